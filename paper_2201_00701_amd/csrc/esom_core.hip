// Landmark preparation, the exact FP64 path, and kernel launchers.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "embed_kernel.h"
#include "esom_internal.h"

namespace esom {

// ---------------------------------------------------------------- preparation

// Centroid of the landmarks (FP64 sum, rounded to FP32), zero-padded to dp.
// Also resets the per-call fallback list and the landmark norm maximum, and
// counts the points of this call.
__global__ void prep_centroid(const float *__restrict__ L, int g, int d, int dp,
                              float *__restrict__ cent, float *__restrict__ lmax,
                              unsigned long long *__restrict__ counters, long long n_points) {
    for (int t = threadIdx.x; t < dp; t += blockDim.x) {
        double s = 0.0;
        if (t < d)
            for (int j = 0; j < g; ++j) s += (double)L[(size_t)j * d + t];
        cent[t] = t < d ? (float)(s / (double)g) : 0.f;
    }
    if (threadIdx.x == 0) {
        *lmax = 0.f;
        counters[C_FB_LEN] = 0ull;
        counters[C_POINTS] += (unsigned long long)n_points;
    }
}

// One thread per (padded) landmark: centred row, squared norm, MFMA operand
// entries, the zero-padded FP32 copy for exact rescoring, and the norm max.
__global__ void prep_landmarks(const float *__restrict__ L, int g, int gpad, int d, int dp,
                               int mode, const float *__restrict__ cent, void *__restrict__ A,
                               float *__restrict__ norms, float *__restrict__ Lpad,
                               float *__restrict__ lmax) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= gpad) return;
    const int t = j / TILE, m = j % TILE;
    const int dc = dp / 16;
    const bool real = j < g;
    double nrm = 0.0;
    for (int q = 0; q < dp; ++q) {
        const float lv = (real && q < d) ? L[(size_t)j * d + q] : 0.f;
        const float c = (real && q < d) ? lv - cent[q] : 0.f;
        nrm += (double)c * (double)c;
        if (real) Lpad[(size_t)j * dp + q] = lv;
        const float a2 = -2.f * c;
        if (mode == 1) {
            // A_bf16[t][c][lane = 32 h + m][e], dim = 16 c + 8 h + e
            const int cc = q / 16, hh = (q % 16) / 8, e = q % 8;
            unsigned u = __float_as_uint(a2);
            u += 0x7FFFu + ((u >> 16) & 1u);
            reinterpret_cast<unsigned short *>(A)[(((size_t)t * dc + cc) * 64 + 32 * hh + m) * 8 + e] =
                (unsigned short)(u >> 16);
        } else {
            // A_f32[t][s][lane = 32 h + m], dim = 2 s + h
            const int s = q / 2, hh = q % 2;
            reinterpret_cast<float *>(A)[((size_t)t * (dp / 2) + s) * 64 + 32 * hh + m] = a2;
        }
    }
    // MFMA 32x32 output row m sits in lane half h = (m / 4) % 2, register r = 4 (m / 8) + m % 4
    const int hh = (m / 4) % 2, r = 4 * (m / 8) + m % 4;
    norms[((size_t)t * 2 + hh) * 16 + r] = real ? (float)nrm : INFINITY;
    if (real) atomicMax(reinterpret_cast<unsigned *>(lmax), __float_as_uint((float)sqrt(nrm) * 1.0000002f));
}

// Pair table inv2[u][v] = 1 / (2 |L_u - L_v|^2) (FP64 differences), -1 when zero.
__global__ void prep_pairs(const float *__restrict__ L, int g, int d, float *__restrict__ inv2) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)g * g) return;
    const int u = (int)(e / g), v = (int)(e % g);
    double s = 0.0;
    for (int q = 0; q < d; ++q) {
        const double df = (double)L[(size_t)v * d + q] - (double)L[(size_t)u * d + q];
        s += df * df;
    }
    inv2[e] = s > 0.0 ? (float)(0.5 / s) : -1.f;
}

hipError_t launch_prep(const Prep &P, const float *L, int mode, unsigned long long *counters,
                       long long n_points, hipStream_t s) {
    hipLaunchKernelGGL(prep_centroid, dim3(1), dim3(256), 0, s, L, P.g, P.d, P.dp, P.cent, P.lmax,
                       counters, n_points);
    const int gpad = P.ntiles * TILE;
    hipLaunchKernelGGL(prep_landmarks, dim3((gpad + 255) / 256), dim3(256), 0, s, L, P.g, gpad, P.d,
                       P.dp, mode, P.cent, P.A, P.norms, P.Lpad, P.lmax);
    const long long gg = (long long)P.g * P.g;
    hipLaunchKernelGGL(prep_pairs, dim3((unsigned)((gg + 255) / 256)), dim3(256), 0, s, L, P.g, P.d,
                       P.inv2);
    return hipGetLastError();
}

// ---------------------------------------------------------------- exact FP64 path

// Recomputes points exactly in FP64: full k-nearest scan with (distance,
// index) order, scores, every pair's segment projection from the
// coordinates, Cramer's rule; the centroid for degenerate neighbourhoods.
// all_points = 1 processes every point (shapes outside the fast kernels).
__global__ void __launch_bounds__(64) embed_exact(EmbedArgs a, int all_points) {
    const long long cnt = all_points
                              ? a.n
                              : (long long)min(a.counters[C_FB_LEN], (unsigned long long)a.n);
    unsigned long long n_fb = 0, n_unc = 0, n_tie = 0, n_ill = 0, n_deg = 0;
    double dd[ESOM_MAX_K + 1];
    int nb[ESOM_MAX_K + 1];
    double dl[ESOM_MAX_K], sc[ESOM_MAX_K];
    const int m = a.k + 1 <= a.g ? a.k + 1 : a.g;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < cnt;
         e += (long long)gridDim.x * blockDim.x) {
        const long long pi = all_points ? e : (long long)a.fb_list[e];
        const unsigned reason = all_points ? 0u : (unsigned)a.fb_reason[e];
        ++n_fb;
        n_unc += (reason & R_UNCERT) ? 1 : 0;
        n_tie += (reason & R_NEARTIE) ? 1 : 0;
        n_ill += (reason & R_ILLCOND) ? 1 : 0;
        const float *xr = a.X + pi * a.ldx;
        for (int q = 0; q < m; ++q) {
            dd[q] = INFINITY;
            nb[q] = -1;
        }
        for (int j = 0; j < a.g; ++j) {
            const float *Lj = a.Lpad + (size_t)j * a.dp;
            double s = 0.0;
            for (int q = 0; q < a.d; ++q) {
                const double df = (double)xr[q] - (double)Lj[q];
                s += df * df;
            }
            if (nb[m - 1] >= 0 && !(s < dd[m - 1])) continue;  // j ascends: ties keep the earlier
            int pos = m - 1;
            while (pos > 0 && (nb[pos - 1] < 0 || s < dd[pos - 1])) {
                dd[pos] = dd[pos - 1];
                nb[pos] = nb[pos - 1];
                --pos;
            }
            dd[pos] = s;
            nb[pos] = j;
        }
        const int k = a.k;
        if (a.knn_idx)
            for (int q = 0; q < k; ++q) a.knn_idx[pi * k + q] = nb[q];
        if (a.knn_d2)
            for (int q = 0; q < k; ++q) a.knn_d2[pi * k + q] = (float)dd[q];
        if (a.knn_only) continue;
        if (nb[k - 1] < 0) {  // non-finite input: no ordered neighbours
            a.out[2 * pi] = NAN;
            a.out[2 * pi + 1] = NAN;
            continue;
        }

        // scores
        for (int q = 0; q < k; ++q) dl[q] = sqrt(dd[q]);
        bool degenerate = dl[0] == dl[k - 1];
        double ssum = 0.0;
        if (!degenerate) {
            double W = 0.0, mu = 0.0;
            for (int q = 0; q < k; ++q) {
                W += 1.0 / (q + 1);
                mu += dl[q] / (q + 1);
            }
            mu /= W;
            double var = 0.0;
            for (int q = 0; q < k; ++q) var += (dl[q] - mu) * (dl[q] - mu) / (q + 1);
            var /= W;
            const bool flat = !(var > 1e-30 * mu * mu);
            for (int q = 0; q < k; ++q) {
                const double ev = flat ? 1.0 : exp((double)a.boost * (mu - dl[q]) / sqrt(var));
                const double cv = a.use_cutoff ? 1.0 - exp((double)a.cutoff * (dl[q] / dl[k - 1] - 1.0))
                                               : 1.0;
                sc[q] = ev * cv;
                ssum += sc[q];
            }
        }
        // pairs: D_uv from the coordinates (FP64)
        double M00 = 0.0, M01 = 0.0, M11 = 0.0, r0 = 0.0, r1 = 0.0;
        if (!degenerate) {
            for (int qi = 0; qi < k; ++qi) {
                const int u = nb[qi];
                const float *Lu = a.Lpad + (size_t)u * a.dp;
                const double lux = a.l2d[2 * u], luy = a.l2d[2 * u + 1];
                for (int qj = qi + 1; qj < k; ++qj) {
                    const int v = nb[qj];
                    const float *Lv = a.Lpad + (size_t)v * a.dp;
                    double HH = 0.0, xH = 0.0;
                    for (int q = 0; q < a.d; ++q) {
                        const double H = (double)Lv[q] - (double)Lu[q];
                        HH += H * H;
                        xH += ((double)xr[q] - (double)Lu[q]) * H;
                    }
                    if (HH == 0.0) continue;
                    const double D = xH / HH;
                    const double hx = (double)a.l2d[2 * v] - lux, hy = (double)a.l2d[2 * v + 1] - luy;
                    const double hh = hx * hx + hy * hy;
                    if (hh == 0.0) continue;
                    const double qw = sc[qi] * sc[qj] * pow(hh, -(double)a.adjust);
                    const double rhs = D + (hx * lux + hy * luy) / hh;
                    M00 += qw * hx * hx / hh;
                    M01 += qw * hx * hy / hh;
                    M11 += qw * hy * hy / hh;
                    r0 += qw * hx * rhs;
                    r1 += qw * hy * rhs;
                }
            }
            for (int q = 0; q < k; ++q) {
                const double gs = (double)a.gravity * sc[q];
                M00 += gs;
                M11 += gs;
                r0 += gs * a.l2d[2 * nb[q]];
                r1 += gs * a.l2d[2 * nb[q] + 1];
            }
        }
        const double det = M00 * M11 - M01 * M01;
        double px, py;
        if (degenerate || !(ssum > 0.0) || !(det > 0.0)) {
            double cx = 0.0, cy = 0.0;
            for (int q = 0; q < k; ++q) {
                cx += a.l2d[2 * nb[q]];
                cy += a.l2d[2 * nb[q] + 1];
            }
            px = cx / k;
            py = cy / k;
            ++n_deg;
        } else {
            px = (r0 * M11 - M01 * r1) / det;
            py = (M00 * r1 - M01 * r0) / det;
        }
        a.out[2 * pi] = (float)px;
        a.out[2 * pi + 1] = (float)py;
    }
    if (n_fb) {
        atomicAdd(&a.counters[all_points ? C_SLOW : C_FALLBACK], n_fb);
        if (n_unc) atomicAdd(&a.counters[C_UNCERT], n_unc);
        if (n_tie) atomicAdd(&a.counters[C_NEARTIE], n_tie);
        if (n_ill) atomicAdd(&a.counters[C_ILLCOND], n_ill);
        if (n_deg) atomicAdd(&a.counters[C_DEGEN], n_deg);
    }
}

hipError_t launch_fallback(const EmbedArgs &a, int num_cus, hipStream_t s) {
    hipLaunchKernelGGL(embed_exact, dim3(num_cus * 4), dim3(64), 0, s, a, 0);
    return hipGetLastError();
}

hipError_t launch_all_to_fallback(const EmbedArgs &a, int num_cus, hipStream_t s) {
    long long blocks = (a.n + 63) / 64;
    if (blocks > (long long)num_cus * 16) blocks = (long long)num_cus * 16;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(embed_exact, dim3((unsigned)blocks), dim3(64), 0, s, a, 1);
    return hipGetLastError();
}

// ---------------------------------------------------------------- main kernel dispatch

// Instantiation units (embed_inst.hip, one object per (mode, KP)); each
// picks the DC instantiation, sizes a persistent grid from the occupancy of
// that kernel, and launches it.
hipError_t launch_main_m0_kp8(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp16(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp32(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp8(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp16(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp32(const EmbedArgs &, int, int, size_t, int, hipStream_t);

hipError_t launch_embed(const EmbedArgs &a, int mode, int kp, int num_cus, hipStream_t s) {
    const int dc = a.dp / 16;
    const int wsm = wave_smem_bytes(kp, a.npair_tiles);
    int wpb = 65536 / wsm;
    if (wpb > 4) wpb = 4;
    if (wpb < 1) wpb = 1;
    const size_t smem = (size_t)wpb * wsm;
    const int block = 64 * wpb;
    if (mode == 0) {
        if (kp == 8) return launch_main_m0_kp8(a, dc, block, smem, num_cus, s);
        if (kp == 16) return launch_main_m0_kp16(a, dc, block, smem, num_cus, s);
        return launch_main_m0_kp32(a, dc, block, smem, num_cus, s);
    }
    if (kp == 8) return launch_main_m1_kp8(a, dc, block, smem, num_cus, s);
    if (kp == 16) return launch_main_m1_kp16(a, dc, block, smem, num_cus, s);
    return launch_main_m1_kp32(a, dc, block, smem, num_cus, s);
}

}  // namespace esom
