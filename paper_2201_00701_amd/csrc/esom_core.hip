// Landmark preparation, the exact FP64 path, and kernel launchers.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "embed_kernel.h"
#include "esom_internal.h"

namespace esom {

// ---------------------------------------------------------------- preparation

// Centroid of the landmarks (FP64 sum, rounded to FP32), zero-padded to dp:
// one block per dimension.  Block 0 also resets the per-call fallback list
// and the landmark norm maximum, and counts the points of this call.
__global__ void prep_centroid(const float *__restrict__ L, int g, int d, int dp,
                              float *__restrict__ cent, float *__restrict__ lmax,
                              unsigned long long *__restrict__ counters, long long n_points) {
    __shared__ double red[256];
    const int t = blockIdx.x;
    double s = 0.0;
    if (t < d)
        for (int j = threadIdx.x; j < g; j += blockDim.x) s += (double)L[(size_t)j * d + t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) cent[t] = t < d ? (float)(red[0] / (double)g) : 0.f;
    if (t == 0 && threadIdx.x == 0) {
        *lmax = 0.f;
        counters[C_FB_LEN] = 0ull;
        counters[C_POINTS] += (unsigned long long)n_points;
    }
}

// One wavefront per (padded) landmark, lanes over dimensions: centred row,
// squared norm (FP64 wave sum), MFMA operand entries, the zero-padded FP32
// copy for exact rescoring, and the norm maximum.
__global__ void prep_landmarks(const float *__restrict__ L, int g, int gpad, int d, int dp,
                               int mode, const float *__restrict__ cent, void *__restrict__ A,
                               float *__restrict__ norms, float *__restrict__ Lpad,
                               float *__restrict__ lmax) {
    const int j = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= gpad) return;
    const int t = j / TILE, m = j % TILE;
    const int dc = dp / 16;
    const bool real = j < g;
    double nrm = 0.0;
    for (int q = lane; q < dp; q += 64) {
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
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nrm += __shfl_xor(nrm, o);
    if (lane == 0) {
        // MFMA 32x32 output row m sits in lane half h = (m / 4) % 2, register r = 4 (m / 8) + m % 4
        const int hh = (m / 4) % 2, r = 4 * (m / 8) + m % 4;
        norms[((size_t)t * 2 + hh) * 16 + r] = real ? (float)nrm : INFINITY;
        if (real)
            atomicMax(reinterpret_cast<unsigned *>(lmax), __float_as_uint((float)sqrt(nrm) * 1.0000002f));
    }
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
    hipLaunchKernelGGL(prep_centroid, dim3(P.dp), dim3(256), 0, s, L, P.g, P.d, P.dp, P.cent,
                       P.lmax, counters, n_points);
    const int gpad = P.ntiles * TILE;
    hipLaunchKernelGGL(prep_landmarks, dim3((gpad + 3) / 4), dim3(256), 0, s, L, P.g, gpad, P.d,
                       P.dp, mode, P.cent, P.A, P.norms, P.Lpad, P.lmax);
    const long long gg = (long long)P.g * P.g;
    hipLaunchKernelGGL(prep_pairs, dim3((unsigned)((gg + 255) / 256)), dim3(256), 0, s, L, P.g, P.d,
                       P.inv2);
    return hipGetLastError();
}

// ---------------------------------------------------------------- exact FP64 path

// (distance, index) lexicographic minimum across the wavefront.
__device__ __forceinline__ void wave_argmin(double &v, int &j) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o);
        const int oj = __shfl_xor(j, o);
        if (ov < v || (ov == v && oj < j)) {
            v = ov;
            j = oj;
        }
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Recomputes points exactly in FP64, one wavefront (block of 64) per point:
// all g distances from the coordinates into LDS, the k (+1) nearest by
// repeated wave-wide (distance, index) minima, the scores, every pair's
// segment projection from the coordinates spread over the lanes, and
// Cramer's rule; the centroid of the neighbours for degenerate
// neighbourhoods.  all_points = 1 processes every point (shapes outside the
// fast kernels), otherwise the fast kernel's list.
__global__ void __launch_bounds__(64) embed_exact(EmbedArgs a, int all_points) {
    extern __shared__ __align__(16) unsigned char esm[];
    double *dist = reinterpret_cast<double *>(esm);        // g
    double *xs = dist + a.g;                                // d
    double *sel_d = xs + a.d;                               // k + 1
    double *sc = sel_d + (ESOM_MAX_K + 1);                  // k
    int *sel_j = reinterpret_cast<int *>(sc + ESOM_MAX_K);  // k + 1
    const int lane = threadIdx.x;
    const long long cnt = all_points
                              ? a.n
                              : (long long)min(a.counters[C_FB_LEN], (unsigned long long)a.n);
    const int k = a.k;
    const int m = k + 1 <= a.g ? k + 1 : a.g;
    unsigned long long n_fb = 0, n_unc = 0, n_tie = 0, n_ill = 0, n_deg = 0;
    for (long long e = blockIdx.x; e < cnt; e += gridDim.x) {
        const long long pi = all_points ? e : (long long)a.fb_list[e];
        const unsigned reason = all_points ? 0u : (unsigned)a.fb_reason[e];
        ++n_fb;
        n_unc += (reason & R_UNCERT) ? 1 : 0;
        n_tie += (reason & R_NEARTIE) ? 1 : 0;
        n_ill += (reason & R_ILLCOND) ? 1 : 0;
        const float *xr = a.X + pi * a.ldx;
        for (int q = lane; q < a.d; q += 64) xs[q] = (double)xr[q];
        __syncthreads();
        for (int j = lane; j < a.g; j += 64) {
            const float *Lj = a.Lpad + (size_t)j * a.dp;
            double s = 0.0;
            for (int q = 0; q < a.d; ++q) {
                const double df = xs[q] - (double)Lj[q];
                s = fma(df, df, s);
            }
            dist[j] = s;
        }
        __syncthreads();
        // m smallest by (distance, index); taken entries become NaN (never minimal)
        bool bad = false;
        for (int r = 0; r < m; ++r) {
            double bv = INFINITY;
            int bj = 0x7fffffff;
            for (int j = lane; j < a.g; j += 64) {
                const double v = dist[j];
                if (v < bv || (v == bv && j < bj)) {
                    bv = v;
                    bj = j;
                }
            }
            wave_argmin(bv, bj);
            if (bj == 0x7fffffff) bad = true;
            if (lane == 0) {
                sel_d[r] = bv;
                sel_j[r] = bj;
                if (bj != 0x7fffffff) dist[bj] = NAN;
            }
            __syncthreads();
        }
        // Neighbours of points listed only for the projection (ill-conditioned,
        // degenerate) were already certified by the fast kernel: keep its outputs.
        const bool hd_reason = all_points || (reason & (R_UNCERT | R_NEARTIE)) || a.knn_only;
        if (lane < k && hd_reason) {
            if (a.knn_idx) a.knn_idx[pi * k + lane] = bad ? -1 : sel_j[lane];
            if (a.knn_d2) a.knn_d2[pi * k + lane] = (float)sel_d[lane];
        }
        if (lane == 0 && a.knn_mark && hd_reason) a.knn_mark[pi] = 1;
        if (a.knn_only) continue;
        if (bad) {
            if (lane == 0) {
                a.out[2 * pi] = NAN;
                a.out[2 * pi + 1] = NAN;
            }
            continue;
        }
        // scores (every lane computes the neighbourhood statistics)
        const double dl0 = sqrt(sel_d[0]), dlk = sqrt(sel_d[k - 1]);
        const bool degenerate = dl0 == dlk;
        double W = 0.0, mu = 0.0;
        for (int q = 0; q < k; ++q) {
            W += 1.0 / (q + 1);
            mu += sqrt(sel_d[q]) / (q + 1);
        }
        mu /= W;
        double var = 0.0;
        for (int q = 0; q < k; ++q) {
            const double t = sqrt(sel_d[q]) - mu;
            var += t * t / (q + 1);
        }
        var /= W;
        const bool flat = !(var > 1e-30 * mu * mu);
        if (lane < k) {
            const double dq = sqrt(sel_d[lane]);
            const double ev = flat ? 1.0 : exp((double)a.boost * (mu - dq) / sqrt(var));
            const double cv = a.use_cutoff ? 1.0 - exp((double)a.cutoff * (dq / dlk - 1.0)) : 1.0;
            sc[lane] = degenerate ? 0.0 : ev * cv;
        }
        __syncthreads();
        // pairs spread over the lanes
        double M00 = 0.0, M01 = 0.0, M11 = 0.0, r0 = 0.0, r1 = 0.0, ssum = 0.0;
        const int npair = k * (k - 1) / 2;
        for (int p = lane; p < npair && !degenerate; p += 64) {
            int qi = 0, rem = p;
            while (rem >= k - 1 - qi) {
                rem -= k - 1 - qi;
                ++qi;
            }
            const int qj = qi + 1 + rem;
            const int u = sel_j[qi], v = sel_j[qj];
            const float *Lu = a.Lpad + (size_t)u * a.dp;
            const float *Lv = a.Lpad + (size_t)v * a.dp;
            double HH = 0.0, xH = 0.0;
            for (int q = 0; q < a.d; ++q) {
                const double H = (double)Lv[q] - (double)Lu[q];
                HH = fma(H, H, HH);
                xH = fma(xs[q] - (double)Lu[q], H, xH);
            }
            if (HH == 0.0) continue;
            const double D = xH / HH;
            const double lux = a.l2d[2 * u], luy = a.l2d[2 * u + 1];
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
        if (lane < k && !degenerate) {
            const double gs = (double)a.gravity * sc[lane];
            M00 += gs;
            M11 += gs;
            r0 += gs * a.l2d[2 * sel_j[lane]];
            r1 += gs * a.l2d[2 * sel_j[lane] + 1];
            ssum += sc[lane];
        }
        M00 = wave_sum(M00);
        M01 = wave_sum(M01);
        M11 = wave_sum(M11);
        r0 = wave_sum(r0);
        r1 = wave_sum(r1);
        ssum = wave_sum(ssum);
        if (lane == 0) {
            const double det = M00 * M11 - M01 * M01;
            double px, py;
            if (degenerate || !(ssum > 0.0) || !(det > 0.0)) {
                double cx = 0.0, cy = 0.0;
                for (int q = 0; q < k; ++q) {
                    cx += a.l2d[2 * sel_j[q]];
                    cy += a.l2d[2 * sel_j[q] + 1];
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
        __syncthreads();
    }
    if (lane == 0 && n_fb) {
        atomicAdd(&a.counters[all_points ? C_SLOW : C_FALLBACK], n_fb);
        if (n_unc) atomicAdd(&a.counters[C_UNCERT], n_unc);
        if (n_tie) atomicAdd(&a.counters[C_NEARTIE], n_tie);
        if (n_ill) atomicAdd(&a.counters[C_ILLCOND], n_ill);
        if (n_deg) atomicAdd(&a.counters[C_DEGEN], n_deg);
    }
}

static size_t exact_smem(const EmbedArgs &a) {
    return sizeof(double) * ((size_t)a.g + a.d + 2 * ESOM_MAX_K + 1) + sizeof(int) * (ESOM_MAX_K + 1);
}

hipError_t launch_fallback(const EmbedArgs &a, int num_cus, hipStream_t s) {
    // The list length is only known on the device: a fixed grid loops over it.
    hipLaunchKernelGGL(embed_exact, dim3(num_cus * 4), dim3(64), exact_smem(a), s, a, 0);
    return hipGetLastError();
}

hipError_t launch_all_to_fallback(const EmbedArgs &a, int num_cus, hipStream_t s) {
    long long blocks = a.n;
    if (blocks > (long long)num_cus * 16) blocks = (long long)num_cus * 16;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(embed_exact, dim3((unsigned)blocks), dim3(64), exact_smem(a), s, a, 1);
    return hipGetLastError();
}

// ---------------------------------------------------------------- projection from given neighbours

hipError_t launch_project(const EmbedArgs &a, int kp, int num_cus, hipStream_t s) {
    const int block = 256, wpb = 4;
    const size_t smem = (size_t)wpb * kp * 64 * 10;
    long long blocks = ((a.n + 63) / 64 + wpb - 1) / wpb;
    if (blocks > (long long)num_cus * 8) blocks = (long long)num_cus * 8;
    if (blocks < 1) blocks = 1;
    if (kp == 8)
        hipLaunchKernelGGL(embed_project<8>, dim3((unsigned)blocks), dim3(block), smem, s, a);
    else if (kp == 16)
        hipLaunchKernelGGL(embed_project<16>, dim3((unsigned)blocks), dim3(block), smem, s, a);
    else
        hipLaunchKernelGGL(embed_project<32>, dim3((unsigned)blocks), dim3(block), smem, s, a);
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

hipError_t launch_embed(const EmbedArgs &a0, int mode, int kp, int num_cus, size_t lds_per_block,
                        hipStream_t s) {
    EmbedArgs a = a0;
    const int dc = a.dp / 16;
    const size_t wsm = (size_t)wave_smem_bytes(kp, a.npair_tiles);
    const size_t rows = ((size_t)a.g * (a.dp + 4) * 4 + 255) & ~(size_t)255;
    // Stage the landmark rows in LDS when a full block of waves (one block per
    // CU: 3 waves per SIMD in BF16 mode, 2 in FP32 mode) still fits beside
    // them; otherwise rescore from global memory with 4-wave blocks, several
    // per CU.
    const int max_wpb = main_max_block(mode, dc, kp) / 64;
    int wpb;
    if (CENT_LDS_BYTES + rows + (size_t)max_wpb * wsm <= lds_per_block) {
        a.lds_rows = 1;
        wpb = max_wpb;
    } else {
        a.lds_rows = 0;
        wpb = (int)((lds_per_block - CENT_LDS_BYTES) / wsm);
        if (wpb > 4) wpb = 4;
        if (wpb < 1) wpb = 1;
    }
    const size_t smem = CENT_LDS_BYTES + (a.lds_rows ? rows : 0) + (size_t)wpb * wsm;
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
