// EmbedSOM projection into 3-D (the paper states the method in 2-D for
// brevity, Section "Landmark-directed dimensionality reduction"): the same
// neighbours, scores and segment projections, with 3-D landmark positions l
// (g x 3) and a 3 x 3 system solved by Cramer's rule.  The k nearest
// landmarks come from the 2-D path's screen and exact selection (k-NN only);
// this kernel then works in FP64 throughout, one wavefront per point:
//   lanes q < k: the exact squared distance of neighbour q, then its rank by
//     (distance, index) and its score;
//   all lanes: the pairs (a < b) spread over the wavefront, each projecting
//     the point on the segment L_u -> L_v directly, D = <x - L_u, H> / |H|^2;
//   wave sums of the six entries of M and three of r, then Cramer's rule,
//   or the centroid of the neighbours' positions for a degenerate
//   neighbourhood or a numerically singular system (det <= 1e-9 (tr/3)^3).
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "esom_internal.h"

namespace esom {

constexpr int E3_WAVES = 4;  // wavefronts per block

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double det3x3(double a00, double a01, double a02, double a10, double a11, double a12,
                                         double a20, double a21, double a22) {
    return a00 * (a11 * a22 - a12 * a21) - a01 * (a10 * a22 - a12 * a20) + a02 * (a10 * a21 - a11 * a20);
}

// Pair p (0 <= p < k (k - 1) / 2) as (a, b), a < b, in row order
// (0,1), (0,2), ..., (0,k-1), (1,2), ...: row a starts at a (2k - a - 1) / 2.
__device__ __forceinline__ void pair_of(int p, int k, int &a, int &b) {
    const double kk = 2.0 * k - 1.0;
    int r = (int)floor((kk - sqrt(kk * kk - 8.0 * p)) * 0.5);
    if (r < 0) r = 0;
    // guard the floating-point root against an off-by-one
    while (r > 0 && r * (2 * k - r - 1) / 2 > p) --r;
    while ((r + 1) * (2 * k - r - 2) / 2 <= p) ++r;
    a = r;
    b = p - r * (2 * k - r - 1) / 2 + r + 1;
}

__global__ void __launch_bounds__(64 * E3_WAVES) embed3_kernel(Embed3Args e) {
    __shared__ int sj[E3_WAVES][64];      // sorted neighbours' landmark indices
    __shared__ double ss[E3_WAVES][64];   // ... their scores
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t nw = (int64_t)gridDim.x * E3_WAVES;
    const int k = e.k;
    const int npairs = k * (k - 1) / 2;
    for (int64_t pi = (int64_t)blockIdx.x * E3_WAVES + wv; pi < e.n; pi += nw) {
        const float *x = e.X + pi * e.ldx;
        // neighbour q on lane q: index and exact squared distance
        int jq = 0;
        bool bad = false;
        double dq = INFINITY;
        if (lane < k) {
            jq = e.knn_idx[pi * k + lane];
            if (jq < 0 || jq >= e.g) {
                bad = true;
                jq = 0;
            }
            const float *Lr = e.L + (size_t)jq * e.d;
            double s = 0.0;
            for (int t = 0; t < e.d; ++t) {
                const double df = (double)x[t] - (double)Lr[t];
                s = fma(df, df, s);
            }
            dq = s;
        }
        if (__ballot(bad) != 0ull) {
            // a point without k finite distances (non-finite input)
            if (lane < 3) e.out[3 * pi + lane] = NAN;
            continue;
        }
        // rank by (distance, index)
        int rank = 0;
        for (int p = 0; p < k; ++p) {
            const double dp = __shfl(dq, p);
            const int jp = __shfl(jq, p);
            rank += (lane < k && (dp < dq || (dp == dq && jp < jq))) ? 1 : 0;
        }
        if (lane < k) sj[wv][rank] = jq;
        // the sorted distances, lane r = rank r
        double d2r = 0.0;
        for (int p = 0; p < k; ++p) {
            const double dp = __shfl(dq, p);
            const int rp = __shfl(rank, p);
            if (rp == lane) d2r = dp;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const int jr = lane < k ? sj[wv][lane] : 0;
        // scores: rank weights 1/(r+1), weighted mean and variance of the
        // distances, exponential, and the cutoff at the k-th
        const double dl = sqrt(d2r);
        const double w = lane < k ? 1.0 / (double)(lane + 1) : 0.0;
        const double mu = wave_sum64(w * dl) / e.Wk;
        const double dev = lane < k ? dl - mu : 0.0;
        const double var = wave_sum64(w * dev * dev) / e.Wk;
        const double d0 = __shfl(dl, 0), dk = __shfl(dl, k - 1);
        const bool degenerate = d0 == dk;
        double s = 0.0;
        if (lane < k && !degenerate) {
            const double ex = var <= 1e-30 * mu * mu ? 1.0 : exp(e.boost * (mu - dl) / sqrt(var));
            const double c = e.use_cutoff ? 1.0 - exp(e.cutoff * (dl / dk - 1.0)) : 1.0;
            s = ex * c;
        }
        if (lane < k) ss[wv][lane] = s;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const double ssum = wave_sum64(s);
        double l3r[3] = {0.0, 0.0, 0.0};
        if (lane < k)
            for (int c = 0; c < 3; ++c) l3r[c] = (double)e.l3[(size_t)3 * jr + c];
        // gravity of neighbour r, then the pairs spread over the lanes
        const double gs = degenerate ? 0.0 : e.gravity * s;
        double m00 = gs, m01 = 0.0, m02 = 0.0, m11 = gs, m12 = 0.0, m22 = gs;
        double r0 = gs * l3r[0], r1 = gs * l3r[1], r2 = gs * l3r[2];
        if (!degenerate) {
            for (int p = lane; p < npairs; p += 64) {
                int a, b;
                pair_of(p, k, a, b);
                const int u = sj[wv][a], v = sj[wv][b];
                const float *Lu = e.L + (size_t)u * e.d, *Lv = e.L + (size_t)v * e.d;
                double HH = 0.0, xH = 0.0;
                for (int t = 0; t < e.d; ++t) {
                    const double lu = Lu[t];
                    const double H = (double)Lv[t] - lu;
                    HH = fma(H, H, HH);
                    xH = fma((double)x[t] - lu, H, xH);
                }
                if (HH == 0.0) continue;  // coincident high-dimensional landmarks
                double h[3], hh = 0.0, hl = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double lu3 = e.l3[(size_t)3 * u + c];
                    h[c] = (double)e.l3[(size_t)3 * v + c] - lu3;
                    hh = fma(h[c], h[c], hh);
                    hl = fma(h[c], lu3, hl);
                }
                if (hh == 0.0) continue;  // coincident 3-D positions
                const double q = ss[wv][a] * ss[wv][b] * pow(hh, -(double)e.adjust);
                const double rhs = xH / HH + hl / hh;
                const double qh = q / hh;
                m00 = fma(qh * h[0], h[0], m00);
                m01 = fma(qh * h[0], h[1], m01);
                m02 = fma(qh * h[0], h[2], m02);
                m11 = fma(qh * h[1], h[1], m11);
                m12 = fma(qh * h[1], h[2], m12);
                m22 = fma(qh * h[2], h[2], m22);
                r0 = fma(q * h[0], rhs, r0);
                r1 = fma(q * h[1], rhs, r1);
                r2 = fma(q * h[2], rhs, r2);
            }
        }
        m00 = wave_sum64(m00);
        m01 = wave_sum64(m01);
        m02 = wave_sum64(m02);
        m11 = wave_sum64(m11);
        m12 = wave_sum64(m12);
        m22 = wave_sum64(m22);
        r0 = wave_sum64(r0);
        r1 = wave_sum64(r1);
        r2 = wave_sum64(r2);
        const double c0 = wave_sum64(l3r[0]), c1 = wave_sum64(l3r[1]), c2 = wave_sum64(l3r[2]);
        if (lane == 0) {
            const double det = det3x3(m00, m01, m02, m01, m11, m12, m02, m12, m22);
            const double tr3 = (m00 + m11 + m22) / 3.0;
            double p0, p1, p2;
            if (degenerate || ssum == 0.0 || !(det > 1e-9 * tr3 * tr3 * tr3)) {
                p0 = c0 / k;
                p1 = c1 / k;
                p2 = c2 / k;
            } else {
                p0 = det3x3(r0, m01, m02, r1, m11, m12, r2, m12, m22) / det;
                p1 = det3x3(m00, r0, m02, m01, r1, m12, m02, r2, m22) / det;
                p2 = det3x3(m00, m01, r0, m01, m11, r1, m02, m12, r2) / det;
            }
            e.out[3 * pi] = (float)p0;
            e.out[3 * pi + 1] = (float)p1;
            e.out[3 * pi + 2] = (float)p2;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

hipError_t launch_embed3(const Embed3Args &e, int num_cus, hipStream_t s) {
    long long blocks = (e.n + E3_WAVES - 1) / E3_WAVES;
    const long long cap = (long long)num_cus * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(embed3_kernel, dim3((unsigned)blocks), dim3(64 * E3_WAVES), 0, s, e);
    return hipGetLastError();
}

}  // namespace esom
