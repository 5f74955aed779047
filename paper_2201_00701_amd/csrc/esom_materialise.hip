// The materialised-distance path: the distance pass and the k-NN selection
// as two kernels with the keys written to device memory between them (the
// separation the paper's "k-NN step" weighs against fusion and leaves for
// extreme d).  It serves the dimensions beyond the fused kernel's register
// budget (d above 64 in FP32 mode, above 128 in BF16 mode, up to 256), which
// otherwise go point by point through the exact FP64 path.
//
//   keys_kernel    one wavefront per 32 points: their centred rows staged in
//                  LDS, every 32-landmark tile of the FP32 MFMA operand
//                  (v_mfma_f32_32x32x2f32, C initialised to |L_j - c|^2)
//                  gives key_ij = |L_j - c|^2 - 2 <x_i - c, L_j - c> for all
//                  landmarks, stored per point in landmark-position order;
//   select_kernel  one wavefront per point: every lane keeps the C smallest
//                  of its keys, the wavefront merges them (C rounds of a wave
//                  minimum), the C candidates are rescored with exact FP32
//                  differences and ranked by (distance, index); the point is
//                  certified when its k-th rescored distance lies below the
//                  smallest non-candidate key by more than the keys' rounding
//                  bound, else it is marked for the exact path, as is a k-th /
//                  (k+1)-th tie FP32 cannot order.
// The projection then runs from these neighbours (embed_project) and the
// exact path takes the marked points.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "embed_kernel.h"
#include "esom_internal.h"

namespace esom {

constexpr int MK_WAVES = 4;  // wavefronts (32 points each) per keys block

__global__ void __launch_bounds__(64 * MK_WAVES) keys_kernel(MatArgs m) {
    extern __shared__ __align__(16) float ksm[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int h = lane >> 5, i32 = lane & 31;
    const int dp = m.dp;
    float *xs = ksm + (size_t)wv * 32 * (dp + 1);  // 32 centred rows, stride dp + 1
    const int64_t p0 = ((int64_t)blockIdx.x * MK_WAVES + wv) * 32;
    if (p0 >= m.n) return;  // whole wavefronts leave together (no block barrier below)
    for (int e = lane; e < 32 * dp; e += 64) {
        const int r = e / dp, c = e % dp;
        const int64_t pi = p0 + r;
        xs[r * (dp + 1) + c] = (pi < m.n && c < m.d) ? m.X[pi * m.ldx + c] - m.cent[c] : 0.f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const float *A = static_cast<const float *>(m.A);
    const float *xrow = xs + i32 * (dp + 1) + h;
    for (int t = 0; t < m.ntiles; ++t) {
        f32x16 acc;
        const float4 *np = reinterpret_cast<const float4 *>(m.norms + (size_t)(t * 2 + h) * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = np[q];
            acc[4 * q] = v.x;
            acc[4 * q + 1] = v.y;
            acc[4 * q + 2] = v.z;
            acc[4 * q + 3] = v.w;
        }
        const float *At = A + (size_t)t * (dp / 2) * 64 + lane;
        for (int s = 0; s < dp / 2; ++s)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(At[(size_t)s * 64], xrow[2 * s], acc, 0, 0, 0);
        // lane (h, i32) holds point i32 and the tile's rows m = 8 (r / 4) + 4 h + r % 4,
        // which are landmark positions 64 (t / 2) + 32 (t % 2) + 2 (4 (m / 8) + m % 4) + (m / 4) % 2
        const int64_t pi = p0 + i32;
        if (pi < m.n) {
            float *krow = m.keys + pi * m.gpad;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * h + (r & 3);
                const int rr = 4 * (row >> 3) + (row & 3), hj = (row >> 2) & 1;
                const int pos = 64 * (t >> 1) + 32 * (t & 1) + 2 * rr + hj;
                krow[pos] = acc[r];
            }
        }
    }
}

// Insertion into an ascending list of C (key, position) entries kept in
// registers (MAT_MAX_C slots, the first C used).
__device__ __forceinline__ void mat_insert(float (&kd)[MAT_MAX_C], int (&kp)[MAT_MAX_C], int C, float v, int pos) {
#pragma unroll
    for (int q = 0; q < MAT_MAX_C; ++q) {
        if (q < C && (v < kd[q] || (v == kd[q] && pos < kp[q]))) {
            const float tv = kd[q];
            const int tp = kp[q];
            kd[q] = v;
            kp[q] = pos;
            v = tv;
            pos = tp;
        }
    }
}

__global__ void __launch_bounds__(256) select_kernel(MatArgs m) {
    __shared__ float cd[4][64];  // per wavefront: rescored candidates
    __shared__ int cj[4][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int C = m.C, k = m.k;
    for (int64_t pi = (int64_t)blockIdx.x * 4 + wv; pi < m.n; pi += nw) {
        const float *krow = m.keys + pi * m.gpad;
        float kd[MAT_MAX_C];
        int kp[MAT_MAX_C];
#pragma unroll
        for (int q = 0; q < MAT_MAX_C; ++q) {
            kd[q] = INFINITY;
            kp[q] = INT32_MAX;
        }
        for (int j = lane; j < m.gpad; j += 64) mat_insert(kd, kp, C, krow[j], j);
        // the (C+1) smallest keys of the point: C candidates and the smallest
        // non-candidate (the certificate's threshold), by C + 1 wave minima
        int cand_pos = -1;
        float cand_key = INFINITY, tau = INFINITY;
        for (int r = 0; r <= C; ++r) {
            float mv = kd[0];
            int mp = kp[0];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const float ov = __shfl_xor(mv, o);
                const int op = __shfl_xor(mp, o);
                if (ov < mv || (ov == mv && op < mp)) {
                    mv = ov;
                    mp = op;
                }
            }
            if (r == C) {
                tau = mv;
                break;
            }
            if (lane == r) {
                cand_pos = mp;
                cand_key = mv;
            }
            if (kp[0] == mp && mp != INT32_MAX) {
#pragma unroll
                for (int q = 0; q + 1 < MAT_MAX_C; ++q) {
                    kd[q] = kd[q + 1];
                    kp[q] = kp[q + 1];
                }
                kd[MAT_MAX_C - 1] = INFINITY;
                kp[MAT_MAX_C - 1] = INT32_MAX;
            }
        }
        (void)cand_key;
        // exact FP32 rescoring of candidate r on lane r (positions past g are padding)
        const float *x = m.X + pi * m.ldx;
        float d2 = INFINITY;
        int jl = INT32_MAX;
        if (lane < C && cand_pos >= 0 && cand_pos < m.g) {
            jl = m.perm[cand_pos];
            const float *Lr = m.Lpad + (size_t)cand_pos * m.dp;
            float s = 0.f;
            for (int t = 0; t < m.d; ++t) {
                const float df = x[t] - Lr[t];
                s = fmaf(df, df, s);
            }
            d2 = s;
        }
        // rank by (distance, landmark index)
        int rank = 0;
        for (int p = 0; p < C; ++p) {
            const float dp2 = __shfl(d2, p);
            const int jp = __shfl(jl, p);
            rank += (lane < C && (dp2 < d2 || (dp2 == d2 && jp < jl))) ? 1 : 0;
        }
        if (lane < C) {
            cd[wv][rank] = d2;
            cj[wv][rank] = jl;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // certificate: every non-candidate's key is >= tau, so its exact
        // distance^2 exceeds tau + |x - c|^2 - E (E the FP32 keys' rounding bound)
        float xn = 0.f;
        if (lane < 32) {
            for (int t = lane; t < m.d; t += 32) {
                const float v = x[t] - m.cent[t];
                xn = fmaf(v, v, xn);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) xn += __shfl_xor(xn, o);
        const float lmax = m.lmax[0];
        const float sx = sqrtf(xn);
        const float facc = (2.f * m.dp + 16.f) * U32 * (sx + lmax) * (sx + lmax);
        const float E = 1.01f * (2.f * (2.f * U32 + U32 * U32) * sx * lmax + facc);
        float rhs = tau + xn - E;
        rhs -= 4.f * U32 * (fabsf(tau) + xn + E);
        const float d2k = cd[wv][k - 1];
        const float d2k1 = C > k ? cd[wv][k] : INFINITY;
        const float rb = (float)(m.dp + 3) * U32;  // rounding bound of a rescored distance
        bool mark = !(tau < INFINITY ? d2k * (1.f + rb) < rhs : d2k < INFINITY);
        if (d2k1 < INFINITY && d2k1 - d2k <= 2.f * rb * d2k1) mark = true;  // k-th / (k+1)-th closer than FP32 orders
        // adjacent entries FP32 cannot order when the caller wants the exact order
        if (m.exact_order)
            for (int q = 1; q < k; ++q)
                if (cd[wv][q] - cd[wv][q - 1] <= 2.f * rb * cd[wv][q]) mark = true;
        if (lane < k) {
            m.knn_idx[pi * k + lane] = cj[wv][lane];
            m.knn_d2[pi * k + lane] = cd[wv][lane];
        }
        if (lane == 0) m.knn_mark[pi] = mark ? 1 : 0;
        __builtin_amdgcn_wave_barrier();
    }
}

hipError_t launch_materialise(const MatArgs &m, int num_cus, hipStream_t s) {
    const long long waves = (m.n + 31) / 32;
    const unsigned kblocks = (unsigned)((waves + MK_WAVES - 1) / MK_WAVES);
    const size_t ksmem = sizeof(float) * (size_t)MK_WAVES * 32 * (m.dp + 1);
    hipLaunchKernelGGL(keys_kernel, dim3(kblocks), dim3(64 * MK_WAVES), ksmem, s, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    long long sblocks = (m.n + 3) / 4;
    if (sblocks > (long long)num_cus * 8) sblocks = (long long)num_cus * 8;
    if (sblocks < 1) sblocks = 1;
    hipLaunchKernelGGL(select_kernel, dim3((unsigned)sblocks), dim3(256), 0, s, m);
    return hipGetLastError();
}

}  // namespace esom
