// Online SOM training support and the fit of added landmarks (supervised
// training of self-organizing maps: the user's 2-D map is the topology, new
// landmarks get high-dimensional positions fitted from their 2-D neighbours).
//
// A training step gathers its batch of points into a contiguous buffer, finds
// each point's best-matching landmark with the exact nearest-landmark path,
// and applies the averaged online update (esom_update.hip, kind 2).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "esom_internal.h"

namespace esom {

// Xb[i] = X[rows[i]] (zeros for rows outside [0, n)); one thread per element.
__global__ void som_gather(const float *__restrict__ X, int64_t n, int64_t ldx, int d,
                           const int32_t *__restrict__ rows, int B, float *__restrict__ Xb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * d) return;
    const int i = (int)(e / d), c = (int)(e % d);
    const int32_t r = rows[i];
    Xb[e] = (r >= 0 && r < n) ? X[(int64_t)r * ldx + c] : 0.f;
}

// nearest[i] = -1 where rows[i] is outside [0, n): that entry presents no point.
__global__ void som_mask(const int32_t *__restrict__ rows, int B, int64_t n, int32_t *__restrict__ nearest) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B && (rows[i] < 0 || rows[i] >= n)) nearest[i] = -1;
}

hipError_t launch_som_gather(const float *X, int64_t n, int64_t ldx, int d, const int32_t *rows, int B,
                             float *Xb, hipStream_t s) {
    const int64_t tot = (int64_t)B * d;
    hipLaunchKernelGGL(som_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, n, ldx, d, rows,
                       B, Xb);
    return hipGetLastError();
}

hipError_t launch_som_mask(const int32_t *rows, int B, int64_t n, int32_t *nearest, hipStream_t s) {
    hipLaunchKernelGGL(som_mask, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, rows, B, n, nearest);
    return hipGetLastError();
}

// Lexicographic order on (squared distance, index).
__device__ __forceinline__ bool lex_before(double a, int ia, double b, int ib) {
    return a < b || (a == b && ia < ib);
}

// One wavefront per added landmark q at 2-D position p_q:
//  1. its kfit nearest 2-D landmarks by (squared distance, index), one per
//     round: each round takes the wave-wide lexicographic minimum among the
//     landmarks that come after the previous round's choice;
//  2. weights w_i = exp(-(d2_i - d2_1) / (2 sigma^2)) (scaled so the nearest
//     weighs 1) and the 3 x 3 weighted normal matrix G of the affine fit
//     z -> A z + c, z = (lx, ly, 1), in FP64 wave sums;
//  3. v = G^-1 (p, 1) by Cramer's rule and coefficients beta_i = w_i (v . z_i),
//     or the weighted mean when G is numerically singular (fewer than three
//     or collinear neighbours);
//  4. out_q = sum_i beta_i L_i, lanes over dimensions.
constexpr int FIT_MAX_K = 64;

__global__ void __launch_bounds__(64) fit_landmarks(const float *__restrict__ L, const float *__restrict__ l2d,
                                                    int g, int d, const float *__restrict__ p, int kfit,
                                                    float sigma, float *__restrict__ out) {
    __shared__ double beta[FIT_MAX_K];
    __shared__ int nbs[FIT_MAX_K];
    const int q = blockIdx.x;
    const int lane = threadIdx.x;
    const double px = (double)p[2 * q], py = (double)p[2 * q + 1];
    double prev_d = -1.0;
    int prev_j = -1;
    double my_d = 0.0;  // lane i keeps neighbour i
    int my_j = -1;
    for (int r = 0; r < kfit; ++r) {
        double bd = INFINITY;
        int bj = 0x7fffffff;
        for (int j = lane; j < g; j += 64) {
            const double dx = (double)l2d[2 * j] - px, dy = (double)l2d[2 * j + 1] - py;
            const double dj = dx * dx + dy * dy;
            if (lex_before(prev_d, prev_j, dj, j) && lex_before(dj, j, bd, bj)) {
                bd = dj;
                bj = j;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double od = __shfl_xor(bd, o);
            const int oj = __shfl_xor(bj, o);
            if (lex_before(od, oj, bd, bj)) {
                bd = od;
                bj = oj;
            }
        }
        prev_d = bd;
        prev_j = bj;
        if (lane == r) {
            my_d = bd;
            my_j = bj;
        }
    }
    const double d0 = __shfl(my_d, 0);
    const bool act = lane < kfit;
    const double w = act ? exp(-(my_d - d0) / (2.0 * (double)sigma * (double)sigma)) : 0.0;
    const double zx = act ? (double)l2d[2 * my_j] : 0.0, zy = act ? (double)l2d[2 * my_j + 1] : 0.0;
    double Gs[7] = {w * zx * zx, w * zx * zy, w * zx, w * zy * zy, w * zy, w, 0.0};
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) Gs[i] += __shfl_xor(Gs[i], o);
    const double G[3][3] = {{Gs[0], Gs[1], Gs[2]}, {Gs[1], Gs[3], Gs[4]}, {Gs[2], Gs[4], Gs[5]}};
    const double W = Gs[5];
    auto det3 = [](const double (&M)[3][3]) {
        return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
               M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    };
    const double det = det3(G);
    const double md = (G[0][0] + G[1][1] + G[2][2]) / 3.0;
    double bt;
    if (kfit >= 3 && det > 1e-12 * md * md * md) {
        const double e[3] = {px, py, 1.0};
        double v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double M[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) M[a][b] = (b == c) ? e[a] : G[a][b];
            v[c] = det3(M) / det;
        }
        bt = w * (v[0] * zx + v[1] * zy + v[2]);
    } else {
        bt = w / W;
    }
    if (act) {
        beta[lane] = bt;
        nbs[lane] = my_j;
    }
    __syncthreads();
    for (int c = lane; c < d; c += 64) {
        double o = 0.0;
        for (int i = 0; i < kfit; ++i) o += beta[i] * (double)L[(size_t)nbs[i] * d + c];
        out[(size_t)q * d + c] = (float)o;
    }
}

hipError_t launch_fit_landmarks(const float *L, const float *l2d, int g, int d, const float *p, int m,
                                int kfit, float sigma, float *out, hipStream_t s) {
    if (m > 0)
        hipLaunchKernelGGL(fit_landmarks, dim3((unsigned)m), dim3(64), 0, s, L, l2d, g, d, p, kfit, sigma, out);
    return hipGetLastError();
}

}  // namespace esom
