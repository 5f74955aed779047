// The paper's kernel families, rebuilt for gfx950 as ablations of the fused
// kernel (Sections "k-NN step" and "Projection step"): plain FP32 throughout,
// as the paper's kernels are, with the paper's work division and caching but
// 64-wide wavefronts.  They compute what the fused path computes (the k
// nearest landmarks; the projection from given neighbours) without its
// screen, certificate or FP64 solve, so that the relative merits of the
// paper's designs can be measured on MI355X.
//
// k-NN (n points, g landmarks, k neighbours; output sorted by (distance, index)):
//   Base        one thread per point; every distance from global memory; the
//               k-array updated by an insertion step from its end.
//   Shared      the same, landmarks staged in LDS tile by tile.
//   GridInsert  a block stages h points and w landmarks, computes the h x w
//               distances cooperatively into LDS, then h threads insert them.
//   Bitonic     k threads per point: a sorted block of the k best and a block
//               of k new distances in LDS; each round sorts the new block
//               (bitonic sort), keeps the k smaller of the two blocks with one
//               comparator stage (best[i] vs new[k-1-i]) and re-sorts them
//               with a bitonic merge.
// Projection (scores, the k (k-1) / 2 segment projections, 2x2 Cramer):
//   Base        one thread per point, everything from global memory.
//   Shared      a block per point: neighbours' rows, distances, scores and
//               2-D positions in LDS; threads share out the pairs and add into
//               private 2x3 accumulators, reduced at the end.
//   Aligned     Shared with rows padded to 16 bytes and float4 transfers.
//   Registers   Aligned with each thread taking a 2 x 2 group of pairs, so
//               every float4 loaded from LDS serves two pairs.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "esom_internal.h"

namespace esom {

__device__ __forceinline__ bool ab_before(float da, int ia, float db, int ib) {
    return da < db || (da == db && ia < ib);
}

// Insertion step from the end of a sorted array of m (distance, index).
__device__ __forceinline__ void ab_insert(float *kd, int *ki, int m, float dv, int iv) {
    if (!ab_before(dv, iv, kd[m - 1], ki[m - 1])) return;
    int pos = m - 1;
    while (pos > 0 && ab_before(dv, iv, kd[pos - 1], ki[pos - 1])) {
        kd[pos] = kd[pos - 1];
        ki[pos] = ki[pos - 1];
        --pos;
    }
    kd[pos] = dv;
    ki[pos] = iv;
}

// ---------------------------------------------------------------- k-NN Base / Shared

template <bool SHARED>
__global__ void __launch_bounds__(256) ab_knn_insert(const float *__restrict__ X, int64_t n, int d,
                                                     const float *__restrict__ L, int g, int k,
                                                     int32_t *__restrict__ oidx, float *__restrict__ od2) {
    extern __shared__ float tileL[];  // SHARED: a tile of landmarks, tile x d
    float kd[ABL_MAX_K];
    int ki[ABL_MAX_K];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    for (int q = 0; q < k; ++q) {
        kd[q] = INFINITY;
        ki[q] = INT32_MAX;
    }
    const float *x = X + (live ? i : 0) * d;
    const int tile = SHARED ? (int)(ABL_LDS_FLOATS / d) : g;
    for (int j0 = 0; j0 < g; j0 += tile) {
        const int nt = g - j0 < tile ? g - j0 : tile;
        if constexpr (SHARED) {
            __syncthreads();
            for (int e = threadIdx.x; e < nt * d; e += blockDim.x) tileL[e] = L[(size_t)j0 * d + e];
            __syncthreads();
        }
        if (!live) continue;
        for (int j = 0; j < nt; ++j) {
            const float *Lj = SHARED ? tileL + (size_t)j * d : L + (size_t)(j0 + j) * d;
            float s = 0.f;
            for (int t = 0; t < d; ++t) {
                const float df = x[t] - Lj[t];
                s = fmaf(df, df, s);
            }
            ab_insert(kd, ki, k, s, j0 + j);
        }
    }
    if (!live) return;
    for (int q = 0; q < k; ++q) {
        oidx[i * k + q] = ki[q];
        od2[i * k + q] = kd[q];
    }
}

// ---------------------------------------------------------------- k-NN GridInsert

// h = blockDim.x points per block (one inserting thread each), w landmarks per
// epoch; all threads compute the h x w distances of an epoch.
__global__ void __launch_bounds__(256) ab_knn_grid(const float *__restrict__ X, int64_t n, int d,
                                                   const float *__restrict__ L, int g, int k, int w,
                                                   int32_t *__restrict__ oidx, float *__restrict__ od2) {
    extern __shared__ float gsm[];
    const int h = blockDim.x;
    float *xs = gsm;                 // h x d points
    float *ls = xs + (size_t)h * d;  // w x d landmarks
    float *ds = ls + (size_t)w * d;  // h x w distances
    float kd[ABL_MAX_K];
    int ki[ABL_MAX_K];
    for (int q = 0; q < k; ++q) {
        kd[q] = INFINITY;
        ki[q] = INT32_MAX;
    }
    const int64_t i0 = (int64_t)blockIdx.x * h;
    for (int e = threadIdx.x; e < h * d; e += blockDim.x) {
        const int64_t r = i0 + e / d;
        xs[e] = r < n ? X[r * d + e % d] : 0.f;
    }
    for (int j0 = 0; j0 < g; j0 += w) {
        const int nt = g - j0 < w ? g - j0 : w;
        __syncthreads();
        for (int e = threadIdx.x; e < nt * d; e += blockDim.x) ls[e] = L[(size_t)j0 * d + e];
        __syncthreads();
        for (int e = threadIdx.x; e < h * nt; e += blockDim.x) {
            const int p = e / nt, j = e % nt;
            float s = 0.f;
            for (int t = 0; t < d; ++t) {
                const float df = xs[p * d + t] - ls[j * d + t];
                s = fmaf(df, df, s);
            }
            ds[p * w + j] = s;
        }
        __syncthreads();
        for (int j = 0; j < nt; ++j) ab_insert(kd, ki, k, ds[threadIdx.x * w + j], j0 + j);
    }
    const int64_t i = i0 + threadIdx.x;
    if (i >= n) return;
    for (int q = 0; q < k; ++q) {
        oidx[i * k + q] = ki[q];
        od2[i * k + q] = kd[q];
    }
}

// ---------------------------------------------------------------- k-NN Bitonic

// Compare-exchange of entries a < b of a block (ascending when up).
__device__ __forceinline__ void ab_cx(float *bd, int *bi, int a, int b, bool up) {
    const float da = bd[a], db = bd[b];
    const int ia = bi[a], ib = bi[b];
    const bool swap = up ? ab_before(db, ib, da, ia) : ab_before(da, ia, db, ib);
    if (swap) {
        bd[a] = db;
        bd[b] = da;
        bi[a] = ib;
        bi[b] = ia;
    }
}

// KB threads (KB = k rounded up to a power of two) per point, blockDim.x / KB
// points per block.  Per point, LDS holds best[KB] and fresh[KB].
__global__ void __launch_bounds__(256) ab_knn_bitonic(const float *__restrict__ X, int64_t n, int d,
                                                      const float *__restrict__ L, int g, int k, int KB,
                                                      int32_t *__restrict__ oidx, float *__restrict__ od2) {
    extern __shared__ float bsm[];
    const int per = blockDim.x / KB;
    const int slot = threadIdx.x / KB, t = threadIdx.x % KB;
    float *bestd = bsm + (size_t)slot * 4 * KB;
    int *besti = reinterpret_cast<int *>(bestd + KB);
    float *newd = bestd + 2 * KB;
    int *newi = reinterpret_cast<int *>(bestd + 3 * KB);
    const int64_t i = (int64_t)blockIdx.x * per + slot;
    const bool live = i < n;
    const float *x = X + (live ? i : 0) * d;
    bestd[t] = INFINITY;
    besti[t] = INT32_MAX;
    for (int j0 = 0; j0 < g; j0 += KB) {
        // a block of KB fresh distances (one per thread)
        const int j = j0 + t;
        float s = INFINITY;
        if (live && j < g) {
            const float *Lj = L + (size_t)j * d;
            s = 0.f;
            for (int q = 0; q < d; ++q) {
                const float df = x[q] - Lj[q];
                s = fmaf(df, df, s);
            }
        }
        newd[t] = s;
        newi[t] = j < g ? j : INT32_MAX;
        __syncthreads();
        // bitonic sort of the fresh block, ascending
        for (int size = 2; size <= KB; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                const int partner = t ^ stride;
                if (partner > t) ab_cx(newd, newi, t, partner, (t & size) == 0);
                __syncthreads();
            }
        }
        // keep the KB smaller of best (ascending) and fresh (ascending): the
        // pairwise minima of best[i] and fresh[KB-1-i] are those, as a bitonic
        // sequence
        if (t < KB / 2) {
            const int a = t, b = KB - 1 - t;
            // two comparators per thread (entries a and b of best)
            float d0 = bestd[a], d1 = newd[b];
            int i0 = besti[a], i1 = newi[b];
            if (ab_before(d1, i1, d0, i0)) {
                bestd[a] = d1;
                besti[a] = i1;
            }
            float e0 = bestd[b], e1 = newd[a];
            int k0 = besti[b], k1 = newi[a];
            if (ab_before(e1, k1, e0, k0)) {
                bestd[b] = e1;
                besti[b] = k1;
            }
        }
        __syncthreads();
        // bitonic merge of the best block back to ascending order
        for (int stride = KB >> 1; stride > 0; stride >>= 1) {
            const int partner = t ^ stride;
            if (partner > t) ab_cx(bestd, besti, t, partner, true);
            __syncthreads();
        }
    }
    if (live && t < k) {
        oidx[i * k + t] = besti[t];
        od2[i * k + t] = bestd[t];
    }
}

hipError_t launch_ablation_knn(int algo, const float *X, int64_t n, int d, const float *L, int g, int k,
                               int32_t *idx, float *d2, hipStream_t s) {
    if (algo == 0 || algo == 1) {
        const unsigned blocks = (unsigned)((n + 255) / 256);
        if (algo == 0)
            hipLaunchKernelGGL(ab_knn_insert<false>, dim3(blocks), dim3(256), 0, s, X, n, d, L, g, k, idx, d2);
        else
            hipLaunchKernelGGL(ab_knn_insert<true>, dim3(blocks), dim3(256), ABL_LDS_FLOATS * sizeof(float), s,
                               X, n, d, L, g, k, idx, d2);
    } else if (algo == 2) {
        // h = 64 points (one wavefront inserting); w landmarks per epoch, at most
        // 128 and as many as a 64 KB block holds (h x d points, w x d
        // landmarks, h x w distances)
        const int h = 64;
        int w = (int)((16384 - (long long)h * d) / (d + h));
        if (w > 128) w = 128;
        if (w < 1) return hipErrorInvalidValue;
        const size_t smem = sizeof(float) * ((size_t)(h + w) * d + (size_t)h * w);
        const unsigned blocks = (unsigned)((n + h - 1) / h);
        hipLaunchKernelGGL(ab_knn_grid, dim3(blocks), dim3(h), smem, s, X, n, d, L, g, k, w, idx, d2);
    } else {
        int KB = 2;  // the merge needs two entries per block
        while (KB < k) KB <<= 1;
        const int threads = 256 >= KB ? 256 : KB;
        const int per = threads / KB;
        const size_t smem = sizeof(float) * 4 * (size_t)KB * per;
        const unsigned blocks = (unsigned)((n + per - 1) / per);
        hipLaunchKernelGGL(ab_knn_bitonic, dim3(blocks), dim3(threads), smem, s, X, n, d, L, g, k, KB, idx, d2);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- projection

struct AbProj {
    const float *X, *L, *l2d;
    const int32_t *idx;
    const float *d2;
    int64_t n;
    int d, g, k, dpad;
    float boost, cutoff, gravity, adjust, Wk;
    int use_cutoff;
    float *out;
};

// Scores of k sorted squared distances (FP32; degenerate -> all zero).
__device__ __forceinline__ bool ab_scores(const AbProj &a, const float *d2, float *s) {
    const int k = a.k;
    float mu = 0.f;
    for (int q = 0; q < k; ++q) mu += sqrtf(d2[q]) / (float)(q + 1);
    mu /= a.Wk;
    float var = 0.f;
    for (int q = 0; q < k; ++q) {
        const float e = sqrtf(d2[q]) - mu;
        var += e * e / (float)(q + 1);
    }
    var /= a.Wk;
    const float dk = sqrtf(d2[k - 1]);
    const bool degenerate = d2[0] == d2[k - 1];
    for (int q = 0; q < k; ++q) {
        const float dq = sqrtf(d2[q]);
        const float e = (var <= 1e-30f * mu * mu) ? 1.f : expf(a.boost * (mu - dq) / sqrtf(var));
        const float c = a.use_cutoff ? 1.f - expf(a.cutoff * (dq / dk - 1.f)) : 1.f;
        s[q] = degenerate ? 0.f : e * c;
    }
    return degenerate;
}

// One pair's contribution (u, v with scores su, sv) to the 2x3 system [M | r].
__device__ __forceinline__ void ab_pair(const AbProj &a, float HH, float xH, float2 lu, float2 lv, float su,
                                        float sv, float (&acc)[5]) {
    if (HH == 0.f) return;
    const float hx = lv.x - lu.x, hy = lv.y - lu.y;
    const float hh = hx * hx + hy * hy;
    if (hh == 0.f) return;
    const float q = su * sv * powf(hh, -a.adjust);
    const float D = xH / HH;
    const float rhs = D + (hx * lu.x + hy * lu.y) / hh;
    acc[0] += q * hx * hx / hh;
    acc[1] += q * hx * hy / hh;
    acc[2] += q * hy * hy / hh;
    acc[3] += q * hx * rhs;
    acc[4] += q * hy * rhs;
}

// Gravity, the 2x2 solve and the output of one point.
__device__ __forceinline__ void ab_solve(const AbProj &a, int64_t i, const int *nb, const float *s,
                                         bool degenerate, float (&acc)[5]) {
    float ssum = 0.f, cx = 0.f, cy = 0.f;
    for (int q = 0; q < a.k; ++q) {
        const float2 lq = reinterpret_cast<const float2 *>(a.l2d)[nb[q]];
        const float gs = a.gravity * s[q];
        acc[0] += gs;
        acc[2] += gs;
        acc[3] += gs * lq.x;
        acc[4] += gs * lq.y;
        ssum += s[q];
        cx += lq.x;
        cy += lq.y;
    }
    const float det = acc[0] * acc[2] - acc[1] * acc[1];
    const float htr = 0.5f * (acc[0] + acc[2]);
    float2 p;
    if (degenerate || ssum == 0.f || !(det > 1e-9f * htr * htr))
        p = make_float2(cx / a.k, cy / a.k);
    else
        p = make_float2((acc[3] * acc[2] - acc[1] * acc[4]) / det, (acc[0] * acc[4] - acc[1] * acc[3]) / det);
    reinterpret_cast<float2 *>(a.out)[i] = p;
}

// Base: one thread per point.
__global__ void __launch_bounds__(256) ab_proj_base(AbProj a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    float d2[ABL_MAX_K], s[ABL_MAX_K];
    int nb[ABL_MAX_K];
    for (int q = 0; q < a.k; ++q) {
        // indices outside [0, g) are a caller error; clamped so that no load leaves L
        nb[q] = min(max(a.idx[i * a.k + q], 0), a.g - 1);
        d2[q] = a.d2[i * a.k + q];
    }
    const bool degenerate = ab_scores(a, d2, s);
    float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    const float *x = a.X + i * a.d;
    if (!degenerate) {
        for (int p = 0; p < a.k; ++p) {
            const float *Lu = a.L + (size_t)nb[p] * a.d;
            const float2 lu = reinterpret_cast<const float2 *>(a.l2d)[nb[p]];
            for (int q = p + 1; q < a.k; ++q) {
                const float *Lv = a.L + (size_t)nb[q] * a.d;
                float HH = 0.f, xH = 0.f;
                for (int t = 0; t < a.d; ++t) {
                    const float H = Lv[t] - Lu[t];
                    HH = fmaf(H, H, HH);
                    xH = fmaf(x[t] - Lu[t], H, xH);
                }
                ab_pair(a, HH, xH, lu, reinterpret_cast<const float2 *>(a.l2d)[nb[q]], s[p], s[q], acc);
            }
        }
    }
    ab_solve(a, i, nb, s, degenerate, acc);
}

// Block-per-point variants.  LDS: the point (dpad floats), the k rows (k x
// dpad), the sorted neighbours' indices, scores and 2-D positions, and the
// per-thread accumulators for the reduction.  MODE 0: Shared (scalar
// accesses, stride d), 1: Aligned (float4, stride dpad), 2: Registers
// (Aligned, 2 x 2 pair groups).
template <int MODE>
__global__ void __launch_bounds__(256) ab_proj_block(AbProj a) {
    extern __shared__ __align__(16) float psm[];
    const int k = a.k;
    const int st = MODE == 0 ? a.d : a.dpad;
    float *xs = psm;                      // dpad
    float *rows = xs + a.dpad;            // k x st
    float *ss = rows + (size_t)k * st;    // k scores
    float *dd = ss + ABL_MAX_K;           // k squared distances
    int *nb = reinterpret_cast<int *>(dd + ABL_MAX_K);  // k indices
    float *red = reinterpret_cast<float *>(nb + ABL_MAX_K);  // 5 x blockDim.x
    for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
        __syncthreads();
        for (int q = threadIdx.x; q < k; q += blockDim.x) {
            nb[q] = min(max(a.idx[i * k + q], 0), a.g - 1);  // see ab_proj_base
            dd[q] = a.d2[i * k + q];
        }
        if constexpr (MODE == 0) {
            for (int e = threadIdx.x; e < a.d; e += blockDim.x) xs[e] = a.X[i * a.d + e];
        } else {
            for (int e = threadIdx.x; e < a.dpad; e += blockDim.x) xs[e] = e < a.d ? a.X[i * a.d + e] : 0.f;
        }
        __syncthreads();
        if constexpr (MODE == 0) {
            for (int e = threadIdx.x; e < k * a.d; e += blockDim.x)
                rows[e] = a.L[(size_t)nb[e / a.d] * a.d + e % a.d];
        } else {
            // padded rows, written as float4 (the source rows are read scalar:
            // their stride d need not be a multiple of 4)
            const int q4 = a.dpad / 4;
            for (int e = threadIdx.x; e < k * q4; e += blockDim.x) {
                const int r = e / q4, c = 4 * (e % q4);
                const float *src = a.L + (size_t)nb[r] * a.d;
                float4 v;
                v.x = c < a.d ? src[c] : 0.f;
                v.y = c + 1 < a.d ? src[c + 1] : 0.f;
                v.z = c + 2 < a.d ? src[c + 2] : 0.f;
                v.w = c + 3 < a.d ? src[c + 3] : 0.f;
                reinterpret_cast<float4 *>(rows + (size_t)r * st)[c / 4] = v;
            }
        }
        if (threadIdx.x == 0) {
            float s[ABL_MAX_K];
            const bool degenerate = ab_scores(a, dd, s);
            for (int q = 0; q < k; ++q) ss[q] = degenerate ? -1.f : s[q];
        }
        __syncthreads();
        const bool degenerate = k > 0 && ss[0] < 0.f;
        float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        if (!degenerate) {
            auto pair_from_rows = [&](int p, int q) {
                const float *Lu = rows + (size_t)p * st, *Lv = rows + (size_t)q * st;
                float HH = 0.f, xH = 0.f;
                if constexpr (MODE == 0) {
                    for (int t = 0; t < a.d; ++t) {
                        const float H = Lv[t] - Lu[t];
                        HH = fmaf(H, H, HH);
                        xH = fmaf(xs[t] - Lu[t], H, xH);
                    }
                } else {
                    for (int t = 0; t < a.dpad / 4; ++t) {
                        const float4 u4 = reinterpret_cast<const float4 *>(Lu)[t];
                        const float4 v4 = reinterpret_cast<const float4 *>(Lv)[t];
                        const float4 x4 = reinterpret_cast<const float4 *>(xs)[t];
                        const float h0 = v4.x - u4.x, h1 = v4.y - u4.y, h2 = v4.z - u4.z, h3 = v4.w - u4.w;
                        HH = fmaf(h0, h0, fmaf(h1, h1, fmaf(h2, h2, fmaf(h3, h3, HH))));
                        xH = fmaf(x4.x - u4.x, h0, fmaf(x4.y - u4.y, h1, fmaf(x4.z - u4.z, h2,
                                                                           fmaf(x4.w - u4.w, h3, xH))));
                    }
                }
                ab_pair(a, HH, xH, reinterpret_cast<const float2 *>(a.l2d)[nb[p]],
                        reinterpret_cast<const float2 *>(a.l2d)[nb[q]], ss[p], ss[q], acc);
            };
            if constexpr (MODE <= 1) {
                const int np = k * (k - 1) / 2;
                for (int pp = threadIdx.x; pp < np; pp += blockDim.x) {
                    // pair pp in row order: (0,1) .. (0,k-1), (1,2) ..
                    int p = 0, rem = pp;
                    while (rem >= k - 1 - p) {
                        rem -= k - 1 - p;
                        ++p;
                    }
                    pair_from_rows(p, p + 1 + rem);
                }
            } else {
                // 2 x 2 groups: rows {2a, 2a+1} x columns {2b, 2b+1} with
                // 2b >= 2a (each unordered pair once, p < q); one float4 of each
                // of the four rows serves the four pairs
                const int kh = (k + 1) / 2;
                const int ng = kh * (kh + 1) / 2;
                for (int gg = threadIdx.x; gg < ng; gg += blockDim.x) {
                    int ga = 0, rem = gg;
                    while (rem >= kh - ga) {
                        rem -= kh - ga;
                        ++ga;
                    }
                    const int gb = ga + rem;
                    const int p0 = 2 * ga, q0 = 2 * gb;
                    float HH[2][2] = {{0.f, 0.f}, {0.f, 0.f}}, xH[2][2] = {{0.f, 0.f}, {0.f, 0.f}};
                    const bool use[2][2] = {{p0 < q0 && q0 < k, p0 < q0 + 1 && q0 + 1 < k},
                                            {p0 + 1 < q0 && p0 + 1 < k && q0 < k,
                                             p0 + 1 < q0 + 1 && p0 + 1 < k && q0 + 1 < k}};
                    const int pr[2] = {p0, p0 + 1 < k ? p0 + 1 : p0};
                    const int qr[2] = {q0 < k ? q0 : 0, q0 + 1 < k ? q0 + 1 : 0};
                    for (int t = 0; t < a.dpad / 4; ++t) {
                        const float4 x4 = reinterpret_cast<const float4 *>(xs)[t];
                        float4 u4[2], v4[2];
                        for (int r = 0; r < 2; ++r) {
                            u4[r] = reinterpret_cast<const float4 *>(rows + (size_t)pr[r] * st)[t];
                            v4[r] = reinterpret_cast<const float4 *>(rows + (size_t)qr[r] * st)[t];
                        }
                        for (int r = 0; r < 2; ++r)
                            for (int c = 0; c < 2; ++c) {
                                const float h0 = v4[c].x - u4[r].x, h1 = v4[c].y - u4[r].y;
                                const float h2 = v4[c].z - u4[r].z, h3 = v4[c].w - u4[r].w;
                                HH[r][c] = fmaf(h0, h0, fmaf(h1, h1, fmaf(h2, h2, fmaf(h3, h3, HH[r][c]))));
                                xH[r][c] = fmaf(x4.x - u4[r].x, h0,
                                                fmaf(x4.y - u4[r].y, h1,
                                                     fmaf(x4.z - u4[r].z, h2, fmaf(x4.w - u4[r].w, h3, xH[r][c]))));
                            }
                    }
                    for (int r = 0; r < 2; ++r)
                        for (int c = 0; c < 2; ++c)
                            if (use[r][c])
                                ab_pair(a, HH[r][c], xH[r][c], reinterpret_cast<const float2 *>(a.l2d)[nb[pr[r]]],
                                        reinterpret_cast<const float2 *>(a.l2d)[nb[qr[c]]], ss[pr[r]], ss[qr[c]],
                                        acc);
                }
            }
        }
        // reduction of the private accumulators (wave shuffles, then LDS)
        for (int c = 0; c < 5; ++c) {
            float v = acc[c];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if ((threadIdx.x & 63) == 0) red[c * 4 + (threadIdx.x >> 6)] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            float tot[5];
            for (int c = 0; c < 5; ++c) {
                tot[c] = 0.f;
                for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot[c] += red[c * 4 + w];
            }
            float s[ABL_MAX_K];
            for (int q = 0; q < k; ++q) s[q] = degenerate ? 0.f : ss[q];
            ab_solve(a, i, nb, s, degenerate, tot);
        }
    }
}

hipError_t launch_ablation_project(int algo, const AbProjArgs &p, int num_cus, hipStream_t s) {
    AbProj a;
    a.X = p.X;
    a.L = p.L;
    a.l2d = p.l2d;
    a.idx = p.idx;
    a.d2 = p.d2;
    a.n = p.n;
    a.d = p.d;
    a.g = p.g;
    a.k = p.k;
    a.dpad = 4 * ((p.d + 3) / 4);
    a.boost = p.boost;
    a.cutoff = p.cutoff;
    a.gravity = p.gravity;
    a.adjust = p.adjust;
    a.Wk = p.Wk;
    a.use_cutoff = p.k < p.g ? 1 : 0;
    a.out = p.out;
    if (algo == 0) {
        hipLaunchKernelGGL(ab_proj_base, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    // block size by k (the paper found 8 .. 128 threads best): one wavefront
    // up to k = 16, two above
    const int threads = p.k <= 16 ? 64 : 128;
    const int st = algo == 1 ? p.d : a.dpad;
    const size_t smem = sizeof(float) * ((size_t)a.dpad + (size_t)p.k * st + 3 * ABL_MAX_K + 5 * 4);
    long long blocks = p.n < (long long)num_cus * 16 ? p.n : (long long)num_cus * 16;
    if (blocks < 1) blocks = 1;
    if (algo == 1)
        hipLaunchKernelGGL(ab_proj_block<0>, dim3((unsigned)blocks), dim3(threads), smem, s, a);
    else if (algo == 2)
        hipLaunchKernelGGL(ab_proj_block<1>, dim3((unsigned)blocks), dim3(threads), smem, s, a);
    else
        hipLaunchKernelGGL(ab_proj_block<2>, dim3((unsigned)blocks), dim3(threads), smem, s, a);
    return hipGetLastError();
}

}  // namespace esom
