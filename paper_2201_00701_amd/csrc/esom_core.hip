// Landmark preparation, the exact FP64 path, and kernel launchers.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "embed_kernel.h"
#include "esom_internal.h"

namespace esom {

// ---------------------------------------------------------------- preparation

// Landmark order.  The screen tiles, the rescoring rows and the pair table
// hold the landmarks in an order where landmarks close in the input space
// get nearby positions: a point's candidates then fill fewer bitmap words,
// and the pair-table entries of its neighbours share cache lines.  The
// order: P = min(64, g) pivots (landmarks floor(i g / P)); each landmark
// joins its nearest pivot; the pivots are chained greedily from pivot 0 (each
// next pivot the nearest one not yet taken); landmarks are sorted by (their
// pivot's place in the chain, distance to the pivot, index).  Only speed
// depends on it: results follow the landmark indices, which the keys carry.
constexpr int ORDER_MAX_P = 64;
constexpr int ASSIGN_PER_BLOCK = 16;  // landmarks per assignment block

// Wavefront minimum of an unsigned value (device library, DPP reduction).
extern "C" __device__ unsigned int __ockl_wfred_min_u32(unsigned int);

__host__ __device__ inline int order_pivots(int g) { return g < ORDER_MAX_P ? g : ORDER_MAX_P; }

// Centroid of the landmarks (FP64 sum, rounded to FP32), zero-padded to dp:
// blocks 0 .. dp-1, one per dimension.  Block 0 also resets the per-call
// fallback list and the landmark maxima (norm, BF16 quantisation error of the
// MFMA operand), and counts the points of this
// call.  Blocks dp .. : the landmarks' nearest pivots (squared FP32
// distance; equal leading bits break to the lower pivot) into pcl[j] and
// that distance into pdist[j]; a pivot's wavefront also writes its row of
// pivot-to-pivot distances into pp.
__global__ void prep_centroid(const float *__restrict__ L, int g, int d, int dp,
                              float *__restrict__ cent, float *__restrict__ lmax,
                              unsigned long long *__restrict__ counters, long long n_points,
                              int *__restrict__ pcl, float *__restrict__ pdist,
                              float *__restrict__ pp) {
    __shared__ double red[256];
    if ((int)blockIdx.x >= dp) {
        // pivot rows staged transposed (dimension-major: lanes read
        // consecutive words), then ASSIGN_PER_BLOCK landmarks, one per
        // wavefront at a time, lane = pivot
        extern __shared__ float pvt[];  // d x 64
        const int P = order_pivots(g);
        for (int e = threadIdx.x; e < d * 64; e += blockDim.x) {
            const int q = e / 64, i = e % 64;
            pvt[e] = i < P ? L[(size_t)(((long long)i * g) / P) * d + q] : 0.f;
        }
        __syncthreads();
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int j0 = ((int)blockIdx.x - dp) * ASSIGN_PER_BLOCK;
        for (int j = j0 + wv; j < j0 + ASSIGN_PER_BLOCK && j < g; j += blockDim.x / 64) {
            const float *Lj = L + (size_t)j * d;
            float s = 0.f;
            for (int q = 0; q < d; ++q) {
                const float df = Lj[q] - pvt[q * 64 + lane];
                s = fmaf(df, df, s);
            }
            const float dd = lane < P ? s : INFINITY;
            {
                const int pi = (int)(((long long)j * P + g - 1) / g);  // the pivot j may be
                if (pi < P && (int)(((long long)pi * g) / P) == j && lane < P) pp[pi * P + lane] = dd;
            }
            // nearest pivot: wave minimum of (distance bits, low 6 bits = pivot)
            const unsigned kv = lane < P ? ((__float_as_uint(dd) & ~63u) | (unsigned)lane) : 0xffffffffu;
            const int best = (int)(__ockl_wfred_min_u32(kv) & 63u);
            if (lane == best) {
                pcl[j] = best;
                pdist[j] = dd;
            }
        }
        return;
    }
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
        lmax[0] = 0.f;
        lmax[1] = 0.f;
        lmax[2] = 0.f;
        lmax[3] = 0.f;
        counters[C_FB_LEN] = 0ull;
        counters[C_POINTS] += (unsigned long long)n_points;
    }
}

// One block orders the landmarks:
//  1. the pivot chain (pivot-to-pivot squared distances from the assignment
//     pass); a pivot's place is its step in the chain;
//  2. each landmark's key (place of its pivot, distance to it, index), 64 bits;
//  3. a counting sort by place (a histogram and its prefix sum), then each
//     landmark's position within its place by counting the smaller keys of
//     the same place only (about g / 64 of them).
// Writes perm (position -> landmark) and ipos (landmark -> position).
__global__ void __launch_bounds__(1024) prep_order(int g, const int *__restrict__ pcl,
                                                   const float *__restrict__ pdist,
                                                   const float *__restrict__ ppg,
                                                   int *__restrict__ perm, int *__restrict__ ipos) {
    extern __shared__ __align__(16) unsigned char osm[];
    const int P = order_pivots(g);
    unsigned long long *key = reinterpret_cast<unsigned long long *>(osm);  // g
    float *pp = reinterpret_cast<float *>(key + g);                          // P x P
    int *place = reinterpret_cast<int *>(pp + ORDER_MAX_P * ORDER_MAX_P);    // P
    int *cnt = place + ORDER_MAX_P;                                          // landmarks per place
    int *start = cnt + ORDER_MAX_P;                                          // first position of a place
    int *fill = start + ORDER_MAX_P;                                         // bucket fill counters
    int *bucket = fill + ORDER_MAX_P;                                        // g: landmarks by place
    const int tid = threadIdx.x;
    for (int e = tid; e < P * P; e += blockDim.x) pp[e] = ppg[e];
    if (tid < ORDER_MAX_P) {
        cnt[tid] = 0;
        fill[tid] = 0;
    }
    __syncthreads();
    // 1. greedy chain over the pivots (one wavefront, lane = pivot): each step
    // takes the nearest pivot not yet taken, by a wave minimum of 32-bit keys
    // (distance bits with the 6 low bits replaced by the pivot number)
    if (tid < 64) {
        bool taken = tid == 0;
        int cur = 0;
        if (tid == 0) place[0] = 0;
        for (int r = 1; r < P; ++r) {
            unsigned kv = 0xffffffffu;
            if (tid < P && !taken) kv = (__float_as_uint(fmaxf(pp[cur * P + tid], 0.f)) & ~63u) | (unsigned)tid;
            cur = (int)(__ockl_wfred_min_u32(kv) & 63u);
            if (tid == cur) taken = true;
            if (tid == 0) place[cur] = r;
        }
    }
    __syncthreads();
    // 2. keys: place (6 bits) | distance bits (31) | index (13); landmarks per place
    for (int j = tid; j < g; j += blockDim.x) {
        const int pl = place[pcl[j]];
        const unsigned db = __float_as_uint(fmaxf(pdist[j], 0.f)) & 0x7fffffffu;
        key[j] = ((unsigned long long)pl << 44) | ((unsigned long long)db << 13) | (unsigned long long)j;
        atomicAdd(&cnt[pl], 1);
    }
    __syncthreads();
    if (tid < 64) {
        // exclusive prefix sum over the places (P <= 64)
        int v = tid < P ? cnt[tid] : 0;
        int incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (tid >= o) incl += t;
        }
        if (tid < P) start[tid] = incl - v;
    }
    __syncthreads();
    // 3. buckets, then the rank within the bucket (keys are distinct)
    for (int j = tid; j < g; j += blockDim.x) {
        const int pl = (int)(key[j] >> 44);
        bucket[start[pl] + atomicAdd(&fill[pl], 1)] = j;
    }
    __syncthreads();
    for (int j = tid; j < g; j += blockDim.x) {
        const unsigned long long kj = key[j];
        const int pl = (int)(kj >> 44);
        const int b0 = start[pl], nb = cnt[pl];
        int pos = b0;
        for (int i = 0; i < nb; ++i) pos += key[bucket[b0 + i]] < kj ? 1 : 0;
        perm[pos] = j;
        ipos[j] = pos;
    }
}

// One wavefront per (padded) landmark, lanes over dimensions: centred row,
// squared norm (FP64 wave sum), MFMA operand entries, the zero-padded FP32
// copy for exact rescoring, and the norm maximum.
__device__ __forceinline__ void prep_landmarks(int blk, const float *__restrict__ L, const int *__restrict__ perm, int g,
                               int gpad, int d, int dp, int mode, const float *__restrict__ cent,
                               void *__restrict__ A, void *__restrict__ A16, float *__restrict__ norms,
                               float *__restrict__ Lpad, float *__restrict__ lmax, unsigned *wmax) {
    // wmax: 4 x (waves per block) words of LDS for the block's four maxima
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int j = blk * nw + wv;
    const int lane = threadIdx.x & 63;
    if (j >= gpad) {
        if (lane == 0) wmax[wv] = wmax[nw + wv] = wmax[2 * nw + wv] = wmax[3 * nw + wv] = 0u;
    } else {
        // Position j sits in tile pair j / 64, screen half j % 2, tile parity
        // (j / 32) % 2 and accumulator register (j / 2) % 16, so that bit b of a
        // candidate-bitmap word (16 parity + register) is position
        // 64 tile_pair + 2 b + half: the two halves of a point's screen
        // interleave, and each sees every other landmark of the order.  MFMA 32x32
        // output row m sits in lane half (m / 4) % 2, register 4 (m / 8) + m % 4.
        const int rr = (j / 2) % 16, hj = j % 2;
        const int t = 2 * (j / 64) + (j / 32) % 2, m = 8 * (rr >> 2) + 4 * hj + (rr & 3);
        const int dc = dp / 16;
        const bool real = j < g;
        const size_t src = real ? (size_t)perm[j] * d : 0;
        // |L_j - c|^2, |BF16 quantisation error of a = -2 (L_j - c)|^2, and for
        // the split a = ah + al + ra (ah = bf16(a), al = bf16(a - ah), both
        // differences exact in FP32) |al|^2 and |ra|^2
        double nrm = 0.0, qe = 0.0, le = 0.0, re = 0.0;
        for (int q = lane; q < dp; q += 64) {
            const float lv = (real && q < d) ? L[src + q] : 0.f;
            const float c = (real && q < d) ? lv - cent[q] : 0.f;
            nrm += (double)c * (double)c;
            if (real) Lpad[(size_t)j * dp + q] = lv;
            const float a2 = -2.f * c;
            {
                // A_bf16[t][c][lane = 32 h + m][e], dim = 16 c + 8 h + e: the
                // BF16 mode's high parts (A) and low parts (A16), or FP32
                // mode's threshold-pass operand (A16)
                const int cc = q / 16, hh = (q % 16) / 8, e = q % 8;
                const size_t at = (((size_t)t * dc + cc) * 64 + 32 * hh + m) * 8 + e;
                unsigned u = __float_as_uint(a2);
                u += 0x7FFFu + ((u >> 16) & 1u);
                const float ah = __uint_as_float(u & 0xFFFF0000u);
                const double qd = (double)ah - (double)a2;
                qe += qd * qd;
                reinterpret_cast<unsigned short *>(mode == 1 ? A : A16)[at] = (unsigned short)(u >> 16);
                if (mode == 1) {
                    const float r1 = a2 - ah;
                    unsigned v = __float_as_uint(r1);
                    v += 0x7FFFu + ((v >> 16) & 1u);
                    const float al = __uint_as_float(v & 0xFFFF0000u);
                    le += (double)al * (double)al;
                    re += (double)(r1 - al) * (double)(r1 - al);
                    reinterpret_cast<unsigned short *>(A16)[at] = (unsigned short)(v >> 16);
                }
            }
            if (mode == 0) {
                // A_f32[t][s][lane = 32 h + m], dim = 2 s + h
                const int s = q / 2, hh = q % 2;
                reinterpret_cast<float *>(A)[((size_t)t * (dp / 2) + s) * 64 + 32 * hh + m] = a2;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            nrm += __shfl_xor(nrm, o);
            qe += __shfl_xor(qe, o);
            le += __shfl_xor(le, o);
            re += __shfl_xor(re, o);
        }
        if (lane == 0) {
            norms[((size_t)t * 2 + hj) * 16 + rr] = real ? (float)nrm : INFINITY;
            // non-negative floats: integer order is float order
            wmax[wv] = real ? __float_as_uint((float)sqrt(nrm) * 1.0000002f) : 0u;
            wmax[nw + wv] = real ? __float_as_uint((float)sqrt(qe) * 1.0000002f) : 0u;
            wmax[2 * nw + wv] = real ? __float_as_uint((float)sqrt(le) * 1.0000002f) : 0u;
            wmax[3 * nw + wv] = real ? __float_as_uint((float)sqrt(re) * 1.0000002f) : 0u;
        }
    }
    // one atomic per block and maximum (the landmark blocks all update the
    // same four words)
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned mv = 0u;
        for (int w = 0; w < nw; ++w) mv = max(mv, wmax[threadIdx.x * nw + w]);
        if (mv) atomicMax(reinterpret_cast<unsigned *>(lmax) + threadIdx.x, mv);
    }
}

// Pair table pairs[u][v] = 1 / (2 |L_u - L_v|^2), the high-dimensional factor
// of the segment coordinate (Section "Projection step": the projection of a
// point onto the segment between two landmarks), from FP64 differences, 0
// when the two landmarks coincide; indexed by landmark positions.  Each entry
// depends only on the two landmarks, so the per-point pair loop needs no
// division and the table serves any 2-D positions; it is exactly symmetric
// (the same FP64 sums either way).  The 2-D factor 1 / |l_v - l_u|^2 is
// formed in the pair loop instead: a second table entry made every pair's
// load 8 bytes, and at 1024 landmarks the table (8 MB) no longer stayed in a
// die's L2.  A 256-thread block computes a 16 x 16 tile of pairs from the two
// 16-row slices of L staged in LDS (row stride d + 1 floats: no bank conflicts
// between the 16 rows a wave reads); rows are read and the table written
// coalesced.
constexpr int PAIR_TILE = 16;

__device__ __forceinline__ void prep_pairs(int blk, float *prs, const float *__restrict__ L,
                                           const int *__restrict__ perm, int g, int d,
                                           float *__restrict__ pairs) {
    // prs: 2 x PAIR_TILE x (d + 1) floats of LDS
    const int ntu = (g + PAIR_TILE - 1) / PAIR_TILE;
    const int u0 = (blk / ntu) * PAIR_TILE, v0 = (blk % ntu) * PAIR_TILE;
    const int rs = d + 1;
    float *Lu = prs, *Lv = prs + PAIR_TILE * rs;
    for (int e = threadIdx.x; e < PAIR_TILE * d; e += blockDim.x) {
        const int r = e / d, q = e % d;
        Lu[r * rs + q] = u0 + r < g ? L[(size_t)perm[u0 + r] * d + q] : 0.f;
        Lv[r * rs + q] = v0 + r < g ? L[(size_t)perm[v0 + r] * d + q] : 0.f;
    }
    __syncthreads();
    const int ty = threadIdx.x / PAIR_TILE, tx = threadIdx.x % PAIR_TILE;
    const int u = u0 + ty, v = v0 + tx;
    if (u >= g || v >= g) return;
    double s = 0.0;
    for (int q = 0; q < d; ++q) {
        const double df = (double)Lv[tx * rs + q] - (double)Lu[ty * rs + q];
        s = fma(df, df, s);
    }
    // FP32 reciprocal (about 1 ulp): the fast kernel uses it in FP32
    pairs[(size_t)u * g + v] = s > 0.0 ? 0.5f * __builtin_amdgcn_rcpf((float)s) : 0.f;
}

// The landmark tables and the pair table in one launch: blocks 0 .. nlb-1
// prepare 4 landmarks each, the others one 16 x 16 tile of pairs each.
__global__ void __launch_bounds__(256) prep_tables(const float *__restrict__ L, const int *__restrict__ perm,
                                                   int g, int gpad, int d, int dp, int mode, int nlb,
                                                   const float *__restrict__ cent, void *__restrict__ A,
                                                   void *__restrict__ A16,
                                                   float *__restrict__ norms, float *__restrict__ Lpad,
                                                   float *__restrict__ lmax, float *__restrict__ pairs) {
    extern __shared__ __align__(16) float prs[];
    if ((int)blockIdx.x < nlb)
        prep_landmarks((int)blockIdx.x, L, perm, g, gpad, d, dp, mode, cent, A, A16, norms, Lpad, lmax,
                       reinterpret_cast<unsigned *>(prs));
    else
        prep_pairs((int)blockIdx.x - nlb, prs, L, perm, g, d, pairs);
}

hipError_t launch_prep(const Prep &P, const float *L, int mode,
                       unsigned long long *counters, long long n_points, hipStream_t s) {
    hipLaunchKernelGGL(prep_centroid, dim3(P.dp + (P.g + ASSIGN_PER_BLOCK - 1) / ASSIGN_PER_BLOCK),
                       dim3(256), sizeof(float) * P.d * 64, s, L, P.g, P.d, P.dp, P.cent, P.lmax, counters,
                       n_points, P.pcl, P.pdist, P.ppiv);
    const size_t osm = sizeof(unsigned long long) * P.g + sizeof(float) * ORDER_MAX_P * ORDER_MAX_P +
                       sizeof(int) * (4 * ORDER_MAX_P + P.g);
    hipLaunchKernelGGL(prep_order, dim3(1), dim3(1024), osm, s, P.g, P.pcl, P.pdist, P.ppiv, P.perm,
                       P.ipos);
    const int gpad = P.ntiles * TILE;
    const int nlb = (gpad + 3) / 4;
    const int ntu = P.need_pairs ? (P.g + PAIR_TILE - 1) / PAIR_TILE : 0;
    hipLaunchKernelGGL(prep_tables, dim3((unsigned)(nlb + ntu * ntu)), dim3(256),
                       sizeof(float) * 2 * PAIR_TILE * (P.d + 1), s, L, P.perm, P.g, gpad, P.d, P.dp, mode,
                       nlb, P.cent, P.A, P.A16, P.norms, P.Lpad, P.lmax, P.pairs);
    return hipGetLastError();
}

// ---------------------------------------------------------------- exact FP64 path

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Recomputes points exactly in FP64, one block of EX_THREADS per point (a
// point's latency sets the duration of the short lists the fast kernel
// leaves, so its work is spread over a block):
//  1. all g distances from FP64 differences into LDS; the landmarks within
//     the point's k-th distance bound (fb_thresh) are collected;
//  2. without a usable bound (none given, or too few or too many within it),
//     the k-th smallest of the threads' own minima bounds the k-th distance
//     (those minima belong to distinct landmarks), and the landmarks within
//     that bound are collected instead;
//  3. the k nearest by (distance, index): each collected landmark's rank is
//     counted against the others; only when too many remain collected does
//     one wavefront take k repeated (distance, index) minima over all g;
//  4. the scores (one neighbour per lane of wavefront 0); the neighbours'
//     rows and 2-D positions into LDS; every pair's segment projection from
//     the coordinates, spread over the threads; block sums;
//  5. Cramer's rule, or the centroid of the neighbours' 2-D positions for a
//     degenerate neighbourhood.
// all_points = 1 processes every point (shapes outside the fast kernels),
// otherwise the fast kernel's list.
constexpr int EX_THREADS = 256;
constexpr int EX_SEL_CAP = 256;  // collected landmarks ranked by counting

// LDS layout (byte offsets).
struct ExLayout {
    size_t nrow, dist, xs, cdist, seld, sc, nl2, red, tmin, bnd, cando, cpos, selj, selp, flags, bytes;
};

__host__ __device__ inline ExLayout ex_layout(int g, int dp, int k) {
    ExLayout L;
    size_t o = 0;
    L.nrow = o;  // k x dp floats: the neighbours' rows
    o += ((sizeof(float) * (size_t)k * dp) + 15) & ~(size_t)15;
    L.dist = o;  // g doubles
    o += sizeof(double) * (size_t)g;
    L.xs = o;  // dp doubles (zero beyond d)
    o += sizeof(double) * (size_t)dp;
    L.cdist = o;  // collected distances
    o += sizeof(double) * EX_SEL_CAP;
    L.seld = o;  // the k nearest: distances
    o += sizeof(double) * ESOM_MAX_K;
    L.sc = o;  // scores
    o += sizeof(double) * ESOM_MAX_K;
    L.nl2 = o;  // the neighbours' 2-D positions
    o += sizeof(double) * 2 * ESOM_MAX_K;
    L.red = o;  // block sums: 6 per wavefront
    o += sizeof(double) * 6 * (EX_THREADS / 64);
    L.tmin = o;  // the threads' minima
    o += sizeof(double) * EX_THREADS;
    L.bnd = o;  // bound from those minima
    o += sizeof(double) * 2;
    L.cando = o;  // collected landmark indices
    o += sizeof(int) * EX_SEL_CAP;
    L.cpos = o;  // collected landmark positions
    o += sizeof(int) * EX_SEL_CAP;
    L.selj = o;  // the k nearest: landmark indices
    o += sizeof(int) * ESOM_MAX_K;
    L.selp = o;  // the k nearest: positions
    o += sizeof(int) * ESOM_MAX_K;
    L.flags = o;  // [0] collected count, [1] no k finite distances
    o += sizeof(int) * 4;
    L.bytes = (o + 15) & ~(size_t)15;
    return L;
}

__device__ __forceinline__ bool lex_less(double a, int ia, double b, int ib) {
    return a < b || (a == b && ia < ib);
}

// Score of a neighbour at distance dl (Section 3: the rank-weighted mean mu
// and variance var of the k distances, the boost exponent, and the cutoff
// factor relative to the k-th distance dlk).  Not inlined: the FP64
// exponentials would otherwise raise the register count of the whole kernel.
__device__ __noinline__ double exact_score(double dl, double dlk, double mu, double var, bool flat,
                                           float boost, float cutoff, int use_cutoff) {
    const double ev = flat ? 1.0 : exp((double)boost * (mu - dl) / sqrt(var));
    const double cv = use_cutoff ? 1.0 - exp((double)cutoff * (dl / dlk - 1.0)) : 1.0;
    return ev * cv;
}

// x^y, not inlined for the same reason.
__device__ __noinline__ double exact_pow(double x, double y) { return pow(x, y); }

__global__ void __launch_bounds__(EX_THREADS) embed_exact(EmbedArgs a, int all_points) {
    extern __shared__ __align__(16) unsigned char esm[];
    const int k = a.k;
    const int g = a.g;
    const int dq = a.dp / 4;  // float4 per row (dp is a multiple of 16)
    const ExLayout Lo = ex_layout(g, a.dp, k);
    float *nrow = reinterpret_cast<float *>(esm + Lo.nrow);
    double *dist = reinterpret_cast<double *>(esm + Lo.dist);
    double *xs = reinterpret_cast<double *>(esm + Lo.xs);
    double *cdist = reinterpret_cast<double *>(esm + Lo.cdist);
    double *sel_d = reinterpret_cast<double *>(esm + Lo.seld);
    double *sc = reinterpret_cast<double *>(esm + Lo.sc);
    double *nl2 = reinterpret_cast<double *>(esm + Lo.nl2);
    double *red = reinterpret_cast<double *>(esm + Lo.red);
    double *tmin = reinterpret_cast<double *>(esm + Lo.tmin);
    double *bnd = reinterpret_cast<double *>(esm + Lo.bnd);
    int *cando = reinterpret_cast<int *>(esm + Lo.cando);
    int *cpos = reinterpret_cast<int *>(esm + Lo.cpos);
    int *sel_j = reinterpret_cast<int *>(esm + Lo.selj);
    int *sel_p = reinterpret_cast<int *>(esm + Lo.selp);
    int *flags = reinterpret_cast<int *>(esm + Lo.flags);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const long long cnt = all_points
                              ? a.n
                              : (long long)min(a.counters[C_FB_LEN], (unsigned long long)a.n);
    unsigned long long n_fb = 0, n_unc = 0, n_tie = 0, n_ill = 0, n_deg = 0;
    // appends landmark position j (index o, distance s) to the collected list
    auto collect = [&](int j, int o, double s) {
        const int slot = atomicAdd(&flags[0], 1);
        if (slot < EX_SEL_CAP) {
            cdist[slot] = s;
            cando[slot] = o;
            cpos[slot] = j;
        }
    };
    for (long long e = blockIdx.x; e < cnt; e += gridDim.x) {
        const long long pi = all_points ? e : (long long)a.fb_list[e];
        const unsigned reason = all_points ? 0u : (unsigned)a.fb_reason[e];
        const double thr = all_points ? (double)INFINITY : (double)a.fb_thresh[e];
        ++n_fb;
        n_unc += (reason & R_UNCERT) ? 1 : 0;
        n_tie += (reason & R_NEARTIE) ? 1 : 0;
        n_ill += (reason & R_ILLCOND) ? 1 : 0;
        const float *xr = a.X + pi * a.ldx;
        for (int q = tid; q < a.dp; q += EX_THREADS) xs[q] = q < a.d ? (double)xr[q] : 0.0;
        if (tid == 0) {
            flags[0] = 0;
            flags[1] = 0;
            bnd[0] = NAN;
        }
        __syncthreads();
        // 1. distances (LDS and rows by landmark position); collect the
        // landmarks within the bound
        const bool use_thr = thr < INFINITY;
        double tm = INFINITY;
        for (int j = tid; j < g; j += EX_THREADS) {
            const int oj = a.perm[j];
            const float4 *Lj = reinterpret_cast<const float4 *>(a.Lpad + (size_t)j * a.dp);
            double s = 0.0;
            for (int q = 0; q < dq; q += 4) {
                float4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = Lj[q + u];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double *xq = xs + 4 * (q + u);
                    const double d0 = xq[0] - (double)v[u].x, d1 = xq[1] - (double)v[u].y;
                    const double d2 = xq[2] - (double)v[u].z, d3 = xq[3] - (double)v[u].w;
                    s = fma(d0, d0, s);
                    s = fma(d1, d1, s);
                    s = fma(d2, d2, s);
                    s = fma(d3, d3, s);
                }
            }
            dist[j] = s;
            tm = fmin(tm, s);
            if (use_thr && s <= thr) collect(j, oj, s);
        }
        __syncthreads();
        int nc = flags[0];
        // 2. no usable bound: the k-th smallest of the threads' minima (by
        // value, then thread) bounds the k-th distance; g >= k landmarks
        // spread over the threads give at least k finite minima
        if (!(nc >= k && nc <= EX_SEL_CAP)) {
            tmin[tid] = tm;
            __syncthreads();
            if (tid == 0) flags[0] = 0;
            int rank = 0;
#pragma unroll 8
            for (int o = 0; o < EX_THREADS; ++o) {
                const double v = tmin[o];
                rank += (v < tm || (v == tm && o < tid)) ? 1 : 0;
            }
            if (rank == k - 1) bnd[0] = tm;
            __syncthreads();
            const double b = bnd[0];  // NaN when distances are not finite: nothing collected
            for (int j = tid; j < g; j += EX_THREADS) {
                const double s = dist[j];
                if (s <= b) collect(j, a.perm[j], s);
            }
            __syncthreads();
            nc = flags[0];
        }
        // 3. the k nearest, sorted by (distance, index)
        if (nc >= k && nc <= EX_SEL_CAP) {
            for (int c = tid; c < nc; c += EX_THREADS) {
                const double dc = cdist[c];
                const int jc = cando[c];
                int rank = 0;
#pragma unroll 4
                for (int o = 0; o < nc; ++o) rank += lex_less(cdist[o], cando[o], dc, jc) ? 1 : 0;
                if (rank < k) {
                    sel_d[rank] = dc;
                    sel_j[rank] = jc;
                    sel_p[rank] = cpos[c];
                }
            }
        } else if (wv == 0) {
            // k repeated minima over all g; taken entries become NaN (never minimal)
            for (int r = 0; r < k; ++r) {
                double bv = INFINITY;
                int bj = 0x7fffffff, bp = 0;  // landmark index, its position
                for (int j = lane; j < g; j += 64) {
                    const double v = dist[j];
                    const int o = a.perm[j];
                    if (v < bv || (v == bv && o < bj)) {
                        bv = v;
                        bj = o;
                        bp = j;
                    }
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(bv, off);
                    const int oj = __shfl_xor(bj, off), op = __shfl_xor(bp, off);
                    if (ov < bv || (ov == bv && oj < bj)) {
                        bv = ov;
                        bj = oj;
                        bp = op;
                    }
                }
                if (lane == 0) {
                    sel_d[r] = bv;
                    sel_j[r] = bj;
                    sel_p[r] = bp;
                    if (bj != 0x7fffffff)
                        dist[bp] = NAN;
                    else
                        flags[1] = 1;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
        }
        __syncthreads();
        const bool bad = flags[1] != 0;
        // Neighbours of points listed only for the projection (ill-conditioned,
        // degenerate) were already certified by the fast kernel: keep its outputs.
        const bool hd_reason = all_points || (reason & (R_UNCERT | R_NEARTIE)) || a.knn_only;
        if (tid < k && hd_reason) {
            if (a.knn_idx) a.knn_idx[pi * k + tid] = bad ? -1 : sel_j[tid];
            if (a.knn_d2) a.knn_d2[pi * k + tid] = (float)sel_d[tid];
        }
        if (tid == 0 && a.knn_mark && hd_reason) a.knn_mark[pi] = 1;
        if (a.knn_only) {
            __syncthreads();
            continue;
        }
        if (bad) {
            if (tid == 0) {
                a.out[2 * pi] = NAN;
                a.out[2 * pi + 1] = NAN;
            }
            __syncthreads();
            continue;
        }
        // 4. scores (wavefront 0, one neighbour per lane; k <= 64)
        const bool degenerate = sqrt(sel_d[0]) == sqrt(sel_d[k - 1]);  // all delta equal
        if (wv == 0) {
            const double dl = lane < k ? sqrt(sel_d[lane]) : 0.0;
            const double wq = lane < k ? 1.0 / (lane + 1) : 0.0;
            const double W = wave_sum(wq);
            const double mu = wave_sum(wq * dl) / W;
            const double var = wave_sum(lane < k ? wq * (dl - mu) * (dl - mu) : 0.0) / W;
            const bool flat = !(var > 1e-30 * mu * mu);
            if (lane < k)
                sc[lane] = degenerate ? 0.0
                                      : exact_score(dl, sqrt(sel_d[k - 1]), mu, var, flat, a.boost,
                                                    a.cutoff, a.use_cutoff);
        }
        // the neighbours' rows and 2-D positions into LDS, then every pair's
        // projection from them, spread over the threads
        for (int e2 = tid; e2 < k * dq; e2 += EX_THREADS) {
            const int q = e2 / dq, c = e2 % dq;
            reinterpret_cast<float4 *>(nrow + (size_t)q * a.dp)[c] =
                reinterpret_cast<const float4 *>(a.Lpad + (size_t)sel_p[q] * a.dp)[c];
        }
        if (tid < 2 * k) nl2[tid] = a.l2d[2 * sel_j[tid >> 1] + (tid & 1)];
        __syncthreads();
        double M00 = 0.0, M01 = 0.0, M11 = 0.0, r0 = 0.0, r1 = 0.0, ssum = 0.0;
        const int npair = k * (k - 1) / 2;
        for (int p = tid; p < npair && !degenerate; p += EX_THREADS) {
            int qi = 0, rem = p;
            while (rem >= k - 1 - qi) {
                rem -= k - 1 - qi;
                ++qi;
            }
            const int qj = qi + 1 + rem;
            const float4 *Lu = reinterpret_cast<const float4 *>(nrow + (size_t)qi * a.dp);
            const float4 *Lv = reinterpret_cast<const float4 *>(nrow + (size_t)qj * a.dp);
            // padded dimensions are 0 in the rows and in xs
            double HH = 0.0, xH = 0.0;
            for (int q = 0; q < dq; ++q) {
                const float4 lu = Lu[q], lv = Lv[q];
                const double *xq = xs + 4 * q;
                const double H0 = (double)lv.x - (double)lu.x, H1 = (double)lv.y - (double)lu.y;
                const double H2 = (double)lv.z - (double)lu.z, H3 = (double)lv.w - (double)lu.w;
                HH = fma(H0, H0, HH);
                HH = fma(H1, H1, HH);
                HH = fma(H2, H2, HH);
                HH = fma(H3, H3, HH);
                xH = fma(xq[0] - (double)lu.x, H0, xH);
                xH = fma(xq[1] - (double)lu.y, H1, xH);
                xH = fma(xq[2] - (double)lu.z, H2, xH);
                xH = fma(xq[3] - (double)lu.w, H3, xH);
            }
            if (HH == 0.0) continue;
            const double D = xH / HH;
            const double lux = nl2[2 * qi], luy = nl2[2 * qi + 1];
            const double hx = nl2[2 * qj] - lux, hy = nl2[2 * qj + 1] - luy;
            const double hh = hx * hx + hy * hy;
            if (hh == 0.0) continue;
            const double qw = sc[qi] * sc[qj] * (a.adjust == 1.0f ? 1.0 / hh : exact_pow(hh, -(double)a.adjust));
            const double rhs = D + (hx * lux + hy * luy) / hh;
            M00 += qw * hx * hx / hh;
            M01 += qw * hx * hy / hh;
            M11 += qw * hy * hy / hh;
            r0 += qw * hx * rhs;
            r1 += qw * hy * rhs;
        }
        if (tid < k && !degenerate) {
            const double gs = (double)a.gravity * sc[tid];
            M00 += gs;
            M11 += gs;
            r0 += gs * nl2[2 * tid];
            r1 += gs * nl2[2 * tid + 1];
            ssum += sc[tid];
        }
        M00 = wave_sum(M00);
        M01 = wave_sum(M01);
        M11 = wave_sum(M11);
        r0 = wave_sum(r0);
        r1 = wave_sum(r1);
        ssum = wave_sum(ssum);
        if (lane == 0) {
            red[6 * wv + 0] = M00;
            red[6 * wv + 1] = M01;
            red[6 * wv + 2] = M11;
            red[6 * wv + 3] = r0;
            red[6 * wv + 4] = r1;
            red[6 * wv + 5] = ssum;
        }
        __syncthreads();
        // 5. solve
        if (tid == 0) {
            double t[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int w = 0; w < EX_THREADS / 64; ++w)
                for (int i = 0; i < 6; ++i) t[i] += red[6 * w + i];
            const double det = t[0] * t[2] - t[1] * t[1];
            const double htr = 0.5 * (t[0] + t[2]);
            double px, py;
            // numerically singular (a rank-deficient system, e.g. one pair and
            // no gravity, has det = 0 up to rounding of either sign): centroid
            if (degenerate || !(t[5] > 0.0) || !(det > SINGULAR_REL * htr * htr)) {
                double cx = 0.0, cy = 0.0;
                for (int q = 0; q < k; ++q) {
                    cx += nl2[2 * q];
                    cy += nl2[2 * q + 1];
                }
                px = cx / k;
                py = cy / k;
                ++n_deg;
            } else {
                px = (t[3] * t[2] - t[1] * t[4]) / det;
                py = (t[0] * t[4] - t[1] * t[3]) / det;
            }
            a.out[2 * pi] = (float)px;
            a.out[2 * pi + 1] = (float)py;
        }
        __syncthreads();
    }
    if (tid == 0 && n_fb) {
        atomicAdd(&a.counters[all_points ? C_SLOW : C_FALLBACK], n_fb);
        if (n_unc) atomicAdd(&a.counters[C_UNCERT], n_unc);
        if (n_tie) atomicAdd(&a.counters[C_NEARTIE], n_tie);
        if (n_ill) atomicAdd(&a.counters[C_ILLCOND], n_ill);
        if (n_deg) atomicAdd(&a.counters[C_DEGEN], n_deg);
    }
}

hipError_t launch_fallback(const EmbedArgs &a, int num_cus, size_t lds_per_block, hipStream_t s) {
    // The list length is only known on the device: a fixed grid loops over it.
    const size_t smem = ex_layout(a.g, a.dp, a.k).bytes;
    if (smem > lds_per_block) return hipErrorInvalidValue;
    hipLaunchKernelGGL(embed_exact, dim3(num_cus * 4), dim3(EX_THREADS), smem, s, a, 0);
    return hipGetLastError();
}

hipError_t launch_all_to_fallback(const EmbedArgs &a, int num_cus, size_t lds_per_block, hipStream_t s) {
    const size_t smem = ex_layout(a.g, a.dp, a.k).bytes;
    if (smem > lds_per_block) return hipErrorInvalidValue;
    long long blocks = a.n;
    if (blocks > (long long)num_cus * 4) blocks = (long long)num_cus * 4;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(embed_exact, dim3((unsigned)blocks), dim3(EX_THREADS), smem, s, a, 1);
    return hipGetLastError();
}

__global__ void reset_fallback(unsigned long long *counters) {
    if (threadIdx.x == 0) counters[C_FB_LEN] = 0ull;
}

hipError_t launch_reset_fallback(unsigned long long *counters, hipStream_t s) {
    hipLaunchKernelGGL(reset_fallback, dim3(1), dim3(64), 0, s, counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------- projection from given neighbours

hipError_t launch_project(const EmbedArgs &a, int kp, int num_cus, hipStream_t s) {
    const int block = 256, wpb = 4;
    const size_t smem = (size_t)wpb * kp * 64 * 10 + sizeof(unsigned short) * (size_t)a.g;
    long long blocks = ((a.n + 63) / 64 + wpb - 1) / wpb;
    if (blocks > (long long)num_cus * 8) blocks = (long long)num_cus * 8;
    if (blocks < 1) blocks = 1;
    if (kp == 8)
        hipLaunchKernelGGL(embed_project<8>, dim3((unsigned)blocks), dim3(block), smem, s, a);
    else if (kp == 16)
        hipLaunchKernelGGL(embed_project<16>, dim3((unsigned)blocks), dim3(block), smem, s, a);
    else if (kp == 20)
        hipLaunchKernelGGL(embed_project<20>, dim3((unsigned)blocks), dim3(block), smem, s, a);
    else if (kp == 24)
        hipLaunchKernelGGL(embed_project<24>, dim3((unsigned)blocks), dim3(block), smem, s, a);
    else
        hipLaunchKernelGGL(embed_project<32>, dim3((unsigned)blocks), dim3(block), smem, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- main kernel dispatch

// Instantiation units (embed_inst.hip, one object per (mode, KP)); each
// picks the DC instantiation, sizes a persistent grid from the occupancy of
// that kernel, and launches it.
hipError_t launch_main_m0_kp8_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp16_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp20_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp20_kf1(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp24_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp32_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp8_kf1(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp16_kf1(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m0_kp32_kf1(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp8_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp16_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp20_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp20_kf1(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp24_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp32_kf0(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp8_kf1(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp16_kf1(const EmbedArgs &, int, int, size_t, int, hipStream_t);
hipError_t launch_main_m1_kp32_kf1(const EmbedArgs &, int, int, size_t, int, hipStream_t);

hipError_t launch_embed(const EmbedArgs &a0, int mode, int kp, int num_cus, size_t lds_per_block,
                        hipStream_t s) {
    EmbedArgs a = a0;
    const int dc = a.dp / 16;
    const size_t wsm = (size_t)wave_smem_bytes(kp, a.k, a.npair_tiles);
    const size_t rows = ((size_t)a.g * (a.dp + 4) * 4 + 255) & ~(size_t)255;
    // Stage the landmark rows in LDS when a full block of waves (one block per
    // CU: 3 or 2 waves per SIMD, main_max_block) still fits beside them;
    // otherwise rescore from global memory with 4-wave blocks, several per CU.
    // The screen operands (A tiles and norms, read by every wave twice per 64
    // points) join them in LDS when that still fits.
    const int max_wpb = main_max_block(mode, dc, kp) / 64;
    int wpb;
    const size_t fixed = CENT_LDS_BYTES + order_lds_bytes(a.g);
    const size_t tiles = tile_lds_bytes(mode, a.ntiles, dc);
    a.lds_tiles = 0;
    if (fixed + rows + (size_t)max_wpb * wsm <= lds_per_block) {
        a.lds_rows = 1;
        wpb = max_wpb;
        if (fixed + rows + tiles + (size_t)max_wpb * wsm <= lds_per_block) a.lds_tiles = 1;
    } else {
        a.lds_rows = 0;
        wpb = (int)((lds_per_block - fixed) / wsm);
        if (wpb > 4) wpb = 4;
        if (wpb < 1) wpb = 1;
    }
    const size_t smem = fixed + (a.lds_rows ? rows : 0) + (a.lds_tiles ? tiles : 0) + (size_t)wpb * wsm;
    const int block = 64 * wpb;
    // k == KP with k < g has its own instantiation (KP 8, 16, 20 and 32)
    const bool kf = a.k == kp && a.kact == kp - 1 && kp != 24;
    if (mode == 0) {
        if (kp == 8) return (kf ? launch_main_m0_kp8_kf1 : launch_main_m0_kp8_kf0)(a, dc, block, smem, num_cus, s);
        if (kp == 16) return (kf ? launch_main_m0_kp16_kf1 : launch_main_m0_kp16_kf0)(a, dc, block, smem, num_cus, s);
        if (kp == 20) return (kf ? launch_main_m0_kp20_kf1 : launch_main_m0_kp20_kf0)(a, dc, block, smem, num_cus, s);
        if (kp == 24) return launch_main_m0_kp24_kf0(a, dc, block, smem, num_cus, s);
        return (kf ? launch_main_m0_kp32_kf1 : launch_main_m0_kp32_kf0)(a, dc, block, smem, num_cus, s);
    }
    if (kp == 8) return (kf ? launch_main_m1_kp8_kf1 : launch_main_m1_kp8_kf0)(a, dc, block, smem, num_cus, s);
    if (kp == 16) return (kf ? launch_main_m1_kp16_kf1 : launch_main_m1_kp16_kf0)(a, dc, block, smem, num_cus, s);
    if (kp == 20) return (kf ? launch_main_m1_kp20_kf1 : launch_main_m1_kp20_kf0)(a, dc, block, smem, num_cus, s);
    if (kp == 24) return launch_main_m1_kp24_kf0(a, dc, block, smem, num_cus, s);
    return (kf ? launch_main_m1_kp32_kf1 : launch_main_m1_kp32_kf0)(a, dc, block, smem, num_cus, s);
}

}  // namespace esom
