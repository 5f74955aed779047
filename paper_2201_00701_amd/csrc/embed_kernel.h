// Fused EmbedSOM kernel for gfx950 (one wavefront = 64 points).
//
// Phase A, screen (MFMA).  The wave holds its 64 points as two 32-point MFMA
// B operands (centred on the landmark centroid) in registers and streams
// 32-landmark A tiles (-2 (L_j - c), prepared once per landmark set).
// v_mfma_f32_32x32x* with C initialised to |L_j - c|^2 gives
//   key_ij = |L_j - c|^2 - 2 <x_i - c, L_j - c>  =  delta_ij^2 - |x_i - c|^2,
// so keys rank the landmarks of a point exactly like the distances do.  In
// the 32x32 output layout lane l holds 16 keys of point (l mod 32); the two
// lanes l and l+32 of a point see disjoint halves of every tile.
//   Pass 1 (BF16 operands) keeps, per lane, the minimum key of 32 landmark
//   groups (register slot x tile parity).  A lane's j-th smallest group
//   minimum bounds from above j distinct keys of its half, so with
//   j = ceil(C/2) the larger of the two lanes' values has at least C keys at
//   or below it; widened by both passes' error bounds it is the threshold tau.
//   Pass 2 recomputes the keys more accurately (FP32 operands in FP32 mode;
//   in BF16 mode both operands split into high and low BF16 parts, three
//   products per element, which leaves an error near 2^-16 of the products
//   instead of 2^-8) and shifts one bit per key (key <= tau) into a per-lane
//   bitmap in LDS: the candidate set, with no capacity limit.
// Phase B, exact selection (one lane = one point).  Every candidate is
// rescored with exact FP32 differences and inserted into a sorted register
// list; keys are doubles packing (delta^2, landmark index) so a plain
// min/max network orders them lexicographically.  A point is certified when
// its k-th rescored distance lies below tau by more than a rigorous bound of
// the screen's rounding error (every non-candidate then lies farther away).
// Phase C, projection (FP32, FP64 solve).  Scores from the k distances; the
// pair terms use D_uv = 1/2 + (delta_u^2 - delta_v^2) / (2 |L_u - L_v|^2)
// (polarisation of the segment projection) with the pair table from the
// landmark preparation; Cramer's rule in FP64.
// Points the fast path cannot vouch for (uncertified screen, k-th/(k+1)-th
// tie below FP32 resolution, ill-conditioned system, degenerate
// neighbourhood) are appended to a list and recomputed by the exact FP64
// kernel afterwards.
#pragma once

#include <float.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "esom_internal.h"

namespace esom {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr float U32 = 5.9604645e-08f;     // 2^-24, FP32 unit roundoff
constexpr float ILL_PAIR = 64.0f;         // max(delta^2)/(2|L_u-L_v|^2) beyond this: exact path
constexpr double ILL_COND = 64.0;         // (tr/2)^2/det beyond this: exact path
constexpr double SINGULAR_REL = 1e-9;     // det <= this (tr/2)^2: singular, centroid
// Cutoff weights below this are recomputed from FP64 distances: c = 1 - exp(A
// (delta_q - delta_k) / delta_k) takes its relative accuracy from the difference
// delta_q - delta_k, which FP32 distances only give to ~u delta_k, so a weight
// c ~ A u carries a relative error near 1 (and a system held only by such a
// weight moves accordingly).  Above it the relative error is at most
// 2 A (d_pad + 3) u / C_REFINE.  Done for k <= 8 (see embed_main).
constexpr float C_REFINE = 1.0f / 32.0f;
constexpr float LN_1M_CREFINE = -0.031748698f;  // ln(1 - C_REFINE)
constexpr int N_REFINE = 4;                      // refined weights per point at most

// Largest block of the fused kernel: 12 waves (3 per SIMD, 168 registers per
// lane) where the register budget of the instantiation allows it (padded
// dimension <= 32, k <= 16), else 8 waves (256 registers).  In FP32 mode the
// 12-wave block leaves no LDS room for the FP32 screen tiles (they stream
// from L2) and spills a few registers once per 64 points, and still runs
// 8% faster at 1M x 32-D with 400 landmarks than 8 waves with the tiles in
// LDS: the third wave per SIMD overlaps one wave's MFMA screen with another's
// VALU phases.
__host__ __device__ constexpr int main_max_block(int mode, int dc, int kp) {
    return (dc <= 2 && kp <= 16) ? 768 : 512;
}

// 1 - exp(z) for z <= 0 with full relative accuracy near 0: Taylor series
// through z^7 for |z| < 1/8 (truncation below 2e-11 relative), else 1 - exp(z)
// directly (then 1 - exp(z) > 0.11 and its rounding is relatively small).
__device__ __forceinline__ float one_minus_exp(float z) {
    if (z > -0.125f) {
        float p = 1.f / 5040.f;
        p = fmaf(p, z, 1.f / 720.f);
        p = fmaf(p, z, 1.f / 120.f);
        p = fmaf(p, z, 1.f / 24.f);
        p = fmaf(p, z, 1.f / 6.f);
        p = fmaf(p, z, 0.5f);
        p = fmaf(p, z, 1.f);
        return fmaxf(-z * p, 0.f);
    }
    return 1.f - __expf(z);
}

__device__ __forceinline__ unsigned bf16_bits_rne(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ double pack_key(float d2, int j) {
    unsigned long long b = (unsigned long long)__double_as_longlong((double)d2);
    return __longlong_as_double((long long)(b | (unsigned long long)j));
}
__device__ __forceinline__ float key_d2(double v) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (float)__longlong_as_double((long long)(b & ~0x1FFFull));
}
__device__ __forceinline__ int key_idx(double v) {
    return (int)((unsigned long long)__double_as_longlong(v) & 0x1FFFull);
}

// Upper bound of the exact k-th nearest squared distance from the rescored
// k-th value d2k: each of the first k rescored values is within (d_pad+3)u of
// its exact value, so k landmarks lie within d2k (1 + 2 (d_pad+3) u); the
// factor 4 leaves room for the FP64 distances of the exact path.  +inf when
// fewer than k candidates were rescored (d2k = +inf).
__device__ __forceinline__ float kth_bound(float d2k, int dp) {
    const float t = d2k * (1.f + 4.f * (float)(dp + 3) * U32);
    return t < FLT_MAX ? t : INFINITY;
}

// Batcher's odd-even merge sort network on N = 2^m inputs (63 comparators for
// 16, 191 for 32), built at compile time.
template <int N>
struct OemNet {
    int a[N * N] = {}, b[N * N] = {};
    int n = 0;
    constexpr OemNet() { sort(0, N - 1); }
    constexpr void merge(int lo, int hi, int r) {
        const int step = 2 * r;
        if (step < hi - lo) {
            merge(lo, hi, step);
            merge(lo + r, hi, step);
            for (int i = lo + r; i < hi - r; i += step) {
                a[n] = i;
                b[n] = i + r;
                ++n;
            }
        } else {
            a[n] = lo;
            b[n] = lo + r;
            ++n;
        }
    }
    constexpr void sort(int lo, int hi) {
        if (hi - lo >= 1) {
            const int mid = lo + (hi - lo) / 2;
            sort(lo, mid);
            sort(mid + 1, hi);
            merge(lo, hi, 1);
        }
    }
};

// Ascending sort of N registers.  The screen sorts bit patterns of
// non-negative floats: for those, integer order is float order and +inf sorts
// last.
template <int N>
__device__ __forceinline__ void sort_regs(int (&v)[N]) {
    constexpr OemNet<N> net{};
#pragma unroll
    for (int c = 0; c < net.n; ++c) {
        const int x = v[net.a[c]], y = v[net.b[c]];
        v[net.a[c]] = min(x, y);
        v[net.b[c]] = max(x, y);
    }
}

// Bitonic merge of N registers holding a bitonic sequence: ascending after.
template <int N>
__device__ __forceinline__ void bitonic_clean(int (&m)[N]) {
#pragma unroll
    for (int st = N / 2; st > 0; st >>= 1)
#pragma unroll
        for (int i = 0; i < N; ++i)
            if ((i & st) == 0) {
                const int x = m[i], y = m[i + st];
                m[i] = min(x, y);
                m[i + st] = max(x, y);
            }
}

// The j-th smallest (1 <= j <= 32) of the 64 values held by a lane (lo[0..15],
// hi[0..15]) and its partner lane (lane ^ 32), the same on both lanes.  Each
// lane orders its own smallest values (16 for j <= 16, else all 32); with two
// ascending lists s and t of length M, min(s[i], t[M - 1 - i]) holds the M
// smallest of their union as a bitonic sequence, which a bitonic merge orders.
// j is uniform.
__device__ __forceinline__ int select_pair_jth(int (&lo)[16], int (&hi)[16], int j) {
    if (j <= 16) {
        sort_regs<16>(lo);
        sort_regs<16>(hi);
        int s[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) s[i] = min(lo[i], hi[15 - i]);
        bitonic_clean<16>(s);
        int u[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) u[i] = min(s[i], __shfl_xor(s[15 - i], 32));
        bitonic_clean<16>(u);
        int t = u[0];
#pragma unroll
        for (int i = 1; i < 16; ++i)
            if (i == j - 1) t = u[i];
        return t;
    }
    int v[32];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        v[i] = lo[i];
        v[16 + i] = hi[i];
    }
    sort_regs<32>(v);
    int u[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) u[i] = min(v[i], __shfl_xor(v[31 - i], 32));
    bitonic_clean<32>(u);
    int t = u[31];
#pragma unroll
    for (int i = 16; i < 31; ++i)
        if (i == j - 1) t = u[i];
    return t;
}

// The j-th smallest (1 <= j <= 32) of the 32 values lo[0..15], hi[0..15].
// For j <= 16: with both halves sorted, min(lo[i], hi[15 - i]) holds the 16
// smallest of the union as a bitonic sequence; its maximum is the 16th
// smallest, and a bitonic merge orders it for smaller j.  j is uniform.
__device__ __forceinline__ int select_jth(int (&lo)[16], int (&hi)[16], int j) {
    if (j <= 16) {
        sort_regs<16>(lo);
        sort_regs<16>(hi);
        int m[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) m[i] = min(lo[i], hi[15 - i]);
        if (j == 16) {
            int t = m[0];
#pragma unroll
            for (int i = 1; i < 16; ++i) t = max(t, m[i]);
            return t;
        }
#pragma unroll
        for (int st = 8; st > 0; st >>= 1)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if ((i & st) == 0) {
                    const int x = m[i], y = m[i + st];
                    m[i] = min(x, y);
                    m[i + st] = max(x, y);
                }
        int t = m[0];
#pragma unroll
        for (int i = 1; i < 16; ++i)
            if (i == j - 1) t = m[i];
        return t;
    }
    int v[32];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        v[i] = lo[i];
        v[16 + i] = hi[i];
    }
    sort_regs<32>(v);
    int t = v[31];
#pragma unroll
    for (int i = 16; i < 32; ++i)
        if (i == j - 1) t = v[i];
    return t;
}

// FP32 minimum as a single instruction: the median of (a, b, ninf) with ninf
// = -inf.  fminf, or a median with a visible -inf constant (which the
// compiler turns into fminf), quiets both operands with an extra instruction
// each.  (Not inline assembly: the compiler must see the read of an MFMA
// result to insert the wait states it needs.)
__device__ __forceinline__ float vmin32(float a, float b, float ninf) {
    return __builtin_amdgcn_fmed3f(a, b, ninf);
}

// x * y as a 24-bit multiply (full rate); the compiler otherwise emits a
// 32-bit multiply, which issues at a quarter of the rate.  x, y < 2^24 and
// x * y < 2^32.
__device__ __forceinline__ unsigned mul24(unsigned x, unsigned y) {
    unsigned r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(x), "s"(y));
    return r;
}
template <int RS>
__device__ __forceinline__ unsigned row_offset(int j) {
    return mul24((unsigned)j, (unsigned)RS);
}

// -inf in a scalar register, opaque to the compiler.
__device__ __forceinline__ float opaque_neg_inf() {
    float r;
    asm volatile("s_mov_b32 %0, 0xff800000" : "=s"(r));
    return r;
}

// FP64 minimum / maximum as single instructions.  fmin/fmax would add a
// quieting step per operand for signalling NaNs, which never occur here (the
// operands are packed keys built by integer operations, or +inf).
__device__ __forceinline__ double vmin64(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double vmax64(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Insert v into the ascending list s; whatever falls off the end updates rej
// (the smallest key ever rejected).
template <int KP>
__device__ __forceinline__ void insert_sorted(double (&s)[KP], double &rej, double v) {
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        const double hi = vmax64(s[q], v);
        asm("v_min_f64 %0, %0, %1" : "+v"(s[q]) : "v"(v));  // in place: no copies of the list
        v = hi;
    }
    rej = vmin64(rej, v);
}

// Next non-empty 64-bit bitmap word of a point: mk marks the non-empty words
// (bit tp = tile pair tp), row = the point's words, stride 32 per tile pair.
// nb = 0 when none is left.
__device__ __forceinline__ void next_word(unsigned long long &mk, const unsigned long long *row,
                                          unsigned long long &nb, int &ntp) {
    nb = 0ull;
    if (mk) {
        ntp = __builtin_ctzll(mk);
        mk &= mk - 1ull;
        nb = row[ntp * 32];
    }
}

template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};
template <int V>
struct IntTag {
    static constexpr int value = V;
};

// LDS bytes of the block-wide centroid copy (padded dimension <= 128).
constexpr int CENT_LDS_BYTES = 512;

// LDS bytes of the block-wide landmark order tables (position -> landmark and
// landmark -> position, 16-bit each, two halves of equal size).
__host__ __device__ inline size_t order_lds_bytes(int g) { return (size_t)(((2 * g + 255) / 256) * 256) * 2; }

// Bytes of the screen's A operand (ntiles tiles of 32 landmarks) and of its
// LDS copy with the norms (16 per lane half and tile), 256-byte aligned.
__host__ __device__ inline size_t tile_a_bytes(int mode, int ntiles, int dc) {
    return (size_t)ntiles * dc * 64 * (mode == 1 ? 16 : 32);
}
__host__ __device__ inline size_t tile_lds_bytes(int mode, int ntiles, int dc) {
    return (tile_a_bytes(mode, ntiles, dc) + (size_t)ntiles * 128 + 255) & ~(size_t)255;
}

// Bytes of LDS one wave needs: candidate bitmaps (2 W words per lane), or for
// KP > 24 the neighbour staging of the pair loop (k entries of 10 bytes per
// lane) in the same space; then thresholds, norms and the per-lane masks of
// non-empty bitmap words.
__host__ __device__ inline int wave_smem_bytes(int kp, int k, int npair_tiles) {
    const int bits = 2 * npair_tiles * 64 * 4;
    const int nbr = kp > 24 ? k * 64 * 10 : 0;
    return (bits > nbr ? bits : nbr) + 512 + 1024;
}

// Centred values x_t - c_t of dimensions 16 c + 8 h + e (e < 8) of the point
// row xr; zero past d and for an invalid point.
__device__ __forceinline__ void centred8(const EmbedArgs &a, const float *xr, const float *centL, int c, int h,
                                         bool valid, float (&v)[8]) {
    if (a.x_vec4) {
        const float4 *x4 = reinterpret_cast<const float4 *>(xr + 16 * c + 8 * h);
        const float4 *c4 = reinterpret_cast<const float4 *>(centL + 16 * c + 8 * h);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const float4 q = valid ? x4[u] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 cv = valid ? c4[u] : make_float4(0.f, 0.f, 0.f, 0.f);
            v[4 * u] = q.x - cv.x;
            v[4 * u + 1] = q.y - cv.y;
            v[4 * u + 2] = q.z - cv.z;
            v[4 * u + 3] = q.w - cv.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int d0 = 16 * c + 8 * h + e;
            v[e] = (valid && d0 < a.d) ? xr[d0] - centL[d0] : 0.f;
        }
    }
}

// Point index of processing slot si < n (the optional locality order).
__device__ __forceinline__ int64_t slot_point(const EmbedArgs &a, int64_t si) {
    return a.pt_order ? (int64_t)a.pt_order[si] : si;
}

template <int MODE, int DC>
struct PointOperand;

template <int DC>
struct PointOperand<1, DC> {  // BF16: lane holds dims 16c + 8h + e of its point
    bf16x8 b[2][DC];
};
template <int DC>
struct PointOperand<0, DC> {  // FP32: lane holds dims 2s + h, s < 8 DC
    float b[2][8 * DC];
};

// One landmark tile's A operand and squared norms, as one lane holds them.
template <int MODE, int DC>
struct TileRegs;
template <int DC>
struct TileRegs<1, DC> {
    u32x4 a[DC];
};
template <int DC>
struct TileRegs<0, DC> {
    float a[8 * DC];
};

// The A operand and the norms come from Abase / Nbase: global memory, or the
// block's LDS copy (the caller's choice, fixed per instantiation so that the
// compiler sees the address space).
template <int MODE, int DC>
__device__ __forceinline__ void load_tile(const void *Abase, int t, int lane, TileRegs<MODE, DC> &T) {
    if constexpr (MODE == 1) {
        const u32x4 *Ap = reinterpret_cast<const u32x4 *>(Abase) + (size_t)t * DC * 64 + lane;
#pragma unroll
        for (int c = 0; c < DC; ++c) T.a[c] = Ap[c * 64];
    } else {
        const float *Ap = reinterpret_cast<const float *>(Abase) + (size_t)t * (8 * DC) * 64 + lane;
#pragma unroll
        for (int s = 0; s < 8 * DC; ++s) T.a[s] = Ap[s * 64];
    }
}

// Keys of tile t for both 32-point halves of the wave: acc[p] = |L|^2 + A B_p.
template <int MODE, int DC>
__device__ __forceinline__ void screen_tile(const float *Nbase, int t, int lane, const TileRegs<MODE, DC> &T,
                                            const PointOperand<MODE, DC> &P, f32x16 (&acc)[2]) {
    f32x16 nrm;
    {
        const float4 *np = reinterpret_cast<const float4 *>(Nbase + (size_t)(t * 2 + (lane >> 5)) * 16);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float4 n = np[i];
            nrm[4 * i] = n.x;
            nrm[4 * i + 1] = n.y;
            nrm[4 * i + 2] = n.z;
            nrm[4 * i + 3] = n.w;
        }
    }
    acc[0] = nrm;
    acc[1] = nrm;
    if constexpr (MODE == 1) {
#pragma unroll
        for (int c = 0; c < DC; ++c) {
            const bf16x8 av = __builtin_bit_cast(bf16x8, T.a[c]);
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, P.b[0][c], acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, P.b[1][c], acc[1], 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int s = 0; s < 8 * DC; ++s) {
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(T.a[s], P.b[0][s], acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(T.a[s], P.b[1][s], acc[1], 0, 0, 0);
        }
    }
}

// Split BF16 keys of tile t: acc[p] = |L|^2 + Al B_p + Ah Bl_p + Ah B_p (the
// small terms first), with A = Ah + Al and B = B_p + Bl_p the high and low
// BF16 parts of the two operands.
template <int DC>
__device__ __forceinline__ void screen_tile_split(const float *Nbase, int t, int lane, const TileRegs<1, DC> &Th,
                                                  const TileRegs<1, DC> &Tl, const PointOperand<1, DC> &P,
                                                  const PointOperand<1, DC> &Pl, f32x16 (&acc)[2]) {
    f32x16 nrm;
    {
        const float4 *np = reinterpret_cast<const float4 *>(Nbase + (size_t)(t * 2 + (lane >> 5)) * 16);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float4 n = np[i];
            nrm[4 * i] = n.x;
            nrm[4 * i + 1] = n.y;
            nrm[4 * i + 2] = n.z;
            nrm[4 * i + 3] = n.w;
        }
    }
    acc[0] = nrm;
    acc[1] = nrm;
#pragma unroll
    for (int c = 0; c < DC; ++c) {
        const bf16x8 al = __builtin_bit_cast(bf16x8, Tl.a[c]);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, P.b[0][c], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, P.b[1][c], acc[1], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < DC; ++c) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, Th.a[c]);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, Pl.b[0][c], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, Pl.b[1][c], acc[1], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < DC; ++c) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, Th.a[c]);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, P.b[0][c], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, P.b[1][c], acc[1], 0, 0, 0);
    }
}

// Cutoff weights c = 1 - exp(A (delta_q - delta_k) / delta_k) of the active
// neighbours whose FP32 value is below C_REFINE, from FP64 distances.  sk: the
// k nearest as sorted (delta^2, index) keys.  d2x(j) returns the FP64 squared
// distance from the lane's point to landmark j; it is called by all lanes
// together, with a valid landmark on every lane.  c decreases along the sorted
// list, so the weights to refine are the lane's last nref active ones: on
// return cref[r-1] holds the weight of neighbour kact - r for r = 1..nref
// (nref <= N_REFINE).  Returns R_NEARTIE when the FP64 distances order a
// refined neighbour after the k-th (the exact path then ranks the point again)
// and R_ILLCOND when more than N_REFINE weights need it (rare: 0.03% of the
// points of 1M x 32-D with 400 landmarks even at k = 16).
template <int KP, class D2X>
__device__ __forceinline__ unsigned refine_cutoffs(const EmbedArgs &a, const double (&sk)[KP], bool valid,
                                                   D2X &&d2x, float (&cref)[N_REFINE], int &nref) {
    nref = 0;
#pragma unroll
    for (int r = 0; r < N_REFINE; ++r) cref[r] = 0.f;
    if (!a.use_cutoff) return 0u;
    float d2k = 0.f;
    int jk = 0;
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        if (q == a.k - 1) {
            d2k = key_d2(sk[q]);
            jk = key_idx(sk[q]);
        }
    }
    // c < C_REFINE  <=>  delta_q / delta_k > 1 + ln(1 - C_REFINE) / A
    const float f = 1.f + LN_1M_CREFINE / a.cutoff;
    const float lim = f > 0.f ? d2k * f * f : 0.f;
#pragma unroll
    for (int q = 0; q < KP; ++q)
        if (valid && q < a.kact && key_d2(sk[q]) > lim) ++nref;
    unsigned reason = 0u;
    if (nref > N_REFINE) {
        reason |= R_ILLCOND;
        nref = N_REFINE;
    }
    if (__ballot(nref > 0) == 0ull) return reason;
    const double d2k64 = d2x(jk);
    const float dk32 = __builtin_amdgcn_sqrtf((float)d2k64);
#pragma unroll
    for (int r = 1; r <= N_REFINE; ++r) {
        if (__ballot(r <= nref) == 0ull) break;
        const bool act = r <= nref;
        int jt = jk;
#pragma unroll
        for (int q = 0; q < KP; ++q)
            if (act && q == a.kact - r) jt = key_idx(sk[q]);
        const double d2t = d2x(jt);
        // only the difference needs FP64: it keeps its relative accuracy
        // through the conversion, and the rest is well conditioned
        const float dd = (float)(d2t - d2k64);
        const float den = (__builtin_amdgcn_sqrtf((float)d2t) + dk32) * dk32;
        const float z = den > 0.f ? a.cutoff * dd / den : 0.f;
        if (act && (d2t > d2k64 || (d2t == d2k64 && jt > jk))) reason |= R_NEARTIE;
        cref[r - 1] = one_minus_exp(z);
    }
    return reason;
}

// Phase C for one point (lane): scores from the k sorted distances, the pair
// terms, the FP64 2x2 solve and the output store.  sk holds the k nearest as
// packed (delta^2, index) keys, ascending.  Returns the accumulated fallback
// reasons; the output is written only when there is none.
// The cutoff weight of neighbour kact - r comes from cref[r-1] for r = 1..nref
// (see refine_cutoffs).
template <int KP>
__device__ __forceinline__ unsigned project_point(const EmbedArgs &a, const double (&sk)[KP],
                                                  int lane, bool valid, long long pi, unsigned reason,
                                                  float *nbD2, float *nbS, unsigned short *nbI,
                                                  const unsigned short *iposL, const float (&cref)[N_REFINE],
                                                  int nref) {
    float d2q[KP], dl[KP], sq[KP], lxq[KP], lyq[KP];
    int jq[KP];
    float mu = 0.f;
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        d2q[q] = (q < a.k) ? key_d2(sk[q]) : 0.f;
        jq[q] = (q < a.k) ? key_idx(sk[q]) : 0;
        dl[q] = __builtin_amdgcn_sqrtf(d2q[q]);
        if (q < a.k) mu = fmaf(dl[q], 1.f / (float)(q + 1), mu);
    }
    float d2k = d2q[0];
#pragma unroll
    for (int q = 0; q < KP; ++q)
        if (q == a.k - 1) d2k = d2q[q];
    mu /= a.Wk;
    float var = 0.f;
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        if (q < a.k) {
            const float e = dl[q] - mu;
            var = fmaf(e * e, 1.f / (float)(q + 1), var);
        }
    }
    var /= a.Wk;
    const float dk = __builtin_amdgcn_sqrtf(d2k);
    // cutoff argument A (delta_q - delta_k) / delta_k from the FP32 distances
    const float cut_scale = a.cutoff * __builtin_amdgcn_rcpf(dk);
    const bool degenerate = d2q[0] == d2k;
    const bool flat = !(var > 1e-30f * mu * mu);
    const float isig = flat ? 0.f : a.boost * rsqrtf(var);
    if (degenerate) reason |= R_DEGEN;
    const float ox = a.l2d[2 * jq[0]], oy = a.l2d[2 * jq[0] + 1];
    float ssum = 0.f;
    float M00 = 0.f, M01 = 0.f, M11 = 0.f, r0 = 0.f, r1 = 0.f;
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        const float2 lv = reinterpret_cast<const float2 *>(a.l2d)[jq[q]];
        lxq[q] = lv.x - ox;
        lyq[q] = lv.y - oy;
    }
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        sq[q] = 0.f;
        if (q < a.k) {
            const float e = flat ? 1.f : __expf((mu - dl[q]) * isig);
            float c = a.use_cutoff ? 1.f - __expf((dl[q] - dk) * cut_scale) : 1.f;
            if constexpr (KP <= 8) {
#pragma unroll
                for (int r = 1; r <= N_REFINE; ++r)
                    if (r <= nref && q == a.kact - r) c = cref[r - 1];
            }
            sq[q] = degenerate ? 0.f : e * c;
            ssum += sq[q];
            const float gs = a.gravity * sq[q];
            M00 += gs;
            M11 += gs;
            r0 = fmaf(gs, lxq[q], r0);
            r1 = fmaf(gs, lyq[q], r1);
        }
    }
    if (!(ssum > 0.f)) reason |= R_DEGEN;

    // pairs (i < j among the neighbours with non-zero score); d2i <= d2j.  The
    // pair (i, j) adds q/|h|^2 h h^T to M and q/|h|^2 h t to r, with h = l_j - l_i,
    // t = D |h|^2 + h.l_i and D its segment coordinate.  Split as q D h plus
    // (q/|h|^2 h h^T) l_i, the second part sums over j into M_i l_i, so a pair
    // costs no dot product; s_i multiplies the sums of base i once.  The pair
    // table supplies 1/(2|L_u - L_v|^2), 0 for coincident landmarks; 1/|h|^2
    // comes from the 2-D difference at hand, and a pair with either length 0
    // gets weight 0, so a skipped pair adds exactly 0.
    float pmax = 0.f;  // largest delta_j^2 / (2 |L_i - L_j|^2) over the pairs
    const bool unit_adjust = a.adjust == 1.0f;
    auto pair_term = [&](auto unit, float d2i, float lxi, float lyi, float d2j, float sj, float lxj,
                         float lyj, float inv, float (&Mi)[3], float (&ri)[2]) {
        const float hx = lxj - lxi, hy = lyj - lyi;
        const float hh = fmaf(hx, hx, hy * hy);
        const float ihh = (inv > 0.f && hh > 0.f) ? __builtin_amdgcn_rcpf(hh) : 0.f;
        const float D = fmaf(d2i - d2j, inv, 0.5f);
        pmax = fmaxf(pmax, d2j * inv);
        float q;
        // unit: adjust == 1 (weight 1 / |h|^2), as a compile-time tag so that
        // the two variants of the pair loop are separate code
        if constexpr (decltype(unit)::value)
            q = sj * ihh;
        else
            q = ihh > 0.f ? sj * exp2f(a.adjust * __log2f(ihh)) : 0.f;
        const float qh = q * ihh, qD = q * D;
        const float qhx = qh * hx, qhy = qh * hy;
        Mi[0] = fmaf(qhx, hx, Mi[0]);
        Mi[1] = fmaf(qhx, hy, Mi[1]);
        Mi[2] = fmaf(qhy, hy, Mi[2]);
        ri[0] = fmaf(qD, hx, ri[0]);
        ri[1] = fmaf(qD, hy, ri[1]);
    };
    // closes base i: r += s_i (r_i + M_i l_i), M += s_i M_i
    auto close_base = [&](bool origin, float si, float lxi, float lyi, const float (&Mi)[3],
                          float (&ri)[2]) {
        if (!origin) {
            ri[0] = fmaf(Mi[0], lxi, fmaf(Mi[1], lyi, ri[0]));
            ri[1] = fmaf(Mi[1], lxi, fmaf(Mi[2], lyi, ri[1]));
        }
        M00 = fmaf(si, Mi[0], M00);
        M01 = fmaf(si, Mi[1], M01);
        M11 = fmaf(si, Mi[2], M11);
        r0 = fmaf(si, ri[0], r0);
        r1 = fmaf(si, ri[1], r1);
    };
    auto run_pairs = [&](auto unit) {
    if constexpr (KP <= 24) {
        // neighbour data in registers (fully unrolled: 276 pair slots at
        // k <= 24, which ran 6% faster at 1M x 48-D, 1024 landmarks, k = 20
        // than the LDS staging below); each row of pair-table loads is issued
        // together, unconditionally (slots past k hold landmark 0, a valid
        // entry, and are never used), addressed by 32-bit byte offsets from
        // the table base (g <= 4096: under 2^26 bytes)
        const char *ptab = reinterpret_cast<const char *>(a.pairs);
#pragma unroll
        for (int qi = 0; qi < KP - 1; ++qi) {
            if (qi < a.kact - 1) {
                const unsigned rowoff = mul24(iposL[jq[qi]], (unsigned)a.g);
                float pv[KP];
#pragma unroll
                for (int qj = qi + 1; qj < KP; ++qj)
                    pv[qj] = *reinterpret_cast<const float *>(ptab + (size_t)((rowoff + iposL[jq[qj]]) * 4u));
                float Mi[3] = {0.f, 0.f, 0.f}, ri[2] = {0.f, 0.f};
#pragma unroll
                for (int qj = qi + 1; qj < KP; ++qj)
                    if (qj < a.kact)
                        pair_term(unit, d2q[qi], lxq[qi], lyq[qi], d2q[qj], sq[qj], lxq[qj], lyq[qj],
                                  pv[qj], Mi, ri);
                // neighbour 0 is the origin of the 2-D frame
                close_base(qi == 0, sq[qi], lxq[qi], lyq[qi], Mi, ri);
            }
        }
    } else {
        // larger neighbourhoods: neighbour data through LDS, inner loop unrolled
        // by 4.  The table is symmetric; entry (u, v) is read at row min(u, v),
        // column max(u, v), so a point's reads cover fewer cache lines (each
        // row only to the right of its own position): 4% faster at 1M x 48-D,
        // 1024 landmarks, k = 20 when this path served that shape.  (With
        // k <= 16 the extra address arithmetic cost more than it saved.)
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            if (q < a.k) {
                nbD2[q * 64 + lane] = d2q[q];
                nbS[q * 64 + lane] = sq[q];
                nbI[q * 64 + lane] = (unsigned short)jq[q];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int qi = 0; qi < a.kact - 1; ++qi) {
            const float d2i = nbD2[qi * 64 + lane], si = nbS[qi * 64 + lane];
            const int ui = nbI[qi * 64 + lane];
            const float2 li = reinterpret_cast<const float2 *>(a.l2d)[ui];
            const float lxi = li.x - ox, lyi = li.y - oy;
            const unsigned pu = iposL[ui];
            float Mi[3] = {0.f, 0.f, 0.f}, ri[2] = {0.f, 0.f};
            for (int qb = qi + 1; qb < a.kact; qb += 4) {
                float pv[4];
                float d2j[4], sj[4], lxj[4], lyj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int qj = qb + u;
                    const bool ok = qj < a.kact;
                    const int vj = ok ? nbI[qj * 64 + lane] : 0;
                    const unsigned pw = iposL[vj];
                    pv[u] = ok ? a.pairs[(size_t)min(pu, pw) * a.g + max(pu, pw)] : 0.f;
                    d2j[u] = ok ? nbD2[qj * 64 + lane] : 0.f;
                    sj[u] = ok ? nbS[qj * 64 + lane] : 0.f;
                    const float2 lv = reinterpret_cast<const float2 *>(a.l2d)[vj];
                    lxj[u] = lv.x - ox;
                    lyj[u] = lv.y - oy;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    pair_term(unit, d2i, lxi, lyi, d2j[u], sj[u], lxj[u], lyj[u], pv[u], Mi, ri);
            }
            close_base(false, si, lxi, lyi, Mi, ri);
        }
        __builtin_amdgcn_wave_barrier();
    }
    };
    if (unit_adjust)
        run_pairs(BoolTag<true>{});
    else
        run_pairs(BoolTag<false>{});
    const bool ill = pmax > ILL_PAIR;
    // 2x2 solve in FP64 (Cramer's rule)
    const double m00 = M00, m01 = M01, m11 = M11, rr0 = r0, rr1 = r1;
    const double det = m00 * m11 - m01 * m01;
    const double tr = m00 + m11;
    if (ill || !(det > 0.0) || 0.25 * tr * tr > ILL_COND * det) reason |= R_ILLCOND;
    if (valid && reason == 0) {
        const double px = (rr0 * m11 - m01 * rr1) / det;
        const double py = (m00 * rr1 - m01 * rr0) / det;
        reinterpret_cast<float2 *>(a.out)[pi] = make_float2((float)((double)ox + px),
                                                            (float)((double)oy + py));
    }
    return reason;
}

// Projection only (phases of scores, pairs and solve) from given k nearest
// landmarks (knn_idx / knn_d2, sorted by (distance, index)), e.g. cached from
// an earlier call with the same high-dimensional landmarks.
template <int KP>
__global__ void __launch_bounds__(256) embed_project(EmbedArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    unsigned char *wsm = smem + (size_t)wave * (KP * 64 * 10);
    float *nbD2 = reinterpret_cast<float *>(wsm);
    float *nbS = nbD2 + KP * 64;
    unsigned short *nbI = reinterpret_cast<unsigned short *>(nbS + KP * 64);
    unsigned short *iposL = reinterpret_cast<unsigned short *>(smem + (size_t)wpb * (KP * 64 * 10));
    for (int e = threadIdx.x; e < a.g; e += blockDim.x) iposL[e] = (unsigned short)a.ipos[e];
    __syncthreads();
    const int64_t nwt = (a.n + 63) / 64;
    // Tile wt goes to block wt mod grid, wave (wt / grid) mod wpb: the last,
    // partial round of tiles then spreads over all blocks (CUs) instead of
    // filling the first few.
    for (int64_t wt = (int64_t)wave * gridDim.x + blockIdx.x; wt < nwt; wt += (int64_t)gridDim.x * wpb) {
        const int64_t pi = wt * 64 + lane;
        const bool valid = pi < a.n;
        // A cached index outside [0, g) (the exact path writes -1 for a point
        // without k finite distances) is never used for a load: it becomes
        // landmark 0 and the point goes to the exact path, which ranks it again.
        double sk[KP];
        bool bad_idx = false;
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            sk[q] = INFINITY;
            if (valid && q < a.k) {
                int j = a.knn_idx[pi * a.k + q];
                if (j < 0 || j >= a.g) {
                    bad_idx = true;
                    j = 0;
                }
                sk[q] = pack_key(a.knn_d2[pi * a.k + q], j);
            }
        }
        unsigned reason = (valid && a.knn_mark && a.knn_mark[pi]) ? (unsigned)R_NEARTIE : 0u;
        if (bad_idx) reason |= R_UNCERT;
        float d2k = INFINITY;
#pragma unroll
        for (int q = 0; q < KP; ++q)
            if (q == a.k - 1) d2k = key_d2(sk[q]);
        const float thr = kth_bound(d2k, a.dp);
        const float *xr = a.X + (valid ? pi : 0) * a.ldx;
        auto d2x = [&](int jl) -> double {
            const float *Lr = a.Lpad + (size_t)iposL[jl] * a.dp;
            double acc = 0.0;
            for (int t = 0; t < a.d; ++t) {
                const double e = (double)xr[t] - (double)Lr[t];
                acc = fma(e, e, acc);
            }
            return acc;
        };
        float cref[N_REFINE] = {};
        int nref = 0;
        if constexpr (KP <= 8) reason |= refine_cutoffs<KP>(a, sk, valid, d2x, cref, nref);
        reason = project_point<KP>(a, sk, lane, valid, pi, reason, nbD2, nbS, nbI, iposL, cref, nref);
        if (valid && reason) {
            const unsigned long long slot = atomicAdd(&a.counters[C_FB_LEN], 1ull);
            a.fb_list[slot] = (int32_t)pi;
            a.fb_reason[slot] = (uint8_t)reason;
            a.fb_thresh[slot] = thr;
        }
    }
}

// ROWS = 1: the block stages the padded landmark rows in LDS for the exact
// rescoring (a.lds_rows); ROWS = 0: rows stream from memory.  The two are
// separate instantiations so that each gets its own register allocation.
// KF = 1: k == KP and k < g (so k - 1 neighbours are active), known at
// compile time: the loops over the sorted list and the pairs lose their
// bounds tests (5% faster at 1M x 32-D with k = 16, 4% at 10M x 64-D).
template <int MODE, int DC, int KP, int ROWS, int KF>
__global__ void __launch_bounds__(main_max_block(MODE, DC, KP)) embed_main(EmbedArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (KF == 1) {
        a.k = KP;
        a.kact = KP - 1;
    }
    constexpr int DP = 16 * DC;
    constexpr int RS = DP + 4;  // LDS row stride (floats): spreads rows over the banks
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int h = lane >> 5;
    const int i32 = lane & 31;
    const int W = a.npair_tiles;
    // Block-wide copies: the centroid (read for every point group), and
    // optionally the landmark rows for exact rescoring.
    float *centL = reinterpret_cast<float *>(smem);
    const size_t tab_bytes = order_lds_bytes(a.g);
    unsigned short *permL = reinterpret_cast<unsigned short *>(smem + CENT_LDS_BYTES);
    unsigned short *iposL = permL + tab_bytes / 4;
    float *rowsL = reinterpret_cast<float *>(smem + CENT_LDS_BYTES + tab_bytes);
    const size_t rows_bytes = ROWS ? (((size_t)a.g * RS * 4 + 255) & ~(size_t)255) : 0;
    // optionally the screen operands (A tiles and norms), read by every wave
    // twice per 64 points
    const size_t a_bytes = tile_a_bytes(MODE, a.ntiles, DC);
    const size_t tiles_bytes = a.lds_tiles ? tile_lds_bytes(MODE, a.ntiles, DC) : 0;
    unsigned char *tilesL = smem + CENT_LDS_BYTES + tab_bytes + rows_bytes;
    const float *normsL = reinterpret_cast<const float *>(tilesL + a_bytes);
    for (int e = threadIdx.x; e < DP; e += blockDim.x) centL[e] = e < a.d ? a.cent[e] : 0.f;
    for (int e = threadIdx.x; e < a.g; e += blockDim.x) {
        permL[e] = (unsigned short)a.perm[e];
        iposL[e] = (unsigned short)a.ipos[e];
    }
    if constexpr (ROWS == 1) {
        for (int e = threadIdx.x; e < a.g * (DP / 4); e += blockDim.x) {
            const int j = e / (DP / 4), q = e % (DP / 4);
            reinterpret_cast<float4 *>(rowsL + (size_t)j * RS)[q] =
                reinterpret_cast<const float4 *>(a.Lpad + (size_t)j * DP)[q];
        }
    }
    if (a.lds_tiles) {
        const size_t nv = (a_bytes + (size_t)a.ntiles * 128) / 16;
        const float4 *srcA = reinterpret_cast<const float4 *>(a.A);
        const float4 *srcN = reinterpret_cast<const float4 *>(a.norms);
        for (size_t e = threadIdx.x; e < nv; e += blockDim.x)
            reinterpret_cast<float4 *>(tilesL)[e] = e < a_bytes / 16 ? srcA[e] : srcN[e - a_bytes / 16];
    }
    __syncthreads();
    unsigned char *wsm = smem + CENT_LDS_BYTES + tab_bytes + rows_bytes + tiles_bytes +
                         (size_t)wave * wave_smem_bytes(KP, a.k, W);
    unsigned *bitsL = reinterpret_cast<unsigned *>(wsm);
    float *nbD2 = reinterpret_cast<float *>(wsm);
    float *nbS = nbD2 + a.k * 64;
    unsigned short *nbI = reinterpret_cast<unsigned short *>(nbS + a.k * 64);
    const int nbr_bytes = KP > 24 ? a.k * 64 * 10 : 0;
    const int tail = (2 * W * 64 * 4 > nbr_bytes) ? 2 * W * 64 * 4 : nbr_bytes;
    float *certL = reinterpret_cast<float *>(wsm + tail);  // 64 certificate bounds (512 B reserved)
    unsigned long long *maskL = reinterpret_cast<unsigned long long *>(certL + 128);

    const float lmax = a.lmax[0];
    const float qa = a.lmax[1];  // max_j |bf16(-2 (L_j - c)) + 2 (L_j - c)|

    unsigned long long st_cand = 0;
    const int64_t nwt = (a.n + 63) / 64;
    // Tile wt goes to block wt mod grid, wave (wt / grid) mod wpb: the last,
    // partial round of tiles then spreads over all blocks (CUs) instead of
    // filling the first few.
    for (int64_t wt = (int64_t)wave * gridDim.x + blockIdx.x; wt < nwt; wt += (int64_t)gridDim.x * wpb) {
        const int64_t pbase = wt * 64;

        // ---------------- point operands (centred), and |x - c|^2.  Pass 1
        // always runs on the BF16 operand; FP32 mode builds its FP32 operand
        // for pass 2 afterwards.
        PointOperand<1, DC> P16, P16lo;  // P16lo: BF16 mode's pass 2
        float xnp[2], dxp[2];  // |x - c|^2 and |bf16(x - c) - (x - c)|^2
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int64_t si = pbase + 32 * p + i32;
            const bool valid = si < a.n;
            const float *xr = a.X + (valid ? slot_point(a, si) : 0) * a.ldx;
            float part = 0.f, dpart = 0.f;
#pragma unroll
            for (int c = 0; c < DC; ++c) {
                float v[8];
                centred8(a, xr, centL, c, h, valid, v);
                unsigned w[4];
#pragma unroll
                for (int e = 0; e < 8; e += 2) {
                    part = fmaf(v[e], v[e], part);
                    part = fmaf(v[e + 1], v[e + 1], part);
                    const unsigned b0 = bf16_bits_rne(v[e]), b1 = bf16_bits_rne(v[e + 1]);
                    // quantisation errors (exact in FP32)
                    const float q0 = __uint_as_float(b0 << 16) - v[e], q1 = __uint_as_float(b1 << 16) - v[e + 1];
                    dpart = fmaf(q0, q0, dpart);
                    dpart = fmaf(q1, q1, dpart);
                    w[e >> 1] = b0 | (b1 << 16);
                }
                u32x4 wv = {w[0], w[1], w[2], w[3]};
                P16.b[p][c] = __builtin_bit_cast(bf16x8, wv);
            }
            xnp[p] = part + __shfl_xor(part, 32);
            dxp[p] = dpart + __shfl_xor(dpart, 32);
        }
        // Rigorous bounds of the screen's rounding error in key units, per
        // point.  With a = -2(L - c) and its BF16 image a + da, x' = x - c and
        // its BF16 image x' + dx: |x'.da + dx.a + dx.da| <= |x'| max|da| + |dx|
        // (max|a| + max|da|) (|dx| exact per point, max|da| from the
        // preparation); plus FP32 accumulation and centring, (2 d_pad + 16) u
        // (|x'| + max|L - c|)^2.  FP32 operands are exact and 2 (2u + u^2) |x'|
        // max|L - c| bounds their products.  The FP32 evaluation of the bound
        // is covered by the factor 1.01.  (The split BF16 keys of pass 2 have
        // their own bound, e2 below.)
        float e16[2], e32[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const float sx = sqrtf(xnp[p]);
            const float facc = (2.f * DP + 16.f) * U32 * (sx + lmax) * (sx + lmax);
            e16[p] = 1.01f * (sx * qa + sqrtf(dxp[p]) * (2.f * lmax + qa) + facc);
            e32[p] = 1.01f * (2.f * (2.f * U32 + U32 * U32) * sx * lmax + facc);
        }

        // ---------------- pass 1: group minima of the BF16 keys; |x - c|^2 is
        // added once per group afterwards (rounding is monotone, so the
        // minimum of the sums equals the sum with the minimum).
        float gmin[2][2][16];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 16; ++r) gmin[p][q][r] = INFINITY;
        const float ninf = opaque_neg_inf();
        auto pass1_consume = [&](const f32x16 (&acc)[2], int half) {
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int r = 0; r < 16; ++r) gmin[p][half][r] = vmin32(gmin[p][half][r], acc[p][r], ninf);
        };
        // one screen pass over all tiles with the operand of precision OM,
        // tiles from the block's LDS copy or from global memory
        auto screen_pass = [&](auto in_lds, auto opm, const auto &Pop, const void *Aglob, auto consume,
                               auto store) {
            constexpr int OM = decltype(opm)::value;
            const void *Ab = decltype(in_lds)::value ? static_cast<const void *>(tilesL) : Aglob;
            const float *Nb = decltype(in_lds)::value ? normsL : a.norms;
            TileRegs<OM, DC> T;
            for (int tp = 0; tp < W; ++tp) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    f32x16 acc[2];
                    load_tile<OM, DC>(Ab, 2 * tp + half, lane, T);
                    screen_tile<OM, DC>(Nb, 2 * tp + half, lane, T, Pop, acc);
                    consume(acc, half);
                }
                store(tp);
            }
        };
        // BF16 mode's pass 2: split operands, high parts from LDS or global
        // memory, low parts from global memory (a.A16)
        auto screen_pass_split = [&](auto in_lds, auto consume, auto store) {
            const void *Ab = decltype(in_lds)::value ? static_cast<const void *>(tilesL) : a.A;
            const float *Nb = decltype(in_lds)::value ? normsL : a.norms;
            TileRegs<1, DC> Th, Tl;
            for (int tp = 0; tp < W; ++tp) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    f32x16 acc[2];
                    load_tile<1, DC>(Ab, 2 * tp + half, lane, Th);
                    load_tile<1, DC>(a.A16, 2 * tp + half, lane, Tl);
                    screen_tile_split<DC>(Nb, 2 * tp + half, lane, Th, Tl, P16, P16lo, acc);
                    consume(acc, half);
                }
                store(tp);
            }
        };
        // BF16 mode's pass 2 for points in locality order: the high product
        // first, which is the pass-1 key (same operands, same order, error at
        // most E16).  A 32-point half whose keys of the tile all exceed its
        // points' tau + E16 + E2 (pass-2 keys then exceed tau) has no candidate
        // there: the low products are skipped and the tile's bits marked "not
        // a candidate".  The points of a wavefront share a neighbourhood, and
        // most tiles hold no candidate of theirs.
        auto screen_pass_split_skip = [&](auto in_lds, auto consume, auto store, const float (&thr)[2]) {
            const void *Ab = decltype(in_lds)::value ? static_cast<const void *>(tilesL) : a.A;
            const float *Nb = decltype(in_lds)::value ? normsL : a.norms;
            TileRegs<1, DC> Th, Tl;
            for (int tp = 0; tp < W; ++tp) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const int t = 2 * tp + half;
                    f32x16 acc[2];
                    load_tile<1, DC>(Ab, t, lane, Th);
                    screen_tile<1, DC>(Nb, t, lane, Th, P16, acc);
                    bool need[2];
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        float m = acc[p][0];
#pragma unroll
                        for (int r = 1; r < 16; ++r) m = vmin32(m, acc[p][r], ninf);
                        need[p] = __ballot(m <= thr[p]) != 0ull;
                    }
                    if (need[0] || need[1]) {
                        load_tile<1, DC>(a.A16, t, lane, Tl);
#pragma unroll
                        for (int p = 0; p < 2; ++p) {
                            if (need[p]) {
#pragma unroll
                                for (int c = 0; c < DC; ++c) {
                                    const bf16x8 al = __builtin_bit_cast(bf16x8, Tl.a[c]);
                                    const bf16x8 ah = __builtin_bit_cast(bf16x8, Th.a[c]);
                                    acc[p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, P16.b[p][c], acc[p], 0, 0, 0);
                                    acc[p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, P16lo.b[p][c], acc[p], 0, 0, 0);
                                }
                            }
                        }
                    }
                    consume(acc, need);
                }
                store(tp);
            }
        };
        // FP32 mode's pass 2 likewise, for points in locality order: the BF16
        // key (the pass-1 key, again) decides whether a half needs the tile's
        // FP32 products.
        auto screen_pass_fp32_skip = [&](auto in_lds, const auto &P32, auto consume, auto store,
                                         const float (&thr)[2]) {
            const void *Ab = decltype(in_lds)::value ? static_cast<const void *>(tilesL) : a.A;
            const float *Nb = decltype(in_lds)::value ? normsL : a.norms;
            TileRegs<1, DC> T16;
            TileRegs<0, DC> T32;
            for (int tp = 0; tp < W; ++tp) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const int t = 2 * tp + half;
                    f32x16 acc[2];
                    load_tile<1, DC>(a.A16, t, lane, T16);
                    screen_tile<1, DC>(a.norms, t, lane, T16, P16, acc);
                    bool need[2];
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        float m = acc[p][0];
#pragma unroll
                        for (int r = 1; r < 16; ++r) m = vmin32(m, acc[p][r], ninf);
                        need[p] = __ballot(m <= thr[p]) != 0ull;
                    }
                    if (need[0] || need[1]) {
                        load_tile<0, DC>(Ab, t, lane, T32);
                        const float4 *np = reinterpret_cast<const float4 *>(Nb + (size_t)(t * 2 + (lane >> 5)) * 16);
#pragma unroll
                        for (int p = 0; p < 2; ++p) {
                            if (need[p]) {
#pragma unroll
                                for (int i = 0; i < 4; ++i) {
                                    const float4 n = np[i];
                                    acc[p][4 * i] = n.x;
                                    acc[p][4 * i + 1] = n.y;
                                    acc[p][4 * i + 2] = n.z;
                                    acc[p][4 * i + 3] = n.w;
                                }
#pragma unroll
                                for (int s = 0; s < 8 * DC; ++s)
                                    acc[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(T32.a[s], P32.b[p][s], acc[p], 0, 0, 0);
                            }
                        }
                    }
                    consume(acc, need);
                }
                store(tp);
            }
        };
        {
            auto no_store = [](int) {};
            if constexpr (MODE == 1) {
                if (a.lds_tiles)
                    screen_pass(BoolTag<true>{}, IntTag<1>{}, P16, a.A, pass1_consume, no_store);
                else
                    screen_pass(BoolTag<false>{}, IntTag<1>{}, P16, a.A, pass1_consume, no_store);
            } else {
                // FP32 mode: the BF16 tiles stream from global memory (the LDS
                // copy holds the FP32 tiles of pass 2)
                screen_pass(BoolTag<false>{}, IntTag<1>{}, P16, a.A16, pass1_consume, no_store);
            }
        }
        // thresholds: the jsel-th smallest of the point's 64 group minima (both
        // lanes' 32; negative values, from rounding, count as 0), as a key, or
        // (pair_select = 0: C above 32, jsel = ceil(C / 2)) the larger of the
        // two lanes' own jsel-th values.  Widened by both error bounds it screens both halves
        // in pass 2: the groups are disjoint, and a landmark counted by a BF16
        // group minimum has an exact key at most E16 above it and a pass-2 key
        // at most E2 above that, so the point has at least C candidates (jsel,
        // or 2 jsel); the certificate uses the pass-2 criterion itself.
        float tbase[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            int v0[16], v1[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                // approximate delta^2 as bit patterns; negative values (rounding)
                // become 0, and integer order is then float order
                v0[r] = max(__float_as_int(gmin[p][0][r] + xnp[p]), 0);
                v1[r] = max(__float_as_int(gmin[p][1][r] + xnp[p]), 0);
            }
            if (a.pair_select) {
                const int tl = min(select_pair_jth(v0, v1, a.jsel), 0x7F7FFFFF);  // +inf -> FLT_MAX
                tbase[p] = __int_as_float(tl);
            } else {
                const int tl = min(select_jth(v0, v1, a.jsel), 0x7F7FFFFF);
                const float own = __int_as_float(tl), oth = __int_as_float(__shfl_xor(tl, 32));
                tbase[p] = fmaxf(own, oth);
            }
        }

        // Pass-2 operands and their error bound e2.  BF16 mode splits the
        // point operand as x' = hi + lo + r (hi the pass-1 operand, lo = bf16(x'
        // - hi), both differences exact in FP32) and the landmark operand as
        // a = ah + al + ra likewise (from the preparation), and forms ah.hi +
        // al.hi + ah.lo, three BF16 products per element.  What it leaves out,
        // a.r - ra.r + al.lo + ra.x', is at most |r| (2 max|L - c| + max|ra|) +
        // max|al| |lo| + max|ra| |x'|; the FP32 accumulation of three chains of
        // d_pad products adds (6 d_pad + 16) u (|x'| + max|L - c|)^2 (the
        // single chain's allowance tripled).  |lo| and |r| are exact per point
        // (the rows are read again: still in cache).  FP32 mode's FP32 operand
        // is exact (e32).
        float e2[2];
        if constexpr (MODE == 1) {
            const float la = a.lmax[2], ra = a.lmax[3];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int64_t si = pbase + 32 * p + i32;
                const bool valid = si < a.n;
                const float *xr = a.X + (valid ? slot_point(a, si) : 0) * a.ldx;
                float lpart = 0.f, rpart = 0.f;
#pragma unroll
                for (int c = 0; c < DC; ++c) {
                    float v[8];
                    centred8(a, xr, centL, c, h, valid, v);
                    unsigned w[4];
#pragma unroll
                    for (int e = 0; e < 8; e += 2) {
                        const float r0 = v[e] - __uint_as_float(bf16_bits_rne(v[e]) << 16);
                        const float r1 = v[e + 1] - __uint_as_float(bf16_bits_rne(v[e + 1]) << 16);
                        const unsigned b0 = bf16_bits_rne(r0), b1 = bf16_bits_rne(r1);
                        const float l0 = __uint_as_float(b0 << 16), l1 = __uint_as_float(b1 << 16);
                        lpart = fmaf(l0, l0, lpart);
                        lpart = fmaf(l1, l1, lpart);
                        rpart = fmaf(r0 - l0, r0 - l0, rpart);
                        rpart = fmaf(r1 - l1, r1 - l1, rpart);
                        w[e >> 1] = b0 | (b1 << 16);
                    }
                    u32x4 wv = {w[0], w[1], w[2], w[3]};
                    P16lo.b[p][c] = __builtin_bit_cast(bf16x8, wv);
                }
                const float nlo = sqrtf(lpart + __shfl_xor(lpart, 32));
                const float nr = sqrtf(rpart + __shfl_xor(rpart, 32));
                const float sx = sqrtf(xnp[p]);
                const float facc3 = (6.f * DP + 16.f) * U32 * (sx + lmax) * (sx + lmax);
                e2[p] = 1.01f * (nr * (2.f * lmax + ra) + la * nlo + ra * sx + facc3);
            }
        } else {
            e2[0] = e32[0];
            e2[1] = e32[1];
        }

        float tau[2], taucert[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            tau[p] = (tbase[p] >= FLT_MAX) ? FLT_MAX : (tbase[p] - xnp[p]) + (e16[p] + e2[p]);
            taucert[p] = tau[p];
        }

        // FP32 mode: the FP32 operand of pass 2 (the rows are still in cache)
        PointOperand<0, DC> P32;
        if constexpr (MODE == 0) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int64_t si = pbase + 32 * p + i32;
                const bool valid = si < a.n;
                const float *xr = a.X + (valid ? slot_point(a, si) : 0) * a.ldx;
#pragma unroll
                for (int s = 0; s < 8 * DC; ++s) {
                    const int dd = 2 * s + h;
                    P32.b[p][s] = (valid && dd < a.d) ? xr[dd] - centL[dd] : 0.f;
                }
            }
        }

        // ---------------- pass 2: candidate bitmaps (key <= tau) into LDS.  The
        // sign of tau - key is shifted in (1 = not a candidate) and the word
        // complemented.  The two screen halves' words of a point and tile pair
        // sit side by side, bit-reversed, as one 64-bit word: bit 32 h + b is
        // position 64 tp + 2 b + h.  A mask per point marks the non-empty words.
        unsigned long long nonempty[2] = {0ull, 0ull};
        {
            unsigned word[2] = {0u, 0u};
            auto pass2_consume = [&](const f32x16 (&acc)[2], int) {
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        word[p] = __builtin_amdgcn_alignbit(word[p], __float_as_uint(tau[p] - acc[p][r]), 31);
            };
            auto pass2_store = [&](int tp) {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const unsigned wd = ~word[p];
                    bitsL[((p * W + tp) * 32 + i32) * 2 + h] = __builtin_bitreverse32(wd);
                    nonempty[p] |= (unsigned long long)(wd != 0u) << tp;
                }
            };
            // a skipped half shifts in 16 "not a candidate" bits
            auto pass2_consume_skip = [&](const f32x16 (&acc)[2], const bool (&need)[2]) {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    if (need[p]) {
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            word[p] = __builtin_amdgcn_alignbit(word[p], __float_as_uint(tau[p] - acc[p][r]), 31);
                    } else {
                        word[p] = (word[p] << 16) | 0xFFFFu;
                    }
                }
            };
            // the skip threshold tau + E16 + E2, rounded up
            float thr[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const float w = e16[p] + e2[p];
                thr[p] = (tau[p] + w) + 4.f * U32 * (fabsf(tau[p]) + w);
            }
            if constexpr (MODE == 1) {
                if (a.pt_order) {
                    if (a.lds_tiles)
                        screen_pass_split_skip(BoolTag<true>{}, pass2_consume_skip, pass2_store, thr);
                    else
                        screen_pass_split_skip(BoolTag<false>{}, pass2_consume_skip, pass2_store, thr);
                } else if (a.lds_tiles) {
                    screen_pass_split(BoolTag<true>{}, pass2_consume, pass2_store);
                } else {
                    screen_pass_split(BoolTag<false>{}, pass2_consume, pass2_store);
                }
            } else {
                // (FP32 mode skips from 48 padded dimensions on, where the FP32
                // products cost most; below, the BF16 operand is not kept live
                // through pass 2, which leaves the 12-wave blocks their registers)
                bool done = false;
                if constexpr (DC >= 3) {
                    if (a.pt_order) {
                        if (a.lds_tiles)
                            screen_pass_fp32_skip(BoolTag<true>{}, P32, pass2_consume_skip, pass2_store, thr);
                        else
                            screen_pass_fp32_skip(BoolTag<false>{}, P32, pass2_consume_skip, pass2_store, thr);
                        done = true;
                    }
                }
                if (!done) {
                    if (a.lds_tiles)
                        screen_pass(BoolTag<true>{}, IntTag<0>{}, P32, a.A, pass2_consume, pass2_store);
                    else
                        screen_pass(BoolTag<false>{}, IntTag<0>{}, P32, a.A, pass2_consume, pass2_store);
                }
            }
        }
        // Certificate bound per point: a non-candidate's exact distance^2
        // exceeds tau + |x - c|^2 - E, with E = e2 the error bound of the keys
        // pass 2 compared.
        if (h == 0) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const float E = e2[p];
                const float tc = taucert[p];
                float rhs = tc + xnp[p] - E;
                rhs -= 4.f * U32 * (fabsf(tc) + xnp[p] + E);
                certL[32 * p + i32] = (tc >= FLT_MAX) ? INFINITY : rhs;
            }
        }
        // masks of the points (p, i32): either screen half's word non-empty
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const unsigned long long both = nonempty[p] | __shfl_xor(nonempty[p], 32);
            if (h == 0) maskL[32 * p + i32] = both;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // ---------------- phase B: one lane per point (lane l <-> slot pbase + l)
        const bool valid = pbase + lane < a.n;
        const int64_t pi = valid ? slot_point(a, pbase + lane) : 0;  // the point's own index
        const float cert_rhs = certL[lane];
        float x[DP];
        {
            const float *xr = a.X + (valid ? pi : 0) * a.ldx;
            if (a.x_vec4) {
#pragma unroll
                for (int t = 0; t < DP / 4; ++t) {
                    const float4 v = reinterpret_cast<const float4 *>(xr)[t];
                    x[4 * t] = v.x;
                    x[4 * t + 1] = v.y;
                    x[4 * t + 2] = v.z;
                    x[4 * t + 3] = v.w;
                }
            } else {
#pragma unroll
                for (int t = 0; t < DP; ++t) x[t] = (t < a.d) ? xr[t < a.d ? t : a.d - 1] : 0.f;
            }
        }
        double sk[KP];
#pragma unroll
        for (int q = 0; q < KP; ++q) sk[q] = INFINITY;
        double rej = INFINITY;
        int m = 0;
        // Each lane walks its own candidates across all its words (one candidate
        // per iteration), so the wave iterates max_l m_l times.  The next
        // non-empty word is read one word ahead.  The loop is wave-uniform (it
        // ends when no lane has a candidate left); a lane without one rescores
        // landmark 0 and inserts +inf, which leaves its list unchanged.  Keeping
        // the insertion out of divergent control flow keeps the list in place
        // in registers.
        {
            unsigned long long mk = valid ? maskL[lane] : 0ull;
            const unsigned long long *row = reinterpret_cast<const unsigned long long *>(bitsL) + h * W * 32 + i32;
            int ntp = 0, ctp = 0;
            unsigned long long nb = 0ull, b = 0ull;
            next_word(mk, row, nb, ntp);
            for (;;) {
                if (b == 0ull && nb != 0ull) {
                    b = nb;
                    ctp = ntp;
                    next_word(mk, row, nb, ntp);
                }
                const bool act = b != 0ull;
                if (__ballot(act) == 0ull) break;
                const int bit = act ? __builtin_ctzll(b) : 0;
                b &= b - 1ull;
                // bit 32 h + pos of a word of tile pair ctp: position 64 ctp + 2 pos + h
                const int j = act ? 64 * ctp + 2 * (bit & 31) + (bit >> 5) : 0;
                float acc = 0.f;
                // rows from the block's LDS copy or from global memory (separate
                // code, so that each load has its own address space)
                auto add_row = [&](const float4 lv, int q) {
                    const float e0 = x[4 * q] - lv.x, e1 = x[4 * q + 1] - lv.y;
                    const float e2 = x[4 * q + 2] - lv.z, e3 = x[4 * q + 3] - lv.w;
                    acc = fmaf(e0, e0, acc);
                    acc = fmaf(e1, e1, acc);
                    acc = fmaf(e2, e2, acc);
                    acc = fmaf(e3, e3, acc);
                };
                if constexpr (ROWS == 1) {
                    const float4 *Lr = reinterpret_cast<const float4 *>(rowsL + row_offset<RS>(j));
#pragma unroll
                    for (int q = 0; q < DP / 4; ++q) add_row(Lr[q], q);
                } else {
                    const float4 *Lr = reinterpret_cast<const float4 *>(a.Lpad + (size_t)j * DP);
#pragma unroll
                    for (int q = 0; q < DP / 4; ++q) add_row(Lr[q], q);
                }
                // keys carry the landmark index (ties break on it), not the position
                insert_sorted<KP>(sk, rej, act ? pack_key(acc, permL[j]) : (double)INFINITY);
                m += act ? 1 : 0;
            }
        }
        __builtin_amdgcn_wave_barrier();

        // k-th and (k+1)-th rescored distances
        float d2k = 0.f, d2k1 = INFINITY;
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            if (q == a.k - 1) d2k = key_d2(sk[q]);
            if (q == a.k) d2k1 = key_d2(sk[q]);
        }
        if (a.k >= KP) d2k1 = (rej < INFINITY) ? key_d2(rej) : INFINITY;
        const float thr = kth_bound(m >= a.k ? d2k : INFINITY, DP);

        unsigned reason = 0;
        {
            const bool cert = d2k * (1.f + (DP + 3) * U32) < cert_rhs;
            if (!cert || m < a.k) reason |= R_UNCERT;
            // two rescored values are ordered correctly when their gap exceeds the sum
            // of their rounding bounds, (d_pad + 3) u each
            if (m > a.k && d2k1 - d2k <= 2.f * (DP + 3) * U32 * d2k1) reason |= R_NEARTIE;
            // When the caller asked for the neighbour list (its first entry is the
            // nearest landmark of the landmark update), adjacent entries closer
            // than the rounding bound go to the exact path too, so the list is
            // ordered by exact distance.  (The serving cache keeps the fast
            // path's own order, which is what a fresh projection uses.)
            if (a.knn_exact_order) {
                float prev = key_d2(sk[0]);
#pragma unroll
                for (int q = 1; q < KP; ++q) {
                    const float cur = key_d2(sk[q]);
                    if (q < a.k && q < m && cur - prev <= 2.f * (DP + 3) * U32 * cur) reason |= R_NEARTIE;
                    prev = cur;
                }
            }
        }

        // FP64 distances for small cutoff weights (k <= 8 only), while the
        // point's row is in registers; landmark rows from the LDS copy or the
        // padded array (zero past d in both).  A weight's FP32 error matters when
        // its pairs compete with gravity alone in some direction, which needs
        // the other neighbours' pairs to be rank-deficient in 2-D: plausible
        // for a few neighbours; with more, the strong pairs fix both directions
        // or the system is flagged as ill-conditioned.  At k <= 16 the code
        // alone cost 8% of this kernel (register pressure), used or not.
        float cref[N_REFINE] = {};
        int nref = 0;
        if constexpr (KP <= 8) {
            if (!a.knn_only) {
                // rows of more than 64 dimensions are read again from memory
                // instead of being kept in registers past the walk
                const float *xr = a.X + (valid ? pi : 0) * a.ldx;
                auto d2x = [&](int jl) -> double {
                    const unsigned pos = iposL[jl];
                    const float4 *Lr = ROWS ? reinterpret_cast<const float4 *>(rowsL + row_offset<RS>(pos))
                                                  : reinterpret_cast<const float4 *>(a.Lpad + (size_t)pos * DP);
                    double acc = 0.0;
                    auto add4 = [&](float4 xv, float4 lv) {
                        const double e0 = (double)xv.x - (double)lv.x;
                        const double e1 = (double)xv.y - (double)lv.y;
                        const double e2 = (double)xv.z - (double)lv.z;
                        const double e3 = (double)xv.w - (double)lv.w;
                        acc = fma(e0, e0, acc);
                        acc = fma(e1, e1, acc);
                        acc = fma(e2, e2, acc);
                        acc = fma(e3, e3, acc);
                    };
                    if constexpr (DC <= 4) {
#pragma unroll
                        for (int q = 0; q < DP / 4; ++q)
                            add4(make_float4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]), Lr[q]);
                    } else {
#pragma unroll 4
                        for (int q = 0; q < DP / 4; ++q) {
                            float4 xv;
                            if (a.x_vec4) {
                                xv = reinterpret_cast<const float4 *>(xr)[q];
                            } else {
                                xv.x = 4 * q < a.d ? xr[min(4 * q, a.d - 1)] : 0.f;
                                xv.y = 4 * q + 1 < a.d ? xr[min(4 * q + 1, a.d - 1)] : 0.f;
                                xv.z = 4 * q + 2 < a.d ? xr[min(4 * q + 2, a.d - 1)] : 0.f;
                                xv.w = 4 * q + 3 < a.d ? xr[min(4 * q + 3, a.d - 1)] : 0.f;
                            }
                            add4(xv, Lr[q]);
                        }
                    }
                    return acc;
                };
                reason |= refine_cutoffs<KP>(a, sk, valid, d2x, cref, nref);
            }
        }

        // knn outputs (the exact path rewrites those of uncertified / near-tie points)
        if (valid && a.knn_mark) a.knn_mark[pi] = (reason & (R_UNCERT | R_NEARTIE)) ? 1 : 0;
        if (valid && (a.knn_idx || a.knn_d2)) {
#pragma unroll
            for (int q = 0; q < KP; ++q) {
                if (q < a.k) {
                    if (a.knn_idx) a.knn_idx[pi * a.k + q] = key_idx(sk[q]);
                    if (a.knn_d2) a.knn_d2[pi * a.k + q] = key_d2(sk[q]);
                }
            }
        }

        if (!a.knn_only) {
            __builtin_amdgcn_wave_barrier();
            reason = project_point<KP>(a, sk, lane, valid, pi, reason, nbD2, nbS, nbI, iposL, cref, nref);
        }
        if (valid && reason) {
            const unsigned long long slot = atomicAdd(&a.counters[C_FB_LEN], 1ull);
            a.fb_list[slot] = (int32_t)pi;
            a.fb_reason[slot] = (uint8_t)reason;
            a.fb_thresh[slot] = thr;
        }
        st_cand += valid ? (unsigned long long)m : 0ull;
    }
    // wave-level totals
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) st_cand += __shfl_xor(st_cand, o);
    if (lane == 0 && st_cand) atomicAdd(&a.counters[C_CAND], st_cand);
}

}  // namespace esom
