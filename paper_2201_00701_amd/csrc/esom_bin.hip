// Locality order of the points for the fused kernel.
//
// The fused kernel's cost at large landmark sets depends on how much the 64
// points of a wavefront share: candidate bitmap words, landmark rows and,
// above all, pair-table lines (g x g entries; 4 MB at g = 1024, which the
// point stream evicts from L2).  Points in input order share little.  Here
// every point gets its nearest of 64 ordering pivots (the landmarks j g / 64,
// the landmark preparation's pivots), and a counting sort by pivot gives the
// fused kernel its processing order; the outputs still go to the points' own
// rows.  The order has no effect on any result.  It needs nothing from the
// landmark preparation, so a context runs it on a second stream beside that.
//
//   bin_zero     clears the counts;
//   bin_keys     one wavefront per 64 points (persistent): the 64 pivots as
//                a BF16 MFMA A operand centred on landmark 0 (built once per
//                block in LDS), keys |P_i - c0|^2 - 2 <x - c0, P_i - c0> for
//                both 32-point halves, the argmin per point (BF16 keys: an
//                approximate nearest pivot, which is all an order needs) into
//                cell[], and a per-block histogram added to hist;
//   bin_scatter  blocks of BIN_CHUNK points: the block's count per pivot, a
//                range per pivot claimed from the global cursors (offset by
//                the prefix sum of hist), and each point written to its slot
//                of order[].  Within a pivot, slots follow block order and,
//                inside a block, arrival order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "embed_kernel.h"
#include "esom_internal.h"

namespace esom {

constexpr int BIN_P = 64;        // ordering pivots (g >= BIN_MIN_G)
constexpr int BIN_WAVES = 4;     // wavefronts per bin_keys block
constexpr int BIN_CHUNK = 4096;  // points per bin_scatter block

__global__ void bin_zero(unsigned *hist) {
    if (threadIdx.x < 2 * BIN_P) hist[threadIdx.x] = 0u;
}

template <int DC>
__global__ void __launch_bounds__(64 * BIN_WAVES) bin_keys(BinArgs b) {
    // the centre (landmark 0, zero past d), the pivot operand (2 tiles x DC
    // chunks x 64 lanes) and its norms in accumulator order ([tile][lane
    // half][16])
    __shared__ float cen[16 * DC];
    __shared__ u32x4 As[2][DC][64];
    __shared__ float Ns[2][2][16];
    __shared__ unsigned hl[BIN_P];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5, i32 = lane & 31;
    if (threadIdx.x < BIN_P) hl[threadIdx.x] = 0u;
    for (int e = threadIdx.x; e < 16 * DC; e += blockDim.x) cen[e] = e < b.d ? b.L[e] : 0.f;
    __syncthreads();
    if (wave == 0) {
        // tile t, row m = lane mod 32 is pivot i = 32 t + m (landmark i g / 64);
        // lane l holds dimensions 16 c + 8 h + e of its row (MFMA A layout)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int64_t j = ((int64_t)(32 * t + i32) * b.g) / BIN_P;
            const float *Lr = b.L + j * b.d;
            float part = 0.f;
#pragma unroll
            for (int c = 0; c < DC; ++c) {
                unsigned w[4];
#pragma unroll
                for (int e = 0; e < 8; e += 2) {
                    const int q0 = 16 * c + 8 * h + e;
                    const float v0 = q0 < b.d ? Lr[q0] - cen[q0] : 0.f;
                    const float v1 = q0 + 1 < b.d ? Lr[q0 + 1] - cen[q0 + 1] : 0.f;
                    part = fmaf(v0, v0, part);
                    part = fmaf(v1, v1, part);
                    w[e >> 1] = bf16_bits_rne(-2.f * v0) | (bf16_bits_rne(-2.f * v1) << 16);
                }
                As[t][c][lane] = u32x4{w[0], w[1], w[2], w[3]};
            }
            const float nr = part + __shfl_xor(part, 32);  // row m's |P - c0|^2 on lanes m, m + 32
            // row m sits in lane half (m / 4) % 2, register 4 (m / 8) + m % 4
            if (h == 0) Ns[t][(i32 >> 2) & 1][4 * (i32 >> 3) + (i32 & 3)] = nr;
        }
    }
    __syncthreads();

    const int64_t nwt = (b.n + 63) / 64;
    for (int64_t wt = (int64_t)wave * gridDim.x + blockIdx.x; wt < nwt; wt += (int64_t)gridDim.x * BIN_WAVES) {
        const int64_t pbase = wt * 64;
        bf16x8 P[2][DC];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int64_t pi = pbase + 32 * p + i32;
            const bool valid = pi < b.n;
            const float *xr = b.X + (valid ? pi : 0) * b.ldx;
#pragma unroll
            for (int c = 0; c < DC; ++c) {
                float v[8];
                if (b.x_vec4) {
                    const float4 *x4 = reinterpret_cast<const float4 *>(xr + 16 * c + 8 * h);
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const float4 q = valid ? x4[u] : make_float4(0.f, 0.f, 0.f, 0.f);
                        const int q0 = 16 * c + 8 * h + 4 * u;
                        v[4 * u] = q.x - cen[q0];
                        v[4 * u + 1] = q.y - cen[q0 + 1];
                        v[4 * u + 2] = q.z - cen[q0 + 2];
                        v[4 * u + 3] = q.w - cen[q0 + 3];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int q = 16 * c + 8 * h + e;
                        v[e] = (valid && q < b.d) ? xr[q] - cen[q] : 0.f;
                    }
                }
                unsigned w[4];
#pragma unroll
                for (int e = 0; e < 8; e += 2) w[e >> 1] = bf16_bits_rne(v[e]) | (bf16_bits_rne(v[e + 1]) << 16);
                P[p][c] = __builtin_bit_cast(bf16x8, u32x4{w[0], w[1], w[2], w[3]});
            }
        }
        // argmin over the lane's 32 rows (two tiles), then over both lane halves
        float best[2] = {INFINITY, INFINITY};
        int brow[2] = {0, 0};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            f32x16 acc[2];
            {
                const float4 *np = reinterpret_cast<const float4 *>(&Ns[t][h][0]);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float4 nv = np[i];
                    acc[0][4 * i] = nv.x;
                    acc[0][4 * i + 1] = nv.y;
                    acc[0][4 * i + 2] = nv.z;
                    acc[0][4 * i + 3] = nv.w;
                }
                acc[1] = acc[0];
            }
#pragma unroll
            for (int c = 0; c < DC; ++c) {
                const bf16x8 av = __builtin_bit_cast(bf16x8, As[t][c][lane]);
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, P[0][c], acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, P[1][c], acc[1], 0, 0, 0);
            }
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = 32 * t + 8 * (r >> 2) + 4 * h + (r & 3);
                    if (acc[p][r] < best[p]) {
                        best[p] = acc[p][r];
                        brow[p] = row;
                    }
                }
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const float ob = __shfl_xor(best[p], 32);
            const int orow = __shfl_xor(brow[p], 32);
            if (ob < best[p] || (ob == best[p] && orow < brow[p])) brow[p] = orow;
        }
        // lane l records point pbase + l (its half's result)
        const int64_t pi = pbase + lane;
        if (pi < b.n) {
            const int cell = h ? brow[1] : brow[0];
            b.cell[pi] = (uint8_t)cell;
            atomicAdd(&hl[cell], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < BIN_P && hl[threadIdx.x]) atomicAdd(&b.hist[threadIdx.x], hl[threadIdx.x]);
}

__global__ void __launch_bounds__(256) bin_scatter(BinArgs b) {
    __shared__ unsigned cnt[BIN_P], fill[BIN_P], base[BIN_P];
    const int64_t i0 = (int64_t)blockIdx.x * BIN_CHUNK;
    const int64_t i1 = i0 + BIN_CHUNK < b.n ? i0 + BIN_CHUNK : b.n;
    if (threadIdx.x < BIN_P) {
        cnt[threadIdx.x] = 0u;
        fill[threadIdx.x] = 0u;
    }
    __syncthreads();
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) atomicAdd(&cnt[b.cell[i]], 1u);
    __syncthreads();
    if (threadIdx.x < BIN_P) {
        // exclusive prefix sum of the places' totals, plus this block's claim
        const unsigned v = b.hist[threadIdx.x];
        unsigned incl = v;
#pragma unroll
        for (int o = 1; o < BIN_P; o <<= 1) {
            const unsigned t = __shfl_up(incl, o);
            if ((int)threadIdx.x >= o) incl += t;
        }
        base[threadIdx.x] = (incl - v) + (cnt[threadIdx.x] ? atomicAdd(&b.hist[BIN_P + threadIdx.x], cnt[threadIdx.x]) : 0u);
    }
    __syncthreads();
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const int c = b.cell[i];
        b.order[base[c] + atomicAdd(&fill[c], 1u)] = (int32_t)i;
    }
}

template <int DC>
static void launch_keys(const BinArgs &b, unsigned blocks, hipStream_t s) {
    hipLaunchKernelGGL(bin_keys<DC>, dim3(blocks), dim3(64 * BIN_WAVES), 0, s, b);
}

hipError_t launch_bin(const BinArgs &b, int num_cus, hipStream_t s) {
    hipLaunchKernelGGL(bin_zero, dim3(1), dim3(2 * BIN_P), 0, s, b.hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    long long blocks = ((b.n + 63) / 64 + BIN_WAVES - 1) / BIN_WAVES;
    if (blocks > (long long)num_cus * 2) blocks = (long long)num_cus * 2;
    if (blocks < 1) blocks = 1;
    switch (b.dp / 16) {
        case 1: launch_keys<1>(b, (unsigned)blocks, s); break;
        case 2: launch_keys<2>(b, (unsigned)blocks, s); break;
        case 3: launch_keys<3>(b, (unsigned)blocks, s); break;
        case 4: launch_keys<4>(b, (unsigned)blocks, s); break;
        case 5: launch_keys<5>(b, (unsigned)blocks, s); break;
        case 6: launch_keys<6>(b, (unsigned)blocks, s); break;
        case 7: launch_keys<7>(b, (unsigned)blocks, s); break;
        case 8: launch_keys<8>(b, (unsigned)blocks, s); break;
        default: return hipErrorInvalidValue;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long sblocks = (b.n + BIN_CHUNK - 1) / BIN_CHUNK;
    hipLaunchKernelGGL(bin_scatter, dim3((unsigned)(sblocks > 0 ? sblocks : 1)), dim3(256), 0, s, b);
    return hipGetLastError();
}

}  // namespace esom
