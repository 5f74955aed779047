// Batch landmark update: nearest-landmark sums and counts, then a k-means or
// batch-SOM blend (semi-supervised model update of the paper's supervision
// section, in data-parallel batch form).
//
// Points are bucketed by nearest landmark with a counting sort (per-block
// LDS histograms, one global scan, per-block range claims), then every
// bucket's rows are summed in FP64 in chunks with coalesced row reads.  FP64
// sums make the result independent of the visiting order up to FP64
// rounding, far below the FP32 output rounding.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "esom_internal.h"

namespace esom {

constexpr int UPD_BLOCK = 256;
constexpr int UPD_CHUNK = 4096;  // points per histogram block / per summing chunk
constexpr int UPD_SCAN = 1024;   // threads of the scan block

// counts[j] += number of points whose nearest landmark is j.
__global__ void upd_hist(const int32_t *__restrict__ nearest, int64_t ld, int64_t n, int g,
                         int *__restrict__ counts) {
    extern __shared__ int hist[];
    for (int j = threadIdx.x; j < g; j += blockDim.x) hist[j] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * UPD_CHUNK;
    const int64_t b1 = b0 + UPD_CHUNK < n ? b0 + UPD_CHUNK : n;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        const int j = nearest[i * ld];
        if (j >= 0 && j < g) atomicAdd(&hist[j], 1);  // invalid indices are ignored
    }
    __syncthreads();
    for (int j = threadIdx.x; j < g; j += blockDim.x)
        if (hist[j]) atomicAdd(&counts[j], hist[j]);
}

// Exclusive scans of the counts (offsets[0..g], cursors) and of the chunks per
// landmark (ceil(count / UPD_CHUNK)), then the chunk table: chunk c covers
// [chunk_start, +UPD_CHUNK) of landmark chunk_landmark's range, landmark by
// landmark.  One block; each thread owns a contiguous run of landmarks.
__global__ void __launch_bounds__(UPD_SCAN) upd_scan(const int *__restrict__ counts, int g,
                                                     int64_t *__restrict__ offsets,
                                                     unsigned long long *__restrict__ cursor,
                                                     int *__restrict__ chunk_landmark,
                                                     int *__restrict__ chunk_start, int *__restrict__ nchunks) {
    __shared__ long long sp[UPD_SCAN];
    __shared__ int sc[UPD_SCAN];
    const int per = (g + UPD_SCAN - 1) / UPD_SCAN;
    const int j0 = threadIdx.x * per, j1 = j0 + per < g ? j0 + per : g;
    long long pts = 0;
    int chk = 0;
    for (int j = j0; j < j1; ++j) {
        pts += counts[j];
        chk += (counts[j] + UPD_CHUNK - 1) / UPD_CHUNK;
    }
    sp[threadIdx.x] = pts;
    sc[threadIdx.x] = chk;
    __syncthreads();
    // inclusive Hillis-Steele scans of the per-thread totals
    for (int o = 1; o < UPD_SCAN; o <<= 1) {
        const long long a = threadIdx.x >= o ? sp[threadIdx.x - o] : 0;
        const int b = threadIdx.x >= o ? sc[threadIdx.x - o] : 0;
        __syncthreads();
        sp[threadIdx.x] += a;
        sc[threadIdx.x] += b;
        __syncthreads();
    }
    long long run = sp[threadIdx.x] - pts;
    int c = sc[threadIdx.x] - chk;
    for (int j = j0; j < j1; ++j) {
        offsets[j] = run;
        cursor[j] = (unsigned long long)run;
        run += counts[j];
        for (int s0 = 0; s0 < counts[j]; s0 += UPD_CHUNK) {
            chunk_landmark[c] = j;
            chunk_start[c] = s0;
            ++c;
        }
    }
    if (threadIdx.x == UPD_SCAN - 1) {
        offsets[g] = sp[UPD_SCAN - 1];
        *nchunks = sc[UPD_SCAN - 1];
    }
}

// Scatter point indices into their landmark's range.
__global__ void upd_scatter(const int32_t *__restrict__ nearest, int64_t ld, int64_t n, int g,
                            unsigned long long *__restrict__ cursor, int32_t *__restrict__ perm) {
    extern __shared__ int sh[];
    int *hist = sh;                                               // g: block histogram
    int *base = sh + g;                                           // g: next slot in the claim
    long long *claim = reinterpret_cast<long long *>(sh + 2 * g);  // g: this block's range start
    for (int j = threadIdx.x; j < g; j += blockDim.x) hist[j] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * UPD_CHUNK;
    const int64_t b1 = b0 + UPD_CHUNK < n ? b0 + UPD_CHUNK : n;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        const int j = nearest[i * ld];
        if (j >= 0 && j < g) atomicAdd(&hist[j], 1);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < g; j += blockDim.x) {
        base[j] = 0;
        claim[j] = hist[j] ? (long long)atomicAdd(&cursor[j], (unsigned long long)hist[j]) : 0;
    }
    __syncthreads();
    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        const int j = nearest[i * ld];
        if (j < 0 || j >= g) continue;
        const int pos = atomicAdd(&base[j], 1);
        perm[claim[j] + pos] = (int32_t)i;
    }
}

// FP64 sums of the rows in one chunk of one landmark's range.  Block = one
// chunk; threads stride over dimensions (rows are read contiguously).
__global__ void upd_sum(const float *__restrict__ X, int64_t ldx, int d,
                        const int32_t *__restrict__ perm, const int64_t *__restrict__ offsets,
                        const int *__restrict__ chunk_landmark, const int *__restrict__ chunk_start,
                        const int *__restrict__ nchunks, double *__restrict__ sums) {
    const int c = blockIdx.x;
    if (c >= *nchunks) return;
    const int j = chunk_landmark[c];
    const int64_t beg = offsets[j] + (int64_t)chunk_start[c];
    int64_t end = beg + UPD_CHUNK;
    if (end > offsets[j + 1]) end = offsets[j + 1];
    // Several rows per pass: the block is split into groups of `tpr` threads per row.
    const int tpr = d <= 32 ? 32 : 64;
    const int rows_per_pass = blockDim.x / tpr;
    const int sub = threadIdx.x / tpr, t0 = threadIdx.x % tpr;
    __shared__ double red[UPD_BLOCK / 32][ESOM_MAX_D];
    double acc[ESOM_MAX_D / 32];
#pragma unroll
    for (int q = 0; q < ESOM_MAX_D / 32; ++q) acc[q] = 0.0;
    for (int64_t r = beg + sub; r < end; r += rows_per_pass) {
        const float *xr = X + (int64_t)perm[r] * ldx;
#pragma unroll
        for (int q = 0; q < ESOM_MAX_D / 32; ++q) {
            const int t = t0 + q * tpr;
            if (t < d) acc[q] += (double)xr[t];
        }
    }
#pragma unroll
    for (int q = 0; q < ESOM_MAX_D / 32; ++q) {
        const int t = t0 + q * tpr;
        if (t < d) red[sub][t] = acc[q];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < d; t += blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < rows_per_pass; ++q) s += red[q][t];
        atomicAdd(&sums[(size_t)j * (d + 1) + t], s);
    }
    if (threadIdx.x == 0) atomicAdd(&sums[(size_t)j * (d + 1) + d], (double)(end - beg));
}

// Blend: one block per landmark j, threads over dimensions.  kind 0: k-means;
// kind 1: batch SOM; kind 2: one online SOM step over a batch of `batch`
// points, the average of the single-point online updates
//   L_j += (alpha / batch) sum_b h_jb (S_b - c_b L_j),
// skipping landmarks with frozen[j] != 0.
__global__ void upd_finalize(const double *__restrict__ sums, const float *__restrict__ l2d, int g,
                             int d, int kind, float alpha, float sigma, float *__restrict__ L,
                             const int *__restrict__ counts, int32_t *__restrict__ counts_out,
                             const uint8_t *__restrict__ frozen, int64_t batch) {
    const int j = blockIdx.x;
    if (j >= g) return;
    if (counts_out && threadIdx.x == 0) counts_out[j] = counts[j];
    if (kind == 2 && frozen && frozen[j]) return;
    double den = 0.0;
    const double s2 = 2.0 * (double)sigma * (double)sigma;
    if (kind == 0) {
        den = sums[(size_t)j * (d + 1) + d];
    } else {
        for (int b = 0; b < g; ++b) {
            double hjb;
            if (sigma == 0.f) {
                hjb = b == j ? 1.0 : 0.0;
            } else {
                const double dx = (double)l2d[2 * j] - (double)l2d[2 * b];
                const double dy = (double)l2d[2 * j + 1] - (double)l2d[2 * b + 1];
                hjb = exp(-(dx * dx + dy * dy) / s2);
            }
            den += hjb * sums[(size_t)b * (d + 1) + d];
        }
    }
    for (int t = threadIdx.x; t < d; t += blockDim.x) {
        double num = 0.0;
        if (kind == 0) {
            num = sums[(size_t)j * (d + 1) + t];
        } else {
            for (int b = 0; b < g; ++b) {
                double hjb;
                if (sigma == 0.f) {
                    hjb = b == j ? 1.0 : 0.0;
                } else {
                    const double dx = (double)l2d[2 * j] - (double)l2d[2 * b];
                    const double dy = (double)l2d[2 * j + 1] - (double)l2d[2 * b + 1];
                    hjb = exp(-(dx * dx + dy * dy) / s2);
                }
                num += hjb * sums[(size_t)b * (d + 1) + t];
            }
        }
        const double Lj = (double)L[(size_t)j * d + t];
        if (kind == 2)
            L[(size_t)j * d + t] = (float)(Lj + (double)alpha / (double)batch * (num - den * Lj));
        else if (den > 0.0)
            L[(size_t)j * d + t] = (float)(Lj + (double)alpha * (num / den - Lj));
    }
}

__global__ void upd_zero(double *__restrict__ sums, size_t ns, int *__restrict__ counts, int g) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < ns) sums[e] = 0.0;
    if (e < (size_t)g) counts[e] = 0;
}

// Workspace layout (bytes, each region 256-aligned), computed by the caller.
size_t update_workspace_bytes(int64_t n, int g, int d) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const int64_t maxchunks = n / UPD_CHUNK + g + 1;
    return al(sizeof(double) * (size_t)g * (d + 1)) + al(sizeof(int) * g) +
           al(sizeof(int64_t) * (g + 1)) + al(sizeof(unsigned long long) * g) +
           al(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)) + 2 * al(sizeof(int) * (size_t)maxchunks) +
           al(sizeof(int));
}

hipError_t launch_update(const UpdateArgs &u, void *ws, int num_cus, hipStream_t s) {
    (void)num_cus;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = static_cast<char *>(ws);
    double *sums = reinterpret_cast<double *>(p);
    p += al(sizeof(double) * (size_t)u.g * (u.d + 1));
    int *counts = reinterpret_cast<int *>(p);
    p += al(sizeof(int) * u.g);
    int64_t *offsets = reinterpret_cast<int64_t *>(p);
    p += al(sizeof(int64_t) * (u.g + 1));
    unsigned long long *cursor = reinterpret_cast<unsigned long long *>(p);
    p += al(sizeof(unsigned long long) * u.g);
    int32_t *perm = reinterpret_cast<int32_t *>(p);
    p += al(sizeof(int32_t) * (size_t)(u.n > 0 ? u.n : 1));
    const int64_t maxchunks = u.n / UPD_CHUNK + u.g + 1;
    int *chunk_landmark = reinterpret_cast<int *>(p);
    p += al(sizeof(int) * (size_t)maxchunks);
    int *chunk_start = reinterpret_cast<int *>(p);
    p += al(sizeof(int) * (size_t)maxchunks);
    int *nchunks = reinterpret_cast<int *>(p);

    const size_t ns = (size_t)u.g * (u.d + 1);
    const size_t nz = ns > (size_t)u.g ? ns : (size_t)u.g;
    hipLaunchKernelGGL(upd_zero, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, sums, ns,
                       counts, u.g);
    const unsigned hblocks = (unsigned)((u.n + UPD_CHUNK - 1) / UPD_CHUNK);
    if (u.n > 0) {
        hipLaunchKernelGGL(upd_hist, dim3(hblocks), dim3(UPD_BLOCK), sizeof(int) * u.g, s, u.nearest,
                           u.nearest_ld, u.n, u.g, counts);
    }
    hipLaunchKernelGGL(upd_scan, dim3(1), dim3(UPD_SCAN), 0, s, counts, u.g, offsets, cursor,
                       chunk_landmark, chunk_start, nchunks);
    if (u.n > 0) {
        const size_t sh = sizeof(int) * 2 * (size_t)u.g + sizeof(long long) * (size_t)u.g;
        hipLaunchKernelGGL(upd_scatter, dim3(hblocks), dim3(UPD_BLOCK), sh, s, u.nearest, u.nearest_ld,
                           u.n, u.g, cursor, perm);
        // Grid sized for the worst case; blocks past the chunk count exit at once.
        hipLaunchKernelGGL(upd_sum, dim3((unsigned)maxchunks), dim3(UPD_BLOCK), 0, s, u.X, u.ldx,
                           u.d, perm, offsets, chunk_landmark, chunk_start, nchunks, sums);
    }
    hipLaunchKernelGGL(upd_finalize, dim3(u.g), dim3(u.d < 256 ? 64 * ((u.d + 63) / 64) : 256), 0, s,
                       sums, u.l2d, u.g, u.d, u.kind, u.alpha, u.sigma, u.L, counts, u.counts,
                       u.frozen, u.batch);
    return hipGetLastError();
}

}  // namespace esom
