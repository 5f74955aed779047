// Graph-mode supervision (Section "Semi-supervised structure reconstruction"):
// the neighbourhood graph of the high-dimensional landmarks, a force-based
// layout of their 2-D positions on that graph, and the duplication and
// removal of landmarks.  The paper names no graph or force law; the graph is
// the kg nearest other landmarks of every landmark and the force law is a
// spring per edge (rest length proportional to the high-dimensional distance)
// plus a softened all-pairs repulsion.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "esom_internal.h"

namespace esom {

// Lexicographic order on (squared distance, index).
__device__ __forceinline__ bool pair_before(double da, int ia, double db, int ib) {
    return da < db || (da == db && ia < ib);
}

// One wavefront per landmark u: every lane scans the landmarks v = lane,
// lane + 64, ... (v != u), keeps its GRAPH_MAX_K nearest in a sorted register
// list, then the wave merges the 64 lists by kg rounds of a wave-wide minimum.
// Distances are FP64 sums of squared differences, added in dimension order
// without fused multiply-adds, so equal distances compare equal exactly as
// in a plain double-precision evaluation.
__global__ void __launch_bounds__(256) landmark_graph_kernel(const float *__restrict__ L, int g, int d,
                                                             int kg, int32_t *__restrict__ nbr,
                                                             float *__restrict__ dist2) {
    const int lane = threadIdx.x & 63;
    const int u = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (u >= g) return;  // whole wavefronts exit together (u is wave-uniform)
    double bd[GRAPH_MAX_K];
    int bi[GRAPH_MAX_K];
#pragma unroll
    for (int q = 0; q < GRAPH_MAX_K; ++q) {
        bd[q] = INFINITY;
        bi[q] = INT32_MAX;
    }
    const float *Lu = L + (size_t)u * d;
    for (int v = lane; v < g; v += 64) {
        if (v == u) continue;
        const float *Lv = L + (size_t)v * d;
        double s = 0.0;
        for (int t = 0; t < d; ++t) {
            const double df = (double)Lv[t] - (double)Lu[t];
            s = __dadd_rn(s, __dmul_rn(df, df));
        }
        // insertion into the lane's sorted list (the list holds at most kg)
        double cd = s;
        int ci = v;
#pragma unroll
        for (int q = 0; q < GRAPH_MAX_K; ++q) {
            if (q < kg && pair_before(cd, ci, bd[q], bi[q])) {
                const double td = bd[q];
                const int ti = bi[q];
                bd[q] = cd;
                bi[q] = ci;
                cd = td;
                ci = ti;
            }
        }
    }
    // merge: kg rounds, each taking the wave-wide smallest head
    for (int r = 0; r < kg; ++r) {
        double md = bd[0];
        int mi = bi[0];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double od = __shfl_xor(md, o);
            const int oi = __shfl_xor(mi, o);
            if (pair_before(od, oi, md, mi)) {
                md = od;
                mi = oi;
            }
        }
        if (lane == 0) {
            nbr[(size_t)u * kg + r] = mi < g ? mi : -1;
            if (dist2) dist2[(size_t)u * kg + r] = mi < g ? (float)md : INFINITY;
        }
        // the lane whose head was taken pops it (indices are unique)
        if (bi[0] == mi && mi < g) {
#pragma unroll
            for (int q = 0; q + 1 < GRAPH_MAX_K; ++q) {
                bd[q] = bd[q + 1];
                bi[q] = bi[q + 1];
            }
            bd[GRAPH_MAX_K - 1] = INFINITY;
            bi[GRAPH_MAX_K - 1] = INT32_MAX;
        }
    }
}

hipError_t launch_landmark_graph(const float *L, int g, int d, int kg, int32_t *nbr, float *dist2,
                                 hipStream_t s) {
    const int waves_per_block = 4;
    const unsigned blocks = (unsigned)((g + waves_per_block - 1) / waves_per_block);
    hipLaunchKernelGGL(landmark_graph_kernel, dim3(blocks), dim3(64 * waves_per_block), 0, s, L, g, d, kg,
                       nbr, dist2);
    return hipGetLastError();
}

// One synchronous layout step, one thread per node u.  The landmarks v are
// visited in tiles of LAYOUT_TILE whose 2-D positions and neighbour lists are
// staged in LDS: every v repels u, and v pulls u along a spring when u-v is an
// edge (v in u's list or u in v's list; an edge listed both ways acts once).
// Forces and the move are summed in FP64 from the positions before the step
// (lin), the new positions go to lout.
constexpr int LAYOUT_TILE = 256;

__global__ void __launch_bounds__(LAYOUT_TILE) layout_step_kernel(
    const float *__restrict__ L, int g, int d, const int32_t *__restrict__ nbr, int kg,
    const float *__restrict__ lin, float *__restrict__ lout, const uint8_t *__restrict__ fixed,
    double scale, double repulsion, double soft2, double step, double max_move) {
    extern __shared__ __align__(16) unsigned char lsm[];
    float2 *tl = reinterpret_cast<float2 *>(lsm);                         // LAYOUT_TILE positions
    int32_t *tn = reinterpret_cast<int32_t *>(tl + LAYOUT_TILE);          // LAYOUT_TILE x kg
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = u < g;
    int32_t own[GRAPH_MAX_K];
#pragma unroll
    for (int q = 0; q < GRAPH_MAX_K; ++q) own[q] = (live && q < kg) ? nbr[(size_t)u * kg + q] : -1;
    const float2 pu = live ? reinterpret_cast<const float2 *>(lin)[u] : make_float2(0.f, 0.f);
    const double ux = pu.x, uy = pu.y;
    double fx = 0.0, fy = 0.0;
    for (int v0 = 0; v0 < g; v0 += LAYOUT_TILE) {
        const int nv = g - v0 < LAYOUT_TILE ? g - v0 : LAYOUT_TILE;
        __syncthreads();
        for (int e = threadIdx.x; e < nv; e += blockDim.x) tl[e] = reinterpret_cast<const float2 *>(lin)[v0 + e];
        for (int e = threadIdx.x; e < nv * kg; e += blockDim.x) tn[e] = nbr[(size_t)v0 * kg + e];
        __syncthreads();
        if (!live) continue;
        for (int e = 0; e < nv; ++e) {
            const int v = v0 + e;
            if (v == u) continue;
            const double dx = (double)tl[e].x - ux, dy = (double)tl[e].y - uy;
            const double r2 = dx * dx + dy * dy;
            bool edge = false;
#pragma unroll
            for (int q = 0; q < GRAPH_MAX_K; ++q) edge |= (q < kg && own[q] == v);
            for (int q = 0; q < kg && !edge; ++q) edge = tn[e * kg + q] == u;
            if (edge) {
                const double r = sqrt(r2);
                if (r > 0.0) {
                    const float *Lu = L + (size_t)u * d, *Lv = L + (size_t)v * d;
                    double hd = 0.0;
                    for (int t = 0; t < d; ++t) {
                        const double df = (double)Lu[t] - (double)Lv[t];
                        hd = fma(df, df, hd);
                    }
                    const double pull = (r - scale * sqrt(hd)) / r;
                    fx = fma(pull, dx, fx);
                    fy = fma(pull, dy, fy);
                }
            }
            const double push = repulsion / (r2 + soft2);
            fx = fma(-push, dx, fx);
            fy = fma(-push, dy, fy);
        }
    }
    if (!live) return;
    double mx = step * fx, my = step * fy;
    const double len = sqrt(mx * mx + my * my);
    if (len > max_move) {
        mx *= max_move / len;
        my *= max_move / len;
    }
    if (fixed && fixed[u]) mx = my = 0.0;
    reinterpret_cast<float2 *>(lout)[u] = make_float2((float)(ux + mx), (float)(uy + my));
}

hipError_t launch_layout_step(const float *L, int g, int d, const int32_t *nbr, int kg, const float *lin,
                              float *lout, const uint8_t *fixed, double scale, double repulsion,
                              double soft, double step, double max_move, hipStream_t s) {
    const unsigned blocks = (unsigned)((g + LAYOUT_TILE - 1) / LAYOUT_TILE);
    const size_t smem = sizeof(float2) * LAYOUT_TILE + sizeof(int32_t) * LAYOUT_TILE * kg;
    hipLaunchKernelGGL(layout_step_kernel, dim3(blocks), dim3(LAYOUT_TILE), smem, s, L, g, d, nbr, kg, lin,
                       lout, fixed, scale, repulsion, soft * soft, step, max_move);
    return hipGetLastError();
}

// Landmark g (a new row) := landmark j, 2-D position shifted by (dx, dy).
__global__ void duplicate_kernel(float *__restrict__ L, float *__restrict__ l2d, int g, int d, int j, float dx,
                                 float dy) {
    for (int t = threadIdx.x; t < d; t += blockDim.x) L[(size_t)g * d + t] = L[(size_t)j * d + t];
    if (threadIdx.x == 0) {
        l2d[2 * g] = l2d[2 * j] + dx;
        l2d[2 * g + 1] = l2d[2 * j + 1] + dy;
    }
}

// Landmark j := landmark g - 1 (the last row moves into the removed slot).
__global__ void remove_kernel(float *__restrict__ L, float *__restrict__ l2d, int g, int d, int j) {
    const int last = g - 1;
    for (int t = threadIdx.x; t < d; t += blockDim.x) L[(size_t)j * d + t] = L[(size_t)last * d + t];
    if (threadIdx.x == 0) {
        l2d[2 * j] = l2d[2 * last];
        l2d[2 * j + 1] = l2d[2 * last + 1];
    }
}

hipError_t launch_duplicate(float *L, float *l2d, int g, int d, int j, float dx, float dy, hipStream_t s) {
    hipLaunchKernelGGL(duplicate_kernel, dim3(1), dim3(256), 0, s, L, l2d, g, d, j, dx, dy);
    return hipGetLastError();
}

hipError_t launch_remove(float *L, float *l2d, int g, int d, int j, hipStream_t s) {
    hipLaunchKernelGGL(remove_kernel, dim3(1), dim3(256), 0, s, L, l2d, g, d, j);
    return hipGetLastError();
}

}  // namespace esom
