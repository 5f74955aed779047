// Explicit instantiations of the fused kernel for one (mode, KP, KF) triple.
// Compiled once per triple with -DINST_MODE=<0|1> -DINST_KP=<8|16|20|24|32>
// -DINST_KF=<0|1> (KF = 1: k == KP, k < g).
#include "embed_kernel.h"

#ifndef INST_MODE
#error "INST_MODE must be defined"
#endif
#ifndef INST_KP
#error "INST_KP must be defined"
#endif
#ifndef INST_KF
#error "INST_KF must be defined"
#endif

#define ESOM_CAT2(a, b, c) a##b##c
#define ESOM_NAME(m, k, f) ESOM_CAT2(launch_main_m, m, _kp##k##_kf##f)
#define ESOM_LAUNCHER(m, k, f) ESOM_NAME(m, k, f)

namespace esom {

template <int MODE, int DC, int KP>
static hipError_t launch_dc(const EmbedArgs &a, int block, size_t smem, int num_cus, hipStream_t s) {
    constexpr int KF = INST_KF;
    auto kern = a.lds_rows ? embed_main<MODE, DC, KP, 1, KF> : embed_main<MODE, DC, KP, 0, KF>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, smem) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int wpb = block / 64;
    const long long waves = (a.n + 63) / 64;
    long long blocks = (waves + wpb - 1) / wpb;
    if (blocks > (long long)per_cu * num_cus) blocks = (long long)per_cu * num_cus;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(block), smem, s, a);
    return hipGetLastError();
}

hipError_t ESOM_LAUNCHER(INST_MODE, INST_KP, INST_KF)(const EmbedArgs &a, int dc, int block, size_t smem,
                                                      int num_cus, hipStream_t s) {
    constexpr int M = INST_MODE, K = INST_KP;
    switch (dc) {
        case 1: return launch_dc<M, 1, K>(a, block, smem, num_cus, s);
        case 2: return launch_dc<M, 2, K>(a, block, smem, num_cus, s);
        case 3: return launch_dc<M, 3, K>(a, block, smem, num_cus, s);
        case 4: return launch_dc<M, 4, K>(a, block, smem, num_cus, s);
#if INST_MODE == 1
        case 5: return launch_dc<M, 5, K>(a, block, smem, num_cus, s);
        case 6: return launch_dc<M, 6, K>(a, block, smem, num_cus, s);
        case 7: return launch_dc<M, 7, K>(a, block, smem, num_cus, s);
        case 8: return launch_dc<M, 8, K>(a, block, smem, num_cus, s);
#endif
        default: return hipErrorInvalidValue;
    }
}

}  // namespace esom
