// Instantiates the dock kernel for BF16 texels.
#include "dock_kernels.inc"
#include "gather_probe.inc"

namespace exs {

hipError_t launch_dock_bf16(const DockArgs& a, int ppl, dim3 grid, dim3 block, size_t lds,
                           hipStream_t st) {
#define EXS_LAUNCH(SS, PP) \
    if (a.S == SS && ppl == PP) { \
        hipLaunchKernelGGL((dock_kernel<SS, PP, TexBF16>), grid, block, lds, st, a); \
        return hipGetLastError(); \
    }
    EXS_LAUNCH(8, 1) EXS_LAUNCH(8, 2) EXS_LAUNCH(8, 4) EXS_LAUNCH(16, 1) EXS_LAUNCH(16, 2)
    EXS_LAUNCH(16, 4) EXS_LAUNCH(32, 1) EXS_LAUNCH(32, 2) EXS_LAUNCH(32, 4)
#undef EXS_LAUNCH
    return hipErrorInvalidValue;
}

const void* dock_kernel_fn_bf16(int S, int ppl) {
#define EXS_FN(SS, PP) \
    if (S == SS && ppl == PP) return reinterpret_cast<const void*>(&dock_kernel<SS, PP, TexBF16>);
    EXS_FN(8, 1) EXS_FN(8, 2) EXS_FN(8, 4) EXS_FN(16, 1) EXS_FN(16, 2) EXS_FN(16, 4)
    EXS_FN(32, 1) EXS_FN(32, 2) EXS_FN(32, 4)
#undef EXS_FN
    return nullptr;
}

hipError_t launch_gather_probe_bf16(const GridDesc* gd, int nb, int64_t blocks, int per_lane,
                                float half, float walk, uint32_t seed, float* out, hipStream_t st) {
    const dim3 grid((unsigned)blocks), block(256);
    switch (nb) {
        case 8: hipLaunchKernelGGL((gather_probe_kernel<TexBF16, 8>), grid, block, 0, st, gd, per_lane, half, walk, seed, out); break;
        case 16: hipLaunchKernelGGL((gather_probe_kernel<TexBF16, 16>), grid, block, 0, st, gd, per_lane, half, walk, seed, out); break;
        case 32: hipLaunchKernelGGL((gather_probe_kernel<TexBF16, 32>), grid, block, 0, st, gd, per_lane, half, walk, seed, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t upload_trig_bf16(const float* t32, const double* t64) {
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_trig32), t32, sizeof(float) * kTrigEntries);
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_trig64), t64, sizeof(double) * kTrigEntries);
}

}  // namespace exs
