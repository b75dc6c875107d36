// Measurement helper: achievable FP32 FMA throughput of the device (VALU,
// unpacked, as the simulation kernels are compiled).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cfsim.h"

namespace {

// eight independent FMA chains per lane; b and c are runtime values so the
// chains cannot be folded, and the sum is stored so they stay live.
// ACC = false: a <- a b + c (three-operand v_fma_f32);
// ACC = true:  a <- b c + a (two-operand accumulate form, v_fmac_f32).
template <bool ACC>
__global__ __launch_bounds__(256) void k_fma_probe(float* out, int iters, float b, float c) {
    float a0 = 1e-3f * (float)threadIdx.x, a1 = a0 + 1.f, a2 = a0 + 2.f, a3 = a0 + 3.f;
    float a4 = a0 + 4.f, a5 = a0 + 5.f, a6 = a0 + 6.f, a7 = a0 + 7.f;
    for (int i = 0; i < iters; ++i) {
        if constexpr (ACC) {
            a0 = __builtin_fmaf(b, c, a0); a1 = __builtin_fmaf(b, c, a1);
            a2 = __builtin_fmaf(b, c, a2); a3 = __builtin_fmaf(b, c, a3);
            a4 = __builtin_fmaf(b, c, a4); a5 = __builtin_fmaf(b, c, a5);
            a6 = __builtin_fmaf(b, c, a6); a7 = __builtin_fmaf(b, c, a7);
        } else {
            a0 = __builtin_fmaf(a0, b, c); a1 = __builtin_fmaf(a1, b, c);
            a2 = __builtin_fmaf(a2, b, c); a3 = __builtin_fmaf(a3, b, c);
            a4 = __builtin_fmaf(a4, b, c); a5 = __builtin_fmaf(a5, b, c);
            a6 = __builtin_fmaf(a6, b, c); a7 = __builtin_fmaf(a7, b, c);
        }
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

}  // namespace

extern "C" cf_status cf_probe_fma(float* out, int32_t n_blocks, int32_t iters, int32_t form, void* stream) {
    if (!out || n_blocks < 1 || iters < 1 || (form != 0 && form != 1)) return CF_EINVAL;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)out) != hipSuccess) {
        (void)hipGetLastError();
        return CF_EINVAL;
    }
    if ((size_t)((const char*)out - (const char*)base) + (size_t)n_blocks * 256 * sizeof(float) > size)
        return CF_EINVAL;
    if (form == 0)
        hipLaunchKernelGGL(k_fma_probe<false>, dim3((unsigned)n_blocks), dim3(256), 0, (hipStream_t)stream, out,
                           iters, 0.9999999f, 1e-7f);
    else
        hipLaunchKernelGGL(k_fma_probe<true>, dim3((unsigned)n_blocks), dim3(256), 0, (hipStream_t)stream, out,
                           iters, 1e-3f, 1e-4f);
    return hipGetLastError() == hipSuccess ? CF_OK : CF_EDEVICE;
}
