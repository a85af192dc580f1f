// Readiness probes: what this GPU sustains right now, measured beside every benchmark (the
// paper checks each node with operational readiness scripts before use, sec. 8).
//   device_copy_kernel: plain streaming copy, 16 bytes per lane, one element per lane and as
//   many workgroups as elements / 256, so the running workgroups sweep memory in order (a
//   grid-stride loop over a fixed grid measured ~12 % slower); the HBM rate a streaming kernel
//   can reach, and the reference for calibrating the HBM traffic counters.  With a second
//   destination it writes every chunk twice: one byte read per two written, the mix of an F
//   stage that turns 4-byte samples into 8-byte ones.
//   mfma_probe_kernel: back-to-back dense MFMAs on register operands, eight independent
//   accumulator chains per wave, two workgroups of four waves per CU; the MFMA rate at the
//   clock the chip holds under that load.
#include "cobalt_internal.h"

namespace cobalt {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int intx16 __attribute__((ext_vector_type(16)));
typedef int intx4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void device_copy_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void device_fanout_kernel(uint4* __restrict__ dst0, uint4* __restrict__ dst1,
                                                            const uint4* __restrict__ src, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) {
        const uint4 v = src[i];
        dst0[i] = v;
        dst1[i] = v;
    }
}

constexpr int kChains = 8;

// Every operand element is 1, so after `iters` rounds each accumulator element holds
// iters * K (K = 16 for FP16, 32 for int8), exact for iters <= 2^19.  Each thread writes that
// value when all of its accumulator elements agree, else -1; the caller checks it.
template <int MODE>
__global__ __launch_bounds__(256, 2) void mfma_probe_kernel(int64_t iters, float* __restrict__ sink) {
    if constexpr (MODE == XM_FP16_SPLIT) {
        half8 one;
#pragma unroll
        for (int e = 0; e < 8; ++e) one[e] = (_Float16)1.0f;
        floatx16 acc[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = floatx16{};
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(one, one, acc[c], 0, 0, 0);
        }
        float v = acc[0][0];
#pragma unroll
        for (int c = 0; c < kChains; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) v = acc[c][r] == acc[0][0] ? v : -1.f;
        sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = v;
    } else {
        const intx4 one = {0x01010101, 0x01010101, 0x01010101, 0x01010101};
        intx16 acc[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = intx16{};
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(one, one, acc[c], 0, 0, 0);
        }
        int v = acc[0][0];
#pragma unroll
        for (int c = 0; c < kChains; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) v = acc[c][r] == acc[0][0] ? v : -1;
        sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = (float)v;
    }
}

}  // namespace

hipError_t launch_device_copy(void* dst, const void* src, int64_t bytes, hipStream_t st) {
    const int64_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const int64_t blocks = (n16 + 255) / 256;   // the loop in the kernel covers sizes beyond 2^30 workgroups
    hipLaunchKernelGGL(device_copy_kernel, dim3((unsigned)(blocks < (1 << 30) ? blocks : (1 << 30))), dim3(256), 0, st,
                       (uint4*)dst, (const uint4*)src, n16);
    return hipGetLastError();
}

hipError_t launch_device_fanout(void* dst0, void* dst1, const void* src, int64_t bytes, hipStream_t st) {
    const int64_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const int64_t blocks = (n16 + 255) / 256;
    hipLaunchKernelGGL(device_fanout_kernel, dim3((unsigned)(blocks < (1 << 30) ? blocks : (1 << 30))), dim3(256), 0, st,
                       (uint4*)dst0, (uint4*)dst1, (const uint4*)src, n16);
    return hipGetLastError();
}

hipError_t launch_mfma_probe(int x_mode, int64_t iters, int workgroups, float* sink, hipStream_t st) {
    if (workgroups <= 0) return hipSuccess;
    switch (x_mode) {
        case XM_FP16_SPLIT:
            hipLaunchKernelGGL(mfma_probe_kernel<XM_FP16_SPLIT>, dim3((unsigned)workgroups), dim3(256), 0, st, iters, sink);
            break;
        case XM_INT8:
            hipLaunchKernelGGL(mfma_probe_kernel<XM_INT8>, dim3((unsigned)workgroups), dim3(256), 0, st, iters, sink);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cobalt
