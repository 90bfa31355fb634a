// Attainable ceilings of the device, for reading the kernels' roofline
// fractions against what a plain kernel reaches rather than the data-sheet
// peaks:
//   k_ceil_copy  float4 stream copy (HBM read + write)
//   k_ceil_fma   eight independent FP32 FMA chains per thread (vector ALU,
//                built without packed FP32)
//   k_ceil_mfma  four independent 16x16x4 FP32 MFMA chains per wavefront
// Each writes a value derived from its chains so that no work is removed.
#include "device_common.h"

namespace pv {

typedef float v4f_c __attribute__((ext_vector_type(4)));

constexpr int kCeilThreads = 256;

__global__ __launch_bounds__(kCeilThreads) void k_ceil_copy(const float4 *src, float4 *dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kCeilThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kCeilThreads)
        dst[i] = src[i];
}

__global__ __launch_bounds__(kCeilThreads) void k_ceil_fma(float *out, int iters) {
    const float m = 0.999f, c = 1e-4f;
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f;
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = fmaf(a[k], m, c);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k];
    out[(size_t)blockIdx.x * kCeilThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kCeilThreads) void k_ceil_mfma(float *out, int iters) {
    const float a = (float)(threadIdx.x & 63) * 1e-4f, b = 1e-3f;
    v4f_c acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = v4f_c{0.f, 0.f, 0.f, (float)k};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[(size_t)blockIdx.x * kCeilThreads + threadIdx.x] = s;
}

hipError_t launch_ceil_copy(const void *src, void *dst, size_t bytes, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_ceil_copy, dim3(blocks), dim3(kCeilThreads), 0, s, (const float4 *)src, (float4 *)dst,
                       bytes / 16);
    return hipGetLastError();
}

hipError_t launch_ceil_fma(float *out, int blocks, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_ceil_fma, dim3(blocks), dim3(kCeilThreads), 0, s, out, iters);
    return hipGetLastError();
}

hipError_t launch_ceil_mfma(float *out, int blocks, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_ceil_mfma, dim3(blocks), dim3(kCeilThreads), 0, s, out, iters);
    return hipGetLastError();
}

}  // namespace pv
