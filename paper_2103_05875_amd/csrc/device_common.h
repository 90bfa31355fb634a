// Device helpers shared by the kernels of the probe-volume library.
#pragma once

#include <hip/hip_fp16.h>

#include "internal.h"

namespace pv {

constexpr int kStack = kStack4;
// A texel whose weight sum is at most this keeps its old value: no ray falls
// usefully inside its lobe. Far above where FP32 weights underflow.
constexpr float kWeightFloor = 1e-20f;

// ---------------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 xyz(float4 a) { return make_float3(a.x, a.y, a.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z), fmaf(a.x, b.y, -a.y * b.x));
}

// XCD-aware block order: the hardware deals consecutive workgroups to the 8
// XCDs in turn; renumber so that each XCD runs one contiguous range of the
// logical work (neighbouring rays share that XCD's L2).
__device__ __forceinline__ int xcd_logical_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

}  // namespace pv
