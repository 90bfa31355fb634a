// Ray directions and the blend kernel.
//   k_raydirs   spherical-Fibonacci ray set under the frame rotation (one
//               thread per ray); also clears the trace's work counters
//   k_blend     weighted means on the FP32 matrix cores, hysteresis, FP32 or
//               FP16 store, guard bands
#include "blend_device.h"

namespace pv {

constexpr int kDirThreads = 256;

// queue: the work counters of the trace that follows, zeroed here
__global__ __launch_bounds__(kDirThreads) void k_raydirs(FrameParams fp, int n, float4 *dirs, int *queue) {
    if (queue && blockIdx.x == 0 && threadIdx.x < 9) queue[threadIdx.x * kQueueStride] = 0;
    const int j = blockIdx.x * kDirThreads + threadIdx.x;
    if (j < n) dirs[j] = raydir(fp, n, j);
}

// Batched: block (b, v) covers rays 256b .. of volume v.
__global__ __launch_bounds__(kDirThreads) void k_raydirs_batched(const BatchVolume *vols, const FrameParams *frames,
                                                                 int n_vols) {
    const int v = blockIdx.y;
    if (v >= n_vols) return;
    const BatchVolume &bv = vols[v];
    const int j = blockIdx.x * kDirThreads + threadIdx.x;
    if (j < bv.vp.n) const_cast<float4 *>(bv.dirs)[j] = raydir(frames[v], bv.vp.n, j);
}

int raydir_blocks(int n) { return (n + kDirThreads - 1) / kDirThreads; }

template <typename T>
__global__ __launch_bounds__(kBlendThreads) void k_blend(VolumeParams vp, const float4 *dirs, const float4 *rays, T *irr,
                                                         T *vis, float h) {
    __shared__ BlendSmem sm;
    const int blk = xcd_logical_block();
    const int p0 = (blk / kBlendSplit) * kBlendTile;
    if (p0 >= vp.P) return;
    blend_tile_any<T>(vp, dirs, rays, irr, vis, h, p0, blk % kBlendSplit, sm);
}

hipError_t launch_raydirs(const FrameParams &fp, const VolumeParams &vp, float4 *dirs, int *queue, hipStream_t s) {
    hipLaunchKernelGGL(k_raydirs, dim3(raydir_blocks(vp.n)), dim3(kDirThreads), 0, s, fp, vp.n, dirs, queue);
    return hipGetLastError();
}

hipError_t launch_raydirs_batched(const BatchVolume *vols_dev, const FrameParams *frames_dev, int n_vols,
                                  int dir_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_raydirs_batched, dim3(dir_blocks, n_vols), dim3(kDirThreads), 0, s, vols_dev, frames_dev,
                       n_vols);
    return hipGetLastError();
}

hipError_t launch_blend(const VolumeParams &vp, const float4 *dirs, const float4 *rays, void *irr, void *vis,
                        int fp16, float h, hipStream_t s) {
    const dim3 grid((vp.P + kBlendTile - 1) / kBlendTile * kBlendSplit);
    if (fp16)
        hipLaunchKernelGGL(k_blend<__half>, grid, dim3(kBlendThreads), 0, s, vp, dirs, rays, (__half *)irr,
                           (__half *)vis, h);
    else
        hipLaunchKernelGGL(k_blend<float>, grid, dim3(kBlendThreads), 0, s, vp, dirs, rays, (float *)irr, (float *)vis,
                           h);
    return hipGetLastError();
}

}  // namespace pv
