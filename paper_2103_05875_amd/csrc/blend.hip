// Ray directions with the blend's weight tables, and the blend kernel.
//   k_raydirs   spherical-Fibonacci ray set under the frame rotation, and for
//               every (texel row, ray) the blend weight, plus partial row sums
//   k_blend     weighted means on the FP32 matrix cores, hysteresis, FP32 or
//               FP16 store, guard bands
#include "blend_device.h"

namespace pv {

constexpr int kRowChunks = kTexRows / 64;  // texel rows per ray-direction block: 64

// Block (b, c) of one volume-frame: rays 64b .. 64b+63 and texel rows
// 64c .. 64c+63. It computes the rays' directions (block c = 0 stores them),
// its slice of the weight table and the slice's partial row sums. Thread
// (row r = tid % 64, quarter u = tid / 64) weighs rays 16u .. 16u+15 for
// row 64c + r and writes them as four 16-byte groups; the four quarters'
// sums are added in a fixed order.
template <int S>
__device__ void raydirs_part(const FrameParams &fp, int n, int sharp, float4 *dirs, const WeightTables &wt, int b,
                             int c) {
    __shared__ float4 sd[kRaysPerPart];
    __shared__ float ps[4][64];
    const int tid = threadIdx.x;
    const int j0 = b * kRaysPerPart, m = min(kRaysPerPart, n - j0);
    if (tid < m) {
        const float4 d = raydir(fp, n, j0 + tid);
        if (c == 0) dirs[j0 + tid] = d;
        sd[tid] = d;
    }
    __syncthreads();
    const int r = tid & 63, u = tid >> 6, t = 64 * c + r;
    const bool irr = t < kIrrRows;
    const int tv = t - kIrrRows;
    const float3 om = irr ? oct_texel_dir(8, t & 7, t >> 3) : oct_texel_dir(16, tv & 15, tv >> 4);
    float s = 0.f;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int jj = 16 * u + 4 * g;
        if (jj >= m) break;  // past n the table keeps its zero padding
        float w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float x = 0.f;
            if (jj + k < m) {
                x = fmaxf(dot3(om, xyz(sd[jj + k])), 0.f);
                if (!irr) x = pow_int<S>(x, sharp);
            }
            w[k] = x;
        }
        s += w[0];
        s += w[1];
        s += w[2];
        s += w[3];
        *reinterpret_cast<float4 *>(wt.w + ((size_t)((j0 + jj) >> 2) * kTexRows + t) * 4) =
            make_float4(w[0], w[1], w[2], w[3]);
    }
    ps[u][r] = s;
    __syncthreads();
    if (u == 0) wt.part[b * kTexRows + t] = ((ps[0][r] + ps[1][r]) + ps[2][r]) + ps[3][r];
}

__device__ __forceinline__ void raydirs_any(const FrameParams &fp, int n, int sharp, float4 *dirs,
                                            const WeightTables &wt, int b, int c) {
    if (sharp == 50)
        raydirs_part<50>(fp, n, sharp, dirs, wt, b, c);
    else
        raydirs_part<0>(fp, n, sharp, dirs, wt, b, c);
}

// queue: the work counters of the trace that follows, zeroed here
__global__ __launch_bounds__(256) void k_raydirs(FrameParams fp, int n, int sharp, float4 *dirs, WeightTables wt,
                                                 int *queue) {
    if (queue && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 9) queue[threadIdx.x * kQueueStride] = 0;
    raydirs_any(fp, n, sharp, dirs, wt, blockIdx.x, blockIdx.y);
}

// Batched: block (b * kRowChunks + c, v) covers rays 64b.. and rows 64c.. of volume v.
__global__ __launch_bounds__(256) void k_raydirs_batched(const BatchVolume *vols, const FrameParams *frames,
                                                         int n_vols) {
    const int v = blockIdx.y;
    if (v >= n_vols) return;
    const BatchVolume &bv = vols[v];
    const int b = blockIdx.x / kRowChunks, c = blockIdx.x - b * kRowChunks;
    if (b >= bv.wt.nparts) return;
    raydirs_any(frames[v], bv.vp.n, bv.vp.vis_sharpness, const_cast<float4 *>(bv.dirs), bv.wt, b, c);
}

template <typename T>
__global__ __launch_bounds__(kBlendThreads) void k_blend(VolumeParams vp, WeightTables wt, const float4 *rays, T *irr,
                                                         T *vis, float h) {
    __shared__ BlendSmem sm;
    const int blk = xcd_logical_block();
    const int p0 = (blk / kBlendSplit) * kBlendTile;
    if (p0 >= vp.P) return;
    blend_tile<T>(vp, wt, rays, irr, vis, h, p0, blk % kBlendSplit, sm);
}

hipError_t launch_raydirs(const FrameParams &fp, const VolumeParams &vp, float4 *dirs, const WeightTables &wt,
                          int *queue, hipStream_t s) {
    hipLaunchKernelGGL(k_raydirs, dim3(wt.nparts, kRowChunks), dim3(256), 0, s, fp, vp.n, vp.vis_sharpness, dirs, wt,
                       queue);
    return hipGetLastError();
}

hipError_t launch_raydirs_batched(const BatchVolume *vols_dev, const FrameParams *frames_dev, int n_vols,
                                  int max_parts, hipStream_t s) {
    hipLaunchKernelGGL(k_raydirs_batched, dim3(max_parts * kRowChunks, n_vols), dim3(256), 0, s, vols_dev, frames_dev,
                       n_vols);
    return hipGetLastError();
}

hipError_t launch_blend(const VolumeParams &vp, const WeightTables &wt, const float4 *rays, void *irr, void *vis,
                        int fp16, float h, hipStream_t s) {
    const dim3 grid((vp.P + kBlendTile - 1) / kBlendTile * kBlendSplit);
    if (fp16)
        hipLaunchKernelGGL(k_blend<__half>, grid, dim3(kBlendThreads), 0, s, vp, wt, rays, (__half *)irr,
                           (__half *)vis, h);
    else
        hipLaunchKernelGGL(k_blend<float>, grid, dim3(kBlendThreads), 0, s, vp, wt, rays, (float *)irr, (float *)vis,
                           h);
    return hipGetLastError();
}

}  // namespace pv
