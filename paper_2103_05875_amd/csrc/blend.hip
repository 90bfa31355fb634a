// Ray directions and the blend kernel.
//   k_raydirs   spherical-Fibonacci ray set under the frame rotation (one
//               thread per ray); also clears the trace's work counters
//   k_blend     weighted means on the FP32 matrix cores, hysteresis, FP32 or
//               FP16 store, guard bands
#include "blend_gemm.h"

namespace pv {

constexpr int kDirThreads = 256;
static_assert(kDirThreads == 256 && kWGroup == 4 && kWGroup * kWStep <= kDirThreads, "a weight-table block: four wavefronts, one step each, one direction per thread");

__host__ __device__ inline int dir_blocks(int n) { return (n + kDirThreads - 1) / kDirThreads; }
__host__ __device__ inline int table_blocks(int mode, int n) {
    return (mode == kBlendBF16x3 || mode == kBlendF32 || mode == kBlendVALU || mode == kBlendBF16x6)
               ? kMTiles * wtab_groups(n)
               : 0;
}

// Blocks [0, dir_blocks): one thread per ray direction; the next
// table_blocks(mode, n) blocks: the weight table after the directions (one
// row tile over one group of steps each). queue: the work counters of the trace that follows,
// zeroed here.
__global__ __launch_bounds__(kDirThreads) void k_raydirs(FrameParams fp, int n, float4 *dirs, int *queue, int mode,
                                                         int sharp) {
    __shared__ float3 sdir[kWGroup * kWStep];
    __shared__ float red[64];
    const int db = dir_blocks(n);
    if ((int)blockIdx.x >= db) {
        weight_table_block(fp, n, sharp, mode, reinterpret_cast<uint8_t *>(dirs) + dirs_span(n), blockIdx.x - db,
                           sdir, red);
        return;
    }
    if (queue && blockIdx.x == 0 && threadIdx.x < 9) queue[threadIdx.x * kQueueStride] = 0;
    const int j = blockIdx.x * kDirThreads + threadIdx.x;
    if (j < n) dirs[j] = raydir(fp, n, j);
}

// Batched: block (b, v) covers rays 256b .. of volume v, or one block of its
// weight table.
__global__ __launch_bounds__(kDirThreads) void k_raydirs_batched(const BatchVolume *vols, const FrameParams *frames,
                                                                 int n_vols) {
    __shared__ float3 sdir[kWGroup * kWStep];
    __shared__ float red[64];
    const int v = blockIdx.y;
    if (v >= n_vols) return;
    const BatchVolume &bv = vols[v];
    const int n = bv.vp.n, db = dir_blocks(n);
    if ((int)blockIdx.x >= db) {
        if ((int)blockIdx.x - db < table_blocks(bv.vp.blend_mode, n))
            weight_table_block(frames[v], n, bv.vp.vis_sharpness, bv.vp.blend_mode,
                               reinterpret_cast<uint8_t *>(const_cast<float4 *>(bv.dirs)) + dirs_span(n),
                               blockIdx.x - db, sdir, red);
        return;
    }
    const int j = blockIdx.x * kDirThreads + threadIdx.x;
    if (j < n) const_cast<float4 *>(bv.dirs)[j] = raydir(frames[v], n, j);
}

int raydir_blocks(int n) { return dir_blocks(n); }
int weight_blocks(int mode, int n) { return table_blocks(mode, n); }

template <typename T>
__global__ __launch_bounds__(kBlendThreads) void k_blend(VolumeParams vp, const float4 *dirs, const float4 *rays, T *irr,
                                                         T *vis, float h) {
    __shared__ BlendSmem sm;
    const int blk = xcd_logical_block();
    const int p0 = (blk / kBlendSplit) * kBlendTile;
    if (p0 >= vp.P) return;
    blend_tile_any<T>(vp, dirs, rays, irr, vis, h, p0, blk % kBlendSplit, sm);
}

// One block per 16-probe column group, G row-group wavefronts (one kernel
// per grouping, so that the small groups are not held to the registers of
// the large ones).
template <typename T, int MODE, int G>
__device__ __forceinline__ void blend_gemm_grid(const VolumeParams &vp, const float4 *dirs, const float4 *rays, T *irr,
                                                T *vis, float h) {
    __shared__ BlendSmemGemm<T> sm;
    const int cg = xcd_logical_block();
    if (cg >= blend_column_groups(vp.P)) return;
    blend_gemm_block<T, MODE, G>(vp, dirs, rays, irr, vis, h, cg, sm);
}

template <typename T, int MODE, int G>
__global__ __launch_bounds__(64 * G) void k_blend_gemm(VolumeParams vp, const float4 *dirs, const float4 *rays, T *irr,
                                                       T *vis, float h) {
    blend_gemm_grid<T, MODE, G>(vp, dirs, rays, irr, vis, h);
}

// Binary16 maps in four-wavefront blocks (the large volumes): at most 128
// registers per lane, so that four wavefronts share a SIMD and every block
// of the encode-size grid is resident at once (the FP32 image's LDS allows
// two blocks per CU whatever the registers).
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_blend_gemm_h4(
    VolumeParams vp, const float4 *dirs, const float4 *rays, __half *irr, __half *vis, float h) {
    blend_gemm_grid<__half, MODE, 4>(vp, dirs, rays, irr, vis, h);
}

hipError_t launch_raydirs(const FrameParams &fp, const VolumeParams &vp, float4 *dirs, int *queue, hipStream_t s) {
    hipLaunchKernelGGL(k_raydirs, dim3(dir_blocks(vp.n) + table_blocks(vp.blend_mode, vp.n)), dim3(kDirThreads), 0, s, fp,
                       vp.n, dirs, queue, vp.blend_mode, vp.vis_sharpness);
    return hipGetLastError();
}

hipError_t launch_raydirs_batched(const BatchVolume *vols_dev, const FrameParams *frames_dev, int n_vols,
                                  int dir_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_raydirs_batched, dim3(dir_blocks, n_vols), dim3(kDirThreads), 0, s, vols_dev, frames_dev,
                       n_vols);
    return hipGetLastError();
}

int blend_blocks(int P, int mode) {
    if (mode == kBlendTiles) return (P + kBlendTile - 1) / kBlendTile * kBlendSplit;
    return blend_column_groups(P);
}

template <typename T, int MODE>
static void launch_gemm(bool g4, dim3 grid, const VolumeParams &vp, const float4 *dirs, const float4 *rays, T *irr,
                        T *vis, float h, hipStream_t s) {
    if (!g4)
        hipLaunchKernelGGL((k_blend_gemm<T, MODE, 8>), grid, dim3(512), 0, s, vp, dirs, rays, irr, vis, h);
    else if constexpr (std::is_same_v<T, __half>)
        hipLaunchKernelGGL((k_blend_gemm_h4<MODE>), grid, dim3(256), 0, s, vp, dirs, rays, irr, vis, h);
    else
        hipLaunchKernelGGL((k_blend_gemm<T, MODE, 4>), grid, dim3(256), 0, s, vp, dirs, rays, irr, vis, h);
}

template <typename T>
static hipError_t launch_blend_t(const VolumeParams &vp, const float4 *dirs, const float4 *rays, T *irr, T *vis,
                                 float h, hipStream_t s) {
    const dim3 grid(blend_blocks(vp.P, vp.blend_mode));
    const bool g4 = blend_row_groups(vp.P) == 4;
    switch (vp.blend_mode) {
    case kBlendBF16x3:
        launch_gemm<T, kBlendBF16x3>(g4, grid, vp, dirs, rays, irr, vis, h, s);
        break;
    case kBlendF32:
        launch_gemm<T, kBlendF32>(g4, grid, vp, dirs, rays, irr, vis, h, s);
        break;
    case kBlendVALU:
        launch_gemm<T, kBlendVALU>(g4, grid, vp, dirs, rays, irr, vis, h, s);
        break;
    case kBlendBF16x6:
        launch_gemm<T, kBlendBF16x6>(g4, grid, vp, dirs, rays, irr, vis, h, s);
        break;
    default:
        hipLaunchKernelGGL(k_blend<T>, grid, dim3(kBlendThreads), 0, s, vp, dirs, rays, irr, vis, h);
    }
    return hipGetLastError();
}

hipError_t launch_blend(const VolumeParams &vp, const float4 *dirs, const float4 *rays, void *irr, void *vis,
                        int fp16, float h, hipStream_t s) {
    if (fp16) return launch_blend_t<__half>(vp, dirs, rays, (__half *)irr, (__half *)vis, h, s);
    return launch_blend_t<float>(vp, dirs, rays, (float *)irr, (float *)vis, h, s);
}

}  // namespace pv
