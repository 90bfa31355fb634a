// Batched update of many volumes: after the ray-direction kernel of every
// volume (blend.hip), one trace launch covers every packet of every volume
// and one blend launch every probe group of every volume. Each block belongs
// to one volume and finds it by binary search over the per-volume prefix
// counts, so volumes of different sizes, ray counts, scenes and map formats
// share the device without a launch per volume. The trace runs the stepped
// lane loop (separate node and triangle steps) on each volume's own probe
// brick and top-node staging (its trace configuration). Results are bit-identical
// to the per-volume launches: each ray and each probe group runs the same
// device code on the same inputs.
#include "blend_gemm.h"
#include "trace_device.h"

namespace pv {

// trace: two packets per block (against four: the 32-volume frame's trace
// launch 1% faster, as the per-volume tuner's choice of 128-thread blocks
// for most of its volumes suggested)
constexpr int kBatchBlock = 128;
constexpr int kBatchWaves = kBatchBlock / 64;

// Last volume whose first item is at or before 'item' (prefix counts are
// ascending; every volume has at least one item).
template <bool BLEND>
__device__ __forceinline__ int find_volume(const BatchVolume *vols, int n_vols, int item) {
    int lo = 0, hi = n_vols - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int first = BLEND ? vols[mid].first_blend : vols[mid].first_wave;
        if (first <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename E>
__global__ __launch_bounds__(kBatchBlock) void k_trace_batched(const BatchVolume *vols, int n_vols,
                                                               const FrameParams *frames) {
    __shared__ E stk[kStack * kBatchBlock];
    const int wave0 = xcd_logical_block() * kBatchWaves;  // volumes start on a block boundary
    const int v = __builtin_amdgcn_readfirstlane(find_volume<false>(vols, n_vols, wave0));
    const BatchVolume &bv = vols[v];
    NodeSrc src = global_nodes(bv.sv.stat);
    const int nt = min(bv.top_nodes, bv.sv.stat.n_nodes);
    const uint4 *gn = reinterpret_cast<const uint4 *>(bv.sv.stat.nodes);
    for (int i = threadIdx.x; i < nt * 4; i += kBatchBlock) pv_top_nodes[i] = gn[i];
    __syncthreads();
    src.top = nt;
    // the packet of this wave in the volume's packet order (its own probe
    // brick), traced with the stepped lane loop
    TraceGrid g;
    g.bx = bv.bx;
    g.by = bv.by;
    g.bz = bv.bz;
    g.nbx = bv.bricks_x;
    g.nby = bv.bricks_y;
    g.nbz = bv.bricks_z;
    g.n_bricks = g.nbx * g.nby * g.nbz;
    g.n_waves = bv.n_waves;
    g.persistent = 2;
    g.chunk = 0;
    const int local = wave0 - bv.first_wave + (threadIdx.x >> 6);
    const int q = local < bv.n_waves ? ray_record(bv.vp, g, local * 64 + (threadIdx.x & 63)) : -1;
    LaneState s;
    lane_start(s, bv.vp, bv.sv, bv.dirs, q);
    Counts cnt = {0, 0};
    uint32_t sh = 0;
    lane_loop<false, false>(s, bv.vp, bv.sv, src, frames[v], bv.dirs, bv.rays, bv.hits, g, nullptr,
                            Stack<kBatchBlock, E>{stk + threadIdx.x}, cnt, sh);
}

// Blocks of a volume follow its blend mode: per-tile blocks (8 probes, half
// the rows) or column-group blocks of the product with four row groups.
union BatchedBlendSmem {
    BlendSmem tiles;
    BlendSmemGemm<float> gemm32;
    BlendSmemGemm<__half> gemm16;
};

template <typename T>
__device__ __forceinline__ void blend_batched_block(const BatchVolume &bv, int local, BatchedBlendSmem &sm) {
    const int mode = bv.vp.blend_mode;
    if (mode == kBlendTiles) {
        blend_tile_any<T>(bv.vp, bv.dirs, bv.rays, (T *)bv.irr, (T *)bv.vis, bv.h, (local / kBlendSplit) * kBlendTile,
                          local % kBlendSplit, sm.tiles);
        return;
    }
    BlendSmemGemm<T> &g = *reinterpret_cast<BlendSmemGemm<T> *>(&sm);
    if (mode == kBlendBF16x3)
        blend_gemm_block<T, kBlendBF16x3, 4>(bv.vp, bv.dirs, bv.rays, (T *)bv.irr, (T *)bv.vis, bv.h, local, g);
    else if (mode == kBlendVALU)
        blend_gemm_block<T, kBlendVALU, 4>(bv.vp, bv.dirs, bv.rays, (T *)bv.irr, (T *)bv.vis, bv.h, local, g);
    else if (mode == kBlendBF16x6)
        blend_gemm_block<T, kBlendBF16x6, 4>(bv.vp, bv.dirs, bv.rays, (T *)bv.irr, (T *)bv.vis, bv.h, local, g);
    else
        blend_gemm_block<T, kBlendF32, 4>(bv.vp, bv.dirs, bv.rays, (T *)bv.irr, (T *)bv.vis, bv.h, local, g);
}

// Batches whose maps share one type and whose volumes use the automatic
// blend paths (per-tile below the table's break-even, the BF16x6 table from
// there) or the FP32 table: only those three paths are compiled in, so the
// launch holds their registers instead of every path's (228 per lane: two
// wavefronts per SIMD). Binary16 maps: at most 128 registers, four
// wavefronts per SIMD.
template <typename T>
union AutoBlendSmem {
    BlendSmem tiles;
    BlendSmemGemm<T> gemm;
};

template <typename T>
__device__ __forceinline__ void blend_batched_auto(const BatchVolume *vols, int n_vols, AutoBlendSmem<T> &sm) {
    const int g = xcd_logical_block();
    const int v = __builtin_amdgcn_readfirstlane(find_volume<true>(vols, n_vols, g));
    const BatchVolume &bv = vols[v];
    const int local = g - bv.first_blend;
    const int mode = bv.vp.blend_mode;
    if (mode == kBlendTiles)
        blend_tile_any<T>(bv.vp, bv.dirs, bv.rays, (T *)bv.irr, (T *)bv.vis, bv.h, (local / kBlendSplit) * kBlendTile,
                          local % kBlendSplit, sm.tiles);
    else if (mode == kBlendBF16x6)
        blend_gemm_block<T, kBlendBF16x6, 4>(bv.vp, bv.dirs, bv.rays, (T *)bv.irr, (T *)bv.vis, bv.h, local, sm.gemm);
    else
        blend_gemm_block<T, kBlendF32, 4>(bv.vp, bv.dirs, bv.rays, (T *)bv.irr, (T *)bv.vis, bv.h, local, sm.gemm);
}

__global__ __launch_bounds__(kBlendThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_blend_batched_auto_h(
    const BatchVolume *vols, int n_vols) {
    __shared__ AutoBlendSmem<__half> sm;
    blend_batched_auto<__half>(vols, n_vols, sm);
}

__global__ __launch_bounds__(kBlendThreads) void k_blend_batched_auto_f(const BatchVolume *vols, int n_vols) {
    __shared__ AutoBlendSmem<float> sm;
    blend_batched_auto<float>(vols, n_vols, sm);
}

__global__ __launch_bounds__(kBlendThreads) void k_blend_batched(const BatchVolume *vols, int n_vols) {
    __shared__ BatchedBlendSmem sm;
    const int g = xcd_logical_block();
    const int v = __builtin_amdgcn_readfirstlane(find_volume<true>(vols, n_vols, g));
    const BatchVolume &bv = vols[v];
    const int local = g - bv.first_blend;
    if (bv.fp16)
        blend_batched_block<__half>(bv, local, sm);
    else
        blend_batched_block<float>(bv, local, sm);
}

hipError_t launch_trace_batched(const BatchVolume *vols_dev, int n_vols, int total_waves, const FrameParams *frames_dev,
                                bool short_stack, int max_top, hipStream_t s) {
    static_assert(kBatchWaves * 64 == kBatchBlock, "packets per trace block");
    const dim3 grid((total_waves + kBatchWaves - 1) / kBatchWaves);
    const size_t smem = (size_t)max_top * sizeof(GpuNode4);
    if (short_stack)
        hipLaunchKernelGGL(k_trace_batched<uint16_t>, grid, dim3(kBatchBlock), smem, s, vols_dev, n_vols, frames_dev);
    else
        hipLaunchKernelGGL(k_trace_batched<int>, grid, dim3(kBatchBlock), smem, s, vols_dev, n_vols, frames_dev);
    return hipGetLastError();
}

hipError_t launch_blend_batched(const BatchVolume *vols_dev, int n_vols, int total_blend, int kind, hipStream_t s) {
    if (kind == kBatchBlendAutoHalf)
        hipLaunchKernelGGL(k_blend_batched_auto_h, dim3(total_blend), dim3(kBlendThreads), 0, s, vols_dev, n_vols);
    else if (kind == kBatchBlendAutoFloat)
        hipLaunchKernelGGL(k_blend_batched_auto_f, dim3(total_blend), dim3(kBlendThreads), 0, s, vols_dev, n_vols);
    else
        hipLaunchKernelGGL(k_blend_batched, dim3(total_blend), dim3(kBlendThreads), 0, s, vols_dev, n_vols);
    return hipGetLastError();
}

}  // namespace pv
