// Batched update: one persistent launch traces and blends many volumes.
#include "blend_device.h"
#include "trace_device.h"

namespace pv {

// ---------------------------------------------------------------------------
// batched persistent launch
// ---------------------------------------------------------------------------
// Work queue over all volumes: first every trace item (4 waves), then every
// blend group (8 probes). A blend group of volume v waits until all
// trace items of v have completed; every item it waits on was dequeued
// earlier by a running block that never waits on later items, so the
// queue drains. The wait is bounded; on expiry the block records an error
// and skips its item.
constexpr int kBatchBlock = 256;
constexpr long long kSpinLimit = 1ll << 26;

union BatchSmem {
    int stk[kStack * kBatchBlock];
    BlendSmem blend;
};

// Blend group of one volume (a call of its own: its registers are not
// allocated together with the trace path's).
__device__ __attribute__((noinline)) void batched_blend_item(const BatchVolume &bv, int p0, BlendSmem &sm) {
    if (bv.fp16)
        blend_tile<__half>(bv.vp, bv.wt, bv.rays, (__half *)bv.irr, (__half *)bv.vis, bv.h, p0, sm);
    else
        blend_tile<float>(bv.vp, bv.wt, bv.rays, (float *)bv.irr, (float *)bv.vis, bv.h, p0, sm);
}

__device__ __forceinline__ int volume_of_wave(const BatchVolume *vols, int n_vols, int wave) {
    int v = 0;
    while (v + 1 < n_vols && vols[v + 1].first_wave <= wave) ++v;
    return v;
}

__global__ __launch_bounds__(kBatchBlock) void k_batched(const BatchVolume *vols, int n_vols, int wave_items,
                                                        int total_blend, const FrameParams *frames, int *queue,
                                                        int *done, int *status) {
    __shared__ BatchSmem sm;
    __shared__ int item_s;
    const int total = wave_items + total_blend;
    const int wpi = kBatchBlock / 64;  // trace waves per item
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) item_s = atomicAdd(queue, 1);
        __syncthreads();
        // the item is the same for the whole block: keep it (and what is
        // derived from it) in scalar registers
        const int item = __builtin_amdgcn_readfirstlane(item_s);
        if (item >= total) break;
        if (item < wave_items) {
            const int wave = item * wpi + (threadIdx.x >> 6);
            const int v = volume_of_wave(vols, n_vols, wave);
            const BatchVolume &bv = vols[v];
            const int local = wave - bv.first_wave;
            if (local >= 0 && local < bv.n_waves) {
                const int lane = threadIdx.x & 63;
                const int n_bricks = bv.n_waves / bv.vp.n;
                const int j = local / n_bricks, brick = local - j * n_bricks;
                const int bxi = brick % bv.bricks_x, byi = (brick / bv.bricks_x) % bv.bricks_y,
                          bzi = brick / (bv.bricks_x * bv.bricks_y);
                const int x = bxi * 4 + (lane & 3), y = byi * 4 + ((lane >> 2) & 3), z = bzi * 4 + (lane >> 4);
                Counts cnt = {0, 0};
                uint32_t sh = 0;
                if (x < bv.vp.nx && y < bv.vp.ny && z < bv.vp.nz)
                    trace_shade_one<false, false>(bv.vp, bv.sv, global_nodes(bv.sv.stat), frames[v],
                                                               bv.dirs, bv.rays, bv.hits, x, y, z, j,
                                                               Stack<kBatchBlock>{sm.stk + threadIdx.x}, cnt, sh,
                                                               SplitBuffers());
            }
            __threadfence();
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int k = 0; k < wpi; ++k) {
                    const int wk = item * wpi + k;
                    const int vk = volume_of_wave(vols, n_vols, wk);
                    const int lk = wk - vols[vk].first_wave;
                    if (lk >= 0 && lk < vols[vk].n_waves) atomicAdd(&done[vk], 1);
                }
            }
        } else {
            const int g = item - wave_items;
            int v = 0;
            while (v + 1 < n_vols && vols[v + 1].first_blend <= g) ++v;
            v = __builtin_amdgcn_readfirstlane(v);
            const BatchVolume &bv = vols[v];
            if (threadIdx.x == 0) {
                long long spins = 0;
                while (__hip_atomic_load(&done[v], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < bv.n_waves) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > kSpinLimit) {
                        atomicExch(status, 1);
                        break;
                    }
                }
                __threadfence();
            }
            __syncthreads();
            batched_blend_item(bv, (g - bv.first_blend) * kBlendTile, sm.blend);
        }
    }
}

hipError_t launch_batched(const BatchVolume *vols_dev, int n_vols, int total_waves, int total_blend,
                          const FrameParams *frames_dev, int *queue_dev, int *done_dev, int *status_dev,
                          hipStream_t s) {
    const int wave_items = (total_waves + kBatchBlock / 64 - 1) / (kBatchBlock / 64);
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int blocks = cus * 4;
    hipLaunchKernelGGL(k_batched, dim3(blocks), dim3(kBatchBlock), 0, s, vols_dev, n_vols, wave_items, total_blend,
                       frames_dev, queue_dev, done_dev, status_dev);
    return hipGetLastError();
}

}  // namespace pv
