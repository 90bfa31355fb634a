// Trace kernels: closest hit of every (probe, ray) plus direct shading.
//   k_trace         one wavefront = one ray direction over a brick of 64
//                   probes (parallel rays with nearby origins)
//   k_trace_refill  persistent waves whose lanes take new rays as theirs end
//   k_shadow/k_shade  split-shadow variant: dense shadow rays, then shading
#include "trace_device.h"

namespace pv {

// One wavefront = one ray direction j over one brick of probes.
template <bool COUNT, bool SPLIT, class STK>
__device__ __forceinline__ void trace_wave(const VolumeParams &vp, const SceneView &sv, const NodeSrc &src,
                                           const FrameParams &fp, const float4 *dirs, float4 *rays, int32_t *hits,
                                           const TraceGrid &g, int w, STK stk, Counts &cnt, uint32_t &shadow,
                                           const SplitBuffers &split) {
    const int lane = threadIdx.x & 63;
    int j, brick;
    packet_of(vp, w, j, brick);
    const int bxi = brick % g.nbx, byi = (brick / g.nbx) % g.nby, bzi = brick / (g.nbx * g.nby);
    const int x = bxi * g.bx + lane % g.bx;
    const int y = byi * g.by + (lane / g.bx) % g.by;
    const int z = bzi * g.bz + lane / (g.bx * g.by);
    if (x < vp.nx && y < vp.ny && z < vp.nz)
        trace_shade_one<COUNT, SPLIT>(vp, sv, src, fp, dirs, rays, hits, x, y, z, j, stk, cnt, shadow, split);
}

template <bool COUNT, int W, int TOP, bool SPLIT, typename E>
__global__ __launch_bounds__(W) void k_trace(VolumeParams vp, SceneView sv, FrameParams fp, const float4 *dirs,
                                             float4 *rays, int32_t *hits, unsigned long long *counts, TraceGrid g,
                                             int *queue, SplitBuffers split) {
    __shared__ E stk[kStack * W];
    NodeSrc src = global_nodes(sv.stat);
    if (TOP > 0) {
        const int nt = min(TOP, sv.stat.n_nodes);
        const uint4 *gn = reinterpret_cast<const uint4 *>(sv.stat.nodes);
        for (int i = threadIdx.x; i < nt * 4; i += W) pv_top_nodes[i] = gn[i];
        __syncthreads();
        src.top = nt;
    }
    Stack<W, E> st{stk + threadIdx.x};
    Counts cnt = {0, 0};
    uint32_t shadow = 0;
    const int w = xcd_logical_block() * (W / 64) + (threadIdx.x >> 6);
    if (w < g.n_waves) trace_wave<COUNT, SPLIT>(vp, sv, src, fp, dirs, rays, hits, g, w, st, cnt, shadow, split);
    if (COUNT) {
        atomicAdd(&counts[0], (unsigned long long)cnt.nodes);
        atomicAdd(&counts[1], (unsigned long long)cnt.tris);
        atomicAdd(&counts[2], (unsigned long long)shadow);
    }
}

// REFILL = false: one wave per packet, as in k_trace, with the same lane
// state machine (separate node and triangle steps, shadow rays started as
// lanes finish) but no rays taken after the packet's own 64.
template <bool COUNT, int W, int TOP, typename E, bool REFILL>
__global__ __launch_bounds__(W) void k_trace_refill(VolumeParams vp, SceneView sv, FrameParams fp,
                                                    const float4 *dirs, float4 *rays, int32_t *hits,
                                                    unsigned long long *counts, TraceGrid g, int *queue) {
    __shared__ E stk[kStack * W];
    NodeSrc stat_src = global_nodes(sv.stat);
    if (TOP > 0) {
        const int nt = min(TOP, sv.stat.n_nodes);
        const uint4 *gn = reinterpret_cast<const uint4 *>(sv.stat.nodes);
        for (int i = threadIdx.x; i < nt * 4; i += W) pv_top_nodes[i] = gn[i];
        __syncthreads();
        stat_src.top = nt;
    }
    Counts cnt = {0, 0};
    uint32_t shadow = 0;
    LaneState s;
    int q = -1;
    if (!REFILL) {
        // the wave's own packet, then nothing more
        const int w = xcd_logical_block() * (W / 64) + (threadIdx.x >> 6);
        if (w < g.n_waves) q = ray_record(vp, g, w * 64 + (threadIdx.x & 63));
    }
    lane_start(s, vp, sv, dirs, q);
    lane_loop<COUNT, REFILL>(s, vp, sv, stat_src, fp, dirs, rays, hits, g, queue, Stack<W, E>{stk + threadIdx.x}, cnt,
                             shadow);
    if (COUNT) {
        atomicAdd(&counts[0], (unsigned long long)cnt.nodes);
        atomicAdd(&counts[1], (unsigned long long)cnt.tris);
        atomicAdd(&counts[2], (unsigned long long)shadow);
    }
}

// Shadow rays of the split trace: dense any-hit over the compacted queue.
template <bool COUNT, int W, int TOP, typename E>
__global__ __launch_bounds__(W) void k_shadow(SceneView sv, SplitBuffers split, unsigned long long *counts) {
    __shared__ E stk[kStack * W];
    NodeSrc src = global_nodes(sv.stat);
    if (TOP > 0) {
        const int nt = min(TOP, sv.stat.n_nodes);
        const uint4 *gn = reinterpret_cast<const uint4 *>(sv.stat.nodes);
        for (int i = threadIdx.x; i < nt * 4; i += W) pv_top_nodes[i] = gn[i];
        __syncthreads();
        src.top = nt;
    }
    const NodeSrc dyn_src = global_nodes(sv.dyn);
    Stack<W, E> st{stk + threadIdx.x};
    Counts cnt = {0, 0};
    const int n = *split.count;
    // whole wavefronts step together through the queue
    const int nwaves_grid = gridDim.x * (W / 64);
    const int wave = blockIdx.x * (W / 64) + (threadIdx.x >> 6);
    for (int base = wave * 64; base < n; base += nwaves_grid * 64) {
        const int i = base + (threadIdx.x & 63);
        if (i < n) {
            const ShadowEntry e = split.queue[i];
            const Ray sr = make_ray(xyz(e.o_tmax), xyz(e.d_ray));
            bool occ = any_hit<COUNT>(sv.stat, src, sr, 0.f, e.o_tmax.w, st, cnt);
            if (!occ) occ = any_hit<COUNT>(sv.dyn, dyn_src, sr, 0.f, e.o_tmax.w, st, cnt);
            if (occ) {
                const int code = __float_as_int(e.d_ray.w);
                atomicOr(&split.occ[code >> 3], 1u << (code & 7));
            }
        }
    }
    if (COUNT) {
        atomicAdd(&counts[0], (unsigned long long)cnt.nodes);
        atomicAdd(&counts[1], (unsigned long long)cnt.tris);
    }
}

// Shade pass of the split trace: the same light loop as the fused trace, with
// each light's visibility read from the occlusion bits.
__global__ __launch_bounds__(256) void k_shade(VolumeParams vp, SceneView sv, FrameParams fp, const float4 *dirs,
                                               float4 *rays, SplitBuffers split) {
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (size_t)vp.P * vp.n) return;
    const int2 hr = split.hitrec[q];
    if (hr.x < 0 || fp.n_lights == 0) return;
    const int p = (int)(q / vp.n), j = (int)(q - (size_t)p * vp.n);
    const int x = p % vp.nx, y = (p / vp.nx) % vp.ny, z = p / (vp.nx * vp.ny);
    const float3 o = make_float3(fmaf(vp.sx, (float)x, vp.ox), fmaf(vp.sy, (float)y, vp.oy),
                                 fmaf(vp.sz, (float)z, vp.oz));
    const Ray ray = make_ray(o, xyz(dirs[j]));
    const GpuTri *arr = (hr.x & 0x80000000) ? sv.dyn.tris : sv.stat.tris;
    const GpuTri T = arr[hr.x & 0x7fffffff];
    float3 nrm, xh;
    hit_frame(T, ray, o, __int_as_float(hr.y), nrm, xh);
    const float4 alb = sv.mats[2 * tri_id(T)];
    const uint32_t occ = split.occ[q];
    float4 rec = rays[q];
    float3 L = make_float3(rec.x, rec.y, rec.z);
    for (int li = 0; li < fp.n_lights; ++li) {
        float cosv, d2, smax;
        float3 so, sd;
        if (!light_setup(fp, li, sv.eps, nrm, xh, cosv, d2, so, sd, smax)) continue;
        if (!((occ >> li) & 1u)) light_add(fp, li, alb, cosv, d2, L);
    }
    rays[q] = make_float4(L.x, L.y, L.z, rec.w);
}

template <bool COUNT, int W, int TOP, bool SPLIT, typename E>
static hipError_t launch_trace_t(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp,
                                 const float4 *dirs, float4 *rays, int32_t *hits, unsigned long long *counts,
                                 const TraceGrid &g, int *queue, const SplitBuffers &split, hipStream_t s) {
    const size_t smem = (size_t)TOP * sizeof(GpuNode4);
    if (g.persistent == 1 && !SPLIT) {
        // as many waves as fit on the device at once; each deals itself rays
        int dev = 0, cus = 256, per_cu = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_refill<COUNT, W, TOP, E, true>, W, smem);
        const long long need = ((long long)g.n_waves * 64 + W - 1) / W;
        const unsigned blocks =
            (unsigned)std::max(1ll, std::min<long long>((long long)cus * std::max(per_cu, 1), need));
        hipLaunchKernelGGL((k_trace_refill<COUNT, W, TOP, E, true>), dim3(blocks), dim3(W), smem, s, vp, sv, fp, dirs,
                           rays, hits, counts, g, queue);
        return hipGetLastError();
    }
    if (g.persistent == 2 && !SPLIT) {
        const unsigned blocks = (unsigned)(((long long)g.n_waves * 64 + W - 1) / W);
        hipLaunchKernelGGL((k_trace_refill<COUNT, W, TOP, E, false>), dim3(blocks), dim3(W), smem, s, vp, sv, fp, dirs,
                           rays, hits, counts, g, queue);
        return hipGetLastError();
    }
    const unsigned blocks = (unsigned)(((long long)g.n_waves * 64 + W - 1) / W);
    hipLaunchKernelGGL((k_trace<COUNT, W, TOP, SPLIT, E>), dim3(blocks), dim3(W), smem, s, vp, sv, fp, dirs, rays, hits,
                       counts, g, queue, split);
    return hipGetLastError();
}

template <bool COUNT, bool SPLIT>
static hipError_t launch_trace_c(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp,
                                 const float4 *dirs, float4 *rays, int32_t *hits, unsigned long long *counts,
                                 const TraceConfig &tc, const TraceGrid &g, int *queue, const SplitBuffers &split,
                                 hipStream_t s) {
    const bool short_stack = stack_fits_u16(sv);
#define PV_TRACE_CASE(Wv, Tv)                                                                                      \
    if (tc.block == Wv && tc.top_nodes == Tv)                                                                     \
        return short_stack                                                                                        \
                   ? launch_trace_t<COUNT, Wv, Tv, SPLIT, uint16_t>(vp, sv, fp, dirs, rays, hits, counts, g, queue, \
                                                                    split, s)                                     \
                   : launch_trace_t<COUNT, Wv, Tv, SPLIT, int>(vp, sv, fp, dirs, rays, hits, counts, g, queue, split, s);
    PV_TRACE_CASE(128, 0)
    PV_TRACE_CASE(128, 21)
    PV_TRACE_CASE(128, 85)
    PV_TRACE_CASE(256, 0)
    PV_TRACE_CASE(256, 21)
    PV_TRACE_CASE(256, 85)
#undef PV_TRACE_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_trace(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp, const float4 *dirs,
                        float4 *rays, int32_t *hits, unsigned long long *counts, const TraceConfig &tc, int *queue,
                        const SplitBuffers &split, hipStream_t s) {
    TraceGrid g;
    g.bx = tc.bx;
    g.by = tc.by;
    g.bz = tc.bz;
    g.nbx = (vp.nx + tc.bx - 1) / tc.bx;
    g.nby = (vp.ny + tc.by - 1) / tc.by;
    g.nbz = (vp.nz + tc.bz - 1) / tc.bz;
    g.n_bricks = g.nbx * g.nby * g.nbz;
    g.n_waves = g.n_bricks * vp.n;
    g.persistent = (tc.persistent == 1 && queue == nullptr) ? 0 : tc.persistent;
    g.chunk = (g.n_waves + 7) / 8;
    const bool split_mode = tc.split_shadows && split.queue != nullptr;
    if (counts) {
        if (split_mode) return launch_trace_c<true, true>(vp, sv, fp, dirs, rays, hits, counts, tc, g, queue, split, s);
        return launch_trace_c<true, false>(vp, sv, fp, dirs, rays, hits, counts, tc, g, queue, split, s);
    }
    if (split_mode) return launch_trace_c<false, true>(vp, sv, fp, dirs, rays, hits, counts, tc, g, queue, split, s);
    return launch_trace_c<false, false>(vp, sv, fp, dirs, rays, hits, counts, tc, g, queue, split, s);
}

template <bool COUNT, int W, int TOP, typename E>
static hipError_t launch_shadow_t(const SceneView &sv, const SplitBuffers &split, unsigned long long *counts,
                                  hipStream_t s) {
    int dev = 0, cus = 256, per_cu = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_shadow<COUNT, W, TOP, E>, W,
                                                       (size_t)TOP * sizeof(GpuNode4));
    const long long cap_blocks = (split.capacity + W - 1) / W;
    const unsigned blocks = (unsigned)std::max(1ll, std::min<long long>((long long)cus * std::max(per_cu, 1), cap_blocks));
    hipLaunchKernelGGL((k_shadow<COUNT, W, TOP, E>), dim3(blocks), dim3(W), (size_t)TOP * sizeof(GpuNode4), s, sv, split,
                       counts);
    return hipGetLastError();
}

hipError_t launch_shadow(const SceneView &sv, const SplitBuffers &split, const TraceConfig &tc,
                         unsigned long long *counts, hipStream_t s) {
    const bool short_stack = stack_fits_u16(sv);
#define PV_SHADOW_CASE(Wv, Tv)                                                                 \
    if (tc.block == Wv && tc.top_nodes == Tv) {                                                \
        if (short_stack)                                                                       \
            return counts ? launch_shadow_t<true, Wv, Tv, uint16_t>(sv, split, counts, s)      \
                          : launch_shadow_t<false, Wv, Tv, uint16_t>(sv, split, counts, s);    \
        return counts ? launch_shadow_t<true, Wv, Tv, int>(sv, split, counts, s)               \
                      : launch_shadow_t<false, Wv, Tv, int>(sv, split, counts, s);             \
    }
    PV_SHADOW_CASE(128, 0)
    PV_SHADOW_CASE(128, 21)
    PV_SHADOW_CASE(128, 85)
    PV_SHADOW_CASE(256, 0)
    PV_SHADOW_CASE(256, 21)
    PV_SHADOW_CASE(256, 85)
#undef PV_SHADOW_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_shade(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp, const float4 *dirs,
                        float4 *rays, const SplitBuffers &split, hipStream_t s) {
    const long long n = (long long)vp.P * vp.n;
    hipLaunchKernelGGL(k_shade, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, vp, sv, fp, dirs, rays, split);
    return hipGetLastError();
}

}  // namespace pv
