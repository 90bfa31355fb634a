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
    const int j = w / g.n_bricks, brick = w - j * g.n_bricks;
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

// ---------------------------------------------------------------------------
// Persistent trace with per-lane ray refill
// ---------------------------------------------------------------------------
// The wavefront-per-packet trace idles a lane from the moment its ray ends
// until the slowest ray of the packet ends, and runs a node's leaf triangles
// inside the node step, so one lane's leaf stalls the other 63. Here every
// lane is a small state machine over (primary ray through the static BVH,
// then the dynamic BVH; per light a shadow ray through both), and the wave
// loop does one of three things per iteration:
//   - node step: lanes with no pending triangles visit their next node; the
//     node's hit leaf children become a pending triangle mask
//   - triangle step: lanes with pending triangles test one of them
//   - transition: lanes whose traversal ended move to the next stage (shade,
//     shadow ray, write the record), idle lanes take new rays from the work
//     queues
// Node or triangle step is chosen by how many lanes are waiting for each
// (weighted by their cost); transitions wait until enough lanes need one.
// Each lane runs exactly the operations of the per-packet trace, in the same
// order, so the records are bit-identical; only the interleaving of lanes
// differs. Rays are numbered as in the per-packet trace (packet of one
// direction over one brick, 64 per packet) and dealt out from 8 queues, one
// per XCD, in runs of consecutive rays.
constexpr int kRefillAt = 16;      // transitions once this many lanes wait
constexpr int kNodeCost = 3;       // node step ~ 3 triangle steps (instructions)

enum : int { kPrimStat = 0, kPrimDyn = 1, kShadStat = 2, kShadDyn = 3 };

struct LaneState {
    // current traversal
    Ray ray;
    float tmax;         // closest: best distance so far; any hit: shadow length
    int node;           // next node, -1 when the stack is exhausted
    int sp;
    int tbase;          // first triangle slot of the pending leaf triangles
    uint32_t tmask;     // pending leaf triangles (bit i = slot tbase + i)
    int stage;
    bool occluded;
    // the ray's job
    int q;              // record index (probe * n + direction), -1 idle
    int best, best_id;  // closest hit: leaf-order slot and original id
    bool best_dyn;
    float tbest;        // closest hit distance (kept while shadow rays run)
    float3 L;
    float dist;
    int li;             // light of the current shadow ray
    float cosv, d2;
};

__device__ __forceinline__ void start_traversal(LaneState &s, const DeviceBvh &bvh) {
    s.node = bvh.n_nodes > 0 ? 0 : -1;
    s.sp = 0;
    s.tmask = 0u;
}

__device__ __forceinline__ float3 probe_origin(const VolumeParams &vp, int p) {
    const int x = p % vp.nx, y = (p / vp.nx) % vp.ny, z = p / (vp.nx * vp.ny);
    return make_float3(fmaf(vp.sx, (float)x, vp.ox), fmaf(vp.sy, (float)y, vp.oy), fmaf(vp.sz, (float)z, vp.oz));
}

// Starts the shadow ray of the first light at or after s.li that faces the
// hit; false when none is left. The hit frame is recomputed from the primary
// ray and the hit triangle with the operations of the per-packet trace.
template <bool COUNT>
__device__ __forceinline__ bool next_light(LaneState &s, const VolumeParams &vp, const SceneView &sv,
                                           const FrameParams &fp, const float4 *dirs, uint32_t &shadow_rays) {
    if (s.best < 0) return false;
    const int p = s.q / vp.n, j = s.q - p * vp.n;
    const float3 o = probe_origin(vp, p);
    const Ray pr = make_ray(o, xyz(dirs[j]));
    const GpuTri T = (s.best_dyn ? sv.dyn.tris : sv.stat.tris)[s.best];
    float3 nrm, xh;
    hit_frame(T, pr, o, s.tbest, nrm, xh);
    for (; s.li < fp.n_lights; ++s.li) {
        float smax;
        float3 so, sd;
        if (!light_setup(fp, s.li, sv.eps, nrm, xh, s.cosv, s.d2, so, sd, smax)) continue;
        s.ray = make_ray(so, sd);
        s.tmax = smax;
        s.stage = kShadStat;
        s.occluded = false;
        start_traversal(s, sv.stat);
        if (COUNT) shadow_rays++;
        return true;
    }
    return false;
}

// Moves a lane whose traversal ended to its next traversal, or writes its
// record and leaves it idle.
template <bool COUNT>
__device__ void lane_transition(LaneState &s, const VolumeParams &vp, const SceneView &sv, const FrameParams &fp,
                                const float4 *dirs, float4 *rays, int32_t *hits, uint32_t &shadow_rays) {
    if (s.stage == kPrimStat && sv.dyn.n_nodes > 0) {
        s.stage = kPrimDyn;
        start_traversal(s, sv.dyn);
        return;
    }
    if (s.stage == kShadStat && !s.occluded && sv.dyn.n_nodes > 0) {
        s.stage = kShadDyn;
        start_traversal(s, sv.dyn);
        return;
    }
    if (s.stage <= kPrimDyn) {
        // primary ray done: emission or sky, then the lights
        s.tbest = s.tmax;
        if (s.best >= 0) {
            const float4 emi = sv.mats[2 * s.best_id + 1];
            s.L = make_float3(emi.x, emi.y, emi.z);
            s.dist = fminf(s.tbest, vp.max_distance);
        } else {
            s.L = make_float3(vp.sky[0], vp.sky[1], vp.sky[2]);
            s.dist = vp.max_distance;
        }
        s.li = 0;
    } else {
        // shadow ray done
        if (!s.occluded) light_add(fp, s.li, sv.mats[2 * s.best_id], s.cosv, s.d2, s.L);
        ++s.li;
    }
    if (next_light<COUNT>(s, vp, sv, fp, dirs, shadow_rays)) return;
    rays[s.q] = make_float4(s.L.x, s.L.y, s.L.z, s.dist);
    if (hits) hits[s.q] = s.best_id;
    s.q = -1;
}

// Ray number r (packet order) -> record index, or -1 for a lane of a ragged
// brick that lies outside the grid.
__device__ __forceinline__ int ray_record(const VolumeParams &vp, const TraceGrid &g, int r) {
    const int w = r >> 6, lane = r & 63;
    const int j = w / g.n_bricks, brick = w - j * g.n_bricks;
    const int bxi = brick % g.nbx, byi = (brick / g.nbx) % g.nby, bzi = brick / (g.nbx * g.nby);
    const int x = bxi * g.bx + lane % g.bx;
    const int y = byi * g.by + (lane / g.bx) % g.by;
    const int z = bzi * g.bz + lane / (g.bx * g.by);
    if (x >= vp.nx || y >= vp.ny || z >= vp.nz) return -1;
    return (x + vp.nx * (y + vp.ny * z)) * vp.n + j;
}

template <bool COUNT, int W, int TOP, typename E>
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
    const uint4 *dyn_nodes = reinterpret_cast<const uint4 *>(sv.dyn.nodes);
    Stack<W, E> stk_l{stk + threadIdx.x};
    Counts cnt = {0, 0};
    uint32_t shadow = 0;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const long long total = (long long)g.n_waves * 64;
    const int chunk = (int)((total + 7) / 8);

    LaneState s;
    s.q = -1;
    s.node = -1;
    s.tmask = 0u;
    s.stage = kPrimStat;
    int k = 0;                                   // queues visited (wave-uniform)
    const int home = (blockIdx.x & 7);
    bool exhausted = false;

    while (true) {
        const bool act = s.q >= 0 && (s.node >= 0 || s.tmask != 0u);
        const bool fin = s.q >= 0 && !act;
        const int n_act = __popcll(__ballot(act));
        const int n_fin = __popcll(__ballot(fin));
        const int n_idle = exhausted ? 0 : __popcll(__ballot(s.q < 0));
        if (n_act == 0 && n_fin == 0 && exhausted) break;
        // transitions when enough lanes wait for one, or when the finished
        // lanes outnumber the ones still tracing (the end of the queues)
        if (n_act == 0 || n_fin + n_idle >= kRefillAt || n_fin > n_act) {
            if (fin) lane_transition<COUNT>(s, vp, sv, fp, dirs, rays, hits, shadow);
            // deal new rays to idle lanes, consecutive rays to consecutive idle lanes
            unsigned long long idle = __ballot(s.q < 0);
            while (idle != 0ull && !exhausted) {
                const int want = __popcll(idle);
                const int qk = (home + k) & 7;
                int base = 0;
                if (lane == 0) base = atomicAdd(&queue[qk], want);
                base = __shfl(base, 0);
                const long long lo = (long long)qk * chunk;
                const long long hi = min(total, lo + chunk);
                if (lo + base >= hi) {
                    if (++k == 8) exhausted = true;
                    continue;
                }
                if (s.q < 0) {
                    const long long r = lo + base + __popcll(idle & below);
                    if (r < hi) {
                        const int q = ray_record(vp, g, (int)r);
                        if (q >= 0) {
                            const int p = q / vp.n, j = q - p * vp.n;
                            s.q = q;
                            s.ray = make_ray(probe_origin(vp, p), xyz(dirs[j]));
                            s.tmax = INFINITY;
                            s.best = -1;
                            s.best_id = -1;
                            s.best_dyn = false;
                            s.stage = kPrimStat;
                            start_traversal(s, sv.stat);
                        }
                    }
                }
                idle = __ballot(s.q < 0);
            }
            continue;
        }
        const int n_tri = __popcll(__ballot(act && s.tmask != 0u));
        const int n_node = n_act - n_tri;
        const bool dyn = (s.stage & 1) != 0;
        const bool any = s.stage >= kShadStat;
        if (n_tri * kNodeCost >= n_node) {
            // triangle step
            if (act && s.tmask != 0u) {
                const int i = __builtin_ctz(s.tmask);
                s.tmask &= s.tmask - 1u;
                const int slot = s.tbase + i;
                const GpuTri T = (dyn ? sv.dyn.tris : sv.stat.tris)[slot];
                float t;
                if (COUNT) cnt.tris++;
                if (tri_cross(T, s.ray, t) && t > 0.f) {
                    if (any) {
                        if (t < s.tmax) {
                            s.occluded = true;
                            s.node = -1;
                            s.tmask = 0u;
                        }
                    } else if (t < s.tmax || (t == s.tmax && tri_id(T) < s.best_id)) {
                        s.tmax = t;
                        s.best = slot;
                        s.best_id = tri_id(T);
                        s.best_dyn = dyn;
                    }
                }
            }
        } else if (act && s.tmask == 0u) {
            // node step
            uint4 w0, w1, w2, w3;
            if (dyn) {
                const uint4 *qn = dyn_nodes + 4 * (size_t)s.node;
                w0 = qn[0];
                w1 = qn[1];
                w2 = qn[2];
                w3 = qn[3];
            } else {
                stat_src.load(s.node, w0, w1, w2, w3);
            }
            Node4Hits h;
            box4(w0, w1, w2, w3, s.ray, 0.f, s.tmax, h);
            if (COUNT) cnt.nodes++;
            // hit leaf children become the pending triangle mask
            s.tmask = leaf_mask(h, s.tbase);
            int ids[4];
            const int mi = sort_inner(h, ids);
            if (mi > 0) {
                if (mi > 3) stk_l.push(s.sp, ids[3]);
                if (mi > 2) stk_l.push(s.sp, ids[2]);
                if (mi > 1) stk_l.push(s.sp, ids[1]);
                s.node = ids[0];
            } else {
                s.node = s.sp == 0 ? -1 : stk_l.pop(s.sp);
            }
        }
    }
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
    if (g.persistent && !SPLIT) {
        // as many waves as fit on the device at once; each deals itself rays
        int dev = 0, cus = 256, per_cu = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_refill<COUNT, W, TOP, E>, W, smem);
        const long long need = ((long long)g.n_waves * 64 + W - 1) / W;
        const unsigned blocks =
            (unsigned)std::max(1ll, std::min<long long>((long long)cus * std::max(per_cu, 1), need));
        hipLaunchKernelGGL((k_trace_refill<COUNT, W, TOP, E>), dim3(blocks), dim3(W), smem, s, vp, sv, fp, dirs, rays,
                           hits, counts, g, queue);
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
    g.persistent = tc.persistent && queue != nullptr;
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
