// Data layouts and launch parameters of the trace: BVH nodes and triangles,
// scene / volume / frame parameter blocks, the trace launch shape and its
// work counters. Shared by the host side and the kernels; not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "probestream.h"

namespace pv {

// ---------------------------------------------------------------------------
// Device data layouts
// ---------------------------------------------------------------------------

// Triangle in leaf order: its three vertices exactly as given (v0.w = the
// original triangle id as int bits; v1.w, v2.w unused). Vertices shared by
// neighbouring triangles are bit-identical, which the watertight triangle
// test relies on.
struct alignas(16) GpuTri {
    float4 v0, v1, v2;
};

struct GpuNode4;

struct DeviceBvh {
    GpuNode4 *nodes = nullptr;
    GpuTri *tris = nullptr;
    int n_nodes = 0;
    int n_tris = 0;
};

// Inner-node depth limit of the binary tree the builder starts from.
constexpr int kMaxDepth = 32;
constexpr int kLeafMax = 4;

// 4-wide node with 8-bit quantized child boxes, one 64-byte line:
//   w0 = origin.x, origin.y, origin.z (float bits), exps = ex | ey<<8 | ez<<16
//        (biased exponents: scale_a = 2^(e_a - 127), so lo = origin + q*scale)
//   w1 = bytes qlo_x[4] | qhi_x[4] | qlo_y[4] | qhi_y[4]  (byte c = child c)
//   w2 = bytes qlo_z[4] | qhi_z[4] | leaf[4] | leaf_base
//        leaf byte c = count | offset << 3: count (1..4) triangles of a leaf
//        child starting at triangle slot leaf_base + offset; 0 for an inner
//        or empty slot. The leaf children's triangles are consecutive slots
//        in child order, so offsets stay below 16.
//   w3 = child[4]: inner node index (leaf byte 0), first triangle of a leaf,
//        or -1 for an empty slot
// Quantization rounds outward (floor / ceil), so decoded boxes contain the
// exact ones.
struct alignas(16) GpuNode4 {
    uint4 w0, w1, w2, w3;
};

struct HostBvh4 {
    std::vector<GpuNode4> nodes;
    std::vector<GpuTri> tris;
    int depth = 0;
    int stack_need = 0;  // worst-case traversal stack entries (proved bound)
};

// Stack entries the 4-wide traversal may hold at once.
constexpr int kStack4 = 32;

// Leaf triangle slots a BVH over n triangles may hold (large triangles are
// split into several references, at most doubling the count).
inline size_t bvh_max_refs(int n) { return 2 * (size_t)(n > 0 ? n : 0); }

// Builds the 4-wide quantized BVH (collapsed from the binary SAH tree, with
// the binary depth limit lowered until the worst-case stack fits kStack4).
bool build_bvh4(const float *tri9, int n, int id_base, HostBvh4 &out, std::string &err);

// ---------------------------------------------------------------------------
// Kernel parameter blocks (passed by value)
// ---------------------------------------------------------------------------
struct FrameParams {
    float rot[9];
    int n_lights;
    float light_pos[PV_MAX_LIGHTS][3];
    float light_int[PV_MAX_LIGHTS][3];
};

struct VolumeParams {
    int nx, ny, nz, P, n;
    float ox, oy, oz, sx, sy, sz;
    float max_distance;
    float sky[3];
    int vis_sharpness;
    int blend_mode;     // BlendMode of the frame's blend (never kBlendAuto)
    // When set (second bounce on), the trace also writes every ray's hit
    // record [P][n]: x = leaf-order triangle slot with bit 31 set for the
    // dynamic BVH, or -1 for a miss; y = hit distance (float bits).
    int2 *hitrec;
};

struct SceneView {
    DeviceBvh stat;
    DeviceBvh dyn;
    const float4 *mats;   // [n_triangles][2]: albedo, emission
    float eps;            // shadow-ray offset
};

// Launch shape of the trace: probe brick per wavefront (bx*by*bz = 64); the
// schedule (one wave per packet; persistent waves with per-lane ray refill
// from per-XCD work queues; one wave per packet with stepped lanes); the
// number of top BVH nodes staged in LDS (0, 21 or 85 = the top 1, 3 or 4
// levels); threads per block (128 or 256).
struct TraceConfig {
    int bx = 4, by = 4, bz = 4;
    int persistent = 2;     // 0 packet, 1 persistent with ray refill, 2 packet with stepped lanes
    int top_nodes = 21;
    int block = 256;
    int split_shadows = 0;  // 1: shadow rays in a compacted second pass
};

// Buffers of the split-shadow trace (per volume): hit record per ray
// (leaf-order triangle index with bit 31 set for the dynamic BVH, distance),
// occlusion bits per ray (bit l = light l occluded), shadow-ray queue.
struct ShadowEntry {
    float4 o_tmax;   // origin, tmax
    float4 d_ray;    // direction, (ray index * 8 + light) as int bits
};
struct SplitBuffers {
    int2 *hitrec = nullptr;
    uint32_t *occ = nullptr;
    ShadowEntry *queue = nullptr;
    int *count = nullptr;      // queue length (zeroed by the ray-direction kernel)
    long long capacity = 0;
};

// Work counters of one volume's trace: one per XCD, each on its own 128-byte
// line (the XCDs do not share a contended line), then the split-shadow queue
// length.
constexpr int kQueueStride = 32;                       // ints between counters
constexpr int kQueueInts = 9 * kQueueStride;           // 8 counters + shadow count
inline int *queue_counter(int *q, int k) { return q + k * kQueueStride; }

// Trace (and, in split-shadow mode, the shadow and shade passes).
hipError_t launch_trace(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp, const float4 *dirs,
                        float4 *rays, int32_t *hits, unsigned long long *counts, const TraceConfig &tc,
                        int *queue, const SplitBuffers &split, hipStream_t s);
hipError_t launch_shadow(const SceneView &sv, const SplitBuffers &split, const TraceConfig &tc,
                         unsigned long long *counts, hipStream_t s);
hipError_t launch_shade(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp, const float4 *dirs,
                        float4 *rays, const SplitBuffers &split, hipStream_t s);
}  // namespace pv
