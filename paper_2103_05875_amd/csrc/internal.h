// Internal declarations shared by the host side and the kernels of the
// probe-volume library. Not part of the public ABI.
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

// BVH node with both child boxes (64 bytes, one node fetch tests two boxes).
//   bx = (lo.x[0], lo.x[1], hi.x[0], hi.x[1]), by, bz likewise
//   meta = (child[0], child[1], count[0], count[1]) as int bits
// count > 0: leaf, child = first triangle of the leaf in the reordered
// triangle array; count == 0: inner node index, or -1 for an empty slot
// (its box is empty so it is never entered).
struct alignas(16) GpuNode {
    float4 bx, by, bz;
    int4 meta;
};

// Triangle in leaf order: v0 (w = original triangle id as int bits),
// e1 = v1 - v0, e2 = v2 - v0 (w unused).
struct alignas(16) GpuTri {
    float4 v0, e1, e2;
};

struct GpuNode4;

struct DeviceBvh {
    GpuNode4 *nodes = nullptr;
    GpuTri *tris = nullptr;
    int n_nodes = 0;
    int n_tris = 0;
};

// Host BVH build result.
struct HostBvh {
    std::vector<GpuNode> nodes;
    std::vector<GpuTri> tris;
    int depth = 0;
};

// Maximum inner-node depth the builder produces; the traversal stack holds
// at most this many entries.
constexpr int kMaxDepth = 32;
constexpr int kLeafMax = 4;

// Builds a BVH over triangles (tri9: [n][9] float) with original ids
// id_base + i. Returns false if a triangle is not finite.
bool build_bvh(const float *tri9, int n, int id_base, HostBvh &out, std::string &err);

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
};

struct SceneView {
    DeviceBvh stat;
    DeviceBvh dyn;
    const float4 *mats;   // [n_triangles][2]: albedo, emission
    float eps;            // shadow-ray offset
};

// Blend weight tables of one volume-frame, written by the ray-direction
// kernel (rows: 64 irradiance texels, then 256 visibility texels):
//   w[((j / 4) * kTexRows + t) * 4 + j % 4]  weight of ray j for texel row t;
//                                            rays n .. (n rounded up to a
//                                            multiple of 128) - 1 weigh 0
//   part[b * kTexRows + t]                   sum of row t over rays
//                                            kRaysPerPart*b .. +kRaysPerPart-1
// The blend sums the parts in order b = 0, 1, ... for the row totals.
constexpr int kTexRows = 64 + 256;
constexpr int kRaysPerPart = 64;
constexpr int kBlendTile = 8;  // probes per blend block
struct WeightTables {
    float *w = nullptr;
    float *part = nullptr;
    int k4 = 0;
    int nparts = 0;
};
inline size_t weight_table_floats(int n) { return (size_t)((n + 127) / 128) * 128 * kTexRows; }
inline size_t weight_part_floats(int n) { return (size_t)((n + kRaysPerPart - 1) / kRaysPerPart) * kTexRows; }

// Work description of one volume for the batched launch.
struct BatchVolume {
    VolumeParams vp;
    SceneView sv;
    const float4 *dirs;
    WeightTables wt;
    float4 *rays;
    int32_t *hits;
    void *irr;
    void *vis;
    float h;          // effective hysteresis of this frame
    int fp16;
    int first_wave;   // prefix over volumes of trace packets (multiple of 4)
    int n_waves;
    int first_blend;  // prefix over volumes of blend groups
    int n_blend;
    int bricks_x, bricks_y, bricks_z;
};

// Launch shape of the trace: probe brick per wavefront (bx*by*bz = 64),
// persistent grid with per-lane ray refill from per-XCD work queues or one
// wave per packet, number of
// top BVH nodes staged in LDS (0, 21 or 85 = the top 1, 3 or 4 levels), and
// threads per block (128 or 256).
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

// ---------------------------------------------------------------------------
// Launchers (trace.hip, blend.hip, batched.hip, pack.hip)
// ---------------------------------------------------------------------------
// Work counters of one volume's trace: one per XCD, each on its own 128-byte
// line (the XCDs do not share a contended line), then the split-shadow queue
// length.
constexpr int kQueueStride = 32;                       // ints between counters
constexpr int kQueueInts = 9 * kQueueStride;           // 8 counters + shadow count
inline int *queue_counter(int *q, int k) { return q + k * kQueueStride; }

// Directions and weight tables; the 9 work counters are zeroed for the trace that follows
hipError_t launch_raydirs(const FrameParams &fp, const VolumeParams &vp, float4 *dirs, const WeightTables &wt,
                          int *queue, hipStream_t s);
hipError_t launch_trace(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp, const float4 *dirs,
                        float4 *rays, int32_t *hits, unsigned long long *counts, const TraceConfig &tc,
                        int *queue, const SplitBuffers &split, hipStream_t s);
hipError_t launch_shadow(const SceneView &sv, const SplitBuffers &split, const TraceConfig &tc,
                         unsigned long long *counts, hipStream_t s);
hipError_t launch_shade(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp, const float4 *dirs,
                        float4 *rays, const SplitBuffers &split, hipStream_t s);
hipError_t launch_blend(const VolumeParams &vp, const WeightTables &wt, const float4 *rays, void *irr, void *vis,
                        int fp16, float h, hipStream_t s);
// Batched trace / blend over every volume of a batch (descriptors on the
// device; each volume's first_wave a multiple of 4).
hipError_t launch_trace_batched(const BatchVolume *vols_dev, int n_vols, int total_waves, const FrameParams *frames_dev,
                                bool short_stack, hipStream_t s);
hipError_t launch_blend_batched(const BatchVolume *vols_dev, int n_vols, int total_blend, hipStream_t s);
hipError_t launch_raydirs_batched(const BatchVolume *vols_dev, const FrameParams *frames_dev, int n_vols,
                                  int max_parts, hipStream_t s);

struct PackBuffers {
    const uint16_t *cur_irr, *cur_vis;   // tiles
    uint16_t *ref_irr, *ref_vis;         // interiors
    uint8_t *mask_irr, *mask_vis;
    int4 *tiles;      // per tile of 16 probes: changed counts (irr, vis) and last changed probe
                      // (irr, vis), replaced by their exclusive prefix by the mask kernel
    uint32_t *done;   // [0] mask blocks finished, [1] compaction blocks finished (both left 0),
                      // [2] K_irr, [3] K_vis
    uint8_t *packet;
};
hipError_t launch_pack_mask(const PackBuffers &b, int P, float tau_irr, float tau_vis, hipStream_t s);
hipError_t launch_pack_compact(const PackBuffers &b, int P, uint32_t client, uint32_t seq, hipStream_t s);
constexpr int kPackTile = 16;  // probes per pack block
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace pv
