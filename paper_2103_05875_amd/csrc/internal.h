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

struct DeviceBvh {
    GpuNode *nodes = nullptr;
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

// Work description of one volume for the batched launch.
struct BatchVolume {
    VolumeParams vp;
    SceneView sv;
    const float4 *dirs;
    float4 *rays;
    int32_t *hits;
    void *irr;
    void *vis;
    float h;          // effective hysteresis of this frame
    int fp16;
    int first_wave;   // prefix over volumes of trace waves
    int n_waves;
    int first_blend;  // prefix over volumes of blend groups
    int n_blend;
    int bricks_x, bricks_y, bricks_z;
};

// ---------------------------------------------------------------------------
// Launchers (kernels.hip)
// ---------------------------------------------------------------------------
hipError_t launch_raydirs(const FrameParams &fp, int n, float4 *dirs, hipStream_t s);
hipError_t launch_trace(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp, const float4 *dirs,
                        float4 *rays, int32_t *hits, unsigned long long *counts, hipStream_t s);
hipError_t launch_blend(const VolumeParams &vp, const float4 *dirs, const float4 *rays, void *irr, void *vis,
                        int fp16, float h, hipStream_t s);
hipError_t launch_batched(const BatchVolume *vols_dev, int n_vols, int total_waves, int total_blend,
                          const FrameParams *frames_dev, int *queue_dev, int *done_dev, int *status_dev,
                          hipStream_t s);
hipError_t launch_raydirs_batched(const FrameParams *frames_dev, const int *ns_dev, float4 *const *dirs_dev,
                                  int n_vols, hipStream_t s);

struct PackBuffers {
    const uint16_t *cur_irr, *cur_vis;   // tiles
    uint16_t *ref_irr, *ref_vis;         // interiors
    uint8_t *mask_irr, *mask_vis;
    uint32_t *rank_irr, *rank_vis;
    uint8_t *packet;
};
hipError_t launch_pack_mask(const PackBuffers &b, int P, float tau_irr, float tau_vis, hipStream_t s);
hipError_t launch_pack_scan(const PackBuffers &b, int P, uint32_t client, uint32_t seq, hipStream_t s);
hipError_t launch_pack_compact(const PackBuffers &b, int P, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace pv
