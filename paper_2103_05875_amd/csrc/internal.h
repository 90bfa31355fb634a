// Internal declarations shared by the host side and the kernels of the
// probe-volume library. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "probestream.h"
#include "trace_layout.h"

namespace pv {

constexpr int kTexRows = 64 + 256;  // texel rows of the blend: 64 irradiance, then 256 visibility
constexpr int kBlendTile = 8;       // probes per block of the per-tile blend

// Blend paths (pv_blend_mode values; see blend_device.h):
//   kBlendBF16x3  weight table, products on the BF16 matrix cores as three
//                 products of high and low halves (FP32 accumulate)
//   kBlendF32     weight table, FP32 matrix cores
//   kBlendTiles   weights evaluated per 8-probe tile in registers, FP32
//                 matrix cores (no table)
//   kBlendVALU    weight table, FP32 vector FMAs
//   kBlendBF16x6  weight table, BF16 matrix cores: operands split into three
//                 BF16 parts, the six products down to 2^-18 (FP32 accumulate)
enum BlendMode : int { kBlendAuto = 0, kBlendBF16x3 = 1, kBlendF32 = 2, kBlendTiles = 3, kBlendVALU = 4, kBlendBF16x6 = 5 };
// The default path of a volume of P probes: the per-tile weights below
// kTableMinProbes (a table costs a pass over every weight per frame, which
// small volumes do not earn back), the three-part BF16 table product from
// there (as accurate as the FP32 products and 1.2-1.6x faster).
constexpr int kTableMinProbes = 2048;
inline int auto_blend_mode(int P) { return P >= kTableMinProbes ? kBlendBF16x6 : kBlendTiles; }

// The per-volume-frame weight table follows the ray directions in their
// buffer: steps of kWStep rays x kMTiles row tiles of 16 texel rows x 64
// lanes x 32 bytes (the lane's MFMA A-operand fragment of that step: eight
// FP32 weights, or eight BF16 high halves then eight low halves; 48 bytes
// for kBlendBF16x6: high, middle and low parts), then per group of kWGroup
// steps the kTexRows FP32 partial row totals. The buffer is sized for the
// widest layout.
constexpr int kWStep = 32;
constexpr int kMTiles = kTexRows / 16;
__host__ __device__ inline size_t dirs_span(int n) { return ((size_t)n * 16 + 255) / 256 * 256; }
__host__ __device__ inline size_t wtab_steps(int n) { return (size_t)(n + kWStep - 1) / kWStep; }
__host__ __device__ inline int wtab_lane_bytes(int mode) { return mode == kBlendBF16x6 ? 48 : 32; }
__host__ __device__ inline size_t wtab_rows_offset(int n, int mode) {
    return wtab_steps(n) * kMTiles * 64 * wtab_lane_bytes(mode);
}
// Table blocks take groups of kWGroup steps; each group leaves its own row
// of kTexRows partial totals, which the blend adds in order.
constexpr int kWGroup = 4;
__host__ __device__ inline int wtab_groups(int n) { return (int)((wtab_steps(n) + kWGroup - 1) / kWGroup); }
__host__ __device__ inline size_t wtab_bytes(int n) {
    return wtab_rows_offset(n, kBlendBF16x6) + (size_t)wtab_groups(n) * kTexRows * 4;
}

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
    int first_wave;   // prefix over volumes of trace packets (multiple of 4)
    int n_waves;
    int first_blend;  // prefix over volumes of blend groups
    int n_blend;
    int first_bounce; // prefix over volumes of second-bounce blocks (0 blocks without it)
    int n_bounce;
    uint8_t *active;  // probe activity (classifying volumes), else null
    int first_classify; // prefix over volumes of classification blocks (0 blocks without it)
    int n_classify;
    int bricks_x, bricks_y, bricks_z;
    int bx, by, bz;   // the volume's probe brick (64 probes per trace packet)
    int top_nodes;    // top BVH nodes the volume's trace blocks stage in LDS (0, 21 or 85)
};

// ---------------------------------------------------------------------------
// Launchers (trace.hip, blend.hip, batched.hip, bounce.hip, pack.hip)
// ---------------------------------------------------------------------------
// Ray directions; the 9 work counters are zeroed for the trace that follows
// (plus the weight table after the directions when the blend mode uses one)
hipError_t launch_raydirs(const FrameParams &fp, const VolumeParams &vp, float4 *dirs, int *queue, hipStream_t s);
int raydir_blocks(int n);
int weight_blocks(int mode, int n);  // extra blocks of the direction launch that build the table
int blend_blocks(int P, int mode);  // 256-thread blocks of one volume's blend
hipError_t launch_blend(const VolumeParams &vp, const float4 *dirs, const float4 *rays, void *irr, void *vis,
                        int fp16, float h, hipStream_t s);
// Batched trace / blend over every volume of a batch (descriptors on the
// device; each volume's first_wave a multiple of 4).
hipError_t launch_trace_batched(const BatchVolume *vols_dev, int n_vols, int total_waves, const FrameParams *frames_dev,
                                bool short_stack, int max_top, hipStream_t s);
// Which batched blend kernel a batch takes: every path and map type, or one
// map type with the per-tile, FP32-table and BF16x6-table paths only.
enum : int { kBatchBlendAny = 0, kBatchBlendAutoHalf = 1, kBatchBlendAutoFloat = 2 };
hipError_t launch_blend_batched(const BatchVolume *vols_dev, int n_vols, int total_blend, int kind, hipStream_t s);
hipError_t launch_raydirs_batched(const BatchVolume *vols_dev, const FrameParams *frames_dev, int n_vols,
                                  int dir_blocks, hipStream_t s);

// Attainable ceilings (ceilings.hip): stream copy, FP32 FMA chains, FP32
// MFMA chains; 'out' holds blocks * 256 floats.
hipError_t launch_ceil_copy(const void *src, void *dst, size_t bytes, int blocks, hipStream_t s);
hipError_t launch_ceil_fma(float *out, int blocks, int iters, hipStream_t s);
hipError_t launch_ceil_mfma(float *out, int blocks, int iters, hipStream_t s);

// Second bounce (bounce.hip): adds albedo x the stored maps' query to every
// hit record's radiance (vp.hitrec must be set); the client query.
int bounce_blocks(int P, int n);
hipError_t launch_bounce(const VolumeParams &vp, const SceneView &sv, const float4 *dirs, float4 *rays,
                         const void *irr, const void *vis, int fp16, hipStream_t s);
hipError_t launch_bounce_batched(const BatchVolume *vols_dev, int n_vols, int total_blocks, hipStream_t s);
hipError_t launch_probe_query(const VolumeParams &vp, const void *irr, const void *vis, int fp16, const float *pts,
                              const float *nrms, float *out, long long n, hipStream_t s);

struct PackBuffers {
    const uint16_t *cur_irr, *cur_vis;   // tiles
    uint16_t *ref_irr, *ref_vis;         // interiors
    uint8_t *mask_irr, *mask_vis;
    uint32_t *tsum;   // per tile of kPackTile probes: its own summary (changed counts, last two
                      // changed probes per texture) in 32 bits, written by the mask pass
    int4 *tiles;      // per tile, written by the scan: changed counts (irr, vis) and last changed
                      // probe (irr, vis) of the tiles before it
    int2 *tiles2;     // per tile, likewise: the changed probe before the last one (irr, vis)
    uint32_t *totals; // K_irr, K_vis, last and second-last changed irradiance probe (written by the scan)
    unsigned long long *cks; // checksum counters: kCksGroups group words and one final word, 128 bytes
                             // apart; zero between packs (the last adder of each word resets it)
    uint8_t *packet;
    const uint8_t *active;  // [P] volume's active probes, or null (all)
    const uint8_t *view;    // [P] client's visible set, or null (all)
};
hipError_t launch_pack_mask(const PackBuffers &b, int P, float tau_irr, float tau_vis, hipStream_t s);
hipError_t launch_pack_scan(const PackBuffers &b, int P, hipStream_t s);
hipError_t launch_pack_compact(const PackBuffers &b, int P, uint32_t client, uint32_t seq, hipStream_t s);
constexpr int kPackTile = 8;   // probes per pack block
// Up to this many tiles every compaction block reduces the tile summaries
// itself and the scan launch is skipped (its few microseconds of launch
// latency exceed the redundant reads); above it the one-block scan runs.
constexpr int kPackFusedTiles = 2048;
bool pack_fused(int P);
// The packet checksum is summed by the compaction blocks themselves: each
// adds its share to one of kCksGroups group words (tile % kCksGroups), the
// last block of a group adds the group's sum to the final word, the last of
// those writes the header. A word holds its adders' count in bits 48-63 and
// their sum in bits 0-47 (at most 256 shares of 32 bits per group at 8,192
// tiles), so one 64-bit atomic add both adds and tells a block whether it is
// the last; no fence or second launch is needed.
constexpr int kCksGroups = 32;
constexpr int kCksStride = 16;  // 64-bit words between counters (128 bytes)
constexpr size_t kCksBytes = (size_t)(kCksGroups + 1) * kCksStride * 8;
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
// Pack without allocation (pack.hip): intermediates live in a static device
// array sized for kNoAllocMaxProbes probes; its address on a device is taken
// once with that device current (noalloc_scratch_init, from pv_ctx_create).
constexpr int kNoAllocMaxProbes = PV_MAX_PROBES;
constexpr size_t kNoAllocScratchBytes = 8192 * 16 + 8192 * 8 + 4352 + 8192 * 4 + 256 + 65536 + 65536;
hipError_t noalloc_scratch_init(int device);
unsigned char *noalloc_scratch(int device);  // null before noalloc_scratch_init on that device
hipError_t launch_pack_noalloc(unsigned char *scratch_dev, const uint16_t *cur_irr, const uint16_t *cur_vis,
                               uint16_t *ref_irr, uint16_t *ref_vis, int P, float tau_irr, float tau_vis,
                               uint32_t client, uint32_t seq, uint8_t *packet, hipStream_t s);

// Client-side unpack (receive.hip). The packet's header has been checked on
// the host; the index and the checksum are checked on the device before any
// texel is written.
struct RxStatus {
    uint32_t sum;      // payload checksum accumulated on the device
    int bad_index;     // 1: an index entry is out of range or not increasing
};
struct RxBuffers {
    const uint8_t *pkt;   // device copy of the packet
    int P, K_irr, K_vis;
    uint32_t checksum;    // from the header
    long long payload_words;
    uint16_t *irr, *vis;  // the client's tiles (with guard bands)
    int *idx;             // [K_irr + K_vis] decoded probe numbers
    RxStatus *status;
};
hipError_t launch_receive(const RxBuffers &b, hipStream_t s);

// Probe selection (select.hip): activity from the frame's hit records, and
// a client's visible set from a spherical view at its position.
hipError_t launch_classify(const VolumeParams &vp, const SceneView &sv, const float4 *dirs, uint8_t *active,
                           hipStream_t s);
hipError_t launch_client_view(const VolumeParams &vp, const SceneView &sv, float ex, float ey, float ez, int n_rays,
                              uint8_t *view, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t s);
int classify_blocks(int P);
hipError_t launch_classify_batched(const BatchVolume *vols_dev, int n_vols, int total_blocks, hipStream_t s);

// Entropy stage (entropy.hip).
constexpr int kEntStreams = 11;  // index section, 6 irradiance planes, 4 visibility planes
struct EntBuffers {
    const uint8_t *pkt;      // the packet (its header gives the stream sizes)
    uint32_t *hist;          // [11][256], zeroed before the histogram
    uint8_t *lens;           // [11][256]
    uint32_t *codes;         // [11][256]
    uint32_t *chunk_bits;    // [11][max_chunks]
    unsigned long long *chunk_off;  // [11][max_chunks] byte offsets in the container
    unsigned long long *total;      // container bytes
    uint8_t *out;            // the container
    int max_chunks;          // chunks of the longest possible stream
};
struct EntChunk {
    int stream, n_sym;
    unsigned int bits;
    unsigned long long in_off, out_off;  // container / packet byte offsets
};
// Chunks per decode block (one wavefront, one chunk per lane; the decode of a
// chunk is a serial chain of LDS lookups, so fewer chunks per wavefront
// spread the chains over more SIMDs).
constexpr int kEntDecodeChunks = 8;
struct EntBlock {
    int stream, first, n;    // up to kEntDecodeChunks consecutive chunks of one stream
};
struct EntDecode {
    const uint8_t *in;       // the container
    unsigned long long stream_base[kEntStreams];  // offsets of the streams' tables
    const EntChunk *chunks;
    const EntBlock *blocks;
    int n_blocks;
    uint8_t *pkt;            // decoded packet (index padding cleared by the host)
};
hipError_t launch_entropy_hist(const EntBuffers &e, int max_chunks, hipStream_t s);
hipError_t launch_entropy_encode(const EntBuffers &e, int max_chunks, hipStream_t s);  // after the tables
hipError_t launch_entropy_decode(const EntDecode &d, hipStream_t s);

// Codec surfaces (yuv.hip): plane sizes for P probes, C tiles per atlas row.
struct YuvDims {
    long long w, h;    // irradiance planes (samples)
    long long wv, hv;  // visibility planes
};
inline YuvDims yuv_dims(int P, int C) {
    const long long rows = (P + C - 1) / C;
    return YuvDims{8ll * C, 8 * rows, (64ll * C + 2) / 3, 16 * rows};
}
hipError_t launch_yuv_encode(const uint16_t *irr, const uint16_t *vis, int P, int C, float k, uint16_t *irr_planes,
                             uint8_t *vis_planes, const YuvDims &d, hipStream_t s);
hipError_t launch_yuv_decode(const uint16_t *irr_planes, const uint8_t *vis_planes, int P, int C, uint32_t *codes,
                             uint16_t *vis, const YuvDims &d, hipStream_t s);

}  // namespace pv
