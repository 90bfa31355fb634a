/*
 * probestream.h -- C ABI of the MI355X (gfx950) probe-volume update and
 * lossless delta-pack library.
 *
 * The operations follow "A Distributed, Decoupled System for Losslessly
 * Streaming Dynamic Light Probes to Thin Clients" (Stengel et al. 2021):
 *
 *   - a GI server computes view-independent probe textures from the current
 *     scene state (Section 3.1, architecture overview): pv_update_probes;
 *   - each probe holds an octahedral irradiance map (8x8 interior texels in a
 *     10x10 tile) and a visibility map of mean distance and mean squared
 *     distance (16x16 interior in an 18x18 tile) (Section 3.2, Eq. 1 and
 *     Eq. 2 and the visibility paragraph); the update itself is the
 *     irradiance-volume method the paper adopts (Section 3.2, first
 *     paragraph): rays per probe, closest hit, shading, cosine-weighted blend
 *     with hysteresis, guard-band copy;
 *   - for each client the server keeps last-transmitted textures, selects the
 *     probes that changed (Section 3.4, change thresholding), drops the
 *     guard bands and sends an index-based update with a delta-coded 2-byte
 *     probe index buffer (Section 3.4, repacking and update textures), with
 *     every FP16 value split into its two bytes (Section 3.3, visibility
 *     encoding): pv_pack_delta.
 *
 * Conventions
 *   - Every call returns a pv_status; outputs are written only on PV_OK and
 *     pv_last_error() (thread-local) describes the last failure.
 *   - Work is enqueued asynchronously on the given HIP stream (a
 *     hipStream_t passed as void*; NULL is HIP's default stream, as in HIP
 *     itself). Device faults surface as PV_ERR_DEVICE at the next pv_sync
 *     or blocking call.
 *   - The library owns every handle and all device memory (maps, client
 *     references, BVHs, ray buffers, packets). Host arrays passed in are
 *     copied before the call returns and never retained. Device pointers
 *     handed out (pv_get_maps, pv_get_rays, pv_packet_device) are borrowed:
 *     valid until the handle is destroyed, contents valid until the next
 *     update / pack on that handle.
 *   - Handles are not thread-safe. Different volumes may be updated on
 *     different streams concurrently; a scene may be shared by volumes.
 *   - destroy(NULL) is PV_OK.
 */
#ifndef PROBESTREAM_H
#define PROBESTREAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* every entry point below is exported from the shared library */
#pragma GCC visibility push(default)

typedef struct pv_ctx pv_ctx;
typedef struct pv_scene pv_scene;
typedef struct pv_volume pv_volume;
typedef struct pv_client pv_client;

typedef enum {
    PV_OK = 0,
    PV_ERR_ARG = -1,         /* invalid argument (message says which) */
    PV_ERR_OOM = -2,         /* device or host allocation failed */
    PV_ERR_DEVICE = -3,      /* HIP runtime / device error */
    PV_ERR_STATE = -4,       /* call not valid in the handle's state */
    PV_ERR_CAPACITY = -5,    /* caller buffer or memory budget too small */
    PV_ERR_UNSUPPORTED = -6  /* valid request the library does not implement */
} pv_status;

typedef enum { PV_MAP_FP32 = 0, PV_MAP_FP16 = 1 } pv_map_format;

/* pv_volume_desc.flags */
#define PV_FIRST_FRAME_NO_HISTORY 1u /* first update of a volume uses h = 0 */
#define PV_KEEP_HITS 2u              /* keep the hit triangle id of every ray */
/* Second bounce (Sec. 3.2's shading-time query applied during the update):
 * every hit adds its albedo times the volume's query (pv_probe_query) at the
 * hit point moved off the surface along its normal by a tenth of the
 * smallest probe spacing, evaluated on the maps as they stand before the
 * frame's blend. Repeated frames thus accumulate multiple bounces. Costs an
 * 8-byte hit record per ray and one more launch per update. */
#define PV_MULTI_BOUNCE 4u
/* Probe activity (Sec. 3.4: only active probes are worth sending): every
 * update classifies each probe from its rays -- inactive when more than a
 * quarter of them hit a triangle from behind (the side its normal
 * (v1 - v0) x (v2 - v0) points away from, i.e. the probe sits inside a
 * solid; scenes wind triangles with normals out of solids) or when none
 * hits anything closer than the cell diagonal |spacing| -- and the pack
 * sends active probes only. Costs an 8-byte hit record per ray, P bytes
 * and one launch per update. Before the first update every probe counts as
 * active. */
#define PV_CLASSIFY 8u

#define PV_MAX_LIGHTS 8
#define PV_MAX_PROBES 65536          /* the 2-byte probe index (Section 3.4) */
#define PV_MAX_RAYS 4096

/*
 * A regular probe grid. Probe p = x + nx*(y + ny*z) sits at
 * origin + spacing * (x, y, z). Ray directions: a spherical-Fibonacci set of
 * rays_per_probe directions under the frame's rotation, shared by every probe.
 * Maps: irradiance tiles [P][3][irr_res+2][irr_res+2] and visibility tiles
 * [P][2][vis_res+2][vis_res+2] (channel-planar, row-major, 1-texel guard
 * band), FP32 or FP16 storage, FP32 arithmetic. The library supports
 * irr_res = 8 and vis_res = 16 (the paper's 10x10 and 18x18 tiles).
 */
typedef struct {
    int nx, ny, nz;
    float origin[3], spacing[3];
    int rays_per_probe;      /* 1 .. PV_MAX_RAYS */
    int irr_res, vis_res;    /* 8, 16 */
    float hysteresis;        /* h in [0, 1): new = h*old + (1-h)*estimate */
    float max_distance;      /* distances are clamped to this (> 0) */
    int vis_sharpness;       /* visibility weight = max(0, cos)^s, s in [1, 128] */
    pv_map_format format;
    float sky[3];            /* radiance of rays that leave the scene */
    uint32_t flags;          /* PV_FIRST_FRAME_NO_HISTORY | PV_KEEP_HITS | PV_MULTI_BOUNCE | PV_CLASSIFY */
} pv_volume_desc;

typedef struct {
    float pos[3];
    float intensity[3];      /* radiant intensity (inverse-square falloff) */
} pv_point_light;

/*
 * Triangle scene. positions: n_vertices*3 floats; indices: n_triangles*3;
 * albedo: n_triangles*3 (diffuse reflectance per triangle); emission:
 * n_triangles*3 or NULL. The last n_dynamic_triangles triangles may be moved
 * per frame with pv_scene_set_dynamic. lights: the default lights of a
 * frame that passes none. Triangles are two-sided.
 */
typedef struct {
    int n_vertices;
    const float *positions;
    int n_triangles;
    const uint32_t *indices;
    const float *albedo;
    const float *emission;
    int n_dynamic_triangles;
    int n_lights;
    const pv_point_light *lights;
} pv_scene_desc;

/* Per-frame input: the ray-set rotation (row-major 3x3, a proper rotation)
 * and the point lights (n_lights = 0 and lights = NULL: the scene's). */
typedef struct {
    float rotation[9];
    int n_lights;
    const pv_point_light *lights;
} pv_frame;

const char *pv_last_error(void);
const char *pv_version(void);

/* Context bound to one HIP device; owns a default stream. */
pv_status pv_ctx_create(int hip_device, pv_ctx **out);
pv_status pv_ctx_destroy(pv_ctx *ctx);

/*
 * The scene the server traces probe rays against (Sec. 3.1). Copies the
 * scene to the device and builds its BVH on the host (binned surface-area
 * heuristic). Inputs must be finite and indices < n_vertices.
 * The shadow-ray offset is 1e-4 times the diagonal of the bounding box of
 * the static triangles.
 */
pv_status pv_scene_create(pv_ctx *ctx, const pv_scene_desc *desc, pv_scene **out);
/* New positions (n_dynamic_triangles*9 floats, host) of the dynamic
 * triangles, in effect for work enqueued on 'stream' after this call. */
pv_status pv_scene_set_dynamic(pv_scene *scene, const float *positions, void *stream);
pv_status pv_scene_destroy(pv_scene *scene);
/* Copy of the scene's device BVH (dynamic = 0: the static triangles; 1: the
 * dynamic ones as of the last pv_scene_set_dynamic), synchronous, for
 * inspection and for replaying the traversal on the host. counts receives
 * (nodes, triangle slots) and eps the shadow-ray offset; with NULL buffers
 * only those are returned. Nodes: 64 bytes each, breadth first from the
 * root at 0, as four 16-byte words:
 *   w0: origin x, y, z (float), per-axis exponents e_x | e_y << 8 | e_z << 16
 *       (a child box coordinate is origin + q * 2^(e - 127), q a byte)
 *   w1: bytes q_lo_x[4] | q_hi_x[4] | q_lo_y[4] | q_hi_y[4] (byte c = child c)
 *   w2: bytes q_lo_z[4] | q_hi_z[4] | leaf[4] | first leaf slot (u32);
 *       leaf byte = count (bits 0-2, 0 for an inner child) | slot offset
 *       from the first leaf slot (bits 3-6)
 *   w3: child[4] (int32): inner node index, or -1 for an empty slot
 * Triangle slots: 48 bytes, vertices v0, v1, v2 as float4 (v0.w = the
 * triangle's index as int32 bits); a triangle may fill several slots.
 * PV_ERR_CAPACITY when a buffer is smaller than counts require. */
pv_status pv_scene_read_bvh(pv_scene *scene, int dynamic, void *nodes_host, uint64_t nodes_cap, void *tris_host,
                            uint64_t tris_cap, int64_t counts[2], float *eps);

/* A probe volume (Sec. 3.2: a regular grid of probes, each with an
 * octahedral irradiance tile and a visibility tile of mean and mean squared
 * distance, both with a one-texel guard band). Maps zeroed, frame counter 0.
 * PV_ERR_ARG for an invalid descriptor, PV_ERR_OOM when device memory runs
 * out (nothing is left allocated). */
pv_status pv_create_volume(pv_ctx *ctx, const pv_volume_desc *desc, pv_volume **out);
pv_status pv_volume_destroy(pv_volume *vol);
/* Device bytes pv_create_volume would allocate for desc (admission). */
pv_status pv_volume_footprint(const pv_volume_desc *desc, uint64_t *bytes);
/* The scene the volume's rays are traced against (Sec. 3.1); the scene is
 * borrowed and must outlive the volume's updates. */
pv_status pv_set_scene(pv_volume *vol, pv_scene *scene);

/*
 * One full update (async; Sec. 3.1 server ray tracing of probe textures,
 * Sec. 3.2 blend of the rays into the irradiance and visibility maps, Eq. 1
 * and Eq. 2, with hysteresis): ray directions, trace + shade every
 * (probe, ray), blend both maps with hysteresis, rebuild guard bands.
 * A texel whose weight sum over the rays is at most 1e-20 keeps its value.
 * Ray records are kept in the volume's ray buffer (pv_get_rays).
 */
pv_status pv_update_probes(pv_volume *vol, const pv_frame *frame, void *stream);
/*
 * pv_update_probes for a pipeline of frames (the same kernels and results):
 * the ray directions and the trace are enqueued at once, and the kernels
 * after them, which rewrite what a pack of the previous frame reads (the
 * maps, the probe activity), first wait for 'event' (a hipEvent_t passed as
 * void*, recorded by the caller after those packs, e.g. on another stream).
 * The packs of frame f then overlap the directions and trace of frame f + 1.
 * PV_ERR_ARG when event is NULL.
 */
pv_status pv_update_probes_after(pv_volume *vol, const pv_frame *frame, void *stream, void *event);

/*
 * The same update for n volumes in one go, enqueued on 'stream': three
 * launches whatever n is -- ray directions of every volume, the trace of
 * every wavefront packet of every volume, the blend of
 * every probe group of every volume -- so small volumes share the device
 * instead of each filling it alone. Results are bit-identical to n
 * pv_update_probes calls with the default trace launch shape.
 */
pv_status pv_update_probes_batched(pv_volume *const *vols, const pv_frame *frames, int n, void *stream);

/*
 * A captured HIP graph of the batched update of a fixed set of volumes:
 * copy nodes refreshing the device-resident descriptors and frame
 * parameters from pinned host memory, then the three batched kernels.
 * pv_batch_graph_launch writes the frames into the pinned buffer (waiting for
 * the graph's previous launch to finish first) and launches the graph on
 * 'stream'; results equal pv_update_probes_batched. The volumes must outlive
 * the graph.
 */
typedef struct pv_batch_graph pv_batch_graph;
pv_status pv_batch_graph_create(pv_volume *const *vols, int n, pv_batch_graph **out);
pv_status pv_batch_graph_launch(pv_batch_graph *graph, const pv_frame *frames, void *stream);
pv_status pv_batch_graph_destroy(pv_batch_graph *graph);

/*
 * Blend + hysteresis + guard bands from externally supplied ray records
 * (device pointer, [P][rays_per_probe] x float4 {L.r, L.g, L.b, distance}),
 * with the directions of 'frame'. Advances the frame counter like an update.
 */
pv_status pv_blend_rays(pv_volume *vol, const pv_frame *frame, const void *rays_dev, void *stream);

/* Borrowed device pointers to the current tiles, densely packed in the
 * volume's map format (float or binary16): irradiance [P][3][10][10]
 * (channel r, g, b; 8x8 interior with its guard band), visibility
 * [P][2][18][18] (mean distance, mean squared distance; 16x16 interior).
 * Probe p's tiles start at element p * 300 and p * 648: no padding. */
pv_status pv_get_maps(pv_volume *vol, void **irr_dev, void **vis_dev);
/* Borrowed device pointers: ray records [P][n] float4, hit triangle ids
 * [P][n] int32 (-1 = miss; NULL unless PV_KEEP_HITS), directions [n] float4. */
pv_status pv_get_rays(pv_volume *vol, void **rays_dev, void **hits_dev, void **dirs_dev);
/*
 * Shading query of the volume's current maps (Sec. 3.2: probe visibility by
 * a Chebyshev test on the stored mean and mean-squared distances), the step
 * a client runs per shaded point: the mean radiance arriving at point i
 * around normal i, as the weighted mean over the eight probes at the corners
 * of the grid cell holding the point (clamped to the grid) of each probe's
 * irradiance tile filtered bilinearly in the normal's direction. A probe's
 * weight is its trilinear weight, times var / (var + (d - mu)^2) when the
 * point's distance d from it exceeds the mean distance mu its visibility
 * tile records in that direction (var = mu2 - mu^2, floored at 0; var = 0
 * excludes the probe). 0 when every weight vanishes.
 * points_dev, normals_dev: device float [n][3] (normals non-zero, any
 * length); out_dev: device float [n][3], written. Asynchronous on 'stream';
 * n = 0 does nothing. FP32 arithmetic on FP32 or FP16 maps.
 */
pv_status pv_probe_query(pv_volume *vol, const float *points_dev, const float *normals_dev, int64_t n, float *out_dev,
                         void *stream);
/* Replace the maps from host memory (checkpoint import) and set the frame
 * counter; synchronous. */
pv_status pv_set_maps(pv_volume *vol, const void *irr_host, const void *vis_host, int64_t frame);
/* Copy the maps to host memory (checkpoint export); synchronous. */
pv_status pv_read_maps(pv_volume *vol, void *irr_host, void *vis_host, int64_t *frame);

/*
 * Per-client server state: last-transmitted interiors (all-zero bits at
 * creation, i.e. the first pack sends every probe that is not all zero) and
 * a device packet buffer sized for a full update. FP16 volumes only.
 */
pv_status pv_client_create(pv_volume *vol, uint32_t client_id, pv_client **out);
pv_status pv_client_destroy(pv_client *client);
/* Zero the client's reference: the next pack resends everything (as a
 * video I-frame would after loss). */
pv_status pv_client_reset(pv_client *client, void *stream);
pv_status pv_client_footprint(const pv_volume_desc *desc, uint64_t *bytes);

/*
 * Build the client's next packet on the device (async) from the volume's
 * current maps (Sec. 3.3: binary16 texels split into two byte planes;
 * Sec. 3.4: change thresholding against the client's last-transmitted
 * textures, probe index buffer). A probe is sent for a texture when any interior texel
 * differs from the client's reference: bit pattern differs (tau = 0), or
 * |cur - ref| > tau exactly (tau > 0). Sent probes are written to the
 * reference. Packet layout (little endian):
 *   header 32 B: u32 magic 0x4B505650 ("PVPK"), u16 version 1, u16 32,
 *                u32 client, u32 seq, u32 P, u32 K_irr, u32 K_vis,
 *                u32 checksum
 *   index: K_irr then K_vis u16 entries, delta coded (first = probe index,
 *          then difference to the previous sent probe), zero padded to a
 *          multiple of 16 bytes
 *   irradiance planes (R lo, R hi, G lo, G hi, B lo, B hi), each K_irr*64
 *          bytes: byte k*64 + t = that byte of cur XOR ref for the k-th sent
 *          probe, interior texel t = row*8 + column
 *   visibility planes (mean lo, mean hi, mean^2 lo, mean^2 hi), K_vis*256 B
 *   checksum = sum over payload u32 words w_i (i from 0 after the header) of
 *          fmix32(w_i ^ (i * 0x9E3779B9)) mod 2^32 (MurmurHash3 finaliser).
 * seq counts the client's packs from 0.
 */
pv_status pv_pack_delta(pv_client *client, float tau_irr, float tau_vis, void *stream);
/* Borrowed device pointer to the packet buffer and its capacity. */
pv_status pv_packet_device(pv_client *client, const void **packet_dev, uint64_t *capacity);
/* Synchronous: wait for the last pack on 'stream', copy only the packet's
 * bytes to host_buf (Sec. 4: only the compressed data crosses to the host).
 * PV_ERR_CAPACITY with *bytes = needed size when cap is too small;
 * PV_ERR_STATE before the first pack. */
pv_status pv_packet_download(pv_client *client, void *host_buf, uint64_t cap, uint64_t *bytes, void *stream);
/* Synchronous: wait for the last pack on 'stream' and copy the packet into
 * the client's own pinned host staging (allocated, or grown, on first use
 * to the packet's size); *host_ptr receives that borrowed pointer, valid
 * until the next pv_packet_stage or pv_packet_download on the client or its
 * destruction, and *bytes the packet's size. For callers that copy the
 * bytes out themselves: one device-to-host transfer at pinned rate (Sec. 4:
 * only the packet crosses to the host). PV_ERR_STATE before the first pack,
 * PV_ERR_OOM when the staging cannot be allocated. */
pv_status pv_packet_stage(pv_client *client, const void **host_ptr, uint64_t *bytes, void *stream);
/* Client reference export / import (host buffers [P][3][64] and
 * [P][2][256] uint16, plus the sequence counter); synchronous. Lets a
 * server evict a client's state from HBM and bring it back later. */
pv_status pv_client_read_state(pv_client *client, void *ref_irr_host, void *ref_vis_host, uint32_t *seq);
pv_status pv_client_set_state(pv_client *client, const void *ref_irr_host, const void *ref_vis_host, uint32_t seq);
/* pv_pack_delta without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops that may not
 * call hipMalloc). Same computation, kernels and packet layout as
 * pv_pack_delta, on caller-owned device buffers:
 *   cur_irr, cur_vis  the current FP16 tiles, [P][3][10][10] and
 *                     [P][2][18][18] binary16 (the volume map layout);
 *   ref_irr, ref_vis  the client's reference interiors, [P][3][64] and
 *                     [P][2][256] binary16 (all zero = nothing sent yet);
 *                     read, and sent probes written (in place);
 *   packet            receives the packet; packet_cap must hold a full
 *                     resend (the size of a packet with K_irr = K_vis = P),
 *                     else PV_ERR_CAPACITY. The header gives its size.
 * client_id and seq go into the header. Every pointer 16-byte aligned.
 * Changed masks, tile summaries, totals and checksum counters live in one
 * static device array per GPU of 356.5 KiB (held until the process ends;
 * the counters are cleared once when the context takes its address and
 * every call leaves them at zero),
 * which limits n_probes to 65,536 (PV_ERR_ARG beyond). All calls on one GPU
 * share that array: calls that overlap on a GPU (different streams, or
 * threads) race and must be ordered by the caller. Asynchronous on 'stream';
 * calls no allocating routine. Not timed by pv_ctx_set_timing. */
pv_status pv_pack_delta_noalloc(pv_ctx *ctx, const uint16_t *cur_irr, const uint16_t *cur_vis, uint16_t *ref_irr,
                                uint16_t *ref_vis, int n_probes, float tau_irr, float tau_vis, uint32_t client_id,
                                uint32_t seq, uint8_t *packet, uint64_t packet_cap, void *stream);
/* Changed-probe masks of the last pack (device, [P] uint8 each). */
pv_status pv_get_masks(pv_client *client, void **mask_irr_dev, void **mask_vis_dev);

/* Activity of the last update, [P] uint8 (1 = active), device memory owned
 * by the volume; PV_ERR_STATE without PV_CLASSIFY. */
pv_status pv_get_active(pv_volume *vol, const void **active_dev);
/*
 * Server-side client-view culling (Sec. 3.4: the probes that may shade
 * points visible from the client, estimated by a spherical view from its
 * position): n_rays spherical-Fibonacci directions (no rotation) are traced
 * from eye against the volume's scene; every probe at a corner of the grid
 * cell (clamped to the grid) holding a hit point joins the client's view.
 * From then on pv_pack_delta sends only probes in the view (and active,
 * with PV_CLASSIFY); probes outside keep their reference. Asynchronous on
 * 'stream'. n_rays in [1, 2^22]; eye finite.
 */
pv_status pv_client_set_view(pv_client *client, const float eye[3], int n_rays, void *stream);
/* Back to no view culling. */
pv_status pv_client_clear_view(pv_client *client);
/* The client's view mask [P] uint8, or NULL when no view is set. */
pv_status pv_client_get_view(pv_client *client, const void **view_dev);

/* Wait for the stream (NULL: the whole device); report asynchronous device
 * errors. */
pv_status pv_sync(void *stream);

/*
 * Client side (Sec. 3.4: the client keeps its textures, applies index-based
 * probe updates and rebuilds the guard bands the packets leave out). A
 * receiver holds FP16 tiles in the layout of pv_volume_desc (irradiance
 * [P][3][10][10], visibility [P][2][18][18], guard bands included), all-zero
 * bits at creation -- the state of a new pv_client's reference.
 */
typedef struct pv_receiver pv_receiver;
pv_status pv_receiver_create(pv_ctx *ctx, int n_probes, pv_receiver **out);
pv_status pv_receiver_destroy(pv_receiver *rcv);
/*
 * Apply one packet (host memory, the pv_pack_delta layout) asynchronously
 * on 'stream': copied through pinned staging, the index decoded, the
 * payload checksum recomputed, and -- only when the index is valid (every
 * probe in range, strictly increasing) and the checksum matches -- each
 * sent probe's byte planes XORed into its interior texels, written with
 * their guard copies. A packet that fails those checks leaves the tiles
 * unchanged. Header errors are returned at once: PV_ERR_ARG (magic, probe
 * count, size), PV_ERR_UNSUPPORTED (version). Consecutive applies are
 * ordered on the device whatever streams they use.
 */
pv_status pv_receiver_apply(pv_receiver *rcv, const void *packet, uint64_t bytes, void *stream);
/* Waits for the last apply: *result 0 = applied, -2 = checksum mismatch,
 * -4 = invalid index (both: tiles unchanged); *seq (may be NULL) = sequence
 * number of the last packet known to be applied. PV_ERR_STATE before the
 * first apply. */
pv_status pv_receiver_status(pv_receiver *rcv, int *result, uint32_t *seq);
/* Borrowed device pointers to the tiles (uint16 binary16 bit patterns). */
pv_status pv_receiver_get_maps(pv_receiver *rcv, void **irr_dev, void **vis_dev);
/* Copy the tiles to host memory; synchronous. */
pv_status pv_receiver_read_maps(pv_receiver *rcv, void *irr_host, void *vis_host);

/*
 * Entropy stage (lossless; the paper's own stage is HEVC, not built here):
 * the client's last packet coded on the device with a canonical Huffman
 * code per byte stream -- stream 0 the index section (2 (K_irr + K_vis)
 * bytes, no padding), 1..6 the irradiance planes, 7..10 the visibility
 * planes. Per stream: code lengths by Huffman's algorithm over the byte
 * values that occur (the two lightest nodes merged first, leaves before
 * internal nodes on equal weight, leaves ordered by (count, value)), limited
 * to 12 bits by halving every count (rounded up) and rebuilding; canonical
 * codes in (length, value) order; the stream cut into chunks of 1,024 bytes,
 * each coded most significant bit first and padded to 32 bits.
 * Container (little endian): u32 0x43485650 ("PVHC"), u32 version 1, the
 * 32-byte packet header, then per stream 128 bytes of code lengths (value
 * 2i in the low nibble of byte i), u32 n_chunks, u32 bits[n_chunks], and
 * the chunks' bytes.
 * pv_entropy_encode: after pv_pack_delta, on 'stream'; returns once the
 *   histograms are on the host (it waits for the stream up to that point;
 *   the code tables are built on the host) with the coding kernels queued.
 * pv_entropy_download: synchronous; PV_ERR_CAPACITY (with *bytes set) when
 *   cap is too small; PV_ERR_STATE before the first encode.
 * pv_receiver_apply_compressed: decodes a container on the device and
 *   applies the packet as pv_receiver_apply does (same checks and status);
 *   container structure errors: PV_ERR_ARG at once.
 */
pv_status pv_entropy_encode(pv_client *client, void *stream);
pv_status pv_entropy_download(pv_client *client, void *host_buf, uint64_t cap, uint64_t *bytes, void *stream);
pv_status pv_receiver_apply_compressed(pv_receiver *rcv, const void *container, uint64_t bytes, void *stream);

/*
 * Codec surfaces (Sec. 3.3): a volume's textures as the planes a lossless
 * video encoder takes, and back. Probe p occupies atlas tile
 * (p % tiles_per_row, p / tiles_per_row); guard bands are left out; tiles
 * past the last probe are zero. rows = ceil(n_probes / tiles_per_row).
 *   irradiance: three planes (Y = R, U = G, V = B) of uint16, each
 *     [8 rows][8 tiles_per_row]; sample = code << 6 with the 10-bit code
 *     rint(value * k) clamped to [0, 1023], k the FP32 value nearest
 *     1023 / irr_scale, the product in FP32 (ties to even);
 *   visibility: three planes (Y, U, V) of uint8, each
 *     [16 rows][ceil(64 tiles_per_row / 3)]: the bytes of a texel row
 *     (per texel mean lo, mean hi, mean^2 lo, mean^2 hi) dealt in order to
 *     Y, U, V of consecutive samples, so three texels fill four samples;
 *     missing bytes zero.
 * pv_yuv_dims: dims = {irradiance width, height, visibility width, height}.
 * pv_encode_yuv: from an FP16 volume's current maps (PV_ERR_UNSUPPORTED for
 *   FP32 maps); planes are caller-owned device buffers of 3 x w x h samples
 *   each, plane after plane; asynchronous on 'stream'.
 * pv_decode_yuv: planes back to A2RGB10 codes [n_probes][64] (R | G << 10 |
 *   B << 20, alpha 0; texel t = row * 8 + column) and visibility bit
 *   patterns [n_probes][2][256]; caller-owned device buffers; asynchronous.
 * Both: n_probes and tiles_per_row in [1, 65536], else PV_ERR_ARG.
 */
pv_status pv_yuv_dims(int n_probes, int tiles_per_row, int64_t dims[4]);
pv_status pv_encode_yuv(pv_volume *vol, float irr_scale, int tiles_per_row, uint16_t *irr_planes_dev,
                        uint8_t *vis_planes_dev, void *stream);
pv_status pv_decode_yuv(pv_ctx *ctx, int n_probes, int tiles_per_row, const uint16_t *irr_planes_dev,
                        const uint8_t *vis_planes_dev, uint32_t *irr_codes_dev, uint16_t *vis_dev, void *stream);

/*
 * Launch shape of the trace kernel (a tuning choice; every shape computes
 * identical results): probes per wavefront packet as a brick
 * brick[0] x brick[1] x brick[2] = 64 of one ray direction (this also fixes
 * the order in which rays are dealt out), the grid and schedule: one
 * wavefront per packet (persistent 0); a persistent grid whose lanes each take
 * a new ray from per-XCD work queues as soon as theirs ends, with node visits
 * and leaf triangle tests scheduled as separate wave steps (persistent 1); one
 * wavefront per packet with those separate steps and each lane's shadow rays
 * started as soon as its primary ray ends (persistent 2), the number
 * of top BVH nodes staged in LDS (0, 21 or 85: one, three or four levels),
 * threads per block (128 or 256), and whether shadow rays are traced inside
 * the primary kernel (0) or appended to a compacted queue and traced by a
 * dense second kernel, then applied by a shade kernel (1; the primary kernel
 * then runs one wavefront per packet whatever 'persistent' says). Defaults:
 * 4x4x4, 2, 21, 256, 0.
 */
typedef struct {
    int brick[3];
    int persistent;
    int top_nodes;
    int block_threads;
    int split_shadows;
} pv_trace_config;

/* Numeric path of the blend (Sec. 3.2's weighted means as one matrix
 * product per texture: weights x ray records). The weights are shared by
 * every probe of a volume-frame; except for PV_BLEND_TILES they are
 * evaluated once per frame into a table. PV_BLEND_BF16X3: BF16 matrix cores,
 * weights and records split into high and low BF16 halves, three products
 * per term with FP32 accumulation (about 2^-16 relative per term).
 * PV_BLEND_F32: FP32 matrix cores. PV_BLEND_TILES: FP32 matrix cores with
 * the weights evaluated again by every 8-probe tile (no table).
 * PV_BLEND_VALU: the table on FP32 vector FMAs. PV_BLEND_BF16X6: BF16
 * matrix cores, weights and records split into three BF16 parts (high,
 * middle, low), the six products down to 2^-18 of the term with FP32
 * accumulation (about 2^-25 relative per term). PV_BLEND_AUTO (the default
 * of a new volume) resolves to PV_BLEND_TILES below 2,048 probes and to
 * PV_BLEND_BF16X6 from there. Every path but PV_BLEND_BF16X3 meets the FP32
 * blend's 1e-5 bound. Takes effect from the next update; the mode is
 * reported as resolved. */
enum { PV_BLEND_AUTO = 0, PV_BLEND_BF16X3 = 1, PV_BLEND_F32 = 2, PV_BLEND_TILES = 3, PV_BLEND_VALU = 4,
       PV_BLEND_BF16X6 = 5 };
pv_status pv_volume_set_blend_mode(pv_volume *vol, int mode);
pv_status pv_volume_get_blend_mode(pv_volume *vol, int *mode);
pv_status pv_volume_set_trace_config(pv_volume *vol, const pv_trace_config *cfg);
pv_status pv_volume_get_trace_config(pv_volume *vol, pv_trace_config *cfg);

/* Kernel stages that can be timed with HIP events. */
typedef enum {
    PV_STAGE_RAYDIRS = 0,
    PV_STAGE_TRACE = 1,
    PV_STAGE_BLEND = 2,
    PV_STAGE_PACK_MASK = 3,
    PV_STAGE_PACK_SCAN = 4,
    PV_STAGE_PACK_COMPACT = 5,
    PV_STAGE_BATCHED = 6,
    PV_STAGE_SHADOW = 7,
    PV_STAGE_SHADE = 8,
    PV_STAGE_PACK_FINISH = 9, /* the packet checksum (above 4,096 probes) */
    PV_STAGE_BOUNCE = 10,
    PV_STAGE_UNPACK = 11,
    PV_STAGE_CODEC = 12,
    PV_STAGE_SELECT = 13,
    PV_STAGE_ENTROPY = 14,
    PV_STAGE_COUNT = 15
} pv_stage;

/* When enabled, every kernel launch of the context is bracketed by a pair
 * of HIP events recorded on the launch stream. */
pv_status pv_ctx_set_timing(pv_ctx *ctx, int enable);
/* Synchronous: total milliseconds and launch counts per stage since the
 * previous call (which are then reset). Arrays of PV_STAGE_COUNT. */
pv_status pv_ctx_stage_times(pv_ctx *ctx, double *ms, uint64_t *launches);

/* Instrumented trace of one frame (for measurement): the same work as
 * pv_update_probes with per-ray counts of node and triangle tests,
 * summed into counts[0] (node visits, four child boxes each), counts[1] (triangle
 * tests), counts[2] (shadow rays). Synchronous. */
pv_status pv_trace_counts(pv_volume *vol, const pv_frame *frame, uint64_t counts[3]);

/* Attainable ceilings of the context's device (for measurement: what a plain
 * kernel reaches, beside the data-sheet peaks):
 *   PV_CEIL_COPY      float4 copy of 1 GiB; rate in bytes/s, read + write
 *   PV_CEIL_FMA_F32   eight independent FP32 FMA chains per thread, no
 *                     packed FP32; rate in FLOP/s (FMA = 2)
 *   PV_CEIL_MFMA_F32  four independent 16x16x4 FP32 MFMA chains per
 *                     wavefront; rate in FLOP/s
 * 32 wavefronts per compute unit; one untimed warm-up, then the fastest of
 * 'reps' launches (HIP events on the context's stream). Allocates and frees
 * its own buffers (2 GiB for the copy). Synchronous. PV_ERR_ARG for an
 * unknown kind or reps < 1, PV_ERR_OOM when the buffers cannot be allocated.
 * Measurement support only; no part of the paper's method. */
enum { PV_CEIL_COPY = 0, PV_CEIL_FMA_F32 = 1, PV_CEIL_MFMA_F32 = 2 };
pv_status pv_measure_ceiling(pv_ctx *ctx, int kind, int reps, double *rate);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif

#endif /* PROBESTREAM_H */
