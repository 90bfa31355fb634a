// C ABI of the probe-volume library: handles, validation, device memory,
// launch sequencing. Kernels live in trace.hip, blend.hip, batched.hip,
// bounce.hip, select.hip, pack.hip, entropy.hip, receive.hip and yuv.hip,
// the BVH builder in bvh.cpp.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "blend_layout.h"
#include "packet_format.h"

using namespace pv;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static pv_status fail(pv_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return fail(PV_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" const char *pv_last_error(void) { return g_err.c_str(); }
extern "C" const char *pv_version(void) { return "probestream 1.0 gfx950"; }

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
// Device and pinned host buffers of one batched launch. Launches in flight
// on different streams use different slots; a slot is reused only after
// its previous launch has finished (its event).
struct BatchSlot {
    BatchVolume *batch_dev = nullptr;
    FrameParams *frames_dev = nullptr;
    int cap = 0;
    void *stage_host = nullptr;
    hipEvent_t done = nullptr;
};

struct pv_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    static constexpr int kRing = 8;
    BatchSlot slots[kRing];
    int slot_next = 0;
    unsigned long long *counts_dev = nullptr;
    // optional per-stage event timing
    struct Timed {
        int stage;
        hipEvent_t a, b;
    };
    bool timing = false;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
};

// Runs 'launch' and, when timing is on, brackets it with events on 's'.
template <class F>
static hipError_t timed(pv_ctx *c, int stage, hipStream_t s, F launch) {
    if (!c->timing) return launch();
    hipEvent_t ev[2];
    for (int i = 0; i < 2; ++i) {
        if (!c->pool.empty()) {
            ev[i] = c->pool.back();
            c->pool.pop_back();
        } else {
            hipError_t e = hipEventCreate(&ev[i]);
            if (e != hipSuccess) return e;
        }
    }
    hipError_t e = hipEventRecord(ev[0], s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(ev[1], s);
    c->pending.push_back({stage, ev[0], ev[1]});
    return e;
}

struct pv_scene {
    pv_ctx *ctx = nullptr;
    int n_static = 0, n_dyn = 0;
    DeviceBvh stat;
    float4 *mats = nullptr;
    float eps = 1e-4f;
    std::vector<pv_point_light> lights;
    // dynamic triangles: ring of device BVH slots fed from pinned staging
    static constexpr int kRing = 4;
    GpuNode4 *dyn_nodes[kRing] = {};
    GpuTri *dyn_tris[kRing] = {};
    void *dyn_stage[kRing] = {};
    hipEvent_t dyn_use[kRing] = {};
    bool dyn_used[kRing] = {};
    int dyn_nodes_n[kRing] = {};
    int dyn_tris_n[kRing] = {};
    int dyn_slot = 0;
    size_t dyn_node_cap = 0, dyn_tri_cap = 0;
};

struct pv_volume {
    pv_ctx *ctx = nullptr;
    pv_volume_desc desc;
    int P = 0, n = 0;
    size_t elem = 4;
    void *irr = nullptr, *vis = nullptr;
    float4 *rays = nullptr, *dirs = nullptr;
    int32_t *hits = nullptr;
    int2 *hitrec = nullptr;  // hit records (PV_MULTI_BOUNCE or PV_CLASSIFY)
    uint8_t *active = nullptr;  // [P] probe activity of the last update (PV_CLASSIFY)
    int *queue = nullptr;  // work counters (queue_counter: 0..7 per XCD, 8 shadow-queue length)
    int64_t frame = 0;
    pv_scene *scene = nullptr;
    TraceConfig tc;
    SplitBuffers split;    // allocated on first use of the split-shadow trace
    int blend_mode = kBlendF32;     // resolved BlendMode
};

struct pv_client {
    pv_volume *vol = nullptr;
    uint32_t id = 0, seq = 0;
    uint16_t *ref_irr = nullptr, *ref_vis = nullptr;
    uint8_t *mask_irr = nullptr, *mask_vis = nullptr;
    int4 *tiles = nullptr;         // per-tile summaries of the last mask pass
    uint32_t *totals = nullptr;    // changed-probe totals of the last scan
    int2 *tiles2 = nullptr;        // per-tile second-last changed probes
    unsigned long long *cks = nullptr;  // checksum counters (zero between packs)
    uint32_t *tsum = nullptr;      // per-tile own summaries
    uint8_t *packet = nullptr;
    uint64_t packet_cap = 0;
    uint32_t *hdr_host = nullptr;  // pinned, 32 bytes
    uint8_t *stage_host = nullptr; // pinned packet staging (grown on demand)
    uint64_t stage_cap = 0;
    uint8_t *view = nullptr;       // [P] visible set of the last pv_client_set_view
    bool view_on = false;
    // entropy stage (allocated on first use)
    EntBuffers ent = {};
    uint64_t ent_cap = 0;
    unsigned long long *ent_total_host = nullptr;  // pinned
    uint8_t *ent_tables_host = nullptr;            // pinned: histograms, then lengths and codes
};

// NULL is HIP's default stream, as in the HIP API itself.
static hipStream_t pick(pv_ctx *, void *s) { return (hipStream_t)s; }

static uint64_t irr_bytes(int P, size_t elem) { return (uint64_t)P * 3 * 100 * elem; }
static uint64_t vis_bytes(int P, size_t elem) { return (uint64_t)P * 2 * 324 * elem; }
static uint64_t packet_capacity(int P) { return packet_bytes((uint64_t)P, (uint64_t)P); }

template <typename T>
static pv_status dev_alloc(T **p, size_t bytes, const char *what) {
    *p = nullptr;
    if (bytes == 0) return PV_OK;
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(PV_ERR_OOM, std::string("device allocation of ") + what + " (" + std::to_string(bytes) +
                                    " bytes) failed: " + hipGetErrorString(e));
    }
    return PV_OK;
}

#define PV_TRY(expr)                      \
    do {                                  \
        pv_status s_ = (expr);            \
        if (s_ != PV_OK) return s_;       \
    } while (0)

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" pv_status pv_ctx_create(int hip_device, pv_ctx **out) {
    if (!out) return fail(PV_ERR_ARG, "out is NULL");
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (hip_device < 0 || hip_device >= count)
        return fail(PV_ERR_ARG, "hip_device " + std::to_string(hip_device) + " out of range");
    HIP_TRY(hipSetDevice(hip_device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PV_ERR_UNSUPPORTED, std::string("built for gfx950, device is ") + prop.gcnArchName);
    // the no-allocation pack's scratch array: its address on this device
    HIP_TRY(noalloc_scratch_init(hip_device));
    pv_ctx *c = new pv_ctx();
    c->device = hip_device;
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return fail(PV_ERR_DEVICE, std::string("stream: ") + hipGetErrorString(e));
    }
    for (int i = 0; i < pv_ctx::kRing; ++i) HIP_TRY(hipEventCreateWithFlags(&c->slots[i].done, hipEventDisableTiming));
    *out = c;
    return PV_OK;
}

extern "C" pv_status pv_ctx_destroy(pv_ctx *c) {
    if (!c) return PV_OK;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    hipDeviceSynchronize();
    hipFree(c->counts_dev);
    for (int i = 0; i < pv_ctx::kRing; ++i) {
        BatchSlot &b = c->slots[i];
        hipFree(b.batch_dev);
        hipFree(b.frames_dev);
        if (b.stage_host) hipHostFree(b.stage_host);
        if (b.done) hipEventDestroy(b.done);
    }
    for (auto &t : c->pending) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    for (auto e : c->pool) hipEventDestroy(e);
    hipStreamDestroy(c->stream);
    delete c;
    return PV_OK;
}

extern "C" pv_status pv_ctx_set_timing(pv_ctx *c, int enable) {
    if (!c) return fail(PV_ERR_ARG, "ctx is NULL");
    c->timing = enable != 0;
    return PV_OK;
}

extern "C" pv_status pv_ctx_stage_times(pv_ctx *c, double *ms, uint64_t *launches) {
    if (!c || !ms || !launches) return fail(PV_ERR_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(c->device));
    for (int i = 0; i < PV_STAGE_COUNT; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    for (auto &t : c->pending) {
        HIP_TRY(hipEventSynchronize(t.b));
        float m = 0.f;
        HIP_TRY(hipEventElapsedTime(&m, t.a, t.b));
        ms[t.stage] += m;
        launches[t.stage] += 1;
        c->pool.push_back(t.a);
        c->pool.push_back(t.b);
    }
    c->pending.clear();
    return PV_OK;
}

// ---------------------------------------------------------------------------
// scene
// ---------------------------------------------------------------------------
static bool finite_all(const float *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

static pv_status upload_bvh(const HostBvh4 &hb, DeviceBvh &db, hipStream_t s) {
    db.n_nodes = (int)hb.nodes.size();
    db.n_tris = (int)hb.tris.size();
    PV_TRY(dev_alloc(&db.nodes, hb.nodes.size() * sizeof(GpuNode4), "BVH nodes"));
    PV_TRY(dev_alloc(&db.tris, hb.tris.size() * sizeof(GpuTri), "BVH triangles"));
    if (db.n_nodes) HIP_TRY(hipMemcpyAsync(db.nodes, hb.nodes.data(), hb.nodes.size() * sizeof(GpuNode4), hipMemcpyHostToDevice, s));
    if (db.n_tris) HIP_TRY(hipMemcpyAsync(db.tris, hb.tris.data(), hb.tris.size() * sizeof(GpuTri), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PV_OK;
}

static pv_status validate_lights(int n, const pv_point_light *l) {
    if (n < 0 || n > PV_MAX_LIGHTS) return fail(PV_ERR_ARG, "n_lights must be in [0, 8]");
    if (n > 0 && !l) return fail(PV_ERR_ARG, "lights is NULL");
    for (int i = 0; i < n; ++i)
        if (!finite_all(l[i].pos, 3) || !finite_all(l[i].intensity, 3))
            return fail(PV_ERR_ARG, "light " + std::to_string(i) + " is not finite");
    return PV_OK;
}

static void destroy_scene(pv_scene *s) {
    if (!s) return;
    hipFree(s->stat.nodes);
    hipFree(s->stat.tris);
    hipFree(s->mats);
    for (int i = 0; i < pv_scene::kRing; ++i) {
        hipFree(s->dyn_nodes[i]);
        hipFree(s->dyn_tris[i]);
        if (s->dyn_stage[i]) hipHostFree(s->dyn_stage[i]);
        if (s->dyn_use[i]) hipEventDestroy(s->dyn_use[i]);
    }
    delete s;
}

static pv_status set_dynamic_impl(pv_scene *s, const float *pos, hipStream_t st);

extern "C" pv_status pv_scene_create(pv_ctx *ctx, const pv_scene_desc *d, pv_scene **out) {
    if (!ctx || !d || !out) return fail(PV_ERR_ARG, "NULL argument");
    if (d->n_triangles < 0 || d->n_vertices < 0) return fail(PV_ERR_ARG, "negative counts");
    if (d->n_dynamic_triangles < 0 || d->n_dynamic_triangles > d->n_triangles)
        return fail(PV_ERR_ARG, "n_dynamic_triangles must be in [0, n_triangles]");
    if (d->n_triangles > 0 && (!d->positions || !d->indices || !d->albedo))
        return fail(PV_ERR_ARG, "positions, indices and albedo are required");
    if (d->n_vertices > 0 && !finite_all(d->positions, 3ull * d->n_vertices))
        return fail(PV_ERR_ARG, "vertex positions must be finite");
    PV_TRY(validate_lights(d->n_lights, d->lights));
    const int T = d->n_triangles;
    for (int64_t i = 0; i < 3ll * T; ++i)
        if (d->indices[i] >= (uint32_t)d->n_vertices)
            return fail(PV_ERR_ARG, "triangle index out of range at " + std::to_string(i));
    if (T > 0 && !finite_all(d->albedo, 3ull * T)) return fail(PV_ERR_ARG, "albedo must be finite");
    if (T > 0 && d->emission && !finite_all(d->emission, 3ull * T)) return fail(PV_ERR_ARG, "emission must be finite");
    HIP_TRY(hipSetDevice(ctx->device));
    pv_scene *s = new pv_scene();
    s->ctx = ctx;
    s->n_dyn = d->n_dynamic_triangles;
    s->n_static = T - s->n_dyn;
    s->lights.assign(d->lights, d->lights + d->n_lights);
    std::vector<float> tri9((size_t)T * 9);
    for (int t = 0; t < T; ++t)
        for (int v = 0; v < 3; ++v)
            for (int k = 0; k < 3; ++k) tri9[9 * (size_t)t + 3 * v + k] = d->positions[3 * (size_t)d->indices[3 * (size_t)t + v] + k];
    // shadow offset from the static bounding box (all triangles if none is static)
    const int ns = s->n_static > 0 ? s->n_static : T;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int t = 0; t < ns; ++t)
        for (int v = 0; v < 3; ++v)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], (double)tri9[9 * (size_t)t + 3 * v + k]);
                hi[k] = std::max(hi[k], (double)tri9[9 * (size_t)t + 3 * v + k]);
            }
    double diag = ns > 0 ? std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                     (hi[2] - lo[2]) * (hi[2] - lo[2]))
                         : 1.0;
    s->eps = (float)(1e-4 * diag);
    HostBvh4 hb;
    std::string err;
    if (!build_bvh4(tri9.data(), s->n_static, 0, hb, err)) {
        destroy_scene(s);
        return fail(PV_ERR_ARG, err);
    }
    pv_status st = upload_bvh(hb, s->stat, ctx->stream);
    if (st != PV_OK) {
        destroy_scene(s);
        return st;
    }
    std::vector<float4> mats((size_t)std::max(T, 1) * 2);
    for (int t = 0; t < T; ++t) {
        mats[2 * t] = make_float4(d->albedo[3 * t], d->albedo[3 * t + 1], d->albedo[3 * t + 2], 0.f);
        mats[2 * t + 1] = d->emission ? make_float4(d->emission[3 * t], d->emission[3 * t + 1], d->emission[3 * t + 2], 0.f)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    st = dev_alloc(&s->mats, mats.size() * sizeof(float4), "materials");
    if (st != PV_OK) {
        destroy_scene(s);
        return st;
    }
    hipError_t e = hipMemcpy(s->mats, mats.data(), mats.size() * sizeof(float4), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        destroy_scene(s);
        return fail(PV_ERR_DEVICE, std::string("materials upload: ") + hipGetErrorString(e));
    }
    if (s->n_dyn > 0) {
        // a tree over m leaf slots has fewer than m inner nodes
        s->dyn_node_cap = bvh_max_refs(s->n_dyn);
        s->dyn_tri_cap = bvh_max_refs(s->n_dyn);
        for (int i = 0; i < pv_scene::kRing; ++i) {
            st = dev_alloc(&s->dyn_nodes[i], s->dyn_node_cap * sizeof(GpuNode4), "dynamic BVH nodes");
            if (st == PV_OK) st = dev_alloc(&s->dyn_tris[i], s->dyn_tri_cap * sizeof(GpuTri), "dynamic triangles");
            if (st == PV_OK && hipHostMalloc(&s->dyn_stage[i], s->dyn_node_cap * sizeof(GpuNode4) + s->dyn_tri_cap * sizeof(GpuTri)) != hipSuccess)
                st = fail(PV_ERR_OOM, "pinned staging for dynamic triangles");
            if (st == PV_OK && hipEventCreateWithFlags(&s->dyn_use[i], hipEventDisableTiming) != hipSuccess)
                st = fail(PV_ERR_DEVICE, "event");
            if (st != PV_OK) {
                destroy_scene(s);
                return st;
            }
        }
        s->dyn_slot = pv_scene::kRing - 1;
        st = set_dynamic_impl(s, tri9.data() + 9 * (size_t)s->n_static, ctx->stream);
        if (st == PV_OK) st = hipStreamSynchronize(ctx->stream) == hipSuccess ? PV_OK : fail(PV_ERR_DEVICE, "sync");
        if (st != PV_OK) {
            destroy_scene(s);
            return st;
        }
    }
    *out = s;
    return PV_OK;
}

static pv_status set_dynamic_impl(pv_scene *s, const float *pos, hipStream_t st) {
    if (!finite_all(pos, 9ull * s->n_dyn)) return fail(PV_ERR_ARG, "dynamic positions must be finite");
    HostBvh4 hb;
    std::string err;
    if (!build_bvh4(pos, s->n_dyn, s->n_static, hb, err)) return fail(PV_ERR_ARG, err);
    if (hb.nodes.size() > s->dyn_node_cap || hb.tris.size() > s->dyn_tri_cap)
        return fail(PV_ERR_STATE, "dynamic BVH larger than its slot");
    const int k = (s->dyn_slot + 1) % pv_scene::kRing;
    // the slot may still be read by earlier work: wait for its last use
    if (s->dyn_used[k]) HIP_TRY(hipEventSynchronize(s->dyn_use[k]));
    char *stage = (char *)s->dyn_stage[k];
    const size_t nb = hb.nodes.size() * sizeof(GpuNode4), tb = hb.tris.size() * sizeof(GpuTri);
    std::memcpy(stage, hb.nodes.data(), nb);
    std::memcpy(stage + s->dyn_node_cap * sizeof(GpuNode4), hb.tris.data(), tb);
    HIP_TRY(hipMemcpyAsync(s->dyn_nodes[k], stage, nb, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->dyn_tris[k], stage + s->dyn_node_cap * sizeof(GpuNode4), tb, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(s->dyn_use[k], st));
    s->dyn_used[k] = true;
    s->dyn_nodes_n[k] = (int)hb.nodes.size();
    s->dyn_tris_n[k] = (int)hb.tris.size();
    s->dyn_slot = k;
    return PV_OK;
}

extern "C" pv_status pv_scene_set_dynamic(pv_scene *s, const float *positions, void *stream) {
    if (!s || !positions) return fail(PV_ERR_ARG, "NULL argument");
    if (s->n_dyn == 0) return fail(PV_ERR_STATE, "scene has no dynamic triangles");
    HIP_TRY(hipSetDevice(s->ctx->device));
    return set_dynamic_impl(s, positions, pick(s->ctx, stream));
}

extern "C" pv_status pv_scene_destroy(pv_scene *s) {
    if (!s) return PV_OK;
    hipSetDevice(s->ctx->device);
    hipDeviceSynchronize();
    destroy_scene(s);
    return PV_OK;
}

static SceneView scene_view(pv_scene *s) {
    SceneView v;
    v.stat = s->stat;
    v.dyn = DeviceBvh();
    if (s->n_dyn > 0) {
        v.dyn.nodes = s->dyn_nodes[s->dyn_slot];
        v.dyn.tris = s->dyn_tris[s->dyn_slot];
        v.dyn.n_nodes = s->dyn_nodes_n[s->dyn_slot];
        v.dyn.n_tris = s->dyn_tris_n[s->dyn_slot];
    }
    v.mats = s->mats;
    v.eps = s->eps;
    return v;
}

extern "C" pv_status pv_scene_read_bvh(pv_scene *s, int dynamic, void *nodes_host, uint64_t nodes_cap,
                                       void *tris_host, uint64_t tris_cap, int64_t counts[2], float *eps) {
    if (!s || !counts) return fail(PV_ERR_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(s->ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    const SceneView v = scene_view(s);
    const DeviceBvh &b = dynamic ? v.dyn : v.stat;
    counts[0] = b.n_nodes;
    counts[1] = b.n_tris;
    if (eps) *eps = v.eps;
    const uint64_t nb = (uint64_t)b.n_nodes * sizeof(GpuNode4), tb = (uint64_t)b.n_tris * sizeof(GpuTri);
    if (!nodes_host || !tris_host) return PV_OK;
    if (nodes_cap < nb || tris_cap < tb) return fail(PV_ERR_CAPACITY, "buffers smaller than the BVH");
    if (nb) HIP_TRY(hipMemcpy(nodes_host, b.nodes, nb, hipMemcpyDeviceToHost));
    if (tb) HIP_TRY(hipMemcpy(tris_host, b.tris, tb, hipMemcpyDeviceToHost));
    return PV_OK;
}

static pv_status note_scene_use(pv_scene *s, hipStream_t st) {
    if (s->n_dyn > 0) HIP_TRY(hipEventRecord(s->dyn_use[s->dyn_slot], st));
    return PV_OK;
}

// ---------------------------------------------------------------------------
// volume
// ---------------------------------------------------------------------------
static pv_status validate_desc(const pv_volume_desc *d) {
    if (!d) return fail(PV_ERR_ARG, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(PV_ERR_ARG, "grid dimensions must be >= 1");
    const long long P = (long long)d->nx * d->ny * d->nz;
    if (P > PV_MAX_PROBES) return fail(PV_ERR_ARG, "at most 65536 probes per volume (2-byte probe index)");
    if (d->rays_per_probe < 1 || d->rays_per_probe > PV_MAX_RAYS) return fail(PV_ERR_ARG, "rays_per_probe must be in [1, 4096]");
    if (!(d->hysteresis >= 0.f && d->hysteresis < 1.f)) return fail(PV_ERR_ARG, "hysteresis must be in [0, 1)");
    if (!(d->max_distance > 0.f) || !std::isfinite(d->max_distance)) return fail(PV_ERR_ARG, "max_distance must be finite and > 0");
    if (d->vis_sharpness < 1 || d->vis_sharpness > 128) return fail(PV_ERR_ARG, "vis_sharpness must be in [1, 128]");
    if (d->format != PV_MAP_FP32 && d->format != PV_MAP_FP16) return fail(PV_ERR_ARG, "unknown map format");
    if (!finite_all(d->origin, 3) || !finite_all(d->spacing, 3) || !finite_all(d->sky, 3))
        return fail(PV_ERR_ARG, "origin, spacing and sky must be finite");
    if (d->irr_res != 8 || d->vis_res != 16)
        return fail(PV_ERR_UNSUPPORTED, "supported: irr_res = 8 and vis_res = 16");
    if (!(d->spacing[0] > 0.f && d->spacing[1] > 0.f && d->spacing[2] > 0.f))
        return fail(PV_ERR_ARG, "spacing must be > 0 on every axis");
    if (d->flags & ~(PV_FIRST_FRAME_NO_HISTORY | PV_KEEP_HITS | PV_MULTI_BOUNCE | PV_CLASSIFY))
        return fail(PV_ERR_ARG, "unknown flags");
    return PV_OK;
}

static uint64_t volume_bytes(const pv_volume_desc *d) {
    const int P = d->nx * d->ny * d->nz, n = d->rays_per_probe;
    const size_t elem = d->format == PV_MAP_FP16 ? 2 : 4;
    uint64_t b = irr_bytes(P, elem) + vis_bytes(P, elem) + 512 + (uint64_t)P * n * 16 + dirs_span(n) +
                 wtab_bytes(n) + (uint64_t)kQueueInts * 4;
    if (d->flags & PV_KEEP_HITS) b += (uint64_t)P * n * 4;
    if (d->flags & (PV_MULTI_BOUNCE | PV_CLASSIFY)) b += (uint64_t)P * n * 8;
    if (d->flags & PV_CLASSIFY) b += (uint64_t)P;
    return b;
}

extern "C" pv_status pv_volume_footprint(const pv_volume_desc *d, uint64_t *bytes) {
    PV_TRY(validate_desc(d));
    if (!bytes) return fail(PV_ERR_ARG, "bytes is NULL");
    *bytes = volume_bytes(d);
    return PV_OK;
}

static void free_volume(pv_volume *v) {
    hipFree(v->irr);
    hipFree(v->vis);
    hipFree(v->rays);
    hipFree(v->dirs);
    hipFree(v->hits);
    hipFree(v->hitrec);
    hipFree(v->active);
    hipFree(v->queue);
    hipFree(v->split.hitrec);
    hipFree(v->split.occ);
    hipFree(v->split.queue);
    delete v;
}

extern "C" pv_status pv_create_volume(pv_ctx *ctx, const pv_volume_desc *d, pv_volume **out) {
    if (!ctx || !out) return fail(PV_ERR_ARG, "NULL argument");
    PV_TRY(validate_desc(d));
    HIP_TRY(hipSetDevice(ctx->device));
    pv_volume *v = new pv_volume();
    v->ctx = ctx;
    v->desc = *d;
    v->P = d->nx * d->ny * d->nz;
    v->n = d->rays_per_probe;
    v->elem = d->format == PV_MAP_FP16 ? 2 : 4;
    v->blend_mode = auto_blend_mode(v->P);
    // 256 bytes of slack: vector loads of a ragged last tile stay in bounds
    pv_status st = dev_alloc(&v->irr, irr_bytes(v->P, v->elem) + 256, "irradiance maps");
    if (st == PV_OK) st = dev_alloc(&v->vis, vis_bytes(v->P, v->elem) + 256, "visibility maps");
    if (st == PV_OK) st = dev_alloc(&v->rays, (size_t)v->P * v->n * 16, "ray buffer");
    // the ray directions, then the blend's weight table
    if (st == PV_OK) st = dev_alloc(&v->dirs, dirs_span(v->n) + wtab_bytes(v->n), "directions and blend weights");
    if (st == PV_OK && (d->flags & PV_KEEP_HITS)) st = dev_alloc(&v->hits, (size_t)v->P * v->n * 4, "hit ids");
    if (st == PV_OK && (d->flags & (PV_MULTI_BOUNCE | PV_CLASSIFY)))
        st = dev_alloc(&v->hitrec, (size_t)v->P * v->n * sizeof(int2), "hit records");
    if (st == PV_OK && (d->flags & PV_CLASSIFY)) {
        st = dev_alloc(&v->active, (size_t)v->P, "probe activity");
        // every probe counts as active until the first update classifies it
        if (st == PV_OK && launch_fill_u8(v->active, (size_t)v->P, 1, ctx->stream) != hipSuccess)
            st = fail(PV_ERR_DEVICE, "fill");
    }
    if (st == PV_OK) st = dev_alloc(&v->queue, kQueueInts * sizeof(int), "work queues");
    if (st == PV_OK && launch_zero(v->irr, irr_bytes(v->P, v->elem), ctx->stream) != hipSuccess) st = fail(PV_ERR_DEVICE, "zero fill");
    if (st == PV_OK && launch_zero(v->vis, vis_bytes(v->P, v->elem), ctx->stream) != hipSuccess) st = fail(PV_ERR_DEVICE, "zero fill");
    if (st == PV_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(PV_ERR_DEVICE, "sync after zero fill");
    if (st != PV_OK) {
        free_volume(v);
        return st;
    }
    *out = v;
    return PV_OK;
}

extern "C" pv_status pv_volume_destroy(pv_volume *v) {
    if (!v) return PV_OK;
    hipSetDevice(v->ctx->device);
    hipDeviceSynchronize();
    free_volume(v);
    return PV_OK;
}

extern "C" pv_status pv_set_scene(pv_volume *v, pv_scene *s) {
    if (!v || !s) return fail(PV_ERR_ARG, "NULL argument");
    if (s->ctx != v->ctx) return fail(PV_ERR_ARG, "scene and volume belong to different contexts");
    v->scene = s;
    return PV_OK;
}

static pv_status frame_params(const pv_frame *f, const pv_scene *s, FrameParams &fp) {
    if (!f) return fail(PV_ERR_ARG, "frame is NULL");
    if (!finite_all(f->rotation, 9)) return fail(PV_ERR_ARG, "rotation must be finite");
    // a proper rotation: orthonormal rows to FP32 rounding
    const float *R = f->rotation;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double dot = (double)R[3 * a] * R[3 * b] + (double)R[3 * a + 1] * R[3 * b + 1] + (double)R[3 * a + 2] * R[3 * b + 2];
            if (std::fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-4) return fail(PV_ERR_ARG, "rotation is not orthonormal");
        }
    std::memcpy(fp.rot, R, sizeof(fp.rot));
    const pv_point_light *L = f->lights;
    int nl = f->n_lights;
    if (nl == 0 && !L && s) {
        L = s->lights.data();
        nl = (int)s->lights.size();
    }
    PV_TRY(validate_lights(nl, L));
    fp.n_lights = nl;
    for (int i = 0; i < nl; ++i)
        for (int k = 0; k < 3; ++k) {
            fp.light_pos[i][k] = L[i].pos[k];
            fp.light_int[i][k] = L[i].intensity[k];
        }
    return PV_OK;
}

static VolumeParams volume_params(const pv_volume *v) {
    VolumeParams p;
    const pv_volume_desc &d = v->desc;
    p.nx = d.nx;
    p.ny = d.ny;
    p.nz = d.nz;
    p.P = v->P;
    p.n = v->n;
    p.ox = d.origin[0];
    p.oy = d.origin[1];
    p.oz = d.origin[2];
    p.sx = d.spacing[0];
    p.sy = d.spacing[1];
    p.sz = d.spacing[2];
    p.max_distance = d.max_distance;
    for (int k = 0; k < 3; ++k) p.sky[k] = d.sky[k];
    p.vis_sharpness = d.vis_sharpness;
    p.blend_mode = v->blend_mode;
    p.hitrec = v->hitrec;
    return p;
}

static float effective_h(const pv_volume *v) {
    return (v->frame == 0 && (v->desc.flags & PV_FIRST_FRAME_NO_HISTORY)) ? 0.f : v->desc.hysteresis;
}

// Split-shadow buffers sized for this frame's lights (grown when needed).
static pv_status ensure_split(pv_volume *v, int n_lights, hipStream_t s) {
    const long long need = (long long)v->P * v->n * std::max(n_lights, 1);
    if (v->split.hitrec && v->split.capacity >= need) return PV_OK;
    HIP_TRY(hipStreamSynchronize(s));
    hipFree(v->split.hitrec);
    hipFree(v->split.occ);
    hipFree(v->split.queue);
    v->split = SplitBuffers();
    PV_TRY(dev_alloc(&v->split.hitrec, (size_t)v->P * v->n * sizeof(int2), "hit records"));
    PV_TRY(dev_alloc(&v->split.occ, (size_t)v->P * v->n * sizeof(uint32_t), "occlusion bits"));
    PV_TRY(dev_alloc(&v->split.queue, (size_t)need * sizeof(ShadowEntry), "shadow queue"));
    v->split.count = queue_counter(v->queue, 8);
    v->split.capacity = need;
    return PV_OK;
}

// Enqueues ray directions + trace (+ shadow + shade passes in split mode).
static pv_status enqueue_trace(pv_volume *v, const FrameParams &fp, const SceneView &sv, unsigned long long *counts,
                               hipStream_t s) {
    pv_ctx *c = v->ctx;
    const VolumeParams vp = volume_params(v);
    const bool split = v->tc.split_shadows != 0;
    if (split) PV_TRY(ensure_split(v, fp.n_lights, s));
    const SplitBuffers sb = split ? v->split : SplitBuffers();
    HIP_TRY(timed(c, PV_STAGE_RAYDIRS, s, [&] { return launch_raydirs(fp, vp, v->dirs, v->queue, s); }));
    HIP_TRY(timed(c, PV_STAGE_TRACE, s,
                  [&] { return launch_trace(vp, sv, fp, v->dirs, v->rays, v->hits, counts, v->tc, v->queue, sb, s); }));
    if (split && fp.n_lights > 0) {
        HIP_TRY(timed(c, PV_STAGE_SHADOW, s, [&] { return launch_shadow(sv, sb, v->tc, counts, s); }));
        HIP_TRY(timed(c, PV_STAGE_SHADE, s, [&] { return launch_shade(vp, sv, fp, v->dirs, v->rays, sb, s); }));
    }
    return PV_OK;
}

static pv_status update_probes(pv_volume *v, const pv_frame *f, void *stream, void *after_trace) {
    if (!v) return fail(PV_ERR_ARG, "volume is NULL");
    if (!v->scene) return fail(PV_ERR_STATE, "no scene set on the volume");
    FrameParams fp;
    PV_TRY(frame_params(f, v->scene, fp));
    HIP_TRY(hipSetDevice(v->ctx->device));
    hipStream_t s = pick(v->ctx, stream);
    const VolumeParams vp = volume_params(v);
    pv_ctx *c = v->ctx;
    const SceneView sv = scene_view(v->scene);
    const int fp16 = v->desc.format == PV_MAP_FP16;
    const float h = effective_h(v);
    PV_TRY(enqueue_trace(v, fp, sv, nullptr, s));
    // the kernels from here on rewrite what a pack of the previous frame
    // reads (the maps, the activity): they wait for the caller's event
    if (after_trace) HIP_TRY(hipStreamWaitEvent(s, (hipEvent_t)after_trace, 0));
    if (v->active)
        HIP_TRY(timed(c, PV_STAGE_SELECT, s, [&] { return launch_classify(vp, sv, v->dirs, v->active, s); }));
    if (v->desc.flags & PV_MULTI_BOUNCE)
        HIP_TRY(timed(c, PV_STAGE_BOUNCE, s,
                      [&] { return launch_bounce(vp, sv, v->dirs, v->rays, v->irr, v->vis, fp16, s); }));
    HIP_TRY(timed(c, PV_STAGE_BLEND, s, [&] { return launch_blend(vp, v->dirs, v->rays, v->irr, v->vis, fp16, h, s); }));
    PV_TRY(note_scene_use(v->scene, s));
    v->frame++;
    return PV_OK;
}

extern "C" pv_status pv_update_probes(pv_volume *v, const pv_frame *f, void *stream) {
    return update_probes(v, f, stream, nullptr);
}

extern "C" pv_status pv_update_probes_after(pv_volume *v, const pv_frame *f, void *stream, void *event) {
    if (!event) return fail(PV_ERR_ARG, "event is NULL");
    return update_probes(v, f, stream, event);
}

extern "C" pv_status pv_trace_counts(pv_volume *v, const pv_frame *f, uint64_t counts[3]) {
    if (!v || !counts) return fail(PV_ERR_ARG, "NULL argument");
    if (!v->scene) return fail(PV_ERR_STATE, "no scene set on the volume");
    FrameParams fp;
    PV_TRY(frame_params(f, v->scene, fp));
    HIP_TRY(hipSetDevice(v->ctx->device));
    pv_ctx *c = v->ctx;
    if (!c->counts_dev) PV_TRY(dev_alloc(&c->counts_dev, 4 * sizeof(unsigned long long), "counters"));
    hipStream_t s = c->stream;
    HIP_TRY(launch_zero(c->counts_dev, 4 * sizeof(unsigned long long), s));
    const bool timing = c->timing;
    c->timing = false;
    const pv_status st = enqueue_trace(v, fp, scene_view(v->scene), c->counts_dev, s);
    c->timing = timing;
    PV_TRY(st);
    PV_TRY(note_scene_use(v->scene, s));
    unsigned long long host[4];
    HIP_TRY(hipMemcpyAsync(host, c->counts_dev, sizeof(host), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < 3; ++i) counts[i] = host[i];
    return PV_OK;
}

extern "C" pv_status pv_measure_ceiling(pv_ctx *c, int kind, int reps, double *rate) {
    if (!c || !rate) return fail(PV_ERR_ARG, "NULL argument");
    if (kind < PV_CEIL_COPY || kind > PV_CEIL_MFMA_F32) return fail(PV_ERR_ARG, "unknown ceiling kind");
    if (reps < 1) return fail(PV_ERR_ARG, "reps must be >= 1");
    HIP_TRY(hipSetDevice(c->device));
    int cus = 256;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    const int blocks = cus * 8;  // 32 wavefronts per CU
    const size_t copy_bytes = (size_t)1 << 30;
    const int fma_iters = 4096, mfma_iters = 1024;
    void *a = nullptr, *b = nullptr;
    pv_status st = PV_OK;
    if (kind == PV_CEIL_COPY) {
        st = dev_alloc(&a, copy_bytes, "ceiling copy source");
        if (st == PV_OK) st = dev_alloc(&b, copy_bytes, "ceiling copy destination");
    } else {
        st = dev_alloc(&a, (size_t)blocks * 256 * sizeof(float), "ceiling output");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == PV_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(PV_ERR_DEVICE, "event create");
    hipStream_t s = c->stream;
    auto run = [&]() -> hipError_t {
        if (kind == PV_CEIL_COPY) return launch_ceil_copy(a, b, copy_bytes, blocks, s);
        if (kind == PV_CEIL_FMA_F32) return launch_ceil_fma((float *)a, blocks, fma_iters, s);
        return launch_ceil_mfma((float *)a, blocks, mfma_iters, s);
    };
    double best_ms = 0.0;
    for (int r = -1; st == PV_OK && r < reps; ++r) {  // one untimed warm-up
        if (hipEventRecord(e0, s) != hipSuccess || run() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess) {
            st = fail(PV_ERR_DEVICE, "ceiling kernel");
            break;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = fail(PV_ERR_DEVICE, "event time");
        if (r >= 0 && (best_ms == 0.0 || ms < best_ms)) best_ms = ms;
    }
    if (st == PV_OK) {
        const double threads = (double)blocks * 256;
        const double work = kind == PV_CEIL_COPY    ? 2.0 * (double)copy_bytes
                            : kind == PV_CEIL_FMA_F32 ? threads * fma_iters * 8 * 2
                                                      : threads / 64 * mfma_iters * 4 * 2048.0;
        *rate = work / (best_ms * 1e-3);
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(a);
    hipFree(b);
    return st;
}

extern "C" pv_status pv_blend_rays(pv_volume *v, const pv_frame *f, const void *rays_dev, void *stream) {
    if (!v || !rays_dev) return fail(PV_ERR_ARG, "NULL argument");
    FrameParams fp;
    PV_TRY(frame_params(f, v->scene, fp));
    HIP_TRY(hipSetDevice(v->ctx->device));
    hipStream_t s = pick(v->ctx, stream);
    const VolumeParams vp = volume_params(v);
    pv_ctx *c = v->ctx;
    const float h = effective_h(v);
    HIP_TRY(timed(c, PV_STAGE_RAYDIRS, s, [&] { return launch_raydirs(fp, vp, v->dirs, nullptr, s); }));
    HIP_TRY(timed(c, PV_STAGE_BLEND, s, [&] {
        return launch_blend(vp, v->dirs, (const float4 *)rays_dev, v->irr, v->vis, v->desc.format == PV_MAP_FP16, h, s);
    }));
    v->frame++;
    return PV_OK;
}

extern "C" pv_status pv_volume_set_blend_mode(pv_volume *v, int mode) {
    if (!v) return fail(PV_ERR_ARG, "volume is NULL");
    if (mode < PV_BLEND_AUTO || mode > PV_BLEND_BF16X6) return fail(PV_ERR_ARG, "unknown blend mode");
    v->blend_mode = mode == PV_BLEND_AUTO ? auto_blend_mode(v->P) : mode;
    return PV_OK;
}

extern "C" pv_status pv_volume_get_blend_mode(pv_volume *v, int *mode) {
    if (!v || !mode) return fail(PV_ERR_ARG, "NULL argument");
    *mode = v->blend_mode;
    return PV_OK;
}

extern "C" pv_status pv_volume_set_trace_config(pv_volume *v, const pv_trace_config *c) {
    if (!v || !c) return fail(PV_ERR_ARG, "NULL argument");
    if (c->brick[0] < 1 || c->brick[1] < 1 || c->brick[2] < 1 || c->brick[0] * c->brick[1] * c->brick[2] != 64)
        return fail(PV_ERR_ARG, "brick must hold 64 probes");
    if (c->persistent < 0 || c->persistent > 2) return fail(PV_ERR_ARG, "persistent must be 0, 1 or 2");
    if (c->top_nodes != 0 && c->top_nodes != 21 && c->top_nodes != 85) return fail(PV_ERR_ARG, "top_nodes must be 0, 21 or 85");
    if (c->block_threads != 128 && c->block_threads != 256) return fail(PV_ERR_ARG, "block_threads must be 128 or 256");
    if (c->split_shadows != 0 && c->split_shadows != 1) return fail(PV_ERR_ARG, "split_shadows must be 0 or 1");
    v->tc.bx = c->brick[0];
    v->tc.by = c->brick[1];
    v->tc.bz = c->brick[2];
    v->tc.persistent = c->persistent;
    v->tc.top_nodes = c->top_nodes;
    v->tc.block = c->block_threads;
    v->tc.split_shadows = c->split_shadows;
    return PV_OK;
}

extern "C" pv_status pv_volume_get_trace_config(pv_volume *v, pv_trace_config *c) {
    if (!v || !c) return fail(PV_ERR_ARG, "NULL argument");
    c->brick[0] = v->tc.bx;
    c->brick[1] = v->tc.by;
    c->brick[2] = v->tc.bz;
    c->persistent = v->tc.persistent;
    c->top_nodes = v->tc.top_nodes;
    c->block_threads = v->tc.block;
    c->split_shadows = v->tc.split_shadows;
    return PV_OK;
}

extern "C" pv_status pv_get_maps(pv_volume *v, void **irr, void **vis) {
    if (!v || !irr || !vis) return fail(PV_ERR_ARG, "NULL argument");
    *irr = v->irr;
    *vis = v->vis;
    return PV_OK;
}

extern "C" pv_status pv_get_rays(pv_volume *v, void **rays, void **hits, void **dirs) {
    if (!v) return fail(PV_ERR_ARG, "NULL argument");
    if (rays) *rays = v->rays;
    if (hits) *hits = v->hits;
    if (dirs) *dirs = v->dirs;
    return PV_OK;
}

extern "C" pv_status pv_probe_query(pv_volume *v, const float *pts, const float *nrms, int64_t n, float *out,
                                    void *stream) {
    if (!v) return fail(PV_ERR_ARG, "volume is NULL");
    if (n < 0) return fail(PV_ERR_ARG, "n must be >= 0");
    if (n == 0) return PV_OK;
    if (!pts || !nrms || !out) return fail(PV_ERR_ARG, "NULL buffer");
    if (n > (int64_t)1 << 31) return fail(PV_ERR_ARG, "at most 2^31 points per call");
    HIP_TRY(hipSetDevice(v->ctx->device));
    const int fp16 = v->desc.format == PV_MAP_FP16;
    HIP_TRY(launch_probe_query(volume_params(v), v->irr, v->vis, fp16, pts, nrms, out, (long long)n,
                               pick(v->ctx, stream)));
    return PV_OK;
}

extern "C" pv_status pv_set_maps(pv_volume *v, const void *irr, const void *vis, int64_t frame) {
    if (!v || !irr || !vis) return fail(PV_ERR_ARG, "NULL argument");
    if (frame < 0) return fail(PV_ERR_ARG, "frame must be >= 0");
    HIP_TRY(hipSetDevice(v->ctx->device));
    HIP_TRY(hipStreamSynchronize(v->ctx->stream));
    HIP_TRY(hipMemcpy(v->irr, irr, irr_bytes(v->P, v->elem), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(v->vis, vis, vis_bytes(v->P, v->elem), hipMemcpyHostToDevice));
    v->frame = frame;
    return PV_OK;
}

extern "C" pv_status pv_read_maps(pv_volume *v, void *irr, void *vis, int64_t *frame) {
    if (!v || !irr || !vis) return fail(PV_ERR_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(v->ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(irr, v->irr, irr_bytes(v->P, v->elem), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(vis, v->vis, vis_bytes(v->P, v->elem), hipMemcpyDeviceToHost));
    if (frame) *frame = v->frame;
    return PV_OK;
}

// ---------------------------------------------------------------------------
// batched update
// ---------------------------------------------------------------------------
static pv_status ensure_slot(pv_ctx *c, BatchSlot &b, int n) {
    if (n <= b.cap) return PV_OK;
    hipFree(b.batch_dev);
    hipFree(b.frames_dev);
    if (b.stage_host) hipHostFree(b.stage_host);
    b.batch_dev = nullptr;
    b.frames_dev = nullptr;
    b.stage_host = nullptr;
    b.cap = 0;
    PV_TRY(dev_alloc(&b.batch_dev, sizeof(BatchVolume) * n, "batch descriptors"));
    PV_TRY(dev_alloc(&b.frames_dev, sizeof(FrameParams) * n, "batch frames"));
    const size_t bytes = (sizeof(BatchVolume) + sizeof(FrameParams)) * n + 256;
    HIP_TRY(hipHostMalloc(&b.stage_host, bytes));
    b.cap = n;
    return PV_OK;
}

// ---------------------------------------------------------------------------
// captured batched frame
// ---------------------------------------------------------------------------
struct pv_batch_graph {
    pv_ctx *ctx = nullptr;
    std::vector<pv_volume *> vols;
    BatchSlot slot;           // device descriptors + pinned staging owned by the graph
    size_t o_b = 0, o_f = 0, bytes = 0;
    int waves = 0, blend = 0, bounce = 0, classify = 0, dir_blocks = 0;
    int blend_kind = kBatchBlendAny;  // the captured blend kernel (kBatchBlend*)
    bool short_stack = true;
    int max_top = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
};

// Fills the pinned staging of a batch: descriptors and frames; returns the
// packet, blend-group and second-bounce block totals, the most ray-direction
// blocks of a volume, whether every BVH of the batch fits 16-bit stack
// entries, and the most top nodes a volume stages.
static pv_status fill_batch(pv_volume *const *vols, const pv_frame *frames, int n, char *h, size_t *offs, int &waves,
                            int &blend, int &bounce, int &classify, int &dir_blocks, bool &short_stack,
                            int &max_top) {
    std::vector<BatchVolume> bv(n);
    std::vector<FrameParams> fps(n);
    std::memset(fps.data(), 0, sizeof(FrameParams) * n);
    waves = 0;
    blend = 0;
    bounce = 0;
    classify = 0;
    dir_blocks = 0;
    short_stack = true;
    max_top = 0;
    for (int i = 0; i < n; ++i) {
        pv_volume *v = vols[i];
        if (frames) PV_TRY(frame_params(&frames[i], v->scene, fps[i]));
        BatchVolume &b = bv[i];
        b.vp = volume_params(v);
        b.sv = scene_view(v->scene);
        short_stack = short_stack && b.sv.stat.n_nodes <= 65536 && b.sv.dyn.n_nodes <= 65536;
        b.dirs = v->dirs;
        dir_blocks = std::max(dir_blocks, raydir_blocks(v->n) + weight_blocks(v->blend_mode, v->n));
        b.rays = v->rays;
        b.hits = v->hits;
        b.irr = v->irr;
        b.vis = v->vis;
        b.h = effective_h(v);
        b.fp16 = v->desc.format == PV_MAP_FP16;
        // the volume's own trace shape: probe brick and staged top nodes (the
        // batched trace always runs the stepped lanes in 128-thread blocks)
        b.bx = v->tc.bx;
        b.by = v->tc.by;
        b.bz = v->tc.bz;
        b.top_nodes = v->tc.top_nodes;
        max_top = std::max(max_top, b.top_nodes);
        b.bricks_x = (v->desc.nx + b.bx - 1) / b.bx;
        b.bricks_y = (v->desc.ny + b.by - 1) / b.by;
        b.bricks_z = (v->desc.nz + b.bz - 1) / b.bz;
        b.n_waves = b.bricks_x * b.bricks_y * b.bricks_z * v->n;
        waves = (waves + 3) / 4 * 4;  // a multiple of the packets per trace block: each volume starts on a block boundary
        b.first_wave = waves;
        waves += b.n_waves;
        b.n_blend = blend_blocks(v->P, v->blend_mode);
        b.first_blend = blend;
        blend += b.n_blend;
        b.n_bounce = (v->desc.flags & PV_MULTI_BOUNCE) ? bounce_blocks(v->P, v->n) : 0;
        b.first_bounce = bounce;
        bounce += b.n_bounce;
        b.active = v->active;
        b.n_classify = v->active ? classify_blocks(v->P) : 0;
        b.first_classify = classify;
        classify += b.n_classify;
    }
    size_t off = 0;
    auto put = [&](const void *src, size_t bytes) {
        std::memcpy(h + off, src, bytes);
        size_t o = off;
        off += (bytes + 15) / 16 * 16;
        return o;
    };
    offs[0] = put(bv.data(), sizeof(BatchVolume) * n);
    offs[1] = put(fps.data(), sizeof(FrameParams) * n);  // zeros when no frames are given yet
    offs[2] = off;
    return PV_OK;
}

// The batched blend kernel for these volumes (kBatchBlend*).
static int batch_blend_kind(pv_volume *const *vols, int n) {
    bool half = true, flt = true;
    for (int i = 0; i < n; ++i) {
        const int m = vols[i]->blend_mode;
        if (m != kBlendTiles && m != kBlendF32 && m != kBlendBF16x6) return kBatchBlendAny;
        const bool h = vols[i]->desc.format == PV_MAP_FP16;
        half = half && h;
        flt = flt && !h;
    }
    return half ? kBatchBlendAutoHalf : flt ? kBatchBlendAutoFloat : kBatchBlendAny;
}

static pv_status check_batch(pv_volume *const *vols, int n, pv_ctx **ctx) {
    if (!vols || n < 1) return fail(PV_ERR_ARG, "need at least one volume");
    pv_ctx *c = vols[0] ? vols[0]->ctx : nullptr;
    if (!c) return fail(PV_ERR_ARG, "volume 0 is NULL");
    for (int i = 0; i < n; ++i) {
        if (!vols[i]) return fail(PV_ERR_ARG, "volume " + std::to_string(i) + " is NULL");
        if (vols[i]->ctx != c) return fail(PV_ERR_ARG, "volumes belong to different contexts");
        if (!vols[i]->scene) return fail(PV_ERR_STATE, "volume " + std::to_string(i) + " has no scene");
        for (int k = 0; k < i; ++k)
            if (vols[k] == vols[i]) return fail(PV_ERR_ARG, "a volume appears twice in one batch");
    }
    *ctx = c;
    return PV_OK;
}

extern "C" pv_status pv_update_probes_batched(pv_volume *const *vols, const pv_frame *frames, int n, void *stream) {
    if (!frames) return fail(PV_ERR_ARG, "frames is NULL");
    pv_ctx *c = nullptr;
    PV_TRY(check_batch(vols, n, &c));
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = pick(c, stream);
    BatchSlot &slot = c->slots[c->slot_next];
    c->slot_next = (c->slot_next + 1) % pv_ctx::kRing;
    HIP_TRY(hipEventSynchronize(slot.done));  // the slot's previous launch has finished
    PV_TRY(ensure_slot(c, slot, n));
    size_t offs[3];
    int waves, blend, bounce, classify, dir_blocks, max_top;
    bool short_stack;
    char *h = (char *)slot.stage_host;
    PV_TRY(fill_batch(vols, frames, n, h, offs, waves, blend, bounce, classify, dir_blocks, short_stack, max_top));
    HIP_TRY(hipMemcpyAsync(slot.batch_dev, h + offs[0], sizeof(BatchVolume) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(slot.frames_dev, h + offs[1], sizeof(FrameParams) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(timed(c, PV_STAGE_RAYDIRS, s,
                  [&] { return launch_raydirs_batched(slot.batch_dev, slot.frames_dev, n, dir_blocks, s); }));
    HIP_TRY(timed(c, PV_STAGE_BATCHED, s,
                  [&] { return launch_trace_batched(slot.batch_dev, n, waves, slot.frames_dev, short_stack, max_top, s); }));
    if (classify > 0)
        HIP_TRY(timed(c, PV_STAGE_SELECT, s, [&] { return launch_classify_batched(slot.batch_dev, n, classify, s); }));
    if (bounce > 0)
        HIP_TRY(timed(c, PV_STAGE_BOUNCE, s, [&] { return launch_bounce_batched(slot.batch_dev, n, bounce, s); }));
    const int kind = batch_blend_kind(vols, n);
    HIP_TRY(timed(c, PV_STAGE_BLEND, s, [&] { return launch_blend_batched(slot.batch_dev, n, blend, kind, s); }));
    HIP_TRY(hipEventRecord(slot.done, s));
    for (int i = 0; i < n; ++i) {
        PV_TRY(note_scene_use(vols[i]->scene, s));
        vols[i]->frame++;
    }
    return PV_OK;
}

static void free_graph(pv_batch_graph *g) {
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    if (g->done) hipEventDestroy(g->done);
    BatchSlot &b = g->slot;
    hipFree(b.batch_dev);
    hipFree(b.frames_dev);
    if (b.stage_host) hipHostFree(b.stage_host);
    delete g;
}

extern "C" pv_status pv_batch_graph_create(pv_volume *const *vols, int n, pv_batch_graph **out) {
    if (!out) return fail(PV_ERR_ARG, "out is NULL");
    pv_ctx *c = nullptr;
    PV_TRY(check_batch(vols, n, &c));
    HIP_TRY(hipSetDevice(c->device));
    pv_batch_graph *g = new pv_batch_graph();
    g->ctx = c;
    g->vols.assign(vols, vols + n);
    pv_status st = ensure_slot(c, g->slot, n);
    if (st == PV_OK && hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess)
        st = fail(PV_ERR_DEVICE, "event");
    size_t offs[3];
    if (st == PV_OK)
        st = fill_batch(vols, nullptr, n, (char *)g->slot.stage_host, offs, g->waves, g->blend, g->bounce,
                        g->classify, g->dir_blocks, g->short_stack, g->max_top);
    if (st != PV_OK) {
        free_graph(g);
        return st;
    }
    g->o_b = offs[0];
    g->o_f = offs[1];
    g->bytes = offs[2];
    // capture on a private stream: copy nodes, ray directions, trace, blend
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    BatchSlot &b = g->slot;
    char *h = (char *)b.stage_host;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = hipMemcpyAsync(b.batch_dev, h + g->o_b, sizeof(BatchVolume) * n, hipMemcpyHostToDevice, cs);
    if (e == hipSuccess) e = hipMemcpyAsync(b.frames_dev, h + g->o_f, sizeof(FrameParams) * n, hipMemcpyHostToDevice, cs);
    if (e == hipSuccess) e = launch_raydirs_batched(b.batch_dev, b.frames_dev, n, g->dir_blocks, cs);
    if (e == hipSuccess) e = launch_trace_batched(b.batch_dev, n, g->waves, b.frames_dev, g->short_stack, g->max_top, cs);
    if (e == hipSuccess && g->classify > 0) e = launch_classify_batched(b.batch_dev, n, g->classify, cs);
    if (e == hipSuccess && g->bounce > 0) e = launch_bounce_batched(b.batch_dev, n, g->bounce, cs);
    g->blend_kind = batch_blend_kind(vols, n);
    if (e == hipSuccess) e = launch_blend_batched(b.batch_dev, n, g->blend, g->blend_kind, cs);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) {
        g->graph = graph;
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    } else if (graph) {
        hipGraphDestroy(graph);
    }
    hipStreamDestroy(cs);
    if (e != hipSuccess) {
        free_graph(g);
        return fail(PV_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *out = g;
    return PV_OK;
}

extern "C" pv_status pv_batch_graph_launch(pv_batch_graph *g, const pv_frame *frames, void *stream) {
    if (!g || !frames) return fail(PV_ERR_ARG, "NULL argument");
    pv_ctx *c = g->ctx;
    HIP_TRY(hipSetDevice(c->device));
    const int n = (int)g->vols.size();
    for (int i = 0; i < n; ++i)
        if (!g->vols[i]->scene) return fail(PV_ERR_STATE, "a volume of the graph has no scene");
    // the copy node reads the pinned buffer when the graph runs: the previous
    // launch must have finished before it is rewritten
    if (g->launched) HIP_TRY(hipEventSynchronize(g->done));
    size_t offs[3];
    int waves, blend, bounce, classify, dir_blocks, max_top;
    bool short_stack;
    PV_TRY(fill_batch(g->vols.data(), frames, n, (char *)g->slot.stage_host, offs, waves, blend, bounce, classify,
                      dir_blocks, short_stack, max_top));
    if (waves != g->waves || blend != g->blend || bounce != g->bounce || classify != g->classify ||
        short_stack != g->short_stack || max_top != g->max_top || batch_blend_kind(g->vols.data(), n) != g->blend_kind)
        return fail(PV_ERR_STATE,
                    "a volume of the graph changed scene, trace shape or blend path since the graph was captured");
    hipStream_t s = pick(c, stream);
    HIP_TRY(timed(c, PV_STAGE_BATCHED, s, [&] { return hipGraphLaunch(g->exec, s); }));
    HIP_TRY(hipEventRecord(g->done, s));
    g->launched = true;
    for (int i = 0; i < n; ++i) {
        PV_TRY(note_scene_use(g->vols[i]->scene, s));
        g->vols[i]->frame++;
    }
    return PV_OK;
}

extern "C" pv_status pv_batch_graph_destroy(pv_batch_graph *g) {
    if (!g) return PV_OK;
    hipSetDevice(g->ctx->device);
    if (g->launched) hipEventSynchronize(g->done);
    free_graph(g);
    return PV_OK;
}

// ---------------------------------------------------------------------------
// client + pack
// ---------------------------------------------------------------------------
extern "C" pv_status pv_client_footprint(const pv_volume_desc *d, uint64_t *bytes) {
    PV_TRY(validate_desc(d));
    if (!bytes) return fail(PV_ERR_ARG, "bytes is NULL");
    const uint64_t P = (uint64_t)d->nx * d->ny * d->nz;
    *bytes = P * (192 + 512) * 2 + 3 * P + (P + kPackTile - 1) / kPackTile * 20 + 16 + packet_capacity((int)P);
    return PV_OK;
}

static void free_client(pv_client *c) {
    hipFree(c->ref_irr);
    hipFree(c->ref_vis);
    hipFree(c->mask_irr);
    hipFree(c->mask_vis);
    hipFree(c->tiles);
    hipFree(c->totals);
    hipFree(c->tiles2);
    hipFree(c->cks);
    hipFree(c->tsum);
    hipFree(c->packet);
    hipFree(c->view);
    hipFree(c->ent.hist);
    hipFree(c->ent.lens);
    hipFree(c->ent.codes);
    hipFree(c->ent.chunk_bits);
    hipFree(c->ent.chunk_off);
    hipFree(c->ent.total);
    hipFree(c->ent.out);
    if (c->ent_total_host) hipHostFree(c->ent_total_host);
    if (c->ent_tables_host) hipHostFree(c->ent_tables_host);
    if (c->hdr_host) hipHostFree(c->hdr_host);
    if (c->stage_host) hipHostFree(c->stage_host);
    delete c;
}

extern "C" pv_status pv_client_create(pv_volume *v, uint32_t id, pv_client **out) {
    if (!v || !out) return fail(PV_ERR_ARG, "NULL argument");
    if (v->desc.format != PV_MAP_FP16)
        return fail(PV_ERR_UNSUPPORTED, "delta packing is defined on FP16 maps (FP32 byte planes not built)");
    HIP_TRY(hipSetDevice(v->ctx->device));
    pv_client *c = new pv_client();
    c->vol = v;
    c->id = id;
    const int P = v->P;
    c->packet_cap = packet_capacity(P);
    pv_status st = dev_alloc(&c->ref_irr, (size_t)P * 192 * 2, "irradiance reference");
    if (st == PV_OK) st = dev_alloc(&c->ref_vis, (size_t)P * 512 * 2, "visibility reference");
    if (st == PV_OK) st = dev_alloc(&c->mask_irr, (size_t)P, "mask");
    if (st == PV_OK) st = dev_alloc(&c->mask_vis, (size_t)P, "mask");
    if (st == PV_OK) st = dev_alloc(&c->tiles, (size_t)(P + kPackTile - 1) / kPackTile * sizeof(int4), "tile summaries");
    if (st == PV_OK) st = dev_alloc(&c->totals, 4 * sizeof(uint32_t), "pack totals");
    if (st == PV_OK) st = dev_alloc(&c->tiles2, (size_t)(P + kPackTile - 1) / kPackTile * sizeof(int2), "tile summaries");
    if (st == PV_OK) st = dev_alloc(&c->cks, kCksBytes, "pack checksum counters");
    if (st == PV_OK) st = dev_alloc(&c->tsum, (size_t)(P + kPackTile - 1) / kPackTile * 4, "tile summaries");
    if (st == PV_OK) st = dev_alloc(&c->packet, c->packet_cap, "packet");
    if (st == PV_OK) st = dev_alloc(&c->view, (size_t)P, "client view");
    if (st == PV_OK && hipHostMalloc((void **)&c->hdr_host, 32) != hipSuccess) st = fail(PV_ERR_OOM, "pinned header");
    hipStream_t s = v->ctx->stream;
    if (st == PV_OK && (launch_zero(c->ref_irr, (size_t)P * 192 * 2, s) != hipSuccess ||
                        launch_zero(c->ref_vis, (size_t)P * 512 * 2, s) != hipSuccess ||
                        launch_zero(c->mask_irr, (size_t)P, s) != hipSuccess ||
                        launch_zero(c->mask_vis, (size_t)P, s) != hipSuccess ||
                        launch_zero(c->packet, 32, s) != hipSuccess ||
                        launch_zero(c->cks, kCksBytes, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
        st = fail(PV_ERR_DEVICE, "client initialisation");
    if (st != PV_OK) {
        free_client(c);
        return st;
    }
    *out = c;
    return PV_OK;
}

extern "C" pv_status pv_client_destroy(pv_client *c) {
    if (!c) return PV_OK;
    hipSetDevice(c->vol->ctx->device);
    hipDeviceSynchronize();
    free_client(c);
    return PV_OK;
}

extern "C" pv_status pv_client_reset(pv_client *c, void *stream) {
    if (!c) return fail(PV_ERR_ARG, "client is NULL");
    HIP_TRY(hipSetDevice(c->vol->ctx->device));
    hipStream_t s = pick(c->vol->ctx, stream);
    HIP_TRY(launch_zero(c->ref_irr, (size_t)c->vol->P * 192 * 2, s));
    HIP_TRY(launch_zero(c->ref_vis, (size_t)c->vol->P * 512 * 2, s));
    return PV_OK;
}

extern "C" pv_status pv_pack_delta(pv_client *c, float tau_irr, float tau_vis, void *stream) {
    if (!c) return fail(PV_ERR_ARG, "client is NULL");
    if (!(tau_irr >= 0.f) || !(tau_vis >= 0.f) || !std::isfinite(tau_irr) || !std::isfinite(tau_vis))
        return fail(PV_ERR_ARG, "thresholds must be finite and >= 0");
    pv_volume *v = c->vol;
    HIP_TRY(hipSetDevice(v->ctx->device));
    hipStream_t s = pick(v->ctx, stream);
    PackBuffers b;
    b.cur_irr = (const uint16_t *)v->irr;
    b.cur_vis = (const uint16_t *)v->vis;
    b.ref_irr = c->ref_irr;
    b.ref_vis = c->ref_vis;
    b.mask_irr = c->mask_irr;
    b.mask_vis = c->mask_vis;
    b.tiles = c->tiles;
    b.totals = c->totals;
    b.tiles2 = c->tiles2;
    b.cks = c->cks;
    b.tsum = c->tsum;
    b.packet = c->packet;
    b.active = v->active;
    b.view = c->view_on ? c->view : nullptr;
    pv_ctx *cx = v->ctx;
    const int P = v->P;
    const uint32_t id = c->id, seq = c->seq;
    HIP_TRY(timed(cx, PV_STAGE_PACK_MASK, s, [&] { return launch_pack_mask(b, P, tau_irr, tau_vis, s); }));
    if (!pack_fused(P)) HIP_TRY(timed(cx, PV_STAGE_PACK_SCAN, s, [&] { return launch_pack_scan(b, P, s); }));
    HIP_TRY(timed(cx, PV_STAGE_PACK_COMPACT, s, [&] { return launch_pack_compact(b, P, id, seq, s); }));
    c->seq++;
    return PV_OK;
}

extern "C" pv_status pv_pack_delta_noalloc(pv_ctx *cx, const uint16_t *cur_irr, const uint16_t *cur_vis,
                                           uint16_t *ref_irr, uint16_t *ref_vis, int n_probes, float tau_irr,
                                           float tau_vis, uint32_t client_id, uint32_t seq, uint8_t *packet,
                                           uint64_t packet_cap, void *stream) {
    if (!cx || !cur_irr || !cur_vis || !ref_irr || !ref_vis || !packet) return fail(PV_ERR_ARG, "NULL argument");
    if (n_probes < 1 || n_probes > kNoAllocMaxProbes)
        return fail(PV_ERR_ARG, "n_probes " + std::to_string(n_probes) + " outside [1, " +
                                    std::to_string(kNoAllocMaxProbes) + "] (the scratch array's limit)");
    if (!(tau_irr >= 0.f) || !(tau_vis >= 0.f) || !std::isfinite(tau_irr) || !std::isfinite(tau_vis))
        return fail(PV_ERR_ARG, "thresholds must be finite and >= 0");
    const uintptr_t align = (uintptr_t)cur_irr | (uintptr_t)cur_vis | (uintptr_t)ref_irr | (uintptr_t)ref_vis |
                            (uintptr_t)packet;
    if (align & 15u) return fail(PV_ERR_ARG, "maps, references and packet must be 16-byte aligned");
    if (packet_cap < packet_capacity(n_probes))
        return fail(PV_ERR_CAPACITY, "packet buffer needs " + std::to_string(packet_capacity(n_probes)) +
                                         " bytes (a full resend)");
    HIP_TRY(hipSetDevice(cx->device));
    unsigned char *scr = noalloc_scratch(cx->device);
    if (!scr) return fail(PV_ERR_STATE, "scratch array not set up on this device");
    HIP_TRY(launch_pack_noalloc(scr, cur_irr, cur_vis, ref_irr, ref_vis, n_probes, tau_irr, tau_vis, client_id, seq,
                                packet, pick(cx, stream)));
    return PV_OK;
}

extern "C" pv_status pv_client_read_state(pv_client *c, void *ri, void *rv, uint32_t *seq) {
    if (!c || !ri || !rv) return fail(PV_ERR_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(c->vol->ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(ri, c->ref_irr, (size_t)c->vol->P * 192 * 2, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(rv, c->ref_vis, (size_t)c->vol->P * 512 * 2, hipMemcpyDeviceToHost));
    if (seq) *seq = c->seq;
    return PV_OK;
}

extern "C" pv_status pv_client_set_state(pv_client *c, const void *ri, const void *rv, uint32_t seq) {
    if (!c || !ri || !rv) return fail(PV_ERR_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(c->vol->ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(c->ref_irr, ri, (size_t)c->vol->P * 192 * 2, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->ref_vis, rv, (size_t)c->vol->P * 512 * 2, hipMemcpyHostToDevice));
    c->seq = seq;
    return PV_OK;
}

extern "C" pv_status pv_packet_device(pv_client *c, const void **p, uint64_t *cap) {
    if (!c || !p || !cap) return fail(PV_ERR_ARG, "NULL argument");
    *p = c->packet;
    *cap = c->packet_cap;
    return PV_OK;
}

extern "C" pv_status pv_get_masks(pv_client *c, void **mi, void **mv) {
    if (!c || !mi || !mv) return fail(PV_ERR_ARG, "NULL argument");
    *mi = c->mask_irr;
    *mv = c->mask_vis;
    return PV_OK;
}

// Waits for the last pack on s and copies the whole packet into the
// client's pinned staging (D2H at full PCIe rate, no pageable bounce).
static pv_status stage_packet(pv_client *c, hipStream_t s, uint64_t *bytes) {
    HIP_TRY(hipMemcpyAsync(c->hdr_host, c->packet, 32, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint32_t K_irr = c->hdr_host[kHdrKIrr], K_vis = c->hdr_host[kHdrKVis];
    if (c->hdr_host[kHdrMagic] != kPacketMagic) return fail(PV_ERR_STATE, "no packet has been built");
    const uint64_t total = packet_bytes(K_irr, K_vis);
    if (total > c->stage_cap) {
        if (c->stage_host) hipHostFree(c->stage_host);
        c->stage_host = nullptr;
        c->stage_cap = 0;
        if (hipHostMalloc((void **)&c->stage_host, total) != hipSuccess) return fail(PV_ERR_OOM, "pinned packet staging");
        c->stage_cap = total;
    }
    std::memcpy(c->stage_host, c->hdr_host, 32);
    if (total > 32) HIP_TRY(hipMemcpyAsync(c->stage_host + 32, c->packet + 32, total - 32, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *bytes = total;
    return PV_OK;
}

extern "C" pv_status pv_packet_download(pv_client *c, void *host, uint64_t cap, uint64_t *bytes, void *stream) {
    if (!c || !bytes) return fail(PV_ERR_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(c->vol->ctx->device));
    hipStream_t s = pick(c->vol->ctx, stream);
    HIP_TRY(hipMemcpyAsync(c->hdr_host, c->packet, 32, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->hdr_host[kHdrMagic] != kPacketMagic) return fail(PV_ERR_STATE, "no packet has been built");
    const uint64_t total = packet_bytes(c->hdr_host[kHdrKIrr], c->hdr_host[kHdrKVis]);
    *bytes = total;
    if (!host || cap < total) return fail(PV_ERR_CAPACITY, "packet needs " + std::to_string(total) + " bytes");
    PV_TRY(stage_packet(c, s, bytes));
    std::memcpy(host, c->stage_host, total);
    return PV_OK;
}

extern "C" pv_status pv_packet_stage(pv_client *c, const void **host_ptr, uint64_t *bytes, void *stream) {
    if (!c || !host_ptr || !bytes) return fail(PV_ERR_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(c->vol->ctx->device));
    PV_TRY(stage_packet(c, pick(c->vol->ctx, stream), bytes));
    *host_ptr = c->stage_host;
    return PV_OK;
}

extern "C" pv_status pv_sync(void *stream) {
    hipError_t e = stream ? hipStreamSynchronize((hipStream_t)stream) : hipDeviceSynchronize();
    if (e != hipSuccess) return fail(PV_ERR_DEVICE, std::string("device error: ") + hipGetErrorString(e));
    return PV_OK;
}


// ---------------------------------------------------------------------------
// receiver (client-side unpack)
// ---------------------------------------------------------------------------
struct pv_receiver {
    pv_ctx *ctx = nullptr;
    int P = 0;
    uint16_t *irr = nullptr, *vis = nullptr;  // tiles with guard bands
    int *idx = nullptr;
    RxStatus *status = nullptr;
    uint8_t *pkt = nullptr;                   // device copy of the packet being applied
    uint8_t *stage = nullptr;                 // pinned staging of the host packet
    uint64_t cap = 0;
    hipEvent_t copied = nullptr, done = nullptr;
    bool used = false;
    uint32_t checksum = 0, seq = 0, last_seq = 0;
    bool pending = false;
    // compressed packets: device container, chunk list and decode tables;
    // pinned staging of the container and chunk list
    uint8_t *ent_in = nullptr;
    EntChunk *ent_chunks = nullptr;
    EntBlock *ent_blocks = nullptr;
    uint64_t ent_in_cap = 0, ent_chunk_cap = 0, ent_block_cap = 0;
    uint8_t *ent_stage = nullptr;
    uint64_t ent_stage_cap = 0;
};

static void free_receiver(pv_receiver *r) {
    hipFree(r->irr);
    hipFree(r->vis);
    hipFree(r->idx);
    hipFree(r->status);
    hipFree(r->pkt);
    hipFree(r->ent_in);
    hipFree(r->ent_chunks);
    hipFree(r->ent_blocks);
    if (r->ent_stage) hipHostFree(r->ent_stage);
    if (r->stage) hipHostFree(r->stage);
    if (r->copied) hipEventDestroy(r->copied);
    if (r->done) hipEventDestroy(r->done);
    delete r;
}

extern "C" pv_status pv_receiver_create(pv_ctx *ctx, int n_probes, pv_receiver **out) {
    if (!ctx || !out) return fail(PV_ERR_ARG, "NULL argument");
    if (n_probes < 1 || n_probes > PV_MAX_PROBES) return fail(PV_ERR_ARG, "n_probes must be in [1, 65536]");
    HIP_TRY(hipSetDevice(ctx->device));
    pv_receiver *r = new pv_receiver();
    r->ctx = ctx;
    r->P = n_probes;
    r->cap = packet_capacity(n_probes);
    pv_status st = dev_alloc(&r->irr, irr_bytes(r->P, 2), "receiver irradiance tiles");
    if (st == PV_OK) st = dev_alloc(&r->vis, vis_bytes(r->P, 2), "receiver visibility tiles");
    if (st == PV_OK) st = dev_alloc(&r->idx, (size_t)2 * r->P * sizeof(int), "receiver index");
    if (st == PV_OK) st = dev_alloc(&r->status, sizeof(RxStatus), "receiver status");
    if (st == PV_OK) st = dev_alloc(&r->pkt, r->cap, "receiver packet buffer");
    if (st == PV_OK && hipHostMalloc((void **)&r->stage, r->cap) != hipSuccess)
        st = fail(PV_ERR_OOM, "pinned packet staging");
    if (st == PV_OK && (hipEventCreateWithFlags(&r->copied, hipEventDisableTiming) != hipSuccess ||
                        hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess))
        st = fail(PV_ERR_DEVICE, "event");
    if (st == PV_OK && launch_zero(r->irr, irr_bytes(r->P, 2), ctx->stream) != hipSuccess) st = fail(PV_ERR_DEVICE, "zero fill");
    if (st == PV_OK && launch_zero(r->vis, vis_bytes(r->P, 2), ctx->stream) != hipSuccess) st = fail(PV_ERR_DEVICE, "zero fill");
    if (st == PV_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(PV_ERR_DEVICE, "sync after zero fill");
    if (st != PV_OK) {
        free_receiver(r);
        return st;
    }
    *out = r;
    return PV_OK;
}

extern "C" pv_status pv_receiver_destroy(pv_receiver *r) {
    if (!r) return PV_OK;
    hipSetDevice(r->ctx->device);
    if (r->used) hipEventSynchronize(r->done);
    free_receiver(r);
    return PV_OK;
}

static uint32_t get_u32(const uint8_t *p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

// Header of a packet for receiver r: magic, version, probe count, sent
// counts; returns the packet size in *size.
static pv_status check_packet_header(const pv_receiver *r, const uint8_t *h, uint64_t *size) {
    if (get_u32(h + 4 * kHdrMagic) != kPacketMagic) return fail(PV_ERR_ARG, "not a probe packet (magic)");
    if (get_u32(h + 4 * kHdrVersion) != kPacketVersion) return fail(PV_ERR_UNSUPPORTED, "packet version");
    if (get_u32(h + 4 * kHdrProbes) != (uint32_t)r->P) return fail(PV_ERR_ARG, "packet is for another probe count");
    const uint32_t K_irr = get_u32(h + 4 * kHdrKIrr), K_vis = get_u32(h + 4 * kHdrKVis);
    if (K_irr > (uint32_t)r->P || K_vis > (uint32_t)r->P) return fail(PV_ERR_ARG, "more sent probes than probes");
    *size = packet_bytes(K_irr, K_vis);
    return PV_OK;
}

// Verifies and applies the packet now in r->pkt (ordered on s), header h.
static pv_status receive_on_device(pv_receiver *r, const uint8_t *h, hipStream_t s) {
    const uint32_t K_irr = get_u32(h + 4 * kHdrKIrr), K_vis = get_u32(h + 4 * kHdrKVis);
    const uint64_t bytes = packet_bytes(K_irr, K_vis);
    RxBuffers b;
    b.pkt = r->pkt;
    b.P = r->P;
    b.K_irr = (int)K_irr;
    b.K_vis = (int)K_vis;
    b.checksum = get_u32(h + 4 * kHdrChecksum);
    b.payload_words = (long long)(bytes - kPacketHeader) / 4;
    b.irr = r->irr;
    b.vis = r->vis;
    b.idx = r->idx;
    b.status = r->status;
    HIP_TRY(timed(r->ctx, PV_STAGE_UNPACK, s, [&] { return launch_receive(b, s); }));
    HIP_TRY(hipEventRecord(r->done, s));
    r->used = true;
    r->checksum = b.checksum;
    r->seq = get_u32(h + 4 * kHdrSeq);
    r->pending = true;
    return PV_OK;
}

extern "C" pv_status pv_receiver_apply(pv_receiver *r, const void *packet, uint64_t bytes, void *stream) {
    if (!r || !packet) return fail(PV_ERR_ARG, "NULL argument");
    const uint8_t *h = (const uint8_t *)packet;
    if (bytes < (uint64_t)kPacketHeader) return fail(PV_ERR_ARG, "packet shorter than its header");
    uint64_t size = 0;
    PV_TRY(check_packet_header(r, h, &size));
    if (bytes != size) return fail(PV_ERR_ARG, "packet size does not match its header");
    HIP_TRY(hipSetDevice(r->ctx->device));
    hipStream_t s = pick(r->ctx, stream);
    // the staging buffer is free once the previous copy has run; the device
    // packet buffer once the previous unpack has (ordered on this stream)
    if (r->used) {
        HIP_TRY(hipEventSynchronize(r->copied));
        HIP_TRY(hipStreamWaitEvent(s, r->done, 0));
    }
    std::memcpy(r->stage, packet, bytes);
    HIP_TRY(hipMemcpyAsync(r->pkt, r->stage, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(r->copied, s));
    return receive_on_device(r, h, s);
}

extern "C" pv_status pv_receiver_status(pv_receiver *r, int *result, uint32_t *seq) {
    if (!r || !result) return fail(PV_ERR_ARG, "NULL argument");
    if (!r->used) return fail(PV_ERR_STATE, "no packet has been applied");
    HIP_TRY(hipSetDevice(r->ctx->device));
    HIP_TRY(hipEventSynchronize(r->done));
    RxStatus st;
    HIP_TRY(hipMemcpy(&st, r->status, sizeof st, hipMemcpyDeviceToHost));
    *result = st.bad_index ? -4 : (st.sum != r->checksum ? -2 : 0);
    if (r->pending && *result == 0) r->last_seq = r->seq;
    r->pending = false;
    if (seq) *seq = r->last_seq;
    return PV_OK;
}

extern "C" pv_status pv_receiver_get_maps(pv_receiver *r, void **irr, void **vis) {
    if (!r || !irr || !vis) return fail(PV_ERR_ARG, "NULL argument");
    *irr = r->irr;
    *vis = r->vis;
    return PV_OK;
}

extern "C" pv_status pv_receiver_read_maps(pv_receiver *r, void *irr, void *vis) {
    if (!r || !irr || !vis) return fail(PV_ERR_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(r->ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(irr, r->irr, irr_bytes(r->P, 2), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(vis, r->vis, vis_bytes(r->P, 2), hipMemcpyDeviceToHost));
    return PV_OK;
}

// ---------------------------------------------------------------------------
// codec surfaces
// ---------------------------------------------------------------------------
static pv_status check_layout(int P, int C) {
    if (P < 1 || P > PV_MAX_PROBES) return fail(PV_ERR_ARG, "n_probes must be in [1, 65536]");
    if (C < 1 || C > PV_MAX_PROBES) return fail(PV_ERR_ARG, "tiles_per_row must be in [1, 65536]");
    return PV_OK;
}

extern "C" pv_status pv_yuv_dims(int n_probes, int tiles_per_row, int64_t dims[4]) {
    if (!dims) return fail(PV_ERR_ARG, "dims is NULL");
    PV_TRY(check_layout(n_probes, tiles_per_row));
    const YuvDims d = yuv_dims(n_probes, tiles_per_row);
    dims[0] = d.w;
    dims[1] = d.h;
    dims[2] = d.wv;
    dims[3] = d.hv;
    return PV_OK;
}

extern "C" pv_status pv_encode_yuv(pv_volume *v, float irr_scale, int tiles_per_row, uint16_t *irr_planes,
                                   uint8_t *vis_planes, void *stream) {
    if (!v || !irr_planes || !vis_planes) return fail(PV_ERR_ARG, "NULL argument");
    if (v->desc.format != PV_MAP_FP16) return fail(PV_ERR_UNSUPPORTED, "codec surfaces need FP16 maps");
    if (!(irr_scale > 0.f) || !std::isfinite(irr_scale)) return fail(PV_ERR_ARG, "irr_scale must be finite and > 0");
    PV_TRY(check_layout(v->P, tiles_per_row));
    HIP_TRY(hipSetDevice(v->ctx->device));
    const float k = (float)(1023.0 / (double)irr_scale);
    const YuvDims d = yuv_dims(v->P, tiles_per_row);
    hipStream_t s = pick(v->ctx, stream);
    HIP_TRY(timed(v->ctx, PV_STAGE_CODEC, s, [&] {
        return launch_yuv_encode((const uint16_t *)v->irr, (const uint16_t *)v->vis, v->P, tiles_per_row, k,
                                 irr_planes, vis_planes, d, s);
    }));
    return PV_OK;
}

extern "C" pv_status pv_decode_yuv(pv_ctx *ctx, int n_probes, int tiles_per_row, const uint16_t *irr_planes,
                                   const uint8_t *vis_planes, uint32_t *irr_codes, uint16_t *vis, void *stream) {
    if (!ctx || !irr_planes || !vis_planes || !irr_codes || !vis) return fail(PV_ERR_ARG, "NULL argument");
    PV_TRY(check_layout(n_probes, tiles_per_row));
    HIP_TRY(hipSetDevice(ctx->device));
    const YuvDims d = yuv_dims(n_probes, tiles_per_row);
    hipStream_t s = pick(ctx, stream);
    HIP_TRY(timed(ctx, PV_STAGE_CODEC, s, [&] {
        return launch_yuv_decode(irr_planes, vis_planes, n_probes, tiles_per_row, irr_codes, vis, d, s);
    }));
    return PV_OK;
}

// ---------------------------------------------------------------------------
// probe selection
// ---------------------------------------------------------------------------
extern "C" pv_status pv_get_active(pv_volume *v, const void **active_dev) {
    if (!v || !active_dev) return fail(PV_ERR_ARG, "NULL argument");
    if (!v->active) return fail(PV_ERR_STATE, "volume was created without PV_CLASSIFY");
    *active_dev = v->active;
    return PV_OK;
}

extern "C" pv_status pv_client_set_view(pv_client *c, const float eye[3], int n_rays, void *stream) {
    if (!c || !eye) return fail(PV_ERR_ARG, "NULL argument");
    if (!finite_all(eye, 3)) return fail(PV_ERR_ARG, "eye must be finite");
    if (n_rays < 1 || n_rays > (1 << 22)) return fail(PV_ERR_ARG, "n_rays must be in [1, 4194304]");
    pv_volume *v = c->vol;
    if (!v->scene) return fail(PV_ERR_STATE, "no scene set on the client's volume");
    HIP_TRY(hipSetDevice(v->ctx->device));
    hipStream_t s = pick(v->ctx, stream);
    const VolumeParams vp = volume_params(v);
    const SceneView sv = scene_view(v->scene);
    HIP_TRY(launch_fill_u8(c->view, (size_t)v->P, 0, s));
    HIP_TRY(timed(v->ctx, PV_STAGE_SELECT, s,
                  [&] { return launch_client_view(vp, sv, eye[0], eye[1], eye[2], n_rays, c->view, s); }));
    PV_TRY(note_scene_use(v->scene, s));
    c->view_on = true;
    return PV_OK;
}

extern "C" pv_status pv_client_clear_view(pv_client *c) {
    if (!c) return fail(PV_ERR_ARG, "NULL argument");
    c->view_on = false;
    return PV_OK;
}

extern "C" pv_status pv_client_get_view(pv_client *c, const void **view_dev) {
    if (!c || !view_dev) return fail(PV_ERR_ARG, "NULL argument");
    *view_dev = c->view_on ? c->view : nullptr;
    return PV_OK;
}

// ---------------------------------------------------------------------------
// entropy stage
// ---------------------------------------------------------------------------
static constexpr int kHufChunk = 1024;
static constexpr uint32_t kContainerMagic = 0x43485650u;  // "PVHC"

static int max_chunks_of(int P) { return (int)(((int64_t)P * kVisPlaneBytes + kHufChunk - 1) / kHufChunk); }

// Huffman code lengths of one histogram: the two lightest nodes merged
// first, a leaf before an internal node of equal weight, leaves in (count,
// value) order; a lone symbol gets length 1; while the longest code exceeds
// 12 bits every count is halved (rounded up) and the lengths rebuilt.
static void huffman_lengths(const uint32_t *hist, uint8_t *len) {
    std::vector<uint64_t> cnt(hist, hist + 256);
    for (;;) {
        std::vector<std::pair<uint64_t, int>> leaves;
        for (int v = 0; v < 256; ++v)
            if (cnt[v]) leaves.push_back({cnt[v], v});
        std::memset(len, 0, 256);
        const int n = (int)leaves.size();
        if (n == 0) return;
        if (n == 1) {
            len[leaves[0].second] = 1;
            return;
        }
        std::sort(leaves.begin(), leaves.end());
        // nodes 0..n-1 are the leaves, n.. the merged nodes in creation order
        std::vector<uint64_t> w(2 * n);
        std::vector<int> parent(2 * n, -1);
        for (int i = 0; i < n; ++i) w[i] = leaves[i].first;
        int li = 0, mi = n, me = n;
        while ((n - li) + (me - mi) > 1) {
            int pick[2];
            for (int &pk : pick) pk = (li < n && (mi >= me || w[li] <= w[mi])) ? li++ : mi++;
            w[me] = w[pick[0]] + w[pick[1]];
            parent[pick[0]] = parent[pick[1]] = me;
            ++me;
        }
        std::vector<int> depth(me, 0);
        for (int i = me - 2; i >= 0; --i) depth[i] = depth[parent[i]] + 1;
        int longest = 0;
        for (int i = 0; i < n; ++i) {
            len[leaves[i].second] = (uint8_t)depth[i];
            longest = std::max(longest, depth[i]);
        }
        if (longest <= 12) return;
        for (auto &x : cnt) x = (x + 1) / 2;
    }
}

// Canonical codes: in (length, value) order, each code the previous one plus
// one, shifted left by the length difference.
static void canonical_codes_host(const uint8_t *len, uint32_t *code) {
    uint32_t c = 0;
    int prev = 0;
    bool first = true;
    for (int L = 1; L <= 12; ++L)
        for (int v = 0; v < 256; ++v)
            if (len[v] == L) {
                c = first ? 0u : (c + 1u) << (L - prev);
                first = false;
                prev = L;
                code[v] = c;
            }
    for (int v = 0; v < 256; ++v)
        if (!len[v]) code[v] = 0;
}

extern "C" pv_status pv_entropy_encode(pv_client *c, void *stream) {
    if (!c) return fail(PV_ERR_ARG, "client is NULL");
    pv_volume *v = c->vol;
    HIP_TRY(hipSetDevice(v->ctx->device));
    hipStream_t s = pick(v->ctx, stream);
    const int mc = max_chunks_of(v->P);
    if (!c->ent.out) {
        c->ent.max_chunks = mc;
        // worst case: 12 bits per byte, plus tables and per-chunk padding
        c->ent_cap = 8 + kPacketHeader + (uint64_t)kEntStreams * (132 + 8ull * mc) + c->packet_cap * 3 / 2 + 64;
        PV_TRY(dev_alloc(&c->ent.hist, kEntStreams * 256 * sizeof(uint32_t), "entropy histograms"));
        PV_TRY(dev_alloc(&c->ent.lens, kEntStreams * 256, "code lengths"));
        PV_TRY(dev_alloc(&c->ent.codes, kEntStreams * 256 * sizeof(uint32_t), "codes"));
        PV_TRY(dev_alloc(&c->ent.chunk_bits, (size_t)kEntStreams * mc * sizeof(uint32_t), "chunk bits"));
        PV_TRY(dev_alloc(&c->ent.chunk_off, (size_t)kEntStreams * mc * sizeof(unsigned long long), "chunk offsets"));
        PV_TRY(dev_alloc(&c->ent.total, sizeof(unsigned long long), "container size"));
        PV_TRY(dev_alloc(&c->ent.out, c->ent_cap, "container"));
        if (hipHostMalloc((void **)&c->ent_total_host, sizeof(unsigned long long)) != hipSuccess)
            return fail(PV_ERR_OOM, "pinned container size");
        if (hipHostMalloc((void **)&c->ent_tables_host, kEntStreams * 256 * (4 + 1 + 4)) != hipSuccess)
            return fail(PV_ERR_OOM, "pinned code tables");
    }
    c->ent.pkt = c->packet;
    uint32_t *hist = reinterpret_cast<uint32_t *>(c->ent_tables_host);
    uint8_t *lens = c->ent_tables_host + kEntStreams * 256 * 4;
    uint32_t *codes = reinterpret_cast<uint32_t *>(lens + kEntStreams * 256);
    HIP_TRY(launch_zero(c->ent.hist, kEntStreams * 256 * sizeof(uint32_t), s));
    HIP_TRY(timed(v->ctx, PV_STAGE_ENTROPY, s, [&] { return launch_entropy_hist(c->ent, mc, s); }));
    HIP_TRY(hipMemcpyAsync(hist, c->ent.hist, kEntStreams * 256 * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < kEntStreams; ++k) {
        huffman_lengths(hist + 256 * k, lens + 256 * k);
        canonical_codes_host(lens + 256 * k, codes + 256 * k);
    }
    HIP_TRY(hipMemcpyAsync(c->ent.lens, lens, kEntStreams * 256, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->ent.codes, codes, kEntStreams * 256 * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(timed(v->ctx, PV_STAGE_ENTROPY, s, [&] { return launch_entropy_encode(c->ent, mc, s); }));
    return PV_OK;
}

extern "C" pv_status pv_entropy_download(pv_client *c, void *host, uint64_t cap, uint64_t *bytes, void *stream) {
    if (!c || !bytes) return fail(PV_ERR_ARG, "NULL argument");
    if (!c->ent.out) return fail(PV_ERR_STATE, "no packet has been entropy coded");
    HIP_TRY(hipSetDevice(c->vol->ctx->device));
    hipStream_t s = pick(c->vol->ctx, stream);
    HIP_TRY(hipMemcpyAsync(c->ent_total_host, c->ent.total, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint64_t total = *c->ent_total_host;
    *bytes = total;
    if (!host || cap < total) return fail(PV_ERR_CAPACITY, "container needs " + std::to_string(total) + " bytes");
    HIP_TRY(hipMemcpyAsync(host, c->ent.out, total, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PV_OK;
}

template <typename T>
static pv_status grow(T **p, uint64_t &cap, uint64_t need, const char *what) {
    if (need <= cap) return PV_OK;
    hipFree(*p);
    *p = nullptr;
    cap = 0;
    PV_TRY(dev_alloc(p, need * sizeof(T), what));
    cap = need;
    return PV_OK;
}

extern "C" pv_status pv_receiver_apply_compressed(pv_receiver *r, const void *container, uint64_t bytes, void *stream) {
    if (!r || !container) return fail(PV_ERR_ARG, "NULL argument");
    const uint8_t *in = (const uint8_t *)container;
    if (bytes < 8 + (uint64_t)kPacketHeader) return fail(PV_ERR_ARG, "container shorter than its header");
    if (get_u32(in) != kContainerMagic) return fail(PV_ERR_ARG, "not a compressed probe packet (magic)");
    if (get_u32(in + 4) != 1u) return fail(PV_ERR_UNSUPPORTED, "container version");
    const uint8_t *h = in + 8;
    uint64_t size = 0;
    PV_TRY(check_packet_header(r, h, &size));
    const uint64_t Ki = get_u32(h + 4 * kHdrKIrr), Kv = get_u32(h + 4 * kHdrKVis);
    const uint64_t idx = packet_index_bytes(Ki, Kv);
    // the container's structure, from its tables
    std::vector<EntChunk> chunks;
    std::vector<EntBlock> blocks;
    EntDecode d;
    uint64_t off = 8 + kPacketHeader;
    for (int k = 0; k < kEntStreams; ++k) {
        uint64_t start, n;
        if (k == 0) {
            start = kPacketHeader;
            n = 2 * (Ki + Kv);
        } else if (k <= kIrrPlanes) {
            start = kPacketHeader + idx + (k - 1) * Ki * kIrrPlaneBytes;
            n = Ki * kIrrPlaneBytes;
        } else {
            start = kPacketHeader + idx + kIrrPlanes * Ki * kIrrPlaneBytes + (k - 1 - kIrrPlanes) * Kv * kVisPlaneBytes;
            n = Kv * kVisPlaneBytes;
        }
        const uint64_t nch = (n + kHufChunk - 1) / kHufChunk;
        if (off + 132 + 4 * nch > bytes) return fail(PV_ERR_ARG, "container truncated (tables)");
        d.stream_base[k] = off;
        for (int i = 0; i < 128; ++i)
            if ((in[off + i] & 15) > 12 || (in[off + i] >> 4) > 12) return fail(PV_ERR_ARG, "code length above 12 bits");
        if (get_u32(in + off + 128) != nch) return fail(PV_ERR_ARG, "chunk count does not match the header");
        const uint8_t *bits_tab = in + off + 132;
        off += 132 + 4 * nch;
        for (uint64_t c = 0; c < nch; c += kEntDecodeChunks)
            blocks.push_back(EntBlock{k, (int)(chunks.size() + c), (int)std::min<uint64_t>(kEntDecodeChunks, nch - c)});
        for (uint64_t c = 0; c < nch; ++c) {
            const uint32_t bits = get_u32(bits_tab + 4 * c);
            const uint64_t n_sym = std::min<uint64_t>(kHufChunk, n - c * kHufChunk);
            if (bits < n_sym || bits > 12 * n_sym) return fail(PV_ERR_ARG, "chunk bit count out of range");
            EntChunk e;
            e.stream = k;
            e.n_sym = (int)n_sym;
            e.bits = bits;
            e.in_off = off;
            e.out_off = start + c * kHufChunk;
            chunks.push_back(e);
            off += (bits + 31) / 32 * 4;
        }
    }
    if (off != bytes) return fail(PV_ERR_ARG, "container size does not match its tables");
    HIP_TRY(hipSetDevice(r->ctx->device));
    hipStream_t s = pick(r->ctx, stream);
    if (r->used) {
        HIP_TRY(hipEventSynchronize(r->copied));
        HIP_TRY(hipStreamWaitEvent(s, r->done, 0));
    }
    const uint64_t chunk_bytes = chunks.size() * sizeof(EntChunk);
    const uint64_t block_bytes = blocks.size() * sizeof(EntBlock);
    const uint64_t stage_need = (bytes + 15) / 16 * 16 + (chunk_bytes + 15) / 16 * 16 + block_bytes;
    if (stage_need > r->ent_stage_cap) {
        if (r->ent_stage) hipHostFree(r->ent_stage);
        r->ent_stage = nullptr;
        r->ent_stage_cap = 0;
        if (hipHostMalloc((void **)&r->ent_stage, stage_need) != hipSuccess) return fail(PV_ERR_OOM, "pinned staging");
        r->ent_stage_cap = stage_need;
    }
    PV_TRY(grow(&r->ent_in, r->ent_in_cap, bytes, "container buffer"));
    PV_TRY(grow(&r->ent_chunks, r->ent_chunk_cap, std::max<uint64_t>(chunks.size(), 1), "chunk list"));
    PV_TRY(grow(&r->ent_blocks, r->ent_block_cap, std::max<uint64_t>(blocks.size(), 1), "decode blocks"));
    const uint64_t cpos = (bytes + 15) / 16 * 16, bpos = cpos + (chunk_bytes + 15) / 16 * 16;
    std::memcpy(r->ent_stage, in, bytes);
    if (chunk_bytes) std::memcpy(r->ent_stage + cpos, chunks.data(), chunk_bytes);
    if (block_bytes) std::memcpy(r->ent_stage + bpos, blocks.data(), block_bytes);
    HIP_TRY(hipMemcpyAsync(r->ent_in, r->ent_stage, bytes, hipMemcpyHostToDevice, s));
    if (chunk_bytes) HIP_TRY(hipMemcpyAsync(r->ent_chunks, r->ent_stage + cpos, chunk_bytes, hipMemcpyHostToDevice, s));
    if (block_bytes) HIP_TRY(hipMemcpyAsync(r->ent_blocks, r->ent_stage + bpos, block_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(r->copied, s));
    // the index section's zero padding is not coded: clear its last 16 bytes
    // before the decode writes the entries among them
    if (idx >= 16) HIP_TRY(launch_zero(r->pkt + kPacketHeader + idx - 16, 16, s));
    d.in = r->ent_in;
    d.chunks = r->ent_chunks;
    d.blocks = r->ent_blocks;
    d.n_blocks = (int)blocks.size();
    d.pkt = r->pkt;
    HIP_TRY(timed(r->ctx, PV_STAGE_UNPACK, s, [&] { return launch_entropy_decode(d, s); }));
    return receive_on_device(r, h, s);
}
