// gfx950 kernels of the probe-volume update and the lossless delta pack.
//
//   k_raydirs   spherical-Fibonacci ray set under the frame rotation
//   k_trace     closest hit (BVH, per-lane stack in LDS) + direct shading with
//               a shadow ray; one wavefront = one ray direction x a 4x4x4 brick
//               of probes, so the 64 rays of a wave are parallel and start
//               close together (coherent traversal)
//   k_blend     cosine / cosine^s weighted means over the rays, hysteresis,
//               FP32 or FP16 store, guard bands written by scatter
//   k_pack_*    change mask, ordered compaction, XOR byte planes, reference
//               update, checksum
#include <hip/hip_fp16.h>

#include "internal.h"

namespace pv {

constexpr int kTraceBlock = 128;  // two wavefronts
constexpr int kStack = kStack4;
constexpr int kBlendBlock = 256;
constexpr int kBlendProbes = 4;
constexpr int kBlendChunk = 256;
// A texel whose weight sum is at most this keeps its old value: no ray falls
// usefully inside its lobe. Far above where FP32 weights underflow.
constexpr float kWeightFloor = 1e-20f;

// ---------------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 xyz(float4 a) { return make_float3(a.x, a.y, a.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z), fmaf(a.x, b.y, -a.y * b.x));
}

// XCD-aware block order: the hardware deals consecutive workgroups to the 8
// XCDs in turn; renumber so that each XCD runs one contiguous range of the
// logical work (neighbouring rays share that XCD's L2).
__device__ __forceinline__ int xcd_logical_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// ---------------------------------------------------------------------------
// ray directions
// ---------------------------------------------------------------------------
__device__ void raydir_one(const FrameParams &fp, int n, int i, float4 *dirs) {
    // z evenly spaced in (-1, 1); azimuth steps by the golden angle
    const double z = 1.0 - (2.0 * i + 1.0) / n;
    const double a = (double)i * 0.61803398874989484820;  // frac(i * (phi - 1))
    const double az = 6.28318530717958647692 * (a - floor(a));
    const double rr = sqrt(fmax(0.0, 1.0 - z * z));
    const double sx = rr * cos(az), sy = rr * sin(az);
    const float *R = fp.rot;
    dirs[i] = make_float4((float)(R[0] * sx + R[1] * sy + R[2] * z), (float)(R[3] * sx + R[4] * sy + R[5] * z),
                          (float)(R[6] * sx + R[7] * sy + R[8] * z), 0.f);
}

__global__ void k_raydirs(FrameParams fp, int n, float4 *dirs, int *queue) {
    if (queue && blockIdx.x == 0 && threadIdx.x < 16) queue[threadIdx.x] = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += blockDim.x * gridDim.x) raydir_one(fp, n, i, dirs);
}

__global__ void k_raydirs_batched(const FrameParams *fps, const int *ns, float4 *const *dirs, int n_vols) {
    const int v = blockIdx.x;
    if (v >= n_vols) return;
    const int n = ns[v];
    for (int i = threadIdx.x; i < n; i += blockDim.x) raydir_one(fps[v], n, i, dirs[v]);
}

// ---------------------------------------------------------------------------
// traversal
// ---------------------------------------------------------------------------
struct Ray {
    float3 o, d, inv, oinv;
};

__device__ __forceinline__ Ray make_ray(float3 o, float3 d) {
    Ray r;
    r.o = o;
    r.d = d;
    // keep 1/d finite so the slab products never form inf - inf
    float dx = fabsf(d.x) < 1e-20f ? copysignf(1e-20f, d.x) : d.x;
    float dy = fabsf(d.y) < 1e-20f ? copysignf(1e-20f, d.y) : d.y;
    float dz = fabsf(d.z) < 1e-20f ? copysignf(1e-20f, d.z) : d.z;
    r.inv = make_float3(__builtin_amdgcn_rcpf(dx), __builtin_amdgcn_rcpf(dy), __builtin_amdgcn_rcpf(dz));
    r.oinv = make_float3(o.x * r.inv.x, o.y * r.inv.y, o.z * r.inv.z);
    return r;
}

// Two-sided Moller-Trumbore: true when the ray line crosses the triangle
// (barycentrics inside, det != 0); t receives the distance along the ray.
__device__ __forceinline__ bool tri_cross(const GpuTri &T, const Ray &r, float &t) {
    const float3 e1 = xyz(T.e1), e2 = xyz(T.e2);
    const float3 p = cross3(r.d, e2);
    const float det = dot3(e1, p);
    const float inv = __builtin_amdgcn_rcpf(det);
    const float3 s = r.o - xyz(T.v0);
    const float u = dot3(s, p) * inv;
    const float3 q = cross3(s, e1);
    const float v = dot3(r.d, q) * inv;
    t = dot3(e2, q) * inv;
    // written so that NaN (det == 0) fails every test
    return (u >= 0.f) && (v >= 0.f) && (u + v <= 1.f) && (t == t);
}

__device__ __forceinline__ int tri_id(const GpuTri &T) { return __float_as_int(T.v0.w); }

struct Counts {
    uint32_t nodes, tris;
};

// Per-lane traversal stack in LDS: entry sp of lane 'col' at stk[sp*W + col].
template <int W>
struct Stack {
    int *base;
    __device__ __forceinline__ void push(int &sp, int v) { base[(sp++) * W] = v; }
    __device__ __forceinline__ int pop(int &sp) { return base[(--sp) * W]; }
};

// Four quantized child boxes of a node against [tmin, tmax]. The byte
// coordinates decode as origin + q * 2^e; the slab distance of a plane is
// (origin + q*s - o) / d = q * (s/d) + (origin - o)/d, one FMA per plane.
struct Node4Hits {
    float tn[4];
    bool hit[4];
    int child[4];
    int count[4];
};

__device__ __forceinline__ float ubyte(uint32_t w, int c) { return (float)((w >> (8 * c)) & 0xffu); }

__device__ __forceinline__ void box4(const uint4 w0, const uint4 w1, const uint4 w2, const uint4 w3, const Ray &r,
                                     float tmin, float tmax, Node4Hits &o) {
    const float ax = __uint_as_float((w0.w & 0xffu) << 23) * r.inv.x;
    const float ay = __uint_as_float(((w0.w >> 8) & 0xffu) << 23) * r.inv.y;
    const float az = __uint_as_float(((w0.w >> 16) & 0xffu) << 23) * r.inv.z;
    const float bx = (__uint_as_float(w0.x) - r.o.x) * r.inv.x;
    const float by = (__uint_as_float(w0.y) - r.o.y) * r.inv.y;
    const float bz = (__uint_as_float(w0.z) - r.o.z) * r.inv.z;
    o.child[0] = (int)w3.x;
    o.child[1] = (int)w3.y;
    o.child[2] = (int)w3.z;
    o.child[3] = (int)w3.w;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float x0 = fmaf(ubyte(w1.x, c), ax, bx), x1 = fmaf(ubyte(w1.y, c), ax, bx);
        const float y0 = fmaf(ubyte(w1.z, c), ay, by), y1 = fmaf(ubyte(w1.w, c), ay, by);
        const float z0 = fmaf(ubyte(w2.x, c), az, bz), z1 = fmaf(ubyte(w2.y, c), az, bz);
        const float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), tmin));
        const float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tmax));
        o.tn[c] = tn;
        o.hit[c] = tn <= tf && o.child[c] >= 0;
        o.count[c] = (int)((w2.z >> (8 * c)) & 0xffu);
    }
}

// Orders the hit inner children by entry distance; returns how many.
__device__ __forceinline__ int sort_inner(const Node4Hits &h, int ids[4]) {
    float k[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bool inner = h.hit[c] && h.count[c] == 0;
        k[c] = inner ? h.tn[c] : 3.0e38f;
        ids[c] = h.child[c];
    }
    int m = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) m += (h.hit[c] && h.count[c] == 0) ? 1 : 0;
#define PV_CSWAP(a, b)                                   \
    if (k[b] < k[a]) {                                   \
        const float tk = k[a];                           \
        k[a] = k[b];                                     \
        k[b] = tk;                                       \
        const int ti = ids[a];                           \
        ids[a] = ids[b];                                 \
        ids[b] = ti;                                     \
    }
    PV_CSWAP(0, 1)
    PV_CSWAP(2, 3)
    PV_CSWAP(0, 2)
    PV_CSWAP(1, 3)
    PV_CSWAP(1, 2)
#undef PV_CSWAP
    return m;
}

// LDS copy of the top BVH nodes (dynamic shared memory of the trace kernel).
extern __shared__ uint4 pv_top_nodes[];

// Node fetch: the first 'top' nodes (breadth-first order, so the top levels)
// may be staged in LDS; the rest come from global memory.
struct NodeSrc {
    const uint4 *global;
    int top;
    __device__ __forceinline__ void load(int node, uint4 &w0, uint4 &w1, uint4 &w2, uint4 &w3) const {
        if (node < top) {
            w0 = pv_top_nodes[4 * node];
            w1 = pv_top_nodes[4 * node + 1];
            w2 = pv_top_nodes[4 * node + 2];
            w3 = pv_top_nodes[4 * node + 3];
        } else {
            const uint4 *q = global + 4 * (size_t)node;
            w0 = q[0];
            w1 = q[1];
            w2 = q[2];
            w3 = q[3];
        }
    }
};

__device__ __forceinline__ NodeSrc global_nodes(const DeviceBvh &bvh) {
    return NodeSrc{reinterpret_cast<const uint4 *>(bvh.nodes), 0};
}

// The hit inner children in slot order (any-hit traversal needs no order).
__device__ __forceinline__ int collect_inner(const Node4Hits &h, int ids[4]) {
    int m = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bool inner = h.hit[c] && h.count[c] == 0;
        ids[c] = h.child[c];
        m += inner ? 1 : 0;
    }
    // move the hit inner ones to the front without dynamic indexing
    int out[4] = {-1, -1, -1, -1};
    int w = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bool inner = h.hit[c] && h.count[c] == 0;
        out[0] = (inner && w == 0) ? ids[c] : out[0];
        out[1] = (inner && w == 1) ? ids[c] : out[1];
        out[2] = (inner && w == 2) ? ids[c] : out[2];
        out[3] = (inner && w == 3) ? ids[c] : out[3];
        w += inner ? 1 : 0;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) ids[c] = out[c];
    return m;
}

// The hit leaf children of a node as a mask over its leaf triangle slots:
// the builder stores a node's leaf triangles back to back in slot order, so
// bit i stands for slot base + i, and walking the bits upward tests the
// triangles in the order child 0..3, first..last.
__device__ __forceinline__ uint32_t leaf_mask(const Node4Hits &h, int &base) {
    base = -1;
#pragma unroll
    for (int c = 3; c >= 0; --c) base = h.count[c] > 0 ? h.child[c] : base;
    uint32_t m = 0u;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (h.hit[c] && h.count[c] > 0) m |= ((1u << h.count[c]) - 1u) << (h.child[c] - base);
    return m;
}

// Closest hit in one BVH; updates (tbest, best tri index, best array) when a
// nearer hit is found; equal distances go to the smaller original id.
// Leaves are tested where they are met; hit inner children are visited
// nearest first, the others pushed (the builder bounds the stack).
template <bool COUNT, int W>
__device__ void closest(const DeviceBvh &bvh, const NodeSrc &src, const Ray &r, float tmin, float &tbest, int &best,
                        int &best_id, const GpuTri *&best_arr, Stack<W> stk, Counts &cnt) {
    if (bvh.n_nodes == 0) return;
    int node = 0, sp = 0;
    while (true) {
        Node4Hits h;
        uint4 w0, w1, w2, w3;
        src.load(node, w0, w1, w2, w3);
        box4(w0, w1, w2, w3, r, tmin, tbest, h);
        if (COUNT) cnt.nodes++;
        int base;
        for (uint32_t m = leaf_mask(h, base); m != 0u; m &= m - 1u) {
            const int k = base + __builtin_ctz(m);
            const GpuTri T = bvh.tris[k];
            float t;
            if (COUNT) cnt.tris++;
            if (tri_cross(T, r, t) && t > tmin && (t < tbest || (t == tbest && tri_id(T) < best_id))) {
                tbest = t;
                best = k;
                best_id = tri_id(T);
                best_arr = bvh.tris;
            }
        }
        int ids[4];
        const int m = sort_inner(h, ids);
        if (m > 0) {
            // constant indices keep ids[] in registers
            if (m > 3) stk.push(sp, ids[3]);
            if (m > 2) stk.push(sp, ids[2]);
            if (m > 1) stk.push(sp, ids[1]);
            node = ids[0];
        } else {
            if (sp == 0) break;
            node = stk.pop(sp);
        }
    }
}

// Any hit with tmin < t < tmax in one BVH.
template <bool COUNT, int W>
__device__ bool any_hit(const DeviceBvh &bvh, const NodeSrc &src, const Ray &r, float tmin, float tmax, Stack<W> stk,
                        Counts &cnt) {
    if (bvh.n_nodes == 0) return false;
    int node = 0, sp = 0;
    while (true) {
        Node4Hits h;
        uint4 w0, w1, w2, w3;
        src.load(node, w0, w1, w2, w3);
        box4(w0, w1, w2, w3, r, tmin, tmax, h);
        if (COUNT) cnt.nodes++;
        int base;
        for (uint32_t m = leaf_mask(h, base); m != 0u; m &= m - 1u) {
            float t;
            if (COUNT) cnt.tris++;
            if (tri_cross(bvh.tris[base + __builtin_ctz(m)], r, t) && t > tmin && t < tmax) return true;
        }
        int ids[4];
        const int m = collect_inner(h, ids);
        if (m > 0) {
            // constant indices keep ids[] in registers
            if (m > 3) stk.push(sp, ids[3]);
            if (m > 2) stk.push(sp, ids[2]);
            if (m > 1) stk.push(sp, ids[1]);
            node = ids[0];
        } else {
            if (sp == 0) return false;
            node = stk.pop(sp);
        }
    }
}

// Geometry of a hit: unit normal facing the ray origin and the hit point.
__device__ __forceinline__ void hit_frame(const GpuTri &T, const Ray &ray, float3 o, float t, float3 &nrm,
                                          float3 &xh) {
    nrm = cross3(xyz(T.e1), xyz(T.e2));
    const float il = rsqrtf(dot3(nrm, nrm));
    nrm = make_float3(nrm.x * il, nrm.y * il, nrm.z * il);
    if (dot3(nrm, ray.d) > 0.f) nrm = make_float3(-nrm.x, -nrm.y, -nrm.z);
    xh = make_float3(fmaf(t, ray.d.x, o.x), fmaf(t, ray.d.y, o.y), fmaf(t, ray.d.z, o.z));
}

// Light li at a hit: cosine, squared distance, and the shadow ray from the
// offset point towards the light. Returns false when the light is behind.
__device__ __forceinline__ bool light_setup(const FrameParams &fp, int li, float eps, float3 nrm, float3 xh,
                                            float &cosv, float &d2, float3 &so, float3 &sd, float &smax) {
    const float3 lp = make_float3(fp.light_pos[li][0], fp.light_pos[li][1], fp.light_pos[li][2]);
    const float3 lv = lp - xh;
    d2 = dot3(lv, lv);
    const float dl = sqrtf(d2);
    cosv = dot3(nrm, lv) / dl;
    if (!(cosv > 0.f)) return false;
    so = make_float3(fmaf(eps, nrm.x, xh.x), fmaf(eps, nrm.y, xh.y), fmaf(eps, nrm.z, xh.z));
    sd = lp - so;
    const float slen = sqrtf(dot3(sd, sd));
    const float isl = 1.0f / slen;
    sd = make_float3(sd.x * isl, sd.y * isl, sd.z * isl);
    smax = slen - eps;
    return true;
}

// Adds light li's direct contribution (the light is visible).
__device__ __forceinline__ void light_add(const FrameParams &fp, int li, float4 alb, float cosv, float d2, float3 &L) {
    const float g = cosv / d2 * 0.31830988618379067f;  // 1/pi
    L.x = fmaf(alb.x * fp.light_int[li][0], g, L.x);
    L.y = fmaf(alb.y * fp.light_int[li][1], g, L.y);
    L.z = fmaf(alb.z * fp.light_int[li][2], g, L.z);
}

// Trace and shade the ray of probe (x, y, z), direction j; writes its record.
// SPLIT: instead of tracing shadow rays here, record the hit and append the
// shadow rays to the volume's queue (one atomic per wavefront and light).
template <bool COUNT, int W, bool SPLIT>
__device__ void trace_shade_one(const VolumeParams &vp, const SceneView &sv, const NodeSrc &stat_src,
                                const FrameParams &fp, const float4 *dirs, float4 *rays, int32_t *hits, int x, int y,
                                int z, int j, Stack<W> stk, Counts &cnt, uint32_t &shadow_rays,
                                const SplitBuffers &split) {
    const NodeSrc dyn_src = global_nodes(sv.dyn);
    const float3 o = make_float3(fmaf(vp.sx, (float)x, vp.ox), fmaf(vp.sy, (float)y, vp.oy),
                                 fmaf(vp.sz, (float)z, vp.oz));
    const float4 dj = dirs[j];
    const Ray ray = make_ray(o, xyz(dj));
    float tbest = INFINITY;
    int best = -1, best_id = -1;
    const GpuTri *arr = nullptr;
    closest<COUNT, W>(sv.stat, stat_src, ray, 0.f, tbest, best, best_id, arr, stk, cnt);
    closest<COUNT, W>(sv.dyn, dyn_src, ray, 0.f, tbest, best, best_id, arr, stk, cnt);
    const size_t p = (size_t)x + (size_t)vp.nx * ((size_t)y + (size_t)vp.ny * z);
    const size_t q = p * vp.n + j;
    float3 L;
    float dist;
    float3 nrm, xh;
    float4 alb = make_float4(0.f, 0.f, 0.f, 0.f);
    if (best >= 0) {
        const GpuTri T = arr[best];
        hit_frame(T, ray, o, tbest, nrm, xh);
        alb = sv.mats[2 * best_id];
        const float4 emi = sv.mats[2 * best_id + 1];
        L = make_float3(emi.x, emi.y, emi.z);
        dist = fminf(tbest, vp.max_distance);
    } else {
        L = make_float3(vp.sky[0], vp.sky[1], vp.sky[2]);
        dist = vp.max_distance;
    }
    if (!SPLIT) {
        if (best >= 0) {
            for (int li = 0; li < fp.n_lights; ++li) {
                float cosv, d2, smax;
                float3 so, sd;
                if (!light_setup(fp, li, sv.eps, nrm, xh, cosv, d2, so, sd, smax)) continue;
                const Ray sr = make_ray(so, sd);
                if (COUNT) shadow_rays++;
                bool occ = any_hit<COUNT, W>(sv.stat, stat_src, sr, 0.f, smax, stk, cnt);
                if (!occ) occ = any_hit<COUNT, W>(sv.dyn, dyn_src, sr, 0.f, smax, stk, cnt);
                if (!occ) light_add(fp, li, alb, cosv, d2, L);
            }
        }
    } else {
        split.hitrec[q] = make_int2(best < 0 ? -1 : (best | (arr == sv.dyn.tris ? (int)0x80000000 : 0)),
                                    __float_as_int(tbest));
        split.occ[q] = 0u;
        const int lane = threadIdx.x & 63;
        for (int li = 0; li < fp.n_lights; ++li) {
            float cosv = 0.f, d2 = 0.f, smax = 0.f;
            float3 so = make_float3(0.f, 0.f, 0.f), sd = so;
            const bool need = best >= 0 && light_setup(fp, li, sv.eps, nrm, xh, cosv, d2, so, sd, smax);
            const unsigned long long m = __ballot(need);
            if (m == 0) continue;
            const int leader = __ffsll((long long)m) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(split.count, __popcll(m));
            base = __shfl(base, leader);
            if (need) {
                const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
                split.queue[slot].o_tmax = make_float4(so.x, so.y, so.z, smax);
                split.queue[slot].d_ray = make_float4(sd.x, sd.y, sd.z, __int_as_float((int)(q * 8 + li)));
                if (COUNT) shadow_rays++;
            }
        }
    }
    rays[q] = make_float4(L.x, L.y, L.z, dist);
    if (hits) hits[q] = best_id;
}

struct TraceGrid {
    int bx, by, bz;        // brick shape (64 probes)
    int nbx, nby, nbz;     // bricks per axis
    int n_bricks, n_waves; // n_waves = n_bricks * rays per probe
    int persistent;
    int chunk;             // waves per XCD queue (persistent)
};

// One wavefront = one ray direction j over one brick of probes.
template <bool COUNT, int W, bool SPLIT>
__device__ __forceinline__ void trace_wave(const VolumeParams &vp, const SceneView &sv, const NodeSrc &src,
                                           const FrameParams &fp, const float4 *dirs, float4 *rays, int32_t *hits,
                                           const TraceGrid &g, int w, Stack<W> stk, Counts &cnt, uint32_t &shadow,
                                           const SplitBuffers &split) {
    const int lane = threadIdx.x & 63;
    const int j = w / g.n_bricks, brick = w - j * g.n_bricks;
    const int bxi = brick % g.nbx, byi = (brick / g.nbx) % g.nby, bzi = brick / (g.nbx * g.nby);
    const int x = bxi * g.bx + lane % g.bx;
    const int y = byi * g.by + (lane / g.bx) % g.by;
    const int z = bzi * g.bz + lane / (g.bx * g.by);
    if (x < vp.nx && y < vp.ny && z < vp.nz)
        trace_shade_one<COUNT, W, SPLIT>(vp, sv, src, fp, dirs, rays, hits, x, y, z, j, stk, cnt, shadow, split);
}

template <bool COUNT, int W, int TOP, bool SPLIT>
__global__ __launch_bounds__(W) void k_trace(VolumeParams vp, SceneView sv, FrameParams fp, const float4 *dirs,
                                             float4 *rays, int32_t *hits, unsigned long long *counts, TraceGrid g,
                                             int *queue, SplitBuffers split) {
    __shared__ int stk[kStack * W];
    NodeSrc src = global_nodes(sv.stat);
    if (TOP > 0) {
        const int nt = min(TOP, sv.stat.n_nodes);
        const uint4 *gn = reinterpret_cast<const uint4 *>(sv.stat.nodes);
        for (int i = threadIdx.x; i < nt * 4; i += W) pv_top_nodes[i] = gn[i];
        __syncthreads();
        src.top = nt;
    }
    Stack<W> st{stk + threadIdx.x};
    Counts cnt = {0, 0};
    uint32_t shadow = 0;
    const int w = xcd_logical_block() * (W / 64) + (threadIdx.x >> 6);
    if (w < g.n_waves) trace_wave<COUNT, W, SPLIT>(vp, sv, src, fp, dirs, rays, hits, g, w, st, cnt, shadow, split);
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

template <bool COUNT, int W, int TOP>
__global__ __launch_bounds__(W) void k_trace_refill(VolumeParams vp, SceneView sv, FrameParams fp,
                                                    const float4 *dirs, float4 *rays, int32_t *hits,
                                                    unsigned long long *counts, TraceGrid g, int *queue) {
    __shared__ int stk[kStack * W];
    NodeSrc stat_src = global_nodes(sv.stat);
    if (TOP > 0) {
        const int nt = min(TOP, sv.stat.n_nodes);
        const uint4 *gn = reinterpret_cast<const uint4 *>(sv.stat.nodes);
        for (int i = threadIdx.x; i < nt * 4; i += W) pv_top_nodes[i] = gn[i];
        __syncthreads();
        stat_src.top = nt;
    }
    const uint4 *dyn_nodes = reinterpret_cast<const uint4 *>(sv.dyn.nodes);
    Stack<W> stk_l{stk + threadIdx.x};
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
template <bool COUNT, int W, int TOP>
__global__ __launch_bounds__(W) void k_shadow(SceneView sv, SplitBuffers split, unsigned long long *counts) {
    __shared__ int stk[kStack * W];
    NodeSrc src = global_nodes(sv.stat);
    if (TOP > 0) {
        const int nt = min(TOP, sv.stat.n_nodes);
        const uint4 *gn = reinterpret_cast<const uint4 *>(sv.stat.nodes);
        for (int i = threadIdx.x; i < nt * 4; i += W) pv_top_nodes[i] = gn[i];
        __syncthreads();
        src.top = nt;
    }
    const NodeSrc dyn_src = global_nodes(sv.dyn);
    Stack<W> st{stk + threadIdx.x};
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
            bool occ = any_hit<COUNT, W>(sv.stat, src, sr, 0.f, e.o_tmax.w, st, cnt);
            if (!occ) occ = any_hit<COUNT, W>(sv.dyn, dyn_src, sr, 0.f, e.o_tmax.w, st, cnt);
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

// ---------------------------------------------------------------------------
// blend
// ---------------------------------------------------------------------------
// Centre direction of interior texel (i, j) of an N x N octahedral map.
__device__ __forceinline__ float3 oct_texel_dir(int N, int i, int j) {
    const float u = (2.0f * i + 1.0f) / N - 1.0f;
    const float w = (2.0f * j + 1.0f) / N - 1.0f;
    float x = u, y = w;
    const float zz = 1.0f - fabsf(u) - fabsf(w);
    if (zz < 0.f) {
        x = (1.0f - fabsf(w)) * (u >= 0.f ? 1.f : -1.f);
        y = (1.0f - fabsf(u)) * (w >= 0.f ? 1.f : -1.f);
    }
    const float il = rsqrtf(x * x + y * y + zz * zz);
    return make_float3(x * il, y * il, zz * il);
}

template <int S>
__device__ __forceinline__ float pow_int(float x, int s) {
    if (S == 50) {
        const float x2 = x * x, x4 = x2 * x2, x8 = x4 * x4, x16 = x8 * x8, x32 = x16 * x16;
        return x32 * x16 * x2;
    }
    float r = 1.f, b = x;
    for (int e = s; e > 0; e >>= 1) {
        if (e & 1) r *= b;
        b *= b;
    }
    return r;
}

template <typename T>
__device__ __forceinline__ float load_map(const T *p);
template <>
__device__ __forceinline__ float load_map<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float load_map<__half>(const __half *p) { return __half2float(*p); }

template <typename T>
__device__ __forceinline__ T to_map(float v);
template <>
__device__ __forceinline__ float to_map<float>(float v) { return v; }
template <>
__device__ __forceinline__ __half to_map<__half>(float v) { return __float2half_rn(v); }

// Store interior texel (i, j) of an N x N map into its (N+2)^2 tile together
// with every guard texel that replicates it. Across an edge the octahedral
// square continues mirrored, so a texel on the top row also lands on the
// top guard row at the mirrored column, and so on; the four corner guard
// texels replicate the diagonally opposite interior corner.
template <typename T>
__device__ __forceinline__ void store_with_guard(T *tile, int N, int i, int j, T v) {
    const int S = N + 2;
    tile[(j + 1) * S + (i + 1)] = v;
    if (j == 0) tile[0 * S + (N - i)] = v;
    if (j == N - 1) tile[(N + 1) * S + (N - i)] = v;
    if (i == 0) tile[(N - j) * S + 0] = v;
    if (i == N - 1) tile[(N - j) * S + (N + 1)] = v;
    if (i == N - 1 && j == N - 1) tile[0] = v;
    if (i == 0 && j == N - 1) tile[N + 1] = v;
    if (i == N - 1 && j == 0) tile[(N + 1) * S] = v;
    if (i == 0 && j == 0) tile[(N + 1) * S + (N + 1)] = v;
}

struct BlendSmem {
    float4 sd[kBlendChunk];
    float4 sL[kBlendProbes][kBlendChunk];
    float2 sR[kBlendProbes][kBlendChunk];
};

// One block: Q probes (Q = 1, 2 or 4); thread t owns visibility texel t of
// all Q probes and irradiance texel (t mod 64) of probe t/64 (threads with
// t/64 >= Q skip the irradiance). Each sum runs over the rays in the same
// order whatever Q is, so every Q gives identical bits.
template <typename T, int S, int Q = kBlendProbes>
__device__ void blend_group(const VolumeParams &vp, const float4 *dirs, const float4 *rays, T *irr, T *vis,
                            float h, int p0, BlendSmem &sm) {
    float4 *sd = sm.sd;
    float4 (*sL)[kBlendChunk] = sm.sL;
    float2 (*sR)[kBlendChunk] = sm.sR;
    const int tid = threadIdx.x;
    const int n = vp.n, P = vp.P;
    const float3 wv = oct_texel_dir(16, tid & 15, tid >> 4);
    const int ti = tid & 63, qi = tid >> 6;
    const float3 wi = oct_texel_dir(8, ti & 7, ti >> 3);
    float sv = 0.f, a1[kBlendProbes], a2[kBlendProbes];
#pragma unroll
    for (int q = 0; q < kBlendProbes; ++q) a1[q] = a2[q] = 0.f;
    float sw = 0.f, ar = 0.f, ag = 0.f, ab = 0.f;
    for (int j0 = 0; j0 < n; j0 += kBlendChunk) {
        const int m = min(kBlendChunk, n - j0);
        __syncthreads();
        for (int k = tid; k < m; k += kBlendBlock) sd[k] = dirs[j0 + k];
        for (int k = tid; k < Q * m; k += kBlendBlock) {
            const int q = k / m, jj = k - q * m, p = p0 + q;
            const float4 rec = p < P ? rays[(size_t)p * n + j0 + jj] : make_float4(0.f, 0.f, 0.f, 0.f);
            sL[q][jj] = rec;
            sR[q][jj] = make_float2(rec.w, rec.w * rec.w);
        }
        __syncthreads();
        for (int jj = 0; jj < m; ++jj) {
            const float3 d = xyz(sd[jj]);
            const float cv = fmaxf(dot3(wv, d), 0.f);
            const float v = pow_int<S>(cv, vp.vis_sharpness);
            sv += v;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const float2 rr = sR[q][jj];
                a1[q] = fmaf(v, rr.x, a1[q]);
                a2[q] = fmaf(v, rr.y, a2[q]);
            }
            const float ci = fmaxf(dot3(wi, d), 0.f);
            const float4 L = sL[qi < Q ? qi : 0][jj];
            sw += ci;
            ar = fmaf(ci, L.x, ar);
            ag = fmaf(ci, L.y, ag);
            ab = fmaf(ci, L.z, ab);
        }
    }
    const float g = 1.0f - h;
    // visibility: 2 channels, 18x18 tiles
    if (sv > kWeightFloor) {
        const float isv = 1.0f / sv;
        const int i = tid & 15, jr = tid >> 4;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int p = p0 + q;
            if (p >= P) break;
            T *base = vis + (size_t)p * 2 * 324;
            const float est[2] = {a1[q] * isv, a2[q] * isv};
            for (int c = 0; c < 2; ++c) {
                T *tile = base + c * 324;
                float nv = est[c];
                if (h > 0.f) nv = fmaf(h, load_map<T>(tile + (jr + 1) * 18 + (i + 1)), g * est[c]);
                store_with_guard<T>(tile, 16, i, jr, to_map<T>(nv));
            }
        }
    }
    // irradiance: 3 channels, 10x10 tiles
    const int p = p0 + qi;
    if (qi < Q && p < P && sw > kWeightFloor) {
        const float isw = 1.0f / sw;
        const int i = ti & 7, jr = ti >> 3;
        T *base = irr + (size_t)p * 3 * 100;
        const float est[3] = {ar * isw, ag * isw, ab * isw};
        for (int c = 0; c < 3; ++c) {
            T *tile = base + c * 100;
            float nv = est[c];
            if (h > 0.f) nv = fmaf(h, load_map<T>(tile + (jr + 1) * 10 + (i + 1)), g * est[c]);
            store_with_guard<T>(tile, 8, i, jr, to_map<T>(nv));
        }
    }
}

template <typename T, int S, int Q>
__global__ __launch_bounds__(kBlendBlock) void k_blend(VolumeParams vp, const float4 *dirs, const float4 *rays,
                                                      T *irr, T *vis, float h) {
    __shared__ BlendSmem sm;
    const int p0 = xcd_logical_block() * Q;
    if (p0 >= vp.P) return;
    blend_group<T, S, Q>(vp, dirs, rays, irr, vis, h, p0, sm);
}

// ---------------------------------------------------------------------------
// batched persistent launch
// ---------------------------------------------------------------------------
// Work queue over all volumes: first every trace item (4 waves), then every
// blend group (4 probes). A blend group of volume v waits until all
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
        const int item = item_s;
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
                    trace_shade_one<false, kBatchBlock, false>(bv.vp, bv.sv, global_nodes(bv.sv.stat), frames[v],
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
            const int p0 = (g - bv.first_blend) * kBlendProbes;
            if (bv.fp16) {
                if (bv.vp.vis_sharpness == 50)
                    blend_group<__half, 50>(bv.vp, bv.dirs, bv.rays, (__half *)bv.irr, (__half *)bv.vis, bv.h, p0,
                                            sm.blend);
                else
                    blend_group<__half, 0>(bv.vp, bv.dirs, bv.rays, (__half *)bv.irr, (__half *)bv.vis, bv.h, p0,
                                           sm.blend);
            } else {
                if (bv.vp.vis_sharpness == 50)
                    blend_group<float, 50>(bv.vp, bv.dirs, bv.rays, (float *)bv.irr, (float *)bv.vis, bv.h, p0,
                                           sm.blend);
                else
                    blend_group<float, 0>(bv.vp, bv.dirs, bv.rays, (float *)bv.irr, (float *)bv.vis, bv.h, p0,
                                          sm.blend);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// pack
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ uint32_t word_hash(uint32_t w, uint32_t word_index) {
    return fmix32(w ^ (word_index * 0x9E3779B9u));
}

__device__ __forceinline__ bool texel_changed(uint16_t a, uint16_t b, float tau) {
    if (tau == 0.f) return a != b;
    // binary16 values are exact in double and so is their difference
    const double da = (double)__half2float(__ushort_as_half(a));
    const double db = (double)__half2float(__ushort_as_half(b));
    return fabs(da - db) > (double)tau;
}

// The pack works on tiles of kPackQ consecutive probes. Their FP16 tiles are
// contiguous in HBM (600 B and 1,296 B per probe) and start on 16-byte
// boundaries (kPackQ * 600 and kPackQ * 1,296 are multiples of 16), so a block
// stages them into LDS with aligned 16-byte loads (map allocations carry 256
// bytes of slack, so the last vector of a ragged tail stays in bounds). Work
// is then split into row units of 8 interior texels of one channel:
// irradiance 3 x 8 rows per probe, visibility 2 x 16 rows x 2 halves.
constexpr int kPackQ = 16;
constexpr int kPackThreads = 256;
constexpr int kIrrUnits = 3 * 8;       // per probe
constexpr int kVisUnits = 2 * 16 * 2;  // per probe

struct PackSmem {
    uint4 irr[kPackQ * 600 / 16];
    uint4 vis[kPackQ * 1296 / 16];
    int changed[kPackQ][2];
    uint32_t part[kPackThreads / 64];
};

__device__ __forceinline__ void stage_tiles(const PackBuffers &b, int p0, int P, PackSmem &sm) {
    const int n = min(kPackQ, P - p0);
    const uint4 *gi = reinterpret_cast<const uint4 *>(b.cur_irr + (size_t)p0 * 300);
    const uint4 *gv = reinterpret_cast<const uint4 *>(b.cur_vis + (size_t)p0 * 648);
    const int vi = (n * 600 + 15) / 16, vv = (n * 1296 + 15) / 16;
    for (int i = threadIdx.x; i < vi; i += kPackThreads) sm.irr[i] = gi[i];
    for (int i = threadIdx.x; i < vv; i += kPackThreads) sm.vis[i] = gv[i];
}

// Unit u of the tile (irradiance units first): probe q, texture (0 irr,
// 1 vis), channel c, first interior texel t0 (multiple of 8).
struct Unit {
    int q, tex, c, t0, N;
};

__device__ __forceinline__ Unit unit_of(int u) {
    Unit r;
    if (u < kPackQ * kIrrUnits) {
        r.q = u / kIrrUnits;
        const int w = u - r.q * kIrrUnits;
        r.tex = 0;
        r.c = w / 8;
        r.t0 = (w % 8) * 8;
        r.N = 8;
    } else {
        const int v = u - kPackQ * kIrrUnits;
        r.q = v / kVisUnits;
        const int w = v - r.q * kVisUnits;
        r.tex = 1;
        r.c = w / 32;
        r.t0 = (w % 32) * 8;
        r.N = 16;
    }
    return r;
}

// The 8 current texels of a unit from the staged tiles.
__device__ __forceinline__ void unit_cur(const PackSmem &sm, const Unit &u, uint16_t cur[8]) {
    const uint16_t *base = u.tex == 0 ? reinterpret_cast<const uint16_t *>(sm.irr) + u.q * 300 + u.c * 100
                                      : reinterpret_cast<const uint16_t *>(sm.vis) + u.q * 648 + u.c * 324;
    const int S = u.N + 2, row = u.t0 / u.N, col = u.t0 - row * u.N;
    const uint16_t *src = base + (row + 1) * S + col + 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) cur[i] = src[i];
}

__device__ __forceinline__ uint16_t *unit_ref(const PackBuffers &b, int p, const Unit &u) {
    return u.tex == 0 ? b.ref_irr + (size_t)p * 192 + u.c * 64 + u.t0 : b.ref_vis + (size_t)p * 512 + u.c * 256 + u.t0;
}

__device__ __forceinline__ void unpack8(uint4 v, uint16_t r[8]) {
    r[0] = v.x & 0xffff;
    r[1] = v.x >> 16;
    r[2] = v.y & 0xffff;
    r[3] = v.y >> 16;
    r[4] = v.z & 0xffff;
    r[5] = v.z >> 16;
    r[6] = v.w & 0xffff;
    r[7] = v.w >> 16;
}

// Change mask of every probe: any interior texel differs (tau = 0) or
// |cur - ref| > tau.
__global__ __launch_bounds__(kPackThreads) void k_pack_mask(PackBuffers b, int P, float tau_irr, float tau_vis) {
    __shared__ PackSmem sm;
    const int p0 = blockIdx.x * kPackQ;
    if (p0 >= P) return;
    if (threadIdx.x < kPackQ * 2) sm.changed[threadIdx.x >> 1][threadIdx.x & 1] = 0;
    stage_tiles(b, p0, P, sm);
    __syncthreads();
    const int n = min(kPackQ, P - p0);
    const int units = kPackQ * (kIrrUnits + kVisUnits);
    for (int u = threadIdx.x; u < units; u += kPackThreads) {
        const Unit un = unit_of(u);
        if (un.q >= n) continue;
        uint16_t cur[8], ref[8];
        unit_cur(sm, un, cur);
        unpack8(*reinterpret_cast<const uint4 *>(unit_ref(b, p0 + un.q, un)), ref);
        const float tau = un.tex == 0 ? tau_irr : tau_vis;
        bool ch = false;
#pragma unroll
        for (int i = 0; i < 8; ++i) ch |= texel_changed(cur[i], ref[i], tau);
        if (ch) atomicOr(&sm.changed[un.q][un.tex], 1);
    }
    __syncthreads();
    if (threadIdx.x < n) {
        b.mask_irr[p0 + threadIdx.x] = (uint8_t)sm.changed[threadIdx.x][0];
        b.mask_vis[p0 + threadIdx.x] = (uint8_t)sm.changed[threadIdx.x][1];
    }
}

constexpr int kScanBlock = 1024;

// Inclusive scans across the block with wavefront shuffles and one LDS step.
__device__ __forceinline__ void block_scan2(int &a, int &m, int *sh_a, int *sh_m, int &total_a) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int ya = __shfl_up(a, off), ym = __shfl_up(m, off);
        if (lane >= off) {
            a += ya;
            m = max(m, ym);
        }
    }
    if (lane == 63) {
        sh_a[wv] = a;
        sh_m[wv] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kScanBlock / 64; ++w) {
            sh_a[w] += sh_a[w - 1];
            sh_m[w] = max(sh_m[w], sh_m[w - 1]);
        }
    }
    __syncthreads();
    if (wv > 0) {
        a += sh_a[wv - 1];
        m = max(m, sh_m[wv - 1]);
    }
    total_a = sh_a[kScanBlock / 64 - 1];
    __syncthreads();
}

// One block: ordered ranks of the changed probes, delta-coded index buffers,
// the header, and the checksum share of the index section.
__global__ __launch_bounds__(kScanBlock) void k_pack_scan(PackBuffers b, int P, uint32_t client, uint32_t seq) {
    __shared__ int sh_a[kScanBlock / 64], sh_m[kScanBlock / 64];
    __shared__ uint32_t shu[kScanBlock / 64];
    const int tid = threadIdx.x;
    // per-thread ranges of a multiple of 16 probes, read as 16-byte vectors
    // (mask arrays are padded to 65,536 zero bytes)
    const int per = 16 * ((P + kScanBlock * 16 - 1) / (kScanBlock * 16));
    const int lo = min(P, tid * per), hi = min(P, lo + per);
    int ki = 0, kv = 0, last_i = -1, last_v = -1;
    for (int p = lo; p < hi; p += 16) {
        const uint4 mi = *reinterpret_cast<const uint4 *>(b.mask_irr + p);
        const uint4 mv = *reinterpret_cast<const uint4 *>(b.mask_vis + p);
        const uint32_t wi[4] = {mi.x, mi.y, mi.z, mi.w}, wv[4] = {mv.x, mv.y, mv.z, mv.w};
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const bool ci = (wi[i >> 2] >> (8 * (i & 3))) & 0xffu, cv = (wv[i >> 2] >> (8 * (i & 3))) & 0xffu;
            if (ci && p + i < hi) {
                ++ki;
                last_i = p + i;
            }
            if (cv && p + i < hi) {
                ++kv;
                last_v = p + i;
            }
        }
    }
    // inclusive scans; exclusive values are the inclusive ones minus this thread's
    int ai = ki, mi = last_i, av = kv, mv = last_v, K_irr, K_vis;
    block_scan2(ai, mi, sh_a, sh_m, K_irr);
    block_scan2(av, mv, sh_a, sh_m, K_vis);
    // exclusive max: the previous threads' last changed probe
    int prev_i = __shfl_up(mi, 1), prev_v = __shfl_up(mv, 1);
    __shared__ int wlast_i[kScanBlock / 64], wlast_v[kScanBlock / 64];
    if ((tid & 63) == 63) {
        wlast_i[tid >> 6] = mi;
        wlast_v[tid >> 6] = mv;
    }
    __syncthreads();
    if ((tid & 63) == 0) {
        prev_i = (tid >> 6) > 0 ? wlast_i[(tid >> 6) - 1] : -1;
        prev_v = (tid >> 6) > 0 ? wlast_v[(tid >> 6) - 1] : -1;
    }
    uint8_t *pk = b.packet;
    uint16_t *idx_i = reinterpret_cast<uint16_t *>(pk + 32);
    uint16_t *idx_v = idx_i + K_irr;
    int k_i = ai - ki, k_v = av - kv;
    for (int p0 = lo; p0 < hi; p0 += 16) {
        const uint4 mi = *reinterpret_cast<const uint4 *>(b.mask_irr + p0);
        const uint4 mv = *reinterpret_cast<const uint4 *>(b.mask_vis + p0);
        const uint32_t wi[4] = {mi.x, mi.y, mi.z, mi.w}, wv[4] = {mv.x, mv.y, mv.z, mv.w};
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int p = p0 + i;
            if (p >= hi) break;
            if ((wi[i >> 2] >> (8 * (i & 3))) & 0xffu) {
                b.rank_irr[p] = k_i;
                idx_i[k_i] = (uint16_t)(k_i == 0 ? p : p - prev_i);
                prev_i = p;
                ++k_i;
            }
            if ((wv[i >> 2] >> (8 * (i & 3))) & 0xffu) {
                b.rank_vis[p] = k_v;
                idx_v[k_v] = (uint16_t)(k_v == 0 ? p : p - prev_v);
                prev_v = p;
                ++k_v;
            }
        }
    }
    const int idx_bytes = ((2 * (K_irr + K_vis) + 15) / 16) * 16;
    if (tid < 16) {  // zero the padding after the entries
        const int pos = 2 * (K_irr + K_vis) + tid;
        if (pos < idx_bytes) pk[32 + pos] = 0;
    }
    __syncthreads();
    // checksum of the index section (payload words 0 .. idx_bytes/4 - 1)
    uint32_t part = 0;
    const uint32_t *words = reinterpret_cast<const uint32_t *>(pk + 32);
    for (int wi = tid; wi < idx_bytes / 4; wi += kScanBlock) part += word_hash(words[wi], (uint32_t)wi);
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((tid & 63) == 0) shu[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) {
        uint32_t sum = 0;
        for (int k = 0; k < kScanBlock / 64; ++k) sum += shu[k];
        uint32_t *h = reinterpret_cast<uint32_t *>(pk);
        h[0] = 0x4B505650u;
        h[1] = 1u | (32u << 16);
        h[2] = client;
        h[3] = seq;
        h[4] = (uint32_t)P;
        h[5] = (uint32_t)K_irr;
        h[6] = (uint32_t)K_vis;
        h[7] = sum;
    }
}

// XOR byte planes of the sent probes, reference update, checksum share.
__global__ __launch_bounds__(kPackThreads) void k_pack_compact(PackBuffers b, int P) {
    __shared__ PackSmem sm;
    const int p0 = blockIdx.x * kPackQ;
    if (p0 >= P) return;
    const int n = min(kPackQ, P - p0);
    // skip the tile when none of its probes is sent (uniform per block)
    bool any = false;
    for (int q = 0; q < n; ++q) any |= (b.mask_irr[p0 + q] | b.mask_vis[p0 + q]) != 0;
    if (!any) return;
    stage_tiles(b, p0, P, sm);
    __syncthreads();
    const uint32_t *h = reinterpret_cast<const uint32_t *>(b.packet);
    const int K_irr = (int)h[5], K_vis = (int)h[6];
    const int idx_bytes = ((2 * (K_irr + K_vis) + 15) / 16) * 16;
    uint8_t *planes_i = b.packet + 32 + idx_bytes;
    uint8_t *planes_v = planes_i + (size_t)K_irr * 6 * 64;
    uint32_t part = 0;
    const int units = kPackQ * (kIrrUnits + kVisUnits);
    for (int u = threadIdx.x; u < units; u += kPackThreads) {
        const Unit un = unit_of(u);
        if (un.q >= n) continue;
        const int p = p0 + un.q;
        if (!(un.tex == 0 ? b.mask_irr[p] : b.mask_vis[p])) continue;
        uint16_t cur[8], ref[8];
        unit_cur(sm, un, cur);
        uint16_t *rp = unit_ref(b, p, un);
        unpack8(*reinterpret_cast<const uint4 *>(rp), ref);
        uint32_t lo[2] = {0, 0}, hi[2] = {0, 0};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint16_t x = cur[i] ^ ref[i];
            lo[i >> 2] |= (uint32_t)(x & 0xff) << (8 * (i & 3));
            hi[i >> 2] |= (uint32_t)(x >> 8) << (8 * (i & 3));
        }
        const int K = un.tex == 0 ? K_irr : K_vis;
        const int k = un.tex == 0 ? (int)b.rank_irr[p] : (int)b.rank_vis[p];
        const size_t NN = (size_t)un.N * un.N, plane_bytes = (size_t)K * NN;
        uint8_t *dlo = (un.tex == 0 ? planes_i : planes_v) + (size_t)(2 * un.c) * plane_bytes + (size_t)k * NN + un.t0;
        uint8_t *dhi = dlo + plane_bytes;
        *reinterpret_cast<uint2 *>(dlo) = make_uint2(lo[0], lo[1]);
        *reinterpret_cast<uint2 *>(dhi) = make_uint2(hi[0], hi[1]);
        *reinterpret_cast<uint4 *>(rp) =
            make_uint4((uint32_t)cur[0] | ((uint32_t)cur[1] << 16), (uint32_t)cur[2] | ((uint32_t)cur[3] << 16),
                       (uint32_t)cur[4] | ((uint32_t)cur[5] << 16), (uint32_t)cur[6] | ((uint32_t)cur[7] << 16));
        const uint32_t wlo = (uint32_t)((dlo - (b.packet + 32)) >> 2), whi = (uint32_t)((dhi - (b.packet + 32)) >> 2);
        part += word_hash(lo[0], wlo) + word_hash(lo[1], wlo + 1) + word_hash(hi[0], whi) + word_hash(hi[1], whi + 1);
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((threadIdx.x & 63) == 0) sm.part[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kPackThreads / 64; ++w) s += sm.part[w];
        atomicAdd(reinterpret_cast<uint32_t *>(b.packet) + 7, s);
    }
}

__global__ void k_zero(uint32_t *p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)blockDim.x * gridDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_raydirs(const FrameParams &fp, int n, float4 *dirs, int *queue, hipStream_t s) {
    hipLaunchKernelGGL(k_raydirs, dim3((n + 255) / 256), dim3(256), 0, s, fp, n, dirs, queue);
    return hipGetLastError();
}

hipError_t launch_raydirs_batched(const FrameParams *frames_dev, const int *ns_dev, float4 *const *dirs_dev,
                                  int n_vols, hipStream_t s) {
    hipLaunchKernelGGL(k_raydirs_batched, dim3(n_vols), dim3(256), 0, s, frames_dev, ns_dev, dirs_dev, n_vols);
    return hipGetLastError();
}

template <bool COUNT, int W, int TOP, bool SPLIT>
static hipError_t launch_trace_t(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp,
                                 const float4 *dirs, float4 *rays, int32_t *hits, unsigned long long *counts,
                                 const TraceGrid &g, int *queue, const SplitBuffers &split, hipStream_t s) {
    const size_t smem = (size_t)TOP * sizeof(GpuNode4);
    if (g.persistent && !SPLIT) {
        // as many waves as fit on the device at once; each deals itself rays
        int dev = 0, cus = 256, per_cu = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_refill<COUNT, W, TOP>, W, smem);
        const long long need = ((long long)g.n_waves * 64 + W - 1) / W;
        const unsigned blocks =
            (unsigned)std::max(1ll, std::min<long long>((long long)cus * std::max(per_cu, 1), need));
        hipLaunchKernelGGL((k_trace_refill<COUNT, W, TOP>), dim3(blocks), dim3(W), smem, s, vp, sv, fp, dirs, rays,
                           hits, counts, g, queue);
        return hipGetLastError();
    }
    const unsigned blocks = (unsigned)(((long long)g.n_waves * 64 + W - 1) / W);
    hipLaunchKernelGGL((k_trace<COUNT, W, TOP, SPLIT>), dim3(blocks), dim3(W), smem, s, vp, sv, fp, dirs, rays, hits,
                       counts, g, queue, split);
    return hipGetLastError();
}

template <bool COUNT, bool SPLIT>
static hipError_t launch_trace_c(const VolumeParams &vp, const SceneView &sv, const FrameParams &fp,
                                 const float4 *dirs, float4 *rays, int32_t *hits, unsigned long long *counts,
                                 const TraceConfig &tc, const TraceGrid &g, int *queue, const SplitBuffers &split,
                                 hipStream_t s) {
#define PV_TRACE_CASE(Wv, Tv)                                                                                   \
    if (tc.block == Wv && tc.top_nodes == Tv)                                                                  \
        return launch_trace_t<COUNT, Wv, Tv, SPLIT>(vp, sv, fp, dirs, rays, hits, counts, g, queue, split, s);
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

template <bool COUNT, int W, int TOP>
static hipError_t launch_shadow_t(const SceneView &sv, const SplitBuffers &split, unsigned long long *counts,
                                  hipStream_t s) {
    int dev = 0, cus = 256, per_cu = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_shadow<COUNT, W, TOP>, W,
                                                       (size_t)TOP * sizeof(GpuNode4));
    const long long cap_blocks = (split.capacity + W - 1) / W;
    const unsigned blocks = (unsigned)std::max(1ll, std::min<long long>((long long)cus * std::max(per_cu, 1), cap_blocks));
    hipLaunchKernelGGL((k_shadow<COUNT, W, TOP>), dim3(blocks), dim3(W), (size_t)TOP * sizeof(GpuNode4), s, sv, split,
                       counts);
    return hipGetLastError();
}

hipError_t launch_shadow(const SceneView &sv, const SplitBuffers &split, const TraceConfig &tc,
                         unsigned long long *counts, hipStream_t s) {
#define PV_SHADOW_CASE(Wv, Tv)                                                           \
    if (tc.block == Wv && tc.top_nodes == Tv)                                            \
        return counts ? launch_shadow_t<true, Wv, Tv>(sv, split, counts, s)              \
                      : launch_shadow_t<false, Wv, Tv>(sv, split, counts, s);
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

template <typename T, int S>
static hipError_t launch_blend_t(const VolumeParams &vp, const float4 *dirs, const float4 *rays, void *irr, void *vis,
                                 float h, hipStream_t s) {
    // probes per block: enough blocks to give every CU several
    const int Q = vp.P >= 4096 ? 4 : (vp.P >= 2048 ? 2 : 1);
#define PV_BLEND_Q(Qv)                                                                                      \
    if (Q == Qv) {                                                                                         \
        hipLaunchKernelGGL((k_blend<T, S, Qv>), dim3((vp.P + Qv - 1) / Qv), dim3(kBlendBlock), 0, s, vp, dirs, \
                           rays, (T *)irr, (T *)vis, h);                                                   \
        return hipGetLastError();                                                                          \
    }
    PV_BLEND_Q(4)
    PV_BLEND_Q(2)
    PV_BLEND_Q(1)
#undef PV_BLEND_Q
    return hipErrorInvalidValue;
}

hipError_t launch_blend(const VolumeParams &vp, const float4 *dirs, const float4 *rays, void *irr, void *vis,
                        int fp16, float h, hipStream_t s) {
    const bool s50 = vp.vis_sharpness == 50;
    if (fp16) return s50 ? launch_blend_t<__half, 50>(vp, dirs, rays, irr, vis, h, s)
                         : launch_blend_t<__half, 0>(vp, dirs, rays, irr, vis, h, s);
    return s50 ? launch_blend_t<float, 50>(vp, dirs, rays, irr, vis, h, s)
               : launch_blend_t<float, 0>(vp, dirs, rays, irr, vis, h, s);
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

hipError_t launch_pack_mask(const PackBuffers &b, int P, float tau_irr, float tau_vis, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_mask, dim3((P + kPackQ - 1) / kPackQ), dim3(kPackThreads), 0, s, b, P, tau_irr, tau_vis);
    return hipGetLastError();
}

hipError_t launch_pack_scan(const PackBuffers &b, int P, uint32_t client, uint32_t seq, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_scan, dim3(1), dim3(kScanBlock), 0, s, b, P, client, seq);
    return hipGetLastError();
}

hipError_t launch_pack_compact(const PackBuffers &b, int P, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_compact, dim3((P + kPackQ - 1) / kPackQ), dim3(kPackThreads), 0, s, b, P);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p, words);
    return hipGetLastError();
}

}  // namespace pv
