// Ray traversal and direct shading, device side: quantized 4-wide BVH
// nodes, Moller-Trumbore triangles, per-lane LDS stack, closest / any hit,
// and the shading of one probe ray (emission, point lights with shadow rays,
// sky). Used by the trace kernels and by the batched kernel.
#pragma once

#include "device_common.h"

namespace pv {

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

// Node indices of both BVHs fit the 16-bit stack entries.
inline bool stack_fits_u16(const SceneView &sv) { return sv.stat.n_nodes <= 65536 && sv.dyn.n_nodes <= 65536; }

struct Counts {
    uint32_t nodes, tris;
};

// Per-lane traversal stack in LDS: entry sp of lane 'col' at stk[sp*W + col].
// E = uint16_t halves the LDS when every BVH of the scene has at most 65536
// nodes (more waves fit on a CU); E = int otherwise.
template <int W, typename E = int>
struct Stack {
    E *base;
    __device__ __forceinline__ void push(int &sp, int v) { base[(sp++) * W] = (E)v; }
    __device__ __forceinline__ int pop(int &sp) { return (int)base[(--sp) * W]; }
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
template <bool COUNT, class STK>
__device__ void closest(const DeviceBvh &bvh, const NodeSrc &src, const Ray &r, float tmin, float &tbest, int &best,
                        int &best_id, const GpuTri *&best_arr, STK stk, Counts &cnt) {
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
template <bool COUNT, class STK>
__device__ bool any_hit(const DeviceBvh &bvh, const NodeSrc &src, const Ray &r, float tmin, float tmax, STK stk,
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
template <bool COUNT, bool SPLIT, class STK>
__device__ void trace_shade_one(const VolumeParams &vp, const SceneView &sv, const NodeSrc &stat_src,
                                const FrameParams &fp, const float4 *dirs, float4 *rays, int32_t *hits, int x, int y,
                                int z, int j, STK stk, Counts &cnt, uint32_t &shadow_rays,
                                const SplitBuffers &split) {
    const NodeSrc dyn_src = global_nodes(sv.dyn);
    const float3 o = make_float3(fmaf(vp.sx, (float)x, vp.ox), fmaf(vp.sy, (float)y, vp.oy),
                                 fmaf(vp.sz, (float)z, vp.oz));
    const float4 dj = dirs[j];
    const Ray ray = make_ray(o, xyz(dj));
    float tbest = INFINITY;
    int best = -1, best_id = -1;
    const GpuTri *arr = nullptr;
    closest<COUNT>(sv.stat, stat_src, ray, 0.f, tbest, best, best_id, arr, stk, cnt);
    closest<COUNT>(sv.dyn, dyn_src, ray, 0.f, tbest, best, best_id, arr, stk, cnt);
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
                bool occ = any_hit<COUNT>(sv.stat, stat_src, sr, 0.f, smax, stk, cnt);
                if (!occ) occ = any_hit<COUNT>(sv.dyn, dyn_src, sr, 0.f, smax, stk, cnt);
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

}  // namespace pv
