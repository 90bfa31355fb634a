// Ray traversal and direct shading, device side: quantized 4-wide BVH
// nodes, watertight triangle tests, per-lane LDS stack, closest / any hit,
// and the shading of one probe ray (emission, point lights with shadow rays,
// sky). Used by the trace kernels and by the batched kernel.
#pragma once

#include "device_common.h"

namespace pv {

// ---------------------------------------------------------------------------
// traversal
// ---------------------------------------------------------------------------
struct Ray {
    float3 o, d, inv;
    // The ray's shear (Woop, Benthin and Wald 2013, "Watertight ray/triangle
    // intersection"): kz is the axis of the largest |d| and (kx, ky, kz) the
    // cyclic order ending in it; a point p relative to the origin maps to
    // (p_kx - sx p_kz, p_ky - sy p_kz, sz p_kz) with sx = d_kx / d_kz,
    // sy = d_ky / d_kz, sz = 1 / d_kz: the ray becomes the +z axis and the
    // third coordinate the ray parameter.
    float3 shear;  // sx, sy, sz
    int kz;
};

// Per-lane choice between a and b as one bitfield insert (no branch).
__device__ __forceinline__ float pick(bool c, float a, float b) {
    const uint32_t m = c ? 0xffffffffu : 0u;
    return __uint_as_float((m & __float_as_uint(a)) | (~m & __float_as_uint(b)));
}

// v with its axes rotated cyclically so that axis kz comes last; K = 0, 1, 2
// is that axis known at compile time, K = -1 takes it from kz.
template <int K = -1>
__device__ __forceinline__ float3 rotate_to_z(float3 v, int kz) {
    if (K == 0) return make_float3(v.y, v.z, v.x);
    if (K == 1) return make_float3(v.z, v.x, v.y);
    if (K == 2) return v;
    const bool k0 = kz == 0, k1 = kz == 1;
    return make_float3(pick(k0, v.y, pick(k1, v.z, v.x)), pick(k0, v.z, pick(k1, v.x, v.y)),
                       pick(k0, v.x, pick(k1, v.y, v.z)));
}

__device__ __forceinline__ Ray make_ray(float3 o, float3 d) {
    Ray r;
    r.o = o;
    r.d = d;
    // keep 1/d finite so the slab products never form inf - inf
    float dx = fabsf(d.x) < 1e-20f ? copysignf(1e-20f, d.x) : d.x;
    float dy = fabsf(d.y) < 1e-20f ? copysignf(1e-20f, d.y) : d.y;
    float dz = fabsf(d.z) < 1e-20f ? copysignf(1e-20f, d.z) : d.z;
    r.inv = make_float3(__builtin_amdgcn_rcpf(dx), __builtin_amdgcn_rcpf(dy), __builtin_amdgcn_rcpf(dz));
    const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    r.kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
    const float3 dr = rotate_to_z(d, r.kz);
    const float sz = __builtin_amdgcn_rcpf(dr.z);
    r.shear = make_float3(dr.x * sz, dr.y * sz, sz);
    return r;
}

// Signed double areas of the projected triangle's edges, products rounded
// separately (no fused multiply-add), so that the edge (P, Q) gives exactly
// the negated value of (Q, P): two triangles sharing an edge then agree on
// which side of it a ray passes.
__device__ __forceinline__ void edge_areas(float ax, float ay, float bx, float by, float cx, float cy, float &u,
                                           float &v, float &w) {
#pragma clang fp contract(off)
    u = cx * by - cy * bx;
    v = ax * cy - ay * cx;
    w = bx * ay - by * ax;
}

// Two-sided watertight ray/triangle test (Woop, Benthin and Wald 2013): each
// vertex relative to the origin is sheared into the ray's frame by one fixed
// function of that vertex, and the ray crosses the triangle when the three
// edge areas do not have mixed signs (a ray through a shared edge or vertex
// is inside at least one of the triangles there, never neither). True when
// the ray line crosses the triangle; t receives the ray parameter of the
// crossing as the barycentric mean of the vertices' parameters (within
// about 1e-6 of the scene's extent, enough to order hits; the hit a ray
// keeps gets its distance again from plane_t).
template <int K>
__device__ __forceinline__ bool tri_cross_k(const GpuTri &T, const Ray &r, float &t) {
    const float3 A = rotate_to_z<K>(xyz(T.v0) - r.o, r.kz);
    const float3 B = rotate_to_z<K>(xyz(T.v1) - r.o, r.kz);
    const float3 C = rotate_to_z<K>(xyz(T.v2) - r.o, r.kz);
    const float sx = r.shear.x, sy = r.shear.y, sz = r.shear.z;
    float u, v, w;
    edge_areas(fmaf(-sx, A.z, A.x), fmaf(-sy, A.z, A.y), fmaf(-sx, B.z, B.x), fmaf(-sy, B.z, B.y),
               fmaf(-sx, C.z, C.x), fmaf(-sy, C.z, C.y), u, v, w);
    const float lo = fminf(u, fminf(v, w)), hi = fmaxf(u, fmaxf(v, w));
    const float det = u + v + w;
    t = sz * fmaf(u, A.z, fmaf(v, B.z, w * C.z)) * __builtin_amdgcn_rcpf(det);
    // written so that NaN (det == 0: a ray in the plane) fails
    return !(lo < 0.f && hi > 0.f) && det != 0.f && (t == t);
}

// The rays of a packet share one direction and so one projection axis:
// when every testing lane has the same, the rotation is resolved at compile
// time (a wave-uniform branch); otherwise per lane.
__device__ __forceinline__ bool tri_cross(const GpuTri &T, const Ray &r, float &t) {
    const int k0 = __builtin_amdgcn_readfirstlane(r.kz);
    if (__all(r.kz == k0)) {
        if (k0 == 0) return tri_cross_k<0>(T, r, t);
        if (k0 == 1) return tri_cross_k<1>(T, r, t);
        return tri_cross_k<2>(T, r, t);
    }
    return tri_cross_k<-1>(T, r, t);
}

// Ray parameter where (o, d) meets the plane of T: n . (v0 - o) / n . d with
// n = (v1 - v0) x (v2 - v0). A few ulps even on a large triangle met close to
// the origin, where the barycentric mean of far vertices' parameters loses
// up to 1e-3 of a short distance to cancellation.
__device__ __forceinline__ float plane_t(const GpuTri &T, float3 o, float3 d) {
    const float3 v0 = xyz(T.v0);
    const float3 n = cross3(xyz(T.v1) - v0, xyz(T.v2) - v0);
    return dot3(n, v0 - o) * __builtin_amdgcn_rcpf(dot3(n, d));
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
// Per axis the entry plane is the low one when the direction is positive
// (the FMA is monotonic in q, so it is the smaller distance, exactly what a
// min of the two would pick) and the high one otherwise.
struct Node4Hits {
    float tn[4];
    bool hit[4];
    int child[4];
    int count[4];
    int leaf_base;       // first triangle slot of the node's leaf children
    uint32_t leaf_bits;  // hit leaf triangles: bit i = slot leaf_base + i
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
    const bool sx = __float_as_uint(r.inv.x) >> 31, sy = __float_as_uint(r.inv.y) >> 31,
               sz = __float_as_uint(r.inv.z) >> 31;
    const uint32_t nx = sx ? w1.y : w1.x, fx = sx ? w1.x : w1.y;
    const uint32_t ny = sy ? w1.w : w1.z, fy = sy ? w1.z : w1.w;
    const uint32_t nz = sz ? w2.y : w2.x, fz = sz ? w2.x : w2.y;
    o.leaf_base = (int)w2.w;
    o.leaf_bits = 0u;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float xn = fmaf(ubyte(nx, c), ax, bx), xf = fmaf(ubyte(fx, c), ax, bx);
        const float yn = fmaf(ubyte(ny, c), ay, by), yf = fmaf(ubyte(fy, c), ay, by);
        const float zn = fmaf(ubyte(nz, c), az, bz), zf = fmaf(ubyte(fz, c), az, bz);
        const float tn = fmaxf(fmaxf(xn, yn), fmaxf(zn, tmin));
        const float tf = fminf(fminf(xf, yf), fminf(zf, tmax));
        o.tn[c] = tn;
        o.hit[c] = tn <= tf && o.child[c] >= 0;
        const uint32_t lb = (w2.z >> (8 * c)) & 0xffu;
        o.count[c] = (int)(lb & 7u);
        // triangles offset .. offset + count - 1 of the node's leaf slots
        if (o.hit[c] && (lb & 7u)) o.leaf_bits |= ((1u << (lb & 7u)) - 1u) << (lb >> 3);
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
    base = h.leaf_base;
    return h.leaf_bits;
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

// Hit record of a ray (layout in VolumeParams::hitrec).
__device__ __forceinline__ int2 hit_record(int slot, bool dyn, float t) {
    return make_int2(slot < 0 ? -1 : (slot | (dyn ? (int)0x80000000 : 0)), __float_as_int(t));
}

// Geometry of a hit: unit normal facing the ray origin and the hit point.
__device__ __forceinline__ void hit_frame(const GpuTri &T, const Ray &ray, float3 o, float t, float3 &nrm,
                                          float3 &xh) {
    nrm = cross3(xyz(T.v1) - xyz(T.v0), xyz(T.v2) - xyz(T.v0));
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
    if (best >= 0) tbest = plane_t(arr[best], o, ray.d);
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
        split.hitrec[q] = hit_record(best, arr == sv.dyn.tris, tbest);
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
    if (vp.hitrec) vp.hitrec[q] = hit_record(best, arr == sv.dyn.tris, tbest);
}

struct TraceGrid {
    int bx, by, bz;        // brick shape (64 probes)
    int nbx, nby, nbz;     // bricks per axis
    int n_bricks, n_waves; // n_waves = n_bricks * rays per probe
    int persistent;
    int chunk;             // waves per XCD queue (persistent)
};

// ---------------------------------------------------------------------------
// Stepped lanes: per-lane state machine of the trace
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
// Scheduling weights, measured on the city and encode workloads (2% faster
// than 16 and 3, which were set before the BVH's split references made
// triangle tests rarer):
constexpr int kRefillAt = 32;      // transitions once this many lanes wait
constexpr int kNodeCost = 4;       // triangle step once its lanes x 4 >= the lanes waiting for a node

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
        // primary ray done: its distance from the hit triangle's plane, then
        // emission or sky, then the lights
        s.tbest = s.tmax;
        if (s.best >= 0) {
            const int p = s.q / vp.n, j = s.q - p * vp.n;
            s.tbest = plane_t((s.best_dyn ? sv.dyn.tris : sv.stat.tris)[s.best], probe_origin(vp, p), xyz(dirs[j]));
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
    if (vp.hitrec) vp.hitrec[s.q] = hit_record(s.best, s.best_dyn, s.tbest);
    s.q = -1;
}

// Packet w -> (ray direction j, brick): brick-major, every direction of a
// brick before the next brick, so that each XCD's contiguous share of the
// packets (its blocks, or its refill queue) covers a contiguous set of bricks
// and its L2 holds the scene around them rather than around every brick.
__device__ __forceinline__ void packet_of(const VolumeParams &vp, int w, int &j, int &brick) {
    brick = w / vp.n;
    j = w - brick * vp.n;
}

// Ray number r (packet order) -> record index, or -1 for a lane of a ragged
// brick that lies outside the grid.
__device__ __forceinline__ int ray_record(const VolumeParams &vp, const TraceGrid &g, int r) {
    const int w = r >> 6, lane = r & 63;
    int j, brick;
    packet_of(vp, w, j, brick);
    const int bxi = brick % g.nbx, byi = (brick / g.nbx) % g.nby, bzi = brick / (g.nbx * g.nby);
    const int x = bxi * g.bx + lane % g.bx;
    const int y = byi * g.by + (lane / g.bx) % g.by;
    const int z = bzi * g.bz + lane / (g.bx * g.by);
    if (x >= vp.nx || y >= vp.ny || z >= vp.nz) return -1;
    return (x + vp.nx * (y + vp.ny * z)) * vp.n + j;
}

// The wave's lane loop (see above): runs until every lane is idle and, with
// REFILL, the work queues are empty. Lanes start idle or with a primary ray
// set up by the caller.
template <bool COUNT, bool REFILL, class STK>
__device__ void lane_loop(LaneState &s, const VolumeParams &vp, const SceneView &sv, const NodeSrc &stat_src,
                          const FrameParams &fp, const float4 *dirs, float4 *rays, int32_t *hits, const TraceGrid &g,
                          int *queue, STK stk_l, Counts &cnt, uint32_t &shadow) {
    const uint4 *dyn_nodes = reinterpret_cast<const uint4 *>(sv.dyn.nodes);
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const long long total = (long long)g.n_waves * 64;
    const int chunk = (int)((total + 7) / 8);
    int k = 0;                                   // queues visited (wave-uniform)
    const int home = (blockIdx.x & 7);
    bool exhausted = !REFILL;
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
                if (lane == 0) base = atomicAdd(queue + qk * kQueueStride, want);
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
}

// Sets lane state s to the primary ray of record q (q >= 0) or idle.
__device__ __forceinline__ void lane_start(LaneState &s, const VolumeParams &vp, const SceneView &sv,
                                           const float4 *dirs, int q) {
    s.q = -1;
    s.node = -1;
    s.tmask = 0u;
    s.stage = kPrimStat;
    if (q < 0) return;
    const int p = q / vp.n, j = q - p * vp.n;
    s.q = q;
    s.ray = make_ray(probe_origin(vp, p), xyz(dirs[j]));
    s.tmax = INFINITY;
    s.best = -1;
    s.best_id = -1;
    s.best_dyn = false;
    start_traversal(s, sv.stat);
}

}  // namespace pv
