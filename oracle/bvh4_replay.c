/*
 * bvh4_replay.c -- host replay of the GPU trace's traversal work, for
 * checking the device's instrumented counts (node visits, triangle tests,
 * shadow rays) that the benchmark turns into FLOP per launch.
 *
 * TEST INFRASTRUCTURE ONLY, built into liboracle.so beside oracle.c and
 * called by the test suite alone. It reads the library's device BVH as
 * plain data in the layout the public header documents for
 * pv_scene_read_bvh (4-wide nodes with byte-quantized child boxes,
 * triangle slots with exact vertices) and shares no code with the HIP
 * path: the walk below is written from that layout and from the traversal
 * the GPU performs, which is the algorithm, not the library's source:
 *   - closest hit over the static BVH, then the dynamic one, nearest inner
 *     child first (children ordered by entry distance), the others stacked;
 *     a node's hit leaf triangles tested in slot order; culling by the best
 *     distance so far;
 *   - the triangle test of Woop, Benthin and Wald (2013): vertices relative
 *     to the origin rotated so the dominant axis of the direction comes
 *     last, sheared by (d_kx, d_ky)/d_kz, edge areas from separately
 *     rounded products, no mixed signs; ray parameter as the barycentric
 *     mean of the vertices' parameters, the kept hit's from its plane;
 *   - per point light facing the hit, one any-hit shadow ray from the hit
 *     point moved eps along the normal, through both BVHs.
 * Arithmetic is FP32 with the same fused multiply-adds, so counts agree
 * with the device's except where its approximate reciprocals flip a
 * decision at a box or triangle boundary (rare).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RP_API __attribute__((visibility("default")))

typedef struct { float x, y, z; } f3;

static f3 mk(float x, float y, float z) { f3 r = {x, y, z}; return r; }
static f3 sub(f3 a, f3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static float dot(f3 a, f3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
static f3 cross(f3 a, f3 b)
{
    return mk(fmaf(a.y, b.z, -(a.z * b.y)), fmaf(a.z, b.x, -(a.x * b.z)), fmaf(a.x, b.y, -(a.y * b.x)));
}
static float ubits(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t fbits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

typedef struct {
    const uint32_t *nodes;  /* [n_nodes][16] */
    const float *tris;      /* [n_tris][12] */
    int n_nodes;
} bvh_t;

typedef struct {
    f3 o, inv, shear;
    int kz;
} ray_t;

/* axis kz moved last, cyclic order kept */
static f3 rot(f3 v, int kz)
{
    if (kz == 0) return mk(v.y, v.z, v.x);
    if (kz == 1) return mk(v.z, v.x, v.y);
    return v;
}

static ray_t make_ray(f3 o, f3 d)
{
    ray_t r;
    r.o = o;
    float dx = fabsf(d.x) < 1e-20f ? copysignf(1e-20f, d.x) : d.x;
    float dy = fabsf(d.y) < 1e-20f ? copysignf(1e-20f, d.y) : d.y;
    float dz = fabsf(d.z) < 1e-20f ? copysignf(1e-20f, d.z) : d.z;
    r.inv = mk(1.0f / dx, 1.0f / dy, 1.0f / dz);
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    r.kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
    f3 dr = rot(d, r.kz);
    float sz = 1.0f / dr.z;
    r.shear = mk(dr.x * sz, dr.y * sz, sz);
    return r;
}

static f3 vert(const float *t, int k) { return mk(t[4 * k], t[4 * k + 1], t[4 * k + 2]); }
static int tri_index(const float *t) { int32_t i; memcpy(&i, &t[3], 4); return i; }

/* watertight crossing; *t = barycentric ray parameter */
static int crosses(const float *T, const ray_t *r, float *t)
{
    f3 A = rot(sub(vert(T, 0), r->o), r->kz), B = rot(sub(vert(T, 1), r->o), r->kz),
       C = rot(sub(vert(T, 2), r->o), r->kz);
    float sx = r->shear.x, sy = r->shear.y, sz = r->shear.z;
    float ax = fmaf(-sx, A.z, A.x), ay = fmaf(-sy, A.z, A.y);
    float bx = fmaf(-sx, B.z, B.x), by = fmaf(-sy, B.z, B.y);
    float cx = fmaf(-sx, C.z, C.x), cy = fmaf(-sy, C.z, C.y);
    float p1 = cx * by, p2 = cy * bx, p3 = ax * cy, p4 = ay * cx, p5 = bx * ay, p6 = by * ax;
    float u = p1 - p2, v = p3 - p4, w = p5 - p6;
    float lo = fminf(u, fminf(v, w)), hi = fmaxf(u, fmaxf(v, w));
    float det = u + v + w;
    float num = sz * fmaf(u, A.z, fmaf(v, B.z, w * C.z));
    *t = num * (1.0f / det);
    return !(lo < 0.f && hi > 0.f) && det != 0.f && (*t == *t);
}

static float plane_param(const float *T, f3 o, f3 d)
{
    f3 v0 = vert(T, 0);
    f3 n = cross(sub(vert(T, 1), v0), sub(vert(T, 2), v0));
    return dot(n, sub(v0, o)) * (1.0f / dot(n, d));
}

typedef struct {
    uint64_t nodes, tris;
} cnt_t;

/* The four child boxes of node k against [tmin, tmax]: entry distances,
 * hit flags, and the node's hit leaf triangles as a mask over its slots. */
static void node_boxes(const uint32_t *w, const ray_t *r, float tmin, float tmax, float tn[4], int hit[4],
                       int child[4], int cnt[4], int *base, uint32_t *bits)
{
    float ax = ubits((w[3] & 0xffu) << 23) * r->inv.x;
    float ay = ubits(((w[3] >> 8) & 0xffu) << 23) * r->inv.y;
    float az = ubits(((w[3] >> 16) & 0xffu) << 23) * r->inv.z;
    float bx = (ubits(w[0]) - r->o.x) * r->inv.x;
    float by = (ubits(w[1]) - r->o.y) * r->inv.y;
    float bz = (ubits(w[2]) - r->o.z) * r->inv.z;
    int sx = fbits(r->inv.x) >> 31, sy = fbits(r->inv.y) >> 31, sz = fbits(r->inv.z) >> 31;
    /* per axis the entry plane is the low byte for a positive direction */
    uint32_t nx = sx ? w[5] : w[4], fx = sx ? w[4] : w[5];
    uint32_t ny = sy ? w[7] : w[6], fy = sy ? w[6] : w[7];
    uint32_t nz = sz ? w[9] : w[8], fz = sz ? w[8] : w[9];
    *base = (int)w[11];
    *bits = 0u;
    for (int c = 0; c < 4; ++c) {
        child[c] = (int32_t)w[12 + c];
        float xn = fmaf((float)((nx >> (8 * c)) & 0xffu), ax, bx), xf = fmaf((float)((fx >> (8 * c)) & 0xffu), ax, bx);
        float yn = fmaf((float)((ny >> (8 * c)) & 0xffu), ay, by), yf = fmaf((float)((fy >> (8 * c)) & 0xffu), ay, by);
        float zn = fmaf((float)((nz >> (8 * c)) & 0xffu), az, bz), zf = fmaf((float)((fz >> (8 * c)) & 0xffu), az, bz);
        float a = fmaxf(fmaxf(xn, yn), fmaxf(zn, tmin));
        float b = fminf(fminf(xf, yf), fminf(zf, tmax));
        tn[c] = a;
        hit[c] = a <= b && child[c] >= 0;
        uint32_t lb = (w[10] >> (8 * c)) & 0xffu;
        cnt[c] = (int)(lb & 7u);
        if (hit[c] && (lb & 7u)) *bits |= ((1u << (lb & 7u)) - 1u) << (lb >> 3);
    }
}

/* hit inner children, nearest entry first (a five-exchange sorting network,
 * stable for equal distances as the device's) */
static int order_inner(const float tn[4], const int hit[4], const int child[4], const int cnt[4], int ids[4])
{
    float k[4];
    int m = 0;
    for (int c = 0; c < 4; ++c) {
        int inner = hit[c] && cnt[c] == 0;
        k[c] = inner ? tn[c] : 3.0e38f;
        ids[c] = child[c];
        m += inner;
    }
    static const int net[5][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}, {1, 2}};
    for (int e = 0; e < 5; ++e) {
        int a = net[e][0], b = net[e][1];
        if (k[b] < k[a]) {
            float tk = k[a]; k[a] = k[b]; k[b] = tk;
            int ti = ids[a]; ids[a] = ids[b]; ids[b] = ti;
        }
    }
    return m;
}

#define RP_STACK 64

/* Closest hit (any = 0) or any hit in (0, tmax) (any = 1) in one BVH. */
static int walk(const bvh_t *b, const ray_t *r, int any, float *tmax, int *best_slot, int *best_id, cnt_t *cnt)
{
    if (b->n_nodes == 0) return 0;
    int stack[RP_STACK], sp = 0, node = 0, found = 0;
    for (;;) {
        float tn[4];
        int hit[4], child[4], nc[4], base, ids[4];
        uint32_t bits;
        node_boxes(b->nodes + 16 * (size_t)node, r, 0.f, *tmax, tn, hit, child, nc, &base, &bits);
        cnt->nodes++;
        int m = order_inner(tn, hit, child, nc, ids);  /* culled with the distance before the leaves */
        for (; bits; bits &= bits - 1u) {
            int slot = base + __builtin_ctz(bits);
            const float *T = b->tris + 12 * (size_t)slot;
            float t;
            cnt->tris++;
            if (!crosses(T, r, &t) || !(t > 0.f)) continue;
            if (any) {
                if (t < *tmax) return 1;
            } else if (t < *tmax || (t == *tmax && tri_index(T) < *best_id)) {
                *tmax = t;
                *best_slot = slot;
                *best_id = tri_index(T);
                found = 1;
            }
        }
        if (m > 0) {
            if (sp + 3 > RP_STACK) return -1;
            if (m > 3) stack[sp++] = ids[3];
            if (m > 2) stack[sp++] = ids[2];
            if (m > 1) stack[sp++] = ids[1];
            node = ids[0];
        } else {
            if (sp == 0) break;
            node = stack[--sp];
        }
    }
    return found;
}

/*
 * Replays the trace of every (probe, ray) of a volume: probe p at
 * (ox + sx*x, oy + sy*y, oz + sz*z) (one fused multiply-add per axis),
 * p = x + nx*(y + ny*z); directions dirs[n][4] as the device computed them
 * (FP32); lights [n_lights][6] (position, intensity; only positions used);
 * eps the shadow-ray offset. Adds node visits, triangle tests and shadow
 * rays to counts[0..2]. Returns 0, or -1 when a stack overflows.
 */
RP_API int rp_trace_counts(const uint32_t *snodes, int s_nodes, const float *stris, const uint32_t *dnodes,
                           int d_nodes, const float *dtris, int nx, int ny, int nz, const float origin[3],
                           const float spacing[3], int n, const float *dirs, int n_lights, const float *lights,
                           float eps, uint64_t counts[3])
{
    bvh_t bs = {snodes, stris, s_nodes}, bd = {dnodes, dtris, d_nodes};
    const long long P = (long long)nx * ny * nz;
    uint64_t nodes = 0, tris = 0, shadow = 0;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nodes, tris, shadow) reduction(| : bad)
    for (long long p = 0; p < P; ++p) {
        const int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((long long)nx * ny));
        const f3 o = mk(fmaf(spacing[0], (float)x, origin[0]), fmaf(spacing[1], (float)y, origin[1]),
                        fmaf(spacing[2], (float)z, origin[2]));
        for (int j = 0; j < n; ++j) {
            const f3 d = mk(dirs[4 * j], dirs[4 * j + 1], dirs[4 * j + 2]);
            ray_t r = make_ray(o, d);
            cnt_t c = {0, 0};
            float tb = INFINITY;
            int slot = -1, id = -1, in_dyn = 0;
            int f = walk(&bs, &r, 0, &tb, &slot, &id, &c);
            int g = walk(&bd, &r, 0, &tb, &slot, &id, &c);
            if (f < 0 || g < 0) bad = 1;
            if (g > 0) in_dyn = 1;
            if (slot >= 0) {
                const float *T = (in_dyn ? dtris : stris) + 12 * (size_t)slot;
                const float t = plane_param(T, o, d);
                /* hit frame: unit normal facing the origin, hit point */
                f3 v0 = vert(T, 0);
                f3 nr = cross(sub(vert(T, 1), v0), sub(vert(T, 2), v0));
                const float il = 1.0f / sqrtf(dot(nr, nr));
                nr = mk(nr.x * il, nr.y * il, nr.z * il);
                if (dot(nr, d) > 0.f) nr = mk(-nr.x, -nr.y, -nr.z);
                const f3 xh = mk(fmaf(t, d.x, o.x), fmaf(t, d.y, o.y), fmaf(t, d.z, o.z));
                for (int li = 0; li < n_lights; ++li) {
                    const f3 lp = mk(lights[6 * li], lights[6 * li + 1], lights[6 * li + 2]);
                    const f3 lv = sub(lp, xh);
                    const float dl = sqrtf(dot(lv, lv));
                    const float cosv = dot(nr, lv) / dl;
                    if (!(cosv > 0.f)) continue;
                    const f3 so = mk(fmaf(eps, nr.x, xh.x), fmaf(eps, nr.y, xh.y), fmaf(eps, nr.z, xh.z));
                    f3 sd = sub(lp, so);
                    const float slen = sqrtf(dot(sd, sd));
                    const float isl = 1.0f / slen;
                    sd = mk(sd.x * isl, sd.y * isl, sd.z * isl);
                    float smax = slen - eps;
                    ray_t sr = make_ray(so, sd);
                    int s0 = -1, s1 = -1;
                    shadow++;
                    int occ = walk(&bs, &sr, 1, &smax, &s0, &s1, &c);
                    if (occ < 0) bad = 1;
                    if (occ <= 0) {
                        int occ2 = walk(&bd, &sr, 1, &smax, &s0, &s1, &c);
                        if (occ2 < 0) bad = 1;
                    }
                }
            }
            nodes += c.nodes;
            tris += c.tris;
        }
    }
    counts[0] += nodes;
    counts[1] += tris;
    counts[2] += shadow;
    return bad ? -1 : 0;
}
