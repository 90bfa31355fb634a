/*
 * oracle.c -- plain, slow FP64 CPU oracle for the dynamic probe-volume update
 * and the lossless delta packing of "A Distributed, Decoupled System for
 * Losslessly Streaming Dynamic Light Probes to Thin Clients" (Stengel et al.,
 * 2021).
 *
 * TEST INFRASTRUCTURE ONLY. It is called by the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark. The product library never links,
 * loads or calls it, and the two share no code, headers or tables.
 *
 * What it follows:
 *   - Section 3.2: octahedral irradiance (10x10 texels with a 1-texel guard
 *     band) and visibility (18x18, mean distance and mean squared distance)
 *     maps per probe, from the irradiance-volume method the paper adopts.
 *     The paper does not restate that method's update; the steps below are
 *     the published irradiance-volume reading: spherical-Fibonacci rays under
 *     one random rotation per frame, closest hit, direct shading, cosine
 *     (irradiance) and cosine-power (visibility) weighted means, hysteresis,
 *     guard-band copy by the octahedral fold.
 *   - Section 3.2 (streaming probe visibility): the shading-time query of a
 *     volume -- trilinear over the eight probes around the point, bilinear
 *     octahedral lookup through the guard bands, and the Chebyshev bound of
 *     the (mean, mean squared) distances as a per-probe visibility weight --
 *     used as the second bounce of an update when requested (each hit adds
 *     its albedo times the query of the maps as they stood before the frame).
 *   - Section 3.3 (visibility encoding): each FP16 value split into its two
 *     bytes.
 *   - Section 3.4 (repacking, update textures, change thresholding): guard
 *     bands dropped, index-based update with a delta-encoded 2-byte probe
 *     index buffer, per-client last-transmitted textures, a probe is sent
 *     when it is not identical (or beyond a threshold) to what was last sent,
 *     and sent data is written to the last-transmitted texture.
 *
 * Everything floating point is IEEE double, with no fused multiply-add
 * contraction (build with -ffp-contract=off). FP32 inputs are taken as data.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_API __attribute__((visibility("default")))

/* ======================================================================== */
/* IEEE 754 binary16 <-> double                                              */
/* ======================================================================== */

/* Exact value of a binary16 bit pattern. */
OR_API double or_half_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 0x1f;
    int m = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)m, -24);                 /* zero / subnormal */
    else if (e == 31)
        v = m ? NAN : INFINITY;
    else
        v = ldexp((double)(m + 1024), e - 25);     /* 1.m * 2^(e-15) */
    return sign ? -v : v;
}

/* Round a double to the nearest binary16, ties to even; overflow to inf. */
OR_API uint16_t or_double_to_half(double x)
{
    uint16_t sign = signbit(x) ? 0x8000 : 0;
    double a = fabs(x);
    if (isnan(x))
        return sign | 0x7e00;
    if (a >= 65520.0)                    /* half-way above 65504 rounds to inf */
        return sign | 0x7c00;
    if (a < ldexp(1.0, -14)) {           /* subnormal: multiple of 2^-24 */
        double m = nearbyint(ldexp(a, 24)); /* default mode: ties to even */
        return sign | (uint16_t)m;       /* m == 1024 is the smallest normal */
    }
    int e;
    double f = frexp(a, &e);             /* a = f * 2^e, f in [0.5, 1) */
    double m = nearbyint(ldexp(f, 11));  /* 11 significant bits */
    int E = e - 1 + 15;
    if (m == 2048.0) {
        m = 1024.0;
        E += 1;
    }
    if (E >= 31)
        return sign | 0x7c00;
    return sign | (uint16_t)(E << 10) | (uint16_t)((int)m - 1024);
}

OR_API void or_round_half_array(const double *in, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = or_half_to_double(or_double_to_half(in[i]));
}

/* ======================================================================== */
/* Octahedral map (Cigolle et al. 2014; the map the probe textures use)      */
/* ======================================================================== */

static double sgn_pos(double v) { return v >= 0.0 ? 1.0 : -1.0; }

/* (u, w) in [-1,1]^2 -> unit direction. */
OR_API void or_oct_decode(double u, double w, double out[3])
{
    double x = u, y = w, z = 1.0 - fabs(u) - fabs(w);
    if (z < 0.0) {
        x = (1.0 - fabs(w)) * sgn_pos(u);
        y = (1.0 - fabs(u)) * sgn_pos(w);
    }
    double len = sqrt(x * x + y * y + z * z);
    out[0] = x / len;
    out[1] = y / len;
    out[2] = z / len;
}

/* Unit direction -> (u, w) in [-1,1]^2. */
OR_API void or_oct_encode(const double v[3], double out[2])
{
    double s = fabs(v[0]) + fabs(v[1]) + fabs(v[2]);
    double px = v[0] / s, py = v[1] / s;
    if (v[2] < 0.0) {
        double qx = (1.0 - fabs(py)) * sgn_pos(px);
        double qy = (1.0 - fabs(px)) * sgn_pos(py);
        px = qx;
        py = qy;
    }
    out[0] = px;
    out[1] = py;
}

/* Direction of the centre of interior texel (i, j) of an N x N map. */
static void texel_dir(int N, int i, int j, double out[3])
{
    double u = 2.0 * (i + 0.5) / N - 1.0;
    double w = 2.0 * (j + 0.5) / N - 1.0;
    or_oct_decode(u, w, out);
}

/* All N*N texel-centre directions, row-major (t = j*N + i), [N*N][3]. */
OR_API void or_texel_dirs(int N, double *out)
{
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i)
            texel_dir(N, i, j, out + 3 * (j * N + i));
}

/* ======================================================================== */
/* Ray directions: spherical Fibonacci set rotated by R (Keinert et al. 2015) */
/* ======================================================================== */

OR_API void or_ray_dirs(int n, const float R[9], double *out)
{
    const double golden_frac = (sqrt(5.0) - 1.0) * 0.5;  /* Phi - 1 */
    const double two_pi = 6.283185307179586476925286766559;
    for (int i = 0; i < n; ++i) {
        double z = 1.0 - (2.0 * i + 1.0) / n;
        double a = i * golden_frac;
        double phi = two_pi * (a - floor(a));
        double s = sqrt(fmax(0.0, 1.0 - z * z));
        double sf[3] = {s * cos(phi), s * sin(phi), z};
        for (int k = 0; k < 3; ++k)
            out[3 * i + k] = (double)R[3 * k + 0] * sf[0] +
                             (double)R[3 * k + 1] * sf[1] +
                             (double)R[3 * k + 2] * sf[2];
    }
}

/* ======================================================================== */
/* Scene: triangles + object-median BVH (the oracle's own, binary)           */
/* ======================================================================== */

typedef struct {
    double lo[3], hi[3];
    int left, right;   /* children (inner) */
    int first, count;  /* triangle range in 'order' (leaf when count > 0) */
} or_node;

typedef struct or_scene {
    int ntri;
    double *tri;    /* [ntri][9]  v0, v1, v2 */
    double *alb;    /* [ntri][3] */
    double *emi;    /* [ntri][3] */
    int *order;     /* leaf order -> triangle index */
    or_node *nodes;
    int nnodes;
    double eps;     /* shadow-ray offset: 1e-4 * static bounding-box diagonal */
    double diag;    /* static bounding-box diagonal */
} or_scene;

static double *g_sort_key;  /* used only inside the single-threaded build */

static int cmp_key(const void *a, const void *b)
{
    double ka = g_sort_key[*(const int *)a], kb = g_sort_key[*(const int *)b];
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (*(const int *)a) - (*(const int *)b);
}

static int build_node(or_scene *s, int first, int count, double *cent)
{
    int id = s->nnodes++;
    or_node *nd = &s->nodes[id];
    for (int k = 0; k < 3; ++k) {
        nd->lo[k] = INFINITY;
        nd->hi[k] = -INFINITY;
    }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = first; i < first + count; ++i) {
        const double *t = s->tri + 9 * s->order[i];
        for (int v = 0; v < 3; ++v)
            for (int k = 0; k < 3; ++k) {
                nd->lo[k] = fmin(nd->lo[k], t[3 * v + k]);
                nd->hi[k] = fmax(nd->hi[k], t[3 * v + k]);
            }
        for (int k = 0; k < 3; ++k) {
            clo[k] = fmin(clo[k], cent[3 * s->order[i] + k]);
            chi[k] = fmax(chi[k], cent[3 * s->order[i] + k]);
        }
    }
    if (count <= 4) {
        nd->first = first;
        nd->count = count;
        nd->left = nd->right = -1;
        return id;
    }
    int axis = 0;
    for (int k = 1; k < 3; ++k)
        if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
    for (int i = first; i < first + count; ++i)
        g_sort_key[s->order[i]] = cent[3 * s->order[i] + axis];
    qsort(s->order + first, count, sizeof(int), cmp_key);
    int half = count / 2;
    int l = build_node(s, first, half, cent);
    int r = build_node(s, first + half, count - half, cent);
    nd = &s->nodes[id];  /* (array does not move: preallocated) */
    nd->left = l;
    nd->right = r;
    nd->first = 0;
    nd->count = 0;
    return id;
}

/* tri9: [ntri][3][3] float32 vertex positions; n_static: leading triangles
 * that define the scene extent (and so the shadow offset). */
OR_API or_scene *or_scene_create(int ntri, const float *tri9, const float *albedo,
                                 const float *emission, int n_static)
{
    or_scene *s = (or_scene *)calloc(1, sizeof(or_scene));
    s->ntri = ntri;
    s->tri = (double *)malloc(sizeof(double) * 9 * (ntri > 0 ? ntri : 1));
    s->alb = (double *)malloc(sizeof(double) * 3 * (ntri > 0 ? ntri : 1));
    s->emi = (double *)malloc(sizeof(double) * 3 * (ntri > 0 ? ntri : 1));
    s->order = (int *)malloc(sizeof(int) * (ntri > 0 ? ntri : 1));
    s->nodes = (or_node *)malloc(sizeof(or_node) * (2 * (ntri > 0 ? ntri : 1)));
    for (int64_t i = 0; i < 9 * (int64_t)ntri; ++i) s->tri[i] = tri9[i];
    for (int64_t i = 0; i < 3 * (int64_t)ntri; ++i) {
        s->alb[i] = albedo[i];
        s->emi[i] = emission ? emission[i] : 0.0;
    }
    int ns = n_static > 0 ? n_static : ntri;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < ns && i < ntri; ++i)
        for (int v = 0; v < 3; ++v)
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], s->tri[9 * i + 3 * v + k]);
                hi[k] = fmax(hi[k], s->tri[9 * i + 3 * v + k]);
            }
    s->diag = ntri > 0 ? sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                              (hi[2] - lo[2]) * (hi[2] - lo[2]))
                       : 1.0;
    s->eps = 1e-4 * s->diag;
    s->nnodes = 0;
    if (ntri > 0) {
        double *cent = (double *)malloc(sizeof(double) * 3 * ntri);
        for (int i = 0; i < ntri; ++i) {
            s->order[i] = i;
            for (int k = 0; k < 3; ++k)
                cent[3 * i + k] = (s->tri[9 * i + k] + s->tri[9 * i + 3 + k] + s->tri[9 * i + 6 + k]) / 3.0;
        }
        g_sort_key = (double *)malloc(sizeof(double) * ntri);
        build_node(s, 0, ntri, cent);
        free(g_sort_key);
        g_sort_key = NULL;
        free(cent);
    }
    return s;
}

OR_API void or_scene_destroy(or_scene *s)
{
    if (!s) return;
    free(s->tri);
    free(s->alb);
    free(s->emi);
    free(s->order);
    free(s->nodes);
    free(s);
}

OR_API double or_scene_eps(const or_scene *s) { return s->eps; }
OR_API double or_scene_diag(const or_scene *s) { return s->diag; }

/* Moller-Trumbore (1997) in double: ray o + t d against triangle k.
 * Returns 0 when the ray is parallel to the plane; otherwise t and the
 * signed distances (world units) of the plane hit point to the three edges
 * (all >= 0 inside). */
static int tri_isect(const or_scene *s, int k, const double o[3], const double d[3],
                     double *t_out, double edge_dist[3])
{
    const double *v = s->tri + 9 * k;
    double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    double p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    double tv[3] = {o[0] - v[0], o[1] - v[1], o[2] - v[2]};
    double b1 = (tv[0] * p[0] + tv[1] * p[1] + tv[2] * p[2]) * inv;
    double q[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
    double b2 = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * inv;
    double t = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * inv;
    double b0 = 1.0 - b1 - b2;
    /* distances to edges: b_i * (2 area) / |opposite edge| */
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double area2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    double e12[3] = {v[6] - v[3], v[7] - v[4], v[8] - v[5]};
    double l12 = sqrt(e12[0] * e12[0] + e12[1] * e12[1] + e12[2] * e12[2]);
    double l20 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
    double l01 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    edge_dist[0] = l12 > 0 ? b0 * area2 / l12 : b0;
    edge_dist[1] = l20 > 0 ? b1 * area2 / l20 : b1;
    edge_dist[2] = l01 > 0 ? b2 * area2 / l01 : b2;
    *t_out = t;
    return 1;
}

/* Slab test of the box widened by 'pad'; returns entry distance or INFINITY. */
static double box_enter(const or_node *nd, const double o[3], const double d[3], double pad, double tmax)
{
    double t0 = -INFINITY, t1 = INFINITY;
    for (int k = 0; k < 3; ++k) {
        double lo = nd->lo[k] - pad, hi = nd->hi[k] + pad;
        if (d[k] == 0.0) {
            if (o[k] < lo || o[k] > hi) return INFINITY;
            continue;
        }
        double a = (lo - o[k]) / d[k], b = (hi - o[k]) / d[k];
        if (a > b) { double tmp = a; a = b; b = tmp; }
        if (a > t0) t0 = a;
        if (b < t1) t1 = b;
    }
    if (t0 > t1 || t1 < -pad || t0 > tmax) return INFINITY;
    return t0;
}

/* Result of one ray query with a margin 'm' (world units):
 *   nominal: closest exact hit with t > tmin (ties: smaller triangle index);
 *   near:    1 when the answer could change under a perturbation of size m
 *            (a triangle within m of its edges or of tmin/tmax, or two
 *            different triangles within m of the nominal distance);
 *   ties:    the other triangles that are equally valid answers at margin m:
 *            those within 2m of the nominal distance, and those the ray
 *            passes within m of (edges or tmin) in front of the first sure
 *            hit. */
#define OR_MAX_TIES 8
typedef struct {
    int tri;
    double t;
    int near;
    int nties;
    int ties[OR_MAX_TIES];
    double ties_t[OR_MAX_TIES];
} or_hit;

#define OR_STACK 128

static or_hit closest_hit(const or_scene *s, const double o[3], const double d[3], double tmin, double m)
{
    or_hit h;
    memset(&h, 0, sizeof h);
    h.tri = -1;
    h.t = INFINITY;
    if (s->ntri == 0) return h;
    double t_limit = INFINITY;  /* closest 'sure' distance so far + margin */
    int stack[OR_STACK];
    int sp = 0;
    stack[sp++] = 0;
    /* Possible hits close to the front are kept to decide 'near' at the end. */
    double poss_t[64];
    int poss_id[64], poss_sure[64], npos = 0, overflow = 0;
    while (sp) {
        const or_node *nd = &s->nodes[stack[--sp]];
        if (box_enter(nd, o, d, m, t_limit) == INFINITY) continue;
        if (nd->count > 0) {
            for (int i = nd->first; i < nd->first + nd->count; ++i) {
                int k = s->order[i];
                double t, ed[3];
                if (!tri_isect(s, k, o, d, &t, ed)) continue;
                double emin = fmin(ed[0], fmin(ed[1], ed[2]));
                int exact = (t > tmin) && emin >= 0.0;
                int possible = (t > tmin - m) && emin >= -m;
                int sure = (t > tmin + m) && emin >= m;
                if (exact && (t < h.t || (t == h.t && k < h.tri))) {
                    h.t = t;
                    h.tri = k;
                }
                if (sure && t + m < t_limit) t_limit = t + m;
                if (possible) {
                    if (npos < 64) {
                        poss_t[npos] = t;
                        poss_id[npos] = k;
                        poss_sure[npos] = sure;
                        ++npos;
                    } else {
                        overflow = 1;
                    }
                }
            }
        } else {
            if (sp + 2 > OR_STACK) { h.near = 1; continue; }
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
    /* near: any possible-but-not-sure triangle in front of the sure front, or
     * another triangle within 2m of the nominal distance. */
    double front = h.tri >= 0 ? h.t : INFINITY;
    if (t_limit < front + m) front = t_limit - m;
    for (int i = 0; i < npos; ++i) {
        if (poss_t[i] > front + 2.0 * m) continue;
        const int graze = !poss_sure[i];
        const int same_depth = fabs(poss_t[i] - h.t) <= 2.0 * m;
        if (graze) h.near = 1;
        if (poss_id[i] != h.tri && (graze || same_depth)) {
            h.near = 1;
            int dup = 0;
            for (int k = 0; k < h.nties; ++k) dup |= h.ties[k] == poss_id[i];
            if (!dup && h.nties < OR_MAX_TIES) {
                h.ties[h.nties] = poss_id[i];
                h.ties_t[h.nties] = poss_t[i];
                h.nties++;
            }
        }
    }
    if (overflow) h.near = 1;
    return h;
}

/* Any hit with tmin < t < tmax. Returns 1 if occluded; *near as above. */
static int occluded(const or_scene *s, const double o[3], const double d[3], double tmin, double tmax,
                    double m, int *near)
{
    *near = 0;
    if (s->ntri == 0) return 0;
    int hit = 0, sure_hit = 0, possible_hit = 0;
    int stack[OR_STACK];
    int sp = 0;
    stack[sp++] = 0;
    while (sp) {
        const or_node *nd = &s->nodes[stack[--sp]];
        if (box_enter(nd, o, d, m, tmax + m) == INFINITY) continue;
        if (nd->count > 0) {
            for (int i = nd->first; i < nd->first + nd->count; ++i) {
                double t, ed[3];
                if (!tri_isect(s, s->order[i], o, d, &t, ed)) continue;
                double emin = fmin(ed[0], fmin(ed[1], ed[2]));
                if (t > tmin && t < tmax && emin >= 0.0) hit = 1;
                if (t > tmin + m && t < tmax - m && emin >= m) sure_hit = 1;
                if (t > tmin - m && t < tmax + m && emin >= -m) possible_hit = 1;
            }
            if (sure_hit) break;
        } else {
            if (sp + 2 > OR_STACK) { *near = 1; continue; }
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
    if (!sure_hit && possible_hit) *near = 1;
    return hit;
}

/* ======================================================================== */
/* Volume parameters                                                          */
/* ======================================================================== */

typedef struct {
    int nx, ny, nz;
    int n;              /* rays per probe */
    int irr_res, vis_res;
    int vis_sharpness;  /* exponent of the visibility cosine weight */
    int first_frame_no_history;
    double origin[3], spacing[3];
    double hysteresis, max_distance;
    double sky[3];
} or_volume;

static void probe_origin(const or_volume *v, int p, double o[3])
{
    int x = p % v->nx, y = (p / v->nx) % v->ny, z = p / (v->nx * v->ny);
    o[0] = v->origin[0] + v->spacing[0] * x;
    o[1] = v->origin[1] + v->spacing[1] * y;
    o[2] = v->origin[2] + v->spacing[2] * z;
}

/* ======================================================================== */
/* Shading of one hit                                                         */
/* ======================================================================== */

/* Radiance leaving triangle k at point x towards the probe (direction d of
 * the primary ray), with geometric normal n (already facing the probe).
 * Direct Lambertian lighting from point lights with a shadow ray, plus the
 * triangle's emission. lo/hi widen where a shadow decision is ambiguous. */
static void shade_hit(const or_scene *s, int k, const double x[3], const double n[3], int nlights,
                      const float *lights, double m, double Lnom[3], double Llo[3], double Lhi[3])
{
    const double inv_pi = 0.31830988618379067153776752674503;
    for (int c = 0; c < 3; ++c) Lnom[c] = Llo[c] = Lhi[c] = s->emi[3 * k + c];
    for (int li = 0; li < nlights; ++li) {
        const float *L = lights + 6 * li;
        double l[3] = {L[0] - x[0], L[1] - x[1], L[2] - x[2]};
        double dist2 = l[0] * l[0] + l[1] * l[1] + l[2] * l[2];
        double dist = sqrt(dist2);
        double cosv = (n[0] * l[0] + n[1] * l[1] + n[2] * l[2]) / dist;
        if (!(cosv > 0.0)) continue;
        /* shadow ray from the offset point towards the light */
        double so[3] = {x[0] + s->eps * n[0], x[1] + s->eps * n[1], x[2] + s->eps * n[2]};
        double sd[3] = {L[0] - so[0], L[1] - so[1], L[2] - so[2]};
        double slen = sqrt(sd[0] * sd[0] + sd[1] * sd[1] + sd[2] * sd[2]);
        for (int c = 0; c < 3; ++c) sd[c] /= slen;
        int near = 0;
        int occ = occluded(s, so, sd, 0.0, slen - s->eps, m, &near);
        for (int c = 0; c < 3; ++c) {
            double contrib = s->alb[3 * k + c] * inv_pi * (double)L[3 + c] * cosv / dist2;
            if (!occ) Lnom[c] += contrib;
            if (near) {
                Lhi[c] += contrib;           /* either decision is acceptable */
            } else if (!occ) {
                Llo[c] += contrib;
                Lhi[c] += contrib;
            }
        }
    }
}

/* Hit geometry for triangle k along ray (o, d) at distance t. Returns the
 * normal facing the ray origin; *grazing set when |cos| is tiny. */
static void hit_frame(const or_scene *s, int k, const double o[3], const double d[3], double t, double x[3],
                      double n[3], int *grazing)
{
    const double *v = s->tri + 9 * k;
    double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int c = 0; c < 3; ++c) n[c] /= len;
    double nd = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    if (nd > 0.0)
        for (int c = 0; c < 3; ++c) n[c] = -n[c];
    *grazing = fabs(nd) < 1e-6;
    for (int c = 0; c < 3; ++c) x[c] = o[c] + t * d[c];
}

/* ======================================================================== */
/* Probe query (second bounce)                                               */
/* ======================================================================== */
/* Bilinear lookup in one probe's tile of C channel maps ([C][(N+2)^2],
 * channel planes, row-major) in direction d. Interior texel i is centred at
 * tile coordinate i + 1 (guard texels at 0 and N+1), so the octahedral
 * coordinate u lands at s = (u + 1) N / 2 + 0.5 and the four texels around s
 * are always inside the tile: the guard bands carry the fold across the
 * square's edges. */
OR_API void or_probe_lookup(const double *tile, int N, int C, const double d[3], double *out)
{
    double uv[2];
    or_oct_encode(d, uv);
    const int S = N + 2;
    double sx = (uv[0] + 1.0) * 0.5 * N + 0.5, sy = (uv[1] + 1.0) * 0.5 * N + 0.5;
    int x0 = (int)floor(sx), y0 = (int)floor(sy);
    if (x0 > N) x0 = N;
    if (y0 > N) y0 = N;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    const double fx = sx - x0, fy = sy - y0;
    for (int c = 0; c < C; ++c) {
        const double *t = tile + (size_t)c * S * S;
        const double a = t[y0 * S + x0], b = t[y0 * S + x0 + 1];
        const double e = t[(y0 + 1) * S + x0], f = t[(y0 + 1) * S + x0 + 1];
        out[c] = (1.0 - fy) * ((1.0 - fx) * a + fx * b) + fy * ((1.0 - fx) * e + fx * f);
    }
}

/* Mean radiance arriving at point x around normal n, from the volume's
 * stored maps (irr [P][3][(Ni+2)^2], vis [P][2][(Nv+2)^2]): the probes at the
 * corners of the grid cell holding x (clamped to the grid) weighted
 * trilinearly and by the Chebyshev bound of their visibility moments in the
 * direction of x, each looked up in direction n; 0 when every weight
 * vanishes. */
OR_API void or_probe_query(const or_volume *v, const double *irr, const double *vis, const double x[3],
                           const double n[3], double out[3])
{
    const int dims[3] = {v->nx, v->ny, v->nz};
    int c0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        const double g = (x[a] - v->origin[a]) / v->spacing[a];
        if (dims[a] == 1) {
            c0[a] = 0;
            f[a] = 0.0;
            continue;
        }
        int c = (int)floor(g);
        if (c < 0) c = 0;
        if (c > dims[a] - 2) c = dims[a] - 2;
        double t = g - c;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        c0[a] = c;
        f[a] = t;
    }
    const int Ni = v->irr_res, Nv = v->vis_res;
    const size_t ti = (size_t)3 * (Ni + 2) * (Ni + 2), tv = (size_t)2 * (Nv + 2) * (Nv + 2);
    double acc[3] = {0.0, 0.0, 0.0}, wsum = 0.0;
    for (int corner = 0; corner < 8; ++corner) {
        int idx[3];
        double w = 1.0;
        int skip = 0;
        for (int a = 0; a < 3; ++a) {
            const int bit = (corner >> a) & 1;
            if (bit && dims[a] == 1) skip = 1;
            idx[a] = c0[a] + bit;
            w *= bit ? f[a] : 1.0 - f[a];
        }
        if (skip) continue;
        const int p = idx[0] + v->nx * (idx[1] + v->ny * idx[2]);
        double pp[3];
        probe_origin(v, p, pp);
        const double vec[3] = {x[0] - pp[0], x[1] - pp[1], x[2] - pp[2]};
        const double dist = sqrt(vec[0] * vec[0] + vec[1] * vec[1] + vec[2] * vec[2]);
        if (dist > 0.0) {
            const double dir[3] = {vec[0] / dist, vec[1] / dist, vec[2] / dist};
            double mom[2];
            or_probe_lookup(vis + (size_t)p * tv, Nv, 2, dir, mom);
            if (dist > mom[0]) {
                const double var = fmax(mom[1] - mom[0] * mom[0], 0.0);
                const double dd = dist - mom[0];
                w *= var / (var + dd * dd);
            }
        }
        double e[3];
        or_probe_lookup(irr + (size_t)p * ti, Ni, 3, n, e);
        for (int c = 0; c < 3; ++c) acc[c] += w * e[c];
        wsum += w;
    }
    for (int c = 0; c < 3; ++c) out[c] = wsum > 1e-20 ? acc[c] / wsum : 0.0;
}

/* Stored maps a second bounce reads: the nominal trajectory and the lower
 * and upper tie-bound trajectories ([0] nominal, [1] lower, [2] upper). */
typedef struct {
    const double *irr[3], *vis[3];
} or_prev_maps;

/* Adds the second bounce to a hit's radiance: albedo times the mean
 * radiance queried at the hit point moved off the surface along its normal
 * by a tenth of the smallest probe spacing (so that the probes' own
 * distance record of that surface does not shadow it). The nominal answer
 * reads the nominal maps; lo/hi span the answers on all three trajectories
 * (a lower-precision side's maps lie between the bound maps) and widen by
 * 'rel' of the term (the sides' stored maps also differ by rounding). */
static void add_indirect(const or_scene *s, const or_volume *v, const or_prev_maps *pm, int k, const double x[3],
                         const double n[3], double rel, double L[3], double Llo[3], double Lhi[3])
{
    const double bias = 0.1 * fmin(v->spacing[0], fmin(v->spacing[1], v->spacing[2]));
    const double xb[3] = {x[0] + bias * n[0], x[1] + bias * n[1], x[2] + bias * n[2]};
    double e[3][3];
    for (int m = 0; m < 3; ++m) or_probe_query(v, pm->irr[m], pm->vis[m], xb, n, e[m]);
    for (int c = 0; c < 3; ++c) {
        const double a = s->alb[3 * k + c];
        const double ind = a * e[0][c];
        double lo = ind, hi = ind;
        for (int m = 1; m < 3; ++m) {
            lo = fmin(lo, a * e[m][c]);
            hi = fmax(hi, a * e[m][c]);
        }
        L[c] += ind;
        Llo[c] += lo - rel * fabs(lo);
        Lhi[c] += hi + rel * fabs(hi);
    }
}

/* Distance along (o, d) to the plane of triangle k (for a candidate that a
 * perturbed ray found). */
static double plane_t(const or_scene *s, int k, const double o[3], const double d[3])
{
    const double *v = s->tri + 9 * k;
    double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double nd = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    double num = n[0] * (v[0] - o[0]) + n[1] * (v[1] - o[1]) + n[2] * (v[2] - o[2]);
    return nd != 0.0 ? num / nd : INFINITY;
}

/* ======================================================================== */
/* Trace + shade every (probe, ray)                                           */
/* ======================================================================== */

/*
 * Per ray q = p*n + j (p = x + nx*(y + ny*z)):
 *   L_nom[3q..], r_nom[q]  : the FP64 answer (closest hit, shading, distance);
 *   L_lo/L_hi, r_lo/r_hi   : bounds over every answer that an evaluation in
 *                            lower precision could legitimately produce:
 *                            hit candidates found by perturbing the ray origin
 *                            by +-delta along each axis when the ray is near a
 *                            tie, triangles within the tie margin of the
 *                            nominal distance (coplanar or crossing surfaces),
 *                            and either shadow decision when a shadow ray is
 *                            near a tie;
 *   hit[q]                 : nominal triangle (-1 = miss);
 *   cand[q*maxc..], ncand  : the accepted triangle set (nominal first).
 * delta_rel scales the perturbation with the scene diagonal.
 */
OR_API int or_trace_shade(const or_scene *s, const or_volume *v, const float R[9], int nlights,
                          const float *lights, double delta_rel, double *L_nom, double *L_lo, double *L_hi,
                          double *r_nom, double *r_lo, double *r_hi, int32_t *hit, double *hit_t,
                          int32_t *cand, int32_t *ncand, int maxc, int nthreads, const double *const *prev,
                          double ind_rel)
{
    /* prev: NULL (no second bounce) or six maps: irr, vis (nominal), irr_lo,
     * vis_lo, irr_hi, vis_hi; a NULL bound pair falls back to the nominal */
    or_prev_maps pm;
    const or_prev_maps *pmp = NULL;
    if (prev) {
        for (int m = 0; m < 3; ++m) {
            const int have = prev[2 * m] && prev[2 * m + 1];
            pm.irr[m] = have ? prev[2 * m] : prev[0];
            pm.vis[m] = have ? prev[2 * m + 1] : prev[1];
        }
        pmp = &pm;
    }
    const int P = v->nx * v->ny * v->nz;
    const int n = v->n;
    double *dirs = (double *)malloc(sizeof(double) * 3 * n);
    or_ray_dirs(n, R, dirs);
    const double delta = delta_rel * s->diag;
    const double m = 2.0 * delta;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int p = 0; p < P; ++p) {
        double o[3];
        probe_origin(v, p, o);
        for (int j = 0; j < n; ++j) {
            int64_t q = (int64_t)p * n + j;
            const double *d = dirs + 3 * j;
            or_hit h = closest_hit(s, o, d, 0.0, m);
            int cands[16];
            double cand_t[16];
            int nc = 0;
            cand_t[nc] = h.t;
            cands[nc++] = h.tri;
            if (h.near) {
                for (int a = 0; a < 3; ++a)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        double op[3] = {o[0], o[1], o[2]};
                        op[a] += sg * delta;
                        or_hit hp = closest_hit(s, op, d, 0.0, 0.0);
                        int seen = 0;
                        for (int c = 0; c < nc; ++c) seen |= cands[c] == hp.tri;
                        if (!seen && nc < 16) {
                            cand_t[nc] = hp.t;
                            cands[nc++] = hp.tri;
                        }
                    }
                /* triangles at the same distance (coplanar or crossing
                 * surfaces), and triangles the ray grazes in front of the
                 * first sure hit, are equally valid answers */
                for (int k = 0; k < h.nties; ++k) {
                    int seen = 0;
                    for (int c = 0; c < nc; ++c) seen |= cands[c] == h.ties[k];
                    if (!seen && nc < 16) {
                        cand_t[nc] = h.ties_t[k];
                        cands[nc++] = h.ties[k];
                    }
                }
            }
            double Ln[3], rn;
            double Llo[3] = {INFINITY, INFINITY, INFINITY}, Lhi[3] = {-INFINITY, -INFINITY, -INFINITY};
            double rlo = INFINITY, rhi = -INFINITY;
            for (int c = 0; c < nc; ++c) {
                int k = cands[c];
                double Lc[3], Lcl[3], Lch[3], rc;
                if (k < 0) {
                    for (int ch = 0; ch < 3; ++ch) Lc[ch] = Lcl[ch] = Lch[ch] = v->sky[ch];
                    rc = v->max_distance;
                } else {
                    double t = h.t;
                    if (c > 0) {
                        t = plane_t(s, k, o, d);
                        if (!(t > 0.0 && t < INFINITY)) t = cand_t[c];
                    }
                    double x[3], nrm[3];
                    int grazing;
                    hit_frame(s, k, o, d, t, x, nrm, &grazing);
                    shade_hit(s, k, x, nrm, nlights, lights, m, Lc, Lcl, Lch);
                    if (pmp) add_indirect(s, v, pmp, k, x, nrm, ind_rel, Lc, Lcl, Lch);
                    if (grazing) {  /* the other side is acceptable too */
                        double nf[3] = {-nrm[0], -nrm[1], -nrm[2]}, a[3], b[3], e[3];
                        shade_hit(s, k, x, nf, nlights, lights, m, a, b, e);
                        if (pmp) add_indirect(s, v, pmp, k, x, nf, ind_rel, a, b, e);
                        for (int ch = 0; ch < 3; ++ch) {
                            Lcl[ch] = fmin(Lcl[ch], b[ch]);
                            Lch[ch] = fmax(Lch[ch], e[ch]);
                        }
                    }
                    rc = fmin(t, v->max_distance);
                }
                if (c == 0) {
                    for (int ch = 0; ch < 3; ++ch) Ln[ch] = Lc[ch];
                    rn = rc;
                }
                for (int ch = 0; ch < 3; ++ch) {
                    Llo[ch] = fmin(Llo[ch], Lcl[ch]);
                    Lhi[ch] = fmax(Lhi[ch], Lch[ch]);
                }
                rlo = fmin(rlo, rc);
                rhi = fmax(rhi, rc);
            }
            for (int ch = 0; ch < 3; ++ch) {
                L_nom[3 * q + ch] = Ln[ch];
                if (L_lo) L_lo[3 * q + ch] = Llo[ch];
                if (L_hi) L_hi[3 * q + ch] = Lhi[ch];
            }
            r_nom[q] = rn;
            if (r_lo) r_lo[q] = rlo;
            if (r_hi) r_hi[q] = rhi;
            if (hit) hit[q] = h.tri;
            if (hit_t) hit_t[q] = h.t;
            if (cand && ncand) {
                int keep = nc < maxc ? nc : maxc;
                for (int c = 0; c < maxc; ++c) cand[q * maxc + c] = c < keep ? cands[c] : -2;
                ncand[q] = keep;
            }
        }
    }
    free(dirs);
    return 0;
}

/* Closest hit for arbitrary rays (for intersection pins). */
OR_API void or_closest_hits(const or_scene *s, int nrays, const double *o, const double *d, int32_t *tri,
                            double *t, int32_t *near, double margin)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < nrays; ++i) {
        or_hit h = closest_hit(s, o + 3 * i, d + 3 * i, 0.0, margin);
        tri[i] = h.tri;
        t[i] = h.t;
        if (near) near[i] = h.near;
    }
}

/* Brute-force closest hit over every triangle (no BVH), for pinning the BVH. */
OR_API void or_closest_hits_brute(const or_scene *s, int nrays, const double *o, const double *d, int32_t *tri,
                                  double *t)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < nrays; ++i) {
        int best = -1;
        double bt = INFINITY;
        for (int k = 0; k < s->ntri; ++k) {
            double tk, ed[3];
            if (!tri_isect(s, k, o + 3 * i, d + 3 * i, &tk, ed)) continue;
            if (tk > 0.0 && fmin(ed[0], fmin(ed[1], ed[2])) >= 0.0 && (tk < bt || (tk == bt && k < best))) {
                bt = tk;
                best = k;
            }
        }
        tri[i] = best;
        t[i] = bt;
    }
}

/* ======================================================================== */
/* Border (guard band) copy by the octahedral fold                            */
/* ======================================================================== */

/* One C-channel tile set [P][C][N+2][N+2] (doubles). The source of each
 * guard texel is the interior texel that the octahedral fold puts next to
 * it: across an edge the map continues mirrored (u -> -u on the top and
 * bottom edges, w -> -w on the left and right edges), and all four corners
 * of the square are the same direction. */
OR_API void or_border(int P, int C, int N, double *tiles)
{
    const int S = N + 2;
    for (int64_t pc = 0; pc < (int64_t)P * C; ++pc) {
        double *T = tiles + pc * S * S;
#define AT(x, y) T[(y) * S + (x)]
        for (int x = 1; x <= N; ++x) {
            AT(x, 0) = AT(N + 1 - x, 1);
            AT(x, N + 1) = AT(N + 1 - x, N);
        }
        for (int y = 1; y <= N; ++y) {
            AT(0, y) = AT(1, N + 1 - y);
            AT(N + 1, y) = AT(N, N + 1 - y);
        }
        AT(0, 0) = AT(N, N);
        AT(N + 1, 0) = AT(1, N);
        AT(0, N + 1) = AT(N, 1);
        AT(N + 1, N + 1) = AT(1, 1);
#undef AT
    }
}

/* ======================================================================== */
/* Blend with hysteresis                                                      */
/* ======================================================================== */

/*
 * est_irr[t][c] = sum_j w_tj L_jc / sum_j w_tj,      w_tj = max(0, omega_t . d_j)
 * est_vis[t]    = (sum_j v_tj r_j, sum_j v_tj r_j^2) / sum_j v_tj,  v_tj = w_tj^s
 * new = h*old + (1-h)*est (h = 0 on the first frame when requested); a texel
 * whose weight sum is at most OR_WEIGHT_FLOOR keeps its old value (no ray
 * lies in its lobe to any useful degree; the floor sits far above where FP32
 * weights underflow, so the decision does not depend on precision). With fp16 set each new value
 * is rounded to binary16 (ties to even) before it is stored. Then the guard
 * bands are rebuilt.
 * irr: [P][3][Ni+2][Ni+2], vis: [P][2][Nv+2][Nv+2], updated in place.
 */
#define OR_WEIGHT_FLOOR 1e-20

OR_API void or_blend_update(const or_volume *v, const double *dirs, const double *L, const double *r, int first,
                            int fp16, double *irr, double *vis, int nthreads)
{
    const int P = v->nx * v->ny * v->nz, n = v->n;
    const int Ni = v->irr_res, Nv = v->vis_res, Si = Ni + 2, Sv = Nv + 2;
    const double h = (first && v->first_frame_no_history) ? 0.0 : v->hysteresis;
    double *om_i = (double *)malloc(sizeof(double) * 3 * Ni * Ni);
    double *om_v = (double *)malloc(sizeof(double) * 3 * Nv * Nv);
    or_texel_dirs(Ni, om_i);
    or_texel_dirs(Nv, om_v);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < P; ++p) {
        const double *Lp = L + (int64_t)p * n * 3;
        const double *rp = r + (int64_t)p * n;
        for (int t = 0; t < Ni * Ni; ++t) {
            double acc[3] = {0, 0, 0}, ws = 0;
            for (int j = 0; j < n; ++j) {
                double c = om_i[3 * t] * dirs[3 * j] + om_i[3 * t + 1] * dirs[3 * j + 1] +
                           om_i[3 * t + 2] * dirs[3 * j + 2];
                double w = c > 0.0 ? c : 0.0;
                ws += w;
                for (int ch = 0; ch < 3; ++ch) acc[ch] += w * Lp[3 * j + ch];
            }
            int i = t % Ni, jj = t / Ni;
            for (int ch = 0; ch < 3; ++ch) {
                double *dst = irr + (((int64_t)p * 3 + ch) * Si + (jj + 1)) * Si + (i + 1);
                if (ws > OR_WEIGHT_FLOOR) {
                    double nv = h * (*dst) + (1.0 - h) * (acc[ch] / ws);
                    *dst = fp16 ? or_half_to_double(or_double_to_half(nv)) : nv;
                }
            }
        }
        for (int t = 0; t < Nv * Nv; ++t) {
            double a1 = 0, a2 = 0, ws = 0;
            for (int j = 0; j < n; ++j) {
                double c = om_v[3 * t] * dirs[3 * j] + om_v[3 * t + 1] * dirs[3 * j + 1] +
                           om_v[3 * t + 2] * dirs[3 * j + 2];
                double w = c > 0.0 ? pow(c, (double)v->vis_sharpness) : 0.0;
                ws += w;
                a1 += w * rp[j];
                a2 += w * rp[j] * rp[j];
            }
            int i = t % Nv, jj = t / Nv;
            double est[2] = {a1 / ws, a2 / ws};
            for (int ch = 0; ch < 2; ++ch) {
                double *dst = vis + (((int64_t)p * 2 + ch) * Sv + (jj + 1)) * Sv + (i + 1);
                if (ws > OR_WEIGHT_FLOOR) {
                    double nv = h * (*dst) + (1.0 - h) * est[ch];
                    *dst = fp16 ? or_half_to_double(or_double_to_half(nv)) : nv;
                }
            }
        }
    }
    or_border(P, 3, Ni, irr);
    or_border(P, 2, Nv, vis);
    free(om_i);
    free(om_v);
}

/* ======================================================================== */
/* Lossless delta pack (changed-probe selection, byte planes, index buffer)   */
/* ======================================================================== */

/*
 * Packet byte layout (all little endian):
 *   header (32 B): u32 magic 'PVPK' (0x4B505650), u16 version (1), u16 header
 *                  bytes (32), u32 client, u32 seq, u32 P, u32 K_irr,
 *                  u32 K_vis, u32 checksum
 *   index section: K_irr u16 (delta-coded changed irradiance probes), then
 *                  K_vis u16 (visibility), zero-padded to a multiple of 16 B
 *   irradiance planes: for c in (R,G,B), b in (low, high): K_irr * Ni^2 bytes,
 *                  byte (k*Ni^2 + t) = byte b of cur XOR byte b of ref for
 *                  the k-th changed probe, interior texel t (row-major)
 *   visibility planes: same for (mean, mean^2), Nv^2 texels.
 * Delta code: e_0 = idx_0, e_k = idx_k - idx_{k-1}.
 * checksum = sum over the payload's u32 words w_i of fmix32(w_i ^ (i * 0x9E3779B9)),
 *   modulo 2^32 (fmix32 = the MurmurHash3 32-bit finaliser).
 */
static uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

OR_API uint32_t or_payload_checksum(const uint8_t *payload, int64_t bytes)
{
    uint32_t sum = 0;
    for (int64_t i = 0; i < bytes / 4; ++i) {
        uint32_t w = (uint32_t)payload[4 * i] | ((uint32_t)payload[4 * i + 1] << 8) |
                     ((uint32_t)payload[4 * i + 2] << 16) | ((uint32_t)payload[4 * i + 3] << 24);
        sum += fmix32(w ^ (uint32_t)((uint32_t)i * 0x9E3779B9u));
    }
    return sum;
}

static void put_u32(uint8_t *p, uint32_t v)
{
    p[0] = v & 0xff;
    p[1] = (v >> 8) & 0xff;
    p[2] = (v >> 16) & 0xff;
    p[3] = (v >> 24) & 0xff;
}
static uint32_t get_u32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

/* Interior texel (c, t) of a tile set [P][C][N+2][N+2] (uint16). */
static uint16_t tile_interior(const uint16_t *tiles, int C, int N, int p, int c, int t)
{
    int S = N + 2;
    int i = t % N, j = t / N;
    return tiles[(((int64_t)p * C + c) * S + (j + 1)) * S + (i + 1)];
}

static int probe_changed(const uint16_t *cur, const uint16_t *ref, int C, int N, int p, double tau)
{
    for (int c = 0; c < C; ++c)
        for (int t = 0; t < N * N; ++t) {
            uint16_t a = tile_interior(cur, C, N, p, c, t);
            uint16_t b = ref[((int64_t)p * C + c) * N * N + t];
            if (tau == 0.0) {
                if (a != b) return 1;
            } else {
                if (fabs(or_half_to_double(a) - or_half_to_double(b)) > tau) return 1;
            }
        }
    return 0;
}

OR_API int64_t or_packet_bytes(int K_irr, int K_vis, int Ni, int Nv)
{
    int64_t idx = 2 * (int64_t)(K_irr + K_vis);
    idx = (idx + 15) / 16 * 16;
    return 32 + idx + (int64_t)K_irr * 6 * Ni * Ni + (int64_t)K_vis * 4 * Nv * Nv;
}

/*
 * cur_irr/cur_vis: current FP16 tiles (with guard bands);
 * ref_irr/ref_vis: the client's last-transmitted interiors [P][C][N*N]
 *                  (updated in place for the probes that are sent).
 * tau_* = 0: a probe is changed when any interior FP16 bit pattern differs;
 * tau_* > 0: when some |cur - ref| (exact, in double) is strictly > tau.
 * Returns the packet size, or -(needed size) when cap is too small (nothing
 * is modified then).
 */
OR_API int64_t or_pack(int P, int Ni, int Nv, const uint16_t *cur_irr, const uint16_t *cur_vis, uint16_t *ref_irr,
                       uint16_t *ref_vis, double tau_irr, double tau_vis, uint32_t client, uint32_t seq,
                       uint8_t *out, int64_t cap, uint8_t *mask_irr, uint8_t *mask_vis, const uint8_t *eligible)
{
    /* eligible (NULL: every probe): the probes that may be sent at all
     * (active, and in the client's view when one is set, Sec. 3.4) */
    uint8_t *mi = (uint8_t *)malloc(P > 0 ? P : 1), *mv = (uint8_t *)malloc(P > 0 ? P : 1);
    int K_irr = 0, K_vis = 0;
    for (int p = 0; p < P; ++p) {
        const int ok = eligible ? eligible[p] != 0 : 1;
        mi[p] = (uint8_t)(ok && probe_changed(cur_irr, ref_irr, 3, Ni, p, tau_irr));
        mv[p] = (uint8_t)(ok && probe_changed(cur_vis, ref_vis, 2, Nv, p, tau_vis));
        K_irr += mi[p];
        K_vis += mv[p];
    }
    if (mask_irr) memcpy(mask_irr, mi, P);
    if (mask_vis) memcpy(mask_vis, mv, P);
    int64_t total = or_packet_bytes(K_irr, K_vis, Ni, Nv);
    if (total > cap) {
        free(mi);
        free(mv);
        return -total;
    }
    memset(out, 0, total);
    uint8_t *hdr = out;
    put_u32(hdr + 0, 0x4B505650u);
    hdr[4] = 1;
    hdr[5] = 0;
    hdr[6] = 32;
    hdr[7] = 0;
    put_u32(hdr + 8, client);
    put_u32(hdr + 12, seq);
    put_u32(hdr + 16, (uint32_t)P);
    put_u32(hdr + 20, (uint32_t)K_irr);
    put_u32(hdr + 24, (uint32_t)K_vis);
    /* index buffers */
    uint8_t *ix = out + 32;
    int prev = 0, k = 0;
    for (int p = 0; p < P; ++p)
        if (mi[p]) {
            uint16_t e = (uint16_t)(k == 0 ? p : p - prev);
            ix[2 * k] = e & 0xff;
            ix[2 * k + 1] = e >> 8;
            prev = p;
            ++k;
        }
    prev = 0;
    k = 0;
    for (int p = 0; p < P; ++p)
        if (mv[p]) {
            uint16_t e = (uint16_t)(k == 0 ? p : p - prev);
            ix[2 * (K_irr + k)] = e & 0xff;
            ix[2 * (K_irr + k) + 1] = e >> 8;
            prev = p;
            ++k;
        }
    int64_t idx_bytes = (2 * (int64_t)(K_irr + K_vis) + 15) / 16 * 16;
    uint8_t *planes_irr = out + 32 + idx_bytes;
    uint8_t *planes_vis = planes_irr + (int64_t)K_irr * 6 * Ni * Ni;
    /* irradiance planes + reference update */
    k = 0;
    for (int p = 0; p < P; ++p) {
        if (!mi[p]) continue;
        for (int c = 0; c < 3; ++c)
            for (int t = 0; t < Ni * Ni; ++t) {
                uint16_t a = tile_interior(cur_irr, 3, Ni, p, c, t);
                uint16_t *rf = &ref_irr[((int64_t)p * 3 + c) * Ni * Ni + t];
                uint16_t x = a ^ *rf;
                planes_irr[(int64_t)(2 * c + 0) * K_irr * Ni * Ni + (int64_t)k * Ni * Ni + t] = x & 0xff;
                planes_irr[(int64_t)(2 * c + 1) * K_irr * Ni * Ni + (int64_t)k * Ni * Ni + t] = x >> 8;
                *rf = a;
            }
        ++k;
    }
    k = 0;
    for (int p = 0; p < P; ++p) {
        if (!mv[p]) continue;
        for (int c = 0; c < 2; ++c)
            for (int t = 0; t < Nv * Nv; ++t) {
                uint16_t a = tile_interior(cur_vis, 2, Nv, p, c, t);
                uint16_t *rf = &ref_vis[((int64_t)p * 2 + c) * Nv * Nv + t];
                uint16_t x = a ^ *rf;
                planes_vis[(int64_t)(2 * c + 0) * K_vis * Nv * Nv + (int64_t)k * Nv * Nv + t] = x & 0xff;
                planes_vis[(int64_t)(2 * c + 1) * K_vis * Nv * Nv + (int64_t)k * Nv * Nv + t] = x >> 8;
                *rf = a;
            }
        ++k;
    }
    put_u32(hdr + 28, or_payload_checksum(out + 32, total - 32));
    free(mi);
    free(mv);
    return total;
}

/*
 * Client side of the round trip: verify and apply a packet to the client's
 * FP16 tiles [P][C][N+2][N+2] (XOR into the interiors of the listed probes,
 * then rebuild every guard band). Returns 0 on success, <0 on a malformed
 * packet (1 = bad magic/size, 2 = checksum, 3 = probe count, 4 = index).
 * *seq_out receives the packet's sequence number.
 */
OR_API int or_client_apply(const uint8_t *pkt, int64_t bytes, int P, int Ni, int Nv, uint16_t *cli_irr,
                           uint16_t *cli_vis, uint32_t *seq_out)
{
    if (bytes < 32 || get_u32(pkt) != 0x4B505650u) return -1;
    int K_irr = (int)get_u32(pkt + 20), K_vis = (int)get_u32(pkt + 24);
    if ((int)get_u32(pkt + 16) != P) return -3;
    if (K_irr > P || K_vis > P || or_packet_bytes(K_irr, K_vis, Ni, Nv) != bytes) return -1;
    if (or_payload_checksum(pkt + 32, bytes - 32) != get_u32(pkt + 28)) return -2;
    if (seq_out) *seq_out = get_u32(pkt + 12);
    const uint8_t *ix = pkt + 32;
    int64_t idx_bytes = (2 * (int64_t)(K_irr + K_vis) + 15) / 16 * 16;
    const uint8_t *pi = pkt + 32 + idx_bytes;
    const uint8_t *pv = pi + (int64_t)K_irr * 6 * Ni * Ni;
    for (int pass = 0; pass < 2; ++pass) {
        int K = pass ? K_vis : K_irr, C = pass ? 2 : 3, N = pass ? Nv : Ni;
        const uint8_t *pl = pass ? pv : pi;
        const uint8_t *ixs = ix + 2 * (pass ? K_irr : 0);
        uint16_t *tiles = pass ? cli_vis : cli_irr;
        int S = N + 2;
        int p = 0;
        for (int k = 0; k < K; ++k) {
            int e = ixs[2 * k] | (ixs[2 * k + 1] << 8);
            p = k == 0 ? e : p + e;
            if (p >= P || (k > 0 && e == 0)) return -4;
            for (int c = 0; c < C; ++c)
                for (int t = 0; t < N * N; ++t) {
                    uint16_t lo = pl[(int64_t)(2 * c) * K * N * N + (int64_t)k * N * N + t];
                    uint16_t hi = pl[(int64_t)(2 * c + 1) * K * N * N + (int64_t)k * N * N + t];
                    int i = t % N, j = t / N;
                    tiles[(((int64_t)p * C + c) * S + (j + 1)) * S + (i + 1)] ^= (uint16_t)(lo | (hi << 8));
                }
        }
    }
    /* guard bands of the uint16 tiles (same fold as or_border) */
    for (int pass = 0; pass < 2; ++pass) {
        int C = pass ? 2 : 3, N = pass ? Nv : Ni, S = N + 2;
        uint16_t *tiles = pass ? cli_vis : cli_irr;
        for (int64_t pc = 0; pc < (int64_t)P * C; ++pc) {
            uint16_t *T = tiles + pc * S * S;
#define AT(x, y) T[(y) * S + (x)]
            for (int x = 1; x <= N; ++x) {
                AT(x, 0) = AT(N + 1 - x, 1);
                AT(x, N + 1) = AT(N + 1 - x, N);
            }
            for (int y = 1; y <= N; ++y) {
                AT(0, y) = AT(1, N + 1 - y);
                AT(N + 1, y) = AT(N, N + 1 - y);
            }
            AT(0, 0) = AT(N, N);
            AT(N + 1, 0) = AT(1, N);
            AT(0, N + 1) = AT(N, 1);
            AT(N + 1, N + 1) = AT(1, 1);
#undef AT
        }
    }
    return 0;
}

OR_API int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ======================================================================== */
/* Codec surfaces (Sec. 3.3, memory layout figure)                           */
/* ======================================================================== */
/*
 * Probe p occupies atlas tile (p % C, p / C); unused tiles of the last row
 * are zero. Guard bands are not part of the surfaces (Sec. 3.4 repacking).
 *
 * Irradiance: each channel's normalised value becomes a 10-bit unsigned
 * code, shifted into the top 10 bits of a 16-bit sample (low 6 bits zero);
 * R, G, B are the Y, U, V planes of a YUV444 surface, each [8 rows][8 C]
 * per atlas row of tiles. The code is decided in FP32: the FP32 product of
 * the value and k (the FP32 value nearest 1023 / scale), rounded to the
 * nearest integer (ties to even), clamped to [0, 1023].
 *
 * Visibility: a row of x RG16F texels is 4x bytes (per texel mean lo, mean
 * hi, mean^2 lo, mean^2 hi); byte m goes to YUV sample m / 3, channel m % 3
 * (Y, U, V), so three texels fill four YUV samples (YUVY, UVYU, VYUV) and a
 * plane row holds ceil(4x / 3) samples (x = 16 C), missing bytes zero.
 */
static int ceil_div(int a, int b) { return (a + b - 1) / b; }

OR_API void or_yuv_dims(int P, int C, int64_t out[4])
{
    const int rows = ceil_div(P, C);
    out[0] = 8 * (int64_t)C;                 /* irradiance plane width */
    out[1] = 8 * (int64_t)rows;              /* irradiance plane height */
    out[2] = ceil_div(4 * 16 * C, 3);        /* visibility plane width x' */
    out[3] = 16 * (int64_t)rows;             /* visibility plane height */
}

OR_API uint16_t or_irr_code(float v, float k)
{
    float x = v * k;
    x = rintf(x);
    if (!(x > 0.0f)) return 0;
    if (x > 1023.0f) return 1023;
    return (uint16_t)x;
}

/* irr: FP16-valued tiles as doubles [P][3][10][10]; vis: binary16 bit
 * patterns [P][2][18][18]. */
OR_API void or_yuv_encode(int P, int C, const double *irr, const uint16_t *vis, float k, uint16_t *irr_planes,
                          uint8_t *vis_planes)
{
    int64_t d[4];
    or_yuv_dims(P, C, d);
    const int64_t W = d[0], H = d[1], Wv = d[2], Hv = d[3];
    memset(irr_planes, 0, sizeof(uint16_t) * 3 * W * H);
    memset(vis_planes, 0, 3 * Wv * Hv);
    for (int p = 0; p < P; ++p) {
        const int tx = p % C, ty = p / C;
        for (int c = 0; c < 3; ++c)
            for (int j = 0; j < 8; ++j)
                for (int i = 0; i < 8; ++i) {
                    const float v = (float)irr[(((int64_t)p * 3 + c) * 10 + j + 1) * 10 + i + 1];
                    irr_planes[((int64_t)c * H + ty * 8 + j) * W + tx * 8 + i] = (uint16_t)(or_irr_code(v, k) << 6);
                }
        for (int j = 0; j < 16; ++j)
            for (int i = 0; i < 16; ++i) {
                const int64_t row = (int64_t)ty * 16 + j, col = (int64_t)tx * 16 + i;
                for (int b = 0; b < 4; ++b) {
                    const uint16_t h = vis[(((int64_t)p * 2 + b / 2) * 18 + j + 1) * 18 + i + 1];
                    const uint8_t byte = (uint8_t)(b % 2 ? h >> 8 : h & 0xFF);
                    const int64_t m = 4 * col + b;
                    vis_planes[((m % 3) * Hv + row) * Wv + m / 3] = byte;
                }
            }
    }
}

/* Inverse: irr_codes [P][64] = R | G << 10 | B << 20 (A2RGB10, alpha 0),
 * vis_bits [P][2][256] binary16 interiors. */
OR_API void or_yuv_decode(int P, int C, const uint16_t *irr_planes, const uint8_t *vis_planes, uint32_t *irr_codes,
                          uint16_t *vis_bits)
{
    int64_t d[4];
    or_yuv_dims(P, C, d);
    const int64_t W = d[0], H = d[1], Wv = d[2], Hv = d[3];
    for (int p = 0; p < P; ++p) {
        const int tx = p % C, ty = p / C;
        for (int t = 0; t < 64; ++t) {
            const int i = t % 8, j = t / 8;
            uint32_t code = 0;
            for (int c = 0; c < 3; ++c)
                code |= (uint32_t)(irr_planes[((int64_t)c * H + ty * 8 + j) * W + tx * 8 + i] >> 6) << (10 * c);
            irr_codes[(int64_t)p * 64 + t] = code;
        }
        for (int t = 0; t < 256; ++t) {
            const int i = t % 16, j = t / 16;
            const int64_t row = (int64_t)ty * 16 + j, col = (int64_t)tx * 16 + i;
            uint8_t by[4];
            for (int b = 0; b < 4; ++b) {
                const int64_t m = 4 * col + b;
                by[b] = vis_planes[((m % 3) * Hv + row) * Wv + m / 3];
            }
            vis_bits[((int64_t)p * 2 + 0) * 256 + t] = (uint16_t)(by[0] | (by[1] << 8));
            vis_bits[((int64_t)p * 2 + 1) * 256 + t] = (uint16_t)(by[2] | (by[3] << 8));
        }
    }
}

/* ======================================================================== */
/* Entropy stage: canonical Huffman coding of the packet's byte streams      */
/* ======================================================================== */
/*
 * Streams of a packet: 0 = the index section (2 (K_irr + K_vis) bytes, no
 * padding), 1..6 = the irradiance planes (K_irr * 64 bytes each), 7..10 =
 * the visibility planes (K_vis * 256 bytes each). Each stream gets its own
 * code over byte symbols:
 *   - code lengths by Huffman's algorithm over the symbols that occur,
 *     merging the two lightest nodes first, leaves before internal nodes
 *     on equal weight, leaves ordered by (count, symbol); a single symbol
 *     gets length 1; if the longest code exceeds OR_HUF_MAX bits, every
 *     count is halved (rounded up) and the lengths rebuilt;
 *   - canonical codes: symbols sorted by (length, symbol), each code the
 *     previous plus one, shifted left by the length difference;
 *   - the stream is cut into chunks of OR_HUF_CHUNK symbols, each coded
 *     most significant bit first and padded to a multiple of 32 bits.
 * Container: u32 magic 0x43485650 ("PVHC"), u32 version 1, the 32-byte
 * packet header, then per stream: u8 lengths[256] as 128 bytes of nibbles
 * (symbol 2i in the low nibble), u32 n_chunks, u32 bits[n_chunks], then the
 * chunks' 32-bit words, chunk after chunk (each word's bytes in big-endian
 * order, i.e. the bit stream's byte order).
 */
#define OR_HUF_MAX 12
#define OR_HUF_CHUNK 1024
#define OR_HUF_STREAMS 11

typedef struct {
    int64_t w;
    int sym;   /* leaf symbol, or -1 */
    int a, b;  /* children (internal) */
} or_hnode;

static int cmp_leaf(const void *x, const void *y)
{
    const or_hnode *p = (const or_hnode *)x, *q = (const or_hnode *)y;
    if (p->w != q->w) return p->w < q->w ? -1 : 1;
    return p->sym - q->sym;
}

static void huf_depths(const or_hnode *nd, int i, int d, uint8_t *len)
{
    if (nd[i].sym >= 0) {
        len[nd[i].sym] = (uint8_t)(d > 0 ? d : 1);
        return;
    }
    huf_depths(nd, nd[i].a, d + 1, len);
    huf_depths(nd, nd[i].b, d + 1, len);
}

/* Code lengths of a histogram (0 for absent symbols). */
OR_API void or_huf_lengths(const uint64_t hist[256], uint8_t len[256])
{
    int64_t h[256];
    for (int s = 0; s < 256; ++s) h[s] = (int64_t)hist[s];
    for (;;) {
        or_hnode nd[512];
        int nl = 0;
        for (int s = 0; s < 256; ++s)
            if (h[s] > 0) {
                nd[nl].w = h[s];
                nd[nl].sym = s;
                nd[nl].a = nd[nl].b = -1;
                ++nl;
            }
        memset(len, 0, 256);
        if (nl == 0) return;
        qsort(nd, nl, sizeof(or_hnode), cmp_leaf);
        /* two queues: leaves nd[0..nl), internal nodes appended after them */
        int li = 0, ii = nl, ie = nl;
        while ((nl - li) + (ie - ii) > 1) {
            int pick[2];
            for (int k = 0; k < 2; ++k) {
                if (li < nl && (ii >= ie || nd[li].w <= nd[ii].w))
                    pick[k] = li++;
                else
                    pick[k] = ii++;
            }
            nd[ie].w = nd[pick[0]].w + nd[pick[1]].w;
            nd[ie].sym = -1;
            nd[ie].a = pick[0];
            nd[ie].b = pick[1];
            ++ie;
        }
        huf_depths(nd, ie - 1, 0, len);
        int mx = 0;
        for (int s = 0; s < 256; ++s) mx = len[s] > mx ? len[s] : mx;
        if (mx <= OR_HUF_MAX) return;
        for (int s = 0; s < 256; ++s) h[s] = (h[s] + 1) / 2;
    }
}

/* Canonical codes of a length table. */
OR_API void or_huf_codes(const uint8_t len[256], uint32_t code[256])
{
    uint32_t c = 0;
    int prev = 0, first = 1;
    for (int L = 1; L <= OR_HUF_MAX; ++L)
        for (int s = 0; s < 256; ++s)
            if (len[s] == L) {
                if (first) {
                    c = 0;
                    first = 0;
                } else {
                    c = (c + 1) << (L - prev);
                }
                prev = L;
                code[s] = c;
            }
    for (int s = 0; s < 256; ++s)
        if (!len[s]) code[s] = 0;
}

static void stream_span(const uint8_t *pkt, int k, const uint8_t **p, int64_t *n)
{
    const int64_t Ki = get_u32(pkt + 20), Kv = get_u32(pkt + 24);
    const int64_t idx = (2 * (Ki + Kv) + 15) / 16 * 16;
    if (k == 0) {
        *p = pkt + 32;
        *n = 2 * (Ki + Kv);
    } else if (k <= 6) {
        *p = pkt + 32 + idx + (int64_t)(k - 1) * Ki * 64;
        *n = Ki * 64;
    } else {
        *p = pkt + 32 + idx + 6 * Ki * 64 + (int64_t)(k - 7) * Kv * 256;
        *n = Kv * 256;
    }
}

/* Encodes a packet; returns the container size (or -size needed when cap is
 * too small). */
OR_API int64_t or_huf_encode(const uint8_t *pkt, uint8_t *out, int64_t cap)
{
    int64_t total = 8 + 32;
    uint8_t lens[OR_HUF_STREAMS][256];
    uint32_t codes[OR_HUF_STREAMS][256];
    for (int k = 0; k < OR_HUF_STREAMS; ++k) {
        const uint8_t *p;
        int64_t n;
        stream_span(pkt, k, &p, &n);
        uint64_t hist[256] = {0};
        for (int64_t i = 0; i < n; ++i) hist[p[i]]++;
        or_huf_lengths(hist, lens[k]);
        or_huf_codes(lens[k], codes[k]);
        const int64_t nch = (n + OR_HUF_CHUNK - 1) / OR_HUF_CHUNK;
        total += 128 + 4 + 4 * nch;
        for (int64_t c = 0; c < nch; ++c) {
            int64_t bits = 0;
            for (int64_t i = c * OR_HUF_CHUNK; i < n && i < (c + 1) * OR_HUF_CHUNK; ++i) bits += lens[k][p[i]];
            total += (bits + 31) / 32 * 4;
        }
    }
    if (total > cap) return -total;
    memset(out, 0, total);
    put_u32(out, 0x43485650u);
    put_u32(out + 4, 1u);
    memcpy(out + 8, pkt, 32);
    uint8_t *w = out + 40;
    for (int k = 0; k < OR_HUF_STREAMS; ++k) {
        const uint8_t *p;
        int64_t n;
        stream_span(pkt, k, &p, &n);
        for (int i = 0; i < 128; ++i) w[i] = (uint8_t)(lens[k][2 * i] | (lens[k][2 * i + 1] << 4));
        w += 128;
        const int64_t nch = (n + OR_HUF_CHUNK - 1) / OR_HUF_CHUNK;
        put_u32(w, (uint32_t)nch);
        uint8_t *bits_tab = w + 4;
        w += 4 + 4 * nch;
        for (int64_t c = 0; c < nch; ++c) {
            int64_t bit = 0;
            for (int64_t i = c * OR_HUF_CHUNK; i < n && i < (c + 1) * OR_HUF_CHUNK; ++i) {
                const int L = lens[k][p[i]];
                const uint32_t cd = codes[k][p[i]];
                for (int b = L - 1; b >= 0; --b, ++bit)
                    if ((cd >> b) & 1u) w[bit >> 3] |= (uint8_t)(0x80u >> (bit & 7));
            }
            put_u32(bits_tab + 4 * c, (uint32_t)bit);
            w += (bit + 31) / 32 * 4;
        }
    }
    return total;
}

/* Decodes a container back into the packet (its size from the header);
 * returns the packet size, or -1 on a malformed container. */
OR_API int64_t or_huf_decode(const uint8_t *in, int64_t bytes, uint8_t *pkt, int64_t cap)
{
    if (bytes < 40 || get_u32(in) != 0x43485650u || get_u32(in + 4) != 1u) return -1;
    const uint8_t *hdr = in + 8;
    const int64_t Ki = get_u32(hdr + 20), Kv = get_u32(hdr + 24);
    const int64_t size = or_packet_bytes((int)Ki, (int)Kv, 8, 16);
    if (size > cap) return -1;
    memset(pkt, 0, size);
    memcpy(pkt, hdr, 32);
    const uint8_t *r = in + 40, *end = in + bytes;
    for (int k = 0; k < OR_HUF_STREAMS; ++k) {
        const uint8_t *p;
        int64_t n;
        stream_span(pkt, k, &p, &n);
        uint8_t *dst = (uint8_t *)p;
        if (r + 132 > end) return -1;
        uint8_t len[256];
        uint32_t code[256];
        for (int i = 0; i < 128; ++i) {
            len[2 * i] = r[i] & 15;
            len[2 * i + 1] = r[i] >> 4;
        }
        or_huf_codes(len, code);
        r += 128;
        const int64_t nch = get_u32(r);
        if (nch != (n + OR_HUF_CHUNK - 1) / OR_HUF_CHUNK) return -1;
        const uint8_t *bits_tab = r + 4;
        r += 4 + 4 * nch;
        for (int64_t c = 0; c < nch; ++c) {
            const int64_t nbits = get_u32(bits_tab + 4 * c);
            if (r + (nbits + 31) / 32 * 4 > end) return -1;
            int64_t bit = 0;
            for (int64_t i = c * OR_HUF_CHUNK; i < n && i < (c + 1) * OR_HUF_CHUNK; ++i) {
                /* read bit by bit until a code matches (plain prefix decoding) */
                uint32_t acc = 0;
                int L = 0, found = -1;
                while (found < 0) {
                    if (L >= OR_HUF_MAX || bit >= nbits) return -1;
                    acc = (acc << 1) | ((r[bit >> 3] >> (7 - (bit & 7))) & 1u);
                    ++bit;
                    ++L;
                    for (int s = 0; s < 256 && found < 0; ++s)
                        if (len[s] == L && code[s] == acc) found = s;
                }
                dst[i] = (uint8_t)found;
            }
            r += (nbits + 31) / 32 * 4;
        }
    }
    /* the index section's padding is zero by the packet format */
    return size;
}
