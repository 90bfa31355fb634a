// Shading-time query of a probe volume, device side (Sec. 3.2: the stored
// mean and mean-squared distances weight each probe by a Chebyshev test).
//
// The mean radiance arriving at a point x around a normal n is a weighted
// mean over the eight probes at the corners of the grid cell holding x
// (clamped to the grid): each probe's weight is its trilinear weight, times
// var / (var + (d - mu)^2) when the point lies beyond the probe's mean
// recorded distance mu in its direction (d = |x - probe|, var = mu2 - mu^2 of
// the bilinearly filtered visibility moments); its value is its irradiance
// tile filtered bilinearly in the direction n. The guard bands make the
// bilinear footprint valid at every direction. All four texel fetches of a
// lookup use one integer offset into the tile.
#pragma once

#include "blend_device.h"
#include "trace_device.h"

namespace pv {

constexpr int kIrrN = 8;    // irradiance interior resolution
constexpr int kVisN = 16;   // visibility interior resolution

// Octahedral coordinates of a non-zero vector (Cigolle et al. 2014; the sign
// of zero is +1, the lower hemisphere folds outwards).
__device__ __forceinline__ float2 oct_encode(float3 v) {
    const float s = fabsf(v.x) + fabsf(v.y) + fabsf(v.z);
    float px = v.x / s, py = v.y / s;
    if (v.z < 0.f) {
        const float qx = (1.f - fabsf(py)) * (px >= 0.f ? 1.f : -1.f);
        const float qy = (1.f - fabsf(px)) * (py >= 0.f ? 1.f : -1.f);
        px = qx;
        py = qy;
    }
    return make_float2(px, py);
}

// Bilinear footprint of octahedral coordinates in an N x N tile with guard
// band: interior texel i is centred at tile coordinate i + 1, so the lower
// left texel of the footprint lies in [0, N] on both axes.
struct Footprint {
    int off;      // y0 * (N + 2) + x0
    float fx, fy;
};

template <int N>
__device__ __forceinline__ Footprint footprint(float2 uv) {
    const float sx = (uv.x + 1.f) * 0.5f * N + 0.5f, sy = (uv.y + 1.f) * 0.5f * N + 0.5f;
    int x0 = (int)floorf(sx), y0 = (int)floorf(sy);
    x0 = min(max(x0, 0), N);
    y0 = min(max(y0, 0), N);
    Footprint f;
    f.off = y0 * (N + 2) + x0;
    f.fx = sx - (float)x0;
    f.fy = sy - (float)y0;
    return f;
}

template <int N, typename T>
__device__ __forceinline__ float bilinear(const T *plane, const Footprint &f) {
    const float a = load_map<T>(plane + f.off), b = load_map<T>(plane + f.off + 1);
    const float e = load_map<T>(plane + f.off + N + 2), g = load_map<T>(plane + f.off + N + 3);
    return (1.f - f.fy) * ((1.f - f.fx) * a + f.fx * b) + f.fy * ((1.f - f.fx) * e + f.fx * g);
}

// Grid cell of x on one axis: first corner index and the fraction towards
// the second (both clamped; a one-probe axis has no second corner).
__device__ __forceinline__ void cell_axis(float x, float o, float s, int dim, int &c, float &f) {
    if (dim == 1) {
        c = 0;
        f = 0.f;
        return;
    }
    const float g = (x - o) / s;
    c = min(max((int)floorf(g), 0), dim - 2);
    f = fminf(fmaxf(g - (float)c, 0.f), 1.f);
}

template <typename T>
__device__ float3 probe_query(const VolumeParams &vp, const T *irr, const T *vis, float3 x, float3 n) {
    constexpr int Si = (kIrrN + 2) * (kIrrN + 2), Sv = (kVisN + 2) * (kVisN + 2);
    int cx, cy, cz;
    float fx, fy, fz;
    cell_axis(x.x, vp.ox, vp.sx, vp.nx, cx, fx);
    cell_axis(x.y, vp.oy, vp.sy, vp.ny, cy, fy);
    cell_axis(x.z, vp.oz, vp.sz, vp.nz, cz, fz);
    const Footprint fi = footprint<kIrrN>(oct_encode(n));
    float3 acc = make_float3(0.f, 0.f, 0.f);
    float wsum = 0.f;
    for (int corner = 0; corner < 8; ++corner) {
        const int bx = corner & 1, by = (corner >> 1) & 1, bz = corner >> 2;
        if ((bx && vp.nx == 1) || (by && vp.ny == 1) || (bz && vp.nz == 1)) continue;
        float w = (bx ? fx : 1.f - fx) * (by ? fy : 1.f - fy) * (bz ? fz : 1.f - fz);
        const int p = (cx + bx) + vp.nx * ((cy + by) + vp.ny * (cz + bz));
        const float3 v = x - probe_origin(vp, p);
        const float dist = sqrtf(dot3(v, v));
        if (dist > 0.f) {
            const Footprint fv = footprint<kVisN>(oct_encode(v));
            const T *tv = vis + (size_t)p * 2 * Sv;
            const float mu = bilinear<kVisN>(tv, fv), mu2 = bilinear<kVisN>(tv + Sv, fv);
            if (dist > mu) {
                const float var = fmaxf(fmaf(-mu, mu, mu2), 0.f);
                const float dd = dist - mu;
                w *= var > 0.f ? var / (var + dd * dd) : 0.f;
            }
        }
        const T *ti = irr + (size_t)p * 3 * Si;
        acc.x += w * bilinear<kIrrN>(ti, fi);
        acc.y += w * bilinear<kIrrN>(ti + Si, fi);
        acc.z += w * bilinear<kIrrN>(ti + 2 * Si, fi);
        wsum += w;
    }
    if (!(wsum > kWeightFloor)) return make_float3(0.f, 0.f, 0.f);
    return make_float3(acc.x / wsum, acc.y / wsum, acc.z / wsum);
}

// Distance by which the second bounce moves a hit point off its surface
// along the normal before the query: a tenth of the smallest probe spacing.
__device__ __forceinline__ float bounce_bias(const VolumeParams &vp) {
    return 0.1f * fminf(vp.sx, fminf(vp.sy, vp.sz));
}

// Second bounce of ray record q: albedo times the query of the stored maps
// at the biased hit point, added to the record's radiance.
template <typename T>
__device__ __forceinline__ void bounce_one(const VolumeParams &vp, const SceneView &sv, const float4 *dirs,
                                           float4 *rays, const T *irr, const T *vis, int q) {
    const int2 rec = vp.hitrec[q];
    if (rec.x == -1) return;
    const bool dyn = rec.x < 0;
    const GpuTri tri = (dyn ? sv.dyn.tris : sv.stat.tris)[rec.x & 0x7fffffff];
    const int p = q / vp.n, j = q - p * vp.n;
    const float3 o = probe_origin(vp, p);
    const Ray ray = make_ray(o, xyz(dirs[j]));
    float3 nrm, xh;
    hit_frame(tri, ray, o, __int_as_float(rec.y), nrm, xh);
    const float b = bounce_bias(vp);
    const float3 xb = make_float3(fmaf(b, nrm.x, xh.x), fmaf(b, nrm.y, xh.y), fmaf(b, nrm.z, xh.z));
    const float3 e = probe_query<T>(vp, irr, vis, xb, nrm);
    const float4 alb = sv.mats[2 * tri_id(tri)];
    float4 r = rays[q];
    r.x += alb.x * e.x;
    r.y += alb.y * e.y;
    r.z += alb.z * e.z;
    rays[q] = r;
}

}  // namespace pv
