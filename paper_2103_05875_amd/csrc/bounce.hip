// Second bounce of an update and the shading query of a volume (Sec. 3.2).
//
//   k_bounce         after the trace: every hit adds its albedo times the
//                    query of the maps as they stand before this frame's
//                    blend (the previous frame's result); one thread a ray
//   k_bounce_batched the same over every volume of a batch that asks for it
//   k_probe_query    a client's shading query at given points and normals
//
// The query gathers from eight probes' tiles per point; the maps of a volume
// are a few MB and stay in L2, so the kernels are bound by the gathers, not
// by HBM. Threads of a block take consecutive rays, i.e. rays of one or two
// probes, which share their eight probes.
#include "probe_query.h"

namespace pv {

constexpr int kBounceThreads = 256;

template <typename T>
__global__ __launch_bounds__(kBounceThreads) void k_bounce(VolumeParams vp, SceneView sv, const float4 *dirs,
                                                           float4 *rays, const T *irr, const T *vis) {
    const long long q = (long long)xcd_logical_block() * kBounceThreads + threadIdx.x;
    if (q >= (long long)vp.P * vp.n) return;
    bounce_one<T>(vp, sv, dirs, rays, irr, vis, (int)q);
}

// Last volume whose first bounce block is at or before 'item' (prefix counts
// ascending; a volume without the second bounce has no blocks and shares its
// first block number with the next volume, which the search then picks).
__device__ __forceinline__ int find_bounce_volume(const BatchVolume *vols, int n_vols, int item) {
    int lo = 0, hi = n_vols - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vols[mid].first_bounce <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBounceThreads) void k_bounce_batched(const BatchVolume *vols, int n_vols) {
    const int g = xcd_logical_block();
    const int v = __builtin_amdgcn_readfirstlane(find_bounce_volume(vols, n_vols, g));
    const BatchVolume &bv = vols[v];
    const long long q = (long long)(g - bv.first_bounce) * kBounceThreads + threadIdx.x;
    if (q >= (long long)bv.vp.P * bv.vp.n) return;
    if (bv.fp16)
        bounce_one<__half>(bv.vp, bv.sv, bv.dirs, bv.rays, (const __half *)bv.irr, (const __half *)bv.vis, (int)q);
    else
        bounce_one<float>(bv.vp, bv.sv, bv.dirs, bv.rays, (const float *)bv.irr, (const float *)bv.vis, (int)q);
}

template <typename T>
__global__ __launch_bounds__(kBounceThreads) void k_probe_query(VolumeParams vp, const T *irr, const T *vis,
                                                                const float *pts, const float *nrms, float *out,
                                                                long long n) {
    const long long i = (long long)blockIdx.x * kBounceThreads + threadIdx.x;
    if (i >= n) return;
    const float3 x = make_float3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
    const float3 nn = make_float3(nrms[3 * i], nrms[3 * i + 1], nrms[3 * i + 2]);
    const float3 e = probe_query<T>(vp, irr, vis, x, nn);
    out[3 * i] = e.x;
    out[3 * i + 1] = e.y;
    out[3 * i + 2] = e.z;
}

int bounce_blocks(int P, int n) { return (int)(((long long)P * n + kBounceThreads - 1) / kBounceThreads); }

hipError_t launch_bounce(const VolumeParams &vp, const SceneView &sv, const float4 *dirs, float4 *rays,
                         const void *irr, const void *vis, int fp16, hipStream_t s) {
    const dim3 grid(bounce_blocks(vp.P, vp.n));
    if (fp16)
        hipLaunchKernelGGL(k_bounce<__half>, grid, dim3(kBounceThreads), 0, s, vp, sv, dirs, rays,
                           (const __half *)irr, (const __half *)vis);
    else
        hipLaunchKernelGGL(k_bounce<float>, grid, dim3(kBounceThreads), 0, s, vp, sv, dirs, rays,
                           (const float *)irr, (const float *)vis);
    return hipGetLastError();
}

hipError_t launch_bounce_batched(const BatchVolume *vols_dev, int n_vols, int total_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_bounce_batched, dim3(total_blocks), dim3(kBounceThreads), 0, s, vols_dev, n_vols);
    return hipGetLastError();
}

hipError_t launch_probe_query(const VolumeParams &vp, const void *irr, const void *vis, int fp16, const float *pts,
                              const float *nrms, float *out, long long n, hipStream_t s) {
    const dim3 grid((unsigned)((n + kBounceThreads - 1) / kBounceThreads));
    if (fp16)
        hipLaunchKernelGGL(k_probe_query<__half>, grid, dim3(kBounceThreads), 0, s, vp, (const __half *)irr,
                           (const __half *)vis, pts, nrms, out, n);
    else
        hipLaunchKernelGGL(k_probe_query<float>, grid, dim3(kBounceThreads), 0, s, vp, (const float *)irr,
                           (const float *)vis, pts, nrms, out, n);
    return hipGetLastError();
}

}  // namespace pv
