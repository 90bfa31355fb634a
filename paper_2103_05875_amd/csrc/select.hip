// Probe selection (Sec. 3.4): which probes a client is sent at all.
//
//   k_classify     per probe, from the frame's hit records: inactive when
//                  more than a quarter of its rays hit a triangle from
//                  behind (the probe sits inside a solid) or when none hits
//                  anything closer than the cell diagonal (no surface near
//                  enough for it to shade); one wavefront per probe
//   k_client_view  a spherical view from the client's position: closest hit
//                  of each spherical-Fibonacci direction, and every probe at
//                  a corner of the grid cell holding the hit point marked as
//                  potentially visible; one thread per ray
// The pack then sends a changed probe only when it is active and (once a
// view is set) in the client's view.
#include "probe_query.h"

namespace pv {

constexpr int kClassifyThreads = 256;  // four probes per block
constexpr int kViewThreads = 64;

// Probe p, one wavefront.
__device__ __forceinline__ void classify_probe(const VolumeParams &vp, const SceneView &sv, const float4 *dirs,
                                               uint8_t *active, int p, int lane) {
    const float diag = sqrtf(vp.sx * vp.sx + vp.sy * vp.sy + vp.sz * vp.sz);
    int back = 0;
    bool near = false;
    for (int j = lane; j < vp.n; j += 64) {
        const int2 rec = vp.hitrec[(size_t)p * vp.n + j];
        if (rec.x == -1) continue;
        const GpuTri tri = (rec.x < 0 ? sv.dyn.tris : sv.stat.tris)[rec.x & 0x7fffffff];
        const float3 nrm = cross3(xyz(tri.v1) - xyz(tri.v0), xyz(tri.v2) - xyz(tri.v0));
        back += dot3(nrm, xyz(dirs[j])) > 0.f ? 1 : 0;
        near |= __int_as_float(rec.y) < diag;
    }
    for (int off = 32; off > 0; off >>= 1) back += __shfl_xor(back, off);
    const bool any_near = __ballot(near) != 0ull;
    if (lane == 0) active[p] = (uint8_t)(4 * back <= vp.n && any_near);
}

__global__ __launch_bounds__(kClassifyThreads) void k_classify(VolumeParams vp, SceneView sv, const float4 *dirs,
                                                               uint8_t *active) {
    const int p = blockIdx.x * (kClassifyThreads / 64) + (threadIdx.x >> 6);
    if (p >= vp.P) return;
    classify_probe(vp, sv, dirs, active, p, threadIdx.x & 63);
}

// Every classifying volume of a batch: blocks find their volume by binary
// search over the prefix block counts (volumes without classification have
// no blocks and share their first block number with the next volume).
__global__ __launch_bounds__(kClassifyThreads) void k_classify_batched(const BatchVolume *vols, int n_vols) {
    const int g = blockIdx.x;
    int lo = 0, hi = n_vols - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vols[mid].first_classify <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchVolume &bv = vols[__builtin_amdgcn_readfirstlane(lo)];
    const int p = (g - bv.first_classify) * (kClassifyThreads / 64) + (threadIdx.x >> 6);
    if (p >= bv.vp.P) return;
    classify_probe(bv.vp, bv.sv, bv.dirs, bv.active, p, threadIdx.x & 63);
}

template <typename E>
__global__ __launch_bounds__(kViewThreads) void k_client_view(VolumeParams vp, SceneView sv, FrameParams fp, float ex,
                                                              float ey, float ez, int n_rays, uint8_t *view) {
    __shared__ E stk[kStack * kViewThreads];
    const int i = blockIdx.x * kViewThreads + threadIdx.x;
    if (i >= n_rays) return;
    const float3 eye = make_float3(ex, ey, ez);
    const Ray ray = make_ray(eye, xyz(raydir(fp, n_rays, i)));
    float tbest = INFINITY;
    int best = -1, best_id = -1;
    const GpuTri *arr = nullptr;
    Counts cnt = {0, 0};
    Stack<kViewThreads, E> stk_l{stk + threadIdx.x};
    closest<false>(sv.stat, global_nodes(sv.stat), ray, 0.f, tbest, best, best_id, arr, stk_l, cnt);
    closest<false>(sv.dyn, global_nodes(sv.dyn), ray, 0.f, tbest, best, best_id, arr, stk_l, cnt);
    if (best < 0) return;
    tbest = plane_t(arr[best], eye, ray.d);
    const float3 x = make_float3(fmaf(tbest, ray.d.x, ex), fmaf(tbest, ray.d.y, ey), fmaf(tbest, ray.d.z, ez));
    int cx, cy, cz;
    float fx, fy, fz;
    cell_axis(x.x, vp.ox, vp.sx, vp.nx, cx, fx);
    cell_axis(x.y, vp.oy, vp.sy, vp.ny, cy, fy);
    cell_axis(x.z, vp.oz, vp.sz, vp.nz, cz, fz);
    for (int corner = 0; corner < 8; ++corner) {
        const int bx = corner & 1, by = (corner >> 1) & 1, bz = corner >> 2;
        if ((bx && vp.nx == 1) || (by && vp.ny == 1) || (bz && vp.nz == 1)) continue;
        view[(cx + bx) + vp.nx * ((cy + by) + vp.ny * (cz + bz))] = 1;   // every writer stores 1
    }
}

__global__ void k_fill_u8(uint8_t *p, size_t n, uint8_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)blockDim.x * gridDim.x)
        p[i] = v;
}

hipError_t launch_classify(const VolumeParams &vp, const SceneView &sv, const float4 *dirs, uint8_t *active,
                           hipStream_t s) {
    const int per = kClassifyThreads / 64;
    hipLaunchKernelGGL(k_classify, dim3((vp.P + per - 1) / per), dim3(kClassifyThreads), 0, s, vp, sv, dirs, active);
    return hipGetLastError();
}

int classify_blocks(int P) { return (P + kClassifyThreads / 64 - 1) / (kClassifyThreads / 64); }

hipError_t launch_classify_batched(const BatchVolume *vols_dev, int n_vols, int total_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_classify_batched, dim3(total_blocks), dim3(kClassifyThreads), 0, s, vols_dev, n_vols);
    return hipGetLastError();
}

hipError_t launch_client_view(const VolumeParams &vp, const SceneView &sv, float ex, float ey, float ez, int n_rays,
                              uint8_t *view, hipStream_t s) {
    FrameParams fp = {};
    fp.rot[0] = fp.rot[4] = fp.rot[8] = 1.f;
    const dim3 grid((n_rays + kViewThreads - 1) / kViewThreads);
    if (stack_fits_u16(sv))
        hipLaunchKernelGGL(k_client_view<uint16_t>, grid, dim3(kViewThreads), 0, s, vp, sv, fp, ex, ey, ez, n_rays,
                           view);
    else
        hipLaunchKernelGGL(k_client_view<int>, grid, dim3(kViewThreads), 0, s, vp, sv, fp, ex, ey, ez, n_rays, view);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t s) {
    const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>(1024, (n + 255) / 256));
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace pv
