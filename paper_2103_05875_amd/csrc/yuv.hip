// Codec surfaces (Sec. 3.3): the probe textures laid out as the inputs of a
// lossless video encoder, and back.
//
// Probe p occupies atlas tile (p % C, p / C); guard bands are left out
// (Sec. 3.4); tiles past the last probe are zero.
//   irradiance: 10-bit code of each normalised channel value (FP32: rint of
//     the value times k, clamped to [0, 1023]) in the top 10 bits of a
//     16-bit sample; R, G, B are the Y, U, V planes of a YUV444 surface,
//     [8 ceil(P / C)] x [8 C] samples each
//   visibility: each RG16F texel is four bytes (mean lo, mean hi, mean^2 lo,
//     mean^2 hi); byte m of a texel row goes to sample m / 3 of plane m % 3,
//     so three texels fill four YUV samples; a row of x = 16 C texels is
//     ceil(4 x / 3) samples, the missing bytes zero
// Irradiance: one thread per output sample (encode) or texel (decode);
// visibility encode: one thread per three texels (four samples per plane),
// written out through LDS as 32-bit words;
// the writes of a wavefront are contiguous, the reads gather short runs
// from the tiles. All of it is a pure permutation of bytes plus one rounding
// per irradiance value, so the kernels are bound by HBM.
#include "device_common.h"

namespace pv {

constexpr int kYuvThreads = 256;

__device__ __forceinline__ uint32_t irr_code(float v, float k) {
    const float x = __builtin_rintf(v * k);
    if (!(x > 0.f)) return 0u;
    return x > 1023.f ? 1023u : (uint32_t)x;
}

__global__ __launch_bounds__(kYuvThreads) void k_yuv_irr_encode(const uint16_t *irr, int P, int C, float k,
                                                                uint16_t *planes, int W, int H) {
    const long long idx = (long long)blockIdx.x * kYuvThreads + threadIdx.x;
    if (idx >= (long long)W * H) return;
    const int row = (int)(idx / W), col = (int)(idx - (long long)row * W);
    const int p = (row >> 3) * C + (col >> 3), j = row & 7, i = col & 7;
    const size_t plane = (size_t)W * H;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        uint16_t s = 0;
        if (p < P) {
            const uint16_t h = irr[(((size_t)p * 3 + c) * 10 + j + 1) * 10 + i + 1];
            s = (uint16_t)(irr_code(__half2float(__ushort_as_half(h)), k) << 6);
        }
        planes[c * plane + idx] = s;
    }
}

// One thread per group of three texels of a row (twelve bytes): it reads
// each texel's two 16-bit values once and puts byte 3k + c of the group,
// sample k of plane c, into LDS; the block then writes its run of each
// plane's row (up to 1,024 samples) as aligned 32-bit words, bytes only at
// the run's two ends (words aligned in memory, whatever the planes' base).
// Block (x, y): row x, groups 256y ..
__global__ __launch_bounds__(kYuvThreads) void k_yuv_vis_encode(const uint16_t *vis, int P, int C, uint8_t *planes,
                                                                int Wv, int Hv) {
    __shared__ uint8_t sm[3][4 * kYuvThreads];
    const int x = 16 * C, G = (x + 2) / 3;
    const int row = blockIdx.x, g0 = blockIdx.y * kYuvThreads, g = g0 + threadIdx.x;
    const int ty = row >> 4, j = row & 15;
    uint32_t tex[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int col = 3 * g + t, p = ty * C + (col >> 4), i = col & 15;
        tex[t] = 0u;
        if (g < G && col < x && p < P) {
            const size_t at = (((size_t)p * 2) * 18 + j + 1) * 18 + i + 1;
            tex[t] = (uint32_t)vis[at] | ((uint32_t)vis[at + 18 * 18] << 16);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int m = 3 * k + c;
            sm[c][4 * threadIdx.x + k] = (uint8_t)(tex[m >> 2] >> (8 * (m & 3)));
        }
    __syncthreads();
    const int u0 = 4 * g0, len = min(4 * kYuvThreads, Wv - u0);
    const size_t plane = (size_t)Wv * Hv;
    const long long mis = (long long)((uintptr_t)planes & 3);  // the base's offset from a word boundary
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const long long a0 = (long long)(c * plane + (size_t)row * Wv + u0);
        const long long A = ((a0 + mis) & ~3ll) - mis;  // index of the aligned word holding a0
        const int nwords = (int)((a0 + len - A + 3) >> 2);
        for (int w = threadIdx.x; w < nwords; w += kYuvThreads) {
            const long long at = A + 4ll * w;
            if (at >= a0 && at + 4 <= a0 + len) {
                const int o = (int)(at - a0);
                *reinterpret_cast<uint32_t *>(planes + at) = (uint32_t)sm[c][o] | ((uint32_t)sm[c][o + 1] << 8) |
                                                             ((uint32_t)sm[c][o + 2] << 16) |
                                                             ((uint32_t)sm[c][o + 3] << 24);
            } else {
                for (int bb = 0; bb < 4; ++bb)
                    if (at + bb >= a0 && at + bb < a0 + len) planes[at + bb] = sm[c][at + bb - a0];
            }
        }
    }
}

__global__ __launch_bounds__(kYuvThreads) void k_yuv_irr_decode(const uint16_t *planes, int P, int C, int W, int H,
                                                                uint32_t *codes) {
    const long long idx = (long long)blockIdx.x * kYuvThreads + threadIdx.x;
    if (idx >= (long long)P * 64) return;
    const int p = (int)(idx >> 6), t = (int)(idx & 63);
    const int row = (p / C) * 8 + (t >> 3), col = (p % C) * 8 + (t & 7);
    const size_t plane = (size_t)W * H, at = (size_t)row * W + col;
    uint32_t code = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) code |= (uint32_t)(planes[c * plane + at] >> 6) << (10 * c);
    codes[idx] = code;
}

__global__ __launch_bounds__(kYuvThreads) void k_yuv_vis_decode(const uint8_t *planes, int P, int C, int Wv, int Hv,
                                                                uint16_t *vis) {
    const long long idx = (long long)blockIdx.x * kYuvThreads + threadIdx.x;
    if (idx >= (long long)P * 256) return;
    const int p = (int)(idx >> 8), t = (int)(idx & 255);
    const int row = (p / C) * 16 + (t >> 4), col = (p % C) * 16 + (t & 15);
    const size_t plane = (size_t)Wv * Hv, base = (size_t)row * Wv;
    uint32_t by[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const long long m = 4ll * col + b;
        by[b] = planes[(m % 3) * plane + base + m / 3];
    }
    vis[((size_t)p * 2) * 256 + t] = (uint16_t)(by[0] | (by[1] << 8));
    vis[((size_t)p * 2 + 1) * 256 + t] = (uint16_t)(by[2] | (by[3] << 8));
}

static dim3 yuv_grid(long long n) { return dim3((unsigned)((n + kYuvThreads - 1) / kYuvThreads)); }

hipError_t launch_yuv_encode(const uint16_t *irr, const uint16_t *vis, int P, int C, float k, uint16_t *irr_planes,
                             uint8_t *vis_planes, const YuvDims &d, hipStream_t s) {
    hipLaunchKernelGGL(k_yuv_irr_encode, yuv_grid(d.w * d.h), dim3(kYuvThreads), 0, s, irr, P, C, k, irr_planes,
                       (int)d.w, (int)d.h);
    const int groups = (16 * C + 2) / 3;
    hipLaunchKernelGGL(k_yuv_vis_encode, dim3((unsigned)d.hv, (groups + kYuvThreads - 1) / kYuvThreads),
                       dim3(kYuvThreads), 0, s, vis, P, C, vis_planes, (int)d.wv, (int)d.hv);
    return hipGetLastError();
}

hipError_t launch_yuv_decode(const uint16_t *irr_planes, const uint8_t *vis_planes, int P, int C, uint32_t *codes,
                             uint16_t *vis, const YuvDims &d, hipStream_t s) {
    hipLaunchKernelGGL(k_yuv_irr_decode, yuv_grid((long long)P * 64), dim3(kYuvThreads), 0, s, irr_planes, P, C,
                       (int)d.w, (int)d.h, codes);
    hipLaunchKernelGGL(k_yuv_vis_decode, yuv_grid((long long)P * 256), dim3(kYuvThreads), 0, s, vis_planes, P, C,
                       (int)d.wv, (int)d.hv, vis);
    return hipGetLastError();
}

}  // namespace pv
