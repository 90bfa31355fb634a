// Blend of ray records into the octahedral maps, device side.
//
// Per probe p and texel t the estimate is a weighted mean over the probe's
// rays (Sec. 3.2, Eq. 1 and 2): irradiance texels (64 of them, 8x8) weight
// ray j by max(0, w_t . d_j) and average its radiance; visibility texels
// (256, 16x16) weight it by max(0, w_t . d_j)^s and average its distance and
// squared distance. The weights depend on the texel and the ray, not on the
// probe, because every probe of a volume-frame shares one ray set; so the
// blend of a volume is one matrix product per texture,
//   E_irr[t][(p, c)] = sum_j W_irr[t][j] * L[p][j][c]   (t < 64,  c = r, g, b)
//   E_vis[t][(p, c)] = sum_j W_vis[t][j] * R[p][j][c]   (t < 256, c = r, r^2)
// followed by a division by the weight row sums, the hysteresis lerp with
// the stored value, rounding to the map format and the guard-band copy.
// The products run on the FP32 matrix cores (16x16x4 MFMA, FP32 accumulate).
#pragma once

#include "device_common.h"
#include "blend_layout.h"

namespace pv {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kIrrRows = 64;          // irradiance interior texels
constexpr int kBlendThreads = 256;    // four wavefronts
constexpr int kBlendK = 128;          // rays staged in LDS per step
static_assert(kBlendK == 128, "the weight tables are zero-padded to a multiple of 128 rays");
static_assert(kBlendSplit == 2 && kBlendThreads == 256, "blend_tile maps 2 x 4 waves onto the texel rows");

// Direction i of the n-ray spherical-Fibonacci set, rotated by the frame's
// rotation (FP64 arithmetic, rounded to FP32 once).
__device__ __forceinline__ float4 raydir(const FrameParams &fp, int n, int i) {
    // z evenly spaced in (-1, 1); azimuth steps by the golden angle
    const double z = 1.0 - (2.0 * i + 1.0) / n;
    const double a = (double)i * 0.61803398874989484820;  // frac(i * (phi - 1))
    const double az = 6.28318530717958647692 * (a - floor(a));
    const double rr = sqrt(fmax(0.0, 1.0 - z * z));
    const double sx = rr * cos(az), sy = rr * sin(az);
    const float *R = fp.rot;
    return make_float4((float)(R[0] * sx + R[1] * sy + R[2] * z), (float)(R[3] * sx + R[4] * sy + R[5] * z),
                       (float)(R[6] * sx + R[7] * sy + R[8] * z), 0.f);
}

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

// x^s by repeated squaring (s = 50: x^32 x^16 x^2).
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
    float4 rec[kBlendK][kBlendTile];  // ray records of the tile's probes
    float rows[kTexRows];             // weight row totals
};

// New value of one texel-channel: estimate = sum / total, lerped with the
// stored value by h (h = 0: no history), rounded to the map format, written
// with its guard copies. A texel whose total is at most the floor keeps its
// value.
template <typename T>
__device__ __forceinline__ void blend_store(T *tile, int N, int t, float sum, float total, float h) {
    if (!(total > kWeightFloor)) return;
    const int i = t % N, jr = t / N;
    const float est = sum * (1.0f / total);
    float nv = est;
    if (h > 0.f) nv = fmaf(h, load_map<T>(tile + (jr + 1) * (N + 2) + (i + 1)), (1.0f - h) * est);
    store_with_guard<T>(tile, N, i, jr, to_map<T>(nv));
}

// Blend of probes p0 .. p0+7, rows half 'part' (0 or 1), by one block of
// four wavefronts; the two halves of a tile are independent blocks.
//
// 16x16x4 FP32 MFMA operand layout (lane l of the wave): A[m][k] with
// m = l % 16, k = l / 16; B[k][n] with k = l / 16, n = l % 16; result
// D[m][n] in register r with m = 4 (l / 16) + r, n = l % 16.
// Columns n of B: visibility n = 8 c + q (channel c = r or r^2, probe q);
// irradiance tile 0 n = 8 c + q (c = red, green), tile 1 n = q (blue; the
// upper eight columns are zero). The 8 waves of a tile (g = 4 part + wave)
// each own three 16-row MFMA tiles: visibility rows 32g .. 32g+31 and
// irradiance rows 16 (g / 2) .. +15 of colour tile g % 2.
template <typename T>
__device__ void blend_tile(const VolumeParams &vp, const WeightTables &wt, const float4 *rays, T *irr, T *vis,
                           float h, int p0, int part, BlendSmem &sm) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int g = part * 4 + (tid >> 6);
    const int n = vp.n, P = vp.P;
    const int col = lane & 15, krow = lane >> 4;
    const int q = col & 7, half = col >> 3;
    const int ctile = g & 1;  // irradiance colour tile: 0 = red/green, 1 = blue

    for (int t = tid; t < kTexRows; t += kBlendThreads) {
        float s = 0.f;
        for (int b = 0; b < wt.nparts; ++b) s += wt.part[b * kTexRows + t];
        sm.rows[t] = s;
    }
    v4f acc_i = {0.f, 0.f, 0.f, 0.f};
    v4f acc_v0 = acc_i, acc_v1 = acc_i;
    const int row_i = 16 * (g >> 1) + col;
    const int row_v = kIrrRows + 32 * g + col;

    for (int j0 = 0; j0 < n; j0 += kBlendK) {
        const int m = min(kBlendK, n - j0);
        __syncthreads();
        // consecutive threads fill consecutive LDS records (8 probes of one
        // ray, then the next ray): conflict-free stores, 128-byte runs of
        // each probe's rays in global memory
        for (int e = tid; e < kBlendK * kBlendTile; e += kBlendThreads) {
            const int jj = e / kBlendTile, pq = e - jj * kBlendTile, p = p0 + pq;
            sm.rec[jj][pq] = (p < P && jj < m) ? rays[(size_t)p * n + j0 + jj] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();
        // steps of 4 rays, in groups of 4 steps: the records past m are
        // staged as zeros and the table is zero past n (padded to kBlendK).
        // The weights of the next group are loaded while the current one
        // runs on the matrix cores.
        const int steps = ((m + 15) >> 4) << 2;
        const float *wg = wt.w + (size_t)(j0 >> 2) * (4 * kTexRows) + krow;
        float nxt[4][3];
        auto load_group = [&](int k0, float a[4][3]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float *w = wg + (size_t)(k0 + u) * (4 * kTexRows);
                a[u][0] = w[4 * row_i];
                a[u][1] = w[4 * row_v];
                a[u][2] = w[4 * (row_v + 16)];
            }
        };
        load_group(0, nxt);
        for (int k0 = 0; k0 < steps; k0 += 4) {
            float cur[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int x = 0; x < 3; ++x) cur[u][x] = nxt[u][x];
            if (k0 + 4 < steps) load_group(k0 + 4, nxt);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 r4 = sm.rec[4 * (k0 + u) + krow][q];
                const float bv = half ? r4.w * r4.w : r4.w;
                const float bi = ctile ? (half ? 0.f : r4.z) : (half ? r4.y : r4.x);
                acc_i = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[u][0], bi, acc_i, 0, 0, 0);
                acc_v0 = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[u][1], bv, acc_v0, 0, 0, 0);
                acc_v1 = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[u][2], bv, acc_v1, 0, 0, 0);
            }
        }
    }

    const int p = p0 + q;
    if (p >= P) return;
    T *itile = irr + (size_t)p * 3 * 100;
    T *vtile = vis + (size_t)p * 2 * 324;
    const int ch = ctile ? 2 : half;  // irradiance channel of this lane's column
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ti = 16 * (g >> 1) + 4 * krow + r;
        if (!(ctile && half)) blend_store<T>(itile + ch * 100, 8, ti, acc_i[r], sm.rows[ti], h);
        const int tv0 = 32 * g + 4 * krow + r, tv1 = tv0 + 16;
        blend_store<T>(vtile + half * 324, 16, tv0, acc_v0[r], sm.rows[kIrrRows + tv0], h);
        blend_store<T>(vtile + half * 324, 16, tv1, acc_v1[r], sm.rows[kIrrRows + tv1], h);
    }
}

}  // namespace pv
