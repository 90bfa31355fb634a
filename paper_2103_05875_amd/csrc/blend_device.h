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
constexpr int kBlendK = 128;          // rays staged in LDS per chunk
static_assert(kBlendK <= kBlendThreads && kBlendK * kBlendTile % kBlendThreads == 0, "chunk staging");
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

// Four consecutive texels of a map row held as raw words: loaded early and
// taken apart where they are used, so that the load is waited for there
// (rows of interior texels start at any two-byte boundary).
template <typename T>
struct Texels4;
template <>
struct Texels4<__half> {
    uint2 w;
    __device__ __forceinline__ void load(const __half *p) { __builtin_memcpy(&w, p, sizeof(w)); }
    __device__ __forceinline__ __half get(int r) const {
        const uint32_t x = r < 2 ? w.x : w.y;
        return __ushort_as_half((unsigned short)((r & 1) ? x >> 16 : x & 0xffffu));
    }
    __device__ __forceinline__ float getf(int r) const { return __half2float(get(r)); }
};
template <>
struct Texels4<float> {
    uint4 w;
    __device__ __forceinline__ void load(const float *p) { __builtin_memcpy(&w, p, sizeof(w)); }
    __device__ __forceinline__ float get(int r) const {
        return __uint_as_float(r == 0 ? w.x : r == 1 ? w.y : r == 2 ? w.z : w.w);
    }
    __device__ __forceinline__ float getf(int r) const { return get(r); }
};

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
    float4 dir[kBlendK];              // the chunk's ray directions (zero past n)
    float rows[kTexRows];             // weight row totals
};

// New value of one texel-channel: estimate = sum / total, lerped with the
// stored value 'old' by h (h = 0: no history), rounded to the map format,
// written with its guard copies. A texel whose total is at most the floor
// keeps its value.
template <typename T>
__device__ __forceinline__ void blend_store(T *tile, int N, int t, float sum, float total, float h, float old) {
    if (!(total > kWeightFloor)) return;
    const int i = t % N, jr = t / N;
    const float est = sum * (1.0f / total);
    float nv = est;
    if (h > 0.f) nv = fmaf(h, old, (1.0f - h) * est);
    store_with_guard<T>(tile, N, i, jr, to_map<T>(nv));
}

// Interior texel t of an N x N map in its (N+2)^2 tile.
__device__ __forceinline__ int interior(int N, int t) { return (t / N + 1) * (N + 2) + t % N + 1; }

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
//
// The A operand (the weights) is computed in registers: lane l evaluates
// its three rows' weights for ray 4 step + l / 16 from the ray direction
// staged in LDS, and also sums them, so a wave holds the weight row totals
// of its own rows with no weight table in memory. Ray records arrive in
// 128-ray chunks through LDS; the next chunk is loaded into registers while
// the current one runs on the matrix cores, and the stored values the
// hysteresis needs are loaded before the products.
template <typename T, int S>
__device__ void blend_tile(const VolumeParams &vp, const float4 *dirs, const float4 *rays, T *irr, T *vis, float h,
                           int p0, int part, BlendSmem &sm) {
    constexpr int kStage = kBlendK * kBlendTile / kBlendThreads;  // records each thread stages per chunk
    const int tid = threadIdx.x, lane = tid & 63;
    const int g = part * 4 + (tid >> 6);
    const int n = vp.n, P = vp.P, sharp = vp.vis_sharpness;
    const int col = lane & 15, krow = lane >> 4;
    const int q = col & 7, half = col >> 3;
    const int ctile = g & 1;  // irradiance colour tile: 0 = red/green, 1 = blue
    const int p = p0 + q;
    const bool has_i = !(ctile && half);  // the blue tile's upper columns are zero

    // texel directions of this lane's A rows (irradiance ti_a; visibility tv_a, tv_a + 16)
    const int ti_a = 16 * (g >> 1) + col, tv_a = 32 * g + col;
    const float3 om_i = oct_texel_dir(8, ti_a & 7, ti_a >> 3);
    const float3 om_v0 = oct_texel_dir(16, tv_a & 15, tv_a >> 4);
    const float3 om_v1 = oct_texel_dir(16, (tv_a + 16) & 15, (tv_a + 16) >> 4);

    // the lane's output tiles (irradiance channel: red/green by column
    // half, or blue) and their stored values (rows 4 krow + r)
    T *itile = irr + ((size_t)min(p, P - 1) * 3 + (ctile ? 2 : half)) * 100;
    T *vtile = vis + ((size_t)min(p, P - 1) * 2 + half) * 324;
    // (rows 4 krow .. 4 krow + 3 are four consecutive texels of one tile
    // row; the tiles above are those of a probe inside the volume, so every
    // lane loads, used or not, and no load waits in a branch of its own)
    Texels4<T> old_i, old_v0, old_v1;
    {
        const int ti = 16 * (g >> 1) + 4 * krow, tv0 = 32 * g + 4 * krow;
        old_i.load(itile + interior(8, ti));
        old_v0.load(vtile + interior(16, tv0));
        old_v1.load(vtile + interior(16, tv0 + 16));
    }

    // chunk staging: consecutive threads take consecutive LDS records (8
    // probes of one ray, then the next ray): conflict-free stores, 128-byte
    // runs of each probe's rays in global memory
    float4 rr[kStage], dr;
    auto fetch = [&](int j0) {
        const int m = min(kBlendK, n - j0);
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int e = tid + u * kBlendThreads, jj = e / kBlendTile, pp = p0 + e % kBlendTile;
            rr[u] = (pp < P && jj < m) ? rays[(size_t)pp * n + j0 + jj] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        dr = (tid < m) ? dirs[j0 + tid] : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    fetch(0);

    v4f acc_i = {0.f, 0.f, 0.f, 0.f};
    v4f acc_v0 = acc_i, acc_v1 = acc_i;
    float s_i = 0.f, s_v0 = 0.f, s_v1 = 0.f;
    for (int j0 = 0; j0 < n; j0 += kBlendK) {
        const int m = min(kBlendK, n - j0);
        __syncthreads();  // every wave is done with the previous chunk
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int e = tid + u * kBlendThreads;
            sm.rec[e / kBlendTile][e % kBlendTile] = rr[u];
        }
        if (tid < kBlendK) sm.dir[tid] = dr;
        __syncthreads();
        if (j0 + kBlendK < n) fetch(j0 + kBlendK);
        // steps of 4 rays, unrolled by 4: past m the staged directions and
        // records are zero, so the weights and products add exact zeros
        const int steps = ((m + 15) >> 4) << 2;
        for (int k0 = 0; k0 < steps; k0 += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = 4 * (k0 + u) + krow;
                const float4 r4 = sm.rec[j][q];
                const float3 d = xyz(sm.dir[j]);
                const float w_i = fmaxf(dot3(om_i, d), 0.f);
                const float w_v0 = pow_int<S>(fmaxf(dot3(om_v0, d), 0.f), sharp);
                const float w_v1 = pow_int<S>(fmaxf(dot3(om_v1, d), 0.f), sharp);
                s_i += w_i;
                s_v0 += w_v0;
                s_v1 += w_v1;
                const float bv = half ? r4.w * r4.w : r4.w;
                const float bi = ctile ? (half ? 0.f : r4.z) : (half ? r4.y : r4.x);
                acc_i = __builtin_amdgcn_mfma_f32_16x16x4f32(w_i, bi, acc_i, 0, 0, 0);
                acc_v0 = __builtin_amdgcn_mfma_f32_16x16x4f32(w_v0, bv, acc_v0, 0, 0, 0);
                acc_v1 = __builtin_amdgcn_mfma_f32_16x16x4f32(w_v1, bv, acc_v1, 0, 0, 0);
            }
        }
    }

    // row totals: the four lanes of a row (l / 16 = 0 .. 3) hold partial
    // sums; after the two exchanges all four hold the same total
    s_i += __shfl_xor(s_i, 16);
    s_i += __shfl_xor(s_i, 32);
    s_v0 += __shfl_xor(s_v0, 16);
    s_v0 += __shfl_xor(s_v0, 32);
    s_v1 += __shfl_xor(s_v1, 16);
    s_v1 += __shfl_xor(s_v1, 32);
    if (krow == 0) {
        if (ctile == 0) sm.rows[ti_a] = s_i;  // both colour tiles compute the same irradiance rows
        sm.rows[kIrrRows + tv_a] = s_v0;
        sm.rows[kIrrRows + tv_a + 16] = s_v1;
    }
    __syncthreads();

    if (p >= P) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ti = 16 * (g >> 1) + 4 * krow + r;
        if (has_i) blend_store<T>(itile, 8, ti, acc_i[r], sm.rows[ti], h, old_i.getf(r));
        const int tv0 = 32 * g + 4 * krow + r, tv1 = tv0 + 16;
        blend_store<T>(vtile, 16, tv0, acc_v0[r], sm.rows[kIrrRows + tv0], h, old_v0.getf(r));
        blend_store<T>(vtile, 16, tv1, acc_v1[r], sm.rows[kIrrRows + tv1], h, old_v1.getf(r));
    }
}

// Both sharpness forms of the blend (s = 50 is unrolled; every path that
// blends a volume dispatches the same way, so their results are identical).
template <typename T>
__device__ __forceinline__ void blend_tile_any(const VolumeParams &vp, const float4 *dirs, const float4 *rays, T *irr,
                                               T *vis, float h, int p0, int part, BlendSmem &sm) {
    if (vp.vis_sharpness == 50)
        blend_tile<T, 50>(vp, dirs, rays, irr, vis, h, p0, part, sm);
    else
        blend_tile<T, 0>(vp, dirs, rays, irr, vis, h, p0, part, sm);
}

}  // namespace pv
