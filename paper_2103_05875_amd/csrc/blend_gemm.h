// The blend as a matrix product over a per-frame weight table, device side.
//
// The weights W[t][j] (texel row t, ray j: max(0, w_t . d_j), to the power s
// for visibility rows) are shared by every probe of a volume-frame, so they
// are evaluated once per frame, by extra blocks of the ray-direction launch,
// into a table laid out as the matrix cores' A operand: per step of 32 rays,
// per tile of 16 rows, per lane, 32 bytes. The blend then multiplies that
// table with the ray records of 16 probes per wavefront:
//   E_irr[t][q] (channel c) = sum_j W[t][j] L[q][j][c]   t < 64
//   E_vis[t][q] (channel c) = sum_j W[64 + t][j] R_c[q][j]  (R = r, r^2)
// A block owns 16 probes (their records staged through LDS, shared by its
// wavefronts) and each of its wavefronts a group of the 44 output tiles of
// 16 x 16 (row tiles x channels; four groups of 10 to 12, or eight of four
// to six), so each weight fragment a wavefront loads feeds two or three
// products and each ray record up to five.
//
// Two numeric paths:
//   BF16x3: 16x16x32 BF16 MFMA. Weights and records are split into a BF16
//           high half and a BF16 low half (x = hi + lo + O(2^-18 x)), and
//           each product is hi*hi + hi*lo + lo*hi with FP32 accumulation:
//           about 2^-16 of relative error per term, far below the binary16
//           spacing (2^-11) of the maps it serves.
//   F32:    16x16x4 FP32 MFMA, eight k-steps per 32 rays.
// Operand layouts (lane l): 16x16x32 BF16: A[l%16][8(l/16) + i], B[8(l/16)
// + i][l%16], i < 8; 16x16x4 FP32: A[l%16][l/16], B[l/16][l%16]; both give
// D[4(l/16) + r][l%16] in accumulator register r.
#pragma once

#include <type_traits>

#include "blend_device.h"

namespace pv {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_bits(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
__device__ __forceinline__ float bf16_value(unsigned short b) { return __uint_as_float((uint32_t)b << 16); }

// Weight of texel row m (0-63 irradiance, 64-319 visibility) for direction d.
template <int S>
__device__ __forceinline__ float row_weight(float3 om, bool vis_row, int sharp, float3 d) {
    const float c = fmaxf(dot3(om, d), 0.f);
    return vis_row ? pow_int<S>(c, sharp) : c;
}

__device__ __forceinline__ float3 row_dir(int m) {
    return m < 64 ? oct_texel_dir(8, m & 7, m >> 3) : oct_texel_dir(16, (m - 64) & 15, (m - 64) >> 4);
}

// Table rows of one 16-row tile over a group of four 32-ray steps by a
// 256-thread block: the block first puts the group's 128 directions into LDS
// (the same FP32 values as the direction kernel), then wavefront w evaluates
// the tile's weights of step 4 g + w. The group's row sums (each lane's sum,
// then across the four lanes of a row, then the four wavefronts' sums in
// order) go to the group's row of partial totals; the blend adds the groups'
// partials in order, so every run gives the same totals. sdir: 128 float3,
// red: 64 floats of LDS.
template <int S>
__device__ void weight_tile_block(const FrameParams &fp, int n, int sharp, int mode, uint8_t *tab, int mt, int grp,
                                  float3 *sdir, float *red) {
    const int j0 = grp * kWGroup * kWStep;
    if ((int)threadIdx.x < kWGroup * kWStep && j0 + (int)threadIdx.x < n)
        sdir[threadIdx.x] = xyz(raydir(fp, n, j0 + threadIdx.x));
    __syncthreads();
    const int lane = threadIdx.x & 63, q = lane & 15, kq = lane >> 4, wv = threadIdx.x >> 6;
    const int m = 16 * mt + q;
    const bool vis_row = m >= 64;
    const float3 om = row_dir(m);
    const int steps = (n + kWStep - 1) / kWStep;
    float sum = 0.f;
    for (int s = kWGroup * grp + wv; s < min(steps, kWGroup * (grp + 1)); s += 4) {
        uint4 *dst = reinterpret_cast<uint4 *>(tab + (((size_t)s * kMTiles + mt) * 64 + lane) * wtab_lane_bytes(mode));
        if (mode == kBlendBF16x6) {
            // three parts: x = hi + mid + lo + O(2^-27 x); each difference is
            // exact in FP32 (it drops the leading bits the part took)
            unsigned short hi[8], mi[8], lo[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int j = s * kWStep + 8 * kq + i;
                const float w = j < n ? row_weight<S>(om, vis_row, sharp, sdir[j - j0]) : 0.f;
                sum += w;
                hi[i] = bf16_bits(w);
                const float r = w - bf16_value(hi[i]);
                mi[i] = bf16_bits(r);
                lo[i] = bf16_bits(r - bf16_value(mi[i]));
            }
            dst[0] = make_uint4(hi[0] | (uint32_t)hi[1] << 16, hi[2] | (uint32_t)hi[3] << 16,
                                hi[4] | (uint32_t)hi[5] << 16, hi[6] | (uint32_t)hi[7] << 16);
            dst[1] = make_uint4(mi[0] | (uint32_t)mi[1] << 16, mi[2] | (uint32_t)mi[3] << 16,
                                mi[4] | (uint32_t)mi[5] << 16, mi[6] | (uint32_t)mi[7] << 16);
            dst[2] = make_uint4(lo[0] | (uint32_t)lo[1] << 16, lo[2] | (uint32_t)lo[3] << 16,
                                lo[4] | (uint32_t)lo[5] << 16, lo[6] | (uint32_t)lo[7] << 16);
        } else if (mode == kBlendBF16x3) {
            unsigned short hi[8], lo[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int j = s * kWStep + 8 * kq + i;
                const float w = j < n ? row_weight<S>(om, vis_row, sharp, sdir[j - j0]) : 0.f;
                sum += w;
                hi[i] = bf16_bits(w);
                lo[i] = bf16_bits(w - bf16_value(hi[i]));
            }
            dst[0] = make_uint4(hi[0] | (uint32_t)hi[1] << 16, hi[2] | (uint32_t)hi[3] << 16,
                                hi[4] | (uint32_t)hi[5] << 16, hi[6] | (uint32_t)hi[7] << 16);
            dst[1] = make_uint4(lo[0] | (uint32_t)lo[1] << 16, lo[2] | (uint32_t)lo[3] << 16,
                                lo[4] | (uint32_t)lo[5] << 16, lo[6] | (uint32_t)lo[7] << 16);
        } else if (mode == kBlendVALU) {
            // rows 4 r4 .. 4 r4 + 3 of the tile side by side per ray of the
            // step, so that a lane's four rows are one 16-byte load
            float *dv = reinterpret_cast<float *>(tab + ((size_t)s * kMTiles + mt) * 64 * 32);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = 4 * i + kq, j = s * kWStep + k;
                const float w = j < n ? row_weight<S>(om, vis_row, sharp, sdir[j - j0]) : 0.f;
                sum += w;
                dv[((q >> 2) * kWStep + k) * 4 + (q & 3)] = w;
            }
        } else {
            float w[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int j = s * kWStep + 4 * i + kq;
                w[i] = j < n ? row_weight<S>(om, vis_row, sharp, sdir[j - j0]) : 0.f;
                sum += w[i];
            }
            dst[0] = make_uint4(__float_as_uint(w[0]), __float_as_uint(w[1]), __float_as_uint(w[2]),
                                __float_as_uint(w[3]));
            dst[1] = make_uint4(__float_as_uint(w[4]), __float_as_uint(w[5]), __float_as_uint(w[6]),
                                __float_as_uint(w[7]));
        }
    }
    sum += __shfl_xor(sum, 16);
    sum += __shfl_xor(sum, 32);
    if (kq == 0) red[wv * 16 + q] = sum;
    __syncthreads();
    if (threadIdx.x < 16)
        reinterpret_cast<float *>(tab + wtab_rows_offset(n, mode))[grp * kTexRows + 16 * mt + threadIdx.x] =
            ((red[threadIdx.x] + red[16 + threadIdx.x]) + red[32 + threadIdx.x]) + red[48 + threadIdx.x];
}

// Table block b of the direction launch: row tile b % kMTiles, step group
// b / kMTiles.
__device__ __forceinline__ void weight_table_block(const FrameParams &fp, int n, int sharp, int mode, uint8_t *tab,
                                                   int b, float3 *sdir, float *red) {
    const int mt = b % kMTiles, grp = b / kMTiles;
    if (sharp == 50)
        weight_tile_block<50>(fp, n, sharp, mode, tab, mt, grp, sdir, red);
    else
        weight_tile_block<0>(fp, n, sharp, mode, tab, mt, grp, sdir, red);
}

__device__ __forceinline__ const uint8_t *weight_table(const float4 *dirs, int n) {
    return reinterpret_cast<const uint8_t *>(dirs) + dirs_span(n);
}

// ---------------------------------------------------------------------------
// the product
// ---------------------------------------------------------------------------
// Channel c of a ray record: radiance r, g, b (c < 3), distance, distance^2.
__device__ __forceinline__ float channel(float4 r, int c) {
    return c == 0 ? r.x : c == 1 ? r.y : c == 2 ? r.z : c == 3 ? r.w : r.w * r.w;
}

// Output tiles of a wavefront: NI irradiance row tiles (three channels)
// from irradiance tile I0, NV visibility row tiles (two channels) from
// visibility tile V0.
template <int I0, int NI, int V0, int NV>
struct TileSet {
    static constexpr int kRowTiles = NI + NV;
    static constexpr int kTiles = 3 * NI + 2 * NV;
    static constexpr int kChannels = NI > 0 ? (NV > 0 ? 5 : 3) : 2;  // record channels used
    static constexpr int kC0 = NI > 0 ? 0 : 3;                        // first of them
    v4f acc[kTiles];
    // global row tile (0-3 irradiance, 4-19 visibility) of row tile t
    __device__ static constexpr int mtile(int t) { return t < NI ? I0 + t : 4 + V0 + (t - NI); }
};

// A fragment of row tile mt at step s for this lane (32 bytes).
__device__ __forceinline__ void load_frag(const uint8_t *tab, int s, int mt, uint4 &a0, uint4 &a1) {
    const uint4 *p = reinterpret_cast<const uint4 *>(tab) + (((size_t)s * kMTiles + mt) * 64 + (threadIdx.x & 63)) * 2;
    a0 = p[0];
    a1 = p[1];
}

// The three-part fragment of the BF16x6 table (48 bytes: high, middle, low).
__device__ __forceinline__ void load_frag3(const uint8_t *tab, int s, int mt, uint4 *a) {
    const uint4 *p = reinterpret_cast<const uint4 *>(tab) + (((size_t)s * kMTiles + mt) * 64 + (threadIdx.x & 63)) * 3;
    a[0] = p[0];
    a[1] = p[1];
    a[2] = p[2];
}

// Records of one 32-ray step of a column group, shared through LDS by the
// group's row-group wavefronts (loaded once, coalesced: consecutive threads
// take consecutive records of a probe). A probe's row is padded by one
// record so that the fragment reads of 16 probes spread over the banks.
struct BlendRecs {
    float4 r[2][16][kWStep + 1];
};

// The block's 16 probe tiles in LDS for the epilogue, in the maps' own
// layout: irradiance [16][3][10][10] then visibility [16][2][18][18] of the
// map type (30,336 bytes in binary16); shares its LDS with the records.
template <typename T>
struct BlendImage {
    static constexpr int kIrrElems = 16 * 3 * 100, kVisElems = 16 * 2 * 324;
    static constexpr int kBytes = (kIrrElems + kVisElems) * (int)sizeof(T);
    static_assert(kIrrElems * sizeof(T) % 16 == 0 && kBytes % 16 == 0, "16-byte chunks");
    T v[kIrrElems + kVisElems];
};

// Split-BF16 records of one step, split once per block at staging: per
// buffer, channel (r, g, b, distance, distance^2), part and probe, the
// 32 rays as 16 words of two BF16 values (ray 2w in the low half), so that
// a lane's operand (rays 8 kq .. 8 kq + 7 of probe q) is one aligned
// 16-byte read and a wavefront's 64 reads cover 1 KB without conflicts.
struct BlendRecsBF {
    uint32_t w[2][5][3][16][kWStep / 2];  // parts: high, low (BF16x3) or high, middle, low (BF16x6)
};

template <typename T>
struct BlendSmemGemm {
    union {
        BlendRecs recs;
        BlendRecsBF bf;
        BlendImage<T> img;
    };
    float rows[kTexRows];  // row totals: the table's step-group partials added in order
};

// Tile element (y, x) of an (N + 2)^2 tile -> the element whose value it
// holds: itself inside, across an edge the interior texel the octahedral
// fold puts next to it (rows first, then columns, which also maps the
// corners to the diagonally opposite interior corner).
__device__ __forceinline__ int guard_source(int N, int y, int x) {
    if (y == 0 || y == N + 1) {
        y = y == 0 ? 1 : N;
        x = N + 1 - x;
    }
    if (x == 0 || x == N + 1) {
        x = x == 0 ? 1 : N;
        y = N + 1 - y;
    }
    return y * (N + 2) + x;
}

// Guard texels of one texture of the block's LDS image: tile k (of
// n_tiles, (N + 2)^2 elements each from 'base'), border element g (G = 4N + 4
// per tile: the top row, the bottom row, then the left and right columns
// between them) takes the value of its interior source. Only guard texels
// are written and only interiors read.
template <typename T, int N>
__device__ __forceinline__ void fill_guards(T *base, int n_tiles) {
    constexpr int S = N + 2, G = 4 * N + 4;
    for (int i = threadIdx.x; i < n_tiles * G; i += blockDim.x) {
        const int k = i / G, g = i - k * G;
        int y, x;
        if (g < 2 * S) {
            y = g < S ? 0 : S - 1;
            x = g < S ? g : g - S;
        } else {
            const int r = g - 2 * S;
            x = r < N ? 0 : S - 1;
            y = 1 + (r < N ? r : r - N);
        }
        T *tile = base + k * S * S;
        tile[y * S + x] = tile[guard_source(N, y, x)];
    }
}

// Moves the tiles of probes p0 .. p0 + np - 1 between the maps and the
// block's LDS image in 16-byte chunks, U per thread in flight (to_lds: load
// the stored tiles; else write the image out whole). An odd probe count
// leaves half a chunk of binary16 irradiance (648 elements per probe are
// always whole chunks).
template <typename T, bool TO_LDS, int U>
__device__ __forceinline__ void image_move(T *irr, T *vis, int p0, int np, BlendImage<T> &img) {
    constexpr int kPer = 16 / (int)sizeof(T);
    static_assert(U == 2 || U == 4, "two or four chunks in flight");
    const int ni = np * 300 / kPer, nc = ni + np * 648 / kPer;
    const int tail = np * 300 - ni * kPer;
    if ((int)threadIdx.x < tail) {
        const int e = ni * kPer + threadIdx.x;
        if (TO_LDS)
            img.v[e] = irr[(size_t)p0 * 300 + e];
        else
            irr[(size_t)p0 * 300 + e] = img.v[e];
    }
    uint4 *gi = reinterpret_cast<uint4 *>(irr + (size_t)p0 * 300), *gv = reinterpret_cast<uint4 *>(vis + (size_t)p0 * 648);
    uint4 *li = reinterpret_cast<uint4 *>(img.v), *lv = reinterpret_cast<uint4 *>(img.v + BlendImage<T>::kIrrElems);
    // chunk c of the source and of the destination (irradiance chunks
    // first); each side stays in its own address space
    auto get = [&](int c) -> uint4 {
        if constexpr (TO_LDS)
            return c < ni ? gi[c] : gv[c - ni];
        else
            return c < ni ? li[c] : lv[c - ni];
    };
    auto put = [&](int c, uint4 x) {
        if constexpr (TO_LDS) {
            if (c < ni)
                li[c] = x;
            else
                lv[c - ni] = x;
        } else {
            if (c < ni)
                gi[c] = x;
            else
                gv[c - ni] = x;
        }
    };
    for (int c0 = threadIdx.x; c0 < nc; c0 += U * blockDim.x) {
        const int c1 = c0 + blockDim.x, c2 = c1 + blockDim.x, c3 = c2 + blockDim.x;
        const uint4 x0 = get(c0);
        const uint4 x1 = c1 < nc ? get(c1) : uint4{};
        const uint4 x2 = U == 4 && c2 < nc ? get(c2) : uint4{};
        const uint4 x3 = U == 4 && c3 < nc ? get(c3) : uint4{};
        put(c0, x0);
        if (c1 < nc) put(c1, x1);
        if (U == 4 && c2 < nc) put(c2, x2);
        if (U == 4 && c3 < nc) put(c3, x3);
    }
}

// s_waitcnt operand: vmcnt(2), no wait on the export and LDS/scalar counters
// (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
constexpr int kWaitVm2 = 2 | (7 << 4) | (15 << 8);

// Prefetch of step s's records for the split-BF16 products: thread t < 256
// takes rays 2 (t % 16) and 2 (t % 16) + 1 of probe t / 16 (32 contiguous
// bytes; threads above load record 0 and stage nothing), and at staging
// writes both rays' BF16 parts of every channel (the same split as the
// weights: two parts, x = hi + lo + O(2^-18 x), or three).
template <int PARTS>
struct RecPrefetchBF {
    float4 v[2];
    bool keep[2];
    __device__ __forceinline__ void load(const float4 *rays, int n, int P, int cg, int s) {
        const int t = threadIdx.x, qq = t >> 4, k = 2 * (t & 15);
        const int p = 16 * cg + qq, j = s * kWStep + k;
        const bool ok = t < 256 && p < P;
        // every lane loads (record 0 in place of one outside the volume), so
        // that every wavefront has the same loads in flight; the zeros are
        // applied at staging
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            keep[u] = ok && j + u < n;
            v[u] = rays[keep[u] ? (size_t)p * n + j + u : 0];
        }
    }
    __device__ __forceinline__ void store(BlendRecsBF &sm, int buf) const {
        const int t = threadIdx.x;
        if (t >= 256) return;
        const int qq = t >> 4, w = t & 15;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const float x0 = keep[0] ? channel(v[0], c) : 0.f, x1 = keep[1] ? channel(v[1], c) : 0.f;
            const unsigned short h0 = bf16_bits(x0), h1 = bf16_bits(x1);
            const float r0 = x0 - bf16_value(h0), r1 = x1 - bf16_value(h1);
            const unsigned short m0 = bf16_bits(r0), m1 = bf16_bits(r1);
            sm.w[buf][c][0][qq][w] = (uint32_t)h0 | (uint32_t)h1 << 16;
            sm.w[buf][c][1][qq][w] = (uint32_t)m0 | (uint32_t)m1 << 16;
            if constexpr (PARTS == 3) {
                const unsigned short l0 = bf16_bits(r0 - bf16_value(m0)), l1 = bf16_bits(r1 - bf16_value(m1));
                sm.w[buf][c][2][qq][w] = (uint32_t)l0 | (uint32_t)l1 << 16;
            }
        }
    }
};

// Prefetch of step s's records by the block's NT threads into registers.
template <int NT>
struct RecPrefetch {
    static constexpr int kPer = 16 * kWStep / NT;
    float4 v[kPer];
    bool keep[kPer];
    __device__ __forceinline__ void load(const float4 *rays, int n, int P, int cg, int s) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = threadIdx.x + u * NT, qq = e / kWStep, k = e % kWStep;
            const int p = 16 * cg + qq, j = s * kWStep + k;
            keep[u] = p < P && j < n;
            v[u] = rays[keep[u] ? (size_t)p * n + j : 0];  // record 0 in place of one outside
        }
    }
    __device__ __forceinline__ void store(BlendRecs &sm, int buf) const {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = threadIdx.x + u * NT;
            sm.r[buf][e / kWStep][e % kWStep] = keep[u] ? v[u] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
};

// One wavefront of the blend: probes 16 cg .. 16 cg + 15 (the block's column
// group; NT threads of G row-group wavefronts), its tile set, all steps,
// then the epilogue (estimate = sum / row total, hysteresis, store with
// guard copies, through the block's LDS image of its tiles). The next
// step's records (into LDS, by the whole block) and weight fragments are
// loaded while the current products run.
template <typename T, int MODE, int NT, int I0, int NI, int V0, int NV>
__device__ void blend_gemm_tiles(const VolumeParams &vp, const float4 *dirs, const float4 *rays, T *irr, T *vis,
                                 float h, int cg, BlendSmemGemm<T> &smu) {
    BlendRecs &sm = smu.recs;
    BlendRecsBF &sb = smu.bf;
    using TS = TileSet<I0, NI, V0, NV>;
    constexpr int RT = TS::kRowTiles, NC = TS::kChannels, C0 = TS::kC0;
    const int lane = threadIdx.x & 63, q = lane & 15, kq = lane >> 4;
    const int n = vp.n, P = vp.P;
    const int p = 16 * cg + q;
    const bool live = p < P;
    const uint8_t *tab = weight_table(dirs, n);
    const int steps = (n + kWStep - 1) / kWStep;
    // weight fragments of every row tile of the wavefront for the current
    // step, requested at the step's start in four-wavefront blocks (a second
    // set for the next step would cost the registers of a wavefront per
    // SIMD on the encode-size grid); eight-wavefront blocks (small volumes,
    // fewer blocks than resident slots) have registers to spare and request
    // the next step's fragments one step ahead
    constexpr bool kAhead = NT == 512 && MODE != kBlendVALU;
    // the same blocks (one per CU: the latency of their loads, not their
    // products, sets their pace) request the records two steps ahead, into
    // two register sets taken in turn (the others one step ahead, into one),
    // and take the stored interior texels of their outputs into registers
    // first, in flight under the products, instead of loading the block's
    // tiles into LDS after them
    constexpr bool kDeep = kAhead;
    Texels4<T> old[kDeep ? TS::kTiles : 1];
    if constexpr (kDeep) {
        if (live) {
#pragma unroll
            for (int t = 0; t < TS::kRowTiles; ++t) {
                const bool it = t < NI;
                const int N = it ? 8 : 16, nch = it ? 3 : 2;
                const int mloc = it ? I0 + t : V0 + (t - NI);
                const int acc0 = it ? 3 * t : 3 * NI + 2 * (t - NI);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (c >= nch) continue;
                    const T *tile = it ? irr + (size_t)p * 300 + c * 100 : vis + (size_t)p * 648 + c * 324;
                    old[acc0 + c].load(tile + interior(N, 16 * mloc + 4 * kq));
                }
            }
        }
    }
    TS ts;
#pragma unroll
    for (int t = 0; t < TS::kTiles; ++t) ts.acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    // records through LDS: split into BF16 parts at staging for the split
    // products, else whole FP32 records
    constexpr bool kSplit = MODE == kBlendBF16x3 || MODE == kBlendBF16x6;
    constexpr int kParts = MODE == kBlendBF16x6 ? 3 : 2;
    using PF = std::conditional_t<kSplit, RecPrefetchBF<kParts>, RecPrefetch<NT>>;
    PF pf0, pf1;
    pf0.load(rays, n, P, cg, 0);
    {
        // the row totals of the epilogue: the table's step-group partials,
        // added in order
        const float *part = reinterpret_cast<const float *>(tab + wtab_rows_offset(n, MODE));
        const int groups = wtab_groups(n);
        for (int m = threadIdx.x; m < kTexRows; m += NT) {
            float t = part[m];
            for (int g = 1; g < groups; ++g) t += part[g * kTexRows + m];
            smu.rows[m] = t;
        }
    }
    if constexpr (kSplit)
        pf0.store(sb, 0);
    else
        pf0.store(sm, 0);
    __syncthreads();
    // fragment parts held per row tile: three for BF16x6 (whose
    // four-wavefront blocks load them tile by tile in the product loop)
    constexpr int kFp = MODE == kBlendBF16x6 ? 3 : 2;
    constexpr bool kTileByTile = MODE == kBlendBF16x6 && !kAhead;
    uint4 acur[kTileByTile ? 1 : RT][kFp], anext[kAhead ? RT : 1][kFp];
    auto load_parts = [&](int step, int t, uint4 *a) {
        if constexpr (kFp == 3)
            load_frag3(tab, step, TS::mtile(t), a);
        else
            load_frag(tab, step, TS::mtile(t), a[0], a[1]);
    };
    if constexpr (kAhead) {
#pragma unroll
        for (int t = 0; t < RT; ++t) load_parts(0, t, acur[t]);
    }
    // (after the fragments: a step's first wait leaves in flight only the
    // newest loads, the records of the next step). The loads of these
    // blocks do not depend on the step count (past the last step they
    // repeat its fragments and take record 0, which is never staged), so
    // that every wait below counts the same loads on every path
    if constexpr (kDeep) pf1.load(rays, n, P, cg, 1);
    const int np = min(16, P - 16 * cg);
    // step s: 'ld' takes the records of step s + 2 (kDeep) or s + 1, 'st'
    // holds those of step s + 1 and stages them into LDS at the end
    auto step = [&](int s, PF &ld, PF &st) {
        const int buf = s & 1;
        if constexpr (kDeep) {
            // everything but the two newest loads (this step's fragments
            // arrived with the last step's copy; the next step's records stay
            // in flight), so that the products below wait for nothing; then
            // the next step's fragments and, after them, the records two
            // steps ahead, in that order
            __builtin_amdgcn_s_waitcnt(kWaitVm2);
#pragma unroll
            for (int t = 0; t < RT; ++t) load_parts(min(s + 1, steps - 1), t, anext[t]);
            __builtin_amdgcn_sched_barrier(0);
            ld.load(rays, n, P, cg, s + 2);
        } else {
            if (s + 1 < steps) ld.load(rays, n, P, cg, s + 1);
        }
        if constexpr (!kAhead && MODE != kBlendVALU && MODE != kBlendBF16x6) {
#pragma unroll
            for (int t = 0; t < RT; ++t) load_frag(tab, s, TS::mtile(t), acur[t][0], acur[t][1]);
        }
        if constexpr (MODE == kBlendVALU) {
            // vector FMAs: the lane's rows 4 kq .. 4 kq + 3 of every row tile
            // against its probe's records, four rays at a time
            const float4 *wt = reinterpret_cast<const float4 *>(tab) + (size_t)s * kMTiles * 128;
#pragma unroll 1
            for (int k0 = 0; k0 < kWStep; k0 += 4) {
                float rc[4][NC];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float4 r = sm.r[buf][q][k0 + i];
#pragma unroll
                    for (int c = 0; c < NC; ++c) rc[i][c] = channel(r, C0 + c);
                }
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const bool it = t < NI;
                    const int nch = it ? 3 : 2;
                    const int acc0 = it ? 3 * t : 3 * NI + 2 * (t - NI);
                    const int ch0 = it ? 0 : NC - 2;
                    const float4 *w = wt + TS::mtile(t) * 128 + kq * kWStep + k0;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float4 wv = w[i];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if (c >= nch) continue;
                            v4f &a = ts.acc[acc0 + c];
                            const float x = rc[i][ch0 + c];
                            a[0] = fmaf(wv.x, x, a[0]);
                            a[1] = fmaf(wv.y, x, a[1]);
                            a[2] = fmaf(wv.z, x, a[2]);
                            a[3] = fmaf(wv.w, x, a[3]);
                        }
                    }
                }
            }
        } else {
            // the step's operand fragments: BF16x3 rays 8 kq .. 8 kq + 7 (high
            // and low halves, staged split), F32 ray 4 i + kq of probe q
            bf16x8 bp[kParts][NC];
            float bf[NC][8];
            if constexpr (kSplit) {
#pragma unroll
                for (int k = 0; k < kParts; ++k) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        bp[k][c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&sb.w[buf][C0 + c][k][q][4 * kq]));
                }
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float4 r = sm.r[buf][q][4 * i + kq];
#pragma unroll
                    for (int c = 0; c < NC; ++c) bf[c][i] = channel(r, C0 + c);
                }
            }
            // the products, ordered so that consecutive matrix instructions
            // feed different accumulators (each accumulator still takes its
            // terms in the same order)
            // products (weight part, record part): BF16x3 (0,0) (0,1) (1,0);
            // BF16x6 also (0,2) (2,0) (1,1), the terms down to 2^-18 of the
            // product
            constexpr int kPa[6] = {0, 0, 1, 0, 2, 1}, kPb[6] = {0, 1, 0, 2, 0, 1};
            if constexpr (kTileByTile) {
                // row tile by row tile, its three weight parts loaded for its
                // six products (three parts of every row tile at once would
                // not leave four wavefronts per SIMD)
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const bool it = t < NI;
                    const int nch = it ? 3 : 2;
                    const int acc0 = it ? 3 * t : 3 * NI + 2 * (t - NI);
                    const int ch0 = it ? 0 : NC - 2;
                    uint4 a3[3];
                    load_frag3(tab, s, TS::mtile(t), a3);
#pragma unroll
                    for (int pk = 0; pk < 6; ++pk) {
                        const bf16x8 aw = __builtin_bit_cast(bf16x8, a3[kPa[pk]]);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if (c >= nch) continue;
                            v4f &a = ts.acc[acc0 + c];
                            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bp[kPb[pk]][ch0 + c], a, 0, 0, 0);
                        }
                    }
                }
            } else if constexpr (kSplit) {
                constexpr int kProducts = MODE == kBlendBF16x6 ? 6 : 3;
#pragma unroll
                for (int pk = 0; pk < kProducts; ++pk) {
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        const bool it = t < NI;
                        const int nch = it ? 3 : 2;
                        const int acc0 = it ? 3 * t : 3 * NI + 2 * (t - NI);
                        const int ch0 = it ? 0 : NC - 2;  // first channel slot of the tile's texture
                        const bf16x8 aw = __builtin_bit_cast(bf16x8, acur[t][kPa[pk]]);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if (c >= nch) continue;
                            v4f &a = ts.acc[acc0 + c];
                            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bp[kPb[pk]][ch0 + c], a, 0, 0, 0);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        const bool it = t < NI;
                        const int nch = it ? 3 : 2;
                        const int acc0 = it ? 3 * t : 3 * NI + 2 * (t - NI);
                        const int ch0 = it ? 0 : NC - 2;
                        const uint4 aw = acur[t][i >> 2];
                        const float w = __uint_as_float((i & 3) == 0 ? aw.x : (i & 3) == 1 ? aw.y : (i & 3) == 2 ? aw.z : aw.w);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if (c >= nch) continue;
                            v4f &a = ts.acc[acc0 + c];
                            a = __builtin_amdgcn_mfma_f32_16x16x4f32(w, bf[ch0 + c][i], a, 0, 0, 0);
                        }
                    }
                }
            }
        }
        // every wavefront is done with the other buffer since the last step's barrier
        if (s + 1 < steps) {
            if constexpr (kSplit)
                st.store(sb, buf ^ 1);
            else
                st.store(sm, buf ^ 1);
            if constexpr (kAhead) {
#pragma unroll
                for (int t = 0; t < RT; ++t) {
#pragma unroll
                    for (int k = 0; k < kFp; ++k) acur[t][k] = anext[t][k];
                }
            }
        }
        __syncthreads();
    };
    if constexpr (kDeep) {
        // (the loop is entered only from its last step, so that no wait at
        // its head has to cover loads issued by the first)
        for (int s = 0;;) {
            step(s, pf0, pf1);
            if (++s == steps) break;
            step(s, pf1, pf0);
            if (++s == steps) break;
        }
    } else {
        for (int s = 0; s < steps; ++s) step(s, pf0, pf0);
    }
    // epilogue, through the block's LDS image of its probes' tiles: the
    // stored tiles are loaded (coalesced; eight-wavefront blocks hold their
    // outputs' stored interior texels already), each wavefront replaces its
    // interior texels by the new values (estimate = sum / row total,
    // hysteresis, the map's rounding; a texel whose total is at most the
    // floor keeps its value), the guard texels are copied from their
    // interior sources in LDS, and the tiles are written back whole
    BlendImage<T> &img = smu.img;
    if constexpr (!kDeep) {
        image_move<T, true, 1024 / NT>(irr, vis, 16 * cg, np, img);
        __syncthreads();
    }
    const float *rows = smu.rows;
    if (live) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const bool it = t < NI;
            const int N = it ? 8 : 16, nch = it ? 3 : 2;
            const int mloc = it ? I0 + t : V0 + (t - NI);
            const int acc0 = it ? 3 * t : 3 * NI + 2 * (t - NI);
            float total[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) total[r] = rows[(it ? 0 : 64) + 16 * mloc + 4 * kq + r];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c >= nch) continue;
                T *tile = it ? img.v + (q * 3 + c) * 100 : img.v + BlendImage<T>::kIrrElems + (q * 2 + c) * 324;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float w = total[r];
                    T &dst = tile[interior(N, 16 * mloc + 4 * kq + r)];
                    T prev;
                    if constexpr (kDeep) {
                        // every interior texel of the image is written here
                        prev = old[acc0 + c].get(r);
                        if (!(w > kWeightFloor)) dst = prev;
                    } else {
                        prev = dst;
                    }
                    if (!(w > kWeightFloor)) continue;
                    const float est = ts.acc[acc0 + c][r] * (1.0f / w);
                    dst = to_map<T>(h > 0.f ? fmaf(h, load_map<T>(&prev), (1.0f - h) * est) : est);
                }
            }
        }
    }
    __syncthreads();
    fill_guards<T, 8>(img.v, 3 * np);
    fill_guards<T, 16>(img.v + BlendImage<T>::kIrrElems, 2 * np);
    __syncthreads();
    image_move<T, false, 1024 / NT>(irr, vis, 16 * cg, np, img);
}

// Row groups of a volume's blend: G row-group wavefronts per 16-probe column
// group, one block per column group (G = 4 for large volumes and in the
// batched launch, 8 for small volumes so that enough wavefronts run; which
// wavefront computes a tile does not change its result).
__host__ __device__ inline int blend_row_groups(int P) { return (P + 15) / 16 >= 512 ? 4 : 8; }
__host__ __device__ inline int blend_column_groups(int P) { return (P + 15) / 16; }

template <typename T, int MODE, int G>
__device__ __forceinline__ void blend_gemm_block(const VolumeParams &vp, const float4 *dirs, const float4 *rays, T *irr,
                                                 T *vis, float h, int cg, BlendSmemGemm<T> &sm) {
    constexpr int NT = 64 * G;
    const int g = threadIdx.x >> 6;
    if (G == 4) {
        // irradiance (12 tiles) | visibility rows 0-95 (12) | 96-175 (10) | 176-255 (10)
        switch (g) {
        case 0: blend_gemm_tiles<T, MODE, NT, 0, 4, 0, 0>(vp, dirs, rays, irr, vis, h, cg, sm); break;
        case 1: blend_gemm_tiles<T, MODE, NT, 0, 0, 0, 6>(vp, dirs, rays, irr, vis, h, cg, sm); break;
        case 2: blend_gemm_tiles<T, MODE, NT, 0, 0, 6, 5>(vp, dirs, rays, irr, vis, h, cg, sm); break;
        default: blend_gemm_tiles<T, MODE, NT, 0, 0, 11, 5>(vp, dirs, rays, irr, vis, h, cg, sm); break;
        }
        return;
    }
    // eight groups: two of irradiance (6 tiles each), six of visibility (6, 6, 6, 6, 4, 4)
    switch (g) {
    case 0: blend_gemm_tiles<T, MODE, NT, 0, 2, 0, 0>(vp, dirs, rays, irr, vis, h, cg, sm); break;
    case 1: blend_gemm_tiles<T, MODE, NT, 2, 2, 0, 0>(vp, dirs, rays, irr, vis, h, cg, sm); break;
    case 2: blend_gemm_tiles<T, MODE, NT, 0, 0, 0, 3>(vp, dirs, rays, irr, vis, h, cg, sm); break;
    case 3: blend_gemm_tiles<T, MODE, NT, 0, 0, 3, 3>(vp, dirs, rays, irr, vis, h, cg, sm); break;
    case 4: blend_gemm_tiles<T, MODE, NT, 0, 0, 6, 3>(vp, dirs, rays, irr, vis, h, cg, sm); break;
    case 5: blend_gemm_tiles<T, MODE, NT, 0, 0, 9, 3>(vp, dirs, rays, irr, vis, h, cg, sm); break;
    case 6: blend_gemm_tiles<T, MODE, NT, 0, 0, 12, 2>(vp, dirs, rays, irr, vis, h, cg, sm); break;
    default: blend_gemm_tiles<T, MODE, NT, 0, 0, 14, 2>(vp, dirs, rays, irr, vis, h, cg, sm); break;
    }
}

}  // namespace pv
