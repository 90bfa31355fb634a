// Lossless delta pack of FP16 probe tiles for one client: change masks,
// ordered compaction with a delta-coded index buffer, XOR byte planes against
// the client's last-transmitted state, reference update, checksum.
#include <mutex>
#include <vector>

#include "device_common.h"
#include "packet_format.h"

namespace pv {

// ---------------------------------------------------------------------------
// pack
// ---------------------------------------------------------------------------

// |a - b| > tau for binary16 a, b, decided exactly. A difference of two
// binary16 values is a multiple of 2^-24: below 1 it has fewer than 24
// significant bits and binary32 holds it exactly; at or above 1 its binary32
// rounding stays at or above 1. So for tau < 1 the binary32 difference gives
// the exact answer; larger thresholds take the difference in binary64.
__device__ __forceinline__ bool texel_changed(uint16_t a, uint16_t b, float tau, bool narrow) {
    if (tau == 0.f) return a != b;
    const float fa = __half2float(__ushort_as_half(a)), fb = __half2float(__ushort_as_half(b));
    if (narrow) return fabsf(fa - fb) > tau;
    return fabs((double)fa - (double)fb) > (double)tau;
}

// The pack works on tiles of kPackQ consecutive probes. Their FP16 tiles are
// contiguous in HBM (600 B and 1,296 B per probe) and start on 16-byte
// boundaries (kPackQ * 600 and kPackQ * 1,296 are multiples of 16), so a block
// stages them into LDS with aligned 16-byte loads; a ragged last tile of odd
// length ends its irradiance run with one 8-byte load, so no load reads past
// the maps (which may be caller-owned buffers of exactly P tiles). Work
// is then split into row units of 8 interior texels of one channel:
// irradiance 3 x 8 rows per probe, visibility 2 x 16 rows x 2 halves.
constexpr int kPackQ = kPackTile;
static_assert(kPackQ * 600 % 16 == 0 && kPackQ * 1296 % 16 == 0 && kPackQ <= 64, "aligned staging, one ballot");
constexpr int kPackThreads = 256;
constexpr int kIrrUnits = 3 * 8;       // per probe
constexpr int kVisUnits = 2 * 16 * 2;  // per probe

struct PackSmem {
    uint4 irr[kPackQ * 600 / 16];
    uint4 vis[kPackQ * 1296 / 16];
    int changed[kPackQ][2];
    uint32_t part[kPackThreads / 64];
};

__device__ __forceinline__ void stage_tiles(const PackBuffers &b, int p0, int P, PackSmem &sm) {
    const int n = min(kPackQ, P - p0);
    const uint4 *gi = reinterpret_cast<const uint4 *>(b.cur_irr + (size_t)p0 * 300);
    const uint4 *gv = reinterpret_cast<const uint4 *>(b.cur_vis + (size_t)p0 * 648);
    // n * 1296 is a multiple of 16; n * 600 leaves 8 bytes when n is odd
    const int vi = n * 600 / 16, vv = n * 1296 / 16;
    // every chunk of the thread is requested before any is stored, so that
    // their latencies overlap (a load-store loop waits for each load in
    // turn); a thread past the run takes the run's last chunk, loading and
    // storing the same bytes as its owner (unconditional stores keep each
    // load from being moved next to its store)
    constexpr int kI = (kPackQ * 600 / 16 + kPackThreads - 1) / kPackThreads;
    constexpr int kV = (kPackQ * 1296 / 16 + kPackThreads - 1) / kPackThreads;
    uint4 ri[kI], rv[kV];
#pragma unroll
    for (int u = 0; u < kI; ++u) ri[u] = gi[min((int)threadIdx.x + u * kPackThreads, vi - 1)];
#pragma unroll
    for (int u = 0; u < kV; ++u) rv[u] = gv[min((int)threadIdx.x + u * kPackThreads, vv - 1)];
    if ((n & 1) && threadIdx.x == 0)
        reinterpret_cast<uint2 *>(sm.irr)[2 * vi] = reinterpret_cast<const uint2 *>(gi)[2 * vi];
#pragma unroll
    for (int u = 0; u < kI; ++u) sm.irr[min((int)threadIdx.x + u * kPackThreads, vi - 1)] = ri[u];
#pragma unroll
    for (int u = 0; u < kV; ++u) sm.vis[min((int)threadIdx.x + u * kPackThreads, vv - 1)] = rv[u];
}

// Unit u of the tile (irradiance units first): probe q, texture (0 irr,
// 1 vis), channel c, first interior texel t0 (multiple of 8).
struct Unit {
    int q, tex, c, t0, N;
};

__device__ __forceinline__ Unit unit_of(int u) {
    Unit r;
    if (u < kPackQ * kIrrUnits) {
        r.q = u / kIrrUnits;
        const int w = u - r.q * kIrrUnits;
        r.tex = 0;
        r.c = w / 8;
        r.t0 = (w % 8) * 8;
        r.N = 8;
    } else {
        const int v = u - kPackQ * kIrrUnits;
        r.q = v / kVisUnits;
        const int w = v - r.q * kVisUnits;
        r.tex = 1;
        r.c = w / 32;
        r.t0 = (w % 32) * 8;
        r.N = 16;
    }
    return r;
}

// The 8 current texels of a unit from the staged tiles.
__device__ __forceinline__ void unit_cur(const PackSmem &sm, const Unit &u, uint16_t cur[8]) {
    const uint16_t *base = u.tex == 0 ? reinterpret_cast<const uint16_t *>(sm.irr) + u.q * 300 + u.c * 100
                                      : reinterpret_cast<const uint16_t *>(sm.vis) + u.q * 648 + u.c * 324;
    const int S = u.N + 2, row = u.t0 / u.N, col = u.t0 - row * u.N;
    const uint16_t *src = base + (row + 1) * S + col + 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) cur[i] = src[i];
}

__device__ __forceinline__ uint16_t *unit_ref(const PackBuffers &b, int p, const Unit &u) {
    return u.tex == 0 ? b.ref_irr + (size_t)p * 192 + u.c * 64 + u.t0 : b.ref_vis + (size_t)p * 512 + u.c * 256 + u.t0;
}

__device__ __forceinline__ void unpack8(uint4 v, uint16_t r[8]) {
    r[0] = v.x & 0xffff;
    r[1] = v.x >> 16;
    r[2] = v.y & 0xffff;
    r[3] = v.y >> 16;
    r[4] = v.z & 0xffff;
    r[5] = v.z >> 16;
    r[6] = v.w & 0xffff;
    r[7] = v.w >> 16;
}

// Summary of a run of tiles: changed counts (irradiance, visibility) and the
// last two changed probes of each texture (-1: none). Index entries are
// deltas to the previous changed probe, so the entry just before a tile's
// first one is last - second of the tiles before it.
struct TileSum {
    int ci, cv, li, lv, si, sv;
};

__device__ __forceinline__ TileSum tile_sum_none() { return TileSum{0, 0, -1, -1, -1, -1}; }

// Sums and the top two probes of the union (probes of different tiles are
// distinct): associative and commutative.
__device__ __forceinline__ TileSum tile_merge(const TileSum &a, const TileSum &c) {
    TileSum r;
    r.ci = a.ci + c.ci;
    r.cv = a.cv + c.cv;
    r.li = max(a.li, c.li);
    r.si = max(min(a.li, c.li), max(a.si, c.si));
    r.lv = max(a.lv, c.lv);
    r.sv = max(min(a.lv, c.lv), max(a.sv, c.sv));
    return r;
}

// A tile's own summary in 32 bits (the mask pass's output): changed counts
// (0-8) in bits 0-3 and 4-7, then the offsets in the tile (0-7, 15 = none)
// of the last irradiance, last visibility, second-last irradiance and
// second-last visibility changed probe in bits 8-11, 12-15, 16-19, 20-23.
__device__ __forceinline__ uint32_t pack_tile_sum(const TileSum &v, int p0) {
    auto off = [p0](int p) { return p < 0 ? 15u : (uint32_t)(p - p0); };
    return (uint32_t)v.ci | (uint32_t)v.cv << 4 | off(v.li) << 8 | off(v.lv) << 12 | off(v.si) << 16 |
           off(v.sv) << 20;
}

__device__ __forceinline__ TileSum unpack_tile_sum(uint32_t x, int p0) {
    auto at = [x, p0](int sh) { const int o = (int)(x >> sh) & 15; return o == 15 ? -1 : p0 + o; };
    return TileSum{(int)(x & 15u), (int)(x >> 4 & 15u), at(8), at(12), at(16), at(20)};
}

__device__ __forceinline__ TileSum own_tile_sum(const PackBuffers &b, int t) {
    return unpack_tile_sum(b.tsum[t], t * kPackQ);
}

// The scan's output: the summary of the tiles before tile t.
__device__ __forceinline__ TileSum load_tile_sum(const PackBuffers &b, int t) {
    const int4 x = b.tiles[t];
    const int2 y = b.tiles2[t];
    return TileSum{x.x, x.y, x.z, x.w, y.x, y.y};
}

__device__ __forceinline__ void store_tile_sum(const PackBuffers &b, int t, const TileSum &v) {
    b.tiles[t] = make_int4(v.ci, v.cv, v.li, v.lv);
    b.tiles2[t] = make_int2(v.si, v.sv);
}

__device__ __forceinline__ TileSum shfl_tile_sum(const TileSum &v, int src) {
    return TileSum{__shfl(v.ci, src), __shfl(v.cv, src), __shfl(v.li, src),
                   __shfl(v.lv, src), __shfl(v.si, src), __shfl(v.sv, src)};
}

__device__ __forceinline__ TileSum shfl_up_tile_sum(const TileSum &v, int off) {
    return TileSum{__shfl_up(v.ci, off), __shfl_up(v.cv, off), __shfl_up(v.li, off),
                   __shfl_up(v.lv, off), __shfl_up(v.si, off), __shfl_up(v.sv, off)};
}

__device__ __forceinline__ TileSum shfl_xor_tile_sum(const TileSum &v, int off) {
    return TileSum{__shfl_xor(v.ci, off), __shfl_xor(v.cv, off), __shfl_xor(v.li, off),
                   __shfl_xor(v.lv, off), __shfl_xor(v.si, off), __shfl_xor(v.sv, off)};
}

// Change mask of one tile (every thread of the block): any interior texel
// differs (tau = 0) or |cur - ref| > tau. The tile's current texels are
// staged in sm (and stay there for a compaction in the same block); the
// masks and the tile's 32-bit summary (changed counts and the last two
// changed probes per texture) are written for the prefix.
__device__ void mask_tile(const PackBuffers &b, int P, int tile, float tau_irr, float tau_vis, PackSmem &sm) {
    const int p0 = tile * kPackQ;
    if (threadIdx.x < kPackQ * 2) sm.changed[threadIdx.x >> 1][threadIdx.x & 1] = 0;
    const int n = min(kPackQ, P - p0);
    constexpr int units = kPackQ * (kIrrUnits + kVisUnits);
    constexpr int kPer = (units + kPackThreads - 1) / kPackThreads;
    // the thread's reference rows are requested with the tile staging
    uint4 refv[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int u = threadIdx.x + i * kPackThreads;
        refv[i] = make_uint4(0u, 0u, 0u, 0u);
        if (u < units) {
            const Unit un = unit_of(u);
            if (un.q < n) refv[i] = *reinterpret_cast<const uint4 *>(unit_ref(b, p0 + un.q, un));
        }
    }
    stage_tiles(b, p0, P, sm);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int u = threadIdx.x + i * kPackThreads;
        if (u >= units) continue;
        const Unit un = unit_of(u);
        if (un.q >= n) continue;
        uint16_t cur[8], ref[8];
        unit_cur(sm, un, cur);
        unpack8(refv[i], ref);
        const float tau = un.tex == 0 ? tau_irr : tau_vis;
        const bool narrow = tau < 1.f;
        bool ch = false;
#pragma unroll
        for (int t = 0; t < 8; ++t) ch |= texel_changed(cur[t], ref[t], tau, narrow);
        // many units of a probe may set its flag: plain stores of the same
        // value (LDS atomics on one address serialize)
        if (ch) __hip_atomic_store(&sm.changed[un.q][un.tex], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    if (threadIdx.x < n) {
        // only eligible probes are sent: active, and in the client's view
        const int p = p0 + threadIdx.x;
        if ((b.active && !b.active[p]) || (b.view && !b.view[p])) {
            sm.changed[threadIdx.x][0] = 0;
            sm.changed[threadIdx.x][1] = 0;
        }
        b.mask_irr[p] = (uint8_t)sm.changed[threadIdx.x][0];
        b.mask_vis[p] = (uint8_t)sm.changed[threadIdx.x][1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        TileSum t = tile_sum_none();
        for (int q = 0; q < n; ++q) {
            if (sm.changed[q][0]) {
                t.ci++;
                t.si = t.li;
                t.li = p0 + q;
            }
            if (sm.changed[q][1]) {
                t.cv++;
                t.sv = t.lv;
                t.lv = p0 + q;
            }
        }
        b.tsum[tile] = pack_tile_sum(t, p0);
    }
}

__global__ __launch_bounds__(kPackThreads) void k_pack_mask(PackBuffers b, int P, float tau_irr, float tau_vis) {
    __shared__ PackSmem sm;
    if ((int)blockIdx.x * kPackQ >= P) return;
    mask_tile(b, P, blockIdx.x, tau_irr, tau_vis, sm);
}

constexpr int kScanThreads = 1024;

// Exclusive prefix (tile_merge) of every thread's value across the block, and
// the block's total: wavefront shuffles, then the wavefront totals.
__device__ __forceinline__ TileSum block_exclusive_scan(const TileSum &v, TileSum *sh, TileSum &total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    TileSum inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const TileSum o = shfl_up_tile_sum(inc, off);
        if (lane >= off) inc = tile_merge(o, inc);
    }
    if (lane == 63) sh[wv] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        TileSum run = tile_sum_none();
        for (int k = 0; k < kScanThreads / 64; ++k) {
            const TileSum w = sh[k];
            sh[k] = run;
            run = tile_merge(run, w);
        }
        sh[kScanThreads / 64] = run;
    }
    __syncthreads();
    TileSum ex = shfl_up_tile_sum(inc, 1);
    if (lane == 0) ex = tile_sum_none();
    total = sh[kScanThreads / 64];
    return tile_merge(sh[wv], ex);
}

// One block: writes for every tile the summary of the tiles before it and
// stores the totals (K_irr, K_vis, and the last two changed
// irradiance probes) in totals[0..3].
__global__ __launch_bounds__(kScanThreads) void k_pack_scan(PackBuffers b, int n_tiles) {
    __shared__ TileSum sh[kScanThreads / 64 + 1];
    const int per = (n_tiles + kScanThreads - 1) / kScanThreads;
    const int lo = min(n_tiles, (int)threadIdx.x * per), hi = min(n_tiles, lo + per);
    TileSum mine = tile_sum_none();
    for (int t = lo; t < hi; ++t) mine = tile_merge(mine, own_tile_sum(b, t));
    TileSum total;
    TileSum run = block_exclusive_scan(mine, sh, total);
    for (int t = lo; t < hi; ++t) {
        const TileSum v = own_tile_sum(b, t);
        store_tile_sum(b, t, run);
        run = tile_merge(run, v);
    }
    if (threadIdx.x == 0) {
        b.totals[0] = (uint32_t)total.ci;
        b.totals[1] = (uint32_t)total.cv;
        b.totals[2] = (uint32_t)total.li;
        b.totals[3] = (uint32_t)total.si;
    }
}

// The summary of tiles [0, upto) and of all n_tiles, reduced by the whole
// block from the mask pass's tile summaries (every thread must call it).
template <int T>
__device__ __forceinline__ void reduce_tiles(const PackBuffers &b, int n_tiles, int upto, TileSum &before,
                                             TileSum &total, TileSum *sh) {
    TileSum pre = tile_sum_none(), tot = tile_sum_none();
#pragma unroll 4
    for (int t = threadIdx.x; t < n_tiles; t += T) {
        const TileSum v = own_tile_sum(b, t);
        tot = tile_merge(tot, v);
        if (t < upto) pre = tile_merge(pre, v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        pre = tile_merge(pre, shfl_xor_tile_sum(pre, off));
        tot = tile_merge(tot, shfl_xor_tile_sum(tot, off));
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[2 * wv] = pre;
        sh[2 * wv + 1] = tot;
    }
    __syncthreads();
    before = tile_sum_none();
    total = tile_sum_none();
    for (int w = 0; w < T / 64; ++w) {
        before = tile_merge(before, sh[2 * w]);
        total = tile_merge(total, sh[2 * w + 1]);
    }
    __syncthreads();
}

// Per-block scratch of a tile's compaction.
struct CompactShared {
    int rank_s[kPackQ][2];
    int any_s;
};

// Compaction of one tile (every thread of the block): its changed probes'
// ranks (the summary before the tile plus the changed lanes below), their
// delta-coded index entries, XOR byte planes and reference update; returns
// the thread's share of the checksum. The checksum (the sum of every
// payload word's hash, an order-free integer sum) is split by word: a tile
// hashes its plane words and the index words whose second entry is its own
// (the entry before its first comes from the last two changed probes before
// the tile; the first visibility entry pairs with the last irradiance
// entry), and the tile holding the index's last entry also the zero
// padding. staged: the tile's current texels are already in sm.
__device__ uint32_t compact_tile(const PackBuffers &b, int P, int tile, const TileSum &before, const TileSum &tot,
                                 PackSmem &sm, bool staged, CompactShared &cs) {
    const int p0 = tile * kPackQ;
    const int n = min(kPackQ, P - p0);
    const int K_irr = tot.ci, K_vis = tot.cv, M = K_irr + K_vis;
    const int idx_bytes = ((2 * M + 15) / 16) * 16;
    uint16_t *idx = reinterpret_cast<uint16_t *>(b.packet + 32);  // irradiance entries, then visibility
    uint32_t part = 0;
    if (threadIdx.x < 64) {
        // lane q owns probe p0 + q; its rank counts the changed lanes below
        // it, its predecessor is the highest of them (or the last one before
        // the tile)
        const int q = threadIdx.x, p = p0 + q;
        const bool ci = q < n && b.mask_irr[p] != 0, cv = q < n && b.mask_vis[p] != 0;
        const unsigned long long below = (1ull << q) - 1ull;
        const unsigned long long bi = __ballot(ci), bvv = __ballot(cv);
        const unsigned long long mi = bi & below, mv = bvv & below;
        if (q == 0) cs.any_s = (bi | bvv) != 0ull;
        const int ki = before.ci + __popcll(mi), kv = before.cv + __popcll(mv);
        const int prev_i = mi ? p0 + 63 - __clzll((long long)mi) : before.li;
        const int prev_v = mv ? p0 + 63 - __clzll((long long)mv) : before.lv;
        const uint32_t ei = (uint16_t)(ki == 0 ? p : p - prev_i), ev = (uint16_t)(kv == 0 ? p : p - prev_v);
        // the entry before each one: a lane below in the tile, or from the
        // last two changed probes before the tile (or overall, for the first
        // visibility entry)
        const uint32_t ei_lane = __shfl(ei, mi ? 63 - __clzll((long long)mi) : 0);
        const uint32_t ev_lane = __shfl(ev, mv ? 63 - __clzll((long long)mv) : 0);
        if (q < kPackQ) {
            cs.rank_s[q][0] = ci ? ki : -1;
            cs.rank_s[q][1] = cv ? kv : -1;
        }
        if (ci) idx[ki] = (uint16_t)ei;
        if (cv) idx[K_irr + kv] = (uint16_t)ev;
        for (int tex = 0; tex < 2; ++tex) {
            if (!(tex == 0 ? ci : cv)) continue;
            const int c = tex == 0 ? ki : K_irr + kv;
            const uint32_t e = tex == 0 ? ei : ev;
            if (c & 1) {
                uint32_t pe;
                if (tex == 0)
                    pe = mi ? ei_lane : (uint16_t)(ki == 1 ? before.li : before.li - before.si);
                else if (mv)
                    pe = ev_lane;
                else if (kv > 0)
                    pe = (uint16_t)(kv == 1 ? before.lv : before.lv - before.sv);
                else
                    pe = (uint16_t)(K_irr == 1 ? tot.li : tot.li - tot.si);
                part += word_hash(pe | (e << 16), (uint32_t)(c - 1) / 2);
            }
            if (c == M - 1) {
                // the last entry: its word if it opens one, then the zero padding
                if (!(c & 1)) part += word_hash(e, (uint32_t)c / 2);
                for (int j = M; j < idx_bytes / 2; ++j) idx[j] = 0;
                for (int w = (M + 1) / 2; w < idx_bytes / 4; ++w) part += word_hash(0u, (uint32_t)w);
            }
        }
    }
    __syncthreads();
    if (cs.any_s) {
        if (!staged) {
            stage_tiles(b, p0, P, sm);
            __syncthreads();
        }
        uint8_t *planes_i = b.packet + 32 + idx_bytes;
        uint8_t *planes_v = planes_i + (size_t)K_irr * 6 * 64;
        const int units = kPackQ * (kIrrUnits + kVisUnits);
        for (int u = threadIdx.x; u < units; u += kPackThreads) {
            const Unit un = unit_of(u);
            if (un.q >= n) continue;
            const int k = cs.rank_s[un.q][un.tex];
            if (k < 0) continue;
            const int p = p0 + un.q;
            uint16_t cur[8], ref[8];
            unit_cur(sm, un, cur);
            uint16_t *rp = unit_ref(b, p, un);
            unpack8(*reinterpret_cast<const uint4 *>(rp), ref);
            uint32_t lo[2] = {0, 0}, hi[2] = {0, 0};
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint16_t x = cur[i] ^ ref[i];
                lo[i >> 2] |= (uint32_t)(x & 0xff) << (8 * (i & 3));
                hi[i >> 2] |= (uint32_t)(x >> 8) << (8 * (i & 3));
            }
            const int K = un.tex == 0 ? K_irr : K_vis;
            const size_t NN = (size_t)un.N * un.N, plane_bytes = (size_t)K * NN;
            uint8_t *dlo = (un.tex == 0 ? planes_i : planes_v) + (size_t)(2 * un.c) * plane_bytes + (size_t)k * NN + un.t0;
            uint8_t *dhi = dlo + plane_bytes;
            *reinterpret_cast<uint2 *>(dlo) = make_uint2(lo[0], lo[1]);
            *reinterpret_cast<uint2 *>(dhi) = make_uint2(hi[0], hi[1]);
            *reinterpret_cast<uint4 *>(rp) =
                make_uint4((uint32_t)cur[0] | ((uint32_t)cur[1] << 16), (uint32_t)cur[2] | ((uint32_t)cur[3] << 16),
                           (uint32_t)cur[4] | ((uint32_t)cur[5] << 16), (uint32_t)cur[6] | ((uint32_t)cur[7] << 16));
            const uint32_t wlo = (uint32_t)((dlo - (b.packet + 32)) >> 2), whi = (uint32_t)((dhi - (b.packet + 32)) >> 2);
            part += word_hash(lo[0], wlo) + word_hash(lo[1], wlo + 1) + word_hash(hi[0], whi) + word_hash(hi[1], whi + 1);
        }
    }
    // the block's scratch is reused by its next tile
    __syncthreads();
    return part;
}

// The block's sum of its threads' shares (every thread must call it; thread
// 0 receives the sum).
__device__ __forceinline__ uint32_t block_sum(uint32_t part, uint32_t *sh) {
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = part;
    __syncthreads();
    uint32_t sum = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kPackThreads / 64; ++w) sum += sh[w];
    return sum;
}

__device__ __forceinline__ void write_header(const PackBuffers &b, int P, int K_irr, int K_vis, uint32_t client,
                                             uint32_t seq) {
    uint32_t *h = reinterpret_cast<uint32_t *>(b.packet);
    h[kHdrMagic] = kPacketMagic;
    h[kHdrVersion] = kPacketVersion;
    h[kHdrClient] = client;
    h[kHdrSeq] = seq;
    h[kHdrProbes] = (uint32_t)P;
    h[kHdrKIrr] = (uint32_t)K_irr;
    h[kHdrKVis] = (uint32_t)K_vis;
}

// The checksum share of tile 'tile' (thread 0): added to its group's word;
// the group's last adder resets that word and adds the group's sum to the
// final word, whose last adder resets it and writes the header checksum.
// Sums are modulo 2^32 (the checksum is a sum of word hashes, so shares add
// in any order); a word's low 48 bits hold at most 256 shares.
__device__ __forceinline__ void add_checksum_share(const PackBuffers &b, int n_tiles, int tile, uint32_t share) {
    constexpr unsigned long long kOne = 1ull << 48;
    const int g = tile % kCksGroups;
    const int members = (n_tiles - g + kCksGroups - 1) / kCksGroups;
    unsigned long long *gw = b.cks + (size_t)g * kCksStride;
    const unsigned long long old = atomicAdd(gw, kOne | share);
    if ((int)(old >> 48) != members - 1) return;
    atomicExch(gw, 0ull);
    const uint32_t gsum = (uint32_t)(old + share);
    unsigned long long *fw = b.cks + (size_t)kCksGroups * kCksStride;
    const unsigned long long fold = atomicAdd(fw, kOne | gsum);
    if ((int)(fold >> 48) != min(kCksGroups, n_tiles) - 1) return;
    atomicExch(fw, 0ull);
    reinterpret_cast<uint32_t *>(b.packet)[kHdrChecksum] = (uint32_t)(fold + gsum);
}

// Compaction, one block per tile. FUSED: the block reduces the tile
// summaries itself (small tile counts, no scan launch); otherwise the scan
// left the summary before the tile and the totals. Each block adds its
// checksum share (add_checksum_share); block 0 writes the rest of the header.
template <bool FUSED>
__global__ __launch_bounds__(kPackThreads) void k_pack_compact(PackBuffers b, int P, uint32_t client, uint32_t seq) {
    __shared__ PackSmem sm;
    __shared__ CompactShared cs;
    __shared__ TileSum red[2 * kPackThreads / 64];
    const int tile = blockIdx.x;
    const int n_tiles = (P + kPackQ - 1) / kPackQ;
    TileSum before, tot;
    if (FUSED) {
        reduce_tiles<kPackThreads>(b, n_tiles, tile, before, tot, red);
    } else {
        before = load_tile_sum(b, tile);
        tot = tile_sum_none();
        tot.ci = (int)b.totals[0];
        tot.cv = (int)b.totals[1];
        tot.li = (int)b.totals[2];
        tot.si = (int)b.totals[3];
    }
    const uint32_t part = compact_tile(b, P, tile, before, tot, sm, false, cs);
    const uint32_t sum = block_sum(part, sm.part);
    if (threadIdx.x == 0) {
        if (tile == 0) write_header(b, P, tot.ci, tot.cv, client, seq);
        add_checksum_share(b, n_tiles, tile, sum);
    }
}

__global__ void k_zero(uint32_t *p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)blockDim.x * gridDim.x)
        p[i] = 0u;
}

hipError_t launch_pack_mask(const PackBuffers &b, int P, float tau_irr, float tau_vis, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_mask, dim3((P + kPackQ - 1) / kPackQ), dim3(kPackThreads), 0, s, b, P, tau_irr, tau_vis);
    return hipGetLastError();
}

hipError_t launch_pack_scan(const PackBuffers &b, int P, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_scan, dim3(1), dim3(kScanThreads), 0, s, b, (P + kPackQ - 1) / kPackQ);
    return hipGetLastError();
}

bool pack_fused(int P) { return (P + kPackQ - 1) / kPackQ <= kPackFusedTiles; }

hipError_t launch_pack_compact(const PackBuffers &b, int P, uint32_t client, uint32_t seq, hipStream_t s) {
    if (pack_fused(P))
        hipLaunchKernelGGL(k_pack_compact<true>, dim3((P + kPackQ - 1) / kPackQ), dim3(kPackThreads), 0, s, b, P,
                           client, seq);
    else
        hipLaunchKernelGGL(k_pack_compact<false>, dim3((P + kPackQ - 1) / kPackQ), dim3(kPackThreads), 0, s, b, P,
                           client, seq);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p, words);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pack without allocation: the per-call intermediates (masks, tile
// summaries, totals, checksum counters) in one static device array
// ---------------------------------------------------------------------------
// Layout of the array for up to kNoAllocMaxProbes probes (offsets in bytes,
// each section 256-byte aligned).
constexpr int kNoAllocTiles = (kNoAllocMaxProbes + kPackTile - 1) / kPackTile;
constexpr size_t kScrTiles = 0;
constexpr size_t kScrTiles2 = kScrTiles + (size_t)kNoAllocTiles * sizeof(int4);
constexpr size_t kScrCks = kScrTiles2 + ((size_t)kNoAllocTiles * sizeof(int2) + 255) / 256 * 256;
constexpr size_t kScrTsum = kScrCks + (kCksBytes + 255) / 256 * 256;
constexpr size_t kScrTotals = kScrTsum + ((size_t)kNoAllocTiles * 4 + 255) / 256 * 256;
constexpr size_t kScrMaskIrr = kScrTotals + 256;
constexpr size_t kScrMaskVis = kScrMaskIrr + ((size_t)kNoAllocMaxProbes + 255) / 256 * 256;
constexpr size_t kScrEnd = kScrMaskVis + ((size_t)kNoAllocMaxProbes + 255) / 256 * 256;
static_assert(kScrEnd == kNoAllocScratchBytes, "scratch layout and its stated size agree");

// One copy per device; each GPU the library runs on holds it until the
// process ends. Host code never passes this name to a kernel: it uses the
// device address that hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<unsigned char *> g_scratch_ptr;  // per device, null until set up

hipError_t noalloc_scratch_init(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    // the checksum counters start at zero; every pack leaves them at zero
    e = hipMemset((unsigned char *)ptr + kScrCks, 0, kCksBytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (unsigned char *)ptr;
    return hipSuccess;
}

unsigned char *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < (int)g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

// The pack's launch sequence over caller-owned maps, reference and packet,
// with every intermediate in the device's scratch array (ptr from
// noalloc_scratch). Every intermediate is written before it is read, and
// the checksum counters are back at zero when a call ends, so nothing is
// cleared between calls.
hipError_t launch_pack_noalloc(unsigned char *scr, const uint16_t *cur_irr, const uint16_t *cur_vis, uint16_t *ref_irr,
                               uint16_t *ref_vis, int P, float tau_irr, float tau_vis, uint32_t client, uint32_t seq,
                               uint8_t *packet, hipStream_t s) {
    PackBuffers b;
    b.cur_irr = cur_irr;
    b.cur_vis = cur_vis;
    b.ref_irr = ref_irr;
    b.ref_vis = ref_vis;
    b.mask_irr = scr + kScrMaskIrr;
    b.mask_vis = scr + kScrMaskVis;
    b.tiles = reinterpret_cast<int4 *>(scr + kScrTiles);
    b.totals = reinterpret_cast<uint32_t *>(scr + kScrTotals);
    b.tiles2 = reinterpret_cast<int2 *>(scr + kScrTiles2);
    b.cks = reinterpret_cast<unsigned long long *>(scr + kScrCks);
    b.tsum = reinterpret_cast<uint32_t *>(scr + kScrTsum);
    b.packet = packet;
    b.active = nullptr;
    b.view = nullptr;
    hipError_t e = launch_pack_mask(b, P, tau_irr, tau_vis, s);
    if (e == hipSuccess && !pack_fused(P)) e = launch_pack_scan(b, P, s);
    if (e == hipSuccess) e = launch_pack_compact(b, P, client, seq, s);
    return e;
}

}  // namespace pv
