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

__device__ __forceinline__ bool texel_changed(uint16_t a, uint16_t b, float tau) {
    if (tau == 0.f) return a != b;
    // binary16 values are exact in double and so is their difference
    const double da = (double)__half2float(__ushort_as_half(a));
    const double db = (double)__half2float(__ushort_as_half(b));
    return fabs(da - db) > (double)tau;
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
    for (int i = threadIdx.x; i < vi; i += kPackThreads) sm.irr[i] = gi[i];
    for (int i = threadIdx.x; i < vv; i += kPackThreads) sm.vis[i] = gv[i];
    if ((n & 1) && threadIdx.x == 0)
        reinterpret_cast<uint2 *>(sm.irr)[2 * vi] = reinterpret_cast<const uint2 *>(gi)[2 * vi];
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

// Change mask of every probe: any interior texel differs (tau = 0) or
// |cur - ref| > tau. Each block also leaves a summary of its tile (changed
// counts and last changed probe per texture) for the scan.
__global__ __launch_bounds__(kPackThreads) void k_pack_mask(PackBuffers b, int P, float tau_irr, float tau_vis) {
    __shared__ PackSmem sm;
    const int p0 = blockIdx.x * kPackQ;
    if (p0 >= P) return;
    if (threadIdx.x < kPackQ * 2) sm.changed[threadIdx.x >> 1][threadIdx.x & 1] = 0;
    stage_tiles(b, p0, P, sm);
    __syncthreads();
    const int n = min(kPackQ, P - p0);
    const int units = kPackQ * (kIrrUnits + kVisUnits);
    for (int u = threadIdx.x; u < units; u += kPackThreads) {
        const Unit un = unit_of(u);
        if (un.q >= n) continue;
        uint16_t cur[8], ref[8];
        unit_cur(sm, un, cur);
        unpack8(*reinterpret_cast<const uint4 *>(unit_ref(b, p0 + un.q, un)), ref);
        const float tau = un.tex == 0 ? tau_irr : tau_vis;
        bool ch = false;
#pragma unroll
        for (int i = 0; i < 8; ++i) ch |= texel_changed(cur[i], ref[i], tau);
        if (ch) atomicOr(&sm.changed[un.q][un.tex], 1);
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
        int4 s = make_int4(0, 0, -1, -1);
        for (int q = 0; q < n; ++q) {
            if (sm.changed[q][0]) {
                s.x++;
                s.z = p0 + q;
            }
            if (sm.changed[q][1]) {
                s.y++;
                s.w = p0 + q;
            }
        }
        b.tiles[blockIdx.x] = s;
    }
}

constexpr int kScanThreads = 1024;

// Inclusive scan of (sum, sum, max, max) across the block: wavefront
// shuffles, then the wavefront totals.
__device__ __forceinline__ int4 block_scan_tiles(int4 v, int4 *sh) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int a = __shfl_up(v.x, off), c = __shfl_up(v.y, off), z = __shfl_up(v.z, off), w = __shfl_up(v.w, off);
        if (lane >= off) {
            v.x += a;
            v.y += c;
            v.z = max(v.z, z);
            v.w = max(v.w, w);
        }
    }
    if (lane == 63) sh[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < kScanThreads / 64; ++k) {
            sh[k].x += sh[k - 1].x;
            sh[k].y += sh[k - 1].y;
            sh[k].z = max(sh[k].z, sh[k - 1].z);
            sh[k].w = max(sh[k].w, sh[k - 1].w);
        }
    __syncthreads();
    if (wv > 0) {
        const int4 o = sh[wv - 1];
        v.x += o.x;
        v.y += o.y;
        v.z = max(v.z, o.z);
        v.w = max(v.w, o.w);
    }
    return v;
}

// One block: replaces every tile summary by the exclusive prefix of the tiles
// before it (changed counts, last changed probe) and stores the totals
// K_irr, K_vis in totals[0], totals[1]; clears the packet checksum.
__global__ __launch_bounds__(kScanThreads) void k_pack_scan(PackBuffers b, int n_tiles) {
    __shared__ int4 sh[kScanThreads / 64];
    const int per = (n_tiles + kScanThreads - 1) / kScanThreads;
    const int lo = min(n_tiles, (int)threadIdx.x * per), hi = min(n_tiles, lo + per);
    int4 mine = make_int4(0, 0, -1, -1);
    for (int t = lo; t < hi; ++t) {
        const int4 s = b.tiles[t];
        mine.x += s.x;
        mine.y += s.y;
        mine.z = max(mine.z, s.z);
        mine.w = max(mine.w, s.w);
    }
    const int4 inc = block_scan_tiles(mine, sh);
    int4 run = make_int4(inc.x - mine.x, inc.y - mine.y, -1, -1);
    // exclusive max: the previous thread's inclusive value
    const int pz = __shfl_up(inc.z, 1), pw = __shfl_up(inc.w, 1);
    if ((threadIdx.x & 63) != 0) {
        run.z = pz;
        run.w = pw;
    } else if (threadIdx.x > 0) {
        run.z = sh[(threadIdx.x >> 6) - 1].z;
        run.w = sh[(threadIdx.x >> 6) - 1].w;
    }
    for (int t = lo; t < hi; ++t) {
        const int4 s = b.tiles[t];
        b.tiles[t] = run;
        run.x += s.x;
        run.y += s.y;
        run.z = max(run.z, s.z);
        run.w = max(run.w, s.w);
    }
    if (threadIdx.x == kScanThreads - 1) {
        b.totals[0] = (uint32_t)inc.x;
        b.totals[1] = (uint32_t)inc.y;
        reinterpret_cast<uint32_t *>(b.packet)[7] = 0u;
    }
}

// Sums (x, y) and maxima (z, w) of the mask pass's tile summaries over
// tiles [0, upto) and the totals over all n_tiles, reduced by the whole
// block (every thread must call it).
template <int T>
__device__ __forceinline__ void reduce_tiles(const int4 *tiles, int n_tiles, int upto, int4 &before, int2 &total,
                                             int4 *sh) {
    int4 pre = make_int4(0, 0, -1, -1);
    int2 tot = make_int2(0, 0);
    for (int t = threadIdx.x; t < n_tiles; t += T) {
        const int4 v = tiles[t];
        tot.x += v.x;
        tot.y += v.y;
        if (t < upto) {
            pre.x += v.x;
            pre.y += v.y;
            pre.z = max(pre.z, v.z);
            pre.w = max(pre.w, v.w);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        pre.x += __shfl_xor(pre.x, off);
        pre.y += __shfl_xor(pre.y, off);
        pre.z = max(pre.z, __shfl_xor(pre.z, off));
        pre.w = max(pre.w, __shfl_xor(pre.w, off));
        tot.x += __shfl_xor(tot.x, off);
        tot.y += __shfl_xor(tot.y, off);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[2 * wv] = pre;
        sh[2 * wv + 1] = make_int4(tot.x, tot.y, 0, 0);
    }
    __syncthreads();
    before = make_int4(0, 0, -1, -1);
    total = make_int2(0, 0);
    for (int w = 0; w < T / 64; ++w) {
        const int4 a = sh[2 * w], c = sh[2 * w + 1];
        before.x += a.x;
        before.y += a.y;
        before.z = max(before.z, a.z);
        before.w = max(before.w, a.w);
        total.x += c.x;
        total.y += c.y;
    }
    __syncthreads();
}

// Compaction of one tile: its changed probes' ranks (the tile's prefix plus
// the changed lanes below), their delta-coded index entries, XOR byte planes
// and reference update, and the plane words' checksum share (summed by the
// finish kernel with the index section's). FUSED: the block reduces the
// tile summaries itself (small tile counts, no scan launch); otherwise the
// scan left the prefix in the tile's summary and the totals.
template <bool FUSED>
__global__ __launch_bounds__(kPackThreads) void k_pack_compact(PackBuffers b, int P) {
    __shared__ PackSmem sm;
    __shared__ int rank_s[kPackQ][2];
    __shared__ int any_s;
    __shared__ int4 red[2 * kPackThreads / 64];
    const int tile = blockIdx.x, p0 = tile * kPackQ;
    const int n = min(kPackQ, P - p0);
    int4 before;
    int K_irr, K_vis;
    if (FUSED) {
        int2 tot;
        reduce_tiles<kPackThreads>(b.tiles, (P + kPackQ - 1) / kPackQ, tile, before, tot, red);
        K_irr = tot.x;
        K_vis = tot.y;
    } else {
        before = b.tiles[tile];
        K_irr = (int)b.totals[0];
        K_vis = (int)b.totals[1];
    }
    const int idx_bytes = ((2 * (K_irr + K_vis) + 15) / 16) * 16;
    uint16_t *idx_i = reinterpret_cast<uint16_t *>(b.packet + 32);
    uint16_t *idx_v = idx_i + K_irr;
    if (threadIdx.x < 64) {
        // ranks and index entries of the tile's changed probes: lane q owns
        // probe p0 + q; its rank counts the changed lanes below it, its
        // predecessor is the highest of them (or the last one before the tile)
        const int q = threadIdx.x, p = p0 + q;
        const bool ci = q < n && b.mask_irr[p] != 0, cv = q < n && b.mask_vis[p] != 0;
        const unsigned long long below = (1ull << q) - 1ull;
        const unsigned long long bi = __ballot(ci), bvv = __ballot(cv);
        const unsigned long long mi = bi & below, mv = bvv & below;
        if (q == 0) any_s = (bi | bvv) != 0ull;
        if (q < kPackQ) {
            rank_s[q][0] = rank_s[q][1] = -1;
            if (ci) {
                const int k = before.x + __popcll(mi);
                const int prev = mi ? p0 + 63 - __clzll((long long)mi) : before.z;
                idx_i[k] = (uint16_t)(k == 0 ? p : p - prev);
                rank_s[q][0] = k;
            }
            if (cv) {
                const int k = before.y + __popcll(mv);
                const int prev = mv ? p0 + 63 - __clzll((long long)mv) : before.w;
                idx_v[k] = (uint16_t)(k == 0 ? p : p - prev);
                rank_s[q][1] = k;
            }
        }
    }
    __syncthreads();
    uint32_t part = 0;
    if (any_s) {
        stage_tiles(b, p0, P, sm);
        __syncthreads();
        uint8_t *planes_i = b.packet + 32 + idx_bytes;
        uint8_t *planes_v = planes_i + (size_t)K_irr * 6 * 64;
        const int units = kPackQ * (kIrrUnits + kVisUnits);
        for (int u = threadIdx.x; u < units; u += kPackThreads) {
            const Unit un = unit_of(u);
            if (un.q >= n) continue;
            const int k = rank_s[un.q][un.tex];
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
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((threadIdx.x & 63) == 0) sm.part[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kPackThreads / 64; ++w) s += sm.part[w];
        b.partial[tile] = s;
    }
}

// One block: pads and hashes the index section, adds the compaction blocks'
// plane hashes, writes the header (FUSED: the totals from the tile summaries).
template <bool FUSED>
__global__ __launch_bounds__(kScanThreads) void k_pack_finish(PackBuffers b, int P, int n_tiles, uint32_t client,
                                                             uint32_t seq) {
    __shared__ uint32_t sh[kScanThreads / 64];
    __shared__ int4 red[2 * kScanThreads / 64];
    int K_irr, K_vis;
    if (FUSED) {
        int4 none;
        int2 tot;
        reduce_tiles<kScanThreads>(b.tiles, n_tiles, 0, none, tot, red);
        K_irr = tot.x;
        K_vis = tot.y;
    } else {
        K_irr = (int)b.totals[0];
        K_vis = (int)b.totals[1];
    }
    const int idx_bytes = ((2 * (K_irr + K_vis) + 15) / 16) * 16;
    uint8_t *pk = b.packet;
    if (threadIdx.x < 16) {
        const int pos = 2 * (K_irr + K_vis) + threadIdx.x;
        if (pos < idx_bytes) pk[32 + pos] = 0;
    }
    __syncthreads();
    uint32_t s = 0;
    const uint32_t *words = reinterpret_cast<const uint32_t *>(pk + 32);
    for (int wi = threadIdx.x; wi < idx_bytes / 4; wi += kScanThreads) s += word_hash(words[wi], (uint32_t)wi);
    for (int t = threadIdx.x; t < n_tiles; t += kScanThreads) s += b.partial[t];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) tot += sh[w];
        uint32_t *h = reinterpret_cast<uint32_t *>(pk);
        h[kHdrMagic] = kPacketMagic;
        h[kHdrVersion] = kPacketVersion;
        h[kHdrClient] = client;
        h[kHdrSeq] = seq;
        h[kHdrProbes] = (uint32_t)P;
        h[kHdrKIrr] = (uint32_t)K_irr;
        h[kHdrKVis] = (uint32_t)K_vis;
        h[kHdrChecksum] = tot;
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

hipError_t launch_pack_compact(const PackBuffers &b, int P, hipStream_t s) {
    if (pack_fused(P))
        hipLaunchKernelGGL(k_pack_compact<true>, dim3((P + kPackQ - 1) / kPackQ), dim3(kPackThreads), 0, s, b, P);
    else
        hipLaunchKernelGGL(k_pack_compact<false>, dim3((P + kPackQ - 1) / kPackQ), dim3(kPackThreads), 0, s, b, P);
    return hipGetLastError();
}

hipError_t launch_pack_finish(const PackBuffers &b, int P, uint32_t client, uint32_t seq, hipStream_t s) {
    const int n_tiles = (P + kPackQ - 1) / kPackQ;
    if (pack_fused(P))
        hipLaunchKernelGGL(k_pack_finish<true>, dim3(1), dim3(kScanThreads), 0, s, b, P, n_tiles, client, seq);
    else
        hipLaunchKernelGGL(k_pack_finish<false>, dim3(1), dim3(kScanThreads), 0, s, b, P, n_tiles, client, seq);
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
// summaries, totals, checksum shares) in one static device array
// ---------------------------------------------------------------------------
// Layout of the array for up to kNoAllocMaxProbes probes (offsets in bytes,
// each section 256-byte aligned).
constexpr int kNoAllocTiles = (kNoAllocMaxProbes + kPackTile - 1) / kPackTile;
constexpr size_t kScrTiles = 0;
constexpr size_t kScrPartial = kScrTiles + (size_t)kNoAllocTiles * sizeof(int4);
constexpr size_t kScrTotals = kScrPartial + ((size_t)kNoAllocTiles * 4 + 255) / 256 * 256;
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
    g_scratch_ptr[device] = (unsigned char *)ptr;
    return hipSuccess;
}

unsigned char *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < (int)g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

// The pack's launch sequence over caller-owned maps, reference and packet,
// with every intermediate in the device's scratch array (ptr from
// noalloc_scratch). Every intermediate is written before it is read, so
// nothing is cleared between calls.
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
    b.partial = reinterpret_cast<uint32_t *>(scr + kScrPartial);
    b.packet = packet;
    b.active = nullptr;
    b.view = nullptr;
    hipError_t e = launch_pack_mask(b, P, tau_irr, tau_vis, s);
    if (e == hipSuccess && !pack_fused(P)) e = launch_pack_scan(b, P, s);
    if (e == hipSuccess) e = launch_pack_compact(b, P, s);
    if (e == hipSuccess) e = launch_pack_finish(b, P, client, seq, s);
    return e;
}

}  // namespace pv
