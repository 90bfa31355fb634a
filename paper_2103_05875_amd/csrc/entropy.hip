// Entropy stage of a delta packet: a canonical Huffman code per byte stream
// (the index section, six irradiance planes, four visibility planes),
// streams cut into 1,024-symbol chunks so that both directions run in
// parallel. Layout in probestream.h at pv_entropy_encode.
//
// Encode, reading the packet sizes from its device header:
//   k_ent_hist    byte histograms (LDS counts, one atomic per bin and block)
//   (host)        code lengths and canonical codes from the 11 histograms:
//                 a few hundred sequential steps per stream, which a single
//                 GPU lane runs at LDS latency and the host in microseconds
//   k_ent_count   bits of every chunk
//   k_ent_layout  one block: container offsets of every chunk, the header
//                 and the per-stream tables
//   k_ent_encode  one block per chunk: codes placed by a block scan of their
//                 lengths into LDS words, written out in stream byte order
// Decode: k_ent_decode, blocks of one stream's chunks: the block builds the
// stream's 12-bit lookup table in LDS, then each thread decodes one chunk.
#include "device_common.h"
#include "packet_format.h"

namespace pv {

constexpr int kEntChunk = 1024;
constexpr int kEntMaxBits = 12;
constexpr int kEntThreads = 256;
constexpr int kEntPerThread = kEntChunk / kEntThreads;  // 4
constexpr int kEntChunkWords = kEntChunk * kEntMaxBits / 32;
constexpr int kHistSpan = 16 * kEntChunk;  // bytes per histogram block (few global atomics per bin)

// Byte span of stream k of a packet whose header is h.
__device__ __forceinline__ void ent_span(const uint8_t *pkt, int k, const uint8_t *&p, long long &n) {
    const uint32_t *h = reinterpret_cast<const uint32_t *>(pkt);
    const long long Ki = h[kHdrKIrr], Kv = h[kHdrKVis];
    const long long idx = (long long)packet_index_bytes(Ki, Kv);
    if (k == 0) {
        p = pkt + kPacketHeader;
        n = 2 * (Ki + Kv);
    } else if (k <= kIrrPlanes) {
        p = pkt + kPacketHeader + idx + (k - 1) * Ki * kIrrPlaneBytes;
        n = Ki * kIrrPlaneBytes;
    } else {
        p = pkt + kPacketHeader + idx + kIrrPlanes * Ki * kIrrPlaneBytes + (k - 1 - kIrrPlanes) * Kv * kVisPlaneBytes;
        n = Kv * kVisPlaneBytes;
    }
}

__global__ __launch_bounds__(kEntThreads) void k_ent_hist(EntBuffers e) {
    __shared__ uint32_t h[256];
    const int k = blockIdx.y;
    const uint8_t *p;
    long long n;
    ent_span(e.pkt, k, p, n);
    const long long b0 = (long long)blockIdx.x * kHistSpan;
    if (b0 >= n) return;
    h[threadIdx.x] = 0;
    __syncthreads();
    // the XOR planes are mostly zero bytes: zeros are counted per wavefront
    // with a ballot, the other values with one LDS atomic each
    const long long b1 = min(n, b0 + kHistSpan);
    for (long long i = b0 + threadIdx.x; i < b0 + kHistSpan; i += kEntThreads) {
        const bool in = i < b1;
        const uint8_t v = in ? p[i] : 1;
        const unsigned long long z = __ballot(in && v == 0);
        if ((threadIdx.x & 63) == 0 && z) atomicAdd(&h[0], (uint32_t)__popcll(z));
        if (in && v != 0) atomicAdd(&h[v], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&e.hist[k * 256 + threadIdx.x], h[threadIdx.x]);
}

// Canonical codes of a length table (one wavefront; lane l returns the codes
// of symbols l, l + 64, l + 128, l + 192): the first code of each length is
// the previous length's first code plus its count, shifted left once; a
// symbol's code is its length's first code plus the number of symbols of
// that length with a smaller value.
__device__ __forceinline__ void canonical_codes(const uint8_t *len, uint32_t code[4]) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    uint32_t count[kEntMaxBits + 1];
    unsigned long long m[4][kEntMaxBits + 1];
    for (int L = 1; L <= kEntMaxBits; ++L) {
        count[L] = 0;
        for (int g = 0; g < 4; ++g) {
            m[g][L] = __ballot(len[lane + 64 * g] == L);
            count[L] += __popcll(m[g][L]);
        }
    }
    uint32_t first[kEntMaxBits + 2];
    first[1] = 0;
    for (int L = 2; L <= kEntMaxBits + 1; ++L) first[L] = (first[L - 1] + count[L - 1]) << 1;
    for (int g = 0; g < 4; ++g) {
        const int L = len[lane + 64 * g];
        code[g] = 0;
        if (L == 0) continue;
        uint32_t r = __popcll(m[g][L] & below);
        for (int h = 0; h < g; ++h) r += __popcll(m[h][L]);
        code[g] = first[L] + r;
    }
}

__device__ __forceinline__ uint32_t ent_block_sum(uint32_t v, uint32_t *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < kEntThreads / 64; ++w) t += sh[w];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kEntThreads) void k_ent_count(EntBuffers e) {
    __shared__ uint32_t sh[kEntThreads / 64];
    const int k = blockIdx.y, c = blockIdx.x;
    const uint8_t *p;
    long long n;
    ent_span(e.pkt, k, p, n);
    const long long b0 = (long long)c * kEntChunk;
    if (b0 >= n) return;
    const uint8_t *len = e.lens + k * 256;
    uint32_t bits = 0;
    for (int j = 0; j < kEntPerThread; ++j) {
        const long long i = b0 + threadIdx.x * kEntPerThread + j;
        if (i < n) bits += len[p[i]];
    }
    bits = ent_block_sum(bits, sh);
    if (threadIdx.x == 0) e.chunk_bits[(size_t)k * e.max_chunks + c] = bits;
}

__device__ __forceinline__ void put_be32(uint8_t *q, uint32_t v) {
    q[0] = (uint8_t)(v >> 24);
    q[1] = (uint8_t)(v >> 16);
    q[2] = (uint8_t)(v >> 8);
    q[3] = (uint8_t)v;
}
__device__ __forceinline__ void put_le32(uint8_t *q, uint32_t v) {
    q[0] = (uint8_t)v;
    q[1] = (uint8_t)(v >> 8);
    q[2] = (uint8_t)(v >> 16);
    q[3] = (uint8_t)(v >> 24);
}

constexpr int kLayoutThreads = 1024;

// Exclusive scan of one value per thread over a block of kLayoutThreads;
// *total receives the sum.
__device__ __forceinline__ unsigned long long layout_scan(unsigned long long v, unsigned long long *sh,
                                                          unsigned long long *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long u = __shfl_up(incl, off);
        if (lane >= off) incl += u;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    unsigned long long before = 0, all = 0;
    for (int q = 0; q < kLayoutThreads / 64; ++q) {
        if (q < w) before += sh[q];
        all += sh[q];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// One block: the container's layout. Per stream the tables (128 + 4 + 4
// n_chunks bytes), then its chunks; chunk_off[k * max_chunks + c] = byte
// offset of the chunk's words. Each stream's chunk sizes are scanned by
// the whole block (each thread a contiguous run of chunks).
__global__ __launch_bounds__(kLayoutThreads) void k_ent_layout(EntBuffers e) {
    __shared__ unsigned long long base[kEntStreams + 1];
    __shared__ unsigned long long sh[kLayoutThreads / 64];
    const uint32_t *h = reinterpret_cast<const uint32_t *>(e.pkt);
    unsigned long long off = 8 + kPacketHeader;
    for (int k = 0; k < kEntStreams; ++k) {
        const uint8_t *p;
        long long n;
        ent_span(e.pkt, k, p, n);
        const long long nch = (n + kEntChunk - 1) / kEntChunk;
        if (threadIdx.x == 0) base[k] = off;
        off += 128 + 4 + 4 * nch;
        const long long per = (nch + kLayoutThreads - 1) / kLayoutThreads;
        const long long c0 = min(nch, (long long)threadIdx.x * per), c1 = min(nch, c0 + per);
        unsigned long long mine = 0;
        for (long long c = c0; c < c1; ++c) mine += (e.chunk_bits[(size_t)k * e.max_chunks + c] + 31) / 32 * 4;
        unsigned long long all;
        unsigned long long o = off + layout_scan(mine, sh, &all);
        for (long long c = c0; c < c1; ++c) {
            e.chunk_off[(size_t)k * e.max_chunks + c] = o;
            o += (e.chunk_bits[(size_t)k * e.max_chunks + c] + 31) / 32 * 4;
        }
        off += all;
    }
    if (threadIdx.x == 0) {
        base[kEntStreams] = off;
        *e.total = off;
        put_le32(e.out, 0x43485650u);
        put_le32(e.out + 4, 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kPacketHeader / 4; i += blockDim.x) put_le32(e.out + 8 + 4 * i, h[i]);
    for (int k = 0; k < kEntStreams; ++k) {
        const uint8_t *p;
        long long n;
        ent_span(e.pkt, k, p, n);
        const long long nch = (n + kEntChunk - 1) / kEntChunk;
        uint8_t *t = e.out + base[k];
        const uint8_t *len = e.lens + k * 256;
        for (int i = threadIdx.x; i < 128; i += blockDim.x) t[i] = (uint8_t)(len[2 * i] | (len[2 * i + 1] << 4));
        if (threadIdx.x == 0) put_le32(t + 128, (uint32_t)nch);
        for (long long c = threadIdx.x; c < nch; c += blockDim.x)
            put_le32(t + 132 + 4 * c, e.chunk_bits[(size_t)k * e.max_chunks + c]);
    }
}

__global__ __launch_bounds__(kEntThreads) void k_ent_encode(EntBuffers e) {
    __shared__ uint32_t words[kEntChunkWords];
    __shared__ uint32_t sh[kEntThreads / 64 + 1];
    const int k = blockIdx.y, c = blockIdx.x;
    const uint8_t *p;
    long long n;
    ent_span(e.pkt, k, p, n);
    const long long b0 = (long long)c * kEntChunk;
    if (b0 >= n) return;
    const uint8_t *len = e.lens + k * 256;
    const uint32_t *code = e.codes + k * 256;
    uint8_t sym[kEntPerThread];
    uint32_t bits = 0;
    for (int j = 0; j < kEntPerThread; ++j) {
        const long long i = b0 + threadIdx.x * kEntPerThread + j;
        sym[j] = i < n ? p[i] : 0;
        bits += i < n ? len[sym[j]] : 0;
    }
    for (int i = threadIdx.x; i < kEntChunkWords; i += kEntThreads) words[i] = 0;
    // exclusive scan of the threads' bit counts
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = bits;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(incl, off);
        if (lane >= off) incl += u;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int q = 0; q < w; ++q) before += sh[q];
    uint32_t pos = before + incl - bits;
    for (int j = 0; j < kEntPerThread; ++j) {
        const long long i = b0 + threadIdx.x * kEntPerThread + j;
        if (i >= n) break;
        const int L = len[sym[j]];
        const uint32_t cd = code[sym[j]];
        // the code's bits occupy stream bits pos .. pos+L-1, MSB first
        const int wi = pos >> 5, sh0 = pos & 31;
        const int room = 32 - sh0;
        if (L <= room) {
            atomicOr(&words[wi], cd << (room - L));
        } else {
            atomicOr(&words[wi], cd >> (L - room));
            atomicOr(&words[wi + 1], cd << (32 - (L - room)));
        }
        pos += L;
    }
    __syncthreads();
    const uint32_t total = sh[0] + sh[1] + sh[2] + sh[3];
    uint8_t *dst = e.out + e.chunk_off[(size_t)k * e.max_chunks + c];
    for (uint32_t i = threadIdx.x; i < (total + 31) / 32; i += kEntThreads) put_be32(dst + 4 * i, words[i]);
}

// ---------------------------------------------------------------------------
// decode
// ---------------------------------------------------------------------------
// Blocks of chunks of one stream (block list from the host): the stream's
// lookup table for the next 12 stream bits (symbol | length << 8) built in
// LDS from its length table, then one chunk per thread.
__global__ __launch_bounds__(64) void k_ent_decode(EntDecode d) {
    __shared__ uint8_t len[256];
    __shared__ uint16_t lut[1 << kEntMaxBits];
    const EntBlock blk = d.blocks[blockIdx.x];
    const uint8_t *t = d.in + d.stream_base[blk.stream];
    const int lane = threadIdx.x;
    for (int s = lane; s < 256; s += 64) len[s] = (s & 1) ? (t[s >> 1] >> 4) : (t[s >> 1] & 15);
    for (int v = lane; v < (1 << kEntMaxBits); v += 64) lut[v] = 0;
    __syncthreads();
    uint32_t code[4];
    canonical_codes(len, code);
    for (int g = 0; g < 4; ++g) {
        const int s = lane + 64 * g, L = len[s];
        if (L == 0) continue;
        const uint32_t lo = code[g] << (kEntMaxBits - L), hi = (code[g] + 1) << (kEntMaxBits - L);
        for (uint32_t v = lo; v < hi && v < (1u << kEntMaxBits); ++v) lut[v] = (uint16_t)(s | (L << 8));
    }
    __syncthreads();
    if (lane >= blk.n) return;
    const EntChunk ch = d.chunks[blk.first + lane];
    // chunks start on 4-byte boundaries of the container
    const uint32_t *src = reinterpret_cast<const uint32_t *>(d.in + ch.in_off);
    uint8_t *dst = d.pkt + ch.out_off;
    // a 64-bit window of the stream, refilled a 32-bit word at a time (the
    // words hold the stream's bytes in order: big-endian)
    unsigned long long win = 0;
    int have = 0;
    const uint32_t nwords = (ch.bits + 31) / 32;
    uint32_t next = 1;
    uint32_t ahead = nwords > 0 ? src[0] : 0u;   // the next word, loaded one refill early
    // decoded bytes leave four at a time (chunks start on 4-byte boundaries
    // of the packet), a ragged tail byte by byte
    uint32_t out = 0;
    for (int i = 0; i < ch.n_sym; ++i) {
        if (have <= 32) {
            const uint32_t w = __builtin_bswap32(ahead);
            ahead = next < nwords ? src[next] : 0u;
            ++next;
            win |= (unsigned long long)w << (32 - have);
            have += 32;
        }
        const uint16_t e = lut[win >> (64 - kEntMaxBits)];
        const int L = e >> 8;
        out |= (uint32_t)(e & 0xFF) << (8 * (i & 3));
        if ((i & 3) == 3) {
            *reinterpret_cast<uint32_t *>(dst + i - 3) = out;
            out = 0;
        }
        win <<= L;
        have -= L;
    }
    for (int i = ch.n_sym & ~3; i < ch.n_sym; ++i) dst[i] = (uint8_t)(out >> (8 * (i & 3)));
}

hipError_t launch_entropy_hist(const EntBuffers &e, int max_chunks, hipStream_t s) {
    hipLaunchKernelGGL(k_ent_hist, dim3((max_chunks * kEntChunk + kHistSpan - 1) / kHistSpan, kEntStreams),
                       dim3(kEntThreads), 0, s, e);
    return hipGetLastError();
}

hipError_t launch_entropy_encode(const EntBuffers &e, int max_chunks, hipStream_t s) {
    hipLaunchKernelGGL(k_ent_count, dim3(max_chunks, kEntStreams), dim3(kEntThreads), 0, s, e);
    hipLaunchKernelGGL(k_ent_layout, dim3(1), dim3(kLayoutThreads), 0, s, e);
    hipLaunchKernelGGL(k_ent_encode, dim3(max_chunks, kEntStreams), dim3(kEntThreads), 0, s, e);
    return hipGetLastError();
}

hipError_t launch_entropy_decode(const EntDecode &d, hipStream_t s) {
    if (d.n_blocks > 0) hipLaunchKernelGGL(k_ent_decode, dim3(d.n_blocks), dim3(64), 0, s, d);
    return hipGetLastError();
}

}  // namespace pv
