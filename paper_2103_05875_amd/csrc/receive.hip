// Client-side unpack of delta packets (Sec. 3.4: the client keeps its
// textures and applies index-based probe updates; the guard bands, dropped
// for transmission, are rebuilt on arrival).
//
// Three launches per packet, in stream order:
//   k_rx_index     one block: decodes the delta-coded index of both textures
//                  into absolute probe numbers with a block-wide scan, flags
//                  an invalid index (probe out of range, or not strictly
//                  increasing), and clears the checksum accumulator
//   k_rx_checksum  sums the payload word hashes (one atomic add per block)
//   k_rx_apply     one block per sent probe and texture: if the index was
//                  valid and the checksum matches the header, XORs the two
//                  byte planes of each channel into the interior texel and
//                  writes it with its guard copies; otherwise writes nothing
// so a corrupt packet leaves the client state as it was.
#include "blend_device.h"
#include "packet_format.h"

namespace pv {

constexpr int kRxScanThreads = 1024;
constexpr int kRxThreads = 256;

// Inclusive scan of one value per thread over a block of kRxScanThreads.
__device__ __forceinline__ uint32_t rx_block_scan(uint32_t v, uint32_t *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    if (lane == 63) sh[w] = v;
    __syncthreads();
    if (w == 0) {
        uint32_t s = lane < kRxScanThreads / 64 ? sh[lane] : 0u;
        for (int off = 1; off < kRxScanThreads / 64; off <<= 1) {
            const uint32_t u = __shfl_up(s, off);
            if (lane >= off) s += u;
        }
        if (lane < kRxScanThreads / 64) sh[lane] = s;
    }
    __syncthreads();
    const uint32_t before = w > 0 ? sh[w - 1] : 0u;
    __syncthreads();
    return v + before;
}

// Decodes K entries starting at entry 'first' of the index section into
// idx[first ..]; returns whether any entry is invalid (this thread's part).
__device__ bool rx_decode(const RxBuffers &b, int first, int K, uint32_t *sh) {
    const uint8_t *ix = b.pkt + kPacketHeader + 2 * (size_t)first;
    const int per = (K + kRxScanThreads - 1) / kRxScanThreads;
    const int k0 = min(K, (int)threadIdx.x * per), k1 = min(K, k0 + per);
    uint32_t local = 0;
    for (int k = k0; k < k1; ++k) local += (uint32_t)ix[2 * k] | ((uint32_t)ix[2 * k + 1] << 8);
    // a valid index sums to less than 65536, so 32-bit partial sums of an
    // invalid one stay exact too (at most 65536 entries of at most 65535)
    uint32_t p = rx_block_scan(local, sh) - local;
    bool bad = false;
    for (int k = k0; k < k1; ++k) {
        const uint32_t e = (uint32_t)ix[2 * k] | ((uint32_t)ix[2 * k + 1] << 8);
        p += e;
        bad |= p >= (uint32_t)b.P || (k > 0 && e == 0);
        b.idx[first + k] = (int)p;
    }
    return bad;
}

__global__ __launch_bounds__(kRxScanThreads) void k_rx_index(RxBuffers b) {
    __shared__ uint32_t sh[kRxScanThreads / 64];
    bool bad = rx_decode(b, 0, b.K_irr, sh);
    bad |= rx_decode(b, b.K_irr, b.K_vis, sh);
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) {
        b.status->bad_index = bad ? 1 : 0;
        b.status->sum = 0u;
    }
}

__global__ __launch_bounds__(kRxThreads) void k_rx_checksum(RxBuffers b) {
    __shared__ uint32_t sh[kRxThreads / 64];
    const uint32_t *words = reinterpret_cast<const uint32_t *>(b.pkt + kPacketHeader);
    uint32_t s = 0;
    for (long long i = (long long)blockIdx.x * kRxThreads + threadIdx.x; i < b.payload_words;
         i += (long long)gridDim.x * kRxThreads)
        s += word_hash(words[i], (uint32_t)i);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kRxThreads / 64; ++w) t += sh[w];
        atomicAdd(&b.status->sum, t);
    }
}

template <int N, int C>
__device__ __forceinline__ void rx_probe(uint16_t *tiles, const uint8_t *planes, int K, int k, int p) {
    constexpr int NN = N * N, S = N + 2;
    for (int e = threadIdx.x; e < C * NN; e += kRxThreads) {
        const int c = e / NN, t = e - c * NN;
        const uint32_t lo = planes[(size_t)(2 * c) * K * NN + (size_t)k * NN + t];
        const uint32_t hi = planes[(size_t)(2 * c + 1) * K * NN + (size_t)k * NN + t];
        uint16_t *tile = tiles + ((size_t)p * C + c) * S * S;
        const int i = t % N, j = t / N;
        const uint16_t v = tile[(j + 1) * S + (i + 1)] ^ (uint16_t)(lo | (hi << 8));
        store_with_guard<uint16_t>(tile, N, i, j, v);
    }
}

__global__ __launch_bounds__(kRxThreads) void k_rx_apply(RxBuffers b) {
    if (b.status->bad_index || b.status->sum != b.checksum) return;
    const uint8_t *pi = b.pkt + kPacketHeader + packet_index_bytes(b.K_irr, b.K_vis);
    const int g = blockIdx.x;
    if (g < b.K_irr) {
        rx_probe<8, 3>(b.irr, pi, b.K_irr, g, b.idx[g]);
    } else {
        const uint8_t *pv = pi + (size_t)b.K_irr * kIrrPlanes * kIrrPlaneBytes;
        const int k = g - b.K_irr;
        rx_probe<16, 2>(b.vis, pv, b.K_vis, k, b.idx[b.K_irr + k]);
    }
}

hipError_t launch_receive(const RxBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_rx_index, dim3(1), dim3(kRxScanThreads), 0, s, b);
    const long long words = b.payload_words;
    const unsigned blocks = (unsigned)std::max(1ll, std::min(1024ll, (words + kRxThreads - 1) / kRxThreads));
    hipLaunchKernelGGL(k_rx_checksum, dim3(blocks), dim3(kRxThreads), 0, s, b);
    if (b.K_irr + b.K_vis > 0)
        hipLaunchKernelGGL(k_rx_apply, dim3(b.K_irr + b.K_vis), dim3(kRxThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace pv
