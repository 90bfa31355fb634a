// Delta packet format shared by the server-side pack and the client-side
// receiver (layout in probestream.h at pv_pack_delta): header words, section
// sizes and the payload checksum.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pv {

constexpr uint32_t kPacketMagic = 0x4B505650u;              // "PVPK"
constexpr uint32_t kPacketVersion = 1u | (32u << 16);       // version 1, 32-byte header
constexpr int kPacketHeader = 32;
constexpr int kIrrPlaneBytes = 64;    // per sent probe and plane (8 x 8 texels)
constexpr int kVisPlaneBytes = 256;   // 16 x 16
constexpr int kIrrPlanes = 6, kVisPlanes = 4;

// Header word indices (u32, little endian).
enum { kHdrMagic = 0, kHdrVersion, kHdrClient, kHdrSeq, kHdrProbes, kHdrKIrr, kHdrKVis, kHdrChecksum };

__host__ __device__ inline uint64_t packet_index_bytes(uint64_t K_irr, uint64_t K_vis) {
    return (2 * (K_irr + K_vis) + 15) / 16 * 16;
}

__host__ __device__ inline uint64_t packet_bytes(uint64_t K_irr, uint64_t K_vis) {
    return kPacketHeader + packet_index_bytes(K_irr, K_vis) + K_irr * kIrrPlanes * kIrrPlaneBytes +
           K_vis * kVisPlanes * kVisPlaneBytes;
}

// Checksum term of payload word i: fmix32 (MurmurHash3's finaliser) of the
// word XOR i times the 32-bit golden ratio. The checksum is the wrapping sum
// of the terms, so any partition of the words can be summed in any order.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ uint32_t word_hash(uint32_t w, uint32_t word_index) {
    return fmix32(w ^ (word_index * 0x9E3779B9u));
}

}  // namespace pv
