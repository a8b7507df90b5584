// Philox4x32-10 counter-based generator for device code (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11),
// written from the published round function: two 32x32->64 multiplies by
// fixed odd constants, an xor with the key, a word permutation, and a Weyl
// key schedule between the ten rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qiht {

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u;
    constexpr uint32_t kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u;
    constexpr uint32_t kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kWeylA;
            k1 += kWeylB;
        }
        // full 32 x 32 -> 64 products (one v_mad_u64_u32 each)
        const uint64_t pa = static_cast<uint64_t>(kMulA) * c.x;
        const uint64_t pb = static_cast<uint64_t>(kMulB) * c.z;
        const uint32_t pa_hi = static_cast<uint32_t>(pa >> 32), pa_lo = static_cast<uint32_t>(pa);
        const uint32_t pb_hi = static_cast<uint32_t>(pb >> 32), pb_lo = static_cast<uint32_t>(pb);
        c = make_uint4(pb_hi ^ c.y ^ k0, pb_lo, pa_hi ^ c.w ^ k1, pa_lo);
    }
    return c;
}

// Word for stream element e: word (e & 3) of block (e >> 2, stream, real).
struct PhiloxStream {
    uint32_t k0, k1, stream, real;
    uint64_t cached_block = ~0ull;
    uint4 words;

    __device__ __forceinline__ uint32_t word(uint64_t e) {
        const uint64_t blk = e >> 2;
        if (blk != cached_block) {
            cached_block = blk;
            words = philox10(make_uint4(static_cast<uint32_t>(blk),
                                        static_cast<uint32_t>(blk >> 32),
                                        stream, real),
                             k0, k1);
        }
        switch (e & 3) {
            case 0: return words.x;
            case 1: return words.y;
            case 2: return words.z;
            default: return words.w;
        }
    }
};

}  // namespace qiht
