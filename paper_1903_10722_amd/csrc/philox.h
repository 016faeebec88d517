// philox.h -- Philox4x64-10 counter-based generator for gfx950 device code.
//
// Definition: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11.  One block maps a 4 x 64-bit counter and a 2 x 64-bit
// key to 4 x 64-bit words through 10 rounds; each round multiplies counter
// words 0 and 2 by the two Philox multipliers (full 128-bit products), and
// the key is advanced by the two Weyl increments before every round but the
// first.
//
// Stream convention of this library: key = (seed, instance id); counter =
// (block index, island << 32 | slot, sub << 32 | generation, purpose).  Draw
// d of a stream is the (d % 2 == 0 ? low : high) 32-bit half of word
// (d % 8) / 2 of block d / 8.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flowshop {

enum Purpose : uint32_t { kInit = 3, kCell = 4, kPair = 5, kMlpInit = 7, kMlpBatch = 8 };

struct Block4 {
    uint64_t w[4];
};

__device__ __forceinline__ Block4 philox4x64_10(uint64_t x0, uint64_t x1, uint64_t x2, uint64_t x3,
                                                uint64_t k0, uint64_t k1)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round != 0) {
            k0 += kWeylA;
            k1 += kWeylB;
        }
        const uint64_t pa_lo = kMulA * x0, pa_hi = __umul64hi(kMulA, x0);
        const uint64_t pb_lo = kMulB * x2, pb_hi = __umul64hi(kMulB, x2);
        const uint64_t y0 = pb_hi ^ x1 ^ k0;
        const uint64_t y2 = pa_hi ^ x3 ^ k1;
        x0 = y0;
        x1 = pb_lo;
        x2 = y2;
        x3 = pa_lo;
    }
    Block4 b;
    b.w[0] = x0;
    b.w[1] = x1;
    b.w[2] = x2;
    b.w[3] = x3;
    return b;
}

__device__ __forceinline__ Block4 stream_block(uint64_t seed, uint64_t inst, uint32_t island, uint32_t slot,
                                               uint32_t sub, uint32_t gen, uint32_t purpose, uint32_t block)
{
    return philox4x64_10((uint64_t)block, ((uint64_t)island << 32) | slot, ((uint64_t)sub << 32) | gen,
                         (uint64_t)purpose, seed, inst);
}

// 32-bit draw d (0..7) of a block; d must be a compile-time constant after
// unrolling so that the word index stays in registers.
__device__ __forceinline__ uint32_t draw32(const Block4& b, int d)
{
    const uint64_t w = b.w[(d & 7) >> 1];
    return (d & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
}

// Integer in [0, r): high half of the 64-bit product (multiply-shift).
__device__ __forceinline__ uint32_t below(uint32_t u, uint32_t r)
{
    return (uint32_t)(((uint64_t)u * (uint64_t)r) >> 32);
}

}  // namespace flowshop
