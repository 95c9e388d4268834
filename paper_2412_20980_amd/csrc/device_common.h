// Device-side helpers shared by the kernels of the HIP library: the
// Philox4x32-10 counter-based generator, the integer maps built on it, and
// small bit-set utilities.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gapa {

// Random streams: the top byte of counter word 3 says which decision a draw
// feeds; the low 24 bits count rejection attempts.
enum Stream : uint32_t {
    kStreamInit = 0,
    kStreamSelect = 1,
    kStreamXover = 2,
    kStreamRepair = 3,
    kStreamMutate = 4,
};
constexpr uint32_t kMaxAttempts = 1u << 24;

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32 -> 64-bit products of counter words 0 and 2 whose halves are swapped
// and xored with the other counter words and the round key; the key advances
// by the golden-ratio and sqrt(3)-1 Weyl constants between rounds.
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 64-bit product is one v_mad_u64_u32 (both halves at once)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// The counter of a draw is (slot, individual, generation, stream<<24 | attempt)
// and the key is the 64-bit seed split into its low and high words.
__device__ __forceinline__ Words4 draw(uint64_t seed, uint32_t slot, uint32_t ind, uint32_t gen,
                                       uint32_t stream, uint32_t attempt)
{
    return philox4x32_10(slot, ind, gen, (stream << 24) | attempt, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Integer in [0, m): high word of the 64-bit product w * m.
__device__ __forceinline__ uint32_t bounded(uint32_t w, uint32_t m)
{
    return __umulhi(w, m);
}

__device__ __forceinline__ bool test_bit(const uint32_t *bits, uint32_t i)
{
    return (bits[i >> 5] >> (i & 31)) & 1u;
}

// Workgroups go to the chip's eight XCDs in turn (workgroup b to XCD b mod 8),
// each XCD with its own L2.  This maps workgroup b of nblk to a tile so that
// every XCD takes one contiguous range of tiles: neighbouring tiles that share
// cache lines are then read through the same L2.  A bijection on [0, nblk).
__device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t nblk)
{
    const int32_t q = nblk >> 3, r = nblk & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

}  // namespace gapa
