// Device-side counter-based hash for the Monte Carlo trials.
//
// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel Random
// Numbers: As Easy as 1, 2, 3", SC'11): each round multiplies counter words 0
// and 2 by two fixed odd constants into 128-bit products; the new counter is
// (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)), and the
// key advances by two Weyl constants between rounds.  The key (rng_seed,
// domain) is uniform across a wavefront, so the key schedule runs on the
// scalar unit.
//
// One call serves eight consecutive trials: the counter is (id, t >> 3, 0, 0)
// and trial t takes 32-bit half (t & 1) of output word (t & 7) >> 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imsim {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;

constexpr uint64_t kDomainIcArc = 1;
constexpr uint64_t kDomainLtNode = 2;

struct Block4 {
    uint64_t w0, w1, w2, w3;
};

// Full 128-bit product of two 64-bit words from four 32 x 32 -> 64 partial
// products: a*b = al*bl + 2^32 (al*bh + ah*bl) + 2^64 ah*bh, with the middle
// terms accumulated so that no partial sum overflows 64 bits.
__device__ __forceinline__ void mul_wide(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi)
{
    const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32);
    const uint32_t bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
    const uint64_t p0 = (uint64_t)al * bl;
    const uint64_t t = (uint64_t)al * bh + (p0 >> 32);
    const uint64_t u = (uint64_t)ah * bl + (uint32_t)t;
    hi = (uint64_t)ah * bh + ((t >> 32) + (u >> 32));
    lo = (u << 32) | (uint32_t)p0;
}

// Philox4x64-10 of counter (c0, c1, 0, 0) under key (k0, k1).
__device__ __forceinline__ Block4 philox_block(uint64_t c0, uint64_t c1, uint64_t k0, uint64_t k1)
{
    uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t lo_a, hi_a, lo_b, hi_b;
        mul_wide(kPhiloxM0, x0, lo_a, hi_a);
        mul_wide(kPhiloxM1, x2, lo_b, hi_b);
        const uint64_t n0 = hi_b ^ x1 ^ k0;
        const uint64_t n2 = hi_a ^ x3 ^ k1;
        x0 = n0;
        x1 = lo_b;
        x2 = n2;
        x3 = lo_a;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return Block4{x0, x1, x2, x3};
}

// The 32-bit value of lane j (0..7) of a block.
__device__ __forceinline__ uint32_t block_lane(const Block4& b, uint32_t j)
{
    const uint64_t w = (j >> 1) == 0 ? b.w0 : (j >> 1) == 1 ? b.w1 : (j >> 1) == 2 ? b.w2 : b.w3;
    return (j & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
}

__device__ __forceinline__ uint32_t hash32(uint64_t rng_seed, uint64_t domain, uint64_t trial, uint64_t id)
{
    const Block4 b = philox_block(id, trial >> 3, rng_seed, domain);
    return block_lane(b, (uint32_t)(trial & 7));
}

}  // namespace imsim
