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

// The same function with a different instruction schedule, used for the IC
// arc coins: the middle partial products are summed by one v_mad_u64_u32
// (mid = xh*ml + xl*mh, whose carry out of bit 64 has weight 2^96) and the
// columns above bit 32 by a 32-bit carry chain, the first round skips the
// product of the zero word x2, and each three-way XOR is one v_bitop3_b32 per
// half.  Both forms give identical words; which one the compiler turns into
// faster code depends on the call site (measured on MI355X: the IC coin walk
// of the word-local tasks 1.6x faster with this form, the LT threshold draws
// 4-16% slower, so each site keeps the faster one).
__device__ __forceinline__ void mul_wide_chain(uint64_t x, uint64_t m, uint64_t& lo, uint64_t& hi)
{
    const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
    const uint32_t ml = (uint32_t)m, mh = (uint32_t)(m >> 32);
    const uint64_t p0 = (uint64_t)xl * ml;
    const uint64_t p1 = (uint64_t)xl * mh;
    const uint64_t p3 = (uint64_t)xh * mh;
    const uint64_t mid = (uint64_t)xh * ml + p1;
    const uint32_t cm = mid < p1 ? 1u : 0u;
    uint32_t c1, c2, c3;
    const uint32_t lo_h = __builtin_addc((uint32_t)(p0 >> 32), (uint32_t)mid, 0u, &c1);
    const uint32_t hi_l = __builtin_addc((uint32_t)p3, (uint32_t)(mid >> 32), c1, &c2);
    const uint32_t hi_h = __builtin_addc((uint32_t)(p3 >> 32), cm, c2, &c3);
    lo = ((uint64_t)lo_h << 32) | (uint32_t)p0;
    hi = ((uint64_t)hi_h << 32) | hi_l;
}

__device__ __forceinline__ uint64_t xor3_64(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t l = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0x96);
    const uint32_t h = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), 0x96);
    return (uint64_t)l | ((uint64_t)h << 32);
}

__device__ __forceinline__ Block4 philox_block_chain(uint64_t c0, uint64_t c1, uint64_t k0, uint64_t k1)
{
    uint64_t x0, x1, x2, x3;
    {
        uint64_t lo_a, hi_a;
        mul_wide_chain(c0, kPhiloxM0, lo_a, hi_a);
        x0 = c1 ^ k0;
        x1 = 0;
        x2 = hi_a ^ k1;
        x3 = lo_a;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        uint64_t lo_a, hi_a, lo_b, hi_b;
        mul_wide_chain(x0, kPhiloxM0, lo_a, hi_a);
        mul_wide_chain(x2, kPhiloxM1, lo_b, hi_b);
        const uint64_t n0 = xor3_64(hi_b, x1, k0);
        const uint64_t n2 = xor3_64(hi_a, x3, k1);
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
    // the form the simulation uses for this domain
    const Block4 b = domain == kDomainIcArc ? philox_block_chain(id, trial >> 3, rng_seed, domain)
                                            : philox_block(id, trial >> 3, rng_seed, domain);
    return block_lane(b, (uint32_t)(trial & 7));
}

}  // namespace imsim
