// philox.hpp -- device Philox4x32-10 for gfx950.
//
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds
// of two 32x32->64-bit multiplies and xors, with the 64-bit key bumped by the
// Weyl increments between rounds.  Written for the GPU library alone.  The key
// and the t/tag/stream counter words are wave-uniform, so the compiler keeps
// them, and the key schedule, in scalar registers; only the index word and the
// products are per-lane.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swccl {

struct U4 {
    uint32_t v0, v1, v2, v3;
};

// a ^ b ^ k in one gfx950 three-input bit operation (truth table 0x96 is the
// parity of the three inputs); k is wave-uniform.
__device__ __forceinline__ uint32_t xor3_vvs(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = static_cast<uint64_t>(0xD2511F53u) * c0;  // one v_mad_u64_u32
        const uint64_t b = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        uint32_t n0, n2;
        if (r == 0) {  // c1..c3 may still be wave-uniform: leave the first round to the compiler
            n0 = static_cast<uint32_t>(b >> 32) ^ c1 ^ k0;
            n2 = static_cast<uint32_t>(a >> 32) ^ c3 ^ k1;
        } else {
            n0 = xor3_vvs(static_cast<uint32_t>(b >> 32), c1, k0);
            n2 = xor3_vvs(static_cast<uint32_t>(a >> 32), c3, k1);
        }
        c1 = static_cast<uint32_t>(b);
        c3 = static_cast<uint32_t>(a);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// The same block with the key schedule given: rk[2r] and rk[2r + 1] are the
// two key words of round r (the key bumped r times), read from scalar memory
// where the caller keeps them rather than recomputed.
template <typename RK>
__device__ __forceinline__ U4 philox4x32_10_rk(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, RK *rk)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t b = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t k0 = rk[2 * r], k1 = rk[2 * r + 1];
        uint32_t n0, n2;
        if (r == 0) {
            n0 = static_cast<uint32_t>(b >> 32) ^ c1 ^ k0;
            n2 = static_cast<uint32_t>(a >> 32) ^ c3 ^ k1;
        } else {
            n0 = xor3_vvs(static_cast<uint32_t>(b >> 32), c1, k0);
            n2 = xor3_vvs(static_cast<uint32_t>(a >> 32), c3, k1);
        }
        c1 = static_cast<uint32_t>(b);
        c3 = static_cast<uint32_t>(a);
        c0 = n0;
        c2 = n2;
    }
    return U4{c0, c1, c2, c3};
}

// Word j (0..3) of a block, by selects rather than branches.
__device__ __forceinline__ uint32_t pick(const U4 &b, uint32_t j)
{
    const uint32_t lo = (j & 1u) ? b.v1 : b.v0, hi = (j & 1u) ? b.v3 : b.v2;
    return (j & 2u) ? hi : lo;
}

// floor(w * q / 2^32): one uniform state in 0..q-1 from a 32-bit word.
__device__ __forceinline__ uint32_t draw_state(uint32_t w, uint32_t q)
{
    return static_cast<uint32_t>((static_cast<uint64_t>(w) * q) >> 32);
}

}  // namespace swccl
