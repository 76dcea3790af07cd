// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the
// published multipliers and Weyl key increments.  Shared by the device code of
// the tempering chains and of the learned proposal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

// Rounds R0 .. R1-1 of Philox4x32 on the counter block c (in place); round r
// uses the key (k0 + r W0, k1 + r W1).  Running the rounds in pieces lets a
// kernel spread one block's arithmetic over several memory waits.
template <int R0, int R1>
__device__ __forceinline__ void philox4x32_rounds(uint32_t (&c)[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = R0; r < R1; ++r) {
        const uint32_t kr0 = k0 + (uint32_t)r * 0x9E3779B9u;
        const uint32_t kr1 = k1 + (uint32_t)r * 0xBB67AE85u;
        // each 32x32->64 product as one 64-bit multiply (one v_mad_u64_u32
        // on the vector unit instead of a v_mul_lo_u32 and a v_mul_hi_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        // three-input XOR in one instruction (v_bitop3_b32, truth table 0x96);
        // rounds 0 and 1 keep plain XORs, whose operands are often wave-uniform
        // (counter words shared by the wave), so they stay on the scalar unit
        const uint32_t n0 = r >= 2 ? __builtin_amdgcn_bitop3_b32(hi1, c[1], kr0, 0x96) : hi1 ^ c[1] ^ kr0;
        const uint32_t n2 = r >= 2 ? __builtin_amdgcn_bitop3_b32(hi0, c[3], kr1, 0x96) : hi0 ^ c[3] ^ kr1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t (&out)[4])
{
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
    philox4x32_rounds<0, 10>(out, k0, k1);
}

}  // namespace sk
