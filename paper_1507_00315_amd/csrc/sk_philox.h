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

// The first four rounds of a block whose counter is (b_lo, b_hi, w2, w3)
// with b_lo, b_hi and w2 shared by the wave and w3 not: split into the part
// that involves only the shared words (four values per block, which a kernel
// can compute for 64 blocks at once, one block per lane, and read back one
// block at a time) and the part that involves w3.  Rounds 1 to 3 of the
// shared part are the products and XORs that never meet w3:
//   round 0: u0 = hi(M0 b_lo) ^ k1 (word 2 is u0 ^ w3); word 0 is
//            hi(M1 w2) ^ b_hi ^ k0, word 3 lo(M0 b_lo);
//   round 1: word 2 becomes hi(M0 word0) ^ word3 ^ (k1 + W1) =: t, word 3
//            lo(M0 word0);
//   round 2: u1 = hi(M1 t) ^ (k0 + 2 W0), u2 = lo(M0 word0) ^ (k1 + 2 W1);
//   round 3: u3 = lo(M1 t) ^ (k0 + 3 W0).
struct PhiloxShared {
    uint32_t u0, u1, u2, u3;
};

__device__ __forceinline__ PhiloxShared philox4x32_shared(uint32_t b_lo, uint32_t b_hi, uint32_t w2, uint32_t k0,
                                                          uint32_t k1)
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * b_lo;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * w2;
    const uint32_t word0 = (uint32_t)(p1 >> 32) ^ b_hi ^ k0;
    const uint64_t q0 = (uint64_t)0xD2511F53u * word0;
    const uint32_t t = (uint32_t)(q0 >> 32) ^ (uint32_t)p0 ^ (k1 + 0xBB67AE85u);
    const uint64_t q1 = (uint64_t)0xCD9E8D57u * t;
    PhiloxShared u;
    u.u0 = (uint32_t)(p0 >> 32) ^ k1;
    u.u1 = (uint32_t)(q1 >> 32) ^ (k0 + 2u * 0x9E3779B9u);
    u.u2 = (uint32_t)q0 ^ (k1 + 2u * 0xBB67AE85u);
    u.u3 = (uint32_t)q1 ^ (k0 + 3u * 0x9E3779B9u);
    return u;
}

// Rounds 0 to 3 of the block from its shared part u and the lane's word w3;
// l1 = lo(M1 w2) ^ (k0 + W0), the same for every block of the wave.  The
// result equals philox4x32_rounds<0, 4> on the counter (b_lo, b_hi, w2, w3).
__device__ __forceinline__ void philox4x32_first4(const PhiloxShared& u, uint32_t l1, uint32_t w3, uint32_t k1,
                                                  uint32_t (&c)[4])
{
    // round 1 (round 0 leaves word 2 = u0 ^ w3; its other words are shared)
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (u.u0 ^ w3);
    const uint32_t x0 = (uint32_t)(p1 >> 32) ^ l1, x1 = (uint32_t)p1;
    // round 2
    const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    const uint32_t y0 = u.u1 ^ x1, y2 = (uint32_t)(p0 >> 32) ^ u.u2, y3 = (uint32_t)p0;
    // round 3
    const uint64_t r0 = (uint64_t)0xD2511F53u * y0;
    const uint64_t r1 = (uint64_t)0xCD9E8D57u * y2;
    c[0] = (uint32_t)(r1 >> 32) ^ u.u3;
    c[1] = (uint32_t)r1;
    c[2] = __builtin_amdgcn_bitop3_b32((uint32_t)(r0 >> 32), y3, k1 + 3u * 0xBB67AE85u, 0x96);
    c[3] = (uint32_t)r0;
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
