// Exact modular product-and-accumulate in fp64 for gfx950 (device side).
//
// The sum of Lemma 2.1 is taken modulo primes p with 2^45 < p < 2^46
// (Sec. 2.2: "modulo a number of co-primes", recombined by CRT on the host).
// CDNA4 runs fp64 FMA at the full vector rate, so residues live in fp64
// registers as exact integers (|value| < 2^53) and every reduction is
//     q = nearest integer to h / p    (fma(h, 1/p, 1.5*2^52) - 1.5*2^52)
//     s = h - q p                     (one fma; exact, |s| <= 0.75 p)
// with the low half of a wide product recovered exactly by l = fma(a, b, -a*b).
//
// Factors of one term are grouped: groups are exact fp64 products of up to
// 16 factors (|g| < 2^53).  Bounds checked on the host for every instance:
//   |g0 * g1| < 2^96  (so |q| < 2^51 for p > 2^45),  |g_i| < 2^50 for i >= 2.
// Residues stay in [-p, p]; accumulators absorb 64 terms (64 * 2^46 + p < 2^53)
// before they are reduced again.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_internal.h"

namespace sk {

constexpr double kRoundMagic = 6755399441055744.0;  // 1.5 * 2^52

// Nearest integer to h * pinv for |h * pinv| < 2^51, as an exact fp64 integer.
__device__ __forceinline__ double quot_nearest(double h, double pinv)
{
    return __builtin_fma(h, pinv, kRoundMagic) - kRoundMagic;
}

// x mod p, balanced: |result| <= 0.75 p (x an exact integer, |x| < 2^51 p).
__device__ __forceinline__ double reduce_balanced(double x, double p, double pinv)
{
    return __builtin_fma(quot_nearest(x, pinv), -p, x);
}

// Exact group products of the 4*NQ slot values (each |f| <= 64); group gi
// multiplies quads [qb[gi], qb[gi+1]).
template <int NQ, int G>
__device__ __forceinline__ void group_products(const int32_t* f, const int32_t* qb, double* g)
{
    double q[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int32_t a = f[4 * i] * f[4 * i + 1];
        const int32_t b = f[4 * i + 2] * f[4 * i + 3];
        q[i] = (double)(a * b);
    }
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
        double v = 1.0;
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (i >= qb[gi] && i < qb[gi + 1]) v *= q[i];
        g[gi] = v;
    }
}

// acc[i] += (neg ? -1 : +1) * (g0 g1 ... g_{G-1} mod p_i), exactly, for i < P.
template <int G>
__device__ __forceinline__ void accumulate_term(const double* g, const double* prime,
                                                const double* pinv, int P, bool neg, double* acc)
{
    if constexpr (G == 1) {
#pragma unroll
        for (int i = 0; i < kMaxPrimes; ++i) {
            if (i < P) {
                const double r = reduce_balanced(g[0], prime[i], pinv[i]);
                acc[i] += neg ? -r : r;
            }
        }
    } else {
        const double h = g[0] * g[1];
        const double l = __builtin_fma(g[0], g[1], -h);
#pragma unroll
        for (int i = 0; i < kMaxPrimes; ++i) {
            if (i < P) {
                const double s = __builtin_fma(quot_nearest(h, pinv[i]), -prime[i], h);
                if constexpr (G == 2) {
                    acc[i] += neg ? -s : s;
                    acc[i] += neg ? -l : l;
                } else {
                    double r = s + l;
#pragma unroll
                    for (int gi = 2; gi < G; ++gi) {
                        const double h2 = r * g[gi];
                        const double l2 = __builtin_fma(r, g[gi], -h2);
                        const double s2 = __builtin_fma(quot_nearest(h2, pinv[i]), -prime[i], h2);
                        if (gi == G - 1) {
                            acc[i] += neg ? -s2 : s2;
                            acc[i] += neg ? -l2 : l2;
                        } else {
                            r = s2 + l2;
                        }
                    }
                }
            }
        }
    }
}

// Sum over the 64 lanes of a wavefront (exact while the total is < 2^53).
__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------- reduction
//
// Residues leave a wavefront as exact fp64 integers.  The device sums them per
// prime as unsigned integers in [0, p) into 128-bit accumulators (a low word
// and a carry count, both updated by 64-bit atomics): the sum is exact and
// does not depend on the order of the additions, so it is the same on every
// run, and the host reduces it modulo p once.  With p < 2^46 and fewer than
// 2^32 additions the total stays below 2^78.

// x mod p in [0, p) for an exact fp64 integer x with |x| < 2^51 p.
__device__ __forceinline__ uint64_t canonical_residue(double x, double p, double pinv)
{
    double y = reduce_balanced(x, p, pinv);  // |y| <= 0.75 p
    if (y < 0.0) y += p;
    return (uint64_t)y;
}

// acc[0] += v with the carry out of the low word counted in acc[1].  Works on
// global memory and on LDS (the atomics then stay in the workgroup).
__device__ __forceinline__ void add_u128(unsigned long long* acc, uint64_t v)
{
    const unsigned long long old = atomicAdd(acc, (unsigned long long)v);
    if (old + v < old) atomicAdd(acc + 1, 1ull);
}

// Adds a 128-bit (low, carries) pair into a device accumulator.
__device__ __forceinline__ void add_u128_pair(unsigned long long* acc, unsigned long long lo,
                                              unsigned long long hi)
{
    const unsigned long long old = atomicAdd(acc, lo);
    const unsigned long long carry = (old + lo < old) ? 1ull : 0ull;
    if (hi + carry) atomicAdd(acc + 1, hi + carry);
}

// Workgroup stage of the single-count launches (256 threads = 4 wavefronts,
// every thread of the workgroup must call it): the residues of the
// block's waves (res, the same in every lane of a wave; a wave with active ==
// false contributes 0) meet in LDS, and one thread per prime adds their sum
// (below 2^48) to acc[2 i], acc[2 i + 1].
template <int PMAX>
__device__ __forceinline__ void workgroup_accumulate(const double (&res)[PMAX], int P, const double* prime,
                                                     const double* pinv, bool active,
                                                     unsigned long long* __restrict__ acc)
{
    __shared__ uint64_t part[4][PMAX];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < PMAX; ++i)
            if (i < P) part[w][i] = active ? canonical_residue(res[i], prime[i], pinv[i]) : 0;
    }
    __syncthreads();
    if ((int)threadIdx.x < P) {
        uint64_t s = 0;
#pragma unroll
        for (int i = 0; i < PMAX; ++i)
            if (i == (int)threadIdx.x) s = part[0][i] + part[1][i] + part[2][i] + part[3][i];
        if (s) add_u128(acc + 2 * threadIdx.x, s);
    }
}

}  // namespace sk
