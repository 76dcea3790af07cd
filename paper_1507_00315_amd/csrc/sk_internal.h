// Internal definitions shared by the host planner and the gfx950 kernels.
// Not part of the public ABI (include/skolem.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

constexpr int kMaxN = 32;       // pairs
constexpr int kMaxVars = 64;    // sign variables (= 2n)
constexpr int kMaxSlots = 32;   // factor slots (4 per quad)
constexpr int kMaxPrimes = 4;   // primes per pass
constexpr int kLaneBits = 6;    // 64 lanes of a wavefront = 6 sign variables

// Exact fp64 modular arithmetic needs primes in (2^45, 2^46): see exact_common.h.
constexpr double kPrimeLo = 35184372088832.0;  // 2^45
constexpr double kPrimeHi = 70368744177664.0;  // 2^46

// One slot of the product: the pair sum f_k of one difference d_k, or a
// dummy slot whose value is the constant 1.
//   value = (L - 2 * popcount((X ^ (X >> d)) & M)) >> halve
// X: position-space sign mask (bit pos-1 set <=> x_pos = -1)
// M: bit p-1 set for every p with p and p + d both in the position set
// L: |{p : p, p+d in P}|  (the value of f_k at x = +1...+1)
struct SlotDesc {
    uint64_t mask;
    int32_t d;
    int32_t len;
    int32_t halve;   // 1 if L is even: f_k is then even for every x, stored as f_k / 2
    int32_t pad;
};

// Arguments of one launch of the exact kernel.  Passed by value (kernarg).
struct ExactArgs {
    SlotDesc slot[kMaxSlots];
    int32_t var_pos[kMaxVars];   // position of each sign variable, ascending
    double prime[kMaxPrimes];
    double pinv[kMaxPrimes];     // fl(1/p)
    int32_t nprimes;
    int32_t m;          // sign variables (2n)
    int32_t n_lane;     // variables enumerated across the 64 lanes (<= 6)
    int32_t n_walk;     // variables walked in Gray-code order inside a job (ranks 1..n_walk)
    int32_t n_job;      // job variables (ranks n_walk+1 .. n_walk+n_job)
    int32_t job_bits_per_chunk;  // low job variables enumerated inside one chunk
    uint64_t chunk_base;         // chunk index of wave 0 (when chunk_ids == nullptr)
    const uint64_t* chunk_ids;   // device array, one chunk id per wave, or nullptr
    uint64_t n_waves;            // waves with work in this launch
    int32_t lane_valid_bits;     // lanes >= 2^lane_valid_bits contribute nothing
    int32_t qb[5];               // product group g covers quads [qb[g], qb[g+1])
    unsigned long long* acc;     // device: nprimes x (low word, carries) sums of the
                                 // waves' residues in [0, p); nullptr: one output row per wave
    int32_t larsen;              // 1: the inclusion-exclusion sum (0/1 variables, see exact_v2_body.h)
    int32_t pad1;
    uint64_t x_extra;            // bits ORed into every sign mask (position 1's value for larsen)
};

// Reversal weights (Lemma 2.3).  For Skolem and Langford pairings the term
// at x equals the term at the reversed vector, mapped back to x_1 = +1 by a
// global negation: x'_i = x_2n x_(2n+1-i).  For odd positions j1, j2 whose
// mirrors 2n+1-j1, 2n+1-j2 (even) are also job variables, the products
//     u = x_j1 x_j2,   v = x_(2n+1-j1) x_(2n+1-j2)
// swap under that map (the x_2n factors cancel) and are unchanged by the
// negation of the even positions (Lemma 2.4).  A job (wave-uniform setting of
// the job variables) gets weight 2 if, at the first quadruple with u != v,
// u = +1, weight 0 if u = -1 there (the partner job carries it), and weight 1
// if u = v for every quadruple.  Jobs of weight 0 are skipped.
constexpr int kRevMax = 4;
struct RevMasks {
    uint64_t u[kRevMax];  // bits j1-1, j2-1
    uint64_t v[kRevMax];  // bits of the mirrors
    int32_t r;            // quadruples in use (0: no reversal weighting)
    int32_t pad;
};

// Arguments of one launch of the specialised exact kernel (exact_v2_body.h);
// everything about the instance itself is compiled in.
//
// The launch is persistent: its waves pull work items from a queue (a device
// counter, zero before the launch) until the launch's items are exhausted.
// Item i is 2^item_job_bits consecutive jobs of chunk i >> (job_bits_per_chunk
// - item_job_bits) of the launch; the launch's chunk c is chunk_ids[c], or
// chunk_base + c.
struct ExactArgsV2 {
    RevMasks rev;
    double prime[kMaxPrimes];
    double pinv[kMaxPrimes];
    int32_t job_bits_per_chunk;  // low job variables enumerated inside one chunk
    int32_t item_job_bits;       // jobs per work item: 2^item_job_bits (<= 2^job_bits_per_chunk)
    uint64_t chunk_base;         // chunk index of the launch's chunk 0 (when chunk_ids == nullptr)
    const uint64_t* chunk_ids;   // device array, one chunk id per chunk of the launch, or nullptr
    uint64_t n_chunks;           // chunks of this launch
    uint32_t n_items;            // work items of this launch (n_chunks << (jb - item_job_bits))
    uint32_t pad0;
    uint32_t* counter;           // device: next work item (0 before the launch)
    unsigned long long* acc;     // total mode: as ExactArgs::acc
    unsigned long long* rows;    // row mode (acc == nullptr): n_chunks x P (low word, carries)
                                 // sums of each chunk's residues in [0, p), zero before the launch
    uint64_t x_extra;            // as ExactArgs::x_extra
};

// Device accumulators of one pass: at most this many primes (several launch
// batches of primes), each a (low word, carries) pair of uint64.
constexpr int kAccSlots = 16;

// Quad boundaries of the product groups: group gi covers quads
// [quad_begin(nq, g, gi), quad_begin(nq, g, gi + 1)).
__host__ __device__ constexpr int quad_begin(int nq, int g, int gi)
{
    return gi * (nq / g) + (gi < nq % g ? gi : nq % g);
}

}  // namespace sk
