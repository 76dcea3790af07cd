// Parallel tempering for the approximate count (Sec. 3, Algorithm 2) on gfx950.
//
// One wavefront runs one ladder: lane j is inverse temperature beta_j (j < M
// <= 64).  Every lane owns one configuration slot in LDS -- the placements a_k
// of the n pairs (bytes) and the occupancy of every bin (bytes) -- and its
// energy E (empty bins).  An exchange of neighbouring levels swaps the slot
// indices of two lanes, which moves the whole configuration between levels.
//
// Per iteration (Algorithm 2's order):
//   1. the energy histogram of every level is incremented (LDS), the exact
//      form of Ratio(j) accumulation;
//   2. every level proposes one move: pair k uniform, placement uniform
//      (Sec. 3), accepted with min(1, exp(-beta_j dE));
//   3. neighbouring levels exchange configurations with min(1,
//      exp(-(beta_{j+1} - beta_j)(E_j - E_{j+1}))): even pairs on even
//      iterations, odd pairs on odd iterations.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the seed, one
// block of four words per (iteration, ladder, level): word 0 picks the pair,
// word 1 the placement, word 2 decides the move, word 3 (level j) decides the
// exchange of (j, j+1).  Accept/reject compares the word with a threshold
// floor(2^32 exp(-b e)) computed on the host, so the decisions are bit-exact
// reproducible.  Initial configurations use counters (0xFFFFFFF0 + block,
// 0xFFFFFFFF, ladder, level).
//
// Cost model: with 1024 ladders there is one wave on each SIMD, and one wave
// issues about one instruction per five cycles whatever the instruction; the
// loop is written for the fewest instructions per iteration: the two 32-bit
// products of a Philox round as single 64-bit multiplies, the exchange test
// and the upper/lower roles as wave-uniform lane masks on the scalar unit,
// lane shifts without copies, slots addressed by their LDS address, the slot
// address and the energy packed in one register, positions stored less one,
// Philox blocks split across the iteration boundary, the wave-uniform part of
// their first rounds drawn 64 blocks at a time, and the loop and pair-parity
// bookkeeping on the scalar unit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_philox.h"
#include "sk_pt.h"

namespace sk {

// Placement index -> left position of pair k, stored less one (positions
// 1..2n as 0..2n-1, so that a placement index is its own position), for the
// variant's position set (V: 0 Skolem, 1 Langford, 2 hooked; a compile-time
// constant, so the hooked case costs the other two nothing).  Hooked:
// positions 1..2n-1 and 2n+1; the first 2n-1-d placements end at or below
// 2n-1, the last one ends at 2n+1.
template <int V>
__device__ __forceinline__ int placement(int n, int d, int idx)
{
    if constexpr (V == 2) return idx >= 2 * n - 1 - d ? 2 * n - d : idx;
    return idx;
}

// The value held by lane + 1 / lane - 1 (wavefront shifts by one lane, DPP;
// every lane is active where these are used).  At the ends of the wavefront
// the lane reads 0 (bound control), which the callers never use and which
// keeps every index formed from it in range; a shift that writes every lane
// needs no copy of the old value.
__device__ __forceinline__ int from_lane_above(int x)
{
    return __builtin_amdgcn_mov_dpp(x, 0x130 /* wave_shl:1 */, 0xF, 0xF, true);
}
__device__ __forceinline__ int from_lane_below(int x)
{
    return __builtin_amdgcn_mov_dpp(x, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}

template <int V>
__device__ __forceinline__ int pair_diff(int k)
{
    return k + 1 + (V == 1);
}

template <int V>
__device__ __forceinline__ int placements_of(int n, int d)
{
    return 2 * n - d - (V == 2 && d == 1);
}

// A byte of LDS addressed by its 32-bit LDS address.
typedef __attribute__((address_space(3))) uint8_t lds_byte;

__device__ __forceinline__ lds_byte* lds_at(int addr)
{
    return (lds_byte*)(uintptr_t)(uint32_t)addr;
}

// Layout of the 64 configuration slots in LDS, chosen per variant by
// measurement: rows (a slot's bytes adjacent, slots slot_bytes apart) or
// columns (element i of every slot adjacent: byte base + 64 i of the slot).
// The LDS bank conflicts of the lanes' byte accesses depend on the layout and
// on the chains' positions: columns made the Langford chains 7 % faster, the
// Skolem chains 2.5 % and the hooked chains 4 % slower.
template <int V>
constexpr int kSlotShift = V == 1 ? 6 : 0;

// One byte array of a configuration slot: element i at byte base + (i << SHIFT).
template <int SHIFT>
struct SlotBytes {
    int base;
    __device__ __forceinline__ lds_byte& operator[](int i) const { return *lds_at(base + (i << SHIFT)); }
};

template <int V>
__global__ void __launch_bounds__(64) pt_ladder_kernel(const PtArgs a)
{
    extern __shared__ uint8_t lds[];
    const int lane = threadIdx.x;
    const uint32_t ladder = a.ladder_base + blockIdx.x;
    const int M = a.levels;
    const int n = a.n;
    const int top = a.top;
    const int H = top + 1;
    // n placements, then the occupancies of positions 1..top at bytes 0..top-1 (the host sizes
    // top + 1 of them), rounded to an odd number of 4-byte words
    const int slot_bytes = a.slot_bytes;
    uint32_t* hist = (uint32_t*)(lds + (size_t)64 * slot_bytes);  // M x H
    uint32_t* swap_thr = hist + M * H;                              // M x H, copy of a.swap_thr
    const bool live = lane < M;

    for (int i = lane; i < M * H; i += 64) {
        hist[i] = 0;
        swap_thr[i] = a.swap_thr[i];
    }

    // Every lane, also the ones above the top level, owns a configuration slot
    // and runs the moves on it, so that the iteration needs no lane-dependent
    // branch.  Those lanes never take part in an exchange (so their slots stay
    // their own), their histogram increments are 0 and go to row 0, and their
    // results are never written out.
    // LDS address of the lane's current slot (the address itself, not an
    // offset from the array, so that the slot moves between lanes as a plain
    // value and its bytes are addressed without an add per access)
    constexpr int SH = kSlotShift<V>;
    int sb = (int)(uint32_t)(uintptr_t)(lds_byte*)lds + (SH ? lane : lane * slot_bytes);
    int E = 0;
    // accepted moves; accepted exchanges counted at the upper level of the
    // pair (a lane mask the scalar unit forms), moved to the lower level
    // after the loop
    uint32_t mv_acc = 0, up_acc = 0;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const uint32_t T1 = live ? a.move_thr[lane * 2 + 0] : 0u;
    const uint32_t T2 = live ? a.move_thr[lane * 2 + 1] : 0u;
    const uint32_t hinc = live ? 1u : 0u;
    // (the two thresholds are in registers before the loop starts, so that
    // the loop holds no wait for their loads)
    asm volatile("" ::"v"(T1), "v"(T2));
    uint32_t* const hrow = hist + (live ? lane * H : 0);
    const uint32_t* const trow = swap_thr + (live ? lane * H : 0);
    // The lanes that are the lower level of an exchange pair, one lane mask
    // per parity of the iteration (wave-uniform, so the exchange's lane logic
    // runs on the scalar unit): lane j with j + 1 < M and j of that parity.
    uint64_t lower_mask[2] = {0, 0};
    for (int j = 0; j + 1 < M; ++j) lower_mask[j & 1] |= 1ull << j;
    {
        const SlotBytes<SH> s{sb}, occ{sb + (n << SH)};
        for (int p = 0; p <= top; ++p) occ[p] = 0;
        if (live && a.state_in) {
            const uint8_t* src = a.state_in + ((size_t)ladder * M + lane) * n;
            for (int k = 0; k < n; ++k) s[k] = (uint8_t)(src[k] - 1);
        } else {
            for (int blk = 0; blk * 4 < n; ++blk) {
                uint32_t r[4];
                philox4x32_10(0xFFFFFFF0u + (uint32_t)blk, 0xFFFFFFFFu, ladder, (uint32_t)lane, k0, k1, r);
                for (int t = 0; t < 4 && blk * 4 + t < n; ++t) {
                    const int k = blk * 4 + t;
                    const int d = pair_diff<V>(k);
                    const int idx = (int)__umulhi(r[t], (uint32_t)placements_of<V>(n, d));
                    s[k] = (uint8_t)placement<V>(n, d, idx);
                }
            }
        }
        for (int k = 0; k < n; ++k) {
            const int d = pair_diff<V>(k);
            occ[s[k]]++;
            occ[s[k] + d]++;
        }
        for (int p = 0; p < top; ++p)  // (position p + 1; the hooked set has no position 2n)
            if (!(V == 2 && p == 2 * n - 1) && occ[p] == 0) ++E;
    }
    __syncthreads();

    // Software pipeline.  Each Philox block is drawn in two halves of five
    // rounds that fill the waits for the two dependent LDS round trips of an
    // iteration (the four occupancies; the exchange threshold): iteration it
    // holds the words of it (r) and the block of it + 1 after its first half
    // (q), finishes q during the first round trip -- its word 0 picks the next
    // pair -- and draws the first half of the block of it + 2 during the
    // second.  The byte s[k] that the next move starts from is read in the
    // second round trip, for each of the three slots the lane can hold after
    // the exchange (its own, the one above, the one below), and picked once
    // the exchange is decided.  The scheduling barriers keep each half between
    // a read and the first use of its value.  (A block split across the
    // iteration boundary leaves two word copies per iteration where a block
    // drawn whole two iterations ahead left six.)
    uint32_t r[4], q[4] = {(uint32_t)(a.it_begin + 1), (uint32_t)((a.it_begin + 1) >> 32), ladder, (uint32_t)lane};
    philox4x32_10((uint32_t)a.it_begin, (uint32_t)(a.it_begin >> 32), ladder, (uint32_t)lane, k0, k1, r);
    philox4x32_rounds<0, 5>(q, k0, k1);
    int k = (int)__umulhi(r[0], (uint32_t)n);
    int a_old = *lds_at(sb + (k << SH));
    // (an opaque start value for a_old: without it the compiler treats the
    // loop's a_old as a byte, and the iteration takes one instruction more)
    asm("" : "+v"(a_old));
    // The loop runs over the counter of the block that the iteration draws
    // (it + 2), tested for equality, which the scalar unit does on 64 bits;
    // the lower lanes of the iteration's exchange pairs alternate by an XOR.
    const uint64_t it_end = a.it_end > a.it_begin ? a.it_end : a.it_begin;
    uint64_t lower = lower_mask[a.it_begin & 1];
    const uint64_t lower_flip = lower_mask[0] ^ lower_mask[1];
    // The slot address and the energy travel together through the exchange:
    // se = slot address << 16 | 4 E (the address is below 2^15, E at most
    // 2n + 1, never negative), so one lane shift and one select move both,
    // and 4 E is the byte offset of E's entry in the histogram and threshold
    // rows.
    static_assert(64 * (kPtMaxN + (2 * kPtMaxN + 2) + 3 + 4) < (1 << 15) && 4 * (2 * kPtMaxN + 1) < (1 << 16),
                  "the 64 slots (the kernel declares no other LDS before them) and 4 E must fit their halves");
    int se = (sb << 16) | (E << 2);
    const uint64_t ic_end = it_end + 2;
    // The Philox counter words 0..2 are the block number and the ladder,
    // shared by the wave: the parts of a block's first rounds that involve
    // only them are drawn for a group of 64 blocks at once, one per lane, and
    // each iteration reads its block's values from the lane that holds them
    // (three vector reads per iteration, one value being the same for the
    // whole group, where the scalar unit took about a dozen instructions).
    const uint32_t l1 = (uint32_t)((uint64_t)0xCD9E8D57u * ladder) ^ (k0 + 0x9E3779B9u);
    uint64_t ic = a.it_begin + 2;
    while (ic != ic_end) {
        const uint64_t gbase = ic & ~(uint64_t)63;  // this group of 64 block numbers
        const uint64_t gb = gbase + (uint64_t)lane;
        const PhiloxShared ug = philox4x32_shared((uint32_t)gb, (uint32_t)(gb >> 32), ladder, k0, k1);
        const uint64_t gend = ic_end - gbase < 64 ? ic_end : gbase + 64;
        do {
            const int li = (int)((uint32_t)ic & 63u);
            PhiloxShared u;
            u.u0 = (uint32_t)__builtin_amdgcn_readlane((int)ug.u0, li);
            u.u1 = (uint32_t)__builtin_amdgcn_readlane((int)ug.u1, li);
            u.u2 = (uint32_t)__builtin_amdgcn_readlane((int)ug.u2, li);
            u.u3 = (uint32_t)__builtin_amdgcn_readlane((int)ug.u3, li);
            // 1. move (pair k, whose current left position a_old was read ahead)
            const SlotBytes<SH> s{se >> 16}, occ{(se >> 16) + (n << SH)};
            const int d = pair_diff<V>(k);
            const int idx = (int)__umulhi(r[1], (uint32_t)placements_of<V>(n, d));
            const int a_new = placement<V>(n, d, idx);
            const int b_old = a_old + d, b_new = a_new + d;
            // the four occupancies in one round trip; the positions may coincide
            // (a_new == a_old, a_new == b_old, b_new == a_old), which the energy
            // change and the final counts account for in registers
            const int o1 = occ[a_old], o2 = occ[b_old], o3 = occ[a_new], o4 = occ[b_new];
            // 2. record the energy before the move (LDS atomic add, no read-back;
            // each level owns its row); issued behind the reads it does not feed
            atomicAdd((uint32_t*)((char*)hrow + (se & 0xffff)), hinc);  // hrow[E]
            __builtin_amdgcn_sched_barrier(0);
            philox4x32_rounds<5, 10>(q, k0, k1);  // the next block is complete
            __builtin_amdgcn_sched_barrier(0);
            const int c3 = o3 - (a_new == a_old) - (a_new == b_old);  // after removing pair k
            const int c4 = o4 - (b_new == a_old) - (b_new == b_old);
            const int de = (o1 == 1) + (o2 == 1) - (c3 == 0) - (c4 == 0);
            const bool acc = de <= 0 || r[2] < (de == 1 ? T1 : T2);
            // final counts of the (possibly repeated) four positions, written
            // whether or not the move is accepted (a rejected move writes back what
            // it read); a repeated position receives the same value from every write
            const int ac = acc ? 1 : 0;
            occ[a_old] = (uint8_t)(o1 + ac * ((a_old == a_new) + (a_old == b_new) - 1));
            occ[b_old] = (uint8_t)(o2 + ac * ((b_old == a_new) + (b_old == b_new) - 1));
            occ[a_new] = (uint8_t)(acc ? c3 + 1 : o3);
            occ[b_new] = (uint8_t)(acc ? c4 + 1 : o4);
            s[k] = (uint8_t)(acc ? a_new : a_old);
            se += (ac * de) << 2;
            mv_acc += ac;
            // 3. exchange (j, j+1) with j of the iteration's parity; the threshold
            // is read for every lane (index clamped at 0, where it is not needed),
            // and the next move's s[k] for the three candidate slots (after the
            // writes above, so they see this move)
            const int se_up = from_lane_above(se);
            const int se_dn = from_lane_below(se);
            const int dx4 = (se & 0xffff) - (se_up & 0xffff);  // 4 (E - E_up)
            const uint32_t thr = *(const uint32_t*)((const char*)trow + (dx4 > 0 ? dx4 : 0));
            const int k_next = (int)__umulhi(q[0], (uint32_t)n);
            const int v_own = *lds_at((se >> 16) + (k_next << SH));
            const int v_up = *lds_at((se_up >> 16) + (k_next << SH));
            const int v_dn = *lds_at((se_dn >> 16) + (k_next << SH));
            uint32_t c[4];
            __builtin_amdgcn_sched_barrier(0);
            philox4x32_first4(u, l1, (uint32_t)lane, k1, c);  // the block after next, first half
            philox4x32_rounds<4, 5>(c, k0, k1);
            __builtin_amdgcn_sched_barrier(0);
            // the exchange test as lane masks: the lower lanes of this parity whose
            // energy does not rise or whose word is under the threshold
            const uint64_t sw_mask =
                lower & (__builtin_amdgcn_ballot_w64(dx4 <= 0) | __builtin_amdgcn_ballot_w64(r[3] < thr));
            const bool sw = __builtin_amdgcn_inverse_ballot_w64(sw_mask);
            // the upper level of an accepted exchange: the lane above a lane with
            // sw set (the mask shifted by one lane)
            const uint64_t up_mask = sw_mask << 1;
            const bool upper = __builtin_amdgcn_inverse_ballot_w64(up_mask);
            se = sw ? se_up : (upper ? se_dn : se);
            a_old = sw ? v_up : (upper ? v_dn : v_own);
            {
                // up_acc += upper, the mask as the carry-in of one add
                uint64_t carry_out;
                asm("v_addc_co_u32_e64 %0, %1, 0, %0, %2" : "+v"(up_acc), "=s"(carry_out) : "s"(up_mask));
            }
            k = k_next;
            lower ^= lower_flip;
    #pragma unroll
            for (int i = 0; i < 4; ++i) {
                r[i] = q[i];
                q[i] = c[i];
            }
            // (the loop tests the incremented block counter itself, so that it is
            // neither recomputed from the iteration number nor copied)
            ++ic;
            asm("" : "+s"(ic));
        } while (ic != gend);
    }
    E = (se & 0xffff) >> 2;
    sb = (int)((uint32_t)se >> 16);
    const uint32_t sw_acc = (uint32_t)from_lane_above((int)up_acc);
    __syncthreads();

    // outputs: histograms, acceptance counts, states in level order
    for (int i = lane; i < M * H; i += 64) a.hist_out[(size_t)ladder * M * H + i] += hist[i];
    if (live) {
        a.move_acc[(size_t)ladder * M + lane] += mv_acc;
        a.swap_acc[(size_t)ladder * M + lane] += sw_acc;
        a.energy_out[(size_t)ladder * M + lane] = E;
        const SlotBytes<SH> s{sb};
        uint8_t* dst = a.state_out + ((size_t)ladder * M + lane) * n;
        for (int k = 0; k < n; ++k) dst[k] = (uint8_t)(s[k] + 1);
    }
}

hipError_t launch_pt_ladders(unsigned ladders, size_t lds_bytes, hipStream_t stream, const PtArgs& a)
{
    switch (a.variant) {
        case 0: hipLaunchKernelGGL(pt_ladder_kernel<0>, dim3(ladders), dim3(64), lds_bytes, stream, a); break;
        case 1: hipLaunchKernelGGL(pt_ladder_kernel<1>, dim3(ladders), dim3(64), lds_bytes, stream, a); break;
        case 2: hipLaunchKernelGGL(pt_ladder_kernel<2>, dim3(ladders), dim3(64), lds_bytes, stream, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sk
