// Exact sign-vector sum (Lemma 2.1), tuned kernel body for gfx950.
//
// Same decomposition as the reference body (exact_v1.hip): one wavefront per
// chunk, lanes enumerate the six highest sign variables, jobs enumerate the
// middle ones, and inside a job the lowest n_walk variables are visited in
// binary-reflected Gray-code order (Sec. 2.1: one sign flip per step, the pair
// sums updated by a linear number of additions).
//
// What is specialised here:
//   * Every pair sum is split as f_k = A_k + B_k.  A_k collects the pairs that
//     touch a lane variable; no walked variable is in such a pair (the plan
//     guarantees it), so A_k is fixed for the whole walk and lives per lane.
//     B_k collects the pairs of wave-uniform variables and lives in scalar
//     registers: the scalar unit updates it while the vector unit multiplies.
//   * Factors with an even pair count L_k are kept halved (f_k is even for
//     every sign vector then), shrinking the exact products.
//   * Two factors share a 32-bit register as packed 16-bit integers.  The
//     scalar copy of B is held with a bias of 2^14 per half and updated by
//     ordinary 32-bit adds of "integer-encoded" pairs (lo + 65536*hi), which
//     never carry between the halves.
//   * The lowest INNER walked variables (set Q) flip inside a fully unrolled
//     block of 2^(INNER+1) steps; their flip positions, the states of the other
//     Q variables and the step signs are compile-time constants.  For each
//     q in Q the scalar unit keeps N_q = the vector of (scaled) sums of q's
//     neighbours outside Q, so a flip of q is one scalar add per register pair
//     plus a compile-time constant for the pairs inside Q.
//   * The middle step of the block flips walked variable INNER (compile-time
//     position); the step between blocks flips a higher walked variable chosen
//     by a uniform branch over compile-time cases.
//   * Products: packed 16-bit multiply (two pair products per instruction),
//     one 24-bit multiply per quad reading both halves (SDWA), conversion to
//     fp64, exact fp64 group products, then the fp64 residue chain of
//     exact_common.h per prime.
//   * Where the plan needs three or more product groups (n >= 22), the walk
//     runs the cheaper two-group chain on the first group and the product of
//     the others, keeps per-lane maxima of the two values whose range makes
//     that chain exact, and evaluates a segment of 2^9 steps again with the
//     full chain when a lane of the wave went beyond it.
//   * Launches are persistent: waves pull work items (a few jobs of one
//     chunk) from a device counter until the launch's items run out.
//
// LARSEN = true evaluates the inclusion-exclusion sum of Sec. 2 (the third
// counting approach) with the same machinery: the variables are y in {0, 1}
// (1: position occupied, a set bit of the masks), the factors are
// N_k(y) = sum_i y_i y_(i+d_k) >= 0 (nothing halved), a flip of y_q changes
// N_k by +-(y_(q-d_k) + y_(q+d_k)), and the term's sign (-1)^(empty
// positions) is the parity of the set bits, as for the sign sum (2n is
// even).  Position 1 is not fixed: the host runs both of its values.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "exact_common.h"
#include "sk_internal.h"
#include "sk_plan.h"

namespace sk {

template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, E>(f);
    }
}

typedef short short2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(short2_t, a) + __builtin_bit_cast(short2_t, b));
}

__device__ __forceinline__ uint32_t pk_mul(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(short2_t, a) * __builtin_bit_cast(short2_t, b));
}

// product of the two sign-extended 16-bit halves of x
__device__ __forceinline__ int32_t mul_halves(uint32_t x)
{
    int32_t r;
    asm volatile("v_mul_i32_i24_sdwa %0, sext(%1), sext(%1) dst_sel:DWORD dst_unused:UNUSED_PAD "
                 "src0_sel:WORD_0 src1_sel:WORD_1"
                 : "=v"(r)
                 : "v"(x));
    return r;
}

constexpr uint32_t kHalfBias = 0x4000u;

template <int V, int N, int P, int INNER, bool LARSEN = false>
struct ExactV2 {
    static constexpr PlanCE PL = make_plan_ce(N, V, kWalkCap, LARSEN);
    static_assert(PL.ok, "no plan");
    static constexpr int NS = 4 * PL.nq;  // slots
    static constexpr int NP = NS / 2;     // packed slot pairs
    static constexpr int NQ = PL.nq;
    static constexpr int G = PL.G;
    static constexpr int W = PL.n_walk;
    static constexpr int M = PL.m;
    static_assert(PL.n_lane == 6, "tuned body needs six lane variables");
    static_assert(W >= INNER + 1, "walk too short for the unrolled block");
    static constexpr int D = 1 << (INNER + 1);  // steps per unrolled block

    // ranks below the lane ranks sit at position rank + 1 (the hooked gap is
    // at the top, among the lane ranks)
    static constexpr bool contiguous_low()
    {
        for (int r = 0; r < M - 6; ++r)
            if (PL.pos[r] != r + 1) return false;
        return true;
    }
    static_assert(contiguous_low(), "unexpected position layout");

    static constexpr bool in_set(int p) { return p >= 1 && p <= 64 && ((PL.pset >> (p - 1)) & 1); }
    static constexpr int qpos(int b) { return 2 + b; }  // position of inner walked variable b
    static constexpr bool is_inner(int p) { return p >= 2 && p < 2 + INNER; }
    // change of a pair term per unit neighbour value when one end flips:
    // x_q x_r moves by 2 x_r (1 for a halved factor); y_q y_r by y_r
    static constexpr int g_of(int s) { return PL.slot_k[s] < 0 ? 0 : (LARSEN || PL.slot_halve[s] ? 1 : 2); }
    static constexpr uint64_t lane_posmask()
    {
        uint64_t m = 0;
        for (int b = 0; b < 6; ++b) m |= 1ull << (PL.pos[M - 6 + b] - 1);
        return m;
    }
    // edges of slot s touching a lane variable / between uniform variables
    static constexpr uint64_t mask_lane(int s)
    {
        const uint64_t lp = lane_posmask();
        return PL.slot_k[s] < 0 ? 0 : (PL.slot_mask[s] & (lp | (lp >> PL.slot_d[s])));
    }
    static constexpr uint64_t mask_unif(int s) { return PL.slot_k[s] < 0 ? 0 : (PL.slot_mask[s] & ~mask_lane(s)); }
    static constexpr int popc_ce(uint64_t x)
    {
        int c = 0;
        while (x) {
            c += (int)(x & 1);
            x >>= 1;
        }
        return c;
    }
    // inner state (bit b set <=> x = -1) at local step i of a block
    static constexpr int state(int i) { return (i ^ (i >> 1)) & ((1 << INNER) - 1); }
    // value of inner variable b in state st: x = -1 (bit set) or +1; y = bit
    static constexpr int xval_state(int st, int b) { return LARSEN ? ((st >> b) & 1) : (((st >> b) & 1) ? -1 : 1); }
    // whether the flip of inner variable b from state st raises the factors:
    // x from -1 to +1, y from 0 to 1
    static constexpr bool flip_raises(int st, int b) { return LARSEN ? !((st >> b) & 1) : ((st >> b) & 1); }
    static constexpr int ctz_ce(int i)
    {
        int c = 0;
        while (!(i & 1)) {
            i >>= 1;
            ++c;
        }
        return c;
    }
    // integer-encoded constant for pair p at inner flip of step i:
    // sum over slots of g_s * (sum of x of Q-neighbours of the flipped q at distance d_s)
    static constexpr int inner_const_slot(int i, int s)
    {
        const int b = ctz_ce(i);
        const int st = state(i - 1);
        if (PL.slot_k[s] < 0) return 0;
        int sum = 0;
        for (int b2 = 0; b2 < INNER; ++b2) {
            if (b2 == b) continue;
            const int dist = qpos(b) > qpos(b2) ? qpos(b) - qpos(b2) : qpos(b2) - qpos(b);
            if (dist == PL.slot_d[s]) sum += xval_state(st, b2);
        }
        return g_of(s) * sum;
    }
    static constexpr int32_t inner_const_pair(int i, int p)
    {
        return (int32_t)inner_const_slot(i, 2 * p) + 65536 * (int32_t)inner_const_slot(i, 2 * p + 1);
    }
    // slot whose difference equals dist (-1 if none)
    static constexpr int slot_of_diff(int dist)
    {
        for (int s = 0; s < NS; ++s)
            if (PL.slot_k[s] >= 0 && PL.slot_d[s] == dist) return s;
        return -1;
    }

    // value of the variable at position p: x = +1 / -1 (bit clear / set), or y = bit
    __device__ static __forceinline__ int xbit(uint64_t XU, int p)
    {
        if constexpr (LARSEN) return (int)((XU >> (p - 1)) & 1);
        else return 1 - 2 * (int)((XU >> (p - 1)) & 1);
    }
    // pair terms of slot s on the edges `mask` of sign mask X: the sum of
    // x_i x_(i+d) (L - 2 * disagreeing pairs) or of y_i y_(i+d)
    __device__ static __forceinline__ int pair_sum(uint64_t X, uint64_t mask, int d)
    {
        if constexpr (LARSEN) return (int)__builtin_popcountll(X & (X >> d) & mask);
        else return popc_ce(mask) - 2 * (int)__builtin_popcountll((X ^ (X >> d)) & mask);
    }

    // Scalar state for a job: B (biased, integer-encoded pairs) and N_q.
    struct Uniform {
        uint64_t XU;
        uint32_t B[NP];
        int32_t Nq[INNER][NP];
    };

    __device__ static __forceinline__ void init_uniform(Uniform& u)
    {
        static_for<0, NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            int32_t bh[2];
            static_for<0, 2>([&](auto hc) {
                constexpr int s = 2 * p + decltype(hc)::value;
                if constexpr (PL.slot_k[s] < 0) {
                    bh[decltype(hc)::value] = 0;
                } else {
                    constexpr uint64_t mu = mask_unif(s);
                    constexpr int d = PL.slot_d[s];
                    const int B = pair_sum(u.XU, mu, d);
                    if constexpr (PL.slot_halve[s]) {
                        constexpr int c = popc_ce(mu) & 1;
                        bh[decltype(hc)::value] = (B - c) >> 1;
                    } else {
                        bh[decltype(hc)::value] = B;
                    }
                }
            });
            u.B[p] = (uint32_t)(bh[0] + (int32_t)kHalfBias) + 65536u * (uint32_t)(bh[1] + (int32_t)kHalfBias);
        });
        static_for<0, INNER>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            constexpr int q = qpos(b);
            static_for<0, NP>([&](auto pc) {
                constexpr int p = decltype(pc)::value;
                int32_t nh[2];
                static_for<0, 2>([&](auto hc) {
                    constexpr int s = 2 * p + decltype(hc)::value;
                    int sum = 0;
                    if constexpr (PL.slot_k[s] >= 0) {
                        constexpr int d = PL.slot_d[s];
                        if constexpr (in_set(q - d) && !is_inner(q - d)) sum += xbit(u.XU, q - d);
                        if constexpr (in_set(q + d) && !is_inner(q + d)) sum += xbit(u.XU, q + d);
                    }
                    nh[decltype(hc)::value] = g_of(s) * sum;
                });
                u.Nq[b][p] = nh[0] + 65536 * nh[1];
            });
        });
    }

    // Flip of the uniform walked variable at position R (not in Q).
    template <int R>
    __device__ static __forceinline__ void flip_outer(Uniform& u)
    {
        // per unit neighbour value, the factors move by -x_r g (sign sum) or by
        // +1 / -1 as y_r goes 0 -> 1 / 1 -> 0 (inclusion-exclusion); the sign
        // sum keeps its own expressions (the same values; the compiler
        // allocates registers better for them)
        const int xr = xbit(u.XU, R);  // value before the flip
        static_for<0, NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            int32_t dh[2];
            static_for<0, 2>([&](auto hc) {
                constexpr int s = 2 * p + decltype(hc)::value;
                int sum = 0;
                if constexpr (PL.slot_k[s] >= 0) {
                    constexpr int d = PL.slot_d[s];
                    if constexpr (in_set(R - d)) sum += xbit(u.XU, R - d);
                    if constexpr (in_set(R + d)) sum += xbit(u.XU, R + d);
                }
                if constexpr (LARSEN) dh[decltype(hc)::value] = (1 - 2 * xr) * sum;
                else dh[decltype(hc)::value] = -xr * g_of(s) * sum;
            });
            u.B[p] += (uint32_t)(dh[0] + 65536 * dh[1]);
        });
        static_for<0, INNER>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            constexpr int s = slot_of_diff(R - qpos(b));
            if constexpr (s >= 0) {
                constexpr int32_t unit = (s & 1) ? 65536 : 1;
                if constexpr (LARSEN) u.Nq[b][s / 2] += (1 - 2 * xr) * unit;
                else u.Nq[b][s / 2] += -2 * xr * g_of(s) * unit;
            }
        });
        u.XU ^= 1ull << (R - 1);
    }

    // Flip of inner variable b = ctz(i) at local step i (compile time).
    template <int I>
    __device__ static __forceinline__ void flip_inner(Uniform& u)
    {
        constexpr int b = ctz_ce(I);
        constexpr bool up = flip_raises(state(I - 1), b);
        static_for<0, NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int32_t c = inner_const_pair(I, p);
            if constexpr (up) {
                u.B[p] += (uint32_t)u.Nq[b][p];
                if constexpr (c != 0) u.B[p] += (uint32_t)c;
            } else {
                u.B[p] -= (uint32_t)u.Nq[b][p];
                if constexpr (c != 0) u.B[p] -= (uint32_t)c;
            }
        });
        u.XU ^= 1ull << (qpos(b) - 1);
    }

    template <int LO>
    __device__ static __forceinline__ void flip_walk_bit(Uniform& u, int bit)
    {
        if constexpr (LO < W) {
            if (bit == LO) flip_outer<2 + LO>(u);
            else flip_walk_bit<LO + 1>(u, bit);
        }
    }

    // Term at the current state: acc += sign * prod_k f'_k (mod p_i).  With
    // two product groups the exact low part l of g0 g1 does not depend on the
    // prime; it is summed once in accl and added to every prime's sum when the
    // block is reduced.
    // FAST (G >= 3): the two-group chain of G = 2 on g0 = group 0 (below
    // 2^53 by the plan's bound) and g1 = the product of every other group.  It
    // is exact only while |g1| < 2^53 and |g0 g1| < 2^96, which the plan does
    // not guarantee; the running maxima of both go to mx, and the caller
    // evaluates the segment again without FAST if they were reached.
    template <bool NEG, bool FAST = false>
    __device__ static __forceinline__ void term(const uint32_t (&A)[NP], const Uniform& u, const double (&pr)[P],
                                                const double (&pinv)[P], double (&acc)[P], double& accl,
                                                double (&mx)[2])
    {
        uint32_t f[NP];
        static_for<0, NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            f[p] = pk_add(A[p], u.B[p]);
        });
        double q[NQ];
        static_for<0, NQ>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            q[i] = (double)mul_halves(pk_mul(f[2 * i], f[2 * i + 1]));
        });
        if constexpr (FAST) {
            static_assert(G >= 3, "the fast chain merges groups 1 .. G-1");
            constexpr int q1 = PL.qb[1];
            double g0 = q[0];
            static_for<1, q1>([&](auto jc) { g0 *= q[decltype(jc)::value]; });
            double g1 = q[q1];
            static_for<q1 + 1, NQ>([&](auto jc) { g1 *= q[decltype(jc)::value]; });
            const double h = g0 * g1;
            const double l = __builtin_fma(g0, g1, -h);
            mx[0] = __builtin_fmax(mx[0], __builtin_fabs(g1));
            mx[1] = __builtin_fmax(mx[1], __builtin_fabs(h));
            static_for<0, P>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const double s = __builtin_fma(quot_nearest(h, pinv[i]), -pr[i], h);
                acc[i] = NEG ? acc[i] - s : acc[i] + s;
            });
            accl = NEG ? accl - l : accl + l;
            return;
        }
        double g[G];
        static_for<0, G>([&](auto gc) {
            constexpr int gi = decltype(gc)::value;
            constexpr int q0 = PL.qb[gi], q1 = PL.qb[gi + 1];
            double v = q[q0];
            static_for<q0 + 1, q1>([&](auto jc) { v *= q[decltype(jc)::value]; });
            g[gi] = v;
        });
        if constexpr (G == 1) {
            static_for<0, P>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const double r = reduce_balanced(g[0], pr[i], pinv[i]);
                acc[i] = NEG ? acc[i] - r : acc[i] + r;
            });
        } else {
            const double h = g[0] * g[1];
            const double l = __builtin_fma(g[0], g[1], -h);
            static_for<0, P>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const double s = __builtin_fma(quot_nearest(h, pinv[i]), -pr[i], h);
                if constexpr (G == 2) {
                    acc[i] = NEG ? acc[i] - s : acc[i] + s;
                } else {
                    double r = s + l;
                    static_for<2, G>([&](auto gc) {
                        constexpr int gi = decltype(gc)::value;
                        const double h2 = r * g[gi];
                        const double l2 = __builtin_fma(r, g[gi], -h2);
                        const double s2 = __builtin_fma(quot_nearest(h2, pinv[i]), -pr[i], h2);
                        if constexpr (gi == G - 1) {
                            acc[i] = NEG ? acc[i] - s2 : acc[i] + s2;
                            acc[i] = NEG ? acc[i] - l2 : acc[i] + l2;
                        } else {
                            r = s2 + l2;
                        }
                    });
                }
            });
            if constexpr (G == 2) accl = NEG ? accl - l : accl + l;
        }
    }
};

// A 64-bit value read from the first active lane.  The builtin works on int:
// each half goes back through uint32_t before widening, so that a low word
// with bit 31 set is not sign-extended into the high word.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x)
{
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

// A wave-uniform 64-bit value copied into a vector register pair (it keeps no
// scalar registers while it waits).
__device__ __forceinline__ uint64_t vgpr_copy(uint64_t x)
{
    uint64_t r;
    asm("v_mov_b64 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// Blocks per segment of the two-group chain (G >= 3): 2^4 blocks of 32 steps,
// 2^15 sign vectors over the wave (64 blocks: the L(28) slice 3.5 % slower,
// n = 24 the same).
constexpr uint64_t kFastSegBlocks = 16;

// Jobs [j_begin, j_end) of one chunk (chunk id, 2^jb jobs) evaluated by the
// calling wavefront and added to acc_tot (per lane, balanced residues: the
// wave's sum is the sum over the lanes).  x_extra: bits ORed into every job's
// mask (position 1's value for LARSEN).
template <int V, int N, int P, int INNER, bool LARSEN = false>
__device__ __forceinline__ void exact_v2_jobs(uint64_t chunk, int jb, uint64_t j_begin, uint64_t j_end,
                                              const RevMasks& rev, const double (&pr)[P], const double (&pinv)[P],
                                              double (&acc_tot)[P], uint64_t x_extra = 0)
{
    using K = ExactV2<V, N, P, INNER, LARSEN>;
    constexpr PlanCE PL = K::PL;
    constexpr int NP = K::NP;
    constexpr int W = K::W;
    constexpr int M = K::M;
    constexpr int D = K::D;

    const int lane = threadIdx.x & 63;
    // lane variables
    uint64_t XL = 0;
    static_for<0, 6>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        constexpr int p = PL.pos[M - 6 + b];
        XL |= (uint64_t)((lane >> b) & 1) << (p - 1);
    });
    const int lane_parity = __builtin_popcount(lane) & 1;

    const uint64_t xu_chunk = (chunk << (1 + W + jb)) | x_extra;
    for (uint64_t j = j_begin; j < j_end; ++j) {
        const uint64_t xu_job = xu_chunk | (j << (1 + W));
        // reversal weight of this job (wave-uniform: job variables only)
        int w = 1;
        for (int q = 0; q < rev.r; ++q) {
            const int pu = __builtin_popcountll(xu_job & rev.u[q]) & 1;  // 0: u = +1
            const int pv = __builtin_popcountll(xu_job & rev.v[q]) & 1;
            if (pu != pv) {
                w = pu == 0 ? 2 : 0;
                break;
            }
        }
        if (w == 0) continue;
        typename K::Uniform u;
        u.XU = xu_job;
        K::init_uniform(u);
        // per-lane part A of every slot (pairs touching a lane variable)
        uint32_t A[NP];
        const uint64_t X = u.XU | XL;
        static_for<0, NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            int32_t ah[2];
            static_for<0, 2>([&](auto hc) {
                constexpr int s = 2 * p + decltype(hc)::value;
                if constexpr (PL.slot_k[s] < 0) {
                    ah[decltype(hc)::value] = 1;
                } else {
                    constexpr uint64_t ml = K::mask_lane(s);
                    constexpr int d = PL.slot_d[s];
                    const int Av = K::pair_sum(X, ml, d);
                    if constexpr (PL.slot_halve[s]) {
                        constexpr int c = K::popc_ce(K::mask_unif(s)) & 1;
                        ah[decltype(hc)::value] = (Av + c) >> 1;
                    } else {
                        ah[decltype(hc)::value] = Av;
                    }
                }
            });
            A[p] = ((uint32_t)(ah[0] - (int32_t)kHalfBias) & 0xFFFFu) |
                   ((uint32_t)(ah[1] - (int32_t)kHalfBias) << 16);
        });
        const int neg0 = (__builtin_popcountll(u.XU) + lane_parity) & 1;

        double acc[P];
        double mx[2] = {0.0, 0.0};
        // Blocks [b0, b1) of the walk of the job: D steps each, the step between
        // blocks flipping the walked variable of the block index's lowest set bit.
        auto walk = [&](auto fast, uint64_t b0, uint64_t b1) {
            constexpr bool FAST = decltype(fast)::value;
            for (uint64_t ds = b0; ds < b1; ++ds) {
                if (ds > 0) K::template flip_walk_bit<INNER + 1>(u, INNER + 1 + (int)__builtin_ctzll(ds));
                // |accl| <= D * 2^43 (low parts of products below 2^96)
                double accl = 0.0;
                static_for<0, D>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    if constexpr (i > 0) {
                        if constexpr (K::ctz_ce(i) < INNER) K::template flip_inner<i>(u);
                        else K::template flip_outer<2 + INNER>(u);
                    }
                    K::template term<(i & 1) != 0, FAST>(A, u, pr, pinv, acc, accl, mx);
                });
                static_for<0, P>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    acc[i] = reduce_balanced(acc[i] + accl, pr[i], pinv[i]);
                });
            }
        };
        // the job's weight (Lemma 2.3) and sign, applied to each part of its sum
        auto add_to_total = [&]() {
            static_for<0, P>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const double aw = w == 2 ? acc[i] + acc[i] : acc[i];  // |aw| <= 1.5 p
                acc_tot[i] = reduce_balanced(neg0 ? acc_tot[i] - aw : acc_tot[i] + aw, pr[i], pinv[i]);
            });
        };
        constexpr uint64_t nblocks = 1ull << (W - (INNER + 1));
        if constexpr (K::G >= 3) {
            // Segments of kFastSegBlocks blocks with the two-group chain.  A
            // segment in which some term left that chain's exact range (rare:
            // the largest products come from nearly periodic sign vectors) is
            // evaluated again with the full chain, from its first sign vector:
            // the scalar state is a function of the sign mask alone, so the
            // mask at the segment's start (kept in the wave's LDS slot, which
            // costs no register) restores it.  Each segment's sum goes to the
            // total once it is final.
            constexpr uint64_t seg = nblocks < kFastSegBlocks ? nblocks : kFastSegBlocks;
            __shared__ uint64_t seg_mask[4];  // one slot per wave of the workgroup
            const int wslot = (int)(threadIdx.x >> 6) & 3;
            for (uint64_t s0 = 0; s0 < nblocks; s0 += seg) {
                if (lane == 0) seg_mask[wslot] = u.XU;
#pragma unroll
                for (int i = 0; i < P; ++i) acc[i] = 0.0;
                mx[0] = 0.0;
                mx[1] = 0.0;
                walk(std::true_type{}, s0, s0 + seg);
                const bool out_of_range = mx[0] >= 0x1p53 || mx[1] >= 0x1p96;
                if (__builtin_amdgcn_ballot_w64(out_of_range) != 0) {
                    u.XU = uniform_u64(seg_mask[wslot]);
                    K::init_uniform(u);
#pragma unroll
                    for (int i = 0; i < P; ++i) acc[i] = 0.0;
                    walk(std::false_type{}, s0, s0 + seg);
                }
                add_to_total();
            }
        } else {
#pragma unroll
            for (int i = 0; i < P; ++i) acc[i] = 0.0;
            walk(std::false_type{}, 0, nblocks);
            add_to_total();
        }
    }
}

// One whole chunk; returns in every lane the wave's residues (balanced, exact
// fp64 integers).
template <int V, int N, int P, int INNER, bool LARSEN = false>
__device__ __forceinline__ void exact_v2_chunk(uint64_t chunk, int jb, const RevMasks& rev, const double (&pr)[P],
                                               const double (&pinv)[P], double (&res)[P], uint64_t x_extra = 0)
{
    double acc[P];
#pragma unroll
    for (int i = 0; i < P; ++i) acc[i] = 0.0;
    exact_v2_jobs<V, N, P, INNER, LARSEN>(chunk, jb, 0, 1ull << jb, rev, pr, pinv, acc, x_extra);
#pragma unroll
    for (int i = 0; i < P; ++i) res[i] = wave_sum_f64(acc[i]);
}

// A wave-uniform fp64 value copied into a vector register pair, so that it
// takes no scalar registers: the scalar unit's pair-sum state (B and the N_q)
// of the large instances needs all of them, and the primes and their inverses
// are read only as fp64 operands.
__device__ __forceinline__ double in_vgpr(double x)
{
    double r;
    asm("v_mov_b64 %0, %1" : "=v"(r) : "s"(x));
    return r;
}


// Persistent launch: every wave pulls work items (2^item_job_bits jobs of one
// chunk) from the launch's queue until it is empty.  Total mode (acc): each
// wave keeps one running residue per prime over all its items, and the
// workgroup adds the sums to the device accumulators at the end.  Row mode
// (rows): each item's residues are added to its chunk's row.  Small items keep
// every SIMD busy until the queue drains, whatever the number of waves that
// fit on it.
template <int V, int N, int P, int INNER, bool LARSEN = false>
__global__ void __launch_bounds__(256) exact_v2_kernel(const ExactArgsV2 a)
{
    const int lane = threadIdx.x & 63;
    double pr[P], pinv[P], tot[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        pr[i] = in_vgpr(a.prime[i]);
        pinv[i] = in_vgpr(a.pinv[i]);
        tot[i] = 0.0;
    }
    const int jb = a.job_bits_per_chunk;
    const int ib = a.item_job_bits;
    const int sub = jb - ib;  // items per chunk: 2^sub
    bool any = false;
    // A wave can claim at most n_items items; the trip bound guarantees that
    // every wave leaves the loop whatever the counter returns.
    for (uint32_t trip = 0; trip <= a.n_items; ++trip) {
        // Every lane takes part in the atomic (lane 0 adds 1, the others 0) and
        // the claimed index is read from lane 0: no lane-dependent branch
        // precedes the broadcast.
        const uint32_t old = atomicAdd(a.counter, lane == 0 ? 1u : 0u);
        const uint32_t idx = __builtin_amdgcn_readlane(old, 0);
        if (idx >= a.n_items) break;  // every wave leaves once the queue is empty
        const uint64_t c = (uint64_t)idx >> sub;
        const uint64_t j0 = ((uint64_t)idx & ((1ull << sub) - 1)) << ib;
        const uint64_t chunk = uniform_u64(a.chunk_ids ? a.chunk_ids[c] : a.chunk_base + c);
        double part[P];
#pragma unroll
        for (int i = 0; i < P; ++i) part[i] = 0.0;
        exact_v2_jobs<V, N, P, INNER, LARSEN>(chunk, jb, j0, j0 + (1ull << ib), a.rev, pr, pinv, part, a.x_extra);
        if (a.rows) {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const double r = wave_sum_f64(part[i]);
                if (lane == 0) add_u128(a.rows + 2 * (c * P + i), canonical_residue(r, pr[i], pinv[i]));
            }
        } else {
#pragma unroll
            for (int i = 0; i < P; ++i) tot[i] = reduce_balanced(tot[i] + part[i], pr[i], pinv[i]);
            any = true;
        }
    }
    if (a.acc) {
        // sums of whole launches: wave butterfly, workgroup stage, then the
        // device accumulators
        double res[P];
#pragma unroll
        for (int i = 0; i < P; ++i) res[i] = wave_sum_f64(tot[i]);
        workgroup_accumulate<P>(res, P, pr, pinv, any, a.acc);
    }
}

}  // namespace sk

