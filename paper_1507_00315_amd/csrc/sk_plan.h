// Instance plan for the exact sum, computable at compile time (the tuned
// kernel is specialised per (variant, n)) and at run time (the host).
//
// For a variant and n it fixes:
//   * the position set P and the differences d_k (Sec. 1.1, Sec. 1.2),
//   * the split of the 2n sign variables (ordered by position) into
//       rank 0            x at position 1, fixed to +1 (Lemma 2.2),
//       walk ranks        1 .. n_walk, visited in Gray-code order,
//       job ranks         the ones between (chunk bits on top),
//       lane ranks        the 6 highest, one combination per lane,
//     with n_walk as large as possible such that no walked variable forms a
//     pair (i, i + d_k) with a lane variable,
//   * the factor slots: factor k sits in one of 4*nq slots; slots form quads
//     and quads form G groups whose exact products stay below 2^53 (and the
//     host-checked bounds of the modular chain hold),
//   * which factors are stored halved (f_k is even for every x when the
//     number of pairs L_k at distance d_k is even).
//
// The inclusion-exclusion sum (larsen = true) uses the same split with 0/1
// variables (1: position occupied) and factors N_k = number of occupied
// pairs at distance d_k, 0 <= N_k <= L_k: nothing is halved, and the walk is
// the longest possible (no reversal quadruples).
#pragma once

#include <stdint.h>

#include "sk_internal.h"

namespace sk {

struct PlanCE {
    bool ok = false;
    int n = 0, variant = 0, m = 0, top = 0;
    int pos[kMaxVars] = {};
    int d[kMaxN] = {};
    uint64_t pset = 0;
    int n_lane = 0, n_walk = 0, n_job = 0;
    int nq = 0, G = 0, halved = 0;
    int qb[5] = {};  // group g covers quads [qb[g], qb[g+1])
    // per slot (4*nq used); factor index -1 = constant-1 slot
    int slot_k[kMaxSlots] = {};
    int slot_d[kMaxSlots] = {};
    uint64_t slot_mask[kMaxSlots] = {};
    int slot_len[kMaxSlots] = {};
    int slot_halve[kMaxSlots] = {};
};

constexpr int kWalkCap = 20;

__host__ __device__ constexpr unsigned __int128 u128_max1(uint64_t x) { return x ? x : 1; }

__host__ __device__ constexpr PlanCE make_plan_ce(int n, int variant, int walk_cap = kWalkCap, bool larsen = false)
{
    PlanCE P{};
    if (variant < 0 || variant > 2) return P;
    if (n < 1 || n > kMaxN || (variant == 2 && n > kMaxN - 1)) return P;
    P.n = n;
    P.variant = variant;
    P.top = variant == 2 ? 2 * n + 1 : 2 * n;
    for (int p = 1; p <= P.top; ++p) {
        if (variant == 2 && p == 2 * n) continue;
        P.pos[P.m++] = p;
        P.pset |= 1ull << (p - 1);
    }
    for (int k = 1; k <= n; ++k) P.d[k - 1] = variant == 1 ? k + 1 : k;
    P.n_lane = kLaneBits < P.m - 1 ? kLaneBits : P.m - 1;
    {
        // For Skolem and Langford instances from n = 15 on the walk stops at
        // n - 9 variables (one or two short of the longest walk), so that the
        // job variables hold the mirror pairs of eight middle positions: four
        // reversal quadruples (Lemma 2.3), which skip 15/32 of the jobs
        // instead of 7/16.  A job walks 2^(n-9) sign vectors per lane, at
        // least 2^11 for the instances that dominate a count (n >= 20), so
        // the per-job set-up stays below a percent there.
        const int cap = (!larsen && variant != 2 && n >= 15 && n - 9 < walk_cap) ? n - 9 : walk_cap;
        const int dmax = P.d[n - 1];
        int w = 0;
        while (w + 1 <= P.m - 1 - P.n_lane && w + 1 <= cap && P.pos[w + 1] + dmax < P.pos[P.m - P.n_lane])
            ++w;
        P.n_walk = w;
    }
    P.n_job = P.m - 1 - P.n_lane - P.n_walk;

    // factors
    uint64_t fmask[kMaxN] = {};
    int flen[kMaxN] = {}, fhalve[kMaxN] = {};
    uint64_t fbound[kMaxN] = {};
    for (int k = 0; k < n; ++k) {
        for (int p = 1; p + P.d[k] <= P.top; ++p) {
            if (((P.pset >> (p - 1)) & 1) && ((P.pset >> (p + P.d[k] - 1)) & 1)) {
                fmask[k] |= 1ull << (p - 1);
                ++flen[k];
            }
        }
        fhalve[k] = (!larsen && flen[k] % 2 == 0 && flen[k] > 0) ? 1 : 0;
        fbound[k] = (uint64_t)(flen[k] >> fhalve[k]);
        P.halved += fhalve[k];
    }
    // factor order: bound descending, then k ascending (insertion sort)
    int order[kMaxN] = {};
    for (int k = 0; k < n; ++k) order[k] = k;
    for (int i = 1; i < n; ++i) {
        int v = order[i], j = i - 1;
        while (j >= 0 && (fbound[order[j]] < fbound[v] || (fbound[order[j]] == fbound[v] && order[j] > v))) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = v;
    }
    P.nq = (n + 3) / 4;
    const unsigned __int128 two53 = (unsigned __int128)1 << 53, two50 = (unsigned __int128)1 << 50,
                            two96 = (unsigned __int128)1 << 96;
    for (int G = 1; G <= 4 && G <= P.nq; ++G) {
        // every split of the nq quads into G consecutive groups (ordered sizes)
        int sizes[4] = {1, 1, 1, 1};
        for (;;) {
            int tot = 0;
            for (int g = 0; g < G; ++g) tot += sizes[g];
            if (tot == P.nq) {
                for (int heur = 0; heur < 4; ++heur) {
                    int cap[4] = {}, cnt[4] = {};
                    unsigned __int128 prod[4] = {1, 1, 1, 1};
                    int member[4][kMaxSlots] = {};
                    for (int g = 0; g < G; ++g) cap[g] = 4 * sizes[g];
                    // budget (bits) per group: the first two share 96, the rest 50
                    int budget[4] = {};
                    for (int g = 0; g < G; ++g) budget[g] = G == 1 ? 52 : (g < 2 ? 48 : 49);
                    bool fits = true;
                    for (int i = 0; i < n && fits; ++i) {
                        const int k = order[i];
                        int best = -1;
                        if (heur == 2) {
                            // largest factors first into the groups past the first two
                            // (they only feed the 50-bit chain), then balance g0, g1
                            for (int g = 2; g < G && best < 0; ++g)
                                if (cnt[g] < cap[g] && prod[g] * u128_max1(fbound[k]) < two50) best = g;
                            if (best < 0) {
                                for (int g = 0; g < 2 && g < G; ++g) {
                                    if (cnt[g] >= cap[g]) continue;
                                    if (best < 0 || prod[g] < prod[best]) best = g;
                                }
                            }
                        }
                        if (heur == 3) {
                            // fill the groups from the last one down, largest factors first
                            for (int g = G - 1; g >= 0 && best < 0; --g) {
                                if (cnt[g] >= cap[g]) continue;
                                if (g >= 2 && prod[g] * u128_max1(fbound[k]) >= two50) continue;
                                best = g;
                            }
                        }
                        for (int g = 0; g < G && heur < 2; ++g) {
                            if (cnt[g] >= cap[g]) continue;
                            if (best < 0) {
                                best = g;
                                continue;
                            }
                            if (heur == 0) {
                                if (prod[g] < prod[best]) best = g;
                            } else {
                                // most remaining budget: compare prod / 2^budget
                                const unsigned __int128 lhs = prod[g] << (unsigned)(52 - budget[g]);
                                const unsigned __int128 rhs = prod[best] << (unsigned)(52 - budget[best]);
                                if (lhs < rhs) best = g;
                            }
                        }
                        if (best < 0) {
                            fits = false;
                            break;
                        }
                        member[best][cnt[best]++] = k;
                        prod[best] *= u128_max1(fbound[k]);
                        if (prod[best] >= two53) fits = false;
                    }
                    if (!fits) continue;
                    for (int g = 2; g < G; ++g)
                        if (prod[g] >= two50) fits = false;
                    if (fits && G >= 2 && prod[1] > two96 / prod[0]) fits = false;
                    if (!fits) continue;
                    P.G = G;
                    P.qb[0] = 0;
                    for (int g = 0; g < G; ++g) P.qb[g + 1] = P.qb[g] + sizes[g];
                    int s = 0;
                    for (int g = 0; g < G; ++g) {
                        const int end = 4 * P.qb[g + 1];
                        for (int i = 0; i < cnt[g]; ++i, ++s) {
                            const int k = member[g][i];
                            P.slot_k[s] = k;
                            P.slot_d[s] = P.d[k];
                            P.slot_mask[s] = fmask[k];
                            P.slot_len[s] = flen[k];
                            P.slot_halve[s] = fhalve[k];
                        }
                        for (; s < end; ++s) {
                            P.slot_k[s] = -1;
                            P.slot_d[s] = 0;
                            P.slot_mask[s] = 0;
                            P.slot_len[s] = 1;
                            P.slot_halve[s] = 0;
                        }
                    }
                    for (; s < kMaxSlots; ++s) {
                        P.slot_k[s] = -1;
                        P.slot_len[s] = 1;
                    }
                    P.ok = true;
                    return P;
                }
            }
            // next composition (odometer over sizes[0..G-1], each 1..nq)
            int g = 0;
            while (g < G && ++sizes[g] > P.nq) sizes[g++] = 1;
            if (g == G) break;
        }
    }
    return P;
}

// Fewest primes in (2^45, 2^46) whose product exceeds n! * 2^8.  Every ordered
// count is at most n!: the leftmost uncovered position always starts a new
// pair, so a pairing is fixed by the order in which labels are used.  The
// library's primes are the largest below 2^46, each above 2^45.999, so k of
// them cover 45.999 k bits; log2(n!) is tabulated in thousandths of a bit,
// rounded up.
__host__ __device__ constexpr int primes_for(int n)
{
    constexpr int lg_fact_milli[33] = {0,     0,     1000,  2585,  4585,  6907,  9492,  12300, 15300,
                                       18470, 21792, 25251, 28836, 32536, 36344, 40251, 44251, 48338,
                                       52508, 56756, 61078, 65470, 69930, 74453, 79038, 83682, 88382,
                                       93137, 97945, 102803, 107710, 112664, 117664};
    const int need = lg_fact_milli[n < 0 ? 0 : (n > 32 ? 32 : n)] + 8000;
    int k = 1;
    while (k < kMaxPrimes && k * 45999 < need) ++k;
    return k;
}

}  // namespace sk
