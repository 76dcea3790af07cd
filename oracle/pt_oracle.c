/*
 * CPU oracle for the approximate count of Sec. 3 ("Approximate Counting
 * Algorithm", Algorithm 2) of "Counting Skolem Sequences" (arXiv 1507.00315).
 *
 * TEST INFRASTRUCTURE ONLY (see skolem_oracle.c): nothing in the product
 * library links or calls this file.
 *
 * The relaxed problem (Sec. 3): n pairs of balls, pair k occupies positions
 * a_k and a_k + d_k of the position set P (every such placement allowed, balls
 * may share a bin).  A configuration is C = (a_1..a_n); its energy E(C) is the
 * number of empty bins.  Configurations with E = 0 are exactly the pairings.
 * Z(beta) = sum_C exp(-beta E(C)); Z(0) = prod_k L_k (L_k placements of pair k),
 * Z(infinity) = number of ordered pairings.
 *
 * A chain at inverse temperature beta picks a pair k uniformly, proposes a
 * uniform placement for it and accepts with min(1, exp(-beta dE)) (Sec. 3;
 * Algorithm 2 prints the test as "p <= random" -- the usual Metropolis test,
 * accept when a uniform draw falls below p, is taken here).  Neighbouring
 * temperatures exchange configurations with min(1, exp(-(b_{j+1}-b_j)(E_j -
 * E_{j+1}))).  Ratio(j) accumulates exp(-(b_{j+1} - b_j) E) at level j before
 * the moves of every iteration; here the accumulation is kept exactly as a
 * histogram of energies per level, from which the host forms the ratios.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), written from that definition.  Counter
 * layout (c0, c1, c2, c3) = (iteration low 32, iteration high 32, ladder, level);
 * initial configurations use c1 = 0xFFFFFFFF and c0 = 0xFFFFFFF0 + block.
 * Draws: r0 -> pair index floor(r0 n / 2^32); r1 -> placement index
 * floor(r1 L_k / 2^32) into the ascending list of placements; r2 -> accept the
 * move iff dE <= 0 or r2 < T(beta_j, dE); r3 -> accept the exchange of levels
 * (j, j+1) iff the energy difference gives dE' <= 0 or level j's r3 <
 * T(b_{j+1} - b_j, E_j - E_{j+1}); T(b, e) = floor(2^32 exp(-b e)) computed in
 * double precision with the C library's exp.
 *
 * Exchange schedule: schedule 0 = the sweep of Algorithm 2 (pairs (j, j+1) for
 * j = 0, 1, ..., M-2 one after the other); schedule 1 = even pairs on even
 * iterations, odd pairs on odd iterations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ Philox */

static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
    }
    memcpy(out, c, sizeof(c));
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------ problem */

/* Pairs n <= PT_MAXN, positions 1..top with top <= 2 PT_MAXN + 1. */
#define PT_MAXN 40
#define PT_MAXTOP (2 * PT_MAXN + 1)

typedef struct {
    int n, m, top;
    int d[PT_MAXN];
    int L[PT_MAXN];
    int start[PT_MAXN][PT_MAXTOP]; /* ascending placements of pair k */
    char in_set[PT_MAXTOP + 2];    /* in_set[p]: position p belongs to P */
} relaxed;

static int setup(int n, int variant, relaxed *R)
{
    if (n < 1 || n > PT_MAXN || variant < 0 || variant > 2) return -1;
    memset(R, 0, sizeof(*R));
    R->n = n;
    R->top = (variant == 2) ? 2 * n + 1 : 2 * n;
    for (int p = 1; p <= R->top; ++p) {
        if (variant == 2 && p == 2 * n) continue;
        R->in_set[p] = 1;
        R->m++;
    }
    for (int k = 0; k < n; ++k) {
        R->d[k] = (variant == 1) ? k + 2 : k + 1;
        for (int a = 1; a + R->d[k] <= R->top; ++a)
            if (R->in_set[a] && R->in_set[a + R->d[k]]) R->start[k][R->L[k]++] = a;
        if (R->L[k] == 0) return 1; /* no configuration at all */
    }
    return 0;
}

/* Energy: number of bins of P holding no ball. */
static int energy(const relaxed *R, const int *occ)
{
    int e = 0;
    for (int p = 1; p <= R->top; ++p)
        if (R->in_set[p] && occ[p] == 0) ++e;
    return e;
}

/* Number of placements with each energy, by enumerating all of them.
 * hist must hold top + 1 entries.  Returns 0 on success. */
int orc_energy_histogram(int n, int variant, uint64_t *hist)
{
    relaxed R;
    const int rc = setup(n, variant, &R);
    if (rc < 0) return -1;
    memset(hist, 0, sizeof(uint64_t) * (R.top + 1));
    if (rc > 0) return 0; /* Z(0) = 0 */
    int idx[PT_MAXN] = {0};
    int occ[PT_MAXTOP + 2];
    for (;;) {
        memset(occ, 0, sizeof(occ));
        for (int k = 0; k < n; ++k) {
            occ[R.start[k][idx[k]]]++;
            occ[R.start[k][idx[k]] + R.d[k]]++;
        }
        hist[energy(&R, occ)]++;
        int k = 0;
        while (k < n && ++idx[k] == R.L[k]) idx[k++] = 0;
        if (k == n) break;
    }
    return 0;
}

static uint32_t threshold(double b, int e)
{
    if (e <= 0) return 0xFFFFFFFFu; /* unused: always accept */
    const double t = ldexp(exp(-b * (double)e), 32);
    if (t >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)t;
}

typedef struct {
    int a[PT_MAXN];
    int occ[PT_MAXTOP + 2];
    int e;
} chain_state;

static void place(const relaxed *R, chain_state *s, int k, int a, int sign)
{
    s->occ[a] += sign;
    s->occ[a + R->d[k]] += sign;
}

/*
 * One ladder of M levels for `iters` iterations.
 *   beta[M]          ascending inverse temperatures
 *   hist[M][top+1]   accumulated energy histogram (added to, not cleared)
 *   move_acc[M]      accepted moves per level (added to)
 *   swap_acc[M]      accepted exchanges of levels (j, j+1) (added to)
 *   swap_try[M]      attempted exchanges of levels (j, j+1) (added to)
 *   final_a[M][n]    placements at the end (level order), may be NULL
 *   final_e[M]       energies at the end, may be NULL
 * Returns 0 on success.
 */
int orc_pt_ladder(int n, int variant, int M, const double *beta, uint64_t iters, uint64_t seed,
                  uint32_t ladder, int schedule, uint64_t *hist, uint64_t *move_acc, uint64_t *swap_acc,
                  uint64_t *swap_try, int *final_a, int *final_e)
{
    relaxed R;
    if (setup(n, variant, &R) || M < 1 || M > 64) return -1;
    const int H = R.top + 1;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    chain_state *st = (chain_state *)calloc((size_t)M, sizeof(chain_state));
    uint32_t (*Tm)[5] = calloc((size_t)M, sizeof(*Tm));
    uint32_t *Ts = (uint32_t *)calloc((size_t)M * (R.top + 1), sizeof(uint32_t));
    if (!st || !Tm || !Ts) {
        free(st);
        free(Tm);
        free(Ts);
        return -2;
    }
    for (int j = 0; j < M; ++j) {
        for (int e = 1; e <= 4; ++e) Tm[j][e] = threshold(beta[j], e);
        if (j + 1 < M)
            for (int e = 1; e <= R.top; ++e) Ts[j * (R.top + 1) + e] = threshold(beta[j + 1] - beta[j], e);
    }
    /* initial configurations: uniform placements */
    for (int j = 0; j < M; ++j) {
        for (int blk = 0; blk * 4 < n; ++blk) {
            const uint32_t ctr[4] = {0xFFFFFFF0u + (uint32_t)blk, 0xFFFFFFFFu, ladder, (uint32_t)j};
            uint32_t r[4];
            philox4x32_10(ctr, key, r);
            for (int t = 0; t < 4 && blk * 4 + t < n; ++t) {
                const int k = blk * 4 + t;
                const int idx = (int)(((uint64_t)r[t] * (uint64_t)R.L[k]) >> 32);
                st[j].a[k] = R.start[k][idx];
                place(&R, &st[j], k, st[j].a[k], +1);
            }
        }
        st[j].e = energy(&R, st[j].occ);
    }
    uint32_t (*rnd)[4] = calloc((size_t)M, sizeof(*rnd));
    for (uint64_t it = 0; it < iters; ++it) {
        /* 1: record the energies (Ratio accumulation) */
        for (int j = 0; j < M; ++j) hist[j * H + st[j].e]++;
        /* 2: one Metropolis move per level */
        for (int j = 0; j < M; ++j) {
            const uint32_t ctr[4] = {(uint32_t)it, (uint32_t)(it >> 32), ladder, (uint32_t)j};
            philox4x32_10(ctr, key, rnd[j]);
            chain_state *s = &st[j];
            const int k = (int)(((uint64_t)rnd[j][0] * (uint64_t)n) >> 32);
            const int idx = (int)(((uint64_t)rnd[j][1] * (uint64_t)R.L[k]) >> 32);
            const int a_new = R.start[k][idx];
            const int a_old = s->a[k];
            place(&R, s, k, a_old, -1);
            place(&R, s, k, a_new, +1);
            const int e_new = energy(&R, s->occ);
            const int de = e_new - s->e;
            if (de <= 0 || rnd[j][2] < Tm[j][de]) {
                s->a[k] = a_new;
                s->e = e_new;
                move_acc[j]++;
            } else {
                place(&R, s, k, a_new, -1);
                place(&R, s, k, a_old, +1);
            }
        }
        /* 3: exchanges of neighbouring levels */
        for (int j = (schedule == 1 ? (int)(it & 1) : 0); j + 1 < M; j += (schedule == 1 ? 2 : 1)) {
            swap_try[j]++;
            const int de = st[j].e - st[j + 1].e;
            if (de <= 0 || rnd[j][3] < Ts[j * (R.top + 1) + de]) {
                chain_state tmp = st[j];
                st[j] = st[j + 1];
                st[j + 1] = tmp;
                swap_acc[j]++;
            }
        }
    }
    if (final_a)
        for (int j = 0; j < M; ++j)
            for (int k = 0; k < n; ++k) final_a[j * n + k] = st[j].a[k];
    if (final_e)
        for (int j = 0; j < M; ++j) final_e[j] = st[j].e;
    free(rnd);
    free(st);
    free(Tm);
    free(Ts);
    return 0;
}
