/*
 * CPU oracle for the exact counts of "Counting Skolem Sequences"
 * (Assarpour, Bar-Noy, Liu; arXiv 1507.00315).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * Everything here is plain and slow on purpose:
 *
 *   orc_count_backtrack   -- the plain definition of the count: the number of
 *                            ordered placements (a_1..a_n) of n pairs with
 *                            differences d_k into the position set P, every
 *                            position used once (Sec. 1.1 for Skolem and
 *                            Langford, Sec. 1.2 for hooked Skolem).  Search
 *                            order: the pair with the largest difference is
 *                            placed first, at every position where it fits,
 *                            left to right (the backtracking approach described
 *                            at the start of Sec. 2).
 *   orc_chunk_partial_direct
 *                         -- the signed sign-vector sum of Lemma 2.1 restricted
 *                            to the sign vectors that agree with a fixed partial
 *                            assignment, taken modulo p.  Each term evaluates
 *                            every pair sum f_k from scratch, as Algorithm 1
 *                            does.
 *   orc_chunk_partial_gray
 *                         -- the same sum, visiting the sign vectors in Gray
 *                            code order and updating the pair sums by the
 *                            single sign flip between neighbours (the speed-up
 *                            the paper describes after Algorithm 1).
 *
 * Positions are 1-based.  A position set is a 64-bit mask with bit (pos-1)
 * set for each member.  Variants: 0 = Skolem (P = 1..2n, d_k = k),
 * 1 = Langford (P = 1..2n, d_k = k+1), 2 = hooked Skolem
 * (P = 1..2n-1 and 2n+1, d_k = k).
 *
 * Arithmetic modulo p uses unsigned __int128 products and the C '%' operator;
 * p must satisfy 2 < p < 2^63.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

/* ------------------------------------------------------------------ */
/* Problem statement                                                   */
/* ------------------------------------------------------------------ */

/* Fills pos[0..m-1] (ascending) and d[0..n-1] (ascending); returns m, or -1. */
int orc_instance(int n, int variant, int *pos, int *d)
{
    if (n < 1 || variant < 0 || variant > 2) return -1;
    int top = (variant == 2) ? 2 * n + 1 : 2 * n;
    if (top > 64) return -1;
    int m = 0;
    for (int p = 1; p <= top; p++) {
        if (variant == 2 && p == 2 * n) continue; /* the hook: position 2n is empty */
        pos[m++] = p;
    }
    for (int k = 1; k <= n; k++) d[k - 1] = (variant == 1) ? k + 1 : k;
    return m;
}

static uint64_t position_mask(const int *pos, int m)
{
    uint64_t s = 0;
    for (int i = 0; i < m; i++) s |= 1ull << (pos[i] - 1);
    return s;
}

/* ------------------------------------------------------------------ */
/* Backtracking count                                                  */
/* ------------------------------------------------------------------ */

/* Places pairs k = kk, kk-1, ..., 0 (d ascending, so the largest goes first)
 * into the free positions; returns the number of complete placements. */
static uint64_t place(int kk, uint64_t free_pos, const int *d, int top)
{
    if (kk < 0) return 1;
    uint64_t total = 0;
    int dk = d[kk];
    for (int a = 1; a + dk <= top; a++) {
        uint64_t both = (1ull << (a - 1)) | (1ull << (a + dk - 1));
        if ((free_pos & both) == both) total += place(kk - 1, free_pos & ~both, d, top);
    }
    return total;
}

typedef struct {
    int n, top;
    const int *d;
    uint64_t set;
    int n_items;
    int *item_a, *item_b; /* positions of the two largest pairs */
    int next;
    pthread_mutex_t lock;
    uint64_t total;
} bt_job;

static void *bt_worker(void *arg)
{
    bt_job *J = (bt_job *)arg;
    uint64_t mine = 0;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int i = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (i >= J->n_items) break;
        int a = J->item_a[i], b = J->item_b[i];
        uint64_t free_pos = J->set;
        uint64_t pa = (1ull << (a - 1)) | (1ull << (a + J->d[J->n - 1] - 1));
        free_pos &= ~pa;
        if (J->n >= 2) {
            uint64_t pb = (1ull << (b - 1)) | (1ull << (b + J->d[J->n - 2] - 1));
            free_pos &= ~pb;
            mine += place(J->n - 3, free_pos, J->d, J->top);
        } else {
            mine += 1;
        }
    }
    pthread_mutex_lock(&J->lock);
    J->total += mine;
    pthread_mutex_unlock(&J->lock);
    return NULL;
}

/* Ordered count C(n) (reflections distinct).  threads <= 0 means 1. */
uint64_t orc_count_backtrack(int n, int variant, int threads)
{
    int pos[64], d[64];
    int m = orc_instance(n, variant, pos, d);
    if (m < 0) return 0;
    int top = pos[m - 1];
    uint64_t set = position_mask(pos, m);
    if (threads <= 1 || n < 2) return place(n - 1, set, d, top);

    /* Work items: every compatible placement of the two largest pairs. */
    int cap = 64 * 64, cnt = 0;
    int *ia = (int *)malloc(sizeof(int) * cap), *ib = (int *)malloc(sizeof(int) * cap);
    for (int a = 1; a + d[n - 1] <= top; a++) {
        uint64_t pa = (1ull << (a - 1)) | (1ull << (a + d[n - 1] - 1));
        if ((set & pa) != pa) continue;
        for (int b = 1; b + d[n - 2] <= top; b++) {
            uint64_t pb = (1ull << (b - 1)) | (1ull << (b + d[n - 2] - 1));
            if ((set & pb) != pb || (pa & pb)) continue;
            ia[cnt] = a;
            ib[cnt] = b;
            cnt++;
        }
    }
    bt_job J;
    J.n = n; J.top = top; J.d = d; J.set = set; J.n_items = cnt;
    J.item_a = ia; J.item_b = ib; J.next = 0; J.total = 0;
    pthread_mutex_init(&J.lock, NULL);
    if (threads > 256) threads = 256;
    pthread_t th[256];
    for (int t = 0; t < threads; t++) pthread_create(&th[t], NULL, bt_worker, &J);
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.lock);
    free(ia);
    free(ib);
    return J.total;
}

/* ------------------------------------------------------------------ */
/* Sign-vector sums (Lemma 2.1), restricted to a partial assignment    */
/* ------------------------------------------------------------------ */

/* Residue of a signed 128-bit integer in [0, p). */
static uint64_t mod_signed(i128 v, uint64_t p)
{
    i128 r = v % (i128)p;
    if (r < 0) r += p;
    return (uint64_t)r;
}

/* Product of the pair sums, modulo p.  Factors are multiplied exactly in
 * 128-bit integers while that is safe and reduced with '%' otherwise. */
static uint64_t product_mod(const int *f, int n, uint64_t p)
{
    i128 acc = 1;
    for (int k = 0; k < n; k++) {
        i128 a = acc < 0 ? -acc : acc;
        if (a > ((i128)1 << 110)) acc = (i128)mod_signed(acc, p);
        acc *= f[k];
    }
    return mod_signed(acc, p);
}

/* sign x_pos for a 'negative' bit mask: bit (pos-1) set means x = -1 */
static inline int xval(uint64_t neg, int p) { return ((neg >> (p - 1)) & 1) ? -1 : 1; }

/* f_k for every k, computed from scratch from the full sign vector. */
static void pair_sums_direct(uint64_t neg, uint64_t set, const int *d, int n, int top, int *f)
{
    for (int k = 0; k < n; k++) {
        int s = 0;
        for (int p = 1; p + d[k] <= top; p++) {
            if (!((set >> (p - 1)) & 1) || !((set >> (p + d[k] - 1)) & 1)) continue;
            s += xval(neg, p) * xval(neg, p + d[k]);
        }
        f[k] = s;
    }
}

static int popcount64(uint64_t x) { return __builtin_popcountll(x); }

/*
 * Sum over every sign vector x in {+1,-1}^P that agrees with the fixed
 * assignment (positions in fixed_mask take x = -1 where fixed_neg has the bit
 * set, +1 otherwise) of  (prod_i x_i) * prod_k f_k(x),  modulo p.
 * The free positions are enumerated in plain binary order; each term is
 * evaluated from scratch.
 */
uint64_t orc_chunk_partial_direct(int n, int variant, uint64_t fixed_mask, uint64_t fixed_neg,
                                  uint64_t p)
{
    int pos[64], d[64], f[64];
    int m = orc_instance(n, variant, pos, d);
    if (m < 0 || p < 3) return 0;
    int top = pos[m - 1];
    uint64_t set = position_mask(pos, m);
    int freep[64], nf = 0;
    for (int i = 0; i < m; i++)
        if (!((fixed_mask >> (pos[i] - 1)) & 1)) freep[nf++] = pos[i];
    uint64_t base = fixed_neg & fixed_mask & set;
    uint64_t acc = 0;
    for (uint64_t t = 0; t < (1ull << nf); t++) {
        uint64_t neg = base;
        for (int j = 0; j < nf; j++)
            if ((t >> j) & 1) neg |= 1ull << (freep[j] - 1);
        pair_sums_direct(neg, set, d, n, top, f);
        uint64_t prod = product_mod(f, n, p);
        int sign_neg = popcount64(neg & set) & 1;
        uint64_t term = sign_neg ? (prod == 0 ? 0 : p - prod) : prod;
        acc = (uint64_t)(((u128)acc + term) % p);
    }
    return acc;
}

/*
 * The same sum, visiting the free positions in binary-reflected Gray code
 * order: step t flips the free position with index ctz(t), and each pair sum
 * changes by -2 x_q (x_{q-d_k} + x_{q+d_k}) where q is the flipped position
 * and x_q its value before the flip (neighbours outside P contribute 0).
 * The free positions split into 2^split_bits sub-ranges (the top free
 * positions fixed per sub-range) that run on separate threads.
 */
typedef struct {
    int n, m, top, nf;
    const int *d;
    uint64_t set, base;
    const int *freep;
    uint64_t p;
    int split_bits;
    int next;
    pthread_mutex_t lock;
    uint64_t acc;
} gray_job;

static uint64_t gray_range(const gray_job *G, uint64_t hi_bits)
{
    int n = G->n, nf_lo = G->nf - G->split_bits;
    uint64_t neg = G->base;
    for (int j = 0; j < G->split_bits; j++)
        if ((hi_bits >> j) & 1) neg |= 1ull << (G->freep[nf_lo + j] - 1);
    int f[64];
    pair_sums_direct(neg, G->set, G->d, n, G->top, f);
    int sign_neg = popcount64(neg & G->set) & 1;
    uint64_t p = G->p, acc = 0;
    for (uint64_t t = 0;; t++) {
        if (t > 0) {
            int j = __builtin_ctzll(t);
            int q = G->freep[j];
            int xq = xval(neg, q);
            for (int k = 0; k < n; k++) {
                int nb = 0;
                int lo = q - G->d[k], hi = q + G->d[k];
                if (lo >= 1 && ((G->set >> (lo - 1)) & 1)) nb += xval(neg, lo);
                if (hi <= G->top && ((G->set >> (hi - 1)) & 1)) nb += xval(neg, hi);
                f[k] += -2 * xq * nb;
            }
            neg ^= 1ull << (q - 1);
            sign_neg ^= 1;
        }
        uint64_t prod = product_mod(f, n, p);
        uint64_t term = sign_neg ? (prod == 0 ? 0 : p - prod) : prod;
        acc = (uint64_t)(((u128)acc + term) % p);
        if (t + 1 == (1ull << nf_lo)) break;
    }
    return acc;
}

static void *gray_worker(void *arg)
{
    gray_job *G = (gray_job *)arg;
    for (;;) {
        pthread_mutex_lock(&G->lock);
        int i = G->next++;
        pthread_mutex_unlock(&G->lock);
        if (i >= (1 << G->split_bits)) break;
        uint64_t r = gray_range(G, (uint64_t)i);
        pthread_mutex_lock(&G->lock);
        G->acc = (uint64_t)(((u128)G->acc + r) % G->p);
        pthread_mutex_unlock(&G->lock);
    }
    return NULL;
}

uint64_t orc_chunk_partial_gray(int n, int variant, uint64_t fixed_mask, uint64_t fixed_neg,
                                uint64_t p, int threads)
{
    int pos[64], d[64];
    int m = orc_instance(n, variant, pos, d);
    if (m < 0 || p < 3) return 0;
    int freep[64], nf = 0;
    for (int i = 0; i < m; i++)
        if (!((fixed_mask >> (pos[i] - 1)) & 1)) freep[nf++] = pos[i];
    gray_job G;
    G.n = n; G.m = m; G.top = pos[m - 1]; G.nf = nf; G.d = d;
    G.set = position_mask(pos, m);
    G.base = fixed_neg & fixed_mask & G.set;
    G.freep = freep; G.p = p; G.next = 0; G.acc = 0;
    int sb = 0;
    if (threads > 1) {
        while ((1 << sb) < 4 * threads && sb < 8) sb++;
    }
    if (sb > nf) sb = nf;
    G.split_bits = sb;
    pthread_mutex_init(&G.lock, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    for (int t = 0; t < threads; t++) pthread_create(&th[t], NULL, gray_worker, &G);
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&G.lock);
    return G.acc;
}

/* ------------------------------------------------------------------ */
/* Inclusion-exclusion (the third counting approach of Sec. 2)         */
/* ------------------------------------------------------------------ */
/*
 * The universe is every placement of the n pairs inside the position set
 * with overlaps allowed; A_i holds the placements that leave position i
 * empty.  A placement is a pairing exactly when it leaves no position empty,
 * so by inclusion-exclusion over the sets S of positions forced empty,
 *
 *     C(n) = sum_{S subset of P} (-1)^|S| prod_k N_k(P \ S),
 *
 * N_k(T) = number of a with a, a + d_k both in T.  orc_larsen_partial sums
 * the terms whose S agrees with a fixed part (fixed_mask: positions decided;
 * fixed_empty: those of them in S), each term from scratch, modulo p.
 */
typedef struct {
    int m, n, top;
    const int *pos, *d;
    uint64_t set, fixed_mask, fixed_empty, p;
    int freep[64], nf;
    int split_bits;
    int next;
    pthread_mutex_t lock;
    uint64_t acc;
} ie_job;

/* sum over the free positions' subsets with the top split_bits free
 * positions set by hi, modulo p */
static uint64_t ie_range(const ie_job *J, uint64_t hi)
{
    const int nlow = J->nf - J->split_bits;
    uint64_t acc = 0;
    for (uint64_t lo = 0; lo < (1ull << nlow); lo++) {
        uint64_t empty = J->fixed_empty & J->fixed_mask;
        uint64_t bits = lo | (hi << nlow);
        for (int i = 0; i < J->nf; i++)
            if ((bits >> i) & 1) empty |= 1ull << (J->freep[i] - 1);
        const uint64_t T = J->set & ~empty;
        u128 prod = 1;
        for (int k = 0; k < J->n; k++) {
            uint64_t c = 0;
            for (int a = 1; a + J->d[k] <= J->top; a++)
                if (((T >> (a - 1)) & 1) && ((T >> (a + J->d[k] - 1)) & 1)) c++;
            prod = (prod * c) % J->p;
        }
        if (__builtin_popcountll(empty & J->set) & 1)
            acc = (uint64_t)(((u128)acc + J->p - (uint64_t)prod) % J->p);
        else
            acc = (uint64_t)(((u128)acc + (uint64_t)prod) % J->p);
    }
    return acc;
}

static void *ie_worker(void *arg)
{
    ie_job *J = (ie_job *)arg;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int i = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (i >= (1 << J->split_bits)) break;
        uint64_t r = ie_range(J, (uint64_t)i);
        pthread_mutex_lock(&J->lock);
        J->acc = (uint64_t)(((u128)J->acc + r) % J->p);
        pthread_mutex_unlock(&J->lock);
    }
    return NULL;
}

uint64_t orc_larsen_partial(int n, int variant, uint64_t fixed_mask, uint64_t fixed_empty, uint64_t p,
                            int threads)
{
    int pos[64], d[64];
    int m = orc_instance(n, variant, pos, d);
    if (m < 0 || p < 3) return 0;
    ie_job J;
    memset(&J, 0, sizeof(J));
    J.m = m; J.n = n; J.top = pos[m - 1]; J.pos = pos; J.d = d;
    J.set = position_mask(pos, m);
    J.fixed_mask = fixed_mask & J.set;
    J.fixed_empty = fixed_empty;
    J.p = p;
    for (int i = 0; i < m; i++)
        if (!((J.fixed_mask >> (pos[i] - 1)) & 1)) J.freep[J.nf++] = pos[i];
    int sb = 0;
    if (threads > 1)
        while ((1 << sb) < 4 * threads && sb < 8) sb++;
    if (sb > J.nf) sb = J.nf;
    J.split_bits = sb;
    pthread_mutex_init(&J.lock, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    for (int t = 0; t < threads; t++) pthread_create(&th[t], NULL, ie_worker, &J);
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.lock);
    return J.acc;
}
