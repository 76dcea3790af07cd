/*
 * skolem.h -- C ABI of the MI355X (gfx950) library for counting Skolem,
 * Langford and hooked Skolem pairings, after "Counting Skolem Sequences"
 * (Assarpour, Bar-Noy, Liu; arXiv 1507.00315).
 *
 * Problems (Sec. 1.1, Sec. 1.2):
 *   SK_SKOLEM   split {1..2n} into n pairs (a_k, a_k + k), k = 1..n.
 *   SK_LANGFORD split {1..2n} into n pairs (a_k, a_k + k + 1): the two copies
 *               of k have k numbers between them.
 *   SK_HOOKED   split {1..2n-1, 2n+1} into n pairs (a_k, a_k + k).
 *
 * Method (Sec. 2.1, Lemma 2.1): the number of ordered pairings C(n) is the
 * coefficient of x_1...x_{2n} in prod_k f_k with f_k = sum_i x_i x_{i+d_k},
 * equal to 2^{-2n} times the sum over x in {+1,-1}^{2n} of (prod x) prod_k f_k.
 * The library evaluates the half of the sum with the first sign fixed to +1
 * (Lemma 2.2), further reduced by the even-position symmetry (Lemma 2.4) and
 * the reversal symmetry (Lemma 2.3), visits sign vectors in Gray-code order on
 * the GPU, takes the products modulo several primes below 2^46 and recombines
 * them on the host by the Chinese remainder theorem (Sec. 2.2).
 *
 * Conventions for every entry point:
 *   - All pointers are host pointers unless the name says dev_.
 *   - The caller owns every buffer it passes; the library keeps no pointer to
 *     it after the call returns.
 *   - Device workspace: the exact-sum entry points take a dev_workspace of
 *     ws_bytes bytes (device memory on the current device, e.g. a torch
 *     uint8 tensor's data pointer, 256-byte aligned), sized by
 *     sk_workspace_bytes or sk_partial_workspace_bytes.  It is used only
 *     during the call; its contents on entry do not matter.  NULL: the
 *     library allocates what the call needs and frees it before returning.
 *     A workspace that is too small gives SK_ENOMEM before any work starts.
 *   - A stream argument is a hipStream_t passed as void*; NULL means the
 *     library's own stream.  Calls return after their work has completed.
 *   - Errors are reported only through the status code.  On error, outputs
 *     are left untouched.  No C++ exception crosses this interface.
 *   - Calls are thread-safe with respect to each other except where noted.
 */
#ifndef SKOLEM_H
#define SKOLEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SK_SKOLEM = 0, SK_LANGFORD = 1, SK_HOOKED = 2 } sk_variant;

typedef enum {
    SK_OK = 0,
    SK_EINVAL = -1,   /* bad argument: n out of range, unknown variant, bad chunk id, NULL output */
    SK_ERANGE = -2,   /* the requested primes do not cover the range the result needs */
    SK_EDEVICE = -3,  /* a HIP runtime error; sk_last_error() has the runtime's message */
    SK_ECHECK = -4,   /* a self-check failed: the result is not trusted (silent-error guard) */
    SK_ENOMEM = -5,   /* host or device allocation failed, or a workspace is too small */
    SK_EABORTED = -6, /* the progress callback asked to stop */
    SK_ENOLIB = -7    /* the library was built without a kernel for this instance shape */
} sk_status;

/* Flags for sk_count / sk_instance.flags */
#define SK_ORDERED     0x1u /* count reflections as distinct (A004075 / A176127 style);
                               default: reflections counted once for Skolem and Langford,
                               n > 1 (Sec. 1.3); hooked counts are never halved */
#define SK_NO_SHORTCUT 0x2u /* evaluate the sum even when the existence conditions
                               (Sec. 1.1) already give 0 */
#define SK_VERIFY      0x4u /* run the whole sum a second time modulo a disjoint set of
                               primes and require both results to agree (the analogue of
                               the paper's duplicate GPU jobs, Sec. 1.3) */
#define SK_NO_SYMMETRY 0x8u /* evaluate every sign vector with x_1 = +1.  By default, when
                               the term is invariant under negating the even positions
                               (Lemma 2.4; for every variant this holds exactly when the
                               existence conditions do), only the half with the highest
                               chunk variable (an even position) at +1 is evaluated and
                               the sum is doubled; and for Skolem and Langford pairings
                               the reversal symmetry (Lemma 2.3) weights the settings of
                               the middle job variables by 0, 1 or 2 so that about half
                               of the remaining work is skipped (sk_stats.reversal_quads) */

/* Unsigned 128-bit integer; every count with n <= 32 fits. */
typedef struct { uint64_t lo, hi; } sk_u128;

/* Launch shape.  Zero in a field means "library default / autotuned".
 *   log2_chunk_terms : sign vectors per chunk (the batched launch: per work item)
 *   waves_per_launch : single counts: chunks per kernel launch (the host splits
 *                      the work into launches of this many chunks; the tuned
 *                      kernel's persistent waves, 8 per SIMD, pull small work
 *                      items of the launch's chunks from a queue, the
 *                      reference kernel runs one wavefront per chunk); the
 *                      batched launch: its persistent wavefronts
 *   primes           : primes per pass for sk_count (1..4); default the fewest
 *                      whose product exceeds n! * 2^8 (n! bounds every count)
 *   kernel           : kernel body: 0 = the tuned body when built for the
 *                      instance, else the reference; 1 = reference; 2 = tuned
 *                      (SK_ENOLIB if not built)
 *   primes_per_item  : batched launch: 0 = every work item (chunk) takes all
 *                      of its instance's primes; 1 = one prime per work item
 *                      (where that kernel is built; else 0)                    */
typedef struct {
    int log2_chunk_terms;
    int waves_per_launch;
    int primes;
    int kernel;
    int primes_per_item;
} sk_tuning;

/* One instance of a batched count. */
typedef struct {
    int n;
    int variant;     /* sk_variant */
    unsigned flags;  /* SK_ORDERED | SK_NO_SHORTCUT | SK_VERIFY | SK_NO_SYMMETRY */
} sk_instance;

/* Timing and shape of the last completed call on this thread. */
typedef struct {
    double kernel_ms;        /* sum of kernel durations (HIP events on the launch stream) */
    double wall_ms;          /* whole call, host clock */
    uint64_t terms;          /* sign vectors evaluated (x_1 fixed; fewer when the
                                symmetries apply: symmetry_halved, reversal_quads) */
    uint64_t launches;       /* kernel launches */
    uint64_t chunks;         /* wavefront work units */
    int nprimes;             /* primes used per pass */
    int passes;              /* 1, or 2 with SK_VERIFY */
    int log2_chunk_terms;
    int kernel_variant;      /* which kernel body ran (see sk_kernel_name) */
    double ms_per_launch_avg;
    uint64_t primes[8];
    int symmetry_halved;     /* 1 if the Lemma 2.4 half was evaluated and doubled */
    int reversal_quads;      /* reversal weighting (Lemma 2.3): quadruples in use, 0 if none */
} sk_stats;

/* Progress callback: return nonzero to abort (the call then returns SK_EABORTED). */
typedef int (*sk_progress_fn)(void *ctx, uint64_t terms_done, uint64_t terms_total);

/* Selects the HIP device used by later calls of this thread (default 0) and
 * does the library's set-up for it (its stream, the fixed workspace of
 * sk_count_batch_noalloc), if not done yet. */
sk_status sk_set_device(int device);

/*
 * sk_count -- exact number of pairings for (n, variant), Sec. 2.
 *   n       : 1..32 (Skolem, Langford), 1..31 (hooked)
 *   flags   : SK_ORDERED | SK_NO_SHORTCUT | SK_VERIFY | SK_NO_SYMMETRY
 *   out     : receives the count
 * Errors: SK_EINVAL, SK_EDEVICE, SK_ECHECK (CRT result above the a priori bound
 * n!, or the SK_VERIFY passes disagree), SK_ENOLIB.
 */
sk_status sk_count(int n, int variant, unsigned flags, sk_u128 *out);

/* sk_count with a launch shape (NULL: defaults), a device workspace (see the
 * conventions; NULL: internal), a stream, a progress callback (NULL: none) and
 * a statistics record (NULL: not wanted). */
sk_status sk_count_ex(int n, int variant, unsigned flags, const sk_tuning *tune,
                      void *dev_workspace, size_t ws_bytes, void *stream,
                      sk_progress_fn progress, void *progress_ctx,
                      sk_stats *stats, sk_u128 *out);

/*
 * sk_count_larsen -- the same exact count by the third approach of Sec. 2,
 * inclusion-exclusion over the positions a placement leaves empty: with the
 * universe of all placements of the n pairs inside the position set
 * (overlaps allowed) and A_i the placements avoiding position i,
 *     C(n) = sum_{S subset of P} (-1)^|S| prod_k N_k(P \ S),
 * N_k(T) = number of a with a, a + d_k in T.  The 2^(2n) terms are visited in
 * Gray-code order on the GPU (occupancy bits instead of signs; nothing is
 * halved and no symmetry is used) and summed modulo the same primes as
 * sk_count.  An independent cross-check of sk_count.  Arguments, flags
 * (SK_NO_SYMMETRY has no effect), errors: as sk_count_ex; SK_ENOLIB where
 * the instance shape has no kernel (the reference body covers every n).
 */
sk_status sk_count_larsen(int n, int variant, unsigned flags, const sk_tuning *tune,
                          void *dev_workspace, size_t ws_bytes, void *stream,
                          sk_stats *stats, sk_u128 *out);

/*
 * sk_workspace_bytes -- device workspace that sk_count_ex, sk_count_larsen,
 * sk_count_part and sk_count_batch need for these k instances and launch shape: the 128-bit
 * per-prime accumulators of the on-device reduction (Sec. 2.2: the parts'
 * results are put together at the end) and the work counter of the batched
 * launch.  0 on bad input.  Host only.
 */
size_t sk_workspace_bytes(const sk_instance *inst, size_t k, const sk_tuning *tune);

/*
 * sk_partial_workspace_bytes -- device workspace sk_partial_chunks needs for
 * nchunks chunks and nprimes primes with this launch shape: the accumulators
 * and work-queue counter, then one row of 128-bit sums and one chunk id per
 * chunk of a launch.  0 on bad input.
 */
size_t sk_partial_workspace_bytes(int n, int variant, size_t nchunks, int nprimes,
                                  const sk_tuning *tune);

/*
 * sk_count_part / sk_count_combine -- one count split into independent jobs
 * (Sec. 2.2: the sign space is split, the parts run on different GPUs, and the
 * results are put together at the end).  sk_count_part evaluates the part-th
 * of `parts` equal shares of the work sk_count would do for (n, variant,
 * flags) and returns its sum modulo each of the count's primes (the
 * sk_describe(n, variant).primes largest primes below 2^46), Lemma 2.4
 * doubling and reversal weights included; separate calls (processes, GPUs,
 * machines) may compute the parts.  sk_count_combine (host only) adds the
 * parts' residues and finishes the count exactly as sk_count does (CRT, bound
 * check, reflections).
 *   parts    : a power of two, at most the number of chunks of the count
 *              (SK_EINVAL otherwise); part < parts
 *   residues : sk_count_part: sk_describe(...).primes outputs in [0, p);
 *              sk_count_combine: parts x primes, row k from part k
 * The shares follow the library's own chunking of the instance, so all parts
 * of one count must come from the same build (and the same tune).
 * SK_VERIFY is not accepted by sk_count_part.  Errors: as sk_count.
 */
sk_status sk_count_part(int n, int variant, unsigned flags, uint64_t part, uint64_t parts,
                        const sk_tuning *tune, void *dev_workspace, size_t ws_bytes,
                        void *stream, sk_progress_fn progress, void *progress_ctx,
                        sk_stats *stats, uint64_t *residues);
sk_status sk_count_combine(int n, int variant, unsigned flags, const uint64_t *residues, uint64_t parts,
                           sk_u128 *out);

/*
 * sk_count_batch -- exact counts of k instances (Sec. 2) in persistent kernel
 * launches: wavefronts pull (instance, chunk) work items from one global queue,
 * so instances of very different size share the GPU without a tail per
 * instance.  The instances are grouped (n = 12, 13; the mixed set Skolem 16,
 * 17, 20, 21, Langford 15, 16, 19, 20, hooked 14, 15; the other 14 <= n <= 21;
 * 22 <= n <= 25: the persistent kernel of a group holds the tuned body of each
 * of its instances), one launch per group that holds instances (at most 16);
 * instances outside the groups, and instances with tune->kernel == 1 or a
 * larger prime count, are counted by separate launches in the same call.
 *   inst  : k instances (k >= 1); out: k counts, in order
 *   tune  : NULL = the shape found by sk_autotune_batch for this instance set
 *           (cached per GPU model; without a cached shape 2^22 sign vectors
 *           per work item and 8 waves per SIMD), else log2_chunk_terms (sign
 *           vectors per work item) and waves_per_launch (persistent grid)
 *   dev_workspace, ws_bytes : see the conventions (sk_workspace_bytes)
 *   stats : NULL or receives the totals of the call
 * Reduction: each wavefront's residues are summed per instance and prime in
 * its workgroup's LDS, then into 128-bit device accumulators; the host reads
 * one sum per instance and prime.
 * Errors: as sk_count; SK_EINVAL for k == 0 or a bad instance; SK_ENOMEM for
 * a workspace below sk_workspace_bytes.
 */
sk_status sk_count_batch(const sk_instance *inst, size_t k, const sk_tuning *tune,
                         void *dev_workspace, size_t ws_bytes, void *stream,
                         sk_stats *stats, sk_u128 *out);

/*
 * sk_count_batch_noalloc -- sk_count_batch for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The device workspace is a fixed array of the
 * library, 4096 bytes on each GPU it runs on, held until the process ends;
 * the call makes no hipMalloc, hipFree, event or stream (the per-device
 * set-up -- the library's stream and the array's address -- is done by
 * sk_set_device, or else by the first call on a device).  Every call on one
 * GPU uses that GPU's array and clears what it needs at its start: calls
 * that overlap on one GPU (threads, streams) race and must not be made.
 * stats->kernel_ms is the host-clock time of the launches (no events).
 * Errors: as sk_count_batch; SK_ENOMEM if the instances need more workspace
 * than the fixed array holds (sk_workspace_bytes).
 */
sk_status sk_count_batch_noalloc(const sk_instance *inst, size_t k, const sk_tuning *tune,
                                 void *stream, sk_stats *stats, sk_u128 *out);

/*
 * sk_autotune_batch -- times the batched launch of these instances, group by
 * group, on a fraction of their work (1/4, less above 2^42 sign vectors)
 * for a grid of (sign vectors per work item) x (waves per SIMD) x (primes per
 * work item, where built), stores the fastest shape of each group in the cache
 * file ($SK_TUNE_CACHE, default ~/.cache/skolem_mi355x_tune.txt) keyed by GPU
 * model and instance set, and returns that of the group with the most sign
 * vectors.  Instances that sk_count_batch counts by separate launches (no
 * batched kernel, or no pairing exists) are left out.  best_rate (nullable)
 * receives the returned shape's sign vectors per second.
 * Errors: SK_ENOLIB if no instance of the set runs in a batched launch.
 */
sk_status sk_autotune_batch(const sk_instance *inst, size_t k, void *stream, sk_tuning *best,
                            double *best_rate);

/*
 * sk_sign_sum_residues -- the half-sum of Lemma 2.1 with x_1 = +1, before the
 * division by 2^{2n-1}:  H = sum_{x : x_1 = +1} (prod x) prod_k f_k(x),
 * reduced modulo each given prime.
 *   primes   : nprimes (1..8) odd primes with 2^45 < p < 2^46 (caller's choice)
 *   tune     : launch shape and kernel body (NULL: defaults)
 *   residues : nprimes outputs, H mod p in [0, p)
 * Errors: SK_EINVAL (prime out of range), SK_EDEVICE, SK_ENOLIB.
 */
sk_status sk_sign_sum_residues(int n, int variant, const uint64_t *primes, int nprimes,
                               const sk_tuning *tune, void *stream, uint64_t *residues);

/*
 * sk_partial_chunks -- per-chunk partial sums (Sec. 2.2: the sign space split
 * into independent parts whose results are added at the end).
 *
 * Chunk definition.  Order the 2n sign variables by position.  Variable 1 is
 * fixed to +1.  The six variables at the highest positions are never fixed by
 * a chunk.  A chunk of a split into 2^c chunks fixes the c variables directly
 * below those six: bit b of the chunk id sets x = -1 (bit set) or +1 (clear)
 * for the variable with 1-based rank (2n - 6 - c + 1 + b) in position order.
 * A chunk then holds 2^(2n-1-c) sign vectors.
 *
 *   log2_chunks : c, 0 <= c <= 2n - 7 - (the count of low variables the
 *                 kernel walks; sk_max_chunk_bits gives the largest legal c)
 *   chunk_ids   : nchunks ids, each < 2^c (repeats allowed)
 *   primes      : nprimes (1..8) primes with 2^45 < p < 2^46, or NULL for the
 *                 nprimes largest primes below 2^46 (the ones sk_count uses)
 *   tune        : waves_per_launch and kernel fields are used (NULL: defaults)
 *   dev_workspace, ws_bytes : see the conventions (sk_partial_workspace_bytes)
 *   residues_out: nchunks x nprimes, row-major, each the chunk's signed sum
 *                 of (prod x) prod_k f_k(x) modulo the prime, in [0, p)
 * Errors: SK_EINVAL, SK_EDEVICE, SK_ENOLIB, SK_ENOMEM (workspace too small).
 */
sk_status sk_partial_chunks(int n, int variant, int log2_chunks, const uint64_t *chunk_ids,
                            size_t nchunks, const uint64_t *primes, int nprimes,
                            const sk_tuning *tune, void *dev_workspace, size_t ws_bytes,
                            void *stream, uint64_t *residues_out);

/* Totals of the last sk_count, sk_count_ex, sk_count_batch,
 * sk_sign_sum_residues or sk_partial_chunks call made by this thread. */
sk_status sk_last_stats(sk_stats *out);


/* ------------------------------------------------------------------------
 * Approximate counting by parallel tempering (Sec. 3, Algorithm 2).
 *
 * Relaxed problem: pair k may sit at any placement (a_k, a_k + d_k) inside the
 * position set, pairs may overlap; the energy of a configuration is its number
 * of empty positions.  Z(beta) = sum exp(-beta E); Z(0) = prod_k L_k counts all
 * configurations, Z(infinity) the ordered pairings.  Each ladder runs M chains
 * at 0 = beta_0 < beta_1 < ... < beta_{M-1}; per iteration every level records
 * its energy, makes one Metropolis move and neighbouring levels attempt an
 * exchange (even pairs on even iterations, odd pairs on odd ones).  The
 * estimate of a ladder is Z(0) * prod_j Ratio(j) with Ratio(j) the mean of
 * exp(-(beta_{j+1} - beta_j) E) at level j and the last ratio the fraction of
 * samples with E = 0 at beta_{M-1} (beta_M = infinity).  Randomness: Philox4x32-10
 * keyed by the seed, counter (iteration, ladder, level).
 * ---------------------------------------------------------------------- */

#define SK_PROPOSAL_UNIFORM 0 /* pair uniform, placement uniform (Sec. 3) */
#define SK_PROPOSAL_LEARNED 1 /* MLP proposal with Metropolis-Hastings correction */

/*
 * Learned proposal (not in the paper; an extension of Sec. 3's chains).  A
 * network q(k, a' | C, beta) over single-pair moves is trained on states the
 * chains generate and used as an extra Metropolis-Hastings move: each chain of
 * levels first_level..M-1 proposes (k, a') ~ q(. | C) and accepts with
 * min(1, exp(-beta (E(C') - E(C))) q(k, a_k | C') / q(k, a' | C)), so every
 * level keeps exp(-beta E) as its stationary law.  The run:
 *   1. train_iterations plain iterations (not recorded); the configurations
 *      of the learned levels at `snapshots` evenly spaced points form the
 *      training pool;
 *   2. train_steps Adam steps (learning rate lr) on minibatches of the pool;
 *   3. the recorded iterations, with one learned move of the learned levels
 *      after every plain_per_learned plain iterations (network frozen).
 * Learned moves use Philox counters (move index, 0xFFFFFFFE, ladder, level):
 * word 0 picks the move, word 1 decides it.
 */
typedef struct {
    int hidden1, hidden2;       /* hidden widths (0: 256) */
    int first_level;            /* levels first_level..M-1 take learned moves */
    uint64_t plain_per_learned; /* plain iterations per learned move, >= 1 */
    uint64_t train_iterations;  /* plain iterations that feed the training pool */
    int snapshots;              /* pool snapshots taken during them, >= 1 */
    int train_steps;            /* Adam steps (0: use params as given) */
    int minibatch;              /* states per Adam step */
    double lr;                  /* Adam learning rate */
    uint64_t init_seed;         /* initial weights when params is NULL */
    float *params;              /* NULL, or sk_mlp_param_count floats: the initial
                                   network in, the trained one out */
} sk_learned_params;

typedef struct {
    int levels;          /* M, 2..64 */
    const double *beta;  /* M ascending inverse temperatures, beta[0] == 0 */
    int ladders;         /* independent ladders, >= 1 (one wavefront each) */
    uint64_t iterations; /* per ladder */
    uint64_t seed;       /* Philox key */
    int proposal;        /* SK_PROPOSAL_* */
    unsigned flags;      /* SK_ORDERED: estimate the ordered count */
    uint64_t segment;    /* iterations per kernel launch (0: 2^24); chains carry over */
    uint64_t burn_in;    /* iterations run first and not recorded */
    const sk_learned_params *learned; /* SK_PROPOSAL_LEARNED only */
} sk_pt_params;

typedef struct {
    double mean_energy[64]; /* per level, pooled over ladders */
    double move_accept[64]; /* accepted moves / iterations */
    double swap_accept[64]; /* accepted exchanges of (j, j+1) / attempts */
    double ratio[64];       /* Ratio(j) from the pooled histograms */
    double gpu_ms;          /* kernel time (HIP events) */
    double wall_ms;
    uint64_t moves;         /* ladders x levels x iterations */
    int levels, ladders;
    double learned_accept[64]; /* accepted learned moves that changed the configuration
                                  / learned moves, per level */
    uint64_t learned_moves;    /* learned moves per chain of a learned level */
    double train_ms;           /* GPU time of the training phase (included in gpu_ms) */
    double train_loss;         /* mean cross-entropy of the last Adam minibatch */
    /* Equilibration check: the estimate and its standard error from the first
     * and from the second half of the recorded iterations (for a learned run,
     * split at the first learned move past the middle), and
     * half_z = (second - first) / sqrt(se_first^2 + se_second^2).  The
     * standard error of sk_approx measures the spread between ladders only;
     * chains that are still equilibrating bias every ladder the same way and
     * show as |half_z| well above 2 (0 when the run is too short to split). */
    double estimate_half[2];
    double std_error_half[2];
    double half_z;
} sk_pt_stats;

/* Energy bins per level: 2n + 1 (Skolem, Langford) or 2n + 2 (hooked); -1 on
 * bad input.  Host only. */
int sk_pt_bins(int n, int variant);

/*
 * sk_pt_run -- runs the ladders and returns the raw chain statistics.
 *   hist     : ladders x levels x sk_pt_bins(n, variant) energy counts (filled)
 *   move_acc : ladders x levels accepted moves (filled)
 *   swap_acc : ladders x levels accepted exchanges of (j, j+1) (filled)
 *   state    : NULL or ladders x levels x n final placements a_k (1-based
 *              positions), in level order
 *   energy   : NULL or ladders x levels final energies
 *   Burn-in and training iterations advance the chains but are not recorded;
 *   their Philox counters precede the recorded ones (iteration numbers run
 *   on from 0 across all phases).
 * Errors: SK_EINVAL (bad ladder: beta[0] != 0, not ascending, levels out of
 * range, no configuration; bad learned parameters), SK_EDEVICE.
 */
sk_status sk_pt_run(int n, int variant, const sk_pt_params *p, void *stream, uint64_t *hist,
                    uint64_t *move_acc, uint64_t *swap_acc, uint8_t *state, int32_t *energy);

/*
 * sk_approx -- approximate count (reflections counted once for Skolem and
 * Langford unless p->flags has SK_ORDERED): mean of the ladders' estimates and
 * its standard error (sample standard deviation / sqrt(ladders); 0 for one
 * ladder).  stats may be NULL.
 */
sk_status sk_approx(int n, int variant, const sk_pt_params *p, void *stream, double *estimate,
                    double *std_error, sk_pt_stats *stats);

/*
 * sk_pt_tune_ladder -- inverse temperatures 0 = beta_0 < ... < beta_{M-1} =
 * beta_max chosen as the last paragraph of Sec. 3 prescribes: every exchange
 * of neighbouring levels is accepted with probability at least `target` (the
 * paper: one half), with no more levels than that takes.  Starting from
 * {0, beta_max}, pilot runs (plain moves, `pilot_iterations` burn-in and as
 * many recorded iterations on `ladders` ladders, Philox key seed + round)
 * measure the acceptance of each neighbouring pair; a level is inserted in
 * the middle of every pair below the target (the arithmetic mean next to
 * beta = 0, the geometric mean elsewhere), lowest acceptance first, until no
 * pair is below the target or max_levels (<= 64) is reached.
 *   beta_out    : max_levels doubles, the ladder (levels_out of them)
 *   accept_out  : NULL or max_levels doubles, the last pilot's acceptance of
 *                 the exchange (j, j+1); if max_levels stopped the search,
 *                 some are below the target
 * Errors: SK_EINVAL (bad instance or arguments), SK_EDEVICE.
 */
sk_status sk_pt_tune_ladder(int n, int variant, double beta_max, double target, int max_levels,
                            int ladders, uint64_t pilot_iterations, uint64_t seed, void *stream,
                            double *beta_out, int *levels_out, double *accept_out);

/* ------------------------------------------------------------------------
 * The proposal network (fp32, device-resident while a call runs).
 *
 * Input of configuration C at inverse temperature beta (din = T + 2n + 2
 * values, T = largest position): occupancy indicator of each position 1..T,
 * a_k / T for each pair, 1 if pair k shares a position with another pair,
 * beta, E(C) / |P|.  Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
 * z = W3 h2 + b3 with dout = n * T logits, entry k * T + (a' - 1) for pair k
 * at a'; q is the softmax over the valid placements.  Training target: the
 * heat-bath law p*(k, a') proportional to exp(-beta E(C with a_k = a')),
 * loss the mean cross-entropy -sum p* log q.
 * Parameters: one flat fp32 array, row-major (out x in) weights,
 *   W1[h1][din] b1[h1] W2[h2][h1] b2[h2] W3[dout][h2] b3[dout].
 * states: batch x n placements a_k (1-based left positions, uint8), each a
 * valid placement (else SK_EINVAL); betas: batch doubles (used as fp32).
 * All buffers are host memory owned by the caller.  h1, h2 = 0 mean 256.
 * ---------------------------------------------------------------------- */

/* Number of parameters (0 on bad input). */
size_t sk_mlp_param_count(int n, int variant, int h1, int h2);

/* Gaussian initial weights (standard deviation scale / sqrt(fan in)), zero
 * biases.  Host only. */
sk_status sk_mlp_init(int n, int variant, int h1, int h2, uint64_t seed, double scale, float *params);

/* logits: batch x (n * T) (entries of impossible placements are left as
 * computed; q ignores them). */
sk_status sk_mlp_forward(int n, int variant, int h1, int h2, const float *params, const uint8_t *states,
                         const double *betas, int batch, void *stream, float *logits);

/* Mean cross-entropy over the batch and its gradient (param layout). */
sk_status sk_mlp_loss_grad(int n, int variant, int h1, int h2, const float *params, const uint8_t *states,
                           const double *betas, int batch, void *stream, double *loss, float *grads);

/* steps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, moments from zero) on
 * minibatches of the nstates states: step t uses rows (t * minibatch + i) mod
 * nstates, i < minibatch.  params is updated in place; last_loss (nullable)
 * receives the last minibatch's mean loss before its update. */
sk_status sk_mlp_train(int n, int variant, int h1, int h2, float *params, const uint8_t *states,
                       const double *betas, int nstates, int steps, int minibatch, double lr, void *stream,
                       double *last_loss);

/* One learned Metropolis-Hastings move per state.  The move (k, a') is the
 * first entry j (in k * T + a' - 1 order over valid placements) whose
 * cumulative q exceeds w_pick * 2^-32 times the total; it is accepted when
 * w_acc * 2^-32 < min(1, exp(-beta dE) q(k, a_k | C') / q(k, a' | C)).
 * out_states: resulting states; accepted, proposed (batch x n), logq_forward
 * (log q(k, a' | C)) and logq_reverse (log q(k, a_k | C')) are nullable. */
sk_status sk_mlp_mh_step(int n, int variant, int h1, int h2, const float *params, const uint8_t *states,
                         const double *betas, const uint32_t *w_pick, const uint32_t *w_acc, int batch,
                         void *stream, uint8_t *out_states, uint8_t *accepted, uint8_t *proposed,
                         float *logq_forward, float *logq_reverse);

/* Largest legal log2_chunks for sk_partial_chunks (negative on bad input). */
int sk_max_chunk_bits(int n, int variant);

/* How the library splits the sign variables of (n, variant).  Host only. */
typedef struct {
    int m;            /* sign variables, 2n */
    int n_lane;       /* highest variables enumerated across the 64 lanes */
    int n_walk;       /* lowest free variables walked in Gray-code order */
    int n_job;        /* the variables between them (chunk and job bits) */
    int quads;        /* factor slots / 4 */
    int groups;       /* exact fp64 product groups per term */
    int halved;       /* factors with an even number of pairs, stored as f_k / 2 */
    int primes;       /* primes per pass chosen by sk_count */
    int slot_factor[32]; /* factor index k-1 in each slot, -1 for a constant-1 slot */
    int symmetric;    /* 1 if the term is invariant under negating the even positions
                         (Lemma 2.4), so sk_count evaluates half the sign vectors */
    int reversal_quads; /* reversal (Lemma 2.3) quadruples sk_count uses with the tuned
                           kernel; it then evaluates 1/2 + 2^-(r+1) of the remaining jobs */
} sk_plan_desc;

sk_status sk_describe(int n, int variant, sk_plan_desc *out);

/* The same for the inclusion-exclusion sum of sk_count_larsen (0/1 variables:
 * nothing halved, symmetric = reversal_quads = 0).  Host only. */
sk_status sk_describe_larsen(int n, int variant, sk_plan_desc *out);

/* Describes a status code (static string). */
const char *sk_strerror(sk_status s);

/* Message of the last HIP error seen by this thread ("" if none). */
const char *sk_last_error(void);

/* Decimal text of x into buf (NUL-terminated); returns the length, or -1 if
 * len is too small. */
int sk_u128_to_decimal(sk_u128 x, char *buf, size_t len);

/* Name of a kernel body, for reports and profiles. */
const char *sk_kernel_name(int kernel_variant);

#ifdef __cplusplus
}
#endif

#endif /* SKOLEM_H */
