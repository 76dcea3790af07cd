// Host side of the tempering path (Sec. 3, Algorithm 2): threshold tables,
// segmenting of long runs, the estimator and its standard error.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/skolem.h"
#include "sk_mlp.h"
#include "sk_mlp_net.h"
#include "sk_pt.h"

namespace sk {

const char* set_last_error(const std::string& msg);
int current_device();

// floor(2^32 exp(-b e)), saturated; the Metropolis test accepts when a 32-bit
// uniform word is below it.
static uint32_t accept_threshold(double b, int e)
{
    const double t = std::ldexp(std::exp(-b * (double)e), 32);
    if (t >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)t;
}

struct Relaxed {
    int n = 0, variant = 0, top = 0, m = 0;
    std::vector<char> in_set;  // in_set[p]: position p belongs to P (p = 0..top)
    std::vector<int> L;        // placements of each pair
};

static bool relaxed_of(int n, int variant, Relaxed& R)
{
    if (n < 1 || n > kPtMaxN || variant < 0 || variant > 2) return false;
    R.n = n;
    R.variant = variant;
    R.top = variant == 2 ? 2 * n + 1 : 2 * n;
    R.in_set.assign(R.top + 1, 0);
    for (int p = 1; p <= R.top; ++p) {
        if (variant == 2 && p == 2 * n) continue;
        R.in_set[p] = 1;
        ++R.m;
    }
    for (int k = 0; k < n; ++k) {
        const int d = variant == 1 ? k + 2 : k + 1;
        int c = 0;
        for (int a = 1; a + d <= R.top; ++a)
            if (R.in_set[a] && R.in_set[a + d]) ++c;
        R.L.push_back(c);
    }
    return true;
}

#define PT_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            set_last_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
            return SK_EDEVICE;                                                        \
        }                                                                             \
    } while (0)

#define PT_OK(expr)                             \
    do {                                        \
        sk_status s_ = (expr);                  \
        if (s_ != SK_OK) return s_;             \
    } while (0)

// What a run reports besides the recorded statistics.
struct PtExtra {
    double gpu_ms = 0, train_ms = 0, train_loss = 0;
    uint64_t learned_moves = 0;
    std::vector<uint64_t> learned_acc;  // ladders x levels
    bool want_half = false;             // record the histograms of the first part of the run
    std::vector<uint64_t> hist_first;   // ladders x levels x bins, recorded iterations [0, first_iters)
    uint64_t first_iters = 0;
};

// Device state of one run: thresholds, the two configuration buffers the
// segments alternate between, and the recorded statistics.
struct PtDevice {
    uint32_t *mt = nullptr, *st = nullptr;
    uint8_t *sa = nullptr, *sb = nullptr;
    int32_t* e = nullptr;
    uint64_t *h = nullptr, *ma = nullptr, *sw = nullptr, *la = nullptr, *h1 = nullptr;
    float* beta_f = nullptr;
    uint8_t *pool = nullptr;
    float* pool_beta = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    uint8_t* cur = nullptr;  // configurations after the last segment (nullptr: fresh start)
    ~PtDevice()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (void* p : {(void*)mt, (void*)st, (void*)sa, (void*)sb, (void*)e, (void*)h, (void*)ma, (void*)sw,
                        (void*)la, (void*)beta_f, (void*)pool, (void*)pool_beta, (void*)h1})
            if (p) (void)hipFree(p);
    }
};

// Enqueues plain iterations [it0, it1) in launches of at most seg iterations.
// An empty range still launches once if refresh is set or no configuration
// exists yet: that launch draws (or copies) the configurations and writes
// their energies.
static sk_status enqueue_plain(PtDevice& D, PtArgs a, int ladders, size_t lds, uint64_t seg, uint64_t it0,
                               uint64_t it1, hipStream_t stream, bool refresh = false)
{
    if (it0 == it1 && D.cur && !refresh) return SK_OK;
    for (uint64_t it = it0; it < it1 || it == it0; it += seg) {
        a.it_begin = it;
        a.it_end = std::min<uint64_t>(it1, it + seg);
        a.state_in = D.cur;
        a.state_out = (D.cur == D.sa) ? D.sb : D.sa;
        for (int base = 0; base < ladders; base += 65535) {
            a.ladder_base = (uint32_t)base;
            const unsigned cnt = (unsigned)std::min(65535, ladders - base);
            PT_HIP(launch_pt_ladders(cnt, lds, stream, a));
        }
        D.cur = a.state_out;
    }
    return SK_OK;
}

static sk_status clear_stats(PtDevice& D, size_t nh, size_t nl, hipStream_t stream)
{
    PT_HIP(hipMemsetAsync(D.h, 0, nh * sizeof(uint64_t), stream));
    PT_HIP(hipMemsetAsync(D.ma, 0, nl * sizeof(uint64_t), stream));
    PT_HIP(hipMemsetAsync(D.sw, 0, nl * sizeof(uint64_t), stream));
    if (D.la) PT_HIP(hipMemsetAsync(D.la, 0, nl * sizeof(uint64_t), stream));
    return SK_OK;
}

static sk_status elapsed(PtDevice& D, hipStream_t stream, double& ms_out)
{
    PT_HIP(hipEventRecord(D.e1, stream));
    PT_HIP(hipEventSynchronize(D.e1));
    float ms = 0.f;
    PT_HIP(hipEventElapsedTime(&ms, D.e0, D.e1));
    ms_out += ms;
    return SK_OK;
}

// Chains per learned batch (the network's activations are sized for it).
constexpr long kLearnBatch = 65536;

// One learned move of every chain of levels j0..M-1, in batches.
static sk_status learned_move(MlpNet& net, PtDevice& D, int n, int M, int j0, long chains, uint64_t seed,
                              uint32_t step, hipStream_t stream)
{
    const int nsel = M - j0;
    for (long base = 0; base < chains; base += kLearnBatch) {
        const int B = (int)std::min<long>(kLearnBatch, chains - base);
        PT_HIP(launch_gather(n, D.cur, M, j0, nsel, base, D.beta_f, B, net.s_sel, net.betaf, stream));
        PT_HIP(launch_words(seed, step, j0, nsel, base, B, net.w_pick, net.w_acc, stream));
        PT_OK(net.mh_step(B, M, j0, nsel, base, D.cur, D.la, nullptr, stream));
    }
    return SK_OK;
}

// Runs burn-in (and for the learned proposal, the training phase), then
// p->iterations recorded iterations; outputs are filled (not added).
static sk_status pt_run_impl(const Relaxed& R, const sk_pt_params* p, hipStream_t stream, uint64_t* hist,
                             uint64_t* move_acc, uint64_t* swap_acc, uint8_t* state, int32_t* energy, PtExtra* ex)
{
    const int M = p->levels, Lad = p->ladders, H = R.top + 1, n = R.n;
    const bool learned = p->proposal == SK_PROPOSAL_LEARNED;
    std::vector<uint32_t> mt(2 * M), stt((size_t)M * H, 0);
    for (int j = 0; j < M; ++j) {
        mt[2 * j] = accept_threshold(p->beta[j], 1);
        mt[2 * j + 1] = accept_threshold(p->beta[j], 2);
        if (j + 1 < M)
            for (int e = 1; e < H; ++e) stt[(size_t)j * H + e] = accept_threshold(p->beta[j + 1] - p->beta[j], e);
    }
    // host sources of queued copies are declared before D, whose destructor
    // (hipFree) waits for the device, so they outlive every copy on any path
    const std::vector<float> beta_f(p->beta, p->beta + M);
    PtDevice D;
    const size_t nst = (size_t)Lad * M * n, nh = (size_t)Lad * M * H, nl = (size_t)Lad * M;
    // an odd number of LDS words per slot: the lanes' byte accesses at the same offset in
    // their slots spread over the banks (an even stride, 16 words at n = 20, made S(20)
    // 2 % slower)
    int slot_bytes = (n + H + 3) & ~3;
    if ((slot_bytes / 4) % 2 == 0) slot_bytes += 4;
    // LDS: 64 configuration slots, the histograms and the exchange thresholds
    const size_t lds = (size_t)64 * slot_bytes + 2 * (size_t)M * H * sizeof(uint32_t);
    // iterations per launch; LDS counters stay below 2^32
    const uint64_t seg = (p->segment > 0 && p->segment <= (1ull << 30)) ? p->segment : (1ull << 24);
    PT_HIP(hipMalloc(&D.mt, mt.size() * sizeof(uint32_t)));
    PT_HIP(hipMalloc(&D.st, stt.size() * sizeof(uint32_t)));
    PT_HIP(hipMalloc(&D.sa, nst));
    PT_HIP(hipMalloc(&D.sb, nst));
    PT_HIP(hipMalloc(&D.e, nl * sizeof(int32_t)));
    PT_HIP(hipMalloc(&D.h, nh * sizeof(uint64_t)));
    PT_HIP(hipMalloc(&D.ma, nl * sizeof(uint64_t)));
    PT_HIP(hipMalloc(&D.sw, nl * sizeof(uint64_t)));
    if (ex && ex->want_half) PT_HIP(hipMalloc(&D.h1, nh * sizeof(uint64_t)));
    PT_HIP(hipEventCreate(&D.e0));
    PT_HIP(hipEventCreate(&D.e1));
    PT_HIP(hipMemcpyAsync(D.mt, mt.data(), mt.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    PT_HIP(hipMemcpyAsync(D.st, stt.data(), stt.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream));

    PtArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    a.variant = R.variant;
    a.top = R.top;
    a.levels = M;
    a.slot_bytes = slot_bytes;
    a.seed = p->seed;
    a.move_thr = D.mt;
    a.swap_thr = D.st;
    a.energy_out = D.e;
    a.hist_out = D.h;
    a.move_acc = D.ma;
    a.swap_acc = D.sw;

    double gpu_ms = 0, train_ms = 0, train_loss = 0;
    uint64_t it = 0;  // iteration counter across all phases (Philox counters)
    uint64_t learned_moves = 0;
    MlpNet net;
    const sk_learned_params* L = p->learned;
    const int j0 = learned ? L->first_level : 0;
    const long chains = (long)Lad * (M - j0);

    PT_HIP(hipEventRecord(D.e0, stream));
    PT_OK(clear_stats(D, nh, nl, stream));
    if (p->burn_in > 0) {
        PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it + p->burn_in, stream));
        it += p->burn_in;
    }
    if (learned) {
        MlpGeo g;
        if (!mlp_geometry(n, R.variant, g)) return SK_EINVAL;
        PT_OK(net.init(g, L->hidden1, L->hidden2, stream));
        if (L->params) {
            PT_HIP(hipMemcpyAsync(net.P, L->params, net.count * sizeof(float), hipMemcpyHostToDevice, stream));
        } else {
            std::vector<float> init(net.count);
            PT_OK(sk_mlp_init(n, R.variant, L->hidden1, L->hidden2, L->init_seed, 1.0, init.data()));
            PT_HIP(hipMemcpyAsync(net.P, init.data(), net.count * sizeof(float), hipMemcpyHostToDevice, stream));
            PT_HIP(hipStreamSynchronize(stream));
        }
        PT_HIP(hipMalloc(&D.beta_f, M * sizeof(float)));
        PT_HIP(hipMalloc(&D.la, nl * sizeof(uint64_t)));
        PT_HIP(hipMemcpyAsync(D.beta_f, beta_f.data(), M * sizeof(float), hipMemcpyHostToDevice, stream));
        PT_HIP(hipMemsetAsync(D.la, 0, nl * sizeof(uint64_t), stream));
        if (L->train_steps > 0) {
            // training pool: the learned levels' configurations at each snapshot
            const int S = L->snapshots;
            const long N = chains * S;
            PT_HIP(hipMalloc(&D.pool, (size_t)N * n));
            PT_HIP(hipMalloc(&D.pool_beta, (size_t)N * sizeof(float)));
            for (int snap = 0; snap < S; ++snap) {
                const uint64_t len = L->train_iterations / S + (snap + 1 == S ? L->train_iterations % S : 0);
                PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it + len, stream));
                it += len;
                PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it, stream));
                for (long base = 0; base < chains; base += kLearnBatch) {
                    const int B = (int)std::min<long>(kLearnBatch, chains - base);
                    PT_HIP(launch_gather(n, D.cur, M, j0, M - j0, base, D.beta_f, B,
                                         D.pool + ((size_t)snap * chains + base) * n,
                                         D.pool_beta + (size_t)snap * chains + base, stream));
                }
            }
            double before = 0;
            PT_OK(elapsed(D, stream, before));
            PT_HIP(hipEventRecord(D.e0, stream));
            PT_OK(net.reserve((int)std::min<long>(L->minibatch, kLearnBatch)));
            PT_OK(net.train_pool(D.pool, D.pool_beta, (int)N, L->train_steps,
                                 (int)std::min<long>(L->minibatch, kLearnBatch), (float)L->lr, stream, &train_loss));
            PT_OK(elapsed(D, stream, train_ms));
            gpu_ms += before + train_ms;
            PT_HIP(hipEventRecord(D.e0, stream));
            net.free_batch();
            // both pointers cleared before any error is returned, so the
            // destructor never frees them a second time
            const hipError_t fa = hipFree(D.pool), fb = hipFree(D.pool_beta);
            D.pool = nullptr;
            D.pool_beta = nullptr;
            PT_HIP(fa);
            PT_HIP(fb);
        } else if (L->train_iterations > 0) {
            PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it + L->train_iterations, stream));
            it += L->train_iterations;
        }
        PT_OK(net.reserve((int)std::min<long>(chains, kLearnBatch)));
        PT_OK(clear_stats(D, nh, nl, stream));
        PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it, stream));
        // recorded phase: plain blocks, each followed by a learned move
        const uint64_t blk = L->plain_per_learned;
        uint64_t done = 0;
        while (done < p->iterations) {
            const uint64_t len = std::min<uint64_t>(blk, p->iterations - done);
            PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it + len, stream));
            it += len;
            done += len;
            if (len == blk) {
                PT_OK(learned_move(net, D, n, M, j0, chains, p->seed, (uint32_t)learned_moves, stream));
                ++learned_moves;
            }
            if (D.h1 && ex->first_iters == 0 && 2 * done >= p->iterations) {
                PT_HIP(hipMemcpyAsync(D.h1, D.h, nh * sizeof(uint64_t), hipMemcpyDeviceToDevice, stream));
                ex->first_iters = done;
            }
        }
        // energies of the configurations the last learned move left
        if (learned_moves > 0) PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it, stream, true));
    } else {
        PT_OK(clear_stats(D, nh, nl, stream));
        // with the halves wanted, the histograms after the first half are copied
        const uint64_t first = D.h1 ? p->iterations / 2 : p->iterations;
        PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it + first, stream));
        it += first;
        if (D.h1) {
            PT_HIP(hipMemcpyAsync(D.h1, D.h, nh * sizeof(uint64_t), hipMemcpyDeviceToDevice, stream));
            ex->first_iters = first;
            PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it + (p->iterations - first), stream));
            it += p->iterations - first;
        }
    }
    PT_OK(enqueue_plain(D, a, Lad, lds, seg, it, it, stream));  // zero iterations: initial states
    PT_OK(elapsed(D, stream, gpu_ms));

    PT_HIP(hipMemcpyAsync(hist, D.h, nh * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    PT_HIP(hipMemcpyAsync(move_acc, D.ma, nl * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    PT_HIP(hipMemcpyAsync(swap_acc, D.sw, nl * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    if (state) PT_HIP(hipMemcpyAsync(state, D.cur, nst, hipMemcpyDeviceToHost, stream));
    if (energy) PT_HIP(hipMemcpyAsync(energy, D.e, nl * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    if (D.h1) {
        ex->hist_first.resize(nh);
        PT_HIP(hipMemcpyAsync(ex->hist_first.data(), D.h1, nh * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    }
    if (ex && D.la) {
        ex->learned_acc.resize(nl);
        PT_HIP(hipMemcpyAsync(ex->learned_acc.data(), D.la, nl * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    }
    PT_HIP(hipStreamSynchronize(stream));
    if (ex) {
        ex->gpu_ms = gpu_ms;
        ex->train_ms = train_ms;
        ex->train_loss = train_loss;
        ex->learned_moves = learned_moves;
    }
    if (learned && L->params && L->train_steps > 0)
        PT_HIP(hipMemcpy(L->params, net.P, net.count * sizeof(float), hipMemcpyDeviceToHost));
    return SK_OK;
}

// Per ladder: Z(0) prod_j Ratio(j) (Sec. 3), the last ratio taken to
// beta = infinity (fraction of samples with E = 0); halved for reflections.
// Then the mean over the ladders and its standard error.
static void estimate_of(const Relaxed& R, const sk_pt_params* p, const uint64_t* hist, bool halve, double& mean,
                        double& se)
{
    const int M = p->levels, Lad = p->ladders, H = R.top + 1;
    double logz0 = 0;
    for (int x : R.L) logz0 += std::log((double)x);
    std::vector<double> est(Lad);
    for (int l = 0; l < Lad; ++l) {
        double lg = logz0;
        bool zero = false;
        for (int j = 0; j < M; ++j) {
            const uint64_t* h = &hist[((size_t)l * M + j) * H];
            double tot = 0, num = 0;
            for (int e = 0; e < H; ++e) tot += (double)h[e];
            if (j + 1 < M) {
                const double db = p->beta[j + 1] - p->beta[j];
                for (int e = 0; e < H; ++e) num += (double)h[e] * std::exp(-db * e);
            } else {
                num = (double)h[0];
            }
            if (num <= 0 || tot <= 0) {
                zero = true;
                break;
            }
            lg += std::log(num / tot);
        }
        est[l] = zero ? 0.0 : std::exp(lg) * (halve ? 0.5 : 1.0);
    }
    mean = 0;
    for (double x : est) mean += x;
    mean /= Lad;
    double var = 0;
    for (double x : est) var += (x - mean) * (x - mean);
    se = Lad > 1 ? std::sqrt(var / (Lad - 1) / Lad) : 0.0;
}

static sk_status check_params(const Relaxed& R, const sk_pt_params* p)
{
    if (!p || !p->beta || p->levels < 2 || p->levels > kPtMaxLevels || p->ladders < 1) return SK_EINVAL;
    if (p->beta[0] != 0.0) return SK_EINVAL;
    for (int j = 1; j < p->levels; ++j)
        if (!(p->beta[j] > p->beta[j - 1]) || !std::isfinite(p->beta[j])) return SK_EINVAL;
    for (int x : R.L)
        if (x == 0) return SK_EINVAL;  // no configuration at all
    if (p->proposal == SK_PROPOSAL_UNIFORM) return SK_OK;
    if (p->proposal != SK_PROPOSAL_LEARNED) return SK_EINVAL;
    const sk_learned_params* L = p->learned;
    if (!L || L->first_level < 0 || L->first_level >= p->levels || L->plain_per_learned < 1 || L->hidden1 < 0 ||
        L->hidden2 < 0 || L->hidden1 > 4096 || L->hidden2 > 4096)
        return SK_EINVAL;
    if (L->train_steps < 0) return SK_EINVAL;
    if (L->train_steps > 0 &&
        (L->snapshots < 1 || L->minibatch < 1 || !(L->lr > 0) || L->train_iterations < (uint64_t)L->snapshots))
        return SK_EINVAL;
    if (L->train_steps == 0 && !L->params) return SK_EINVAL;  // an untrained fresh network is of no use
    return SK_OK;
}

}  // namespace sk

using namespace sk;

extern "C" {

int sk_pt_bins(int n, int variant)
{
    Relaxed R;
    if (!relaxed_of(n, variant, R)) return -1;
    return R.top + 1;
}

sk_status sk_pt_run(int n, int variant, const sk_pt_params* p, void* stream, uint64_t* hist, uint64_t* move_acc,
                    uint64_t* swap_acc, uint8_t* state, int32_t* energy)
{
    Relaxed R;
    if (!relaxed_of(n, variant, R) || !hist || !move_acc || !swap_acc) return SK_EINVAL;
    sk_status s = check_params(R, p);
    if (s != SK_OK) return s;
    if (hipSetDevice(current_device()) != hipSuccess) return SK_EDEVICE;
    hipStream_t st = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (!st) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) return SK_EDEVICE;
        st = own;
    }
    s = pt_run_impl(R, p, st, hist, move_acc, swap_acc, state, energy, nullptr);
    if (own) (void)hipStreamDestroy(own);
    return s;
}

sk_status sk_approx(int n, int variant, const sk_pt_params* p, void* stream, double* estimate, double* std_error,
                    sk_pt_stats* stats)
{
    auto t0 = std::chrono::steady_clock::now();
    Relaxed R;
    if (!relaxed_of(n, variant, R) || !estimate) return SK_EINVAL;
    sk_status s = check_params(R, p);
    if (s != SK_OK) return s;
    if (hipSetDevice(current_device()) != hipSuccess) return SK_EDEVICE;
    const int M = p->levels, Lad = p->ladders, H = R.top + 1;
    std::vector<uint64_t> hist((size_t)Lad * M * H), ma((size_t)Lad * M), sw((size_t)Lad * M);
    hipStream_t st = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (!st) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) return SK_EDEVICE;
        st = own;
    }
    PtExtra ex;
    ex.want_half = p->iterations >= 2;
    s = pt_run_impl(R, p, st, hist.data(), ma.data(), sw.data(), nullptr, nullptr, &ex);
    if (own) (void)hipStreamDestroy(own);
    if (s != SK_OK) return s;

    // Z(0) = prod_k L_k times the ratios of every ladder; mean and standard error
    const bool halve = !(p->flags & SK_ORDERED) && variant != SK_HOOKED && n > 1;
    double mean = 0, se = 0;
    estimate_of(R, p, hist.data(), halve, mean, se);
    // the same from each half of the recorded iterations: a short run whose
    // chains are still equilibrating gives halves that differ by more than
    // their standard errors allow (the bias is common to all ladders, so the
    // spread between ladders does not show it)
    double half_est[2] = {0, 0}, half_se[2] = {0, 0}, half_z = 0;
    if (!ex.hist_first.empty() && ex.first_iters > 0 && ex.first_iters < p->iterations) {
        std::vector<uint64_t> second(hist.size());
        for (size_t i = 0; i < hist.size(); ++i) second[i] = hist[i] - ex.hist_first[i];
        estimate_of(R, p, ex.hist_first.data(), halve, half_est[0], half_se[0]);
        estimate_of(R, p, second.data(), halve, half_est[1], half_se[1]);
        const double den = std::sqrt(half_se[0] * half_se[0] + half_se[1] * half_se[1]);
        half_z = den > 0 ? (half_est[1] - half_est[0]) / den : 0.0;
    }
    *estimate = mean;
    if (std_error) *std_error = se;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->estimate_half[0] = half_est[0];
        stats->estimate_half[1] = half_est[1];
        stats->std_error_half[0] = half_se[0];
        stats->std_error_half[1] = half_se[1];
        stats->half_z = half_z;
        stats->levels = M;
        stats->ladders = Lad;
        stats->gpu_ms = ex.gpu_ms;
        stats->train_ms = ex.train_ms;
        stats->train_loss = ex.train_loss;
        stats->learned_moves = ex.learned_moves;
        stats->moves = (uint64_t)Lad * M * p->iterations;
        for (int j = 0; j < M; ++j) {
            double tot = 0, se_sum = 0, num = 0, acc = 0, swa = 0;
            for (int l = 0; l < Lad; ++l) {
                const uint64_t* h = &hist[((size_t)l * M + j) * H];
                for (int e = 0; e < H; ++e) {
                    tot += (double)h[e];
                    se_sum += (double)h[e] * e;
                    if (j + 1 < M) num += (double)h[e] * std::exp(-(p->beta[j + 1] - p->beta[j]) * e);
                    else if (e == 0) num += (double)h[e];
                }
                acc += (double)ma[(size_t)l * M + j];
                swa += (double)sw[(size_t)l * M + j];
            }
            stats->mean_energy[j] = tot > 0 ? se_sum / tot : 0;
            stats->ratio[j] = tot > 0 ? num / tot : 0;
            stats->move_accept[j] = p->iterations ? acc / ((double)Lad * p->iterations) : 0;
            // exchanges of (j, j+1) are attempted on every other iteration
            const double tries = (double)Lad * (double)((p->iterations + ((j & 1) ? 0 : 1)) / 2);
            stats->swap_accept[j] = (j + 1 < M && tries > 0) ? swa / tries : 0;
            if (!ex.learned_acc.empty() && ex.learned_moves > 0) {
                double la = 0;
                for (int l = 0; l < Lad; ++l) la += (double)ex.learned_acc[(size_t)l * M + j];
                stats->learned_accept[j] = la / ((double)Lad * (double)ex.learned_moves);
            }
        }
        stats->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return SK_OK;
}

sk_status sk_pt_tune_ladder(int n, int variant, double beta_max, double target, int max_levels, int ladders,
                            uint64_t pilot_iterations, uint64_t seed, void* stream, double* beta_out,
                            int* levels_out, double* accept_out)
{
    Relaxed R;
    if (!relaxed_of(n, variant, R) || !beta_out || !levels_out) return SK_EINVAL;
    if (!(beta_max > 0) || !std::isfinite(beta_max) || !(target > 0 && target < 1) || max_levels < 2 ||
        max_levels > kPtMaxLevels || ladders < 1 || pilot_iterations < 2)
        return SK_EINVAL;
    for (int x : R.L)
        if (x == 0) return SK_EINVAL;
    if (hipSetDevice(current_device()) != hipSuccess) return SK_EDEVICE;
    hipStream_t st = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (!st) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) return SK_EDEVICE;
        st = own;
    }
    std::vector<double> beta = {0.0, beta_max};
    std::vector<double> acc;
    sk_status s = SK_OK;
    for (int round = 0; round < 64; ++round) {
        const int M = (int)beta.size();
        sk_pt_params p;
        std::memset(&p, 0, sizeof(p));
        p.levels = M;
        p.beta = beta.data();
        p.ladders = ladders;
        p.iterations = pilot_iterations;
        p.burn_in = pilot_iterations;
        p.seed = seed + (uint64_t)round;
        p.proposal = SK_PROPOSAL_UNIFORM;
        const int H = R.top + 1;
        std::vector<uint64_t> hist((size_t)ladders * M * H), ma((size_t)ladders * M), sw((size_t)ladders * M);
        s = pt_run_impl(R, &p, st, hist.data(), ma.data(), sw.data(), nullptr, nullptr, nullptr);
        if (s != SK_OK) break;
        // pooled acceptance of the exchange (j, j+1), attempted on every other iteration
        acc.assign(M - 1, 0.0);
        for (int j = 0; j + 1 < M; ++j) {
            double swa = 0;
            for (int l = 0; l < ladders; ++l) swa += (double)sw[(size_t)l * M + j];
            const double tries = (double)ladders * (double)((pilot_iterations + ((j & 1) ? 0 : 1)) / 2);
            acc[j] = tries > 0 ? swa / tries : 0.0;
        }
        // a level in the middle of every pair below the target, lowest
        // acceptance first while levels remain
        std::vector<int> low;
        for (int j = 0; j + 1 < M; ++j)
            if (acc[j] < target) low.push_back(j);
        if (low.empty() || M >= max_levels) break;
        std::sort(low.begin(), low.end(), [&](int x, int y) { return acc[x] < acc[y]; });
        if ((int)low.size() > max_levels - M) low.resize(max_levels - M);
        std::sort(low.begin(), low.end());
        std::vector<double> nb;
        size_t li = 0;
        for (int j = 0; j < M; ++j) {
            nb.push_back(beta[j]);
            if (li < low.size() && low[li] == j) {
                nb.push_back(beta[j] == 0.0 ? 0.5 * beta[j + 1] : std::sqrt(beta[j] * beta[j + 1]));
                ++li;
            }
        }
        beta.swap(nb);
    }
    if (own) (void)hipStreamDestroy(own);
    if (s != SK_OK) return s;
    *levels_out = (int)beta.size();
    for (size_t j = 0; j < beta.size(); ++j) beta_out[j] = beta[j];
    if (accept_out) {
        for (size_t j = 0; j < beta.size(); ++j) accept_out[j] = j < acc.size() ? acc[j] : 0.0;
    }
    return SK_OK;
}

}  // extern "C"
