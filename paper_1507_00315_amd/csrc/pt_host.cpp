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
    uint64_t pset = 0;
    std::vector<int> L;  // placements of each pair
};

static bool relaxed_of(int n, int variant, Relaxed& R)
{
    if (n < 1 || n > 32 || variant < 0 || variant > 2 || (variant == 2 && n > 31)) return false;
    R.n = n;
    R.variant = variant;
    R.top = variant == 2 ? 2 * n + 1 : 2 * n;
    for (int p = 1; p <= R.top; ++p) {
        if (variant == 2 && p == 2 * n) continue;
        R.pset |= 1ull << (p - 1);
        ++R.m;
    }
    for (int k = 0; k < n; ++k) {
        const int d = variant == 1 ? k + 2 : k + 1;
        int c = 0;
        for (int a = 1; a + d <= R.top; ++a)
            if (((R.pset >> (a - 1)) & 1) && ((R.pset >> (a + d - 1)) & 1)) ++c;
        R.L.push_back(c);
    }
    return true;
}

#define PT_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            set_last_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
            status = SK_EDEVICE;                                                      \
            goto done;                                                                \
        }                                                                             \
    } while (0)

// Runs every ladder for p->iterations iterations; outputs are filled (not added).
static sk_status pt_run_impl(const Relaxed& R, const sk_pt_params* p, hipStream_t stream, uint64_t* hist,
                             uint64_t* move_acc, uint64_t* swap_acc, uint8_t* state, int32_t* energy, double* gpu_ms)
{
    const int M = p->levels, Lad = p->ladders, H = R.top + 1, n = R.n;
    sk_status status = SK_OK;
    std::vector<uint32_t> mt(2 * M), st((size_t)M * H, 0);
    for (int j = 0; j < M; ++j) {
        mt[2 * j] = accept_threshold(p->beta[j], 1);
        mt[2 * j + 1] = accept_threshold(p->beta[j], 2);
        if (j + 1 < M)
            for (int e = 1; e < H; ++e) st[(size_t)j * H + e] = accept_threshold(p->beta[j + 1] - p->beta[j], e);
    }
    uint32_t *d_mt = nullptr, *d_st = nullptr;
    uint8_t *d_sa = nullptr, *d_sb = nullptr;
    int32_t* d_e = nullptr;
    uint64_t *d_h = nullptr, *d_ma = nullptr, *d_sw = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t nst = (size_t)Lad * M * n, nh = (size_t)Lad * M * H, nl = (size_t)Lad * M;
    const int slot_bytes = (n + H + 3) & ~3;
    const size_t lds = (size_t)64 * slot_bytes + (size_t)M * H * sizeof(uint32_t);
    // iterations per launch; LDS counters stay below 2^32
    const uint64_t seg = (p->segment > 0 && p->segment <= (1ull << 30)) ? p->segment : (1ull << 24);
    float total_ms = 0.f;
    PT_HIP(hipMalloc(&d_mt, mt.size() * sizeof(uint32_t)));
    PT_HIP(hipMalloc(&d_st, st.size() * sizeof(uint32_t)));
    PT_HIP(hipMalloc(&d_sa, nst));
    PT_HIP(hipMalloc(&d_sb, nst));
    PT_HIP(hipMalloc(&d_e, nl * sizeof(int32_t)));
    PT_HIP(hipMalloc(&d_h, nh * sizeof(uint64_t)));
    PT_HIP(hipMalloc(&d_ma, nl * sizeof(uint64_t)));
    PT_HIP(hipMalloc(&d_sw, nl * sizeof(uint64_t)));
    PT_HIP(hipEventCreate(&e0));
    PT_HIP(hipEventCreate(&e1));
    PT_HIP(hipMemcpyAsync(d_mt, mt.data(), mt.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    PT_HIP(hipMemcpyAsync(d_st, st.data(), st.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    PT_HIP(hipMemsetAsync(d_h, 0, nh * sizeof(uint64_t), stream));
    PT_HIP(hipMemsetAsync(d_ma, 0, nl * sizeof(uint64_t), stream));
    PT_HIP(hipMemsetAsync(d_sw, 0, nl * sizeof(uint64_t), stream));
    {
        PtArgs a;
        std::memset(&a, 0, sizeof(a));
        a.n = n;
        a.variant = R.variant;
        a.top = R.top;
        a.levels = M;
        a.pset = R.pset;
        a.slot_bytes = slot_bytes;
        a.seed = p->seed;
        a.move_thr = d_mt;
        a.swap_thr = d_st;
        a.energy_out = d_e;
        a.hist_out = d_h;
        a.move_acc = d_ma;
        a.swap_acc = d_sw;
        uint8_t* cur_in = nullptr;
        uint8_t* cur_out = d_sa;
        for (uint64_t it = 0; it < p->iterations || it == 0; it += seg) {
            a.it_begin = it;
            a.it_end = std::min<uint64_t>(p->iterations, it + seg);
            a.state_in = cur_in;
            a.state_out = cur_out;
            // ladders in groups of at most 65535 blocks
            PT_HIP(hipEventRecord(e0, stream));
            for (int base = 0; base < Lad; base += 65535) {
                a.ladder_base = (uint32_t)base;
                const unsigned cnt = (unsigned)std::min(65535, Lad - base);
                PT_HIP(launch_pt_ladders(cnt, lds, stream, a));
            }
            PT_HIP(hipEventRecord(e1, stream));
            PT_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            PT_HIP(hipEventElapsedTime(&ms, e0, e1));
            total_ms += ms;
            cur_in = cur_out;
            cur_out = (cur_out == d_sa) ? d_sb : d_sa;
            if (p->iterations == 0) break;
        }
        PT_HIP(hipMemcpyAsync(hist, d_h, nh * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
        PT_HIP(hipMemcpyAsync(move_acc, d_ma, nl * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
        PT_HIP(hipMemcpyAsync(swap_acc, d_sw, nl * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
        if (state) PT_HIP(hipMemcpyAsync(state, cur_in, nst, hipMemcpyDeviceToHost, stream));
        if (energy) PT_HIP(hipMemcpyAsync(energy, d_e, nl * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        PT_HIP(hipStreamSynchronize(stream));
    }
    if (gpu_ms) *gpu_ms = total_ms;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void* ptr : {(void*)d_mt, (void*)d_st, (void*)d_sa, (void*)d_sb, (void*)d_e, (void*)d_h, (void*)d_ma,
                      (void*)d_sw})
        if (ptr) (void)hipFree(ptr);
    return status;
}

static sk_status check_params(const Relaxed& R, const sk_pt_params* p)
{
    if (!p || !p->beta || p->levels < 2 || p->levels > kPtMaxLevels || p->ladders < 1) return SK_EINVAL;
    if (p->beta[0] != 0.0) return SK_EINVAL;
    for (int j = 1; j < p->levels; ++j)
        if (!(p->beta[j] > p->beta[j - 1]) || !std::isfinite(p->beta[j])) return SK_EINVAL;
    for (int x : R.L)
        if (x == 0) return SK_EINVAL;  // no configuration at all
    if (p->proposal != SK_PROPOSAL_UNIFORM) return SK_ENOLIB;
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
    double ms = 0;
    s = pt_run_impl(R, p, st, hist.data(), ma.data(), sw.data(), nullptr, nullptr, &ms);
    if (own) (void)hipStreamDestroy(own);
    if (s != SK_OK) return s;

    // Z(0) = prod_k L_k; per ladder: Z(0) prod_j Ratio(j) (Sec. 3), the last
    // ratio taken to beta = infinity (fraction of samples with E = 0).
    double logz0 = 0;
    for (int x : R.L) logz0 += std::log((double)x);
    const bool halve = !(p->flags & SK_ORDERED) && variant != SK_HOOKED && n > 1;
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
    double mean = 0;
    for (double x : est) mean += x;
    mean /= Lad;
    double var = 0;
    for (double x : est) var += (x - mean) * (x - mean);
    const double se = Lad > 1 ? std::sqrt(var / (Lad - 1) / Lad) : 0.0;
    *estimate = mean;
    if (std_error) *std_error = se;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->levels = M;
        stats->ladders = Lad;
        stats->gpu_ms = ms;
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
        }
        stats->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return SK_OK;
}

}  // extern "C"
