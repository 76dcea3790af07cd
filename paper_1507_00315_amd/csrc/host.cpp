// Host side of the exact counting library: instance planning, prime choice,
// launch splitting, residue collection and Chinese-remainder recombination.
// Implements the C ABI declared in include/skolem.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/skolem.h"
#include "sk_internal.h"

namespace sk {

using u128 = unsigned __int128;

using ExactKernelFn = void (*)(const ExactArgs, double*);
ExactKernelFn exact_v1_lookup(int nq, int g);

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;
static thread_local int g_device = 0;
static thread_local sk_stats g_stats;

static sk_status hip_fail(hipError_t e, const char* what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return SK_EDEVICE;
}

#define SK_HIP(call)                                        \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, #call);   \
    } while (0)

// ------------------------------------------------------------------ numbers

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod(r, a, m);
        a = mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin for 64-bit integers (bases: first 12 primes).
static bool is_prime_u64(uint64_t x)
{
    if (x < 2) return false;
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t b : bases) {
        if (x % b == 0) return x == b;
    }
    uint64_t d = x - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (uint64_t b : bases) {
        uint64_t y = powmod(b, d, x);
        if (y == 1 || y == x - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            y = mulmod(y, y, x);
            if (y == x - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

// The first `count` primes below 2^46, skipping the first `skip` of them.
static std::vector<uint64_t> default_primes(int count, int skip)
{
    static std::vector<uint64_t> cache;
    const int need = count + skip;
    uint64_t x = cache.empty() ? ((1ull << 46) - 1) : cache.back() - 2;
    while ((int)cache.size() < need) {
        if (is_prime_u64(x)) cache.push_back(x);
        x -= 2;
    }
    return std::vector<uint64_t>(cache.begin() + skip, cache.begin() + need);
}

// Little-endian multi-word unsigned integer (enough for products of 8 primes).
struct Big {
    uint64_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    void mul_add(uint64_t m, uint64_t a)
    {
        u128 carry = a;
        for (int i = 0; i < 8; ++i) {
            u128 t = (u128)w[i] * m + carry;
            w[i] = (uint64_t)t;
            carry = t >> 64;
        }
    }
    int cmp(const Big& o) const
    {
        for (int i = 7; i >= 0; --i) {
            if (w[i] != o.w[i]) return w[i] < o.w[i] ? -1 : 1;
        }
        return 0;
    }
    bool fits128() const
    {
        for (int i = 2; i < 8; ++i)
            if (w[i]) return false;
        return true;
    }
};

// Garner's algorithm: the x in [0, prod p) with x = r_i mod p_i.
static Big crt(const std::vector<uint64_t>& r, const std::vector<uint64_t>& p)
{
    const size_t k = p.size();
    std::vector<uint64_t> a(k);  // mixed-radix digits
    for (size_t i = 0; i < k; ++i) {
        // x_i = (r_i - (a_0 + a_1 p_0 + ... )) / (p_0...p_{i-1}) mod p_i
        uint64_t v = r[i] % p[i];
        uint64_t prodm = 1 % p[i];
        uint64_t acc = 0;
        for (size_t j = 0; j < i; ++j) {
            acc = (uint64_t)(((u128)acc + mulmod(a[j] % p[i], prodm, p[i])) % p[i]);
            prodm = mulmod(prodm, p[j] % p[i], p[i]);
        }
        uint64_t diff = (v + p[i] - acc) % p[i];
        a[i] = mulmod(diff, powmod(prodm, p[i] - 2, p[i]), p[i]);
    }
    Big x;
    for (size_t i = k; i-- > 0;) {
        x.mul_add(p[i], a[i]);  // Horner: x = x * p_i + a_i
    }
    return x;
}

static Big factorial_big(int n)
{
    Big f;
    f.w[0] = 1;
    for (int i = 2; i <= n; ++i) f.mul_add((uint64_t)i, 0);
    return f;
}

// ------------------------------------------------------------------ planning

struct Plan {
    int n = 0, variant = 0, m = 0;
    int pos[kMaxVars];
    int d[kMaxN];
    uint64_t pset = 0;
    int n_lane = 0, n_walk = 0, n_job = 0;
    int nq = 0, G = 0;
    int halved = 0;          // number of factors stored as f_k / 2
    SlotDesc slot[kMaxSlots];
    bool zero_factor = false;  // some f_k is identically 0 (no pairs at that distance)
};

static bool existence(int n, int v)
{
    int r = n % 4;
    if (v == SK_SKOLEM) return r == 0 || r == 1;
    if (v == SK_LANGFORD) return r == 0 || r == 3;
    return r == 2 || r == 3;
}

static int max_walk_bits(const Plan& P, int walk_cap)
{
    // Walked variables (ranks 1..w) must share no pair with a lane variable:
    // pos[w] + d_max < pos[m - n_lane].  Later kernels rely on it.
    const int dmax = P.d[P.n - 1];
    int w = 0;
    while (w + 1 <= P.m - 1 - P.n_lane && w + 1 <= walk_cap &&
           P.pos[w + 1] + dmax < P.pos[P.m - P.n_lane])
        ++w;
    return w;
}

static sk_status make_plan(int n, int variant, Plan& P, int walk_cap = 20)
{
    if (variant < 0 || variant > 2) return SK_EINVAL;
    if (n < 1 || n > kMaxN || (variant == SK_HOOKED && n > kMaxN - 1)) return SK_EINVAL;
    P.n = n;
    P.variant = variant;
    const int top = variant == SK_HOOKED ? 2 * n + 1 : 2 * n;
    P.m = 0;
    for (int p = 1; p <= top; ++p) {
        if (variant == SK_HOOKED && p == 2 * n) continue;
        P.pos[P.m++] = p;
        P.pset |= 1ull << (p - 1);
    }
    for (int k = 1; k <= n; ++k) P.d[k - 1] = variant == SK_LANGFORD ? k + 1 : k;
    P.n_lane = std::min(kLaneBits, P.m - 1);
    P.n_walk = max_walk_bits(P, walk_cap);
    P.n_job = P.m - 1 - P.n_lane - P.n_walk;

    // Factor descriptors and bounds.
    struct Fac { int k; uint64_t mask; int len, halve; uint64_t bound; };
    std::vector<Fac> fac;
    for (int k = 0; k < n; ++k) {
        Fac f{};
        f.k = k;
        for (int p = 1; p + P.d[k] <= top; ++p) {
            if (((P.pset >> (p - 1)) & 1) && ((P.pset >> (p + P.d[k] - 1)) & 1)) {
                f.mask |= 1ull << (p - 1);
                ++f.len;
            }
        }
        f.halve = (f.len % 2 == 0 && f.len > 0) ? 1 : 0;
        f.bound = (uint64_t)(f.len >> f.halve);
        if (f.len == 0) P.zero_factor = true;
        fac.push_back(f);
    }
    P.halved = 0;
    for (auto& f : fac) P.halved += f.halve;

    // Group factors: quads of 4 slots, G groups of consecutive quads.  Try the
    // smallest G whose exactness bounds hold; factors placed greedily (largest
    // bound first into the group with the smallest product so far).
    P.nq = (n + 3) / 4;
    std::vector<Fac> order = fac;
    std::sort(order.begin(), order.end(), [](const Fac& a, const Fac& b) { return a.bound > b.bound; });
    for (int G = 1; G <= std::min(4, P.nq); ++G) {
        std::vector<std::vector<Fac>> grp(G);
        std::vector<double> lg(G, 0.0);
        std::vector<int> cap(G);
        for (int g = 0; g < G; ++g) cap[g] = 4 * (quad_begin(P.nq, G, g + 1) - quad_begin(P.nq, G, g));
        bool ok = true;
        for (auto& f : order) {
            int best = -1;
            for (int g = 0; g < G; ++g) {
                if ((int)grp[g].size() < cap[g] && (best < 0 || lg[g] < lg[best])) best = g;
            }
            if (best < 0) { ok = false; break; }
            grp[best].push_back(f);
            lg[best] += std::log2((double)std::max<uint64_t>(f.bound, 1));
        }
        if (!ok) continue;
        // exact bound checks
        std::vector<u128> gb(G, 1);
        for (int g = 0; g < G; ++g)
            for (auto& f : grp[g]) gb[g] *= std::max<uint64_t>(f.bound, 1);
        const u128 two53 = (u128)1 << 53, two50 = (u128)1 << 50, two96 = (u128)1 << 96;
        for (int g = 0; g < G; ++g) {
            if (gb[g] >= two53) ok = false;
            if (g >= 2 && gb[g] >= two50) ok = false;
        }
        if (ok && G >= 2) {
            // gb[0] * gb[1] < 2^96, computed without overflow
            const u128 a = gb[0], b = gb[1];
            if (a != 0 && b > two96 / a) ok = false;
        }
        if (!ok) continue;
        P.G = G;
        int s = 0;
        for (int g = 0; g < G; ++g) {
            const int end = 4 * quad_begin(P.nq, G, g + 1);
            for (auto& f : grp[g]) {
                P.slot[s].mask = f.mask;
                P.slot[s].d = P.d[f.k];
                P.slot[s].len = f.len;
                P.slot[s].halve = f.halve;
                P.slot[s].pad = f.k;
                ++s;
            }
            for (; s < end; ++s) P.slot[s] = SlotDesc{0, 0, 1, 0, -1};
        }
        return SK_OK;
    }
    return SK_ENOLIB;
}


// ------------------------------------------------------------------ device

struct DeviceCtx {
    bool ready = false;
    hipStream_t stream = nullptr;
    int cus = 0;
};

static DeviceCtx g_ctx[64];

static sk_status device_ctx(DeviceCtx** out)
{
    if (g_device < 0 || g_device >= 64) return SK_EINVAL;
    DeviceCtx& c = g_ctx[g_device];
    SK_HIP(hipSetDevice(g_device));
    if (!c.ready) {
        hipDeviceProp_t prop;
        SK_HIP(hipGetDeviceProperties(&prop, g_device));
        c.cus = prop.multiProcessorCount;
        SK_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
        c.ready = true;
    }
    *out = &c;
    return SK_OK;
}

static uint64_t fp_to_residue(double v, uint64_t p)
{
    const int64_t x = (int64_t)v;  // exact: |v| < 2^53 and integral
    int64_t r = x % (int64_t)p;
    if (r < 0) r += (int64_t)p;
    return (uint64_t)r;
}

struct SumRequest {
    const Plan* plan = nullptr;
    std::vector<uint64_t> primes;
    int log2_chunk_terms = 0;  // 0: default
    int waves_per_launch = 0;
    // listed-chunk mode
    const uint64_t* chunk_ids = nullptr;
    size_t nchunks = 0;
    int chunk_bits = -1;
    hipStream_t stream = nullptr;
    sk_progress_fn progress = nullptr;
    void* progress_ctx = nullptr;
};

// Runs the kernel over the requested chunks.  Total mode: out has one residue
// per prime (sum over all chunks).  Listed mode: out has nchunks x nprimes.
// Residues are of the kernel's sum (factors with even L_k stored halved).
static sk_status run_sum(const SumRequest& R, std::vector<uint64_t>& out, sk_stats& st)
{
    const Plan& P = *R.plan;
    const int np = (int)R.primes.size();
    if (np < 1 || np > kMaxPrimes) return SK_EINVAL;
    for (uint64_t p : R.primes) {
        if ((double)p <= kPrimeLo || (double)p >= kPrimeHi || !(p & 1)) return SK_EINVAL;
    }
    ExactKernelFn fn = exact_v1_lookup(P.nq, P.G);
    if (!fn) return SK_ENOLIB;

    ExactArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int s = 0; s < kMaxSlots; ++s) a.slot[s] = (s < 4 * P.nq) ? P.slot[s] : SlotDesc{0, 0, 1, 0, -1};
    for (int i = 0; i < P.m; ++i) a.var_pos[i] = P.pos[i];
    for (int i = 0; i < np; ++i) {
        a.prime[i] = (double)R.primes[i];
        a.pinv[i] = 1.0 / (double)R.primes[i];
    }
    a.nprimes = np;
    a.m = P.m;
    a.n_lane = P.n_lane;
    a.n_walk = P.n_walk;
    a.n_job = P.n_job;
    a.lane_valid_bits = P.n_lane;

    const bool listed = R.chunk_ids != nullptr;
    int jb;
    uint64_t nchunks;
    if (listed) {
        if (R.chunk_bits < 0 || R.chunk_bits > P.n_job) return SK_EINVAL;
        jb = P.n_job - R.chunk_bits;
        nchunks = R.nchunks;
        for (size_t i = 0; i < R.nchunks; ++i) {
            if (R.chunk_bits < 64 && (R.chunk_ids[i] >> R.chunk_bits) != 0) return SK_EINVAL;
        }
    } else {
        // Default chunk: enough chunks to give every SIMD many waves (2^14
        // chunks), at most 2^31 sign vectors per chunk.
        const int log2_terms = R.log2_chunk_terms > 0
                                   ? R.log2_chunk_terms
                                   : std::min(31, P.n_lane + P.n_walk + std::max(0, P.n_job - 14));
        jb = log2_terms - P.n_lane - P.n_walk;
        jb = std::max(0, std::min(jb, P.n_job));
        nchunks = 1ull << (P.n_job - jb);
    }
    a.job_bits_per_chunk = jb;
    const uint64_t terms_per_chunk = 1ull << (P.n_lane + P.n_walk + jb);
    const uint64_t terms_total = nchunks * terms_per_chunk;

    DeviceCtx* ctx;
    sk_status stt = device_ctx(&ctx);
    if (stt != SK_OK) return stt;
    hipStream_t stream = R.stream ? R.stream : ctx->stream;

    uint64_t wpl = R.waves_per_launch > 0 ? (uint64_t)R.waves_per_launch : (uint64_t)ctx->cus * 4 * 8;
    wpl = std::min<uint64_t>(wpl, nchunks);

    double* d_out = nullptr;
    uint64_t* d_ids = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<double> h_out(wpl * np);
    sk_status status = SK_OK;
    auto fail = [&](hipError_t e, const char* what) {
        status = hip_fail(e, what);
    };
    hipError_t e;
    if ((e = hipMalloc(&d_out, wpl * np * sizeof(double))) != hipSuccess) { fail(e, "hipMalloc"); goto done; }
    if (listed) {
        if ((e = hipMalloc(&d_ids, wpl * sizeof(uint64_t))) != hipSuccess) { fail(e, "hipMalloc"); goto done; }
    }
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        fail(e, "hipEventCreate");
        goto done;
    }
    if (listed) out.assign(nchunks * np, 0);
    else out.assign(np, 0);

    for (uint64_t base = 0; base < nchunks; base += wpl) {
        const uint64_t nw = std::min<uint64_t>(wpl, nchunks - base);
        a.n_waves = nw;
        a.chunk_base = base;
        a.chunk_ids = nullptr;
        if (listed) {
            if ((e = hipMemcpyAsync(d_ids, R.chunk_ids + base, nw * sizeof(uint64_t), hipMemcpyHostToDevice,
                                    stream)) != hipSuccess) { fail(e, "hipMemcpyAsync"); goto done; }
            a.chunk_ids = d_ids;
        }
        const unsigned blocks = (unsigned)((nw + 3) / 4);
        if ((e = hipEventRecord(e0, stream)) != hipSuccess) { fail(e, "hipEventRecord"); goto done; }
        hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), 0, stream, a, d_out);
        if ((e = hipGetLastError()) != hipSuccess) { fail(e, "kernel launch"); goto done; }
        if ((e = hipEventRecord(e1, stream)) != hipSuccess) { fail(e, "hipEventRecord"); goto done; }
        if ((e = hipMemcpyAsync(h_out.data(), d_out, nw * np * sizeof(double), hipMemcpyDeviceToHost,
                                stream)) != hipSuccess) { fail(e, "hipMemcpyAsync"); goto done; }
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) { fail(e, "hipStreamSynchronize"); goto done; }
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { fail(e, "hipEventElapsedTime"); goto done; }
        st.kernel_ms += ms;
        st.launches += 1;
        for (uint64_t w = 0; w < nw; ++w) {
            for (int i = 0; i < np; ++i) {
                const uint64_t r = fp_to_residue(h_out[w * np + i], R.primes[i]);
                if (listed) out[(base + w) * np + i] = r;
                else out[i] = (uint64_t)(((u128)out[i] + r) % R.primes[i]);
            }
        }
        if (R.progress && R.progress(R.progress_ctx, (base + nw) * terms_per_chunk, terms_total)) {
            status = SK_EABORTED;
            goto done;
        }
    }
    st.terms += terms_total;
    st.chunks += nchunks;
    st.log2_chunk_terms = P.n_lane + P.n_walk + jb;
    st.kernel_variant = 1;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d_out) (void)hipFree(d_out);
    if (d_ids) (void)hipFree(d_ids);
    return status;
}

static int primes_needed(int n)
{
    // C <= n! (the leftmost uncovered position always starts a new pair, so a
    // pairing is fixed by a sequence of distinct labels); want prod p > n! 2^8
    // with every prime above 2^45.
    double bits = 8.0;
    for (int i = 2; i <= n; ++i) bits += std::log2((double)i);
    int k = (int)std::ceil(bits / 45.0);
    return std::max(1, std::min(k, kMaxPrimes));
}

static uint64_t inv_pow2_scaled(uint64_t h, int e, uint64_t p)
{
    // h * 2^{-e} mod p
    const uint64_t inv2 = (p + 1) / 2;
    return mulmod(h, powmod(inv2, (uint64_t)e, p), p);
}

}  // namespace sk

using namespace sk;

extern "C" {

sk_status sk_set_device(int device)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return SK_EDEVICE;
    if (device < 0 || device >= count) return SK_EINVAL;
    g_device = device;
    return SK_OK;
}

static sk_status count_impl(int n, int variant, unsigned flags, const sk_tuning* tune, void* stream,
                            sk_progress_fn progress, void* pctx, sk_stats* stats_out, sk_u128* out)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!out) return SK_EINVAL;
    Plan P;
    sk_status s = make_plan(n, variant, P);
    if (s != SK_OK) return s;
    sk_stats st;
    std::memset(&st, 0, sizeof(st));
    u128 result = 0;
    if (!existence(n, variant) && !(flags & SK_NO_SHORTCUT)) {
        result = 0;
    } else {
        const int np = (tune && tune->primes > 0) ? std::max(primes_needed(n), std::min(tune->primes, kMaxPrimes)) : primes_needed(n);
        const int passes = (flags & SK_VERIFY) ? 2 : 1;
        Big first;
        for (int pass = 0; pass < passes; ++pass) {
            SumRequest R;
            R.plan = &P;
            R.primes = default_primes(np, pass * np);
            R.log2_chunk_terms = (tune && tune->log2_chunk_terms > 0) ? tune->log2_chunk_terms : 0;
            R.waves_per_launch = tune ? tune->waves_per_launch : 0;
            R.stream = (hipStream_t)stream;
            R.progress = progress;
            R.progress_ctx = pctx;
            std::vector<uint64_t> res;
            s = run_sum(R, res, st);
            if (s != SK_OK) return s;
            // C = H / 2^{m-1} with H = 2^{halved} * (kernel sum)
            for (int i = 0; i < np; ++i) res[i] = inv_pow2_scaled(res[i], P.m - 1 - P.halved, R.primes[i]);
            Big c = crt(res, R.primes);
            if (c.cmp(factorial_big(n)) > 0 || !c.fits128()) {
                g_last_error = "CRT result exceeds the bound n!";
                return SK_ECHECK;
            }
            if (pass == 0) first = c;
            else if (c.cmp(first) != 0) {
                g_last_error = "verification pass with disjoint primes disagrees";
                return SK_ECHECK;
            }
            for (int i = 0; i < np; ++i) st.primes[pass * np + i] = R.primes[i];
        }
        st.nprimes = np;
        st.passes = passes;
        result = ((u128)first.w[1] << 64) | first.w[0];
    }
    if (!(flags & SK_ORDERED) && variant != SK_HOOKED && n > 1) {
        if (result & 1) {
            g_last_error = "ordered count is odd; reflections must pair up";
            return SK_ECHECK;
        }
        result >>= 1;
    }
    out->lo = (uint64_t)result;
    out->hi = (uint64_t)(result >> 64);
    st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st.ms_per_launch_avg = st.launches ? st.kernel_ms / (double)st.launches : 0.0;
    g_stats = st;
    if (stats_out) *stats_out = st;
    return SK_OK;
}

sk_status sk_count(int n, int variant, unsigned flags, sk_u128* out)
{
    return count_impl(n, variant, flags, nullptr, nullptr, nullptr, nullptr, nullptr, out);
}

sk_status sk_count_ex(int n, int variant, unsigned flags, const sk_tuning* tune, void* stream,
                      sk_progress_fn progress, void* progress_ctx, sk_stats* stats, sk_u128* out)
{
    return count_impl(n, variant, flags, tune, stream, progress, progress_ctx, stats, out);
}

sk_status sk_sign_sum_residues(int n, int variant, const uint64_t* primes, int nprimes,
                               const sk_tuning* tune, void* stream, uint64_t* residues)
{
    if (!primes || !residues || nprimes < 1 || nprimes > kMaxPrimes) return SK_EINVAL;
    Plan P;
    sk_status s = make_plan(n, variant, P);
    if (s != SK_OK) return s;
    SumRequest R;
    R.plan = &P;
    R.primes.assign(primes, primes + nprimes);
    R.log2_chunk_terms = (tune && tune->log2_chunk_terms > 0) ? tune->log2_chunk_terms : 0;
    R.waves_per_launch = tune ? tune->waves_per_launch : 0;
    R.stream = (hipStream_t)stream;
    std::vector<uint64_t> res;
    sk_stats st;
    std::memset(&st, 0, sizeof(st));
    s = run_sum(R, res, st);
    if (s != SK_OK) return s;
    for (int i = 0; i < nprimes; ++i) residues[i] = mulmod(res[i], powmod(2, (uint64_t)P.halved, primes[i]), primes[i]);
    g_stats = st;
    return SK_OK;
}

int sk_max_chunk_bits(int n, int variant)
{
    Plan P;
    if (make_plan(n, variant, P) != SK_OK) return -1;
    return P.n_job;
}

sk_status sk_describe(int n, int variant, sk_plan_desc* out)
{
    if (!out) return SK_EINVAL;
    Plan P;
    sk_status s = make_plan(n, variant, P);
    if (s != SK_OK) return s;
    out->m = P.m;
    out->n_lane = P.n_lane;
    out->n_walk = P.n_walk;
    out->n_job = P.n_job;
    out->quads = P.nq;
    out->groups = P.G;
    out->halved = P.halved;
    out->primes = primes_needed(n);
    for (int i = 0; i < 32; ++i) out->slot_factor[i] = (i < 4 * P.nq) ? P.slot[i].pad : -1;
    return SK_OK;
}

sk_status sk_partial_chunks(int n, int variant, int log2_chunks, const uint64_t* chunk_ids, size_t nchunks,
                            const uint64_t* primes, int nprimes, void* stream, uint64_t* residues_out)
{
    if (!chunk_ids || !primes || !residues_out || nprimes < 1 || nprimes > kMaxPrimes) return SK_EINVAL;
    Plan P;
    sk_status s = make_plan(n, variant, P);
    if (s != SK_OK) return s;
    if (log2_chunks < 0 || log2_chunks > P.n_job) return SK_EINVAL;
    if (nchunks == 0) return SK_OK;
    SumRequest R;
    R.plan = &P;
    R.primes.assign(primes, primes + nprimes);
    R.chunk_ids = chunk_ids;
    R.nchunks = nchunks;
    R.chunk_bits = log2_chunks;
    R.stream = (hipStream_t)stream;
    std::vector<uint64_t> res;
    sk_stats st;
    std::memset(&st, 0, sizeof(st));
    s = run_sum(R, res, st);
    if (s != SK_OK) return s;
    for (size_t c = 0; c < nchunks; ++c)
        for (int i = 0; i < nprimes; ++i)
            residues_out[c * nprimes + i] =
                mulmod(res[c * nprimes + i], powmod(2, (uint64_t)P.halved, primes[i]), primes[i]);
    g_stats = st;
    return SK_OK;
}

const char* sk_strerror(sk_status s)
{
    switch (s) {
        case SK_OK: return "ok";
        case SK_EINVAL: return "invalid argument";
        case SK_ERANGE: return "primes do not cover the result range";
        case SK_EDEVICE: return "HIP device error";
        case SK_ECHECK: return "self-check failed";
        case SK_ENOMEM: return "out of memory";
        case SK_EABORTED: return "aborted by progress callback";
        case SK_ENOLIB: return "no kernel built for this instance shape";
    }
    return "unknown status";
}

const char* sk_last_error(void) { return g_last_error.c_str(); }

int sk_u128_to_decimal(sk_u128 x, char* buf, size_t len)
{
    u128 v = ((u128)x.hi << 64) | x.lo;
    char tmp[48];
    int k = 0;
    do {
        tmp[k++] = (char)('0' + (int)(v % 10));
        v /= 10;
    } while (v);
    if ((size_t)k + 1 > len || !buf) return -1;
    for (int i = 0; i < k; ++i) buf[i] = tmp[k - 1 - i];
    buf[k] = 0;
    return k;
}

const char* sk_kernel_name(int kernel_variant)
{
    switch (kernel_variant) {
        case 1: return "exact_v1_kernel";
        case 2: return "exact_v2_kernel";
    }
    return "none";
}

}  // extern "C"
