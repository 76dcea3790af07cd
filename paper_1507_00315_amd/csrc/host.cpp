// Host side of the exact counting library: instance planning, prime choice,
// launch splitting, residue collection and Chinese-remainder recombination.
// Implements the C ABI declared in include/skolem.h.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/skolem.h"
#include "sk_internal.h"
#include "sk_plan.h"
#include "sk_batch.h"

namespace sk {

using u128 = unsigned __int128;

using ExactKernelFn = void (*)(const ExactArgs, double*);
ExactKernelFn exact_v1_lookup(int nq, int g);

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;
static thread_local int g_device = 0;
static thread_local sk_stats g_stats;

const char* set_last_error(const std::string& msg)
{
    g_last_error = msg;
    return g_last_error.c_str();
}

int current_device() { return g_device; }

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
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
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
    int qb[5] = {};          // product group g covers quads [qb[g], qb[g+1])
    int halved = 0;          // number of factors stored as f_k / 2
    SlotDesc slot[kMaxSlots];
    bool zero_factor = false;  // some f_k is identically 0 (no pairs at that distance)
    bool larsen = false;       // plan of the inclusion-exclusion sum (nothing halved)
};

static bool existence(int n, int v)
{
    int r = n % 4;
    if (v == SK_SKOLEM) return r == 0 || r == 1;
    if (v == SK_LANGFORD) return r == 0 || r == 3;
    return r == 2 || r == 3;
}

// Lemma 2.4 generalised to every variant: negating the sign variables at even
// positions multiplies prod x by (-1)^(even positions in P) and f_k by -1 when
// d_k is odd (exactly one end of each pair is even), by +1 when d_k is even.
// The term is invariant when the total exponent is even -- for Skolem,
// Langford and hooked pairings exactly the existence conditions of Sec. 1.1.
static bool hat_symmetric(const Plan& P)
{
    int e = 0;
    for (int i = 0; i < P.m; ++i) e += (P.pos[i] % 2 == 0);
    for (int k = 0; k < P.n; ++k) e += (P.d[k] % 2 == 1);
    return e % 2 == 0;
}

// Reversal quadruples (Lemma 2.3; see RevMasks): odd positions j whose mirror
// 2n+1-j is also a job variable, the highest job variable (the one the Lemma
// 2.4 half fixes) excluded, taken nearest the middle first, two per quadruple.
// Skolem and Langford only (the hooked position set is not symmetric).
static RevMasks reversal_masks(const Plan& P)
{
    RevMasks rv;
    std::memset(&rv, 0, sizeof(rv));
    if (P.variant == SK_HOOKED) return rv;
    const int lo = P.n_walk + 1, hi = P.n_walk + P.n_job;  // job ranks
    const int top = 2 * P.n;                                // positions 1..2n, rank = position - 1
    std::vector<int> js;
    for (int rank = lo; rank < hi; ++rank) {
        const int j = P.pos[rank];
        const int jm = top + 1 - j;
        if (j % 2 == 0) continue;  // each mirror pair has exactly one odd member
        const int rm = jm - 1;
        if (rm < lo || rm >= hi) continue;
        js.push_back(j);
    }
    std::sort(js.begin(), js.end(), [&](int a, int b) { return std::abs(2 * a - top - 1) < std::abs(2 * b - top - 1); });
    rv.r = std::min<int>(kRevMax, (int)js.size() / 2);
    for (int q = 0; q < rv.r; ++q) {
        const int j1 = js[2 * q], j2 = js[2 * q + 1];
        rv.u[q] = (1ull << (j1 - 1)) | (1ull << (j2 - 1));
        rv.v[q] = (1ull << (top - j1)) | (1ull << (top - j2));
    }
    return rv;
}

// Sign vectors evaluated out of `total` when r reversal quadruples are in use:
// weight-0 jobs are 1/4 + 1/8 + ... + 1/2^(r+1) of all jobs.
static uint64_t reversal_evaluated(uint64_t total, int r)
{
    return r == 0 ? total : (total >> (r + 1)) * ((1ull << r) + 1);
}

static sk_status make_plan(int n, int variant, Plan& P, bool larsen = false)
{
    if (variant < 0 || variant > 2) return SK_EINVAL;
    if (n < 1 || n > kMaxN || (variant == SK_HOOKED && n > kMaxN - 1)) return SK_EINVAL;
    const PlanCE C = make_plan_ce(n, variant, kWalkCap, larsen);
    P.larsen = larsen;
    if (!C.ok) return SK_ENOLIB;
    P.n = C.n;
    P.variant = C.variant;
    P.m = C.m;
    for (int i = 0; i < C.m; ++i) P.pos[i] = C.pos[i];
    for (int k = 0; k < n; ++k) P.d[k] = C.d[k];
    P.pset = C.pset;
    P.n_lane = C.n_lane;
    P.n_walk = C.n_walk;
    P.n_job = C.n_job;
    P.nq = C.nq;
    P.G = C.G;
    for (int g = 0; g < 5; ++g) P.qb[g] = C.qb[g];
    P.halved = C.halved;
    P.zero_factor = false;
    for (int s = 0; s < kMaxSlots; ++s) {
        if (s < 4 * C.nq && C.slot_k[s] >= 0) {
            P.slot[s] = SlotDesc{C.slot_mask[s], C.slot_d[s], C.slot_len[s], C.slot_halve[s], C.slot_k[s]};
            if (C.slot_len[s] == 0) P.zero_factor = true;
        } else {
            P.slot[s] = SlotDesc{0, 0, 1, 0, -1};
        }
    }
    return SK_OK;
}

// ------------------------------------------------------------------ device

// Fixed device workspace of sk_count_batch_noalloc, for callers that cannot
// allocate: every GPU the library runs on holds its own copy until the
// process ends.  In host code this name is only a handle for
// hipGetSymbolAddress; the device address is DeviceCtx::scratch.
constexpr size_t kScratchBytes = 4096;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceCtx {
    bool ready = false;
    hipStream_t stream = nullptr;
    int cus = 0;
    void* scratch = nullptr;  // this device's copy of `scratch`
};

static DeviceCtx g_ctx[64];
static std::mutex g_ctx_mu;

// Per-device set-up, once per device with that device current: the library's
// stream, the CU count and the address of the fixed workspace.
static sk_status device_ctx(DeviceCtx** out)
{
    if (g_device < 0 || g_device >= 64) return SK_EINVAL;
    DeviceCtx& c = g_ctx[g_device];
    SK_HIP(hipSetDevice(g_device));
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if (!c.ready) {
        hipDeviceProp_t prop;
        SK_HIP(hipGetDeviceProperties(&prop, g_device));
        c.cus = prop.multiProcessorCount;
        void* addr = nullptr;
        SK_HIP(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)));
        c.scratch = addr;
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
    int kernel = 0;  // 0 best, 1 reference, 2 tuned
    sk_progress_fn progress = nullptr;
    void* progress_ctx = nullptr;
    // total mode: evaluate only the chunks whose highest chunk variable (an
    // even position) is +1, and double (valid when hat_symmetric)
    bool half = false;
    // total mode, tuned kernel: reversal weights (Lemma 2.3)
    bool reverse = false;
    // total mode: only the part-th of `parts` equal, consecutive ranges of
    // chunk indices (parts a power of two not above the chunk count)
    uint64_t part = 0, parts = 1;
    // device workspace (nullptr: allocated and freed inside the call)
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // time the launches with HIP events (kernel_ms); off in the call that
    // allocates nothing
    bool timing = true;
};

// Device workspace of run_sum: the accumulators of a total (kAccSlots
// (low word, carries) pairs), the work-queue counter of a launch, then, for
// listed chunks, one row of up to kMaxPrimes 128-bit sums (the reference
// kernel: fp64 residues) and one chunk id per chunk of a launch.
constexpr size_t kSumAccBytes = (size_t)kAccSlots * 2 * sizeof(unsigned long long);
constexpr size_t kSumWsBytes = kSumAccBytes + 256;

static size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t sum_ws_bytes(bool listed, uint64_t chunks_per_launch)
{
    if (!listed) return kSumWsBytes;
    return kSumWsBytes + round256(chunks_per_launch * kMaxPrimes * 2 * sizeof(unsigned long long)) +
           round256(chunks_per_launch * sizeof(uint64_t));
}

// Work items of the tuned kernel: at least 2^kItemLog2Steps Gray-code steps
// per lane (the claim of an item is one atomic round trip), otherwise as small
// as possible, so that the queue drains evenly.
constexpr int kItemLog2Steps = 14;

hipError_t launch_zero_words(void* p, uint64_t n, hipStream_t stream);

// ------------------------------------------------------------------ kernels

using ExactV2Fn = void (*)(const ExactArgsV2);

struct V2Entry {
    ExactV2Fn fn = nullptr;
    int nprimes = 0;
    int inner = 0;
};

static V2Entry& v2_slot(int variant, int n, bool larsen = false)
{
    static V2Entry table[2][3][kMaxN + 1];
    return table[larsen ? 1 : 0][variant][n];
}

int register_exact_v2(int variant, int n, int nprimes, int inner, bool larsen, ExactV2Fn fn)
{
    if (variant < 0 || variant > 2 || n < 1 || n > kMaxN) return 0;
    V2Entry& e = v2_slot(variant, n, larsen);
    e.fn = fn;
    e.nprimes = nprimes;
    e.inner = inner;
    return 1;
}

// Kernel body used for (plan, requested kernel): 2 = tuned (when built for
// this instance), 1 = reference.
static int pick_kernel(const Plan& P, int requested)
{
    if (requested == 1) return 1;
    if (v2_slot(P.variant, P.n, P.larsen).fn) return 2;
    return requested == 2 ? -1 : 1;
}

// Runs the kernel over the requested chunks.  Total mode: out has one residue
// per prime (sum over all chunks).  Listed mode: out has nchunks x nprimes.
// Residues are of the kernel's sum (factors with even L_k stored halved).
static sk_status run_sum(const SumRequest& R, std::vector<uint64_t>& out, sk_stats& st)
{
    const Plan& P = *R.plan;
    const int np = (int)R.primes.size();
    if (np < 1 || np > 2 * kMaxPrimes) return SK_EINVAL;
    for (uint64_t p : R.primes) {
        if ((double)p <= kPrimeLo || (double)p >= kPrimeHi || !(p & 1)) return SK_EINVAL;
    }
    const int kv = pick_kernel(P, R.kernel);
    if (kv < 0) return SK_ENOLIB;
    ExactKernelFn fn1 = nullptr;
    ExactV2Fn fn2 = nullptr;
    int batch = 0;  // primes per launch
    if (kv == 2) {
        fn2 = v2_slot(P.variant, P.n, P.larsen).fn;
        batch = v2_slot(P.variant, P.n, P.larsen).nprimes;
    } else {
        fn1 = exact_v1_lookup(P.nq, P.G);
        if (!fn1) return SK_ENOLIB;
        batch = std::min(np, kMaxPrimes);
    }

    const bool listed = R.chunk_ids != nullptr;
    if (P.larsen && (listed || R.half || R.reverse)) return SK_EINVAL;
    // the inclusion-exclusion sum leaves position 1 free: both of its values
    const int x0_passes = P.larsen ? 2 : 1;
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
    const bool half = !listed && R.half && nchunks >= 2;
    if (half) nchunks >>= 1;
    uint64_t chunk_offset = 0;
    if (!listed && R.parts > 1) {
        if ((R.parts & (R.parts - 1)) != 0 || R.part >= R.parts || R.parts > nchunks) {
            g_last_error = "parts must be a power of two not above the number of chunks (" +
                           std::to_string(nchunks) + "), part < parts";
            return SK_EINVAL;
        }
        nchunks /= R.parts;
        chunk_offset = R.part * nchunks;
    }
    const RevMasks rev = (!listed && R.reverse && kv == 2) ? reversal_masks(P) : RevMasks{};
    const int rev_r = rev.r;
    const uint64_t terms_per_chunk = 1ull << (P.n_lane + P.n_walk + jb);
    const int nbatches = (np + batch - 1) / batch;
    const uint64_t terms_total = nchunks * terms_per_chunk * (uint64_t)nbatches * x0_passes;

    DeviceCtx* ctx;
    sk_status stt = device_ctx(&ctx);
    if (stt != SK_OK) return stt;
    hipStream_t stream = R.stream ? R.stream : ctx->stream;

    // chunks per launch (the reference kernel: one wave each)
    uint64_t wpl = R.waves_per_launch > 0 ? (uint64_t)R.waves_per_launch : (uint64_t)ctx->cus * 4 * 8;
    wpl = std::min<uint64_t>(wpl, nchunks);
    // jobs per work item of the tuned kernel, 2^item_bits (kItemLog2Steps);
    // a launch's items are counted in 32 bits
    int item_bits = std::max(0, std::min(jb, kItemLog2Steps - P.n_walk));
    {
        int lw = 0;
        while ((1ull << lw) < wpl) ++lw;
        while (item_bits < jb && lw + (jb - item_bits) > 31) ++item_bits;
    }
    if (np > kAccSlots || (uint64_t)nbatches * batch > (uint64_t)kAccSlots) return SK_EINVAL;

    const size_t need = sum_ws_bytes(listed, wpl);
    unsigned char* ws = (unsigned char*)R.ws;
    bool own_ws = false;
    unsigned long long* d_acc = nullptr;
    uint32_t* d_counter = nullptr;
    double* d_out = nullptr;              // listed rows of the reference kernel
    unsigned long long* d_rows = nullptr; // listed rows of the tuned kernel (same memory)
    uint64_t* d_ids = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<double> h_out(listed && kv == 1 ? wpl * batch : 0);
    std::vector<unsigned long long> h_rows(listed && kv == 2 ? wpl * batch * 2 : 0);
    std::vector<unsigned long long> h_acc((size_t)2 * nbatches * batch);
    sk_status status = SK_OK;
    hipError_t e;
    uint64_t terms_done = 0;
    auto t_host = std::chrono::steady_clock::now();
    auto fail = [&](hipError_t err, const char* what) { status = hip_fail(err, what); };
    if (ws && R.ws_bytes < need) {
        g_last_error = "workspace of " + std::to_string(R.ws_bytes) + " bytes, " + std::to_string(need) + " needed";
        return SK_ENOMEM;
    }
    if (!ws) {
        if ((e = hipMalloc(&ws, need)) != hipSuccess) { fail(e, "hipMalloc"); goto done; }
        own_ws = true;
    }
    d_acc = (unsigned long long*)ws;
    d_counter = (uint32_t*)(ws + kSumAccBytes);
    if (listed) {
        d_out = (double*)(ws + kSumWsBytes);
        d_rows = (unsigned long long*)(ws + kSumWsBytes);
        d_ids = (uint64_t*)(ws + kSumWsBytes + round256(wpl * kMaxPrimes * 2 * sizeof(unsigned long long)));
    } else if ((e = launch_zero_words(d_acc, 2 * (uint64_t)nbatches * batch, stream)) != hipSuccess) {
        fail(e, "zero accumulators");
        goto done;
    }
    if (R.timing) {
        if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
            fail(e, "hipEventCreate");
            goto done;
        }
    }
    if (listed) out.assign(nchunks * np, 0);
    else out.assign(np, 0);

    for (int pass = 0; pass < nbatches * x0_passes; ++pass) {
        const int bt = pass % nbatches;
        const uint64_t x_extra = pass / nbatches;  // position 1 (bit 0) occupied in the second pass
        // primes of this launch batch; the last batch repeats its last prime
        std::vector<uint64_t> bp(batch);
        for (int i = 0; i < batch; ++i) bp[i] = R.primes[std::min(np - 1, bt * batch + i)];
        const int live = std::min(batch, np - bt * batch);
        // total mode: this batch's primes own accumulator slots bt*batch ..
        unsigned long long* acc = listed ? nullptr : d_acc + 2 * (size_t)bt * batch;
        ExactArgs a1;
        ExactArgsV2 a2;
        std::memset(&a1, 0, sizeof(a1));
        std::memset(&a2, 0, sizeof(a2));
        if (kv == 1) {
            for (int s = 0; s < kMaxSlots; ++s) a1.slot[s] = (s < 4 * P.nq) ? P.slot[s] : SlotDesc{0, 0, 1, 0, -1};
            for (int i = 0; i < P.m; ++i) a1.var_pos[i] = P.pos[i];
            for (int i = 0; i < batch; ++i) {
                a1.prime[i] = (double)bp[i];
                a1.pinv[i] = 1.0 / (double)bp[i];
            }
            a1.nprimes = batch;
            a1.m = P.m;
            a1.n_lane = P.n_lane;
            a1.n_walk = P.n_walk;
            a1.n_job = P.n_job;
            a1.lane_valid_bits = P.n_lane;
            for (int g = 0; g < 5; ++g) a1.qb[g] = P.qb[g];
            a1.job_bits_per_chunk = jb;
            a1.acc = acc;
            a1.larsen = P.larsen ? 1 : 0;
            a1.x_extra = x_extra;
        } else {
            for (int i = 0; i < batch; ++i) {
                a2.prime[i] = (double)bp[i];
                a2.pinv[i] = 1.0 / (double)bp[i];
            }
            a2.job_bits_per_chunk = jb;
            a2.item_job_bits = item_bits;
            if (rev_r > 0) a2.rev = rev;
            a2.acc = acc;
            a2.counter = d_counter;
            a2.rows = listed ? d_rows : nullptr;
            a2.x_extra = x_extra;
        }
        for (uint64_t base = 0; base < nchunks; base += wpl) {
            const uint64_t nw = std::min<uint64_t>(wpl, nchunks - base);
            const uint64_t* ids = nullptr;
            if (listed) {
                if ((e = hipMemcpyAsync(d_ids, R.chunk_ids + base, nw * sizeof(uint64_t), hipMemcpyHostToDevice,
                                        stream)) != hipSuccess) { fail(e, "hipMemcpyAsync"); goto done; }
                ids = d_ids;
            }
            // reference kernel: one wave per chunk; tuned kernel: persistent
            // waves (8 per SIMD, or one per item) over the launch's items
            const uint64_t n_items = nw << (jb - item_bits);
            const uint64_t grid_waves = kv == 1 ? nw : std::min<uint64_t>(n_items, (uint64_t)ctx->cus * 4 * 8);
            const unsigned blocks = (unsigned)((grid_waves + 3) / 4);
            if (kv == 2) {
                if ((e = launch_zero_words(d_counter, 1, stream)) != hipSuccess) { fail(e, "zero counter"); goto done; }
                if (listed && (e = launch_zero_words(d_rows, nw * batch * 2, stream)) != hipSuccess) {
                    fail(e, "zero rows");
                    goto done;
                }
            }
            if (e0 && (e = hipEventRecord(e0, stream)) != hipSuccess) { fail(e, "hipEventRecord"); goto done; }
            if (kv == 1) {
                a1.n_waves = nw;
                a1.chunk_base = chunk_offset + base;
                a1.chunk_ids = ids;
                hipLaunchKernelGGL(fn1, dim3(blocks), dim3(256), 0, stream, a1, d_out);
            } else {
                a2.n_chunks = nw;
                a2.n_items = (uint32_t)n_items;
                a2.chunk_base = chunk_offset + base;
                a2.chunk_ids = ids;
                hipLaunchKernelGGL(fn2, dim3(blocks), dim3(256), 0, stream, a2);
            }
            if ((e = hipGetLastError()) != hipSuccess) { fail(e, "kernel launch"); goto done; }
            if (e1 && (e = hipEventRecord(e1, stream)) != hipSuccess) { fail(e, "hipEventRecord"); goto done; }
            if (listed && kv == 1) {
                if ((e = hipMemcpyAsync(h_out.data(), d_out, nw * batch * sizeof(double), hipMemcpyDeviceToHost,
                                        stream)) != hipSuccess) { fail(e, "hipMemcpyAsync"); goto done; }
            }
            if (listed && kv == 2) {
                if ((e = hipMemcpyAsync(h_rows.data(), d_rows, nw * batch * 2 * sizeof(unsigned long long),
                                        hipMemcpyDeviceToHost, stream)) != hipSuccess) {
                    fail(e, "hipMemcpyAsync");
                    goto done;
                }
            }
            if ((e = hipStreamSynchronize(stream)) != hipSuccess) { fail(e, "hipStreamSynchronize"); goto done; }
            if (e0) {
                float ms = 0.f;
                if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { fail(e, "hipEventElapsedTime"); goto done; }
                st.kernel_ms += ms;
            }
            st.launches += 1;
            if (listed) {
                for (uint64_t w = 0; w < nw; ++w)
                    for (int i = 0; i < live; ++i) {
                        const int gi = bt * batch + i;
                        if (kv == 1) {
                            out[(base + w) * np + gi] = fp_to_residue(h_out[w * batch + i], R.primes[gi]);
                        } else {
                            const size_t r = 2 * (w * batch + i);
                            out[(base + w) * np + gi] =
                                (uint64_t)((((u128)h_rows[r + 1] << 64) | h_rows[r]) % R.primes[gi]);
                        }
                    }
            }
            terms_done += nw * terms_per_chunk;
            if (R.progress && R.progress(R.progress_ctx, terms_done, terms_total)) {
                status = SK_EABORTED;
                goto done;
            }
        }
    }
    if (!listed) {
        // one 128-bit sum per prime: (carries * 2^64 + low word) mod p
        if ((e = hipMemcpyAsync(h_acc.data(), d_acc, h_acc.size() * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, stream)) != hipSuccess) { fail(e, "hipMemcpyAsync"); goto done; }
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) { fail(e, "hipStreamSynchronize"); goto done; }
        for (int i = 0; i < np; ++i)
            out[i] = (uint64_t)((((u128)h_acc[2 * i + 1] << 64) | h_acc[2 * i]) % R.primes[i]);
        if (half)
            for (int i = 0; i < np; ++i) out[i] = (uint64_t)(((u128)out[i] * 2) % R.primes[i]);
    }
    if (!R.timing)
        st.kernel_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host).count();
    st.terms += reversal_evaluated(nchunks * terms_per_chunk, rev_r) * x0_passes;
    st.reversal_quads = rev_r;
    st.chunks += nchunks;
    st.log2_chunk_terms = P.n_lane + P.n_walk + jb;
    st.kernel_variant = kv;
    st.symmetry_halved = half ? 1 : 0;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (own_ws) (void)hipFree(ws);
    return status;
}

static int primes_needed(int n) { return primes_for(n); }

static uint64_t inv_pow2_scaled(uint64_t h, int e, uint64_t p)
{
    // h * 2^{-e} mod p
    const uint64_t inv2 = (p + 1) / 2;
    return mulmod(h, powmod(inv2, (uint64_t)e, p), p);
}

// Kernel-sum residues (halved factors) -> ordered count, with the range check.
static sk_status residues_to_count(const Plan& P, const std::vector<uint64_t>& primes, std::vector<uint64_t> res,
                                   Big& out)
{
    // C = H / 2^{m-1} with H = 2^{halved} * (kernel sum)
    for (size_t i = 0; i < primes.size(); ++i) res[i] = inv_pow2_scaled(res[i], P.m - 1 - P.halved, primes[i]);
    Big c = crt(res, primes);
    if (c.cmp(factorial_big(P.n)) > 0 || !c.fits128()) {
        g_last_error = "CRT result exceeds the bound n!";
        return SK_ECHECK;
    }
    out = c;
    return SK_OK;
}

static sk_status halve_reported(int n, int variant, unsigned flags, u128& result)
{
    if (!(flags & SK_ORDERED) && variant != SK_HOOKED && n > 1) {
        if (result & 1) {
            g_last_error = "ordered count is odd; reflections must pair up";
            return SK_ECHECK;
        }
        result >>= 1;
    }
    return SK_OK;
}

}  // namespace sk


namespace sk {

// ------------------------------------------------------------------ batch

// Device workspace of the counting entry points (sk_count_ex, sk_count_part,
// sk_count_batch): one batched launch's accumulators and counter, which also
// hold the accumulators of a separate count.
constexpr size_t kCountWsBytes = kBatchWsBytes > kSumWsBytes ? kBatchWsBytes : kSumWsBytes;

static BatchLaunchFn g_batch_fn[kBatchGroups][2];

int register_batch_kernel(int group, int ppi, BatchLaunchFn fn)
{
    if (group < 0 || group >= kBatchGroups || ppi < 0 || ppi > 1) return 0;
    g_batch_fn[group][ppi] = fn;
    return 1;
}

// Group whose batched kernel holds the tuned body of (variant, n), or -1.
static int batch_group(int variant, int n)
{
    const int g = batch_group_of(variant, n);
    if (g < 0 || !g_batch_fn[g][0] || !v2_slot(variant, n).fn) return -1;
    return g;
}

struct BatchJob {
    const Plan* plan;
    std::vector<uint64_t> primes;  // primes_for(n) of them
    std::vector<uint64_t> res;     // out: kernel-sum residues
    uint64_t terms = 0;
    bool half = false;             // Lemma 2.4 half (see SumRequest::half)
    bool reverse = false;          // reversal weights (see SumRequest::reverse)
};

// One persistent launch over the chunks of every job.  probe_shift > 0 runs
// only the first 2^-probe_shift of each job's chunks (used by the autotuner).
// ws: device workspace of at least kBatchWsBytes (nullptr: allocated here).
static sk_status run_batch(std::vector<BatchJob>& jobs, int group, int log2_chunk, uint64_t waves, int ppi,
                           hipStream_t stream, int probe_shift, sk_stats& st, double* kernel_ms,
                           void* ws_in = nullptr, bool timing = true)
{
    if (jobs.empty()) return SK_OK;
    if ((int)jobs.size() > kBatchMaxInstances || group < 0 || group >= kBatchGroups || ppi < 0 || ppi > 1)
        return SK_EINVAL;
    const BatchLaunchFn launch = g_batch_fn[group][ppi];
    if (!launch) return SK_ENOLIB;
    DeviceCtx* ctx;
    sk_status s = device_ctx(&ctx);
    if (s != SK_OK) return s;
    if (!stream) stream = ctx->stream;

    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    // largest work per item first, so the short instances fill the tail
    std::vector<size_t> order(jobs.size());
    for (size_t i = 0; i < jobs.size(); ++i) order[i] = i;
    std::vector<uint64_t> nch(jobs.size());
    for (size_t b = 0; b < jobs.size(); ++b) {
        const Plan& P = *jobs[b].plan;
        if (batch_group(P.variant, P.n) != group || (int)jobs[b].primes.size() != primes_for(P.n)) return SK_ENOLIB;
        int jb = log2_chunk - P.n_lane - P.n_walk;
        jb = std::max(0, std::min(jb, P.n_job));
        a.inst[b].variant = P.variant;
        a.inst[b].n = P.n;
        a.inst[b].nprimes = (int32_t)jobs[b].primes.size();
        a.inst[b].jb = jb;
        if (jobs[b].reverse) a.inst[b].rev = reversal_masks(P);
        for (size_t i = 0; i < jobs[b].primes.size(); ++i) {
            a.inst[b].prime[i] = (double)jobs[b].primes[i];
            a.inst[b].pinv[i] = 1.0 / (double)jobs[b].primes[i];
        }
        uint64_t total = 1ull << (P.n_job - jb);
        if (jobs[b].half && total < 2) jobs[b].half = false;
        if (jobs[b].half) total >>= 1;
        uint64_t use = std::max<uint64_t>(1, total >> probe_shift);
        nch[b] = use;
        jobs[b].terms = reversal_evaluated(use << (P.n_lane + P.n_walk + jb), a.inst[b].rev.r);
        st.reversal_quads = std::max(st.reversal_quads, (int)a.inst[b].rev.r);
    }
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) {
        return (jobs[x].terms / nch[x]) > (jobs[y].terms / nch[y]);
    });
    uint64_t n_items = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        a.first[k] = (uint32_t)n_items;
        a.slot_inst[k] = (int32_t)order[k];
        // one prime per item: each chunk is P items
        n_items += nch[order[k]] * (ppi == 1 ? jobs[order[k]].primes.size() : 1);
        if (n_items >= (1ull << 32)) return SK_EINVAL;
    }
    a.first[order.size()] = (uint32_t)n_items;
    a.nslots = (int32_t)order.size();
    a.n_items = (uint32_t)n_items;

    unsigned char* ws = (unsigned char*)ws_in;
    bool own_ws = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<unsigned long long> h_acc(kBatchAccBytes / sizeof(unsigned long long));
    hipError_t e;
    sk_status status = SK_OK;
    auto fail = [&](hipError_t err, const char* what) { status = hip_fail(err, what); };
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, (waves + 3) / 4);
    float ms = 0.f;
    auto t_host = std::chrono::steady_clock::now();
    if (!ws) {
        if ((e = hipMalloc(&ws, kBatchWsBytes)) != hipSuccess) { fail(e, "hipMalloc"); goto done; }
        own_ws = true;
    }
    a.acc = (unsigned long long*)ws;
    a.counter = (uint32_t*)(ws + kBatchAccBytes);
    if (timing) {
        if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
            fail(e, "hipEventCreate");
            goto done;
        }
    }
    // accumulators and counter: one 8-byte word per accumulator half, one for the counter
    if ((e = launch_zero_words(ws, kBatchAccBytes / 8 + 1, stream)) != hipSuccess) { fail(e, "zero workspace"); goto done; }
    if (e0 && (e = hipEventRecord(e0, stream)) != hipSuccess) { fail(e, "hipEventRecord"); goto done; }
    if ((e = launch(blocks, stream, a)) != hipSuccess) { fail(e, "batch launch"); goto done; }
    if (e1 && (e = hipEventRecord(e1, stream)) != hipSuccess) { fail(e, "hipEventRecord"); goto done; }
    if ((e = hipMemcpyAsync(h_acc.data(), a.acc, kBatchAccBytes, hipMemcpyDeviceToHost, stream)) != hipSuccess) {
        fail(e, "hipMemcpyAsync");
        goto done;
    }
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) { fail(e, "hipStreamSynchronize"); goto done; }
    if (e0) {
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { fail(e, "hipEventElapsedTime"); goto done; }
    } else {
        ms = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host).count();
    }
    for (size_t b = 0; b < jobs.size(); ++b) {
        BatchJob& j = jobs[b];
        j.res.assign(j.primes.size(), 0);
        for (size_t i = 0; i < j.primes.size(); ++i) {
            const size_t w = 2 * (b * kMaxPrimes + i);
            j.res[i] = (uint64_t)((((u128)h_acc[w + 1] << 64) | h_acc[w]) % j.primes[i]);
        }
    }
    for (auto& j : jobs)
        if (j.half)
            for (size_t i = 0; i < j.primes.size(); ++i) j.res[i] = (uint64_t)(((u128)j.res[i] * 2) % j.primes[i]);
    if (kernel_ms) *kernel_ms = ms;
    st.kernel_ms += ms;
    st.launches += 1;
    st.chunks += n_items;
    // sign vectors evaluated: every one once per item that holds it
    for (auto& j : jobs) st.terms += j.terms * (ppi == 1 ? j.primes.size() : 1);
    st.log2_chunk_terms = log2_chunk;
    st.kernel_variant = 3;
    for (auto& j : jobs)
        if (j.half) st.symmetry_halved = 1;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (own_ws) (void)hipFree(ws);
    return status;
}

// ----- autotune cache: (arch, CUs, instance list) -> launch shape

struct BatchShape {
    int log2_chunk = 27;
    uint64_t waves = 0;
    int ppi = 0;  // primes per work item: 0 all, 1 one
};

static std::mutex g_tune_mu;
static std::map<std::string, BatchShape> g_tune;
static bool g_tune_loaded = false;

static std::string tune_path()
{
    const char* p = std::getenv("SK_TUNE_CACHE");
    if (p && *p) return p;
    const char* h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/skolem_mi355x_tune.txt";
}

// One line per instance set: key, log2 sign vectors per item, waves, and
// (optionally) primes per item.
static void tune_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    std::ifstream f(tune_path());
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        BatchShape b;
        if (is >> key >> b.log2_chunk >> b.waves) {
            if (!(is >> b.ppi) || b.ppi < 0 || b.ppi > 1) b.ppi = 0;
            g_tune[key] = b;
        }
    }
}

static void tune_store()
{
    const std::string path = tune_path();
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) {
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i) {  // create the directory without a shell
            if (i == dir.size() || dir[i] == '/') {
                std::string sub = dir.substr(0, i);
                (void)::mkdir(sub.c_str(), 0755);
            }
        }
    }
    std::ofstream f(path, std::ios::trunc);
    for (auto& kv : g_tune)
        f << kv.first << " " << kv.second.log2_chunk << " " << kv.second.waves << " " << kv.second.ppi << "\n";
}

static std::string tune_key(const std::vector<const Plan*>& plans)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, g_device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    for (auto& ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    std::ostringstream os;
    os << arch << "|" << cus;
    std::vector<std::string> names;
    for (auto* p : plans) names.push_back(std::to_string(p->variant) + "." + std::to_string(p->n));
    std::sort(names.begin(), names.end());
    for (auto& nm : names) os << "|" << nm;
    return os.str();
}

// Times the batched launch of one group's instances on a fraction of every
// instance's chunks (1/4, or less for groups above 2^40 sign vectors) for
// each candidate shape and keeps the fastest in sign vectors of the count per
// second.  The probe must be large: the tail of a launch (waves without
// items) weighs as much more in a probe as the probe is smaller, and a small
// probe favours fewer waves than the full launch wants.  Candidates: 2^22 ..
// 2^28 sign vectors per work item, 2 .. 8 persistent waves per SIMD, and
// where the group has a kernel for it one prime per work item instead of all
// of them.  Smaller work items balance the tail of the launch better; one
// prime per item repeats the pair sums and products for every prime.
static sk_status autotune(const std::vector<const Plan*>& plans, int group, hipStream_t stream, BatchShape* best_out,
                          double* best_rate)
{
    DeviceCtx* ctx;
    sk_status s = device_ctx(&ctx);
    if (s != SK_OK) return s;
    uint64_t total = 0;
    for (auto* p : plans) total += 1ull << (p->m - 1 - (hat_symmetric(*p) ? 1 : 0));
    int shift = 2;
    while (shift < 20 && (total >> shift) > (1ull << 40)) ++shift;
    const int lcs[] = {22, 24, 26, 28};
    const int wps[] = {2, 4, 6, 8};
    double best = -1.0;
    for (int ppi = 0; ppi <= 1; ++ppi) {
        if (!g_batch_fn[group][ppi]) continue;
        for (int lc : lcs) {
            for (int wp : wps) {
                std::vector<BatchJob> jobs;
                for (auto* p : plans) {
                    // the same work per item as the production batch: Lemma 2.4
                    // half and reversal weights (weight-0 jobs skipped in a chunk)
                    BatchJob j;
                    j.plan = p;
                    j.primes = default_primes(primes_for(p->n), 0);
                    j.half = hat_symmetric(*p);
                    j.reverse = true;
                    jobs.push_back(j);
                }
                sk_stats st;
                std::memset(&st, 0, sizeof(st));
                double ms = 0;
                const uint64_t waves = (uint64_t)ctx->cus * 4 * wp;
                s = run_batch(jobs, group, lc, waves, ppi, stream, shift, st, &ms);
                if (s != SK_OK) return s;
                uint64_t covered = 0;
                for (auto& j : jobs) covered += j.terms;
                const double rate = (double)covered / (ms * 1e-3);
                if (rate > best) {
                    best = rate;
                    best_out->log2_chunk = lc;
                    best_out->waves = waves;
                    best_out->ppi = ppi;
                }
            }
        }
    }
    if (best_rate) *best_rate = best;
    return SK_OK;
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
    DeviceCtx* ctx;
    return device_ctx(&ctx);
}

static sk_status count_impl(int n, int variant, unsigned flags, const sk_tuning* tune, void* ws, size_t ws_bytes,
                            void* stream, sk_progress_fn progress, void* pctx, sk_stats* stats_out, sk_u128* out,
                            bool timing = true)
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
            R.kernel = tune ? tune->kernel : 0;
            R.stream = (hipStream_t)stream;
            R.progress = progress;
            R.progress_ctx = pctx;
            R.half = !(flags & SK_NO_SYMMETRY) && hat_symmetric(P);
            R.reverse = !(flags & SK_NO_SYMMETRY);
            R.ws = ws;
            R.ws_bytes = ws_bytes;
            R.timing = timing;
            std::vector<uint64_t> res;
            s = run_sum(R, res, st);
            if (s != SK_OK) return s;
            Big c;
            s = residues_to_count(P, R.primes, res, c);
            if (s != SK_OK) return s;
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
    s = halve_reported(n, variant, flags, result);
    if (s != SK_OK) return s;
    out->lo = (uint64_t)result;
    out->hi = (uint64_t)(result >> 64);
    st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st.ms_per_launch_avg = st.launches ? st.kernel_ms / (double)st.launches : 0.0;
    g_stats = st;
    if (stats_out) *stats_out = st;
    return SK_OK;
}

sk_status sk_count_larsen(int n, int variant, unsigned flags, const sk_tuning* tune, void* dev_workspace,
                          size_t ws_bytes, void* stream, sk_stats* stats_out, sk_u128* out)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!out) return SK_EINVAL;
    Plan P;
    sk_status s = make_plan(n, variant, P, true);
    if (s != SK_OK) return s;
    sk_stats st;
    std::memset(&st, 0, sizeof(st));
    u128 result = 0;
    if (existence(n, variant) || (flags & SK_NO_SHORTCUT)) {
        const int np = (tune && tune->primes > 0) ? std::max(primes_needed(n), std::min(tune->primes, kMaxPrimes))
                                                  : primes_needed(n);
        const int passes = (flags & SK_VERIFY) ? 2 : 1;
        Big first;
        for (int pass = 0; pass < passes; ++pass) {
            SumRequest R;
            R.plan = &P;
            R.primes = default_primes(np, pass * np);
            R.log2_chunk_terms = (tune && tune->log2_chunk_terms > 0) ? tune->log2_chunk_terms : 0;
            R.waves_per_launch = tune ? tune->waves_per_launch : 0;
            R.kernel = tune ? tune->kernel : 0;
            R.stream = (hipStream_t)stream;
            R.ws = dev_workspace;
            R.ws_bytes = ws_bytes;
            std::vector<uint64_t> res;
            s = run_sum(R, res, st);
            if (s != SK_OK) return s;
            // the sum is the ordered count itself: no power of two to divide out
            Big c = crt(res, R.primes);
            if (c.cmp(factorial_big(P.n)) > 0 || !c.fits128()) {
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
    s = halve_reported(n, variant, flags, result);
    if (s != SK_OK) return s;
    out->lo = (uint64_t)result;
    out->hi = (uint64_t)(result >> 64);
    st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st.ms_per_launch_avg = st.launches ? st.kernel_ms / (double)st.launches : 0.0;
    g_stats = st;
    if (stats_out) *stats_out = st;
    return SK_OK;
}

sk_status sk_count_part(int n, int variant, unsigned flags, uint64_t part, uint64_t parts, const sk_tuning* tune,
                        void* dev_workspace, size_t ws_bytes, void* stream, sk_progress_fn progress,
                        void* progress_ctx, sk_stats* stats_out, uint64_t* residues)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!residues || parts == 0 || part >= parts || (flags & SK_VERIFY)) return SK_EINVAL;
    Plan P;
    sk_status s = make_plan(n, variant, P);
    if (s != SK_OK) return s;
    const int np = primes_needed(n);
    sk_stats st;
    std::memset(&st, 0, sizeof(st));
    std::vector<uint64_t> res(np, 0);
    SumRequest R;
    R.plan = &P;
    R.primes = default_primes(np, 0);
    if (existence(n, variant) || (flags & SK_NO_SHORTCUT)) {
        R.log2_chunk_terms = (tune && tune->log2_chunk_terms > 0) ? tune->log2_chunk_terms : 0;
        R.waves_per_launch = tune ? tune->waves_per_launch : 0;
        R.kernel = tune ? tune->kernel : 0;
        R.stream = (hipStream_t)stream;
        R.progress = progress;
        R.progress_ctx = progress_ctx;
        R.half = !(flags & SK_NO_SYMMETRY) && hat_symmetric(P);
        R.reverse = !(flags & SK_NO_SYMMETRY);
        R.part = part;
        R.parts = parts;
        R.ws = dev_workspace;
        R.ws_bytes = ws_bytes;
        s = run_sum(R, res, st);
        if (s != SK_OK) return s;
    }
    for (int i = 0; i < np; ++i) {
        residues[i] = res[i];
        st.primes[i] = R.primes[i];
    }
    st.nprimes = np;
    st.passes = 1;
    st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st.ms_per_launch_avg = st.launches ? st.kernel_ms / (double)st.launches : 0.0;
    g_stats = st;
    if (stats_out) *stats_out = st;
    return SK_OK;
}

sk_status sk_count_combine(int n, int variant, unsigned flags, const uint64_t* residues, uint64_t parts,
                           sk_u128* out)
{
    if (!residues || !out || parts == 0) return SK_EINVAL;
    Plan P;
    sk_status s = make_plan(n, variant, P);
    if (s != SK_OK) return s;
    const int np = primes_needed(n);
    const std::vector<uint64_t> primes = default_primes(np, 0);
    std::vector<uint64_t> res(np, 0);
    for (uint64_t k = 0; k < parts; ++k)
        for (int i = 0; i < np; ++i) {
            const uint64_t r = residues[k * np + i];
            if (r >= primes[i]) return SK_EINVAL;
            res[i] = (uint64_t)(((u128)res[i] + r) % primes[i]);
        }
    u128 result = 0;
    if (existence(n, variant) || (flags & SK_NO_SHORTCUT)) {
        Big c;
        s = residues_to_count(P, primes, res, c);
        if (s != SK_OK) return s;
        result = ((u128)c.w[1] << 64) | c.w[0];
    }
    s = halve_reported(n, variant, flags, result);
    if (s != SK_OK) return s;
    out->lo = (uint64_t)result;
    out->hi = (uint64_t)(result >> 64);
    return SK_OK;
}

sk_status sk_count(int n, int variant, unsigned flags, sk_u128* out)
{
    return count_impl(n, variant, flags, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, out);
}

sk_status sk_count_ex(int n, int variant, unsigned flags, const sk_tuning* tune, void* dev_workspace,
                      size_t ws_bytes, void* stream, sk_progress_fn progress, void* progress_ctx, sk_stats* stats,
                      sk_u128* out)
{
    return count_impl(n, variant, flags, tune, dev_workspace, ws_bytes, stream, progress, progress_ctx, stats, out);
}


// Splits a batch into the instances of each batched group (at most
// kBatchMaxInstances per group) and those counted by separate launches:
// instances outside every group, with no tuned body, or with a tuning the
// batched kernels cannot run (the reference body, more primes).  Instances
// with no pairing (Sec. 1.1) are in neither list unless the shortcut is off.
static void partition_batch(const sk_instance* inst, size_t k, const sk_tuning* tune,
                            std::vector<std::vector<int>>& batched, std::vector<int>& separate)
{
    batched.assign(kBatchGroups, {});
    separate.clear();
    for (size_t i = 0; i < k; ++i) {
        const bool needed = existence(inst[i].n, inst[i].variant) || (inst[i].flags & SK_NO_SHORTCUT);
        if (!needed) continue;
        const int g = batch_group(inst[i].variant, inst[i].n);
        const bool can = g >= 0 && !(tune && (tune->kernel == 1 || tune->primes > primes_for(inst[i].n)));
        if (can && (int)batched[g].size() < kBatchMaxInstances) batched[g].push_back((int)i);
        else separate.push_back((int)i);
    }
}

// sk_count_batch on a given device workspace (nullptr: each launch allocates
// its own); timing = false times the call by the host clock instead of HIP
// events.
static sk_status batch_impl(const sk_instance* inst, size_t k, const sk_tuning* tune, void* ws, size_t ws_bytes,
                            void* stream, sk_stats* stats, sk_u128* out, bool timing)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!inst || !out || k == 0) return SK_EINVAL;
    if (ws && ws_bytes < kCountWsBytes) {
        g_last_error = "workspace of " + std::to_string(ws_bytes) + " bytes, " + std::to_string(kCountWsBytes) +
                       " needed";
        return SK_ENOMEM;
    }
    std::vector<Plan> plans(k);
    for (size_t i = 0; i < k; ++i) {
        sk_status s = make_plan(inst[i].n, inst[i].variant, plans[i]);
        if (s != SK_OK) return s;
    }
    sk_stats st;
    std::memset(&st, 0, sizeof(st));
    std::vector<u128> result(k, 0);
    // instances of each batched group, and those counted by separate launches
    std::vector<std::vector<int>> batched;
    std::vector<int> separate;
    partition_batch(inst, k, tune, batched, separate);
    DeviceCtx* ctx;
    {
        sk_status s = device_ctx(&ctx);
        if (s != SK_OK) return s;
    }
    for (int g = 0; g < kBatchGroups; ++g) {
        if (batched[g].empty()) continue;
        std::vector<const Plan*> bp;
        for (int i : batched[g]) bp.push_back(&plans[i]);
        // default shape when neither the caller nor the autotune cache has one:
        // work items of 2^22 sign vectors, 8 persistent waves per SIMD
        BatchShape shape;
        shape.log2_chunk = 22;
        shape.waves = (uint64_t)ctx->cus * 4 * 8;
        if (tune && tune->log2_chunk_terms > 0) {
            shape.log2_chunk = tune->log2_chunk_terms;
            if (tune->waves_per_launch > 0) shape.waves = (uint64_t)tune->waves_per_launch;
            shape.ppi = tune->primes_per_item == 1 ? 1 : 0;
        } else {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_load();
            auto it = g_tune.find(tune_key(bp));
            if (it != g_tune.end()) shape = it->second;
        }
        if (shape.ppi == 1 && !g_batch_fn[g][1]) shape.ppi = 0;
        int passes = 1;
        for (int i : batched[g])
            if (inst[i].flags & SK_VERIFY) passes = 2;
        std::vector<Big> first(k);
        for (int pass = 0; pass < passes; ++pass) {
            std::vector<BatchJob> jobs;
            std::vector<int> who;
            for (int i : batched[g]) {
                if (pass == 1 && !(inst[i].flags & SK_VERIFY)) continue;
                BatchJob j;
                j.plan = &plans[i];
                j.half = !(inst[i].flags & SK_NO_SYMMETRY) && hat_symmetric(plans[i]);
                j.reverse = !(inst[i].flags & SK_NO_SYMMETRY);
                const int np = primes_for(plans[i].n);
                j.primes = default_primes(np, pass * np);
                jobs.push_back(j);
                who.push_back(i);
            }
            sk_status s = run_batch(jobs, g, shape.log2_chunk, shape.waves, shape.ppi, (hipStream_t)stream, 0, st,
                                    nullptr, ws, timing);
            if (s != SK_OK) return s;
            for (size_t b = 0; b < jobs.size(); ++b) {
                const int i = who[b];
                Big cnt;
                s = residues_to_count(plans[i], jobs[b].primes, jobs[b].res, cnt);
                if (s != SK_OK) return s;
                if (pass == 0) {
                    first[i] = cnt;
                    result[i] = ((u128)cnt.w[1] << 64) | cnt.w[0];
                } else if (cnt.cmp(first[i]) != 0) {
                    g_last_error = "verification pass with disjoint primes disagrees";
                    return SK_ECHECK;
                }
            }
        }
        st.passes = std::max(st.passes, passes);
    }
    for (int i : separate) {
        sk_stats s1;
        sk_u128 o;
        sk_status s = count_impl(inst[i].n, inst[i].variant, inst[i].flags | SK_ORDERED, tune, ws, ws_bytes, stream,
                                 nullptr, nullptr, &s1, &o, timing);
        if (s != SK_OK) return s;
        result[i] = ((u128)o.hi << 64) | o.lo;
        st.kernel_ms += s1.kernel_ms;
        st.launches += s1.launches;
        st.terms += s1.terms;
        st.chunks += s1.chunks;
    }
    for (size_t i = 0; i < k; ++i) {
        sk_status s = halve_reported(inst[i].n, inst[i].variant, inst[i].flags, result[i]);
        if (s != SK_OK) return s;
    }
    for (size_t i = 0; i < k; ++i) {
        out[i].lo = (uint64_t)result[i];
        out[i].hi = (uint64_t)(result[i] >> 64);
    }
    st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st.ms_per_launch_avg = st.launches ? st.kernel_ms / (double)st.launches : 0.0;
    g_stats = st;
    if (stats) *stats = st;
    return SK_OK;
}

sk_status sk_count_batch(const sk_instance* inst, size_t k, const sk_tuning* tune, void* dev_workspace,
                         size_t ws_bytes, void* stream, sk_stats* stats, sk_u128* out)
{
    return batch_impl(inst, k, tune, dev_workspace, ws_bytes, stream, stats, out, true);
}

sk_status sk_count_batch_noalloc(const sk_instance* inst, size_t k, const sk_tuning* tune, void* stream,
                                 sk_stats* stats, sk_u128* out)
{
    if (!inst || !out || k == 0) return SK_EINVAL;
    const size_t need = sk_workspace_bytes(inst, k, tune);
    if (need == 0) return SK_EINVAL;
    if (need > kScratchBytes) {
        g_last_error = "needs " + std::to_string(need) + " bytes of device workspace; the fixed workspace holds " +
                       std::to_string(kScratchBytes);
        return SK_ENOMEM;
    }
    DeviceCtx* ctx;
    sk_status s = device_ctx(&ctx);
    if (s != SK_OK) return s;
    return batch_impl(inst, k, tune, ctx->scratch, kScratchBytes, stream, stats, out, false);
}

size_t sk_workspace_bytes(const sk_instance* inst, size_t k, const sk_tuning* tune)
{
    (void)tune;
    if (!inst || k == 0) return 0;
    for (size_t i = 0; i < k; ++i) {
        Plan P;
        if (make_plan(inst[i].n, inst[i].variant, P) != SK_OK) return 0;
    }
    return kCountWsBytes;
}

size_t sk_partial_workspace_bytes(int n, int variant, size_t nchunks, int nprimes, const sk_tuning* tune)
{
    Plan P;
    if (make_plan(n, variant, P) != SK_OK || nprimes < 1 || nprimes > 2 * kMaxPrimes) return 0;
    DeviceCtx* ctx;
    uint64_t wpl = 0;
    if (tune && tune->waves_per_launch > 0) wpl = (uint64_t)tune->waves_per_launch;
    else if (device_ctx(&ctx) == SK_OK) wpl = (uint64_t)ctx->cus * 4 * 8;
    else return 0;
    return sum_ws_bytes(true, std::max<uint64_t>(1, std::min<uint64_t>(wpl, nchunks)));
}

sk_status sk_autotune_batch(const sk_instance* inst, size_t k, void* stream, sk_tuning* best, double* best_rate)
{
    if (!inst || k == 0 || !best) return SK_EINVAL;
    std::vector<Plan> plans(k);
    for (size_t i = 0; i < k; ++i) {
        sk_status s = make_plan(inst[i].n, inst[i].variant, plans[i]);
        if (s != SK_OK) return s;
    }
    // the groups sk_count_batch would launch for these instances; the ones it
    // counts by separate launches have no shape to tune
    std::vector<std::vector<int>> batched;
    std::vector<int> separate;
    partition_batch(inst, k, nullptr, batched, separate);
    std::vector<std::vector<const Plan*>> groups(kBatchGroups);
    bool any = false;
    for (int g = 0; g < kBatchGroups; ++g) {
        for (int i : batched[g]) groups[g].push_back(&plans[i]);
        any = any || !groups[g].empty();
    }
    if (!any) {
        g_last_error = "no instance of this set runs in a batched launch";
        return SK_ENOLIB;
    }
    // every group is tuned and cached; the shape returned is that of the group
    // with the most sign vectors
    BatchShape out;
    double out_rate = 0, most = -1;
    for (int g = 0; g < kBatchGroups; ++g) {
        if (groups[g].empty()) continue;
        BatchShape shape;
        double rate = 0;
        sk_status s = autotune(groups[g], g, (hipStream_t)stream, &shape, &rate);
        if (s != SK_OK) return s;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_load();
            g_tune[tune_key(groups[g])] = shape;
            tune_store();
        }
        double work = 0;
        for (auto* p : groups[g]) work += std::ldexp(1.0, p->m - 1);
        if (work > most) {
            most = work;
            out = shape;
            out_rate = rate;
        }
    }
    if (best_rate) *best_rate = out_rate;
    std::memset(best, 0, sizeof(*best));
    best->log2_chunk_terms = out.log2_chunk;
    best->waves_per_launch = (int)out.waves;
    best->primes_per_item = out.ppi;
    return SK_OK;
}

sk_status sk_sign_sum_residues(int n, int variant, const uint64_t* primes, int nprimes,
                               const sk_tuning* tune, void* stream, uint64_t* residues)
{
    if (!primes || !residues || nprimes < 1 || nprimes > 2 * kMaxPrimes) return SK_EINVAL;
    Plan P;
    sk_status s = make_plan(n, variant, P);
    if (s != SK_OK) return s;
    SumRequest R;
    R.plan = &P;
    R.primes.assign(primes, primes + nprimes);
    R.log2_chunk_terms = (tune && tune->log2_chunk_terms > 0) ? tune->log2_chunk_terms : 0;
    R.waves_per_launch = tune ? tune->waves_per_launch : 0;
    R.kernel = tune ? tune->kernel : 0;
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

static sk_status describe_impl(int n, int variant, bool larsen, sk_plan_desc* out)
{
    if (!out) return SK_EINVAL;
    Plan P;
    sk_status s = make_plan(n, variant, P, larsen);
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
    out->symmetric = larsen ? 0 : (hat_symmetric(P) ? 1 : 0);
    out->reversal_quads = larsen ? 0 : reversal_masks(P).r;
    return SK_OK;
}

sk_status sk_describe(int n, int variant, sk_plan_desc* out) { return describe_impl(n, variant, false, out); }

sk_status sk_describe_larsen(int n, int variant, sk_plan_desc* out) { return describe_impl(n, variant, true, out); }

sk_status sk_partial_chunks(int n, int variant, int log2_chunks, const uint64_t* chunk_ids, size_t nchunks,
                            const uint64_t* primes, int nprimes, const sk_tuning* tune, void* dev_workspace,
                            size_t ws_bytes, void* stream, uint64_t* residues_out)
{
    if (!chunk_ids || !residues_out || nprimes < 1 || nprimes > 2 * kMaxPrimes) return SK_EINVAL;
    std::vector<uint64_t> dflt;
    if (!primes) {
        dflt = default_primes(nprimes, 0);
        primes = dflt.data();
    }
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
    R.waves_per_launch = tune ? tune->waves_per_launch : 0;
    R.kernel = tune ? tune->kernel : 0;
    R.stream = (hipStream_t)stream;
    std::vector<uint64_t> res;
    sk_stats st;
    std::memset(&st, 0, sizeof(st));
    R.ws = dev_workspace;
    R.ws_bytes = ws_bytes;
    s = run_sum(R, res, st);
    if (s != SK_OK) return s;
    for (size_t c = 0; c < nchunks; ++c)
        for (int i = 0; i < nprimes; ++i)
            residues_out[c * nprimes + i] =
                mulmod(res[c * nprimes + i], powmod(2, (uint64_t)P.halved, primes[i]), primes[i]);
    g_stats = st;
    return SK_OK;
}

sk_status sk_last_stats(sk_stats* out)
{
    if (!out) return SK_EINVAL;
    *out = g_stats;
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
        case 3: return "exact_batch_kernel";
    }
    return "none";
}

}  // extern "C"
