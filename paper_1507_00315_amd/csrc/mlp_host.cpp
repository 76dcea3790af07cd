// Host side of the learned proposal: the network's device buffers, forward and
// backward passes built from the MLP kernels, Adam training, and the C ABI
// entry points that expose each piece.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/skolem.h"
#include "sk_mlp.h"
#include "sk_mlp_net.h"

namespace sk {

const char* set_last_error(const std::string& msg);
int current_device();

bool mlp_geometry(int n, int variant, MlpGeo& g)
{
    if (n < 1 || n > 32 || variant < 0 || variant > 2 || (variant == 2 && n > 31)) return false;
    g.n = n;
    g.variant = variant;
    g.T = variant == 2 ? 2 * n + 1 : 2 * n;
    g.m = 0;
    g.pset = 0;
    for (int p = 1; p <= g.T; ++p) {
        if (variant == 2 && p == 2 * n) continue;
        g.pset |= 1ull << (p - 1);
        ++g.m;
    }
    return true;
}

#define NET_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            set_last_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
            return SK_EDEVICE;                                                             \
        }                                                                                  \
    } while (0)

MlpNet::~MlpNet() { release(); }

void MlpNet::free_batch()
{
    for (void** p : {(void**)&X, (void**)&H1, (void**)&H2, (void**)&Z, (void**)&X2, (void**)&Z2, (void**)&loss,
                     (void**)&betaf, (void**)&s_sel, (void**)&s_new, (void**)&mk, (void**)&mold, (void**)&e_old,
                     (void**)&e_new, (void**)&lq_f, (void**)&lq_r, (void**)&w_pick, (void**)&w_acc})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    cap = 0;
}

void MlpNet::release()
{
    for (float** p : {&P, &Gr, &Mo, &Ve, &ws})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    free_batch();
}

sk_status MlpNet::init(const MlpGeo& geo, int h1_, int h2_, hipStream_t s)
{
    g = geo;
    din = g.T + 2 * g.n + 2;
    h1 = h1_ > 0 ? h1_ : 256;
    h2 = h2_ > 0 ? h2_ : 256;
    dout = g.n * g.T;
    off_W1 = 0;
    off_b1 = off_W1 + (size_t)h1 * din;
    off_W2 = off_b1 + h1;
    off_b2 = off_W2 + (size_t)h2 * h1;
    off_W3 = off_b2 + h2;
    off_b3 = off_W3 + (size_t)dout * h2;
    count = off_b3 + dout;
    NET_HIP(hipMalloc(&P, count * sizeof(float)));
    NET_HIP(hipMalloc(&Gr, count * sizeof(float)));
    NET_HIP(hipMalloc(&Mo, count * sizeof(float)));
    NET_HIP(hipMalloc(&Ve, count * sizeof(float)));
    NET_HIP(hipMemsetAsync(Mo, 0, count * sizeof(float), s));
    NET_HIP(hipMemsetAsync(Ve, 0, count * sizeof(float), s));
    // split-K workspace: up to 16 partial copies of the largest weight matrix
    ws_floats = 16 * (long)std::max({(size_t)h1 * din, (size_t)h2 * h1, (size_t)dout * h2});
    NET_HIP(hipMalloc(&ws, (size_t)ws_floats * sizeof(float)));
    adam_t = 0;
    return SK_OK;
}

sk_status MlpNet::reserve(int B)
{
    if (B <= cap) return SK_OK;
    free_batch();
    NET_HIP(hipMalloc(&X, (size_t)B * din * sizeof(float)));
    NET_HIP(hipMalloc(&X2, (size_t)B * din * sizeof(float)));
    NET_HIP(hipMalloc(&H1, (size_t)B * h1 * sizeof(float)));
    NET_HIP(hipMalloc(&H2, (size_t)B * h2 * sizeof(float)));
    NET_HIP(hipMalloc(&Z, (size_t)B * dout * sizeof(float)));
    NET_HIP(hipMalloc(&Z2, (size_t)B * std::max(dout, h1 + h2) * sizeof(float)));
    NET_HIP(hipMalloc(&loss, (size_t)B * sizeof(float)));
    NET_HIP(hipMalloc(&betaf, (size_t)B * sizeof(float)));
    NET_HIP(hipMalloc(&s_sel, (size_t)B * g.n));
    NET_HIP(hipMalloc(&s_new, (size_t)B * g.n));
    for (int32_t** p : {&mk, &mold, &e_old, &e_new}) NET_HIP(hipMalloc(p, (size_t)B * sizeof(int32_t)));
    for (float** p : {&lq_f, &lq_r}) NET_HIP(hipMalloc(p, (size_t)B * sizeof(float)));
    for (uint32_t** p : {&w_pick, &w_acc}) NET_HIP(hipMalloc(p, (size_t)B * sizeof(uint32_t)));
    cap = B;
    return SK_OK;
}

static GemmArgs gemm(long M, long N, long K, const float* A, long sam, long sak, const float* B, long sbk, long sbn,
                     float* C, long scm, long scn)
{
    GemmArgs a;
    std::memset(&a, 0, sizeof(a));
    a.M = M;
    a.N = N;
    a.K = K;
    a.A = A;
    a.sam = sam;
    a.sak = sak;
    a.B = B;
    a.sbk = sbk;
    a.sbn = sbn;
    a.C = C;
    a.scm = scm;
    a.scn = scn;
    a.alpha = 1.f;
    return a;
}

hipError_t MlpNet::run_gemm(GemmArgs a, hipStream_t s)
{
    a.ws = ws;
    a.ws_floats = ws_floats;
    return launch_gemm(a, s);
}

// Z_out = MLP(X_in) for B rows (activations kept in H1, H2).
sk_status MlpNet::forward(const float* Xin, float* Zout, int B, hipStream_t s)
{
    GemmArgs a = gemm(B, h1, din, Xin, din, 1, P + off_W1, 1, din, H1, h1, 1);
    a.bias = P + off_b1;
    a.relu = 1;
    NET_HIP(run_gemm(a, s));
    a = gemm(B, h2, h1, H1, h1, 1, P + off_W2, 1, h1, H2, h2, 1);
    a.bias = P + off_b2;
    a.relu = 1;
    NET_HIP(run_gemm(a, s));
    a = gemm(B, dout, h2, H2, h2, 1, P + off_W3, 1, h2, Zout, dout, 1);
    a.bias = P + off_b3;
    NET_HIP(run_gemm(a, s));
    return SK_OK;
}

// Gradient of the mean cross-entropy for B states (features already in X,
// forward already run into Z); Gr receives the gradient.
sk_status MlpNet::backward(const uint8_t* states, int B, hipStream_t s)
{
    NET_HIP(launch_target_grad(g, states, betaf, B, Z, dout, 1.f / (float)B, loss, s));
    // dW3 = dZ^T H2, db3 = colsum dZ
    GemmArgs a = gemm(dout, h2, B, Z, 1, dout, H2, h2, 1, Gr + off_W3, h2, 1);
    NET_HIP(run_gemm(a, s));
    NET_HIP(launch_colsum(Z, B, dout, dout, 1.f, Gr + off_b3, s));
    // dA2 = (dZ W3) * [H2 > 0]  (into Z2 as scratch, B x h2)
    a = gemm(B, h2, dout, Z, dout, 1, P + off_W3, h2, 1, Z2, h2, 1);
    a.relu_ref = H2;
    NET_HIP(run_gemm(a, s));
    a = gemm(h2, h1, B, Z2, 1, h2, H1, h1, 1, Gr + off_W2, h1, 1);
    NET_HIP(run_gemm(a, s));
    NET_HIP(launch_colsum(Z2, B, h2, h2, 1.f, Gr + off_b2, s));
    // dA1 = (dA2 W2) * [H1 > 0]  (Z2 holds at least B x (h2 + h1) floats)
    float* dA1 = Z2 + (size_t)B * h2;
    a = gemm(B, h1, h2, Z2, h2, 1, P + off_W2, h1, 1, dA1, h1, 1);
    a.relu_ref = H1;
    NET_HIP(run_gemm(a, s));
    a = gemm(h1, din, B, dA1, 1, h1, X, din, 1, Gr + off_W1, din, 1);
    NET_HIP(run_gemm(a, s));
    NET_HIP(launch_colsum(dA1, B, h1, h1, 1.f, Gr + off_b1, s));
    return SK_OK;
}

sk_status MlpNet::set_betas(const double* betas, int B, hipStream_t s)
{
    std::vector<float> bf(betas, betas + B);
    NET_HIP(hipMemcpyAsync(betaf, bf.data(), B * sizeof(float), hipMemcpyHostToDevice, s));
    NET_HIP(hipStreamSynchronize(s));
    return SK_OK;
}

sk_status MlpNet::mh_step(int B, int M, int j0, int nsel, long base, uint8_t* dst, uint64_t* acc_count,
                          uint8_t* accepted, hipStream_t s)
{
    sk_status st;
    NET_HIP(launch_features(g, s_sel, betaf, B, X, din, e_old, s));
    if ((st = forward(X, Z, B, s)) != SK_OK) return st;
    NET_HIP(launch_sample(g, s_sel, Z, dout, w_pick, B, s_new, mk, mold, lq_f, s));
    NET_HIP(launch_features(g, s_new, betaf, B, X2, din, e_new, s));
    if ((st = forward(X2, Z2, B, s)) != SK_OK) return st;
    NET_HIP(launch_logq(g, Z2, dout, mk, mold, B, lq_r, s));
    NET_HIP(launch_accept(g.n, s_new, e_old, e_new, lq_f, lq_r, betaf, w_acc, B, M, j0, nsel, base, dst, acc_count,
                          accepted, s));
    return SK_OK;
}

sk_status MlpNet::train_pool(const uint8_t* pool, const float* pool_beta, int N, int steps, int B, float lr,
                             hipStream_t s, double* last_loss)
{
    sk_status st;
    for (int step = 0; step < steps; ++step) {
        // rows (step * B + i) mod N, as at most two contiguous runs per wrap
        int filled = 0;
        long r = (long)(((unsigned long long)step * (unsigned long long)B) % (unsigned long long)N);
        while (filled < B) {
            const int run = (int)std::min<long>(B - filled, N - r);
            NET_HIP(hipMemcpyAsync(s_sel + (size_t)filled * g.n, pool + (size_t)r * g.n, (size_t)run * g.n,
                                   hipMemcpyDeviceToDevice, s));
            NET_HIP(hipMemcpyAsync(betaf + filled, pool_beta + r, (size_t)run * sizeof(float),
                                   hipMemcpyDeviceToDevice, s));
            filled += run;
            r = 0;
        }
        NET_HIP(launch_features(g, s_sel, betaf, B, X, din, nullptr, s));
        if ((st = forward(X, Z, B, s)) != SK_OK) return st;
        if ((st = backward(s_sel, B, s)) != SK_OK) return st;
        if ((st = adam_step(lr, s)) != SK_OK) return st;
    }
    if (last_loss) {
        *last_loss = 0;
        if (steps > 0) {
            std::vector<float> lv(B);
            NET_HIP(hipMemcpyAsync(lv.data(), loss, (size_t)B * sizeof(float), hipMemcpyDeviceToHost, s));
            NET_HIP(hipStreamSynchronize(s));
            double t = 0;
            for (float v : lv) t += v;
            *last_loss = t / B;
        }
    }
    return SK_OK;
}

sk_status MlpNet::adam_step(float lr, hipStream_t s)
{
    ++adam_t;
    NET_HIP(launch_adam(P, Gr, Mo, Ve, (long)count, lr, 0.9f, 0.999f, 1e-8f, adam_t, s));
    return SK_OK;
}

}  // namespace sk

using namespace sk;

namespace {

struct Scoped {
    hipStream_t s = nullptr, own = nullptr;
    explicit Scoped(void* stream)
    {
        s = (hipStream_t)stream;
        if (!s && hipStreamCreateWithFlags(&own, hipStreamNonBlocking) == hipSuccess) s = own;
    }
    ~Scoped()
    {
        if (own) (void)hipStreamDestroy(own);
    }
};

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

sk_status setup_net(int n, int variant, int h1, int h2, const float* params, MlpNet& net, hipStream_t s)
{
    MlpGeo g;
    if (!mlp_geometry(n, variant, g) || !params) return SK_EINVAL;
    if (hipSetDevice(current_device()) != hipSuccess) return SK_EDEVICE;
    sk_status st = net.init(g, h1, h2, s);
    if (st != SK_OK) return st;
    if (hipMemcpyAsync(net.P, params, net.count * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess)
        return SK_EDEVICE;
    return SK_OK;
}

sk_status check_states(const MlpGeo& g, const uint8_t* states, int B)
{
    // every placement must be valid: the kernels index bins with it
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < g.n; ++k) {
            const int a = states[(size_t)b * g.n + k];
            const int d = g.variant == 1 ? k + 2 : k + 1;
            if (a < 1 || a + d > g.T || !((g.pset >> (a - 1)) & 1) || !((g.pset >> (a + d - 1)) & 1))
                return SK_EINVAL;
        }
    return SK_OK;
}

}  // namespace

namespace {

// uploads B host states and their inverse temperatures into net.s_sel / betaf
sk_status upload_batch(MlpNet& net, const uint8_t* states, const double* betas, int B, hipStream_t s)
{
    sk_status st;
    if ((st = check_states(net.g, states, B)) != SK_OK) return st;
    if ((st = net.reserve(B)) != SK_OK) return st;
    if (hipMemcpyAsync(net.s_sel, states, (size_t)B * net.g.n, hipMemcpyHostToDevice, s) != hipSuccess)
        return SK_EDEVICE;
    return net.set_betas(betas, B, s);
}

double mean_loss(MlpNet& net, int B, hipStream_t s, sk_status& st)
{
    std::vector<float> lv(B);
    if (hipMemcpyAsync(lv.data(), net.loss, (size_t)B * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        st = SK_EDEVICE;
        return 0;
    }
    double t = 0;
    for (float v : lv) t += v;
    return t / B;
}

}  // namespace

extern "C" {

size_t sk_mlp_param_count(int n, int variant, int h1, int h2)
{
    MlpGeo g;
    if (!mlp_geometry(n, variant, g) || h1 < 0 || h2 < 0) return 0;
    h1 = h1 > 0 ? h1 : 256;
    h2 = h2 > 0 ? h2 : 256;
    const size_t din = g.T + 2 * g.n + 2, dout = (size_t)g.n * g.T;
    return (size_t)h1 * din + h1 + (size_t)h2 * h1 + h2 + dout * h2 + dout;
}

sk_status sk_mlp_init(int n, int variant, int h1, int h2, uint64_t seed, double scale, float* params)
{
    MlpGeo g;
    if (!mlp_geometry(n, variant, g) || !params || h1 < 0 || h2 < 0) return SK_EINVAL;
    h1 = h1 > 0 ? h1 : 256;
    h2 = h2 > 0 ? h2 : 256;
    const int din = g.T + 2 * g.n + 2, dout = g.n * g.T;
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    float* p = params;
    auto layer = [&](int out, int in) {
        const double sd = scale / std::sqrt((double)in);
        for (long i = 0; i < (long)out * in; ++i) *p++ = (float)(nd(rng) * sd);
        for (int i = 0; i < out; ++i) *p++ = 0.f;
    };
    layer(h1, din);
    layer(h2, h1);
    layer(dout, h2);
    return SK_OK;
}

sk_status sk_mlp_forward(int n, int variant, int h1, int h2, const float* params, const uint8_t* states,
                         const double* betas, int batch, void* stream, float* logits)
{
    if (!states || !betas || !logits || batch < 1) return SK_EINVAL;
    Scoped sc(stream);
    MlpNet net;
    sk_status st = setup_net(n, variant, h1, h2, params, net, sc.s);
    if (st != SK_OK) return st;
    if ((st = upload_batch(net, states, betas, batch, sc.s)) != SK_OK) return st;
    if (launch_features(net.g, net.s_sel, net.betaf, batch, net.X, net.din, nullptr, sc.s) != hipSuccess)
        return SK_EDEVICE;
    if ((st = net.forward(net.X, net.Z, batch, sc.s)) != SK_OK) return st;
    if (hipMemcpyAsync(logits, net.Z, (size_t)batch * net.dout * sizeof(float), hipMemcpyDeviceToHost, sc.s) !=
            hipSuccess ||
        hipStreamSynchronize(sc.s) != hipSuccess)
        return SK_EDEVICE;
    return SK_OK;
}

sk_status sk_mlp_loss_grad(int n, int variant, int h1, int h2, const float* params, const uint8_t* states,
                           const double* betas, int batch, void* stream, double* loss, float* grads)
{
    if (!states || !betas || !grads || batch < 1) return SK_EINVAL;
    Scoped sc(stream);
    MlpNet net;
    sk_status st = setup_net(n, variant, h1, h2, params, net, sc.s);
    if (st != SK_OK) return st;
    if ((st = upload_batch(net, states, betas, batch, sc.s)) != SK_OK) return st;
    if (launch_features(net.g, net.s_sel, net.betaf, batch, net.X, net.din, nullptr, sc.s) != hipSuccess)
        return SK_EDEVICE;
    if ((st = net.forward(net.X, net.Z, batch, sc.s)) != SK_OK) return st;
    if ((st = net.backward(net.s_sel, batch, sc.s)) != SK_OK) return st;
    if (hipMemcpyAsync(grads, net.Gr, net.count * sizeof(float), hipMemcpyDeviceToHost, sc.s) != hipSuccess)
        return SK_EDEVICE;
    const double l = mean_loss(net, batch, sc.s, st);
    if (st != SK_OK) return st;
    if (loss) *loss = l;
    return SK_OK;
}

sk_status sk_mlp_train(int n, int variant, int h1, int h2, float* params, const uint8_t* states, const double* betas,
                       int nstates, int steps, int minibatch, double lr, void* stream, double* last_loss)
{
    if (!params || !states || !betas || nstates < 1 || steps < 0 || minibatch < 1 || !(lr > 0)) return SK_EINVAL;
    Scoped sc(stream);
    MlpNet net;
    sk_status st = setup_net(n, variant, h1, h2, params, net, sc.s);
    if (st != SK_OK) return st;
    MlpGeo g = net.g;
    if ((st = check_states(g, states, nstates)) != SK_OK) return st;
    if ((st = net.reserve(minibatch)) != SK_OK) return st;
    DevBuf pool, pbeta;
    std::vector<float> bf(betas, betas + nstates);
    if (hipMalloc(&pool.p, (size_t)nstates * n) != hipSuccess ||
        hipMalloc(&pbeta.p, (size_t)nstates * sizeof(float)) != hipSuccess)
        return SK_EDEVICE;
    if (hipMemcpyAsync(pool.p, states, (size_t)nstates * n, hipMemcpyHostToDevice, sc.s) != hipSuccess ||
        hipMemcpyAsync(pbeta.p, bf.data(), (size_t)nstates * sizeof(float), hipMemcpyHostToDevice, sc.s) !=
            hipSuccess)
        return SK_EDEVICE;
    if ((st = net.train_pool((const uint8_t*)pool.p, (const float*)pbeta.p, nstates, steps, minibatch, (float)lr,
                             sc.s, last_loss)) != SK_OK)
        return st;
    if (hipMemcpyAsync(params, net.P, net.count * sizeof(float), hipMemcpyDeviceToHost, sc.s) != hipSuccess ||
        hipStreamSynchronize(sc.s) != hipSuccess)
        return SK_EDEVICE;
    return SK_OK;
}

sk_status sk_mlp_mh_step(int n, int variant, int h1, int h2, const float* params, const uint8_t* states,
                         const double* betas, const uint32_t* w_pick, const uint32_t* w_acc, int batch, void* stream,
                         uint8_t* out_states, uint8_t* accepted, uint8_t* proposed, float* logq_forward,
                         float* logq_reverse)
{
    if (!states || !betas || !w_pick || !w_acc || !out_states || batch < 1) return SK_EINVAL;
    Scoped sc(stream);
    MlpNet net;
    sk_status st = setup_net(n, variant, h1, h2, params, net, sc.s);
    if (st != SK_OK) return st;
    if ((st = upload_batch(net, states, betas, batch, sc.s)) != SK_OK) return st;
    DevBuf dst, dacc;
    if (hipMalloc(&dst.p, (size_t)batch * n) != hipSuccess || hipMalloc(&dacc.p, (size_t)batch) != hipSuccess)
        return SK_EDEVICE;
    if (hipMemcpyAsync(dst.p, states, (size_t)batch * n, hipMemcpyHostToDevice, sc.s) != hipSuccess ||
        hipMemcpyAsync(net.w_pick, w_pick, (size_t)batch * 4, hipMemcpyHostToDevice, sc.s) != hipSuccess ||
        hipMemcpyAsync(net.w_acc, w_acc, (size_t)batch * 4, hipMemcpyHostToDevice, sc.s) != hipSuccess)
        return SK_EDEVICE;
    if ((st = net.mh_step(batch, batch, 0, 0, 0, (uint8_t*)dst.p, nullptr, (uint8_t*)dacc.p, sc.s)) != SK_OK) return st;
    bool ok = hipMemcpyAsync(out_states, dst.p, (size_t)batch * n, hipMemcpyDeviceToHost, sc.s) == hipSuccess;
    if (accepted) ok = ok && hipMemcpyAsync(accepted, dacc.p, batch, hipMemcpyDeviceToHost, sc.s) == hipSuccess;
    if (proposed)
        ok = ok && hipMemcpyAsync(proposed, net.s_new, (size_t)batch * n, hipMemcpyDeviceToHost, sc.s) == hipSuccess;
    if (logq_forward)
        ok = ok && hipMemcpyAsync(logq_forward, net.lq_f, (size_t)batch * 4, hipMemcpyDeviceToHost, sc.s) == hipSuccess;
    if (logq_reverse)
        ok = ok && hipMemcpyAsync(logq_reverse, net.lq_r, (size_t)batch * 4, hipMemcpyDeviceToHost, sc.s) == hipSuccess;
    if (!ok || hipStreamSynchronize(sc.s) != hipSuccess) return SK_EDEVICE;
    return SK_OK;
}

}  // extern "C"
