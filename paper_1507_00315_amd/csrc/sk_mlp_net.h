// Device-resident proposal network: parameters, Adam moments, activations.
// Parameter layout (fp32, one flat buffer, row-major weights, out x in):
//   W1[h1][din] b1[h1] W2[h2][h1] b2[h2] W3[dout][h2] b3[dout]
// with din = T + 2n + 2 and dout = n * T.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/skolem.h"
#include "sk_mlp.h"

namespace sk {

bool mlp_geometry(int n, int variant, MlpGeo& g);

struct MlpNet {
    MlpGeo g{};
    int din = 0, h1 = 0, h2 = 0, dout = 0;
    size_t off_W1 = 0, off_b1 = 0, off_W2 = 0, off_b2 = 0, off_W3 = 0, off_b3 = 0, count = 0;
    float *P = nullptr, *Gr = nullptr, *Mo = nullptr, *Ve = nullptr;  // params, grads, Adam moments
    float* ws = nullptr;  // split-K workspace of the GEMMs
    long ws_floats = 0;
    // per-batch buffers for up to cap states: features X (B x din), hidden
    // activations H1, H2, logits Z (B x dout); X2, Z2 hold the second forward
    // pass of a proposal (at C') and the backward scratch
    float *X = nullptr, *H1 = nullptr, *H2 = nullptr, *Z = nullptr, *X2 = nullptr, *Z2 = nullptr;
    float *loss = nullptr, *betaf = nullptr;
    // Metropolis-Hastings step buffers (B entries each)
    uint8_t *s_sel = nullptr, *s_new = nullptr;
    int32_t *mk = nullptr, *mold = nullptr, *e_old = nullptr, *e_new = nullptr;
    float *lq_f = nullptr, *lq_r = nullptr;
    uint32_t *w_pick = nullptr, *w_acc = nullptr;
    int cap = 0;
    int adam_t = 0;

    MlpNet() = default;
    MlpNet(const MlpNet&) = delete;
    MlpNet& operator=(const MlpNet&) = delete;
    ~MlpNet();
    void release();
    void free_batch();
    // allocates parameters, gradient and Adam moments (moments zeroed on s)
    sk_status init(const MlpGeo& geo, int h1, int h2, hipStream_t s);
    sk_status reserve(int B);
    sk_status set_betas(const double* betas, int B, hipStream_t s);
    hipError_t run_gemm(GemmArgs a, hipStream_t s);
    sk_status forward(const float* Xin, float* Zout, int B, hipStream_t s);
    sk_status backward(const uint8_t* states, int B, hipStream_t s);
    sk_status adam_step(float lr, hipStream_t s);
    // one learned Metropolis-Hastings move for the B configurations in s_sel
    // (inverse temperatures in betaf, words in w_pick / w_acc); accepted ones
    // are written to dst (row mapping of launch_accept)
    sk_status mh_step(int B, int M, int j0, int nsel, long base, uint8_t* dst, uint64_t* acc_count,
                      uint8_t* accepted, hipStream_t s);
    // steps Adam steps on minibatches of B rows taken cyclically from a
    // device pool of N configurations (row i of step t: (t * B + i) mod N)
    sk_status train_pool(const uint8_t* pool, const float* pool_beta, int N, int steps, int B, float lr,
                         hipStream_t s, double* last_loss);
};

}  // namespace sk
