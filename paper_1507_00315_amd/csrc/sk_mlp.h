// Shared definitions of the learned-proposal kernels (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

// Geometry of the relaxed problem for the kernels.
struct MlpGeo {
    int32_t n, variant, T, m;  // pairs, variant, bins 1..T, |P|
    uint64_t pset;             // bit p-1 set for p in P
};

// C[m, n] = alpha * sum_k A[m, k] B[k, n] (+ bias[n]) (+ C if accumulate),
// then max(., 0) if relu, then 0 where relu_ref[m, n] <= 0 (if given).
// With a workspace, short-and-wide products (few output tiles, long K) are
// split along K and the partials summed in a fixed order.
// Element (i, j) of a matrix X sits at X[i * s_i + j * s_j].
struct GemmArgs {
    long M, N, K;
    const float* A;
    long sam, sak;
    const float* B;
    long sbk, sbn;
    float* C;
    long scm, scn;
    const float* bias;
    const float* relu_ref;
    int relu;
    int accumulate;
    float alpha;
    float* ws;       // nullptr, or a workspace of ws_floats floats that allows split-K
    long ws_floats;
};

hipError_t launch_features(const MlpGeo& g, const uint8_t* states, const float* beta, int B, float* X, int ldx,
                           int32_t* energy, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s);
hipError_t launch_colsum(const float* Y, long M, long N, long ld, float alpha, float* out, hipStream_t s);
hipError_t launch_target_grad(const MlpGeo& g, const uint8_t* states, const float* beta, int B, float* Z, int ldz,
                              float scale, float* loss, hipStream_t s);
hipError_t launch_sample(const MlpGeo& g, const uint8_t* states, const float* Z, int ldz, const uint32_t* uword,
                         int B, uint8_t* states_new, int32_t* move_k, int32_t* move_old, float* logq_fwd,
                         hipStream_t s);
hipError_t launch_logq(const MlpGeo& g, const float* Z, int ldz, const int32_t* move_k, const int32_t* move_old,
                       int B, float* logq_rev, hipStream_t s);
hipError_t launch_accept(int n, const uint8_t* proposed, const int32_t* e_old, const int32_t* e_new,
                         const float* logq_fwd, const float* logq_rev, const float* beta, const uint32_t* uword, int B,
                         int M, int j0, int nsel, long base, uint8_t* dst, uint64_t* acc_count, uint8_t* accepted,
                         hipStream_t s);
hipError_t launch_gather(int n, const uint8_t* all, int M, int j0, int nsel, long base, const float* beta_level,
                         int B, uint8_t* sel, float* beta_sel, hipStream_t s);
hipError_t launch_words(uint64_t seed, uint32_t step, int j0, int nsel, long base, int B, uint32_t* w_pick,
                        uint32_t* w_acc, hipStream_t s);
hipError_t launch_adam(float* P, const float* G, float* M, float* V, long n, float lr, float b1, float b2, float eps,
                       int t, hipStream_t s);

}  // namespace sk
