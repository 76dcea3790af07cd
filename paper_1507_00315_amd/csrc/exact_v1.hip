// Exact sign-vector sum (Lemma 2.1), reference kernel body for gfx950.
//
// One wavefront evaluates one chunk of the half-sum (x_1 = +1, Lemma 2.2):
//   * the 64 lanes enumerate the n_lane highest sign variables,
//   * the wave walks 2^job_bits_per_chunk jobs (low job variables), and
//   * inside a job every lane visits the n_walk lowest free variables in
//     binary-reflected Gray-code order (Sec. 2.1, after Algorithm 1).
// Each term is (prod x) * prod_k f_k(x) with f_k the pair sums.  Factors with
// an even number of pairs L_k are always even and enter as f_k / 2.
//
// This body recomputes every pair sum from the sign mask at every step
// (popcount form); it is the simple, obviously-correct kernel that the tuned
// body (exact_v2.hip) is tested against.  The product path is shared.
// With a.larsen it evaluates the inclusion-exclusion sum instead (0/1
// variables, factors = occupied pairs at distance d_k; see exact_v2_body.h).
#include <hip/hip_runtime.h>

#include "exact_common.h"
#include "sk_internal.h"

namespace sk {

template <int NQ, int G>
__global__ void __launch_bounds__(256) exact_v1_kernel(const ExactArgs a, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const bool active = wave < a.n_waves;  // wave-uniform
    const int P = a.nprimes;
    double res[kMaxPrimes] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
        const uint64_t chunk = a.chunk_ids ? a.chunk_ids[wave] : a.chunk_base + wave;

        uint64_t x_fixed = a.x_extra;
        for (int b = 0; b < a.n_lane; ++b)
            if ((lane >> b) & 1) x_fixed |= 1ull << (a.var_pos[a.m - a.n_lane + b] - 1);
        const int cb = a.n_job - a.job_bits_per_chunk;
        for (int b = 0; b < cb; ++b)
            if ((chunk >> b) & 1)
                x_fixed |= 1ull << (a.var_pos[1 + a.n_walk + a.job_bits_per_chunk + b] - 1);

        double acc[kMaxPrimes] = {0.0, 0.0, 0.0, 0.0};
        const uint64_t njobs = 1ull << a.job_bits_per_chunk;
        const uint64_t nsteps = 1ull << a.n_walk;
        for (uint64_t j = 0; j < njobs; ++j) {
            uint64_t X = x_fixed;
            for (int b = 0; b < a.job_bits_per_chunk; ++b)
                if ((j >> b) & 1) X |= 1ull << (a.var_pos[1 + a.n_walk + b] - 1);
            const bool neg0 = __popcll(X) & 1;
            double accj[kMaxPrimes] = {0.0, 0.0, 0.0, 0.0};
            for (uint64_t t = 0; t < nsteps; ++t) {
                if (t) X ^= 1ull << (a.var_pos[1 + __builtin_ctzll(t)] - 1);
                int32_t f[4 * NQ];
#pragma unroll
                for (int s = 0; s < 4 * NQ; ++s) {
                    if (a.larsen) {  // occupied pairs at distance d_k; a constant-1 slot has no pairs
                        f[s] = __popcll(X & (X >> a.slot[s].d) & a.slot[s].mask) + (a.slot[s].pad < 0 ? 1 : 0);
                    } else {
                        const int c = __popcll((X ^ (X >> a.slot[s].d)) & a.slot[s].mask);
                        f[s] = (a.slot[s].len - 2 * c) >> a.slot[s].halve;
                    }
                }
                double g[G];
                group_products<NQ, G>(f, a.qb, g);
                accumulate_term<G>(g, a.prime, a.pinv, P, (t & 1) != 0, accj);
                if ((t & 63) == 63) {
                    for (int i = 0; i < kMaxPrimes; ++i)
                        if (i < P) accj[i] = reduce_balanced(accj[i], a.prime[i], a.pinv[i]);
                }
            }
            for (int i = 0; i < kMaxPrimes; ++i) {
                if (i < P) {
                    const double r = reduce_balanced(accj[i], a.prime[i], a.pinv[i]);
                    acc[i] = reduce_balanced(neg0 ? acc[i] - r : acc[i] + r, a.prime[i], a.pinv[i]);
                }
            }
        }
        const bool valid = lane < (1 << a.n_lane);
#pragma unroll
        for (int i = 0; i < kMaxPrimes; ++i) {
            if (i < P) {
                const double v = wave_sum_f64(valid ? acc[i] : 0.0);
                res[i] = v;
                if (lane == 0 && !a.acc) out[wave * P + i] = v;
            }
        }
    }
    // sums of whole launches: workgroup stage, then the device accumulators
    if (a.acc) workgroup_accumulate<kMaxPrimes>(res, P, a.prime, a.pinv, active, a.acc);
}

#define SK_V1_INST(NQ, G) \
    template __global__ void exact_v1_kernel<NQ, G>(const ExactArgs, double* __restrict__);

SK_V1_INST(1, 1)
SK_V1_INST(2, 1) SK_V1_INST(2, 2)
SK_V1_INST(3, 1) SK_V1_INST(3, 2) SK_V1_INST(3, 3)
SK_V1_INST(4, 1) SK_V1_INST(4, 2) SK_V1_INST(4, 3) SK_V1_INST(4, 4)
SK_V1_INST(5, 1) SK_V1_INST(5, 2) SK_V1_INST(5, 3) SK_V1_INST(5, 4)
SK_V1_INST(6, 1) SK_V1_INST(6, 2) SK_V1_INST(6, 3) SK_V1_INST(6, 4)
SK_V1_INST(7, 1) SK_V1_INST(7, 2) SK_V1_INST(7, 3) SK_V1_INST(7, 4)
SK_V1_INST(8, 1) SK_V1_INST(8, 2) SK_V1_INST(8, 3) SK_V1_INST(8, 4)

// Clears n 64-bit words: accumulators and counters are cleared by a kernel on
// the caller's stream rather than by a memset node, so a captured sequence of
// calls replays the clearing too.
__global__ void __launch_bounds__(256) zero_words_kernel(unsigned long long* __restrict__ p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_zero_words(void* p, uint64_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)(n / 256 + 1 < 64 ? n / 256 + 1 : 64);
    hipLaunchKernelGGL(zero_words_kernel, dim3(blocks), dim3(256), 0, stream, (unsigned long long*)p, n);
    return hipGetLastError();
}

using ExactKernelFn = void (*)(const ExactArgs, double*);

ExactKernelFn exact_v1_lookup(int nq, int g)
{
#define SK_V1_CASE(NQ, G) \
    if (nq == NQ && g == G) return exact_v1_kernel<NQ, G>;
    SK_V1_CASE(1, 1)
    SK_V1_CASE(2, 1) SK_V1_CASE(2, 2)
    SK_V1_CASE(3, 1) SK_V1_CASE(3, 2) SK_V1_CASE(3, 3)
    SK_V1_CASE(4, 1) SK_V1_CASE(4, 2) SK_V1_CASE(4, 3) SK_V1_CASE(4, 4)
    SK_V1_CASE(5, 1) SK_V1_CASE(5, 2) SK_V1_CASE(5, 3) SK_V1_CASE(5, 4)
    SK_V1_CASE(6, 1) SK_V1_CASE(6, 2) SK_V1_CASE(6, 3) SK_V1_CASE(6, 4)
    SK_V1_CASE(7, 1) SK_V1_CASE(7, 2) SK_V1_CASE(7, 3) SK_V1_CASE(7, 4)
    SK_V1_CASE(8, 1) SK_V1_CASE(8, 2) SK_V1_CASE(8, 3) SK_V1_CASE(8, 4)
#undef SK_V1_CASE
    return nullptr;
}

}  // namespace sk
