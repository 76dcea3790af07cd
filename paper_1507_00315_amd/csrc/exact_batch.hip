// Persistent batched launch of the tuned exact kernel: many instances (n,
// variant) of uneven size in one kernel.  Wavefronts pull work items (instance,
// chunk) from a global atomic counter until the list is exhausted; each item is
// one chunk of one instance, evaluated by the specialisation compiled for that
// instance (a wave-uniform branch).  Reduction: the wave's residues (butterfly
// over the lanes) go into a per-workgroup LDS table, one (low word, carries)
// pair per instance and prime; when the workgroup's waves have left the loop
// the table is added to the device accumulators.  The host reads one 128-bit
// sum per instance and prime and reduces it modulo the prime.
//
// The set of specialisations compiled into this kernel is SK_BATCH_CASES (the
// host keeps the same list); other instances are counted by separate launches.
#include <algorithm>

#include "exact_v2_body.h"
#include "sk_batch.h"

namespace sk {

constexpr int kBatchInner = 4;

template <int V, int N>
__device__ __forceinline__ void batch_case(uint64_t chunk, const BatchInstance& in, unsigned long long* tab)
{
    constexpr int P = primes_for(N);
    double pr[P], pinv[P], res[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        pr[i] = in.prime[i];
        pinv[i] = in.pinv[i];
    }
    exact_v2_chunk<V, N, P, kBatchInner>(chunk, in.jb, in.rev, pr, pinv, res);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < P; ++i) add_u128(tab + 2 * i, canonical_residue(res[i], pr[i], pinv[i]));
    }
}

constexpr int kBatchTab = kBatchMaxInstances * kMaxPrimes * 2;

__global__ void __launch_bounds__(256) exact_batch_kernel(const BatchArgs a)
{
    __shared__ unsigned long long tab[kBatchTab];
    for (int i = threadIdx.x; i < kBatchTab; i += blockDim.x) tab[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    // A wave can claim at most n_items items; the trip bound guarantees that
    // every wave leaves the loop whatever the counter returns.
    for (uint64_t trip = 0; trip <= a.n_items; ++trip) {
        // Every lane takes part in the atomic (lane 0 adds 1, the others 0) and
        // the claimed index is read from lane 0 explicitly: no lane-dependent
        // branch precedes the broadcast, so no lane can reach it without lane 0's
        // value.
        const uint32_t old = atomicAdd(a.counter, lane == 0 ? 1u : 0u);
        const uint32_t idx = __builtin_amdgcn_readlane(old, 0);
        if (idx >= a.n_items) break;  // every wave leaves once the list is exhausted
        int s = 0;
        while (s + 1 < a.nslots && idx >= a.first[s + 1]) ++s;  // wave-uniform
        const int inst = a.slot_inst[s];
        const uint64_t chunk = idx - a.first[s];
        const BatchInstance& in = a.inst[inst];
        unsigned long long* t = tab + inst * kMaxPrimes * 2;
        switch (in.kind) {
#define SK_BATCH_CASE(KIND, V, N) \
    case KIND:                    \
        batch_case<V, N>(chunk, in, t); \
        break;
            SK_BATCH_CASES(SK_BATCH_CASE)
#undef SK_BATCH_CASE
            default:
                break;
        }
    }
    __syncthreads();  // every wave of the workgroup has left the loop
    for (int i = threadIdx.x; i < kBatchTab / 2; i += blockDim.x) {
        const unsigned long long lo = tab[2 * i], hi = tab[2 * i + 1];
        if (lo | hi) add_u128_pair(a.acc + 2 * i, lo, hi);
    }
}

}  // namespace sk

namespace sk {

hipError_t launch_exact_batch(unsigned blocks, hipStream_t stream, const BatchArgs& a)
{
    hipLaunchKernelGGL(exact_batch_kernel, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

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
    const unsigned blocks = (unsigned)std::min<uint64_t>(64, (n + 255) / 256);
    hipLaunchKernelGGL(zero_words_kernel, dim3(blocks), dim3(256), 0, stream, (unsigned long long*)p, n);
    return hipGetLastError();
}

}  // namespace sk
