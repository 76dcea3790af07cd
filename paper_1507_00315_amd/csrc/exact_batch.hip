// Persistent batched launch of the tuned exact kernel: many instances (n,
// variant) of uneven size in one kernel.  Wavefronts pull work items (instance,
// chunk) from a global atomic counter until the list is exhausted; each item is
// one chunk of one instance, evaluated by the specialisation compiled for that
// instance (a wave-uniform branch), and its residues are written to the item's
// output row.  The host adds the rows of each instance modulo its primes.
//
// The set of specialisations compiled into this kernel is SK_BATCH_CASES (the
// host keeps the same list); other instances are counted by separate launches.
#include "exact_v2_body.h"
#include "sk_batch.h"

namespace sk {

constexpr int kBatchInner = 4;

template <int V, int N>
__device__ __forceinline__ void batch_case(uint64_t chunk, const BatchInstance& in, double* out_row)
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
        for (int i = 0; i < P; ++i) out_row[i] = res[i];
    }
}

__global__ void __launch_bounds__(256) exact_batch_kernel(const BatchArgs a)
{
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
        const uint64_t item = uniform_u64(a.items[idx]);
        const int inst = (int)(item >> kBatchChunkBits);
        const uint64_t chunk = item & ((1ull << kBatchChunkBits) - 1);
        const BatchInstance& in = a.inst[inst];
        double* row = a.out + (uint64_t)idx * kMaxPrimes;
        switch (in.kind) {
#define SK_BATCH_CASE(KIND, V, N) \
    case KIND:                    \
        batch_case<V, N>(chunk, in, row); \
        break;
            SK_BATCH_CASES(SK_BATCH_CASE)
#undef SK_BATCH_CASE
            default:
                break;
        }
    }
}

}  // namespace sk

namespace sk {

hipError_t launch_exact_batch(unsigned blocks, hipStream_t stream, const BatchArgs& a)
{
    hipLaunchKernelGGL(exact_batch_kernel, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace sk
