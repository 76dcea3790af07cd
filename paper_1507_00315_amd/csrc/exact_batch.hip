// Persistent batched launch of the tuned exact kernel: many instances (n,
// variant) of uneven size in one kernel.  Wavefronts pull work items (instance,
// chunk[, prime]) from a global atomic counter until the list is exhausted;
// each item is one chunk of one instance, evaluated by the specialisation
// compiled for that instance (a wave-uniform branch).  Reduction: the wave's
// residues (butterfly over the lanes) go into a per-workgroup LDS table, one
// (low word, carries) pair per instance and prime; when the workgroup's waves
// have left the loop the table is added to the device accumulators.  The host
// reads one 128-bit sum per instance and prime and reduces it modulo the prime.
//
// The build compiles this file once per group and primes-per-item setting,
//   -DSK_BATCH_GROUP=g -DSK_BATCH_PPI=p,
// each unit holding the tuned body of every (variant, n) of group g
// (batch_group_of in sk_batch.h) and registering its launcher with the host.
#include "exact_v2_body.h"
#include "sk_batch.h"

#ifndef SK_BATCH_GROUP
#define SK_BATCH_GROUP 1
#endif
#ifndef SK_BATCH_PPI
#define SK_BATCH_PPI 0
#endif

namespace sk {

constexpr int kBatchInner = 4;

template <int V, int N>
constexpr bool batch_supported()
{
    constexpr PlanCE P = make_plan_ce(N, V);
    return P.ok && P.n_lane == 6 && P.n_walk >= kBatchInner + 1;
}

// One work item of instance `in`: chunk `item` with all its primes (PPI = 0),
// or chunk item / P with prime item % P (PPI = 1).  Lane 0 adds the residues
// to the workgroup's table row `tab` of the instance.
template <int PPI, int V, int N>
__device__ __forceinline__ void batch_case(uint64_t item, const BatchInstance& in, unsigned long long* tab)
{
    constexpr int PN = primes_for(N);
    constexpr int P = PPI == 1 ? 1 : PN;
    const uint64_t chunk = PPI == 1 ? item / PN : item;
    const int p0 = PPI == 1 ? (int)(item % PN) : 0;  // wave-uniform
    double pr[P], pinv[P], res[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        pr[i] = in.prime[p0 + i];
        pinv[i] = in.pinv[p0 + i];
    }
    exact_v2_chunk<V, N, P, kBatchInner>(chunk, in.jb, in.rev, pr, pinv, res);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < P; ++i) add_u128(tab + 2 * (p0 + i), canonical_residue(res[i], pr[i], pinv[i]));
    }
}

// Branch to the specialisation of (V, n) among the n in [N, group G's highest]
// that belong to group G.
template <int G, int PPI, int V, int N>
__device__ __forceinline__ void dispatch_n(int n, uint64_t item, const BatchInstance& in, unsigned long long* tab)
{
    if constexpr (N <= batch_group_hi(G)) {
        if constexpr (batch_group_of(V, N) == G && batch_supported<V, N>()) {
            if (n == N) {
                batch_case<PPI, V, N>(item, in, tab);
                return;
            }
        }
        dispatch_n<G, PPI, V, N + 1>(n, item, in, tab);
    }
}

constexpr int kBatchTab = kBatchMaxInstances * kMaxPrimes * 2;

template <int G, int PPI>
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
        const uint64_t item = idx - a.first[s];
        const BatchInstance& in = a.inst[inst];
        unsigned long long* t = tab + inst * kMaxPrimes * 2;
        constexpr int lo = batch_group_lo(G);
        switch (in.variant) {
            case 0: dispatch_n<G, PPI, 0, lo>(in.n, item, in, t); break;
            case 1: dispatch_n<G, PPI, 1, lo>(in.n, item, in, t); break;
            case 2: dispatch_n<G, PPI, 2, lo>(in.n, item, in, t); break;
            default: break;
        }
    }
    __syncthreads();  // every wave of the workgroup has left the loop
    for (int i = threadIdx.x; i < kBatchTab / 2; i += blockDim.x) {
        const unsigned long long lo = tab[2 * i], hi = tab[2 * i + 1];
        if (lo | hi) add_u128_pair(a.acc + 2 * i, lo, hi);
    }
}

static hipError_t launch(unsigned blocks, hipStream_t stream, const BatchArgs& a)
{
    hipLaunchKernelGGL((exact_batch_kernel<SK_BATCH_GROUP, SK_BATCH_PPI>), dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

static const int registered = register_batch_kernel(SK_BATCH_GROUP, SK_BATCH_PPI, launch);

}  // namespace sk
