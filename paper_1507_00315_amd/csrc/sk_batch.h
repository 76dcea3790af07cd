// Shared definitions of the persistent batched launch (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_internal.h"

namespace sk {

// Groups of the batched launch.  Group g's persistent kernel holds the tuned
// body of every (variant, n) that batch_group_of assigns to it (a wave-uniform
// branch picks it per work item); a batched count runs one launch per group
// that holds instances.  Group 1 is the mixed-instance workload (Skolem 16,
// 17, 20, 21; Langford 15, 16, 19, 20; hooked 14, 15) alone: a kernel's
// registers are the most any of its bodies needs, and these ten need the
// fewest; group 3 holds the other bodies with 14 <= n <= 21.
constexpr int kBatchGroups = 4;

__host__ __device__ constexpr int batch_group_of(int variant, int n)
{
    if ((variant == 0 && (n == 16 || n == 17 || n == 20 || n == 21)) ||
        (variant == 1 && (n == 15 || n == 16 || n == 19 || n == 20)) || (variant == 2 && (n == 14 || n == 15)))
        return 1;
    if (variant < 0 || variant > 2) return -1;
    if (n >= 12 && n <= 13) return 0;
    if (n >= 14 && n <= 21) return 3;
    if (n >= 22 && n <= 25) return 2;
    return -1;
}

// Smallest and largest n of a group.
__host__ __device__ constexpr int batch_group_lo(int g) { return g == 0 ? 12 : g == 2 ? 22 : 14; }
__host__ __device__ constexpr int batch_group_hi(int g) { return g == 0 ? 13 : g == 2 ? 25 : 21; }

constexpr int kBatchMaxInstances = 16;

struct BatchInstance {
    RevMasks rev;     // reversal weights of the instance (r = 0: none)
    int32_t variant;  // the specialisation: (variant, n)
    int32_t n;
    int32_t jb;       // job bits enumerated inside one chunk
    int32_t nprimes;  // primes of the instance (primes_for(n))
    double prime[kMaxPrimes];
    double pinv[kMaxPrimes];
};

// Work items are numbered 0 .. n_items - 1 in the order they are handed out:
// processing slot s (instances sorted by work per item, largest first) owns
// items [first[s], first[s + 1]).  With one prime per item (a kernel built
// with PPI = 1) item first[s] + c is chunk c / P, prime c % P of instance
// slot_inst[s]; with all primes per item (PPI = 0) it is chunk c.  Residue
// sums go to acc, kBatchMaxInstances x kMaxPrimes (low word, carries) pairs,
// instance-major.
struct BatchArgs {
    BatchInstance inst[kBatchMaxInstances];
    uint32_t first[kBatchMaxInstances + 1];
    int32_t slot_inst[kBatchMaxInstances];
    int32_t nslots;
    uint32_t n_items;
    uint32_t* counter;        // device: next item (set to 0 before the launch)
    unsigned long long* acc;  // device: accumulators (set to 0 before the launch)
};

// Device workspace of one batched launch: the accumulators, then the counter.
constexpr size_t kBatchAccBytes = (size_t)kBatchMaxInstances * kMaxPrimes * 2 * sizeof(unsigned long long);
constexpr size_t kBatchWsBytes = kBatchAccBytes + 256;

// Launcher of group g's kernel with ppi primes per work item (0: all of the
// instance's, 1: one); each build unit of exact_batch.hip registers its own.
using BatchLaunchFn = hipError_t (*)(unsigned blocks, hipStream_t stream, const BatchArgs& a);
int register_batch_kernel(int group, int ppi, BatchLaunchFn fn);

}  // namespace sk
