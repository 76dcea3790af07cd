// Shared definitions of the persistent batched launch (host and device).
#pragma once

#include <stdint.h>

#include "sk_internal.h"

namespace sk {

// Specialisations compiled into the persistent batched kernel:
// X(kind, variant, n).  The set is the mixed-instance workload (Skolem n = 16,
// 17, 20, 21; Langford n = 15, 16, 19, 20; hooked n = 14, 15).
#define SK_BATCH_CASES(X) \
    X(0, 0, 16)           \
    X(1, 0, 17)           \
    X(2, 0, 20)           \
    X(3, 0, 21)           \
    X(4, 1, 15)           \
    X(5, 1, 16)           \
    X(6, 1, 19)           \
    X(7, 1, 20)           \
    X(8, 2, 14)           \
    X(9, 2, 15)

constexpr int kBatchMaxInstances = 16;

struct BatchInstance {
    RevMasks rev;  // reversal weights of the instance (r = 0: none)
    int32_t kind;  // case of SK_BATCH_CASES
    int32_t jb;    // job bits enumerated inside one chunk
    double prime[kMaxPrimes];
    double pinv[kMaxPrimes];
};

// Work items are numbered 0 .. n_items - 1 in the order they are handed out:
// processing slot s (instances sorted by work per item, largest first) owns
// items [first[s], first[s + 1]), item first[s] + c being chunk c of instance
// slot_inst[s].  Residue sums go to acc, kBatchMaxInstances x kMaxPrimes
// (low word, carries) pairs, instance-major.
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

}  // namespace sk
