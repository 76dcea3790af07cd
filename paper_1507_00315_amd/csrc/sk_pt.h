// Shared definitions of the tempering kernels (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

constexpr int kPtMaxLevels = 64;
constexpr int kPtMaxN = 40;  // pairs (positions up to 2n + 1 <= 81, bytes in LDS)

struct PtArgs {
    int32_t n, variant, top, levels;
    int32_t slot_bytes;       // LDS bytes per configuration slot
    uint32_t ladder_base;     // ladder id of block 0
    uint64_t seed;
    uint64_t it_begin, it_end;
    const uint32_t* move_thr;  // levels x 2: floor(2^32 exp(-beta_j e)), e = 1, 2
    const uint32_t* swap_thr;  // levels x (top+1): floor(2^32 exp(-(beta_{j+1}-beta_j) e))
    const uint8_t* state_in;   // ladders x levels x n placements, or nullptr (fresh start)
    uint8_t* state_out;        // ladders x levels x n
    int32_t* energy_out;       // ladders x levels
    uint64_t* hist_out;        // ladders x levels x (top+1), added to
    uint64_t* move_acc;        // ladders x levels, added to
    uint64_t* swap_acc;        // ladders x levels (exchange of j and j+1), added to
};

hipError_t launch_pt_ladders(unsigned ladders, size_t lds_bytes, hipStream_t stream, const PtArgs& a);

}  // namespace sk
