// Vector-instruction issue rates of one SIMD on gfx950: a calibration
// program for the cost model of the tempering kernel (one wave per SIMD).
//
// Each wave runs a loop of 32 vector instructions per trip, as eight
// independent chains (throughput) or one chain (latency), for three
// instructions: v_add_u32, v_mad_u64_u32 and v_bitop3_b32.  The launch holds
// 1 or 4 waves per SIMD (1024 or 4096 single-wave workgroups on 256 CUs x 4
// SIMDs).  Printed per case: cycles at 2.4 GHz per wave-instruction per
// SIMD, i.e. kernel time x 2.4e9 / (instructions per wave x waves per SIMD).
// Every thread writes one word to out[blockIdx.x * 64 + threadIdx.x]; the
// buffer holds grid x 64 words.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#define CHECK(x)                                                                      \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "issue_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

template <int KIND, bool CHAIN>
__global__ void __launch_bounds__(64) probe(uint32_t* out, int trips, uint32_t seed)
{
    uint32_t x[8];
    uint64_t y[8];
    const uint32_t m = 0xD2511F53u ^ (seed & 1);
    for (int j = 0; j < 8; ++j) {
        x[j] = threadIdx.x * 7919u + j * 104729u + seed;
        y[j] = x[j];
    }
    for (int t = 0; t < trips; ++t) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int j0 = 0; j0 < 8; ++j0) {
                const int j = CHAIN ? 0 : j0;
                if constexpr (KIND == 0) {
                    asm volatile("v_add_u32 %0, %1, %2" : "=v"(x[j]) : "v"(x[j]), "v"(m));
                } else if constexpr (KIND == 1) {
                    uint64_t carry;
                    asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4"
                                 : "=v"(y[j]), "=s"(carry)
                                 : "v"((uint32_t)y[j]), "v"(m), "v"(y[j]));
                } else {
                    asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96"
                                 : "=v"(x[j])
                                 : "v"(x[j]), "v"(m), "v"(x[(j + 1) & 7]));
                }
            }
        }
    }
    uint32_t s = 0;
    for (int j = 0; j < 8; ++j) s += x[j] + (uint32_t)y[j] + (uint32_t)(y[j] >> 32);
    out[blockIdx.x * 64 + threadIdx.x] = s;
}

typedef void (*ProbeFn)(uint32_t*, int, uint32_t);

int main()
{
    const ProbeFn fns[6] = {probe<0, false>, probe<0, true>, probe<1, false>,
                            probe<1, true>,  probe<2, false>, probe<2, true>};
    const char* names[6] = {"v_add_u32", "v_add_u32", "v_mad_u64_u32", "v_mad_u64_u32", "v_bitop3_b32",
                            "v_bitop3_b32"};
    const int max_grid = 4096, trips = 1 << 16;
    uint32_t* out = nullptr;
    CHECK(hipMalloc(&out, (size_t)max_grid * 64 * sizeof(uint32_t)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int grid : {1024, 4096}) {
        for (int k = 0; k < 6; ++k) {
            hipLaunchKernelGGL(fns[k], dim3(grid), dim3(64), 0, 0, out, 16, 1u);  // warm-up
            CHECK(hipGetLastError());
            CHECK(hipDeviceSynchronize());
            CHECK(hipEventRecord(e0, 0));
            hipLaunchKernelGGL(fns[k], dim3(grid), dim3(64), 0, 0, out, trips, 1u);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1, 0));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            const double per_wave = (double)trips * 32.0, waves_per_simd = grid / 1024.0;
            printf("{\"instruction\": \"%s\", \"chains\": %d, \"waves_per_simd\": %d, \"ms\": %.3f, "
                   "\"cycles_per_wave_instr_per_simd\": %.3f}\n",
                   names[k], (k & 1) ? 1 : 8, grid / 1024, ms, ms * 1e-3 * 2.4e9 / (per_wave * waves_per_simd));
            fflush(stdout);
        }
    }
    CHECK(hipFree(out));
    return 0;
}
