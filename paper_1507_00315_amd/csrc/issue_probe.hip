// Vector-instruction issue rates of one SIMD on gfx950: a calibration
// program for the cost models of the kernels (the tempering kernel runs one
// wave per SIMD, the exact kernels eight).
//
// Each wave runs a loop of 32 vector instructions per trip, as eight
// independent chains (throughput) or one chain (latency).  Kinds: the 32-bit
// integer add, the 64-bit multiply-add and the three-input bit operation of
// the tempering loop; the packed 16-bit add and multiply, the 24-bit
// multiply, the int-to-fp64 conversion and the fp64 fma, add and multiply of
// the exact kernels' walk; and a mix of those seven in the walk's
// proportions (per 32: 8 packed adds, 4 of each other).  The launch holds 1,
// 4 or 8 waves per SIMD (1024, 4096 or 8192 single-wave workgroups on 256 CUs
// x 4 SIMDs).  Printed per case: cycles at 2.4 GHz per wave-instruction per
// SIMD, i.e. kernel time x 2.4e9 / (instructions per wave x waves per SIMD).
// Every thread writes one word to out[blockIdx.x * 64 + threadIdx.x]; the
// buffer holds 8192 x 64 words.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#define CHECK(x)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            fprintf(stderr, "issue_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                         \
        }                                                                                     \
    } while (0)

enum Kind {
    kAdd,
    kMad64,
    kBitop3,
    kPkAdd16,
    kPkMul16,
    kMul24,
    kCvtF64,
    kFmaF64,
    kAddF64,
    kMulF64,
    kMix,
    kKinds
};

template <int KIND>
__device__ __forceinline__ void one(int j, uint32_t (&x)[8], uint64_t (&y)[8], double (&z)[8], uint32_t m, double dm)
{
    if constexpr (KIND == kAdd) {
        asm volatile("v_add_u32 %0, %1, %2" : "=v"(x[j]) : "v"(x[j]), "v"(m));
    } else if constexpr (KIND == kMad64) {
        uint64_t carry;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(y[j]), "=s"(carry) : "v"((uint32_t)y[j]), "v"(m), "v"(y[j]));
    } else if constexpr (KIND == kBitop3) {
        asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(x[j]) : "v"(x[j]), "v"(m), "v"(x[(j + 1) & 7]));
    } else if constexpr (KIND == kPkAdd16) {
        asm volatile("v_pk_add_u16 %0, %1, %2" : "=v"(x[j]) : "v"(x[j]), "v"(m));
    } else if constexpr (KIND == kPkMul16) {
        asm volatile("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(x[j]) : "v"(x[j]), "v"(m));
    } else if constexpr (KIND == kMul24) {
        asm volatile("v_mul_i32_i24 %0, %1, %2" : "=v"(x[j]) : "v"(x[j]), "v"(m));
    } else if constexpr (KIND == kCvtF64) {
        asm volatile("v_cvt_f64_i32 %0, %1" : "=v"(z[j]) : "v"(x[j]));
    } else if constexpr (KIND == kFmaF64) {
        asm volatile("v_fma_f64 %0, %1, %2, %3" : "=v"(z[j]) : "v"(z[j]), "v"(dm), "v"(z[j]));
    } else if constexpr (KIND == kAddF64) {
        asm volatile("v_add_f64 %0, %1, %2" : "=v"(z[j]) : "v"(z[j]), "v"(dm));
    } else if constexpr (KIND == kMulF64) {
        asm volatile("v_mul_f64 %0, %1, %2" : "=v"(z[j]) : "v"(z[j]), "v"(dm));
    }
}

template <int KIND, bool CHAIN>
__global__ void __launch_bounds__(64) probe(uint32_t* out, int trips, uint32_t seed)
{
    uint32_t x[8];
    uint64_t y[8];
    double z[8];
    const uint32_t m = 0xD2511F53u ^ (seed & 1);
    const double dm = 0.5 + (double)(seed & 1);
    for (int j = 0; j < 8; ++j) {
        x[j] = threadIdx.x * 7919u + j * 104729u + seed;
        y[j] = x[j];
        z[j] = (double)x[j];
    }
    for (int t = 0; t < trips; ++t) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int j0 = 0; j0 < 8; ++j0) {
                const int j = CHAIN ? 0 : j0;
                if constexpr (KIND == kMix) {
                    // per 8: two packed adds, one of each other kind of the walk
                    if (j0 < 2) one<kPkAdd16>(j, x, y, z, m, dm);
                    else if (j0 == 2) one<kPkMul16>(j, x, y, z, m, dm);
                    else if (j0 == 3) one<kMul24>(j, x, y, z, m, dm);
                    else if (j0 == 4) one<kCvtF64>(j, x, y, z, m, dm);
                    else if (j0 == 5) one<kFmaF64>(j, x, y, z, m, dm);
                    else if (j0 == 6) one<kAddF64>(j, x, y, z, m, dm);
                    else one<kMulF64>(j, x, y, z, m, dm);
                } else {
                    one<KIND>(j, x, y, z, m, dm);
                }
            }
        }
    }
    uint32_t s = 0;
    for (int j = 0; j < 8; ++j) s += x[j] + (uint32_t)y[j] + (uint32_t)(y[j] >> 32) + (uint32_t)(int)z[j];
    out[blockIdx.x * 64 + threadIdx.x] = s;
}

typedef void (*ProbeFn)(uint32_t*, int, uint32_t);

struct Case {
    ProbeFn fn;
    const char* name;
    int chains;
};

int main()
{
    const Case cases[] = {
        {probe<kAdd, false>, "v_add_u32", 8},          {probe<kAdd, true>, "v_add_u32", 1},
        {probe<kMad64, false>, "v_mad_u64_u32", 8},    {probe<kMad64, true>, "v_mad_u64_u32", 1},
        {probe<kBitop3, false>, "v_bitop3_b32", 8},    {probe<kBitop3, true>, "v_bitop3_b32", 1},
        {probe<kPkAdd16, false>, "v_pk_add_u16", 8},   {probe<kPkMul16, false>, "v_pk_mul_lo_u16", 8},
        {probe<kMul24, false>, "v_mul_i32_i24", 8},    {probe<kCvtF64, false>, "v_cvt_f64_i32", 8},
        {probe<kFmaF64, false>, "v_fma_f64", 8},       {probe<kAddF64, false>, "v_add_f64", 8},
        {probe<kMulF64, false>, "v_mul_f64", 8},       {probe<kMix, false>, "walk mix", 8},
    };
    const int n_cases = (int)(sizeof(cases) / sizeof(cases[0]));
    const int max_grid = 8192, trips = 1 << 16;
    uint32_t* out = nullptr;
    CHECK(hipMalloc(&out, (size_t)max_grid * 64 * sizeof(uint32_t)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int grid : {1024, 4096, 8192}) {
        for (int k = 0; k < n_cases; ++k) {
            hipLaunchKernelGGL(cases[k].fn, dim3(grid), dim3(64), 0, 0, out, 16, 1u);  // warm-up
            CHECK(hipGetLastError());
            CHECK(hipDeviceSynchronize());
            CHECK(hipEventRecord(e0, 0));
            hipLaunchKernelGGL(cases[k].fn, dim3(grid), dim3(64), 0, 0, out, trips, 1u);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1, 0));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            const double per_wave = (double)trips * 32.0, waves_per_simd = grid / 1024.0;
            printf("{\"instruction\": \"%s\", \"chains\": %d, \"waves_per_simd\": %d, \"ms\": %.3f, "
                   "\"cycles_per_wave_instr_per_simd\": %.3f}\n",
                   cases[k].name, cases[k].chains, grid / 1024, ms,
                   ms * 1e-3 * 2.4e9 / (per_wave * waves_per_simd));
            fflush(stdout);
        }
    }
    CHECK(hipFree(out));
    return 0;
}
