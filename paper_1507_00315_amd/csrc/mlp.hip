// Learned proposal for the tempering chains: a small MLP over the chain state
// whose output is a distribution q(k, a' | C) over single-pair moves; the chain
// stays exact through the Metropolis-Hastings ratio q(C'->C) / q(C->C').
// Trained on chain states to match the heat-bath distribution over single-pair
// moves, p*(k, a') proportional to exp(-beta E(C with a_k = a')).
//
// Kernels here (fp32):
//   * mlp_features_kernel   state -> input vector (bin occupancy indicators,
//                           a_k / T, per-pair collision flags, beta, E / 2n)
//   * gemm_kernel           C = alpha * op(A) op(B) (+ bias, ReLU, ReLU mask,
//                           accumulate), MFMA v_mfma_f32_32x32x2f32 on 64x64 tiles
//   * gemm_nt_kernel        the same for large products whose operands are both
//                           contiguous along k, on 128x64 tiles with float4 loads
//   * colsum_kernel         bias gradients (column sums)
//   * mlp_target_grad_kernel  masked softmax of the logits, heat-bath target,
//                           cross-entropy and dL/dz = (q - p*) / B, one wave per state
//   * mlp_sample_kernel     draw (k, a') from q by inverting its cumulative
//                           distribution, build C', its energy change and log q
//   * mlp_logq_kernel       log q of the reverse move at C'
//   * mlp_accept_kernel     Metropolis-Hastings decision and write-back
//   * adam_kernel           one Adam step (Kingma and Ba, 2015)
//   * mlp_gather_kernel / mlp_words_kernel  select the chains of a ladder set
//                           that take learned moves, and draw their Philox words
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sk_mlp.h"
#include "sk_philox.h"

namespace sk {

typedef float float16v __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------ features

__device__ __forceinline__ int geo_diff(const MlpGeo& g, int k) { return g.variant == 1 ? k + 2 : k + 1; }
__device__ __forceinline__ bool geo_in(const MlpGeo& g, int p) { return p >= 1 && p <= g.T && ((g.pset >> (p - 1)) & 1); }

__global__ void __launch_bounds__(256) mlp_features_kernel(MlpGeo g, const uint8_t* __restrict__ states,
                                                           const float* __restrict__ beta, int B, float* __restrict__ X,
                                                           int ldx, int32_t* __restrict__ energy_out)
{
    __shared__ uint8_t occ_all[256 * 72];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B) return;
    uint8_t* occ = occ_all + threadIdx.x * 72;
    for (int p = 0; p <= g.T; ++p) occ[p] = 0;
    const uint8_t* s = states + (size_t)t * g.n;
    for (int k = 0; k < g.n; ++k) {
        occ[s[k]]++;
        occ[s[k] + geo_diff(g, k)]++;
    }
    float* x = X + (size_t)t * ldx;
    int E = 0;
    for (int p = 1; p <= g.T; ++p) {
        x[p - 1] = occ[p] > 0 ? 1.f : 0.f;
        if (geo_in(g, p) && occ[p] == 0) ++E;
    }
    for (int k = 0; k < g.n; ++k) {
        const int a = s[k];
        x[g.T + k] = (float)a / (float)g.T;
        x[g.T + g.n + k] = (occ[a] > 1 || occ[a + geo_diff(g, k)] > 1) ? 1.f : 0.f;
    }
    x[g.T + 2 * g.n] = beta[t];
    x[g.T + 2 * g.n + 1] = (float)E / (float)g.m;
    for (int c = g.T + 2 * g.n + 2; c < ldx; ++c) x[c] = 0.f;
    if (energy_out) energy_out[t] = E;
}

// ------------------------------------------------------------------ GEMM

constexpr int kTile = 64, kTk = 16;

// Element i (0..2047) of a 64 x kTk operand tile: its (row within the tile, k)
// pair.  Consecutive threads take consecutive addresses in memory: along the
// row index when that is the contiguous dimension, else along k.
__device__ __forceinline__ void tile_coords(int e, bool row_fast, int& rr, int& kk)
{
    if (row_fast) {
        rr = e % kTile;
        kk = e / kTile;
    } else {
        kk = e % kTk;
        rr = e / kTk;
    }
}

__global__ void __launch_bounds__(256) gemm_kernel(const GemmArgs a)
{
    __shared__ float As[kTk][kTile + 4];
    __shared__ float Bs[kTk][kTile + 4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const long m0 = (long)blockIdx.y * kTile, n0 = (long)blockIdx.x * kTile;
    // split-K: block z of gridDim.z takes the K range [k_lo, k_hi)
    const long kc = (a.K + gridDim.z - 1) / gridDim.z;
    const long kcr = (kc + kTk - 1) / kTk * kTk;
    const long k_lo = (long)blockIdx.z * kcr;
    const long k_hi = k_lo + kcr < a.K ? k_lo + kcr : a.K;
    float16v acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;

    const bool a_mfast = a.sam == 1;  // consecutive m contiguous in memory
    const bool b_nfast = a.sbn == 1;
    constexpr int kPer = kTile * kTk / 256;  // elements of each operand per thread
    // The next tile's elements are loaded into registers while the MFMAs work
    // on the current one (held in LDS), so the global loads' latency hides
    // behind the arithmetic.
    // (32-bit offsets: launch_gemm checks that every operand index fits)
    float ra[kPer], rb[kPer];
    const int M = (int)a.M, N = (int)a.N, kh = (int)k_hi;
    const int sam = (int)a.sam, sak = (int)a.sak, sbk = (int)a.sbk, sbn = (int)a.sbn;
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = tid + 256 * i;
            int mm, kk, nn, kb;
            tile_coords(e, a_mfast, mm, kk);
            tile_coords(e, b_nfast, nn, kb);
            const int gm = (int)m0 + mm, gk = k0 + kk, gn = (int)n0 + nn, gkb = k0 + kb;
            ra[i] = (gm < M && gk < kh) ? a.A[gm * sam + gk * sak] : 0.f;
            rb[i] = (gn < N && gkb < kh) ? a.B[gkb * sbk + gn * sbn] : 0.f;
        }
    };
    if (k_lo < k_hi) load((int)k_lo);
    for (int k0 = (int)k_lo; k0 < kh; k0 += kTk) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = tid + 256 * i;
            int mm, kk, nn, kb;
            tile_coords(e, a_mfast, mm, kk);
            tile_coords(e, b_nfast, nn, kb);
            As[kk][mm] = ra[i];
            Bs[kb][nn] = rb[i];
        }
        __syncthreads();
        if (k0 + kTk < kh) load(k0 + kTk);
#pragma unroll
        for (int kk = 0; kk < kTk; kk += 2) {
            const float av = As[kk + (lane >> 5)][wm * 32 + (lane & 31)];
            const float bv = Bs[kk + (lane >> 5)][wn * 32 + (lane & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = wn * 32 + (lane & 31);
        const long gm = m0 + row, gn = n0 + col;
        if (gridDim.z > 1) {
            // partial sums of this K range, combined by splitk_reduce_kernel
            if (gm < a.M && gn < a.N) a.ws[((long)blockIdx.z * a.M + gm) * a.N + gn] = acc[r];
            continue;
        }
        if (gm < a.M && gn < a.N) {
            float v = a.alpha * acc[r];
            if (a.bias) v += a.bias[gn];
            float* c = a.C + gm * a.scm + gn * a.scn;
            if (a.accumulate) v += *c;
            if (a.relu) v = v > 0.f ? v : 0.f;
            if (a.relu_ref && !(a.relu_ref[gm * a.scm + gn * a.scn] > 0.f)) v = 0.f;
            *c = v;
        }
    }
}

// Large products with both operands contiguous along k (A[m, k] at m*sam + k,
// B[k, n] at n*sbn + k: the forward passes X W^T): 128 x 64 output tiles,
// each wave a 64 x 32 quarter as two MFMA blocks sharing their B operand,
// operands loaded as float4 (the launcher checks K % 16 == 0, 16-byte
// alignment and the 32-bit index range).  The MFMAs take the k pairs in the
// same order as gemm_kernel's, so every output is bit-identical to it.
constexpr int kBigM = 128, kBigN = 64;

__global__ void __launch_bounds__(256) gemm_nt_kernel(const GemmArgs a)
{
    __shared__ float As[kTk][kBigM + 4];
    __shared__ float Bs[kTk][kBigN + 4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * kBigM, n0 = blockIdx.x * kBigN;
    const int M = (int)a.M, N = (int)a.N, K = (int)a.K, sam = (int)a.sam, sbn = (int)a.sbn;
    float16v acc[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[bi][r] = 0.f;

    // thread t loads k quad (t & 3) of A rows (t >> 2), (t >> 2) + 64 and of
    // B column (t >> 2)
    const int kq = tid & 3, rr = tid >> 2;
    float4 pa[2], pb;
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int gm = min(m0 + rr + 64 * i, M - 1);
            pa[i] = *reinterpret_cast<const float4*>(a.A + gm * sam + k0 + 4 * kq);
        }
        const int gn = min(n0 + rr, N - 1);
        pb = *reinterpret_cast<const float4*>(a.B + gn * sbn + k0 + 4 * kq);
    };
    load(0);
    for (int k0 = 0; k0 < K; k0 += kTk) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row = rr + 64 * i;
            const bool va = m0 + row < M;
            As[4 * kq + 0][row] = va ? pa[i].x : 0.f;
            As[4 * kq + 1][row] = va ? pa[i].y : 0.f;
            As[4 * kq + 2][row] = va ? pa[i].z : 0.f;
            As[4 * kq + 3][row] = va ? pa[i].w : 0.f;
        }
        {
            const bool vb = n0 + rr < N;
            Bs[4 * kq + 0][rr] = vb ? pb.x : 0.f;
            Bs[4 * kq + 1][rr] = vb ? pb.y : 0.f;
            Bs[4 * kq + 2][rr] = vb ? pb.z : 0.f;
            Bs[4 * kq + 3][rr] = vb ? pb.w : 0.f;
        }
        __syncthreads();
        if (k0 + kTk < K) load(k0 + kTk);
#pragma unroll
        for (int kk = 0; kk < kTk; kk += 2) {
            const int kr = kk + (lane >> 5), c = lane & 31;
            const float a0 = As[kr][wm * 64 + c], a1 = As[kr][wm * 64 + 32 + c];
            const float b0 = Bs[kr][wn * 32 + c];
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int gm = m0 + wm * 64 + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int gn = n0 + wn * 32 + (lane & 31);
            if (gm < M && gn < N) {
                float v = a.alpha * acc[bi][r];
                if (a.bias) v += a.bias[gn];
                float* cp = a.C + (long)gm * a.scm + (long)gn * a.scn;
                if (a.accumulate) v += *cp;
                if (a.relu) v = v > 0.f ? v : 0.f;
                if (a.relu_ref && !(a.relu_ref[(long)gm * a.scm + (long)gn * a.scn] > 0.f)) v = 0.f;
                *cp = v;
            }
        }
}

// Sum of the split-K partials in z order (deterministic) and the epilogue of
// gemm_kernel.
__global__ void __launch_bounds__(256) splitk_reduce_kernel(const GemmArgs a, int splits)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.M * a.N) return;
    const long gm = i / a.N, gn = i % a.N;
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += a.ws[(long)z * a.M * a.N + i];
    v *= a.alpha;
    if (a.bias) v += a.bias[gn];
    float* c = a.C + gm * a.scm + gn * a.scn;
    if (a.accumulate) v += *c;
    if (a.relu) v = v > 0.f ? v : 0.f;
    if (a.relu_ref && !(a.relu_ref[gm * a.scm + gn * a.scn] > 0.f)) v = 0.f;
    *c = v;
}

// column sums: out[n] = alpha * sum_m Y[m * ld + n].  One block per 64
// columns: wave w adds rows w, w + 4, ... in that order, with lane = column
// (coalesced 256-byte rows); the four partial sums meet in LDS.  The rows are
// loaded 16 at a time ahead of their additions, so the loads' latencies
// overlap while the order of the additions stays fixed.
__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ Y, long M, long N, long ld,
                                                     float alpha, float* __restrict__ out)
{
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long n = (long)blockIdx.x * 64 + lane;
    double s = 0.0;
    if (n < N) {
        constexpr int kAhead = 16;
        long m = wv;
        for (; m + 4 * (kAhead - 1) < M; m += 4 * kAhead) {
            float v[kAhead];
#pragma unroll
            for (int j = 0; j < kAhead; ++j) v[j] = Y[(m + 4 * j) * ld + n];
#pragma unroll
            for (int j = 0; j < kAhead; ++j) s += v[j];
        }
        for (; m < M; m += 4) s += Y[m * ld + n];
    }
    part[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && n < N) out[n] = (float)(alpha * (part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]));
}

// ------------------------------------------------------------------ softmax

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_sumf(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// E(C with pair k moved from ao to ap) - E(C), from the occupancy of C.
// Removing the pair empties ao / ao + d if they held one ball; adding it at ap
// then ap + d fills them if they were empty after the removal.
__device__ __forceinline__ int move_delta(const uint8_t* occ, int ao, int ap, int d)
{
    int de = (occ[ao] == 1) + (occ[ao + d] == 1);
    const int o1 = occ[ap] - (ap == ao) - (ap == ao + d);
    const int o2 = occ[ap + d] - (ap + d == ao) - (ap + d == ao + d);
    de -= (o1 == 0) + (o2 == 0);
    return de;
}

// Walks the entries j = j0, j0 + step, ... of the n x T logit matrix keeping
// (k, c) = (j / T, j % T) up to date without a division per entry.
struct EntryWalk {
    int k, c, qs, rs, T;
    __device__ EntryWalk(int j0, int step, int T_) : k(j0 / T_), c(j0 % T_), qs(step / T_), rs(step % T_), T(T_) {}
    __device__ void next()
    {
        k += qs;
        c += rs;
        if (c >= T) {
            c -= T;
            ++k;
        }
    }
};

// placement index a' - 1 valid for pair k?
__device__ __forceinline__ bool move_valid(const MlpGeo& g, int k, int ap)
{
    const int d = geo_diff(g, k);
    return geo_in(g, ap) && geo_in(g, ap + d);
}

// One wave per state: dz = (q - p*) * scale on valid entries (0 elsewhere),
// loss[state] = -sum p* log q.  z is overwritten by dz.
__global__ void __launch_bounds__(256) mlp_target_grad_kernel(MlpGeo g, const uint8_t* __restrict__ states,
                                                              const float* __restrict__ beta, int B,
                                                              float* __restrict__ Z, int ldz, float scale,
                                                              float* __restrict__ loss)
{
    __shared__ uint8_t occ_all[4][72];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int t = blockIdx.x * 4 + wv;
    if (t >= B) return;
    uint8_t* occ = occ_all[wv];
    const uint8_t* s = states + (size_t)t * g.n;
    // the occupancy lives in this wave's own LDS row; a wave's LDS accesses
    // complete in program order, so a wave barrier (no workgroup barrier: waves
    // of the last block may have left) orders the writes before the reads
    for (int p = lane; p <= g.T; p += 64) occ[p] = 0;
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        for (int k = 0; k < g.n; ++k) {
            occ[s[k]]++;
            occ[s[k] + geo_diff(g, k)]++;
        }
    }
    __builtin_amdgcn_wave_barrier();
    int E = 0;
    for (int p = 1 + lane; p <= g.T; p += 64)
        if (geo_in(g, p) && occ[p] == 0) ++E;
    for (int o = 32; o >= 1; o >>= 1) E += __shfl_xor(E, o, 64);
    const float bt = beta[t];
    float* z = Z + (size_t)t * ldz;
    const int D = g.n * g.T;
    // pass 1: maxima of z and of -beta E'
    float zmax = -INFINITY, emin = INFINITY;
    EntryWalk w1(lane, 64, g.T);
    for (int j = lane; j < D; j += 64, w1.next()) {
        const int k = w1.k, ap = w1.c + 1;
        if (!move_valid(g, k, ap)) continue;
        zmax = fmaxf(zmax, z[j]);
        const int de = move_delta(occ, s[k], ap, geo_diff(g, k));
        emin = fminf(emin, (float)(E + de));
    }
    zmax = wave_max(zmax);
    emin = -wave_max(-emin);
    // pass 2: normalisers
    float zs = 0.f, ps = 0.f;
    EntryWalk w2(lane, 64, g.T);
    for (int j = lane; j < D; j += 64, w2.next()) {
        const int k = w2.k, ap = w2.c + 1;
        if (!move_valid(g, k, ap)) continue;
        zs += __expf(z[j] - zmax);
        const int de = move_delta(occ, s[k], ap, geo_diff(g, k));
        ps += __expf(-bt * ((float)(E + de) - emin));
    }
    zs = wave_sumf(zs);
    ps = wave_sumf(ps);
    const float lzs = __logf(zs);
    // pass 3: gradient and loss
    float l = 0.f;
    EntryWalk w3(lane, 64, g.T);
    for (int j = lane; j < D; j += 64, w3.next()) {
        const int k = w3.k, ap = w3.c + 1;
        if (!move_valid(g, k, ap)) {
            z[j] = 0.f;
            continue;
        }
        const int de = move_delta(occ, s[k], ap, geo_diff(g, k));
        const float pt = __expf(-bt * ((float)(E + de) - emin)) / ps;
        const float lq = z[j] - zmax - lzs;
        l -= pt * lq;
        z[j] = (__expf(lq) - pt) * scale;
    }
    l = wave_sumf(l);
    if (lane == 0 && loss) loss[t] = l;
}

// One wave per state: sample (k, a') from the masked softmax of z with the
// uniform word u (inverse cumulative distribution in lane order of j), write
// C' into states_new, the move and log q(k, a' | C).  The state's logits are
// read from HBM once, coalesced, into LDS (entry j at j + j/32, so that the
// lanes' runs of 32 consecutive entries fall in distinct banks); every pass
// reads them there.
constexpr int kMaxD = 32 * 64;  // n T for n <= 32 pairs

__global__ void __launch_bounds__(256) mlp_sample_kernel(MlpGeo g, const uint8_t* __restrict__ states,
                                                         const float* __restrict__ Z, int ldz,
                                                         const uint32_t* __restrict__ uword, int B,
                                                         uint8_t* __restrict__ states_new,
                                                         int32_t* __restrict__ move_k, int32_t* __restrict__ move_old,
                                                         float* __restrict__ logq_fwd)
{
    __shared__ float zl_all[4][kMaxD + kMaxD / 32];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int t = blockIdx.x * 4 + wv;
    if (t >= B) return;
    const float* z = Z + (size_t)t * ldz;
    float* zl = zl_all[wv];
    const int D = g.n * g.T;
    for (int j = lane; j < D; j += 64) zl[j + (j >> 5)] = z[j];
    // the wave's own LDS writes complete before any lane reads them
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float zmax = -INFINITY;
    EntryWalk w1(lane, 64, g.T);
    for (int j = lane; j < D; j += 64, w1.next())
        if (move_valid(g, w1.k, w1.c + 1)) zmax = fmaxf(zmax, zl[j + (j >> 5)]);
    zmax = wave_max(zmax);
    // each lane owns a contiguous run of entries [lane*R, lane*R + R)
    const int R = (D + 63) / 64;
    float part = 0.f;
    EntryWalk w2(lane * R, 1, g.T);
    for (int i = 0; i < R; ++i, w2.next()) {
        const int j = lane * R + i;
        if (j < D && move_valid(g, w2.k, w2.c + 1)) part += __expf(zl[j + (j >> 5)] - zmax);
    }
    // exclusive prefix over lanes
    float incl = part;
    for (int o = 1; o < 64; o <<= 1) {
        const float v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    const float total = __shfl(incl, 63, 64);
    const float excl = incl - part;
    const float target_mass = ((float)uword[t] * 2.3283064365386963e-10f) * total;
    // the lane whose run holds the target (last lane with excl <= target and mass > 0)
    int owner = (excl <= target_mass && part > 0.f) ? lane : -1;
    for (int o = 32; o >= 1; o >>= 1) owner = max(owner, __shfl_xor(owner, o, 64));
    int chosen = -1;
    if (lane == owner) {
        float c = excl;
        int last_valid = -1;
        EntryWalk w3(lane * R, 1, g.T);
        for (int i = 0; i < R; ++i, w3.next()) {
            const int j = lane * R + i;
            if (j >= D || !move_valid(g, w3.k, w3.c + 1)) continue;
            last_valid = j;
            c += __expf(zl[j + (j >> 5)] - zmax);
            if (c > target_mass) {
                chosen = j;
                break;
            }
        }
        if (chosen < 0) chosen = last_valid;
    }
    chosen = __shfl(chosen, owner < 0 ? 0 : owner, 64);
    if (lane == 0) {
        const uint8_t* s = states + (size_t)t * g.n;
        // no mass at all (non-finite logits): propose staying put, which the
        // acceptance test then keeps
        if (chosen < 0) chosen = s[0] - 1;
        const int k = chosen / g.T, ap = chosen % g.T + 1;
        uint8_t* sn = states_new + (size_t)t * g.n;
        for (int q = 0; q < g.n; ++q) sn[q] = s[q];
        move_k[t] = k;
        move_old[t] = s[k];
        sn[k] = (uint8_t)ap;
        logq_fwd[t] = z[chosen] - zmax - __logf(total);
    }
}

// log q(k, a_old | C') from the logits at C'
__global__ void __launch_bounds__(256) mlp_logq_kernel(MlpGeo g, const float* __restrict__ Z, int ldz,
                                                       const int32_t* __restrict__ move_k,
                                                       const int32_t* __restrict__ move_old, int B,
                                                       float* __restrict__ logq_rev)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int t = blockIdx.x * 4 + wv;
    if (t >= B) return;
    const float* z = Z + (size_t)t * ldz;
    const int D = g.n * g.T;
    float zmax = -INFINITY;
    EntryWalk w1(lane, 64, g.T);
    for (int j = lane; j < D; j += 64, w1.next())
        if (move_valid(g, w1.k, w1.c + 1)) zmax = fmaxf(zmax, z[j]);
    zmax = wave_max(zmax);
    float zs = 0.f;
    EntryWalk w2(lane, 64, g.T);
    for (int j = lane; j < D; j += 64, w2.next())
        if (move_valid(g, w2.k, w2.c + 1)) zs += __expf(z[j] - zmax);
    zs = wave_sumf(zs);
    if (lane == 0) logq_rev[t] = z[move_k[t] * g.T + move_old[t] - 1] - zmax - __logf(zs);
}

// Metropolis-Hastings decision for chain t: accept C' with probability
// min(1, exp(-beta (E' - E)) q(k, a_old | C') / q(k, a' | C)); the uniform is
// word * 2^-32.  The accepted configuration is written to row dst(t) of dst:
// t itself when nsel == 0, else (c / nsel) * M + j0 + c % nsel with
// c = base + t (the chain's place among ladders x levels).  acc_count[row]
// counts accepted moves that change the configuration.
__global__ void __launch_bounds__(256) mlp_accept_kernel(int n, const uint8_t* __restrict__ proposed,
                                                         const int32_t* __restrict__ e_old,
                                                         const int32_t* __restrict__ e_new,
                                                         const float* __restrict__ logq_fwd,
                                                         const float* __restrict__ logq_rev,
                                                         const float* __restrict__ beta,
                                                         const uint32_t* __restrict__ uword, int B, int M, int j0,
                                                         int nsel, long base, uint8_t* __restrict__ dst,
                                                         uint64_t* __restrict__ acc_count,
                                                         uint8_t* __restrict__ accepted)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B) return;
    const float la = -beta[t] * (float)(e_new[t] - e_old[t]) + logq_rev[t] - logq_fwd[t];
    const bool acc = la >= 0.f || (float)uword[t] * 2.3283064365386963e-10f < __expf(la);
    const long c = base + t;
    const size_t row = nsel == 0 ? (size_t)t : (size_t)(c / nsel) * M + j0 + c % nsel;
    if (accepted) accepted[t] = acc ? 1 : 0;
    if (acc) {
        bool changed = false;
        for (int k = 0; k < n; ++k) {
            const uint8_t v = proposed[(size_t)t * n + k];
            changed |= dst[row * n + k] != v;
            dst[row * n + k] = v;
        }
        if (acc_count && changed) acc_count[row] += 1;
    }
}

// Chain c = base + t of the learned set (levels j0..M-1 of every ladder, c =
// ladder * nsel + level - j0): copy its configuration and inverse temperature
// into row t of the compact batch.
__global__ void __launch_bounds__(256) mlp_gather_kernel(int n, const uint8_t* __restrict__ all, int M, int j0,
                                                         int nsel, long base, const float* __restrict__ beta_level,
                                                         int B, uint8_t* __restrict__ sel,
                                                         float* __restrict__ beta_sel)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B) return;
    const long c = base + t;
    const size_t row = (size_t)(c / nsel) * M + j0 + c % nsel;
    for (int k = 0; k < n; ++k) sel[(size_t)t * n + k] = all[row * n + k];
    beta_sel[t] = beta_level[j0 + c % nsel];
}

// Philox words of learned move `step` for chain c = base + t: counter (step,
// 0xFFFFFFFE, ladder, level); word 0 picks the move, word 1 decides it.
__global__ void __launch_bounds__(256) mlp_words_kernel(uint64_t seed, uint32_t step, int j0, int nsel, long base,
                                                        int B, uint32_t* __restrict__ w_pick,
                                                        uint32_t* __restrict__ w_acc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B) return;
    const long c = base + t;
    uint32_t r[4];
    philox4x32_10(step, 0xFFFFFFFEu, (uint32_t)(c / nsel), (uint32_t)(j0 + c % nsel), (uint32_t)seed,
                  (uint32_t)(seed >> 32), r);
    w_pick[t] = r[0];
    w_acc[t] = r[1];
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ P, const float* __restrict__ G,
                                                   float* __restrict__ M, float* __restrict__ V, long n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float m = b1 * M[i] + (1.f - b1) * g;
    const float v = b2 * V[i] + (1.f - b2) * g * g;
    M[i] = m;
    V[i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ------------------------------------------------------------------ launchers

hipError_t launch_features(const MlpGeo& g, const uint8_t* states, const float* beta, int B, float* X, int ldx,
                           int32_t* energy, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_features_kernel, dim3((B + 255) / 256), dim3(256), 0, s, g, states, beta, B, X, ldx,
                       energy);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& a, hipStream_t s)
{
    if (a.M <= 0 || a.N <= 0) return hipSuccess;
    // the kernel indexes A and B with 32-bit offsets
    auto span = [](long rows, long sr, long cols, long sc) {
        return (rows - 1) * (sr < 0 ? -sr : sr) + (cols - 1) * (sc < 0 ? -sc : sc);
    };
    if (a.K > 0 && (span(a.M, a.sam, a.K, a.sak) >= (1L << 31) || span(a.K, a.sbk, a.N, a.sbn) >= (1L << 31) ||
                    a.sam < 0 || a.sak < 0 || a.sbk < 0 || a.sbn < 0))
        return hipErrorInvalidValue;
    const long tiles = ((a.N + kTile - 1) / kTile) * ((a.M + kTile - 1) / kTile);
    // split K when the tiles alone leave most of the 256 CUs idle and K is
    // long; the partials go to the workspace (splits x M x N floats)
    // large products with both operands contiguous along k: 128 x 64 tiles
    const long big_tiles = ((a.N + kBigN - 1) / kBigN) * ((a.M + kBigM - 1) / kBigM);
    if (a.sak == 1 && a.sbk == 1 && a.K % kTk == 0 && a.sam % 4 == 0 && a.sbn % 4 == 0 &&
        (reinterpret_cast<uintptr_t>(a.A) & 15) == 0 && (reinterpret_cast<uintptr_t>(a.B) & 15) == 0 &&
        big_tiles >= 1024) {
        hipLaunchKernelGGL(gemm_nt_kernel, dim3((unsigned)((a.N + kBigN - 1) / kBigN),
                                                (unsigned)((a.M + kBigM - 1) / kBigM)),
                           dim3(256), 0, s, a);
        return hipGetLastError();
    }
    int splits = 1;
    if (a.ws && tiles < 256 && a.K >= 8 * kTk) {
        const long by_occ = (512 + tiles - 1) / tiles, by_k = a.K / (4 * kTk);
        splits = (int)std::min<long>({16, by_occ, by_k, a.ws_floats / (a.M * a.N)});
        if (splits < 2) splits = 1;
    }
    hipLaunchKernelGGL(gemm_kernel,
                       dim3((unsigned)((a.N + kTile - 1) / kTile), (unsigned)((a.M + kTile - 1) / kTile), splits),
                       dim3(256), 0, s, a);
    if (splits > 1) {
        const long mn = a.M * a.N;
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, a, splits);
    }
    return hipGetLastError();
}

hipError_t launch_colsum(const float* Y, long M, long N, long ld, float alpha, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((N + 63) / 64)), dim3(256), 0, s, Y, M, N, ld, alpha, out);
    return hipGetLastError();
}

hipError_t launch_target_grad(const MlpGeo& g, const uint8_t* states, const float* beta, int B, float* Z, int ldz,
                              float scale, float* loss, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_target_grad_kernel, dim3((B + 3) / 4), dim3(256), 0, s, g, states, beta, B, Z, ldz, scale,
                       loss);
    return hipGetLastError();
}

hipError_t launch_sample(const MlpGeo& g, const uint8_t* states, const float* Z, int ldz, const uint32_t* uword,
                         int B, uint8_t* states_new, int32_t* move_k, int32_t* move_old, float* logq_fwd,
                         hipStream_t s)
{
    hipLaunchKernelGGL(mlp_sample_kernel, dim3((B + 3) / 4), dim3(256), 0, s, g, states, Z, ldz, uword, B, states_new,
                       move_k, move_old, logq_fwd);
    return hipGetLastError();
}

hipError_t launch_logq(const MlpGeo& g, const float* Z, int ldz, const int32_t* move_k, const int32_t* move_old,
                       int B, float* logq_rev, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_logq_kernel, dim3((B + 3) / 4), dim3(256), 0, s, g, Z, ldz, move_k, move_old, B, logq_rev);
    return hipGetLastError();
}

hipError_t launch_adam(float* P, const float* G, float* M, float* V, long n, float lr, float b1, float b2, float eps,
                       int t, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, G, M, V, n, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_accept(int n, const uint8_t* proposed, const int32_t* e_old, const int32_t* e_new,
                         const float* logq_fwd, const float* logq_rev, const float* beta, const uint32_t* uword, int B,
                         int M, int j0, int nsel, long base, uint8_t* dst, uint64_t* acc_count, uint8_t* accepted,
                         hipStream_t s)
{
    hipLaunchKernelGGL(mlp_accept_kernel, dim3((B + 255) / 256), dim3(256), 0, s, n, proposed, e_old, e_new, logq_fwd,
                       logq_rev, beta, uword, B, M, j0, nsel, base, dst, acc_count, accepted);
    return hipGetLastError();
}

hipError_t launch_gather(int n, const uint8_t* all, int M, int j0, int nsel, long base, const float* beta_level,
                         int B, uint8_t* sel, float* beta_sel, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_gather_kernel, dim3((B + 255) / 256), dim3(256), 0, s, n, all, M, j0, nsel, base,
                       beta_level, B, sel, beta_sel);
    return hipGetLastError();
}

hipError_t launch_words(uint64_t seed, uint32_t step, int j0, int nsel, long base, int B, uint32_t* w_pick,
                        uint32_t* w_acc, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_words_kernel, dim3((B + 255) / 256), dim3(256), 0, s, seed, step, j0, nsel, base, B,
                       w_pick, w_acc);
    return hipGetLastError();
}

}  // namespace sk
