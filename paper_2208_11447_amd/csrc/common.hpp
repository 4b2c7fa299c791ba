// Shared device helpers of the skfab HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace skfab {

constexpr int WAVE = 64;
constexpr int KMAX = 8;                 // largest truncation length of the fused step
constexpr int NSC_MAX = 2 * KMAX + 1;   // partial scalars per Arnoldi step
constexpr int MMAX = 256;               // largest Krylov dimension (register-resident small problem)
constexpr int SMAX = 1024;              // largest sketch size
constexpr double BREAKDOWN_TOL = 1e-14; // lucky-breakdown threshold on h_{j+1,j} / ||A v_j||

// ---------------------------------------------------------------- sketch hash
// SplitMix64 (Steele, Lea & Flood 2014): n-th output of the generator seeded with
// x is mix(x + n * gamma).  The sparse-sign sketch reads 4*ceil(zeta/8) outputs
// per column i, starting at n = 4*ceil(zeta/8)*i + 1.
constexpr uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Rows (distinct, Floyd's sampling) and signs (+1/-1 as double) of sketch column i.
template <int ZETA>
__device__ __forceinline__ void sketch_column(uint64_t seed, uint64_t i, int s,
                                              int (&rows)[ZETA], double (&sgn)[ZETA]) {
    constexpr int OUTS = 4 * ((ZETA + 7) / 8);
    uint32_t w[2 * OUTS];
    uint64_t z = seed + (i * (uint64_t)OUTS + 1ull) * SM_GAMMA;
#pragma unroll
    for (int t = 0; t < OUTS; ++t) {
        uint64_t o = sm_mix(z);
        w[2 * t] = (uint32_t)o;
        w[2 * t + 1] = (uint32_t)(o >> 32);
        z += SM_GAMMA;
    }
#pragma unroll
    for (int q = 0; q < ZETA; ++q) {
        const uint32_t j = (uint32_t)(s - ZETA + q);
        uint32_t r = (uint32_t)(((uint64_t)(w[q] >> 1) * (uint64_t)(j + 1u)) >> 31);
        bool dup = false;
#pragma unroll
        for (int p = 0; p < q; ++p) dup |= (rows[p] == (int)r);
        rows[q] = dup ? (int)j : (int)r;
        sgn[q] = (w[q] & 1u) ? -1.0 : 1.0;
    }
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
    return v;
}

// Deterministic block sum (fixed tree); `scratch` holds >= blockDim/64 doubles.
// Every thread returns the total.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += scratch[i];
    return t;
}

__device__ __forceinline__ double block_max(double v, double* scratch) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double t = scratch[0];
    for (int i = 1; i < nw; ++i) t = fmax(t, scratch[i]);
    return t;
}

__device__ __forceinline__ void lds_add(double* p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// XCD-aware chunk index: blocks are dispatched round-robin over the 8 XCDs of the
// MI355X; remap so that the blocks of one XCD own a contiguous range of chunks
// (neighbouring rows, shared L2).  G must be a multiple of 8.
__device__ __forceinline__ int xcd_chunk(int g, int G) {
    return (g & 7) * (G >> 3) + (g >> 3);
}

}  // namespace skfab
