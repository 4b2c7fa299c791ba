// Shared device helpers of the skfab HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace skfab {

constexpr int WAVE = 64;
constexpr int KMAX = 8;                 // largest truncation length of the fused step
constexpr int NSC_MAX = 2 * KMAX + 1;   // partial scalars per Arnoldi step
constexpr int MMAX = 512;               // largest Krylov dimension
constexpr int CT_NMAX = 200;            // largest Krylov dimension of the contour form (exp, sGMRES)
constexpr int NODE_SLOTS_CT = 512;      // concurrent complex node solves (2 m^2 doubles of scratch each)
constexpr int CT_KFIRST = 32;           // trapezoidal levels K = 32, 64, ..., CT_KMAX intervals
constexpr int CT_KMAX = 1024;
constexpr int SMAX = 1024;              // largest sketch size
constexpr int STEP_GMAX_1024 = 256;     // step-kernel blocks at most, per 1024 threads of block size
constexpr int PACKED_BLOCK = 512;       // threads per block of the batched step's packed form
constexpr int PACKED_RMAX = 4;          // right-hand sides per problem that the packed form carries
constexpr double BREAKDOWN_TOL = 1e-14; // lucky-breakdown threshold on h_{j+1,j} / ||A v_j||

// ------------------------------------------------------------ precisions
// Storage/arithmetic policies of the Krylov recurrence:
//   V = basis storage, W = SpMV arithmetic and A u storage, A = matrix values.
struct bf16s { uint16_t bits; };

__device__ __forceinline__ float bf16_to_f32(bf16s h) { return __uint_as_float((uint32_t)h.bits << 16); }
__device__ __forceinline__ bf16s f32_to_bf16(float f) {  // round to nearest even
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return bf16s{(uint16_t)(r >> 16)};
}

struct PrecF64 { using V = double; using W = double; using A = double; };
struct PrecF32 { using V = float; using W = float; using A = float; };
struct PrecBF16 { using V = bf16s; using W = float; using A = float; };

template <typename W> __device__ __forceinline__ W to_w(double x) { return (W)x; }
template <typename W> __device__ __forceinline__ W to_w(float x) { return (W)x; }
template <typename W> __device__ __forceinline__ W to_w(bf16s x) { return (W)bf16_to_f32(x); }

// Stores of the basis and of A u_j with the non-temporal hint: every vector is
// read again only in later launches, after the whole matrix has streamed past;
// the hint keeps it from displacing the matrix in the caches (measured: 2 % per
// step on the 3D 128^3 workload; non-temporal loads were slower).
template <typename T> __device__ __forceinline__ void store_nt(T v, T* p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_nt(bf16s v, bf16s* p) { __builtin_nontemporal_store(v.bits, &p->bits); }

// Device memory seen through the global address space.  A pointer read from memory
// (rather than passed as a kernel argument) is generic to the compiler, which then
// reaches it with flat instructions; these also count against the LDS wait counter,
// so that every LDS access waits for all loads in flight.  Typed this way, the
// accesses compile to global instructions.
#define GAS __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GAS T* gptr(T* p) { return (GAS T*)p; }
template <typename T> __device__ __forceinline__ T gload(const GAS T* p) { return *p; }

// Raw buffer stores: a resource covering nbytes from base (wave-uniform); the
// hardware drops stores at byte offsets >= nbytes.  A row-guarded tail thus needs
// no per-lane branch (guarded stores in branches were each made to wait for the
// previous one).  Word 3 of the descriptor is the gfx9-family raw-buffer format.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(void* base, int nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, nbytes, 0x00020000);
}
__device__ __forceinline__ void buf_store_f64(double v, __amdgpu_buffer_rsrc_t r, int byte_off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, byte_off, 0, 0);
}
__device__ __forceinline__ bf16s gload(const GAS bf16s* p) { return bf16s{p->bits}; }
template <typename T> __device__ __forceinline__ void store_nt(T v, GAS T* p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_nt(bf16s v, GAS bf16s* p) { __builtin_nontemporal_store(v.bits, &p->bits); }

template <typename V> struct Store;
template <> struct Store<double> {
    __device__ static double put(double x) { return x; }
};
template <> struct Store<float> {
    __device__ static float put(float x) { return x; }
    __device__ static float put(double x) { return (float)x; }
};
template <> struct Store<bf16s> {
    __device__ static bf16s put(float x) { return f32_to_bf16(x); }
};

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

// Broadcast of a double from a wave-uniform lane through two scalar reads
// (no LDS crossbar round trip).
__device__ __forceinline__ int readlane_i32(int v, int src_lane) {
    return __builtin_amdgcn_readlane(v, src_lane);
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int src_lane) {
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), src_lane);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), src_lane);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double bcast_lane(double v, int src_lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src_lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src_lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane permutation within rows of 16 lanes by a DPP control (quad_perm / mirror).
template <int CTRL>
__device__ __forceinline__ double dpp_perm(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave sum with short latency: DPP butterflies inside each row of 16 lanes
// (quad_perm [1,0,3,2], [2,3,0,1], row_half_mirror, row_mirror), then the four row
// sums read through scalar registers.  Fixed order; every lane gets the total.
__device__ __forceinline__ double wave_sum_fast(double v) {
    v += dpp_perm<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_perm<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_perm<0x141>(v);  // row_half_mirror
    v += dpp_perm<0x140>(v);  // row_mirror
    return (bcast_lane(v, 0) + bcast_lane(v, 16)) + (bcast_lane(v, 32) + bcast_lane(v, 48));
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

// Deterministic sum of NV values per thread over the block, through LDS: a fixed
// three-level tree (BLOCK -> 64 -> 8 -> 1 per value).  `sc` must hold
// NV * (BLOCK + 72) doubles; the totals are returned in out[0..NV) (LDS), visible
// to every thread on return.  Far shorter dependency chains than per-value
// shuffle reductions.
template <int NV, int BLOCK>
__device__ void block_reduce_multi(const double (&v)[NV], double* sc, double* out) {
    static_assert(BLOCK % 64 == 0, "block of whole wavefronts");
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NV; ++i) sc[i * BLOCK + tid] = v[i];
    __syncthreads();
    double* s1 = sc + NV * BLOCK;
    for (int t = tid; t < NV * 64; t += BLOCK) {
        const int i = t >> 6, l = t & 63;
        double a0 = 0.0, a1 = 0.0;
        int q = l;
        for (; q + 64 < BLOCK; q += 128) { a0 += sc[i * BLOCK + q]; a1 += sc[i * BLOCK + q + 64]; }
        if (q < BLOCK) a0 += sc[i * BLOCK + q];
        s1[t] = a0 + a1;
    }
    __syncthreads();
    double* s2 = s1 + NV * 64;
    for (int t = tid; t < NV * 8; t += BLOCK) {
        const double* p = s1 + (t >> 3) * 64 + (t & 7) * 8;
        s2[t] = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    }
    __syncthreads();
    for (int t = tid; t < NV; t += BLOCK) {
        const double* p = s2 + t * 8;
        out[t] = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    }
    __syncthreads();
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
