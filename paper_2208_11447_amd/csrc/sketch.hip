// Test hooks for the sparse-sign sketch: the pattern of a range of columns, and
// S v for a single vector (per-block partial sums in fixed order, then a
// column-ordered reduction).
#include "common.hpp"

namespace skfab {

template <int ZETA>
__global__ void sketch_pattern_kernel(int64_t col0, int64_t ncols, int s, uint64_t seed,
                                      int32_t* rows, int8_t* signs) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncols;
         i += (int64_t)gridDim.x * blockDim.x) {
        int r[ZETA];
        double sg[ZETA];
        sketch_column<ZETA>(seed, (uint64_t)(col0 + i), s, r, sg);
#pragma unroll
        for (int q = 0; q < ZETA; ++q) {
            rows[i * ZETA + q] = r[q];
            signs[i * ZETA + q] = (sg[q] > 0.0) ? 1 : -1;
        }
    }
}

template <int ZETA>
__global__ __launch_bounds__(256) void sketch_apply_partial_kernel(int64_t n, int s, uint64_t seed,
                                                                   const double* v, double* part) {
    extern __shared__ double bins[];  // [4][s]
    const int nw = 256 / WAVE;
    for (int i = threadIdx.x; i < nw * s; i += 256) bins[i] = 0.0;
    __syncthreads();
    double* my = bins + (threadIdx.x / WAVE) * s;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = min(n, r0 + per);
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        int rows[ZETA];
        double sg[ZETA];
        sketch_column<ZETA>(seed, (uint64_t)r, s, rows, sg);
        const double x = v[r];
#pragma unroll
        for (int q = 0; q < ZETA; ++q) lds_add(my + rows[q], sg[q] * x);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < s; i += 256) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += bins[w * s + i];
        part[(int64_t)blockIdx.x * s + i] = t;
    }
}

__global__ void sketch_apply_reduce_kernel(const double* part, int G, int s, double scale, double* Sv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s) return;
    double t = 0.0;
    for (int g = 0; g < G; ++g) t += part[(int64_t)g * s + i];
    Sv[i] = t * scale;
}

hipError_t launch_sketch_pattern(int64_t col0, int64_t ncols, int s, int zeta, uint64_t seed,
                                 int32_t* rows, int8_t* signs, hipStream_t st) {
    int64_t g64 = (ncols + 255) / 256;
    const int grid = (int)(g64 < 4096 ? (g64 > 0 ? g64 : 1) : 4096);
    switch (zeta) {
        case 2: hipLaunchKernelGGL(sketch_pattern_kernel<2>, dim3(grid), dim3(256), 0, st, col0, ncols, s, seed, rows, signs); break;
        case 4: hipLaunchKernelGGL(sketch_pattern_kernel<4>, dim3(grid), dim3(256), 0, st, col0, ncols, s, seed, rows, signs); break;
        case 16: hipLaunchKernelGGL(sketch_pattern_kernel<16>, dim3(grid), dim3(256), 0, st, col0, ncols, s, seed, rows, signs); break;
        default: hipLaunchKernelGGL(sketch_pattern_kernel<8>, dim3(grid), dim3(256), 0, st, col0, ncols, s, seed, rows, signs); break;
    }
    return hipGetLastError();
}

int sketch_apply_blocks(int64_t n) {
    int64_t g = (n + 4095) / 4096;
    return (int)(g < 256 ? (g > 0 ? g : 1) : 256);
}

hipError_t launch_sketch_apply(int64_t n, int s, int zeta, uint64_t seed, const double* v, double* Sv,
                               double* part, hipStream_t st) {
    const int G = sketch_apply_blocks(n);
    const size_t lds = (size_t)(256 / WAVE) * s * sizeof(double);
    switch (zeta) {
        case 2: hipLaunchKernelGGL(sketch_apply_partial_kernel<2>, dim3(G), dim3(256), lds, st, n, s, seed, v, part); break;
        case 4: hipLaunchKernelGGL(sketch_apply_partial_kernel<4>, dim3(G), dim3(256), lds, st, n, s, seed, v, part); break;
        case 16: hipLaunchKernelGGL(sketch_apply_partial_kernel<16>, dim3(G), dim3(256), lds, st, n, s, seed, v, part); break;
        default: hipLaunchKernelGGL(sketch_apply_partial_kernel<8>, dim3(G), dim3(256), lds, st, n, s, seed, v, part); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sketch_apply_reduce_kernel, dim3((s + 255) / 256), dim3(256), 0, st, part, G, s,
                       1.0 / sqrt((double)zeta), Sv);
    return hipGetLastError();
}

}  // namespace skfab
