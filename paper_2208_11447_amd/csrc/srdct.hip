// Subsampled randomized DCT sketch S = sqrt(N/s) P F E (Section 5.1) applied to the
// stored Krylov basis as one dense contraction.
//
// With this sketch the fused step kernel forms no sketch; after the recurrence the
// extended sketched basis [S v_1 .. S v_m, S u_{m+1}] is S times the stored basis
// columns (rescaled by 1/eta_j), a dense s x N by N x (m+1) product: the one place
// in the path where the work is a true dense contraction, so it runs on the FP64
// matrix cores (V_MFMA_F64_16X16X4_F64, one wavefront per 16 x 16 output tile and
// K-chunk, partial tiles summed afterwards in a fixed order).
//
// F_P = sqrt(N/s) P F E is generated once per solve into the workspace, column-major
// (s x N, ld s): F_P[i + s k] = sqrt(N/s) c(r_i) cos(pi r_i (2k + 1) / (2N)) e_k with
// r_i = rows[i], e_k = signs[k], c(0) = sqrt(1/N), c(r) = sqrt(2/N); the angle is
// reduced exactly in integers (r_i (2k + 1) mod 4N) before cospi.
#include "common.hpp"
#include "device_state.hpp"

namespace skfab {

constexpr int SR_TILE = 16;

__global__ __launch_bounds__(256) void srdct_matrix_kernel(int s, int64_t N, const int8_t* __restrict__ signs,
                                                           const int32_t* __restrict__ rows, double* __restrict__ FP) {
    const double sc = sqrt((double)N / (double)s);
    const double c0 = sqrt(1.0 / (double)N), c1 = sqrt(2.0 / (double)N);
    const int64_t total = (int64_t)s * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % s);
        const int64_t k = e / s;
        const int64_t r = rows[i];
        const int64_t q = (r * (2 * k + 1)) % (4 * N);
        const double v = cospi((double)q / (double)(2 * N));
        FP[e] = sc * (r == 0 ? c0 : c1) * v * (double)signs[k];
    }
}

// part[chunk][j][i] (i < s_pad = tiles_i 16, j < tiles_j 16) = sum over k in the chunk of
// F_P[i + s k] U[k + ldU j]; columns j >= ncols and rows i >= s contribute zeros.
// MFMA operand layout (16 x 4 by 4 x 16, FP64): lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; the 16 x 16 result holds D[l / 16 + 4 r][l % 16] in register r
// (checked against the oracle's S V, row by row, by the SRDCT hook test).
template <typename VT>
__global__ __launch_bounds__(64) void srdct_gemm_kernel(const double* __restrict__ FP, int s, int64_t N,
                                                        const VT* __restrict__ U, int64_t ldU, int ncols, int64_t kc,
                                                        double* __restrict__ part) {
    typedef double v4d __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x;
    const int ti = blockIdx.x, tj = blockIdx.y, chunk = blockIdx.z;
    const int s_pad = gridDim.x * SR_TILE, c_pad = gridDim.y * SR_TILE;
    const int ai = ti * SR_TILE + (lane & 15);
    const int bj = tj * SR_TILE + (lane & 15);
    const int kq = lane >> 4;
    const int64_t k0 = (int64_t)chunk * kc;
    const int64_t k1 = min(N, k0 + kc);
    const bool arow = ai < s, bcol = bj < ncols;
    const double* Ap = FP + (arow ? ai : 0);
    const VT* Bp = U + (int64_t)(bcol ? bj : 0) * ldU;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    int64_t k = k0;
    // four k-steps of 4 per iteration, every load issued before the first product
    for (; k + 16 <= k1; k += 16) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t kk = k + 4 * u + kq;
            a[u] = arow ? Ap[(int64_t)s * kk] : 0.0;
            b[u] = bcol ? to_w<double>(Bp[kk]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
    for (; k < k1; k += 4) {
        const int64_t kk = k + kq;
        const bool in = kk < k1;
        const double a = (arow && in) ? Ap[(int64_t)s * kk] : 0.0;
        const double b = (bcol && in) ? to_w<double>(Bp[kk]) : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    double* out = part + (int64_t)chunk * s_pad * c_pad;
    const int j = tj * SR_TILE + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = ti * SR_TILE + kq + 4 * r;
        out[(int64_t)j * s_pad + i] = acc[r];
    }
}

// SV[i + ldS j] = sum_chunk part[chunk][j][i] (fixed order) times scale_j: 1/eta_j for
// j < m_used, 1 for the extension column j = m_used, 0 beyond (and for i >= s).
// With ctrl == nullptr every column is scaled by 1 (test hook).
__global__ __launch_bounds__(256) void srdct_reduce_kernel(const double* __restrict__ part, int nchunks, int s,
                                                           int s_pad, int c_pad, int ncols, const DevCtrl* ctrl,
                                                           const double* __restrict__ eta, double* __restrict__ SV,
                                                           int64_t ldS) {
    const int mu = ctrl ? ctrl->m_used : ncols;
    const int64_t total = (int64_t)ncols * s;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % s), j = (int)(e / s);
        double t = 0.0;
        for (int c = 0; c < nchunks; ++c) t += part[(int64_t)c * s_pad * c_pad + (int64_t)j * s_pad + i];
        const double scale = !ctrl ? 1.0 : (j < mu ? 1.0 / eta[j] : (j == mu ? 1.0 : 0.0));
        SV[(int64_t)j * ldS + i] = t * scale;
    }
}

// Launch geometry of the contraction: tiles of 16 x 16 and K-chunks enough for about
// 2048 wavefronts in flight (at least 16 k per chunk).
struct SrdctPlan {
    int ti, tj, nchunks;
    int64_t kc;
};

SrdctPlan srdct_plan(int s, int64_t N, int ncols) {
    SrdctPlan P;
    P.ti = (s + SR_TILE - 1) / SR_TILE;
    P.tj = (ncols + SR_TILE - 1) / SR_TILE;
    const int64_t tiles = (int64_t)P.ti * P.tj;
    int64_t nc = (2048 + tiles - 1) / tiles;
    const int64_t maxc = (N + 15) / 16;
    if (nc > maxc) nc = maxc;
    if (nc < 1) nc = 1;
    P.kc = ((N + nc - 1) / nc + 15) / 16 * 16;
    P.nchunks = (int)((N + P.kc - 1) / P.kc);
    return P;
}

size_t srdct_part_doubles(int s, int64_t N, int ncols) {
    const SrdctPlan P = srdct_plan(s, N, ncols);
    return (size_t)P.nchunks * P.ti * SR_TILE * P.tj * SR_TILE;
}

hipError_t launch_srdct_matrix(int s, int64_t N, const int8_t* signs, const int32_t* rows, double* FP,
                               hipStream_t st) {
    const int64_t total = (int64_t)s * N;
    int64_t g = (total + 255) / 256;
    hipLaunchKernelGGL(srdct_matrix_kernel, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(256), 0, st, s, N, signs,
                       rows, FP);
    return hipGetLastError();
}

// SV (ld ldS) <- F_P U[:, 0..ncols), scaled as in srdct_reduce_kernel.
hipError_t launch_srdct_sketch(const double* FP, int s, int64_t N, const void* U, int64_t ldU, int ncols, int prec,
                               double* part, const DevCtrl* ctrl, const double* eta, double* SV, int64_t ldS,
                               hipStream_t st) {
    const SrdctPlan P = srdct_plan(s, N, ncols);
    const dim3 grid(P.ti, P.tj, P.nchunks);
    if (prec == 1)
        hipLaunchKernelGGL(srdct_gemm_kernel<float>, grid, dim3(64), 0, st, FP, s, N, static_cast<const float*>(U),
                           ldU, ncols, P.kc, part);
    else if (prec == 2)
        hipLaunchKernelGGL(srdct_gemm_kernel<bf16s>, grid, dim3(64), 0, st, FP, s, N, static_cast<const bf16s*>(U),
                           ldU, ncols, P.kc, part);
    else
        hipLaunchKernelGGL(srdct_gemm_kernel<double>, grid, dim3(64), 0, st, FP, s, N,
                           static_cast<const double*>(U), ldU, ncols, P.kc, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)ncols * s;
    int64_t g = (total + 255) / 256;
    hipLaunchKernelGGL(srdct_reduce_kernel, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, st, part,
                       P.nchunks, s, P.ti * SR_TILE, P.tj * SR_TILE, ncols, ctrl, eta, SV, ldS);
    return hipGetLastError();
}

}  // namespace skfab
