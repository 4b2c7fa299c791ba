// Closed-form sketched FOM for f(z) = exp(-tau z): y = exp(-tau H_hat) beta e_1
// (eq. sfom3 in the form of the Section 2.2 remark, H_hat = H_m + x_hat e_m^T with
// x_hat the sketched least-squares coefficients of the extension vector).
//
// exp of the dense m x m matrix uses scaling and squaring with the [13/13] Pade
// approximant (Higham, SIAM J. Matrix Anal. Appl. 26 (2005)): A <- A / 2^s with
// alpha(A) <= theta_13, U = A (A6 (c13 A6 + c11 A4 + c9 A2) + c7 A6 + c5 A4 + c3 A2 + c1 I),
// V = A6 (c12 A6 + c10 A4 + c8 A2) + c6 A6 + c4 A4 + c2 A2 + c0 I, X = (V - U)^-1 (V + U),
// then s squarings.  The scaling uses alpha(A) = min_p max(||A^p||^(1/p),
// ||A^(p+1)||^(1/(p+1))) over p(p-1) <= 27 instead of ||A||: the backward-error
// series of the [13/13] approximant starts at x^27, and Al-Mohy & Higham (SIAM J.
// Matrix Anal. Appl. 31 (2009), Thm. 4.2) bound such a series at A by its
// absolute-coefficient series at alpha_p(A).  For the projected matrix of a basis
// with a well-conditioned prefix cut from a dependent tail, ||A|| is dominated by
// one large last column while the powers are not, and scaling by ||A|| would square
// many times over and amplify the rounding of each product.  Dense products use an
// LDS-tiled FP64 GEMM; the Pade solve an LU factorisation with partial pivoting
// (one block) and one wavefront per right-hand-side column.
#include "common.hpp"
#include "device_state.hpp"

namespace skfab {

// H_hat (column-major, ld m) scaled by -tau, and ||.||_1 into ctrl->logdet's
// neighbour field (norm1).  One wave:  x = R^-1 r by back substitution, then
// H_hat = H(:mu,:mu) + x e_mu^T.
__global__ __launch_bounds__(64) void hhat_kernel(const DevCtrl* ctrl, int m, const double* T1r, const double* X,
                                                  int s, const double* H, double tau, double* Ahat, double* norm1) {
    __shared__ double xs[MMAX];
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const int lane = threadIdx.x;
    const int64_t ldh = m + 1;
    // r = R_e[:mu, mu] (column mu of the QR'd extended sketch)
    for (int i = lane; i < mu; i += 64) xs[i] = X[i + (int64_t)s * mu];
    __syncthreads();
    for (int i = mu - 1; i >= 0; --i) {
        double part = 0.0;
        for (int j = i + 1 + lane; j < mu; j += 64) part = fma(T1r[(int64_t)i * m + j], xs[j], part);
        part = wave_sum(part);
        if (lane == 0) xs[i] = (xs[i] - part) / T1r[(int64_t)i * m + i];
        __syncthreads();
    }
    double nrm = 0.0;
    for (int j = 0; j < mu; ++j) {
        double colsum = 0.0;
        for (int i = lane; i < mu; i += 64) {
            double h = 0.0;
            if (i <= j + 1) {
                if (i == j + 1) h = H[(j + 1) + ldh * j];
                else h = H[i + ldh * j];
            }
            if (j == mu - 1) h += xs[i];
            const double a = -tau * h;
            Ahat[i + (int64_t)m * j] = a;
            colsum += fabs(a);
        }
        colsum = wave_sum(colsum);
        nrm = fmax(nrm, colsum);
    }
    if (lane == 0) *norm1 = nrm;
}

// Elementwise: D = a*P + b*Q + c*R + d*I over mu x mu (ld m); any of Q, R may be null.
__global__ void combine_kernel(const DevCtrl* ctrl, int m, double a, const double* P, double b, const double* Q,
                               double c, const double* R, double d, double* D) {
    const int mu = ctrl->m_used;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < mu * mu; idx += gridDim.x * blockDim.x) {
        const int i = idx % mu, j = idx / mu;
        const int64_t o = i + (int64_t)m * j;
        double v = a * P[o];
        if (Q) v = fma(b, Q[o], v);
        if (R) v = fma(c, R[o], v);
        if (i == j) v += d;
        D[o] = v;
    }
}

// C = A B (+ beta C) for mu x mu column-major matrices (ld m); 32x32 tiles, 2x2 per thread.
__global__ __launch_bounds__(256) void dgemm_kernel(const DevCtrl* ctrl, int m, const double* A, const double* B,
                                                    double beta, double* C) {
    __shared__ double As[32][33];
    __shared__ double Bs[32][33];
    const int mu = ctrl->m_used;
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    if (i0 >= mu || j0 >= mu) return;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
    for (int k0 = 0; k0 < mu; k0 += 32) {
        for (int idx = threadIdx.x; idx < 1024; idx += 256) {
            const int r = idx & 31, cc = idx >> 5;
            const int gi = i0 + r, gk = k0 + cc;
            As[r][cc] = (gi < mu && gk < mu) ? A[gi + (int64_t)m * gk] : 0.0;
            const int gk2 = k0 + r, gj = j0 + cc;
            Bs[r][cc] = (gk2 < mu && gj < mu) ? B[gk2 + (int64_t)m * gj] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < 32; ++kk) {
            const double a0 = As[tx][kk], a1 = As[tx + 16][kk];
            const double b0 = Bs[kk][ty], b1 = Bs[kk][ty + 16];
            c00 = fma(a0, b0, c00);
            c01 = fma(a0, b1, c01);
            c10 = fma(a1, b0, c10);
            c11 = fma(a1, b1, c11);
        }
        __syncthreads();
    }
    const double cv[2][2] = {{c00, c01}, {c10, c11}};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int gi = i0 + tx + 16 * a, gj = j0 + ty + 16 * b;
            if (gi < mu && gj < mu) {
                const int64_t o = gi + (int64_t)m * gj;
                C[o] = (beta != 0.0) ? fma(beta, C[o], cv[a][b]) : cv[a][b];
            }
        }
}

// In-place LU with partial pivoting of the mu x mu matrix Q (ld m), one block.
__global__ __launch_bounds__(1024) void lu_kernel(DevCtrl* ctrl, int m, double* Q, int* piv) {
    __shared__ double vmax[16];
    __shared__ int imax[16];
    __shared__ int s_p;
    const int mu = ctrl->m_used;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int k = 0; k < mu; ++k) {
        // pivot: argmax |Q[i,k]|, i >= k (ties -> smallest index)
        double bv = -1.0;
        int bi = k;
        for (int i = k + tid; i < mu; i += 1024) {
            const double v = fabs(Q[i + (int64_t)m * k]);
            if (v > bv) { bv = v; bi = i; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { vmax[wid] = bv; imax[wid] = bi; }
        __syncthreads();
        if (tid == 0) {
            double b = vmax[0];
            int p = imax[0];
            for (int w = 1; w < 16; ++w)
                if (vmax[w] > b || (vmax[w] == b && imax[w] < p)) { b = vmax[w]; p = imax[w]; }
            s_p = p;
            piv[k] = p;
            if (b == 0.0) ctrl->status = 3;
        }
        __syncthreads();
        const int p = s_p;
        if (p != k)
            for (int j = tid; j < mu; j += 1024) {
                const double t = Q[k + (int64_t)m * j];
                Q[k + (int64_t)m * j] = Q[p + (int64_t)m * j];
                Q[p + (int64_t)m * j] = t;
            }
        __syncthreads();
        const double pivv = Q[k + (int64_t)m * k];
        for (int i = k + 1 + tid; i < mu; i += 1024) Q[i + (int64_t)m * k] /= pivv;
        __syncthreads();
        const int n = mu - k - 1;
        for (int idx = tid; idx < n * n; idx += 1024) {
            const int i = k + 1 + idx % n, j = k + 1 + idx / n;
            Q[i + (int64_t)m * j] = fma(-Q[i + (int64_t)m * k], Q[k + (int64_t)m * j], Q[i + (int64_t)m * j]);
        }
        __syncthreads();
    }
}

// Solve Q X = P column by column with the LU factors (one wave per column); X may alias P.
__global__ __launch_bounds__(256) void lu_solve_cols_kernel(const DevCtrl* ctrl, int m, const double* LU,
                                                            const int* piv, double* P) {
    const int mu = ctrl->m_used;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (col >= mu) return;
    double* x = P + (int64_t)m * col;
    // row interchanges (sequential, lane 0), then make them visible to the wave
    if (lane == 0)
        for (int k = 0; k < mu; ++k) {
            const int p = piv[k];
            if (p != k) { const double t = x[k]; x[k] = x[p]; x[p] = t; }
        }
    __threadfence_block();
    // forward substitution with unit lower L (column oriented)
    for (int k = 0; k < mu; ++k) {
        const double xk = x[k];
        for (int i = k + 1 + lane; i < mu; i += 64) x[i] = fma(-LU[i + (int64_t)m * k], xk, x[i]);
        __threadfence_block();
    }
    // back substitution with U
    for (int k = mu - 1; k >= 0; --k) {
        double xk = 0.0;
        if (lane == 0) { xk = x[k] / LU[k + (int64_t)m * k]; x[k] = xk; }
        xk = __shfl(xk, 0, 64);
        for (int i = lane; i < k; i += 64) x[i] = fma(-LU[i + (int64_t)m * k], xk, x[i]);
        __threadfence_block();
    }
}

// ||P_q||_1 of the mu x mu matrices P_q (ld m) into norm1[q], one block each.
struct NormArgs {
    const double* P[6];
};
__global__ __launch_bounds__(256) void norm1_kernel(const DevCtrl* ctrl, int m, NormArgs a, double* norm1) {
    __shared__ double scratch[4];
    const int mu = ctrl->m_used;
    const double* P = a.P[blockIdx.x];
    double mx = 0.0;
    for (int j = threadIdx.x; j < mu; j += blockDim.x) {
        double c = 0.0;
        for (int i = 0; i < mu; ++i) c += fabs(P[i + (int64_t)m * j]);
        mx = fmax(mx, c);
    }
    mx = block_max(mx, scratch);
    if (threadIdx.x == 0) norm1[blockIdx.x] = mx;
}

// y[i] = beta * X[i, 0]
__global__ void first_column_kernel(const DevCtrl* ctrl, const double* X, const double* eta, double* y) {
    const int mu = ctrl->m_used;
    for (int i = threadIdx.x; i < mu; i += blockDim.x) y[i] = eta[0] * X[i];
}

hipError_t launch_hhat(const DevCtrl* ctrl, int m, const double* T1r, const double* X, int s, const double* H,
                       double tau, double* Ahat, double* norm1, hipStream_t st) {
    hipLaunchKernelGGL(hhat_kernel, dim3(1), dim3(64), 0, st, ctrl, m, T1r, X, s, H, tau, Ahat, norm1);
    return hipGetLastError();
}

hipError_t launch_combine(const DevCtrl* ctrl, int m, double a, const double* P, double b, const double* Q,
                          double c, const double* R, double d, double* D, hipStream_t st) {
    const int n = m * m;
    hipLaunchKernelGGL(combine_kernel, dim3((n + 255) / 256), dim3(256), 0, st, ctrl, m, a, P, b, Q, c, R, d, D);
    return hipGetLastError();
}

hipError_t launch_dgemm(const DevCtrl* ctrl, int m, const double* A, const double* B, double beta, double* C,
                        hipStream_t st) {
    const int t = (m + 31) / 32;
    hipLaunchKernelGGL(dgemm_kernel, dim3(t, t), dim3(256), 0, st, ctrl, m, A, B, beta, C);
    return hipGetLastError();
}

hipError_t launch_lu(DevCtrl* ctrl, int m, double* Q, int* piv, hipStream_t st) {
    hipLaunchKernelGGL(lu_kernel, dim3(1), dim3(1024), 0, st, ctrl, m, Q, piv);
    return hipGetLastError();
}

hipError_t launch_lu_solve_cols(const DevCtrl* ctrl, int m, const double* LU, const int* piv, double* P,
                                hipStream_t st) {
    hipLaunchKernelGGL(lu_solve_cols_kernel, dim3((m + 3) / 4), dim3(256), 0, st, ctrl, m, LU, piv, P);
    return hipGetLastError();
}

hipError_t launch_norm1(const DevCtrl* ctrl, int m, const double* const* P, int count, double* norm1,
                        hipStream_t st) {
    NormArgs a;
    for (int q = 0; q < 6; ++q) a.P[q] = q < count ? P[q] : nullptr;
    hipLaunchKernelGGL(norm1_kernel, dim3(count), dim3(256), 0, st, ctrl, m, a, norm1);
    return hipGetLastError();
}

hipError_t launch_first_column(const DevCtrl* ctrl, const double* X, const double* eta, double* y, hipStream_t st) {
    hipLaunchKernelGGL(first_column_kernel, dim3(1), dim3(256), 0, st, ctrl, X, eta, y);
    return hipGetLastError();
}

}  // namespace skfab
