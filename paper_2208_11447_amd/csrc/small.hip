// The small sketched problem of sketched FOM / sketched GMRES on the device.
//
// Formulation.  With the k-truncated Arnoldi relation (Section 2.2 remark and
// eq. H_hat)  A V_m = V_m H_m + u_{m+1} e_m^T  (u_{m+1} the unnormalised next
// vector), the sketched basis satisfies  S A V_m = [S V_m, S u_{m+1}] Hbar  with
// Hbar = [H_m; e_m^T].  A Householder QR  [S V_m, S u_{m+1}] = Q_e R_e  gives, for
// every shift t, the (m+1) x m upper Hessenberg pencil
//
//     P(t) = t R_e[:, :m] + K0,     K0 = R_e Hbar,
//
// and with Q_e^T S b = beta R_e[0,0] e_1:
//   * sketched Galerkin condition (eq. ym_hat):  P(t)[:m, :] y(t) = beta R_00 e_1
//   * sketched GMRES (eq. sgmres integrand):       y(t) = argmin || beta R_00 e_1 - P(t) y ||
// The approximants are V_m int y(t) dmu(t) (sFOM, sGMRES).  For z^(-1/2) the
// integral is the Gauss-Chebyshev rule after t = (1-x)/(1+x) (Section 5.1) with the
// spectral scaling t -> sigma t, sigma = |det H_hat|^(1/m) (geometric mean of the
// eigenvalue moduli of the projected matrix), and the adaptive order update
// l <- floor(sqrt(2) l) of Section 4.1.  Every node is an O(m^2) Hessenberg solve
// (partial pivoting) or Givens least-squares solve, one wavefront per node.
#include "common.hpp"
#include "device_state.hpp"

namespace skfab {

constexpr int QR_NB = 16;        // Householder panel width
constexpr int NODE_SLOTS = 256;  // concurrent quadrature nodes (scratch slots)

// ------------------------------------------------------------ utilities
__global__ void fill_kernel(double* p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void init_ctrl_kernel(DevCtrl* c, int m) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->m_used = m; c->stop = 0; c->status = 0; c->l_used = 0; c->converged = 0; c->l_prev = 0;
        c->beta = 0.0; c->sigma = 1.0; c->eps_est = 0.0; c->rcond = 0.0; c->logdet = 0.0;
    }
}

// ------------------------------------------------------- Householder QR
// Panel factorisation of columns [c0, c0+nb) of X (s x ncols, ld s), rows c0..s-1,
// in LDS.  Householder vectors are stored below the diagonal (unit diagonal
// implied), R on and above it; T (nb x nb, upper) is the compact-WY factor.
__global__ __launch_bounds__(1024) void qr_panel_kernel(double* X, int s, int c0, const DevCtrl* ctrl,
                                                        double* Tws) {
    extern __shared__ double P[];  // [QR_NB][nrows]
    __shared__ double red[16][QR_NB];
    __shared__ double wv[QR_NB];
    __shared__ double tau[QR_NB];
    __shared__ double G[QR_NB][QR_NB];
    __shared__ double sc[3];
    const int ncols = ctrl->m_used + 1;
    if (ctrl->m_used == 0 || c0 >= ncols) return;
    const int pc = min(QR_NB, ncols - c0);
    const int nrows = s - c0;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
    for (int idx = tid; idx < pc * nrows; idx += nt) {
        const int cc = idx / nrows, r = idx - cc * nrows;
        P[idx] = X[(int64_t)(c0 + r) + (int64_t)s * (c0 + cc)];
    }
    __syncthreads();
    for (int cc = 0; cc < pc; ++cc) {
        double* pcol = P + cc * nrows;
        double part = 0.0;
        for (int r = cc + 1 + tid; r < nrows; r += nt) part = fma(pcol[r], pcol[r], part);
        part = wave_sum(part);
        if (lane == 0) red[wid][0] = part;
        __syncthreads();
        if (tid == 0) {
            double sig2 = 0.0;
            for (int i = 0; i < nw; ++i) sig2 += red[i][0];
            const double alpha = pcol[cc];
            if (sig2 == 0.0) {
                tau[cc] = 0.0; sc[0] = 0.0; sc[1] = alpha;
            } else {
                const double nrm = sqrt(alpha * alpha + sig2);
                const double beta = (alpha >= 0.0) ? -nrm : nrm;
                tau[cc] = (beta - alpha) / beta;
                sc[0] = 1.0 / (alpha - beta);
                sc[1] = beta;
            }
        }
        __syncthreads();
        const double scale = sc[0], tcc = tau[cc];
        for (int r = cc + 1 + tid; r < nrows; r += nt) pcol[r] *= scale;
        __syncthreads();
        if (tid == 0) pcol[cc] = sc[1];
        // w_{c2} = v^T P[:, c2] for the remaining panel columns
        double acc[QR_NB];
#pragma unroll
        for (int c2 = 0; c2 < QR_NB; ++c2) acc[c2] = 0.0;
        for (int r = cc + tid; r < nrows; r += nt) {
            const double vr = (r == cc) ? 1.0 : pcol[r];
#pragma unroll
            for (int c2 = 0; c2 < QR_NB; ++c2)
                if (c2 > cc && c2 < pc) acc[c2] = fma(vr, P[c2 * nrows + r], acc[c2]);
        }
#pragma unroll
        for (int c2 = 0; c2 < QR_NB; ++c2) {
            if (c2 > cc && c2 < pc) {
                const double t = wave_sum(acc[c2]);
                if (lane == 0) red[wid][c2] = t;
            }
        }
        __syncthreads();
        if (tid < QR_NB && tid > cc && tid < pc) {
            double t = 0.0;
            for (int i = 0; i < nw; ++i) t += red[i][tid];
            wv[tid] = t;
        }
        __syncthreads();
        for (int idx = tid; idx < (pc - cc - 1) * (nrows - cc); idx += nt) {
            const int c2 = cc + 1 + idx / (nrows - cc);
            const int r = cc + idx % (nrows - cc);
            const double vr = (r == cc) ? 1.0 : pcol[r];
            P[c2 * nrows + r] -= tcc * wv[c2] * vr;
        }
        __syncthreads();
    }
    // Gram of the Householder vectors (unit diagonal, zero above) for T
    for (int pair = wid; pair < pc * pc; pair += nw) {
        const int i = pair / pc, l = pair % pc;
        if (l < i) {
            double t = 0.0;
            for (int r = i + lane; r < nrows; r += 64) {
                const double yi = (r == i) ? 1.0 : P[i * nrows + r];
                const double yl = P[l * nrows + r];  // r >= i > l: strictly below diag
                t = fma(yi, yl, t);
            }
            t = wave_sum(t);
            if (lane == 0) G[l][i] = t;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double T[QR_NB][QR_NB];
        for (int i = 0; i < QR_NB; ++i)
            for (int l = 0; l < QR_NB; ++l) T[i][l] = 0.0;
        for (int i = 0; i < pc; ++i) {
            T[i][i] = tau[i];
            for (int l = 0; l < i; ++l) {
                double t = 0.0;
                for (int q = l; q < i; ++q) t += T[l][q] * G[q][i];
                T[l][i] = -tau[i] * t;
            }
        }
        for (int i = 0; i < QR_NB; ++i)
            for (int l = 0; l < QR_NB; ++l) Tws[i * QR_NB + l] = T[i][l];
    }
    for (int idx = tid; idx < pc * nrows; idx += nt) {
        const int cc = idx / nrows, r = idx - cc * nrows;
        X[(int64_t)(c0 + r) + (int64_t)s * (c0 + cc)] = P[idx];
    }
}

// Trailing update C <- (I - Y T Y^T)^T C for columns c0+nb .. ncols-1, one block per column.
__global__ __launch_bounds__(256) void qr_update_kernel(double* X, int s, int c0, const DevCtrl* ctrl,
                                                        const double* Tws) {
    __shared__ double red[4][QR_NB];
    __shared__ double W[QR_NB], Z[QR_NB];
    const int ncols = ctrl->m_used + 1;
    if (ctrl->m_used == 0 || c0 >= ncols) return;
    const int pc = min(QR_NB, ncols - c0);
    const int d = c0 + pc + blockIdx.x;
    if (d >= ncols) return;
    const int nrows = s - c0;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const double* Y = X + (int64_t)c0 + (int64_t)s * c0;  // Y[r + s*i]
    double* C = X + (int64_t)c0 + (int64_t)s * d;
    double acc[QR_NB];
#pragma unroll
    for (int i = 0; i < QR_NB; ++i) acc[i] = 0.0;
    for (int r = tid; r < nrows; r += 256) {
        const double cr = C[r];
#pragma unroll
        for (int i = 0; i < QR_NB; ++i) {
            if (i < pc && r >= i) {
                const double yi = (r == i) ? 1.0 : Y[r + (int64_t)s * i];
                acc[i] = fma(yi, cr, acc[i]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < QR_NB; ++i) {
        const double t = wave_sum(acc[i]);
        if (lane == 0) red[wid][i] = t;
    }
    __syncthreads();
    if (tid < QR_NB) W[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
    if (tid < QR_NB) {
        double t = 0.0;
        for (int l = 0; l <= tid; ++l) t += Tws[l * QR_NB + tid] * W[l];  // (T^T W)_tid
        Z[tid] = (tid < pc) ? t : 0.0;
    }
    __syncthreads();
    for (int r = tid; r < nrows; r += 256) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < QR_NB; ++i) {
            if (i < pc && r >= i) {
                const double yi = (r == i) ? 1.0 : Y[r + (int64_t)s * i];
                t = fma(yi, Z[i], t);
            }
        }
        C[r] -= t;
    }
}

// --------------------------------------------------------- pencil setup
// K0 = R_e Hbar ((mu+1) x mu, row-major, ld = m), T1 = R_e[:, :mu] (row-major),
// where Hbar = [H(:mu, :mu); e_mu^T] and H is banded (k+1 diagonals).
__global__ void pencil_setup_kernel(const double* X, int s, int m, int k, const DevCtrl* ctrl, const double* H,
                                    double* K0r, double* T1r) {
    const int mu = ctrl->m_used;
    const int64_t ldh = m + 1;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < (mu + 1) * mu; idx += gridDim.x * blockDim.x) {
        const int i = idx / mu, jj = idx - i * mu;
        // T1
        T1r[(int64_t)i * m + jj] = (i <= jj) ? X[i + (int64_t)s * jj] : 0.0;
        // K0[i][jj] = sum_l R_e[i][l] Hbar[l][jj], l in [max(0, jj-k+1), jj+1], R_e upper triangular
        double t = 0.0;
        const int l0 = max(max(0, jj - k + 1), i);
        for (int l = l0; l <= jj + 1; ++l) {
            const double hb = (l == jj + 1) ? ((jj == mu - 1) ? 1.0 : H[(jj + 1) + ldh * jj]) : H[l + ldh * jj];
            t = fma(X[i + (int64_t)s * l], hb, t);
        }
        K0r[(int64_t)i * m + jj] = (i <= jj + 1) ? t : 0.0;
    }
}

// ------------------------------------------------ one-wave pencil solves
// Solves with P(a) = a T1 + K0 (upper Hessenberg), right-hand side rhs0 e_1.
//   LS = false: square system P[:mu] y = rhs0 e_1 (Gaussian elimination with
//               partial pivoting between the two candidate rows of each column)
//   LS = true:  least squares min || rhs0 e_1 - P y || over the (mu+1) x mu pencil
//               (Givens rotations)
// The triangular factor is written row-major into Ubuf (mu x mu, ld = m) and read
// back by the back substitution.  One wavefront; columns j = lane + 64 q.
// Returns log|det| and the sign of det(P[:mu]) for the square case in *logdet / *sgn.
constexpr int QMAX = MMAX / WAVE;

template <bool LS>
__device__ void pencil_solve_wave(int mu, int m, double a, const double* __restrict__ T1r,
                                  const double* __restrict__ K0r, double rhs0, double* __restrict__ Ubuf,
                                  double* __restrict__ Urhs, double* __restrict__ y, double* logdet, double* sgn) {
    const int lane = threadIdx.x & 63;
    double carry[QMAX], next[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        const int jj = lane + WAVE * q;
        carry[q] = (jj < mu) ? fma(a, T1r[jj], K0r[jj]) : 0.0;
    }
    double rc = rhs0, rn = 0.0;
    double ld = 0.0, sg = 1.0;
    const int last = LS ? mu : mu - 1;  // number of eliminations
    for (int kk = 0; kk < last; ++kk) {
        const double* t1 = T1r + (int64_t)(kk + 1) * m;
        const double* k0 = K0r + (int64_t)(kk + 1) * m;
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            const int jj = lane + WAVE * q;
            next[q] = (jj >= kk && jj < mu) ? fma(a, t1[jj], k0[jj]) : 0.0;
        }
        rn = 0.0;
        const int ql = kk / WAVE, ll = kk % WAVE;
        double pk = 0.0, nk = 0.0;
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            if (q == ql) { pk = __shfl(carry[q], ll, WAVE); nk = __shfl(next[q], ll, WAVE); }
        }
        double* urow = Ubuf + (int64_t)kk * m;
        if (!LS) {
            const bool swp = fabs(nk) > fabs(pk);
            if (swp) {
#pragma unroll
                for (int q = 0; q < QMAX; ++q) { const double t = carry[q]; carry[q] = next[q]; next[q] = t; }
                const double t = rc; rc = rn; rn = t;
                const double tp = pk; pk = nk; nk = tp;
                sg = -sg;
            }
            const double l = (pk != 0.0) ? nk / pk : 0.0;
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
                const int jj = lane + WAVE * q;
                if (jj >= kk && jj < mu) urow[jj] = carry[q];
                next[q] = fma(-l, carry[q], next[q]);
            }
            if (lane == 0) Urhs[kk] = rc;
            rn = fma(-l, rc, rn);
            ld += log(fabs(pk));
            if (pk < 0.0) sg = -sg;
        } else {
            const double r = hypot(pk, nk);
            const double c = (r != 0.0) ? pk / r : 1.0;
            const double sn = (r != 0.0) ? nk / r : 0.0;
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
                const int jj = lane + WAVE * q;
                const double top = fma(c, carry[q], sn * next[q]);
                const double bot = fma(-sn, carry[q], c * next[q]);
                if (jj >= kk && jj < mu) urow[jj] = top;
                next[q] = bot;
            }
            const double rtop = fma(c, rc, sn * rn);
            const double rbot = fma(-sn, rc, c * rn);
            if (lane == 0) Urhs[kk] = rtop;
            rn = rbot;
        }
#pragma unroll
        for (int q = 0; q < QMAX; ++q) carry[q] = next[q];
        rc = rn;
    }
    if (!LS) {
        // last row of U
        const int kk = mu - 1;
        const int ql = kk / WAVE, ll = kk % WAVE;
        double pk = 0.0;
#pragma unroll
        for (int q = 0; q < QMAX; ++q)
            if (q == ql) pk = __shfl(carry[q], ll, WAVE);
        if (lane == ll) Ubuf[(int64_t)kk * m + kk] = pk;
        if (lane == 0) Urhs[kk] = rc;
        ld += log(fabs(pk));
        if (pk < 0.0) sg = -sg;
    }
    __threadfence_block();  // Ubuf / Urhs written by this wave become visible to all of its lanes
    // back substitution, y distributed: y[lane + 64 q]
    double yv[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) yv[q] = 0.0;
    for (int kk = mu - 1; kk >= 0; --kk) {
        const double* urow = Ubuf + (int64_t)kk * m;
        double part = 0.0;
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            const int jj = lane + WAVE * q;
            if (jj > kk && jj < mu) part = fma(urow[jj], yv[q], part);
        }
        part = wave_sum(part);
        const double ukk = urow[kk];
        const double yk = (Urhs[kk] - part) / ukk;
        const int ql = kk / WAVE, ll = kk % WAVE;
#pragma unroll
        for (int q = 0; q < QMAX; ++q)
            if (q == ql && lane == ll) yv[q] = yk;
    }
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        const int jj = lane + WAVE * q;
        if (jj < mu) y[jj] = yv[q];
    }
    if (logdet) *logdet = ld;
    if (sgn) *sgn = sg;
}

// Node 0 (a = 0): log|det P[:mu]| and its sign (square case), the spectral scale
// sigma = |det H_hat|^(1/mu) = exp((log|det K0[:mu]| - sum log|R_jj|)/mu), rcond of
// R, the branch check for z^(-1/2), and -- for f = 1/z -- the solution itself.
__global__ __launch_bounds__(64) void pencil_setup_scalars_kernel(int m, int s, const double* X, const DevCtrl* ctrl_c,
                                                                  DevCtrl* ctrl, const double* eta,
                                                                  const double* T1r, const double* K0r,
                                                                  double* Ubuf, double* Urhs, double* y0,
                                                                  int is_ls, int branch_check) {
    const int mu = ctrl_c->m_used;
    if (mu == 0) return;
    const int lane = threadIdx.x;
    // R diagonal statistics
    double lr = 0.0, rmin = 1e308, rmax = 0.0, rs = 1.0;
    for (int j = lane; j < mu; j += 64) {
        const double d = X[j + (int64_t)s * j];
        lr += log(fabs(d));
        rmin = fmin(rmin, fabs(d));
        rmax = fmax(rmax, fabs(d));
        if (d < 0.0) rs = -rs;
    }
    lr = wave_sum(lr);
    rmax = wave_max(rmax);
    rmin = -wave_max(-rmin);
    // product of signs: count negatives
    double neg = (rs < 0.0) ? 1.0 : 0.0;
    neg = wave_sum(neg);
    const double beta = eta[0];
    const double rhs0 = beta * X[0];
    double ld = 0.0, sg = 1.0;
    if (is_ls)
        pencil_solve_wave<true>(mu, m, 0.0, T1r, K0r, rhs0, Ubuf, Urhs, y0, nullptr, nullptr);
    else
        pencil_solve_wave<false>(mu, m, 0.0, T1r, K0r, rhs0, Ubuf, Urhs, y0, &ld, &sg);
    if (lane == 0) {
        ctrl->beta = beta;
        ctrl->rcond = (rmax > 0.0) ? rmin / rmax : 0.0;
        if (!(rmin > 2.220446049250313e-16 * rmax)) ctrl->status = 3;  // SKFAB_ERR_RANK
        if (!is_ls) {
            const double lg = (ld - lr) / mu;
            ctrl->logdet = ld - lr;
            ctrl->sigma = exp(lg);
            const int negs = (int)neg;
            const double sdet = sg * ((negs & 1) ? -1.0 : 1.0);  // sign of det H_hat
            if (branch_check && sdet < 0.0 && ctrl->status == 0) ctrl->status = 4;  // SKFAB_ERR_BRANCH
            if (!isfinite(lg) && ctrl->status == 0) ctrl->status = 3;
        }
    }
}

// sigma for the least-squares case: use the square pencil's scale as well.
// (Called before the LS setup kernel; see host sequence.)

// ------------------------------------------------ quadrature levels
struct QuadArgs {
    const DevCtrl* ctrl;
    const double* T1r;
    const double* K0r;
    double* Ubuf;     // [NODE_SLOTS][m*m]
    double* Urhs;     // [NODE_SLOTS][m]
    double* nodebuf;  // [l][m] weighted node solutions
    int m, l, is_ls;
    double rhs0_unused;
};

__global__ __launch_bounds__(256) void quad_level_kernel(QuadArgs qa, const double* X, int s, const double* eta) {
    if (qa.ctrl->converged || qa.ctrl->status != 0) return;
    const int mu = qa.ctrl->m_used;
    if (mu == 0) return;
    const double sigma = qa.ctrl->sigma;
    const double rhs0 = eta[0] * X[0];
    const int wave = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
    const int nwaves_total = gridDim.x * (blockDim.x / WAVE);
    const int slot = wave;  // < NODE_SLOTS by construction of the grid
    double* U = qa.Ubuf + (int64_t)slot * qa.m * qa.m;
    double* Ur = qa.Urhs + (int64_t)slot * qa.m;
    const int l = qa.l;
    for (int i = wave; i < l; i += nwaves_total) {
        const double x = cos((2.0 * i + 1.0) * M_PI / (2.0 * l));
        const double t = (1.0 - x) / (1.0 + x);
        const double w = (2.0 / l) / (1.0 + x);
        double* yi = qa.nodebuf + (int64_t)i * qa.m;
        if (qa.is_ls)
            pencil_solve_wave<true>(mu, qa.m, t * sigma, qa.T1r, qa.K0r, rhs0 * w, U, Ur, yi, nullptr, nullptr);
        else
            pencil_solve_wave<false>(mu, qa.m, t * sigma, qa.T1r, qa.K0r, rhs0 * w, U, Ur, yi, nullptr, nullptr);
    }
}

// q_l = sqrt(sigma) * sum_i nodebuf[i] (fixed order); on the first level store it,
// afterwards compare with the previous rule in the whitened norm ||R_e[:mu,:mu] (.)||
// (Section 4.1 acceptance test) and either accept or keep the new rule.
__global__ __launch_bounds__(256) void quad_reduce_kernel(DevCtrl* ctrl, const double* nodebuf, int m, int l,
                                                          int first, double tol, const double* T1r,
                                                          double* qprev, double* qcur, double* y) {
    __shared__ double scratch[4];
    __shared__ double diff[MMAX];
    __shared__ double cur[MMAX];
    if (ctrl->converged || ctrl->status != 0) return;
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const double sq = sqrt(ctrl->sigma);
    for (int jj = threadIdx.x; jj < mu; jj += 256) {
        double t = 0.0;
        for (int i = 0; i < l; ++i) t += nodebuf[(int64_t)i * m + jj];
        t *= sq;
        cur[jj] = t;
        diff[jj] = t - qprev[jj];
        qcur[jj] = t;
    }
    __syncthreads();
    if (first) {
        for (int jj = threadIdx.x; jj < mu; jj += 256) qprev[jj] = cur[jj];
        if (threadIdx.x == 0) ctrl->l_prev = l;
        return;
    }
    // whitened norms: R = T1[:mu, :mu] (upper triangular, row-major)
    double nd = 0.0, nc = 0.0;
    for (int i = threadIdx.x; i < mu; i += 256) {
        double td = 0.0, tc = 0.0;
        for (int jj = i; jj < mu; ++jj) {
            const double r = T1r[(int64_t)i * m + jj];
            td = fma(r, diff[jj], td);
            tc = fma(r, cur[jj], tc);
        }
        nd = fma(td, td, nd);
        nc = fma(tc, tc, nc);
    }
    nd = block_sum(nd, scratch);
    nc = block_sum(nc, scratch);
    const bool ok = sqrt(nd) <= tol * sqrt(nc);
    __syncthreads();
    for (int jj = threadIdx.x; jj < mu; jj += 256) {
        if (ok) y[jj] = cur[jj];
        else qprev[jj] = cur[jj];
    }
    if (threadIdx.x == 0) {
        if (ok) { ctrl->converged = 1; ctrl->l_used = l; }
        else ctrl->l_prev = l;
        if (!isfinite(nd) || !isfinite(nc)) ctrl->status = 5;
    }
}

__global__ void quad_fail_kernel(DevCtrl* ctrl) {
    if (threadIdx.x == 0 && ctrl->status == 0 && !ctrl->converged && ctrl->m_used > 0) ctrl->status = 5;
}

// y = p(H_hat) beta e_1 by Horner, H_hat z = R^-1 (K0[:mu] z); one block of 64 threads.
__global__ __launch_bounds__(64) void poly_kernel(const DevCtrl* ctrl, int m, const double* T1r, const double* K0r,
                                                  const double* eta, const double* coef, int npoly, double* y) {
    __shared__ double z[MMAX], t[MMAX];
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const int lane = threadIdx.x;
    const double beta = eta[0];
    for (int j = lane; j < mu; j += 64) z[j] = (j == 0) ? coef[npoly - 1] * beta : 0.0;
    __syncthreads();
    for (int d = npoly - 2; d >= 0; --d) {
        // t = K0[:mu] z
        for (int i = lane; i < mu; i += 64) {
            double acc = 0.0;
            for (int jj = max(0, i - 1); jj < mu; ++jj) acc = fma(K0r[(int64_t)i * m + jj], z[jj], acc);
            t[i] = acc;
        }
        __syncthreads();
        // z = R^-1 t (back substitution, serial over rows, parallel dot)
        for (int i = mu - 1; i >= 0; --i) {
            double part = 0.0;
            for (int jj = i + 1 + lane; jj < mu; jj += 64) part = fma(T1r[(int64_t)i * m + jj], z[jj], part);
            part = wave_sum(part);
            if (lane == 0) z[i] = (t[i] - part) / T1r[(int64_t)i * m + i];
            __syncthreads();
        }
        if (lane == 0) z[0] += coef[d] * beta;
        __syncthreads();
    }
    for (int j = lane; j < mu; j += 64) y[j] = z[j];
}

// ys[j] = y[j] / eta_j (basis stored unnormalised), zero beyond m_used; eps monitor.
__global__ __launch_bounds__(256) void finish_coeffs_kernel(DevCtrl* ctrl, int m, const double* y, const double* eta,
                                                            const double* colnorm2, double* ys, double* yout) {
    __shared__ double scratch[4];
    const int mu = ctrl->m_used;
    double e = 0.0;
    for (int j = threadIdx.x; j < m; j += 256) {
        const double yj = (j < mu) ? y[j] : 0.0;
        ys[j] = (j < mu) ? yj / eta[j] : 0.0;
        if (yout) yout[j] = yj;
        if (j < mu) e = fmax(e, fabs(colnorm2[j] - 1.0));
    }
    e = block_max(e, scratch);
    if (threadIdx.x == 0) {
        ctrl->eps_est = e;
        ctrl->beta = (mu > 0) ? eta[0] : 0.0;
    }
}

// x = U ys (N x mu times mu), rows parallel, coalesced over the basis columns.
__global__ __launch_bounds__(256) void assemble_kernel(const double* __restrict__ U, int64_t ldU, int64_t N, int m,
                                                       const DevCtrl* ctrl, const double* __restrict__ ys,
                                                       double* __restrict__ x) {
    __shared__ double c[MMAX];
    const int mu = ctrl->m_used;
    for (int j = threadIdx.x; j < m; j += blockDim.x) c[j] = (j < mu) ? ys[j] : 0.0;
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int j = 0;
        for (; j + 3 < mu; j += 4) {
            a0 = fma(U[r + ldU * j], c[j], a0);
            a1 = fma(U[r + ldU * (j + 1)], c[j + 1], a1);
            a2 = fma(U[r + ldU * (j + 2)], c[j + 2], a2);
            a3 = fma(U[r + ldU * (j + 3)], c[j + 3], a3);
        }
        for (; j < mu; ++j) a0 = fma(U[r + ldU * j], c[j], a0);
        x[r] = (a0 + a1) + (a2 + a3);
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_init_ctrl(DevCtrl* c, int m, hipStream_t st) {
    hipLaunchKernelGGL(init_ctrl_kernel, dim3(1), dim3(64), 0, st, c, m);
    return hipGetLastError();
}

hipError_t launch_qr(double* X, int s, int ncols_max, const DevCtrl* ctrl, double* Tws, hipStream_t st) {
    for (int c0 = 0; c0 < ncols_max; c0 += QR_NB) {
        const size_t lds = (size_t)QR_NB * (s - c0) * sizeof(double);
        hipLaunchKernelGGL(qr_panel_kernel, dim3(1), dim3(1024), lds, st, X, s, c0, ctrl, Tws);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int rest = ncols_max - c0 - QR_NB;
        if (rest > 0) {
            hipLaunchKernelGGL(qr_update_kernel, dim3(rest), dim3(256), 0, st, X, s, c0, ctrl, Tws);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_pencil_setup(const double* X, int s, int m, int k, const DevCtrl* ctrl, const double* H,
                               double* K0r, double* T1r, hipStream_t st) {
    const int n = (m + 1) * m;
    hipLaunchKernelGGL(pencil_setup_kernel, dim3((n + 255) / 256), dim3(256), 0, st, X, s, m, k, ctrl, H, K0r, T1r);
    return hipGetLastError();
}

hipError_t launch_pencil_scalars(int m, int s, const double* X, DevCtrl* ctrl, const double* eta,
                                 const double* T1r, const double* K0r, double* Ubuf, double* Urhs, double* y0,
                                 int is_ls, int branch_check, hipStream_t st) {
    hipLaunchKernelGGL(pencil_setup_scalars_kernel, dim3(1), dim3(64), 0, st, m, s, X, ctrl, ctrl, eta, T1r, K0r,
                       Ubuf, Urhs, y0, is_ls, branch_check);
    return hipGetLastError();
}

hipError_t launch_quad_level(const DevCtrl* ctrl, const double* T1r, const double* K0r, double* Ubuf, double* Urhs,
                             double* nodebuf, int m, int l, int is_ls, const double* X, int s, const double* eta,
                             hipStream_t st) {
    QuadArgs qa{ctrl, T1r, K0r, Ubuf, Urhs, nodebuf, m, l, is_ls, 0.0};
    int waves = l < NODE_SLOTS ? l : NODE_SLOTS;
    int blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(quad_level_kernel, dim3(blocks), dim3(256), 0, st, qa, X, s, eta);
    return hipGetLastError();
}

hipError_t launch_quad_reduce(DevCtrl* ctrl, const double* nodebuf, int m, int l, int first, double tol,
                              const double* T1r, double* qprev, double* qcur, double* y, hipStream_t st) {
    hipLaunchKernelGGL(quad_reduce_kernel, dim3(1), dim3(256), 0, st, ctrl, nodebuf, m, l, first, tol, T1r, qprev,
                       qcur, y);
    return hipGetLastError();
}

hipError_t launch_quad_fail(DevCtrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(quad_fail_kernel, dim3(1), dim3(64), 0, st, ctrl);
    return hipGetLastError();
}

hipError_t launch_poly(const DevCtrl* ctrl, int m, const double* T1r, const double* K0r, const double* eta,
                       const double* coef, int npoly, double* y, hipStream_t st) {
    hipLaunchKernelGGL(poly_kernel, dim3(1), dim3(64), 0, st, ctrl, m, T1r, K0r, eta, coef, npoly, y);
    return hipGetLastError();
}

hipError_t launch_finish_coeffs(DevCtrl* ctrl, int m, const double* y, const double* eta, const double* colnorm2,
                                double* ys, double* yout, hipStream_t st) {
    hipLaunchKernelGGL(finish_coeffs_kernel, dim3(1), dim3(256), 0, st, ctrl, m, y, eta, colnorm2, ys, yout);
    return hipGetLastError();
}

hipError_t launch_assemble(const double* U, int64_t ldU, int64_t N, int m, const DevCtrl* ctrl, const double* ys,
                           double* x, hipStream_t st) {
    int64_t g = (N + 255) / 256;
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)(g < 8192 ? g : 8192)), dim3(256), 0, st, U, ldU, N, m, ctrl,
                       ys, x);
    return hipGetLastError();
}

}  // namespace skfab
