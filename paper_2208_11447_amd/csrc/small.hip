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
//   * sketched Galerkin condition (eq. ym_hat):  P(t)[:m, :] y(t) = beta R_00 e_1,
//     i.e. R (t I + H_hat) y(t) = beta R_00 e_1 with H_hat = H_m + (R^-1 R_e[:m, m]) e_m^T,
//     solved as (t I + H_hat) y(t) = beta e_1 (no factor R: its condition number
//     would otherwise multiply the rounding error of every node solve)
//   * sketched GMRES (eq. sgmres integrand):       y(t) = argmin || beta R_00 e_1 - P(t) y ||
// The approximants are V_m int y(t) dmu(t) (sFOM, sGMRES).  For z^(-1/2) the
// integral is the Gauss-Chebyshev rule after t = (1-x)/(1+x) (Section 5.1) with the
// spectral scaling t -> sigma t, sigma = sqrt(|theta|_min |theta|_max) over the
// eigenvalues of the projected matrix (estimated by power and inverse iteration),
// and the adaptive order update
// l <- floor(sqrt(2) l) of Section 4.1 (accepting an order at the rounding floor
// QUAD_FLOOR when the requested tolerance is out of reach).  Every node is an
// O(m^2) Hessenberg solve (partial pivoting) or Givens least-squares solve, one
// wavefront per node.
#include "common.hpp"
#include "device_state.hpp"

namespace skfab {

constexpr int QR_NB = 16;        // Householder panel width
constexpr int NODE_SLOTS = 1024;  // concurrent quadrature nodes (scratch slots)
// Rounding floor of the adaptive quadrature test: an order whose relative difference
// to the previous one is below this and no longer decreasing is accepted even when
// the requested tolerance lies below what the node solves can resolve.
constexpr double QUAD_FLOOR = 1e-10;

// ------------------------------------------------------------ utilities
__global__ void fill_kernel(double* p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__device__ __forceinline__ void init_ctrl_body(DevCtrl* c, int m) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->m_used = m; c->stop = 0; c->status = 0; c->l_used = 0; c->converged = 0; c->l_prev = 0;
        c->beta = 0.0; c->sigma = 1.0; c->eps_est = 0.0; c->rcond = 0.0; c->logdet = 0.0;
        c->qdiff_prev = INFINITY;
        c->col_wide = 0;
        c->flags = 0;
        c->quad_diff = 0.0;
        c->relres = -1.0;  // set by the Arnoldi-relation check (sparse-sign sketch only)
        c->m_basis = m;
        c->ct_a = 0.0; c->ct_c = 0.0; c->ct_tmax = 0.0;
    }
}

__global__ void init_ctrl_kernel(DevCtrl* c, int m) { init_ctrl_body(c, m); }

// Batched forms below take blockIdx.y as the unit index and read the unit's
// pointers from a SmallUnit array; blockIdx.x keeps its single-problem meaning.
__global__ void init_ctrl_batched_kernel(const SmallUnit* __restrict__ units) {
    const SmallUnit& u = units[blockIdx.y];
    init_ctrl_body(u.ctrl, u.m);
}

// ------------------------------------------------------- Householder QR
// Panel factorisation of columns [c0, c0+nb) of X (s x ncols, ld s), rows c0..s-1.
// Wave w holds panel columns CPW w .. CPW w + CPW - 1 in registers, lane l the rows
// l + 64 i (i < RPW).  Column cc's reflector is formed by the wave that holds it and
// published through LDS (two buffers, one barrier per column); every wave then
// applies it to its later columns and takes the Gram entries <v_l, v_cc> of its
// earlier ones (for T), each with one wave reduction.  Householder vectors are
// stored below the diagonal (unit diagonal implied), R on and above it; T (nb x nb,
// upper) is the compact-WY factor.
constexpr int QR_NT = 256;
constexpr int QR_CPW = QR_NB / (QR_NT / WAVE);  // panel columns per wavefront

template <int RPW>
__device__ __forceinline__ void qr_panel_body(double* X, int s, int c0, const DevCtrl* ctrl, double* Tws) {
    __shared__ double vbuf[2][WAVE * RPW];
    __shared__ double tau[QR_NB];
    __shared__ double G[QR_NB][QR_NB];
    const int ncols = ctrl->m_used + 1;
    if (ctrl->m_used == 0 || c0 >= ncols) return;
    const int pc = min(QR_NB, ncols - c0);
    const int nrows = s - c0;  // <= WAVE * RPW (launcher)
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double a[QR_CPW][RPW];
#pragma unroll
    for (int q = 0; q < QR_CPW; ++q)
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int c = wid * QR_CPW + q, r = lane + WAVE * i;
            a[q][i] = (c < pc && r < nrows) ? X[(int64_t)(c0 + r) + (int64_t)s * (c0 + c)] : 0.0;
        }
    if (tid < QR_NB * QR_NB) G[tid / QR_NB][tid % QR_NB] = 0.0;
    for (int cc = 0; cc < pc; ++cc) {
        double* vb = vbuf[cc & 1];
        // the wave holding column cc (all earlier reflectors applied) forms v_cc
#pragma unroll
        for (int q = 0; q < QR_CPW; ++q) {
            if (wid * QR_CPW + q != cc) continue;
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < RPW; ++i)
                if (lane + WAVE * i > cc) t = fma(a[q][i], a[q][i], t);
            const double sig2 = wave_sum_fast(t);
            const double alpha = bcast_lane(a[q][0], cc);  // row cc < QR_NB: lane cc of i = 0
            double beta, tc, scale;
            if (sig2 == 0.0) {
                beta = alpha; tc = 0.0; scale = 0.0;
            } else {
                const double nrm = sqrt(alpha * alpha + sig2);
                beta = (alpha >= 0.0) ? -nrm : nrm;
                tc = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                const int r = lane + WAVE * i;
                double v = 0.0;
                if (r > cc) { v = scale * a[q][i]; a[q][i] = v; }
                else if (r == cc) { v = 1.0; a[q][i] = beta; }
                if (r < nrows) vb[r] = v;
            }
            if (lane == 0) tau[cc] = tc;
        }
        __syncthreads();
        double v[RPW];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = lane + WAVE * i;
            v[i] = (r < nrows) ? vb[r] : 0.0;
        }
        const double tc = tau[cc];
        double part[QR_CPW];
#pragma unroll
        for (int q = 0; q < QR_CPW; ++q) {
            part[q] = 0.0;
#pragma unroll
            for (int i = 0; i < RPW; ++i) part[q] = fma(v[i], a[q][i], part[q]);
        }
        // v_cc vanishes above row cc: for a later column this is v^T x, for an
        // earlier column l it meets only v_l's rows below its diagonal (= <v_l, v_cc>)
#pragma unroll
        for (int q = 0; q < QR_CPW; ++q) part[q] = wave_sum_fast(part[q]);
#pragma unroll
        for (int q = 0; q < QR_CPW; ++q) {
            const int c = wid * QR_CPW + q;
            if (c > cc && c < pc) {
                const double w = tc * part[q];
#pragma unroll
                for (int i = 0; i < RPW; ++i) a[q][i] = fma(-w, v[i], a[q][i]);
            } else if (c < cc && lane == 0) {
                G[c][cc] = part[q];
            }
        }
    }
    __syncthreads();
    // compact-WY factor T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]: row l of T needs only
    // its own earlier entries, so lane l builds row l alone (no barrier)
    if (tid < QR_NB) {
        const int l = tid;
        double trow[QR_NB];
#pragma unroll
        for (int i = 0; i < QR_NB; ++i) {
            double v = 0.0;
            if (i < pc && i == l) {
                v = tau[i];
            } else if (i < pc && i > l) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < QR_NB; ++q)
                    if (q >= l && q < i) t += trow[q] * G[q][i];
                v = -tau[i] * t;
            }
            trow[i] = v;
        }
#pragma unroll
        for (int i = 0; i < QR_NB; ++i) Tws[l * QR_NB + i] = trow[i];
    }
    // rows c0 .. s-1 of each panel column through a buffer resource ending at row
    // s-1 (an empty one for columns beyond the panel): no per-lane guard
    const int wu = __builtin_amdgcn_readfirstlane(wid);
#pragma unroll
    for (int q = 0; q < QR_CPW; ++q) {
        const int c = wu * QR_CPW + q;
        const __amdgpu_buffer_rsrc_t rs =
            buf_rsrc(X + (int64_t)c0 + (int64_t)s * (c0 + min(c, pc - 1)), (c < pc) ? nrows * 8 : 0);
#pragma unroll
        for (int i = 0; i < RPW; ++i) buf_store_f64(a[q][i], rs, (lane + WAVE * i) * 8);
    }
}

template <int RPW>
__global__ __launch_bounds__(QR_NT) void qr_panel_kernel(double* X, int s, int c0, const DevCtrl* ctrl,
                                                          double* Tws) {
    qr_panel_body<RPW>(X, s, c0, ctrl, Tws);
}

template <int RPW>
__global__ __launch_bounds__(QR_NT) void qr_panel_batched_kernel(const SmallUnit* __restrict__ units, int s, int c0) {
    const SmallUnit& u = units[blockIdx.y];
    qr_panel_body<RPW>(u.SV, s, c0, u.ctrl, u.Tws);
}

// Trailing update C <- (I - Y T Y^T)^T C for columns c0+nb .. ncols-1, one block per column.
__device__ __forceinline__ void qr_update_body(double* X, int s, int c0, const DevCtrl* ctrl, const double* Tws) {
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
    constexpr int RPT = SMAX / 256;
    double cv[RPT], yv[RPT][QR_NB];
    // all loads first (one memory round trip)
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int r = tid + 256 * k;
        cv[k] = (r < nrows) ? C[r] : 0.0;
#pragma unroll
        for (int i = 0; i < QR_NB; ++i)
            yv[k][i] = (r < nrows && i < pc && r > i) ? Y[r + (int64_t)s * i] : ((r == i && i < pc) ? 1.0 : 0.0);
    }
    double acc[QR_NB];
#pragma unroll
    for (int i = 0; i < QR_NB; ++i) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < RPT; ++k) t = fma(yv[k][i], cv[k], t);
        acc[i] = wave_sum_fast(t);
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < QR_NB; ++i) red[wid][i] = acc[i];
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
    // rows beyond the column's end fall outside the buffer resource (no guard)
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(C, nrows * 8);
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int r = tid + 256 * k;
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < QR_NB; ++i) t = fma(yv[k][i], Z[i], t);
        buf_store_f64(cv[k] - t, rs, r * 8);
    }
}

__global__ __launch_bounds__(256) void qr_update_kernel(double* X, int s, int c0, const DevCtrl* ctrl,
                                                        const double* Tws) {
    qr_update_body(X, s, c0, ctrl, Tws);
}

__global__ __launch_bounds__(256) void qr_update_batched_kernel(const SmallUnit* __restrict__ units, int s, int c0) {
    const SmallUnit& u = units[blockIdx.y];
    qr_update_body(u.SV, s, c0, u.ctrl, u.Tws);
}

// --------------------------------------------------------- pencil setup
// K0 = R_e Hbar ((mu+1) x mu, row-major, ld = m), T1 = R_e[:, :mu] (row-major),
// where Hbar = [H(:mu, :mu); e_mu^T] and H is banded (k+1 diagonals).
__device__ __forceinline__ void pencil_setup_body(const double* X, int s, int m, int k, const DevCtrl* ctrl,
                                                  const double* H, double* K0r, double* T1r) {
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

__global__ void pencil_setup_kernel(const double* X, int s, int m, int k, const DevCtrl* ctrl, const double* H,
                                    double* K0r, double* T1r) {
    pencil_setup_body(X, s, m, k, ctrl, H, K0r, T1r);
}

__global__ void pencil_setup_batched_kernel(const SmallUnit* __restrict__ units, int s, int m, int k) {
    const SmallUnit& u = units[blockIdx.y];
    pencil_setup_body(u.SV, s, m, k, u.ctrl, u.H, u.K0r, u.T1r);
}

// ------------------------------------------------ one-wave pencil solves
// Helpers of the one-wavefront Hessenberg solves below (vectors distributed as
// index lane + 64 q over the lanes of the wavefront).

// raw entries of row kk of T1 and K0, columns >= c0 (zero elsewhere); combined into
// P(a) = a T1 + K0 only when the row is used, so the loads stay in flight.
// T1r == nullptr stands for T1 = I (the square systems a I + H_hat).
template <int QM>
struct PRow {
    double t[QM], k[QM];
};

template <int QM>
__device__ __forceinline__ void load_pencil_row(PRow<QM>& row, int kk, int c0, int mu, int m,
                                                const double* __restrict__ T1r, const double* __restrict__ K0r) {
    const int lane = threadIdx.x & 63;
    const double* k0 = K0r + (int64_t)kk * m;
    if (T1r) {
        const double* t1 = T1r + (int64_t)kk * m;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int jj = lane + WAVE * q;
            const bool in = jj >= c0 && jj < mu;
            row.t[q] = in ? t1[jj] : 0.0;
            row.k[q] = in ? k0[jj] : 0.0;
        }
    } else {  // T1 = I
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int jj = lane + WAVE * q;
            const bool in = jj >= c0 && jj < mu;
            row.t[q] = (in && jj == kk) ? 1.0 : 0.0;
            row.k[q] = in ? k0[jj] : 0.0;
        }
    }
}

template <int QM>
__device__ __forceinline__ void combine_row(double (&row)[QM], const PRow<QM>& r, double a) {
#pragma unroll
    for (int q = 0; q < QM; ++q) row[q] = fma(a, r.t[q], r.k[q]);
}


// value of the distributed vector v at index i (wave-uniform i)
template <int QM>
__device__ __forceinline__ double dist_get(const double (&v)[QM], int i) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < QM; ++q)
        if (q == i / WAVE) t = v[q];
    return bcast_lane(t, i % WAVE);
}

template <int QM>
__device__ __forceinline__ void dist_set(double (&v)[QM], int i, double x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < QM; ++q)
        if (q == i / WAVE && lane == i % WAVE) v[q] = x;
}

// ----------------------------------------------------- spectral scale sigma
// sigma ~ sqrt(theta_small theta_max), the scale that balances the Gauss-Chebyshev
// rule's error at both ends of the spectrum of H_hat (the sketched Ritz values).
// theta_max: power iteration with H_hat, the mean of log ||H x|| over the second half
// of SIG_IT normalised steps (settles on the modulus also for a complex dominant
// pair).  theta_small = beta / ||H_hat^-1 beta e_1||, from the a = 0 node solve the
// kernel makes anyway: the smallest scale of the spectrum as the right-hand side
// sees it.  On the batched workload this lands within 0.05x..4x of the eigenvalue
// optimum sqrt(|theta|_min |theta|_max), where the rule converges within a few
// hundred nodes; the geometric mean of all moduli (|det H_hat|^(1/mu)) was 9x..90x
// off and needed up to 1395.  That mean is the fallback if an estimate is not finite.
constexpr int SIG_IT = 10;

__device__ __forceinline__ void sig_start(int mu, double* xs) {
    const int lane = threadIdx.x & 63;
    // a fixed start vector with every component nonzero
    double t = 0.0;
    for (int i = lane; i < mu; i += WAVE) {
        const double v = 1.0 + 0.25 * (double)((i * 7) % 11);
        xs[i] = v;
        t = fma(v, v, t);
    }
    t = wave_sum(t);
    __syncthreads();
    const double r = 1.0 / sqrt(t);
    for (int i = lane; i < mu; i += WAVE) xs[i] *= r;
    __syncthreads();
}

// ys <- ys / ||ys||; returns log ||ys|| (before the scaling); xs <- the scaled ys
__device__ __forceinline__ double sig_normalise(int mu, double* xs, const double* ys) {
    const int lane = threadIdx.x & 63;
    double t = 0.0;
    for (int i = lane; i < mu; i += WAVE) t = fma(ys[i], ys[i], t);
    t = wave_sum(t);
    const double r = 1.0 / sqrt(t);
    __syncthreads();
    for (int i = lane; i < mu; i += WAVE) xs[i] = ys[i] * r;
    __syncthreads();
    return 0.5 * log(t);
}

// ------------------------------------------------- conditioning of R (Section 2.1)
// The remark after eq. (sFOM''') suggests a numerical pseudoinverse in place of
// R_m^-1 when SV_m, and so R_m, is extremely ill-conditioned.  The one used here
// is the truncated QR one in the order of the Krylov basis: the leading blocks
// R_j = R[:j, :j] are the QR factors of the prefixes SV_j (the same Householder
// steps), kappa_F(R_j) = ||R_j||_F ||R_j^-1||_F never decreases with j, and the
// approximant is formed from the longest prefix with kappa_F(R_j) <= cmax.
// R_j^-1 is the leading block of R^-1, so one inverse gives every prefix: column
// c of R^-1 (support rows 0..c) is a back substitution, one wavefront per column.
// The prefix then looks to the rest of the small problem exactly like a run of
// j steps: its extension column S u_{j+1} = h_{j+1,j} S v_{j+1} is, after the first
// j reflectors, h_{j+1,j} times rows 0..j of the factored column j.
constexpr int RC_NT = 256;  // wavefronts per block of the column kernel: 4

// cnd[c] = ||R^-1 e_c||^2, cnd[m + 1 + c] = ||R[:c+1, c]||^2 for c < mu.
template <int QM>
__device__ __forceinline__ void rinv_col_body(int c, const double* __restrict__ X, int s,
                                              const DevCtrl* ctrl, int m, double* __restrict__ cnd) {
    const int mu = ctrl->m_used;
    if (c >= mu) return;
    const int lane = threadIdx.x & 63;
    double r[QM], dinv[QM];
    double g = 0.0;
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int i = lane + WAVE * q;
        r[q] = (i == c) ? 1.0 : 0.0;
        dinv[q] = (i <= c) ? 1.0 / X[i + (int64_t)s * i] : 0.0;
        const double v = (i <= c) ? X[i + (int64_t)s * c] : 0.0;
        g = fma(v, v, g);
    }
    // x = R^-1 e_c, columns of R from c down to 0, BF columns in flight
    constexpr int BF = 4;
    double cb[BF][QM];
#pragma unroll
    for (int f = 0; f < BF; ++f) {
        const int col = c - f;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = lane + WAVE * q;
            cb[f][q] = (col >= 0 && i < col) ? X[i + (int64_t)s * col] : 0.0;
        }
    }
    for (int l = c; l >= 0; --l) {
        const double xl = dist_get(r, l) * dist_get(dinv, l);
        dist_set(r, l, xl);
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = lane + WAVE * q;
            if (i < l) r[q] = fma(-cb[0][q], xl, r[q]);
        }
#pragma unroll
        for (int f = 0; f + 1 < BF; ++f)
#pragma unroll
            for (int q = 0; q < QM; ++q) cb[f][q] = cb[f + 1][q];
        const int col = l - BF;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = lane + WAVE * q;
            cb[BF - 1][q] = (col >= 0 && i < col) ? X[i + (int64_t)s * col] : 0.0;
        }
    }
    double n = 0.0;
#pragma unroll
    for (int q = 0; q < QM; ++q)
        if (lane + WAVE * q <= c) n = fma(r[q], r[q], n);
    n = wave_sum(n);
    g = wave_sum(g);
    if (lane == 0) {
        cnd[c] = n;
        cnd[m + 1 + c] = g;
    }
}

template <int QM>
__global__ __launch_bounds__(RC_NT) void rinv_col_kernel(const double* X, int s, const DevCtrl* ctrl, int m,
                                                         double* cnd) {
    rinv_col_body<QM>(blockIdx.x * (RC_NT / WAVE) + (threadIdx.x >> 6), X, s, ctrl, m, cnd);
}

template <int QM>
__global__ __launch_bounds__(RC_NT) void rinv_col_batched_kernel(const SmallUnit* __restrict__ units, int s, int m) {
    const SmallUnit& u = units[blockIdx.y];
    rinv_col_body<QM>(blockIdx.x * (RC_NT / WAVE) + (threadIdx.x >> 6), u.SV, s, u.ctrl, m, u.cnd);
}

// The prefix: kappa_F(R_j) from the prefix sums of cnd (fixed order: per-lane
// chunks, then an exclusive scan of the 64 chunk sums by lane 0), j' = the number of
// prefixes within cmax.  rcond reports 1 / kappa_F of the factor used.  If
// j' < mu, column j' of X becomes the extension column of the j'-step problem and
// m_used drops to j' (flag bit 0).  One wavefront.
__device__ __forceinline__ void cond_trunc_body(DevCtrl* ctrl, double* X, int s, const double* H, int64_t ldh,
                                                int m, const double* cnd, double cmax) {
    __shared__ double fsum[WAVE + 1], gsum[WAVE + 1];
    __shared__ int cnt[WAVE];
    __shared__ double kap[WAVE];
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const int lane = threadIdx.x;
    const int per = (mu + WAVE - 1) / WAVE;
    const int c0 = min(lane * per, mu), c1 = min(c0 + per, mu);
    auto fin = [](double v) { return (v <= 1.7976931348623157e308) ? v : INFINITY; };  // NaN -> inf
    double fs = 0.0, gs = 0.0;
    for (int c = c0; c < c1; ++c) { fs += fin(cnd[c]); gs += fin(cnd[m + 1 + c]); }
    fsum[lane + 1] = fs;
    gsum[lane + 1] = gs;
    __syncthreads();
    if (lane == 0) {
        fsum[0] = 0.0; gsum[0] = 0.0;
        for (int i = 1; i <= WAVE; ++i) { fsum[i] += fsum[i - 1]; gsum[i] += gsum[i - 1]; }
    }
    __syncthreads();
    double F = fsum[lane], G = gsum[lane];
    int n = 0;
    double klast = 0.0;
    for (int c = c0; c < c1; ++c) {
        F += fin(cnd[c]);
        G += fin(cnd[m + 1 + c]);
        const double k = sqrt(F * G);
        if (k <= cmax) { ++n; klast = k; }
    }
    cnt[lane] = n;
    kap[lane] = klast;
    __syncthreads();
    if (lane == 0) {
        int mp = 0;
        double kp = 0.0;
        for (int i = 0; i < WAVE; ++i) {
            if (cnt[i] > 0) kp = kap[i];
            mp += cnt[i];
        }
        ctrl->m_basis = mu;
        ctrl->rcond = (mp > 0 && kp > 0.0) ? 1.0 / kp : 0.0;
        if (mp == 0) {
            if (ctrl->status == 0) ctrl->status = 3;  // SKFAB_ERR_RANK: R_11 = 0
        } else if (mp < mu) {
            ctrl->m_used = mp;
            ctrl->flags |= 1;
        }
        cnt[0] = mp;
    }
    __syncthreads();
    const int mp = cnt[0];
    if (mp > 0 && mp < mu) {
        const double h = H[mp + ldh * (mp - 1)];
        for (int i = lane; i <= mp; i += WAVE) X[i + (int64_t)s * mp] *= h;
    }
}

__global__ __launch_bounds__(64) void cond_trunc_kernel(DevCtrl* ctrl, double* X, int s, const double* H, int m,
                                                        const double* cnd, double cmax) {
    cond_trunc_body(ctrl, X, s, H, m + 1, m, cnd, cmax);
}

__global__ __launch_bounds__(64) void cond_trunc_batched_kernel(const SmallUnit* __restrict__ units, int s, int m,
                                                                double cmax) {
    const SmallUnit& u = units[blockIdx.y];
    cond_trunc_body(u.ctrl, u.SV, s, u.H, m + 1, m, u.cnd, cmax);
}

// ------------------------------------------------------------- H_hat rows
// H_hat = H_mu + x e_mu^T with x = R^-1 r, r = R_e[:mu, mu] (the extension column
// of the QR'd sketch): the projected matrix of the sketched FOM in the basis V_m
// (remark of Section 2.2).  Written row-major into Hh (ld m) for the square node
// systems (t I + H_hat) y = beta e_1.  Block 0 (1024 threads) computes x by
// blocked back substitution: for each 64-column block from the right, its
// diagonal block is solved from LDS by wavefront 0 (one lane per row) while the
// other wavefronts already hold the block's columns of the rows above (one
// wavefront per row: a coalesced read and a wavefront sum) and the next diagonal
// block; every read of T1 is thus in flight during a solve.  Blocks 1..ncb copy
// H's first mu - 1 columns into Hh meanwhile (one column per wavefront); with ncb
// = 0 (the batched form, where the units already fill the device) block 0 copies
// them itself first.
constexpr int HH_NT = 1024;
constexpr int HH_B = 64;
constexpr int HH_CB = 15;

template <int QM>
__device__ __forceinline__ void hhat_rows_body(int blk, int ncb, const DevCtrl* ctrl, int m, int s,
                                              const double* __restrict__ X, const double* __restrict__ T1r,
                                              const double* __restrict__ H, double* __restrict__ Hh) {
    __shared__ double xs[MMAX];
    __shared__ double D[HH_B][HH_B + 1];
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int NWV = HH_NT / WAVE;
    const int64_t ldh = m + 1;
    if (blk > 0 || ncb == 0) {
        // column j of H into column j of the row-major Hh (QM * 64 >= m rows: every
        // read is issued before the first store)
        const int nbk = (ncb > 0) ? ncb : 1, bk = (ncb > 0) ? blk - 1 : 0;
        for (int j = bk * NWV + wid; j < mu - 1; j += nbk * NWV) {
            double v[QM];
#pragma unroll
            for (int q = 0; q < QM; ++q) v[q] = H[min(lane + WAVE * q, mu - 1) + ldh * j];
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int i = lane + WAVE * q;
                if (i < mu) Hh[(int64_t)i * m + j] = v[q];
            }
        }
        if (blk > 0) return;
    }
    // rows above a diagonal block held by one wavefront: w, w + NWV, ... (< QM * 64 - 64)
    constexpr int UR = (QM * WAVE - HH_B) / NWV;
    constexpr int DPT = HH_B * HH_B / HH_NT;  // entries of a diagonal block per thread
    for (int i = tid; i < mu; i += HH_NT) xs[i] = X[i + (int64_t)s * mu];
    int kb = ((mu - 1) / HH_B) * HH_B;
    {
        const int nb = mu - kb;
#pragma unroll
        for (int u = 0; u < DPT; ++u) {
            const int idx = tid + HH_NT * u, a = idx / HH_B, b = idx % HH_B;
            if (a < nb && b < nb) D[a][b] = (b >= a) ? T1r[(int64_t)(kb + a) * m + (kb + b)] : 0.0;
        }
    }
    for (; kb >= 0; kb -= HH_B) {
        const int nb = min(HH_B, mu - kb);
        const int rlast = max(kb - 1, 0);
        double pr[UR];
#pragma unroll
        for (int t = 0; t < UR; ++t)
            pr[t] = T1r[(int64_t)min(wid + NWV * t, rlast) * m + kb + min(lane, nb - 1)];
        const int kn = kb - HH_B;  // next block (full width)
        double dn[DPT];
#pragma unroll
        for (int u = 0; u < DPT; ++u) {
            const int idx = tid + HH_NT * u, a = idx / HH_B, b = idx % HH_B;
            const int rn = min(max(kn, 0) + a, mu - 1), cn = min(max(kn, 0) + b, mu - 1);
            dn[u] = (kn >= 0 && b >= a) ? T1r[(int64_t)rn * m + cn] : 0.0;
        }
        __syncthreads();  // D and the previous update of xs complete
        if (wid == 0) {
            const bool in = lane < nb;
            double r = in ? xs[kb + lane] : 0.0;
            const double di = in ? 1.0 / D[lane][lane] : 0.0;
            double dc = D[lane][nb - 1];
            for (int a = nb - 1; a >= 0; --a) {
                const double dnx = D[lane][a > 0 ? a - 1 : 0];  // next column, read off the chain
                const double xa = bcast_lane(r * di, a);
                r = (lane < a) ? fma(-dc, xa, r) : ((lane == a) ? xa : r);
                dc = dnx;
            }
            if (in) xs[kb + lane] = r;
        }
        __syncthreads();  // x of the block complete; D free
        if (kn >= 0) {
#pragma unroll
            for (int u = 0; u < DPT; ++u) {
                const int idx = tid + HH_NT * u;
                D[idx / HH_B][idx % HH_B] = dn[u];
            }
        }
        // rows above the block: xs[i] -= R[i, kb:kb+nb] x[kb:kb+nb]
        const double xb = (lane < nb) ? xs[kb + lane] : 0.0;
#pragma unroll
        for (int t = 0; t < UR; ++t) {
            const int i = wid + NWV * t;
            if (i < kb) {
                const double v = wave_sum((lane < nb) ? pr[t] * xb : 0.0);
                if (lane == 0) xs[i] -= v;
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < mu; i += HH_NT) Hh[(int64_t)i * m + (mu - 1)] = H[i + ldh * (mu - 1)] + xs[i];
}

template <int QM>
__global__ __launch_bounds__(HH_NT) void hhat_rows_kernel(const DevCtrl* ctrl, int m, int s, const double* X,
                                                         const double* T1r, const double* H, double* Hh) {
    hhat_rows_body<QM>(blockIdx.x, HH_CB, ctrl, m, s, X, T1r, H, Hh);
}

template <int QM>
__global__ __launch_bounds__(HH_NT) void hhat_rows_batched_kernel(const SmallUnit* __restrict__ units, int m, int s) {
    const SmallUnit& u = units[blockIdx.y];
    hhat_rows_body<QM>(0, 0, u.ctrl, m, s, u.SV, u.T1r, u.H, u.Hh);
}

// Solves with P(a) = a T1 + K0 (upper Hessenberg), right-hand side rhs0 e_1.
//   LS = false: square system P[:mu] y = rhs0 e_1 (Gaussian elimination with
//               partial pivoting between the two candidate rows of each column)
//   LS = true:  least squares min || rhs0 e_1 - P y || over the (mu+1) x mu pencil
//               (Givens rotations)
// One wavefront; vectors are distributed as index lane + 64 q.  The triangular
// factor goes column-major into Ucol (column jj at jj * m), read back column by
// column by the (reduction-free) back substitution.  With DET the sign of
// det(P[:mu]) is returned in *sgn (row swaps times the signs of the pivots) and
// the pivots are left on the diagonal of Ucol for the caller.
template <bool LS, bool DET, int QM>
__device__ void pencil_solve_wave(int mu, int m, double a, const double* __restrict__ T1r,
                                  const double* __restrict__ K0r, double rhs0, double* __restrict__ Ucol,
                                  const double* rhsv, double* __restrict__ y, double* logdet, double* sgn) {
    const int lane = threadIdx.x & 63;
    constexpr int PF = QM <= 4 ? 4 : 2;  // rows of the pencil in flight ahead of the elimination
    double carry[QM], next[QM];
    PRow<QM> pref[PF];
    double rv[QM], ud[QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) { rv[q] = 0.0; ud[q] = 1.0; }
    {
        PRow<QM> r0;
        load_pencil_row(r0, 0, 0, mu, m, T1r, K0r);
        combine_row(carry, r0, a);
    }
    const int last = LS ? mu : mu - 1;  // number of eliminations; rows 1..last are read
#pragma unroll
    for (int f = 0; f < PF; ++f)
        if (1 + f <= last) load_pencil_row(pref[f], 1 + f, f, mu, m, T1r, K0r);
    // right-hand side rhs0 e_1, or (square case) the vector rhsv, read row by row
    double rc = (!LS && rhsv) ? rhsv[0] : rhs0;
    double sg = 1.0;
    for (int kk = 0; kk < last; ++kk) {
        combine_row(next, pref[0], a);
#pragma unroll
        for (int f = 0; f + 1 < PF; ++f) pref[f] = pref[f + 1];
        // keep PF rows in flight while this column is eliminated
        if (kk + 1 + PF <= last) load_pencil_row(pref[PF - 1], kk + 1 + PF, kk + PF, mu, m, T1r, K0r);
        double rn = (!LS && rhsv) ? rhsv[kk + 1] : 0.0;
        double pk = dist_get(carry, kk);
        double nk = dist_get(next, kk);
        double* ucol = Ucol + kk;  // row kk of U: element (kk, jj) at jj * m + kk
        if (!LS) {
            if (fabs(nk) > fabs(pk)) {
#pragma unroll
                for (int q = 0; q < QM; ++q) { const double t = carry[q]; carry[q] = next[q]; next[q] = t; }
                const double tr = rn; rn = rc; rc = tr;
                const double tp = pk; pk = nk; nk = tp;
                if (DET) sg = -sg;
            }
            const double l = (pk != 0.0) ? nk / pk : 0.0;
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int jj = lane + WAVE * q;
                if (jj >= kk && jj < mu) ucol[(int64_t)jj * m] = carry[q];
                next[q] = fma(-l, carry[q], next[q]);
            }
            dist_set(rv, kk, rc);
            dist_set(ud, kk, pk);
            rn = fma(-l, rc, rn);
        } else {
            const double r = sqrt(fma(pk, pk, nk * nk));
            const double rinv = (r != 0.0) ? 1.0 / r : 0.0;
            const double c = (r != 0.0) ? pk * rinv : 1.0;
            const double sn = nk * rinv;
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int jj = lane + WAVE * q;
                const double top = fma(c, carry[q], sn * next[q]);
                const double bot = fma(-sn, carry[q], c * next[q]);
                if (jj >= kk && jj < mu) ucol[(int64_t)jj * m] = top;
                next[q] = bot;
            }
            dist_set(rv, kk, c * rc);
            dist_set(ud, kk, r);
            rn = -sn * rc;
        }
#pragma unroll
        for (int q = 0; q < QM; ++q) carry[q] = next[q];
        rc = rn;
    }
    if (!LS) {
        // last diagonal entry
        const int kk = mu - 1;
        const double pk = dist_get(carry, kk);
        if (lane == kk % WAVE) Ucol[(int64_t)kk * m + kk] = pk;
        dist_set(rv, kk, rc);
        dist_set(ud, kk, pk);
    }
    if (DET) {
        double neg = 0.0;
#pragma unroll
        for (int q = 0; q < QM; ++q)
            if (lane + WAVE * q < mu && ud[q] < 0.0) neg += 1.0;
        neg = wave_sum_fast(neg);
        if (((int)neg) & 1) sg = -sg;
    }
    // reciprocals of the diagonal, all at once
    double dinv[QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) dinv[q] = (lane + WAVE * q < mu) ? 1.0 / ud[q] : 0.0;
    __threadfence_block();  // Ucol written by this wave becomes visible to all of its lanes
    // column-oriented back substitution: y_k = r_k / U_kk, then r_i -= U_ik y_k (i < k)
    constexpr int BF = QM <= 4 ? 4 : 2;  // columns of U in flight
    double yv[QM], cbuf[BF][QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) yv[q] = 0.0;
#pragma unroll
    for (int f = 0; f < BF; ++f) {
        const int col = mu - 1 - f;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = lane + WAVE * q;
            cbuf[f][q] = (col >= 0 && i < col) ? Ucol[(int64_t)col * m + i] : 0.0;
        }
    }
    for (int kk = mu - 1; kk >= 0; --kk) {
        const double yk = dist_get(rv, kk) * dist_get(dinv, kk);
        dist_set(yv, kk, yk);
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = lane + WAVE * q;
            if (i < kk) rv[q] = fma(-cbuf[0][q], yk, rv[q]);
        }
#pragma unroll
        for (int f = 0; f + 1 < BF; ++f)
#pragma unroll
            for (int q = 0; q < QM; ++q) cbuf[f][q] = cbuf[f + 1][q];
        const int col = kk - BF;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = lane + WAVE * q;
            cbuf[BF - 1][q] = (col >= 0 && i < col) ? Ucol[(int64_t)col * m + i] : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int jj = lane + WAVE * q;
        if (jj < mu) y[jj] = yv[q];
    }
    if (logdet) *logdet = 0.0;
    if (sgn) *sgn = sg;
}

// Node 0 (a = 0): log|det H_hat| and its sign (square case), the spectral scale
// sigma (see sig_start), the branch check for z^(-1/2) (a negative determinant means
// an odd number of negative real eigenvalues), and -- for f = 1/z -- the solution
// itself (H_hat y = beta e_1, or the least-squares pencil problem for sGMRES).
template <int QM>
__device__ __forceinline__ void pencil_scalars_body(int m, int s, const double* X, const DevCtrl* ctrl_c,
                                                   DevCtrl* ctrl, const double* eta, const double* T1r,
                                                   const double* K0r, const double* Hh, double* Ubuf, double* Urhs,
                                                   double* y0, int is_ls, int branch_check) {
    const int mu = ctrl_c->m_used;
    if (mu == 0) return;
    const int lane = threadIdx.x;
    const double beta = eta[0];
    double ld = 0.0, sg = 1.0;
    if (is_ls) {
        pencil_solve_wave<true, false, QM>(mu, m, 0.0, T1r, K0r, beta * X[0], Ubuf, nullptr, y0, nullptr, nullptr);
    } else {
        // H_hat y = beta e_1: the a = 0 system of the square case, and det H_hat
        pencil_solve_wave<false, true, QM>(mu, m, 0.0, nullptr, Hh, beta, Ubuf, nullptr, y0, nullptr, &sg);
        // log|det| = sum log|U_kk| (sg already holds the sign: row swaps and pivot signs)
        double lu = 0.0;
        for (int kk = lane; kk < mu; kk += 64) lu += log(fabs(Ubuf[(int64_t)kk * m + kk]));
        ld = wave_sum_fast(lu);
    }
    double lsig = NAN;
    if (!is_ls) {
        // sigma as in the band form: power iteration with the rows of H_hat (one row per
        // step across the lanes), the small scale from y0 = H_hat^-1 beta e_1
        __shared__ double xs[MMAX], ys[MMAX];
        double lmax = 0.0;
        __syncthreads();  // y0 of the a = 0 solve complete
        double y2 = 0.0;
        for (int i = lane; i < mu; i += WAVE) y2 = fma(y0[i], y0[i], y2);
        const double lsmall = log(beta) - 0.5 * log(wave_sum(y2));
        sig_start(mu, xs);
        for (int it = 0; it < SIG_IT; ++it) {
            for (int i = 0; i < mu; ++i) {
                double t = 0.0;
                for (int jj = max(i - 1, 0) + lane; jj < mu; jj += WAVE) t = fma(Hh[(int64_t)i * m + jj], xs[jj], t);
                t = wave_sum(t);
                if (lane == 0) ys[i] = t;
            }
            __syncthreads();
            const double l = sig_normalise(mu, xs, ys);
            if (it >= SIG_IT / 2) lmax += l;
        }
        lsig = 0.5 * (lmax / (SIG_IT / 2) + lsmall);
    }
    if (lane == 0) {
        ctrl->beta = beta;
        if (!is_ls) {
            const double lg = ld / mu;
            ctrl->logdet = ld;
            ctrl->sigma = isfinite(lsig) ? exp(lsig) : exp(lg);
            const double sdet = sg;  // sign of det H_hat
            if (branch_check && sdet < 0.0 && ctrl->status == 0) ctrl->status = 4;  // SKFAB_ERR_BRANCH
            if (!isfinite(lg) && ctrl->status == 0) ctrl->status = 3;
        }
    }
}

template <int QM>
__global__ __launch_bounds__(64) void pencil_setup_scalars_kernel(int m, int s, const double* X, const DevCtrl* ctrl_c,
                                                                  DevCtrl* ctrl, const double* eta,
                                                                  const double* T1r, const double* K0r,
                                                                  const double* Hh, double* Ubuf, double* Urhs,
                                                                  double* y0, int is_ls, int branch_check) {
    pencil_scalars_body<QM>(m, s, X, ctrl_c, ctrl, eta, T1r, K0r, Hh, Ubuf, Urhs, y0, is_ls, branch_check);
}

template <int QM>
__global__ __launch_bounds__(64) void pencil_scalars_batched_kernel(const SmallUnit* __restrict__ units, int m, int s,
                                                                    int is_ls, int branch_check) {
    const SmallUnit& u = units[blockIdx.y];
    pencil_scalars_body<QM>(m, s, u.SV, u.ctrl, u.ctrl, u.eta, u.T1r, u.K0r, u.Hh, u.Ubuf, u.Urhs, u.y0, is_ls,
                            branch_check);
}

// sigma for the least-squares case: use the square pencil's scale as well.
// (Called before the LS setup kernel; see host sequence.)

// ------------------------------------------------ quadrature levels
// One launch evaluates every node of a group of consecutive orders (the nodes
// are independent, Section 5.3); the reduction then applies the acceptance test
// of Section 4.1 to the orders in sequence.
template <int QM>
__device__ __forceinline__ void quad_level_body(const DevCtrl* ctrl, const QuadGroup& grp, const double* T1r,
                                               const double* K0r, const double* Hh, double* Ubuf, double* Urhs,
                                               double* nodebuf, int m, int is_ls, const double* X,
                                               const double* eta) {
    if (ctrl->converged || ctrl->status != 0) return;
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const double sigma = ctrl->sigma;
    // least squares: the pencil t R + R_e Hbar with rhs beta R_00 e_1; square:
    // t I + H_hat with rhs beta e_1 (the same solution, without the factor R)
    const double rhs0 = is_ls ? eta[0] * X[0] : eta[0];
    const int wave = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
    const int nwaves_total = gridDim.x * (blockDim.x / WAVE);
    double* U = Ubuf + (int64_t)wave * m * m;   // slot = global wave index < NODE_SLOTS
    double* Ur = Urhs + (int64_t)wave * m;
    for (int i = wave; i < grp.total; i += nwaves_total) {
        int lev = 0;
        while (lev + 1 < grp.nlev && i >= grp.lev_off[lev + 1]) ++lev;
        const int l = grp.lev_l[lev];
        const int ii = i - grp.lev_off[lev];
        const double x = cos((2.0 * ii + 1.0) * M_PI / (2.0 * l));
        const double t = (1.0 - x) / (1.0 + x);
        const double w = (2.0 / l) / (1.0 + x);
        double* yi = nodebuf + (int64_t)i * m;
        if (is_ls)
            pencil_solve_wave<true, false, QM>(mu, m, t * sigma, T1r, K0r, rhs0 * w, U, nullptr, yi, nullptr, nullptr);
        else
            pencil_solve_wave<false, false, QM>(mu, m, t * sigma, nullptr, Hh, rhs0 * w, U, nullptr, yi, nullptr, nullptr);
    }
}

// ------------------------------------------------ banded square node solves
// In the square case the node systems are (a I + H_hat) y = rhs0 e_1 with
// H_hat = H_m + r e_m^T: H_m from the k-truncated recurrence is zero outside
// i-1 <= c <= i+k-1, so a row of H_hat holds at most k+1 band entries plus its
// last-column entry.  Gaussian elimination with partial pivoting keeps that shape
// (two candidate rows per column), so one lane solves one node in O(m k).  The
// operations on the band entries are those of the dense Hessenberg elimination.
constexpr int BAND_NT = 256;

// Band rows of H_hat (row-major, ld m) into LDS: Bs[i KB + d] = H_hat[i][i-1+d] for
// 0 <= i-1+d < mu-1 (KB = k+1), Ls[i] = H_hat[i][mu-1]; whole block.
template <int KB>
__device__ __forceinline__ void load_band(const double* __restrict__ Hh, int m, int mu, double* Bs, double* Ls) {
    for (int idx = threadIdx.x; idx < mu * KB; idx += blockDim.x) {
        const int i = idx / KB, d = idx - i * KB, c = i - 1 + d;
        Bs[idx] = (c >= 0 && c < mu - 1) ? Hh[(int64_t)i * m + c] : 0.0;
    }
    for (int i = threadIdx.x; i < mu; i += blockDim.x) Ls[i] = Hh[(int64_t)i * m + (mu - 1)];
}

// One node on the calling lane: y (stride 1) <- (a I + H_hat)^-1 rhs0 e_1.  Row kk
// of U goes to Us[(kk (KB+2) + f) fstride], f = 0: reciprocal of the pivot (one
// division per row: the multiplier and the back substitution both use it),
// 1..KB-1: entries right of the pivot, KB: last column, KB+1: transformed
// right-hand side.  With DET, the last pivot's reciprocal goes to field 0 of row
// mu-1 (so that field 0 of row kk holds 1 / pivot_kk for every kk < mu) and *neg =
// parity of row swaps plus negative pivots (sign of the determinant).
template <int KB, bool DET>
__device__ __forceinline__ void band_node_solve(int mu, double a, double rhs0, const double* Bs, const double* Ls,
                                                double* __restrict__ Us, int64_t fstride, double* __restrict__ y,
                                                int* neg, const double* rhsv = nullptr) {
    constexpr int F = KB + 2;
    double c[KB];  // carry row: columns kk .. kk+KB-1 (the last slot is zero on entry)
#pragma unroll
    for (int d = 0; d + 1 < KB; ++d) c[d] = Bs[d + 1];
    c[KB - 1] = 0.0;
    double cL = Ls[0], cR = rhsv ? rhsv[0] : rhs0;
    if (mu > 1) c[0] += a;
    else cL += a;
    int ng = 0;
    for (int kk = 0; kk + 1 < mu; ++kk) {
        double n[KB];
#pragma unroll
        for (int d = 0; d < KB; ++d) n[d] = Bs[(kk + 1) * KB + d];
        double nL = Ls[kk + 1], nR = rhsv ? rhsv[kk + 1] : 0.0;
        if (kk + 2 < mu) n[1] += a;  // the diagonal of row kk+1 (in the last column for the last row)
        else nL += a;
        if (fabs(n[0]) > fabs(c[0])) {
#pragma unroll
            for (int d = 0; d < KB; ++d) { const double t = c[d]; c[d] = n[d]; n[d] = t; }
            double t = cL; cL = nL; nL = t;
            t = cR; cR = nR; nR = t;
            ng ^= 1;
        }
        const double p = c[0];
        const double rp = 1.0 / p;
        const double l = (p != 0.0) ? n[0] * rp : 0.0;
        double* u = Us + (int64_t)kk * F * fstride;
        u[0] = rp;
#pragma unroll
        for (int d = 1; d < KB; ++d) u[d * fstride] = c[d];
        u[KB * fstride] = cL;
        u[(KB + 1) * fstride] = cR;
        if (DET && p < 0.0) ng ^= 1;
#pragma unroll
        for (int d = 0; d + 1 < KB; ++d) c[d] = fma(-l, c[d + 1], n[d + 1]);
        c[KB - 1] = 0.0;
        cL = fma(-l, cL, nL);
        cR = fma(-l, cR, nR);
    }
    // last pivot: column mu-1 lives in the last-column slot
    const double pl = cL;
    const double rpl = 1.0 / pl;
    if (DET) {
        if (pl < 0.0) ng ^= 1;
        Us[(int64_t)(mu - 1) * F * fstride] = rpl;
    }
    const double ylast = cR * rpl;
    y[mu - 1] = ylast;
    // back substitution, columns in descending order as in the dense elimination;
    // yw[d] = y[kk+1+d] (zero beyond column mu-2: those band slots hold zeros).  The
    // fields of the next BPD rows are in flight while a row is used (clamped row
    // indices: unconditional loads, re-reading row 0 at the end).
    constexpr int BPD = 4;
    double yw[KB];
#pragma unroll
    for (int d = 0; d < KB; ++d) yw[d] = 0.0;
    double nu[BPD][F];
#pragma unroll
    for (int q = 0; q < BPD; ++q) {
        const double* u = Us + (int64_t)max(mu - 2 - q, 0) * F * fstride;
#pragma unroll
        for (int f = 0; f < F; ++f) nu[q][f] = u[f * fstride];
    }
    for (int kk = mu - 2; kk >= 0; --kk) {
        double cu[F];
#pragma unroll
        for (int f = 0; f < F; ++f) cu[f] = nu[0][f];
#pragma unroll
        for (int q = 0; q + 1 < BPD; ++q)
#pragma unroll
            for (int f = 0; f < F; ++f) nu[q][f] = nu[q + 1][f];
        {
            const double* u = Us + (int64_t)max(kk - BPD, 0) * F * fstride;
#pragma unroll
            for (int f = 0; f < F; ++f) nu[BPD - 1][f] = u[f * fstride];
        }
        double sres = fma(-cu[KB], ylast, cu[KB + 1]);
#pragma unroll
        for (int d = KB - 1; d >= 1; --d) sres = fma(-cu[d], yw[d - 1], sres);
        const double yk = sres * cu[0];
        y[kk] = yk;
#pragma unroll
        for (int d = KB - 1; d >= 1; --d) yw[d] = yw[d - 1];
        yw[0] = yk;
    }
    if (DET) *neg = ng;
}

// Nodes of a quadrature group, square case, one lane per node.  Ubuf holds the
// U rows of the group's nodes, field-major (node index fastest, stride grp.total:
// a group of one high order can hold more than NODE_SLOTS nodes).
template <int KB>
__device__ __forceinline__ void quad_level_band_body(const DevCtrl* ctrl, const QuadGroup& grp,
                                                     const double* __restrict__ Hh, double* Ubuf,
                                                     double* nodebuf, int m, const double* eta) {
    __shared__ double Bs[MMAX * KB];
    __shared__ double Ls[MMAX];
    if (ctrl->converged || ctrl->status != 0) return;
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    load_band<KB>(Hh, m, mu, Bs, Ls);
    __syncthreads();
    const int i = blockIdx.x * BAND_NT + threadIdx.x;
    if (i >= grp.total) return;
    int lev = 0;
    while (lev + 1 < grp.nlev && i >= grp.lev_off[lev + 1]) ++lev;
    const int l = grp.lev_l[lev];
    const int ii = i - grp.lev_off[lev];
    const double x = cos((2.0 * ii + 1.0) * M_PI / (2.0 * l));
    const double t = (1.0 - x) / (1.0 + x);
    const double w = (2.0 / l) / (1.0 + x);
    band_node_solve<KB, false>(mu, t * ctrl->sigma, eta[0] * w, Bs, Ls, Ubuf + i, grp.total,
                               nodebuf + (int64_t)i * m, nullptr);
}

template <int KB>
__global__ __launch_bounds__(BAND_NT) void quad_level_band_kernel(const DevCtrl* ctrl, QuadGroup grp,
                                                                  const double* Hh, double* Ubuf, double* nodebuf,
                                                                  int m, const double* eta) {
    quad_level_band_body<KB>(ctrl, grp, Hh, Ubuf, nodebuf, m, eta);
}

template <int KB>
__global__ __launch_bounds__(BAND_NT) void quad_level_band_batched_kernel(const SmallUnit* __restrict__ units,
                                                                          QuadGroup grp, int m) {
    const SmallUnit& u = units[blockIdx.y];
    quad_level_band_body<KB>(u.ctrl, grp, u.Hh, u.Ubuf, u.nodebuf, m, u.eta);
}

// Square case of the pencil scalars with the band elimination: beta, H_hat y0 = beta e_1 (lane 0), log|det H_hat|, sigma and the
// sign of det H_hat for the branch test.  One wavefront.
template <int KB>
__device__ __forceinline__ void pencil_scalars_band_body(int m, int s, const double* X, DevCtrl* ctrl,
                                                         const double* eta, const double* Hh, double* Ubuf,
                                                         double* y0, int branch_check) {
    __shared__ double Bs[MMAX * KB];
    __shared__ double Ls[MMAX];
    __shared__ double Us[MMAX * (KB + 2)];  // U rows of the one node (fstride 1)
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const int lane = threadIdx.x;
    (void)Ubuf;
    (void)X;
    (void)s;
    load_band<KB>(Hh, m, mu, Bs, Ls);
    __syncthreads();
    const double beta = eta[0];
    int ng = 0;
    if (lane == 0) band_node_solve<KB, true>(mu, 0.0, beta, Bs, Ls, Us, 1, y0, &ng);
    __syncthreads();
    // log|det H_hat| = sum log|pivot| = -sum log|1 / pivot| over the U rows, all
    // lanes (a log per pivot on the solving lane would lengthen its serial chain)
    double lu = 0.0;
    for (int kk = lane; kk < mu; kk += WAVE) lu += log(fabs(Us[kk * (KB + 2)]));
    const double ld = -wave_sum_fast(lu);
    // sigma: |theta|_max by power iteration (rows of H_hat over the lanes), the small
    // scale from y0 = H_hat^-1 beta e_1 (written by lane 0 above, visible after the barrier)
    __shared__ double xs[MMAX], ys[MMAX];
    double lmax = 0.0;
    double y2 = 0.0;
    for (int i = lane; i < mu; i += WAVE) y2 = fma(y0[i], y0[i], y2);
    const double lsmall = log(beta) - 0.5 * log(wave_sum(y2));
    sig_start(mu, xs);
    for (int it = 0; it < SIG_IT; ++it) {
        for (int i = lane; i < mu; i += WAVE) {
            double t = Ls[i] * xs[mu - 1];
#pragma unroll
            for (int d = 0; d < KB; ++d) {
                const int c = i - 1 + d;
                if (c >= 0 && c < mu - 1) t = fma(Bs[i * KB + d], xs[c], t);
            }
            ys[i] = t;
        }
        __syncthreads();
        const double l = sig_normalise(mu, xs, ys);
        if (it >= SIG_IT / 2) lmax += l;
    }
    const double lsig = 0.5 * (lmax / (SIG_IT / 2) + lsmall);  // log sqrt(theta_max theta_small)
    if (lane == 0) {
        ctrl->beta = beta;
        const double lg = ld / mu;
        ctrl->logdet = ld;
        ctrl->sigma = isfinite(lsig) ? exp(lsig) : exp(lg);
        if (branch_check && ng && ctrl->status == 0) ctrl->status = 4;  // SKFAB_ERR_BRANCH: det H_hat < 0
        if (!isfinite(lg) && ctrl->status == 0) ctrl->status = 3;
    }
}

template <int KB>
__global__ __launch_bounds__(64) void pencil_scalars_band_kernel(int m, int s, const double* X, DevCtrl* ctrl,
                                                                 const double* eta, const double* Hh, double* Ubuf,
                                                                 double* y0, int branch_check) {
    pencil_scalars_band_body<KB>(m, s, X, ctrl, eta, Hh, Ubuf, y0, branch_check);
}

template <int KB>
__global__ __launch_bounds__(64) void pencil_scalars_band_batched_kernel(const SmallUnit* __restrict__ units, int m,
                                                                         int s, int branch_check) {
    const SmallUnit& u = units[blockIdx.y];
    pencil_scalars_band_body<KB>(m, s, u.SV, u.ctrl, u.eta, u.Hh, u.Ubuf, u.y0, branch_check);
}

template <int QM>
__global__ __launch_bounds__(256) void quad_level_kernel(const DevCtrl* ctrl, QuadGroup grp, const double* T1r,
                                                         const double* K0r, const double* Hh, double* Ubuf,
                                                         double* Urhs, double* nodebuf, int m, int is_ls,
                                                         const double* X, const double* eta) {
    quad_level_body<QM>(ctrl, grp, T1r, K0r, Hh, Ubuf, Urhs, nodebuf, m, is_ls, X, eta);
}

template <int QM>
__global__ __launch_bounds__(256) void quad_level_batched_kernel(const SmallUnit* __restrict__ units, QuadGroup grp,
                                                                 int m, int is_ls) {
    const SmallUnit& u = units[blockIdx.y];
    quad_level_body<QM>(u.ctrl, grp, u.T1r, u.K0r, u.Hh, u.Ubuf, u.Urhs, u.nodebuf, m, is_ls, u.SV, u.eta);
}

// For each level of the group: q_l = sqrt(sigma) sum_i nodebuf[i] (fixed order), and
// the whitened norms ||R q_l||, ||R (q_l - q_{l-1})|| (R = R_e[:mu,:mu]); levels are
// summed in parallel (one wavefront each), then the acceptance test of Section 4.1
// is applied in sequence: the sequence's first level only seeds qprev; accept q_l
// when ||R (q_l - q_prev)|| <= tol ||R q_l||.

__device__ __forceinline__ void quad_reduce_body(DevCtrl* ctrl, const QuadGroup& grp, const double* nodebuf, int m,
                                                double tol, const double* T1r, double* qprev, double* y,
                                                double* qlev) {
    __shared__ double nd[MAX_GROUP_LEVELS], nc[MAX_GROUP_LEVELS];
    __shared__ double qs[MAX_GROUP_LEVELS + 1][MMAX];
    if (ctrl->converged || ctrl->status != 0) return;
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const double sq = sqrt(ctrl->sigma);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // q of every level (row 0 of qs holds the previous group's last rule)
    for (int jj = threadIdx.x; jj < mu; jj += 1024) qs[0][jj] = qprev[jj];
    for (int lev = wid; lev < grp.nlev; lev += 16) {
        const int l = grp.lev_l[lev], off = grp.lev_off[lev];
        for (int jj = lane; jj < mu; jj += 64) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int i = 0;
            for (; i + 3 < l; i += 4) {
                a0 += nodebuf[(int64_t)(off + i) * m + jj];
                a1 += nodebuf[(int64_t)(off + i + 1) * m + jj];
                a2 += nodebuf[(int64_t)(off + i + 2) * m + jj];
                a3 += nodebuf[(int64_t)(off + i + 3) * m + jj];
            }
            for (; i < l; ++i) a0 += nodebuf[(int64_t)(off + i) * m + jj];
            qs[lev + 1][jj] = ((a0 + a1) + (a2 + a3)) * sq;
        }
    }
    __syncthreads();
    // whitened norms, one wavefront per level: rows of R spread over lanes
    for (int lev = wid; lev < grp.nlev; lev += 16) {
        double td_all = 0.0, tc_all = 0.0;
        for (int i = lane; i < mu; i += 64) {
            double d0 = 0.0, d1 = 0.0, c0 = 0.0, c1 = 0.0;
            int jj = i;
            for (; jj + 1 < mu; jj += 2) {
                const double r0 = T1r[(int64_t)i * m + jj], r1 = T1r[(int64_t)i * m + jj + 1];
                d0 = fma(r0, qs[lev + 1][jj] - qs[lev][jj], d0);
                d1 = fma(r1, qs[lev + 1][jj + 1] - qs[lev][jj + 1], d1);
                c0 = fma(r0, qs[lev + 1][jj], c0);
                c1 = fma(r1, qs[lev + 1][jj + 1], c1);
            }
            if (jj < mu) {
                const double r0 = T1r[(int64_t)i * m + jj];
                d0 = fma(r0, qs[lev + 1][jj] - qs[lev][jj], d0);
                c0 = fma(r0, qs[lev + 1][jj], c0);
            }
            td_all = fma(d0 + d1, d0 + d1, td_all);
            tc_all = fma(c0 + c1, c0 + c1, tc_all);
        }
        td_all = wave_sum(td_all);
        tc_all = wave_sum(tc_all);
        if (lane == 0) { nd[lev] = td_all; nc[lev] = tc_all; }
    }
    __syncthreads();
    int acc_lev = -1;
    int last = grp.nlev - 1;
    bool bad = false, floor_acc = false;
    double dprev = ctrl->qdiff_prev, dacc = 0.0;
    for (int lev = 0; lev < grp.nlev; ++lev) {
        if (grp.first && lev == 0) continue;
        if (!isfinite(nd[lev]) || !isfinite(nc[lev])) { bad = true; last = lev; break; }
        // relative difference of consecutive orders; accepted below tol, or at the
        // rounding floor: below QUAD_FLOOR and no longer falling (d > d_prev / 2), or
        // below QUAD_FLOOR at the final order of the sequence
        const double d = (nc[lev] > 0.0) ? sqrt(nd[lev] / nc[lev]) : (nd[lev] > 0.0 ? INFINITY : 0.0);
        const bool final_order = grp.last && lev == grp.nlev - 1;
        if (d <= tol || (d <= QUAD_FLOOR && (d > 0.5 * dprev || final_order))) {
            acc_lev = lev;
            dacc = d;
            floor_acc = d > tol;
            break;
        }
        dprev = d;
    }
    if (acc_lev >= 0) {
        for (int jj = threadIdx.x; jj < mu; jj += 1024) y[jj] = qs[acc_lev + 1][jj];
    } else {
        for (int jj = threadIdx.x; jj < mu; jj += 1024) qprev[jj] = qs[last + 1][jj];
    }
    if (threadIdx.x == 0) {
        if (acc_lev >= 0) {
            ctrl->converged = 1;
            ctrl->l_used = grp.lev_l[acc_lev];
            ctrl->quad_diff = dacc;
            if (floor_acc) ctrl->flags |= 2;
        }
        else { ctrl->l_prev = grp.lev_l[last]; ctrl->qdiff_prev = dprev; }
        if (bad) ctrl->status = 5;
    }
}

__global__ __launch_bounds__(1024) void quad_reduce_kernel(DevCtrl* ctrl, QuadGroup grp, const double* nodebuf, int m,
                                                           double tol, const double* T1r, double* qprev, double* y,
                                                           double* qlev) {
    quad_reduce_body(ctrl, grp, nodebuf, m, tol, T1r, qprev, y, qlev);
}

__global__ __launch_bounds__(1024) void quad_reduce_batched_kernel(const SmallUnit* __restrict__ units, QuadGroup grp,
                                                                   int m, double tol) {
    const SmallUnit& u = units[blockIdx.y];
    quad_reduce_body(u.ctrl, grp, u.nodebuf, m, tol, u.T1r, u.qprev, u.y0, nullptr);
}

__global__ void quad_fail_kernel(DevCtrl* ctrl) {
    if (threadIdx.x == 0 && ctrl->status == 0 && !ctrl->converged && ctrl->m_used > 0) ctrl->status = 5;
}

__global__ void quad_fail_batched_kernel(const SmallUnit* __restrict__ units) {
    DevCtrl* ctrl = units[blockIdx.y].ctrl;
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
__device__ __forceinline__ void finish_coeffs_body(DevCtrl* ctrl, int m, const double* y, const double* eta,
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

__global__ __launch_bounds__(256) void finish_coeffs_kernel(DevCtrl* ctrl, int m, const double* y, const double* eta,
                                                            const double* colnorm2, double* ys, double* yout) {
    finish_coeffs_body(ctrl, m, y, eta, colnorm2, ys, yout);
}

__global__ __launch_bounds__(256) void finish_coeffs_batched_kernel(const SmallUnit* __restrict__ units, int m) {
    const SmallUnit& u = units[blockIdx.y];
    finish_coeffs_body(u.ctrl, m, u.y0, u.eta, u.colnorm2, u.ys, u.y);
}

// x = U ys (N x mu times mu), rows parallel, coalesced over the basis columns; the
// basis is read in its storage type and accumulated in FP64.
template <typename VT>
__device__ __forceinline__ void assemble_body(const VT* __restrict__ U, int64_t ldU, int64_t N, int m,
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
            a0 = fma(to_w<double>(U[r + ldU * j]), c[j], a0);
            a1 = fma(to_w<double>(U[r + ldU * (j + 1)]), c[j + 1], a1);
            a2 = fma(to_w<double>(U[r + ldU * (j + 2)]), c[j + 2], a2);
            a3 = fma(to_w<double>(U[r + ldU * (j + 3)]), c[j + 3], a3);
        }
        for (; j < mu; ++j) a0 = fma(to_w<double>(U[r + ldU * j]), c[j], a0);
        x[r] = (a0 + a1) + (a2 + a3);
    }
}

template <typename VT>
__global__ __launch_bounds__(256) void assemble_kernel(const VT* __restrict__ U, int64_t ldU, int64_t N, int m,
                                                       const DevCtrl* ctrl, const double* __restrict__ ys,
                                                       double* __restrict__ x) {
    assemble_body<VT>(U, ldU, N, m, ctrl, ys, x);
}

template <typename VT>
__global__ __launch_bounds__(256) void assemble_batched_kernel(const SmallUnit* __restrict__ units, int m) {
    const SmallUnit& u = units[blockIdx.y];
    assemble_body<VT>(static_cast<const VT*>(u.U), u.ldU, u.N, m, u.ctrl, u.ys, u.x);
}

// Second pass of the two-pass form (Section 4.2): x += ys[j] u_j with the basis
// vector u_j just regenerated in its ring column (x = 0 before j = 0).  Steps at or
// beyond m_used (breakdown, or the conditioned prefix) add nothing.
template <typename VT>
__global__ __launch_bounds__(256) void accum_basis_kernel(const VT* __restrict__ Uj, int64_t N, int j,
                                                          const DevCtrl* ctrl, const double* __restrict__ ys,
                                                          double* __restrict__ x) {
    const int mu = ctrl->m_used;
    const bool add = j < mu;
    const double c = add ? ys[j] : 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
        const double base = (j == 0) ? 0.0 : x[r];
        x[r] = add ? fma(c, to_w<double>(Uj[r]), base) : base;
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_accum_basis(const void* Uj, int64_t N, int j, const DevCtrl* ctrl, const double* ys, double* x,
                              int prec, hipStream_t st) {
    int64_t g = (N + 255) / 256;
    const dim3 grid((unsigned)(g < 4096 ? g : 4096));
    if (prec == 1)
        hipLaunchKernelGGL(accum_basis_kernel<float>, grid, dim3(256), 0, st, static_cast<const float*>(Uj), N, j,
                           ctrl, ys, x);
    else if (prec == 2)
        hipLaunchKernelGGL(accum_basis_kernel<bf16s>, grid, dim3(256), 0, st, static_cast<const bf16s*>(Uj), N, j,
                           ctrl, ys, x);
    else
        hipLaunchKernelGGL(accum_basis_kernel<double>, grid, dim3(256), 0, st, static_cast<const double*>(Uj), N, j,
                           ctrl, ys, x);
    return hipGetLastError();
}

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

// Rows per lane of a panel with nrows rows (nrows <= SMAX = 64 * 16).
static int qr_rpw(int nrows) { return nrows <= 128 ? 2 : (nrows <= 256 ? 4 : (nrows <= 512 ? 8 : 16)); }

hipError_t launch_qr(double* X, int s, int ncols_max, const DevCtrl* ctrl, double* Tws, hipStream_t st) {
    for (int c0 = 0; c0 < ncols_max; c0 += QR_NB) {
        switch (qr_rpw(s - c0)) {
            case 2: hipLaunchKernelGGL(qr_panel_kernel<2>, dim3(1), dim3(QR_NT), 0, st, X, s, c0, ctrl, Tws); break;
            case 4: hipLaunchKernelGGL(qr_panel_kernel<4>, dim3(1), dim3(QR_NT), 0, st, X, s, c0, ctrl, Tws); break;
            case 8: hipLaunchKernelGGL(qr_panel_kernel<8>, dim3(1), dim3(QR_NT), 0, st, X, s, c0, ctrl, Tws); break;
            default: hipLaunchKernelGGL(qr_panel_kernel<16>, dim3(1), dim3(QR_NT), 0, st, X, s, c0, ctrl, Tws); break;
        }
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

hipError_t launch_hhat_rows(const DevCtrl* ctrl, int m, int s, const double* X, const double* T1r, const double* H,
                            double* Hh, hipStream_t st) {
    if (m <= 256)
        hipLaunchKernelGGL(hhat_rows_kernel<4>, dim3(1 + HH_CB), dim3(HH_NT), 0, st, ctrl, m, s, X, T1r, H, Hh);
    else
        hipLaunchKernelGGL(hhat_rows_kernel<8>, dim3(1 + HH_CB), dim3(HH_NT), 0, st, ctrl, m, s, X, T1r, H, Hh);
    return hipGetLastError();
}

// Square case with the band elimination: window k <= 4 and U rows that fit the
// node scratch (m >= k + 3); otherwise the dense one-wave elimination.
static bool band_ok(int k, int m) { return k >= 1 && k <= 4 && m >= k + 3; }

#define BAND_DISPATCH(KB_RT, LAUNCH)          \
    switch (KB_RT) {                          \
        case 2: { constexpr int KB = 2; LAUNCH; break; } \
        case 3: { constexpr int KB = 3; LAUNCH; break; } \
        case 4: { constexpr int KB = 4; LAUNCH; break; } \
        default: { constexpr int KB = 5; LAUNCH; break; } \
    }

hipError_t launch_pencil_scalars(int m, int s, const double* X, DevCtrl* ctrl, const double* eta,
                                 const double* T1r, const double* K0r, const double* Hh, double* Ubuf, double* Urhs,
                                 double* y0, int is_ls, int branch_check, int k, hipStream_t st) {
    if (!is_ls && band_ok(k, m)) {
        BAND_DISPATCH(k + 1, hipLaunchKernelGGL(pencil_scalars_band_kernel<KB>, dim3(1), dim3(64), 0, st, m, s, X,
                                                ctrl, eta, Hh, Ubuf, y0, branch_check));
        return hipGetLastError();
    }
    if (m <= 256)
        hipLaunchKernelGGL(pencil_setup_scalars_kernel<4>, dim3(1), dim3(64), 0, st, m, s, X, ctrl, ctrl, eta, T1r,
                           K0r, Hh, Ubuf, Urhs, y0, is_ls, branch_check);
    else
        hipLaunchKernelGGL(pencil_setup_scalars_kernel<8>, dim3(1), dim3(64), 0, st, m, s, X, ctrl, ctrl, eta, T1r,
                           K0r, Hh, Ubuf, Urhs, y0, is_ls, branch_check);
    return hipGetLastError();
}

hipError_t launch_quad_group(const DevCtrl* ctrl, const QuadGroup& g, const double* T1r, const double* K0r,
                             const double* Hh, double* Ubuf, double* Urhs, double* nodebuf, int m, int is_ls,
                             const double* X, const double* eta, int k, hipStream_t st) {
    // one lane per node; the U rows of all g.total nodes, (k + 3) m doubles each, fit the
    // NODE_SLOTS x m x m node scratch when g.total (k + 3) <= NODE_SLOTS m
    if (!is_ls && band_ok(k, m) && (int64_t)g.total * (k + 3) <= (int64_t)NODE_SLOTS * m) {
        const int blocks = (g.total + BAND_NT - 1) / BAND_NT;
        BAND_DISPATCH(k + 1, hipLaunchKernelGGL(quad_level_band_kernel<KB>, dim3(blocks), dim3(BAND_NT), 0, st, ctrl,
                                                g, Hh, Ubuf, nodebuf, m, eta));
        return hipGetLastError();
    }
    const int waves = g.total < NODE_SLOTS ? g.total : NODE_SLOTS;
    const int blocks = (waves + 3) / 4;
    if (m <= 256)
        hipLaunchKernelGGL(quad_level_kernel<4>, dim3(blocks), dim3(256), 0, st, ctrl, g, T1r, K0r, Hh, Ubuf, Urhs,
                           nodebuf, m, is_ls, X, eta);
    else
        hipLaunchKernelGGL(quad_level_kernel<8>, dim3(blocks), dim3(256), 0, st, ctrl, g, T1r, K0r, Hh, Ubuf, Urhs,
                           nodebuf, m, is_ls, X, eta);
    return hipGetLastError();
}

hipError_t launch_quad_reduce(DevCtrl* ctrl, const QuadGroup& g, const double* nodebuf, int m, double tol,
                              const double* T1r, double* qprev, double* y, hipStream_t st) {
    hipLaunchKernelGGL(quad_reduce_kernel, dim3(1), dim3(1024), 0, st, ctrl, g, nodebuf, m, tol, T1r, qprev, y,
                       nullptr);
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

hipError_t launch_assemble(const void* U, int64_t ldU, int64_t N, int m, const DevCtrl* ctrl, const double* ys,
                           double* x, int prec, hipStream_t st) {
    int64_t g = (N + 255) / 256;
    const dim3 grid((unsigned)(g < 8192 ? g : 8192));
    if (prec == 1)
        hipLaunchKernelGGL(assemble_kernel<float>, grid, dim3(256), 0, st, static_cast<const float*>(U), ldU, N, m,
                           ctrl, ys, x);
    else if (prec == 2)
        hipLaunchKernelGGL(assemble_kernel<bf16s>, grid, dim3(256), 0, st, static_cast<const bf16s*>(U), ldU, N, m,
                           ctrl, ys, x);
    else
        hipLaunchKernelGGL(assemble_kernel<double>, grid, dim3(256), 0, st, static_cast<const double*>(U), ldU, N, m,
                           ctrl, ys, x);
    return hipGetLastError();
}


// ------------------------------------------------------- batched launchers
// Every unit uses the common leading dimensions m (= m_max) and s (= s_max).
hipError_t launch_init_ctrl_batched(const SmallUnit* units, int nunits, hipStream_t st) {
    hipLaunchKernelGGL(init_ctrl_batched_kernel, dim3(1, nunits), dim3(64), 0, st, units);
    return hipGetLastError();
}

hipError_t launch_cond_trunc(double* X, int s, int m, DevCtrl* ctrl, const double* H, double* cnd, double cmax,
                             hipStream_t st) {
    const int blocks = (m + RC_NT / WAVE - 1) / (RC_NT / WAVE);
    if (m <= 256)
        hipLaunchKernelGGL(rinv_col_kernel<4>, dim3(blocks), dim3(RC_NT), 0, st, X, s, ctrl, m, cnd);
    else
        hipLaunchKernelGGL(rinv_col_kernel<8>, dim3(blocks), dim3(RC_NT), 0, st, X, s, ctrl, m, cnd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cond_trunc_kernel, dim3(1), dim3(64), 0, st, ctrl, X, s, H, m, cnd, cmax);
    return hipGetLastError();
}

hipError_t launch_cond_trunc_batched(const SmallUnit* units, int nunits, int s, int m, double cmax, hipStream_t st) {
    const int blocks = (m + RC_NT / WAVE - 1) / (RC_NT / WAVE);
    if (m <= 256)
        hipLaunchKernelGGL(rinv_col_batched_kernel<4>, dim3(blocks, nunits), dim3(RC_NT), 0, st, units, s, m);
    else
        hipLaunchKernelGGL(rinv_col_batched_kernel<8>, dim3(blocks, nunits), dim3(RC_NT), 0, st, units, s, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cond_trunc_batched_kernel, dim3(1, nunits), dim3(64), 0, st, units, s, m, cmax);
    return hipGetLastError();
}

hipError_t launch_qr_batched(const SmallUnit* units, int nunits, int s, int ncols_max, hipStream_t st) {
    for (int c0 = 0; c0 < ncols_max; c0 += QR_NB) {
        const dim3 g(1, nunits);
        switch (qr_rpw(s - c0)) {
            case 2: hipLaunchKernelGGL(qr_panel_batched_kernel<2>, g, dim3(QR_NT), 0, st, units, s, c0); break;
            case 4: hipLaunchKernelGGL(qr_panel_batched_kernel<4>, g, dim3(QR_NT), 0, st, units, s, c0); break;
            case 8: hipLaunchKernelGGL(qr_panel_batched_kernel<8>, g, dim3(QR_NT), 0, st, units, s, c0); break;
            default: hipLaunchKernelGGL(qr_panel_batched_kernel<16>, g, dim3(QR_NT), 0, st, units, s, c0); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int rest = ncols_max - c0 - QR_NB;
        if (rest > 0) {
            hipLaunchKernelGGL(qr_update_batched_kernel, dim3(rest, nunits), dim3(256), 0, st, units, s, c0);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_pencil_setup_batched(const SmallUnit* units, int nunits, int s, int m, int k, hipStream_t st) {
    const int n = (m + 1) * m;
    hipLaunchKernelGGL(pencil_setup_batched_kernel, dim3((n + 255) / 256, nunits), dim3(256), 0, st, units, s, m, k);
    return hipGetLastError();
}

hipError_t launch_hhat_rows_batched(const SmallUnit* units, int nunits, int m, int s, hipStream_t st) {
    if (m <= 256)
        hipLaunchKernelGGL(hhat_rows_batched_kernel<4>, dim3(1, nunits), dim3(HH_NT), 0, st, units, m, s);
    else
        hipLaunchKernelGGL(hhat_rows_batched_kernel<8>, dim3(1, nunits), dim3(HH_NT), 0, st, units, m, s);
    return hipGetLastError();
}

hipError_t launch_pencil_scalars_batched(const SmallUnit* units, int nunits, int m, int s, int is_ls, int branch_check,
                                         int k, hipStream_t st) {
    // the band U rows of the one node: (k + 3) m doubles of the unit's node scratch
    if (!is_ls && band_ok(k, m)) {
        BAND_DISPATCH(k + 1, hipLaunchKernelGGL(pencil_scalars_band_batched_kernel<KB>, dim3(1, nunits), dim3(64), 0,
                                                st, units, m, s, branch_check));
        return hipGetLastError();
    }
    if (m <= 256)
        hipLaunchKernelGGL(pencil_scalars_batched_kernel<4>, dim3(1, nunits), dim3(64), 0, st, units, m, s, is_ls,
                           branch_check);
    else
        hipLaunchKernelGGL(pencil_scalars_batched_kernel<8>, dim3(1, nunits), dim3(64), 0, st, units, m, s, is_ls,
                           branch_check);
    return hipGetLastError();
}

// slots: quadrature scratch slots (wavefronts) per unit; Ubuf holds slots x m x m per unit
hipError_t launch_quad_group_batched(const SmallUnit* units, int nunits, const QuadGroup& g, int m, int is_ls,
                                     int slots, int k, hipStream_t st) {
    // one lane per node; U rows of the group's nodes: g.total (k + 3) m doubles of the
    // unit's slots x m x m scratch
    if (!is_ls && band_ok(k, m) && (int64_t)g.total * (k + 3) <= (int64_t)slots * m) {
        const int blocks = (g.total + BAND_NT - 1) / BAND_NT;
        BAND_DISPATCH(k + 1, hipLaunchKernelGGL(quad_level_band_batched_kernel<KB>, dim3(blocks, nunits),
                                                dim3(BAND_NT), 0, st, units, g, m));
        return hipGetLastError();
    }
    const int waves = g.total < slots ? g.total : slots;
    const int blocks = (waves + 3) / 4;
    if (m <= 256)
        hipLaunchKernelGGL(quad_level_batched_kernel<4>, dim3(blocks, nunits), dim3(256), 0, st, units, g, m, is_ls);
    else
        hipLaunchKernelGGL(quad_level_batched_kernel<8>, dim3(blocks, nunits), dim3(256), 0, st, units, g, m, is_ls);
    return hipGetLastError();
}

hipError_t launch_quad_reduce_batched(const SmallUnit* units, int nunits, const QuadGroup& g, int m, double tol,
                                      hipStream_t st) {
    hipLaunchKernelGGL(quad_reduce_batched_kernel, dim3(1, nunits), dim3(1024), 0, st, units, g, m, tol);
    return hipGetLastError();
}

hipError_t launch_quad_fail_batched(const SmallUnit* units, int nunits, hipStream_t st) {
    hipLaunchKernelGGL(quad_fail_batched_kernel, dim3(1, nunits), dim3(64), 0, st, units);
    return hipGetLastError();
}

hipError_t launch_finish_coeffs_batched(const SmallUnit* units, int nunits, int m, hipStream_t st) {
    hipLaunchKernelGGL(finish_coeffs_batched_kernel, dim3(1, nunits), dim3(256), 0, st, units, m);
    return hipGetLastError();
}

hipError_t launch_assemble_batched(const SmallUnit* units, int nunits, int64_t nmax, int m, int prec,
                                   hipStream_t st) {
    int64_t g = (nmax + 255) / 256;
    const dim3 grid((unsigned)(g < 1024 ? g : 1024), nunits);
    if (prec == 1)
        hipLaunchKernelGGL(assemble_batched_kernel<float>, grid, dim3(256), 0, st, units, m);
    else if (prec == 2)
        hipLaunchKernelGGL(assemble_batched_kernel<bf16s>, grid, dim3(256), 0, st, units, m);
    else
        hipLaunchKernelGGL(assemble_batched_kernel<double>, grid, dim3(256), 0, st, units, m);
    return hipGetLastError();
}

}  // namespace skfab
