// k-truncated Arnoldi recurrence with on-the-fly sparse-sign sketches, one fused
// kernel per step (Algorithm 2 of arXiv 2208.11447, basis part; truncation rule of
// Section 2.2).
//
// Step j (0-based) forms the next unnormalised basis vector from the previous
// step's data and multiplies it by A in the same pass:
//
//   u_j = A v_{j-1} - sum_{i in window} h_{i,j-1} v_i        (j >= 1),  u_0 = b
//       = W_{j-1} / eta_{j-1} - sum_i (h_{i,j-1} / eta_i) U_i
//   W_j = A u_j,   S u_j,  S W_j,  and the dot products needed for step j+1's
//   coefficients: ||u_j||^2, <u_j, W_j>, ||W_j||^2, <U_l, W_j>, <u_j, U_l>
//   for the k-1 previous vectors l of the window.
//
// The stored basis is U (v_j = u_j / eta_j with eta_j = ||u_j||); the sketches are
// rescaled by 1/eta_j when the per-block partial sums are reduced.  The truncated
// modified Gram-Schmidt coefficients are obtained from the dot products and the
// Gram entries of the window (h_i = <v_i, w> - sum_{l<i} h_l <v_i, v_l>), which
// equals sequential MGS for the stored vectors.  Entries of u_j needed by the
// SpMV at neighbouring rows are recomputed from W_{j-1} and the window with the
// same fused multiply-add sequence, so the SpMV input equals the stored U_j bit
// for bit.
//
// Determinism: every sum has a fixed order (per-wave LDS bins, fixed block trees,
// partial arrays reduced in block order).
#include "common.hpp"
#include "device_state.hpp"

namespace skfab {

// ----------------------------------------------------------- coefficients
// Turns the reduced dot products of step p into eta_p, h_{.,p}, the Gram
// entries of v_p and the coefficients of u_{p+1}.  Runs on one thread.
// Returns false on breakdown (m_used set to p, or 0 for b = 0).
template <int KW>
__device__ bool step_coefficients(const double* red, int p, int k, int m, bool writer,
                                  const StepArgs& a, double* coef) {
    const double uu = red[0], uw = red[1], ww = red[2];
    const double eta_p = sqrt(uu);
    bool ok;
    if (p == 0) {
        ok = eta_p > 0.0;
    } else {
        ok = eta_p > BREAKDOWN_TOL * a.wnorm[p - 1];
    }
    if (!ok) {
        if (writer) {
            a.ctrl->m_used = p;
            a.ctrl->stop = 1;
            if (p >= 1) a.H[p + (int64_t)(m + 1) * (p - 1)] = eta_p;
        }
        return false;
    }
    const double wn = sqrt(ww) / eta_p;
    const int nwp = min(k, p + 1);  // window(p) = {p-nwp+1 .. p}
    double d[KW], gp[KW], h[KW];
#pragma unroll
    for (int o = 0; o < KW; ++o) { d[o] = 0.0; gp[o] = 0.0; h[o] = 0.0; }
    d[0] = uw / (eta_p * eta_p);
#pragma unroll
    for (int o = 1; o < KW; ++o) {
        if (o < nwp) {
            const double eo = a.eta[p - o];
            d[o] = red[3 + (o - 1)] / (eo * eta_p);
            gp[o] = red[3 + (KW - 1) + (o - 1)] / (eta_p * eo);
        }
    }
    // modified Gram-Schmidt order: ascending i = p - o, i.e. descending o
#pragma unroll
    for (int o = KW - 1; o >= 0; --o) {
        if (o < nwp) {
            const int i = p - o;
            double hi = d[o];
#pragma unroll
            for (int o2 = KW - 1; o2 > o; --o2) {
                if (o2 < nwp) {
                    const int l = p - o2;
                    const double gil = (o == 0) ? gp[o2] : a.gram[(int64_t)i * KMAX + (i - l - 1)];
                    hi -= h[o2] * gil;
                }
            }
            h[o] = hi;
        }
    }
    if (coef) {
        coef[0] = 1.0 / eta_p;
#pragma unroll
        for (int o = 0; o < KW; ++o) {
            const double eo = (o == 0) ? eta_p : ((o < nwp) ? a.eta[p - o] : 1.0);
            coef[1 + o] = (o < nwp) ? -h[o] / eo : 0.0;
        }
    }
    if (writer) {
        a.eta[p] = eta_p;
        a.wnorm[p] = wn;
        const int64_t ldh = m + 1;
        for (int o = 0; o < nwp; ++o) a.H[(p - o) + ldh * p] = h[o];
        if (p >= 1) a.H[p + ldh * (p - 1)] = eta_p;
        for (int o = 1; o < nwp; ++o) a.gram[(int64_t)p * KMAX + (o - 1)] = gp[o];
    }
    return true;
}

// Reduce the [NSC][G] partial scalars of the previous step (fixed order).
template <int KW, int BLOCK>
__device__ void reduce_prev_scalars(const double* scal_prev, int G, double* red, double* scratch) {
    constexpr int NSC = 2 * KW + 1;
    for (int sc = 0; sc < NSC; ++sc) {
        double v = 0.0;
        for (int g = threadIdx.x; g < G; g += BLOCK) v += scal_prev[(int64_t)sc * G + g];
        v = block_sum(v, scratch);
        if (threadIdx.x == 0) red[sc] = v;
    }
    __syncthreads();
}

// ------------------------------------------------------------- step kernel
template <int KW, int ZETA, int BLOCK>
__global__ __launch_bounds__(BLOCK) void arnoldi_step_kernel(StepArgs a) {
    extern __shared__ double bins[];  // [BLOCK/64][2s]
    __shared__ double red[NSC_MAX];
    __shared__ double coef[KMAX + 1];
    __shared__ double scratch[BLOCK / WAVE];
    __shared__ int s_ok;

    if (a.ctrl->stop) return;
    constexpr int NSC = 2 * KW + 1;
    const int j = a.j, k = a.k, s = a.s, G = a.G;
    const int tid = threadIdx.x;

    if (j > 0) {
        reduce_prev_scalars<KW, BLOCK>(a.scal_prev, G, red, scratch);
        if (tid == 0) s_ok = step_coefficients<KW>(red, j - 1, k, a.m, blockIdx.x == 0, a, coef) ? 1 : 0;
        __syncthreads();
        if (!s_ok) return;
    } else if (tid == 0) {
        coef[0] = 1.0;
        for (int o = 0; o < KW; ++o) coef[1 + o] = 0.0;
    }
    // zero the per-wave sketch bins
    const int nwaves = BLOCK / WAVE;
    for (int i = tid; i < nwaves * 2 * s; i += BLOCK) bins[i] = 0.0;
    __syncthreads();

    const int nwin = (j == 0) ? 0 : min(k, j);   // vectors j-1 .. j-nwin form u_j
    const int ndot = min(k - 1, j);              // vectors j-1 .. j-ndot enter the dots
    const double alpha = coef[0];
    double cf[KW];
#pragma unroll
    for (int o = 0; o < KW; ++o) cf[o] = coef[1 + o];

    const double* __restrict__ base = (j == 0) ? a.b : a.Wprev;
    const double* Uo[KW];
#pragma unroll
    for (int o = 0; o < KW; ++o) Uo[o] = a.U + (int64_t)((o < nwin) ? (j - 1 - o) : 0) * a.ldU;
    double* __restrict__ Uj = a.U + (int64_t)(a.extend ? 0 : j) * a.ldU;
    double* binV = bins + (tid / WAVE) * 2 * s;
    double* binAV = binV + s;

    double acc_uu = 0.0, acc_uw = 0.0, acc_ww = 0.0;
    double acc_lw[KW], acc_ul[KW];
#pragma unroll
    for (int o = 0; o < KW; ++o) { acc_lw[o] = 0.0; acc_ul[o] = 0.0; }

    const int chunk = xcd_chunk(blockIdx.x, G);
    const int64_t r_begin = (int64_t)chunk * a.rows_per_chunk;
    const int64_t r_end = min(a.N, r_begin + a.rows_per_chunk);

    for (int64_t r0 = r_begin; r0 < r_end; r0 += BLOCK) {
        const int64_t r = r0 + tid;
        if (r < r_end) {
            double uo[KW];
            double u = alpha * base[r];
#pragma unroll
            for (int o = 0; o < KW; ++o) {
                uo[o] = (o < nwin) ? Uo[o][r] : 0.0;
                if (o < nwin) u = fma(cf[o], uo[o], u);
            }
            if (a.extend) {
                acc_uu = fma(u, u, acc_uu);
                int rows[ZETA];
                double sg[ZETA];
                sketch_column<ZETA>(a.seed, (uint64_t)r, s, rows, sg);
#pragma unroll
                for (int q = 0; q < ZETA; ++q) lds_add(binV + rows[q], sg[q] * u);
                continue;
            }
            Uj[r] = u;
            const int e0 = a.rowptr[r], e1 = a.rowptr[r + 1];
            double w = 0.0;
            for (int e = e0; e < e1; ++e) {
                const int c = a.col[e];
                double x = alpha * base[c];
#pragma unroll
                for (int o = 0; o < KW; ++o)
                    if (o < nwin) x = fma(cf[o], Uo[o][c], x);
                w = fma(a.val[e], x, w);
            }
            a.Wcur[r] = w;
            acc_uu = fma(u, u, acc_uu);
            acc_uw = fma(u, w, acc_uw);
            acc_ww = fma(w, w, acc_ww);
#pragma unroll
            for (int o = 0; o < KW - 1; ++o) {
                if (o < ndot) {
                    acc_lw[o] = fma(uo[o], w, acc_lw[o]);
                    acc_ul[o] = fma(u, uo[o], acc_ul[o]);
                }
            }
            int rows[ZETA];
            double sg[ZETA];
            sketch_column<ZETA>(a.seed, (uint64_t)r, s, rows, sg);
#pragma unroll
            for (int q = 0; q < ZETA; ++q) {
                lds_add(binV + rows[q], sg[q] * u);
                lds_add(binAV + rows[q], sg[q] * w);
            }
        }
    }

    // partial scalars of this block
    double vals[NSC];
    vals[0] = acc_uu; vals[1] = acc_uw; vals[2] = acc_ww;
#pragma unroll
    for (int o = 0; o < KW - 1; ++o) { vals[3 + o] = acc_lw[o]; vals[3 + (KW - 1) + o] = acc_ul[o]; }
#pragma unroll
    for (int sc = 0; sc < NSC; ++sc) {
        const double t = block_sum(vals[sc], scratch);
        if (tid == 0) a.scal_cur[(int64_t)sc * G + blockIdx.x] = t;
    }
    __syncthreads();
    double* dst = a.skpart + (int64_t)blockIdx.x * 2 * s;
    for (int i = tid; i < 2 * s; i += BLOCK) {
        double t = 0.0;
        for (int wv = 0; wv < nwaves; ++wv) t += bins[wv * 2 * s + i];
        dst[i] = t;
    }
}

// Coefficients of the last step (eta_{m-1}, h_{., m-1}) and breakdown check.
template <int KW>
__global__ __launch_bounds__(256) void arnoldi_finalize_kernel(StepArgs a) {
    __shared__ double red[NSC_MAX];
    __shared__ double scratch[256 / WAVE];
    if (a.ctrl->stop) return;
    reduce_prev_scalars<KW, 256>(a.scal_prev, a.G, red, scratch);
    if (threadIdx.x == 0) step_coefficients<KW>(red, a.j - 1, a.k, a.m, true, a, nullptr);
}

// SV[:, j] = inv_sqrt_zeta / eta_j * sum_g part_j[g][0:s], SAV likewise from [s:2s]
// for j < m_used; column m_used of SV receives S u_{m_used} unnormalised (the
// extension vector of the Arnoldi relation).  One block per column j = 0..m.
__global__ __launch_bounds__(256) void sketch_reduce_kernel(const double* skpart, int G, int s, int m,
                                                           double inv_sqrt_zeta, const DevCtrl* ctrl,
                                                           const double* eta, double* SV, double* SAV,
                                                           double* colnorm2) {
    __shared__ double scratch[4];
    const int j = blockIdx.x;
    const int m_used = ctrl->m_used;
    const bool valid = j <= m_used && m_used > 0;
    const double scale = (j < m_used) ? inv_sqrt_zeta / eta[j] : inv_sqrt_zeta;
    const double* src = skpart + (int64_t)j * G * 2 * s;
    double nrm = 0.0;
    for (int i = threadIdx.x; i < 2 * s; i += 256) {
        double t = 0.0;
        if (valid && (i < s || j < m_used))
            for (int g = 0; g < G; ++g) t += src[(int64_t)g * 2 * s + i];
        t *= scale;
        if (i < s) {
            SV[(int64_t)j * s + i] = t;
            nrm = fma(t, t, nrm);
        } else if (j < m) {
            SAV[(int64_t)j * s + (i - s)] = (j < m_used) ? t : 0.0;
        }
    }
    nrm = block_sum(nrm, scratch);
    if (threadIdx.x == 0 && j < m) colnorm2[j] = (j < m_used) ? nrm : 1.0;
}

// eta_m and h_{m+1,m} from the extension step's partial ||u_m||^2.
__global__ __launch_bounds__(256) void extension_finalize_kernel(const double* scal, int G, int m, DevCtrl* ctrl,
                                                                 double* eta, double* H) {
    __shared__ double scratch[4];
    if (ctrl->stop) return;
    double v = 0.0;
    for (int g = threadIdx.x; g < G; g += 256) v += scal[g];
    v = block_sum(v, scratch);
    if (threadIdx.x == 0) {
        eta[m] = sqrt(v);
        H[m + (int64_t)(m + 1) * (m - 1)] = sqrt(v);
    }
}

// relres = ||SAV - [SV, S u] Hbar1||_F / ||SAV||_F over the first m_used columns,
// Hbar1 = [H; e_mu^T] (Arnoldi relation in the sketched space).  One block.
__global__ __launch_bounds__(256) void arnoldi_check_kernel(const double* SV, const double* SAV, const double* H,
                                                           int s, int m, int k, DevCtrl* ctrl) {
    __shared__ double scratch[4];
    const int mu = ctrl->m_used;
    double num = 0.0, den = 0.0;
    for (int idx = threadIdx.x; idx < s * mu; idx += 256) {
        const int jj = idx / s, i = idx - jj * s;
        double t = SAV[(int64_t)jj * s + i];
        den = fma(t, t, den);
        for (int l = max(0, jj - k + 1); l <= jj + 1; ++l) {
            const double hb = (l == jj + 1) ? ((jj == mu - 1) ? 1.0 : H[(jj + 1) + (int64_t)(m + 1) * jj])
                                            : H[l + (int64_t)(m + 1) * jj];
            t = fma(-SV[(int64_t)l * s + i], hb, t);
        }
        num = fma(t, t, num);
    }
    num = block_sum(num, scratch);
    den = block_sum(den, scratch);
    if (threadIdx.x == 0) ctrl->relres = (den > 0.0) ? sqrt(num / den) : 0.0;
}

// V[:, j] = U[:, j] / eta_j (zero beyond m_used); test hook only.
__global__ void normalize_basis_kernel(const double* U, int64_t ldU, int64_t N, int m,
                                       const DevCtrl* ctrl, const double* eta, double* V) {
    const int j = blockIdx.y;
    const int m_used = ctrl->m_used;
    const double sc = (j < m_used) ? 1.0 / eta[j] : 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x)
        V[(int64_t)j * N + r] = (j < m_used) ? U[(int64_t)j * ldU + r] * sc : 0.0;
}

// ---------------------------------------------------------------- launchers
template <int KW, int ZETA>
static hipError_t launch_step_t(const StepArgs& a, int block, hipStream_t st) {
    const size_t lds = (size_t)(block / WAVE) * 2 * a.s * sizeof(double);
    if (block == 1024) {
        hipLaunchKernelGGL((arnoldi_step_kernel<KW, ZETA, 1024>), dim3(a.G), dim3(1024), lds, st, a);
    } else if (block == 512) {
        hipLaunchKernelGGL((arnoldi_step_kernel<KW, ZETA, 512>), dim3(a.G), dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL((arnoldi_step_kernel<KW, ZETA, 256>), dim3(a.G), dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

template <int ZETA>
static hipError_t launch_step_z(const StepArgs& a, int block, hipStream_t st) {
    switch (a.k) {
        case 1: return launch_step_t<1, ZETA>(a, block, st);
        case 2: return launch_step_t<2, ZETA>(a, block, st);
        case 3: return launch_step_t<3, ZETA>(a, block, st);
        case 4: return launch_step_t<4, ZETA>(a, block, st);
        default: return launch_step_t<8, ZETA>(a, block, st);
    }
}

hipError_t launch_arnoldi_step(const StepArgs& a, int zeta, int block, hipStream_t st) {
    switch (zeta) {
        case 2: return launch_step_z<2>(a, block, st);
        case 4: return launch_step_z<4>(a, block, st);
        case 16: return launch_step_z<16>(a, block, st);
        default: return launch_step_z<8>(a, block, st);
    }
}

hipError_t launch_arnoldi_finalize(const StepArgs& a, hipStream_t st) {
    switch (a.k) {
        case 1: hipLaunchKernelGGL((arnoldi_finalize_kernel<1>), dim3(1), dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((arnoldi_finalize_kernel<2>), dim3(1), dim3(256), 0, st, a); break;
        case 3: hipLaunchKernelGGL((arnoldi_finalize_kernel<3>), dim3(1), dim3(256), 0, st, a); break;
        case 4: hipLaunchKernelGGL((arnoldi_finalize_kernel<4>), dim3(1), dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((arnoldi_finalize_kernel<8>), dim3(1), dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_sketch_reduce(const double* skpart, int G, int s, int m, int zeta, const DevCtrl* ctrl,
                                const double* eta, double* SV, double* SAV, double* colnorm2, hipStream_t st) {
    hipLaunchKernelGGL(sketch_reduce_kernel, dim3(m + 1), dim3(256), 0, st, skpart, G, s, m,
                       1.0 / sqrt((double)zeta), ctrl, eta, SV, SAV, colnorm2);
    return hipGetLastError();
}

hipError_t launch_extension_finalize(const double* scal, int G, int m, DevCtrl* ctrl, double* eta, double* H,
                                     hipStream_t st) {
    hipLaunchKernelGGL(extension_finalize_kernel, dim3(1), dim3(256), 0, st, scal, G, m, ctrl, eta, H);
    return hipGetLastError();
}

hipError_t launch_arnoldi_check(const double* SV, const double* SAV, const double* H, int s, int m, int k,
                                DevCtrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(arnoldi_check_kernel, dim3(1), dim3(256), 0, st, SV, SAV, H, s, m, k, ctrl);
    return hipGetLastError();
}

hipError_t launch_normalize_basis(const double* U, int64_t ldU, int64_t N, int m, const DevCtrl* ctrl,
                                  const double* eta, double* V, hipStream_t st) {
    int64_t gx64 = (N + 255) / 256;
    int gx = (int)(gx64 < 1024 ? gx64 : 1024);
    hipLaunchKernelGGL(normalize_basis_kernel, dim3(gx, m), dim3(256), 0, st, U, ldU, N, m, ctrl, eta, V);
    return hipGetLastError();
}

}  // namespace skfab
