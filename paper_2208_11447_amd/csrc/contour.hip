// Sketched GMRES for f(z) = exp(-tau z) by a contour integral (Section 1, Sections
// 4.1 and 5.2).  Cauchy's formula with the paper's measure dmu(t) = dt / (2 pi i):
//
//     exp(-tau A) b = 1/(2 pi i) int_Gamma exp(tau t) (t I + A)^-1 b dt,
//
// Gamma around the negated spectrum.  The sketched GMRES approximant (eq. sGMRES)
// replaces (t I + A)^-1 b by V_m y(t), y(t) = (t SV_m + SAV_m)^+ S b, which the
// pencil form of the small problem gives as the least-squares solution of
// min || beta R_00 e_1 - (t R + K0) y || (R = R_e[:, :m], K0 = R_e Hbar) -- here at
// complex t.  Algorithm 2 places Gamma around the sketched Ritz values (the
// eigenvalues of H_hat, negated); Section 5.2 uses the parabola
// t(theta) = a + i theta - c theta^2.
//
//   contour_setup_kernel: eigenvalues of H_hat (Francis QR with small bulges on the
//     Hessenberg matrix, one block, the matrix in LDS) and the parabola;
//   contour_level_kernel: the trapezoidal rule's nodes, one wavefront per node
//     (complex Givens least squares), each node's contribution
//     Im(W_k y(t_k)) to the rule, summed and tested by quad_reduce_kernel.
//
// Parabola (in units u = tau t, mu_j = -tau theta_j, X = max Re mu_j): only the
// mu_j with Re mu_j >= X - CT_L matter; apex alpha = X + 1; curvature kappa =
// min(CT_KAPPA_MAX, min_j (alpha - Re mu_j) / (2 (Im mu_j)^2)) over the relevant
// complex mu_j (each one halfway between the axis and the parabola); truncation
// |v| <= v_max with alpha - kappa v_max^2 = X - CT_L.  In t: a = alpha / tau,
// c = kappa tau, theta_max = v_max / tau.
//
// Rule: trapezoidal in theta, step h = theta_max / K, nodes theta_k = k h,
// k = 0..K.  A, b and S are real, so the integrand at -theta is minus the
// conjugate of the one at theta and the rule folds to
// (h / pi) sum_k c_k Im(exp(tau t_k) t'_k y(t_k)), c_0 = 1/2, c_k = 1 otherwise,
// t'(theta) = i - 2 c theta.  K = 32, 64, ..., CT_KMAX under the relative test of
// Section 4.1 (in the whitened norm ||R q||).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "device_state.hpp"

namespace skfab {

__device__ __forceinline__ double wave_min(double v) { return -wave_max(-v); }

constexpr double CT_L = 45.0;
constexpr double CT_KAPPA_MAX = 0.25;

// ------------------------------------------------ Hessenberg eigenvalues
// H_hat = H_m + r e_m^T is upper Hessenberg.  Its eigenvalues are found by the
// Francis QR iteration with small bulges (eigenvalues only: each step acts on the
// active block), one block, the matrix in LDS in FP64: row i from column
// max(i - 1, 0) (CT_HQR_CAP doubles for n <= CT_NMAX).  A sweep chases up to
// HQ_NB bulges of two shifts each, HQ_DS rows apart; the shifts are eigenvalues
// of the trailing 2 HQ_NB x 2 HQ_NB block.  A bulge leaves at most three entries
// below the subdiagonal, at (k+2, k), (k+3, k+1) and (k+3, k) after its step at
// row k: those two below the diagonal live in slot row % HQ_P of one array after
// the matrix, those three below in slot row % HQ_P of another (the entries of a
// chain span fewer than HQ_P rows), and all are zero between sweeps.
// Balancing by powers of two (a diagonal similarity, exact) comes first: the last
// column of H_hat can be orders of magnitude larger than the band.
constexpr int CT_HQR_CAP = CT_NMAX + (CT_NMAX - 1) * (CT_NMAX + 2) / 2;
constexpr int HQ_P = 32;     // slot period of the entries below the subdiagonal
constexpr int HQ_NB = 4;     // bulges of a sweep at most
constexpr int HQ_DS = 4;     // rows between consecutive bulges of a chain
constexpr int HQ_NS = 2 * HQ_NB;
constexpr int HQ_NMIN = 24;  // smaller active blocks take one bulge (shifts of the trailing 2 x 2)
static_assert(HQ_NB * HQ_DS + 4 <= HQ_P, "the sub-subdiagonal entries of a chain map to distinct slots");
constexpr int HQ_LDS = CT_HQR_CAP + 2 * HQ_P;  // the matrix and the two slot arrays
// Threads of the eigenvalue kernel (NT): every wavefront takes the same (uniform)
// decisions from the same LDS values; the row and column updates of a chain step
// (at most HQ_NB (n + 1) entries each) are spread over all of them.  1024 threads
// for n > HQ_NSMALL; 256 below, where every sweep takes one bulge (measured: the
// shift eigenvalues and the chain's fill and drain cost more than they save on
// such short blocks, and fewer wavefronts make the barriers cheaper).
constexpr int HQ_NSMALL = 63;
static_assert(HQ_NB * (HQ_NSMALL + 1) <= 256 && HQ_NB * (CT_NMAX + 1) <= 1024, "one entry per thread and phase");

__device__ __forceinline__ int hq_off(int i, int n) { return (i == 0) ? 0 : n + (i - 1) * (2 * n - i + 2) / 2; }

// address of entry (i, j), j >= i - 3, by arithmetic alone (a load never waits on
// a branch, so the loads of an update are in flight together)
__device__ __forceinline__ double* hq_at(double* Hs, int i, int j, int n) {
    const int d = i - j;
    const int band = hq_off(i, n) + j - (i > 0 ? i - 1 : 0);
    return Hs + ((d <= 1) ? band : CT_HQR_CAP + ((d == 2) ? 0 : HQ_P) + (i & (HQ_P - 1)));
}

__device__ __forceinline__ void hq_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Balancing by wavefront 0 alone (its LDS accesses ordered by wavefront fences),
// the other wavefronts waiting at one barrier at the end.
__device__ void hq_balance(double* Hs, int n) {
    if (threadIdx.x < WAVE) {
        const int lane = threadIdx.x;
        for (int sweep = 0; sweep < 40; ++sweep) {
            bool done = true;
            for (int i = 0; i < n; ++i) {
                double c = 0.0, r = 0.0;
                for (int q = lane; q < min(i + 2, n); q += WAVE)
                    if (q != i) c += fabs(*hq_at(Hs, q, i, n));
                for (int q = (i > 0 ? i - 1 : 0) + lane; q < n; q += WAVE)
                    if (q != i) r += fabs(*hq_at(Hs, i, q, n));
                c = wave_sum(c);
                r = wave_sum(r);
                if (c == 0.0 || r == 0.0) continue;
                double gg = 0.5 * r, f = 1.0;
                const double s = c + r;
                for (int t = 0; t < 2100 && c < gg; ++t) { f *= 2.0; c *= 4.0; }
                gg = 2.0 * r;
                for (int t = 0; t < 2100 && c >= gg; ++t) { f *= 0.5; c *= 0.25; }
                if ((c + r) / f < 0.95 * s) {
                    done = false;
                    const double fi = 1.0 / f;
                    hq_wave_sync();  // every lane has its sums before any scaling
                    for (int q = (i > 0 ? i - 1 : 0) + lane; q < n; q += WAVE) *hq_at(Hs, i, q, n) *= fi;
                    hq_wave_sync();
                    for (int q = lane; q < min(i + 2, n); q += WAVE) *hq_at(Hs, q, i, n) *= f;
                    hq_wave_sync();
                }
            }
            if (done) break;
        }
    }
    __syncthreads();
}

// Householder reflector P = I - tau v v^T with P (x, y, z)^T = (alpha, 0, 0)^T, into
// out = (v0, v1, v2, tau, alpha); tau = 0 (no reflection) when x = y = z = 0.
__device__ __forceinline__ void hq_reflector(double x, double y, double z, double* out) {
    const double nx = sqrt(x * x + y * y + z * z);
    if (nx == 0.0) {
        out[0] = out[1] = out[2] = out[3] = out[4] = 0.0;
        return;
    }
    const double alpha = (x >= 0.0) ? -nx : nx;
    const double v0 = x - alpha;
    out[0] = v0;
    out[1] = y;
    out[2] = z;
    out[3] = 2.0 / (v0 * v0 + y * y + z * z);
    out[4] = alpha;
}

// Eigenvalues of the ns x ns upper Hessenberg matrix W (row-major, ld HQ_NS, in
// LDS) by the double-shift iteration, on the 64 lanes of one wavefront (uniform
// decisions; a reflector's row and column updates one entry per lane, ordered by
// wavefront fences); into er, ei.  Returns false without convergence in 30 ns steps.

__device__ bool hq_small_eigs(double* W, int ns, double* er, double* ei) {
    const int lane = threadIdx.x & 63;
    auto w = [&](int i, int j) -> double& { return W[i * HQ_NS + j]; };
    double nrm = 0.0;
    for (int e = lane; e < ns * ns; e += WAVE) nrm += fabs(w(e / ns, e % ns));
    nrm = wave_sum(nrm);
    const double eps = 2.3e-16;
    int hi = ns - 1, its = 0, total = 0;
    while (hi >= 0) {
        int l = 0;
        for (int c = hi; c > 0; --c) {
            double sd = fabs(w(c - 1, c - 1)) + fabs(w(c, c));
            if (sd == 0.0) sd = nrm;
            if (fabs(w(c, c - 1)) <= eps * sd) { l = c; break; }
        }
        hq_wave_sync();
        if (l > 0 && lane == 0) w(l, l - 1) = 0.0;
        if (l == hi) {
            if (lane == 0) { er[hi] = w(hi, hi); ei[hi] = 0.0; }
            hq_wave_sync();
            --hi;
            its = 0;
            continue;
        }
        if (l == hi - 1) {
            const double p = w(hi - 1, hi - 1), q = w(hi - 1, hi), r = w(hi, hi - 1), s = w(hi, hi);
            const double hm = 0.5 * (p - s), disc = hm * hm + q * r;
            if (lane == 0) {
                if (disc >= 0.0) {
                    const double z = hm + copysign(sqrt(disc), hm);
                    er[hi - 1] = s + z;
                    er[hi] = (z != 0.0) ? s - q * r / z : s + z;
                    ei[hi - 1] = ei[hi] = 0.0;
                } else {
                    const double im = sqrt(-disc);
                    er[hi - 1] = er[hi] = s + hm;
                    ei[hi - 1] = im;
                    ei[hi] = -im;
                }
            }
            hq_wave_sync();
            hi -= 2;
            its = 0;
            continue;
        }
        if (total >= 30 * ns) return false;
        double sh, dt;
        if (its == 10 || its == 20) {
            const double x = fabs(w(hi, hi - 1)) + fabs(w(hi - 1, hi - 2));
            sh = 1.5 * x;
            dt = x * x;
        } else {
            const double p = w(hi - 1, hi - 1), q = w(hi - 1, hi), r = w(hi, hi - 1), s = w(hi, hi);
            sh = p + s;
            dt = p * s - q * r;
        }
        ++its;
        ++total;
        const double h00 = w(l, l), h01 = w(l, l + 1), h10 = w(l + 1, l), h11 = w(l + 1, l + 1);
        double x = h00 * h00 + h01 * h10 - sh * h00 + dt, y = h10 * (h00 + h11 - sh), z = h10 * w(l + 2, l + 1);
        hq_wave_sync();
        for (int k = l; k <= hi - 1; ++k) {
            const bool three = k <= hi - 2;
            if (k > l) {
                x = w(k, k - 1);
                y = w(k + 1, k - 1);
                z = three ? w(k + 2, k - 1) : 0.0;
            }
            double rf[5];
            hq_reflector(x, y, three ? z : 0.0, rf);
            const double v0 = rf[0], v1 = rf[1], v2 = rf[2], tau = rf[3];
            hq_wave_sync();  // every lane has read x, y, z
            if (tau == 0.0) continue;
            {
                const int j = max(l, k - 1) + lane;
                if (j <= hi) {
                    if (j == k - 1) {
                        w(k, j) = rf[4];
                        w(k + 1, j) = 0.0;
                        if (three) w(k + 2, j) = 0.0;
                    } else {
                        const double r0 = w(k, j), r1 = w(k + 1, j), r2 = three ? w(k + 2, j) : 0.0;
                        const double d = tau * (v0 * r0 + v1 * r1 + v2 * r2);
                        w(k, j) = r0 - d * v0;
                        w(k + 1, j) = r1 - d * v1;
                        if (three) w(k + 2, j) = r2 - d * v2;
                    }
                }
            }
            hq_wave_sync();
            {
                const int i = l + lane;
                if (i <= min(k + 3, hi)) {
                    const double c0 = w(i, k), c1 = w(i, k + 1), c2 = three ? w(i, k + 2) : 0.0;
                    const double d = tau * (v0 * c0 + v1 * c1 + v2 * c2);
                    w(i, k) = c0 - d * v0;
                    w(i, k + 1) = c1 - d * v1;
                    if (three) w(i, k + 2) = c2 - d * v2;
                }
            }
            hq_wave_sync();
        }
    }
    return true;
}

// Eigenvalues of the n x n Hessenberg matrix in Hs into wr, wi; every control
// decision uniform.  Returns false when the iteration has not converged within
// 30 n sweeps.
template <int NT>
__device__ bool hqr_eigs(double* Hs, int n, double* __restrict__ wr, double* __restrict__ wi) {
    __shared__ double W[HQ_NS * HQ_NS];      // trailing block for the shifts
    __shared__ double ser[HQ_NS], sei[HQ_NS];
    __shared__ double shs[HQ_NB], shd[HQ_NB];  // shift pairs: sum and product
    __shared__ int s_nb;
    __shared__ double rfl[HQ_NB][5];          // reflector of each bulge in a chain step
    const int lane = threadIdx.x & 63;
    const int tid = threadIdx.x;
    auto g = [&](int i, int j) -> double { return *hq_at(Hs, i, j, n); };
    double nrm = 0.0;  // size of the matrix for the deflation test of zero diagonals
    for (int i = lane; i < n; i += WAVE)
        for (int j = (i > 0 ? i - 1 : 0); j < n; ++j) nrm += fabs(g(i, j));
    nrm = wave_sum(nrm);
    const double eps = 2.3e-16;
    int hi = n - 1, its = 0, total = 0;
    while (hi >= 0) {
        // start l of the unreduced block that ends at hi: the largest l in 1..hi with a
        // negligible H[l][l-1] (0 if none), 64 candidates per pass
        int l = 0;
        for (int top = hi; top > 0; top -= WAVE) {
            const int c = top - lane;
            bool small = false;
            if (c > 0) {
                double sd = fabs(g(c - 1, c - 1)) + fabs(g(c, c));
                if (sd == 0.0) sd = nrm;
                small = fabs(g(c, c - 1)) <= eps * sd;
            }
            const unsigned long long hit = __ballot(small);
            if (hit) {
                l = top - (__ffsll((long long)hit) - 1);
                break;
            }
        }
        __syncthreads();
        if (l > 0 && tid == 0) *hq_at(Hs, l, l - 1, n) = 0.0;
        __syncthreads();
        if (l == hi) {
            if (tid == 0) { wr[hi] = g(hi, hi); wi[hi] = 0.0; }
            --hi;
            its = 0;
            continue;
        }
        if (l == hi - 1) {
            // 2 x 2 block [[p, q], [r, s]]
            const double p = g(hi - 1, hi - 1), q = g(hi - 1, hi), r = g(hi, hi - 1), s = g(hi, hi);
            const double hm = 0.5 * (p - s), disc = hm * hm + q * r;
            if (tid == 0) {
                if (disc >= 0.0) {
                    const double z = hm + copysign(sqrt(disc), hm);
                    wr[hi - 1] = s + z;
                    wr[hi] = (z != 0.0) ? s - q * r / z : s + z;
                    wi[hi - 1] = 0.0;
                    wi[hi] = 0.0;
                } else {
                    const double im = sqrt(-disc);
                    wr[hi - 1] = s + hm;
                    wr[hi] = s + hm;
                    wi[hi - 1] = im;
                    wi[hi] = -im;
                }
            }
            hi -= 2;
            its = 0;
            continue;
        }
        if (total >= 30 * n) return false;
        ++its;
        ++total;
        // the sweep's shifts: eigenvalues of the trailing HQ_NS x HQ_NS block, paired
        // (conjugate pairs, then real ones in ascending order); one pair from the
        // trailing 2 x 2 block for small active blocks, or ad hoc after 10 and 20
        // sweeps without deflation
        const bool multi = NT >= 1024 && hi - l + 1 >= HQ_NMIN && its != 10 && its != 20;
        bool small_ok = false;
        if (multi && tid < WAVE) {  // wavefront 0: the trailing block's eigenvalues
            const int b0 = hi - HQ_NS + 1;
            for (int e = lane; e < HQ_NS * HQ_NS; e += WAVE) {
                const int i = e / HQ_NS, j = e % HQ_NS;
                W[e] = (i - j <= 1) ? g(b0 + i, b0 + j) : 0.0;
            }
            hq_wave_sync();
            small_ok = hq_small_eigs(W, HQ_NS, ser, sei);
        }
        if (tid == 0) {
            int nb = 0;
            if (multi) {
                if (small_ok) {
                    for (int i = 0; i < HQ_NS && nb < HQ_NB; ++i)
                        if (sei[i] > 0.0) {
                            shs[nb] = 2.0 * ser[i];
                            shd[nb] = ser[i] * ser[i] + sei[i] * sei[i];
                            ++nb;
                        }
                    double rr[HQ_NS];
                    int nr = 0;
                    for (int i = 0; i < HQ_NS; ++i)
                        if (sei[i] == 0.0) {
                            double v = ser[i];
                            int q = nr++;
                            for (; q > 0 && rr[q - 1] > v; --q) rr[q] = rr[q - 1];
                            rr[q] = v;
                        }
                    for (int i = 0; i + 1 < nr && nb < HQ_NB; i += 2) {
                        shs[nb] = rr[i] + rr[i + 1];
                        shd[nb] = rr[i] * rr[i + 1];
                        ++nb;
                    }
                }
            }
            if (nb == 0) {
                if (its == 10 || its == 20) {
                    const double x = fabs(g(hi, hi - 1)) + fabs(g(hi - 1, hi - 2));
                    shs[0] = 1.5 * x;
                    shd[0] = x * x;
                } else {
                    const double p = g(hi - 1, hi - 1), q = g(hi - 1, hi), r = g(hi, hi - 1), s = g(hi, hi);
                    shs[0] = p + s;
                    shd[0] = p * s - q * r;
                }
                nb = 1;
            }
            s_nb = nb;
        }
        __syncthreads();
        const int nb = s_nb;
        if (nb == 1) {
            // one bulge: every thread forms the reflector itself (no record in LDS)
            const double sh = shs[0], dt = shd[0];
            const double h00 = g(l, l), h01 = g(l, l + 1), h10 = g(l + 1, l), h11 = g(l + 1, l + 1);
            double x = h00 * h00 + h01 * h10 - sh * h00 + dt;
            double y = h10 * (h00 + h11 - sh);
            double z = h10 * g(l + 2, l + 1);
            for (int k = l; k <= hi - 1; ++k) {
                const bool three = k <= hi - 2;
                if (k > l) {
                    x = g(k, k - 1);
                    y = g(k + 1, k - 1);
                    z = three ? g(k + 2, k - 1) : 0.0;
                }
                const double nx = sqrt(x * x + y * y + z * z);
                __syncthreads();  // every thread has read x, y, z
                if (nx == 0.0) continue;
                const double alpha = (x >= 0.0) ? -nx : nx;
                const double v0 = x - alpha;
                const double v1 = y, v2 = three ? z : 0.0;
                const double tau = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
                for (int j = max(l, k - 1) + tid; j <= hi; j += NT) {
                    double* p0 = hq_at(Hs, k, j, n);
                    double* p1 = hq_at(Hs, k + 1, j, n);
                    if (j == k - 1) {
                        *p0 = alpha;
                        *p1 = 0.0;
                        if (three) *hq_at(Hs, k + 2, j, n) = 0.0;
                        continue;
                    }
                    const double r0 = *p0, r1 = *p1;
                    const double r2 = three ? *hq_at(Hs, k + 2, j, n) : 0.0;
                    const double d = tau * (v0 * r0 + v1 * r1 + v2 * r2);
                    *p0 = r0 - d * v0;
                    *p1 = r1 - d * v1;
                    if (three) *hq_at(Hs, k + 2, j, n) = r2 - d * v2;
                }
                __syncthreads();
                const int rl = min(k + 3, hi);
                for (int i = l + tid; i <= rl; i += NT) {
                    double* p0 = hq_at(Hs, i, k, n);
                    double* p1 = hq_at(Hs, i, k + 1, n);
                    const double c0 = *p0, c1 = *p1;
                    const double c2 = three ? *hq_at(Hs, i, k + 2, n) : 0.0;
                    const double d = tau * (v0 * c0 + v1 * c1 + v2 * c2);
                    *p0 = c0 - d * v0;
                    *p1 = c1 - d * v1;
                    if (three) *hq_at(Hs, i, k + 2, n) = c2 - d * v2;
                }
                __syncthreads();
            }
            continue;
        }
        // the chain: at step t bulge b is at row k = l + t - b HQ_DS.  Each step forms
        // every bulge's reflector, applies them all from the left (disjoint rows),
        // then all from the right (disjoint columns).
        const int last = hi - 1;
        const int nsteps = (last - l) + (nb - 1) * HQ_DS + 1;
        for (int t = 0; t < nsteps; ++t) {
            if (tid < nb) {
                const int b = tid, k = l + t - b * HQ_DS;
                if (k >= l && k <= last) {
                    const bool three = k <= hi - 2;
                    double x, y, z;
                    if (k == l) {
                        const double sh = shs[b], dt = shd[b];
                        const double h00 = g(l, l), h01 = g(l, l + 1), h10 = g(l + 1, l), h11 = g(l + 1, l + 1);
                        x = h00 * h00 + h01 * h10 - sh * h00 + dt;
                        y = h10 * (h00 + h11 - sh);
                        z = h10 * g(l + 2, l + 1);
                    } else {
                        x = g(k, k - 1);
                        y = g(k + 1, k - 1);
                        z = three ? g(k + 2, k - 1) : 0.0;
                    }
                    hq_reflector(x, y, three ? z : 0.0, rfl[b]);
                }
            }
            __syncthreads();
            // from the left: bulge b on rows k..k+2, columns max(l, k-1)..hi; column
            // k-1 (k > l) is the annihilated bulge, written exactly: (alpha, 0, 0).  The
            // entry of a thread follows from l, hi and t alone; a bulge whose reflector
            // is the identity (tau = 0: x = y = z = 0) changes nothing.
            for (int e = tid; e < HQ_NB * (n + 1); e += NT) {
                int rem = e, b = -1, k = 0;
#pragma unroll
                for (int q = 0; q < HQ_NB; ++q) {
                    const int kq = l + t - q * HQ_DS;
                    const int cnt = (q < nb && kq >= l && kq <= last) ? hi - max(l, kq - 1) + 1 : 0;
                    if (b < 0) {
                        if (rem < cnt) { b = q; k = kq; } else rem -= cnt;
                    }
                }
                if (b < 0) break;
                const bool three = k <= hi - 2;
                const int j = max(l, k - 1) + rem;
                double* p0 = hq_at(Hs, k, j, n);
                double* p1 = hq_at(Hs, k + 1, j, n);
                double* p2 = hq_at(Hs, k + 2, j, n);  // (unused for a two-row reflector)
                const double v0 = rfl[b][0], v1 = rfl[b][1], v2 = rfl[b][2], tau = rfl[b][3];
                if (j == k - 1) {
                    if (tau != 0.0) {
                        *p0 = rfl[b][4];
                        *p1 = 0.0;
                        if (three) *p2 = 0.0;
                    }
                } else {
                    const double r0 = *p0, r1 = *p1, r2 = three ? *p2 : 0.0;
                    const double d = tau * (v0 * r0 + v1 * r1 + v2 * r2);
                    *p0 = r0 - d * v0;
                    *p1 = r1 - d * v1;
                    if (three) *p2 = r2 - d * v2;
                }
            }
            __syncthreads();
            // from the right: bulge b on columns k..k+2, rows l..min(k+3, hi)
            for (int e = tid; e < HQ_NB * (n + 1); e += NT) {
                int rem = e, b = -1, k = 0;
#pragma unroll
                for (int q = 0; q < HQ_NB; ++q) {
                    const int kq = l + t - q * HQ_DS;
                    const int cnt = (q < nb && kq >= l && kq <= last) ? min(kq + 3, hi) - l + 1 : 0;
                    if (b < 0) {
                        if (rem < cnt) { b = q; k = kq; } else rem -= cnt;
                    }
                }
                if (b < 0) break;
                const bool three = k <= hi - 2;
                const int i = l + rem;
                double* p0 = hq_at(Hs, i, k, n);
                double* p1 = hq_at(Hs, i, k + 1, n);
                double* p2 = hq_at(Hs, i, k + 2, n);
                const double v0 = rfl[b][0], v1 = rfl[b][1], v2 = rfl[b][2], tau = rfl[b][3];
                const double c0 = *p0, c1 = *p1, c2 = three ? *p2 : 0.0;
                const double d = tau * (v0 * c0 + v1 * c1 + v2 * c2);
                *p0 = c0 - d * v0;
                *p1 = c1 - d * v1;
                if (three) *p2 = c2 - d * v2;
            }
            __syncthreads();
        }
    }
    return true;
}

// One block of NT threads: the Ritz values (eigenvalues of H_hat, row-major,
// ld m) into ritz[0..mu) (real parts) and ritz[m..m+mu) (imaginary parts), then
// the parabola into the control block (sigma = 1: the rule carries its own scale).
template <int NT>
__global__ __launch_bounds__(NT) void contour_setup_kernel(DevCtrl* ctrl, int m, const double* __restrict__ Hh,
                                                            double tau, double* __restrict__ ritz) {
    __shared__ double Hs[HQ_LDS];  // the matrix and the slots of the entries below the subdiagonal
    if (ctrl->status != 0) return;
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 2 * HQ_P) Hs[CT_HQR_CAP + threadIdx.x] = 0.0;
    for (int i = 0; i < mu; ++i)
        for (int j = (i > 0 ? i - 1 : 0) + (int)threadIdx.x; j < mu; j += NT)
            Hs[hq_off(i, mu) + j - (i > 0 ? i - 1 : 0)] = Hh[(int64_t)i * m + j];
    __syncthreads();
    hq_balance(Hs, mu);
    double* wr = ritz;
    double* wi = ritz + m;
    const bool ok = hqr_eigs<NT>(Hs, mu, wr, wi);
    __threadfence_block();
    __syncthreads();
    if (!ok) {
        if (threadIdx.x == 0) ctrl->status = 5;  // no contour: the eigenvalue iteration did not converge
        return;
    }
    // the parabola (comment at the top of the file)
    double top = -INFINITY;
    for (int i = lane; i < mu; i += WAVE) top = fmax(top, -tau * wr[i]);
    top = wave_max(top);
    const double alpha = top + 1.0;
    double kap = CT_KAPPA_MAX;
    for (int i = lane; i < mu; i += WAVE) {
        const double re = -tau * wr[i], im = tau * wi[i];
        if (re >= top - CT_L && im != 0.0) kap = fmin(kap, (alpha - re) / (2.0 * im * im));
    }
    kap = wave_min(kap);
    if (threadIdx.x == 0) {
        const double vmax = sqrt((alpha - top + CT_L) / kap);
        ctrl->ct_a = alpha / tau;
        ctrl->ct_c = kap * tau;
        ctrl->ct_tmax = vmax / tau;
        ctrl->sigma = 1.0;
        if (!isfinite(ctrl->ct_a) || !isfinite(ctrl->ct_c) || !isfinite(ctrl->ct_tmax)) ctrl->status = 5;
    }
}

// ------------------------------------------------ complex least squares per node
// min || rhs0 e_1 - (t T1 + K0) y || over the (mu+1) x mu Hessenberg pencil with
// complex t = tr + i ti (T1 = R, K0 = R_e Hbar, real, row-major, ld m), by complex
// Givens rotations G = [[conj(c), conj(s)], [-s, c]], c = p / r, s = q / r,
// r = sqrt(|p|^2 + |q|^2) (real and positive: the triangular factor has a real
// diagonal).  One wavefront; vectors distributed as index lane + 64 q; the factor
// goes column-major into Ure, Uim (column jj at jj * m).
template <int QM>
__device__ void cpencil_ls_wave(int mu, int m, double tr, double ti, const double* __restrict__ T1r,
                                const double* __restrict__ K0r, double rhs0, double* __restrict__ Ure,
                                double* __restrict__ Uim, double (&yre)[QM], double (&yim)[QM]) {
    const int lane = threadIdx.x & 63;
    double cre[QM], cim[QM], nre[QM], nim[QM];
    double rvr[QM], rvi[QM], ud[QM];
    auto load_row = [&](int kk, int c0, double (&re)[QM], double (&im)[QM]) {
        const double* t1 = T1r + (int64_t)kk * m;
        const double* k0 = K0r + (int64_t)kk * m;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int jj = lane + WAVE * q;
            const bool in = jj >= c0 && jj < mu;
            const double a = in ? t1[jj] : 0.0, b = in ? k0[jj] : 0.0;
            re[q] = fma(tr, a, b);
            im[q] = ti * a;
        }
    };
    auto get = [&](const double (&v)[QM], int i) -> double {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < QM; ++q)
            if (q == i / WAVE) t = v[q];
        return bcast_lane(t, i % WAVE);
    };
    auto set = [&](double (&v)[QM], int i, double x) {
#pragma unroll
        for (int q = 0; q < QM; ++q)
            if (q == i / WAVE && lane == i % WAVE) v[q] = x;
    };
#pragma unroll
    for (int q = 0; q < QM; ++q) { rvr[q] = 0.0; rvi[q] = 0.0; ud[q] = 1.0; }
    load_row(0, 0, cre, cim);
    double rcr = rhs0, rci = 0.0;
    for (int kk = 0; kk < mu; ++kk) {
        load_row(kk + 1, kk, nre, nim);
        const double pr = get(cre, kk), pi = get(cim, kk), qr = get(nre, kk), qi = get(nim, kk);
        const double r = sqrt(pr * pr + pi * pi + qr * qr + qi * qi);
        const double rinv = (r != 0.0) ? 1.0 / r : 0.0;
        const double car = (r != 0.0) ? pr * rinv : 1.0, cai = pi * rinv;  // c
        const double sr = qr * rinv, si = qi * rinv;                       // s
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int jj = lane + WAVE * q;
            // top = conj(c) carry + conj(s) next; bottom = -s carry + c next
            const double tre = car * cre[q] + cai * cim[q] + sr * nre[q] + si * nim[q];
            const double tim = car * cim[q] - cai * cre[q] + sr * nim[q] - si * nre[q];
            const double bre = -(sr * cre[q] - si * cim[q]) + (car * nre[q] - cai * nim[q]);
            const double bim = -(sr * cim[q] + si * cre[q]) + (car * nim[q] + cai * nre[q]);
            if (jj >= kk && jj < mu) {
                Ure[(int64_t)jj * m + kk] = tre;
                Uim[(int64_t)jj * m + kk] = tim;
            }
            cre[q] = bre;
            cim[q] = bim;
        }
        // right-hand side: row kk gets conj(c) rc, the carry -s rc (the next row's rhs is 0)
        set(rvr, kk, car * rcr + cai * rci);
        set(rvi, kk, car * rci - cai * rcr);
        set(ud, kk, r);
        const double nr = -(sr * rcr - si * rci), ni = -(sr * rci + si * rcr);
        rcr = nr;
        rci = ni;
    }
    __threadfence_block();
    // back substitution, columns in descending order: y_k = rv_k / U_kk, rv_i -= U_ik y_k
#pragma unroll
    for (int q = 0; q < QM; ++q) { yre[q] = 0.0; yim[q] = 0.0; }
    for (int kk = mu - 1; kk >= 0; --kk) {
        const double di = 1.0 / get(ud, kk);
        const double ykr = get(rvr, kk) * di, yki = get(rvi, kk) * di;
        set(yre, kk, ykr);
        set(yim, kk, yki);
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = lane + WAVE * q;
            if (i < kk) {
                const double ur = Ure[(int64_t)kk * m + i], ui = Uim[(int64_t)kk * m + i];
                rvr[q] -= ur * ykr - ui * yki;
                rvi[q] -= ur * yki + ui * ykr;
            }
        }
    }
}

// The nodes of a group of trapezoidal levels (grp.lev_l[lev] = K + 1 nodes of the
// rule with K intervals), one wavefront per node; node i of level lev writes
// (h / pi) c_k Im(exp(tau t_k) t'_k y(t_k)) to nodebuf[i m ..].
template <int QM>
__global__ __launch_bounds__(256) void contour_level_kernel(const DevCtrl* ctrl, QuadGroup grp, double tau,
                                                             const double* __restrict__ T1r,
                                                             const double* __restrict__ K0r, double* Ubuf,
                                                             double* __restrict__ nodebuf, int m,
                                                             const double* __restrict__ X,
                                                             const double* __restrict__ eta) {
    if (ctrl->converged || ctrl->status != 0) return;
    const int mu = ctrl->m_used;
    if (mu == 0) return;
    const int lane = threadIdx.x & 63;
    const double a = ctrl->ct_a, c = ctrl->ct_c, tmax = ctrl->ct_tmax;
    const double rhs0 = eta[0] * X[0];
    const int wave = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
    const int nwaves_total = gridDim.x * (blockDim.x / WAVE);
    double* Ure = Ubuf + (int64_t)wave * 2 * m * m;  // slot = global wave index < NODE_SLOTS / 2
    double* Uim = Ure + (int64_t)m * m;
    for (int i = wave; i < grp.total; i += nwaves_total) {
        int lev = 0;
        while (lev + 1 < grp.nlev && i >= grp.lev_off[lev + 1]) ++lev;
        const int K = grp.lev_l[lev] - 1;
        const int kk = i - grp.lev_off[lev];
        const double h = tmax / K;
        const double th = h * kk;
        const double tr = a - c * th * th, ti = th;  // t(theta)
        // W = (h / pi) c_k exp(tau t) t'(theta), t' = -2 c theta + i
        const double mag = (kk == 0 ? 0.5 : 1.0) * (h / M_PI) * exp(tau * tr);
        const double er = mag * cos(tau * ti), ei = mag * sin(tau * ti);
        const double dr = -2.0 * c * th, di = 1.0;
        const double Wr = er * dr - ei * di, Wi = er * di + ei * dr;
        double yre[QM], yim[QM];
        cpencil_ls_wave<QM>(mu, m, tr, ti, T1r, K0r, rhs0, Ure, Uim, yre, yim);
        double* out = nodebuf + (int64_t)i * m;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int jj = lane + WAVE * q;
            if (jj < mu) out[jj] = Wr * yim[q] + Wi * yre[q];  // Im(W y)
        }
    }
}

hipError_t launch_contour_setup(DevCtrl* ctrl, int m, const double* Hh, double tau, double* ritz, hipStream_t st) {
    if (m <= HQ_NSMALL)
        hipLaunchKernelGGL(contour_setup_kernel<256>, dim3(1), dim3(256), 0, st, ctrl, m, Hh, tau, ritz);
    else
        hipLaunchKernelGGL(contour_setup_kernel<1024>, dim3(1), dim3(1024), 0, st, ctrl, m, Hh, tau, ritz);
    return hipGetLastError();
}

hipError_t launch_contour_level(const DevCtrl* ctrl, const QuadGroup& g, double tau, const double* T1r,
                                const double* K0r, double* Ubuf, double* nodebuf, int m, const double* X,
                                const double* eta, hipStream_t st) {
    const int slots = NODE_SLOTS_CT;
    const int waves = g.total < slots ? g.total : slots;
    const int blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(contour_level_kernel<4>, dim3(blocks), dim3(256), 0, st, ctrl, g, tau, T1r, K0r, Ubuf,
                       nodebuf, m, X, eta);
    return hipGetLastError();
}

}  // namespace skfab
