// Adaptive choice of m (Section 4.3): the basis is nested, so the sketched FOM
// approximant of any m' below the current step can be formed from the data the
// recurrence has already written.  These kernels take a snapshot of the first m'
// steps in the form of the small-problem input (normalised basis), evaluate the
// relative stopping estimate between two checkpoints, and rescale the accepted
// coefficients to the stored (unnormalised) basis.
#include "common.hpp"
#include "device_state.hpp"

namespace skfab {

// Small-problem input of the first mp steps: SVs[:, j] = S v_j (j < mp),
// SVs[:, mp] = eta_mp S v_mp = S u_mp (the unnormalised extension), Hs = H[:mp+1, :mp]
// (ld mp + 1), eta_s = (beta, 1, 1, ...), colnorm2 = 1 and SAV = 0 (relation check off).
__global__ __launch_bounds__(256) void snapshot_kernel(const double* __restrict__ SV, int s,
                                                       const double* __restrict__ H, int64_t ldh,
                                                       const double* __restrict__ eta, int mp,
                                                       double* __restrict__ SVs, double* __restrict__ Hs,
                                                       double* __restrict__ etas, double* __restrict__ cn2,
                                                       double* __restrict__ SAVs) {
    const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x, nt = (int64_t)gridDim.x * 256;
    const double emp = eta[mp];
    const int64_t n1 = (int64_t)s * (mp + 1);
    for (int64_t i = tid; i < n1; i += nt) {
        const int64_t j = i / s;
        SVs[i] = (j < mp) ? SV[i] : emp * SV[i];
    }
    const int64_t n2 = (int64_t)(mp + 1) * mp;
    for (int64_t i = tid; i < n2; i += nt) {
        const int64_t j = i / (mp + 1), r = i - j * (mp + 1);
        Hs[i] = H[r + ldh * j];
    }
    for (int64_t i = tid; i < mp + 2; i += nt) etas[i] = (i == 0) ? eta[0] : 1.0;
    for (int64_t i = tid; i < mp + 1; i += nt) cn2[i] = 1.0;
    const int64_t n3 = (int64_t)s * mp;
    for (int64_t i = tid; i < n3; i += nt) SAVs[i] = 0.0;
}

// out[0] = || SV (y - [yp; 0]) || / || SV y || * sqrt((1 + e) / (1 - e)),
// e = max_{j < mp} | ||SV_j||^2 - 1 |  (+inf when there is no previous checkpoint or
// the small problem reported a failure); out[1] = that status; ysave = y.
__global__ __launch_bounds__(256) void adaptive_est_kernel(const double* __restrict__ SV, int s, int mp,
                                                           const double* __restrict__ y,
                                                           const double* __restrict__ yp, int mprev,
                                                           const DevCtrl* __restrict__ sctrl,
                                                           double* __restrict__ out, double* __restrict__ ysave) {
    __shared__ double ysh[MMAX], dsh[MMAX];
    __shared__ double scratch[4];
    const int tid = threadIdx.x;
    for (int j = tid; j < mp; j += 256) {
        const double v = y[j];
        ysh[j] = v;
        dsh[j] = v - ((j < mprev) ? yp[j] : 0.0);
    }
    __syncthreads();
    double num = 0.0, den = 0.0;
    for (int i = tid; i < s; i += 256) {
        double a = 0.0, c = 0.0;
        for (int j = 0; j < mp; ++j) {
            const double x = SV[i + (int64_t)s * j];
            a = fma(x, ysh[j], a);
            c = fma(x, dsh[j], c);
        }
        den = fma(a, a, den);
        num = fma(c, c, num);
    }
    double e = 0.0;
    for (int j = tid; j < mp; j += 256) {
        double cn = 0.0;
        for (int i = 0; i < s; ++i) {
            const double x = SV[i + (int64_t)s * j];
            cn = fma(x, x, cn);
        }
        e = fmax(e, fabs(cn - 1.0));
    }
    num = block_sum(num, scratch);
    den = block_sum(den, scratch);
    e = block_max(e, scratch);
    for (int j = tid; j < mp; j += 256) ysave[j] = ysh[j];
    if (tid == 0) {
        const int st = sctrl->status;
        double est = INFINITY;
        if (mprev > 0 && st == 0 && e < 1.0) {
            if (den > 0.0) est = sqrt(num / den) * sqrt((1.0 + e) / (1.0 - e));
            else est = (num == 0.0) ? 0.0 : INFINITY;
        }
        out[0] = est;
        out[1] = (double)st;
    }
}

// ys[j] = y[j] / eta[j], j < mp: coefficients of the stored basis u_j = eta_j v_j.
__global__ __launch_bounds__(256) void rescale_coeffs_kernel(const double* __restrict__ y,
                                                             const double* __restrict__ eta, int mp,
                                                             double* __restrict__ ys) {
    for (int j = threadIdx.x; j < mp; j += 256) ys[j] = y[j] / eta[j];
}

hipError_t launch_snapshot(const double* SV, int s, const double* H, int64_t ldh, const double* eta, int mp,
                           double* SVs, double* Hs, double* etas, double* cn2, double* SAVs, hipStream_t st) {
    const int64_t n = (int64_t)s * (mp + 1);
    int64_t g = (n + 255) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(snapshot_kernel, dim3((unsigned)g), dim3(256), 0, st, SV, s, H, ldh, eta, mp, SVs, Hs, etas,
                       cn2, SAVs);
    return hipGetLastError();
}

hipError_t launch_adaptive_est(const double* SV, int s, int mp, const double* y, const double* yp, int mprev,
                               const DevCtrl* sctrl, double* out, double* ysave, hipStream_t st) {
    hipLaunchKernelGGL(adaptive_est_kernel, dim3(1), dim3(256), 0, st, SV, s, mp, y, yp, mprev, sctrl, out, ysave);
    return hipGetLastError();
}

hipError_t launch_rescale_coeffs(const double* y, const double* eta, int mp, double* ys, hipStream_t st) {
    hipLaunchKernelGGL(rescale_coeffs_kernel, dim3(1), dim3(256), 0, st, y, eta, mp, ys);
    return hipGetLastError();
}

}  // namespace skfab
