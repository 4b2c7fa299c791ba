// Kernels of the learned controller of (m, k, s): cheap matrix features
// (Gershgorin bounds) and the network 16 -> 64 -> 64 -> 3 (ReLU hidden layers,
// linear output, FP32) with its mean-squared-error gradient and Adam update.
//
// Parameter vector (row-major): W1 [64][16], b1 [64], W2 [64][64], b2 [64],
// W3 [3][64], b3 [3].  Loss L = (1 / (3 B)) sum_{b,o} (y_bo - t_bo)^2.  Every sum
// has a fixed order (one thread per output, sequential over the contraction), so
// results are reproducible run to run.  The contractions are tiny (B x 64 x 64);
// plain FP32 FMA throughput is not the limit, launch latency is.
#include "common.hpp"
#include "device_state.hpp"

namespace skfab {

constexpr int MLP_IN = 16, MLP_HID = 64, MLP_OUT = 3;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_HID * MLP_IN, OFF_W2 = OFF_B1 + MLP_HID,
              OFF_B2 = OFF_W2 + MLP_HID * MLP_HID, OFF_W3 = OFF_B2 + MLP_HID, OFF_B3 = OFF_W3 + MLP_OUT * MLP_HID,
              MLP_PARAMS = OFF_B3 + MLP_OUT;

// ------------------------------------------------------- Gershgorin bounds
// Per row: a_ii -/+ sum_{j != i} |a_ij|; block partials of min / max, then one block.
__global__ __launch_bounds__(256) void gershgorin_kernel(const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val, int64_t N,
                                                         double* __restrict__ part) {
    __shared__ double scratch[4];
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += (int64_t)gridDim.x * 256) {
        double d = 0.0, off = 0.0;
        for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
            if (col[e] == r) d += val[e];
            else off += fabs(val[e]);
        }
        lo = fmin(lo, d - off);
        hi = fmax(hi, d + off);
    }
    lo = -block_max(-lo, scratch);
    hi = block_max(hi, scratch);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = lo; part[2 * blockIdx.x + 1] = hi; }
}

__global__ __launch_bounds__(256) void gershgorin_finish_kernel(const double* __restrict__ part, int nb,
                                                                double* __restrict__ out) {
    __shared__ double scratch[4];
    double lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < nb; i += 256) { lo = fmin(lo, part[2 * i]); hi = fmax(hi, part[2 * i + 1]); }
    lo = -block_max(-lo, scratch);
    hi = block_max(hi, scratch);
    if (threadIdx.x == 0) { out[0] = lo; out[1] = hi; }
}

// ------------------------------------------------------------------ network
// Z = in W^T + bias (B x nout), A = relu(Z) or Z; one thread per output.
__global__ __launch_bounds__(256) void dense_fwd_kernel(const float* __restrict__ in, int B, int nin,
                                                        const float* __restrict__ W, const float* __restrict__ bias,
                                                        int nout, float* __restrict__ Z, float* __restrict__ A,
                                                        int relu) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= B * nout) return;
    const int b = idx / nout, o = idx - b * nout;
    const float* x = in + (int64_t)b * nin;
    const float* w = W + (int64_t)o * nin;
    float z = bias[o];
    for (int i = 0; i < nin; ++i) z = fmaf(w[i], x[i], z);
    if (Z) Z[idx] = z;
    A[idx] = relu ? fmaxf(z, 0.0f) : z;
}

// dY = 2 (Y - T) / (3 B) and the loss, one block (fixed-order sums).
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                       int B, float* __restrict__ dY, float* __restrict__ loss) {
    __shared__ double scratch[4];
    const int n = B * MLP_OUT;
    const float sc = 2.0f / (float)n;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const float d = Y[i] - T[i];
        dY[i] = sc * d;
        acc += (double)d * (double)d;
    }
    acc = block_sum(acc, scratch);
    if (threadIdx.x == 0 && loss) *loss = (float)(acc / n);
}

// dIn[b][i] = (sum_o dZ[b][o] W[o][i]) * (Zin[b][i] > 0)
__global__ __launch_bounds__(256) void dense_bwd_input_kernel(const float* __restrict__ dZ, int B, int nout,
                                                              const float* __restrict__ W, int nin,
                                                              const float* __restrict__ Zin,
                                                              float* __restrict__ dIn) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= B * nin) return;
    const int b = idx / nin, i = idx - b * nin;
    const float* dz = dZ + (int64_t)b * nout;
    float t = 0.0f;
    for (int o = 0; o < nout; ++o) t = fmaf(dz[o], W[(int64_t)o * nin + i], t);
    dIn[idx] = (Zin[idx] > 0.0f) ? t : 0.0f;
}

// gW[o][i] = sum_b dZ[b][o] in[b][i] (i < nin), gb[o] = sum_b dZ[b][o] (i == nin)
__global__ __launch_bounds__(256) void dense_bwd_weight_kernel(const float* __restrict__ dZ, int B, int nout,
                                                               const float* __restrict__ in, int nin,
                                                               float* __restrict__ gW, float* __restrict__ gb) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= nout * (nin + 1)) return;
    const int o = idx / (nin + 1), i = idx - o * (nin + 1);
    float t = 0.0f;
    if (i < nin) {
        for (int b = 0; b < B; ++b) t = fmaf(dZ[(int64_t)b * nout + o], in[(int64_t)b * nin + i], t);
        gW[(int64_t)o * nin + i] = t;
    } else {
        for (int b = 0; b < B; ++b) t += dZ[(int64_t)b * nout + o];
        gb[o] = t;
    }
}

// Adam (Kingma & Ba 2015) with the bias corrections c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m1, float* __restrict__ m2, int n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float m = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = m;
    m2[i] = v;
    p[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// ---------------------------------------------------------------- launchers
static inline int nblk(int n) { return (n + 255) / 256; }

int gershgorin_blocks(int64_t N) {
    const int64_t b = (N + 255) / 256;
    return (int)(b < 1024 ? b : 1024);
}

hipError_t launch_gershgorin(const int32_t* rowptr, const int32_t* col, const double* val, int64_t N, double* part,
                             double* out, hipStream_t st) {
    const int nb = gershgorin_blocks(N);
    hipLaunchKernelGGL(gershgorin_kernel, dim3(nb), dim3(256), 0, st, rowptr, col, val, N, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gershgorin_finish_kernel, dim3(1), dim3(256), 0, st, part, nb, out);
    return hipGetLastError();
}

int mlp_param_count() { return MLP_PARAMS; }

// workspace floats: Z1, A1, Z2, A2 (B x 64 each), Y, dY (B x 3), dZ2, dZ1 (B x 64)
size_t mlp_ws_floats(int B) { return (size_t)B * (6 * MLP_HID + 2 * MLP_OUT); }

struct MlpWs {
    float *Z1, *A1, *Z2, *A2, *Y, *dY, *dZ2, *dZ1;
};

static MlpWs mlp_carve(float* ws, int B) {
    MlpWs w;
    const size_t h = (size_t)B * MLP_HID, o = (size_t)B * MLP_OUT;
    w.Z1 = ws; w.A1 = w.Z1 + h; w.Z2 = w.A1 + h; w.A2 = w.Z2 + h; w.Y = w.A2 + h; w.dY = w.Y + o;
    w.dZ2 = w.dY + o; w.dZ1 = w.dZ2 + h;
    return w;
}

static hipError_t mlp_fwd(const float* X, int B, const float* p, const MlpWs& w, float* Y, hipStream_t st) {
    hipLaunchKernelGGL(dense_fwd_kernel, dim3(nblk(B * MLP_HID)), dim3(256), 0, st, X, B, MLP_IN, p + OFF_W1,
                       p + OFF_B1, MLP_HID, w.Z1, w.A1, 1);
    hipLaunchKernelGGL(dense_fwd_kernel, dim3(nblk(B * MLP_HID)), dim3(256), 0, st, w.A1, B, MLP_HID, p + OFF_W2,
                       p + OFF_B2, MLP_HID, w.Z2, w.A2, 1);
    hipLaunchKernelGGL(dense_fwd_kernel, dim3(nblk(B * MLP_OUT)), dim3(256), 0, st, w.A2, B, MLP_HID, p + OFF_W3,
                       p + OFF_B3, MLP_OUT, (float*)nullptr, Y, 0);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* X, int B, const float* p, float* Y, float* ws, hipStream_t st) {
    return mlp_fwd(X, B, p, mlp_carve(ws, B), Y, st);
}

hipError_t launch_mlp_loss_grad(const float* X, const float* T, int B, const float* p, float* g, float* loss,
                                float* ws, hipStream_t st) {
    const MlpWs w = mlp_carve(ws, B);
    hipError_t e = mlp_fwd(X, B, p, w, w.Y, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mse_grad_kernel, dim3(1), dim3(256), 0, st, w.Y, T, B, w.dY, loss);
    // layer 3
    hipLaunchKernelGGL(dense_bwd_weight_kernel, dim3(nblk(MLP_OUT * (MLP_HID + 1))), dim3(256), 0, st, w.dY, B,
                       MLP_OUT, w.A2, MLP_HID, g + OFF_W3, g + OFF_B3);
    hipLaunchKernelGGL(dense_bwd_input_kernel, dim3(nblk(B * MLP_HID)), dim3(256), 0, st, w.dY, B, MLP_OUT,
                       p + OFF_W3, MLP_HID, w.Z2, w.dZ2);
    // layer 2
    hipLaunchKernelGGL(dense_bwd_weight_kernel, dim3(nblk(MLP_HID * (MLP_HID + 1))), dim3(256), 0, st, w.dZ2, B,
                       MLP_HID, w.A1, MLP_HID, g + OFF_W2, g + OFF_B2);
    hipLaunchKernelGGL(dense_bwd_input_kernel, dim3(nblk(B * MLP_HID)), dim3(256), 0, st, w.dZ2, B, MLP_HID,
                       p + OFF_W2, MLP_HID, w.Z1, w.dZ1);
    // layer 1
    hipLaunchKernelGGL(dense_bwd_weight_kernel, dim3(nblk(MLP_HID * (MLP_IN + 1))), dim3(256), 0, st, w.dZ1, B,
                       MLP_HID, X, MLP_IN, g + OFF_W1, g + OFF_B1);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, const float* g, float* m1, float* m2, int n, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(n)), dim3(256), 0, st, p, g, m1, m2, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace skfab
