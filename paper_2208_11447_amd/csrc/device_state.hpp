// Device-side state of one solve, shared by host launchers and kernels.
#pragma once
#include <stdint.h>
#include <stddef.h>

namespace skfab {

// Control block at the start of the workspace.  Written by kernels, read back by
// the host only in synchronising calls.
struct DevCtrl {
    int32_t m_used;     // Krylov dimension in use (m unless a breakdown occurred)
    int32_t stop;       // set once the recurrence has broken down
    int32_t status;     // skfab_status of device-detected numerical failures
    int32_t l_used;     // accepted quadrature order
    int32_t converged;  // quadrature convergence flag
    int32_t l_prev;     // order of the rule held in qprev
    int32_t pad[2];
    double beta;        // ||b||
    double sigma;       // spectral scale of the quadrature
    double eps_est;     // max_j | ||S v_j||^2 - 1 |
    double rcond;       // min |R_jj| / max |R_jj|
    double logdet;      // log |det H_hat|
    double relres;      // ||S A V - [S V, S u_{m+1}] Hbar||_F / ||S A V||_F (Arnoldi relation check)
    double pad2[2];
};

// Arguments of the fused Arnoldi step kernel.
struct StepArgs {
    int64_t N;
    int64_t rows_per_chunk;
    int64_t ldU;
    const int32_t* rowptr;
    const int32_t* col;
    const double* val;
    const double* b;
    double* U;            // ldU x m, unnormalised basis u_j (v_j = u_j / eta_j)
    double* Wcur;         // A u_j (this step)
    const double* Wprev;  // A u_{j-1}
    const double* scal_prev;  // [NSC_MAX][G] partial scalars of step j-1
    double* scal_cur;         // [NSC_MAX][G] partial scalars of step j
    double* skpart;           // [G][2s] partial sketches of step j (S u_j | S A u_j)
    DevCtrl* ctrl;
    double* eta;    // [m]   ||u_j||
    double* wnorm;  // [m]   ||A v_j||
    double* H;      // [(m+1) x m] truncated MGS coefficients
    double* gram;   // [m][KMAX] <v_j, v_{j-1-q}>
    uint64_t seed;
    int32_t s, k, j, m, G;
    int32_t extend;   // 1: form u_m and its sketch only (no product with A)
    int32_t pad;
};

}  // namespace skfab
