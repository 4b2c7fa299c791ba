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
    int32_t col_wide;   // set by the SELL conversion when some |col - row| exceeds the int16 range
    int32_t flags;      // bit 0: basis truncated to its conditioned prefix (Section 2.1 remedy);
                        // bit 1: quadrature order accepted at the rounding floor, not at tol
    double beta;        // ||b||
    double sigma;       // spectral scale of the quadrature
    double eps_est;     // max_j | ||S v_j||^2 - 1 |
    double rcond;       // 1 / kappa_F(R) of the whitening factor used
    double logdet;      // log |det H_hat|
    double relres;      // ||S A V - [S V, S u_{m+1}] Hbar||_F / ||S A V||_F (Arnoldi relation check)
    double qdiff_prev;  // relative difference of the last two quadrature orders tested
    double quad_diff;   // relative difference at the accepted quadrature order
    int64_t sell_total; // entries of the SELL-64 copy of A (padded)
    int32_t sell_ok;    // 1: the SELL-64 copy fits the workspace and is used
    int32_t col16;      // 1: the SELL-64 copy stores column offsets col - row as int16
    int32_t ndict;      // distinct values of A seen by the conversion (0.0 included)
    int32_t dict_over;  // set when A has more distinct values than the value table holds
    int32_t dict8;      // 1: the SELL-64 copy stores 8-bit indices into the value table
    int32_t m_basis;    // basis length built (m_used before the conditioning truncation)
    double ct_a, ct_c, ct_tmax;  // contour t(theta) = a + i theta - c theta^2, |theta| <= tmax (exp, sGMRES)
};

// Value table of the SELL-64 copy (one per matrix): when A has at most DICT_MAX
// distinct values (0.0, the padding value, always among them), each stored entry
// is a uint8 index into `table`.  `keys` is the open-addressing set the conversion
// builds (DICT_SLOTS slots, empty = DICT_EMPTY), `slot_idx` its slot -> index map.
constexpr int DICT_MAX = 256;
constexpr int DICT_SLOTS = 512;
constexpr uint64_t DICT_EMPTY = ~0ull;
struct DictBuf {
    uint64_t keys[DICT_SLOTS];
    int32_t slot_idx[DICT_SLOTS];
    double table[DICT_MAX];
};

// Launch shape of the step kernel for one problem (host side): block size, grid
// G (a multiple of 8, at most STEP_GMAX_1024 * 1024 / block) and the contiguous
// slice / row chunks of the G blocks.
struct Launch {
    int block;
    int G;
    int64_t nslices;
    int64_t slices_per_chunk;
    int64_t rows_per_chunk;
};

// Arguments of the fused Arnoldi step kernel.
struct StepArgs {
    int64_t N;
    int64_t ldU;
    // CSR (fallback) and its SELL-64 copy: slice sl holds rows 64 sl .. 64 sl + 63,
    // entry q of row 64 sl + l at sl_ptr[sl] + 64 q + l, sl_len[sl] entries per row;
    // sl_col holds int32 columns, or int16 offsets col - row when ctrl->col16 is set.
    const int32_t* rowptr;
    const int32_t* col;
    const double* val;
    const int64_t* sl_ptr;
    const int32_t* sl_len;
    const int32_t* sl_col;
    const void* sl_val;   // values in the precision's matrix type, or uint8 table indices (ctrl->dict8)
    const double* sl_table;  // the value table (DictBuf::table) for the uint8 form
    int64_t nslices;
    int64_t slices_per_chunk;
    int64_t rows_per_chunk;
    const double* b;
    void* U;              // ldU x m, unnormalised basis u_j (v_j = u_j / eta_j), basis storage type
    void* Wcur;           // A u_j (this step), SpMV type
    const void* Wprev;    // A u_{j-1}
    const double* scal_prev;  // [NSC_MAX][G] partial scalars of step j-1
    double* scal_cur;         // [NSC_MAX][G] partial scalars of step j
    const double* skp_prev;   // [2s][G] partial sketches of step j-1 (bin-major, XCD slot order)
    double* skp_cur;          // [2s][G] partial sketches of step j (S u_j | S A u_j)
    double* SV;               // s x (m+1): S v_0 .. S v_{m-1}, then S u_m unnormalised
    double* SAV;              // s x m
    DevCtrl* ctrl;
    double* eta;    // [m+2] ||u_j||
    double* wnorm;  // [m]   ||A v_j||
    double* H;      // [(m+1) x m] truncated MGS coefficients
    double* gram;   // [m][KMAX] <v_j, v_{j-1-q}>
    const DevCtrl* sctrl;  // control block of the SELL-64 conversion of A (sell_ok)
    int64_t ldS;      // leading dimension of SV, SAV (>= s; rows s.. stay zero)
    int64_t ldH;      // leading dimension of H (>= m + 1)
    uint64_t seed;
    double inv_sqrt_zeta;
    int32_t s, k, j, m, G;
    int32_t extend;   // 1: form u_m and its sketch only (no product with A)
    int32_t uring;    // columns of U: basis vector c lives in column c % uring (m, or k + 1
                      // for the two-pass form, whose first pass keeps only the window; m + 1
                      // with keep_ext)
    int32_t nosketch; // 1: no sparse-sign sketch in the step (the SRDCT sketch is applied to
                      // the stored basis afterwards)
    int32_t keep_ext; // 1: the extension pass stores u_m in column m % uring
    int32_t sav;      // 1: also sketch A u_j (S A V_m, read only by the Arnoldi relation check)
};

// One (problem, right-hand side) pair of a batched solve: the step arguments
// that do not depend on j, and the double-buffered arrays selected by j's parity.
struct BatchStepUnit {
    StepArgs a;
    void* W[2];
    double* scal[2];
    double* skp[2];
};

// Per-unit pointers of the batched small problem and assembly.  Every unit's
// small arrays use the batch's common leading dimensions (m_max, s_max); the
// unit's own Krylov dimension is its control block's m_used.
struct SmallUnit {
    DevCtrl* ctrl;
    double *SV, *SAV, *H, *eta, *colnorm2, *chk, *Tws, *K0r, *T1r, *Hh, *Ubuf, *Urhs, *nodebuf, *qprev, *y0, *ys, *y;
    double* cnd;  // [2 (m_max + 1)] column norms of R^-1 and of R (conditioning test)
    const void* U;
    int64_t ldU, N;
    double* x;
    int32_t m, pad;
};

// A group of consecutive quadrature orders evaluated by one launch.
constexpr int MAX_GROUP_LEVELS = 16;
struct QuadGroup {
    int32_t nlev;
    int32_t total;                       // nodes in the group
    int32_t lev_l[MAX_GROUP_LEVELS];     // order of each level
    int32_t lev_off[MAX_GROUP_LEVELS];   // first node of each level
    int32_t first;                       // 1: the group starts the sequence (its first level seeds qprev)
    int32_t last;                        // 1: the group ends the sequence (its last level is the final order)
};

}  // namespace skfab
