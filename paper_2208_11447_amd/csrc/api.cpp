// C ABI of libskfab: validation, workspace layout and the launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/skfab.h"
#include "common.hpp"
#include "device_state.hpp"

namespace skfab {
hipError_t launch_arnoldi_step(const StepArgs& a, int zeta, int block, int prec, hipStream_t st);
hipError_t launch_arnoldi_tail(const StepArgs& a, double* colnorm2, hipStream_t st);
hipError_t launch_arnoldi_check(const double* SV, const double* SAV, const double* H, int s, int m, int k,
                                DevCtrl* ctrl, double* part, hipStream_t st);
int64_t sell_scan_blocks(int64_t nslices);
hipError_t launch_sell_convert(const int32_t* rowptr, const int32_t* col, const double* val, int64_t N,
                               int64_t nslices, int64_t capacity, DevCtrl* ctrl, int32_t* sl_len, int64_t* sl_ptr,
                               int64_t* bsum, int32_t* sl_col, void* sl_val, DictBuf* dict, int use_dict, int prec,
                               hipStream_t st);
hipError_t launch_normalize_basis(const void* U, int64_t ldU, int64_t N, int m, const DevCtrl* ctrl,
                                  const double* eta, double* V, int prec, hipStream_t st);
hipError_t launch_sketch_pattern(int64_t col0, int64_t ncols, int s, int zeta, uint64_t seed, int32_t* rows,
                                 int8_t* signs, hipStream_t st);
hipError_t launch_sketch_apply(int64_t n, int s, int zeta, uint64_t seed, const double* v, double* Sv,
                               double* part, hipStream_t st);
int sketch_apply_blocks(int64_t n);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_init_ctrl(DevCtrl* c, int m, hipStream_t st);
hipError_t launch_qr(double* X, int s, int ncols_max, const DevCtrl* ctrl, double* Tws, hipStream_t st);
hipError_t launch_cond_trunc(double* X, int s, int m, DevCtrl* ctrl, const double* H, double* cnd, double cmax,
                             hipStream_t st);
hipError_t launch_cond_trunc_batched(const SmallUnit* units, int nunits, int s, int m, double cmax, hipStream_t st);
// launch rule of the step kernel (arnoldi.hip)
int step_block_fit(int block, int s);
Launch step_launch(int64_t N, int s, int k);
hipError_t launch_pencil_setup(const double* X, int s, int m, int k, const DevCtrl* ctrl, const double* H,
                               double* K0r, double* T1r, hipStream_t st);
hipError_t launch_hhat_rows(const DevCtrl* ctrl, int m, int s, const double* X, const double* T1r, const double* H,
                            double* Hh, hipStream_t st);
hipError_t launch_hhat_rows_batched(const SmallUnit* units, int nunits, int m, int s, hipStream_t st);
hipError_t launch_pencil_scalars(int m, int s, const double* X, DevCtrl* ctrl, const double* eta,
                                 const double* T1r, const double* K0r, const double* Hh, double* Ubuf, double* Urhs,
                                 double* y0, int is_ls, int branch_check, int k, hipStream_t st);
hipError_t launch_quad_group(const DevCtrl* ctrl, const QuadGroup& g, const double* T1r, const double* K0r,
                             const double* Hh, double* Ubuf, double* Urhs, double* nodebuf, int m, int is_ls,
                             const double* X, const double* eta, int k, hipStream_t st);
hipError_t launch_contour_setup(DevCtrl* ctrl, int m, const double* Hh, double tau, double* ritz, hipStream_t st);
hipError_t launch_contour_level(const DevCtrl* ctrl, const QuadGroup& g, double tau, const double* T1r,
                                const double* K0r, double* Ubuf, double* nodebuf, int m, const double* X,
                                const double* eta, hipStream_t st);
hipError_t launch_quad_reduce(DevCtrl* ctrl, const QuadGroup& g, const double* nodebuf, int m, double tol,
                              const double* T1r, double* qprev, double* y, hipStream_t st);
hipError_t launch_quad_fail(DevCtrl* ctrl, hipStream_t st);
hipError_t launch_poly(const DevCtrl* ctrl, int m, const double* T1r, const double* K0r, const double* eta,
                       const double* coef, int npoly, double* y, hipStream_t st);
hipError_t launch_finish_coeffs(DevCtrl* ctrl, int m, const double* y, const double* eta, const double* colnorm2,
                                double* ys, double* yout, hipStream_t st);
hipError_t launch_assemble(const void* U, int64_t ldU, int64_t N, int m, const DevCtrl* ctrl, const double* ys,
                           double* x, int prec, hipStream_t st);
hipError_t launch_norm1(const DevCtrl* ctrl, int m, const double* const* P, int count, double* norm1,
                        hipStream_t st);
hipError_t launch_accum_basis(const void* Uj, int64_t N, int j, const DevCtrl* ctrl, const double* ys, double* x,
                              int prec, hipStream_t st);
hipError_t launch_colnorm(const double* SV, int s, int m, const DevCtrl* ctrl, double* colnorm2, hipStream_t st);
size_t srdct_part_doubles(int s, int64_t N, int ncols);
hipError_t launch_srdct_matrix(int s, int64_t N, const int8_t* signs, const int32_t* rows, double* FP,
                               hipStream_t st);
hipError_t launch_srdct_sketch(const double* FP, int s, int64_t N, const void* U, int64_t ldU, int ncols, int prec,
                               double* part, const DevCtrl* ctrl, const double* eta, double* SV, int64_t ldS,
                               hipStream_t st);
hipError_t launch_hhat(const DevCtrl* ctrl, int m, const double* T1r, const double* X, int s, const double* H,
                       double tau, double* Ahat, double* norm1, hipStream_t st);
hipError_t launch_combine(const DevCtrl* ctrl, int m, double a, const double* P, double b, const double* Q,
                          double c, const double* R, double d, double* D, hipStream_t st);
hipError_t launch_dgemm(const DevCtrl* ctrl, int m, const double* A, const double* B, double beta, double* C,
                        hipStream_t st);
hipError_t launch_lu(DevCtrl* ctrl, int m, double* Q, int* piv, hipStream_t st);
hipError_t launch_lu_solve_cols(const DevCtrl* ctrl, int m, const double* LU, const int* piv, double* P,
                                hipStream_t st);
hipError_t launch_first_column(const DevCtrl* ctrl, const double* X, const double* eta, double* y, hipStream_t st);
hipError_t launch_arnoldi_step_batched(const BatchStepUnit* units, const int* base, int nact, int R, int j, int k,
                                       int g0, int grid, int block, int smax, int prec, hipStream_t st);
size_t packed_step_lds(int block, int R, int smax);
hipError_t launch_arnoldi_step_packed(const BatchStepUnit* units, const int* base, int nprob, int R, int j, int grid,
                                      int smax, int prec, hipStream_t st);
hipError_t launch_arnoldi_tail_batched(const BatchStepUnit* units, const SmallUnit* small, int nunits, int smax,
                                       int mmax, hipStream_t st);
hipError_t launch_arnoldi_check_batched(const SmallUnit* small, int nunits, int smax, int mmax, int k,
                                        hipStream_t st);
hipError_t launch_init_ctrl_batched(const SmallUnit* units, int nunits, hipStream_t st);
hipError_t launch_qr_batched(const SmallUnit* units, int nunits, int s, int ncols_max, hipStream_t st);
hipError_t launch_pencil_setup_batched(const SmallUnit* units, int nunits, int s, int m, int k, hipStream_t st);
hipError_t launch_pencil_scalars_batched(const SmallUnit* units, int nunits, int m, int s, int is_ls, int branch_check,
                                         int k, hipStream_t st);
hipError_t launch_quad_group_batched(const SmallUnit* units, int nunits, const QuadGroup& g, int m, int is_ls,
                                     int slots, int k, hipStream_t st);
hipError_t launch_quad_reduce_batched(const SmallUnit* units, int nunits, const QuadGroup& g, int m, double tol,
                                      hipStream_t st);
hipError_t launch_quad_fail_batched(const SmallUnit* units, int nunits, hipStream_t st);
hipError_t launch_finish_coeffs_batched(const SmallUnit* units, int nunits, int m, hipStream_t st);
hipError_t launch_assemble_batched(const SmallUnit* units, int nunits, int64_t nmax, int m, int prec,
                                   hipStream_t st);
hipError_t launch_snapshot(const double* SV, int s, const double* H, int64_t ldh, const double* eta, int mp,
                           double* SVs, double* Hs, double* etas, double* cn2, double* SAVs, hipStream_t st);
hipError_t launch_adaptive_est(const double* SV, int s, int mp, const double* y, const double* yp, int mprev,
                               const DevCtrl* sctrl, double* out, double* ysave, hipStream_t st);
hipError_t launch_rescale_coeffs(const double* y, const double* eta, int mp, double* ys, hipStream_t st);
int gershgorin_blocks(int64_t N);
hipError_t launch_gershgorin(const int32_t* rowptr, const int32_t* col, const double* val, int64_t N, double* part,
                             double* out, hipStream_t st);
int mlp_param_count();
size_t mlp_ws_floats(int B);
hipError_t launch_mlp_forward(const float* X, int B, const float* p, float* Y, float* ws, hipStream_t st);
hipError_t launch_mlp_loss_grad(const float* X, const float* T, int B, const float* p, float* g, float* loss,
                                float* ws, hipStream_t st);
hipError_t launch_mlp_adam(float* p, const float* g, float* m1, float* m2, int n, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t st);
constexpr int QR_NB_HOST = 16;
constexpr int NODE_SLOTS_HOST = 1024;
}  // namespace skfab

using namespace skfab;

namespace skfab {
skfab_status noalloc_init_device(int device);
int ctx_device(const skfab_ctx* ctx);
}  // namespace skfab

struct skfab_ctx {
    int device;
    hipStream_t stream;
    // optional timing of kernel classes (0: Arnoldi step, 1: assembly): a run of
    // consecutive launches of a class as one interval, isolated launches every
    // stride-th one
    bool timing = false;
    int32_t stride = 1;             // every stride-th isolated launch of a class is timed
    int64_t tick[2] = {0, 0};       // isolated launches of each class seen while enabled
    std::vector<hipEvent_t> ev[2];  // start/stop pairs, flattened
    std::vector<int32_t> nl[2];     // launches covered by each pair
    size_t used[2] = {0, 0};
    double acc_ms[2] = {0.0, 0.0};
    int64_t count[2] = {0, 0};
    // batched solves: launch shape of the step kernel, and the host copy of the
    // unit descriptors (kept alive until the next batched call has synchronised)
    int batch_block = 1024;
    int batch_spw = 1;
    // the packed form of the batched step (one block per chunk for all of a
    // problem's right-hand sides) where it applies: k = 2, 512-thread blocks, the
    // steps 2 <= j < m, the Arnoldi relation check off, its bins within the LDS.
    // Off unless set or chosen by the autotuner: in FP64 its registers spill.
    bool batch_packed = false;
    std::vector<char> batch_host;
    // the SELL copy may store A's values as uint8 indices into a value table when A
    // has at most 256 distinct values (FP64 form only: for 4-byte values the table
    // lookup costs more than the 3 bytes per entry it saves)
    bool value_table = true;
    // the step kernels also sketch A u_j (S A V_m) and the small problem checks the
    // Arnoldi relation against it (info.arnoldi_relres); off: neither (relres -1)
    bool arnoldi_check = false;
};

int skfab::ctx_device(const skfab_ctx* ctx) { return ctx ? ctx->device : -1; }

namespace {
constexpr size_t TIMING_PAIRS = 2048;

// Sum the durations of the recorded pairs of class c and recycle them.
hipError_t timing_flush(skfab_ctx* ctx, int c) {
    if (ctx->used[c] == 0) return hipSuccess;
    hipError_t e = hipEventSynchronize(ctx->ev[c][2 * ctx->used[c] - 1]);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < ctx->used[c]; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ctx->ev[c][2 * i], ctx->ev[c][2 * i + 1]);
        if (e != hipSuccess) return e;
        ctx->acc_ms[c] += ms;
        ctx->count[c] += ctx->nl[c][i];
    }
    ctx->used[c] = 0;
    return hipSuccess;
}

// An open interval of class c (stop == nullptr: not timed).
struct Span {
    hipEvent_t stop = nullptr;
    int c = 0;
    size_t i = 0;
};

// Opens the interval of the next launch of class c, or with run = true of a run of
// consecutive launches of class c (always timed: one pair of events for the whole
// run keeps the events' own cost out of the per-launch mean).  Intervals of one
// class do not nest.
hipError_t timing_begin(skfab_ctx* ctx, int c, hipStream_t st, Span* sp, bool run = false) {
    sp->stop = nullptr;
    if (!ctx || !ctx->timing) return hipSuccess;
    if (!run && ctx->tick[c]++ % ctx->stride != 0) return hipSuccess;
    if (ctx->used[c] == TIMING_PAIRS) {
        hipError_t e = timing_flush(ctx, c);
        if (e != hipSuccess) return e;
    }
    const size_t i = ctx->used[c]++;
    sp->stop = ctx->ev[c][2 * i + 1];
    sp->c = c;
    sp->i = i;
    return hipEventRecord(ctx->ev[c][2 * i], st);
}

// Closes the interval; it counts as `launches` launches of its class.
hipError_t timing_end(skfab_ctx* ctx, const Span& sp, hipStream_t st, int launches = 1) {
    if (!sp.stop) return hipSuccess;
    ctx->nl[sp.c][sp.i] = launches;
    return hipEventRecord(sp.stop, st);
}

// Drops an interval that will not be closed (a launch of the run failed).
void timing_cancel(skfab_ctx* ctx, const Span& sp) {
    if (sp.stop && ctx->used[sp.c] == sp.i + 1) --ctx->used[sp.c];
}
}  // namespace

namespace {

constexpr size_t ALIGN = 256;
constexpr int EXP_BUFS = 10;  // dense m x m work matrices of the exponential

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int next_order(int l) {
    // floor(sqrt(2) * l) exactly: largest q with q*q <= 2*l*l
    const int64_t t = 2LL * l * l;
    int64_t q = (int64_t)std::sqrt((double)t);
    while (q * q > t) --q;
    while ((q + 1) * (q + 1) <= t) ++q;
    return (int)q;
}

struct Layout {
    size_t ctrl, eta, wnorm, H, gram, colnorm2, scal, U, W, skpart, SV, SAV, Tws, K0r, T1r, Hh, Ubuf, Urhs, nodebuf,
        qprev, qcur, y, ys, y0, poly, expbuf, piv, norm1, chk, cnd, srfp, srpart, sl_len, sl_ptr, bsum, sl_col, sl_val, dict, total;
    int64_t ldU;
    int64_t sell_capacity;
    int lnodes;
    Launch L;
};

std::vector<int> order_sequence(int l1, int l2, int lmax) {
    std::vector<int> seq{l1, l2};
    while (true) {
        const int nx = next_order(seq.back());
        if (nx > lmax) break;
        seq.push_back(nx);
    }
    return seq;
}

// Consecutive orders packed into launches of at most NODE_SLOTS nodes (a single
// order larger than that forms its own group).
std::vector<QuadGroup> quad_groups(int l1, int l2, int lmax) {
    const std::vector<int> seq = order_sequence(l1, l2, lmax);
    std::vector<QuadGroup> out;
    QuadGroup g;
    std::memset(&g, 0, sizeof(g));
    g.first = 1;
    for (int l : seq) {
        if (g.nlev > 0 && (g.total + l > NODE_SLOTS_HOST || g.nlev == MAX_GROUP_LEVELS)) {
            out.push_back(g);
            std::memset(&g, 0, sizeof(g));
        }
        g.lev_l[g.nlev] = l;
        g.lev_off[g.nlev] = g.total;
        g.total += l;
        g.nlev += 1;
    }
    if (g.nlev > 0) out.push_back(g);
    if (!out.empty()) out.back().last = 1;
    return out;
}

// Trapezoidal levels of the contour rule (K = CT_KFIRST, 2 CT_KFIRST, ..., CT_KMAX
// intervals, K + 1 nodes each), packed like quad_groups.
std::vector<QuadGroup> contour_groups() {
    std::vector<QuadGroup> out;
    QuadGroup g;
    std::memset(&g, 0, sizeof(g));
    g.first = 1;
    for (int K = CT_KFIRST; K <= CT_KMAX; K *= 2) {
        const int l = K + 1;
        if (g.nlev > 0 && (g.total + l > NODE_SLOTS_HOST || g.nlev == MAX_GROUP_LEVELS)) {
            out.push_back(g);
            std::memset(&g, 0, sizeof(g));
        }
        g.lev_l[g.nlev] = l;
        g.lev_off[g.nlev] = g.total;
        g.total += l;
        g.nlev += 1;
    }
    if (g.nlev > 0) out.push_back(g);
    if (!out.empty()) out.back().last = 1;
    return out;
}

int max_level_nodes(int l1, int l2, int lmax) {
    int mx = 0;
    for (const QuadGroup& g : quad_groups(l1, l2, lmax)) mx = g.total > mx ? g.total : mx;
    for (const QuadGroup& g : contour_groups()) mx = g.total > mx ? g.total : mx;
    return mx;
}

// bytes of the basis (V), SpMV (W) and matrix-value (A) element types of a precision
size_t vbytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }
size_t wbytes(int prec) { return prec == 0 ? 8 : 4; }

Layout make_layout(int64_t N, int64_t nnz, int m, int s, int l1, int l2, int lmax, int npoly, bool with_basis,
                   int prec, int k = 1, int ucols = 0, bool srdct = false) {
    Layout ly;
    ly.L = step_launch(N > 0 ? N : 1, s, k);
    ly.ldU = (N + 63) / 64 * 64;
    ly.lnodes = max_level_nodes(l1, l2, lmax);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t d = sizeof(double);
    const int G = ly.L.G;
    ly.ctrl = take(sizeof(DevCtrl));
    ly.eta = take((m + 2) * d);
    ly.wnorm = take((m + 2) * d);
    ly.H = take((size_t)(m + 1) * m * d);
    ly.gram = take((size_t)(m + 1) * KMAX * d);
    ly.colnorm2 = take((m + 1) * d);
    ly.scal = take((size_t)2 * NSC_MAX * G * d);
    ly.U = with_basis ? take((size_t)ly.ldU * (ucols > 0 ? ucols : m) * vbytes(prec)) : take(0);
    ly.W = with_basis ? take((size_t)2 * ly.ldU * wbytes(prec)) : take(0);
    ly.skpart = with_basis ? take((size_t)2 * G * 2 * s * d) : take(0);
    // SELL-64 copy of A: room for 25% more entries than nnz plus one padded row per slice
    ly.sell_capacity = with_basis ? nnz + nnz / 4 + 64 * ly.L.nslices : 0;
    ly.sl_len = with_basis ? take((size_t)ly.L.nslices * sizeof(int32_t)) : take(0);
    ly.sl_ptr = with_basis ? take((size_t)ly.L.nslices * sizeof(int64_t)) : take(0);
    ly.bsum = with_basis ? take((size_t)sell_scan_blocks(ly.L.nslices) * sizeof(int64_t)) : take(0);
    ly.sl_col = with_basis ? take((size_t)ly.sell_capacity * sizeof(int32_t)) : take(0);
    ly.sl_val = with_basis ? take((size_t)ly.sell_capacity * wbytes(prec)) : take(0);
    ly.dict = with_basis ? take(sizeof(DictBuf)) : take(0);
    ly.chk = take((size_t)2 * m * d);
    ly.cnd = take((size_t)2 * (m + 1) * d);
    // SRDCT sketch: F_P (s x N) and the partial tiles of the contraction
    ly.srfp = (srdct && with_basis) ? take((size_t)s * N * d) : take(0);
    ly.srpart = (srdct && with_basis) ? take(srdct_part_doubles(s, N, m + 1) * d) : take(0);
    ly.SV = take((size_t)s * (m + 1) * d);
    ly.SAV = take((size_t)s * m * d);
    ly.Tws = take((size_t)QR_NB_HOST * QR_NB_HOST * d);
    ly.K0r = take((size_t)(m + 1) * m * d);
    ly.T1r = take((size_t)(m + 1) * m * d);
    ly.Hh = take((size_t)m * m * d);
    ly.Ubuf = take((size_t)NODE_SLOTS_HOST * m * m * d);
    ly.Urhs = take((size_t)NODE_SLOTS_HOST * m * d);
    ly.nodebuf = take((size_t)ly.lnodes * m * d);
    ly.qprev = take(m * d);
    ly.qcur = take(m * d);
    ly.y = take(m * d);
    ly.ys = take(m * d);
    ly.y0 = take(m * d);
    ly.poly = take((size_t)(npoly > 0 ? npoly : 1) * d);
    ly.expbuf = take((size_t)EXP_BUFS * m * m * d);
    ly.piv = take((size_t)m * sizeof(int));
    ly.norm1 = take(6 * d);
    ly.total = off;
    return ly;
}

struct Ptrs {
    DevCtrl* ctrl;
    void *U, *W;
    double *eta, *wnorm, *H, *gram, *colnorm2, *scal, *skpart, *SV, *SAV, *Tws, *K0r, *T1r, *Hh, *Ubuf, *Urhs,
        *nodebuf, *qprev, *qcur, *y, *ys, *y0, *poly, *expbuf, *norm1, *chk, *cnd, *srfp, *srpart;
    void* sl_val;
    DictBuf* dict;
    int* piv;
    int32_t *sl_len, *sl_col;
    int64_t *sl_ptr, *bsum;
};

Ptrs carve(void* ws, const Layout& ly) {
    char* b = static_cast<char*>(ws);
    Ptrs p;
    p.ctrl = reinterpret_cast<DevCtrl*>(b + ly.ctrl);
    auto D = [&](size_t o) { return reinterpret_cast<double*>(b + o); };
    p.eta = D(ly.eta); p.wnorm = D(ly.wnorm); p.H = D(ly.H); p.gram = D(ly.gram); p.colnorm2 = D(ly.colnorm2);
    p.scal = D(ly.scal); p.U = b + ly.U; p.W = b + ly.W; p.skpart = D(ly.skpart); p.SV = D(ly.SV); p.SAV = D(ly.SAV);
    p.Tws = D(ly.Tws); p.K0r = D(ly.K0r); p.T1r = D(ly.T1r); p.Hh = D(ly.Hh); p.Ubuf = D(ly.Ubuf);
    p.Urhs = D(ly.Urhs);
    p.nodebuf = D(ly.nodebuf); p.qprev = D(ly.qprev); p.qcur = D(ly.qcur); p.y = D(ly.y); p.ys = D(ly.ys);
    p.y0 = D(ly.y0); p.poly = D(ly.poly); p.expbuf = D(ly.expbuf); p.norm1 = D(ly.norm1);
    p.piv = reinterpret_cast<int*>(b + ly.piv);
    p.chk = D(ly.chk);
    p.cnd = D(ly.cnd);
    p.srfp = D(ly.srfp);
    p.srpart = D(ly.srpart);
    p.sl_val = b + ly.sl_val;
    p.dict = reinterpret_cast<DictBuf*>(b + ly.dict);
    p.sl_len = reinterpret_cast<int32_t*>(b + ly.sl_len);
    p.sl_col = reinterpret_cast<int32_t*>(b + ly.sl_col);
    p.sl_ptr = reinterpret_cast<int64_t*>(b + ly.sl_ptr);
    p.bsum = reinterpret_cast<int64_t*>(b + ly.bsum);
    return p;
}

void defaults(const skfab_params* p, int* l1, int* l2, int* lmax, double* tol) {
    *l1 = p->l1 > 0 ? p->l1 : 32;
    *l2 = p->l2 > 0 ? p->l2 : 45;
    *lmax = p->lmax > 0 ? p->lmax : 1395;
    *tol = p->quad_tol > 0.0 ? p->quad_tol : 1e-13;
}

bool zeta_ok(int z) { return z == 2 || z == 4 || z == 8 || z == 16; }

// Columns of the stored basis U: all m, or the k + 1 of the window (two-pass form).
int basis_columns(const skfab_params* p) {
    if (p->sketch == SKFAB_SKETCH_SRDCT) return p->m + 1;  // u_{m+1} kept for the sketch
    return p->two_pass ? p->k + 1 : p->m;
}

// Largest kappa_F of the basis prefix used (Section 2.1 remedy): the caller's, or the
// precision's default.
double cond_max_of(const skfab_params* p) {
    if (p->cond_max > 0.0) return p->cond_max;
    return p->prec == SKFAB_PREC_FP64 ? SKFAB_COND_MAX_FP64
                                      : (p->prec == SKFAB_PREC_FP32 ? SKFAB_COND_MAX_FP32 : SKFAB_COND_MAX_BF16);
}

skfab_status validate(const skfab_csr* A, const skfab_params* p, bool need_matrix) {
    if (!p) return SKFAB_ERR_ARG;
    if (need_matrix) {
        if (!A || !A->rowptr || !A->col || !A->val) return SKFAB_ERR_ARG;
        if (A->val_type != SKFAB_VAL_F64) return SKFAB_ERR_ARG;
        if (A->n <= 0 || A->nnz < 0 || A->nnz > INT32_MAX) return SKFAB_ERR_SHAPE;
    }
    if (p->f < 0 || p->f > 3 || p->method < 0 || p->method > 2) return SKFAB_ERR_ARG;
    if (p->prec < SKFAB_PREC_FP64 || p->prec > SKFAB_PREC_FP32_BF16BASIS) return SKFAB_ERR_ARG;
    if (!(p->cond_max == 0.0 || p->cond_max >= 1.0)) return SKFAB_ERR_ARG;
    if (p->two_pass != 0 && p->two_pass != 1) return SKFAB_ERR_ARG;
    if (p->sketch != SKFAB_SKETCH_SPARSE_SIGN && p->sketch != SKFAB_SKETCH_SRDCT) return SKFAB_ERR_ARG;
    if (p->sketch == SKFAB_SKETCH_SRDCT) {
        // the SRDCT sketch is applied to the stored basis: one pass only
        if (p->two_pass) return SKFAB_ERR_ARG;
        if (need_matrix && (!p->srdct_signs || !p->srdct_rows)) return SKFAB_ERR_ARG;
    }
    // reduced precisions are built for the default sketch density and k <= 4
    if (p->prec != SKFAB_PREC_FP64 && (p->zeta != 8 || p->k > 4)) return SKFAB_ERR_ARG;
    if (p->m < 1 || p->m > MMAX) return SKFAB_ERR_SHAPE;
    if (p->k < 1 || p->k > KMAX || p->k > p->m) return SKFAB_ERR_SHAPE;
    if (p->s <= p->m || p->s > SMAX) return SKFAB_ERR_SHAPE;
    if (need_matrix && p->s > A->n) return SKFAB_ERR_SHAPE;
    if (p->sketch == SKFAB_SKETCH_SPARSE_SIGN && (!zeta_ok(p->zeta) || p->zeta > p->s)) return SKFAB_ERR_SHAPE;
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    if (l1 < 1 || l2 <= l1 || lmax < l2) return SKFAB_ERR_ARG;
    if (p->f == SKFAB_F_POLY) {
        if (!p->poly || p->npoly < 1 || p->npoly > p->m) return SKFAB_ERR_ARG;
        if (p->method != SKFAB_SFOM_CLOSED) return SKFAB_ERR_ARG;
    }
    if (p->f == SKFAB_F_EXP) {
        if (!(p->fparam >= 0.0)) return SKFAB_ERR_ARG;
        if (p->method == SKFAB_SFOM_QUAD) return SKFAB_ERR_ARG;
        // sketched GMRES by the contour rule: tau > 0 (the integrand's decay), m <= CT_NMAX
        if (p->method == SKFAB_SGMRES_QUAD && (!(p->fparam > 0.0) || p->m > CT_NMAX)) return SKFAB_ERR_ARG;
    }
    return SKFAB_OK;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return SKFAB_ERR_HIP;     \
    } while (0)

// k-truncated Arnoldi with sketches, plus the extension vector u_m (Algorithm 2, basis part):
// arnoldi_setup (control block, SELL copy of A, step arguments), one arnoldi_step per
// j = 0..m (j = m forms the extension only), arnoldi_tail (its sketch and eta_m).
skfab_status arnoldi_setup(const skfab_csr* A, const double* b, const skfab_params* p, const Layout& ly,
                           const Ptrs& w, bool value_table, hipStream_t st, StepArgs* out) {
    const int m = p->m, s = p->s;
    HIP_TRY(launch_init_ctrl(w.ctrl, m, st));
    HIP_TRY(launch_sell_convert(A->rowptr, A->col, static_cast<const double*>(A->val), A->n, ly.L.nslices,
                                ly.sell_capacity, w.ctrl, w.sl_len, w.sl_ptr, w.bsum, w.sl_col, w.sl_val, w.dict,
                                (value_table && p->prec == SKFAB_PREC_FP64) ? 1 : 0, p->prec, st));
    StepArgs& a = *out;
    std::memset(&a, 0, sizeof(a));
    a.N = A->n;
    a.ldU = ly.ldU;
    a.rowptr = A->rowptr;
    a.col = A->col;
    a.val = static_cast<const double*>(A->val);
    a.sl_ptr = w.sl_ptr;
    a.sl_len = w.sl_len;
    a.sl_col = w.sl_col;
    a.sl_val = w.sl_val;
    a.sl_table = w.dict->table;
    a.nslices = ly.L.nslices;
    a.slices_per_chunk = ly.L.slices_per_chunk;
    a.rows_per_chunk = ly.L.rows_per_chunk;
    a.b = b;
    a.U = w.U;
    a.SV = w.SV;
    a.SAV = w.SAV;
    a.ctrl = w.ctrl;
    a.sctrl = w.ctrl;
    a.ldS = s;
    a.ldH = m + 1;
    a.eta = w.eta;
    a.wnorm = w.wnorm;
    a.H = w.H;
    a.gram = w.gram;
    a.seed = p->seed;
    a.inv_sqrt_zeta = 1.0 / std::sqrt((double)p->zeta);
    a.s = s;
    a.k = p->k;
    a.m = m;
    a.G = ly.L.G;
    a.uring = basis_columns(p);
    a.nosketch = p->sketch == SKFAB_SKETCH_SRDCT ? 1 : 0;
    a.keep_ext = a.nosketch;
    HIP_TRY(launch_fill(w.H, (int64_t)(m + 1) * m, 0.0, st));
    return SKFAB_OK;
}

// One step launch.  time_each: the launch is timed on its own (every stride-th);
// false inside a run that the caller times as a whole.
skfab_status arnoldi_step(skfab_ctx* ctx, StepArgs& a, const skfab_params* p, const Layout& ly, const Ptrs& w,
                          int j, hipStream_t st, bool time_each = true) {
    const int64_t nsc = (int64_t)NSC_MAX * ly.L.G;
    const int64_t nsk = (int64_t)2 * p->s * ly.L.G;
    a.j = j;
    a.extend = (j == p->m) ? 1 : 0;
    a.Wcur = static_cast<char*>(w.W) + (int64_t)(j & 1) * ly.ldU * wbytes(p->prec);
    a.Wprev = static_cast<char*>(w.W) + (int64_t)((j + 1) & 1) * ly.ldU * wbytes(p->prec);
    a.scal_prev = w.scal + ((j + 1) & 1) * nsc;
    a.scal_cur = w.scal + (j & 1) * nsc;
    a.skp_prev = w.skpart + ((j + 1) & 1) * nsk;
    a.skp_cur = w.skpart + (j & 1) * nsk;
    Span sp;
    const bool timed = time_each && j < p->m;  // the extension pass has no product with A
    if (timed) HIP_TRY(timing_begin(ctx, 0, st, &sp));
    HIP_TRY(launch_arnoldi_step(a, p->zeta, ly.L.block, p->prec, st));
    if (timed) HIP_TRY(timing_end(ctx, sp, st));
    return SKFAB_OK;
}

skfab_status arnoldi_tail(StepArgs& a, const skfab_params* p, const Layout& ly, const Ptrs& w, hipStream_t st) {
    const int m = p->m;
    a.scal_prev = w.scal + (m & 1) * (int64_t)NSC_MAX * ly.L.G;
    a.skp_prev = w.skpart + (m & 1) * (int64_t)2 * p->s * ly.L.G;
    HIP_TRY(launch_arnoldi_tail(a, w.colnorm2, st));
    return SKFAB_OK;
}

skfab_status run_arnoldi(skfab_ctx* ctx, const skfab_csr* A, const double* b, const skfab_params* p,
                         const Layout& ly, const Ptrs& w, hipStream_t st, StepArgs* out = nullptr,
                         bool sav = false) {
    StepArgs local;
    StepArgs& a = out ? *out : local;
    skfab_status r = arnoldi_setup(A, b, p, ly, w, ctx->value_table, st, &a);
    if (r != SKFAB_OK) return r;
    a.sav = sav ? 1 : 0;
    // steps 0 .. m-1 (each with its product by A) are timed as one run; the
    // extension pass j = m is not timed
    Span sp;
    HIP_TRY(timing_begin(ctx, 0, st, &sp, true));
    for (int j = 0; j < p->m; ++j) {
        r = arnoldi_step(ctx, a, p, ly, w, j, st, false);
        if (r != SKFAB_OK) {
            timing_cancel(ctx, sp);
            return r;
        }
    }
    HIP_TRY(timing_end(ctx, sp, st, p->m));
    r = arnoldi_step(ctx, a, p, ly, w, p->m, st, false);
    if (r != SKFAB_OK) return r;
    return arnoldi_tail(a, p, ly, w, st);
}

// y0 = exp(-tau H_hat) beta e_1 by [13/13] Pade scaling and squaring.  The powers
// A^2 .. A^6 are formed unscaled; their 1-norms come back to the host once and
// choose the number of squarings s from alpha(A) (see csrc/expm.hip); the powers
// are then scaled by 2^(-p s), exactly (powers of two).
skfab_status run_expm(const skfab_params* p, const Ptrs& w, hipStream_t st) {
    const int m = p->m, s = p->s;
    double* B[EXP_BUFS];
    for (int i = 0; i < EXP_BUFS; ++i) B[i] = w.expbuf + (size_t)i * m * m;
    double *A = B[0], *A2 = B[1], *A4 = B[2], *A6 = B[3], *T = B[4], *W1 = B[5], *U = B[6], *V = B[7], *Q = B[8],
           *X2 = B[9];
    HIP_TRY(launch_fill(w.norm1, 6, 0.0, st));
    HIP_TRY(launch_fill(w.y0, m, 0.0, st));
    HIP_TRY(launch_hhat(w.ctrl, m, w.T1r, w.SV, s, w.H, p->fparam, A, w.norm1, st));
    HIP_TRY(launch_dgemm(w.ctrl, m, A, A, 0.0, A2, st));
    HIP_TRY(launch_dgemm(w.ctrl, m, A, A2, 0.0, T, st));    // A^3
    HIP_TRY(launch_dgemm(w.ctrl, m, A2, A2, 0.0, A4, st));
    HIP_TRY(launch_dgemm(w.ctrl, m, A, A4, 0.0, W1, st));   // A^5
    HIP_TRY(launch_dgemm(w.ctrl, m, A4, A2, 0.0, A6, st));
    {
        const double* P[5] = {A2, T, A4, W1, A6};
        HIP_TRY(launch_norm1(w.ctrl, m, P, 5, w.norm1 + 1, st));
    }
    double nrm[6] = {0, 0, 0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(nrm, w.norm1, sizeof(nrm), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int q = 0; q < 6; ++q)
        if (!std::isfinite(nrm[q])) return SKFAB_OK;  // m_used == 0 or overflow: y0 stays as initialised
    // d_k = ||A^k||^(1/k); alpha = min over p = 1..5 of max(d_p, d_{p+1})
    double d[7];
    for (int k = 1; k <= 6; ++k) d[k] = std::pow(nrm[k - 1], 1.0 / k);
    double alpha = INFINITY;
    for (int q = 1; q <= 5; ++q) alpha = std::min(alpha, std::max(d[q], d[q + 1]));
    const double theta13 = 5.371920351148152;  // Higham (2005), Table 2.3
    int sq = 0;
    if (alpha > theta13) sq = (int)std::ceil(std::log2(alpha / theta13));
    if (sq > 0) {
        HIP_TRY(launch_combine(w.ctrl, m, std::ldexp(1.0, -sq), A, 0, nullptr, 0, nullptr, 0.0, A, st));
        HIP_TRY(launch_combine(w.ctrl, m, std::ldexp(1.0, -2 * sq), A2, 0, nullptr, 0, nullptr, 0.0, A2, st));
        HIP_TRY(launch_combine(w.ctrl, m, std::ldexp(1.0, -4 * sq), A4, 0, nullptr, 0, nullptr, 0.0, A4, st));
        HIP_TRY(launch_combine(w.ctrl, m, std::ldexp(1.0, -6 * sq), A6, 0, nullptr, 0, nullptr, 0.0, A6, st));
    }
    double c[14];
    c[0] = 1.0;
    for (int j = 0; j < 13; ++j) c[j + 1] = c[j] * (13.0 - j) / ((26.0 - j) * (j + 1.0));
    // U = A (A6 (c13 A6 + c11 A4 + c9 A2) + c7 A6 + c5 A4 + c3 A2 + c1 I)
    HIP_TRY(launch_combine(w.ctrl, m, c[13], A6, c[11], A4, c[9], A2, 0.0, T, st));
    HIP_TRY(launch_dgemm(w.ctrl, m, A6, T, 0.0, W1, st));
    HIP_TRY(launch_combine(w.ctrl, m, 1.0, W1, c[7], A6, c[5], A4, 0.0, W1, st));
    HIP_TRY(launch_combine(w.ctrl, m, 1.0, W1, c[3], A2, 0, nullptr, c[1], W1, st));
    HIP_TRY(launch_dgemm(w.ctrl, m, A, W1, 0.0, U, st));
    // V = A6 (c12 A6 + c10 A4 + c8 A2) + c6 A6 + c4 A4 + c2 A2 + c0 I
    HIP_TRY(launch_combine(w.ctrl, m, c[12], A6, c[10], A4, c[8], A2, 0.0, T, st));
    HIP_TRY(launch_dgemm(w.ctrl, m, A6, T, 0.0, V, st));
    HIP_TRY(launch_combine(w.ctrl, m, 1.0, V, c[6], A6, c[4], A4, 0.0, V, st));
    HIP_TRY(launch_combine(w.ctrl, m, 1.0, V, c[2], A2, 0, nullptr, c[0], V, st));
    // Q = V - U, P = V + U (into T); X = Q^-1 P
    HIP_TRY(launch_combine(w.ctrl, m, 1.0, V, -1.0, U, 0, nullptr, 0.0, Q, st));
    HIP_TRY(launch_combine(w.ctrl, m, 1.0, V, 1.0, U, 0, nullptr, 0.0, T, st));
    HIP_TRY(launch_lu(w.ctrl, m, Q, w.piv, st));
    HIP_TRY(launch_lu_solve_cols(w.ctrl, m, Q, w.piv, T, st));
    double* cur = T;
    double* nxt = X2;
    for (int i = 0; i < sq; ++i) {
        HIP_TRY(launch_dgemm(w.ctrl, m, cur, cur, 0.0, nxt, st));
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    HIP_TRY(launch_first_column(w.ctrl, cur, w.eta, w.y0, st));
    return SKFAB_OK;
}

// Small problem and coefficients y (unnormalised-basis coefficients in w.ys).
skfab_status run_small(const skfab_params* p, const Layout& ly, const Ptrs& w, hipStream_t st,
                       bool check = false) {
    const int m = p->m, s = p->s;
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    if (p->method == SKFAB_SFOM_CLOSED) tol = 1e-13;
    const bool ls = p->method == SKFAB_SGMRES_QUAD;
    if (check && p->sketch == SKFAB_SKETCH_SPARSE_SIGN)  // (the SRDCT path forms no S A V_m)
        HIP_TRY(launch_arnoldi_check(w.SV, w.SAV, w.H, s, m, p->k, w.ctrl, w.chk, st));
    HIP_TRY(launch_qr(w.SV, s, m + 1, w.ctrl, w.Tws, st));
    // Section 2.1 remedy: the longest basis prefix whose sketch is conditioned
    HIP_TRY(launch_cond_trunc(w.SV, s, m, w.ctrl, w.H, w.cnd, cond_max_of(p), st));
    HIP_TRY(launch_pencil_setup(w.SV, s, m, p->k, w.ctrl, w.H, w.K0r, w.T1r, st));
    HIP_TRY(launch_hhat_rows(w.ctrl, m, s, w.SV, w.T1r, w.H, w.Hh, st));
    const int branch = (p->f == SKFAB_F_INVSQRT && !ls) ? 1 : 0;
    // square system at t = 0: sigma, rcond, branch check; for 1/z with sFOM also the solution
    HIP_TRY(launch_pencil_scalars(m, s, w.SV, w.ctrl, w.eta, w.T1r, w.K0r, w.Hh, w.Ubuf, w.Urhs, w.y0, 0, branch,
                                  p->k, st));
    if (p->f == SKFAB_F_INV) {
        if (ls)
            HIP_TRY(launch_pencil_scalars(m, s, w.SV, w.ctrl, w.eta, w.T1r, w.K0r, w.Hh, w.Ubuf, w.Urhs, w.y0, 1, 0,
                                          p->k, st));
        HIP_TRY(launch_finish_coeffs(w.ctrl, m, w.y0, w.eta, w.colnorm2, w.ys, w.y, st));
        return SKFAB_OK;
    }
    if (p->f == SKFAB_F_POLY) {
        HIP_TRY(hipMemcpyAsync(w.poly, p->poly, sizeof(double) * p->npoly, hipMemcpyHostToDevice, st));
        HIP_TRY(launch_poly(w.ctrl, m, w.T1r, w.K0r, w.eta, w.poly, p->npoly, w.y0, st));
        HIP_TRY(launch_finish_coeffs(w.ctrl, m, w.y0, w.eta, w.colnorm2, w.ys, w.y, st));
        return SKFAB_OK;
    }
    if (p->f == SKFAB_F_EXP && ls) {
        // sketched GMRES by the contour rule (Sections 4.1, 5.2): Ritz values and the
        // parabola, then trapezoidal levels under the Section 4.1 test
        HIP_TRY(launch_contour_setup(w.ctrl, m, w.Hh, p->fparam, w.expbuf, st));
        for (const QuadGroup& g : contour_groups()) {
            HIP_TRY(launch_contour_level(w.ctrl, g, p->fparam, w.T1r, w.K0r, w.Ubuf, w.nodebuf, m, w.SV, w.eta, st));
            HIP_TRY(launch_quad_reduce(w.ctrl, g, w.nodebuf, m, tol, w.T1r, w.qprev, w.y0, st));
        }
        HIP_TRY(launch_quad_fail(w.ctrl, st));
        HIP_TRY(launch_finish_coeffs(w.ctrl, m, w.y0, w.eta, w.colnorm2, w.ys, w.y, st));
        return SKFAB_OK;
    }
    if (p->f == SKFAB_F_EXP) {
        skfab_status r = run_expm(p, w, st);
        if (r != SKFAB_OK) return r;
        HIP_TRY(launch_finish_coeffs(w.ctrl, m, w.y0, w.eta, w.colnorm2, w.ys, w.y, st));
        return SKFAB_OK;
    }
    // z^(-1/2): adaptive Gauss-Chebyshev (Section 4.1 / 5.1), orders evaluated in groups
    for (const QuadGroup& g : quad_groups(l1, l2, lmax)) {
        HIP_TRY(launch_quad_group(w.ctrl, g, w.T1r, w.K0r, w.Hh, w.Ubuf, w.Urhs, w.nodebuf, m, ls ? 1 : 0, w.SV,
                                  w.eta, p->k, st));
        HIP_TRY(launch_quad_reduce(w.ctrl, g, w.nodebuf, m, tol, w.T1r, w.qprev, w.y0, st));
    }
    HIP_TRY(launch_quad_fail(w.ctrl, st));
    HIP_TRY(launch_finish_coeffs(w.ctrl, m, w.y0, w.eta, w.colnorm2, w.ys, w.y, st));
    return SKFAB_OK;
}

// Storage form of A used by the step kernel (skfab_info.a_format).
int32_t a_format(const DevCtrl& c) { return c.sell_ok ? (c.col16 ? 2 : 1) | (c.dict8 ? 4 : 0) : 0; }

skfab_status solve_one(skfab_ctx* ctx, const skfab_csr* A, const double* b, double* x, const skfab_params* p,
                       void* ws, size_t ws_bytes, skfab_info* info);
bool multi_rhs_batched(const skfab_params* p, int nrhs);
skfab_batch_problem one_problem(const skfab_csr* A, const double* b, int64_t ldb, double* x, int64_t ldx,
                                const skfab_params* p);
size_t batch_ws_total(int32_t nprob, const skfab_batch_problem* probs, int32_t nrhs, const skfab_params* p);

// skfab_info from a control block (a_format from the control block of the SELL copy).
void ctrl_to_info(const DevCtrl& c, int32_t aformat, skfab_info* o) {
    o->status = c.status;
    o->m_used = c.m_used;
    o->l_used = c.l_used;
    o->a_format = aformat;
    o->eps_est = c.eps_est;
    o->rcond_R = c.rcond;
    o->sigma = c.sigma;
    o->beta = c.beta;
    o->arnoldi_relres = c.relres;
    o->quad_diff = c.quad_diff;
    o->flags = c.flags;
    o->m_basis = c.m_basis;
}

skfab_status read_info(const Ptrs& w, hipStream_t st, skfab_info* info) {
    if (!info) return SKFAB_OK;
    DevCtrl c;
    HIP_TRY(hipMemcpyAsync(&c, w.ctrl, sizeof(DevCtrl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    ctrl_to_info(c, a_format(c), info);
    return SKFAB_OK;
}

}  // namespace

extern "C" {

int32_t skfab_version(void) { return SKFAB_VERSION_MAJOR * 100 + SKFAB_VERSION_MINOR; }

const char* skfab_status_string(int32_t s) {
    switch (s) {
        case SKFAB_OK: return "ok";
        case SKFAB_ERR_ARG: return "invalid argument";
        case SKFAB_ERR_SHAPE: return "invalid shape (need 1 <= k <= min(m,8), m < s <= min(N,1024), m <= 512)";
        case SKFAB_ERR_RANK: return "sketched basis numerically rank deficient";
        case SKFAB_ERR_BRANCH: return "projected matrix has an eigenvalue on the branch cut";
        case SKFAB_ERR_QUAD: return "adaptive quadrature did not converge";
        case SKFAB_ERR_HIP: return "HIP runtime error";
        case SKFAB_ERR_WORKSPACE: return "workspace missing or too small";
        case SKFAB_ERR_TOO_LARGE: return "problem needs more workspace than skfab_solve_noalloc's static buffer";
        default: return "unknown status";
    }
}

skfab_status skfab_create(skfab_ctx** ctx, int32_t device, void* hip_stream) {
    if (!ctx) return SKFAB_ERR_ARG;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return SKFAB_ERR_HIP;
    if (device < 0 || device >= n) return SKFAB_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return SKFAB_ERR_HIP;
    skfab_ctx* c = new (std::nothrow) skfab_ctx;
    if (!c) return SKFAB_ERR_ARG;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    // the device address of skfab_solve_noalloc's static workspace, once per device
    const skfab_status st = skfab::noalloc_init_device(device);
    if (st != SKFAB_OK) {
        delete c;
        return st;
    }
    *ctx = c;
    return SKFAB_OK;
}

skfab_status skfab_set_stream(skfab_ctx* ctx, void* hip_stream) {
    if (!ctx) return SKFAB_ERR_ARG;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return SKFAB_OK;
}

skfab_status skfab_destroy(skfab_ctx* ctx) {
    if (ctx) {
        for (int c = 0; c < 2; ++c)
            for (hipEvent_t e : ctx->ev[c]) (void)hipEventDestroy(e);
    }
    delete ctx;
    return SKFAB_OK;
}

skfab_status skfab_timing_enable(skfab_ctx* ctx, int32_t enable) {
    if (!ctx || enable < 0) return SKFAB_ERR_ARG;
    if (enable && ctx->ev[0].empty()) {
        if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
        for (int c = 0; c < 2; ++c) {
            ctx->ev[c].resize(2 * TIMING_PAIRS);
            ctx->nl[c].assign(TIMING_PAIRS, 1);
            for (auto& e : ctx->ev[c]) HIP_TRY(hipEventCreate(&e));
        }
    }
    if (!enable && ctx->timing) {
        for (int c = 0; c < 2; ++c) HIP_TRY(timing_flush(ctx, c));
    }
    ctx->timing = enable != 0;
    ctx->stride = enable > 0 ? enable : 1;
    ctx->tick[0] = ctx->tick[1] = 0;
    return SKFAB_OK;
}

skfab_status skfab_timing_read(skfab_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches) {
    if (!ctx || kernel < 0 || kernel > 1 || !total_ms || !launches) return SKFAB_ERR_ARG;
    HIP_TRY(timing_flush(ctx, kernel));
    *total_ms = ctx->acc_ms[kernel];
    *launches = ctx->count[kernel];
    ctx->acc_ms[kernel] = 0.0;
    ctx->count[kernel] = 0;
    return SKFAB_OK;
}

skfab_status skfab_workspace_bytes(const skfab_csr* A, const skfab_params* p, int32_t nrhs, size_t* bytes) {
    if (!bytes || !A || !p || nrhs < 1) return SKFAB_ERR_ARG;
    skfab_status v = validate(A, p, false);
    if (v != SKFAB_OK) return v;
    if (A->n <= 0) return SKFAB_ERR_SHAPE;
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    size_t total = make_layout(A->n, A->nnz, p->m, p->s, l1, l2, lmax, p->npoly, true, p->prec, p->k,
                               basis_columns(p), p->sketch == SKFAB_SKETCH_SRDCT).total;
    if (nrhs > 1 && multi_rhs_batched(p, nrhs)) {
        const skfab_batch_problem q = one_problem(A, nullptr, 0, nullptr, 0, p);
        const size_t tb = batch_ws_total(1, &q, nrhs, p);
        total = tb > total ? tb : total;
    }
    *bytes = total;
    return SKFAB_OK;
}

skfab_status skfab_solve(skfab_ctx* ctx, const skfab_csr* A, const double* b, int64_t ldb, int32_t nrhs, double* x,
                         int64_t ldx, const skfab_params* p, void* ws, size_t ws_bytes, skfab_info* info) {
    if (!ctx || !b || !x || !A || nrhs < 1) return SKFAB_ERR_ARG;
    if (nrhs > 1 && (ldb < A->n || ldx < A->n)) return SKFAB_ERR_SHAPE;
    if (nrhs == 1) return solve_one(ctx, A, b, x, p, ws, ws_bytes, info);
    skfab_status v = validate(A, p, true);
    if (v != SKFAB_OK) return v;
    if (multi_rhs_batched(p, nrhs)) {
        // one problem with nrhs right-hand sides: the batched form, whose step launch
        // serves every column from the same rows of A
        const skfab_batch_problem q = one_problem(A, b, ldb, x, ldx, p);
        return skfab_solve_batched(ctx, 1, &q, nrhs, p, ws, ws_bytes, info);
    }
    // other functions / shapes: the columns one after another in the same workspace
    for (int r = 0; r < nrhs; ++r) {
        v = solve_one(ctx, A, b + (int64_t)r * ldb, x + (int64_t)r * ldx, p, ws, ws_bytes, info ? info + r : nullptr);
        if (v != SKFAB_OK) return v;
    }
    return SKFAB_OK;
}

skfab_status skfab_solve_reckless(skfab_ctx* ctx, const skfab_csr* A, const double* b, double* x,
                                  const skfab_params* p, int32_t s_max, double eps_max, void* ws, size_t ws_bytes,
                                  skfab_info* info, int32_t* s_used) {
    if (!ctx || !A || !b || !x || !p || !info) return SKFAB_ERR_ARG;
    if (!(eps_max > 0.0) || s_max < p->s || p->two_pass || p->sketch != SKFAB_SKETCH_SPARSE_SIGN) return SKFAB_ERR_ARG;
    skfab_params q = *p;
    q.s = s_max;  // the largest attempt must fit (shape and workspace) before the first runs
    skfab_status v = validate(A, &q, true);
    if (v != SKFAB_OK) return v;
    size_t need = 0;
    v = skfab_workspace_bytes(A, &q, 1, &need);
    if (v != SKFAB_OK) return v;
    if (!ws || ws_bytes < need) return SKFAB_ERR_WORKSPACE;
    int32_t s = p->s;
    for (;;) {
        q.s = s;
        v = solve_one(ctx, A, b, x, &q, ws, ws_bytes, info);
        if (v != SKFAB_OK) return v;
        const bool ok = info->status == SKFAB_OK && info->eps_est <= eps_max;
        if (ok || s >= s_max) break;
        s = (2 * (int64_t)s < s_max) ? 2 * s : s_max;
    }
    if (s_used) *s_used = s;
    return SKFAB_OK;
}

}  // extern "C"

namespace {

skfab_status solve_one(skfab_ctx* ctx, const skfab_csr* A, const double* b, double* x, const skfab_params* p,
                       void* ws, size_t ws_bytes, skfab_info* info) {
    if (!ctx || !b || !x) return SKFAB_ERR_ARG;
    skfab_status v = validate(A, p, true);
    if (v != SKFAB_OK) return v;
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    const Layout ly = make_layout(A->n, A->nnz, p->m, p->s, l1, l2, lmax, p->npoly, true, p->prec, p->k,
                                  basis_columns(p), p->sketch == SKFAB_SKETCH_SRDCT);
    if (!ws || ws_bytes < ly.total || (reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    const Ptrs w = carve(ws, ly);
    hipStream_t st = ctx->stream;
    const bool srdct = p->sketch == SKFAB_SKETCH_SRDCT;
    if (srdct) HIP_TRY(launch_srdct_matrix(p->s, A->n, p->srdct_signs, p->srdct_rows, w.srfp, st));
    StepArgs a;
    skfab_status r = run_arnoldi(ctx, A, b, p, ly, w, st, &a, ctx->arnoldi_check);
    if (r != SKFAB_OK) return r;
    if (srdct) {
        // [S v_1 .. S v_m, S u_{m+1}]: the stored basis times F_P (FP64 matrix cores)
        HIP_TRY(launch_srdct_sketch(w.srfp, p->s, A->n, w.U, ly.ldU, p->m + 1, p->prec, w.srpart, w.ctrl, w.eta,
                                    w.SV, p->s, st));
        HIP_TRY(launch_colnorm(w.SV, p->s, p->m, w.ctrl, w.colnorm2, st));
    }
    r = run_small(p, ly, w, st, ctx->arnoldi_check);
    if (r != SKFAB_OK) return r;
    if (p->two_pass) {
        // Section 4.2, second pass: the same step launches regenerate u_0 .. u_{m-1}
        // (bitwise: every sum has a fixed order), each added to x as it appears
        const size_t vb = vbytes(p->prec);
        for (int j = 0; j < p->m; ++j) {
            r = arnoldi_step(ctx, a, p, ly, w, j, st);
            if (r != SKFAB_OK) return r;
            const char* uj = static_cast<const char*>(w.U) + (size_t)(j % (p->k + 1)) * ly.ldU * vb;
            HIP_TRY(launch_accum_basis(uj, A->n, j, w.ctrl, w.ys, x, p->prec, st));
        }
        return read_info(w, st, info);
    }
    Span sp;
    HIP_TRY(timing_begin(ctx, 1, st, &sp));
    HIP_TRY(launch_assemble(w.U, ly.ldU, A->n, p->m, w.ctrl, w.ys, x, p->prec, st));
    HIP_TRY(timing_end(ctx, sp, st));
    return read_info(w, st, info);
}

}  // namespace

extern "C" {

skfab_status skfab_arnoldi(skfab_ctx* ctx, const skfab_csr* A, const double* b, const skfab_params* p, double* V,
                           double* SV, double* SAV, double* H, void* ws, size_t ws_bytes, skfab_info* info) {
    if (!ctx || !b) return SKFAB_ERR_ARG;
    skfab_status v = validate(A, p, true);
    if (v == SKFAB_ERR_ARG && p && p->f == SKFAB_F_EXP) v = SKFAB_OK;  // the basis does not depend on f
    if (v != SKFAB_OK) return v;
    if (p->two_pass || p->sketch != SKFAB_SKETCH_SPARSE_SIGN) return SKFAB_ERR_ARG;  // hook of the fused sketch
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    const Layout ly = make_layout(A->n, A->nnz, p->m, p->s, l1, l2, lmax, p->npoly, true, p->prec, p->k);
    if (!ws || ws_bytes < ly.total || (reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    const Ptrs w = carve(ws, ly);
    hipStream_t st = ctx->stream;
    skfab_status r = run_arnoldi(ctx, A, b, p, ly, w, st, nullptr, true);  // SAV is exported
    if (r != SKFAB_OK) return r;
    const int m = p->m, s = p->s;
    if (V) HIP_TRY(launch_normalize_basis(w.U, ly.ldU, A->n, m, w.ctrl, w.eta, V, p->prec, st));
    if (SV) HIP_TRY(hipMemcpyAsync(SV, w.SV, sizeof(double) * s * m, hipMemcpyDeviceToDevice, st));
    if (SAV) HIP_TRY(hipMemcpyAsync(SAV, w.SAV, sizeof(double) * s * m, hipMemcpyDeviceToDevice, st));
    if (H) HIP_TRY(hipMemcpyAsync(H, w.H, sizeof(double) * (m + 1) * m, hipMemcpyDeviceToDevice, st));
    if (info) {
        HIP_TRY(launch_finish_coeffs(w.ctrl, m, w.y, w.eta, w.colnorm2, w.ys, nullptr, st));
        return read_info(w, st, info);
    }
    return SKFAB_OK;
}

skfab_status skfab_small_workspace_bytes(const skfab_params* p, size_t* bytes) {
    if (!bytes || !p) return SKFAB_ERR_ARG;
    skfab_status v = validate(nullptr, p, false);
    if (v != SKFAB_OK) return v;
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    *bytes = make_layout(0, 0, p->m, p->s, l1, l2, lmax, p->npoly, false, 0).total;
    return SKFAB_OK;
}

skfab_status skfab_small_problem(skfab_ctx* ctx, const double* SVext, const double* Hbar, double beta,
                                 const skfab_params* p, double* y, void* ws, size_t ws_bytes, skfab_info* info) {
    if (!ctx || !SVext || !Hbar || !y) return SKFAB_ERR_ARG;
    skfab_status v = validate(nullptr, p, false);
    if (v != SKFAB_OK) return v;
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    const Layout ly = make_layout(0, 0, p->m, p->s, l1, l2, lmax, p->npoly, false, 0);
    if (!ws || ws_bytes < ly.total || (reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    const Ptrs w = carve(ws, ly);
    hipStream_t st = ctx->stream;
    const int m = p->m, s = p->s;
    HIP_TRY(launch_init_ctrl(w.ctrl, m, st));
    // the caller's basis is normalised: eta = 1 except eta[0] = beta (used for S b = beta S v_1)
    HIP_TRY(launch_fill(w.eta, m + 2, 1.0, st));
    HIP_TRY(hipMemcpyAsync(w.eta, &beta, sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w.SV, SVext, sizeof(double) * s * (m + 1), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(w.H, Hbar, sizeof(double) * (m + 1) * m, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_fill(w.colnorm2, m + 1, 1.0, st));
    // SAV is not an input here: the Arnoldi-relation check is skipped (relres = 0)
    HIP_TRY(launch_fill(w.SAV, (int64_t)s * m, 0.0, st));
    skfab_params q = *p;
    skfab_status r = run_small(&q, ly, w, st, true);  // the caller supplies S A V_m
    if (r != SKFAB_OK) return r;
    // run_small leaves y / eta in ys; with eta_j = 1 for j >= 1 only ys[0] differs
    HIP_TRY(hipMemcpyAsync(y, w.y, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    return read_info(w, st, info);
}

skfab_status skfab_sketch_pattern(skfab_ctx* ctx, int64_t col0, int64_t ncols, int32_t s, int32_t zeta,
                                  uint64_t seed, int32_t* rows, int8_t* signs) {
    if (!ctx || !rows || !signs || col0 < 0 || ncols < 0) return SKFAB_ERR_ARG;
    if (!zeta_ok(zeta) || zeta > s || s < 1) return SKFAB_ERR_SHAPE;
    if (ncols == 0) return SKFAB_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    HIP_TRY(launch_sketch_pattern(col0, ncols, s, zeta, seed, rows, signs, ctx->stream));
    return SKFAB_OK;
}

size_t skfab_sketch_ws_bytes(int64_t n, int32_t s) {
    if (n <= 0 || s <= 0) return 0;
    return (size_t)sketch_apply_blocks(n) * s * sizeof(double);
}

skfab_status skfab_sketch_apply(skfab_ctx* ctx, int64_t n, int32_t s, int32_t zeta, uint64_t seed, const double* v,
                                double* Sv, void* ws, size_t ws_bytes) {
    if (!ctx || !v || !Sv || n <= 0) return SKFAB_ERR_ARG;
    if (!zeta_ok(zeta) || zeta > s || s < 1 || s > SMAX) return SKFAB_ERR_SHAPE;
    if (!ws || ws_bytes < skfab_sketch_ws_bytes(n, s)) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    HIP_TRY(launch_sketch_apply(n, s, zeta, seed, v, Sv, static_cast<double*>(ws), ctx->stream));
    return SKFAB_OK;
}

}  // extern "C"

// ===================================================================== batch
namespace {

constexpr int BATCH_MAX_PROBLEMS = 4096;
constexpr int BATCH_MAX_RHS = 4;
constexpr int BATCH_GMAX = 256;     // step-kernel blocks per (problem, rhs) at most
static_assert(BATCH_GMAX <= STEP_GMAX_1024, "the step kernel reduces at most STEP_GMAX_1024 * 1024 / block partials");
constexpr int BATCH_SLOTS = 128;    // quadrature scratch slots per unit

struct BatchProbLayout {
    int64_t N, nnz, ldU, nslices, capacity;
    size_t sl_len, sl_ptr, bsum, sl_col, sl_val, dict;
};

struct BatchUnitLayout {
    size_t U, W, scal, skp, small, ubuf, nodebuf;
};

struct BatchLayout {
    int nprob, R, nunits, mmax, smax, lnodes;
    int64_t nmax;
    std::vector<int> order;            // problems by decreasing m (stable)
    std::vector<BatchProbLayout> prob; // indexed by original problem
    std::vector<BatchUnitLayout> unit; // indexed by sorted position * R + r
    size_t ctrl, steps, smalls, base;  // ctrl array, descriptor arrays, base[nprob+1]
    size_t small_begin, small_end;     // contiguous per-unit small region (zero-filled per call)
    size_t small_bytes;                // bytes of one unit's small block
    // offsets inside one unit's small block
    size_t o_eta, o_wnorm, o_H, o_gram, o_colnorm2, o_chk, o_cnd, o_SV, o_SAV, o_Tws, o_K0r, o_T1r, o_Hh, o_Urhs, o_qprev, o_y,
        o_ys, o_y0;
    size_t total;
};

skfab_status validate_batch(int32_t nprob, const skfab_batch_problem* probs, int32_t nrhs, const skfab_params* p,
                            bool need_data) {
    if (!probs || !p || nprob < 1 || nprob > BATCH_MAX_PROBLEMS) return SKFAB_ERR_ARG;
    if (nrhs < 1 || nrhs > BATCH_MAX_RHS) return SKFAB_ERR_ARG;
    if (p->f != SKFAB_F_INVSQRT && p->f != SKFAB_F_INV) return SKFAB_ERR_ARG;
    if (p->method < 0 || p->method > 2) return SKFAB_ERR_ARG;
    if (p->prec < SKFAB_PREC_FP64 || p->prec > SKFAB_PREC_FP32_BF16BASIS) return SKFAB_ERR_ARG;
    if (!(p->cond_max == 0.0 || p->cond_max >= 1.0)) return SKFAB_ERR_ARG;
    if (p->two_pass) return SKFAB_ERR_ARG;  // the batched form keeps every basis
    if (p->sketch != SKFAB_SKETCH_SPARSE_SIGN) return SKFAB_ERR_ARG;
    if (p->zeta != 8 || p->k < 1 || p->k > 4) return SKFAB_ERR_ARG;
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    if (l1 < 1 || l2 <= l1 || lmax < l2) return SKFAB_ERR_ARG;
    for (int i = 0; i < nprob; ++i) {
        const skfab_batch_problem& q = probs[i];
        if (need_data && (!q.A.rowptr || !q.A.col || !q.A.val || !q.B || !q.X)) return SKFAB_ERR_ARG;
        if (q.A.val_type != SKFAB_VAL_F64) return SKFAB_ERR_ARG;
        if (q.A.n <= 0 || q.A.nnz < 0 || q.A.nnz > INT32_MAX) return SKFAB_ERR_SHAPE;
        if (q.m < 1 || q.m > MMAX) return SKFAB_ERR_SHAPE;
        if (p->k > q.m) return SKFAB_ERR_SHAPE;
        if (q.s <= q.m || q.s > SMAX || q.s > q.A.n) return SKFAB_ERR_SHAPE;
        if ((q.ldb != 0 && q.ldb < q.A.n) || (q.ldx != 0 && q.ldx < q.A.n)) return SKFAB_ERR_SHAPE;
    }
    return SKFAB_OK;
}

// Multi-RHS solves of skfab_solve go through the batched form when it covers them.
bool multi_rhs_batched(const skfab_params* p, int nrhs) {
    return nrhs >= 1 && nrhs <= BATCH_MAX_RHS && !p->two_pass && p->sketch == SKFAB_SKETCH_SPARSE_SIGN &&
           (p->f == SKFAB_F_INVSQRT || p->f == SKFAB_F_INV) &&
           p->zeta == 8 && p->k >= 1 && p->k <= 4;
}

skfab_batch_problem one_problem(const skfab_csr* A, const double* b, int64_t ldb, double* x, int64_t ldx,
                                const skfab_params* p) {
    skfab_batch_problem q;
    std::memset(&q, 0, sizeof(q));
    q.A = *A;
    q.B = b;
    q.X = x;
    q.m = p->m;
    q.s = p->s;
    q.seed = p->seed;
    q.ldb = ldb;
    q.ldx = ldx;
    return q;
}

BatchLayout make_batch_layout(int32_t nprob, const skfab_batch_problem* probs, int32_t R, const skfab_params* p) {
    BatchLayout L;
    L.nprob = nprob;
    L.R = R;
    L.nunits = nprob * R;
    L.mmax = 0;
    L.smax = 0;
    L.nmax = 0;
    for (int i = 0; i < nprob; ++i) {
        L.mmax = probs[i].m > L.mmax ? probs[i].m : L.mmax;
        L.smax = probs[i].s > L.smax ? probs[i].s : L.smax;
        L.nmax = probs[i].A.n > L.nmax ? probs[i].A.n : L.nmax;
    }
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    L.lnodes = max_level_nodes(l1, l2, lmax);
    L.order.resize(nprob);
    for (int i = 0; i < nprob; ++i) L.order[i] = i;
    std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) { return probs[a].m > probs[b].m; });
    const size_t d = sizeof(double);
    const int mmax = L.mmax, smax = L.smax;
    // one unit's small block
    size_t o = 0;
    auto sub = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    L.o_eta = sub((mmax + 2) * d);
    L.o_wnorm = sub((mmax + 2) * d);
    L.o_H = sub((size_t)(mmax + 1) * mmax * d);
    L.o_gram = sub((size_t)(mmax + 1) * KMAX * d);
    L.o_colnorm2 = sub((mmax + 1) * d);
    L.o_chk = sub((size_t)2 * mmax * d);
    L.o_cnd = sub((size_t)2 * (mmax + 1) * d);
    L.o_SV = sub((size_t)smax * (mmax + 1) * d);
    L.o_SAV = sub((size_t)smax * mmax * d);
    L.o_Tws = sub((size_t)QR_NB_HOST * QR_NB_HOST * d);
    L.o_K0r = sub((size_t)(mmax + 1) * mmax * d);
    L.o_T1r = sub((size_t)(mmax + 1) * mmax * d);
    L.o_Hh = sub((size_t)mmax * mmax * d);
    L.o_Urhs = sub((size_t)BATCH_SLOTS * mmax * d);
    L.o_qprev = sub(mmax * d);
    L.o_y = sub(mmax * d);
    L.o_ys = sub(mmax * d);
    L.o_y0 = sub(mmax * d);
    L.small_bytes = o;

    size_t off = 0;
    auto take = [&](size_t bytes) { size_t r = off; off = align_up(off + bytes); return r; };
    L.ctrl = take((size_t)L.nunits * sizeof(DevCtrl));
    L.steps = take((size_t)L.nunits * sizeof(BatchStepUnit));
    L.smalls = take((size_t)L.nunits * sizeof(SmallUnit));
    L.base = take((size_t)(nprob + 1) * sizeof(int));
    L.prob.resize(nprob);
    for (int i = 0; i < nprob; ++i) {
        BatchProbLayout& q = L.prob[i];
        q.N = probs[i].A.n;
        q.nnz = probs[i].A.nnz;
        q.ldU = (q.N + 63) / 64 * 64;
        q.nslices = (q.N + 63) / 64;
        q.capacity = q.nnz + q.nnz / 4 + 64 * q.nslices;
        q.sl_len = take((size_t)q.nslices * sizeof(int32_t));
        q.sl_ptr = take((size_t)q.nslices * sizeof(int64_t));
        q.bsum = take((size_t)sell_scan_blocks(q.nslices) * sizeof(int64_t));
        q.sl_col = take((size_t)q.capacity * sizeof(int32_t));
        q.sl_val = take((size_t)q.capacity * wbytes(p->prec));
        q.dict = take(sizeof(DictBuf));
    }
    L.unit.resize(L.nunits);
    for (int qi = 0; qi < nprob; ++qi) {
        const int pi = L.order[qi];
        const BatchProbLayout& q = L.prob[pi];
        for (int r = 0; r < R; ++r) {
            BatchUnitLayout& u = L.unit[qi * R + r];
            u.U = take((size_t)q.ldU * probs[pi].m * vbytes(p->prec));
            u.W = take((size_t)2 * q.ldU * wbytes(p->prec));
            u.scal = take((size_t)2 * NSC_MAX * BATCH_GMAX * d);
            u.skp = take((size_t)2 * BATCH_GMAX * 2 * probs[pi].s * d);
        }
    }
    L.small_begin = off;
    for (int u = 0; u < L.nunits; ++u) L.unit[u].small = take(L.small_bytes);
    L.small_end = off;
    for (int u = 0; u < L.nunits; ++u) {
        L.unit[u].ubuf = take((size_t)BATCH_SLOTS * mmax * mmax * d);
        L.unit[u].nodebuf = take((size_t)L.lnodes * mmax * d);
    }
    L.total = off;
    return L;
}

size_t batch_ws_total(int32_t nprob, const skfab_batch_problem* probs, int32_t nrhs, const skfab_params* p) {
    return make_batch_layout(nprob, probs, nrhs, p).total;
}

// Step-kernel blocks of a problem with `nslices` SELL slices: about `spw` slices per
// wavefront, a multiple of 8 (whole XCD groups), at most BATCH_GMAX.
int batch_blocks(int64_t nslices, int block, int spw) {
    const int64_t per_block = (int64_t)(block / WAVE) * spw;
    int64_t G = (nslices + per_block - 1) / per_block;
    if (G > BATCH_GMAX) G = BATCH_GMAX;
    G = (G + 7) / 8 * 8;
    return (int)G;
}

struct BatchPlan {
    std::vector<int> G;     // by sorted position
    std::vector<int> base;  // [nprob + 1], sorted order
};

BatchPlan batch_plan(const BatchLayout& L, int block, int spw) {
    BatchPlan P;
    P.G.resize(L.nprob);
    P.base.resize(L.nprob + 1);
    P.base[0] = 0;
    for (int qi = 0; qi < L.nprob; ++qi) {
        P.G[qi] = batch_blocks(L.prob[L.order[qi]].nslices, block, spw);
        P.base[qi + 1] = P.base[qi] + L.R * P.G[qi];
    }
    return P;
}

// Host images of the unit descriptors and the base table, for a launch plan.
void batch_descriptors(const BatchLayout& L, const BatchPlan& P, const skfab_batch_problem* probs,
                       const skfab_params* p, char* dev, std::vector<char>& host, bool sav) {
    host.assign(L.base + (size_t)(L.nprob + 1) * sizeof(int), 0);
    BatchStepUnit* su = reinterpret_cast<BatchStepUnit*>(host.data() + L.steps);
    SmallUnit* sm = reinterpret_cast<SmallUnit*>(host.data() + L.smalls);
    int* base = reinterpret_cast<int*>(host.data() + L.base);
    DevCtrl* ctrl = reinterpret_cast<DevCtrl*>(dev + L.ctrl);
    for (int qi = 0; qi < L.nprob; ++qi) {
        const int pi = L.order[qi];
        const skfab_batch_problem& q = probs[pi];
        const BatchProbLayout& ql = L.prob[pi];
        for (int r = 0; r < L.R; ++r) {
            const int u = qi * L.R + r;
            const BatchUnitLayout& ul = L.unit[u];
            char* sb = dev + ul.small;
            StepArgs a;
            std::memset(&a, 0, sizeof(a));
            a.N = ql.N;
            a.ldU = ql.ldU;
            a.rowptr = q.A.rowptr;
            a.col = q.A.col;
            a.val = static_cast<const double*>(q.A.val);
            a.sl_ptr = reinterpret_cast<const int64_t*>(dev + ql.sl_ptr);
            a.sl_len = reinterpret_cast<const int32_t*>(dev + ql.sl_len);
            a.sl_col = reinterpret_cast<const int32_t*>(dev + ql.sl_col);
            a.sl_val = dev + ql.sl_val;
            a.sl_table = reinterpret_cast<const DictBuf*>(dev + ql.dict)->table;
            a.nslices = ql.nslices;
            a.slices_per_chunk = (ql.nslices + P.G[qi] - 1) / P.G[qi];
            a.rows_per_chunk = (ql.N + P.G[qi] - 1) / P.G[qi];
            a.b = q.B + (int64_t)r * (q.ldb > 0 ? q.ldb : ql.N);
            a.U = dev + ul.U;
            a.SV = reinterpret_cast<double*>(sb + L.o_SV);
            a.SAV = reinterpret_cast<double*>(sb + L.o_SAV);
            a.sav = sav ? 1 : 0;
            a.ctrl = ctrl + u;
            a.sctrl = ctrl + qi * L.R;  // the SELL copy is converted once per problem
            a.eta = reinterpret_cast<double*>(sb + L.o_eta);
            a.wnorm = reinterpret_cast<double*>(sb + L.o_wnorm);
            a.H = reinterpret_cast<double*>(sb + L.o_H);
            a.gram = reinterpret_cast<double*>(sb + L.o_gram);
            a.ldS = L.smax;
            a.ldH = L.mmax + 1;
            a.seed = q.seed;
            a.inv_sqrt_zeta = 1.0 / std::sqrt((double)p->zeta);
            a.s = q.s;
            a.k = p->k;
            a.m = q.m;
            a.uring = q.m;
            a.G = P.G[qi];
            BatchStepUnit& b = su[u];
            b.a = a;
            const size_t wb = (size_t)ql.ldU * wbytes(p->prec);
            b.W[0] = dev + ul.W;
            b.W[1] = dev + ul.W + wb;
            b.scal[0] = reinterpret_cast<double*>(dev + ul.scal);
            b.scal[1] = b.scal[0] + (size_t)NSC_MAX * BATCH_GMAX;
            b.skp[0] = reinterpret_cast<double*>(dev + ul.skp);
            b.skp[1] = b.skp[0] + (size_t)BATCH_GMAX * 2 * q.s;
            SmallUnit& m = sm[u];
            m.ctrl = ctrl + u;
            m.SV = a.SV;
            m.SAV = a.SAV;
            m.H = a.H;
            m.eta = a.eta;
            m.colnorm2 = reinterpret_cast<double*>(sb + L.o_colnorm2);
            m.chk = reinterpret_cast<double*>(sb + L.o_chk);
            m.cnd = reinterpret_cast<double*>(sb + L.o_cnd);
            m.Tws = reinterpret_cast<double*>(sb + L.o_Tws);
            m.K0r = reinterpret_cast<double*>(sb + L.o_K0r);
            m.T1r = reinterpret_cast<double*>(sb + L.o_T1r);
            m.Hh = reinterpret_cast<double*>(sb + L.o_Hh);
            m.Ubuf = reinterpret_cast<double*>(dev + ul.ubuf);
            m.Urhs = reinterpret_cast<double*>(sb + L.o_Urhs);
            m.nodebuf = reinterpret_cast<double*>(dev + ul.nodebuf);
            m.qprev = reinterpret_cast<double*>(sb + L.o_qprev);
            m.y0 = reinterpret_cast<double*>(sb + L.o_y0);
            m.ys = reinterpret_cast<double*>(sb + L.o_ys);
            m.y = reinterpret_cast<double*>(sb + L.o_y);
            m.U = a.U;
            m.ldU = ql.ldU;
            m.N = ql.N;
            m.x = q.X + (int64_t)r * (q.ldx > 0 ? q.ldx : ql.N);
            m.m = q.m;
            m.pad = 0;
        }
    }
    for (int qi = 0; qi <= L.nprob; ++qi) base[qi] = P.base[qi];
}

// Arnoldi part of a batch: control blocks, SELL copies, then one launch per step j
// over every (problem, rhs) with m_p >= j (the last is the extension pass).
// Step j of a batched solve over the first nact problems (by decreasing m): the
// problems short of their m in the packed form where it applies (a launch of
// P.base[nfull] / R blocks), the others -- and every problem at j < 2 -- in the
// per-unit form.  Both forms keep the same data layout and give the same results.
hipError_t batch_step(const skfab_ctx* ctx, const BatchLayout& L, const BatchPlan& P,
                      const skfab_batch_problem* probs, const skfab_params* p, const BatchStepUnit* su,
                      const int* base, int nact, int j, int block, hipStream_t st, int* nlaunch) {
    int nfull = 0;
    if (ctx->batch_packed && p->k == 2 && !ctx->arnoldi_check && j >= 2 && block == PACKED_BLOCK &&
        packed_step_lds(block, L.R, L.smax) > 0) {
        nfull = nact;
        while (nfull > 0 && probs[L.order[nfull - 1]].m <= j) --nfull;
        // the packed kernel addresses vector entries by 32-bit byte offsets
        for (int qi = 0; qi < nfull; ++qi)
            if (L.prob[L.order[qi]].N >= ((int64_t)1 << 29)) nfull = 0;
    }
    if (nfull > 0) {
        hipError_t e = launch_arnoldi_step_packed(su, base, nfull, L.R, j, P.base[nfull] / L.R, L.smax, p->prec, st);
        if (e != hipSuccess) return e;
        ++*nlaunch;
    }
    if (nact > nfull) {
        hipError_t e = launch_arnoldi_step_batched(su, base, nact, L.R, j, p->k, P.base[nfull],
                                                   P.base[nact] - P.base[nfull], block, L.smax, p->prec, st);
        if (e != hipSuccess) return e;
        ++*nlaunch;
    }
    return hipSuccess;
}

skfab_status run_batch_arnoldi(skfab_ctx* ctx, const BatchLayout& L, const BatchPlan& P,
                               const skfab_batch_problem* probs, const skfab_params* p, char* dev, int block,
                               int jmax, hipStream_t st) {
    const SmallUnit* sm = reinterpret_cast<const SmallUnit*>(dev + L.smalls);
    const BatchStepUnit* su = reinterpret_cast<const BatchStepUnit*>(dev + L.steps);
    const int* base = reinterpret_cast<const int*>(dev + L.base);
    DevCtrl* ctrl = reinterpret_cast<DevCtrl*>(dev + L.ctrl);
    HIP_TRY(launch_fill(reinterpret_cast<double*>(dev + L.small_begin),
                        (int64_t)((L.small_end - L.small_begin) / sizeof(double)), 0.0, st));
    HIP_TRY(launch_init_ctrl_batched(sm, L.nunits, st));
    for (int qi = 0; qi < L.nprob; ++qi) {
        const int pi = L.order[qi];
        const BatchProbLayout& q = L.prob[pi];
        HIP_TRY(launch_sell_convert(probs[pi].A.rowptr, probs[pi].A.col, static_cast<const double*>(probs[pi].A.val),
                                    q.N, q.nslices, q.capacity, ctrl + qi * L.R,
                                    reinterpret_cast<int32_t*>(dev + q.sl_len),
                                    reinterpret_cast<int64_t*>(dev + q.sl_ptr),
                                    reinterpret_cast<int64_t*>(dev + q.bsum),
                                    reinterpret_cast<int32_t*>(dev + q.sl_col), dev + q.sl_val,
                                    reinterpret_cast<DictBuf*>(dev + q.dict),
                                    (ctx->value_table && p->prec == SKFAB_PREC_FP64) ? 1 : 0, p->prec, st));
    }
    int nact = L.nprob;
    // the step launches follow one another with nothing between them: one run
    Span sp;
    HIP_TRY(timing_begin(ctx, 0, st, &sp, true));
    int nlaunch = 0;
    for (int j = 0; j <= jmax; ++j) {
        while (nact > 0 && probs[L.order[nact - 1]].m < j) --nact;
        if (nact == 0) break;
        const hipError_t e = batch_step(ctx, L, P, probs, p, su, base, nact, j, block, st, &nlaunch);
        if (e != hipSuccess) {
            timing_cancel(ctx, sp);
            return SKFAB_ERR_HIP;
        }
    }
    HIP_TRY(timing_end(ctx, sp, st, nlaunch));
    return SKFAB_OK;
}

skfab_status run_batch_small(const BatchLayout& L, const skfab_params* p, char* dev, hipStream_t st,
                             bool check) {
    const SmallUnit* sm = reinterpret_cast<const SmallUnit*>(dev + L.smalls);
    const BatchStepUnit* su = reinterpret_cast<const BatchStepUnit*>(dev + L.steps);
    const int n = L.nunits, m = L.mmax, s = L.smax;
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    if (p->method == SKFAB_SFOM_CLOSED) tol = 1e-13;
    const bool ls = p->method == SKFAB_SGMRES_QUAD;
    HIP_TRY(launch_arnoldi_tail_batched(su, sm, n, s, m, st));
    if (check) HIP_TRY(launch_arnoldi_check_batched(sm, n, s, m, p->k, st));
    HIP_TRY(launch_qr_batched(sm, n, s, m + 1, st));
    HIP_TRY(launch_cond_trunc_batched(sm, n, s, m, cond_max_of(p), st));
    HIP_TRY(launch_pencil_setup_batched(sm, n, s, m, p->k, st));
    HIP_TRY(launch_hhat_rows_batched(sm, n, m, s, st));
    const int branch = (p->f == SKFAB_F_INVSQRT && !ls) ? 1 : 0;
    HIP_TRY(launch_pencil_scalars_batched(sm, n, m, s, 0, branch, p->k, st));
    if (p->f == SKFAB_F_INV) {
        if (ls) HIP_TRY(launch_pencil_scalars_batched(sm, n, m, s, 1, 0, p->k, st));
    } else {
        for (const QuadGroup& g : quad_groups(l1, l2, lmax)) {
            HIP_TRY(launch_quad_group_batched(sm, n, g, m, ls ? 1 : 0, BATCH_SLOTS, p->k, st));
            HIP_TRY(launch_quad_reduce_batched(sm, n, g, m, tol, st));
        }
        HIP_TRY(launch_quad_fail_batched(sm, n, st));
    }
    HIP_TRY(launch_finish_coeffs_batched(sm, n, m, st));
    return SKFAB_OK;
}

skfab_status batch_prepare(skfab_ctx* ctx, int32_t nprob, const skfab_batch_problem* probs, int32_t nrhs,
                           const skfab_params* p, void* ws, size_t ws_bytes, BatchLayout* L) {
    if (!ctx) return SKFAB_ERR_ARG;
    skfab_status v = validate_batch(nprob, probs, nrhs, p, true);
    if (v != SKFAB_OK) return v;
    *L = make_batch_layout(nprob, probs, nrhs, p);
    if (!ws || ws_bytes < L->total || (reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    // the previous call's descriptor upload may still read the host copy
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SKFAB_OK;
}

skfab_status batch_upload(skfab_ctx* ctx, const BatchLayout& L, const BatchPlan& P, const skfab_batch_problem* probs,
                          const skfab_params* p, char* dev) {
    batch_descriptors(L, P, probs, p, dev, ctx->batch_host, ctx->arnoldi_check);
    HIP_TRY(hipMemcpyAsync(dev + L.steps, ctx->batch_host.data() + L.steps, ctx->batch_host.size() - L.steps,
                           hipMemcpyHostToDevice, ctx->stream));
    return SKFAB_OK;
}

}  // namespace

extern "C" {

skfab_status skfab_batch_workspace_bytes(int32_t nprob, const skfab_batch_problem* probs, int32_t nrhs,
                                         const skfab_params* p, size_t* bytes) {
    if (!bytes) return SKFAB_ERR_ARG;
    skfab_status v = validate_batch(nprob, probs, nrhs, p, false);
    if (v != SKFAB_OK) return v;
    *bytes = make_batch_layout(nprob, probs, nrhs, p).total;
    return SKFAB_OK;
}

size_t skfab_srdct_ws_bytes(int64_t n, int32_t s, int32_t ncols) {
    if (n < 1 || s < 1 || ncols < 1) return 0;
    return align_up((size_t)s * n * sizeof(double)) + align_up(srdct_part_doubles(s, n, ncols) * sizeof(double));
}

skfab_status skfab_srdct_apply(skfab_ctx* ctx, int64_t n, int32_t s, const int8_t* signs, const int32_t* rows,
                               const double* V, int64_t ldv, int32_t ncols, double* SV, void* ws, size_t ws_bytes) {
    if (!ctx || !signs || !rows || !V || !SV) return SKFAB_ERR_ARG;
    if (n < 1 || s < 1 || s > n || ncols < 1 || ldv < n) return SKFAB_ERR_SHAPE;
    const size_t need = skfab_srdct_ws_bytes(n, s, ncols);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    double* FP = static_cast<double*>(ws);
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + align_up((size_t)s * n * sizeof(double)));
    HIP_TRY(launch_srdct_matrix(s, n, signs, rows, FP, ctx->stream));
    HIP_TRY(launch_srdct_sketch(FP, s, n, V, ldv, ncols, 0, part, nullptr, nullptr, SV, s, ctx->stream));
    return SKFAB_OK;
}

skfab_status skfab_set_arnoldi_check(skfab_ctx* ctx, int32_t enable) {
    if (!ctx || (enable != 0 && enable != 1)) return SKFAB_ERR_ARG;
    ctx->arnoldi_check = enable != 0;
    return SKFAB_OK;
}

skfab_status skfab_set_value_table(skfab_ctx* ctx, int32_t enable) {
    if (!ctx || (enable != 0 && enable != 1)) return SKFAB_ERR_ARG;
    ctx->value_table = enable != 0;
    return SKFAB_OK;
}

skfab_status skfab_batch_set_tuning(skfab_ctx* ctx, const skfab_batch_tuning* t) {
    if (!ctx || !t) return SKFAB_ERR_ARG;
    if (t->block != 256 && t->block != 512 && t->block != 1024) return SKFAB_ERR_ARG;
    if (t->slices_per_wave < 1 || t->slices_per_wave > 64) return SKFAB_ERR_ARG;
    if (t->packed != 0 && t->packed != 1) return SKFAB_ERR_ARG;
    ctx->batch_block = t->block;
    ctx->batch_spw = t->slices_per_wave;
    ctx->batch_packed = t->packed != 0;
    return SKFAB_OK;
}

skfab_status skfab_batch_get_tuning(skfab_ctx* ctx, skfab_batch_tuning* t) {
    if (!ctx || !t) return SKFAB_ERR_ARG;
    t->block = ctx->batch_block;
    t->slices_per_wave = ctx->batch_spw;
    t->packed = ctx->batch_packed ? 1 : 0;
    return SKFAB_OK;
}

skfab_status skfab_solve_batched(skfab_ctx* ctx, int32_t nprob, const skfab_batch_problem* probs, int32_t nrhs,
                                 const skfab_params* p, void* ws, size_t ws_bytes, skfab_info* info) {
    BatchLayout L;
    skfab_status r = batch_prepare(ctx, nprob, probs, nrhs, p, ws, ws_bytes, &L);
    if (r != SKFAB_OK) return r;
    char* dev = static_cast<char*>(ws);
    hipStream_t st = ctx->stream;
    const int block = step_block_fit(ctx->batch_block, L.smax);
    const BatchPlan P = batch_plan(L, block, ctx->batch_spw);
    r = batch_upload(ctx, L, P, probs, p, dev);
    if (r != SKFAB_OK) return r;
    r = run_batch_arnoldi(ctx, L, P, probs, p, dev, block, L.mmax, st);
    if (r != SKFAB_OK) return r;
    r = run_batch_small(L, p, dev, st, ctx->arnoldi_check);
    if (r != SKFAB_OK) return r;
    const SmallUnit* sm = reinterpret_cast<const SmallUnit*>(dev + L.smalls);
    Span sp;
    HIP_TRY(timing_begin(ctx, 1, st, &sp));
    HIP_TRY(launch_assemble_batched(sm, L.nunits, L.nmax, L.mmax, p->prec, st));
    HIP_TRY(timing_end(ctx, sp, st));
    if (!info) return SKFAB_OK;
    std::vector<DevCtrl> c(L.nunits);
    HIP_TRY(hipMemcpyAsync(c.data(), dev + L.ctrl, sizeof(DevCtrl) * L.nunits, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int qi = 0; qi < L.nprob; ++qi) {
        const int pi = L.order[qi];
        for (int rr = 0; rr < L.R; ++rr) {
            // the problem's SELL flags sit in its first unit
            ctrl_to_info(c[qi * L.R + rr], a_format(c[qi * L.R]), &info[pi * L.R + rr]);
        }
    }
    return SKFAB_OK;
}

skfab_status skfab_batch_autotune(skfab_ctx* ctx, int32_t nprob, const skfab_batch_problem* probs, int32_t nrhs,
                                  const skfab_params* p, void* ws, size_t ws_bytes, int32_t steps,
                                  skfab_batch_tuning* chosen) {
    BatchLayout L;
    skfab_status r = batch_prepare(ctx, nprob, probs, nrhs, p, ws, ws_bytes, &L);
    if (r != SKFAB_OK) return r;
    if (steps < 1) steps = 4;
    char* dev = static_cast<char*>(ws);
    hipStream_t st = ctx->stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int blocks[3] = {256, 512, 1024};
    const int spws[7] = {1, 2, 4, 8, 16, 32, 64};
    float best = 1e30f;
    int bb = ctx->batch_block, bs = ctx->batch_spw;
    bool bp = ctx->batch_packed;
    const bool timing = ctx->timing, packed0 = ctx->batch_packed;
    ctx->timing = false;
    // candidates: block x slices per wave, and for 512-thread blocks also the packed
    // form (timed over the same steps; it applies from step 2 on)
    for (int ci = 0; ci < 4 * 7 && r == SKFAB_OK; ++ci) {
        const int bi = (ci / 7 < 3) ? ci / 7 : 1, si = ci % 7;
        const bool packed = ci >= 3 * 7;
        if (packed && (p->k != 2 || packed_step_lds(blocks[bi], L.R, L.smax) == 0)) continue;
        if (step_block_fit(blocks[bi], L.smax) != blocks[bi]) continue;  // bins do not fit LDS
        ctx->batch_packed = packed;
        {
            const BatchPlan P = batch_plan(L, blocks[bi], spws[si]);
            // the step launches of a candidate time j = 1 .. steps (j = 0 has no
            // previous step to reduce and is run untimed first)
            if (hipStreamSynchronize(st) != hipSuccess) { r = SKFAB_ERR_HIP; break; }
            r = batch_upload(ctx, L, P, probs, p, dev);
            if (r != SKFAB_OK) break;
            r = run_batch_arnoldi(ctx, L, P, probs, p, dev, blocks[bi], 0, st);
            if (r != SKFAB_OK) break;
            if (hipEventRecord(e0, st) != hipSuccess) { r = SKFAB_ERR_HIP; break; }
            const BatchStepUnit* su = reinterpret_cast<const BatchStepUnit*>(dev + L.steps);
            const int* base = reinterpret_cast<const int*>(dev + L.base);
            int nact = L.nprob, nl = 0;
            for (int j = 1; j <= steps; ++j) {
                while (nact > 0 && probs[L.order[nact - 1]].m < j) --nact;
                if (nact == 0) break;
                if (batch_step(ctx, L, P, probs, p, su, base, nact, j, blocks[bi], st, &nl) != hipSuccess) {
                    r = SKFAB_ERR_HIP;
                    break;
                }
            }
            if (r != SKFAB_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { r = SKFAB_ERR_HIP; break; }
            if (ms < best) { best = ms; bb = blocks[bi]; bs = spws[si]; bp = packed; }
        }
    }
    ctx->timing = timing;
    ctx->batch_packed = packed0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != SKFAB_OK) return r;
    ctx->batch_block = bb;
    ctx->batch_spw = bs;
    ctx->batch_packed = bp;
    if (chosen) { chosen->block = bb; chosen->slices_per_wave = bs; chosen->packed = bp ? 1 : 0; }
    return SKFAB_OK;
}

}  // extern "C"

// ============================================================ adaptive m
namespace {

struct AdaptiveLayout {
    Layout main, snap;
    size_t snap_off, ysave_off, out_off, total;
};

AdaptiveLayout make_adaptive_layout(const skfab_csr* A, const skfab_params* p) {
    int l1, l2, lmax;
    double tol;
    defaults(p, &l1, &l2, &lmax, &tol);
    AdaptiveLayout L;
    L.main = make_layout(A->n, A->nnz, p->m, p->s, l1, l2, lmax, p->npoly, true, p->prec, p->k);
    L.snap = make_layout(0, 0, p->m, p->s, l1, l2, lmax, p->npoly, false, 0);
    L.snap_off = align_up(L.main.total);
    L.ysave_off = align_up(L.snap_off + L.snap.total);
    L.out_off = align_up(L.ysave_off + (size_t)2 * p->m * sizeof(double));
    L.total = align_up(L.out_off + 2 * sizeof(double));
    return L;
}

void fill_info(const DevCtrl& c, skfab_info* info) { ctrl_to_info(c, a_format(c), info); }

}  // namespace

extern "C" {

skfab_status skfab_adaptive_workspace_bytes(const skfab_csr* A, const skfab_params* p, size_t* bytes) {
    if (!bytes || !A || !p) return SKFAB_ERR_ARG;
    skfab_status v = validate(A, p, false);
    if (v != SKFAB_OK) return v;
    if (A->n <= 0) return SKFAB_ERR_SHAPE;
    *bytes = make_adaptive_layout(A, p).total;
    return SKFAB_OK;
}

skfab_status skfab_solve_adaptive(skfab_ctx* ctx, const skfab_csr* A, const double* b, double* x,
                                  const skfab_params* p, int32_t m0, int32_t d, double tol, void* ws,
                                  size_t ws_bytes, skfab_info* info, int32_t* m_stop, double* estimate) {
    if (!ctx || !b || !x) return SKFAB_ERR_ARG;
    skfab_status v = validate(A, p, true);
    if (v != SKFAB_OK) return v;
    if (p->method != SKFAB_SFOM_CLOSED || p->two_pass || p->sketch != SKFAB_SKETCH_SPARSE_SIGN) return SKFAB_ERR_ARG;
    if (d < 1 || m0 < p->k || m0 > p->m || !(tol > 0.0)) return SKFAB_ERR_ARG;
    const AdaptiveLayout L = make_adaptive_layout(A, p);
    if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    char* base = static_cast<char*>(ws);
    const Ptrs w = carve(ws, L.main);
    double* ysave[2] = {reinterpret_cast<double*>(base + L.ysave_off),
                        reinterpret_cast<double*>(base + L.ysave_off) + p->m};
    double* dout = reinterpret_cast<double*>(base + L.out_off);
    hipStream_t st = ctx->stream;
    const int m = p->m, s = p->s;
    int l1, l2, lmax;
    double qtol;
    defaults(p, &l1, &l2, &lmax, &qtol);
    StepArgs a;
    skfab_status r = arnoldi_setup(A, b, p, L.main, w, ctx->value_table, st, &a);
    if (r != SKFAB_OK) return r;
    int mprev = 0, cur = 0;
    bool broke = false;
    double est = INFINITY;
    for (int j = 0; j <= m; ++j) {
        r = arnoldi_step(ctx, a, p, L.main, w, j, st);
        if (r != SKFAB_OK) return r;
        const int mp = j - 1;
        if (broke || j < 1 || mp < m0 || (mp - m0) % d != 0 || mp >= m) continue;
        // checkpoint mp: the first mp steps as a small problem of their own
        const Layout sl = make_layout(0, 0, mp, s, l1, l2, lmax, p->npoly, false, 0);
        const Ptrs sw = carve(base + L.snap_off, sl);
        HIP_TRY(launch_init_ctrl(sw.ctrl, mp, st));
        HIP_TRY(launch_snapshot(w.SV, s, w.H, m + 1, w.eta, mp, sw.SV, sw.H, sw.eta, sw.colnorm2, sw.SAV, st));
        skfab_params q = *p;
        q.m = mp;
        r = run_small(&q, sl, sw, st);
        if (r != SKFAB_OK) return r;
        HIP_TRY(launch_adaptive_est(w.SV, s, mp, sw.y, ysave[1 - cur], mprev, sw.ctrl, dout, ysave[cur], st));
        double hout[2];
        DevCtrl mc;
        HIP_TRY(hipMemcpyAsync(hout, dout, sizeof(hout), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&mc, w.ctrl, sizeof(DevCtrl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (mc.stop && mc.m_used <= mp) { broke = true; continue; }  // the final solve is exact
        est = hout[0];
        if (est <= tol) {
            HIP_TRY(launch_rescale_coeffs(sw.y, w.eta, mp, sw.ys, st));
            HIP_TRY(launch_assemble(w.U, L.main.ldU, A->n, mp, sw.ctrl, sw.ys, x, p->prec, st));
            if (m_stop) *m_stop = mp;
            if (estimate) *estimate = est;
            if (info) {
                DevCtrl c;
                HIP_TRY(hipMemcpyAsync(&c, sw.ctrl, sizeof(DevCtrl), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                fill_info(c, info);
            }
            return SKFAB_OK;
        }
        mprev = mp;
        cur = 1 - cur;
    }
    // no checkpoint passed (or a breakdown): the full solve at m, judged against the last checkpoint
    r = arnoldi_tail(a, p, L.main, w, st);
    if (r != SKFAB_OK) return r;
    r = run_small(p, L.main, w, st);
    if (r != SKFAB_OK) return r;
    HIP_TRY(launch_adaptive_est(w.SV, s, m, w.y, ysave[1 - cur], broke ? 0 : mprev, w.ctrl, dout, ysave[cur], st));
    HIP_TRY(launch_assemble(w.U, L.main.ldU, A->n, m, w.ctrl, w.ys, x, p->prec, st));
    double hout[2];
    DevCtrl c;
    HIP_TRY(hipMemcpyAsync(hout, dout, sizeof(hout), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&c, w.ctrl, sizeof(DevCtrl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (m_stop) *m_stop = c.m_used;
    if (estimate) *estimate = broke ? 0.0 : hout[0];
    if (info) fill_info(c, info);
    return SKFAB_OK;
}

// ------------------------------------------------------- controller support
size_t skfab_gershgorin_ws_bytes(int64_t n) {
    if (n <= 0) return 0;
    return (size_t)2 * gershgorin_blocks(n) * sizeof(double);
}

skfab_status skfab_gershgorin(skfab_ctx* ctx, const skfab_csr* A, double* bounds, void* ws, size_t ws_bytes) {
    if (!ctx || !A || !bounds || !A->rowptr || !A->col || !A->val) return SKFAB_ERR_ARG;
    if (A->val_type != SKFAB_VAL_F64) return SKFAB_ERR_ARG;
    if (A->n <= 0) return SKFAB_ERR_SHAPE;
    if (!ws || ws_bytes < skfab_gershgorin_ws_bytes(A->n)) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    HIP_TRY(launch_gershgorin(A->rowptr, A->col, static_cast<const double*>(A->val), A->n,
                              static_cast<double*>(ws), bounds, ctx->stream));
    return SKFAB_OK;
}

int32_t skfab_mlp_param_count(void) { return mlp_param_count(); }

size_t skfab_mlp_ws_bytes(int32_t batch) {
    if (batch <= 0) return 0;
    return mlp_ws_floats(batch) * sizeof(float);
}

skfab_status skfab_mlp_forward(skfab_ctx* ctx, const float* X, int32_t B, const float* params, float* Y, void* ws,
                               size_t ws_bytes) {
    if (!ctx || !X || !params || !Y || B <= 0) return SKFAB_ERR_ARG;
    if (!ws || ws_bytes < skfab_mlp_ws_bytes(B)) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    HIP_TRY(launch_mlp_forward(X, B, params, Y, static_cast<float*>(ws), ctx->stream));
    return SKFAB_OK;
}

skfab_status skfab_mlp_loss_grad(skfab_ctx* ctx, const float* X, const float* T, int32_t B, const float* params,
                                 float* grad, float* loss, void* ws, size_t ws_bytes) {
    if (!ctx || !X || !T || !params || !grad || B <= 0) return SKFAB_ERR_ARG;
    if (!ws || ws_bytes < skfab_mlp_ws_bytes(B)) return SKFAB_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    HIP_TRY(launch_mlp_loss_grad(X, T, B, params, grad, loss, static_cast<float*>(ws), ctx->stream));
    return SKFAB_OK;
}

skfab_status skfab_mlp_adam(skfab_ctx* ctx, float* params, const float* grad, float* m1, float* m2, int32_t t,
                            float lr, float beta1, float beta2, float eps) {
    if (!ctx || !params || !grad || !m1 || !m2 || t < 1) return SKFAB_ERR_ARG;
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return SKFAB_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SKFAB_ERR_HIP;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, t)));
    HIP_TRY(launch_mlp_adam(params, grad, m1, m2, mlp_param_count(), lr, beta1, beta2, eps, c1, c2, ctx->stream));
    return SKFAB_OK;
}

}  // extern "C"
