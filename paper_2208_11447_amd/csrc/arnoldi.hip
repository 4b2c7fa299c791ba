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
// The stored basis is U (v_j = u_j / eta_j with eta_j = ||u_j||).  The truncated
// modified Gram-Schmidt coefficients are obtained from the dot products and the
// Gram entries of the window (h_i = <v_i, w> - sum_{l<i} h_l <v_i, v_l>), which
// equals sequential MGS for the stored vectors.  Entries of u_j needed by the
// SpMV at neighbouring rows are recomputed from W_{j-1} and the window with the
// same fused multiply-add sequence, so the SpMV input equals the stored U_j bit
// for bit.
//
// Layout and mapping: A is copied once per solve into SELL-64 (slices of 64 rows
// = one wavefront, entries of a slice interleaved so every load of the column
// indices and values is coalesced); each wavefront owns one slice at a time and
// every lane one row.  Blocks own contiguous ranges of slices, assigned so that
// the blocks of one XCD own neighbouring rows (shared L2 for the gathers).
//
// Sketches: per-wave LDS bins (64-lane FP64 LDS atomics, deterministic within a
// wavefront), combined in wave order per block and written bin-major into a
// [2s][G] partial array; the next step's blocks reduce it in slot order and
// write S v_j and S A v_j (scaled by 1/eta_j) into SV, SAV.  Every sum has a
// fixed order: results are bitwise reproducible run to run.
#include <type_traits>

#include "common.hpp"
#include "device_state.hpp"

namespace skfab {

// ----------------------------------------------------------- coefficients
// Window values read by the coefficients of step p, fetched by thread t < KW^2 at
// the start of the next launch so that their latency overlaps the reductions:
// win[0] = ||A v_{p-1}||, win[o] = eta_{p-o} (1 <= o < KW), and
// win[KW + (o-1) KW + o2] = <v_{p-o}, v_{p-o2}> (1 <= o < o2 < KW); 0 where absent.
// (unconditional loads from clamped addresses, then a select: a load inside a
// branch, or from a selected pointer, would be waited for before the loads that
// follow it are issued)
template <int KW>
__device__ __forceinline__ double window_value(const StepArgs& a, int p, int t) {
    const int q = t - KW, o = 1 + q / KW, o2 = q % KW;
    const bool okw = t == 0 && p >= 1;
    const bool oke = t > 0 && t < KW && p - t >= 0;
    const bool okg = t >= KW && t < KW * KW && o2 > o && p - o2 >= 0;
    const double vw = gptr(a.wnorm)[okw ? p - 1 : 0];
    const double ve = gptr(a.eta)[oke ? p - t : 0];
    const double vg = gptr(a.gram)[okg ? (int64_t)(p - o) * KMAX + (o2 - o - 1) : 0];
    return okw ? vw : (oke ? ve : (okg ? vg : 0.0));
}

// Turns the reduced dot products of step p into eta_p, h_{.,p}, the Gram
// entries of v_p and the coefficients of u_{p+1}.  Runs on one thread.
// Returns false on breakdown (m_used set to p, or 0 for b = 0).
template <int KW>
__device__ bool step_coefficients(const double* red, const double* win, int p, int k, bool writer,
                                  const StepArgs& a, double* coef) {
    const double uu = red[0], uw = red[1], ww = red[2];
    const double eta_p = sqrt(uu);
    bool ok;
    if (p == 0) {
        ok = eta_p > 0.0;
    } else {
        ok = eta_p > BREAKDOWN_TOL * win[0];
    }
    if (coef) coef[KMAX + 1] = eta_p;
    if (!ok) {
        if (writer) {
            a.ctrl->m_used = p;
            a.ctrl->stop = 1;
            if (p >= 1) a.H[p + a.ldH * (p - 1)] = eta_p;
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
            const double eo = win[o];
            d[o] = red[3 + (o - 1)] / (eo * eta_p);
            gp[o] = red[3 + (KW - 1) + (o - 1)] / (eta_p * eo);
        }
    }
    // modified Gram-Schmidt order: ascending i = p - o, i.e. descending o
#pragma unroll
    for (int o = KW - 1; o >= 0; --o) {
        if (o < nwp) {
            double hi = d[o];
#pragma unroll
            for (int o2 = KW - 1; o2 > o; --o2) {
                if (o2 < nwp) {
                    const double gil = (o == 0) ? gp[o2] : win[KW + (o - 1) * KW + o2];
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
            const double eo = (o == 0) ? eta_p : ((o < nwp) ? win[o] : 1.0);
            coef[1 + o] = (o < nwp) ? -h[o] / eo : 0.0;
        }
    }
    if (writer) {
        a.eta[p] = eta_p;
        a.wnorm[p] = wn;
        const int64_t ldh = a.ldH;
        for (int o = 0; o < nwp; ++o) a.H[(p - o) + ldh * p] = h[o];
        if (p >= 1) a.H[p + ldh * (p - 1)] = eta_p;
        for (int o = 1; o < nwp; ++o) a.gram[(int64_t)p * KMAX + (o - 1)] = gp[o];
    }
    return true;
}

// Bins [c0, c1) of the reduction of step p's sketch partials (slots summed in
// fixed order), one wavefront per bin; used only when a block owns more bins than
// it has wavefronts.  Bin i < s goes to SV[:, p] (scale_v), bin s + i to SAV[:, p]
// (scale_av, skipped when write_av is false).
template <int BLOCK>
__device__ void reduce_prev_sketch_tail(const double* skp, int G, int s, int64_t ldS, int p, int c0, int c1,
                                        double scale_v, double scale_av, bool write_av, double* SV, double* SAV) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    constexpr int NW = BLOCK / WAVE;
    for (int bin = c0 + wid; bin < c1; bin += NW) {
        if (bin >= s && !write_av) continue;
        const double* src = skp + (int64_t)bin * G;
        double t = 0.0;
        for (int g = lane; g < G; g += WAVE) t += src[g];
        t = wave_sum(t);
        if (lane == 0) {
            if (bin < s) SV[(int64_t)p * ldS + bin] = t * scale_v;
            else SAV[(int64_t)p * ldS + (bin - s)] = t * scale_av;
        }
    }
}

// ------------------------------------------------------------- step kernel
#define NW_OF(BLOCK) ((BLOCK) / 64)
// SELL entries per load batch (fewer for wide windows to bound register use).  Seven
// covers a 7-point stencil row in one batch: an eighth slot would cost a guarded
// load and three gathers per row for nothing (measured 2.3 us per step, 3D 128^3).
template <int KW> struct SellBatch { static constexpr int value = KW <= 2 ? 7 : (KW <= 4 ? 4 : 1); };

// P: storage/arithmetic policy (PrecF64, PrecF32, PrecBF16).  The basis u_j is
// formed in the SpMV type W, rounded to the basis type V for storage, and the
// rounded value is what enters the product with A, the sketch and the dots (so
// the stored basis, its sketch and its image under A stay consistent).  Dot
// products and sketch bins accumulate in FP64.
//
// The body serves both the single-problem kernel and the batched one: `bid` is
// the block's index among the G blocks of its (problem, right-hand side) pair.
template <int KW, int ZETA, int BLOCK, typename P, bool PREFETCH>
__device__ __forceinline__ void step_body(StepArgs a, const int bid) {
    using VT = typename P::V;
    using WT = typename P::W;
    using AT = typename P::A;
    extern __shared__ double bins[];  // [BLOCK/64][2s]
    __shared__ double red[NSC_MAX];
    __shared__ double coef[KMAX + 2];
    __shared__ double win[KW * KW];
    __shared__ int2 meta[NW_OF(BLOCK)][WAVE];  // per-wave ring: (entries, offset / 64) of 64 slices
    __shared__ double scratch[BLOCK / WAVE];
    __shared__ int s_ok;
    __shared__ int s_prog;  // slices finished by the block's wavefronts (main loop)
    __shared__ WT dtab[DICT_MAX];  // the matrix's value table (uint8 form of the SELL copy)

    const int sell_flag = gptr(a.sctrl)->sell_ok;  // issued with the control-block loads
    const int col16 = gptr(a.sctrl)->col16;
    const int dict8 = gptr(a.sctrl)->dict8;
    const WT dval = (WT)(AT)gptr(a.sl_table)[threadIdx.x & (DICT_MAX - 1)];  // (written to LDS in the prologue)
    // A breakdown detected by an earlier step ends the recurrence (the step that
    // detects it still runs its prologue to write the extension column).  The test
    // is made only after every load of the prologue has been issued, so that the
    // control block's latency overlaps theirs.
    const int stop_flag = gptr(a.ctrl)->stop, stop_m = gptr(a.ctrl)->m_used;
    const bool stopped = stop_flag && stop_m < a.j - 1;
    constexpr int NSC = 2 * KW + 1;
    constexpr int NW = BLOCK / WAVE;
    const int j = a.j, k = a.k, s = a.s, G = a.G;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;

    // SELL path: every slice's entry count and offset are read once per window of 64
    // slices (lane i fetching the wave's i-th slice) into a per-wave LDS ring, so a
    // slice's loads wait neither on a metadata load from memory nor on the stores of
    // the previous slice.  The first window is requested before the prologue so that
    // its latency overlaps the reductions.
    const int chunk = xcd_chunk(bid, G);
    const int64_t sl0 = (int64_t)chunk * a.slices_per_chunk + wid;
    const int64_t sl1 = min(a.nslices, (int64_t)(chunk + 1) * a.slices_per_chunk);
    // (loaded from a clamped, always valid index and masked only when written to
    // LDS after the prologue: a guarded load would be waited for on the spot)
    const int64_t itl0 = sl0 + (int64_t)lane * NW;
    const bool win_in = !a.extend && itl0 < sl1;
    const int64_t itl0c = win_in ? itl0 : 0;
    const GAS int32_t* __restrict__ sl_len = gptr(a.sl_len);
    const GAS int64_t* __restrict__ sl_ptr = gptr(a.sl_ptr);
    const int wlen = sl_len[itl0c];
    const int64_t wptr = sl_ptr[itl0c];

    if (j > 0) {
        // issue every load of the prologue before any reduction: the partial scalars
        // of step j-1 (G per scalar), this block's share of its sketch partials, and
        // the window's eta / Gram entries used by the coefficients
        // (fixed trip counts and clamped indices: every load is issued before the first
        // is used; the host never launches more than STEP_GMAX_1024 * 1024 / BLOCK blocks)
        constexpr int GM = STEP_GMAX_1024 * (1024 / BLOCK);
        constexpr int GPT = (GM + BLOCK - 1) / BLOCK;  // partial slots per thread
        constexpr int GPL = (GM + WAVE - 1) / WAVE;    // slots per lane of one sketch bin
        double sv[NSC];
        {
            double ld[NSC][GPT];
#pragma unroll
            for (int q = 0; q < GPT; ++q) {
                const int g = tid + q * BLOCK, gc = (g < G) ? g : 0;
#pragma unroll
                for (int sc = 0; sc < NSC; ++sc) ld[sc][q] = gptr(a.scal_prev)[(int64_t)sc * G + gc];
            }
#pragma unroll
            for (int sc = 0; sc < NSC; ++sc) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < GPT; ++q)  // mask by a factor 0 / 1: exact, and no branch
                    t = fma((tid + q * BLOCK < G) ? 1.0 : 0.0, ld[sc][q], t);
                sv[sc] = t;
            }
        }
        const double wv = window_value<KW>(a, j - 1, tid);  // nonzero for tid < KW^2 only
        const int nb = a.sav ? 2 * s : s;  // bins of S u_{j-1} (and of S A u_{j-1})
        const int b0 = (bid * nb) / G;        // bid nb <= 1024 * 2048: 32-bit arithmetic
        const int b1 = ((bid + 1) * nb) / G;
        // sketch partial sums of this block's bins (one wavefront per bin)
        double skv = 0.0;
        int mybin = -1;
        if (b0 + wid < b1) {
            mybin = b0 + wid;
            const GAS double* src = gptr(a.skp_prev) + (int64_t)mybin * G;
            double ld[GPL];
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                const int g = lane + q * WAVE;
                ld[q] = src[(g < G) ? g : 0];
            }
            double t0 = 0.0, t1 = 0.0;  // even slots of 64 into t0, odd into t1
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                const double mk = (lane + q * WAVE < G) ? 1.0 : 0.0;
                if (q & 1) t1 = fma(mk, ld[q], t1);
                else t0 = fma(mk, ld[q], t0);
            }
            skv = t0 + t1;
        }
        if (stopped) return;
        if (tid < KW * KW) win[tid] = wv;
        if (tid < DICT_MAX) dtab[tid] = dval;
        // every thread's scalar partials reduced in a fixed tree through the (not yet
        // used) sketch-bin region of LDS (its first barrier also publishes win and dtab)
        block_reduce_multi<NSC, BLOCK>(sv, bins, red);
        if (tid == 0) s_ok = step_coefficients<KW>(red, win, j - 1, k, bid == 0, a, coef) ? 1 : 0;
        skv = wave_sum(skv);
        // the bin region is free again: the other wavefronts clear it meanwhile
        if (wid > 0)
            for (int i = tid - WAVE; i < NW * 2 * s; i += BLOCK - WAVE) bins[i] = 0.0;
        if (tid == WAVE) s_prog = 0;
        __syncthreads();
        // S v_{j-1}, S A v_{j-1}; after a breakdown, S u_{j-1} unnormalised (extension column)
        const double eta_p = coef[KMAX + 1];
        const bool ok = s_ok != 0;
        if (mybin >= 0 && lane == 0) {
            if (mybin < s) gptr(a.SV)[(int64_t)(j - 1) * a.ldS + mybin] = skv * (ok ? a.inv_sqrt_zeta / eta_p : a.inv_sqrt_zeta);
            else if (ok) gptr(a.SAV)[(int64_t)(j - 1) * a.ldS + (mybin - s)] = skv * (a.inv_sqrt_zeta / eta_p);
        }
        // bins beyond one per wave (only when 2s > 16 G): fall back to the generic loop
        if (b1 - b0 > NW)
            reduce_prev_sketch_tail<BLOCK>(a.skp_prev, G, s, a.ldS, j - 1, b0 + NW, b1,
                                           ok ? a.inv_sqrt_zeta / eta_p : a.inv_sqrt_zeta,
                                           a.inv_sqrt_zeta / eta_p, ok && a.sav, a.SV, a.SAV);
        if (!ok) return;
    } else {
        if (stopped) return;
        if (tid == 0) {
            coef[0] = 1.0;
            for (int o = 0; o < KW; ++o) coef[1 + o] = 0.0;
        }
        for (int i = tid; i < NW * 2 * s; i += BLOCK) bins[i] = 0.0;
        if (tid == 0) s_prog = 0;
        if (tid < DICT_MAX) dtab[tid] = dval;
        __syncthreads();
    }

    meta[wid][lane] = win_in ? make_int2(wlen, (int)(wptr >> 6)) : make_int2(0, 0);
    const int nwin_all = (j == 0) ? 0 : min(k, j);   // vectors j-1 .. j-nwin form u_j
    const int ndot = min(k - 1, j);              // vectors j-1 .. j-ndot enter the dots
    const double alpha = coef[0];
    double cf[KW];
#pragma unroll
    for (int o = 0; o < KW; ++o) cf[o] = coef[1 + o];

    const GAS WT* __restrict__ Wp = gptr(static_cast<const WT*>(a.Wprev));
    const GAS double* __restrict__ b0p = gptr(a.b);
    const bool first_all = (j == 0);
    // basis vector c in column c % uring (a ring of k + 1 columns in the two-pass form)
    const int ur = a.uring;
    const GAS VT* Uo[KW];
#pragma unroll
    for (int o = 0; o < KW; ++o) Uo[o] = gptr(static_cast<const VT*>(a.U)) + (int64_t)((o < nwin_all) ? (j - 1 - o) % ur : 0) * a.ldU;
    GAS VT* __restrict__ Uj = gptr(static_cast<VT*>(a.U)) + (int64_t)(j % ur) * a.ldU;
    const bool store_u = !a.extend || a.keep_ext;
    const bool sketch = !a.nosketch;
    GAS WT* __restrict__ Wc = gptr(static_cast<WT*>(a.Wcur));
    const GAS AT* __restrict__ slv = gptr(static_cast<const AT*>(a.sl_val));
    const GAS int32_t* __restrict__ sl_col = gptr(a.sl_col);
    const GAS int16_t* __restrict__ slo = gptr(reinterpret_cast<const int16_t*>(a.sl_col));
    const GAS uint8_t* __restrict__ sl8 = gptr(reinterpret_cast<const uint8_t*>(a.sl_val));
    const GAS int32_t* __restrict__ rowptr = gptr(a.rowptr);
    const GAS int32_t* __restrict__ colp = gptr(a.col);
    const GAS double* __restrict__ valp = gptr(a.val);
    const WT alpha_w = (WT)alpha;
    WT cf_w[KW];
#pragma unroll
    for (int o = 0; o < KW; ++o) cf_w[o] = (WT)cf[o];
    double* binV = bins + wid * 2 * s;
    double* binAV = binV + s;

    double acc_uu = 0.0, acc_uw = 0.0, acc_ww = 0.0;
    double acc_lw[KW], acc_ul[KW];
#pragma unroll
    for (int o = 0; o < KW; ++o) { acc_lw[o] = 0.0; acc_ul[o] = 0.0; }

    const bool sell = sell_flag != 0;
    // rows of this block: SELL slices [sl0, sl1) or CSR rows [r_begin, r_end)
    int64_t it0, it1, step;
    if (sell) {
        it0 = sl0;
        it1 = sl1;
        step = NW;
    } else {
        const int64_t r_begin = (int64_t)chunk * a.rows_per_chunk;
        it0 = r_begin + tid;
        it1 = min(a.N, r_begin + a.rows_per_chunk);
        step = BLOCK;
    }
    constexpr int SB = SellBatch<KW>::value;
    const bool pre = sell && !a.extend;
    // the loop twice: once for the steps whose window is full (j >= k, every test of
    // the window length folded away), once for the first k steps
    auto main_loop = [&](auto full_tag, auto dict_tag) __attribute__((always_inline)) {
    constexpr bool FULL = decltype(full_tag)::value;
    constexpr bool DICT = decltype(dict_tag)::value;  // values as uint8 indices into dtab
    const bool first = FULL ? false : first_all;
    const int nwin = FULL ? KW : nwin_all;
    int wbase = 0;
    int iter = 0;
    // metadata of the slice at loop position idx (slice index itn) from the wavefront's
    // ring, refilled with the next 64 slices when it runs out
    auto ring = [&](int64_t itn, int idx) {
        if (idx - wbase == WAVE) {
            wbase += WAVE;
            const int64_t itl = itn + (int64_t)lane * step;
            const int nl = (itl < it1) ? sl_len[itl] : 0;
            const int np = (itl < it1) ? (int)(sl_ptr[itl] >> 6) : 0;
            meta[wid][lane] = make_int2(nl, np);
        }
        return meta[wid][idx - wbase];
    };
    // Batched form, with the value table and windows up to 2 wide: the next slice's
    // metadata and the column data of its first batch are requested while the
    // current slice is processed, so that a slice waits for one memory round trip
    // (its value indices travel with its gathers) instead of two.  (Measured: 2 %
    // faster in the batched form; slower in the single-problem one, whose main
    // loop then runs at the register limit, and slower with 8-byte values, where
    // the loop was bound by bandwidth.  Wider windows have no registers left.)
    constexpr bool PFC = PREFETCH && DICT && KW <= 2;
    int lenN = 0;
    int64_t e0N = 0;
    int pcol[SB];
    auto prefetch = [&](int64_t itn, int idx) {
        const int2 md = ring(itn, idx);
        lenN = md.x;
        e0N = ((int64_t)md.y << 6) + lane;
#pragma unroll
        for (int q = 0; q < SB; ++q) {
            if (q < lenN) pcol[q] = col16 ? (int)slo[e0N + (int64_t)q * WAVE] : sl_col[e0N + (int64_t)q * WAVE];
            else pcol[q] = 0;
        }
    };
    if (PFC && pre && it0 < it1) prefetch(it0, 0);
    for (int64_t it = it0; it < it1; it += step, ++iter) {
        const int64_t r = sell ? it * WAVE + lane : it;
        const bool valid = r < a.N;
        int len = 0;
        int64_t e0 = 0;
        bool pf_done = !(PFC && pre) || it + step >= it1;  // the next slice's prefetch is issued
        if (pre) {
            // the four wavefronts of a SIMD share its issue slots, which go to the oldest
            // first: with equal static shares the youngest would finish last.  A
            // wavefront behind the block's average takes the higher priority instead
            // (timing only: the slices each wavefront owns do not change).
            const int done = __hip_atomic_load(&s_prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (done > iter * NW) __builtin_amdgcn_s_setprio(3);
            else __builtin_amdgcn_s_setprio(0);
            if constexpr (PFC) {
                len = lenN;
                e0 = e0N;
            } else {
                const int2 md = ring(it, iter);
                len = md.x;
                e0 = ((int64_t)md.y << 6) + lane;
            }
        }
        // the row's own inputs of u_j: requested before the matrix entries and used
        // only after the product, which needs u_j at the neighbours, not at the row
        // (for the widest windows only W: holding all k values through the product
        // would spill registers)
        WT wrow = (WT)0;
        VT urow[KW];
        if (valid) {
            wrow = first ? (WT)b0p[r] : Wp[r];
            if constexpr (KW <= 4) {
#pragma unroll
                for (int o = 0; o < KW; ++o)
                    if (o < nwin) urow[o] = gload(Uo[o] + r);
            }
        }
        WT w = (WT)0;
        if (!a.extend) {
            if (sell) {
                // entries in batches of SB: all index and value loads of a batch, then all
                // gathers, then the products -- one memory round trip per batch
                const int32_t rr = valid ? (int32_t)r : 0;  // offsets of rows beyond N are 0
                for (int q0 = 0; q0 < len; q0 += SB) {
                    int cc[SB], vi[SB];
                    WT vv[SB], xb[SB], xu[SB][KW];
                    if (PFC && q0 == 0) {
#pragma unroll
                        for (int q = 0; q < SB; ++q) {
                            const bool in = q < len;
                            cc[q] = in ? (col16 ? rr + pcol[q] : pcol[q]) : 0;
                            vi[q] = in ? (int)sl8[e0 + (int64_t)q * WAVE] : 0;
                        }
                    } else if (col16) {
                        // every offset and value load issued before the first offset is
                        // used (converting each offset as it arrives would serialise them)
#pragma unroll
                        for (int q = 0; q < SB; ++q) {
                            const bool in = q0 + q < len;
                            cc[q] = in ? (int32_t)slo[e0 + (int64_t)(q0 + q) * WAVE] : 0;
                            if constexpr (DICT) vi[q] = in ? (int)sl8[e0 + (int64_t)(q0 + q) * WAVE] : 0;
                            else vv[q] = in ? (WT)slv[e0 + (int64_t)(q0 + q) * WAVE] : (WT)0;
                        }
#pragma unroll
                        for (int q = 0; q < SB; ++q) cc[q] = (q0 + q < len) ? rr + cc[q] : 0;
                    } else {
#pragma unroll
                        for (int q = 0; q < SB; ++q) {
                            const bool in = q0 + q < len;
                            cc[q] = in ? sl_col[e0 + (int64_t)(q0 + q) * WAVE] : 0;
                            if constexpr (DICT) vi[q] = in ? (int)sl8[e0 + (int64_t)(q0 + q) * WAVE] : 0;
                            else vv[q] = in ? (WT)slv[e0 + (int64_t)(q0 + q) * WAVE] : (WT)0;
                        }
                    }
                    if constexpr (DICT && !PFC) {
#pragma unroll
                        for (int q = 0; q < SB; ++q) vv[q] = (q0 + q < len) ? dtab[vi[q]] : (WT)0;
                    }
#pragma unroll
                    for (int q = 0; q < SB; ++q) {
                        xb[q] = first ? (WT)b0p[cc[q]] : Wp[cc[q]];
#pragma unroll
                        for (int o = 0; o < KW; ++o) xu[q][o] = (o < nwin) ? to_w<WT>(gload(Uo[o] + cc[q])) : (WT)0;
                    }
                    if constexpr (PFC) {
                        if (!pf_done) {  // the next slice's column data, behind this slice's gathers
                            prefetch(it + step, iter + 1);
                            pf_done = true;
                        }
#pragma unroll
                        for (int q = 0; q < SB; ++q) vv[q] = (q0 + q < len) ? dtab[vi[q]] : (WT)0;
                    }
#pragma unroll
                    for (int q = 0; q < SB; ++q) {
                        WT x = alpha_w * xb[q];
#pragma unroll
                        for (int o = 0; o < KW; ++o)
                            if (o < nwin) x = fma(cf_w[o], xu[q][o], x);
                        x = to_w<WT>(Store<VT>::put(x));
                        w = fma(vv[q], x, w);
                    }
                }
                if constexpr (PFC) {
                    if (!pf_done) {  // (an empty slice)
                        prefetch(it + step, iter + 1);
                        pf_done = true;
                    }
                }
            } else if (valid) {
                const int e0 = rowptr[r], e1 = rowptr[r + 1];
                for (int e = e0; e < e1; ++e) {
                    const int c = colp[e];
                    WT x = alpha_w * (first ? (WT)b0p[c] : Wp[c]);
#pragma unroll
                    for (int o = 0; o < KW; ++o)
                        if (o < nwin) x = fma(cf_w[o], to_w<WT>(gload(Uo[o] + c)), x);
                    x = to_w<WT>(Store<VT>::put(x));
                    w = fma((WT)valp[e], x, w);
                }
            }
        }
        // u_j at the row, with the same operations as at the gathered columns
        if constexpr (KW > 4) {
            if (valid) {
#pragma unroll
                for (int o = 0; o < KW; ++o)
                    if (o < nwin) urow[o] = gload(Uo[o] + r);
            }
        }
        WT uo[KW];
        WT u = (WT)0;
        if (valid) {
            u = alpha_w * wrow;
#pragma unroll
            for (int o = 0; o < KW; ++o) {
                uo[o] = (o < nwin) ? to_w<WT>(urow[o]) : (WT)0;
                if (o < nwin) u = fma(cf_w[o], uo[o], u);
            }
        } else {
#pragma unroll
            for (int o = 0; o < KW; ++o) uo[o] = (WT)0;
        }
        const VT us = Store<VT>::put(u);
        u = to_w<WT>(us);  // the stored value is the one used everywhere
        if (store_u && valid) store_nt(us, &Uj[r]);
        if (!a.extend && valid) store_nt(w, &Wc[r]);
        if (valid) {
            const double ud = (double)u, wd = (double)w;
            acc_uu = fma(ud, ud, acc_uu);
            acc_uw = fma(ud, wd, acc_uw);
            acc_ww = fma(wd, wd, acc_ww);
#pragma unroll
            for (int o = 0; o < KW - 1; ++o) {
                if (o < ndot) {
                    acc_lw[o] = fma((double)uo[o], wd, acc_lw[o]);
                    acc_ul[o] = fma(ud, (double)uo[o], acc_ul[o]);
                }
            }
            if (sketch) {
                int rows[ZETA];
                double sg[ZETA];
                sketch_column<ZETA>(a.seed, (uint64_t)r, s, rows, sg);
#pragma unroll
                for (int q = 0; q < ZETA; ++q) lds_add(binV + rows[q], sg[q] * ud);
                if (!a.extend && a.sav) {
#pragma unroll
                    for (int q = 0; q < ZETA; ++q) lds_add(binAV + rows[q], sg[q] * wd);
                }
            }
        }
        if (pre && lane == 0) __hip_atomic_fetch_add(&s_prog, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    };
    auto run = [&](auto dict_tag) __attribute__((always_inline)) {
        if constexpr (KW <= 4) {  // (for the widest window the second copy would spill registers)
            if (nwin_all == KW && !first_all) main_loop(std::integral_constant<bool, true>(), dict_tag);
            else main_loop(std::integral_constant<bool, false>(), dict_tag);
        } else {
            main_loop(std::integral_constant<bool, false>(), dict_tag);
        }
    };
    if (dict8 && sell) run(std::integral_constant<bool, true>());
    else run(std::integral_constant<bool, false>());
    __builtin_amdgcn_s_setprio(0);

    // partial sketches, bin-major; slot = chunk keeps one XCD's slots contiguous
    __syncthreads();
    for (int i = tid; i < (a.sav ? 2 * s : s); i += BLOCK) {
        double t = 0.0;
        for (int wv = 0; wv < NW; ++wv) t += bins[wv * 2 * s + i];
        gptr(a.skp_cur)[(int64_t)i * G + chunk] = t;
    }
    // partial scalars of this block, reduced through the (now free) bin region
    double vals[NSC];
    vals[0] = acc_uu; vals[1] = acc_uw; vals[2] = acc_ww;
#pragma unroll
    for (int o = 0; o < KW - 1; ++o) { vals[3 + o] = acc_lw[o]; vals[3 + (KW - 1) + o] = acc_ul[o]; }
    __syncthreads();
    block_reduce_multi<NSC, BLOCK>(vals, bins, red);
    if (tid < NSC) gptr(a.scal_cur)[(int64_t)tid * G + bid] = red[tid];
}

template <int KW, int ZETA, int BLOCK, typename P>
__global__ __launch_bounds__(BLOCK) void arnoldi_step_kernel(StepArgs a) {
    step_body<KW, ZETA, BLOCK, P, false>(a, blockIdx.x);
}

// Unit (problem, right-hand side) of a block of the batched step launch.
// Problems are ordered by decreasing m and problem q owns the blocks
// [base[q], base[q+1]); within it block g' serves right-hand side (g' / 8) % R
// and local block 8 (g' / 8R) + g' % 8, so the R blocks that read the same rows
// of A are dispatched one after another onto the same XCD (A read once from HBM,
// shared through L2) and the local index keeps the XCD-contiguous chunk mapping.
struct BatchLookup {
    int unit;
    int bid;
};

__device__ __forceinline__ BatchLookup batch_lookup(const int* __restrict__ base, int nact, int R, int g) {
    int lo = 0, hi = nact;  // base[lo] <= g < base[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= g) lo = mid; else hi = mid;
    }
    const int gp = g - base[lo];
    BatchLookup r;
    r.unit = lo * R + (gp >> 3) % R;
    r.bid = (gp / (8 * R)) * 8 + (gp & 7);
    return r;
}

template <int KW, int ZETA, int BLOCK, typename P>
__global__ __launch_bounds__(BLOCK) void arnoldi_step_batched_kernel(const BatchStepUnit* __restrict__ units,
                                                                     const int* __restrict__ base, int nact, int R,
                                                                     int j, int g0) {
    const BatchLookup lk = batch_lookup(base, nact, R, g0 + (int)blockIdx.x);
    const BatchStepUnit& u = units[lk.unit];
    StepArgs a = u.a;
    a.j = j;
    a.extend = (j == a.m) ? 1 : 0;
    a.Wcur = u.W[j & 1];
    a.Wprev = u.W[(j + 1) & 1];
    a.scal_prev = u.scal[(j + 1) & 1];
    a.scal_cur = u.scal[j & 1];
    a.skp_prev = u.skp[(j + 1) & 1];
    a.skp_cur = u.skp[j & 1];
    step_body<KW, ZETA, BLOCK, P, true>(a, lk.bid);
}

// ------------------------------------------- batched step: all right-hand sides
// One block serves chunk `bid` of problem q for all R of its right-hand sides
// (units q R .. q R + R - 1): a slice's metadata, column offsets and value
// indices, and a row's sketch hash, are loaded or computed once for all of them,
// and each wavefront has the gathers of every right-hand side in flight at once.
// For the steps 2 <= j < m with k = 2 (full window, no extension pass, no sketch
// of A u_j), SELL form of A.  Chunks, per-wavefront slices, bins, partials and the
// order of every sum are those of the per-unit form (step_body), so the two forms
// agree bit for bit and may alternate from step to step.  A block takes the LDS of
// R sets of bins, [NW][R][s] doubles (R <= RM).
// Load / store at element i of a uniform (per-block) base through a 32-bit byte
// offset: the global instructions then take the base in scalar registers and only
// the offset in a vector register (the host keeps 8 N below 2^32 for this form).
template <typename T>
__device__ __forceinline__ T ld_off(const GAS T* base, uint32_t i) {
    return gload(reinterpret_cast<const GAS T*>(reinterpret_cast<const GAS char*>(base) + i * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st_off(GAS T* base, uint32_t i, T v) {
    store_nt(v, reinterpret_cast<GAS T*>(reinterpret_cast<GAS char*>(base) + i * (uint32_t)sizeof(T)));
}

template <int ZETA, int BLOCK, typename P, int RM>
__global__ __launch_bounds__(BLOCK) void arnoldi_step_packed_kernel(const BatchStepUnit* __restrict__ units,
                                                                    const int* __restrict__ base, int nprob, int R,
                                                                    int j) {
    using VT = typename P::V;
    using WT = typename P::W;
    using AT = typename P::A;
    constexpr int KW = 2;
    constexpr int NSC = 2 * KW + 1;
    constexpr int NW = BLOCK / WAVE;
    constexpr int SB = 5;  // entries per load batch (the gathers of RM units must fit the registers)
    extern __shared__ double bins[];  // [NW][R][s]; the reductions' scratch before and after the loop
    __shared__ double red[RM * NSC];
    __shared__ double coef[RM][KMAX + 2];
    __shared__ double win[RM][KW * KW];
    __shared__ int2 meta[NW][WAVE];
    __shared__ int s_ok[RM];
    __shared__ int s_prog;
    __shared__ WT dtab[DICT_MAX];

    // problem of this block: base[q] = R x (blocks of the problems before q)
    const int g = blockIdx.x;
    int lo = 0, hi = nprob;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= g * R) lo = mid; else hi = mid;
    }
    const int bid = g - base[lo] / R;
    const BatchStepUnit* __restrict__ un = units + (int64_t)lo * R;
    const StepArgs& a0 = un[0].a;  // fields shared by the problem's units
    const int sell_flag = gptr(a0.sctrl)->sell_ok;
    const int col16 = gptr(a0.sctrl)->col16;
    const int dict8 = gptr(a0.sctrl)->dict8;
    const WT dval = (WT)(AT)gptr(a0.sl_table)[threadIdx.x & (DICT_MAX - 1)];
    const int k = a0.k, s = a0.s, G = a0.G;
    const int64_t N = a0.N, ldS = a0.ldS;
    const uint64_t seed = a0.seed;
    const double isz = a0.inv_sqrt_zeta;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int p = j - 1;  // the step whose reductions this block finishes

    const int chunk = xcd_chunk(bid, G);
    const int64_t sl0 = (int64_t)chunk * a0.slices_per_chunk + wid;
    const int64_t sl1 = min(a0.nslices, (int64_t)(chunk + 1) * a0.slices_per_chunk);
    const int64_t itl0 = sl0 + (int64_t)lane * NW;
    const bool win_in = itl0 < sl1;
    const int64_t itl0c = win_in ? itl0 : 0;
    const GAS int32_t* __restrict__ sl_len = gptr(a0.sl_len);
    const GAS int64_t* __restrict__ sl_ptr = gptr(a0.sl_ptr);
    const int wlen = sl_len[itl0c];
    const int64_t wptr = sl_ptr[itl0c];

    // ------------------------------------------------ prologue, every unit
    constexpr int GM = STEP_GMAX_1024 * (1024 / BLOCK);
    constexpr int GPT = (GM + BLOCK - 1) / BLOCK;
    constexpr int GPL = (GM + WAVE - 1) / WAVE;
    bool stopped[RM];
    double sv[RM * NSC];
    double skv[RM];
    const int b0 = (bid * s) / G, b1 = ((bid + 1) * s) / G;
    const int mybin = (b0 + wid < b1) ? b0 + wid : -1;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const bool in = r < R;
        const BatchStepUnit& u = un[in ? r : 0];
        const GAS DevCtrl* cr = gptr(u.a.ctrl);
        stopped[r] = !in || (cr->stop && cr->m_used < j - 1);
        const GAS double* sp = gptr(u.scal[(j + 1) & 1]);
        double ld[NSC][GPT];
#pragma unroll
        for (int q = 0; q < GPT; ++q) {
            const int gg = tid + q * BLOCK, gc = (gg < G) ? gg : 0;
#pragma unroll
            for (int sc = 0; sc < NSC; ++sc) ld[sc][q] = sp[(int64_t)sc * G + gc];
        }
#pragma unroll
        for (int sc = 0; sc < NSC; ++sc) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < GPT; ++q) t = fma((tid + q * BLOCK < G) ? 1.0 : 0.0, ld[sc][q], t);
            sv[r * NSC + sc] = t;
        }
        const double wv = window_value<KW>(u.a, p, tid & (KW * KW - 1));
        if (tid < KW * KW) win[r][tid] = wv;
        double t0 = 0.0, t1 = 0.0;
        if (mybin >= 0) {
            const GAS double* src = gptr(u.skp[(j + 1) & 1]) + (int64_t)mybin * G;
            double lb[GPL];
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                const int gg = lane + q * WAVE;
                lb[q] = src[(gg < G) ? gg : 0];
            }
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                const double mk = (lane + q * WAVE < G) ? 1.0 : 0.0;
                if (q & 1) t1 = fma(mk, lb[q], t1);
                else t0 = fma(mk, lb[q], t0);
            }
        }
        skv[r] = t0 + t1;
    }
    bool any = false;
#pragma unroll
    for (int r = 0; r < RM; ++r) any |= !stopped[r];
    if (!any) return;
    if (tid < DICT_MAX) dtab[tid] = dval;
    block_reduce_multi<RM * NSC, BLOCK>(sv, bins, red);
    if (tid < RM) {  // thread r: the coefficients of unit r
        const int r = tid;
        bool st = true;
#pragma unroll
        for (int q = 0; q < RM; ++q)
            if (q == r) st = stopped[q];
        bool ok = false;
        if (!st) ok = step_coefficients<KW>(red + r * NSC, win[r], p, k, bid == 0, un[r].a, coef[r]);
        s_ok[r] = ok ? 1 : 0;
    }
#pragma unroll
    for (int r = 0; r < RM; ++r) skv[r] = wave_sum(skv[r]);
    if (wid > 0)
        for (int i = tid - WAVE; i < NW * R * s; i += BLOCK - WAVE) bins[i] = 0.0;
    if (tid == WAVE) s_prog = 0;
    __syncthreads();
    bool act[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        act[r] = !stopped[r] && s_ok[r] != 0;
        if (stopped[r]) continue;
        const BatchStepUnit& u = un[r];
        const double eta_p = coef[r][KMAX + 1];
        const bool ok = s_ok[r] != 0;
        if (mybin >= 0 && lane == 0) gptr(u.a.SV)[(int64_t)p * ldS + mybin] = skv[r] * (ok ? isz / eta_p : isz);
        if (b1 - b0 > NW)
            reduce_prev_sketch_tail<BLOCK>(u.skp[(j + 1) & 1], G, s, ldS, p, b0 + NW, b1,
                                           ok ? isz / eta_p : isz, isz / eta_p, false, u.a.SV, u.a.SAV);
    }
    bool anyact = false;
#pragma unroll
    for (int r = 0; r < RM; ++r) anyact |= act[r];
    if (!anyact) return;

    // ------------------------------------------------ main loop
    meta[wid][lane] = win_in ? make_int2(wlen, (int)(wptr >> 6)) : make_int2(0, 0);
    double alpha[RM];
    WT alpha_w[RM], cf_w[RM][KW];
    const GAS WT* Wp[RM];
    const GAS VT* Uo[RM][KW];
    GAS VT* Uj[RM];
    GAS WT* Wc[RM];
    double* binV[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const BatchStepUnit& u = un[act[r] ? r : 0];
        alpha[r] = coef[r][0];
        alpha_w[r] = (WT)alpha[r];
#pragma unroll
        for (int o = 0; o < KW; ++o) cf_w[r][o] = (WT)coef[r][1 + o];
        Wp[r] = gptr(static_cast<const WT*>(u.W[(j + 1) & 1]));
        Wc[r] = gptr(static_cast<WT*>(u.W[j & 1]));
        const int ur = u.a.uring;
#pragma unroll
        for (int o = 0; o < KW; ++o)
            Uo[r][o] = gptr(static_cast<const VT*>(u.a.U)) + (int64_t)((j - 1 - o) % ur) * u.a.ldU;
        Uj[r] = gptr(static_cast<VT*>(u.a.U)) + (int64_t)(j % ur) * u.a.ldU;
        binV[r] = bins + (wid * R + r) * s;
    }
    const GAS AT* __restrict__ slv = gptr(static_cast<const AT*>(a0.sl_val));
    const GAS int32_t* __restrict__ sl_col = gptr(a0.sl_col);
    const GAS int16_t* __restrict__ slo = gptr(reinterpret_cast<const int16_t*>(a0.sl_col));
    const GAS uint8_t* __restrict__ sl8 = gptr(reinterpret_cast<const uint8_t*>(a0.sl_val));
    const GAS int32_t* __restrict__ rowptr = gptr(a0.rowptr);
    const GAS int32_t* __restrict__ colp = gptr(a0.col);
    const GAS double* __restrict__ valp = gptr(a0.val);

    double acc[RM][NSC];
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int i = 0; i < NSC; ++i) acc[r][i] = 0.0;

    const bool sell = sell_flag != 0;
    int64_t it0, it1, step;
    if (sell) {
        it0 = sl0;
        it1 = sl1;
        step = NW;
    } else {
        const int64_t r_begin = (int64_t)chunk * a0.rows_per_chunk;
        it0 = r_begin + tid;
        it1 = min(N, r_begin + a0.rows_per_chunk);
        step = BLOCK;
    }
    auto main_loop = [&](auto dict_tag) __attribute__((always_inline)) {
        constexpr bool DICT = decltype(dict_tag)::value;
        int wbase = 0, iter = 0;
        auto ring = [&](int64_t itn, int idx) {
            if (idx - wbase == WAVE) {
                wbase += WAVE;
                const int64_t itl = itn + (int64_t)lane * step;
                const int nl = (itl < it1) ? sl_len[itl] : 0;
                const int np = (itl < it1) ? (int)(sl_ptr[itl] >> 6) : 0;
                meta[wid][lane] = make_int2(nl, np);
            }
            return meta[wid][idx - wbase];
        };
        for (int64_t it = it0; it < it1; it += step, ++iter) {
            const int64_t rw = sell ? it * WAVE + lane : it;
            const bool valid = rw < N;
            int len = 0;
            int64_t e0 = 0;
            if (sell) {
                const int done = __hip_atomic_load(&s_prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (done > iter * NW) __builtin_amdgcn_s_setprio(3);
                else __builtin_amdgcn_s_setprio(0);
                const int2 md = ring(it, iter);
                len = md.x;
                e0 = ((int64_t)md.y << 6) + lane;
            }
            WT wrow[RM];
            VT urow[RM][KW];
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                wrow[r] = (WT)0;
                if (valid && act[r]) {
                    wrow[r] = ld_off(Wp[r], (uint32_t)rw);
#pragma unroll
                    for (int o = 0; o < KW; ++o) urow[r][o] = ld_off(Uo[r][o], (uint32_t)rw);
                }
            }
            WT w[RM];
#pragma unroll
            for (int r = 0; r < RM; ++r) w[r] = (WT)0;
            if (sell) {
                const int32_t rr = valid ? (int32_t)rw : 0;
                for (int q0 = 0; q0 < len; q0 += SB) {
                    int cc[SB], vi[SB];
                    WT vv[SB];
#pragma unroll
                    for (int q = 0; q < SB; ++q) {
                        const bool in = q0 + q < len;
                        cc[q] = in ? (col16 ? (int32_t)slo[e0 + (int64_t)(q0 + q) * WAVE]
                                            : sl_col[e0 + (int64_t)(q0 + q) * WAVE]) : 0;
                        if constexpr (DICT) vi[q] = in ? (int)sl8[e0 + (int64_t)(q0 + q) * WAVE] : 0;
                        else vv[q] = in ? (WT)slv[e0 + (int64_t)(q0 + q) * WAVE] : (WT)0;
                    }
                    if (col16) {
#pragma unroll
                        for (int q = 0; q < SB; ++q) cc[q] = (q0 + q < len) ? rr + cc[q] : 0;
                    }
                    if constexpr (DICT) {
#pragma unroll
                        for (int q = 0; q < SB; ++q) vv[q] = (q0 + q < len) ? dtab[vi[q]] : (WT)0;
                    }
                    WT xb[RM][SB], xu[RM][SB][KW];
#pragma unroll
                    for (int r = 0; r < RM; ++r) {
                        if (!act[r]) continue;
#pragma unroll
                        for (int q = 0; q < SB; ++q) {
                            xb[r][q] = ld_off(Wp[r], (uint32_t)cc[q]);
#pragma unroll
                            for (int o = 0; o < KW; ++o) xu[r][q][o] = to_w<WT>(ld_off(Uo[r][o], (uint32_t)cc[q]));
                        }
                    }
#pragma unroll
                    for (int r = 0; r < RM; ++r) {
                        if (!act[r]) continue;
#pragma unroll
                        for (int q = 0; q < SB; ++q) {
                            WT x = alpha_w[r] * xb[r][q];
#pragma unroll
                            for (int o = 0; o < KW; ++o) x = fma(cf_w[r][o], xu[r][q][o], x);
                            x = to_w<WT>(Store<VT>::put(x));
                            w[r] = fma(vv[q], x, w[r]);
                        }
                    }
                }
            } else if (valid) {
                const int e0r = rowptr[rw], e1r = rowptr[rw + 1];
                for (int e = e0r; e < e1r; ++e) {
                    const int c = colp[e];
                    const WT av = (WT)valp[e];
#pragma unroll
                    for (int r = 0; r < RM; ++r) {
                        if (!act[r]) continue;
                        WT x = alpha_w[r] * Wp[r][c];
#pragma unroll
                        for (int o = 0; o < KW; ++o) x = fma(cf_w[r][o], to_w<WT>(gload(Uo[r][o] + c)), x);
                        x = to_w<WT>(Store<VT>::put(x));
                        w[r] = fma(av, x, w[r]);
                    }
                }
            }
            if (valid) {
                int rows[ZETA];
                double sg[ZETA];
                sketch_column<ZETA>(seed, (uint64_t)rw, s, rows, sg);
#pragma unroll
                for (int r = 0; r < RM; ++r) {
                    if (!act[r]) continue;
                    WT u = alpha_w[r] * wrow[r];
                    WT uo[KW];
#pragma unroll
                    for (int o = 0; o < KW; ++o) {
                        uo[o] = to_w<WT>(urow[r][o]);
                        u = fma(cf_w[r][o], uo[o], u);
                    }
                    const VT us = Store<VT>::put(u);
                    u = to_w<WT>(us);
                    st_off(Uj[r], (uint32_t)rw, us);
                    st_off(Wc[r], (uint32_t)rw, w[r]);
                    const double ud = (double)u, wd = (double)w[r];
                    acc[r][0] = fma(ud, ud, acc[r][0]);
                    acc[r][1] = fma(ud, wd, acc[r][1]);
                    acc[r][2] = fma(wd, wd, acc[r][2]);
                    acc[r][3] = fma((double)uo[0], wd, acc[r][3]);
                    acc[r][4] = fma(ud, (double)uo[0], acc[r][4]);
#pragma unroll
                    for (int q = 0; q < ZETA; ++q) lds_add(binV[r] + rows[q], sg[q] * ud);
                }
            }
            if (sell && lane == 0) __hip_atomic_fetch_add(&s_prog, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };
    if (dict8 && sell) main_loop(std::integral_constant<bool, true>());
    else main_loop(std::integral_constant<bool, false>());
    __builtin_amdgcn_s_setprio(0);

    // ------------------------------------------------ epilogue, every unit
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        if (!act[r]) continue;
        GAS double* dst = gptr(un[r].skp[j & 1]);
        for (int i = tid; i < s; i += BLOCK) {
            double t = 0.0;
            for (int wv = 0; wv < NW; ++wv) t += bins[(wv * R + r) * s + i];
            dst[(int64_t)i * G + chunk] = t;
        }
    }
    double vals[RM * NSC];
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int i = 0; i < NSC; ++i) vals[r * NSC + i] = acc[r][i];
    __syncthreads();
    block_reduce_multi<RM * NSC, BLOCK>(vals, bins, red);
    if (tid < RM * NSC) {
        const int r = tid / NSC, i = tid % NSC;
        if (act[r]) gptr(un[r].scal[j & 1])[(int64_t)i * G + bid] = red[tid];
    }
}

// After the extension step m: S u_m (unnormalised) into SV[:, m_used], eta_m and
// h_{m+1,m} (unless the recurrence broke down earlier, in which case the step
// that detected it already wrote the extension column), then ||S v_j||^2 for the
// epsilon monitor.  One wavefront per sketch bin in the first ceil(s/4) blocks.
__device__ __forceinline__ void tail_body(const StepArgs& a) {
    const int m = a.m, s = a.s, G = a.G;
    const int lane = threadIdx.x & 63;
    const int bin = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (a.ctrl->stop) return;
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        double v = 0.0;
        for (int g = lane; g < G; g += 64) v += a.scal_prev[g];
        v = wave_sum_fast(v);
        if (lane == 0) {
            a.eta[m] = sqrt(v);
            a.H[m + a.ldH * (m - 1)] = sqrt(v);
        }
    }
    if (bin < s) {
        const double* src = a.skp_prev + (int64_t)bin * G;
        double t0 = 0.0, t1 = 0.0;
        int g = lane;
        for (; g + 64 < G; g += 128) { t0 += src[g]; t1 += src[g + 64]; }
        if (g < G) t0 += src[g];
        const double t = wave_sum_fast(t0 + t1);
        if (lane == 0) a.SV[(int64_t)m * a.ldS + bin] = t * a.inv_sqrt_zeta;
    }
}

__global__ __launch_bounds__(256) void arnoldi_tail_kernel(StepArgs a) { tail_body(a); }

// Batched tail: blockIdx.y = unit, arguments of its last (extension) step.
__global__ __launch_bounds__(256) void arnoldi_tail_batched_kernel(const BatchStepUnit* __restrict__ units) {
    const BatchStepUnit& u = units[blockIdx.y];
    StepArgs a = u.a;
    a.scal_prev = u.scal[a.m & 1];
    a.skp_prev = u.skp[a.m & 1];
    tail_body(a);
}

// ||S v_j||^2 for the epsilon monitor, one wavefront per column.
__device__ __forceinline__ void colnorm_body(const double* SV, int s, int m, const DevCtrl* ctrl,
                                             double* colnorm2) {
    const int lane = threadIdx.x & 63;
    const int jj = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (jj >= m) return;
    const int mu = ctrl->m_used;
    double t = 0.0;
    if (jj < mu)
        for (int i = lane; i < s; i += 64) {
            const double x = SV[(int64_t)jj * s + i];
            t = fma(x, x, t);
        }
    t = wave_sum_fast(t);
    if (lane == 0) colnorm2[jj] = (jj < mu) ? t : 1.0;
}

__global__ __launch_bounds__(256) void colnorm_kernel(const double* SV, int s, int m, const DevCtrl* ctrl,
                                                      double* colnorm2) {
    colnorm_body(SV, s, m, ctrl, colnorm2);
}

__global__ __launch_bounds__(256) void colnorm_batched_kernel(const SmallUnit* __restrict__ units, int s, int m) {
    const SmallUnit& u = units[blockIdx.y];
    colnorm_body(u.SV, s, m, u.ctrl, u.colnorm2);
}

// relres = ||SAV - [SV, S u] Hbar1||_F / ||SAV||_F over the first m_used columns,
// Hbar1 = [H; e_mu^T] (Arnoldi relation in the sketched space).  One block per
// column, partial sums in part[2 m]; the last block to finish would need an
// atomic, so the final sum is taken by the small-problem kernels instead.
__device__ __forceinline__ void check_body(const double* SV, const double* SAV, const double* H, int s, int m,
                                           int k, const DevCtrl* ctrl, double* part) {
    __shared__ double scratch[4];
    const int mu = ctrl->m_used;
    const int jj = blockIdx.x;
    double num = 0.0, den = 0.0;
    if (jj < mu) {
        for (int i = threadIdx.x; i < s; i += 256) {
            double t = SAV[(int64_t)jj * s + i];
            den = fma(t, t, den);
            for (int l = max(0, jj - k + 1); l <= jj + 1; ++l) {
                const double hb = (l == jj + 1) ? ((jj == mu - 1) ? 1.0 : H[(jj + 1) + (int64_t)(m + 1) * jj])
                                                : H[l + (int64_t)(m + 1) * jj];
                t = fma(-SV[(int64_t)l * s + i], hb, t);
            }
            num = fma(t, t, num);
        }
    }
    num = block_sum(num, scratch);
    den = block_sum(den, scratch);
    if (threadIdx.x == 0) { part[jj] = num; part[m + jj] = den; }
}

__global__ __launch_bounds__(256) void arnoldi_check_kernel(const double* SV, const double* SAV, const double* H,
                                                           int s, int m, int k, const DevCtrl* ctrl, double* part) {
    check_body(SV, SAV, H, s, m, k, ctrl, part);
}

__global__ __launch_bounds__(256) void arnoldi_check_batched_kernel(const SmallUnit* __restrict__ units, int s, int m,
                                                                   int k) {
    const SmallUnit& u = units[blockIdx.y];
    check_body(u.SV, u.SAV, u.H, s, m, k, u.ctrl, u.chk);
}

__device__ __forceinline__ void check_finish_body(const double* part, int m, DevCtrl* ctrl) {
    __shared__ double scratch[4];
    double num = 0.0, den = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) { num += part[i]; den += part[m + i]; }
    num = block_sum(num, scratch);
    den = block_sum(den, scratch);
    if (threadIdx.x == 0) ctrl->relres = (den > 0.0) ? sqrt(num / den) : 0.0;
}

__global__ __launch_bounds__(256) void arnoldi_check_finish_kernel(const double* part, int m, DevCtrl* ctrl) {
    check_finish_body(part, m, ctrl);
}

__global__ __launch_bounds__(256) void arnoldi_check_finish_batched_kernel(const SmallUnit* __restrict__ units, int m) {
    const SmallUnit& u = units[blockIdx.y];
    check_finish_body(u.chk, m, u.ctrl);
}

// V[:, j] = U[:, j] / eta_j (zero beyond m_used); test hook only.
template <typename VT>
__global__ void normalize_basis_kernel(const VT* U, int64_t ldU, int64_t N, int m,
                                       const DevCtrl* ctrl, const double* eta, double* V) {
    const int j = blockIdx.y;
    const int m_used = ctrl->m_used;
    const double sc = (j < m_used) ? 1.0 / eta[j] : 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x)
        V[(int64_t)j * N + r] = (j < m_used) ? to_w<double>(U[(int64_t)j * ldU + r]) * sc : 0.0;
}

// ------------------------------------------------------ SELL-64 conversion
// Value set of A (open addressing over DICT_SLOTS slots, linear probing).
__device__ __forceinline__ int dict_hash(uint64_t bits) { return (int)((bits * 0x9E3779B97F4A7C15ull) >> 55); }

// Inserts `bits` into a set in LDS: 1 if it was not there, 0 if it was, -1 if full.
__device__ __forceinline__ int dict_insert_lds(uint64_t* keys, uint64_t bits) {
    const int h = dict_hash(bits);
    for (int t = 0; t < DICT_SLOTS; ++t) {
        const int sl = (h + t) & (DICT_SLOTS - 1);
        const uint64_t k = keys[sl];
        if (k == bits) return 0;
        if (k == DICT_EMPTY) {
            const uint64_t prev = atomicCAS((unsigned long long*)&keys[sl], (unsigned long long)DICT_EMPTY,
                                            (unsigned long long)bits);
            if (prev == DICT_EMPTY) return 1;
            if (prev == bits) return 0;
        }
    }
    return -1;
}

// The same for the matrix's set in device memory (agent-scope atomics: blocks on
// every XCD insert into it); counts the values in ctrl->ndict.
__device__ __forceinline__ bool dict_insert_global(DictBuf* d, DevCtrl* ctrl, uint64_t bits) {
    const int h = dict_hash(bits);
    for (int t = 0; t < DICT_SLOTS; ++t) {
        const int sl = (h + t) & (DICT_SLOTS - 1);
        const uint64_t k = __hip_atomic_load(&d->keys[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == bits) return true;
        if (k == DICT_EMPTY) {
            const uint64_t prev = atomicCAS((unsigned long long*)&d->keys[sl], (unsigned long long)DICT_EMPTY,
                                            (unsigned long long)bits);
            if (prev == DICT_EMPTY) {
                atomicAdd(&ctrl->ndict, 1);
                return true;
            }
            if (prev == bits) return true;
        }
    }
    return false;
}

// The matrix's value set emptied, with 0.0 (the padding value) in it; one block.
__global__ __launch_bounds__(DICT_SLOTS) void sell_dict_reset_kernel(DictBuf* d, DevCtrl* ctrl) {
    const int t = threadIdx.x;
    d->keys[t] = (t == dict_hash(0ull)) ? 0ull : DICT_EMPTY;
    if (t == 0) {
        ctrl->ndict = 1;
        ctrl->dict_over = 0;
        ctrl->dict8 = 0;
    }
}

// sl_len[sl] = max row length in slice sl (one wavefront per slice); ctrl->col_wide
// is raised when a column lies outside [row - 32768, row + 32767], i.e. when the
// 16-bit offset form of the column indices cannot be used.  With use_dict, every
// value of A goes into the matrix's value set (through a per-block set in LDS, so
// that only values new to the block reach device memory); ctrl->dict_over is raised
// when the set overflows.
__global__ __launch_bounds__(256) void sell_len_kernel(const int32_t* rowptr, const int32_t* col, const double* val,
                                                       int64_t N, int64_t nslices, int32_t* sl_len, DevCtrl* ctrl,
                                                       DictBuf* dict, int use_dict) {
    __shared__ uint64_t lkeys[DICT_SLOTS];
    const int lane = threadIdx.x & 63;
    if (use_dict) {
        for (int t = threadIdx.x; t < DICT_SLOTS; t += 256) lkeys[t] = DICT_EMPTY;
        __syncthreads();
    }
    bool over = false;
    uint64_t last = 0ull;  // the lane's last value found in the set (0.0 is always there)
    for (int64_t sl = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); sl < nslices; sl += (int64_t)gridDim.x * 4) {
        const int64_t r = sl * 64 + lane;
        const int e0 = (r < N) ? rowptr[r] : 0, e1 = (r < N) ? rowptr[r + 1] : 0;
        int len = e1 - e0;
        int wide = 0;
        // entries in groups of 8: all loads of a group issued before any is used
        for (int g0 = e0; g0 < e1; g0 += 8) {
            int cb[8];
            uint64_t vb[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool in = g0 + q < e1;
                cb[q] = in ? col[g0 + q] : (int)r;
                vb[q] = (in && use_dict) ? (uint64_t)__double_as_longlong(val[g0 + q]) : 0ull;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t d = (int64_t)cb[q] - r;
                wide |= (d < -32768 || d > 32767) ? 1 : 0;
                const uint64_t bits = vb[q];
                if (use_dict && !over && bits != last) {
                    const int ins = (bits == DICT_EMPTY) ? -1 : dict_insert_lds(lkeys, bits);
                    if (ins < 0 || (ins == 1 && !dict_insert_global(dict, ctrl, bits))) over = true;
                    last = bits;
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            len = max(len, __shfl_xor(len, off, 64));
            wide |= __shfl_xor(wide, off, 64);
        }
        if (lane == 0) {
            sl_len[sl] = len;
            if (wide) atomicOr(&ctrl->col_wide, 1);
        }
    }
    if (over) atomicOr(&ctrl->dict_over, 1);
}

constexpr int SCAN_CH = 4096;  // slices per scan block

// per-block sums of 64 * sl_len
__global__ __launch_bounds__(1024) void sell_scan_sums_kernel(const int32_t* sl_len, int64_t nslices, int64_t* bsum) {
    __shared__ double scratch[16];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CH;
    double t = 0.0;  // exact for totals below 2^53
    for (int i = threadIdx.x; i < SCAN_CH; i += 1024)
        if (base + i < nslices) t += 64.0 * sl_len[base + i];
    t = block_sum(t, scratch);
    if (threadIdx.x == 0) bsum[blockIdx.x] = (int64_t)t;
}

// Exclusive prefix sum of one value per thread over a block of 1024 threads
// (integers: exact in any order), and the block total.  Scans within each
// wavefront by shuffles, then across the 16 wavefront totals.
__device__ __forceinline__ int64_t block_exclusive_scan_1024(int64_t v, int64_t* wsum, int64_t* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int64_t w = (lane < 16) ? wsum[lane] : 0;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const int64_t y = __shfl_up(w, off, 64);
            if (lane >= off) w += y;
        }
        if (lane < 16) wsum[16 + lane] = w;  // inclusive scan of the wavefront totals
    }
    __syncthreads();
    *total = wsum[16 + 15];
    return ((wid > 0) ? wsum[16 + wid - 1] : 0) + x - v;
}

// exclusive scan of the block sums (one block: a sequential sum per thread, then
// the block scan)
__global__ __launch_bounds__(1024) void sell_scan_top_kernel(int64_t* bsum, int64_t nb, int64_t capacity,
                                                             DevCtrl* ctrl, DictBuf* dict, int use_dict) {
    __shared__ int64_t wsum[32];
    __shared__ int sh_ok;
    __shared__ int wcnt[16];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t i0 = threadIdx.x * per, i1 = min(nb, i0 + per);
    int64_t t = 0;
    for (int64_t i = i0; i < i1; ++i) t += bsum[i];
    int64_t total = 0;
    int64_t run = block_exclusive_scan_1024(t, wsum, &total);
    if (threadIdx.x == 0) {
        ctrl->sell_total = total;
        ctrl->sell_ok = (total <= capacity) ? 1 : 0;
        ctrl->col16 = ctrl->col_wide ? 0 : 1;
        sh_ok = (total <= capacity) ? 1 : 0;
    }
    __syncthreads();
    for (int64_t i = i0; i < i1; ++i) { const int64_t v = bsum[i]; bsum[i] = run; run += v; }
    // value table: the occupied slots of the value set numbered in slot order
    const bool use = use_dict && sh_ok && !ctrl->dict_over && ctrl->ndict <= DICT_MAX;
    const int tid = threadIdx.x;
    uint64_t k = DICT_EMPTY;
    if (use && tid < DICT_SLOTS) k = dict->keys[tid];
    const bool occ = k != DICT_EMPTY;
    const uint64_t mask = __ballot(occ);
    if ((tid & 63) == 0) wcnt[tid >> 6] = __popcll(mask);
    __syncthreads();
    if (use && tid < DICT_SLOTS) {
        int idx = __popcll(mask & ((1ull << (tid & 63)) - 1ull));
        for (int w = 0; w < (tid >> 6); ++w) idx += wcnt[w];
        dict->slot_idx[tid] = occ ? idx : -1;
        if (occ) dict->table[idx] = __longlong_as_double((long long)k);
    }
    if (tid == 0) ctrl->dict8 = use ? 1 : 0;
}

// sl_ptr = exclusive prefix of 64 * sl_len (block-local scan plus block offset)
__global__ __launch_bounds__(1024) void sell_scan_apply_kernel(const int32_t* sl_len, int64_t nslices,
                                                               const int64_t* boff, int64_t* sl_ptr) {
    __shared__ int64_t wsum[32];
    constexpr int PER = SCAN_CH / 1024;
    const int64_t base = (int64_t)blockIdx.x * SCAN_CH + (int64_t)threadIdx.x * PER;
    int64_t loc[PER];
    int64_t t = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        loc[i] = (base + i < nslices) ? 64 * (int64_t)sl_len[base + i] : 0;
        t += loc[i];
    }
    int64_t total = 0;
    int64_t run = boff[blockIdx.x] + block_exclusive_scan_1024(t, wsum, &total);
    for (int i = 0; i < PER; ++i) {
        if (base + i < nslices) sl_ptr[base + i] = run;
        run += loc[i];
    }
}

// interleaved copy; padding entries have value 0 and their own row as column
// (offset 0 in the int16 form, also for the rows beyond N of the last slice)
template <typename AT>
__global__ __launch_bounds__(256) void sell_fill_kernel(const int32_t* rowptr, const int32_t* col, const double* val,
                                                        int64_t N, int64_t nslices, const DevCtrl* ctrl,
                                                        const int64_t* sl_ptr, const int32_t* sl_len,
                                                        int32_t* sl_col, AT* sl_val, const DictBuf* dict) {
    __shared__ uint64_t lkeys[DICT_SLOTS];
    __shared__ int lidx[DICT_SLOTS];
    if (!ctrl->sell_ok) return;
    const bool c16 = ctrl->col16 != 0;
    const bool d8 = ctrl->dict8 != 0;
    if (d8) {  // (block-uniform)
        for (int t = threadIdx.x; t < DICT_SLOTS; t += 256) {
            lkeys[t] = dict->keys[t];
            lidx[t] = dict->slot_idx[t];
        }
        __syncthreads();
    }
    // table index of a value (every value of A, and 0.0, is in the set)
    auto index_of = [&](double v) -> uint8_t {
        const uint64_t bits = (uint64_t)__double_as_longlong(v);
        const int h = dict_hash(bits);
        for (int t = 0; t < DICT_SLOTS; ++t) {
            const int sl = (h + t) & (DICT_SLOTS - 1);
            if (lkeys[sl] == bits) return (uint8_t)lidx[sl];
        }
        return 0;
    };
    int16_t* sl_off = reinterpret_cast<int16_t*>(sl_col);
    uint8_t* sl_v8 = reinterpret_cast<uint8_t*>(sl_val);
    const int lane = threadIdx.x & 63;
    for (int64_t sl = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); sl < nslices; sl += (int64_t)gridDim.x * 4) {
        const int64_t r = sl * 64 + lane;
        const int len = sl_len[sl];
        const int e0 = (r < N) ? rowptr[r] : 0;
        const int rl = (r < N) ? rowptr[r + 1] - e0 : 0;
        const int32_t self = (r < N) ? (int32_t)r : 0;
        const int64_t o = sl_ptr[sl] + lane;
        for (int q0 = 0; q0 < len; q0 += 8) {
            int cb[8];
            double vb[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool real = q0 + q < rl;
                cb[q] = real ? col[e0 + q0 + q] : self;
                vb[q] = real ? val[e0 + q0 + q] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (q0 + q < len) {
                    if (c16) sl_off[o + (int64_t)(q0 + q) * 64] = (int16_t)((r < N) ? cb[q] - r : 0);
                    else sl_col[o + (int64_t)(q0 + q) * 64] = cb[q];
                    if (d8) sl_v8[o + (int64_t)(q0 + q) * 64] = index_of(vb[q]);
                    else sl_val[o + (int64_t)(q0 + q) * 64] = (AT)vb[q];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- launchers
template <int KW, int ZETA, typename P>
static hipError_t launch_step_t(const StepArgs& a, int block, hipStream_t st) {
    // the dynamic region holds the per-wave sketch bins, and in the prologue and
    // epilogue the scratch of the (2 KW + 1)-value block reduction
    const size_t bins = (size_t)(block / WAVE) * 2 * a.s;
    const size_t red = (size_t)(2 * KW + 1) * (block + 72);
    const size_t lds = (bins > red ? bins : red) * sizeof(double);
    if (block == 1024) {
        hipLaunchKernelGGL((arnoldi_step_kernel<KW, ZETA, 1024, P>), dim3(a.G), dim3(1024), lds, st, a);
    } else if (block == 512) {
        hipLaunchKernelGGL((arnoldi_step_kernel<KW, ZETA, 512, P>), dim3(a.G), dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL((arnoldi_step_kernel<KW, ZETA, 256, P>), dim3(a.G), dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

template <int ZETA>
static hipError_t launch_step_z(const StepArgs& a, int block, hipStream_t st) {
    switch (a.k) {
        case 1: return launch_step_t<1, ZETA, PrecF64>(a, block, st);
        case 2: return launch_step_t<2, ZETA, PrecF64>(a, block, st);
        case 3: return launch_step_t<3, ZETA, PrecF64>(a, block, st);
        case 4: return launch_step_t<4, ZETA, PrecF64>(a, block, st);
        default: return launch_step_t<8, ZETA, PrecF64>(a, block, st);
    }
}

// reduced precision: zeta = 8, k <= 4
template <typename P>
static hipError_t launch_step_p(const StepArgs& a, int block, hipStream_t st) {
    switch (a.k) {
        case 1: return launch_step_t<1, 8, P>(a, block, st);
        case 2: return launch_step_t<2, 8, P>(a, block, st);
        case 3: return launch_step_t<3, 8, P>(a, block, st);
        default: return launch_step_t<4, 8, P>(a, block, st);
    }
}

// ----------------------------------------------------------- launch rule
// Largest step-kernel block (from `block` down to 256) whose LDS fits the CU's
// 160 KiB with 4 KiB spare: per-wave sketch bins (2s doubles, shared with the
// reduction scratch) and the per-wave slice-metadata ring (64 x 8 bytes).
int step_block_fit(int block, int s) {
    const size_t lds_budget = 156 * 1024;
    auto lds_of = [&](int bl) {
        const size_t bins = (size_t)(bl / 64) * 2 * s, red = (size_t)(2 * KMAX + 1) * (bl + 72);
        return (bins > red ? bins : red) * sizeof(double) + (size_t)(bl / 64) * 64 * 8 + DICT_MAX * sizeof(double);
    };
    while (block > 256 && lds_of(block) > lds_budget) block /= 2;
    return block;
}

Launch step_launch(int64_t N, int s, int k) {
    // windows wider than 4 (k > 4) need more than the 128 registers per thread that
    // a 1024-thread block leaves; 512-thread blocks allow 256
    int block = step_block_fit(k > 4 ? 512 : 1024, s);
    if (N < (int64_t)block * 256) block = 256;  // small problems: more, smaller blocks
    Launch L;
    L.block = block;
    L.nslices = (N + 63) / 64;
    const int waves = block / 64;
    int64_t G = (L.nslices + waves - 1) / waves;
    const int64_t gmax = (int64_t)STEP_GMAX_1024 * (1024 / block);
    if (G > gmax) G = gmax;
    G = (G + 7) / 8 * 8;
    L.G = (int)G;
    L.slices_per_chunk = (L.nslices + G - 1) / G;
    L.rows_per_chunk = (N + G - 1) / G;
    return L;
}

hipError_t launch_arnoldi_step(const StepArgs& a, int zeta, int block, int prec, hipStream_t st) {
    if (prec == 1) return launch_step_p<PrecF32>(a, block, st);
    if (prec == 2) return launch_step_p<PrecBF16>(a, block, st);
    switch (zeta) {
        case 2: return launch_step_z<2>(a, block, st);
        case 4: return launch_step_z<4>(a, block, st);
        case 16: return launch_step_z<16>(a, block, st);
        default: return launch_step_z<8>(a, block, st);
    }
}

hipError_t launch_arnoldi_tail(const StepArgs& a, double* colnorm2, hipStream_t st) {
    hipLaunchKernelGGL(arnoldi_tail_kernel, dim3((a.s + 3) / 4), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colnorm_kernel, dim3((a.m + 3) / 4), dim3(256), 0, st, a.SV, a.s, a.m, a.ctrl, colnorm2);
    return hipGetLastError();
}

hipError_t launch_colnorm(const double* SV, int s, int m, const DevCtrl* ctrl, double* colnorm2, hipStream_t st) {
    hipLaunchKernelGGL(colnorm_kernel, dim3((m + 3) / 4), dim3(256), 0, st, SV, s, m, ctrl, colnorm2);
    return hipGetLastError();
}

hipError_t launch_arnoldi_check(const double* SV, const double* SAV, const double* H, int s, int m, int k,
                                DevCtrl* ctrl, double* part, hipStream_t st) {
    hipLaunchKernelGGL(arnoldi_check_kernel, dim3(m), dim3(256), 0, st, SV, SAV, H, s, m, k, ctrl, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(arnoldi_check_finish_kernel, dim3(1), dim3(256), 0, st, part, m, ctrl);
    return hipGetLastError();
}

hipError_t launch_normalize_basis(const void* U, int64_t ldU, int64_t N, int m, const DevCtrl* ctrl,
                                  const double* eta, double* V, int prec, hipStream_t st) {
    int64_t gx64 = (N + 255) / 256;
    int gx = (int)(gx64 < 1024 ? gx64 : 1024);
    if (prec == 1)
        hipLaunchKernelGGL(normalize_basis_kernel<float>, dim3(gx, m), dim3(256), 0, st, static_cast<const float*>(U),
                           ldU, N, m, ctrl, eta, V);
    else if (prec == 2)
        hipLaunchKernelGGL(normalize_basis_kernel<bf16s>, dim3(gx, m), dim3(256), 0, st, static_cast<const bf16s*>(U),
                           ldU, N, m, ctrl, eta, V);
    else
        hipLaunchKernelGGL(normalize_basis_kernel<double>, dim3(gx, m), dim3(256), 0, st,
                           static_cast<const double*>(U), ldU, N, m, ctrl, eta, V);
    return hipGetLastError();
}

int64_t sell_scan_blocks(int64_t nslices) { return (nslices + SCAN_CH - 1) / SCAN_CH; }

hipError_t launch_sell_convert(const int32_t* rowptr, const int32_t* col, const double* val, int64_t N,
                               int64_t nslices, int64_t capacity, DevCtrl* ctrl, int32_t* sl_len, int64_t* sl_ptr,
                               int64_t* bsum, int32_t* sl_col, void* sl_val, DictBuf* dict, int use_dict, int prec,
                               hipStream_t st) {
    const int64_t g64 = (nslices + 3) / 4;
    const unsigned g = (unsigned)(g64 < 65536 ? g64 : 65536);
    hipLaunchKernelGGL(sell_dict_reset_kernel, dim3(1), dim3(DICT_SLOTS), 0, st, dict, ctrl);
    hipLaunchKernelGGL(sell_len_kernel, dim3(g), dim3(256), 0, st, rowptr, col, val, N, nslices, sl_len, ctrl, dict,
                       use_dict);
    const int64_t nb = sell_scan_blocks(nslices);
    hipLaunchKernelGGL(sell_scan_sums_kernel, dim3((unsigned)nb), dim3(1024), 0, st, sl_len, nslices, bsum);
    hipLaunchKernelGGL(sell_scan_top_kernel, dim3(1), dim3(1024), 0, st, bsum, nb, capacity, ctrl, dict, use_dict);
    hipLaunchKernelGGL(sell_scan_apply_kernel, dim3((unsigned)nb), dim3(1024), 0, st, sl_len, nslices, bsum, sl_ptr);
    if (prec == 0)
        hipLaunchKernelGGL(sell_fill_kernel<double>, dim3(g), dim3(256), 0, st, rowptr, col, val, N, nslices, ctrl,
                           sl_ptr, sl_len, sl_col, static_cast<double*>(sl_val), dict);
    else
        hipLaunchKernelGGL(sell_fill_kernel<float>, dim3(g), dim3(256), 0, st, rowptr, col, val, N, nslices, ctrl,
                           sl_ptr, sl_len, sl_col, static_cast<float*>(sl_val), dict);
    return hipGetLastError();
}


// ------------------------------------------------------- batched launchers
template <int KW, int ZETA, typename P>
static hipError_t launch_step_batched_t(const BatchStepUnit* units, const int* base, int nact, int R, int j,
                                        int g0, int grid, int block, int smax, hipStream_t st) {
    const size_t bins = (size_t)(block / WAVE) * 2 * smax;
    const size_t red = (size_t)(2 * KW + 1) * (block + 72);
    const size_t lds = (bins > red ? bins : red) * sizeof(double);
    if (block == 1024)
        hipLaunchKernelGGL((arnoldi_step_batched_kernel<KW, ZETA, 1024, P>), dim3(grid), dim3(1024), lds, st, units,
                           base, nact, R, j, g0);
    else if (block == 512)
        hipLaunchKernelGGL((arnoldi_step_batched_kernel<KW, ZETA, 512, P>), dim3(grid), dim3(512), lds, st, units,
                           base, nact, R, j, g0);
    else
        hipLaunchKernelGGL((arnoldi_step_batched_kernel<KW, ZETA, 256, P>), dim3(grid), dim3(256), lds, st, units,
                           base, nact, R, j, g0);
    return hipGetLastError();
}

template <typename P>
static hipError_t launch_step_batched_p(const BatchStepUnit* units, const int* base, int nact, int R, int j, int k,
                                        int g0, int grid, int block, int smax, hipStream_t st) {
    switch (k) {
        case 1: return launch_step_batched_t<1, 8, P>(units, base, nact, R, j, g0, grid, block, smax, st);
        case 2: return launch_step_batched_t<2, 8, P>(units, base, nact, R, j, g0, grid, block, smax, st);
        case 3: return launch_step_batched_t<3, 8, P>(units, base, nact, R, j, g0, grid, block, smax, st);
        default: return launch_step_batched_t<4, 8, P>(units, base, nact, R, j, g0, grid, block, smax, st);
    }
}

// Batched step launch (sketch density 8, k <= 4), per-unit form: `grid` blocks
// starting at block g0 of the launch plan, the first nact problems (by decreasing
// m) active.
hipError_t launch_arnoldi_step_batched(const BatchStepUnit* units, const int* base, int nact, int R, int j, int k,
                                       int g0, int grid, int block, int smax, int prec, hipStream_t st) {
    if (prec == 1) return launch_step_batched_p<PrecF32>(units, base, nact, R, j, k, g0, grid, block, smax, st);
    if (prec == 2) return launch_step_batched_p<PrecBF16>(units, base, nact, R, j, k, g0, grid, block, smax, st);
    return launch_step_batched_p<PrecF64>(units, base, nact, R, j, k, g0, grid, block, smax, st);
}

// LDS of the packed form's block (dynamic part: R sets of bins per wavefront, or
// the reductions' scratch), or 0 when it does not fit beside the static part.
size_t packed_step_lds(int block, int R, int smax) {
    constexpr int RM = PACKED_RMAX, NSC = 5;
    if (block != PACKED_BLOCK || R < 1 || R > RM) return 0;
    const size_t bins = (size_t)(block / WAVE) * R * smax;
    const size_t red = (size_t)RM * NSC * (block + 72);
    const size_t lds = (bins > red ? bins : red) * sizeof(double);
    const size_t stat = (size_t)(block / WAVE) * WAVE * 8 + DICT_MAX * sizeof(double) + 1024;
    return (lds + stat <= 156 * 1024) ? lds : 0;
}

// Batched step launch, packed form (k = 2, 2 <= j < m of every problem in the
// first nprob): one block per chunk of a problem for all its R right-hand sides.
hipError_t launch_arnoldi_step_packed(const BatchStepUnit* units, const int* base, int nprob, int R, int j, int grid,
                                      int smax, int prec, hipStream_t st) {
    const size_t lds = packed_step_lds(PACKED_BLOCK, R, smax);
    if (lds == 0) return hipErrorInvalidValue;
    if (prec == 1)
        hipLaunchKernelGGL((arnoldi_step_packed_kernel<8, PACKED_BLOCK, PrecF32, PACKED_RMAX>), dim3(grid),
                           dim3(PACKED_BLOCK), lds, st, units, base, nprob, R, j);
    else if (prec == 2)
        hipLaunchKernelGGL((arnoldi_step_packed_kernel<8, PACKED_BLOCK, PrecBF16, PACKED_RMAX>), dim3(grid),
                           dim3(PACKED_BLOCK), lds, st, units, base, nprob, R, j);
    else
        hipLaunchKernelGGL((arnoldi_step_packed_kernel<8, PACKED_BLOCK, PrecF64, PACKED_RMAX>), dim3(grid),
                           dim3(PACKED_BLOCK), lds, st, units, base, nprob, R, j);
    return hipGetLastError();
}

hipError_t launch_arnoldi_tail_batched(const BatchStepUnit* units, const SmallUnit* small, int nunits, int smax,
                                       int mmax, hipStream_t st) {
    hipLaunchKernelGGL(arnoldi_tail_batched_kernel, dim3((smax + 3) / 4, nunits), dim3(256), 0, st, units);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colnorm_batched_kernel, dim3((mmax + 3) / 4, nunits), dim3(256), 0, st, small, smax, mmax);
    return hipGetLastError();
}

hipError_t launch_arnoldi_check_batched(const SmallUnit* small, int nunits, int smax, int mmax, int k,
                                        hipStream_t st) {
    hipLaunchKernelGGL(arnoldi_check_batched_kernel, dim3(mmax, nunits), dim3(256), 0, st, small, smax, mmax, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(arnoldi_check_finish_batched_kernel, dim3(1, nunits), dim3(256), 0, st, small, mmax);
    return hipGetLastError();
}

}  // namespace skfab
