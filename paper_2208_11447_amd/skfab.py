"""Python binding of libskfab with the C ABI's names.

PyTorch is used only to hold device memory and to name the HIP stream; every
step of the method runs in the library's kernels.  Device arrays are torch CUDA
(HIP) tensors; the functions marshal pointers and sizes and raise
``SkfabError`` on a non-OK status.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _native as N

FUNCS = {"invsqrt": N.SKFAB_F_INVSQRT, "exp": N.SKFAB_F_EXP, "inv": N.SKFAB_F_INV, "poly": N.SKFAB_F_POLY}
METHODS = {"sfom": N.SKFAB_SFOM_CLOSED, "sfom_quad": N.SKFAB_SFOM_QUAD, "sgmres": N.SKFAB_SGMRES_QUAD}
PRECS = {"fp64": N.SKFAB_PREC_FP64, "fp32": N.SKFAB_PREC_FP32, "bf16basis": N.SKFAB_PREC_FP32_BF16BASIS}


class SkfabError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = N.lib().skfab_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def _check(status: int, where: str):
    if status != N.SKFAB_OK:
        raise SkfabError(status, where)


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _require_device(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")


@dataclass
class CSR:
    """Device CSR matrix (int32 indices, float64 values)."""
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def n(self) -> int:
        return self.rowptr.numel() - 1

    def c_struct(self) -> N.skfab_csr:
        _require_device(self.rowptr, torch.int32, "rowptr")
        _require_device(self.col, torch.int32, "col")
        _require_device(self.val, torch.float64, "val")
        return N.skfab_csr(self.n, self.col.numel(), self.rowptr.data_ptr(), self.col.data_ptr(),
                           self.val.data_ptr(), N.SKFAB_VAL_F64)

    @staticmethod
    def from_numpy(rowptr, col, val, device="cuda"):
        return CSR(torch.as_tensor(rowptr, dtype=torch.int32, device=device),
                   torch.as_tensor(col, dtype=torch.int32, device=device),
                   torch.as_tensor(val, dtype=torch.float64, device=device))


def make_params(f="invsqrt", m=50, k=2, s=200, zeta=8, seed=0, method="sfom", fparam=0.0, poly=None,
                l1=32, l2=45, lmax=1395, quad_tol=1e-13, prec="fp64", cond_max=0.0,
                two_pass=False, srdct=None) -> N.skfab_params:
    """Method parameters.  srdct: None for the sparse-sign sketch, or (signs, rows) device
    tensors (int8[N], int32[s]) of the SRDCT sketch (kept alive by the returned struct)."""
    p = N.skfab_params()
    p.f = FUNCS[f] if isinstance(f, str) else int(f)
    p.fparam = float(fparam)
    p.method = METHODS[method] if isinstance(method, str) else int(method)
    p.m, p.k, p.s, p.zeta, p.seed = int(m), int(k), int(s), int(zeta), int(seed)
    p.l1, p.l2, p.lmax, p.quad_tol = int(l1), int(l2), int(lmax), float(quad_tol)
    p.prec = PRECS[prec] if isinstance(prec, str) else int(prec)
    p.cond_max = float(cond_max)
    p.two_pass = 1 if two_pass else 0
    if srdct is not None:
        signs, rows = srdct
        _require_device(signs, torch.int8, "srdct signs")
        _require_device(rows, torch.int32, "srdct rows")
        p.sketch = N.SKFAB_SKETCH_SRDCT
        p.srdct_signs = signs.data_ptr()
        p.srdct_rows = rows.data_ptr()
        p._srdct_keepalive = (signs, rows)
    else:
        p.sketch = N.SKFAB_SKETCH_SPARSE_SIGN
    if poly is not None:
        arr = (C.c_double * len(poly))(*[float(c) for c in poly])
        p.poly = C.cast(arr, C.POINTER(C.c_double))
        p.npoly = len(poly)
        p._poly_keepalive = arr
    else:
        p.poly = None
        p.npoly = 0
    return p


class Context:
    """skfab_create / skfab_destroy around a device and a torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = device
        self.stream = stream or torch.cuda.current_stream(device)
        self.handle = C.c_void_p()
        _check(N.lib().skfab_create(C.byref(self.handle), device, C.c_void_p(self.stream.cuda_stream)),
               "skfab_create")

    def set_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        _check(N.lib().skfab_set_stream(self.handle, C.c_void_p(stream.cuda_stream)), "skfab_set_stream")

    def close(self):
        if self.handle:
            N.lib().skfab_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def skfab_version() -> int:
    return N.lib().skfab_version()


def skfab_workspace_bytes(A: CSR | int, p: N.skfab_params, nrhs: int = 1) -> int:
    if isinstance(A, CSR):
        csr = N.skfab_csr(A.n, A.col.numel(), None, None, None, N.SKFAB_VAL_F64)
    else:
        csr = N.skfab_csr(int(A), 0, None, None, None, N.SKFAB_VAL_F64)
    out = C.c_size_t()
    _check(N.lib().skfab_workspace_bytes(C.byref(csr), C.byref(p), int(nrhs), C.byref(out)),
           "skfab_workspace_bytes")
    return out.value


def alloc_workspace(nbytes: int, device=None) -> torch.Tensor:
    """Device bytes for the library (torch caching allocator; 256-byte aligned)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def skfab_solve(ctx: Context, A: CSR, b: torch.Tensor, x: torch.Tensor, p: N.skfab_params,
                ws: torch.Tensor, want_info: bool = True):
    """x <- f(A) b.  b, x: (N,) tensors (one right-hand side; returns one skfab_info)
    or (nrhs, N) tensors (row r = column r of the C ABI's column-major N x nrhs;
    returns a list of nrhs skfab_info)."""
    _require_device(b, torch.float64, "b")
    _require_device(x, torch.float64, "x")
    if b.shape != x.shape or b.dim() not in (1, 2) or b.shape[-1] != A.n:
        raise ValueError("b and x must both be (N,) or (nrhs, N) tensors of the matrix's size")
    nrhs = 1 if b.dim() == 1 else int(b.shape[0])
    csr = A.c_struct()
    info = (N.skfab_info * nrhs)() if want_info else None
    st = N.lib().skfab_solve(ctx.handle, C.byref(csr), _ptr(b), A.n, nrhs, _ptr(x), A.n, C.byref(p), _ptr(ws),
                             ws.numel(), info)
    _check(st, "skfab_solve")
    if info is None:
        return None
    return info[0] if b.dim() == 1 else [info[r] for r in range(nrhs)]


def skfab_solve_noalloc(ctx: Context, A: CSR, b: torch.Tensor, x: torch.Tensor, p: N.skfab_params,
                        want_info: bool = True):
    """x <- f(A) b (one right-hand side) with the library's static device workspace:
    the call allocates nothing."""
    _require_device(b, torch.float64, "b")
    _require_device(x, torch.float64, "x")
    if b.shape != x.shape or b.dim() != 1 or b.shape[0] != A.n:
        raise ValueError("b and x must be (N,) tensors of the matrix's size")
    csr = A.c_struct()
    info = N.skfab_info() if want_info else None
    st = N.lib().skfab_solve_noalloc(ctx.handle, C.byref(csr), _ptr(b), _ptr(x), C.byref(p),
                                     C.byref(info) if info is not None else None)
    _check(st, "skfab_solve_noalloc")
    return info


def skfab_solve_reckless(ctx: Context, A: CSR, b: torch.Tensor, x: torch.Tensor, p: N.skfab_params, s_max: int,
                         eps_max: float, ws: torch.Tensor):
    """x <- f(A) b with the sketch size chosen by the computation: p.s first, doubled
    (up to s_max) while the solve fails or the embedding monitor exceeds eps_max.
    Returns (info, s_used); ws must hold the workspace of the s = s_max solve."""
    _require_device(b, torch.float64, "b")
    _require_device(x, torch.float64, "x")
    if b.shape != x.shape or b.dim() != 1 or b.shape[0] != A.n:
        raise ValueError("b and x must be (N,) tensors of the matrix's size")
    csr = A.c_struct()
    info = N.skfab_info()
    s_used = C.c_int32(0)
    st = N.lib().skfab_solve_reckless(ctx.handle, C.byref(csr), _ptr(b), _ptr(x), C.byref(p), int(s_max),
                                      float(eps_max), _ptr(ws), ws.numel(), C.byref(info), C.byref(s_used))
    _check(st, "skfab_solve_reckless")
    return info, s_used.value


def skfab_arnoldi(ctx: Context, A: CSR, b: torch.Tensor, p: N.skfab_params, V=None, SV=None, SAV=None, H=None,
                  ws: torch.Tensor = None, want_info: bool = True):
    csr = A.c_struct()
    info = N.skfab_info() if want_info else None
    st = N.lib().skfab_arnoldi(ctx.handle, C.byref(csr), _ptr(b), C.byref(p), _ptr(V), _ptr(SV), _ptr(SAV),
                               _ptr(H), _ptr(ws), ws.numel(), C.byref(info) if info is not None else None)
    _check(st, "skfab_arnoldi")
    return info


def skfab_small_workspace_bytes(p: N.skfab_params) -> int:
    out = C.c_size_t()
    _check(N.lib().skfab_small_workspace_bytes(C.byref(p), C.byref(out)), "skfab_small_workspace_bytes")
    return out.value


def skfab_small_problem(ctx: Context, SVext: torch.Tensor, Hbar: torch.Tensor, beta: float, p: N.skfab_params,
                        y: torch.Tensor, ws: torch.Tensor):
    info = N.skfab_info()
    st = N.lib().skfab_small_problem(ctx.handle, _ptr(SVext), _ptr(Hbar), float(beta), C.byref(p), _ptr(y),
                                     _ptr(ws), ws.numel(), C.byref(info))
    _check(st, "skfab_small_problem")
    return info


def skfab_sketch_pattern(ctx: Context, col0: int, ncols: int, s: int, zeta: int, seed: int,
                         rows: torch.Tensor, signs: torch.Tensor):
    _require_device(rows, torch.int32, "rows")
    _require_device(signs, torch.int8, "signs")
    _check(N.lib().skfab_sketch_pattern(ctx.handle, col0, ncols, s, zeta, seed, _ptr(rows), _ptr(signs)),
           "skfab_sketch_pattern")


def skfab_sketch_ws_bytes(n: int, s: int) -> int:
    return N.lib().skfab_sketch_ws_bytes(n, s)


def skfab_sketch_apply(ctx: Context, n: int, s: int, zeta: int, seed: int, v: torch.Tensor, Sv: torch.Tensor,
                       ws: torch.Tensor):
    _require_device(v, torch.float64, "v")
    _require_device(Sv, torch.float64, "Sv")
    _check(N.lib().skfab_sketch_apply(ctx.handle, n, s, zeta, seed, _ptr(v), _ptr(Sv), _ptr(ws), ws.numel()),
           "skfab_sketch_apply")


def skfab_srdct_ws_bytes(n: int, s: int, ncols: int) -> int:
    return N.lib().skfab_srdct_ws_bytes(int(n), int(s), int(ncols))


def skfab_srdct_apply(ctx: Context, signs: torch.Tensor, rows: torch.Tensor, V: torch.Tensor, SV: torch.Tensor,
                      ws: torch.Tensor):
    """SV <- S V for the SRDCT sketch; V: (ncols, n) tensor (row c = column c of the C ABI's
    column-major n x ncols), SV: (ncols, s)."""
    _require_device(signs, torch.int8, "signs")
    _require_device(rows, torch.int32, "rows")
    _require_device(V, torch.float64, "V")
    _require_device(SV, torch.float64, "SV")
    ncols, n = V.shape
    s = rows.numel()
    if SV.shape != (ncols, s) or signs.numel() != n:
        raise ValueError("shapes: V (ncols, n), SV (ncols, s), signs (n,), rows (s,)")
    _check(N.lib().skfab_srdct_apply(ctx.handle, n, s, _ptr(signs), _ptr(rows), _ptr(V), n, ncols, _ptr(SV),
                                     _ptr(ws), ws.numel()), "skfab_srdct_apply")


def skfab_set_arnoldi_check(ctx: Context, enable: bool = True):
    """Sketch A u_j as well and report the Arnoldi relation residual in
    info.arnoldi_relres (off by default: -1)."""
    _check(N.lib().skfab_set_arnoldi_check(ctx.handle, 1 if enable else 0), "skfab_set_arnoldi_check")


def skfab_set_value_table(ctx: Context, enable: bool = True):
    """Value-table (uint8 index) storage of A's values in the SELL copy when A has at
    most 256 distinct values; on by default (enable=False: always the plain form)."""
    _check(N.lib().skfab_set_value_table(ctx.handle, 1 if enable else 0), "skfab_set_value_table")


def skfab_timing_enable(ctx: Context, enable: bool = True, stride: int = 1):
    """Event timing of the timed kernel classes (off: enable=False): runs of consecutive
    step launches as one interval each, isolated launches every stride-th."""
    _check(N.lib().skfab_timing_enable(ctx.handle, int(stride) if enable else 0), "skfab_timing_enable")


def skfab_timing_read(ctx: Context, kernel: int = 0):
    """(total milliseconds, launches) of kernel class 0 (Arnoldi step) or 1 (assembly) since the last read."""
    ms = C.c_double()
    n = C.c_int64()
    _check(N.lib().skfab_timing_read(ctx.handle, kernel, C.byref(ms), C.byref(n)), "skfab_timing_read")
    return ms.value, n.value


# ----------------------------------------------------------------- batches
@dataclass
class BatchProblem:
    """One problem of a batch: device CSR, right-hand sides B and results X as
    (nrhs, N) contiguous float64 tensors (row r = column r of the C ABI's
    column-major N x nrhs), Krylov dimension m, sketch size s and sketch seed."""
    A: CSR
    B: torch.Tensor
    X: torch.Tensor
    m: int
    s: int
    seed: int = 0


def _batch_array(probs, need_data: bool = True):
    arr = (N.skfab_batch_problem * len(probs))()
    for i, q in enumerate(probs):
        if need_data:
            _require_device(q.B, torch.float64, "B")
            _require_device(q.X, torch.float64, "X")
            if q.B.shape != q.X.shape or q.B.dim() != 2 or q.B.shape[1] != q.A.n:
                raise ValueError("B and X must be (nrhs, N) tensors of the problem's size")
            arr[i].A = q.A.c_struct()
            arr[i].B = q.B.data_ptr()
            arr[i].X = q.X.data_ptr()
        else:
            arr[i].A = N.skfab_csr(q.A.n, q.A.col.numel(), None, None, None, N.SKFAB_VAL_F64)
        arr[i].m, arr[i].s, arr[i].seed = int(q.m), int(q.s), int(q.seed)
    return arr


def _nrhs(probs) -> int:
    r = {int(q.B.shape[0]) for q in probs}
    if len(r) != 1:
        raise ValueError("every problem of a batch needs the same number of right-hand sides")
    return r.pop()


def skfab_batch_workspace_bytes(probs, p: N.skfab_params, nrhs: int | None = None) -> int:
    nr = _nrhs(probs) if nrhs is None else int(nrhs)
    out = C.c_size_t()
    _check(N.lib().skfab_batch_workspace_bytes(len(probs), _batch_array(probs, False), nr, C.byref(p),
                                               C.byref(out)), "skfab_batch_workspace_bytes")
    return out.value


def skfab_solve_batched(ctx: Context, probs, p: N.skfab_params, ws: torch.Tensor, want_info: bool = True):
    """X_p[r] <- f(A_p) B_p[r] for every problem p and right-hand side r; returns a
    list (per problem) of lists (per right-hand side) of skfab_info, or None."""
    nr = _nrhs(probs)
    arr = _batch_array(probs)
    info = (N.skfab_info * (len(probs) * nr))() if want_info else None
    st = N.lib().skfab_solve_batched(ctx.handle, len(probs), arr, nr, C.byref(p), _ptr(ws), ws.numel(), info)
    _check(st, "skfab_solve_batched")
    if info is None:
        return None
    return [[info[i * nr + r] for r in range(nr)] for i in range(len(probs))]


def skfab_batch_set_tuning(ctx: Context, block: int, slices_per_wave: int, packed: bool = False):
    t = N.skfab_batch_tuning(int(block), int(slices_per_wave), 1 if packed else 0)
    _check(N.lib().skfab_batch_set_tuning(ctx.handle, C.byref(t)), "skfab_batch_set_tuning")


def skfab_batch_get_tuning(ctx: Context):
    """(block, slices_per_wave, packed) of the context's batched step launches."""
    t = N.skfab_batch_tuning()
    _check(N.lib().skfab_batch_get_tuning(ctx.handle, C.byref(t)), "skfab_batch_get_tuning")
    return t.block, t.slices_per_wave, bool(t.packed)


def skfab_batch_autotune(ctx: Context, probs, p: N.skfab_params, ws: torch.Tensor, steps: int = 4):
    """Time every launch shape of the batched step kernel on this batch (and the
    packed form for 512-thread blocks); keeps and returns the fastest
    (block, slices_per_wave, packed)."""
    nr = _nrhs(probs)
    t = N.skfab_batch_tuning()
    _check(N.lib().skfab_batch_autotune(ctx.handle, len(probs), _batch_array(probs), nr, C.byref(p), _ptr(ws),
                                        ws.numel(), int(steps), C.byref(t)), "skfab_batch_autotune")
    return t.block, t.slices_per_wave, bool(t.packed)


# -------------------------------------------------------------- adaptive m
def skfab_adaptive_workspace_bytes(A: CSR | int, p: N.skfab_params) -> int:
    n = A.n if isinstance(A, CSR) else int(A)
    nnz = A.col.numel() if isinstance(A, CSR) else 0
    csr = N.skfab_csr(n, nnz, None, None, None, N.SKFAB_VAL_F64)
    out = C.c_size_t()
    _check(N.lib().skfab_adaptive_workspace_bytes(C.byref(csr), C.byref(p), C.byref(out)),
           "skfab_adaptive_workspace_bytes")
    return out.value


def skfab_solve_adaptive(ctx: Context, A: CSR, b: torch.Tensor, x: torch.Tensor, p: N.skfab_params, m0: int,
                         d: int, tol: float, ws: torch.Tensor):
    """Returns (info, m_stop, estimate)."""
    _require_device(b, torch.float64, "b")
    _require_device(x, torch.float64, "x")
    csr = A.c_struct()
    info = N.skfab_info()
    ms = C.c_int32()
    est = C.c_double()
    _check(N.lib().skfab_solve_adaptive(ctx.handle, C.byref(csr), _ptr(b), _ptr(x), C.byref(p), int(m0), int(d),
                                        float(tol), _ptr(ws), ws.numel(), C.byref(info), C.byref(ms),
                                        C.byref(est)), "skfab_solve_adaptive")
    return info, ms.value, est.value


# ------------------------------------------------------ controller kernels
def skfab_gershgorin(ctx: Context, A: CSR, bounds: torch.Tensor, ws: torch.Tensor):
    _require_device(bounds, torch.float64, "bounds")
    csr = A.c_struct()
    _check(N.lib().skfab_gershgorin(ctx.handle, C.byref(csr), _ptr(bounds), _ptr(ws), ws.numel()),
           "skfab_gershgorin")


def skfab_gershgorin_ws_bytes(n: int) -> int:
    return N.lib().skfab_gershgorin_ws_bytes(int(n))


def skfab_mlp_param_count() -> int:
    return N.lib().skfab_mlp_param_count()


def skfab_mlp_ws_bytes(batch: int) -> int:
    return N.lib().skfab_mlp_ws_bytes(int(batch))


def skfab_mlp_forward(ctx: Context, X: torch.Tensor, params: torch.Tensor, Y: torch.Tensor, ws: torch.Tensor):
    for t, nm in ((X, "X"), (params, "params"), (Y, "Y")):
        _require_device(t, torch.float32, nm)
    _check(N.lib().skfab_mlp_forward(ctx.handle, _ptr(X), X.shape[0], _ptr(params), _ptr(Y), _ptr(ws),
                                     ws.numel()), "skfab_mlp_forward")


def skfab_mlp_loss_grad(ctx: Context, X: torch.Tensor, T: torch.Tensor, params: torch.Tensor, grad: torch.Tensor,
                        loss: torch.Tensor | None, ws: torch.Tensor):
    for t, nm in ((X, "X"), (T, "T"), (params, "params"), (grad, "grad")):
        _require_device(t, torch.float32, nm)
    _check(N.lib().skfab_mlp_loss_grad(ctx.handle, _ptr(X), _ptr(T), X.shape[0], _ptr(params), _ptr(grad),
                                       _ptr(loss), _ptr(ws), ws.numel()), "skfab_mlp_loss_grad")


def skfab_mlp_adam(ctx: Context, params: torch.Tensor, grad: torch.Tensor, m1: torch.Tensor, m2: torch.Tensor,
                   t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    _check(N.lib().skfab_mlp_adam(ctx.handle, _ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), int(t), float(lr),
                                  float(beta1), float(beta2), float(eps)), "skfab_mlp_adam")
