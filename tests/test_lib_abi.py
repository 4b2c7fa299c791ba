"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and rejects bad shapes on the host (no device work)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2208_11447_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skfab.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(skfab_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_names():
    assert sorted(N.EXPORTED) == declared_functions()


def test_library_exports_every_symbol():
    lib = N.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(skfab_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def _params(**kw):
    p = N.skfab_params()
    p.f, p.method, p.m, p.k, p.s, p.zeta, p.seed = 0, 0, 50, 2, 200, 8, 0
    p.l1, p.l2, p.lmax, p.quad_tol, p.prec = 32, 45, 1395, 1e-13, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _ws(n, **kw):
    csr = N.skfab_csr(n, 5 * n, None, None, None, 0)
    out = C.c_size_t()
    st = N.lib().skfab_workspace_bytes(C.byref(csr), C.byref(_params(**kw)), 1, C.byref(out))
    return st, out.value


def test_workspace_multi_rhs():
    """nrhs > 1 through the batched form needs at least the room of nrhs bases;
    nrhs < 1 is refused."""
    csr = N.skfab_csr(100_000, 500_000, None, None, None, 0)
    out1, out4 = C.c_size_t(), C.c_size_t()
    p = _params(m=100, s=200)
    assert N.lib().skfab_workspace_bytes(C.byref(csr), C.byref(p), 1, C.byref(out1)) == N.SKFAB_OK
    assert N.lib().skfab_workspace_bytes(C.byref(csr), C.byref(p), 4, C.byref(out4)) == N.SKFAB_OK
    assert out4.value >= 4 * 100_000 * 100 * 8 > out1.value
    assert N.lib().skfab_workspace_bytes(C.byref(csr), C.byref(p), 0, C.byref(out1)) == N.SKFAB_ERR_ARG


def test_workspace_sizes_grow_with_problem():
    st1, a = _ws(10_000)
    st2, b = _ws(2_097_152, m=200, s=400)
    assert st1 == st2 == N.SKFAB_OK
    assert b > a > 0
    # the basis dominates: N * m doubles
    assert b >= 2_097_152 * 200 * 8


@pytest.mark.parametrize("kw,status", [
    (dict(m=200, s=200), N.SKFAB_ERR_SHAPE),   # m < s violated
    (dict(k=0), N.SKFAB_ERR_SHAPE),
    (dict(k=9, m=50), N.SKFAB_ERR_SHAPE),      # k above the fused-kernel limit
    (dict(m=600, s=1000), N.SKFAB_ERR_SHAPE),  # m above the small-problem limit
    (dict(prec=1, k=8, m=50), N.SKFAB_ERR_ARG),  # reduced precision needs k <= 4
    (dict(prec=3), N.SKFAB_ERR_ARG),
    (dict(s=2000), N.SKFAB_ERR_SHAPE),
    (dict(zeta=3), N.SKFAB_ERR_SHAPE),
    (dict(f=7), N.SKFAB_ERR_ARG),
    (dict(method=1, f=3), N.SKFAB_ERR_ARG),    # polynomial needs the closed form
    (dict(l1=45, l2=32), N.SKFAB_ERR_ARG),
    (dict(f=1, method=2, fparam=0.0), N.SKFAB_ERR_ARG),           # contour form needs tau > 0
    (dict(f=1, method=2, fparam=0.01, m=201, s=402), N.SKFAB_ERR_ARG),  # ... and m <= 200
    (dict(f=1, method=1, fparam=0.01), N.SKFAB_ERR_ARG),          # no sFOM-quadrature form for exp
])
def test_host_validation(kw, status):
    st, _ = _ws(10_000, **kw)
    assert st == status


def test_contour_form_accepted():
    """exp with sketched GMRES (the contour rule) passes host validation."""
    st, nbytes = _ws(10_000, f=1, method=2, fparam=0.01, m=50, s=200)
    assert st == N.SKFAB_OK and nbytes > 0


def test_reckless_host_validation():
    """skfab_solve_reckless rejects null arguments before touching any device."""
    lib = N.lib()
    info = N.skfab_info()
    used = C.c_int32(0)
    p = N.skfab_params()
    assert lib.skfab_solve_reckless(None, None, None, None, C.byref(p), 400, 0.5, None, 0, C.byref(info),
                                    C.byref(used)) == N.SKFAB_ERR_ARG
    assert lib.skfab_solve_reckless(None, None, None, None, None, 400, 0.5, None, 0, None, None) == N.SKFAB_ERR_ARG


def test_value_table_switch_validation():
    """skfab_set_value_table rejects a null context before touching any device."""
    lib = N.lib()
    assert lib.skfab_set_value_table(None, 1) == N.SKFAB_ERR_ARG
    assert lib.skfab_set_value_table(None, 0) == N.SKFAB_ERR_ARG


def test_status_strings():
    lib = N.lib()
    for s in range(8):
        assert lib.skfab_status_string(s)
    assert lib.skfab_status_string(99) == b"unknown status"


def _batch(sizes, ms, ss=None):
    arr = (N.skfab_batch_problem * len(sizes))()
    for i, (n, m) in enumerate(zip(sizes, ms)):
        arr[i].A = N.skfab_csr(n, 5 * n, None, None, None, 0)
        arr[i].m = m
        arr[i].s = 2 * m if ss is None else ss[i]
        arr[i].seed = i
    return arr


def _batch_ws(sizes, ms, nrhs=4, ss=None, **kw):
    out = C.c_size_t()
    st = N.lib().skfab_batch_workspace_bytes(len(sizes), _batch(sizes, ms, ss), nrhs, C.byref(_params(**kw)),
                                             C.byref(out))
    return st, out.value


def test_batch_workspace_holds_every_basis():
    sizes, ms = [65_536, 262_144, 1_048_576], [80, 250, 160]
    st, nbytes = _batch_ws(sizes, ms)
    assert st == N.SKFAB_OK
    # four right-hand sides per problem, each with its own N x m basis
    assert nbytes >= sum(4 * 8 * n * m for n, m in zip(sizes, ms))
    st1, one = _batch_ws(sizes, ms, nrhs=1)
    assert st1 == N.SKFAB_OK and one < nbytes


@pytest.mark.parametrize("kw,nrhs,status", [
    (dict(), 5, N.SKFAB_ERR_ARG),            # at most 4 right-hand sides
    (dict(), 0, N.SKFAB_ERR_ARG),
    (dict(f=1), 4, N.SKFAB_ERR_ARG),         # exp is not offered batched
    (dict(zeta=4), 4, N.SKFAB_ERR_ARG),      # batched kernels: 8 nonzeros per column
    (dict(k=5), 4, N.SKFAB_ERR_ARG),
    (dict(prec=3), 4, N.SKFAB_ERR_ARG),
])
def test_batch_host_validation(kw, nrhs, status):
    st, _ = _batch_ws([10_000, 20_000], [50, 60], nrhs=nrhs, **kw)
    assert st == status


def test_batch_shape_validation():
    assert _batch_ws([10_000], [50], ss=[50])[0] == N.SKFAB_ERR_SHAPE       # s > m
    assert _batch_ws([100], [50], ss=[200])[0] == N.SKFAB_ERR_SHAPE        # s <= N
    assert _batch_ws([10_000], [600], ss=[1000])[0] == N.SKFAB_ERR_SHAPE   # m <= 512
    out = C.c_size_t()
    assert N.lib().skfab_batch_workspace_bytes(0, _batch([10], [2]), 1, C.byref(_params()),
                                               C.byref(out)) == N.SKFAB_ERR_ARG
