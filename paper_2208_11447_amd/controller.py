"""Learned controller of (m, k, s) for sketched FOM at a requested tolerance.

A small network (16 -> 64 -> 64 -> 3, ReLU, FP32; forward, gradient and Adam in
the library's HIP kernels) maps cheap features of a problem to the Krylov
dimension m, the truncation length k and the sketch-size factor s / m that
the plain adaptive-m method (Section 4.3 stopping estimate, checked every d
steps) would need. The controlled solve starts its checks at the predicted m, so
a good prediction costs two small problems and one synchronisation instead of
one per checkpoint. The plain adaptive-m solve is both the fallback (the checks
continue past the prediction, and a full adaptive run follows if the capped
dimension is reached) and the arbiter (every accepted result passes its stopping
test).

Features (16): log n_x, log n_y, log n_z (n_z = 1 in 2D), log D, log(1 + c_x),
log(1 + c_y), log(1 + c_z), signed logs of the Gershgorin bounds (device
kernel), log ||b||, and signed logs of the three smallest and three largest
real parts of the Ritz values of a 10-step Arnoldi probe (the probe runs on the
device; the 10 x 10 eigenvalue problem is solved on the host).

Training data come from runs of the method itself: random 2D/3D
convection-diffusion problems, each solved by the adaptive-m method for every
(k, s/m) in {2, 4} x {2, 4}; the label is the successful configuration of least
work m (k + 3) (HBM traffic per step grows with the k window vectors plus A u_j
in and u_j, A u_j out).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import skfab as sk

N_FEATURES = 16
K_CHOICES = (2, 4)
S_FACTORS = (2, 4)
M_CAP = 240           # largest Krylov dimension the controller works with
CHECK_D = 10          # checkpoint spacing of the adaptive-m method
PROBE_M, PROBE_K, PROBE_S = 10, 8, 40


@dataclass
class ProblemSpec:
    """A convection-diffusion operator (grid n per axis, dim 2 or 3, diffusion D,
    convection per axis) and the seed of its right-hand side."""
    n: int
    dim: int
    diffusion: float
    convection: tuple
    rhs_seed: int

    @property
    def N(self) -> int:
        return self.n ** self.dim

    def build(self, device="cuda"):
        from workloads import convdiff_csr, gaussian_rhs
        rp, col, val = convdiff_csr(self.n, self.dim, self.diffusion, np.asarray(self.convection, dtype=float))
        A = sk.CSR.from_numpy(rp, col, val, device=device)
        b = torch.as_tensor(gaussian_rhs(rp.size - 1, self.rhs_seed), device=device)
        return A, b


def random_specs(count: int, seed: int):
    """Random 2D / 3D problems: 2D grids n in 40..120, 3D grids n in 12..24,
    diffusion in [0.5, 2], convection per axis in [0, 150]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        dim = int(rng.choice([2, 3]))
        n = int(rng.integers(40, 121)) if dim == 2 else int(rng.integers(12, 25))
        D = float(rng.uniform(0.5, 2.0))
        c = tuple(float(v) for v in rng.uniform(0.0, 150.0, size=dim))
        out.append(ProblemSpec(n, dim, D, c, int(rng.integers(0, 2**31 - 1))))
    return out


def _slog(x: float) -> float:
    return math.copysign(math.log1p(abs(x)), x)


class Runner:
    """Device context and scratch shared by feature extraction and solves."""

    def __init__(self, device: int = 0):
        self.ctx = sk.Context(device)
        self.bounds = torch.zeros(2, dtype=torch.float64, device="cuda")

    def features(self, spec: ProblemSpec, A: sk.CSR, b: torch.Tensor) -> np.ndarray:
        gws = sk.alloc_workspace(sk.skfab_gershgorin_ws_bytes(A.n))
        sk.skfab_gershgorin(self.ctx, A, self.bounds, gws)
        p = sk.make_params(m=PROBE_M, k=PROBE_K, s=PROBE_S)
        ws = sk.alloc_workspace(sk.skfab_workspace_bytes(A, p))
        H = torch.zeros((PROBE_M, PROBE_M + 1), dtype=torch.float64, device="cuda")
        info = sk.skfab_arnoldi(self.ctx, A, b, p, None, None, None, H, ws)
        lo, hi = self.bounds.cpu().numpy()
        Hm = H.cpu().numpy().T[:info.m_used, :info.m_used]
        re = np.sort(np.linalg.eigvals(Hm).real) if Hm.size else np.zeros(1)
        re = np.concatenate([re, np.repeat(re[-1:], max(0, 6 - re.size))])
        nz = spec.n if spec.dim == 3 else 1
        conv = list(spec.convection) + [0.0] * (3 - len(spec.convection))
        f = [math.log(spec.n), math.log(spec.n), math.log(nz), math.log(spec.diffusion),
             math.log1p(conv[0]), math.log1p(conv[1]), math.log1p(conv[2]),
             _slog(lo), _slog(hi), math.log(max(info.beta, 1e-300))]
        f += [_slog(v) for v in re[:3]] + [_slog(v) for v in re[-3:]]
        return np.asarray(f, dtype=np.float32)

    def adaptive(self, A, b, k: int, sfac: int, m0: int, m_max: int, tol: float):
        """Plain adaptive-m solve; returns (x, info, m_stop, estimate, seconds)."""
        m_max = min(m_max, M_CAP, 1024 // sfac - 1)
        p = sk.make_params(f="invsqrt", m=m_max, k=k, s=min(sfac * m_max, A.n - 1), zeta=8)
        ws = sk.alloc_workspace(sk.skfab_adaptive_workspace_bytes(A, p))
        x = torch.empty_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info, m_stop, est = sk.skfab_solve_adaptive(self.ctx, A, b, x, p, max(m0, k), CHECK_D, tol, ws)
        torch.cuda.synchronize()
        return x, info, m_stop, est, time.perf_counter() - t0


def label_problem(runner: Runner, spec: ProblemSpec, tol: float):
    """Features and the label (log m, k, s/m) of one problem, from adaptive-m runs
    of every configuration; returns (features, label, runs) or None if no
    configuration met the tolerance."""
    A, b = spec.build()
    feats = runner.features(spec, A, b)
    best = None
    runs = 0
    for k in K_CHOICES:
        for sf in S_FACTORS:
            _, info, m_stop, est, _ = runner.adaptive(A, b, k, sf, 10, M_CAP, tol)
            runs += 1
            if info.status != 0 or not (est <= tol):
                continue
            work = m_stop * (k + 3)
            if best is None or work < best[0]:
                best = (work, m_stop, k, sf)
    if best is None:
        return feats, None, runs
    _, m_stop, k, sf = best
    return feats, np.asarray([math.log(m_stop), k - 3.0, sf - 3.0], dtype=np.float32), runs


@dataclass
class Model:
    params: torch.Tensor                # device float32 [param_count]
    mu: np.ndarray                      # feature standardisation
    sd: np.ndarray
    history: list = field(default_factory=list)


def train(runner: Runner, X: np.ndarray, Y: np.ndarray, steps: int = 3000, lr: float = 2e-3, seed: int = 0,
          log_every: int = 0) -> Model:
    """Full-batch Adam on the device kernels (forward + gradient + update per step)."""
    P = sk.skfab_mlp_param_count()
    mu = X.mean(axis=0)
    sd = X.std(axis=0) + 1e-6
    Xs = torch.as_tensor((X - mu) / sd, dtype=torch.float32, device="cuda").contiguous()
    T = torch.as_tensor(Y, dtype=torch.float32, device="cuda").contiguous()
    params = torch.as_tensor(init_params(seed), dtype=torch.float32, device="cuda")
    grad = torch.zeros_like(params)
    m1 = torch.zeros_like(params)
    m2 = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = sk.alloc_workspace(sk.skfab_mlp_ws_bytes(Xs.shape[0]))
    hist = []
    for t in range(1, steps + 1):
        sk.skfab_mlp_loss_grad(runner.ctx, Xs, T, params, grad, loss, ws)
        sk.skfab_mlp_adam(runner.ctx, params, grad, m1, m2, t, lr)
        if log_every and (t % log_every == 0 or t == 1):
            hist.append((t, float(loss.item())))
    if not hist or hist[-1][0] != steps:
        sk.skfab_mlp_loss_grad(runner.ctx, Xs, T, params, grad, loss, ws)
        hist.append((steps, float(loss.item())))
    assert P == params.numel()
    return Model(params, mu, sd, hist)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, in the library's layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((64, 16), (64, 64), (3, 64)):
        lim = math.sqrt(6.0 / cols)
        parts += [rng.uniform(-lim, lim, size=rows * cols), np.zeros(rows)]
    return np.concatenate(parts).astype(np.float32)


def predict(runner: Runner, model: Model, feats: np.ndarray):
    """(m, k, s/m) predictions for a batch of feature rows, on the device kernels."""
    X = torch.as_tensor((np.atleast_2d(feats) - model.mu) / model.sd, dtype=torch.float32,
                        device="cuda").contiguous()
    Y = torch.empty((X.shape[0], 3), dtype=torch.float32, device="cuda")
    ws = sk.alloc_workspace(sk.skfab_mlp_ws_bytes(X.shape[0]))
    sk.skfab_mlp_forward(runner.ctx, X, model.params, Y, ws)
    out = []
    for y in Y.cpu().numpy():
        m = int(min(M_CAP, max(CHECK_D + 2, math.ceil(math.exp(float(y[0])) * 1.1))))
        k = 2 if y[1] < 0 else 4
        sf = 2 if y[2] < 0 else 4
        out.append((m, k, sf))
    return out


def checkpoints(m0: int, m_stop: int, d: int = CHECK_D) -> int:
    """Small problems an adaptive run from m0 evaluates before stopping at m_stop."""
    return max(0, (m_stop - m0) // d) + 1


def controlled_solve(runner: Runner, model: Model, spec: ProblemSpec, A, b, tol: float, feats=None):
    """Solve with the predicted configuration: checks at m_pred - d and m_pred,
    continuing every d steps up to m_pred + 6 d; a full plain adaptive-m run if
    that does not pass.  Returns (x, info, m_stop, estimate, seconds, fallback,
    checks), checks = small problems evaluated (both runs on a fallback)."""
    t0 = time.perf_counter()
    if feats is None:
        feats = runner.features(spec, A, b)
    m, k, sf = predict(runner, model, feats)[0]
    m_max = min(M_CAP, m + 6 * CHECK_D)
    m0 = max(k, m - CHECK_D)
    x, info, m_stop, est, _ = runner.adaptive(A, b, k, sf, m0, m_max, tol)
    checks = checkpoints(m0, m_stop)
    fallback = False
    if info.status != 0 or not (est <= tol):
        fallback = True
        x, info, m_stop, est, _ = runner.adaptive(A, b, 2, 2, 10, M_CAP, tol)
        checks += checkpoints(10, m_stop)
    torch.cuda.synchronize()
    return x, info, m_stop, est, time.perf_counter() - t0, fallback, checks
