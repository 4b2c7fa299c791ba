#!/usr/bin/env python3
"""Benchmark: sketched-FOM f(A)b solves per second on one MI355X.

Workload (default): 3D convection-diffusion on a 128^3 grid (N = 2,097,152,
7-point upwind stencil, diffusion 1, convection (100,100,100), CSR FP64),
f(z) = z^(-1/2), b ~ N(0,1) seed 0, m = 200, k = 2, s = 400 sparse-sign sketch
with 8 nonzeros per column (seed 0), sketched FOM closed form.

One timed step = one complete solve with the inputs already resident in HBM:
the implicit sketch, m fused Arnoldi steps (SpMV + truncated Gram-Schmidt dots +
both sketches), the extension vector, the sketch reduction, the whitening QR,
the Hessenberg pencil, the adaptive quadrature and the assembly x = V_m y.

The JSON line also carries
  roofline:     the fused Arnoldi step kernel (dominant): algorithmic bytes per
                launch / its mean duration, timed with HIP events recorded by the
                library on the solve stream during the timed region, against
                the 8 TB/s HBM peak;
  cpu_baseline: the FP64 oracle on a bounded sample of the same workload on this
                host's CPU, scaled to solves/s;
  parity:       relative 2-norm error of the timed GPU result against the oracle
                on the full workload (same sketch, m, k).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="convdiff3d_n128_m200",
                    help="a single-problem workload, 'batch64x4' for the batched form (64 problems x 4 rhs), "
                         "'controller' for the learned controller against plain adaptive-m, or 'paper51' for "
                         "the convergence table of the paper's convection-diffusion experiment")
    ap.add_argument("--train-problems", type=int, default=2500,
                    help="controller: training problems (4 method runs each)")
    ap.add_argument("--test-problems", type=int, default=256, help="controller: held-out problems")
    ap.add_argument("--nprob", type=int, default=64, help="problems of the batched workload")
    ap.add_argument("--no-autotune", action="store_true", help="batched form: keep the default launch shape")
    ap.add_argument("--save-outputs", default=None, metavar="NPZ",
                    help="batched form: save every pair's status, m_used, ||x|| and x at a fixed sample of "
                         "entries, for the offline oracle check (--check-outputs)")
    ap.add_argument("--check-outputs", default=None, metavar="NPZ",
                    help="CPU only: check the saved batched outputs against the oracle (right-hand side 0 of "
                         "every problem and every pair with a nonzero status) and print the table")
    ap.add_argument("--reckless", action="store_true",
                    help="batched form: after the timed batches, re-solve every refused pair with "
                         "skfab_solve_reckless (s doubled from 4m up to min(8m, 1024) while the solve fails or the "
                         "embedding monitor exceeds 0.5) and report how many it recovers")
    ap.add_argument("--tuning", default=None, metavar="BLOCK,SPW[,PACKED]",
                    help="batched form: fixed launch shape (threads per block, slices per wavefront, and 1 / 0 "
                         "for the packed form or not, default 0)")
    ap.add_argument("--f", default="invsqrt", choices=["invsqrt", "inv", "exp"],
                    help="f(z): z^(-1/2), 1/z, or exp(-tau z) (sfom: closed form; sgmres: contour rule)")
    ap.add_argument("--tau", type=float, default=1e-2, help="tau of f(z) = exp(-tau z)")
    ap.add_argument("--quad-tol", type=float, default=1e-13,
                    help="tolerance of the adaptive quadrature (Section 4.1 test) for sfom_quad and sgmres")
    ap.add_argument("--method", default="sfom", choices=["sfom", "sfom_quad", "sgmres"])
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16basis"],
                    help="storage/arithmetic of A, the basis and the SpMV (small problem and assembly stay FP64)")
    ap.add_argument("--no-parity", action="store_true", help="skip the full-size oracle comparison")
    ap.add_argument("--plain-values", action="store_true",
                    help="single-problem workloads: store A's values in the SELL copy as they are, not as "
                         "indices into a table of its distinct values")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-solves", type=int, default=3,
                    help="full oracle solves timed for cpu_baseline (median; the first also gives the parity)")
    ap.add_argument("--no-timing-events", action="store_true")
    ap.add_argument("--timing-stride", type=int, default=8,
                    help="single-problem workloads: HIP events bracket every n-th assembly launch of the timed "
                         "region (the step launches of each solve are timed as one run, every one counted); "
                         "the events cost a few microseconds of queue time each, so timing every isolated launch "
                         "would lower the solves/s figure they are quoted with")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of this many GiB (5 times) and report its GB/s; "
                         "used to scale rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--summarize", default=None, choices=["trace", "counters"],
                    help="CPU only: write a text summary of rocprofv3 CSV output (-f csv): 'trace' from one "
                         "--kernel-trace --stats run, 'counters' from four --pmc runs (FETCH_SIZE, WRITE_SIZE of "
                         "the workload, then of the copy calibration); see --prof-dirs")
    ap.add_argument("--prof-dirs", default="", help="comma-separated rocprofv3 output folders (-d)")
    ap.add_argument("--prof-json", default=None, help="the JSON line bench.py printed in the profiled run")
    ap.add_argument("--prof-copy-json", default=None,
                    help="the JSON line of the --copy-calibration run profiled for the counter scale")
    ap.add_argument("--prof-title", default="", help="summary title line")
    ap.add_argument("--prof-cmd", action="append", default=[], help="command(s) that made the output")
    ap.add_argument("--prof-out", default=None, help="summary file to write")
    return ap.parse_args()


def _prof_rows(root: str, suffix: str):
    """Rows of every rocprofv3 CSV file under `root` whose name ends in `suffix`."""
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {root}")
    return rows


def _kernel_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_means(root: str, counter: str):
    """{kernel name: (dispatches, mean counter value per dispatch)} of one --pmc run."""
    acc = {}
    for r in _prof_rows(root, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        name = r["Kernel_Name"]
        n, t = acc.get(name, (0, 0.0))
        acc[name] = (n + 1, t + float(r["Counter_Value"]))
    return {k: (n, t / n) for k, (n, t) in acc.items()}


def summarize_profile(args):
    """Text summary of rocprofv3 CSV output for profiles/ (see --summarize)."""
    dirs = [d for d in args.prof_dirs.split(",") if d]
    run = {}
    if args.prof_json:
        with open(args.prof_json) as fh:
            run = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    roof = run.get("roofline", {})
    lines = [f"# {args.prof_title}"] + [f"# command: {c}" for c in args.prof_cmd]
    lines.append(f"# kernel sources sha256 ({', '.join(os.path.basename(r) for r in KERNEL_SOURCES)}): "
                 f"{_kernel_sha()}")
    if args.summarize == "trace":
        rows = _prof_rows(dirs[0], "kernel_stats.csv")
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        total = sum(float(r["TotalDurationNs"]) for r in rows)
        if run:
            lines.append(f"# bench line of the same run: value {run.get('value')} {run.get('unit')}, "
                         f"ms_per_step {run.get('ms_per_step')}, step kernel by HIP events "
                         f"{roof.get('mean_launch_us', roof.get('step_ms_per_batch'))} "
                         f"{'us per launch' if 'mean_launch_us' in roof else 'ms per batch'}")
        lines.append("# columns: kernel, calls, total, mean, share of GPU time")
        for r in rows:
            t = float(r["TotalDurationNs"])
            name = r["Name"][:90]
            lines.append(f"{name:<92s}{int(r['Calls']):>7d}  {t / 1e6:>10.3f} ms  {float(r['AverageNs']) / 1e3:>10.2f} us"
                         f"  {100 * t / total:>6.2f} %")
    else:
        fetch, write, cfetch, cwrite = (_counter_means(dirs[0], "FETCH_SIZE"), _counter_means(dirs[1], "WRITE_SIZE"),
                                        _counter_means(dirs[2], "FETCH_SIZE"), _counter_means(dirs[3], "WRITE_SIZE"))
        # the calibration copy: the dispatch with the most bytes in each calibration run
        cf = max(v for _, v in cfetch.values())
        cw = max(v for _, v in cwrite.values())
        with open(args.prof_copy_json) as fh:
            cj = json.loads([ln for ln in fh if ln.startswith("{")][-1])
        step = [k for k in fetch if "arnoldi_step" in k]
        if len(step) != 1:
            raise SystemExit(f"expected one step kernel, found {step}")
        kname = step[0]
        nd, fk = fetch[kname]
        _, wk = write[kname]
        lines.append(f"# calibration: device copy reading {cj['copy_bytes_read']} B and writing "
                     f"{cj['copy_bytes_written']} B: FETCH_SIZE {cf:.1f} KiB, WRITE_SIZE {cw:.1f} KiB per dispatch")
        fs = cj["copy_bytes_read"] / 1024 / cf
        ws_ = cj["copy_bytes_written"] / 1024 / cw
        lines += [f"fetch_scale: {fs:.4f}", f"write_scale: {ws_:.4f}", f"kernel: {kname}", f"dispatches: {nd}",
                  f"fetch_kib_per_dispatch: {fk:.1f}", f"write_kib_per_dispatch: {wk:.1f}"]
        per_dispatch = 1024 * (fk * fs + wk * ws_)
        if "bytes_per_batch" in roof:
            per_batch_launches = roof["launches"] / run["steps"]
            batches = nd / per_batch_launches
            traffic = per_dispatch * nd / batches
            alg = roof["bytes_per_batch"]
            lines += [f"batches: {batches:.2f}", f"traffic_bytes_per_batch: {int(traffic)}",
                      f"algorithmic_bytes_per_batch: {alg}"]
        else:
            traffic = per_dispatch
            alg = roof["bytes_per_launch"]
            lines += [f"traffic_bytes_per_launch: {int(traffic)}", f"algorithmic_bytes_per_launch: {alg}"]
        lines += [f"traffic_over_algorithmic: {traffic / alg:.4f}", f"source_sha256: {_kernel_sha()}",
                  "# other kernels of the same runs (mean KiB per dispatch, unscaled): FETCH_SIZE / WRITE_SIZE"]
        for k in sorted(fetch, key=lambda k: -fetch[k][0] * fetch[k][1])[:12]:
            if k == kname:
                continue
            lines.append(f"#   {k[:86]:<88s}{fetch[k][0]:>6d}  {fetch[k][1]:>12.1f}  {write.get(k, (0, 0.0))[1]:>12.1f}")
    text = "\n".join(lines) + "\n"
    if args.prof_out:
        with open(args.prof_out, "w") as fh:
            fh.write(text)
    print(text, end="")


def copy_calibration(gib: float):
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n,
                      "copy_gbs": round(16 * n / dt / 1e9, 1)}), flush=True)


# bytes per element of (A values, basis vectors u_j, products A u_j) per precision form
PREC_BYTES = {"fp64": (8, 8, 8), "fp32": (4, 4, 4), "bf16basis": (4, 2, 4)}
PREC_DTYPE = {"fp64": "f64", "fp32": "f32", "bf16basis": "bf16+f32"}


def step_kernel_bytes(N: int, nnz: int, k: int, prec: str = "fp64") -> int:
    """Algorithmic HBM bytes of one fused Arnoldi step (int32 indices, implicit sketch):
    A once (nnz values + 4 nnz columns + 4 (N+1) row pointers), the k window vectors and
    A u_{j-1} read once, u_j and A u_j written once.  FP64: 12 nnz + 4(N+1) + 8(k+1)N + 16N."""
    ab, vb, wb = PREC_BYTES[prec]
    return (ab + 4) * nnz + 4 * (N + 1) + (k * vb + wb) * N + (vb + wb) * N


# the step kernel, its launch rule and the headers they share: the recorded counters
# belong to these sources and are dropped (traffic null) once any of them changes
KERNEL_SOURCES = ("paper_2208_11447_amd/csrc/arnoldi.hip", "paper_2208_11447_amd/csrc/common.hpp",
                  "paper_2208_11447_amd/csrc/device_state.hpp")


def storage_name(a_format: int) -> str:
    """Storage of A in the Arnoldi steps as reported by skfab_info.a_format."""
    if a_format == 0:
        return "csr"
    cols = "int16_offsets" if a_format & 3 == 2 else "int32_cols"
    vals = "uint8_value_table" if a_format & 4 else "values"
    return f"sell64_{cols}_{vals}"


def recorded_traffic(workload: str, prec: str, field: str = "traffic_bytes_per_launch"):
    """HBM bytes per step-kernel launch (per batch for the batched workload: field
    traffic_bytes_per_batch) from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of
    this workload (each counter scaled by its reading for a plain device copy of known size),
    or None when there is no summary or the step kernel's sources (or its launch code) have
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"arnoldi_step_{workload}_{prec}_hbm_counters.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if not line.startswith("#") and ":" in line:
                key, val = line.split(":", 1)
                fields[key.strip()] = val.strip()
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    if fields.get("source_sha256") != h.hexdigest():
        return None
    return int(fields[field])


def host_threads() -> int:
    """CPU threads this process may use: its affinity set, capped by OMP_NUM_THREADS
    when that is set (a GPU machine gives each GPU a share of its cores)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_legs(cfg, arrays, b, x_gpu, f, method, reps, tau=0.0, quad_tol=1e-13):
    """The oracle as it stands, on the same workload: `reps` full solves (sketch
    construction, m truncated-Arnoldi steps, small problem, assembly) with the BLAS
    pool at the host's thread share.  The first solve also gives the parity of the
    GPU result.  Returns (parity error, cpu_baseline dict or None)."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import arnoldi as oarn
    from oracle import methods as ometh
    from oracle import sketch as osk

    rp, col, val = arrays
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    threads = host_threads()
    from oracle import contour as ocont
    solve = {"sfom": lambda arn: ometh.sfom_closed(arn, f, tau),
             "sgmres": (lambda arn: ocont.sgmres_contour(arn, tau, tol=quad_tol)) if f == "exp"
             else (lambda arn: ometh.sgmres(arn, f, tol=quad_tol)),
             "sfom_quad": lambda arn: ometh.sfom_quad(arn, f, tol=1e-13)}[method]
    times, t_arn, err = [], [], None
    with threadpool_limits(limits=threads):
        for r in range(max(1, reps)):
            t0 = time.perf_counter()
            S = osk.sparse_sign_matrix(N, cfg["s"], cfg["zeta"], cfg["sketch_seed"])
            t1 = time.perf_counter()
            arn = oarn.truncated_arnoldi(A, b, cfg["m"], cfg["k"], S)
            t2 = time.perf_counter()
            xr = solve(arn).x
            times.append(time.perf_counter() - t0)
            t_arn.append(t2 - t1)
            if r == 0:
                err = float(np.linalg.norm(x_gpu - xr) / np.linalg.norm(xr))
            print(f"# oracle solve {r + 1}/{reps}: {times[-1]:.1f} s", file=sys.stderr, flush=True)
    if reps < 1:
        return err, None
    med = float(np.median(times))
    nnz = int(rp[-1])
    arn_bytes = cfg["m"] * step_kernel_bytes(N, nnz, cfg["k"])
    cpu = {"value": round(1.0 / med, 5), "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"median of {len(times)} full oracle solves of this workload (sketch build, "
                     f"{cfg['m']} truncated-Arnoldi steps, small problem, assembly); NumPy/SciPy BLAS pool "
                     f"{threads} threads, scipy.sparse products single-threaded",
           "sec_per_solve": [round(t, 2) for t in times],
           "arnoldi_gbs": round(arn_bytes / float(np.median(t_arn)) / 1e9, 2),
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    return err, cpu


def batch_step_bytes(Ns, nnzs, ms, R, k, prec):
    """Algorithmic bytes of every step launch of a batched solve, summed: in step j
    each problem with m_p >= j reads A once for its R right-hand sides (its blocks
    share it through L2) and each pair moves its own vectors (as step_kernel_bytes)."""
    ab, vb, wb = PREC_BYTES[prec]
    total = 0
    for N, nnz, m in zip(Ns, nnzs, ms):
        a_bytes = (ab + 4) * nnz + 4 * (N + 1)
        vec = (k * vb + wb) * N + (vb + wb) * N
        total += m * (a_bytes + R * vec)   # steps j = 0 .. m-1 (the extension pass has no product)
    return total


def run_batched(args):
    """The batched form: 64 2D convection-diffusion problems (grids 256^2..1024^2,
    convection U[10, 200], m U{80..250}, s = 2m, k = 2), 4 right-hand sides each,
    one skfab_solve_batched call per step of the benchmark."""
    import numpy as np
    import torch

    from paper_2208_11447_amd import skfab as sk
    from workloads import batched_problem_params, convdiff_csr

    R = 4
    params = batched_problem_params(args.nprob)
    probs, hosts = [], []
    t0 = time.perf_counter()
    for i, q in enumerate(params):
        rp, col, val = convdiff_csr(q["n"], 2, 1.0, q["c"])
        N = rp.size - 1
        B = np.random.default_rng(q["rhs_seedseq"]).standard_normal((R, N))
        A = sk.CSR.from_numpy(rp, col, val)
        Bt = torch.as_tensor(B, device="cuda")
        probs.append(sk.BatchProblem(A, Bt, torch.empty_like(Bt), m=q["m"], s=q["s"], seed=q["sketch_seed"]))
        hosts.append((rp, col, val, B))
        if i % 16 == 15:
            print(f"# generated {i + 1} problems ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    Ns = [q.A.n for q in probs]
    nnzs = [q.A.col.numel() for q in probs]
    ms = [q.m for q in probs]
    p = sk.make_params(f=args.f, k=2, zeta=8, method=args.method, quad_tol=1e-13, prec=args.prec)
    nbytes = sk.skfab_batch_workspace_bytes(probs, p)
    ws = sk.alloc_workspace(nbytes)
    ctx = sk.Context(0)
    print(f"# batch: {len(probs)} problems x {R} rhs, N {min(Ns)}..{max(Ns)} (sum {sum(Ns)}), m {min(ms)}..{max(ms)}, "
          f"workspace {nbytes / 2**30:.1f} GiB, prec {args.prec}", file=sys.stderr, flush=True)
    tuning = None
    if args.tuning:
        vals = [int(v) for v in args.tuning.split(",")]
        blk, spw, packed = vals[0], vals[1], bool(vals[2]) if len(vals) > 2 else False
        sk.skfab_batch_set_tuning(ctx, blk, spw, packed)
        tuning = (blk, spw, packed)
    elif not args.no_autotune:
        t = time.perf_counter()
        tuning = sk.skfab_batch_autotune(ctx, probs, p, ws, steps=4)
        print(f"# autotuned launch shape: block {tuning[0]}, {tuning[1]} slices per wavefront, packed form "
              f"{tuning[2]} ({time.perf_counter() - t:.1f} s)", file=sys.stderr, flush=True)
    else:
        tuning = sk.skfab_batch_get_tuning(ctx)
    info = sk.skfab_solve_batched(ctx, probs, p, ws)
    bad = [(i, r, info[i][r].status) for i in range(len(probs)) for r in range(R) if info[i][r].status != 0]
    for _ in range(args.warmup):
        sk.skfab_solve_batched(ctx, probs, p, ws, want_info=False)
    torch.cuda.synchronize()
    # every launch timed: the launches differ in size (units drop out as their m is reached)
    sk.skfab_timing_enable(ctx, True)
    sk.skfab_timing_read(ctx, 0)
    sk.skfab_timing_read(ctx, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sk.skfab_solve_batched(ctx, probs, p, ws, want_info=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step, n_step = sk.skfab_timing_read(ctx, 0)
    ms_asm, n_asm = sk.skfab_timing_read(ctx, 1)
    sk.skfab_timing_enable(ctx, False)
    step_bytes = batch_step_bytes(Ns, nnzs, ms, R, 2, args.prec) * args.steps
    achieved = step_bytes / (ms_step / 1e3) / 1e9
    asm_bytes = sum(R * (PREC_BYTES[args.prec][1] * N * m + 8 * N) for N, m in zip(Ns, ms)) * n_asm
    print(f"# timed {args.steps} batches in {elapsed:.3f} s; {len(bad)} pairs with a nonzero status {bad[:4]}",
          file=sys.stderr, flush=True)
    reck = None
    if args.reckless and bad:
        # the sketch size chosen by the computation for the pairs the batch refused
        s_cap = lambda i: min(4 * probs[i].s, 1024)  # (the library's largest sketch)
        s_mx = max(s_cap(i) for i, _, _ in bad)
        pr = sk.make_params(f=args.f, m=max(ms), k=2, zeta=8, s=s_mx, method=args.method, quad_tol=1e-13,
                            prec=args.prec)
        big = max(range(len(probs)), key=lambda i: Ns[i])
        wsr = sk.alloc_workspace(sk.skfab_workspace_bytes(probs[big].A, pr))
        rec, used, t0 = 0, [], time.perf_counter()
        for i, r, _ in bad:
            pq = sk.make_params(f=args.f, m=probs[i].m, k=2, zeta=8, s=2 * probs[i].s, seed=probs[i].seed,
                                method=args.method, quad_tol=1e-13, prec=args.prec)
            xr = torch.empty_like(probs[i].B[r])
            inf_r, s_u = sk.skfab_solve_reckless(ctx, probs[i].A, probs[i].B[r].contiguous(), xr, pq,
                                                 s_cap(i), 0.5, wsr)
            used.append([int(i), int(r), int(s_u), int(inf_r.status)])
            if inf_r.status == 0:
                rec += 1
                probs[i].X[r].copy_(xr)
                info[i][r] = inf_r
        torch.cuda.synchronize()
        reck = {"recovered": rec, "refused": len(bad), "seconds": round(time.perf_counter() - t0, 3),
                "s_start": "4m", "s_max": "min(8m, 1024)", "eps_max": 0.5, "pairs": used}
        print(f"# reckless s: {rec} of {len(bad)} refused pairs recovered", file=sys.stderr, flush=True)
    if args.save_outputs:
        s_used = {(p_[0], p_[1]): p_[2] for p_ in reck["pairs"]} if reck else None
        save_batch_outputs(args.save_outputs, probs, info, R, s_used)
    # parity on a bounded sample: the two smallest problems, first right-hand side
    parity = None
    if not args.no_parity:
        from oracle import arnoldi as oarn
        from oracle import methods as ometh
        from oracle import sketch as osk
        import scipy.sparse as sp
        errs = []
        for i in np.argsort(Ns)[:2]:
            rp, col, val, B = hosts[i]
            N = rp.size - 1
            A = sp.csr_matrix((val, col, rp), shape=(N, N))
            S = osk.sparse_sign_matrix(N, probs[i].s, 8, probs[i].seed)
            arn = oarn.truncated_arnoldi(A, B[0], probs[i].m, 2, S)
            xr = ometh.sfom_closed(arn, args.f).x if args.method == "sfom" else ometh.sgmres(arn, args.f,
                                                                                             tol=1e-13).x
            xg = probs[i].X[0].cpu().numpy()
            errs.append(float(np.linalg.norm(xg - xr) / np.linalg.norm(xr)))
        parity = {"rel_err_vs_oracle_max": max(errs), "sample": "problems with the two smallest N, rhs 0",
                  "tol": 1e-10 if args.prec == "fp64" else None}
        print(f"# parity vs oracle (sample): {errs}", file=sys.stderr, flush=True)
    solves = len(probs) * R
    ok = solves - len(bad)
    out = {
        "metric": "f(A)b solves/s and SpMV+sketch HBM GB/s at rel. err 1e-8 vs FP64 oracle",
        # pairs that end with a nonzero status are not counted as solves
        "value": round(ok * args.steps / elapsed, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": f"batch{len(probs)}x{R}_convdiff2d_{args.f}_{args.method}"
                   + ("" if args.prec == "fp64" else f"_{args.prec}"),
                   "problems": len(probs), "rhs_per_problem": R, "pairs_per_step": solves,
                   "solves_per_step": ok,
                   "N_range": [min(Ns), max(Ns)], "N_sum": sum(Ns), "m_range": [min(ms), max(ms)], "k": 2,
                   "s": "2m", "zeta": 8, "prec": args.prec, "tuning": tuning,
                   "a_storage": sorted({storage_name(info[i][0].a_format) for i in range(len(probs))}),
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     # counters are recorded per launch shape (null for a shape without a record)
                     "traffic": recorded_traffic(f"{args.workload}_t{tuning[0]}x{tuning[1]}"
                                                 + ("p" if tuning[2] else ""), args.prec,
                                                 "traffic_bytes_per_batch"),
                     "kernel": ("arnoldi_step_packed_kernel + arnoldi_step_batched_kernel" if tuning and tuning[2]
                                else "arnoldi_step_batched_kernel"), "bytes_per_batch": step_bytes // args.steps,
                     "launches": n_step, "step_ms_per_batch": round(ms_step / args.steps, 3),
                     "assembly_gbs": round(asm_bytes / (ms_asm / 1e3) / 1e9, 1) if n_asm else None},
        "cpu_baseline": None,
        "parity": parity,
        "nonzero_status_pairs": len(bad),
        "reckless_s": reck,
        "nonzero_status_list": [[int(i), int(r), int(st)] for i, r, st in bad],
    }
    print(json.dumps(out), flush=True)


SAMPLE_ENTRIES = 4096


def sample_index(N: int):
    """Fixed entries of a result kept by --save-outputs: evenly spaced over 0..N-1."""
    import numpy as np
    return np.unique(np.linspace(0, N - 1, SAMPLE_ENTRIES).astype(np.int64))


def save_batch_outputs(path, probs, info, R, s_used=None):
    """Every pair's status, m_used, flags, ||x||, x at the sample entries and the
    sketch size its result used (s_used: {(problem, rhs): s} for the pairs the
    s-adaptive solve redid, else the problem's s)."""
    import numpy as np
    rows = []
    for i, q in enumerate(probs):
        idx = sample_index(q.A.n)
        X = q.X.cpu().numpy()
        for r in range(R):
            rows.append((i, r, info[i][r].status, info[i][r].m_used, info[i][r].flags,
                         float(np.linalg.norm(X[r])), X[r][idx], (s_used or {}).get((i, r), q.s)))
    np.savez_compressed(path, prob=np.array([r[0] for r in rows]), rhs=np.array([r[1] for r in rows]),
                        s=np.array([r[7] for r in rows]),
                        status=np.array([r[2] for r in rows]), m_used=np.array([r[3] for r in rows]),
                        flags=np.array([r[4] for r in rows]), xnorm=np.array([r[5] for r in rows]),
                        xs=np.array([np.pad(r[6], (0, SAMPLE_ENTRIES - r[6].size)) for r in rows]))
    print(f"# saved {len(rows)} pair outputs to {path}", file=sys.stderr, flush=True)


def _oracle_pair(job):
    """One (problem, rhs) pair of the batched workload through the oracle (worker)."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import arnoldi as oarn
    from oracle import methods as ometh
    from oracle import sketch as osk
    from workloads import batched_problem_params, convdiff_csr

    pi, r, nprob, s = job
    q = batched_problem_params(nprob)[pi]
    with threadpool_limits(limits=1):
        rp, col, val = convdiff_csr(q["n"], 2, 1.0, q["c"])
        N = rp.size - 1
        A = sp.csr_matrix((val, col, rp), shape=(N, N))
        b = np.random.default_rng(q["rhs_seedseq"]).standard_normal((4, N))[r]
        S = osk.sparse_sign_matrix(N, s, 8, q["sketch_seed"])
        arn = oarn.truncated_arnoldi(A, b, q["m"], 2, S)
        out = {"N": N, "m": q["m"], "s": s}
        try:
            res = ometh.sfom_closed(arn, "invsqrt")
            out.update(verdict="ok", m_used=res.m_used, xnorm=float(np.linalg.norm(res.x)),
                       xs=res.x[sample_index(N)])
        except ometh.BranchError:
            w = ometh.whiten(ometh.regularize(arn)[0])
            ev = np.linalg.eigvals(w.M)
            neg = ev[(np.abs(ev.imag) <= 1e-12 * np.max(np.abs(ev))) & (ev.real <= 0)]
            out.update(verdict="branch", m_used=ometh.conditioned_prefix(arn),
                       cut_eigs=[float(v.real) for v in neg])
    return pi, r, out


def check_batch_outputs(path, nprob):
    """Oracle check of saved batched outputs (CPU): right-hand side 0 of every
    problem, every pair with a nonzero status and every pair the s-adaptive solve
    redid, through the oracle's own run of the same pair at the sketch size the
    saved result used.  A pair the GPU solved is compared on the sampled entries
    and on ||x||; a pair the GPU refused is classified by what the oracle does
    with it."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor

    d = np.load(path)
    from workloads import batched_problem_params
    qs = batched_problem_params(nprob)
    pairs = {(int(p), int(r)): k for k, (p, r) in enumerate(zip(d["prob"], d["rhs"]))}
    s_of = {pr: (int(d["s"][k]) if "s" in d else qs[pr[0]]["s"]) for pr, k in pairs.items()}
    todo = sorted({(p, 0) for p in range(nprob)} | {pr for pr, k in pairs.items() if d["status"][k] != 0}
                  | {pr for pr in pairs if s_of[pr] != qs[pr[0]]["s"]})
    rows = []
    worst = 0.0
    with ProcessPoolExecutor(max_workers=host_threads()) as ex:
        results = sorted(ex.map(_oracle_pair, [(p, r, nprob, s_of[(p, r)]) for p, r in todo]),
                         key=lambda t: (t[0], t[1]))
    print("problem rhs N m s gpu_status oracle gpu_m_used oracle_m_used rel_err_sampled rel_err_norm cut_eigs",
          flush=True)
    for pi, r, o in results:
        k = pairs[(pi, r)]
        gst = int(d["status"][k])
        e = en = "-"
        if o["verdict"] == "ok" and gst == 0:
            xs = d["xs"][k][: o["xs"].size]
            ev = float(np.linalg.norm(xs - o["xs"]) / np.linalg.norm(o["xs"]))
            evn = abs(float(d["xnorm"][k]) - o["xnorm"]) / o["xnorm"]
            worst = max(worst, ev, evn)
            e, en = f"{ev:.2e}", f"{evn:.2e}"
        rows.append((pi, r, o["N"], o["m"], o["s"], gst, o["verdict"], int(d["m_used"][k]), o["m_used"], e, en,
                     ",".join(f"{v:.3g}" for v in o.get("cut_eigs", [])) or "-"))
        print(" ".join(str(v) for v in rows[-1]), flush=True)
    agree = sum(1 for row in rows if (row[5] == 0) == (row[6] == "ok"))
    print(json.dumps({"checked_pairs": len(rows), "status_agrees_with_oracle": agree,
                      "max_rel_err_sampled": worst}), flush=True)


def run_paper51(args):
    """The paper's convection-diffusion experiment (Section 5.1): 100 x 100 grid,
    diffusion 1e-3, unit convection in direction [1, -1], b = ones / ||ones||, k = 4,
    s = 400, f = z^(-1/2).  For m = 10, 20, ..., 200 and both sketches (the paper's
    SRDCT and the sparse sign of the other workloads) the device solves with sketched
    FOM in closed form, sketched FOM by quadrature and sketched GMRES; errors against
    the reference A^(-1/2) b (sparse direct quadrature, no Krylov space) beside the
    error of the best approximation from K_m(A, b) (orthogonal projection)."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    from oracle import arnoldi as oarn
    from oracle import methods as ometh
    from oracle import reference
    from oracle import sketch as osk
    from paper_2208_11447_amd import skfab as sk
    from workloads import config, convdiff_csr, ones_rhs, srdct_draws

    cfg = config("paper51_convdiff2d_n100")
    rp, col, val = convdiff_csr(cfg["n"], 2, cfg["diffusion"], cfg["convection"], paper_direction=True)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    b = ones_rhs(N)
    t0 = time.perf_counter()
    truth = reference.invsqrt_apply(A, b, tol=1e-13)
    print(f"# reference A^(-1/2) b in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    full = oarn.full_arnoldi(A, b, cfg["m"])
    Q, _ = np.linalg.qr(full.V)
    nt = np.linalg.norm(truth)
    ms = list(range(10, cfg["m"] + 1, 10))
    best = {m: float(np.linalg.norm(truth - Q[:, :m] @ (Q[:, :m].T @ truth)) / nt) for m in ms}
    Ad = sk.CSR.from_numpy(rp, col, val)
    bd = torch.as_tensor(b, device="cuda")
    x = torch.empty_like(bd)
    ctx = sk.Context(0)
    signs, rows = srdct_draws(N, cfg["s"], cfg["sketch_seed"])
    sketches = {"srdct": (torch.as_tensor(signs, device="cuda"), torch.as_tensor(rows, device="cuda")),
                "sparse_sign": None}
    table = []
    for m in ms:
        row = {"m": m, "best": best[m]}
        for name, sr in sketches.items():
            # sFOM by quadrature at the tolerance of the paper's experiments (1e-7, Section 5.3)
            for method, qtol in (("sfom", 1e-13), ("sfom_quad", 1e-7), ("sgmres", 1e-13)):
                p = sk.make_params(f="invsqrt", m=m, k=cfg["k"], s=cfg["s"], zeta=cfg["zeta"], seed=cfg["sketch_seed"],
                                   method=method, quad_tol=qtol, srdct=sr)
                ws = sk.alloc_workspace(sk.skfab_workspace_bytes(Ad, p))
                info = sk.skfab_solve(ctx, Ad, bd, x, p, ws)
                e = float(np.linalg.norm(x.cpu().numpy() - truth) / nt) if info.status == 0 else None
                row[f"{name}_{method}"] = e
                row[f"{name}_{method}_status"] = int(info.status)
                if method == "sfom":
                    row[f"{name}_m_used"] = int(info.m_used)
                if method == "sfom_quad":
                    row[f"{name}_sfom_quad_l"] = int(info.l_used)
                    xq = x.cpu().numpy()
            # the closed form by a dense matrix function (the oracle: Schur square root of
            # the projected matrix), for the same sketch, against the device's quadrature
            S = osk.srdct_matrix(N, signs, rows) if sr is not None else osk.sparse_sign_matrix(N, cfg["s"], 8,
                                                                                               cfg["sketch_seed"])
            xo = ometh.sfom_closed(oarn.truncated_arnoldi(A, b, m, cfg["k"], S), "invsqrt").x
            row[f"{name}_quad_vs_dense_closed"] = float(np.linalg.norm(xq - xo) / np.linalg.norm(xo))
        table.append(row)
        print("# " + json.dumps(row), file=sys.stderr, flush=True)
    # closed form and quadrature of sketched FOM coincide (the paper's observation)
    gap = max(r[f"{n}_quad_vs_dense_closed"] for r in table for n in sketches)
    out = {"metric": "relative error of f(A)b approximants vs m (Section 5.1 convection-diffusion)",
           "config": {"workload": "paper51_convdiff2d_n100", "N": N, "k": cfg["k"], "s": cfg["s"],
                      "f": "invsqrt", "rhs": "ones/||ones||", "sketches": list(sketches)},
           "max_rel_gap_sfom_quad_tol1e-7_vs_dense_closed_form": gap, "table": table}
    print(json.dumps(out), flush=True)


def run_controller(args):
    """The learned controller: labels from 4 adaptive-m runs per training problem
    ((k, s/m) in {2, 4} x {2, 4}, tol 1e-8), full-batch training on the device
    kernels, then held-out problems solved by plain adaptive-m (k = 2, s = 2 m_cap,
    checks every 10 steps from m = 10) and by the controlled solve (features, network,
    checks from the predicted m, adaptive fallback)."""
    import numpy as np
    import torch

    from paper_2208_11447_amd import controller as ctl

    tol = 1e-8
    runner = ctl.Runner(0)
    t0 = time.perf_counter()
    X, Y, runs = [], [], 0
    specs = ctl.random_specs(args.train_problems, seed=11)
    for i, spec in enumerate(specs):
        f, lab, r = ctl.label_problem(runner, spec, tol)
        runs += r
        if lab is not None:
            X.append(f)
            Y.append(lab)
        if (i + 1) % 100 == 0:
            print(f"# labelled {i + 1} problems, {runs} runs ({time.perf_counter() - t0:.0f} s)", file=sys.stderr,
                  flush=True)
    t_label = time.perf_counter() - t0
    X, Y = np.asarray(X), np.asarray(Y)
    t0 = time.perf_counter()
    model = ctl.train(runner, X, Y, steps=3000, lr=2e-3, log_every=1000)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"# trained on {len(X)} labelled problems in {t_train:.1f} s, loss {model.history}", file=sys.stderr,
          flush=True)
    rows = []
    for i, spec in enumerate(ctl.random_specs(args.test_problems, seed=12)):
        A, b = spec.build()
        _, ip, mp, ep, sp_ = runner.adaptive(A, b, 2, 2, 10, ctl.M_CAP, tol)
        _, ic, mc, ec, sc, fb, _ = ctl.controlled_solve(runner, model, spec, A, b, tol)
        rows.append((ip.status == 0 and ep <= tol, ic.status == 0 and ec <= tol, sp_, sc, mp, mc, fb))
        if (i + 1) % 64 == 0:
            print(f"# evaluated {i + 1} held-out problems", file=sys.stderr, flush=True)
    ok_p = [r for r in rows if r[0]]
    t_p = sum(r[2] for r in ok_p)
    t_c = sum(r[3] for r in ok_p)
    out = {
        "metric": "f(A)b solves/s at rel. err 1e-8 (stopping estimate), learned controller vs plain adaptive-m",
        "value": round(len(ok_p) / t_c, 2) if t_c > 0 else None,
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "config": {"workload": "controller_convdiff2d3d", "train_problems": args.train_problems,
                   "method_runs": runs, "labelled": int(len(X)), "test_problems": args.test_problems,
                   "tol": tol, "network": "16-64-64-3 relu fp32", "train_steps": 3000},
        "plain_adaptive_solves_per_s": round(len(ok_p) / t_p, 2) if t_p > 0 else None,
        "speedup": round(t_p / t_c, 3) if t_c > 0 else None,
        "held_out_met_by_plain": len(ok_p),
        "held_out_met_by_controller": sum(1 for r in rows if r[1]),
        "controller_meets_tol_where_plain_does": sum(1 for r in ok_p if r[1]),
        "krylov_steps_plain": int(sum(r[4] for r in ok_p)),
        "krylov_steps_controller": int(sum(r[5] for r in ok_p)),
        "fallbacks": int(sum(r[6] for r in ok_p)),
        "label_seconds": round(t_label, 1),
        "train_seconds": round(t_train, 2),
        "train_loss": model.history,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.check_outputs:
        check_batch_outputs(args.check_outputs, args.nprob)
        return
    if args.summarize:
        summarize_profile(args)
        return
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2208_11447_amd import skfab as sk
    from workloads import config, convdiff_csr, gaussian_rhs

    if args.workload == "batch64x4":
        run_batched(args)
        return
    if args.workload == "controller":
        run_controller(args)
        return
    if args.workload == "paper51":
        run_paper51(args)
        return
    cfg = config(args.workload)
    rp, col, val = convdiff_csr(cfg["n"], cfg["dim"], cfg["diffusion"], cfg["convection"])
    N = rp.size - 1
    nnz = int(rp[-1])
    b = gaussian_rhs(N, cfg["rhs_seed"])
    dev = torch.device("cuda:0")
    A = sk.CSR.from_numpy(rp, col, val, device=dev)
    bd = torch.as_tensor(b, device=dev)
    x = torch.empty_like(bd)
    p = sk.make_params(f=args.f, m=cfg["m"], k=cfg["k"], s=cfg["s"], zeta=cfg["zeta"], seed=cfg["sketch_seed"],
                       method=args.method, quad_tol=args.quad_tol, prec=args.prec,
                       fparam=args.tau if args.f == "exp" else 0.0)
    ws = sk.alloc_workspace(sk.skfab_workspace_bytes(A, p), device=dev)
    ctx = sk.Context(0)
    if args.plain_values:
        sk.skfab_set_value_table(ctx, False)
    print(f"# workload {args.workload}: N={N} nnz={nnz} m={cfg['m']} k={cfg['k']} s={cfg['s']} "
          f"f={args.f} method={args.method} prec={args.prec}", file=sys.stderr, flush=True)

    info = sk.skfab_solve(ctx, A, bd, x, p, ws)
    if info.status != 0:
        raise RuntimeError(f"solve status {info.status}")
    for _ in range(args.warmup):
        sk.skfab_solve(ctx, A, bd, x, p, ws, want_info=False)
    torch.cuda.synchronize()

    timing = not args.no_timing_events
    if timing:
        sk.skfab_timing_enable(ctx, True, stride=args.timing_stride)
        sk.skfab_timing_read(ctx, 0)
        sk.skfab_timing_read(ctx, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sk.skfab_solve(ctx, A, bd, x, p, ws, want_info=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    roof = None
    if timing:
        ms_step, n_step = sk.skfab_timing_read(ctx, 0)
        ms_asm, n_asm = sk.skfab_timing_read(ctx, 1)
        sk.skfab_timing_enable(ctx, False)
        per_launch_s = ms_step / 1e3 / max(n_step, 1)
        nbytes = step_kernel_bytes(N, nnz, cfg["k"], args.prec)
        achieved = nbytes / per_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(args.workload, args.prec),
                "kernel": "arnoldi_step_kernel", "bytes_per_launch": nbytes,
                "mean_launch_us": round(per_launch_s * 1e6, 2), "launches": n_step,
                "timed": "every step launch j < m of every timed solve: one event pair per solve's run of m "
                         "launches (gaps between launches included)",
                "assembly_gbs": round((PREC_BYTES[args.prec][1] * N * cfg["m"] + 8 * N) / (ms_asm / 1e3 / max(n_asm, 1)) / 1e9, 1)
                if n_asm else None}
    x_host = x.cpu().numpy()
    print(f"# timed {args.steps} solves in {elapsed:.3f} s; m_used={info.m_used} l_used={info.l_used} "
          f"sigma={info.sigma:.4g} rcond={info.rcond_R:.3e} eps_est={info.eps_est:.3f} "
          f"relres={info.arnoldi_relres:.2e}", file=sys.stderr, flush=True)

    parity = None
    cpu = None
    if not (args.no_parity and args.no_cpu_baseline):
        reps = 0 if args.no_cpu_baseline else args.cpu_solves
        err, cpu = oracle_legs(cfg, (rp, col, val), b, x_host, args.f, args.method, reps,
                               tau=args.tau if args.f == "exp" else 0.0, quad_tol=args.quad_tol)
        if not args.no_parity:
            parity = {"rel_err_vs_oracle": err, "tol": 1e-10 if args.prec == "fp64" else None}
            print(f"# parity vs oracle: {err:.3e}", file=sys.stderr, flush=True)

    value = args.steps / elapsed
    out = {
        "metric": "f(A)b solves/s and SpMV+sketch HBM GB/s at rel. err 1e-8 vs FP64 oracle",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}_{args.f}_{args.method}"
                   + ("" if args.prec == "fp64" else f"_{args.prec}"), "grid": f"{cfg['n']}^{cfg['dim']}",
                   "N": N, "nnz": nnz, "m": cfg["m"], "k": cfg["k"], "s": cfg["s"], "zeta": cfg["zeta"],
                   "f": args.f, "method": args.method, "prec": args.prec,
                   **({"tau": args.tau} if args.f == "exp" else {}),
                   "a_storage": storage_name(info.a_format), "parallelism": "single-gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "small_problem": {"status": int(info.status), "m_used": int(info.m_used), "quad_order": int(info.l_used),
                          "quad_diff": float(info.quad_diff), "flags": int(info.flags)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
