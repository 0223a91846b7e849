#!/usr/bin/env python3
"""Benchmark: sign(H) + one structure-preserving spectral division step of
H = [[A, B], [-B, -A]] at n = 4096 (A, B of size m = 2048), Casida-like blocks.

One "step" is one pseudosym_divide call (estimate alpha/beta, two Zolotarev steps,
Sigma-orthonormal basis of the positive invariant subspace, decoupled H_+) on inputs
already resident in device memory.  Prints one JSON line (rank 0, one GPU).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--modes ...] [--no-cpu]
                    [--workload casida_n4096|ill_separated_n16384|batched_256|eig_n128|
                                eig_n4096|adjoint_n2048]

modes      : fp64 / mixed (precision of the Zolotarev steps) x basis (Alg. 6, or
             "-core": the basis from the half-size core); all are timed and reported,
             the primary one (the first of mixed-core, mixed, fp64-core, fp64 that was
             run) gives `value`.
value      : TFLOP/s of the primary mode = nominal algorithmic flops of the executed
             variant / measured time (flop convention below).
roofline   : the large-tile FP64 GEMM kernel (the dominant kernel class), its
             algorithmic flops per launch over its average launch duration, timed
             with HIP events around each launch on the library's stream during a
             separate instrumented pass over the same K steps.
cpu_baseline: the FP64 CPU oracle (Alg. 8 with LDL^T solves on the full matrix),
             timed on one shifted solve of Eq:LDLZolo at full size and scaled to the
             whole divide; the same leg computes the reference eigenvalues used for
             the relative eigenvalue error.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sign-fn+divide time & TFLOP/s at n=4096, mixed vs FP64, rel eig err ≤1e-10"
PEAK = {"f64": 78.6, "f32": 157.3}   # MI355X dense matrix-core peaks, TFLOP/s


def nominal_flops(m: int, r: int, step2_terms: int, basis: str = "alg6") -> float:
    """Algorithmic flops of the executed divide (standard LAPACK conventions: GEMM 2mnk,
    SYRK n^2 k, POTRF m^3/3, TRTRI m^3/3, triangular x full m^3, upper x lower
    triangular 2m^3/3, upper x upper triangular m^3/3)."""
    m3 = float(m) ** 3
    setup = 2 * (m3 / 3 + m3 / 3) + 2 * (2 * m3 / 3)        # chol+inverse of A+-B, Y0, Y0^-1
    step1 = m3 + r * (m3 / 3 + m3 / 3 + m3 / 3) + 2 * m3     # X^T X, r x (POTRF, TRTRI, W W^T), X(I+N)
    if step2_terms > 0:
        step2 = m3 + max(step2_terms - 2, 0) * 2 * m3 + 2 * m3   # X^T X, Horner, X T
    else:
        step2 = step1
    if basis == "core":
        # R_M^-1 U, R_K^-T (.), chol+inverse of G, (.) R_G^-1, R_K^-1 R_G^-1, H_+ (upper half)
        tail = m3 + m3 + 2 * m3 / 3 + m3 + m3 / 3 + m3 / 3
    else:
        assemble = 4 * m3                                     # S12 = W_M U R_K, S21 = R_M^T U W_K^T
        bases = 2 * m3 / 3 + m3                               # chol+inverse of (I+A_s)/2, B_s C^{-1}
        decouple = 2 * m3 + 2 * m3                            # R_M a, R_K b, F^T F (K = 2m)
        tail = assemble + bases + decouple
    return setup + step1 + step2 + tail


def gpu_leg(args, a, b):
    import numpy as np
    import torch
    from paper_2203_08900_amd import api

    A = torch.tensor(a, dtype=torch.float64, device="cuda:0")
    B = torch.tensor(b, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    out = {}
    for mode in args.modes:
        kw = dict(precision=mode.split("-")[0], r=args.r,
                  basis="core" if mode.endswith("-core") else "alg6")
        for _ in range(args.warmup):
            api.divide(A, B, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            Qp, Hp, info = api.divide(A, B, **kw)
            infos.append(info)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        info = infos[-1]
        flops = nominal_flops(args.m, info["r"], info["step2_terms"], kw["basis"])
        # instrumented pass: per-phase and per-launch kernel times
        gl, gms, gfl = 0, 0.0, 0.0
        phase = [0.0] * 8
        for _ in range(args.steps):
            _, _, ti = api.divide(A, B, timing=2, **kw)
            gl += ti["gemm_launches"]
            gms += ti["gemm_ms"]
            gfl += ti["gemm_flops"]
            phase = [p + q / args.steps for p, q in zip(phase, ti["phase_ms"])]
        torch.cuda.synchronize()
        Hh = Hp.cpu().numpy()
        w = np.linalg.eigvalsh(0.5 * (Hh + Hh.T))   # host LAPACK: the check, not the path
        out[mode] = {
            "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12, "flops": flops,
            "info": info, "w": np.sort(w), "phase_ms": phase,
            "gemm": {"launches": gl, "ms": gms, "flops": gfl},
        }
    return out


def batched_leg(args):
    """256 independent problems, m_i uniform over {32..512}: one batched call (worker
    streams) against the same problems called one at a time."""
    import numpy as np
    import torch
    from paper_2203_08900_amd import api, inputs

    sizes = inputs.batched_sizes(256, 2)
    probs = [inputs.small_dense(mi, i) for i, mi in enumerate(sizes)]
    As = [torch.tensor(a, dtype=torch.float64, device="cuda:0") for a, _ in probs]
    Bs = [torch.tensor(b, dtype=torch.float64, device="cuda:0") for _, b in probs]
    out = {}
    for mode in args.modes:
        kw = dict(precision=mode.split("-")[0], r=args.r,
                  basis="core" if mode.endswith("-core") else "alg6")
        for _ in range(args.warmup):
            api.divide_batched(As, Bs, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, Hs, infos = api.divide_batched(As, Bs, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        t0 = time.perf_counter()
        for A, B in zip(As, Bs):
            api.divide(A, B, **kw)
        torch.cuda.synchronize()
        ms_seq = (time.perf_counter() - t0) * 1e3
        flops = sum(nominal_flops(mi, inf["r"], inf["step2_terms"], kw["basis"])
                    for mi, inf in zip(sizes, infos))
        err = 0.0
        for i in range(0, 256, 32):
            a, b = probs[i]
            lam = np.sort(np.sqrt(np.linalg.eigvals((a - b) @ (a + b)).real))
            w = np.sort(np.linalg.eigvalsh(0.5 * (Hs[i] + Hs[i].T).cpu().numpy()))
            err = max(err, float(np.max(np.abs(w - lam) / lam)))
        out[mode] = {"ms": ms, "tflops": flops / (ms * 1e-3) / 1e12, "ms_one_at_a_time": ms_seq,
                     "rel_eig_err_sampled": err}
    primary = next((k for k in ("mixed-core", "mixed", "fp64-core", "fp64") if k in out),
                   args.modes[0])
    return {"metric": "batched sign-fn+divide, 256 problems n_i in {64..1024}", "value":
            out[primary]["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": out[primary]["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64" if primary.startswith("fp64") else "f32+f64",
            "data": "synthetic", "config": {"workload": "batched_256: m_i uniform over {32..512} "
                                            "(seed 2), small_dense(m_i, i) blocks",
                                            "problems": 256, "precision": primary},
            "modes": out}


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, out


def eig_leg(args):
    """All eigenpairs (pseudosym_eig): n = 128 (the plain-method case, seed 0) or
    n = 4096 (the Casida-like workload); error against the oracle's definition."""
    import numpy as np
    import torch
    from oracle import eig as eg
    from oracle import sign as sg
    from paper_2203_08900_amd import api, inputs

    if args.workload == "eig_n128":
        m = 64
        a, b = inputs.small_dense(m, 0)
        desc = "small_dense m=64 (n=128) seed 0: A = Q diag(U[1,10]) Q^T, ||B|| = 0.5 lambda_min(A)"
    else:
        m = 2048
        a, b = inputs.casida_like(m, 1)
        desc = "casida_like m=2048 (n=4096) seed 1"
    A = torch.tensor(a, dtype=torch.float64, device="cuda:0")
    B = torch.tensor(b, dtype=torch.float64, device="cuda:0")
    ms, (lam, V, info) = _timed(lambda: api.eig(A, B), args.steps, args.warmup)
    lam_ref, _ = eg.eig_casida(a, b)
    lam = lam.cpu().numpy()
    Vn = V.cpu().numpy()
    h = sg.casida_matrix(a, b)
    res = float(np.abs(h @ Vn - Vn * lam[None, :]).max() / np.abs(h).max())
    err = float(np.max(np.abs(lam - lam_ref) / np.abs(lam_ref)))
    return {"metric": "all eigenpairs of H (pseudosym_eig)", "value": ms, "unit": "ms",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": desc, "n": 2 * m, "m": m},
            "rel_eig_err": err, "residual": res, "splits": info["eig_splits"],
            "leaves": info["eig_leaves"], "max_jacobi_sweeps": info["eig_sweeps"]}


def adjoint_leg(args):
    """Forward (sign blocks + eigen-decomposition) and backward (adjoint) of the
    differentiable sign at n = 2048: casida_like(1024, 3), loss trace(W P_+)."""
    import numpy as np
    import torch
    from oracle import grad as gr
    from paper_2203_08900_amd import api, inputs

    m = 1024
    a, b = inputs.casida_like(m, 3)
    w = inputs.gradient_weight(m, 1003)
    A = torch.tensor(a, dtype=torch.float64, device="cuda:0")
    B = torch.tensor(b, dtype=torch.float64, device="cuda:0")
    ms_f, (SA, SB, lam, V, _) = _timed(lambda: api.sign_fwd(A, B), args.steps, args.warmup)
    gsa = torch.tensor(0.5 * (w[:m, :m] - w[m:, m:]).T, dtype=torch.float64, device="cuda:0")
    gsb = torch.tensor(0.5 * (w[m:, :m] - w[:m, m:]).T, dtype=torch.float64, device="cuda:0")
    ms_b, (gA, gB) = _timed(lambda: api.sign_bwd(lam, V, gsa, gsb), args.steps, args.warmup)
    ra, rb = gr.projector_loss_grad(a, b, w)
    err = float(max(np.linalg.norm(gA.cpu().numpy() - ra) / np.linalg.norm(ra),
                    np.linalg.norm(gB.cpu().numpy() - rb) / np.linalg.norm(rb)))
    return {"metric": "gradient of trace(W P_+) w.r.t. (A, B)", "value": ms_f + ms_b,
            "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_f + ms_b, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "casida_like m=1024 (n=2048) seed 3, W symmetric Gaussian "
                                   "seed 1003", "n": 2 * m, "m": m},
            "forward_ms": ms_f, "backward_ms": ms_b, "rel_grad_err_vs_oracle": err}


def copy_probe(nbytes: int = 512 << 20):
    """A plain streaming kernel of known size: y = -x over nbytes of FP64 (reads and
    writes nbytes each)."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()


def kernel_source_hash(paths) -> str:
    """sha256 (first 16 hex digits) of the concatenated kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


GEMM_SOURCES = [os.path.join(ROOT, "paper_2203_08900_amd", "csrc", f)
                for f in ("gemm_f64.hip", "gemm_tile.h")]


def traffic_from_profile(kernel_srcs):
    """HBM bytes per launch of the large-tile GEMM from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "gemm_f64_128x128_traffic_casida_n4096.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash(kernel_srcs):
        return None
    return float(kv["hbm_bytes_per_launch"])


def cpu_leg(args, a, b, lam_pos=None):
    """The oracle: one shifted LDL^T solve of Eq:LDLZolo at full size (the unit that
    dominates the paper-literal divide), and the reference eigenvalues (the oracle's
    definition, unless the construction fixes them)."""
    import numpy as np
    import scipy.linalg as sla

    from oracle import eig as eg
    from oracle import sign as sg
    from oracle import zolotarev as zol

    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    m = a.shape[0]
    t_eig = time.perf_counter()
    if lam_pos is None:
        lam, _ = eg.eig_casida(a, b)
        lp = lam[:m]
    else:
        lp = lam_pos
    t_eig = time.perf_counter() - t_eig
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(m)
    alpha, beta = 1.01 * lp.max(), 0.99 * lp.min()
    x = h / alpha
    co = zol.coefficients(beta / alpha, args.r)
    t0 = time.perf_counter()
    xtsx = x.T @ (sigma[:, None] * x)
    t_gram = time.perf_counter() - t0
    t0 = time.perf_counter()
    z = xtsx + co.c[0] * np.diag(sigma)
    lu, d, perm = sla.ldl(z, lower=True)
    w = sg.ldl_solve(lu, d, perm, np.diag(sigma))
    _ = x @ w
    t_shift = time.perf_counter() - t0
    t_total = 2 * (t_gram + args.r * t_shift)
    return {"t_shift": t_shift, "t_gram": t_gram, "t_total": t_total, "threads": threads,
            "lam_pos": lp, "t_eig": t_eig}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="casida_n4096",
                    choices=["casida_n4096", "ill_separated_n16384", "batched_256", "eig_n128",
                             "eig_n4096", "adjoint_n2048"])
    ap.add_argument("--m", type=int, default=0, help="override the half size m")
    ap.add_argument("--r", type=int, default=8)
    ap.add_argument("--modes", default="fp64,mixed,fp64-core,mixed-core")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain device copy of 512 MiB three times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    args = ap.parse_args()
    args.modes = [s for s in args.modes.split(",") if s]
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the method is benchmarked "
              "at its real single-GPU shape and this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    from paper_2203_08900_amd import inputs

    if args.copy_probe:
        copy_probe()
    exact = None
    if args.workload == "batched_256":
        print(json.dumps(batched_leg(args)), flush=True)
        return
    if args.workload in ("eig_n128", "eig_n4096"):
        print(json.dumps(eig_leg(args)), flush=True)
        return
    if args.workload == "adjoint_n2048":
        print(json.dumps(adjoint_leg(args)), flush=True)
        return
    if args.workload == "casida_n4096":
        args.m = args.m or 2048
        args.seed = 1
        a, b = inputs.casida_like(args.m, args.seed)
        desc = (f"casida_like m={args.m} (n={2 * args.m}) seed 1: A = diag(U[0.2,5]) + rank-64 "
                "PSD coupling (norm 0.05), B rank-64 symmetric, ||B|| = 0.3 lambda_min(A)")
    else:
        args.m = args.m or 8192
        args.seed = 4
        a, b, mu = inputs.ill_separated(args.m, args.seed)
        exact = np.sqrt(mu)
        desc = (f"ill_separated m={args.m} (n={2 * args.m}) seed 4: eig((A-B)(A+B)) = mu, "
                "log-uniform in [1e-6, 1], l = 1e-3")
    g = gpu_leg(args, a, b)
    primary = next((k for k in ("mixed-core", "mixed", "fp64-core", "fp64") if k in g),
                   args.modes[0])
    res = g[primary]

    cpu = None
    rel_err = {}
    if exact is not None:
        for mode, r in g.items():
            rel_err[mode] = float(np.max(np.abs(r["w"] - exact) / exact))
    if not args.no_cpu:
        c = cpu_leg(args, a, b, exact)
        for mode, r in g.items():
            rel_err[mode] = float(np.max(np.abs(r["w"] - c["lam_pos"]) / c["lam_pos"]))
        cpu_tflops = res["flops"] / c["t_total"] / 1e12
        cpu = {
            "value": cpu_tflops, "unit": "TFLOP/s", "cores": c["threads"], "kind": "oracle",
            "sample": (f"one of the 2r = {2 * args.r} shifted LDL^T solves of Eq:LDLZolo on the full "
                       f"{2 * args.m}x{2 * args.m} matrix ({c['t_shift']:.2f} s) plus one Gram product "
                       f"({c['t_gram']:.2f} s), scaled to the divide as 2 x (Gram + r solves) = "
                       f"{c['t_total']:.1f} s; the flop numerator is the GPU variant's nominal count"),
        }

    gm = res["gemm"]
    roof = None
    if gm["launches"] > 0 and gm["ms"] > 0:
        achieved = gm["flops"] / (gm["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK["f64"], "unit": "TFLOP/s",
                "frac": achieved / PEAK["f64"],
                "traffic": traffic_from_profile(GEMM_SOURCES),
                "kernel": "gemm_mfma_kernel<double,128,128,4,4>",
                "launches_per_step": gm["launches"] / args.steps,
                "avg_launch_ms": gm["ms"] / gm["launches"],
                "flops_per_launch": gm["flops"] / gm["launches"]}

    line = {
        "metric": METRIC,
        "value": res["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if primary.startswith("fp64") else "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc,
                   "n": 2 * args.m, "m": args.m, "r": args.r, "precision": primary,
                   "step2_terms": res["info"]["step2_terms"],
                   "nominal_gflop": res["flops"] / 1e9},
        "roofline": roof,
        "cpu_baseline": cpu,
        "rel_eig_err": rel_err.get(primary),
        "modes": {k: {"ms": v["ms"], "tflops": v["tflops"], "rel_eig_err": rel_err.get(k),
                      "phase_ms": [round(x, 4) for x in v["phase_ms"]],
                      "alpha": v["info"]["alpha"], "beta": v["info"]["beta"],
                      "restarts": v["info"]["restarts"]} for k, v in g.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
