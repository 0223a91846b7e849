#!/usr/bin/env python3
"""Benchmark: sign(H) + one structure-preserving spectral division step of
H = [[A, B], [-B, -A]] at n = 4096 (A, B of size m = 2048), Casida-like blocks.

One "step" is one pseudosym_divide call (estimate alpha/beta, two Zolotarev steps,
Sigma-orthonormal basis of the positive invariant subspace, decoupled H_+) on inputs
already resident in device memory.  Prints one JSON line (rank 0, one GPU).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--modes ...] [--no-cpu]
                    [--workload casida_n4096|ill_separated_n16384|batched_256|eig_n128|
                                eig_n4096|adjoint_n2048|general_n5000|bse2_n2048]

modes      : fp64 / mixed (precision of the Zolotarev steps) x basis (Alg. 6, or
             "-core": the basis from the half-size core, or "-ldl": Alg. 7 with the
             pivoted LDL^T); all are timed and reported,
             the primary one (the first of mixed-core, mixed, fp64-core, fp64 that was
             run) gives `value`.
value      : TFLOP/s of the primary mode = nominal algorithmic flops of the executed
             variant / measured time (flop convention below).
roofline   : the kernel class with the largest summed GPU time in the primary mode
             (a separate instrumented pass over the same K steps brackets every launch
             of the matrix-core kernels with HIP events on the stream it runs on): its
             algorithmic flops per launch over its average launch duration, against
             the matrix-core peak of its precision; "kernels" lists every class.
cpu_baseline: the FP64 CPU oracle (Alg. 8 with LDL^T solves on the full matrix, Alg. 6
             bases, the decoupled block), one whole divide timed on the host; the
             same leg computes the reference eigenvalues used for the relative
             eigenvalue error.
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
        # X^T X (symmetric: m^3), Horner products of commuting symmetric factors (symmetric
        # results: m^3 each), X T (2 m^3)
        step2 = m3 + max(step2_terms - 2, 0) * m3 + 2 * m3
    else:
        step2 = step1
    if basis == "core":
        # R_M^-1 U, R_K^-T (.), chol+inverse of G, (.) R_G^-1, R_K^-1 R_G^-1, H_+ (upper half)
        tail = m3 + m3 + 2 * m3 / 3 + m3 + m3 / 3 + m3 / 3
    else:
        assemble = 4 * m3                                     # S12 = W_M U R_K, S21 = R_M^T U W_K^T
        if basis == "ldl":
            # Alg. 7: rank-m pivoted LDL^T of the 2m x 2m Sigma P_+, sum over pivots j of
            # (2m - j)^2 for j < m = 7m^3/3
            bases = 7 * m3 / 3
        else:
            bases = 2 * m3 / 3 + m3                           # chol+inverse of (I+A_s)/2, B_s C^{-1}
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
        kw = mode_options(mode, args.r)
        # a tuning table applies to the precision and basis it was measured on
        t = args.tuning_table
        api.set_gemm_tuning(t["entries"] if t and (t["precision"], t["basis"]) ==
                            (kw["precision"], kw["basis"]) and kw["refine"] == "rr" else [])
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
        nk = len(api.KERNEL_CLASSES)
        kl, kms, kfl = [0] * nk, [0.0] * nk, [0.0] * nk
        phase = [0.0] * 8
        for _ in range(args.steps):
            _, _, ti = api.divide(A, B, timing=2, **kw)
            for c in range(nk):
                kl[c] += ti["kclass_launches"][c]
                kms[c] += ti["kclass_ms"][c]
                kfl[c] += ti["kclass_flops"][c]
            phase = [p + q / args.steps for p, q in zip(phase, ti["phase_ms"])]
        torch.cuda.synchronize()
        Hh = Hp.cpu().numpy()
        w = np.linalg.eigvalsh(0.5 * (Hh + Hh.T))   # host LAPACK: the check, not the path
        out[mode] = {
            "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12, "flops": flops,
            "info": info, "w": np.sort(w), "phase_ms": phase,
            "kclass": {"launches": kl, "ms": kms, "flops": kfl},
        }
    return out


def mode_options(mode: str, r: int):
    """precision[-core|-ldl][-norefine]: FP64 or mixed steps, Alg. 6, the core basis or
    Alg. 7, and the FP64 refinement (default) or none (the mixed path's result before
    refinement)."""
    parts = mode.split("-")
    return dict(precision=parts[0], r=r,
                basis="core" if "core" in parts else ("ldl" if "ldl" in parts else "alg6"),
                refine="none" if "norefine" in parts else "rr")


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
        kw = mode_options(mode, args.r)
        if kw["basis"] == "ldl":   # the batched call offers Alg. 6 and the core basis
            continue
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
        # instrumented pass: per-class kernel times (the class pipelines then run without
        # graphs; each reports its classes in its first problem's record)
        nk = len(api.KERNEL_CLASSES)
        kc = {"launches": [0] * nk, "ms": [0.0] * nk, "flops": [0.0] * nk}
        for _ in range(args.steps):
            _, _, tinfos = api.divide_batched(As, Bs, timing=2, **kw)
            for ti in tinfos:
                for c in range(nk):
                    kc["launches"][c] += ti["kclass_launches"][c]
                    kc["ms"][c] += ti["kclass_ms"][c]
                    kc["flops"][c] += ti["kclass_flops"][c]
        torch.cuda.synchronize()
        out[mode] = {"ms": ms, "tflops": flops / (ms * 1e-3) / 1e12, "ms_one_at_a_time": ms_seq,
                     "rel_eig_err_sampled": err, "kclass": kc}
    primary = next((k for k in ("mixed-core", "mixed", "fp64-core", "fp64") if k in out),
                   args.modes[0])
    return {"metric": "batched sign-fn+divide, 256 problems n_i in {64..1024}", "value":
            out[primary]["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": out[primary]["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64" if primary.startswith("fp64") else "f32+f64",
            "data": "synthetic", "config": {"workload": "batched_256: m_i uniform over {32..512} "
                                            "(seed 2), small_dense(m_i, i) blocks",
                                            "problems": 256, "precision": primary},
            # per-class times are summed over the worker streams, which run at once
            "roofline": roofline(out[primary]["kclass"], args.steps, out[primary]["ms"]),
            "modes": {k: {q: v for q, v in e.items() if q != "kclass"} for k, e in out.items()}}


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
            "leaves": info["eig_leaves"], "max_jacobi_sweeps": info["eig_sweeps"],
            "zolotarev_steps": info["eig_steps"], "restarts": info["eig_restarts"]}


def adjoint_leg(args):
    """Forward and backward of the differentiable sign at n = 2048: casida_like(1024, 3),
    loss trace(W P_+).  Primary: the stored-factor adjoint (sign pipeline keeping the
    iteration's factors, reverse mode through them); beside it the eigenbasis adjoint
    (sign blocks + eigen-decomposition, divided differences)."""
    import numpy as np
    import torch
    from oracle import grad as gr
    from paper_2203_08900_amd import api, inputs

    m = 1024
    a, b = inputs.casida_like(m, 3)
    w = inputs.gradient_weight(m, 1003)
    A = torch.tensor(a, dtype=torch.float64, device="cuda:0")
    B = torch.tensor(b, dtype=torch.float64, device="cuda:0")
    gsa = torch.tensor(0.5 * (w[:m, :m] - w[m:, m:]).T, dtype=torch.float64, device="cuda:0")
    gsb = torch.tensor(0.5 * (w[m:, :m] - w[:m, m:]).T, dtype=torch.float64, device="cuda:0")
    ra, rb = gr.projector_loss_grad(a, b, w)

    def err_of(gA, gB):
        return float(max(np.linalg.norm(gA.cpu().numpy() - ra) / np.linalg.norm(ra),
                         np.linalg.norm(gB.cpu().numpy() - rb) / np.linalg.norm(rb)))

    ms_fi, (_, _, store, _) = _timed(lambda: api.sign_fwd_iter(A, B), args.steps, args.warmup)
    ms_bi, (gA, gB) = _timed(lambda: api.sign_bwd_iter(store, gsa, gsb), args.steps,
                             args.warmup)
    err_i = err_of(gA, gB)
    ms_f, (SA, SB, lam, V, _) = _timed(lambda: api.sign_fwd(A, B), args.steps, args.warmup)
    ms_b, (gA, gB) = _timed(lambda: api.sign_bwd(lam, V, gsa, gsb), args.steps, args.warmup)
    err = err_of(gA, gB)
    return {"metric": "gradient of trace(W P_+) w.r.t. (A, B)", "value": ms_fi + ms_bi,
            "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_fi + ms_bi, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "casida_like m=1024 (n=2048) seed 3, W symmetric Gaussian "
                                   "seed 1003", "n": 2 * m, "m": m,
                       "adjoint": "stored iteration factors"},
            "forward_ms": ms_fi, "backward_ms": ms_bi, "rel_grad_err_vs_oracle": err_i,
            "eigenbasis": {"forward_ms": ms_f, "backward_ms": ms_b,
                           "rel_grad_err_vs_oracle": err}}


def general_leg(args):
    """Division of the random definite pseudosymmetric matrices of the paper's experiments
    (any signature, H = Sigma Q D Q^T, D equally spaced in [1, kappa]): the n = 5000
    matrix of the runtime table at kappa = 1e2 (time per divide, backward error), and the
    n = 250 backward-error experiment (10 matrices per kappa, kappa = 1e1 .. 1e12), with
    the Alg. 6 bases (the headline time) and with the bases from the projectors of the
    congruent symmetric T."""
    import numpy as np
    import torch
    from paper_2203_08900_amd import api, inputs

    n = args.m or 5000
    h, sig = inputs.general_sigma(n, 0, 1e2)
    H = torch.tensor(h, dtype=torch.float64, device="cuda:0")
    ms, (Qp, Qm, Hp, Hm, _, info) = _timed(lambda: api.divide_general(H, sig), args.steps,
                                           args.warmup)
    kc = kclass_sums(lambda: api.divide_general(H, sig, timing=2)[5], args.steps)
    Hs = torch.tensor(sig[:, None] * h, dtype=torch.float64, device="cuda:0")
    bwd = float(torch.linalg.norm(Qp.T @ Hs @ Qm) / torch.linalg.norm(H))
    # the bases from the projectors of T (no sign(H) formed)
    ms_c, (Qpc, Qmc, _, _, _, info_c) = _timed(
        lambda: api.divide_general(H, sig, basis="congruent"), args.steps, args.warmup)
    bwd_c = float(torch.linalg.norm(Qpc.T @ Hs @ Qmc) / torch.linalg.norm(H))

    def sweep_of(basis, kappas):
        out = {}
        for kappa in kappas:
            errs = []
            for seed in range(10):
                h2, s2 = inputs.general_sigma(250, 100 + seed, kappa)
                H2 = torch.tensor(h2, dtype=torch.float64, device="cuda:0")
                qp, qm, _, _, _, inf = api.divide_general(H2, s2, raise_on_error=False,
                                                          basis=basis)
                if inf["rc"] != 0:
                    errs.append(float("nan"))
                    continue
                S2 = torch.tensor(s2[:, None] * h2, dtype=torch.float64, device="cuda:0")
                errs.append(float(torch.linalg.norm(qp.T @ S2 @ qm) / torch.linalg.norm(H2)))
            ok = [e for e in errs if e == e]
            out[f"{kappa:g}"] = {"mean": float(np.mean(ok)) if ok else None,
                                 "max": float(np.max(ok)) if ok else None,
                                 "failures": len(errs) - len(ok)}
        return out

    kappas = () if args.no_sweep else (1e1, 1e2, 1e4, 1e6, 1e8, 1e10, 1e12)
    sweep = sweep_of("alg6", kappas)
    sweep_c = sweep_of("congruent", kappas)
    return {"metric": "spectral division of a definite pseudosymmetric matrix, any signature",
            "value": ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"general_sigma n={n} seed 0 kappa=1e2: H = Sigma Q D Q^T, "
                                   "random signature, D = linspace(1, kappa)", "n": n,
                       "r_plus": int(np.sum(sig > 0))},
            "roofline": roofline(kc, args.steps, ms),
            "steps_taken": info["steps"], "restarts": info["restarts"], "backward_error": bwd,
            "cond_est": info["cond_est"],
            "backward_error_n250": sweep,
            "congruent_basis": {"ms": ms_c, "backward_error": bwd_c,
                                "steps_taken": info_c["steps"],
                                "backward_error_n250": sweep_c}}


def bse_leg(args):
    """The complex Casida form Eq:BSE2 (A, B Hermitian) at complex m = 1024 (n = 2048):
    sign + division in FP64 and mixed precision, Alg. 6 and the core basis.  The rate
    counts the complex algorithm's flops (one complex multiply-add = 8 real flops, 4x the
    real count at the same m); the library computes it on the realified real form at
    half-size 2m, whose real flops are twice that.  Relative eigenvalue error of H_+
    against the positive eigenvalues of H from LAPACK's complex eigensolver on the host."""
    import numpy as np
    import torch
    from paper_2203_08900_amd import api, inputs

    m = args.m or 1024
    a, b = inputs.bse2_like(m, 1)
    A = torch.tensor(a, dtype=torch.complex128, device="cuda:0")
    B = torch.tensor(b, dtype=torch.complex128, device="cuda:0")
    h = np.block([[a, b], [-b, -a]])
    lam = np.linalg.eigvals(h).real
    lam = np.sort(lam[lam > 0])
    modes = {}
    for mode in ("fp64", "mixed", "fp64-core", "mixed-core"):
        kw = mode_options(mode, args.r)
        ms, (Qp, Hp, info) = _timed(lambda: api.divide_hermitian(A, B, **kw), args.steps,
                                    args.warmup)
        Hh = Hp.cpu().numpy()
        w = np.sort(np.linalg.eigvalsh(0.5 * (Hh + Hh.conj().T)))
        flops = 4.0 * nominal_flops(m, info["r"], info["step2_terms"], kw["basis"])
        modes[mode] = {"ms": ms, "tflops": flops / (ms * 1e-3) / 1e12,
                       "rel_eig_err": float(np.max(np.abs(w - lam) / lam))}
    kw = mode_options("mixed-core", args.r)
    kc = kclass_sums(lambda: api.divide_hermitian(A, B, timing=2, **kw)[2], args.steps)
    primary = modes["mixed-core"]
    return {"metric": "sign-fn+divide time & TFLOP/s, complex Casida form (Eq:BSE2)",
            "value": primary["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": primary["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": f"bse2_like m={m} (n={2 * m}) seed 1: A = U diag(U[1,10]) U^H, "
                                   "B Hermitian Gaussian, ||B|| = 0.5 lambda_min(A)",
                       "n": 2 * m, "m": m, "precision": "mixed-core"},
            "roofline": roofline(kc, args.steps, primary["ms"]),
            "rel_eig_err": primary["rel_eig_err"], "modes": modes}


TUNING_DIR = os.path.join(ROOT, "paper_2203_08900_amd", "tuning")


def install_tuning(args):
    """Load the GEMM tuning table the run asks for (args.tuning_table; the casida workload
    installs it for the modes of its precision and basis, the others for the whole run);
    returns its path or None."""
    args.tuning_table = None
    if args.tuning == "none":
        return None
    path = args.tuning
    if path == "auto":
        path = os.path.join(TUNING_DIR, f"{args.workload}.json")
        if not os.path.exists(path):
            return None
        import torch
        if json.load(open(path)).get("device") != torch.cuda.get_device_name(0):
            return None
    args.tuning_table = json.load(open(path))
    if args.workload != "casida_n4096":
        from paper_2203_08900_amd import autotune
        autotune.load(path)
    return os.path.relpath(path, ROOT)


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


_CSRC = os.path.join(ROOT, "paper_2203_08900_amd", "csrc")
# per kernel class: the committed HBM-traffic summary and the sources the kernel is
# built from (the counters only count while those sources are unchanged)
TRAFFIC_PROFILES = {
    0: ("chol_step_wide_f64_traffic_casida_n4096.txt", ["chol_f64.hip", "chol_block.h", "gemm_tile.h"]),
    3: ("gemm_f64_128x128_traffic_casida_n4096.txt", ["gemm_f64.hip", "gemm_tile.h"]),
    4: ("gemm_f64_64x64_traffic_casida_n4096.txt", ["gemm_f64.hip", "gemm_tile.h"]),
}
CLASS_DTYPE = ["f64", "f64", "f32", "f64", "f64", "f32"]


def kclass_sums(call, steps):
    """Per-class kernel sums (launches, ms, algorithmic flops) over `steps` calls of
    call() -> info made with timing = 2."""
    import torch
    from paper_2203_08900_amd import api
    nk = len(api.KERNEL_CLASSES)
    kc = {"launches": [0] * nk, "ms": [0.0] * nk, "flops": [0.0] * nk}
    for _ in range(steps):
        ti = call()
        for c in range(nk):
            kc["launches"][c] += ti["kclass_launches"][c]
            kc["ms"][c] += ti["kclass_ms"][c]
            kc["flops"][c] += ti["kclass_flops"][c]
    torch.cuda.synchronize()
    return kc


def roofline(kc, steps, step_ms, traffic=None):
    """The roofline object of a step from per-class kernel sums over `steps` instrumented
    steps (launches, ms, algorithmic flops per class): every class's achieved rate against
    its peak, and the class with the largest summed time as the dominant kernel.
    traffic(cls) gives that class's HBM bytes per launch from a committed counter
    summary of this workload, or None."""
    kernels = []
    for cls, name in enumerate(api_classes()):
        if kc["launches"][cls] == 0 or kc["ms"][cls] <= 0:
            continue
        ach = kc["flops"][cls] / (kc["ms"][cls] * 1e-3) / 1e12
        peak = PEAK[CLASS_DTYPE[cls]]
        kernels.append({"kernel": name, "launches_per_step": kc["launches"][cls] / steps,
                        "ms_per_step": kc["ms"][cls] / steps,
                        "avg_launch_ms": kc["ms"][cls] / kc["launches"][cls],
                        "achieved": ach, "peak": peak, "frac": ach / peak,
                        "share_of_step": kc["ms"][cls] / steps / step_ms})
    if not kernels:
        return None
    k = max(kernels, key=lambda e: e["ms_per_step"])
    cls = api_classes().index(k["kernel"])
    return {"bound": "mfma", "achieved": k["achieved"], "peak": k["peak"], "unit": "TFLOP/s",
            "frac": k["frac"], "traffic": traffic(cls) if traffic else None,
            "kernel": k["kernel"], "launches_per_step": k["launches_per_step"],
            "avg_launch_ms": k["avg_launch_ms"],
            "flops_per_launch": kc["flops"][cls] / kc["launches"][cls],
            "kernels": kernels}


def traffic_from_profile(cls):
    """HBM bytes per launch of kernel class `cls` from the committed counter summary, or
    None when there is none or the kernel sources changed since the counters were taken."""
    if cls not in TRAFFIC_PROFILES:
        return None
    name, srcs = TRAFFIC_PROFILES[cls]
    kernel_srcs = [os.path.join(_CSRC, f) for f in srcs]
    path = os.path.join(ROOT, "profiles", name)
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


def host_cpu():
    """CPU model, physical cores and the BLAS thread count of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:  # pragma: no cover
        pass
    try:
        import psutil
        phys = psutil.cpu_count(logical=False)
    except Exception:  # pragma: no cover
        phys = None
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    return model, phys, threads


def cpu_leg(args, a, b, lam_pos=None, whole=True):
    """The oracle on the host: one whole divide (Alg. 8 with Bunch-Kaufman LDL^T solves on
    the full 2m x 2m matrix, alpha and beta from the definition, Alg. 6 bases, the
    decoupled block), timed once, and the reference eigenvalues (the oracle's definition,
    unless the construction fixes them)."""
    from oracle import divide as dv
    from oracle import eig as eg

    model, phys, threads = host_cpu()
    m = a.shape[0]
    t_eig = time.perf_counter()
    if lam_pos is None:
        lam, _ = eg.eig_casida(a, b)
        lp = lam[:m]
    else:
        lp = lam_pos
    t_eig = time.perf_counter() - t_eig
    t_total = None
    if whole:
        t0 = time.perf_counter()
        dv.divide_casida(a, b, r=args.r)
        t_total = time.perf_counter() - t0
    return {"t_total": t_total, "threads": threads, "model": model, "physical_cores": phys,
            "lam_pos": lp, "t_eig": t_eig}


def api_classes():
    from paper_2203_08900_amd import api
    return api.KERNEL_CLASSES


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="casida_n4096",
                    choices=["casida_n4096", "ill_separated_n16384", "batched_256", "eig_n128",
                             "eig_n4096", "adjoint_n2048", "general_n5000", "bse2_n2048"])
    ap.add_argument("--m", type=int, default=0, help="override the half size m")
    ap.add_argument("--tuning", default="auto",
                    help="GEMM tuning table (JSON of paper_2203_08900_amd.autotune) to install "
                         "before timing; 'auto': the package's table for this workload when it "
                         "was made on this device type; 'none': the built-in choices")
    ap.add_argument("--r", type=int, default=8)
    ap.add_argument("--modes",
                    default="fp64,mixed,fp64-core,mixed-core,mixed-core-norefine,mixed-ldl")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="general_n5000: skip the n = 250 backward-error sweeps")
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
    tuning_used = install_tuning(args)
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
    if args.workload == "general_n5000":
        print(json.dumps(general_leg(args)), flush=True)
        return
    if args.workload == "bse2_n2048":
        print(json.dumps(bse_leg(args)), flush=True)
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
        c = cpu_leg(args, a, b, exact, whole=args.workload == "casida_n4096")
        for mode, r in g.items():
            rel_err[mode] = float(np.max(np.abs(r["w"] - c["lam_pos"]) / c["lam_pos"]))
        if c["t_total"] is not None:
            cpu = {
                "value": res["flops"] / c["t_total"] / 1e12, "unit": "TFLOP/s",
                "cores": c["threads"], "kind": "oracle",
                "sample": (f"one whole oracle divide at n = {2 * args.m} (Alg. 8 with Bunch-Kaufman "
                           f"LDL^T solves on the full matrix, alpha and beta from the definition, "
                           f"Alg. 6 bases, H_+), {c['t_total']:.1f} s on {c['threads']} BLAS "
                           f"threads of a {c['model']} ({c['physical_cores']} physical cores); "
                           f"the flop numerator is the GPU variant's nominal count"),
                "seconds": c["t_total"], "cpu_model": c["model"],
                "physical_cores": c["physical_cores"],
            }

    roof = roofline(res["kclass"], args.steps, res["ms"], traffic_from_profile)

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
        "gemm_tuning": (None if tuning_used is None else
                        {"table": tuning_used, "precision": args.tuning_table["precision"],
                         "basis": args.tuning_table["basis"]}),
        "rel_eig_err_before_refinement": rel_err.get("mixed-core-norefine"),
        "modes": {k: {"ms": v["ms"], "tflops": v["tflops"], "rel_eig_err": rel_err.get(k),
                      "phase_ms": [round(x, 4) for x in v["phase_ms"]],
                      "alpha": v["info"]["alpha"], "beta": v["info"]["beta"],
                      "restarts": v["info"]["restarts"]} for k, v in g.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
