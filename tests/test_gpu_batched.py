"""Batched division of independent problems of uneven sizes (pseudosym_divide_batched).

A problem alone in its padded size runs the single-problem pipeline on one of the
handle's worker streams, so its result must equal, bit for bit, the one
pseudosym_divide returns for it; problems that share a padded size run as one batched
pipeline and agree with single calls to rounding.  A sample is also checked against
the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import divide as dv
from oracle import sign as sg
from paper_2203_08900_amd import api, inputs

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def test_batched_matches_single_and_oracle():
    sizes = [17, 300, 64, 1, 130, 65, 200, 33, 250, 96, 7, 180]
    probs = [inputs.small_dense(mi, 100 + i) for i, mi in enumerate(sizes)]
    As = [dev(a) for a, _ in probs]
    Bs = [dev(b) for _, b in probs]
    print(f"[batched] sizes {sizes}", flush=True)
    Qs, Hs, infos = api.divide_batched(As, Bs)
    assert all(inf["status"] == 0 for inf in infos)
    padded = [(mi + 63) // 64 for mi in sizes]
    for i, (A, B) in enumerate(zip(As, Bs)):
        Q1, H1, _ = api.divide(A, B)
        if padded.count(padded[i]) == 1:     # alone in its size: the single pipeline
            assert torch.equal(Q1, Qs[i]) and torch.equal(H1, Hs[i])
        else:                                # a class: the same results to rounding
            w1 = np.linalg.eigvalsh(0.5 * (H1 + H1.T).cpu().numpy())
            w2 = np.linalg.eigvalsh(0.5 * (Hs[i] + Hs[i].T).cpu().numpy())
            assert np.max(np.abs(w1 - w2) / w1) < 1e-12
    for i in (0, 1, 4):
        a, b = probs[i]
        m = sizes[i]
        amax, amin = sg.abs_eig_bounds(sg.casida_matrix(a, b), sg.casida_sigma(m))
        ref = dv.divide_casida(a, b, alpha=1.01 * amax, beta=0.99 * amin)
        w = np.linalg.eigvalsh(0.5 * (Hs[i] + Hs[i].T).cpu().numpy())
        lam = np.sort(np.linalg.eigvalsh(0.5 * (ref["H_plus"] + ref["H_plus"].T)))
        assert np.max(np.abs(w - lam) / lam) < 1e-12


def test_batched_mixed_and_empty():
    assert api.divide_batched([], []) == ([], [], [])
    sizes = [40, 120, 260]
    probs = [inputs.small_dense(mi, 7 + i) for i, mi in enumerate(sizes)]
    Qs, Hs, infos = api.divide_batched([dev(a) for a, _ in probs], [dev(b) for _, b in probs],
                                       precision="mixed")
    for (a, b), H, inf, m in zip(probs, Hs, infos, sizes):
        assert inf["status"] == 0
        # below the padded size 1024 a mixed request runs every shift in FP64 (the FP32
        # group's extra launches cost more than they save there): FP64 accuracy
        assert inf["shifts_fp64"][0] == inf["r"]
        lam = np.sqrt(np.linalg.eigvals((a - b) @ (a + b)).real)
        w = np.linalg.eigvalsh(0.5 * (H + H.T).cpu().numpy())
        assert np.max(np.abs(np.sort(w) - np.sort(lam)) / np.sort(lam)) < 1e-12


def test_batched_bad_arguments():
    a, b = inputs.small_dense(8, 1)
    with pytest.raises(api.PseudosymError):
        api.divide_batched([dev(a)], [dev(b)], r=9)


@pytest.mark.parametrize("basis", ["core", "alg6"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_classes_match_single(precision, basis):
    """Problems of one padded size run as one batched pipeline (per-problem bounds,
    coefficients and shifts in device arrays), with either basis.  The arithmetic per
    problem is the single path's with sums split differently, so the results agree with
    single calls to rounding: same eigenvalues of H_+ to 1e-12, Sigma-orthonormal Q_+,
    and the same subspace (P_+ = Q_+ Q_+^T Sigma)."""
    sizes = [40, 50, 60, 33, 130, 140, 150, 129, 7, 300, 310, 290, 64, 1, 2, 3]
    probs = [inputs.small_dense(mi, 300 + i) for i, mi in enumerate(sizes)]
    As = [dev(a) for a, _ in probs]
    Bs = [dev(b) for _, b in probs]
    print(f"[classes] {precision} {basis} sizes {sizes}", flush=True)
    Qs, Hs, infos = api.divide_batched(As, Bs, precision=precision, basis=basis)
    assert all(inf["status"] == 0 for inf in infos)
    for i, (A, B) in enumerate(zip(As, Bs)):
        m = sizes[i]
        Q1, H1, _ = api.divide(A, B, precision=precision, basis=basis)
        sig = torch.cat([torch.ones(m, dtype=torch.float64, device="cuda"),
                         -torch.ones(m, dtype=torch.float64, device="cuda")])
        G = Qs[i].T @ (sig[:, None] * Qs[i])
        assert (G - torch.eye(m, dtype=torch.float64, device="cuda")).abs().max().item() < 1e-12
        P1 = Q1 @ Q1.T * sig[None, :]
        P2 = Qs[i] @ Qs[i].T * sig[None, :]
        assert (P1 - P2).abs().max().item() < 1e-11
        w1 = np.linalg.eigvalsh(0.5 * (H1 + H1.T).cpu().numpy())
        w2 = np.linalg.eigvalsh(0.5 * (Hs[i] + Hs[i].T).cpu().numpy())
        assert np.max(np.abs(w1 - w2) / w1) < 1e-12
    for i in (0, 4, 9):
        a, b = probs[i]
        lam = np.sort(np.sqrt(np.linalg.eigvals((a - b) @ (a + b)).real))
        w = np.sort(np.linalg.eigvalsh(0.5 * (Hs[i] + Hs[i].T).cpu().numpy()))
        assert np.max(np.abs(w - lam) / lam) < 1e-11


@pytest.mark.parametrize("basis", ["core", "alg6"])
def test_batched_graph_replays_match_direct_launches(basis):
    """Classes captured as HIP graphs: the first call captures and launches, later calls
    replay; every replay, with other device work and synchronizations in between, must
    equal the direct launches bit for bit (the same kernels in the same order)."""
    sizes = [70, 100, 127, 65, 200, 240, 256, 33, 40]   # classes of padded 128 and 256
    probs = [inputs.small_dense(mi, 300 + i) for i, mi in enumerate(sizes)]
    As = [dev(a) for a, _ in probs]
    Bs = [dev(b) for _, b in probs]
    print(f"[batched graphs] {basis} sizes {sizes}", flush=True)
    api.set_graphs(False)
    Q0, H0, i0 = api.divide_batched(As, Bs, basis=basis)
    assert all(inf["status"] == 0 for inf in i0)
    api.set_graphs(True)
    try:
        for rep in range(4):
            Qs, Hs, infos = api.divide_batched(As, Bs, basis=basis)
            assert all(inf["status"] == 0 for inf in infos)
            for q0, q1, h0, h1 in zip(Q0, Qs, H0, Hs):
                assert torch.equal(q0, q1) and torch.equal(h0, h1), rep
            x = torch.randn(512, 512, dtype=torch.float64, device="cuda")
            (x @ x).sum().item()                      # eager work between the replays
            torch.cuda.synchronize()
    finally:
        api.set_graphs(True)


def test_batched_timing_reports_each_class_once():
    """timing == 2 on a batched call: the class pipelines run without graphs and report
    their kernel classes in one record each (their first completed problem), problems
    alone in their size report their own; the results equal the untimed call's bit for
    bit (the same kernels in the same order)."""
    sizes = [70, 100, 127, 65, 200, 240, 256, 33, 300]   # classes of 128 and 256, 300 alone
    probs = [inputs.small_dense(mi, 400 + i) for i, mi in enumerate(sizes)]
    As = [dev(a) for a, _ in probs]
    Bs = [dev(b) for _, b in probs]
    print(f"[batched timing] sizes {sizes}", flush=True)
    Q0, H0, _ = api.divide_batched(As, Bs, basis="core")
    Q1, H1, infos = api.divide_batched(As, Bs, basis="core", timing=2)
    assert all(inf["status"] == 0 for inf in infos)
    for q0, q1, h0, h1 in zip(Q0, Q1, H0, H1):
        assert torch.equal(q0, q1) and torch.equal(h0, h1)
    timed = [i for i, inf in enumerate(infos) if sum(inf["kclass_launches"]) > 0]
    padded = [(mi + 63) // 64 for mi in sizes]
    classes = {p for p in padded if padded.count(p) > 1}
    alone = [i for i, p in enumerate(padded) if padded.count(p) == 1]
    # one record per class plus every problem that ran alone
    assert len(timed) == len(classes) + len(alone)
    assert set(alone) <= set(timed)
    assert sorted({padded[i] for i in timed if i not in alone}) == sorted(classes)
    for i in timed:
        inf = infos[i]
        assert all(ms >= 0.0 for ms in inf["kclass_ms"])
        assert sum(inf["kclass_flops"]) > 0.0
