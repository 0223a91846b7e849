"""The comparison iterations of Tab:ItRuntime on the GPU (ps_opts.iteration): Sigma-DWH
(the step of Alg. 8 with r = 1) and the scaled Newton iteration with the Byers-Xu scaling.
Each runs the oracle's step schedule (same l = beta/alpha: the same number of steps) and
reaches sign(H) by its definition; for the Casida form and for any signature."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import iterations as it
from oracle import sign as sg
from paper_2203_08900_amd import api, inputs

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("which", ["dwh", "newton"])
@pytest.mark.parametrize("m,seed,kind", [(64, 0, "dense"), (200, 3, "dense"), (300, 11, "casida")])
def test_comparison_iteration_casida(which, m, seed, kind):
    print(f"[iterations] {which} m={m}", flush=True)
    a, b = inputs.small_dense(m, seed) if kind == "dense" else inputs.casida_like(m, seed, rank=16)
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(m)
    amax, amin = sg.abs_eig_bounds(h, sigma)
    al, be = 1.01 * amax, 0.99 * amin
    SA, SB, info = api.sign(dev(a), dev(b), alpha=al, beta=be, iteration=which)
    assert info["status"] == 0 and info["r"] == 1
    sched = it.dwh_schedule(be / al) if which == "dwh" else it.newton_schedule(be / al)
    assert info["steps"] == len(sched)
    s = sg.sign_definition(h, sigma)
    scale = np.abs(s).max()
    assert np.abs(SA.cpu().numpy() - s[:m, :m]).max() < 1e-12 * scale
    assert np.abs(SB.cpu().numpy() - s[:m, m:]).max() < 1e-12 * scale
    # the whole division also runs on these iterations
    Qp, Hp, inf2 = api.divide(dev(a), dev(b), iteration=which, basis="core")
    w = np.linalg.eigvalsh(0.5 * (Hp + Hp.T).cpu().numpy())
    lam = np.sort(np.abs(np.linalg.eigvals(h).real))[::2]
    assert inf2["status"] == 0 and np.max(np.abs(np.sort(w) - lam) / lam) < 1e-11


@pytest.mark.parametrize("which", ["dwh", "newton"])
def test_comparison_iteration_general_signature(which):
    n = 150
    h, sig = inputs.general_sigma(n, 21, 1e2)
    H = dev(h)
    Qp, Qm, Hp, Hm, S, info = api.divide_general(H, sig, want_sign=True, iteration=which)
    assert info["status"] == 0
    ell = info["beta"] / info["alpha"]
    sched = it.dwh_schedule(ell) if which == "dwh" else it.newton_schedule(ell)
    assert info["steps"] == len(sched)
    s = sg.sign_definition(h, sig)
    assert np.abs(S.cpu().numpy() - s).max() < 1e-10 * np.abs(s).max()


def test_comparison_iteration_rejects_mixed():
    a, b = inputs.small_dense(20, 1)
    with pytest.raises(api.PseudosymError):
        api.sign(dev(a), dev(b), iteration="dwh", precision="mixed")
