"""GPU parity of pseudosym_divide_general (definite pseudosymmetric H of any signature,
the random matrices of Sec. 6.1) against the oracle.

The oracle runs Alg. 8 with LDL^T solves on H itself; the GPU runs the same rational
iteration on the congruent symmetric T = R Sigma R^T.  Both converge to sign(H), so the
GPU's sign is compared with the definition, and its bases and blocks element by element
with Alg. 6 (as printed, the leading-index Cholesky factors) applied to the definition's
sign.  Alg. 6 factors the leading blocks of +-Sigma P_+-, whose condition numbers c
(up to ~1e6 for a random Sigma) bound the accuracy of the bases: the tolerances scale
with them (measured errors ~1e-17 c)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bases as bs
from oracle import divide as dv
from oracle import sign as sg
from paper_2203_08900_amd import api, inputs

pytestmark = pytest.mark.gpu


def rel(x, y):
    return np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)


CASES = [(2, 7, 10.0), (17, 1, 10.0), (60, 2, 1e2), (100, 3, 1e4), (250, 4, 10.0),
         (250, 5, 1e6), (700, 6, 1e3)]


@pytest.mark.parametrize("n,seed,kappa", CASES)
def test_general_division_parity(n, seed, kappa):
    print(f"[general] n={n} seed={seed} kappa={kappa:g}", flush=True)
    h, sig = inputs.general_sigma(n, seed, kappa)
    p = int(np.sum(sig > 0))
    q = n - p
    H = torch.tensor(h, dtype=torch.float64, device="cuda")
    Qp, Qm, Hp, Hm, S, info = api.divide_general(H, sig, want_sign=True)
    assert info["status"] == 0 and info["steps"] == 2 and info["restarts"] == 0
    # the condition estimate: cond(Sigma H) = kappa (D spans [1, kappa]), from below
    print(f"[general] cond_est {info['cond_est']:.3g}", flush=True)
    assert 0.5 * kappa <= info["cond_est"] <= kappa * (1.0 + 1e-8)
    Qp, Qm, Hp, Hm, S = (x.cpu().numpy() for x in (Qp, Qm, Hp, Hm, S))
    s_def = sg.sign_definition(h, sig)
    assert np.abs(S - s_def).max() < 1e-12 * kappa * np.abs(s_def).max()
    # the oracle's Alg. 6 on the definition's sign, and its decoupled blocks
    qp_ref, qm_ref = bs.alg6_bases_general(s_def, sig)
    hp_ref, hm_ref, _ = dv.decouple(h, sig, qp_ref, qm_ref)
    pp = 0.5 * (np.eye(n) + s_def)
    sp, sm = sig[:, None] * pp, -(sig[:, None] * (np.eye(n) - pp))
    cnd = max(np.linalg.cond(sp[:p, :p]) if p else 1.0, np.linalg.cond(sm[:q, :q]) if q else 1.0)
    tol = max(1e-15 * cnd, 1e-13) * kappa
    if p:
        assert rel(Qp, qp_ref) < tol
        assert rel(Hp, hp_ref) < tol
        assert np.abs(Qp.T @ (sig[:, None] * Qp) - np.eye(p)).max() < tol
    if q:
        assert rel(Qm, qm_ref) < tol
        assert rel(Hm, hm_ref) < tol
        assert np.abs(Qm.T @ (sig[:, None] * Qm) + np.eye(q)).max() < tol
    # eigenvalues: H_+ holds the positive ones, H_- the negative ones (nonsymmetric
    # LAPACK eigensolver on H as the reference)
    lam = np.linalg.eigvals(h).real
    scale = np.abs(lam).max()
    etol = max(1e-13 * kappa, 1e-14 * cnd) * scale
    if p:
        assert np.abs(np.sort(np.linalg.eigvalsh(0.5 * (Hp + Hp.T))) - np.sort(lam[lam > 0])).max() < etol
    if q:
        assert np.abs(np.sort(np.linalg.eigvalsh(0.5 * (Hm + Hm.T))) - np.sort(lam[lam < 0])).max() < etol
    # the paper's backward error (Sec. 6.1: below 1e-9 for all methods)
    if p and q:
        bwd = np.linalg.norm(Qp.T @ (sig[:, None] * h) @ Qm) / np.linalg.norm(h)
        print(f"[general] backward error {bwd:.2e}", flush=True)
        assert bwd < 1e-9


def test_general_one_signed():
    """Sigma = I: H = M is SPD, sign(H) = I, Q_+ = I, H_+ = H, no negative part."""
    n = 70
    hg, sg_gen = inputs.general_sigma(n, 9, 50.0)
    h = sg_gen[:, None] * hg                                 # Q D Q^T, symmetric positive definite
    h = 0.5 * (h + h.T)
    sig = np.ones(n)
    H = torch.tensor(h, dtype=torch.float64, device="cuda")
    Qp, Qm, Hp, Hm, S, info = api.divide_general(H, sig, want_sign=True)
    assert info["status"] == 0 and Qm.shape == (n, 0) and Hm.shape == (0, 0)
    assert np.abs(S.cpu().numpy() - np.eye(n)).max() < 1e-13
    assert np.abs(Qp.cpu().numpy() - np.eye(n)).max() < 1e-13
    assert rel(Hp.cpu().numpy(), h) < 1e-13


def test_general_bad_signs():
    h, sig = inputs.general_sigma(10, 1, 5.0)
    sig = sig.copy()
    sig[3] = 0.5
    H = torch.tensor(h, dtype=torch.float64, device="cuda")
    with pytest.raises(api.PseudosymError):
        api.divide_general(H, sig)
