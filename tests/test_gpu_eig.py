"""GPU parity of pseudosym_eig (all eigenpairs of H) against the oracle's definition.

The oracle diagonalizes Sigma*H and Sigma simultaneously (Thm. EVREalSigmaOrth) and
returns the eigenpairs in the canonical order and normalization: positive eigenvalues
ascending, lambda[m+i] = -lambda[i], V^T Sigma V = diag(I, -I), each column's entry of
largest modulus positive.  The GPU result comes from one structure-preserving division
(Alg. 3, Alg. 6) and the symmetric divide-and-conquer of Alg. 2 / Alg. 4 on H_+ with
Jacobi leaves; it is unique in this normalization wherever the eigenvalues are simple.

Tolerances (FP64): eigenvalues 1e-11 relative; eigenvectors of eigenvalues whose
relative gap to their neighbours exceeds 1e-4 within 1e-8 (perturbation theory bounds
the error by ~ u ||H|| / gap); for all columns the residual ||H V - V Lambda|| and
||V^T Sigma V - diag(I, -I)|| below 1e-11 relative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import eig as eg
from oracle import sign as sg
from paper_2203_08900_amd import api, inputs

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


CASES = [(1, 3, "dense"), (2, 4, "dense"), (17, 5, "dense"), (64, 0, "dense"),
         (65, 6, "dense"), (100, 1, "dense"), (150, 8, "dense"), (300, 11, "dense"),
         (420, 12, "casida")]


def make(m, seed, kind):
    return inputs.small_dense(m, seed) if kind == "dense" else inputs.casida_like(m, seed, rank=16)


def check(a, b, lam, V, info, m):
    lam_ref, v_ref = eg.eig_casida(a, b)
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(m)
    assert np.array_equal(lam[m:], -lam[:m])
    assert np.all(np.diff(lam[:m]) >= 0)
    assert np.max(np.abs(lam - lam_ref) / np.abs(lam_ref)) < 1e-11
    # invariants for every column
    sig_hat = np.concatenate([np.ones(m), -np.ones(m)])
    assert np.abs(V.T @ (sigma[:, None] * V) - np.diag(sig_hat)).max() < 1e-11
    res = np.abs(h @ V - V * lam[None, :]).max() / np.abs(h).max()
    assert res < 1e-11
    assert np.array_equal(V[:m, m:], V[m:, :m]) and np.array_equal(V[m:, m:], V[:m, :m])
    # unique columns against the definition
    lp = lam_ref[:m]
    gap = np.full(m, np.inf)
    if m > 1:
        d = np.diff(lp) / lp[1:]
        gap[1:] = np.minimum(gap[1:], d)
        gap[:-1] = np.minimum(gap[:-1], d)
    simple = np.concatenate([gap > 1e-4, gap > 1e-4])
    assert np.abs(V[:, simple] - v_ref[:, simple]).max() < 1e-8


@pytest.mark.parametrize("m,seed,kind", CASES)
def test_eig_parity(m, seed, kind):
    print(f"[eig parity] m={m} seed={seed} kind={kind}", flush=True)
    a, b = make(m, seed, kind)
    lam, V, info = api.eig(dev(a), dev(b))
    assert info["status"] == 0
    if m > 64:
        assert info["eig_splits"] >= 1 and info["eig_leaves"] >= 2
    check(a, b, lam.cpu().numpy(), V.cpu().numpy(), info, m)


def test_eig_values_only_and_commuting_blocks():
    """Eigenvalues without vectors; commuting A, B give lambda = sqrt(alpha^2 - beta^2)."""
    m = 90
    rng = np.random.default_rng(7)
    q = inputs.haar(rng, m)
    alv = rng.uniform(1.0, 4.0, m)
    bev = alv * rng.uniform(-0.9, 0.9, m)
    a = 0.5 * (((q * alv) @ q.T) + ((q * alv) @ q.T).T)
    b = 0.5 * (((q * bev) @ q.T) + ((q * bev) @ q.T).T)
    lam, V, info = api.eig(dev(a), dev(b), want_vectors=False)
    assert V is None and info["status"] == 0
    exact = np.sort(np.sqrt(alv ** 2 - bev ** 2))
    lam = lam.cpu().numpy()
    assert np.max(np.abs(lam[:m] - exact) / exact) < 1e-12
    assert np.array_equal(lam[m:], -lam[:m])


def test_eig_b_zero():
    """B = 0: H = diag(A, -A); the eigenpairs are those of A."""
    a, _ = inputs.small_dense(80, 9)
    b = np.zeros_like(a)
    lam, V, info = api.eig(dev(a), dev(b))
    w = np.linalg.eigvalsh(a)
    lam = lam.cpu().numpy()
    assert np.max(np.abs(lam[:80] - w) / w) < 1e-12
    check(a, b, lam, V.cpu().numpy(), info, 80)


@pytest.mark.timeout(600)
def test_eig_casida_m1024():
    """A larger case with several recursion levels (m = 1024, n = 2048)."""
    m = 1024
    a, b = inputs.casida_like(m, 3)
    print("[eig] m=1024", flush=True)
    lam, V, info = api.eig(dev(a), dev(b))
    assert info["status"] == 0 and info["eig_splits"] >= 15
    check(a, b, lam.cpu().numpy(), V.cpu().numpy(), info, m)


def check_clusters(a, b, lam, V, m):
    """Checks that hold with multiple eigenvalues: values against the definition,
    Sigma-orthonormality, the residual, the +-pairing, and for every group of equal
    eigenvalues the projector onto its eigenspace (unique) against the oracle's."""
    lam_ref, v_ref = eg.eig_casida(a, b)
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(m)
    assert np.array_equal(lam[m:], -lam[:m])
    assert np.all(np.diff(lam[:m]) >= 0)
    assert np.max(np.abs(lam - lam_ref) / np.abs(lam_ref)) < 1e-12
    sig_hat = np.concatenate([np.ones(m), -np.ones(m)])
    assert np.abs(V.T @ (sigma[:, None] * V) - np.diag(sig_hat)).max() < 1e-11
    assert np.abs(h @ V - V * lam[None, :]).max() / np.abs(h).max() < 1e-11
    # group the positive eigenvalues by relative gaps above 1e-8
    lp = lam_ref[:m]
    cuts = np.where(np.diff(lp) / lp[1:] > 1e-8)[0] + 1
    for grp in np.split(np.arange(m), cuts):
        proj = V[:, grp] @ (V[:, grp].T * sigma[None, :])
        pref = v_ref[:, grp] @ (v_ref[:, grp].T * sigma[None, :])
        assert np.abs(proj - pref).max() < 1e-9 * max(1.0, np.abs(pref).max())


@pytest.mark.parametrize("m,a0,b0", [(100, 3.0, 1.0), (300, 2.5, -0.7), (90, 4.0, 0.0)])
def test_eig_multiple_of_identity(m, a0, b0):
    """A = aI, B = bI: all m positive eigenvalues equal sqrt(a^2 - b^2), so no shift can
    split a block of the recursion; such blocks are recognized as lambda I and halved as
    they are (Thm. EVREalSigmaOrth: any Sigma-orthonormal basis of the eigenspace is an
    eigenbasis)."""
    print(f"[eig cluster] m={m} a={a0} b={b0}", flush=True)
    a = a0 * np.eye(m)
    b = b0 * np.eye(m)
    lam, V, info = api.eig(dev(a), dev(b))
    assert info["status"] == 0
    assert info["eig_clusters"] >= 1
    lam = lam.cpu().numpy()
    exact = np.sqrt(a0 * a0 - b0 * b0)
    assert np.abs(lam[:m] - exact).max() < 1e-13 * exact
    check_clusters(a, b, lam, V.cpu().numpy(), m)


def test_eig_cluster_inside_spread_spectrum():
    """A 100-fold eigenvalue in the middle of a spectrum spread over two decades: the
    median shifts land on or near it; nudged shifts split the others off and the
    cluster block is then recognized as lambda I."""
    m = 260
    rng = np.random.default_rng(31)
    qm = inputs.haar(rng, m)
    dm = rng.uniform(1.0, 2.0, m)
    mu = 10.0 ** rng.uniform(-1.0, 1.0, m)
    mu[:100] = 1.0                                   # eig((A-B)(A+B)) = mu: 100-fold 1
    q = inputs.haar(rng, m)
    mih = (qm * dm[None, :] ** -0.5) @ qm.T
    k = mih @ ((q * mu[None, :]) @ q.T) @ mih
    mm = (qm * dm[None, :]) @ qm.T
    a = 0.5 * (mm + k)
    b = 0.5 * (mm - k)
    a, b = 0.5 * (a + a.T), 0.5 * (b + b.T)
    print("[eig cluster] m=260 with a 100-fold eigenvalue", flush=True)
    lam, V, info = api.eig(dev(a), dev(b))
    assert info["status"] == 0
    lam = lam.cpu().numpy()
    assert np.sum(np.abs(lam[:m] - 1.0) < 1e-12) == 100
    check_clusters(a, b, lam, V.cpu().numpy(), m)
