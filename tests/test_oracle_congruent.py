"""Pins for the oracle's bases from the projectors of the congruent symmetric T
(``bases.congruent_bases_general``), for a definite pseudosymmetric H of any signature.

Checked against what does not depend on the construction: the spectral projectors of H
from its eigendecomposition (Lemma SignProj), invariance H Q_+- = Q_+- H_+- and
Sigma-orthonormality (Thm. DefDivConq), the eigenvalues from LAPACK's nonsymmetric
solver (Thm. EVREalSigmaOrth: r_+ positive, r_- negative), and the closed form at
Sigma = +-I (with sign(T) = +-I the pivots are 0, 1, ... and Q is upper triangular and
orthogonal with a positive diagonal, hence the identity).  At cond(Sigma H) = 1e12 the
backward error stays at rounding level where Alg. 6 on sign(H) loses cond(M) u.
"""
import numpy as np
import pytest

from oracle import bases as bs
from oracle import divide as dv
from oracle import sign as sg
from paper_2203_08900_amd import inputs


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_one_signed_closed_form(sign):
    n = 40
    rng = np.random.default_rng(3)
    x = rng.standard_normal((n, n))
    m = x @ x.T + n * np.eye(n)
    sigma = np.full(n, sign)
    h = sigma[:, None] * m
    qp, qm, hp, hm = bs.congruent_bases_general(h, sigma, u=sign * np.eye(n))
    q, hq = (qp, hp) if sign > 0 else (qm, hm)
    assert (qp.shape[1], qm.shape[1]) == ((n, 0) if sign > 0 else (0, n))
    assert np.abs(q - np.eye(n)).max() < 1e-13
    assert np.abs(hq - h).max() < 1e-12 * np.abs(h).max()


@pytest.mark.parametrize("n,seed,kappa", [(2, 1, 10.0), (31, 2, 1e3), (120, 3, 1e5)])
def test_projectors_invariance_and_eigenvalues(n, seed, kappa):
    h, sigma = inputs.general_sigma(n, seed, kappa)
    p = int(np.sum(sigma > 0))
    q = n - p
    qp, qm, hp, hm = bs.congruent_bases_general(h, sigma)
    assert qp.shape == (n, p) and qm.shape == (n, q)
    s_def = sg.sign_definition(h, sigma)            # from the eigendecomposition of H
    pp = 0.5 * (np.eye(n) + s_def)
    tol = 1e-14 * kappa
    sq = lambda x: sigma[:, None] * x
    if p:
        assert np.abs(qp @ sq(qp).T - pp).max() < tol * max(1.0, np.abs(pp).max())
        assert np.abs(qp.T @ sq(qp) - np.eye(p)).max() < tol
        assert np.abs(h @ qp - qp @ hp).max() < tol * np.abs(h).max() * np.abs(qp).max()
    if q:
        assert np.abs(-(qm @ sq(qm).T) - (np.eye(n) - pp)).max() < tol * max(1.0, np.abs(pp).max())
        assert np.abs(qm.T @ sq(qm) + np.eye(q)).max() < tol
        assert np.abs(h @ qm - qm @ hm).max() < tol * np.abs(h).max() * np.abs(qm).max()
    if p and q:
        assert np.abs(qp.T @ sq(qm)).max() < tol
    lam = np.sort(np.linalg.eigvals(h).real)
    scale = np.abs(lam).max()
    if p:
        assert np.abs(np.sort(np.linalg.eigvalsh(hp)) - lam[lam > 0]).max() < tol * scale
    if q:
        assert np.abs(np.sort(np.linalg.eigvalsh(hm)) - lam[lam < 0]).max() < tol * scale


def test_given_sign_matches_iteration():
    h, sigma = inputs.general_sigma(80, 5, 1e4)
    m = sigma[:, None] * h
    r = np.linalg.cholesky(0.5 * (m + m.T)).T
    t = (r * sigma[None, :]) @ r.T
    w, v = np.linalg.eigh(0.5 * (t + t.T))
    u = (v * np.sign(w)) @ v.T
    a = bs.congruent_bases_general(h, sigma)
    b = bs.congruent_bases_general(h, sigma, u=u)
    for x, y in zip(a, b):
        assert np.linalg.norm(x - y) <= 1e-11 * np.linalg.norm(y)


@pytest.mark.parametrize("seed", [11, 12])
def test_accurate_where_alg6_is_not(seed):
    h, sigma = inputs.general_sigma(150, seed, 1e12)
    qp, qm, hp, hm = bs.congruent_bases_general(h, sigma)
    hp2, hm2, bwd = dv.decouple(h, sigma, qp, qm)
    assert bwd < 1e-13
    assert np.abs(hp - hp2).max() < 1e-12 * np.abs(hp2).max()
    assert np.abs(hm - hm2).max() < 1e-12 * np.abs(hm2).max()
    p, q = qp.shape[1], qm.shape[1]
    assert np.abs(qp.T @ (sigma[:, None] * qp) - np.eye(p)).max() < 1e-11
    assert np.abs(qm.T @ (sigma[:, None] * qm) + np.eye(q)).max() < 1e-11
    # Alg. 6 on sign(H) from the eigendecomposition of the pencil
    op, om = bs.alg6_bases_general(sg.sign_definition(h, sigma), sigma)
    assert dv.decouple(h, sigma, op, om)[2] > 1e3 * bwd


def test_divide_general_congruent_option():
    h, sigma = inputs.general_sigma(90, 13, 1e6)
    res = dv.divide_general(h, sigma, basis="congruent")
    qp, qm, _, _ = bs.congruent_bases_general(h, sigma)
    assert np.abs(res["Q_plus"] - qp).max() == 0.0 and np.abs(res["Q_minus"] - qm).max() == 0.0
    assert res["backward_error"] < 1e-14
