"""Pins for the oracle's Alg. 7 with the pivoted 1x1 LDL^T (``bases.pivoted_ldl_factor``,
``bases.alg7_pivoted_bases``).

With the candidate set as large as the matrix the pivot rule is complete diagonal
pivoting, which LAPACK's pivoted Cholesky (xPSTRF, a separate implementation) computes:
pivots must agree exactly and the factor to rounding.  With a small candidate set the
factor must still reproduce a rank-k positive semidefinite matrix, each panel must start
at the global largest Schur diagonal, and the bases must be Sigma-orthonormal with the
projectors of the sign function (Lemma SignProj, Thm. DefDivConq).
"""
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from oracle import bases as bs
from oracle import divide as dv
from oracle import eig as eg
from oracle import sign as sg
from paper_2203_08900_amd import inputs


def rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


@pytest.mark.parametrize("n,keep,panel", [(40, 40, 8), (90, 60, 16), (130, 130, 64), (200, 77, 64)])
def test_complete_pivoting_is_lapack_pstrf(n, keep, panel):
    rng = np.random.default_rng(n)
    g = rng.standard_normal((n, n))
    a = g @ g.T + 0.1 * np.eye(n)
    c, piv = bs.pivoted_ldl_factor(a, keep, panel=panel, cand=n)
    lf, lp, _, info = lapack.dpstrf(a, lower=1)
    assert info == 0
    lp = lp - 1
    assert np.array_equal(piv, lp[:keep])
    lf = np.tril(lf)
    assert np.abs(c[lp] - lf[:, :keep]).max() < 1e-12 * np.abs(lf).max()


@pytest.mark.parametrize("n,k,cand", [(150, 70, 40), (256, 200, 100), (97, 97, 128)])
def test_restricted_candidates_factor_rank_k(n, k, cand):
    rng = np.random.default_rng(7 + n)
    g = rng.standard_normal((n, k)) * rng.uniform(0.1, 3.0, k)
    z = g @ g.T
    c, piv = bs.pivoted_ldl_factor(z, k, panel=32, cand=cand)
    assert len(set(piv.tolist())) == k
    assert rel(c @ c.T, z) < 1e-12
    # lower trapezoidal in pivot order: pivot j has no entries right of column j
    cp = c[piv]
    assert np.abs(np.triu(cp, 1)).max() == 0.0
    assert np.all(np.diag(cp) > 0)
    # the first pivot of every panel is the largest Schur diagonal over all free rows
    for t0 in range(0, k, 32):
        schur = np.diag(z) - np.sum(c[:, :t0] ** 2, axis=1)
        schur[piv[:t0]] = -np.inf
        assert piv[t0] == int(np.argmax(schur))


def test_non_positive_pivot_raises():
    z = np.diag([1.0, 2.0, 0.0, 0.0])
    c, piv = bs.pivoted_ldl_factor(z, 2, panel=2, cand=4)
    assert list(piv) == [1, 0]
    with pytest.raises(np.linalg.LinAlgError):
        bs.pivoted_ldl_factor(z, 3, panel=2, cand=4)


def test_casida_bases():
    a, b = inputs.small_dense(64, 0)
    m = a.shape[0]
    res = dv.divide_casida(a, b, r=8, basis="alg7-pivoted")
    s, sigma, h = res["S"], res["sigma"], res["H"]
    qp, qm = res["Q_plus"], res["Q_minus"]
    pp, pm = bs.projectors(s)
    assert np.linalg.norm(qp.T @ (sigma[:, None] * qp) - np.eye(m)) < 1e-13
    assert np.linalg.norm(qm.T @ (sigma[:, None] * qm) + np.eye(m)) < 1e-13
    assert rel(qp @ qp.T * sigma[None, :], pp) < 1e-13
    assert rel(qm @ qm.T * (-sigma[None, :]), pm) < 1e-13
    assert res["backward_error"] < 1e-13
    lam, _ = eg.eig_casida(a, b)
    w = np.linalg.eigvalsh(0.5 * (res["H_plus"] + res["H_plus"].T))
    assert np.max(np.abs(w - lam[:m]) / lam[:m]) < 1e-12


@pytest.mark.parametrize("seed", [0, 2])
def test_general_sigma_more_accurate_than_alg6(seed):
    """Sec. 6.1 matrices with kappa = 1e8: the leading blocks Alg. 6 factors can be
    ill-conditioned, the pivoted factorization picks well-conditioned pivots."""
    h, sigma = inputs.general_sigma(120, seed, 1e8)
    s, _ = sg.zolo_pd(h, sigma, r=8)
    p = int(np.sum(sigma > 0))
    qp, qm = bs.alg7_pivoted_bases(s, sigma)
    assert qp.shape[1] == p and qm.shape[1] == sigma.size - p
    e7 = np.linalg.norm(qp.T @ (sigma[:, None] * qp) - np.eye(p))
    q6, _ = bs.alg6_bases_general(s, sigma)
    e6 = np.linalg.norm(q6.T @ (sigma[:, None] * q6) - np.eye(p))
    assert e7 < 1e-13 and e7 < 1e-3 * e6
    _, _, bwd = dv.decouple(h, sigma, qp, qm)
    assert bwd < 1e-9                                   # the paper's Example 1 bound
