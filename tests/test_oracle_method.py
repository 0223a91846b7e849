"""Pins for the oracle's sign iteration, bases, decoupling and eigen-decomposition.

Each check ties the oracle to something it does not compute itself: closed forms
for commuting blocks, invariants the paper proves (Lemma SignProj, Thm.
EVREalSigmaOrth, Thm. DefDivConq, Lemma IterOnSelfAdj), multiprecision brute
force on tiny inputs, a second LAPACK route, and the numbers of Sec. 6.
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import bases as bs
from oracle import divide as dv
from oracle import eig as eg
from oracle import sign as sg
from oracle import zolotarev as zol
from paper_2203_08900_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def pi_swap(m):
    z = np.zeros((m, m))
    return np.block([[z, np.eye(m)], [np.eye(m), z]])


def rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


@pytest.fixture(scope="module")
def small():
    a, b = inputs.small_dense(64, 0)
    return a, b, dv.divide_casida(a, b, r=8, keep_iterates=True)


# ----------------------------------------------------------------------------- LDL^T solve
def test_ldl_solve_matches_dense_solve():
    rng = np.random.default_rng(7)
    n = 40
    g = rng.standard_normal((n, n))
    z = g + g.T + np.diag(np.where(np.arange(n) % 2 == 0, 1.0, -1.0))   # symmetric indefinite
    rhs = rng.standard_normal((n, 5))
    lu, d, perm = sla.ldl(z, lower=True)
    y = sg.ldl_solve(lu, d, perm, rhs)
    assert rel(y, np.linalg.solve(z, rhs)) < 1e-11


# ----------------------------------------------------------------------------- closed forms
@pytest.mark.parametrize("m", [1, 3, 17])
def test_commuting_blocks_closed_form(m):
    """A, B with a common eigenbasis: H splits into 2x2 blocks [[a, b], [-b, -a]] whose
    square is (a^2 - b^2) I, so sign(H) = [[A, B], [-B, -A]] with a_i, b_i divided by
    lambda_i = sqrt(a_i^2 - b_i^2)."""
    rng = np.random.default_rng(m)
    q = inputs.haar(rng, m)
    al = rng.uniform(1.0, 4.0, m)
    be = al * rng.uniform(-0.9, 0.9, m)
    a = (q * al) @ q.T
    b = (q * be) @ q.T
    lam = np.sqrt(al ** 2 - be ** 2)
    s_ref = sg.casida_matrix((q * (al / lam)) @ q.T, (q * (be / lam)) @ q.T)
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(m)
    s, rec = sg.zolo_pd(h, sigma, r=8)
    assert rel(s, s_ref) < 1e-13
    assert rec.restarts == 0
    lam_o, _ = eg.eig_casida(a, b)
    assert np.allclose(lam_o[:m], np.sort(lam), rtol=1e-13)
    assert np.allclose(lam_o[m:], -np.sort(lam), rtol=1e-13)


def test_b_zero_special_case():
    a, _ = inputs.small_dense(12, 3)
    b = np.zeros_like(a)
    m = 12
    res = dv.divide_casida(a, b)
    assert rel(res["S"], np.diag(sg.casida_sigma(m))) < 1e-13
    qp = res["Q_plus"]
    assert np.abs(qp[:m] - np.eye(m)).max() < 1e-13 and np.abs(qp[m:]).max() < 1e-13
    assert rel(res["H_plus"], a) < 1e-13


# ----------------------------------------------------------------------------- Alg. 8
def test_paper_iteration_matches_definition(small):
    a, b, res = small
    h, sigma, s = res["H"], res["sigma"], res["S"]
    assert rel(s, sg.sign_definition(h, sigma)) < 1e-13
    assert rel(sg.sign_definition(h, sigma), sg.sign_definition_geev(h)) < 1e-12
    rec = res["record"]
    assert rec.restarts == 0 and len(rec.changes) == 1
    assert rec.changes[0] <= GOLDEN["stopping_rule"]["u"] ** (1.0 / 17)


def test_sign_invariants(small):
    a, b, res = small
    m = a.shape[0]
    h, s = res["H"], res["S"]
    eye = np.eye(2 * m)
    j = np.diag(sg.casida_sigma(m))
    assert np.linalg.norm(s @ s - eye) / np.sqrt(2 * m) < 1e-13              # S^2 = I
    assert np.linalg.norm(j @ s - (j @ s).T) / np.linalg.norm(s) < 1e-13     # J S = S^T J
    assert np.linalg.norm(h @ s - s @ h) / np.linalg.norm(h) < 1e-13
    p = pi_swap(m)
    assert np.linalg.norm(p @ s @ p + s) / np.linalg.norm(s) < 1e-13         # Pi S Pi = -S
    assert abs(np.trace(s)) < 1e-11                                          # p = m positive


def test_iterates_act_on_eigenvalues(small):
    """Lemma IterOnSelfAdj: X_1 = g(H / alpha) with g = hat Z, so the eigenvalues of X_1
    are sign(lambda) hat Z(|lambda| / alpha; l)."""
    a, b, res = small
    rec = res["record"]
    x1 = rec.iterates[0]
    lam, _ = eg.eig_casida(a, b)
    co = rec.coeffs[0]
    pred = np.array([np.sign(v) * float(zol.zhat(abs(v) / rec.alpha, co)) for v in lam])
    got = np.sort(np.linalg.eigvals(x1).real)
    assert np.max(np.abs(np.sort(pred) - got)) < 1e-13


def test_third_step_is_stationary(small):
    a, b, res = small
    rec = res["record"]
    co3 = zol.coefficients(min(rec.coeffs[1].ell_next, 1 - 1e-15), 8)
    x3 = sg.ldl_zolo_step(res["S"], res["sigma"], co3)
    assert rel(x3, res["S"]) < 1e-14


def test_restart_path_fires_and_converges():
    """Overestimating beta (l too large) leaves small eigenvalues outside [l, 1]; the
    stopping test of Alg. 8 then restarts from X2 and the result is still sign(H)."""
    a, b = inputs.small_dense(24, 5)
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(24)
    amax, amin = sg.abs_eig_bounds(h, sigma)
    assert amin < 0.25 * amax
    s, rec = sg.zolo_pd(h, sigma, r=2, alpha=amax, beta=0.9 * amax)
    assert rec.restarts >= 1
    assert rel(s, sg.sign_definition(h, sigma)) < 1e-12


# ----------------------------------------------------------------------------- bases
def test_alg6_bases(small):
    a, b, res = small
    m = a.shape[0]
    s, sigma = res["S"], res["sigma"]
    qp, qm = res["Q_plus"], res["Q_minus"]
    pp, pm = bs.projectors(s)
    assert np.linalg.norm(qp.T @ (sigma[:, None] * qp) - np.eye(m)) < 1e-12
    # Q_- pivots on the leading block of -Sigma P_- = (A_s - I)/2, which is nearly
    # singular when B is small against A: Alg. 6 loses accuracy there (Sec. 6.2 reports
    # such losses for the Cholesky bases), so its Sigma-orthonormality is looser
    assert np.linalg.norm(qm.T @ (sigma[:, None] * qm) + np.eye(m)) < 1e-9
    assert rel(pp @ qp, qp) < 1e-13 and rel(pm @ qm, qm) < 1e-12
    assert rel(qp @ qp.T * sigma[None, :], pp) < 1e-13                         # P_+ = Q Q^T Sigma
    top = qp[:m]
    assert np.abs(np.triu(top, 1)).max() == 0.0 and np.all(np.diag(top) > 0)   # canonical form
    # Q_- spans range(Pi Q_+) (F3 of the Casida structure)
    piqp = pi_swap(m) @ qp
    assert rel(pm @ piqp, piqp) < 1e-13


def test_alg6_printed_q_minus_leaves_the_subspace(small):
    a, b, res = small
    m = a.shape[0]
    _, qm_printed = bs.alg6_cholesky_bases_as_printed(res["S"], m)
    _, pm = bs.projectors(res["S"])
    assert rel(pm @ qm_printed, qm_printed) > 1e-3


def test_alg7_bases_and_decoupling(small):
    a, b, res = small
    m = a.shape[0]
    s, sigma, h = res["S"], res["sigma"], res["H"]
    qp, qm = bs.alg7_ldl_bases(s, sigma)
    pp, pm = bs.projectors(s)
    assert np.linalg.norm(qp.T @ (sigma[:, None] * qp) - np.eye(m)) < 1e-12
    assert np.linalg.norm(qm.T @ (sigma[:, None] * qm) + np.eye(m)) < 1e-12
    assert rel(qp @ qp.T * sigma[None, :], pp) < 1e-13
    hp, hm, bwd = dv.decouple(h, sigma, qp, qm)
    assert bwd < 1e-13
    lam, _ = eg.eig_casida(a, b)
    assert np.max(np.abs(np.linalg.eigvalsh(hp) - lam[:m]) / lam[:m]) < 1e-12


def test_decoupled_blocks(small):
    a, b, res = small
    m = a.shape[0]
    hp, hm = res["H_plus"], res["H_minus"]
    assert np.linalg.norm(hp - hp.T) < 1e-13 * np.linalg.norm(hp)
    w = np.linalg.eigvalsh(0.5 * (hp + hp.T))
    assert w.min() > 0                                                       # Thm. DefDivConq
    assert np.linalg.eigvalsh(0.5 * (hm + hm.T)).max() < 0
    lam, _ = eg.eig_casida(a, b)
    assert np.max(np.abs(w - lam[:m]) / lam[:m]) < 1e-12
    assert res["backward_error"] < 1e-13


def test_alg4_orthogonal_bases():
    rng = np.random.default_rng(11)
    n = 30
    q = inputs.haar(rng, n)
    d = np.concatenate([rng.uniform(0.5, 2, 12), -rng.uniform(0.5, 2, 18)])
    a = (q * d) @ q.T
    s = sg.zolo_pd_symmetric(a)
    qp, qm = bs.alg4_orthogonal_bases(s)
    assert qp.shape[1] == 12 and qm.shape[1] == 18
    v = np.hstack([qp, qm])
    assert np.linalg.norm(v.T @ v - np.eye(n)) < 1e-12
    blk = v.T @ a @ v
    assert np.linalg.norm(blk[:12, 12:]) < 1e-12


# ----------------------------------------------------------------------------- eigen-decomposition
def test_eigenvalues_pairs_and_squares(small):
    a, b, _ = small
    m = a.shape[0]
    lam, v = eg.eig_casida(a, b)
    assert np.all(lam[:m] > 0) and np.all(lam[m:] < 0)
    assert np.max(np.abs(lam[m:] + lam[:m]) / lam[:m]) < 1e-13
    km = np.sort(np.linalg.eigvals((a - b) @ (a + b)).real)
    assert np.max(np.abs(lam[:m] ** 2 - km) / km) < 1e-12
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(m)
    assert np.linalg.norm(h @ v - v * lam[None, :]) / np.linalg.norm(h) < 1e-13
    vsv = v.T @ (sigma[:, None] * v)
    assert np.linalg.norm(vsv - np.diag(np.concatenate([np.ones(m), -np.ones(m)]))) < 1e-12
    assert np.abs(v[:, m:] - pi_swap(m) @ v[:, :m]).max() < 1e-12      # V_- = Pi V_+


def test_eigenvalues_brute_force_multiprecision():
    a, b = inputs.small_dense(5, 21)
    h = sg.casida_matrix(a, b)
    with mp.workdps(40):
        ev = mp.eig(mp.matrix(h.tolist()), left=False, right=False)
        ref = sorted([float(mp.re(x)) for x in ev])
    lam, _ = eg.eig_casida(a, b)
    ref = np.array(ref)
    pos = np.sort(ref[ref > 0])
    neg = np.sort(ref[ref < 0])[::-1]
    assert np.max(np.abs(np.concatenate([pos, neg]) - lam) / np.abs(lam)) < 1e-13


def test_alg2_recursion_reaches_definition(small):
    a, b, res = small
    hp = 0.5 * (res["H_plus"] + res["H_plus"].T)
    w, v = eg.alg2_symmetric_dc(hp)
    ref = np.linalg.eigvalsh(hp)
    assert np.max(np.abs(w - ref) / ref) < 1e-10
    assert np.linalg.norm(v.T @ v - np.eye(hp.shape[0])) < 1e-10


# ----------------------------------------------------------------------------- Sec. 6 numbers
def _example1_matrix(n, kappa, seed):
    """Example 1 generator: A = Sigma Q D Q^T, Sigma random +-1, D = linspace(1, kappa)."""
    rng = np.random.default_rng(seed)
    sigma = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    q = inputs.haar(rng, n)
    d = np.linspace(1.0, kappa, n)
    return sigma[:, None] * ((q * d) @ q.T), sigma


@pytest.mark.parametrize("kappa", [10.0, 1e4])
def test_example1_backward_error_bound(kappa):
    n = 120
    h, sigma = _example1_matrix(n, kappa, 0)
    s, rec = sg.zolo_pd(h, sigma, r=8)
    qp, qm = bs.alg7_ldl_bases(s, sigma)
    _, _, bwd = dv.decouple(h, sigma, qp, qm)
    assert bwd < GOLDEN["example1_backward_error_bound"]["bound"]
    if kappa == 10.0:
        assert bwd < 100 * GOLDEN["example1_backward_error_bound"]["zolo_avg_kappa10"]
    assert int(np.sum(sigma > 0)) == qp.shape[1]          # p positive eigenvalues


@pytest.mark.parametrize("m,seed,mu_lo", [(5, 1, 1e-2), (60, 3, 1e-3), (150, 8, 1e-6)])
def test_sign_definition_against_construction(m, seed, mu_lo):
    """The ill-separated construction fixes sign(H) in closed form (products of its own
    spectral factors, no eigensolver); the definition through the definite pencil must
    reproduce it, and the column form must equal the full one."""
    a, b, _, fac = inputs.ill_separated(m, seed, mu_lo=mu_lo, return_factors=True)
    As, Bs = sg.sign_blocks_from_spectral_factors(*fac)
    s = sg.sign_definition(sg.casida_matrix(a, b), sg.casida_sigma(m))
    scale = np.abs(s).max()
    # rounding of A, B (~1e-16 relative) moves sign(H) by about that over the squared
    # spectral gap, min|lambda|^2 = mu_lo (measured: 2.4e-13 at 1e-4, 2.4e-11 at 1e-6)
    tol = 1e-16 / mu_lo
    for blk, ref in ((s[:m, :m], As), (s[:m, m:], Bs), (s[m:, :m], -Bs), (s[m:, m:], -As)):
        assert np.abs(blk - ref).max() < tol * scale
    cols = [0, m // 2, m - 1]
    ca, cb = sg.sign_columns_from_spectral_factors(*fac, cols)
    assert np.abs(ca - As[:, cols]).max() < 1e-13 * scale
    assert np.abs(cb - Bs[:, cols]).max() < 1e-13 * scale


@pytest.mark.parametrize("n,seed,kappa", [(60, 1, 10.0), (120, 3, 1e4), (97, 5, 1e2)])
def test_general_sigma_division(n, seed, kappa):
    """Any signature (Sec. 6.1 matrices): Alg. 8 on H reaches the definition of sign(H);
    rank P_+ = number of +1 in Sigma (Thm. EVREalSigmaOrth); the Alg. 6 bases are
    (Sigma, +-I)-orthonormal and invariant; H_+ holds the positive eigenvalues of H and
    H_- the negative ones (a second LAPACK route, the nonsymmetric eigensolver); the
    backward error stays below the paper's 1e-9 (Fig. BackErr_all)."""
    h, sig = inputs.general_sigma(n, seed, kappa)
    ref = dv.divide_general(h, sig)
    s = ref["S"]
    p = int(np.sum(sig > 0))
    assert np.abs(s - sg.sign_definition(h, sig)).max() < 1e-12 * kappa * np.abs(s).max()
    assert int(round(np.trace(0.5 * (np.eye(n) + s)))) == p
    qp, qm = ref["Q_plus"], ref["Q_minus"]
    assert qp.shape == (n, p) and qm.shape == (n, n - p)
    # Alg. 6 factors the leading blocks of +-Sigma P_+-, whose condition numbers (up to
    # ~1e6 here for a random Sigma) bound the accuracy of the bases (measured ~1e-17 cond)
    pp = 0.5 * (np.eye(n) + s)
    sp, sm = sig[:, None] * pp, -(sig[:, None] * (np.eye(n) - pp))
    cnd = max(np.linalg.cond(sp[:p, :p]), np.linalg.cond(sm[:n - p, :n - p]))
    tol = 1e-15 * max(cnd, kappa)
    assert np.abs(qp.T @ (sig[:, None] * qp) - np.eye(p)).max() < tol
    assert np.abs(qm.T @ (sig[:, None] * qm) + np.eye(n - p)).max() < tol
    assert np.abs(pp @ qp - qp).max() < tol and np.abs(pp @ qm).max() < tol
    lam = np.linalg.eigvals(h).real
    wp = np.linalg.eigvalsh(0.5 * (ref["H_plus"] + ref["H_plus"].T))
    wm = np.linalg.eigvalsh(0.5 * (ref["H_minus"] + ref["H_minus"].T))
    scale = np.abs(lam).max()
    # H_+- inherit the bases' departure from Sigma-orthonormality (above)
    etol = max(1e-13 * kappa, 1e-14 * cnd) * scale
    assert np.abs(np.sort(wp) - np.sort(lam[lam > 0])).max() < etol
    assert np.abs(np.sort(wm) - np.sort(lam[lam < 0])).max() < etol
    assert ref["backward_error"] < 1e-9
    assert len(ref["record"].changes) == 1          # two Zolotarev steps, no restart


def test_general_bases_reduce_to_casida_case():
    """With Sigma = diag(I_m, -I_m) the general Alg. 6 is the block form used for H of
    Casida type."""
    a, b = inputs.small_dense(30, 2)
    h = sg.casida_matrix(a, b)
    sig = sg.casida_sigma(30)
    s = sg.sign_definition(h, sig)
    qp, qm = bs.alg6_bases_general(s, sig)
    qp2, qm2 = bs.alg6_cholesky_bases(s, 30)
    # the same factorizations; they differ only in how the leading block is symmetrized
    assert np.abs(qp - qp2).max() < 1e-12 and np.abs(qm - qm2).max() < 1e-11


@pytest.mark.parametrize("which", ["dwh", "newton"])
def test_comparison_iterations_reach_sign(which):
    """Sigma-DWH (Eq:LDLZolo with r = 1) and the scaled Newton iteration reach the
    definition of sign(H) and pass their stopping tests (u^{1/3}, u^{1/2})."""
    from oracle import iterations as it
    a, b = inputs.small_dense(50, 3)
    h = sg.casida_matrix(a, b)
    sig = sg.casida_sigma(50)
    amax, amin = sg.abs_eig_bounds(h, sig)
    sd = sg.sign_definition(h, sig)
    if which == "dwh":
        s, steps, change = it.sign_dwh(h, sig, 1.01 * amax, 0.99 * amin)
        assert change <= (2.0 ** -53) ** (1 / 3)
    else:
        s, steps, change = it.sign_newton(h, 1.01 * amax, 0.99 * amin)
        assert change <= (2.0 ** -53) ** (1 / 2)
    assert np.abs(s - sd).max() < 1e-13 * np.abs(sd).max()
