"""Matrix sign function of a definite pseudosymmetric matrix - oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``zolo_pd``: Alg. 8 (hyperbolic Zolo-PD) on the full n x n matrix, in FP64.
  Both steps use the LDL^T form of the iteration, Eq:LDLZolo:
      Z_j = X^T Sigma X + c_{2j-1} Sigma = P L D L^T P^T   (Bunch-Kaufman, scipy ``ldl``)
      X_new = hat C (X + sum_j a_j X Z_j^{-1} Sigma).
  The paper computes the first step with the inverse-free form Eq:HRZolo through
  the LDLIQR2 factorization of its reference [BenNP22], which is not part of the
  text; both forms evaluate the same rational function (Lemma HRnoInv) and the
  paper states that the LDL^T form is safe once the iterate is well conditioned,
  so the oracle uses the LDL^T form for both steps.  The stopping test
  ||X2 - X1||_F / ||X2||_F <= u^{1/(2r+1)} and the restart "A <- X2, go back to
  the estimation step" are taken as printed, with u = 2^-53.
* ``sign_definition``: sign(H) = V diag(sign lambda) V^{-1} (eq:signDef), with V
  from the simultaneous diagonalization of Sigma*H (SPD) and Sigma used in the
  proof of Thm. EVREalSigmaOrth, i.e. the symmetric-definite pencil
  Sigma x = mu (Sigma H) x, lambda = 1/mu.
* ``sign_definition_geev``: the same definition through LAPACK's nonsymmetric
  eigensolver, as an independent cross-check.
* ``zolo_pd_symmetric``: the Zolotarev iteration Eq:ZoloIt1 with M = I for a
  symmetric matrix (used by the symmetric divide-and-conquer of Alg. 2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from . import zolotarev as zol

U_DOUBLE = 2.0 ** -53


def casida_matrix(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """H = [[A, B], [-B, -A]] (Eq:Casida)."""
    return np.block([[a, b], [-b, -a]])


def casida_sigma(m: int) -> np.ndarray:
    """Diagonal of Sigma = diag(I_m, -I_m)."""
    return np.concatenate([np.ones(m), -np.ones(m)])


# --------------------------------------------------------------------------- LDL^T solve
def ldl_solve(lu: np.ndarray, d: np.ndarray, perm: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Solve Z Y = rhs given scipy's Bunch-Kaufman factorization Z = lu d lu^T.

    ``lu[perm]`` is unit lower triangular and ``d`` is block diagonal with 1x1 and
    2x2 blocks (the P, L, D factors of Eq:LDLZolo).
    """
    lp = lu[perm]
    t = sla.solve_triangular(lp, rhs[perm], lower=True, unit_diagonal=True)
    s = np.empty_like(t)
    n = d.shape[0]
    i = 0
    while i < n:
        if i + 1 < n and d[i + 1, i] != 0.0:
            s[i:i + 2] = np.linalg.solve(d[i:i + 2, i:i + 2], t[i:i + 2])
            i += 2
        else:
            s[i] = t[i] / d[i, i]
            i += 1
    yp = sla.solve_triangular(lp, s, lower=True, trans="T", unit_diagonal=True)
    y = np.empty_like(yp)
    y[perm] = yp
    return y


def ldl_zolo_step(x: np.ndarray, sigma: np.ndarray, co: zol.ZoloCoeffs) -> np.ndarray:
    """One step of Eq:LDLZolo: X <- hat C (X + sum_j a_j X Z_j^{-1} Sigma)."""
    sig = np.diag(sigma)
    xtsx = x.T @ (sigma[:, None] * x)
    acc = x.copy()
    for j in range(co.r):
        z = xtsx + co.c[2 * j] * sig                  # c_{2j-1} (0-based index 2j)
        lu, d, perm = sla.ldl(z, lower=True)
        acc += co.a[j] * (x @ ldl_solve(lu, d, perm, sig))
    return co.chat * acc


# --------------------------------------------------------------------------- definitions
def pencil_eig(h: np.ndarray, sigma: np.ndarray):
    """Eigenpairs of a definite pseudosymmetric H from the pencil (Sigma, Sigma H).

    The pencil solver gives X with X^T (Sigma H) X = I and X^T Sigma X = diag(mu)
    (the simultaneous diagonalization in the proof of Thm. EVREalSigmaOrth); then
    H X = X diag(1/mu) and X^{-1} = X^T Sigma H.  Returns (lam, X, X^{-1}) with
    lam = 1/mu in the solver's order.
    """
    sh = sigma[:, None] * h
    sh = 0.5 * (sh + sh.T)
    mu, xv = sla.eigh(np.diag(sigma), sh)
    lam = 1.0 / mu
    xinv = xv.T @ sh
    return lam, xv, xinv


def abs_eig_bounds(h: np.ndarray, sigma: np.ndarray):
    """(max |lambda|, min |lambda|) of a definite pseudosymmetric matrix (definition)."""
    lam, _, _ = pencil_eig(h, sigma)
    a = np.abs(lam)
    return float(a.max()), float(a.min())


def sign_definition(h: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """sign(H) = V diag(sign lambda) V^{-1} (eq:signDef) via the definite pencil."""
    lam, xv, xinv = pencil_eig(h, sigma)
    return (xv * np.sign(lam)[None, :]) @ xinv


def sign_definition_geev(h: np.ndarray) -> np.ndarray:
    """sign(H) = V diag(sign Re lambda) V^{-1} through the nonsymmetric eigensolver."""
    lam, v = np.linalg.eig(h)
    s = (v * np.sign(lam.real)[None, :]) @ np.linalg.inv(v)
    return s.real


def sign_blocks_from_spectral_factors(qm: np.ndarray, dm: np.ndarray, q: np.ndarray,
                                      mu: np.ndarray):
    """Closed form of the blocks (A_s, B_s) of sign(H) = [[A_s, B_s], [-B_s, -A_s]] when
    A + B = M = q_M diag(d_M) q_M^T and A - B = K = M^{-1/2} q diag(mu) q^T M^{-1/2}.

    With Q_h = [[I, I], [I, -I]] / sqrt(2), Q_h H Q_h = [[0, K], [M, 0]] =: X, and
    eq:signDef gives sign(X) = X (X^2)^{-1/2} = [[0, K (MK)^{-1/2}], [M (KM)^{-1/2}, 0]].
    For this K, KM = M^{-1/2} q diag(mu) q^T M^{1/2}, so
        S12 = K (MK)^{-1/2} = M^{-1/2} q diag(mu^{1/2}) q^T M^{-1/2},
        S21 = M (KM)^{-1/2} = M^{1/2} q diag(mu^{-1/2}) q^T M^{1/2},
    and Q_h [[0, S12], [S21, 0]] Q_h has blocks A_s = (S21 + S12)/2, B_s = (S21 - S12)/2.
    Only matrix products of the factors: usable at sizes where no eigensolver is.
    Returns (A_s, B_s) and a function cols(j) giving the columns j of both blocks
    at O(m^2 len(j)) cost."""
    mh = (qm * np.sqrt(dm)[None, :]) @ qm.T
    mih = (qm * (1.0 / np.sqrt(dm))[None, :]) @ qm.T
    cp = (q * np.sqrt(mu)[None, :]) @ q.T
    cm = (q * (1.0 / np.sqrt(mu))[None, :]) @ q.T
    s12 = mih @ (cp @ mih)
    s21 = mh @ (cm @ mh)
    return 0.5 * (s21 + s12), 0.5 * (s21 - s12)


def sign_columns_from_spectral_factors(qm, dm, q, mu, cols):
    """Columns `cols` of A_s and B_s (same closed form as above), applying every factor
    to the few columns instead of forming the m x m products."""
    e = np.zeros((qm.shape[0], len(cols)))
    e[np.asarray(cols), np.arange(len(cols))] = 1.0

    def apply(diag_m, diag_mu, x):
        x = qm @ (diag_m[:, None] * (qm.T @ x))
        x = q @ (diag_mu[:, None] * (q.T @ x))
        return qm @ (diag_m[:, None] * (qm.T @ x))

    s12 = apply(1.0 / np.sqrt(dm), np.sqrt(mu), e)
    s21 = apply(np.sqrt(dm), 1.0 / np.sqrt(mu), e)
    return 0.5 * (s21 + s12), 0.5 * (s21 - s12)


# --------------------------------------------------------------------------- Alg. 8
@dataclass
class ZoloRecord:
    r: int
    alpha: float
    beta: float
    ell: List[float] = field(default_factory=list)       # ell at the start of each step
    changes: List[float] = field(default_factory=list)   # ||X2-X1||_F/||X2||_F per attempt
    restarts: int = 0
    iterates: List[np.ndarray] = field(default_factory=list)
    coeffs: list = field(default_factory=list)


def zolo_pd(h: np.ndarray, sigma: np.ndarray, r: int = 8,
            alpha: Optional[float] = None, beta: Optional[float] = None,
            max_restarts: int = 2, keep_iterates: bool = False, u: float = U_DOUBLE):
    """Alg. 8: S = sign(H) for Sigma*H positive definite.  Returns (S, record)."""
    if alpha is None or beta is None:
        a_est, b_est = abs_eig_bounds(h, sigma)
        alpha = a_est if alpha is None else alpha
        beta = b_est if beta is None else beta
    rec = ZoloRecord(r=r, alpha=float(alpha), beta=float(beta))
    x = h / alpha
    ell = beta / alpha
    tol = u ** (1.0 / (2 * r + 1))
    for attempt in range(max_restarts + 1):
        s1, s2 = zol.two_step_schedule(ell, r)
        rec.ell += [s1.ell, s2.ell]
        rec.coeffs += [s1, s2]
        x1 = ldl_zolo_step(x, sigma, s1)
        x2 = ldl_zolo_step(x1, sigma, s2)
        if keep_iterates:
            rec.iterates += [x1, x2]
        change = np.linalg.norm(x2 - x1) / np.linalg.norm(x2)
        rec.changes.append(float(change))
        if change <= tol:
            return x2, rec
        # restart from X2: estimate its eigenvalue moduli and scale again
        rec.restarts += 1
        a_est, b_est = abs_eig_bounds(x2, sigma)
        x = x2 / a_est
        ell = min(b_est / a_est, 1.0 - 1e-15)
    return x2, rec


# --------------------------------------------------------------------------- symmetric Zolo-PD
def zolo_pd_symmetric(a: np.ndarray, r: int = 8, alpha: Optional[float] = None,
                      beta: Optional[float] = None, max_restarts: int = 2,
                      u: float = U_DOUBLE):
    """sign(A) of a symmetric nonsingular A by Eq:ZoloIt1 with M = I (Cholesky solves)."""
    if alpha is None or beta is None:
        w = np.abs(np.linalg.eigvalsh(0.5 * (a + a.T)))
        alpha = float(w.max()) if alpha is None else alpha
        beta = float(w.min()) if beta is None else beta
    x = a / alpha
    ell = min(beta / alpha, 1.0 - 1e-12)     # all |lambda| equal: X0 is already orthogonal
    tol = u ** (1.0 / (2 * r + 1))
    n = a.shape[0]
    for _ in range(max_restarts + 1):
        s1, s2 = zol.two_step_schedule(ell, r)
        xs = [x]
        for co in (s1, s2):
            xk = xs[-1]
            g = xk.T @ xk
            acc = xk.copy()
            for j in range(co.r):
                cf = sla.cho_factor(g + co.c[2 * j] * np.eye(n))
                acc += co.a[j] * sla.cho_solve(cf, xk.T).T
            xs.append(co.chat * acc)
        x1, x2 = xs[1], xs[2]
        if np.linalg.norm(x2 - x1) / np.linalg.norm(x2) <= tol:
            return 0.5 * (x2 + x2.T)
        w = np.abs(np.linalg.eigvalsh(0.5 * (x2 + x2.T)))
        x = x2 / w.max()
        ell = min(w.min() / w.max(), 1.0 - 1e-15)
    return 0.5 * (x2 + x2.T)
