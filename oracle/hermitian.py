"""The complex Bethe-Salpeter forms (Sec. 5) - oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Eq:BSE2: H = [[A, B], [-B, -A]] with A, B Hermitian (the complex Casida form).
* Eq:BSE1: H = [[A, B], [-conj(B), -conj(A)]] with A Hermitian and B complex symmetric.
Both are pseudo-Hermitian for Sigma = diag(I_m, -I_m) and definite when Sigma H is
Hermitian positive definite (Sec. 5).  Everything here is complex arithmetic taken
from the definitions: sign(H) by the definite pencil (Thm. EVREalSigmaOrth) or by a
general eigensolver (eq:signDef), Alg. 6 with conjugate transposes, and the decoupled
block of Thm. DefDivConq.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def bse2_matrix(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """H = [[A, B], [-B, -A]] (Eq:BSE2)."""
    return np.block([[a, b], [-b, -a]])


def bse1_matrix(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """H = [[A, B], [-conj(B), -conj(A)]] (Eq:BSE1; B^H = conj(B) for symmetric B)."""
    return np.block([[a, b], [-b.conj(), -a.conj()]])


def sigma_of(m: int) -> np.ndarray:
    return np.concatenate([np.ones(m), -np.ones(m)])


def sign_pencil(h: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """sign(H) through the definite pencil: M = Sigma H = L L^H (Hermitian positive
    definite), T = L^H Sigma L Hermitian and L^H H L^{-H} = T, so
    sign(H) = L^{-H} sign(T) L^H with sign(T) = W sign(Lambda) W^H (eigh)."""
    m_mat = sigma[:, None] * h
    m_mat = 0.5 * (m_mat + m_mat.conj().T)
    l = np.linalg.cholesky(m_mat)                       # M = L L^H
    t = l.conj().T @ (sigma[:, None] * l)
    t = 0.5 * (t + t.conj().T)
    lam, w = np.linalg.eigh(t)
    st = (w * np.sign(lam)[None, :]) @ w.conj().T
    lh = l.conj().T
    return sla.solve_triangular(lh, st @ lh, lower=False)   # L^{-H} sign(T) L^H


def sign_geev(h: np.ndarray) -> np.ndarray:
    """sign(H) = V diag(sign Re lambda) V^{-1} by the general complex eigensolver."""
    lam, v = np.linalg.eig(h)
    return (v * np.sign(lam.real)[None, :]) @ np.linalg.inv(v)


def alg6_plus(s: np.ndarray, m: int) -> np.ndarray:
    """Alg. 6 for Sigma = diag(I_m, -I_m) in complex arithmetic: P_+ = (I + S)/2,
    C = chol(P_+(1:m, 1:m)) upper (C^H C), Q_+ = [C^H; P_+(m+1:2m, 1:m) C^{-1}]."""
    n = s.shape[0]
    pp = 0.5 * (np.eye(n) + s)
    lead = 0.5 * (pp[:m, :m] + pp[:m, :m].conj().T)
    c = sla.cholesky(lead, lower=False)
    bottom = sla.solve_triangular(c, pp[m:, :m].T, trans="T").T   # P_21 C^{-1}
    return np.vstack([c.conj().T, bottom])


def decouple_plus(h: np.ndarray, sigma: np.ndarray, q_plus: np.ndarray) -> np.ndarray:
    """H_+ = Q_+^H Sigma H Q_+ (Thm. DefDivConq), Hermitian positive definite."""
    return q_plus.conj().T @ ((sigma[:, None] * h) @ q_plus)


def positive_eigenvalues(h: np.ndarray) -> np.ndarray:
    """The positive eigenvalues of H, ascending, by the general complex eigensolver."""
    lam = np.linalg.eigvals(h).real
    return np.sort(lam[lam > 0])
