"""Eigen-decomposition of definite pseudosymmetric matrices - oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``eig_definite``: the plain definition.  Sigma*H is SPD, so Sigma and Sigma*H
  are diagonalized simultaneously (proof of Thm. EVREalSigmaOrth); the pencil
  solver returns X with X^T Sigma H X = I and X^T Sigma X = diag(1/lambda), and
  V = X |Lambda|^{1/2} satisfies V^T Sigma V = diag(+-1) (Eq:VSigmaOrth).
* ``canonical``: the ordering and normalization used to compare results.  The
  paper lists the p positive eigenvalues first, then the negative ones
  (Thm. EVREalSigmaOrth); within each group the order is |lambda| ascending, so
  that for the Casida form lambda[m+i] = -lambda[i].  Each eigenvector is scaled
  to v^T Sigma v = +-1 and its sign is chosen so that its entry of largest
  modulus (lowest index on ties) is positive.
* ``alg2_symmetric_dc``: Alg. 2 (symmetric spectral divide-and-conquer) with the
  Zolotarev sign iteration and the Alg. 4 bases; the shift is the median of the
  diagonal (the paper leaves the shift choice open), nudged when it does not
  split the spectrum.
"""
from __future__ import annotations

import numpy as np

from . import bases as bs
from . import sign as sg


def canonical_sign(v: np.ndarray) -> np.ndarray:
    """Flip each column so its largest-modulus entry (lowest index on ties) is positive."""
    idx = np.argmax(np.abs(v), axis=0)
    s = np.sign(v[idx, np.arange(v.shape[1])])
    s[s == 0] = 1.0
    return v * s[None, :]


def canonical(lam: np.ndarray, v: np.ndarray, sigma: np.ndarray):
    """Order positives |lambda| ascending then negatives |lambda| ascending; normalize V."""
    pos = np.where(lam > 0)[0]
    neg = np.where(lam < 0)[0]
    pos = pos[np.argsort(lam[pos], kind="stable")]
    neg = neg[np.argsort(-lam[neg], kind="stable")]
    order = np.concatenate([pos, neg])
    lam = lam[order]
    v = v[:, order]
    nrm = np.sqrt(np.abs(np.einsum("ij,i,ij->j", v, sigma, v)))
    v = v / nrm[None, :]
    return lam, canonical_sign(v)


def eig_definite(h: np.ndarray, sigma: np.ndarray):
    """All eigenpairs of a definite pseudosymmetric H, canonical order (plain definition)."""
    lam, xv, _ = sg.pencil_eig(h, sigma)
    return canonical(lam, xv, sigma)


def eig_casida(a: np.ndarray, b: np.ndarray):
    """Eigenpairs of H = [[A, B], [-B, -A]] in canonical order."""
    m = a.shape[0]
    return eig_definite(sg.casida_matrix(a, b), sg.casida_sigma(m))


def alg2_symmetric_dc(a: np.ndarray, r: int = 8, leaf: int = 1):
    """Alg. 2: orthogonal V and eigenvalues of symmetric A by recursive sign splits."""
    n = a.shape[0]
    if n <= leaf:
        if n == 1:
            return np.array([a[0, 0]]), np.ones((1, 1))
        w, v = np.linalg.eigh(a)
        return w, v
    diag = np.sort(np.diag(a))
    shift = float(np.median(diag))
    for attempt in range(8):
        shifted = a - shift * np.eye(n)
        s = sg.zolo_pd_symmetric(shifted, r=r)
        pp = 0.5 * (np.eye(n) + s)
        rk = int(round(np.trace(pp)))
        if 0 < rk < n:
            break
        lo, hi = diag[0], diag[-1]
        shift = shift + (hi - lo) * (0.25 if rk == n else -0.25) / (attempt + 1)
    else:
        w, v = np.linalg.eigh(a)
        return w, v
    qp, qm = bs.alg4_orthogonal_bases(s)
    v0 = np.hstack([qp, qm])
    a11 = qp.T @ a @ qp
    a22 = qm.T @ a @ qm
    w1, v1 = alg2_symmetric_dc(0.5 * (a11 + a11.T), r, leaf)
    w2, v2 = alg2_symmetric_dc(0.5 * (a22 + a22.T), r, leaf)
    v = v0 @ np.block([[v1, np.zeros((v1.shape[0], v2.shape[1]))],
                       [np.zeros((v2.shape[0], v1.shape[1])), v2]])
    w = np.concatenate([w1, w2])
    order = np.argsort(w, kind="stable")
    return w[order], v[:, order]
