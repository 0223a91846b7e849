"""One step of structure-preserving spectral division for definite H - oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Alg. 3 with the simplifications of Sec. 5 for a definite pseudosymmetric H:
the shift is sigma = 0, the rank of P_+ is known (p = number of +1 entries of
Sigma, Thm. EVREalSigmaOrth), S = sign(H) comes from Alg. 8, the bases from
Alg. 6 or Alg. 7, and by Thm. DefDivConq the decoupled blocks are
    H_+ = Q_+^dagger H Q_+ = Q_+^T Sigma H Q_+        (hat Sigma_+ = I, SPD)
    H_- = Q_-^dagger H Q_- = -Q_-^T Sigma H Q_-       (hat Sigma_- = -I, negative definite).
The accuracy measure is the paper's backward error ||Q_+^T Sigma H Q_-||_F / ||H||_F
(Example 1, Sec. 6.1).
"""
from __future__ import annotations

import numpy as np

from . import bases as bs
from . import sign as sg


def decouple(h: np.ndarray, sigma: np.ndarray, q_plus: np.ndarray, q_minus: np.ndarray):
    """(H_+, H_-, backward error) for given bases (Thm. DefDivConq)."""
    sh = sigma[:, None] * h
    h_plus = q_plus.T @ sh @ q_plus
    h_minus = -(q_minus.T @ sh @ q_minus)
    bwd = np.linalg.norm(q_plus.T @ sh @ q_minus) / np.linalg.norm(h)
    return h_plus, h_minus, float(bwd)


def divide_casida(a: np.ndarray, b: np.ndarray, r: int = 8, alpha=None, beta=None,
                  basis: str = "alg6", max_restarts: int = 2, keep_iterates: bool = False):
    """Spectral division of H = [[A, B], [-B, -A]] with A +- B SPD.

    Returns a dict with S, Q_+, Q_-, H_+, H_-, the backward error and the
    Zolotarev record of Alg. 8.
    """
    m = a.shape[0]
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(m)
    s, rec = sg.zolo_pd(h, sigma, r=r, alpha=alpha, beta=beta,
                        max_restarts=max_restarts, keep_iterates=keep_iterates)
    if basis == "alg6":
        try:
            qp, qm = bs.alg6_cholesky_bases(s, m)
        except np.linalg.LinAlgError:
            # the leading block of -Sigma P_- is singular (e.g. B = 0): Alg. 6 breaks down
            # for Q_- (Sec. 5.1 notes such breakdowns); take Q_+ from Alg. 6 and Q_- from Alg. 7
            qp = bs.alg6_cholesky_bases_plus(s, m)
            qm = bs.alg7_ldl_bases(s, sigma)[1]
    elif basis == "alg7":
        qp, qm = bs.alg7_ldl_bases(s, sigma)
    elif basis == "alg7-pivoted":
        qp, qm = bs.alg7_pivoted_bases(s, sigma)
    else:
        raise ValueError(basis)
    hp, hm, bwd = decouple(h, sigma, qp, qm)
    return {"H": h, "sigma": sigma, "S": s, "Q_plus": qp, "Q_minus": qm,
            "H_plus": hp, "H_minus": hm, "backward_error": bwd, "record": rec}


def divide_general(h: np.ndarray, sigma: np.ndarray, r: int = 8, alpha=None, beta=None,
                   max_restarts: int = 2, basis: str = "alg6"):
    """Spectral division of a definite pseudosymmetric H for any signature Sigma
    (Sigma H symmetric positive definite; Sec. 5 and the matrices of Sec. 6.1): sign(H)
    by Alg. 8 with LDL^T solves on H, bases by Alg. 6 as printed (leading indices,
    Q_- with the sign of Thm. HRisLDL) or by Alg. 7 with the pivoted 1x1 LDL^T
    (basis = "alg7-pivoted"), or from the projectors of the congruent symmetric T
    (basis = "congruent", ``bases.congruent_bases_general``, sign(T) by Alg. 8 on T),
    decoupled blocks and backward error."""
    s, rec = sg.zolo_pd(h, sigma, r=r, alpha=alpha, beta=beta, max_restarts=max_restarts)
    if basis == "alg6":
        qp, qm = bs.alg6_bases_general(s, sigma)
    elif basis == "alg7-pivoted":
        qp, qm = bs.alg7_pivoted_bases(s, sigma)
    elif basis == "congruent":
        qp, qm, _, _ = bs.congruent_bases_general(h, sigma)
    else:
        raise ValueError(basis)
    hp, hm, bwd = decouple(h, sigma, qp, qm)
    return {"H": h, "sigma": sigma, "S": s, "Q_plus": qp, "Q_minus": qm,
            "H_plus": hp, "H_minus": hm, "backward_error": bwd, "record": rec}
