"""Invariant-subspace bases from the matrix sign function - oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``alg6_cholesky_bases``: Alg. 6 for a definite pseudosymmetric matrix with
  Sigma = diag(I_p, -I_q).  Q_{1,+} = chol(P_+(1:p,1:p)) (upper factor, R^T R),
  Q_+ = [Q_{1,+}^T; P_+(p+1:n,1:p) Q_{1,+}^{-1}].  For Q_- the printed formula
  [Sigma Q_{1,-}^T; P_-(..) Q_{1,-}^{-1}] drops the factor hat Sigma_- = -I that
  Thm. HRisLDL puts into H = Sigma R^T hat Sigma; without it the two blocks have
  inconsistent signs and the columns leave range(P_-).  The oracle applies the
  theorem as stated: with -Sigma P_- = R^T R (R from the Cholesky factor of the
  leading q x q block, as printed), Q_- = Sigma R^T hat Sigma = -Sigma R^T.
* ``alg7_ldl_bases``: Alg. 7, the truncated pivoted LDL^T variant: ldl(Sigma P_+)
  = L D L^T, diagonalize the 1x1/2x2 blocks of D, keep the p largest entries,
  Q_+ = Sigma L V(:,1:p) D(1:p,1:p)^{1/2}; likewise with ldl(-Sigma P_-).
* ``pivoted_ldl_factor`` / ``alg7_pivoted_bases``: Alg. 7 with the LDL^T of Sigma P_+
  (and of -Sigma P_-) taken with 1x1 pivots and diagonal pivoting.  Both matrices are
  positive semidefinite with known rank (Thm. DefDivConq, Thm. EVREalSigmaOrth), so D
  is diagonal, its eigen-decomposition in step 4 is the identity, and the pivots come
  out in the order the truncation keeps.  Pivot rule (the paper leaves the pivoting to
  its ldl): per panel of `panel` columns, the `cand` largest diagonal entries of the
  current Schur complement (ties: lower index) are the candidates, and each pivot is
  the largest Schur diagonal among the remaining candidates (ties: lower index).  With
  `cand` at least the matrix size this is complete diagonal pivoting (LAPACK xPSTRF).
* ``congruent_bases_general``: for any signature, the bases from the projectors of the
  congruent symmetric T = R Sigma R^T (M = Sigma H = R^T R): H = R^{-1} T R, so the
  projectors of H are R^{-1} (I +- sign(T))/2 R and their ranges are W = R^{-1} applied to
  the ranges of Z_+- = (I +- sign(T))/2, symmetric positive semidefinite of rank r_+-.
  Z_+- = C C^T by the pivoted LDL^T above, V = W C, and Q = V R_G^{-1} with the Cholesky
  factor of the Sigma-Gram matrix +-V^T Sigma V (positive definite, Thm. DefDivConq).  Not
  one of the paper's listings: it avoids forming sign(H), whose projectors lose
  cond(M) u of accuracy, and is exact in exact arithmetic.
* ``alg4_orthogonal_bases``: Alg. 4 for a symmetric matrix: r_+ = trace(P_+),
  lower Cholesky factor of the leading r_+ block of P_+ extended by
  P_+(r_++1:n,1:r_+) Q_{1,+}^{-T}; the second half uses P_- throughout (the
  printed final line refers to P_+, which cannot give a basis of range(P_-)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def projectors(s: np.ndarray):
    """P_+ = (I + S)/2, P_- = (I - S)/2 (Lemma SignProj)."""
    n = s.shape[0]
    eye = np.eye(n)
    return 0.5 * (eye + s), 0.5 * (eye - s)


def alg6_cholesky_bases(s: np.ndarray, p: int):
    """Alg. 6 with Sigma = diag(I_p, -I_{n-p}).  Returns (Q_+, Q_-)."""
    n = s.shape[0]
    q = n - p
    sigma = np.concatenate([np.ones(p), -np.ones(q)])
    pp, pm = projectors(s)
    # positive part: Q_{1,+} = chol(Sigma(1:p,1:p) P_+(1:p,1:p)), upper, R^T R
    c_plus = sla.cholesky(sigma[:p, None] * pp[:p, :p], lower=False)
    top = (sigma[:p, None] * c_plus.T)
    bottom = sla.solve_triangular(c_plus, pp[p:, :p].T, trans="T", lower=False).T  # P21 C^{-1}
    q_plus = np.vstack([top, bottom])
    # negative part: -Sigma P_- = R^T R with R = [C, C^{-T} T_12] (pivot on the leading q rows)
    t = -(sigma[:, None] * pm)
    c_minus = sla.cholesky(t[:q, :q], lower=False)
    r_rest = sla.solve_triangular(c_minus, t[:q, q:], trans="T", lower=False)    # C^{-T} T_12
    rt = np.vstack([c_minus.T, r_rest.T])            # R^T (n x q)
    q_minus = -(sigma[:, None] * rt)                 # Sigma R^T hat Sigma_-, hat Sigma_- = -I
    return q_plus, q_minus


def alg6_cholesky_bases_plus(s: np.ndarray, p: int):
    """The Q_+ half of Alg. 6 only."""
    n = s.shape[0]
    sigma = np.concatenate([np.ones(p), -np.ones(n - p)])
    pp, _ = projectors(s)
    c_plus = sla.cholesky(sigma[:p, None] * pp[:p, :p], lower=False)
    bottom = sla.solve_triangular(c_plus, pp[p:, :p].T, trans="T", lower=False).T
    return np.vstack([sigma[:p, None] * c_plus.T, bottom])


def alg6_bases_general(s: np.ndarray, sigma: np.ndarray):
    """Alg. 6 for any signature Sigma (diagonal entries +-1 in any order), with r_+ and
    r_- the numbers of +1 and -1 entries (Thm. EVREalSigmaOrth).  As printed, the
    Cholesky factors come from the leading r_+ (resp. r_-) rows and columns of Sigma P_+
    (resp. -Sigma P_-), whatever signs Sigma has there:
        Q_{1,+} = chol(Sigma(1:r_+) P_+(1:r_+, 1:r_+))  (upper, R^T R),
        Q_+ = [Sigma(1:r_+) Q_{1,+}^T; P_+(r_+ + 1:n, 1:r_+) Q_{1,+}^{-1}].
    Q_- takes the sign of Thm. HRisLDL (see the module docstring): with
    -Sigma P_- = R^T R pivoted on the leading r_- indices, Q_- = Sigma R^T hat Sigma_-,
        Q_- = [-Sigma(1:r_-) Q_{1,-}^T; P_-(r_- + 1:n, 1:r_-) Q_{1,-}^{-1}].
    Returns (Q_+, Q_-)."""
    n = s.shape[0]
    p = int(np.sum(sigma > 0))
    q = n - p
    pp, pm = projectors(s)
    sp = sigma[:, None] * pp
    c_plus = sla.cholesky(0.5 * (sp[:p, :p] + sp[:p, :p].T), lower=False)
    top = sigma[:p, None] * c_plus.T
    bottom = sla.solve_triangular(c_plus, pp[p:, :p].T, trans="T", lower=False).T
    q_plus = np.vstack([top, bottom])
    sm = -(sigma[:, None] * pm)
    c_minus = sla.cholesky(0.5 * (sm[:q, :q] + sm[:q, :q].T), lower=False)
    top_m = -(sigma[:q, None] * c_minus.T)
    bottom_m = sla.solve_triangular(c_minus, pm[q:, :q].T, trans="T", lower=False).T
    q_minus = np.vstack([top_m, bottom_m])
    return q_plus, q_minus


def alg6_cholesky_bases_as_printed(s: np.ndarray, p: int):
    """Alg. 6 exactly as printed (kept only to document the sign error of Q_-)."""
    n = s.shape[0]
    q = n - p
    sigma = np.concatenate([np.ones(p), -np.ones(q)])
    pp, pm = projectors(s)
    c_plus = sla.cholesky(sigma[:p, None] * pp[:p, :p], lower=False)
    q_plus = np.vstack([sigma[:p, None] * c_plus.T,
                        sla.solve_triangular(c_plus, pp[p:, :p].T, trans="T").T])
    c_minus = sla.cholesky(-(sigma[:q, None] * pm[:q, :q]), lower=False)
    q_minus = np.vstack([sigma[:q, None] * c_minus.T,
                         sla.solve_triangular(c_minus, pm[q:, :q].T, trans="T").T])
    return q_plus, q_minus


def _truncated_ldl_basis(mat: np.ndarray, keep: int, sigma: np.ndarray):
    """Sigma L V(:,1:keep) D(1:keep,1:keep)^{1/2} from ldl(mat) (Alg. 7 steps 3-5)."""
    lu, d, _perm = sla.ldl(mat, lower=True)
    w, v = np.linalg.eigh(0.5 * (d + d.T))      # D is block diagonal: its eigen-decomposition
    order = np.argsort(w)[::-1]                  # descending
    w = w[order][:keep]
    v = v[:, order][:, :keep]
    if np.any(w <= 0):
        raise np.linalg.LinAlgError("truncated LDL^T: non-positive retained pivot")
    return sigma[:, None] * ((lu @ v) * np.sqrt(w)[None, :])


def alg7_ldl_bases(s: np.ndarray, sigma: np.ndarray):
    """Alg. 7 for general Sigma (p = number of +1 entries).  Returns (Q_+, Q_-)."""
    p = int(np.sum(sigma > 0))
    q = s.shape[0] - p
    pp, pm = projectors(s)
    q_plus = _truncated_ldl_basis(sigma[:, None] * pp, p, sigma)
    q_minus = _truncated_ldl_basis(-(sigma[:, None] * pm), q, sigma)
    return q_plus, q_minus


def pivoted_ldl_factor(z: np.ndarray, keep: int, panel: int = 64, cand: int = 128):
    """Truncated LDL^T with 1x1 pivots of the symmetric positive semidefinite z (Alg. 7
    steps 3-5): returns (C, piv) with C = L D^{1/2} restricted to the first `keep`
    pivots, rows in the original order (so z ~ C C^T when z has rank `keep`), and the
    pivot indices in the order taken.  Pivot rule as in the module docstring."""
    if cand < panel:
        raise ValueError("a panel needs at least as many candidates as pivots")
    z = 0.5 * (np.array(z, dtype=np.float64) + np.array(z, dtype=np.float64).T)
    n = z.shape[0]
    c = np.zeros((n, keep))
    piv = []
    free = np.ones(n, dtype=bool)
    for t0 in range(0, keep, panel):
        nb = min(panel, keep - t0)
        d = np.diag(z).copy()
        idx = np.flatnonzero(free)
        order = np.lexsort((idx, -d[idx]))          # largest first, then lower index
        cands = idx[order[:min(cand, idx.size)]]
        # greedy pivoting inside the candidate block (right-looking, one column a pivot)
        cd = d[cands].copy()
        cfree = np.ones(cands.size, dtype=bool)
        cb = np.zeros((cands.size, nb))
        slots = []
        for jj in range(nb):
            live = np.flatnonzero(cfree)
            if live.size == 0:
                raise np.linalg.LinAlgError("pivoted LDL^T: no candidate left")
            best = live[np.lexsort((cands[live], -cd[live]))[0]]
            if not cd[best] > 0.0:
                raise np.linalg.LinAlgError("pivoted LDL^T: non-positive retained pivot")
            sq = np.sqrt(cd[best])
            col = (z[cands, cands[best]] - cb[:, :jj] @ cb[best, :jj]) / sq
            col[best] = sq
            col[~cfree] = 0.0
            cb[:, jj] = col
            cfree[best] = False
            cd[cfree] -= col[cfree] ** 2
            slots.append(best)
        pp = cands[slots]
        lpp = cb[slots, :]                           # nb x nb, lower triangular
        # the panel for every row: z(:, pivots) L_pp^{-T}; rows pivoted earlier are zero,
        # the pivot rows are L_pp itself
        cp = sla.solve_triangular(lpp, z[:, pp].T, lower=True).T
        cp[~free] = 0.0
        cp[pp] = lpp
        c[:, t0:t0 + nb] = cp
        z = z - cp @ cp.T
        free[pp] = False
        piv.extend(int(i) for i in pp)
    return c, np.array(piv, dtype=np.int64)


def ldl_matrices(s: np.ndarray, sigma: np.ndarray):
    """Sigma P_+ = (Sigma S + Sigma)/2 and -Sigma P_- = (Sigma S - Sigma)/2, symmetrized
    (Sigma S is symmetric for the sign of a Sigma-self-adjoint matrix)."""
    ss = sigma[:, None] * s
    ss = 0.5 * (ss + ss.T)
    return 0.5 * (ss + np.diag(sigma)), 0.5 * (ss - np.diag(sigma))


def alg7_pivoted_bases(s: np.ndarray, sigma: np.ndarray, panel: int = 64, cand: int = 128):
    """Alg. 7 with the pivoted 1x1 LDL^T above: Q_+ = Sigma C_+ with C_+ C_+^T = Sigma P_+
    (rank p), Q_- = Sigma C_- with C_- C_-^T = -Sigma P_- (rank n - p).  Returns (Q_+, Q_-)."""
    p = int(np.sum(sigma > 0))
    q = s.shape[0] - p
    zp, zm = ldl_matrices(s, sigma)
    cp, _ = pivoted_ldl_factor(zp, p, panel, cand) if p else (np.zeros((s.shape[0], 0)), None)
    cm, _ = pivoted_ldl_factor(zm, q, panel, cand) if q else (np.zeros((s.shape[0], 0)), None)
    return sigma[:, None] * cp, sigma[:, None] * cm


def congruent_bases_general(h: np.ndarray, sigma: np.ndarray, u=None):
    """Bases of the two invariant subspaces of a definite pseudosymmetric H (Sigma H
    symmetric positive definite, any signature) from the projectors of the congruent
    symmetric T (module docstring).  Steps: M = sym(Sigma H) = R^T R, W = R^{-1},
    T = R Sigma R^T, U = sign(T) (given as `u`, else Alg. 8 on T with Cholesky solves);
    for (a, k) = (+1, r_+) and (-1, r_-): C C^T = (I + a U)/2 (rank k, pivoted 1x1 LDL^T),
    V = W C, a V^T Sigma V = R_G^T R_G, Q = V R_G^{-1}, and the decoupled block
    a Q^T Sigma H Q = a (R Q)^T (R Q) = a F^T F with F = C R_G^{-1} (R V = C).
    Returns (Q_+, Q_-, H_+, H_-)."""
    from . import sign as sg
    n = h.shape[0]
    m = sigma[:, None] * h
    m = 0.5 * (m + m.T)
    r = sla.cholesky(m, lower=False)
    w = sla.solve_triangular(r, np.eye(n), lower=False)
    if u is None:
        t = (r * sigma[None, :]) @ r.T
        u = sg.zolo_pd_symmetric(0.5 * (t + t.T))
    u = 0.5 * (u + u.T)
    out = []
    for a in (1.0, -1.0):
        k = int(np.sum(sigma * a > 0))
        if k == 0:
            out.append((np.zeros((n, 0)), np.zeros((0, 0))))
            continue
        c, _ = pivoted_ldl_factor(0.5 * (np.eye(n) + a * u), k)
        v = w @ c
        g = a * (v.T @ (sigma[:, None] * v))
        rg = sla.cholesky(0.5 * (g + g.T), lower=False)
        d = sla.solve_triangular(rg, np.eye(k), lower=False)
        f = c @ d
        out.append((v @ d, a * (f.T @ f)))
    (qp, hp), (qm, hm) = out
    return qp, qm, hp, hm


def alg4_orthogonal_bases(s: np.ndarray):
    """Alg. 4 for symmetric A with S = sign(A).  Returns (Q_+, Q_-), Q^T Q = I."""
    n = s.shape[0]
    pp, pm = projectors(s)
    r_plus = int(round(np.trace(pp)))
    r_minus = n - r_plus
    out = []
    for proj, rk in ((pp, r_plus), (pm, r_minus)):
        if rk == 0:
            out.append(np.zeros((n, 0)))
            continue
        l1 = sla.cholesky(proj[:rk, :rk], lower=True)        # Q_1 Q_1^T = P(1:rk,1:rk)
        lower = sla.solve_triangular(l1, proj[rk:, :rk].T, lower=True).T  # P21 Q_1^{-T}
        out.append(np.vstack([l1, lower]))
    return out[0], out[1]
