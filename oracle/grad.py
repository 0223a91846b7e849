"""Reference derivatives of the matrix sign function of H = [[A, B], [-B, -A]] - oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper differentiates nothing; the derivative asked of the library is that of
its sign function (eq:signDef) and of the spectral projector P_+ = (I + sign(H))/2
(the projector of Lemma SignProj onto the invariant subspace of the positive
eigenvalues).  The oracle writes the plain definitions out:

* ``frechet_adjoint``: for a diagonalizable H = V diag(lambda) V^{-1} and a scalar
  function f, the Frechet derivative is L(H, E) = V (F o (V^{-1} E V)) V^{-1} with the
  divided differences F_ij = (f(lambda_i) - f(lambda_j)) / (lambda_i - lambda_j)
  (f'(lambda_i) on the diagonal; 0 for the sign function, whose eigenvalues here
  stay away from 0).  Its adjoint with respect to <X, Y> = trace(X^T Y) is
  L*(H, G) = V^{-T} (F o (V^T G V^{-T})) V^T.  V and lambda come from the
  simultaneous diagonalization of Sigma*H and Sigma (``sign.pencil_eig``).
* ``grad_blocks``: H depends on (A, B) through dH = [[dA, dB], [-dB, -dA]], so for a
  loss with dL = <G_H, dH> the gradients are G11 - G22 (for A) and G12 - G21 (for
  B).  A and B are symmetric, so the gradient is reported as the symmetric part
  (the reading that makes <grad, E> the derivative along every symmetric E).
* ``projector_loss`` / ``projector_loss_grad``: L(A, B) = trace(W P_+) and its
  gradient; dL/dS = W^T / 2.
* ``sign_block_grad``: the gradient for a loss given through the blocks of
  sign(H) = [[S_A, S_B], [-S_B, -S_A]]: dL = <g_A, dS_A> + <g_B, dS_B> equals
  <G_S, dS> with G_S = [[g_A, g_B], [0, 0]].
"""
from __future__ import annotations

import numpy as np

from . import sign as sg


def _sym(x: np.ndarray) -> np.ndarray:
    return 0.5 * (x + x.T)


def frechet_adjoint_sign(h: np.ndarray, sigma: np.ndarray, g: np.ndarray) -> np.ndarray:
    """L*(H, G) for f = sign, by the divided-difference (Daleckii-Krein) formula."""
    lam, v, vinv = sg.pencil_eig(h, sigma)
    s = np.sign(lam)
    diff = lam[:, None] - lam[None, :]
    same = s[:, None] == s[None, :]
    f = np.where(same, 0.0, (s[:, None] - s[None, :]) / np.where(same, 1.0, diff))
    return vinv.T @ (f * (v.T @ g @ vinv.T)) @ v.T


def grad_blocks(gh: np.ndarray, m: int):
    """(dL/dA, dL/dB) from dL/dH, symmetric parts."""
    g11, g12 = gh[:m, :m], gh[:m, m:]
    g21, g22 = gh[m:, :m], gh[m:, m:]
    return _sym(g11 - g22), _sym(g12 - g21)


def sign_block_grad(a: np.ndarray, b: np.ndarray, ga: np.ndarray, gb: np.ndarray):
    """Gradient w.r.t. (A, B) of a loss whose gradient w.r.t. (S_A, S_B) is (ga, gb)."""
    m = a.shape[0]
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(m)
    gs = np.zeros((2 * m, 2 * m))
    gs[:m, :m] = ga
    gs[:m, m:] = gb
    return grad_blocks(frechet_adjoint_sign(h, sigma, gs), m)


def projector_loss(a: np.ndarray, b: np.ndarray, w: np.ndarray) -> float:
    """trace(W P_+), P_+ = (I + sign(H)) / 2, sign by its definition."""
    m = a.shape[0]
    s = sg.sign_definition(sg.casida_matrix(a, b), sg.casida_sigma(m))
    return float(np.trace(w @ (0.5 * (np.eye(2 * m) + s))))


def projector_loss_grad(a: np.ndarray, b: np.ndarray, w: np.ndarray):
    """(dL/dA, dL/dB) of trace(W P_+)."""
    m = a.shape[0]
    h = sg.casida_matrix(a, b)
    sigma = sg.casida_sigma(m)
    return grad_blocks(frechet_adjoint_sign(h, sigma, 0.5 * w.T), m)
