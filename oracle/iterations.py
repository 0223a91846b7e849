"""The comparison iterations of Sec. 6 (Tab:ItRuntime) for the matrix sign function of a
definite pseudosymmetric H - oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Sigma-DWH: the Zolotarev step of Alg. 8 with r = 1 (the dynamically weighted Halley
  iteration, text after Eq:Compcis), repeated with the l-recurrence l <- hat Z(l; l)
  until the scalar recurrence reaches 1 - 1e-15, plus one step for the stopping test
  ||X_k - X_{k-1}||_F / ||X_k||_F <= u^{1/3} (convergence rate 3).  Each step is taken
  in the LDL^T form of Eq:LDLZolo on the full H ("Sigma DWH with LDL^T").
* Scaled Newton for the sign function, X <- (mu X + (mu X)^{-1}) / 2, with the scaling
  of Byers and Xu that the paper uses ("suboptimal scaling"): for eigenvalue moduli in
  [l, 1], mu_0 = 1 / sqrt(l); afterwards the moduli lie in [1, u_k] with
  u_1 = (mu_0 + 1/mu_0) / 2 and mu_k = 1 / sqrt(u_k), u_{k+1} = (mu_k + 1/mu_k) / 2.
  Steps are taken until u_k - 1 <= 1e-15, plus one for the stopping test with
  u^{1/2} (convergence rate 2).  The inverse is LAPACK's (LU with pivoting).
The step counts these schedules give are the ones Tab:ItRuntime reports (5, 6, 6 and
7, 9, 9 at kappa = 1e2, 1e8, 1e12); the tests pin that.
"""
from __future__ import annotations

import math

import numpy as np

from . import sign as sg
from . import zolotarev as zol

U_DOUBLE = 2.0 ** -53


def dwh_schedule(ell: float, tol: float = 1e-15, max_steps: int = 30):
    """Coefficients of the r = 1 steps: until 1 - l <= tol, then one more."""
    out = []
    while len(out) < max_steps:
        co = zol.coefficients(min(ell, 1.0 - 1e-16), 1)
        out.append(co)
        done = 1.0 - ell <= tol
        ell = min(co.ell_next, 1.0 - 1e-16)
        if done:
            break
        if 1.0 - ell <= tol:
            out.append(zol.coefficients(ell, 1))   # the step of the stopping test
            break
    return out


def newton_schedule(ell: float, tol: float = 1e-15, max_steps: int = 60):
    """Scalings mu_k of the scaled Newton steps for eigenvalue moduli in [ell, 1]."""
    mus = [1.0 / math.sqrt(ell)]
    u = 0.5 * (mus[0] + 1.0 / mus[0])
    while len(mus) < max_steps:
        mu = 1.0 / math.sqrt(u)
        mus.append(mu)
        if u - 1.0 <= tol:
            break
        u = 0.5 * (mu + 1.0 / mu)
    return mus


def sign_dwh(h: np.ndarray, sigma: np.ndarray, alpha: float, beta: float):
    """Sigma-DWH with LDL^T solves (Eq:LDLZolo, r = 1).  Returns (S, steps, last change)."""
    x = h / alpha
    prev = None
    steps = dwh_schedule(beta / alpha)
    for co in steps:
        prev, x = x, sg.ldl_zolo_step(x, sigma, co)
    change = float(np.linalg.norm(x - prev) / np.linalg.norm(x))
    return x, len(steps), change


def sign_newton(h: np.ndarray, alpha: float, beta: float):
    """Scaled Newton iteration for sign(H).  Returns (S, steps, last change)."""
    x = h / alpha
    prev = None
    mus = newton_schedule(beta / alpha)
    for mu in mus:
        prev, x = x, 0.5 * (mu * x + np.linalg.inv(mu * x))
    change = float(np.linalg.norm(x - prev) / np.linalg.norm(x))
    return x, len(mus), change
