"""Zolotarev coefficients for the matrix sign iteration, in multiprecision.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Sec. 5.2 (Subsec:DefZolo) of the paper:

* Eq:Compcis: c_i = l^2 sn^2(u_i; l') / cn^2(u_i; l'),  i = 1..2r,
  with l' = sqrt(1 - l^2), K' = K(l') and u_i = i K' / (2r + 1).
  Reading: the unlabelled argument "i K'/(2r+1)" uses the summation index i
  (not the imaginary unit); the Jacobi functions take the modulus l', i.e. the
  parameter m = l'^2 = 1 - l^2.
* Eq:hatZ: hat Z(x; l) = hat C x prod_j (x^2 + c_{2j}) / (x^2 + c_{2j-1}),
  hat C = prod_j (1 + c_{2j-1}) / (1 + c_{2j}), so that hat Z(1; l) = 1.
* Eq:ZPartialFrac / Eq:ZPartialFrac2: hat Z(x) = hat C x (1 + sum_j a_j /
  (x^2 + c_{2j-1})).  Reading: the printed a_j multiplies the two products; the
  residue of the partial fraction is their quotient,
  a_j = - prod_k (c_{2j-1} - c_{2k}) / prod_{k != j} (c_{2j-1} - c_{2k-1}).
* Alg. 8: l_next = hat Z(l; l) = hat C l prod_j (l^2 + c_{2j}) / (l^2 + c_{2j-1}).

All arithmetic runs in mpmath at ``dps`` decimal digits; results are returned as
Python floats (rounded once) and, on request, as mpf values.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import mpmath as mp

DEFAULT_DPS = 60


@dataclass
class ZoloCoeffs:
    """Coefficients of one Zolotarev step (Eq:Compcis, Eq:hatZ, Eq:ZPartialFrac2)."""
    ell: float
    r: int
    c: List[float]        # c_1..c_2r   (index 0 holds c_1)
    a: List[float]        # a_1..a_r
    chat: float           # hat C
    ell_next: float       # hat Z(ell; ell)
    c_mp: list = None
    a_mp: list = None
    chat_mp: object = None
    ell_next_mp: object = None

    def c_odd(self) -> List[float]:
        """The pole shifts c_{2j-1}, j = 1..r."""
        return [self.c[2 * j] for j in range(self.r)]


def _coeffs_mp(ell, r: int):
    """c_1..c_2r, a_1..a_r, hat C, hat Z(ell; ell) as mpf values at the current precision."""
    ell = mp.mpf(ell)
    mparam = 1 - ell * ell                 # parameter of the complementary modulus l'
    kprime = mp.ellipk(mparam)             # K' = K(l')
    c = []
    for i in range(1, 2 * r + 1):
        u = i * kprime / (2 * r + 1)
        sn = mp.ellipfun("sn", u, m=mparam)
        cn = mp.ellipfun("cn", u, m=mparam)
        c.append(ell * ell * (sn * sn) / (cn * cn))
    a = []
    for j in range(1, r + 1):
        cj = c[2 * j - 2]                                        # c_{2j-1}
        num = mp.fprod([cj - c[2 * k - 1] for k in range(1, r + 1)])              # c_{2k}
        den = mp.fprod([cj - c[2 * k - 2] for k in range(1, r + 1) if k != j])    # c_{2k-1}
        a.append(-num / den)
    chat = mp.fprod([(1 + c[2 * j - 2]) / (1 + c[2 * j - 1]) for j in range(1, r + 1)])
    ell_next = chat * ell * mp.fprod(
        [(ell * ell + c[2 * j - 1]) / (ell * ell + c[2 * j - 2]) for j in range(1, r + 1)])
    return c, a, chat, ell_next


def coefficients(ell, r: int, dps: int = DEFAULT_DPS) -> ZoloCoeffs:
    """Coefficients of hat Z_{2r+1}(x; ell) for 0 < ell < 1 (Eq:Compcis, Eq:hatZ)."""
    if r < 1:
        raise ValueError("r must be >= 1")
    with mp.workdps(dps):
        if not (0 < mp.mpf(ell) < 1):
            raise ValueError("ell must lie in (0, 1)")
        c, a, chat, ell_next = _coeffs_mp(ell, r)
        return ZoloCoeffs(
            ell=float(mp.mpf(ell)), r=r,
            c=[float(v) for v in c], a=[float(v) for v in a],
            chat=float(chat), ell_next=float(ell_next),
            c_mp=c, a_mp=a, chat_mp=chat, ell_next_mp=ell_next)


def zhat(x, co: ZoloCoeffs, dps: int = DEFAULT_DPS):
    """hat Z(x; ell) in product form (Eq:hatZ), evaluated in multiprecision."""
    with mp.workdps(dps):
        x = mp.mpf(x)
        p = mp.fprod([(x * x + co.c_mp[2 * j + 1]) / (x * x + co.c_mp[2 * j])
                      for j in range(co.r)])
        return co.chat_mp * x * p


def zhat_partial_fraction(x, co: ZoloCoeffs, dps: int = DEFAULT_DPS):
    """hat Z(x; ell) in partial-fraction form (Eq:ZPartialFrac)."""
    with mp.workdps(dps):
        x = mp.mpf(x)
        s = 1 + mp.fsum([co.a_mp[j] / (x * x + co.c_mp[2 * j]) for j in range(co.r)])
        return co.chat_mp * x * s


def two_step_schedule(ell, r: int, dps: int = DEFAULT_DPS):
    """Coefficients for the two steps of Alg. 8: step 1 at ell, step 2 at ell_1 = hat Z(ell; ell)."""
    s1 = coefficients(ell, r, dps)
    with mp.workdps(dps):
        ell1 = s1.ell_next_mp
        if ell1 >= 1:
            ell1 = 1 - mp.mpf(10) ** (-dps + 5)
        s2 = coefficients(ell1, r, dps)
    return s1, s2


def choose_r(ell, tol: float = 1e-15, r_max: int = 8, dps: int = DEFAULT_DPS) -> int:
    """Smallest r <= r_max for which two steps map [ell, 1] into [1 - tol, 1].

    The paper picks r from a table of its reference [NakF16] that is not part of
    the text; this computes the same criterion directly from the l-recurrence.
    """
    for r in range(1, r_max + 1):
        s1, s2 = two_step_schedule(ell, r, dps)
        with mp.workdps(dps):
            if 1 - s2.ell_next_mp <= tol:
                return r
    return r_max
