"""Pins for the oracle's Zolotarev coefficients (Sec. 5.2, Eq:Compcis, Eq:hatZ,
Eq:ZPartialFrac2, Alg. 8).  Every check compares against something other than
the oracle's own formulas: a published closed form, an identity of the Jacobi
elliptic functions, the Chebyshev alternation of a best approximation, the
composition property, or numbers the paper prints.
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import zolotarev as zol

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def dwh_closed_form(ell):
    """Dynamically weighted Halley weights (Nakatsukasa, Bai, Gygi 2010), which the paper
    identifies with the r = 1 Zolotarev function (text after Eq:Compcis)."""
    ell = mp.mpf(ell)
    gam = mp.cbrt(4 * (1 - ell ** 2) / ell ** 4)
    a = mp.sqrt(1 + gam) + mp.sqrt(8 - 4 * gam + 8 * (2 - ell ** 2) / (ell ** 2 * mp.sqrt(1 + gam))) / 2
    b = (a - 1) ** 2 / 4
    c = a + b - 1
    return a, b, c


@pytest.mark.parametrize("ell", [0.5, 0.1, 1e-2, 1e-4, 1e-6])
def test_r1_equals_dwh(ell):
    # x (a + b x^2) / (1 + c x^2) = hat C x (x^2 + c_2) / (x^2 + c_1)
    with mp.workdps(60):
        a, b, c = dwh_closed_form(ell)
        co = zol.coefficients(ell, 1)
        assert abs(co.c_mp[0] - 1 / c) / (1 / c) < mp.mpf(10) ** -40
        assert abs(co.c_mp[1] - a / b) / (a / b) < mp.mpf(10) ** -40
        assert abs(co.chat_mp - b / c) / (b / c) < mp.mpf(10) ** -40
        e = mp.mpf(ell)
        lnext = e * (a + b * e ** 2) / (1 + c * e ** 2)
        assert abs(co.ell_next_mp - lnext) < mp.mpf(10) ** -40


@pytest.mark.parametrize("r", [1, 2, 5, 8])
@pytest.mark.parametrize("ell", [1e-12, 1e-3, 0.04, 0.5])
def test_reflection_identity(r, ell):
    # sn(K'-u) = cn(u)/dn(u), cn(K'-u) = l sn(u)/dn(u)  =>  c_i c_{2r+1-i} = l^2
    co = zol.coefficients(ell, r)
    with mp.workdps(60):
        for i in range(1, 2 * r + 1):
            prod = co.c_mp[i - 1] * co.c_mp[2 * r - i]
            assert abs(prod - mp.mpf(ell) ** 2) / mp.mpf(ell) ** 2 < mp.mpf(10) ** -45


@pytest.mark.parametrize("r,ell", [(1, 0.3), (2, 0.05), (3, 0.01), (8, 0.04)])
def test_coefficients_ordered_and_residues_positive(r, ell):
    co = zol.coefficients(ell, r)
    assert all(co.c[i] < co.c[i + 1] for i in range(2 * r - 1))
    assert all(a > 0 for a in co.a)
    assert 0 < co.chat < 1


@pytest.mark.parametrize("r,ell", [(1, 0.3), (2, 0.05), (3, 0.02), (4, 0.2)])
def test_equioscillation(r, ell):
    """Best rational approximation of sign on [l,1]: hat Z attains its minimum hat Z(l)
    at r+1 points (x = l and r interior points) and its maximum 1 at r+1 points
    (r interior points and x = 1), alternating: 2r + 2 alternation points."""
    co = zol.coefficients(ell, r)
    f = lambda x: float(zol.zhat(x, co, dps=30))
    xs = np.geomspace(ell, 1.0, 20001)
    ys = np.array([f(x) for x in xs])
    lo, hi = ys.min(), ys.max()
    assert hi == pytest.approx(1.0, abs=1e-12)
    assert lo == pytest.approx(co.ell_next, rel=1e-9)
    inner_max = [i for i in range(1, len(ys) - 1) if ys[i] >= ys[i - 1] and ys[i] >= ys[i + 1]]
    inner_min = [i for i in range(1, len(ys) - 1) if ys[i] <= ys[i - 1] and ys[i] <= ys[i + 1]]
    assert len(inner_max) == r and len(inner_min) == r
    amp = 1.0 - co.ell_next
    for i in inner_max:
        assert abs(ys[i] - 1.0) < 2e-3 * amp
    for i in inner_min:
        assert abs(ys[i] - co.ell_next) < 2e-3 * amp
    ext = sorted([0, len(xs) - 1] + inner_max + inner_min)
    kinds = ["min" if (i == 0 or i in inner_min) else "max" for i in ext]
    assert all(kinds[k] != kinds[k + 1] for k in range(len(kinds) - 1))
    assert len(ext) == 2 * r + 2


@pytest.mark.parametrize("r,ell", [(1, 1e-3), (2, 0.05), (2, 1e-6), (3, 1e-8)])
def test_composition_property(r, ell):
    """hat Z_{2r+1}(hat Z_{2r+1}(x; l); l_1) = hat Z_{(2r+1)^2}(x; l) (text before Eq:hatZ)."""
    rr = ((2 * r + 1) ** 2 - 1) // 2
    with mp.workdps(70):
        s1, s2 = zol.two_step_schedule(ell, r, dps=70)
        big = zol.coefficients(ell, rr, dps=70)
        for x in [ell, 2 * ell, 0.1, 0.37, 0.9, 1.0]:
            lhs = zol.zhat(zol.zhat(x, s1, 70), s2, 70)
            rhs = zol.zhat(x, big, 70)
            assert abs(lhs - rhs) < mp.mpf(10) ** -35


def test_two_step_bound_printed():
    g = GOLDEN["two_step_bound"]
    r, ell = g["r"], g["ell_min"]
    s1, s2 = zol.two_step_schedule(ell, r)
    with mp.workdps(60):
        # minimum of the composed function on [l, 1] is attained at x = l
        assert s2.ell_next_mp >= mp.mpf(g["lower_bound"])
        for x in np.geomspace(ell, 1.0, 200):
            v = zol.zhat(zol.zhat(x, s1), s2)
            assert mp.mpf(g["lower_bound"]) <= v <= 1 + mp.mpf(10) ** -40


@pytest.mark.parametrize("r,ell", [(2, 0.05), (8, 0.04), (8, 1e-10)])
def test_partial_fraction_quotient_reading(r, ell):
    """Eq:ZPartialFrac2 must be a quotient: the product form of Eq:hatZ and the partial
    fractions agree; the printed product would not."""
    co = zol.coefficients(ell, r)
    with mp.workdps(60):
        for x in [ell, 0.2, 0.5, 1.0, 3.0]:
            assert abs(zol.zhat(x, co) - zol.zhat_partial_fraction(x, co)) < mp.mpf(10) ** -40
        assert abs(zol.zhat(1.0, co) - 1) < mp.mpf(10) ** -45
        # the literal product reading gives a different function
        bad = []
        for j in range(1, r + 1):
            cj = co.c_mp[2 * j - 2]
            bad.append(-mp.fprod([cj - co.c_mp[2 * k - 1] for k in range(1, r + 1)])
                       * mp.fprod([cj - co.c_mp[2 * k - 2] for k in range(1, r + 1) if k != j]))
        x = mp.mpf("0.5")
        val = co.chat_mp * x * (1 + mp.fsum([bad[j] / (x * x + co.c_mp[2 * j]) for j in range(r)]))
        assert abs(val - zol.zhat(x, co)) > mp.mpf(10) ** -6


def _scalar_iterations(ell, r, tol=1e-15, kmax=40):
    k = 0
    with mp.workdps(60):
        e = mp.mpf(ell)
        while 1 - e > tol and k < kmax:
            co = zol.coefficients(e, r)
            e = co.ell_next_mp
            k += 1
    return k


def test_iteration_counts_table1():
    """Tab:ItRuntime: Zolo-PD (r = 8) takes 2 steps for kappa = 1e2, 1e8, 1e12; the r = 1
    variant (Sigma-DWH) reports 5, 6, 6, i.e. the scalar count plus the one extra
    iteration its stopping test needs."""
    g = GOLDEN["table1_iterations"]
    for kappa, z, d in zip(g["kappa"], g["hyperbolic_zolo_pd"], g["sigma_dwh_ldliqr2"]):
        ell = 1.0 / kappa
        assert _scalar_iterations(ell, 8) == z
        assert _scalar_iterations(ell, 1) + 1 == d


def test_choose_r_rule_monotone():
    rs = [zol.choose_r(e) for e in [0.5, 0.1, 1e-2, 1e-4, 1e-8, 1e-12, 1e-16]]
    assert rs == sorted(rs)
    assert rs[-1] <= 8


@pytest.mark.parametrize("ell", [0.5, 0.2, 0.1, 0.04, 0.01, 1e-3, 1e-6, 1e-10])
def test_choose_r_against_composite_function(ell):
    """The rule for r (Alg. 8 takes it from a table that is not in the text): the smallest
    r whose two steps reach 1 - 1e-15 at x = l.  By the composition property of Sec. 5.2,
    two steps of hat Z_{2r+1} are the single function hat Z_{(2r+1)^2}(x; l), whose value
    at l comes from its own coefficients (degree parameter R = ((2r+1)^2 - 1)/2 = 2r(r+1)),
    not from the two-step schedule.  The returned r must meet the bound and r - 1 must not."""
    tol = mp.mpf("1e-15")
    r = zol.choose_r(ell)
    with mp.workdps(60):
        assert 1 - zol.coefficients(ell, 2 * r * (r + 1)).ell_next_mp <= tol
        if r > 1:
            assert 1 - zol.coefficients(ell, 2 * (r - 1) * r).ell_next_mp > tol


def test_comparison_iteration_counts_table1():
    """Tab:ItRuntime: Sigma-DWH takes 5, 6, 6 steps and the scaled Newton iteration 7, 9, 9
    at kappa = 1e2, 1e8, 1e12.  The oracle's schedules (r = 1 steps until the l-recurrence
    reaches 1 - 1e-15 plus the step of the stopping test; Newton with the Byers-Xu
    scaling until the modulus interval reaches [1, 1 + 1e-15] plus one) give those counts."""
    from oracle import iterations as it
    g = GOLDEN["table1_iterations"]
    for kappa, d, nw in zip(g["kappa"], g["sigma_dwh_ldliqr2"], g["newton"]):
        assert len(it.dwh_schedule(1.0 / kappa)) == d
        assert len(it.newton_schedule(1.0 / kappa)) == nw


def test_newton_scaling_scalar_map():
    """The scaled Newton map x -> (mu x + 1/(mu x))/2 with the schedule's scalings takes
    every modulus in [l, 1] into [1, 1 + 1e-15] (evaluated in multiprecision)."""
    from oracle import iterations as it
    for ell in (1e-1, 1e-4, 1e-10):
        mus = it.newton_schedule(ell)
        with mp.workdps(50):
            xs = [mp.mpf(ell) * (mp.mpf(1) / ell) ** (mp.mpf(k) / 20) for k in range(21)]
            for mu in mus:
                xs = [(mu * x + 1 / (mu * x)) / 2 for x in xs]
            assert max(abs(x - 1) for x in xs) <= mp.mpf("2e-15")
