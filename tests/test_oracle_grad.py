"""Pins of the oracle's derivatives (oracle/grad.py) against what the mathematics fixes:
central finite differences of the definitions, and the closed form of the commuting
case, where sign(H) has blocks Q diag(alpha/lambda) Q^T and Q diag(beta/lambda) Q^T
with lambda = sqrt(alpha^2 - beta^2)."""
import numpy as np
import pytest

from oracle import grad as gr
from oracle import sign as sg
from paper_2203_08900_amd import inputs


def sym(x):
    return 0.5 * (x + x.T)


def sign_blocks(a, b):
    m = a.shape[0]
    s = sg.sign_definition(sg.casida_matrix(a, b), sg.casida_sigma(m))
    return s[:m, :m], s[:m, m:]


@pytest.mark.parametrize("m,seed", [(3, 0), (6, 1), (10, 2)])
def test_projector_loss_gradient_vs_central_differences(m, seed):
    a, b = inputs.small_dense(m, seed)
    rng = np.random.default_rng(50 + seed)
    w = sym(rng.standard_normal((2 * m, 2 * m)))
    ga, gb = gr.projector_loss_grad(a, b, w)
    h = 1e-5
    for _ in range(4):
        ea = sym(rng.standard_normal((m, m)))
        eb = sym(rng.standard_normal((m, m)))
        fd = (gr.projector_loss(a + h * ea, b + h * eb, w)
              - gr.projector_loss(a - h * ea, b - h * eb, w)) / (2 * h)
        an = np.sum(ga * ea) + np.sum(gb * eb)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


@pytest.mark.parametrize("m,seed", [(4, 3), (9, 4)])
def test_sign_block_gradient_vs_central_differences(m, seed):
    a, b = inputs.small_dense(m, seed)
    rng = np.random.default_rng(70 + seed)
    g_a = rng.standard_normal((m, m))
    g_b = rng.standard_normal((m, m))
    ga, gb = gr.sign_block_grad(a, b, g_a, g_b)

    def loss(aa, bb):
        sa, sb = sign_blocks(aa, bb)
        return np.sum(g_a * sa) + np.sum(g_b * sb)

    h = 1e-5
    for _ in range(4):
        ea = sym(rng.standard_normal((m, m)))
        eb = sym(rng.standard_normal((m, m)))
        fd = (loss(a + h * ea, b + h * eb) - loss(a - h * ea, b - h * eb)) / (2 * h)
        an = np.sum(ga * ea) + np.sum(gb * eb)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_commuting_closed_form():
    m = 7
    rng = np.random.default_rng(11)
    q = inputs.haar(rng, m)
    al = rng.uniform(1.0, 3.0, m)
    be = al * rng.uniform(-0.8, 0.8, m)
    lam = np.sqrt(al ** 2 - be ** 2)
    a = sym((q * al) @ q.T)
    b = sym((q * be) @ q.T)
    p = rng.standard_normal(m)
    qq = rng.standard_normal(m)
    g_a = (q * p) @ q.T
    g_b = (q * qq) @ q.T
    ga, gb = gr.sign_block_grad(a, b, g_a, g_b)
    # L = sum p_i alpha_i / lambda_i + q_i beta_i / lambda_i along commuting directions
    dl_da = (-p * be ** 2 - qq * al * be) / lam ** 3
    dl_db = (p * al * be + qq * al ** 2) / lam ** 3
    e = rng.standard_normal(m)
    ec = (q * e) @ q.T
    assert abs(np.sum(ga * ec) - np.sum(dl_da * e)) < 1e-12 * np.abs(dl_da).sum()
    assert abs(np.sum(gb * ec) - np.sum(dl_db * e)) < 1e-12 * np.abs(dl_db).sum()


def test_gradient_is_symmetric_and_zero_for_constant_loss():
    a, b = inputs.small_dense(5, 6)
    ga, gb = gr.projector_loss_grad(a, b, np.eye(10))   # trace(P_+) = m for every H
    assert np.abs(ga).max() < 1e-12 and np.abs(gb).max() < 1e-12
    w = sym(np.random.default_rng(1).standard_normal((10, 10)))
    ga, gb = gr.projector_loss_grad(a, b, w)
    assert np.array_equal(ga, ga.T) and np.array_equal(gb, gb.T)
