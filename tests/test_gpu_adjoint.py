"""Adjoint of the sign function on the GPU (pseudosym_sign_fwd / pseudosym_sign_bwd and
the torch.autograd.Function around them) against the oracle's divided-difference
gradient (oracle/grad.py) and against central differences of the GPU forward.

Tolerances: the adjoint is four FP64 GEMMs in the eigenbasis, so against the oracle it
agrees to ~1e-12 relative (1e-10 allowed); central differences with h = 1e-5 carry a
truncation error ~h^2 and a rounding error ~1e-14 / h relative, so they are compared
to 1e-7 relative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grad as gr
from oracle import sign as sg
from paper_2203_08900_amd import api, inputs

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


def sym(x):
    return 0.5 * (x + x.T)


@pytest.mark.parametrize("m,seed", [(1, 0), (37, 1), (100, 2), (200, 5)])
def test_sign_bwd_matches_oracle(m, seed):
    print(f"[adjoint] m={m}", flush=True)
    a, b = inputs.small_dense(m, seed)
    rng = np.random.default_rng(seed + 10)
    g_a = rng.standard_normal((m, m))
    g_b = rng.standard_normal((m, m))
    SA, SB, lam, V, info = api.sign_fwd(dev(a), dev(b))
    assert info["status"] == 0
    s = sg.sign_definition(sg.casida_matrix(a, b), sg.casida_sigma(m))
    assert rel(SA.cpu().numpy(), s[:m, :m]) < 1e-12
    ga, gb = api.sign_bwd(lam, V, dev(g_a), dev(g_b))
    ra, rb = gr.sign_block_grad(a, b, g_a, g_b)
    assert rel(ga.cpu().numpy(), ra) < 1e-10 and rel(gb.cpu().numpy(), rb) < 1e-10


def _projector_loss_torch(SA, SB, W, m):
    I = torch.eye(m, dtype=torch.float64, device=SA.device)
    P = 0.5 * torch.cat([torch.cat([I + SA, SB], 1), torch.cat([-SB, I - SA], 1)], 0)
    return torch.trace(W @ P)


def test_autograd_projector_loss_small():
    m = 64
    a, b = inputs.small_dense(m, 0)
    w = sym(np.random.default_rng(3).standard_normal((2 * m, 2 * m)))
    A = dev(a).requires_grad_(True)
    B = dev(b).requires_grad_(True)
    SA, SB = api.PseudosymSign.apply(A, B)
    L = _projector_loss_torch(SA, SB, dev(w), m)
    L.backward()
    ra, rb = gr.projector_loss_grad(a, b, w)
    assert abs(L.item() - gr.projector_loss(a, b, w)) < 1e-10 * abs(L.item())
    assert rel(A.grad.cpu().numpy(), ra) < 1e-10 and rel(B.grad.cpu().numpy(), rb) < 1e-10


@pytest.mark.timeout(600)
def test_config_m1024_vs_finite_differences_and_oracle():
    """n = 2048: casida_like(1024, 3), W = symmetric Gaussian (seed 1003)."""
    m = 1024
    a, b = inputs.casida_like(m, 3)
    w = inputs.gradient_weight(m, 1003)
    W = dev(w)
    print("[adjoint] m=1024 forward/backward", flush=True)
    A = dev(a).requires_grad_(True)
    B = dev(b).requires_grad_(True)
    SA, SB = api.PseudosymSign.apply(A, B)
    L = _projector_loss_torch(SA, SB, W, m)
    L.backward()
    gA, gB = A.grad.cpu().numpy(), B.grad.cpu().numpy()
    # central differences of the GPU forward, fixed bounds so both sides run the same
    # rational iteration
    amax, amin = sg.abs_eig_bounds(sg.casida_matrix(a, b), sg.casida_sigma(m))
    al, be = 1.05 * amax, 0.95 * amin

    def loss(aa, bb):
        sa, sb, _ = api.sign(dev(aa), dev(bb), alpha=al, beta=be)
        return _projector_loss_torch(sa, sb, W, m).item()

    h = 1e-5
    rng = np.random.default_rng(2024)
    dirs = []
    for _ in range(8):
        ea = sym(rng.standard_normal((m, m)))
        eb = sym(rng.standard_normal((m, m)))
        nrm = np.sqrt(np.sum(ea ** 2) + np.sum(eb ** 2))
        dirs.append((ea / nrm, eb / nrm))
    for k in range(16):
        i, j = rng.integers(0, m, 2)
        e = np.zeros((m, m))
        e[i, j] = e[j, i] = 1.0
        dirs.append((e, np.zeros((m, m))) if k % 2 == 0 else (np.zeros((m, m)), e))
    print("[adjoint] m=1024 finite differences", flush=True)
    scale = np.sqrt(np.sum(gA ** 2) + np.sum(gB ** 2))
    for ea, eb in dirs:
        fd = (loss(a + h * ea, b + h * eb) - loss(a - h * ea, b - h * eb)) / (2 * h)
        an = np.sum(gA * ea) + np.sum(gB * eb)
        assert abs(fd - an) <= 1e-7 * scale
    print("[adjoint] m=1024 oracle gradient", flush=True)
    ra, rb = gr.projector_loss_grad(a, b, w)
    assert rel(gA, ra) < 1e-10 and rel(gB, rb) < 1e-10


# ---- the stored-factor adjoint (pseudosym_sign_fwd_iter / pseudosym_sign_bwd_iter):
# reverse mode through the forward's own composition (Cholesky of A +- B, Y0 = R_M R_K^T,
# the Zolotarev steps with their stored inverse factors, the sign-block products).  It
# differentiates the rational approximation of sign that two steps reach (error below
# 1e-15), so against the oracle's exact divided differences it agrees to rounding
# (1e-10 allowed, as for the eigenbasis adjoint).

@pytest.mark.parametrize("m,seed", [(1, 0), (37, 1), (100, 2), (200, 5)])
def test_sign_bwd_iter_matches_oracle(m, seed):
    print(f"[adjoint iter] m={m}", flush=True)
    a, b = inputs.small_dense(m, seed)
    rng = np.random.default_rng(seed + 10)
    g_a = rng.standard_normal((m, m))
    g_b = rng.standard_normal((m, m))
    SA, SB, store, info = api.sign_fwd_iter(dev(a), dev(b))
    assert info["status"] == 0 and info["step2_terms"] == 0
    s = sg.sign_definition(sg.casida_matrix(a, b), sg.casida_sigma(m))
    assert rel(SA.cpu().numpy(), s[:m, :m]) < 1e-12
    ga, gb = api.sign_bwd_iter(store, dev(g_a), dev(g_b))
    ra, rb = gr.sign_block_grad(a, b, g_a, g_b)
    assert rel(ga.cpu().numpy(), ra) < 1e-10 and rel(gb.cpu().numpy(), rb) < 1e-10


def test_sign_bwd_iter_through_a_restart():
    """An overestimated beta makes the stopping test restart: the store then holds four
    steps joined by the rescaling X0 = X2 / alpha_2, and the gradient is still the
    oracle's."""
    m = 48
    a, b = inputs.small_dense(m, 5)
    amax, amin = sg.abs_eig_bounds(sg.casida_matrix(a, b), sg.casida_sigma(m))
    rng = np.random.default_rng(7)
    g_a, g_b = rng.standard_normal((m, m)), rng.standard_normal((m, m))
    SA, SB, store, info = api.sign_fwd_iter(dev(a), dev(b), alpha=amax, beta=0.9 * amax, r=2)
    assert info["status"] == 0 and info["restarts"] >= 1 and info["steps"] >= 4
    ga, gb = api.sign_bwd_iter(store, dev(g_a), dev(g_b))
    ra, rb = gr.sign_block_grad(a, b, g_a, g_b)
    assert rel(ga.cpu().numpy(), ra) < 1e-9 and rel(gb.cpu().numpy(), rb) < 1e-9


def test_sign_iter_store_after_failed_forward():
    """A forward that fails (A + B not definite) leaves the store marked empty: the
    backward refuses it (-3) rather than use the factors of an earlier forward."""
    m = 16
    a, b = inputs.small_dense(m, 1)
    SA, SB, store, info = api.sign_fwd_iter(dev(a), dev(b))
    assert info["status"] == 0
    g = dev(np.eye(m))
    api.sign_bwd_iter(store, g, g)                     # a complete forward: accepted
    _, _, same, info2 = api.sign_fwd_iter(dev(-a), dev(b), store=store, raise_on_error=False)
    assert same is store and info2["rc"] == 1          # not definite
    with pytest.raises(api.PseudosymError) as e:
        api.sign_bwd_iter(store, g, g)
    assert e.value.code == -3


def test_sign_iter_arguments():
    a, b = inputs.small_dense(16, 1)
    with pytest.raises(api.PseudosymError) as e:
        api.sign_fwd_iter(dev(a), dev(b), precision="mixed")
    assert e.value.code == -12
    with pytest.raises(api.PseudosymError) as e:
        api.sign_fwd_iter(dev(a), dev(b), max_restarts=4)
    assert e.value.code == -12


@pytest.mark.timeout(600)
def test_autograd_iter_m1024_vs_oracle_and_eigenbasis_adjoint():
    """n = 2048 (the gradient workload): the stored-factor backward against the oracle's
    gradient and against the eigenbasis adjoint."""
    m = 1024
    a, b = inputs.casida_like(m, 3)
    w = inputs.gradient_weight(m, 1003)
    W = dev(w)
    print("[adjoint iter] m=1024", flush=True)
    grads = []
    for fn in (api.PseudosymSignIter, api.PseudosymSign):
        A = dev(a).requires_grad_(True)
        B = dev(b).requires_grad_(True)
        SA, SB = fn.apply(A, B)
        L = _projector_loss_torch(SA, SB, W, m)
        L.backward()
        grads.append((A.grad.cpu().numpy(), B.grad.cpu().numpy()))
    (ia, ib), (ea, eb) = grads
    assert rel(ia, ea) < 1e-10 and rel(ib, eb) < 1e-10
    ra, rb = gr.projector_loss_grad(a, b, w)
    assert rel(ia, ra) < 1e-10 and rel(ib, rb) < 1e-10
