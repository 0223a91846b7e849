"""GPU parity of the complex Bethe-Salpeter forms (Sec. 5: Eq:BSE2 and Eq:BSE1) against
the oracle's complex arithmetic (``oracle.hermitian``).

The library realifies the complex blocks and runs the real pipeline at half-size 2m; the
oracle never realifies: its sign(H) comes from the definite pencil in complex arithmetic,
Alg. 6 and H_+ from conjugate transposes.  Sign blocks, the Alg. 6 basis (unique: the top
block is lower triangular with a positive real diagonal) and H_+ are compared element
by element; the core basis through its unique projector."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import hermitian as hm
from paper_2203_08900_amd import api, inputs

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.complex128, device="cuda")


def host(x):
    return x.cpu().numpy()


def rel(x, y):
    return np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)


CASES = [(1, 0), (17, 1), (100, 2), (300, 3)]


@pytest.mark.parametrize("m,seed", CASES)
def test_bse2_sign_parity(m, seed):
    print(f"[bse2 sign] m={m} seed={seed}", flush=True)
    a, b = inputs.bse2_like(m, seed)
    s = hm.sign_pencil(hm.bse2_matrix(a, b), hm.sigma_of(m))
    SA, SB, info = api.sign_hermitian(dev(a), dev(b))
    assert info["status"] == 0 and info["steps"] == 2
    scale = np.abs(s).max()
    assert np.abs(host(SA) - s[:m, :m]).max() < 1e-11 * scale
    assert np.abs(host(SB) - s[:m, m:]).max() < 1e-11 * scale


@pytest.mark.parametrize("m,seed", CASES)
def test_bse2_divide_alg6_parity(m, seed):
    print(f"[bse2 divide] m={m} seed={seed}", flush=True)
    a, b = inputs.bse2_like(m, seed)
    h = hm.bse2_matrix(a, b)
    sig = hm.sigma_of(m)
    s = hm.sign_pencil(h, sig)
    q_ref = hm.alg6_plus(s, m)
    hp_ref = hm.decouple_plus(h, sig, q_ref)
    Qp, Hp, info = api.divide_hermitian(dev(a), dev(b))
    assert info["status"] == 0
    Qp, Hp = host(Qp), host(Hp)
    assert rel(Qp, q_ref) < 1e-10
    assert rel(Hp, hp_ref) < 1e-10
    assert np.abs(Qp.conj().T @ (sig[:, None] * Qp) - np.eye(m)).max() < 1e-12
    top = Qp[:m]
    assert np.abs(np.triu(top, 1)).max() == 0.0
    assert np.all(np.diag(top).real > 0) and np.abs(np.diag(top).imag).max() < 1e-12
    w = np.linalg.eigvalsh(0.5 * (Hp + Hp.conj().T))
    lam = hm.positive_eigenvalues(h)
    assert np.max(np.abs(w - lam) / lam) < 1e-12


@pytest.mark.parametrize("m,seed", [(17, 4), (300, 5)])
def test_bse2_divide_core_basis(m, seed):
    """The core basis spans the same subspace: the projector Q_+ Q_+^H Sigma = P_+."""
    print(f"[bse2 core] m={m} seed={seed}", flush=True)
    a, b = inputs.bse2_like(m, seed)
    h = hm.bse2_matrix(a, b)
    sig = hm.sigma_of(m)
    s = hm.sign_pencil(h, sig)
    Qp, Hp, info = api.divide_hermitian(dev(a), dev(b), basis="core")
    assert info["status"] == 0
    Qp, Hp = host(Qp), host(Hp)
    pp = 0.5 * (np.eye(2 * m) + s)
    assert np.abs(Qp @ (Qp.conj().T * sig[None, :]) - pp).max() < 1e-11
    assert np.abs(Qp.conj().T @ (sig[:, None] * Qp) - np.eye(m)).max() < 1e-12
    w = np.linalg.eigvalsh(0.5 * (Hp + Hp.conj().T))
    lam = hm.positive_eigenvalues(h)
    assert np.max(np.abs(w - lam) / lam) < 1e-12


@pytest.mark.parametrize("m,seed", CASES)
def test_bse1_sign_parity(m, seed):
    print(f"[bse1 sign] m={m} seed={seed}", flush=True)
    a, b = inputs.bse1_like(m, seed)
    s = hm.sign_pencil(hm.bse1_matrix(a, b), hm.sigma_of(m))
    SA, SB, info = api.sign_bse(dev(a), dev(b))
    assert info["status"] == 0
    SA, SB = host(SA), host(SB)
    scale = np.abs(s).max()
    assert np.abs(SA - s[:m, :m]).max() < 1e-11 * scale
    assert np.abs(SB - s[:m, m:]).max() < 1e-11 * scale
    assert np.abs(SB - SB.T).max() < 1e-11 * scale          # complex symmetric block


@pytest.mark.timeout(300)
def test_bse2_mixed_precision_m600():
    """Realified half-size 1200 (padded 1216 >= 1024): the mixed mode runs its FP32
    shifts, whose factorizations compute the two copies of each complex entry in
    different orders; the polar factor is projected back onto the realified form before
    the bases, so Q_+ keeps FP64 Sigma-orthonormality (without the projection: 6e-9 for
    the core basis) and the Rayleigh-Ritz eigenvalues of H_+ meet the 1e-10 target."""
    m = 600
    print("[bse2 mixed] m=600", flush=True)
    a, b = inputs.bse2_like(m, 6)
    h = hm.bse2_matrix(a, b)
    sig = hm.sigma_of(m)
    lam = hm.positive_eigenvalues(h)
    for basis in ("alg6", "core"):
        Qp, Hp, info = api.divide_hermitian(dev(a), dev(b), precision="mixed", basis=basis)
        assert info["status"] == 0 and 0 < info["shifts_fp64"][0] < info["r"]
        Qp, Hp = host(Qp), host(Hp)
        # the bounds of the real mixed division at half-size 1100
        orth = np.abs(Qp.conj().T @ (sig[:, None] * Qp) - np.eye(m)).max()
        w = np.linalg.eigvalsh(0.5 * (Hp + Hp.conj().T))
        err = np.max(np.abs(w - lam) / lam)
        print(f"[bse2 mixed] {basis}: Sigma-orthonormality {orth:.2e}, relative eigenvalue "
              f"error {err:.2e}", flush=True)
        assert orth < 1e-11
        assert err < 1e-10


def test_complex_argument_checks():
    a, b = inputs.bse2_like(8, 1)
    with pytest.raises(TypeError):
        api.sign_hermitian(torch.tensor(a.real, device="cuda"), torch.tensor(b.real, device="cuda"))
    with pytest.raises(api.PseudosymError):
        api.divide_hermitian(dev(a), dev(b), basis="ldl")
    with pytest.raises(api.PseudosymError):
        api.sign_bse(dev(a), dev(b), max_steps=1)
