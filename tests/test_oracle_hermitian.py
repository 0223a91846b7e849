"""Pins for the oracle's complex Bethe-Salpeter forms (``oracle.hermitian``).

The two routes to sign(H) share nothing: the definite pencil (Cholesky of Sigma H and a
Hermitian eigensolver) and LAPACK's general complex eigensolver.  With real blocks the
complex functions must reduce to the real oracle's (a separate implementation).  The
structure of the sign function (an odd function keeps the block form), the projector
identities and the eigenvalues of H_+ tie the rest to the paper's statements (Sec. 5,
Thm. EVREalSigmaOrth, Thm. DefDivConq)."""
import numpy as np
import pytest

from oracle import bases as bs
from oracle import hermitian as hm
from oracle import sign as sg
from paper_2203_08900_amd import inputs


@pytest.mark.parametrize("m,seed", [(1, 0), (9, 1), (40, 2), (90, 3)])
def test_bse2_sign_two_routes_and_structure(m, seed):
    a, b = inputs.bse2_like(m, seed)
    assert np.allclose(a, a.conj().T) and np.allclose(b, b.conj().T)
    h = hm.bse2_matrix(a, b)
    sig = hm.sigma_of(m)
    s = hm.sign_pencil(h, sig)
    assert np.abs(s - hm.sign_geev(h)).max() < 1e-12
    assert np.abs(s @ s - np.eye(2 * m)).max() < 1e-12
    ss = sig[:, None] * s
    assert np.abs(ss - ss.conj().T).max() < 1e-12           # Sigma S Hermitian
    x, y = s[:m, :m], s[:m, m:]
    assert np.abs(s[m:, :m] + y).max() < 1e-12 and np.abs(s[m:, m:] + x).max() < 1e-12
    assert np.abs(x - x.conj().T).max() < 1e-12 and np.abs(y - y.conj().T).max() < 1e-12


@pytest.mark.parametrize("m,seed", [(1, 4), (9, 5), (40, 6)])
def test_bse1_sign_structure(m, seed):
    a, b = inputs.bse1_like(m, seed)
    assert np.allclose(b, b.T)
    h = hm.bse1_matrix(a, b)
    sig = hm.sigma_of(m)
    s = hm.sign_pencil(h, sig)
    assert np.abs(s - hm.sign_geev(h)).max() < 1e-12
    x, y = s[:m, :m], s[:m, m:]
    assert np.abs(s[m:, :m] + y.conj()).max() < 1e-12
    assert np.abs(s[m:, m:] + x.conj()).max() < 1e-12
    assert np.abs(x - x.conj().T).max() < 1e-12 and np.abs(y - y.T).max() < 1e-12
    lam = np.linalg.eigvals(h)
    pos = np.sort(lam.real[lam.real > 0])
    neg = np.sort(-lam.real[lam.real < 0])
    assert pos.size == m and np.abs(pos - neg).max() < 1e-12 * pos.max()   # +-lambda pairs


def test_real_blocks_reduce_to_the_real_oracle():
    a, b = inputs.small_dense(30, 7)
    m = 30
    h = hm.bse2_matrix(a.astype(complex), b.astype(complex))
    sig = hm.sigma_of(m)
    s = hm.sign_pencil(h, sig)
    s_real = sg.sign_definition(sg.casida_matrix(a, b), sg.casida_sigma(m))
    assert np.abs(s - s_real).max() < 1e-13
    assert np.abs(hm.alg6_plus(s, m) - bs.alg6_cholesky_bases_plus(s_real, m)).max() < 1e-12


@pytest.mark.parametrize("m,seed", [(9, 1), (40, 2), (120, 8)])
def test_bse2_alg6_basis_and_block(m, seed):
    a, b = inputs.bse2_like(m, seed)
    h = hm.bse2_matrix(a, b)
    sig = hm.sigma_of(m)
    s = hm.sign_pencil(h, sig)
    q = hm.alg6_plus(s, m)
    assert np.abs(q.conj().T @ (sig[:, None] * q) - np.eye(m)).max() < 1e-12
    pp = 0.5 * (np.eye(2 * m) + s)
    assert np.abs(pp @ q - q).max() < 1e-12
    top = q[:m]
    assert np.abs(np.triu(top, 1)).max() == 0.0
    assert np.all(np.abs(np.diag(top).imag) == 0.0) and np.all(np.diag(top).real > 0)
    hp = hm.decouple_plus(h, sig, q)
    assert np.abs(hp - hp.conj().T).max() < 1e-12 * np.abs(hp).max()
    w = np.linalg.eigvalsh(0.5 * (hp + hp.conj().T))
    assert np.max(np.abs(w - hm.positive_eigenvalues(h)) / w) < 1e-12
