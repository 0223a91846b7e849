"""Seeded synthetic workloads for the block pseudosymmetric eigenproblem.

Every generator returns the two symmetric m x m blocks (A, B) of
H = [[A, B], [-B, -A]] (the Casida form, Sec. 5, Eq:Casida) as float64 NumPy
arrays with A + B and A - B symmetric positive definite, i.e. Sigma*H is positive
definite for Sigma = diag(I_m, -I_m) (the "definite" case of Sec. 5).

This module only builds inputs.  It holds none of the method's arithmetic and is
the one piece of code that both the GPU path and the CPU oracle consume.  The
paper's own application matrices (the LiF and N2H4 Bethe-Salpeter matrices of
Sec. 6.2) are not available; these synthetic families stand in for them with the
same block structure and definiteness.

Workload families (draw order matters for reproducibility and is fixed here):

* ``small_dense(m, seed)`` - A = Q diag(U[1,10]) Q^T with Q Haar-orthogonal,
  B = sym(Gaussian) scaled to ||B||_2 = 0.5 * lambda_min(A).  Used at m = 64
  (n = 128) and, per problem, by the batched family.
* ``casida_like(m, seed)`` - A = diag(sorted U[0.2, 5]) + a positive
  semidefinite rank-64 Gaussian coupling of spectral norm 0.05,
  B = symmetric rank-64 Gaussian with random signs scaled to
  ||B||_2 = 0.3 * lambda_min(A).  Used at m = 2048 (n = 4096) and m = 1024.
* ``batched(count, seed)`` - sizes m_i drawn uniformly from {32, ..., 512},
  problem i is ``small_dense(m_i, i)``.
* ``ill_separated(m, seed)`` - A = (M + K)/2, B = (M - K)/2 with
  M = Q_M diag(U[1,2]) Q_M^T and K = M^{-1/2} Q diag(mu) Q^T M^{-1/2},
  mu log-uniform in [1e-6, 1] with both ends pinned, so that the
  eigenvalues of (A - B)(A + B) = K M are exactly mu (spectral gap ratio 1e6).
* ``gradient_weight(m, seed)`` - a symmetric Gaussian 2m x 2m weight W.
* ``general_sigma(n, seed, kappa)`` - H = Sigma Q D Q^T with a random signature Sigma,
  Q orthonormalized from U[0, 1) entries and D equally spaced in [1, kappa]: the
  random definite pseudosymmetric matrices of the paper's experiments (Sec. 6.1).
* ``bse2_like(m, seed)`` / ``bse1_like(m, seed)`` - complex blocks of the
  Bethe-Salpeter forms (Sec. 5): A = U diag(U[1,10]) U^H with U Haar-unitary, and B
  Hermitian (Eq:BSE2) or complex symmetric (Eq:BSE1) from a complex Gaussian, scaled to
  ||B||_2 = 0.5 lambda_min(A), so that Sigma H is Hermitian positive definite.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar",
    "small_dense",
    "casida_like",
    "batched_sizes",
    "batched",
    "ill_separated",
    "gradient_weight",
    "general_sigma",
    "bse2_like",
    "bse1_like",
    "workload",
    "WORKLOADS",
]


def haar(rng: np.random.Generator, m: int) -> np.ndarray:
    """Haar-distributed orthogonal m x m matrix (QR of a Gaussian, sign-fixed)."""
    g = rng.standard_normal((m, m))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def _sym(x: np.ndarray) -> np.ndarray:
    return 0.5 * (x + x.T)


def _spec_norm_sym(x: np.ndarray) -> float:
    w = np.linalg.eigvalsh(x)
    return float(max(abs(w[0]), abs(w[-1])))


def small_dense(m: int, seed: int):
    """A = Q diag(U[1,10]) Q^T, B = sym(N(0,1)) with ||B||_2 = 0.5 lambda_min(A)."""
    rng = np.random.default_rng(seed)
    q = haar(rng, m)
    d = rng.uniform(1.0, 10.0, m)
    a = _sym((q * d[None, :]) @ q.T)
    g = rng.standard_normal((m, m))
    b = _sym(g)
    lam_min = float(np.linalg.eigvalsh(a)[0])
    b *= 0.5 * lam_min / _spec_norm_sym(b)
    return np.ascontiguousarray(a), np.ascontiguousarray(_sym(b))


def casida_like(m: int, seed: int, rank: int = 64, coupling: float = 0.05,
                b_ratio: float = 0.3):
    """Diagonal-dominant Casida-like blocks with low-rank coupling."""
    rng = np.random.default_rng(seed)
    d = np.sort(rng.uniform(0.2, 5.0, m))
    g = rng.standard_normal((m, rank))
    c = g @ g.T
    c *= coupling / _spec_norm_sym(c)
    a = _sym(np.diag(d) + c)
    g2 = rng.standard_normal((m, rank))
    s = rng.standard_normal(rank)
    b = _sym((g2 * s[None, :]) @ g2.T)
    lam_min = float(np.linalg.eigvalsh(a)[0])
    b *= b_ratio * lam_min / _spec_norm_sym(b)
    return np.ascontiguousarray(a), np.ascontiguousarray(_sym(b))


def batched_sizes(count: int = 256, seed: int = 2, lo: int = 32, hi: int = 512):
    """Uneven half-sizes m_i uniform over {lo, ..., hi} (n_i = 2 m_i)."""
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.integers(lo, hi + 1, count)]


def batched(count: int = 256, seed: int = 2):
    """List of (A_i, B_i) from ``small_dense(m_i, i)``."""
    return [small_dense(mi, i) for i, mi in enumerate(batched_sizes(count, seed))]


def _blocks_from_factors(qm, dm, q, mu):
    """A, B with A + B = M = qm diag(dm) qm^T and A - B = K = M^{-1/2} q diag(mu) q^T M^{-1/2},
    so that K M, and (A - B)(A + B), have the eigenvalues mu."""
    mmat = _sym((qm * dm[None, :]) @ qm.T)
    m_inv_half = _sym((qm * (dm ** -0.5)[None, :]) @ qm.T)
    kcore = _sym((q * mu[None, :]) @ q.T)
    k = _sym(m_inv_half @ kcore @ m_inv_half)
    a = _sym(0.5 * (mmat + k))
    b = _sym(0.5 * (mmat - k))
    return a, b


def isolated_small(m: int, seed: int, small: float = 1e-3, lo: float = 0.1, hi: float = 1.0):
    """Blocks whose H has one positive eigenvalue `small` far below the others
    (log-uniform in [lo, hi], ends pinned): a core with an isolated smallest singular
    value, the case where a lower bound beta that misses it leaves a single direction
    outside [beta, alpha].  Returns (A, B, the positive eigenvalues sorted)."""
    rng = np.random.default_rng(seed)
    qm = haar(rng, m)
    dm = rng.uniform(1.0, 2.0, m)
    lam = 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), m)
    lam[0] = small
    lam[1] = lo
    lam[-1] = hi
    q = haar(rng, m)
    a, b = _blocks_from_factors(qm, dm, q, lam ** 2)
    return np.ascontiguousarray(a), np.ascontiguousarray(b), np.sort(lam)


def ill_separated(m: int, seed: int, mu_lo: float = 1e-6, mu_hi: float = 1.0,
                  return_factors: bool = False):
    """Blocks whose (A-B)(A+B) has eigenvalues exactly mu (log-uniform, ends pinned).

    With ``return_factors`` also returns the draws the blocks are built from,
    (q_M, d_M, q, mu) in draw order (mu unsorted), for references that use the
    construction itself."""
    rng = np.random.default_rng(seed)
    qm = haar(rng, m)
    dm = rng.uniform(1.0, 2.0, m)
    mu = 10.0 ** rng.uniform(np.log10(mu_lo), np.log10(mu_hi), m)
    mu[0] = mu_lo
    mu[-1] = mu_hi
    q = haar(rng, m)
    a, b = _blocks_from_factors(qm, dm, q, mu)
    if return_factors:
        return (np.ascontiguousarray(a), np.ascontiguousarray(b), np.sort(mu),
                (qm, dm, q, mu.copy()))
    return np.ascontiguousarray(a), np.ascontiguousarray(b), np.sort(mu)


def general_sigma(n: int, seed: int, kappa: float):
    """A definite pseudosymmetric H = Sigma Q D Q^T of any signature, as in the paper's
    random experiments (Sec. 6.1): Sigma with +1 or -1 on the diagonal with equal
    probability, Q the orthogonal factor of a matrix of U[0, 1) entries, D equally
    spaced values from 1 to kappa.  Returns (H, sigma)."""
    rng = np.random.default_rng(seed)
    sigma = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    q, _ = np.linalg.qr(rng.random((n, n)))
    d = np.linspace(1.0, kappa, n)
    m = _sym((q * d[None, :]) @ q.T)
    h = sigma[:, None] * m
    return np.ascontiguousarray(h), sigma


def _complex_blocks(m: int, seed: int, hermitian_b: bool):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    q, r = np.linalg.qr(g)
    q = q * (np.diag(r) / np.abs(np.diag(r)))[None, :].conj()
    d = rng.uniform(1.0, 10.0, m)
    a = (q * d[None, :]) @ q.conj().T
    a = 0.5 * (a + a.conj().T)
    g2 = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    b = 0.5 * (g2 + (g2.conj().T if hermitian_b else g2.T))
    lam_min = float(np.linalg.eigvalsh(a)[0])
    b *= 0.5 * lam_min / float(np.linalg.norm(b, 2))
    return np.ascontiguousarray(a), np.ascontiguousarray(b)


def bse2_like(m: int, seed: int):
    """Complex Casida form (Eq:BSE2): A, B Hermitian, A +- B Hermitian positive definite."""
    return _complex_blocks(m, seed, True)


def bse1_like(m: int, seed: int):
    """Bethe-Salpeter form (Eq:BSE1): A Hermitian, B complex symmetric, with
    [[A, B], [conj(B), conj(A)]] Hermitian positive definite."""
    return _complex_blocks(m, seed, False)


def gradient_weight(m: int, seed: int) -> np.ndarray:
    """Symmetric Gaussian weight W (2m x 2m) for the loss trace(W P_+)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((2 * m, 2 * m))
    return np.ascontiguousarray(_sym(g))


# Named workloads: (description, callable returning (A, B)).
WORKLOADS = {
    "casida_n128_plain": ("m=64 Haar/U[1,10] blocks, seed 0", lambda: small_dense(64, 0)),
    "casida_n4096": ("m=2048 Casida-like blocks, seed 1", lambda: casida_like(2048, 1)),
    "casida_n2048_grad": ("m=1024 Casida-like blocks, seed 3", lambda: casida_like(1024, 3)),
    "ill_separated_n16384": ("m=8192 ill-separated blocks, seed 4",
                             lambda: ill_separated(8192, 4)[:2]),
}


def workload(name: str):
    return WORKLOADS[name][1]()
