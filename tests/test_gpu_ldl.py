"""GPU parity of the Alg. 7 bases (opts.basis = PS_BASIS_LDL: truncated LDL^T of Sigma P_+
with 1x1 pivots and diagonal pivoting) against the oracle's same factorization
(``oracle.bases.alg7_pivoted_bases``) applied to the oracle's sign(H).

The pivot rule (panel candidates = the largest Schur diagonals, greedy pivots among
them, ties to the lower index) fixes the basis uniquely, so Q_+ (and Q_- for a general
signature) and the decoupled blocks are compared element by element; the invariants
that hold for any valid basis (Sigma-orthonormality, the projector P_+ = Q_+ Q_+^T Sigma,
the eigenvalues of H_+) are checked as well."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bases as bs
from oracle import divide as dv
from oracle import eig as eg
from oracle import sign as sg
from paper_2203_08900_amd import api, inputs

pytestmark = pytest.mark.gpu


def rel(x, y):
    ny = np.linalg.norm(y)
    return np.linalg.norm(x - y) / (ny if ny > 0 else 1.0)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


CASES = [(1, 2, "dense"), (17, 5, "dense"), (64, 0, "dense"), (100, 1, "dense"),
         (130, 7, "casida"), (300, 11, "dense"), (420, 12, "casida")]


@pytest.mark.parametrize("m,seed,kind", CASES)
def test_ldl_divide_parity(m, seed, kind):
    """n = 2m from 2 to 840: one panel and several, ragged last panels (m = 17, 100,
    130, 300, 420 pivots), fewer rows than candidates (n < 128)."""
    print(f"[ldl divide] m={m} seed={seed} kind={kind}", flush=True)
    a, b = inputs.small_dense(m, seed) if kind == "dense" else inputs.casida_like(m, seed, rank=16)
    amax, amin = sg.abs_eig_bounds(sg.casida_matrix(a, b), sg.casida_sigma(m))
    al, be = 1.01 * amax, 0.99 * amin
    ref = dv.divide_casida(a, b, alpha=al, beta=be, basis="alg7-pivoted")
    Qp, Hp, info = api.divide(dev(a), dev(b), alpha=al, beta=be, basis="ldl")
    assert info["status"] == 0
    Qp, Hp = Qp.cpu().numpy(), Hp.cpu().numpy()
    assert rel(Qp, ref["Q_plus"]) < 1e-10
    assert rel(Hp, ref["H_plus"]) < 1e-10
    sigma = sg.casida_sigma(m)
    assert np.abs(Qp.T @ (sigma[:, None] * Qp) - np.eye(m)).max() < 1e-12
    pp = 0.5 * (np.eye(2 * m) + ref["S"])
    assert np.abs(Qp @ (Qp.T * sigma[None, :]) - pp).max() < 1e-11
    lam, _ = eg.eig_casida(a, b)
    w = np.linalg.eigvalsh(0.5 * (Hp + Hp.T))
    assert np.max(np.abs(w - lam[:m]) / lam[:m]) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ldl_matches_alg6_subspace_m1100(precision):
    """m = 1100 (n = 2200, 18 panels, padded 2240; mixed runs its FP32 shifts there): the
    Alg. 7 basis spans the Alg. 6 subspace, Q_ldl = Q_6 G with G orthogonal, and
    H_+ = G^T H_+(Alg. 6) G."""
    m = 1100
    print(f"[ldl vs alg6] m={m} {precision}", flush=True)
    a, b = inputs.casida_like(m, 9)
    A, B = dev(a), dev(b)
    Q6, H6, i6 = api.divide(A, B, precision=precision)
    Ql, Hl, il = api.divide(A, B, precision=precision, basis="ldl")
    assert i6["status"] == 0 and il["status"] == 0
    sig = torch.cat([torch.ones(m), -torch.ones(m)]).to(torch.float64).cuda()
    g = Q6.t() @ (sig[:, None] * Ql)
    eye = torch.eye(m, dtype=torch.float64, device="cuda")
    assert (g.t() @ g - eye).abs().max().item() < 1e-10
    assert (Q6 @ g - Ql).abs().max().item() < 1e-10 * Ql.abs().max().item()
    # Sigma-orthonormal to the accuracy of the sign: FP64, or the mixed sign after its
    # FP64 refinement (the same bound as for the Alg. 6 basis in mixed precision)
    orth = 1e-12 if precision == "fp64" else 1e-11
    assert (Ql.t() @ (sig[:, None] * Ql) - eye).abs().max().item() < orth
    assert (g.t() @ H6 @ g - Hl).abs().max().item() < 1e-10 * Hl.abs().max().item()


# kappa up to 1e6: beyond cond(M) ~ 1e7 the Cholesky form of the first Zolotarev step
# limits the sign itself (and any basis built from it); the oracle's pins cover Alg. 7
# with an exact sign at kappa = 1e8
GCASES = [(5, 3, 10.0), (120, 0, 1e6), (250, 4, 10.0), (250, 2, 1e6), (700, 6, 1e3)]


@pytest.mark.parametrize("n,seed,kappa", GCASES)
def test_ldl_general_parity(n, seed, kappa):
    """Any signature (Sec. 6.1 matrices): Q_+- by Alg. 7 from the GPU's sign against the
    oracle's Alg. 7 on the definition's sign, Sigma-orthonormality to the accuracy of the
    sign, and the paper's backward error bound."""
    print(f"[ldl general] n={n} seed={seed} kappa={kappa:g}", flush=True)
    h, sig = inputs.general_sigma(n, seed, kappa)
    p = int(np.sum(sig > 0))
    q = n - p
    H = dev(h)
    Qp, Qm, Hp, Hm, S, info = api.divide_general(H, sig, want_sign=True, basis="ldl")
    assert info["status"] == 0
    Qp, Qm, Hp, Hm, S = (x.cpu().numpy() for x in (Qp, Qm, Hp, Hm, S))
    s_def = sg.sign_definition(h, sig)
    qp_ref, qm_ref = bs.alg7_pivoted_bases(s_def, sig)
    hp_ref, hm_ref, _ = dv.decouple(h, sig, qp_ref, qm_ref)
    # the sign carries ~1e-13 kappa; the pivoted factors do not amplify it further
    tol = 1e-12 * kappa
    # With S^2 = I + F, Sigma P_+ = C C^T + (a residual of order F) and sigma_min(C) >= 1,
    # so C^T Sigma C - I is of the order of ||F||: the bases are Sigma-orthonormal to the
    # accuracy of the sign as an involution (which the Cholesky form of the first step
    # loses past cond(M) ~ 1e7), whatever the conditioning of leading blocks.
    f2 = np.linalg.norm(S @ S - np.eye(n), 2)
    orth = 10.0 * f2 + 1e-12
    e7 = 0.0
    if p:
        assert rel(Qp, qp_ref) < tol
        assert rel(Hp, hp_ref) < tol
        e7 = np.abs(Qp.T @ (sig[:, None] * Qp) - np.eye(p)).max()
        assert e7 < orth
    if q:
        assert rel(Qm, qm_ref) < tol
        assert rel(Hm, hm_ref) < tol
        assert np.abs(Qm.T @ (sig[:, None] * Qm) + np.eye(q)).max() < orth
    _, _, bwd = dv.decouple(h, sig, Qp, Qm)
    assert bwd < 1e-9                                       # the paper's Example 1 bound
    if kappa >= 1e6:
        Q6, _, _, _, _, i6 = api.divide_general(H, sig)
        assert i6["status"] == 0
        Q6 = Q6.cpu().numpy()
        e6 = np.abs(Q6.T @ (sig[:, None] * Q6) - np.eye(p)).max()
        print(f"[ldl general] ||S^2 - I|| {f2:.2e}  Sigma-orthonormality: "
              f"Alg. 7 {e7:.2e}, Alg. 6 {e6:.2e}", flush=True)


def test_ldl_argument_limits():
    """Alg. 7 is offered for the single divisions only, and up to padded 2m = 16384: the
    recursion and the batched call reject it before any launch, and so does a size
    beyond the limit (fake non-null pointers: nothing is read)."""
    lib = api.load()
    a, b = inputs.small_dense(8, 1)
    with pytest.raises(api.PseudosymError):
        api.eig(dev(a), dev(b), basis="ldl")
    opts = api.make_opts(basis="ldl")
    h = api._handle(0, torch.cuda.current_stream().cuda_stream)
    fake = ctypes.c_void_p(256)
    info = api.PsInfo()
    rc = lib.pseudosym_divide(h.handle, 8193, fake, 8193, fake, 8193, fake, 2 * 8193, fake, 8193,
                              ctypes.byref(opts), ctypes.byref(info))
    assert rc == -11
    m = (ctypes.c_int * 1)(8)
    ld = (ctypes.c_int * 1)(8)
    ld2 = (ctypes.c_int * 1)(16)
    ptrs = (ctypes.c_void_p * 1)(256)
    rc = lib.pseudosym_divide_batched(h.handle, 1, m, ptrs, ld, ptrs, ld, ptrs, ld2, ptrs, ld,
                                      ctypes.byref(opts), None)
    assert rc == -12
