"""ctypes binding of libpseudosym.so (C-ABI in include/pseudosym.h).

Argument marshalling only: every step of the computation runs in the HIP library.
PyTorch supplies device memory (inputs, outputs, the workspace) and the stream.
Tensors are float64 on a ROCm device; symmetric m x m inputs can be passed in
either memory order.  Matrices returned by the library are column-major, which the
functions expose as transposed views of row-major tensors.

The library must have been built (``python -m paper_2203_08900_amd.build``);
loading fails loudly otherwise.  There is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpseudosym.so")

PS_PREC_FP64 = 0
PS_PREC_MIXED = 1
PS_BASIS_ALG6 = 0
PS_BASIS_CORE = 1
PS_BASIS_LDL = 2
PS_BASIS_CONGRUENT = 3
# kernel classes of info["kclass_*"] (PS_KC_* in the header)
KERNEL_CLASSES = ["chol_step_kernel<double,wide>", "chol_step_kernel<double,narrow>",
                  "chol_step_kernel<float>", "gemm_mfma_kernel<double,128x128>",
                  "gemm_mfma_kernel<double,64x64>", "gemm_mfma_kernel<float>"]

STATUS = {
    0: "ok", 1: "not definite", 2: "shift breakdown", 3: "not converged",
    4: "HIP error", 5: "no workspace", 6: "basis breakdown",
}


class PsOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("r", ctypes.c_int),
        ("max_restarts", ctypes.c_int),
        ("max_steps", ctypes.c_int),
        ("lanczos_steps", ctypes.c_int),
        ("timing", ctypes.c_int),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("mixed_kappa", ctypes.c_double),
        ("step2_series", ctypes.c_int),
        ("basis", ctypes.c_int),
        ("iteration", ctypes.c_int),
        ("refine", ctypes.c_int),
    ]


class PsGemmTune(ctypes.Structure):
    _fields_ = [("key", ctypes.c_ulonglong), ("tile", ctypes.c_int), ("ksplit", ctypes.c_int),
                ("streamk", ctypes.c_int), ("ms", ctypes.c_float), ("ms_default", ctypes.c_float),
                ("launches", ctypes.c_int)]


class PsInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("steps", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("r", ctypes.c_int),
        ("shifts_fp64", ctypes.c_int * 2),
        ("failed_step", ctypes.c_int),
        ("failed_mask", ctypes.c_int),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("ell", ctypes.c_double * 4),
        ("step_change", ctypes.c_double),
        ("sigma_est", ctypes.c_double * 2),
        ("phase_ms", ctypes.c_double * 8),
        ("step2_terms", ctypes.c_int),
        ("gemm_launches", ctypes.c_int),
        ("gemm_ms", ctypes.c_double),
        ("gemm_flops", ctypes.c_double),
        ("eig_splits", ctypes.c_int),
        ("eig_leaves", ctypes.c_int),
        ("eig_sweeps", ctypes.c_int),
        ("eig_steps", ctypes.c_int),
        ("eig_restarts", ctypes.c_int),
        ("eig_clusters", ctypes.c_int),
        ("kclass_launches", ctypes.c_int * 8),
        ("kclass_ms", ctypes.c_double * 8),
        ("kclass_flops", ctypes.c_double * 8),
        ("delta_norm_est", ctypes.c_double),
        ("bounds_rejected", ctypes.c_int),
        ("cond_est", ctypes.c_double),
    ]

    def as_dict(self):
        return {
            "status": self.status, "steps": self.steps, "restarts": self.restarts,
            "r": self.r, "shifts_fp64": list(self.shifts_fp64),
            "failed_step": self.failed_step, "failed_mask": self.failed_mask,
            "alpha": self.alpha, "beta": self.beta, "ell": list(self.ell),
            "step_change": self.step_change, "sigma_est": list(self.sigma_est),
            "phase_ms": list(self.phase_ms), "step2_terms": self.step2_terms,
            "gemm_launches": self.gemm_launches, "gemm_ms": self.gemm_ms,
            "gemm_flops": self.gemm_flops, "eig_splits": self.eig_splits,
            "eig_leaves": self.eig_leaves, "eig_sweeps": self.eig_sweeps,
            "eig_steps": self.eig_steps, "eig_restarts": self.eig_restarts,
            "eig_clusters": self.eig_clusters,
            "kclass_launches": list(self.kclass_launches),
            "kclass_ms": list(self.kclass_ms), "kclass_flops": list(self.kclass_flops),
            "delta_norm_est": self.delta_norm_est, "bounds_rejected": self.bounds_rejected,
            "cond_est": self.cond_est,
        }


EXPORTS = [
    "ps_opts_default", "ps_create", "ps_destroy", "ps_set_stream", "ps_workspace_size",
    "ps_set_workspace", "ps_workspace_size_batched", "ps_set_worker_streams",
    "ps_zolotarev_coeffs", "ps_set_graphs", "ps_set_gemm_tuning", "ps_autotune_divide",
    "pseudosym_sign", "pseudosym_divide",
    "pseudosym_divide_static", "pseudosym_divide_general", "pseudosym_eig",
    "pseudosym_divide_batched", "pseudosym_sign_fwd", "pseudosym_sign_bwd",
    "ps_sign_store_size", "pseudosym_sign_fwd_iter", "pseudosym_sign_bwd_iter",
    "pseudosym_sign_full",
    "pseudosym_sign_hermitian", "pseudosym_divide_hermitian", "pseudosym_sign_bse",
    "ps_status_string",
]

# worker streams lent to each handle (batched calls and the recursion use up to six)
N_WORKER_STREAMS = 6

_lib = None
_lock = threading.Lock()


def load():
    """Load libpseudosym.so and declare the C signatures (raises if not built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2203_08900_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, ip, dp, sz = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
        hp = ctypes.c_void_p
        lib.ps_opts_default.argtypes = [ctypes.POINTER(PsOpts)]
        lib.ps_opts_default.restype = None
        lib.ps_create.argtypes = [ctypes.POINTER(hp), vp]
        lib.ps_create.restype = ip
        lib.ps_destroy.argtypes = [hp]
        lib.ps_destroy.restype = ip
        lib.ps_set_stream.argtypes = [hp, vp]
        lib.ps_set_stream.restype = ip
        lib.ps_workspace_size.argtypes = [ip, ctypes.POINTER(PsOpts), ip]
        lib.ps_workspace_size.restype = sz
        lib.ps_set_workspace.argtypes = [hp, vp, sz]
        lib.ps_set_workspace.restype = ip
        lib.ps_workspace_size_batched.argtypes = [ip, ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(PsOpts)]
        lib.ps_workspace_size_batched.restype = sz
        lib.ps_set_worker_streams.argtypes = [hp, ip, ctypes.POINTER(ctypes.c_void_p)]
        lib.ps_set_worker_streams.restype = ip
        lib.ps_zolotarev_coeffs.argtypes = [ctypes.c_double, ip, dp, dp, dp, dp]
        lib.ps_zolotarev_coeffs.restype = ip
        lib.ps_set_graphs.argtypes = [hp, ip]
        lib.ps_set_graphs.restype = ip
        lib.ps_set_gemm_tuning.argtypes = [hp, ctypes.POINTER(PsGemmTune), ip]
        lib.ps_set_gemm_tuning.restype = ip
        mat = [hp, ip, vp, ip, vp, ip]
        lib.ps_autotune_divide.argtypes = mat + [ctypes.POINTER(PsOpts), ctypes.POINTER(PsGemmTune),
                                                 ip, ctypes.POINTER(ctypes.c_int)]
        lib.ps_autotune_divide.restype = ip
        lib.pseudosym_sign.argtypes = mat + [vp, vp, ip, ctypes.POINTER(PsOpts), ctypes.POINTER(PsInfo)]
        lib.pseudosym_sign.restype = ip
        lib.pseudosym_divide.argtypes = mat + [vp, ip, vp, ip, ctypes.POINTER(PsOpts),
                                               ctypes.POINTER(PsInfo)]
        lib.pseudosym_divide.restype = ip
        lib.pseudosym_divide_static.argtypes = mat + [vp, ip, vp, ip, ctypes.POINTER(PsOpts),
                                                      ctypes.POINTER(PsInfo)]
        lib.pseudosym_divide_static.restype = ip
        for name in ("pseudosym_sign_hermitian", "pseudosym_sign_bse"):
            fn = getattr(lib, name)
            fn.argtypes = mat + [vp, vp, ip, ctypes.POINTER(PsOpts), ctypes.POINTER(PsInfo)]
            fn.restype = ip
        lib.pseudosym_divide_hermitian.argtypes = mat + [vp, ip, vp, ip, ctypes.POINTER(PsOpts),
                                                         ctypes.POINTER(PsInfo)]
        lib.pseudosym_divide_hermitian.restype = ip
        lib.pseudosym_divide_general.argtypes = [hp, ip, vp, ip, ctypes.POINTER(ctypes.c_double),
                                                 vp, ip, vp, ip, vp, ip, vp, ip, vp, ip,
                                                 ctypes.POINTER(PsOpts), ctypes.POINTER(PsInfo)]
        lib.pseudosym_divide_general.restype = ip
        lib.pseudosym_eig.argtypes = mat + [vp, vp, ip, ctypes.POINTER(PsOpts),
                                            ctypes.POINTER(PsInfo)]
        lib.pseudosym_eig.restype = ip
        iarr = ctypes.POINTER(ctypes.c_int)
        parr = ctypes.POINTER(ctypes.c_void_p)
        lib.pseudosym_divide_batched.argtypes = [hp, ip, iarr, parr, iarr, parr, iarr, parr, iarr,
                                                 parr, iarr, ctypes.POINTER(PsOpts),
                                                 ctypes.POINTER(PsInfo)]
        lib.pseudosym_divide_batched.restype = ip
        lib.pseudosym_sign_fwd.argtypes = mat + [vp, vp, ip, vp, vp, ip, ctypes.POINTER(PsOpts),
                                                 ctypes.POINTER(PsInfo)]
        lib.pseudosym_sign_fwd.restype = ip
        lib.pseudosym_sign_bwd.argtypes = [hp, ip, vp, vp, ip, vp, vp, ip, vp, vp, ip]
        lib.pseudosym_sign_bwd.restype = ip
        lib.pseudosym_sign_full.argtypes = [hp, ip, vp, vp, ip, vp, ip]
        lib.pseudosym_sign_full.restype = ip
        lib.ps_sign_store_size.argtypes = [ip, ctypes.POINTER(PsOpts)]
        lib.ps_sign_store_size.restype = sz
        lib.pseudosym_sign_fwd_iter.argtypes = mat + [vp, vp, ip, vp, sz, ctypes.POINTER(PsOpts),
                                                      ctypes.POINTER(PsInfo)]
        lib.pseudosym_sign_fwd_iter.restype = ip
        lib.pseudosym_sign_bwd_iter.argtypes = [hp, ip, vp, vp, vp, ip, vp, vp, ip]
        lib.pseudosym_sign_bwd_iter.restype = ip
        lib.ps_status_string.argtypes = [ip]
        lib.ps_status_string.restype = ctypes.c_char_p
        _lib = lib
        return lib


def zolotarev_coeffs(ell: float, r: int):
    """Host-side coefficients (no GPU needed): dict with c, a, chat, ell_next."""
    lib = load()
    c = (ctypes.c_double * 16)()
    a = (ctypes.c_double * 8)()
    chat = ctypes.c_double()
    nxt = ctypes.c_double()
    rc = lib.ps_zolotarev_coeffs(float(ell), int(r), c, a, ctypes.byref(chat), ctypes.byref(nxt))
    if rc != 0:
        raise ValueError(f"ps_zolotarev_coeffs({ell}, {r}) failed")
    return {"c": list(c[:2 * r]), "a": list(a[:r]), "chat": chat.value, "ell_next": nxt.value}


ITERATIONS = {"zolo": 0, "dwh": 1, "newton": 2}
REFINES = {"none": 0, "rr": 1, "ns": 2}


def make_opts(precision="fp64", r=8, max_restarts=2, max_steps=0, lanczos_steps=20,
              timing=False, alpha=0.0, beta=0.0, mixed_kappa=20.0,
              step2_series=True, basis="alg6", iteration="zolo", refine="rr") -> PsOpts:
    lib = load()
    o = PsOpts()
    lib.ps_opts_default(ctypes.byref(o))
    o.precision = {"fp64": PS_PREC_FP64, "mixed": PS_PREC_MIXED}[precision] \
        if isinstance(precision, str) else int(precision)
    o.r = int(r)
    o.max_restarts = int(max_restarts)
    o.max_steps = int(max_steps)
    o.lanczos_steps = int(lanczos_steps)
    o.timing = int(timing) if not isinstance(timing, bool) else (1 if timing else 0)
    o.alpha = float(alpha or 0.0)
    o.beta = float(beta or 0.0)
    o.mixed_kappa = float(mixed_kappa)
    o.step2_series = 1 if step2_series else 0
    o.basis = {"alg6": PS_BASIS_ALG6, "core": PS_BASIS_CORE, "ldl": PS_BASIS_LDL,
               "congruent": PS_BASIS_CONGRUENT}[basis] \
        if isinstance(basis, str) else int(basis)
    o.iteration = ITERATIONS[iteration] if isinstance(iteration, str) else int(iteration)
    o.refine = REFINES[refine] if isinstance(refine, str) else int(refine)
    return o


class PseudosymError(RuntimeError):
    def __init__(self, code, info=None):
        self.code = code
        self.info = info
        super().__init__(f"pseudosym status {code}: {STATUS.get(code, 'invalid argument')}")


@dataclass
class _HandleState:
    handle: ctypes.c_void_p
    workspace: object
    ws_bytes: int
    streams: list = None      # torch streams lent to the handle (kept alive here)


_handles = {}


def _torch():
    import torch
    return torch


def _handle(device, stream_ptr):
    """One library handle per (device, stream), with a torch-owned workspace."""
    key = (device, stream_ptr)
    st = _handles.get(key)
    if st is None:
        torch = _torch()
        lib = load()
        h = ctypes.c_void_p()
        rc = lib.ps_create(ctypes.byref(h), ctypes.c_void_p(stream_ptr))
        if rc != 0:
            raise PseudosymError(rc)
        # PyTorch supplies the streams of the concurrent parts (default priority)
        streams = [torch.cuda.Stream(device=device) for _ in range(N_WORKER_STREAMS)]
        arr = (ctypes.c_void_p * len(streams))(*[x.cuda_stream for x in streams])
        rc = lib.ps_set_worker_streams(h, len(streams), arr)
        if rc != 0:
            raise PseudosymError(rc)
        st = _HandleState(h, None, 0, streams)
        _handles[key] = st
    return st


def _prepare(A, B):
    torch = _torch()
    for t, name in ((A, "A"), (B, "B")):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name} must be a float64 tensor on a ROCm device")
        if t.dim() != 2 or t.shape[0] != t.shape[1]:
            raise ValueError(f"{name} must be square")
    if A.shape != B.shape or A.device != B.device:
        raise ValueError("A and B must have the same shape and device")
    return A.contiguous(), B.contiguous()


def _ensure_workspace(st, lib, m, opts, what, device, need=None):
    torch = _torch()
    if need is None:
        need = int(lib.ps_workspace_size(int(m), ctypes.byref(opts), int(what)))
    if st.ws_bytes < need:
        st.workspace = torch.empty(need + 256, dtype=torch.uint8, device=device)
        st.ws_bytes = need
        base = st.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        rc = lib.ps_set_workspace(st.handle, ctypes.c_void_p(aligned), ctypes.c_size_t(need))
        if rc != 0:
            raise PseudosymError(rc)


def _call_setup(A, B, opts, what):
    torch = _torch()
    lib = load()
    A, B = _prepare(A, B)
    m = A.shape[0]
    dev = A.device
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        st = _handle(dev.index, stream.cuda_stream)
        _ensure_workspace(st, lib, m, opts, what, dev)
    return lib, st, A, B, m


def sign(A, B, raise_on_error=True, full=False, **kw):
    """Blocks (SA, SB) of sign(H), H = [[A, B], [-B, -A]].  Returns (SA, SB, info), or with
    full=True (SA, SB, S, info) with S the whole 2m x 2m sign(H)."""
    torch = _torch()
    opts = make_opts(**kw)
    lib, st, A, B, m = _call_setup(A, B, opts, 0)
    SA = torch.empty((m, m), dtype=torch.float64, device=A.device)
    SB = torch.empty((m, m), dtype=torch.float64, device=A.device)
    info = PsInfo()
    rc = lib.pseudosym_sign(st.handle, m, A.data_ptr(), m, B.data_ptr(), m, SA.data_ptr(),
                            SB.data_ptr(), m, ctypes.byref(opts), ctypes.byref(info))
    if rc != 0 and raise_on_error:
        raise PseudosymError(rc, info.as_dict())
    # the library writes column-major; SA, SB are symmetric up to rounding, return the
    # column-major view so that entry (i, j) is the library's (i, j)
    out = info.as_dict() | {"rc": rc}
    if not full:
        return SA.t(), SB.t(), out
    St = torch.empty((2 * m, 2 * m), dtype=torch.float64, device=A.device)
    if rc == 0:
        rc2 = lib.pseudosym_sign_full(st.handle, m, SA.data_ptr(), SB.data_ptr(), m,
                                      St.data_ptr(), 2 * m)
        if rc2 != 0:
            raise PseudosymError(rc2)
    return SA.t(), SB.t(), St.t(), out


def divide(A, B, raise_on_error=True, **kw):
    """Q_+ (2m x m) and H_+ (m x m) of one spectral division step.  Returns (Qp, Hp, info)."""
    torch = _torch()
    opts = make_opts(**kw)
    lib, st, A, B, m = _call_setup(A, B, opts, 1)
    Qt = torch.empty((m, 2 * m), dtype=torch.float64, device=A.device)  # column-major 2m x m
    Hp = torch.empty((m, m), dtype=torch.float64, device=A.device)
    info = PsInfo()
    rc = lib.pseudosym_divide(st.handle, m, A.data_ptr(), m, B.data_ptr(), m, Qt.data_ptr(),
                              2 * m, Hp.data_ptr(), m, ctypes.byref(opts), ctypes.byref(info))
    if rc != 0 and raise_on_error:
        raise PseudosymError(rc, info.as_dict())
    return Qt.t(), Hp.t(), info.as_dict() | {"rc": rc}


def _complex_call(name, A, B, out_rows, raise_on_error, kw):
    """Complex blocks in, two complex outputs (out_rows x m and m x m) back, column-major
    for the library (the transposed contiguous copy of a row-major tensor)."""
    torch = _torch()
    lib = load()
    for t, nm in ((A, "A"), (B, "B")):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
            raise TypeError(f"{nm} must be a complex128 tensor on a ROCm device")
        if t.dim() != 2 or t.shape[0] != t.shape[1]:
            raise ValueError(f"{nm} must be square")
    if A.shape != B.shape or A.device != B.device:
        raise ValueError("A and B must have the same shape and device")
    m = A.shape[0]
    Ac, Bc = A.t().contiguous(), B.t().contiguous()      # column-major storage
    opts = make_opts(**kw)
    dev = A.device
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        st = _handle(dev.index, stream.cuda_stream)
        _ensure_workspace(st, lib, m, opts, 5, dev)
    O1 = torch.empty((m, out_rows), dtype=torch.complex128, device=dev)   # column-major
    O2 = torch.empty((m, m), dtype=torch.complex128, device=dev)
    info = PsInfo()
    if name == "pseudosym_divide_hermitian":
        rc = lib.pseudosym_divide_hermitian(st.handle, m, Ac.data_ptr(), m, Bc.data_ptr(), m,
                                            O1.data_ptr(), out_rows, O2.data_ptr(), m,
                                            ctypes.byref(opts), ctypes.byref(info))
    else:   # sign blocks: one leading dimension for both
        rc = getattr(lib, name)(st.handle, m, Ac.data_ptr(), m, Bc.data_ptr(), m, O1.data_ptr(),
                                O2.data_ptr(), m, ctypes.byref(opts), ctypes.byref(info))
    if rc != 0 and raise_on_error:
        raise PseudosymError(rc, info.as_dict())
    return O1.t(), O2.t(), info.as_dict() | {"rc": rc}


def sign_hermitian(A, B, raise_on_error=True, **kw):
    """Blocks (SA, SB) of sign(H), H = [[A, B], [-B, -A]] with A, B Hermitian (Eq:BSE2;
    complex128 device tensors).  Returns (SA, SB, info)."""
    return _complex_call("pseudosym_sign_hermitian", A, B, A.shape[0], raise_on_error, kw)


def divide_hermitian(A, B, raise_on_error=True, **kw):
    """Q_+ (2m x m) and H_+ (m x m) for H = [[A, B], [-B, -A]] with A, B Hermitian
    (Eq:BSE2).  Returns (Qp, Hp, info)."""
    return _complex_call("pseudosym_divide_hermitian", A, B, 2 * A.shape[0], raise_on_error, kw)


def sign_bse(A, B, raise_on_error=True, **kw):
    """Blocks (SA, SB) of sign(H), H = [[A, B], [-conj(B), -conj(A)]] with A Hermitian
    and B complex symmetric (Eq:BSE1).  Returns (SA, SB, info)."""
    return _complex_call("pseudosym_sign_bse", A, B, A.shape[0], raise_on_error, kw)


def divide_general(H, sigma, want_sign=False, raise_on_error=True, **kw):
    """One spectral division of a definite pseudosymmetric H (n x n, float64 on the device)
    for any signature sigma (n values +-1; Sigma H symmetric positive definite).
    Returns (Qp, Qm, Hp, Hm, S, info): Qp n x r_+, Qm n x r_-, Hp r_+ x r_+, Hm r_- x r_-,
    S = sign(H) (n x n) when want_sign, else None."""
    import numpy as np
    torch = _torch()
    lib = load()
    if not isinstance(H, torch.Tensor) or H.dtype != torch.float64 or not H.is_cuda:
        raise TypeError("H must be a float64 tensor on a ROCm device")
    if H.dim() != 2 or H.shape[0] != H.shape[1]:
        raise ValueError("H must be square")
    n = H.shape[0]
    sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64).reshape(-1))
    if sig.shape[0] != n:
        raise ValueError("sigma must have n entries")
    p = int(np.sum(sig > 0))
    q = n - p
    opts = make_opts(**kw)
    Hc = H.t().contiguous()            # column-major storage of H
    dev = H.device
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        st = _handle(dev.index, stream.cuda_stream)
        _ensure_workspace(st, lib, n, opts, 4, dev)
    f64 = dict(dtype=torch.float64, device=dev)
    Qpt = torch.empty((max(p, 1), n), **f64)
    Qmt = torch.empty((max(q, 1), n), **f64)
    Hpt = torch.empty((max(p, 1), max(p, 1)), **f64)
    Hmt = torch.empty((max(q, 1), max(q, 1)), **f64)
    St = torch.empty((n, n), **f64) if want_sign else None
    info = PsInfo()
    rc = lib.pseudosym_divide_general(
        st.handle, n, Hc.data_ptr(), n, sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        St.data_ptr() if St is not None else None, n, Qpt.data_ptr(), n, Qmt.data_ptr(), n,
        Hpt.data_ptr(), max(p, 1), Hmt.data_ptr(), max(q, 1), ctypes.byref(opts),
        ctypes.byref(info))
    if rc != 0 and raise_on_error:
        raise PseudosymError(rc, info.as_dict())
    return (Qpt[:p].t(), Qmt[:q].t(), Hpt[:p, :p].t(), Hmt[:q, :q].t(),
            St.t() if St is not None else None, info.as_dict() | {"rc": rc})


def eig(A, B, want_vectors=True, raise_on_error=True, **kw):
    """Eigenvalues (2m) and, optionally, eigenvectors (2m x 2m) of H.  Returns (lam, V, info)."""
    torch = _torch()
    opts = make_opts(**kw)
    lib, st, A, B, m = _call_setup(A, B, opts, 2)
    lam = torch.empty(2 * m, dtype=torch.float64, device=A.device)
    Vt = torch.empty((2 * m, 2 * m), dtype=torch.float64, device=A.device) if want_vectors else None
    info = PsInfo()
    rc = lib.pseudosym_eig(st.handle, m, A.data_ptr(), m, B.data_ptr(), m, lam.data_ptr(),
                           Vt.data_ptr() if Vt is not None else None, 2 * m,
                           ctypes.byref(opts), ctypes.byref(info))
    if rc != 0 and raise_on_error:
        raise PseudosymError(rc, info.as_dict())
    return lam, (Vt.t() if Vt is not None else None), info.as_dict() | {"rc": rc}


def divide_batched(As, Bs, raise_on_error=True, **kw):
    """pseudosym_divide for lists of independent problems (sizes may differ).
    Returns (list of Qp, list of Hp, list of info)."""
    torch = _torch()
    opts = make_opts(**kw)
    lib = load()
    pairs = [_prepare(A, B) for A, B in zip(As, Bs)]
    n = len(pairs)
    if n == 0:
        return [], [], []
    dev = pairs[0][0].device
    ms = [A.shape[0] for A, _ in pairs]
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        st = _handle(dev.index, stream.cuda_stream)
        need = int(lib.ps_workspace_size_batched(n, (ctypes.c_int * n)(*ms), ctypes.byref(opts)))
        _ensure_workspace(st, lib, 0, opts, 1, dev, need=need)
    Qts = [torch.empty((mi, 2 * mi), dtype=torch.float64, device=dev) for mi in ms]
    Hps = [torch.empty((mi, mi), dtype=torch.float64, device=dev) for mi in ms]
    I = ctypes.c_int * n
    P = ctypes.c_void_p * n
    m_arr = I(*ms)
    two_m = I(*[2 * mi for mi in ms])
    infos = (PsInfo * n)()
    rc = lib.pseudosym_divide_batched(
        st.handle, n, m_arr, P(*[A.data_ptr() for A, _ in pairs]), m_arr,
        P(*[B.data_ptr() for _, B in pairs]), m_arr, P(*[q.data_ptr() for q in Qts]), two_m,
        P(*[h.data_ptr() for h in Hps]), m_arr, ctypes.byref(opts), infos)
    if rc != 0 and raise_on_error:
        raise PseudosymError(rc)
    return ([q.t() for q in Qts], [h.t() for h in Hps],
            [infos[i].as_dict() | {"rc": rc} for i in range(n)])


def set_graphs(enable=True, device=None):
    """Capture and replay the batched pipeline's class launch sequences as HIP graphs
    (default on) or issue every launch directly; applies to the handle of the current
    stream on `device` and its workers."""
    torch = _torch()
    lib = load()
    dev = torch.device("cuda", device if device is not None else torch.cuda.current_device())
    with torch.cuda.device(dev):
        st = _handle(dev.index, torch.cuda.current_stream(dev).cuda_stream)
    rc = lib.ps_set_graphs(st.handle, 1 if enable else 0)
    if rc != 0:
        raise PseudosymError(rc)


def autotune_divide(A, B, **kw):
    """Time every distinct GEMM launch of one pseudosym_divide under each tile, split-K and
    schedule choice it can take.  Returns a list of dicts (key, tile, ksplit, streamk, ms,
    ms_default, launches); no division result."""
    opts = make_opts(**kw)
    lib, st, A, B, m = _call_setup(A, B, opts, 6)
    cap = 256
    out = (PsGemmTune * cap)()
    count = ctypes.c_int(0)
    rc = lib.ps_autotune_divide(st.handle, m, A.data_ptr(), m, B.data_ptr(), m, ctypes.byref(opts),
                                out, cap, ctypes.byref(count))
    if rc != 0:
        raise PseudosymError(rc)
    return [{"key": f"{out[i].key:016x}", "tile": out[i].tile, "ksplit": out[i].ksplit,
             "streamk": out[i].streamk, "ms": out[i].ms, "ms_default": out[i].ms_default,
             "launches": out[i].launches} for i in range(min(count.value, cap))]


def set_gemm_tuning(entries, device=None):
    """Install a GEMM tuning table (a list of dicts as autotune_divide returns, or []) on the
    handle of the current stream on `device` and its workers."""
    torch = _torch()
    lib = load()
    dev = torch.device("cuda", device if device is not None else torch.cuda.current_device())
    with torch.cuda.device(dev):
        st = _handle(dev.index, torch.cuda.current_stream(dev).cuda_stream)
    n = len(entries)
    arr = (PsGemmTune * max(n, 1))()
    for i, e in enumerate(entries):
        arr[i].key = int(e["key"], 16) if isinstance(e["key"], str) else int(e["key"])
        arr[i].tile, arr[i].ksplit, arr[i].streamk = int(e["tile"]), int(e["ksplit"]), int(e["streamk"])
    rc = lib.ps_set_gemm_tuning(st.handle, arr, n)
    if rc != 0:
        raise PseudosymError(rc)


def _colmajor(x):
    """Contiguous buffer holding x in column-major order."""
    return x.t().contiguous()


def sign_fwd(A, B, raise_on_error=True, **kw):
    """Sign blocks plus the eigen-decomposition the adjoint reuses.
    Returns (SA, SB, lam, V, info)."""
    torch = _torch()
    opts = make_opts(**kw)
    lib, st, A, B, m = _call_setup(A, B, opts, 2)
    SA = torch.empty((m, m), dtype=torch.float64, device=A.device)
    SB = torch.empty((m, m), dtype=torch.float64, device=A.device)
    lam = torch.empty(2 * m, dtype=torch.float64, device=A.device)
    Vt = torch.empty((2 * m, 2 * m), dtype=torch.float64, device=A.device)
    info = PsInfo()
    rc = lib.pseudosym_sign_fwd(st.handle, m, A.data_ptr(), m, B.data_ptr(), m, SA.data_ptr(),
                                SB.data_ptr(), m, lam.data_ptr(), Vt.data_ptr(), 2 * m,
                                ctypes.byref(opts), ctypes.byref(info))
    if rc != 0 and raise_on_error:
        raise PseudosymError(rc, info.as_dict())
    return SA.t(), SB.t(), lam, Vt.t(), info.as_dict() | {"rc": rc}


def sign_bwd(lam, V, gSA, gSB):
    """(dL/dA, dL/dB) from (dL/dSA, dL/dSB) and the forward's lam, V."""
    torch = _torch()
    lib = load()
    m = gSA.shape[0]
    dev = V.device
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        st = _handle(dev.index, stream.cuda_stream)
        need = int(lib.ps_workspace_size(int(m), None, 3))
        _ensure_workspace(st, lib, m, None, 3, dev, need=need)
    Vc = _colmajor(V.to(torch.float64))
    ga_in = _colmajor(gSA.to(torch.float64))
    gb_in = _colmajor(gSB.to(torch.float64))
    lam = lam.contiguous()
    gA = torch.empty((m, m), dtype=torch.float64, device=dev)
    gB = torch.empty((m, m), dtype=torch.float64, device=dev)
    rc = lib.pseudosym_sign_bwd(st.handle, m, lam.data_ptr(), Vc.data_ptr(), 2 * m,
                                ga_in.data_ptr(), gb_in.data_ptr(), m, gA.data_ptr(),
                                gB.data_ptr(), m)
    if rc != 0:
        raise PseudosymError(rc)
    return gA.t(), gB.t()


class SignStore:
    """Device memory holding the factors pseudosym_sign_fwd_iter keeps for the backward
    (a torch buffer and its 256-byte aligned address)."""

    def __init__(self, nbytes, device, m):
        torch = _torch()
        self.buffer = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self.ptr = (self.buffer.data_ptr() + 255) // 256 * 256
        self.nbytes = nbytes
        self.m = m


def sign_fwd_iter(A, B, raise_on_error=True, store=None, **kw):
    """Sign blocks plus the iteration's stored factors, which the adjoint reuses (FP64).
    `store`: a SignStore of an earlier call to reuse when it is large enough.
    Returns (SA, SB, store, info)."""
    torch = _torch()
    opts = make_opts(**kw)
    lib, st, A, B, m = _call_setup(A, B, opts, 0)
    need = int(lib.ps_sign_store_size(m, ctypes.byref(opts)))
    if store is None or store.nbytes < need or store.buffer.device != A.device:
        store = SignStore(need, A.device, m)
    store.m = m
    SA = torch.empty((m, m), dtype=torch.float64, device=A.device)
    SB = torch.empty((m, m), dtype=torch.float64, device=A.device)
    info = PsInfo()
    rc = lib.pseudosym_sign_fwd_iter(st.handle, m, A.data_ptr(), m, B.data_ptr(), m,
                                     SA.data_ptr(), SB.data_ptr(), m, ctypes.c_void_p(store.ptr),
                                     ctypes.c_size_t(store.nbytes), ctypes.byref(opts),
                                     ctypes.byref(info))
    if rc != 0 and raise_on_error:
        raise PseudosymError(rc, info.as_dict())
    return SA.t(), SB.t(), store, info.as_dict() | {"rc": rc}


def sign_bwd_iter(store, gSA, gSB):
    """(dL/dA, dL/dB) from (dL/dSA, dL/dSB) and the forward's stored factors."""
    torch = _torch()
    lib = load()
    m = store.m
    dev = store.buffer.device
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        st = _handle(dev.index, stream.cuda_stream)
        _ensure_workspace(st, lib, m, make_opts(), 7, dev)
    ga_in = _colmajor(gSA.to(torch.float64))
    gb_in = _colmajor(gSB.to(torch.float64))
    gA = torch.empty((m, m), dtype=torch.float64, device=dev)
    gB = torch.empty((m, m), dtype=torch.float64, device=dev)
    rc = lib.pseudosym_sign_bwd_iter(st.handle, m, ctypes.c_void_p(store.ptr), ga_in.data_ptr(),
                                     gb_in.data_ptr(), m, gA.data_ptr(), gB.data_ptr(), m)
    if rc != 0:
        raise PseudosymError(rc)
    return gA.t(), gB.t()


def _make_autograd():
    torch = _torch()

    class PseudosymSign(torch.autograd.Function):
        """(A, B) -> blocks (S_A, S_B) of sign([[A, B], [-B, -A]]), differentiable: the
        backward is the library's adjoint, which reuses the forward's eigenvectors."""

        @staticmethod
        def forward(ctx, A, B):
            SA, SB, lam, V, _ = sign_fwd(A.detach(), B.detach())
            ctx.save_for_backward(lam, V)
            return SA, SB

        @staticmethod
        def backward(ctx, gSA, gSB):
            lam, V = ctx.saved_tensors
            if gSA is None:
                gSA = torch.zeros_like(V[: V.shape[0] // 2, : V.shape[0] // 2])
            if gSB is None:
                gSB = torch.zeros_like(V[: V.shape[0] // 2, : V.shape[0] // 2])
            return sign_bwd(lam, V, gSA, gSB)

    class PseudosymSignIter(torch.autograd.Function):
        """(A, B) -> (S_A, S_B) as PseudosymSign, with the backward by reverse mode through
        the iteration on the factors its forward stored (no eigen-decomposition)."""

        @staticmethod
        def forward(ctx, A, B):
            SA, SB, store, _ = sign_fwd_iter(A.detach(), B.detach())
            ctx.store = store
            return SA, SB

        @staticmethod
        def backward(ctx, gSA, gSB):
            store = ctx.store
            m = store.m
            dev = store.buffer.device
            if gSA is None:
                gSA = torch.zeros((m, m), dtype=torch.float64, device=dev)
            if gSB is None:
                gSB = torch.zeros((m, m), dtype=torch.float64, device=dev)
            return sign_bwd_iter(store, gSA, gSB)

    return PseudosymSign, PseudosymSignIter


def __getattr__(name):
    if name in ("PseudosymSign", "PseudosymSignIter"):
        a, b = _make_autograd()
        globals()["PseudosymSign"] = a
        globals()["PseudosymSignIter"] = b
        return globals()[name]
    raise AttributeError(name)
