"""Host-side checks of the HIP library that need no GPU: it loads, exports every
entry point the C header declares, validates arguments before touching a device,
and its host-side Zolotarev coefficients (extended-precision AGM) agree with the
multiprecision oracle."""
import ctypes
import os
import re

import mpmath as mp
import pytest

from oracle import zolotarev as zol
from paper_2203_08900_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pseudosym.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\**\s+\**([a-z_]+)\s*\(", txt, flags=re.M)))


def test_library_loads_and_exports_header_symbols():
    lib = api.load()
    names = header_functions()
    assert "pseudosym_sign" in names and "pseudosym_divide" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) <= set(api.EXPORTS)


def test_argument_errors_before_any_launch():
    lib = api.load()
    o = api.make_opts()
    info = api.PsInfo()
    rc = lib.pseudosym_sign(None, 4, None, 4, None, 4, None, None, 4, ctypes.byref(o),
                            ctypes.byref(info))
    assert rc == -1                                  # null handle is argument 1
    rc = lib.pseudosym_eig(None, 4, None, 4, None, 4, None, None, 8, ctypes.byref(o),
                           ctypes.byref(info))
    assert rc == -1
    rc = lib.pseudosym_divide_batched(None, 1, None, None, None, None, None, None, None, None,
                                      None, ctypes.byref(o), None)
    assert rc == -1
    assert lib.ps_workspace_size(64, ctypes.byref(o), 2) > lib.ps_workspace_size(
        64, ctypes.byref(o), 1) > lib.ps_workspace_size(64, ctypes.byref(o), 0) > 0
    assert lib.ps_zolotarev_coeffs(0.0, 8, None, None, None, None) == -1
    assert lib.ps_zolotarev_coeffs(0.5, 9, None, None, None, None) == -1
    assert lib.ps_status_string(1).decode().startswith("not definite")


@pytest.mark.parametrize("r", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("ell", [1e-12, 1e-8, 1e-6, 1e-3, 0.04, 0.108, 0.5, 0.9, 0.999])
def test_host_coefficients_match_oracle(ell, r):
    got = api.zolotarev_coeffs(ell, r)
    ref = zol.coefficients(ell, r)
    tol = 4e-16
    for x, y in zip(got["c"], ref.c):
        assert abs(x - y) <= tol * abs(y)
    for x, y in zip(got["a"], ref.a):
        assert abs(x - y) <= tol * abs(y)
    assert abs(got["chat"] - ref.chat) <= tol * ref.chat
    assert abs(got["ell_next"] - ref.ell_next) <= 1e-15


def test_host_coefficients_tiny_ell():
    # the two-step bound of Sec. 5.2 is stated down to l = 1e-16
    got = api.zolotarev_coeffs(1e-16, 8)
    ref = zol.coefficients(1e-16, 8)
    for x, y in zip(got["c"], ref.c):
        assert abs(x - y) <= 4e-16 * abs(y)
    assert abs(got["ell_next"] - ref.ell_next) <= 4e-16 * ref.ell_next


def test_workspace_and_stream_arguments_host_only():
    """The caller owns every device buffer and stream: the batched workspace size is a
    host computation, and the stream call validates its arguments before anything else."""
    lib = api.load()
    n = 5
    ms = (ctypes.c_int * n)(40, 300, 64, 300, 7)
    o = api.make_opts()
    full = lib.ps_workspace_size_batched(n, ms, ctypes.byref(o))
    assert full > 0
    # at least one share per worker holding the largest single problem
    one = lib.ps_workspace_size(300, ctypes.byref(o), 1)
    assert full >= min(n, 6) * (one - 256)
    assert lib.ps_workspace_size_batched(0, ms, None) == 0
    assert lib.ps_workspace_size_batched(n, None, None) == 0
    bad = (ctypes.c_int * 2)(5, 0)
    assert lib.ps_workspace_size_batched(2, bad, None) == 0
    assert lib.ps_set_worker_streams(None, 0, None) == -1


def test_sign_store_and_adjoint_workspace_sizes_host_only():
    """The stored-factor adjoint's sizes are host computations: the store holds a 256-value
    header, R_M, R_K, W_M, W_K, U and per Zolotarev step its input and r factors, for
    2 (1 + max_restarts) steps; its backward's workspace is kind 7."""
    lib = api.load()
    o = api.make_opts(r=8, max_restarts=2)
    mp = 320                                          # m = 300 padded to 64
    steps = 2 * (1 + 2)
    assert lib.ps_sign_store_size(300, ctypes.byref(o)) == (256 + (5 + steps * 9) * mp * mp) * 8
    o0 = api.make_opts(r=0, max_restarts=0)           # r = 0 stores the largest r
    assert lib.ps_sign_store_size(300, ctypes.byref(o0)) == (256 + (5 + 2 * 9) * mp * mp) * 8
    assert lib.ps_sign_store_size(0, ctypes.byref(o)) == 0
    assert lib.ps_sign_store_size(300, ctypes.byref(api.make_opts(max_restarts=4))) == 0
    w7 = lib.ps_workspace_size(300, ctypes.byref(o), 7)
    assert w7 >= (13 + 2 * 8 + 8) * mp * mp * 8
    assert lib.pseudosym_sign_bwd_iter(None, 4, None, None, None, 4, None, None, 4) == -1


def _c_struct_fields(name):
    txt = open(HEADER).read()
    body = txt[:txt.index("} " + name + ";")]
    body = body[body.rindex("typedef struct {"):]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    out = []
    for decl in re.findall(r"(?:int|double)\s+([^;]+);", body):
        for part in decl.split(","):
            out.append(re.sub(r"\[.*\]", "", part).strip())
    return out


def test_binding_structs_match_the_header():
    """The ctypes mirrors of ps_opts and ps_info declare the header's fields in its order."""
    assert [n for n, _ in api.PsOpts._fields_] == _c_struct_fields("ps_opts")
    assert [n for n, _ in api.PsInfo._fields_] == _c_struct_fields("ps_info")
