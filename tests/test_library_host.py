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
