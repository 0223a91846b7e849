"""pseudosym_divide_static: the division with no workspace, for callers that cannot
allocate device memory.  Called through the C-ABI and compared with pseudosym_divide on
the same inputs: the same kernels on a different scratch area, so the results are equal
bit for bit.  Two calls in a row, the second smaller (the static area keeps the first
call's contents); sizes beyond the area are refused with -2."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2203_08900_amd import api, inputs

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def static_divide(A, B, **kw):
    lib = api.load()
    m = A.shape[0]
    opts = api.make_opts(**kw)
    stream = torch.cuda.current_stream()
    st = api._handle(A.device.index, stream.cuda_stream)
    Qt = torch.empty((m, 2 * m), dtype=torch.float64, device=A.device)
    Hp = torch.empty((m, m), dtype=torch.float64, device=A.device)
    info = api.PsInfo()
    rc = lib.pseudosym_divide_static(st.handle, m, A.data_ptr(), m, B.data_ptr(), m,
                                     Qt.data_ptr(), 2 * m, Hp.data_ptr(), m,
                                     ctypes.byref(opts), ctypes.byref(info))
    return rc, Qt.t(), Hp.t(), info.as_dict()


@pytest.mark.parametrize("basis,precision", [("alg6", "fp64"), ("core", "fp64"), ("core", "mixed")])
def test_static_divide_matches_divide(basis, precision):
    for m, seed in ((512, 41), (200, 42)):          # the second call is smaller
        print(f"[static divide] m={m} {basis} {precision}", flush=True)
        a, b = inputs.small_dense(m, seed)
        A, B = dev(a), dev(b)
        rc, Qs, Hs, info = static_divide(A, B, basis=basis, precision=precision)
        assert rc == 0 and info["status"] == 0
        Qd, Hd, _ = api.divide(A, B, basis=basis, precision=precision)
        assert torch.equal(Qs, Qd) and torch.equal(Hs, Hd)


def test_static_divide_refuses_large_sizes():
    a, b = inputs.casida_like(1024, 3, rank=16)
    rc, _, _, _ = static_divide(dev(a), dev(b))
    assert rc == -2
