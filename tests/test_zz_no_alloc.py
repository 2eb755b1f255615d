"""The allocation-free inverse (scratch in the library's static device
array) against the workspace inverse, through the C ABI: two calls in a row,
the second on a smaller problem, each bit for bit equal to lsh_dev_inverse
on the same input; and a problem whose scratch exceeds the static array is
refused before any device work."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call_static(lsh, A, info):
    prec = lsh.LSH_FP64 if A.dtype.itemsize == 16 else lsh.LSH_FP32
    b, c, _ = A.shape
    return lsh.lib().lsh_dev_inverse_static(prec, ctypes.c_void_p(A.data_ptr()), c, c, c * c, b,
                                            ctypes.c_void_p(info.data_ptr()), lsh._stream())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_scratch_inverse_equals_workspace_inverse(prec):
    import torch
    from paper_2007_12718_amd import lsh
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    rng = np.random.default_rng(5)
    # first call: the blocked path (order above the in-LDS limit), several matrices;
    # second call: smaller (the in-LDS path), fewer matrices
    for (b, c) in ((3, 300), (2, 40)):
        a = rng.standard_normal((b, c, c)) + 1j * rng.standard_normal((b, c, c)) + 4 * np.eye(c)
        A1 = torch.from_numpy(a).to(dt).cuda()
        A2 = A1.clone()
        ref, info_ref = lsh.dev_inverse(A1)
        info = torch.full((b,), -1, dtype=torch.int32, device="cuda")
        assert _call_static(lsh, A2, info) == lsh.LSH_OK
        torch.cuda.synchronize()
        assert torch.equal(A2, ref), (b, c)
        assert torch.equal(info, info_ref) and int(info.abs().sum()) == 0
        exact = np.linalg.inv(a)
        tol = 1e-11 if prec == "fp64" else 1e-4
        assert np.abs(A2.cpu().numpy() - exact).max() <= tol * np.abs(exact).max()


def test_static_scratch_inverse_rejects_oversized_problem():
    import torch
    from paper_2007_12718_amd import lsh
    c, b = 1024, 4  # FP64 blocked-path scratch of about 75 MiB > 32 MiB
    A = torch.zeros((1, 1, 1), dtype=torch.complex128, device="cuda")
    info = torch.zeros(b, dtype=torch.int32, device="cuda")
    rc = lsh.lib().lsh_dev_inverse_static(lsh.LSH_FP64, ctypes.c_void_p(A.data_ptr()), c, c, c * c, b,
                                          ctypes.c_void_p(info.data_ptr()), lsh._stream())
    assert rc == lsh.LSH_ERR_WORKSPACE_TOO_SMALL
    assert b"static scratch" in lsh.lib().lsh_last_error()
