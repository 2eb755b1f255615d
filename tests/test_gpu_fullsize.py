"""Full size: the fourier-1024 workload (N = 1,048,576, kappa = 200 pi, random
Fourier contrast in [-1, 0.9], order-10 operator; FP32 HBS at tol 1e-4, leaf 8,
proxy width 2, automatic merge form), built with lsh_build and solved with
lsh_solve exactly as the headline timing does.

The dense oracle cannot form or factor A at N = 2^20, so these are the checks
it can make at this size:
  * sampled rows of A x, each by the oracle's direct sum over all 2^20
    sources, and all of A x against the oracle's FFT operator;
  * the FGMRES solution solves the system: the relative residual
    ||f - A sigma|| / ||f||, with A applied by the oracle, is at most the
    GMRES tolerance 1e-10, and sampled rows of it by direct sum are each at
    most 1e-10 ||f||;
  * the HBS preconditioner M approximates A^{-1}: ||A M x - x|| / ||x|| for
    a random x, with A from the oracle.

Tolerances: the FFT operator in FP64 over a 2048 x 2048 embedding carries a
relative error of order eps log2(2048^2) ~ 5e-15 of max |y|; 1e-12 leaves a
factor 200.  The preconditioner bound is 0.1: the compression at tol 1e-4
with FP32 factors measures 3.0e-2 on a random x (GMRES converges in 7
steps); a dropped level, a wrong sibling block or a transposed factor gives
O(1).
"""
import numpy as np
import pytest

from oracle import dense, fftop
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["fp32", "fp64"])
def full(request):
    import torch
    from paper_2007_12718_amd import lsh
    w = synth.largest()
    b_d = torch.from_numpy(w.b).cuda()
    u_d = torch.from_numpy(w.u_inc).cuda()
    P, F = lsh.build(w.n, w.kappa, b_d, op_order=w.op_order, leaf=w.leaf, tol=w.tol,
                     proxy_width=w.proxy_width, prec=request.param, merge="auto")
    Koff = dense.kernel_offsets(w.n, w.kappa, w.op_order)
    op = fftop.FFTOperator(w.n, w.kappa, w.op_order)
    yield w, P, F, b_d, u_d, Koff, op
    F.close()
    P.close()


def _rows(n, count, seed):
    """Random targets plus the four corners and the centre."""
    rng = np.random.default_rng(seed)
    N = n * n
    fixed = [0, n - 1, N - n, N - 1, (n // 2) * n + n // 2]
    return np.concatenate([fixed, rng.integers(0, N, count)])


def test_full_size_operator(full):
    import torch
    w, P, F, b_d, u_d, Koff, op = full
    rng = np.random.default_rng(11)
    x = rng.standard_normal((w.n, w.n)) + 1j * rng.standard_normal((w.n, w.n))
    y = P.apply_operator(b_d, torch.from_numpy(x).cuda()).cpu().numpy().reshape(-1)
    ymax = np.max(np.abs(y))
    rows = _rows(w.n, 48, 12)
    yr = dense.apply_rows(Koff, w.b, x, w.kappa, rows)
    assert np.max(np.abs(y[rows] - yr)) <= 1e-12 * ymax
    yf = op.apply(w.b, x).reshape(-1)
    assert np.max(np.abs(y - yf)) <= 1e-12 * ymax


def test_full_size_solve_residual(full):
    w, P, F, b_d, u_d, Koff, op = full
    sig, _, info, rc = F.solve(u_d, tol=w.gmres_tol, maxit=100, want_u=False)
    assert rc == 0 and info.iterations <= 20
    s = sig.cpu().numpy().reshape(w.n, w.n)
    f = dense.rhs(w.b, w.u_inc[0], w.kappa)
    r = f - op.apply(w.b, s).reshape(-1)
    fn = np.linalg.norm(f)
    rel = np.linalg.norm(r) / fn
    print(f"fourier-1024: {info.iterations} iterations, oracle residual {rel:.3e}")
    assert rel <= w.gmres_tol
    rows = _rows(w.n, 32, 13)
    rr = f[rows] - dense.apply_rows(Koff, w.b, s, w.kappa, rows)
    assert np.max(np.abs(rr)) <= w.gmres_tol * fn


def test_full_size_preconditioner(full):
    import torch
    w, P, F, b_d, u_d, Koff, op = full
    rng = np.random.default_rng(14)
    x = rng.standard_normal((w.n, w.n)) + 1j * rng.standard_normal((w.n, w.n))
    z = F.apply_precond(torch.from_numpy(x).cuda()).cpu().numpy()
    e = np.linalg.norm(op.apply(w.b, z).reshape(-1) - x.reshape(-1)) / np.linalg.norm(x)
    print(f"fourier-1024: ||A M x - x|| / ||x|| = {e:.3e}")
    assert e <= 0.1
