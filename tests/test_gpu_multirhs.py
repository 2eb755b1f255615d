"""Several right-hand sides at once: the lockstep FGMRES (one preconditioner
and one operator application per iteration for a group of up to eight
right-hand sides, each with its own Krylov basis and stopping test), the
multi-vector leaf and box products behind it, and groups split at eight.

Tolerances: solves to a 1e-13 GMRES residual match the dense LU oracle to
1e-9 relative (cond(A) below ~1e3 here). A multi-column preconditioner
apply equals column-by-column applies up to the rounding of the factor's
precision (the products of a level switch from matrix-vector to MFMA
matrix-matrix kernels once the level has more than 32 box vectors).
"""
import numpy as np
import pytest

from oracle import dense
import synth

pytestmark = pytest.mark.gpu


def cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _fields(n, kappa, nr, seed):
    """Plane waves from nr directions, every third replaced by a random field
    and one all-zero right-hand side (a degenerate column)."""
    rng = np.random.default_rng(seed)
    u = np.stack([synth.plane_wave(n, kappa, 2 * np.pi * r / nr) for r in range(nr)])
    for r in range(1, nr, 3):
        u[r] = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    u[nr // 2] = 0
    return u


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nr", [3, 11])
def test_multi_rhs_solve_matches_dense(prec, nr):
    from paper_2007_12718_amd import lsh
    n, kappa = 48, 2 * np.pi * 6
    b = synth.bumps(n, np.random.default_rng(40 + nr))
    uinc = _fields(n, kappa, nr, nr)
    D = dense.DenseSolver(n, kappa, 10, b)
    sig, u = D.solve(uinc)
    P = lsh.Plan(n, kappa, op_order=10, leaf=6, tol=1e-4, proxy_width=2, prec=prec)
    F = lsh.Factor(P, cuda(b))
    s, uu, info, rc = F.solve(cuda(uinc), tol=1e-13, maxit=60)
    assert rc == 0 and info.true_residual < 1e-13
    s, uu = s.cpu().numpy(), uu.cpu().numpy()
    for r in range(nr):
        if r == nr // 2:
            assert not np.any(s[r]) and not np.any(uu[r])
            continue
        assert rel(s[r], sig[r]) <= 1e-9, r
        assert rel(uu[r], u[r]) <= 1e-9, r
    # the last column's iteration count is that of its own one-column solve
    s1, _, info1, rc1 = F.solve(cuda(uinc[-1:]), tol=1e-13, maxit=60)
    assert rc1 == 0 and abs(info.iterations - info1.iterations) <= 1
    assert rel(s[-1], s1.cpu().numpy()[0]) <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_rhs_adjoint_matches_dense(prec):
    from paper_2007_12718_amd import lsh
    n, kappa, nr = 48, 2 * np.pi * 6, 9
    b = synth.bumps(n, np.random.default_rng(7))
    rng = np.random.default_rng(8)
    g = rng.standard_normal((nr, n, n)) + 1j * rng.standard_normal((nr, n, n))
    ref = dense.DenseSolver(n, kappa, 6, b).solve_adjoint(g.reshape(nr, -1))
    P = lsh.Plan(n, kappa, op_order=6, leaf=6, tol=1e-4, proxy_width=2, prec=prec)
    F = lsh.Factor(P, cuda(b), transpose=True)
    lam, info, rc = F.solve_adjoint(cuda(g), tol=1e-13, maxit=60)
    assert rc == 0 and info.true_residual < 1e-13
    lam = lam.cpu().numpy().reshape(nr, -1)
    for r in range(nr):
        assert rel(lam[r], ref[r]) <= 1e-9, r


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
@pytest.mark.parametrize("transpose", [False, True])
def test_multi_column_apply_equals_columns(prec, tol, transpose):
    from paper_2007_12718_amd import lsh
    n, nr = 64, 6
    kappa = 2 * np.pi * 6
    b = synth.bumps(n, np.random.default_rng(3))
    P = lsh.Plan(n, kappa, op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec=prec)
    F = lsh.Factor(P, cuda(b), transpose=transpose)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((nr, n, n)) + 1j * rng.standard_normal((nr, n, n))
    y = F.apply_precond(cuda(x), transpose=transpose).cpu().numpy()
    for r in range(nr):
        y1 = F.apply_precond(cuda(x[r:r + 1]), transpose=transpose).cpu().numpy()[0]
        assert rel(y[r], y1) <= tol, r


def test_multi_rhs_unpreconditioned_matches_dense():
    from paper_2007_12718_amd import lsh
    n, kappa, nr = 32, 2 * np.pi * 3, 4
    b = synth.gaussian_b(n)
    uinc = _fields(n, kappa, nr, 1)
    sig, _ = dense.DenseSolver(n, kappa, 8, b).solve(uinc)
    P = lsh.Plan(n, kappa, op_order=8, leaf=8, tol=1e-4, proxy_width=2, prec="fp64")
    F = lsh.Factor(P, cuda(b))
    s, _, info, rc = F.solve(cuda(uinc), tol=1e-13, maxit=150, precondition=False)
    assert rc == 0
    s = s.cpu().numpy()
    for r in range(nr):
        if r != nr // 2:
            assert rel(s[r], sig[r]) <= 1e-10, r
