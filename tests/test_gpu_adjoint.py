"""GPU parity of the adjoint path: M^T (Algorithm 2 transposed), the
transposed-HBS-preconditioned adjoint solve, the receiver adjoint and the
b-gradient, against the oracle's dense adjoint and finite differences."""
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


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_transpose_apply_dot_product(prec, tol):
    from paper_2007_12718_amd import lsh
    w = synth.small(32)
    P = lsh.Plan(w.n, w.kappa, op_order=4, leaf=8, tol=1e-4, proxy_width=2, prec=prec)
    F = lsh.Factor(P, cuda(w.b), transpose=True)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 32, 32)) + 1j * rng.standard_normal((1, 32, 32))
    y = rng.standard_normal((1, 32, 32)) + 1j * rng.standard_normal((1, 32, 32))
    My = F.apply_precond(cuda(y)).cpu().numpy()
    MTx = F.apply_precond(cuda(x), transpose=True).cpu().numpy()
    a, b = np.sum(x * My), np.sum(MTx * y)
    assert abs(a - b) <= tol * abs(a)


def test_transpose_apply_full_rank_equals_dense():
    from paper_2007_12718_amd import lsh
    w = synth.small(32)
    A = dense.dense_A(w.b, dense.dense_K(32, w.kappa, 4), w.kappa)
    P = lsh.Plan(32, w.kappa, op_order=4, leaf=8, tol=0.0, proxy_width=2, prec="fp64")
    F = lsh.Factor(P, cuda(w.b), transpose=True)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 32, 32)) + 1j * rng.standard_normal((2, 32, 32))
    q = F.apply_precond(cuda(x), transpose=True).cpu().numpy()
    for r in range(2):
        assert rel(q[r], np.linalg.solve(A.T, x[r].reshape(-1))) <= 1e-11


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_solve_matches_dense(prec):
    from paper_2007_12718_amd import lsh
    n, kappa = 48, 2 * np.pi * 6
    b = synth.bumps(n, np.random.default_rng(48))
    D = dense.DenseSolver(n, kappa, 10, b)
    rng = np.random.default_rng(5)
    g = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    ref = D.solve_adjoint(g.reshape(2, -1))
    P = lsh.Plan(n, kappa, op_order=10, leaf=6, tol=1e-4, proxy_width=2, prec=prec)
    F = lsh.Factor(P, cuda(b), transpose=True)
    lam, info, rc = F.solve_adjoint(cuda(g), tol=1e-13, maxit=60)
    assert rc == 0 and info.true_residual < 1e-13 and info.iterations <= 15
    assert rel(lam.cpu().numpy().reshape(2, -1), ref) <= 1e-9


def test_receiver_adjoint_matches_oracle():
    from paper_2007_12718_amd import lsh
    n, kappa = 40, 21.0
    pts = synth.receivers(12, 0.7)
    rng = np.random.default_rng(7)
    g = rng.standard_normal((3, 12)) + 1j * rng.standard_normal((3, 12))
    P = lsh.Plan(n, kappa, op_order=4, leaf=5, tol=1e-4, proxy_width=2, prec="fp64")
    out = P.eval_points_adjoint(cuda(g), cuda(pts)).cpu().numpy().reshape(3, -1)
    E = dense.receiver_matrix(n, kappa, pts)
    ref = g @ E.conj()
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def _problem(n=32):
    kappa = 2 * np.pi * 4
    b = 0.6 * synth.gaussian_b(n, amp=1.0, width=0.18)
    U = np.stack([synth.plane_wave(n, kappa, t) for t in (0.0, 2.1)])
    pts = synth.receivers(8, 0.7)
    tgt = np.random.default_rng(3).standard_normal((2, 8)) * 1e-2
    return n, kappa, b, U, pts, tgt


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autograd_gradient_matches_dense_adjoint(prec):
    import torch
    from paper_2007_12718_amd import lsh
    n, kappa, b, U, pts, tgt = _problem()
    Lref, gref = dense.misfit_loss_and_grad(n, kappa, 10, b, U, pts, tgt)
    P = lsh.Plan(n, kappa, op_order=10, leaf=8, tol=1e-4, proxy_width=2, prec=prec)
    bt = cuda(b).requires_grad_(True)
    ur = lsh.receiver_field(bt, cuda(U), cuda(pts), P, tol=1e-13)
    L = torch.sum(torch.abs(ur - cuda(tgt)) ** 2)
    L.backward()
    assert float(L) == pytest.approx(Lref, rel=1e-9)
    assert rel(bt.grad.cpu().numpy().ravel(), gref) <= 1e-8


def test_autograd_gradient_matches_finite_differences():
    import torch
    from paper_2007_12718_amd import lsh
    n, kappa, b, U, pts, tgt = _problem()
    P = lsh.Plan(n, kappa, op_order=10, leaf=8, tol=1e-4, proxy_width=2, prec="fp64")

    def loss(bb, grad=False):
        t = cuda(bb).requires_grad_(grad)
        ur = lsh.receiver_field(t, cuda(U), cuda(pts), P, tol=1e-14)
        L = torch.sum(torch.abs(ur - cuda(tgt)) ** 2)
        if grad:
            L.backward()
            return float(L), t.grad.cpu().numpy().ravel()
        return float(L)

    L0, g = loss(b, True)
    rng = np.random.default_rng(41)
    idx = np.argsort(-np.abs(g))[:40]
    eps = 1e-4
    for k in rng.choice(idx, 6, replace=False):
        bp, bm = b.copy().ravel(), b.copy().ravel()
        bp[k] += eps
        bm[k] -= eps
        fd = (loss(bp.reshape(n, n)) - loss(bm.reshape(n, n))) / (2 * eps)
        assert g[k] == pytest.approx(fd, rel=1e-5)
