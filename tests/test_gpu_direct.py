"""Direct-solver mode (lsh_desc.hbs_order = 6, 8, 10): the HBS of the
order-p matrix, whose correction stencil reaches into the leaf, sibling and
proxy blocks, against the oracle's order-p compression and the dense LU.

Tolerances: block entries are table lookups (1e-13 relative); the full-rank
form is exact (dense LU to 1e-11); at tol 1e-10 with a 3-layer ring the
HBS inverse of the order-10 matrix solves the order-10 system to 1e-8
(the oracle's own figure is 1.7e-10 at 64 x 64; GPU and oracle pivots
differ within ties).
"""
import numpy as np
import pytest

from oracle import dense, hbs
import synth

pytestmark = pytest.mark.gpu


def cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("order", [6, 10])
def test_order_p_blocks_are_table_lookups(order):
    from paper_2007_12718_amd import lsh
    w = synth.small(32)
    P = lsh.Plan(w.n, w.kappa, op_order=order, leaf=8, tol=1e-8, proxy_width=3, prec="fp64", hbs_order=order)
    C = hbs.Compression(w.n, w.kappa, 8, 1e-8, 3, order=order)
    L, _ = P.ranks()
    for l in range(L):
        J, cand, U = P.level(l + 1)
        skel = cand[J]
        a = skel + np.array(C.tree.box(l + 1, 0)[:2])
        b = skel + np.array(C.tree.box(l + 1, 1)[:2])
        ref = C.gblock(a, b)
        assert np.abs(P.block(l).cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
        # the level's ID is valid for its proxy columns (plain G on the ring and
        # the corrected near-neighbour entries)
        ox, oy, sx, sy = C.tree.box(l + 1, 0)
        A = C.proxy_block(cand, hbs.proxy_ring(sx, sy, 3))
        U = U.cpu().numpy()
        assert np.linalg.norm(A - U @ A[J]) <= 10 * 1e-8 * np.linalg.norm(A)
    assert np.abs(P.block(-1).cpu().numpy() - C.Gleaf).max() <= 1e-13 * np.abs(C.Gleaf).max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_order10_full_rank_equals_dense(prec, tol):
    from paper_2007_12718_amd import lsh
    w = synth.small(32)
    sig, _ = dense.DenseSolver(w.n, w.kappa, 10, w.b).solve(w.u_inc)
    P = lsh.Plan(w.n, w.kappa, op_order=10, leaf=8, tol=0.0, proxy_width=3, prec=prec, hbs_order=10)
    F = lsh.Factor(P, cuda(w.b))
    f = dense.rhs(w.b, w.u_inc, w.kappa).reshape(1, w.n, w.n)
    assert rel(F.apply_precond(cuda(f)).cpu().numpy(), sig[0]) <= tol


@pytest.mark.parametrize("merge", ["schur", "auto"])
def test_order10_direct_solve_matches_dense_and_oracle(merge):
    from paper_2007_12718_amd import lsh
    n, kappa = 64, 2 * np.pi * 5
    b = synth.bumps(n, np.random.default_rng(10))
    uinc = synth.plane_wave(n, kappa, 0.3)[None]
    D = dense.DenseSolver(n, kappa, 10, b)
    sig, u = D.solve(uinc)
    f = dense.rhs(b, uinc, kappa).reshape(1, n, n)
    P, F = lsh.build(n, kappa, cuda(b), op_order=10, leaf=8, tol=1e-10, proxy_width=3, prec="fp64",
                     merge=merge, hbs_order=10)
    q = F.apply_precond(cuda(f)).cpu().numpy()[0]
    assert rel(q, sig[0]) <= 1e-8
    M = hbs.Inverse(hbs.Compression(n, kappa, 8, 1e-10, 3, order=10), b)
    assert rel(q, M.apply(f)) <= 1e-8
    # as a preconditioner for the same order, FGMRES is done in one or two steps
    s, uu, info, rc = F.solve(cuda(uinc), tol=1e-12, maxit=10)
    assert rc == 0 and info.iterations <= 2
    assert rel(s.cpu().numpy(), sig) <= 1e-10 and rel(uu.cpu().numpy(), u) <= 1e-10


def test_stencil_wider_than_proxy_ring_is_rejected():
    from paper_2007_12718_amd import lsh
    with pytest.raises(lsh.LshError) as e:
        lsh.Plan(32, 20.0, op_order=10, leaf=8, tol=1e-10, proxy_width=2, prec="fp64", hbs_order=10)
    assert e.value.code == -1
    with pytest.raises(lsh.LshError):
        lsh.Plan(32, 20.0, op_order=10, leaf=8, tol=1e-10, proxy_width=3, prec="fp64", hbs_order=5)
