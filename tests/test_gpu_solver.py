"""GPU parity of the hot path against the oracle (all through the C ABI).

Tolerances: FP64 kernel entries and FFT operator to 1e-13 relative; the
exact (full-rank) HBS inverse equals the dense LU solution to 1e-11 (FP64)
or 1e-5 (FP32); solves are run to a 1e-13 GMRES residual and must match the
dense LU density to 1e-9 relative (||d sigma|| <= cond(A) * res with cond(A)
up to ~1e3 here).
"""
import numpy as np
import pytest

from oracle import dense, fftop, hbs
import synth

pytestmark = pytest.mark.gpu


def cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def small():
    w = synth.small(32)
    D = dense.DenseSolver(w.n, w.kappa, 4, w.b)
    sig, u = D.solve(w.u_inc)
    return w, D, sig, u


def test_offset_table(small):
    from paper_2007_12718_amd import lsh
    from oracle import quadrature as quad
    w = small[0]
    P = lsh.Plan(w.n, w.kappa, op_order=4, leaf=8, tol=1e-10, proxy_width=3, prec="fp64")
    T = P.table().cpu().numpy()
    D = T.shape[0] - 1
    h = 1.0 / w.n
    dy, dx = np.meshgrid(np.arange(D + 1), np.arange(D + 1), indexing="ij")
    r = h * np.hypot(dx, dy)
    ref = np.empty_like(T)
    ref[r > 0] = h * h * quad.green(w.kappa, r[r > 0])
    ref[0, 0] = h * h * quad.correction_weights(4, w.kappa * h)[(0, 0)]
    err = np.abs(T - ref) / np.abs(ref)
    assert err.max() <= 1e-13, err.max()


@pytest.mark.parametrize("n,order,use_b", [(20, 10, True), (32, 6, True), (32, 8, False), (24, 4, True)])
def test_operator_matches_dense(n, order, use_b):
    from paper_2007_12718_amd import lsh
    rng = np.random.default_rng(n + order)
    kappa = 17.0
    b = rng.uniform(-1, 0.9, (n, n))
    x = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    leaf = 4 if n % 4 == 0 and (n // 4) & (n // 4 - 1) == 0 else (n if n < 12 else 3)
    if n == 20:
        leaf = 5
    P = lsh.Plan(n, kappa, op_order=order, leaf=leaf, tol=1e-4, proxy_width=2, prec="fp64")
    y = P.apply_operator(cuda(b) if use_b else None, cuda(x)).cpu().numpy()
    K = dense.dense_K(n, kappa, order)
    for r in range(2):
        ref = (dense.dense_A(b, K, kappa) @ x[r].reshape(-1)) if use_b else K @ x[r].reshape(-1)
        assert np.abs(y[r].reshape(-1) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n,leaf", [(48, 6), (96, 6), (128, 8), (192, 6), (384, 6), (512, 8), (768, 6),
                                    (1536, 6)])
def test_operator_matches_oracle_fft(n, leaf):
    """Every transform length the operator uses, 2n rounded up to a power of
    two from 128 to 4096 (sides that fill half the padded length and sides
    that do not), against the oracle's numpy FFT operator; the relative error
    bound is as for the dense check."""
    import torch
    from paper_2007_12718_amd import lsh
    rng = np.random.default_rng(n)
    kappa = 0.3 * n
    b = rng.uniform(-1, 0.9, (n, n))
    x = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    P = lsh.Plan(n, kappa, op_order=10, leaf=leaf, tol=1e-3, proxy_width=2, prec="fp32")
    try:
        y = P.apply_operator(cuda(b), cuda(x)).cpu().numpy()
        k = P.apply_operator(None, cuda(x)).cpu().numpy()
    finally:
        P.close()
    torch.cuda.empty_cache()
    op = fftop.FFTOperator(n, kappa, 10)
    yr, kr = op.apply(b, x), op.conv(x)
    assert np.abs(y - yr).max() <= 1e-13 * np.abs(yr).max()
    assert np.abs(k - kr).max() <= 1e-13 * np.abs(kr).max()


@pytest.mark.parametrize("n,tol,width,method,alpha", [(32, 1e-10, 3, "panel", 1), (64, 1e-4, 2, "panel", 1),
                                                      (128, 1e-5, 2, "panel", 1), (64, 1e-4, 2, "block", 1),
                                                      (128, 1e-5, 2, "block", 1), (64, 1e-4, 2, "block", 0.75),
                                                      (128, 1e-5, 2, "block", 0.5), (128, 1e-4, 2, "block", 0.25)])
def test_level_ids_valid_and_ranks_match_oracle(n, tol, width, method, alpha, monkeypatch):
    """The pivots are not unique (the boxes and proxy rings are symmetric, so
    column norms tie exactly).  Each level's ID must hold U[J] = I and
    approximate the proxy matrix to the tolerance, with the oracle's rank
    (+-2 for ties and for alpha-greedy pivoting).  tol 1e-10 runs the CPQR
    path, the others the Gram path: one-pivot panels ("panel") or the
    block-pivoted left-looking Cholesky ("block": alpha = 1 takes the greedy
    pivots, alpha < 1 alpha-greedy ones, several per step)."""
    from paper_2007_12718_amd import lsh
    monkeypatch.setenv("LSH_ROWID", method)
    monkeypatch.setenv("LSH_BP_ALPHA", str(alpha))
    w = synth.small(n)
    P = lsh.Plan(w.n, w.kappa, op_order=4, leaf=8, tol=tol, proxy_width=width, prec="fp64")
    C = hbs.Compression(w.n, w.kappa, 8, tol, width)
    L, ranks = P.ranks()
    assert L == C.tree.L
    assert np.array_equal(P.level(L)[1], C.cand[L])
    for l in range(L, 0, -1):
        J, cand, U = P.level(l)
        U = U.cpu().numpy()
        assert abs(len(J) - C.ranks()[l]) <= 2, (l, len(J), C.ranks()[l])
        assert np.array_equal(U[J], np.eye(len(J)))
        ox, oy, sx, sy = C.tree.box(l, 0)
        A = C.gblock(cand, hbs.proxy_ring(sx, sy, width))
        assert np.linalg.norm(A - U @ A[J]) <= 10 * tol * np.linalg.norm(A), l


def test_sibling_blocks_are_table_lookups(small):
    from paper_2007_12718_amd import lsh
    w = small[0]
    P = lsh.Plan(w.n, w.kappa, op_order=4, leaf=8, tol=1e-6, proxy_width=2, prec="fp64")
    C = hbs.Compression(w.n, w.kappa, 8, 1e-6, 2)
    L, _ = P.ranks()
    for l in range(L):
        J, cand, _ = P.level(l + 1)
        skel = cand[J]
        a = skel + np.array(C.tree.box(l + 1, 0)[:2])
        b = skel + np.array(C.tree.box(l + 1, 1)[:2])
        ref = C.gblock(a, b)
        assert np.abs(P.block(l).cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(P.block(-1).cpu().numpy() - C.Gleaf).max() <= 1e-13 * np.abs(C.Gleaf).max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_full_rank_inverse_equals_dense(small, prec, tol):
    from paper_2007_12718_amd import lsh
    w, D, sig, _ = small
    P = lsh.Plan(w.n, w.kappa, op_order=4, leaf=8, tol=0.0, proxy_width=2, prec=prec)
    F = lsh.Factor(P, cuda(w.b))
    f = dense.rhs(w.b, w.u_inc, w.kappa).reshape(1, w.n, w.n)
    q = F.apply_precond(cuda(f)).cpu().numpy()
    assert rel(q, sig[0]) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_compressed_inverse_matches_oracle(small, prec):
    """Both sides approximate (I + B G)^{-1} to the compression tolerance; the
    skeleton choice is not unique (ties), so agreement is to O(tol)."""
    from paper_2007_12718_amd import lsh
    w, D = small[0], small[1]
    tol = 1e-8
    P = lsh.Plan(w.n, w.kappa, op_order=4, leaf=8, tol=tol, proxy_width=3, prec=prec)
    M = hbs.Inverse(hbs.Compression(w.n, w.kappa, 8, tol, 3), w.b)
    F = lsh.Factor(P, cuda(w.b))
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, w.n, w.n)) + 1j * rng.standard_normal((2, w.n, w.n))
    q = F.apply_precond(cuda(x)).cpu().numpy()
    for r in range(2):
        assert rel(q[r], M.apply(x[r])) <= (1e-6 if prec == "fp64" else 2e-5)


def test_small_config_direct_and_gmres(small):
    from paper_2007_12718_amd import lsh
    w, D, sig, u = small
    P = lsh.Plan(w.n, w.kappa, op_order=4, leaf=8, tol=1e-10, proxy_width=3, prec="fp64")
    F = lsh.Factor(P, cuda(w.b))
    f = dense.rhs(w.b, w.u_inc, w.kappa).reshape(1, w.n, w.n)
    q = F.apply_precond(cuda(f)).cpu().numpy()
    assert rel(q, sig[0]) <= 1e-8          # HBS at tol 1e-10 as a direct solver
    s, uu, info, rc = F.solve(cuda(w.u_inc), tol=1e-13, maxit=20)
    assert rc == 0 and info.iterations <= 4 and info.true_residual < 1e-13
    assert rel(s.cpu().numpy(), sig) <= 1e-11
    assert rel(uu.cpu().numpy(), u) <= 1e-11


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,leaf,order", [(64, 8, 6), (48, 6, 10)])
def test_bumps_solve_matches_dense(prec, n, leaf, order):
    from paper_2007_12718_amd import lsh
    kappa = 2 * np.pi * 6
    b = synth.bumps(n, np.random.default_rng(n))
    uinc = synth.plane_wave(n, kappa)[None]
    D = dense.DenseSolver(n, kappa, order, b)
    sig, _ = D.solve(uinc)
    P = lsh.Plan(n, kappa, op_order=order, leaf=leaf, tol=1e-4, proxy_width=2, prec=prec)
    F = lsh.Factor(P, cuda(b))
    s, _, info, rc = F.solve(cuda(uinc), tol=1e-13, maxit=60)
    assert rc == 0 and info.true_residual < 1e-13
    assert info.iterations <= 15
    assert rel(s.cpu().numpy(), sig) <= 1e-9


def test_unpreconditioned_gmres_matches_dense():
    from paper_2007_12718_amd import lsh
    n, kappa = 32, 2 * np.pi * 3
    b = synth.gaussian_b(n)
    uinc = synth.plane_wave(n, kappa)[None]
    sig, _ = dense.DenseSolver(n, kappa, 8, b).solve(uinc)
    P = lsh.Plan(n, kappa, op_order=8, leaf=8, tol=1e-4, proxy_width=2, prec="fp64")
    F = lsh.Factor(P, cuda(b))
    s, _, info, rc = F.solve(cuda(uinc), tol=1e-13, maxit=150, precondition=False)
    assert rc == 0 and rel(s.cpu().numpy(), sig) <= 1e-10


def test_eval_points_matches_oracle():
    import torch
    from paper_2007_12718_amd import lsh
    n, kappa = 40, 25.0
    rng = np.random.default_rng(3)
    sig = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))
    pts = synth.receivers(16, 0.7)
    P = lsh.Plan(n, kappa, op_order=4, leaf=5, tol=1e-4, proxy_width=2, prec="fp64")
    out = P.eval_points(cuda(sig), cuda(pts)).cpu().numpy()
    E = dense.receiver_matrix(n, kappa, pts)
    ref = sig.reshape(3, -1) @ E.T
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("merge", ["auto", "lowrank"])
@pytest.mark.parametrize("prec,fl", [("fp64", 1), ("fp64", 2), ("fp32", 1)])
def test_full_top_levels_keep_candidates(small, prec, fl, merge):
    """Levels 1..full_levels keep every candidate (U = I, no row ID): their
    ranks are their candidate counts, the HBS below is compressed as usual,
    and the inverse and its transpose still match the dense ones to the
    compression tolerance (FP64 at 1e-10: to 1e-8; FP32: to 2e-5)."""
    from paper_2007_12718_amd import lsh
    w, D, sig, _ = small
    P = lsh.Plan(w.n, w.kappa, op_order=4, leaf=8, tol=1e-10, proxy_width=3, prec=prec, merge=merge,
                 full_levels=fl)
    L, r = P.ranks()
    for l in range(1, fl + 1):
        assert r[l] == 2 * r[l + 1]
    F = lsh.Factor(P, cuda(w.b), transpose=True)
    f = dense.rhs(w.b, w.u_inc, w.kappa).reshape(1, w.n, w.n)
    q = F.apply_precond(cuda(f)).cpu().numpy()
    bound = 1e-8 if prec == "fp64" else 2e-5
    assert rel(q, sig[0]) <= bound
    A = dense.dense_A(w.b, dense.dense_K(w.n, w.kappa, 4), w.kappa)
    x = np.random.default_rng(3).standard_normal((1, w.n, w.n)) + 0j
    qt = F.apply_precond(cuda(x), transpose=True).cpu().numpy()
    assert rel(qt[0], np.linalg.solve(A.T, x[0].reshape(-1)).reshape(w.n, w.n)) <= bound


@pytest.mark.parametrize("prec,fl", [("fp64", 0), ("fp32", 0), ("fp32", 1)])
def test_pipelined_build_equals_separate_calls(prec, fl):
    """lsh_build (plan and factor overlapped by level) computes exactly what
    lsh_plan_create + lsh_factor_create compute."""
    from paper_2007_12718_amd import lsh
    n, kappa = 64, 2 * np.pi * 6
    b = synth.bumps(n, np.random.default_rng(9))
    P1 = lsh.Plan(n, kappa, op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec=prec, full_levels=fl)
    F1 = lsh.Factor(P1, cuda(b))
    P2, F2 = lsh.build(n, kappa, cuda(b), op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec=prec, full_levels=fl)
    assert P1.ranks() == P2.ranks()
    x = np.random.default_rng(1).standard_normal((1, n, n)) + 0j
    assert np.array_equal(F1.apply_precond(cuda(x)).cpu().numpy(), F2.apply_precond(cuda(x)).cpu().numpy())
    s1 = F1.solve(cuda(synth.plane_wave(n, kappa)[None]), tol=1e-12)[0].cpu().numpy()
    s2 = F2.solve(cuda(synth.plane_wave(n, kappa)[None]), tol=1e-12)[0].cpu().numpy()
    assert np.array_equal(s1, s2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reused_workspaces_give_identical_factor(prec):
    """Plans and factors live in caller-owned workspaces with arbitrary
    contents: builds into workspaces full of 0xff bytes (NaN patterns), or
    reused after a build for another b, compute bit for bit what a build into
    zeroed memory computes."""
    import torch
    from paper_2007_12718_amd import lsh
    n, kappa = 64, 2 * np.pi * 6
    kw = dict(op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec=prec, transpose=True)
    b1 = synth.bumps(n, np.random.default_rng(21))
    b2 = synth.bumps(n, np.random.default_rng(22))
    x = np.random.default_rng(2).standard_normal((1, n, n)) + 0j

    def run(b, ws):
        P, F = lsh.build(n, kappa, cuda(b), workspaces=ws, **kw)
        y = F.apply_precond(cuda(x)).cpu().numpy()
        yt = F.apply_precond(cuda(x), transpose=True).cpu().numpy()
        s, _, info, rc = F.solve(cuda(synth.plane_wave(n, kappa)[None]), tol=1e-12)
        F.close()
        P.close()
        return y, yt, s.cpu().numpy()

    pw, fw = lsh.build_workspaces(n, kappa, **kw)
    r1 = run(b1, (torch.zeros_like(pw), torch.zeros_like(fw)))
    pw.fill_(255)
    fw.fill_(255)
    run(b2, (pw, fw))
    r3 = run(b1, (pw, fw))
    for a, c in zip(r1, r3):
        assert np.array_equal(a, c)


@pytest.mark.parametrize("prec,merge,fl", [("fp32", "auto", 0), ("fp64", "auto", 0), ("fp32", "lowrank", 0),
                                           ("fp64", "schur", 0), ("fp32", "auto", 1)])
def test_workspace_bounds_hold(prec, merge, fl):
    """The plan and factor use at most the workspace the queries ask for
    (the factor's exact size given the plan is within lsh_build's bound), and
    a workspace one granule short is refused with
    LSH_ERR_WORKSPACE_TOO_SMALL before any device work."""
    import ctypes
    from paper_2007_12718_amd import lsh
    n, kappa = 64, 2 * np.pi * 6
    b = synth.bumps(n, np.random.default_rng(4))
    P = lsh.Plan(n, kappa, op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec=prec, merge=merge, full_levels=fl)
    used, size = P.workspace_used()
    assert 0 < used <= size
    for tr in (False, True):
        pb, fb = lsh.build_workspaces(n, kappa, op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec=prec,
                                      merge=merge, transpose=tr, full_levels=fl)
        assert size == pb.numel()
        F = lsh.Factor(P, cuda(b), transpose=tr)
        u, z = F.workspace_used()
        assert 0 < u <= z <= fb.numel()
        if tr:
            F.apply_precond(cuda(np.ones((1, n, n), complex)), transpose=True)
            u, z = F.workspace_used()
            assert u <= z
        F.close()
    nb = ctypes.c_size_t(0)
    rc = lsh.lib().lsh_plan_workspace(ctypes.byref(P.desc), ctypes.byref(nb))
    assert rc == 0 and nb.value == size
    small = lsh.workspace(nb.value - 256)
    h = ctypes.c_void_p()
    rc = lsh.lib().lsh_plan_create(ctypes.byref(P.desc), ctypes.c_void_p(small.data_ptr()), nb.value - 256,
                                   lsh._stream(), ctypes.byref(h))
    assert rc == lsh.LSH_ERR_WORKSPACE_TOO_SMALL and not h.value
    assert b"workspace" in lsh.lib().lsh_last_error()
    P.close()


@pytest.mark.parametrize("nrhs", [1, 3])
def test_not_converged_returns_best_iterate(nrhs):
    """maxit below what the tolerance needs: LSH_NOT_CONVERGED, and sigma is
    the FGMRES iterate after maxit steps, whose true residual is reported and
    lies between the tolerance and the residual of x0 = 0."""
    from paper_2007_12718_amd import lsh
    n, kappa = 32, 2 * np.pi * 4
    b = synth.bumps(n, np.random.default_rng(5))
    U = np.stack([synth.plane_wave(n, kappa, t) for t in np.linspace(0, 2, nrhs)])
    P = lsh.Plan(n, kappa, op_order=10, leaf=8, tol=1e-4, proxy_width=2, prec="fp32")
    F = lsh.Factor(P, cuda(b))
    sig, _, info, rc = F.solve(cuda(U), tol=1e-13, maxit=2, want_u=False)
    assert rc == lsh.LSH_NOT_CONVERGED
    assert info.iterations == 2 and 1e-13 < info.true_residual < 1.0
    A = dense.dense_A(b, dense.dense_K(n, kappa, 10), kappa)
    for r in range(nrhs):
        f = dense.rhs(b, U[r], kappa)
        res = np.linalg.norm(f - A @ sig[r].cpu().numpy().reshape(-1)) / np.linalg.norm(f)
        assert 1e-13 < res < 1.0 and res <= info.true_residual * (1 + 1e-6)
    # the same factor then converges with enough iterations
    sig2, _, info2, rc2 = F.solve(cuda(U), tol=1e-12, maxit=50, want_u=False)
    assert rc2 == lsh.LSH_OK and info2.true_residual < 1e-12


def test_nonfinite_b_rejected_by_factor_and_build():
    from paper_2007_12718_amd import lsh
    n, kappa = 32, 2 * np.pi * 4
    b = synth.gaussian_b(n)
    for bad in (np.nan, np.inf):
        bb = b.copy()
        bb[7, 3] = bad
        P = lsh.Plan(n, kappa, op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec="fp32")
        with pytest.raises(lsh.LshError) as e1:
            lsh.Factor(P, cuda(bb))
        assert e1.value.code == lsh.LSH_ERR_INPUT_NONFINITE
        with pytest.raises(lsh.LshError) as e2:
            lsh.build(n, kappa, cuda(bb), op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec="fp64")
        assert e2.value.code == lsh.LSH_ERR_INPUT_NONFINITE
        # the plan is still usable after the failed factor
        F = lsh.Factor(P, cuda(b))
        sig, _, info, rc = F.solve(cuda(synth.plane_wave(n, kappa)[None]), tol=1e-10)
        assert rc == lsh.LSH_OK
