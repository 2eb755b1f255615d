"""Plan cache (universal compression): row IDs reused across b, across
grids with the same kappa h, and through a file.  A cached ID must give
exactly the plan a cold build gives: the same pivots, U, ranks and, through
the factor, bitwise the same preconditioner.  Grids whose h differ by a
power of two scale the whole table by a power of two (h^2), which moves no
pivot and no bit of U, so those plans agree bitwise too."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _plan_arrays(P):
    L, ranks = P.ranks()
    out = [ranks]
    for l in range(1, L + 1):
        J, cand, U = P.level(l)
        out += [J, cand, U.cpu().numpy()]
    for l in range(L):
        LR = P.lowrank(l)
        out.append(None if LR is None else [t.cpu().numpy() for t in LR])
    return out


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        if isinstance(x, list):
            _same(x, y)
        elif x is None or y is None:
            assert x is None and y is None
        else:
            assert np.array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_cached_plan_equals_cold_plan(prec):
    from paper_2007_12718_amd import lsh
    lsh.plan_cache_clear()
    n, kappa = 64, 2 * np.pi * 6
    b = synth.bumps(n, np.random.default_rng(1))
    x = np.random.default_rng(2).standard_normal((1, n, n)) + 0j
    kw = dict(op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec=prec)
    P0, F0 = lsh.build(n, kappa, cuda(b), **kw)                     # cache off
    P1, F1 = lsh.build(n, kappa, cuda(b), plan_cache=True, **kw)    # fills the cache
    e1, _ = lsh.plan_cache_info()
    P2, F2 = lsh.build(n, kappa, cuda(b), plan_cache=True, **kw)    # every ID from the cache
    e2, _ = lsh.plan_cache_info()
    assert e1 > 0 and e2 == e1
    ref = _plan_arrays(P0)
    _same(_plan_arrays(P1), ref)
    _same(_plan_arrays(P2), ref)
    y0 = F0.apply_precond(cuda(x)).cpu().numpy()
    for F in (F1, F2):
        assert np.array_equal(F.apply_precond(cuda(x)).cpu().numpy(), y0)
    lsh.plan_cache_clear()
    assert lsh.plan_cache_info()[0] == 0


def test_cache_serves_a_smaller_grid_with_the_same_kappa_h():
    from paper_2007_12718_amd import lsh
    lsh.plan_cache_clear()
    kw = dict(op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec="fp32")
    lsh.Plan(128, 2 * np.pi * 12, plan_cache=True, **kw)
    e1, _ = lsh.plan_cache_info()
    P1 = lsh.Plan(64, 2 * np.pi * 6, plan_cache=True, **kw)    # same kappa h: all levels are hits
    assert lsh.plan_cache_info()[0] == e1
    P0 = lsh.Plan(64, 2 * np.pi * 6, **kw)
    _same(_plan_arrays(P1), _plan_arrays(P0))
    lsh.plan_cache_clear()


def test_cache_file_round_trip(tmp_path):
    from paper_2007_12718_amd import lsh
    lsh.plan_cache_clear()
    n, kappa = 64, 2 * np.pi * 6
    b = synth.bumps(n, np.random.default_rng(3))
    x = np.random.default_rng(4).standard_normal((1, n, n)) + 0j
    kw = dict(op_order=6, leaf=8, tol=1e-4, proxy_width=2, prec="fp32")
    P1, F1 = lsh.build(n, kappa, cuda(b), plan_cache=True, **kw)
    e1, by1 = lsh.plan_cache_info()
    path = tmp_path / "plans.lshpc"
    lsh.plan_cache_save(path)
    lsh.plan_cache_clear()
    lsh.plan_cache_load(path)
    assert lsh.plan_cache_info() == (e1, by1)
    P2, F2 = lsh.build(n, kappa, cuda(b), plan_cache=True, **kw)
    assert lsh.plan_cache_info()[0] == e1
    _same(_plan_arrays(P2), _plan_arrays(P1))
    assert np.array_equal(F1.apply_precond(cuda(x)).cpu().numpy(), F2.apply_precond(cuda(x)).cpu().numpy())
    bad = tmp_path / "bad.lshpc"
    bad.write_bytes(b"not a cache")
    with pytest.raises(lsh.LshError):
        lsh.plan_cache_load(bad)
    lsh.plan_cache_clear()
