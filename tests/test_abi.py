"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-side correction weights agree with the oracle (no GPU call)."""
import os
import re

import numpy as np
import pytest

from oracle import quadrature as quad

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("lsh.h", "lsh_dev.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"^(?:int|const char\*)\s+(lsh_\w+)\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2007_12718_amd import lsh
    lib = lsh.lib()
    decl = _declared()
    assert len(decl) >= 15
    missing = [n for n in decl if not hasattr(lib, n)]
    assert not missing, missing
    assert set(lsh.EXPORTED) == decl


@pytest.mark.parametrize("order", [4, 6, 8, 10])
@pytest.mark.parametrize("kh", [0.05, 0.49, 1.3])
def test_host_weights_match_oracle(order, kh):
    from paper_2007_12718_amd import lsh
    off, tau = lsh.lsh_correction_weights(order, kh)
    ref = quad.correction_weights(order, kh)
    assert len(off) == len(ref)
    for (dx, dy), t in zip(off, tau):
        assert abs(t - ref[(int(dx), int(dy))]) <= 1e-14 * max(1.0, abs(ref[(int(dx), int(dy))]))


def test_bad_arguments_are_reported_not_raised():
    from paper_2007_12718_amd import lsh
    with pytest.raises(lsh.LshError) as e:
        lsh.lsh_correction_weights(5, 0.3)
    assert e.value.code == -1
    # the fused-apply threshold: -1 (the default) and above; a host-only call
    with pytest.raises(lsh.LshError) as e:
        lsh.apply_fused_levels(-2)
    assert e.value.code == -1
    lsh.apply_fused_levels(-1)


def test_library_sources_allocate_no_device_memory():
    """Every device buffer comes from a caller's workspace: no allocation or
    free call of the HIP runtime appears in the library's sources."""
    csrc = os.path.join(ROOT, "paper_2007_12718_amd", "csrc")
    pat = re.compile(r"\bhip(Malloc\w*|Free\w*|ExtMalloc\w*|MallocAsync|HostMalloc)\s*\(")
    hits = []
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cpp", ".hpp")):
            for i, line in enumerate(open(os.path.join(csrc, f)), 1):
                if pat.search(line):
                    hits.append(f"{f}:{i}: {line.strip()}")
    assert not hits, hits


def _desc(lsh, n, prec="fp32", merge="auto", tol=1e-4):
    return lsh.LshDesc(n=n, h=1.0 / n, x0=-0.5, y0=-0.5, kappa=2 * np.pi * n / 10.24, op_order=10, leaf=8,
                       tol=tol, proxy_width=2, hbs_prec=lsh.LSH_FP32 if prec == "fp32" else lsh.LSH_FP64,
                       merge=lsh.MERGE[merge], hbs_order=4, plan_cache=0)


def test_workspace_queries_are_host_only_and_consistent():
    import ctypes
    from paper_2007_12718_amd import lsh
    L = lsh.lib()
    prev = 0
    for n in (32, 64, 256, 1024):
        for prec in ("fp32", "fp64"):
            d = _desc(lsh, n, prec)
            p, pb, fb, fbt = (ctypes.c_size_t(0) for _ in range(4))
            assert L.lsh_plan_workspace(ctypes.byref(d), ctypes.byref(p)) == 0
            assert L.lsh_build_workspace(ctypes.byref(d), 0, ctypes.byref(pb), ctypes.byref(fb)) == 0
            assert L.lsh_build_workspace(ctypes.byref(d), lsh.LSH_FACTOR_TRANSPOSE, ctypes.byref(pb),
                                         ctypes.byref(fbt)) == 0
            assert p.value == pb.value and 0 < fb.value < fbt.value
            assert p.value % 256 == 0 and fb.value % 256 == 0
        assert p.value > prev
        prev = p.value
    d = _desc(lsh, 30)  # n / leaf not a power of two
    assert L.lsh_plan_workspace(ctypes.byref(d), ctypes.byref(p)) == lsh.LSH_ERR_INVALID_ARG


def test_full_levels_validated_and_bounded():
    """full_levels lies in [0, L); keeping the top levels whole can only
    raise the plan's bound (their ranks become their candidate counts)."""
    import ctypes
    from paper_2007_12718_amd import lsh
    L = lsh.lib()
    p0, p1 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    d = _desc(lsh, 256)  # 256 / 8 = 32 leaves a side: L = 10 levels below the root
    assert L.lsh_plan_workspace(ctypes.byref(d), ctypes.byref(p0)) == 0
    d.full_levels = 1
    assert L.lsh_plan_workspace(ctypes.byref(d), ctypes.byref(p1)) == 0
    assert p1.value >= p0.value
    for bad in (-1, 10, 11):
        d.full_levels = bad
        assert L.lsh_plan_workspace(ctypes.byref(d), ctypes.byref(p1)) == lsh.LSH_ERR_INVALID_ARG
    d.full_levels = 9
    assert L.lsh_plan_workspace(ctypes.byref(d), ctypes.byref(p1)) == 0
