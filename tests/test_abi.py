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
