"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, and its host-only pieces agree with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polarbp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\([^;{]*\)\s*;", src)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("polar_construct", "polar_encode", "bp_decode", "pp_mt_bp_decode",
                 "pp_mt_bp_decode_batched", "wbp_forward", "wbp_backward"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1911_08868_amd as pbp
    L = ctypes.CDLL(pbp.library_path())
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(pbp._lib.EXPORTS) == _declared()


def test_strerror():
    import paper_1911_08868_amd as pbp
    L = pbp.lib()
    assert L.polar_strerror(0) == b"success"
    assert L.polar_strerror(-1) == b"invalid argument"
    assert L.polar_strerror(-2) == b"not supported by this library"


@pytest.mark.parametrize("n,k,Q,seed", [(10, 3, 8, 0), (10, 4, 8, 7), (10, 5, 8, 123),
                                        (10, 10, 8, 5), (12, 5, 8, 9), (6, 2, 8, 1), (3, 3, 8, 4)])
def test_pool_matches_oracle(orc, n, k, Q, seed):
    import paper_1911_08868_amd as pbp
    assert np.array_equal(pbp.trellis_pool(n, k, Q, seed), orc.trellis_pool(n, k, Q, seed))


def test_pool_rejects_bad_arguments():
    import paper_1911_08868_amd as pbp
    with pytest.raises(pbp.PolarError):
        pbp.trellis_pool(10, 11, 8, 0)
    with pytest.raises(pbp.PolarError):
        pbp.trellis_pool(10, 3, 9, 0)
