"""Host-side checks of libtem: the library loads, exports every entry point
declared in include/tem.h, and its C++ symbolic phase reproduces the
oracle's nested-dissection ordering and supernodal row sets bit for bit."""
import os
import re

import numpy as np
import pytest

from oracle.fem import HexMesh
from oracle.ordering import analyse, factor_flops, nnz_L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tem.h")).read()
    return sorted(set(re.findall(r"\b(tem_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2605_19951_amd import tem
    L = tem.load_library()
    names = _declared()
    assert "tem_factor_poles" in names and "tem_vjp" in names
    for n in names:
        assert hasattr(L, n), n
    assert sorted(tem.EXPORTS) == names


@pytest.mark.parametrize("dims,leaf", [((8, 8, 8), 4), ((10, 9, 7), 4), ((16, 16, 16), 4),
                                       ((18, 18, 18), 4), ((12, 6, 9), 3), ((5, 5, 5), 2),
                                       # edge cases: the smallest mesh, leaf size 1 (empty
                                       # separators), one supernode, a thin column of cells
                                       ((2, 2, 2), 4), ((2, 3, 4), 1), ((6, 6, 6), 1000),
                                       ((2, 2, 9), 2)])
def test_symbolic_bit_exact_against_oracle(dims, leaf):
    from paper_2605_19951_amd import symbolic_host
    lib = symbolic_host(*dims, leaf_max=leaf)
    mesh = HexMesh(*dims, 1.0)
    nodes, perm, iperm = analyse(mesh, leaf_max=leaf)
    assert np.array_equal(lib["perm"], perm.astype(np.int32))
    assert lib["n_supernodes"] == len(nodes)
    assert np.array_equal(lib["sn_ptr"][:-1], np.array([nd.first for nd in nodes], np.int32))
    assert lib["sn_ptr"][-1] == len(perm)
    assert np.array_equal(lib["sn_parent"], np.array([nd.parent for nd in nodes], np.int32))
    rows = np.concatenate([nd.rows for nd in nodes]).astype(np.int32)
    assert np.array_equal(lib["rows"], rows)
    sizes = np.diff(lib["rows_ptr"])
    assert np.array_equal(sizes, np.array([len(nd.rows) for nd in nodes]))
    assert lib["nnz_l"] == nnz_L(nodes)
    assert lib["flops_per_pole"] == pytest.approx(factor_flops(nodes), rel=1e-12)
    assert lib["max_front"] == max(nd.last - nd.first + len(nd.rows) for nd in nodes)


def test_symbolic_rejects_bad_sizes():
    from paper_2605_19951_amd import TemError, symbolic_host
    with pytest.raises(TemError):
        symbolic_host(1, 4, 4)
