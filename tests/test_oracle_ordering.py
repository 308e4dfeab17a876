"""Pins of the oracle's nested-dissection ordering and supernodal symbolic
structure: a hand-counted 4^3 example, bijection, separator property,
box-surface invariant, and a brute-force boolean elimination game."""
import numpy as np
import pytest

from oracle.fem import HexMesh
from oracle.ordering import analyse, cell_adjacency, nested_dissection


def test_hand_counted_4cubed_leaf2():
    # 4^3 cells, leaves of side <= 2: root splits x at 2 (24 separator
    # edges: 12 y-edges and 12 z-edges in the plane x = 2), each half splits
    # y at 2 (6 x-edges + 4 z-edges), each quarter splits z at 2 (2 x-edges
    # + 2 y-edges), and the eight 2^3 leaves hold 6 interior edges each.
    mesh = HexMesh(4, 4, 4, 1.0)
    nodes, perm = nested_dissection(mesh, leaf_max=2)
    assert len(nodes) == 15
    sizes = [len(nd.cols) for nd in nodes]
    assert sizes == [6, 6, 4, 6, 6, 4, 10, 6, 6, 4, 6, 6, 4, 10, 24]
    root = nodes[-1]
    assert root.box == ((0, 4), (0, 4), (0, 4))
    for e in root.cols:
        d, i, j, k = mesh.edge_geometry(e)
        assert d in (1, 2) and i == 2
    assert nodes[0].box == ((0, 2), (0, 2), (0, 2))
    assert nodes[6].box == ((0, 2), (0, 4), (0, 4))
    assert sorted(perm.tolist()) == list(range(108))


@pytest.mark.parametrize("n", [6, 8, 9])
def test_bijection_and_separator_property(n):
    mesh = HexMesh(n, n, n, 1.0)
    nodes, perm, iperm = analyse(mesh)
    N = len(perm)
    assert np.array_equal(np.sort(perm), np.arange(N))
    A = cell_adjacency(mesh)
    Ap = A[perm][:, perm].tocoo()
    for nd in nodes:
        if not nd.children:
            continue
        c1, c2 = (nodes[c] for c in nd.children)
        r1 = (Ap.row >= c1.sub_first) & (Ap.row < c1.last)
        r2 = (Ap.col >= c2.sub_first) & (Ap.col < c2.last)
        assert not np.any(r1 & r2)


def _surface_unknowns(mesh, box):
    (x0, x1), (y0, y1), (z0, z1) = box
    cnt = 0
    for e in mesh.unknown_edges():
        d, i, j, k = mesh.edge_geometry(e)
        lo = [i, j, k]
        hi = [i + (d == 0), j + (d == 1), k + (d == 2)]
        inside = all(b[0] <= l and u <= b[1] for l, u, b in zip(lo, hi, box))
        if not inside:
            continue
        on_face = any(lo[a] == hi[a] == box[a][0] or lo[a] == hi[a] == box[a][1] for a in range(3))
        cnt += on_face
    return cnt


def test_update_rows_are_box_surface():
    mesh = HexMesh(8, 8, 8, 1.0)
    nodes, perm, iperm = analyse(mesh)
    for nd in nodes:
        assert len(nd.rows) == _surface_unknowns(mesh, nd.box)
        # every update row is a column of an ancestor
        anc = set()
        p = nd.parent
        while p >= 0:
            anc.update(range(nodes[p].first, nodes[p].last))
            p = nodes[p].parent
        assert set(nd.rows.tolist()) <= anc


def _elimination_game(Ap):
    """Boolean Cholesky structure of the (symmetric) pattern, eliminating
    in natural order: returns the list of row sets of each column of L."""
    N = Ap.shape[0]
    B = Ap.toarray() != 0
    cols = []
    for j in range(N):
        nb = np.flatnonzero(B[j + 1:, j]) + j + 1
        cols.append(nb)
        if len(nb):
            B[np.ix_(nb, nb)] = True
    return cols


@pytest.mark.parametrize("n", [6, 8])
def test_symbolic_matches_elimination_game(n):
    mesh = HexMesh(n, n, n, 1.0)
    nodes, perm, iperm = analyse(mesh)
    A = cell_adjacency(mesh)
    Ap = A[perm][:, perm].tocsr()
    struct = _elimination_game(Ap)
    for nd in nodes:
        front = set(range(nd.first, nd.last)) | set(nd.rows.tolist())
        union = set()
        for j in range(nd.first, nd.last):
            rows = set(struct[j].tolist())
            assert rows <= front                   # struct(L) inside the front
            union |= rows
        assert union - set(range(nd.first, nd.last)) == set(nd.rows.tolist())
