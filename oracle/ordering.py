"""Nested-dissection ordering and supernodal symbolic structure (CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

All shifted matrices A_i = K - xi_i M share one sparsity pattern, so one
ordering and one symbolic structure serve every pole (section "Computational
performance": identical sparsity for all shifted systems).  The paper hands
this to MUMPS; here it is specified exactly so that two independent
implementations (this one and the library's C++ one) must agree bit for bit.

Ordering (recursive geometric nested dissection on boxes of cells
B = [x0,x1) x [y0,y1) x [z0,z1), node coordinates):
  * S(B) = unknown edges lying in the closed box but not on its surface;
  * if the longest side is <= leaf_max, B is a leaf supernode with columns
    S(B);
  * otherwise split the longest side (ties: x before y before z) at
    p = lo + (hi - lo) // 2; the separator is the set of edges lying in the
    plane at p, inside the closed box and not on its surface; the children
    are [lo, p) and [p, hi) along that axis;
  * post-order numbering: low child, high child, then the node itself;
    within a supernode columns go in increasing canonical edge id.
Symbolic structure: U_s = (adj(cols(s)) U (U_c over children c)) minus the
columns of s and of its descendants, sorted by new index, where adj is the
"shares a cell" relation between unknown edges (the structural pattern of K
and M).

Pins (tests/test_oracle_ordering.py): perm is a bijection; the separator
property (no entry of K couples two sibling subtrees); a hand-checked 4^3
example; U_s against a brute-force boolean elimination game on the permuted
pattern; |U_s| = number of unknown edges on the surface of the box.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import HexMesh


class Supernode:
    __slots__ = ("box", "cols", "children", "parent", "first", "last", "rows", "sub_first", "level")

    def __init__(self, box, cols, children):
        self.box = box
        self.cols = cols          # canonical edge ids, increasing
        self.children = children  # indices of child supernodes
        self.parent = -1
        self.first = -1           # first new index of its columns
        self.last = -1            # one past the last new index
        self.sub_first = -1       # first new index of its subtree
        self.rows = None          # U_s as new indices, increasing
        self.level = 0            # depth from the root (root = 0)


def _box_interior_edges(mesh: HexMesh, box):
    (x0, x1), (y0, y1), (z0, z1) = box
    out = []
    # x-edges: i in [x0, x1), j in (y0, y1), k in (z0, z1)
    for k in range(z0 + 1, z1):
        for j in range(y0 + 1, y1):
            for i in range(x0, x1):
                out.append(mesh.ex(i, j, k))
    for k in range(z0 + 1, z1):
        for j in range(y0, y1):
            for i in range(x0 + 1, x1):
                out.append(mesh.ey(i, j, k))
    for k in range(z0, z1):
        for j in range(y0 + 1, y1):
            for i in range(x0 + 1, x1):
                out.append(mesh.ez(i, j, k))
    return out


def _plane_edges(mesh: HexMesh, box, axis, p):
    """Edges lying in the plane {coordinate axis = p}, inside the closed box,
    not on the box surface."""
    (x0, x1), (y0, y1), (z0, z1) = box
    out = []
    if axis == 0:
        for k in range(z0 + 1, z1):
            for j in range(y0, y1):
                out.append(mesh.ey(p, j, k))
        for k in range(z0, z1):
            for j in range(y0 + 1, y1):
                out.append(mesh.ez(p, j, k))
    elif axis == 1:
        for k in range(z0 + 1, z1):
            for i in range(x0, x1):
                out.append(mesh.ex(i, p, k))
        for k in range(z0, z1):
            for i in range(x0 + 1, x1):
                out.append(mesh.ez(i, p, k))
    else:
        for j in range(y0 + 1, y1):
            for i in range(x0, x1):
                out.append(mesh.ex(i, j, p))
        for j in range(y0, y1):
            for i in range(x0 + 1, x1):
                out.append(mesh.ey(i, j, p))
    return out


def nested_dissection(mesh: HexMesh, leaf_max=4):
    """Supernodes in post-order (list index = supernode id) and perm, where
    perm[new] = unknown index (position among unknowns in increasing
    canonical order)."""
    nodes = []

    def rec(box, level):
        sides = [box[d][1] - box[d][0] for d in range(3)]
        if max(sides) <= leaf_max:
            cols = sorted(_box_interior_edges(mesh, box))
            nodes.append(Supernode(box, cols, []))
            nodes[-1].level = level
            return len(nodes) - 1
        axis = int(np.argmax(sides))          # first maximum: x, then y, then z
        lo, hi = box[axis]
        p = lo + (hi - lo) // 2
        b1 = list(box)
        b2 = list(box)
        b1[axis] = (lo, p)
        b2[axis] = (p, hi)
        c1 = rec(tuple(b1), level + 1)
        c2 = rec(tuple(b2), level + 1)
        cols = sorted(_plane_edges(mesh, box, axis, p))
        nodes.append(Supernode(box, cols, [c1, c2]))
        nodes[-1].level = level
        me = len(nodes) - 1
        nodes[c1].parent = me
        nodes[c2].parent = me
        return me

    rec(((0, mesh.nx), (0, mesh.ny), (0, mesh.nz)), 0)
    unk = mesh.unknown_edges()
    pos = -np.ones(mesh.n_edges, dtype=np.int64)
    pos[unk] = np.arange(len(unk))
    perm = []
    for s, nd in enumerate(nodes):
        nd.first = len(perm)
        perm.extend(int(pos[e]) for e in nd.cols)
        nd.last = len(perm)
        if nd.children:
            nd.sub_first = nodes[nd.children[0]].sub_first
        else:
            nd.sub_first = nd.first
    perm = np.asarray(perm, dtype=np.int64)
    return nodes, perm


def cell_adjacency(mesh: HexMesh):
    """Boolean pattern (CSR, unknown indices) of the relation 'two unknown
    edges belong to a common cell' (includes the diagonal)."""
    ce = mesh.cell_edges()
    unk = mesh.unknown_edges()
    pos = -np.ones(mesh.n_edges, dtype=np.int64)
    pos[unk] = np.arange(len(unk))
    loc = pos[ce]
    ii = np.repeat(loc, 12, axis=1)
    jj = np.tile(loc, (1, 12))
    keep = (ii >= 0) & (jj >= 0)
    N = len(unk)
    A = sp.coo_matrix((np.ones(keep.sum()), (ii[keep], jj[keep])), shape=(N, N)).tocsr()
    A.sum_duplicates()
    A.data[:] = 1.0
    return A


def symbolic(mesh: HexMesh, nodes, perm):
    """Fill in U_s (rows) for every supernode, as sorted new indices."""
    N = len(perm)
    iperm = np.empty(N, dtype=np.int64)
    iperm[perm] = np.arange(N)
    A = cell_adjacency(mesh)
    # permuted pattern: row new index -> neighbour new indices
    Ap = A[perm][:, perm].tocsr()
    for s, nd in enumerate(nodes):
        parts = [Ap.indices[Ap.indptr[nd.first]:Ap.indptr[nd.last]].astype(np.int64)]
        for c in nd.children:
            parts.append(nodes[c].rows)
        cand = np.unique(np.concatenate(parts)) if parts else np.zeros(0, np.int64)
        keep = (cand < nd.sub_first) | (cand >= nd.last)
        nd.rows = cand[keep]
    return iperm


def analyse(mesh: HexMesh, leaf_max=4):
    nodes, perm = nested_dissection(mesh, leaf_max)
    iperm = symbolic(mesh, nodes, perm)
    return nodes, perm, iperm


def factor_flops(nodes):
    """Real flops of the complex partial LDL^T over all fronts:
    8 * ((k+u)^3 - u^3) / 6 (complex multiply-add = 8 real flops)."""
    tot = 0.0
    for nd in nodes:
        k = nd.last - nd.first
        u = len(nd.rows)
        tot += 8.0 * ((k + u) ** 3 - u ** 3) / 6.0
    return tot


def nnz_L(nodes):
    return sum((nd.last - nd.first) * (nd.last - nd.first + 1) // 2
               + (nd.last - nd.first) * len(nd.rows) for nd in nodes)
