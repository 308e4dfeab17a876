"""Host-side analysis of tetrahedral meshes (no GPU): the graph nested
dissection and supernodal structure of tem_symbolic_tet_host against a
brute-force elimination of the permuted pattern."""
import numpy as np
import pytest

from oracle import tet as ot
from tem_inputs.tet import kuhn_mesh

tem = pytest.importorskip("paper_2605_19951_amd.tem")


def _lib_or_skip():
    try:
        tem.load_library()
    except ImportError as e:
        pytest.skip(str(e))


def unknown_graph(topo):
    """Pairs of unknowns sharing a tetrahedron (from the oracle's topology)."""
    adj = [set() for _ in range(len(topo.unknown))]
    for t in range(len(topo.tets)):
        us = [int(topo.pos[e]) for e in topo.tet_edges[t] if topo.pos[e] >= 0]
        for a in us:
            adj[a].update(us)
    return adj


def eliminate(adj, perm):
    """Column structures of L (rows below the diagonal) from the
    elimination game on the permuted graph."""
    n = len(perm)
    iperm = np.empty(n, np.int64)
    iperm[perm] = np.arange(n)
    g = [set(int(iperm[w]) for w in adj[perm[q]]) - {q} for q in range(n)]
    cols = []
    for j in range(n):
        lower = sorted(i for i in g[j] if i > j)
        cols.append(lower)
        for a in lower:
            g[a].update(b for b in lower if b != a)
    return cols


@pytest.mark.parametrize("shape,leaf", [((5, 4, 4), 2), ((4, 4, 4), 1), ((3, 3, 3), 4)])
def test_graph_nested_dissection_structure(shape, leaf):
    _lib_or_skip()
    nx, ny, nz = shape
    me = kuhn_mesh(nx, ny, nz, 10.0, 1, 0.15, np.random.default_rng(nx * 7 + leaf))
    sym = tem.symbolic_tet_host(me.xyz, me.tets, leaf)
    topo = ot.TetTopology(me.xyz, me.tets)
    adj = unknown_graph(topo)
    N = len(topo.unknown)
    assert sym["n_unknowns"] == N
    assert sym["nnz_a"] == sum(len(a) for a in adj)
    perm = sym["perm"]
    assert np.array_equal(np.sort(perm), np.arange(N))
    sp_, par = sym["sn_ptr"], sym["sn_parent"]
    ns = len(par)
    assert sp_[0] == 0 and sp_[-1] == N and (np.diff(sp_) > 0).all()
    assert par[-1] == -1 and all(par[s] > s for s in range(ns - 1))
    # within a supernode the columns follow the unknown (canonical) order
    for s in range(ns):
        cols = perm[sp_[s]:sp_[s + 1]]
        assert (np.diff(cols) > 0).all()
    # U_s holds the column structures of L over the supernode (minus the
    # supernode: the exact fill), and is what the multifrontal assembly
    # produces: (neighbours of the supernode's columns, plus the children's
    # update rows) outside the supernode's subtree, all of them later
    lcols = eliminate(adj, perm)
    rp, rows = sym["rows_ptr"], sym["rows"]
    iperm = np.empty(N, np.int64)
    iperm[perm] = np.arange(N)
    sub_first = list(sp_[:-1])
    for s in range(ns):
        if par[s] >= 0:
            sub_first[par[s]] = min(sub_first[par[s]], sub_first[s])
    nnz_l, exact = 0, 0
    for s in range(ns):
        U = rows[rp[s]:rp[s + 1]]
        fill = set()
        for j in range(sp_[s], sp_[s + 1]):
            fill.update(lcols[j])
        fill -= set(range(sp_[s], sp_[s + 1]))
        assert fill <= set(U), s
        front = set()
        for j in range(sp_[s], sp_[s + 1]):
            front.update(int(iperm[w]) for w in adj[perm[j]])
        for c in np.nonzero(par == s)[0]:
            front.update(rows[rp[c]:rp[c + 1]])
        front = {r for r in front if r < sub_first[s] or r >= sp_[s + 1]}
        assert sorted(front) == list(U), s
        assert len(U) == 0 or U[0] >= sp_[s + 1]
        k = sp_[s + 1] - sp_[s]
        exact += sum(len(lcols[j]) + 1 for j in range(sp_[s], sp_[s + 1]))
        nnz_l += k * (k + 1) // 2 + k * len(U)
        # an update row lies in the parent's columns or its update rows
        if par[s] >= 0 and len(U):
            p = par[s]
            inpar = set(range(sp_[p], sp_[p + 1])) | set(rows[rp[p]:rp[p + 1]])
            assert set(U) <= inpar
    assert sym["nnz_l"] == nnz_l
    # the supernodes' dense triangles and any rows a child brings past its
    # true parent cost some explicit zeros; keep that bounded once the
    # graph is split at all (a single leaf is one dense front)
    if ns > 1:
        assert nnz_l <= 1.5 * exact, (nnz_l, exact)


def test_tet_host_rejects_bad_meshes():
    _lib_or_skip()
    me = kuhn_mesh(2, 2, 2, 10.0, 1, 0.0)
    bad = me.tets.copy()
    bad[0, 1] = bad[0, 0]                       # repeated node
    with pytest.raises(tem.TemError):
        tem.symbolic_tet_host(me.xyz, bad)
    flat = me.xyz.copy()
    flat[:, 2] = 0.0                            # zero volumes
    with pytest.raises(tem.TemError):
        tem.symbolic_tet_host(flat, me.tets)
    dup = np.concatenate([me.tets, me.tets[:1]])   # a face of three tetrahedra
    with pytest.raises(tem.TemError):
        tem.symbolic_tet_host(me.xyz, dup)


def test_disconnected_mesh_gets_a_valid_tree():
    """Two blocks of cubes that share no node: the split between them cuts no
    edge, so the separator is a single unknown; the structure still holds
    the exact fill."""
    _lib_or_skip()
    a = kuhn_mesh(3, 3, 3, 10.0, 1, 0.1, np.random.default_rng(8))
    b = kuhn_mesh(3, 3, 3, 10.0, 1, 0.1, np.random.default_rng(9))
    xyz = np.concatenate([a.xyz, b.xyz + np.array([100.0, 0.0, 0.0])])
    tets = np.concatenate([a.tets, b.tets + len(a.xyz)]).astype(np.int32)
    sym = tem.symbolic_tet_host(xyz, tets, 1)
    topo = ot.TetTopology(xyz, tets)
    adj = unknown_graph(topo)
    N = len(topo.unknown)
    assert sym["n_unknowns"] == N
    perm, sp_, par = sym["perm"], sym["sn_ptr"], sym["sn_parent"]
    assert np.array_equal(np.sort(perm), np.arange(N))
    ns = len(par)
    assert par[-1] == -1 and all(par[s] > s for s in range(ns - 1))
    assert sp_[-1] - sp_[-2] == 1          # the root: a one-unknown separator
    lcols = eliminate(adj, perm)
    rp, rows = sym["rows_ptr"], sym["rows"]
    for s in range(ns):
        fill = set()
        for j in range(sp_[s], sp_[s + 1]):
            fill.update(lcols[j])
        fill -= set(range(sp_[s], sp_[s + 1]))
        assert fill <= set(rows[rp[s]:rp[s + 1]]), s
