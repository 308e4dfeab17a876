"""Pins of the oracle's edge-element operators (section "Spatial
discretization"): closed-form element matrices against quadrature of the
explicit basis, discrete de Rham identities, symmetry/definiteness, and the
input numbering convention."""
import numpy as np
import pytest

import tem_inputs as ti
from oracle.fem import (HexMesh, assemble, basis_curls, basis_values, element_mass_unit,
                        element_stiffness, face_edge_incidence)
from oracle.tem import MU0


def _gauss_tensor(h, npts=3):
    x, w = np.polynomial.legendre.leggauss(npts)
    x = 0.5 * h * (x + 1.0)
    w = 0.5 * h * w
    for a in range(npts):
        for b in range(npts):
            for c in range(npts):
                yield x[a], x[b], x[c], w[a] * w[b] * w[c]


@pytest.mark.parametrize("h", [1.0, 25.0, 50.0])
def test_element_matrices_match_quadrature(h):
    Mq = np.zeros((12, 12))
    Kq = np.zeros((12, 12))
    for x, y, z, w in _gauss_tensor(h):
        N = basis_values(h, x, y, z)
        C = basis_curls(h, x, y, z)
        Mq += w * N @ N.T
        Kq += w * C @ C.T
    Kq /= MU0
    Me = element_mass_unit(h)
    Ke = element_stiffness(h, MU0)
    assert np.max(np.abs(Me - Mq)) <= 1e-14 * np.max(np.abs(Mq))
    assert np.max(np.abs(Ke - Kq)) <= 1e-13 * np.max(np.abs(Kq))


@pytest.mark.parametrize("h", [1.0, 25.0])
def test_element_matrices_closed_form(h):
    # Closed forms worked out by hand from the 1-D integrals of the linear
    # hat functions (int phi_a phi_b = h m1[a, b], phi_a' = s_a / h with
    # s_0 = -1, s_1 = +1), independent of the oracle's basis functions.  An
    # edge along axis d starting at node offsets o (0/1 per axis) has
    # N = e_d prod_{t != d} phi_{o_t}(x_t) / h, so
    #   int N_p . N_q = h prod_{t != d} m1[o_t, o'_t]           (same d)
    #   mu int curl N_p . curl N_q
    #     = (1/h) sum_{t != d} s_{o_t} s_{o'_t} m1[o_u, o'_u]   (same d, u the third axis)
    #     = -(1/h) s_{o_{d'}} s_{o'_d} m1[o_u, o'_u]            (directions d != d', u the third)
    m1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
    sg = np.array([-1.0, 1.0])
    mesh = HexMesh(1, 1, 1, h)
    geo = [mesh.edge_geometry(e) for e in mesh.cell_edges()[0]]
    Mc = np.zeros((12, 12))
    Kc = np.zeros((12, 12))
    for p, (d, *op) in enumerate(geo):
        for q, (d2, *oq) in enumerate(geo):
            if d == d2:
                t1, t2 = [t for t in range(3) if t != d]
                Mc[p, q] = h * m1[op[t1], oq[t1]] * m1[op[t2], oq[t2]]
                Kc[p, q] = (sg[op[t1]] * sg[oq[t1]] * m1[op[t2], oq[t2]]
                            + sg[op[t2]] * sg[oq[t2]] * m1[op[t1], oq[t1]]) / h
            else:
                u = 3 - d - d2
                Kc[p, q] = -sg[op[d2]] * sg[oq[d]] * m1[op[u], oq[u]] / h
    # the hand derivation itself: symmetric, curl-free on element gradients
    assert np.array_equal(Kc, Kc.T)
    Ge = np.zeros((12, 8))
    for p, (d, i, j, k) in enumerate(geo):
        a = (i, j, k)
        b = list(a)
        b[d] += 1
        Ge[p, a[0] + 2 * a[1] + 4 * a[2]] -= 1.0
        Ge[p, b[0] + 2 * b[1] + 4 * b[2]] += 1.0
    assert np.max(np.abs(Kc @ Ge)) <= 1e-15 / h
    assert np.max(np.abs(element_mass_unit(h) - Mc)) <= 1e-15 * h
    assert np.max(np.abs(element_stiffness(h, MU0) * MU0 - Kc)) <= 1e-14 / h


def test_basis_degrees_of_freedom_are_line_integrals():
    # int over edge e' of N_e . t_e' = delta_{e e'} (2-point Gauss is exact).
    h = 2.0
    mesh = HexMesh(1, 1, 1, h)
    ce = mesh.cell_edges()[0]
    g, gw = np.polynomial.legendre.leggauss(2)
    s = 0.5 * h * (g + 1.0)
    sw = 0.5 * h * gw
    for le, e in enumerate(ce):
        d, i, j, k = mesh.edge_geometry(e)
        val = np.zeros(12)
        for t, wt in zip(s, sw):
            p = np.array([i * h, j * h, k * h], float)
            p[d] += t
            val += wt * basis_values(h, *p)[:, d]
        expect = np.zeros(12)
        expect[le] = 1.0
        assert np.allclose(val, expect, atol=1e-14)


def test_curl_is_face_combination():
    # curl N_e = sum_f C[f, e] w_f with unit-flux face functions.
    h = 3.0
    C = face_edge_incidence()
    for x, y, z, _ in _gauss_tensor(h, 2):
        curls = basis_curls(h, x, y, z)
        faces = np.zeros((6, 3))
        for d in range(3):
            s = (x, y, z)[d]
            faces[2 * d, d] = (1.0 - s / h) / h ** 2
            faces[2 * d + 1, d] = (s / h) / h ** 2
        assert np.allclose(curls, C.T @ faces, atol=1e-15)


def test_element_curl_of_gradient_vanishes():
    C = face_edge_incidence()
    mesh = HexMesh(1, 1, 1, 1.0)
    G = mesh.gradient().toarray()           # 12 x 8 for one cell
    ce = mesh.cell_edges()[0]
    Gl = G[ce]
    assert np.array_equal(C @ Gl, np.zeros((6, 8)))
    Ke = element_stiffness(1.0, MU0)
    assert np.max(np.abs(Ke @ Gl)) <= 1e-15 * np.max(np.abs(Ke))


def test_global_identities_8cubed():
    wl = ti.tiny_workload()
    me = wl.mesh
    mesh = HexMesh(me.nx, me.ny, me.nz, me.h)
    K, M = assemble(mesh, wl.sigma, MU0)
    # exact symmetry
    assert abs(K - K.T).max() == 0.0 and abs(M - M.T).max() == 0.0
    # M is SPD
    np.linalg.cholesky(M.toarray())
    # K is SPSD and annihilates gradients of interior nodal functions
    unk = mesh.unknown_edges()
    G = mesh.gradient()
    nodes_int = [mesh.node(i, j, k) for k in range(1, me.nz) for j in range(1, me.ny)
                 for i in range(1, me.nx)]
    Gi = G[:, nodes_int]
    # gradients of interior nodal functions live on unknown edges only
    other = np.setdiff1d(np.arange(mesh.n_edges), unk)
    assert abs(Gi[other]).max() == 0.0
    KG = K @ Gi[unk]
    assert abs(KG).max() <= 1e-14 * abs(K).max()
    # loop sources are discretely divergence free; Bz receivers see no gradient
    assert np.array_equal(G.T @ wl.F, np.zeros((G.shape[1], wl.S)))
    wl2 = ti.smooth_workload(16, 2, S=3, m=8, K=4, g=4, seed=9)
    m2 = HexMesh(16, 16, 16, 25.0)
    Q = wl2.rx.dense(m2.n_edges)
    assert np.max(np.abs(Q @ m2.gradient().toarray())) == 0.0
    assert np.array_equal(m2.gradient().T @ wl2.F, np.zeros((m2.n_nodes(), wl2.S)))


def test_numbering_matches_input_convention():
    me = ti.Mesh(5, 4, 3, 1.0, 1)
    mesh = HexMesh(5, 4, 3, 1.0)
    assert mesh.n_edges == me.n_edges
    for (i, j, k) in [(0, 0, 0), (4, 4, 3), (2, 1, 2)]:
        assert mesh.ex(i, j, k) == me.xedge(i, j, k)
    for (i, j, k) in [(0, 0, 0), (5, 3, 3), (2, 1, 2)]:
        assert mesh.ey(i, j, k) == me.yedge(i, j, k)
    for (i, j, k) in [(0, 0, 0), (5, 4, 2), (2, 1, 2)]:
        assert mesh.ez(i, j, k) == me.zedge(i, j, k)
    unk = mesh.unknown_edges()
    assert len(unk) == 3 * 0 + (5 * 3 * 2 + 4 * 4 * 2 + 4 * 3 * 3)
    assert all(mesh.is_unknown(e) for e in unk)


def test_assembly_counts_match_combinatorics():
    # n^3 mesh: 3 n (n+1)^2 edges, 3 n (n-1)^2 unknowns; K is 'shares a cell'.
    for n in (4, 8):
        mesh = HexMesh(n, n, n, 1.0)
        K, M = assemble(mesh, np.ones(n ** 3), MU0)
        assert mesh.n_edges == 3 * n * (n + 1) ** 2
        assert K.shape[0] == 3 * n * (n - 1) ** 2
    # 8^3: 31,008 structural entries of K, 8,664 nonzero entries of M
    mesh = HexMesh(8, 8, 8, 1.0)
    K, M = assemble(mesh, np.ones(512), MU0)
    assert K.nnz == 31008
    assert np.count_nonzero(M.data) == 8664
