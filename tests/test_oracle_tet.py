"""Pins of the tetrahedral oracle (oracle/tet.py) against quadrature, the
de Rham identities, Stokes' theorem and the divergence theorem, and of its
forward map against the adjoint identity and finite differences."""
import math

import numpy as np
import pytest

from oracle import tet as ot
from tem_inputs import MU0
from tem_inputs.tet import delaunay_workload, kuhn_mesh, tet_workload

# quadrature exact for quadratics on a tetrahedron: -1/20 of the vertex
# values plus 1/5 of the edge-midpoint values, times the volume
def quad2(x, f):
    vol = abs(np.linalg.det(np.array([x[1] - x[0], x[2] - x[0], x[3] - x[0]]))) / 6.0
    s = -sum(f(x[i]) for i in range(4)) / 20.0
    s = s + sum(f(0.5 * (x[i] + x[j])) for i, j in ot.LOCAL_EDGES) / 5.0
    return vol * s, vol


def nedelec_fields():
    """The six fields a (unit axes) and b x x (unit axes) spanning the local
    lowest-order edge space; value and curl as functions of x."""
    out = []
    for k in range(3):
        a = np.eye(3)[k]
        out.append((lambda x, a=a: a, np.zeros(3)))
    for k in range(3):
        b = np.eye(3)[k]
        out.append((lambda x, b=b: np.cross(b, x), 2.0 * b))
    return out


def edge_dof(f, xa, xb):
    # line integral of a linear field along the segment: midpoint rule
    return f(0.5 * (xa + xb)) @ (xb - xa)


@pytest.fixture(scope="module")
def small_mesh():
    return kuhn_mesh(4, 4, 4, 25.0, 1, 0.15, np.random.default_rng(3))


def test_numbering_matches_inputs(small_mesh):
    topo = ot.TetTopology(small_mesh.xyz, small_mesh.tets)
    assert np.array_equal(topo.edges, small_mesh.edges)
    assert np.array_equal(topo.faces, small_mesh.faces)
    # a conforming mesh: every face has one or two tetrahedra
    assert all(len(t) in (1, 2) for t in topo.face_tets)


def test_element_matrices_on_the_local_space(small_mesh):
    rng = np.random.default_rng(0)
    fields = nedelec_fields()
    for c in rng.choice(small_mesh.n_tets, 5, replace=False):
        x = small_mesh.xyz[small_mesh.tets[c]] - small_mesh.xyz[small_mesh.tets[c]].mean(0)
        Ke, Me = ot.edge_element(x, MU0)
        U = np.array([[edge_dof(f, x[i], x[j]) for (f, _) in fields] for i, j in ot.LOCAL_EDGES])
        assert abs(np.linalg.det(U)) > 1e-6 * np.abs(U).max() ** 6
        for a, (fa, ca) in enumerate(fields):
            for b, (fb, cb) in enumerate(fields):
                q, vol = quad2(x, lambda p: fa(p) @ fb(p))
                m = U[:, a] @ Me @ U[:, b]
                assert abs(m - q) <= 1e-12 * vol * 625.0, (a, b, m, q)
                k = U[:, a] @ Ke @ U[:, b]
                assert abs(k - vol * (ca @ cb) / MU0) <= 1e-12 * vol / MU0, (a, b, k)


def test_assembled_forms_and_gradient_kernel(small_mesh):
    topo = ot.TetTopology(small_mesh.xyz, small_mesh.tets)
    rng = np.random.default_rng(1)
    sigma = np.exp(rng.uniform(-3, 0, small_mesh.n_tets))
    K, M = ot.assemble_all(topo, sigma, MU0)
    a, b = rng.standard_normal(3), rng.standard_normal(3) / 50.0
    f = lambda p: a + np.cross(b, p)
    xyz = small_mesh.xyz
    u = np.array([edge_dof(f, xyz[e0], xyz[e1]) for e0, e1 in topo.edges])
    qm, qk = 0.0, 0.0
    for c, t in enumerate(small_mesh.tets):
        q, vol = quad2(xyz[t], lambda p: f(p) @ f(p))
        qm += sigma[c] * q
        qk += vol * 4.0 * (b @ b) / MU0
    assert abs(u @ (M @ u) - qm) <= 1e-11 * qm
    assert abs(u @ (K @ u) - qk) <= 1e-11 * qk
    G = topo.gradient()
    KG = K @ G
    assert abs(KG).max() <= 1e-12 * abs(K).max()
    # restricted to the unknowns, gradients of interior-node functions too
    Ku, Mu = ot.assemble(topo, sigma, MU0)
    Gi = G[topo.unknown][:, topo.inner_nodes]
    assert abs(Ku @ Gi).max() <= 1e-12 * abs(Ku).max()
    # symmetric, and M positive definite on the unknowns
    assert abs(Mu - Mu.T).max() <= 1e-15 * abs(Mu).max()
    assert abs(Ku - Ku.T).max() <= 1e-15 * abs(Ku).max()
    assert np.linalg.eigvalsh(Mu.toarray()).min() > 0.0


def test_receivers_and_sources_against_stokes():
    wl = tet_workload(8, 2, S=2, m=4, K=4, g=2, seed=21)
    me = wl.mesh
    topo = ot.TetTopology(me.xyz, me.tets)
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal(3), rng.standard_normal(3)
    f = lambda p: a + np.cross(b, p)
    u = np.array([edge_dof(f, me.xyz[e0], me.xyz[e1]) for e0, e1 in topo.edges])
    Q = wl.rx.dense(me.n_edges)
    assert np.allclose(Q @ u, -2.0 * b[2], rtol=1e-12, atol=0)
    # loops: closed (no circulation of a gradient) and 2 b_z (loop area)
    phi = rng.standard_normal(me.n_nodes)
    assert np.allclose(wl.F.T @ (topo.gradient() @ phi), 0.0, atol=1e-12)
    for s in range(wl.S):
        es = np.nonzero(wl.F[:, s])[0]
        assert len(es) == 8
        # walk the loop in the direction of f to get its polygon
        nxt = {}
        for e in es:
            p, q = topo.edges[e]
            if wl.F[e, s] < 0:
                p, q = q, p
            nxt[int(p)] = int(q)
        ring, v = [], next(iter(nxt))
        for _ in range(8):
            ring.append(v)
            v = nxt[v]
        assert v == ring[0]
        P = me.xyz[ring, :2]
        area = 0.5 * sum(P[k, 0] * P[(k + 1) % 8, 1] - P[(k + 1) % 8, 0] * P[k, 1] for k in range(8))
        assert area > 0   # counter-clockwise seen from +z
        assert abs(wl.F[:, s] @ u - 2.0 * b[2] * area) <= 1e-10 * abs(b[2]) * area


def test_rt0_element_on_the_local_space(small_mesh):
    rng = np.random.default_rng(4)
    for c in rng.choice(small_mesh.n_tets, 5, replace=False):
        x = small_mesh.xyz[small_mesh.tets[c]]
        Me = ot.rt0_element(x)
        ctr = x.mean(0)
        fields = [lambda p, k=k: np.eye(3)[k] for k in range(3)] + [lambda p: p - ctr]
        V = np.zeros((4, 4))
        for p, fc in enumerate(ot.LOCAL_FACES):
            y = x[list(fc)]
            n = np.cross(y[1] - y[0], y[2] - y[0])
            if n @ (y[0] - x[p]) < 0:
                n = -n                    # outward
            cf = y.mean(0)
            for k, f in enumerate(fields):
                V[p, k] = f(cf) @ n / 2.0   # flux of a linear field: centroid rule
        for k in range(4):
            for l in range(4):
                q, vol = quad2(x, lambda p: fields[k](p) @ fields[l](p))
                assert abs(V[:, k] @ Me @ V[:, l] - q) <= 1e-11 * max(abs(q), vol * 25.0)
        # divergence theorem: the outward fluxes of x - c sum to 3 |T|
        assert abs(V[:, 3].sum() - 3.0 * vol) <= 1e-12 * vol


def test_rt0_regulariser_structure(small_mesh):
    topo = ot.TetTopology(small_mesh.xyz, small_mesh.tets)
    params = np.arange(0, small_mesh.n_tets, 2)      # every other tetrahedron
    params = np.unique(np.concatenate([params, np.arange(small_mesh.n_tets // 2)]))
    R, diag, D, lo, hi = ot.rt0_regulariser(topo, params)
    L = D @ sp_diag(1.0 / diag) @ D.T
    assert abs(L @ np.ones(len(params))).max() <= 1e-12 * abs(L).max()
    assert abs((R.T @ R) - L).max() <= 1e-12 * abs(L).max()
    assert (diag > 0).all() and (lo < hi).all()
    # every face in R is shared by two parameter tetrahedra
    n2 = sum(1 for ts in topo.face_tets if len(ts) == 2
             and all(np.isin([t for t, _ in ts], params)))
    assert R.shape[0] == n2


def sp_diag(v):
    import scipy.sparse as sp
    return sp.diags(v)


@pytest.fixture(scope="module")
def tiny_tet():
    wl = tet_workload(6, 2, S=1, m=5, K=6, g=2, seed=23)
    orc = ot.OracleTetTEM(wl.mesh.xyz, wl.mesh.tets, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col,
                          wl.rx.val, wl.poles.xi, wl.poles.alpha, wl.params, wl.mu)
    return wl, orc


def test_forward_adjoint_identity(tiny_tet):
    wl, orc = tiny_tet
    rng = np.random.default_rng(5)
    v = rng.standard_normal(len(wl.params))
    d = orc.data()
    w = rng.standard_normal(d.shape)
    jv = orc.jvp(v)
    jtw = orc.vjp(w)
    lhs, rhs = np.sum(jv * w), v @ jtw
    assert abs(lhs - rhs) <= 1e-10 * np.linalg.norm(jv) * np.linalg.norm(w)


def test_forward_finite_differences(tiny_tet):
    wl, orc = tiny_tet
    rng = np.random.default_rng(6)
    v = rng.standard_normal(len(wl.params))
    v /= np.linalg.norm(v)
    m0 = np.log(wl.sigma[wl.params])
    orc.set_model(m0)
    jv = orc.jvp(v)
    h = 1e-4
    orc.set_model(m0 + h * v)
    dp = orc.data()
    orc.set_model(m0 - h * v)
    dm = orc.data()
    orc.set_model(m0)
    fd = (dp - dm) / (2 * h)
    assert np.linalg.norm(fd - jv) <= 1e-6 * np.linalg.norm(jv)


def test_assembled_forms_on_a_delaunay_mesh():
    """The global forms of a field a + b x x and K G = 0 on a mesh with no
    structure (Delaunay of random points, slivers included)."""
    wl = delaunay_workload(300, S=1, R=2, m=3, K=3, seed=62)
    me = wl.mesh
    topo = ot.TetTopology(me.xyz, me.tets)
    assert np.array_equal(topo.edges, me.edges)
    rng = np.random.default_rng(7)
    K, M = ot.assemble_all(topo, wl.sigma, MU0)
    a, b = rng.standard_normal(3), rng.standard_normal(3) / 500.0
    f = lambda p: a + np.cross(b, p)
    u = np.array([edge_dof(f, me.xyz[e0], me.xyz[e1]) for e0, e1 in topo.edges])
    qm, qk = 0.0, 0.0
    for c, t in enumerate(me.tets):
        q, vol = quad2(me.xyz[t], lambda p: f(p) @ f(p))
        qm += wl.sigma[c] * q
        qk += vol * 4.0 * (b @ b) / MU0
    assert abs(u @ (M @ u) - qm) <= 1e-10 * qm
    assert abs(u @ (K @ u) - qk) <= 1e-10 * qk
    assert abs(K @ topo.gradient()).max() <= 1e-11 * abs(K).max()
