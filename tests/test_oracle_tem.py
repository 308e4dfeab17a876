"""Pins of the oracle's shifted solves, time assembly, Jacobian products and
LSQR against things the paper and the mathematics fix independently."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import tem_inputs as ti
from oracle.fem import HexMesh
from oracle.tem import OracleTEM, first_difference, gauss_newton_step, lsqr


def make(wl, sigma=None):
    me = wl.mesh
    return OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma if sigma is None else sigma, wl.F,
                     wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.xi, wl.poles.alpha, wl.params)


@pytest.fixture(scope="module")
def tiny():
    wl = ti.tiny_workload()
    return wl, make(wl)


def test_pole_table_properties(tiny):
    wl, _ = tiny
    pt = wl.poles
    assert np.all(pt.xi.imag > 0)              # no real pole: 2 Re would double count it
    assert pt.alpha.shape == (20, 8)
    assert np.max(pt.err) < 5e-3
    # the rational function is real-valued and close to exp(-t z) on z >= 0
    z = np.logspace(-2, 12, 777)
    for j in (0, 10, 19):
        assert np.max(np.abs(np.exp(-pt.t[j] * z) - pt.r(j, z))) <= pt.err[j] * 1.5 + 1e-12


def test_sparse_solve_matches_dense_lapack(tiny):
    """Two backward-stable FP64 solvers agree to kappa * u on g itself (the
    air gradient modes make A_i ill conditioned, kappa ~ 1e8) and to near
    round-off on what the receivers observe and on the residual."""
    wl, o = tiny
    Qd = o.Q.toarray()
    for i in (0, 3, 7):
        A = o.A(i).toarray()
        g_dense = np.linalg.solve(A, o.F.astype(complex))
        g = o.solve(i, o.F)
        assert np.linalg.norm(g - g_dense) <= 1e-8 * np.linalg.norm(g_dense)
        assert np.linalg.norm(Qd @ (g - g_dense)) <= 1e-11 * np.linalg.norm(Qd @ g_dense)
        assert np.linalg.norm(o.F - A @ g) <= 1e-13 * np.linalg.norm(o.F)


def test_conjugate_pole_symmetry(tiny):
    """The oracle's own shifted solve at a pole and at its conjugate:
    g(conj xi) = conj(g(xi)) since K, M and f are real."""
    wl, _ = tiny
    me = wl.mesh
    xi = wl.poles.xi[2]
    o2 = OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                   np.array([xi, np.conj(xi)]), wl.poles.alpha[:, :2], wl.params)
    g = o2.solve(0, o2.F)
    gc = o2.solve(1, o2.F)
    assert np.linalg.norm(gc - np.conj(g)) <= 1e-13 * np.linalg.norm(g)


def test_divergence_invariant(tiny):
    # G^T f = 0 and G^T K = 0 give G^T M g_i = 0 for every pole.
    wl, o = tiny
    me = wl.mesh
    mesh = HexMesh(me.nx, me.ny, me.nz, me.h)
    nodes_int = [mesh.node(i, j, k) for k in range(1, me.nz) for j in range(1, me.ny)
                 for i in range(1, me.nx)]
    Gi = mesh.gradient()[:, nodes_int][o.unk]
    G = o.solve_poles()
    for i in range(G.shape[0]):
        Mg = o.M @ G[i]
        lhs = Gi.T @ Mg
        assert np.linalg.norm(lhs) <= 1e-12 * abs(Gi).sum(0).max() * np.linalg.norm(Mg)


def test_dense_eigendecomposition_pins_rational_approximation(tiny):
    """u_RA(t) = V r_t(Lambda) V^T f exactly (both are the rational function
    of M^{-1} K applied to b), and ||u_RA - u_exact||_M <= eps(t) ||b||_M
    with eps(t) the scalar error at the pencil's eigenvalues."""
    wl, o = tiny
    Kd = o.K.toarray()
    Md = o.M.toarray()
    lam, V = sla.eigh(Kd, Md)
    lam = np.maximum(lam, 0.0)
    f = o.F[:, 0]
    b = np.linalg.solve(Md, f)
    bM = math.sqrt(b @ Md @ b)
    o.solve_poles()
    for j in (0, 5, 10, 19):
        t = wl.poles.t[j]
        u_ra = o.fields(j)[:, 0]
        u_ra_eig = V @ (wl.poles.r(j, lam) * (V.T @ f))
        dlt = u_ra - u_ra_eig
        # M-norm: the only norm in which M^{-1}K is self-adjoint; the
        # Euclidean difference is dominated by air gradient modes, which are
        # determined only to kappa * u by either route.
        assert math.sqrt(dlt @ Md @ dlt) <= 1e-10 * bM
        Qd = o.Q.toarray()
        assert np.linalg.norm(Qd @ dlt) <= 1e-8 * np.linalg.norm(Qd @ u_ra_eig) + 1e-15
        u_ex = V @ (np.exp(-t * lam) * (V.T @ f))
        eps = np.max(np.abs(np.exp(-t * lam) - wl.poles.r(j, lam)))
        err = u_ra - u_ex
        assert math.sqrt(err @ Md @ err) <= 1.0001 * eps * bM + 1e-12 * bM
    # the eigen route itself against the matrix exponential
    t = wl.poles.t[10]
    u_expm = sla.expm(-t * np.linalg.solve(Md, Kd)) @ b
    u_ex = V @ (np.exp(-t * lam) * (V.T @ f))
    dx = u_expm - u_ex
    assert math.sqrt(dx @ Md @ dx) <= 1e-8 * math.sqrt(u_ex @ Md @ u_ex)


def test_data_is_Q_of_fields(tiny):
    wl, o = tiny
    d = o.data()
    assert d.shape == (1, 20, 5)
    Qd = wl.rx.dense(wl.mesh.n_edges)[:, o.unk]
    for j in (0, 7, 19):
        assert np.allclose(d[0, j], Qd @ o.fields(j)[:, 0], rtol=1e-12, atol=1e-25)


@pytest.fixture(scope="module")
def small_bz():
    wl = ti.smooth_workload(10, 2, S=2, m=6, K=8, g=2, seed=11)
    return wl, make(wl)


def test_adjoint_identity(small_bz):
    wl, o = small_bz
    rng = np.random.default_rng(0)
    v = rng.standard_normal(len(wl.params))
    w = rng.standard_normal(o.data().shape)
    a = np.vdot(o.jvp(v).reshape(-1), w.reshape(-1))
    b = np.vdot(v, o.vjp(w))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_taylor_remainders(small_bz):
    wl, o = small_bz
    rng = np.random.default_rng(1)
    m0 = np.log(wl.sigma[wl.params])
    dm = rng.standard_normal(len(m0))
    o.set_model(m0)
    d0 = o.data()
    jv = o.jvp(dm)
    hs = [0.1 / 2 ** k for k in range(5)]
    e0, e1 = [], []
    for h in hs:
        o.set_model(m0 + h * dm)
        dh = o.data()
        e0.append(np.linalg.norm(dh - d0))
        e1.append(np.linalg.norm(dh - d0 - h * jv))
    o.set_model(m0)
    s0 = np.polyfit(np.log(hs), np.log(e0), 1)[0]
    s1 = np.polyfit(np.log(hs), np.log(e1), 1)[0]
    assert abs(s0 - 1.0) < 0.1
    assert abs(s1 - 2.0) < 0.1


def test_central_differences_match_vjp(small_bz):
    wl, o = small_bz
    rng = np.random.default_rng(2)
    m0 = np.log(wl.sigma[wl.params])
    o.set_model(m0)
    w = rng.standard_normal(o.data().shape)
    grad = o.vjp(w)
    h = 1e-3
    for _ in range(3):
        dirn = rng.standard_normal(len(m0))
        dirn /= np.linalg.norm(dirn)
        o.set_model(m0 + h * dirn)
        dp = np.vdot(o.data().reshape(-1), w.reshape(-1))
        o.set_model(m0 - h * dirn)
        dmn = np.vdot(o.data().reshape(-1), w.reshape(-1))
        fd = (dp - dmn) / (2 * h)
        assert abs(fd - grad @ dirn) <= 1e-5 * np.linalg.norm(grad)
    o.set_model(m0)


def test_lsqr_matches_scipy_and_lstsq():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 12))
    b = rng.standard_normal(40)
    x, _ = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, 12, 12)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    B = rng.standard_normal((300, 80))
    c = rng.standard_normal(300)
    x, _ = lsqr(lambda v: B @ v, lambda u: B.T @ u, c, 80, 20)
    xs = spla.lsqr(B, c, atol=0, btol=0, conlim=0, iter_lim=20)[0]
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def _krylov_lstsq(A, b, k):
    """min ||A x - b|| over x in K_k(A^T A, A^T b), with an orthonormal
    basis of the Krylov space from Arnoldi (modified Gram-Schmidt, twice)
    on the normal operator and a dense least-squares solve."""
    q = A.T @ b
    Q = [q / np.linalg.norm(q)]
    for _ in range(k - 1):
        z = A.T @ (A @ Q[-1])
        for _pass in range(2):
            for qq in Q:
                z = z - (qq @ z) * qq
        Q.append(z / np.linalg.norm(z))
    V = np.stack(Q, axis=1)
    y = np.linalg.lstsq(A @ V, b, rcond=None)[0]
    return V @ y


def test_reorthogonalised_lsqr_is_the_krylov_least_squares_solution():
    """On an ill-conditioned operator (singular values from 1 to 1e-8) the
    reorthogonalised LSQR iterate after k steps is the least-squares solution
    over the k-dimensional Krylov space; plain LSQR agrees with it while its
    vectors are still orthogonal and drifts away later."""
    rng = np.random.default_rng(8)
    m, n = 200, 120
    U = np.linalg.qr(rng.standard_normal((m, n)))[0]
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = U @ np.diag(np.logspace(0, -8, n)) @ V.T
    b = rng.standard_normal(m)
    mv, rmv = (lambda v: A @ v), (lambda u: A.T @ u)
    for k in (3, 10, 30):
        x, hist = lsqr(mv, rmv, b, n, k, reorth=True)
        ref = _krylov_lstsq(A, b, k)
        assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)
        # the residual estimate is the residual norm of the iterate
        assert abs(hist[-1] - np.linalg.norm(b - A @ x)) <= 1e-8 * np.linalg.norm(b)
    xp, _ = lsqr(mv, rmv, b, n, 3)
    xr, _ = lsqr(mv, rmv, b, n, 3, reorth=True)
    assert np.linalg.norm(xp - xr) <= 1e-12 * np.linalg.norm(xr)


def test_lsqr_degenerate_right_hand_sides():
    # b = 0: x = 0 and a zero residual; A^T b = 0 (b orthogonal to the range
    # of A): x = 0 is the least-squares solution and ||r|| = ||b|| throughout.
    # Both end the bidiagonalisation at once (rho = 0), as in SciPy's LSQR.
    rng = np.random.default_rng(5)
    A = np.zeros((30, 6))
    A[:10] = rng.standard_normal((10, 6))
    x, hist = lsqr(lambda v: A @ v, lambda u: A.T @ u, np.zeros(30), 6, 5)
    assert np.array_equal(x, np.zeros(6)) and hist == [0.0] * 5
    x, hist = lsqr(lambda v: A @ v, lambda u: A.T @ u, np.zeros(30), 6, 5, reorth=True)
    assert np.array_equal(x, np.zeros(6)) and hist == [0.0] * 5
    b = np.zeros(30)
    b[10:] = rng.standard_normal(20)
    x, hist = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, 6, 5)
    assert np.array_equal(x, np.zeros(6))
    assert np.allclose(hist, np.linalg.norm(b), rtol=1e-15)
    xs = spla.lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=5)[0]
    assert np.array_equal(xs, np.zeros(6))


def test_first_difference_operator():
    R = first_difference(3, 2, 2)
    # faces between earth cells: x: 2*2*2, y: 3*1*2, z: 3*2*1
    assert R.shape == (8 + 6 + 6, 12)
    assert np.allclose(R @ np.ones(12), 0.0)
    assert np.all(np.abs(R).sum(1) == 2)


def test_gauss_newton_step_with_explicit_jacobian():
    """On a tiny model (2x2x2 earth parameters), LSQR run for P iterations on
    the implicit operator equals the dense least-squares step with the
    Jacobian assembled column by column from jvp."""
    wl = ti.smooth_workload(8, 2, S=1, m=4, K=5, g=2, seed=12)
    me = wl.mesh
    params = np.array([me.cell(i, j, k) for k in (2, 3) for j in (3, 4) for i in (3, 4)],
                      dtype=np.int32)
    o = OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col,
                  wl.rx.val, wl.poles.xi, wl.poles.alpha, params)
    m_true = np.log(wl.sigma[params])
    o.set_model(m_true)
    d_obs = o.data().reshape(-1)
    wd = 1.0 / (0.03 * np.abs(d_obs) + 1e-12)
    m0 = m_true + 0.3
    R = first_difference(2, 2, 2)
    P = len(params)
    dm, hist, b = gauss_newton_step(o, m0, d_obs, wd, m0, 1.0, R, P)
    dmr, _, _ = gauss_newton_step(o, m0, d_obs, wd, m0, 1.0, R, P, reorth=True)
    o.set_model(m0)
    J = np.stack([o.jvp(e).reshape(-1) for e in np.eye(P)], axis=1)
    Aug = np.vstack([wd[:, None] * J, R.toarray()])
    ref = np.linalg.lstsq(Aug, b, rcond=None)[0]
    assert np.linalg.norm(dm - ref) <= 1e-8 * np.linalg.norm(ref)
    assert np.linalg.norm(dmr - ref) <= 1e-8 * np.linalg.norm(ref)
    # after fewer iterations: the least-squares solution over the Krylov space
    for k in (2, 5):
        dmk, _, _ = gauss_newton_step(o, m0, d_obs, wd, m0, 1.0, R, k, reorth=True)
        o.set_model(m0)
        refk = _krylov_lstsq(Aug, b, k)
        assert np.linalg.norm(dmk - refk) <= 1e-8 * np.linalg.norm(refk)
