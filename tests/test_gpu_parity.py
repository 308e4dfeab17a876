"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 factors 1e-9, FP32 factors with FP64 GMRES refinement
1e-6 (relative), on the quantities the method outputs (data at all times,
J v, J^T w) and on the receiver view Q g_i of the pole solutions.  The full
vectors g_i are compared in the M-norm (the air gradient modes make A_i
ill conditioned, kappa ~ 1e8, so any FP64 solver fixes g_i itself only to
kappa * u in the Euclidean norm)."""
import numpy as np
import pytest

import tem_inputs as ti
from oracle.fem import HexMesh, assemble
from oracle.tem import OracleTEM

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle(wl):
    me = wl.mesh
    return OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                     wl.poles.xi, wl.poles.alpha, wl.params)


class Run:
    """A factored GPU context for one workload and precision, plus the oracle."""

    def __init__(self, wl, prec, leaf=4):
        torch = _torch()
        from paper_2605_19951_amd import Tem
        self.torch = torch
        self.wl = wl
        me = wl.mesh
        self.dev = torch.device("cuda:0")
        print("case %s prec=%d N-mesh=%s S=%d m=%d" % (wl.name, prec, (me.nx, me.ny, me.nz), wl.S,
                                                       len(wl.poles.xi)), flush=True)
        self.t = Tem(0)
        self.t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0,
                        torch.tensor(wl.sigma, device=self.dev), wl.params)
        self.info = self.t.analyse(leaf)
        self.t.factor_poles(wl.poles.xi, prec)
        self.F = torch.tensor(wl.F.T.copy(), device=self.dev)
        K, R = len(wl.poles.t), wl.rx.n
        self.d = torch.zeros((wl.S, K, R), dtype=torch.float64, device=self.dev)
        self.G = torch.zeros((len(wl.poles.xi), wl.S, me.n_edges), dtype=torch.complex128,
                             device=self.dev)
        self.ir = self.t.forward(self.F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, self.d)
        self.o = _oracle(wl)


def _env_run(wl, prec, env):
    """Run with the library's schedule knobs (read by tem_create) set to env."""
    import os
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return Run(wl, prec)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _wide(wl, prec):
    """Run with the big-block sweep schedule forced on every level."""
    return _env_run(wl, prec, {"TEM_SWEEP_BLOCK": "64", "TEM_SWEEP_BIG_LIMIT": "1000000"})


def C16():
    return ti.smooth_workload(16, 2, S=2, m=6, K=9, g=4, seed=22)


def RK13():
    """13^3 workload whose poles and residues come from RKFIT (six conjugate
    pairs fitted to exp(-t z) at its seven times) instead of the contour."""
    from paper_2605_19951_amd import rkfit
    wl = ti.smooth_workload(13, 2, S=3, m=6, K=7, g=2, seed=21)
    tab = rkfit.rkfit_exp(wl.poles.t, 6)
    wl.poles = ti.PoleTable(t=tab.t, xi=tab.xi, alpha=tab.alpha, err=tab.err)
    return wl


def S17():
    """12^3 mesh with seventeen loop sources on a grid of centres (loops may
    share edges; each column of F is still one loop)."""
    wl = ti.smooth_workload(12, 2, S=1, m=3, K=5, g=2, seed=24)
    centres = [(cx, cy) for cx in range(3, 10, 2) for cy in range(3, 10, 2)][:16] + [(6, 6)]
    wl.F = ti.source_matrix(wl.mesh, centres)
    return wl


CASES = {
    "tiny64": lambda: Run(ti.tiny_workload(), 0),
    "tiny32": lambda: Run(ti.tiny_workload(), 1),
    "r13_64": lambda: Run(ti.smooth_workload(13, 2, S=3, m=5, K=7, g=2, seed=21), 0),
    "r13_32": lambda: Run(ti.smooth_workload(13, 2, S=3, m=5, K=7, g=2, seed=21), 1),
    "c16_64": lambda: Run(ti.smooth_workload(16, 2, S=2, m=6, K=9, g=4, seed=22), 0),
    "c16_32": lambda: Run(ti.smooth_workload(16, 2, S=2, m=6, K=9, g=4, seed=22), 1),
    "w16_64": lambda: _wide(ti.smooth_workload(16, 2, S=2, m=6, K=9, g=4, seed=22), 0),
    "w16_32": lambda: _wide(ti.smooth_workload(16, 2, S=2, m=6, K=9, g=4, seed=22), 1),
    # twelve right-hand sides: the FP32 forward sweep's two-block path (S > 8)
    "s12_32": lambda: Run(ti.smooth_workload(16, 2, S=12, m=3, K=5, g=2, seed=23), 1),
    # seventeen right-hand sides: solved in two blocks of nine (the second
    # padded with a zero right-hand side), both precisions
    # an RKFIT pole/residue table through the whole path, both precisions
    "rk13_64": lambda: Run(RK13(), 0),
    "rk13_32": lambda: Run(RK13(), 1),
    "s17_64": lambda: Run(S17(), 0),
    "s17_32": lambda: Run(S17(), 1),
    # factor panel schedules (the 13^3 root separator has 312 columns): 64-column
    # left-looking panels, and 96-column right-looking panels (recursion halves
    # of 32 and 64 columns)
    "p64_32": lambda: _env_run(ti.smooth_workload(13, 2, S=3, m=5, K=7, g=2, seed=21), 1,
                               {"TEM_PANEL": "64"}),
    "p96rl_64": lambda: _env_run(ti.smooth_workload(13, 2, S=3, m=5, K=7, g=2, seed=21), 0,
                                 {"TEM_PANEL": "96", "TEM_LEFT_LOOKING": "0"}),
    # every front-update variant the autotuner or the knobs can select, on every
    # level of a 16^3 tree (fronts up to 712 rows): FP32 64x64 with four real
    # products, 128x64 with three and four, 128x128 (four); FP64 64x64 with three
    "u64m4_32": lambda: _env_run(C16(), 1, {"TEM_UPDATE_TILE": "64", "TEM_UPDATE_3M": "none"}),
    "u128x64m3_32": lambda: _env_run(C16(), 1, {"TEM_UPDATE_TILE": "128x64",
                                                "TEM_UPDATE_3M": "f32"}),
    "u128x64m4_32": lambda: _env_run(C16(), 1, {"TEM_UPDATE_TILE": "128x64",
                                                "TEM_UPDATE_3M": "none"}),
    "u128_32": lambda: _env_run(C16(), 1, {"TEM_UPDATE_TILE": "128", "TEM_UPDATE_3M": "none"}),
    "u64m3_64": lambda: _env_run(C16(), 0, {"TEM_UPDATE_TILE": "64", "TEM_UPDATE_3M": "f64"}),
}
UPDATE_VARIANTS = ["u64m4_32", "u128x64m3_32", "u128x64m4_32", "u128_32", "u64m3_64"]
_cache = {}


def get(name):
    if name not in _cache:
        _cache[name] = CASES[name]()
    return _cache[name]


TOL = {0: 1e-9, 1: 1e-6}


def test_assembly_matches_oracle():
    r = get("r13_64")
    wl = r.wl
    me = wl.mesh
    perm, rowptr, col, kv, mv = r.t.export_operators()
    mesh = HexMesh(me.nx, me.ny, me.nz, me.h)
    K, M = assemble(mesh, wl.sigma, ti.MU0)
    Kp = K[perm][:, perm].tocsr()
    Mp = M[perm][:, perm].tocsr()
    Kp.sort_indices()
    Mp.sort_indices()
    assert np.array_equal(Kp.indptr, rowptr) and np.array_equal(Kp.indices, col)
    assert np.max(np.abs(kv - Kp.data)) <= 4 * np.finfo(float).eps * np.max(np.abs(kv))
    assert np.max(np.abs(mv - Mp.data)) <= 4 * np.finfo(float).eps * np.max(np.abs(Mp.data))
    # symbolic info agrees with the oracle
    from oracle.ordering import analyse, factor_flops
    nodes, operm, _ = analyse(mesh)
    assert np.array_equal(perm, operm.astype(np.int32))
    assert r.info["flops_per_pole"] == pytest.approx(factor_flops(nodes), rel=1e-12)


@pytest.mark.parametrize("name", list(CASES))
def test_pole_solutions(name):
    r = get(name)
    tol = TOL[int(name.endswith("32"))]
    assert r.ir["n_unconverged"] == 0
    G = r.G
    r.t.solve_poles(r.F, G)
    g = G.cpu().numpy()[:, :, r.o.unk].transpose(0, 2, 1)          # (m, N, S)
    gref = r.o.solve_poles()
    Q = r.o.Q
    for i in range(g.shape[0]):
        dq = Q @ (g[i] - gref[i])
        assert np.linalg.norm(dq) <= tol * np.linalg.norm(Q @ gref[i])
        dg = g[i] - gref[i]
        mn = np.sqrt(np.abs(np.sum(np.conj(dg) * (r.o.M @ dg))))
        mr = np.sqrt(np.abs(np.sum(np.conj(gref[i]) * (r.o.M @ gref[i]))))
        assert mn <= 10 * tol * mr
        res = r.o.F - r.o.A(i) @ g[i]
        assert np.linalg.norm(res) <= 1.5e-10 * np.linalg.norm(r.o.F)
    # boundary edges are zero
    other = np.setdiff1d(np.arange(r.wl.mesh.n_edges), r.o.unk)
    assert np.all(G.cpu().numpy()[:, :, other] == 0)


@pytest.mark.parametrize("name", list(CASES))
def test_data_all_times(name):
    r = get(name)
    tol = TOL[int(name.endswith("32"))]
    d = r.d.cpu().numpy()
    dref = r.o.data()
    cond = r.o.data_condition()
    assert np.all(np.abs(d - dref) <= tol * cond + 1e-300)
    for j in range(d.shape[1]):
        nrm = np.linalg.norm(dref[:, j])
        assert np.linalg.norm(d[:, j] - dref[:, j]) <= tol * max(nrm, np.linalg.norm(cond[:, j]))


@pytest.mark.parametrize("name", ["r13_64", "r13_32", "c16_64", "c16_32", "w16_64", "w16_32",
                                  "s12_32", "s17_64", "s17_32", "rk13_64", "rk13_32"]
                         + UPDATE_VARIANTS)
def test_jvp_vjp(name):
    r = get(name)
    torch = r.torch
    tol = TOL[int(name.endswith("32"))]
    rng = np.random.default_rng(5)
    P = len(r.wl.params)
    v = rng.standard_normal(P)
    w = rng.standard_normal(tuple(r.d.shape))
    jv = torch.zeros_like(r.d)
    jtw = torch.zeros(P, dtype=torch.float64, device=r.dev)
    r.t.jvp(torch.tensor(v, device=r.dev), jv)
    r.t.vjp(torch.tensor(w, device=r.dev), jtw)
    jv_ref = r.o.jvp(v)
    jtw_ref = r.o.vjp(w)
    assert np.linalg.norm(jv.cpu().numpy() - jv_ref) <= tol * np.linalg.norm(jv_ref)
    assert np.linalg.norm(jtw.cpu().numpy() - jtw_ref) <= tol * np.linalg.norm(jtw_ref)
    # adjoint identity on the GPU results
    a = np.vdot(jv.cpu().numpy().ravel(), w.ravel())
    b = np.vdot(v, jtw.cpu().numpy())
    assert abs(a - b) <= 10 * tol * max(abs(a), abs(b))


@pytest.mark.parametrize("name", UPDATE_VARIANTS)
def test_update_variant_needs_no_extra_refinement(name):
    """A forced update kernel factors as accurately as the default one: its
    forward needs at most one refinement solve more than the default kernel's
    on any pole and source (the rounding of the two kernels differs)."""
    r = get(name)
    base = get("c16_32" if name.endswith("32") else "c16_64")
    assert np.max(r.ir["iters"]) <= np.max(base.ir["iters"]) + 1


def test_block_inverse_sweep_matches_triangle_sweep():
    """FP32 factors: the wide fronts' diagonal blocks applied through their
    explicit inverses (column blocks of 64, every level wide) give the same
    single unrefined FP32 solve as the triangle kernels (blocks of 512, no
    inverses), to FP32 rounding, on every pole and source; the data of both
    refined solves agree to the refinement tolerance."""
    inv = _env_run(C16(), 1, {"TEM_SWEEP_BLOCK": "64", "TEM_SWEEP_BIG_LIMIT": "1000000"})
    tri = _env_run(C16(), 1, {"TEM_SWEEP_BLOCK": "512", "TEM_SWEEP_BIG_LIMIT": "1000000"})
    torch = inv.torch
    wl = inv.wl
    d1 = []
    for r in (inv, tri):
        d = torch.zeros_like(r.d)
        ir = r.t.forward(r.F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d,
                         ir=dict(rtol=1e-10, max_iter=1), allow_noconv=True)
        rel = np.asarray(ir["rel"])
        print("one FP32 solve: worst relative residual %.2e" % rel.max(), flush=True)
        assert rel.max() < 1e-4
        d1.append(d.cpu().numpy())
    scale = np.abs(d1[1]).max()
    assert np.abs(d1[0] - d1[1]).max() <= 1e-4 * scale
    assert np.max(inv.ir["iters"]) <= np.max(tri.ir["iters"]) + 1
    assert np.abs(inv.d.cpu().numpy() - tri.d.cpu().numpy()).max() <= 1e-8 * scale


def test_unknown_update_knob_is_refused():
    """tem_create rejects a TEM_UPDATE_TILE or TEM_UPDATE_3M value it does not know."""
    _torch()
    import os
    from paper_2605_19951_amd import Tem, TemError
    for k, v in (("TEM_UPDATE_TILE", "96"), ("TEM_UPDATE_3M", "yes")):
        old = os.environ.get(k)
        os.environ[k] = v
        try:
            with pytest.raises(TemError) as e:
                Tem(0)
            assert k in str(e.value)
        finally:
            if old is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = old


def test_bitwise_determinism():
    r = get("c16_32")
    torch = r.torch
    d2 = torch.zeros_like(r.d)
    r.t.forward(r.F, r.wl.rx.ptr, r.wl.rx.col, r.wl.rx.val, r.wl.poles.alpha, d2)
    d3 = torch.zeros_like(r.d)
    r.t.forward(r.F, r.wl.rx.ptr, r.wl.rx.col, r.wl.rx.val, r.wl.poles.alpha, d3)
    assert torch.equal(d2, d3)


def test_state_machine_and_argument_errors():
    torch = _torch()
    from paper_2605_19951_amd import Tem, TemError
    from paper_2605_19951_amd.tem import TEM_EINVAL, TEM_ESTATE
    wl = ti.tiny_workload()
    me = wl.mesh
    dev = torch.device("cuda:0")
    t = Tem(0)
    with pytest.raises(TemError) as e:
        t.analyse()
    assert e.value.status == TEM_ESTATE
    bad = torch.tensor(wl.sigma, device=dev)
    bad[3] = -1.0
    with pytest.raises(TemError) as e:
        t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0, bad, wl.params)
    assert e.value.status == TEM_EINVAL
    t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0, torch.tensor(wl.sigma, device=dev), wl.params)
    with pytest.raises(TemError) as e:
        t.factor_poles(wl.poles.xi)
    assert e.value.status == TEM_ESTATE
    t.analyse()
    with pytest.raises(TemError) as e:
        t.factor_poles(np.conj(wl.poles.xi))          # Im < 0 rejected
    assert e.value.status == TEM_EINVAL
    t.factor_poles(wl.poles.xi, 0)
    d = torch.zeros((1, 20, 5), dtype=torch.float64, device=dev)
    v = torch.zeros(len(wl.params), dtype=torch.float64, device=dev)
    with pytest.raises(TemError) as e:
        t.jvp(v, d)
    assert e.value.status == TEM_ESTATE
    # a forward call that is refused (a receiver column past the last edge)
    # leaves no survey behind: Jv is refused until a forward call succeeds
    F = torch.tensor(wl.F.T.copy(), device=dev)
    K, R = len(wl.poles.t), wl.rx.n
    d = torch.zeros((wl.S, K, R), dtype=torch.float64, device=dev)
    t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
    jv = torch.zeros_like(d)
    t.jvp(v, jv)
    bad_col = np.array(wl.rx.col, np.int32).copy()
    bad_col[0] = me.n_edges
    with pytest.raises(TemError) as e:
        t.forward(F, wl.rx.ptr, bad_col, wl.rx.val, wl.poles.alpha, d)
    assert e.value.status == TEM_EINVAL
    with pytest.raises(TemError) as e:
        t.jvp(v, jv)
    assert e.value.status == TEM_ESTATE
    t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
    t.jvp(v, jv)
    # more than 1024 right-hand sides are refused, with the survey dropped
    F1025 = F[:1].repeat(1025, 1).contiguous()
    d1025 = torch.zeros((1025, K, R), dtype=torch.float64, device=dev)
    with pytest.raises(TemError) as e:
        t.forward(F1025, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d1025)
    assert e.value.status == TEM_EINVAL
    with pytest.raises(TemError) as e:
        t.jvp(v, jv)
    assert e.value.status == TEM_ESTATE
    t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
    t.jvp(v, jv)
    t.close()
