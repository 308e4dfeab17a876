"""GPU checks at the full sizes of the benchmark workloads, through the C
ABI, in the configuration bench.py times (autotuned update kernels, FP32
factors with FP64 refinement, and FP64 factors).

The oracle's direct solves are too slow at these sizes (~20 min per pole at
64^3), so the checks are properties that hold at any size, evaluated with
the oracle's own assembly, observation and time assembly:

* sampled pole solutions g_is satisfy ||f_s - (K - xi_i M) g_is|| <= 1e-9
  ||f_s|| with K and M assembled by the oracle, not by the library;
* the data equal the oracle's time assembly of the GPU's Q g_is at every
  time, within the summation condition;
* FP32 + refinement and FP64 data agree to 1e-8;
* <J v, w> = <v, J^T w> on the GPU results;
* 48^3 differentiation workload: central differences of <d(m), w> along 32
  random unit directions (h = 1e-3) match <J^T w, dir> to 1e-5 ||J^T w||;
  one Gauss-Newton
  step with 20 LSQR iterations has a non-increasing residual estimate;
* the twelve-mesh ragged batch gives the data of the meshes run one at a
  time."""
import math
import os
import sys

import numpy as np
import pytest

import tem_inputs as ti
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


def test_hex64_precision_workload_properties():
    torch = _torch()
    from paper_2605_19951_amd import Tem
    wl = ti.workload(2)
    me = wl.mesh
    m, S, K, R = len(wl.poles.xi), wl.S, len(wl.poles.t), wl.rx.n
    dev = torch.device("cuda:0")
    print("case hex64_precision: 64^3, 16 poles, 8 sources", flush=True)
    t = Tem(0)
    t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0, torch.tensor(wl.sigma, device=dev), wl.params)
    t.analyse()
    o = _oracle(wl)
    F = torch.tensor(wl.F.T.copy(), device=dev)
    G = torch.zeros((m, S, me.n_edges), dtype=torch.complex128, device=dev)
    data = {}
    for prec in (1, 0):
        print("precision %d" % prec, flush=True)
        if prec == 1:
            t.autotune(wl.poles.xi, prec)
        t.factor_poles(wl.poles.xi, prec)
        d = torch.zeros((S, K, R), dtype=torch.float64, device=dev)
        ir = t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
        assert ir["n_unconverged"] == 0
        t.solve_poles(F, G)
        Gh = G.cpu().numpy()[:, :, o.unk]                       # (m, S, N)
        # independent residuals with the oracle's K and M
        for i, s in [(0, 0), (m // 2, S // 2), (m - 1, S - 1)]:
            g = Gh[i, s]
            r = o.F[:, s] - (o.K @ g - wl.poles.xi[i] * (o.M @ g))
            assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(o.F[:, s])
        # data = the oracle's time assembly of the GPU's observations
        Y = np.stack([o.Q @ Gh[i].T for i in range(m)])          # (m, R, S)
        dref, cond = o._combine(Y), o._combine_condition(Y)
        dh = d.cpu().numpy()
        assert np.all(np.abs(dh - dref) <= 1e-12 * cond + 1e-300)
        data[prec] = dh
    assert np.linalg.norm(data[1] - data[0]) <= 1e-8 * np.linalg.norm(data[0])
    # adjoint identity through the FP64 factors
    rng = np.random.default_rng(9)
    v = torch.tensor(rng.standard_normal(len(wl.params)), device=dev)
    w = torch.tensor(rng.standard_normal((S, K, R)), device=dev)
    jv = torch.zeros((S, K, R), dtype=torch.float64, device=dev)
    jtw = torch.zeros(len(wl.params), dtype=torch.float64, device=dev)
    t.jvp(v, jv)
    t.vjp(w, jtw)
    a = float((jv * w).sum())
    b = float((v * jtw).sum())
    assert abs(a - b) <= 1e-9 * max(abs(a), abs(b))
    t.close()


def test_hex48_differentiation_workload():
    torch = _torch()
    from paper_2605_19951_amd import FP32_IR, Tem
    wl = ti.workload(3)
    ex = wl.extra
    me = wl.mesh
    S, K, R, P = wl.S, len(wl.poles.t), wl.rx.n, len(wl.params)
    dev = torch.device("cuda:0")
    print("case hex48_differentiation: 48^3, P = %d, 16 sources" % P, flush=True)
    t = Tem(0)
    t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0, torch.tensor(wl.sigma, device=dev), wl.params)
    t.analyse()
    F = torch.tensor(wl.F.T.copy(), device=dev)
    m_true = torch.tensor(ex["m_true"], device=dev)
    w = torch.tensor(ex["noise"], device=dev)

    def phi(mv):
        t.set_model(mv)
        t.factor_poles(wl.poles.xi, FP32_IR)
        d = torch.zeros((S, K, R), dtype=torch.float64, device=dev)
        t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
        return d

    d0 = phi(m_true)
    jtw = torch.zeros(P, dtype=torch.float64, device=dev)
    t.vjp(w, jtw)
    grad = jtw.cpu().numpy()
    h = ex["fd_h"]
    worst = 0.0
    for k, dirn in enumerate(ex["fd_dirs"]):
        dt = torch.tensor(dirn, device=dev)
        fp = float((phi(m_true + h * dt) * w).sum())
        fm = float((phi(m_true - h * dt) * w).sum())
        fd = (fp - fm) / (2 * h)
        worst = max(worst, abs(fd - grad @ dirn) / np.linalg.norm(grad))
    print("central differences, 32 directions: worst |fd - <J^T w, dir>| / ||J^T w|| = %.2e"
          % worst, flush=True)
    assert worst <= 1e-5
    # one Gauss-Newton step with 20 LSQR iterations from the reference model
    dh = d0.cpu().numpy()
    sd = ex["eps_r"] * np.abs(dh) + ex["eps_a"]
    d_obs = torch.tensor(dh + sd * ex["noise"], device=dev)
    wd = torch.tensor(1.0 / sd, device=dev)
    m0 = torch.tensor(ex["m0"], device=dev)
    phi(m0)
    dm = torch.zeros(P, dtype=torch.float64, device=dev)
    hist = t.gn_step(d_obs, wd, m0, torch.tensor(ex["m_ref"], device=dev), ex["lam"],
                     ex["lsqr_iters"], dm)
    assert len(hist) == 20 and np.all(np.isfinite(hist))
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    assert hist[-1] < hist[0]
    assert torch.isfinite(dm).all()
    t.close()


def test_ragged_batch_of_twelve_meshes_equals_one_at_a_time():
    torch = _torch()
    from paper_2605_19951_amd import FP32_IR, Tem
    wls = ti.ragged_batch()
    K = len(wls[0].poles.t)
    dev = torch.device("cuda:0")
    print("case ragged batch: 12 meshes 16^3 .. 40^3", flush=True)
    singles = []
    for wl in wls:
        me = wl.mesh
        t = Tem(0)
        t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0, torch.tensor(wl.sigma, device=dev),
                   wl.params)
        t.analyse()
        t.factor_poles(wl.poles.xi, FP32_IR)
        d = torch.zeros((wl.S, K, wl.rx.n), dtype=torch.float64, device=dev)
        t.forward(torch.tensor(wl.F.T.copy(), device=dev), wl.rx.ptr, wl.rx.col, wl.rx.val,
                  wl.poles.alpha, d)
        singles.append(d.cpu().numpy().reshape(-1))
        t.close()
    t = Tem(0)
    t.assemble_batch([(w.mesh.nx, w.mesh.ny, w.mesh.nz, w.mesh.h) for w in wls], ti.MU0,
                     torch.tensor(np.concatenate([w.sigma for w in wls]), device=dev))
    t.analyse()
    t.factor_poles_batch([w.poles.xi for w in wls], FP32_IR)
    F = torch.tensor(np.concatenate([w.F.T.reshape(-1) for w in wls]), device=dev)
    d = torch.zeros(sum(w.S * K * w.rx.n for w in wls), dtype=torch.float64, device=dev)
    ir = t.forward_batch(F, [w.S for w in wls], [(w.rx.ptr, w.rx.col, w.rx.val) for w in wls],
                         [w.poles.alpha for w in wls], d)
    assert ir["n_unconverged"] == 0
    db = d.cpu().numpy()
    ds = np.concatenate(singles)
    assert np.linalg.norm(db - ds) <= 1e-10 * np.linalg.norm(ds)
    # the batch's 16^3 and 18^3 meshes against the oracle run on each alone
    off = 0
    for wl in wls[:2]:
        n = wl.S * K * wl.rx.n
        o = _oracle(wl)
        dref, cond = o.data(), o.data_condition()
        dm = db[off:off + n].reshape(dref.shape)
        assert np.all(np.abs(dm - dref) <= 1e-6 * cond + 1e-300), wl.name
        off += n
    t.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("golden file %s not written (tests/golden/make_*.py)" % name)
    return np.load(path)


@pytest.mark.parametrize("prec", [0, 1])
def test_hex32_workload_against_oracle_outputs(prec):
    """The whole 32^3 workload (12 poles, 4 sources, 40 times) against the
    oracle's stored outputs (tests/golden/make_hex32_fp64.py): Q g of every
    pole and source, the data at every time within tol * the summation
    condition, J v and J^T w normwise; tol 1e-9 with FP64 factors, 1e-6 with
    FP32 factors and refinement."""
    torch = _torch()
    sys.path.insert(0, GOLDEN)
    from make_hex32_fp64 import seeded_vectors
    from paper_2605_19951_amd import Tem
    g = _golden("hex32_fp64.npz")
    wl = ti.workload(1)
    me = wl.mesh
    m, S, K, R, P = len(wl.poles.xi), wl.S, len(wl.poles.t), wl.rx.n, len(wl.params)
    tol = 1e-9 if prec == 0 else 1e-6
    dev = torch.device("cuda:0")
    print("case hex32 golden prec=%d" % prec, flush=True)
    t = Tem(0)
    t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0, torch.tensor(wl.sigma, device=dev), wl.params)
    t.analyse()
    t.factor_poles(wl.poles.xi, prec)
    F = torch.tensor(wl.F.T.copy(), device=dev)
    d = torch.zeros((S, K, R), dtype=torch.float64, device=dev)
    ir = t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
    assert ir["n_unconverged"] == 0
    dh = d.cpu().numpy()
    assert np.all(np.abs(dh - g["d"]) <= tol * g["cond"] + 1e-300)
    for j in range(K):
        assert np.linalg.norm(dh[:, j] - g["d"][:, j]) <= tol * max(
            np.linalg.norm(g["d"][:, j]), np.linalg.norm(g["cond"][:, j]))
    G = torch.zeros((m, S, me.n_edges), dtype=torch.complex128, device=dev)
    t.solve_poles(F, G)
    o = _oracle(wl)      # assembly and observation operator only (no solves)
    Gh = G.cpu().numpy()[:, :, o.unk]
    for i in range(m):
        qg = o.Q @ Gh[i].T                                      # (R, S)
        assert np.linalg.norm(qg - g["qg"][i]) <= tol * np.linalg.norm(g["qg"][i])
    v, w = seeded_vectors(P, (S, K, R))
    jv = torch.zeros_like(d)
    jtw = torch.zeros(P, dtype=torch.float64, device=dev)
    t.jvp(torch.tensor(v, device=dev), jv)
    t.vjp(torch.tensor(w, device=dev), jtw)
    e_jv = np.linalg.norm(jv.cpu().numpy() - g["jv"]) / np.linalg.norm(g["jv"])
    e_jtw = np.linalg.norm(jtw.cpu().numpy() - g["jtw"]) / np.linalg.norm(g["jtw"])
    print("hex32 prec=%d: J v rel err %.2e, J^T w rel err %.2e" % (prec, e_jv, e_jtw), flush=True)
    assert e_jv <= tol and e_jtw <= tol
    t.close()


@pytest.mark.parametrize("prec", [1, 0])
def test_hex64_pole_against_oracle_outputs(prec):
    """One pole of the 64^3 precision workload (8 sources, 60 times) against
    the oracle's stored outputs for it (tests/golden/make_hex64_pole.py):
    Q g for all sources, that pole's data term at every time within tol * its
    summation condition, its J v term and its J^T w term (norm, two seeded
    projections and 4096 seeded cells) for the benchmark's seeded v and w;
    tol 1e-6 with FP32 factors and refinement, 1e-9 with FP64 factors."""
    torch = _torch()
    from paper_2605_19951_amd import Tem
    g = _golden("hex64_pole.npz")
    wl = ti.workload(2)
    me = wl.mesh
    i = int(g["pole"])
    S, K, R, P = wl.S, len(wl.poles.t), wl.rx.n, len(wl.params)
    tol = 1e-9 if prec == 0 else 1e-6
    xi, alpha = wl.poles.xi[i:i + 1], wl.poles.alpha[:, i:i + 1]
    dev = torch.device("cuda:0")
    print("case hex64 pole %d prec=%d" % (i, prec), flush=True)
    t = Tem(0)
    t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0, torch.tensor(wl.sigma, device=dev), wl.params)
    t.analyse()
    t.factor_poles(xi, prec)
    F = torch.tensor(wl.F.T.copy(), device=dev)
    d = torch.zeros((S, K, R), dtype=torch.float64, device=dev)
    ir = t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, alpha, d)
    assert ir["n_unconverged"] == 0
    dh = d.cpu().numpy()
    assert np.all(np.abs(dh - g["d"]) <= tol * g["cond"] + 1e-300)
    G = torch.zeros((1, S, me.n_edges), dtype=torch.complex128, device=dev)
    t.solve_poles(F, G)
    o = _oracle(wl)      # assembly and observation operator only (no solves)
    qg = o.Q @ G.cpu().numpy()[0][:, o.unk].T
    e_qg = np.linalg.norm(qg - g["qg"]) / np.linalg.norm(g["qg"])
    rng = np.random.default_rng(7)       # drawn as the benchmark draws them
    v = rng.standard_normal(P)
    w = rng.standard_normal((S, K, R))
    jv = torch.zeros_like(d)
    jtw = torch.zeros(P, dtype=torch.float64, device=dev)
    t.jvp(torch.tensor(v, device=dev), jv)
    t.vjp(torch.tensor(w, device=dev), jtw)
    jv, jtw = jv.cpu().numpy(), jtw.cpu().numpy()
    e_jv = np.linalg.norm(jv - g["jv"]) / np.linalg.norm(g["jv"])
    e_norm = abs(np.linalg.norm(jtw) - g["jtw_norm"]) / g["jtw_norm"]
    samp = jtw[g["jtw_idx"]]
    e_samp = np.linalg.norm(samp - g["jtw_sample"]) / np.linalg.norm(g["jtw_sample"])
    proj = np.random.default_rng(11)
    proj.choice(P, 4096, replace=False)           # the draw of the sample cells
    vecs = proj.standard_normal((2, P))
    e_proj = np.max(np.abs(vecs @ jtw - g["jtw_proj"]) /
                    (np.linalg.norm(vecs, axis=1) * g["jtw_norm"]))
    print("hex64 pole %d prec=%d: Q g %.2e, J v %.2e, |J^T w| %.2e, sample %.2e, proj %.2e"
          % (i, prec, e_qg, e_jv, e_norm, e_samp, e_proj), flush=True)
    assert max(e_qg, e_jv, e_norm, e_samp, e_proj) <= tol
    t.close()


def test_hex32_fp64_workload_sampled_poles_against_oracle():
    """32^3 FP64 workload (12 poles, 4 sources, 40 times): the first and last
    pole solved by the oracle (SuperLU on its own ordering) against the GPU's
    solutions of the same poles, in the quantities of the parity tests."""
    torch = _torch()
    from paper_2605_19951_amd import FP64, Tem
    wl = ti.workload(1)
    me = wl.mesh
    m, S = len(wl.poles.xi), wl.S
    dev = torch.device("cuda:0")
    print("case hex32_fp64: 32^3, 12 poles, 4 sources", flush=True)
    t = Tem(0)
    t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0, torch.tensor(wl.sigma, device=dev), wl.params)
    t.analyse()
    t.factor_poles(wl.poles.xi, FP64)
    F = torch.tensor(wl.F.T.copy(), device=dev)
    G = torch.zeros((m, S, me.n_edges), dtype=torch.complex128, device=dev)
    ir = t.solve_poles(F, G)
    assert ir["n_unconverged"] == 0
    o = _oracle(wl)
    Gh = G.cpu().numpy()[:, :, o.unk]
    for i in (0, m - 1):
        gref = o.solve(i, o.F)                                  # (N, S)
        g = Gh[i].T
        assert np.linalg.norm(o.Q @ (g - gref)) <= 1e-9 * np.linalg.norm(o.Q @ gref)
        dg = g - gref
        mn = np.sqrt(abs(np.sum(np.conj(dg) * (o.M @ dg))))
        mr = np.sqrt(abs(np.sum(np.conj(gref) * (o.M @ gref))))
        assert mn <= 1e-8 * mr
    t.close()
