"""GPU checks of the differentiation path: the autograd wrapper's gradient
against central finite differences of the forward map, and one
Gauss-Newton/LSQR step against the oracle's LSQR on its own operator."""
import math

import numpy as np
import pytest

import tem_inputs as ti
from oracle.tem import OracleTEM, first_difference, gauss_newton_step

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(prec, n=12, S=2, m=6, K=6, g=2, seed=31):
    torch = _torch()
    from paper_2605_19951_amd import Tem
    from paper_2605_19951_amd.autograd import TEMProblem
    wl = ti.smooth_workload(n, 2, S=S, m=m, K=K, g=g, seed=seed)
    me = wl.mesh
    dev = torch.device("cuda:0")
    t = Tem(0)
    t.assemble(me.nx, me.ny, me.nz, me.h, ti.MU0, torch.tensor(wl.sigma, device=dev), wl.params)
    t.analyse()
    F = torch.tensor(wl.F.T.copy(), device=dev)
    prob = TEMProblem(t, F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.xi, wl.poles.alpha, prec)
    return torch, wl, t, prob, dev


@pytest.mark.parametrize("prec", [0, 1])
def test_autograd_gradient_matches_finite_differences(prec):
    torch, wl, t, prob, dev = _setup(prec)
    from paper_2605_19951_amd.autograd import tem_forward
    rng = np.random.default_rng(3)
    m0 = torch.tensor(np.log(wl.sigma[wl.params]), device=dev, requires_grad=True)
    w = torch.tensor(rng.standard_normal(prob.data_shape()), device=dev)
    d = tem_forward(m0, prob)
    (d * w).sum().backward()
    grad = m0.grad.detach().cpu().numpy()
    h = 1e-3
    for _ in range(4):
        dirn = rng.standard_normal(len(wl.params))
        dirn /= np.linalg.norm(dirn)
        dt = torch.tensor(dirn, device=dev)
        with torch.no_grad():
            fp = (tem_forward(m0.detach() + h * dt, prob) * w).sum().item()
            fm = (tem_forward(m0.detach() - h * dt, prob) * w).sum().item()
        fd = (fp - fm) / (2 * h)
        assert abs(fd - grad @ dirn) <= 1e-5 * np.linalg.norm(grad)
    t.close()


def _gn_inputs(wl, o):
    m_true = np.log(wl.sigma[wl.params])
    d_true = o.data().reshape(-1)
    noise = np.random.default_rng(4).standard_normal(d_true.shape)
    sd = 0.03 * np.abs(d_true) + 1e-9
    return m_true, d_true + noise * sd, 1.0 / sd


@pytest.mark.parametrize("prec", [0, 1])
def test_gauss_newton_step_20_iterations_matches_oracle(prec):
    """Twenty LSQR iterations on a 12^3 problem with 288 data (2 sources,
    4 x 4 receivers, 9 times) and 1,440 parameters: the library's LSQR
    reorthogonalises its v vectors, as the oracle's does here, so both stay
    within rounding of the least-squares solution over the 20-dimensional
    Krylov space (plain LSQR moves by O(1e-2) under 1e-12 perturbations of
    the operator on this problem)."""
    torch, wl, t, prob, dev = _setup(prec, n=12, S=2, m=6, K=9, g=4, seed=33)
    me = wl.mesh
    o = OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                  wl.poles.xi, wl.poles.alpha, wl.params)
    m_true, d_obs, wd = _gn_inputs(wl, o)
    assert d_obs.size == 288
    m0 = np.full(len(m_true), math.log(1e-2))
    R = first_difference(me.nx, me.ny, me.k_if)
    iters = 20
    dm_ref, hist_ref, _ = gauss_newton_step(o, m0, d_obs, wd, m0, 1.0, R, iters, reorth=True)
    mt = torch.tensor(m0, device=dev)
    t.set_model(mt)
    t.factor_poles(wl.poles.xi, prec)
    d = torch.zeros(prob.data_shape(), dtype=torch.float64, device=dev)
    t.forward(prob.F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
    dm = torch.zeros(len(m0), dtype=torch.float64, device=dev)
    shp = prob.data_shape()
    hist = t.gn_step(torch.tensor(d_obs.reshape(shp), device=dev),
                     torch.tensor(wd.reshape(shp), device=dev), mt, mt.clone(), 1.0, iters, dm)
    err = np.linalg.norm(dm.cpu().numpy() - dm_ref) / np.linalg.norm(dm_ref)
    herr = np.max(np.abs(hist - hist_ref) / np.abs(hist_ref))
    print("GN 20 its prec=%d: dm rel err %.2e, residual estimates %.2e" % (prec, err, herr),
          flush=True)
    assert err <= 1e-6
    assert herr <= 1e-6
    t.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_gauss_newton_step_matches_oracle(prec):
    """Four LSQR iterations on a 20-datum problem, and the degenerate step."""
    torch, wl, t, prob, dev = _setup(prec, n=10, S=1, m=5, K=5, g=2, seed=32)
    me = wl.mesh
    o = OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                  wl.poles.xi, wl.poles.alpha, wl.params)
    m_true = np.log(wl.sigma[wl.params])
    d_true = o.data().reshape(-1)
    noise = np.random.default_rng(4).standard_normal(d_true.shape)
    sd = 0.03 * np.abs(d_true) + 1e-9
    d_obs = d_true + noise * sd
    wd = 1.0 / sd
    m0 = np.full(len(m_true), math.log(1e-2))
    R = first_difference(me.nx, me.ny, me.k_if)
    iters = 4
    dm_ref, hist_ref, _ = gauss_newton_step(o, m0, d_obs, wd, m0, 1.0, R, iters, reorth=True)
    # GPU
    mt = torch.tensor(m0, device=dev)
    t.set_model(mt)
    t.factor_poles(wl.poles.xi, prec)
    d = torch.zeros(prob.data_shape(), dtype=torch.float64, device=dev)
    t.forward(prob.F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
    dm = torch.zeros(len(m0), dtype=torch.float64, device=dev)
    shp = prob.data_shape()
    hist = t.gn_step(torch.tensor(d_obs.reshape(shp), device=dev),
                     torch.tensor(wd.reshape(shp), device=dev), mt, mt.clone(), 1.0, iters, dm)
    tol = 1e-9 if prec == 0 else 1e-6
    assert np.linalg.norm(dm.cpu().numpy() - dm_ref) <= tol * np.linalg.norm(dm_ref)
    assert np.allclose(hist, hist_ref, rtol=10 * tol)
    # degenerate step: the model fits its own data and equals the reference,
    # so the least-squares right-hand side is zero and LSQR ends at once
    # (the oracle's LSQR does the same: tests/test_oracle_tem.py)
    dm.fill_(1.0)
    hist0 = t.gn_step(d.clone(), torch.tensor(wd.reshape(shp), device=dev), mt, mt.clone(), 1.0,
                      iters, dm)
    assert torch.count_nonzero(dm).item() == 0
    assert np.array_equal(hist0, np.zeros(iters))
    t.close()


@pytest.mark.parametrize("prec,lam0,conv,max_gn", [(0, 1.0, 0.0, 3), (1, 1.0, 0.0, 3),
                                                    (0, 3e4, 0.1, 4), (1, 3e4, 0.1, 4)])
def test_inversion_loop_matches_oracle(prec, lam0, conv, max_gn):
    """Gauss-Newton iterations with the backtracking line search and lambda
    cooling (tem_invert) against the oracle's loop on a 10^3 problem (one
    loop, 4 x 4 receivers, 6 times, 5 poles).  With lambda0 = 1 the second
    iteration backtracks (the quadratic model picks eta ~ 0.39); with
    lambda0 = 3e4 and conv_rtol = 0.1 the third iteration's small decrease
    halves lambda.  The decisions (accepted, trials, stop, lambda) must be
    equal, chi^2, phi, the slope and eta agree to 1e-6, and so does the
    final model."""
    from oracle.inversion import Problem, invert
    torch, wl, t, prob, dev = _setup(prec, n=10, S=1, m=5, K=6, g=4, seed=41)
    me = wl.mesh
    o = OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                  wl.poles.xi, wl.poles.alpha, wl.params)
    d_true = o.data().reshape(-1)
    shape = o.data().shape
    sd = 0.03 * np.abs(d_true) + 1e-9
    d_obs = d_true + sd * np.random.default_rng(2).standard_normal(d_true.shape)

    def fwd(m):
        o.set_model(m)
        return o.data().reshape(-1)

    def jv(m, v):
        o.set_model(m)
        return o.jvp(v).reshape(-1)

    def jtw(m, w):
        o.set_model(m)
        return o.vjp(w.reshape(shape))

    R = first_difference(me.nx, me.ny, me.k_if)
    m0 = np.full(len(wl.params), math.log(1e-2))
    kw = dict(conv_rtol=conv) if conv > 0 else {}
    m_fin, log_ref = invert(Problem(fwd, jv, jtw, R, d_obs, 1.0 / sd, m0), m0, lam0,
                            max_gn=max_gn, lsqr_iters=8, **kw)
    mt = torch.tensor(m0, device=dev)
    t.set_model(mt)
    t.factor_poles(wl.poles.xi, prec)
    d = torch.zeros(shape, dtype=torch.float64, device=dev)
    t.forward(prob.F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
    log = t.invert(torch.tensor(d_obs.reshape(shape), device=dev),
                   torch.tensor((1.0 / sd).reshape(shape), device=dev), mt,
                   torch.tensor(m0, device=dev), lam0, max_gn, 8, conv_rtol=conv)
    print("invert prec=%d lam0=%g: %s" % (prec, lam0, [(r["accepted"], r["trials"], r["lam"],
                                                        round(r["eta"], 4)) for r in log]),
          flush=True)
    assert len(log) == len(log_ref)
    for r, q in zip(log, log_ref):
        assert r["lam"] == q["lam"]
        assert bool(r["stop"]) == ("stop" in q)
        assert r["chi2"] == pytest.approx(q["chi2"], rel=1e-6)
        assert r["phi"] == pytest.approx(q["phi"], rel=1e-6)
        if "stop" in q:
            continue
        assert r["accepted"] == q["accepted"] and r["trials"] == q["trials"]
        assert r["slope"] == pytest.approx(q["slope"], rel=1e-6)
        assert r["eta"] == pytest.approx(q["eta"], rel=1e-6)
        assert r["phi_new"] == pytest.approx(q["phi_new"], rel=1e-6)
        assert r["seconds"] > 0 and 0 < r["factor_seconds"] <= r["seconds"]
    if lam0 == 1.0:
        assert any(r["trials"] > 1 for r in log)
    else:
        assert log[-1]["lam"] < lam0
    mg = mt.cpu().numpy()
    assert np.linalg.norm(mg - m_fin) <= 1e-6 * np.linalg.norm(m_fin)
    t.close()
