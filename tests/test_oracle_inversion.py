"""Pins of the oracle's Gauss-Newton inversion loop (section "Optimization"):
the quadratic-model trial step, the backtracking line search, the objective's
gradient, a linear forward map where each accepted model is the closed-form
regularised least-squares solution, and the Armijo and cooling rules along a
nonlinear run.  CPU only."""
import math

import numpy as np
import pytest

import tem_inputs as ti
from oracle.inversion import Problem, invert, line_search, next_trial
from oracle.tem import OracleTEM, first_difference


def test_next_trial_is_the_minimiser_of_an_exact_quadratic():
    a, b, c = 2.0, -3.0, 5.0           # phi(s) = a + b s + c s^2, minimiser 0.3
    assert next_trial(a, b, 1.0, a + b + c) == pytest.approx(0.3, rel=1e-15)
    # the minimiser is kept in [eta/10, eta/2]
    assert next_trial(a, -0.1, 1.0, a - 0.1 + 50.0) == pytest.approx(0.1)
    assert next_trial(a, -9.0, 1.0, a - 9.0 + 5.0) == pytest.approx(0.5)
    # a concave (or linear) model halves the step
    assert next_trial(a, -1.0, 0.4, a - 0.4 - 0.1) == pytest.approx(0.2)


def test_line_search_on_a_quadratic():
    a, b, c = 1.0, -4.0, 10.0          # the full step increases phi: 7 > 1
    phi = lambda s: a + b * s + c * s * s  # noqa: E731
    ok, eta, val, trials = line_search(phi, a, b)
    assert ok and trials == 2
    assert eta == pytest.approx(0.2, rel=1e-14) and val == pytest.approx(phi(0.2), rel=1e-14)
    assert val <= a + 1e-4 * eta * b
    # a full step that meets the condition is taken at once
    ok, eta, _, trials = line_search(lambda s: a + b * s + 0.1 * s * s, a, b)
    assert ok and eta == 1.0 and trials == 1
    # no descent anywhere (phi rises although the slope says it falls): the
    # quadratic through phi(0) = a, slope -1 and phi(eta) = a + eta has its
    # minimiser at eta / 4, so the trials are 1, 1/4, 1/16; the next, 1/64,
    # is below the floor 1/32 and the step is rejected
    ok, eta, _, trials = line_search(lambda s: a + s, a, -1.0, eta_min=1.0 / 32.0)
    assert not ok and trials == 3 and eta == pytest.approx(1.0 / 16.0)


def _linear_problem(seed=3, nd=40, P=12):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((nd, P))
    wd = 1.0 / (0.1 + rng.random(nd))
    m_true = rng.standard_normal(P)
    d_obs = G @ m_true + 0.05 * rng.standard_normal(nd) / wd
    R = first_difference(3, 2, 2).toarray()
    m_ref = np.zeros(P)
    prob = Problem(lambda m: G @ m, lambda m, v: G @ v, lambda m, w: G.T @ w, R, d_obs, wd,
                   m_ref)
    return prob, G, wd, d_obs, R, m_ref


def test_gradient_of_the_objective_matches_central_differences():
    prob, G, wd, d_obs, R, m_ref = _linear_problem()
    rng = np.random.default_rng(4)
    m = rng.standard_normal(12)
    lam = 0.7
    phi = lambda x: sum(w * p for w, p in zip((1.0, lam), prob.parts(prob.forward(x), x)))  # noqa
    g = prob.gradient(m, prob.forward(m), lam)
    for _ in range(3):
        e = rng.standard_normal(12)
        h = 1e-4
        fd = (phi(m + h * e) - phi(m - h * e)) / (2 * h)
        assert fd == pytest.approx(g @ e, rel=1e-8)


def test_linear_forward_map_gives_the_regularised_least_squares_models():
    """With d(m) = G m and LSQR run to the parameter count, an accepted step is
    the minimiser of phi at that lambda; the next step at the same lambda
    cannot decrease phi, so lambda is halved, and the following accepted model
    is the minimiser at lambda/2."""
    prob, G, wd, d_obs, R, m_ref = _linear_problem()
    W2 = wd * wd

    def closed_form(lam):
        A = G.T @ (W2[:, None] * G) + lam * R.T @ R
        return np.linalg.solve(A, G.T @ (W2 * d_obs) + lam * R.T @ (R @ m_ref))

    lam0 = 2.0
    m, log = invert(prob, np.ones(12), lam0, max_gn=3, lsqr_iters=12, chi2_target=0.0)
    assert log[0]["accepted"] and log[0]["eta"] == 1.0 and log[0]["trials"] == 1
    assert [r["lam"] for r in log] == [lam0, lam0, lam0 / 2]
    assert np.linalg.norm(m - closed_form(lam0 / 2)) <= 1e-8 * np.linalg.norm(closed_form(lam0 / 2))
    # each iteration starts from the previous accepted model
    assert log[1]["phi"] == pytest.approx(log[0]["phi_new"], rel=1e-12)


def test_nonlinear_run_keeps_the_armijo_and_cooling_rules():
    """d(m) = arctan(G m) from a start where the linearisation overshoots
    (backtracking needed) with a heavy initial regularisation (cooling
    needed) down to chi^2 <= 1."""
    rng = np.random.default_rng(6)
    nd, P = 60, 12
    G = 0.5 * rng.standard_normal((nd, P))
    m_true = 0.3 * rng.standard_normal(P)
    d_obs = np.arctan(G @ m_true) + 0.01 * rng.standard_normal(nd)
    wd = np.full(nd, 100.0)
    R = first_difference(3, 2, 2).toarray()
    prob = Problem(lambda m: np.arctan(G @ m), lambda m, v: (G @ v) / (1 + (G @ m) ** 2),
                   lambda m, w: G.T @ (w / (1 + (G @ m) ** 2)), R, d_obs, wd, np.zeros(P))
    m, log = invert(prob, 3.0 * np.ones(P), 1000.0, max_gn=25, lsqr_iters=6, chi2_target=1.0)
    assert any(r.get("trials", 1) > 1 for r in log)          # backtracking was needed
    assert log[-1]["lam"] < 1000.0                          # lambda was cooled
    assert log[-1].get("stop") == "chi2" and log[-1]["chi2"] <= 1.0
    for k, r in enumerate(log[:-1]):
        assert r["slope"] < 0.0
        if r["accepted"]:
            assert r["phi_new"] <= r["phi"] + 1e-4 * r["eta"] * r["slope"]
        cooled = (not r["accepted"]) or (r["phi"] - r["phi_new"]) < 1e-2 * r["phi"]
        assert log[k + 1]["lam"] == (r["lam"] / 2 if cooled else r["lam"])


def test_small_tem_inversion_decreases_the_misfit():
    """The loop on the oracle's TEM forward map (10^3 mesh, 4 x 4 receivers):
    three Gauss-Newton iterations from a half-space lower chi^2."""
    wl = ti.smooth_workload(10, 2, S=1, m=5, K=6, g=4, seed=41)
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
    prob = Problem(fwd, jv, jtw, R, d_obs, 1.0 / sd, m0)
    m, log = invert(prob, m0, 1.0, max_gn=3, lsqr_iters=8)
    assert log[-1].get("phi_new", log[-1]["phi"]) < log[0]["phi"]
    assert all(r["slope"] < 0 for r in log if "slope" in r)
