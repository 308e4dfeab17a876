"""Pins of the RKFIT pole/residue generator (section "Rational approximation
using RKFIT"; Berljafa & Guettel's RKFIT): exact recovery of the poles of
rational data, the roots of the real partial-fraction form, the error against
the exact exponential, and a table from it driving the oracle's solves on a
small mesh within the scalar error bound.  Host-only, no GPU."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import tem_inputs as ti
from oracle.tem import OracleTEM
from paper_2605_19951_amd import rkfit


def _rational(z, xi, al):
    return 2.0 * ((1.0 / (z[:, None] - xi[None, :])) @ al.T).real.T


def test_recovers_the_poles_of_rational_data():
    # Data that are exactly 2 Re sum_i a_ji / (z - xi_i) with common poles:
    # one RKFIT step finds those poles from an unrelated start, the next
    # confirms the fixed point, and the residues are the a_ji.
    rng = np.random.default_rng(1)
    xs = np.array([-50 + 300j, 200 + 2000j, -1e3 + 1e4j, 5e3 + 8e4j])
    z = np.concatenate([[0.0], np.logspace(0, 7, 400)])
    al = rng.standard_normal((5, 4)) + 1j * rng.standard_normal((5, 4))
    F = _rational(z, xs, al)
    start = np.array([-10 + 100j, 1e2 + 1e3j, 1e3 + 1e4j, 1e4 + 1e5j])
    xi, alpha, info = rkfit.rkfit(z, F, start)
    o1 = np.argsort(np.abs(xs))
    assert np.max(np.abs(xi - xs[o1]) / np.abs(xs[o1])) <= 1e-9
    assert np.max(np.abs(alpha - al[:, o1])) <= 1e-8 * np.max(np.abs(al))
    assert info["misfits"][1] <= 1e-13
    assert info["stop"] == "converged"


def test_roots_of_the_real_partial_fraction_form():
    rng = np.random.default_rng(2)
    xi = rng.standard_normal(6) + 1j * (np.abs(rng.standard_normal(6)) + 0.1)
    a, bb, c0 = rng.standard_normal(6), rng.standard_normal(6), 0.7
    lam = rkfit._roots(c0, a, bb, xi)
    assert len(lam) == 12
    # exactly conjugate (a real matrix) ...
    up, dn = np.sort_complex(lam[lam.imag > 0]), np.sort_complex(np.conj(lam[lam.imag < 0]))
    assert len(up) + len(dn) + np.sum(lam.imag == 0) == 12
    assert np.array_equal(up, dn)
    # ... and roots of g(z) = c0 + sum_k a_k Re 1/(z - xi_k) + bb_k Im 1/(z - xi_k)
    for x in lam:
        w = 1.0 / (x - xi)
        wc = 1.0 / (x - np.conj(xi))
        g = c0 + np.sum(a * (w + wc) / 2.0 + bb * (w - wc) / 2j)
        scale = abs(c0) + np.sum((np.abs(a) + np.abs(bb)) * np.maximum(np.abs(w), np.abs(wc)))
        assert abs(g) <= 1e-12 * scale


@pytest.mark.parametrize("p", [8, 12, 16])
def test_exp_table_error_and_gain_over_the_contour(p):
    t = ti.log_times(1e-5, 1e-2, 60)
    tab = rkfit.rkfit_exp(t, p)
    assert tab.xi.shape == (p,) and tab.alpha.shape == (60, p) and np.all(tab.xi.imag > 0)
    # the reported error is the definition, evaluated here on other points
    zc = np.concatenate([[0.0], np.sort(np.random.default_rng(p).uniform(-3, 14, 20000))])
    zc[1:] = 10.0 ** zc[1:]
    err = np.array([np.max(np.abs(np.exp(-tj * zc) - tab.r(j, zc))) for j, tj in enumerate(t)])
    assert np.all(err <= 1.05 * tab.err + 1e-15)
    # near-best common poles beat the hyperbolic contour at the same count
    contour = ti.pole_table(p, 1e-5, 1e-2, 60)
    gain = {8: 1.5, 12: 3.0, 16: 10.0}[p]
    assert tab.err.max() * gain <= contour.err.max()


@pytest.mark.parametrize("p", [4, 6])
def test_real_roots_end_the_iteration_with_a_valid_table(p):
    # With few pairs a step's denominator can have real roots, which the
    # 2 Re form cannot hold: the iteration stops and returns the best
    # conjugate-pair iterate so far (the start included).
    t = ti.log_times(1e-5, 1e-2, 60)
    tab = rkfit.rkfit_exp(t, p)
    assert tab.info["stop"] == "real poles"
    assert np.all(tab.xi.imag > 0) and tab.alpha.shape == (60, p)
    fits = tab.info["misfits"]
    assert fits[tab.info["best_step"]] == min(fits)
    assert tab.err.max() <= ti.pole_table(p, 1e-5, 1e-2, 60).err.max() * 1.05


def test_rkfit_table_drives_the_oracle_within_the_scalar_bound():
    """The oracle's u(t) = 2 Re sum_i alpha_i (K - xi_i M)^{-1} f with an RKFIT
    table equals r_t(M^{-1} K) b, so its M-norm error against the exact
    exp(-t M^{-1} K) b is at most the scalar error at the pencil's eigenvalues
    times ||b||_M."""
    wl = ti.tiny_workload()
    me = wl.mesh
    t = wl.poles.t
    tab = rkfit.rkfit_exp(t, len(wl.poles.xi))
    o = OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                  tab.xi, tab.alpha, wl.params)
    lam, V = sla.eigh(o.K.toarray(), o.M.toarray())
    lam = np.maximum(lam, 0.0)
    Md = o.M.toarray()
    f = o.F[:, 0]
    b = np.linalg.solve(Md, f)
    bM = math.sqrt(b @ Md @ b)
    o.solve_poles()
    for j in (0, 7, 13, len(t) - 1):
        u = o.fields(j)[:, 0]
        u_ex = V @ (np.exp(-t[j] * lam) * (V.T @ f))
        eps = np.max(np.abs(np.exp(-t[j] * lam) - tab.r(j, lam)))
        assert eps <= tab.err[j] * 1.05 + 1e-15
        e = u - u_ex
        assert math.sqrt(e @ Md @ e) <= 1.0001 * eps * bM + 1e-12 * bM


def test_argument_checks():
    t = ti.log_times(1e-5, 1e-2, 10)
    with pytest.raises(ValueError):
        rkfit.rkfit_exp(-t, 4)
    with pytest.raises(ValueError):
        rkfit.rkfit_exp(t, 0)
    with pytest.raises(ValueError):
        rkfit.rkfit_exp(t, 2, xi0=np.array([1 - 1j, 2 + 1j]))
    with pytest.raises(ValueError):
        rkfit.rkfit(np.linspace(0, 1, 5), np.ones((1, 5)), np.array([1j, 2j]))
