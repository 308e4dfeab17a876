"""Gauss-Newton inversion with backtracking line search and lambda cooling
(FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Optimization": at iteration nu the update dm solves the linearised
least-squares problem by LSQR; a backtracking line search starts from the
full step eta = 1 and shrinks eta until the Armijo condition

    phi(m + eta dm) <= phi(m) + c1 eta grad phi(m)^T dm,   c1 = 1e-4,

holds, with a lower bound on eta; a quadratic model of phi along dm (from
phi(0), its slope and phi at the last trial) proposes the next trial; the
regularisation weight lambda is kept while the objective still decreases and
halved once it stops decreasing, unless the data fit has reached
chi^2 ~ 1.  Here

    phi(m) = ||W_d (d(m) - d_obs)||^2 + lambda ||R (m - m_ref)||^2,
    grad phi(m) = 2 (J^T W_d^2 (d(m) - d_obs) + lambda R^T R (m - m_ref)),
    chi^2 = ||W_d (d(m) - d_obs)||^2 / n_data.

Readings (the paper gives the rules, not the constants): the next trial is
the minimiser of the quadratic through phi(0), phi'(0) and phi(eta), kept
in [eta/10, eta/2] (plain halving when the quadratic is not convex); eta is
not taken below eta_min: if no trial down to eta_min meets the Armijo
condition the step is rejected, m stays, and lambda is halved; an accepted
step whose relative decrease of phi is below conv_rtol also counts as
convergence at this lambda and halves it.

Pins: tests/test_oracle_inversion.py (a linear forward map, where an accepted
step is the closed-form regularised least-squares model; an exactly quadratic
line function, where the first interpolated trial is its exact minimiser;
the Armijo inequality and the cooling rule along a nonlinear run).
"""
from __future__ import annotations

import numpy as np

from .tem import lsqr


def next_trial(phi0, slope, eta, phi_eta):
    """Next step length after a failed trial at eta: the minimiser of the
    quadratic q(s) = phi0 + slope s + c s^2 with q(eta) = phi_eta, kept in
    [eta/10, eta/2]; eta/2 when c <= 0."""
    c = (phi_eta - phi0 - slope * eta) / (eta * eta)
    if not c > 0.0:
        return 0.5 * eta
    s = -slope / (2.0 * c)
    return min(max(s, 0.1 * eta), 0.5 * eta)


def line_search(phi_at, phi0, slope, c1=1e-4, eta_min=1.0 / 32.0):
    """Backtracking from eta = 1 until phi_at(eta) <= phi0 + c1 eta slope.
    Returns (accepted, eta, phi(eta), trials); when no eta >= eta_min is
    accepted, accepted is False and eta, phi are those of the last trial."""
    eta = 1.0
    trials = 0
    while True:
        val = phi_at(eta)
        trials += 1
        if val <= phi0 + c1 * eta * slope:
            return True, eta, val, trials
        nxt = next_trial(phi0, slope, eta, val)
        if nxt < eta_min:
            return False, eta, val, trials
        eta = nxt


class Problem:
    """The pieces of the objective: forward(m) -> d (flat), jvp(m, v),
    vjp(m, w) (flat data vectors), R (sparse or dense first differences)."""

    def __init__(self, forward, jvp, vjp, R, d_obs, wd, m_ref):
        self.forward, self.jvp, self.vjp, self.R = forward, jvp, vjp, R
        self.d_obs = np.asarray(d_obs, float)
        self.wd = np.asarray(wd, float)
        self.m_ref = np.asarray(m_ref, float)

    def parts(self, d, m):
        r = self.wd * (d - self.d_obs)
        g = self.R @ (m - self.m_ref)
        return float(r @ r), float(g @ g)

    def step(self, m, d, lam, iters):
        """LSQR (reorthogonalised) on [W_d J; sqrt(lam) R] dm = -[W_d (d - d_obs);
        sqrt(lam) R (m - m_ref)]."""
        sl = np.sqrt(lam)
        nd = d.size
        b = -np.concatenate([self.wd * (d - self.d_obs), sl * (self.R @ (m - self.m_ref))])

        def mv(v):
            return np.concatenate([self.wd * self.jvp(m, v), sl * (self.R @ v)])

        def rmv(u):
            return self.vjp(m, self.wd * u[:nd]) + sl * (self.R.T @ u[nd:])

        dm, hist = lsqr(mv, rmv, b, m.size, iters, reorth=True)
        return dm, hist

    def gradient(self, m, d, lam):
        return 2.0 * (self.vjp(m, self.wd * self.wd * (d - self.d_obs)) +
                      lam * (self.R.T @ (self.R @ (m - self.m_ref))))


def invert(prob: Problem, m0, lam0, max_gn, lsqr_iters, c1=1e-4, eta_min=1.0 / 32.0,
           conv_rtol=1e-2, chi2_target=1.0):
    """Gauss-Newton iterations with line search and lambda cooling.  Returns
    the final model and one record per iteration (lambda, chi^2 and phi at
    the start, accepted, eta, trials, phi after)."""
    m = np.array(m0, float)
    lam = float(lam0)
    d = prob.forward(m)
    nd = d.size
    log = []
    for _ in range(max_gn):
        mis, reg = prob.parts(d, m)
        phi = mis + lam * reg
        chi2 = mis / nd
        if chi2 <= chi2_target:
            log.append(dict(lam=lam, chi2=chi2, phi=phi, stop="chi2"))
            break
        dm, _ = prob.step(m, d, lam, lsqr_iters)
        slope = float(prob.gradient(m, d, lam) @ dm)
        trial = {}

        def phi_at(eta):
            mt = m + eta * dm
            dt = prob.forward(mt)
            a, b = prob.parts(dt, mt)
            trial["m"], trial["d"] = mt, dt
            return a + lam * b

        ok, eta, phit, trials = line_search(phi_at, phi, slope, c1, eta_min)
        rec = dict(lam=lam, chi2=chi2, phi=phi, slope=slope, accepted=ok, eta=eta, trials=trials,
                   phi_new=phit if ok else phi)
        log.append(rec)
        if ok:
            m, d = trial["m"], trial["d"]
            if (phi - phit) < conv_rtol * phi:
                lam *= 0.5
        else:
            lam *= 0.5
    return m, log
