"""Poles and residues for the rational approximation of exp(-t z): RKFIT.

The method approximates u(t_j) = exp(-t_j M^{-1} K) u_0 by a rational
function of type (m-1, m) whose m poles are shared by every time t_j
(section "Rational approximation using RKFIT"):

    r_j(z) = 2 Re sum_i alpha_i^[j] / (z - xi_i),   Im xi_i > 0,

so that u(t_j) ~ 2 Re sum_i alpha_i^[j] (K - xi_i M)^{-1} f (conjugate poles
implicit through 2 Re).  The poles come from RKFIT (Berljafa & Guettel, "The
RKFIT algorithm for nonlinear rational approximation", SIAM J. Sci. Comput.
39, 2017), here for the scalar problem the paper reduces to: A = diag(z) on a
set of sample points z_k >= 0 covering the spectrum, weights b, and the
functions F_j = exp(-t_j A).

One RKFIT step, as used here.  Let q be the current denominator (the poles).
The rational Krylov space W_{m+1} = {p(A) q(A)^{-1} b : deg p <= m} holds the
candidates v = q^(A) q(A)^{-1} b for a new denominator q^; its subspace
W_m = {p(A) q(A)^{-1} b : deg p <= m-1} holds the strictly proper numerators.
If F_j b were exactly p_j(A) q^(A)^{-1} b, then F_j v = p_j(A) q(A)^{-1} b would
lie in W_m for every j.  RKFIT therefore takes the unit vector v^ in W_{m+1}
that minimises sum_j ||(I - P_m) F_j v^||^2 (P_m the orthogonal projector onto
W_m) -- a smallest singular vector -- and the roots of its q^ become the new
poles.  The step is repeated until the poles settle; the residues are then
the weighted least-squares numerators, r_j(A) b = P_m F_j b.

The spaces are spanned by partial fractions of the current poles in a real
form (b, b Re 1/(z - xi), b Im 1/(z - xi) for each conjugate pair), so the
data, the minimiser and q^ are real and the new poles again come in conjugate
pairs.  The roots of c0 + sum_k C_k / (z - P_k) are the eigenvalues of the
rank-one update diag(P) - (C / c0) 1^T.

Host-only set-up (NumPy); the tables it returns are the xi / alpha inputs of
tem_factor_poles and tem_forward.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class RationalTable:
    """r_j(z) = 2 Re sum_i alpha[j, i] / (z - xi[i]) for the times t[j].

    xi: (p,) complex, Im > 0 (the p conjugate pairs of the m = 2p poles).
    alpha: (K, p) complex.  err: (K,) largest |exp(-t_j z) - r_j(z)| over the
    check points.  info: iterations, pole changes, misfits."""
    t: np.ndarray
    xi: np.ndarray
    alpha: np.ndarray
    err: np.ndarray
    info: dict = field(default_factory=dict)

    def r(self, j, z):
        z = np.asarray(z, dtype=float)
        return 2.0 * ((1.0 / (z[..., None] - self.xi)) @ self.alpha[j]).real


def default_nodes(t, n=2000):
    """Sample points for times t: z = 0 and n log-spaced points from 1e-2/t_max
    (where exp(-t z) ~ 1 for every t) to 1e6/t_min (where it is ~ 0)."""
    t = np.asarray(t, float)
    lo, hi = 1e-2 / t.max(), 1e6 / t.min()
    return np.concatenate([[0.0], np.logspace(math.log10(lo), math.log10(hi), n)])


def initial_poles(t, n_pairs):
    """Starting poles: n_pairs points on a hyperbolic contour around the
    positive real axis (the parametrisation of Weideman & Trefethen, Math.
    Comp. 76, 2007), xi_k = conj(-mu (1 + sin(i th_k - 0.2))), th_k = (k - 1/2)
    h, mu = 0.1 / sqrt(t_min t_max), h = min(1.2, 2.5 / sqrt(n_pairs))."""
    t = np.asarray(t, float)
    mu = 0.1 / math.sqrt(t.min() * t.max())
    h = min(1.2, 2.5 / math.sqrt(n_pairs))
    th = (np.arange(1, n_pairs + 1) - 0.5) * h
    return np.conj(-mu * (1.0 + np.sin(1j * th - 0.2)))


def _real_fractions(z, xi):
    """Columns Re 1/(z - xi_i), Im 1/(z - xi_i) for each pole of a pair."""
    w = 1.0 / (z[:, None] - xi[None, :])
    out = np.empty((len(z), 2 * len(xi)))
    out[:, 0::2] = w.real
    out[:, 1::2] = w.imag
    return out


def relocate(z, b, targets, xi):
    """One RKFIT step: new pole pairs from the pairs xi.

    z (N,) sample points, b (N,) weights, targets (K, N) values F_j(z_k).
    Returns (new xi with Im > 0, sigma_min, the real roots found if any)."""
    Phi_m = b[:, None] * _real_fractions(z, xi)             # spans W_m
    Phi = np.hstack([b[:, None], Phi_m])                     # spans W_{m+1}
    Q, R = np.linalg.qr(Phi)
    Vm, _ = np.linalg.qr(Phi_m)
    blocks = []
    for f in targets:
        FQ = f[:, None] * Q
        blocks.append(FQ - Vm @ (Vm.T @ FQ))
    S = np.vstack(blocks)
    _, sv, Vt = np.linalg.svd(S, full_matrices=False)
    y = Vt[-1]
    c = np.linalg.solve(R, y)                                # coefficients in Phi
    c0 = c[0]
    a, bb = c[1::2], c[2::2]
    if not np.isfinite(c0) or abs(c0) <= 1e-14 * np.abs(c).max():
        raise ValueError("RKFIT: the new denominator lost degree (constant term ~ 0)")
    lam = _roots(c0, a, bb, xi)
    return lam[lam.imag > 0], sv[-1], lam[lam.imag == 0]


def _roots(c0, a, bb, xi):
    """Roots of g(z) = c0 + sum_k (a_k Re 1/(z - xi_k) + bb_k Im 1/(z - xi_k)).

    In complex partial fractions g = c0 + sum_k C_k/(z - xi_k) + conj(C_k)/(z -
    conj(xi_k)) with C_k = (a_k - i bb_k)/2, whose roots are the eigenvalues of
    diag(P) - (C / c0) 1^T (P the poles).  The similarity by the blocks
    [[1, 1], [-i, i]] / sqrt 2 of each conjugate pair makes that matrix real:
    the blocks [[Re xi_k, -Im xi_k], [Im xi_k, Re xi_k]] on the diagonal, minus
    u e^T, where u holds (a_k, -bb_k) / c0 in the two rows of pair k and e is
    1 in the first column of every pair and 0 in the second.  A real matrix
    has exactly conjugate complex eigenvalues and exactly real ones."""
    p = len(xi)
    Mr = np.zeros((2 * p, 2 * p))
    for k, x in enumerate(xi):
        Mr[2 * k:2 * k + 2, 2 * k:2 * k + 2] = [[x.real, -x.imag], [x.imag, x.real]]
    u = np.empty(2 * p)
    u[0::2] = a / c0
    u[1::2] = -bb / c0
    Mr[:, 0::2] -= u[:, None]
    return np.linalg.eigvals(Mr)


def residues(z, b, targets, xi):
    """Weighted least-squares numerators for the poles xi: alpha (K, p)."""
    Phi_m = b[:, None] * _real_fractions(z, xi)
    coef, *_ = np.linalg.lstsq(Phi_m, (targets * b[None, :]).T, rcond=None)
    a, bb = coef[0::2], coef[1::2]
    # a Re w + bb Im w = 2 Re[((a - i bb) / 2) w]
    return ((a - 1j * bb) / 2.0).T


def max_error(t, xi, alpha, zchk):
    R = 1.0 / (zchk[:, None] - xi[None, :])
    return np.array([np.max(np.abs(np.exp(-tj * zchk) - 2.0 * (R @ alpha[j]).real))
                     for j, tj in enumerate(t)])


def misfit(z, b, targets, xi, alpha):
    """Relative least-squares misfit sqrt(sum_j ||b (F_j - r_j)||^2 / sum_j
    ||b F_j||^2) on the sample points: the quantity RKFIT minimises."""
    R = 1.0 / (z[:, None] - xi[None, :])
    fit = 2.0 * (R @ alpha.T).real.T
    return float(np.linalg.norm(b * (targets - fit)) / np.linalg.norm(b * targets))


def rkfit(z, targets, xi0, weights=None, max_iter=10, tol=1e-10):
    """RKFIT for real functions sampled at real points z with common poles.

    z        (N,) sample points (real; no pole may lie on them).
    targets  (K, N) real values F_j(z_k).
    xi0      (p,) starting poles, Im > 0 (m = 2 p poles with the conjugates).
    weights  (N,) positive weights b (default: ones).
    Returns (xi, alpha, info): poles (p,) with Im > 0 sorted by modulus,
    residues (K, p) with F_j(z) ~ 2 Re sum_i alpha[j, i] / (z - xi[i]), and
    info.  Runs up to max_iter relocation steps and keeps the iterate (the
    start included) with the smallest least-squares misfit, as RKFIT does:
    the steps may end in a cycle between iterates of similar quality rather
    than at a fixed point.  It stops early when no pole moves by more than
    tol relative to its size, or when a step's denominator has real roots
    (which the 2 Re form cannot hold) or loses degree.  info records the
    misfit of every iterate, the largest relative pole move of every step,
    the chosen step and why the loop ended."""
    from scipy.optimize import linear_sum_assignment

    z = np.asarray(z, float)
    targets = np.atleast_2d(np.asarray(targets, float))
    b = np.ones_like(z) if weights is None else np.asarray(weights, float)
    xi = np.asarray(xi0, complex)
    p = len(xi)
    if z.ndim != 1 or targets.shape[1] != len(z) or b.shape != z.shape or np.any(b <= 0):
        raise ValueError("rkfit: targets must be (K, N) over N points with N positive weights")
    if p < 1 or not np.all(xi.imag > 0):
        raise ValueError("rkfit: need at least one starting pole, all with Im > 0")
    if len(z) <= 2 * p + 1:
        raise ValueError("rkfit: need more sample points than 2 p + 1")
    alpha = residues(z, b, targets, xi)
    fits = [misfit(z, b, targets, xi, alpha)]
    best = (fits[0], 0, xi, alpha)
    moves = []
    stop = "max_iter"
    for it in range(1, max_iter + 1):
        try:
            new, _, real = relocate(z, b, targets, xi)
        except ValueError:
            stop = "degree"
            break
        if len(real) or len(new) != p:
            stop = "real poles"
            break
        C = np.abs(new[:, None] - xi[None, :]) / np.abs(xi[None, :])
        r, c = linear_sum_assignment(C)
        moves.append(float(C[r, c].max()))
        xi = new
        alpha = residues(z, b, targets, xi)
        fits.append(misfit(z, b, targets, xi, alpha))
        if fits[-1] < best[0]:
            best = (fits[-1], it, xi, alpha)
        if moves[-1] <= tol:
            stop = "converged"
            break
    _, it_best, xi, alpha = best
    order = np.argsort(np.abs(xi))
    return xi[order], alpha[:, order], dict(misfits=fits, pole_moves=moves, best_step=it_best,
                                            stop=stop)


def rkfit_exp(t, n_pairs, nodes=None, weights=None, xi0=None, max_iter=10, tol=1e-10,
              zchk=None) -> RationalTable:
    """Common poles for exp(-t_j z), j = 1..K, by RKFIT (see rkfit).

    t        (K,) times (s), > 0.
    n_pairs  number p of conjugate pole pairs (m = 2 p poles, p systems).
    nodes    sample points z >= 0 (default: default_nodes(t)).
    weights  per-node weights (default: ones).
    xi0      starting poles, Im > 0 (default: initial_poles(t, n_pairs)).
    zchk     points for the reported largest error (default: z = 0 and 8000
             log-spaced points over [1e-3 / t_max, 1e9 / t_min])."""
    t = np.asarray(t, float)
    if t.ndim != 1 or len(t) == 0 or not np.all(t > 0) or not np.all(np.isfinite(t)):
        raise ValueError("rkfit_exp: times must be a non-empty vector of positive values")
    if n_pairs < 1:
        raise ValueError("rkfit_exp: need at least one pole pair")
    z = default_nodes(t) if nodes is None else np.asarray(nodes, float)
    if np.any(z < 0):
        raise ValueError("rkfit_exp: sample points must be >= 0 (the spectrum of M^-1 K)")
    xi0 = initial_poles(t, n_pairs) if xi0 is None else np.asarray(xi0, complex)
    if len(xi0) != n_pairs:
        raise ValueError("rkfit_exp: xi0 needs n_pairs poles")
    targets = np.exp(-t[:, None] * z[None, :])
    xi, alpha, info = rkfit(z, targets, xi0, weights, max_iter, tol)
    zc = np.concatenate([[0.0], np.logspace(math.log10(1e-3 / t.max()),
                                            math.log10(1e9 / t.min()), 8000)]) \
        if zchk is None else np.asarray(zchk, float)
    err = max_error(t, xi, alpha, zc)
    return RationalTable(t=t, xi=xi, alpha=alpha, err=err, info=info)
