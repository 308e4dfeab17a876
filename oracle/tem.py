"""Shifted solves, time assembly, data, Jv, J^T w and LSQR (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``solve_poles``: g_is = (K - xi_i M)^{-1} f_s, the solution of each shifted
  system (Algorithm 1; "derivative of the inverse" subsection defines g_i the
  same way).  The plain definition is the solution of a linear system, so a
  library sparse LU (SuperLU, complex128) is the step that computes it, on
  the matrix permuted by the oracle's own nested-dissection ordering:
  g = P^T (P A P^T)^{-1} P f.
* ``fields`` / ``data``: u(t_j) = 2 Re sum_i alpha_i^[j] g_i (the partial
  fraction form of the rational approximation) and d_j = Q u(t_j) (section
  "The Inverse Problem"), data stacked as d[s, j, r].
* ``jvp``: J v = 2 Re sum_i alpha_i^[j] xi_i Q A_i^{-1} [dM/dm g_i v]
  (section "Jacobian computation"), with m = ln sigma so that the slice of
  dM/dm for cell c is sigma_c times the unit-conductivity element mass
  (chain rule; the paper's sentence on the slices speaks of unit
  conductivity, which is the derivative with respect to sigma itself).
* ``vjp``: J^T w = 2 Re sum_i xi_i [dM/dm g_i]^T A_i^{-1} Q^T (sum_j
  alpha_i^[j] w_j), plain transpose (A_i is complex symmetric).
* ``lsqr``: Paige & Saunders (1982) LSQR on [W_d J; sqrt(lam) R] with a
  first-difference R over faces shared by two earth cells (section
  "Optimization"; the RT0 operator of the section "Regularization" reduces
  to first differences on a uniform hex mesh up to scale and boundary
  treatment).

Pins: tests/test_oracle_tem.py (dense eigen-decomposition of the 8^3 pencil
reproduces the rational approximation exactly and the exact exponential
within the scalar error bound; conjugate-pole symmetry; divergence
invariants; SuperLU against dense LAPACK solves; adjoint test; Taylor
slopes 1 and 2; central finite differences; LSQR against SciPy's LSQR and,
after P iterations on a tiny problem, against the dense least-squares
solution, and on degenerate right-hand sides, b = 0 and A^T b = 0; the
reorthogonalised LSQR against the least-squares solution over the Krylov
space K_k(A^T A, A^T b) built densely, and against plain LSQR in its first
iterations).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import HexMesh, assemble, element_mass_unit
from .ordering import nested_dissection

MU0 = 4.0e-7 * math.pi


class OracleTEM:
    """FP64 forward map and derivatives for one mesh, conductivity and
    survey.  Inputs are the canonical-edge arrays of ``tem_inputs``."""

    def __init__(self, nx, ny, nz, h, sigma, F_edges, q_ptr, q_col, q_val,
                 xi, alpha, params, mu=MU0):
        self.mesh = HexMesh(nx, ny, nz, h)
        self.mu = mu
        self.sigma = np.asarray(sigma, float).copy()
        self.params = np.asarray(params, np.int64)
        self.xi = np.asarray(xi, complex)
        self.alpha = np.asarray(alpha, complex)            # (K, m)
        unk = self.mesh.unknown_edges()
        self.unk = unk
        self.pos = -np.ones(self.mesh.n_edges, dtype=np.int64)
        self.pos[unk] = np.arange(len(unk))
        self.F = np.asarray(F_edges, float)[unk]           # (N, S)
        R = len(q_ptr) - 1
        Qe = sp.csr_matrix((np.asarray(q_val, float), np.asarray(q_col), np.asarray(q_ptr)),
                           shape=(R, self.mesh.n_edges))
        self.Q = Qe[:, unk].tocsr()                        # (R, N)
        self.ce = self.pos[self.mesh.cell_edges()]         # (n_cells, 12)
        self.Me1 = element_mass_unit(self.mesh.h)
        self._assemble()

    # ---------------------------------------------------------------
    def _assemble(self):
        self.K, self.M = assemble(self.mesh, self.sigma, self.mu)
        self._lu = {}
        self.G = None

    def set_sigma(self, sigma):
        self.sigma = np.asarray(sigma, float).copy()
        self._assemble()

    def set_model(self, m):
        """m = ln sigma on the parameter cells; other cells unchanged."""
        s = self.sigma.copy()
        s[self.params] = np.exp(m)
        self.set_sigma(s)

    def A(self, i):
        return (self.K - self.xi[i] * self.M).astype(complex).tocsc()

    def ordering(self):
        if getattr(self, "_perm", None) is None:
            self._perm = nested_dissection(self.mesh)[1]
        return self._perm

    def lu(self, i):
        if i not in self._lu:
            p = self.ordering()
            Ap = self.A(i)[p][:, p].tocsc()
            self._lu[i] = spla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                                    options=dict(SymmetricMode=True))
        return self._lu[i]

    def solve(self, i, B):
        p = self.ordering()
        B = np.asarray(B, complex)
        x = self.lu(i).solve(B[p])
        out = np.empty_like(x)
        out[p] = x
        return out

    # ---------------------------------------------------------------
    def solve_poles(self):
        """G[i] = A_i^{-1} F, shape (m, N, S) complex."""
        self.G = np.stack([self.solve(i, self.F) for i in range(len(self.xi))])
        return self.G

    def fields(self, j):
        """u(t_j) over unknowns, (N, S)."""
        if self.G is None:
            self.solve_poles()
        return 2.0 * np.einsum("i,ins->ns", self.alpha[j], self.G).real

    def _combine(self, Y):
        """Y: (m, R, S) complex -> d[s, j, r] = 2 Re sum_i alpha_ij Y[i, r, s]."""
        return 2.0 * np.einsum("ji,irs->sjr", self.alpha, Y).real

    def _combine_condition(self, Y):
        """Summation condition c[s, j, r] = sum_i 2 |alpha_ij| |Y[i, r, s]|."""
        return 2.0 * np.einsum("ji,irs->sjr", np.abs(self.alpha), np.abs(Y))

    def observe(self, G):
        return np.stack([self.Q @ G[i] for i in range(G.shape[0])])   # (m, R, S)

    def data(self):
        if self.G is None:
            self.solve_poles()
        return self._combine(self.observe(self.G))

    def data_condition(self):
        if self.G is None:
            self.solve_poles()
        return self._combine_condition(self.observe(self.G))

    # ---------------------------------------------------------------
    def dM_apply(self, g, v):
        """(dM/dm g) v = sum_p v_p sigma_c Me1 g|_c, c = params[p]; g (N, S)."""
        N, S = g.shape
        out = np.zeros((N, S), dtype=complex)
        cells = self.params
        loc = self.ce[cells]                                  # (P, 12)
        gl = np.where(loc[:, :, None] >= 0, g[np.maximum(loc, 0)], 0.0)   # (P, 12, S)
        w = (np.asarray(v, float) * self.sigma[cells])[:, None, None]
        contrib = w * np.einsum("ab,pbs->pas", self.Me1, gl)  # (P, 12, S)
        ok = loc >= 0
        np.add.at(out, loc[ok], contrib[ok])
        return out

    def jvp(self, v):
        if self.G is None:
            self.solve_poles()
        Y = []
        for i in range(len(self.xi)):
            rhs = self.xi[i] * self.dM_apply(self.G[i], v)
            Y.append(self.Q @ self.solve(i, rhs))
        return self._combine(np.stack(Y))

    def vjp(self, w):
        """w: (S, K, R) real -> (P,) real."""
        if self.G is None:
            self.solve_poles()
        w = np.asarray(w, float)
        cells = self.params
        loc = self.ce[cells]
        ok = (loc >= 0)
        out = np.zeros(len(cells))
        for i in range(len(self.xi)):
            wt = np.einsum("j,sjr->rs", self.alpha[:, i], w)          # (R, S) complex
            lam = self.solve(i, self.Q.T @ wt)                         # (N, S)
            gl = np.where(ok[:, :, None], self.G[i][np.maximum(loc, 0)], 0.0)
            ll = np.where(ok[:, :, None], lam[np.maximum(loc, 0)], 0.0)
            bil = np.einsum("pas,ab,pbs->p", gl, self.Me1, ll)
            out += 2.0 * (self.xi[i] * bil).real
        return out * self.sigma[cells]


# ---------------------------------------------------------------------------
# regularisation and LSQR
# ---------------------------------------------------------------------------
def first_difference(nx, ny, nz_earth):
    """R: one row m_a - m_b per face shared by two earth cells a < b,
    rows ordered x-faces, y-faces, z-faces, each by the lower cell index.
    Earth cell (i, j, k) is parameter i + nx (j + ny k)."""
    rows, cols, vals = [], [], []
    r = 0

    def p(i, j, k):
        return i + nx * (j + ny * k)
    for d in range(3):
        for k in range(nz_earth):
            for j in range(ny):
                for i in range(nx):
                    i2, j2, k2 = i + (d == 0), j + (d == 1), k + (d == 2)
                    if i2 >= nx or j2 >= ny or k2 >= nz_earth:
                        continue
                    rows += [r, r]
                    cols += [p(i2, j2, k2), p(i, j, k)]
                    vals += [1.0, -1.0]
                    r += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(r, nx * ny * nz_earth))


def lsqr(matvec, rmatvec, b, n, iters, reorth=False):
    """LSQR (Paige & Saunders 1982), x0 = 0, no damping, fixed number of
    iterations.  Returns x and the per-iteration estimates of ||r||.
    When the bidiagonalisation ends (rho = 0: A^T b = 0, or the Krylov space
    is exhausted) x already solves the problem; it is returned as is and the
    remaining estimates repeat the last one.

    reorth: orthogonalise each new v against all earlier v twice (modified
    Gram-Schmidt) before normalising it (one-sided reorthogonalisation,
    Simon & Zha 2000).  In exact arithmetic the v are already orthonormal
    and the iterates are those of plain LSQR; in floating point plain LSQR
    loses that orthogonality after a few iterations on these ill-conditioned
    weighted operators, and its iterates then move by O(1) under rounding
    perturbations, while the reorthogonalised ones stay within rounding of
    the Krylov least-squares solution."""
    x = np.zeros(n)
    u = np.array(b, float)
    beta = np.linalg.norm(u)
    if beta > 0:
        u = u / beta
    v = rmatvec(u)
    alpha = np.linalg.norm(v)
    if alpha > 0:
        v = v / alpha
    w = v.copy()
    basis = [v.copy()]
    phibar = beta
    rhobar = alpha
    hist = []
    for _ in range(iters):
        u = matvec(v) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0:
            u = u / beta
        v = rmatvec(u) - beta * v
        if reorth:
            for _pass in range(2):
                for q in basis:
                    v = v - (q @ v) * q
        alpha = np.linalg.norm(v)
        if alpha > 0:
            v = v / alpha
        basis.append(v.copy())
        rho = math.hypot(rhobar, beta)
        if rho == 0.0:
            hist.extend([phibar] * (iters - len(hist)))
            break
        c = rhobar / rho
        s = beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        hist.append(phibar)
    return x, hist


def gauss_newton_step(orc: OracleTEM, m, d_obs, wd, m_ref, lam, Rmat, iters, reorth=False):
    """One Gauss-Newton update dm from LSQR on
    min || [W_d J; sqrt(lam) R] dm + [W_d (d(m) - d_obs); sqrt(lam) R (m - m_ref)] ||
    (reorth: LSQR with one-sided reorthogonalisation, see ``lsqr``)."""
    orc.set_model(m)
    d = orc.data().reshape(-1)
    sl = math.sqrt(lam)
    b = -np.concatenate([wd * (d - d_obs), sl * (Rmat @ (m - m_ref))])
    nd = d.size
    shape = orc.data().shape

    def mv(v):
        return np.concatenate([wd * orc.jvp(v).reshape(-1), sl * (Rmat @ v)])

    def rmv(u):
        return orc.vjp((wd * u[:nd]).reshape(shape)) + sl * (Rmat.T @ u[nd:])

    dm, hist = lsqr(mv, rmv, b, len(m), iters, reorth)
    return dm, hist, b
