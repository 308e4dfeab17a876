"""Lowest-order Nedelec edge elements and the RT0 smoothness operator on
tetrahedral meshes (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``edge_element``: the 6 x 6 element matrices of one tetrahedron for the
  section "Spatial discretization" (curl-conforming lowest-order elements
  on tetrahedra): basis of the edge from local node i to local node j is
  lambda_i grad lambda_j - lambda_j grad lambda_i (line integral 1 along
  that edge, 0 along the others), so
  M_T[(ij),(kl)] = int lambda_i lambda_k grad lambda_j . grad lambda_l - ...
  with int lambda_p lambda_q = |T| (1 + delta_pq) / 20, and
  K_T[(ij),(kl)] = (4 |T| / mu) (grad lambda_i x grad lambda_j) .
  (grad lambda_k x grad lambda_l).
* ``assemble``: K = sum_T K_T, M = sum_T sigma_T M_T over the canonical
  edges (oriented from the lower to the higher node id), restricted to the
  edges not on the outer boundary (a face of only one tetrahedron), as the
  tangential-E condition of the governing equations asks.
* ``rt0_element`` / ``rt0_regulariser``: the section "Regularization".  The
  face function of face f (opposite local node p) is s (x - x_p) / (3 |T|),
  s = +1 for the normal pointing out of T, so that its flux through f is
  s and its divergence s / |T|: D[T, f] = int_T div = s.  The lumped mass
  keeps the diagonal of the assembled RT0 mass (reading: the paper allows a
  diagonal or lumped form and fixes neither); faces are those shared by two
  parameter tetrahedra (the flux through the other faces is taken as zero),
  L = D diag(M_div)^-1 D^T and R = diag(M_div)^-1/2 D^T, one row per face
  (m_b - m_a) / sqrt(M_ff) with a < b parameter indices, so R^T R = L.
* ``OracleTetTEM``: the forward map, Jv and J^T w of ``oracle.tem`` on these
  operators (the time assembly, data, solves and Jacobian formulas are the
  same; only the element mass of each parameter cell is per tetrahedron).
  Its sparse LU uses SuperLU's own minimum-degree column ordering.

Pins (tests/test_oracle_tet.py): on each tetrahedron the local space is
exactly the fields a + b x x, so its element matrices are fixed by their
values on the six interpolants of a and b x x; the test compares them with
an independent quadrature rule exact for quadratics (vertex and edge
midpoint values), and K_T with |T| |2b|^2 / mu; the assembled forms of a
global field a + b x x with the same quadrature per tetrahedron; K G = 0
for the discrete gradient; the dB_z/dt receiver rows and the loop source
against the curl and the circulation of b x x; RT0 element matrices on the
fields a + c x (exact quadrature) and D by the divergence theorem; L 1 = 0;
the forward map through the adjoint identity and central finite
differences of the data in m.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .tem import OracleTEM

# local edges (i, j) of a tetrahedron, i < j in local node order
LOCAL_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
# local faces: the face opposite local node p
LOCAL_FACES = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]


def bary_gradients(x):
    """Gradients of the barycentric functions of the tetrahedron with
    vertices x (4, 3), and its volume."""
    J = np.array([x[1] - x[0], x[2] - x[0], x[3] - x[0]])
    Ji = np.linalg.inv(J)
    g = np.empty((4, 3))
    g[1:] = Ji.T
    g[0] = -g[1:].sum(axis=0)
    return g, abs(np.linalg.det(J)) / 6.0


def edge_element(x, mu):
    """(K_T, M_T with unit conductivity), both 6 x 6, local edge order and
    local orientation (local node i -> j)."""
    g, vol = bary_gradients(x)

    def ll(p, q):
        return vol * (2.0 if p == q else 1.0) / 20.0

    Me = np.zeros((6, 6))
    Ke = np.zeros((6, 6))
    for a, (i, j) in enumerate(LOCAL_EDGES):
        for b, (k, l) in enumerate(LOCAL_EDGES):
            Me[a, b] = (ll(i, k) * g[j] @ g[l] - ll(i, l) * g[j] @ g[k]
                        - ll(j, k) * g[i] @ g[l] + ll(j, l) * g[i] @ g[k])
            Ke[a, b] = 4.0 * vol / mu * np.cross(g[i], g[j]) @ np.cross(g[k], g[l])
    return Ke, Me


class TetTopology:
    """Own numbering of the canonical edges and faces (must agree with the
    input convention; checked by a test), the interior edges and the edges
    and signs of every tetrahedron."""

    def __init__(self, xyz, tets):
        self.xyz = np.asarray(xyz, float)
        self.tets = np.asarray(tets, np.int64)
        nn = len(self.xyz)
        el = []
        for t in self.tets:
            for i, j in LOCAL_EDGES:
                a, b = int(t[i]), int(t[j])
                el.append((min(a, b), max(a, b)))
        self.edges = np.array(sorted(set(el)), np.int64)
        key = {tuple(e): q for q, e in enumerate(self.edges)}
        nt = len(self.tets)
        self.tet_edges = np.empty((nt, 6), np.int64)
        self.tet_signs = np.empty((nt, 6))
        for c, t in enumerate(self.tets):
            for a, (i, j) in enumerate(LOCAL_EDGES):
                p, q = int(t[i]), int(t[j])
                self.tet_edges[c, a] = key[(min(p, q), max(p, q))]
                self.tet_signs[c, a] = 1.0 if p < q else -1.0
        # faces and the tetrahedra on each side
        fl = {}
        for c, t in enumerate(self.tets):
            for p, f in enumerate(LOCAL_FACES):
                k = tuple(sorted(int(t[v]) for v in f))
                fl.setdefault(k, []).append((c, p))
        self.faces = np.array(sorted(fl), np.int64)
        self.face_tets = [fl[tuple(f)] for f in self.faces]
        bnd_edges = set()
        for f, ts in zip(self.faces, self.face_tets):
            if len(ts) == 1:
                a, b, c3 = (int(v) for v in f)
                bnd_edges.update([(a, b), (a, c3), (b, c3)])
        self.n_nodes = nn
        self.unknown = np.array([q for q, e in enumerate(self.edges)
                                 if (int(e[0]), int(e[1])) not in bnd_edges], np.int64)
        self.pos = -np.ones(len(self.edges), np.int64)
        self.pos[self.unknown] = np.arange(len(self.unknown))
        bnd_nodes = set()
        for f, ts in zip(self.faces, self.face_tets):
            if len(ts) == 1:
                bnd_nodes.update(int(v) for v in f)
        self.inner_nodes = np.array([v for v in range(nn) if v not in bnd_nodes], np.int64)

    def gradient(self):
        """Discrete gradient over all canonical edges and all nodes:
        (G phi)_e = phi_b - phi_a for e = (a, b)."""
        ne = len(self.edges)
        r = np.repeat(np.arange(ne), 2)
        c = self.edges.reshape(-1)
        v = np.tile([-1.0, 1.0], ne)
        return sp.csr_matrix((v, (r, c)), shape=(ne, self.n_nodes))


def element_matrices(topo: TetTopology, mu):
    """Per tetrahedron K_T and unit M_T in the canonical edge orientation
    (local matrices times the edge signs on both sides)."""
    nt = len(topo.tets)
    Ks = np.empty((nt, 6, 6))
    Ms = np.empty((nt, 6, 6))
    for c, t in enumerate(topo.tets):
        Ke, Me = edge_element(topo.xyz[t], mu)
        s = topo.tet_signs[c]
        Ks[c] = Ke * np.outer(s, s)
        Ms[c] = Me * np.outer(s, s)
    return Ks, Ms


def assemble_all(topo: TetTopology, sigma, mu, Ks=None, Ms=None):
    """K and M over all canonical edges (no boundary condition)."""
    if Ks is None:
        Ks, Ms = element_matrices(topo, mu)
    ne = len(topo.edges)
    r = np.repeat(topo.tet_edges, 6, axis=1).reshape(-1)
    c = np.tile(topo.tet_edges, (1, 6)).reshape(-1)
    K = sp.csr_matrix((Ks.reshape(-1), (r, c)), shape=(ne, ne))
    M = sp.csr_matrix(((Ms * np.asarray(sigma, float)[:, None, None]).reshape(-1), (r, c)),
                      shape=(ne, ne))
    return K, M


def assemble(topo: TetTopology, sigma, mu, Ks=None, Ms=None):
    """K and M restricted to the interior edges (unknown order = increasing
    canonical edge id)."""
    K, M = assemble_all(topo, sigma, mu, Ks, Ms)
    u = topo.unknown
    return K[u][:, u].tocsr(), M[u][:, u].tocsr()


# ---------------------------------------------------------------------------
# RT0 regularisation
# ---------------------------------------------------------------------------
def rt0_element(x):
    """(M_T 4 x 4, signs s_f) of the face functions s (x - x_p) / (3|T|) of
    the faces opposite local nodes p = 0..3, s = +1 (outward normal)."""
    _, vol = bary_gradients(x)
    # int_T (x - x_p).(x - x_q) dx with the exact second moments
    c = x.mean(axis=0)
    S2 = vol / 20.0 * (np.einsum("ia,ib->ab", x - c, x - c))   # int (x-c)(x-c)^T
    Me = np.empty((4, 4))
    for p in range(4):
        for q in range(4):
            dp, dq = c - x[p], c - x[q]
            Me[p, q] = (np.trace(S2) + vol * dp @ dq) / (9.0 * vol * vol)
    return Me


def rt0_regulariser(topo: TetTopology, params):
    """R (faces shared by two parameter tetrahedra x P), the lumped mass
    diagonal per face and D (P x faces)."""
    params = np.asarray(params, np.int64)
    pid = -np.ones(len(topo.tets), np.int64)
    pid[params] = np.arange(len(params))
    rows_lo, rows_hi, diag = [], [], []
    for f, ts in enumerate(topo.face_tets):
        if len(ts) != 2:
            continue
        (c1, p1), (c2, p2) = ts
        if pid[c1] < 0 or pid[c2] < 0:
            continue
        m = 0.0
        for c, p in ts:
            m += rt0_element(topo.xyz[topo.tets[c]])[p, p]
        a, b = sorted((int(pid[c1]), int(pid[c2])))
        rows_lo.append(a)
        rows_hi.append(b)
        diag.append(m)
    nf = len(diag)
    diag = np.asarray(diag)
    # D: the face's flux leaves the tetrahedron of parameter a (+1) and
    # enters that of b (-1); R row = (m_b - m_a) / sqrt(M_ff) = -D^T m / sqrt
    D = sp.csr_matrix((np.concatenate([np.ones(nf), -np.ones(nf)]),
                       (np.concatenate([rows_lo, rows_hi]), np.concatenate([np.arange(nf)] * 2))),
                      shape=(len(params), nf))
    w = 1.0 / np.sqrt(diag)
    R = sp.csr_matrix((np.concatenate([-w, w]),
                       (np.concatenate([np.arange(nf)] * 2), np.concatenate([rows_lo, rows_hi]))),
                      shape=(nf, len(params)))
    return R, diag, D, np.asarray(rows_lo), np.asarray(rows_hi)


# ---------------------------------------------------------------------------
# forward map
# ---------------------------------------------------------------------------
class OracleTetTEM(OracleTEM):
    """``OracleTEM`` on a tetrahedral mesh: sigma per tetrahedron, the
    parameters are tetrahedra, F and Q over canonical edges."""

    def __init__(self, xyz, tets, sigma, F_edges, q_ptr, q_col, q_val, xi, alpha, params, mu):
        self.topo = TetTopology(xyz, tets)
        self.mu = mu
        self.sigma = np.asarray(sigma, float).copy()
        self.params = np.asarray(params, np.int64)
        self.xi = np.asarray(xi, complex)
        self.alpha = np.asarray(alpha, complex)
        unk = self.topo.unknown
        self.unk = unk
        self.pos = self.topo.pos
        self.F = np.asarray(F_edges, float)[unk]
        ne = len(self.topo.edges)
        Qe = sp.csr_matrix((np.asarray(q_val, float), np.asarray(q_col), np.asarray(q_ptr)),
                           shape=(len(q_ptr) - 1, ne))
        self.Q = Qe[:, unk].tocsr()
        self.ce = self.pos[self.topo.tet_edges]          # (n_tets, 6), -1 on the boundary
        self.Ks, self.Ms = element_matrices(self.topo, mu)
        self._assemble()

    def _assemble(self):
        self.K, self.M = assemble(self.topo, self.sigma, self.mu, self.Ks, self.Ms)
        self._lu = {}
        self.G = None

    def lu(self, i):
        if i not in self._lu:
            self._lu[i] = spla.splu(self.A(i), permc_spec="MMD_AT_PLUS_A")
        return self._lu[i]

    def solve(self, i, B):
        return self.lu(i).solve(np.asarray(B, complex))

    def dM_apply(self, g, v):
        """(dM/dm g) v = sum_p v_p sigma_c M_c g|_c, c = params[p]."""
        N, S = g.shape
        out = np.zeros((N, S), dtype=complex)
        cells = self.params
        loc = self.ce[cells]
        gl = np.where(loc[:, :, None] >= 0, g[np.maximum(loc, 0)], 0.0)
        w = (np.asarray(v, float) * self.sigma[cells])[:, None, None]
        contrib = w * np.einsum("pab,pbs->pas", self.Ms[cells], gl)
        ok = loc >= 0
        np.add.at(out, loc[ok], contrib[ok])
        return out

    def vjp(self, w):
        if self.G is None:
            self.solve_poles()
        w = np.asarray(w, float)
        cells = self.params
        loc = self.ce[cells]
        ok = loc >= 0
        Mc = self.Ms[cells]
        out = np.zeros(len(cells))
        for i in range(len(self.xi)):
            wt = np.einsum("j,sjr->rs", self.alpha[:, i], w)
            lam = self.solve(i, self.Q.T @ wt)
            gl = np.where(ok[:, :, None], self.G[i][np.maximum(loc, 0)], 0.0)
            ll = np.where(ok[:, :, None], lam[np.maximum(loc, 0)], 0.0)
            out += 2.0 * (self.xi[i] * np.einsum("pas,pab,pbs->p", gl, Mc, ll)).real
        return out * self.sigma[cells]
