"""Lowest-order edge elements on a uniform hexahedral mesh (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the section "Spatial discretization": K u + M du/dt = 0 with K the
curl-curl stiffness (1/mu) int curl N_a . curl N_b and M the conductivity
weighted mass int sigma N_a . N_b, both restricted to the edges not on the
outer boundary (the tangential-E boundary condition of the governing
equations).  The paper uses tetrahedra; the workloads here are uniform hex
meshes with the lowest-order edge (Nedelec) element, degrees of freedom =
line integrals of E along the edges.

Pins (tests/test_oracle_fem.py): element matrices against tensor Gauss
quadrature of the explicitly written basis functions; the discrete de Rham
identities curl(grad) = 0 and K grad = 0; symmetry and definiteness of M.
Through the forward map of ``oracle.tem``, the exact whole-space step-off
transient of a square loop (closed form from the diffusion Green's function)
pins K, M, mu and the seeded source and receiver rows at two resolutions,
with an error that falls under refinement (tests/test_oracle_physics.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# local edge order in a cell: direction-major (x, y, z); within a direction
# the two transverse offsets (a, b) in order (0,0), (1,0), (0,1), (1,1), where
# for x-edges (a, b) = (dy, dz), for y-edges (dx, dz), for z-edges (dx, dy).
_AB = [(0, 0), (1, 0), (0, 1), (1, 1)]


class HexMesh:
    """Own implementation of the canonical numbering (must agree with the
    input convention; checked by a test)."""

    def __init__(self, nx, ny, nz, h):
        self.nx, self.ny, self.nz, self.h = nx, ny, nz, float(h)
        self.Ex = nx * (ny + 1) * (nz + 1)
        self.Ey = (nx + 1) * ny * (nz + 1)
        self.Ez = (nx + 1) * (ny + 1) * nz
        self.n_edges = self.Ex + self.Ey + self.Ez
        self.n_cells = nx * ny * nz

    # canonical ids ---------------------------------------------------
    def ex(self, i, j, k):
        return i + self.nx * (j + (self.ny + 1) * k)

    def ey(self, i, j, k):
        return self.Ex + i + (self.nx + 1) * (j + self.ny * k)

    def ez(self, i, j, k):
        return self.Ex + self.Ey + i + (self.nx + 1) * (j + (self.ny + 1) * k)

    def edge_geometry(self, e):
        """(direction, i, j, k) of canonical edge e."""
        if e < self.Ex:
            i = e % self.nx
            r = e // self.nx
            return 0, i, r % (self.ny + 1), r // (self.ny + 1)
        e -= self.Ex
        if e < self.Ey:
            i = e % (self.nx + 1)
            r = e // (self.nx + 1)
            return 1, i, r % self.ny, r // self.ny
        e -= self.Ey
        i = e % (self.nx + 1)
        r = e // (self.nx + 1)
        return 2, i, r % (self.ny + 1), r // (self.ny + 1)

    def is_unknown(self, e):
        d, i, j, k = self.edge_geometry(e)
        if d == 0:
            return 0 < j < self.ny and 0 < k < self.nz
        if d == 1:
            return 0 < i < self.nx and 0 < k < self.nz
        return 0 < i < self.nx and 0 < j < self.ny

    def unknown_edges(self):
        """Canonical ids of the interior edges, increasing: unknown n is
        edge unknown_edges()[n]."""
        nx, ny, nz = self.nx, self.ny, self.nz
        k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx), indexing="ij")
        mx = ((j > 0) & (j < ny) & (k > 0) & (k < nz)).reshape(-1)
        k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny), np.arange(nx + 1), indexing="ij")
        my = ((i > 0) & (i < nx) & (k > 0) & (k < nz)).reshape(-1)
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
        mz = ((i > 0) & (i < nx) & (j > 0) & (j < ny)).reshape(-1)
        return np.flatnonzero(np.concatenate([mx, my, mz])).astype(np.int64)

    def cell_edges(self):
        """(n_cells, 12) canonical edge ids in local order."""
        k, j, i = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx),
                              indexing="ij")
        i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)
        cols = []
        for a, b in _AB:
            cols.append(self.ex(i, j + a, k + b))
        for a, b in _AB:
            cols.append(self.ey(i + a, j, k + b))
        for a, b in _AB:
            cols.append(self.ez(i + a, j + b, k))
        return np.stack(cols, axis=1).astype(np.int64)

    def n_nodes(self):
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    def node(self, i, j, k):
        return i + (self.nx + 1) * (j + (self.ny + 1) * k)

    def gradient(self):
        """Discrete gradient G (n_edges x n_nodes): (G phi)_e =
        phi(end) - phi(start) for an edge oriented along +axis."""
        rows, cols, vals = [], [], []
        for e in range(self.n_edges):
            d, i, j, k = self.edge_geometry(e)
            a = self.node(i, j, k)
            b = self.node(i + (d == 0), j + (d == 1), k + (d == 2))
            rows += [e, e]
            cols += [b, a]
            vals += [1.0, -1.0]
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.n_edges, self.n_nodes()))


# ---------------------------------------------------------------------------
# element matrices (closed form)
# ---------------------------------------------------------------------------
def element_mass_unit(h):
    """int N_a . N_b over one cube of side h, unit conductivity.  For two
    edges of the same direction with transverse offsets (a,b), (a',b') the
    value is h * m(a,a') m(b,b') with the 1-D linear mass m = [[1/3,1/6],
    [1/6,1/3]]; edges of different directions are orthogonal."""
    m1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
    blk = np.zeros((4, 4))
    for p, (a, b) in enumerate(_AB):
        for q, (a2, b2) in enumerate(_AB):
            blk[p, q] = h * m1[a, a2] * m1[b, b2]
    M = np.zeros((12, 12))
    for d in range(3):
        M[4 * d:4 * d + 4, 4 * d:4 * d + 4] = blk
    return M


def face_edge_incidence():
    """6 x 12 circulation matrix C: row f = face (direction d = f // 2,
    offset f % 2 along d), +1/-1 for edges traversed with/against their
    orientation when going around the face counter-clockwise about +d.
    Stokes: (curl E) . n integrated over the face = sum_e C[f, e] u_e."""
    C = np.zeros((6, 12))

    def lx(a, b):   # x-edge, (dy, dz)
        return _AB.index((a, b))

    def ly(a, b):   # y-edge, (dx, dz)
        return 4 + _AB.index((a, b))

    def lz(a, b):   # z-edge, (dx, dy)
        return 8 + _AB.index((a, b))

    for o in (0, 1):
        # x-face at dx = o: (curl E)_x = dEz/dy - dEy/dz
        f = 0 + o
        C[f, lz(o, 1)] += 1
        C[f, lz(o, 0)] -= 1
        C[f, ly(o, 1)] -= 1
        C[f, ly(o, 0)] += 1
        # y-face at dy = o: (curl E)_y = dEx/dz - dEz/dx
        f = 2 + o
        C[f, lx(o, 1)] += 1
        C[f, lx(o, 0)] -= 1
        C[f, lz(1, o)] -= 1
        C[f, lz(0, o)] += 1
        # z-face at dz = o: (curl E)_z = dEy/dx - dEx/dy
        f = 4 + o
        C[f, ly(1, o)] += 1
        C[f, ly(0, o)] -= 1
        C[f, lx(1, o)] -= 1
        C[f, lx(0, o)] += 1
    return C


def element_stiffness(h, mu):
    """(1/mu) int curl N_a . curl N_b = (1/mu) C^T Mf C, with Mf the mass
    matrix of the unit-flux face functions n (1 - s/h)/h^2 (and s/h):
    Mf = 1/(6h) [[2,1],[1,2]] per direction.  Exact because the curl of
    every edge function is the combination sum_f C[f,e] w_f of face
    functions."""
    C = face_edge_incidence()
    Mf = np.zeros((6, 6))
    for d in range(3):
        Mf[2 * d:2 * d + 2, 2 * d:2 * d + 2] = np.array([[2.0, 1.0], [1.0, 2.0]]) / (6.0 * h)
    return (C.T @ Mf @ C) / mu


# explicit basis functions, for the quadrature pin -----------------------
def basis_values(h, x, y, z):
    """Values (12, 3) of the edge functions at local point (x,y,z) in
    [0,h]^3: x-edge (a,b) is x_hat (1/h) l_a(y) l_b(z) with l_0(s) = 1 -
    s/h, l_1(s) = s/h, and so on."""
    def l(o, s):
        return (1.0 - s / h) if o == 0 else (s / h)
    out = np.zeros((12, 3))
    for p, (a, b) in enumerate(_AB):
        out[p, 0] = l(a, y) * l(b, z) / h
        out[4 + p, 1] = l(a, x) * l(b, z) / h
        out[8 + p, 2] = l(a, x) * l(b, y) / h
    return out


def basis_curls(h, x, y, z):
    """Analytic curls (12, 3) of the edge functions."""
    def l(o, s):
        return (1.0 - s / h) if o == 0 else (s / h)

    def dl(o):
        return (-1.0 / h) if o == 0 else (1.0 / h)
    out = np.zeros((12, 3))
    for p, (a, b) in enumerate(_AB):
        # N = x_hat f(y,z)/h: curl = (0, df/dz, -df/dy)/h
        out[p, 1] = l(a, y) * dl(b) / h
        out[p, 2] = -dl(a) * l(b, z) / h
        # N = y_hat f(x,z)/h: curl = (-df/dz, 0, df/dx)/h
        out[4 + p, 0] = -l(a, x) * dl(b) / h
        out[4 + p, 2] = dl(a) * l(b, z) / h
        # N = z_hat f(x,y)/h: curl = (df/dy, -df/dx, 0)/h
        out[8 + p, 0] = l(a, x) * dl(b) / h
        out[8 + p, 1] = -dl(a) * l(b, y) / h
    return out


# ---------------------------------------------------------------------------
# global assembly
# ---------------------------------------------------------------------------
def assemble(mesh: HexMesh, sigma, mu):
    """K and M over the unknown (interior) edges, in increasing canonical
    order, as scipy CSR (FP64).  K = sum_c Ke, M = sum_c sigma_c Me1."""
    ce = mesh.cell_edges()
    unk = mesh.unknown_edges()
    pos = -np.ones(mesh.n_edges, dtype=np.int64)
    pos[unk] = np.arange(len(unk))
    Ke = element_stiffness(mesh.h, mu)
    Me = element_mass_unit(mesh.h)
    loc = pos[ce]                               # (n_cells, 12)
    ii = np.repeat(loc, 12, axis=1)             # row index per (a, b)
    jj = np.tile(loc, (1, 12))
    keep = (ii >= 0) & (jj >= 0)
    kv = np.broadcast_to(Ke.reshape(1, 144), ii.shape)
    mv = np.asarray(sigma, float)[:, None] * Me.reshape(1, 144)
    N = len(unk)
    K = sp.coo_matrix((kv[keep], (ii[keep], jj[keep])), shape=(N, N)).tocsr()
    M = sp.coo_matrix((mv[keep], (ii[keep], jj[keep])), shape=(N, N)).tocsr()
    K.sum_duplicates()
    M.sum_duplicates()
    return K, M


def element_mass_blocks(mesh: HexMesh):
    """Per cell: (n_cells, 12) unknown positions (-1 for boundary) and the
    unit-conductivity element mass, for the derivative dM/dm_c."""
    ce = mesh.cell_edges()
    unk = mesh.unknown_edges()
    pos = -np.ones(mesh.n_edges, dtype=np.int64)
    pos[unk] = np.arange(len(unk))
    return pos[ce], element_mass_unit(mesh.h)
