"""Seeded tetrahedral meshes and their survey arrays (inputs only).

Like the package root, this module holds none of the method's arithmetic:
it produces a conforming tetrahedral mesh (node coordinates and the four
nodes of every tetrahedron), the canonical edge and face numbering every
other array is expressed in, conductivities per tetrahedron, the source
right-hand sides and the receiver functionals.

Mesh recipe: an nx x ny x nz box of cubes of side h, each cube split into
six tetrahedra around its main diagonal (the Kuhn/Freudenthal subdivision,
conforming across cubes), then every node moved by a seeded uniform offset
of at most ``jitter * h`` per coordinate: nodes on the outer boundary move
only within their boundary plane(s), and nodes on the air-earth interface
plane only within that plane, so that the interface stays flat and the
loops and receivers on it stay horizontal.  The jitter makes every element
matrix different (an unstructured mesh in all but connectivity); nothing
downstream uses the cube structure.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import itertools

import numpy as np

from . import MU0, SIGMA_AIR, PoleTable, Receivers, _csr, _streams, pole_table

# the six tetrahedra of a cube: paths from corner (0,0,0) to (1,1,1) along
# the axes in every order (corner offsets as bit masks x=1, y=2, z=4)
_KUHN = []
for _perm in itertools.permutations(range(3)):
    _c, _path = 0, [0]
    for _a in _perm:
        _c |= 1 << _a
        _path.append(_c)
    _KUHN.append(tuple(_path))


@dataclass
class TetMesh:
    """Conforming tetrahedral mesh.

    xyz: (n_nodes, 3) float64 coordinates (m); tets: (n_tets, 4) int32 node
    ids.  Canonical edges are the distinct node pairs (a, b), a < b, of the
    tetrahedra sorted lexicographically, oriented from a to b; canonical
    faces are the distinct sorted node triples, sorted lexicographically.
    ``cube`` gives the cube each tetrahedron came from (for building the
    inputs only) and ``z_if`` the height of the interface plane."""
    xyz: np.ndarray
    tets: np.ndarray
    nx: int
    ny: int
    nz: int
    h: float
    n_air: int
    cube: np.ndarray
    z_if: float
    edges: np.ndarray = field(init=False)
    faces: np.ndarray = field(init=False)

    def __post_init__(self):
        t = np.sort(self.tets, axis=1)
        pairs = np.stack([t[:, [0, 0, 0, 1, 1, 2]], t[:, [1, 2, 3, 2, 3, 3]]], axis=2)
        self.edges = np.unique(pairs.reshape(-1, 2), axis=0).astype(np.int32)
        tri = np.stack([t[:, [0, 0, 0, 1]], t[:, [1, 1, 2, 2]], t[:, [2, 3, 3, 3]]], axis=2)
        self.faces = np.unique(tri.reshape(-1, 3), axis=0).astype(np.int32)
        self._keys = self.edges[:, 0].astype(np.int64) * len(self.xyz) + self.edges[:, 1]

    @property
    def n_nodes(self):
        return len(self.xyz)

    @property
    def n_tets(self):
        return len(self.tets)

    @property
    def n_edges(self):
        return len(self.edges)

    def node(self, i, j, k):
        return i + (self.nx + 1) * (j + (self.ny + 1) * k)

    def edge_id(self, a, b):
        """Canonical id of the edge between nodes a and b, and the sign of
        the direction a -> b relative to its orientation."""
        lo, hi = (a, b) if a < b else (b, a)
        key = lo * np.int64(self.n_nodes) + hi
        keys = self._keys
        pos = int(np.searchsorted(keys, key))
        if pos >= len(keys) or keys[pos] != key:
            raise KeyError((a, b))
        return pos, (1.0 if a < b else -1.0)


def kuhn_mesh(nx, ny, nz, h, n_air, jitter=0.15, rng=None):
    """The jittered six-tetrahedra-per-cube mesh of the module docstring."""
    n1 = (nx + 1, ny + 1, nz + 1)
    k_if = nz - n_air
    I, J, K = np.meshgrid(np.arange(n1[0]), np.arange(n1[1]), np.arange(n1[2]), indexing="ij")
    ijk = np.stack([I.T.reshape(-1), J.T.reshape(-1), K.T.reshape(-1)], axis=1)   # node order
    xyz = ijk.astype(float) * h
    if jitter > 0.0:
        rng = rng if rng is not None else np.random.default_rng(0)
        d = rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
        fixed = np.zeros(xyz.shape, bool)
        for a, n in enumerate((nx, ny, nz)):
            fixed[:, a] |= (ijk[:, a] == 0) | (ijk[:, a] == n)
        fixed[:, 2] |= ijk[:, 2] == k_if
        d[fixed] = 0.0
        xyz = xyz + d
    tets, cube = [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = i + nx * (j + ny * k)
                corner = [(i + (b & 1)) + n1[0] * ((j + ((b >> 1) & 1)) + n1[1] * (k + ((b >> 2) & 1)))
                          for b in range(8)]
                for path in _KUHN:
                    tets.append([corner[b] for b in path])
                    cube.append(c)
    return TetMesh(xyz, np.asarray(tets, np.int32), nx, ny, nz, float(h), n_air,
                   np.asarray(cube, np.int64), float(k_if * h))


def earth_tets(mesh: TetMesh):
    """Tetrahedra below the interface (from cubes under it), increasing."""
    k = mesh.cube // (mesh.nx * mesh.ny)
    return np.nonzero(k < mesh.nz - mesh.n_air)[0].astype(np.int32)


def sigma_from_cubes(mesh: TetMesh, sigma_cubes):
    """Conductivity per tetrahedron: that of the cube it came from."""
    return np.asarray(sigma_cubes, float)[mesh.cube]


def loop_source(mesh: TetMesh, centres, current=1.0, half=1):
    """f per loop (n_edges, S): +/- current on the edges of a square loop of
    2*half x 2*half cubes on the interface plane, counter-clockwise seen from
    +z (the line integral of the source trace against each edge function)."""
    F = np.zeros((mesh.n_edges, len(centres)))
    k = mesh.nz - mesh.n_air
    for s, (cx, cy) in enumerate(centres):
        ring = ([(i, cy - half) for i in range(cx - half, cx + half)]
                + [(cx + half, j) for j in range(cy - half, cy + half)]
                + [(i, cy + half) for i in range(cx + half, cx - half, -1)]
                + [(cx - half, j) for j in range(cy + half, cy - half, -1)])
        for p in range(len(ring)):
            a = mesh.node(*ring[p], k)
            b = mesh.node(*ring[(p + 1) % len(ring)], k)
            e, sg = mesh.edge_id(a, b)
            F[e, s] += sg * current
    return F


def bz_receivers_quads(mesh: TetMesh, quads):
    """dB_z/dt receivers on interface quadrilaterals (ci, cj) (nodes
    [ci, ci+1] x [cj, cj+1] of the interface plane, moved by the jitter but
    still horizontal): row = -(circulation of E counter-clockwise seen from
    +z) / (area of the quadrilateral), the quadrilateral mean of dB_z/dt
    (dB/dt = -curl E, Stokes, edge degrees of freedom are line integrals)."""
    k = mesh.nz - mesh.n_air
    rows = []
    for ci, cj in quads:
        ring = [mesh.node(ci, cj, k), mesh.node(ci + 1, cj, k),
                mesh.node(ci + 1, cj + 1, k), mesh.node(ci, cj + 1, k)]
        p = mesh.xyz[ring, :2]
        area = 0.5 * abs(sum(p[q, 0] * p[(q + 1) % 4, 1] - p[(q + 1) % 4, 0] * p[q, 1]
                             for q in range(4)))
        row = []
        for q in range(4):
            e, sg = mesh.edge_id(ring[q], ring[(q + 1) % 4])
            row.append((e, -sg / area))
        rows.append(row)
    r = _csr(rows)
    r.kind = "bz"
    return r


@dataclass
class TetWorkload:
    name: str
    mesh: TetMesh
    sigma: np.ndarray            # (n_tets,) float64
    F: np.ndarray                # (n_edges, S) canonical edge order
    rx: Receivers
    poles: PoleTable
    params: np.ndarray           # (P,) int32 earth tetrahedra
    mu: float = MU0
    extra: dict = field(default_factory=dict)

    @property
    def S(self):
        return self.F.shape[1]


def tet_workload(n=8, n_air=2, h=25.0, S=2, m=8, K=12, g=3, jitter=0.15, seed=11, name=None):
    """n^3 cubes (6 n^3 tetrahedra), h = 25 m, n_air air layers
    (1e-6 S/m), earth 0.01 S/m with a seeded (n/8)^3-cube block of 1 S/m
    (at least 1 cube), S loops of 2 x 2 cubes on the interface placed from
    a seeded stream, a g x g grid of dB_z/dt receivers (two-cube spacing
    around the centre), m contour poles and K times in [1e-5, 1e-2] s."""
    r_mesh, r_blk, r_src, r_noise, r_dir = _streams(seed)
    mesh = kuhn_mesh(n, n, n, h, n_air, jitter, r_mesh)
    k_if = n - n_air
    s = np.full((n, n, n), SIGMA_AIR)
    s[:k_if] = 0.01
    b = max(1, n // 8)
    i0 = int(r_blk.integers(1, n - b))
    j0 = int(r_blk.integers(1, n - b))
    k0 = int(r_blk.integers(1, max(2, k_if - b)))
    s[k0:k0 + b, j0:j0 + b, i0:i0 + b] = 1.0
    sigma = sigma_from_cubes(mesh, s.reshape(-1))
    cs = []
    for _ in range(10000):
        if len(cs) == S:
            break
        cx = int(r_src.integers(2, n - 1))
        cy = int(r_src.integers(2, n - 1))
        if all(abs(cx - a) >= 3 or abs(cy - bb) >= 3 for a, bb in cs):
            cs.append((cx, cy))
    if len(cs) < S:
        raise ValueError("cannot place %d loops on %d^3 cubes" % (S, n))
    F = loop_source(mesh, cs)
    quads = [(n // 2 + 2 * a - g, n // 2 + 2 * bq - g) for bq in range(g) for a in range(g)]
    quads = [(min(max(ci, 0), n - 1), min(max(cj, 0), n - 1)) for ci, cj in quads]
    rx = bz_receivers_quads(mesh, quads)
    wl = TetWorkload(name or "tet%d" % n, mesh, sigma, F, rx, pole_table(m, 1e-5, 1e-2, K),
                     earth_tets(mesh))
    wl.extra["rng_noise"] = r_noise
    wl.extra["rng_dir"] = r_dir
    return wl


def delaunay_workload(n_points=700, L=500.0, S=2, R=6, m=5, K=6, seed=61):
    """A mesh with no structure at all: the Delaunay tetrahedralisation
    (scipy.spatial.Delaunay, joggled input so every cell is a tetrahedron)
    of the eight corners of an L-cube and n_points seeded uniform points
    inside it.  Air (1e-6 S/m) above z = 0.8 L by tetrahedron centroid,
    earth 0.01 S/m with a 1 S/m box [0.3, 0.6] L x [0.3, 0.6] L x
    [0.4, 0.6] L; S current-element sources of unit current on seeded edges
    between interior points, R tangential-E receivers (mean field along the
    edge: e^T / length) on further such edges; m contour poles and K times in
    [1e-5, 1e-2] s.  Parameters are the earth tetrahedra."""
    import scipy.spatial as ss
    r_pts, r_src, r_rx, r_noise, r_dir = _streams(seed)
    corners = np.array([[x, y, z] for z in (0.0, L) for y in (0.0, L) for x in (0.0, L)])
    pts = np.vstack([corners, r_pts.uniform(0.02 * L, 0.98 * L, (n_points, 3))])
    tets = ss.Delaunay(pts, qhull_options="QJ").simplices.astype(np.int32)
    mesh = TetMesh(pts, tets, 0, 0, 0, float(L), 0, np.zeros(len(tets), np.int64), 0.8 * L)
    cen = pts[tets].mean(axis=1)
    sigma = np.where(cen[:, 2] > 0.8 * L, SIGMA_AIR, 0.01)
    blk = ((cen[:, 0] > 0.3 * L) & (cen[:, 0] < 0.6 * L) & (cen[:, 1] > 0.3 * L)
           & (cen[:, 1] < 0.6 * L) & (cen[:, 2] > 0.4 * L) & (cen[:, 2] < 0.6 * L))
    sigma[blk] = 1.0
    inner = np.nonzero((mesh.edges[:, 0] >= 8) & (mesh.edges[:, 1] >= 8))[0]
    pick = r_src.choice(inner, S + R, replace=False)
    F = np.zeros((mesh.n_edges, S))
    for s in range(S):
        F[pick[s], s] = 1.0
    rows = []
    for e in pick[S:]:
        a, b = mesh.edges[e]
        rows.append([(int(e), 1.0 / float(np.linalg.norm(pts[b] - pts[a])))])
    rx = _csr(rows)
    rx.kind = "edge"
    params = np.nonzero(cen[:, 2] <= 0.8 * L)[0].astype(np.int32)
    wl = TetWorkload("delaunay%d" % n_points, mesh, sigma, F, rx, pole_table(m, 1e-5, 1e-2, K),
                     params)
    wl.extra["rng_noise"] = r_noise
    wl.extra["rng_dir"] = r_dir
    return wl
