"""Seeded synthetic inputs for the pole-shifted TEM solves.

This package is shared by the oracle and by the GPU path, and deliberately
holds none of the method's arithmetic (no assembly, no solves, no time
assembly, no Jacobian).  It produces the *inputs* of the forward map as the
paper states it (section "Rational approximation using RKFIT" and section
"The Inverse Problem"):

* a uniform hexahedral mesh description and the canonical edge numbering that
  every array below is expressed in;
* cell conductivities sigma (S/m), earth-cell parameter lists;
* source right-hand sides f (the discrete initial condition M u(0) = f of the
  semi-discrete system, one column per transmitter loop);
* receiver functionals Q (rows of the observation operator);
* observation times and the pole/residue table {xi_i}, {alpha_i^[j]} of the
  rational approximation, which the paper treats as precomputed data that is
  independent of the spatial discretisation.

The paper's own meshes and RKFIT tables are not available, so every workload
is synthetic; the recipes are documented with each function.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

MU0 = 4.0e-7 * math.pi          # magnetic permeability used everywhere (H/m)
SIGMA_AIR = 1.0e-6              # air conductivity (S/m)


# --------------------------------------------------------------------------
# mesh description and canonical edge numbering (input convention only)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Mesh:
    """Uniform hexahedral mesh of nx*ny*nz cubic cells of side h (metres).

    z points up; cell layer k = nz-1 is the top.  The top ``n_air`` cell
    layers are air; the air-earth interface is the node plane
    ``k_if = nz - n_air``.

    Canonical edge ids: x-edges (i,j,k), i<nx, j<=ny, k<=nz, id
    i + nx*(j + (ny+1)*k); then y-edges (i,j,k), i<=nx, j<ny, k<=nz, id
    Ex + i + (nx+1)*(j + ny*k); then z-edges (i,j,k), i<=nx, j<=ny, k<nz, id
    Ex + Ey + i + (nx+1)*(j + (ny+1)*k).  Every edge is oriented along +axis.
    Cell (i,j,k) has index i + nx*(j + ny*k).
    """
    nx: int
    ny: int
    nz: int
    h: float
    n_air: int

    @property
    def k_if(self) -> int:
        return self.nz - self.n_air

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_xedges(self) -> int:
        return self.nx * (self.ny + 1) * (self.nz + 1)

    @property
    def n_yedges(self) -> int:
        return (self.nx + 1) * self.ny * (self.nz + 1)

    @property
    def n_zedges(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * self.nz

    @property
    def n_edges(self) -> int:
        return self.n_xedges + self.n_yedges + self.n_zedges

    def xedge(self, i, j, k):
        return i + self.nx * (j + (self.ny + 1) * k)

    def yedge(self, i, j, k):
        return self.n_xedges + i + (self.nx + 1) * (j + self.ny * k)

    def zedge(self, i, j, k):
        return self.n_xedges + self.n_yedges + i + (self.nx + 1) * (j + (self.ny + 1) * k)

    def cell(self, i, j, k):
        return i + self.nx * (j + self.ny * k)


# --------------------------------------------------------------------------
# conductivity models
# --------------------------------------------------------------------------
def _place_block(rng, mesh: Mesh, b: int, margin: int):
    """Seeded lower corner of a b^3 block at least ``margin`` cells away from
    the sides, the bottom and the air-earth interface."""
    hi_x = mesh.nx - margin - b
    hi_y = mesh.ny - margin - b
    hi_z = mesh.k_if - margin - b
    if hi_x < margin or hi_y < margin or hi_z < margin:
        raise ValueError("mesh too small for the anomalous block")
    ci = int(rng.integers(margin, hi_x + 1))
    cj = int(rng.integers(margin, hi_y + 1))
    ck = int(rng.integers(margin, hi_z + 1))
    return ci, cj, ck


def sigma_block_halfspace(mesh: Mesh, rng, sigma_earth=0.01, sigma_block=1.0, b=2):
    """Half-space of ``sigma_earth`` under ``n_air`` air layers, plus one
    seeded b^3 block of ``sigma_block`` fully inside the earth."""
    s = np.full((mesh.nz, mesh.ny, mesh.nx), sigma_earth)
    s[mesh.k_if:, :, :] = SIGMA_AIR
    ci, cj, ck = _place_block(rng, mesh, b, 1)
    s[ck:ck + b, cj:cj + b, ci:ci + b] = sigma_block
    return s.reshape(-1)


def sigma_smooth_random(mesh: Mesh, rng_field, rng_block, b: int,
                        mean_log10=-2.0, sd_log10=0.5, corr_cells=4.0,
                        sigma_block=1.0):
    """log10(sigma) = mean + sd * z on earth cells, where z is white noise
    smoothed by a Gaussian filter of ``corr_cells`` cells (reflecting ends)
    and standardised to mean 0, sd 1; plus a seeded b^3 block of
    ``sigma_block`` at least two cells from the sides, the bottom and the
    interface; air cells are SIGMA_AIR."""
    from scipy.ndimage import gaussian_filter
    z = rng_field.standard_normal((mesh.k_if, mesh.ny, mesh.nx))
    z = gaussian_filter(z, sigma=corr_cells, mode="reflect")
    z = (z - z.mean()) / z.std()
    s = np.full((mesh.nz, mesh.ny, mesh.nx), SIGMA_AIR)
    s[:mesh.k_if] = 10.0 ** (mean_log10 + sd_log10 * z)
    ci, cj, ck = _place_block(rng_block, mesh, b, 2)
    s[ck:ck + b, cj:cj + b, ci:ci + b] = sigma_block
    return s.reshape(-1)


def earth_cells(mesh: Mesh) -> np.ndarray:
    """Indices (increasing) of the cells below the interface: the model
    parameters m = ln(sigma) live on these."""
    n = mesh.nx * mesh.ny * mesh.k_if
    return np.arange(n, dtype=np.int32)


# --------------------------------------------------------------------------
# sources: square loops on the interface plane
# --------------------------------------------------------------------------
def loop_edges(mesh: Mesh, cx: int, cy: int, half: int = 1):
    """Edges and signs of a square loop of 2*half x 2*half cells on node
    plane k_if spanning nodes [cx-half, cx+half] x [cy-half, cy+half],
    counter-clockwise seen from +z (the workloads use half = 1: a 2x2-cell
    loop)."""
    k = mesh.k_if
    out = []
    for i in range(cx - half, cx + half):           # y = cy-half, +x
        out.append((mesh.xedge(i, cy - half, k), +1.0))
    for j in range(cy - half, cy + half):           # x = cx+half, +y
        out.append((mesh.yedge(cx + half, j, k), +1.0))
    for i in range(cx + half - 1, cx - half - 1, -1):   # y = cy+half, -x
        out.append((mesh.xedge(i, cy + half, k), -1.0))
    for j in range(cy + half - 1, cy - half - 1, -1):   # x = cx-half, -y
        out.append((mesh.yedge(cx - half, j, k), -1.0))
    return out


def seeded_loop_centres(mesh: Mesh, rng, n_loops: int, margin=3):
    """Centres at least ``margin`` nodes from the sides; two loops differ by
    at least 3 nodes in x or in y, so their edges never overlap."""
    cs = []
    tries = 0
    while len(cs) < n_loops:
        tries += 1
        if tries > 100000:
            raise RuntimeError("cannot place loops")
        cx = int(rng.integers(margin, mesh.nx - margin + 1))
        cy = int(rng.integers(margin, mesh.ny - margin + 1))
        if all(abs(cx - a) >= 3 or abs(cy - b) >= 3 for a, b in cs):
            cs.append((cx, cy))
    return cs


def source_matrix(mesh: Mesh, centres, current=1.0, half=1):
    """f for each loop as a dense (n_edges, S) float64 array in canonical
    edge numbering: +/- current on loop edges (the line integral of the
    source trace against each edge basis function), zero elsewhere.  Loops
    have 2*half x 2*half cells."""
    F = np.zeros((mesh.n_edges, len(centres)))
    for s, (cx, cy) in enumerate(centres):
        for e, sg in loop_edges(mesh, cx, cy, half):
            F[e, s] += sg * current
    return F


# --------------------------------------------------------------------------
# receivers: rows of the observation operator Q (canonical edge columns)
# --------------------------------------------------------------------------
@dataclass
class Receivers:
    """Observation operator as CSR over canonical edges (R rows)."""
    ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    kind: str

    @property
    def n(self) -> int:
        return len(self.ptr) - 1

    def dense(self, n_edges):
        Q = np.zeros((self.n, n_edges))
        for r in range(self.n):
            for p in range(self.ptr[r], self.ptr[r + 1]):
                Q[r, self.col[p]] += self.val[p]
        return Q


def _csr(rows):
    ptr = [0]
    col, val = [], []
    for row in rows:
        for c, v in row:
            col.append(c)
            val.append(v)
        ptr.append(len(col))
    return Receivers(np.asarray(ptr, np.int64), np.asarray(col, np.int32),
                     np.asarray(val, np.float64), "")


def edge_receivers_at(mesh: Mesh, edges):
    """Tangential-E receivers: mean field along each given edge (row =
    e^T / h, since the degree of freedom is the line integral)."""
    r = _csr([[(int(e), 1.0 / mesh.h)] for e in edges])
    r.kind = "edge"
    return r


def edge_receivers(mesh: Mesh):
    """Five tangential-E receivers: mean field along y-edges on the
    interface plane (row = e^T / h) at j = ny/2-1 and i in {1, 2, nx-2,
    nx-1}, plus the y-edge at i = nx-2 one layer below the interface."""
    j = mesh.ny // 2 - 1
    k = mesh.k_if
    es = [mesh.yedge(i, j, k) for i in (1, 2, mesh.nx - 2, mesh.nx - 1)]
    es.append(mesh.yedge(mesh.nx - 2, j, k - 1))
    return edge_receivers_at(mesh, es)


def bz_receivers_at(mesh: Mesh, faces):
    """dB_z/dt receivers on the given horizontal interface faces (ci, cj)
    (the face spans nodes [ci, ci+1] x [cj, cj+1] on plane k_if).  The row
    is -(circulation of E around the face, counter-clockwise from +z) / h^2,
    since dB/dt = -curl E and the edge degrees of freedom are line
    integrals: the face mean of dB_z/dt."""
    k = mesh.k_if
    w = 1.0 / (mesh.h * mesh.h)
    rows = [[(mesh.xedge(ci, cj, k), -w),
             (mesh.yedge(ci + 1, cj, k), -w),
             (mesh.xedge(ci, cj + 1, k), +w),
             (mesh.yedge(ci, cj, k), +w)] for (ci, cj) in faces]
    r = _csr(rows)
    r.kind = "bz"
    return r


def bz_receivers(mesh: Mesh, g: int):
    """g x g grid of dB_z/dt receivers on horizontal interface faces with
    two-cell spacing around the mesh centre (rows as ``bz_receivers_at``)."""
    faces = [(mesh.nx // 2 + 2 * a - g, mesh.ny // 2 + 2 * b - g)
             for b in range(g) for a in range(g)]
    return bz_receivers_at(mesh, faces)


# --------------------------------------------------------------------------
# times, poles and residues
# --------------------------------------------------------------------------
def log_times(t1, tK, K):
    return np.logspace(math.log10(t1), math.log10(tK), K)


@dataclass
class PoleTable:
    """u(t_j) ~ 2 Re sum_i alpha[j, i] (K - xi_i M)^{-1} f.

    xi: (m,) complex with Im > 0 (conjugate poles implicit through 2 Re).
    alpha: (K, m) complex.  err: (K,) max |exp(-t z) - r_t(z)| over a dense
    grid z in {0} U [1e-2, 1e13] (an a-posteriori estimate of the scalar
    approximation error for each time)."""
    t: np.ndarray
    xi: np.ndarray
    alpha: np.ndarray
    err: np.ndarray
    params: dict = field(default_factory=dict)

    def r(self, j, z):
        """Scalar rational function r_{t_j}(z) = 2 Re sum_i alpha_ij/(z - xi_i)."""
        z = np.asarray(z, dtype=float)
        R = 1.0 / (z[..., None] - self.xi)
        return 2.0 * (R @ self.alpha[j]).real


def _fit_residues(xi, t, zfit):
    R = 1.0 / (zfit[:, None] - xi[None, :])
    A = np.hstack([2.0 * R.real, -2.0 * R.imag])
    m = len(xi)
    al = np.zeros((len(t), m), complex)
    for j, tj in enumerate(t):
        sol = np.linalg.lstsq(A, np.exp(-tj * zfit), rcond=None)[0]
        al[j] = sol[:m] + 1j * sol[m:]
    return al


def _max_err(xi, al, t, zchk):
    R = 1.0 / (zchk[:, None] - xi[None, :])
    return np.array([np.max(np.abs(np.exp(-tj * zchk) - 2.0 * (R @ al[j]).real))
                     for j, tj in enumerate(t)])


def pole_table(m: int, t1: float, tK: float, K: int) -> PoleTable:
    """Poles on a hyperbolic contour enclosing the positive real axis
    (Weideman & Trefethen 2007 style), xi_k = conj(-mu (1 + sin(i th_k -
    a))), th_k = (k - 1/2) h_th, with a = 0.2 and mu = 0.1/sqrt(t1 tK);
    residues for every time by linear least squares of exp(-t z) on
    z in {0} U logspace(-1, 12, 1500).  h_th is picked from a fixed grid to
    minimise the worst error.  The paper uses RKFIT near-best poles, which
    are not available; this table stands in for them and is an input to
    both the oracle and the GPU path."""
    a = 0.2
    mu = 0.1 / math.sqrt(t1 * tK)
    t = log_times(t1, tK, K)
    zfit = np.concatenate([[0.0], np.logspace(-1, 12, 1500)])
    zchk = np.concatenate([[0.0], np.logspace(-2, 13, 6000)])
    best = None
    for hth in np.arange(0.40, 1.2001, 0.05):
        th = (np.arange(1, m + 1) - 0.5) * hth
        xi = np.conj(-mu * (1.0 + np.sin(1j * th - a)))
        al = _fit_residues(xi, t, zfit)
        err = _max_err(xi, al, t, zchk)
        if best is None or err.max() < best[0]:
            best = (err.max(), hth, xi, al, err)
    _, hth, xi, al, err = best
    return PoleTable(t=t, xi=xi, alpha=al, err=err,
                     params=dict(a=a, mu=mu, h_theta=float(hth)))


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    mesh: Mesh
    sigma: np.ndarray            # (n_cells,) float64
    F: np.ndarray                # (n_edges, S) float64, canonical edge order
    rx: Receivers
    poles: PoleTable
    params: np.ndarray           # (P,) int32 earth-cell ids
    extra: dict = field(default_factory=dict)

    @property
    def S(self):
        return self.F.shape[1]


def _streams(seed, k=5):
    ss = np.random.SeedSequence(seed).spawn(k)
    return [np.random.default_rng(s) for s in ss]


def tiny_workload(n=8, h=50.0, n_air=2, m=8, K=20, seed=1):
    """Plain-method case: n^3 cells, h = 50 m, two air layers, earth
    0.01 S/m with a seeded 2x2x2 block of 1 S/m, one centred loop, five
    tangential-E receivers, m poles, K times in [1e-5, 1e-2] s."""
    mesh = Mesh(n, n, n, h, n_air)
    r_sig, r_blk, r_src, r_noise, r_dir = _streams(seed)
    sigma = sigma_block_halfspace(mesh, r_blk)
    F = source_matrix(mesh, [(n // 2, n // 2)])
    return Workload("hex%d_fp64_plain" % n, mesh, sigma, F, edge_receivers(mesh),
                    pole_table(m, 1e-5, 1e-2, K), earth_cells(mesh))


def smooth_workload(n, n_air, S, m, K, g, seed, h=25.0, block=None, name=None):
    """n^3 cells, h = 25 m, n_air air layers, smoothed random earth with a
    seeded 1 S/m block of (n/8)^3 cells, S seeded loops, g x g dB_z/dt
    receivers, m poles and K times in [1e-5, 1e-2] s."""
    mesh = Mesh(n, n, n, h, n_air)
    r_sig, r_blk, r_src, r_noise, r_dir = _streams(seed)
    b = block if block is not None else max(1, n // 8)
    sigma = sigma_smooth_random(mesh, r_sig, r_blk, b)
    F = source_matrix(mesh, seeded_loop_centres(mesh, r_src, S))
    wl = Workload(name or "hex%d" % n, mesh, sigma, F, bz_receivers(mesh, g),
                  pole_table(m, 1e-5, 1e-2, K), earth_cells(mesh))
    wl.extra["rng_noise"] = r_noise
    wl.extra["rng_dir"] = r_dir
    return wl


def workload(index: int) -> Workload:
    """The five seeded workloads (seed = index + 1):
    0: 8^3 h=50 plain FP64 case; 1: 32^3 FP64; 2: 64^3 precision case;
    3: 48^3 differentiation case; see ``ragged_batch`` for the batch case."""
    if index == 0:
        return tiny_workload(seed=1)
    if index == 1:
        return smooth_workload(32, 4, S=4, m=12, K=40, g=4, seed=2, name="hex32_fp64")
    if index == 2:
        return smooth_workload(64, 8, S=8, m=16, K=60, g=4, seed=3, name="hex64_precision")
    if index == 3:
        wl = smooth_workload(48, 7, S=16, m=16, K=30, g=5, seed=4, name="hex48_differentiation")
        wl.extra.update(inversion_inputs(wl))
        return wl
    raise ValueError(index)


def four_block_workload(n=32, h=5.0, n_air=8, m=21, K=31, seed=6, poles=None):
    """Uniform-hex analogue of the paper's inversion example (section
    "Synthetic examples"): a 0.1 S/m half-space under n_air air layers with
    two conductive (1 S/m) and two resistive (0.01 S/m) blocks of 5 x 5 x 1
    cells (25 x 25 x 5 m at h = 5 m) whose tops lie 2 cells (10 m) below the
    surface, at the four corners of a square around the centre; one square
    loop of 8 x 8 cells (40 m) centred on the surface; a 7 x 7 grid of
    dB_z/dt receivers with 3-cell (15 m) spacing around the centre; K times
    log-spaced in [1e-6, 1e-3] s; m poles (the contour table unless ``poles``
    (a PoleTable) is given).  Parameters are all earth cells.  The paper's
    receiver grid is stated both as 7 x 7 with 15 m spacing and as spanning
    -60..60 m (which 7 stations at 15 m do not reach); the spacing is kept.
    The noise draws (for the observed data) come from the seeded stream."""
    mesh = Mesh(n, n, n, h, n_air)
    s = np.full((mesh.nz, mesh.ny, mesh.nx), SIGMA_AIR)
    s[:mesh.k_if] = 0.1
    c = n // 2
    k = mesh.k_if - 3                     # one layer, its top 2 cells below the interface
    for (i0, j0), val in (((c - 7, c - 7), 1.0), ((c + 2, c + 2), 1.0),
                          ((c + 2, c - 7), 0.01), ((c - 7, c + 2), 0.01)):
        s[k, j0:j0 + 5, i0:i0 + 5] = val
    F = source_matrix(mesh, [(c, c)], half=4)
    faces = [(c + 3 * (a - 3) - 1, c + 3 * (b - 3) - 1) for b in range(7) for a in range(7)]
    rx = bz_receivers_at(mesh, faces)
    pt = poles if poles is not None else pole_table(m, 1e-6, 1e-3, K)
    wl = Workload("hex%d_four_blocks" % n, mesh, s.reshape(-1), F, rx, pt, earth_cells(mesh))
    wl.extra["rng_noise"] = _streams(seed)[3]
    return wl


def inversion_inputs(wl: Workload, eps_r=0.03, eps_a=1e-9, n_dirs=32):
    """Inputs of one Gauss-Newton step: true model ln(sigma) on earth cells,
    starting/reference model ln(0.01), regularisation weight 1, unit-normal
    noise draws (scaled by eps_r |d| + eps_a once d is known) and unit
    random directions for the finite-difference gradient check."""
    P = len(wl.params)
    m_true = np.log(wl.sigma[wl.params])
    m0 = np.full(P, math.log(1e-2))
    R = wl.rx.n
    K = len(wl.poles.t)
    noise = wl.extra["rng_noise"].standard_normal((wl.S, K, R))
    dirs = wl.extra["rng_dir"].standard_normal((n_dirs, P))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    return dict(m_true=m_true, m0=m0, m_ref=m0.copy(), lam=1.0, eps_r=eps_r,
                eps_a=eps_a, noise=noise, fd_dirs=dirs, fd_h=1e-3, lsqr_iters=20)


def ragged_batch(seed=5):
    """Twelve meshes n = round(16 + 24 k / 11), k = 0..11, h = 25 m,
    round(n/8) air layers, S ~ U{1..4} loops, m ~ U{8..16} poles, 16
    receivers, 40 times; each mesh draws from its own substream."""
    rng = np.random.default_rng(seed)
    sizes = [int(round(16 + 24 * k / 11)) for k in range(12)]
    out = []
    for k, n in enumerate(sizes):
        S = int(rng.integers(1, 5))
        m = int(rng.integers(8, 17))
        out.append(smooth_workload(n, max(1, int(round(n / 8))), S=S, m=m, K=40, g=4,
                                   seed=seed * 1000 + k, name="hex%d_b%d" % (n, k)))
    return out


def small_ragged_batch(seed=7):
    """A ragged batch small enough for the oracle: three meshes of 12, 13
    and 14 cells per side (2 air layers), 1..3 loops, 4..7 poles, 9 times,
    3 x 3 receivers; each mesh draws from its own substream."""
    rng = np.random.default_rng(seed)
    out = []
    for k, n in enumerate((12, 13, 14)):
        S = int(rng.integers(1, 4))
        m = int(rng.integers(4, 8))
        out.append(smooth_workload(n, 2, S=S, m=m, K=9, g=3, seed=seed * 1000 + k,
                                   name="hex%d_sb%d" % (n, k)))
    return out

