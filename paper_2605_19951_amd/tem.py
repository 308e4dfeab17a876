"""Thin ctypes binding of libtem (the C ABI in include/tem.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device arrays are torch tensors on the context's GPU (torch is
used for device memory and streams); host arrays are numpy arrays.  The
method names follow the C calls (tem_assemble -> Tem.assemble, ...).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libtem.so")

TEM_OK, TEM_EINVAL, TEM_ENOMEM, TEM_EDEVICE, TEM_ESTATE, TEM_EPIVOT, TEM_ENOCONV = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_IR = 0, 1
_STATUS = {0: "TEM_OK", -1: "TEM_EINVAL", -2: "TEM_ENOMEM", -3: "TEM_EDEVICE", -4: "TEM_ESTATE",
           -5: "TEM_EPIVOT", -6: "TEM_ENOCONV"}

# every entry point declared in include/tem.h
EXPORTS = ["tem_create", "tem_destroy", "tem_last_error", "tem_assemble", "tem_set_model",
           "tem_export_operators", "tem_analyse", "tem_symbolic_host", "tem_factor_poles",
           "tem_solve_poles", "tem_forward", "tem_jvp", "tem_vjp", "tem_get_stats",
           "tem_set_profiling", "tem_gn_step", "tem_assemble_batch", "tem_factor_poles_batch",
           "tem_forward_batch", "tem_autotune", "tem_autotune_level", "tem_vjp_noalloc",
           "tem_invert", "tem_set_params_batch", "tem_jvp_batch", "tem_vjp_batch",
           "tem_assemble_tet", "tem_symbolic_tet_host"]


class TemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class Mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
                ("mu", C.c_double)]


class TetMesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_tets", C.c_int64), ("xyz", C.c_void_p),
                ("tets", C.c_void_p), ("mu", C.c_double)]


class AnalyseOpts(C.Structure):
    _fields_ = [("leaf_max_cells", C.c_int32)]


class SymbolicInfo(C.Structure):
    _fields_ = [("n_unknowns", C.c_int64), ("nnz_a", C.c_int64), ("nnz_l", C.c_int64),
                ("n_rows_total", C.c_int64), ("n_supernodes", C.c_int32),
                ("n_levels", C.c_int32), ("max_front", C.c_int32), ("reserved", C.c_int32),
                ("flops_per_pole", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class FactorOpts(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_int64), ("max_group", C.c_int32),
                ("reserved", C.c_int32)]


class AutotuneReport(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("n_levels", C.c_int32),
                ("candidate_ms", C.c_double * 8), ("candidate_tile", C.c_int32 * 8),
                ("candidate_m3", C.c_int32 * 8), ("tuned_ms", C.c_double)]


class InvertOpts(C.Structure):
    _fields_ = [("lambda0", C.c_double), ("chi2_target", C.c_double), ("c1", C.c_double),
                ("eta_min", C.c_double), ("conv_rtol", C.c_double), ("max_gn", C.c_int32),
                ("lsqr_iters", C.c_int32)]


class InvertRecord(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("chi2", C.c_double), ("phi", C.c_double),
                ("slope", C.c_double), ("eta", C.c_double), ("phi_new", C.c_double),
                ("seconds", C.c_double), ("factor_seconds", C.c_double),
                ("accepted", C.c_int32), ("trials", C.c_int32), ("lsqr_iters", C.c_int32),
                ("stop", C.c_int32)]


class IrOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("reserved", C.c_int32)]


class IrStats(C.Structure):
    _fields_ = [("iters", C.POINTER(C.c_int32)), ("final_rel_res", C.POINTER(C.c_double)),
                ("n_unconverged", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_poles", C.c_int32), ("n_groups", C.c_int32), ("group_size", C.c_int32),
                ("precision", C.c_int32), ("factor_bytes", C.c_int64),
                ("workspace_bytes", C.c_int64), ("n_tiny_pivots", C.c_int32),
                ("last_solves", C.c_int32), ("factor_ms", C.c_double), ("solve_ms", C.c_double),
                ("update_ms", C.c_double), ("update_flops", C.c_double),
                ("update_launches", C.c_int64), ("sweep_ms", C.c_double),
                ("sweep_bytes", C.c_double), ("sweeps", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib_handle = None


def load_library(path: str = LIB_PATH):
    """Load libtem.so (raises if it has not been built: there is no fallback)."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(path):
        raise ImportError("libtem.so not built (%s); run __graft_entry__.build()" % path)
    L = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
    sig = {
        "tem_create": ([C.POINTER(vp), C.c_int, vp], C.c_int),
        "tem_destroy": ([vp], None),
        "tem_last_error": ([vp], C.c_char_p),
        "tem_assemble": ([vp, C.POINTER(Mesh), dp, i32, vp], C.c_int),
        "tem_set_model": ([vp, dp], C.c_int),
        "tem_export_operators": ([vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
        "tem_analyse": ([vp, C.POINTER(AnalyseOpts), C.POINTER(SymbolicInfo)], C.c_int),
        "tem_symbolic_host": ([i32, i32, i32, i32, C.POINTER(SymbolicInfo), vp, vp, vp, vp, vp],
                              C.c_int),
        "tem_factor_poles": ([vp, i32, vp, C.c_int, C.POINTER(FactorOpts)], C.c_int),
        "tem_solve_poles": ([vp, i32, dp, dp, C.POINTER(IrOpts), C.POINTER(IrStats)], C.c_int),
        "tem_forward": ([vp, i32, dp, i32, vp, vp, vp, i32, vp, C.POINTER(IrOpts), dp,
                         C.POINTER(IrStats)], C.c_int),
        "tem_jvp": ([vp, dp, dp, C.POINTER(IrOpts), C.POINTER(IrStats)], C.c_int),
        "tem_vjp": ([vp, dp, dp, C.POINTER(IrOpts), C.POINTER(IrStats)], C.c_int),
        "tem_vjp_noalloc": ([vp, dp, dp, C.POINTER(IrOpts), C.POINTER(IrStats)], C.c_int),
        "tem_get_stats": ([vp, C.POINTER(Stats)], C.c_int),
        "tem_set_profiling": ([vp, i32], C.c_int),
        "tem_gn_step": ([vp, dp, dp, dp, dp, C.c_double, i32, dp, vp, C.POINTER(IrOpts)], C.c_int),
        "tem_invert": ([vp, dp, dp, dp, dp, C.POINTER(InvertOpts), C.POINTER(IrOpts), vp,
                        C.POINTER(C.c_int32)], C.c_int),
        "tem_assemble_batch": ([vp, i32, vp, dp], C.c_int),
        "tem_assemble_tet": ([vp, C.POINTER(TetMesh), dp, i32, vp], C.c_int),
        "tem_symbolic_tet_host": ([C.POINTER(TetMesh), i32, C.POINTER(SymbolicInfo), vp, vp, vp,
                                   vp, vp], C.c_int),
        "tem_autotune": ([vp, i32, vp, C.c_int, C.POINTER(AutotuneReport)], C.c_int),
        "tem_autotune_level": ([vp, C.c_int, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
                               C.c_int),
        "tem_factor_poles_batch": ([vp, vp, vp, C.c_int, C.POINTER(FactorOpts)], C.c_int),
        "tem_set_params_batch": ([vp, vp, vp], C.c_int),
        "tem_jvp_batch": ([vp, dp, dp, C.POINTER(IrOpts), C.POINTER(IrStats)], C.c_int),
        "tem_vjp_batch": ([vp, dp, dp, C.POINTER(IrOpts), C.POINTER(IrStats)], C.c_int),
        "tem_forward_batch": ([vp, vp, dp, vp, vp, vp, vp, i32, vp, C.POINTER(IrOpts), dp,
                               C.POINTER(IrStats)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib_handle = L
    return L


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _dev(t, dtype_name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a torch tensor on the GPU")
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError("expected dtype %s, got %s" % (dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (shape, tuple(t.shape)))
    return C.c_void_p(t.data_ptr())


def symbolic_host(nx, ny, nz, leaf_max=4):
    """Host-only symbolic analysis (no GPU): dict with perm, sn_ptr,
    sn_parent, rows_ptr, rows and the info fields."""
    L = load_library()
    info = SymbolicInfo()
    st = L.tem_symbolic_host(nx, ny, nz, leaf_max, C.byref(info), None, None, None, None, None)
    if st != TEM_OK:
        raise TemError(st, "tem_symbolic_host failed")
    N, ns, nr = info.n_unknowns, info.n_supernodes, info.n_rows_total
    perm = np.zeros(N, np.int32)
    sn_ptr = np.zeros(ns + 1, np.int32)
    par = np.zeros(ns, np.int32)
    rptr = np.zeros(ns + 1, np.int64)
    rows = np.zeros(max(nr, 1), np.int32)
    st = L.tem_symbolic_host(nx, ny, nz, leaf_max, C.byref(info), perm.ctypes.data_as(C.c_void_p),
                             sn_ptr.ctypes.data_as(C.c_void_p), par.ctypes.data_as(C.c_void_p),
                             rptr.ctypes.data_as(C.c_void_p), rows.ctypes.data_as(C.c_void_p))
    if st != TEM_OK:
        raise TemError(st, "tem_symbolic_host failed")
    out = info.as_dict()
    out.update(perm=perm, sn_ptr=sn_ptr, sn_parent=par, rows_ptr=rptr, rows=rows[:nr])
    return out


def _tet_mesh(xyz, tets, mu):
    xyz, _ = _host(xyz, np.float64)
    tets, _ = _host(tets, np.int32)
    if xyz.ndim != 2 or xyz.shape[1] != 3 or tets.ndim != 2 or tets.shape[1] != 4:
        raise ValueError("expected xyz (n_nodes, 3) and tets (n_tets, 4)")
    m = TetMesh(len(xyz), len(tets), xyz.ctypes.data_as(C.c_void_p),
                tets.ctypes.data_as(C.c_void_p), mu)
    return m, (xyz, tets)


def symbolic_tet_host(xyz, tets, leaf_max=4, mu=4.0e-7 * np.pi):
    """Host-only analysis of a tetrahedral mesh (no GPU); as symbolic_host."""
    L = load_library()
    mesh, keep = _tet_mesh(xyz, tets, mu)
    info = SymbolicInfo()
    st = L.tem_symbolic_tet_host(C.byref(mesh), leaf_max, C.byref(info), None, None, None, None,
                                 None)
    if st != TEM_OK:
        raise TemError(st, "tem_symbolic_tet_host failed")
    N, ns, nr = info.n_unknowns, info.n_supernodes, info.n_rows_total
    perm = np.zeros(N, np.int32)
    sn_ptr = np.zeros(ns + 1, np.int32)
    par = np.zeros(ns, np.int32)
    rptr = np.zeros(ns + 1, np.int64)
    rows = np.zeros(max(nr, 1), np.int32)
    st = L.tem_symbolic_tet_host(C.byref(mesh), leaf_max, C.byref(info),
                                 perm.ctypes.data_as(C.c_void_p), sn_ptr.ctypes.data_as(C.c_void_p),
                                 par.ctypes.data_as(C.c_void_p), rptr.ctypes.data_as(C.c_void_p),
                                 rows.ctypes.data_as(C.c_void_p))
    if st != TEM_OK:
        raise TemError(st, "tem_symbolic_tet_host failed")
    del keep
    out = info.as_dict()
    out.update(perm=perm, sn_ptr=sn_ptr, sn_parent=par, rows_ptr=rptr, rows=rows[:nr])
    return out


class Tem:
    """One library context (one mesh, its factors and cached solutions)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.L = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("libtem needs a GPU")
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = self.L.tem_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if st != TEM_OK:
            raise TemError(st, self.L.tem_last_error(None).decode())
        self.h = h
        self.n_params = 0
        self.npole = 0
        self.S = 0

    def close(self):
        if getattr(self, "h", None):
            self.L.tem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st, allow=()):
        if st != TEM_OK and st not in allow:
            raise TemError(st, self.L.tem_last_error(self.h).decode())
        return st

    # -----------------------------------------------------------------
    def assemble(self, nx, ny, nz, h, mu, sigma, params):
        params, pp = _host(params, np.int32)
        self.mesh = Mesh(nx, ny, nz, h, mu)
        self.n_cells = nx * ny * nz
        self.n_edges = nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz
        self._chk(self.L.tem_assemble(self.h, C.byref(self.mesh), _dev(sigma, "float64", (self.n_cells,)),
                                      len(params), pp))
        self.n_params = len(params)

    def assemble_tet(self, xyz, tets, mu, sigma, params):
        """Tetrahedral mesh: xyz (n_nodes, 3), tets (n_tets, 4) host arrays,
        sigma a device float64 tensor per tetrahedron, params tetrahedron ids."""
        params, pp = _host(params, np.int32)
        mesh, keep = _tet_mesh(xyz, tets, mu)
        self.n_cells = int(mesh.n_tets)
        self._chk(self.L.tem_assemble_tet(self.h, C.byref(mesh),
                                          _dev(sigma, "float64", (self.n_cells,)), len(params), pp))
        del keep
        t = np.sort(np.asarray(tets, np.int64), axis=1)
        pairs = np.concatenate([t[:, [a, b]] for a, b in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))])
        self.n_edges = len(np.unique(pairs, axis=0))
        self.n_params = len(params)

    def set_model(self, m):
        self._chk(self.L.tem_set_model(self.h, _dev(m, "float64", (self.n_params,))))

    def analyse(self, leaf_max=4):
        info = SymbolicInfo()
        self._chk(self.L.tem_analyse(self.h, C.byref(AnalyseOpts(leaf_max)), C.byref(info)))
        self.info = info.as_dict()
        return self.info

    def export_operators(self):
        N, nnz = C.c_int64(), C.c_int64()
        self._chk(self.L.tem_export_operators(self.h, C.byref(N), C.byref(nnz), None, None, None,
                                              None, None))
        perm = np.zeros(N.value, np.int32)
        rowptr = np.zeros(N.value + 1, np.int64)
        col = np.zeros(nnz.value, np.int32)
        kv = np.zeros(nnz.value)
        mv = np.zeros(nnz.value)
        self._chk(self.L.tem_export_operators(self.h, None, None, *(a.ctypes.data_as(C.c_void_p)
                                                                   for a in (perm, rowptr, col, kv, mv))))
        return perm, rowptr, col, kv, mv

    def factor_poles(self, xi, precision=FP32_IR, mem_budget_bytes=0, max_group=0):
        xi = np.asarray(xi, complex)
        buf, bp = _host(np.stack([xi.real, xi.imag], axis=1).reshape(-1), np.float64)
        self._chk(self.L.tem_factor_poles(self.h, len(xi), bp, int(precision),
                                          C.byref(FactorOpts(int(mem_budget_bytes), int(max_group), 0))))
        self.npole = len(xi)

    @staticmethod
    def _ir(ir):
        if ir is None:
            return None
        return C.byref(IrOpts(float(ir.get("rtol", 0.0)), int(ir.get("max_iter", 0)), 0))

    def _stats_struct(self, n):
        it = np.zeros(n, np.int32)
        rr = np.zeros(n)
        s = IrStats(it.ctypes.data_as(C.POINTER(C.c_int32)), rr.ctypes.data_as(C.POINTER(C.c_double)), 0, 0)
        return s, it, rr

    def solve_poles(self, F, G=None, ir=None, allow_noconv=False):
        """F: (S, n_edges) float64 on the GPU (column s = f_s); G: optional
        (m, S, n_edges) complex128 output.  Returns IR statistics."""
        S = F.shape[0]
        s, it, rr = self._stats_struct(self.npole * S)
        st = self.L.tem_solve_poles(self.h, S, _dev(F, "float64", (S, self.n_edges)),
                                    None if G is None else _dev(G, "complex128", (self.npole, S, self.n_edges)),
                                    self._ir(ir), C.byref(s))
        self._chk(st, (TEM_ENOCONV,) if allow_noconv else ())
        self.S = S
        return dict(iters=it.reshape(self.npole, S), rel=rr.reshape(self.npole, S),
                    n_unconverged=s.n_unconverged, status=st)

    def forward(self, F, q_ptr, q_col, q_val, alpha, d, ir=None, allow_noconv=False):
        """d (S, K, R) float64 on the GPU receives 2 Re sum_i alpha_ji Q g_is."""
        S = F.shape[0]
        qp, qpp = _host(q_ptr, np.int64)
        qc, qcp = _host(q_col, np.int32)
        qv, qvp = _host(q_val, np.float64)
        alpha = np.asarray(alpha, complex)
        K = alpha.shape[0]
        al, alp = _host(np.stack([alpha.real, alpha.imag], axis=2).reshape(-1), np.float64)
        R = len(qp) - 1
        s, it, rr = self._stats_struct(self.npole * S)
        st = self.L.tem_forward(self.h, S, _dev(F, "float64", (S, self.n_edges)), R, qpp, qcp, qvp,
                                K, alp, self._ir(ir), _dev(d, "float64", (S, K, R)), C.byref(s))
        self._chk(st, (TEM_ENOCONV,) if allow_noconv else ())
        self.S, self.K, self.R = S, K, R
        return dict(iters=it.reshape(self.npole, S), rel=rr.reshape(self.npole, S),
                    n_unconverged=s.n_unconverged, status=st)

    def _dshape(self):
        return (self.S, self.K, self.R) if hasattr(self, "K") else None

    def jvp(self, v, jv, ir=None):
        s, it, rr = self._stats_struct(max(self.npole * self.S, 1))
        self._chk(self.L.tem_jvp(self.h, _dev(v, "float64", (self.n_params,)),
                                 _dev(jv, "float64", self._dshape()), self._ir(ir), C.byref(s)))
        return dict(iters=it.reshape(self.npole, self.S), rel=rr.reshape(self.npole, self.S))

    def vjp(self, w, jtw, ir=None):
        s, it, rr = self._stats_struct(max(self.npole * self.S, 1))
        self._chk(self.L.tem_vjp(self.h, _dev(w, "float64", self._dshape()),
                                 _dev(jtw, "float64", (self.n_params,)), self._ir(ir), C.byref(s)))
        return dict(iters=it.reshape(self.npole, self.S), rel=rr.reshape(self.npole, self.S))

    def vjp_noalloc(self, w, jtw, ir=None):
        """tem_vjp_noalloc: J^T w with all work space in the library's static
        scratch array (no device allocation)."""
        s, it, rr = self._stats_struct(max(self.npole * self.S, 1))
        self._chk(self.L.tem_vjp_noalloc(self.h, _dev(w, "float64", self._dshape()),
                                         _dev(jtw, "float64", (self.n_params,)), self._ir(ir),
                                         C.byref(s)))
        return dict(iters=it.reshape(self.npole, self.S), rel=rr.reshape(self.npole, self.S))

    def gn_step(self, d_obs, wd, m, m_ref, lam, iters, dm, ir=None):
        """One Gauss-Newton step by LSQR; returns the residual estimates."""
        hist = np.zeros(iters)
        shp = self._dshape()
        self._chk(self.L.tem_gn_step(self.h, _dev(d_obs, "float64", shp), _dev(wd, "float64", shp),
                                     _dev(m, "float64", (self.n_params,)),
                                     _dev(m_ref, "float64", (self.n_params,)), float(lam), int(iters),
                                     _dev(dm, "float64", (self.n_params,)),
                                     hist.ctypes.data_as(C.c_void_p), self._ir(ir)))
        return hist

    def invert(self, d_obs, wd, m, m_ref, lambda0, max_gn, lsqr_iters, chi2_target=0.0,
               c1=0.0, eta_min=0.0, conv_rtol=0.0, ir=None):
        """Gauss-Newton inversion from the model of the last forward (tem_invert);
        m (P,) float64 on the GPU is updated in place.  Returns one dict per
        iteration."""
        shp = self._dshape()
        opts = InvertOpts(float(lambda0), float(chi2_target), float(c1), float(eta_min),
                          float(conv_rtol), int(max_gn), int(lsqr_iters))
        recs = (InvertRecord * int(max_gn))()
        n = C.c_int32(0)
        self._chk(self.L.tem_invert(self.h, _dev(d_obs, "float64", shp), _dev(wd, "float64", shp),
                                    _dev(m, "float64", (self.n_params,)),
                                    _dev(m_ref, "float64", (self.n_params,)), C.byref(opts),
                                    self._ir(ir), C.cast(recs, C.c_void_p), C.byref(n)))
        out = []
        for r in recs[:n.value]:
            d = {f: getattr(r, f) for f, _ in r._fields_}
            d["lam"] = d.pop("lambda_")
            d["accepted"] = bool(d["accepted"])
            out.append(d)
        return out

    def autotune(self, xi, precision=FP32_IR):
        """Time the front-update variants level by level and keep the fastest
        per level (tem_autotune).  Returns the report and the per-level choice."""
        xi = np.asarray(xi, complex)
        buf, bp = _host(np.stack([xi.real, xi.imag], axis=1).reshape(-1), np.float64)
        rep = AutotuneReport()
        self._chk(self.L.tem_autotune(self.h, len(xi), bp, int(precision), C.byref(rep)))
        self.npole = len(xi)
        n = rep.n_candidates
        levels = []
        for L in range(rep.n_levels):
            tl, m3 = C.c_int32(), C.c_int32()
            self._chk(self.L.tem_autotune_level(self.h, int(precision), L, C.byref(tl), C.byref(m3)))
            levels.append((tl.value, m3.value))
        return dict(candidate_ms=list(rep.candidate_ms[:n]),
                    candidates=list(zip(rep.candidate_tile[:n], rep.candidate_m3[:n])),
                    tuned_ms=rep.tuned_ms, levels=levels)

    # ------------------------------------------------------- ragged batches
    def assemble_batch(self, meshes, mu, sigma):
        """meshes: list of (nx, ny, nz, h); sigma: float64 GPU tensor of all
        cells, mesh after mesh.  Puts the context in batch mode."""
        arr = (Mesh * len(meshes))(*[Mesh(int(a), int(b), int(c), float(h), float(mu))
                                     for a, b, c, h in meshes])
        self._bmeshes = arr
        self.batch = [tuple(m) for m in meshes]
        self.batch_edges = [a * (b + 1) * (c + 1) + (a + 1) * b * (c + 1) + (a + 1) * (b + 1) * c
                            for a, b, c, _ in meshes]
        ncell = sum(a * b * c for a, b, c, _ in meshes)
        self._chk(self.L.tem_assemble_batch(self.h, len(meshes), C.cast(arr, C.c_void_p),
                                            _dev(sigma, "float64", (ncell,))))

    def factor_poles_batch(self, xi_list, precision=FP32_IR, mem_budget_bytes=0, max_group=0):
        """xi_list: one array of poles (Im > 0) per mesh."""
        m, mp = _host([len(x) for x in xi_list], np.int32)
        xi = np.concatenate([np.asarray(x, complex) for x in xi_list])
        buf, bp = _host(np.stack([xi.real, xi.imag], axis=1).reshape(-1), np.float64)
        self._chk(self.L.tem_factor_poles_batch(self.h, mp, bp, int(precision),
                                                C.byref(FactorOpts(int(mem_budget_bytes),
                                                                   int(max_group), 0))))
        self.batch_m = [len(x) for x in xi_list]

    def forward_batch(self, F, S, receivers, alpha_list, d, ir=None, allow_noconv=False):
        """F: float64 GPU tensor, mesh b's (S[b], n_edges_b) block after the
        previous ones; receivers: list of (q_ptr, q_col, q_val) per mesh;
        alpha_list: (K, m_b) complex residues per mesh; d: float64 GPU tensor
        receiving mesh b's (S[b], K, R_b) block after the previous ones."""
        B = len(S)
        Sa, sp = _host(S, np.int32)
        Ra, rp = _host([len(q[0]) - 1 for q in receivers], np.int32)
        qp, qpp = _host(np.concatenate([np.asarray(q[0], np.int64) for q in receivers]), np.int64)
        qc, qcp = _host(np.concatenate([np.asarray(q[1], np.int32) for q in receivers]), np.int32)
        qv, qvp = _host(np.concatenate([np.asarray(q[2], np.float64) for q in receivers]),
                        np.float64)
        K = np.asarray(alpha_list[0]).shape[0]
        al = np.concatenate([np.asarray(a, complex).reshape(-1) for a in alpha_list])
        alb, alp = _host(np.stack([al.real, al.imag], axis=1).reshape(-1), np.float64)
        nf = sum(int(S[b]) * self.batch_edges[b] for b in range(B))
        nd = sum(int(S[b]) * K * int(Ra[b]) for b in range(B))
        MP, Smax = max(self.batch_m), int(max(S))
        s, it, rr = self._stats_struct(B * MP * Smax)
        st = self.L.tem_forward_batch(self.h, sp, _dev(F, "float64", (nf,)), rp, qpp, qcp, qvp, K,
                                      alp, self._ir(ir), _dev(d, "float64", (nd,)), C.byref(s))
        self._chk(st, (TEM_ENOCONV,) if allow_noconv else ())
        self._bsurvey = dict(nd=nd, nsys=B * MP * Smax, shape=(B, MP, Smax))
        return dict(iters=it.reshape(B, MP, Smax), rel=rr.reshape(B, MP, Smax),
                    n_unconverged=s.n_unconverged, status=st)

    def set_params_batch(self, params_list):
        """params_list: one array of parameter cell ids per mesh of the batch."""
        n, npp = _host([len(p) for p in params_list], np.int32)
        cells, cp = _host(np.concatenate([np.asarray(p, np.int32) for p in params_list]),
                          np.int32)
        self._chk(self.L.tem_set_params_batch(self.h, npp, cp))
        self.batch_params = [len(p) for p in params_list]

    def jvp_batch(self, v, jv, ir=None):
        """v: float64 GPU tensor of all meshes' parameters; jv: like forward_batch's d."""
        P = sum(self.batch_params)
        s, it, rr = self._stats_struct(self._bsurvey["nsys"])
        self._chk(self.L.tem_jvp_batch(self.h, _dev(v, "float64", (P,)),
                                       _dev(jv, "float64", (self._bsurvey["nd"],)), self._ir(ir),
                                       C.byref(s)))
        return dict(iters=it.reshape(self._bsurvey["shape"]))

    def vjp_batch(self, w, jtw, ir=None):
        """w: like forward_batch's d; jtw: float64 GPU tensor of all meshes' parameters."""
        P = sum(self.batch_params)
        s, it, rr = self._stats_struct(self._bsurvey["nsys"])
        self._chk(self.L.tem_vjp_batch(self.h, _dev(w, "float64", (self._bsurvey["nd"],)),
                                       _dev(jtw, "float64", (P,)), self._ir(ir), C.byref(s)))
        return dict(iters=it.reshape(self._bsurvey["shape"]))

    def set_profiling(self, enable=True):
        self._chk(self.L.tem_set_profiling(self.h, 1 if enable else 0))

    def stats(self):
        s = Stats()
        self._chk(self.L.tem_get_stats(self.h, C.byref(s)))
        return s.as_dict()
