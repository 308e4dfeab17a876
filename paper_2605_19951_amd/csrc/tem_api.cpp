// C ABI of libtem: context, state machine, symbolic maps, and the host
// orchestration of the batched factorisation, the solves with FP64
// refinement, the time assembly and the Jacobian products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <limits>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tem.h"
#include "host_mesh.h"
#include "tem_internal.h"

using namespace tem;

namespace {

// text of the calling thread's last failed tem_create
thread_local std::string g_create_error;

// Work space of the allocation-free entry points (tem_vjp_noalloc): one
// static device array per GPU, held from the module's load until the
// process ends.  Host code never passes `scratch` itself to a kernel (its
// host-side name is not a device address): tem_create looks up the array's
// device address once per device and every use goes through that pointer.
constexpr size_t SCRATCH_BYTES = size_t(256) << 20;
constexpr int SCRATCH_MAX_DEVICES = 64;
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// device address of `scratch` on the current device `dev` (looked up once)
hipError_t scratch_setup(int dev) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = ptr;
  return hipSuccess;
}

void *scratch_ptr(int dev) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// set while an allocation-free call runs on this thread: any device
// allocation attempted then fails instead of calling hipMalloc
thread_local bool t_no_alloc = false;

// ------------------------------------------------------------ device buffer
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  bool borrowed = false;   // p lies in the static scratch array (not owned)
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p && !borrowed) hipFree(p);
    p = nullptr;
    bytes = 0;
    borrowed = false;
  }
  // Freeing and mapping tens of GB takes seconds, so buffers that are
  // rebuilt with the same size (factors, arenas) keep their allocation.
  hipError_t alloc(size_t b) {
    if (b == bytes && p) return hipSuccess;
    if (t_no_alloc) return hipErrorOutOfMemory;
    release();
    if (b == 0) return hipSuccess;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = b;
    return hipSuccess;
  }
  template <typename T>
  T *as() const {
    return (T *)p;
  }
};

// Host-to-device copies from pageable host memory complete before these
// helpers return, so the host buffer may be reused or freed right away.
template <typename T>
hipError_t upload(DBuf &b, const std::vector<T> &v, hipStream_t st) {
  hipError_t e = b.alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (e != hipSuccess) return e;
  if (v.empty()) return hipSuccess;
  e = hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t h2d(void *dst, const void *src, size_t bytes, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

struct LevelInfo {
  std::vector<int32_t> nodes;
  int64_t lvl_begin = 0;           // offset in the device level-node list
  int n = 0;
  int max_k = 0, max_u = 0, max_n = 0;
  int max_u_child[2] = {0, 0};
  int64_t panel_begin = 0, panel_end = 0;   // per-pole element range
  int64_t amap_begin = 0, amap_end = 0;
  int64_t cb_size = 0;             // elements per pole
  int64_t w_rows = 0;              // update rows per pole
  // extend-add column lists per child slot: [xa, xm) go to the panels,
  // [xm, xe) to the contribution blocks (offsets into d_xcols)
  int64_t xa[2] = {0, 0}, xm[2] = {0, 0}, xe[2] = {0, 0};
};

struct Tiles {
  // update tiles of shape `tile` covering the lower trapezoid with columns
  // [cbeg, cend) of an n-row front (the enumeration of k_front_update)
  static int64_t count(int64_t n, int64_t cbeg, int64_t cend, int tile) {
    if (cbeg >= cend) return 0;
    const int64_t tc = upd_tile_cols(tile), tr = upd_tile_rows(tile), r = tr / tc;
    const int64_t nct = (cend - cbeg + tc - 1) / tc, nrt = (n - cbeg + tr - 1) / tr;
    int64_t tot = 0;
    for (int64_t ct = 0; ct < nct; ++ct) tot += nrt - ct / r;
    return tot;
  }
};

// One multifrontal system: symbolic structure, pattern and device maps.
// The edge system holds the shifted matrices of all poles; the nodal system
// holds the gradient-space matrix G^T M G used by the refinement.
struct MF {
  bool nodes = false;
  Symbolic sym;
  Pattern pat;
  std::vector<int32_t> perm;
  int64_t N = 0;
  DBuf d_rowptr, d_col, d_row_ent, d_ent_new;
  DBuf d_first, d_k, d_u, d_rows_off, d_rows, d_rel, d_panel_off, d_cb_off, d_w_off, d_gmap_off,
      d_gmap0, d_gmap1, d_child0, d_child1, d_lvl_nodes, d_amap_csr, d_amap_pos, d_xcols;
  std::vector<LevelInfo> levels;   // by depth (0 = root)
  int64_t pole_stride = 0;         // panel elements per pole
  int64_t cb_stride = 0;           // max level CB elements per pole
  int64_t w_rows_max = 0;
  DBuf w_t, w_w0, w_w1;            // sweep work space
  DBuf d_np;                       // batch: poles of each front's mesh (else empty)
  // explicit inverses of the BB-column diagonal blocks of the wide fronts
  // (levels with max_k > BB): per front the offset of its first block in
  // one pole's region of x_stride elements (k_diag_inverse)
  DBuf d_xoff;
  int64_t x_stride = 0;
  int x_bb = 0;
  // row blocks of the FP64 residual (edge system; see launch_residual_blk)
  int64_t rb_n = 0;
  bool rb_packed = false;   // some row has more than RB_NNZ entries
  DBuf d_rb_row, d_rb_rows, d_rb_hoff, d_rb_h, d_lcol;
  std::vector<int32_t> h_np;
  // poles of front s among the g slots starting at p0
  int present(int s, int p0, int g) const {
    if (h_np.empty()) return g;
    return std::max(0, std::min(g, h_np[s] - p0));
  }
};

}  // namespace

struct tem_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // stages
  bool assembled = false, analysed = false, factored = false, solved = false, surveyed = false;
  // mesh
  tem_mesh mesh{};
  MeshTopo mt;
  // tetrahedral mesh (tem_assemble_tet): topology, coordinates and
  // connectivity on the device, element matrices [36][n_tets], the
  // element-to-entry gather lists of the pattern, each row's tetrahedra and
  // each tetrahedron's six new edge indices
  bool tet = false;
  TetTopo tt;
  double tet_mu = 0.0;
  DBuf d_xyz, d_tetv, d_tsign, d_Kt, d_Mt, d_ent_ptr, d_ent_src, d_et_ptr, d_et_src, d_tet_new;
  // and its gradient-space system: unit nodal blocks [16][n_tets], the
  // gather lists of the nodal pattern, each node's signed edges (CSR)
  DBuf d_Lt, d_nent_ptr, d_nent_src, d_node_ptr;
  double Ke[144], Me[144];
  std::vector<int32_t> params;
  int leaf = 4;
  MF ed;                           // edge system (ordering used by the device pattern)
  MF nd;                           // nodal gradient-space system
  // device: mesh and operators
  DBuf d_K, d_M, d_cell_new, d_sigma, d_params, d_Ke, d_Me, d_Le;
  // nodal matrix G^T M G (values on nd's pattern), zeros, its factor
  DBuf d_Ln, d_Lzero, d_nfactor, d_nxi, d_edge_nodes, d_node_edges, d_nvec, d_ncoef;
  bool nodal_ready = false;
  bool aux = true;                 // gradient-space correction in FP32 refinement
  int64_t sweep_bb = 256;          // big column block of the wide-front sweeps
  int64_t sweep_big_limit = 1024;  // fronts x poles below which a level is "wide"
  int upd_tile = UPD_T64;          // FP32 update tile shape (FP64: 64 x 64)
  int panel_w = 8 * NB;            // columns per factorisation panel (multiple of NB)
  bool left_looking = true;        // panels take all earlier panels' updates at once
  bool upd_m3_f32 = true;          // 3M complex products in the FP32 update
  bool upd_m3_f64 = false;         // 3M complex products in the FP64 update
  // Autotuned update variant per tree level of the edge system, by
  // precision (empty: the defaults above); see tem_autotune.
  struct UpdCfg {
    int tile;
    bool m3;
  };
  std::vector<UpdCfg> tuned[2];    // [0] FP64, [1] FP32
  bool forcing = false;            // tem_autotune: every level uses `forced`
  UpdCfg forced{UPD_T64, false};
  // tem_autotune: start/end events per (pole group, level) of the edge
  // factorisation, [(group * levels + L) * 2 + {0, 1}]
  bool lvl_timing = false;
  int lvl_group = 0;
  std::vector<hipEvent_t> lvl_ev;
  // HIP graph of the all-pole edge sweep, replayed by every refinement step;
  // valid while the factors, the vector and its shape are those captured
  bool use_graphs = true;
  hipStream_t cap_stream = nullptr;
  // the nodal factorisation runs on its own stream beside the edge factor
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // start/end of the device time of a factorisation or solve call (made once
  // by tem_create, so no error path of those calls leaks events)
  hipEvent_t t_ev[2] = {nullptr, nullptr};
  DBuf d_ncb0, d_ncb1;                  // nodal contribution-block arenas
  std::vector<double> h_ncoef;          // host copy of the correction coefficients
  struct SweepGraph {
    hipGraphExec_t exec = nullptr;
    const void *x = nullptr, *factor = nullptr, *xinv = nullptr;
    const void *ws[3] = {nullptr, nullptr, nullptr};
    int S = 0, npole = 0;
  } sgraph[2];                     // [0] FP64 factors, [1] FP32 factors
  // Batch of meshes (B > 0): the per-mesh contexts in `sub` assemble and
  // analyse each mesh; this context holds the merged block-diagonal edge and
  // nodal systems (mesh b owns edge rows [row_off[b], row_off[b+1]), matrix
  // entries [nnz_off[b], nnz_off[b+1]), nodal rows [node_off[b], ...)).
  // Pole tables are [mesh][MP], MP the largest pole count; absent poles of a
  // mesh are padding that no kernel computes.
  int B = 0;
  std::vector<tem_ctx *> sub;
  std::vector<int64_t> row_off, nnz_off, node_off, nnz_node_off, cell_off;
  std::vector<int> np_mesh;
  int MP = 0;
  DBuf d_row_seg, d_nnz_seg;
  std::vector<int32_t> h_node_edges, h_edge_nodes;   // nodal incidence (host copies)
  // survey of the last tem_forward_batch: sources and receivers per mesh,
  // first merged receiver row of each mesh; parameter cells per mesh
  // (tem_set_params_batch): mesh b's parameters are [param_off[b], param_off[b+1])
  std::vector<int> S_mesh, R_mesh;
  std::vector<int64_t> q_row_off, param_off;
  // factors
  int npole = 0;                   // pole slots (a batch: the largest pole count)
  int64_t fac_elems = 0;           // factor elements of the poles present
  tem_precision prec = TEM_FP64;
  std::vector<double> xi;
  DBuf d_xi, d_factor, d_cb0, d_cb1, d_flags;
  DBuf d_xinv;                     // FP32 factors: the wide fronts' block inverses
  bool xinv_ok = false;
  DBuf d_nxinv;                    // the same for the nodal factor (FP64, real)
  bool nxinv_ok = false;
  int n_groups = 0, group_size = 0;
  int n_tiny = 0;
  double factor_ms = 0.0, solve_ms = 0.0;
  int last_solves = 0;
  // solve state
  int S = 0;
  DBuf d_g;                        // cached g [pole][N][S] complex double
  DBuf d_fnew;                     // sources [N][S] real (new ordering)
  // survey
  int R = 0, K = 0;
  DBuf d_qptr, d_qcol, d_qval, d_alpha;
  // regularisation rows w_r (m_hi - m_lo) over faces shared by two
  // parameter cells (hex: w = 1, d_reg_w empty; tetrahedra: RT0 weights)
  int64_t n_reg = 0;
  DBuf d_reg_lo, d_reg_hi, d_reg_incp, d_reg_inc, d_reg_w;
  // LSQR work space
  DBuf l_u, l_v, l_w, l_x, l_tmpd, l_tmpm, l_part, l_scal, l_V;
  // inversion work space (tem_invert)
  DBuf inv_d, inv_dt, inv_mt, inv_dm, inv_t1, inv_t2, inv_t3;
  // work space
  DBuf w_x;                        // factor-precision sweep vector
  DBuf v_r, v_z, v_rhs, v_lam, v_vs, v_dots, v_partial, v_inv, v_nrm, v_coef, v_mask;
  DBuf v_aux, v_fblk, v_xblk;
  // Allocation-free calls: while `on`, the work buffers a call needs are
  // carved from the device's static scratch array (bump allocation from
  // `base`) instead of allocated; `saved` keeps each borrowed buffer's own
  // allocation, given back when the call ends.
  struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    bool on = false;
    struct Saved {
      DBuf *b;
      void *p;
      size_t bytes;
    };
    std::vector<Saved> saved;
  } arena;
  // profiling (HIP events around the update launches and the sweeps)
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Span {
    hipEvent_t a, b;
    double work;   // flops (updates) or bytes (sweeps)
    int kind;      // 0 update, 1 sweep
  };
  std::vector<Span> spans;
  double upd_ms = 0, upd_flops = 0, sweep_ms = 0, sweep_bytes = 0;
  int64_t upd_launches = 0, sweeps = 0;

  hipError_t check_last() { return hipGetLastError(); }
};

namespace {

tem_status fail(tem_ctx *c, tem_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

tem_status hip_fail(tem_ctx *c, hipError_t e, const char *where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? TEM_ENOMEM : TEM_EDEVICE, m);
}

#define HIPCHK(expr, where)                     \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(c, e_, where); \
  } while (0)

#define TRY(expr)                  \
  do {                             \
    tem_status s_ = (expr);        \
    if (s_ != TEM_OK) return s_;   \
  } while (0)

int64_t N_of(const tem_ctx *c) { return c->ed.N; }
// canonical edges (the numbering of sources and receiver columns) and cells
int64_t n_ent(const tem_ctx *c) { return c->tet ? c->tt.n_edges : c->mt.n_edges; }
int64_t n_cells_of(const tem_ctx *c) { return c->tet ? c->tt.n_tets : c->mt.n_cells; }
// unknowns per nested-dissection leaf of a tetrahedral mesh for the leaf
// size given in cells per side (about the edges of that many cubes)
int64_t tet_leaf(int leaf) { return 3 * (int64_t)leaf * leaf * leaf; }

// systems per (pole, source) slot: one per mesh of a batch
int n_seg(const tem_ctx *c) { return c->B > 0 ? c->B : 1; }
Seg row_seg(const tem_ctx *c) {
  Seg sg;
  if (c->B > 0) {
    sg.n = c->B;
    sg.off = c->d_row_seg.as<int64_t>();
    sg.stride = c->MP;
  } else {
    sg.stride = c->npole;
  }
  return sg;
}
Seg nnz_seg(const tem_ctx *c) {
  Seg sg = row_seg(c);
  if (c->B > 0) sg.off = c->d_nnz_seg.as<int64_t>();
  return sg;
}

// --------------------------------------------------- assembly on the device
tem_status run_assemble_edges(tem_ctx *c) {
  MF &e = c->ed;
  HIPCHK(launch_assemble_KM(c->stream, e.N, e.d_rowptr.as<int64_t>(), e.d_col.as<int32_t>(),
                            e.d_row_ent.as<int32_t>(), e.d_ent_new.as<int32_t>(), c->mt.nx,
                            c->mt.ny, c->mt.nz, c->d_Ke.as<double>(), c->d_Me.as<double>(),
                            c->d_sigma.as<double>(), c->d_K.as<double>(), c->d_M.as<double>()),
         "assemble kernel");
  return TEM_OK;
}

// Row blocks of the residual: at most RB_ROWS rows and at most RB_HALO
// distinct columns per block, never across a segment start (a mesh of a
// batch).  With positions (3 per row) the rows are taken, segment by
// segment, in Morton order of their position on a grid of about three rows
// per cell, so that a block's rows are neighbours in space and share most of
// their columns (about a third fewer halo rows per row than in elimination
// order); without, in row order.  Each block's halo is its sorted column set
// and lcol gives every entry's position in it; a block holds at most
// RB_ROWS * RB_NNZ entries, and a longer row is refused.
uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t k = 0;
  for (int b = 0; b < 21; ++b)
    k |= ((uint64_t)((x >> b) & 1) << (3 * b)) | ((uint64_t)((y >> b) & 1) << (3 * b + 1)) |
         ((uint64_t)((z >> b) & 1) << (3 * b + 2));
  return k;
}

tem_status build_res_blocks(tem_ctx *c, MF &mf, const std::vector<int64_t> &rowptr,
                            const std::vector<int32_t> &col, const std::vector<int64_t> &seg,
                            const std::vector<double> *pos = nullptr) {
  const int64_t N = (int64_t)rowptr.size() - 1;
  std::vector<int32_t> order(std::max<int64_t>(N, 0));
  for (int64_t q = 0; q < N; ++q) order[q] = (int32_t)q;
  if (pos && (int64_t)pos->size() == 3 * N) {
    for (size_t si = 0; si < seg.size(); ++si) {
      const int64_t a = seg[si], e = si + 1 < seg.size() ? seg[si + 1] : N;
      if (e - a < 2) continue;
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int64_t q = a; q < e; ++q)
        for (int d = 0; d < 3; ++d) {
          lo[d] = std::min(lo[d], (*pos)[3 * q + d]);
          hi[d] = std::max(hi[d], (*pos)[3 * q + d]);
        }
      double vol = 1.0;
      for (int d = 0; d < 3; ++d) vol *= std::max(hi[d] - lo[d], 1e-300);
      const double cs = std::cbrt(vol * 3.0 / (double)(e - a));
      std::vector<std::pair<uint64_t, int32_t>> key(e - a);
      for (int64_t q = a; q < e; ++q) {
        uint32_t g[3];
        for (int d = 0; d < 3; ++d)
          g[d] = (uint32_t)std::min(2097151.0, std::max(0.0, ((*pos)[3 * q + d] - lo[d]) / cs));
        key[q - a] = {morton3(g[0], g[1], g[2]), (int32_t)q};
      }
      std::sort(key.begin(), key.end());
      for (int64_t q = a; q < e; ++q) order[q] = key[q - a].second;
    }
  }
  std::vector<int64_t> brow(1, 0), hoff(1, 0);
  std::vector<int32_t> halo;
  std::vector<uint16_t> lcol(col.size());
  std::vector<int64_t> stamp(std::max<int64_t>(N, 1), -1);
  std::vector<int32_t> pos_(std::max<int64_t>(N, 1), 0);
  std::vector<int32_t> h;
  size_t si = 0;
  int64_t i = 0;
  while (i < N) {
    const int64_t first = order[i];
    while (si + 1 < seg.size() && seg[si + 1] <= first) ++si;
    const int64_t seg_lo = seg[si], seg_end = si + 1 < seg.size() ? seg[si + 1] : N;
    const int64_t blk = (int64_t)brow.size() - 1, i0 = i;
    h.clear();
    int64_t ents = 0;
    while (i < N && i - i0 < RB_ROWS) {
      const int64_t r = order[i];
      if (r < seg_lo || r >= seg_end) break;   // the next segment starts a block
      const int64_t len = rowptr[r + 1] - rowptr[r];
      if (len > (int64_t)RB_ROWS * RB_NNZ)
        return fail(c, TEM_EINVAL, "residual blocks: a row has more than 1056 entries");
      if (len > RB_HALO)
        return fail(c, TEM_EINVAL, "residual blocks: a row has more than 256 distinct columns");
      if (ents + len > (int64_t)RB_ROWS * RB_NNZ) break;   // the block's entries are full
      ents += len;
      int add = 0;
      for (int64_t t = rowptr[r]; t < rowptr[r + 1]; ++t)
        if (stamp[col[t]] != blk) {
          stamp[col[t]] = blk;
          ++add;
          h.push_back(col[t]);
        }
      if ((int64_t)h.size() > RB_HALO) {
        // the row does not fit: undo its new columns (i > i0 here, since a
        // single row has at most RB_HALO columns)
        for (int k = 0; k < add; ++k) {
          stamp[h.back()] = -1;
          h.pop_back();
        }
        break;
      }
      ++i;
    }
    std::sort(h.begin(), h.end());
    for (size_t k = 0; k < h.size(); ++k) pos_[h[k]] = (int32_t)k;
    for (int64_t j = i0; j < i; ++j) {
      const int64_t r = order[j];
      for (int64_t t = rowptr[r]; t < rowptr[r + 1]; ++t) lcol[t] = (uint16_t)pos_[col[t]];
    }
    halo.insert(halo.end(), h.begin(), h.end());
    brow.push_back(i);
    hoff.push_back((int64_t)halo.size());
  }
  hipStream_t st = c->stream;
  mf.rb_n = (int64_t)brow.size() - 1;
  mf.rb_packed = false;
  for (int64_t q = 0; q < N && !mf.rb_packed; ++q) mf.rb_packed = rowptr[q + 1] - rowptr[q] > RB_NNZ;
  HIPCHK(upload(mf.d_rb_row, brow, st), "upload residual blocks");
  HIPCHK(upload(mf.d_rb_rows, order, st), "upload residual blocks");
  HIPCHK(upload(mf.d_rb_hoff, hoff, st), "upload residual blocks");
  HIPCHK(upload(mf.d_rb_h, halo, st), "upload residual blocks");
  HIPCHK(upload(mf.d_lcol, lcol, st), "upload residual blocks");
  return TEM_OK;
}

// Entity positions of the rows of a pattern (3 per row): edge midpoints of
// a hexahedral mesh (cell units) or of a tetrahedral one (coordinates).
std::vector<double> hex_row_positions(const MeshTopo &mt, const std::vector<int32_t> &row_edge) {
  std::vector<double> p(3 * row_edge.size());
  for (size_t q = 0; q < row_edge.size(); ++q) {
    int d, i, j, k;
    mt.geometry(row_edge[q], d, i, j, k);
    p[3 * q] = i + 0.5 * (d == 0);
    p[3 * q + 1] = j + 0.5 * (d == 1);
    p[3 * q + 2] = k + 0.5 * (d == 2);
  }
  return p;
}
std::vector<double> tet_row_positions(const TetTopo &tt, const std::vector<int32_t> &row_edge) {
  std::vector<double> p(3 * row_edge.size());
  for (size_t q = 0; q < row_edge.size(); ++q) {
    const int64_t e = row_edge[q];
    for (int k = 0; k < 3; ++k)
      p[3 * q + k] = 0.5 * (tt.xyz[3 * (size_t)tt.edges[2 * e] + k] +
                            tt.xyz[3 * (size_t)tt.edges[2 * e + 1] + k]);
  }
  return p;
}

tem_status upload_pattern(tem_ctx *c, MF &mf) {
  hipStream_t st = c->stream;
  build_pattern(c->mt, mf.perm, mf.pat, mf.nodes);
  mf.N = (int64_t)mf.perm.size();
  HIPCHK(upload(mf.d_rowptr, mf.pat.rowptr, st), "upload rowptr");
  HIPCHK(upload(mf.d_col, mf.pat.col, st), "upload col");
  HIPCHK(upload(mf.d_row_ent, mf.pat.row_edge, st), "upload row map");
  HIPCHK(upload(mf.d_ent_new, mf.pat.edge_new, st), "upload entity map");
  if (!mf.nodes) {
    const std::vector<double> pos = hex_row_positions(c->mt, mf.pat.row_edge);
    TRY(build_res_blocks(c, mf, mf.pat.rowptr, mf.pat.col, {0}, &pos));
  }
  return TEM_OK;
}

tem_status upload_pattern_and_assemble(tem_ctx *c) {
  hipStream_t st = c->stream;
  TRY(upload_pattern(c, c->ed));
  // cell -> 12 new indices
  std::vector<int32_t> cn((size_t)c->mt.n_cells * 12);
  int64_t ce[12];
  for (int k = 0; k < c->mt.nz; ++k)
    for (int j = 0; j < c->mt.ny; ++j)
      for (int i = 0; i < c->mt.nx; ++i) {
        int64_t cell = i + (int64_t)c->mt.nx * (j + (int64_t)c->mt.ny * k);
        c->mt.cell_edges(i, j, k, ce);
        for (int t = 0; t < 12; ++t) cn[cell * 12 + t] = c->ed.pat.edge_new[ce[t]];
      }
  HIPCHK(upload(c->d_cell_new, cn, st), "upload cell_new");
  const size_t nnz = c->ed.pat.col.size();
  HIPCHK(c->d_K.alloc(sizeof(double) * nnz), "alloc K");
  HIPCHK(c->d_M.alloc(sizeof(double) * nnz), "alloc M");
  return run_assemble_edges(c);
}

// ------------------------------------------ tetrahedral mesh (device side)
tem_status run_assemble_tet(tem_ctx *c, bool with_k) {
  const MF &e = c->ed;
  HIPCHK(launch_tet_gather(c->stream, (int64_t)e.pat.col.size(), c->d_ent_ptr.as<int64_t>(),
                           c->d_ent_src.as<int32_t>(), 36, c->tt.n_tets, c->d_Kt.as<double>(),
                           c->d_Mt.as<double>(), c->d_sigma.as<double>(), with_k,
                           c->d_K.as<double>(), c->d_M.as<double>()),
         "tet gather");
  return TEM_OK;
}

// Pattern in the current ordering, the gather lists from element entries
// (t * 36 + 6 a + b, increasing) to pattern entries, each row's tetrahedra,
// each tetrahedron's new edge indices; element matrices; K and M.
tem_status upload_pattern_and_assemble_tet(tem_ctx *c) {
  hipStream_t st = c->stream;
  MF &e = c->ed;
  const TetTopo &tt = c->tt;
  build_pattern_graph(tt.adj_ptr, tt.adj, e.perm, tt.edge_of_unk, tt.n_edges, e.pat);
  e.N = (int64_t)e.perm.size();
  HIPCHK(upload(e.d_rowptr, e.pat.rowptr, st), "upload rowptr");
  HIPCHK(upload(e.d_col, e.pat.col, st), "upload col");
  HIPCHK(upload(e.d_row_ent, e.pat.row_edge, st), "upload row map");
  HIPCHK(upload(e.d_ent_new, e.pat.edge_new, st), "upload entity map");
  {
    const std::vector<double> pos = tet_row_positions(tt, e.pat.row_edge);
    TRY(build_res_blocks(c, e, e.pat.rowptr, e.pat.col, {0}, &pos));
  }
  const int64_t nt = tt.n_tets, N = e.N;
  const size_t nnz = e.pat.col.size();
  std::vector<int32_t> tn((size_t)nt * 6);
  for (int64_t t = 0; t < nt * 6; ++t) tn[t] = e.pat.edge_new[tt.tet_edges[t]];
  auto entry = [&](int32_t qa, int32_t qb) {
    const int32_t *b = e.pat.col.data() + e.pat.rowptr[qa], *en = e.pat.col.data() + e.pat.rowptr[qa + 1];
    return (int64_t)(std::lower_bound(b, en, qb) - e.pat.col.data());
  };
  std::vector<int64_t> eptr(nnz + 1, 0), etp(N + 1, 0);
  for (int64_t t = 0; t < nt; ++t)
    for (int a = 0; a < 6; ++a) {
      const int32_t qa = tn[t * 6 + a];
      if (qa < 0) continue;
      ++etp[qa + 1];
      for (int b = 0; b < 6; ++b)
        if (tn[t * 6 + b] >= 0) ++eptr[entry(qa, tn[t * 6 + b]) + 1];
    }
  for (size_t k = 0; k < nnz; ++k) eptr[k + 1] += eptr[k];
  for (int64_t q = 0; q < N; ++q) etp[q + 1] += etp[q];
  std::vector<int32_t> esrc(eptr[nnz]), ets(etp[N]);
  std::vector<int64_t> ef(eptr.begin(), eptr.end() - 1), tf(etp.begin(), etp.end() - 1);
  for (int64_t t = 0; t < nt; ++t)
    for (int a = 0; a < 6; ++a) {
      const int32_t qa = tn[t * 6 + a];
      if (qa < 0) continue;
      ets[tf[qa]++] = (int32_t)(t * 6 + a);
      for (int b = 0; b < 6; ++b)
        if (tn[t * 6 + b] >= 0) esrc[ef[entry(qa, tn[t * 6 + b])]++] = (int32_t)(t * 36 + a * 6 + b);
    }
  HIPCHK(upload(c->d_ent_ptr, eptr, st), "upload gather lists");
  HIPCHK(upload(c->d_ent_src, esrc, st), "upload gather lists");
  HIPCHK(upload(c->d_et_ptr, etp, st), "upload row tetrahedra");
  HIPCHK(upload(c->d_et_src, ets, st), "upload row tetrahedra");
  HIPCHK(upload(c->d_tet_new, tn, st), "upload tetrahedron edges");
  HIPCHK(c->d_K.alloc(sizeof(double) * nnz), "alloc K");
  HIPCHK(c->d_M.alloc(sizeof(double) * nnz), "alloc M");
  HIPCHK(c->d_Kt.alloc(sizeof(double) * 36 * (size_t)nt), "alloc element K");
  HIPCHK(c->d_Mt.alloc(sizeof(double) * 36 * (size_t)nt), "alloc element M");
  HIPCHK(c->d_Lt.alloc(sizeof(double) * 16 * (size_t)nt), "alloc nodal blocks");
  HIPCHK(launch_tet_elements(st, nt, c->d_xyz.as<double>(), c->d_tetv.as<int32_t>(),
                             c->d_tsign.as<int8_t>(), c->tet_mu, c->d_Kt.as<double>(),
                             c->d_Mt.as<double>(), c->d_Lt.as<double>()),
         "tet elements");
  return run_assemble_tet(c, true);
}

void release_tet(tem_ctx *c) {
  c->tet = false;
  c->tt = TetTopo();
  for (DBuf *b : {&c->d_xyz, &c->d_tetv, &c->d_tsign, &c->d_Kt, &c->d_Mt, &c->d_ent_ptr,
                  &c->d_ent_src, &c->d_et_ptr, &c->d_et_src, &c->d_tet_new, &c->d_Lt,
                  &c->d_nent_ptr, &c->d_nent_src, &c->d_node_ptr})
    b->release();
}

tem_status build_front_maps(tem_ctx *c, MF &mf);

// The gradient-space system of a tetrahedral mesh (as setup_nodal for
// hexahedra): nested dissection of the interior-node graph, its pattern,
// the gather lists of G^T M G from the unit nodal blocks, each node's
// signed edges and each edge's two nodes (new indices).
tem_status setup_nodal_tet(tem_ctx *c, int leaf) {
  MF &nd = c->nd;
  nd.nodes = true;
  c->nodal_ready = false;
  const TetTopo &tt = c->tt;
  nd.N = 0;
  if (tt.n_inodes == 0) return TEM_OK;
  std::vector<double> xy((size_t)tt.n_inodes * 3);
  for (int64_t u = 0; u < tt.n_inodes; ++u)
    for (int k = 0; k < 3; ++k) xy[3 * u + k] = tt.xyz[3 * (size_t)tt.node_of_unk[u] + k];
  try {
    analyse_graph(tt.n_inodes, tt.nadj_ptr, tt.nadj, xy, (int64_t)leaf * leaf * leaf, nd.sym);
  } catch (const std::exception &ex) {
    return fail(c, TEM_EINVAL, std::string("nodal analysis: ") + ex.what());
  }
  nd.perm = nd.sym.perm;
  hipStream_t st = c->stream;
  build_pattern_graph(tt.nadj_ptr, tt.nadj, nd.perm, tt.node_of_unk, tt.n_nodes, nd.pat);
  nd.N = (int64_t)nd.perm.size();
  HIPCHK(upload(nd.d_rowptr, nd.pat.rowptr, st), "upload nodal rowptr");
  HIPCHK(upload(nd.d_col, nd.pat.col, st), "upload nodal col");
  HIPCHK(upload(nd.d_row_ent, nd.pat.row_edge, st), "upload nodal row map");
  HIPCHK(upload(nd.d_ent_new, nd.pat.edge_new, st), "upload nodal map");
  TRY(build_front_maps(c, nd));
  const int64_t nt = tt.n_tets, Nn = nd.N;
  const size_t nnz = nd.pat.col.size();
  // G^T M G entries from the blocks t * 16 + 4 i + j of interior nodes
  std::vector<int32_t> tn((size_t)nt * 4);
  for (int64_t t = 0; t < nt * 4; ++t) tn[t] = nd.pat.edge_new[tt.tets[t]];
  auto entry = [&](int32_t qa, int32_t qb) {
    const int32_t *b = nd.pat.col.data() + nd.pat.rowptr[qa], *en = nd.pat.col.data() + nd.pat.rowptr[qa + 1];
    return (int64_t)(std::lower_bound(b, en, qb) - nd.pat.col.data());
  };
  std::vector<int64_t> eptr(nnz + 1, 0);
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        if (tn[t * 4 + i] >= 0 && tn[t * 4 + j] >= 0) ++eptr[entry(tn[t * 4 + i], tn[t * 4 + j]) + 1];
  for (size_t k = 0; k < nnz; ++k) eptr[k + 1] += eptr[k];
  std::vector<int32_t> esrc(eptr[nnz]);
  std::vector<int64_t> ef(eptr.begin(), eptr.end() - 1);
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        if (tn[t * 4 + i] >= 0 && tn[t * 4 + j] >= 0)
          esrc[ef[entry(tn[t * 4 + i], tn[t * 4 + j])]++] = (int32_t)(t * 16 + i * 4 + j);
  HIPCHK(upload(c->d_nent_ptr, eptr, st), "upload nodal gather lists");
  HIPCHK(upload(c->d_nent_src, esrc, st), "upload nodal gather lists");
  // node -> signed unknown edges (new indices), edge -> (start, end) nodes
  const Pattern &ep = c->ed.pat;
  std::vector<int64_t> np_(Nn + 1, 0);
  std::vector<int32_t> en((size_t)c->ed.N * 2);
  for (int64_t q = 0; q < c->ed.N; ++q) {
    const int64_t e = ep.row_edge[q];
    const int32_t a = nd.pat.edge_new[tt.edges[2 * e]], b = nd.pat.edge_new[tt.edges[2 * e + 1]];
    en[q * 2] = a;
    en[q * 2 + 1] = b;
    if (a >= 0) ++np_[a + 1];
    if (b >= 0) ++np_[b + 1];
  }
  for (int64_t v = 0; v < Nn; ++v) np_[v + 1] += np_[v];
  std::vector<int32_t> ne(np_[Nn]);
  std::vector<int64_t> nf(np_.begin(), np_.end() - 1);
  for (int64_t q = 0; q < c->ed.N; ++q) {
    if (en[q * 2] >= 0) ne[nf[en[q * 2]]++] = -(int32_t)(q + 1);
    if (en[q * 2 + 1] >= 0) ne[nf[en[q * 2 + 1]]++] = (int32_t)(q + 1);
  }
  HIPCHK(upload(c->d_node_ptr, np_, st), "upload node edges");
  HIPCHK(upload(c->d_node_edges, ne, st), "upload node edges");
  HIPCHK(upload(c->d_edge_nodes, en, st), "upload edge nodes");
  HIPCHK(c->d_Ln.alloc(sizeof(double) * nnz), "alloc nodal values");
  HIPCHK(c->d_Lzero.alloc(sizeof(double) * nnz), "alloc zeros");
  HIPCHK(launch_fill_f64(st, c->d_Lzero.as<double>(), (int64_t)nnz, 0.0), "zeros");
  std::vector<double> zxi = {0.0, 0.0};
  HIPCHK(upload(c->d_nxi, zxi, st), "upload zero shift");
  HIPCHK(hipStreamSynchronize(st), "nodal setup sync");
  return TEM_OK;
}

// Invalidates the factors and pole solutions; their memory stays allocated
// for a refactorisation of the same size (free_factors releases it).
void drop_graphs(tem_ctx *c) {
  for (auto &g : c->sgraph) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    g = tem_ctx::SweepGraph();
  }
}
void drop_factors(tem_ctx *c) {
  c->nodal_ready = false;
  c->factored = false;
  c->xinv_ok = false;
  c->nxinv_ok = false;
  c->solved = false;
  drop_graphs(c);
}
void free_factors(tem_ctx *c) {
  drop_factors(c);
  c->d_factor.release();
  c->d_xinv.release();
  c->d_cb0.release();
  c->d_cb1.release();
  c->d_g.release();
}

// ------------------------------------------------ symbolic maps (host)
// Rows (m_b - m_a) for every face shared by two parameter cells a < b:
// x-faces, then y-faces, then z-faces, each in increasing cell index of the
// lower cell; parameter incidence lists (signed row+1) for the transpose.
tem_status upload_regulariser(tem_ctx *c, const std::vector<int32_t> &lo,
                              const std::vector<int32_t> &hi, const std::vector<double> &w);

tem_status build_regulariser(tem_ctx *c) {
  const MeshTopo &mt = c->mt;
  std::vector<int32_t> pid(mt.n_cells, -1);
  for (size_t p = 0; p < c->params.size(); ++p) pid[c->params[p]] = (int32_t)p;
  std::vector<int32_t> cells(c->params.begin(), c->params.end());
  std::sort(cells.begin(), cells.end());
  std::vector<int32_t> lo, hi;
  for (int d = 0; d < 3; ++d)
    for (int32_t cell : cells) {
      int i = cell % mt.nx, j = (cell / mt.nx) % mt.ny, k = cell / (mt.nx * mt.ny);
      int i2 = i + (d == 0), j2 = j + (d == 1), k2 = k + (d == 2);
      if (i2 >= mt.nx || j2 >= mt.ny || k2 >= mt.nz) continue;
      int32_t nb = pid[i2 + mt.nx * (j2 + mt.ny * k2)];
      if (nb < 0) continue;
      lo.push_back(pid[cell]);
      hi.push_back(nb);
    }
  return upload_regulariser(c, lo, hi, {});
}

// Tetrahedra (section "Regularization"): one row per face shared by two
// parameter tetrahedra a < b, in increasing order of the face's sorted node
// triple, (m_b - m_a) / sqrt(d_f) with d_f the diagonal of the lowest-order
// Raviart-Thomas mass of the face's unit-flux function over both
// tetrahedra (the lumped M_div), so that R^T R = D diag(M_div)^-1 D^T.
tem_status build_regulariser_tet(tem_ctx *c) {
  const TetTopo &tt = c->tt;
  std::vector<int32_t> pid(tt.n_tets, -1);
  for (size_t p = 0; p < c->params.size(); ++p) pid[c->params[p]] = (int32_t)p;
  std::vector<int32_t> lo, hi;
  std::vector<double> w;
  const size_t nf = tt.iface_opp.size() / 2;
  for (size_t f = 0; f < nf; ++f) {
    const int32_t t1 = tt.iface_tets[2 * f], t2 = tt.iface_tets[2 * f + 1];
    if (pid[t1] < 0 || pid[t2] < 0) continue;
    double d = 0.0;
    for (int side = 0; side < 2; ++side) {
      const int32_t t = tt.iface_tets[2 * f + side];
      double x[12], dg[4];
      for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 3; ++k) x[3 * i + k] = tt.xyz[3 * (size_t)tt.tets[4 * (size_t)t + i] + k];
      tet_rt0_diag(x, dg);
      d += dg[tt.iface_opp[2 * f + side]];
    }
    lo.push_back(std::min(pid[t1], pid[t2]));
    hi.push_back(std::max(pid[t1], pid[t2]));
    w.push_back(1.0 / std::sqrt(d));
  }
  return upload_regulariser(c, lo, hi, w);
}

// Rows (lo, hi, optional weights) and the parameter incidence lists
// (signed row+1) of the transpose.
tem_status upload_regulariser(tem_ctx *c, const std::vector<int32_t> &lo,
                              const std::vector<int32_t> &hi, const std::vector<double> &w) {
  const int P = (int)c->params.size();
  std::vector<int64_t> incp(P + 1, 0);
  for (size_t r = 0; r < lo.size(); ++r) {
    incp[lo[r] + 1]++;
    incp[hi[r] + 1]++;
  }
  for (int p = 0; p < P; ++p) incp[p + 1] += incp[p];
  std::vector<int32_t> inc(incp[P]);
  std::vector<int64_t> fill(incp.begin(), incp.end() - 1);
  for (size_t r = 0; r < lo.size(); ++r) {
    inc[fill[lo[r]]++] = -(int32_t)(r + 1);
    inc[fill[hi[r]]++] = (int32_t)(r + 1);
  }
  c->n_reg = (int64_t)lo.size();
  if (w.empty())
    c->d_reg_w.release();
  else
    HIPCHK(upload(c->d_reg_w, w, c->stream), "upload reg weights");
  HIPCHK(upload(c->d_reg_lo, lo, c->stream), "upload reg");
  HIPCHK(upload(c->d_reg_hi, hi, c->stream), "upload reg");
  HIPCHK(upload(c->d_reg_incp, incp, c->stream), "upload reg");
  HIPCHK(upload(c->d_reg_inc, inc, c->stream), "upload reg");
  return TEM_OK;
}

tem_status build_front_maps(tem_ctx *c, MF &mf) {
  const Symbolic &sym = mf.sym;
  const int ns = (int)sym.nodes.size();
  std::vector<int64_t> first(ns), rows_off(ns), panel_off(ns), cb_off(ns), w_off(ns), gmap_off(ns);
  std::vector<int32_t> kk(ns), uu(ns), child0(ns), child1(ns);
  std::vector<int32_t> rel(sym.rows.size(), -1);
  for (int s = 0; s < ns; ++s) {
    const SymNode &nd = sym.nodes[s];
    first[s] = nd.first;
    kk[s] = (int32_t)(nd.last - nd.first);
    uu[s] = (int32_t)nd.nrows;
    rows_off[s] = nd.rows_off;
    child0[s] = nd.child[0];
    child1[s] = nd.child[1];
  }
  // relative maps: each U_s row's position in the parent's front
  for (int s = 0; s < ns; ++s) {
    const SymNode &nd = sym.nodes[s];
    if (nd.parent < 0) {
      if (nd.nrows) return fail(c, TEM_EINVAL, "root supernode has update rows");
      continue;
    }
    const SymNode &pa = sym.nodes[nd.parent];
    const int32_t *prow = sym.rows.data() + pa.rows_off;
    for (int64_t a = 0; a < nd.nrows; ++a) {
      int32_t q = sym.rows[nd.rows_off + a];
      int64_t pos;
      if (q >= pa.first && q < pa.last) {
        pos = q - pa.first;
      } else {
        const int32_t *it = std::lower_bound(prow, prow + pa.nrows, q);
        if (it == prow + pa.nrows || *it != q)
          return fail(c, TEM_EINVAL, "update row missing from the parent front");
        pos = (pa.last - pa.first) + (it - prow);
      }
      rel[nd.rows_off + a] = (int32_t)pos;
    }
  }
  // levels (depth); factor/solve order is deepest first
  int nl = sym.n_levels;
  mf.levels.assign(nl, LevelInfo());
  mf.x_bb = 0;   // block-inverse offsets follow the new structure
  for (int s = 0; s < ns; ++s) mf.levels[sym.nodes[s].level].nodes.push_back(s);
  std::vector<int32_t> lvl_nodes;
  int64_t poff = 0;
  mf.cb_stride = 0;
  mf.w_rows_max = 0;
  for (int L = nl - 1; L >= 0; --L) {
    LevelInfo &li = mf.levels[L];
    li.n = (int)li.nodes.size();
    li.lvl_begin = (int64_t)lvl_nodes.size();
    lvl_nodes.insert(lvl_nodes.end(), li.nodes.begin(), li.nodes.end());
    li.panel_begin = poff;
    int64_t cbo = 0, wo = 0;
    for (int s : li.nodes) {
      int64_t n = (int64_t)kk[s] + uu[s];
      panel_off[s] = poff;
      poff += panel_size(n, kk[s]);
      cb_off[s] = cbo;
      cbo += (int64_t)uu[s] * uu[s];
      w_off[s] = wo;
      wo += uu[s];
      li.max_k = std::max(li.max_k, kk[s]);
      li.max_u = std::max(li.max_u, uu[s]);
      li.max_n = std::max(li.max_n, (int)n);
      for (int sl = 0; sl < 2; ++sl) {
        int ch = sym.nodes[s].child[sl];
        if (ch >= 0) li.max_u_child[sl] = std::max(li.max_u_child[sl], uu[ch]);
      }
    }
    li.panel_end = poff;
    li.cb_size = cbo;
    li.w_rows = wo;
    mf.cb_stride = std::max(mf.cb_stride, cbo);
    mf.w_rows_max = std::max(mf.w_rows_max, wo);
  }
  mf.pole_stride = poff;
  // original-entry map, level by level (deepest first)
  std::vector<int32_t> amap_csr;
  std::vector<int64_t> amap_pos;
  const Pattern &pat = mf.pat;
  for (int L = nl - 1; L >= 0; --L) {
    LevelInfo &li = mf.levels[L];
    li.amap_begin = (int64_t)amap_csr.size();
    for (int s : li.nodes) {
      const SymNode &nd = sym.nodes[s];
      const int64_t k = nd.last - nd.first, n = k + nd.nrows;
      const int32_t *rw = sym.rows.data() + nd.rows_off;
      for (int64_t j = nd.first; j < nd.last; ++j) {
        for (int64_t t = pat.rowptr[j]; t < pat.rowptr[j + 1]; ++t) {
          int32_t r = pat.col[t];
          if (r < j) continue;
          int64_t lr;
          if (r < nd.last) {
            lr = r - nd.first;
          } else {
            const int32_t *it = std::lower_bound(rw, rw + nd.nrows, r);
            if (it == rw + nd.nrows || *it != r)
              return fail(c, TEM_EINVAL, "matrix entry outside its front");
            lr = k + (it - rw);
          }
          amap_csr.push_back((int32_t)t);
          amap_pos.push_back(panel_off[s] + panel_elem(n, lr, j - nd.first));
        }
      }
    }
    li.amap_end = (int64_t)amap_csr.size();
  }
  // extend-add column lists, level by level and child slot by slot
  std::vector<int32_t> xcols;
  for (int L = nl - 1; L >= 0; --L) {
    LevelInfo &li = mf.levels[L];
    for (int sl = 0; sl < 2; ++sl) {
      li.xa[sl] = (int64_t)xcols.size() / 2;
      for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) li.xm[sl] = (int64_t)xcols.size() / 2;
        for (int s : li.nodes) {
          const int ch = sym.nodes[s].child[sl];
          if (ch < 0) continue;
          const SymNode &cn = sym.nodes[ch];
          for (int64_t bcol = 0; bcol < cn.nrows; ++bcol) {
            const bool to_panel = rel[cn.rows_off + bcol] < kk[s];
            if (to_panel != (pass == 0)) continue;
            xcols.push_back(s);
            xcols.push_back((int32_t)bcol);
          }
        }
      }
      li.xe[sl] = (int64_t)xcols.size() / 2;
    }
  }
  // child gather maps for the solves
  std::vector<int32_t> gmap0, gmap1;
  int64_t goff = 0;
  for (int s = 0; s < ns; ++s) {
    const SymNode &nd = sym.nodes[s];
    const int64_t n = (nd.last - nd.first) + nd.nrows;
    gmap_off[s] = goff;
    gmap0.resize(goff + n, -1);
    gmap1.resize(goff + n, -1);
    for (int sl = 0; sl < 2; ++sl) {
      int ch = nd.child[sl];
      if (ch < 0) continue;
      const SymNode &cn = sym.nodes[ch];
      for (int64_t a = 0; a < cn.nrows; ++a) {
        int32_t pos = rel[cn.rows_off + a];
        (sl == 0 ? gmap0 : gmap1)[goff + pos] = (int32_t)a;
      }
    }
    goff += n;
  }
  hipStream_t st = c->stream;
  HIPCHK(upload(mf.d_first, first, st), "upload first");
  HIPCHK(upload(mf.d_k, kk, st), "upload k");
  HIPCHK(upload(mf.d_u, uu, st), "upload u");
  HIPCHK(upload(mf.d_rows_off, rows_off, st), "upload rows_off");
  HIPCHK(upload(mf.d_rows, sym.rows, st), "upload rows");
  HIPCHK(upload(mf.d_rel, rel, st), "upload rel");
  HIPCHK(upload(mf.d_panel_off, panel_off, st), "upload panel_off");
  HIPCHK(upload(mf.d_cb_off, cb_off, st), "upload cb_off");
  HIPCHK(upload(mf.d_w_off, w_off, st), "upload w_off");
  HIPCHK(upload(mf.d_gmap_off, gmap_off, st), "upload gmap_off");
  HIPCHK(upload(mf.d_gmap0, gmap0, st), "upload gmap0");
  HIPCHK(upload(mf.d_gmap1, gmap1, st), "upload gmap1");
  HIPCHK(upload(mf.d_child0, child0, st), "upload child0");
  HIPCHK(upload(mf.d_child1, child1, st), "upload child1");
  HIPCHK(upload(mf.d_lvl_nodes, lvl_nodes, st), "upload levels");
  HIPCHK(upload(mf.d_amap_csr, amap_csr, st), "upload amap_csr");
  HIPCHK(upload(mf.d_amap_pos, amap_pos, st), "upload amap_pos");
  HIPCHK(upload(mf.d_xcols, xcols, st), "upload extend-add lists");
  HIPCHK(hipStreamSynchronize(st), "sync maps");
  return TEM_OK;
}

hipEvent_t ev_get(tem_ctx *c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// time a launch sequence: call before (returns start event or null)
hipEvent_t span_begin(tem_ctx *c) {
  if (!c->profile) return nullptr;
  hipEvent_t a = ev_get(c);
  if (a) hipEventRecord(a, c->stream);
  return a;
}
void span_end(tem_ctx *c, hipEvent_t a, double work, int kind) {
  if (!c->profile || !a) return;
  hipEvent_t b = ev_get(c);
  if (!b) return;
  hipEventRecord(b, c->stream);
  c->spans.push_back({a, b, work, kind});
}
// fold recorded spans into the totals (after a stream synchronisation)
void spans_collect(tem_ctx *c) {
  for (auto &sp : c->spans) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, sp.a, sp.b) != hipSuccess) continue;
    if (sp.kind == 0) {
      c->upd_ms += ms;
      c->upd_flops += sp.work;
      c->upd_launches++;
    } else {
      c->sweep_ms += ms;
      c->sweep_bytes += sp.work;
      c->sweeps++;
    }
  }
  c->spans.clear();
  c->ev_used = 0;
}

template <typename T>
bool upd_m3(const tem_ctx *c) {
  return sizeof(T) == 4 ? c->upd_m3_f32 : c->upd_m3_f64;
}
// Update variant of level L of system mf: autotuned per level for the edge
// system when available, else the context defaults (FP32 tiles other than
// 64 x 64 only where the tallest front has >= 256 rows below cbeg).
template <typename T>
tem_ctx::UpdCfg upd_cfg(const tem_ctx *c, const MF &mf, int L, int64_t rows) {
  tem_ctx::UpdCfg cf{UPD_T64, upd_m3<T>(c)};
  const bool edge = &mf == &c->ed;
  const std::vector<tem_ctx::UpdCfg> &tab = c->tuned[sizeof(T) == 4 ? 1 : 0];
  if (edge && c->forcing)
    cf = c->forced;
  else if (edge && (int)tab.size() > L)
    cf = tab[L];
  else if (sizeof(T) == 4 && rows >= 256)
    cf.tile = c->upd_tile;
  if (sizeof(T) != 4) cf.tile = UPD_T64;   // FP64 runs 64 x 64 tiles only
  if (cf.tile == UPD_T128) cf.m3 = false;   // 4M only
  if (cf.tile != UPD_T64 && rows < 128) cf.tile = UPD_T64;
  return cf;
}

FrontTab front_tab(const MF &mf, int p0 = 0) {
  FrontTab ft;
  ft.np = mf.d_np.p ? mf.d_np.as<int32_t>() : nullptr;
  ft.p0 = p0;
  ft.first = mf.d_first.as<int64_t>();
  ft.k = mf.d_k.as<int32_t>();
  ft.u = mf.d_u.as<int32_t>();
  ft.rows_off = mf.d_rows_off.as<int64_t>();
  ft.rows = mf.d_rows.as<int32_t>();
  ft.rel = mf.d_rel.as<int32_t>();
  ft.panel_off = mf.d_panel_off.as<int64_t>();
  ft.cb_off = mf.d_cb_off.as<int64_t>();
  ft.w_off = mf.d_w_off.as<int64_t>();
  ft.gmap_off = mf.d_gmap_off.as<int64_t>();
  ft.gmap0 = mf.d_gmap0.as<int32_t>();
  ft.gmap1 = mf.d_gmap1.as<int32_t>();
  ft.child0 = mf.d_child0.as<int32_t>();
  ft.child1 = mf.d_child1.as<int32_t>();
  return ft;
}

const int32_t *lvl_ptr(const MF &mf, const LevelInfo &li) {
  return mf.d_lvl_nodes.as<int32_t>() + li.lvl_begin;
}

// ------------------------------------------------------- factorisation
// Factor g matrices Kv - xi_p Mv (p < g) of system mf into F (pole stride
// mf.pole_stride), using the two contribution-block arenas.
template <typename T>
tem_status factor_group(tem_ctx *c, MF &mf, cpx<T> *F, const double *xi, Seg xseg,
                        const double *Kv, const double *Mv, int p0, int g, cpx<T> *arena0,
                        cpx<T> *arena1) {
  hipStream_t st = c->stream;
  FrontTab ft = front_tab(mf, p0);
  cpx<T> *arena[2] = {arena0, arena1};
  const int nl = (int)mf.levels.size();
  const Symbolic &sym = mf.sym;
  const bool lvl_timing = &mf == &c->ed && c->lvl_timing;
  const size_t ev0 = (size_t)c->lvl_group * nl * 2;
  for (int L = nl - 1; L >= 0; --L) {
    const LevelInfo &li = mf.levels[L];
    const int32_t *ln = lvl_ptr(mf, li);
    cpx<T> *cbL = arena[L & 1];
    cpx<T> *cbC = arena[(L + 1) & 1];
    if (lvl_timing) HIPCHK(hipEventRecord(c->lvl_ev[ev0 + 2 * L], st), "level event");
    HIPCHK(launch_fill_zero<T>(st, F + li.panel_begin, li.panel_end - li.panel_begin, g,
                               mf.pole_stride),
           "zero panels");
    HIPCHK(launch_front_assemble<T>(st, li.amap_end - li.amap_begin,
                                    mf.d_amap_csr.as<int32_t>() + li.amap_begin,
                                    mf.d_amap_pos.as<int64_t>() + li.amap_begin, Kv, Mv, xi, xseg,
                                    g, F, mf.pole_stride),
           "front assemble");
    const int2 *xl = mf.d_xcols.as<int2>();
    for (int sl = 0; sl < 2; ++sl)
      HIPCHK(launch_extend_add<T>(st, ft, xl + li.xa[sl], li.xm[sl] - li.xa[sl], sl, g, F,
                                  mf.pole_stride, cbL, cbC, mf.cb_stride),
             "extend-add into panels");
    // Panels of panel_w columns (256 by default), each factored recursively:
    // the left half of a column range is factored, applied to the right half
    // only (one rank-w/2 update), then the right half is factored; 32-column
    // blocks at the bottom take the diagonal and triangular-solve kernels.
    // The finished panel then updates all later columns at once.  This is
    // the arithmetic of 32-column right-looking steps in another order, with
    // deeper and fewer read-modify-write passes over the panel.
    const int PW = c->panel_w;
    auto trailing = [&](int j0, int dw, int ccap) -> tem_status {
      int64_t max_tiles = 0;
      double fl = 0;
      const tem_ctx::UpdCfg cf = upd_cfg<T>(c, mf, L, li.max_n - j0 - dw);
      const int tt = cf.tile;
      for (int s : li.nodes) {
        const SymNode &nd = sym.nodes[s];
        const int64_t k = nd.last - nd.first, n = k + nd.nrows;
        const int64_t c0 = j0 + dw, c1 = std::min<int64_t>(k, ccap);
        if (c0 >= c1) continue;
        max_tiles = std::max(max_tiles, Tiles::count(n, c0, c1, tt));
        if (c->profile) {
          const double w = (double)std::min<int64_t>(dw, k - j0);
          const double a0 = (double)c0, a1 = (double)c1;
          // lower-trapezoid entries of columns [c0, c1): sum (n - col)
          fl += 8.0 * w * ((a1 - a0) * n - (a1 * (a1 - 1) - a0 * (a0 - 1)) / 2.0) *
                mf.present(s, p0, g);
        }
      }
      if (max_tiles == 0) return TEM_OK;
      hipEvent_t ea = span_begin(c);
      HIPCHK(launch_front_update<T>(st, ft, ln, li.n, 0, j0, dw, ccap, max_tiles, g, F,
                                    mf.pole_stride, cbL, mf.cb_stride, tt, cf.m3),
             "trailing update");
      span_end(c, ea, fl, 0);
      return TEM_OK;
    };
    // columns [j0, j0 + NB); jp = j0 - NB folds in the update of the block
    // just factored (the last one these columns need), jp = -1 none
    auto block = [&](int j0, int jp) -> tem_status {
      int max_rows = 0;
      for (int s : li.nodes) {
        const SymNode &nd = sym.nodes[s];
        const int64_t k = nd.last - nd.first, n = k + nd.nrows;
        if (j0 >= k) continue;
        const int64_t w = std::min<int64_t>(NB, k - j0);
        max_rows = std::max<int>(max_rows, (int)(n - j0 - w));
      }
      HIPCHK(launch_panel_diag<T>(st, ft, ln, li.n, j0, jp, g, F, mf.pole_stride,
                                  c->d_flags.as<int>()),
             "panel diag");
      HIPCHK(launch_panel_trsm<T>(st, ft, ln, li.n, j0, jp, max_rows, g, F, mf.pole_stride),
             "panel trsm");
      return TEM_OK;
    };
    // columns [a, a + w) of the panel, w a multiple of NB; a range of two
    // blocks factors the second with the first's update folded in (the rank-NB
    // update of NB columns, a separate launch otherwise)
    std::function<tem_status(int, int)> factor_range = [&](int a, int w) -> tem_status {
      if (a >= li.max_k) return TEM_OK;
      if (w <= NB) return block(a, -1);
      if (w == 2 * NB) {
        TRY(block(a, -1));
        return a + NB < li.max_k ? block(a + NB, a) : TEM_OK;
      }
      const int h = NB * ((w / NB) / 2);
      TRY(factor_range(a, h));
      TRY(trailing(a, h, a + w));
      return factor_range(a + h, w - h);
    };
    for (int P0 = 0; P0 < li.max_k; P0 += PW) {
      if (c->left_looking) {
        if (P0 > 0) TRY(trailing(0, P0, P0 + PW));
        TRY(factor_range(P0, PW));
      } else {
        TRY(factor_range(P0, PW));
        TRY(trailing(P0, PW, 1 << 30));
      }
    }
    int64_t cb_tiles = 0;
    double fl = 0;
    const tem_ctx::UpdCfg cfc = upd_cfg<T>(c, mf, L, li.max_u);
    const int ttc = cfc.tile;
    for (int s : li.nodes) {
      const SymNode &nd = sym.nodes[s];
      const int64_t k = nd.last - nd.first, n = k + nd.nrows;
      if (nd.nrows > 0) cb_tiles = std::max(cb_tiles, Tiles::count(n, k, n, ttc));
      fl += 8.0 * (double)k * (double)nd.nrows * (double)(nd.nrows + 1) / 2.0 *
            mf.present(s, p0, g);
    }
    if (cb_tiles > 0) {   // (the root level has no contribution block)
      hipEvent_t ea = span_begin(c);
      HIPCHK(launch_front_update<T>(st, ft, ln, li.n, 1, 0, 0, 0, cb_tiles, g, F, mf.pole_stride,
                                    cbL, mf.cb_stride, ttc, cfc.m3),
             "contribution update");
      span_end(c, ea, fl, 0);
    }
    for (int sl = 0; sl < 2; ++sl)
      HIPCHK(launch_extend_add<T>(st, ft, xl + li.xm[sl], li.xe[sl] - li.xm[sl], sl, g, F,
                                  mf.pole_stride, cbL, cbC, mf.cb_stride),
             "extend-add into contribution blocks");
    if (lvl_timing) HIPCHK(hipEventRecord(c->lvl_ev[ev0 + 2 * L + 1], st), "level event");
  }
  return TEM_OK;
}

// ---------------------------------------------------------------- sweeps
// Allocation-free mode: give b a region of at least `bytes` of the static
// scratch array (b keeps a region it already took in this call if it is
// large enough).  Fails with TEM_ENOMEM when the array is exhausted.
tem_status arena_take(tem_ctx *c, DBuf &b, size_t bytes, const char *what) {
  tem_ctx::Arena &a = c->arena;
  bool seen = false;
  for (const tem_ctx::Arena::Saved &sv : a.saved)
    if (sv.b == &b) seen = true;
  if (seen && b.bytes >= bytes) return TEM_OK;
  const size_t off = (a.used + 255) & ~(size_t)255;
  if (off > a.cap || bytes > a.cap - off) {
    char buf[224];
    std::snprintf(buf, sizeof(buf),
                  "%s: the work space of an allocation-free call exceeds the %zu MiB static "
                  "scratch (%zu bytes in use, %zu more requested)",
                  what, a.cap >> 20, off, bytes);
    return fail(c, TEM_ENOMEM, buf);
  }
  if (!seen) a.saved.push_back({&b, b.p, b.bytes});
  b.p = a.base + off;
  b.bytes = bytes;
  b.borrowed = true;
  a.used = off + bytes;
  return TEM_OK;
}

// Scope of an allocation-free call: work space from `base` (cap bytes), no
// device allocation on this thread, eager launches (instantiating a graph
// may allocate) and no profiling events; everything restored on exit.
struct ArenaScope {
  tem_ctx *c;
  bool graphs, profile;
  ArenaScope(tem_ctx *cc, void *base, size_t cap) : c(cc) {
    c->arena.base = (char *)base;
    c->arena.cap = cap;
    c->arena.used = 0;
    c->arena.saved.clear();
    c->arena.on = true;
    graphs = c->use_graphs;
    profile = c->profile;
    c->use_graphs = false;
    c->profile = false;
    t_no_alloc = true;
  }
  ~ArenaScope() {
    // the call's kernels have finished with the scratch before the
    // buffers get their own allocations back (every entry point
    // synchronises its stream on success; this covers the error paths)
    hipStreamSynchronize(c->stream);
    for (size_t i = c->arena.saved.size(); i-- > 0;) {
      const tem_ctx::Arena::Saved &sv = c->arena.saved[i];
      sv.b->p = sv.p;
      sv.b->bytes = sv.bytes;
      sv.b->borrowed = false;
    }
    c->arena.saved.clear();
    c->arena.on = false;
    c->use_graphs = graphs;
    c->profile = profile;
    t_no_alloc = false;
  }
};

// Allocate b; if the device is out of memory, give back the contribution-
// block arenas that the factorisation keeps for the next one (they are idle
// once a factorisation has finished) and try once more.
tem_status alloc_or_reclaim(tem_ctx *c, DBuf &b, size_t bytes, const char *what) {
  hipError_t e = b.alloc(bytes);
  if (e == hipErrorOutOfMemory && (c->d_cb0.p || c->d_cb1.p) && !t_no_alloc) {
    (void)hipGetLastError();   // clear the failed allocation's error
    HIPCHK(hipStreamSynchronize(c->stream), "sync before freeing the arenas");
    c->d_cb0.release();
    c->d_cb1.release();
    e = b.alloc(bytes);
  }
  HIPCHK(e, what);
  return TEM_OK;
}

template <typename T>
tem_status ensure_sweep_ws(tem_ctx *c, MF &mf, int npole, int S) {
  const size_t vec = sizeof(cpx<T>) * (size_t)npole * mf.N * S;
  const size_t wb = sizeof(cpx<T>) * (size_t)npole * std::max<int64_t>(mf.w_rows_max, 1) * S;
  if (c->arena.on) {
    TRY(arena_take(c, mf.w_t, vec, "sweep t"));
    TRY(arena_take(c, mf.w_w0, wb, "sweep w0"));
    return arena_take(c, mf.w_w1, wb, "sweep w1");
  }
  if (mf.w_t.bytes < vec) TRY(alloc_or_reclaim(c, mf.w_t, vec, "alloc sweep t"));
  if (mf.w_w0.bytes < wb) TRY(alloc_or_reclaim(c, mf.w_w0, wb, "alloc sweep w0"));
  if (mf.w_w1.bytes < wb) TRY(alloc_or_reclaim(c, mf.w_w1, wb, "alloc sweep w1"));
  return TEM_OK;
}

// in place: x ([pole][N][S], factor precision) <- A_p^{-1} x for npole
// systems whose factors start at F with stride f_stride (0: one shared factor)
template <typename T>
tem_status sweep_levels(tem_ctx *c, MF &mf, const cpx<T> *F, int64_t f_stride, int npole,
                        cpx<T> *x, int S, int p0 = 0, bool real_l = false) {
  TRY(ensure_sweep_ws<T>(c, mf, npole, S));
  hipStream_t st = c->stream;
  FrontTab ft = front_tab(mf, p0);
  const int64_t N = mf.N;
  cpx<T> *W[2] = {mf.w_w0.as<cpx<T>>(), mf.w_w1.as<cpx<T>>()};
  const int64_t ws = std::max<int64_t>(mf.w_rows_max, 1) * S;
  cpx<T> *t = mf.w_t.as<cpx<T>>();
  const int nl = (int)mf.levels.size();
  // Levels whose fronts are few and wide are walked in big column blocks:
  // one workgroup per front solves a BB-wide diagonal block, then many
  // workgroups apply it to the remaining rows (forward) or columns (backward).
  // In FP32 every level wider than BB is: its triangle kernels then keep a
  // whole block range in registers (at most 256 rows).
  const int64_t BB = c->sweep_bb;
  auto big = [&](const LevelInfo &li) {
    return li.max_k > BB &&
           (sizeof(T) == 4 || (int64_t)li.n * npole < c->sweep_big_limit);
  };
  // FP32 edge factors: the wide fronts' BB-column diagonal blocks are
  // applied through their explicit inverses (k_diag_inverse), the block's
  // solution going through t (free during the forward pass, and after
  // bwd init in the backward pass) so that the launch that uses it can
  // write it into x
  // (the nodal factor's, shared by all its virtual poles, for up to eight
  // right-hand sides)
  const cpx<T> *XI = nullptr;
  int64_t xs = 0;   // elements per pole of the inverses
  if constexpr (sizeof(T) == 4) {
    if (&mf == &c->ed && c->xinv_ok && mf.x_bb == BB && !real_l) {
      XI = c->d_xinv.as<cpx<T>>() + (int64_t)p0 * mf.x_stride;
      xs = mf.x_stride;
    }
  } else {
    if (&mf == &c->nd && c->nxinv_ok && mf.x_bb == BB && real_l && f_stride == 0 && S <= 8)
      XI = c->d_nxinv.as<cpx<T>>();
  }
  const int64_t *xoff = mf.d_xoff.as<int64_t>();
  for (int L = nl - 1; L >= 0; --L) {
    const LevelInfo &li = mf.levels[L];
    const int32_t *ln = lvl_ptr(mf, li);
    if (!big(li)) {
      HIPCHK(launch_fwd_tri<T>(st, ft, ln, li.n, npole, S, N, F, f_stride, x, W[(L + 1) & 1], ws,
                               0, (int64_t)1 << 40, real_l),
             "fwd tri");
    } else if (XI) {
      HIPCHK(launch_fwd_child_add<T>(st, ft, ln, li.n, npole, S, N, x, W[(L + 1) & 1], ws),
             "fwd child add");
      for (int64_t cb = 0; cb < li.max_k; cb += BB) {
        HIPCHK(launch_blk_apply<T>(st, ft, ln, li.n, npole, S, N, XI, xs, xoff, (int)BB, cb,
                                   false, real_l, x, t),
               "fwd block inverse");
        HIPCHK(launch_fwd_rows<T>(st, ft, ln, li.n, (int)std::max<int64_t>(0, li.max_k - cb - BB),
                                  npole, S, N, F, f_stride, x, cb, BB, real_l, t),
               "fwd rows");
      }
    } else {
      for (int64_t cb = 0; cb < li.max_k; cb += BB) {
        HIPCHK(launch_fwd_tri<T>(st, ft, ln, li.n, npole, S, N, F, f_stride, x, W[(L + 1) & 1],
                                 ws, cb, BB, real_l),
               "fwd tri");
        HIPCHK(launch_fwd_rows<T>(st, ft, ln, li.n, (int)std::max<int64_t>(0, li.max_k - cb - BB),
                                  npole, S, N, F, f_stride, x, cb, BB, real_l, nullptr),
               "fwd rows");
      }
    }
    HIPCHK(launch_fwd_rect<T>(st, ft, ln, li.n, li.max_u, npole, S, N, F, f_stride, x,
                              W[(L + 1) & 1], W[L & 1], ws, real_l),
           "fwd rect");
  }
  for (int L = 0; L < nl; ++L) {
    const LevelInfo &li = mf.levels[L];
    const int32_t *ln = lvl_ptr(mf, li);
    HIPCHK(launch_bwd_rect<T>(st, ft, ln, li.n, li.max_k, npole, S, N, F, f_stride, x, t, N * S,
                              real_l),
           "bwd rect");
    if (!big(li)) {
      HIPCHK(launch_bwd_tri<T>(st, ft, ln, li.n, npole, S, N, F, f_stride, x, t, N * S, 0,
                               (int64_t)1 << 40, 1, real_l),
             "bwd tri");
    } else {
      HIPCHK(launch_bwd_init<T>(st, ft, ln, li.n, li.max_k, npole, S, N, F, f_stride, x, t, N * S),
             "bwd init");
      const int64_t nbb = (li.max_k + BB - 1) / BB;
      for (int64_t bb = nbb - 1; bb >= 0; --bb) {
        const int64_t cb = bb * BB;
        if (XI) {
          HIPCHK(launch_blk_apply<T>(st, ft, ln, li.n, npole, S, N, XI, xs, xoff, (int)BB, cb,
                                     true, real_l, x, t),
                 "bwd block inverse");
        } else {
          HIPCHK(launch_bwd_tri<T>(st, ft, ln, li.n, npole, S, N, F, f_stride, x, t, N * S, cb,
                                   BB, 0, real_l),
                 "bwd tri");
        }
        HIPCHK(launch_bwd_cols<T>(st, ft, ln, li.n, cb, npole, S, N, F, f_stride, x, BB, real_l,
                                  XI ? t : nullptr),
               "bwd cols");
      }
    }
  }
  return TEM_OK;
}

// Contiguous pole slots [p0, p0 + n) that still have systems to refine.
struct PoleRun {
  int p0, n;
};
std::vector<PoleRun> all_poles(const tem_ctx *c) { return {PoleRun{0, c->npole}}; }
// runs of pole slots with at least one active system ([mesh][pole][s])
std::vector<PoleRun> active_runs(const tem_ctx *c, const std::vector<int> &active, int S) {
  const int m = c->npole, mS = m * S;
  std::vector<char> on(m, 0);
  for (size_t i = 0; i < active.size(); ++i)
    if (active[i]) on[(i % mS) / S] = 1;
  std::vector<PoleRun> runs;
  for (int p = 0; p < m; ++p) {
    if (!on[p]) continue;
    if (!runs.empty() && runs.back().p0 + runs.back().n == p)
      runs.back().n++;
    else
      runs.push_back({p, 1});
  }
  return runs;
}

// edge sweep with the cached pole factors for the poles of `runs`; x is
// the full [pole][N][S] vector (timed when profiling)
// Capture the all-pole sweep of x into a graph on a private stream (the
// caller's stream may be the legacy default stream, which cannot capture).
template <typename T>
tem_status capture_sweep(tem_ctx *c, cpx<T> *x, int S, tem_ctx::SweepGraph &g) {
  TRY(ensure_sweep_ws<T>(c, c->ed, c->npole, S));   // no allocation while capturing
  if (!c->cap_stream)
    HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream");
  hipStream_t saved = c->stream;
  c->stream = c->cap_stream;
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  tem_status s0 = sweep_levels<T>(c, c->ed, c->d_factor.as<cpx<T>>(), c->ed.pole_stride,
                                  c->npole, x, S, 0);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
  c->stream = saved;
  if (s0 != TEM_OK) {
    if (graph) hipGraphDestroy(graph);
    return s0;
  }
  if (e != hipSuccess) return hip_fail(c, e, "end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(c, e, "instantiate sweep graph");
  if (g.exec) hipGraphExecDestroy(g.exec);
  g.exec = exec;
  g.x = x;
  g.factor = c->d_factor.p;
  g.xinv = c->d_xinv.p;
  g.ws[0] = c->ed.w_t.p;
  g.ws[1] = c->ed.w_w0.p;
  g.ws[2] = c->ed.w_w1.p;
  g.S = S;
  g.npole = c->npole;
  return TEM_OK;
}

template <typename T>
tem_status sweep(tem_ctx *c, cpx<T> *x, int S, const std::vector<PoleRun> &runs) {
  const int64_t N = N_of(c);
  if (c->use_graphs && runs.size() == 1 && runs[0].p0 == 0 && runs[0].n == c->npole) {
    tem_ctx::SweepGraph &g = c->sgraph[sizeof(T) == 4 ? 1 : 0];
    // the graph holds the vector, factor and work-space addresses it was
    // captured with; any change (or a grown work space) means a new capture
    TRY(ensure_sweep_ws<T>(c, c->ed, c->npole, S));
    if (!(g.exec && g.x == x && g.factor == c->d_factor.p && g.xinv == c->d_xinv.p && g.S == S &&
          g.npole == c->npole && g.ws[0] == c->ed.w_t.p && g.ws[1] == c->ed.w_w0.p &&
          g.ws[2] == c->ed.w_w1.p))
      TRY(capture_sweep<T>(c, x, S, g));
    hipEvent_t ea = span_begin(c);
    HIPCHK(hipGraphLaunch(g.exec, c->stream), "sweep graph");
    const double bytes = 2.0 * (double)sizeof(cpx<T>) * (double)c->fac_elems +
                         4.0 * (double)sizeof(cpx<T>) * (double)c->npole * N * S;
    span_end(c, ea, bytes, 1);
    return TEM_OK;
  }
  for (const PoleRun &pr : runs) {
    hipEvent_t ea = span_begin(c);
    TRY(sweep_levels<T>(c, c->ed, c->d_factor.as<cpx<T>>() + (int64_t)pr.p0 * c->ed.pole_stride,
                        c->ed.pole_stride, pr.n, x + (int64_t)pr.p0 * N * S, S, pr.p0));
    // each factor entry of the run's poles is read once forward and once
    // backward; the solution vector is read and written in both passes
    const double bytes =
        2.0 * (double)sizeof(cpx<T>) * (double)c->fac_elems * pr.n / std::max(c->npole, 1) +
        4.0 * (double)sizeof(cpx<T>) * (double)pr.n * N * S;
    span_end(c, ea, bytes, 1);
  }
  return TEM_OK;
}

tem_status ensure_vec(tem_ctx *c, DBuf &b, size_t bytes, const char *what) {
  if (c->arena.on) return arena_take(c, b, bytes, what);
  if (b.bytes != bytes) TRY(alloc_or_reclaim(c, b, bytes, what));
  return TEM_OK;
}

int dot_blocks(int64_t N) {
  int64_t b = (N + 8191) / 8192;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 256));
}

// norms of all systems of v -> host, [segment][pole][s] (one segment per
// mesh of a batch, so that each mesh's systems are judged on their own rows)
tem_status sysnorms(tem_ctx *c, const cpx<double> *v, int S, std::vector<double> &out) {
  const int64_t N = N_of(c);
  const int mS = c->npole * S;
  const int B = n_seg(c);
  const int nb = dot_blocks(N);
  TRY(ensure_vec(c, c->v_partial, sizeof(cpx<double>) * (size_t)nb * mS * 2, "alloc partial"));
  TRY(ensure_vec(c, c->v_dots, sizeof(cpx<double>) * (size_t)B * mS * 64, "alloc dots"));
  for (int b = 0; b < B; ++b) {
    const int64_t r0 = c->B > 0 ? c->row_off[b] : 0, r1 = c->B > 0 ? c->row_off[b + 1] : N;
    HIPCHK(launch_batched_dot(c->stream, r1 - r0, c->npole, S, N * S, v + r0 * S, v + r0 * S, true,
                              c->v_partial.as<cpx<double>>(), dot_blocks(r1 - r0),
                              c->v_dots.as<cpx<double>>() + (size_t)b * mS),
           "norm");
  }
  std::vector<cpx<double>> h((size_t)B * mS);
  HIPCHK(hipMemcpyAsync(h.data(), c->v_dots.p, sizeof(cpx<double>) * B * mS,
                        hipMemcpyDeviceToHost, c->stream),
         "norm d2h");
  HIPCHK(hipStreamSynchronize(c->stream), "norm sync");
  out.resize((size_t)B * mS);
  for (size_t i = 0; i < out.size(); ++i) out[i] = std::sqrt(std::max(h[i].re, 0.0));
  return TEM_OK;
}

// Gradient-space (Galerkin) correction of a preconditioned solve:
// z += G (G^T A_p G)^{-1} G^T (r - A_p z), with G^T A_p G = -xi_p G^T M G
// because K G = 0; one FP64 factor of the nodal matrix G^T M G serves every
// pole.  This removes the error the FP32 factors leave on the
// (nearly singular) gradient modes of the low-conductivity region.
tem_status aux_correct(tem_ctx *c, const cpx<double> *r, cpx<double> *z, int S,
                       const std::vector<PoleRun> &runs) {
  hipStream_t st = c->stream;
  const int64_t N = N_of(c), Nn = c->nd.N;
  const int m = c->npole;
  TRY(ensure_vec(c, c->v_aux, sizeof(cpx<double>) * (size_t)m * S * N, "alloc aux residual"));
  TRY(ensure_vec(c, c->d_nvec,
                 sizeof(cpx<double>) * (size_t)(m * S + 16) * std::max<int64_t>(Nn, 1),
                 "alloc nodal vector"));
  cpx<double> *w = c->v_aux.as<cpx<double>>();
  cpx<double> *y = c->d_nvec.as<cpx<double>>();
  const Seg rs = row_seg(c);
  for (const PoleRun &pr : runs) {
    // the shift and coefficient tables are [mesh][pole]: offsetting them
    // by p0 keeps the (mesh, p0 + p) entry under index mesh * stride + p
    const int64_t o = (int64_t)pr.p0 * N * S;
    HIPCHK(launch_residual_blk(st, N, pr.n, S, c->ed.rb_n, c->ed.d_rb_row.as<int64_t>(),
                               c->ed.d_rb_rows.as<int32_t>(),
                               c->ed.d_rb_hoff.as<int64_t>(), c->ed.d_rb_h.as<int32_t>(),
                               c->ed.rb_packed,
                               c->ed.d_rowptr.as<int64_t>(), c->ed.d_lcol.as<uint16_t>(),
                               c->d_K.as<double>(), c->d_M.as<double>(),
                               c->d_xi.as<double>() + 2 * pr.p0, rs, nullptr, r + o, z + o, w + o),
           "aux residual");
    // the nodal factor is the same for every pole: its sweep takes the
    // run's systems packed S2 = 8 to a virtual pole (eight right-hand sides
    // keep its register triangle kernels at two blocks in flight)
    const int nsys = pr.n * S, S2 = std::min(8, nsys), nv = (nsys + S2 - 1) / S2;
    HIPCHK(launch_grad_T(st, Nn, pr.n, S, S2, N, c->tet ? c->d_node_ptr.as<int64_t>() : nullptr,
                         c->d_node_edges.as<int32_t>(), w + o, y),
           "G^T");
    TRY(sweep_levels<double>(c, c->nd, c->d_nfactor.as<cpx<double>>(), 0, nv, y, S2, 0,
                                   /*real_l=*/true));
    HIPCHK(launch_grad_add(st, N, pr.n, S, S2, Nn, c->d_edge_nodes.as<int32_t>(),
                           c->d_ncoef.as<cpx<double>>() + pr.p0, rs, y, z + o),
           "z += G y");
  }
  return TEM_OK;
}

// out = A^{-1} in (approximately, in the factor precision) for the poles of
// `runs`, FP64 in/out; other poles of out are left undefined
tem_status precond(tem_ctx *c, const cpx<double> *in, cpx<double> *out, int S,
                   const std::vector<PoleRun> &runs) {
  hipStream_t st = c->stream;
  const int64_t N = N_of(c);
  const int m = c->npole;
  const int mS = m * S;
  if (c->prec == TEM_FP64) {
    TRY(ensure_vec(c, c->w_x, sizeof(cpx<double>) * (size_t)mS * N, "alloc sweep x"));
    cpx<double> *x = c->w_x.as<cpx<double>>();
    HIPCHK(hipMemcpyAsync(x, in, sizeof(cpx<double>) * (size_t)mS * N, hipMemcpyDeviceToDevice, st),
           "copy rhs");
    TRY(sweep<double>(c, x, S, runs));
    HIPCHK(hipMemcpyAsync(out, x, sizeof(cpx<double>) * (size_t)mS * N, hipMemcpyDeviceToDevice, st),
           "copy sol");
    return TEM_OK;
  }
  TRY(ensure_vec(c, c->w_x, sizeof(cpx<float>) * (size_t)mS * N, "alloc sweep x"));
  const int nb = dot_blocks(N);
  TRY(ensure_vec(c, c->v_partial, sizeof(cpx<double>) * (size_t)nb * mS * 2, "alloc partial"));
  TRY(ensure_vec(c, c->v_dots, sizeof(cpx<double>) * (size_t)n_seg(c) * mS * 64, "alloc dots"));
  TRY(ensure_vec(c, c->v_inv, sizeof(double) * mS, "alloc inv"));
  TRY(ensure_vec(c, c->v_nrm, sizeof(double) * mS, "alloc nrm"));
  HIPCHK(launch_batched_dot(st, N, m, S, N * S, in, in, true, c->v_partial.as<cpx<double>>(), nb,
                            c->v_dots.as<cpx<double>>()),
         "precond norm");
  HIPCHK(launch_norm_scales(st, mS, c->v_dots.as<cpx<double>>(), c->v_inv.as<double>(),
                            c->v_nrm.as<double>()),
         "precond scales");
  cpx<float> *x = c->w_x.as<cpx<float>>();
  HIPCHK(launch_convert_in<float>(st, N * S, m, S, in, c->v_inv.as<double>(), x), "to fp32");
  TRY(sweep<float>(c, x, S, runs));
  HIPCHK(launch_convert_out<float>(st, N * S, m, S, x, c->v_nrm.as<double>(), out), "to fp64");
  if (c->aux && c->nodal_ready) TRY(aux_correct(c, in, out, S, runs));
  return TEM_OK;
}

struct IrResult {
  std::vector<int> iters;
  std::vector<double> rel;
  int unconverged = 0;
  int solves = 0;
};

// Solve A_p x_ps = f_ps for all systems by classical iterative refinement
// (S <= 16).  f either real [N][S] (same for all poles) or complex
// [pole][N][S]; x: [pole][N][S] complex double.  Each step computes the FP64
// residual r = f - A_p x, judges ||r|| / ||f|| per system against rtol,
// solves A_p z = r through the cached factors (FP32 factors: followed by
// the gradient-space correction) and adds z to x.  Only the contiguous runs
// of pole slots that still hold an unconverged system are swept, corrected
// and have their residual recomputed; converged systems keep x and r.
tem_status refine_block(tem_ctx *c, const double *f_real, const cpx<double> *f_cplx, int S,
                        cpx<double> *x, const tem_ir_opts *ir, IrResult &res) {
  hipStream_t st = c->stream;
  const int64_t N = N_of(c);
  const int m = c->npole;
  const int mS = m * S;
  const double rtol = (ir && ir->rtol > 0) ? ir->rtol : 1e-10;
  const int max_iter = (ir && ir->max_iter > 0) ? ir->max_iter : 200;
  const size_t vbytes = sizeof(cpx<double>) * (size_t)mS * N;
  TRY(ensure_vec(c, c->v_r, vbytes, "alloc r"));
  TRY(ensure_vec(c, c->v_z, vbytes, "alloc z"));
  // systems: [mesh][pole][s] (one mesh unless a batch); absent poles of a
  // mesh in a batch are padding and never active
  const int nsys = n_seg(c) * mS;
  std::vector<char> pad(nsys, 0);
  if (c->B > 0)
    for (int b = 0; b < c->B; ++b)
      for (int p = c->np_mesh[b]; p < m; ++p)
        for (int q = 0; q < S; ++q) pad[(size_t)b * mS + p * S + q] = 1;
  TRY(ensure_vec(c, c->v_coef, sizeof(cpx<double>) * (size_t)mS, "alloc coef"));
  TRY(ensure_vec(c, c->v_mask, sizeof(int) * (size_t)nsys, "alloc mask"));
  cpx<double> *r = c->v_r.as<cpx<double>>();
  cpx<double> *z = c->v_z.as<cpx<double>>();
  const double *xi = c->d_xi.as<double>();
  const Seg rs = row_seg(c);
  auto residual = [&](const std::vector<PoleRun> &runs, const cpx<double> *xv) -> tem_status {
    for (const PoleRun &pr : runs) {
      // the shift table is [mesh][pole]: offsetting it by p0 keeps the
      // (mesh, p0 + p) entry under index mesh * stride + p
      const int64_t o = (int64_t)pr.p0 * N * S;
      if (xv)
        HIPCHK(launch_residual_blk(st, N, pr.n, S, c->ed.rb_n, c->ed.d_rb_row.as<int64_t>(),
                                   c->ed.d_rb_rows.as<int32_t>(),
                                   c->ed.d_rb_hoff.as<int64_t>(), c->ed.d_rb_h.as<int32_t>(),
                                   c->ed.rb_packed,
                                   c->ed.d_rowptr.as<int64_t>(), c->ed.d_lcol.as<uint16_t>(),
                                   c->d_K.as<double>(), c->d_M.as<double>(), xi + 2 * pr.p0, rs,
                                   f_real, f_cplx ? f_cplx + o : nullptr, xv + o, r + o),
               "residual");
      else   // x = 0: r = f
        HIPCHK(launch_residual_init(st, N, pr.n, S, f_real, f_cplx ? f_cplx + o : nullptr, r + o),
               "residual");
    }
    return TEM_OK;
  };
  // x = 0, so that r = f and ||r|| = ||f||
  HIPCHK(launch_fill_f64(st, (double *)x, 2 * (int64_t)mS * N, 0.0), "zero x");
  TRY(residual(all_poles(c), nullptr));
  std::vector<double> fn;
  TRY(sysnorms(c, r, S, fn));
  res.iters.assign(nsys, 0);
  res.rel.assign(nsys, 0.0);
  std::vector<int> active(nsys, 1);
  for (int i = 0; i < nsys; ++i)
    if (fn[i] == 0.0 || pad[i]) active[i] = 0;
  {
    std::vector<cpx<double>> one(mS, {1.0, 0.0});
    HIPCHK(h2d(c->v_coef.p, one.data(), sizeof(cpx<double>) * mS, st), "coef");
  }
  int solves = 0;
  std::vector<double> rn = fn;
  for (int it = 0; it <= max_iter; ++it) {
    bool any = false;
    for (int i = 0; i < nsys; ++i) {
      res.rel[i] = (fn[i] > 0 && !pad[i]) ? rn[i] / fn[i] : 0.0;
      if (active[i] && res.rel[i] <= rtol) active[i] = 0;
      any = any || active[i];
    }
    if (!any || it == max_iter) break;
    const std::vector<PoleRun> runs = active_runs(c, active, S);
    HIPCHK(h2d(c->v_mask.p, active.data(), sizeof(int) * nsys, st), "mask");
    TRY(precond(c, r, z, S, runs));
    ++solves;
    for (int i = 0; i < nsys; ++i)
      if (active[i]) res.iters[i]++;
    HIPCHK(launch_batched_axpy(st, N, m, S, c->v_coef.as<cpx<double>>(), 1.0, z, x,
                               c->v_mask.as<int>(), rs),
           "x += z");
    TRY(residual(runs, x));
    TRY(sysnorms(c, r, S, rn));
  }
  res.unconverged = 0;
  for (int i = 0; i < nsys; ++i)
    if (!(res.rel[i] <= rtol)) res.unconverged++;   // NaN counts as unconverged
  res.solves = solves;
  return TEM_OK;
}

// refine_block for any number of right-hand sides: more than 16 are solved
// in equal blocks of at most 16 (the last one padded with zero right-hand
// sides, which count as converged), gathered from and scattered back to the
// [pole][N][S] vectors.  Single meshes only (a batch has <= 16 per mesh).
tem_status refine_solve(tem_ctx *c, const double *f_real, const cpx<double> *f_cplx, int S,
                        cpx<double> *x, const tem_ir_opts *ir, IrResult &res) {
  if (S <= MAX_BLOCK_RHS) return refine_block(c, f_real, f_cplx, S, x, ir, res);
  if (c->B > 0) return fail(c, TEM_EINVAL, "more than 16 sources per mesh in a batch");
  hipStream_t st = c->stream;
  const int64_t N = N_of(c);
  const int m = c->npole;
  const int nblk = (S + MAX_BLOCK_RHS - 1) / MAX_BLOCK_RHS;
  const int Sb = (S + nblk - 1) / nblk;
  // sized for a complex block, so that real and complex calls share it
  TRY(ensure_vec(c, c->v_fblk, sizeof(cpx<double>) * (size_t)m * N * Sb, "alloc rhs block"));
  TRY(ensure_vec(c, c->v_xblk, sizeof(cpx<double>) * (size_t)m * N * Sb, "alloc solution block"));
  res.iters.assign((size_t)m * S, 0);
  res.rel.assign((size_t)m * S, 0.0);
  res.unconverged = 0;
  res.solves = 0;
  for (int b = 0; b < nblk; ++b) {
    const int s0 = b * Sb, cnt = std::min(Sb, S - s0);
    // doubles per element: 1 (real f) or 2 (complex)
    if (f_real)
      HIPCHK(launch_copy_cols(st, N, f_real, S, s0, cnt, c->v_fblk.as<double>(), Sb, 0, Sb),
             "gather rhs block");
    else
      HIPCHK(launch_copy_cols(st, (int64_t)m * N, (const double *)f_cplx, 2 * S, 2 * s0, 2 * cnt,
                              c->v_fblk.as<double>(), 2 * Sb, 0, 2 * Sb),
             "gather rhs block");
    IrResult rb;
    TRY(refine_block(c, f_real ? c->v_fblk.as<double>() : nullptr,
                     f_real ? nullptr : c->v_fblk.as<cpx<double>>(), Sb,
                     c->v_xblk.as<cpx<double>>(), ir, rb));
    HIPCHK(launch_copy_cols(st, (int64_t)m * N, c->v_xblk.as<double>(), 2 * Sb, 0, 2 * cnt,
                            (double *)x, 2 * S, 2 * s0, 2 * cnt),
           "scatter solution block");
    for (int p = 0; p < m; ++p)
      for (int q = 0; q < cnt; ++q) {
        res.iters[(size_t)p * S + s0 + q] = rb.iters[(size_t)p * Sb + q];
        res.rel[(size_t)p * S + s0 + q] = rb.rel[(size_t)p * Sb + q];
        if (!(rb.rel[(size_t)p * Sb + q] <= ((ir && ir->rtol > 0) ? ir->rtol : 1e-10)))
          res.unconverged++;
      }
    res.solves = std::max(res.solves, rb.solves);
  }
  return TEM_OK;
}

void fill_stats(const IrResult &res, tem_ir_stats *stats) {
  if (!stats) return;
  for (size_t i = 0; i < res.iters.size(); ++i) {
    if (stats->iters) stats->iters[i] = res.iters[i];
    if (stats->final_rel_res) stats->final_rel_res[i] = res.rel[i];
  }
  stats->n_unconverged = res.unconverged;
}

}  // namespace

// ------------------------------------------------ nodal gradient system
tem_status setup_nodal(tem_ctx *c, int leaf) {
  MF &nd = c->nd;
  nd.nodes = true;
  c->nodal_ready = false;
  if (c->mt.n_inodes == 0) return TEM_OK;
  try {
    analyse_symbolic(c->mt, leaf, nd.sym, true);
  } catch (const std::exception &ex) {
    return fail(c, TEM_EINVAL, std::string("nodal analysis: ") + ex.what());
  }
  nd.perm = nd.sym.perm;
  TRY(upload_pattern(c, nd));
  TRY(build_front_maps(c, nd));
  // node -> 6 incident edges (new edge indices), edge -> (start, end) nodes
  const MeshTopo &mt = c->mt;
  const Pattern &ep = c->ed.pat;
  std::vector<int32_t> ne((size_t)nd.N * 6);
  for (int64_t q = 0; q < nd.N; ++q) {
    int64_t v = nd.pat.row_edge[q];
    int i = (int)(v % (mt.nx + 1));
    int64_t rr = v / (mt.nx + 1);
    int j = (int)(rr % (mt.ny + 1)), k = (int)(rr / (mt.ny + 1));
    int64_t es[6] = {mt.xedge(i - 1, j, k), mt.xedge(i, j, k), mt.yedge(i, j - 1, k),
                     mt.yedge(i, j, k),     mt.zedge(i, j, k - 1), mt.zedge(i, j, k)};
    for (int t = 0; t < 6; ++t) {
      int32_t qe = ep.edge_new[es[t]];
      if (qe < 0) return fail(c, TEM_EINVAL, "interior node touches a boundary edge");
      ne[q * 6 + t] = qe;
    }
  }
  std::vector<int32_t> en((size_t)c->ed.N * 2);
  for (int64_t q = 0; q < c->ed.N; ++q) {
    int d, i, j, k;
    mt.geometry(ep.row_edge[q], d, i, j, k);
    int64_t a = mt.node(i, j, k), b = mt.node(i + (d == 0), j + (d == 1), k + (d == 2));
    en[q * 2] = nd.pat.edge_new[a];
    en[q * 2 + 1] = nd.pat.edge_new[b];
  }
  HIPCHK(upload(c->d_node_edges, ne, c->stream), "upload node edges");
  HIPCHK(upload(c->d_edge_nodes, en, c->stream), "upload edge nodes");
  c->h_node_edges = std::move(ne);
  c->h_edge_nodes = std::move(en);
  double le[64];
  element_grad_mass(c->mesh.h, le);
  std::vector<double> lev(le, le + 64);
  HIPCHK(upload(c->d_Le, lev, c->stream), "upload Le");
  const size_t nnz = nd.pat.col.size();
  HIPCHK(c->d_Ln.alloc(sizeof(double) * nnz), "alloc nodal values");
  HIPCHK(c->d_Lzero.alloc(sizeof(double) * nnz), "alloc zeros");
  HIPCHK(launch_fill_f64(c->stream, c->d_Lzero.as<double>(), (int64_t)nnz, 0.0), "zeros");
  std::vector<double> zxi = {0.0, 0.0};
  HIPCHK(upload(c->d_nxi, zxi, c->stream), "upload zero shift");
  HIPCHK(hipStreamSynchronize(c->stream), "nodal setup sync");
  return TEM_OK;
}

// assemble G^T M G for the current sigma and factor it (FP64)
// Offsets of the explicit inverses of the wide fronts' BB-column diagonal
// blocks (levels with max_k > BB, the ones the sweeps may walk in blocks):
// per front 2 ((nbb - 1) BB^2 + w_last^2) elements (each block and its
// transpose, w_last the width of the last block), per pole.
tem_status prepare_xinv(tem_ctx *c, MF &mf, int BB) {
  if (mf.x_bb == BB && mf.d_xoff.p) return TEM_OK;
  std::vector<int64_t> off(std::max<size_t>(mf.sym.nodes.size(), 1), 0);
  int64_t tot = 0;
  for (const LevelInfo &li : mf.levels) {
    if (li.max_k <= BB) continue;
    for (int s : li.nodes) {
      const SymNode &nd = mf.sym.nodes[s];
      const int64_t k = nd.last - nd.first;
      if (k <= 0) continue;
      const int64_t nbb = (k + BB - 1) / BB, wl = k - (nbb - 1) * BB;
      off[s] = tot;
      tot += 2 * ((nbb - 1) * (int64_t)BB * BB + wl * wl);
    }
  }
  HIPCHK(upload(mf.d_xoff, off, c->stream), "upload block-inverse offsets");
  mf.x_stride = tot;
  mf.x_bb = BB;
  return TEM_OK;
}

tem_status factor_nodal(tem_ctx *c) {
  MF &nd = c->nd;
  c->nodal_ready = false;
  if (nd.N == 0) return TEM_OK;
  hipStream_t st = c->stream;
  // coefficients -1/xi of the correction, one per pole slot of each mesh;
  // uploaded first: a copy from pageable memory returns only when the
  // stream has reached it, which must not wait for the factor launched below
  // (the host copy is a member, so it outlives the copy in any case)
  {
    const size_t nco = (size_t)n_seg(c) * c->npole;
    std::vector<double> &coef = c->h_ncoef;
    coef.assign(2 * nco, 0.0);
    for (size_t p = 0; p < nco; ++p) {
      std::complex<double> v = -1.0 / std::complex<double>(c->xi[2 * p], c->xi[2 * p + 1]);
      coef[2 * p] = v.real();
      coef[2 * p + 1] = v.imag();
    }
    HIPCHK(upload(c->d_ncoef, coef, st), "upload coefficients");
  }
  if (c->B > 0) {
    // each mesh assembles its block of the merged nodal matrix
    for (int b = 0; b < c->B; ++b) {
      tem_ctx *sb = c->sub[b];
      const MF &snd = sb->nd;
      if (snd.N == 0) continue;
      HIPCHK(launch_assemble_nodal(st, snd.N, snd.d_rowptr.as<int64_t>(), snd.d_col.as<int32_t>(),
                                   snd.d_row_ent.as<int32_t>(), snd.d_ent_new.as<int32_t>(),
                                   sb->mt.nx, sb->mt.ny, sb->mt.nz, sb->d_Le.as<double>(),
                                   sb->d_sigma.as<double>(),
                                   c->d_Ln.as<double>() + c->nnz_node_off[b]),
             "nodal assembly");
    }
  } else if (c->tet) {
    HIPCHK(launch_tet_gather(st, (int64_t)nd.pat.col.size(), c->d_nent_ptr.as<int64_t>(),
                             c->d_nent_src.as<int32_t>(), 16, c->tt.n_tets, nullptr,
                             c->d_Lt.as<double>(), c->d_sigma.as<double>(), false, nullptr,
                             c->d_Ln.as<double>()),
           "nodal assembly");
  } else {
    HIPCHK(launch_assemble_nodal(st, nd.N, nd.d_rowptr.as<int64_t>(), nd.d_col.as<int32_t>(),
                                 nd.d_row_ent.as<int32_t>(), nd.d_ent_new.as<int32_t>(), c->mt.nx,
                                 c->mt.ny, c->mt.nz, c->d_Le.as<double>(),
                                 c->d_sigma.as<double>(), c->d_Ln.as<double>()),
           "nodal assembly");
  }
  // the nodal factor's wide diagonal blocks get explicit inverses too (one
  // real factor for every pole: one region)
  c->nxinv_ok = false;
  const bool xinv = c->sweep_bb <= 256;
  if (xinv) {
    TRY(prepare_xinv(c, nd, (int)c->sweep_bb));
    HIPCHK(c->d_nxinv.alloc(sizeof(cpx<double>) * (size_t)std::max<int64_t>(nd.x_stride, 1)),
           "alloc nodal block inverses");
  }
  HIPCHK(c->d_nfactor.alloc(sizeof(cpx<double>) * (size_t)std::max<int64_t>(nd.pole_stride, 1)),
         "alloc nodal factor");
  const size_t cbb = sizeof(cpx<double>) * (size_t)std::max<int64_t>(nd.cb_stride, 1);
  HIPCHK(c->d_ncb0.alloc(cbb), "alloc nodal cb");
  HIPCHK(c->d_ncb1.alloc(cbb), "alloc nodal cb");
  // the nodal factor is not part of the timed front-update figures
  const bool prof = c->profile;
  c->profile = false;
  tem_status fs = factor_group<double>(c, nd, c->d_nfactor.as<cpx<double>>(), c->d_nxi.as<double>(),
                                       Seg(), c->d_Ln.as<double>(), c->d_Lzero.as<double>(), 0, 1,
                                       c->d_ncb0.as<cpx<double>>(), c->d_ncb1.as<cpx<double>>());
  c->profile = prof;
  TRY(fs);
  if (xinv && nd.x_stride > 0) {
    const FrontTab ft = front_tab(nd, 0);
    for (const LevelInfo &li : nd.levels)
      if (li.max_k > c->sweep_bb)
        HIPCHK(launch_diag_inverse<double>(st, ft, lvl_ptr(nd, li), li.n, li.max_k, 1,
                                           c->d_nfactor.as<cpx<double>>(), 0,
                                           c->d_nxinv.as<cpx<double>>(), 0,
                                           nd.d_xoff.as<int64_t>(), (int)c->sweep_bb),
               "nodal diagonal-block inverses");
    c->nxinv_ok = true;
  }
  // complete once st reaches this point (the caller orders later work after it)
  c->nodal_ready = true;
  return TEM_OK;
}

// Factor every pole slot of c->xi (a table [mesh][npole] for a batch) in
// precision prec; pole groups when the arenas do not fit beside the factors.
tem_status factor_core(tem_ctx *c, tem_precision prec, const tem_factor_opts *opts) {
  const int m = c->npole;
  HIPCHK(upload(c->d_xi, c->xi, c->stream), "upload xi");
  const size_t esz = prec == TEM_FP64 ? sizeof(cpx<double>) : sizeof(cpx<float>);
  const size_t fbytes = esz * (size_t)c->ed.pole_stride * m;
  const size_t cb_pole = esz * (size_t)std::max<int64_t>(c->ed.cb_stride, 1);
  // FP32: the wide fronts' diagonal-block inverses beside the factors
  const bool xinv = prec == TEM_FP32_IR && c->sweep_bb <= 256;
  c->xinv_ok = false;
  if (xinv) TRY(prepare_xinv(c, c->ed, (int)c->sweep_bb));
  const size_t xbytes = xinv ? sizeof(cpx<float>) * (size_t)c->ed.x_stride * m : 0;
  // a factor buffer of another size and the arenas are given back first;
  // the budget counts what is still held as available.
  if (c->d_factor.bytes != fbytes) c->d_factor.release();
  if (c->d_xinv.bytes != xbytes) c->d_xinv.release();
  size_t free_b = 0, total_b = 0;
  HIPCHK(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
  const int64_t held =
      (int64_t)(c->d_factor.bytes + c->d_xinv.bytes + c->d_cb0.bytes + c->d_cb1.bytes);
  int64_t budget = (opts && opts->mem_budget_bytes > 0)
                       ? opts->mem_budget_bytes
                       : (int64_t)(0.92 * (double)free_b) + held;
  const int64_t fixed = (int64_t)(fbytes + xbytes);
  if (fixed + 2 * (int64_t)cb_pole > budget)
    return fail(c, TEM_ENOMEM, "tem_factor_poles: factors do not fit in the memory budget");
  int g = (int)std::min<int64_t>(m, (budget - fixed) / (2 * (int64_t)cb_pole));
  if (opts && opts->max_group > 0) g = std::min(g, (int)opts->max_group);
  g = std::max(g, 1);
  const int ngroups = (m + g - 1) / g;
  g = (m + ngroups - 1) / ngroups;    // balance the groups
  if (c->d_cb0.bytes != cb_pole * g) {
    c->d_cb0.release();
    c->d_cb1.release();
  }
  HIPCHK(c->d_factor.alloc(fbytes), "alloc factors");
  if (xbytes) HIPCHK(c->d_xinv.alloc(xbytes), "alloc block inverses");
  HIPCHK(c->d_cb0.alloc(cb_pole * g), "alloc cb arena");
  HIPCHK(c->d_cb1.alloc(cb_pole * g), "alloc cb arena");
  HIPCHK(hipMemsetAsync(c->d_flags.p, 0, sizeof(int) * 4, c->stream), "clear flags");
  hipEvent_t e0 = c->t_ev[0], e1 = c->t_ev[1];
  if (c->lvl_timing) {
    const size_t need = (size_t)2 * ngroups * c->ed.levels.size();
    while (c->lvl_ev.size() < need) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e), "event");
      c->lvl_ev.push_back(e);
    }
  }
  HIPCHK(hipEventRecord(e0, c->stream), "event");
  // The nodal factor (FP32 mode) does not depend on the edge factor: it
  // runs on a second stream, joined before the factorisation ends, so its
  // small levels fill gaps of the edge factor's.  Autotuning times the edge
  // levels alone, with the nodal factor after them.
  const bool nodal = prec == TEM_FP32_IR && c->aux;
  const bool overlap = nodal && !c->lvl_timing;
  if (overlap) {
    if (!c->aux_stream)
      HIPCHK(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking), "aux stream");
    if (!c->ev_fork) HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "event");
    if (!c->ev_join) HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "event");
    HIPCHK(hipEventRecord(c->ev_fork, c->stream), "fork");
    HIPCHK(hipStreamWaitEvent(c->aux_stream, c->ev_fork, 0), "fork");
    hipStream_t main = c->stream;
    c->stream = c->aux_stream;
    tem_status s = factor_nodal(c);
    c->stream = main;
    if (s == TEM_OK && hipEventRecord(c->ev_join, c->aux_stream) != hipSuccess)
      s = fail(c, TEM_EDEVICE, "join event");
    if (s != TEM_OK) {
      hipStreamSynchronize(c->aux_stream);
      return s;
    }
  }
  for (int p0 = 0; p0 < m; p0 += g) {
    int gg = std::min(g, m - p0);
    c->lvl_group = p0 / g;
    tem_status s =
        prec == TEM_FP64
            ? factor_group<double>(c, c->ed,
                                   c->d_factor.as<cpx<double>>() + (int64_t)p0 * c->ed.pole_stride,
                                   c->d_xi.as<double>() + 2 * p0, nnz_seg(c), c->d_K.as<double>(),
                                   c->d_M.as<double>(), p0, gg, c->d_cb0.as<cpx<double>>(),
                                   c->d_cb1.as<cpx<double>>())
            : factor_group<float>(c, c->ed,
                                  c->d_factor.as<cpx<float>>() + (int64_t)p0 * c->ed.pole_stride,
                                  c->d_xi.as<double>() + 2 * p0, nnz_seg(c), c->d_K.as<double>(),
                                  c->d_M.as<double>(), p0, gg, c->d_cb0.as<cpx<float>>(),
                                  c->d_cb1.as<cpx<float>>());
    if (s != TEM_OK) {
      if (overlap) hipStreamSynchronize(c->aux_stream);
      return s;
    }
  }
  if (xbytes) {
    // the wide fronts' diagonal blocks are final: their inverses, all poles
    const FrontTab ft = front_tab(c->ed, 0);
    for (const LevelInfo &li : c->ed.levels)
      if (li.max_k > c->sweep_bb)
        HIPCHK(launch_diag_inverse<float>(c->stream, ft, lvl_ptr(c->ed, li), li.n, li.max_k, m,
                                          c->d_factor.as<cpx<float>>(), c->ed.pole_stride,
                                          c->d_xinv.as<cpx<float>>(), c->ed.x_stride,
                                          c->ed.d_xoff.as<int64_t>(), (int)c->sweep_bb),
               "diagonal-block inverses");
  }
  if (overlap) HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join, 0), "join");
  // the arenas stay allocated for the next factorisation of this size; a
  // solve that runs out of device memory gives them back (alloc_or_reclaim)
  if (nodal && !overlap) {
    tem_status s = factor_nodal(c);
    if (s != TEM_OK) {
      return s;
    }
  }
  HIPCHK(hipEventRecord(e1, c->stream), "event");
  HIPCHK(hipEventSynchronize(e1), "factor sync");
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  c->factor_ms = ms;
  spans_collect(c);
  int flags[4];
  HIPCHK(hipMemcpy(flags, c->d_flags.p, sizeof(flags), hipMemcpyDeviceToHost), "flags d2h");
  c->n_tiny = flags[1];
  c->n_groups = ngroups;
  c->group_size = g;
  if (flags[0]) {
    return fail(c, TEM_EPIVOT, "tem_factor_poles: zero or non-finite pivot");
  }
  c->factored = true;
  c->xinv_ok = xbytes > 0;
  return TEM_OK;
}

// ------------------------------------------------------------- batches
// Concatenate the meshes' edge (or nodal) systems into one block-diagonal
// system: mesh b's unknowns follow those of meshes 0..b-1, its supernodes
// keep their depths, so one level of the merged forest holds that level of
// every mesh and each launch covers all of them.
tem_status merge_systems(tem_ctx *c, bool nodes) {
  MF &M = nodes ? c->nd : c->ed;
  Symbolic &S = M.sym;
  Pattern &P = M.pat;
  S.nodes.clear();
  S.perm.clear();
  S.iperm.clear();
  S.rows.clear();
  S.n_levels = 0;
  S.max_front = 0;
  S.flops_per_pole = 0.0;
  S.nnz_l = 0;
  P.rowptr.assign(1, 0);
  P.col.clear();
  P.row_edge.clear();
  std::vector<double> posv;   // entity positions of the rows (edge systems)
  P.edge_new.clear();
  M.h_np.clear();
  M.d_np.release();
  std::vector<int64_t> &roff = nodes ? c->node_off : c->row_off;
  std::vector<int64_t> &zoff = nodes ? c->nnz_node_off : c->nnz_off;
  roff.assign(c->B + 1, 0);
  zoff.assign(c->B + 1, 0);
  int64_t r0 = 0, e0 = 0, z0 = 0;
  int node0 = 0;
  int64_t rows0 = 0;
  for (int b = 0; b < c->B; ++b) {
    const tem_ctx *sb = c->sub[b];
    const MF &m = nodes ? sb->nd : sb->ed;
    const int64_t ents = nodes ? sb->mt.n_nodes : sb->mt.n_edges;
    roff[b] = r0;
    zoff[b] = z0;
    for (SymNode nd : m.sym.nodes) {
      nd.first += r0;
      nd.last += r0;
      nd.sub_first += r0;
      if (nd.parent >= 0) nd.parent += node0;
      for (int t = 0; t < 2; ++t)
        if (nd.child[t] >= 0) nd.child[t] += node0;
      nd.rows_off += rows0;
      S.nodes.push_back(nd);
    }
    for (int32_t q : m.sym.rows) S.rows.push_back((int32_t)(q + r0));
    for (int32_t q : m.perm) S.perm.push_back((int32_t)(q + r0));
    for (int32_t q : m.sym.iperm) S.iperm.push_back((int32_t)(q + r0));
    S.n_levels = std::max(S.n_levels, m.sym.n_levels);
    S.max_front = std::max(S.max_front, m.sym.max_front);
    S.flops_per_pole += m.sym.flops_per_pole;
    S.nnz_l += m.sym.nnz_l;
    for (size_t i = 0; i + 1 < m.pat.rowptr.size(); ++i) P.rowptr.push_back(m.pat.rowptr[i + 1] + z0);
    for (int32_t q : m.pat.col) P.col.push_back((int32_t)(q + r0));
    for (int32_t e : m.pat.row_edge) P.row_edge.push_back((int32_t)(e + e0));
    if (!nodes) {
      const std::vector<double> p = hex_row_positions(sb->mt, m.pat.row_edge);
      posv.insert(posv.end(), p.begin(), p.end());
    }
    for (int32_t q : m.pat.edge_new) P.edge_new.push_back(q >= 0 ? (int32_t)(q + r0) : -1);
    r0 += m.N;
    e0 += ents;
    z0 += (int64_t)m.pat.col.size();
    node0 += (int)m.sym.nodes.size();
    rows0 += (int64_t)m.sym.rows.size();
  }
  roff[c->B] = r0;
  zoff[c->B] = z0;
  if (r0 > ((int64_t)1 << 31) - 1 || e0 > ((int64_t)1 << 31) - 1)
    return fail(c, TEM_EINVAL, "tem_analyse: batch too large for 32-bit indices");
  M.nodes = nodes;
  M.perm = S.perm;
  M.N = r0;
  hipStream_t st = c->stream;
  HIPCHK(upload(M.d_rowptr, P.rowptr, st), "upload rowptr");
  HIPCHK(upload(M.d_col, P.col, st), "upload col");
  HIPCHK(upload(M.d_row_ent, P.row_edge, st), "upload row map");
  HIPCHK(upload(M.d_ent_new, P.edge_new, st), "upload entity map");
  if (!nodes) TRY(build_res_blocks(c, M, P.rowptr, P.col, roff, &posv));
  return build_front_maps(c, M);
}

// merged K, M values from the meshes' own (analysed) assemblies
tem_status batch_values(tem_ctx *c) {
  for (int b = 0; b < c->B; ++b) {
    const tem_ctx *sb = c->sub[b];
    const size_t n = sizeof(double) * (size_t)(c->nnz_off[b + 1] - c->nnz_off[b]);
    HIPCHK(hipMemcpyAsync(c->d_K.as<double>() + c->nnz_off[b], sb->d_K.p, n,
                          hipMemcpyDeviceToDevice, c->stream),
           "copy K block");
    HIPCHK(hipMemcpyAsync(c->d_M.as<double>() + c->nnz_off[b], sb->d_M.p, n,
                          hipMemcpyDeviceToDevice, c->stream),
           "copy M block");
  }
  return TEM_OK;
}

// merged systems, segment tables and the nodal incidence of a batch
tem_status batch_analyse(tem_ctx *c) {
  TRY(merge_systems(c, false));
  TRY(merge_systems(c, true));
  hipStream_t st = c->stream;
  HIPCHK(upload(c->d_row_seg, c->row_off, st), "upload row segments");
  HIPCHK(upload(c->d_nnz_seg, c->nnz_off, st), "upload entry segments");
  const size_t nnz = c->ed.pat.col.size();
  HIPCHK(c->d_K.alloc(sizeof(double) * std::max<size_t>(nnz, 1)), "alloc K");
  HIPCHK(c->d_M.alloc(sizeof(double) * std::max<size_t>(nnz, 1)), "alloc M");
  TRY(batch_values(c));
  // nodal incidence in merged numbering
  std::vector<int32_t> ne, en;
  for (int b = 0; b < c->B; ++b) {
    const tem_ctx *sb = c->sub[b];
    for (int32_t q : sb->h_node_edges) ne.push_back((int32_t)(q + c->row_off[b]));
    for (int32_t a : sb->h_edge_nodes) en.push_back(a >= 0 ? (int32_t)(a + c->node_off[b]) : -1);
  }
  if ((int64_t)en.size() != 2 * c->ed.N || (int64_t)ne.size() != 6 * c->nd.N)
    return fail(c, TEM_EINVAL, "tem_analyse: nodal incidence does not match the merged systems");
  HIPCHK(upload(c->d_node_edges, ne, st), "upload node edges");
  HIPCHK(upload(c->d_edge_nodes, en, st), "upload edge nodes");
  const size_t nnn = c->nd.pat.col.size();
  HIPCHK(c->d_Ln.alloc(sizeof(double) * std::max<size_t>(nnn, 1)), "alloc nodal values");
  HIPCHK(c->d_Lzero.alloc(sizeof(double) * std::max<size_t>(nnn, 1)), "alloc zeros");
  HIPCHK(launch_fill_f64(st, c->d_Lzero.as<double>(), (int64_t)std::max<size_t>(nnn, 1), 0.0),
         "zeros");
  std::vector<double> zxi = {0.0, 0.0};
  HIPCHK(upload(c->d_nxi, zxi, st), "upload zero shift");
  HIPCHK(hipStreamSynchronize(st), "batch analyse sync");
  return TEM_OK;
}

void batch_release(tem_ctx *c) {
  for (tem_ctx *sb : c->sub) tem_destroy(sb);
  c->sub.clear();
  c->B = 0;
  c->MP = 0;
  c->np_mesh.clear();
  c->ed.h_np.clear();
  c->ed.d_np.release();
  c->S_mesh.clear();
  c->R_mesh.clear();
  c->q_row_off.clear();
  c->param_off.clear();
}

// =================================================================== ABI
extern "C" {

tem_status tem_create(tem_ctx **out, int hip_device, void *hip_stream) {
  if (!out) {
    g_create_error = "tem_create: out is NULL";
    return TEM_EINVAL;
  }
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    g_create_error = std::string("tem_create: no HIP device: ") + hipGetErrorString(e);
    return TEM_EDEVICE;
  }
  if (hip_device < 0 || hip_device >= ndev) {
    g_create_error = "tem_create: device index out of range";
    return TEM_EINVAL;
  }
  e = hipSetDevice(hip_device);
  if (e != hipSuccess) {
    g_create_error = std::string("tem_create: hipSetDevice: ") + hipGetErrorString(e);
    return TEM_EDEVICE;
  }
  // device address of the static scratch array on this device (once per
  // device; the allocation-free calls use it)
  e = scratch_setup(hip_device);
  if (e != hipSuccess) {
    g_create_error = std::string("tem_create: scratch address: ") + hipGetErrorString(e);
    return TEM_EDEVICE;
  }
  std::unique_ptr<tem_ctx> c(new tem_ctx());
  c->device = hip_device;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    e = hipStreamCreate(&c->stream);
    if (e != hipSuccess) {
      g_create_error = std::string("tem_create: hipStreamCreate: ") + hipGetErrorString(e);
      return TEM_EDEVICE;
    }
    c->own_stream = true;
  }
  // tuning overrides (used by the tests to exercise both sweep schedules)
  if (const char *v = std::getenv("TEM_SWEEP_BLOCK")) {
    long b = std::strtol(v, nullptr, 10);
    if (b >= NB && b % NB == 0) c->sweep_bb = b;
  }
  if (const char *v = std::getenv("TEM_SWEEP_BIG_LIMIT")) {
    long b = std::strtol(v, nullptr, 10);
    if (b >= 0) c->sweep_big_limit = b;
  }
  if (const char *v = std::getenv("TEM_GRAPHS")) c->use_graphs = std::strtol(v, nullptr, 10) != 0;
  if (const char *v = std::getenv("TEM_PANEL")) {   // panel width: a multiple of 32, 32..1024
    const long w = std::strtol(v, nullptr, 10);
    if (w >= NB && w <= 1024 && w % NB == 0) c->panel_w = (int)w;
  }
  if (const char *v = std::getenv("TEM_LEFT_LOOKING")) c->left_looking = std::strtol(v, nullptr, 10) != 0;
  if (const char *v = std::getenv("TEM_UPDATE_TILE")) {   // "64", "128x64" or "128"
    const std::string m(v);
    if (m != "64" && m != "128x64" && m != "128") {
      g_create_error = "tem_create: TEM_UPDATE_TILE must be 64, 128x64 or 128, not '" + m + "'";
      tem_destroy(c.release());
      return TEM_EINVAL;
    }
    c->upd_tile = m == "64" ? UPD_T64 : m == "128" ? UPD_T128 : UPD_T128x64;
  }
  if (const char *v = std::getenv("TEM_UPDATE_3M")) {   // "f32", "f64", "both" or "none"
    const std::string m(v);
    if (m != "f32" && m != "f64" && m != "both" && m != "none") {
      g_create_error = "tem_create: TEM_UPDATE_3M must be f32, f64, both or none, not '" + m + "'";
      tem_destroy(c.release());
      return TEM_EINVAL;
    }
    c->upd_m3_f32 = m == "f32" || m == "both";
    c->upd_m3_f64 = m == "f64" || m == "both";
  }
  e = c->d_flags.alloc(sizeof(int) * 4);
  if (e != hipSuccess) {
    g_create_error = "tem_create: flags allocation failed";
    tem_destroy(c.release());
    return TEM_ENOMEM;
  }
  for (hipEvent_t &ev : c->t_ev) {
    e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      g_create_error = std::string("tem_create: hipEventCreate: ") + hipGetErrorString(e);
      tem_destroy(c.release());
      return TEM_EDEVICE;
    }
  }
  *out = c.release();
  return TEM_OK;
}

void tem_destroy(tem_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  batch_release(c);
  hipStream_t st = c->stream;
  bool own = c->own_stream;
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  for (hipEvent_t e : c->lvl_ev) hipEventDestroy(e);
  drop_graphs(c);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  if (c->aux_stream) hipStreamDestroy(c->aux_stream);
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  for (hipEvent_t e : c->t_ev)
    if (e) hipEventDestroy(e);
  delete c;
  if (own) hipStreamDestroy(st);
}

const char *tem_last_error(const tem_ctx *c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

tem_status tem_assemble(tem_ctx *c, const tem_mesh *mesh, const double *sigma_cells,
                        int32_t n_params, const int32_t *param_cells) {
  if (!c) return TEM_EINVAL;
  if (!mesh || !sigma_cells) return fail(c, TEM_EINVAL, "tem_assemble: NULL mesh or sigma");
  if (mesh->nx < 2 || mesh->ny < 2 || mesh->nz < 2)
    return fail(c, TEM_EINVAL, "tem_assemble: each axis needs at least 2 cells");
  if (!(mesh->h > 0) || !(mesh->mu > 0) || !std::isfinite(mesh->h) || !std::isfinite(mesh->mu))
    return fail(c, TEM_EINVAL, "tem_assemble: h and mu must be positive and finite");
  const int64_t n_cells = (int64_t)mesh->nx * mesh->ny * mesh->nz;
  if ((int64_t)3 * (mesh->nx + 1) * (mesh->ny + 1) * (mesh->nz + 1) > ((int64_t)1 << 31) - 1)
    return fail(c, TEM_EINVAL, "tem_assemble: mesh too large for 32-bit edge ids");
  if (n_params < 0 || (n_params > 0 && !param_cells))
    return fail(c, TEM_EINVAL, "tem_assemble: bad parameter list");
  std::vector<int32_t> prm(param_cells, param_cells + n_params);
  {
    std::vector<char> seen(n_cells, 0);
    for (int32_t p : prm) {
      if (p < 0 || p >= n_cells) return fail(c, TEM_EINVAL, "tem_assemble: parameter cell out of range");
      if (seen[p]) return fail(c, TEM_EINVAL, "tem_assemble: duplicate parameter cell");
      seen[p] = 1;
    }
  }
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  // validate sigma on the host copy
  std::vector<double> sg(n_cells);
  HIPCHK(hipMemcpy(sg.data(), sigma_cells, sizeof(double) * n_cells, hipMemcpyDeviceToHost),
         "tem_assemble: sigma d2h");
  for (double v : sg)
    if (!(v > 0) || !std::isfinite(v))
      return fail(c, TEM_EINVAL, "tem_assemble: sigma must be positive and finite");
  if (c->B > 0) {   // leaving batch mode
    batch_release(c);
    free_factors(c);
    c->assembled = false;
    c->analysed = false;
  }
  if (c->tet) {   // leaving tetrahedral mode
    release_tet(c);
    free_factors(c);
    c->assembled = false;
    c->analysed = false;
  }
  const bool same_mesh = c->assembled && c->mesh.nx == mesh->nx && c->mesh.ny == mesh->ny &&
                         c->mesh.nz == mesh->nz && c->mesh.h == mesh->h && c->mesh.mu == mesh->mu;
  if (same_mesh)
    drop_factors(c);
  else
    free_factors(c);
  if (!same_mesh) {
    c->analysed = false;
    c->assembled = false;
    c->mesh = *mesh;
    c->mt.init(mesh->nx, mesh->ny, mesh->nz);
    element_mass_unit(mesh->h, c->Me);
    element_stiffness(mesh->h, mesh->mu, c->Ke);
    std::vector<double> ke(c->Ke, c->Ke + 144), me(c->Me, c->Me + 144);
    HIPCHK(upload(c->d_Ke, ke, c->stream), "upload Ke");
    HIPCHK(upload(c->d_Me, me, c->stream), "upload Me");
    c->ed.perm.resize(c->mt.n_unknowns);
    for (int64_t q = 0; q < c->mt.n_unknowns; ++q) c->ed.perm[q] = (int32_t)q;
  }
  HIPCHK(c->d_sigma.alloc(sizeof(double) * n_cells), "alloc sigma");
  HIPCHK(hipMemcpyAsync(c->d_sigma.p, sigma_cells, sizeof(double) * n_cells,
                        hipMemcpyDeviceToDevice, c->stream),
         "copy sigma");
  c->params = prm;
  HIPCHK(upload(c->d_params, c->params, c->stream), "upload params");
  TRY(build_regulariser(c));
  if (!same_mesh) {
    TRY(upload_pattern_and_assemble(c));
  } else {
    TRY(run_assemble_edges(c));
  }
  HIPCHK(hipStreamSynchronize(c->stream), "tem_assemble sync");
  c->assembled = true;
  return TEM_OK;
}

tem_status tem_set_model(tem_ctx *c, const double *m) {
  if (!c) return TEM_EINVAL;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_set_model: not available on a batch of meshes");
  if (!c->assembled) return fail(c, TEM_ESTATE, "tem_set_model: call tem_assemble first");
  if (!m) return fail(c, TEM_EINVAL, "tem_set_model: m is NULL");
  if (c->params.empty()) return fail(c, TEM_EINVAL, "tem_set_model: no model parameters");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  const int P = (int)c->params.size();
  std::vector<double> mh(P);
  HIPCHK(hipMemcpy(mh.data(), m, sizeof(double) * P, hipMemcpyDeviceToHost), "m d2h");
  for (double v : mh)
    if (!std::isfinite(v) || std::fabs(v) > 700.0)
      return fail(c, TEM_EINVAL, "tem_set_model: m must be finite with |m| <= 700");
  drop_factors(c);
  HIPCHK(launch_set_sigma_exp(c->stream, P, c->d_params.as<int32_t>(), m, c->d_sigma.as<double>()),
         "set sigma");
  if (c->tet)
    TRY(run_assemble_tet(c, false));
  else
    TRY(run_assemble_edges(c));
  HIPCHK(hipStreamSynchronize(c->stream), "set_model sync");
  return TEM_OK;
}

tem_status tem_export_operators(const tem_ctx *cc, int64_t *n_unknowns, int64_t *nnz,
                                int32_t *perm, int64_t *rowptr, int32_t *col, double *kval,
                                double *mval) {
  tem_ctx *c = const_cast<tem_ctx *>(cc);
  if (!c) return TEM_EINVAL;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_export_operators: not available on a batch of meshes");
  if (!c->assembled) return fail(c, TEM_ESTATE, "tem_export_operators: nothing assembled");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  const int64_t N = N_of(c), nz = (int64_t)c->ed.pat.col.size();
  if (n_unknowns) *n_unknowns = N;
  if (nnz) *nnz = nz;
  if (perm) std::memcpy(perm, c->ed.perm.data(), sizeof(int32_t) * N);
  if (rowptr) std::memcpy(rowptr, c->ed.pat.rowptr.data(), sizeof(int64_t) * (N + 1));
  if (col) std::memcpy(col, c->ed.pat.col.data(), sizeof(int32_t) * nz);
  HIPCHK(hipStreamSynchronize(c->stream), "export sync");
  if (kval) HIPCHK(hipMemcpy(kval, c->d_K.p, sizeof(double) * nz, hipMemcpyDeviceToHost), "K d2h");
  if (mval) HIPCHK(hipMemcpy(mval, c->d_M.p, sizeof(double) * nz, hipMemcpyDeviceToHost), "M d2h");
  return TEM_OK;
}

tem_status tem_analyse(tem_ctx *c, const tem_analyse_opts *opts, tem_symbolic_info *info) {
  if (!c) return TEM_EINVAL;
  if (!c->assembled) return fail(c, TEM_ESTATE, "tem_analyse: call tem_assemble first");
  int leaf = (opts && opts->leaf_max_cells > 0) ? opts->leaf_max_cells : 4;
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  if (c->B > 0 && (!c->analysed || leaf != c->leaf)) {
    free_factors(c);
    tem_analyse_opts so{};
    so.leaf_max_cells = leaf;
    for (int b = 0; b < c->B; ++b) {
      tem_status sb = tem_analyse(c->sub[b], &so, nullptr);
      if (sb != TEM_OK) return fail(c, sb, std::string("mesh ") + std::to_string(b) + ": " +
                                               tem_last_error(c->sub[b]));
    }
    c->leaf = leaf;
    TRY(batch_analyse(c));
    c->analysed = true;
  }
  if (!c->analysed || leaf != c->leaf) {
    c->tuned[0].clear();
    c->tuned[1].clear();
  }
  if (c->B == 0 && c->tet && (!c->analysed || leaf != c->leaf)) {
    free_factors(c);
    const TetTopo &tt = c->tt;
    std::vector<double> mid((size_t)tt.n_unknowns * 3);
    for (int64_t u = 0; u < tt.n_unknowns; ++u) {
      const int64_t e = tt.edge_of_unk[u];
      for (int k = 0; k < 3; ++k)
        mid[3 * u + k] = 0.5 * (tt.xyz[3 * (size_t)tt.edges[2 * e] + k] +
                                tt.xyz[3 * (size_t)tt.edges[2 * e + 1] + k]);
    }
    try {
      analyse_graph(tt.n_unknowns, tt.adj_ptr, tt.adj, mid, tet_leaf(leaf), c->ed.sym);
    } catch (const std::exception &ex) {
      return fail(c, TEM_EINVAL, std::string("tem_analyse: ") + ex.what());
    }
    c->leaf = leaf;
    c->ed.perm = c->ed.sym.perm;
    TRY(upload_pattern_and_assemble_tet(c));
    TRY(build_front_maps(c, c->ed));
    TRY(setup_nodal_tet(c, leaf));
    c->analysed = true;
  }
  if (c->B == 0 && !c->tet && (!c->analysed || leaf != c->leaf)) {
    free_factors(c);
    try {
      analyse_symbolic(c->mt, leaf, c->ed.sym, false);
    } catch (const std::exception &ex) {
      return fail(c, TEM_EINVAL, std::string("tem_analyse: ") + ex.what());
    }
    c->leaf = leaf;
    c->ed.perm = c->ed.sym.perm;
    TRY(upload_pattern_and_assemble(c));
    TRY(build_front_maps(c, c->ed));
    TRY(setup_nodal(c, leaf));
    c->analysed = true;
  }
  if (info) {
    info->n_unknowns = c->ed.N;
    info->nnz_a = (int64_t)c->ed.pat.col.size();
    info->nnz_l = c->ed.sym.nnz_l;
    info->n_rows_total = (int64_t)c->ed.sym.rows.size();
    info->n_supernodes = (int32_t)c->ed.sym.nodes.size();
    info->n_levels = c->ed.sym.n_levels;
    info->max_front = c->ed.sym.max_front;
    info->reserved = 0;
    info->flops_per_pole = c->ed.sym.flops_per_pole;
  }
  return TEM_OK;
}

tem_status tem_symbolic_host(int32_t nx, int32_t ny, int32_t nz, int32_t leaf_max_cells,
                             tem_symbolic_info *info, int32_t *perm, int32_t *sn_ptr,
                             int32_t *sn_parent, int64_t *rows_ptr, int32_t *rows) {
  if (nx < 2 || ny < 2 || nz < 2) return TEM_EINVAL;
  if ((int64_t)3 * (nx + 1) * (ny + 1) * (nz + 1) > ((int64_t)1 << 31) - 1) return TEM_EINVAL;
  MeshTopo mt;
  Symbolic sym;
  try {
    mt.init(nx, ny, nz);
    analyse_symbolic(mt, leaf_max_cells > 0 ? leaf_max_cells : 4, sym);
  } catch (...) {
    return TEM_EINVAL;
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->n_unknowns = mt.n_unknowns;
    info->nnz_l = sym.nnz_l;
    info->n_rows_total = (int64_t)sym.rows.size();
    info->n_supernodes = (int32_t)sym.nodes.size();
    info->n_levels = sym.n_levels;
    info->max_front = sym.max_front;
    info->flops_per_pole = sym.flops_per_pole;
    Pattern pat;
    build_pattern(mt, sym.perm, pat);
    info->nnz_a = (int64_t)pat.col.size();
  }
  const int ns = (int)sym.nodes.size();
  if (perm) std::memcpy(perm, sym.perm.data(), sizeof(int32_t) * sym.perm.size());
  if (sn_ptr) {
    for (int s = 0; s < ns; ++s) sn_ptr[s] = (int32_t)sym.nodes[s].first;
    sn_ptr[ns] = (int32_t)mt.n_unknowns;
  }
  if (sn_parent)
    for (int s = 0; s < ns; ++s) sn_parent[s] = sym.nodes[s].parent;
  if (rows_ptr) {
    for (int s = 0; s < ns; ++s) rows_ptr[s] = sym.nodes[s].rows_off;
    rows_ptr[ns] = (int64_t)sym.rows.size();
  }
  if (rows) std::memcpy(rows, sym.rows.data(), sizeof(int32_t) * sym.rows.size());
  return TEM_OK;
}

// ------------------------------------------------------ tetrahedral meshes
tem_status tem_assemble_tet(tem_ctx *c, const tem_tet_mesh *mesh, const double *sigma_tets,
                            int32_t n_params, const int32_t *param_tets) {
  if (!c) return TEM_EINVAL;
  if (!mesh || !mesh->xyz || !mesh->tets || !sigma_tets)
    return fail(c, TEM_EINVAL, "tem_assemble_tet: NULL mesh arrays or sigma");
  if (!(mesh->mu > 0) || !std::isfinite(mesh->mu))
    return fail(c, TEM_EINVAL, "tem_assemble_tet: mu must be positive and finite");
  if (mesh->n_tets > ((int64_t)1 << 31) / 36 - 1)
    return fail(c, TEM_EINVAL, "tem_assemble_tet: too many tetrahedra for 32-bit element ids");
  TetTopo tt;
  const std::string err = tt.init(mesh->xyz, mesh->tets, mesh->n_nodes, mesh->n_tets);
  if (!err.empty()) return fail(c, TEM_EINVAL, "tem_assemble_tet: " + err);
  if (tt.n_unknowns == 0) return fail(c, TEM_EINVAL, "tem_assemble_tet: no interior edges");
  const int64_t nt = tt.n_tets;
  if (n_params < 0 || (n_params > 0 && !param_tets))
    return fail(c, TEM_EINVAL, "tem_assemble_tet: bad parameter list");
  std::vector<int32_t> prm(param_tets, param_tets + n_params);
  {
    std::vector<char> seen(nt, 0);
    for (int32_t p : prm) {
      if (p < 0 || p >= nt) return fail(c, TEM_EINVAL, "tem_assemble_tet: parameter tetrahedron out of range");
      if (seen[p]) return fail(c, TEM_EINVAL, "tem_assemble_tet: duplicate parameter tetrahedron");
      seen[p] = 1;
    }
  }
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  std::vector<double> sg(nt);
  HIPCHK(hipMemcpy(sg.data(), sigma_tets, sizeof(double) * nt, hipMemcpyDeviceToHost),
         "tem_assemble_tet: sigma d2h");
  for (double v : sg)
    if (!(v > 0) || !std::isfinite(v))
      return fail(c, TEM_EINVAL, "tem_assemble_tet: sigma must be positive and finite");
  if (c->B > 0) batch_release(c);
  free_factors(c);
  release_tet(c);
  c->assembled = false;
  c->analysed = false;
  c->mesh = tem_mesh{};
  c->mt = MeshTopo();
  c->nd.N = 0;
  c->nodal_ready = false;
  c->tuned[0].clear();
  c->tuned[1].clear();
  c->tet = true;
  c->tt = std::move(tt);
  c->tet_mu = mesh->mu;
  hipStream_t st = c->stream;
  HIPCHK(upload(c->d_xyz, c->tt.xyz, st), "upload coordinates");
  HIPCHK(upload(c->d_tetv, c->tt.tets, st), "upload tetrahedra");
  HIPCHK(upload(c->d_tsign, c->tt.tet_signs, st), "upload edge signs");
  HIPCHK(c->d_sigma.alloc(sizeof(double) * nt), "alloc sigma");
  HIPCHK(hipMemcpyAsync(c->d_sigma.p, sigma_tets, sizeof(double) * nt, hipMemcpyDeviceToDevice, st),
         "copy sigma");
  c->params = prm;
  HIPCHK(upload(c->d_params, c->params, st), "upload params");
  TRY(build_regulariser_tet(c));
  c->ed.perm.resize(c->tt.n_unknowns);
  for (int64_t q = 0; q < c->tt.n_unknowns; ++q) c->ed.perm[q] = (int32_t)q;
  TRY(upload_pattern_and_assemble_tet(c));
  HIPCHK(hipStreamSynchronize(st), "tem_assemble_tet sync");
  c->assembled = true;
  return TEM_OK;
}

tem_status tem_symbolic_tet_host(const tem_tet_mesh *mesh, int32_t leaf_max_cells,
                                 tem_symbolic_info *info, int32_t *perm, int32_t *sn_ptr,
                                 int32_t *sn_parent, int64_t *rows_ptr, int32_t *rows) {
  if (!mesh || !mesh->xyz || !mesh->tets) return TEM_EINVAL;
  TetTopo tt;
  Symbolic sym;
  try {
    if (!tt.init(mesh->xyz, mesh->tets, mesh->n_nodes, mesh->n_tets).empty()) return TEM_EINVAL;
    std::vector<double> mid((size_t)tt.n_unknowns * 3);
    for (int64_t u = 0; u < tt.n_unknowns; ++u) {
      const int64_t e = tt.edge_of_unk[u];
      for (int k = 0; k < 3; ++k)
        mid[3 * u + k] = 0.5 * (tt.xyz[3 * (size_t)tt.edges[2 * e] + k] +
                                tt.xyz[3 * (size_t)tt.edges[2 * e + 1] + k]);
    }
    analyse_graph(tt.n_unknowns, tt.adj_ptr, tt.adj, mid,
                  tet_leaf(leaf_max_cells > 0 ? leaf_max_cells : 4), sym);
  } catch (...) {
    return TEM_EINVAL;
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->n_unknowns = tt.n_unknowns;
    info->nnz_a = (int64_t)tt.adj.size();
    info->nnz_l = sym.nnz_l;
    info->n_rows_total = (int64_t)sym.rows.size();
    info->n_supernodes = (int32_t)sym.nodes.size();
    info->n_levels = sym.n_levels;
    info->max_front = sym.max_front;
    info->flops_per_pole = sym.flops_per_pole;
  }
  const int ns = (int)sym.nodes.size();
  if (perm) std::memcpy(perm, sym.perm.data(), sizeof(int32_t) * sym.perm.size());
  if (sn_ptr) {
    for (int s = 0; s < ns; ++s) sn_ptr[s] = (int32_t)sym.nodes[s].first;
    sn_ptr[ns] = (int32_t)tt.n_unknowns;
  }
  if (sn_parent)
    for (int s = 0; s < ns; ++s) sn_parent[s] = sym.nodes[s].parent;
  if (rows_ptr) {
    for (int s = 0; s < ns; ++s) rows_ptr[s] = sym.nodes[s].rows_off;
    rows_ptr[ns] = (int64_t)sym.rows.size();
  }
  if (rows) std::memcpy(rows, sym.rows.data(), sizeof(int32_t) * sym.rows.size());
  return TEM_OK;
}

tem_status tem_factor_poles(tem_ctx *c, int32_t m, const double *xi, tem_precision prec,
                            const tem_factor_opts *opts) {
  if (!c) return TEM_EINVAL;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_factor_poles: not available on a batch of meshes");
  if (!c->analysed) return fail(c, TEM_ESTATE, "tem_factor_poles: call tem_analyse first");
  if (m <= 0 || !xi) return fail(c, TEM_EINVAL, "tem_factor_poles: need m > 0 poles");
  if (m > 65535) return fail(c, TEM_EINVAL, "tem_factor_poles: too many poles");
  if (prec != TEM_FP64 && prec != TEM_FP32_IR)
    return fail(c, TEM_EINVAL, "tem_factor_poles: unknown precision");
  for (int i = 0; i < m; ++i) {
    if (!std::isfinite(xi[2 * i]) || !std::isfinite(xi[2 * i + 1]) || !(xi[2 * i + 1] > 0))
      return fail(c, TEM_EINVAL, "tem_factor_poles: poles need finite values and Im > 0");
  }
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  drop_factors(c);
  if (m != c->npole) c->surveyed = false;   // residues are per pole
  c->w_x.release();
  c->v_fblk.release();
  c->v_xblk.release();
  c->npole = m;
  c->prec = prec;
  c->xi.assign(xi, xi + 2 * m);
  c->fac_elems = c->ed.pole_stride * (int64_t)m;
  return factor_core(c, prec, opts);
}

tem_status tem_solve_poles(tem_ctx *c, int32_t nrhs, const double *F, double *G,
                           const tem_ir_opts *ir, tem_ir_stats *stats) {
  if (!c) return TEM_EINVAL;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_solve_poles: not available on a batch of meshes");
  if (!c->factored) return fail(c, TEM_ESTATE, "tem_solve_poles: call tem_factor_poles first");
  if (nrhs <= 0 || nrhs > 1024 || !F)
    return fail(c, TEM_EINVAL, "tem_solve_poles: need 1 <= nrhs <= 1024 and a source array");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  const int64_t N = N_of(c);
  const int S = nrhs;
  hipStream_t st = c->stream;
  c->solved = false;
  TRY(ensure_vec(c, c->d_fnew, sizeof(double) * (size_t)N * S, "alloc f"));
  HIPCHK(launch_gather_rhs(st, N, S, S, n_ent(c), c->ed.d_row_ent.as<int32_t>(), F,
                           c->d_fnew.as<double>()),
         "gather f");
  TRY(ensure_vec(c, c->d_g, sizeof(cpx<double>) * (size_t)c->npole * N * S, "alloc g"));
  hipEvent_t e0 = c->t_ev[0], e1 = c->t_ev[1];
  HIPCHK(hipEventRecord(e0, st), "event");
  IrResult res;
  tem_status s = refine_solve(c, c->d_fnew.as<double>(), nullptr, S, c->d_g.as<cpx<double>>(), ir, res);
  hipEventRecord(e1, st);
  hipEventSynchronize(e1);
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  if (s != TEM_OK) return s;
  c->solve_ms = ms;
  spans_collect(c);
  c->last_solves = res.solves;
  c->S = S;
  if (G) {
    HIPCHK(launch_scatter_solution(st, N, c->npole, S, n_ent(c), c->ed.d_ent_new.as<int32_t>(),
                                   c->d_g.as<cpx<double>>(), (cpx<double> *)G),
           "scatter g");
  }
  HIPCHK(hipStreamSynchronize(st), "solve sync");
  fill_stats(res, stats);
  c->solved = true;
  if (res.unconverged) {
    double worst = 0;
    for (double v : res.rel) worst = std::max(worst, v);
    char buf[160];
    std::snprintf(buf, sizeof(buf), "tem_solve_poles: %d systems above rtol (worst %.3e) after %d solves",
                  res.unconverged, worst, res.solves);
    return fail(c, TEM_ENOCONV, buf);
  }
  return TEM_OK;
}

static tem_status set_survey(tem_ctx *c, int R, const int64_t *q_ptr, const int32_t *q_col,
                             const double *q_val, int K, const double *alpha) {
  if (R <= 0 || K <= 0 || !q_ptr || !q_col || !q_val || !alpha)
    return fail(c, TEM_EINVAL, "tem_forward: bad receivers or residues");
  if (q_ptr[0] != 0) return fail(c, TEM_EINVAL, "tem_forward: q_ptr[0] must be 0");
  const int64_t nnz = q_ptr[R];
  std::vector<int64_t> qp(R + 1, 0);
  std::vector<int32_t> qc;
  std::vector<double> qv;
  for (int r = 0; r < R; ++r) {
    if (q_ptr[r + 1] < q_ptr[r] || q_ptr[r + 1] > nnz)
      return fail(c, TEM_EINVAL, "tem_forward: q_ptr not monotone");
    for (int64_t t = q_ptr[r]; t < q_ptr[r + 1]; ++t) {
      if (q_col[t] < 0 || q_col[t] >= n_ent(c))
        return fail(c, TEM_EINVAL, "tem_forward: receiver column out of range");
      if (!std::isfinite(q_val[t])) return fail(c, TEM_EINVAL, "tem_forward: non-finite Q value");
      int32_t q = c->ed.pat.edge_new[q_col[t]];
      if (q < 0) continue;   // boundary edge: the field is zero there
      qc.push_back(q);
      qv.push_back(q_val[t]);
    }
    qp[r + 1] = (int64_t)qc.size();
  }
  for (int64_t i = 0; i < 2 * (int64_t)K * c->npole; ++i)
    if (!std::isfinite(alpha[i])) return fail(c, TEM_EINVAL, "tem_forward: non-finite residue");
  std::vector<double> al(alpha, alpha + 2 * (size_t)K * c->npole);
  HIPCHK(upload(c->d_qptr, qp, c->stream), "upload q_ptr");
  HIPCHK(upload(c->d_qcol, qc, c->stream), "upload q_col");
  HIPCHK(upload(c->d_qval, qv, c->stream), "upload q_val");
  HIPCHK(upload(c->d_alpha, al, c->stream), "upload alpha");
  c->R = R;
  c->K = K;
  return TEM_OK;
}

tem_status tem_forward(tem_ctx *c, int32_t S, const double *F, int32_t R, const int64_t *q_ptr,
                       const int32_t *q_col, const double *q_val, int32_t K, const double *alpha,
                       const tem_ir_opts *ir, double *d, tem_ir_stats *stats) {
  if (!c) return TEM_EINVAL;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_forward: not available on a batch of meshes");
  if (!c->factored) return fail(c, TEM_ESTATE, "tem_forward: call tem_factor_poles first");
  if (!d) return fail(c, TEM_EINVAL, "tem_forward: d is NULL");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  // the cached solutions and survey belong together: until this call has
  // both, Jv / J^T w are refused
  c->surveyed = false;
  TRY(set_survey(c, R, q_ptr, q_col, q_val, K, alpha));
  tem_status s = tem_solve_poles(c, S, F, nullptr, ir, stats);
  if (s != TEM_OK && s != TEM_ENOCONV) return s;
  HIPCHK(launch_time_assembly(c->stream, S, K, R, c->npole, N_of(c), S, c->d_qptr.as<int64_t>(),
                              c->d_qcol.as<int32_t>(), c->d_qval.as<double>(),
                              c->d_alpha.as<cpx<double>>(), c->d_g.as<cpx<double>>(), d),
         "time assembly");
  HIPCHK(hipStreamSynchronize(c->stream), "forward sync");
  c->surveyed = true;
  return s;
}

tem_status tem_jvp(tem_ctx *c, const double *v, double *jv, const tem_ir_opts *ir,
                   tem_ir_stats *stats) {
  if (!c) return TEM_EINVAL;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_jvp: not available on a batch of meshes");
  if (!c->surveyed || !c->solved) return fail(c, TEM_ESTATE, "tem_jvp: call tem_forward first");
  if (c->params.empty()) return fail(c, TEM_EINVAL, "tem_jvp: no model parameters");
  if (!v || !jv) return fail(c, TEM_EINVAL, "tem_jvp: NULL argument");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  hipStream_t st = c->stream;
  const int64_t N = N_of(c);
  const int S = c->S, m = c->npole;
  TRY(ensure_vec(c, c->v_vs, sizeof(double) * (size_t)n_cells_of(c), "alloc vs"));
  TRY(ensure_vec(c, c->v_rhs, sizeof(cpx<double>) * (size_t)m * N * S, "alloc rhs"));
  TRY(ensure_vec(c, c->v_lam, sizeof(cpx<double>) * (size_t)m * N * S, "alloc sol"));
  HIPCHK(launch_param_scatter(st, (int)c->params.size(), c->d_params.as<int32_t>(), v,
                              c->d_sigma.as<double>(), n_cells_of(c), c->v_vs.as<double>()),
         "param scatter");
  if (c->tet)
    HIPCHK(launch_jv_rhs_tet(st, N, m, S, S, N * S, c->d_et_ptr.as<int64_t>(),
                             c->d_et_src.as<int32_t>(), c->d_tet_new.as<int32_t>(), c->tt.n_tets,
                             c->v_vs.as<double>(), c->d_Mt.as<double>(), c->d_xi.as<double>(),
                             c->d_g.as<cpx<double>>(), c->v_rhs.as<cpx<double>>()),
           "jv rhs");
  else
    HIPCHK(launch_jv_rhs(st, N, m, S, S, N * S, c->mt.nx, c->mt.ny, c->mt.nz,
                         c->ed.d_row_ent.as<int32_t>(), c->d_cell_new.as<int32_t>(),
                         c->v_vs.as<double>(), c->d_Me.as<double>(), c->d_xi.as<double>(),
                         c->d_g.as<cpx<double>>(), c->v_rhs.as<cpx<double>>()),
           "jv rhs");
  IrResult res;
  TRY(refine_solve(c, nullptr, c->v_rhs.as<cpx<double>>(), S, c->v_lam.as<cpx<double>>(), ir, res));
  HIPCHK(launch_time_assembly(st, S, c->K, c->R, m, N, S, c->d_qptr.as<int64_t>(),
                              c->d_qcol.as<int32_t>(), c->d_qval.as<double>(),
                              c->d_alpha.as<cpx<double>>(), c->v_lam.as<cpx<double>>(), jv),
         "jv time assembly");
  HIPCHK(hipStreamSynchronize(st), "jvp sync");
  spans_collect(c);
  fill_stats(res, stats);
  c->last_solves = res.solves;
  if (res.unconverged) return fail(c, TEM_ENOCONV, "tem_jvp: refinement did not converge");
  return TEM_OK;
}

tem_status tem_vjp(tem_ctx *c, const double *w, double *jtw, const tem_ir_opts *ir,
                   tem_ir_stats *stats) {
  if (!c) return TEM_EINVAL;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_vjp: not available on a batch of meshes");
  if (!c->surveyed || !c->solved) return fail(c, TEM_ESTATE, "tem_vjp: call tem_forward first");
  if (c->params.empty()) return fail(c, TEM_EINVAL, "tem_vjp: no model parameters");
  if (!w || !jtw) return fail(c, TEM_EINVAL, "tem_vjp: NULL argument");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  hipStream_t st = c->stream;
  const int64_t N = N_of(c);
  const int S = c->S, m = c->npole;
  TRY(ensure_vec(c, c->v_rhs, sizeof(cpx<double>) * (size_t)m * N * S, "alloc rhs"));
  TRY(ensure_vec(c, c->v_lam, sizeof(cpx<double>) * (size_t)m * N * S, "alloc sol"));
  HIPCHK(launch_fill_f64(st, (double *)c->v_rhs.p, 2 * N * m * S, 0.0), "zero rhs");
  HIPCHK(launch_jtw_rhs(st, S, S, N * S, c->K, c->R, m, c->d_qptr.as<int64_t>(),
                        c->d_qcol.as<int32_t>(), c->d_qval.as<double>(),
                        c->d_alpha.as<cpx<double>>(), w, c->v_rhs.as<cpx<double>>()),
         "jtw rhs");
  IrResult res;
  TRY(refine_solve(c, nullptr, c->v_rhs.as<cpx<double>>(), S, c->v_lam.as<cpx<double>>(), ir, res));
  if (c->tet)
    HIPCHK(launch_jtw_reduce_tet(st, (int)c->params.size(), m, S, S, N * S,
                                 c->d_params.as<int32_t>(), c->d_tet_new.as<int32_t>(),
                                 c->tt.n_tets, c->d_sigma.as<double>(), c->d_Mt.as<double>(),
                                 c->d_xi.as<double>(), c->d_g.as<cpx<double>>(),
                                 c->v_lam.as<cpx<double>>(), jtw),
           "jtw reduce");
  else
    HIPCHK(launch_jtw_reduce(st, (int)c->params.size(), m, S, S, N * S,
                             c->d_params.as<int32_t>(), c->d_cell_new.as<int32_t>(),
                             c->d_sigma.as<double>(), c->d_Me.as<double>(), c->d_xi.as<double>(),
                             c->d_g.as<cpx<double>>(), c->v_lam.as<cpx<double>>(), jtw),
           "jtw reduce");
  HIPCHK(hipStreamSynchronize(st), "vjp sync");
  spans_collect(c);
  fill_stats(res, stats);
  c->last_solves = res.solves;
  if (res.unconverged) return fail(c, TEM_ENOCONV, "tem_vjp: refinement did not converge");
  return TEM_OK;
}

tem_status tem_vjp_noalloc(tem_ctx *c, const double *w, double *jtw, const tem_ir_opts *ir,
                           tem_ir_stats *stats) {
  if (!c) return TEM_EINVAL;
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  void *base = scratch_ptr(c->device);
  if (!base) return fail(c, TEM_EDEVICE, "tem_vjp_noalloc: no scratch address for this device");
  tem_status s;
  {
    ArenaScope scope(c, base, SCRATCH_BYTES);
    s = tem_vjp(c, w, jtw, ir, stats);
  }
  if (s != TEM_OK && s != TEM_ENOCONV) {
    const std::string m = c->err;
    return fail(c, s, m.compare(0, 16, "tem_vjp_noalloc:") == 0 ? m : "tem_vjp_noalloc: " + m);
  }
  return s;
}

static tem_status lsqr_norm(tem_ctx *c, int64_t n, const double *a, double &out) {
  HIPCHK(launch_rdot(c->stream, n, a, a, c->l_part.as<double>(), c->l_scal.as<double>()), "dot");
  double v = 0;
  HIPCHK(hipMemcpyAsync(&v, c->l_scal.p, sizeof(double), hipMemcpyDeviceToHost, c->stream), "d2h");
  HIPCHK(hipStreamSynchronize(c->stream), "sync");
  out = std::sqrt(std::max(v, 0.0));
  return TEM_OK;
}

// LSQR on the Gauss-Newton least-squares problem at the current model (the
// one the cached factors and solutions belong to).  With slope != NULL also
// returns grad phi(m)^T dm for phi = ||W_d (d - d_obs)||^2 + lambda
// ||R (m - m_ref)||^2: the first bidiagonalisation step gives
// A^T b = alpha_1 beta_1 v_1 = -grad phi / 2, so the slope is
// -2 alpha_1 beta_1 v_1^T dm (no further solve).
tem_status gn_lsqr(tem_ctx *c, const double *d_obs, const double *wd, const double *m,
                   const double *m_ref, double lambda, int32_t iters, double *dm, double *hist,
                   const tem_ir_opts *ir, double *slope) {
  hipStream_t st = c->stream;
  const int64_t nd = (int64_t)c->S * c->K * c->R, nr = c->n_reg, nu = nd + nr;
  const int P = (int)c->params.size();
  const double sl = std::sqrt(lambda);
  TRY(ensure_vec(c, c->l_u, sizeof(double) * nu, "alloc lsqr"));
  TRY(ensure_vec(c, c->l_v, sizeof(double) * P, "alloc lsqr"));
  TRY(ensure_vec(c, c->l_w, sizeof(double) * P, "alloc lsqr"));
  TRY(ensure_vec(c, c->l_x, sizeof(double) * P, "alloc lsqr"));
  TRY(ensure_vec(c, c->l_tmpd, sizeof(double) * nd, "alloc lsqr"));
  TRY(ensure_vec(c, c->l_tmpm, sizeof(double) * P, "alloc lsqr"));
  TRY(ensure_vec(c, c->l_part, sizeof(double) * 64 * std::max(iters + 1, 4), "alloc lsqr"));
  TRY(ensure_vec(c, c->l_scal, sizeof(double) * (iters + 1), "alloc lsqr"));
  // the v vectors of the bidiagonalisation, kept for reorthogonalisation
  TRY(ensure_vec(c, c->l_V, sizeof(double) * (size_t)P * (iters + 1), "alloc lsqr basis"));
  double *Vb = c->l_V.as<double>();
  double *u = c->l_u.as<double>(), *v = c->l_v.as<double>(), *w = c->l_w.as<double>();
  double *x = c->l_x.as<double>(), *td = c->l_tmpd.as<double>(), *tm = c->l_tmpm.as<double>();
  const int32_t *rlo = c->d_reg_lo.as<int32_t>(), *rhi = c->d_reg_hi.as<int32_t>();
  const double *rw = c->d_reg_w.as<double>();
  // A v = [W_d J v ; sqrt(lam) R v] -> u (times a, plus b u)
  auto matvec = [&](const double *vin, double a, double b) -> tem_status {
    TRY(tem_jvp(c, vin, td, ir, nullptr));
    HIPCHK(launch_raxpby(st, nd, a, td, wd, b, u), "u data");
    HIPCHK(launch_reg(st, nr, rlo, rhi, rw, a * sl, vin, b, u + nd), "u reg");
    return TEM_OK;
  };
  // A^T u = J^T (W_d u_d) + sqrt(lam) R^T u_r -> v (times a, plus b v)
  auto rmatvec = [&](double a, double b) -> tem_status {
    HIPCHK(launch_raxpby(st, nd, 1.0, u, wd, 0.0, td), "W u");
    TRY(tem_vjp(c, td, tm, ir, nullptr));
    HIPCHK(launch_raxpby(st, P, a, tm, nullptr, b, v), "v data");
    HIPCHK(launch_regT(st, P, c->d_reg_incp.as<int64_t>(), c->d_reg_inc.as<int32_t>(), rw,
                       a * sl, u + nd, 1.0, v),
           "v reg");
    return TEM_OK;
  };
  // b = -[W_d (d(m) - d_obs); sqrt(lam) R (m - m_ref)]
  HIPCHK(launch_time_assembly(st, c->S, c->K, c->R, c->npole, N_of(c), c->S,
                              c->d_qptr.as<int64_t>(),
                              c->d_qcol.as<int32_t>(), c->d_qval.as<double>(),
                              c->d_alpha.as<cpx<double>>(), c->d_g.as<cpx<double>>(), td),
         "d(m)");
  HIPCHK(launch_raxpby(st, nd, -1.0, d_obs, nullptr, 1.0, td), "d - d_obs");
  HIPCHK(launch_raxpby(st, nd, -1.0, td, wd, 0.0, u), "b data");
  HIPCHK(launch_raxpby(st, P, 1.0, m, nullptr, 0.0, tm), "m");
  HIPCHK(launch_raxpby(st, P, -1.0, m_ref, nullptr, 1.0, tm), "m - m_ref");
  HIPCHK(launch_reg(st, nr, rlo, rhi, rw, -sl, tm, 0.0, u + nd), "b reg");
  double beta, alpha;
  TRY(lsqr_norm(c, nu, u, beta));
  if (beta > 0) HIPCHK(launch_raxpby(st, nu, 0.0, nullptr, nullptr, 1.0 / beta, u), "u /= beta");
  HIPCHK(launch_raxpby(st, P, 0.0, nullptr, nullptr, 0.0, v), "v = 0");
  TRY(rmatvec(1.0, 0.0));
  TRY(lsqr_norm(c, P, v, alpha));
  const double ab1 = alpha * beta;
  if (alpha > 0) HIPCHK(launch_raxpby(st, P, 0.0, nullptr, nullptr, 1.0 / alpha, v), "v /= alpha");
  HIPCHK(launch_raxpby(st, P, 1.0, v, nullptr, 0.0, Vb), "V0 = v");
  HIPCHK(launch_raxpby(st, P, 1.0, v, nullptr, 0.0, w), "w = v");
  HIPCHK(launch_raxpby(st, P, 0.0, nullptr, nullptr, 0.0, x), "x = 0");
  double phibar = beta, rhobar = alpha;
  for (int it = 0; it < iters; ++it) {
    TRY(matvec(v, 1.0, -alpha));                  // u = A v - alpha u
    TRY(lsqr_norm(c, nu, u, beta));
    if (beta > 0) HIPCHK(launch_raxpby(st, nu, 0.0, nullptr, nullptr, 1.0 / beta, u), "u scale");
    TRY(rmatvec(1.0, -beta));                     // v = A^T u - beta v
    // one-sided reorthogonalisation: v against every earlier v, twice
    for (int pass = 0; pass < 2; ++pass)
      HIPCHK(launch_reorth(st, P, it + 1, Vb, v, c->l_part.as<double>(), c->l_scal.as<double>()),
             "reorthogonalise v");
    TRY(lsqr_norm(c, P, v, alpha));
    if (alpha > 0) HIPCHK(launch_raxpby(st, P, 0.0, nullptr, nullptr, 1.0 / alpha, v), "v scale");
    HIPCHK(launch_raxpby(st, P, 1.0, v, nullptr, 0.0, Vb + (size_t)P * (it + 1)), "store v");
    const double rho = std::hypot(rhobar, beta);
    if (rho == 0) {   // the bidiagonalisation has ended: x solves the problem
      if (hist)
        for (int k = it; k < iters; ++k) hist[k] = phibar;
      break;
    }
    const double cs = rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    rhobar = -cs * alpha;
    const double phi = cs * phibar;
    phibar = sn * phibar;
    HIPCHK(launch_raxpby(st, P, phi / rho, w, nullptr, 1.0, x), "x update");
    HIPCHK(launch_raxpby(st, P, 1.0, v, nullptr, -theta / rho, w), "w update");
    if (hist) hist[it] = phibar;
  }
  HIPCHK(hipMemcpyAsync(dm, x, sizeof(double) * P, hipMemcpyDeviceToDevice, st), "dm");
  if (slope) {
    double v1x = 0.0;
    HIPCHK(launch_rdot(st, P, Vb, x, c->l_part.as<double>(), c->l_scal.as<double>()), "v1 . dm");
    HIPCHK(hipMemcpyAsync(&v1x, c->l_scal.p, sizeof(double), hipMemcpyDeviceToHost, st), "d2h");
    HIPCHK(hipStreamSynchronize(st), "sync");
    *slope = -2.0 * ab1 * v1x;
  }
  HIPCHK(hipStreamSynchronize(st), "gn sync");
  return TEM_OK;
}

tem_status tem_gn_step(tem_ctx *c, const double *d_obs, const double *wd, const double *m,
                       const double *m_ref, double lambda, int32_t iters, double *dm,
                       double *hist, const tem_ir_opts *ir) {
  if (!c) return TEM_EINVAL;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_gn_step: not available on a batch of meshes");
  if (!c->surveyed || !c->solved) return fail(c, TEM_ESTATE, "tem_gn_step: call tem_forward first");
  if (c->params.empty()) return fail(c, TEM_EINVAL, "tem_gn_step: no model parameters");
  if (!d_obs || !wd || !m || !m_ref || !dm || iters <= 0 || !(lambda >= 0) || !std::isfinite(lambda))
    return fail(c, TEM_EINVAL, "tem_gn_step: bad argument");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  return gn_lsqr(c, d_obs, wd, m, m_ref, lambda, iters, dm, hist, ir, nullptr);
}

// ------------------------------------------------------------ inversion
// ||a||^2 of n device doubles (host result)
static tem_status sq_norm(tem_ctx *c, int64_t n, const double *a, double &out) {
  double r = 0.0;
  TRY(lsqr_norm(c, n, a, r));
  out = r * r;
  return TEM_OK;
}

// misfit ||W_d (d - d_obs)||^2 and roughness ||R (m - m_ref)||^2 (device
// inputs; work buffers inv_t1 (nd), inv_t2 (P), inv_t3 (n_reg))
static tem_status objective_parts(tem_ctx *c, const double *d, const double *d_obs,
                                  const double *wd, const double *m, const double *m_ref,
                                  double &mis, double &reg) {
  hipStream_t st = c->stream;
  const int64_t nd = (int64_t)c->S * c->K * c->R;
  const int P = (int)c->params.size();
  double *t1 = c->inv_t1.as<double>(), *t2 = c->inv_t2.as<double>(), *t3 = c->inv_t3.as<double>();
  HIPCHK(launch_raxpby(st, nd, 1.0, d, nullptr, 0.0, t1), "d");
  HIPCHK(launch_raxpby(st, nd, -1.0, d_obs, nullptr, 1.0, t1), "d - d_obs");
  HIPCHK(launch_raxpby(st, nd, 1.0, t1, wd, 0.0, t1), "W_d (d - d_obs)");
  TRY(sq_norm(c, nd, t1, mis));
  HIPCHK(launch_raxpby(st, P, 1.0, m, nullptr, 0.0, t2), "m");
  HIPCHK(launch_raxpby(st, P, -1.0, m_ref, nullptr, 1.0, t2), "m - m_ref");
  HIPCHK(launch_reg(st, c->n_reg, c->d_reg_lo.as<int32_t>(), c->d_reg_hi.as<int32_t>(),
                    c->d_reg_w.as<double>(), 1.0, t2, 0.0, t3),
         "R (m - m_ref)");
  TRY(sq_norm(c, c->n_reg, t3, reg));
  return TEM_OK;
}

// the forward map at the context's current model: factor every pole (the
// poles and precision of the last factorisation), solve for the sources of
// the last tem_forward (kept in the new ordering) and assemble the data
// into d; fac_s receives the factorisation's wall time
static tem_status forward_current(tem_ctx *c, const tem_ir_opts *ir, double *d, double &fac_s) {
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<double> xi = c->xi;
  TRY(tem_factor_poles(c, c->npole, xi.data(), c->prec, nullptr));
  fac_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  const int64_t N = N_of(c);
  const int S = c->S;
  TRY(ensure_vec(c, c->d_g, sizeof(cpx<double>) * (size_t)c->npole * N * S, "alloc g"));
  IrResult res;
  TRY(refine_solve(c, c->d_fnew.as<double>(), nullptr, S, c->d_g.as<cpx<double>>(), ir, res));
  spans_collect(c);
  c->last_solves = res.solves;
  if (res.unconverged) return fail(c, TEM_ENOCONV, "refinement did not converge in a forward solve");
  c->solved = true;
  HIPCHK(launch_time_assembly(c->stream, S, c->K, c->R, c->npole, N, S, c->d_qptr.as<int64_t>(),
                              c->d_qcol.as<int32_t>(), c->d_qval.as<double>(),
                              c->d_alpha.as<cpx<double>>(), c->d_g.as<cpx<double>>(), d),
         "time assembly");
  HIPCHK(hipStreamSynchronize(c->stream), "forward sync");
  return TEM_OK;
}

// next trial step length after a failed trial at eta: the minimiser of the
// quadratic through phi(0), phi'(0) = slope and phi(eta), kept in
// [eta/10, eta/2] (eta/2 when that quadratic is not convex)
static double next_trial(double phi0, double slope, double eta, double phi_eta) {
  const double cq = (phi_eta - phi0 - slope * eta) / (eta * eta);
  if (!(cq > 0.0)) return 0.5 * eta;
  const double s = -slope / (2.0 * cq);
  return std::min(std::max(s, 0.1 * eta), 0.5 * eta);
}

tem_status tem_invert(tem_ctx *c, const double *d_obs, const double *wd, double *m,
                      const double *m_ref, const tem_invert_opts *opts, const tem_ir_opts *ir,
                      tem_invert_record *log, int32_t *n_records) {
  if (!c) return TEM_EINVAL;
  if (n_records) *n_records = 0;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_invert: not available on a batch of meshes");
  if (!c->surveyed || !c->solved) return fail(c, TEM_ESTATE, "tem_invert: call tem_forward first");
  if (c->params.empty()) return fail(c, TEM_EINVAL, "tem_invert: no model parameters");
  if (!d_obs || !wd || !m || !m_ref || !opts || !log)
    return fail(c, TEM_EINVAL, "tem_invert: NULL argument");
  const double lam0 = opts->lambda0;
  const double chi2_target = opts->chi2_target > 0 ? opts->chi2_target : 1.0;
  const double c1 = opts->c1 > 0 ? opts->c1 : 1e-4;
  const double eta_min = opts->eta_min > 0 ? opts->eta_min : 1.0 / 32.0;
  const double conv_rtol = opts->conv_rtol > 0 ? opts->conv_rtol : 1e-2;
  if (!(lam0 > 0) || !std::isfinite(lam0) || opts->max_gn <= 0 || opts->lsqr_iters <= 0 ||
      !(eta_min < 1.0) || !(c1 < 1.0))
    return fail(c, TEM_EINVAL, "tem_invert: need lambda0 > 0, max_gn >= 1, lsqr_iters >= 1, "
                               "c1 < 1 and eta_min < 1");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  hipStream_t st = c->stream;
  const int64_t nd = (int64_t)c->S * c->K * c->R;
  const int P = (int)c->params.size();
  TRY(ensure_vec(c, c->inv_d, sizeof(double) * nd, "alloc inversion"));
  TRY(ensure_vec(c, c->inv_dt, sizeof(double) * nd, "alloc inversion"));
  TRY(ensure_vec(c, c->inv_mt, sizeof(double) * P, "alloc inversion"));
  TRY(ensure_vec(c, c->inv_dm, sizeof(double) * P, "alloc inversion"));
  TRY(ensure_vec(c, c->inv_t1, sizeof(double) * nd, "alloc inversion"));
  TRY(ensure_vec(c, c->inv_t2, sizeof(double) * P, "alloc inversion"));
  TRY(ensure_vec(c, c->inv_t3, sizeof(double) * std::max<int64_t>(c->n_reg, 1), "alloc inversion"));
  // LSQR's reduction buffers, sized as gn_lsqr sizes them
  TRY(ensure_vec(c, c->l_part, sizeof(double) * 64 * std::max(opts->lsqr_iters + 1, 4),
                 "alloc inversion"));
  TRY(ensure_vec(c, c->l_scal, sizeof(double) * (opts->lsqr_iters + 1), "alloc inversion"));
  double *d = c->inv_d.as<double>(), *dt = c->inv_dt.as<double>();
  double *mt = c->inv_mt.as<double>(), *dm = c->inv_dm.as<double>();
  // the data at m: the time assembly of the cached solutions
  HIPCHK(launch_time_assembly(st, c->S, c->K, c->R, c->npole, N_of(c), c->S,
                              c->d_qptr.as<int64_t>(), c->d_qcol.as<int32_t>(),
                              c->d_qval.as<double>(), c->d_alpha.as<cpx<double>>(),
                              c->d_g.as<cpx<double>>(), d),
         "d(m0)");
  double lam = lam0;
  int nrec = 0;
  for (int it = 0; it < opts->max_gn; ++it) {
    const auto t0 = std::chrono::steady_clock::now();
    double fac_s = 0.0;
    tem_invert_record rec{};
    double mis, reg;
    TRY(objective_parts(c, d, d_obs, wd, m, m_ref, mis, reg));
    const double phi = mis + lam * reg;
    rec.lambda = lam;
    rec.chi2 = mis / (double)nd;
    rec.phi = phi;
    if (rec.chi2 <= chi2_target) {
      rec.stop = 1;
      log[nrec++] = rec;
      break;
    }
    double slope = 0.0;
    TRY(gn_lsqr(c, d_obs, wd, m, m_ref, lam, opts->lsqr_iters, dm, nullptr, ir, &slope));
    rec.slope = slope;
    rec.lsqr_iters = opts->lsqr_iters;
    double eta = 1.0, phit = phi;
    bool ok = false;
    for (;;) {
      HIPCHK(launch_raxpby(st, P, 1.0, m, nullptr, 0.0, mt), "m_t = m");
      HIPCHK(launch_raxpby(st, P, eta, dm, nullptr, 1.0, mt), "m_t += eta dm");
      TRY(tem_set_model(c, mt));
      TRY(forward_current(c, ir, dt, fac_s));
      double mis_t, reg_t;
      TRY(objective_parts(c, dt, d_obs, wd, mt, m_ref, mis_t, reg_t));
      phit = mis_t + lam * reg_t;
      rec.trials++;
      if (phit <= phi + c1 * eta * slope) {
        ok = true;
        break;
      }
      const double nxt = next_trial(phi, slope, eta, phit);
      if (nxt < eta_min) break;
      eta = nxt;
    }
    rec.accepted = ok ? 1 : 0;
    rec.eta = eta;
    rec.phi_new = ok ? phit : phi;
    if (ok) {
      // the context is factored and solved at m_t already
      HIPCHK(hipMemcpyAsync(m, mt, sizeof(double) * P, hipMemcpyDeviceToDevice, st), "m = m_t");
      HIPCHK(hipMemcpyAsync(d, dt, sizeof(double) * nd, hipMemcpyDeviceToDevice, st), "d = d_t");
      if (phi - phit < conv_rtol * phi) lam *= 0.5;
    } else {
      // back to m: its factors and solutions are needed by the next step
      TRY(tem_set_model(c, m));
      TRY(forward_current(c, ir, d, fac_s));
      lam *= 0.5;
    }
    HIPCHK(hipStreamSynchronize(st), "inversion sync");
    rec.factor_seconds = fac_s;
    rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    log[nrec++] = rec;
  }
  if (n_records) *n_records = nrec;
  return TEM_OK;
}

tem_status tem_set_profiling(tem_ctx *c, int32_t enable) {
  if (!c) return TEM_EINVAL;
  c->profile = enable != 0;
  c->upd_ms = c->upd_flops = c->sweep_ms = c->sweep_bytes = 0;
  c->upd_launches = c->sweeps = 0;
  return TEM_OK;
}

// --------------------------------------------------------- batches
tem_status tem_assemble_batch(tem_ctx *c, int32_t n_mesh, const tem_mesh *meshes,
                              const double *sigma_cells) {
  if (!c) return TEM_EINVAL;
  if (n_mesh <= 0 || n_mesh > 4096 || !meshes || !sigma_cells)
    return fail(c, TEM_EINVAL, "tem_assemble_batch: need 1..4096 meshes and sigma");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  bool same = c->B == n_mesh && c->assembled;
  for (int b = 0; same && b < n_mesh; ++b) {
    const tem_mesh &a = c->sub[b]->mesh, &m = meshes[b];
    same = a.nx == m.nx && a.ny == m.ny && a.nz == m.nz && a.h == m.h && a.mu == m.mu;
  }
  if (!same) {
    free_factors(c);
    batch_release(c);
    if (c->tet) release_tet(c);
    c->assembled = false;
    c->analysed = false;
    c->mesh = tem_mesh{};
    c->mt = MeshTopo();
    c->params.clear();
    for (int b = 0; b < n_mesh; ++b) {
      tem_ctx *sb = nullptr;
      tem_status st = tem_create(&sb, c->device, (void *)c->stream);
      if (st != TEM_OK) {
        batch_release(c);
        return fail(c, st, "tem_assemble_batch: cannot create a mesh context");
      }
      c->sub.push_back(sb);
    }
    c->B = n_mesh;
  } else {
    drop_factors(c);
  }
  c->cell_off.assign(n_mesh + 1, 0);
  for (int b = 0; b < n_mesh; ++b)
    c->cell_off[b + 1] =
        c->cell_off[b] + (int64_t)meshes[b].nx * meshes[b].ny * meshes[b].nz;
  for (int b = 0; b < n_mesh; ++b) {
    tem_status st = tem_assemble(c->sub[b], &meshes[b], sigma_cells + c->cell_off[b], 0, nullptr);
    if (st != TEM_OK) {
      std::string msg = std::string("tem_assemble_batch: mesh ") + std::to_string(b) + ": " +
                        tem_last_error(c->sub[b]);
      batch_release(c);
      c->assembled = false;
      c->analysed = false;
      return fail(c, st, msg);
    }
  }
  if (c->analysed) {
    // same meshes, new conductivities: refresh the merged values
    TRY(batch_values(c));
    HIPCHK(hipStreamSynchronize(c->stream), "tem_assemble_batch sync");
  }
  c->assembled = true;
  return TEM_OK;
}

tem_status tem_factor_poles_batch(tem_ctx *c, const int32_t *m, const double *xi,
                                  tem_precision prec, const tem_factor_opts *opts) {
  if (!c) return TEM_EINVAL;
  if (c->B == 0) return fail(c, TEM_ESTATE, "tem_factor_poles_batch: no batch assembled");
  if (!c->analysed) return fail(c, TEM_ESTATE, "tem_factor_poles_batch: call tem_analyse first");
  if (!m || !xi) return fail(c, TEM_EINVAL, "tem_factor_poles_batch: NULL pole counts or poles");
  if (prec != TEM_FP64 && prec != TEM_FP32_IR)
    return fail(c, TEM_EINVAL, "tem_factor_poles_batch: unknown precision");
  int MP = 0;
  int64_t tot = 0;
  for (int b = 0; b < c->B; ++b) {
    if (m[b] <= 0 || m[b] > 4096)
      return fail(c, TEM_EINVAL, "tem_factor_poles_batch: every mesh needs 1..4096 poles");
    MP = std::max(MP, (int)m[b]);
    tot += m[b];
  }
  for (int64_t i = 0; i < tot; ++i)
    if (!std::isfinite(xi[2 * i]) || !std::isfinite(xi[2 * i + 1]) || !(xi[2 * i + 1] > 0))
      return fail(c, TEM_EINVAL, "tem_factor_poles_batch: poles need finite values and Im > 0");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  drop_factors(c);
  c->surveyed = false;
  c->w_x.release();
  c->v_fblk.release();
  c->v_xblk.release();
  // pole table [mesh][MP]; absent slots repeat the mesh's last pole (never
  // computed: the kernels skip them, the table only stays well defined)
  c->np_mesh.assign(m, m + c->B);
  c->MP = MP;
  c->npole = MP;
  c->prec = prec;
  c->xi.assign(2 * (size_t)c->B * MP, 0.0);
  c->fac_elems = 0;
  int64_t o = 0;
  for (int b = 0; b < c->B; ++b) {
    for (int p = 0; p < MP; ++p) {
      const int64_t src = o + std::min(p, m[b] - 1);
      c->xi[2 * ((size_t)b * MP + p)] = xi[2 * src];
      c->xi[2 * ((size_t)b * MP + p) + 1] = xi[2 * src + 1];
    }
    o += m[b];
    c->fac_elems += (int64_t)m[b] * c->sub[b]->ed.pole_stride;
  }
  // pole count of every merged front
  MF &e = c->ed;
  e.h_np.assign(e.sym.nodes.size(), 0);
  int node0 = 0;
  for (int b = 0; b < c->B; ++b) {
    const int nn = (int)c->sub[b]->ed.sym.nodes.size();
    for (int q = 0; q < nn; ++q) e.h_np[node0 + q] = m[b];
    node0 += nn;
  }
  HIPCHK(upload(e.d_np, e.h_np, c->stream), "upload pole counts");
  return factor_core(c, prec, opts);
}

tem_status tem_forward_batch(tem_ctx *c, const int32_t *S, const double *F, const int32_t *R,
                             const int64_t *q_ptr, const int32_t *q_col, const double *q_val,
                             int32_t K, const double *alpha, const tem_ir_opts *ir, double *d,
                             tem_ir_stats *stats) {
  if (!c) return TEM_EINVAL;
  if (c->B == 0) return fail(c, TEM_ESTATE, "tem_forward_batch: no batch assembled");
  if (!c->factored) return fail(c, TEM_ESTATE, "tem_forward_batch: call tem_factor_poles_batch first");
  if (!S || !F || !R || !q_ptr || !q_col || !q_val || !alpha || !d || K <= 0)
    return fail(c, TEM_EINVAL, "tem_forward_batch: NULL argument or K <= 0");
  const int B = c->B, MP = c->MP;
  int Smax = 0;
  for (int b = 0; b < B; ++b) {
    if (S[b] <= 0 || S[b] > 16) return fail(c, TEM_EINVAL, "tem_forward_batch: need 1 <= S <= 16");
    if (R[b] <= 0) return fail(c, TEM_EINVAL, "tem_forward_batch: need R > 0 receivers");
    Smax = std::max(Smax, (int)S[b]);
  }
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  hipStream_t st = c->stream;
  const int64_t N = N_of(c);
  c->surveyed = false;
  // receivers in merged numbering, residues [mesh][K][MP] (0 for absent poles)
  std::vector<int64_t> qp(1, 0), qrow(B + 1, 0);
  std::vector<int32_t> qc;
  std::vector<double> qv;
  std::vector<double> al(2 * (size_t)B * K * MP, 0.0);
  int64_t po = 0, zo = 0, ao = 0;
  for (int b = 0; b < B; ++b) {
    const tem_ctx *sb = c->sub[b];
    const int64_t *pp = q_ptr + po;
    if (pp[0] != 0) return fail(c, TEM_EINVAL, "tem_forward_batch: each q_ptr block starts at 0");
    for (int r = 0; r < R[b]; ++r) {
      if (pp[r + 1] < pp[r]) return fail(c, TEM_EINVAL, "tem_forward_batch: q_ptr not monotone");
      for (int64_t t = pp[r]; t < pp[r + 1]; ++t) {
        const int32_t e = q_col[zo + t];
        const double v = q_val[zo + t];
        if (e < 0 || e >= sb->mt.n_edges)
          return fail(c, TEM_EINVAL, "tem_forward_batch: receiver column out of range");
        if (!std::isfinite(v)) return fail(c, TEM_EINVAL, "tem_forward_batch: non-finite Q value");
        const int32_t q = sb->ed.pat.edge_new[e];
        if (q < 0) continue;   // boundary edge: the field is zero there
        qc.push_back((int32_t)(q + c->row_off[b]));
        qv.push_back(v);
      }
      qp.push_back((int64_t)qc.size());
    }
    qrow[b + 1] = qrow[b] + R[b];
    zo += pp[R[b]];
    po += R[b] + 1;
    for (int j = 0; j < K; ++j)
      for (int p = 0; p < c->np_mesh[b]; ++p) {
        const double ar = alpha[2 * (ao + (int64_t)j * c->np_mesh[b] + p)];
        const double ai = alpha[2 * (ao + (int64_t)j * c->np_mesh[b] + p) + 1];
        if (!std::isfinite(ar) || !std::isfinite(ai))
          return fail(c, TEM_EINVAL, "tem_forward_batch: non-finite residue");
        al[2 * (((size_t)b * K + j) * MP + p)] = ar;
        al[2 * (((size_t)b * K + j) * MP + p) + 1] = ai;
      }
    ao += (int64_t)K * c->np_mesh[b];
  }
  HIPCHK(upload(c->d_qptr, qp, st), "upload q_ptr");
  HIPCHK(upload(c->d_qcol, qc, st), "upload q_col");
  HIPCHK(upload(c->d_qval, qv, st), "upload q_val");
  HIPCHK(upload(c->d_alpha, al, st), "upload alpha");
  // sources: merged rows [N][Smax], zero columns past a mesh's own count
  c->solved = false;
  TRY(ensure_vec(c, c->d_fnew, sizeof(double) * (size_t)N * Smax, "alloc f"));
  HIPCHK(launch_fill_f64(st, c->d_fnew.as<double>(), N * Smax, 0.0), "zero f");
  int64_t fo = 0;
  for (int b = 0; b < B; ++b) {
    const tem_ctx *sb = c->sub[b];
    HIPCHK(launch_gather_rhs(st, sb->ed.N, S[b], Smax, sb->mt.n_edges,
                             sb->ed.d_row_ent.as<int32_t>(), F + fo,
                             c->d_fnew.as<double>() + c->row_off[b] * Smax),
           "gather f");
    fo += sb->mt.n_edges * S[b];
  }
  TRY(ensure_vec(c, c->d_g, sizeof(cpx<double>) * (size_t)MP * N * Smax, "alloc g"));
  hipEvent_t e0 = c->t_ev[0], e1 = c->t_ev[1];
  HIPCHK(hipEventRecord(e0, st), "event");
  IrResult res;
  tem_status s = refine_solve(c, c->d_fnew.as<double>(), nullptr, Smax, c->d_g.as<cpx<double>>(),
                              ir, res);
  hipEventRecord(e1, st);
  hipEventSynchronize(e1);
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  if (s != TEM_OK) return s;
  c->solve_ms = ms;
  spans_collect(c);
  c->last_solves = res.solves;
  c->S = Smax;
  c->K = K;
  c->S_mesh.assign(S, S + B);
  c->R_mesh.assign(R, R + B);
  c->q_row_off = qrow;
  int64_t dof = 0;
  for (int b = 0; b < B; ++b) {
    HIPCHK(launch_time_assembly(st, S[b], K, R[b], MP, N, Smax, c->d_qptr.as<int64_t>() + qrow[b],
                                c->d_qcol.as<int32_t>(), c->d_qval.as<double>(),
                                c->d_alpha.as<cpx<double>>() + (size_t)b * K * MP,
                                c->d_g.as<cpx<double>>(), d + dof),
           "time assembly");
    dof += (int64_t)S[b] * K * R[b];
  }
  HIPCHK(hipStreamSynchronize(st), "forward sync");
  fill_stats(res, stats);
  c->solved = true;
  c->surveyed = true;
  if (res.unconverged) {
    double worst = 0;
    for (double v : res.rel) worst = std::max(worst, v);
    char buf[160];
    std::snprintf(buf, sizeof(buf),
                  "tem_forward_batch: %d systems above rtol (worst %.3e) after %d solves",
                  res.unconverged, worst, res.solves);
    return fail(c, TEM_ENOCONV, buf);
  }
  return TEM_OK;
}

tem_status tem_set_params_batch(tem_ctx *c, const int32_t *n_params, const int32_t *param_cells) {
  if (!c) return TEM_EINVAL;
  if (c->B == 0) return fail(c, TEM_ESTATE, "tem_set_params_batch: no batch assembled");
  if (!n_params || !param_cells) return fail(c, TEM_EINVAL, "tem_set_params_batch: NULL argument");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  std::vector<int64_t> off(c->B + 1, 0);
  for (int b = 0; b < c->B; ++b) {
    const int64_t nc = c->sub[b]->mt.n_cells;
    if (n_params[b] < 0 || n_params[b] > nc)
      return fail(c, TEM_EINVAL, "tem_set_params_batch: parameter count out of range");
    std::vector<char> seen(nc, 0);
    for (int p = 0; p < n_params[b]; ++p) {
      const int32_t cell = param_cells[off[b] + p];
      if (cell < 0 || cell >= nc || seen[cell])
        return fail(c, TEM_EINVAL, "tem_set_params_batch: cell ids must be distinct and in range");
      seen[cell] = 1;
    }
    off[b + 1] = off[b] + n_params[b];
  }
  for (int b = 0; b < c->B; ++b) {
    tem_ctx *sb = c->sub[b];
    sb->params.assign(param_cells + off[b], param_cells + off[b + 1]);
    HIPCHK(upload(sb->d_params, sb->params, c->stream), "upload params");
  }
  c->param_off = off;
  return TEM_OK;
}

static tem_status batch_jac_check(tem_ctx *c, const char *who, const void *a, const void *b) {
  if (c->B == 0) return fail(c, TEM_ESTATE, std::string(who) + ": no batch assembled");
  if (!c->surveyed || !c->solved)
    return fail(c, TEM_ESTATE, std::string(who) + ": call tem_forward_batch first");
  if ((int)c->param_off.size() != c->B + 1 || c->param_off[c->B] == 0)
    return fail(c, TEM_ESTATE, std::string(who) + ": call tem_set_params_batch first");
  if (!a || !b) return fail(c, TEM_EINVAL, std::string(who) + ": NULL argument");
  return TEM_OK;
}

tem_status tem_jvp_batch(tem_ctx *c, const double *v, double *jv, const tem_ir_opts *ir,
                         tem_ir_stats *stats) {
  if (!c) return TEM_EINVAL;
  TRY(batch_jac_check(c, "tem_jvp_batch", v, jv));
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  hipStream_t st = c->stream;
  const int64_t N = N_of(c);
  const int MP = c->MP, Sm = c->S, B = c->B;
  const int64_t pst = N * Sm;
  int64_t ncell = 1;
  for (int b = 0; b < B; ++b) ncell = std::max<int64_t>(ncell, c->sub[b]->mt.n_cells);
  TRY(ensure_vec(c, c->v_vs, sizeof(double) * (size_t)ncell, "alloc vs"));
  TRY(ensure_vec(c, c->v_rhs, sizeof(cpx<double>) * (size_t)MP * N * Sm, "alloc rhs"));
  TRY(ensure_vec(c, c->v_lam, sizeof(cpx<double>) * (size_t)MP * N * Sm, "alloc sol"));
  cpx<double> *rhs = c->v_rhs.as<cpx<double>>(), *lam = c->v_lam.as<cpx<double>>();
  const cpx<double> *g = c->d_g.as<cpx<double>>();
  HIPCHK(launch_fill_f64(st, (double *)rhs, 2 * (int64_t)MP * N * Sm, 0.0), "zero rhs");
  for (int b = 0; b < B; ++b) {
    const tem_ctx *sb = c->sub[b];
    const int64_t r0 = c->row_off[b] * Sm;
    HIPCHK(launch_param_scatter(st, (int)sb->params.size(), sb->d_params.as<int32_t>(),
                                v + c->param_off[b], sb->d_sigma.as<double>(), sb->mt.n_cells,
                                c->v_vs.as<double>()),
           "param scatter");
    HIPCHK(launch_jv_rhs(st, sb->ed.N, c->np_mesh[b], c->S_mesh[b], Sm, pst, sb->mt.nx, sb->mt.ny,
                         sb->mt.nz, sb->ed.d_row_ent.as<int32_t>(), sb->d_cell_new.as<int32_t>(),
                         c->v_vs.as<double>(), sb->d_Me.as<double>(),
                         c->d_xi.as<double>() + 2 * (size_t)b * MP, g + r0, rhs + r0),
           "jv rhs");
  }
  IrResult res;
  TRY(refine_solve(c, nullptr, rhs, Sm, lam, ir, res));
  int64_t dof = 0;
  for (int b = 0; b < B; ++b) {
    HIPCHK(launch_time_assembly(st, c->S_mesh[b], c->K, c->R_mesh[b], MP, N, Sm,
                                c->d_qptr.as<int64_t>() + c->q_row_off[b], c->d_qcol.as<int32_t>(),
                                c->d_qval.as<double>(),
                                c->d_alpha.as<cpx<double>>() + (size_t)b * c->K * MP, lam,
                                jv + dof),
           "jv time assembly");
    dof += (int64_t)c->S_mesh[b] * c->K * c->R_mesh[b];
  }
  HIPCHK(hipStreamSynchronize(st), "jvp sync");
  spans_collect(c);
  fill_stats(res, stats);
  c->last_solves = res.solves;
  if (res.unconverged) return fail(c, TEM_ENOCONV, "tem_jvp_batch: refinement did not converge");
  return TEM_OK;
}

tem_status tem_vjp_batch(tem_ctx *c, const double *w, double *jtw, const tem_ir_opts *ir,
                         tem_ir_stats *stats) {
  if (!c) return TEM_EINVAL;
  TRY(batch_jac_check(c, "tem_vjp_batch", w, jtw));
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  hipStream_t st = c->stream;
  const int64_t N = N_of(c);
  const int MP = c->MP, Sm = c->S, B = c->B;
  const int64_t pst = N * Sm;
  TRY(ensure_vec(c, c->v_rhs, sizeof(cpx<double>) * (size_t)MP * N * Sm, "alloc rhs"));
  TRY(ensure_vec(c, c->v_lam, sizeof(cpx<double>) * (size_t)MP * N * Sm, "alloc sol"));
  cpx<double> *rhs = c->v_rhs.as<cpx<double>>(), *lam = c->v_lam.as<cpx<double>>();
  const cpx<double> *g = c->d_g.as<cpx<double>>();
  HIPCHK(launch_fill_f64(st, (double *)rhs, 2 * (int64_t)MP * N * Sm, 0.0), "zero rhs");
  int64_t dof = 0;
  for (int b = 0; b < B; ++b) {
    // receivers are in merged rows: the whole vector is the base
    HIPCHK(launch_jtw_rhs(st, c->S_mesh[b], Sm, pst, c->K, c->R_mesh[b], MP,
                          c->d_qptr.as<int64_t>() + c->q_row_off[b], c->d_qcol.as<int32_t>(),
                          c->d_qval.as<double>(),
                          c->d_alpha.as<cpx<double>>() + (size_t)b * c->K * MP, w + dof, rhs),
           "jtw rhs");
    dof += (int64_t)c->S_mesh[b] * c->K * c->R_mesh[b];
  }
  IrResult res;
  TRY(refine_solve(c, nullptr, rhs, Sm, lam, ir, res));
  for (int b = 0; b < B; ++b) {
    const tem_ctx *sb = c->sub[b];
    const int64_t r0 = c->row_off[b] * Sm;
    HIPCHK(launch_jtw_reduce(st, (int)sb->params.size(), c->np_mesh[b], c->S_mesh[b], Sm, pst,
                             sb->d_params.as<int32_t>(), sb->d_cell_new.as<int32_t>(),
                             sb->d_sigma.as<double>(), sb->d_Me.as<double>(),
                             c->d_xi.as<double>() + 2 * (size_t)b * MP, g + r0, lam + r0,
                             jtw + c->param_off[b]),
           "jtw reduce");
  }
  HIPCHK(hipStreamSynchronize(st), "vjp sync");
  spans_collect(c);
  fill_stats(res, stats);
  c->last_solves = res.solves;
  if (res.unconverged) return fail(c, TEM_ENOCONV, "tem_vjp_batch: refinement did not converge");
  return TEM_OK;
}

// ------------------------------------------------------------ autotuning
tem_status tem_autotune(tem_ctx *c, int32_t m, const double *xi, tem_precision prec,
                        tem_autotune_report *rep) {
  if (!c) return TEM_EINVAL;
  if (c->B > 0) return fail(c, TEM_ESTATE, "tem_autotune: not available on a batch of meshes");
  if (!c->analysed) return fail(c, TEM_ESTATE, "tem_autotune: call tem_analyse first");
  if (prec != TEM_FP64 && prec != TEM_FP32_IR)
    return fail(c, TEM_EINVAL, "tem_autotune: unknown precision");
  const int ip = prec == TEM_FP32_IR ? 1 : 0;
  std::vector<tem_ctx::UpdCfg> cand;
  if (ip == 1)
    cand = {{UPD_T64, true}, {UPD_T64, false}, {UPD_T128x64, true}, {UPD_T128x64, false}};
  else
    cand = {{UPD_T64, false}, {UPD_T64, true}};
  const int nl = (int)c->ed.levels.size();
  // t[q][L]: the smaller of two timings of level L under candidate q, taken
  // in two passes over the candidates, the second in reverse order, so that
  // neither the first factorisation of the process nor a drift of the clocks
  // during the runs decides a level.
  const double unset = std::numeric_limits<double>::infinity();
  std::vector<std::vector<double>> t(cand.size(), std::vector<double>(nl, unset));
  c->tuned[ip].clear();
  tem_status st = TEM_OK;
  const size_t nq = cand.size();
  for (size_t run = 0; run < 2 * nq && st == TEM_OK; ++run) {
    const size_t q = run < nq ? run : 2 * nq - 1 - run;
    c->forcing = true;
    c->forced = cand[q];
    c->lvl_timing = true;
    st = tem_factor_poles(c, m, xi, prec, nullptr);
    c->forcing = false;
    c->lvl_timing = false;
    if (st != TEM_OK) break;
    std::vector<double> lv(nl, 0.0);
    for (int grp = 0; grp < c->n_groups; ++grp)
      for (int L = 0; L < nl; ++L) {
        float ms = 0;
        const size_t e = ((size_t)grp * nl + L) * 2;
        if (hipEventElapsedTime(&ms, c->lvl_ev[e], c->lvl_ev[e + 1]) == hipSuccess) lv[L] += ms;
      }
    for (int L = 0; L < nl; ++L) t[q][L] = std::min(t[q][L], lv[L]);
  }
  if (st != TEM_OK) return st;
  std::vector<tem_ctx::UpdCfg> best(nl);
  double tuned = 0;
  for (int L = 0; L < nl; ++L) {
    size_t bq = 0;
    for (size_t q = 1; q < cand.size(); ++q)
      if (t[q][L] < t[bq][L]) bq = q;
    best[L] = cand[bq];
    tuned += t[bq][L];
  }
  c->tuned[ip] = best;
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->n_candidates = (int32_t)cand.size();
    for (size_t q = 0; q < cand.size() && q < 8; ++q) {
      double sum = 0;
      for (int L = 0; L < nl; ++L) sum += t[q][L];
      rep->candidate_ms[q] = sum;
      rep->candidate_tile[q] = cand[q].tile;
      rep->candidate_m3[q] = cand[q].m3 ? 1 : 0;
    }
    rep->tuned_ms = tuned;
    rep->n_levels = nl;
  }
  return TEM_OK;
}

tem_status tem_autotune_level(const tem_ctx *c, tem_precision prec, int32_t level, int32_t *tile,
                              int32_t *m3) {
  if (!c || !tile || !m3) return TEM_EINVAL;
  const std::vector<tem_ctx::UpdCfg> &tab = c->tuned[prec == TEM_FP32_IR ? 1 : 0];
  if (level < 0 || level >= (int)tab.size()) return TEM_ESTATE;
  *tile = tab[level].tile;
  *m3 = tab[level].m3 ? 1 : 0;
  return TEM_OK;
}

tem_status tem_get_stats(const tem_ctx *c, tem_stats *out) {
  if (!c || !out) return TEM_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->n_poles = c->npole;
  out->n_groups = c->n_groups;
  out->group_size = c->group_size;
  out->precision = (int32_t)c->prec;
  out->factor_bytes = (int64_t)c->d_factor.bytes;
  out->workspace_bytes = (int64_t)(c->w_x.bytes + c->ed.w_t.bytes + c->ed.w_w0.bytes + c->ed.w_w1.bytes +
                                   c->v_r.bytes + c->v_z.bytes + c->v_fblk.bytes + c->v_xblk.bytes +
                                   c->v_rhs.bytes + c->v_lam.bytes);
  out->n_tiny_pivots = c->n_tiny;
  out->last_solves = c->last_solves;
  out->factor_ms = c->factor_ms;
  out->solve_ms = c->solve_ms;
  out->update_ms = c->upd_ms;
  out->update_flops = c->upd_flops;
  out->update_launches = c->upd_launches;
  out->sweep_ms = c->sweep_ms;
  out->sweep_bytes = c->sweep_bytes;
  out->sweeps = c->sweeps;
  return TEM_OK;
}

}  // extern "C"
