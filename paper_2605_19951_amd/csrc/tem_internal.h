// Internal declarations shared by the HIP kernels and the host orchestration.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tem {

constexpr int NB = 32;          // panel (column block) width of the factors
constexpr int MAX_BLOCK_RHS = 16;  // right-hand sides per sweep (more are solved in blocks)

// Complex value stored as interleaved (re, im).
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

// -------------------------------------------------------------------------
// Front panel layout ("column-block trapezoid").  A front of n = k + u rows
// keeps its k eliminated columns in blocks of NB columns; block b holds
// columns [NB b, NB b + w_b) for rows [NB b, n) column-major with leading
// dimension n - NB b.  Element (r, c), r >= NB*(c/NB), lives at
// panel_elem(n, r, c).  Within each NB x NB diagonal block the strictly
// lower part holds L, the diagonal holds D, and the strictly upper part
// holds the transpose of the inverse of the unit-lower diagonal block.
// -------------------------------------------------------------------------
__host__ __device__ inline int64_t panel_block_off(int64_t n, int64_t b) {
  // sum over b' < b of NB * (n - NB b')
  return (int64_t)NB * (b * n - (int64_t)NB * (b * (b - 1) / 2));
}
__host__ __device__ inline int64_t panel_elem(int64_t n, int64_t r, int64_t c) {
  int64_t b = c / NB;
  int64_t r0 = NB * b;
  return panel_block_off(n, b) + (c - r0) * (n - r0) + (r - r0);
}
__host__ __device__ inline int64_t panel_size(int64_t n, int64_t k) {
  int64_t nb = (k + NB - 1) / NB;
  if (nb == 0) return 0;
  int64_t last_w = k - NB * (nb - 1);
  return panel_block_off(n, nb - 1) + last_w * (n - NB * (nb - 1));
}

// Device view of the supernodal structure (pole independent).
struct FrontTab {
  const int64_t *first;     // first column (new index)
  const int32_t *k;         // number of columns
  const int32_t *u;         // |U_s|
  const int64_t *rows_off;  // offset of U_s in rows / rel
  const int32_t *rows;      // U_s as new indices
  const int32_t *rel;       // position of each U_s row in the parent's front
  const int64_t *panel_off; // element offset of the panel in one pole's factor
  const int64_t *cb_off;    // element offset of the CB in one pole's level arena
  const int64_t *w_off;     // row offset of the solve update vector in one pole's level arena
  const int64_t *gmap_off;  // offset of the front's child gather maps
  const int32_t *gmap0;     // front position -> row of child 0's update (or -1)
  const int32_t *gmap1;     // front position -> row of child 1's update (or -1)
  const int32_t *child0;
  const int32_t *child1;
  // Ragged pole counts of a batch of meshes: pole slot p0 + z of a launch
  // (z = its pole index) exists for front s only if p0 + z < np[s].  np is
  // null when every front has every pole.
  const int32_t *np;
  int p0;
};

// Contiguous index segments, one per mesh of a batch (rows, matrix entries,
// ...): index i belongs to segment b with off[b] <= i < off[b+1].  Per-mesh
// tables (shifts, coefficients) are indexed [b * stride + pole].  A single
// mesh is n = 1 with off = null.
struct Seg {
  int n = 1;
  const int64_t *off = nullptr;
  int stride = 0;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return hipGetLastError().
// T is float (FP32 factors) or double (FP64 factors).

hipError_t launch_assemble_KM(hipStream_t st, int64_t N, const int64_t *rowptr, const int32_t *col,
                              const int32_t *row_edge, const int32_t *edge_new, int nx, int ny,
                              int nz, const double *Ke, const double *Me, const double *sigma,
                              double *Kv, double *Mv);

template <typename T>
hipError_t launch_fill_zero(hipStream_t st, cpx<T> *base, int64_t count, int npole,
                            int64_t pole_stride);

template <typename T>
hipError_t launch_front_assemble(hipStream_t st, int64_t n_entries, const int32_t *csr,
                                 const int64_t *pos, const double *Kv, const double *Mv,
                                 const double *xi, Seg entry_seg, int npole, cpx<T> *factor,
                                 int64_t pole_stride);

// cols: n_cols (parent front, child column) pairs of child `slot`
template <typename T>
hipError_t launch_extend_add(hipStream_t st, FrontTab ft, const int2 *cols, int64_t n_cols,
                             int slot, int npole, cpx<T> *factor, int64_t f_stride,
                             cpx<T> *cb_parent, cpx<T> *cb_child, int64_t cb_stride);

// Diagonal block and the rows below it of column block j0 / NB; jp = j0 - NB
// makes both first apply the update of the factored block jp, jp = -1 none.
template <typename T>
hipError_t launch_panel_diag(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                             int j0, int jp, int npole, cpx<T> *factor, int64_t f_stride,
                             int *flags);

template <typename T>
hipError_t launch_panel_trsm(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                             int j0, int jp, int max_rows, int npole, cpx<T> *factor,
                             int64_t f_stride);

// Output tile shapes of the front update (rows x columns): 64 x 64; 128 x 64
// and 128 x 128 (FP32 only; 128 x 128 with four real products only).
enum { UPD_T64 = 0, UPD_T128x64 = 1, UPD_T128 = 2 };
inline int upd_tile_rows(int tile) { return tile == UPD_T64 ? 64 : 128; }
inline int upd_tile_cols(int tile) { return tile == UPD_T128 ? 128 : 64; }

// mode 0: trailing update of panel columns [j0+dw, min(k, ccap)) by the
// eliminated columns [j0, j0+dw); mode 1: contribution block
// C = -L21 D L21^T.  tile: one of UPD_T*; max_tiles counted with the same
// shape (column tile t has ceil((n - cbeg) / rows) - floor(t / (rows /
// cols)) row tiles); m3: complex products with three real matrix-core
// products instead of four.
template <typename T>
hipError_t launch_front_update(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                               int mode, int j0, int dw, int ccap, int64_t max_tiles, int npole,
                               cpx<T> *factor, int64_t f_stride, cpx<T> *cb, int64_t cb_stride,
                               int tile, bool m3);

// ------------------------------------------------------------------ solves
// Vectors are [pole][N][S] complex T (S fastest), S <= 16.
// Triangle kernels work on the column range [cb, min(cb + BB, k)); BB >= k
// covers the whole front in one launch (one workgroup per front and pole).
// real_l: the factor's imaginary parts are zero (the register kernels then
// keep and apply its real parts only).
template <typename T>
hipError_t launch_fwd_tri(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                          int npole, int S, int64_t N, const cpx<T> *factor, int64_t f_stride,
                          cpx<T> *x, const cpx<T> *w_child, int64_t w_stride, int64_t cb,
                          int64_t BB, bool real_l = false);
// rows [cb+BB, k) -= L(rows, [cb, cb+BB)) y   (many workgroups per front);
// yin non-null: y is read from rows [cb, cb+BB) of yin and copied into x
template <typename T>
hipError_t launch_fwd_rows(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int max_rows, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, cpx<T> *x, int64_t cb, int64_t BB, bool real_l,
                           const cpx<T> *yin);
// x_j = y_j / d_j - t_j
template <typename T>
hipError_t launch_bwd_init(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int max_k, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, cpx<T> *x, const cpx<T> *t, int64_t t_stride);
// columns [0, cb) -= L([cb, cb+BB), cols)^T x  (many workgroups per front);
// xin non-null: the block's x rows are read from xin and copied into x
template <typename T>
hipError_t launch_bwd_cols(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int64_t cb, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, cpx<T> *x, int64_t BB, bool real_l,
                           const cpx<T> *xin);

// Explicit inverses of the unit-lower BB-column diagonal blocks of the
// fronts of a level (BB a multiple of NB, at most 256): block b of front s
// and its transpose at xoff[s] + 2 b BB^2 of each pole's x_stride-element
// region (column-major, leading dimension = the block's width).
template <typename T>
hipError_t launch_diag_inverse(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                               int max_k, int npole, const cpx<T> *factor, int64_t f_stride,
                               cpx<T> *xinv, int64_t x_stride, const int64_t *xoff, int BB);
// the children's update rows added to the top rows of every front of a level
template <typename T>
hipError_t launch_fwd_child_add(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                                int npole, int S, int64_t N, cpx<T> *x, const cpx<T> *w_child,
                                int64_t w_stride);
// out rows [cb, cb + w) = X_b x rows [cb, cb + w) (upper: X_b^T), b = cb / BB,
// for every front and pole of a level (out and x: [pole][N][S]; x_stride 0:
// one set of inverses for every pole slot; real_l: real inverses; S <= 16,
// FP64 S <= 8)
template <typename T>
hipError_t launch_blk_apply(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                            int npole, int S, int64_t N, const cpx<T> *xinv, int64_t x_stride,
                            const int64_t *xoff, int BB, int64_t cb, bool upper, bool real_l,
                            const cpx<T> *x, cpx<T> *out);

// real_l: the factor's imaginary parts are zero (FP64 only; skips the
// products with them)
template <typename T>
hipError_t launch_fwd_rect(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int max_u, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, const cpx<T> *x, const cpx<T> *w_child,
                           cpx<T> *w_out, int64_t w_stride, bool real_l = false);

template <typename T>
hipError_t launch_bwd_rect(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int max_k, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, const cpx<T> *x, cpx<T> *t, int64_t t_stride,
                           bool real_l = false);

template <typename T>
hipError_t launch_bwd_tri(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                          int npole, int S, int64_t N, const cpx<T> *factor, int64_t f_stride,
                          cpx<T> *x, const cpx<T> *t, int64_t t_stride, int64_t cb, int64_t BB,
                          int init, bool real_l = false);

// ------------------------------------------------------- vector kernels
// r = f for all poles p and rhs s (the residual of x = 0, FP64): f [N][S]
// real (new ordering) or, with f_cplx, [pole][N][S] complex; r [pole][N][S].
hipError_t launch_residual_init(hipStream_t st, int64_t N, int npole, int S,
                                const double *f_real, const cpx<double> *f_cplx, cpx<double> *r);

// Row blocks of the FP64 residual (launch_residual_blk): at most RB_ROWS
// rows per block (neighbours in space: the rows are taken in Morton order of
// their entities' positions) whose columns span at most RB_HALO distinct
// rows (the block's halo), with at most RB_ROWS * RB_NNZ entries in all (any
// row length up to that: rows of at most RB_NNZ entries keep a fixed stride
// in LDS, longer ones need the packed layout); right-hand sides are staged
// RB_SC at a time.
constexpr int RB_ROWS = 32, RB_HALO = 256, RB_NNZ = 33, RB_SC = 8;
// r = f - (K - xi_p M) x (x != NULL) by row blocks: block b holds the rows
// rb_rows[rb_row[b] .. rb_row[b+1]) and halo rows rb_h[rb_hoff[b] ..
// rb_hoff[b+1]); lcol[t] is the position of col[t] in its block's halo.
// Each row's sum runs over its entries in order.  S <= 16.
hipError_t launch_residual_blk(hipStream_t st, int64_t N, int npole, int S, int64_t nblk,
                               const int64_t *rb_row, const int32_t *rb_rows,
                               const int64_t *rb_hoff, const int32_t *rb_h, bool packed,
                               const int64_t *rowptr, const uint16_t *lcol, const double *Kv,
                               const double *Mv, const double *xi, Seg sg, const double *f_real,
                               const cpx<double> *f_cplx, const cpx<double> *x, cpx<double> *r);

// Batched complex dot products over N rows for all (pole, s):
// out[p*S+s] = sum_row conj(a) * b (conj_a) or sum a*b.  Deterministic.
// Pole p's rows start at a + p * pstride (pstride = N * S for whole
// vectors; a row range of a larger vector otherwise).
hipError_t launch_batched_dot(hipStream_t st, int64_t N, int npole, int S, int64_t pstride,
                              const cpx<double> *a, const cpx<double> *b, bool conj_a,
                              cpx<double> *partial, int n_partial_blocks, cpx<double> *out);

// y[p][i][s] += alpha[p*S+s] * x[p][i][s]  (complex alpha per system); mask
// (int per system, may be null) skips systems with mask == 0.
// sign multiplies alpha (use -1 for y -= alpha x)
// With row segments (a batch) the mask is per (segment, pole, s):
// mask[b * npole * S + p * S + s].
hipError_t launch_batched_axpy(hipStream_t st, int64_t N, int npole, int S,
                               const cpx<double> *alpha, double sign, const cpx<double> *x,
                               cpx<double> *y, const int *mask, Seg row_seg = Seg());
// inv[i] = 1/sqrt(Re dots[i]) (1 when zero), nrm[i] = sqrt(Re dots[i])
hipError_t launch_norm_scales(hipStream_t st, int n, const cpx<double> *dots, double *inv,
                              double *nrm);
hipError_t launch_fill_f64(hipStream_t st, double *p, int64_t n, double v);
// dst[row * ldd + d0 + j] = (j < cnt ? src[row * lds + s0 + j] : 0) for
// j < width: a block of columns of row-major arrays (in doubles; a complex
// column is two).  Gathers and scatters blocks of right-hand sides.
hipError_t launch_copy_cols(hipStream_t st, int64_t rows, const double *src, int lds, int s0,
                            int cnt, double *dst, int ldd, int d0, int width);

// conversions between the FP64 refinement vectors and the factor precision,
// with a per-system scale: out = in * scale[p*S+s].
template <typename T>
hipError_t launch_convert_in(hipStream_t st, int64_t n_per_pole, int npole, int S,
                             const cpx<double> *in, const double *scale, cpx<T> *out);
template <typename T>
hipError_t launch_convert_out(hipStream_t st, int64_t n_per_pole, int npole, int S,
                              const cpx<T> *in, const double *scale, cpx<double> *out);

// canonical-edge real array F (n_edges x S, column-major) -> new-ordering
// real rows f_new[q * ldS + s] (ldS >= S), q < N.
hipError_t launch_gather_rhs(hipStream_t st, int64_t N, int S, int ldS, int64_t n_edges,
                             const int32_t *row_edge, const double *F, double *f_new);

// g [pole][N][S] complex (new order) -> G [pole][S][n_edges] complex (canonical).
hipError_t launch_scatter_solution(hipStream_t st, int64_t N, int npole, int S, int64_t n_edges,
                                   const int32_t *edge_new, const cpx<double> *g,
                                   cpx<double> *G);

// Observation + residue time assembly:
// d[s][j][r] = 2 Re sum_i alpha[j][i] sum_q Qval * g[i][Qcol][s]
// g is [pole][N][ldS] (ldS >= S).
hipError_t launch_time_assembly(hipStream_t st, int S, int K, int R, int npole, int64_t N, int ldS,
                                const int64_t *q_ptr, const int32_t *q_col, const double *q_val,
                                const cpx<double> *alpha, const cpx<double> *g, double *d);

// Vectors of the Jacobian kernels are [pole][row][ldS] complex with pole
// stride pstride (elements); S <= ldS right-hand sides are used (a mesh of a
// batch: its rows and sources inside the merged vectors).
//
// Jv right-hand sides: rhs[p][e][s] = xi_p sum_{cells c of e} vs[c] (Me1 g_p|_c)[local]
// with vs[c] = v_param * sigma_c (0 for non-parameter cells); N rows.
hipError_t launch_jv_rhs(hipStream_t st, int64_t N, int npole, int S, int ldS, int64_t pstride,
                         int nx, int ny, int nz, const int32_t *row_edge, const int32_t *cell_new,
                         const double *vs, const double *Me, const double *xi,
                         const cpx<double> *g, cpx<double> *rhs);

// Tetrahedra: element matrices (entry-major Kt/Mt [36][nt], unit
// conductivity mass, edge signs applied; Lt [16][nt] the unit nodal blocks
// |T| g_i . g_j), the entry-owner gather of a pattern from element entries
// src = t * ne + ab (M only unless with_k), and the Jacobian pieces as above with the
// per-tetrahedron masses (et_ptr/et_src: tetrahedra t * 6 + local index of
// each row; tet_new: 6 new indices per tetrahedron, -1 on the boundary).
hipError_t launch_tet_elements(hipStream_t st, int64_t nt, const double *xyz, const int32_t *tets,
                               const int8_t *sgn, double mu, double *Kt, double *Mt, double *Lt);
hipError_t launch_tet_gather(hipStream_t st, int64_t nnz, const int64_t *ent_ptr,
                             const int32_t *ent_src, int ne, int64_t nt, const double *Kt,
                             const double *Mt, const double *sigma, bool with_k, double *Kv,
                             double *Mv);
hipError_t launch_jv_rhs_tet(hipStream_t st, int64_t N, int npole, int S, int ldS, int64_t pstride,
                             const int64_t *et_ptr, const int32_t *et_src, const int32_t *tet_new,
                             int64_t nt, const double *vs, const double *Mt, const double *xi,
                             const cpx<double> *g, cpx<double> *rhs);
hipError_t launch_jtw_reduce_tet(hipStream_t st, int P, int npole, int S, int ldS, int64_t pstride,
                                 const int32_t *params, const int32_t *tet_new, int64_t nt,
                                 const double *sigma, const double *Mt, const double *xi,
                                 const cpx<double> *g, const cpx<double> *lam, double *out);

// sigma[params[p]] = exp(m[p])
hipError_t launch_set_sigma_exp(hipStream_t st, int P, const int32_t *params, const double *m,
                                double *sigma);

hipError_t launch_param_scatter(hipStream_t st, int P, const int32_t *params, const double *v,
                                const double *sigma, int64_t n_cells, double *vs);

// J^T w right-hand sides: rhs[p][e][s] += sum_r Q[r][e] sum_j alpha[j][p] w[s][j][r]
// (rhs zeroed by the caller; alpha is [K][npole])
hipError_t launch_jtw_rhs(hipStream_t st, int S, int ldS, int64_t pstride, int K, int R,
                          int npole, const int64_t *q_ptr, const int32_t *q_col,
                          const double *q_val, const cpx<double> *alpha, const double *w,
                          cpx<double> *rhs);

// (J^T w)_p = 2 Re sum_{i,s} xi_i sigma_c g_is|_c^T Me1 lam_is|_c, c = params[p]
hipError_t launch_jtw_reduce(hipStream_t st, int P, int npole, int S, int ldS, int64_t pstride,
                             const int32_t *params, const int32_t *cell_new, const double *sigma,
                             const double *Me, const double *xi, const cpx<double> *g,
                             const cpx<double> *lam, double *out);

// ----------------------------------------------------- LSQR helpers (FP64)
// v -= V^T (V v): one classical Gram-Schmidt pass of v (n entries) against
// the nv rows of V (row-major, row j at V + j * n); partial: nv * 64
// doubles, h: nv doubles (work space).  Deterministic.
hipError_t launch_reorth(hipStream_t st, int64_t n, int nv, const double *V, double *v,
                         double *partial, double *h);
hipError_t launch_rdot(hipStream_t st, int64_t n, const double *a, const double *b,
                       double *partial /* 256 */, double *out);
hipError_t launch_raxpby(hipStream_t st, int64_t n, double a, const double *x, const double *w,
                         double b, double *y);
// regulariser rows sc w_r (m[hi] - m[lo]) and their transpose (w NULL: 1)
hipError_t launch_reg(hipStream_t st, int64_t nr, const int32_t *lo, const int32_t *hi,
                      const double *w, double sc, const double *m, double a, double *out);
hipError_t launch_regT(hipStream_t st, int P, const int64_t *inc_ptr, const int32_t *inc_row,
                       const double *w, double sc, const double *u, double a, double *out);

// ------------------------------------------------ nodal gradient space
// G^T M G on interior nodes (row-owner gather over the <= 8 cells of a node)
hipError_t launch_assemble_nodal(hipStream_t st, int64_t Nn, const int64_t *rowptr,
                                 const int32_t *col, const int32_t *row_node,
                                 const int32_t *node_new, int nx, int ny, int nz, const double *Le,
                                 const double *sigma, double *Lv);
// out = G^T r  (edge vectors [pole][N][S] -> packed nodal vectors: system
// j = p * S + s in column j % S2 of virtual pole j / S2, [vp][Nn][S2],
// zero past npole * S).  node_ptr NULL: six edges per node in the
// hexahedral order (signs +, -, +, -, +, -); else the node's edges are the
// signed edge+1 entries node_edges[node_ptr[n] .. node_ptr[n+1]) (+ where
// the node ends the edge).
hipError_t launch_grad_T(hipStream_t st, int64_t Nn, int npole, int S, int S2, int64_t N,
                         const int64_t *node_ptr, const int32_t *node_edges, const cpx<double> *r,
                         cpx<double> *out);
// z += coef[pole] * G y
// z += coef * G y with y packed as for launch_grad_T; coef indexed
// [segment of the edge row * row_seg.stride + pole]
hipError_t launch_grad_add(hipStream_t st, int64_t N, int npole, int S, int S2, int64_t Nn,
                           const int32_t *edge_nodes, const cpx<double> *coef, Seg row_seg,
                           const cpx<double> *y, cpx<double> *z);

}  // namespace tem
