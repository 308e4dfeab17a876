// Batched supernodal triangular solves with the cached factors, all poles
// and all right-hand sides of one tree level per launch.
//   forward:  per front, top rows  y_s = L11^{-1} (b_s + child updates)
//             update rows          W_s = (child updates) - L21 y_s
//   backward: per front            t_s = L21^T x(U_s)
//                                  x_s = L11^{-T} (D^{-1} y_s - t_s)
// Vectors are [pole][N][S] complex, S <= 16, in the nested-dissection
// ordering; W arenas hold each front's update rows [row][S].
#include "k_common.h"

namespace tem {

// rows per LDS tile of the backward rectangle kernel (32: 64 registers,
// eight waves per SIMD; 64 rows took 92, five)
constexpr int RT = 32;
constexpr int RTT = 32;  // rows per LDS tile (triangle kernels, keeps LDS under 64 KiB)

// Pointer to column c's data such that element (r, c) is colptr[r].
template <typename T>
__device__ __forceinline__ const cpx<T> *col_ptr(const cpx<T> *P, int64_t n, int64_t c,
                                                 int64_t &ld) {
  const int64_t b = c / NB, r0 = NB * b;
  ld = n - r0;
  return P + panel_block_off(n, b) + (c - r0) * ld - r0;
}

// Stages rows r0 .. r0+nr-1 of columns 0 .. w-1 of a column block (column
// l at Lc + l * ld) into Lt[l][i], zero past nr rows and w columns.  The
// loads go to clamped in-bounds positions and are all issued before any is
// used (256 threads).
template <typename T, int RTS>
__device__ __forceinline__ void stage_tile(cpx<T> (*Lt)[RTS + 1], const cpx<T> *Lc, int64_t ld,
                                           int64_t r0, int nr, int w, int tid) {
  constexpr int PERT = RTS * NB / 256;
  cpx<T> v[PERT];
#pragma unroll
  for (int q = 0; q < PERT; ++q) {
    const int idx = tid + 256 * q, i = idx % RTS, l = idx / RTS;
    v[q] = Lc[(int64_t)min(l, w - 1) * ld + r0 + min(i, nr - 1)];
  }
#pragma unroll
  for (int q = 0; q < PERT; ++q) {
    const int idx = tid + 256 * q, i = idx % RTS, l = idx / RTS;
    Lt[l][i] = (i < nr && l < w) ? v[q] : czero<T>();
  }
}

// Adds the children's update rows into the top rows X of front s (pole p):
// four elements per thread in flight, maps, then child rows, then sums.
template <typename T>
__device__ inline void fwd_child_add(const FrontTab &ft, int s, int p, int64_t k, int S,
                                     cpx<T> *X, const cpx<T> *w_child, int64_t w_stride,
                                     int tid) {
  const int32_t *gm0 = ft.gmap0 + ft.gmap_off[s];
  const int32_t *gm1 = ft.gmap1 + ft.gmap_off[s];
  const int c0 = ft.child0[s], c1 = ft.child1[s];
  const cpx<T> *W0 = c0 >= 0 ? w_child + (int64_t)p * w_stride + ft.w_off[c0] * S : nullptr;
  const cpx<T> *W1 = c1 >= 0 ? w_child + (int64_t)p * w_stride + ft.w_off[c1] * S : nullptr;
  const bool h0 = c0 >= 0 && ft.u[c0] > 0, h1 = c1 >= 0 && ft.u[c1] > 0;
  if (h0 || h1) {
    // four elements per thread in flight: maps, then child rows, then sums
    const int64_t tot = k * S;
    for (int64_t base = tid; base < tot; base += 4 * 256) {
      int g0[4], g1[4];
      cpx<T> xv[4], v0[4], v1[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t id = min(base + 256 * j, tot - 1), q = id / S;
        g0[j] = h0 ? gm0[q] : -1;
        g1[j] = h1 ? gm1[q] : -1;
        xv[j] = X[id];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t id = min(base + 256 * j, tot - 1), c = id % S;
        v0[j] = h0 ? W0[(int64_t)max(g0[j], 0) * S + c] : czero<T>();
        v1[j] = h1 ? W1[(int64_t)max(g1[j], 0) * S + c] : czero<T>();
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t id = base + 256 * j;
        if (id >= tot) continue;
        cpx<T> v = xv[j];
        if (g0[j] >= 0) v = cadd(v, v0[j]);
        if (g1[j] >= 0) v = cadd(v, v1[j]);
        X[id] = v;
      }
    }
  }
}

// ------------------------------------------------------------ forward tri
// Solves the diagonal blocks of columns [cb, ce), ce = min(cb + BB, k), and
// updates only the rows inside that range; cb == 0 first adds the children's
// update rows to all top rows.
template <typename T>
__global__ __launch_bounds__(256) void k_fwd_tri(FrontTab ft, const int32_t *lvl_nodes, int S,
                                                 int64_t N, const cpx<T> *factor,
                                                 int64_t f_stride, cpx<T> *x,
                                                 const cpx<T> *w_child, int64_t w_stride,
                                                 int64_t cb, int64_t BB) {
  const int s = lvl_nodes[blockIdx.x];
  const int p = blockIdx.y;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], n = k + ft.u[s], first = ft.first[s];
  if (k == 0 || cb >= k) return;
  const int64_t ce = min(k, cb + BB);
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];
  cpx<T> *X = x + ((int64_t)p * N + first) * S;     // rows of this front's columns
  const int tid = threadIdx.x;
  if (cb == 0) fwd_child_add<T>(ft, s, p, k, S, X, w_child, w_stride, tid);
  __shared__ cpx<T> Li[NB][NB + 1];   // Li[j][l]: inverse of the unit-lower diagonal block
  __shared__ cpx<T> V[NB][16];
  __shared__ cpx<T> Y[NB][16];
  __shared__ cpx<T> Lt[NB][RTT + 1];   // Lt[l][i] = L(r0 + i, jb + l)
  for (int64_t jb = cb; jb < ce; jb += NB) {
    const int w = (int)min((int64_t)NB, k - jb);
    int64_t ld;
    const cpx<T> *Lc = col_ptr(P, n, jb, ld);   // column jb; column jb+l at Lc + l*ld
    __syncthreads();
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int j = idx % w, l = idx / w;
      // stored transposed in the upper part: Linv[j][l] at (row jb+l, col jb+j)
      // (entries l >= j are read but not used)
      Li[j][l] = Lc[(int64_t)j * ld + jb + l];
    }
    for (int idx = tid; idx < w * S; idx += blockDim.x) V[idx / S][idx % S] = X[(jb) * S + idx];
    __syncthreads();
    for (int idx = tid; idx < w * S; idx += blockDim.x) {
      const int j = idx / S, c = idx % S;
      cpx<T> acc = V[j][c];
      for (int l = 0; l < j; ++l) acc = cfma(Li[j][l], V[l][c], acc);
      Y[j][c] = acc;
      X[jb * S + idx] = acc;
    }
    __syncthreads();
    // rows below inside the range: X[r] -= sum_l L(r, jb+l) Y[l]
    for (int64_t rc = jb + w; rc < ce; rc += RTT) {
      const int nr = (int)min((int64_t)RTT, ce - rc);
      stage_tile<T, RTT>(Lt, Lc, ld, rc, nr, w, tid);
      __syncthreads();
      for (int idx = tid; idx < nr * S; idx += blockDim.x) {
        const int i = idx / S, c = idx % S;
        cpx<T> acc = czero<T>();
        for (int l = 0; l < w; ++l) acc = cfma(Lt[l][i], Y[l][c], acc);
        cpx<T> *q = X + (rc + i) * S + c;
        *q = csub(*q, acc);
      }
      __syncthreads();
    }
  }
}

// Forward triangle for ranges of at most 256 rows.  Thread i owns row
// cb + i of the range and keeps its right-hand sides in registers for the
// whole range, together with its row of the current 32-column block, loaded
// one block ahead (as is the inverse diagonal block).  Per block: the owners
// of the block's rows publish them (V), Y = V + Lo V is formed, Lo the
// strictly lower part of the stored inverse of the unit-lower diagonal
// block, and every later row of the range subtracts its L row times Y.  SP
// (8 or 16) columns are computed for S <= SP right-hand sides, with zero
// factors in place of branches; barriers order LDS only.
template <typename T, int SP, bool RL>
__global__ __launch_bounds__(256) void k_fwd_tri_reg(FrontTab ft, const int32_t *lvl_nodes,
                                                     int S, int64_t N, const cpx<T> *factor,
                                                     int64_t f_stride, cpx<T> *x,
                                                     const cpx<T> *w_child, int64_t w_stride,
                                                     int64_t cb, int64_t BB) {
  constexpr int NT = NB * SP / 256;   // (row, column) tasks per thread in the block solve
  typedef FacVal<T, RL> FV;           // RL: real factor, kept and applied as real
  const int s = lvl_nodes[blockIdx.x];
  const int p = blockIdx.y;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], n = k + ft.u[s], first = ft.first[s];
  if (k == 0 || cb >= k) return;
  const int64_t ce = min(k, cb + BB);
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];
  cpx<T> *X = x + ((int64_t)p * N + first) * S;
  const int tid = threadIdx.x;
  if (cb == 0) fwd_child_add<T>(ft, s, p, k, S, X, w_child, w_stride, tid);
  __syncthreads();
  const int nr = (int)(ce - cb);   // <= 256 (checked by the launcher)
  const bool own = tid < nr;
  const int64_t r = cb + min(tid, nr - 1);
  cpx<T> xr[SP];
#pragma unroll
  for (int c = 0; c < SP; ++c) xr[c] = X[r * S + min(c, S - 1)];
  __shared__ typename FV::type Lo[NB][NB + 1];
  __shared__ cpx<T> V[NB][SP];
  __shared__ cpx<T> Y[NB][SP];
  typename FV::type lv[NB], li[NB * NB / 256];
  // inverse block of columns [jb, jb + NB): Linv[j][l] at (row jb + l,
  // column jb + j); clamped to the last block (entries past w are zeroed)
  auto fetch_li = [&](int64_t jb) {
    jb = min(jb, NB * ((k - 1) / NB));
    const int w = (int)min((int64_t)NB, k - jb);
    int64_t ld;
    const cpx<T> *Lc = col_ptr(P, n, jb, ld);
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
      const int idx = tid + 256 * q, j = idx % NB, l = idx / NB;
      li[q] = FV::of(Lc[(int64_t)min(j, w - 1) * ld + jb + min(l, w - 1)]);
    }
  };
  // the owned row's entries in columns [jb, jb + NB) (rows above the block
  // are clamped to its first row: they are not stored with it)
  auto fetch_lv = [&](int64_t jb) {
    jb = min(jb, NB * ((k - 1) / NB));
    const int w = (int)min((int64_t)NB, k - jb);
    int64_t ld;
    const cpx<T> *Lc = col_ptr(P, n, jb, ld);
    const int64_t rr = max(r, jb);
#pragma unroll
    for (int l = 0; l < NB; ++l) lv[l] = FV::of(Lc[(int64_t)min(l, w - 1) * ld + rr]);
  };
  fetch_li(cb);
  fetch_lv(cb);
  for (int64_t jb = cb; jb < ce; jb += NB) {
    const int w = (int)min((int64_t)NB, k - jb);
    lds_barrier();   // the previous block's readers of Lo, V and Y are done
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
      const int idx = tid + 256 * q, j = idx % NB, l = idx / NB;
      Lo[j][l] = (l < j && j < w) ? li[q] : FV::of(czero<T>());
    }
    fetch_li(jb + NB);
    if (own && r >= jb && r < jb + w) {
#pragma unroll
      for (int c = 0; c < SP; ++c) V[r - jb][c] = xr[c];
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) {   // rows past w of the block: zero
      const int idx = tid + 256 * q, j = idx / SP;
      if (j >= w) V[j][idx % SP] = czero<T>();
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int idx = tid + 256 * q, j = idx / SP, c = idx % SP;
      cpx<T> acc = V[j][c];
#pragma unroll
      for (int l = 0; l < NB; ++l) acc = FV::fma_(Lo[j][l], V[l][c], acc);
      Y[j][c] = acc;
      if (j < w && c < S) X[(jb + j) * S + c] = acc;
    }
    lds_barrier();
    if (own && r >= jb + w) {
#pragma unroll
      for (int l = 0; l < NB; ++l) {
        const typename FV::type a = l < w ? FV::neg(lv[l]) : FV::of(czero<T>());
#pragma unroll
        for (int c = 0; c < SP; ++c) xr[c] = FV::fma_(a, Y[l][c], xr[c]);
      }
    }
    fetch_lv(jb + NB);
  }
}

template <typename T>
hipError_t launch_fwd_tri(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                          int npole, int S, int64_t N, const cpx<T> *factor, int64_t f_stride,
                          cpx<T> *x, const cpx<T> *w_child, int64_t w_stride, int64_t cb,
                          int64_t BB, bool real_l) {
  if (n_nodes <= 0) return hipSuccess;
  // the column blocks of wide fronts (at most 256 rows, one per thread)
  // take the register kernel; whole small fronts, many per level, keep the
  // lighter LDS kernel
  if (S >= 1 && S <= 16 && BB <= 256 && BB % NB == 0 && cb % NB == 0)
    hipLaunchKernelGGL((real_l ? (S <= 8 ? k_fwd_tri_reg<T, 8, true> : k_fwd_tri_reg<T, 16, true>)
                               : (S <= 8 ? k_fwd_tri_reg<T, 8, false>
                                         : k_fwd_tri_reg<T, 16, false>)),
                       dim3(n_nodes, npole), dim3(256), 0, st, ft, lvl_nodes, S, N, factor,
                       f_stride, x, w_child, w_stride, cb, BB);
  else
    hipLaunchKernelGGL(k_fwd_tri<T>, dim3(n_nodes, npole), dim3(256), 0, st, ft, lvl_nodes, S, N,
                       factor, f_stride, x, w_child, w_stride, cb, BB);
  return hipGetLastError();
}

// ------------------------------------------------------------ forward rect
// W_s[a] = child updates at front row k+a  -  sum_j L(k+a, j) y_j
// Forward rect on the matrix cores: per front the update rows are
// W = (children's rows) - L21 Y, a product with few columns (the right-hand
// sides).  A 16 x 16 x 4 MFMA (f32 or f64) multiplies 16 rows of L21 by four
// columns at a time; its 16 output columns hold Re y and Im y of eight
// right-hand sides, so Lr B and Li B (B = [Re Y | Im Y]) give all four real
// products of the complex one: Re(L y) = Lr Re y - Li Im y, Im(L y) =
// Lr Im y + Li Re y.  Operand lane l carries row (or output column) l % 16
// and depth l / 16.  Each wave owns 32 rows and walks all k columns on its
// own (no LDS, no barriers), a chunk of 16 columns at a time
// (FP32 and FP64), loading the next chunk while the current one is multiplied.
// NBK = 1 for S <= 8 right-hand sides, 2 for S <= 16.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
// 16 x 16 x 4 products: FP32 result element i of lane l is row 4 (l / 16) + i,
// FP64 row l / 16 + 4 i (column l % 16 for both); operands as above
template <typename T>
struct Mfma16;
template <>
struct Mfma16<float> {
  using acc_t = floatx4;
  // columns per chunk: 16 keeps two chunks of operands in 75 registers (six
  // waves per SIMD; 32 columns needed 112, four waves)
  static constexpr int KC = 16;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int ld4, int i) { return 4 * ld4 + i; }
};
template <>
struct Mfma16<double> {
  using acc_t = doublex4;
  static constexpr int KC = 16;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int ld4, int i) { return ld4 + 4 * i; }
};
// ROWS = true is the same product for the pivot rows below a block of
// columns of a wide front: X[r] -= sum_{j in [cb, ce)} L(r, j) y_j for rows r
// in [ce, k), ce = min(k, cb + BB), in place.  RL = true: the factor is
// real (its imaginary parts are zero), so the Li products are skipped.
// yin (ROWS only, may be null): y of the block's columns is read from yin
// ([pole][N][S] like x) instead of x, and the workgroups copy those rows of
// yin into x (the explicit-inverse schedule leaves the block's solution
// there; no workgroup of the launch reads x in those rows).
template <typename T, int NBK, bool ROWS, bool RL = false>
__global__ __launch_bounds__(256) void k_fwd_rect_mfma(FrontTab ft, const int32_t *lvl_nodes,
                                                       int S, int64_t N, const cpx<T> *factor,
                                                       int64_t f_stride, cpx<T> *x,
                                                       const cpx<T> *w_child,
                                                       cpx<T> *w_out, int64_t w_stride,
                                                       int64_t cb, int64_t BB, int pf,
                                                       const cpx<T> *yin) {
  using MF = Mfma16<T>;
  using acc_t = typename MF::acc_t;
  constexpr int RB = 2, KC = MF::KC;   // 16-row blocks per wave, columns per chunk
  const int s = lvl_nodes[blockIdx.y];
  // pf > 1: the pole is the fastest part of blockIdx.x (the workgroups of all
  // poles for the same rows run together; a factor shared by all poles is
  // then read once from HBM)
  const int p = pf > 1 ? (int)(blockIdx.x % pf) : (int)blockIdx.z;
  const int64_t bx = pf > 1 ? (int64_t)(blockIdx.x / pf) : (int64_t)blockIdx.x;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], u = ft.u[s], n = k + u, first = ft.first[s];
  // output rows row0 + [0, nrows), depth columns [d0, d1)
  int64_t row0 = k, nrows = u, d0 = 0, d1 = k;
  cpx<T> *X = x + ((int64_t)p * N + first) * S;
  const cpx<T> *Y = X;   // where y of the depth columns is read
  if (ROWS) {
    if (cb >= k) return;
    d0 = cb;
    d1 = min(k, cb + BB);
    row0 = d1;
    nrows = k - d1;
    if (yin) {
      Y = yin + ((int64_t)p * N + first) * S;
      // block rows [d0 + 128 bx, +128) of yin -> x
      const int64_t c0 = d0 + bx * 128, c1 = min(d1, c0 + 128);
      for (int64_t idx = c0 * S + threadIdx.x; idx < c1 * S; idx += 256) X[idx] = Y[idx];
    }
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t aw = bx * 128 + wave * 32;   // first row of the wave
  if (aw >= nrows) return;
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];
  const int lr = lane & 15, ld4 = lane >> 4;   // operand row / output column, depth
  // rows of the two blocks (clamped; rows past u reach no output)
  int32_t rrow[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) rrow[b] = (int32_t)(row0 + min(aw + b * 16 + lr, nrows - 1));
  // B operand: column lr of block nb is Re y_j (lr < 8) or Im y_j, j = 8 nb + lr % 8
  int yj[NBK];
  bool yon[NBK];
#pragma unroll
  for (int nb = 0; nb < NBK; ++nb) {
    const int j = 8 * nb + (lr & 7);
    yon[nb] = j < S;
    yj[nb] = 2 * min(j, S - 1) + (lr >> 3);   // float index inside a row of X
  }
  acc_t r1[RB][NBK], r2[RB][NBK];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int nb = 0; nb < NBK; ++nb) {
      r1[b][nb] = acc_t{0, 0, 0, 0};
      r2[b][nb] = acc_t{0, 0, 0, 0};
    }
  const T *Xf = reinterpret_cast<const T *>(Y);
  // chunk jb into (lv, yv): unconditional loads from clamped addresses (a
  // chunk past the end re-reads the last one and gets y = 0)
  const int64_t jlast = d0 + ((d1 - 1 - d0) / KC) * KC;
  auto load = [&](int64_t jb, cpx<T> (&lv)[KC / 4][RB], T (&yv)[KC / 4][NBK]) {
    const int64_t je = min(jb, jlast);
    int64_t ld;
    const cpx<T> *Lc = col_ptr(P, n, je, ld);   // the chunk lies in one column block
    const T *Xc = Xf + je * 2 * S;
    // 32-bit offsets inside the chunk: column offset <= 31, ld and 2 S below 2^24
    const int32_t lim = (int32_t)(d1 - 1 - je), ldi = (int32_t)ld, colk = (int32_t)(d1 - jb);
#pragma unroll
    for (int q = 0; q < KC / 4; ++q) {
      const int32_t t = 4 * q + ld4, o = min(t, lim);
      const int32_t lo = (int32_t)__umul24((uint32_t)o, (uint32_t)ldi);
#pragma unroll
      for (int b = 0; b < RB; ++b) lv[q][b] = Lc[lo + rrow[b]];
      const int32_t yo = (int32_t)__umul24((uint32_t)o, (uint32_t)(2 * S));
#pragma unroll
      for (int nb = 0; nb < NBK; ++nb)   // a multiply, not a select: the load stays unconditional
        yv[q][nb] = Xc[yo + yj[nb]] * ((t < colk && yon[nb]) ? T(1) : T(0));
    }
  };
  auto mma = [&](const cpx<T> (&lv)[KC / 4][RB], const T (&yv)[KC / 4][NBK]) {
#pragma unroll
    for (int q = 0; q < KC / 4; ++q)
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int nb = 0; nb < NBK; ++nb) {
          r1[b][nb] = MF::mma(lv[q][b].re, yv[q][nb], r1[b][nb]);
          if constexpr (!RL) r2[b][nb] = MF::mma(lv[q][b].im, yv[q][nb], r2[b][nb]);
        }
  };
  // two register sets: the loads of the next chunk are in flight while the
  // current one is multiplied
  cpx<T> la[KC / 4][RB], lb[KC / 4][RB];
  T ya[KC / 4][NBK], yb[KC / 4][NBK];
  load(d0, la, ya);
  for (int64_t jb = d0; jb < d1; jb += 2 * KC) {
    load(jb + KC, lb, yb);
    mma(la, ya);
    if (jb + KC >= d1) break;
    load(jb + 2 * KC, la, ya);
    mma(lb, yb);
  }
  // lanes with lr < 8 hold column j's Lr Re y and Li Re y; lane l ^ 8 holds
  // Lr Im y and Li Im y of the same j
  const int c0 = ft.child0[s], c1 = ft.child1[s];
  const bool h0 = c0 >= 0 && ft.u[c0] > 0, h1 = c1 >= 0 && ft.u[c1] > 0;
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int nb = 0; nb < NBK; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T o1 = __shfl_xor(r1[b][nb][i], 8), o2 = __shfl_xor(r2[b][nb][i], 8);
        const int64_t a = aw + b * 16 + MF::row(ld4, i);
        const int j = 8 * nb + lr;
        if (lr >= 8 || j >= S || a >= nrows) continue;
        cpx<T> v = {-(r1[b][nb][i] - o2), -(o1 + r2[b][nb][i])};
        if (ROWS) {
          cpx<T> *o = X + (row0 + a) * S + j;
          *o = cadd(*o, v);
          continue;
        }
        if (h0) {
          const int g = ft.gmap0[ft.gmap_off[s] + k + a];
          if (g >= 0) v = cadd(v, w_child[(int64_t)p * w_stride + (ft.w_off[c0] + g) * S + j]);
        }
        if (h1) {
          const int g = ft.gmap1[ft.gmap_off[s] + k + a];
          if (g >= 0) v = cadd(v, w_child[(int64_t)p * w_stride + (ft.w_off[c1] + g) * S + j]);
        }
        w_out[(int64_t)p * w_stride + (ft.w_off[s] + a) * S + j] = v;
      }
}

// launches the forward MFMA kernel for S right-hand sides (NBK from S; the
// real-factor variant only exists in FP64)
template <typename T, bool ROWS>
hipError_t fwd_mfma_go(hipStream_t st, dim3 grid, FrontTab ft, const int32_t *lvl_nodes, int S,
                       int64_t N, const cpx<T> *factor, int64_t f_stride, cpx<T> *x,
                       const cpx<T> *w_child, cpx<T> *w_out, int64_t w_stride, int64_t cb,
                       int64_t BB, bool real_l, const cpx<T> *yin = nullptr) {
  if (S < 1 || S > 16) return hipErrorInvalidValue;
  const bool two = S > 8;
  // the poles go into the fastest grid dimension, so that the workgroups of
  // all poles for the same rows run together
  const int pf = (int)grid.z;
  if (pf > 1) {
    grid.x *= pf;
    grid.z = 1;
  }
  if constexpr (sizeof(T) == 8) {
    if (real_l) {
      if (two)
        hipLaunchKernelGGL((k_fwd_rect_mfma<T, 2, ROWS, true>), grid, dim3(256), 0, st, ft,
                           lvl_nodes, S, N, factor, f_stride, x, w_child, w_out, w_stride, cb, BB,
                           pf, yin);
      else
        hipLaunchKernelGGL((k_fwd_rect_mfma<T, 1, ROWS, true>), grid, dim3(256), 0, st, ft,
                           lvl_nodes, S, N, factor, f_stride, x, w_child, w_out, w_stride, cb, BB,
                           pf, yin);
      return hipGetLastError();
    }
  }
  if (two)
    hipLaunchKernelGGL((k_fwd_rect_mfma<T, 2, ROWS>), grid, dim3(256), 0, st, ft, lvl_nodes, S, N,
                       factor, f_stride, x, w_child, w_out, w_stride, cb, BB, pf, yin);
  else
    hipLaunchKernelGGL((k_fwd_rect_mfma<T, 1, ROWS>), grid, dim3(256), 0, st, ft, lvl_nodes, S, N,
                       factor, f_stride, x, w_child, w_out, w_stride, cb, BB, pf, yin);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fwd_rect(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int max_u, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, const cpx<T> *x, const cpx<T> *w_child,
                           cpx<T> *w_out, int64_t w_stride, bool real_l) {
  if (n_nodes <= 0 || max_u <= 0) return hipSuccess;
  dim3 grid((max_u + 127) / 128, n_nodes, npole);
  cpx<T> *xm = const_cast<cpx<T> *>(x);   // read only in this mode
  return fwd_mfma_go<T, false>(st, grid, ft, lvl_nodes, S, N, factor, f_stride, xm, w_child,
                               w_out, w_stride, 0, 0, real_l);
}

// rows [ce, k) of each wide front -= L(rows, [cb, ce)) y, ce = min(k, cb + BB);
// yin: y in rows [cb, ce) of yin, copied into x by the same launch
template <typename T>
hipError_t launch_fwd_rows(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int max_rows, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, cpx<T> *x, int64_t cb, int64_t BB, bool real_l,
                           const cpx<T> *yin) {
  if (n_nodes <= 0) return hipSuccess;
  int64_t nbx = (max_rows + 127) / 128;
  if (yin) nbx = std::max<int64_t>(nbx, (BB + 127) / 128);   // the copy of the block rows
  if (nbx <= 0) return hipSuccess;
  dim3 grid((unsigned)nbx, n_nodes, npole);
  return fwd_mfma_go<T, true>(st, grid, ft, lvl_nodes, S, N, factor, f_stride, x, nullptr,
                              nullptr, 0, cb, BB, real_l, yin);
}

// ----------------------------------------------------------- backward rect
// t[first + jb + l] = sum_a L(k + a, jb + l) x[U_s[a]] for one column block
// On the matrix cores: the RT-row tiles of the panel and the gathered x
// rows are staged through LDS (coalesced loads from clamped positions,
// prefetched into registers one tile ahead, masked when written); the
// products are 16 x 16 x 4 MFMAs whose rows are the block's columns and
// whose 16 result columns hold Re x and Im x of eight right-hand sides (as
// in the forward rect).  Wave w takes columns 16 (w % 2) .. + 15 and rows
// (RT / 2) (w / 2) .. of every tile; the two row halves are summed through
// LDS at the end.  x rows past the tile are staged as zeros (a zero panel
// entry times stale LDS could be NaN).  With the reduction running down the
// column-major panel, MFMA operands loaded straight from HBM would span 16
// columns x 4 rows per instruction (a quarter of each cache line used).
// COLS = true is the same product for a wide front's columns left of a
// block of rows: X[j] -= sum_{r in [cb, ce)} L(r, j) x_r for j < cb, x read
// in place (no gather), ce = min(k, cb + BB).  RL as in the forward kernel.
// xin (COLS only, may be null): the block's x rows are read from xin
// ([pole][N][S]) and copied into x by the launch, as yin in the forward
// kernel.
template <typename T, int NBK, bool COLS, bool RL = false>
__global__ __launch_bounds__(256) void k_bwd_rect_mfma(FrontTab ft, const int32_t *lvl_nodes,
                                                       int S, int64_t N, const cpx<T> *factor,
                                                       int64_t f_stride, cpx<T> *x,
                                                       cpx<T> *t, int64_t t_stride, int64_t cb,
                                                       int64_t BB, int pf, const cpx<T> *xin) {
  using MF = Mfma16<T>;
  using acc_t = typename MF::acc_t;
  const int s = lvl_nodes[blockIdx.y];
  const int p = pf > 1 ? (int)(blockIdx.x % pf) : (int)blockIdx.z;   // as in the forward kernel
  const int64_t bx = pf > 1 ? (int64_t)(blockIdx.x / pf) : (int64_t)blockIdx.x;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], u = ft.u[s], n = k + u, first = ft.first[s];
  const int64_t jb = bx * NB;
  // columns [jb, jb + w) take rows row0 + [0, u) of the panel
  int64_t row0 = k, ncol = k;
  cpx<T> *Xf = x + ((int64_t)p * N + first) * S;
  const cpx<T> *Xr = Xf;   // where the block's x rows are read (COLS)
  if (COLS) {
    if (cb >= k) return;
    row0 = cb;
    ncol = cb;
    if (xin) {
      Xr = xin + ((int64_t)p * N + first) * S;
      // block rows [cb + NB bx, + NB) of xin -> x
      const int64_t c0 = cb + bx * NB, c1 = min(min(k, cb + BB), c0 + NB);
      for (int64_t idx = c0 * S + threadIdx.x; idx < c1 * S; idx += 256) Xf[idx] = Xr[idx];
    }
  }
  if (jb >= ncol) return;
  const int w = (int)min((int64_t)NB, ncol - jb);
  const int64_t nr = COLS ? min(k, cb + BB) - cb : u;   // rows of the reduction
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];
  const cpx<T> *Xp = x + (int64_t)p * N * S;
  const int32_t *rows = ft.rows + ft.rows_off[s];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int mb = wave & 1, rh = wave >> 1;
  const int lr = lane & 15, ld4 = lane >> 4;
  int64_t ld;
  const cpx<T> *Lc = col_ptr(P, n, jb, ld);
  __shared__ cpx<T> Lt[NB][RT + 1];   // Lt[l][i] = L(k + ac + i, jb + l)
  __shared__ cpx<T> Xs[RT * 16 + 1];   // x rows [RT][16] and one sink slot
  cpx<T>(*Xt)[16] = reinterpret_cast<cpx<T>(*)[16]>(Xs);
  acc_t r1[NBK], r2[NBK];
#pragma unroll
  for (int nb = 0; nb < NBK; ++nb) {
    r1[nb] = acc_t{0, 0, 0, 0};
    r2[nb] = acc_t{0, 0, 0, 0};
  }
  // register prefetch of the next RT-row tile: NP panel elements and two x
  // values per thread (clamped in-bounds positions; masked in LDS)
  constexpr int NP = RT * NB / 256;   // panel elements per thread and tile
  cpx<T> pre[NP], px0, px1;
  auto xval = [&](int q, int64_t ac, int na) -> cpx<T> {
    const int idx = tid + 256 * q;
    const int i = min(idx / S, na - 1), c = idx % S;
    if (COLS) return Xr[(row0 + ac + i) * S + c];
    return Xp[(int64_t)rows[ac + i] * S + c];
  };
  auto fetch = [&](int64_t ac) {
    const int na = (int)min((int64_t)RT, nr - ac);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int idx = tid + 256 * q, i = min(idx % RT, na - 1), l = min(idx / RT, w - 1);
      pre[q] = Lc[(int64_t)l * ld + row0 + ac + i];
    }
    px0 = xval(0, ac, na);
    px1 = xval(1, ac, na);
  };
  if (nr > 0) fetch(0);
  for (int64_t ac = 0; ac < nr; ac += RT) {
    const int na = (int)min((int64_t)RT, nr - ac);
    lds_barrier();   // the previous tile's readers are done
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int idx = tid + 256 * q;
      const bool ok = idx % RT < na && idx / RT < w;
      Lt[idx / RT][idx % RT] = ok ? pre[q] : czero<T>();
    }
    // x rows: values of rows < na, zeros for the rows past na (right-hand
    // sides past S are never written: they only reach discarded outputs)
    auto xput = [&](int q, cpx<T> v) {
      const int idx = tid + 256 * q;
      const int i = idx / S;
      Xs[idx < RT * S ? i * 16 + idx % S : RT * 16] = i < na ? v : czero<T>();
    };
    xput(0, px0);
    xput(1, px1);
    lds_barrier();
    if (ac + RT < nr) fetch(ac + RT);
#pragma unroll
    for (int q = 0; q < RT / 8; ++q) {
      const int i = rh * (RT / 2) + 4 * q + ld4;
      const cpx<T> a = Lt[mb * 16 + lr][i];
#pragma unroll
      for (int nb = 0; nb < NBK; ++nb) {
        const cpx<T> xv = Xt[i][8 * nb + (lr & 7)];
        const T b = lr < 8 ? xv.re : xv.im;
        r1[nb] = MF::mma(a.re, b, r1[nb]);
        if constexpr (!RL) r2[nb] = MF::mma(a.im, b, r2[nb]);
      }
    }
  }
  // sum the row halves: waves 2, 3 hand theirs to waves 0, 1 through LDS
  lds_barrier();
  T *red = reinterpret_cast<T *>(&Lt[0][0]);   // [mb][nb][r1/r2][4][64]
  if (rh == 1) {
#pragma unroll
    for (int nb = 0; nb < NBK; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        red[(((mb * NBK + nb) * 2 + 0) * 4 + i) * 64 + lane] = r1[nb][i];
        red[(((mb * NBK + nb) * 2 + 1) * 4 + i) * 64 + lane] = r2[nb][i];
      }
  }
  lds_barrier();
  if (rh == 1) return;
  cpx<T> *To = t + (int64_t)p * t_stride + (first + jb) * S;
#pragma unroll
  for (int nb = 0; nb < NBK; ++nb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T a1 = r1[nb][i] + red[(((mb * NBK + nb) * 2 + 0) * 4 + i) * 64 + lane];
      const T a2 = r2[nb][i] + red[(((mb * NBK + nb) * 2 + 1) * 4 + i) * 64 + lane];
      const T o1 = __shfl_xor(a1, 8), o2 = __shfl_xor(a2, 8);
      const int m = mb * 16 + MF::row(ld4, i), j = 8 * nb + lr;
      if (lr >= 8 || j >= S || m >= w) continue;
      if (COLS) {
        cpx<T> *o = Xf + (jb + m) * S + j;
        *o = csub(*o, cpx<T>{a1 - o2, o1 + a2});
      } else {
        To[m * S + j] = {a1 - o2, o1 + a2};
      }
    }
}

// launches the backward MFMA kernel (as fwd_mfma_go)
template <typename T, bool COLS>
hipError_t bwd_mfma_go(hipStream_t st, dim3 grid, FrontTab ft, const int32_t *lvl_nodes, int S,
                       int64_t N, const cpx<T> *factor, int64_t f_stride, cpx<T> *x, cpx<T> *t,
                       int64_t t_stride, int64_t cb, int64_t BB, bool real_l,
                       const cpx<T> *xin = nullptr) {
  if (S < 1 || S > 16) return hipErrorInvalidValue;
  const bool two = S > 8;
  const int pf = (int)grid.z;   // poles fastest, as in fwd_mfma_go
  if (pf > 1) {
    grid.x *= pf;
    grid.z = 1;
  }
  if constexpr (sizeof(T) == 8) {
    if (real_l) {
      if (two)
        hipLaunchKernelGGL((k_bwd_rect_mfma<T, 2, COLS, true>), grid, dim3(256), 0, st, ft,
                           lvl_nodes, S, N, factor, f_stride, x, t, t_stride, cb, BB, pf, xin);
      else
        hipLaunchKernelGGL((k_bwd_rect_mfma<T, 1, COLS, true>), grid, dim3(256), 0, st, ft,
                           lvl_nodes, S, N, factor, f_stride, x, t, t_stride, cb, BB, pf, xin);
      return hipGetLastError();
    }
  }
  if (two)
    hipLaunchKernelGGL((k_bwd_rect_mfma<T, 2, COLS>), grid, dim3(256), 0, st, ft, lvl_nodes, S, N,
                       factor, f_stride, x, t, t_stride, cb, BB, pf, xin);
  else
    hipLaunchKernelGGL((k_bwd_rect_mfma<T, 1, COLS>), grid, dim3(256), 0, st, ft, lvl_nodes, S, N,
                       factor, f_stride, x, t, t_stride, cb, BB, pf, xin);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bwd_rect(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int max_k, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, const cpx<T> *x, cpx<T> *t, int64_t t_stride,
                           bool real_l) {
  if (n_nodes <= 0 || max_k <= 0) return hipSuccess;
  dim3 grid((max_k + NB - 1) / NB, n_nodes, npole);
  cpx<T> *xm = const_cast<cpx<T> *>(x);   // read only in this mode
  return bwd_mfma_go<T, false>(st, grid, ft, lvl_nodes, S, N, factor, f_stride, xm, t, t_stride,
                               0, 0, real_l);
}

// ------------------------------------------------------------ backward tri
// x_s = L11^{-T} (D^{-1} y_s - t_s), blocks from the last to the first
// (left-looking: each block first gathers the contributions of the rows
// below it inside L11).  With u == 0 the t term is absent.
// Blocks of columns [cb, ce) from the last to the first.  With init the
// right-hand side of each block is D^{-1} y - t (the whole triangle in one
// launch when cb = 0 and BB >= k); without, X already holds that value
// minus the contributions of the rows below ce (k_bwd_init, then the
// column mode of k_bwd_rect_mfma).
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_tri(FrontTab ft, const int32_t *lvl_nodes, int S,
                                                 int64_t N, const cpx<T> *factor,
                                                 int64_t f_stride, cpx<T> *x, const cpx<T> *t,
                                                 int64_t t_stride, int64_t cb, int64_t BB,
                                                 int init) {
  const int s = lvl_nodes[blockIdx.x];
  const int p = blockIdx.y;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], u = ft.u[s], n = k + u, first = ft.first[s];
  if (k == 0 || cb >= k) return;
  const int64_t ce = min(k, cb + BB);
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];
  cpx<T> *X = x + ((int64_t)p * N + first) * S;
  const cpx<T> *Tv = t + (int64_t)p * t_stride + first * S;
  const int tid = threadIdx.x;
  __shared__ cpx<T> Li[NB][NB + 1];
  __shared__ cpx<T> V[NB][16];
  __shared__ cpx<T> Lt[NB][RTT + 1];
  __shared__ cpx<T> Xt[RTT][16];
  const int64_t b_first = cb / NB, b_last = (ce + NB - 1) / NB - 1;
  for (int64_t bi = b_last; bi >= b_first; --bi) {
    const int64_t jb = bi * NB;
    const int w = (int)min((int64_t)NB, k - jb);
    int64_t ld;
    const cpx<T> *Lc = col_ptr(P, n, jb, ld);
    cpx<T> acc[2];
    acc[0] = czero<T>();
    acc[1] = czero<T>();
    // contributions of the already solved rows jb+w .. ce-1
    for (int64_t rc = jb + w; rc < ce; rc += RTT) {
      const int nr = (int)min((int64_t)RTT, ce - rc);
      __syncthreads();
      stage_tile<T, RTT>(Lt, Lc, ld, rc, nr, w, tid);
      for (int idx = tid; idx < nr * S; idx += blockDim.x) Xt[idx / S][idx % S] = X[rc * S + idx];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int idx = tid + 256 * q;
        if (idx < w * S) {
          const int l = idx / S, c = idx % S;
          cpx<T> sacc = acc[q];
          for (int i = 0; i < nr; ++i) sacc = cfma(Lt[l][i], Xt[i][c], sacc);
          acc[q] = sacc;
        }
      }
    }
    __syncthreads();
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int j = idx % w, l = idx / w;
      Li[j][l] = Lc[(int64_t)j * ld + jb + l];   // entries l >= j unused
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      if (idx < w * S) {
        const int l = idx / S, c = idx % S;
        cpx<T> v = X[jb * S + idx];
        if (init) {
          const cpx<T> d = Lc[(int64_t)l * ld + jb + l];
          v = cmul(v, cinv(d));
          if (u > 0) v = csub(v, Tv[jb * S + idx]);
        }
        V[l][c] = csub(v, acc[q]);
      }
    }
    __syncthreads();
    // x_b = Linv^T v_b : x[l] = v[l] + sum_{j > l} Linv[j][l] v[j]
    for (int idx = tid; idx < w * S; idx += blockDim.x) {
      const int l = idx / S, c = idx % S;
      cpx<T> r = V[l][c];
      for (int j = l + 1; j < w; ++j) r = cfma(Li[j][l], V[j][c], r);
      X[jb * S + idx] = r;
    }
    __syncthreads();
  }
}

// Backward triangle for ranges of at most 256 rows, right-looking:
// thread i owns row cb + i and keeps its right-hand side v in registers
// (D^{-1} y - t with init, else the value in x).  Blocks run from the last
// to the first; per block the owners publish v, x_b = v + Lo^T v is formed
// and written out (Lo as in the forward kernel), and every earlier row r of
// the range subtracts sum_l L(jb + l, r) x_b[l], from its own column's
// entries below the block, loaded one block ahead.  SP as in the forward
// kernel.
template <typename T, int SP, bool RL>
__global__ __launch_bounds__(256) void k_bwd_tri_reg(FrontTab ft, const int32_t *lvl_nodes,
                                                     int S, int64_t N, const cpx<T> *factor,
                                                     int64_t f_stride, cpx<T> *x,
                                                     const cpx<T> *t, int64_t t_stride,
                                                     int64_t cb, int64_t BB, int init) {
  constexpr int NT = NB * SP / 256;
  typedef FacVal<T, RL> FV;           // RL: real factor, kept and applied as real
  const int s = lvl_nodes[blockIdx.x];
  const int p = blockIdx.y;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], u = ft.u[s], n = k + u, first = ft.first[s];
  if (k == 0 || cb >= k) return;
  const int64_t ce = min(k, cb + BB);
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];
  cpx<T> *X = x + ((int64_t)p * N + first) * S;
  const cpx<T> *Tv = t + (int64_t)p * t_stride + first * S;
  const int tid = threadIdx.x;
  const int nr = (int)(ce - cb);   // <= 256 (checked by the launcher)
  const bool own = tid < nr;
  const int64_t r = cb + min(tid, nr - 1);
  int64_t ldr;
  const cpx<T> *Lr = col_ptr(P, n, r, ldr);   // column r: element (i, r) at Lr[i]
  const int64_t r0 = NB * (r / NB);
  cpx<T> v[SP];
  {
    const cpx<T> dinv = init ? cinv(Lr[r]) : cpx<T>{T(1), T(0)};
    const bool tt = init && u > 0;
#pragma unroll
    for (int c = 0; c < SP; ++c) {
      const int64_t id = r * S + min(c, S - 1);
      v[c] = cmul(X[id], dinv);
      if (tt) v[c] = csub(v[c], Tv[id]);
    }
  }
  __shared__ typename FV::type Lo[NB][NB + 1];   // Lo[l][j] = Linv[j][l] for l < j < w
  __shared__ cpx<T> V[NB][SP];
  __shared__ cpx<T> Y[NB][SP];
  typename FV::type lv[NB], li[NB * NB / 256];
  const int64_t b_first = cb / NB, b_last = (ce + NB - 1) / NB - 1;
  auto fetch_li = [&](int64_t bi) {
    const int64_t jb = max(bi, b_first) * NB;
    const int w = (int)min((int64_t)NB, k - jb);
    int64_t ld;
    const cpx<T> *Lc = col_ptr(P, n, jb, ld);
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
      const int idx = tid + 256 * q, j = idx % NB, l = idx / NB;
      li[q] = FV::of(Lc[(int64_t)min(j, w - 1) * ld + jb + min(l, w - 1)]);
    }
  };
  // L(jb + l, r) for the block's rows: column r below its own block (rows
  // before the column's block are clamped to it: they are not stored)
  auto fetch_lv = [&](int64_t bi) {
    const int64_t jb = max(bi, b_first) * NB;
    const int w = (int)min((int64_t)NB, k - jb);
#pragma unroll
    for (int l = 0; l < NB; ++l) lv[l] = FV::of(Lr[max(jb + min(l, w - 1), r0)]);
  };
  fetch_li(b_last);
  fetch_lv(b_last);
  for (int64_t bi = b_last; bi >= b_first; --bi) {
    const int64_t jb = bi * NB;
    const int w = (int)min((int64_t)NB, k - jb);
    lds_barrier();   // the previous block's readers of Lo, V and Y are done
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
      const int idx = tid + 256 * q, j = idx % NB, l = idx / NB;
      Lo[l][j] = (l < j && j < w) ? li[q] : FV::of(czero<T>());
    }
    fetch_li(bi - 1);
    if (own && r >= jb && r < jb + w) {
#pragma unroll
      for (int c = 0; c < SP; ++c) V[r - jb][c] = v[c];
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) {   // rows past w of the block: zero
      const int idx = tid + 256 * q, j = idx / SP;
      if (j >= w) V[j][idx % SP] = czero<T>();
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int idx = tid + 256 * q, l = idx / SP, c = idx % SP;
      cpx<T> acc = V[l][c];
#pragma unroll
      for (int j = 0; j < NB; ++j) acc = FV::fma_(Lo[l][j], V[j][c], acc);
      Y[l][c] = acc;
      if (l < w && c < S) X[(jb + l) * S + c] = acc;
    }
    lds_barrier();
    if (own && r < jb) {
#pragma unroll
      for (int l = 0; l < NB; ++l) {
        const typename FV::type a = l < w ? FV::neg(lv[l]) : FV::of(czero<T>());
#pragma unroll
        for (int c = 0; c < SP; ++c) v[c] = FV::fma_(a, Y[l][c], v[c]);
      }
    }
    fetch_lv(bi - 1);
  }
}

template <typename T>
hipError_t launch_bwd_tri(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                          int npole, int S, int64_t N, const cpx<T> *factor, int64_t f_stride,
                          cpx<T> *x, const cpx<T> *t, int64_t t_stride, int64_t cb, int64_t BB,
                          int init, bool real_l) {
  if (n_nodes <= 0) return hipSuccess;
  // the column blocks of wide fronts (at most 256 rows, one per thread)
  // take the register kernel; whole small fronts, many per level, keep the
  // lighter LDS kernel
  if (S >= 1 && S <= 16 && BB <= 256 && BB % NB == 0 && cb % NB == 0)
    hipLaunchKernelGGL((real_l ? (S <= 8 ? k_bwd_tri_reg<T, 8, true> : k_bwd_tri_reg<T, 16, true>)
                               : (S <= 8 ? k_bwd_tri_reg<T, 8, false>
                                         : k_bwd_tri_reg<T, 16, false>)),
                       dim3(n_nodes, npole), dim3(256), 0, st, ft, lvl_nodes, S, N, factor,
                       f_stride, x, t, t_stride, cb, BB, init);
  else
    hipLaunchKernelGGL(k_bwd_tri<T>, dim3(n_nodes, npole), dim3(256), 0, st, ft, lvl_nodes, S, N,
                       factor, f_stride, x, t, t_stride, cb, BB, init);
  return hipGetLastError();
}

// ------------------------------------------------------ backward init
// X[j] = y_j / d_j - t_j for all columns of the front
template <typename T>
__global__ void k_bwd_init(FrontTab ft, const int32_t *lvl_nodes, int S, int64_t N,
                           const cpx<T> *factor, int64_t f_stride, cpx<T> *x, const cpx<T> *t,
                           int64_t t_stride) {
  const int s = lvl_nodes[blockIdx.y];
  const int p = blockIdx.z;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], u = ft.u[s], n = k + u, first = ft.first[s];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k * S) return;
  const int64_t j = idx / S;
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];
  const cpx<T> d = P[panel_elem(n, j, j)];
  cpx<T> *X = x + ((int64_t)p * N + first) * S;
  cpx<T> v = cmul(X[idx], cinv(d));
  if (u > 0) v = csub(v, t[(int64_t)p * t_stride + first * S + idx]);
  X[idx] = v;
}

template <typename T>
hipError_t launch_bwd_init(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int max_k, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, cpx<T> *x, const cpx<T> *t, int64_t t_stride) {
  if (n_nodes <= 0 || max_k <= 0) return hipSuccess;
  dim3 grid(((int64_t)max_k * S + 255) / 256, n_nodes, npole);
  hipLaunchKernelGGL(k_bwd_init<T>, grid, dim3(256), 0, st, ft, lvl_nodes, S, N, factor, f_stride,
                     x, t, t_stride);
  return hipGetLastError();
}

// ------------------------------------------------------ backward cols
// X[j] -= sum_{r in [cb, ce)} L(r, j) x_r for the column blocks of j < cb
// xin: the block's x rows in rows [cb, ce) of xin, copied into x by the
// same launch
template <typename T>
hipError_t launch_bwd_cols(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                           int64_t cb, int npole, int S, int64_t N, const cpx<T> *factor,
                           int64_t f_stride, cpx<T> *x, int64_t BB, bool real_l,
                           const cpx<T> *xin) {
  if (n_nodes <= 0) return hipSuccess;
  int64_t nbx = (cb + NB - 1) / NB;
  if (xin) nbx = std::max<int64_t>(nbx, (BB + NB - 1) / NB);   // the copy of the block rows
  if (nbx <= 0) return hipSuccess;
  dim3 grid((unsigned)nbx, n_nodes, npole);
  return bwd_mfma_go<T, true>(st, grid, ft, lvl_nodes, S, N, factor, f_stride, x, nullptr, 0, cb,
                              BB, real_l, xin);
}

// ------------------------------------------- explicit diagonal-block inverses
// For the wide fronts (levels walked in BB-column blocks) the unit-lower
// diagonal block of columns [b BB, b BB + w), w = min(BB, k - b BB), is
// inverted once per factorisation, so that a sweep applies it as one
// matrix product over many workgroups instead of a chain of NB-column
// steps inside one workgroup per front and pole.  From the stored NB x NB
// diagonal inverses Linv_i (the panel's strictly upper diagonal-block parts)
// and the panel's off-diagonal NB x NB blocks L_iq:
//   X_jj = Linv_j,   X_ij = -Linv_i sum_{j <= q < i} L_iq X_qj   (i > j).
// X (column-major, leading dimension w) and then its transpose (the same
// layout) start at xoff[s] + 2 b BB^2 of the pole's region (x_stride
// elements per pole).  One workgroup per group of CW columns of a block:
// the group's columns of X stay in LDS while its NB-row blocks are formed
// in order.
template <typename T>
__global__ __launch_bounds__(256) void k_diag_inverse(FrontTab ft, const int32_t *lvl_nodes,
                                                      const cpx<T> *factor, int64_t f_stride,
                                                      cpx<T> *xinv, int64_t x_stride,
                                                      const int64_t *xoff, int BB) {
  constexpr int CW = sizeof(T) == 4 ? 16 : 8;   // columns per workgroup
  constexpr int NE = NB * CW / 256;             // entries of a row block per thread
  const int gpb = BB / CW;
  const int s = lvl_nodes[blockIdx.y];
  const int p = blockIdx.z;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], n = k + ft.u[s];
  const int bb = (int)(blockIdx.x / gpb), g = (int)(blockIdx.x % gpb);
  const int64_t cb = (int64_t)bb * BB;
  if (cb >= k) return;
  const int w = (int)min((int64_t)BB, k - cb);
  const int c0 = g * CW;
  if (c0 >= w) return;
  const int j = c0 / NB, nbw = (w + NB - 1) / NB;
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];
  __shared__ cpx<T> Xs[256][CW];        // rows [NB j, w) of the group's columns
  __shared__ cpx<T> Ts[NB][CW];
  __shared__ cpx<T> Lt[NB][NB + 1];     // Linv_i[a][b], b < a
  const int tid = threadIdx.x, a = tid % NB, cg = tid / NB;
  // X_jj = Linv_j: unit diagonal; Linv_j[r][c] (r > c) is stored at (row c, column r)
  for (int idx = tid; idx < NB * CW; idx += 256) {
    const int r = idx / CW, c = idx % CW, cc = c0 + c - NB * j;
    cpx<T> v = czero<T>();
    if (NB * j + r < w && c0 + c < w) {
      if (r == cc)
        v = cpx<T>{T(1), T(0)};
      else if (r > cc)
        v = P[panel_elem(n, cb + NB * j + cc, cb + NB * j + r)];
    }
    Xs[NB * j + r][c] = v;
  }
  __syncthreads();
  for (int i = j + 1; i < nbw; ++i) {
    const int wi = min(NB, w - NB * i);
    for (int idx = tid; idx < NB * NB; idx += 256) {   // Linv_i (consecutive b: one column)
      const int ra = idx / NB, b = idx % NB;
      Lt[ra][b] = (b < ra && ra < wi) ? P[panel_elem(n, cb + NB * i + b, cb + NB * i + ra)]
                                      : czero<T>();
    }
    // T[a][c] = sum_{q in [NB j, NB i)} L(cb + NB i + a, cb + q) X[q][c], the
    // row's entries loaded NB at a time (rows past wi clamped, results unused)
    const int64_t row = cb + NB * i + min(a, wi - 1);
    cpx<T> acc[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) acc[e] = czero<T>();
    for (int q0 = NB * j; q0 < NB * i; q0 += NB) {
      const cpx<T> *Lc = P + panel_block_off(n, (cb + q0) / NB) - (cb + q0) + row;
      const int64_t ld = n - (cb + q0);   // column block of q0: element (r, c) at Lc[(c - q0') ld]
      cpx<T> lq[NB];
#pragma unroll
      for (int l = 0; l < NB; ++l) lq[l] = Lc[(int64_t)l * ld];
#pragma unroll
      for (int l = 0; l < NB; ++l)
#pragma unroll
        for (int e = 0; e < NE; ++e) acc[e] = cfma(lq[l], Xs[q0 + l][cg + 8 * e], acc[e]);
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) Ts[a][cg + 8 * e] = a < wi ? acc[e] : czero<T>();
    __syncthreads();
    // X_ij = -Linv_i T = -(T + Lo_i T)
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int c = cg + 8 * e;
      cpx<T> r = Ts[a][c];
      for (int b = 0; b < a; ++b) r = cfma(Lt[a][b], Ts[b][c], r);
      if (a < wi) Xs[NB * i + a][c] = cpx<T>{-r.re, -r.im};
    }
    __syncthreads();
  }
  // X and its transpose; rows above block j are zero
  cpx<T> *Xo = xinv + (int64_t)p * x_stride + xoff[s] + 2 * (int64_t)bb * BB * BB;
  cpx<T> *XTo = Xo + (int64_t)w * w;
  const int cw = min(CW, w - c0);
  for (int idx = tid; idx < w * cw; idx += 256) {
    const int c = idx / w, r = idx % w;
    Xo[(int64_t)(c0 + c) * w + r] = r < NB * j ? czero<T>() : Xs[r][c];
  }
  for (int idx = tid; idx < w * cw; idx += 256) {
    const int r = idx / cw, c = idx % cw;
    XTo[(int64_t)r * w + c0 + c] = r < NB * j ? czero<T>() : Xs[r][c];
  }
}

template <typename T>
hipError_t launch_diag_inverse(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                               int max_k, int npole, const cpx<T> *factor, int64_t f_stride,
                               cpx<T> *xinv, int64_t x_stride, const int64_t *xoff, int BB) {
  constexpr int CW = sizeof(T) == 4 ? 16 : 8;
  if (n_nodes <= 0 || max_k <= 0) return hipSuccess;
  if (BB < NB || BB > 256 || BB % NB != 0) return hipErrorInvalidValue;
  const int64_t nbb = (max_k + BB - 1) / BB;
  dim3 grid((unsigned)(nbb * (BB / CW)), n_nodes, npole);
  hipLaunchKernelGGL(k_diag_inverse<T>, grid, dim3(256), 0, st, ft, lvl_nodes, factor, f_stride,
                     xinv, x_stride, xoff, BB);
  return hipGetLastError();
}

// The children's update rows added to the top rows of every front of a
// level (the first step of the forward sweep of a wide front).
template <typename T>
__global__ __launch_bounds__(256) void k_fwd_child_add(FrontTab ft, const int32_t *lvl_nodes,
                                                       int S, int64_t N, cpx<T> *x,
                                                       const cpx<T> *w_child, int64_t w_stride) {
  const int s = lvl_nodes[blockIdx.x];
  const int p = blockIdx.y;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s];
  if (k == 0) return;
  cpx<T> *X = x + ((int64_t)p * N + ft.first[s]) * S;
  fwd_child_add<T>(ft, s, p, k, S, X, w_child, w_stride, threadIdx.x);
}

template <typename T>
hipError_t launch_fwd_child_add(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                                int npole, int S, int64_t N, cpx<T> *x, const cpx<T> *w_child,
                                int64_t w_stride) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fwd_child_add<T>, dim3(n_nodes, npole), dim3(256), 0, st, ft, lvl_nodes, S,
                     N, x, w_child, w_stride);
  return hipGetLastError();
}

// out rows [cb, cb + w) = M x rows [cb, cb + w) for every front and pole of
// a level: M = X_b (UPPER false, the forward step) or its transpose (UPPER
// true, the backward step), b = cb / BB.  A workgroup takes one NB-row
// slab of M; its wave q multiplies the slab's q-th NB x NB tile (the tiles
// on the other side of the diagonal are zero and skipped) with x on the
// matrix cores (operands as in the forward rect kernel), and the tiles'
// products are summed through LDS in tile order.
template <typename T, int NBK, bool UPPER, bool RL>
__global__ __launch_bounds__(512) void k_blk_apply(FrontTab ft, const int32_t *lvl_nodes, int S,
                                                   int64_t N, const cpx<T> *xinv,
                                                   int64_t x_stride, const int64_t *xoff, int BB,
                                                   int64_t cb, const cpx<T> *x, cpx<T> *out,
                                                   int pf) {
  using MF = Mfma16<T>;
  using acc_t = typename MF::acc_t;
  const int s = lvl_nodes[blockIdx.y];
  const int p = pf > 1 ? (int)(blockIdx.x % pf) : (int)blockIdx.z;
  const int i = pf > 1 ? (int)(blockIdx.x / pf) : (int)blockIdx.x;   // row slab
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], first = ft.first[s];
  if (cb >= k) return;
  const int w = (int)min((int64_t)BB, k - cb);
  if (NB * i >= w) return;   // uniform over the workgroup
  const int nq = (w + NB - 1) / NB;
  const cpx<T> *M = xinv + (int64_t)p * x_stride + xoff[s] + 2 * (cb / BB) * BB * BB +
                    (UPPER ? (int64_t)w * w : 0);
  __shared__ cpx<T> red[8][NB][8 * NBK];
  const int lane = threadIdx.x & 63;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // column tile
  const bool act = q < nq && (UPPER ? q >= i : q <= i);
  if (act) {
    const int lr = lane & 15, ld4 = lane >> 4;
    int rrow[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) rrow[b] = min(NB * i + 16 * b + lr, w - 1);
    int yj[NBK];
    bool yon[NBK];
#pragma unroll
    for (int nb = 0; nb < NBK; ++nb) {
      const int jj = 8 * nb + (lr & 7);
      yon[nb] = jj < S;
      yj[nb] = 2 * min(jj, S - 1) + (lr >> 3);
    }
    const T *Xv = reinterpret_cast<const T *>(x + ((int64_t)p * N + first + cb) * S);
    cpx<T> lv[NB / 4][2];
    T yv[NB / 4][NBK];
#pragma unroll
    for (int qq = 0; qq < NB / 4; ++qq) {
      const int col = NB * q + 4 * qq + ld4, cc = min(col, w - 1);
#pragma unroll
      for (int b = 0; b < 2; ++b) lv[qq][b] = M[(int64_t)cc * w + rrow[b]];
#pragma unroll
      for (int nb = 0; nb < NBK; ++nb)   // a multiply, not a select: the load stays unconditional
        yv[qq][nb] = Xv[(int64_t)cc * 2 * S + yj[nb]] * ((col < w && yon[nb]) ? T(1) : T(0));
    }
    acc_t r1[2][NBK], r2[2][NBK];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int nb = 0; nb < NBK; ++nb) {
        r1[b][nb] = acc_t{0, 0, 0, 0};
        r2[b][nb] = acc_t{0, 0, 0, 0};
      }
#pragma unroll
    for (int qq = 0; qq < NB / 4; ++qq)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int nb = 0; nb < NBK; ++nb) {
          r1[b][nb] = MF::mma(lv[qq][b].re, yv[qq][nb], r1[b][nb]);
          if constexpr (!RL) r2[b][nb] = MF::mma(lv[qq][b].im, yv[qq][nb], r2[b][nb]);
        }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int nb = 0; nb < NBK; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const T o1 = __shfl_xor(r1[b][nb][e], 8), o2 = __shfl_xor(r2[b][nb][e], 8);
          if (lr < 8)
            red[q][16 * b + MF::row(ld4, e)][8 * nb + lr] =
                cpx<T>{r1[b][nb][e] - o2, o1 + r2[b][nb][e]};
        }
  }
  __syncthreads();
  const int q0 = UPPER ? i : 0, q1 = UPPER ? nq - 1 : i;
  cpx<T> *O = out + ((int64_t)p * N + first + cb) * S;
  for (int idx = threadIdx.x; idx < NB * S; idx += 512) {
    const int ra = idx / S, jj = idx % S;
    const int r = NB * i + ra;
    if (r >= w) continue;
    cpx<T> v = czero<T>();
    for (int qt = q0; qt <= q1; ++qt) v = cadd(v, red[qt][ra][jj]);
    O[(int64_t)r * S + jj] = v;
  }
}

template <typename T, int NBK, bool UPPER>
void blk_apply_go(hipStream_t st, dim3 grid, bool real_l, FrontTab ft, const int32_t *lvl_nodes,
                  int S, int64_t N, const cpx<T> *xinv, int64_t x_stride, const int64_t *xoff,
                  int BB, int64_t cb, const cpx<T> *x, cpx<T> *out, int pf) {
  if (real_l)
    hipLaunchKernelGGL((k_blk_apply<T, NBK, UPPER, true>), grid, dim3(512), 0, st, ft, lvl_nodes,
                       S, N, xinv, x_stride, xoff, BB, cb, x, out, pf);
  else
    hipLaunchKernelGGL((k_blk_apply<T, NBK, UPPER, false>), grid, dim3(512), 0, st, ft, lvl_nodes,
                       S, N, xinv, x_stride, xoff, BB, cb, x, out, pf);
}

// real_l: the inverses are real (a real factor; their imaginary parts are
// zero and skipped).  FP64 takes at most 8 right-hand sides (the LDS of the
// tile sums).
template <typename T>
hipError_t launch_blk_apply(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                            int npole, int S, int64_t N, const cpx<T> *xinv, int64_t x_stride,
                            const int64_t *xoff, int BB, int64_t cb, bool upper, bool real_l,
                            const cpx<T> *x, cpx<T> *out) {
  if (n_nodes <= 0) return hipSuccess;
  if (S < 1 || S > (sizeof(T) == 4 ? 16 : 8) || BB < NB || BB > 256 || BB % NB != 0)
    return hipErrorInvalidValue;
  const int pf = npole;   // poles fastest, as in the rect kernels
  dim3 grid((unsigned)((BB / NB) * pf), n_nodes, 1);
  if constexpr (sizeof(T) == 4) {
    if (S > 8) {
      if (upper)
        blk_apply_go<T, 2, true>(st, grid, real_l, ft, lvl_nodes, S, N, xinv, x_stride, xoff, BB,
                                 cb, x, out, pf);
      else
        blk_apply_go<T, 2, false>(st, grid, real_l, ft, lvl_nodes, S, N, xinv, x_stride, xoff,
                                  BB, cb, x, out, pf);
      return hipGetLastError();
    }
  }
  if (upper)
    blk_apply_go<T, 1, true>(st, grid, real_l, ft, lvl_nodes, S, N, xinv, x_stride, xoff, BB, cb,
                             x, out, pf);
  else
    blk_apply_go<T, 1, false>(st, grid, real_l, ft, lvl_nodes, S, N, xinv, x_stride, xoff, BB, cb,
                              x, out, pf);
  return hipGetLastError();
}

#define TEM_INST_INV(T)                                                                          \
  template hipError_t launch_diag_inverse<T>(hipStream_t, FrontTab, const int32_t *, int, int,   \
                                             int, const cpx<T> *, int64_t, cpx<T> *, int64_t,    \
                                             const int64_t *, int);                              \
  template hipError_t launch_fwd_child_add<T>(hipStream_t, FrontTab, const int32_t *, int, int,  \
                                              int, int64_t, cpx<T> *, const cpx<T> *, int64_t);  \
  template hipError_t launch_blk_apply<T>(hipStream_t, FrontTab, const int32_t *, int, int, int, \
                                          int64_t, const cpx<T> *, int64_t, const int64_t *,     \
                                          int, int64_t, bool, bool, const cpx<T> *, cpx<T> *);
TEM_INST_INV(float)
TEM_INST_INV(double)
#undef TEM_INST_INV

#define TEM_INST(T)                                                                              \
  template hipError_t launch_fwd_tri<T>(hipStream_t, FrontTab, const int32_t *, int, int, int,    \
                                        int64_t, const cpx<T> *, int64_t, cpx<T> *,              \
                                        const cpx<T> *, int64_t, int64_t, int64_t, bool);        \
  template hipError_t launch_fwd_rows<T>(hipStream_t, FrontTab, const int32_t *, int, int, int,   \
                                         int, int64_t, const cpx<T> *, int64_t, cpx<T> *,        \
                                         int64_t, int64_t, bool, const cpx<T> *);                \
  template hipError_t launch_bwd_init<T>(hipStream_t, FrontTab, const int32_t *, int, int, int,   \
                                         int, int64_t, const cpx<T> *, int64_t, cpx<T> *,        \
                                         const cpx<T> *, int64_t);                               \
  template hipError_t launch_bwd_cols<T>(hipStream_t, FrontTab, const int32_t *, int, int64_t,    \
                                         int, int, int64_t, const cpx<T> *, int64_t, cpx<T> *,   \
                                         int64_t, bool, const cpx<T> *);                         \
  template hipError_t launch_fwd_rect<T>(hipStream_t, FrontTab, const int32_t *, int, int, int,   \
                                         int, int64_t, const cpx<T> *, int64_t, const cpx<T> *,  \
                                         const cpx<T> *, cpx<T> *, int64_t, bool);               \
  template hipError_t launch_bwd_rect<T>(hipStream_t, FrontTab, const int32_t *, int, int, int,   \
                                         int, int64_t, const cpx<T> *, int64_t, const cpx<T> *,  \
                                         cpx<T> *, int64_t, bool);                               \
  template hipError_t launch_bwd_tri<T>(hipStream_t, FrontTab, const int32_t *, int, int, int,    \
                                        int64_t, const cpx<T> *, int64_t, cpx<T> *,              \
                                        const cpx<T> *, int64_t, int64_t, int64_t, int, bool);
TEM_INST(float)
TEM_INST(double)
#undef TEM_INST

}  // namespace tem
