// Batched multifrontal complex-symmetric LDL^T of A_i = K - xi_i M:
// front assembly, extend-add, panel factorisation (diagonal block LDL^T with
// the inverse of its unit-lower factor, triangular solve of the rows below)
// and the MFMA trailing / contribution-block updates.  One launch covers
// every front of one tree level for every pole.
#include "k_common.h"

namespace tem {

// ------------------------------------------------------------------ fills
template <typename T>
__global__ void k_fill_zero(cpx<T> *base, int64_t count, int64_t pole_stride) {
  cpx<T> *p = base + (int64_t)blockIdx.y * pole_stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = czero<T>();
}

template <typename T>
hipError_t launch_fill_zero(hipStream_t st, cpx<T> *base, int64_t count, int npole,
                            int64_t pole_stride) {
  if (count <= 0 || npole <= 0) return hipSuccess;
  dim3 grid(grid_1d(count, 256, 4096), npole);
  hipLaunchKernelGGL(k_fill_zero<T>, grid, dim3(256), 0, st, base, count, pole_stride);
  return hipGetLastError();
}

// ------------------------------------------------------ original entries
// factor[pole][pos[i]] = K[csr[i]] - xi * M[csr[i]], xi the pole's shift for
// the mesh that owns matrix entry csr[i] (sg: entry segments)
template <typename T>
__global__ void k_front_assemble(int64_t n, const int32_t *csr, const int64_t *pos,
                                 const double *Kv, const double *Mv, const double *xi, Seg sg,
                                 cpx<T> *factor, int64_t pole_stride) {
  const int p = blockIdx.y;
  cpx<T> *F = factor + (int64_t)p * pole_stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = csr[i];
    const int64_t xo = 2 * ((int64_t)seg_find(sg, e) * sg.stride + p);
    const double xr = xi[xo], xim = xi[xo + 1];
    const double kv = Kv[e], mv = Mv[e];
    cpx<T> v;
    v.re = (T)(kv - xr * mv);
    v.im = (T)(-xim * mv);
    F[pos[i]] = v;
  }
}

template <typename T>
hipError_t launch_front_assemble(hipStream_t st, int64_t n_entries, const int32_t *csr,
                                 const int64_t *pos, const double *Kv, const double *Mv,
                                 const double *xi, Seg sg, int npole, cpx<T> *factor,
                                 int64_t pole_stride) {
  if (n_entries <= 0) return hipSuccess;
  dim3 grid(grid_1d(n_entries, 256, 8192), npole);
  hipLaunchKernelGGL(k_front_assemble<T>, grid, dim3(256), 0, st, n_entries, csr, pos, Kv, Mv,
                     xi, sg, factor, pole_stride);
  return hipGetLastError();
}

// ----------------------------------------------------------- extend-add
// Adds child `slot`'s contribution block into its parent front through the
// relative row map, one column b of the block (rows a >= b) per wave: the
// list holds (parent front, b) pairs.  Columns whose parent position is a
// pivot column of the parent go to the panel (before the parent is
// factored); the others go to the parent's contribution block (after its
// own update has written it).  One slot per launch keeps the scatter free
// of races (two children may hit the same parent entry).
template <typename T>
__global__ __launch_bounds__(256) void k_extend_add(FrontTab ft, const int2 *cols, int64_t n_cols,
                                                    int slot, cpx<T> *factor, int64_t f_stride,
                                                    cpx<T> *cb_par, cpx<T> *cb_ch,
                                                    int64_t cb_stride) {
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.y;
  if (e >= n_cols) return;
  const int s = cols[e].x;
  const int64_t b = cols[e].y;
  if (pole_absent(ft, s, p)) return;
  const int ch = slot == 0 ? ft.child0[s] : ft.child1[s];
  const int64_t uc = ft.u[ch];
  const int64_t kp = ft.k[s], up = ft.u[s], np = kp + up;
  const int32_t *rel = ft.rel + ft.rows_off[ch];
  const cpx<T> *src = cb_ch + (int64_t)p * cb_stride + ft.cb_off[ch] + b * uc;
  const int64_t rb = rel[b];
  cpx<T> *dst;
  if (rb < kp) {   // panel column rb: element (r, rb) at dst[r]
    const int64_t r0 = NB * (rb / NB);
    dst = factor + (int64_t)p * f_stride + ft.panel_off[s] + panel_block_off(np, rb / NB) +
          (rb - r0) * (np - r0) - r0;
  } else {         // contribution-block column rb - kp: element (r, rb) at dst[r]
    dst = cb_par + (int64_t)p * cb_stride + ft.cb_off[s] + (rb - kp) * up - kp;
  }
  for (int64_t a = b + lane; a < uc; a += 64) {
    cpx<T> *q = dst + rel[a];
    *q = cadd(*q, src[a]);
  }
}

template <typename T>
hipError_t launch_extend_add(hipStream_t st, FrontTab ft, const int2 *cols, int64_t n_cols,
                             int slot, int npole, cpx<T> *factor, int64_t f_stride,
                             cpx<T> *cb_parent, cpx<T> *cb_child, int64_t cb_stride) {
  if (n_cols <= 0) return hipSuccess;
  dim3 grid((unsigned)((n_cols + 3) / 4), npole);
  hipLaunchKernelGGL(k_extend_add<T>, grid, dim3(256), 0, st, ft, cols, n_cols, slot, factor,
                     f_stride, cb_parent, cb_child, cb_stride);
  return hipGetLastError();
}

// -------------------------------------------------------- panel diagonal
// LDL^T (no pivoting) of the NB x NB diagonal block of column block j0/NB,
// then the inverse of its unit-lower factor, stored transposed in the
// strictly upper part of the block.  flags[0] |= 1 on a zero or non-finite
// pivot; flags[1] counts tiny pivots.  Both triangular recurrences (the
// elimination and the inverse) run a column step at a time over all the
// entries that step updates.  With jp >= 0 (= j0 - NB) the block first takes
// the update of the factored block jp: A_jj -= L_j,p D_p L_j,p^T (the last
// update of the block, left-looking, in place of a separate launch).
template <typename T>
__global__ __launch_bounds__(256) void k_panel_diag(FrontTab ft, const int32_t *lvl_nodes, int j0,
                                                    int jp, cpx<T> *factor, int64_t f_stride,
                                                    int *flags) {
  const int s = lvl_nodes[blockIdx.x];
  const int p = blockIdx.y;
  if (pole_absent(ft, s, p)) return;
  const int k = ft.k[s];
  if (j0 >= k) return;
  const int w = min(NB, k - j0);
  const int64_t n = (int64_t)k + ft.u[s];
  const int64_t ld = n - j0;
  cpx<T> *blk = factor + (int64_t)p * f_stride + ft.panel_off[s] + panel_block_off(n, j0 / NB);
  __shared__ cpx<T> F[NB][NB + 1];   // F[c][r]
  __shared__ cpx<T> Iv[NB][NB + 1];  // inverse of the unit lower factor, Iv[c][r]
  const int tid = threadIdx.x;
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    const int r = idx % w, c = idx / w;
    F[c][r] = (r >= c) ? blk[(int64_t)c * ld + r] : czero<T>();
  }
  if (jp >= 0) {
    // rows j0 .. j0+w-1 of block jp (below its diagonal block: plain L) and
    // its pivots; Iv is free until the inverse is formed
    const int64_t ldp = n - jp;
    const cpx<T> *bp = factor + (int64_t)p * f_stride + ft.panel_off[s] + panel_block_off(n, jp / NB);
    for (int idx = tid; idx < NB * w; idx += blockDim.x) {
      const int r = idx % w, l = idx / w;
      Iv[l][r] = bp[(int64_t)l * ldp + (j0 - jp) + r];
    }
    if (tid < NB) Iv[tid][NB] = bp[(int64_t)tid * ldp + tid];   // d_l in the pad column
    __syncthreads();
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int r = idx % w, c = idx / w;
      if (r < c) continue;
      cpx<T> acc = F[c][r];
      for (int l = 0; l < NB; ++l) {
        const cpx<T> a = cmul(Iv[l][r], Iv[l][NB]);
        acc = cfma(cpx<T>{-a.re, -a.im}, Iv[l][c], acc);
      }
      F[c][r] = acc;
    }
  }
  __syncthreads();
  const T tiny = sizeof(T) == 4 ? T(1e-30) : T(1e-300);
  for (int j = 0; j < w; ++j) {
    const cpx<T> d = F[j][j];
    const T ad = fabs(d.re) + fabs(d.im);
    if (tid == 0) {
      if (!(ad > T(0)) || !isfinite(d.re) || !isfinite(d.im)) flags[0] = 1;
      else if (ad < tiny) atomicAdd(&flags[1], 1);
    }
    const cpx<T> inv = cinv(d);
    const int nt = w - j - 1;
    for (int idx = tid; idx < nt * nt; idx += blockDim.x) {
      const int rr = j + 1 + idx % nt, cc = j + 1 + idx / nt;
      if (cc <= rr) F[cc][rr] = csub(F[cc][rr], cmul(cmul(F[j][rr], inv), F[j][cc]));
    }
    __syncthreads();
    for (int r = j + 1 + tid; r < w; r += blockDim.x) F[j][r] = cmul(F[j][r], inv);
    __syncthreads();
  }
  // inverse of the unit lower triangular factor by column sweeps: after step
  // l entry l of every column c <= l is final and is eliminated from the
  // rows below it (Iv[c][r] is row r of column c of the inverse)
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    const int r = idx % w, c = idx / w;
    Iv[c][r] = (r == c) ? cpx<T>{T(1), T(0)} : czero<T>();
  }
  __syncthreads();
  for (int l = 0; l + 1 < w; ++l) {
    const int nr = w - l - 1;   // rows l+1 .. w-1 of columns 0 .. l
    for (int idx = tid; idx < (l + 1) * nr; idx += blockDim.x) {
      const int c = idx / nr, r = l + 1 + idx % nr;
      const cpx<T> a = F[l][r];
      Iv[c][r] = cfma(cpx<T>{-a.re, -a.im}, Iv[c][l], Iv[c][r]);
    }
    __syncthreads();
  }
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    const int r = idx % w, c = idx / w;
    // lower part (r >= c): L and D; upper (r < c): transpose of the inverse
    blk[(int64_t)c * ld + r] = (r >= c) ? F[c][r] : Iv[r][c];
  }
}

template <typename T>
hipError_t launch_panel_diag(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                             int j0, int jp, int npole, cpx<T> *factor, int64_t f_stride,
                             int *flags) {
  if (n_nodes <= 0) return hipSuccess;
  if (jp >= 0 && jp != j0 - NB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_panel_diag<T>, dim3(n_nodes, npole), dim3(256), 0, st, ft, lvl_nodes, j0,
                     jp, factor, f_stride, flags);
  return hipGetLastError();
}

// --------------------------------------------------------- panel rows
// Rows below the diagonal block: L[r, j] = (A[r, j] - sum_{l<j} L[r, l] d_l
// L[j, l]) / d_j, one row per thread.  With jp >= 0 (= j0 - NB) each row
// first takes the update of block jp: A[r, j] -= sum_l L[r, jp+l] d_l
// L[j, jp+l] (as in k_panel_diag).
template <typename T>
__global__ __launch_bounds__(256) void k_panel_trsm(FrontTab ft, const int32_t *lvl_nodes, int j0,
                                                    int jp, cpx<T> *factor, int64_t f_stride) {
  const int s = lvl_nodes[blockIdx.y];
  const int p = blockIdx.z;
  if (pole_absent(ft, s, p)) return;
  const int k = ft.k[s];
  if (j0 >= k) return;
  const int w = min(NB, k - j0);
  const int64_t n = (int64_t)k + ft.u[s];
  const int64_t ld = n - j0;
  cpx<T> *blk = factor + (int64_t)p * f_stride + ft.panel_off[s] + panel_block_off(n, j0 / NB);
  __shared__ cpx<T> W[NB][NB];    // W[j][l] = d_l L[j][l]
  __shared__ cpx<T> W2[NB][NB];   // W2[j][l] = d_l L[j0 + j][jp + l] (jp >= 0)
  __shared__ cpx<T> invd[NB];
  const int64_t ldp = n - jp;
  const cpx<T> *bp =
      jp >= 0 ? factor + (int64_t)p * f_stride + ft.panel_off[s] + panel_block_off(n, jp / NB)
              : nullptr;
  const int tid = threadIdx.x;
  const int64_t rloc0 = (int64_t)w + (int64_t)blockIdx.x * blockDim.x;  // block-local row
  if (rloc0 >= ld) return;
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    const int j = idx % w, l = idx / w;
    if (l < j) W[j][l] = cmul(blk[(int64_t)l * ld + l], blk[(int64_t)l * ld + j]);
  }
  if (tid < w) invd[tid] = cinv(blk[(int64_t)tid * ld + tid]);
  if (jp >= 0) {
    for (int idx = tid; idx < w * NB; idx += blockDim.x) {
      const int j = idx % w, l = idx / w;
      W2[j][l] = cmul(bp[(int64_t)l * ldp + l], bp[(int64_t)l * ldp + (j0 - jp) + j]);
    }
  }
  __syncthreads();
  const int64_t r = rloc0 + tid;
  if (r >= ld) return;
  cpx<T> x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < w) x[j] = blk[(int64_t)j * ld + r];
  if (jp >= 0) {
    // row r of block jp, one entry at a time
#pragma unroll 4
    for (int l = 0; l < NB; ++l) {
      const cpx<T> a = bp[(int64_t)l * ldp + (j0 - jp) + r];
      const cpx<T> na = {-a.re, -a.im};
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < w) x[j] = cfma(na, W2[j][l], x[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < w) {
      cpx<T> acc = x[j];
#pragma unroll
      for (int l = 0; l < NB; ++l)
        if (l < j) acc = cfma(cpx<T>{-x[l].re, -x[l].im}, W[j][l], acc);
      x[j] = cmul(acc, invd[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < w) blk[(int64_t)j * ld + r] = x[j];
}

template <typename T>
hipError_t launch_panel_trsm(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                             int j0, int jp, int max_rows, int npole, cpx<T> *factor,
                             int64_t f_stride) {
  if (n_nodes <= 0 || max_rows <= 0) return hipSuccess;
  if (jp >= 0 && jp != j0 - NB) return hipErrorInvalidValue;
  dim3 grid((max_rows + 255) / 256, n_nodes, npole);
  hipLaunchKernelGGL(k_panel_trsm<T>, grid, dim3(256), 0, st, ft, lvl_nodes, j0, jp, factor,
                     f_stride);
  return hipGetLastError();
}

// ------------------------------------------------------ MFMA tile update
// C -= L D L^T on the lower triangle.  TTS x TTS output tiles, 4 waves of
// (TTS/2) x (TTS/2); complex arithmetic as four real MFMAs per depth step on
// split real/imaginary planes staged through LDS; the next depth chunk is
// prefetched into registers while the current one is multiplied.
constexpr int KB = 16;   // depth chunk (divides NB)

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));


// Complex products.  The update is C -= A B^T with A = Ar + i Ai (rows of
// L) and B = Br + i Bi (rows of L D).  With M3 = false four real products
// accumulate Re = Ar Br^T - Ai Bi^T and Im = Ar Bi^T + Ai Br^T; with
// M3 = true three (the 3M method): P1 = Ar Br^T, P2 = Ai Bi^T,
// P3 = (Ar + Ai)(Br + Bi)^T, Re = P1 - P2, Im = P3 - P1 - P2.  The 3M form
// does a quarter fewer matrix-core products and its error stays normwise
// of the order of the unit roundoff (Higham, SIAM J. Matrix Anal. Appl. 13,
// 1992).  Accumulator q of a wave holds NBK x NBK MFMA blocks.
template <typename T>
struct Mfma;
// FP32: blocks of 32 x 32, v_mfma_f32_32x32x2f32 (depth 2 per product;
// operand lane l carries row l % 32, depth l / 32; result element i of lane
// l is row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32)
template <>
struct Mfma<float> {
  static constexpr int BS = 32, DK = 2, NV = 16;
  using acc_t = floatx16;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static void operand(int lane, int &r, int &k) {
    r = lane & 31;
    k = lane >> 5;
  }
  __device__ static void coord(int lane, int i, int &row, int &col) {
    row = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    col = lane & 31;
  }
};
// FP64: blocks of 16 x 16, v_mfma_f64_16x16x4f64 (depth 4; operand lane l
// carries row l % 16, depth l / 16; result element i of lane l is row
// l / 16 + 4 i, column l % 16)
template <>
struct Mfma<double> {
  static constexpr int BS = 16, DK = 4, NV = 4;
  using acc_t = doublex4;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static void operand(int lane, int &r, int &k) {
    r = lane & 15;
    k = lane >> 4;
  }
  __device__ static void coord(int lane, int i, int &row, int &col) {
    row = (lane >> 4) + 4 * i;
    col = lane & 15;
  }
};

template <typename T, int NBR, int NBC, bool M3>
struct WaveAcc {
  using F = Mfma<T>;
  static constexpr int NQ = M3 ? 3 : 2;
  typename F::acc_t q[NQ][NBR][NBC];
  __device__ void zero() {
#pragma unroll
    for (int z = 0; z < NQ; ++z)
#pragma unroll
      for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b)
#pragma unroll
          for (int i = 0; i < F::NV; ++i) q[z][a][b][i] = T(0);
  }
  // Ar, Ai: rows of L for the wave's NBR row blocks (from row ar0 of the LDS
  // planes of width TA); Br, Bi: rows of L for its NBC column blocks (from
  // row br0, width TB); Dr, Di: the pivots of the chunk, applied here
  template <int TA, int TB>
  __device__ void step(const T (*Ar)[TA], const T (*Ai)[TA], const T (*Br)[TB],
                       const T (*Bi)[TB], const T *Dr, const T *Di, int ar0, int br0,
                       int lane) {
    int rr, kh;
    F::operand(lane, rr, kh);
#pragma unroll
    for (int kk = 0; kk < KB; kk += F::DK) {
      T ar[NBR], ai[NBR], br[NBC], bi[NBC];
      const T dr = Dr[kk + kh], di = Di[kk + kh];
#pragma unroll
      for (int a = 0; a < NBR; ++a) {
        ar[a] = Ar[kk + kh][ar0 + a * F::BS + rr];
        ai[a] = Ai[kk + kh][ar0 + a * F::BS + rr];
      }
#pragma unroll
      for (int b = 0; b < NBC; ++b) {
        const T lr = Br[kk + kh][br0 + b * F::BS + rr];
        const T li = Bi[kk + kh][br0 + b * F::BS + rr];
        br[b] = lr * dr - li * di;
        bi[b] = lr * di + li * dr;
      }
#pragma unroll
      for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b) {
          if constexpr (M3) {
            q[0][a][b] = F::mma(ar[a], br[b], q[0][a][b]);
            q[1][a][b] = F::mma(ai[a], bi[b], q[1][a][b]);
            q[2][a][b] = F::mma(ar[a] + ai[a], br[b] + bi[b], q[2][a][b]);
          } else {
            q[0][a][b] = F::mma(-ar[a], br[b], q[0][a][b]);
            q[0][a][b] = F::mma(ai[a], bi[b], q[0][a][b]);
            q[1][a][b] = F::mma(-ar[a], bi[b], q[1][a][b]);
            q[1][a][b] = F::mma(-ai[a], br[b], q[1][a][b]);
          }
        }
    }
  }
  static constexpr int nelem() { return NBR * NBC * F::NV; }
  // element e of this lane -> (row, col) inside the wave's sub-tile
  __device__ static void coord(int lane, int e, int &row, int &col) {
    const int blk = e / F::NV, i = e % F::NV;
    F::coord(lane, i, row, col);
    row += (blk / NBC) * F::BS;
    col += (blk % NBC) * F::BS;
  }
  // the update's increment -A B^T at element e
  __device__ T get_re(int e) const {
    const int a = (e / F::NV) / NBC, b = (e / F::NV) % NBC, i = e % F::NV;
    if constexpr (M3)
      return q[1][a][b][i] - q[0][a][b][i];
    else
      return q[0][a][b][i];
  }
  __device__ T get_im(int e) const {
    const int a = (e / F::NV) / NBC, b = (e / F::NV) % NBC, i = e % F::NV;
    if constexpr (M3)
      return (q[0][a][b][i] + q[1][a][b][i]) - q[2][a][b][i];
    else
      return q[1][a][b][i];
  }
};

// Output tiles of TR rows x TC columns (TR = R TC, R = 1 or 2) over the lower
// trapezoid of columns [cbeg, cend) and rows [cbeg, n), on a row grid
// aligned to TR: tile (ct, rt) covers columns cbeg + TC ct .. and rows
// cbeg + TR rt .., and exists for floor(ct / R) <= rt < nrt, nrt =
// ceil((n - cbeg) / TR).  Numbering in super-column order: column tiles are
// grouped by SUPER_W; inside a group the tiles run by row tile, then column
// tile, so that the tiles in flight share row and column panels.  Returns
// false past the last tile.
constexpr int SUPER_W = 8;
template <int R>
__device__ inline bool trap_tile(int64_t id, int64_t nct, int64_t nrt, int64_t &ct,
                                 int64_t &rt) {
  for (int64_t c0 = 0; c0 < nct; c0 += SUPER_W) {
    const int64_t w = min((int64_t)SUPER_W, nct - c0);
    int64_t here = 0;
    for (int64_t c = c0; c < c0 + w; ++c) here += nrt - c / R;
    if (id >= here) {
      id -= here;
      continue;
    }
    // rows where only a prefix of the group's columns has reached the diagonal
    int64_t r = c0 / R;
    for (; r < nrt; ++r) {
      const int64_t act = min(w, R * (r + 1) - c0);
      if (act >= w) break;
      if (id < act) {
        ct = c0 + id;
        rt = r;
        return true;
      }
      id -= act;
    }
    ct = c0 + id % w;
    rt = r + id / w;
    return true;
  }
  return false;
}
template <int R>
__device__ inline int64_t trap_count(int64_t nct, int64_t nrt) {
  // nct * nrt - sum_{t < nct} floor(t / R), R = 1 or 2
  if (R == 1) return nct * nrt - nct * (nct - 1) / 2;
  const int64_t m = nct / 2;
  return nct * nrt - ((nct & 1) ? m * m : m * (m - 1));
}

// mode 0: depth (eliminated columns) [j0, j0 + dw), updated columns
// [j0 + dw, min(k, ccap)); mode 1: depth [0, k), contribution block.
// TR x TC output tile per workgroup, 4 waves of (TR/2) x (TC/2).
// Waves per SIMD the register allocation must allow: FP32 tiles of 64 x 64
// fit four (at most 128 registers, accumulators included) and tiles of
// 128 x 64 three, without spilling.
template <typename T, int TR, int TC>
constexpr int update_waves() {
  return sizeof(T) != 4 ? 1 : (TR == 64 && TC == 64) ? 4 : (TR == 128 && TC == 64) ? 3 : 1;
}
template <typename T, int TR, int TC, bool M3>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(update_waves<T, TR, TC>())))
void k_front_update(FrontTab ft, const int32_t *lvl_nodes,
                                                      int mode, int j0, int dw, int ccap,
                                                      cpx<T> *factor, int64_t f_stride,
                                                      cpx<T> *cb, int64_t cb_stride) {
  constexpr int R = TR / TC;
  using Acc = WaveAcc<T, TR / 2 / Mfma<T>::BS, TC / 2 / Mfma<T>::BS, M3>;
  const int s = lvl_nodes[blockIdx.y];
  const int p = blockIdx.z;
  if (pole_absent(ft, s, p)) return;
  const int64_t k = ft.k[s], u = ft.u[s], n = k + u;
  int64_t cbeg, cend, l0, l1;
  if (mode == 0) {
    cbeg = (int64_t)j0 + dw;
    cend = min(k, (int64_t)ccap);
    l0 = j0;
    l1 = min((int64_t)j0 + dw, k);
  } else {
    cbeg = k;
    cend = n;
    l0 = 0;
    l1 = k;
  }
  if (cbeg >= cend) return;
  if (mode == 0 && l0 >= l1) return;   // mode 1 with k = 0 writes zeros
  // Work split across the eight XCDs: the grid's x extent is a multiple of
  // 8, workgroups are handed to XCDs round robin, so x % 8 names the XCD and
  // each XCD takes one contiguous eighth of the tile sequence, walked in
  // super-column order so that the tiles in flight on an XCD share row and
  // column panels in its L2.
  const int64_t nct = (cend - cbeg + TC - 1) / TC, nrt = (n - cbeg + TR - 1) / TR;
  const int64_t cnt = trap_count<R>(nct, nrt);
  const int64_t chunk = (cnt + 7) / 8;
  const int64_t loc = blockIdx.x >> 3;
  if (loc >= chunk) return;
  const int64_t id = (int64_t)(blockIdx.x & 7) * chunk + loc;
  if (id >= cnt) return;
  int64_t ct, rt;
  if (!trap_tile<R>(id, nct, nrt, ct, rt)) return;
  const int64_t col0 = cbeg + TC * ct;
  const int64_t row0 = cbeg + TR * rt;
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];

  __shared__ T Ar[2][KB][TR], Ai[2][KB][TR], Br[2][KB][TC], Bi[2][KB][TC];
  __shared__ T Dr[2][KB], Di[2][KB];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the wave index is uniform: computed once on the scalar unit, so that
  // every depth offset below is scalar arithmetic and only the row offset
  // is per lane
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 1, wc = wave >> 1;
  constexpr int PA = TR * KB / 256, PB = TC * KB / 256;   // elements per thread and chunk
  static_assert(TR % 64 == 0 && TC % 64 == 0, "tiles are whole waves wide");
  const int lra = (wave % (TR / 64)) * 64 + lane, lka = (wave / (TR / 64)) * PA;
  const int lrb = (wave % (TC / 64)) * 64 + lane, lkb = (wave / (TC / 64)) * PB;
  // Prefetch of the next depth chunk: unconditional loads from clamped
  // (in-bounds) addresses, so nothing waits on them until the chunk is
  // written to LDS.  No value needs masking there: depth columns past l1
  // get the pivot D = 0, which zeroes their whole contribution (B = L D is
  // formed from the staged D), and rows past n only reach outputs that the
  // epilogue discards.  Clamped rows stay in the panel block: every row
  // index is >= cbeg >= l1.  Threads tid < KB also fetch the pivot of
  // depth column l + tid.
  cpx<T> pa[PA], pb[PB], pd;
  int64_t pl = l0;
  const int32_t rac = (int32_t)min(row0 + lra, n - 1), rbc = (int32_t)min(col0 + lrb, n - 1);
  const int32_t dl = tid % KB;
  auto fetch = [&](int64_t l) {
    const int64_t b = l / NB, r0 = NB * b, ldb = n - r0;
    const cpx<T> *base = P + panel_block_off(n, b) - r0;
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int64_t lc = min(l + lka + q, l1 - 1);
      pa[q] = (base + (lc - r0) * ldb)[rac];
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int64_t lc = min(l + lkb + q, l1 - 1);
      pb[q] = (base + (lc - r0) * ldb)[rbc];
    }
    const int32_t ld = (int32_t)min(l + dl, l1 - 1) - (int32_t)r0;   // 0 <= ld < NB
    pd = (base + r0)[__umul24((uint32_t)ld, (uint32_t)ldb + 1u)];
    pl = l;
  };
  // registers -> LDS buffer bf (columns past l1 get D = 0)
  auto stage = [&](int bf) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      Ar[bf][lka + q][lra] = pa[q].re;
      Ai[bf][lka + q][lra] = pa[q].im;
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      Br[bf][lkb + q][lrb] = pb[q].re;
      Bi[bf][lkb + q][lrb] = pb[q].im;
    }
    if (tid < KB) {
      const bool okd = pl + tid < l1;
      Dr[bf][tid] = okd ? pd.re : T(0);
      Di[bf][tid] = okd ? pd.im : T(0);
    }
  };
  // two LDS buffers: chunk i+1 is loaded while chunk i is multiplied, one
  // barrier per chunk
  Acc acc;
  acc.zero();
  if (l1 > l0) {
    fetch(l0);
    stage(0);
    __syncthreads();
    int bf = 0;
    for (int64_t l = l0; l < l1; l += KB) {
      const bool more = l + KB < l1;
      if (more) fetch(l + KB);
      acc.template step<TR, TC>(Ar[bf], Ai[bf], Br[bf], Bi[bf], Dr[bf], Di[bf], wr * (TR / 2),
                                wc * (TC / 2), lane);
      if (more) stage(bf ^ 1);
      __syncthreads();
      bf ^= 1;
    }
  }
  // epilogue on the lower triangle.  Mode 1 writes the contribution block
  // C = -L21 D L21^T (the children's parts are added after this update).
  // Mode 0 adds into the panel, four entries at a time: their loads are
  // issued together (entries outside the triangle read the tile's corner
  // (row0, col0), which always exists), then the valid ones are stored.
  cpx<T> *Cb = (mode == 1) ? cb + (int64_t)p * cb_stride + ft.cb_off[s] : nullptr;
  cpx<T> *Pw = factor + (int64_t)p * f_stride + ft.panel_off[s];
  constexpr int NE = Acc::nelem(), GE = 4;
  if (mode == 1) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      int rr, cc;
      Acc::coord(lane, e, rr, cc);
      const int64_t row = row0 + wr * (TR / 2) + rr, col = col0 + wc * (TC / 2) + cc;
      if (row >= n || col >= cend || row < col) continue;
      Cb[(col - k) * u + (row - k)] = {acc.get_re(e), acc.get_im(e)};
    }
    return;
  }
#pragma unroll
  for (int e0 = 0; e0 < NE; e0 += GE) {
    cpx<T> *qp[GE];
    bool ok[GE];
    cpx<T> cv[GE];
#pragma unroll
    for (int j = 0; j < GE; ++j) {
      int rr, cc;
      Acc::coord(lane, e0 + j, rr, cc);
      const int64_t row = row0 + wr * (TR / 2) + rr, col = col0 + wc * (TC / 2) + cc;
      ok[j] = !(row >= n || col >= cend || row < col);
      const int64_t r = ok[j] ? row : row0, c = ok[j] ? col : col0;
      qp[j] = Pw + panel_elem(n, r, c);
      cv[j] = *qp[j];
    }
#pragma unroll
    for (int j = 0; j < GE; ++j) {
      if (!ok[j]) continue;
      cpx<T> v = cv[j];
      v.re += acc.get_re(e0 + j);
      v.im += acc.get_im(e0 + j);
      *qp[j] = v;
    }
  }
}

template <typename T>
hipError_t launch_front_update(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                               int mode, int j0, int dw, int ccap, int64_t max_tiles, int npole,
                               cpx<T> *factor, int64_t f_stride, cpx<T> *cb, int64_t cb_stride,
                               int tile, bool m3) {
  if (n_nodes <= 0 || max_tiles <= 0) return hipSuccess;
  dim3 grid((unsigned)(8 * ((max_tiles + 7) / 8)), n_nodes, npole);
#define TEM_UPD(TR, TC, M)                                                                        \
  hipLaunchKernelGGL((k_front_update<T, TR, TC, M>), grid, dim3(256), 0, st, ft, lvl_nodes, mode, \
                     j0, dw, ccap, factor, f_stride, cb, cb_stride)
  if constexpr (sizeof(T) == 4) {
    if (tile == UPD_T128) {   // 4M only: the 3M accumulators do not fit beside it
      TEM_UPD(128, 128, false);
      return hipGetLastError();
    }
    if (tile == UPD_T128x64) {
      if (m3)
        TEM_UPD(128, 64, true);
      else
        TEM_UPD(128, 64, false);
      return hipGetLastError();
    }
  }
  if (tile != UPD_T64) return hipErrorInvalidValue;   // FP64 runs 64 x 64 tiles only
  if (m3)
    TEM_UPD(64, 64, true);
  else
    TEM_UPD(64, 64, false);
#undef TEM_UPD
  return hipGetLastError();
}

// --------------------------------------------------------- instantiation
#define TEM_INST(T)                                                                              \
  template hipError_t launch_fill_zero<T>(hipStream_t, cpx<T> *, int64_t, int, int64_t);         \
  template hipError_t launch_front_assemble<T>(hipStream_t, int64_t, const int32_t *,            \
                                               const int64_t *, const double *, const double *,  \
                                               const double *, Seg, int, cpx<T> *, int64_t);     \
  template hipError_t launch_extend_add<T>(hipStream_t, FrontTab, const int2 *, int64_t, int, int, \
                                           cpx<T> *, int64_t, cpx<T> *, cpx<T> *, int64_t);      \
  template hipError_t launch_panel_diag<T>(hipStream_t, FrontTab, const int32_t *, int, int, int, \
                                           int, cpx<T> *, int64_t, int *);                       \
  template hipError_t launch_panel_trsm<T>(hipStream_t, FrontTab, const int32_t *, int, int, int, \
                                           int, int, cpx<T> *, int64_t);                         \
  template hipError_t launch_front_update<T>(hipStream_t, FrontTab, const int32_t *, int, int,    \
                                             int, int, int, int64_t, int, cpx<T> *, int64_t,      \
                                             cpx<T> *, int64_t, int, bool);
TEM_INST(float)
TEM_INST(double)
#undef TEM_INST

}  // namespace tem
