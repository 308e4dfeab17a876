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
// factor[pole][pos[i]] = K[csr[i]] - xi_pole * M[csr[i]]
template <typename T>
__global__ void k_front_assemble(int64_t n, const int32_t *csr, const int64_t *pos,
                                 const double *Kv, const double *Mv, const double *xi,
                                 cpx<T> *factor, int64_t pole_stride) {
  const int p = blockIdx.y;
  const double xr = xi[2 * p], xim = xi[2 * p + 1];
  cpx<T> *F = factor + (int64_t)p * pole_stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = csr[i];
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
                                 const double *xi, int npole, cpx<T> *factor,
                                 int64_t pole_stride) {
  if (n_entries <= 0) return hipSuccess;
  dim3 grid(grid_1d(n_entries, 256, 8192), npole);
  hipLaunchKernelGGL(k_front_assemble<T>, grid, dim3(256), 0, st, n_entries, csr, pos, Kv, Mv,
                     xi, factor, pole_stride);
  return hipGetLastError();
}

// ----------------------------------------------------------- extend-add
// Adds the lower triangle of child `slot`'s contribution block into the
// parent front through the relative row map.  One slot per launch keeps the
// scatter free of races (two children may hit the same parent entry).
template <typename T>
__global__ void k_extend_add(FrontTab ft, const int32_t *lvl_nodes, int slot, cpx<T> *factor,
                             int64_t f_stride, cpx<T> *cb_par, cpx<T> *cb_ch,
                             int64_t cb_stride) {
  const int s = lvl_nodes[blockIdx.y];
  const int p = blockIdx.z;
  const int ch = slot == 0 ? ft.child0[s] : ft.child1[s];
  if (ch < 0) return;
  const int64_t uc = ft.u[ch];
  const int64_t cnt = uc * uc;
  const int64_t kp = ft.k[s], up = ft.u[s], np = kp + up;
  const int32_t *rel = ft.rel + ft.rows_off[ch];
  const cpx<T> *src = cb_ch + (int64_t)p * cb_stride + ft.cb_off[ch];
  cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];
  cpx<T> *C = cb_par + (int64_t)p * cb_stride + ft.cb_off[s];
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < cnt;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = idx % uc, b = idx / uc;
    if (a < b) continue;
    const int64_t ra = rel[a], rb = rel[b];
    const cpx<T> v = src[idx];
    if (rb < kp) {
      cpx<T> *q = P + panel_elem(np, ra, rb);
      *q = cadd(*q, v);
    } else {
      cpx<T> *q = C + (rb - kp) * up + (ra - kp);
      *q = cadd(*q, v);
    }
  }
}

template <typename T>
hipError_t launch_extend_add(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                             int slot, int max_u_child, int npole, cpx<T> *factor,
                             int64_t f_stride, cpx<T> *cb_parent, cpx<T> *cb_child,
                             int64_t cb_stride) {
  if (n_nodes <= 0 || max_u_child <= 0) return hipSuccess;
  int64_t cnt = (int64_t)max_u_child * max_u_child;
  dim3 grid(grid_1d(cnt, 256, 2048), n_nodes, npole);
  hipLaunchKernelGGL(k_extend_add<T>, grid, dim3(256), 0, st, ft, lvl_nodes, slot, factor,
                     f_stride, cb_parent, cb_child, cb_stride);
  return hipGetLastError();
}

// -------------------------------------------------------- panel diagonal
// LDL^T (no pivoting) of the NB x NB diagonal block of column block j0/NB,
// then the inverse of its unit-lower factor, stored transposed in the
// strictly upper part of the block.  flags[0] |= 1 on a zero or non-finite
// pivot; flags[1] counts tiny pivots.
template <typename T>
__global__ __launch_bounds__(256) void k_panel_diag(FrontTab ft, const int32_t *lvl_nodes, int j0,
                                                    cpx<T> *factor, int64_t f_stride,
                                                    int *flags) {
  const int s = lvl_nodes[blockIdx.x];
  const int p = blockIdx.y;
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
  // inverse of the unit lower triangular factor, one column per thread
  if (tid < w) {
    const int c = tid;
    for (int r = 0; r < w; ++r) Iv[c][r] = czero<T>();
    Iv[c][c] = {T(1), T(0)};
    for (int r = c + 1; r < w; ++r) {
      cpx<T> acc = czero<T>();
      for (int l = c; l < r; ++l) acc = cfma(F[l][r], Iv[c][l], acc);
      Iv[c][r] = {-acc.re, -acc.im};
    }
  }
  __syncthreads();
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    const int r = idx % w, c = idx / w;
    // lower part (r >= c): L and D; upper (r < c): transpose of the inverse
    blk[(int64_t)c * ld + r] = (r >= c) ? F[c][r] : Iv[r][c];
  }
}

template <typename T>
hipError_t launch_panel_diag(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                             int j0, int npole, cpx<T> *factor, int64_t f_stride, int *flags) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_panel_diag<T>, dim3(n_nodes, npole), dim3(256), 0, st, ft, lvl_nodes, j0,
                     factor, f_stride, flags);
  return hipGetLastError();
}

// --------------------------------------------------------- panel rows
// Rows below the diagonal block: L[r, j] = (A[r, j] - sum_{l<j} L[r, l] d_l
// L[j, l]) / d_j, one row per thread.
template <typename T>
__global__ __launch_bounds__(256) void k_panel_trsm(FrontTab ft, const int32_t *lvl_nodes, int j0,
                                                    cpx<T> *factor, int64_t f_stride) {
  const int s = lvl_nodes[blockIdx.y];
  const int p = blockIdx.z;
  const int k = ft.k[s];
  if (j0 >= k) return;
  const int w = min(NB, k - j0);
  const int64_t n = (int64_t)k + ft.u[s];
  const int64_t ld = n - j0;
  cpx<T> *blk = factor + (int64_t)p * f_stride + ft.panel_off[s] + panel_block_off(n, j0 / NB);
  __shared__ cpx<T> W[NB][NB];   // W[j][l] = d_l L[j][l]
  __shared__ cpx<T> invd[NB];
  const int tid = threadIdx.x;
  const int64_t rloc0 = (int64_t)w + (int64_t)blockIdx.x * blockDim.x;  // block-local row
  if (rloc0 >= ld) return;
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    const int j = idx % w, l = idx / w;
    if (l < j) W[j][l] = cmul(blk[(int64_t)l * ld + l], blk[(int64_t)l * ld + j]);
  }
  if (tid < w) invd[tid] = cinv(blk[(int64_t)tid * ld + tid]);
  __syncthreads();
  const int64_t r = rloc0 + tid;
  if (r >= ld) return;
  cpx<T> x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < w) x[j] = blk[(int64_t)j * ld + r];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < w) {
      cpx<T> acc = x[j];
#pragma unroll
      for (int l = 0; l < NB; ++l)
        if (l < j) acc = csub(acc, cmul(x[l], W[j][l]));
      x[j] = cmul(acc, invd[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < w) blk[(int64_t)j * ld + r] = x[j];
}

template <typename T>
hipError_t launch_panel_trsm(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                             int j0, int max_rows, int npole, cpx<T> *factor, int64_t f_stride) {
  if (n_nodes <= 0 || max_rows <= 0) return hipSuccess;
  dim3 grid((max_rows + 255) / 256, n_nodes, npole);
  hipLaunchKernelGGL(k_panel_trsm<T>, grid, dim3(256), 0, st, ft, lvl_nodes, j0, factor,
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

template <typename T, int TTS>
struct WaveAcc;

// FP32: blocks of 32 x 32 (v_mfma_f32_32x32x2f32), NBK x NBK blocks per wave
template <int TTS>
struct WaveAcc<float, TTS> {
  static constexpr int NBK = TTS / 64;
  floatx16 re[NBK][NBK], im[NBK][NBK];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < NBK; ++a)
#pragma unroll
      for (int b = 0; b < NBK; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          re[a][b][i] = 0.f;
          im[a][b][i] = 0.f;
        }
  }
  __device__ void step(const float (*Ar)[TTS], const float (*Ai)[TTS], const float (*Br)[TTS],
                       const float (*Bi)[TTS], int wr, int wc, int lane) {
    const int rr = lane & 31, kh = lane >> 5;
#pragma unroll
    for (int kk = 0; kk < KB; kk += 2) {
      float ar[NBK], ai[NBK], br[NBK], bi[NBK];
#pragma unroll
      for (int a = 0; a < NBK; ++a) {
        ar[a] = Ar[kk + kh][wr * (TTS / 2) + a * 32 + rr];
        ai[a] = Ai[kk + kh][wr * (TTS / 2) + a * 32 + rr];
        br[a] = Br[kk + kh][wc * (TTS / 2) + a * 32 + rr];
        bi[a] = Bi[kk + kh][wc * (TTS / 2) + a * 32 + rr];
      }
#pragma unroll
      for (int a = 0; a < NBK; ++a)
#pragma unroll
        for (int b = 0; b < NBK; ++b) {
          re[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ar[a], br[b], re[a][b], 0, 0, 0);
          re[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[a], bi[b], re[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ar[a], bi[b], im[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai[a], br[b], im[a][b], 0, 0, 0);
        }
    }
  }
  static constexpr int nelem() { return NBK * NBK * 16; }
  // element e of this lane -> (row, col) inside the wave's tile
  __device__ static void coord(int lane, int e, int &row, int &col) {
    const int blk = e >> 4, i = e & 15;
    const int a = blk / NBK, b = blk % NBK;
    row = a * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    col = b * 32 + (lane & 31);
  }
  __device__ float get_re(int e) const { return re[(e >> 4) / NBK][(e >> 4) % NBK][e & 15]; }
  __device__ float get_im(int e) const { return im[(e >> 4) / NBK][(e >> 4) % NBK][e & 15]; }
};

// FP64: blocks of 16 x 16 (v_mfma_f64_16x16x4f64), NBK x NBK blocks per wave
template <int TTS>
struct WaveAcc<double, TTS> {
  static constexpr int NBK = TTS / 32;
  doublex4 re[NBK][NBK], im[NBK][NBK];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < NBK; ++a)
#pragma unroll
      for (int b = 0; b < NBK; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          re[a][b][i] = 0.0;
          im[a][b][i] = 0.0;
        }
  }
  __device__ void step(const double (*Ar)[TTS], const double (*Ai)[TTS], const double (*Br)[TTS],
                       const double (*Bi)[TTS], int wr, int wc, int lane) {
    const int rr = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4) {
      double ar[NBK], ai[NBK], br[NBK], bi[NBK];
#pragma unroll
      for (int a = 0; a < NBK; ++a) {
        ar[a] = Ar[kk + kq][wr * (TTS / 2) + a * 16 + rr];
        ai[a] = Ai[kk + kq][wr * (TTS / 2) + a * 16 + rr];
        br[a] = Br[kk + kq][wc * (TTS / 2) + a * 16 + rr];
        bi[a] = Bi[kk + kq][wc * (TTS / 2) + a * 16 + rr];
      }
#pragma unroll
      for (int a = 0; a < NBK; ++a)
#pragma unroll
        for (int b = 0; b < NBK; ++b) {
          re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar[a], br[b], re[a][b], 0, 0, 0);
          re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], re[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar[a], bi[b], im[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[a], br[b], im[a][b], 0, 0, 0);
        }
    }
  }
  static constexpr int nelem() { return NBK * NBK * 4; }
  __device__ static void coord(int lane, int e, int &row, int &col) {
    const int blk = e >> 2, i = e & 3;
    const int a = blk / NBK, b = blk % NBK;
    row = a * 16 + (lane >> 4) + 4 * i;   // f64 16x16x4 result: row lane/16 + 4i
    col = b * 16 + (lane & 15);
  }
  __device__ double get_re(int e) const { return re[(e >> 2) / NBK][(e >> 2) % NBK][e & 3]; }
  __device__ double get_im(int e) const { return im[(e >> 2) / NBK][(e >> 2) % NBK][e & 3]; }
};

// mode 0: depth (eliminated columns) [j0, j0 + dw), updated columns
// [j0 + dw, min(k, ccap)); mode 1: depth [0, k), contribution block.
template <typename T, int TTS>
__global__ __launch_bounds__(256) void k_front_update(FrontTab ft, const int32_t *lvl_nodes,
                                                      int mode, int j0, int dw, int ccap,
                                                      cpx<T> *factor, int64_t f_stride,
                                                      cpx<T> *cb, int64_t cb_stride) {
  const int s = lvl_nodes[blockIdx.y];
  const int p = blockIdx.z;
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
  if (cbeg >= cend || l0 >= l1) return;
  // linear tile id -> (column tile, row tile) over the lower trapezoid
  int64_t t = blockIdx.x;
  const int64_t nct = (cend - cbeg + TTS - 1) / TTS;
  int64_t ct = 0;
  for (; ct < nct; ++ct) {
    const int64_t cnt = (n - (cbeg + TTS * ct) + TTS - 1) / TTS;
    if (t < cnt) break;
    t -= cnt;
  }
  if (ct >= nct) return;
  const int64_t col0 = cbeg + TTS * ct;
  const int64_t row0 = col0 + TTS * t;
  const cpx<T> *P = factor + (int64_t)p * f_stride + ft.panel_off[s];

  __shared__ T Ar[KB][TTS], Ai[KB][TTS], Br[KB][TTS], Bi[KB][TTS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  constexpr int PER = TTS * KB / 256;   // elements of A (and of B) per thread and chunk
  const int lr = tid % TTS;             // tile row this thread loads
  const int lk = (tid / TTS) * PER;     // first depth column it loads
  cpx<T> pa[PER], pb[PER];
  auto fetch = [&](int64_t l) {
    const int64_t b = l / NB, r0 = NB * b, ldb = n - r0;
    const cpx<T> *base = P + panel_block_off(n, b);
    const int64_t ra = row0 + lr, rb = col0 + lr;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int64_t lc = l + lk + q;
      cpx<T> a = czero<T>(), bb = czero<T>();
      if (lc < l1) {
        const cpx<T> *colp = base + (lc - r0) * ldb - r0;
        if (ra < n) a = colp[ra];
        if (rb < n) bb = cmul(colp[rb], colp[lc]);
      }
      pa[q] = a;
      pb[q] = bb;
    }
  };
  WaveAcc<T, TTS> acc;
  acc.zero();
  fetch(l0);
  for (int64_t l = l0; l < l1; l += KB) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      Ar[lk + q][lr] = pa[q].re;
      Ai[lk + q][lr] = pa[q].im;
      Br[lk + q][lr] = pb[q].re;
      Bi[lk + q][lr] = pb[q].im;
    }
    __syncthreads();
    if (l + KB < l1) fetch(l + KB);
    acc.step(Ar, Ai, Br, Bi, wr, wc, lane);
  }
  // epilogue: C += acc on the lower triangle
  cpx<T> *Cb = (mode == 1) ? cb + (int64_t)p * cb_stride + ft.cb_off[s] : nullptr;
  cpx<T> *Pw = factor + (int64_t)p * f_stride + ft.panel_off[s];
#pragma unroll
  for (int e = 0; e < WaveAcc<T, TTS>::nelem(); ++e) {
    int rr, cc;
    WaveAcc<T, TTS>::coord(lane, e, rr, cc);
    const int64_t row = row0 + wr * (TTS / 2) + rr, col = col0 + wc * (TTS / 2) + cc;
    if (row >= n || col >= cend || row < col) continue;
    cpx<T> *q = (mode == 1) ? Cb + (col - k) * u + (row - k) : Pw + panel_elem(n, row, col);
    cpx<T> v = *q;
    v.re += acc.get_re(e);
    v.im += acc.get_im(e);
    *q = v;
  }
}

template <typename T>
hipError_t launch_front_update(hipStream_t st, FrontTab ft, const int32_t *lvl_nodes, int n_nodes,
                               int mode, int j0, int dw, int ccap, int64_t max_tiles, int npole,
                               cpx<T> *factor, int64_t f_stride, cpx<T> *cb, int64_t cb_stride,
                               int tile) {
  if (n_nodes <= 0 || max_tiles <= 0) return hipSuccess;
  dim3 grid((unsigned)max_tiles, n_nodes, npole);
  if (tile == 128)
    hipLaunchKernelGGL((k_front_update<T, 128>), grid, dim3(256), 0, st, ft, lvl_nodes, mode, j0,
                       dw, ccap, factor, f_stride, cb, cb_stride);
  else
    hipLaunchKernelGGL((k_front_update<T, 64>), grid, dim3(256), 0, st, ft, lvl_nodes, mode, j0,
                       dw, ccap, factor, f_stride, cb, cb_stride);
  return hipGetLastError();
}

// --------------------------------------------------------- instantiation
#define TEM_INST(T)                                                                              \
  template hipError_t launch_fill_zero<T>(hipStream_t, cpx<T> *, int64_t, int, int64_t);         \
  template hipError_t launch_front_assemble<T>(hipStream_t, int64_t, const int32_t *,            \
                                               const int64_t *, const double *, const double *,  \
                                               const double *, int, cpx<T> *, int64_t);          \
  template hipError_t launch_extend_add<T>(hipStream_t, FrontTab, const int32_t *, int, int, int, \
                                           int, cpx<T> *, int64_t, cpx<T> *, cpx<T> *, int64_t);  \
  template hipError_t launch_panel_diag<T>(hipStream_t, FrontTab, const int32_t *, int, int, int, \
                                           cpx<T> *, int64_t, int *);                            \
  template hipError_t launch_panel_trsm<T>(hipStream_t, FrontTab, const int32_t *, int, int, int, \
                                           int, cpx<T> *, int64_t);                              \
  template hipError_t launch_front_update<T>(hipStream_t, FrontTab, const int32_t *, int, int,    \
                                             int, int, int, int64_t, int, cpx<T> *, int64_t,      \
                                             cpx<T> *, int64_t, int);
TEM_INST(float)
TEM_INST(double)
#undef TEM_INST

}  // namespace tem
