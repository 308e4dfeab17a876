// Device helpers shared by the HIP kernel files.
#pragma once

#include "tem_internal.h"

namespace tem {

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
// acc + a*b
template <typename T>
__device__ __forceinline__ cpx<T> cfma(cpx<T> a, cpx<T> b, cpx<T> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
template <typename T>
__device__ __forceinline__ cpx<T> cinv(cpx<T> a) {
  T den = a.re * a.re + a.im * a.im;
  return {a.re / den, -a.im / den};
}
template <typename T>
__device__ __forceinline__ cpx<T> czero() {
  return {T(0), T(0)};
}

// segment of index i (0 for a single mesh)
__device__ __forceinline__ int seg_find(const Seg &sg, int64_t i) {
  if (sg.n <= 1) return 0;
  int lo = 0, hi = sg.n - 1;   // largest b with off[b] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sg.off[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}
// pole slot p of front s is padding (nothing to compute)
__device__ __forceinline__ bool pole_absent(const FrontTab &ft, int s, int p) {
  return ft.np && ft.p0 + p >= ft.np[s];
}

// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS operations (lgkmcnt 0) but not for its global loads and stores,
// which __syncthreads (a workgroup release fence) would drain, so that loads
// issued ahead stay in flight across the barrier.  Not a fence for global
// memory: threads must not exchange data through it across this barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xc07f);   // vmcnt 63, expcnt 7, lgkmcnt 0
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

inline unsigned grid_1d(int64_t n, int block, int64_t cap = 65535 * 16) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace tem
