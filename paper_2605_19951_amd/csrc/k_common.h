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
// acc + a*b for a real a
template <typename T>
__device__ __forceinline__ cpx<T> rfma(T a, cpx<T> b, cpx<T> acc) {
  acc.re = fma(a, b.re, acc.re);
  acc.im = fma(a, b.im, acc.im);
  return acc;
}
// factor entries as the register triangle kernels keep them: complex, or
// the real part alone when the factor is real (its imaginary parts zero)
template <typename T, bool RL>
struct FacVal {
  typedef cpx<T> type;
  __device__ static type of(cpx<T> v) { return v; }
  __device__ static cpx<T> as_cpx(type v) { return v; }
  __device__ static type neg(type v) { return {-v.re, -v.im}; }
  __device__ static cpx<T> fma_(type a, cpx<T> b, cpx<T> acc) { return cfma(a, b, acc); }
};
template <typename T>
struct FacVal<T, true> {
  typedef T type;
  __device__ static type of(cpx<T> v) { return v.re; }
  __device__ static cpx<T> as_cpx(type v) { return {v, T(0)}; }
  __device__ static type neg(type v) { return -v; }
  __device__ static cpx<T> fma_(type a, cpx<T> b, cpx<T> acc) { return rfma(a, b, acc); }
};
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
