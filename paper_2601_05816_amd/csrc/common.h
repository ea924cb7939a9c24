// Shared device/host helpers: complex storage types, precision traits, spinor
// block addressing for the three layouts, XCD-aware block mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lqcd.h"

namespace lq {

// ---------------------------------------------------------------- complex ---
template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
// multiply by +i
template <typename R>
__device__ __forceinline__ cx<R> mul_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__device__ __forceinline__ cx<R> scale(R s, cx<R> a) { return {s * a.re, s * a.im}; }
// acc += a * b
template <typename R>
__device__ __forceinline__ cx<R> cmadd(cx<R> acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// acc += conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cjmadd(cx<R> acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}

// ------------------------------------------------------ precision traits ---
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

template <int PREC>
struct prec_traits;
template <>
struct prec_traits<LQCD_F64> {
  typedef double2 store;   // one complex number in memory
  typedef double real;     // arithmetic type
};
template <>
struct prec_traits<LQCD_F32> {
  typedef float2 store;
  typedef float real;
};
template <>
struct prec_traits<LQCD_F16> {
  typedef h2_t store;
  typedef float real;
};

__device__ __forceinline__ cx<double> ld(const double2* p) {
  double2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ cx<float> ld(const float2* p) {
  float2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ cx<float> ld(const h2_t* p) {
  h2_t v = *p;
  return {(float)v.x, (float)v.y};
}
// the same for a value already in registers
__device__ __forceinline__ cx<double> widen(double2 v) { return {v.x, v.y}; }
__device__ __forceinline__ cx<float> widen(float2 v) { return {v.x, v.y}; }
__device__ __forceinline__ cx<float> widen(h2_t v) { return {(float)v.x, (float)v.y}; }
__device__ __forceinline__ void st(double2* p, cx<double> a) { *p = make_double2(a.re, a.im); }
__device__ __forceinline__ void st(float2* p, cx<float> a) { *p = make_float2(a.re, a.im); }
__device__ __forceinline__ void st(h2_t* p, cx<float> a) {
  h2_t v;
  v.x = (_Float16)a.re;
  v.y = (_Float16)a.im;
  *p = v;
}

typedef double d2v_t __attribute__((ext_vector_type(2)));
typedef float f2v_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_nt(double2* p, cx<double> a) {
  d2v_t v = {a.re, a.im};
  __builtin_nontemporal_store(v, (d2v_t*)p);
}
__device__ __forceinline__ void st_nt(float2* p, cx<float> a) {
  f2v_t v = {a.re, a.im};
  __builtin_nontemporal_store(v, (f2v_t*)p);
}
__device__ __forceinline__ void st_nt(h2_t* p, cx<float> a) {
  h2_t v;
  v.x = (_Float16)a.re;
  v.y = (_Float16)a.im;
  __builtin_nontemporal_store(v, p);
}

// NR consecutive complex numbers (consecutive rhs of one component) with
// one vector access: FP32 x 2 = 16 B, FP16 x 2 = 8 B, FP16 x 4 = 16 B.
typedef float f4v_t __attribute__((ext_vector_type(4)));
typedef _Float16 h4v_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8v_t __attribute__((ext_vector_type(8)));

template <int NR>
__device__ __forceinline__ void ldn(const double2* p, cx<double>* o) {
#pragma unroll
  for (int r = 0; r < NR; ++r) o[r] = ld(p + r);
}
template <int NR>
__device__ __forceinline__ void ldn(const float2* p, cx<float>* o) {
  if (NR == 2) {
    const f4v_t v = *(const f4v_t*)p;
    o[0] = {v.x, v.y};
    o[1] = {v.z, v.w};
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) o[r] = ld(p + r);
  }
}
template <int NR>
__device__ __forceinline__ void ldn(const h2_t* p, cx<float>* o) {
  if (NR == 2) {
    const h4v_t v = *(const h4v_t*)p;
    o[0] = {(float)v[0], (float)v[1]};
    o[1] = {(float)v[2], (float)v[3]};
  } else if (NR == 4) {
    const h8v_t v = *(const h8v_t*)p;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = {(float)v[2 * r], (float)v[2 * r + 1]};
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) o[r] = ld(p + r);
  }
}
template <int NR>
__device__ __forceinline__ void stn(double2* p, const cx<double>* o) {
#pragma unroll
  for (int r = 0; r < NR; ++r) st(p + r, o[r]);
}
template <int NR>
__device__ __forceinline__ void stn(float2* p, const cx<float>* o) {
  if (NR == 2) {
    f4v_t v = {o[0].re, o[0].im, o[1].re, o[1].im};
    *(f4v_t*)p = v;
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) st(p + r, o[r]);
  }
}
template <int NR>
__device__ __forceinline__ void stn(h2_t* p, const cx<float>* o) {
  if (NR == 2) {
    h4v_t v = {(_Float16)o[0].re, (_Float16)o[0].im, (_Float16)o[1].re, (_Float16)o[1].im};
    *(h4v_t*)p = v;
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) st(p + r, o[r]);
  }
}

// ---------------------------------------------------------- block layout ---
// Element (site, comp, rhs) of a spinor block with `nsites` sites, 12
// components per site and nrhs right-hand sides.
template <int LAYOUT>
struct blk {
  // offset of component 0 of (site, rhs)
  __device__ __forceinline__ static size_t base(size_t site, int rhs, size_t nsites, int nrhs) {
    if (LAYOUT == LQCD_LAYOUT2) return site * 12u * (size_t)nrhs + (size_t)rhs;
    if (LAYOUT == LQCD_LAYOUT1) return (site * (size_t)nrhs + (size_t)rhs) * 12u;
    return ((size_t)rhs * nsites + site) * 12u;  // LQCD_RHS_OUTER
  }
  __device__ __forceinline__ static int cstride(int nrhs) { return LAYOUT == LQCD_LAYOUT2 ? nrhs : 1; }
  // work item t -> (site, rhs): the rhs index runs fastest where it is the
  // innermost memory index, the site index otherwise.
  __device__ __forceinline__ static void item(size_t t, size_t nsites, int nrhs, size_t& site, int& rhs) {
    if (LAYOUT == LQCD_RHS_OUTER) {
      rhs = (int)(t / nsites);
      site = t - (size_t)rhs * nsites;
    } else {
      site = t / (size_t)nrhs;
      rhs = (int)(t - site * (size_t)nrhs);
    }
  }
};

// Consecutive workgroups are dispatched round-robin over the 8 XCDs, each
// with a private L2.  Renumber so that XCD k processes a contiguous range of
// the logical block space (a bijection for any grid size).
__device__ __forceinline__ unsigned xcd_block(unsigned bid, unsigned nblk) {
  const unsigned nx = 8;
  unsigned q = nblk / nx, r = nblk % nx;
  unsigned k = bid % nx, i = bid / nx;
  return k * q + (k < r ? k : r) + i;
}

// Sum of x over the lanes of this wavefront that hold the same rhs group
// (lanes congruent modulo G, G a power of two dividing 64), left in lanes
// 0..G-1: a butterfly over lane distances 32, 16, ..., G, in a fixed order.
__device__ __forceinline__ cx<double> wave_group_sum(cx<double> x, int G) {
  for (int s = 32; s >= G; s >>= 1) {
    x.re += __shfl_xor(x.re, s);
    x.im += __shfl_xor(x.im, s);
  }
  return x;
}

// True when an activity mask is given and no rhs of the block is active (a
// lattice of a lock-step batch whose rhs have all converged): the BLAS
// kernels then return at once; their partial sums are only read for active
// rhs.
__device__ __forceinline__ bool none_live(const int* __restrict__ live, int nrhs) {
  if (!live) return false;
  for (int r = 0; r < nrhs; ++r)
    if (live[r]) return false;
  return true;
}

}  // namespace lq
