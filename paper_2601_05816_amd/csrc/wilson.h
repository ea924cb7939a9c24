// Per-site Wilson hopping term on a block of right-hand sides.
//
// For one output site x and one rhs the kernels accumulate
//   hop(x) = sum_mu [ (1 - s gamma_mu) U_mu(x) psi(x+mu) + (1 + s gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
// with s = +1 for D and s = -1 for D^dagger (the adjoint of each hopping term
// flips the sign of gamma_mu), the quantity summed over directions in Algorithm 1.
// Each term is evaluated on a half spinor, as Sec. III-A.1 describes for the
// projected vectors lambda_mu and chi_mu: with psi = (u; d) in upper/lower
// spin pairs and gamma_mu = [[0, B], [B^dag, 0]],
//   (1 + t gamma_mu) psi = (h; t B^dag h),  h = u + t B d,
// so the colour matrix multiplies the 2x3 block h only (two 3x3-by-3 products
// instead of four) and the lower spins are rebuilt from the product.  Every
// B_mu has entries in {0, +-1, +-i}, so the projection is additions only.
#pragma once

#include "common.h"

namespace lq {

template <typename R>
struct spinor {
  cx<R> c[4][3];  // [spin][colour]
};
template <typename R>
struct half_spinor {
  cx<R> c[2][3];
};

// h = u + t B_mu d  (T = t = +-1)
template <int MU, int T, typename R>
__device__ __forceinline__ half_spinor<R> project(const spinor<R>& p) {
  half_spinor<R> h;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> u0 = p.c[0][a], u1 = p.c[1][a], d0 = p.c[2][a], d1 = p.c[3][a];
    cx<R> b0, b1;  // (B d)_0, (B d)_1
    if (MU == 0) { b0 = d0; b1 = d1; }                               // B_0 = 1
    if (MU == 1) { b0 = -mul_i(d1); b1 = -mul_i(d0); }               // B_1 = [[0,-i],[-i,0]]
    if (MU == 2) { b0 = -d1; b1 = d0; }                              // B_2 = [[0,-1],[1,0]]
    if (MU == 3) { b0 = -mul_i(d0); b1 = mul_i(d1); }                // B_3 = [[-i,0],[0,i]]
    if (T > 0) { h.c[0][a] = u0 + b0; h.c[1][a] = u1 + b1; }
    else       { h.c[0][a] = u0 - b0; h.c[1][a] = u1 - b1; }
  }
  return h;
}

// acc += (r; t B_mu^dag r)
template <int MU, int T, typename R>
__device__ __forceinline__ void reconstruct(spinor<R>& acc, const half_spinor<R>& r) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> r0 = r.c[0][a], r1 = r.c[1][a];
    cx<R> l0, l1;  // (B^dag r)_0, (B^dag r)_1
    if (MU == 0) { l0 = r0; l1 = r1; }
    if (MU == 1) { l0 = mul_i(r1); l1 = mul_i(r0); }
    if (MU == 2) { l0 = r1; l1 = -r0; }
    if (MU == 3) { l0 = mul_i(r0); l1 = -mul_i(r1); }
    acc.c[0][a] = acc.c[0][a] + r0;
    acc.c[1][a] = acc.c[1][a] + r1;
    if (T > 0) { acc.c[2][a] = acc.c[2][a] + l0; acc.c[3][a] = acc.c[3][a] + l1; }
    else       { acc.c[2][a] = acc.c[2][a] - l0; acc.c[3][a] = acc.c[3][a] - l1; }
  }
}

template <typename R>
struct su3 {
  cx<R> m[3][3];
};

template <typename S, typename R>
__device__ __forceinline__ su3<R> load_link(const S* __restrict__ u) {
  su3<R> a;
#pragma unroll
  for (int i = 0; i < 9; ++i) a.m[i / 3][i % 3] = ld(u + i);
  return a;
}

// r = U h (ADJ = false) or U^dag h (ADJ = true) for a link held in registers
template <bool ADJ, typename R>
__device__ __forceinline__ half_spinor<R> colour_mul_r(const su3<R>& u, const half_spinor<R>& h) {
  half_spinor<R> r;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> acc = {R(0), R(0)};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (ADJ) acc = cjmadd(acc, u.m[b][a], h.c[s][b]);
        else     acc = cmadd(acc, u.m[a][b], h.c[s][b]);
      }
      r.c[s][a] = acc;
    }
  }
  return r;
}

// r = U h (ADJ = false) or U^dag h (ADJ = true); U row-major 3x3 in memory.
template <bool ADJ, typename S, typename R>
__device__ __forceinline__ half_spinor<R> colour_mul(const S* __restrict__ u, const half_spinor<R>& h) {
  cx<R> m[3][3];
#pragma unroll
  for (int i = 0; i < 9; ++i) m[i / 3][i % 3] = ld(u + i);
  half_spinor<R> r;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> acc = {R(0), R(0)};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (ADJ) acc = cjmadd(acc, m[b][a], h.c[s][b]);
        else     acc = cmadd(acc, m[a][b], h.c[s][b]);
      }
      r.c[s][a] = acc;
    }
  }
  return r;
}

template <typename S, typename R>
__device__ __forceinline__ spinor<R> load_spinor(const S* __restrict__ p, size_t base, int cs) {
  spinor<R> v;
#pragma unroll
  for (int i = 0; i < 12; ++i) v.c[i / 3][i % 3] = ld(p + base + (size_t)i * cs);
  return v;
}

// A spinor as stored (12 storage elements, not yet widened), so that a
// kernel can issue its loads early and project it later.
template <typename S>
struct raw_spinor {
  S c[12];
};
template <typename S>
__device__ __forceinline__ raw_spinor<S> load_raw(const S* __restrict__ p, size_t base, int cs) {
  raw_spinor<S> v;
#pragma unroll
  for (int i = 0; i < 12; ++i) v.c[i] = p[base + (size_t)i * cs];
  return v;
}

// Half spinor h = u + t B_mu d of a stored spinor (project<MU, T> of the
// widened values).  `one` must be 1: for FP16 storage each entry of h is
// then one mixed-precision FMA, fma(d, +-one, u), on the FP16 values as
// loaded, which rounds exactly as the FP32 sum of the widened values but
// needs no conversions first (a run-time 1 keeps the compiler from folding
// the FMA back into an add of converted values).
template <int MU, int T, typename S, typename R>
__device__ __forceinline__ half_spinor<R> project_raw(const raw_spinor<S>& v, R one) {
  (void)one;
  spinor<R> w;
#pragma unroll
  for (int i = 0; i < 12; ++i) w.c[i / 3][i % 3] = widen(v.c[i]);
  return project<MU, T>(w);
}
template <int MU, int T>
__device__ __forceinline__ half_spinor<float> project_raw(const raw_spinor<h2_t>& v, float one) {
  const float s = T > 0 ? one : -one;
  auto mix = [](_Float16 a, float f, _Float16 b) { return __builtin_fmaf((float)a, f, (float)b); };
  half_spinor<float> h;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const h2_t u0 = v.c[a], u1 = v.c[3 + a], d0 = v.c[6 + a], d1 = v.c[9 + a];
    if (MU == 0) {  // B_0 d = (d0, d1)
      h.c[0][a] = {mix(d0.x, s, u0.x), mix(d0.y, s, u0.y)};
      h.c[1][a] = {mix(d1.x, s, u1.x), mix(d1.y, s, u1.y)};
    }
    if (MU == 1) {  // B_1 d = (-i d1, -i d0)
      h.c[0][a] = {mix(d1.y, s, u0.x), mix(d1.x, -s, u0.y)};
      h.c[1][a] = {mix(d0.y, s, u1.x), mix(d0.x, -s, u1.y)};
    }
    if (MU == 2) {  // B_2 d = (-d1, d0)
      h.c[0][a] = {mix(d1.x, -s, u0.x), mix(d1.y, -s, u0.y)};
      h.c[1][a] = {mix(d0.x, s, u1.x), mix(d0.y, s, u1.y)};
    }
    if (MU == 3) {  // B_3 d = (-i d0, i d1)
      h.c[0][a] = {mix(d0.y, s, u0.x), mix(d0.x, -s, u0.y)};
      h.c[1][a] = {mix(d1.y, -s, u1.x), mix(d1.x, s, u1.y)};
    }
  }
  return h;
}

// the projected neighbour straight from storage
template <int MU, int T, typename S, typename R>
__device__ __forceinline__ half_spinor<R> load_project(const S* __restrict__ p, size_t base, int cs, R one) {
  return project_raw<MU, T>(load_raw(p, base, cs), one);
}

template <typename S, typename R>
__device__ __forceinline__ void store_spinor(S* __restrict__ p, size_t base, int cs, const spinor<R>& v) {
#pragma unroll
  for (int i = 0; i < 12; ++i) st(p + base + (size_t)i * cs, v.c[i / 3][i % 3]);
}

// Same, with non-temporal stores: the output is not read again by the
// kernel, so it should not displace reusable neighbour spinors from L2.
template <typename S, typename R>
__device__ __forceinline__ void store_spinor_nt(S* __restrict__ p, size_t base, int cs, const spinor<R>& v) {
#pragma unroll
  for (int i = 0; i < 12; ++i) st_nt(p + base + (size_t)i * cs, v.c[i / 3][i % 3]);
}

// One direction mu: forward neighbour (block offset fb, link U_mu(x) at uf)
// and backward neighbour (block offset bb, link U_mu(x-mu) at ub).
// SG = +1 for D, -1 for D^dagger.
template <int MU, int SG, typename S, typename R>
__device__ __forceinline__ void hop_dir(spinor<R>& acc, const S* __restrict__ psi, int cs, size_t fb,
                                        size_t bb, const S* __restrict__ uf, const S* __restrict__ ub) {
  {
    spinor<R> p = load_spinor<S, R>(psi, fb, cs);
    half_spinor<R> h = project<MU, -SG>(p);
    reconstruct<MU, -SG>(acc, colour_mul<false>(uf, h));
  }
  {
    spinor<R> p = load_spinor<S, R>(psi, bb, cs);
    half_spinor<R> h = project<MU, SG>(p);
    reconstruct<MU, SG>(acc, colour_mul<true>(ub, h));
  }
}

}  // namespace lq
