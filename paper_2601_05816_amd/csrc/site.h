// One-(site, rhs) bodies of the Wilson kernels, shared by the per-lattice
// kernels (dslash.hip) and the persistent batch kernel (batch.hip).
#pragma once

#include "clover.h"
#include "wilson.h"

namespace lq {

struct geo4 {
  int n[4];
  size_t V;
};

inline geo4 make_geo(const lqcd_lattice* lat) {
  geo4 g;
  for (int i = 0; i < 4; ++i) g.n[i] = lat->dims[i];
  g.V = (size_t)g.n[0] * g.n[1] * g.n[2] * g.n[3];
  return g;
}

// eta(site, rhs) = diag psi + hopc hop(psi) at one site and rhs, minus
// C(site) psi(site) when CL (clover field C: 42 packed entries per site)
template <int PREC, int LAYOUT, int SG, bool CL = false>
__device__ __forceinline__ void wilson_full_site(const typename prec_traits<PREC>::store* __restrict__ U,
                                                 const typename prec_traits<PREC>::store* __restrict__ psi,
                                                 typename prec_traits<PREC>::store* __restrict__ eta,
                                                 const geo4& g, int nrhs, typename prec_traits<PREC>::real diag,
                                                 typename prec_traits<PREC>::real hopc, size_t site, int rhs,
                                                 const typename prec_traits<PREC>::store* __restrict__ C = nullptr) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  const size_t V = g.V;
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], n3 = g.n[3];
  size_t r = site;
  const int x3 = (int)(r % n3); r /= n3;
  const int x2 = (int)(r % n2); r /= n2;
  const int x1 = (int)(r % n1);
  const int x0 = (int)(r / n1);
  const size_t s3 = 1, s2 = (size_t)n3, s1 = (size_t)n2 * n3, s0 = (size_t)n1 * n2 * n3;
  const size_t f0 = x0 + 1 < n0 ? site + s0 : site - (size_t)(n0 - 1) * s0;
  const size_t b0 = x0 > 0 ? site - s0 : site + (size_t)(n0 - 1) * s0;
  const size_t f1 = x1 + 1 < n1 ? site + s1 : site - (size_t)(n1 - 1) * s1;
  const size_t b1 = x1 > 0 ? site - s1 : site + (size_t)(n1 - 1) * s1;
  const size_t f2 = x2 + 1 < n2 ? site + s2 : site - (size_t)(n2 - 1) * s2;
  const size_t b2 = x2 > 0 ? site - s2 : site + (size_t)(n2 - 1) * s2;
  const size_t f3 = x3 + 1 < n3 ? site + s3 : site - (size_t)(n3 - 1) * s3;
  const size_t b3 = x3 > 0 ? site - s3 : site + (size_t)(n3 - 1) * s3;
  const int cs = blk<LAYOUT>::cstride(nrhs);
  spinor<R> acc;
#pragma unroll
  for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
  hop_dir<0, SG, S, R>(acc, psi, cs, blk<LAYOUT>::base(f0, rhs, V, nrhs), blk<LAYOUT>::base(b0, rhs, V, nrhs),
                       U + (0 * V + site) * 9, U + (0 * V + b0) * 9);
  hop_dir<1, SG, S, R>(acc, psi, cs, blk<LAYOUT>::base(f1, rhs, V, nrhs), blk<LAYOUT>::base(b1, rhs, V, nrhs),
                       U + (1 * V + site) * 9, U + (1 * V + b1) * 9);
  hop_dir<2, SG, S, R>(acc, psi, cs, blk<LAYOUT>::base(f2, rhs, V, nrhs), blk<LAYOUT>::base(b2, rhs, V, nrhs),
                       U + (2 * V + site) * 9, U + (2 * V + b2) * 9);
  hop_dir<3, SG, S, R>(acc, psi, cs, blk<LAYOUT>::base(f3, rhs, V, nrhs), blk<LAYOUT>::base(b3, rhs, V, nrhs),
                       U + (3 * V + site) * 9, U + (3 * V + b3) * 9);
  const size_t me = blk<LAYOUT>::base(site, rhs, V, nrhs);
  spinor<R> p = load_spinor<S, R>(psi, me, cs);
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    cx<R> a = acc.c[i / 3][i % 3], b = p.c[i / 3][i % 3];
    acc.c[i / 3][i % 3] = {fma(hopc, a.re, diag * b.re), fma(hopc, a.im, diag * b.im)};
  }
  if (CL) {
    const spinor<R> cp = clover_mul<S, R>(C + site * 42, p);
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = acc.c[i / 3][i % 3] - cp.c[i / 3][i % 3];
  }
  store_spinor<S, R>(eta, me, cs, acc);
}

// --------------------------------------------------------- odd-even hop
// out(h) = alpha * xin(h) + beta * hop(in)(h) for one parity-p site h (compact
// index) and rhs, where `in` is a parity (1-p) compact block; xin may be
// null (alpha ignored).  When CL, with per-site packed 42-entry fields
// indexed by site number (either may be null):
//   out(h) = Cout(x) [alpha xin(h) - Cx(x) xin(h) + beta hop(in)(h)].
template <int PREC, int LAYOUT, int SG, bool CL = false>
__device__ __forceinline__ void wilson_eo_site(const typename prec_traits<PREC>::store* __restrict__ U,
                                               const typename prec_traits<PREC>::store* __restrict__ in,
                                               const typename prec_traits<PREC>::store* __restrict__ xin,
                                               typename prec_traits<PREC>::store* __restrict__ out, const geo4& g,
                                               int p, int nrhs, typename prec_traits<PREC>::real alpha,
                                               typename prec_traits<PREC>::real beta, size_t h, int rhs,
                                               const typename prec_traits<PREC>::store* __restrict__ Cx = nullptr,
                                               const typename prec_traits<PREC>::store* __restrict__ Cout = nullptr) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  const size_t V = g.V, Vh = V / 2;
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], n3 = g.n[3];
  const int nh3 = n3 >> 1;
  size_t r = h;
  const int j = (int)(r % nh3); r /= nh3;
  const int x2 = (int)(r % n2); r /= n2;
  const int x1 = (int)(r % n1);
  const int x0 = (int)(r / n1);
  const int x3 = 2 * j + ((p + x0 + x1 + x2) & 1);
  // compact index of a site with the same x3 (row part) and with x3 changed
  const size_t row = ((size_t)(x0 * n1 + x1) * n2 + x2);
  const size_t site = row * n3 + x3;
  const size_t hs0 = (size_t)n1 * n2 * nh3, hs1 = (size_t)n2 * nh3, hs2 = (size_t)nh3;
  const size_t s0 = (size_t)n1 * n2 * n3, s1 = (size_t)n2 * n3, s2 = (size_t)n3;
  // neighbours: compact index (h..) of the other parity and site number (l..)
  size_t hf0, hb0, hf1, hb1, hf2, hb2, hf3, hb3, lb0, lb1, lb2, lb3;
  if (x0 + 1 < n0) hf0 = h + hs0; else hf0 = h - (size_t)(n0 - 1) * hs0;
  if (x0 > 0) { hb0 = h - hs0; lb0 = site - s0; } else { hb0 = h + (size_t)(n0 - 1) * hs0; lb0 = site + (size_t)(n0 - 1) * s0; }
  if (x1 + 1 < n1) hf1 = h + hs1; else hf1 = h - (size_t)(n1 - 1) * hs1;
  if (x1 > 0) { hb1 = h - hs1; lb1 = site - s1; } else { hb1 = h + (size_t)(n1 - 1) * hs1; lb1 = site + (size_t)(n1 - 1) * s1; }
  if (x2 + 1 < n2) hf2 = h + hs2; else hf2 = h - (size_t)(n2 - 1) * hs2;
  if (x2 > 0) { hb2 = h - hs2; lb2 = site - s2; } else { hb2 = h + (size_t)(n2 - 1) * hs2; lb2 = site + (size_t)(n2 - 1) * s2; }
  {
    const int xf = x3 + 1 < n3 ? x3 + 1 : 0;
    const int xb = x3 > 0 ? x3 - 1 : n3 - 1;
    hf3 = row * nh3 + (xf >> 1);
    hb3 = row * nh3 + (xb >> 1);
    lb3 = row * n3 + xb;
  }
  const int cs = blk<LAYOUT>::cstride(nrhs);
  spinor<R> acc;
#pragma unroll
  for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
  hop_dir<0, SG, S, R>(acc, in, cs, blk<LAYOUT>::base(hf0, rhs, Vh, nrhs), blk<LAYOUT>::base(hb0, rhs, Vh, nrhs),
                       U + (0 * V + site) * 9, U + (0 * V + lb0) * 9);
  hop_dir<1, SG, S, R>(acc, in, cs, blk<LAYOUT>::base(hf1, rhs, Vh, nrhs), blk<LAYOUT>::base(hb1, rhs, Vh, nrhs),
                       U + (1 * V + site) * 9, U + (1 * V + lb1) * 9);
  hop_dir<2, SG, S, R>(acc, in, cs, blk<LAYOUT>::base(hf2, rhs, Vh, nrhs), blk<LAYOUT>::base(hb2, rhs, Vh, nrhs),
                       U + (2 * V + site) * 9, U + (2 * V + lb2) * 9);
  hop_dir<3, SG, S, R>(acc, in, cs, blk<LAYOUT>::base(hf3, rhs, Vh, nrhs), blk<LAYOUT>::base(hb3, rhs, Vh, nrhs),
                       U + (3 * V + site) * 9, U + (3 * V + lb3) * 9);
  const size_t me = blk<LAYOUT>::base(h, rhs, Vh, nrhs);
  if (xin) {
    spinor<R> x = load_spinor<S, R>(xin, me, cs);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      cx<R> a = acc.c[i / 3][i % 3], b = x.c[i / 3][i % 3];
      acc.c[i / 3][i % 3] = {fma(beta, a.re, alpha * b.re), fma(beta, a.im, alpha * b.im)};
    }
    if (CL && Cx) {
      const spinor<R> cx_ = clover_mul<S, R>(Cx + site * 42, x);
#pragma unroll
      for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = acc.c[i / 3][i % 3] - cx_.c[i / 3][i % 3];
    }
  } else {
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = scale(beta, acc.c[i / 3][i % 3]);
  }
  if (CL && Cout) acc = clover_mul<S, R>(Cout + site * 42, acc);
  store_spinor<S, R>(out, me, cs, acc);
}

}  // namespace lq
