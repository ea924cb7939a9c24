// Bodies of the time-streaming ("pencil") Wilson kernels, written for one
// block index b of the pencil grid so that the per-lattice kernels (one
// launch, b = blockIdx.x) and the persistent multi-lattice kernel (b walks
// a list of work units) share them.
#pragma once

#include "clover.h"
#include "pencil.h"

namespace lq {

// ---------------------------------------------------------- full lattice
// CL: the clover-improved operator D = D_W - C, C(x) psi(x) subtracted with
// the diagonal term (C: 42 packed entries per site).
template <int PREC, int LAYOUT, int SG, bool CL = false>
__device__ __forceinline__ void wilson_full_p_body(const typename prec_traits<PREC>::store* __restrict__ U,
                                                       const typename prec_traits<PREC>::store* __restrict__ psi,
                                                       typename prec_traits<PREC>::store* __restrict__ eta,
                                                       pencil_geo pg, int nrhs,
                                                       typename prec_traits<PREC>::real diag,
                                                       typename prec_traits<PREC>::real hopc, unsigned b,
                                                       const typename prec_traits<PREC>::store* __restrict__ C =
                                                           nullptr) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  int x, y, z, rhs, t0;
  if (!pencil_item<LAYOUT>(pg, nrhs, x, y, z, rhs, t0, b)) return;
  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  const size_t V = pg.V, S0 = (size_t)NZ * NY * NX;
  const int cs = blk<LAYOUT>::cstride(nrhs);
  const R one = (R)pg.one;
  // column bases (site number at t = 0) of this column and its spatial neighbours
  const size_t c0 = ((size_t)z * NY + y) * NX + x;
  const size_t cxf = c0 - x + (x + 1 < NX ? x + 1 : 0), cxb = c0 - x + (x > 0 ? x - 1 : NX - 1);
  const size_t cyf = c0 + (size_t)((y + 1 < NY ? y + 1 : 0) - y) * NX;
  const size_t cyb = c0 + (size_t)((y > 0 ? y - 1 : NY - 1) - y) * NX;
  const size_t czf = c0 + (size_t)((z + 1 < NZ ? z + 1 : 0) - z) * NY * NX;
  const size_t czb = c0 + (size_t)((z > 0 ? z - 1 : NZ - 1) - z) * NY * NX;
  const S* U0 = U;
  const S* U1 = U + 1 * V * 9;
  const S* U2 = U + 2 * V * 9;
  const S* U3 = U + 3 * V * 9;

  // prologue: the -t hop of site t0 and the projected centre of t0
  spinor<R> acc;
  half_spinor<R> hplus;
  {
    const int tm = t0 > 0 ? t0 - 1 : T - 1;
    const size_t sm = (size_t)tm * S0 + c0;
    spinor<R> pm = load_spinor<S, R>(psi, blk<LAYOUT>::base(sm, rhs, V, nrhs), cs);
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
    add_hop<0, SG, true, S, R>(acc, pm, U0 + sm * 9, hopc);
    const size_t s0 = (size_t)t0 * S0 + c0;
    spinor<R> p0 = load_spinor<S, R>(psi, blk<LAYOUT>::base(s0, rhs, V, nrhs), cs);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      cx<R> a = acc.c[i / 3][i % 3], b = p0.c[i / 3][i % 3];
      acc.c[i / 3][i % 3] = {fma(diag, b.re, a.re), fma(diag, b.im, a.im)};
    }
    if (CL) {
      const spinor<R> c0 = clover_mul<S, R>(C + s0 * 42, p0);
#pragma unroll
      for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = acc.c[i / 3][i % 3] - c0.c[i / 3][i % 3];
    }
    hplus = project<0, SG>(p0);
  }
  for (int it = 0; it < pg.Lt; ++it) {
    const int t = t0 + it;
    const size_t toff = (size_t)t * S0;
    const size_t site = toff + c0;
    // spatial hops (directions 3 = x, 2 = y, 1 = z); FP16 storage projects
    // the loaded values directly (add_hop_at)
    if constexpr (std::is_same<S, h2_t>::value) {
      add_hop_at<3, -SG, false, S, R>(acc, psi, blk<LAYOUT>::base(toff + cxf, rhs, V, nrhs), cs,
          U3 + site * 9, hopc, one);
      add_hop_at<3, SG, true, S, R>(acc, psi, blk<LAYOUT>::base(toff + cxb, rhs, V, nrhs), cs,
          U3 + (toff + cxb) * 9, hopc, one);
      add_hop_at<2, -SG, false, S, R>(acc, psi, blk<LAYOUT>::base(toff + cyf, rhs, V, nrhs), cs,
          U2 + site * 9, hopc, one);
      add_hop_at<2, SG, true, S, R>(acc, psi, blk<LAYOUT>::base(toff + cyb, rhs, V, nrhs), cs,
          U2 + (toff + cyb) * 9, hopc, one);
      add_hop_at<1, -SG, false, S, R>(acc, psi, blk<LAYOUT>::base(toff + czf, rhs, V, nrhs), cs,
          U1 + site * 9, hopc, one);
      add_hop_at<1, SG, true, S, R>(acc, psi, blk<LAYOUT>::base(toff + czb, rhs, V, nrhs), cs,
          U1 + (toff + czb) * 9, hopc, one);
    } else {
      {
        spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cxf, rhs, V, nrhs), cs);
        add_hop<3, -SG, false, S, R>(acc, p, U3 + site * 9, hopc);
      }
      {
        spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cxb, rhs, V, nrhs), cs);
        add_hop<3, SG, true, S, R>(acc, p, U3 + (toff + cxb) * 9, hopc);
      }
      {
        spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cyf, rhs, V, nrhs), cs);
        add_hop<2, -SG, false, S, R>(acc, p, U2 + site * 9, hopc);
      }
      {
        spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cyb, rhs, V, nrhs), cs);
        add_hop<2, SG, true, S, R>(acc, p, U2 + (toff + cyb) * 9, hopc);
      }
      {
        spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + czf, rhs, V, nrhs), cs);
        add_hop<1, -SG, false, S, R>(acc, p, U1 + site * 9, hopc);
      }
      {
        spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + czb, rhs, V, nrhs), cs);
        add_hop<1, SG, true, S, R>(acc, p, U1 + (toff + czb) * 9, hopc);
      }
    }
    // time direction: psi(t+1) gives the +t hop of t, and the centre and the
    // -t hop (through U_0(t)^dagger and the carried projection of psi(t)) of t+1
    const int t1 = t + 1 < T ? t + 1 : 0;
    const size_t s1 = (size_t)t1 * S0 + c0;
    spinor<R> p1 = load_spinor<S, R>(psi, blk<LAYOUT>::base(s1, rhs, V, nrhs), cs);
    add_hop<0, -SG, false, S, R>(acc, p1, U0 + site * 9, hopc);
    if (pg.nt) store_spinor_nt<S, R>(eta, blk<LAYOUT>::base(site, rhs, V, nrhs), cs, acc);
    else store_spinor<S, R>(eta, blk<LAYOUT>::base(site, rhs, V, nrhs), cs, acc);
    if (it + 1 < pg.Lt) {
#pragma unroll
      for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = scale(diag, p1.c[i / 3][i % 3]);
      if (CL) {
        const spinor<R> c1 = clover_mul<S, R>(C + s1 * 42, p1);
#pragma unroll
        for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = acc.c[i / 3][i % 3] - c1.c[i / 3][i % 3];
      }
      reconstruct<0, SG>(acc, hscale(hopc, colour_mul<true>(U0 + site * 9, hplus)));
      hplus = project<0, SG>(p1);
    }
  }
}

// --------------------------------------------------------- odd-even hop
// out(h) = alpha xin(h) + beta hop(in)(h) on parity p; columns are the
// compact (z, y, j) columns, j = x >> 1.  Along t the output site of a
// compact column alternates between x = 2j and 2j + 1; its +-t neighbours
// (parity 1-p) lie in the same compact column at t +- 1 with the same x.
template <int PREC, int LAYOUT, int SG>
__device__ __forceinline__ void wilson_eo_p_body(const typename prec_traits<PREC>::store* __restrict__ U,
                                                     const typename prec_traits<PREC>::store* __restrict__ in,
                                                     const typename prec_traits<PREC>::store* __restrict__ xin,
                                                     typename prec_traits<PREC>::store* __restrict__ out,
                                                     pencil_geo pg, int p, int nrhs,
                                                     typename prec_traits<PREC>::real alpha,
                                                     typename prec_traits<PREC>::real beta,
                                                     const int* __restrict__ live, unsigned b) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  int j, y, z, rhs, t0;
  if (!pencil_item<LAYOUT>(pg, nrhs, j, y, z, rhs, t0, b)) return;
  if (live && !live[rhs]) return;
  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  const int NXh = NX >> 1;
  const size_t V = pg.V, Vh = V / 2;
  const size_t S0 = (size_t)NZ * NY * NX, H0 = S0 / 2;  // site / compact strides of one time slice
  const int cs = blk<LAYOUT>::cstride(nrhs);
  const size_t row = (size_t)z * NY + y;                   // (z, y) row
  const size_t hc = row * NXh + j;                         // compact column base at t = 0
  const size_t hyf = ((size_t)z * NY + (y + 1 < NY ? y + 1 : 0)) * NXh + j;
  const size_t hyb = ((size_t)z * NY + (y > 0 ? y - 1 : NY - 1)) * NXh + j;
  const size_t hzf = ((size_t)(z + 1 < NZ ? z + 1 : 0) * NY + y) * NXh + j;
  const size_t hzb = ((size_t)(z > 0 ? z - 1 : NZ - 1) * NY + y) * NXh + j;
  const size_t lyb = ((size_t)z * NY + (y > 0 ? y - 1 : NY - 1)) * NX;  // site bases (x added later)
  const size_t lzb = ((size_t)(z > 0 ? z - 1 : NZ - 1) * NY + y) * NX;
  const size_t lrow = row * NX;
  const S* U0 = U;
  const S* U1 = U + 1 * V * 9;
  const S* U2 = U + 2 * V * 9;
  const S* U3 = U + 3 * V * 9;
  const int par0 = (p + z + y) & 1;  // x parity offset at t = 0
  const R one = (R)pg.one;

  // One direction per phase: both neighbours and both links are loaded
  // before either term is accumulated, so a wavefront has two hops' loads
  // in flight.  The -t neighbour in(t-1) of the same compact column is
  // loaded again (it was this work item's +t neighbour two steps earlier,
  // an L2 hit) rather than carried: a carried projection costs the
  // registers that the second hop's loads need.
  for (int it = 0; it < pg.Lt; ++it) {
    const int t = t0 + it;
    const int x = 2 * j + ((par0 + t) & 1);
    const size_t site = (size_t)t * S0 + lrow + x;
    const size_t hh = (size_t)t * H0 + hc;
    const size_t toffh = (size_t)t * H0;
    spinor<R> acc;
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
    {
      const int tm = t > 0 ? t - 1 : T - 1, t1 = t + 1 < T ? t + 1 : 0;
      add_hop_pair<0, SG, S, R>(acc, in, blk<LAYOUT>::base((size_t)t1 * H0 + hc, rhs, Vh, nrhs),
                                blk<LAYOUT>::base((size_t)tm * H0 + hc, rhs, Vh, nrhs), cs, U0 + site * 9,
                                U0 + ((size_t)tm * S0 + lrow + x) * 9, one);
    }
    {
      const int xf = x + 1 < NX ? x + 1 : 0, xb = x > 0 ? x - 1 : NX - 1;
      add_hop_pair<3, SG, S, R>(acc, in, blk<LAYOUT>::base(toffh + row * NXh + (xf >> 1), rhs, Vh, nrhs),
                                blk<LAYOUT>::base(toffh + row * NXh + (xb >> 1), rhs, Vh, nrhs), cs, U3 + site * 9,
                                U3 + ((size_t)t * S0 + lrow + xb) * 9, one);
    }
    add_hop_pair<2, SG, S, R>(acc, in, blk<LAYOUT>::base(toffh + hyf, rhs, Vh, nrhs),
                              blk<LAYOUT>::base(toffh + hyb, rhs, Vh, nrhs), cs, U2 + site * 9,
                              U2 + ((size_t)t * S0 + lyb + x) * 9, one);
    add_hop_pair<1, SG, S, R>(acc, in, blk<LAYOUT>::base(toffh + hzf, rhs, Vh, nrhs),
                              blk<LAYOUT>::base(toffh + hzb, rhs, Vh, nrhs), cs, U1 + site * 9,
                              U1 + ((size_t)t * S0 + lzb + x) * 9, one);
    const size_t me = blk<LAYOUT>::base(hh, rhs, Vh, nrhs);
    if (xin) {
      spinor<R> xv = load_spinor<S, R>(xin, me, cs);
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        cx<R> a = acc.c[i / 3][i % 3], b = xv.c[i / 3][i % 3];
        acc.c[i / 3][i % 3] = {fma(beta, a.re, alpha * b.re), fma(beta, a.im, alpha * b.im)};
      }
    } else {
#pragma unroll
      for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = scale(beta, acc.c[i / 3][i % 3]);
    }
    if (pg.nt) store_spinor_nt<S, R>(out, me, cs, acc);
    else store_spinor<S, R>(out, me, cs, acc);
  }
}

template <int NR, typename S, typename R>
__device__ __forceinline__ void load_spinors(const S* __restrict__ p, size_t base, int cs, spinor<R> (&v)[NR]) {
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    cx<R> t[NR];
    ldn<NR>(p + base + (size_t)i * cs, t);
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r].c[i / 3][i % 3] = t[r];
  }
}

template <int NR, typename S, typename R>
__device__ __forceinline__ void store_spinors(S* __restrict__ p, size_t base, int cs, const spinor<R> (&v)[NR]) {
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    cx<R> t[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) t[r] = v[r].c[i / 3][i % 3];
    stn<NR>(p + base + (size_t)i * cs, t);
  }
}

// acc[r] += c (hop term of direction MU, projector sign T) of neighbours p[r], one link for all r
template <int MU, int T, bool ADJ, int NR, typename S, typename R>
__device__ __forceinline__ void add_hops(spinor<R> (&acc)[NR], const spinor<R> (&p)[NR], const S* __restrict__ u,
                                         R c) {
  const su3<R> m = load_link<S, R>(u);
#pragma unroll
  for (int r = 0; r < NR; ++r)
    reconstruct<MU, T>(acc[r], hscale(c, colour_mul_r<ADJ>(m, project<MU, T>(p[r]))));
}

// --------------------------------------------------------- odd-even hop
template <int PREC, int SG, int NR>
__device__ __forceinline__ void wilson_eo_pn_body(const typename prec_traits<PREC>::store* __restrict__ U,
                                                      const typename prec_traits<PREC>::store* __restrict__ in,
                                                      const typename prec_traits<PREC>::store* __restrict__ xin,
                                                      typename prec_traits<PREC>::store* __restrict__ out,
                                                      pencil_geo pg, int p, int nrhs,
                                                      typename prec_traits<PREC>::real alpha,
                                                      typename prec_traits<PREC>::real beta,
                                                      const int* __restrict__ live, unsigned b) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  int j, y, z, g, t0;
  if (!pencil_item<LQCD_LAYOUT2>(pg, nrhs / NR, j, y, z, g, t0, b)) return;
  const int rhs0 = g * NR;
  if (live) {
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) any |= live[rhs0 + r] != 0;
    if (!any) return;
  }
  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  const int NXh = NX >> 1;
  const size_t V = pg.V;
  const size_t S0 = (size_t)NZ * NY * NX, H0 = S0 / 2;
  const int cs = nrhs;
  auto base = [&](size_t h) { return h * 12u * (size_t)nrhs + (size_t)rhs0; };
  const size_t row = (size_t)z * NY + y;
  const size_t hc = row * NXh + j;
  const size_t hyf = ((size_t)z * NY + (y + 1 < NY ? y + 1 : 0)) * NXh + j;
  const size_t hyb = ((size_t)z * NY + (y > 0 ? y - 1 : NY - 1)) * NXh + j;
  const size_t hzf = ((size_t)(z + 1 < NZ ? z + 1 : 0) * NY + y) * NXh + j;
  const size_t hzb = ((size_t)(z > 0 ? z - 1 : NZ - 1) * NY + y) * NXh + j;
  const size_t lyb = ((size_t)z * NY + (y > 0 ? y - 1 : NY - 1)) * NX;
  const size_t lzb = ((size_t)(z > 0 ? z - 1 : NZ - 1) * NY + y) * NX;
  const size_t lrow = row * NX;
  const S* U0 = U;
  const S* U1 = U + 1 * V * 9;
  const S* U2 = U + 2 * V * 9;
  const S* U3 = U + 3 * V * 9;
  const int par0 = (p + z + y) & 1;

  half_spinor<R> q0[NR], q1[NR];
  {
    const int tm = t0 > 0 ? t0 - 1 : T - 1;
    spinor<R> pm[NR];
    load_spinors<NR>(in, base((size_t)tm * H0 + hc), cs, pm);
#pragma unroll
    for (int r = 0; r < NR; ++r) q0[r] = project<0, SG>(pm[r]);
    load_spinors<NR>(in, base((size_t)t0 * H0 + hc), cs, pm);
#pragma unroll
    for (int r = 0; r < NR; ++r) q1[r] = project<0, SG>(pm[r]);
  }
  for (int it = 0; it < pg.Lt; ++it) {
    const int t = t0 + it;
    const int x = 2 * j + ((par0 + t) & 1);
    const size_t site = (size_t)t * S0 + lrow + x;
    const size_t toffh = (size_t)t * H0;
    spinor<R> acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < 12; ++i) acc[r].c[i / 3][i % 3] = {R(0), R(0)};
    {
      const int tm = t > 0 ? t - 1 : T - 1;
      const su3<R> m = load_link<S, R>(U0 + ((size_t)tm * S0 + lrow + x) * 9);
#pragma unroll
      for (int r = 0; r < NR; ++r) reconstruct<0, SG>(acc[r], colour_mul_r<true>(m, q0[r]));
    }
    {
      const int xf = x + 1 < NX ? x + 1 : 0, xb = x > 0 ? x - 1 : NX - 1;
      spinor<R> pn[NR];
      load_spinors<NR>(in, base(toffh + row * NXh + (xf >> 1)), cs, pn);
      add_hops<3, -SG, false, NR, S, R>(acc, pn, U3 + site * 9, R(1));
      load_spinors<NR>(in, base(toffh + row * NXh + (xb >> 1)), cs, pn);
      add_hops<3, SG, true, NR, S, R>(acc, pn, U3 + ((size_t)t * S0 + lrow + xb) * 9, R(1));
    }
    {
      spinor<R> pn[NR];
      load_spinors<NR>(in, base(toffh + hyf), cs, pn);
      add_hops<2, -SG, false, NR, S, R>(acc, pn, U2 + site * 9, R(1));
      load_spinors<NR>(in, base(toffh + hyb), cs, pn);
      add_hops<2, SG, true, NR, S, R>(acc, pn, U2 + ((size_t)t * S0 + lyb + x) * 9, R(1));
    }
    {
      spinor<R> pn[NR];
      load_spinors<NR>(in, base(toffh + hzf), cs, pn);
      add_hops<1, -SG, false, NR, S, R>(acc, pn, U1 + site * 9, R(1));
      load_spinors<NR>(in, base(toffh + hzb), cs, pn);
      add_hops<1, SG, true, NR, S, R>(acc, pn, U1 + ((size_t)t * S0 + lzb + x) * 9, R(1));
    }
    {
      const int t1 = t + 1 < T ? t + 1 : 0;
      spinor<R> pn[NR];
      load_spinors<NR>(in, base((size_t)t1 * H0 + hc), cs, pn);
      add_hops<0, -SG, false, NR, S, R>(acc, pn, U0 + site * 9, R(1));
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        q0[r] = q1[r];
        q1[r] = project<0, SG>(pn[r]);
      }
    }
    const size_t me = base(toffh + hc);
    if (xin) {
      spinor<R> xv[NR];
      load_spinors<NR>(xin, me, cs, xv);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          cx<R> a = acc[r].c[i / 3][i % 3], b = xv[r].c[i / 3][i % 3];
          acc[r].c[i / 3][i % 3] = {fma(beta, a.re, alpha * b.re), fma(beta, a.im, alpha * b.im)};
        }
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < 12; ++i) acc[r].c[i / 3][i % 3] = scale(beta, acc[r].c[i / 3][i % 3]);
    }
    store_spinors<NR>(out, me, cs, acc);
  }
}

// ---------------------------------------------------------- full lattice
template <int PREC, int SG, int NR>
__device__ __forceinline__ void wilson_full_pn_body(const typename prec_traits<PREC>::store* __restrict__ U,
                                                        const typename prec_traits<PREC>::store* __restrict__ psi,
                                                        typename prec_traits<PREC>::store* __restrict__ eta,
                                                        pencil_geo pg, int nrhs,
                                                        typename prec_traits<PREC>::real diag,
                                                        typename prec_traits<PREC>::real hopc, unsigned b) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  int x, y, z, g, t0;
  if (!pencil_item<LQCD_LAYOUT2>(pg, nrhs / NR, x, y, z, g, t0, b)) return;
  const int rhs0 = g * NR;
  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  const size_t V = pg.V, S0 = (size_t)NZ * NY * NX;
  const int cs = nrhs;
  auto base = [&](size_t site) { return site * 12u * (size_t)nrhs + (size_t)rhs0; };
  const size_t c0 = ((size_t)z * NY + y) * NX + x;
  const size_t cxf = c0 - x + (x + 1 < NX ? x + 1 : 0), cxb = c0 - x + (x > 0 ? x - 1 : NX - 1);
  const size_t cyf = c0 + (size_t)((y + 1 < NY ? y + 1 : 0) - y) * NX;
  const size_t cyb = c0 + (size_t)((y > 0 ? y - 1 : NY - 1) - y) * NX;
  const size_t czf = c0 + (size_t)((z + 1 < NZ ? z + 1 : 0) - z) * NY * NX;
  const size_t czb = c0 + (size_t)((z > 0 ? z - 1 : NZ - 1) - z) * NY * NX;
  const S* U0 = U;
  const S* U1 = U + 1 * V * 9;
  const S* U2 = U + 2 * V * 9;
  const S* U3 = U + 3 * V * 9;

  spinor<R> acc[NR];
  half_spinor<R> hplus[NR];
  {
    const int tm = t0 > 0 ? t0 - 1 : T - 1;
    const size_t sm = (size_t)tm * S0 + c0;
    spinor<R> pm[NR];
    load_spinors<NR>(psi, base(sm), cs, pm);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < 12; ++i) acc[r].c[i / 3][i % 3] = {R(0), R(0)};
    add_hops<0, SG, true, NR, S, R>(acc, pm, U0 + sm * 9, hopc);
    load_spinors<NR>(psi, base((size_t)t0 * S0 + c0), cs, pm);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        cx<R> a = acc[r].c[i / 3][i % 3], b = pm[r].c[i / 3][i % 3];
        acc[r].c[i / 3][i % 3] = {fma(diag, b.re, a.re), fma(diag, b.im, a.im)};
      }
      hplus[r] = project<0, SG>(pm[r]);
    }
  }
  for (int it = 0; it < pg.Lt; ++it) {
    const int t = t0 + it;
    const size_t toff = (size_t)t * S0;
    const size_t site = toff + c0;
    {
      spinor<R> pn[NR];
      load_spinors<NR>(psi, base(toff + cxf), cs, pn);
      add_hops<3, -SG, false, NR, S, R>(acc, pn, U3 + site * 9, hopc);
      load_spinors<NR>(psi, base(toff + cxb), cs, pn);
      add_hops<3, SG, true, NR, S, R>(acc, pn, U3 + (toff + cxb) * 9, hopc);
      load_spinors<NR>(psi, base(toff + cyf), cs, pn);
      add_hops<2, -SG, false, NR, S, R>(acc, pn, U2 + site * 9, hopc);
      load_spinors<NR>(psi, base(toff + cyb), cs, pn);
      add_hops<2, SG, true, NR, S, R>(acc, pn, U2 + (toff + cyb) * 9, hopc);
      load_spinors<NR>(psi, base(toff + czf), cs, pn);
      add_hops<1, -SG, false, NR, S, R>(acc, pn, U1 + site * 9, hopc);
      load_spinors<NR>(psi, base(toff + czb), cs, pn);
      add_hops<1, SG, true, NR, S, R>(acc, pn, U1 + (toff + czb) * 9, hopc);
    }
    const int t1 = t + 1 < T ? t + 1 : 0;
    spinor<R> p1[NR];
    load_spinors<NR>(psi, base((size_t)t1 * S0 + c0), cs, p1);
    const su3<R> u0 = load_link<S, R>(U0 + site * 9);
#pragma unroll
    for (int r = 0; r < NR; ++r)
      reconstruct<0, -SG>(acc[r], hscale(hopc, colour_mul_r<false>(u0, project<0, -SG>(p1[r]))));
    store_spinors<NR>(eta, base(site), cs, acc);
    if (it + 1 < pg.Lt) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int i = 0; i < 12; ++i) acc[r].c[i / 3][i % 3] = scale(diag, p1[r].c[i / 3][i % 3]);
        reconstruct<0, SG>(acc[r], hscale(hopc, colour_mul_r<true>(u0, hplus[r])));
        hplus[r] = project<0, SG>(p1[r]);
      }
    }
  }
}

// ------------------------------------------- full lattice, links via LDS
// Same pencil walk; the links of a time step are fetched once per wavefront
// with coalesced loads (one complex number per lane and load) into a
// wave-private LDS slice and read from there by all lanes of a column (the
// rhs that share the column), instead of one vector-memory load per lane and
// link element.  The slices are double-buffered and the loads of step t+1 are
// issued before step t is computed, so their latency overlaps the step.
// Rhs-fastest layouts only; NCW bounds the number of columns one wavefront
// touches (64 / nrhs + 1).
// Link slots per column and step: 0 U_0(x), 1..3 U_mu(x) (mu = 1 z, 2 y, 3 x),
// 4..6 U_mu(x - mu).
// lds_all: a double-buffered slice per wavefront of the workgroup; b: block
// index of the pencil grid.
template <int PREC, int LAYOUT, int SG, int NCW>
__device__ __forceinline__ void wilson_full_pl_body(const typename prec_traits<PREC>::store* __restrict__ U,
                                                    const typename prec_traits<PREC>::store* __restrict__ psi,
                                                    typename prec_traits<PREC>::store* __restrict__ eta,
                                                    pencil_geo pg, int nrhs,
                                                    typename prec_traits<PREC>::real diag,
                                                    typename prec_traits<PREC>::real hopc, unsigned b,
                                                    typename prec_traits<PREC>::store (&lds_all)[4][2][NCW * 63]) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  constexpr int NEL = NCW * 63;            // link elements of a wavefront and step
  constexpr int NE = (NEL + 63) / 64;      // per lane
  const unsigned k8 = b & 7u, ib = b >> 3;
  const unsigned u = ib / pg.bpt, q = ib % pg.bpt;
  const unsigned ngrp = (unsigned)(pg.ntiles + 7) / 8u;
  const unsigned seg = u / ngrp, grp = u % ngrp;  // segment-major: tile groups of one t segment run back to back
  const unsigned tile = grp * 8u + k8;
  if (tile >= (unsigned)pg.ntiles) return;  // whole workgroup idle
  const unsigned CT = (unsigned)pg.TX * pg.TY * pg.TZ;
  const unsigned wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const unsigned tin = q * blockDim.x + threadIdx.x;
  const unsigned tw0 = q * blockDim.x + wave * 64u;
  if (tw0 >= CT * (unsigned)nrhs) return;  // whole wavefront idle (no LDS sharing across waves)
  const unsigned colw0 = tw0 / nrhs;
  unsigned colw1 = (tw0 + 63u) / nrhs;
  if (colw1 > CT - 1) colw1 = CT - 1;
  const int ncw = (int)(colw1 - colw0 + 1);
  const bool active = tin < CT * (unsigned)nrhs;
  const unsigned col = active ? tin / nrhs : colw0;
  const int rhs = (int)(tin % nrhs);
  const int cl = (int)(col - colw0);

  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  const int tx = tile % pg.NTX, ty = (tile / pg.NTX) % pg.NTY, tz = tile / (pg.NTX * pg.NTY);
  const int t0 = (int)seg * pg.Lt;
  const size_t V = pg.V, S0 = (size_t)NZ * NY * NX;
  const int cs = blk<LAYOUT>::cstride(nrhs);
  auto colsite = [&](unsigned c, int& x, int& y, int& z) {
    x = tx * pg.TX + (int)(c % pg.TX);
    y = ty * pg.TY + (int)((c / pg.TX) % pg.TY);
    z = tz * pg.TZ + (int)(c / (pg.TX * pg.TY));
  };
  int x, y, z;
  colsite(col, x, y, z);
  const size_t c0 = ((size_t)z * NY + y) * NX + x;
  const size_t cxf = c0 - x + (x + 1 < NX ? x + 1 : 0), cxb = c0 - x + (x > 0 ? x - 1 : NX - 1);
  const size_t cyf = c0 + (size_t)((y + 1 < NY ? y + 1 : 0) - y) * NX;
  const size_t cyb = c0 + (size_t)((y > 0 ? y - 1 : NY - 1) - y) * NX;
  const size_t czf = c0 + (size_t)((z + 1 < NZ ? z + 1 : 0) - z) * NY * NX;
  const size_t czb = c0 + (size_t)((z > 0 ? z - 1 : NZ - 1) - z) * NY * NX;
  const S* U0 = U;

  // this lane's link elements: source offset at t = 0 and LDS slot, computed once
  size_t goff[NE];
  int lidx[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = (int)lane + 64 * k;
    lidx[k] = -1;
    goff[k] = 0;
    if (e < ncw * 63) {
      const int slot = e / (9 * ncw);
      const int rem = e - slot * 9 * ncw;
      const int c = rem / 9, kk = rem - c * 9;
      int xx, yy, zz;
      colsite(colw0 + (unsigned)c, xx, yy, zz);
      size_t sc = ((size_t)zz * NY + yy) * NX + xx;
      int mu = slot;
      if (slot >= 4) {
        mu = slot - 3;
        if (mu == 1) sc += (size_t)((zz > 0 ? zz - 1 : NZ - 1) - zz) * NY * NX;
        else if (mu == 2) sc += (size_t)((yy > 0 ? yy - 1 : NY - 1) - yy) * NX;
        else sc += (size_t)((xx > 0 ? xx - 1 : NX - 1) - xx);
      }
      goff[k] = ((size_t)mu * V + sc) * 9 + kk;
      lidx[k] = (c * 7 + slot) * 9 + kk;
    }
  }
  S lr[NE];
  auto fetch = [&](int t) {
    const size_t toff9 = (size_t)t * S0 * 9;
#pragma unroll
    for (int k = 0; k < NE; ++k)
      if (lidx[k] >= 0) lr[k] = U[goff[k] + toff9];
  };
  auto put = [&](int buf) {
    S* lds = lds_all[wave][buf];
#pragma unroll
    for (int k = 0; k < NE; ++k)
      if (lidx[k] >= 0) lds[lidx[k]] = lr[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };

  spinor<R> acc;
  half_spinor<R> hplus;
  fetch(t0);
  {
    const int tm = t0 > 0 ? t0 - 1 : T - 1;
    const size_t sm = (size_t)tm * S0 + c0;
    spinor<R> pm = load_spinor<S, R>(psi, blk<LAYOUT>::base(sm, rhs, V, nrhs), cs);
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
    add_hop<0, SG, true, S, R>(acc, pm, U0 + sm * 9, hopc);
    const size_t s0 = (size_t)t0 * S0 + c0;
    spinor<R> p0 = load_spinor<S, R>(psi, blk<LAYOUT>::base(s0, rhs, V, nrhs), cs);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      cx<R> a = acc.c[i / 3][i % 3], bb = p0.c[i / 3][i % 3];
      acc.c[i / 3][i % 3] = {fma(diag, bb.re, a.re), fma(diag, bb.im, a.im)};
    }
    hplus = project<0, SG>(p0);
  }
  put(0);
  for (int it = 0; it < pg.Lt; ++it) {
    const int t = t0 + it;
    const size_t toff = (size_t)t * S0;
    const size_t site = toff + c0;
    const S* L = lds_all[wave][it & 1] + cl * 7 * 9;
    if (it + 1 < pg.Lt) fetch(t + 1);
    {
      spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cxf, rhs, V, nrhs), cs);
      add_hop<3, -SG, false, S, R>(acc, p, L + 3 * 9, hopc);
    }
    {
      spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cxb, rhs, V, nrhs), cs);
      add_hop<3, SG, true, S, R>(acc, p, L + 6 * 9, hopc);
    }
    {
      spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cyf, rhs, V, nrhs), cs);
      add_hop<2, -SG, false, S, R>(acc, p, L + 2 * 9, hopc);
    }
    {
      spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cyb, rhs, V, nrhs), cs);
      add_hop<2, SG, true, S, R>(acc, p, L + 5 * 9, hopc);
    }
    {
      spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + czf, rhs, V, nrhs), cs);
      add_hop<1, -SG, false, S, R>(acc, p, L + 1 * 9, hopc);
    }
    {
      spinor<R> p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + czb, rhs, V, nrhs), cs);
      add_hop<1, SG, true, S, R>(acc, p, L + 4 * 9, hopc);
    }
    const int t1 = t + 1 < T ? t + 1 : 0;
    const size_t s1 = (size_t)t1 * S0 + c0;
    spinor<R> p1 = load_spinor<S, R>(psi, blk<LAYOUT>::base(s1, rhs, V, nrhs), cs);
    add_hop<0, -SG, false, S, R>(acc, p1, L, hopc);
    if (active) {
      if (pg.nt) store_spinor_nt<S, R>(eta, blk<LAYOUT>::base(site, rhs, V, nrhs), cs, acc);
      else store_spinor<S, R>(eta, blk<LAYOUT>::base(site, rhs, V, nrhs), cs, acc);
    }
    if (it + 1 < pg.Lt) {
#pragma unroll
      for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = scale(diag, p1.c[i / 3][i % 3]);
      reconstruct<0, SG>(acc, hscale(hopc, colour_mul<true>(L, hplus)));
      hplus = project<0, SG>(p1);
      put((it + 1) & 1);
    }
  }
}

}  // namespace lq
