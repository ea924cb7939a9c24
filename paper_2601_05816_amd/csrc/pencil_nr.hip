// Pencil Wilson kernels with NR right-hand sides per work item (rhs-innermost
// layout, FP32 and FP16 storage).  The NR rhs of a component are consecutive
// in memory, so one vector access fetches them all (16 B for two FP32 or four
// FP16 numbers, 8 B for two FP16), and each link is loaded once for NR
// projected half spinors.  The arithmetic per site and rhs is the one of
// pencil.hip.  Needs nrhs % NR == 0.
#include "pencil.h"

namespace lq {

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
__global__ __launch_bounds__(256) void k_wilson_eo_pn(const typename prec_traits<PREC>::store* __restrict__ U,
                                                      const typename prec_traits<PREC>::store* __restrict__ in,
                                                      const typename prec_traits<PREC>::store* __restrict__ xin,
                                                      typename prec_traits<PREC>::store* __restrict__ out,
                                                      pencil_geo pg, int p, int nrhs,
                                                      typename prec_traits<PREC>::real alpha,
                                                      typename prec_traits<PREC>::real beta,
                                                      const int* __restrict__ live) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  int j, y, z, g, t0;
  if (!pencil_item<LQCD_LAYOUT2>(pg, nrhs / NR, j, y, z, g, t0)) return;
  const int rhs0 = g * NR;
  if (live) {
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) any |= live[rhs0 + r] != 0;
    if (!any) return;
  }
  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  const int NXh = NX >> 1;
  const size_t V = pg.V, Vh = V / 2;
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
__global__ __launch_bounds__(256) void k_wilson_full_pn(const typename prec_traits<PREC>::store* __restrict__ U,
                                                        const typename prec_traits<PREC>::store* __restrict__ psi,
                                                        typename prec_traits<PREC>::store* __restrict__ eta,
                                                        pencil_geo pg, int nrhs,
                                                        typename prec_traits<PREC>::real diag,
                                                        typename prec_traits<PREC>::real hopc) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  int x, y, z, g, t0;
  if (!pencil_item<LQCD_LAYOUT2>(pg, nrhs / NR, x, y, z, g, t0)) return;
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

// ------------------------------------------------------------- launchers
template <int PREC, int SG, int NR>
static hipError_t go_eo(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                        int nrhs, double alpha, double beta, const int* live, const kcfg& c, hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  pencil_geo pg = make_pencil(lat, nrhs / NR, true, c);
  size_t dyn = 0;
  if (!occupancy_lds(c.occ, 0, &dyn)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_wilson_eo_pn<PREC, SG, NR>), dim3(pencil_blocks(pg)), dim3(256), dyn, s, (const S*)U,
                     (const S*)in, (const S*)xin, (S*)out, pg, p, nrhs, (R)alpha, (R)beta, live);
  return hipSuccess;
}

template <int PREC, int SG, int NR>
static hipError_t go_full(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                          double hopc, const kcfg& c, hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  pencil_geo pg = make_pencil(lat, nrhs / NR, false, c);
  size_t dyn = 0;
  if (!occupancy_lds(c.occ, 0, &dyn)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_wilson_full_pn<PREC, SG, NR>), dim3(pencil_blocks(pg)), dim3(256), dyn, s, (const S*)U,
                     (const S*)psi, (S*)eta, pg, nrhs, (R)diag, (R)hopc);
  return hipSuccess;
}

bool nr_supported(int prec, int layout, int nrhs) {
  return layout == LQCD_LAYOUT2 && (prec == LQCD_F32 || prec == LQCD_F16) && nrhs % 2 == 0;
}

hipError_t wilson_eo_nr(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                        int nrhs, double alpha, double beta, int prec, bool dagger, const int* live, const kcfg& c,
                        hipStream_t s) {
  if (prec == LQCD_F32) {
    hipError_t e = dagger ? go_eo<LQCD_F32, -1, 2>(lat, U, in, xin, out, p, nrhs, alpha, beta, live, c, s)
                   : go_eo<LQCD_F32, 1, 2>(lat, U, in, xin, out, p, nrhs, alpha, beta, live, c, s);
    if (e != hipSuccess) return e;
  } else if (prec == LQCD_F16) {
    hipError_t e = dagger ? go_eo<LQCD_F16, -1, 2>(lat, U, in, xin, out, p, nrhs, alpha, beta, live, c, s)
                   : go_eo<LQCD_F16, 1, 2>(lat, U, in, xin, out, p, nrhs, alpha, beta, live, c, s);
    if (e != hipSuccess) return e;
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t wilson_full_nr(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                          double hopc, int prec, bool dagger, const kcfg& c, hipStream_t s) {
  if (prec == LQCD_F32) {
    hipError_t e = dagger ? go_full<LQCD_F32, -1, 2>(lat, U, psi, eta, nrhs, diag, hopc, c, s)
                   : go_full<LQCD_F32, 1, 2>(lat, U, psi, eta, nrhs, diag, hopc, c, s);
    if (e != hipSuccess) return e;
  } else if (prec == LQCD_F16) {
    hipError_t e = dagger ? go_full<LQCD_F16, -1, 2>(lat, U, psi, eta, nrhs, diag, hopc, c, s)
                   : go_full<LQCD_F16, 1, 2>(lat, U, psi, eta, nrhs, diag, hopc, c, s);
    if (e != hipSuccess) return e;
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lq
