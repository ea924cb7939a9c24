// Pencil Wilson kernels whose links reach the rhs lanes by a row broadcast.
//
// In the rhs-fastest layouts with nrhs a multiple of 16, each 16-lane row of
// a wavefront holds 16 rhs of one column, so every lane of a row needs the
// same links at every time step.  Instead of one vector-memory load per lane
// and link element (63 per step for the full operator, each moving the same
// 16 bytes to 16 lanes), lane k of a row loads link elements k, k+16, k+32,
// k+48 of its column's step (four loads per lane), and each element is moved
// to the whole row with a DPP row broadcast (v_mov_dpp row_newbcast), a VALU
// move.  The vector-memory pipe then carries only the spinors and the
// elements themselves, once; the arithmetic per site and rhs is the one of
// pencil.hip (Algorithm 1's projected hops, the time-direction reuse of the
// streamed spinor), so results agree with the other pencil kernels bit for
// bit.  The loads of step t+1's elements are issued at the top of step t.
#include <type_traits>
#include <utility>

#include "pencil_kernels.h"

namespace lq {

// ------------------------------------------------------- row broadcast
// Value of v in lane N of this lane's 16-lane row (a bit-exact move).
template <int N>
__device__ __forceinline__ double2 rowb(double2 v) {
  long a = __builtin_bit_cast(long, v.x), b = __builtin_bit_cast(long, v.y);
  a = __builtin_amdgcn_update_dpp(0l, a, 0x150 + N, 0xf, 0xf, true);
  b = __builtin_amdgcn_update_dpp(0l, b, 0x150 + N, 0xf, 0xf, true);
  return make_double2(__builtin_bit_cast(double, a), __builtin_bit_cast(double, b));
}
template <int N>
__device__ __forceinline__ float2 rowb(float2 v) {
  long a = __builtin_bit_cast(long, v);
  a = __builtin_amdgcn_update_dpp(0l, a, 0x150 + N, 0xf, 0xf, true);
  return __builtin_bit_cast(float2, a);
}
template <int N>
__device__ __forceinline__ h2_t rowb(h2_t v) {
  int a = __builtin_bit_cast(int, v);
  a = __builtin_amdgcn_update_dpp(0, a, 0x150 + N, 0xf, 0xf, true);
  return __builtin_bit_cast(h2_t, a);
}

// Link slot SLOT (9 elements; element e of the step sits in register e / 16
// of lane e % 16) broadcast to the row and widened to the arithmetic type.
template <int SLOT, typename S, typename R, int... K>
__device__ __forceinline__ su3<R> bc_link_impl(const S* lr, std::integer_sequence<int, K...>) {
  su3<R> m;
  ((m.m[K / 3][K % 3] = widen(rowb<(9 * SLOT + K) % 16>(lr[(9 * SLOT + K) / 16]))), ...);
  return m;
}
template <int SLOT, typename S, typename R>
__device__ __forceinline__ su3<R> bc_link(const S* lr) {
  return bc_link_impl<SLOT, S, R>(lr, std::make_integer_sequence<int, 9>{});
}

// acc += c * (hop term MU, projector sign T) of neighbour p with link m
template <int MU, int T, bool ADJ, typename R>
__device__ __forceinline__ void add_hop_r(spinor<R>& acc, const spinor<R>& p, const su3<R>& m, R c) {
  reconstruct<MU, T>(acc, hscale(c, colour_mul_r<ADJ>(m, project<MU, T>(p))));
}

// the same for the neighbour stored at p[base + i cs] (i = 0..11) with the
// link of slot SLOT; FP16 storage projects the loaded values directly
// (load_project, no separate conversions), FP32 / FP64 widen the spinor
// first, the form their kernels were tuned with
template <int MU, int T, bool ADJ, int SLOT, typename S, typename R>
__device__ __forceinline__ void add_hop_bc(spinor<R>& acc, const S* __restrict__ p, size_t base, int cs,
                                           const S* lr, R c, R one) {
  if constexpr (std::is_same<S, h2_t>::value) {
    const half_spinor<R> h = load_project<MU, T>(p, base, cs, one);
    reconstruct<MU, T>(acc, hscale(c, colour_mul_r<ADJ>(bc_link<SLOT, S, R>(lr), h)));
  } else {
    const spinor<R> v = load_spinor<S, R>(p, base, cs);
    add_hop_r<MU, T, ADJ, R>(acc, v, bc_link<SLOT, S, R>(lr), c);
  }
}

// acc += both hop terms of direction MU (sign SG): forward neighbour at
// in[fb + i cs] with the link of slot SF, backward one at in[bb + i cs] with
// the adjoint of the link of slot SB; both loaded before either is used
template <int MU, int SG, int SF, int SB, typename S, typename R>
__device__ __forceinline__ void add_hop_pair_bc(spinor<R>& acc, const S* __restrict__ in, size_t fb, size_t bb,
                                                int cs, const S* lr, R one) {
  if constexpr (std::is_same<S, h2_t>::value) {
    const half_spinor<R> hf = load_project<MU, -SG>(in, fb, cs, one);
    const half_spinor<R> hb = load_project<MU, SG>(in, bb, cs, one);
    reconstruct<MU, -SG>(acc, colour_mul_r<false>(bc_link<SF, S, R>(lr), hf));
    reconstruct<MU, SG>(acc, colour_mul_r<true>(bc_link<SB, S, R>(lr), hb));
  } else {
    const spinor<R> pf = load_spinor<S, R>(in, fb, cs);
    const spinor<R> pb = load_spinor<S, R>(in, bb, cs);
    reconstruct<MU, -SG>(acc, colour_mul_r<false>(bc_link<SF, S, R>(lr), project<MU, -SG>(pf)));
    reconstruct<MU, SG>(acc, colour_mul_r<true>(bc_link<SB, S, R>(lr), project<MU, SG>(pb)));
  }
}

// ---------------------------------------------------------- full lattice
// Link slots of a step: 0 U_0(x), 1..3 U_mu(x) (mu = 1 z, 2 y, 3 x),
// 4..6 U_mu(x - mu); 63 elements, four per lane.
//
// nrhs is the number of rhs a workgroup's lanes cover, ldr the block's rhs
// count (the memory stride of LAYOUT1 / LAYOUT2); for ldr > nrhs the grid
// holds ldr / nrhs copies of the pencil grid, one rhs chunk each, chunk
// slowest, so the workgroups resident at any time stream one chunk (the
// working set of a time slice is that of nrhs rhs).
//
// XL (variant 7): the workgroup's 256 / nrhs columns are consecutive x of
// one row, so the +-x neighbours of all but the two end columns are the
// spinors the neighbouring columns of the same workgroup stream along t.
// Each column puts the spinor it loads for t+1 into LDS (one slot per
// column, rhs fastest), and at step t the inner columns read their x
// neighbours there; two barriers per step (before the reads, before the
// slot is overwritten).
template <int PREC, int LAYOUT, int SG, bool XL>
__global__ __launch_bounds__(256) void k_wilson_full_pb(const typename prec_traits<PREC>::store* __restrict__ U,
                                                        const typename prec_traits<PREC>::store* __restrict__ psi,
                                                        typename prec_traits<PREC>::store* __restrict__ eta,
                                                        pencil_geo pg, int nrhs, int ldr,
                                                        typename prec_traits<PREC>::real diag,
                                                        typename prec_traits<PREC>::real hopc) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  const R one = (R)pg.one;
  __shared__ S xs[XL ? 256 * 12 : 1];  // the workgroup's columns at one t, [column][12][rhs]
  int x, y, z, rhs, t0;
  // nrhs % 16 == 0: a row of 16 lanes is idle or busy as a whole (with XL the
  // launch guarantees whole workgroups)
  // rhs chunks (ldr > nrhs) run one after another: chunk-major grid
  const unsigned nb = gridDim.x / (unsigned)(ldr / nrhs), chunk = blockIdx.x / nb;
  if (!pencil_item<LAYOUT>(pg, nrhs, x, y, z, rhs, t0, blockIdx.x % nb)) return;
  const int rl = rhs;  // rhs within the chunk (LDS slots), rhs: within the block
  rhs += (int)chunk * nrhs;
  const int lc = (int)threadIdx.x / nrhs, ncw = 256 / nrhs;  // column within the workgroup (XL)
  auto put = [&](const spinor<R>& v) {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const cx<R> c = v.c[i / 3][i % 3];
      st(xs + ((size_t)lc * 12 + i) * nrhs + rl, c);
    }
  };
  auto get = [&](int col) {
    spinor<R> v;
#pragma unroll
    for (int i = 0; i < 12; ++i) v.c[i / 3][i % 3] = ld(xs + ((size_t)col * 12 + i) * nrhs + rl);
    return v;
  };
  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  const size_t V = pg.V, S0 = (size_t)NZ * NY * NX;
  const int cs = blk<LAYOUT>::cstride(ldr);
  const size_t c0 = ((size_t)z * NY + y) * NX + x;
  const size_t cxf = c0 - x + (x + 1 < NX ? x + 1 : 0), cxb = c0 - x + (x > 0 ? x - 1 : NX - 1);
  const size_t cyf = c0 + (size_t)((y + 1 < NY ? y + 1 : 0) - y) * NX;
  const size_t cyb = c0 + (size_t)((y > 0 ? y - 1 : NY - 1) - y) * NX;
  const size_t czf = c0 + (size_t)((z + 1 < NZ ? z + 1 : 0) - z) * NY * NX;
  const size_t czb = c0 + (size_t)((z > 0 ? z - 1 : NZ - 1) - z) * NY * NX;

  // this lane's link elements: offset at t = 0 (advanced by 9 S0 per step)
  const int l16 = (int)(threadIdx.x & 15u);
  size_t goff[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int e = l16 + 16 * j < 63 ? l16 + 16 * j : 62;  // lane 15's fourth element: a harmless repeat
    const int slot = e / 9, kk = e - 9 * (e / 9);
    const int mu = slot == 0 ? 0 : (slot <= 3 ? slot : slot - 3);
    const size_t col = slot <= 3 ? c0 : (slot == 4 ? czb : (slot == 5 ? cyb : cxb));
    goff[j] = ((size_t)mu * V + col) * 9 + kk;
  }
  const size_t step9 = S0 * 9;
  S lr[4], ln[4];

  spinor<R> acc;
  half_spinor<R> hplus;
  {
    const int tm = t0 > 0 ? t0 - 1 : T - 1;
    const size_t sm = (size_t)tm * S0 + c0;
#pragma unroll
    for (int j = 0; j < 4; ++j) lr[j] = U[goff[j] + (size_t)t0 * step9];
    spinor<R> pm = load_spinor<S, R>(psi, blk<LAYOUT>::base(sm, rhs, V, ldr), cs);
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
    add_hop<0, SG, true, S, R>(acc, pm, U + sm * 9, hopc);
    const size_t s0 = (size_t)t0 * S0 + c0;
    spinor<R> p0 = load_spinor<S, R>(psi, blk<LAYOUT>::base(s0, rhs, V, ldr), cs);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      cx<R> a = acc.c[i / 3][i % 3], b = p0.c[i / 3][i % 3];
      acc.c[i / 3][i % 3] = {fma(diag, b.re, a.re), fma(diag, b.im, a.im)};
    }
    hplus = project<0, SG>(p0);
    if (XL) put(p0);
  }
  for (int it = 0; it < pg.Lt; ++it) {
    const int t = t0 + it;
    const size_t toff = (size_t)t * S0;
    const size_t site = toff + c0;
    if (it + 1 < pg.Lt) {
#pragma unroll
      for (int j = 0; j < 4; ++j) ln[j] = U[goff[j] + (size_t)(t + 1) * step9];
    }
    if (XL) __syncthreads();  // every column's spinor at t is in LDS
    if constexpr (std::is_same<S, h2_t>::value) {  // FP16: project the loaded values directly
      const size_t lb = ((size_t)lc * 12) * nrhs + rl;  // this column's slot in LDS
      half_spinor<R> h;
      if (XL && lc + 1 < ncw) h = load_project<3, -SG>(xs, lb + 12 * (size_t)nrhs, nrhs, one);
      else h = load_project<3, -SG>(psi, blk<LAYOUT>::base(toff + cxf, rhs, V, ldr), cs, one);
      reconstruct<3, -SG>(acc, hscale(hopc, colour_mul_r<false>(bc_link<3, S, R>(lr), h)));
      if (XL && lc > 0) h = load_project<3, SG>(xs, lb - 12 * (size_t)nrhs, nrhs, one);
      else h = load_project<3, SG>(psi, blk<LAYOUT>::base(toff + cxb, rhs, V, ldr), cs, one);
      reconstruct<3, SG>(acc, hscale(hopc, colour_mul_r<true>(bc_link<6, S, R>(lr), h)));
    } else {
      {
        spinor<R> p;
        if (XL && lc + 1 < ncw) p = get(lc + 1);
        else p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cxf, rhs, V, ldr), cs);
        add_hop_r<3, -SG, false, R>(acc, p, bc_link<3, S, R>(lr), hopc);
      }
      {
        spinor<R> p;
        if (XL && lc > 0) p = get(lc - 1);
        else p = load_spinor<S, R>(psi, blk<LAYOUT>::base(toff + cxb, rhs, V, ldr), cs);
        add_hop_r<3, SG, true, R>(acc, p, bc_link<6, S, R>(lr), hopc);
      }
    }
    add_hop_bc<2, -SG, false, 2>(acc, psi, blk<LAYOUT>::base(toff + cyf, rhs, V, ldr), cs, lr, hopc, one);
    add_hop_bc<2, SG, true, 5>(acc, psi, blk<LAYOUT>::base(toff + cyb, rhs, V, ldr), cs, lr, hopc, one);
    add_hop_bc<1, -SG, false, 1>(acc, psi, blk<LAYOUT>::base(toff + czf, rhs, V, ldr), cs, lr, hopc, one);
    add_hop_bc<1, SG, true, 4>(acc, psi, blk<LAYOUT>::base(toff + czb, rhs, V, ldr), cs, lr, hopc, one);
    const int t1 = t + 1 < T ? t + 1 : 0;
    const size_t s1 = (size_t)t1 * S0 + c0;
    spinor<R> p1 = load_spinor<S, R>(psi, blk<LAYOUT>::base(s1, rhs, V, ldr), cs);
    const su3<R> u0 = bc_link<0, S, R>(lr);
    add_hop_r<0, -SG, false, R>(acc, p1, u0, hopc);
    if (pg.nt) store_spinor_nt<S, R>(eta, blk<LAYOUT>::base(site, rhs, V, ldr), cs, acc);
    else store_spinor<S, R>(eta, blk<LAYOUT>::base(site, rhs, V, ldr), cs, acc);
    if (it + 1 < pg.Lt) {
#pragma unroll
      for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = scale(diag, p1.c[i / 3][i % 3]);
      reconstruct<0, SG>(acc, hscale(hopc, colour_mul_r<true>(u0, hplus)));
      hplus = project<0, SG>(p1);
#pragma unroll
      for (int j = 0; j < 4; ++j) lr[j] = ln[j];
      if (XL) {
        __syncthreads();  // every column has read its neighbours at t
        put(p1);
      }
    }
  }
}

// --------------------------------------------------------- odd-even hop
// out(h) = alpha xin(h) + beta hop(in)(h) on parity p, compact columns as in
// wilson_eo_p_body.  Link slots of a step: 0 U_0(x), 1 U_0(x - t), 2 U_3(x),
// 3 U_3(x - x^), 4 U_2(x), 5 U_2(x - y^), 6 U_1(x), 7 U_1(x - z^); 72
// elements, five per lane (the output site's x alternates with t, so the
// element addresses are formed per step).  Lanes of converged rhs (`live`)
// take part in the loads and broadcasts and skip only their store.
template <int PREC, int LAYOUT, int SG, bool XL>
__global__ __launch_bounds__(256) void k_wilson_eo_pb(const typename prec_traits<PREC>::store* __restrict__ U,
                                                      const typename prec_traits<PREC>::store* __restrict__ in,
                                                      const typename prec_traits<PREC>::store* __restrict__ xin,
                                                      typename prec_traits<PREC>::store* __restrict__ out,
                                                      pencil_geo pg, int p, int nrhs, int ldr,
                                                      typename prec_traits<PREC>::real alpha,
                                                      typename prec_traits<PREC>::real beta,
                                                      const int* __restrict__ live) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  // XL: the workgroup's columns at one t, [column][12][rhs] (see the kernel's comment)
  __shared__ S xs[XL ? 256 * 12 : 1];
  int j, y, z, rhs, t0;
  const unsigned nb = gridDim.x / (unsigned)(ldr / nrhs), chunk = blockIdx.x / nb;  // as in the full kernel
  if (!pencil_item<LAYOUT>(pg, nrhs, j, y, z, rhs, t0, blockIdx.x % nb)) return;
  const int rl = rhs;
  rhs += (int)chunk * nrhs;
  const bool store_me = !live || live[rhs];
  const int lc = (int)threadIdx.x / nrhs, ncw = 256 / nrhs;  // column within the workgroup (XL)
  const int jbase = j - lc;                                  // the workgroup's first compact column
  auto put = [&](const spinor<R>& v) {
#pragma unroll
    for (int i = 0; i < 12; ++i) st(xs + ((size_t)lc * 12 + i) * nrhs + rl, v.c[i / 3][i % 3]);
  };
  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  const R one = (R)pg.one;
  const int NXh = NX >> 1;
  const size_t V = pg.V, Vh = V / 2;
  const size_t S0 = (size_t)NZ * NY * NX, H0 = S0 / 2;
  const int cs = blk<LAYOUT>::cstride(ldr);
  const size_t row = (size_t)z * NY + y;
  const size_t hc = row * NXh + j;
  const size_t hyf = ((size_t)z * NY + (y + 1 < NY ? y + 1 : 0)) * NXh + j;
  const size_t hyb = ((size_t)z * NY + (y > 0 ? y - 1 : NY - 1)) * NXh + j;
  const size_t hzf = ((size_t)(z + 1 < NZ ? z + 1 : 0) * NY + y) * NXh + j;
  const size_t hzb = ((size_t)(z > 0 ? z - 1 : NZ - 1) * NY + y) * NXh + j;
  const size_t lyb = ((size_t)z * NY + (y > 0 ? y - 1 : NY - 1)) * NX;
  const size_t lzb = ((size_t)(z > 0 ? z - 1 : NZ - 1) * NY + y) * NX;
  const size_t lrow = row * NX;
  const int par0 = (p + z + y) & 1;

  // this lane's link elements: direction, entry, and where the site sits
  // (time t or t-1, row of x / y-1 / z-1, x or x-1), all fixed per lane
  const int l16 = (int)(threadIdx.x & 15u);
  int emu[5], ekk[5];
  bool etm[5], exb[5];
  size_t erow[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const int e = l16 + 16 * q < 72 ? l16 + 16 * q : 71;  // lanes 8-15's fifth element: a harmless repeat
    const int sl = e / 9;
    ekk[q] = e - 9 * sl;
    emu[q] = sl < 2 ? 0 : (sl < 4 ? 3 : (sl < 6 ? 2 : 1));
    etm[q] = sl == 1;
    exb[q] = sl == 3;
    erow[q] = sl == 5 ? lyb : (sl == 7 ? lzb : lrow);
  }
  auto fetch = [&](int t, S (&dst)[5]) {
    const int x = 2 * j + ((par0 + t) & 1);
    const int tm = t > 0 ? t - 1 : T - 1;
    const int xb = x > 0 ? x - 1 : NX - 1;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const size_t site = (size_t)(etm[q] ? tm : t) * S0 + erow[q] + (size_t)(exb[q] ? xb : x);
      dst[q] = U[((size_t)emu[q] * V + site) * 9 + ekk[q]];
    }
  };
  S lr[5], ln[5];
  fetch(t0, lr);
  // FP64: the -t neighbour in(t-1) of step t was the +t neighbour of step
  // t-2 in this compact column, so its -t projection is formed then and
  // carried (qm: for step t, qn: for step t+1), one spinor load less per
  // step (measured faster; in FP32 / FP16 the carried registers cost more
  // than the load, which is reloaded there)
  constexpr bool CARRY = PREC == LQCD_F64;
  half_spinor<R> qm, qn;
  if (CARRY) {
    const int tm = t0 > 0 ? t0 - 1 : T - 1;
    qm = project<0, SG>(load_spinor<S, R>(in, blk<LAYOUT>::base((size_t)tm * H0 + hc, rhs, Vh, ldr), cs));
    const spinor<R> p0 = load_spinor<S, R>(in, blk<LAYOUT>::base((size_t)t0 * H0 + hc, rhs, Vh, ldr), cs);
    qn = project<0, SG>(p0);
    if (XL) put(p0);
  } else if (XL) {
    put(load_spinor<S, R>(in, blk<LAYOUT>::base((size_t)t0 * H0 + hc, rhs, Vh, ldr), cs));
  }
  for (int it = 0; it < pg.Lt; ++it) {
    const int t = t0 + it;
    const int x = 2 * j + ((par0 + t) & 1);
    const size_t hh = (size_t)t * H0 + hc;
    const size_t toffh = (size_t)t * H0;
    if (it + 1 < pg.Lt) fetch(t + 1, ln);
    spinor<R> acc;
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
    // time direction: the +t neighbour in(t+1) of this compact column (with
    // XL at the end of the step: it is the spinor this column puts into LDS
    // for the next step's x neighbours)
    if constexpr (!XL) {
      const int tm = t > 0 ? t - 1 : T - 1, t1 = t + 1 < T ? t + 1 : 0;
      spinor<R> pf = load_spinor<S, R>(in, blk<LAYOUT>::base((size_t)t1 * H0 + hc, rhs, Vh, ldr), cs);
      reconstruct<0, -SG>(acc, colour_mul_r<false>(bc_link<0, S, R>(lr), project<0, -SG>(pf)));
      if (CARRY) {
        reconstruct<0, SG>(acc, colour_mul_r<true>(bc_link<1, S, R>(lr), qm));
        qm = qn;
        qn = project<0, SG>(pf);
      } else {
        spinor<R> pb = load_spinor<S, R>(in, blk<LAYOUT>::base((size_t)tm * H0 + hc, rhs, Vh, ldr), cs);
        reconstruct<0, SG>(acc, colour_mul_r<true>(bc_link<1, S, R>(lr), project<0, SG>(pb)));
      }
    }
    {
      const int xf = x + 1 < NX ? x + 1 : 0, xb = x > 0 ? x - 1 : NX - 1;
      const int jf = xf >> 1, jb = xb >> 1;
      if constexpr (XL) {
        // in(t) of the x neighbours' compact columns: LDS when they belong
        // to this workgroup, else memory
        __syncthreads();  // every column's in(t) is in LDS
        const int cf = jf - jbase, cb = jb - jbase;
        spinor<R> pf, pb;
        if (cf >= 0 && cf < ncw) pf = load_spinor<S, R>(xs, ((size_t)cf * 12) * nrhs + rl, nrhs);
        else pf = load_spinor<S, R>(in, blk<LAYOUT>::base(toffh + row * NXh + jf, rhs, Vh, ldr), cs);
        if (cb >= 0 && cb < ncw) pb = load_spinor<S, R>(xs, ((size_t)cb * 12) * nrhs + rl, nrhs);
        else pb = load_spinor<S, R>(in, blk<LAYOUT>::base(toffh + row * NXh + jb, rhs, Vh, ldr), cs);
        reconstruct<3, -SG>(acc, colour_mul_r<false>(bc_link<2, S, R>(lr), project<3, -SG>(pf)));
        reconstruct<3, SG>(acc, colour_mul_r<true>(bc_link<3, S, R>(lr), project<3, SG>(pb)));
      } else {
        add_hop_pair_bc<3, SG, 2, 3>(acc, in, blk<LAYOUT>::base(toffh + row * NXh + jf, rhs, Vh, ldr),
                                     blk<LAYOUT>::base(toffh + row * NXh + jb, rhs, Vh, ldr), cs, lr, one);
      }
    }
    {
      add_hop_pair_bc<2, SG, 4, 5>(acc, in, blk<LAYOUT>::base(toffh + hyf, rhs, Vh, ldr),
                                        blk<LAYOUT>::base(toffh + hyb, rhs, Vh, ldr), cs, lr, one);
    }
    {
      add_hop_pair_bc<1, SG, 6, 7>(acc, in, blk<LAYOUT>::base(toffh + hzf, rhs, Vh, ldr),
                                        blk<LAYOUT>::base(toffh + hzb, rhs, Vh, ldr), cs, lr, one);
    }
    spinor<R> pnext;  // XL: this column's in(t+1)
    if constexpr (XL) {
      const int tm = t > 0 ? t - 1 : T - 1, t1 = t + 1 < T ? t + 1 : 0;
      pnext = load_spinor<S, R>(in, blk<LAYOUT>::base((size_t)t1 * H0 + hc, rhs, Vh, ldr), cs);
      reconstruct<0, -SG>(acc, colour_mul_r<false>(bc_link<0, S, R>(lr), project<0, -SG>(pnext)));
      if (CARRY) {
        reconstruct<0, SG>(acc, colour_mul_r<true>(bc_link<1, S, R>(lr), qm));
        qm = qn;
        qn = project<0, SG>(pnext);
      } else {
        spinor<R> pb = load_spinor<S, R>(in, blk<LAYOUT>::base((size_t)tm * H0 + hc, rhs, Vh, ldr), cs);
        reconstruct<0, SG>(acc, colour_mul_r<true>(bc_link<1, S, R>(lr), project<0, SG>(pb)));
      }
    }
    const size_t me = blk<LAYOUT>::base(hh, rhs, Vh, ldr);
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
    if (store_me) {
      if (pg.nt) store_spinor_nt<S, R>(out, me, cs, acc);
      else store_spinor<S, R>(out, me, cs, acc);
    }
    if (it + 1 < pg.Lt) {
#pragma unroll
      for (int q = 0; q < 5; ++q) lr[q] = ln[q];
      if constexpr (XL) {
        __syncthreads();  // every column has read its x neighbours at t
        put(pnext);
      }
    }
  }
}

// ------------------------------------------------------------- launchers
// x neighbours through LDS (variant 7): the workgroup's columns are whole
// and consecutive in x (256 / nrhs of them within one tile row of x)
// rhs per workgroup chunk of the full apply: FP64 blocks wider than 16 rhs
// run in chunks of 16 (a time slice's working set is that of 16 rhs; a
// chunk's share of a site component is 256 contiguous bytes, whole cache
// lines), measured 3 % faster at 32 rhs and 7.5 % at 64 on 32^3x64.  In
// FP32 / FP16 a chunk's share is 128 / 64 bytes, so a chunk leaves cache
// lines half used until the next chunk and chunking measured slower; the
// odd-even passes gain nothing measurable, so they run the block at once.
template <int PREC>
static int rhs_chunk(int nrhs) {
  return PREC == LQCD_F64 && nrhs > 16 ? 16 : nrhs;
}

static bool xl_fits(const pencil_geo& pg, int nrhs) {
  if (256 % nrhs) return false;
  const int ncw = 256 / nrhs;
  const size_t items = (size_t)pg.TX * pg.TY * pg.TZ * nrhs;
  return ncw >= 2 && pg.TX % ncw == 0 && items % 256 == 0;
}

template <int PREC, int LAYOUT, int SG>
static hipError_t go_full(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                          double hopc, const kcfg& c, hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  const int w = rhs_chunk<PREC>(nrhs);
  pencil_geo pg = make_pencil(lat, w, false, c);
  const dim3 grid(pencil_blocks(pg) * (unsigned)(nrhs / w));
  size_t dyn = 0;
  if (c.variant == 7 && xl_fits(pg, w)) {
    if (!occupancy_lds(c.occ, 256 * 12 * sizeof(S), &dyn)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_wilson_full_pb<PREC, LAYOUT, SG, true>), grid, dim3(256), dyn, s, (const S*)U,
                       (const S*)psi, (S*)eta, pg, w, nrhs, (R)diag, (R)hopc);
    return hipSuccess;
  }
  if (!occupancy_lds(c.occ, 0, &dyn)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_wilson_full_pb<PREC, LAYOUT, SG, false>), grid, dim3(256), dyn, s, (const S*)U,
                     (const S*)psi, (S*)eta, pg, w, nrhs, (R)diag, (R)hopc);
  return hipSuccess;
}

template <int PREC, int LAYOUT, int SG>
static hipError_t go_eo(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                        int nrhs, double alpha, double beta, const int* live, const kcfg& c, hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  const int w = nrhs;  // one chunk (see rhs_chunk)
  pencil_geo pg = make_pencil(lat, w, true, c);
  const dim3 grid(pencil_blocks(pg) * (unsigned)(nrhs / w));
  size_t dyn = 0;
  if (c.variant == 7 && xl_fits(pg, w)) {
    if (!occupancy_lds(c.occ, 256 * 12 * sizeof(S), &dyn)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_wilson_eo_pb<PREC, LAYOUT, SG, true>), grid, dim3(256), dyn, s, (const S*)U,
                       (const S*)in, (const S*)xin, (S*)out, pg, p, w, nrhs, (R)alpha, (R)beta, live);
    return hipSuccess;
  }
  if (!occupancy_lds(c.occ, 0, &dyn)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_wilson_eo_pb<PREC, LAYOUT, SG, false>), grid, dim3(256), dyn, s, (const S*)U,
                     (const S*)in, (const S*)xin, (S*)out, pg, p, w, nrhs, (R)alpha, (R)beta, live);
  return hipSuccess;
}

#define LQ_BC_KEY(p, l, d) ((p) * 100 + (l) * 10 + (d))
#define LQ_BC_CASE(P, L, D, FN, ...)                     \
  case LQ_BC_KEY(P, L, D): {                             \
    hipError_t e_ = FN<P, L, (D) ? -1 : 1>(__VA_ARGS__); \
    if (e_ != hipSuccess) return e_;                     \
  } break;
#define LQ_BC_CASES(P, FN, ...)                         \
  LQ_BC_CASE(P, LQCD_LAYOUT1, 0, FN, __VA_ARGS__)       \
  LQ_BC_CASE(P, LQCD_LAYOUT1, 1, FN, __VA_ARGS__)       \
  LQ_BC_CASE(P, LQCD_LAYOUT2, 0, FN, __VA_ARGS__)       \
  LQ_BC_CASE(P, LQCD_LAYOUT2, 1, FN, __VA_ARGS__)
#define LQ_BC_DISPATCH(PREC_, LAYOUT_, DAG_, FN, ...)                                                   \
  do {                                                                                                  \
    switch (LQ_BC_KEY(PREC_, LAYOUT_, DAG_)) {                                                          \
      LQ_BC_CASES(LQCD_F64, FN, __VA_ARGS__) LQ_BC_CASES(LQCD_F32, FN, __VA_ARGS__)                     \
      LQ_BC_CASES(LQCD_F16, FN, __VA_ARGS__)                                                            \
      default: return hipErrorInvalidValue;                                                             \
    }                                                                                                   \
  } while (0)

bool bc_supported(int layout, int nrhs) {
  return (layout == LQCD_LAYOUT1 || layout == LQCD_LAYOUT2) && nrhs % 16 == 0;
}

hipError_t wilson_full_bc(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                          double hopc, int layout, int prec, bool dagger, const kcfg& c, hipStream_t s) {
  if (!bc_supported(layout, nrhs)) return hipErrorInvalidValue;
  LQ_BC_DISPATCH(prec, layout, (dagger ? 1 : 0), go_full, lat, U, psi, eta, nrhs, diag, hopc, c, s);
  return hipGetLastError();
}

hipError_t wilson_eo_bc(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                        int nrhs, double alpha, double beta, int layout, int prec, bool dagger, const int* live,
                        const kcfg& c, hipStream_t s) {
  if (!bc_supported(layout, nrhs)) return hipErrorInvalidValue;
  LQ_BC_DISPATCH(prec, layout, (dagger ? 1 : 0), go_eo, lat, U, in, xin, out, p, nrhs, alpha, beta, live, c, s);
  return hipGetLastError();
}

}  // namespace lq
