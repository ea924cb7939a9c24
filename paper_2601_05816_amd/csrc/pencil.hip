// Wilson-Dirac kernels that stream along the time direction ("pencils").
//
// A work item owns one spatial column (z, y, x) and one rhs and walks a
// segment of t values.  The +t neighbour loaded for site t is the centre of
// site t+1 and the -t neighbour of site t+2, so each spinor along t is read
// once and its three uses (Algorithm 1: the diagonal term and the two
// time-direction hops) are served from registers; only
// the six spatial neighbours go through the caches.  The time link U_0(x) is
// shared between the +t hop of site t and the -t hop of site t+1.
//
// Columns are grouped into tiles (TX x TY x TZ).  Workgroup b runs on XCD
// b mod 8 (the dispatcher's round-robin); the eight workgroups of a "tile
// group" at the same position of the dispatch order therefore work on eight
// adjacent tiles at the same time, so that a tile's spatial halo is the
// interior of a tile that another XCD reads in the same time step.  Within
// an XCD the tile's workgroups cover the tile's columns and rhs.  With
// several t segments the order is segment-major: all tile groups of segment
// 0, then of segment 1, ..., so a tile group's z halo at the same t range was
// read by the previous group shortly before (an Infinity Cache hit rather
// than an HBM read).  The mapping is a bijection for any tile shape; the tile
// shape and the number of t segments only change locality.
#include "kernels.h"
#include "pencil_kernels.h"

namespace lq {

// k_wilson_full_p: one launch over the pencil grid of one lattice (body in pencil_kernels.h).
template <int PREC, int LAYOUT, int SG>
__global__ __launch_bounds__(256) void k_wilson_full_p(const typename prec_traits<PREC>::store* __restrict__ U,
                                                       const typename prec_traits<PREC>::store* __restrict__ psi,
                                                       typename prec_traits<PREC>::store* __restrict__ eta,
                                                       pencil_geo pg, int nrhs,
                                                       typename prec_traits<PREC>::real diag,
                                                       typename prec_traits<PREC>::real hopc) {
  wilson_full_p_body<PREC, LAYOUT, SG>(U, psi, eta, pg, nrhs, diag, hopc, blockIdx.x);
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
template <int PREC, int LAYOUT, int SG, int NCW>
__global__ __launch_bounds__(256) void k_wilson_full_pl(const typename prec_traits<PREC>::store* __restrict__ U,
                                                        const typename prec_traits<PREC>::store* __restrict__ psi,
                                                        typename prec_traits<PREC>::store* __restrict__ eta,
                                                        pencil_geo pg, int nrhs,
                                                        typename prec_traits<PREC>::real diag,
                                                        typename prec_traits<PREC>::real hopc) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  constexpr int NEL = NCW * 63;            // link elements of a wavefront and step
  constexpr int NE = (NEL + 63) / 64;      // per lane
  __shared__ S lds_all[4][2][NEL];
  const unsigned b = blockIdx.x;
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

// k_wilson_eo_p: one launch over the pencil grid of one lattice (body in pencil_kernels.h).
template <int PREC, int LAYOUT, int SG>
__global__ __launch_bounds__(256) void k_wilson_eo_p(const typename prec_traits<PREC>::store* __restrict__ U,
                                                     const typename prec_traits<PREC>::store* __restrict__ in,
                                                     const typename prec_traits<PREC>::store* __restrict__ xin,
                                                     typename prec_traits<PREC>::store* __restrict__ out,
                                                     pencil_geo pg, int p, int nrhs,
                                                     typename prec_traits<PREC>::real alpha,
                                                     typename prec_traits<PREC>::real beta,
                                                     const int* __restrict__ live) {
  wilson_eo_p_body<PREC, LAYOUT, SG>(U, in, xin, out, pg, p, nrhs, alpha, beta, live, blockIdx.x);
}

// Clover-improved operator D = D_W - C on the same pencil grid (body in
// pencil_kernels.h with the clover epilogue).  The odd-even clover passes
// stay on the one-(site, rhs)-per-work-item kernels: with the clover
// product added, the pencil version of those passes measured slower.
template <int PREC, int LAYOUT, int SG>
__global__ __launch_bounds__(256) void k_wilson_full_pcl(const typename prec_traits<PREC>::store* __restrict__ U,
                                                         const typename prec_traits<PREC>::store* __restrict__ C,
                                                         const typename prec_traits<PREC>::store* __restrict__ psi,
                                                         typename prec_traits<PREC>::store* __restrict__ eta,
                                                         pencil_geo pg, int nrhs,
                                                         typename prec_traits<PREC>::real diag,
                                                         typename prec_traits<PREC>::real hopc) {
  wilson_full_p_body<PREC, LAYOUT, SG, true>(U, psi, eta, pg, nrhs, diag, hopc, blockIdx.x, C);
}

// ------------------------------------------------------------ configuration
bool occupancy_lds(int occ, size_t static_bytes, size_t* dyn_bytes) {
  *dyn_bytes = 0;
  if (occ <= 0) return true;
  int dev = 0, per_cu = 0, per_wg = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      per_cu <= 0)
    per_cu = 160 * 1024;
  if (hipDeviceGetAttribute(&per_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || per_wg <= 0)
    per_wg = 64 * 1024;
  // allocation granularity is 512 bytes; occ + 1 requests must overflow the CU
  size_t want = ((size_t)per_cu / (size_t)(occ + 1) + 512) & ~(size_t)511;
  if (want * (size_t)occ > (size_t)per_cu || want > (size_t)per_wg) return false;
  *dyn_bytes = want > static_bytes ? want - static_bytes : 0;
  return true;
}

template <int PREC, int LAYOUT, int SG>
static hipError_t launch_full_p(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs,
                                double diag, double hopc, const kcfg& c, hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  pencil_geo pg = make_pencil(lat, nrhs, false, c);
  const dim3 grid(pencil_blocks(pg)), blk(256);
  size_t dyn = 0;
  if (LAYOUT != LQCD_RHS_OUTER && c.variant == 2 && nrhs >= 4) {
    const int ncw = nrhs >= 16 ? 5 : (nrhs >= 8 ? 9 : 17);
    if (!occupancy_lds(c.occ, 8 * (size_t)ncw * 63 * sizeof(S), &dyn)) return hipErrorInvalidConfiguration;
    if (nrhs >= 16)
      hipLaunchKernelGGL((k_wilson_full_pl<PREC, LAYOUT, SG, 5>), grid, blk, dyn, s, (const S*)U, (const S*)psi,
                         (S*)eta, pg, nrhs, (R)diag, (R)hopc);
    else if (nrhs >= 8)
      hipLaunchKernelGGL((k_wilson_full_pl<PREC, LAYOUT, SG, 9>), grid, blk, dyn, s, (const S*)U, (const S*)psi,
                         (S*)eta, pg, nrhs, (R)diag, (R)hopc);
    else
      hipLaunchKernelGGL((k_wilson_full_pl<PREC, LAYOUT, SG, 17>), grid, blk, dyn, s, (const S*)U, (const S*)psi,
                         (S*)eta, pg, nrhs, (R)diag, (R)hopc);
    return hipSuccess;
  }
  if (!occupancy_lds(c.occ, 0, &dyn)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_wilson_full_p<PREC, LAYOUT, SG>), grid, blk, dyn, s, (const S*)U, (const S*)psi, (S*)eta,
                     pg, nrhs, (R)diag, (R)hopc);
  return hipSuccess;
}

template <int PREC, int LAYOUT, int SG>
static hipError_t launch_eo_p(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out,
                              int p, int nrhs, double alpha, double beta, const int* live, const kcfg& c,
                              hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  pencil_geo pg = make_pencil(lat, nrhs, true, c);
  size_t dyn = 0;
  if (!occupancy_lds(c.occ, 0, &dyn)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_wilson_eo_p<PREC, LAYOUT, SG>), dim3(pencil_blocks(pg)), dim3(256), dyn, s, (const S*)U,
                     (const S*)in, (const S*)xin, (S*)out, pg, p, nrhs, (R)alpha, (R)beta, live);
  return hipSuccess;
}

template <int PREC, int LAYOUT, int SG>
static hipError_t launch_full_pcl(const lqcd_lattice* lat, const void* U, const void* C, const void* psi, void* eta,
                                  int nrhs, double diag, double hopc, const kcfg& c, hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  pencil_geo pg = make_pencil(lat, nrhs, false, c);
  size_t dyn = 0;
  if (!occupancy_lds(c.occ, 0, &dyn)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_wilson_full_pcl<PREC, LAYOUT, SG>), dim3(pencil_blocks(pg)), dim3(256), dyn, s, (const S*)U,
                     (const S*)C, (const S*)psi, (S*)eta, pg, nrhs, (R)diag, (R)hopc);
  return hipSuccess;
}

#define LQ_KEY(p, l, d) ((p) * 100 + (l) * 10 + (d))
#define LQ_CASE(P, L, D, FN, ...) \
  case LQ_KEY(P, L, D): {                                \
    hipError_t e_ = FN<P, L, (D) ? -1 : 1>(__VA_ARGS__);  \
    if (e_ != hipSuccess) return e_;                     \
  } break;
#define LQ_CASES_L(P, D, FN, ...)                   \
  LQ_CASE(P, LQCD_RHS_OUTER, D, FN, __VA_ARGS__)    \
  LQ_CASE(P, LQCD_LAYOUT1, D, FN, __VA_ARGS__)      \
  LQ_CASE(P, LQCD_LAYOUT2, D, FN, __VA_ARGS__)
#define LQ_DISPATCH(PREC_, LAYOUT_, DAG_, FN, ...)                                         \
  do {                                                                                     \
    switch (LQ_KEY(PREC_, LAYOUT_, DAG_)) {                                                \
      LQ_CASES_L(LQCD_F64, 0, FN, __VA_ARGS__) LQ_CASES_L(LQCD_F64, 1, FN, __VA_ARGS__)    \
      LQ_CASES_L(LQCD_F32, 0, FN, __VA_ARGS__) LQ_CASES_L(LQCD_F32, 1, FN, __VA_ARGS__)    \
      LQ_CASES_L(LQCD_F16, 0, FN, __VA_ARGS__) LQ_CASES_L(LQCD_F16, 1, FN, __VA_ARGS__)    \
      default: return hipErrorInvalidValue;                                                \
    }                                                                                      \
  } while (0)

hipError_t wilson_full_pencil(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs,
                              double diag, double hopc, int layout, int prec, bool dagger, const kcfg& c,
                              hipStream_t s) {
  LQ_DISPATCH(prec, layout, (dagger ? 1 : 0), launch_full_p, lat, U, psi, eta, nrhs, diag, hopc, c, s);
  return hipGetLastError();
}

hipError_t wilson_eo_pencil(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out,
                            int p, int nrhs, double alpha, double beta, int layout, int prec, bool dagger,
                            const int* live, const kcfg& c, hipStream_t s) {
  LQ_DISPATCH(prec, layout, (dagger ? 1 : 0), launch_eo_p, lat, U, in, xin, out, p, nrhs, alpha, beta, live, c, s);
  return hipGetLastError();
}

hipError_t wilson_full_clover_pencil(const lqcd_lattice* lat, const void* U, const void* C, const void* psi,
                                     void* eta, int nrhs, double diag, double hopc, int layout, int prec, bool dagger,
                                     const kcfg& c, hipStream_t s) {
  LQ_DISPATCH(prec, layout, (dagger ? 1 : 0), launch_full_pcl, lat, U, C, psi, eta, nrhs, diag, hopc, c, s);
  return hipGetLastError();
}

}  // namespace lq
