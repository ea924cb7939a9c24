// Time-streaming Wilson kernel fed by asynchronous global-to-LDS loads.
//
// Same walk as the pencil kernels (a work item owns one spatial column and
// one rhs and steps along t; the time-direction neighbours stay in
// registers), but the seven spinors a step needs (six spatial neighbours and
// psi(t+1)) and the link of each hop are fetched with global_load_lds: the
// data lands in a wave-private ring of LDS slots without occupying vector
// registers, so a wavefront keeps NSLOT - 1 hops in flight while it computes
// the current one.  With register-destination loads the compiler drains the
// memory counter once per hop, which leaves one wavefront per SIMD waiting
// on seven dependent round trips per step.
//
// Fetch k (k = 7 * step + hop) goes to slot k mod NSLOT.  Loads complete in
// issue order, so "fetch k has landed" is s_waitcnt vmcnt(n) with n the
// number of load instructions issued after it: 13 per later fetch (twelve
// spinor components and one link element per lane).  Output stores also
// count in vmcnt; they are issued after some of the fetches being waited
// on, which can only make a wait longer, never shorter.
//
// LDS per wavefront: NSLOT x (12 x 64 + 64) complex elements.  For FP64 and
// NSLOT = 3 a workgroup of four wavefronts takes 156 KiB, one workgroup per
// compute unit, the residency at which an XCD's L2 serves the spatial
// neighbours of its tile.  FP64 storage only (one complex element = one
// 16-byte transfer per lane), rhs-innermost layout, nrhs >= 11.
#include "kernels.h"
#include "pencil.h"

namespace lq {

typedef __attribute__((address_space(3))) void lds_void_t;

// lane i of the wavefront copies its 16-byte element *g to l[i] (l wave-uniform)
__device__ __forceinline__ void dma(const double2* g, double2* l) {
  __builtin_amdgcn_global_load_lds((const void*)g, (lds_void_t*)l, 16, 0, 0);
}

template <int N>
__device__ __forceinline__ void wait_vm() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

typedef double d2v_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned lds_addr(const void* p) {
  return (unsigned)(size_t)(const __attribute__((address_space(3))) void*)p;
}

// Read a lane's 12 spinor components (stride 1 KiB) and a 3x3 link (stride
// 16 B) from LDS.  Written as assembly with its own wait so that the
// compiler, which cannot tell which global-to-LDS transfer a read depends
// on, does not drain every transfer in flight before it (the explicit
// vmcnt waits above order the reads after the transfers they need).  The
// outputs are early-clobber: a read's destination must not reuse the
// address register that the following reads of the block still need.
__device__ __forceinline__ void lds_spinor(unsigned a, spinor<double>& p) {
  d2v_t r0, r1, r2, r3, r4, r5, r6, r7, r8, r9, r10, r11;
  asm volatile(
      "ds_read_b128 %0, %12\n\t"
      "ds_read_b128 %1, %12 offset:1024\n\t"
      "ds_read_b128 %2, %12 offset:2048\n\t"
      "ds_read_b128 %3, %12 offset:3072\n\t"
      "ds_read_b128 %4, %12 offset:4096\n\t"
      "ds_read_b128 %5, %12 offset:5120\n\t"
      "ds_read_b128 %6, %12 offset:6144\n\t"
      "ds_read_b128 %7, %12 offset:7168\n\t"
      "ds_read_b128 %8, %12 offset:8192\n\t"
      "ds_read_b128 %9, %12 offset:9216\n\t"
      "ds_read_b128 %10, %12 offset:10240\n\t"
      "ds_read_b128 %11, %12 offset:11264\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7), "=&v"(r8),
        "=&v"(r9), "=&v"(r10), "=&v"(r11)
      : "v"(a)
      : "memory");
  const d2v_t r[12] = {r0, r1, r2, r3, r4, r5, r6, r7, r8, r9, r10, r11};
#pragma unroll
  for (int c = 0; c < 12; ++c) p.c[c / 3][c % 3] = {r[c].x, r[c].y};
}

__device__ __forceinline__ void lds_link(unsigned a, su3<double>& w) {
  d2v_t r0, r1, r2, r3, r4, r5, r6, r7, r8;
  asm volatile(
      "ds_read_b128 %0, %9\n\t"
      "ds_read_b128 %1, %9 offset:16\n\t"
      "ds_read_b128 %2, %9 offset:32\n\t"
      "ds_read_b128 %3, %9 offset:48\n\t"
      "ds_read_b128 %4, %9 offset:64\n\t"
      "ds_read_b128 %5, %9 offset:80\n\t"
      "ds_read_b128 %6, %9 offset:96\n\t"
      "ds_read_b128 %7, %9 offset:112\n\t"
      "ds_read_b128 %8, %9 offset:128\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7), "=&v"(r8)
      : "v"(a)
      : "memory");
  const d2v_t r[9] = {r0, r1, r2, r3, r4, r5, r6, r7, r8};
#pragma unroll
  for (int i = 0; i < 9; ++i) w.m[i / 3][i % 3] = {r[i].x, r[i].y};
}

template <int MU, int T, bool ADJ, typename R>
__device__ __forceinline__ void add_hop_r(spinor<R>& acc, const spinor<R>& p, const su3<R>& u, R c) {
  reconstruct<MU, T>(acc, hscale(c, colour_mul_r<ADJ>(u, project<MU, T>(p))));
}

// Addresses one lane needs: its own column's neighbour columns (spinors)
// and the column of the link entry it fetches for the wavefront.
struct dma_lane {
  size_t cxf, cxb, cyf, cyb, czf, czb, c0;  // spinor columns (site numbers at t = 0)
  size_t l0, lxb, lyb, lzb;                 // link columns
  int lkk;                                  // link entry 0..8
};

// Issue fetch of hop H (0..5: +x, -x, +y, -y, +z, -z; 6: psi(t+1) and U_0)
// for time slice t into `slot`: 12 spinor transfers and 1 link transfer.
template <int H>
__device__ __forceinline__ void dma_issue(const double2* __restrict__ U, const double2* __restrict__ psi,
                                          double2* slot, const dma_lane& g, int t, int T, size_t S0, size_t V,
                                          int rhs, int nrhs, size_t cstride) {
  constexpr int SP = 12 * 64;
  const size_t toff = (size_t)t * S0;
  size_t sn, ls;
  int mu;
  if (H == 0) { sn = g.cxf; mu = 3; ls = g.l0; }
  if (H == 1) { sn = g.cxb; mu = 3; ls = g.lxb; }
  if (H == 2) { sn = g.cyf; mu = 2; ls = g.l0; }
  if (H == 3) { sn = g.cyb; mu = 2; ls = g.lyb; }
  if (H == 4) { sn = g.czf; mu = 1; ls = g.l0; }
  if (H == 5) { sn = g.czb; mu = 1; ls = g.lzb; }
  if (H == 6) { sn = g.c0; mu = 0; ls = g.l0; }
  const size_t sofs = H == 6 ? (size_t)(t + 1 < T ? t + 1 : 0) * S0 : toff;
  const double2* src = psi + (sn + sofs) * 12u * (size_t)nrhs + (size_t)rhs;
#pragma unroll
  for (int c = 0; c < 12; ++c) dma(src + (size_t)c * cstride, slot + c * 64);
  dma(U + ((size_t)mu * V + ls + toff) * 9 + g.lkk, slot + SP);
}

template <int SG, int NSLOT>
__global__ __launch_bounds__(256) void k_wilson_full_dma(const double2* __restrict__ U,
                                                         const double2* __restrict__ psi,
                                                         double2* __restrict__ eta, pencil_geo pg, int nrhs,
                                                         double diag, double hopc) {
  typedef double2 S;
  typedef double R;
  constexpr int SP = 12 * 64;  // spinor elements of a slot
  constexpr int SL = SP + 64;  // plus one link element per lane
  constexpr int PER_FETCH = 13;
  static_assert(PER_FETCH * (NSLOT - 1) <= 63, "vmcnt field is 6 bits");
  __shared__ S lds_all[4][NSLOT * SL];

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
  if (tw0 >= CT * (unsigned)nrhs) return;  // whole wavefront idle
  const unsigned colw0 = tw0 / nrhs;
  unsigned colw1 = (tw0 + 63u) / nrhs;
  if (colw1 > CT - 1) colw1 = CT - 1;
  const int ncw = (int)(colw1 - colw0 + 1);  // columns of this wavefront (9 * ncw <= 64)
  // idle lanes of a partly idle wavefront still issue every load (valid
  // addresses of the wavefront's first column) so that the per-fetch
  // instruction count is the same for all; they store nothing
  const bool active = tin < CT * (unsigned)nrhs;
  const unsigned col = active ? tin / nrhs : colw0;
  const int rhs = (int)(tin % nrhs);
  const int cl = (int)(col - colw0);
  S* lds = lds_all[wave];

  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  const int tx = tile % pg.NTX, ty = (tile / pg.NTX) % pg.NTY, tz = tile / (pg.NTX * pg.NTY);
  const int t0 = (int)seg * pg.Lt;
  const size_t V = pg.V, S0 = (size_t)NZ * NY * NX;
  dma_lane g;
  {
    const int x = tx * pg.TX + (int)(col % pg.TX);
    const int y = ty * pg.TY + (int)((col / pg.TX) % pg.TY);
    const int z = tz * pg.TZ + (int)(col / (pg.TX * pg.TY));
    g.c0 = ((size_t)z * NY + y) * NX + x;
    g.cxf = g.c0 - x + (x + 1 < NX ? x + 1 : 0);
    g.cxb = g.c0 - x + (x > 0 ? x - 1 : NX - 1);
    g.cyf = g.c0 + (size_t)((y + 1 < NY ? y + 1 : 0) - y) * NX;
    g.cyb = g.c0 + (size_t)((y > 0 ? y - 1 : NY - 1) - y) * NX;
    g.czf = g.c0 + (size_t)((z + 1 < NZ ? z + 1 : 0) - z) * NY * NX;
    g.czb = g.c0 + (size_t)((z > 0 ? z - 1 : NZ - 1) - z) * NY * NX;
    // link entry of this lane: column lane / 9 of the wavefront, entry lane % 9
    const int le = (int)lane < 9 * ncw ? (int)lane : 0;
    const unsigned lc = colw0 + (unsigned)(le / 9);
    g.lkk = le % 9;
    const int lx = tx * pg.TX + (int)(lc % pg.TX);
    const int ly = ty * pg.TY + (int)((lc / pg.TX) % pg.TY);
    const int lz = tz * pg.TZ + (int)(lc / (pg.TX * pg.TY));
    g.l0 = ((size_t)lz * NY + ly) * NX + lx;
    g.lxb = g.l0 - lx + (lx > 0 ? lx - 1 : NX - 1);
    g.lyb = g.l0 + (size_t)((ly > 0 ? ly - 1 : NY - 1) - ly) * NX;
    g.lzb = g.l0 + (size_t)((lz > 0 ? lz - 1 : NZ - 1) - lz) * NY * NX;
  }
  const size_t me = g.c0 * 12u * (size_t)nrhs + (size_t)rhs;  // own element at t = 0
  const size_t tstride = S0 * 12u * (size_t)nrhs;

  // prologue (plain loads): the -t hop of t0 and the projected centre of t0
  spinor<R> acc;
  half_spinor<R> hplus;
  {
    const int tm = t0 > 0 ? t0 - 1 : T - 1;
    spinor<R> pm = load_spinor<S, R>(psi, me + (size_t)tm * tstride, nrhs);
#pragma unroll
    for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
    add_hop_r<0, SG, true, R>(acc, pm, load_link<S, R>(U + ((size_t)tm * S0 + g.c0) * 9), hopc);
    spinor<R> p0 = load_spinor<S, R>(psi, me + (size_t)t0 * tstride, nrhs);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      cx<R> a = acc.c[i / 3][i % 3], bb = p0.c[i / 3][i % 3];
      acc.c[i / 3][i % 3] = {fma(diag, bb.re, a.re), fma(diag, bb.im, a.im)};
    }
    hplus = project<0, SG>(p0);
  }
  wait_vm<0>();  // the fetch accounting below starts from an empty counter

  // ring of NSLOT fetches: fetch k = 7 * step + hop lives in slot k mod NSLOT
  const int K = 7 * pg.Lt;
  int s_take = 0, s_issue = 0;  // slot of the next fetch to consume / to issue
  // issue fetch (t, hop HOP) into the next issue slot; HOP is a constant
  // once the hop loop below is unrolled
#define LQ_ISSUE(HOP, TT)                                                        \
  do {                                                                           \
    S* sl_ = lds + s_issue * SL;                                                 \
    switch (HOP) {                                                               \
      case 0: dma_issue<0>(U, psi, sl_, g, (TT), T, S0, V, rhs, nrhs, cstr); break;    \
      case 1: dma_issue<1>(U, psi, sl_, g, (TT), T, S0, V, rhs, nrhs, cstr); break;    \
      case 2: dma_issue<2>(U, psi, sl_, g, (TT), T, S0, V, rhs, nrhs, cstr); break;    \
      case 3: dma_issue<3>(U, psi, sl_, g, (TT), T, S0, V, rhs, nrhs, cstr); break;    \
      case 4: dma_issue<4>(U, psi, sl_, g, (TT), T, S0, V, rhs, nrhs, cstr); break;    \
      case 5: dma_issue<5>(U, psi, sl_, g, (TT), T, S0, V, rhs, nrhs, cstr); break;    \
      default: dma_issue<6>(U, psi, sl_, g, (TT), T, S0, V, rhs, nrhs, cstr); break;   \
    }                                                                            \
    s_issue = s_issue + 1 == NSLOT ? 0 : s_issue + 1;                            \
  } while (0)
  size_t cstr = (size_t)nrhs;  // component stride (elements)
#pragma unroll
  for (int i = 0; i < NSLOT; ++i)
    if (i < K) LQ_ISSUE(i % 7, t0 + i / 7);

  for (int it = 0; it < pg.Lt; ++it) {
    // opaque copies of the time slice and the component stride: keep the
    // compiler from hoisting the 91 transfer addresses of a step out of the
    // loop (they would occupy ~180 registers)
    int tcur = t0 + it;
    asm volatile("" : "+s"(tcur), "+s"(cstr));
    spinor<R> p;
    su3<R> w;
    // one hop per iteration, not unrolled: a hop's spinor and link are dead
    // once its term is accumulated
#pragma unroll 1
    for (int h = 0; h < 7; ++h) {
      // wait for fetch k = 7 it + h: every later fetch already issued is
      // 13 load instructions younger
      const int k = 7 * it + h;
      if (k + NSLOT - 1 < K) wait_vm<PER_FETCH * (NSLOT - 1)>();
      else wait_vm<0>();
      const unsigned sa = lds_addr(lds + s_take * SL);
      lds_spinor(sa + lane * 16u, p);
      lds_link(sa + (unsigned)(SP + cl * 9) * 16u, w);  // reads complete: the slot can be refilled
      s_take = s_take + 1 == NSLOT ? 0 : s_take + 1;
      if (k + NSLOT < K) {
        const int hn = h + NSLOT;
        LQ_ISSUE(hn >= 7 ? hn - 7 : hn, tcur + (hn >= 7 ? 1 : 0));
      }
      switch (h) {
        case 0: add_hop_r<3, -SG, false, R>(acc, p, w, hopc); break;
        case 1: add_hop_r<3, SG, true, R>(acc, p, w, hopc); break;
        case 2: add_hop_r<2, -SG, false, R>(acc, p, w, hopc); break;
        case 3: add_hop_r<2, SG, true, R>(acc, p, w, hopc); break;
        case 4: add_hop_r<1, -SG, false, R>(acc, p, w, hopc); break;
        case 5: add_hop_r<1, SG, true, R>(acc, p, w, hopc); break;
        default: add_hop_r<0, -SG, false, R>(acc, p, w, hopc); break;  // psi(t+1), U_0(x)
      }
    }
    const size_t mine = me + (size_t)(t0 + it) * tstride;
    if (active) {
      if (pg.nt) store_spinor_nt<S, R>(eta, mine, nrhs, acc);
      else store_spinor<S, R>(eta, mine, nrhs, acc);
    }
    if (it + 1 < pg.Lt) {
#pragma unroll
      for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = scale(diag, p.c[i / 3][i % 3]);
      reconstruct<0, SG>(acc, hscale(hopc, colour_mul_r<true>(w, hplus)));
      hplus = project<0, SG>(p);
    }
  }
#undef LQ_ISSUE
}

// ---------------------------------------------------------------- launchers
bool dma_supported(int prec, int layout, int nrhs) {
  // one link element per lane: 9 entries for each column a wavefront
  // touches, at most 1 + ceil(63 / nrhs) columns for 64 consecutive items
  if (prec != LQCD_F64 || layout != LQCD_LAYOUT2 || nrhs < 1) return false;
  const int ncw = 1 + (63 + nrhs - 1) / nrhs;
  return 9 * ncw <= 64;
}

template <int SG, int NSLOT>
static void go_full_dma(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                        double hopc, const kcfg& c, hipStream_t s) {
  pencil_geo pg = make_pencil(lat, nrhs, false, c);
  hipLaunchKernelGGL((k_wilson_full_dma<SG, NSLOT>), dim3(pencil_blocks(pg)), dim3(256), 0, s, (const double2*)U,
                     (const double2*)psi, (double2*)eta, pg, nrhs, diag, hopc);
}

hipError_t wilson_full_dma(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                           double hopc, int prec, bool dagger, const kcfg& c, hipStream_t s) {
  // FP64 only: one complex element is one 16-byte LDS transfer per lane (the
  // 8-byte transfer an FP32 complex would need does not exist)
  if (prec != LQCD_F64) return hipErrorInvalidValue;
  if (dagger) go_full_dma<-1, 3>(lat, U, psi, eta, nrhs, diag, hopc, c, s);
  else go_full_dma<1, 3>(lat, U, psi, eta, nrhs, diag, hopc, c, s);
  return hipGetLastError();
}

}  // namespace lq
