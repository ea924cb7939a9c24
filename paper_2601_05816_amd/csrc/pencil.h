// Shared pieces of the time-streaming ("pencil") Wilson kernels.
#pragma once

#include <type_traits>

#include "kernels.h"
#include "wilson.h"

namespace lq {

struct pencil_geo {
  int n[4];          // N0 = T, N1 = Z, N2 = Y, N3 = X
  size_t V;
  int TX, TY, TZ;    // column tile (in columns; TX counts compact columns for eo)
  int NTX, NTY, NTZ; // tiles per direction
  int nseg, Lt;      // t segments and their length
  int bpt;           // workgroups per tile and segment
  int ntiles;
  int nt;            // non-temporal output stores
  float one;         // 1, as a run-time value (the FMA form of load_project)
};

// (column coordinates, rhs, t0) of work item threadIdx.x of block b of the
// pencil grid, or false if idle.
template <int LAYOUT>
__device__ __forceinline__ bool pencil_item(const pencil_geo& pg, int nrhs, int& x, int& y, int& z, int& rhs,
                                            int& t0, unsigned b) {
  const unsigned k = b & 7u, i = b >> 3;
  const unsigned u = i / pg.bpt, q = i % pg.bpt;
  const unsigned ngrp = (unsigned)(pg.ntiles + 7) / 8u;
  const unsigned seg = u / ngrp, grp = u % ngrp;  // segment-major: tile groups of one t segment run back to back
  const unsigned tile = grp * 8u + k;
  if (tile >= (unsigned)pg.ntiles) return false;
  const unsigned CT = (unsigned)pg.TX * pg.TY * pg.TZ;
  const unsigned tin = q * blockDim.x + threadIdx.x;
  if (tin >= CT * (unsigned)nrhs) return false;
  unsigned col;
  if (LAYOUT == LQCD_RHS_OUTER) {
    rhs = (int)(tin / CT);
    col = tin % CT;
  } else {
    col = tin / nrhs;
    rhs = (int)(tin % nrhs);
  }
  const int tx = tile % pg.NTX, ty = (tile / pg.NTX) % pg.NTY, tz = tile / (pg.NTX * pg.NTY);
  x = tx * pg.TX + (int)(col % pg.TX);
  y = ty * pg.TY + (int)((col / pg.TX) % pg.TY);
  z = tz * pg.TZ + (int)(col / (pg.TX * pg.TY));
  t0 = (int)seg * pg.Lt;
  return true;
}

template <typename R>
__device__ __forceinline__ half_spinor<R> hscale(R s, half_spinor<R> h) {
#pragma unroll
  for (int i = 0; i < 6; ++i) h.c[i / 3][i % 3] = scale(s, h.c[i / 3][i % 3]);
  return h;
}

// acc += c * (hop term of direction MU with projector sign T) for a loaded
// neighbour p and link u (ADJ: use u^dagger)
template <int MU, int T, bool ADJ, typename S, typename R>
__device__ __forceinline__ void add_hop(spinor<R>& acc, const spinor<R>& p, const S* __restrict__ u, R c) {
  half_spinor<R> h = project<MU, T>(p);
  reconstruct<MU, T>(acc, hscale(c, colour_mul<ADJ>(u, h)));
}

// The same for the neighbour stored at p[base + i cs] (i = 0..11).  FP16
// storage projects the loaded values directly (load_project, no separate
// conversions); FP32 / FP64 widen the spinor first, the form their kernels
// were tuned with.
template <int MU, int T, bool ADJ, typename S, typename R>
__device__ __forceinline__ void add_hop_at(spinor<R>& acc, const S* p, size_t base, int cs, const S* u, R c, R one) {
  if constexpr (std::is_same<S, h2_t>::value) {
    reconstruct<MU, T>(acc, hscale(c, colour_mul<ADJ>(u, load_project<MU, T>(p, base, cs, one))));
  } else {
    spinor<R> v = load_spinor<S, R>(p, base, cs);
    add_hop<MU, T, ADJ, S, R>(acc, v, u, c);
  }
}

// acc += both hop terms of direction MU (sign SG): the forward neighbour at
// in[fb + i cs] with U_MU(x) at uf and the backward one at in[bb + i cs]
// with U_MU(x - MU)^dagger at ub; both neighbours and links are loaded
// before either term is accumulated.  FP16 storage projects as add_hop_at.
template <int MU, int SG, typename S, typename R>
__device__ __forceinline__ void add_hop_pair(spinor<R>& acc, const S* in, size_t fb, size_t bb, int cs, const S* uf,
                                             const S* ub, R one) {
  if constexpr (std::is_same<S, h2_t>::value) {
    half_spinor<R> hf = load_project<MU, -SG>(in, fb, cs, one);
    su3<R> mf = load_link<S, R>(uf);
    half_spinor<R> hb = load_project<MU, SG>(in, bb, cs, one);
    su3<R> mb = load_link<S, R>(ub);
    reconstruct<MU, -SG>(acc, colour_mul_r<false>(mf, hf));
    reconstruct<MU, SG>(acc, colour_mul_r<true>(mb, hb));
  } else {
    spinor<R> pf = load_spinor<S, R>(in, fb, cs);
    su3<R> mf = load_link<S, R>(uf);
    spinor<R> pb = load_spinor<S, R>(in, bb, cs);
    su3<R> mb = load_link<S, R>(ub);
    reconstruct<MU, -SG>(acc, colour_mul_r<false>(mf, project<MU, -SG>(pf)));
    reconstruct<MU, SG>(acc, colour_mul_r<true>(mb, project<MU, SG>(pb)));
  }
}

inline int largest_divisor_at_most(int n, int cap) {
  if (cap < 1) cap = 1;
  for (int d = cap < n ? cap : n; d >= 1; --d)
    if (n % d == 0) return d;
  return 1;
}

// Tile: all of X, then as much of Y and Z as one XCD keeps resident (about
// 16384 work items), but no fewer than eight tiles when the lattice allows;
// segments: enough work items for several waves of residency on the whole
// chip.  Entries of c that are > 0 and divide the
// lattice override the automatic choice.
inline pencil_geo make_pencil(const lqcd_lattice* lat, int nrhs, bool eo, const kcfg& c) {
  pencil_geo pg;
  for (int i = 0; i < 4; ++i) pg.n[i] = lat->dims[i];
  pg.V = (size_t)pg.n[0] * pg.n[1] * pg.n[2] * pg.n[3];
  const int T = pg.n[0], NZ = pg.n[1], NY = pg.n[2], NX = pg.n[3];
  pg.TX = eo ? NX / 2 : NX;
  const int target_cols = (16384 / nrhs) > 0 ? 16384 / nrhs : 1;
  int rest = target_cols / pg.TX;
  if (rest < 1) rest = 1;
  const bool auto_y = !(c.ty > 0 && NY % c.ty == 0), auto_z = !(c.tz > 0 && NZ % c.tz == 0);
  int TY = auto_y ? largest_divisor_at_most(NY, rest) : c.ty;
  int TZ = auto_z ? largest_divisor_at_most(NZ, rest / TY) : c.tz;
  // automatic tiles: at least one tile per XCD where the lattice allows it
  // (a small lattice would otherwise fit one tile and leave seven XCDs idle)
  while ((NY / TY) * (NZ / TZ) < 8) {
    if (auto_z && TZ > 1 && (TZ >= TY || !auto_y)) TZ = largest_divisor_at_most(NZ, TZ / 2);
    else if (auto_y && TY > 1) TY = largest_divisor_at_most(NY, TY / 2);
    else break;
  }
  pg.TY = TY;
  pg.TZ = TZ;
  pg.NTX = 1;
  pg.NTY = NY / TY;
  pg.NTZ = NZ / TZ;
  pg.ntiles = pg.NTY * pg.NTZ;
  const size_t cols = (size_t)pg.TX * NY * NZ;
  int nseg = 1;
  if (c.nseg > 0 && T % c.nseg == 0) {
    nseg = c.nseg;
  } else {
    const size_t want = 524288;
    while (nseg < T && cols * (size_t)nrhs * nseg < want) {
      int next = nseg + 1;
      while (next < T && T % next) ++next;
      nseg = next;
    }
  }
  pg.nseg = nseg;
  pg.Lt = T / nseg;
  const size_t items = (size_t)pg.TX * TY * TZ * nrhs;
  pg.bpt = (int)((items + 255) / 256);
  pg.nt = c.nt;
  pg.one = 1.0f;
  return pg;
}

// Dynamic LDS bytes that cap residency at `occ` workgroups per compute unit
// for a kernel with `static_bytes` of its own LDS: each workgroup asks for a
// little more than 1/(occ+1) of the compute unit's LDS.  occ = 0: no cap.
// Returns false if the cap cannot be expressed on this device (a workgroup
// may not request that much LDS).
bool occupancy_lds(int occ, size_t static_bytes, size_t* dyn_bytes);

inline unsigned pencil_blocks(const pencil_geo& pg) {
  const unsigned ngroups = (unsigned)((pg.ntiles + 7) / 8);
  return ngroups * 8u * (unsigned)pg.nseg * (unsigned)pg.bpt;
}

}  // namespace lq
