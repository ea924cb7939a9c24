// The odd-even Schur complement in one kernel (Sec. III-A.2):
//   eta_e = d psi_e - (1 / 4d) H_eo H_oe psi_e,   d = 4 + m0,
// where H is the hopping sum of the Wilson operator (without its factor 1/2)
// and D_oo = d.  The two-pass apply writes the odd field H_oe psi_e to HBM and
// reads it back; here it never leaves the compute unit.
//
// A workgroup owns a tile of (y, z) rows, each row holding all compact x
// columns of one (y, z), and a chunk of rw right-hand sides, and walks the
// tile along t.  At every time slice it computes the odd field for its
// interior rows and for the rows one step outside the tile in y and z (the
// halo, recomputed rather than shared with the neighbouring tiles), keeps
// that slice in LDS (two slices, double-buffered), and applies H_eo to it for
// the interior rows.  Along t the odd field of a compact column stays in the
// work item that computes it: the +t neighbour of the even output at t is the
// odd field the item has just computed for t + 1, and the -t neighbour is the
// one it computed two steps earlier, carried as the half spinor
// U_0^dagger (1 + s gamma_0) chi that the -t hop needs.
//
// Column geometry (as in the pencil kernels): compact column j of row (y, z)
// holds x = 2j and 2j + 1; at time t its even site is x_e = 2j + ((t+y+z)&1)
// and its odd site x_e ^ 1.  The odd +-t neighbours of the even site (t, x_e)
// are the odd sites of the same compact column at t +- 1 (same x), and its
// +-y / +-z neighbours are the odd sites of column j in the neighbouring rows.
#include "kernels.h"
#include "pencil.h"

namespace lq {

struct schur_geo {
  int n[4];      // T, Z, Y, X
  size_t V;
  int TY, TZ;    // interior rows of a tile: TY x TZ
  int NTY, NTZ, ntiles;
  int rows;      // rows a workgroup computes the odd field for: interior + 2 TZ + 2 TY
  int NXh;       // compact columns per row
  int rw, nch;   // rhs per workgroup and rhs chunks
  int nseg, Lt;  // t segments and their length
  int items;     // active work items per workgroup: rows * NXh * rw
  int nt;        // non-temporal output stores
};

// Region row r -> offset (iy, iz) from the tile origin; interior rows first,
// then the y halo (iy = -1 and TY), then the z halo (iz = -1 and TZ).
__device__ __forceinline__ void schur_row(const schur_geo& g, int r, int& iy, int& iz) {
  const int ni = g.TY * g.TZ;
  if (r < ni) {
    iy = r % g.TY;
    iz = r / g.TY;
  } else if (r < ni + 2 * g.TZ) {
    const int k = r - ni;
    iy = k < g.TZ ? -1 : g.TY;
    iz = k < g.TZ ? k : k - g.TZ;
  } else {
    const int k = r - ni - 2 * g.TZ;
    iz = k < g.TY ? -1 : g.TZ;
    iy = k < g.TY ? k : k - g.TY;
  }
}

// Inverse of schur_row for the rows an interior row's neighbours sit in.
__device__ __forceinline__ int schur_row_of(const schur_geo& g, int iy, int iz) {
  const int ni = g.TY * g.TZ;
  if (iy >= 0 && iy < g.TY && iz >= 0 && iz < g.TZ) return iz * g.TY + iy;
  if (iy < 0) return ni + iz;
  if (iy >= g.TY) return ni + g.TZ + iz;
  if (iz < 0) return ni + 2 * g.TZ + iy;
  return ni + 2 * g.TZ + g.TY + iy;
}

// acc += H_oe psi_e at the odd site (t, x) of row (y, z), compact column j:
// the eight hopping terms, neighbours read from the even block `in`.
template <int PREC, int LAYOUT, int SG>
__device__ __forceinline__ void odd_hop(const typename prec_traits<PREC>::store* __restrict__ U,
                                        const typename prec_traits<PREC>::store* __restrict__ in, const schur_geo& g,
                                        int nrhs, int rhs, int t, int j, int y, int z,
                                        spinor<typename prec_traits<PREC>::real>& acc) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  const int T = g.n[0], NZ = g.n[1], NY = g.n[2], NX = g.n[3], NXh = g.NXh;
  const size_t V = g.V, Vh = V / 2;
  const size_t S0 = (size_t)NZ * NY * NX, H0 = S0 / 2;
  const int cs = blk<LAYOUT>::cstride(nrhs);
  const size_t row = (size_t)z * NY + y, lrow = row * NX;
  const int x = 2 * j + ((1 + t + y + z) & 1);
  const size_t site = (size_t)t * S0 + lrow + x;
  const size_t toffh = (size_t)t * H0;
  const S* U0 = U;
  const S* U1 = U + 1 * V * 9;
  const S* U2 = U + 2 * V * 9;
  const S* U3 = U + 3 * V * 9;
#pragma unroll
  for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
  // one direction at a time: both neighbours and both links are loaded before
  // either term is accumulated, two hops' loads in flight per wavefront
  const int tm = t > 0 ? t - 1 : T - 1, t1 = t + 1 < T ? t + 1 : 0;
  {
    spinor<R> pf = load_spinor<S, R>(in, blk<LAYOUT>::base((size_t)t1 * H0 + row * NXh + j, rhs, Vh, nrhs), cs);
    su3<R> uf = load_link<S, R>(U0 + site * 9);
    spinor<R> pb = load_spinor<S, R>(in, blk<LAYOUT>::base((size_t)tm * H0 + row * NXh + j, rhs, Vh, nrhs), cs);
    su3<R> ub = load_link<S, R>(U0 + ((size_t)tm * S0 + lrow + x) * 9);
    reconstruct<0, -SG>(acc, colour_mul_r<false>(uf, project<0, -SG>(pf)));
    reconstruct<0, SG>(acc, colour_mul_r<true>(ub, project<0, SG>(pb)));
  }
  {
    const int xf = x + 1 < NX ? x + 1 : 0, xb = x > 0 ? x - 1 : NX - 1;
    spinor<R> pf = load_spinor<S, R>(in, blk<LAYOUT>::base(toffh + row * NXh + (xf >> 1), rhs, Vh, nrhs), cs);
    su3<R> uf = load_link<S, R>(U3 + site * 9);
    spinor<R> pb = load_spinor<S, R>(in, blk<LAYOUT>::base(toffh + row * NXh + (xb >> 1), rhs, Vh, nrhs), cs);
    su3<R> ub = load_link<S, R>(U3 + ((size_t)t * S0 + lrow + xb) * 9);
    reconstruct<3, -SG>(acc, colour_mul_r<false>(uf, project<3, -SG>(pf)));
    reconstruct<3, SG>(acc, colour_mul_r<true>(ub, project<3, SG>(pb)));
  }
  {
    const int yf = y + 1 < NY ? y + 1 : 0, yb = y > 0 ? y - 1 : NY - 1;
    spinor<R> pf =
        load_spinor<S, R>(in, blk<LAYOUT>::base(toffh + ((size_t)z * NY + yf) * NXh + j, rhs, Vh, nrhs), cs);
    su3<R> uf = load_link<S, R>(U2 + site * 9);
    spinor<R> pb =
        load_spinor<S, R>(in, blk<LAYOUT>::base(toffh + ((size_t)z * NY + yb) * NXh + j, rhs, Vh, nrhs), cs);
    su3<R> ub = load_link<S, R>(U2 + ((size_t)t * S0 + ((size_t)z * NY + yb) * NX + x) * 9);
    reconstruct<2, -SG>(acc, colour_mul_r<false>(uf, project<2, -SG>(pf)));
    reconstruct<2, SG>(acc, colour_mul_r<true>(ub, project<2, SG>(pb)));
  }
  {
    const int zf = z + 1 < NZ ? z + 1 : 0, zb = z > 0 ? z - 1 : NZ - 1;
    spinor<R> pf =
        load_spinor<S, R>(in, blk<LAYOUT>::base(toffh + ((size_t)zf * NY + y) * NXh + j, rhs, Vh, nrhs), cs);
    su3<R> uf = load_link<S, R>(U1 + site * 9);
    spinor<R> pb =
        load_spinor<S, R>(in, blk<LAYOUT>::base(toffh + ((size_t)zb * NY + y) * NXh + j, rhs, Vh, nrhs), cs);
    su3<R> ub = load_link<S, R>(U1 + ((size_t)t * S0 + ((size_t)zb * NY + y) * NX + x) * 9);
    reconstruct<1, -SG>(acc, colour_mul_r<false>(uf, project<1, -SG>(pf)));
    reconstruct<1, SG>(acc, colour_mul_r<true>(ub, project<1, SG>(pb)));
  }
}

template <typename S, typename R>
__device__ __forceinline__ spinor<R> lds_spinor(const S* __restrict__ buf, int stride, int off) {
  spinor<R> v;
#pragma unroll
  for (int i = 0; i < 12; ++i) v.c[i / 3][i % 3] = widen(buf[i * stride + off]);
  return v;
}

template <typename S, typename R>
__device__ __forceinline__ void lds_put(S* __restrict__ buf, int stride, int off, const spinor<R>& v) {
#pragma unroll
  for (int i = 0; i < 12; ++i) st(buf + i * stride + off, v.c[i / 3][i % 3]);
}

// eta_e = d in + c H_eo H_oe in on the even half lattice (c = -1 / 4d).
// Dynamic LDS: two slices of the odd field over the workgroup's rows,
// 2 x 12 x rows x NXh x rw storage elements.  Every work item of the
// workgroup reaches every barrier: the loop trip count is the same for all,
// and items beyond `items` only skip the arithmetic.
// Work items per workgroup at most: 256 where the arithmetic needs more than
// half of a SIMD's registers per lane (FP64, and FP16 with its conversions).
template <int PREC>
struct schur_max_items {
  static constexpr int value = PREC == LQCD_F32 ? 512 : 256;
};

template <int PREC, int LAYOUT, int SG>
__global__ __launch_bounds__(schur_max_items<PREC>::value) void k_schur_fused(
    const typename prec_traits<PREC>::store* __restrict__ U, const typename prec_traits<PREC>::store* __restrict__ in,
    typename prec_traits<PREC>::store* __restrict__ out, schur_geo g, int nrhs, typename prec_traits<PREC>::real d,
    typename prec_traits<PREC>::real c, const int* __restrict__ live) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  extern __shared__ unsigned char schur_lds[];
  S* slot0 = (S*)schur_lds;
  const int stride = g.rows * g.NXh * g.rw;  // elements between components of one slice
  S* slot1 = slot0 + 12 * stride;

  // block -> (segment, tile, rhs chunk); XCD k runs a contiguous range of
  // tiles, all rhs chunks of a tile on the same XCD (they share links)
  const unsigned L = xcd_block(blockIdx.x, gridDim.x);
  const int ch = (int)(L % (unsigned)g.nch);
  const unsigned u = L / (unsigned)g.nch;
  const int tile = (int)(u % (unsigned)g.ntiles);
  const int seg = (int)(u / (unsigned)g.ntiles);
  const int ty0 = (tile % g.NTY) * g.TY, tz0 = (tile / g.NTY) * g.TZ;

  const int tin = threadIdx.x;
  const bool act = tin < g.items;
  const int rl = tin % g.rw;
  const int col = act ? tin / g.rw : 0;
  const int j = col % g.NXh, r = col / g.NXh;
  const int rhs = ch * g.rw + rl;
  int iy, iz;
  schur_row(g, r, iy, iz);
  const int T = g.n[0], NZ = g.n[1], NY = g.n[2], NX = g.n[3], NXh = g.NXh;
  const int y = (ty0 + iy + NY) % NY, z = (tz0 + iz + NZ) % NZ;
  const bool inner = act && r < g.TY * g.TZ;
  const bool store_me = inner && (!live || live[rhs]);
  const int me = (r * NXh + j) * g.rw + rl;  // this item's offset in a slice

  // neighbour offsets in a slice (interior rows only)
  int oyf = 0, oyb = 0, ozf = 0, ozb = 0;
  if (inner) {
    oyf = (schur_row_of(g, iy + 1, iz) * NXh + j) * g.rw + rl;
    oyb = (schur_row_of(g, iy - 1, iz) * NXh + j) * g.rw + rl;
    ozf = (schur_row_of(g, iy, iz + 1) * NXh + j) * g.rw + rl;
    ozb = (schur_row_of(g, iy, iz - 1) * NXh + j) * g.rw + rl;
  }
  const size_t V = g.V, Vh = V / 2;
  const size_t S0 = (size_t)NZ * NY * NX, H0 = S0 / 2;
  const size_t row = (size_t)z * NY + y, lrow = row * NX;
  const size_t lyb = ((size_t)z * NY + (y > 0 ? y - 1 : NY - 1)) * NX;
  const size_t lzb = ((size_t)(z > 0 ? z - 1 : NZ - 1) * NY + y) * NX;
  const int cs = blk<LAYOUT>::cstride(nrhs);
  const S* U0 = U;
  const S* U1 = U + 1 * V * 9;
  const S* U2 = U + 2 * V * 9;
  const S* U3 = U + 3 * V * 9;
  const int t0 = seg * g.Lt;

  // prologue: the carried -t terms of the outputs at t0 and t0 + 1, and the
  // odd slice t0 in LDS slot 0
  half_spinor<R> cA, cB;
  {
    spinor<R> o;
    if (inner) {
      const int tm = t0 > 0 ? t0 - 1 : T - 1;
      odd_hop<PREC, LAYOUT, SG>(U, in, g, nrhs, rhs, tm, j, y, z, o);
      const int x = 2 * j + ((1 + tm + y + z) & 1);
      cA = colour_mul_r<true>(load_link<S, R>(U0 + ((size_t)tm * S0 + lrow + x) * 9), project<0, SG>(o));
    }
    if (act) {
      odd_hop<PREC, LAYOUT, SG>(U, in, g, nrhs, rhs, t0, j, y, z, o);
      lds_put<S, R>(slot0, stride, me, o);
      if (inner) {
        const int x = 2 * j + ((1 + t0 + y + z) & 1);
        cB = colour_mul_r<true>(load_link<S, R>(U0 + ((size_t)t0 * S0 + lrow + x) * 9), project<0, SG>(o));
      }
    }
  }
  __syncthreads();

  for (int it = 0; it < g.Lt; ++it) {
    const int t = t0 + it;
    const int t1 = t + 1 < T ? t + 1 : 0;
    S* cur = (it & 1) ? slot1 : slot0;
    S* nxt = (it & 1) ? slot0 : slot1;
    spinor<R> acc;
    if (act) {
      // odd field at t + 1: into the other slot (its previous slice, t - 1,
      // was last read before the barrier that ended the previous step)
      spinor<R> on;
      odd_hop<PREC, LAYOUT, SG>(U, in, g, nrhs, rhs, t1, j, y, z, on);
      if (it + 1 < g.Lt) lds_put<S, R>(nxt, stride, me, on);
      if (inner) {
        const int e = (t + y + z) & 1;
        const int xe = 2 * j + e;
        const size_t site = (size_t)t * S0 + lrow + xe;
#pragma unroll
        for (int i = 0; i < 12; ++i) acc.c[i / 3][i % 3] = {R(0), R(0)};
        // +t: the odd field just computed; -t: carried from two steps back
        reconstruct<0, -SG>(acc, colour_mul_r<false>(load_link<S, R>(U0 + site * 9), project<0, -SG>(on)));
        reconstruct<0, SG>(acc, cA);
        cA = cB;
        cB = colour_mul_r<true>(load_link<S, R>(U0 + ((size_t)t1 * S0 + lrow + xe) * 9), project<0, SG>(on));
      }
    }
    if (inner) {
      const int e = (t + y + z) & 1;
      const int xe = 2 * j + e;
      const size_t site = (size_t)t * S0 + lrow + xe;
      const int xb = xe > 0 ? xe - 1 : NX - 1;
      const int jf = e ? (j + 1 < NXh ? j + 1 : 0) : j;  // compact column of x_e + 1
      const int jb = e ? j : (j > 0 ? j - 1 : NXh - 1);  // compact column of x_e - 1
      const int ox = (r * NXh) * g.rw + rl;
      {
        spinor<R> pf = lds_spinor<S, R>(cur, stride, ox + jf * g.rw);
        su3<R> uf = load_link<S, R>(U3 + site * 9);
        spinor<R> pb = lds_spinor<S, R>(cur, stride, ox + jb * g.rw);
        su3<R> ub = load_link<S, R>(U3 + ((size_t)t * S0 + lrow + xb) * 9);
        reconstruct<3, -SG>(acc, colour_mul_r<false>(uf, project<3, -SG>(pf)));
        reconstruct<3, SG>(acc, colour_mul_r<true>(ub, project<3, SG>(pb)));
      }
      {
        spinor<R> pf = lds_spinor<S, R>(cur, stride, oyf);
        su3<R> uf = load_link<S, R>(U2 + site * 9);
        spinor<R> pb = lds_spinor<S, R>(cur, stride, oyb);
        su3<R> ub = load_link<S, R>(U2 + ((size_t)t * S0 + lyb + xe) * 9);
        reconstruct<2, -SG>(acc, colour_mul_r<false>(uf, project<2, -SG>(pf)));
        reconstruct<2, SG>(acc, colour_mul_r<true>(ub, project<2, SG>(pb)));
      }
      {
        spinor<R> pf = lds_spinor<S, R>(cur, stride, ozf);
        su3<R> uf = load_link<S, R>(U1 + site * 9);
        spinor<R> pb = lds_spinor<S, R>(cur, stride, ozb);
        su3<R> ub = load_link<S, R>(U1 + ((size_t)t * S0 + lzb + xe) * 9);
        reconstruct<1, -SG>(acc, colour_mul_r<false>(uf, project<1, -SG>(pf)));
        reconstruct<1, SG>(acc, colour_mul_r<true>(ub, project<1, SG>(pb)));
      }
      const size_t hb = blk<LAYOUT>::base((size_t)t * H0 + row * NXh + j, rhs, Vh, nrhs);
      spinor<R> xv = load_spinor<S, R>(in, hb, cs);
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        cx<R> a = acc.c[i / 3][i % 3], b = xv.c[i / 3][i % 3];
        acc.c[i / 3][i % 3] = {fma(c, a.re, d * b.re), fma(c, a.im, d * b.im)};
      }
      if (store_me) {
        if (g.nt) store_spinor_nt<S, R>(out, hb, cs, acc);
        else store_spinor<S, R>(out, hb, cs, acc);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ host
static int lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 64 * 1024;
  return v;
}
static int lds_per_cu() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || v <= 0)
    return 64 * 1024;
  return v;
}

static size_t schur_lds_bytes(const schur_geo& g, size_t esz) {
  return 2 * 12 * (size_t)g.rows * g.NXh * g.rw * esz;
}

// Geometry for configuration c: tile (c.ty, c.tz; 0 = the largest of 4x4,
// 4x2, 2x2, 2x1, 1x1 that fits), t segments c.nseg (0 = 1), and as many rhs
// per workgroup (a power of two dividing nrhs) as fit max_items work items
// and the LDS share of c.occ workgroups per compute unit (0 = 1).  False when
// no tile fits.
static bool make_schur(const lqcd_lattice* lat, int nrhs, const kcfg& c, size_t esz, int max_items,
                       schur_geo& g) {
  for (int i = 0; i < 4; ++i) g.n[i] = lat->dims[i];
  const int T = g.n[0], NZ = g.n[1], NY = g.n[2], NX = g.n[3];
  g.V = (size_t)T * NZ * NY * NX;
  g.NXh = NX / 2;
  g.nt = c.nt;
  const int occ = c.occ > 0 ? c.occ : 1;
  const size_t budget = std::min((size_t)lds_per_block(), (size_t)lds_per_cu() / (size_t)occ);
  static const int kAuto[][2] = {{4, 4}, {4, 2}, {2, 2}, {2, 1}, {1, 1}};
  int cand[5][2];
  int nc = 0;
  if (c.ty > 0 && c.tz > 0) {
    cand[0][0] = c.ty;
    cand[0][1] = c.tz;
    nc = 1;
  } else {
    for (auto& k : kAuto) {
      cand[nc][0] = k[0];
      cand[nc][1] = k[1];
      ++nc;
    }
  }
  for (int k = 0; k < nc; ++k) {
    const int TY = cand[k][0], TZ = cand[k][1];
    if (NY % TY || NZ % TZ) continue;
    g.TY = TY;
    g.TZ = TZ;
    g.rows = TY * TZ + 2 * TZ + 2 * TY;
    g.rw = 0;
    for (int rw = 1; rw <= nrhs; rw *= 2) {
      if (nrhs % rw) break;
      g.rw = rw;
      if ((size_t)g.rows * g.NXh * rw > (size_t)max_items || schur_lds_bytes(g, esz) > budget) {
        g.rw = rw / 2;
        break;
      }
    }
    if (g.rw < 1) continue;
    g.nch = nrhs / g.rw;
    g.items = g.rows * g.NXh * g.rw;
    g.NTY = NY / TY;
    g.NTZ = NZ / TZ;
    g.ntiles = g.NTY * g.NTZ;
    g.nseg = (c.nseg > 0 && T % c.nseg == 0) ? c.nseg : 1;
    g.Lt = T / g.nseg;
    return true;
  }
  return false;
}

template <int PREC, int LAYOUT, int SG>
static hipError_t go_schur(const lqcd_lattice* lat, const void* U, const void* in, void* out, int nrhs, double d,
                           const int* live, const kcfg& c, hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  schur_geo g;
  if (!make_schur(lat, nrhs, c, sizeof(S), schur_max_items<PREC>::value, g)) return hipErrorInvalidConfiguration;
  const unsigned blocks = (unsigned)g.ntiles * (unsigned)g.nch * (unsigned)g.nseg;
  const unsigned threads = (unsigned)((g.items + 63) / 64 * 64);
  const size_t lds = schur_lds_bytes(g, sizeof(S));
  hipLaunchKernelGGL((k_schur_fused<PREC, LAYOUT, SG>), dim3(blocks), dim3(threads), lds, s, (const S*)U,
                     (const S*)in, (S*)out, g, nrhs, (R)d, (R)(-0.25 / d), live);
  return hipGetLastError();
}

#define LQ_KEY(p, l, dg) ((p) * 100 + (l) * 10 + (dg))
#define LQ_SCASE(P, L, D, ...) \
  case LQ_KEY(P, L, D): return go_schur<P, L, (D) ? -1 : 1>(__VA_ARGS__);
#define LQ_SCASES_L(P, D, ...)                 \
  LQ_SCASE(P, LQCD_RHS_OUTER, D, __VA_ARGS__)  \
  LQ_SCASE(P, LQCD_LAYOUT1, D, __VA_ARGS__)    \
  LQ_SCASE(P, LQCD_LAYOUT2, D, __VA_ARGS__)

bool schur_fused_supported(const lqcd_lattice* lat, int nrhs, int prec, const kcfg& c) {
  schur_geo g;
  const size_t esz = prec == LQCD_F64 ? 16 : prec == LQCD_F32 ? 8 : 4;
  const int max_items = prec == LQCD_F64   ? schur_max_items<LQCD_F64>::value
                        : prec == LQCD_F32 ? schur_max_items<LQCD_F32>::value
                                           : schur_max_items<LQCD_F16>::value;
  return make_schur(lat, nrhs, c, esz, max_items, g);
}

hipError_t schur_fused(const lqcd_lattice* lat, const void* U, const void* in, void* out, int nrhs, double d,
                       int layout, int prec, bool dagger, const int* live, const kcfg& c, hipStream_t s) {
  switch (LQ_KEY(prec, layout, dagger ? 1 : 0)) {
    LQ_SCASES_L(LQCD_F64, 0, lat, U, in, out, nrhs, d, live, c, s)
    LQ_SCASES_L(LQCD_F64, 1, lat, U, in, out, nrhs, d, live, c, s)
    LQ_SCASES_L(LQCD_F32, 0, lat, U, in, out, nrhs, d, live, c, s)
    LQ_SCASES_L(LQCD_F32, 1, lat, U, in, out, nrhs, d, live, c, s)
    LQ_SCASES_L(LQCD_F16, 0, lat, U, in, out, nrhs, d, live, c, s)
    LQ_SCASES_L(LQCD_F16, 1, lat, U, in, out, nrhs, d, live, c, s)
    default: return hipErrorInvalidValue;
  }
}

// The Schur apply the library runs everywhere: the fused kernel when the
// configuration for this problem (forced, or the tuner's entry for the whole
// apply) selects it and the lattice fits, else the two hop passes through
// the odd temporary `tmp` (which the fused kernel does not touch).
hipError_t schur_apply(const lqcd_lattice* lat, const void* U, const void* in, void* out, void* tmp, int nrhs,
                       double d, int layout, int prec, bool dagger, const int* live, hipStream_t s) {
  const kcfg c = choose_cfg(KIND_SCHUR, lat, nrhs, prec, layout);
  if (c.variant == 8 && schur_fused_supported(lat, nrhs, prec, c))
    return schur_fused(lat, U, in, out, nrhs, d, layout, prec, dagger, live, c, s);
  hipError_t e = wilson_eo(lat, U, in, nullptr, tmp, 1, nrhs, 0.0, 1.0, layout, prec, dagger, live, s);
  if (e != hipSuccess) return e;
  return wilson_eo(lat, U, tmp, in, out, 0, nrhs, d, -0.25 / d, layout, prec, dagger, live, s);
}

}  // namespace lq
