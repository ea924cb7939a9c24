// Wilson-Dirac kernels: the full-lattice operator on a block of rhs and the
// odd-even hopping half-operator with an axpy epilogue.
//
// One work item = one (site, rhs) pair; the rhs index runs fastest in LAYOUT2
// and LAYOUT1 so that the 12 components of neighbouring rhs are contiguous
// (LAYOUT2) and a site's links are fetched once per wavefront-row and served
// from cache to all rhs of that site (Sec. III-A.1: the rhs loop fused into the
// site loop so that U is not revisited per rhs).  Algorithm 1's separate
// passes (diagonal, projections, halo, accumulation) collapse into one pass:
// each work item reads its 8 neighbour spinors and 8 links, projects,
// multiplies and reconstructs in registers, and writes its output once.
#include "kernels.h"
#include "site.h"

namespace lq {

// ------------------------------------------------------------ full lattice
template <int PREC, int LAYOUT, int SG>
__global__ __launch_bounds__(256) void k_wilson_full(const typename prec_traits<PREC>::store* __restrict__ U,
                                                     const typename prec_traits<PREC>::store* __restrict__ psi,
                                                     typename prec_traits<PREC>::store* __restrict__ eta, geo4 g,
                                                     int nrhs, typename prec_traits<PREC>::real diag,
                                                     typename prec_traits<PREC>::real hopc) {
  const size_t t = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= g.V * (size_t)nrhs) return;
  size_t site;
  int rhs;
  blk<LAYOUT>::item(t, g.V, nrhs, site, rhs);
  wilson_full_site<PREC, LAYOUT, SG>(U, psi, eta, g, nrhs, diag, hopc, site, rhs);
}

// --------------------------------------------------------- odd-even hop
// out(h) = alpha * xin(h) + beta * hop(in)(h) for the parity-p sites h, where
// `in` is a parity (1-p) compact block.  xin may be null (alpha ignored).
// `live` (nullable, per rhs) masks right-hand sides that need no update.
template <int PREC, int LAYOUT, int SG>
__global__ __launch_bounds__(256) void k_wilson_eo(const typename prec_traits<PREC>::store* __restrict__ U,
                                                   const typename prec_traits<PREC>::store* __restrict__ in,
                                                   const typename prec_traits<PREC>::store* __restrict__ xin,
                                                   typename prec_traits<PREC>::store* __restrict__ out, geo4 g, int p,
                                                   int nrhs, typename prec_traits<PREC>::real alpha,
                                                   typename prec_traits<PREC>::real beta,
                                                   const int* __restrict__ live) {
  const size_t Vh = g.V / 2;
  const size_t t = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= Vh * (size_t)nrhs) return;
  size_t h;
  int rhs;
  blk<LAYOUT>::item(t, Vh, nrhs, h, rhs);
  if (live && !live[rhs]) return;
  wilson_eo_site<PREC, LAYOUT, SG>(U, in, xin, out, g, p, nrhs, alpha, beta, h, rhs);
}

// ------------------------------------------------------------- launchers
static inline unsigned nblocks(size_t items, unsigned bs) { return (unsigned)((items + bs - 1) / bs); }

template <int PREC, int LAYOUT, int SG>
static void launch_full(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                        double hopc, hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  geo4 g = make_geo(lat);
  const size_t items = g.V * (size_t)nrhs;
  hipLaunchKernelGGL((k_wilson_full<PREC, LAYOUT, SG>), dim3(nblocks(items, 256)), dim3(256), 0, s,
                     (const S*)U, (const S*)psi, (S*)eta, g, nrhs, (R)diag, (R)hopc);
}

template <int PREC, int LAYOUT, int SG>
static void launch_eo(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                      int nrhs, double alpha, double beta, const int* live, hipStream_t s) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  geo4 g = make_geo(lat);
  const size_t items = g.V / 2 * (size_t)nrhs;
  hipLaunchKernelGGL((k_wilson_eo<PREC, LAYOUT, SG>), dim3(nblocks(items, 256)), dim3(256), 0, s, (const S*)U,
                     (const S*)in, (const S*)xin, (S*)out, g, p, nrhs, (R)alpha, (R)beta, live);
}

#define LQ_KEY(p, l, d) ((p) * 100 + (l) * 10 + (d))
#define LQ_CASE(P, L, D, FN, ...) \
  case LQ_KEY(P, L, D): FN<P, L, (D) ? -1 : 1>(__VA_ARGS__); break;
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

// DAG_ = 1 selects D^dagger (hopping sign SG = -1)
hipError_t wilson_full(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                       double hopc, int layout, int prec, bool dagger, hipStream_t s) {
  kcfg c = choose_cfg(KIND_FULL, lat, nrhs, prec, layout);
  if (c.variant == 8) c.variant = 7;
  if (c.variant == 6 || c.variant == 7) {
    if (bc_supported(layout, nrhs)) return wilson_full_bc(lat, U, psi, eta, nrhs, diag, hopc, layout, prec, dagger, c, s);
    c.variant = 3;
  }
  if (c.variant == 5) {
    if (dma_supported(prec, layout, nrhs)) return wilson_full_dma(lat, U, psi, eta, nrhs, diag, hopc, prec, dagger, c, s);
    c.variant = 3;
  }
  if (c.variant == 4) {
    if (nr_supported(prec, layout, nrhs)) return wilson_full_nr(lat, U, psi, eta, nrhs, diag, hopc, prec, dagger, c, s);
    c.variant = 3;
  }
  if (c.variant >= 2) return wilson_full_pencil(lat, U, psi, eta, nrhs, diag, hopc, layout, prec, dagger, c, s);
  LQ_DISPATCH(prec, layout, (dagger ? 1 : 0), launch_full, lat, U, psi, eta, nrhs, diag, hopc, s);
  return hipGetLastError();
}

hipError_t wilson_eo(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                     int nrhs, double alpha, double beta, int layout, int prec, bool dagger, const int* live,
                     hipStream_t s) {
  kcfg c = choose_cfg(KIND_EO, lat, nrhs, prec, layout);
  if (c.variant == 8) c.variant = 7;
  if (c.variant == 6 || c.variant == 7) {
    if (bc_supported(layout, nrhs))
      return wilson_eo_bc(lat, U, in, xin, out, p, nrhs, alpha, beta, layout, prec, dagger, live, c, s);
    c.variant = 3;
  }
  if (c.variant == 5) c.variant = 3;
  if (c.variant == 4) {
    if (nr_supported(prec, layout, nrhs))
      return wilson_eo_nr(lat, U, in, xin, out, p, nrhs, alpha, beta, prec, dagger, live, c, s);
    c.variant = 3;
  }
  if (c.variant >= 2)
    return wilson_eo_pencil(lat, U, in, xin, out, p, nrhs, alpha, beta, layout, prec, dagger, live, c, s);
  LQ_DISPATCH(prec, layout, (dagger ? 1 : 0), launch_eo, lat, U, in, xin, out, p, nrhs, alpha, beta, live, s);
  return hipGetLastError();
}

}  // namespace lq
