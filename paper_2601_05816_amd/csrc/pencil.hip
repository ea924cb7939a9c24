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

// k_wilson_full_pl: links of a step through LDS (body in pencil_kernels.h).
template <int PREC, int LAYOUT, int SG, int NCW>
__global__ __launch_bounds__(256) void k_wilson_full_pl(const typename prec_traits<PREC>::store* __restrict__ U,
                                                        const typename prec_traits<PREC>::store* __restrict__ psi,
                                                        typename prec_traits<PREC>::store* __restrict__ eta,
                                                        pencil_geo pg, int nrhs,
                                                        typename prec_traits<PREC>::real diag,
                                                        typename prec_traits<PREC>::real hopc) {
  __shared__ typename prec_traits<PREC>::store lds_all[4][2][NCW * 63];
  wilson_full_pl_body<PREC, LAYOUT, SG, NCW>(U, psi, eta, pg, nrhs, diag, hopc, blockIdx.x, lds_all);
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
