// Pencil Wilson kernels with NR right-hand sides per work item (rhs-innermost
// layout, FP32 and FP16 storage).  The NR rhs of a component are consecutive
// in memory, so one vector access fetches them all (16 B for two FP32 or four
// FP16 numbers, 8 B for two FP16), and each link is loaded once for NR
// projected half spinors.  The arithmetic per site and rhs is the one of
// pencil.hip.  Needs nrhs % NR == 0.
#include "pencil_kernels.h"

namespace lq {

// k_wilson_eo_pn: one launch over the pencil grid of one lattice (body in pencil_kernels.h).
template <int PREC, int SG, int NR>
__global__ __launch_bounds__(256) void k_wilson_eo_pn(const typename prec_traits<PREC>::store* __restrict__ U,
                                                      const typename prec_traits<PREC>::store* __restrict__ in,
                                                      const typename prec_traits<PREC>::store* __restrict__ xin,
                                                      typename prec_traits<PREC>::store* __restrict__ out,
                                                      pencil_geo pg, int p, int nrhs,
                                                      typename prec_traits<PREC>::real alpha,
                                                      typename prec_traits<PREC>::real beta,
                                                      const int* __restrict__ live) {
  wilson_eo_pn_body<PREC, SG, NR>(U, in, xin, out, pg, p, nrhs, alpha, beta, live, blockIdx.x);
}

// k_wilson_full_pn: one launch over the pencil grid of one lattice (body in pencil_kernels.h).
template <int PREC, int SG, int NR>
__global__ __launch_bounds__(256) void k_wilson_full_pn(const typename prec_traits<PREC>::store* __restrict__ U,
                                                        const typename prec_traits<PREC>::store* __restrict__ psi,
                                                        typename prec_traits<PREC>::store* __restrict__ eta,
                                                        pencil_geo pg, int nrhs,
                                                        typename prec_traits<PREC>::real diag,
                                                        typename prec_traits<PREC>::real hopc) {
  wilson_full_pn_body<PREC, SG, NR>(U, psi, eta, pg, nrhs, diag, hopc, blockIdx.x);
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
