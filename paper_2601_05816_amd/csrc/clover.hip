// The improved operator D = D_W - C with a clover field (Sec. III-A.1, the
// equation after eq. (1); Algorithm 1 applies C together with the diagonal):
// the full apply, the site-local inverse of D_oo = (4 + m0) - C_o, and the
// odd-even Schur complement S = D_ee - D_eo D_oo^{-1} D_oe with a
// site-dependent D_oo.  The full apply takes the kernel kind chosen for the
// plain operator (time-streaming pencils or one (site, rhs) per work item,
// both with the clover epilogue); the odd-even passes run one (site, rhs) per
// work item.  The clover field is read once per site and rhs (an L1/L2 hit
// for the other rhs of the site in the rhs-innermost layouts).
#include <stdint.h>

#include "kernels.h"
#include "site.h"

namespace lq {

int fail(int code, const char* fmt, ...);
int check_lattice(const lqcd_lattice* lat);
int check_block(int nrhs, int layout, int prec);
int hip_status(hipError_t e, const char* what);

template <int PREC, int LAYOUT, int SG>
__global__ __launch_bounds__(256) void k_wilson_full_cl(const typename prec_traits<PREC>::store* __restrict__ U,
                                                        const typename prec_traits<PREC>::store* __restrict__ C,
                                                        const typename prec_traits<PREC>::store* __restrict__ psi,
                                                        typename prec_traits<PREC>::store* __restrict__ eta, geo4 g,
                                                        int nrhs, typename prec_traits<PREC>::real diag,
                                                        typename prec_traits<PREC>::real hopc) {
  const size_t t = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= g.V * (size_t)nrhs) return;
  size_t site;
  int rhs;
  blk<LAYOUT>::item(t, g.V, nrhs, site, rhs);
  wilson_full_site<PREC, LAYOUT, SG, true>(U, psi, eta, g, nrhs, diag, hopc, site, rhs, C);
}

template <int PREC, int LAYOUT, int SG>
__global__ __launch_bounds__(256) void k_wilson_eo_cl(const typename prec_traits<PREC>::store* __restrict__ U,
                                                      const typename prec_traits<PREC>::store* __restrict__ in,
                                                      const typename prec_traits<PREC>::store* __restrict__ xin,
                                                      typename prec_traits<PREC>::store* __restrict__ out, geo4 g,
                                                      int p, int nrhs, typename prec_traits<PREC>::real alpha,
                                                      typename prec_traits<PREC>::real beta,
                                                      const int* __restrict__ live,
                                                      const typename prec_traits<PREC>::store* __restrict__ Cx,
                                                      const typename prec_traits<PREC>::store* __restrict__ Cout) {
  const size_t Vh = g.V / 2;
  const size_t t = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= Vh * (size_t)nrhs) return;
  size_t h;
  int rhs;
  blk<LAYOUT>::item(t, Vh, nrhs, h, rhs);
  if (live && !live[rhs]) return;
  wilson_eo_site<PREC, LAYOUT, SG, true>(U, in, xin, out, g, p, nrhs, alpha, beta, h, rhs, Cx, Cout);
}

// out(h) = alpha Cm(x) in(h) on the parity-p compact sites h (x the site of h)
template <int PREC, int LAYOUT>
__global__ __launch_bounds__(256) void k_clover_site_mul(const typename prec_traits<PREC>::store* __restrict__ Cm,
                                                         const typename prec_traits<PREC>::store* __restrict__ in,
                                                         typename prec_traits<PREC>::store* __restrict__ out, geo4 g,
                                                         int p, int nrhs, typename prec_traits<PREC>::real alpha) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  const size_t Vh = g.V / 2;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Vh * (size_t)nrhs) return;
  size_t h;
  int rhs;
  blk<LAYOUT>::item(t, Vh, nrhs, h, rhs);
  const int n1 = g.n[1], n2 = g.n[2], n3 = g.n[3], nh3 = n3 >> 1;
  size_t r = h;
  const int j = (int)(r % nh3); r /= nh3;
  const int x2 = (int)(r % n2); r /= n2;
  const int x1 = (int)(r % n1);
  const int x0 = (int)(r / n1);
  const size_t site = ((size_t)(x0 * n1 + x1) * n2 + x2) * n3 + 2 * j + ((p + x0 + x1 + x2) & 1);
  const int cs = blk<LAYOUT>::cstride(nrhs);
  const size_t me = blk<LAYOUT>::base(h, rhs, Vh, nrhs);
  spinor<R> v = clover_mul<S, R>(Cm + site * 42, load_spinor<S, R>(in, me, cs));
#pragma unroll
  for (int i = 0; i < 12; ++i) v.c[i / 3][i % 3] = scale(alpha, v.c[i / 3][i % 3]);
  store_spinor<S, R>(out, me, cs, v);
}

__device__ __forceinline__ cx<double> up64(cx<double> a) { return a; }
__device__ __forceinline__ cx<double> up64(cx<float> a) { return {(double)a.re, (double)a.im}; }
__device__ __forceinline__ cx<double> cmul(cx<double> a, cx<double> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// Cinv(x) = packed ((d I - C(x)) blocks)^{-1}: one thread per (site, block),
// Gauss-Jordan with partial pivoting in FP64 whatever the storage; a pivot
// below 1e-13 d in magnitude sets *singular.
template <int PREC>
__global__ __launch_bounds__(256) void k_clover_invert(const typename prec_traits<PREC>::store* __restrict__ C,
                                                       typename prec_traits<PREC>::store* __restrict__ Cinv,
                                                       size_t V, double d, int* __restrict__ singular) {
  typedef typename prec_traits<PREC>::store S;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * V) return;
  const S* a = C + (t >> 1) * 42 + 21 * (t & 1);
  S* o = Cinv + (t >> 1) * 42 + 21 * (t & 1);
  const double tiny = (1e-13 * d) * (1e-13 * d);
  cx<double> m[6][12];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 12; ++j) m[i][j] = {0.0, 0.0};
  int k = 6;
  for (int i = 0; i < 6; ++i) {
    const cx<double> di = up64(ld(a + i));
    m[i][i] = {d - di.re, 0.0};
    m[i][6 + i] = {1.0, 0.0};
  }
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j, ++k) {
      const cx<double> u = up64(ld(a + k));
      m[i][j] = {-u.re, -u.im};
      m[j][i] = {-u.re, u.im};
    }
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    double best = m[c][c].re * m[c][c].re + m[c][c].im * m[c][c].im;
    for (int r = c + 1; r < 6; ++r) {
      const double n = m[r][c].re * m[r][c].re + m[r][c].im * m[r][c].im;
      if (n > best) {
        best = n;
        piv = r;
      }
    }
    if (!(best > tiny)) {  // |pivot| below 1e-13 d, or NaN
      *singular = 1;
      return;
    }
    if (piv != c)
      for (int j = 0; j < 12; ++j) {
        const cx<double> tmp = m[c][j];
        m[c][j] = m[piv][j];
        m[piv][j] = tmp;
      }
    const cx<double> pv = m[c][c];
    const cx<double> inv = {pv.re / best, -pv.im / best};  // 1 / pv
    for (int j = 0; j < 12; ++j) m[c][j] = cmul(m[c][j], inv);
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const cx<double> f = m[r][c];
      for (int j = 0; j < 12; ++j) m[r][j] = m[r][j] - cmul(f, m[c][j]);
    }
  }
  typedef typename prec_traits<PREC>::real R;
  k = 6;
  for (int i = 0; i < 6; ++i) st(o + i, cx<R>{(R)m[i][6 + i].re, R(0)});
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j, ++k) st(o + k, cx<R>{(R)m[i][6 + j].re, (R)m[i][6 + j].im});
}

// ------------------------------------------------------------- launchers
static inline unsigned nblk(size_t items) { return (unsigned)((items + 255) / 256); }

#define CL_KEY(p, l, d) ((p) * 100 + (l) * 10 + (d))
#define CL_CASE(P, L, D, ...)                        \
  case CL_KEY(P, L, D): {                            \
    constexpr int PP = P, LL = L, SS = (D) ? -1 : 1; \
    typedef typename prec_traits<PP>::store S;       \
    typedef typename prec_traits<PP>::real R;        \
    __VA_ARGS__;                                     \
  } break;
#define CL_CASES_L(P, D, ...)                                                          \
  CL_CASE(P, LQCD_RHS_OUTER, D, __VA_ARGS__) CL_CASE(P, LQCD_LAYOUT1, D, __VA_ARGS__) \
  CL_CASE(P, LQCD_LAYOUT2, D, __VA_ARGS__)
#define CL_DISPATCH(PREC_, LAYOUT_, DAG_, ...)                                                         \
  switch (CL_KEY(PREC_, LAYOUT_, DAG_)) {                                                              \
    CL_CASES_L(LQCD_F64, 0, __VA_ARGS__) CL_CASES_L(LQCD_F64, 1, __VA_ARGS__)                          \
    CL_CASES_L(LQCD_F32, 0, __VA_ARGS__) CL_CASES_L(LQCD_F32, 1, __VA_ARGS__)                          \
    CL_CASES_L(LQCD_F16, 0, __VA_ARGS__) CL_CASES_L(LQCD_F16, 1, __VA_ARGS__)                          \
    default: return hipErrorInvalidValue;                                                              \
  }

// The full clover apply runs on the pencil kernel whenever the configuration
// chosen for the plain operator of the same problem is a pencil one (the
// clover epilogue adds one site-local block product per site and rhs), else
// on the one-(site, rhs)-per-work-item kernel.  The odd-even passes always
// take the latter (measured faster there at 32^3 x 64, 16 rhs, FP64).
hipError_t wilson_full_clover(const lqcd_lattice* lat, const void* U, const void* C, const void* psi, void* eta,
                              int nrhs, double diag, double hopc, int layout, int prec, bool dagger, hipStream_t s) {
  kcfg c = choose_cfg(KIND_FULL, lat, nrhs, prec, layout);
  if (c.variant >= 2) {
    c.variant = 3;
    return wilson_full_clover_pencil(lat, U, C, psi, eta, nrhs, diag, hopc, layout, prec, dagger, c, s);
  }
  const geo4 g = make_geo(lat);
  CL_DISPATCH(prec, layout, (dagger ? 1 : 0),
              hipLaunchKernelGGL((k_wilson_full_cl<PP, LL, SS>), dim3(nblk(g.V * (size_t)nrhs)), dim3(256), 0, s,
                                 (const S*)U, (const S*)C, (const S*)psi, (S*)eta, g, nrhs, (R)diag, (R)hopc))
  return hipGetLastError();
}

hipError_t wilson_eo_clover(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                            int nrhs, double alpha, double beta, int layout, int prec, bool dagger, const int* live,
                            const void* Cx, const void* Cout, hipStream_t s) {
  const geo4 g = make_geo(lat);
  CL_DISPATCH(prec, layout, (dagger ? 1 : 0),
              hipLaunchKernelGGL((k_wilson_eo_cl<PP, LL, SS>), dim3(nblk(g.V / 2 * (size_t)nrhs)), dim3(256), 0, s,
                                 (const S*)U, (const S*)in, (const S*)xin, (S*)out, g, p, nrhs, (R)alpha, (R)beta,
                                 live, (const S*)Cx, (const S*)Cout))
  return hipGetLastError();
}

hipError_t clover_site_mul(const lqcd_lattice* lat, const void* Cm, const void* in, void* out, int p, int nrhs,
                           double alpha, int layout, int prec, hipStream_t s) {
  const geo4 g = make_geo(lat);
  CL_DISPATCH(prec, layout, 0,
              (void)SS;
              hipLaunchKernelGGL((k_clover_site_mul<PP, LL>), dim3(nblk(g.V / 2 * (size_t)nrhs)), dim3(256), 0, s,
                                 (const S*)Cm, (const S*)in, (S*)out, g, p, nrhs, (R)alpha))
  return hipGetLastError();
}

hipError_t clover_invert(const lqcd_lattice* lat, const void* C, void* Cinv, double d, int prec, int* dflag,
                         hipStream_t s) {
  const size_t V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  switch (prec) {
    case LQCD_F64:
      hipLaunchKernelGGL(k_clover_invert<LQCD_F64>, dim3(nblk(2 * V)), dim3(256), 0, s,
                         (const prec_traits<LQCD_F64>::store*)C, (prec_traits<LQCD_F64>::store*)Cinv, V, d, dflag);
      break;
    case LQCD_F32:
      hipLaunchKernelGGL(k_clover_invert<LQCD_F32>, dim3(nblk(2 * V)), dim3(256), 0, s,
                         (const prec_traits<LQCD_F32>::store*)C, (prec_traits<LQCD_F32>::store*)Cinv, V, d, dflag);
      break;
    case LQCD_F16:
      hipLaunchKernelGGL(k_clover_invert<LQCD_F16>, dim3(nblk(2 * V)), dim3(256), 0, s,
                         (const prec_traits<LQCD_F16>::store*)C, (prec_traits<LQCD_F16>::store*)Cinv, V, d, dflag);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lq

using namespace lq;

extern "C" {

int dirac_apply_clover(const lqcd_lattice* lat, const void* U, const void* C, const void* psi, void* eta, int nrhs,
                       double m0, int layout, int prec, int flags, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, prec))) return rc;
  if (!U || !C || !psi || !eta) return fail(LQCD_ERR_ARG, "dirac_apply_clover: null array pointer");
  if (flags & ~LQCD_DAGGER) return fail(LQCD_ERR_ARG, "dirac_apply_clover: unknown flags 0x%x", flags);
  return hip_status(wilson_full_clover(lat, U, C, psi, eta, nrhs, 4.0 + m0, -0.5, layout, prec,
                                       (flags & LQCD_DAGGER) != 0, (hipStream_t)stream),
                    "dirac_apply_clover launch");
}

int clover_inverse(const lqcd_lattice* lat, const void* C, void* Cinv, double m0, int prec, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (prec != LQCD_F64 && prec != LQCD_F32 && prec != LQCD_F16) return fail(LQCD_ERR_PREC, "unknown precision %d", prec);
  if (!C || !Cinv) return fail(LQCD_ERR_ARG, "clover_inverse: null array pointer");
  hipStream_t s = (hipStream_t)stream;
  int* dflag = nullptr;
  hipError_t e = hipMallocAsync((void**)&dflag, sizeof(int), s);
  if (e != hipSuccess) return hip_status(e, "clover_inverse: flag allocation");
  e = hipMemsetAsync(dflag, 0, sizeof(int), s);
  if (e == hipSuccess) e = clover_invert(lat, C, Cinv, 4.0 + m0, prec, dflag, s);
  int flag = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipError_t e2 = hipFreeAsync(dflag, s);
  if (e != hipSuccess) return hip_status(e, "clover_inverse");
  if (e2 != hipSuccess) return hip_status(e2, "clover_inverse: free flag");
  if (flag) return fail(LQCD_ERR_SINGULAR, "clover_inverse: (4 + m0) - C(x) is singular on some site");
  return LQCD_OK;
}

int dirac_apply_eo_clover(const lqcd_lattice* lat, const void* U, const void* C, const void* Cinv, const void* psi_e,
                          void* eta_e, int nrhs, double m0, int layout, int prec, int flags, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, prec))) return rc;
  if (!U || !C || !Cinv || !psi_e || !eta_e) return fail(LQCD_ERR_ARG, "dirac_apply_eo_clover: null array pointer");
  if (flags & ~LQCD_DAGGER) return fail(LQCD_ERR_ARG, "dirac_apply_eo_clover: unknown flags 0x%x", flags);
  hipStream_t s = (hipStream_t)stream;
  const size_t V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  const size_t esz = prec == LQCD_F64 ? 16 : prec == LQCD_F32 ? 8 : 4;
  void* tmp = nullptr;
  hipError_t e = hipMallocAsync(&tmp, V / 2 * 12 * (size_t)nrhs * esz, s);
  if (e != hipSuccess) return hip_status(e, "dirac_apply_eo_clover: temporary odd block");
  const bool dag = (flags & LQCD_DAGGER) != 0;
  // S psi_e = ((4+m0) - C_e) psi_e - (1/4) H_eo D_oo^{-1} H_oe psi_e, D_oo^{-1} = Cinv on odd sites
  e = wilson_eo_clover(lat, U, psi_e, nullptr, tmp, 1, nrhs, 0.0, 1.0, layout, prec, dag, nullptr, nullptr, Cinv, s);
  if (e == hipSuccess)
    e = wilson_eo_clover(lat, U, tmp, psi_e, eta_e, 0, nrhs, 4.0 + m0, -0.25, layout, prec, dag, nullptr, C, nullptr,
                         s);
  hipError_t e2 = hipFreeAsync(tmp, s);
  if (e != hipSuccess) return hip_status(e, "dirac_apply_eo_clover launch");
  return hip_status(e2, "dirac_apply_eo_clover: free temporary");
}

}  // extern "C"
