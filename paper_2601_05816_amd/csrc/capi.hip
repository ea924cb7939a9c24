// C-ABI entry points: argument validation, status codes, last-error message,
// and the host-side geometry tables.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "kernels.h"

namespace lq {

static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int check_lattice(const lqcd_lattice* lat) {
  if (!lat) return fail(LQCD_ERR_ARG, "lattice pointer is null");
  size_t v = 1;
  for (int i = 0; i < 4; ++i) {
    int n = lat->dims[i];
    if (n < 2 || (n & 1))
      return fail(LQCD_ERR_DIMS, "lattice extent dims[%d] = %d: every extent must be even and >= 2", i, n);
    v *= (size_t)n;
  }
  if (v > ((size_t)1 << 40)) return fail(LQCD_ERR_DIMS, "lattice volume %zu is too large", v);
  return LQCD_OK;
}

int check_block(int nrhs, int layout, int prec) {
  if (nrhs < 1) return fail(LQCD_ERR_ARG, "nrhs = %d: need at least one right-hand side", nrhs);
  if (layout != LQCD_RHS_OUTER && layout != LQCD_LAYOUT1 && layout != LQCD_LAYOUT2)
    return fail(LQCD_ERR_LAYOUT, "unknown layout %d", layout);
  if (prec != LQCD_F64 && prec != LQCD_F32 && prec != LQCD_F16)
    return fail(LQCD_ERR_PREC, "unknown precision %d", prec);
  return LQCD_OK;
}

int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return LQCD_OK;
  return fail(LQCD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace lq

using namespace lq;

extern "C" {

const char* lqcd_last_error(void) { return g_err; }

int lqcd_lattice_tables(const lqcd_lattice* lat, int32_t* nbr, int32_t* eo_site) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  const int n0 = lat->dims[0], n1 = lat->dims[1], n2 = lat->dims[2], n3 = lat->dims[3];
  const size_t V = (size_t)n0 * n1 * n2 * n3;
  if (V > (size_t)INT32_MAX) return fail(LQCD_ERR_DIMS, "volume does not fit int32 site numbers");
  const int n[4] = {n0, n1, n2, n3};
  size_t cnt[2] = {0, 0};
  for (int x0 = 0; x0 < n0; ++x0)
    for (int x1 = 0; x1 < n1; ++x1)
      for (int x2 = 0; x2 < n2; ++x2)
        for (int x3 = 0; x3 < n3; ++x3) {
          const int x[4] = {x0, x1, x2, x3};
          const int32_t site = ((x0 * n1 + x1) * n2 + x2) * n3 + x3;
          if (nbr) {
            for (int mu = 0; mu < 4; ++mu) {
              int y[4], z[4];
              for (int k = 0; k < 4; ++k) y[k] = z[k] = x[k];
              y[mu] = (x[mu] + 1) % n[mu];
              z[mu] = (x[mu] + n[mu] - 1) % n[mu];
              nbr[(size_t)site * 8 + mu] = ((y[0] * n1 + y[1]) * n2 + y[2]) * n3 + y[3];
              nbr[(size_t)site * 8 + 4 + mu] = ((z[0] * n1 + z[1]) * n2 + z[2]) * n3 + z[3];
            }
          }
          if (eo_site) {
            const int p = (x0 + x1 + x2 + x3) & 1;
            eo_site[(size_t)p * (V / 2) + cnt[p]] = site;
          }
          const int p = (x0 + x1 + x2 + x3) & 1;
          cnt[p]++;
        }
  return LQCD_OK;
}

int dirac_apply(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double m0,
                int layout, int prec, int flags, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, prec))) return rc;
  if (!U || !psi || !eta) return fail(LQCD_ERR_ARG, "dirac_apply: null array pointer");
  if (flags & ~LQCD_DAGGER) return fail(LQCD_ERR_ARG, "dirac_apply: unknown flags 0x%x", flags);
  hipError_t e = wilson_full(lat, U, psi, eta, nrhs, 4.0 + m0, -0.5, layout, prec, (flags & LQCD_DAGGER) != 0,
                             (hipStream_t)stream);
  return hip_status(e, "dirac_apply launch");
}

size_t dirac_apply_eo_workspace_bytes(const lqcd_lattice* lat, int nrhs, int prec) {
  if (check_lattice(lat) || nrhs < 1 || (prec != LQCD_F64 && prec != LQCD_F32 && prec != LQCD_F16)) return 0;
  const size_t V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  const size_t esz = prec == LQCD_F64 ? 16 : prec == LQCD_F32 ? 8 : 4;
  return V / 2 * 12 * (size_t)nrhs * esz;
}

int dirac_apply_eo_ws(const lqcd_lattice* lat, const void* U, const void* psi_e, void* eta_e, int nrhs, double m0,
                      int layout, int prec, int flags, void* work, size_t work_bytes, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, prec))) return rc;
  if (!U || !psi_e || !eta_e) return fail(LQCD_ERR_ARG, "dirac_apply_eo_ws: null array pointer");
  if (flags & ~LQCD_DAGGER) return fail(LQCD_ERR_ARG, "dirac_apply_eo_ws: unknown flags 0x%x", flags);
  const double d = 4.0 + m0;
  if (d == 0.0) return fail(LQCD_ERR_SINGULAR, "dirac_apply_eo_ws: 4 + m0 = 0, D_oo is not invertible");
  const size_t need = dirac_apply_eo_workspace_bytes(lat, nrhs, prec);
  if (!work || work_bytes < need)
    return fail(LQCD_ERR_WORKSPACE, "dirac_apply_eo_ws: workspace of %zu bytes given, %zu needed", work_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  const bool dag = (flags & LQCD_DAGGER) != 0;
  hipError_t e = schur_apply(lat, U, psi_e, eta_e, work, nrhs, d, layout, prec, dag, nullptr, s);
  return hip_status(e, "dirac_apply_eo_ws launch");
}

int dirac_apply_eo(const lqcd_lattice* lat, const void* U, const void* psi_e, void* eta_e, int nrhs, double m0,
                   int layout, int prec, int flags, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, prec))) return rc;
  if (!U || !psi_e || !eta_e) return fail(LQCD_ERR_ARG, "dirac_apply_eo: null array pointer");
  if (flags & ~LQCD_DAGGER) return fail(LQCD_ERR_ARG, "dirac_apply_eo: unknown flags 0x%x", flags);
  const double d = 4.0 + m0;
  if (d == 0.0) return fail(LQCD_ERR_SINGULAR, "dirac_apply_eo: 4 + m0 = 0, D_oo is not invertible");
  hipStream_t s = (hipStream_t)stream;
  const size_t V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  const size_t esz = prec == LQCD_F64 ? 16 : prec == LQCD_F32 ? 8 : 4;
  void* tmp = nullptr;
  hipError_t e = hipMallocAsync(&tmp, V / 2 * 12 * (size_t)nrhs * esz, s);
  if (e != hipSuccess) return hip_status(e, "dirac_apply_eo: temporary odd block");
  const bool dag = (flags & LQCD_DAGGER) != 0;
  // S psi_e = (4+m0) psi_e - (1/4) H_eo H_oe psi_e / (4+m0), with D_eo = -H_eo / 2
  e = schur_apply(lat, U, psi_e, eta_e, tmp, nrhs, d, layout, prec, dag, nullptr, s);
  hipError_t e2 = hipFreeAsync(tmp, s);
  if (e != hipSuccess) return hip_status(e, "dirac_apply_eo launch");
  return hip_status(e2, "dirac_apply_eo: free temporary");
}

}  // extern "C"
