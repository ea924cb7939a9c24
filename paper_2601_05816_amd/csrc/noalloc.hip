// dirac_apply_eo without device allocation: the odd half-lattice temporary of
// the Schur apply lives in a fixed array of this library instead of a
// hipMallocAsync block.  The array is a device global, so every GPU the
// library runs on holds its own copy (at its own address) until the process
// ends.  Host code never passes the array's name to a kernel: the address of
// this device's copy is resolved once per device with hipGetSymbolAddress and
// kept; the kernels receive that pointer exactly as they receive the
// temporary in dirac_apply_eo.
#include <mutex>

#include "kernels.h"

namespace lq {
int fail(int code, const char* fmt, ...);
int check_lattice(const lqcd_lattice* lat);
int check_block(int nrhs, int layout, int prec);
int hip_status(hipError_t e, const char* what);
}  // namespace lq

using namespace lq;

static __device__ __align__(256) unsigned char scratch[LQCD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Address of this device's copy of `scratch` (resolved on the first call per
// device, with that device current).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "dirac_apply_eo_noalloc: current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(LQCD_ERR_ARG, "dirac_apply_eo_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e, "dirac_apply_eo_noalloc: scratch address");
    if (!p) return fail(LQCD_ERR_HIP, "dirac_apply_eo_noalloc: scratch address is null");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return LQCD_OK;
}

}  // namespace

extern "C" {

int dirac_apply_eo_noalloc(const lqcd_lattice* lat, const void* U, const void* psi_e, void* eta_e, int nrhs,
                           double m0, int layout, int prec, int flags, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, prec))) return rc;
  if (!U || !psi_e || !eta_e) return fail(LQCD_ERR_ARG, "dirac_apply_eo_noalloc: null array pointer");
  if (flags & ~LQCD_DAGGER) return fail(LQCD_ERR_ARG, "dirac_apply_eo_noalloc: unknown flags 0x%x", flags);
  const double d = 4.0 + m0;
  if (d == 0.0) return fail(LQCD_ERR_SINGULAR, "dirac_apply_eo_noalloc: 4 + m0 = 0, D_oo is not invertible");
  const size_t V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  const size_t esz = prec == LQCD_F64 ? 16 : prec == LQCD_F32 ? 8 : 4;
  const size_t need = V / 2 * 12 * (size_t)nrhs * esz;
  if (need > (size_t)LQCD_NOALLOC_SCRATCH_BYTES)
    return fail(LQCD_ERR_WORKSPACE, "dirac_apply_eo_noalloc: the odd block needs %zu bytes, the fixed scratch holds %zu",
                need, (size_t)LQCD_NOALLOC_SCRATCH_BYTES);
  void* tmp = nullptr;
  if ((rc = scratch_address(&tmp))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const bool dag = (flags & LQCD_DAGGER) != 0;
  // the same apply as dirac_apply_eo; with two hop passes the first writes
  // every entry of the odd block before the second reads it, so nothing is
  // cleared (the fused kernel does not use the array)
  hipError_t e = schur_apply(lat, U, psi_e, eta_e, tmp, nrhs, d, layout, prec, dag, nullptr, s);
  return hip_status(e, "dirac_apply_eo_noalloc launch");
}

}  // extern "C"
