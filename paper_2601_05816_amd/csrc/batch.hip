// Uneven batches: several independent lattices, each with its own gauge
// field, rhs count and mass, in ONE persistent launch.
//
// The work of every problem is cut into units of 256 (site, rhs) items; the
// units of all problems form one list (problem k owns units
// [unit0_k, unit0_k + units_k)).  A fixed grid of workgroups sized to the
// chip's residency walks the list with a stride of the grid size, so a batch
// of lattices from 8^3 x 16 to 24^3 x 48 with 1..32 rhs each keeps every CU
// busy without one launch per lattice.  The per-item arithmetic is the
// one-site body of dslash.hip (rhs-innermost layout).
#include "batch.h"
#include "wilson.h"

namespace lq {

int fail(int code, const char* fmt, ...);
int check_lattice(const lqcd_lattice* lat);
int hip_status(hipError_t e, const char* what);

template <int PREC, int SG>
__global__ __launch_bounds__(256) void k_wilson_batch(batch_desc d) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  for (unsigned long long u = blockIdx.x; u < d.total_units; u += gridDim.x) {
    int k = 0;
    while (k + 1 < d.n && u >= d.p[k + 1].unit0) ++k;
    const batch_prob& pb = d.p[k];
    const size_t nsite = pb.parity < 0 ? pb.g.V : pb.g.V / 2;
    const size_t t = (size_t)(u - pb.unit0) * 256u + threadIdx.x;
    if (t >= nsite * (size_t)pb.nrhs) continue;
    const size_t site = t / pb.nrhs;
    const int rhs = (int)(t % pb.nrhs);
    if (pb.live && !pb.live[rhs]) continue;
    if (pb.parity < 0)
      wilson_full_site<PREC, LQCD_LAYOUT2, SG>((const S*)pb.U, (const S*)pb.in, (S*)pb.out, pb.g, pb.nrhs,
                                               (R)pb.alpha, (R)pb.beta, site, rhs);
    else
      wilson_eo_site<PREC, LQCD_LAYOUT2, SG>((const S*)pb.U, (const S*)pb.in, (const S*)pb.xin, (S*)pb.out, pb.g,
                                             pb.parity, pb.nrhs, (R)pb.alpha, (R)pb.beta, site, rhs);
  }
}

static int g_batch_grid = 0;  // persistent grid size (0 = residency of the chip)

void set_batch_grid(int blocks) { g_batch_grid = blocks > 0 ? blocks : 0; }

unsigned batch_grid_default() {
  static unsigned cached = 0;
  if (!cached) {
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) ncu = 256;
    cached = (unsigned)ncu * 4u;  // four 256-thread workgroups per CU
  }
  return cached;
}

hipError_t wilson_batch(batch_desc& d, int prec, bool dagger, hipStream_t s) {
  unsigned long long units = 0;
  for (int k = 0; k < d.n; ++k) {
    const size_t nsite = d.p[k].parity < 0 ? d.p[k].g.V : d.p[k].g.V / 2;
    d.p[k].unit0 = units;
    units += (nsite * (size_t)d.p[k].nrhs + 255) / 256;
  }
  d.total_units = units;
  if (units == 0) return hipSuccess;
  unsigned grid = g_batch_grid ? (unsigned)g_batch_grid : batch_grid_default();
  if (grid > units) grid = (unsigned)units;
#define BL(P, SGN) hipLaunchKernelGGL((k_wilson_batch<P, SGN>), dim3(grid), dim3(256), 0, s, d)
  switch (prec * 2 + (dagger ? 1 : 0)) {
    case LQCD_F64 * 2: BL(LQCD_F64, 1); break;
    case LQCD_F64 * 2 + 1: BL(LQCD_F64, -1); break;
    case LQCD_F32 * 2: BL(LQCD_F32, 1); break;
    case LQCD_F32 * 2 + 1: BL(LQCD_F32, -1); break;
    case LQCD_F16 * 2: BL(LQCD_F16, 1); break;
    case LQCD_F16 * 2 + 1: BL(LQCD_F16, -1); break;
    default: return hipErrorInvalidValue;
  }
#undef BL
  return hipGetLastError();
}

geo4 make_geo4(const lqcd_lattice* lat) {
  geo4 g;
  for (int i = 0; i < 4; ++i) g.n[i] = lat->dims[i];
  g.V = (size_t)g.n[0] * g.n[1] * g.n[2] * g.n[3];
  return g;
}

}  // namespace lq

using namespace lq;

extern "C" {

int dirac_apply_batch(int nprob, const lqcd_problem* probs, int prec, int flags, void* stream) {
  if (nprob < 1 || nprob > LQCD_MAX_BATCH)
    return fail(LQCD_ERR_ARG, "dirac_apply_batch: %d problems, need 1..%d", nprob, LQCD_MAX_BATCH);
  if (!probs) return fail(LQCD_ERR_ARG, "dirac_apply_batch: probs is null");
  if (prec != LQCD_F64 && prec != LQCD_F32 && prec != LQCD_F16)
    return fail(LQCD_ERR_PREC, "unknown precision %d", prec);
  if (flags & ~LQCD_DAGGER) return fail(LQCD_ERR_ARG, "dirac_apply_batch: unknown flags 0x%x", flags);
  batch_desc d;
  d.n = nprob;
  for (int k = 0; k < nprob; ++k) {
    const lqcd_problem& q = probs[k];
    int rc = check_lattice(&q.lat);
    if (rc) return rc;
    if (q.nrhs < 1) return fail(LQCD_ERR_ARG, "dirac_apply_batch: problem %d has nrhs = %d", k, q.nrhs);
    if (!q.U || !q.psi || !q.eta) return fail(LQCD_ERR_ARG, "dirac_apply_batch: problem %d has a null pointer", k);
    batch_prob& b = d.p[k];
    b.g = make_geo4(&q.lat);
    b.U = q.U;
    b.in = q.psi;
    b.xin = nullptr;
    b.out = q.eta;
    b.live = nullptr;
    b.nrhs = q.nrhs;
    b.parity = -1;
    b.alpha = 4.0 + q.m0;
    b.beta = -0.5;
  }
  return hip_status(wilson_batch(d, prec, (flags & LQCD_DAGGER) != 0, (hipStream_t)stream),
                    "dirac_apply_batch launch");
}

int lqcd_set_batch_grid(int blocks) {
  if (blocks < 0) return fail(LQCD_ERR_ARG, "negative grid size");
  set_batch_grid(blocks);
  return LQCD_OK;
}

}  // extern "C"
