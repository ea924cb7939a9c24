// Uneven batches: several independent lattices, each with its own gauge
// field, rhs count and mass, in ONE persistent launch.
//
// The work of every problem is cut into units of 256 work items; the units
// of all problems form one list (problem k owns units [unit0_k, unit0_k +
// units_k)).  A fixed grid of workgroups sized to the chip's residency walks
// the list with a stride of the grid size, so a batch of lattices from
// 8^3 x 16 to 24^3 x 48 with 1..32 rhs each keeps every CU busy without one
// launch per lattice.  Two kernels: a unit is either 256 (site, rhs) items
// with the one-site body of dslash.hip, or one workgroup of the problem's
// time-streaming pencil grid (pencil_kernels.h) with the tile, segment
// count and store kind the autotuner recorded for that lattice, two rhs per
// work item for FP32 / FP16 blocks with an even rhs count, or (FP32 / FP16,
// 8 or more rhs) with the links of each step staged in LDS where the
// autotuner chose that kernel (variant 2).  Pencil units
// differ in length between lattices, so by default the pencil launch has one
// workgroup per unit (the dispatcher balances them) with the longest units
// first; a set grid size makes it persistent.  Pencil units of a problem
// start at a multiple of 8 and a persistent grid is a multiple of 8, so a
// unit keeps the XCD its pencil grid position assumes.
#include <algorithm>

#include "batch.h"
#include "pencil_kernels.h"
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

// LDS slices of the links-through-LDS body: NCW 5 (16 or more rhs) and 9
// (8 to 15 rhs); fewer rhs (NCW 17) would need 4 x 2 x 17 x 63 elements,
// more than a pencil launch should reserve for every unit.
constexpr int kBatchNcw[2] = {5, 9};

template <int PREC>
constexpr size_t batch_pl_bytes(int ncw) {
  return (size_t)4 * 2 * ncw * 63 * sizeof(typename prec_traits<PREC>::store);
}

template <int PREC, int SG>
__global__ __launch_bounds__(256) void k_wilson_batch_p(batch_desc d) {
  typedef typename prec_traits<PREC>::store S;
  typedef typename prec_traits<PREC>::real R;
  // dynamic LDS: the link slices of the largest links-through-LDS unit (the
  // launch requests them when a problem uses that body)
  extern __shared__ __align__(16) unsigned char batch_lds[];
  for (unsigned long long u = blockIdx.x; u < d.total_units; u += gridDim.x) {
    // the wavefronts of a workgroup leave a unit at different times, and the
    // two links-through-LDS bodies place their per-wavefront slices at
    // different offsets: no wavefront starts a unit before all have left the
    // previous one
    if (d.pl) __syncthreads();
    int k = 0;
    while (k + 1 < d.n && u >= d.p[k + 1].unit0) ++k;
    const batch_prob& pb = d.p[k];
    const unsigned b = (unsigned)(u - pb.unit0);
    const S* U = (const S*)pb.U;
    const S* in = (const S*)pb.in;
    S* out = (S*)pb.out;
    if (pb.parity < 0) {
      if constexpr (PREC != LQCD_F64) {  // (FP64: registers of the other bodies would grow)
        if (pb.ncw == kBatchNcw[0]) {
          wilson_full_pl_body<PREC, LQCD_LAYOUT2, SG, kBatchNcw[0]>(
              U, in, out, pb.pg, pb.nrhs, (R)pb.alpha, (R)pb.beta, b,
              *reinterpret_cast<S(*)[4][2][kBatchNcw[0] * 63]>(batch_lds));
          continue;
        }
        if (pb.ncw == kBatchNcw[1]) {
          wilson_full_pl_body<PREC, LQCD_LAYOUT2, SG, kBatchNcw[1]>(
              U, in, out, pb.pg, pb.nrhs, (R)pb.alpha, (R)pb.beta, b,
              *reinterpret_cast<S(*)[4][2][kBatchNcw[1] * 63]>(batch_lds));
          continue;
        }
      }
      if (PREC != LQCD_F64 && pb.nr == 2)
        wilson_full_pn_body<PREC, SG, (PREC == LQCD_F64 ? 1 : 2)>(U, in, out, pb.pg, pb.nrhs, (R)pb.alpha,
                                                                   (R)pb.beta, b);
      else
        wilson_full_p_body<PREC, LQCD_LAYOUT2, SG>(U, in, out, pb.pg, pb.nrhs, (R)pb.alpha, (R)pb.beta, b);
    } else {
      if (PREC != LQCD_F64 && pb.nr == 2)
        wilson_eo_pn_body<PREC, SG, (PREC == LQCD_F64 ? 1 : 2)>(U, in, (const S*)pb.xin, out, pb.pg, pb.parity,
                                                                 pb.nrhs, (R)pb.alpha, (R)pb.beta, pb.live, b);
      else
        wilson_eo_p_body<PREC, LQCD_LAYOUT2, SG>(U, in, (const S*)pb.xin, out, pb.pg, pb.parity, pb.nrhs,
                                                 (R)pb.alpha, (R)pb.beta, pb.live, b);
    }
  }
}

static int g_batch_grid = 0;  // persistent grid size (0 = residency of the chip)
static int g_batch_kind = 0;
static int g_batch_occ = 0;   // pencil launch: at most this many workgroups per CU (0 = no cap)

void set_batch_grid(int blocks) { g_batch_grid = blocks > 0 ? blocks : 0; }
void set_batch_occupancy(int occ) { g_batch_occ = occ > 0 ? occ : 0; }
void set_batch_kernel(int kind) { g_batch_kind = kind; }
int batch_kernel() { return g_batch_kind; }

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

hipError_t wilson_batch(batch_desc& din, int prec, bool dagger, hipStream_t s) {
  // automatic choice (measured on MI355X with the eight-lattice batch): the
  // pencil kernel for full-lattice applies, the one-site kernel for the
  // odd-even passes of the lock-step solver
  const bool pencil = g_batch_kind == 2 || (g_batch_kind == 0 && din.n > 0 && din.p[0].parity < 0);
  batch_desc d = din;  // the launch's copy: problems may be reordered below
  unsigned long long units = 0;
  size_t pl_bytes = 0;  // LDS of the links-through-LDS units
  if (pencil) {
    const size_t pl_max = 40 * 1024;
    for (int k = 0; k < d.n; ++k) {
      batch_prob& pb = d.p[k];
      lqcd_lattice lat;
      for (int i = 0; i < 4; ++i) lat.dims[i] = pb.g.n[i];
      // kernel, tile, segments and store kind of the autotuner's entry for this lattice
      const bool eo = pb.parity >= 0;
      const kcfg c = choose_cfg(eo ? KIND_EO : KIND_FULL, &lat, pb.nrhs, prec, LQCD_LAYOUT2);
      pb.ncw = 0;
      if (!eo && prec != LQCD_F64 && c.variant == 2 && pb.nrhs >= 8) {
        const int ncw = pb.nrhs >= 16 ? kBatchNcw[0] : kBatchNcw[1];
        const size_t need = prec == LQCD_F32 ? batch_pl_bytes<LQCD_F32>(ncw) : batch_pl_bytes<LQCD_F16>(ncw);
        if (need <= pl_max) {
          pb.ncw = ncw;
          pl_bytes = std::max(pl_bytes, need);
        }
      }
      pb.nr = (!pb.ncw && prec != LQCD_F64 && pb.nrhs % 2 == 0) ? 2 : 1;
      pb.pg = make_pencil(&lat, pb.nrhs / pb.nr, eo, c);
    }
    // longest units (most time steps per workgroup) first, so that the
    // dispatcher does not end the launch on a few long workgroups
    std::stable_sort(d.p, d.p + d.n, [](const batch_prob& a, const batch_prob& b) { return a.pg.Lt > b.pg.Lt; });
  }
  for (int k = 0; k < d.n; ++k) {
    batch_prob& pb = d.p[k];
    pb.unit0 = units;
    if (pencil) {
      units += pencil_blocks(pb.pg);  // a multiple of 8
    } else {
      const size_t nsite = pb.parity >= 0 ? pb.g.V / 2 : pb.g.V;
      units += (nsite * (size_t)pb.nrhs + 255) / 256;
    }
  }
  d.total_units = units;
  d.pl = pl_bytes > 0 ? 1 : 0;
  if (units == 0) return hipSuccess;
  // pencils: one workgroup per unit unless a persistent grid is set (a
  // multiple of 8, so that every unit keeps the XCD its position assumes);
  // one (site, rhs) per item: persistent, four workgroups per CU by default
  unsigned grid;
  if (pencil) grid = g_batch_grid ? (g_batch_grid < 8 ? 8u : (unsigned)g_batch_grid & ~7u) : (unsigned)units;
  else grid = g_batch_grid ? (unsigned)g_batch_grid : batch_grid_default();
  if (grid > units) grid = (unsigned)units;
  size_t dyn = 0;  // residency cap of the pencil launch through its LDS request
  if (pencil && !occupancy_lds(g_batch_occ, 0, &dyn)) dyn = 0;
  if (dyn < pl_bytes) dyn = pl_bytes;
#define BL(K, P, SGN) hipLaunchKernelGGL((K<P, SGN>), dim3(grid), dim3(256), pencil ? dyn : 0, s, d)
#define BL_ALL(K)                                         \
  switch (prec * 2 + (dagger ? 1 : 0)) {                  \
    case LQCD_F64 * 2: BL(K, LQCD_F64, 1); break;         \
    case LQCD_F64 * 2 + 1: BL(K, LQCD_F64, -1); break;    \
    case LQCD_F32 * 2: BL(K, LQCD_F32, 1); break;         \
    case LQCD_F32 * 2 + 1: BL(K, LQCD_F32, -1); break;    \
    case LQCD_F16 * 2: BL(K, LQCD_F16, 1); break;         \
    case LQCD_F16 * 2 + 1: BL(K, LQCD_F16, -1); break;    \
    default: return hipErrorInvalidValue;                 \
  }
  if (pencil) {
    BL_ALL(k_wilson_batch_p)
  } else {
    BL_ALL(k_wilson_batch)
  }
#undef BL_ALL
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

int lqcd_set_batch_kernel(int kind) {
  if (kind < 0 || kind > 2) return fail(LQCD_ERR_ARG, "unknown batch kernel %d", kind);
  set_batch_kernel(kind);
  return LQCD_OK;
}

}  // extern "C"
