// Batched restarted GMRES (Algorithm 2) on the device, with optional
// odd-even preconditioning and FP64 iterative refinement around an FP32 or
// FP16-storage inner solver.
//
// Every rhs runs its own GMRES(m) in lock-step with the others (batched, not
// block Krylov).  One Arnoldi step for all rhs (Algorithm 2, lines 4-5):
//   w = A v_j                      Wilson kernels on the whole block
//   h_kj = <v_k, w>, k <= j        classical Gram-Schmidt: all dots of the step
//                                  in passes of DOT_KB vectors over w
//   w -= sum_k h_kj v_k, |w|^2     one fused pass
//   Givens / gamma / relnorm       one thread per rhs, FP64
//   v_{j+1} = w / |w|
// A rhs whose relnorm falls below tol (or whose Krylov space closes) stops
// taking steps (its lanes are masked) while the others continue; the cycle
// ends when none is left ("max over rhs" exit, line 6).  At the end of a cycle
// each rhs solves its small triangular system and updates x (line 9).  The
// next cycle starts from the true residual b - A x.
#include <math.h>
#include <string.h>

#include <vector>

#include "blas.h"
#include "common.h"
#include "kernels.h"

namespace lq {

int fail(int code, const char* fmt, ...);
int check_lattice(const lqcd_lattice* lat);
int check_block(int nrhs, int layout, int prec);
int hip_status(hipError_t e, const char* what);

typedef cx<double> zd;

// ------------------------------------------------------------ small kernels
// Start of a cycle: beta = |r|, relative residual against bref, activity,
// Givens state reset, scale factor 1/beta for v_0.
__global__ void k_cycle_start(int nrhs, int m, const zd* __restrict__ nrm, const double* __restrict__ bref,
                              double tol, int fixed, int* __restrict__ live, int* __restrict__ steps,
                              zd* __restrict__ g, double* __restrict__ scl, double* __restrict__ beta,
                              int* __restrict__ flags /*[0] active count, [1] nonfinite*/) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double b = sqrt(nrm[r].re);
  beta[r] = b;
  steps[r] = 0;
  const bool finite = isfinite(b);
  if (!finite) atomicAdd(&flags[1], 1);
  const bool act = finite && bref[r] > 0.0 && b > 0.0 && (fixed || b > tol * bref[r]);
  live[r] = act ? 1 : 0;
  scl[r] = act ? 1.0 / b : 0.0;
  for (int k = 0; k <= m; ++k) g[(size_t)r * (m + 1) + k] = {0.0, 0.0};
  g[(size_t)r * (m + 1)] = {b, 0.0};
  if (act) atomicAdd(&flags[0], 1);
}

// Column j of the Hessenberg matrix for every live rhs: apply the previous
// rotations, build the rotation that zeroes h_{j+1,j}, rotate gamma.
__global__ void k_arnoldi_col(int j, int m, int nrhs, const zd* __restrict__ hcol, const zd* __restrict__ nrm,
                              zd* __restrict__ H, double* __restrict__ cs, zd* __restrict__ sn, zd* __restrict__ g,
                              const double* __restrict__ bref, double tol, int fixed, int* __restrict__ live,
                              int* __restrict__ steps, double* __restrict__ est, double* __restrict__ scl) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs || !live[r]) return;
  zd* Hr = H + (size_t)r * (m + 1) * m;  // H[i][j] at Hr[i*m + j]
  double* c = cs + (size_t)r * m;
  zd* s = sn + (size_t)r * m;
  zd* gr = g + (size_t)r * (m + 1);
  for (int k = 0; k <= j; ++k) Hr[(size_t)k * m + j] = hcol[(size_t)k * nrhs + r];
  const double hn = sqrt(nrm[r].re);
  for (int i = 0; i < j; ++i) {
    const zd a = Hr[(size_t)i * m + j], b = Hr[(size_t)(i + 1) * m + j];
    const zd t1 = {c[i] * a.re + (s[i].re * b.re - s[i].im * b.im), c[i] * a.im + (s[i].re * b.im + s[i].im * b.re)};
    // -conj(s) a + c b
    const zd t2 = {-(s[i].re * a.re + s[i].im * a.im) + c[i] * b.re, -(s[i].re * a.im - s[i].im * a.re) + c[i] * b.im};
    Hr[(size_t)i * m + j] = t1;
    Hr[(size_t)(i + 1) * m + j] = t2;
  }
  const zd a = Hr[(size_t)j * m + j];
  const double aa = hypot(a.re, a.im);
  double cj;
  zd sj;
  if (aa == 0.0) {
    cj = 0.0;
    sj = {1.0, 0.0};
  } else {
    const double rr = hypot(aa, hn);
    cj = aa / rr;
    sj = {a.re / aa * hn / rr, a.im / aa * hn / rr};  // (a/|a|) conj(hn) / r, hn real
  }
  c[j] = cj;
  s[j] = sj;
  Hr[(size_t)j * m + j] = {cj * a.re + sj.re * hn, cj * a.im + sj.im * hn};
  Hr[(size_t)(j + 1) * m + j] = {0.0, 0.0};
  const zd gj = gr[j];
  gr[j + 1] = {-(sj.re * gj.re + sj.im * gj.im), -(sj.re * gj.im - sj.im * gj.re)};  // -conj(s) g_j
  gr[j] = {cj * gj.re, cj * gj.im};
  steps[r] = j + 1;
  const double rel = hypot(gr[j + 1].re, gr[j + 1].im) / bref[r];
  est[r] = rel;
  scl[r] = hn > 0.0 ? 1.0 / hn : 0.0;
  if ((!fixed && rel < tol) || hn == 0.0 || !isfinite(rel)) live[r] = 0;
}

__global__ void k_count_live(int nrhs, const int* __restrict__ live, int* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int n = 0;
    for (int r = 0; r < nrhs; ++r) n += live[r];
    *out = n;
  }
}

// Back substitution R y = gamma on the rotated triangle, y[k][rhs].
__global__ void k_lsq(int m, int nrhs, const zd* __restrict__ H, const zd* __restrict__ g,
                      const int* __restrict__ steps, zd* __restrict__ y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const int n = steps[r];
  const zd* Hr = H + (size_t)r * (m + 1) * m;
  const zd* gr = g + (size_t)r * (m + 1);
  for (int i = n - 1; i >= 0; --i) {
    zd acc = gr[i];
    for (int k = i + 1; k < n; ++k) {
      const zd h = Hr[(size_t)i * m + k], yk = y[(size_t)k * nrhs + r];
      acc.re -= h.re * yk.re - h.im * yk.im;
      acc.im -= h.re * yk.im + h.im * yk.re;
    }
    const zd d = Hr[(size_t)i * m + i];
    const double den = d.re * d.re + d.im * d.im;
    y[(size_t)i * nrhs + r] = {(acc.re * d.re + acc.im * d.im) / den, (acc.im * d.re - acc.re * d.im) / den};
  }
}

// out[r] = a * sqrt(nrm[r].re) (+ flag handling): used for |b| and scale factors
__global__ void k_sqrt_scale(int nrhs, const zd* __restrict__ nrm, double a, double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) out[r] = a * sqrt(nrm[r].re);
}

// Per-rhs factors for a refinement step from the outer residual norms:
// fin = c / |r| (into the inner rhs), fout = |r| / c (back into x), 0 for
// rhs that are converged (|r| <= tol |b|) or have a zero source.
__global__ void k_ir_factors(int nrhs, const zd* __restrict__ nrm, const double* __restrict__ bref, double tol,
                             double c, double* __restrict__ fin, double* __restrict__ fout,
                             double* __restrict__ ibref, double* __restrict__ rel, int* __restrict__ flags) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double b = sqrt(nrm[r].re);
  rel[r] = bref[r] > 0.0 ? b / bref[r] : 0.0;
  if (!isfinite(b)) atomicAdd(&flags[1], 1);
  const bool act = isfinite(b) && bref[r] > 0.0 && b > tol * bref[r];
  fin[r] = act ? c / b : 0.0;
  fout[r] = act ? b / c : 0.0;
  ibref[r] = act ? 1.0 : 0.0;
  if (act) atomicAdd(&flags[0], 1);
}

// zero-source rhs: factor 0 (their solution is x = 0), else 1
__global__ void k_zero_mask(int nrhs, const double* __restrict__ bref, double* __restrict__ f) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) f[r] = bref[r] > 0.0 ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- workspace
struct Arena {
  char* base;
  size_t off, cap;
  void* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    void* p = base ? base + off : nullptr;
    off += n;
    return p;
  }
};

static size_t esize(int prec) { return prec == LQCD_F64 ? 16 : prec == LQCD_F32 ? 8 : 4; }

struct Solver {
  lqcd_lattice lat;
  size_t V, nsite, nelem;
  int nrhs, m, eo, mode, plo;
  bool dag;  // solve with D^dagger
  double m0, d;
  hipStream_t s;
  unsigned nblk;
  // device buffers
  const void* U64;
  void* Ulo;
  void *xe, *xo, *be, *bo, *bp;   // FP64 internal vectors (xo, bo only with eo)
  void* r64;                      // FP64 residual (refinement modes)
  void* tmp64;                    // FP64 odd temporary (eo)
  void* basis;                    // m+1 Krylov vectors in the working precision
  void* tmplo;                    // odd temporary in the working precision (eo)
  void* rlo;                      // inner rhs (refinement modes)
  void* dlo;                      // inner solution (refinement modes)
  zd *part, *hcol, *nrm, *H, *sn, *g, *y;
  double *cs, *bref, *ibref, *beta, *scl, *est, *fin, *fout, *rel;
  int *live, *steps, *flags, *nlive;
  hipEvent_t ev[2];

  void layout(Arena& a) {
    const size_t v64 = nelem * 16;
    const int pw = mode == 0 ? LQCD_F64 : plo;
    xe = a.take(v64);
    be = a.take(v64);
    bp = eo ? a.take(v64) : be;
    xo = eo ? a.take(v64) : nullptr;
    bo = eo ? a.take(v64) : nullptr;
    tmp64 = eo ? a.take(v64) : nullptr;
    r64 = mode ? a.take(v64) : nullptr;
    basis = a.take((size_t)(m + 1) * nelem * esize(pw));
    tmplo = (eo && mode) ? a.take(nelem * esize(pw)) : nullptr;
    rlo = mode ? a.take(nelem * esize(pw)) : nullptr;
    dlo = mode ? a.take(nelem * esize(pw)) : nullptr;
    Ulo = mode ? a.take(4 * V * 9 * esize(pw)) : nullptr;
    part = (zd*)a.take((size_t)nblk * DOT_KB * nrhs * sizeof(zd));
    hcol = (zd*)a.take((size_t)(m + 1) * nrhs * sizeof(zd));
    nrm = (zd*)a.take((size_t)nrhs * sizeof(zd));
    H = (zd*)a.take((size_t)nrhs * (m + 1) * m * sizeof(zd));
    sn = (zd*)a.take((size_t)nrhs * m * sizeof(zd));
    g = (zd*)a.take((size_t)nrhs * (m + 1) * sizeof(zd));
    y = (zd*)a.take((size_t)m * nrhs * sizeof(zd));
    cs = (double*)a.take((size_t)nrhs * m * sizeof(double));
    bref = (double*)a.take(nrhs * sizeof(double));
    ibref = (double*)a.take(nrhs * sizeof(double));
    beta = (double*)a.take(nrhs * sizeof(double));
    scl = (double*)a.take(nrhs * sizeof(double));
    est = (double*)a.take(nrhs * sizeof(double));
    fin = (double*)a.take(nrhs * sizeof(double));
    fout = (double*)a.take(nrhs * sizeof(double));
    rel = (double*)a.take(nrhs * sizeof(double));
    live = (int*)a.take(nrhs * sizeof(int));
    steps = (int*)a.take(nrhs * sizeof(int));
    flags = (int*)a.take(2 * sizeof(int));
    nlive = (int*)a.take(2 * sizeof(int));
  }

  void* Vk(int prec, int k) const { return (char*)basis + (size_t)k * nelem * esize(prec); }
  unsigned small_grid() const { return (unsigned)((nrhs + 63) / 64); }

  // out = A in, in the working precision `prec` (A = S with eo, else D)
  hipError_t apply(int prec, const void* in, void* out, const int* lv) {
    const void* U = prec == LQCD_F64 ? U64 : Ulo;
    if (eo) {
      void* t = prec == LQCD_F64 ? tmp64 : tmplo;
      hipError_t e = wilson_eo(&lat, U, in, nullptr, t, 1, nrhs, 0.0, 1.0, LQCD_LAYOUT2, prec, dag, lv, s);
      if (e != hipSuccess) return e;
      return wilson_eo(&lat, U, t, in, out, 0, nrhs, d, -0.25 / d, LQCD_LAYOUT2, prec, dag, lv, s);
    }
    return wilson_full(&lat, U, in, out, nrhs, d, -0.5, LQCD_LAYOUT2, prec, dag, s);
  }

  // |x|^2 per rhs into nrm (scaled by sc)
  hipError_t norms(int prec, const void* x, double sc, const int* lv) {
    hipError_t e = norm_parts(prec, x, nelem, nrhs, lv, part, nblk, s);
    if (e != hipSuccess) return e;
    return reduce_parts(part, nblk, 1, nrhs, sc, nrm, s);
  }
};

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return hip_status(e_, #x); \
  } while (0)

struct HostState {
  std::vector<int> iters, restarts, outer;
  std::vector<double> est;
};

// One batched GMRES(m) solve of A x = b in precision `prec`, vectors scaled by
// `c` (stored value = c x true value).  x holds the initial guess.  Relative
// residuals are measured against bref (device, per rhs).  Runs at most
// max_cycles cycles; returns LQCD_OK or an error code.  Adds the Arnoldi steps
// and cycles of every rhs to hs.
static int run_gmres(Solver& S, int prec, void* x, const void* b, const double* bref_dev, double tol, int max_cycles,
                     int fixed, bool x_zero, double c, HostState& hs, int* host_pinned) {
  const size_t nel = S.nelem;
  const int nrhs = S.nrhs, m = S.m;
  const double sc = 1.0 / (c * c);
  hipStream_t s = S.s;
  std::vector<int> steps_h(nrhs);
  std::vector<double> est_h(nrhs);
  hipEvent_t* ev = S.ev;
  int rc = LQCD_OK;
  for (int cycle = 0; cycle < max_cycles; ++cycle) {
    void* V0 = S.Vk(prec, 0);
    hipError_t e;
    if (cycle == 0 && x_zero) {
      e = convert(prec, b, prec, V0, nel, nrhs, nullptr, s);
      if (e == hipSuccess) e = S.norms(prec, V0, sc, nullptr);
    } else {
      e = S.apply(prec, x, V0, nullptr);
      if (e == hipSuccess) e = b_minus_y(prec, b, V0, nel, nrhs, nullptr, S.part, S.nblk, s);
      if (e == hipSuccess) e = reduce_parts(S.part, S.nblk, 1, nrhs, sc, S.nrm, s);
    }
    if (e != hipSuccess) { rc = hip_status(e, "gmres residual"); break; }
    HIPCHK(hipMemsetAsync(S.flags, 0, 2 * sizeof(int), s));
    hipLaunchKernelGGL(k_cycle_start, dim3(S.small_grid()), dim3(64), 0, s, nrhs, m, S.nrm, bref_dev, tol, fixed,
                       S.live, S.steps, S.g, S.scl, S.beta, S.flags);
    int fl[2];
    HIPCHK(hipMemcpyAsync(fl, S.flags, sizeof fl, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (fl[1]) { rc = fail(LQCD_ERR_NONFINITE, "gmres: non-finite residual norm"); break; }
    if (fl[0] == 0) break;
    {
      std::vector<int> lv(nrhs);
      HIPCHK(hipMemcpy(lv.data(), S.live, nrhs * sizeof(int), hipMemcpyDeviceToHost));
      for (int r = 0; r < nrhs; ++r) hs.restarts[r] += lv[r];
    }
    HIPCHK(scale_rhs(prec, V0, nel, nrhs, S.scl, S.live, s));
    for (int j = 0; j < m; ++j) {
      void* w = S.Vk(prec, j + 1);
      HIPCHK(S.apply(prec, S.Vk(prec, j), w, S.live));
      for (int k0 = 0; k0 <= j; k0 += DOT_KB) {
        const int K = (j + 1 - k0) < DOT_KB ? (j + 1 - k0) : DOT_KB;
        HIPCHK(dot_parts(prec, S.basis, nel, k0, K, w, nel, nrhs, S.live, S.part, S.nblk, s));
        HIPCHK(reduce_parts(S.part, S.nblk, K, nrhs, sc, S.hcol + (size_t)k0 * nrhs, s));
      }
      HIPCHK(cgs_update(prec, S.basis, nel, j + 1, S.hcol, w, nel, nrhs, S.live, S.part, S.nblk, s));
      HIPCHK(reduce_parts(S.part, S.nblk, 1, nrhs, sc, S.nrm, s));
      hipLaunchKernelGGL(k_arnoldi_col, dim3(S.small_grid()), dim3(64), 0, s, j, m, nrhs, S.hcol, S.nrm, S.H, S.cs,
                         S.sn, S.g, bref_dev, tol, fixed, S.live, S.steps, S.est, S.scl);
      HIPCHK(scale_rhs(prec, w, nel, nrhs, S.scl, S.live, s));
      // pipelined exit test: read the live count of the previous step while
      // this one runs
      hipLaunchKernelGGL(k_count_live, dim3(1), dim3(1), 0, s, nrhs, S.live, S.nlive + (j & 1));
      HIPCHK(hipMemcpyAsync(host_pinned + (j & 1), S.nlive + (j & 1), sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipEventRecord(ev[j & 1], s));
      if (j >= 1) {
        HIPCHK(hipEventSynchronize(ev[(j - 1) & 1]));
        if (host_pinned[(j - 1) & 1] == 0) break;
      }
    }
    hipLaunchKernelGGL(k_lsq, dim3(S.small_grid()), dim3(64), 0, s, m, nrhs, S.H, S.g, S.steps, S.y);
    HIPCHK(lincomb(prec, S.basis, nel, m, S.y, S.steps, prec, x, nel, nrhs, 1.0, s));
    HIPCHK(hipMemcpyAsync(steps_h.data(), S.steps, nrhs * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(est_h.data(), S.est, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r) {
      hs.iters[r] += steps_h[r];
      if (steps_h[r]) hs.est[r] = est_h[r];
    }
    x_zero = false;
  }
  return rc;
}

static void defaults(lqcd_solver_params* p) {
  memset(p, 0, sizeof *p);
  p->restart = 30;
  p->max_restarts = 200;
  p->eo = 1;
  p->mode = 0;
  p->tol = 1e-10;
  p->inner_tol = 0.0;
  p->max_outer = 50;
}

static int check_params(const lqcd_solver_params* p) {
  if (!p) return fail(LQCD_ERR_ARG, "gmres: params is null");
  if (p->restart < 1 || p->restart > 64) return fail(LQCD_ERR_ARG, "gmres: restart = %d not in 1..64", p->restart);
  if (p->max_restarts < 1) return fail(LQCD_ERR_ARG, "gmres: max_restarts must be >= 1");
  if (p->mode < 0 || p->mode > 2) return fail(LQCD_ERR_ARG, "gmres: unknown mode %d", p->mode);
  if (!(p->tol >= 0.0)) return fail(LQCD_ERR_ARG, "gmres: tol must be >= 0");
  if (p->mode && p->max_outer < 1) return fail(LQCD_ERR_ARG, "gmres: max_outer must be >= 1");
  return LQCD_OK;
}

static void setup(Solver& S, const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p) {
  S.lat = *lat;
  S.V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  S.eo = p->eo ? 1 : 0;
  S.nsite = S.eo ? S.V / 2 : S.V;
  S.nelem = S.nsite * 12 * (size_t)nrhs;
  S.nrhs = nrhs;
  S.m = p->restart;
  S.mode = p->mode;
  S.plo = p->mode == 1 ? LQCD_F32 : LQCD_F16;
  S.dag = p->dagger != 0;
  S.nblk = reduce_grid(S.nelem);
}

}  // namespace lq

using namespace lq;

extern "C" {

void lqcd_solver_defaults(lqcd_solver_params* p) {
  if (p) defaults(p);
}

size_t gmres_workspace_bytes(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p) {
  if (check_lattice(lat) || nrhs < 1 || check_params(p)) return 0;
  Solver S;
  setup(S, lat, nrhs, p);
  Arena a{nullptr, 0, 0};
  S.layout(a);
  return a.off + 256;
}

int gmres_solve(const lqcd_lattice* lat, const void* U, const void* b, void* x, int nrhs, double m0, int layout,
                const lqcd_solver_params* params, void* work, size_t work_bytes, lqcd_rhs_stats* stats,
                void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, LQCD_F64))) return rc;
  if ((rc = check_params(params))) return rc;
  if (!U || !b || !x) return fail(LQCD_ERR_ARG, "gmres_solve: null array pointer");
  const size_t need = gmres_workspace_bytes(lat, nrhs, params);
  if (!work || work_bytes < need)
    return fail(LQCD_ERR_WORKSPACE, "gmres_solve: workspace of %zu bytes given, %zu needed", work_bytes, need);
  const double d = 4.0 + m0;
  if (d == 0.0 && params->eo) return fail(LQCD_ERR_SINGULAR, "gmres_solve: 4 + m0 = 0, D_oo is not invertible");

  Solver S;
  setup(S, lat, nrhs, params);
  S.m0 = m0;
  S.d = d;
  S.s = (hipStream_t)stream;
  S.U64 = U;
  Arena a{(char*)work, 0, work_bytes};
  a.off = (256 - ((uintptr_t)work & 255)) & 255;
  S.layout(a);
  hipStream_t s = S.s;
  const size_t nel = S.nelem;
  const double tol = params->tol;
  const int fixed = params->fixed_iters ? 1 : 0;
  const int dims[4] = {lat->dims[0], lat->dims[1], lat->dims[2], lat->dims[3]};
  HostState hs;
  hs.iters.assign(nrhs, 0);
  hs.restarts.assign(nrhs, 0);
  hs.outer.assign(nrhs, 0);
  hs.est.assign(nrhs, 0.0);
  int* pinned = nullptr;
  HIPCHK(hipHostMalloc((void**)&pinned, 4 * sizeof(int), hipHostMallocDefault));
  if (hipEventCreateWithFlags(&S.ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&S.ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipHostFree(pinned);
    return fail(LQCD_ERR_HIP, "gmres_solve: event creation failed");
  }

  auto body = [&]() -> int {
    // ingest: ABI layout -> internal vectors; |b| of the full system per rhs
    HIPCHK(pack(layout, true, (void*)b, S.be, S.bo, dims, nrhs, S.eo, s));
    if (S.eo) {
      HIPCHK(norm_parts(LQCD_F64, S.be, nel, nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(reduce_parts(S.part, S.nblk, 1, nrhs, 1.0, S.hcol, s));
      HIPCHK(norm_parts(LQCD_F64, S.bo, nel, nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(reduce_parts(S.part, S.nblk, 1, nrhs, 1.0, S.nrm, s));
      // nrm += hcol (|b_e|^2 + |b_o|^2) via a 2-row reduction of the stored values
      HIPCHK(hipMemcpyAsync(S.part, S.hcol, nrhs * sizeof(zd), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(S.part + nrhs, S.nrm, nrhs * sizeof(zd), hipMemcpyDeviceToDevice, s));
      HIPCHK(reduce_parts(S.part, 2, 1, nrhs, 1.0, S.nrm, s));
    } else {
      HIPCHK(S.norms(LQCD_F64, S.be, 1.0, nullptr));
    }
    hipLaunchKernelGGL(k_sqrt_scale, dim3(S.small_grid()), dim3(64), 0, s, nrhs, S.nrm, 1.0, S.bref);
    bool x_zero = !params->x_is_guess;
    if (params->x_is_guess) {
      HIPCHK(pack(layout, true, x, S.xe, S.xo, dims, nrhs, S.eo, s));
      hipLaunchKernelGGL(k_zero_mask, dim3(S.small_grid()), dim3(64), 0, s, nrhs, S.bref, S.fin);
      HIPCHK(scale_rhs(LQCD_F64, S.xe, nel, nrhs, S.fin, nullptr, s));
    } else {
      HIPCHK(hipMemsetAsync(S.xe, 0, nel * 16, s));
    }
    if (S.eo) {
      // b'_e = b_e - D_eo D_oo^{-1} b_o = b_e + (1/2) H_eo b_o / (4+m0)
      HIPCHK(wilson_eo(&S.lat, U, S.bo, S.be, S.bp, 0, nrhs, 1.0, 0.5 / d, LQCD_LAYOUT2, LQCD_F64, S.dag, nullptr, s));
    }
    if (S.mode == 0) {
      rc = run_gmres(S, LQCD_F64, S.xe, S.bp, S.bref, tol, params->max_restarts, fixed, x_zero, 1.0, hs, pinned);
      if (rc) return rc;
    } else {
      // iterative refinement: FP64 residual and update, inner GMRES in plo
      const int plo = S.plo;
      const double c = plo == LQCD_F16 ? sqrt((double)S.nsite * 12.0) : 1.0;
      const double itol = params->inner_tol > 0 ? params->inner_tol : (plo == LQCD_F32 ? 1e-4 : 1e-2);
      HIPCHK(convert_links(U, plo, S.Ulo, 4 * S.V * 9, s));
      for (int outer = 0; outer < params->max_outer; ++outer) {
        if (outer == 0 && x_zero) {
          HIPCHK(convert(LQCD_F64, S.bp, LQCD_F64, S.r64, nel, nrhs, nullptr, s));
          HIPCHK(S.norms(LQCD_F64, S.r64, 1.0, nullptr));
        } else {
          HIPCHK(S.apply(LQCD_F64, S.xe, S.r64, nullptr));
          HIPCHK(b_minus_y(LQCD_F64, S.bp, S.r64, nel, nrhs, nullptr, S.part, S.nblk, s));
          HIPCHK(reduce_parts(S.part, S.nblk, 1, nrhs, 1.0, S.nrm, s));
        }
        HIPCHK(hipMemsetAsync(S.flags, 0, 2 * sizeof(int), s));
        hipLaunchKernelGGL(k_ir_factors, dim3(S.small_grid()), dim3(64), 0, s, nrhs, S.nrm, S.bref, tol, c, S.fin,
                           S.fout, S.ibref, S.rel, S.flags);
        int fl[2];
        HIPCHK(hipMemcpyAsync(fl, S.flags, sizeof fl, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (fl[1]) return fail(LQCD_ERR_NONFINITE, "gmres: non-finite residual norm in refinement");
        if (fl[0] == 0) break;
        {
          std::vector<double> fo(nrhs);
          HIPCHK(hipMemcpy(fo.data(), S.fout, nrhs * sizeof(double), hipMemcpyDeviceToHost));
          for (int r = 0; r < nrhs; ++r) hs.outer[r] += fo[r] != 0.0;
        }
        HIPCHK(convert(LQCD_F64, S.r64, plo, S.rlo, nel, nrhs, S.fin, s));
        HIPCHK(hipMemsetAsync(S.dlo, 0, nel * esize(plo), s));
        rc = run_gmres(S, plo, S.dlo, S.rlo, S.ibref, itol, 1, 0, true, c, hs, pinned);
        if (rc) return rc;
        HIPCHK(add_scaled(plo, S.dlo, S.xe, nel, nrhs, S.fout, s));
      }
    }
    // reconstruct the odd sites, full-system true residual, write x back
    void* t1 = S.mode ? S.r64 : S.Vk(LQCD_F64, 0);
    double nr_e_scale = 1.0;
    if (S.eo) {
      // x_o = (b_o + (1/2) H_oe x_e) / (4+m0)
      HIPCHK(wilson_eo(&S.lat, U, S.xe, S.bo, S.xo, 1, nrhs, 1.0 / d, 0.5 / d, LQCD_LAYOUT2, LQCD_F64, S.dag, nullptr,
                       s));
      // r_e = b_e - [(4+m0) x_e - (1/2) H_eo x_o]
      HIPCHK(wilson_eo(&S.lat, U, S.xo, S.xe, t1, 0, nrhs, d, -0.5, LQCD_LAYOUT2, LQCD_F64, S.dag, nullptr, s));
      HIPCHK(b_minus_y(LQCD_F64, S.be, t1, nel, nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(reduce_parts(S.part, S.nblk, 1, nrhs, nr_e_scale, S.hcol, s));
      HIPCHK(wilson_eo(&S.lat, U, S.xe, S.xo, S.tmp64, 1, nrhs, d, -0.5, LQCD_LAYOUT2, LQCD_F64, S.dag, nullptr, s));
      HIPCHK(b_minus_y(LQCD_F64, S.bo, S.tmp64, nel, nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(reduce_parts(S.part, S.nblk, 1, nrhs, 1.0, S.nrm, s));
      HIPCHK(hipMemcpyAsync(S.part, S.hcol, nrhs * sizeof(zd), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(S.part + nrhs, S.nrm, nrhs * sizeof(zd), hipMemcpyDeviceToDevice, s));
      HIPCHK(reduce_parts(S.part, 2, 1, nrhs, 1.0, S.nrm, s));
    } else {
      HIPCHK(wilson_full(&S.lat, U, S.xe, t1, nrhs, d, -0.5, LQCD_LAYOUT2, LQCD_F64, S.dag, s));
      HIPCHK(b_minus_y(LQCD_F64, S.be, t1, nel, nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(reduce_parts(S.part, S.nblk, 1, nrhs, 1.0, S.nrm, s));
    }
    HIPCHK(pack(layout, false, x, S.xe, S.xo, dims, nrhs, S.eo, s));
    std::vector<zd> rn(nrhs);
    std::vector<double> bn(nrhs);
    HIPCHK(hipMemcpyAsync(rn.data(), S.nrm, nrhs * sizeof(zd), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(bn.data(), S.bref, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int all = 1;
    for (int r = 0; r < nrhs; ++r) {
      const double tr = bn[r] > 0 ? sqrt(rn[r].re) / bn[r] : 0.0;
      const int conv = (bn[r] == 0.0) || (tr <= tol);
      if (!(tr == tr)) return fail(LQCD_ERR_NONFINITE, "gmres: non-finite true residual for rhs %d", r);
      all &= conv;
      if (stats) {
        stats[r].iters = hs.iters[r];
        stats[r].restarts = hs.restarts[r];
        stats[r].outer_iters = hs.outer[r];
        stats[r].converged = conv;
        stats[r].true_relres = tr;
        stats[r].est_relres = hs.est[r];
      }
    }
    return (all || fixed) ? LQCD_OK : LQCD_NOT_CONVERGED;
  };
  rc = body();
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(S.ev[0]);
  (void)hipEventDestroy(S.ev[1]);
  (void)hipHostFree(pinned);
  return rc;
}

}  // extern "C"
