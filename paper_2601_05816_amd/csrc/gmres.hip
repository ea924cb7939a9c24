// Batched restarted GMRES (Algorithm 2) on the device, with optional
// odd-even preconditioning and FP64 iterative refinement around an FP32 or
// FP16-storage inner solver.
//
// Every rhs runs its own GMRES(m) in lock-step with the others (batched, not
// block Krylov).  One Arnoldi step for all rhs (Algorithm 2):
//   w = A v_j                      Wilson kernels on the whole block
//   h_kj = <v_k, w>, k <= j        classical Gram-Schmidt: all dots of the step
//                                  in passes of DOT_KB vectors over w
//   w -= sum_k h_kj v_k, |w|^2     one fused pass
//   Givens / gamma / relnorm       one thread per rhs, FP64
//   v_{j+1} = w / |w|              FP64 bases: not a pass of its own; the basis
//                                  is kept unnormalised, v_k = s_k u_k with a
//                                  scale s_k per rhs and vector, and the
//                                  scales enter the coefficients of the next
//                                  step.  FP32 / FP16 bases are scaled in a
//                                  pass (unnormalised vectors could leave
//                                  their range over a cycle).
// A rhs whose relnorm falls below tol (or whose Krylov space closes) stops
// taking steps (its lanes are masked) while the others continue; the cycle
// ends when none is left (the "max over rhs" exit of Algorithm 2).  At the end of a cycle
// each rhs solves its small triangular system and updates x.  The
// next cycle starts from the true residual b - A x.
#include <math.h>
#include <string.h>

#include <map>
#include <tuple>
#include <vector>

#include "blas.h"
#include "common.h"
#include "batch.h"
#include "kernels.h"

namespace lq {

int fail(int code, const char* fmt, ...);
int check_lattice(const lqcd_lattice* lat);
int check_block(int nrhs, int layout, int prec);
int hip_status(hipError_t e, const char* what);

typedef cx<double> zd;

// ------------------------------------------------------------ small kernels
// Start of a cycle: beta = |r|, relative residual against bref, activity,
// Givens state reset.  lazy: v_0 = sk[0] r with sk[0] = 1/beta (r stays as
// stored); else scl = 1/beta for an explicit scaling pass and sk[0] = 1.
__global__ void k_cycle_start(int nrhs, int m, const zd* __restrict__ nrm, const double* __restrict__ bref,
                              double tol, int fixed, int lazy, int* __restrict__ live, int* __restrict__ steps,
                              zd* __restrict__ g, double* __restrict__ sk, double* __restrict__ scl,
                              double* __restrict__ beta, int* __restrict__ flags /*[0] active, [1] nonfinite*/) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double b = sqrt(nrm[r].re);
  beta[r] = b;
  steps[r] = 0;
  const bool finite = isfinite(b);
  if (!finite) atomicAdd(&flags[1], 1);
  const bool act = finite && bref[r] > 0.0 && b > 0.0 && (fixed || b > tol * bref[r]);
  live[r] = act ? 1 : 0;
  sk[r] = lazy ? (act ? 1.0 / b : 0.0) : 1.0;
  scl[r] = act ? 1.0 / b : 0.0;
  for (int k = 0; k <= m; ++k) g[(size_t)r * (m + 1) + k] = {0.0, 0.0};
  g[(size_t)r * (m + 1)] = {b, 0.0};
  if (act) atomicAdd(&flags[0], 1);
}

// Column j of the Hessenberg matrix for every live rhs: apply the previous
// rotations, build the rotation that zeroes h_{j+1,j}, rotate gamma.
//
// The basis may be stored unnormalised: v_k = sk[k] u_k.  hcol holds the raw
// dots d_k = <u_k, w> with w = A u_j, nrm holds |u_{j+1}|^2 of the updated
// vector u_{j+1} = w - sum_k sk[k]^2 d_k u_k; the true entries are
// h_kj = sk[k] sk[j] d_k and h_{j+1,j} = sk[j] |u_{j+1}|, and
// sk[j+1] = 1 / |u_{j+1}|.
__global__ void k_arnoldi_col(int j, int m, int nrhs, const zd* __restrict__ hcol, const zd* __restrict__ nrm,
                              zd* __restrict__ H, double* __restrict__ cs, zd* __restrict__ sn, zd* __restrict__ g,
                              const double* __restrict__ bref, double tol, int fixed, int lazy,
                              int* __restrict__ live, int* __restrict__ steps, double* __restrict__ est,
                              double* __restrict__ sk, double* __restrict__ scl) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs || !live[r]) return;
  zd* Hr = H + (size_t)r * (m + 1) * m;  // H[i][j] at Hr[i*m + j]
  double* c = cs + (size_t)r * m;
  zd* s = sn + (size_t)r * m;
  zd* gr = g + (size_t)r * (m + 1);
  const double scj = sk[(size_t)j * nrhs + r];
  for (int k = 0; k <= j; ++k) {
    const double f = sk[(size_t)k * nrhs + r] * scj;
    const zd d = hcol[(size_t)k * nrhs + r];
    Hr[(size_t)k * m + j] = {f * d.re, f * d.im};
  }
  const double un = sqrt(nrm[r].re);
  const double hn = scj * un;
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
  // lazy: v_{j+1} = sk[j+1] u_{j+1}; else the caller scales u_{j+1} by scl
  sk[(size_t)(j + 1) * nrhs + r] = lazy ? (un > 0.0 ? 1.0 / un : 0.0) : 1.0;
  scl[r] = un > 0.0 ? 1.0 / un : 0.0;
  if ((!fixed && rel < tol) || hn == 0.0 || !isfinite(rel)) live[r] = 0;
}

// Coefficients of the fused update u_{j+1} = w - sum_k coef_k u_k for the
// unnormalised basis: coef_k = sk[k]^2 d_k.
__global__ void k_cgs_coef(int K, int nrhs, const zd* __restrict__ d, const double* __restrict__ sk,
                           zd* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * nrhs) return;
  const double f = sk[i] * sk[i];
  coef[i] = {f * d[i].re, f * d[i].im};
}

__global__ void k_count_live(int nrhs, const int* __restrict__ live, int* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int n = 0;
    for (int r = 0; r < nrhs; ++r) n += live[r];
    *out = n;
  }
}

// acc[i] += add[i] (the second CGS pass's dots into the first's)
__global__ void k_add_zd(int n, const zd* __restrict__ add, zd* __restrict__ acc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    acc[i].re += add[i].re;
    acc[i].im += add[i].im;
  }
}

// Back substitution R y = gamma on the rotated triangle, y[k][rhs].
__global__ void k_lsq(int m, int nrhs, const zd* __restrict__ H, const zd* __restrict__ g,
                      const int* __restrict__ steps, const double* __restrict__ sk, zd* __restrict__ y) {
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
  // coefficients of the stored (unnormalised) basis vectors: v_i = sk[i] u_i
  for (int i = 0; i < n; ++i) {
    const double f = sk[(size_t)i * nrhs + r];
    zd& yi = y[(size_t)i * nrhs + r];
    yi = {f * yi.re, f * yi.im};
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


// ------------------------------------------------------------ block GMRES
// All rhs of one lattice expand one block Krylov space K_k(A, R0) (Sec. II);
// a block of b <= 16 rhs is an nrows x b matrix (the rhs-innermost layout).
// Columns that have converged at the start of a cycle are zeroed and carried
// as identity pivots, which decouples them exactly (their least-squares
// coefficients are zero), so the block shrinks without repacking.

// Cycle start: active columns (|r_q| > tol |b_q|; with a fixed iteration
// count every nonzero source) and factors 1 / 0 that zero the others.
__global__ void k_bstart(int b, const zd* __restrict__ nrm, const double* __restrict__ bref, double tol, int fixed,
                         int* __restrict__ act, double* __restrict__ f, int* __restrict__ flags) {
  if (threadIdx.x || blockIdx.x) return;
  int n = 0, bad = 0;
  for (int q = 0; q < b; ++q) {
    const double r = sqrt(nrm[q].re);
    if (!isfinite(r)) bad = 1;
    const bool a = isfinite(r) && bref[q] > 0.0 && r > 0.0 && (fixed || r > tol * bref[q]);
    act[q] = a ? 1 : 0;
    f[q] = a ? 1.0 : 0.0;
    n += a;
  }
  flags[0] = n;
  flags[1] = bad;
}

constexpr int BMX = LQCD_BLOCK_MAX_RHS;  // widest block of the block solver

// G = R^H R for the Gram block G of the active columns (R upper triangular,
// unit rows and columns for the inactive ones) and Rinv = R^-1.  A pivot at
// or below 1e-12 of the largest diagonal entry of G (a diagonal entry of R
// at or below 1e-6 of the largest column norm; the pivots carry rounding
// errors of the order of 1e-16 of G's diagonal, so a smaller threshold would
// not see an exactly dependent column) marks the block numerically rank
// deficient: *bad = 1, that pivot's row is left zero and Rinv unset.
// With deflate (the residual block at a restart) the first such column is
// instead taken out of the cycle (act = 0, f = 0) and *bad = 2: the caller
// zeroes it and factorises again.
__global__ __launch_bounds__(64) void k_bchol(int b, int* __restrict__ act, const zd* __restrict__ G,
                                              zd* __restrict__ R, zd* __restrict__ Rinv, int* __restrict__ bad,
                                              int deflate, double* __restrict__ f) {
  // G and R in LDS; the entries of a row of R right of its pivot are
  // computed in parallel (thread c: column c), columns of R^-1 likewise.
  // Every thread reads the same pivots, so the branches are uniform.
  __shared__ zd g[BMX * BMX], r[BMX * BMX];
  __shared__ int ac[BMX];
  const int tid = threadIdx.x;
  for (int i = tid; i < b * b; i += blockDim.x) {
    g[i] = G[i];
    r[i] = {0.0, 0.0};
  }
  if (tid < b) ac[tid] = act[tid];
  __syncthreads();
  double gmax = 0.0;
  for (int q = 0; q < b; ++q)
    if (ac[q] && g[q * b + q].re > gmax) gmax = g[q * b + q].re;
  int deficient = 0;
  for (int q = 0; q < b; ++q) {
    if (!ac[q]) {  // row q of R stays a unit row
      if (tid == 0) r[q * b + q] = {1.0, 0.0};
      continue;
    }
    double d = g[q * b + q].re;
    for (int p = 0; p < q; ++p) d -= r[p * b + q].re * r[p * b + q].re + r[p * b + q].im * r[p * b + q].im;
    if (!(d > 1e-12 * gmax)) {
      if (deflate) {
        if (tid == 0) {
          act[q] = 0;
          f[q] = 0.0;
          *bad = 2;
        }
        return;
      }
      deficient = 1;
      if (tid == 0) r[q * b + q] = {d > 0.0 ? sqrt(d) : 0.0, 0.0};
      continue;
    }
    const double rq = sqrt(d);
    if (tid == 0) r[q * b + q] = {rq, 0.0};
    const int c = tid;
    if (c > q && c < b && ac[c]) {
      zd z = g[q * b + c];
      for (int p = 0; p < q; ++p) {  // z -= conj(R[p][q]) R[p][c]
        const zd u = r[p * b + q], v = r[p * b + c];
        z.re -= u.re * v.re + u.im * v.im;
        z.im -= u.re * v.im - u.im * v.re;
      }
      r[q * b + c] = {z.re / rq, z.im / rq};
    }
    __syncthreads();
  }
  __syncthreads();
  for (int i = tid; i < b * b; i += blockDim.x) R[i] = r[i];
  if (tid == 0) *bad = deficient;
  if (deficient) return;
  if (tid < b) {  // column c of R^-1 by back substitution, into g
    const int c = tid;
    for (int i = 0; i < b; ++i) g[i * b + c] = {0.0, 0.0};
    g[c * b + c] = {1.0 / r[c * b + c].re, 0.0};
    for (int i = c - 1; i >= 0; --i) {
      zd z = {0.0, 0.0};
      for (int k = i + 1; k <= c; ++k) {
        const zd u = r[i * b + k], v = g[k * b + c];
        z.re += u.re * v.re - u.im * v.im;
        z.im += u.re * v.im + u.im * v.re;
      }
      const double di = r[i * b + i].re;
      g[i * b + c] = {-z.re / di, -z.im / di};
    }
  }
  __syncthreads();
  for (int i = tid; i < b * b; i += blockDim.x) Rinv[i] = g[i];
}

// rotated right-hand side of the cycle's least-squares problem: [S; 0]
__global__ void k_binit(int m, int b, const zd* __restrict__ S, zd* __restrict__ G) {
  const int n = (m + 1) * b * b;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    G[i] = i < b * b ? S[i] : zd{0.0, 0.0};
}

// [x; y] <- [c x + s y; -conj(s) x + c y]
__device__ __forceinline__ void brot(zd& x, zd& y, double c, zd s) {
  const zd nx = {c * x.re + (s.re * y.re - s.im * y.im), c * x.im + (s.re * y.im + s.im * y.re)};
  const zd ny = {-(s.re * x.re + s.im * x.im) + c * y.re, -(s.re * x.im - s.im * x.re) + c * y.im};
  x = nx;
  y = ny;
}

constexpr int BH_CH = 32;  // earlier rotation steps staged in LDS per chunk

// n earlier rotation steps applied to one column of the incoming block:
// x = row cp, w[t] = row cp + 1 + t (t < B) in registers; row cp is final
// after step cp and goes to hcol, row cp + 1 + B enters from lr.  B is a
// template argument so that every index into w is a constant.
template <int B>
__device__ __forceinline__ void bhess_rows(zd& x, zd (&w)[BMX], const double* lc, const zd* ls, const zd* lr, int n,
                                           zd* hcol, size_t mb, int q) {
  for (int i = 0; i < n; ++i) {
#pragma unroll
    for (int t = 0; t < B; ++t) brot(x, w[t], lc[i * B + t], ls[i * B + t]);
    hcol[(size_t)i * mb] = x;
    x = w[0];
#pragma unroll
    for (int t = 0; t < B - 1; ++t) w[t] = w[t + 1];
    w[B - 1] = lr[i * B + q];
  }
}

// Step j of the block Arnoldi process on the small matrices: enter column
// block j of the block Hessenberg matrix (the Gram blocks H_ij, i <= j, and
// the triangular factor R of the new block below them), apply the earlier
// rotations, zero its b subdiagonals with b rotations per column, rotate the
// right-hand side and read the per-rhs residual estimates off the last b
// rows.  flags[0] counts the active columns that are still above tolerance.
//
// Layout of the work: lane q of the first wavefront owns column c0 + q and
// carries the b + 1 rows an earlier rotation step cp touches (rows cp ..
// cp + b) in registers, so the cp-loop is a register chain; the other
// wavefronts stage the rotations and the incoming rows of the next
// BH_CH steps in LDS meanwhile.  The new rotations of the 2b x b diagonal
// block are formed in parallel: the rotation that zeroes subdiagonal entry t
// of a column leaves the pivot with the norm r_t of the pivot and entries
// 0..t, so cosine r_{t-1} / r_t and sine u conj(y_t) / r_t (u the pivot's
// phase) follow from running sums of |y|^2.
__global__ __launch_bounds__(256) void k_bhess(int j, int m, int b, const zd* __restrict__ Hc,
                                               const zd* __restrict__ R, zd* __restrict__ H, double* __restrict__ cs,
                                               zd* __restrict__ sn, zd* __restrict__ G, const int* __restrict__ act,
                                               const double* __restrict__ bref, double tol, int fixed,
                                               double* __restrict__ est, int* __restrict__ flags) {
  __shared__ double lcs[2][BH_CH * BMX];
  __shared__ zd lsn[2][BH_CH * BMX], lrow[2][BH_CH * BMX];
  __shared__ zd hb[2 * BMX * BMX], gb[2 * BMX * BMX];
  __shared__ double rcs[BMX], ry2[BMX];
  __shared__ zd rsn[BMX];
  const int tid = threadIdx.x;
  const size_t mb = (size_t)m * b;
  const int c0 = j * b, nr = (j + 1) * b;
  // row `row` of the incoming column block, column q: a Gram block above
  // row nr, the factor R below
  auto src = [&](int row, int q) -> zd {
    return row < nr ? Hc[(size_t)(row / b) * b * b + (size_t)(row % b) * b + q] : R[(size_t)(row - nr) * b + q];
  };
  // rotations of steps k*BH_CH .. and the rows entering after them
  auto stage = [&](int k, int buf) {
    const int k0 = k * BH_CH, n = min(BH_CH, c0 - k0) * b;
    for (int i = tid - 64; i < n; i += blockDim.x - 64) {
      lcs[buf][i] = cs[(size_t)k0 * b + i];
      lsn[buf][i] = sn[(size_t)k0 * b + i];
      lrow[buf][i] = src(k0 + i / b + 1 + b, i % b);
    }
  };
  zd x = {0.0, 0.0}, w[BMX];
  if (tid < b) {
    x = src(0, tid);
#pragma unroll
    for (int t = 0; t < BMX; ++t) w[t] = t < b ? src(1 + t, tid) : zd{0.0, 0.0};
  }
  const int nch = (c0 + BH_CH - 1) / BH_CH;
  if (tid >= 64 && nch > 0) stage(0, 0);
  for (int i = tid; i < 2 * b * b; i += blockDim.x) gb[i] = G[(size_t)c0 * b + i];
  __syncthreads();
  for (int k = 0; k < nch; ++k) {
    if (tid >= 64 && k + 1 < nch) stage(k + 1, (k + 1) & 1);
    if (tid < b) {
      const int buf = k & 1, k0 = k * BH_CH, n = min(BH_CH, c0 - k0);
      zd* hcol = H + (size_t)k0 * mb + c0 + tid;
      switch (b) {
#define BH_CASE(B)                                                                               \
  case B:                                                                                        \
    bhess_rows<B>(x, w, lcs[buf], lsn[buf], lrow[buf], n, hcol, mb, tid);                        \
    break;
        BH_CASE(1) BH_CASE(2) BH_CASE(3) BH_CASE(4) BH_CASE(5) BH_CASE(6) BH_CASE(7) BH_CASE(8)
        BH_CASE(9) BH_CASE(10) BH_CASE(11) BH_CASE(12) BH_CASE(13) BH_CASE(14) BH_CASE(15) BH_CASE(16)
#undef BH_CASE
      }
    }
    __syncthreads();
  }
  // the 2b x b diagonal block: rows c0 .. c0 + 2b - 1
  if (tid < b) {
    hb[tid] = x;
#pragma unroll
    for (int t = 0; t < BMX; ++t)
      if (t < b) hb[(1 + t) * b + tid] = w[t];
    for (int r = b + 1; r < 2 * b; ++r) hb[r * b + tid] = src(c0 + r, tid);
  }
  __syncthreads();
  for (int q = 0; q < b; ++q) {
    const zd a = hb[q * b + q];
    const double aa2 = a.re * a.re + a.im * a.im;
    zd y = {0.0, 0.0};
    if (tid < b) {
      y = hb[(q + 1 + tid) * b + q];
      ry2[tid] = y.re * y.re + y.im * y.im;
    }
    __syncthreads();
    if (tid < b) {
      double p0 = aa2;  // |pivot|^2 + sum_{s < t} |y_s|^2, the same sums in every lane
      for (int s2 = 0; s2 < tid; ++s2) p0 += ry2[s2];
      const double p1 = p0 + ry2[tid];
      const double r0 = sqrt(p0), r1 = sqrt(p1), aa = sqrt(aa2);
      const zd u = aa > 0.0 ? zd{a.re / aa, a.im / aa} : zd{1.0, 0.0};
      double cc = 1.0;  // nothing to eliminate (also a decoupled inactive column)
      zd ss = {0.0, 0.0};
      if (r1 > 0.0) {
        cc = r0 / r1;
        ss = {(u.re * y.re + u.im * y.im) / r1, (u.im * y.re - u.re * y.im) / r1};
      }
      rcs[tid] = cc;
      rsn[tid] = ss;
      cs[(size_t)(c0 + q) * b + tid] = cc;
      sn[(size_t)(c0 + q) * b + tid] = ss;
      hb[(q + 1 + tid) * b + q] = {0.0, 0.0};
      if (tid == b - 1) hb[q * b + q] = {u.re * r1, u.im * r1};
    }
    __syncthreads();
    if (tid < b && tid > q) {  // later columns of the block
      zd xx = hb[q * b + tid];
#pragma unroll
      for (int t = 0; t < BMX; ++t)
        if (t < b) {
          zd yv = hb[(q + 1 + t) * b + tid];
          brot(xx, yv, rcs[t], rsn[t]);
          hb[(q + 1 + t) * b + tid] = yv;
        }
      hb[q * b + tid] = xx;
    } else if (tid >= 64 && tid < 64 + b) {  // right-hand side
      const int qq = tid - 64;
      zd xx = gb[q * b + qq];
#pragma unroll
      for (int t = 0; t < BMX; ++t)
        if (t < b) {
          zd yv = gb[(q + 1 + t) * b + qq];
          brot(xx, yv, rcs[t], rsn[t]);
          gb[(q + 1 + t) * b + qq] = yv;
        }
      gb[q * b + qq] = xx;
    }
    __syncthreads();
  }
  for (int i = tid; i < 2 * b * b; i += blockDim.x) {
    H[(size_t)(c0 + i / b) * mb + c0 + i % b] = hb[i];
    G[(size_t)c0 * b + i] = gb[i];
  }
  if (tid == 0) flags[0] = 0;
  __syncthreads();
  if (tid < b) {
    double e2 = 0.0;
    for (int r = b; r < 2 * b; ++r) {
      const zd g = gb[r * b + tid];
      e2 += g.re * g.re + g.im * g.im;
    }
    const double e = sqrt(e2);
    if (act[tid]) {
      est[tid] = bref[tid] > 0.0 ? e / bref[tid] : 0.0;
      if (fixed || !(e <= tol * bref[tid])) atomicAdd(&flags[0], 1);
    }
  }
}

// Y = T^-1 G on the rotated upper triangle T of the first n column blocks;
// Y row-major [n b][b].  Column-oriented back substitution: thread k holds
// row k of the right-hand side (all b columns) in registers; once row i is
// solved (by thread i, into LDS) every thread k < i subtracts T[k][i] Y[i].
// Each thread streams its own row of T, BS_PF entries ahead.
constexpr int BS_PF = 4;

__global__ __launch_bounds__(1024) void k_bsolve(int n, int m, int b, const zd* __restrict__ H,
                                                 const zd* __restrict__ G, zd* __restrict__ Y) {
  __shared__ zd ys[2][BMX];
  const int k = threadIdx.x;
  const size_t mb = (size_t)m * b;
  const int nb = n * b;
  zd a[BMX];
  double rden = 0.0;
  zd d = {0.0, 0.0};
  if (k < nb) {
#pragma unroll
    for (int q = 0; q < BMX; ++q) a[q] = q < b ? G[(size_t)k * b + q] : zd{0.0, 0.0};
    d = H[(size_t)k * mb + k];
    const double den = d.re * d.re + d.im * d.im;
    rden = den > 0.0 ? 1.0 / den : 0.0;
  }
  auto fetch = [&](int g0, zd* dst) {  // T[k][g0 .. g0 + BS_PF - 1]
#pragma unroll
    for (int p = 0; p < BS_PF; ++p) {
      const int i = g0 + p;
      dst[p] = (k < i && i < nb) ? H[(size_t)k * mb + i] : zd{0.0, 0.0};
    }
  };
  const int top = (nb + BS_PF - 1) / BS_PF * BS_PF;
  zd hc[BS_PF], hn[BS_PF] = {};
  fetch(top - BS_PF, hc);
  for (int g0 = top - BS_PF; g0 >= 0; g0 -= BS_PF) {
    if (g0 >= BS_PF) fetch(g0 - BS_PF, hn);
#pragma unroll
    for (int p = BS_PF - 1; p >= 0; --p) {
      const int i = g0 + p;
      if (i >= nb) continue;
      const int buf = i & 1;
      if (k == i) {
#pragma unroll
        for (int q = 0; q < BMX; ++q)
          if (q < b) {  // a / d
            const zd y = {(a[q].re * d.re + a[q].im * d.im) * rden, (a[q].im * d.re - a[q].re * d.im) * rden};
            ys[buf][q] = y;
            Y[(size_t)i * b + q] = y;
          }
      }
      __syncthreads();
      if (k < i) {
        const zd h = hc[p];
#pragma unroll
        for (int q = 0; q < BMX; ++q)
          if (q < b) {
            const zd y = ys[buf][q];
            a[q].re -= h.re * y.re - h.im * y.im;
            a[q].im -= h.re * y.im + h.im * y.re;
          }
      }
    }
#pragma unroll
    for (int p = 0; p < BS_PF; ++p) hc[p] = hn[p];
  }
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
  int gs;    // 0 CGS, 1 CGS2, 2 MGS
  bool dag;  // solve with D^dagger
  double m0, d;
  hipStream_t s;
  unsigned nblk;
  // device buffers
  const void* U64;
  void* Ulo;
  // clover term (D = D_W - C): caller's FP64 field, the site-local inverse
  // of D_oo (eo) and working-precision copies (refinement modes)
  bool clov = false;
  const void* C64 = nullptr;
  void *Ci64 = nullptr, *Clo = nullptr, *Cilo = nullptr;
  void *xe, *xo, *be, *bo, *bp;   // FP64 internal vectors (xo, bo only with eo)
  void* r64;                      // FP64 residual (refinement modes)
  void* tmp64;                    // FP64 odd temporary (eo)
  void* basis;                    // m+1 Krylov vectors in the working precision
  void* tmplo;                    // odd temporary in the working precision (eo)
  void* rlo;                      // inner rhs (refinement modes)
  void* dlo;                      // inner solution (refinement modes)
  zd *part, *hcol, *coef, *nrm, *H, *sn, *g, *y;
  zd* hcol2;   // second-pass dots (CGS2)
  double* sk;  // per basis vector and rhs: v_k = sk[k] u_k (the stored vectors are unnormalised)
  double *cs, *bref, *ibref, *beta, *scl, *est, *fin, *fout, *rel;
  int *live, *steps, *flags, *nlive;
  // block GMRES (one block Krylov space for all rhs): block Hessenberg
  // ((m+1) b x m b), its rotations, the rotated right-hand side ((m+1) b x b),
  // the Gram blocks of a step, the triangular factor of the new block and its
  // inverse, the least-squares solution and the Gram partial sums
  bool blk = false;
  unsigned gblk = 0;
  zd *bH = nullptr, *bsn = nullptr, *bG = nullptr, *bHc = nullptr, *bR = nullptr, *bRi = nullptr, *bW = nullptr,
     *bY = nullptr, *bpart = nullptr;
  double* bcs = nullptr;
  int* bact = nullptr;

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
    Ci64 = (clov && eo) ? a.take(V * 42 * 16) : nullptr;
    Clo = (clov && mode) ? a.take(V * 42 * esize(pw)) : nullptr;
    Cilo = (clov && eo && mode) ? a.take(V * 42 * esize(pw)) : nullptr;
    part = (zd*)a.take((size_t)nblk * DOT_KB * nrhs * sizeof(zd));
    hcol = (zd*)a.take((size_t)(m + 1) * nrhs * sizeof(zd));
    hcol2 = gs == 1 ? (zd*)a.take((size_t)(m + 1) * nrhs * sizeof(zd)) : nullptr;
    coef = (zd*)a.take((size_t)(m + 1) * nrhs * sizeof(zd));
    sk = (double*)a.take((size_t)(m + 1) * nrhs * sizeof(double));
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
    if (blk) {
      const size_t b = (size_t)nrhs, mb = (size_t)m * b;
      bH = (zd*)a.take((m + 1) * b * mb * sizeof(zd));
      bsn = (zd*)a.take(mb * b * sizeof(zd));
      bcs = (double*)a.take(mb * b * sizeof(double));
      bG = (zd*)a.take((m + 1) * b * b * sizeof(zd));
      bHc = (zd*)a.take((m + 1) * b * b * sizeof(zd));
      bR = (zd*)a.take(b * b * sizeof(zd));
      bRi = (zd*)a.take(b * b * sizeof(zd));
      bW = (zd*)a.take(b * b * sizeof(zd));
      bY = (zd*)a.take(mb * b * sizeof(zd));
      bpart = (zd*)a.take((size_t)gblk * BG_KB * b * b * sizeof(zd));
      bact = (int*)a.take((b + 8) * sizeof(int));  // activity, breakdown flag, working count, start flags
    }
  }

  void* Vk(int prec, int k) const { return (char*)basis + (size_t)k * nelem * esize(prec); }
  unsigned small_grid() const { return (unsigned)((nrhs + 63) / 64); }

  // out = A in, in the working precision `prec` (A = S with eo, else D)
  hipError_t apply(int prec, const void* in, void* out, const int* lv) {
    const void* U = prec == LQCD_F64 ? U64 : Ulo;
    if (clov) {  // pass 1 tmp_o = D_oo^{-1} H_oe in; pass 2 out = (d - C_e) in - H_eo tmp_o / 4
      const void* Cp = prec == LQCD_F64 ? C64 : Clo;
      if (!eo) return wilson_full_clover(&lat, U, Cp, in, out, nrhs, d, -0.5, LQCD_LAYOUT2, prec, dag, s);
      void* t = prec == LQCD_F64 ? tmp64 : tmplo;
      hipError_t e = wilson_eo_clover(&lat, U, in, nullptr, t, 1, nrhs, 0.0, 1.0, LQCD_LAYOUT2, prec, dag, lv, nullptr,
                                      prec == LQCD_F64 ? Ci64 : Cilo, s);
      if (e != hipSuccess) return e;
      return wilson_eo_clover(&lat, U, t, in, out, 0, nrhs, d, -0.25, LQCD_LAYOUT2, prec, dag, lv, Cp, nullptr, s);
    }
    if (eo) {
      void* t = prec == LQCD_F64 ? tmp64 : tmplo;
      return schur_apply(&lat, U, in, out, t, nrhs, d, LQCD_LAYOUT2, prec, dag, lv, s);
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

// One lattice of a solve: its solver state, its ABI input/output and the
// vectors the current GMRES run works on.
struct Task {
  Solver S;
  const void* U;       // FP64 links (caller's)
  const void* b_abi;
  void* x_abi;
  int layout;
  int abi_nrhs = 0, col0 = 0;  // this task solves columns col0.. of ABI blocks of abi_nrhs rhs (0: all)
  HostState hs;
  void* x;             // solution of the current GMRES run
  const void* b;       // right-hand side of the current GMRES run
  const double* bref;  // per-rhs reference norm of the current run
};

// All lattices of one solve, advanced in lock-step on one stream.  With
// `graph`, the kernels of Arnoldi step j (for every lattice) are captured
// into a HIP graph the first time they run and replayed in later cycles.
// With several lattices, each lattice's Gram-Schmidt and Givens kernels of a
// step run on a stream of its own (forked from and joined back to the
// group's stream around the one batched Wilson launch), so the small
// kernels of different lattices overlap, and lattices with no rhs left in
// the cycle are left out of the launches; captured step graphs are keyed by
// the set of lattices they launch.
struct Group {
  std::vector<Task> T;
  hipStream_t s;
  int m;
  bool graph;
  std::map<std::tuple<int, int, unsigned>, hipGraphExec_t> exec;  // (precision, step j, lattice mask)
  std::map<std::tuple<int, int, unsigned>, int> seen;              // occurrences of uncaptured keys
  int* pinned;                          // 2 ints per lattice
  hipEvent_t ev[2];
  bool block = false;                   // block GMRES (one lattice) instead of batched
  std::vector<hipStream_t> ts;          // per-lattice streams (several lattices only)
  std::vector<hipEvent_t> tev;          // per-lattice join events
  hipEvent_t fork = nullptr;
};

static unsigned mask_of(const std::vector<int>& act) {
  unsigned m = 0;
  for (int k : act) m |= 1u << k;
  return m;
}

// out = A in for every lattice, in precision prec (in/out chosen per task)
template <class In, class Out>
static hipError_t apply_all(Group& G, int prec, In in_of, Out out_of, bool masked, const std::vector<int>& act) {
  if (G.T.size() == 1) {
    Solver& S = G.T[0].S;
    return S.apply(prec, in_of(G.T[0]), out_of(G.T[0]), masked ? S.live : nullptr);
  }
  batch_desc d;
  d.n = (int)act.size();
  if (d.n == 0) return hipSuccess;
  const bool eo = G.T[0].S.eo;
  const bool dag = G.T[0].S.dag;
  for (int i = 0; i < d.n; ++i) {
    Solver& S = G.T[act[i]].S;
    batch_prob& b = d.p[i];
    b.g = make_geo4(&S.lat);
    b.U = prec == LQCD_F64 ? S.U64 : S.Ulo;
    b.live = masked ? S.live : nullptr;
    b.nrhs = S.nrhs;
    if (eo) {  // first hop pass: tmp_o = H_oe in
      b.in = in_of(G.T[act[i]]);
      b.xin = nullptr;
      b.out = prec == LQCD_F64 ? S.tmp64 : S.tmplo;
      b.parity = 1;
      b.alpha = 0.0;
      b.beta = 1.0;
    } else {
      b.in = in_of(G.T[act[i]]);
      b.xin = nullptr;
      b.out = out_of(G.T[act[i]]);
      b.parity = -1;
      b.alpha = S.d;
      b.beta = -0.5;
    }
  }
  hipError_t e = wilson_batch(d, prec, dag, G.s);
  if (e != hipSuccess || !eo) return e;
  for (int i = 0; i < d.n; ++i) {  // second pass: out_e = d in - H_eo tmp_o / (4 d)
    Solver& S = G.T[act[i]].S;
    batch_prob& b = d.p[i];
    b.in = prec == LQCD_F64 ? S.tmp64 : S.tmplo;
    b.xin = in_of(G.T[act[i]]);
    b.out = out_of(G.T[act[i]]);
    b.parity = 0;
    b.alpha = S.d;
    b.beta = -0.25 / S.d;
  }
  return wilson_batch(d, prec, dag, G.s);
}

// The kernels of Arnoldi step j for the lattices in `act` (w = A v_j, CGS,
// Givens, normalisation).
static hipError_t gs_step(Task& t, int prec, int j, int m, double sc, double tol, int fixed, hipStream_t s) {
  Solver& S = t.S;
  hipError_t e;
  const size_t nel = S.nelem;
  void* w = S.Vk(prec, j + 1);
  const int nc = (j + 1) * S.nrhs;
  if (S.gs == 2) {
    // modified Gram-Schmidt: d_k = <u_k, w> against the vector already
    // orthogonalised to u_0 .. u_{k-1}, then w -= sk[k]^2 d_k u_k
    for (int k = 0; k <= j; ++k) {
      if ((e = dot_parts(prec, S.basis, nel, k, 1, w, nel, S.nrhs, S.live, S.part, S.nblk, s)) != hipSuccess) return e;
      if ((e = reduce_parts(S.part, S.nblk, 1, S.nrhs, sc, S.hcol + (size_t)k * S.nrhs, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_cgs_coef, dim3(((k + 1) * S.nrhs + 255) / 256), dim3(256), 0, s, k + 1, S.nrhs, S.hcol,
                         S.sk, S.coef);
      if ((e = cgs_update(prec, S.Vk(prec, k), nel, 1, S.coef + (size_t)k * S.nrhs, w, nel, S.nrhs, S.live, S.part,
                          S.nblk, s)) != hipSuccess)
        return e;
    }
  } else {
    // classical Gram-Schmidt: all dots against the same w, one fused update;
    // CGS2 repeats the pass on the updated vector and adds its dots
    for (int pass = 0; pass < (S.gs == 1 ? 2 : 1); ++pass) {
      zd* hc = pass == 0 ? S.hcol : S.hcol2;
      for (int k0 = 0; k0 <= j; k0 += DOT_KB) {
        const int K = (j + 1 - k0) < DOT_KB ? (j + 1 - k0) : DOT_KB;
        if ((e = dot_parts(prec, S.basis, nel, k0, K, w, nel, S.nrhs, S.live, S.part, S.nblk, s)) != hipSuccess)
          return e;
        if ((e = reduce_parts(S.part, S.nblk, K, S.nrhs, sc, hc + (size_t)k0 * S.nrhs, s)) != hipSuccess) return e;
      }
      hipLaunchKernelGGL(k_cgs_coef, dim3((nc + 255) / 256), dim3(256), 0, s, j + 1, S.nrhs, hc, S.sk, S.coef);
      if ((e = cgs_update(prec, S.basis, nel, j + 1, S.coef, w, nel, S.nrhs, S.live, S.part, S.nblk, s)) !=
          hipSuccess)
        return e;
      if (pass == 1) hipLaunchKernelGGL(k_add_zd, dim3((nc + 255) / 256), dim3(256), 0, s, nc, S.hcol2, S.hcol);
    }
  }
  if ((e = reduce_parts(S.part, (int)cgs_update_parts(prec, nel, S.nrhs, S.nblk), 1, S.nrhs, sc, S.nrm, s)) !=
      hipSuccess)
    return e;
  const int lazy = prec == LQCD_F64;
  hipLaunchKernelGGL(k_arnoldi_col, dim3(S.small_grid()), dim3(64), 0, s, j, m, S.nrhs, S.hcol, S.nrm, S.H, S.cs,
                     S.sn, S.g, t.bref, tol, fixed, lazy, S.live, S.steps, S.est, S.sk, S.scl);
  if (!lazy && (e = scale_rhs(prec, w, nel, S.nrhs, S.scl, S.live, s)) != hipSuccess) return e;
  return hipSuccess;
}

static hipError_t arnoldi_step(Group& G, int prec, int j, double sc, double tol, int fixed,
                               const std::vector<int>& act) {
  hipStream_t s = G.s;
  const int m = G.m;
  hipError_t e = apply_all(
      G, prec, [&](Task& t) -> const void* { return t.S.Vk(prec, j); }, [&](Task& t) -> void* { return t.S.Vk(prec, j + 1); },
      true, act);
  if (e != hipSuccess) return e;
  if (G.ts.empty()) {
    for (int k : act)
      if ((e = gs_step(G.T[k], prec, j, m, sc, tol, fixed, s)) != hipSuccess) return e;
    return hipGetLastError();
  }
  // fork: every lattice's kernels on its own stream after the batched apply; join
  if ((e = hipEventRecord(G.fork, s)) != hipSuccess) return e;
  for (int k : act) {
    if ((e = hipStreamWaitEvent(G.ts[k], G.fork, 0)) != hipSuccess) return e;
    if ((e = gs_step(G.T[k], prec, j, m, sc, tol, fixed, G.ts[k])) != hipSuccess) return e;
    if ((e = hipEventRecord(G.tev[k], G.ts[k])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, G.tev[k], 0)) != hipSuccess) return e;
  }
  return hipGetLastError();
}

// With graphs, a step is captured the second time its (precision, step,
// lattice set) occurs and replayed from then on; a set that occurs once (a
// lattice dropping out at some step of some cycle) runs eagerly instead of
// paying for a capture it would never reuse.
static hipError_t run_step(Group& G, int prec, int j, double sc, double tol, int fixed, const std::vector<int>& act) {
  if (!G.graph) return arnoldi_step(G, prec, j, sc, tol, fixed, act);
  const auto key = std::make_tuple(prec, j, mask_of(act));
  if (!G.exec.count(key) && ++G.seen[key] < 2) return arnoldi_step(G, prec, j, sc, tol, fixed, act);
  hipGraphExec_t& ex = G.exec[key];
  if (!ex) {
    hipError_t e = hipStreamBeginCapture(G.s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e2 = arnoldi_step(G, prec, j, sc, tol, fixed, act);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(G.s, &g);
    if (e2 != hipSuccess) return e2;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
  }
  return hipGraphLaunch(ex, G.s);
}

// One batched GMRES(m) run of A x = b for every lattice, in precision `prec`,
// vectors scaled by `c` (stored value = c x true value).  Each task's x holds
// the initial guess (zero if x_zero).  Runs at most max_cycles cycles.
static int run_gmres(Group& G, int prec, double tol, int max_cycles, int fixed, bool x_zero, double c) {
  const double sc = 1.0 / (c * c);
  hipStream_t s = G.s;
  const int m = G.m;
  const int nt = (int)G.T.size();
  // lattices that may still have work: one whose every rhs is at tolerance at
  // a cycle start keeps its x and takes no further part in this run
  std::vector<int> open(nt);
  for (int k = 0; k < nt; ++k) open[k] = k;
  for (int cycle = 0; cycle < max_cycles && !open.empty(); ++cycle) {
    // true residual r = b - A x into v_0, |r| per rhs
    if (cycle == 0 && x_zero) {
      for (int k : open) {
        Task& t = G.T[k];
        HIPCHK(convert(prec, t.b, prec, t.S.Vk(prec, 0), t.S.nelem, t.S.nrhs, nullptr, s));
        HIPCHK(t.S.norms(prec, t.S.Vk(prec, 0), sc, nullptr));
      }
    } else {
      HIPCHK(apply_all(
          G, prec, [&](Task& t) -> const void* { return t.x; }, [&](Task& t) -> void* { return t.S.Vk(prec, 0); },
          false, open));
      for (int k : open) {
        Task& t = G.T[k];
        HIPCHK(b_minus_y(prec, t.b, t.S.Vk(prec, 0), t.S.nelem, t.S.nrhs, nullptr, t.S.part, t.S.nblk, s));
        HIPCHK(reduce_parts(t.S.part, t.S.nblk, 1, t.S.nrhs, sc, t.S.nrm, s));
      }
    }
    std::vector<int> fl(2 * nt, 0);
    for (int k : open) {
      Solver& S = G.T[k].S;
      HIPCHK(hipMemsetAsync(S.flags, 0, 2 * sizeof(int), s));
      hipLaunchKernelGGL(k_cycle_start, dim3(S.small_grid()), dim3(64), 0, s, S.nrhs, m, S.nrm, G.T[k].bref, tol,
                         fixed, prec == LQCD_F64, S.live, S.steps, S.g, S.sk, S.scl, S.beta, S.flags);
      HIPCHK(hipMemcpyAsync(&fl[2 * k], S.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int> act;
    for (int k : open) {
      if (fl[2 * k + 1]) return fail(LQCD_ERR_NONFINITE, "gmres: non-finite residual norm");
      if (fl[2 * k]) act.push_back(k);
    }
    open = act;
    if (act.empty()) break;
    for (int k : act) {
      Task& t = G.T[k];
      std::vector<int> lv(t.S.nrhs);
      HIPCHK(hipMemcpy(lv.data(), t.S.live, t.S.nrhs * sizeof(int), hipMemcpyDeviceToHost));
      for (int r = 0; r < t.S.nrhs; ++r) t.hs.restarts[r] += lv[r];
      if (prec != LQCD_F64) HIPCHK(scale_rhs(prec, t.S.Vk(prec, 0), t.S.nelem, t.S.nrhs, t.S.scl, t.S.live, s));
    }
    std::vector<int> step_act = act;  // lattices with live rhs in this cycle's steps
    for (int j = 0; j < m; ++j) {
      HIPCHK(run_step(G, prec, j, sc, tol, fixed, step_act));
      // pipelined exit test: read the live counts of the previous step while
      // this one runs; a lattice with none left drops out of the next steps
      for (int k : step_act) {
        Solver& S = G.T[k].S;
        hipLaunchKernelGGL(k_count_live, dim3(1), dim3(1), 0, s, S.nrhs, S.live, S.nlive + (j & 1));
        HIPCHK(hipMemcpyAsync(G.pinned + 2 * k + (j & 1), S.nlive + (j & 1), sizeof(int), hipMemcpyDeviceToHost,
                              s));
      }
      HIPCHK(hipEventRecord(G.ev[j & 1], s));
      if (j >= 1) {
        HIPCHK(hipEventSynchronize(G.ev[(j - 1) & 1]));
        std::vector<int> still;
        for (int k : step_act)
          if (G.pinned[2 * k + ((j - 1) & 1)]) still.push_back(k);
        if (still.empty()) break;
        step_act = still;
      }
    }
    std::vector<std::vector<int>> steps_h(nt);
    std::vector<std::vector<double>> est_h(nt);
    for (int k : act) {
      Task& t = G.T[k];
      Solver& S = t.S;
      hipLaunchKernelGGL(k_lsq, dim3(S.small_grid()), dim3(64), 0, s, m, S.nrhs, S.H, S.g, S.steps, S.sk, S.y);
      HIPCHK(lincomb(prec, S.basis, S.nelem, m, S.y, S.steps, prec, t.x, S.nelem, S.nrhs, 1.0, s));
      steps_h[k].resize(S.nrhs);
      est_h[k].resize(S.nrhs);
      HIPCHK(hipMemcpyAsync(steps_h[k].data(), S.steps, S.nrhs * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(est_h[k].data(), S.est, S.nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    for (int k : act)
      for (int r = 0; r < G.T[k].S.nrhs; ++r) {
        G.T[k].hs.iters[r] += steps_h[k][r];
        if (steps_h[k][r]) G.T[k].hs.est[r] = est_h[k][r];
      }
    x_zero = false;
  }
  return LQCD_OK;
}


// Restarted block GMRES(m) on one lattice, FP64: x (the task's current
// vector) is refined in place; per-rhs statistics go to t.hs.
static int run_block_gmres(Task& t, double tol, int max_cycles, int fixed, bool x_zero) {
  Solver& S = t.S;
  hipStream_t s = S.s;
  const int b = S.nrhs, m = S.m;
  const size_t nel = S.nelem, nrows = nel / b, bb = (size_t)b * b;
  int* bad = S.bact + b;       // rank-deficiency flag of the last factorisation
  int* working = S.bact + b + 1;
  int* startf = S.bact + b + 2;  // 2 ints
  auto V = [&](int k) { return (zd*)S.Vk(LQCD_F64, k); };
  for (int cycle = 0; cycle < max_cycles; ++cycle) {
    zd* v0 = V(0);
    if (cycle == 0 && x_zero) {
      HIPCHK(convert(LQCD_F64, t.b, LQCD_F64, v0, nel, b, nullptr, s));
      HIPCHK(S.norms(LQCD_F64, v0, 1.0, nullptr));
    } else {
      HIPCHK(S.apply(LQCD_F64, t.x, v0, nullptr));
      HIPCHK(b_minus_y(LQCD_F64, t.b, v0, nel, b, nullptr, S.part, S.nblk, s));
      HIPCHK(reduce_parts(S.part, S.nblk, 1, b, 1.0, S.nrm, s));
    }
    hipLaunchKernelGGL(k_bstart, dim3(1), dim3(1), 0, s, b, S.nrm, t.bref, tol, fixed, S.bact, S.fin, startf);
    int st[2];
    std::vector<int> act(b);
    HIPCHK(hipMemcpyAsync(st, startf, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(act.data(), S.bact, b * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st[1]) return fail(LQCD_ERR_NONFINITE, "block gmres: non-finite residual norm");
    if (st[0] == 0) break;
    // thin QR of the residual block R0 = V_0 S; columns that make it rank
    // deficient (dependent on earlier ones) sit out this cycle, one at a time
    int deficient = 0;
    for (int attempt = 0; attempt <= b; ++attempt) {
      HIPCHK(scale_rhs(LQCD_F64, v0, nel, b, S.fin, nullptr, s));
      HIPCHK(bgram_parts(v0, 0, 1, v0, nrows, b, S.bpart, S.gblk, s));
      HIPCHK(bgram_reduce(S.bpart, S.gblk, 1, b, S.bW, s));
      hipLaunchKernelGGL(k_bchol, dim3(1), dim3(64), 0, s, b, S.bact, S.bW, S.bR, S.bRi, bad, 1, S.fin);
      HIPCHK(hipMemcpyAsync(&deficient, bad, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (deficient != 2) break;
    }
    if (deficient) return fail(LQCD_ERR_NONFINITE, "block gmres: residual block could not be factorised");
    HIPCHK(hipMemcpyAsync(act.data(), S.bact, b * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int q = 0; q < b; ++q) t.hs.restarts[q] += act[q];
    HIPCHK(bgemm(v0, nullptr, 0.0, 1.0, v0, 0, 1, S.bRi, nrows, b, s));
    hipLaunchKernelGGL(k_binit, dim3(4), dim3(256), 0, s, m, b, S.bR, S.bG);
    int steps = 0;
    for (int j = 0; j < m; ++j) {
      zd* w = V(j + 1);
      HIPCHK(S.apply(LQCD_F64, V(j), w, nullptr));
      // block classical Gram-Schmidt: H_ij = V_i^H w for i <= j, then w -= sum_i V_i H_ij
      for (int k0 = 0; k0 <= j; k0 += BG_KB) {
        const int K = (j + 1 - k0) < BG_KB ? (j + 1 - k0) : BG_KB;
        HIPCHK(bgram_parts(V(k0), nel, K, w, nrows, b, S.bpart, S.gblk, s));
        HIPCHK(bgram_reduce(S.bpart, S.gblk, K, b, S.bHc + (size_t)k0 * bb, s));
      }
      for (int k0 = 0; k0 <= j; k0 += BM_KB) {
        const int K = (j + 1 - k0) < BM_KB ? (j + 1 - k0) : BM_KB;
        HIPCHK(bgemm(w, w, 1.0, -1.0, V(k0), nel, K, S.bHc + (size_t)k0 * bb, nrows, b, s));
      }
      // thin QR of the new block: w = V_{j+1} R
      HIPCHK(bgram_parts(w, 0, 1, w, nrows, b, S.bpart, S.gblk, s));
      HIPCHK(bgram_reduce(S.bpart, S.gblk, 1, b, S.bW, s));
      hipLaunchKernelGGL(k_bchol, dim3(1), dim3(64), 0, s, b, S.bact, S.bW, S.bR, S.bRi, bad, 0, S.fin);
      hipLaunchKernelGGL(k_bhess, dim3(1), dim3(256), 0, s, j, m, b, S.bHc, S.bR, S.bH, S.bcs, S.bsn, S.bG, S.bact,
                         t.bref, tol, fixed, S.est, working);
      int fl[2];
      HIPCHK(hipMemcpyAsync(fl, bad, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      steps = j + 1;
      if (fl[0] || fl[1] == 0) break;  // rank-deficient block (the step still counts) or all converged
      if (j + 1 < m) HIPCHK(bgemm(w, nullptr, 0.0, 1.0, w, 0, 1, S.bRi, nrows, b, s));
    }
    // least squares and x += [V_0 .. V_{steps-1}] Y
    hipLaunchKernelGGL(k_bsolve, dim3(1), dim3((steps * b + 63) / 64 * 64), 0, s, steps, m, b, S.bH, S.bG, S.bY);
    for (int k0 = 0; k0 < steps; k0 += BM_KB) {
      const int K = (steps - k0) < BM_KB ? (steps - k0) : BM_KB;
      HIPCHK(bgemm(t.x, t.x, 1.0, 1.0, V(k0), nel, K, S.bY + (size_t)k0 * bb, nrows, b, s));
    }
    std::vector<double> est(b);
    HIPCHK(hipMemcpyAsync(est.data(), S.est, b * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int q = 0; q < b; ++q)
      if (act[q]) {
        t.hs.iters[q] += steps;
        t.hs.est[q] = est[q];
      }
    x_zero = false;
  }
  return LQCD_OK;
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
  if (p->gs < 0 || p->gs > 2) return fail(LQCD_ERR_ARG, "gmres: unknown orthogonalisation gs = %d", p->gs);
  if (p->rhs_block < 0) return fail(LQCD_ERR_ARG, "gmres: rhs_block must be >= 0");
  return LQCD_OK;
}

static void setup(Solver& S, const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p, bool clov = false,
                  bool blk = false) {
  S.lat = *lat;
  S.clov = clov;
  S.blk = blk;
  S.V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  S.eo = p->eo ? 1 : 0;
  S.nsite = S.eo ? S.V / 2 : S.V;
  S.nelem = S.nsite * 12 * (size_t)nrhs;
  S.nrhs = nrhs;
  S.m = p->restart;
  S.mode = p->mode;
  S.plo = p->mode == 1 ? LQCD_F32 : LQCD_F16;
  S.gs = blk ? 0 : p->gs;
  S.dag = p->dagger != 0;
  S.nblk = reduce_grid(S.nelem);
  S.gblk = blk ? bgram_blocks(S.nelem / nrhs) : 0;
}

static size_t task_bytes(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p, bool clov = false,
                         bool blk = false) {
  Solver S;
  setup(S, lat, nrhs, p, clov, blk);
  Arena a{nullptr, 0, 0};
  S.layout(a);
  return (a.off + 511) & ~(size_t)255;
}

// |b_e|^2 + |b_o|^2 (or |b|^2) of the task's full-system source into nrm
static hipError_t full_norm2(Task& t, const void* ve, const void* vo, hipStream_t s) {
  Solver& S = t.S;
  hipError_t e;
  if (!S.eo) {
    if ((e = norm_parts(LQCD_F64, ve, S.nelem, S.nrhs, nullptr, S.part, S.nblk, s)) != hipSuccess) return e;
    return reduce_parts(S.part, S.nblk, 1, S.nrhs, 1.0, S.nrm, s);
  }
  if ((e = norm_parts(LQCD_F64, ve, S.nelem, S.nrhs, nullptr, S.part, S.nblk, s)) != hipSuccess) return e;
  if ((e = reduce_parts(S.part, S.nblk, 1, S.nrhs, 1.0, S.hcol, s)) != hipSuccess) return e;
  if ((e = norm_parts(LQCD_F64, vo, S.nelem, S.nrhs, nullptr, S.part, S.nblk, s)) != hipSuccess) return e;
  if ((e = reduce_parts(S.part, S.nblk, 1, S.nrhs, 1.0, S.nrm, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(S.part, S.hcol, S.nrhs * sizeof(zd), hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(S.part + S.nrhs, S.nrm, S.nrhs * sizeof(zd), hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return e;
  return reduce_parts(S.part, 2, 1, S.nrhs, 1.0, S.nrm, s);
}

// The whole solve for a group of lattices: ingest, (refined) GMRES,
// reconstruction, full-system true residual, write-back and statistics.
static int solve_group(Group& G, const lqcd_solver_params* params, lqcd_rhs_stats* stats) {
  hipStream_t s = G.s;
  const double tol = params->tol;
  const int fixed = params->fixed_iters ? 1 : 0;
  const bool x_zero = !params->x_is_guess;
  const int mode = params->mode;
  for (Task& t : G.T) {
    Solver& S = t.S;
    const int dims[4] = {S.lat.dims[0], S.lat.dims[1], S.lat.dims[2], S.lat.dims[3]};
    t.hs.iters.assign(S.nrhs, 0);
    t.hs.restarts.assign(S.nrhs, 0);
    t.hs.outer.assign(S.nrhs, 0);
    t.hs.est.assign(S.nrhs, 0.0);
    HIPCHK(pack(t.layout, true, (void*)t.b_abi, S.be, S.bo, dims, S.nrhs, S.eo, s, t.abi_nrhs, t.col0));
    HIPCHK(full_norm2(t, S.be, S.bo, s));
    hipLaunchKernelGGL(k_sqrt_scale, dim3(S.small_grid()), dim3(64), 0, s, S.nrhs, S.nrm, 1.0, S.bref);
    if (params->x_is_guess) {
      HIPCHK(pack(t.layout, true, t.x_abi, S.xe, S.xo, dims, S.nrhs, S.eo, s, t.abi_nrhs, t.col0));
      hipLaunchKernelGGL(k_zero_mask, dim3(S.small_grid()), dim3(64), 0, s, S.nrhs, S.bref, S.fin);
      HIPCHK(scale_rhs(LQCD_F64, S.xe, S.nelem, S.nrhs, S.fin, nullptr, s));
    } else {
      HIPCHK(hipMemsetAsync(S.xe, 0, S.nelem * 16, s));
    }
    if (S.clov && S.eo) {  // D_oo^{-1} = ((4+m0) - C_o)^{-1}, site by site
      HIPCHK(hipMemsetAsync(S.flags, 0, 2 * sizeof(int), s));
      HIPCHK(clover_invert(&S.lat, S.C64, S.Ci64, S.d, LQCD_F64, S.flags, s));
      int sing = 0;
      HIPCHK(hipMemcpyAsync(&sing, S.flags, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (sing) return fail(LQCD_ERR_SINGULAR, "gmres: (4 + m0) - C(x) is singular on some odd site");
    }
    if (S.eo && S.clov) {  // b'_e = b_e + (1/2) H_eo D_oo^{-1} b_o
      HIPCHK(clover_site_mul(&S.lat, S.Ci64, S.bo, S.tmp64, 1, S.nrhs, 1.0, LQCD_LAYOUT2, LQCD_F64, s));
      HIPCHK(wilson_eo(&S.lat, t.U, S.tmp64, S.be, S.bp, 0, S.nrhs, 1.0, 0.5, LQCD_LAYOUT2, LQCD_F64, S.dag, nullptr,
                       s));
    } else if (S.eo) {  // b'_e = b_e - D_eo D_oo^{-1} b_o = b_e + (1/2) H_eo b_o / (4+m0)
      HIPCHK(wilson_eo(&S.lat, t.U, S.bo, S.be, S.bp, 0, S.nrhs, 1.0, 0.5 / S.d, LQCD_LAYOUT2, LQCD_F64, S.dag,
                       nullptr, s));
    }
  }
  if (mode == 0) {
    for (Task& t : G.T) {
      t.x = t.S.xe;
      t.b = t.S.bp;
      t.bref = t.S.bref;
    }
    int rc = G.block ? run_block_gmres(G.T[0], tol, params->max_restarts, fixed, x_zero)
                     : run_gmres(G, LQCD_F64, tol, params->max_restarts, fixed, x_zero, 1.0);
    if (rc) return rc;
  } else {
    // iterative refinement: FP64 residual and update, inner GMRES in plo
    const int plo = G.T[0].S.plo;
    const double itol = params->inner_tol > 0 ? params->inner_tol : (plo == LQCD_F32 ? 1e-4 : 1e-2);
    for (Task& t : G.T) {
      HIPCHK(convert_links(t.U, plo, t.S.Ulo, 4 * t.S.V * 9, s));
      if (t.S.clov) HIPCHK(convert_links(t.S.C64, plo, t.S.Clo, t.S.V * 42, s));
      if (t.S.clov && t.S.eo) HIPCHK(convert_links(t.S.Ci64, plo, t.S.Cilo, t.S.V * 42, s));
    }
    for (int outer = 0; outer < params->max_outer; ++outer) {
      if (outer == 0 && x_zero) {
        for (Task& t : G.T) {
          HIPCHK(convert(LQCD_F64, t.S.bp, LQCD_F64, t.S.r64, t.S.nelem, t.S.nrhs, nullptr, s));
          HIPCHK(t.S.norms(LQCD_F64, t.S.r64, 1.0, nullptr));
        }
      } else {
        std::vector<int> all(G.T.size());
        for (size_t k = 0; k < all.size(); ++k) all[k] = (int)k;
        HIPCHK(apply_all(
            G, LQCD_F64, [&](Task& t) -> const void* { return t.S.xe; }, [&](Task& t) -> void* { return t.S.r64; },
            false, all));
        for (Task& t : G.T) {
          HIPCHK(b_minus_y(LQCD_F64, t.S.bp, t.S.r64, t.S.nelem, t.S.nrhs, nullptr, t.S.part, t.S.nblk, s));
          HIPCHK(reduce_parts(t.S.part, t.S.nblk, 1, t.S.nrhs, 1.0, t.S.nrm, s));
        }
      }
      const int nt = (int)G.T.size();
      std::vector<int> fl(2 * nt);
      for (int k = 0; k < nt; ++k) {
        Solver& S = G.T[k].S;
        const double c = plo == LQCD_F16 ? sqrt((double)S.nsite * 12.0) : 1.0;
        HIPCHK(hipMemsetAsync(S.flags, 0, 2 * sizeof(int), s));
        hipLaunchKernelGGL(k_ir_factors, dim3(S.small_grid()), dim3(64), 0, s, S.nrhs, S.nrm, S.bref, tol, c, S.fin,
                           S.fout, S.ibref, S.rel, S.flags);
        HIPCHK(hipMemcpyAsync(&fl[2 * k], S.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
      }
      HIPCHK(hipStreamSynchronize(s));
      int active = 0;
      for (int k = 0; k < nt; ++k) {
        if (fl[2 * k + 1]) return fail(LQCD_ERR_NONFINITE, "gmres: non-finite residual norm in refinement");
        active += fl[2 * k];
      }
      if (active == 0) break;
      for (Task& t : G.T) {
        std::vector<double> fo(t.S.nrhs);
        HIPCHK(hipMemcpy(fo.data(), t.S.fout, t.S.nrhs * sizeof(double), hipMemcpyDeviceToHost));
        for (int r = 0; r < t.S.nrhs; ++r) t.hs.outer[r] += fo[r] != 0.0;
        HIPCHK(convert(LQCD_F64, t.S.r64, plo, t.S.rlo, t.S.nelem, t.S.nrhs, t.S.fin, s));
        HIPCHK(hipMemsetAsync(t.S.dlo, 0, t.S.nelem * esize(plo), s));
        t.x = t.S.dlo;
        t.b = t.S.rlo;
        t.bref = t.S.ibref;
      }
      // the F16 scale differs per lattice only through its size; the inner run
      // uses the first lattice's for the dot/norm rescaling, so every lattice
      // of an F16 batch must share its site count (checked by the caller)
      const double c0 = plo == LQCD_F16 ? sqrt((double)G.T[0].S.nsite * 12.0) : 1.0;
      int rc = run_gmres(G, plo, itol, 1, 0, true, c0);
      if (rc) return rc;
      for (Task& t : G.T) HIPCHK(add_scaled(plo, t.S.dlo, t.S.xe, t.S.nelem, t.S.nrhs, t.S.fout, s));
    }
  }
  // reconstruct the odd sites, full-system true residual, write x back
  int all = 1;
  size_t off = 0;
  for (Task& t : G.T) {
    Solver& S = t.S;
    const double d = S.d;
    const int dims[4] = {S.lat.dims[0], S.lat.dims[1], S.lat.dims[2], S.lat.dims[3]};
    void* t1 = S.mode ? S.r64 : S.Vk(LQCD_F64, 0);
    if (S.eo && S.clov) {
      // x_o = D_oo^{-1} (b_o + (1/2) H_oe x_e); r = b - D x with D_pp = (4+m0) - C_p
      HIPCHK(wilson_eo_clover(&S.lat, t.U, S.xe, S.bo, S.xo, 1, S.nrhs, 1.0, 0.5, LQCD_LAYOUT2, LQCD_F64, S.dag,
                              nullptr, nullptr, S.Ci64, s));
      HIPCHK(wilson_eo_clover(&S.lat, t.U, S.xo, S.xe, t1, 0, S.nrhs, d, -0.5, LQCD_LAYOUT2, LQCD_F64, S.dag, nullptr,
                              S.C64, nullptr, s));
      HIPCHK(b_minus_y(LQCD_F64, S.be, t1, S.nelem, S.nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(wilson_eo_clover(&S.lat, t.U, S.xe, S.xo, S.tmp64, 1, S.nrhs, d, -0.5, LQCD_LAYOUT2, LQCD_F64, S.dag,
                              nullptr, S.C64, nullptr, s));
      HIPCHK(b_minus_y(LQCD_F64, S.bo, S.tmp64, S.nelem, S.nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(full_norm2(t, t1, S.tmp64, s));
    } else if (S.clov) {
      HIPCHK(wilson_full_clover(&S.lat, t.U, S.C64, S.xe, t1, S.nrhs, d, -0.5, LQCD_LAYOUT2, LQCD_F64, S.dag, s));
      HIPCHK(b_minus_y(LQCD_F64, S.be, t1, S.nelem, S.nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(reduce_parts(S.part, S.nblk, 1, S.nrhs, 1.0, S.nrm, s));
    } else if (S.eo) {
      // x_o = (b_o + (1/2) H_oe x_e) / (4+m0)
      HIPCHK(wilson_eo(&S.lat, t.U, S.xe, S.bo, S.xo, 1, S.nrhs, 1.0 / d, 0.5 / d, LQCD_LAYOUT2, LQCD_F64, S.dag,
                       nullptr, s));
      // r_e = b_e - [(4+m0) x_e - (1/2) H_eo x_o],  r_o = b_o - [(4+m0) x_o - (1/2) H_oe x_e]
      HIPCHK(wilson_eo(&S.lat, t.U, S.xo, S.xe, t1, 0, S.nrhs, d, -0.5, LQCD_LAYOUT2, LQCD_F64, S.dag, nullptr, s));
      HIPCHK(b_minus_y(LQCD_F64, S.be, t1, S.nelem, S.nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(wilson_eo(&S.lat, t.U, S.xe, S.xo, S.tmp64, 1, S.nrhs, d, -0.5, LQCD_LAYOUT2, LQCD_F64, S.dag, nullptr,
                       s));
      HIPCHK(b_minus_y(LQCD_F64, S.bo, S.tmp64, S.nelem, S.nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(full_norm2(t, t1, S.tmp64, s));
    } else {
      HIPCHK(wilson_full(&S.lat, t.U, S.xe, t1, S.nrhs, d, -0.5, LQCD_LAYOUT2, LQCD_F64, S.dag, s));
      HIPCHK(b_minus_y(LQCD_F64, S.be, t1, S.nelem, S.nrhs, nullptr, S.part, S.nblk, s));
      HIPCHK(reduce_parts(S.part, S.nblk, 1, S.nrhs, 1.0, S.nrm, s));
    }
    HIPCHK(pack(t.layout, false, t.x_abi, S.xe, S.xo, dims, S.nrhs, S.eo, s, t.abi_nrhs, t.col0));
    std::vector<zd> rn(S.nrhs);
    std::vector<double> bn(S.nrhs);
    HIPCHK(hipMemcpyAsync(rn.data(), S.nrm, S.nrhs * sizeof(zd), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(bn.data(), S.bref, S.nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int r = 0; r < S.nrhs; ++r) {
      const double tr = bn[r] > 0 ? sqrt(rn[r].re) / bn[r] : 0.0;
      if (!(tr == tr)) return fail(LQCD_ERR_NONFINITE, "gmres: non-finite true residual for rhs %d", r);
      const int conv = (bn[r] == 0.0) || (tr <= tol);
      all &= conv;
      if (stats) {
        lqcd_rhs_stats& st = stats[off + r];
        st.iters = t.hs.iters[r];
        st.restarts = t.hs.restarts[r];
        st.outer_iters = t.hs.outer[r];
        st.converged = conv;
        st.true_relres = tr;
        st.est_relres = t.hs.est[r];
      }
    }
    off += S.nrhs;
  }
  return (all || fixed) ? LQCD_OK : LQCD_NOT_CONVERGED;
}

// Set up the group's stream, events and pinned buffer, run, and release.
static int run_group(Group& G, const lqcd_solver_params* params, lqcd_rhs_stats* stats, hipStream_t user,
                     bool graph) {
  G.graph = graph;
  G.m = params->restart;
  hipStream_t own = nullptr;
  if (graph) {  // capture needs a stream of its own (not the null stream)
    if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess)
      return fail(LQCD_ERR_HIP, "gmres: stream creation failed");
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) {
      (void)hipEventRecord(e, user);
      (void)hipStreamWaitEvent(own, e, 0);
      (void)hipEventDestroy(e);
    }
    G.s = own;
  } else {
    G.s = user;
  }
  for (Task& t : G.T) t.S.s = G.s;
  G.pinned = nullptr;
  if (hipHostMalloc((void**)&G.pinned, 2 * G.T.size() * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return fail(LQCD_ERR_HIP, "gmres: pinned buffer allocation failed");
  if (hipEventCreateWithFlags(&G.ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&G.ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipHostFree(G.pinned);
    return fail(LQCD_ERR_HIP, "gmres: event creation failed");
  }
  int rc = LQCD_OK;
  if (G.T.size() > 1 && !G.block) {  // per-lattice streams for the Gram-Schmidt kernels of a step
    if (hipEventCreateWithFlags(&G.fork, hipEventDisableTiming) != hipSuccess)
      rc = fail(LQCD_ERR_HIP, "gmres: event creation failed");
    for (size_t k = 0; k < G.T.size() && !rc; ++k) {
      hipStream_t ts = nullptr;
      hipEvent_t te = nullptr;
      if (hipStreamCreateWithFlags(&ts, hipStreamNonBlocking) != hipSuccess) {
        rc = fail(LQCD_ERR_HIP, "gmres: stream creation failed");
        break;
      }
      G.ts.push_back(ts);
      if (hipEventCreateWithFlags(&te, hipEventDisableTiming) != hipSuccess) {
        rc = fail(LQCD_ERR_HIP, "gmres: event creation failed");
        break;
      }
      G.tev.push_back(te);
    }
    if (rc || G.ts.size() != G.T.size() || G.tev.size() != G.T.size()) {
      if (!rc) rc = fail(LQCD_ERR_HIP, "gmres: stream setup failed");
    }
  }
  if (!rc) rc = solve_group(G, params, stats);
  (void)hipStreamSynchronize(G.s);
  for (hipStream_t ts : G.ts) (void)hipStreamSynchronize(ts);
  for (auto& kv : G.exec)
    if (kv.second) (void)hipGraphExecDestroy(kv.second);
  for (hipEvent_t te : G.tev) (void)hipEventDestroy(te);
  for (hipStream_t ts : G.ts) (void)hipStreamDestroy(ts);
  if (G.fork) (void)hipEventDestroy(G.fork);
  (void)hipEventDestroy(G.ev[0]);
  (void)hipEventDestroy(G.ev[1]);
  (void)hipHostFree(G.pinned);
  if (own) (void)hipStreamDestroy(own);
  return rc;
}

}  // namespace lq

using namespace lq;

extern "C" {

void lqcd_solver_defaults(lqcd_solver_params* p) {
  if (p) defaults(p);
}

size_t gmres_workspace_bytes(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p) {
  if (check_lattice(lat) || nrhs < 1 || check_params(p)) return 0;
  const int w = (p->rhs_block > 0 && p->rhs_block < nrhs) ? p->rhs_block : nrhs;
  return task_bytes(lat, w, p) + 256;
}

}  // extern "C"

namespace lq {

// Chunk width of a solve (lqcd_solver_params.rhs_block): the caller's, else
// the full width if the workspace holds it, else among the candidate widths
// the workspace holds the one whose tuned Wilson time (the autotuner's table
// entry for the operator the solve applies most: the odd-even hop pass or
// the full apply, in the inner precision) per rhs is least, counting the
// chunks it takes; without table entries the largest such width.
static int choose_rhs_block(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p, size_t work_bytes,
                            bool clov) {
  if (p->rhs_block > 0) return p->rhs_block < nrhs ? p->rhs_block : nrhs;
  auto fits = [&](int w) { return task_bytes(lat, w, p, clov) + 256 <= work_bytes; };
  if (fits(nrhs)) return nrhs;
  const int prec = p->mode == 0 ? LQCD_F64 : (p->mode == 1 ? LQCD_F32 : LQCD_F16);
  const int kind = p->eo ? KIND_EO : KIND_FULL;
  int best = 0, largest = 0;
  double best_cost = 0.0;
  for (int w : {64, 48, 32, 24, 16, 12, 8, 4, 2, 1}) {
    if (w >= nrhs || !fits(w)) continue;
    if (!largest) largest = w;
    double ms = 0.0;
    if (!tuned_time(kind, lat, w, prec, LQCD_LAYOUT2, &ms)) continue;
    const double cost = ms * (double)((nrhs + w - 1) / w);
    if (!best || cost < best_cost) {
      best = w;
      best_cost = cost;
    }
  }
  return best ? best : largest;
}

// The solve of nrhs rhs in chunks of w consecutive rhs, one after another,
// each with the whole workspace (a chunk is an ordinary solve of its
// columns; the ABI blocks are read and written in place).
static int solve_chunked(const lqcd_lattice* lat, const void* U, const void* C, const void* b, void* x, int nrhs,
                         int w, double m0, int layout, const lqcd_solver_params* params, char* work,
                         lqcd_rhs_stats* stats, hipStream_t stream) {
  int rc_all = LQCD_OK;
  for (int c0 = 0; c0 < nrhs; c0 += w) {
    const int wc = (nrhs - c0) < w ? (nrhs - c0) : w;
    Group G;
    G.T.resize(1);
    Task& t = G.T[0];
    setup(t.S, lat, wc, params, C != nullptr, false);
    t.S.C64 = C;
    t.S.m0 = m0;
    t.S.d = 4.0 + m0;
    t.S.U64 = U;
    t.U = U;
    t.b_abi = b;
    t.x_abi = x;
    t.layout = layout;
    t.abi_nrhs = nrhs;
    t.col0 = c0;
    Arena a{work, 0, 0};
    t.S.layout(a);
    const int rc = run_group(G, params, stats ? stats + c0 : nullptr, stream, params->use_graph != 0);
    if (rc < 0) return rc;
    if (rc == LQCD_NOT_CONVERGED) rc_all = LQCD_NOT_CONVERGED;
  }
  return rc_all;
}

}  // namespace lq

extern "C" {

int gmres_rhs_block(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p, size_t work_bytes) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (nrhs < 1) return fail(LQCD_ERR_ARG, "gmres_rhs_block: nrhs = %d", nrhs);
  if ((rc = check_params(p))) return rc;
  const int w = choose_rhs_block(lat, nrhs, p, work_bytes, false);
  if (!w || task_bytes(lat, w, p) + 256 > work_bytes)
    return fail(LQCD_ERR_WORKSPACE, "gmres_rhs_block: a workspace of %zu bytes holds no chunk", work_bytes);
  return w;
}

static int init_task(Task& t, const lqcd_lattice* lat, const void* U, const void* b, void* x, int nrhs, double m0,
                     int layout, const lqcd_solver_params* p, char* work, const void* C = nullptr,
                     bool blk = false) {
  setup(t.S, lat, nrhs, p, C != nullptr, blk);
  t.S.C64 = C;
  t.S.m0 = m0;
  t.S.d = 4.0 + m0;
  t.S.U64 = U;
  t.U = U;
  t.b_abi = b;
  t.x_abi = x;
  t.layout = layout;
  Arena a{work, 0, 0};
  t.S.layout(a);
  return LQCD_OK;
}

int gmres_solve(const lqcd_lattice* lat, const void* U, const void* b, void* x, int nrhs, double m0, int layout,
                const lqcd_solver_params* params, void* work, size_t work_bytes, lqcd_rhs_stats* stats,
                void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, LQCD_F64))) return rc;
  if ((rc = check_params(params))) return rc;
  if (!U || !b || !x) return fail(LQCD_ERR_ARG, "gmres_solve: null array pointer");
  if (4.0 + m0 == 0.0 && params->eo) return fail(LQCD_ERR_SINGULAR, "gmres_solve: 4 + m0 = 0, D_oo is not invertible");
  const int wb = choose_rhs_block(lat, nrhs, params, work ? work_bytes : 0, false);
  const size_t need = wb ? task_bytes(lat, wb, params) + 256 : task_bytes(lat, 1, params) + 256;
  if (!work || !wb || work_bytes < need)
    return fail(LQCD_ERR_WORKSPACE, "gmres_solve: workspace of %zu bytes given, %zu needed", work_bytes, need);
  char* w = (char*)work + ((256 - ((uintptr_t)work & 255)) & 255);
  if (wb < nrhs) return solve_chunked(lat, U, nullptr, b, x, nrhs, wb, m0, layout, params, w, stats, (hipStream_t)stream);
  Group G;
  G.T.resize(1);
  init_task(G.T[0], lat, U, b, x, nrhs, m0, layout, params, w);
  return run_group(G, params, stats, (hipStream_t)stream, params->use_graph != 0);
}

size_t gmres_workspace_bytes_clover(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p) {
  if (check_lattice(lat) || nrhs < 1 || check_params(p)) return 0;
  const int w = (p->rhs_block > 0 && p->rhs_block < nrhs) ? p->rhs_block : nrhs;
  return task_bytes(lat, w, p, true) + 256;
}

int gmres_solve_clover(const lqcd_lattice* lat, const void* U, const void* C, const void* b, void* x, int nrhs,
                       double m0, int layout, const lqcd_solver_params* params, void* work, size_t work_bytes,
                       lqcd_rhs_stats* stats, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, LQCD_F64))) return rc;
  if ((rc = check_params(params))) return rc;
  if (!U || !C || !b || !x) return fail(LQCD_ERR_ARG, "gmres_solve_clover: null array pointer");
  const int wb = choose_rhs_block(lat, nrhs, params, work ? work_bytes : 0, true);
  const size_t need = wb ? task_bytes(lat, wb, params, true) + 256 : task_bytes(lat, 1, params, true) + 256;
  if (!work || !wb || work_bytes < need)
    return fail(LQCD_ERR_WORKSPACE, "gmres_solve_clover: workspace of %zu bytes given, %zu needed", work_bytes, need);
  char* w = (char*)work + ((256 - ((uintptr_t)work & 255)) & 255);
  if (wb < nrhs) return solve_chunked(lat, U, C, b, x, nrhs, wb, m0, layout, params, w, stats, (hipStream_t)stream);
  Group G;
  G.T.resize(1);
  init_task(G.T[0], lat, U, b, x, nrhs, m0, layout, params, w, C);
  return run_group(G, params, stats, (hipStream_t)stream, params->use_graph != 0);
}

size_t gmres_workspace_bytes_batch(int nprob, const lqcd_problem* probs, const lqcd_solver_params* p) {
  if (nprob < 1 || nprob > LQCD_MAX_BATCH || !probs || check_params(p)) return 0;
  size_t total = 256;
  for (int k = 0; k < nprob; ++k) {
    if (check_lattice(&probs[k].lat) || probs[k].nrhs < 1) return 0;
    total += task_bytes(&probs[k].lat, probs[k].nrhs, p);
  }
  return total;
}

int gmres_solve_batch(int nprob, const lqcd_problem* probs, const lqcd_solver_params* params, void* work,
                      size_t work_bytes, lqcd_rhs_stats* stats, void* stream) {
  if (nprob < 1 || nprob > LQCD_MAX_BATCH)
    return fail(LQCD_ERR_ARG, "gmres_solve_batch: %d problems, need 1..%d", nprob, LQCD_MAX_BATCH);
  if (!probs) return fail(LQCD_ERR_ARG, "gmres_solve_batch: probs is null");
  int rc = check_params(params);
  if (rc) return rc;
  for (int k = 0; k < nprob; ++k) {
    const lqcd_problem& q = probs[k];
    if ((rc = check_lattice(&q.lat))) return rc;
    if (q.nrhs < 1) return fail(LQCD_ERR_ARG, "gmres_solve_batch: problem %d has nrhs = %d", k, q.nrhs);
    if (!q.U || !q.psi || !q.eta) return fail(LQCD_ERR_ARG, "gmres_solve_batch: problem %d has a null pointer", k);
    if (4.0 + q.m0 == 0.0 && params->eo)
      return fail(LQCD_ERR_SINGULAR, "gmres_solve_batch: problem %d has 4 + m0 = 0", k);
    if (params->mode == 2 && q.lat.dims[0] * q.lat.dims[1] * q.lat.dims[2] * q.lat.dims[3] !=
                                 probs[0].lat.dims[0] * probs[0].lat.dims[1] * probs[0].lat.dims[2] * probs[0].lat.dims[3])
      return fail(LQCD_ERR_ARG, "gmres_solve_batch: FP16 refinement needs lattices of one volume");
  }
  const size_t need = gmres_workspace_bytes_batch(nprob, probs, params);
  if (!work || work_bytes < need)
    return fail(LQCD_ERR_WORKSPACE, "gmres_solve_batch: workspace of %zu bytes given, %zu needed", work_bytes, need);
  Group G;
  G.T.resize(nprob);
  char* w = (char*)work + ((256 - ((uintptr_t)work & 255)) & 255);
  for (int k = 0; k < nprob; ++k) {
    const lqcd_problem& q = probs[k];
    init_task(G.T[k], &q.lat, q.U, q.psi, q.eta, q.nrhs, q.m0, LQCD_LAYOUT2, params, w);
    w += task_bytes(&q.lat, q.nrhs, params);
  }
  return run_group(G, params, stats, (hipStream_t)stream, params->use_graph != 0);
}

size_t block_gmres_workspace_bytes(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p) {
  if (check_lattice(lat) || nrhs < 1 || nrhs > LQCD_BLOCK_MAX_RHS || check_params(p) || p->mode != 0) return 0;
  return task_bytes(lat, nrhs, p, false, true) + 256;
}

int block_gmres_solve(const lqcd_lattice* lat, const void* U, const void* b, void* x, int nrhs, double m0, int layout,
                      const lqcd_solver_params* params, void* work, size_t work_bytes, lqcd_rhs_stats* stats,
                      void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, LQCD_F64))) return rc;
  if ((rc = check_params(params))) return rc;
  if (nrhs > LQCD_BLOCK_MAX_RHS)
    return fail(LQCD_ERR_ARG, "block_gmres_solve: nrhs = %d, the block solver takes at most %d", nrhs,
                LQCD_BLOCK_MAX_RHS);
  if (params->mode != 0) return fail(LQCD_ERR_ARG, "block_gmres_solve: only FP64 (mode 0) is supported");
  if (params->use_graph) return fail(LQCD_ERR_ARG, "block_gmres_solve: graph capture is not supported");
  if (!U || !b || !x) return fail(LQCD_ERR_ARG, "block_gmres_solve: null array pointer");
  const size_t need = block_gmres_workspace_bytes(lat, nrhs, params);
  if (!work || work_bytes < need)
    return fail(LQCD_ERR_WORKSPACE, "block_gmres_solve: workspace of %zu bytes given, %zu needed", work_bytes, need);
  if (4.0 + m0 == 0.0 && params->eo)
    return fail(LQCD_ERR_SINGULAR, "block_gmres_solve: 4 + m0 = 0, D_oo is not invertible");
  Group G;
  G.block = true;
  G.T.resize(1);
  char* w = (char*)work + ((256 - ((uintptr_t)work & 255)) & 255);
  init_task(G.T[0], lat, U, b, x, nrhs, m0, layout, params, w, nullptr, true);
  return run_group(G, params, stats, (hipStream_t)stream, false);
}

}  // extern "C"
