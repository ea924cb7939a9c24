// Link force: the gradient of a real loss with respect to the gauge links
// through y = D psi (differentiation of the Sec. III-A.1 operator; the
// derivation is not in the paper, see the formula below).
//
// For dL/dy = g (gradient convention dL = Re <g, dy>) the derivative of D_W
// with respect to the entries of U_mu(x) gives
//   G_mu(x) = -1/2 sum_rhs sum_spin { [(1 - gamma_mu) g(x)] (x) psi(x+mu)^*
//                                    + psi(x) (x) [(1 + gamma_mu) g(x+mu)]^* }
// (colour outer products).  Because (1 -+ gamma)/2 are Hermitian projectors of
// rank two, each spin sum equals the sum over the two components of the
// projected half spinors: sum_s [(1 - gamma) g]_s q_s^* = sum_{s<2} h_s(g) h_s(q)^*
// with h = u - B d (and u + B d for 1 + gamma).  The kernel evaluates
// G = coeff * sum_rhs { h^-(g(x)) (x) h^-(psi(x+mu))^* + h^+(psi(x)) (x) h^+(g(x+mu))^* }
// so coeff = -1/2 is the apply gradient and +1/2 with (g, psi) -> (lambda, x)
// the solve gradient.  With `project`, G is replaced by the su(3) force
// TA(G U^dagger), TA(X) = (X - X^dag)/2 - tr(X - X^dag)/6.
#include "common.h"
#include "wilson.h"

namespace lq {

int fail(int code, const char* fmt, ...);
int check_lattice(const lqcd_lattice* lat);
int check_block(int nrhs, int layout, int prec);
int hip_status(hipError_t e, const char* what);

template <int MU, int SGN, int LAYOUT>
__device__ __forceinline__ void force_dir(cx<double> (&G)[3][3], const double2* __restrict__ g,
                                          const double2* __restrict__ psi, size_t x, size_t xp, size_t V, int nrhs) {
  const int cs = blk<LAYOUT>::cstride(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    // first term: h^-(g(x)) (x) h^-(psi(x+mu))^*
    {
      half_spinor<double> a = project<MU, -1>(load_spinor<double2, double>(g, blk<LAYOUT>::base(x, r, V, nrhs), cs));
      half_spinor<double> b =
          project<MU, -1>(load_spinor<double2, double>(psi, blk<LAYOUT>::base(xp, r, V, nrhs), cs));
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int k = 0; k < 3; ++k) G[i][k] = cjmadd(G[i][k], b.c[s][k], a.c[s][i]);
    }
    // second term: h^+(psi(x)) (x) h^+(g(x+mu))^*
    {
      half_spinor<double> a = project<MU, 1>(load_spinor<double2, double>(psi, blk<LAYOUT>::base(x, r, V, nrhs), cs));
      half_spinor<double> b = project<MU, 1>(load_spinor<double2, double>(g, blk<LAYOUT>::base(xp, r, V, nrhs), cs));
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int k = 0; k < 3; ++k) G[i][k] = cjmadd(G[i][k], b.c[s][k], a.c[s][i]);
    }
  }
}

// one thread per (site, mu)
template <int LAYOUT>
__global__ __launch_bounds__(256) void k_link_force(const double2* __restrict__ U, const double2* __restrict__ g,
                                                    const double2* __restrict__ psi, double2* __restrict__ out,
                                                    int n0, int n1, int n2, int n3, int nrhs, double coeff,
                                                    int project) {
  const size_t V = (size_t)n0 * n1 * n2 * n3;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * V) return;
  const int mu = (int)(t / V);
  const size_t x = t - (size_t)mu * V;
  size_t r = x;
  const int x3 = (int)(r % n3); r /= n3;
  const int x2 = (int)(r % n2); r /= n2;
  const int x1 = (int)(r % n1);
  const int x0 = (int)(r / n1);
  size_t xp;
  if (mu == 0) xp = x0 + 1 < n0 ? x + (size_t)n1 * n2 * n3 : x - (size_t)(n0 - 1) * n1 * n2 * n3;
  else if (mu == 1) xp = x1 + 1 < n1 ? x + (size_t)n2 * n3 : x - (size_t)(n1 - 1) * n2 * n3;
  else if (mu == 2) xp = x2 + 1 < n2 ? x + (size_t)n3 : x - (size_t)(n2 - 1) * n3;
  else xp = x3 + 1 < n3 ? x + 1 : x - (size_t)(n3 - 1);
  cx<double> G[3][3];
#pragma unroll
  for (int i = 0; i < 9; ++i) G[i / 3][i % 3] = {0.0, 0.0};
  if (mu == 0) force_dir<0, 1, LAYOUT>(G, g, psi, x, xp, V, nrhs);
  else if (mu == 1) force_dir<1, 1, LAYOUT>(G, g, psi, x, xp, V, nrhs);
  else if (mu == 2) force_dir<2, 1, LAYOUT>(G, g, psi, x, xp, V, nrhs);
  else force_dir<3, 1, LAYOUT>(G, g, psi, x, xp, V, nrhs);
  double2* o = out + ((size_t)mu * V + x) * 9;
  if (project) {
    // X = G U^dagger, F = (X - X^dag)/2 - tr(X - X^dag)/6 I
    const double2* u = U + ((size_t)mu * V + x) * 9;
    cx<double> X[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        cx<double> a = {0.0, 0.0};
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          const double2 ukl = u[k * 3 + l];
          a = cjmadd(a, cx<double>{ukl.x, ukl.y}, cx<double>{coeff * G[i][l].re, coeff * G[i][l].im});
        }
        X[i][k] = a;
      }
    double tr_im = (X[0][0].im + X[1][1].im + X[2][2].im) / 3.0;  // tr(X - X^dag)/6 = i Im tr X / 3
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double re = 0.5 * (X[i][k].re - X[k][i].re);
        double im = 0.5 * (X[i][k].im + X[k][i].im) - (i == k ? tr_im : 0.0);
        o[i * 3 + k] = make_double2(re, im);
      }
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) o[i] = make_double2(coeff * G[i / 3][i % 3].re, coeff * G[i / 3][i % 3].im);
  }
}

// out[rhs] = sum_sites sum_comp conj(a) b over a full-lattice block (any layout)
template <int LAYOUT>
__global__ __launch_bounds__(256) void k_block_dot(const double2* __restrict__ a, const double2* __restrict__ b,
                                                   size_t V, int nrhs, double2* __restrict__ out) {
  // one workgroup per rhs, fixed-order tree reduction
  const int r = blockIdx.x;
  const int cs = blk<LAYOUT>::cstride(nrhs);
  cx<double> acc = {0.0, 0.0};
  for (size_t s = threadIdx.x; s < V; s += blockDim.x) {
    const size_t base = blk<LAYOUT>::base(s, r, V, nrhs);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const double2 x = a[base + (size_t)c * cs], y = b[base + (size_t)c * cs];
      acc = cjmadd(acc, cx<double>{x.x, x.y}, cx<double>{y.x, y.y});
    }
  }
  __shared__ cx<double> sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = make_double2(sh[0].re, sh[0].im);
}

}  // namespace lq

using namespace lq;

extern "C" {

int link_force(const lqcd_lattice* lat, const void* U, const void* g, const void* psi, void* G, int nrhs, int layout,
               double coeff, int project, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, LQCD_F64))) return rc;
  if (!g || !psi || !G || (project && !U)) return fail(LQCD_ERR_ARG, "link_force: null array pointer");
  const size_t V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  const unsigned nb = (unsigned)((4 * V + 255) / 256);
  hipStream_t s = (hipStream_t)stream;
#define LF(L)                                                                                                    \
  hipLaunchKernelGGL((k_link_force<L>), dim3(nb), dim3(256), 0, s, (const double2*)U, (const double2*)g,         \
                     (const double2*)psi, (double2*)G, lat->dims[0], lat->dims[1], lat->dims[2], lat->dims[3],  \
                     nrhs, coeff, project)
  if (layout == LQCD_RHS_OUTER) LF(LQCD_RHS_OUTER);
  else if (layout == LQCD_LAYOUT1) LF(LQCD_LAYOUT1);
  else LF(LQCD_LAYOUT2);
#undef LF
  return hip_status(hipGetLastError(), "link_force launch");
}

int block_dot(const lqcd_lattice* lat, const void* a, const void* b, int nrhs, int layout, void* out,
              void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, LQCD_F64))) return rc;
  if (!a || !b || !out) return fail(LQCD_ERR_ARG, "block_dot: null array pointer");
  const size_t V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  hipStream_t s = (hipStream_t)stream;
#define BD(L)                                                                                                   \
  hipLaunchKernelGGL((k_block_dot<L>), dim3(nrhs), dim3(256), 0, s, (const double2*)a, (const double2*)b, V,   \
                     nrhs, (double2*)out)
  if (layout == LQCD_RHS_OUTER) BD(LQCD_RHS_OUTER);
  else if (layout == LQCD_LAYOUT1) BD(LQCD_LAYOUT1);
  else BD(LQCD_LAYOUT2);
#undef BD
  return hip_status(hipGetLastError(), "block_dot launch");
}

}  // extern "C"
