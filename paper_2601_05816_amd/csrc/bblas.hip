// Tall-skinny block kernels of block GMRES on rhs-innermost FP64 blocks
// [nrows][b] (b <= 16 right-hand sides per row): the block Gram products
// H_k = V_k^H W and the block combinations out = alpha Y + beta sum_k V_k C_k
// with b x b coefficient blocks C_k.  These are dense contractions (K =
// nrows for the Gram products, K = b for the combinations), so they run on
// the FP64 matrix cores: v_mfma_f64_16x16x4f64 with a complex product split
// into three real products (Gauss: for (a + ib)(c + id), k1 = c (a + b),
// k2 = a (d - c), k3 = b (c + d), real part k1 - k3, imaginary part k1 + k2),
// which at b = 16 rhs keeps the matrix-core time per byte below the HBM time.  Operand layouts of that instruction (lane l of a
// wavefront): A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, and D[i][j]
// in lane j + 16 (i % 4), element i / 4 (checked on the device).
#include <hip/hip_runtime.h>

#include "blas.h"
#include "common.h"

namespace lq {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef cx<double> zd;

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// parts[p][k][i b + j] = sum over the rows of workgroup p of
// conj(V_k[row][i]) W[row][j] for k < K.  A wavefront takes four rows per
// step: lane l loads element (row0 + l / 16, l % 16) of V_k and of W, i.e.
// the A operand V_k^T (i = column of V, k = row) and the B operand W; the four
// wavefronts' sums are added in LDS (fixed order).  K is a template parameter
// so that the K + 1 loads of a step are unconditional and issue together;
// SELF (K = 1, V = W) forms W^H W from one load.  Lanes past the last row or
// column load element 0 (which exists) and zero it.
template <int K, bool SELF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_bgram(const zd* V, size_t vstride, const zd* W, size_t nrows, int b,
                                               size_t rows_per_blk, zd* __restrict__ parts) {
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = l & 15, kq = l >> 4;
  const size_t r0 = (size_t)blockIdx.x * rows_per_blk;
  const size_t r1 = r0 + rows_per_blk < nrows ? r0 + rows_per_blk : nrows;
  d4 p1[K], p2[K], p3[K];
#pragma unroll
  for (int k = 0; k < K; ++k) p1[k] = p2[k] = p3[k] = d4{0.0, 0.0, 0.0, 0.0};
  for (size_t q = r0 + 4 * (size_t)wave; q < r1; q += 16) {
    const size_t row = q + kq;
    const bool ok = row < r1 && col < b;
    const size_t at = ok ? row * b + col : 0;
    zd w = W[at];
    zd v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = SELF ? w : V[(size_t)k * vstride + at];
    if (!ok) {
      w = zd{0.0, 0.0};
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = zd{0.0, 0.0};
    }
    // conj(v) w: a = v.re, b = -v.im, c = w.re, d = w.im
    const double wd = w.im - w.re, ws = w.re + w.im;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      p1[k] = mfma(v[k].re - v[k].im, w.re, p1[k]);
      p2[k] = mfma(v[k].re, wd, p2[k]);
      p3[k] = mfma(-v[k].im, ws, p3[k]);
    }
  }
  __shared__ d4 red[3][2][64];
  const size_t bb = (size_t)b * b;
  zd* out = parts + (size_t)blockIdx.x * K * bb;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    d4 hr = p1[k] - p3[k], hi = p1[k] + p2[k];
    if (wave) {
      red[wave - 1][0][l] = hr;
      red[wave - 1][1][l] = hi;
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        hr += red[u][0][l];
        hi += red[u][1][l];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = kq + 4 * v;
        if (i < b && col < b) out[(size_t)k * bb + (size_t)i * b + col] = zd{hr[v], hi[v]};
      }
    }
    __syncthreads();
  }
}

// out[o] = sum_p parts[p][o], o < n, p < np: 64 consecutive outputs per
// workgroup (coalesced rows of the partial sums), wavefront u sums the
// partials p = u mod 4 in increasing order, then the four sums are added in
// LDS (a fixed order, so the result is deterministic).
__global__ __launch_bounds__(256) void k_bgram_reduce(const zd* __restrict__ parts, int np, int n,
                                                      zd* __restrict__ out) {
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + l;
  zd acc = {0.0, 0.0};
  if (o < n) {
#pragma unroll 8
    for (int p = wave; p < np; p += 4) {
      const zd v = parts[(size_t)p * n + o];
      acc.re += v.re;
      acc.im += v.im;
    }
  }
  __shared__ zd sh[4][64];
  sh[wave][l] = acc;
  __syncthreads();
  if (wave == 0 && o < n) {
    zd t = sh[0][l];
    for (int u = 1; u < 4; ++u) {
      t.re += sh[u][l].re;
      t.im += sh[u][l].im;
    }
    out[o] = t;
  }
}

// out[row][c] = alpha Y[row][c] + beta sum_k sum_r V_k[row][r] C_k[r][c]
// (Y is not read when alpha = 0; out may alias Y or V_0: every wavefront
// reads its 16-row tile completely before it writes it).  A wavefront works
// on 16 rows: lane l loads the A operand (i = row, k = r) straight from V_k,
// element (row0 + l % 16, 4 s + l / 16) for the four steps s (independent
// loads, no staging); the coefficients are the B operand (k = r, j = c),
// held in LDS.
template <int KB>
__global__ __launch_bounds__(256) void k_bgemm(zd* out, const zd* Y, double alpha, double beta, const zd* V,
                                               size_t vstride, int K, const zd* __restrict__ C, size_t nrows, int b) {
  __shared__ zd cl[KB][16][16];  // coefficient blocks, zero-padded to 16 x 16
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = l & 15, kq = l >> 4;
  const size_t bb = (size_t)b * b;
  for (int e = threadIdx.x; e < KB * 256; e += blockDim.x) {
    const int k = e >> 8, r = (e >> 4) & 15, c = e & 15;
    cl[k][r][c] = (k < K && r < b && c < b) ? C[(size_t)k * bb + (size_t)r * b + c] : zd{0.0, 0.0};
  }
  __syncthreads();
  const size_t ntiles = (nrows + 15) / 16;
  for (size_t t = (size_t)blockIdx.x * 4 + wave; t < ntiles; t += (size_t)gridDim.x * 4) {
    const size_t t0 = t * 16;
    const bool rok = t0 + col < nrows;  // this lane's A row exists
    d4 k1 = {0.0, 0.0, 0.0, 0.0}, k2 = k1, k3 = k1;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      if (k < K) {
        const zd* src = V + (size_t)k * vstride + (t0 + col) * b;
        zd a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int r = 4 * s + kq;
          a[s] = (rok && r < b) ? src[r] : zd{0.0, 0.0};
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          if (4 * s < b) {  // uniform: skip steps past the last coefficient row
            const zd c = cl[k][4 * s + kq][col];
            // a = A.re, b = A.im, c = C.re, d = C.im
            k1 = mfma(a[s].re + a[s].im, c.re, k1);
            k2 = mfma(a[s].re, c.im - c.re, k2);
            k3 = mfma(a[s].im, c.re + c.im, k3);
          }
        }
      }
    }
    const d4 dr = k1 - k3, di = k1 + k2;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const size_t row = t0 + kq + 4 * v;
      if (row < nrows && col < b) {
        const size_t e = row * b + col;
        zd o = {beta * dr[v], beta * di[v]};
        if (alpha != 0.0) {
          const zd y = Y[e];
          o.re += alpha * y.re;
          o.im += alpha * y.im;
        }
        out[e] = o;
      }
    }
  }
}

unsigned bgram_blocks(size_t nrows) {
  size_t n = (nrows + 255) / 256;
  if (n > 1024) n = 1024;
  return n < 1 ? 1u : (unsigned)n;
}

hipError_t bgram_parts(const void* V, size_t vstride, int K, const void* W, size_t nrows, int b, void* parts,
                       unsigned nblk, hipStream_t s) {
  if (b < 1 || b > 16 || K < 1 || K > BG_KB) return hipErrorInvalidValue;
  size_t rpb = (nrows + nblk - 1) / nblk;
  rpb = (rpb + 15) & ~(size_t)15;
  const zd* Vz = (const zd*)V;
  const zd* Wz = (const zd*)W;
  zd* P = (zd*)parts;
  switch (K) {
    case 1:
      if (V == W)
        hipLaunchKernelGGL((k_bgram<1, true>), dim3(nblk), dim3(256), 0, s, Vz, vstride, Wz, nrows, b, rpb, P);
      else
        hipLaunchKernelGGL((k_bgram<1, false>), dim3(nblk), dim3(256), 0, s, Vz, vstride, Wz, nrows, b, rpb, P);
      break;
    case 2:
      hipLaunchKernelGGL((k_bgram<2, false>), dim3(nblk), dim3(256), 0, s, Vz, vstride, Wz, nrows, b, rpb, P);
      break;
#define LQ_BGRAM_CASE(KK)                                                                                  \
  case KK:                                                                                                 \
    hipLaunchKernelGGL((k_bgram<KK, false>), dim3(nblk), dim3(256), 0, s, Vz, vstride, Wz, nrows, b, rpb, P); \
    break;
    LQ_BGRAM_CASE(3) LQ_BGRAM_CASE(4) LQ_BGRAM_CASE(5) LQ_BGRAM_CASE(6) LQ_BGRAM_CASE(7)
#undef LQ_BGRAM_CASE
    default:
      hipLaunchKernelGGL((k_bgram<8, false>), dim3(nblk), dim3(256), 0, s, Vz, vstride, Wz, nrows, b, rpb, P);
      break;
  }
  return hipGetLastError();
}

hipError_t bgram_reduce(const void* parts, unsigned nblk, int K, int b, void* out, hipStream_t s) {
  const int n = K * b * b;
  hipLaunchKernelGGL(k_bgram_reduce, dim3((n + 63) / 64), dim3(256), 0, s, (const zd*)parts, (int)nblk, n, (zd*)out);
  return hipGetLastError();
}

hipError_t bgemm(void* out, const void* Y, double alpha, double beta, const void* V, size_t vstride, int K,
                 const void* C, size_t nrows, int b, hipStream_t s) {
  if (b < 1 || b > 16 || K < 0 || K > BM_KB) return hipErrorInvalidValue;
  const size_t ntiles = (nrows + 15) / 16;
  size_t grid = (ntiles + 3) / 4;
  if (grid > 2048) grid = 2048;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_bgemm<BM_KB>), dim3((unsigned)grid), dim3(256), 0, s, (zd*)out, (const zd*)Y, alpha, beta,
                     (const zd*)V, vstride, K, (const zd*)C, nrows, b);
  return hipGetLastError();
}

}  // namespace lq
