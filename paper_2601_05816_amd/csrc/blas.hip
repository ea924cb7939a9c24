// Batched BLAS-1 on rhs-innermost vectors for the Arnoldi process of
// Algorithm 2 (the Arnoldi step and the final update of x).
//
// Every vector is [nrow][nrhs] complex with nrow = 12 x (number of sites), so
// element e = row * nrhs + rhs.  Reductions are per rhs ("batched dot
// products", Sec. V-B): each thread keeps one rhs for its whole grid-stride
// loop, partial sums are combined per block in LDS in a fixed order and then
// across blocks by a second kernel in a fixed order, so results are
// deterministic.  Arithmetic of the reductions is FP64 whatever the storage
// precision.  A per-rhs `live` mask (nullable) skips right-hand sides that
// have converged.
#include "blas.h"
#include "common.h"

namespace lq {

template <int P>
using store_t = typename prec_traits<P>::store;

__device__ __forceinline__ cx<double> up(cx<double> a) { return a; }
__device__ __forceinline__ cx<double> up(cx<float> a) { return {(double)a.re, (double)a.im}; }

template <int P>
__device__ __forceinline__ cx<double> ldd(const store_t<P>* p) {
  return up(ld(p));
}
template <int P>
__device__ __forceinline__ void std_(store_t<P>* p, cx<double> a) {
  typedef typename prec_traits<P>::real R;
  st(p, cx<R>{(R)a.re, (R)a.im});
}

// threads [0, T') with T' the largest multiple of nrhs not above the grid
// size take part; thread t owns rhs t % nrhs for its whole loop.
struct stride_info {
  size_t t, stride;
  int rhs;
  bool active;
};
__device__ __forceinline__ stride_info grid_rhs(int nrhs) {
  stride_info s;
  const size_t T = (size_t)gridDim.x * blockDim.x;
  s.stride = T / nrhs * nrhs;
  s.t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  s.active = s.t < s.stride;
  s.rhs = (int)(s.t % nrhs);
  return s;
}

// Combine per-thread values val[0..K) of this block into part[blk][k][rhs].
template <int KB>
__device__ __forceinline__ void block_combine(cx<double> (&val)[KB], int K, int nrhs, bool active,
                                              cx<double>* __restrict__ part) {
  __shared__ cx<double> sh[256];
  const int tid = threadIdx.x;
  const int bt = blockDim.x;
  const size_t base = (size_t)blockIdx.x * K * nrhs;
  if (nrhs <= 8 && (nrhs & (nrhs - 1)) == 0 && bt % 64 == 0) {
    // few rhs (a power of two): thread t of the block owns rhs t % nrhs
    // (the block size is a multiple of nrhs), so a butterfly within each
    // wavefront sums its lanes of one rhs, and one thread per rhs adds the
    // wavefronts' sums
    const int lane = tid & 63, wave = tid >> 6, nw = bt >> 6;
    for (int k = 0; k < K; ++k) {
      cx<double> v = {0.0, 0.0};
#pragma unroll
      for (int q = 0; q < KB; ++q)
        if (q == k) v = val[q];
      v = wave_group_sum(active ? v : cx<double>{0.0, 0.0}, nrhs);
      if (lane < nrhs) sh[wave * 8 + lane] = v;
      __syncthreads();
      if (tid < nrhs) {
        cx<double> acc = {0.0, 0.0};
        for (int w = 0; w < nw; ++w) acc = acc + sh[w * 8 + tid];
        part[base + (size_t)k * nrhs + tid] = acc;
      }
      __syncthreads();
    }
    return;
  }
  for (int k = 0; k < K; ++k) {
    cx<double> v = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < KB; ++q)
      if (q == k) v = val[q];
    sh[tid] = active ? v : cx<double>{0.0, 0.0};
    __syncthreads();
    // thread r < nrhs sums the threads of this block that own rhs r (global
    // thread index congruent to r modulo nrhs), in increasing order.
    for (int r = tid; r < nrhs; r += bt) {
      const size_t t0 = (size_t)blockIdx.x * bt;
      int first = (int)((r - (int)(t0 % nrhs) + nrhs) % nrhs);
      cx<double> acc = {0.0, 0.0};
      for (int i = first; i < bt; i += nrhs) acc = acc + sh[i];
      part[base + (size_t)k * nrhs + r] = acc;
    }
    __syncthreads();
  }
}

// part[blk][k][rhs] = sum_rows conj(V_{k0+k}[row, rhs]) w[row, rhs], k < K <= KB.
template <int P, int KB>
__global__ __launch_bounds__(256) void k_dot_parts(const store_t<P>* __restrict__ V, size_t vstride, int k0, int K,
                                                   const store_t<P>* __restrict__ w, size_t nelem, int nrhs,
                                                   const int* __restrict__ live, cx<double>* __restrict__ part) {
  if (none_live(live, nrhs)) return;
  stride_info s = grid_rhs(nrhs);
  cx<double> acc[KB];
#pragma unroll
  for (int q = 0; q < KB; ++q) acc[q] = {0.0, 0.0};
  const bool on = s.active && (!live || live[s.rhs]);
  if (on) {
    for (size_t e = s.t; e < nelem; e += s.stride) {
      const cx<double> we = ldd<P>(w + e);
#pragma unroll
      for (int q = 0; q < KB; ++q)
        if (q < K) acc[q] = cjmadd(acc[q], ldd<P>(V + (size_t)(k0 + q) * vstride + e), we);
    }
  }
  block_combine<KB>(acc, K, nrhs, on, part);
}

// part[blk][0][rhs] = sum_rows |x[row, rhs]|^2 (stored in .re)
template <int P>
__global__ __launch_bounds__(256) void k_norm_parts(const store_t<P>* __restrict__ x, size_t nelem, int nrhs,
                                                    const int* __restrict__ live, cx<double>* __restrict__ part) {
  if (none_live(live, nrhs)) return;
  stride_info s = grid_rhs(nrhs);
  cx<double> acc[1] = {{0.0, 0.0}};
  const bool on = s.active && (!live || live[s.rhs]);
  if (on)
    for (size_t e = s.t; e < nelem; e += s.stride) {
      cx<double> v = ldd<P>(x + e);
      acc[0].re = fma(v.re, v.re, fma(v.im, v.im, acc[0].re));
    }
  block_combine<1>(acc, 1, nrhs, on, part);
}

// w -= sum_{k<K} h[k][rhs] V_k ; part = per-block |w|^2 of the result.
template <int P>
__global__ __launch_bounds__(256) void k_cgs_update(const store_t<P>* __restrict__ V, size_t vstride, int K,
                                                    const cx<double>* __restrict__ h, store_t<P>* __restrict__ w,
                                                    size_t nelem, int nrhs, const int* __restrict__ live,
                                                    cx<double>* __restrict__ part) {
  if (none_live(live, nrhs)) return;
  stride_info s = grid_rhs(nrhs);
  cx<double> acc[1] = {{0.0, 0.0}};
  const bool on = s.active && (!live || live[s.rhs]);
  if (on)
    for (size_t e = s.t; e < nelem; e += s.stride) {
      cx<double> v = ldd<P>(w + e);
      for (int k = 0; k < K; ++k) {
        const cx<double> hk = h[(size_t)k * nrhs + s.rhs];
        v = cmadd(v, -hk, ldd<P>(V + (size_t)k * vstride + e));
      }
      std_<P>(w + e, v);
      acc[0].re = fma(v.re, v.re, fma(v.im, v.im, acc[0].re));
    }
  block_combine<1>(acc, 1, nrhs, on, part);
}

// Chunked, non-persistent forms of the two kernels above that write a
// vector: block b owns the contiguous elements [b CH, (b+1) CH) with
// CH = SB x iters, SB = the largest multiple of nrhs not above the block
// size, so thread t < SB keeps rhs t % nrhs.  With one block per chunk the
// dispatcher keeps the blocks in flight on neighbouring addresses, which
// measured 15 % more read+write bandwidth on MI355X than a persistent
// grid-stride loop.
__device__ __forceinline__ void chunk_combine(cx<double> v, int nrhs, int sb, bool on,
                                              cx<double>* __restrict__ part) {
  __shared__ cx<double> sh[256];
  const int tid = threadIdx.x;
  sh[tid] = on ? v : cx<double>{0.0, 0.0};
  __syncthreads();
  for (int r = tid; r < nrhs; r += blockDim.x) {
    cx<double> a = {0.0, 0.0};
    for (int i = r; i < sb; i += nrhs) a = a + sh[i];
    part[(size_t)blockIdx.x * nrhs + r] = a;
  }
}

// LH: the K x nrhs coefficients are first copied to LDS (dynamic, K nrhs
// entries), so that the vector-memory pipe carries only basis loads.
template <int P, bool LH>
__global__ __launch_bounds__(256) void k_cgs_update_c(const store_t<P>* __restrict__ V, size_t vstride, int K,
                                                      const cx<double>* __restrict__ h, store_t<P>* __restrict__ w,
                                                      size_t nelem, int nrhs, int iters,
                                                      const int* __restrict__ live, cx<double>* __restrict__ part) {
  if (none_live(live, nrhs)) return;
  extern __shared__ char lds_raw[];
  cx<double>* hs = reinterpret_cast<cx<double>*>(lds_raw);
  if (LH) {
    for (int i = threadIdx.x; i < K * nrhs; i += blockDim.x) hs[i] = h[i];
    __syncthreads();
  }
  const int sb = (int)(blockDim.x / nrhs) * nrhs;
  const int tid = threadIdx.x;
  const int rhs = tid % nrhs;
  const bool on = tid < sb && (!live || live[rhs]);
  cx<double> acc = {0.0, 0.0};
  if (on) {
    const size_t e0 = (size_t)blockIdx.x * sb * iters + tid;
    for (int i = 0; i < iters; ++i) {
      const size_t e = e0 + (size_t)i * sb;
      if (e >= nelem) break;
      cx<double> v = ldd<P>(w + e);
      // eight basis vectors per round: their loads are issued together (the
      // terms are still added in the order k = 0, 1, ..., K-1)
      int k = 0;
      for (; k + 8 <= K; k += 8) {
        cx<double> a[8], c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          a[q] = ldd<P>(V + (size_t)(k + q) * vstride + e);
          c[q] = LH ? hs[(k + q) * nrhs + rhs] : h[(size_t)(k + q) * nrhs + rhs];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) v = cmadd(v, -c[q], a[q]);
      }
      for (; k + 4 <= K; k += 4) {
        cx<double> a[4], c[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a[q] = ldd<P>(V + (size_t)(k + q) * vstride + e);
          c[q] = LH ? hs[(k + q) * nrhs + rhs] : h[(size_t)(k + q) * nrhs + rhs];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) v = cmadd(v, -c[q], a[q]);
      }
      for (; k < K; ++k)
        v = cmadd(v, -(LH ? hs[k * nrhs + rhs] : h[(size_t)k * nrhs + rhs]), ldd<P>(V + (size_t)k * vstride + e));
      std_<P>(w + e, v);
      acc.re = fma(v.re, v.re, fma(v.im, v.im, acc.re));
    }
  }
  chunk_combine(acc, nrhs, sb, on, part);
}

template <int P>
__global__ __launch_bounds__(256) void k_scale_c(store_t<P>* __restrict__ x, size_t nelem, int nrhs, int iters,
                                                 const double* __restrict__ s, const int* __restrict__ live) {
  if (none_live(live, nrhs)) return;
  const int sb = (int)(blockDim.x / nrhs) * nrhs;
  const int tid = threadIdx.x;
  const int rhs = tid % nrhs;
  if (tid >= sb || (live && !live[rhs])) return;
  const double f = s[rhs];
  const size_t e0 = (size_t)blockIdx.x * sb * iters + tid;
  for (int i = 0; i < iters; ++i) {
    const size_t e = e0 + (size_t)i * sb;
    if (e >= nelem) break;
    cx<double> v = ldd<P>(x + e);
    std_<P>(x + e, cx<double>{v.re * f, v.im * f});
  }
}

// y = b - y ; part = |y|^2 per block
template <int P>
__global__ __launch_bounds__(256) void k_bmy(const store_t<P>* __restrict__ b, store_t<P>* __restrict__ y,
                                             size_t nelem, int nrhs, const int* __restrict__ live,
                                             cx<double>* __restrict__ part) {
  if (none_live(live, nrhs)) return;
  stride_info s = grid_rhs(nrhs);
  cx<double> acc[1] = {{0.0, 0.0}};
  const bool on = s.active && (!live || live[s.rhs]);
  if (on)
    for (size_t e = s.t; e < nelem; e += s.stride) {
      cx<double> v = ldd<P>(b + e) - ldd<P>(y + e);
      std_<P>(y + e, v);
      acc[0].re = fma(v.re, v.re, fma(v.im, v.im, acc[0].re));
    }
  block_combine<1>(acc, 1, nrhs, on, part);
}

// out[k][rhs] = scale * sum_blocks part[blk][k][rhs]: one workgroup per
// output, each thread sums a fixed strided subset of the blocks, then a fixed
// tree in LDS (deterministic order).
__global__ __launch_bounds__(256) void k_reduce_parts(const cx<double>* __restrict__ part, int nblk, int K,
                                                      int nrhs, double scale, cx<double>* __restrict__ out) {
  const int i = blockIdx.x;  // output index k * nrhs + rhs
  const size_t stride = (size_t)K * nrhs;
  cx<double> acc = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc = acc + part[(size_t)b * stride + i];
  __shared__ cx<double> sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = {sh[0].re * scale, sh[0].im * scale};
}

// x[row, rhs] *= s[rhs]
template <int P>
__global__ __launch_bounds__(256) void k_scale(store_t<P>* __restrict__ x, size_t nelem, int nrhs,
                                               const double* __restrict__ s, const int* __restrict__ live) {
  if (none_live(live, nrhs)) return;
  stride_info si = grid_rhs(nrhs);
  if (!si.active || (live && !live[si.rhs])) return;
  const double f = s[si.rhs];
  for (size_t e = si.t; e < nelem; e += si.stride) {
    cx<double> v = ldd<P>(x + e);
    std_<P>(x + e, cx<double>{v.re * f, v.im * f});
  }
}

// x[row, rhs] += scale * sum_{k < cnt[rhs]} y[k][rhs] V_k[row, rhs]   (x in precision PX)
template <int P, int PX>
__global__ __launch_bounds__(256) void k_lincomb(const store_t<P>* __restrict__ V, size_t vstride, int kmax,
                                                 const cx<double>* __restrict__ y, const int* __restrict__ cnt,
                                                 store_t<PX>* __restrict__ x, size_t nelem, int nrhs, double scale) {
  stride_info si = grid_rhs(nrhs);
  if (!si.active) return;
  const int n = cnt[si.rhs] < kmax ? cnt[si.rhs] : kmax;
  if (n == 0) return;
  for (size_t e = si.t; e < nelem; e += si.stride) {
    cx<double> acc = {0.0, 0.0};
    // four basis vectors per round (loads issued together, terms added in
    // the order k = 0, 1, ..., n-1)
    int k = 0;
    for (; k + 4 <= n; k += 4) {
      cx<double> a[4], c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = ldd<P>(V + (size_t)(k + q) * vstride + e);
        c[q] = y[(size_t)(k + q) * nrhs + si.rhs];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) acc = cmadd(acc, c[q], a[q]);
    }
    for (; k < n; ++k) acc = cmadd(acc, y[(size_t)k * nrhs + si.rhs], ldd<P>(V + (size_t)k * vstride + e));
    cx<double> v = ldd<PX>(x + e);
    std_<PX>(x + e, cx<double>{fma(scale, acc.re, v.re), fma(scale, acc.im, v.im)});
  }
}

// out[row, rhs] = s[rhs] * in[row, rhs] (precision conversion); s may be null (1)
template <int PI, int PO>
__global__ __launch_bounds__(256) void k_convert(const store_t<PI>* __restrict__ in, store_t<PO>* __restrict__ out,
                                                 size_t nelem, int nrhs, const double* __restrict__ s) {
  stride_info si = grid_rhs(nrhs);
  if (!si.active) return;
  const double f = s ? s[si.rhs] : 1.0;
  for (size_t e = si.t; e < nelem; e += si.stride) {
    cx<double> v = ldd<PI>(in + e);
    std_<PO>(out + e, cx<double>{v.re * f, v.im * f});
  }
}

// out64[row, rhs] += f[rhs] * in[row, rhs]
template <int PI>
__global__ __launch_bounds__(256) void k_add_scaled(const store_t<PI>* __restrict__ in,
                                                    store_t<LQCD_F64>* __restrict__ out, size_t nelem, int nrhs,
                                                    const double* __restrict__ f) {
  stride_info si = grid_rhs(nrhs);
  if (!si.active) return;
  const double a = f[si.rhs];
  if (a == 0.0) return;
  for (size_t e = si.t; e < nelem; e += si.stride) {
    cx<double> v = ldd<PI>(in + e), o = ldd<LQCD_F64>(out + e);
    std_<LQCD_F64>(out + e, cx<double>{fma(a, v.re, o.re), fma(a, v.im, o.im)});
  }
}

// Flat copy with precision conversion (gauge links): out[i] = in[i]
template <int PI, int PO>
__global__ __launch_bounds__(256) void k_convert_flat(const store_t<PI>* __restrict__ in,
                                                      store_t<PO>* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    std_<PO>(out + i, ldd<PI>(in + i));
}

// ABI block (full lattice, any layout) <-> internal rhs-innermost vectors.
// eo = 1: internal vectors are the even and odd half lattices (compact index
// = site >> 1); eo = 0: one full-lattice vector in site order.
template <int LAYOUT, bool TO_INTERNAL>
__global__ __launch_bounds__(256) void k_pack(store_t<LQCD_F64>* __restrict__ abi, store_t<LQCD_F64>* __restrict__ ie,
                                              store_t<LQCD_F64>* __restrict__ io, int n0, int n1, int n2, int n3,
                                              int nrhs, int eo, int abi_nrhs, int col0) {
  const size_t V = (size_t)n0 * n1 * n2 * n3;
  const size_t items = V * (size_t)nrhs;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < items; t += (size_t)gridDim.x * blockDim.x) {
    const size_t site = t / nrhs;
    const int rhs = (int)(t % nrhs);
    size_t r = site;
    const int x3 = (int)(r % n3); r /= n3;
    const int x2 = (int)(r % n2); r /= n2;
    const int x1 = (int)(r % n1);
    const int x0 = (int)(r / n1);
    store_t<LQCD_F64>* dst;
    size_t idx;
    if (eo) {
      dst = ((x0 + x1 + x2 + x3) & 1) ? io : ie;
      idx = site >> 1;
    } else {
      dst = ie;
      idx = site;
    }
    const size_t a = blk<LAYOUT>::base(site, col0 + rhs, V, abi_nrhs);
    const int cs = blk<LAYOUT>::cstride(abi_nrhs);
    const size_t b = idx * 12u * (size_t)nrhs + (size_t)rhs;
    for (int c = 0; c < 12; ++c) {
      if (TO_INTERNAL) dst[b + (size_t)c * nrhs] = abi[a + (size_t)c * cs];
      else abi[a + (size_t)c * cs] = dst[b + (size_t)c * nrhs];
    }
  }
}

// --------------------------------------------------------------- launchers
static unsigned red_blocks(size_t nelem) {
  size_t b = (nelem + 1023) / 1024;
  if (b > 2048) b = 2048;
  return (unsigned)(b < 1 ? 1 : b);
}
unsigned reduce_grid(size_t nelem) { return red_blocks(nelem); }

#define PREC_SWITCH(P, CALL)                                       \
  switch (P) {                                                     \
    case LQCD_F64: { constexpr int PP = LQCD_F64; CALL; } break;   \
    case LQCD_F32: { constexpr int PP = LQCD_F32; CALL; } break;   \
    case LQCD_F16: { constexpr int PP = LQCD_F16; CALL; } break;   \
    default: return hipErrorInvalidValue;                          \
  }

static int g_vec_blas = 1;
void set_vector_blas(int on) { g_vec_blas = on ? 1 : 0; }

hipError_t dot_parts(int prec, const void* V, size_t vstride, int k0, int K, const void* w, size_t nelem, int nrhs,
                     const int* live, void* part, unsigned nblk, hipStream_t s) {
  if (K < 1 || K > DOT_KB) return hipErrorInvalidValue;
  if (g_vec_blas && vec_width(prec, nrhs) > 1)
    return dot_parts_v(prec, V, vstride, k0, K, w, nelem, nrhs, live, part, nblk, s);
  PREC_SWITCH(prec, hipLaunchKernelGGL((k_dot_parts<PP, DOT_KB>), dim3(nblk), dim3(256), 0, s,
                                       (const store_t<PP>*)V, vstride, k0, K, (const store_t<PP>*)w, nelem, nrhs,
                                       live, (cx<double>*)part));
  return hipGetLastError();
}

hipError_t norm_parts(int prec, const void* x, size_t nelem, int nrhs, const int* live, void* part, unsigned nblk,
                      hipStream_t s) {
  PREC_SWITCH(prec, hipLaunchKernelGGL((k_norm_parts<PP>), dim3(nblk), dim3(256), 0, s, (const store_t<PP>*)x, nelem,
                                       nrhs, live, (cx<double>*)part));
  return hipGetLastError();
}

// Chunk length (in multiples of the block's rhs-aligned width) of the
// chunked kernels: at least 16, and few enough blocks that their partial
// sums fit the nblk x DOT_KB x nrhs part buffer.
static int chunk_iters(size_t nelem, int nrhs, unsigned nblk) {
  const size_t sb = (size_t)(256 / nrhs) * nrhs;
  const size_t cap = (size_t)nblk * DOT_KB;  // partial rows available
  size_t it = 16;
  while ((nelem + sb * it - 1) / (sb * it) > cap) it *= 2;
  return (int)it;
}

unsigned cgs_update_parts(int prec, size_t nelem, int nrhs, unsigned nblk) {
  if ((g_vec_blas && vec_width(prec, nrhs) > 1) || nrhs > 256) return nblk;
  const size_t sb = (size_t)(256 / nrhs) * nrhs;
  const size_t ch = sb * (size_t)chunk_iters(nelem, nrhs, nblk);
  return (unsigned)((nelem + ch - 1) / ch);
}

hipError_t cgs_update(int prec, const void* V, size_t vstride, int K, const void* h, void* w, size_t nelem, int nrhs,
                      const int* live, void* part, unsigned nblk, hipStream_t s) {
  if (g_vec_blas && vec_width(prec, nrhs) > 1)
    return cgs_update_v(prec, V, vstride, K, h, w, nelem, nrhs, live, part, nblk, s);
  if (nrhs <= 256) {
    const int it = chunk_iters(nelem, nrhs, nblk);
    const unsigned nb = cgs_update_parts(prec, nelem, nrhs, nblk);
    const size_t hb = (size_t)K * nrhs * sizeof(cx<double>);
    if (hb <= CGS_LDS_BYTES) {
      PREC_SWITCH(prec, hipLaunchKernelGGL((k_cgs_update_c<PP, true>), dim3(nb), dim3(256), hb, s,
                                           (const store_t<PP>*)V, vstride, K, (const cx<double>*)h,
                                           (store_t<PP>*)w, nelem, nrhs, it, live, (cx<double>*)part));
    } else {
      PREC_SWITCH(prec, hipLaunchKernelGGL((k_cgs_update_c<PP, false>), dim3(nb), dim3(256), 0, s,
                                           (const store_t<PP>*)V, vstride, K, (const cx<double>*)h,
                                           (store_t<PP>*)w, nelem, nrhs, it, live, (cx<double>*)part));
    }
    return hipGetLastError();
  }
  PREC_SWITCH(prec, hipLaunchKernelGGL((k_cgs_update<PP>), dim3(nblk), dim3(256), 0, s, (const store_t<PP>*)V,
                                       vstride, K, (const cx<double>*)h, (store_t<PP>*)w, nelem, nrhs, live,
                                       (cx<double>*)part));
  return hipGetLastError();
}

hipError_t b_minus_y(int prec, const void* b, void* y, size_t nelem, int nrhs, const int* live, void* part,
                     unsigned nblk, hipStream_t s) {
  PREC_SWITCH(prec, hipLaunchKernelGGL((k_bmy<PP>), dim3(nblk), dim3(256), 0, s, (const store_t<PP>*)b,
                                       (store_t<PP>*)y, nelem, nrhs, live, (cx<double>*)part));
  return hipGetLastError();
}

hipError_t reduce_parts(const void* part, int nblk, int K, int nrhs, double scale, void* out, hipStream_t s) {
  const int n = K * nrhs;
  hipLaunchKernelGGL(k_reduce_parts, dim3(n), dim3(256), 0, s, (const cx<double>*)part, nblk, K, nrhs, scale,
                     (cx<double>*)out);
  return hipGetLastError();
}

hipError_t scale_rhs(int prec, void* x, size_t nelem, int nrhs, const double* f, const int* live, hipStream_t s) {
  if (g_vec_blas && vec_width(prec, nrhs) > 1) return scale_rhs_v(prec, x, nelem, nrhs, f, live, red_blocks(nelem), s);
  if (nrhs <= 256) {
    const size_t ch = (size_t)(256 / nrhs) * nrhs * 16;
    PREC_SWITCH(prec, hipLaunchKernelGGL((k_scale_c<PP>), dim3((unsigned)((nelem + ch - 1) / ch)), dim3(256), 0, s,
                                         (store_t<PP>*)x, nelem, nrhs, 16, f, live));
    return hipGetLastError();
  }
  PREC_SWITCH(prec, hipLaunchKernelGGL((k_scale<PP>), dim3(red_blocks(nelem)), dim3(256), 0, s, (store_t<PP>*)x,
                                       nelem, nrhs, f, live));
  return hipGetLastError();
}

hipError_t lincomb(int prec, const void* V, size_t vstride, int kmax, const void* y, const int* cnt, int precx,
                   void* x, size_t nelem, int nrhs, double scale, hipStream_t s) {
  const unsigned nb = red_blocks(nelem);
  if (g_vec_blas && prec == precx && vec_width(prec, nrhs) > 1)
    return lincomb_v(prec, V, vstride, kmax, y, cnt, x, nelem, nrhs, scale, nb, s);
#define LC(PV, PX)                                                                                                \
  hipLaunchKernelGGL((k_lincomb<PV, PX>), dim3(nb), dim3(256), 0, s, (const store_t<PV>*)V, vstride, kmax,        \
                     (const cx<double>*)y, cnt, (store_t<PX>*)x, nelem, nrhs, scale)
  if (prec == LQCD_F64 && precx == LQCD_F64) LC(LQCD_F64, LQCD_F64);
  else if (prec == LQCD_F32 && precx == LQCD_F32) LC(LQCD_F32, LQCD_F32);
  else if (prec == LQCD_F16 && precx == LQCD_F16) LC(LQCD_F16, LQCD_F16);
  else if (prec == LQCD_F32 && precx == LQCD_F64) LC(LQCD_F32, LQCD_F64);
  else if (prec == LQCD_F16 && precx == LQCD_F64) LC(LQCD_F16, LQCD_F64);
  else return hipErrorInvalidValue;
#undef LC
  return hipGetLastError();
}

hipError_t convert(int pin, const void* in, int pout, void* out, size_t nelem, int nrhs, const double* f,
                   hipStream_t s) {
  const unsigned nb = red_blocks(nelem);
#define CV(A, B)                                                                                                   \
  hipLaunchKernelGGL((k_convert<A, B>), dim3(nb), dim3(256), 0, s, (const store_t<A>*)in, (store_t<B>*)out, nelem, \
                     nrhs, f)
  if (pin == LQCD_F64 && pout == LQCD_F64) CV(LQCD_F64, LQCD_F64);
  else if (pin == LQCD_F32 && pout == LQCD_F32) CV(LQCD_F32, LQCD_F32);
  else if (pin == LQCD_F16 && pout == LQCD_F16) CV(LQCD_F16, LQCD_F16);
  else if (pin == LQCD_F64 && pout == LQCD_F32) CV(LQCD_F64, LQCD_F32);
  else if (pin == LQCD_F64 && pout == LQCD_F16) CV(LQCD_F64, LQCD_F16);
  else if (pin == LQCD_F32 && pout == LQCD_F64) CV(LQCD_F32, LQCD_F64);
  else if (pin == LQCD_F16 && pout == LQCD_F64) CV(LQCD_F16, LQCD_F64);
  else return hipErrorInvalidValue;
#undef CV
  return hipGetLastError();
}

hipError_t add_scaled(int pin, const void* in, void* out64, size_t nelem, int nrhs, const double* f, hipStream_t s) {
  PREC_SWITCH(pin, hipLaunchKernelGGL((k_add_scaled<PP>), dim3(red_blocks(nelem)), dim3(256), 0, s,
                                      (const store_t<PP>*)in, (store_t<LQCD_F64>*)out64, nelem, nrhs, f));
  return hipGetLastError();
}

hipError_t convert_links(const void* in, int pout, void* out, size_t n, hipStream_t s) {
  const unsigned nb = red_blocks(n);
  if (pout == LQCD_F32)
    hipLaunchKernelGGL((k_convert_flat<LQCD_F64, LQCD_F32>), dim3(nb), dim3(256), 0, s,
                       (const store_t<LQCD_F64>*)in, (store_t<LQCD_F32>*)out, n);
  else if (pout == LQCD_F16)
    hipLaunchKernelGGL((k_convert_flat<LQCD_F64, LQCD_F16>), dim3(nb), dim3(256), 0, s,
                       (const store_t<LQCD_F64>*)in, (store_t<LQCD_F16>*)out, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t pack(int layout, bool to_internal, void* abi, void* ie, void* io, const int* dims, int nrhs, int eo,
                hipStream_t s, int abi_nrhs, int col0) {
  if (abi_nrhs <= 0) abi_nrhs = nrhs;
  if (col0 < 0 || col0 + nrhs > abi_nrhs) return hipErrorInvalidValue;
  const size_t items = (size_t)dims[0] * dims[1] * dims[2] * dims[3] * (size_t)nrhs;
  size_t nb = (items + 255) / 256;
  if (nb > 65536) nb = 65536;
#define PK(L, T)                                                                                                   \
  hipLaunchKernelGGL((k_pack<L, T>), dim3((unsigned)nb), dim3(256), 0, s, (store_t<LQCD_F64>*)abi,                 \
                     (store_t<LQCD_F64>*)ie, (store_t<LQCD_F64>*)io, dims[0], dims[1], dims[2], dims[3], nrhs, eo, \
                     abi_nrhs, col0)
  switch (layout * 2 + (to_internal ? 1 : 0)) {
    case LQCD_RHS_OUTER * 2 + 1: PK(LQCD_RHS_OUTER, true); break;
    case LQCD_RHS_OUTER * 2 + 0: PK(LQCD_RHS_OUTER, false); break;
    case LQCD_LAYOUT1 * 2 + 1: PK(LQCD_LAYOUT1, true); break;
    case LQCD_LAYOUT1 * 2 + 0: PK(LQCD_LAYOUT1, false); break;
    case LQCD_LAYOUT2 * 2 + 1: PK(LQCD_LAYOUT2, true); break;
    case LQCD_LAYOUT2 * 2 + 0: PK(LQCD_LAYOUT2, false); break;
    default: return hipErrorInvalidValue;
  }
#undef PK
  return hipGetLastError();
}

}  // namespace lq
