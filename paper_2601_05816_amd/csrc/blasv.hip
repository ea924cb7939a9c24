// Vector-width variants of the batched BLAS-1 kernels for the low-precision
// Krylov bases of the refinement modes: each lane moves VW consecutive rhs of
// one row with one 16-byte access (VW = 2 for FP32, 4 for FP16 storage),
// instead of one 8- or 4-byte access per rhs.  Needs nrhs % VW == 0 (the
// launchers in blas.hip fall back to the scalar kernels otherwise).  Partial
// sums per lane are FP64 for VW = 2 and FP32 for VW = 4; block and
// cross-block sums are FP64 in a fixed order, as in blas.hip.
#include "blas.h"
#include "common.h"

namespace lq {


template <int P>
struct vio;
template <>
struct vio<LQCD_F32> {
  enum { VW = 2 };
  typedef double acc_t;
  typedef float2 store;
  typedef f4v_t raw;  // one 16-byte access as loaded
  typedef double ct;  // dot products: FP64 products of FP32 values (exact)
  __device__ static __forceinline__ raw load_raw(const float2* p) { return *(const f4v_t*)p; }
  __device__ static __forceinline__ void unpack(const raw& v, cx<double> (&o)[2]) {
    o[0] = {v.x, v.y};
    o[1] = {v.z, v.w};
  }
  __device__ static __forceinline__ void load(const float2* p, cx<double> (&o)[2]) { unpack(load_raw(p), o); }
  __device__ static __forceinline__ void save(float2* p, const cx<double> (&o)[2]) {
    f4v_t v = {(float)o[0].re, (float)o[0].im, (float)o[1].re, (float)o[1].im};
    *(f4v_t*)p = v;
  }
};
template <>
struct vio<LQCD_F16> {
  enum { VW = 4 };
  typedef float acc_t;
  typedef h2_t store;
  typedef h8v_t raw;  // one 16-byte access as loaded
  typedef float ct;   // dot products: FP32 products of FP16 values (exact: 11-bit significands)
  __device__ static __forceinline__ raw load_raw(const h2_t* p) { return *(const h8v_t*)p; }
  __device__ static __forceinline__ void unpack(const raw& v, cx<double> (&o)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = {(double)(float)v[2 * i], (double)(float)v[2 * i + 1]};
  }
  __device__ static __forceinline__ void unpack(const raw& v, cx<float> (&o)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = {(float)v[2 * i], (float)v[2 * i + 1]};
  }
  __device__ static __forceinline__ void load(const h2_t* p, cx<double> (&o)[4]) { unpack(load_raw(p), o); }
  __device__ static __forceinline__ void save(h2_t* p, const cx<double> (&o)[4]) {
    h8v_t v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[2 * i] = (_Float16)(float)o[i].re;
      v[2 * i + 1] = (_Float16)(float)o[i].im;
    }
    *(h8v_t*)p = v;
  }
};

// Thread t owns rhs group gr = t % G (rhs gr*VW .. gr*VW+VW-1) of rows
// row0, row0 + rstride, ... with G = nrhs / VW.
struct vsched {
  size_t row0, rstride;
  int gr;
  bool active;
};
__device__ __forceinline__ vsched vgrid(int G) {
  vsched s;
  const size_t T = (size_t)gridDim.x * blockDim.x;
  const size_t Tp = T / G * G;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  s.active = t < Tp;
  s.gr = (int)(t % G);
  s.row0 = t / G;
  s.rstride = Tp / G;
  return s;
}

// part[blk][k][rhs] from per-thread values val[k][v] of rhs gr*VW + v
template <int KB, int VW, typename A>
__device__ __forceinline__ void vblock_combine(A (&re)[KB][VW], A (&im)[KB][VW], int K, int nrhs, bool active,
                                               cx<double>* __restrict__ part) {
  __shared__ cx<double> sh[256];
  const int tid = threadIdx.x, bt = blockDim.x;
  const int G = nrhs / VW;
  const size_t base = (size_t)blockIdx.x * K * nrhs;
  const size_t t0 = (size_t)blockIdx.x * bt;
  if (G <= 8 && (G & (G - 1)) == 0 && bt % 64 == 0) {
    // few rhs groups (a power of two): thread t owns group t % G, so a
    // butterfly within each wavefront sums its lanes of one group, and one
    // thread per group adds the wavefronts' sums
    const int lane = tid & 63, wave = tid >> 6, nw = bt >> 6;
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        cx<double> x = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < KB; ++q)
          if (q == k) x = {(double)re[q][v], (double)im[q][v]};
        x = wave_group_sum(active ? x : cx<double>{0.0, 0.0}, G);
        if (lane < G) sh[wave * 8 + lane] = x;
        __syncthreads();
        if (tid < G) {
          cx<double> a = {0.0, 0.0};
          for (int w = 0; w < nw; ++w) a = a + sh[w * 8 + tid];
          part[base + (size_t)k * nrhs + (size_t)tid * VW + v] = a;
        }
        __syncthreads();
      }
    }
    return;
  }
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      cx<double> x = {0.0, 0.0};
#pragma unroll
      for (int q = 0; q < KB; ++q)
        if (q == k) x = {(double)re[q][v], (double)im[q][v]};
      sh[tid] = active ? x : cx<double>{0.0, 0.0};
      __syncthreads();
      for (int g = tid; g < G; g += bt) {
        const int first = (int)((g - (int)(t0 % G) + G) % G);
        cx<double> a = {0.0, 0.0};
        for (int i = first; i < bt; i += G) a = a + sh[i];
        part[base + (size_t)k * nrhs + (size_t)g * VW + v] = a;
      }
      __syncthreads();
    }
  }
}

// K (the number of basis vectors, 1..DOT_KB) is a template parameter, so
// that the K + 1 loads of a row are unconditional and issue together.
template <int P, int K>
__global__ __launch_bounds__(256) void k_dot_parts_v(const typename vio<P>::store* __restrict__ V, size_t vstride,
                                                     int k0, const typename vio<P>::store* __restrict__ w,
                                                     size_t nrow, int nrhs, const int* __restrict__ live,
                                                     cx<double>* __restrict__ part) {
  constexpr int KB = K;
  if (none_live(live, nrhs)) return;
  constexpr int VW = vio<P>::VW;
  typedef typename vio<P>::acc_t A;
  const int G = nrhs / VW;
  vsched s = vgrid(G);
  A re[KB][VW], im[KB][VW];
#pragma unroll
  for (int q = 0; q < KB; ++q)
#pragma unroll
    for (int v = 0; v < VW; ++v) re[q][v] = im[q][v] = A(0);
  bool on = s.active;
  if (on && live) {
    bool any = false;
#pragma unroll
    for (int v = 0; v < VW; ++v) any |= live[s.gr * VW + v] != 0;
    on = any;
  }
  if (on) {
    for (size_t row = s.row0; row < nrow; row += s.rstride) {
      const size_t e = row * nrhs + (size_t)s.gr * VW;
      typedef typename vio<P>::ct C;
      cx<C> we[VW];
      vio<P>::unpack(vio<P>::load_raw(w + e), we);
      // Basis vectors in groups of DG, software-pipelined: the loads of
      // group g + 1 are issued before the products of group g, and a
      // scheduling barrier keeps the compiler from hoisting every load to
      // the top (which overflows the registers for large K).  The loads stay
      // in their 16-byte form until used.
      constexpr int DG = 4;
      typename vio<P>::raw vr[KB];
#pragma unroll
      for (int q = 0; q < DG && q < KB; ++q) vr[q] = vio<P>::load_raw(V + (size_t)(k0 + q) * vstride + e);
#pragma unroll
      for (int g = 0; g < KB; g += DG) {
#pragma unroll
        for (int q = g + DG; q < g + 2 * DG && q < KB; ++q)
          vr[q] = vio<P>::load_raw(V + (size_t)(k0 + q) * vstride + e);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = g; q < g + DG && q < KB; ++q) {
          cx<C> ve[VW];
          vio<P>::unpack(vr[q], ve);
#pragma unroll
          for (int v = 0; v < VW; ++v) {
            // conj(v) w
            re[q][v] += (A)(ve[v].re * we[v].re + ve[v].im * we[v].im);
            im[q][v] += (A)(ve[v].re * we[v].im - ve[v].im * we[v].re);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  vblock_combine<KB, VW, A>(re, im, K, nrhs, on, part);
}

// LH: the K x nrhs coefficients are first copied to LDS (dynamic, K nrhs
// entries), so that the vector-memory pipe carries only basis loads.
template <int P, bool LH>
__global__ __launch_bounds__(256) void k_cgs_update_v(const typename vio<P>::store* __restrict__ V, size_t vstride,
                                                      int K, const cx<double>* __restrict__ h,
                                                      typename vio<P>::store* __restrict__ w, size_t nrow, int nrhs,
                                                      const int* __restrict__ live, cx<double>* __restrict__ part) {
  if (none_live(live, nrhs)) return;
  extern __shared__ char lds_raw[];
  cx<double>* hs = reinterpret_cast<cx<double>*>(lds_raw);
  constexpr int VW = vio<P>::VW;
  typedef typename vio<P>::acc_t A;
  const int G = nrhs / VW;
  if (LH) {
    // [k][v][group]: the lanes of a wavefront read G consecutive entries for
    // one (k, v), not G entries VW apart (fewer LDS bank conflicts)
    for (int i = threadIdx.x; i < K * nrhs; i += blockDim.x) {
      const int k = i / nrhs, r = i - k * nrhs;
      hs[((size_t)k * VW + r % VW) * G + r / VW] = h[i];
    }
    __syncthreads();
  }
  vsched s = vgrid(G);
  A re[1][VW], im[1][VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) re[0][v] = im[0][v] = A(0);
  bool on = s.active;
  if (on && live) {
    bool any = false;
#pragma unroll
    for (int v = 0; v < VW; ++v) any |= live[s.gr * VW + v] != 0;
    on = any;
  }
  if (on) {
    for (size_t row = s.row0; row < nrow; row += s.rstride) {
      const size_t e = row * nrhs + (size_t)s.gr * VW;
      cx<double> x[VW];
      vio<P>::load(w + e, x);
      // four basis vectors per round, loads issued together, terms added in
      // the order k = 0, 1, ..., K-1
      int k = 0;
      for (; k + 4 <= K; k += 4) {
        cx<double> ve[4][VW];
#pragma unroll
        for (int q = 0; q < 4; ++q) vio<P>::load(V + (size_t)(k + q) * vstride + e, ve[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int v = 0; v < VW; ++v) {
            const cx<double> c = LH ? hs[((k + q) * VW + v) * G + s.gr] : h[(k + q) * nrhs + s.gr * VW + v];
            x[v] = cmadd(x[v], -c, ve[q][v]);
          }
      }
      for (; k < K; ++k) {
        cx<double> ve[VW];
        vio<P>::load(V + (size_t)k * vstride + e, ve);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          const cx<double> c = LH ? hs[(k * VW + v) * G + s.gr] : h[k * nrhs + s.gr * VW + v];
          x[v] = cmadd(x[v], -c, ve[v]);
        }
      }
      vio<P>::save(w + e, x);
#pragma unroll
      for (int v = 0; v < VW; ++v) re[0][v] += (A)(x[v].re * x[v].re + x[v].im * x[v].im);
    }
  }
  vblock_combine<1, VW, A>(re, im, 1, nrhs, on, part);
}

template <int P>
__global__ __launch_bounds__(256) void k_scale_v(typename vio<P>::store* __restrict__ x, size_t nrow, int nrhs,
                                                 const double* __restrict__ f, const int* __restrict__ live) {
  if (none_live(live, nrhs)) return;
  constexpr int VW = vio<P>::VW;
  const int G = nrhs / VW;
  vsched s = vgrid(G);
  if (!s.active) return;
  double fs[VW];
  bool any = false;
#pragma unroll
  for (int v = 0; v < VW; ++v) {
    const int r = s.gr * VW + v;
    const bool lv = !live || live[r];
    fs[v] = lv ? f[r] : 1.0;
    any |= lv;
  }
  if (!any) return;
  for (size_t row = s.row0; row < nrow; row += s.rstride) {
    const size_t e = row * nrhs + (size_t)s.gr * VW;
    cx<double> a[VW];
    vio<P>::load(x + e, a);
#pragma unroll
    for (int v = 0; v < VW; ++v) a[v] = {a[v].re * fs[v], a[v].im * fs[v]};
    vio<P>::save(x + e, a);
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_lincomb_v(const typename vio<P>::store* __restrict__ V, size_t vstride,
                                                   int kmax, const cx<double>* __restrict__ y,
                                                   const int* __restrict__ cnt, typename vio<P>::store* __restrict__ x,
                                                   size_t nrow, int nrhs, double scale) {
  constexpr int VW = vio<P>::VW;
  const int G = nrhs / VW;
  vsched s = vgrid(G);
  if (!s.active) return;
  int n[VW], nmax = 0;
#pragma unroll
  for (int v = 0; v < VW; ++v) {
    const int c = cnt[s.gr * VW + v];
    n[v] = c < kmax ? c : kmax;
    nmax = n[v] > nmax ? n[v] : nmax;
  }
  if (nmax == 0) return;
  for (size_t row = s.row0; row < nrow; row += s.rstride) {
    const size_t e = row * nrhs + (size_t)s.gr * VW;
    cx<double> acc[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[v] = {0.0, 0.0};
    // four basis vectors per round (loads issued together, in their 16-byte
    // form; terms added in the order k = 0, 1, ...)
    int k = 0;
    for (; k + 4 <= nmax; k += 4) {
      typename vio<P>::raw vr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) vr[q] = vio<P>::load_raw(V + (size_t)(k + q) * vstride + e);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cx<double> ve[VW];
        vio<P>::unpack(vr[q], ve);
#pragma unroll
        for (int v = 0; v < VW; ++v)
          if (k + q < n[v]) acc[v] = cmadd(acc[v], y[(size_t)(k + q) * nrhs + s.gr * VW + v], ve[v]);
      }
    }
    for (; k < nmax; ++k) {
      cx<double> ve[VW];
      vio<P>::load(V + (size_t)k * vstride + e, ve);
#pragma unroll
      for (int v = 0; v < VW; ++v)
        if (k < n[v]) acc[v] = cmadd(acc[v], y[(size_t)k * nrhs + s.gr * VW + v], ve[v]);
    }
    cx<double> xv[VW];
    vio<P>::load(x + e, xv);
#pragma unroll
    for (int v = 0; v < VW; ++v) xv[v] = {fma(scale, acc[v].re, xv[v].re), fma(scale, acc[v].im, xv[v].im)};
    vio<P>::save(x + e, xv);
  }
}

// ------------------------------------------------------------ launchers
int vec_width(int prec, int nrhs) {
  if (prec == LQCD_F32 && nrhs % 2 == 0) return 2;
  if (prec == LQCD_F16 && nrhs % 4 == 0) return 4;
  return 1;
}

#define VSWITCH(P, CALL)                                             \
  switch (P) {                                                       \
    case LQCD_F32: { constexpr int PP = LQCD_F32; CALL; } break;     \
    case LQCD_F16: { constexpr int PP = LQCD_F16; CALL; } break;     \
    default: return hipErrorInvalidValue;                            \
  }

template <int P>
static hipError_t dot_v(const void* V, size_t vstride, int k0, int K, const void* w, size_t nrow, int nrhs,
                        const int* live, void* part, unsigned nblk, hipStream_t s) {
  typedef const typename vio<P>::store* In;
#define LQ_DOT_V(KK)                                                                                          \
  case KK:                                                                                                    \
    hipLaunchKernelGGL((k_dot_parts_v<P, KK>), dim3(nblk), dim3(256), 0, s, (In)V, vstride, k0, (In)w, nrow, \
                       nrhs, live, (cx<double>*)part);                                                        \
    break;
  switch (K) {
    LQ_DOT_V(1) LQ_DOT_V(2) LQ_DOT_V(3) LQ_DOT_V(4) LQ_DOT_V(5) LQ_DOT_V(6) LQ_DOT_V(7) LQ_DOT_V(8)
    LQ_DOT_V(9) LQ_DOT_V(10) LQ_DOT_V(11) LQ_DOT_V(12) LQ_DOT_V(13) LQ_DOT_V(14) LQ_DOT_V(15) LQ_DOT_V(16)
    default: return hipErrorInvalidValue;
  }
#undef LQ_DOT_V
  return hipGetLastError();
}
static_assert(DOT_KB == 16, "dot_v instantiates K = 1..16");

hipError_t dot_parts_v(int prec, const void* V, size_t vstride, int k0, int K, const void* w, size_t nelem, int nrhs,
                       const int* live, void* part, unsigned nblk, hipStream_t s) {
  const size_t nrow = nelem / nrhs;
  if (prec == LQCD_F32) return dot_v<LQCD_F32>(V, vstride, k0, K, w, nrow, nrhs, live, part, nblk, s);
  if (prec == LQCD_F16) return dot_v<LQCD_F16>(V, vstride, k0, K, w, nrow, nrhs, live, part, nblk, s);
  return hipErrorInvalidValue;
}

hipError_t cgs_update_v(int prec, const void* V, size_t vstride, int K, const void* h, void* w, size_t nelem,
                        int nrhs, const int* live, void* part, unsigned nblk, hipStream_t s) {
  const size_t nrow = nelem / nrhs;
  const size_t hb = (size_t)K * nrhs * sizeof(cx<double>);
  if (hb <= CGS_LDS_BYTES) {
    VSWITCH(prec, hipLaunchKernelGGL((k_cgs_update_v<PP, true>), dim3(nblk), dim3(256), hb, s,
                                     (const typename vio<PP>::store*)V, vstride, K, (const cx<double>*)h,
                                     (typename vio<PP>::store*)w, nrow, nrhs, live, (cx<double>*)part));
  } else {
    VSWITCH(prec, hipLaunchKernelGGL((k_cgs_update_v<PP, false>), dim3(nblk), dim3(256), 0, s,
                                     (const typename vio<PP>::store*)V, vstride, K, (const cx<double>*)h,
                                     (typename vio<PP>::store*)w, nrow, nrhs, live, (cx<double>*)part));
  }
  return hipGetLastError();
}

hipError_t scale_rhs_v(int prec, void* x, size_t nelem, int nrhs, const double* f, const int* live, unsigned nblk,
                       hipStream_t s) {
  const size_t nrow = nelem / nrhs;
  VSWITCH(prec, hipLaunchKernelGGL((k_scale_v<PP>), dim3(nblk), dim3(256), 0, s, (typename vio<PP>::store*)x, nrow,
                                   nrhs, f, live));
  return hipGetLastError();
}

hipError_t lincomb_v(int prec, const void* V, size_t vstride, int kmax, const void* y, const int* cnt, void* x,
                     size_t nelem, int nrhs, double scale, unsigned nblk, hipStream_t s) {
  const size_t nrow = nelem / nrhs;
  VSWITCH(prec, hipLaunchKernelGGL((k_lincomb_v<PP>), dim3(nblk), dim3(256), 0, s,
                                   (const typename vio<PP>::store*)V, vstride, kmax, (const cx<double>*)y, cnt,
                                   (typename vio<PP>::store*)x, nrow, nrhs, scale));
  return hipGetLastError();
}

}  // namespace lq
