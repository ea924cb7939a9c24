// STREAM-style HBM probe: the empirical memory ceiling against which the
// paper measures its kernels (Sec. V-A, eq. (4): STREAM Triad bandwidth times
// arithmetic intensity).  Copy and triad over double arrays with 16-byte
// vector accesses and a grid-stride loop sized to the chip.
#include "common.h"

namespace lq {
int fail(int code, const char* fmt, ...);
int hip_status(hipError_t e, const char* what);

// Each thread moves U 16-byte elements per iteration (independent loads in
// flight), consecutive threads consecutive elements; stores are non-temporal
// when NT (a pure stream has no reuse).
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_copy(const double2* __restrict__ a, double2* __restrict__ b, size_t n2) {
  const size_t T = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * T < n2; i += U * T) {
    d2v_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = *(const d2v_t*)(a + i + u * T);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (NT) __builtin_nontemporal_store(v[u], (d2v_t*)(b + i + u * T));
      else *(d2v_t*)(b + i + u * T) = v[u];
    }
  }
  for (; i < n2; i += T) b[i] = a[i];
}

template <int U, bool NT>
__global__ __launch_bounds__(256) void k_triad(double2* __restrict__ a, const double2* __restrict__ b,
                                               const double2* __restrict__ c, double s, size_t n2) {
  const size_t T = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * T < n2; i += U * T) {
    d2v_t x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x[u] = *(const d2v_t*)(b + i + u * T);
      y[u] = *(const d2v_t*)(c + i + u * T);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      d2v_t r = {fma(s, y[u].x, x[u].x), fma(s, y[u].y, x[u].y)};
      if (NT) __builtin_nontemporal_store(r, (d2v_t*)(a + i + u * T));
      else *(d2v_t*)(a + i + u * T) = r;
    }
  }
  for (; i < n2; i += T) {
    const double2 x = b[i], y = c[i];
    a[i] = make_double2(fma(s, y.x, x.x), fma(s, y.y, x.y));
  }
}
// One block per contiguous chunk of 256 x U elements (no grid-stride loop):
// the dispatcher keeps the blocks in flight on neighbouring addresses, the
// fastest streaming form measured on MI355X.  Loads and stores bypass cache
// allocation (a pure stream).
template <int U>
__global__ __launch_bounds__(256) void k_copy_chunk(const double2* __restrict__ a, double2* __restrict__ b,
                                                    size_t n2) {
  const size_t base = (size_t)blockIdx.x * 256 * U + threadIdx.x;
  d2v_t v[U];
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (base + u * 256 < n2) v[u] = __builtin_nontemporal_load((const d2v_t*)(a + base + u * 256));
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (base + u * 256 < n2) __builtin_nontemporal_store(v[u], (d2v_t*)(b + base + u * 256));
}

template <int U>
__global__ __launch_bounds__(256) void k_triad_chunk(double2* __restrict__ a, const double2* __restrict__ b,
                                                     const double2* __restrict__ c, double s, size_t n2) {
  const size_t base = (size_t)blockIdx.x * 256 * U + threadIdx.x;
  d2v_t x[U], y[U];
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (base + u * 256 < n2) {
      x[u] = __builtin_nontemporal_load((const d2v_t*)(b + base + u * 256));
      y[u] = __builtin_nontemporal_load((const d2v_t*)(c + base + u * 256));
    }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (base + u * 256 < n2) {
      d2v_t r = {fma(s, y[u].x, x[u].x), fma(s, y[u].y, x[u].y)};
      __builtin_nontemporal_store(r, (d2v_t*)(a + base + u * 256));
    }
}
}  // namespace lq

using namespace lq;

extern "C" int lqcd_hbm_probe(int kind, double* a, double* b, const double* c, size_t n, int reps, double* ms,
                              void* stream) {
  if (!a || !b || (kind == 1 && !c) || !ms || (n & 1) || n == 0)
    return fail(LQCD_ERR_ARG, "lqcd_hbm_probe: bad arguments (n must be even and > 0)");
  if (kind != 0 && kind != 1) return fail(LQCD_ERR_ARG, "lqcd_hbm_probe: kind must be 0 (copy) or 1 (triad)");
  if (reps < 1) reps = 5;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t n2 = n / 2;
  // best of a few launch shapes: persistent grid-stride loops (workgroups
  // per CU, non-temporal stores) and one block per chunk
  double best = 1e300;
  for (int shape = 0; shape < 5; ++shape) {
  const size_t per_cu = shape < 2 ? 8 : 16;
  const bool nt = shape & 1;
  size_t nb = (size_t)ncu * per_cu;
  if (nb * 256 > n2) nb = (n2 + 255) / 256;
  if (shape == 4) {
    nb = (n2 + 1023) / 1024;  // chunks of 256 x 4 elements
    if (nb > 0xffffffffull) continue;
  }
  auto launch = [&]() {
    if (shape == 4) {
      if (kind == 0)
        hipLaunchKernelGGL((k_copy_chunk<4>), dim3((unsigned)nb), dim3(256), 0, s, (const double2*)a, (double2*)b, n2);
      else
        hipLaunchKernelGGL((k_triad_chunk<4>), dim3((unsigned)nb), dim3(256), 0, s, (double2*)a, (const double2*)b,
                           (const double2*)c, 3.0, n2);
    } else if (kind == 0) {
      if (nt) hipLaunchKernelGGL((k_copy<4, true>), dim3((unsigned)nb), dim3(256), 0, s, (const double2*)a, (double2*)b, n2);
      else hipLaunchKernelGGL((k_copy<4, false>), dim3((unsigned)nb), dim3(256), 0, s, (const double2*)a, (double2*)b, n2);
    } else {
      if (nt)
        hipLaunchKernelGGL((k_triad<4, true>), dim3((unsigned)nb), dim3(256), 0, s, (double2*)a, (const double2*)b,
                           (const double2*)c, 3.0, n2);
      else
        hipLaunchKernelGGL((k_triad<4, false>), dim3((unsigned)nb), dim3(256), 0, s, (double2*)a, (const double2*)b,
                           (const double2*)c, 3.0, n2);
    }
  };
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(LQCD_ERR_HIP, "lqcd_hbm_probe: event creation failed");
  launch();
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  (void)hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_status(e, "lqcd_hbm_probe");
  if (t / reps < best) best = t / reps;
  }
  *ms = best;
  return hip_status(hipGetLastError(), "lqcd_hbm_probe launch");
}
