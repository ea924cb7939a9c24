// Clover term C(x) of the improved operator D = D_W - C (Sec. III-A.1):
// block-diagonal with two Hermitian 6x6 blocks per site, 42 complex numbers.
// Block b acts on spins (2b, 2b+1) x colour, index 3 s + c within the block;
// storage per block: its 6 diagonal entries (real parts used), then the 15
// entries above the diagonal row by row.
#pragma once

#include "wilson.h"

namespace lq {

// r = A v for one packed Hermitian 6x6 block
template <typename S, typename R>
__device__ __forceinline__ void herm6_mul(const S* __restrict__ a, const cx<R> (&v)[6], cx<R> (&r)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const R d = ld(a + i).re;
    r[i] = {d * v[i].re, d * v[i].im};
  }
  int k = 6;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j, ++k) {
      const cx<R> u = ld(a + k);
      r[i] = cmadd(r[i], u, v[j]);   // A_ij v_j
      r[j] = cjmadd(r[j], u, v[i]);  // A_ji v_i = conj(A_ij) v_i
    }
}

// C(x) v for one site's packed 42 entries
template <typename S, typename R>
__device__ __forceinline__ spinor<R> clover_mul(const S* __restrict__ c, const spinor<R>& v) {
  spinor<R> out;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    cx<R> in[6], r[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) in[i] = v.c[2 * b + i / 3][i % 3];
    herm6_mul<S, R>(c + 21 * b, in, r);
#pragma unroll
    for (int i = 0; i < 6; ++i) out.c[2 * b + i / 3][i % 3] = r[i];
  }
  return out;
}

}  // namespace lq
