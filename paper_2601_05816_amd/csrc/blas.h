// Internal launchers of the batched BLAS-1 kernels (blas.hip).  Vectors are
// rhs-innermost [nrow][nrhs] complex in precision `prec`; nelem = nrow*nrhs.
// Reduction outputs are complex double.  `part` buffers hold nblk*K*nrhs
// complex doubles; nblk must be reduce_grid(nelem).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace lq {

constexpr int DOT_KB = 16;  // dot products computed per pass over w
// coefficient blocks of at most this many bytes are staged in LDS by the
// Gram-Schmidt update kernels
constexpr size_t CGS_LDS_BYTES = 32768;

unsigned reduce_grid(size_t nelem);
hipError_t dot_parts(int prec, const void* V, size_t vstride, int k0, int K, const void* w, size_t nelem, int nrhs,
                     const int* live, void* part, unsigned nblk, hipStream_t s);
hipError_t norm_parts(int prec, const void* x, size_t nelem, int nrhs, const int* live, void* part, unsigned nblk,
                      hipStream_t s);
hipError_t cgs_update(int prec, const void* V, size_t vstride, int K, const void* h, void* w, size_t nelem, int nrhs,
                      const int* live, void* part, unsigned nblk, hipStream_t s);
// number of partial-sum blocks cgs_update leaves in `part` (reduce that many)
unsigned cgs_update_parts(int prec, size_t nelem, int nrhs, unsigned nblk);
hipError_t b_minus_y(int prec, const void* b, void* y, size_t nelem, int nrhs, const int* live, void* part,
                     unsigned nblk, hipStream_t s);
hipError_t reduce_parts(const void* part, int nblk, int K, int nrhs, double scale, void* out, hipStream_t s);
hipError_t scale_rhs(int prec, void* x, size_t nelem, int nrhs, const double* f, const int* live, hipStream_t s);
hipError_t lincomb(int prec, const void* V, size_t vstride, int kmax, const void* y, const int* cnt, int precx,
                   void* x, size_t nelem, int nrhs, double scale, hipStream_t s);
// out = f[rhs] * in (f may be null); add = true: out += f[rhs] * in
hipError_t convert(int pin, const void* in, int pout, void* out, size_t nelem, int nrhs, const double* f,
                   hipStream_t s);
hipError_t add_scaled(int pin, const void* in, void* out64, size_t nelem, int nrhs, const double* f, hipStream_t s);
hipError_t convert_links(const void* in, int pout, void* out, size_t n, hipStream_t s);
// columns col0 .. col0+nrhs-1 of an ABI block of abi_nrhs rhs <-> an
// internal block of nrhs rhs (abi_nrhs = 0: the ABI block has nrhs rhs)
hipError_t pack(int layout, bool to_internal, void* abi, void* ie, void* io, const int* dims, int nrhs, int eo,
                hipStream_t s, int abi_nrhs = 0, int col0 = 0);

// Block kernels of block GMRES (bblas.hip), FP64 blocks [nrows][b], b <= 16,
// on the FP64 matrix cores.  bgram_parts writes nblk partial sums of the
// K Gram blocks V_k^H W (K <= BG_KB, each b x b, row-major), which
// bgram_reduce adds into out; nblk = bgram_blocks(nrows).
// bgemm: out = alpha Y + beta sum_k V_k C_k, K <= BM_KB coefficient blocks.
constexpr int BG_KB = 8;
constexpr int BM_KB = 8;
unsigned bgram_blocks(size_t nrows);
hipError_t bgram_parts(const void* V, size_t vstride, int K, const void* W, size_t nrows, int b, void* parts,
                       unsigned nblk, hipStream_t s);
hipError_t bgram_reduce(const void* parts, unsigned nblk, int K, int b, void* out, hipStream_t s);
hipError_t bgemm(void* out, const void* Y, double alpha, double beta, const void* V, size_t vstride, int K,
                 const void* C, size_t nrows, int b, hipStream_t s);

// 16-byte-per-lane variants for FP32 / FP16 bases (blasv.hip); the scalar
// launchers above dispatch to them when vec_width(prec, nrhs) > 1.
int vec_width(int prec, int nrhs);
void set_vector_blas(int on);
hipError_t dot_parts_v(int prec, const void* V, size_t vstride, int k0, int K, const void* w, size_t nelem, int nrhs,
                       const int* live, void* part, unsigned nblk, hipStream_t s);
hipError_t cgs_update_v(int prec, const void* V, size_t vstride, int K, const void* h, void* w, size_t nelem,
                        int nrhs, const int* live, void* part, unsigned nblk, hipStream_t s);
hipError_t scale_rhs_v(int prec, void* x, size_t nelem, int nrhs, const double* f, const int* live, unsigned nblk,
                       hipStream_t s);
hipError_t lincomb_v(int prec, const void* V, size_t vstride, int kmax, const void* y, const int* cnt, void* x,
                     size_t nelem, int nrhs, double scale, unsigned nblk, hipStream_t s);

}  // namespace lq
