// Internal launchers shared by the C-ABI and the solver (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/lqcd.h"

namespace lq {

// eta = diag * psi + hopc * hop(psi) on the full lattice (hop with the sign of
// D, or of D^dagger when `dagger`).
hipError_t wilson_full(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                       double hopc, int layout, int prec, bool dagger, hipStream_t s);

// out = alpha * xin + beta * hop(in) on the parity-p half lattice, `in` on
// parity 1-p; xin and live may be null.
hipError_t wilson_eo(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                     int nrhs, double alpha, double beta, int layout, int prec, bool dagger, const int* live,
                     hipStream_t s);

// Time-streaming ("pencil") variants of the two kernels above (pencil.hip).
hipError_t wilson_full_pencil(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs,
                              double diag, double hopc, int layout, int prec, bool dagger, hipStream_t s);
hipError_t wilson_eo_pencil(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out,
                            int p, int nrhs, double alpha, double beta, int layout, int prec, bool dagger,
                            const int* live, hipStream_t s);
// Kernel choice: 0 automatic, 1 one site per work item, 2 pencils; pencil[3]
// = (tile Y, tile Z, t segments) overrides, 0 = automatic (pencil may be null).
void set_variant(int v, const int* pencil);
int get_variant();

}  // namespace lq
