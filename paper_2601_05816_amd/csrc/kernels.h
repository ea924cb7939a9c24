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

// Kernel configuration of one apply.  variant: 1 one (site, rhs) per work
// item, 2 time-streaming pencils with links staged in LDS, 3 pencils without
// staging, 4 pencils with two rhs per work item (FP32/FP16, rhs-innermost,
// even nrhs; otherwise treated as 3), 5 pencils fed by global-to-LDS loads
// (FP64, rhs-innermost, nrhs >= 11, full operator; otherwise treated as 3), 6 pencils whose links
// reach the rhs lanes of a column by row broadcasts (rhs-fastest layouts, nrhs % 16 == 0; otherwise
// treated as 3), 7 as 6 with the +-x neighbours of a workgroup's inner columns read from LDS
// (lattices whose x rows hold whole workgroups; otherwise treated as 6), 8 the Schur complement in
// one kernel (schur.hip; selects that kernel for a whole Schur apply, is treated as 7 by the full
// operator and by a single odd-even hop pass); ty, tz, nseg: pencil tile and t segments
// (0 = automatic); nt: non-temporal output stores; occ: at most this many
// workgroups per compute unit (0 = no cap), enforced through the LDS request.
struct kcfg {
  int variant, ty, tz, nseg, nt, occ;
};
// Tuning kinds: a full-operator apply, one odd-even hop pass, a whole Schur apply.
enum { KIND_FULL = 0, KIND_EO = 1, KIND_SCHUR = 2 };

// Time-streaming ("pencil") variants of the two kernels above (pencil.hip).
hipError_t wilson_full_pencil(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs,
                              double diag, double hopc, int layout, int prec, bool dagger, const kcfg& c,
                              hipStream_t s);
hipError_t wilson_eo_pencil(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out,
                            int p, int nrhs, double alpha, double beta, int layout, int prec, bool dagger,
                            const int* live, const kcfg& c, hipStream_t s);
// the same pencils for D = D_W - C (the epilogue of wilson_full_clover)
hipError_t wilson_full_clover_pencil(const lqcd_lattice* lat, const void* U, const void* C, const void* psi,
                                     void* eta, int nrhs, double diag, double hopc, int layout, int prec, bool dagger,
                                     const kcfg& c, hipStream_t s);

// Pencil kernels with two rhs per work item (pencil_nr.hip): rhs-innermost
// layout, FP32 / FP16 storage, even nrhs.
bool nr_supported(int prec, int layout, int nrhs);
hipError_t wilson_eo_nr(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                        int nrhs, double alpha, double beta, int prec, bool dagger, const int* live, const kcfg& c,
                        hipStream_t s);
hipError_t wilson_full_nr(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                          double hopc, int prec, bool dagger, const kcfg& c, hipStream_t s);

// Pencil kernel fed by global-to-LDS loads (pencil_dma.hip): FP64 storage,
// rhs-innermost layout, nrhs >= 11.
bool dma_supported(int prec, int layout, int nrhs);
hipError_t wilson_full_dma(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                           double hopc, int prec, bool dagger, const kcfg& c, hipStream_t s);

// Pencil kernels with links moved to the rhs lanes by row broadcasts
// (pencil_bc.hip): rhs-fastest layouts, nrhs a multiple of 16, any precision.
bool bc_supported(int layout, int nrhs);
hipError_t wilson_full_bc(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, double diag,
                          double hopc, int layout, int prec, bool dagger, const kcfg& c, hipStream_t s);
hipError_t wilson_eo_bc(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                        int nrhs, double alpha, double beta, int layout, int prec, bool dagger, const int* live,
                        const kcfg& c, hipStream_t s);

// The Schur complement eta_e = d in - (1/4d) H_eo H_oe in (schur.hip).
// schur_apply runs the fused kernel when the configuration for KIND_SCHUR
// selects it (variant 8) and the lattice fits, else the two hop passes
// through tmp (an odd block of nrhs spinors; untouched by the fused kernel).
bool schur_fused_supported(const lqcd_lattice* lat, int nrhs, int prec, const kcfg& c);
hipError_t schur_fused(const lqcd_lattice* lat, const void* U, const void* in, void* out, int nrhs, double d,
                       int layout, int prec, bool dagger, const int* live, const kcfg& c, hipStream_t s);
hipError_t schur_apply(const lqcd_lattice* lat, const void* U, const void* in, void* out, void* tmp, int nrhs,
                       double d, int layout, int prec, bool dagger, const int* live, hipStream_t s);

// The clover-improved operator (clover.hip): one (site, rhs) per work item.
// Full: eta = diag psi - C psi + hopc hop(psi).  Odd-even half (out on
// parity p, in on 1-p): out = Cout [alpha xin - Cx xin + beta hop(in)], Cx and
// Cout per-site packed 42-entry fields (either may be null).
hipError_t wilson_full_clover(const lqcd_lattice* lat, const void* U, const void* C, const void* psi, void* eta,
                              int nrhs, double diag, double hopc, int layout, int prec, bool dagger, hipStream_t s);
hipError_t wilson_eo_clover(const lqcd_lattice* lat, const void* U, const void* in, const void* xin, void* out, int p,
                            int nrhs, double alpha, double beta, int layout, int prec, bool dagger, const int* live,
                            const void* Cx, const void* Cout, hipStream_t s);
// out = alpha Cm in on the parity-p half lattice (a site-local block multiply)
hipError_t clover_site_mul(const lqcd_lattice* lat, const void* Cm, const void* in, void* out, int p, int nrhs,
                           double alpha, int layout, int prec, hipStream_t s);
hipError_t clover_invert(const lqcd_lattice* lat, const void* C, void* Cinv, double d, int prec, int* dflag,
                         hipStream_t s);

// Configuration for an apply (tune.hip): the process-wide forced setting if
// any, else the autotuner's entry for these arguments, else the default.
kcfg choose_cfg(int kind, const lqcd_lattice* lat, int nrhs, int prec, int layout);
// The autotuner's measured time of one launch for these arguments, if it has an entry.
bool tuned_time(int kind, const lqcd_lattice* lat, int nrhs, int prec, int layout, double* ms);
void set_variant(int v, const int* pencil);

}  // namespace lq
