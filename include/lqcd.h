/*
 * lqcd.h - C interface of the multi-right-hand-side Wilson-Dirac library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library applies the Wilson-Dirac operator (Sec. III-A.1) to a block of
 * nrhs spinor fields in one pass, applies its odd-even Schur complement
 * (Sec. III-A.2, odd-even preconditioning), and solves D x = b for every rhs
 * with the batched restarted GMRES of Algorithm 2, optionally as iterative
 * refinement around an FP32 or FP16-storage operator.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: dims[0..3] = (N0, N1, N2, N3), N0 = time is slowest, N3 fastest;
 *   every extent even and >= 2; periodic in all four directions.  A site
 *   (x0,x1,x2,x3) has number ((x0*N1 + x1)*N2 + x2)*N3 + x3 (Sec. III-A.1,
 *   positional numbering; the printed stride formula is read as this
 *   mixed-radix form).  V = N0*N1*N2*N3.
 * Parity: (x0+x1+x2+x3) mod 2; parity 0 is "even".  A half-lattice (compact)
 *   vector of parity p lists the V/2 sites of that parity in ascending site
 *   number; the compact index of site n is n >> 1.
 * Complex numbers are interleaved (re, im) (Sec. III-B, complex storage):
 *   LQCD_F64 = 2 x double, LQCD_F32 = 2 x float, LQCD_F16 = 2 x IEEE half.
 * Spinor: 12 complex per site and rhs, component 3*spin + colour.
 *   Gamma matrices: chiral basis, gamma_mu = [[0, B_mu], [B_mu^dag, 0]],
 *   B_0 = 1, B_k = -i sigma_k; gamma_0 is time.
 * Gauge field U: [4][V][3][3] complex, direction-major, each 3x3 link
 *   row-major (Sec. III-A.1, storage of U_mu), same precision as the spinors.
 * Spinor block layouts (eq. (1) and eq. (3), Sec. III-B):
 *   LQCD_RHS_OUTER [nrhs][V][12]  one contiguous field per rhs
 *   LQCD_LAYOUT1   [V][nrhs][12]  the paper's Layout 1
 *   LQCD_LAYOUT2   [V][12][nrhs]  the paper's Layout 2 (rhs innermost); the
 *                                 fastest layout on this hardware
 *   For half-lattice vectors replace V by V/2 and the site by its compact index.
 * Operator (Sec. III-A.1, no clover term, a = 1):
 *   D psi(x) = (4+m0) psi(x) - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                                  + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ].
 * Memory: every array pointer is a DEVICE pointer owned by the caller, aligned
 *   to its complex type; no call keeps a pointer after it returns.  Input and
 *   output blocks must not overlap.
 * Streams: every call is enqueued on `stream` (a hipStream_t; NULL = the null
 *   stream) and returns without synchronising, except gmres_solve.
 * Errors: 0 = success; a negative LQCD_ERR_* code leaves outputs unspecified
 *   and sets a per-thread message readable with lqcd_last_error().
 */
#ifndef LQCD_H
#define LQCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int32_t dims[4]; } lqcd_lattice;

enum lqcd_prec { LQCD_F64 = 0, LQCD_F32 = 1, LQCD_F16 = 2 };
enum lqcd_layout { LQCD_RHS_OUTER = 0, LQCD_LAYOUT1 = 1, LQCD_LAYOUT2 = 2 };
enum lqcd_flags { LQCD_DAGGER = 1 };

enum lqcd_status {
  LQCD_OK = 0,
  LQCD_NOT_CONVERGED = 1,   /* warning: x holds the last iterate, stats are filled */
  LQCD_ERR_ARG = -1,        /* null pointer, nrhs < 1, bad parameter */
  LQCD_ERR_DIMS = -2,       /* an extent odd or < 2, or sizes overflow */
  LQCD_ERR_LAYOUT = -3,
  LQCD_ERR_PREC = -4,
  LQCD_ERR_HIP = -5,        /* a HIP runtime call or kernel launch failed */
  LQCD_ERR_WORKSPACE = -6,  /* workspace missing or smaller than required */
  LQCD_ERR_SINGULAR = -7,   /* 4 + m0 = 0: the odd-odd block is not invertible */
  LQCD_ERR_NONFINITE = -8   /* a NaN or Inf appeared in a norm of the solve */
};

/* Message describing the last non-zero status returned on this thread. */
const char* lqcd_last_error(void);

/* Geometry tables on the HOST (Sec. III-A.1 site numbering).
 * nbr (may be NULL): [V][8] int32, columns 0..3 = site of x + mu_hat,
 *   4..7 = site of x - mu_hat, periodic.
 * eo_site (may be NULL): [2][V/2] int32, row p = the parity-p sites in
 *   ascending order.  Returns LQCD_ERR_DIMS for invalid extents. */
int lqcd_lattice_tables(const lqcd_lattice* lat, int32_t* nbr, int32_t* eo_site);

/* Kernel selection for the Wilson kernels (process-wide; for tuning and
 * tests).  variant 0 = automatic, 1 = one (site, rhs) per work item,
 * 2 = time-streaming pencils.  pencil (may be NULL) = {tile Y, tile Z, number
 * of t segments} for variant 2; 0 entries are chosen automatically, values
 * that do not divide the lattice fall back to automatic.  Every choice
 * computes the same sums; results agree to rounding.  Not thread-safe
 * against concurrent applies. */
int lqcd_set_kernel_variant(int variant, const int32_t* pencil);

/* eta = D psi (flags & LQCD_DAGGER: eta = D^dagger psi) for every rhs
 * (Sec. III-A.1 operator, Algorithm 1 fused into one pass; the rhs loop is
 * fused into the site loop as in the block form of eq. (1)).
 * U: gauge field in precision `prec`; psi, eta: full-lattice blocks of nrhs
 * rhs in `layout` and `prec`.  LQCD_F16 computes in FP32 and rounds eta to
 * half precision. */
int dirac_apply(const lqcd_lattice* lat, const void* U, const void* psi, void* eta,
                int nrhs, double m0, int layout, int prec, int flags, void* stream);

/* eta_e = S psi_e with S = D_ee - D_eo D_oo^{-1} D_oe, the even-site Schur
 * complement (Sec. III-A.2, odd-even preconditioning); with LQCD_DAGGER,
 * S^dagger.  psi_e, eta_e: even half-lattice blocks.  Needs 4 + m0 != 0
 * (else LQCD_ERR_SINGULAR).  Uses a temporary odd half-lattice block that the
 * library allocates with hipMallocAsync on `stream`. */
int dirac_apply_eo(const lqcd_lattice* lat, const void* U, const void* psi_e, void* eta_e,
                   int nrhs, double m0, int layout, int prec, int flags, void* stream);

/* Parameters of gmres_solve (Algorithm 2). */
typedef struct {
  int32_t restart;       /* Krylov length m per cycle (restartLen); 1..64, default 30 */
  int32_t max_restarts;  /* cap on restart cycles per solve (restartNum), default 200 */
  int32_t eo;            /* 1: solve the even Schur system and reconstruct the odd sites */
  int32_t mode;          /* 0: FP64 GMRES; 1: FP64 refinement around FP32 inner GMRES;
                            2: FP64 refinement around FP16-storage / FP32-arithmetic inner GMRES */
  int32_t x_is_guess;    /* 1: x holds the initial guess on entry; 0: start from x = 0 */
  int32_t fixed_iters;   /* 1: ignore tol and run exactly max_restarts x restart steps */
  double tol;            /* target ||b_i - D x_i|| <= tol ||b_i|| of the FULL system, per rhs */
  double inner_tol;      /* relative tolerance of each inner solve (modes 1, 2); 0 = default */
  int32_t max_outer;     /* cap on refinement steps (modes 1, 2), default 50 */
  int32_t reserved;
} lqcd_solver_params;

/* Per-rhs results of gmres_solve (HOST memory, nrhs entries). */
typedef struct {
  int32_t iters;         /* Arnoldi steps taken (all cycles, inner steps in modes 1, 2) */
  int32_t restarts;      /* restart cycles started */
  int32_t outer_iters;   /* refinement steps (modes 1, 2), 0 in mode 0 */
  int32_t converged;     /* 1 if true_relres <= tol */
  double true_relres;    /* ||b - D x|| / ||b|| of the full system, evaluated in FP64 */
  double est_relres;     /* last |gamma_{j+1}| / ||b|| estimate of the (inner) GMRES */
} lqcd_rhs_stats;

/* Fill p with the defaults listed above. */
void lqcd_solver_defaults(lqcd_solver_params* p);

/* Device workspace in bytes that gmres_solve needs for these arguments. */
size_t gmres_workspace_bytes(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p);

/* Solve D x_i = b_i for i = 0..nrhs-1 with batched restarted GMRES
 * (Algorithm 2: every rhs runs its own GMRES(m) in lock-step; classical
 * Gram-Schmidt with one fused pass for all dots of a step; complex Givens
 * rotations and the Hessenberg least-squares solve in FP64 on the device).
 * U: FP64 gauge field; b, x: FP64 full-lattice blocks in `layout`.
 * work: device workspace of at least gmres_workspace_bytes() bytes.
 * stats: HOST array of nrhs entries (may be NULL).
 * Synchronises `stream` once per restart cycle (to read the convergence
 * flags) and at exit.  Returns LQCD_OK when every rhs reached tol,
 * LQCD_NOT_CONVERGED otherwise, or an error code. */
int gmres_solve(const lqcd_lattice* lat, const void* U, const void* b, void* x, int nrhs,
                double m0, int layout, const lqcd_solver_params* params, void* work,
                size_t work_bytes, lqcd_rhs_stats* stats, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LQCD_H */
