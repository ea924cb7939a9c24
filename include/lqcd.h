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
 * 2 = time-streaming pencils with the links of each step staged in LDS,
 * 3 = pencils without LDS staging, 4 = pencils with two rhs per work item
 * (FP32 / FP16 storage, LQCD_LAYOUT2, even nrhs; otherwise as 3), 5 = pencils
 * whose neighbour spinors and links arrive through asynchronous
 * global-to-LDS loads, several hops in flight per wavefront (full operator,
 * FP64, LQCD_LAYOUT2, nrhs >= 11; otherwise as 3), 6 = pencils whose
 * links reach the 16 rhs lanes of a column by row broadcasts, one load per
 * link element and row (LQCD_LAYOUT1 / LQCD_LAYOUT2, nrhs a multiple of 16,
 * any precision, full operator and odd-even hops; otherwise as 3; the FP64
 * full operator runs blocks of more than 16 rhs in chunks of 16, one chunk
 * after another across the grid, so a time slice's working set is that of
 * 16 rhs), 7 = variant 6 whose workgroups (256 / nrhs consecutive x columns,
 * 16 for a chunked FP64 block, compact
 * columns for the odd-even hops) pass their streamed spinors through LDS so
 * that the inner columns read their +-x neighbours there (lattices whose x
 * extent does not hold whole workgroups run as 6),
 * 8 = the Schur apply of dirac_apply_eo(_ws/_noalloc) and of the odd-even
 * solvers in one kernel (Sec. III-A.2): a workgroup computes the odd field
 * H_oe psi_e for its tile of (y, z) rows and the rows around it into LDS,
 * one time slice at a time, and applies H_eo there, so the odd field never
 * reaches memory (any layout and precision; tile_y, tile_z: interior tile,
 * wg_per_cu 1 or 2: the LDS share a workgroup may use; a lattice whose x
 * rows do not fit a workgroup runs the two hop passes; the full operator
 * and single odd-even hop passes run as 7).
 * pencil (may be NULL) = {tile Y, tile Z,
 * number of t segments} for variants 2 and 3; 0 entries are chosen automatically, values
 * that do not divide the lattice fall back to automatic.  Every choice
 * computes the same sums; results agree to rounding.  Not thread-safe
 * against concurrent applies. */
int lqcd_set_kernel_variant(int variant, const int32_t* pencil);

/* Full kernel configuration (for tuning and tests; process-wide).
 * variant: 0 automatic (the autotuner's entry for the arguments, else the
 * default), 1 to 8 as above; tile_y, tile_z, segments: pencil tile and t
 * segments (0 = automatic); nontemporal: 1 = output stores bypass L2
 * allocation; wg_per_cu (0..8): pencil variants run at most this many
 * workgroups per compute unit at a time (0 = no cap; the cap is imposed
 * through the LDS request and an apply whose cap the device cannot express
 * returns LQCD_ERR_HIP).  NULL restores automatic selection.  ms is ignored. */
typedef struct {
  int32_t variant, tile_y, tile_z, segments, nontemporal, wg_per_cu;
  double ms;  /* measured time of one launch (filled by the autotuner) */
} lqcd_kernel_config;
int lqcd_set_kernel_config(const lqcd_kernel_config* cfg);

/* Autotuner: times every candidate kernel configuration for this apply
 * (eo = 0: the full operator, eo = 1: one odd-even hop pass, the kernel a
 * two-pass Schur apply runs twice) on the caller's buffers (eta is
 * overwritten; for eo, psi and eta are half-lattice blocks), reps launches
 * each, and records the fastest for automatic selection by every later apply
 * with the same lattice, nrhs, precision and layout.  With eo it then times
 * the whole Schur apply, the two passes against the fused kernel (variant 8),
 * and records that choice too (a temporary odd block is allocated for it).
 * Synchronises `stream`.  best (may be NULL) receives the hop-pass winner and
 * its time per launch. */
int lqcd_autotune(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, int prec,
                  int layout, int eo, int reps, lqcd_kernel_config* best, void* stream);
/* Write / read the autotuner's table (text, one entry per line).  Load
 * returns the number of entries read or a negative error. */
int lqcd_tune_save(const char* path);
int lqcd_tune_load(const char* path);
void lqcd_tune_clear(void);

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
 * (else LQCD_ERR_SINGULAR).  Two hop passes through a temporary odd
 * half-lattice block that the library allocates with hipMallocAsync on
 * `stream`, or the fused kernel (variant 8) where the tuner or the forced
 * configuration selects it. */
int dirac_apply_eo(const lqcd_lattice* lat, const void* U, const void* psi_e, void* eta_e,
                   int nrhs, double m0, int layout, int prec, int flags, void* stream);

/* dirac_apply_eo with the odd temporary in a caller workspace (device, at
 * least dirac_apply_eo_workspace_bytes() = V/2 x 12 x nrhs complex numbers
 * of `prec`; LQCD_ERR_WORKSPACE if smaller): no allocation, the same
 * kernels.  The workspace size is 0 for invalid arguments. */
size_t dirac_apply_eo_workspace_bytes(const lqcd_lattice* lat, int nrhs, int prec);
int dirac_apply_eo_ws(const lqcd_lattice* lat, const void* U, const void* psi_e, void* eta_e,
                      int nrhs, double m0, int layout, int prec, int flags, void* work,
                      size_t work_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Schur apply as dirac_apply_eo, with its odd half-lattice temporary in a
 * fixed device array of LQCD_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends.  Calls no hipMalloc, hipFree
 * or allocating routine; the caller passes U, psi_e and eta_e as for
 * dirac_apply_eo.  Returns LQCD_ERR_WORKSPACE when the odd block
 * (V/2 x 12 x nrhs complex numbers of `prec`) is larger than the array.
 * The first call on a device, with that device current, resolves the
 * array's address there (hipGetSymbolAddress).  All calls on one device
 * share its array, so calls that overlap on one device (other streams,
 * other threads) race; nothing in the array needs clearing between calls. */
#define LQCD_NOALLOC_SCRATCH_BYTES (256u << 20)
int dirac_apply_eo_noalloc(const lqcd_lattice* lat, const void* U, const void* psi_e, void* eta_e,
                           int nrhs, double m0, int layout, int prec, int flags, void* stream);

/* ---- the clover-improved operator D = D_W - C (Sec. III-A.1) ---- */

/* Clover field C: [V][42] complex in the precision `prec` (same storage as
 * U), device pointer, caller-owned.  Per site two Hermitian 6x6 blocks
 * (Sec. III-A.1: "block-diagonal, each block Hermitian, 42 numbers"): block b
 * acts on spins (2b, 2b+1) x colour with index 3 s + c inside the block, and
 * is stored as its 6 diagonal entries (only the real parts are read) followed
 * by the 15 entries above the diagonal row by row ((0,1), (0,2), ..., (4,5)).
 *
 * eta = D psi = D_W psi - C psi (Algorithm 1 with C), or with
 * flags = LQCD_DAGGER eta = D^dagger psi = D_W^dagger psi - C psi (C is
 * Hermitian).  Arguments, layouts and errors as dirac_apply. */
int dirac_apply_clover(const lqcd_lattice* lat, const void* U, const void* C, const void* psi, void* eta, int nrhs,
                       double m0, int layout, int prec, int flags, void* stream);

/* Cinv[x] = ((4 + m0) I - C(x))^{-1} for every site, in the same packed
 * storage (the inverse of a Hermitian block is Hermitian): the site-local
 * inverse D_oo^{-1} of the odd-even Schur complement.  Computed in FP64 and
 * stored in `prec`.  C, Cinv: device [V][42], caller-owned, distinct.
 * Synchronises `stream`; returns LQCD_ERR_SINGULAR if a block has a pivot
 * below 1e-13 (4 + m0) in magnitude (Cinv is then unspecified). */
int clover_inverse(const lqcd_lattice* lat, const void* C, void* Cinv, double m0, int prec, void* stream);

/* eta_e = S psi_e with S = D_ee - D_eo D_oo^{-1} D_oe (Sec. III-A.2 with the
 * clover term): D_ee = (4 + m0) - C on even sites, D_oo^{-1} = Cinv (from
 * clover_inverse with the same m0) on odd sites.  flags = LQCD_DAGGER gives
 * S^dagger.  psi_e, eta_e: even half-lattice blocks as dirac_apply_eo.  Uses
 * a temporary odd block allocated with hipMallocAsync on `stream`. */
int dirac_apply_eo_clover(const lqcd_lattice* lat, const void* U, const void* C, const void* Cinv, const void* psi_e,
                          void* eta_e, int nrhs, double m0, int layout, int prec, int flags, void* stream);

/* ---- uneven batches of independent lattices ---- */
#define LQCD_MAX_BATCH 16

/* One lattice of a batch: its own gauge field, rhs count and mass.  psi and
 * eta are full-lattice blocks in LQCD_LAYOUT2. */
typedef struct {
  lqcd_lattice lat;
  const void* U;
  const void* psi;
  void* eta;
  int32_t nrhs;
  int32_t reserved;
  double m0;
} lqcd_problem;

/* eta_k = D_k psi_k (or D_k^dagger psi_k) for every problem k in ONE
 * persistent launch (the batched evaluation of Algorithm 1 over several
 * lattices of different size and rhs count).  1 <= nprob <= LQCD_MAX_BATCH;
 * all problems share the precision `prec`.  Same results as one dirac_apply
 * per problem up to rounding (the same sums; the pencil kernel's order of
 * the terms is that of the pencil variants of dirac_apply). */
int dirac_apply_batch(int nprob, const lqcd_problem* probs, int prec, int flags, void* stream);

/* Grid size of the batch launch: 0 = the kernel's default (one (site, rhs)
 * per item: four persistent workgroups per CU; pencils: one workgroup per
 * work unit, longest units first); > 0 = a persistent grid of that many
 * workgroups (the pencil kernel rounds it down to a multiple of 8). */
int lqcd_set_batch_grid(int blocks);

/* Kernel of the batch launch (process-wide): 0 automatic (2 for the full
 * operator, 1 for the odd-even passes of gmres_solve_batch, the faster of
 * the two for each on MI355X), 1 one (site, rhs) per work item, 2
 * time-streaming pencils with each
 * lattice's autotuned tile and segment count (two rhs per work item for
 * FP32 / FP16 blocks with even nrhs).  Returns LQCD_ERR_ARG for other values. */
int lqcd_set_batch_kernel(int kind);

/* Autotuner for the batch launch: times both kernels with their default
 * grid and persistent grids of 1, 2, 4, 8 and 16 workgroups per CU, the
 * pencil kernel also with its residency capped at 1 or 2 workgroups per CU
 * (eta overwritten), keeps the fastest grid (lqcd_set_batch_grid), cap and kernel
 * (lqcd_set_batch_kernel: 1 if the one-site kernel wins, else the automatic
 * choice) and returns the winner in best_kernel, best_grid (either may be
 * NULL). */
int lqcd_autotune_batch(int nprob, const lqcd_problem* probs, int prec, int reps, int* best_kernel, int* best_grid,
                        void* stream);

/* Measured HBM ceiling (a STREAM-style probe, the paper's empirical memory
 * ceiling of Sec. V-A, eq. (4)): kind 0 = copy b = a, 1 = triad
 * a = b + s c, over n doubles per array (device buffers a, b, c of n doubles;
 * c unused for copy).  Tries five launch shapes (persistent grids of 8 or 16
 * workgroups per CU with plain or non-temporal stores, and one workgroup per
 * contiguous chunk with non-temporal loads and stores), each launched `reps`
 * times, and returns the best mean time per launch in *ms.  Synchronises
 * `stream`.  The grid of the chunked shape is n / 2048 workgroups, so n may
 * not exceed 2^42. */
int lqcd_hbm_probe(int kind, double* a, double* b, const double* c, size_t n, int reps, double* ms, void* stream);

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
  int32_t dagger;        /* 1: solve D^dagger x = b instead (the adjoint solve of a gradient) */
  int32_t use_graph;     /* 1: capture each Arnoldi step (all lattices) in a HIP graph and replay it */
  int32_t rhs_block;     /* gmres_solve / gmres_solve_clover solve the rhs in chunks of this many
                            consecutive rhs, one after another (eq. (1)'s block of b rhs, b = this width):
                            the workspace is that of one chunk.  0 = chosen by the library: the full
                            width if the workspace holds it, else among the widths it holds the one
                            with the least tuned apply time per rhs (largest width without table
                            entries); see gmres_rhs_block */
  int32_t gs;            /* orthogonalisation of the batched Arnoldi step (Algorithm 2 leaves it open):
                            0 classical Gram-Schmidt, one pass for all dots (default); 1 CGS2, a second
                            CGS pass against the updated vector; 2 modified Gram-Schmidt, one
                            vector at a time.  Block GMRES ignores it (block CGS + Cholesky QR) */
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

/* Device workspace in bytes that gmres_solve needs for these arguments: for
 * p->rhs_block = w in 1..nrhs-1 that of one chunk of w rhs, else that of all
 * nrhs rhs at once. */
size_t gmres_workspace_bytes(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p);

/* The chunk width gmres_solve uses for these arguments and a workspace of
 * work_bytes: p->rhs_block if it is in 1..nrhs, else the library's choice
 * (see lqcd_solver_params.rhs_block); LQCD_ERR_WORKSPACE if not even one
 * rhs fits. */
int gmres_rhs_block(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p, size_t work_bytes);

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

/* gmres_solve for the clover-improved operator D = D_W - C (C as for
 * dirac_apply_clover, FP64, device [V][42], caller-owned).  With eo the
 * Schur complement uses D_oo^{-1} = ((4+m0) - C_o)^{-1}, computed in the
 * workspace (LQCD_ERR_SINGULAR if singular); the refinement modes convert
 * C and D_oo^{-1} to the working precision.  Workspace from
 * gmres_workspace_bytes_clover; everything else as gmres_solve. */
size_t gmres_workspace_bytes_clover(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p);
int gmres_solve_clover(const lqcd_lattice* lat, const void* U, const void* C, const void* b, void* x, int nrhs,
                       double m0, int layout, const lqcd_solver_params* params, void* work, size_t work_bytes,
                       lqcd_rhs_stats* stats, void* stream);

/* Batched solves over independent lattices (uneven sizes and rhs counts):
 * problem k solves D_k x_k = b_k with b = probs[k].psi and x = probs[k].eta
 * (FP64, full-lattice LQCD_LAYOUT2 blocks, links probs[k].U in FP64), all
 * lattices advancing in lock-step through one GMRES driver; the Wilson
 * applies of every step run in one persistent launch for all lattices.  With
 * params->use_graph the kernels of each Arnoldi step are captured once and
 * replayed as a HIP graph.  stats: sum of nrhs entries, problem by problem.
 * FP16 refinement (mode 2) needs lattices of equal volume. */
size_t gmres_workspace_bytes_batch(int nprob, const lqcd_problem* probs, const lqcd_solver_params* p);
int gmres_solve_batch(int nprob, const lqcd_problem* probs, const lqcd_solver_params* params, void* work,
                      size_t work_bytes, lqcd_rhs_stats* stats, void* stream);

/* Block GMRES: all rhs of the block expand ONE block Krylov subspace
 * K_k(A, R0) = span{R0, A R0, ..., A^{k-1} R0} of the residual block R0 (the
 * block Krylov space of Sec. II that the paper contrasts with its batched
 * solver), and every rhs minimises its residual over that shared space.
 * Restarted block GMRES(m): thin QR of the residual block (Cholesky QR), per
 * step the block apply W = A V_j, block classical Gram-Schmidt
 * H_ij = V_i^H W, W -= V_i H_ij (tall-skinny products on the FP64 matrix
 * cores), Cholesky QR W = V_{j+1} H_{j+1,j}, and the block Hessenberg
 * least-squares problem by complex Givens rotations on the device.  A cycle
 * ends after `restart` steps, when every rhs is below tol, or when the new
 * block is numerically rank deficient; rhs already converged at a restart
 * are left out of the next cycle.
 * Arguments as gmres_solve, with 1 <= nrhs <= LQCD_BLOCK_MAX_RHS, mode 0
 * (FP64) and use_graph 0 only (LQCD_ERR_ARG otherwise); eo, dagger,
 * fixed_iters, x_is_guess, tol and max_restarts as there.  stats[i].iters
 * counts the block steps during which rhs i was active.  Workspace from
 * block_gmres_workspace_bytes (0 for invalid arguments).  Synchronises
 * `stream` once per block step and at every restart. */
#define LQCD_BLOCK_MAX_RHS 16
size_t block_gmres_workspace_bytes(const lqcd_lattice* lat, int nrhs, const lqcd_solver_params* p);
int block_gmres_solve(const lqcd_lattice* lat, const void* U, const void* b, void* x, int nrhs, double m0,
                      int layout, const lqcd_solver_params* params, void* work, size_t work_bytes,
                      lqcd_rhs_stats* stats, void* stream);

/* Gradient of a real loss with respect to the links through y = D psi
 * (differentiation of the Sec. III-A.1 operator): with dL = Re <g, dy> and
 * gradients of complex entries taken as dL/dRe + i dL/dIm,
 *   G_mu(x) = coeff * sum_rhs sum_spin { [(1 - gamma_mu) g(x)] (x) psi(x+mu)^*
 *                                        + psi(x) (x) [(1 + gamma_mu) g(x+mu)]^* }
 * (colour outer products).  coeff = -1/2 gives dL/dU of an apply with
 * upstream gradient g; for a solve x = D^-1 eta pass g = lambda = D^-dag dL/dx,
 * psi = x and coeff = +1/2.  project = 1 returns instead the su(3) force
 * TA(G U_mu(x)^dag), the steepest-ascent direction for U -> exp(h Q) U.
 * U: FP64 gauge field (read only when project = 1); g, psi: FP64
 * full-lattice blocks in `layout`; G: [4][V][3][3] FP64 output. */
int link_force(const lqcd_lattice* lat, const void* U, const void* g, const void* psi, void* G, int nrhs,
               int layout, double coeff, int project, void* stream);

/* out[i] = sum over sites and components of conj(a_i) b_i for every rhs i
 * (FP64 full-lattice blocks in `layout`; out: nrhs complex doubles, device). */
int block_dot(const lqcd_lattice* lat, const void* a, const void* b, int nrhs, int layout, void* out,
              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LQCD_H */
