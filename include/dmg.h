/*
 * dmg.h -- deflated adaptive-multigrid solver for the 2D Schwinger-model
 * Wilson-Dirac system D x = b on one AMD MI355X (gfx950).
 *
 * The method is that of Whyte, Wilcox and Morgan, "Deflated GMRES with
 * Multigrid for Lattice QCD" (Methods section): a three-grid adaptive
 * multigrid preconditioner for an outer FGMRES(8); GMRES(2) pre- and
 * post-smoothing on the fine and intermediate grids; a partial intermediate
 * solve to 0.2 ||b||; and a deflated coarse solve, GMRES-DR(m, k) on the first
 * coarse call and GMRES-Proj(m, k) on every later call, reusing the k
 * eigenvectors.  Cost is counted in matrix-vector products (Mvps) per grid and
 * in fine-equivalent Mvps, eq. (1) of the Results section.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex numbers are interleaved (re, im) pairs of the element type:
 *    double for DMG_FP64 data, float for DMG_FP32 data.
 *  - Fine lattice Nx x Nt, site s = x + Nx * t.  A fine field has 2 complex
 *    components per site, layout [t][x][spin].  A blocked (intermediate or
 *    coarse) field has 24 complex components per site, layout [T][X][24];
 *    components 0..11 have chirality +, 12..23 chirality - (Gamma_5 =
 *    diag(I_12, -I_12)).  Blocking is 4 x 4 sites; block (X, T) holds the
 *    sites x in [4X, 4X+4), t in [4T, 4T+4).
 *  - Multi-RHS fields (nrhs > 1) are nrhs single fields stored back to back.
 *  - ptr_kind selects where caller buffers live: DMG_PTR_HOST (copied through
 *    the context's stream, call returns after the result is on the host) or
 *    DMG_PTR_DEVICE (stream-ordered on the context's stream, not synchronised).
 *  - Every call returns a dmg_status.  Negative values are errors, positive
 *    values warnings; the message of the calling thread's last failure is
 *    dmg_last_error().
 *    Nothing throws or aborts across the ABI.
 *  - Handles are owned by the caller and released with the matching
 *    *_destroy call, which accepts NULL.  A hierarchy refers to its gauge and
 *    context; destroy dependants first.
 */
#ifndef DMG_H
#define DMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int dmg_status;
enum {
  DMG_OK = 0,
  DMG_W_NOT_CONVERGED = 1,   /* solve stopped at its iteration cap; best iterate written */
  DMG_E_INVALID = -1,        /* bad argument, shape or state */
  DMG_E_NONFINITE = -2,      /* NaN or Inf in an input */
  DMG_E_HIP = -3,            /* HIP runtime error */
  DMG_E_BUDGET = -4,         /* allocation would exceed the context's HBM budget */
  DMG_E_NOMEM = -5,          /* device allocation failed */
  DMG_E_BREAKDOWN = -6       /* numerical breakdown (rank-deficient block, singular small system) */
};

enum { DMG_PTR_HOST = 0, DMG_PTR_DEVICE = 1 };

/* Precision of the multigrid preconditioner.  The outer FGMRES (Arnoldi
 * vectors, orthogonalisation, least squares, true residual) is always FP64. */
/* DMG_FP32_BF16: FP32 fields and arithmetic with the intermediate-grid operator D-hat stored in
 * bfloat16 (each part of every block entry rounded to FP32, then to bfloat16, nearest even);
 * a preconditioner precision (and a precision of the level-1 operator hooks).
 * DMG_FP32_BF16C: FP32 fields and arithmetic with the coarse-grid operator D_c rounded to
 * bfloat16 the same way (FP32 accumulation; the rounded entries are held as FP32 values, since
 * the persistent coarse kernel loads them into registers once per solve); the deflation space
 * is built in FP64 on the unrounded D_c.  A preconditioner precision of dmg_solve and the pools
 * (not of the lockstep forms) and of the single-field level-2 operator hook. */
typedef enum { DMG_FP64 = 0, DMG_FP32 = 1, DMG_FP32_BF16 = 2, DMG_FP32_BF16C = 3 } dmg_precision;

typedef struct dmg_context dmg_context;
typedef struct dmg_gauge dmg_gauge;
typedef struct dmg_hierarchy dmg_hierarchy;
typedef struct dmg_deflation dmg_deflation;

/* Device allocator hooks.  alloc(bytes, user) returns device memory or NULL;
 * free(ptr, user) releases it.  NULL hooks mean hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} dmg_allocator;

/* ---------------------------------------------------------------- context */

/* Bind a device and a HIP stream (hipStream_t, NULL = default stream).  The
 * caller keeps the stream.  hbm_budget (bytes, 0 = unlimited) caps the device
 * memory the context may hold; allocations beyond it fail with DMG_E_BUDGET. */
dmg_status dmg_context_create(int device, void* hip_stream, const dmg_allocator* alloc,
                              size_t hbm_budget, dmg_context** out);
void dmg_context_destroy(dmg_context* ctx);
/* Message of the calling thread's last call on ctx ("" if it succeeded; the text is
 * kept per host thread).  Valid until that thread's next call on ctx. */
const char* dmg_last_error(const dmg_context* ctx);
/* Bytes of device memory currently held by the context. */
size_t dmg_context_bytes_in_use(const dmg_context* ctx);
/* Changes the HBM budget (0: none).  Memory already held is kept even when it
 * exceeds the new budget; later allocations past it fail with DMG_E_BUDGET. */
dmg_status dmg_context_set_budget(dmg_context* ctx, size_t hbm_budget);

/* Kernel timing: for the kernels whose bit (1 << DMG_KT_*) is set in `mask`, the
 * library brackets every launch with HIP events on the context's stream
 * (mask 0 turns timing off).  Reading synchronises the stream and returns, per
 * kernel, the summed event time, the launch count and the work units processed
 * (coarse solve: Arnoldi steps; intermediate stencil: blocked sites; multi-RHS
 * stencils: sites x right-hand-side lanes).  Every call of dmg_kernel_timer resets
 * the sums.
 *   DMG_KT_COARSE_PROJ      persistent coarse GMRES-Proj kernel (dmg_solve)
 *   DMG_KT_BLOCK_APPLY_INT  single-field intermediate block stencil, FP64
 *   DMG_KT_BLOCK_BATCHED    multi-RHS block stencil, levels 1 and 2 (lockstep solves,
 *                           batches, dmg_hierarchy_apply_batched)
 *   DMG_KT_WILSON_BATCHED   multi-RHS fine Wilson stencil (same callers) */
enum {
  DMG_KT_COARSE_PROJ = 0,
  DMG_KT_BLOCK_APPLY_INT = 1,
  DMG_KT_BLOCK_BATCHED = 2,
  DMG_KT_WILSON_BATCHED = 3,
  DMG_KT_COUNT = 4
};
dmg_status dmg_kernel_timer(dmg_context* ctx, int mask);
dmg_status dmg_kernel_timer_read(dmg_context* ctx, int kernel, double* total_ms, long long* launches,
                                 long long* units);

/* ------------------------------------------------------------------ gauge */

/* Upload U(1) links U_mu(x, t) = exp(i theta[t][x][mu]) (mu = 0: x, 1: t;
 * host array of 2 * Nx * Nt doubles, radians).  With t_antiperiodic != 0 the
 * fermion sees antiperiodic time boundaries (the links on the last time slice
 * enter D with a minus sign).  The array is copied; FP64 and FP32 copies are
 * kept on the device.  DMG_E_INVALID if Nx or Nt is odd or < 4;
 * DMG_E_NONFINITE on a non-finite angle. */
dmg_status dmg_gauge_create(dmg_context* ctx, int Nx, int Nt, const double* theta,
                            int t_antiperiodic, dmg_gauge** out);
void dmg_gauge_destroy(dmg_gauge* g);

/* out = D in (dagger = 0) or D^dagger in (dagger = 1), D the Wilson-Dirac
 * operator of the Methods section in the r = 1, "m0 + 2" normalisation:
 *   (D psi)(s) = (m0 + 2) psi(s) - 1/2 sum_mu [ (1 - g_mu) U_mu(s) psi(s + mu)
 *                                           + (1 + g_mu) U_mu(s - mu)^* psi(s - mu) ]
 * with g_0 = sigma_1, g_1 = sigma_2; D^dagger = sigma_3 D sigma_3.
 * in/out: nrhs fine fields of precision p; in and out must not overlap. */
dmg_status dmg_apply_dirac(dmg_context* ctx, const dmg_gauge* g, double m0, int dagger,
                           dmg_precision p, const void* in, void* out, int nrhs, int ptr_kind);

/* -------------------------------------------------------------- hierarchy */

typedef struct {
  int nvec;              /* near-null vectors per level (12) */
  double null_tol;       /* CG tolerance of D D^dagger e = -D D^dagger x (1e-4) */
  int null_max_iters;    /* CG iteration cap per level (2000) */
} dmg_setup_params;

/* Build the three-grid hierarchy (Methods section): for each of the two
 * coarsenings, 12 near-null vectors psi = x + e from D D^dagger e = -D D^dagger x
 * solved by CG to null_tol; global orthonormalisation; chiral doubling with
 * (1 +- gamma_5)/2; restriction to 4 x 4 blocks and local orthonormalisation
 * (the columns of P); Galerkin operator P^dagger A P.
 *   start0: nvec fine fields (FP64, layout above) -- the random x of level 0;
 *   start1: nvec intermediate fields (FP64, 24 * (Nx/4) * (Nt/4) complex each).
 * With inject_nullvecs != 0 the two arrays are taken as the finished near-null
 * vectors psi instead and no CG is run (used to check the rest of the setup).
 * Nx and Nt must be divisible by 16 (DMG_E_INVALID).  DMG_E_BREAKDOWN if a
 * local block loses rank.  The hierarchy is device resident and FP64; FP32
 * copies of every operator are made for the mixed-precision form. */
dmg_status dmg_setup(dmg_context* ctx, const dmg_gauge* g, double m0, const dmg_setup_params* prm,
                     const void* start0, const void* start1, int inject_nullvecs, int ptr_kind,
                     dmg_hierarchy** out);
void dmg_hierarchy_destroy(dmg_hierarchy* h);

/* Parts of a hierarchy that can be copied out (parity checks, checkpoints). */
typedef enum {
  DMG_PART_NULLVECS = 0,  /* level 0 or 1: nvec fields psi before orthonormalisation */
  DMG_PART_P = 1,         /* level 0 or 1: prolongator, [site][dof][12] complex; dof 2 or 24;
                             entry (s, a, k) is column 12 * c(a) + k of block B(s) */
  DMG_PART_BLOCKS = 2,    /* level 1 or 2: operator blocks [S][d][col][row] complex (each 24 x 24
                             block column-major), d = 0 self, 1 +x, 2 -x, 3 +t, 4 -t: the
                             coupling from site S + d into site S */
  DMG_PART_SETUP_ITERS = 3 /* level 0 or 1: nvec int32 CG iteration counts */
} dmg_part;
/* Copy a part to a caller-owned host buffer of exactly the part's size in
 * bytes (DMG_E_INVALID otherwise); dmg_hierarchy_part_bytes reports it. */
dmg_status dmg_hierarchy_export(dmg_hierarchy* h, int level, int part, void* host_buf, size_t bytes);
size_t dmg_hierarchy_part_bytes(const dmg_hierarchy* h, int level, int part);

/* Operator and transfer hooks on one level of a hierarchy (parity checks).
 *   DMG_OP_APPLY:    out = A_level in        (level 0, 1, 2)
 *   DMG_OP_APPLY_DAG: out = A_level^dagger in (level 0, 1, 2)
 *   DMG_OP_RESTRICT: out = P_level^dagger in (level 0 or 1: level -> level + 1)
 *   DMG_OP_PROLONG:  out = P_level in        (level 0 or 1: level + 1 -> level)
 * Buffers are single fields of precision p (DMG_FP32_BF16: FP32 fields; the level-1 operator
 * reads its BF16-stored blocks).  DMG_E_INVALID for another precision. */
enum { DMG_OP_APPLY = 0, DMG_OP_APPLY_DAG = 1, DMG_OP_RESTRICT = 2, DMG_OP_PROLONG = 3 };
/* The multi-right-hand-side kernels of dmg_solve_batched on nrhs fields at once
 * (parity hook): op DMG_OP_APPLY, DMG_OP_RESTRICT or DMG_OP_PROLONG as above; in and
 * out hold nrhs consecutive fields of precision p (1 <= nrhs <= 64).  Block stencils
 * (FP32 and FP64) with 16 or more right-hand sides run on the matrix cores; mfma = 0
 * forces the vector-FMA kernel instead. */
dmg_status dmg_hierarchy_apply_batched(dmg_hierarchy* h, int level, int op, dmg_precision p, const void* in,
                                       void* out, int nrhs, int ptr_kind, int mfma);
dmg_status dmg_hierarchy_apply(dmg_hierarchy* h, int level, int op, dmg_precision p,
                               const void* in, void* out, int ptr_kind);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): dmg_hierarchy_apply_batched without any device or
 * pinned allocation.  The lane-interleaved copies of in and out that the multi-RHS kernels
 * work on live in a static device array of DMG_STATIC_SCRATCH_BYTES per GPU, held from the
 * library's load until the process ends.
 *   in, out: DEVICE pointers (nrhs consecutive fields of precision p, as in
 *     dmg_hierarchy_apply_batched); the call is stream-ordered on the context's stream and
 *     returns without synchronising.  The caller owns in and out.
 *   The lane-interleaved input (rounded up to 256 bytes) plus output, element size x field
 *   length x nrhs rounded up to a power of two, must fit DMG_STATIC_SCRATCH_BYTES;
 *   larger requests fail with DMG_E_INVALID (nothing is launched).
 *   Every call on one GPU shares that GPU's array: calls whose work overlaps on the device
 *   (other streams, other host threads, other contexts of the same device) race and must be
 *   ordered by the caller.  The array needs no clearing between calls (every element a call
 *   reads was written earlier in that call).
 *   Results are bitwise those of dmg_hierarchy_apply_batched (same kernels; a launch form
 *   not tuned yet is the default form, and all forms give the same bits).  No autotuning
 *   runs and no kernel timer events are recorded. */
#define DMG_STATIC_SCRATCH_BYTES (64u << 20)
dmg_status dmg_hierarchy_apply_batched_static(dmg_hierarchy* h, int level, int op, dmg_precision p, const void* in,
                                              void* out, int nrhs, int mfma);

/* -------------------------------------------------------------- deflation */

/* Coarse-grid deflation space (Methods section): EMPTY until the first coarse
 * solve runs GMRES-DR(m, k), which leaves A V_k = V_{k+1} Hbar_k; READY after
 * that, when every coarse solve is GMRES-Proj(m, k).  Tied to one hierarchy.
 * Sizes: 1 <= k < m <= 256 and k <= 64 (DMG_E_INVALID otherwise).  Spaces with m <= 63
 * and k <= 31 whose deflated restart fits one workgroup's LDS (every such space with
 * m <= 40) use the short-cycle solvers (persistent coarse kernels); larger ones (the
 * paper's (200, 40)) the long-cycle FP64 solvers, one launch per Arnoldi sub-step, also
 * under an FP32 preconditioner.  The lockstep and batch forms need m - k <= 24. */
dmg_status dmg_deflation_create(dmg_hierarchy* h, int m, int k, dmg_deflation** out);
/* Fill the space now by GMRES-DR on the given coarse right-hand side (FP64,
 * 24 * (Nx/16) * (Nt/16) complex) to tol. */
dmg_status dmg_deflation_build(dmg_deflation* d, const void* rhs, double tol, int ptr_kind);
void dmg_deflation_reset(dmg_deflation* d);
int dmg_deflation_ready(const dmg_deflation* d);
/* Copy the space out: V (n x (k+1), column j at offset j * n) and Hbar
 * ((k+1) x k, column-major), FP64 complex.  Either buffer may be NULL. */
dmg_status dmg_deflation_export(const dmg_deflation* d, void* V, void* H, int* k_out);
void dmg_deflation_destroy(dmg_deflation* d);

/* ------------------------------------------------------------------ solve */

typedef struct {
  double tol;              /* outer true relative residual (1e-8) */
  int outer_m;             /* FGMRES restart length (8) */
  int max_outer_iters;     /* cap on outer Arnoldi steps (400) */
  int smooth_steps;        /* GMRES smoother steps (2) */
  double int_tol;          /* partial intermediate solve, relative (0.2) */
  int int_m;               /* its FGMRES restart length (8) */
  int int_max_iters;       /* its iteration cap (16) */
  double coarse_tol_first; /* GMRES-DR tolerance on the first coarse call (1e-8) */
  double coarse_tol_later; /* GMRES-Proj tolerance afterwards (1e-2) */
  int coarse_max_iters;    /* cap on coarse Arnoldi steps per call (5000) */
  dmg_precision precond;   /* preconditioner precision (outer is FP64) */
  int use_x0;              /* 1: x holds the initial guess */
  int coarse_persistent;   /* each GMRES-Proj coarse solve as one persistent kernel in one
                              cooperative launch (1, the default; the runtime places the whole
                              grid at once), or 0: one launch per Arnoldi sub-step.  Other values
                              are DMG_E_INVALID */
  int int_mode;            /* intermediate grid: 0 partial solve (FGMRES(int_m) to int_tol, the
                              default); 1 one intermediate cycle (smoothing-only treatment) */
  int graphs;              /* lockstep solves (dmg_solve_batched, dmg_batch_*): 1 replays each
                              coarse GMRES-Proj cycle as one captured HIP graph (default, unless a
                              batched-kernel timer is on); 0 launches its kernels one by one.
                              Results are the same either way */
} dmg_solve_params;

typedef struct {
  int outer_iters;
  int converged;
  long long fine_mvps, int_mvps, coarse_mvps;
  double fine_equiv_mvps;   /* eq. (1) */
  double true_rel_resid;    /* ||b - D x|| / ||b|| in FP64 */
  int coarse_calls, coarse_dr_calls;
  double elapsed_ms;
} dmg_solve_stats;

/* Autotuning of the lockstep stencils (process-wide, all contexts).  The multi-RHS block
 * stencil on the matrix cores has launch forms with 64, 32 or 16 right-hand sides per
 * workgroup (form 0, 1, 2; as nb allows) and the FP32 multi-RHS Wilson stencil forms with
 * 256, 128, 512, 64 or 1024 threads per workgroup (form 0 .. 4).  All forms of a kernel compute
 * the same bits.  Unless off, a lockstep workspace (dmg_solve_batched, dmg_batch_create)
 * and dmg_hierarchy_apply_batched time every form of a shape (sites, lanes, precision)
 * the first time they meet it and keep the fastest for the life of the process.
 *   dmg_autotune: mode 0 off (form 0 everywhere), 1 on (default), 2 on and forget the
 *     choices made so far.  DMG_E_INVALID for another mode.
 *   dmg_autotune_force: kernel DMG_TUNE_BLOCK or DMG_TUNE_WILSON; form >= 0 is used for
 *     every shape (out-of-range forms fall back to form 0), -1 restores the tuned choice.
 *   dmg_autotune_report: one line per tuned shape (kernel, precision, sites, lanes, chosen
 *     form, microseconds per launch of each form) into buf (NUL-terminated, truncated to
 *     len); returns the length the full report needs, NUL included. */
enum { DMG_TUNE_BLOCK = 0, DMG_TUNE_WILSON = 1 };
int dmg_autotune(int mode);
int dmg_autotune_force(int kernel, int form);
size_t dmg_autotune_report(char* buf, size_t len);

/* Fill p with the paper's defaults.  GMRES-DR (first coarse call, and the fine-grid
 * comparison solver) also ends when, with the relative residual already at or below 1e-10,
 * a cycle lowers it by less than 1 % (a tolerance such as 1e-15 that the arithmetic cannot
 * reach). */
void dmg_solve_params_default(dmg_solve_params* p);
void dmg_setup_params_default(dmg_setup_params* p);

/* Solve D x = b for nrhs fine right-hand sides (FP64), one after the other,
 * sharing the hierarchy and the deflation space (Sec. 2-3: the space found by
 * GMRES-DR in the first coarse solve serves every later coarse solve through
 * GMRES-Proj).  d == NULL gives the non-deflated comparison method: every coarse
 * solve is CG on the normal equations D_c D_c^dagger y = b_c, x = D_c^dagger y, to
 * coarse_tol_first.  b and x hold nrhs fields of 2 * Nx * Nt complex doubles
 * ([t][x][spin], interleaved re/im).  stats: array of nrhs entries (may be NULL).
 * Returns DMG_OK, or DMG_W_NOT_CONVERGED if some RHS hit its cap (best iterate
 * written). */
dmg_status dmg_solve(dmg_context* ctx, dmg_hierarchy* h, dmg_deflation* d, const dmg_solve_params* prm,
                     const void* b, void* x, int nrhs, int ptr_kind, dmg_solve_stats* stats);

/* Fine-grid comparison solvers without multigrid (the paper's baselines, Results):
 *   DMG_FINE_CGNE        CG on D D^dagger y = b, x = D^dagger y, all nrhs fields in one
 *                        batched CG (m, k ignored); stats: outer_iters = CG iterations,
 *                        fine_mvps = 2 per iteration + 1
 *   DMG_FINE_GMRES_DR    GMRES-DR(m, k) on D from 0 for each right-hand side with a fresh
 *                        deflation space (2 <= m <= 256, 1 <= k < m, k <= 64; the paper's
 *                        fine-grid runs use (200, 40)); outer_iters = Arnoldi steps
 *   DMG_FINE_GMRES_PROJ  GMRES-DR(m, k) on the first right-hand side, whose final space
 *                        A V_k = V_{k+1} Hbar_k then serves GMRES-Proj(m, k) (projection over
 *                        the space, then GMRES(m - k) cycles) on every later right-hand side of
 *                        the call (the paper's multiple right-hand-side comparison); sizes as
 *                        above; coarse_dr_calls = 1 on the first right-hand side only
 * All stop at relative residual tol (max_iters: CG iterations or Arnoldi steps) and report
 * the true relative residual.  b, x: nrhs fields (host or device by ptr_kind).  Sizes that
 * the short-cycle state does not hold (as for the coarse deflation space above) run the
 * long-cycle solvers: FP64 state in device memory, the harmonic-Ritz restart in one
 * workgroup. */
enum { DMG_FINE_CGNE = 0, DMG_FINE_GMRES_DR = 1, DMG_FINE_GMRES_PROJ = 2 };
dmg_status dmg_solve_fine(dmg_context* ctx, dmg_hierarchy* h, int method, int m, int k, double tol, int max_iters,
                          const void* b, void* x, int nrhs, int ptr_kind, dmg_solve_stats* stats);

/* Solves D x = b for nrhs right-hand sides of one hierarchy jointly: the method of
 * dmg_solve (outer FGMRES(outer_m), the three-grid cycle with the partial
 * intermediate solve, GMRES-Proj coarse solves) advanced in lockstep, every launch
 * covering all right-hand sides (multi-RHS stencils, transfers, Gram-Schmidt and
 * projection kernels) while each right-hand side keeps its own Krylov state and
 * stopping decisions.  The deflation space is shared and read only, so d must be
 * READY (Sec. 2-3: the eigenvectors found once serve all later right-hand sides).
 * Layout of b and x as in dmg_solve (nrhs consecutive fields).  Limits: 1 <= nrhs
 * <= 64; outer_m, int_m and d's m - k at most 24; smooth_steps 2; use_x0 0
 * (DMG_E_INVALID otherwise).  stats (nrhs entries, may be NULL): Mvp counts are
 * the lockstep applications made while that right-hand side was iterating;
 * elapsed_ms is the whole call.  Iterates agree with dmg_solve's to rounding
 * (different reduction order).  The workspace is kept in the hierarchy between
 * calls with the same shape. */
dmg_status dmg_solve_batched(dmg_context* ctx, dmg_hierarchy* h, dmg_deflation* d, const dmg_solve_params* prm,
                             const void* b, void* x, int nrhs, int ptr_kind, dmg_solve_stats* stats);

/* ---------------------------------------------------------------------------
 * Batch: iteration-level continuous batching on one hierarchy (serving form).
 *
 * The slots of a batch are the lanes of dmg_solve_batched's lockstep engine: a
 * request joins a free slot between outer FGMRES(outer_m) cycles (x starts at 0),
 * every step runs whole cycles of all running slots in one set of multi-RHS
 * launches, and a slot leaves when its true relative residual reaches tol or it hit
 * max_outer_iters.  A slot's arithmetic depends only on its own data and on the
 * batch's lane count (capacity rounded up to a power of two), so a request gets the
 * same result alone or in any mix on batches of equal capacity.  The deflation space
 * must be READY and is only read.
 *
 * Each batch runs on a device stream of its own, so the steps of different batches
 * overlap on the device: admit, step and retire calls on different batches may come
 * from different host threads at once (create and destroy do not overlap other calls
 * on the context; calls on one batch come from one thread at a time).  admit and
 * retire order that stream against the context's stream, so device b and x stay
 * stream-ordered on the context's stream as elsewhere.
 *
 *   admit(slot, b)        FREE -> RUNNING (DONE at once for b = 0)
 *   step(min_iters)       ceil(min_iters / outer_m) lockstep cycles; finished -> DONE
 *   retire(slot, x)       DONE -> FREE, returns the solution and its statistics
 * ------------------------------------------------------------------------- */
typedef struct dmg_batch dmg_batch;
#define DMG_BATCH_MAX_LANES 64
enum { DMG_SLOT_FREE = 0, DMG_SLOT_RUNNING = 1, DMG_SLOT_DONE = 2 };

/* capacity in [1, 64]; parameter limits as dmg_solve_batched.  Errors: DMG_E_INVALID,
 * DMG_E_BUDGET / DMG_E_NOMEM (workspace). */
dmg_status dmg_batch_create(dmg_hierarchy* h, dmg_deflation* d, int capacity, const dmg_solve_params* prm,
                            dmg_batch** out);
/* b: one fine field (host or device by ptr_kind).  DMG_E_INVALID if the slot is not
 * FREE; DMG_E_NONFINITE for a non-finite host b. */
dmg_status dmg_batch_admit(dmg_batch* bt, int slot, const void* b, int ptr_kind);
/* n_done (may be NULL): slots now DONE. */
dmg_status dmg_batch_step(dmg_batch* bt, int min_iters, int* n_done);
/* x: one fine field (host or device); stats may be NULL (elapsed_ms from admission).
 * Returns DMG_OK or DMG_W_NOT_CONVERGED; DMG_E_INVALID if the slot is not DONE. */
dmg_status dmg_batch_retire(dmg_batch* bt, int slot, void* x, int ptr_kind, dmg_solve_stats* stats);
/* DMG_SLOT_* of a slot, or -1 for a bad index. */
int dmg_batch_slot_state(dmg_batch* bt, int slot);
void dmg_batch_destroy(dmg_batch* bt);

/* ---------------------------------------------------------------------------
 * Pool: independent solves of any resident hierarchy, overlapped on the device.
 *
 * A pool owns `capacity` slots.  Each slot has its own device stream, host worker
 * thread and solver workspace, so the solves of different slots overlap on the
 * device.  A slot takes one right-hand side of any hierarchy of the batch's context
 * (different configurations and lattice sizes may share a pool); slots join and
 * leave between steps:
 *
 *   admit(slot, h, d, b)  -> slot RUNNING        (FREE slots only)
 *   step(min_iters)       -> every RUNNING slot with no advance in flight starts one:
 *                            whole FGMRES(m) cycles until it ran at least min_iters
 *                            more outer iterations or finished (then it becomes
 *                            DONE).  Returns once some advance has ended; the others
 *                            go on in the background, so short solves are retired
 *                            and their slots refilled while long ones run.
 *   retire(slot, x)       -> DONE slot returns its solution and becomes FREE
 *
 * The calls on one pool come from one host thread.
 * The outer FGMRES cycles are never cut, so a solve performs the same arithmetic
 * whatever the step sizes and whichever other solves share the pool; the result
 * is bitwise that of dmg_solve with the same parameters and deflation state.
 * The deflation space of an admitted solve must be READY (dmg_deflation_build, or
 * an earlier dmg_solve) and is only read, so results do not depend on arrival
 * order; d == NULL selects the non-deflated method.  A hierarchy and its deflation
 * space must outlive the slots that use them and must not be rebuilt or reset
 * while admitted.  Persistent coarse solves are launched cooperatively, so the runtime
 * places the whole grid at once and no workgroup of it waits behind the other slots'
 * kernels.  At most DMG_POOL_MAX_SLOTS slots.
 * ------------------------------------------------------------------------- */
typedef struct dmg_pool dmg_pool;
#define DMG_POOL_MAX_SLOTS 8

/* prm: solve parameters of every slot (NULL: defaults).  Errors: DMG_E_INVALID (capacity outside [1, DMG_POOL_MAX_SLOTS], bad
 * parameters), DMG_E_HIP (stream creation). */
dmg_status dmg_pool_create(dmg_context* ctx, int capacity, const dmg_solve_params* prm, dmg_pool** out);
/* Copies b (one fine field of h, host or device by ptr_kind) into the slot and
 * allocates the slot's workspace for h (DMG_E_BUDGET past the context's HBM
 * budget: the request is not admitted and the slot stays FREE).  DMG_E_INVALID if
 * the slot is not FREE, h belongs to another context, or d is not READY. */
dmg_status dmg_pool_admit(dmg_pool* bt, int slot, dmg_hierarchy* h, dmg_deflation* d, const void* b,
                           int ptr_kind);
/* Starts an advance on every idle RUNNING slot as described above and waits until
 * one advance (of any slot) has ended; returns at once if none is in flight.
 * n_done (may be NULL): slots now DONE.  A solve that fails becomes DONE with its
 * error, reported by retire; step itself fails only on invalid arguments. */
dmg_status dmg_pool_step(dmg_pool* bt, int min_iters, int* n_done);
/* Copies the slot's solution to x (host or device by ptr_kind), fills stats (may be
 * NULL; elapsed_ms runs from admission) and frees the slot.  Returns the solve's
 * status (DMG_OK, DMG_W_NOT_CONVERGED or its error; dmg_last_error has the text).
 * DMG_E_INVALID if the slot is not DONE. */
dmg_status dmg_pool_retire(dmg_pool* bt, int slot, void* x, int ptr_kind, dmg_solve_stats* stats);
/* DMG_SLOT_* of a slot, or -1 for a bad slot index. */
int dmg_pool_slot_state(dmg_pool* bt, int slot);
/* Waits for advances in flight, the slots' streams and threads, then releases
 * everything; tolerates NULL. */
void dmg_pool_destroy(dmg_pool* bt);

#ifdef __cplusplus
}
#endif
#endif /* DMG_H */
