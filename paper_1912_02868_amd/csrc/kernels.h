// Host launchers of the libdmg kernels.  Every launcher enqueues on `st` and
// returns without synchronising.  Vectors are interleaved complex arrays of the
// element type R (double or float); small-dense state is always FP64.
#pragma once

#include "common.h"

namespace dmg {

// ---------------------------------------------------------------- stencils (stencil.hip)
// Fine Wilson-Dirac operator; U has the fermion boundary sign folded in.
// With `sub` non-null the output is sub - D in (a residual in one pass).
template <typename R>
void launch_wilson(hipStream_t st, const cx<R>* U, const cx<R>* in, cx<R>* out, double m0, int Nx, int Nt,
                   int dagger, int nrhs, const int* skip = nullptr, const cx<R>* sub = nullptr);
// Blocked-lattice operator: 5 blocks of 24 x 24 per site, stored [S][d][col][row].
template <typename R>
void launch_block_apply(hipStream_t st, const cx<R>* A, const cx<R>* in, cx<R>* out, int Lx, int Lt, int dagger,
                        const int* skip = nullptr, const cx<R>* sub = nullptr);
// Restriction out = P^dagger in and prolongation out (+)= P in.  P is [site][dof][12] on the
// finer lattice Lx x Lt with `dof` components per site.
template <typename R>
void launch_restrict(hipStream_t st, const cx<R>* P, const cx<R>* fine, cx<R>* coarse, int Lx, int Lt, int dof);
template <typename R>
void launch_prolong(hipStream_t st, const cx<R>* P, const cx<R>* coarse, cx<R>* fine, int Lx, int Lt, int dof,
                    int accumulate);

// ---------------------------------------------------------------- vector kernels (blas.hip)
// Number of workgroups the reduction kernels use for a vector of n complex entries.
int red_blocks(int64_t n);

// Arnoldi step on basis V (columns V + i * ld), the new vector w = A v_j already stored in
// column j + 1.  Classical Gram-Schmidt applied twice, then ||w||, then the Givens update of
// the least-squares problem; the last step normalises column j + 1.  All four kernels
// return at once when st->done is set.
template <typename R>
void launch_arnoldi_orth(hipStream_t s, cx<R>* V, int64_t ld, int64_t n, int j, KState* ks, double2* partials,
                         unsigned* counter);
// One-pass variant for solves that only precondition: h = V^H w and ||w||^2 in one reduction,
// the norm from their difference, w = (w - V h) / hn; when that difference cancels, ks->pass2
// is set and launch_arnoldi_pass2 must follow (exact second pass, norm, Givens, scaling).
template <typename R>
void launch_arnoldi_orth1(hipStream_t s, cx<R>* V, int64_t ld, int64_t n, int j, KState* ks, double2* partials,
                          unsigned* counter);
template <typename R>
void launch_arnoldi_pass2(hipStream_t s, cx<R>* V, int64_t ld, int64_t n, int j, KState* ks, double2* partials,
                          unsigned* counter);

// x (+)= sum_i coef[i] * V_i, coef = ks->y (use_u = 0) or ks->u (use_u = 1), count = ks->steps (+1 if use_u)
template <typename R, typename RX>
void launch_combine(hipStream_t s, cx<RX>* x, const cx<R>* V, int64_t ld, int64_t n, const KState* ks, int use_u,
                    int accumulate);
// y = a * x + b * y  (a, b real)
template <typename R>
void launch_axpby(hipStream_t s, int64_t n, double a, const cx<R>* x, double b, cx<R>* y);
// y = x - y
template <typename R>
void launch_xmy(hipStream_t s, int64_t n, const cx<R>* x, cx<R>* y);
// precision casts
void launch_cast_d2f(hipStream_t s, int64_t n, const double2* x, float2* y);
void launch_cast_f2d(hipStream_t s, int64_t n, const float2* x, double2* y);
// out[0] = ||x||^2 (deterministic, FP64 accumulation)
template <typename R>
void launch_norm2(hipStream_t s, int64_t n, const cx<R>* x, double* out, double2* partials, unsigned* counter);
// Starts a cycle: ks->beta = ||r||, V_0 = r / beta, g = c = beta e_1, state reset, and the
// stopping threshold tol_abs = tol_rel * bnorm.  set_bnorm = 1 first records bnorm = ||r||
// (a solve that starts from x0 = 0); otherwise bnorm is kept from launch_set_bnorm.
template <typename R>
void launch_cycle_start(hipStream_t s, const cx<R>* r, cx<R>* V0, int64_t n, KState* ks, double tol_rel,
                        int set_bnorm, double2* partials, unsigned* counter);
template <typename R>
void launch_set_bnorm(hipStream_t s, int64_t n, const cx<R>* x, KState* ks, double2* partials, unsigned* counter);
// multi-dot out[i] = V_i^H w, i < nv (deterministic); result to device array
template <typename R>
void launch_multidot(hipStream_t s, const cx<R>* V, int64_t ld, int nv, const cx<R>* w, int64_t n, double2* out,
                     double2* partials, unsigned* counter);
// w -= sum_i coef[i] V_i, i < nv (coef FP64 device array)
template <typename R>
void launch_multi_axpy(hipStream_t s, cx<R>* w, const cx<R>* V, int64_t ld, int nv, const double2* coef, int64_t n,
                       double sign);
// V_out[:, j] = sum_i V_in[:, i] * P[i + ldp * j], i < rows, j < cols (basis rotation)
template <typename R>
void launch_basis_rotate(hipStream_t s, const cx<R>* Vin, cx<R>* Vout, int64_t ld, int64_t n, const double2* P,
                         int ldp, int rows, int cols);
// y = x * scale (scale on device, FP64)
template <typename R>
void launch_scale_dev(hipStream_t s, int64_t n, const cx<R>* x, cx<R>* y, const double* scale, int invert_sqrt);
void launch_rank_test(hipStream_t s, const double* before, const double* after, double rel2, int* status);

// Two-step GMRES smoother from x0 = 0 given w1 = A v and w2 = A w1: y = c0 v + c1 w1
// minimising || v - A y ||, and r = v - A y (skipped when r is null).  coef: 2 device double2.
template <typename R>
void launch_smooth2(hipStream_t s, const cx<R>* v, const cx<R>* w1, const cx<R>* w2, int64_t n, double2* coef,
                    cx<R>* y, cx<R>* r, double2* partials, unsigned* counter);
// z = a x + b y
template <typename R>
void launch_axpbyz(hipStream_t s, int64_t n, double a, const cx<R>* x, double b, const cx<R>* y, cx<R>* z);

// ---------------------------------------------------------------- small dense (dense.hip)
// Back-substitution y = R^{-1} g for the completed steps; then u = c - H y.
void launch_ls_solve(hipStream_t s, KState* ks);
// GMRES-DR deflated restart (harmonic Ritz, k smallest, new Hbar_k, c, rotations) on the
// small matrices.  Writes the (m+1) x (k+1) basis change to Pout (ld m+1).
// final_mode = 1: last compression (harmonic residual direction instead of s).
// work: device scratch of dr_work_elems(m, k) entries; status[0] stays 0 on success.  warm = 1
// lets the eigenvalue iteration start from the previous restart's eigenvalues held in work
// (restarts after the first of one solve, same m and k).
size_t dr_work_elems(int m, int k);
// whether the one-workgroup restart holds (m, k) in LDS (else the long-cycle solvers run)
bool dr_restart_fits(int m, int k);
void launch_dr_restart(hipStream_t s, KState* ks, int m, int k, double2* Pout, int final_mode, double2* work,
                       int* status, int warm);
// After a restart: rotations for the full (k+1) x k block and the rotated rhs.
void launch_qr_block(hipStream_t s, KState* ks, int k);
// GMRES-Proj projection: given c = V_{k+1}^H r in ks->c, d = argmin ||c - Hbar_k d|| using the
// stored deflation matrix Hk ((k+1) x k column-major, ld k+1); y = d, u = Hbar_k d.
void launch_proj_solve(hipStream_t s, const double2* Hk, int k, KState* ks);

// ---------------------------------------------------------------- persistent coarse solve (coarse.hip)
// One cooperative launch per GMRES-Proj(m, k) coarse solve from x = 0; DM and DP are the
// projection matrices of launch_defl_prepare.  Returns 0 (nothing
// launched) when the grid cannot be co-resident; xchg holds 2 n entries; out_iters / out_relres receive the Arnoldi
// steps taken and the final recurrence residual relative to ||b||.  flags: barrier words
// (coarse_proj_flag_words(G) needed, zeroed by the launcher); err: set on a barrier timeout.
// coop = 1: cooperative launch; 0: plain launch (the grid fits the device by construction).
template <typename R>
int launch_coarse_proj(hipStream_t st, const cx<R>* A, int Lx, int Lt, const cx<R>* DV, const double2* DM,
                       const double2* DP, int k,
                       const cx<R>* b, cx<R>* x, double tol, int mm, int max_iters, cx<R>* xchg,
                       double2* partials, size_t partials_elems, int* out_iters, double* out_relres,
                       unsigned* flags, size_t flag_words, int* err, int groups, int coop);
size_t coarse_proj_flag_words(int G);
// Arnoldi part of one GMRES-DR cycle on the coarse grid (FP64) as one persistent launch: extends
// V (ld = n, columns 0 .. j0 orthonormal) and the cycle's state ks from column j0 up to m, or
// until ks->tol_abs or a breakdown; nrot_bound >= ks->nrot on entry.  Returns 1 if launched,
// 0 if the shape does not fit (the caller takes the kernel-per-step path).  flags as for
// launch_coarse_proj; err set on a barrier timeout.
int launch_coarse_arnoldi(hipStream_t st, const double2* A, int Lx, int Lt, double2* V, KState* ks, int nrot_bound,
                          int j0, int m, double2* xchg, double2* partials, size_t partials_elems, unsigned* flags,
                          size_t flag_words, int* err);

// Projection matrices of a deflation space: M = Hbar_k^+ (k x (k+1)) and Pi = Hbar_k M
// ((k+1) x (k+1)), column-major.
void launch_defl_prepare(hipStream_t s, const double2* Hk, int k, double2* M, double2* Pi);

// ---------------------------------------------------------------- setup (setup.hip)
// Batched CG on A A^dagger for nvec fields (x, r, p, q stored as nvec consecutive fields).
void launch_cg_scalars(hipStream_t s, int nvec, const double* pq, const double* rr_new, double* rr, double* alpha,
                       double* beta, int* active, const double* b2, double tol2, int* iters, int phase);
template <typename R>
void launch_cg_update(hipStream_t s, int64_t n, int nvec, cx<R>* x, cx<R>* r, cx<R>* p, const cx<R>* q,
                      const double* alpha, const double* beta, const int* active, int phase);
void launch_batched_dots(hipStream_t s, int64_t n, int nvec, const double2* a, const double2* b, double* out,
                         double2* partials, unsigned* counter);
// Chiral split + local MGS2 per (block, chirality): vectors (nvec fields, already globally
// orthonormal) -> P [site][dof][12].  status[0] set to 1 on rank loss.
void launch_local_ortho(hipStream_t s, const double2* vecs, int64_t n, int nvec, double2* P, int Lx, int Lt, int dof,
                        int* status);
// Wilson operator as 2 x 2 blocks [s][d][col][row] (d: self, +x, -x, +t, -t).
void launch_wilson_blocks(hipStream_t s, const double2* U, double m0, int Nx, int Nt, double2* blocks);
// Galerkin: coarse blocks [S][d][col][row] (24 x 24) from fine blocks [s][d][col][row] (dof x dof).
void launch_galerkin(hipStream_t s, const double2* fineA, const double2* P, int Lx, int Lt, int dof, double2* coarseA);
void launch_d2f(hipStream_t s, int64_t ncomplex, const double2* x, float2* y);
// BF16 copy of FP64 blocks (re, im each rounded to FP32, then to bfloat16, nearest even)
void launch_d2bf16(hipStream_t s, int64_t ncomplex, const double2* x, bf16c* y);
// each part rounded to FP32, then to bfloat16 (nearest even), kept as FP32
void launch_d2bf16f(hipStream_t s, int64_t ncomplex, const double2* x, float2* y);
// block stencil with BF16-stored blocks, FP32 vectors and arithmetic
void launch_block_apply_bf16(hipStream_t st, const bf16c* A, const float2* in, float2* out, int Lx, int Lt,
                             int dagger, const int* skip, const float2* sub);

}  // namespace dmg
