// Multi-right-hand-side (lockstep) kernels.  A batched field holds nb right-hand
// sides interleaved: entry e of right-hand side r sits at e * nb + r, so a wavefront
// reads consecutive right-hand sides of one entry and a matrix entry is loaded once
// for all of them.  nb is a power of two <= 64; every right-hand side has its own
// small-dense state (BS) and its own convergence flags.
#pragma once

#include <string>

#include "common.h"

namespace dmg {

constexpr int MB = 24;   // longest Krylov cycle of the batched solver
constexpr int MQ = 34;   // most quantities of one batched reduction (>= MB + 2, >= k + 1)
constexpr int NBMAX = 64;

// Per right-hand-side state of a batched Krylov cycle (device memory, FP64).
struct BS {
  double2 H[(MB + 1) * MB];   // unrotated Arnoldi matrix, column j at H + j * (MB + 1)
  double2 Rm[(MB + 1) * MB];  // rotated factor (upper triangular)
  double2 g[MB + 1];          // rotated right-hand side
  double2 c[MQ];              // unrotated right-hand side / projection coefficients
  double2 y[MQ];              // least-squares or projection solution
  double2 u[MQ];              // residual coordinates c - H y / projected image
  double2 h2[MB + 1];         // second Gram-Schmidt pass
  double2 rs[MB];             // rotation q acts on rows (q, q + 1)
  double rc[MB];
  double beta, bnorm, tol_abs, est, wn0;
  int steps;   // Arnoldi columns completed in this cycle
  int done;    // no further steps in this cycle
  int active;  // this right-hand side takes part in the current solve
  int brk;     // breakdown
  int cap;     // steps allowed in this cycle
  int pass2;   // the current Arnoldi step needs a second Gram-Schmidt pass
};
// Every right-hand side of bs[0..nb) has done set (flags written by earlier kernels).  A
// workgroup vote: every thread of a workgroup of at least nb threads calls it.
__device__ inline bool lanes_all_done(const BS* bs, int nb) {
  return __syncthreads_and(threadIdx.x < (unsigned)nb ? bs[threadIdx.x].done : 1) != 0;
}
// Host copy of a BS tail (beta .. cap), read back after a cycle.
struct BSTail {
  double beta, bnorm, tol_abs, est, wn0;
  int steps, done, active, brk, cap, pass2;
};

int bred_blocks(int64_t n_entries);

// Autotuning (process-wide): launch forms that give the same bits, timed once per shape.
enum { TK_BLOCK = 0, TK_WILSON = 1, TK_COUNT = 2 };
int tuned_form(int kernel, int prec_bytes, int sites, int nb);  // 0 (default form) until tuned
// time the forms of the batched block / Wilson stencil on these buffers (in is read, out written)
template <typename R>
void b_tune_block(hipStream_t s, const cx<R>* A, const cx<R>* in, cx<R>* out, int Lx, int Lt, int nb,
                  bool mfma = true);
template <typename R>
void b_tune_wilson(hipStream_t s, const cx<R>* U, const cx<R>* in, cx<R>* out, double m0, int Nx, int Nt, int nb);
void b_tune_block_bf16(hipStream_t s, const bf16c* A, const float2* in, float2* out, int Lx, int Lt, int nb,
                       bool mfma = true);
void b_tune_mode(int mode);              // 0 off (default forms), 1 on, 2 on and forget earlier choices
void b_tune_force(int kernel, int form);  // form >= 0 overrides the choice; -1 restores it
std::string b_tune_report();
size_t bred_partials(int nb);  // double2 entries of reduction scratch

// ||x_r||^2 per right-hand side; mode 0: out[r]; mode 3: bs[r].bnorm = ||x_r||;
// mode 1: cycle start (beta, g = c = beta e1, tol_abs = tol_rel * bnorm, done when beta
// is 0 or below tol_abs, inactive right-hand sides done with no steps); mode 2: as 1
// and bnorm = beta first.  Once every right-hand side is done, the batched stencils given
// bs as their skip set and the Arnoldi kernels return at once.
template <typename R>
void launch_b_norm(hipStream_t s, const cx<R>* x, int64_t n, int nb, BS* bs, double tol_rel, int mode, double* out,
                   double2* part);
// *flag = 1 when every right-hand side of bs is done, else 0
void launch_b_all_done(hipStream_t s, const BS* bs, int nb, int* flag);
// y = x / beta_r (0 when beta_r == 0)
template <typename R>
void launch_b_scale_beta(hipStream_t s, const cx<R>* x, cx<R>* y, int64_t n, int nb, const BS* bs);
// Arnoldi step j on batched basis V (field stride ld entries): classical Gram-Schmidt
// with the norm from ||w||^2 - ||h||^2, and a second pass only for the right-hand sides
// where that difference cancels (below eta ||w||^2); Givens update; a right-hand side is
// done once it converged, broke down or took cap steps.  eta: 1e-8 for FP64 vectors,
// 1e-4 for FP32.  anyp2: device flag of the step (some right-hand side needs a second pass).
template <typename R>
void launch_b_arnoldi(hipStream_t s, cx<R>* V, int64_t ld, int64_t n, int nb, int j, BS* bs, int* anyp2,
                      double2* part);
// y = Rm^{-1} g, u = c - H y per active right-hand side
void launch_b_ls_solve(hipStream_t s, BS* bs, int nb);
// x (+)= sum_i coef_i V_i with coef = y (steps terms) or u (steps + 1 terms); active only
template <typename R>
void launch_b_combine(hipStream_t s, cx<R>* x, const cx<R>* V, int64_t ld, int64_t n, int nb, const BS* bs,
                      int use_u, int accumulate);
// two-step GMRES smoother from w1 = A v, w2 = A w1 (coef: 2 * nb double2 scratch)
template <typename R>
void launch_b_smooth2(hipStream_t s, const cx<R>* v, const cx<R>* w1, const cx<R>* w2, int64_t n, int nb,
                      double2* coef, cx<R>* y, cx<R>* r, double2* part);
// GMRES-Proj projection over a shared deflation basis DV (k + 1 single fields):
// c = DV^H r, y = M c, u = Pi c per active right-hand side; then x += DV_k y, r -= DV u.
template <typename R>
void launch_b_project(hipStream_t s, const cx<R>* DV, int k, const double2* M, const double2* Pi, cx<R>* x, cx<R>* r,
                      int64_t n, int nb, BS* bs, double2* part);
// stencils on batched fields (sub: out = sub - A in; skip: return at once when every
// right-hand side of the state array skip[0..nb) is done)
template <typename R>
void launch_b_wilson(hipStream_t s, const cx<R>* U, const cx<R>* in, cx<R>* out, double m0, int Nx, int Nt, int nb,
                     const cx<R>* sub, const BS* skip = nullptr);
template <typename R>
void launch_b_block(hipStream_t s, const cx<R>* A, const cx<R>* in, cx<R>* out, int Lx, int Lt, int nb,
                    const cx<R>* sub, const BS* skip = nullptr, bool mfma = true);
// block stencil with BF16-stored blocks, FP32 fields and arithmetic
void launch_b_block_bf16(hipStream_t s, const bf16c* A, const float2* in, float2* out, int Lx, int Lt, int nb,
                         const float2* sub, const BS* skip = nullptr, bool mfma = true);
template <typename R>
void launch_b_restrict(hipStream_t s, const cx<R>* P, const cx<R>* fine, cx<R>* coarse, int Lx, int Lt, int dof,
                       int nb);
template <typename R>
void launch_b_prolong(hipStream_t s, const cx<R>* P, const cx<R>* coarse, cx<R>* fine, int Lx, int Lt, int dof, int nb,
                      int accumulate);
// nrhs consecutive fields of n entries <-> batched field (right-hand sides nrhs..nb-1 zero)
template <typename T>
void launch_b_gather(hipStream_t s, const T* in, T* out, int64_t n, int nrhs, int nb);
template <typename T>
void launch_b_scatter(hipStream_t s, const T* in, T* out, int64_t n, int nrhs, int nb);
// lane r of a batched field: dst lane = src lane (src null: zero)
void launch_b_lane_copy(hipStream_t s, const double2* src, double2* dst, int64_t n, int nb, int r);
// to_lane = 1: lane r of out = single field in; 0: single field out = lane r of in
void launch_b_lane_io(hipStream_t s, const double2* in, double2* out, int64_t n, int nb, int r, int to_lane);
// per right-hand-side flags for the next cycle: bs[r].active = st[2r], bs[r].cap = st[2r+1]
void launch_b_set_state(hipStream_t s, BS* bs, const int* st, int nb);

}  // namespace dmg
