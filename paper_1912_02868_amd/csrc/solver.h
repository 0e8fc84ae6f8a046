// Multigrid hierarchy, deflation space and Krylov solvers of libdmg (host
// orchestration of the device kernels).
#pragma once

#include <chrono>
#include <memory>

#include "kernels.h"

namespace dmg {

// Device memory owned through the context (allocator hooks + budget).
struct DevBuf {
  dmg_context* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void alloc(dmg_context* c, size_t b);
  void release();
  template <typename T> T* as() const { return (T*)p; }
};

// One level's operator: the fine Wilson-Dirac stencil or a 24-dof block stencil.
struct Op {
  int kind = 0;  // 0 Wilson, 1 block stencil
  int Lx = 0, Lt = 0;
  int64_t n = 0;  // complex entries of one field
  const double2* U64 = nullptr;
  const float2* U32 = nullptr;
  double m0 = 0.0;
  const double2* A64 = nullptr;
  const float2* A32 = nullptr;
  const bf16c* A16 = nullptr;  // set: FP32 applies read these BF16 blocks instead of A32
  // out = A in (sub null) or out = sub - A in
  dmg_context* ctx = nullptr;  // for the kernel timer
  int timer_id = -1;            // DMG_KT_* of this operator's stencil, or -1
  void apply(hipStream_t s, const double2* in, double2* out, int dag, const int* skip,
             const double2* sub = nullptr) const {
    hipEvent_t ta = (timer_id >= 0 && ctx) ? timer_mark(ctx, timer_id, s) : nullptr;
    if (kind == 0) launch_wilson<double>(s, U64, in, out, m0, Lx, Lt, dag, 1, skip, sub);
    else launch_block_apply<double>(s, A64, in, out, Lx, Lt, dag, skip, sub);
    if (ta) timer_span(ctx, timer_id, ta, timer_mark(ctx, timer_id, s), (long long)Lx * Lt);
  }
  void apply(hipStream_t s, const float2* in, float2* out, int dag, const int* skip,
             const float2* sub = nullptr) const {
    if (kind == 0) launch_wilson<float>(s, U32, in, out, m0, Lx, Lt, dag, 1, skip, sub);
    else if (A16) launch_block_apply_bf16(s, A16, in, out, Lx, Lt, dag, skip, sub);
    else launch_block_apply<float>(s, A32, in, out, Lx, Lt, dag, skip, sub);
  }
};

struct Transfer {  // P from level l (Lx x Lt sites, dof per site) to level l + 1
  int Lx = 0, Lt = 0, dof = 0;
  const double2* P64 = nullptr;
  const float2* P32 = nullptr;
  const double2* P(const double2*) const { return P64; }
  const float2* P(const float2*) const { return P32; }
};

// Status fields of a KState read back to the host (layout of KState's tail).
struct KStatus {
  int nrot, steps, done, breakdown;
  double tol_abs, est, beta, wn0, bnorm;
  int pass2;
};

// Krylov workspace: basis V (m + 1 fields), optional Z (m fields), small-dense state.
struct KWS {
  int m = 0;
  int64_t n = 0;
  DevBuf V, Z, ks;
  void alloc(dmg_context* c, int m_, int64_t n_, size_t esize, bool flexible);
  KState* state() const { return ks.as<KState>(); }
};

struct Counters {
  long long mv[3] = {0, 0, 0};
  int coarse_calls = 0, dr_calls = 0;
};

template <typename R> struct Precond;
struct BWork;                 // lane engine of the lockstep multi-right-hand-side solve
void destroy_bwork(BWork* b);
struct BigWS;                 // workspace of the long-cycle GMRES-DR / GMRES-Proj (bigkrylov.hip)
void destroy_bigws(BigWS* b);

// Mutable state of one solve in flight: its stream, reduction scratch, status mirror,
// Mvp counters and every Krylov workspace.  A hierarchy owns one (for dmg_solve and
// the setup); each slot of a batch owns another, so solves on different streams share
// only the read-only operators and the frozen deflation space.
struct Work {
  dmg_context* ctx = nullptr;  // allocator, budget, error text
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DevBuf partials, counters, flags;
  KStatus* host_status = nullptr;  // pinned
  Counters cnt;
  // outer FGMRES (FP64)
  KWS outer;
  DevBuf ob, ox, or_, oz32, ov32, bn2;
  std::unique_ptr<Precond<double>> pc64;
  std::unique_ptr<Precond<float>> pc32;
  // GMRES-DR (FP64)
  KWS dr;
  DevBuf dr_Vtmp, dr_P, dr_work, dr_coef;
  DevBuf dr_xchg, dr_flags;  // persistent GMRES-DR cycle: exchange field, barrier flags
  int dr_m = 0, dr_k = 0;
  BigWS* big = nullptr;      // long-cycle solvers (allocated on first use)
  // state of a resumable outer solve (one right-hand side)
  struct Run {
    dmg_hierarchy* h = nullptr;
    dmg_deflation* d = nullptr;
    dmg_solve_params p{};
    const double2* b = nullptr;
    double2* x = nullptr;
    double bnorm = 0.0, rel = 0.0;
    int iters = 0;
    bool conv = false, done = false;
    std::chrono::steady_clock::time_point t0;
  } run;
  void init(dmg_context* c, hipStream_t s, bool owns);
  Work();
  ~Work();
};

}  // namespace dmg

struct dmg_deflation {
  dmg_hierarchy* h = nullptr;
  int m = 30, k = 10;
  int kk = 0;      // vectors actually stored (k, or the whole Krylov space if shorter)
  int ready = 0;
  int cast_ready = 0;  // FP32 copy of V up to date
  dmg::DevBuf V64, V32, H;  // V: n_c x (kk + 1); H: (kk + 1) x kk column-major, ld kk + 1
  dmg::DevBuf M, Pi;        // projection matrices Hbar^+ (kk x (kk+1)) and Hbar Hbar^+
};

struct dmg_hierarchy {
  dmg_context* ctx = nullptr;
  const dmg_gauge* g = nullptr;
  double m0 = 0.0;
  dmg_setup_params prm{};
  dmg::Op op[3];
  dmg::Transfer tr[2];
  dmg::DevBuf A64[3], A32[3], P64[2], P32[2], null[2];
  dmg::DevBuf A16;  // BF16 copy of the level-1 blocks
  dmg::Op op16;     // level-1 operator reading them (FP32 applies)
  dmg::DevBuf A32c16;  // level-2 blocks rounded to bfloat16, held as FP32
  dmg::Op opc16;       // level-2 operator reading them (FP32 applies)
  int setup_iters[2][64] = {};
  dmg::Work main;  // workspace of dmg_solve, the setup and the deflation build (context stream)
  dmg::BWork* bwork = nullptr;  // workspace of dmg_solve_batched (kept between calls)
  dmg_hierarchy();
  ~dmg_hierarchy();
};

namespace dmg {

// setup (near-null vectors, prolongators, Galerkin operators), on h->main
void build_hierarchy(dmg_hierarchy* h, const double2* start0, const double2* start1, int inject);
// GMRES-DR on the operator of level lvl (2: coarse) in FP64 from x = 0; fills the
// deflation space.  Returns the Arnoldi steps taken.
// persistent: the Arnoldi part of every cycle as one persistent launch where it fits
int coarse_gmres_dr(dmg_hierarchy* h, Work* w, dmg_deflation* d, const double2* b, double2* x, double tol,
                    int max_iters, int lvl = 2, int persistent = 1);
// fine-grid comparison solvers without multigrid: CG on D D^dagger (x = D^dagger y) for
// nrhs fields at once, or GMRES-DR(m, k) per right-hand side
dmg_status fine_solve(dmg_hierarchy* h, int method, int m, int k, double tol, int max_iters, const double2* b,
                      double2* x, int nrhs, dmg_solve_stats* st);
// outer solve of one right-hand side (device buffers b, x; x holds x0 when use_x0) on workspace w
dmg_status outer_solve(dmg_hierarchy* h, Work* w, dmg_deflation* d, const dmg_solve_params* p, const double2* b,
                       double2* x, dmg_solve_stats* st);
// The same solve in three parts: begin (initial residual), advance by whole FGMRES cycles
// until at least `min_iters` more outer iterations ran or the solve ended (returns true
// once it ended), finish (statistics).  The arithmetic does not depend on how the
// advance calls split the cycles.
void outer_begin(dmg_hierarchy* h, Work* w, dmg_deflation* d, const dmg_solve_params* p, const double2* b,
                 double2* x);
bool outer_advance(Work* w, int min_iters);
dmg_status outer_finish(Work* w, dmg_solve_stats* st);
// allocate every buffer a solve of h with these parameters touches on workspace w
void prepare_work(dmg_hierarchy* h, Work* w, dmg_deflation* d, const dmg_solve_params* p);
// FP32 copy of a ready deflation space (made once, on w's stream, which is synchronised)
void prepare_deflation_fp32(Work* w, dmg_deflation* d);
// lockstep solve of nrhs right-hand sides (batched fields in device memory, RHS-major)
dmg_status batched_solve(dmg_hierarchy* h, dmg_deflation* d, const dmg_solve_params* p, const double2* b, double2* x,
                         int nrhs, dmg_solve_stats* st);
void sync_status(Work* w, const KState* ks, KStatus* out);
// Long-cycle GMRES-DR(m, k) on A from x = 0 (m <= 256, k <= 64, FP64); fills d (V_{k+1}, Hbar_k and the
// projection matrices) when d is not null.  Returns the Arnoldi steps taken.
int big_gmres_dr(dmg_context* ctx, Work* w, const Op& A, int m, int k, const double2* b, double2* x, double tol,
                 int max_iters, dmg_deflation* d);
// Long-cycle GMRES-Proj(m, k) on A from x = 0 over the ready space d; returns the Arnoldi steps taken and
// the final residual estimate relative to ||b|| in rel_est.
int big_gmres_proj(Work* w, const Op& A, const dmg_deflation* d, const double2* b, double2* x, double tol,
                   int max_iters, double* rel_est);
// deflation spaces beyond the short-cycle state (m > 64, k > 31, or a restart too large for one
// workgroup's LDS) use the long-cycle solvers
inline bool big_deflation(int m, int k) { return m > MMAX || k > 31 || !dr_restart_fits(m, k); }

}  // namespace dmg
