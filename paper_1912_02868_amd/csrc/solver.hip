// Host orchestration of the deflated three-grid solve (Methods section):
// hierarchy setup, the GMRES(2) smoother, the intermediate and fine cycles, the
// partial intermediate solve, the deflated coarse solve (GMRES-DR, then
// GMRES-Proj), and the outer FP64 FGMRES(8).  All arithmetic runs in the device
// kernels; the host only enqueues them and reads back the few scalars that
// decide control flow (one status read per Arnoldi step of the outer and
// intermediate solves, one per cycle of the coarse solves).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include <limits>
#include <vector>

#include "bigkrylov.h"
#include "solver.h"

namespace dmg {

static_assert(offsetof(KState, steps) == offsetof(KState, nrot) + 4, "KState tail layout");
static_assert(offsetof(KState, tol_abs) == offsetof(KState, nrot) + 16, "KState tail layout");
static_assert(offsetof(KState, bnorm) == offsetof(KState, nrot) + offsetof(KStatus, bnorm), "KState tail layout");

void DevBuf::alloc(dmg_context* c, size_t b) {
  release();
  ctx = c;
  p = dev_alloc(c, b);
  bytes = b;
}
void DevBuf::release() {
  if (p) dev_free(ctx, p, bytes);
  p = nullptr;
  bytes = 0;
}

void KWS::alloc(dmg_context* c, int m_, int64_t n_, size_t esize, bool flexible) {
  m = m_;
  n = n_;
  V.alloc(c, esize * (size_t)n * (m + 1));
  if (flexible) Z.alloc(c, esize * (size_t)n * m);
  ks.alloc(c, sizeof(KState));
  DMG_HIP(hipMemsetAsync(ks.p, 0, sizeof(KState), c->stream));
}

void sync_status(Work* w, const KState* ks, KStatus* out) {
  hipStream_t s = w->stream;
  DMG_HIP(hipMemcpyAsync(w->host_status, &ks->nrot, sizeof(KStatus), hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  *out = *w->host_status;
}

static double read_double(Work* w, const double* p) {
  hipStream_t s = w->stream;
  DMG_HIP(hipMemcpyAsync(w->host_status, p, sizeof(double), hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  double v;
  std::memcpy(&v, w->host_status, sizeof(double));
  return v;
}

static double2* PART(Work* w) { return w->partials.as<double2>(); }
static unsigned* CNT(Work* w) { return w->counters.as<unsigned>(); }

Work::Work() = default;

void Work::init(dmg_context* c, hipStream_t s, bool owns) {
  ctx = c;
  stream = s;
  own_stream = owns;
  DMG_HIP(hipHostMalloc((void**)&host_status, 256, hipHostMallocDefault));
  partials.alloc(c, sizeof(double2) * 80 * 1024);
  counters.alloc(c, sizeof(unsigned) * 64);
  flags.alloc(c, sizeof(int) * 64);
  DMG_HIP(hipMemsetAsync(counters.p, 0, sizeof(unsigned) * 64, s));
  DMG_HIP(hipMemsetAsync(flags.p, 0, sizeof(int) * 64, s));
}

Work::~Work() {
  if (stream) (void)hipStreamSynchronize(stream);
  destroy_bigws(big);
  big = nullptr;
  pc64.reset();
  pc32.reset();
  if (host_status) (void)hipHostFree(host_status);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// ---------------------------------------------------------------- coarse GMRES-DR (FP64)
static void ensure_dr(dmg_hierarchy* h, Work* w, int m, int k, int lvl = 2) {
  const int64_t n = h->op[lvl].n;
  if (w->dr_m == m && w->dr_k == k && w->dr.V.p && w->dr.n == n) return;
  w->dr.alloc(w->ctx, m, n, sizeof(double2), false);
  w->dr_Vtmp.alloc(w->ctx, sizeof(double2) * (size_t)n * (k + 1));
  w->dr_P.alloc(w->ctx, sizeof(double2) * (size_t)(m + 1) * (k + 1));
  w->dr_work.alloc(w->ctx, sizeof(double2) * dr_work_elems(m, k));
  w->dr_coef.alloc(w->ctx, sizeof(double2) * (MMAX + 2));
  w->dr_xchg.alloc(w->ctx, sizeof(double2) * (size_t)n);
  w->dr_flags.alloc(w->ctx, sizeof(unsigned) * coarse_proj_flag_words(256));
  w->dr_m = m;
  w->dr_k = k;
}

static void check_dr_status(Work* w) {
  int st = 0;
  DMG_HIP(hipMemcpyAsync(&st, w->flags.as<int>(), sizeof(int), hipMemcpyDeviceToHost, w->stream));
  DMG_HIP(hipStreamSynchronize(w->stream));
  DMG_CHECK(st == 0, DMG_E_BREAKDOWN, "GMRES-DR restart failed (singular Hessenberg or eigenvalue iteration)");
}

int coarse_gmres_dr(dmg_hierarchy* h, Work* w, dmg_deflation* d, const double2* b, double2* x, double tol,
                    int max_iters, int lvl, int persistent) {
  const int m = d->m, k = d->k;
  if (big_deflation(m, k)) {
    const int it = big_gmres_dr(h->ctx, w, h->op[lvl], m, k, b, x, tol, max_iters, d);
    w->cnt.dr_calls++;
    return it;
  }
  DMG_CHECK(m <= MMAX && k >= 1 && k < m, DMG_E_INVALID, "GMRES-DR sizes");
  ensure_dr(h, w, m, k, lvl);
  hipStream_t s = w->stream;
  const Op& A = h->op[lvl];
  const int64_t n = A.n;
  KState* ks = w->dr.state();
  double2* V = w->dr.V.as<double2>();
  int* status = w->flags.as<int>();
  int* err_d = w->flags.as<int>() + 12;  // grid-barrier timeout of the persistent cycle
  DMG_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
  DMG_HIP(hipMemsetAsync(err_d, 0, sizeof(int), s));
  DMG_HIP(hipMemsetAsync(x, 0, sizeof(double2) * n, s));
  launch_cycle_start<double>(s, b, V, n, ks, tol, 1, PART(w), CNT(w));
  int j0 = 0, iters = 0, restarts = 0;
  KStatus st{};
  double prev_est = -1.0;
  for (;;) {
    // the rotations on entry: none in the first cycle, the restart block's k (k + 1) / 2 later
    const bool pers = persistent && A.kind == 1 &&
                      launch_coarse_arnoldi(s, A.A64, A.Lx, A.Lt, V, ks, j0 == 0 ? 0 : k * (k + 1) / 2, j0, m,
                                            w->dr_xchg.as<double2>(), PART(w), w->partials.bytes / sizeof(double2),
                                            w->dr_flags.as<unsigned>(), w->dr_flags.bytes / sizeof(unsigned), err_d);
    if (!pers)
      for (int j = j0; j < m; ++j) {
        A.apply(s, V + (int64_t)j * n, V + (int64_t)(j + 1) * n, 0, &ks->done);
        launch_arnoldi_orth<double>(s, V, n, n, j, ks, PART(w), CNT(w));
      }
    launch_ls_solve(s, ks);
    launch_combine<double, double>(s, x, V, n, n, ks, 0, 1);
    if (pers) {
      // the cycle's status and the grid barrier's error word in one round trip
      static_assert(sizeof(KStatus) <= 128, "the error word follows the status in the 256-byte pinned buffer");
      int* herr = (int*)((char*)w->host_status + 128);
      DMG_HIP(hipMemcpyAsync(w->host_status, &ks->nrot, sizeof(KStatus), hipMemcpyDeviceToHost, s));
      DMG_HIP(hipMemcpyAsync(herr, err_d, sizeof(int), hipMemcpyDeviceToHost, s));
      DMG_HIP(hipStreamSynchronize(s));
      st = *w->host_status;
      DMG_CHECK(*herr == 0, DMG_E_HIP, "persistent GMRES-DR cycle: grid barrier timed out");
    } else {
      sync_status(w, ks, &st);
    }
    iters += st.steps - j0;
    w->cnt.mv[2] += st.steps - j0;
    if (st.done || iters >= max_iters) break;
    // in the rounding regime (relative residual <= 1e-10), a cycle that lowers the residual by
    // less than 1 % ends the solve (a tolerance the arithmetic cannot reach)
    if (prev_est > 0.0 && st.est > 0.99 * prev_est && st.est <= 1e-10 * st.bnorm) break;
    prev_est = st.est;
    // deflated restart: keep the k smallest harmonic Ritz vectors and the residual
    launch_dr_restart(s, ks, m, k, w->dr_P.as<double2>(), 0, w->dr_work.as<double2>(), status, restarts++ > 0);
    launch_basis_rotate<double>(s, V, w->dr_Vtmp.as<double2>(), n, n, w->dr_P.as<double2>(), m + 1, m + 1, k + 1);
    DMG_HIP(hipMemcpyAsync(V, w->dr_Vtmp.p, sizeof(double2) * n * (k + 1), hipMemcpyDeviceToDevice, s));
    // re-orthogonalise v_{k+1} against v_1 .. v_k
    double2* coef = w->dr_coef.as<double2>();
    launch_multidot<double>(s, V, n, k, V + (int64_t)k * n, n, coef, PART(w), CNT(w));
    launch_multi_axpy<double>(s, V + (int64_t)k * n, V, n, k, coef, n, 1.0);
    launch_norm2<double>(s, n, V + (int64_t)k * n, (double*)(coef + MMAX), PART(w), CNT(w));
    launch_scale_dev<double>(s, n, V + (int64_t)k * n, V + (int64_t)k * n, (const double*)(coef + MMAX), 1);
    j0 = k;
  }
  check_dr_status(w);
  // store the deflation space A V_k = V_{k+1} Hbar_k
  const int cols = st.steps;
  if (cols > k && !st.breakdown) {
    launch_dr_restart(s, ks, cols, k, w->dr_P.as<double2>(), 1, w->dr_work.as<double2>(), status, 0);
    d->V64.alloc(h->ctx, sizeof(double2) * (size_t)n * (k + 1));
    d->H.alloc(h->ctx, sizeof(double2) * (size_t)(k + 1) * k);
    launch_basis_rotate<double>(s, V, d->V64.as<double2>(), n, n, w->dr_P.as<double2>(), cols + 1, cols + 1, k + 1);
    DMG_HIP(hipMemcpy2DAsync(d->H.p, sizeof(double2) * (k + 1), ks->H, sizeof(double2) * (MMAX + 1),
                             sizeof(double2) * (k + 1), k, hipMemcpyDeviceToDevice, s));
    d->kk = k;
    check_dr_status(w);
  } else {
    const int kk = std::max(cols, 1);
    d->V64.alloc(h->ctx, sizeof(double2) * (size_t)n * (kk + 1));
    d->H.alloc(h->ctx, sizeof(double2) * (size_t)(kk + 1) * kk);
    DMG_HIP(hipMemcpyAsync(d->V64.p, V, sizeof(double2) * n * (kk + 1), hipMemcpyDeviceToDevice, s));
    DMG_HIP(hipMemcpy2DAsync(d->H.p, sizeof(double2) * (kk + 1), ks->H, sizeof(double2) * (MMAX + 1),
                             sizeof(double2) * (kk + 1), kk, hipMemcpyDeviceToDevice, s));
    d->kk = kk;
  }
  d->M.alloc(h->ctx, sizeof(double2) * (size_t)d->kk * (d->kk + 1));
  d->Pi.alloc(h->ctx, sizeof(double2) * (size_t)(d->kk + 1) * (d->kk + 1));
  launch_defl_prepare(s, d->H.as<double2>(), d->kk, d->M.as<double2>(), d->Pi.as<double2>());
  d->ready = 1;
  d->cast_ready = 0;
  w->cnt.dr_calls++;
  return iters;
}

// ---------------------------------------------------------------- batched CG on A A^dagger (FP64)
// x_f = argmin for A A^dagger x_f = b_f, f < nvec, each stopping at ||r_f|| <= tol ||b_f||.
static void cg_normal(dmg_hierarchy* h, Work* w, int lvl, int nvec, const double2* b, double2* x, double tol, int max_iters,
                      int* iters_host) {
  hipStream_t s = w->stream;
  const Op& A = h->op[lvl];
  const int64_t n = A.n;
  const size_t fb = sizeof(double2) * (size_t)n * nvec;
  DevBuf r, p, q, t, sc;
  r.alloc(h->ctx, fb);
  p.alloc(h->ctx, fb);
  q.alloc(h->ctx, fb);
  t.alloc(h->ctx, fb);
  // scalars: pq[2 nvec], rrn[2 nvec], rr[nvec], alpha, beta, b2 (doubles); active, iters (ints)
  sc.alloc(h->ctx, sizeof(double) * 8 * 64 + sizeof(int) * 2 * 64);
  double* pq = sc.as<double>();
  double* rrn = pq + 128;
  double* rr = rrn + 128;
  double* alpha = rr + 64;
  double* beta = alpha + 64;
  double* b2 = beta + 64;
  int* active = (int*)(b2 + 64);
  int* its = active + 64;
  DMG_CHECK(nvec <= 64, DMG_E_INVALID, "too many CG fields");
  auto normal = [&](const double2* in, double2* out) {
    if (A.kind == 0) {
      launch_wilson<double>(s, A.U64, in, t.as<double2>(), A.m0, A.Lx, A.Lt, 1, nvec);
      launch_wilson<double>(s, A.U64, t.as<double2>(), out, A.m0, A.Lx, A.Lt, 0, nvec);
    } else {
      for (int f = 0; f < nvec; ++f) {
        launch_block_apply<double>(s, A.A64, in + f * n, t.as<double2>() + f * n, A.Lx, A.Lt, 1);
        launch_block_apply<double>(s, A.A64, t.as<double2>() + f * n, out + f * n, A.Lx, A.Lt, 0);
      }
    }
    w->cnt.mv[lvl] += 2 * nvec;
  };
  DMG_HIP(hipMemsetAsync(x, 0, fb, s));
  DMG_HIP(hipMemcpyAsync(r.p, b, fb, hipMemcpyDeviceToDevice, s));
  DMG_HIP(hipMemcpyAsync(p.p, b, fb, hipMemcpyDeviceToDevice, s));
  launch_batched_dots(s, n, nvec, b, b, rrn, PART(w), CNT(w));
  // rr = b2 = ||b||^2, all active
  std::vector<int> ones(nvec, 1), zeros(nvec, 0);
  DMG_HIP(hipMemcpyAsync(active, ones.data(), sizeof(int) * nvec, hipMemcpyHostToDevice, s));
  DMG_HIP(hipMemcpyAsync(its, zeros.data(), sizeof(int) * nvec, hipMemcpyHostToDevice, s));
  DMG_HIP(hipMemcpy2DAsync(rr, sizeof(double), rrn, 2 * sizeof(double), sizeof(double), nvec,
                           hipMemcpyDeviceToDevice, s));
  DMG_HIP(hipMemcpy2DAsync(b2, sizeof(double), rrn, 2 * sizeof(double), sizeof(double), nvec,
                           hipMemcpyDeviceToDevice, s));
  std::vector<int> act(nvec);
  for (int it = 1; it <= max_iters; ++it) {
    normal(p.as<double2>(), q.as<double2>());
    launch_batched_dots(s, n, nvec, p.as<double2>(), q.as<double2>(), pq, PART(w), CNT(w));
    launch_cg_scalars(s, nvec, pq, rrn, rr, alpha, beta, active, b2, tol * tol, its, 0);
    launch_cg_update<double>(s, n, nvec, x, r.as<double2>(), p.as<double2>(), q.as<double2>(), alpha, beta, active, 0);
    launch_batched_dots(s, n, nvec, r.as<double2>(), r.as<double2>(), rrn, PART(w), CNT(w));
    launch_cg_scalars(s, nvec, pq, rrn, rr, alpha, beta, active, b2, tol * tol, its, 1);
    launch_cg_update<double>(s, n, nvec, x, r.as<double2>(), p.as<double2>(), q.as<double2>(), alpha, beta, active, 1);
    if (it % 4 == 0 || it == max_iters) {
      DMG_HIP(hipMemcpyAsync(act.data(), active, sizeof(int) * nvec, hipMemcpyDeviceToHost, s));
      DMG_HIP(hipStreamSynchronize(s));
      bool any = false;
      for (int f = 0; f < nvec; ++f) any = any || act[f];
      if (!any) break;
    }
  }
  if (iters_host) DMG_HIP(hipMemcpyAsync(iters_host, its, sizeof(int) * nvec, hipMemcpyDeviceToHost, s));
  // the work fields are freed on return: let the stream drain first
  DMG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- setup
// Global orthonormalisation: modified Gram-Schmidt over the whole lattice, two passes.
// Modified Gram-Schmidt applied twice, vectors in index order.  A vector whose norm falls
// below 1e-12 of its norm before the passes makes the set rank-deficient (DMG_E_BREAKDOWN), the
// criterion of the local orthonormalisation.
static void global_mgs2(dmg_hierarchy* h, Work* w, double2* W, int64_t n, int nvec) {
  hipStream_t s = w->stream;
  DevBuf coef;
  coef.alloc(h->ctx, sizeof(double2) * 4);
  double2* c = coef.as<double2>();
  int* status = w->flags.as<int>();
  DMG_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
  for (int k = 0; k < nvec; ++k) {
    double2* wk = W + (int64_t)k * n;
    launch_norm2<double>(s, n, wk, (double*)(c + 3), PART(w), CNT(w));
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < k; ++j) {
        launch_multidot<double>(s, W + (int64_t)j * n, n, 1, wk, n, c, PART(w), CNT(w));
        launch_multi_axpy<double>(s, wk, W + (int64_t)j * n, n, 1, c, n, 1.0);
      }
    launch_norm2<double>(s, n, wk, (double*)(c + 2), PART(w), CNT(w));
    launch_rank_test(s, (const double*)(c + 3), (const double*)(c + 2), 1e-24, status);
    launch_scale_dev<double>(s, n, wk, wk, (const double*)(c + 2), 1);
  }
  int st = 0;
  DMG_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  DMG_CHECK(st == 0, DMG_E_BREAKDOWN, "global orthonormalisation: the near-null vectors are linearly dependent");
}

void build_hierarchy(dmg_hierarchy* h, const double2* start0, const double2* start1, int inject) {
  Work* w = &h->main;
  hipStream_t s = w->stream;
  const int nvec = h->prm.nvec;
  DMG_CHECK(nvec == NV, DMG_E_INVALID, "the blocked layout holds 12 near-null vectors per chirality");
  for (int lvl = 0; lvl < 2; ++lvl) {
    const Op& A = h->op[lvl];
    const int64_t n = A.n;
    const size_t fb = sizeof(double2) * (size_t)n * nvec;
    const double2* start = lvl == 0 ? start0 : start1;
    h->null[lvl].alloc(h->ctx, fb);
    double2* psi = h->null[lvl].as<double2>();
    if (inject) {
      DMG_HIP(hipMemcpyAsync(psi, start, fb, hipMemcpyDeviceToDevice, s));
    } else {
      // b = -A A^dagger x ; solve A A^dagger e = b ; psi = x + e
      DevBuf bb, tt;
      bb.alloc(h->ctx, fb);
      tt.alloc(h->ctx, fb);
      double2* b = bb.as<double2>();
      if (A.kind == 0) {
        launch_wilson<double>(s, A.U64, start, tt.as<double2>(), A.m0, A.Lx, A.Lt, 1, nvec);
        launch_wilson<double>(s, A.U64, tt.as<double2>(), b, A.m0, A.Lx, A.Lt, 0, nvec);
      } else {
        for (int f = 0; f < nvec; ++f) {
          launch_block_apply<double>(s, A.A64, start + f * n, tt.as<double2>() + f * n, A.Lx, A.Lt, 1);
          launch_block_apply<double>(s, A.A64, tt.as<double2>() + f * n, b + f * n, A.Lx, A.Lt, 0);
        }
      }
      launch_axpby<double>(s, n * nvec, 0.0, b, -1.0, b);
      cg_normal(h, w, lvl, nvec, b, psi, h->prm.null_tol, h->prm.null_max_iters, h->setup_iters[lvl]);
      launch_axpby<double>(s, n * nvec, 1.0, start, 1.0, psi);
    }
    // global orthonormalisation (on a copy), chiral split + local orthonormalisation
    DevBuf W;
    W.alloc(h->ctx, fb);
    DMG_HIP(hipMemcpyAsync(W.p, psi, fb, hipMemcpyDeviceToDevice, s));
    global_mgs2(h, w, W.as<double2>(), n, nvec);
    const int dof = lvl == 0 ? 2 : NC;
    const int64_t pe = (int64_t)A.Lx * A.Lt * dof * NV;
    h->P64[lvl].alloc(h->ctx, sizeof(double2) * pe);
    h->P32[lvl].alloc(h->ctx, sizeof(float2) * pe);
    int* status = w->flags.as<int>();
    DMG_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
    launch_local_ortho(s, W.as<double2>(), n, nvec, h->P64[lvl].as<double2>(), A.Lx, A.Lt, dof, status);
    int st = 0;
    DMG_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
    DMG_HIP(hipStreamSynchronize(s));
    DMG_CHECK(st == 0, DMG_E_BREAKDOWN, "local orthonormalisation lost rank in a block");
    launch_d2f(s, pe, h->P64[lvl].as<double2>(), h->P32[lvl].as<float2>());
    h->tr[lvl] = Transfer{A.Lx, A.Lt, dof, h->P64[lvl].as<double2>(), h->P32[lvl].as<float2>()};
    // Galerkin operator of the next level
    const int CLx = A.Lx / BLK, CLt = A.Lt / BLK;
    const int64_t ce = (int64_t)CLx * CLt * 5 * NC * NC;
    h->A64[lvl + 1].alloc(h->ctx, sizeof(double2) * ce);
    h->A32[lvl + 1].alloc(h->ctx, sizeof(float2) * ce);
    if (lvl == 0) {
      DevBuf wb;
      wb.alloc(h->ctx, sizeof(double2) * (size_t)A.Lx * A.Lt * 5 * 4);
      launch_wilson_blocks(s, A.U64, A.m0, A.Lx, A.Lt, wb.as<double2>());
      launch_galerkin(s, wb.as<double2>(), h->P64[0].as<double2>(), A.Lx, A.Lt, 2, h->A64[1].as<double2>());
      DMG_HIP(hipStreamSynchronize(s));
    } else {
      launch_galerkin(s, h->A64[1].as<double2>(), h->P64[1].as<double2>(), A.Lx, A.Lt, NC, h->A64[2].as<double2>());
    }
    launch_d2f(s, ce, h->A64[lvl + 1].as<double2>(), h->A32[lvl + 1].as<float2>());
    Op& C = h->op[lvl + 1];
    C.ctx = h->ctx;
    C.timer_id = lvl == 0 ? DMG_KT_BLOCK_APPLY_INT : -1;
    C.kind = 1;
    C.Lx = CLx;
    C.Lt = CLt;
    C.n = (int64_t)CLx * CLt * NC;
    C.A64 = h->A64[lvl + 1].as<double2>();
    C.A32 = h->A32[lvl + 1].as<float2>();
    if (lvl == 0) {
      h->A16.alloc(h->ctx, sizeof(bf16c) * ce);
      launch_d2bf16(s, ce, h->A64[1].as<double2>(), h->A16.as<bf16c>());
      h->op16 = C;
      h->op16.A16 = h->A16.as<bf16c>();
    } else {
      h->A32c16.alloc(h->ctx, sizeof(float2) * ce);
      launch_d2bf16f(s, ce, h->A64[2].as<double2>(), h->A32c16.as<float2>());
      h->opc16 = C;
      h->opc16.A32 = h->A32c16.as<float2>();
    }
    DMG_HIP(hipStreamSynchronize(s));
  }
}

// ---------------------------------------------------------------- preconditioner (precision R)
template <typename R>
struct Precond {
  using T = cx<R>;
  dmg_hierarchy* h;
  Work* w;
  int smooth_steps = 2;
  KWS sm[2];                       // smoother bases, levels 0 and 1
  DevBuf y[2], r[2], r2[2], sv[2];  // cycle vectors
  KWS e1;                          // partial intermediate solve (flexible)
  DevBuf e1r, e1x, bh;
  DevBuf bc, ec, bc64, ec64, pr;   // coarse vectors
  KWS proj;                        // GMRES-Proj cycles
  int proj_m = 0;
  DevBuf xchg;                     // exchange field of the persistent coarse solve
  DevBuf bflags;                   // its grid-barrier flags
  DevBuf cg_y;                     // CGNE iterate of the non-deflated coarse solve
  const dmg_solve_params* p = nullptr;
  dmg_deflation* defl = nullptr;
  bool bf16 = false;   // FP32 with the BF16-stored intermediate operator
  bool bf16c = false;  // FP32 with the BF16-rounded coarse operator

  Precond(dmg_hierarchy* hh, Work* ww) : h(hh), w(ww) {}
  const Op& op(int l) const { return (l == 1 && bf16) ? h->op16 : (l == 2 && bf16c) ? h->opc16 : h->op[l]; }

  hipStream_t S() const { return w->stream; }
  const T* Pm(int lvl) const { return (const T*)h->tr[lvl].P((const T*)nullptr); }

  void ensure(const dmg_solve_params* prm, dmg_deflation* d) {
    p = prm;
    defl = d;
    bf16 = sizeof(R) == sizeof(float) && prm->precond == DMG_FP32_BF16;
    bf16c = sizeof(R) == sizeof(float) && prm->precond == DMG_FP32_BF16C;
    dmg_context* c = w->ctx;
    const size_t es = sizeof(T);
    if (!sm[0].V.p || smooth_steps != prm->smooth_steps) {
      smooth_steps = prm->smooth_steps;
      for (int l = 0; l < 2; ++l) {
        const int64_t n = h->op[l].n;
        sm[l].alloc(c, smooth_steps, n, es, false);
        y[l].alloc(c, es * n);
        r[l].alloc(c, es * n);
        r2[l].alloc(c, es * n);
        sv[l].alloc(c, es * n);
      }
      const int64_t n2 = h->op[2].n;
      bc.alloc(c, es * n2);
      ec.alloc(c, es * n2);
      pr.alloc(c, es * n2);
      bc64.alloc(c, sizeof(double2) * n2);
      ec64.alloc(c, sizeof(double2) * n2);
    }
    if (!e1.V.p || e1.m != prm->int_m) {
      const int64_t n1 = h->op[1].n;
      e1.alloc(c, prm->int_m, n1, es, true);
      e1r.alloc(c, es * n1);
      e1x.alloc(c, es * n1);
      bh.alloc(c, es * n1);
    }
    const int pm = d ? d->m : 1;
    if (!proj.V.p || proj_m < pm) {
      proj.alloc(c, pm, h->op[2].n, es, false);
      proj_m = pm;
    }
    if (d && prm->coarse_persistent) {
      if (!xchg.p) xchg.alloc(c, 2 * es * h->op[2].n);  // two halves (halo form)
      if (!bflags.p) bflags.alloc(c, sizeof(unsigned) * coarse_proj_flag_words(256));
    }
    if (!d && !cg_y.p) cg_y.alloc(c, sizeof(double2) * h->op[2].n);
  }

  // GMRES(s) from x = 0 on level lvl: y = approximate A^{-1} v; r = v - A y from the
  // least-squares relation when requested (no extra matrix-vector product).  Two steps
  // (the paper's smoother) use the fused kernels: w1 = A v, w2 = A w1, one Gram reduction
  // with the 2 x 2 solve, one combination.  Other step counts run the Arnoldi kernels.
  void smooth(int lvl, const T* v, T* yout, T* rout) {
    KWS& ws = sm[lvl];
    KState* ks = ws.state();
    T* V = ws.V.as<T>();
    const int64_t n = ws.n;
    if (smooth_steps == 2) {
      op(lvl).apply(S(), v, V, 0, nullptr);
      op(lvl).apply(S(), V, V + n, 0, nullptr);
      w->cnt.mv[lvl] += 2;
      launch_smooth2<R>(S(), v, V, V + n, n, ks->y, yout, rout, PART(w), CNT(w));
      return;
    }
    launch_cycle_start<R>(S(), v, V, n, ks, -1.0, 1, PART(w), CNT(w));
    for (int j = 0; j < smooth_steps; ++j) {
      op(lvl).apply(S(), V + j * n, V + (j + 1) * n, 0, &ks->done);
      launch_arnoldi_orth<R>(S(), V, n, n, j, ks, PART(w), CNT(w));
      w->cnt.mv[lvl]++;
    }
    launch_ls_solve(S(), ks);
    launch_combine<R, R>(S(), yout, V, n, n, ks, 0, 0);
    if (rout) launch_combine<R, R>(S(), rout, V, n, n, ks, 1, 0);
  }

  // GMRES-Proj(m, k): projection over the deflation space, then GMRES(m - k) cycles.
  void gmres_proj(const T* b, T* x, double tol) {
    dmg_deflation* d = defl;
    const Op& A = op(2);
    const int64_t n = A.n;
    const int k = d->kk;
    const int mm = std::max(d->m - k, 1);
    const T* DV = dvec(d);
    const double2* DH = d->H.as<double2>();
    if (p->coarse_persistent) {
      if (!xchg.p) xchg.alloc(w->ctx, 2 * sizeof(T) * n);
      int* it_d = w->flags.as<int>() + 8;
      double* rr_d = (double*)(w->flags.as<int>() + 16);
      const T* Ab = (const T*)(sizeof(R) == sizeof(double) ? (const void*)A.A64 : (const void*)A.A32);
      if (!bflags.p) bflags.alloc(w->ctx, sizeof(unsigned) * coarse_proj_flag_words(256));
      int* err_d = w->flags.as<int>() + 9;  // read back together with the step count
      hipEvent_t ta = timer_mark(h->ctx, DMG_KT_COARSE_PROJ, S());
      if (launch_coarse_proj<R>(S(), Ab, A.Lx, A.Lt, DV, d->M.as<double2>(), d->Pi.as<double2>(), k, b, x, tol, mm,
                                p->coarse_max_iters,
                                xchg.as<T>(), PART(w), w->partials.bytes / sizeof(double2), it_d, rr_d,
                                bflags.as<unsigned>(), bflags.bytes / sizeof(unsigned), err_d, 0,
                                p->coarse_persistent == 1 ? 1 : 0)) {
        (void)err_d;  // step count and barrier status are read once per outer solve
        timer_span(h->ctx, DMG_KT_COARSE_PROJ, ta, timer_mark(h->ctx, DMG_KT_COARSE_PROJ, S()), 0);
        return;
      }
    }
    KState* ks = proj.state();
    T* V = proj.V.as<T>();
    T* rr = pr.as<T>();
    DMG_HIP(hipMemsetAsync(x, 0, sizeof(T) * n, S()));
    DMG_HIP(hipMemcpyAsync(rr, b, sizeof(T) * n, hipMemcpyDeviceToDevice, S()));
    launch_set_bnorm<R>(S(), n, b, ks, PART(w), CNT(w));
    int iters = 0;
    KStatus st{};
    for (;;) {
      launch_multidot<R>(S(), DV, n, k + 1, rr, n, ks->c, PART(w), CNT(w));
      launch_proj_solve(S(), DH, k, ks);
      launch_combine<R, R>(S(), x, DV, n, n, ks, 0, 1);
      launch_multi_axpy<R>(S(), rr, DV, n, k + 1, ks->u, n, 1.0);
      launch_cycle_start<R>(S(), rr, V, n, ks, tol, 0, PART(w), CNT(w));
      for (int j = 0; j < mm; ++j) {
        A.apply(S(), V + j * n, V + (j + 1) * n, 0, &ks->done);
        launch_arnoldi_orth<R>(S(), V, n, n, j, ks, PART(w), CNT(w));
      }
      launch_ls_solve(S(), ks);
      launch_combine<R, R>(S(), x, V, n, n, ks, 0, 1);
      launch_combine<R, R>(S(), rr, V, n, n, ks, 1, 0);
      sync_status(w, ks, &st);
      iters += st.steps;
      w->cnt.mv[2] += st.steps;
      if (st.est <= st.tol_abs || st.breakdown || iters >= p->coarse_max_iters) break;
    }
  }

  const T* dvec(dmg_deflation* d);

  void coarse_solve(const T* b, T* x) {
    w->cnt.coarse_calls++;
    if (!defl) {
      coarse_cgne(b, x);
      return;
    }
    if (!defl->ready) {
      const int64_t n = h->op[2].n;
      if constexpr (sizeof(R) == sizeof(double)) {
        coarse_gmres_dr(h, w, defl, (const double2*)b, (double2*)x, p->coarse_tol_first, p->coarse_max_iters, 2,
                        p->coarse_persistent);
      } else {
        launch_cast_f2d(S(), n, (const float2*)b, bc64.as<double2>());
        coarse_gmres_dr(h, w, defl, bc64.as<double2>(), ec64.as<double2>(), p->coarse_tol_first, p->coarse_max_iters, 2,
                        p->coarse_persistent);
        launch_cast_d2f(S(), n, ec64.as<double2>(), (float2*)x);
      }
      return;
    }
    if (big_deflation(defl->m, defl->k)) {
      // long cycles: GMRES-Proj in FP64 on the kernel-per-step path (also under an FP32 preconditioner)
      const int64_t n = h->op[2].n;
      double rel = 0.0;
      if constexpr (sizeof(R) == sizeof(double)) {
        big_gmres_proj(w, h->op[2], defl, (const double2*)b, (double2*)x, p->coarse_tol_later, p->coarse_max_iters,
                       &rel);
      } else {
        launch_cast_f2d(S(), n, (const float2*)b, bc64.as<double2>());
        big_gmres_proj(w, h->op[2], defl, bc64.as<double2>(), ec64.as<double2>(), p->coarse_tol_later,
                       p->coarse_max_iters, &rel);
        launch_cast_d2f(S(), n, ec64.as<double2>(), (float2*)x);
      }
      return;
    }
    double tol = p->coarse_tol_later;
    if (sizeof(R) == sizeof(float)) tol = std::max(tol, 1e-5);
    gmres_proj(b, x, tol);
  }

  // non-deflated comparison: CG on D_c D_c^dagger y = b, x = D_c^dagger y (FP64)
  void coarse_cgne(const T* b, T* x) {
    const int64_t n = h->op[2].n;
    const double2* b64;
    if constexpr (sizeof(R) == sizeof(double)) b64 = (const double2*)b;
    else {
      launch_cast_f2d(S(), n, (const float2*)b, bc64.as<double2>());
      b64 = bc64.as<double2>();
    }
    if (!cg_y.p) cg_y.alloc(w->ctx, sizeof(double2) * n);
    int it = 0;
    cg_normal(h, w, 2, 1, b64, cg_y.as<double2>(), p->coarse_tol_first, p->coarse_max_iters, &it);
    double2* x64 = (sizeof(R) == sizeof(double)) ? (double2*)x : ec64.as<double2>();
    op(2).apply(S(), cg_y.as<double2>(), x64, 1, nullptr);
    w->cnt.mv[2]++;
    if constexpr (sizeof(R) == sizeof(float)) launch_cast_d2f(S(), n, ec64.as<double2>(), (float2*)x);
  }

  // intermediate cycle M1: smooth, coarse correction, smooth
  void cycle1(const T* v, T* out) {
    const int64_t n = h->op[1].n;
    T* y1 = y[1].as<T>();
    T* r1 = r[1].as<T>();
    T* q = r2[1].as<T>();
    T* s1 = sv[1].as<T>();
    smooth(1, v, y1, r1);
    launch_restrict<R>(S(), Pm(1), r1, bc.as<T>(), h->tr[1].Lx, h->tr[1].Lt, NC);
    coarse_solve(bc.as<T>(), ec.as<T>());
    launch_prolong<R>(S(), Pm(1), ec.as<T>(), y1, h->tr[1].Lx, h->tr[1].Lt, NC, 1);
    op(1).apply(S(), y1, q, 0, nullptr, v);  // q = v - D_hat y1
    w->cnt.mv[1]++;
    smooth(1, q, s1, nullptr);
    launch_axpbyz<R>(S(), n, 1.0, y1, 1.0, s1, out);
  }

  // partial intermediate solve E1: FGMRES(int_m) on D_hat with M1 to int_tol ||b||
  void partial_solve(const T* b, T* x) {
    const Op& A = op(1);
    const int64_t n = A.n;
    KState* ks = e1.state();
    T* V = e1.V.as<T>();
    T* Z = e1.Z.as<T>();
    DMG_HIP(hipMemsetAsync(x, 0, sizeof(T) * n, S()));
    const T* rr = b;
    int iters = 0;
    bool first = true;
    KStatus st{};
    while (iters < p->int_max_iters) {
      launch_cycle_start<R>(S(), rr, V, n, ks, p->int_tol, first ? 1 : 0, PART(w), CNT(w));
      first = false;
      const int mm = std::min(e1.m, p->int_max_iters - iters);
      for (int j = 0; j < mm; ++j) {
        cycle1(V + j * n, Z + j * n);
        A.apply(S(), Z + j * n, V + (j + 1) * n, 0, nullptr);
        w->cnt.mv[1]++;
        launch_arnoldi_orth1<R>(S(), V, n, n, j, ks, PART(w), CNT(w));
        sync_status(w, ks, &st);
        if (st.pass2) {
          launch_arnoldi_pass2<R>(S(), V, n, n, j, ks, PART(w), CNT(w));
          sync_status(w, ks, &st);
        }
        if (st.done) break;
      }
      launch_ls_solve(S(), ks);
      launch_combine<R, R>(S(), x, Z, n, n, ks, 0, 1);
      iters += st.steps;
      if (st.est <= st.tol_abs || st.breakdown || iters >= p->int_max_iters) break;
      T* res = e1r.as<T>();
      A.apply(S(), x, res, 0, nullptr, b);
      w->cnt.mv[1]++;
      rr = res;
    }
  }

  // fine cycle M0: smooth, partial intermediate solve, smooth
  void cycle0(const T* v, T* out) {
    const int64_t n = h->op[0].n;
    T* y0 = y[0].as<T>();
    T* r0 = r[0].as<T>();
    T* q = r2[0].as<T>();
    T* s0 = sv[0].as<T>();
    smooth(0, v, y0, r0);
    launch_restrict<R>(S(), Pm(0), r0, bh.as<T>(), h->tr[0].Lx, h->tr[0].Lt, 2);
    if (p->int_mode == 1) cycle1(bh.as<T>(), e1x.as<T>());
    else partial_solve(bh.as<T>(), e1x.as<T>());
    launch_prolong<R>(S(), Pm(0), e1x.as<T>(), y0, h->tr[0].Lx, h->tr[0].Lt, 2, 1);
    op(0).apply(S(), y0, q, 0, nullptr, v);  // q = v - D y0
    w->cnt.mv[0]++;
    smooth(0, q, s0, nullptr);
    launch_axpbyz<R>(S(), n, 1.0, y0, 1.0, s0, out);
  }
};

template <>
const double2* Precond<double>::dvec(dmg_deflation* d) {
  return d->V64.as<double2>();
}
template <>
const float2* Precond<float>::dvec(dmg_deflation* d) {
  if (!d->cast_ready) {
    const int64_t n = h->op[2].n;
    d->V32.alloc(w->ctx, sizeof(float2) * (size_t)n * (d->kk + 1));
    launch_cast_d2f(S(), n * (d->kk + 1), d->V64.as<double2>(), d->V32.as<float2>());
    d->cast_ready = 1;
  }
  return d->V32.as<float2>();
}

// ---------------------------------------------------------------- outer FGMRES (FP64)
void prepare_work(dmg_hierarchy* h, Work* w, dmg_deflation* d, const dmg_solve_params* p) {
  DMG_CHECK(p->outer_m >= 1 && p->outer_m <= MMAX && p->int_m >= 1 && p->int_m <= MMAX && p->smooth_steps >= 1 &&
                p->smooth_steps <= MMAX,
            DMG_E_INVALID, "restart lengths must lie in [1, 64]");
  DMG_CHECK(!d || d->h == h, DMG_E_INVALID, "deflation space belongs to another hierarchy");
  const int64_t n = h->op[0].n;
  DMG_CHECK(p->precond == DMG_FP64 || p->precond == DMG_FP32 || p->precond == DMG_FP32_BF16 ||
                p->precond == DMG_FP32_BF16C,
            DMG_E_INVALID, "preconditioner precision");
  const bool fp32 = p->precond != DMG_FP64;
  if (!w->outer.V.p || w->outer.m != p->outer_m || w->outer.n != n) {
    w->outer.alloc(w->ctx, p->outer_m, n, sizeof(double2), true);
    w->or_.alloc(w->ctx, sizeof(double2) * n);
    w->bn2.alloc(w->ctx, sizeof(double) * 4);
    w->ov32.release();
    w->oz32.release();
  }
  if (fp32 && !w->ov32.p) {
    w->ov32.alloc(w->ctx, sizeof(float2) * n);
    w->oz32.alloc(w->ctx, sizeof(float2) * n);
  }
  // a preconditioner workspace serves any hierarchy with the same level sizes
  auto same = [&](const dmg_hierarchy* o) {
    for (int l = 0; l < 3; ++l)
      if (o->op[l].n != h->op[l].n || o->op[l].Lx != h->op[l].Lx) return false;
    return true;
  };
  if (fp32) {
    if (w->pc32 && w->pc32->h != h && !same(w->pc32->h)) w->pc32.reset();
    if (!w->pc32) w->pc32.reset(new Precond<float>(h, w));
    w->pc32->h = h;
    w->pc32->ensure(p, d);
  } else {
    if (w->pc64 && w->pc64->h != h && !same(w->pc64->h)) w->pc64.reset();
    if (!w->pc64) w->pc64.reset(new Precond<double>(h, w));
    w->pc64->h = h;
    w->pc64->ensure(p, d);
  }
  if (d && d->m != w->dr_m) {
    // GMRES-DR workspace, used when this solve builds the deflation space
    ensure_dr(h, w, d->m, d->k);
  }
}

void prepare_deflation_fp32(Work* w, dmg_deflation* d) {
  if (!d || !d->ready || d->cast_ready) return;
  const int64_t n = d->h->op[2].n;
  d->V32.alloc(w->ctx, sizeof(float2) * (size_t)n * (d->kk + 1));
  launch_cast_d2f(w->stream, n * (d->kk + 1), d->V64.as<double2>(), d->V32.as<float2>());
  DMG_HIP(hipStreamSynchronize(w->stream));
  d->cast_ready = 1;
}

void outer_begin(dmg_hierarchy* h, Work* w, dmg_deflation* d, const dmg_solve_params* p, const double2* b,
                 double2* x) {
  Work::Run& R = w->run;
  R = Work::Run{};
  R.t0 = std::chrono::steady_clock::now();
  R.h = h;
  R.d = d;
  R.p = *p;
  R.b = b;
  R.x = x;
  prepare_work(h, w, d, &R.p);
  hipStream_t s = w->stream;
  w->cnt = Counters{};
  // device accumulators of the persistent coarse solves: [8] Arnoldi steps, [9] barrier timeout
  DMG_HIP(hipMemsetAsync(w->flags.as<int>() + 8, 0, 2 * sizeof(int), s));
  const Op& A = h->op[0];
  const int64_t n = A.n;
  KState* ks = w->outer.state();
  double2* r = w->or_.as<double2>();
  double* scal = w->bn2.as<double>();
  if (R.p.use_x0) {
    A.apply(s, x, r, 0, nullptr);
    w->cnt.mv[0]++;
    launch_xmy<double>(s, n, b, r);
  } else {
    DMG_HIP(hipMemsetAsync(x, 0, sizeof(double2) * n, s));
    DMG_HIP(hipMemcpyAsync(r, b, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
  }
  launch_norm2<double>(s, n, b, scal, PART(w), CNT(w));
  launch_set_bnorm<double>(s, n, b, ks, PART(w), CNT(w));
  R.bnorm = std::sqrt(read_double(w, scal));
  if (R.bnorm == 0.0) {
    DMG_HIP(hipMemsetAsync(x, 0, sizeof(double2) * n, s));
    R.conv = true;
    R.done = true;
    return;
  }
  // initial residual check (x0 given)
  launch_norm2<double>(s, n, r, scal, PART(w), CNT(w));
  R.rel = std::sqrt(read_double(w, scal)) / R.bnorm;
  R.conv = R.rel <= R.p.tol;
  R.done = R.conv;
}

bool outer_advance(Work* w, int min_iters) {
  Work::Run& R = w->run;
  if (R.done) return true;
  dmg_hierarchy* h = R.h;
  const dmg_solve_params* p = &R.p;
  hipStream_t s = w->stream;
  const Op& A = h->op[0];
  const int64_t n = A.n;
  const bool fp32 = p->precond != DMG_FP64;
  if (fp32) w->pc32->ensure(p, R.d);
  else w->pc64->ensure(p, R.d);
  KState* ks = w->outer.state();
  double2* V = w->outer.V.as<double2>();
  double2* Z = w->outer.Z.as<double2>();
  double2* r = w->or_.as<double2>();
  double* scal = w->bn2.as<double>();
  double2* x = R.x;
  const int start = R.iters;
  KStatus st{};
  while (!R.conv && R.iters < p->max_outer_iters && R.iters - start < min_iters) {
    launch_cycle_start<double>(s, r, V, n, ks, p->tol, 0, PART(w), CNT(w));
    const int mm = std::min(p->outer_m, p->max_outer_iters - R.iters);
    for (int j = 0; j < mm; ++j) {
      double2* vj = V + (int64_t)j * n;
      double2* zj = Z + (int64_t)j * n;
      if (fp32) {
        launch_cast_d2f(s, n, vj, w->ov32.as<float2>());
        w->pc32->cycle0(w->ov32.as<float2>(), w->oz32.as<float2>());
        launch_cast_f2d(s, n, w->oz32.as<float2>(), zj);
      } else {
        w->pc64->cycle0(vj, zj);
      }
      A.apply(s, zj, V + (int64_t)(j + 1) * n, 0, nullptr);
      w->cnt.mv[0]++;
      launch_arnoldi_orth1<double>(s, V, n, n, j, ks, PART(w), CNT(w));
      sync_status(w, ks, &st);
      if (st.pass2) {
        launch_arnoldi_pass2<double>(s, V, n, n, j, ks, PART(w), CNT(w));
        sync_status(w, ks, &st);
      }
      if (st.done) break;
    }
    launch_ls_solve(s, ks);
    launch_combine<double, double>(s, x, Z, n, n, ks, 0, 1);
    R.iters += st.steps;
    // true residual r = b - D x
    A.apply(s, x, r, 0, nullptr, R.b);
    w->cnt.mv[0]++;
    launch_norm2<double>(s, n, r, scal, PART(w), CNT(w));
    R.rel = std::sqrt(read_double(w, scal)) / R.bnorm;
    R.conv = R.rel <= p->tol;
    if (st.steps == 0) {
      R.done = true;
      break;
    }
  }
  if (R.conv || R.iters >= p->max_outer_iters) R.done = true;
  return R.done;
}

dmg_status outer_finish(Work* w, dmg_solve_stats* stout) {
  Work::Run& R = w->run;
  dmg_hierarchy* h = R.h;
  hipStream_t s = w->stream;
  DMG_HIP(hipMemcpyAsync(w->host_status, w->flags.as<int>() + 8, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  {
    const int* hs = (const int*)w->host_status;
    DMG_CHECK(hs[1] == 0, DMG_E_HIP, "persistent coarse solve: a grid-barrier wait timed out");
    w->cnt.mv[2] += hs[0];
    if (h->ctx->timing & (1 << DMG_KT_COARSE_PROJ)) {
      std::lock_guard<std::mutex> lk(h->ctx->mu);
      h->ctx->pending_units[DMG_KT_COARSE_PROJ] += hs[0];
    }
  }
  if (stout) {
    dmg_solve_stats& o = *stout;
    o.outer_iters = R.iters;
    o.converged = R.conv ? 1 : 0;
    o.fine_mvps = w->cnt.mv[0];
    o.int_mvps = w->cnt.mv[1];
    o.coarse_mvps = w->cnt.mv[2];
    const double n0 = (double)h->op[0].n, n1 = (double)h->op[1].n, n2 = (double)h->op[2].n;
    o.fine_equiv_mvps = w->cnt.mv[0] + n1 / n0 * w->cnt.mv[1] + n2 / n0 * w->cnt.mv[2];
    o.true_rel_resid = R.rel;
    o.coarse_calls = w->cnt.coarse_calls;
    o.coarse_dr_calls = w->cnt.dr_calls;
    o.elapsed_ms = std::chrono::duration<double, std::milli>(t1 - R.t0).count();
  }
  return R.conv ? DMG_OK : DMG_W_NOT_CONVERGED;
}

// ---------------------------------------------------------------- fine-grid comparison solvers
dmg_status fine_solve(dmg_hierarchy* h, int method, int m, int k, double tol, int max_iters, const double2* b,
                      double2* x, int nrhs, dmg_solve_stats* stout) {
  Work* w = &h->main;
  hipStream_t s = w->stream;
  const Op& A = h->op[0];
  const int64_t n = A.n;
  std::vector<dmg_solve_stats> st(nrhs);
  bool all = true;
  if (method == DMG_FINE_CGNE) {
    auto t0 = std::chrono::steady_clock::now();
    DevBuf y;
    y.alloc(h->ctx, sizeof(double2) * n * nrhs);
    std::vector<int> its(nrhs, 0);
    w->cnt = Counters{};
    cg_normal(h, w, 0, nrhs, b, y.as<double2>(), tol, max_iters, its.data());
    for (int f = 0; f < nrhs; ++f) A.apply(s, y.as<double2>() + f * n, x + f * n, 1, nullptr);
    DevBuf rn, dy, scal;
    rn.alloc(h->ctx, sizeof(double2) * n);
    scal.alloc(h->ctx, sizeof(double) * 2);
    auto t1 = std::chrono::steady_clock::now();
    for (int f = 0; f < nrhs; ++f) {
      double2* yf = y.as<double2>() + f * n;
      double2* xf = x + f * n;
      double v[2];
      auto true_residual = [&]() {  // rn = b - D x, v = (||rn||^2, ||b||^2)
        A.apply(s, xf, rn.as<double2>(), 0, nullptr, b + f * n);
        launch_norm2<double>(s, n, rn.as<double2>(), scal.as<double>(), PART(w), CNT(w));
        launch_norm2<double>(s, n, b + f * n, scal.as<double>() + 1, PART(w), CNT(w));
        DMG_HIP(hipMemcpyAsync(v, scal.p, sizeof(v), hipMemcpyDeviceToHost, s));
        DMG_HIP(hipStreamSynchronize(s));
      };
      true_residual();
      // Near the critical mass the recursively updated residual of CG on D D^dagger drifts from
      // the true one (by about 1e-8 relative at a mass gap of 1e-4): while the true residual is
      // above tol, CG is restarted on D D^dagger dy = b - D x from dy = 0 and y += dy.
      int passes = 0;
      while (passes < 8 && its[f] < max_iters && v[1] > 0.0 && std::sqrt(v[0] / v[1]) > tol) {
        if (!dy.p) dy.alloc(h->ctx, sizeof(double2) * n);
        const double tol_r = 0.9 * tol * std::sqrt(v[1] / v[0]);  // relative to ||b - D x||
        int it = 0;
        cg_normal(h, w, 0, 1, rn.as<double2>(), dy.as<double2>(), tol_r, max_iters - its[f], &it);
        its[f] += it;
        launch_axpby<double>(s, n, 1.0, dy.as<double2>(), 1.0, yf);
        A.apply(s, yf, xf, 1, nullptr);
        ++passes;
        true_residual();
      }
      dmg_solve_stats& o = st[f];
      o = dmg_solve_stats{};
      o.outer_iters = its[f];
      o.fine_mvps = 2LL * its[f] + 1 + 2LL * passes;
      o.fine_equiv_mvps = (double)o.fine_mvps;
      o.true_rel_resid = v[1] > 0.0 ? std::sqrt(v[0] / v[1]) : 0.0;
      o.converged = o.true_rel_resid <= tol * (1.0 + 1e-6) ? 1 : 0;
      o.elapsed_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
      all = all && o.converged;
    }
  } else {
    // GMRES-DR(m, k) with a fresh space per right-hand side, or (DMG_FINE_GMRES_PROJ) GMRES-DR on the
    // first right-hand side and GMRES-Proj(m, k) over its space on every later one
    DMG_CHECK(m >= 2 && m <= MBIG && k >= 1 && k < m && k <= KBIG, DMG_E_INVALID, "fine GMRES-DR sizes");
    const bool proj = method == DMG_FINE_GMRES_PROJ;
    const bool big = proj || big_deflation(m, k);
    dmg_deflation d;
    d.h = h;
    d.m = m;
    d.k = k;
    DevBuf rn, scal;
    rn.alloc(h->ctx, sizeof(double2) * n);
    scal.alloc(h->ctx, sizeof(double) * 2);
    for (int f = 0; f < nrhs; ++f) {
      auto t0 = std::chrono::steady_clock::now();
      w->cnt = Counters{};
      int it;
      const bool first = !proj || f == 0;
      if (!big) it = coarse_gmres_dr(h, w, &d, b + f * n, x + f * n, tol, max_iters, 0);
      else if (first) it = big_gmres_dr(h->ctx, w, A, m, k, b + f * n, x + f * n, tol, max_iters, proj ? &d : nullptr);
      else it = big_gmres_proj(w, A, &d, b + f * n, x + f * n, tol, max_iters, nullptr);
      A.apply(s, x + f * n, rn.as<double2>(), 0, nullptr, b + f * n);
      launch_norm2<double>(s, n, rn.as<double2>(), scal.as<double>(), PART(w), CNT(w));
      launch_norm2<double>(s, n, b + f * n, scal.as<double>() + 1, PART(w), CNT(w));
      double v[2];
      DMG_HIP(hipMemcpyAsync(v, scal.p, sizeof(v), hipMemcpyDeviceToHost, s));
      DMG_HIP(hipStreamSynchronize(s));
      auto t1 = std::chrono::steady_clock::now();
      dmg_solve_stats& o = st[f];
      o = dmg_solve_stats{};
      o.outer_iters = it;
      o.fine_mvps = it;
      o.fine_equiv_mvps = (double)it;
      o.true_rel_resid = v[1] > 0.0 ? std::sqrt(v[0] / v[1]) : 0.0;
      o.converged = o.true_rel_resid <= tol * (1.0 + 1e-6) ? 1 : 0;
      o.coarse_dr_calls = first ? 1 : 0;
      o.elapsed_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
      all = all && o.converged;
    }
  }
  if (stout)
    for (int f = 0; f < nrhs; ++f) stout[f] = st[f];
  return all ? DMG_OK : DMG_W_NOT_CONVERGED;
}

dmg_status outer_solve(dmg_hierarchy* h, Work* w, dmg_deflation* d, const dmg_solve_params* p, const double2* b,
                       double2* x, dmg_solve_stats* stout) {
  outer_begin(h, w, d, p, b, x);
  outer_advance(w, std::numeric_limits<int>::max());
  return outer_finish(w, stout);
}

}  // namespace dmg

dmg_hierarchy::dmg_hierarchy() = default;
dmg_hierarchy::~dmg_hierarchy() { dmg::destroy_bwork(bwork); }
