// Lockstep multi-right-hand-side solve: the method of the single-field solver (outer
// FGMRES with the three-grid cycle, partial intermediate solve, GMRES-Proj coarse
// solves over a shared deflation space) applied to nb right-hand sides at once.
// Every right-hand side keeps its own Krylov state and stopping decisions; each
// launch processes all of them, so a matrix entry is read once per launch for the
// whole batch and the launch latency of the small coarse grid is shared.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <memory>
#include <vector>

#include "mrhs.h"
#include "solver.h"

namespace dmg {

// Krylov basis of one level for nb right-hand sides: V (m + 1 batched fields), Z (m
// fields when flexible), per right-hand-side state, and device flags (0: all done, as
// read by the host; 1: an Arnoldi step needs a second pass).
struct BKry {
  int m = 0;
  int64_t n = 0;
  DevBuf V, Z, bs, flag;
  void alloc(dmg_context* c, hipStream_t s, int m_, int64_t n_, int nb, size_t es, bool flexible) {
    m = m_;
    n = n_;
    const size_t fb = es * (size_t)n * nb;
    V.alloc(c, fb * (m + 1));
    DMG_HIP(hipMemsetAsync(V.p, 0, V.bytes, s));
    if (flexible) {
      Z.alloc(c, fb * m);
      DMG_HIP(hipMemsetAsync(Z.p, 0, Z.bytes, s));
    }
    bs.alloc(c, sizeof(BS) * nb);
    DMG_HIP(hipMemsetAsync(bs.p, 0, bs.bytes, s));
    flag.alloc(c, sizeof(int) * 4);
    DMG_HIP(hipMemsetAsync(flag.p, 0, flag.bytes, s));
  }
  BS* st() const { return bs.as<BS>(); }
  int* flags() const { return flag.as<int>(); }
  int* anyp2() const { return flag.as<int>() + 1; }
};

// Shared scratch of one batched solve.
struct BShared {
  dmg_context* ctx = nullptr;
  hipStream_t s = nullptr;
  int nb = 0;
  DevBuf part, coef;
  BSTail* tail = nullptr;  // pinned, nb entries
  int* hflag = nullptr;    // pinned
  ~BShared() {
    if (tail) (void)hipHostFree(tail);
    if (hflag) (void)hipHostFree(hflag);
  }
  void init(dmg_context* c, hipStream_t st, int nb_) {
    ctx = c;
    s = st;
    nb = nb_;
    part.alloc(c, sizeof(double2) * bred_partials(nb));
    coef.alloc(c, sizeof(double2) * 2 * NBMAX);
    DMG_HIP(hipHostMalloc((void**)&tail, sizeof(BSTail) * NBMAX, hipHostMallocDefault));
    DMG_HIP(hipHostMalloc((void**)&hflag, sizeof(int) * 4, hipHostMallocDefault));
  }
  double2* P() const { return part.as<double2>(); }
  // tails of all right-hand sides of a state array (synchronises the stream)
  void read_tails(const BS* bs) {
    DMG_HIP(hipMemcpy2DAsync(tail, sizeof(BSTail), (const char*)bs + offsetof(BS, beta), sizeof(BS), sizeof(BSTail),
                             nb, hipMemcpyDeviceToHost, s));
    DMG_HIP(hipStreamSynchronize(s));
  }
  // every right-hand side of bs is done (flag: a device int; synchronises the stream)
  bool all_done(const BS* bs, int* flag) {
    launch_b_all_done(s, bs, nb, flag);
    DMG_HIP(hipMemcpyAsync(hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    DMG_HIP(hipStreamSynchronize(s));
    return hflag[0] != 0;
  }
  void set_state(BS* bs, const std::vector<int>& act, const std::vector<int>& cap) {
    std::vector<int> st(2 * nb);
    for (int r = 0; r < nb; ++r) {
      st[2 * r] = act[r];
      st[2 * r + 1] = cap[r];
    }
    launch_b_set_state(s, bs, st.data(), nb);
  }
};

static_assert(offsetof(BS, pass2) - offsetof(BS, beta) + sizeof(int) == sizeof(BSTail), "BS tail layout");

// The three-grid preconditioner on batched fields in precision R.
template <typename R>
struct BPre {
  using T = cx<R>;
  dmg_hierarchy* h = nullptr;
  dmg_deflation* d = nullptr;
  const dmg_solve_params* p = nullptr;
  BShared* sh = nullptr;
  int nb = 0;
  DevBuf smw[2], y[2], r[2], q[2], sv[2];
  BKry e1;
  DevBuf e1r, e1x, bh;
  DevBuf bc, ec, pr;
  BKry proj;
  long long mv[3] = {0, 0, 0};

  // One GMRES-Proj cycle of the coarse solve replayed as a captured HIP graph (its ~190
  // kernels have no host decision inside; their arguments are baked in and keyed below).
  hipStream_t cap_s = nullptr;  // capture stream (capture needs a stream other than the null stream)
  hipStream_t cur = nullptr;    // set while capturing
  hipGraphExec_t cyc = nullptr;
  const void* cyc_key[6] = {};
  double cyc_tol = 0.0;
  int cyc_k = -1, cyc_m = -1;

  ~BPre() {
    if (cyc) (void)hipGraphExecDestroy(cyc);
    if (cap_s) (void)hipStreamDestroy(cap_s);
  }
  hipStream_t S() const { return cur ? cur : sh->s; }
  // FP32 with the BF16-stored intermediate operator
  bool bf16() const { return sizeof(R) == sizeof(float) && p->precond == DMG_FP32_BF16; }
  int64_t N(int l) const { return h->op[l].n; }
  const T* Pm(int l) const { return (const T*)h->tr[l].P((const T*)nullptr); }

  void alloc(dmg_hierarchy* hh, dmg_deflation* dd, const dmg_solve_params* pp, BShared* s, int nb_) {
    h = hh;
    d = dd;
    p = pp;
    sh = s;
    nb = nb_;
    dmg_context* c = h->ctx;
    const size_t es = sizeof(T);
    auto field = [&](DevBuf& b, int l, int count) {
      b.alloc(c, es * (size_t)N(l) * nb * count);
      DMG_HIP(hipMemsetAsync(b.p, 0, b.bytes, S()));
    };
    for (int l = 0; l < 2; ++l) {
      field(smw[l], l, 2);
      field(y[l], l, 1);
      field(r[l], l, 1);
      field(q[l], l, 1);
      field(sv[l], l, 1);
    }
    e1.alloc(c, S(), p->int_m, N(1), nb, es, true);
    field(e1r, 1, 1);
    field(e1x, 1, 1);
    field(bh, 1, 1);
    field(bc, 2, 1);
    field(ec, 2, 1);
    field(pr, 2, 1);
    proj.alloc(c, S(), std::max(d->m - d->kk, 1), N(2), nb, es, false);
    // launch forms of this lane count's stencils, timed once per shape on the (zeroed) scratch fields
    const bool f64 = sizeof(R) == sizeof(double);
    const Op& A0 = h->op[0];
    const T* U = (const T*)(f64 ? (const void*)A0.U64 : (const void*)A0.U32);
    b_tune_wilson<R>(S(), U, smw[0].as<T>(), smw[0].as<T>() + N(0) * nb, A0.m0, A0.Lx, A0.Lt, nb);
    for (int l = 1; l < 3; ++l) {
      const Op& A = h->op[l];
      const T* Ab = (const T*)(f64 ? (const void*)A.A64 : (const void*)A.A32);
      if (l == 1 && bf16())
        b_tune_block_bf16(S(), h->A16.as<bf16c>(), (const float2*)smw[1].as<T>(), (float2*)(smw[1].as<T>() + N(1) * nb),
                          A.Lx, A.Lt, nb);
      else if (l == 1) b_tune_block<R>(S(), Ab, smw[1].as<T>(), smw[1].as<T>() + N(1) * nb, A.Lx, A.Lt, nb);
      else b_tune_block<R>(S(), Ab, bc.as<T>(), ec.as<T>(), A.Lx, A.Lt, nb);
    }
  }

  void apply(int l, const T* in, T* out, const T* sub, const BS* skip) {
    const Op& A = h->op[l];
    dmg_context* c = h->ctx;
    const int kt = A.kind == 0 ? DMG_KT_WILSON_BATCHED : DMG_KT_BLOCK_BATCHED;
    hipEvent_t ta = timer_mark(c, kt, S());
    if (A.kind == 0) {
      const T* U = (const T*)(sizeof(R) == sizeof(double) ? (const void*)A.U64 : (const void*)A.U32);
      launch_b_wilson<R>(S(), U, in, out, A.m0, A.Lx, A.Lt, nb, sub, skip);
    } else if (l == 1 && bf16()) {
      launch_b_block_bf16(S(), h->A16.as<bf16c>(), (const float2*)in, (float2*)out, A.Lx, A.Lt, nb,
                          (const float2*)sub, skip);
    } else {
      const T* Ab = (const T*)(sizeof(R) == sizeof(double) ? (const void*)A.A64 : (const void*)A.A32);
      launch_b_block<R>(S(), Ab, in, out, A.Lx, A.Lt, nb, sub, skip);
    }
    if (ta) timer_span(c, kt, ta, timer_mark(c, kt, S()), (long long)A.Lx * A.Lt * nb);
  }

  // two-step GMRES smoother from 0 (fused form): y = approximate A^{-1} v, r = v - A y
  void smooth(int l, const T* v, T* yout, T* rout) {
    T* w1 = smw[l].as<T>();
    T* w2 = w1 + N(l) * nb;
    apply(l, v, w1, nullptr, nullptr);
    apply(l, w1, w2, nullptr, nullptr);
    mv[l] += 2;
    launch_b_smooth2<R>(S(), v, w1, w2, N(l), nb, sh->coef.as<double2>(), yout, rout, sh->P());
  }

  const T* dvec() const {
    return (const T*)(sizeof(R) == sizeof(double) ? (const void*)d->V64.p : (const void*)d->V32.p);
  }

  // projection over the deflation space, then one GMRES(m - k) cycle, for every active lane
  void coarse_cycle_kernels(T* x, T* rr, double tol) {
    const int64_t n = N(2);
    const int k = d->kk, mm = proj.m;
    T* V = proj.V.as<T>();
    const int64_t ld = n * nb;
    BS* bs = proj.st();
    launch_b_project<R>(S(), dvec(), k, d->M.as<double2>(), d->Pi.as<double2>(), x, rr, n, nb, bs, sh->P());
    launch_b_norm<R>(S(), rr, n, nb, bs, tol, 1, nullptr, sh->P());
    launch_b_scale_beta<R>(S(), rr, V, n, nb, bs);
    for (int j = 0; j < mm; ++j) {
      apply(2, V + j * ld, V + (j + 1) * ld, nullptr, bs);
      launch_b_arnoldi<R>(S(), V, ld, n, nb, j, bs, proj.anyp2(), sh->P());
    }
    launch_b_ls_solve(S(), bs, nb);
    launch_b_combine<R>(S(), x, V, ld, n, nb, bs, 0, 1);
    launch_b_combine<R>(S(), rr, V, ld, n, nb, bs, 1, 0);
  }

  void coarse_cycle(T* x, T* rr, double tol) {
    const int timed = (1 << DMG_KT_BLOCK_BATCHED) | (1 << DMG_KT_WILSON_BATCHED);
    if (!p->graphs || (h->ctx->timing & timed)) {
      coarse_cycle_kernels(x, rr, tol);
      return;
    }
    const void* key[6] = {x, rr, proj.V.p, dvec(), d->M.p, d->Pi.p};
    bool same = cyc && cyc_tol == tol && cyc_k == d->kk && cyc_m == proj.m;
    for (int i = 0; i < 6; ++i) same = same && key[i] == cyc_key[i];
    if (!same) {
      if (cyc) {
        DMG_HIP(hipGraphExecDestroy(cyc));
        cyc = nullptr;
      }
      if (!cap_s) DMG_HIP(hipStreamCreateWithFlags(&cap_s, hipStreamNonBlocking));
      DMG_HIP(hipStreamBeginCapture(cap_s, hipStreamCaptureModeThreadLocal));
      cur = cap_s;
      hipGraph_t g = nullptr;
      try {
        coarse_cycle_kernels(x, rr, tol);
      } catch (...) {
        cur = nullptr;
        (void)hipStreamEndCapture(cap_s, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      cur = nullptr;
      DMG_HIP(hipStreamEndCapture(cap_s, &g));
      const hipError_t e = hipGraphInstantiate(&cyc, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      DMG_HIP(e);
      for (int i = 0; i < 6; ++i) cyc_key[i] = key[i];
      cyc_tol = tol;
      cyc_k = d->kk;
      cyc_m = proj.m;
    }
    DMG_HIP(hipGraphLaunch(cyc, sh->s));
  }

  // GMRES-Proj(m, k) from x = 0 on the coarse grid, one stopping decision per right-hand side
  void coarse_solve(const T* b, T* x) {
    const int64_t n = N(2);
    const int mm = proj.m;
    double tol = p->coarse_tol_later;
    if (sizeof(R) == sizeof(float)) tol = std::max(tol, 1e-5);
    T* rr = pr.as<T>();
    const int64_t ld = n * nb;
    BS* bs = proj.st();
    DMG_HIP(hipMemsetAsync(x, 0, sizeof(T) * ld, S()));
    DMG_HIP(hipMemcpyAsync(rr, b, sizeof(T) * ld, hipMemcpyDeviceToDevice, S()));
    std::vector<int> act(nb, 1), cap(nb, mm), it(nb, 0);
    sh->set_state(bs, act, cap);
    launch_b_norm<R>(S(), b, n, nb, bs, 0.0, 3, nullptr, sh->P());
    for (;;) {
      coarse_cycle(x, rr, tol);
      sh->read_tails(bs);
      int most = 0;
      bool any = false;
      for (int r = 0; r < nb; ++r) {
        const BSTail& t = sh->tail[r];
        if (!act[r]) continue;
        it[r] += t.steps;
        most = std::max(most, t.steps);
        const bool stop = t.est <= t.tol_abs || t.brk || it[r] >= p->coarse_max_iters || t.steps == 0;
        act[r] = stop ? 0 : 1;
        any = any || !stop;
      }
      mv[2] += most;
      if (!any) break;
      sh->set_state(bs, act, cap);
    }
  }

  // intermediate cycle M1: smooth, coarse correction, smooth
  void cycle1(const T* v, T* out) {
    const int64_t n = N(1);
    T* y1 = y[1].as<T>();
    T* r1 = r[1].as<T>();
    T* q1 = q[1].as<T>();
    T* s1 = sv[1].as<T>();
    smooth(1, v, y1, r1);
    launch_b_restrict<R>(S(), Pm(1), r1, bc.as<T>(), h->tr[1].Lx, h->tr[1].Lt, NC, nb);
    coarse_solve(bc.as<T>(), ec.as<T>());
    launch_b_prolong<R>(S(), Pm(1), ec.as<T>(), y1, h->tr[1].Lx, h->tr[1].Lt, NC, nb, 1);
    apply(1, y1, q1, v, nullptr);  // q = v - D_hat y1
    mv[1]++;
    smooth(1, q1, s1, nullptr);
    launch_axpbyz<R>(S(), n * nb, 1.0, y1, 1.0, s1, out);
  }

  // partial intermediate solve: FGMRES(int_m) on D_hat with M1 to int_tol ||b|| (per RHS)
  void partial_solve(const T* b, T* x) {
    const int64_t n = N(1);
    const int64_t ld = n * nb;
    BS* bs = e1.st();
    T* V = e1.V.as<T>();
    T* Z = e1.Z.as<T>();
    DMG_HIP(hipMemsetAsync(x, 0, sizeof(T) * ld, S()));
    const T* rr = b;
    std::vector<int> act(nb, 1), cap(nb, std::min(e1.m, p->int_max_iters)), it(nb, 0);
    bool first = true;
    for (;;) {
      sh->set_state(bs, act, cap);
      launch_b_norm<R>(S(), rr, n, nb, bs, p->int_tol, first ? 2 : 1, nullptr, sh->P());
      launch_b_scale_beta<R>(S(), rr, V, n, nb, bs);
      first = false;
      int jmax = 0;
      for (int r = 0; r < nb; ++r)
        if (act[r]) jmax = std::max(jmax, cap[r]);
      for (int j = 0; j < jmax; ++j) {
        cycle1(V + j * ld, Z + j * ld);
        apply(1, Z + j * ld, V + (j + 1) * ld, nullptr, bs);
        mv[1]++;
        launch_b_arnoldi<R>(S(), V, ld, n, nb, j, bs, e1.anyp2(), sh->P());
        if (sh->all_done(bs, e1.flags())) break;
      }
      launch_b_ls_solve(S(), bs, nb);
      launch_b_combine<R>(S(), x, Z, ld, n, nb, bs, 0, 1);
      sh->read_tails(bs);
      bool any = false;
      for (int r = 0; r < nb; ++r) {
        const BSTail& t = sh->tail[r];
        if (!act[r]) continue;
        it[r] += t.steps;
        const bool stop = t.est <= t.tol_abs || t.brk || it[r] >= p->int_max_iters;
        act[r] = stop ? 0 : 1;
        cap[r] = std::min(e1.m, p->int_max_iters - it[r]);
        any = any || !stop;
      }
      if (!any) break;
      T* res = e1r.as<T>();
      apply(1, x, res, b, nullptr);
      mv[1]++;
      rr = res;
    }
  }

  // fine cycle M0: smooth, partial intermediate solve, smooth
  void cycle0(const T* v, T* out) {
    const int64_t n = N(0);
    T* y0 = y[0].as<T>();
    T* r0 = r[0].as<T>();
    T* q0 = q[0].as<T>();
    T* s0 = sv[0].as<T>();
    smooth(0, v, y0, r0);
    launch_b_restrict<R>(S(), Pm(0), r0, bh.as<T>(), h->tr[0].Lx, h->tr[0].Lt, 2, nb);
    partial_solve(bh.as<T>(), e1x.as<T>());
    launch_b_prolong<R>(S(), Pm(0), e1x.as<T>(), y0, h->tr[0].Lx, h->tr[0].Lt, 2, nb, 1);
    apply(0, y0, q0, v, nullptr);  // q = v - D y0
    mv[0]++;
    smooth(0, q0, s0, nullptr);
    launch_axpbyz<R>(S(), n * nb, 1.0, y0, 1.0, s0, out);
  }
};

// Lane engine: nb interleaved right-hand sides ("lanes") advanced by lockstep outer
// FGMRES cycles.  A lane joins between cycles (its x starts at 0, its residual at b)
// and leaves when it converged or reached its iteration cap; a lane's arithmetic
// depends only on its own data and on nb, never on the other lanes.
struct BWork {
  dmg_hierarchy* h = nullptr;
  int nb = 0, outer_m = 0, int_m = 0, precond = -1, dm = 0, dk = 0;
  const dmg_deflation* d = nullptr;
  dmg_solve_params p{};
  BShared sh;
  BKry outer;
  DevBuf B, X, Rr, v32, z32, rn;
  BPre<double> pc64;
  BPre<float> pc32;
  // per-lane host state
  std::vector<int> act, it, conv;
  std::vector<double> rel, bn;
  std::vector<long long> mvr;
  std::vector<std::chrono::steady_clock::time_point> t_in;
  long long mv_prev[3] = {0, 0, 0};
  // a lane batch (dmg_batch_*) runs on a stream of its own, ordered against the context's
  // stream by `ev` where caller buffers are read or written
  hipStream_t own = nullptr;
  hipEvent_t ev = nullptr;

  ~BWork() {  // the members' buffers are released after this body: the own stream is idle by then
    if (own) {
      (void)hipStreamSynchronize(own);
      (void)hipStreamDestroy(own);
    }
    if (ev) (void)hipEventDestroy(ev);
  }
  void init(dmg_hierarchy* hh, dmg_deflation* dd, const dmg_solve_params* pp, int nb_, bool own_stream);
  // the own stream waits for the work queued so far on the context's stream (device memory
  // from the context's allocator and caller buffers are ordered on that stream)
  void order_after_ctx() {
    if (!own) return;
    DMG_HIP(hipEventRecord(ev, h->ctx->stream));
    DMG_HIP(hipStreamWaitEvent(own, ev, 0));
  }
  void reset_lanes();
  void start_lanes(const std::vector<int>& lanes);  // B lanes hold the right-hand sides
  void cycle();                                     // one outer cycle of every active lane
  bool any_active() const {
    for (int r = 0; r < nb; ++r)
      if (act[r]) return true;
    return false;
  }
  void stats(int r, dmg_solve_stats* o, std::chrono::steady_clock::time_point now) const;
};

void destroy_bwork(BWork* b) {
  if (b && b->sh.s) (void)hipStreamSynchronize(b->sh.s);
  delete b;
}

void BWork::init(dmg_hierarchy* hh, dmg_deflation* dd, const dmg_solve_params* pp, int nb_, bool own_stream) {
  h = hh;
  d = dd;
  p = *pp;
  nb = nb_;
  outer_m = p.outer_m;
  int_m = p.int_m;
  precond = p.precond;
  dm = dd->m;
  dk = dd->kk;
  dmg_context* c = h->ctx;
  if (own_stream) {
    DMG_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    DMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  hipStream_t s = own ? own : c->stream;
  if (own) order_after_ctx();
  sh.init(c, s, nb);
  const int64_t n0 = h->op[0].n;
  const size_t fb = sizeof(double2) * (size_t)n0 * nb;
  outer.alloc(c, s, p.outer_m, n0, nb, sizeof(double2), true);
  B.alloc(c, fb);
  X.alloc(c, fb);
  Rr.alloc(c, fb);
  for (DevBuf* b : {&B, &X, &Rr}) DMG_HIP(hipMemsetAsync(b->p, 0, b->bytes, s));
  rn.alloc(c, sizeof(double) * NBMAX);
  if (p.precond != DMG_FP64) {
    v32.alloc(c, fb / 2);
    z32.alloc(c, fb / 2);
    pc32.alloc(h, dd, &p, &sh, nb);
  } else {
    pc64.alloc(h, dd, &p, &sh, nb);
  }
  reset_lanes();
}

void BWork::reset_lanes() {
  act.assign(nb, 0);
  it.assign(nb, 0);
  conv.assign(nb, 0);
  rel.assign(nb, 0.0);
  bn.assign(nb, 0.0);
  mvr.assign(3 * nb, 0);
  t_in.assign(nb, std::chrono::steady_clock::now());
}

void BWork::start_lanes(const std::vector<int>& lanes) {
  hipStream_t s = sh.s;
  const int64_t n = h->op[0].n;
  BS* bs = outer.st();
  // ||b|| of every lane (the other lanes' values are recomputed unchanged)
  launch_b_norm<double>(s, B.as<double2>(), n, nb, bs, 0.0, 3, nullptr, sh.P());
  for (int r : lanes) {
    launch_b_lane_copy(s, B.as<double2>(), Rr.as<double2>(), n, nb, r);
    launch_b_lane_copy(s, (const double2*)nullptr, X.as<double2>(), n, nb, r);
  }
  sh.read_tails(bs);
  const auto now = std::chrono::steady_clock::now();
  for (int r : lanes) {
    bn[r] = sh.tail[r].bnorm;
    it[r] = 0;
    rel[r] = bn[r] > 0.0 ? 1.0 : 0.0;
    conv[r] = bn[r] == 0.0 ? 1 : 0;
    act[r] = bn[r] > 0.0 ? 1 : 0;
    for (int l = 0; l < 3; ++l) mvr[3 * r + l] = 0;
    t_in[r] = now;
  }
}

void BWork::cycle() {
  hipStream_t s = sh.s;
  const bool fp32 = precond != DMG_FP64;
  const Op& A = h->op[0];
  const int64_t n = A.n;
  const int64_t ld = n * nb;
  double2* Bp = B.as<double2>();
  double2* Xp = X.as<double2>();
  double2* Rp = Rr.as<double2>();
  double2* V = outer.V.as<double2>();
  double2* Z = outer.Z.as<double2>();
  BS* bs = outer.st();
  auto pc_mv = [&](int l) { return fp32 ? pc32.mv[l] : pc64.mv[l]; };
  std::vector<int> cap(nb, 0);
  for (int r = 0; r < nb; ++r) {
    if (act[r] && it[r] >= p.max_outer_iters) act[r] = 0;
    cap[r] = act[r] ? std::min(p.outer_m, p.max_outer_iters - it[r]) : 0;
  }
  sh.set_state(bs, act, cap);
  launch_b_norm<double>(s, Rp, n, nb, bs, p.tol, 1, nullptr, sh.P());
  launch_b_scale_beta<double>(s, Rp, V, n, nb, bs);
  long long fine = 0;
  for (int j = 0; j < p.outer_m; ++j) {
    double2* vj = V + j * ld;
    double2* zj = Z + j * ld;
    if (fp32) {
      launch_cast_d2f(s, ld, vj, v32.as<float2>());
      pc32.cycle0(v32.as<float2>(), z32.as<float2>());
      launch_cast_f2d(s, ld, z32.as<float2>(), zj);
    } else {
      pc64.cycle0(vj, zj);
    }
    hipEvent_t ta = timer_mark(h->ctx, DMG_KT_WILSON_BATCHED, s);
    launch_b_wilson<double>(s, A.U64, zj, V + (j + 1) * ld, A.m0, A.Lx, A.Lt, nb, nullptr, bs);
    if (ta) timer_span(h->ctx, DMG_KT_WILSON_BATCHED, ta, timer_mark(h->ctx, DMG_KT_WILSON_BATCHED, s),
                       (long long)A.Lx * A.Lt * nb);
    fine++;
    launch_b_arnoldi<double>(s, V, ld, n, nb, j, bs, outer.anyp2(), sh.P());
    if (sh.all_done(bs, outer.flags())) break;
  }
  launch_b_ls_solve(s, bs, nb);
  launch_b_combine<double>(s, Xp, Z, ld, n, nb, bs, 0, 1);
  launch_b_wilson<double>(s, A.U64, Xp, Rp, A.m0, A.Lx, A.Lt, nb, Bp, nullptr);  // Rr = B - D X
  fine++;
  launch_b_norm<double>(s, Rp, n, nb, bs, 0.0, 0, rn.as<double>(), sh.P());
  std::vector<double> rnh(nb);
  DMG_HIP(hipMemcpyAsync(rnh.data(), rn.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  sh.read_tails(bs);
  long long dl[3];
  for (int l = 0; l < 3; ++l) {
    dl[l] = pc_mv(l) - mv_prev[l];
    mv_prev[l] = pc_mv(l);
  }
  dl[0] += fine;
  for (int r = 0; r < nb; ++r) {
    if (!act[r]) continue;
    const BSTail& t = sh.tail[r];
    it[r] += t.steps;
    for (int l = 0; l < 3; ++l) mvr[3 * r + l] += dl[l];
    rel[r] = std::sqrt(rnh[r]) / bn[r];
    conv[r] = rel[r] <= p.tol ? 1 : 0;
    if (conv[r] || t.steps == 0 || it[r] >= p.max_outer_iters) act[r] = 0;
  }
}

void BWork::stats(int r, dmg_solve_stats* o, std::chrono::steady_clock::time_point now) const {
  *o = dmg_solve_stats{};
  o->outer_iters = it[r];
  o->converged = conv[r];
  o->fine_mvps = mvr[3 * r];
  o->int_mvps = mvr[3 * r + 1];
  o->coarse_mvps = mvr[3 * r + 2];
  const double n0 = (double)h->op[0].n, n1 = (double)h->op[1].n, n2 = (double)h->op[2].n;
  o->fine_equiv_mvps = o->fine_mvps + n1 / n0 * o->int_mvps + n2 / n0 * o->coarse_mvps;
  o->true_rel_resid = rel[r];
  o->elapsed_ms = std::chrono::duration<double, std::milli>(now - t_in[r]).count();
}

BWork* create_bwork(dmg_hierarchy* h, dmg_deflation* d, const dmg_solve_params* p, int nb, bool own_stream) {
  BWork* w = new BWork();
  try {
    w->init(h, d, p, nb, own_stream);
  } catch (...) {
    delete w;
    throw;
  }
  return w;
}

static BWork* get_bwork(dmg_hierarchy* h, dmg_deflation* d, const dmg_solve_params* p, int nb) {
  BWork* w = h->bwork;
  if (w && w->nb == nb && w->outer_m == p->outer_m && w->int_m == p->int_m && w->precond == p->precond && w->d == d &&
      w->dm == d->m && w->dk == d->kk) {
    w->p = *p;
    w->reset_lanes();
    return w;
  }
  destroy_bwork(w);
  h->bwork = nullptr;
  h->bwork = create_bwork(h, d, p, nb, false);
  return h->bwork;
}

dmg_status batched_solve(dmg_hierarchy* h, dmg_deflation* d, const dmg_solve_params* p, const double2* b, double2* x,
                         int nrhs, dmg_solve_stats* stout) {
  int nb = 1;
  while (nb < nrhs) nb *= 2;
  BWork* w = get_bwork(h, d, p, nb);
  hipStream_t s = w->sh.s;
  const int64_t n = h->op[0].n;
  launch_b_gather(s, b, w->B.as<double2>(), n, nrhs, nb);
  std::vector<int> lanes(nrhs);
  for (int r = 0; r < nrhs; ++r) lanes[r] = r;
  w->start_lanes(lanes);
  while (w->any_active()) w->cycle();
  launch_b_scatter(s, w->X.as<double2>(), x, n, nrhs, nb);
  DMG_HIP(hipStreamSynchronize(s));
  const auto now = std::chrono::steady_clock::now();
  bool all = true;
  for (int r = 0; r < nrhs; ++r) {
    all = all && w->conv[r];
    if (stout) w->stats(r, stout + r, now);
  }
  return all ? DMG_OK : DMG_W_NOT_CONVERGED;
}

}  // namespace dmg

// ---------------------------------------------------------------- continuous batching (dmg_batch_*)
// The lanes of the engine are slots that requests join and leave between outer cycles.
using namespace dmg;

struct dmg_batch {
  dmg_hierarchy* h = nullptr;
  dmg_deflation* d = nullptr;
  int cap = 0;
  BWork* w = nullptr;
  std::vector<int> state;
  ~dmg_batch() { destroy_bwork(w); }
};

extern "C" {

dmg_status dmg_batch_create(dmg_hierarchy* h, dmg_deflation* d, int capacity, const dmg_solve_params* prm,
                            dmg_batch** out) {
  if (!h || !out) return DMG_E_INVALID;
  *out = nullptr;
  return guarded(h->ctx, [&]() -> dmg_status {
    DMG_CHECK(capacity >= 1 && capacity <= NBMAX, DMG_E_INVALID, "batch capacity outside [1, 64]");
    DMG_CHECK(d && d->h == h && d->ready, DMG_E_INVALID,
              "batch_create: the deflation space must belong to the hierarchy and be built");
    dmg_solve_params p;
    dmg_solve_params_default(&p);
    if (prm) p = *prm;
    DMG_CHECK(p.tol > 0.0 && p.int_tol > 0.0 && p.coarse_tol_later > 0.0 && p.max_outer_iters >= 1 &&
                  p.int_max_iters >= 1 && p.coarse_max_iters >= 1 && p.outer_m >= 1 && p.outer_m <= MB &&
                  p.int_m >= 1 && p.int_m <= MB && p.smooth_steps == 2 && !p.use_x0 && d->m - d->kk <= MB &&
                  p.int_mode == 0 && (p.precond == DMG_FP64 || p.precond == DMG_FP32 || p.precond == DMG_FP32_BF16),
              DMG_E_INVALID, "batch parameters (restart lengths <= 24, two smoothing steps, no x0, partial "
                             "intermediate solve, a precision of the lockstep form)");
    if (p.precond != DMG_FP64) prepare_deflation_fp32(&h->main, d);
    int nb = 1;
    while (nb < capacity) nb *= 2;
    std::unique_ptr<dmg_batch> bt(new dmg_batch());
    bt->h = h;
    bt->d = d;
    bt->cap = capacity;
    bt->w = create_bwork(h, d, &p, nb, true);
    bt->state.assign(capacity, DMG_SLOT_FREE);
    DMG_HIP(hipStreamSynchronize(bt->w->sh.s));
    DMG_HIP(hipStreamSynchronize(h->ctx->stream));
    *out = bt.release();
    return DMG_OK;
  });
}

dmg_status dmg_batch_admit(dmg_batch* bt, int slot, const void* b, int ptr_kind) {
  if (!bt) return DMG_E_INVALID;
  dmg_context* c = bt->h->ctx;
  return guarded(c, [&]() -> dmg_status {
    DMG_CHECK(slot >= 0 && slot < bt->cap && b, DMG_E_INVALID, "batch_admit: bad arguments");
    DMG_CHECK(ptr_kind == DMG_PTR_HOST || ptr_kind == DMG_PTR_DEVICE, DMG_E_INVALID, "batch_admit: pointer kind");
    DMG_CHECK(bt->state[slot] == DMG_SLOT_FREE, DMG_E_INVALID, "batch_admit: slot is busy");
    BWork* w = bt->w;
    const int64_t n = bt->h->op[0].n;
    hipStream_t s = w->sh.s;
    DevBuf tmp;
    const double2* src = (const double2*)b;
    w->order_after_ctx();  // a device b is ordered on the context's stream
    if (ptr_kind == DMG_PTR_HOST) {
      const double* v = (const double*)b;
      for (int64_t i = 0; i < 2 * n; ++i)
        DMG_CHECK(std::isfinite(v[i]), DMG_E_NONFINITE, "non-finite right-hand side");
      tmp.alloc(c, sizeof(double2) * n);
      DMG_HIP(hipMemcpyAsync(tmp.p, b, sizeof(double2) * n, hipMemcpyHostToDevice, s));
      src = tmp.as<double2>();
    }
    launch_b_lane_io(s, src, w->B.as<double2>(), n, w->nb, slot, 1);
    w->start_lanes({slot});  // synchronises the stream
    bt->state[slot] = w->act[slot] ? DMG_SLOT_RUNNING : DMG_SLOT_DONE;
    return DMG_OK;
  });
}

dmg_status dmg_batch_step(dmg_batch* bt, int min_iters, int* n_done) {
  if (!bt) return DMG_E_INVALID;
  return guarded(bt->h->ctx, [&]() -> dmg_status {
    DMG_CHECK(min_iters >= 1, DMG_E_INVALID, "batch_step: min_iters must be >= 1");
    BWork* w = bt->w;
    const int cycles = (min_iters + w->p.outer_m - 1) / w->p.outer_m;
    for (int c = 0; c < cycles && w->any_active(); ++c) w->cycle();
    int k = 0;
    for (int i = 0; i < bt->cap; ++i) {
      if (bt->state[i] == DMG_SLOT_RUNNING && !w->act[i]) bt->state[i] = DMG_SLOT_DONE;
      k += bt->state[i] == DMG_SLOT_DONE ? 1 : 0;
    }
    if (n_done) *n_done = k;
    return DMG_OK;
  });
}

dmg_status dmg_batch_retire(dmg_batch* bt, int slot, void* x, int ptr_kind, dmg_solve_stats* stats) {
  if (!bt) return DMG_E_INVALID;
  dmg_context* c = bt->h->ctx;
  return guarded(c, [&]() -> dmg_status {
    DMG_CHECK(slot >= 0 && slot < bt->cap && x, DMG_E_INVALID, "batch_retire: bad arguments");
    DMG_CHECK(ptr_kind == DMG_PTR_HOST || ptr_kind == DMG_PTR_DEVICE, DMG_E_INVALID, "batch_retire: pointer kind");
    DMG_CHECK(bt->state[slot] == DMG_SLOT_DONE, DMG_E_INVALID, "batch_retire: slot has no finished solve");
    BWork* w = bt->w;
    const int64_t n = bt->h->op[0].n;
    hipStream_t s = w->sh.s;
    w->order_after_ctx();
    if (ptr_kind == DMG_PTR_HOST) {
      DevBuf tmp;
      tmp.alloc(c, sizeof(double2) * n);
      launch_b_lane_io(s, w->X.as<double2>(), tmp.as<double2>(), n, w->nb, slot, 0);
      DMG_HIP(hipMemcpyAsync(x, tmp.p, sizeof(double2) * n, hipMemcpyDeviceToHost, s));
      DMG_HIP(hipStreamSynchronize(s));
    } else {  // x is written in order on the context's stream
      launch_b_lane_io(s, w->X.as<double2>(), (double2*)x, n, w->nb, slot, 0);
      DMG_HIP(hipEventRecord(w->ev, s));
      DMG_HIP(hipStreamWaitEvent(c->stream, w->ev, 0));
    }
    if (stats) w->stats(slot, stats, std::chrono::steady_clock::now());
    bt->state[slot] = DMG_SLOT_FREE;
    return w->conv[slot] ? DMG_OK : DMG_W_NOT_CONVERGED;
  });
}

int dmg_batch_slot_state(dmg_batch* bt, int slot) {
  if (!bt || slot < 0 || slot >= bt->cap) return -1;
  return bt->state[slot];
}

void dmg_batch_destroy(dmg_batch* bt) { delete bt; }

}  // extern "C"
