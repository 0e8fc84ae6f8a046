// Pool of independent solves: slots with their own stream, host worker thread and
// solver workspace, each taking a right-hand side of any hierarchy.  The solves of
// different slots overlap on the device; each advances by whole outer FGMRES
// cycles, so its arithmetic is the same alone or in a mix.
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <thread>

#include "solver.h"

using namespace dmg;

struct dmg_pool {
  struct Slot {
    Work w;
    int state = DMG_SLOT_FREE;
    bool begun = false;
    dmg_hierarchy* h = nullptr;
    dmg_deflation* d = nullptr;
    DevBuf b, x;
    dmg_status status = DMG_OK;
    std::string err;
    dmg_solve_stats stats{};
    bool go = false;    // an advance is requested
    bool busy = false;  // an advance is in flight (the worker owns the slot)
    int iters = 1;
    std::chrono::steady_clock::time_point t_admit;
    std::thread th;
  };
  dmg_context* ctx = nullptr;
  int cap = 0;
  dmg_solve_params p{};
  std::vector<std::unique_ptr<Slot>> slots;
  std::mutex mu;
  std::condition_variable cv_go, cv_done;
  long long completions = 0;  // advances finished
  bool quit = false;

  void worker(int i);
  ~dmg_pool();
};

void dmg_pool::worker(int i) {
  Slot& sl = *slots[i];
  (void)hipSetDevice(ctx->device);
  for (;;) {
    int iters;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_go.wait(lk, [&] { return quit || sl.go; });
      if (quit) return;
      sl.go = false;
      iters = sl.iters;
    }
    bool done = false;
    dmg_status status = DMG_OK;
    std::string err;
    try {
      if (!sl.begun) {
        outer_begin(sl.h, &sl.w, sl.d, &p, sl.b.as<double2>(), sl.x.as<double2>());
        sl.w.run.t0 = sl.t_admit;
        sl.begun = true;
      }
      if (outer_advance(&sl.w, iters)) {
        status = outer_finish(&sl.w, &sl.stats);
        done = true;
      }
    } catch (const Error& e) {
      status = e.code;
      err = e.msg;
      done = true;
      (void)hipStreamSynchronize(sl.w.stream);
      (void)hipGetLastError();
    } catch (const std::exception& e) {
      status = DMG_E_INVALID;
      err = e.what();
      done = true;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (done) {
      sl.status = status;
      sl.err = err;
      sl.state = DMG_SLOT_DONE;
    }
    sl.busy = false;
    ++completions;
    cv_done.notify_all();
  }
}

dmg_pool::~dmg_pool() {
  {
    std::unique_lock<std::mutex> lk(mu);
    cv_done.wait(lk, [&] {
      for (auto& s : slots)
        if (s->busy) return false;
      return true;
    });
    quit = true;
  }
  cv_go.notify_all();
  for (auto& s : slots)
    if (s->th.joinable()) s->th.join();
  slots.clear();  // each Work waits for its stream before releasing memory
}

extern "C" {

dmg_status dmg_pool_create(dmg_context* ctx, int capacity, const dmg_solve_params* prm, dmg_pool** out) {
  if (!ctx || !out) return DMG_E_INVALID;
  *out = nullptr;
  return guarded(ctx, [&]() -> dmg_status {
    DMG_CHECK(capacity >= 1 && capacity <= DMG_POOL_MAX_SLOTS, DMG_E_INVALID, "pool capacity outside [1, 8]");
    dmg_solve_params p;
    dmg_solve_params_default(&p);
    if (prm) p = *prm;
    DMG_CHECK(p.tol > 0.0 && p.int_tol > 0.0 && p.coarse_tol_first > 0.0 && p.coarse_tol_later > 0.0 &&
                  p.max_outer_iters >= 1 && p.int_max_iters >= 1 && p.coarse_max_iters >= 1 &&
                  p.outer_m >= 1 && p.outer_m <= MMAX && p.int_m >= 1 && p.int_m <= MMAX &&
                  p.smooth_steps >= 1 && p.smooth_steps <= MMAX && !p.use_x0 &&
                  (p.coarse_persistent == 0 || p.coarse_persistent == 1),
              DMG_E_INVALID, "pool solve parameters (use_x0 is not supported)");
    std::unique_ptr<dmg_pool> pl(new dmg_pool());
    pl->ctx = ctx;
    pl->cap = capacity;
    pl->p = p;
    for (int i = 0; i < capacity; ++i) {
      pl->slots.emplace_back(new dmg_pool::Slot());
      hipStream_t s = nullptr;
      DMG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      pl->slots.back()->w.init(ctx, s, true);
    }
    DMG_HIP(hipStreamSynchronize(ctx->stream));
    for (auto& s : pl->slots) DMG_HIP(hipStreamSynchronize(s->w.stream));
    for (int i = 0; i < capacity; ++i) {
      dmg_pool* raw = pl.get();
      pl->slots[i]->th = std::thread([raw, i] { raw->worker(i); });
    }
    *out = pl.release();
    return DMG_OK;
  });
}

dmg_status dmg_pool_admit(dmg_pool* pl, int slot, dmg_hierarchy* h, dmg_deflation* d, const void* b,
                           int ptr_kind) {
  if (!pl) return DMG_E_INVALID;
  return guarded(pl->ctx, [&]() -> dmg_status {
    DMG_CHECK(slot >= 0 && slot < pl->cap && h && b, DMG_E_INVALID, "pool_admit: bad arguments");
    DMG_CHECK(ptr_kind == DMG_PTR_HOST || ptr_kind == DMG_PTR_DEVICE, DMG_E_INVALID, "pool_admit: pointer kind");
    dmg_pool::Slot& sl = *pl->slots[slot];
    {
      std::lock_guard<std::mutex> lk(pl->mu);
      DMG_CHECK(sl.state == DMG_SLOT_FREE, DMG_E_INVALID, "pool_admit: slot is busy");
    }
    DMG_CHECK(h->ctx == pl->ctx, DMG_E_INVALID, "pool_admit: hierarchy belongs to another context");
    DMG_CHECK(!d || (d->h == h && d->ready), DMG_E_INVALID,
              "pool_admit: the deflation space must belong to the hierarchy and be built");
    const int64_t n = h->op[0].n;
    const size_t fb = sizeof(double2) * n;
    if (ptr_kind == DMG_PTR_HOST) {
      const double* v = (const double*)b;
      for (int64_t i = 0; i < 2 * n; ++i)
        DMG_CHECK(std::isfinite(v[i]), DMG_E_NONFINITE, "non-finite right-hand side");
    }
    // workspace for h first: a budget failure leaves the slot FREE
    prepare_work(h, &sl.w, d, &pl->p);
    if (pl->p.precond != DMG_FP64) prepare_deflation_fp32(&sl.w, d);
    // workspace initialisation may have been queued on the context's stream
    DMG_HIP(hipStreamSynchronize(pl->ctx->stream));
    if (sl.b.bytes != fb) {
      DMG_HIP(hipStreamSynchronize(sl.w.stream));
      sl.b.alloc(pl->ctx, fb);
      sl.x.alloc(pl->ctx, fb);
    }
    hipStream_t s = sl.w.stream;
    if (ptr_kind == DMG_PTR_HOST) {
      DMG_HIP(hipMemcpyAsync(sl.b.p, b, fb, hipMemcpyHostToDevice, s));
      DMG_HIP(hipStreamSynchronize(s));
    } else {
      // device input: order the copy after the caller's stream
      hipEvent_t e;
      DMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      DMG_HIP(hipEventRecord(e, pl->ctx->stream));
      DMG_HIP(hipStreamWaitEvent(s, e, 0));
      DMG_HIP(hipEventDestroy(e));
      DMG_HIP(hipMemcpyAsync(sl.b.p, b, fb, hipMemcpyDeviceToDevice, s));
    }
    sl.h = h;
    sl.d = d;
    sl.t_admit = std::chrono::steady_clock::now();
    sl.begun = false;
    sl.status = DMG_OK;
    sl.err.clear();
    sl.stats = dmg_solve_stats{};
    std::lock_guard<std::mutex> lk(pl->mu);
    sl.state = DMG_SLOT_RUNNING;
    return DMG_OK;
  });
}

dmg_status dmg_pool_step(dmg_pool* pl, int min_iters, int* n_done) {
  if (!pl) return DMG_E_INVALID;
  return guarded(pl->ctx, [&]() -> dmg_status {
    DMG_CHECK(min_iters >= 1, DMG_E_INVALID, "pool_step: min_iters must be >= 1");
    std::unique_lock<std::mutex> lk(pl->mu);
    const long long c0 = pl->completions;
    int busy = 0;
    for (auto& s : pl->slots) {
      if (s->state == DMG_SLOT_RUNNING && !s->busy) {
        s->busy = true;
        s->go = true;
        s->iters = min_iters;
      }
      busy += s->busy ? 1 : 0;
    }
    pl->cv_go.notify_all();
    if (busy) pl->cv_done.wait(lk, [&] { return pl->completions != c0; });
    if (n_done) {
      int k = 0;
      for (auto& s : pl->slots) k += s->state == DMG_SLOT_DONE ? 1 : 0;
      *n_done = k;
    }
    return DMG_OK;
  });
}

dmg_status dmg_pool_retire(dmg_pool* pl, int slot, void* x, int ptr_kind, dmg_solve_stats* stats) {
  if (!pl) return DMG_E_INVALID;
  dmg_context* c = pl->ctx;
  dmg_status st = guarded(c, [&]() -> dmg_status {
    DMG_CHECK(slot >= 0 && slot < pl->cap && x, DMG_E_INVALID, "pool_retire: bad arguments");
    DMG_CHECK(ptr_kind == DMG_PTR_HOST || ptr_kind == DMG_PTR_DEVICE, DMG_E_INVALID, "pool_retire: pointer kind");
    dmg_pool::Slot& sl = *pl->slots[slot];
    {
      std::lock_guard<std::mutex> lk(pl->mu);
      DMG_CHECK(sl.state == DMG_SLOT_DONE && !sl.busy, DMG_E_INVALID, "pool_retire: slot has no finished solve");
      sl.state = DMG_SLOT_FREE;
    }
    if (stats) *stats = sl.stats;
    if (sl.status < 0) throw Error{sl.status, sl.err};
    hipStream_t s = sl.w.stream;
    const size_t fb = sl.x.bytes;
    DMG_HIP(hipMemcpyAsync(x, sl.x.p, fb, ptr_kind == DMG_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                           s));
    if (ptr_kind == DMG_PTR_HOST) {
      DMG_HIP(hipStreamSynchronize(s));
    } else {
      // device output: make the caller's stream wait for the copy
      hipEvent_t e;
      DMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      DMG_HIP(hipEventRecord(e, s));
      DMG_HIP(hipStreamWaitEvent(c->stream, e, 0));
      DMG_HIP(hipEventDestroy(e));
    }
    return sl.status;
  });
  return st;
}

int dmg_pool_slot_state(dmg_pool* pl, int slot) {
  if (!pl || slot < 0 || slot >= pl->cap) return -1;
  std::lock_guard<std::mutex> lk(pl->mu);
  return pl->slots[slot]->state;
}

void dmg_pool_destroy(dmg_pool* pl) { delete pl; }

}  // extern "C"
