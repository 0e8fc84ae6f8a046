// Long-cycle GMRES-DR(m, k) and GMRES-Proj(m, k) on any FP64 operator of a hierarchy
// (Methods section; the paper's sizes are m = 200, k = 40).  The Arnoldi vectors stay in
// device memory and every step is a handful of kernels: the operator, classical Gram-Schmidt
// applied twice (multi-vector dot products and updates in chunks of 64 vectors), the norm,
// and one small kernel that appends the column to the Hessenberg matrix and updates its
// Givens QR (KBig, bigkrylov.h).  The harmonic-Ritz restart runs in one workgroup.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "bigkrylov.h"
#include "solver.h"

namespace dmg {

static_assert(offsetof(KBig, steps) == offsetof(KBig, nrot) + 4, "KBig tail layout");
static_assert(offsetof(KBig, tol_abs) == offsetof(KBig, nrot) + 16, "KBig tail layout");
static_assert(offsetof(KBig, bnorm) == offsetof(KBig, nrot) + offsetof(KBigStatus, bnorm), "KBig tail layout");

constexpr int BT_RESTART = 256;
constexpr int BT_SMALL = 256;
constexpr int CHUNK = 64;  // vectors per multi-vector dot product / update launch

struct DevTeam {
  double2* shm;
  __device__ int tid() const { return threadIdx.x; }
  __device__ int size() const { return blockDim.x; }
  __device__ bool lead() const { return threadIdx.x == 0; }
  __device__ void sync() const { __syncthreads(); }
};

__global__ void __launch_bounds__(BT_RESTART) k_big_restart(KBig* kb, int m, int k, double2* P, int final_mode,
                                                            double2* work, int* status) {
  __shared__ double2 shm[2 * LDBIG + 16];
  DevTeam tm{shm};
  const int st = big_restart_body(tm, kb, m, k, P, final_mode, work);
  if (st != 0 && threadIdx.x == 0) status[0] = st;
}

__global__ void __launch_bounds__(BT_SMALL) k_big_column(KBig* kb, int j) {
  __shared__ double2 shm[LDBIG + 1];
  DevTeam tm{shm};
  big_column_body(tm, kb, j);
}

__global__ void __launch_bounds__(BT_SMALL) k_big_lssolve(KBig* kb) {
  __shared__ double2 shm[LDBIG + 1];
  DevTeam tm{shm};
  big_lssolve_body(tm, kb);
}

// fresh cycle from a residual of squared norm rn2[0]: beta e1, no rotations; bnorm = beta when
// set_bnorm, and tol_abs = tol_rel * bnorm
__global__ void k_big_start(KBig* kb, const double* rn2, double tol_rel, int set_bnorm) {
  const double beta = sqrt(rn2[0] > 0.0 ? rn2[0] : 0.0);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < LDBIG * MBIG; e += gridDim.x * blockDim.x) {
    kb->H[e] = mk(0.0, 0.0);
    kb->R[e] = mk(0.0, 0.0);
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < LDBIG; i += blockDim.x) {
      kb->c[i] = mk(i == 0 ? beta : 0.0, 0.0);
      kb->g[i] = kb->c[i];
      kb->y[i] = mk(0.0, 0.0);
      kb->u[i] = kb->c[i];
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (set_bnorm) kb->bnorm = beta;
    kb->beta = beta;
    kb->tol_abs = tol_rel * kb->bnorm;
    kb->est = beta;
    kb->nrot = 0;
    kb->steps = 0;
    kb->breakdown = 0;
    kb->done = (beta == 0.0 || beta <= kb->tol_abs) ? 1 : 0;
  }
}

// projection over a deflation space: d = M c, u = Pi c (M: k x (k+1), Pi: (k+1) x (k+1),
// column-major)
__global__ void k_big_project(const double2* M, const double2* Pi, const double2* c, int k, double2* d,
                              double2* u) {
  const int t = threadIdx.x;
  for (int r = t; r < 2 * k + 1; r += blockDim.x) {
    double2 acc = mk(0.0, 0.0);
    if (r < k) {
      for (int j = 0; j <= k; ++j) cfma(acc, M[r + k * j], c[j]);
      d[r] = acc;
    } else {
      const int i = r - k;
      for (int j = 0; j <= k; ++j) cfma(acc, Pi[i + (k + 1) * j], c[j]);
      u[i] = acc;
    }
  }
}

// M = Hbar^+ and Pi = Hbar Hbar^+ of a full-rank (k+1) x k matrix through its QR (Gram-Schmidt
// twice): Hbar = Q R, M = R^{-1} Q^H, Pi = Q Q^H.  One workgroup; work: (k+1) k + k k entries.
__global__ void __launch_bounds__(BT_SMALL) k_big_proj_prepare(const double2* H, int k, double2* M, double2* Pi,
                                                               double2* work, int* status) {
  __shared__ double2 sh[KBIG + 2];
  const int t = threadIdx.x, nt = blockDim.x;
  const int K1 = k + 1;
  double2* Q = work;            // K1 x k
  double2* R = work + K1 * k;   // k x k
  for (int e = t; e < K1 * k; e += nt) Q[e] = H[e];
  for (int e = t; e < k * k; e += nt) R[e] = mk(0.0, 0.0);
  __syncthreads();
  for (int q = 0; q < k; ++q) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int p = t; p < q; p += nt) {
        double2 d = mk(0.0, 0.0);
        for (int r = 0; r < K1; ++r) cfmac(d, Q[r + K1 * p], Q[r + K1 * q]);
        sh[p] = d;
        R[p + k * q] = cadd(R[p + k * q], d);
      }
      __syncthreads();
      for (int r = t; r < K1; r += nt) {
        double2 acc = Q[r + K1 * q];
        for (int p = 0; p < q; ++p) acc = csub(acc, cmul(sh[p], Q[r + K1 * p]));
        Q[r + K1 * q] = acc;
      }
      __syncthreads();
    }
    if (t == 0) {
      double n2 = 0.0;
      for (int r = 0; r < K1; ++r) n2 += cabs2(Q[r + K1 * q]);
      const double nn = sqrt(n2);
      if (!(nn > 0.0)) status[0] = 3;
      sh[KBIG + 1] = mk(nn > 0.0 ? 1.0 / nn : 0.0, 0.0);
      R[q + k * q] = mk(nn, 0.0);
    }
    __syncthreads();
    for (int r = t; r < K1; r += nt) Q[r + K1 * q] = cscale(Q[r + K1 * q], sh[KBIG + 1].x);
    __syncthreads();
  }
  // M[:, j] = R^{-1} conj(Q[j, :])^T, one column per thread
  for (int j = t; j < K1; j += nt) {
    for (int i = k - 1; i >= 0; --i) {
      double2 acc = cconj(Q[j + K1 * i]);
      for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(R[i + k * l], M[l + k * j]));
      const double2 d = R[i + k * i];
      M[i + k * j] = (d.x == 0.0 && d.y == 0.0) ? mk(0.0, 0.0) : cdiv(acc, d);
    }
  }
  for (int e = t; e < K1 * K1; e += nt) {
    const int i = e % K1, j = e / K1;
    double2 acc = mk(0.0, 0.0);
    for (int l = 0; l < k; ++l) cfma(acc, Q[i + K1 * l], cconj(Q[j + K1 * l]));
    Pi[e] = acc;
  }
}

// ---------------------------------------------------------------- host side
struct BigWS {
  int m = 0;
  int64_t n = 0;
  DevBuf V, Vtmp, ks, work, P, coef, nrm, r, status;
  KBig* state() const { return ks.as<KBig>(); }
};

void destroy_bigws(BigWS* b) { delete b; }

static BigWS* big_ws(Work* w, int m, int64_t n) {
  if (!w->big) w->big = new BigWS();
  BigWS* b = w->big;
  if (b->m < m || b->n != n) {
    b->V.alloc(w->ctx, sizeof(double2) * (size_t)n * (m + 1));
    b->Vtmp.alloc(w->ctx, sizeof(double2) * (size_t)n * (KBIG + 1));
    b->r.alloc(w->ctx, sizeof(double2) * (size_t)n);
    b->m = m;
    b->n = n;
  }
  if (!b->ks.p) {
    b->ks.alloc(w->ctx, sizeof(KBig));
    b->work.alloc(w->ctx, sizeof(double2) * big_restart_work_elems());
    b->P.alloc(w->ctx, sizeof(double2) * (size_t)LDBIG * (KBIG + 1));
    b->coef.alloc(w->ctx, sizeof(double2) * 2 * LDBIG);
    b->nrm.alloc(w->ctx, sizeof(double) * 4);
    b->status.alloc(w->ctx, sizeof(int) * 4);
    DMG_HIP(hipMemsetAsync(b->ks.p, 0, sizeof(KBig), w->stream));
  }
  return b;
}

static KBigStatus big_status(Work* w, BigWS* b) {
  static_assert(sizeof(KBigStatus) <= 256, "status staged in the workspace's pinned buffer");
  DMG_HIP(hipMemcpyAsync(w->host_status, &b->state()->nrot, sizeof(KBigStatus), hipMemcpyDeviceToHost, w->stream));
  DMG_HIP(hipStreamSynchronize(w->stream));
  KBigStatus st;
  std::memcpy(&st, w->host_status, sizeof(st));
  return st;
}

// out[0 .. nv) = V^H w over nv vectors of V (ld n), in chunks
static void big_dots(Work* w, const double2* V, int64_t n, int nv, const double2* x, double2* out) {
  for (int c0 = 0; c0 < nv; c0 += CHUNK)
    launch_multidot<double>(w->stream, V + (int64_t)c0 * n, n, std::min(CHUNK, nv - c0), x, n, out + c0,
                            w->partials.as<double2>(), w->counters.as<unsigned>());
}
// x -= sign * V coef over nv vectors, in chunks
static void big_axpy(Work* w, double2* x, const double2* V, int64_t n, int nv, const double2* coef, double sign) {
  for (int c0 = 0; c0 < nv; c0 += CHUNK)
    launch_multi_axpy<double>(w->stream, x, V + (int64_t)c0 * n, n, std::min(CHUNK, nv - c0), coef + c0, n, sign);
}

// v_0 = r / ||r|| and a fresh cycle state
static void big_cycle_start(Work* w, BigWS* b, const double2* r, double tol_rel, bool set_bnorm) {
  hipStream_t s = w->stream;
  launch_norm2<double>(s, b->n, r, b->nrm.as<double>(), w->partials.as<double2>(), w->counters.as<unsigned>());
  hipLaunchKernelGGL(k_big_start, dim3(64), dim3(256), 0, s, b->state(), (const double*)b->nrm.p, tol_rel,
                     set_bnorm ? 1 : 0);
  DMG_LAUNCH_CHECK();
  launch_scale_dev<double>(s, b->n, r, b->V.as<double2>(), b->nrm.as<double>(), 1);
}

// Arnoldi steps j0 .. m-1 (or until the state is done); returns the status after the last one
static KBigStatus big_arnoldi(Work* w, BigWS* b, const Op& A, int j0, int m) {
  hipStream_t s = w->stream;
  KBig* kb = b->state();
  const int64_t n = b->n;
  double2* V = b->V.as<double2>();
  KBigStatus st = big_status(w, b);
  for (int j = j0; j < m && !st.done; ++j) {
    double2* wv = V + (int64_t)(j + 1) * n;
    A.apply(s, V + (int64_t)j * n, wv, 0, nullptr);
    launch_norm2<double>(s, n, wv, &kb->wn0, w->partials.as<double2>(), w->counters.as<unsigned>());
    big_dots(w, V, n, j + 1, wv, kb->h1);
    big_axpy(w, wv, V, n, j + 1, kb->h1, 1.0);
    big_dots(w, V, n, j + 1, wv, kb->h2);
    big_axpy(w, wv, V, n, j + 1, kb->h2, 1.0);
    launch_norm2<double>(s, n, wv, &kb->wn, w->partials.as<double2>(), w->counters.as<unsigned>());
    hipLaunchKernelGGL(k_big_column, dim3(1), dim3(BT_SMALL), 0, s, kb, j);
    DMG_LAUNCH_CHECK();
    launch_scale_dev<double>(s, n, wv, wv, &kb->wn, 1);
    w->cnt.mv[A.kind == 0 ? 0 : 2]++;
    st = big_status(w, b);
  }
  return st;
}

static void big_restart(Work* w, BigWS* b, int m, int k, int final_mode) {
  hipStream_t s = w->stream;
  int* status = b->status.as<int>();
  DMG_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_big_restart, dim3(1), dim3(BT_RESTART), 0, s, b->state(), m, k, b->P.as<double2>(), final_mode,
                     b->work.as<double2>(), status);
  DMG_LAUNCH_CHECK();
  int st = 0;
  DMG_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  DMG_CHECK(st == 0, DMG_E_BREAKDOWN,
            st == 1 ? "long-cycle GMRES-DR restart: singular Hessenberg block"
                    : "long-cycle GMRES-DR restart: the eigenvalue iteration did not converge");
}

// V_{0..k} <- V_{0..m} P, then v_k re-orthogonalised against v_0 .. v_{k-1}
static void big_rotate_basis(Work* w, BigWS* b, int m, int k) {
  hipStream_t s = w->stream;
  const int64_t n = b->n;
  double2* V = b->V.as<double2>();
  launch_basis_rotate<double>(s, V, b->Vtmp.as<double2>(), n, n, b->P.as<double2>(), m + 1, m + 1, k + 1);
  DMG_HIP(hipMemcpyAsync(V, b->Vtmp.p, sizeof(double2) * n * (k + 1), hipMemcpyDeviceToDevice, s));
  double2* coef = b->coef.as<double2>();
  double2* vk = V + (int64_t)k * n;
  big_dots(w, V, n, k, vk, coef);
  big_axpy(w, vk, V, n, k, coef, 1.0);
  launch_norm2<double>(s, n, vk, b->nrm.as<double>(), w->partials.as<double2>(), w->counters.as<unsigned>());
  launch_scale_dev<double>(s, n, vk, vk, b->nrm.as<double>(), 1);
}

int big_gmres_dr(dmg_context* ctx, Work* w, const Op& A, int m, int k, const double2* b_in, double2* x, double tol,
                 int max_iters, dmg_deflation* d) {
  DMG_CHECK(m >= 2 && m <= MBIG && k >= 1 && k < m && k <= KBIG, DMG_E_INVALID, "long-cycle GMRES-DR sizes");
  hipStream_t s = w->stream;
  const int64_t n = A.n;
  BigWS* b = big_ws(w, m, n);
  KBig* kb = b->state();
  double2* V = b->V.as<double2>();
  DMG_HIP(hipMemsetAsync(x, 0, sizeof(double2) * n, s));
  big_cycle_start(w, b, b_in, tol, true);
  int j0 = 0, iters = 0;
  double prev = -1.0;
  KBigStatus st{};
  for (;;) {
    st = big_arnoldi(w, b, A, j0, m);
    hipLaunchKernelGGL(k_big_lssolve, dim3(1), dim3(BT_SMALL), 0, s, kb);
    DMG_LAUNCH_CHECK();
    big_axpy(w, x, V, n, st.steps, kb->y, -1.0);
    iters += st.steps - j0;
    if (st.done || iters >= max_iters) break;
    // the stagnation exit of the short-cycle solver (a tolerance the arithmetic cannot reach)
    if (prev > 0.0 && st.est > 0.99 * prev && st.est <= 1e-10 * st.bnorm) break;
    prev = st.est;
    big_restart(w, b, m, k, 0);
    big_rotate_basis(w, b, m, k);
    j0 = k;
  }
  if (d) {
    // the stored space A V_k = V_{k+1} Hbar_k: one more compression with the harmonic residual
    const int cols = st.steps;
    const int kk = (cols > k && !st.breakdown) ? k : std::max(cols, 1);
    if (cols > k && !st.breakdown) {
      big_restart(w, b, cols, k, 1);
      big_rotate_basis(w, b, cols, k);
    }
    d->V64.alloc(ctx, sizeof(double2) * (size_t)n * (kk + 1));
    d->H.alloc(ctx, sizeof(double2) * (size_t)(kk + 1) * kk);
    DMG_HIP(hipMemcpyAsync(d->V64.p, V, sizeof(double2) * n * (kk + 1), hipMemcpyDeviceToDevice, s));
    DMG_HIP(hipMemcpy2DAsync(d->H.p, sizeof(double2) * (kk + 1), kb->H, sizeof(double2) * LDBIG,
                             sizeof(double2) * (kk + 1), kk, hipMemcpyDeviceToDevice, s));
    d->kk = kk;
    d->M.alloc(ctx, sizeof(double2) * (size_t)kk * (kk + 1));
    d->Pi.alloc(ctx, sizeof(double2) * (size_t)(kk + 1) * (kk + 1));
    int* status = b->status.as<int>();
    DMG_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_big_proj_prepare, dim3(1), dim3(BT_SMALL), 0, s, d->H.as<double2>(), kk, d->M.as<double2>(),
                       d->Pi.as<double2>(), b->work.as<double2>(), status);
    DMG_LAUNCH_CHECK();
    int ps = 0;
    DMG_HIP(hipMemcpyAsync(&ps, status, sizeof(int), hipMemcpyDeviceToHost, s));
    DMG_HIP(hipStreamSynchronize(s));
    DMG_CHECK(ps == 0, DMG_E_BREAKDOWN, "long-cycle GMRES-DR: rank-deficient deflation block");
    d->ready = 1;
    d->cast_ready = 0;
  }
  return iters;
}

int big_gmres_proj(Work* w, const Op& A, const dmg_deflation* d, const double2* b_in, double2* x, double tol,
                   int max_iters, double* rel_est) {
  DMG_CHECK(d && d->ready && d->m <= MBIG && d->kk <= KBIG, DMG_E_INVALID, "long-cycle GMRES-Proj: deflation space");
  hipStream_t s = w->stream;
  const int64_t n = A.n;
  const int k = d->kk;
  const int mm = std::max(d->m - k, 1);
  BigWS* b = big_ws(w, mm, n);
  KBig* kb = b->state();
  double2* V = b->V.as<double2>();
  double2* r = b->r.as<double2>();
  const double2* DV = d->V64.as<double2>();
  double2* cvec = b->coef.as<double2>();
  double2* dd = cvec + LDBIG;
  double2* uu = kb->h2;  // scratch outside an Arnoldi step
  DMG_HIP(hipMemsetAsync(x, 0, sizeof(double2) * n, s));
  DMG_HIP(hipMemcpyAsync(r, b_in, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
  // ||b|| into the state (a zero-length cycle start on b itself)
  launch_norm2<double>(s, n, b_in, b->nrm.as<double>(), w->partials.as<double2>(), w->counters.as<unsigned>());
  hipLaunchKernelGGL(k_big_start, dim3(64), dim3(256), 0, s, kb, (const double*)b->nrm.p, tol, 1);
  DMG_LAUNCH_CHECK();
  KBigStatus st = big_status(w, b);
  const double bnorm = st.bnorm;
  int iters = 0;
  double est = bnorm;
  if (bnorm == 0.0) {
    if (rel_est) *rel_est = 0.0;
    return 0;
  }
  for (;;) {
    // projection over the deflation space: minimise || r - A V_k d || with A V_k = V_{k+1} Hbar_k
    big_dots(w, DV, n, k + 1, r, cvec);
    hipLaunchKernelGGL(k_big_project, dim3(1), dim3(128), 0, s, d->M.as<double2>(), d->Pi.as<double2>(),
                       (const double2*)cvec, k, dd, uu);
    DMG_LAUNCH_CHECK();
    big_axpy(w, x, DV, n, k, dd, -1.0);
    big_axpy(w, r, DV, n, k + 1, uu, 1.0);
    // one GMRES(m - k) cycle from r
    big_cycle_start(w, b, r, tol, false);
    st = big_status(w, b);
    est = st.beta;
    if (st.done) break;
    st = big_arnoldi(w, b, A, 0, mm);
    hipLaunchKernelGGL(k_big_lssolve, dim3(1), dim3(BT_SMALL), 0, s, kb);
    DMG_LAUNCH_CHECK();
    big_axpy(w, x, V, n, st.steps, kb->y, -1.0);
    // r = V_{steps+1} u (the residual from the Arnoldi relation)
    launch_basis_rotate<double>(s, V, r, n, n, kb->u, LDBIG, st.steps + 1, 1);
    iters += st.steps;
    est = st.est;
    if (st.est <= st.tol_abs || st.breakdown || iters >= max_iters) break;
  }
  if (rel_est) *rel_est = est / bnorm;
  return iters;
}

}  // namespace dmg
