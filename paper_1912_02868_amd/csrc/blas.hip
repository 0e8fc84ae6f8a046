// Vector kernels of the Krylov solvers: Gram-Schmidt dot products and updates,
// norms, linear combinations and casts.  Reductions are deterministic: each
// workgroup writes its partial sums, and the last workgroup to finish (counted
// with one atomic ticket) adds the partials in workgroup order and runs the
// small epilogue of the step (Hessenberg entries, Givens update).
#include <algorithm>

#include "kernels.h"

namespace dmg {

constexpr int RB = 256;          // threads per reduction workgroup
constexpr int RW = RB / 64;      // wavefronts per reduction workgroup
constexpr int MAXRED = 128;      // largest reduction grid (the last workgroup adds <= RB partials per quantity)
constexpr int QB = 8;            // quantities whose loads are issued together
constexpr int NROT_LDS = 128;    // Givens rotations staged in LDS by the update

int red_blocks(int64_t n) {
  int64_t b = (n + RB - 1) / RB;
  if (b < 1) b = 1;
  if (b > MAXRED) b = MAXRED;
  return (int)b;
}

__device__ inline double2 wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// Sum `v` over the workgroup for quantity q; result valid through wg_result after a barrier.
__device__ inline void wg_accumulate(double2 (*lds)[MMAX + 2], int q, double2 v) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6][q] = v;
}

__device__ inline double2 wg_result(double2 (*lds)[MMAX + 2], int q) {
  double2 r = lds[0][q];
  for (int w = 1; w < RW; ++w) r = cadd(r, lds[w][q]);
  return r;
}

// Ticket: true in exactly one (the last) workgroup, after all partials are visible.
// The partial sums travel with device-scope atomic stores and loads, which go to the device's
// coherence point rather than a compute die's own L2: each wavefront waits for its own stores
// to complete before the workgroup barrier and the ticket, and the last workgroup loads the
// partials after its ticket returned.  No fence is needed, so no L2 write-back or invalidation
// (which a device-scope fence costs on every workgroup, and which would also evict the vectors
// the next kernels read).
__device__ inline void st_dev(double2* p, double2 v) {
  __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double2 ld_dev(const double2* p) {
  return mk(__hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
            __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ inline bool last_block(unsigned* counter) {
  __shared__ int am_last;
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's partial stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned t = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (t == gridDim.x * gridDim.y - 1) ? 1 : 0;
  }
  __syncthreads();
  if (am_last && threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return am_last != 0;
}

// Per-workgroup partial dots conj(V_i) . w for i < nv (and ||w||^2 as quantity nv when
// with_norm), QB quantities per pass so their loads are in flight together.  Leaves the
// workgroup sums in lds (read with wg_result after a barrier).
template <typename R>
__device__ void block_dots(const cx<R>* __restrict__ V, int64_t ld, int nv, const cx<R>* __restrict__ w, int64_t n,
                           bool with_norm, double2 (*lds)[MMAX + 2]) {
  const int64_t stride = (int64_t)gridDim.x * RB;
  const int64_t e0 = (int64_t)blockIdx.x * RB + threadIdx.x;
  for (int i0 = 0; i0 < nv; i0 += QB) {
    double2 acc[QB];
#pragma unroll
    for (int u = 0; u < QB; ++u) acc[u] = mk(0.0, 0.0);
    for (int64_t e = e0; e < n; e += stride) {
      const double2 wv = to_d(w[e]);
      double2 vv[QB];
#pragma unroll
      for (int u = 0; u < QB; ++u) vv[u] = (i0 + u < nv) ? to_d(V[(int64_t)(i0 + u) * ld + e]) : mk(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < QB; ++u) cfmac(acc[u], vv[u], wv);
    }
#pragma unroll
    for (int u = 0; u < QB; ++u)
      if (i0 + u < nv) wg_accumulate(lds, i0 + u, acc[u]);
  }
  if (with_norm) {
    double2 acc = mk(0.0, 0.0);
    for (int64_t e = e0; e < n; e += stride) acc.x += cabs2(to_d(w[e]));
    wg_accumulate(lds, nv, acc);
  }
}

// Publish the workgroup sums of quantities q < nq as partials[q][blockIdx].
__device__ inline void publish(double2 (*lds)[MMAX + 2], int nq, double2* partials) {
  __syncthreads();
  for (int q = threadIdx.x; q < nq; q += RB) st_dev(&partials[(int64_t)q * gridDim.x + blockIdx.x], wg_result(lds, q));
}

// In the last workgroup: res[q] = sum over workgroups of partials[q][b], in a fixed order,
// with all threads loading.  res is in LDS; ends with a barrier.
__device__ void last_sums(const double2* partials, int nq, double2 (*lds)[MMAX + 2], double2* res) {
  const int nblk = gridDim.x;
  const int t = threadIdx.x;
  for (int q0 = 0; q0 < nq; q0 += QB) {
    double2 v[QB];
#pragma unroll
    for (int u = 0; u < QB; ++u) v[u] = (q0 + u < nq && t < nblk) ? ld_dev(&partials[(int64_t)(q0 + u) * nblk + t]) : mk(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < QB; ++u)
      if (q0 + u < nq) wg_accumulate(lds, q0 + u, v[u]);
  }
  __syncthreads();
  for (int q = t; q < nq; q += RB) res[q] = wg_result(lds, q);
  __syncthreads();
}

// ---------------------------------------------------------------- Givens update
// Column j of the Hessenberg (already in ks->H) is rotated by the stored rotations and a
// new one that annihilates its subdiagonal; the right-hand side g follows.  All threads of
// the workgroup stage the column and the rotations in LDS; thread 0 does the serial part.
__device__ void givens_update(KState* ks, int j) {
  constexpr int LD = MMAX + 1;
  __shared__ double2 col[MMAX + 2];
  __shared__ double rcs[NROT_LDS];
  __shared__ double2 rss[NROT_LDS];
  __shared__ int rps[NROT_LDS];
  __shared__ double2 gg[2];
  const int t = threadIdx.x;
  const int nrot = ks->nrot;
  for (int i = t; i <= j + 1; i += RB) col[i] = ks->H[LD * j + i];
  for (int q = t; q < nrot && q < NROT_LDS; q += RB) {
    rcs[q] = ks->rot_c[q];
    rss[q] = ks->rot_s[q];
    rps[q] = ks->rot_p[q];
  }
  if (t == 0) {
    gg[0] = ks->g[j];
    gg[1] = ks->g[j + 1];
  }
  __syncthreads();
  if (t == 0) {
    for (int q = 0; q < nrot; ++q) {
      const bool in_lds = q < NROT_LDS;
      const int p = in_lds ? rps[q] : ks->rot_p[q];
      if (p + 1 > j + 1) continue;
      const double c = in_lds ? rcs[q] : ks->rot_c[q];
      const double2 s = in_lds ? rss[q] : ks->rot_s[q];
      const double2 a = col[p], b = col[p + 1];
      col[p] = cadd(cscale(a, c), cmul(s, b));
      col[p + 1] = csub(cscale(b, c), cmul(cconj(s), a));
    }
    // new rotation on rows (j, j+1) zeroing col[j+1]
    const double2 a = col[j], b = col[j + 1];
    const double na = sqrt(cabs2(a)), nb = sqrt(cabs2(b));
    double c;
    double2 s;
    if (nb == 0.0) {
      c = 1.0; s = mk(0.0, 0.0);
    } else if (na == 0.0) {
      c = 0.0; s = cscale(cconj(b), 1.0 / nb);
    } else {
      const double nr = sqrt(na * na + nb * nb);
      c = na / nr;
      s = cscale(cmul(cconj(b), a), 1.0 / (na * nr));
    }
    col[j] = cadd(cscale(a, c), cmul(s, b));
    col[j + 1] = mk(0.0, 0.0);
    const double2 gj = gg[0], gj1 = gg[1];
    const double2 ng0 = cadd(cscale(gj, c), cmul(s, gj1));
    const double2 ng1 = csub(cscale(gj1, c), cmul(cconj(s), gj));
    ks->g[j] = ng0;
    ks->g[j + 1] = ng1;
    ks->rot_p[nrot] = j;
    ks->rot_c[nrot] = c;
    ks->rot_s[nrot] = s;
    ks->nrot = nrot + 1;
    ks->est = sqrt(cabs2(ng1));
    ks->steps = j + 1;
  }
  __syncthreads();
  for (int i = t; i <= j + 1; i += RB) ks->R[LD * j + i] = col[i];
}

// ---------------------------------------------------------------- Arnoldi kernels
// (a) h_i = V_i^H w (i <= j) and ||w||^2; w is column j+1.
template <typename R>
__global__ void __launch_bounds__(RB) k_arn_dots1(const cx<R>* __restrict__ V, int64_t ld, int64_t n, int j,
                                                  KState* ks, double2* partials, unsigned* counter) {
  if (ks->done) return;
  __shared__ double2 lds[RW][MMAX + 2];
  __shared__ double2 res[MMAX + 2];
  const cx<R>* w = V + (int64_t)(j + 1) * ld;
  block_dots<R>(V, ld, j + 1, w, n, true, lds);
  publish(lds, j + 2, partials);
  if (!last_block(counter)) return;
  last_sums(partials, j + 2, lds, res);
  constexpr int LD = MMAX + 1;
  for (int q = threadIdx.x; q <= MMAX; q += RB) {
    if (q <= j) ks->H[LD * j + q] = res[q];
    else if (q > j + 1) ks->H[LD * j + q] = mk(0.0, 0.0);
  }
  if (threadIdx.x == 0) ks->wn0 = sqrt(res[j + 1].x);
}

// (b) w -= sum_i H[i, j] V_i; then h2_i = V_i^H w; H[i, j] += h2_i.
template <typename R>
__global__ void __launch_bounds__(RB) k_arn_update_dots2(cx<R>* __restrict__ V, int64_t ld, int64_t n, int j,
                                                         KState* ks, double2* partials, unsigned* counter) {
  if (ks->done) return;
  __shared__ double2 lds[RW][MMAX + 2];
  __shared__ double2 coef[MMAX + 2];
  constexpr int LD = MMAX + 1;
  for (int i = threadIdx.x; i <= j; i += RB) coef[i] = ks->H[LD * j + i];
  __syncthreads();
  cx<R>* w = V + (int64_t)(j + 1) * ld;
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double2 acc = to_d(w[e]);
    for (int i = 0; i <= j; ++i) acc = csub(acc, cmul(coef[i], to_d(V[(int64_t)i * ld + e])));
    w[e] = from_d<R>(acc);
  }
  block_dots<R>(V, ld, j + 1, w, n, false, lds);
  publish(lds, j + 1, partials);
  if (!last_block(counter)) return;
  last_sums(partials, j + 1, lds, coef);
  for (int q = threadIdx.x; q <= j; q += RB) {
    ks->h2[q] = coef[q];
    ks->H[LD * j + q] = cadd(ks->H[LD * j + q], coef[q]);
  }
}

// (c) w -= sum_i h2_i V_i; ||w|| -> H[j+1, j]; Givens update; convergence flag.
template <typename R>
__global__ void __launch_bounds__(RB) k_arn_update_norm(cx<R>* __restrict__ V, int64_t ld, int64_t n, int j,
                                                        KState* ks, double2* partials, unsigned* counter) {
  if (ks->done) return;
  __shared__ double2 lds[RW][MMAX + 2];
  __shared__ double2 coef[MMAX + 2];
  constexpr int LD = MMAX + 1;
  for (int i = threadIdx.x; i <= j; i += RB) coef[i] = ks->h2[i];
  __syncthreads();
  cx<R>* w = V + (int64_t)(j + 1) * ld;
  const int64_t stride = (int64_t)gridDim.x * RB;
  double2 nrm = mk(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double2 acc = to_d(w[e]);
    for (int i = 0; i <= j; ++i) acc = csub(acc, cmul(coef[i], to_d(V[(int64_t)i * ld + e])));
    const cx<R> st = from_d<R>(acc);
    w[e] = st;
    nrm.x += cabs2(to_d(st));
  }
  wg_accumulate(lds, 0, nrm);
  publish(lds, 1, partials);
  if (!last_block(counter)) return;
  last_sums(partials, 1, lds, coef);
  double hn = sqrt(coef[0].x);
  const bool brk = !(hn > 1e-12 * ks->wn0);
  if (brk) hn = 0.0;
  if (threadIdx.x == 0) ks->H[LD * j + j + 1] = mk(hn, 0.0);
  __syncthreads();
  givens_update(ks, j);
  if (threadIdx.x == 0) {
    if (brk) { ks->breakdown = 1; ks->est = 0.0; }
    if (brk || ks->est <= ks->tol_abs) ks->done = 1;
  }
}

// (d) V_{j+1} = w / h_{j+1, j}
template <typename R>
__global__ void __launch_bounds__(RB) k_arn_normalize(cx<R>* __restrict__ V, int64_t ld, int64_t n, int j,
                                                      const KState* ks) {
  if (ks->done && ks->breakdown) return;
  constexpr int LD = MMAX + 1;
  const double hn = ks->H[LD * j + j + 1].x;
  if (hn == 0.0) return;
  const double inv = 1.0 / hn;
  cx<R>* w = V + (int64_t)(j + 1) * ld;
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double2 v = to_d(w[e]);
    w[e] = from_d<R>(cscale(v, inv));
  }
}

// One-pass classical Gram-Schmidt with the Pythagorean norm, for Krylov solves that only
// precondition (the partial intermediate solve): (a1) h = V^H w and ||w||^2 in one reduction;
// the last workgroup forms hn^2 = ||w||^2 - ||h||^2 and, unless that cancels to eta ||w||^2 or
// less, stores h_{j+1,j} = hn and does the column's Givens update and convergence test as
// k_arn_update_norm does; (b1) w = (w - V h) / hn.  Where it cancels, ks->pass2 = 1, (b1) leaves
// w - V h unscaled and the caller runs the exact second pass (k_arn_dots2, k_arn_update_norm,
// k_arn_normalize).  In exact arithmetic the same column as the two-pass form.
template <typename R>
__global__ void __launch_bounds__(RB) k_arn_dots_all(const cx<R>* __restrict__ V, int64_t ld, int64_t n, int j,
                                                     KState* ks, double2* partials, unsigned* counter, double eta) {
  if (ks->done) return;
  __shared__ double2 lds[RW][MMAX + 2];
  __shared__ double2 res[MMAX + 2];
  const cx<R>* w = V + (int64_t)(j + 1) * ld;
  block_dots<R>(V, ld, j + 1, w, n, true, lds);
  publish(lds, j + 2, partials);
  if (!last_block(counter)) return;
  last_sums(partials, j + 2, lds, res);
  constexpr int LD = MMAX + 1;
  for (int q = threadIdx.x; q <= MMAX; q += RB) {
    if (q <= j) ks->H[LD * j + q] = res[q];
    else if (q > j + 1) ks->H[LD * j + q] = mk(0.0, 0.0);
  }
  __shared__ int one_pass;
  if (threadIdx.x == 0) {
    const double ww = res[j + 1].x;
    double hh = 0.0;
    for (int q = 0; q <= j; ++q) hh += cabs2(res[q]);
    const double hn2 = ww - hh;
    ks->wn0 = sqrt(ww);
    one_pass = hn2 > eta * ww ? 1 : 0;
    ks->pass2 = one_pass ? 0 : 1;
    if (one_pass) ks->H[LD * j + j + 1] = mk(sqrt(hn2), 0.0);
  }
  __syncthreads();
  if (!one_pass) return;
  givens_update(ks, j);
  if (threadIdx.x == 0 && ks->est <= ks->tol_abs) ks->done = 1;
}

template <typename R>
__global__ void __launch_bounds__(RB) k_arn_update1(cx<R>* __restrict__ V, int64_t ld, int64_t n, int j,
                                                    const KState* ks) {
  if (ks->done && ks->breakdown) return;
  __shared__ double2 coef[MMAX + 2];
  constexpr int LD = MMAX + 1;
  for (int i = threadIdx.x; i <= j; i += RB) coef[i] = ks->H[LD * j + i];
  __syncthreads();
  const double inv = ks->pass2 ? 1.0 : 1.0 / ks->H[LD * j + j + 1].x;
  cx<R>* w = V + (int64_t)(j + 1) * ld;
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double2 acc = to_d(w[e]);
    for (int i = 0; i <= j; ++i) acc = csub(acc, cmul(coef[i], to_d(V[(int64_t)i * ld + e])));
    w[e] = from_d<R>(cscale(acc, inv));
  }
}

// second pass after k_arn_update1 left w - V h: h2 = V^H w, H[i, j] += h2_i
template <typename R>
__global__ void __launch_bounds__(RB) k_arn_dots2(const cx<R>* __restrict__ V, int64_t ld, int64_t n, int j,
                                                  KState* ks, double2* partials, unsigned* counter) {
  if (ks->done) return;
  __shared__ double2 lds[RW][MMAX + 2];
  __shared__ double2 coef[MMAX + 2];
  constexpr int LD = MMAX + 1;
  const cx<R>* w = V + (int64_t)(j + 1) * ld;
  block_dots<R>(V, ld, j + 1, w, n, false, lds);
  publish(lds, j + 1, partials);
  if (!last_block(counter)) return;
  last_sums(partials, j + 1, lds, coef);
  for (int q = threadIdx.x; q <= j; q += RB) {
    ks->h2[q] = coef[q];
    ks->H[LD * j + q] = cadd(ks->H[LD * j + q], coef[q]);
  }
}

template <typename R>
void launch_arnoldi_orth1(hipStream_t s, cx<R>* V, int64_t ld, int64_t n, int j, KState* ks, double2* partials,
                          unsigned* counter) {
  const int G = red_blocks(n);
  // DMG_ARNOLDI_TWO_PASS=1 takes the second pass at every step (read at each call)
  const char* e = getenv("DMG_ARNOLDI_TWO_PASS");
  const double eta = (e && *e && *e != '0') ? 2.0 : (sizeof(R) == sizeof(float) ? 1e-4 : 1e-8);
  hipLaunchKernelGGL(k_arn_dots_all<R>, dim3(G), dim3(RB), 0, s, V, ld, n, j, ks, partials, counter, eta);
  hipLaunchKernelGGL(k_arn_update1<R>, dim3(G), dim3(RB), 0, s, V, ld, n, j, (const KState*)ks);
  DMG_LAUNCH_CHECK();
}

template <typename R>
void launch_arnoldi_pass2(hipStream_t s, cx<R>* V, int64_t ld, int64_t n, int j, KState* ks, double2* partials,
                          unsigned* counter) {
  const int G = red_blocks(n);
  hipLaunchKernelGGL(k_arn_dots2<R>, dim3(G), dim3(RB), 0, s, V, ld, n, j, ks, partials, counter);
  hipLaunchKernelGGL(k_arn_update_norm<R>, dim3(G), dim3(RB), 0, s, V, ld, n, j, ks, partials, counter);
  hipLaunchKernelGGL(k_arn_normalize<R>, dim3(G), dim3(RB), 0, s, V, ld, n, j, ks);
  DMG_LAUNCH_CHECK();
}

template <typename R>
void launch_arnoldi_orth(hipStream_t s, cx<R>* V, int64_t ld, int64_t n, int j, KState* ks, double2* partials,
                         unsigned* counter) {
  const int G = red_blocks(n);
  hipLaunchKernelGGL(k_arn_dots1<R>, dim3(G), dim3(RB), 0, s, V, ld, n, j, ks, partials, counter);
  hipLaunchKernelGGL(k_arn_update_dots2<R>, dim3(G), dim3(RB), 0, s, V, ld, n, j, ks, partials, counter);
  hipLaunchKernelGGL(k_arn_update_norm<R>, dim3(G), dim3(RB), 0, s, V, ld, n, j, ks, partials, counter);
  hipLaunchKernelGGL(k_arn_normalize<R>, dim3(G), dim3(RB), 0, s, V, ld, n, j, ks);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- two-step GMRES smoother
// GMRES(2) from x0 = 0 minimises || v - A (c0 v + c1 A v) || over (c0, c1): the least-squares
// fit of v by [w1, w2] = [A v, A^2 v].  One reduction forms the Gram entries
// (w1.w1, w1.w2, w2.w2, w1.v, w2.v); the last workgroup solves the 2 x 2 normal equations
// (falling back to the one-term fit when [w1, w2] is numerically rank one).
// coef receives c0, c1 (double2 each).
template <typename R>
__global__ void __launch_bounds__(RB) k_smooth2_dots(const cx<R>* __restrict__ v, const cx<R>* __restrict__ w1,
                                                     const cx<R>* __restrict__ w2, int64_t n, double2* coef,
                                                     double2* partials, unsigned* counter) {
  __shared__ double2 lds[RW][MMAX + 2];
  __shared__ double2 res[8];
  const int64_t stride = (int64_t)gridDim.x * RB;
  double2 a11 = mk(0.0, 0.0), a12 = mk(0.0, 0.0), a22 = mk(0.0, 0.0), b1 = mk(0.0, 0.0), b2 = mk(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    const double2 vv = to_d(v[e]), x1 = to_d(w1[e]), x2 = to_d(w2[e]);
    a11.x += cabs2(x1);
    cfmac(a12, x1, x2);
    a22.x += cabs2(x2);
    cfmac(b1, x1, vv);
    cfmac(b2, x2, vv);
  }
  wg_accumulate(lds, 0, a11);
  wg_accumulate(lds, 1, a12);
  wg_accumulate(lds, 2, a22);
  wg_accumulate(lds, 3, b1);
  wg_accumulate(lds, 4, b2);
  publish(lds, 5, partials);
  if (!last_block(counter)) return;
  last_sums(partials, 5, lds, res);
  if (threadIdx.x == 0) {
    const double g11 = res[0].x, g22 = res[2].x;
    const double2 g12 = res[1], r1 = res[3], r2 = res[4];
    double2 c0 = mk(0.0, 0.0), c1 = mk(0.0, 0.0);
    const double det = g11 * g22 - cabs2(g12);  // Gram determinant (>= 0)
    if (g11 > 0.0 && det > 1e-13 * g11 * g22) {
      // [g11 g12; conj(g12) g22] [c0; c1] = [r1; r2]
      const double inv = 1.0 / det;
      c0 = cscale(csub(cscale(r1, g22), cmul(g12, r2)), inv);
      c1 = cscale(csub(cscale(r2, g11), cmul(cconj(g12), r1)), inv);
    } else if (g11 > 0.0) {
      c0 = cscale(r1, 1.0 / g11);
    }
    coef[0] = c0;
    coef[1] = c1;
  }
}

// y = c0 v + c1 w1;  r = v - c0 w1 - c1 w2 (r optional)
template <typename R>
__global__ void __launch_bounds__(RB) k_smooth2_combine(const cx<R>* __restrict__ v, const cx<R>* __restrict__ w1,
                                                        const cx<R>* __restrict__ w2, int64_t n, const double2* coef,
                                                        cx<R>* __restrict__ y, cx<R>* __restrict__ r) {
  const double2 c0 = coef[0], c1 = coef[1];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const double2 vv = to_d(v[e]), x1 = to_d(w1[e]);
    double2 yv = mk(0.0, 0.0);
    cfma(yv, c0, vv);
    cfma(yv, c1, x1);
    y[e] = from_d<R>(yv);
    if (r) {
      double2 rv = vv;
      rv = csub(rv, cmul(c0, x1));
      rv = csub(rv, cmul(c1, to_d(w2[e])));
      r[e] = from_d<R>(rv);
    }
  }
}

template <typename R>
void launch_smooth2(hipStream_t s, const cx<R>* v, const cx<R>* w1, const cx<R>* w2, int64_t n, double2* coef,
                    cx<R>* y, cx<R>* r, double2* partials, unsigned* counter) {
  hipLaunchKernelGGL(k_smooth2_dots<R>, dim3(red_blocks(n)), dim3(RB), 0, s, v, w1, w2, n, coef, partials, counter);
  const int64_t nb = std::min<int64_t>((n + RB - 1) / RB, 2048);
  hipLaunchKernelGGL(k_smooth2_combine<R>, dim3((unsigned)nb), dim3(RB), 0, s, v, w1, w2, n, (const double2*)coef, y,
                     r);
  DMG_LAUNCH_CHECK();
}

// z = a x + b y  (separate output)
template <typename R>
__global__ void k_axpbyz(int64_t n, double a, const cx<R>* __restrict__ x, double b, const cx<R>* __restrict__ y,
                         cx<R>* __restrict__ z) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const double2 xv = to_d(x[e]), yv = to_d(y[e]);
    z[e] = from_d<R>(mk(a * xv.x + b * yv.x, a * xv.y + b * yv.y));
  }
}

template <typename R>
void launch_axpbyz(hipStream_t s, int64_t n, double a, const cx<R>* x, double b, const cx<R>* y, cx<R>* z) {
  const int64_t nb = std::min<int64_t>((n + RB - 1) / RB, 2048);
  hipLaunchKernelGGL(k_axpbyz<R>, dim3((unsigned)nb), dim3(RB), 0, s, n, a, x, b, y, z);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- combinations
template <typename R>
__global__ void __launch_bounds__(RB) k_combine(cx<R>* __restrict__ x, const cx<R>* __restrict__ V, int64_t ld,
                                                int64_t n, const KState* ks, int use_u, int accumulate) {
  __shared__ double2 coef[MMAX + 2];
  const int cnt = ks->steps + (use_u ? 1 : 0);
  const double2* src = use_u ? ks->u : ks->y;
  for (int i = threadIdx.x; i < cnt; i += RB) coef[i] = src[i];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double2 acc = accumulate ? to_d(x[e]) : mk(0.0, 0.0);
    for (int i = 0; i < cnt; ++i) cfma(acc, coef[i], to_d(V[(int64_t)i * ld + e]));
    x[e] = from_d<R>(acc);
  }
}

template <typename R, typename RX>
void launch_combine(hipStream_t s, cx<RX>* x, const cx<R>* V, int64_t ld, int64_t n, const KState* ks, int use_u,
                    int accumulate) {
  static_assert(sizeof(R) == sizeof(RX), "combine: same precision");
  hipLaunchKernelGGL(k_combine<R>, dim3(red_blocks(n)), dim3(RB), 0, s, (cx<R>*)x, V, ld, n, ks, use_u, accumulate);
  DMG_LAUNCH_CHECK();
}

template <typename R>
__global__ void k_axpby(int64_t n, double a, const cx<R>* __restrict__ x, double b, cx<R>* __restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const double2 xv = to_d(x[e]), yv = to_d(y[e]);
    y[e] = from_d<R>(mk(a * xv.x + b * yv.x, a * xv.y + b * yv.y));
  }
}

template <typename R>
void launch_axpby(hipStream_t s, int64_t n, double a, const cx<R>* x, double b, cx<R>* y) {
  hipLaunchKernelGGL(k_axpby<R>, dim3(red_blocks(n)), dim3(RB), 0, s, n, a, x, b, y);
  DMG_LAUNCH_CHECK();
}

template <typename R>
void launch_xmy(hipStream_t s, int64_t n, const cx<R>* x, cx<R>* y) {
  launch_axpby<R>(s, n, 1.0, x, -1.0, y);
}

__global__ void k_d2f(int64_t n, const double2* __restrict__ x, float2* __restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
    y[e] = make_float2((float)x[e].x, (float)x[e].y);
}
__global__ void k_f2d(int64_t n, const float2* __restrict__ x, double2* __restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
    y[e] = make_double2((double)x[e].x, (double)x[e].y);
}
void launch_cast_d2f(hipStream_t s, int64_t n, const double2* x, float2* y) {
  hipLaunchKernelGGL(k_d2f, dim3(red_blocks(n)), dim3(RB), 0, s, n, x, y);
  DMG_LAUNCH_CHECK();
}
void launch_cast_f2d(hipStream_t s, int64_t n, const float2* x, double2* y) {
  hipLaunchKernelGGL(k_f2d, dim3(red_blocks(n)), dim3(RB), 0, s, n, x, y);
  DMG_LAUNCH_CHECK();
}
void launch_d2f(hipStream_t s, int64_t n, const double2* x, float2* y) { launch_cast_d2f(s, n, x, y); }

// ---------------------------------------------------------------- norms and cycle start
// mode 0: out[0] = ||x||^2
// mode 1: start a cycle from x: beta = ||x||, state reset, g = c = beta e1,
//         tol_abs = tol_rel * bnorm (bnorm kept from an earlier call)
// mode 2: as mode 1 and first set bnorm = ||x|| (the right-hand side of the solve)
// mode 3: bnorm = ||x|| only
template <typename R>
__global__ void __launch_bounds__(RB) k_norm2(int64_t n, const cx<R>* __restrict__ x, double* out, KState* ks,
                                              double tol_rel, int mode, double2* partials, unsigned* counter) {
  __shared__ double2 lds[RW][MMAX + 2];
  __shared__ double2 res[2];
  const int64_t stride = (int64_t)gridDim.x * RB;
  double2 acc = mk(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) acc.x += cabs2(to_d(x[e]));
  wg_accumulate(lds, 0, acc);
  publish(lds, 1, partials);
  if (!last_block(counter)) return;
  last_sums(partials, 1, lds, res);
  if (threadIdx.x == 0) {
    const double s2 = res[0].x;
    if (mode == 0) { out[0] = s2; return; }
    const double beta = sqrt(s2);
    if (mode == 2 || mode == 3) ks->bnorm = beta;
    if (mode == 3) return;
    ks->beta = beta;
    ks->est = beta;
    ks->tol_abs = tol_rel * ks->bnorm;
    ks->steps = 0;
    ks->nrot = 0;
    ks->breakdown = 0;
    ks->done = (beta == 0.0 || beta <= ks->tol_abs) ? 1 : 0;
  }
  if (mode == 1 || mode == 2) {
    const double beta = sqrt(res[0].x);
    for (int i = threadIdx.x; i <= MMAX; i += RB) {
      ks->g[i] = (i == 0) ? mk(beta, 0.0) : mk(0.0, 0.0);
      ks->c[i] = (i == 0) ? mk(beta, 0.0) : mk(0.0, 0.0);
    }
  }
}

template <typename R>
void launch_norm2(hipStream_t s, int64_t n, const cx<R>* x, double* out, double2* partials, unsigned* counter) {
  hipLaunchKernelGGL(k_norm2<R>, dim3(red_blocks(n)), dim3(RB), 0, s, n, x, out, (KState*)nullptr, 0.0, 0, partials,
                     counter);
  DMG_LAUNCH_CHECK();
}

template <typename R>
void launch_set_bnorm(hipStream_t s, int64_t n, const cx<R>* x, KState* ks, double2* partials, unsigned* counter) {
  hipLaunchKernelGGL(k_norm2<R>, dim3(red_blocks(n)), dim3(RB), 0, s, n, x, (double*)nullptr, ks, 0.0, 3, partials,
                     counter);
  DMG_LAUNCH_CHECK();
}

// y = x / beta with beta = ks->beta (zero vector if beta == 0)
template <typename R>
__global__ void k_scale_beta(int64_t n, const cx<R>* __restrict__ x, cx<R>* __restrict__ y, const KState* ks) {
  const double beta = ks->beta;
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
    y[e] = from_d<R>(cscale(to_d(x[e]), inv));
}

template <typename R>
void launch_cycle_start(hipStream_t s, const cx<R>* r, cx<R>* V0, int64_t n, KState* ks, double tol_rel,
                        int set_bnorm, double2* partials, unsigned* counter) {
  hipLaunchKernelGGL(k_norm2<R>, dim3(red_blocks(n)), dim3(RB), 0, s, n, r, (double*)nullptr, ks, tol_rel,
                     set_bnorm ? 2 : 1, partials, counter);
  hipLaunchKernelGGL(k_scale_beta<R>, dim3(red_blocks(n)), dim3(RB), 0, s, n, r, V0, (const KState*)ks);
  DMG_LAUNCH_CHECK();
}

// y = x * scale[0]  (invert_sqrt: y = x / sqrt(scale[0]))
template <typename R>
__global__ void k_scale_dev(int64_t n, const cx<R>* __restrict__ x, cx<R>* __restrict__ y, const double* scale,
                            int invert_sqrt) {
  double f = scale[0];
  if (invert_sqrt) f = f > 0.0 ? 1.0 / sqrt(f) : 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
    y[e] = from_d<R>(cscale(to_d(x[e]), f));
}

// status[0] = 1 unless after > rel2 * before (squared norms of a vector before and after it was
// orthogonalised against earlier ones: the set has lost rank)
__global__ void k_rank_test(const double* before, const double* after, double rel2, int* status) {
  const double b = before[0], a = after[0];
  if (!(a > rel2 * b) || !(a > 0.0)) status[0] = 1;
}

void launch_rank_test(hipStream_t s, const double* before, const double* after, double rel2, int* status) {
  hipLaunchKernelGGL(k_rank_test, dim3(1), dim3(1), 0, s, before, after, rel2, status);
  DMG_LAUNCH_CHECK();
}

template <typename R>
void launch_scale_dev(hipStream_t s, int64_t n, const cx<R>* x, cx<R>* y, const double* scale, int invert_sqrt) {
  hipLaunchKernelGGL(k_scale_dev<R>, dim3(red_blocks(n)), dim3(RB), 0, s, n, x, y, scale, invert_sqrt);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- multi-dot / multi-axpy / basis rotation
template <typename R>
__global__ void __launch_bounds__(RB) k_multidot(const cx<R>* __restrict__ V, int64_t ld, int nv,
                                                 const cx<R>* __restrict__ w, int64_t n, double2* out,
                                                 double2* partials, unsigned* counter) {
  __shared__ double2 lds[RW][MMAX + 2];
  __shared__ double2 res[MMAX + 2];
  block_dots<R>(V, ld, nv, w, n, false, lds);
  publish(lds, nv, partials);
  if (!last_block(counter)) return;
  last_sums(partials, nv, lds, res);
  for (int q = threadIdx.x; q < nv; q += RB) out[q] = res[q];
}

template <typename R>
void launch_multidot(hipStream_t s, const cx<R>* V, int64_t ld, int nv, const cx<R>* w, int64_t n, double2* out,
                     double2* partials, unsigned* counter) {
  hipLaunchKernelGGL(k_multidot<R>, dim3(red_blocks(n)), dim3(RB), 0, s, V, ld, nv, w, n, out, partials, counter);
  DMG_LAUNCH_CHECK();
}

template <typename R>
__global__ void __launch_bounds__(RB) k_multi_axpy(cx<R>* __restrict__ w, const cx<R>* __restrict__ V, int64_t ld,
                                                   int nv, const double2* coef_g, int64_t n, double sign) {
  __shared__ double2 coef[MMAX + 2];
  for (int i = threadIdx.x; i < nv; i += RB) coef[i] = cscale(coef_g[i], sign);
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double2 acc = to_d(w[e]);
    for (int i = 0; i < nv; ++i) acc = csub(acc, cmul(coef[i], to_d(V[(int64_t)i * ld + e])));
    w[e] = from_d<R>(acc);
  }
}

template <typename R>
void launch_multi_axpy(hipStream_t s, cx<R>* w, const cx<R>* V, int64_t ld, int nv, const double2* coef, int64_t n,
                       double sign) {
  hipLaunchKernelGGL(k_multi_axpy<R>, dim3(red_blocks(n)), dim3(RB), 0, s, w, V, ld, nv, coef, n, sign);
  DMG_LAUNCH_CHECK();
}

// Vout[:, jc] = sum_i P[i, jc] Vin[:, i]: one thread per (entry, output column), the sum in i order.
template <typename R>
__global__ void __launch_bounds__(RB) k_basis_rotate(const cx<R>* __restrict__ Vin, cx<R>* __restrict__ Vout,
                                                     int64_t ld, int64_t n, const double2* __restrict__ P, int ldp,
                                                     int rows, int cols) {
  const int jc = blockIdx.y;
  const double2* pc = P + (int64_t)ldp * jc;
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double2 acc = mk(0.0, 0.0);
    for (int i = 0; i < rows; ++i) cfma(acc, pc[i], to_d(Vin[(int64_t)i * ld + e]));
    Vout[(int64_t)jc * ld + e] = from_d<R>(acc);
  }
}

template <typename R>
void launch_basis_rotate(hipStream_t s, const cx<R>* Vin, cx<R>* Vout, int64_t ld, int64_t n, const double2* P,
                         int ldp, int rows, int cols) {
  int64_t gx = (n + RB - 1) / RB;
  if (gx > 1024) gx = 1024;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_basis_rotate<R>, dim3((unsigned)gx, (unsigned)cols), dim3(RB), 0, s, Vin, Vout, ld, n, P, ldp,
                     rows, cols);
  DMG_LAUNCH_CHECK();
}

#define INST(R)                                                                                                     \
  template void launch_arnoldi_orth<R>(hipStream_t, cx<R>*, int64_t, int64_t, int, KState*, double2*, unsigned*); \
  template void launch_arnoldi_orth1<R>(hipStream_t, cx<R>*, int64_t, int64_t, int, KState*, double2*, unsigned*); \
  template void launch_arnoldi_pass2<R>(hipStream_t, cx<R>*, int64_t, int64_t, int, KState*, double2*, unsigned*); \
  template void launch_combine<R, R>(hipStream_t, cx<R>*, const cx<R>*, int64_t, int64_t, const KState*, int, int); \
  template void launch_axpby<R>(hipStream_t, int64_t, double, const cx<R>*, double, cx<R>*);                       \
  template void launch_xmy<R>(hipStream_t, int64_t, const cx<R>*, cx<R>*);                                         \
  template void launch_norm2<R>(hipStream_t, int64_t, const cx<R>*, double*, double2*, unsigned*);                  \
  template void launch_cycle_start<R>(hipStream_t, const cx<R>*, cx<R>*, int64_t, KState*, double, int, double2*,  \
                                      unsigned*);                                                                   \
  template void launch_set_bnorm<R>(hipStream_t, int64_t, const cx<R>*, KState*, double2*, unsigned*);              \
  template void launch_multidot<R>(hipStream_t, const cx<R>*, int64_t, int, const cx<R>*, int64_t, double2*,       \
                                   double2*, unsigned*);                                                            \
  template void launch_multi_axpy<R>(hipStream_t, cx<R>*, const cx<R>*, int64_t, int, const double2*, int64_t,     \
                                     double);                                                                       \
  template void launch_basis_rotate<R>(hipStream_t, const cx<R>*, cx<R>*, int64_t, int64_t, const double2*, int,   \
                                       int, int);                                                                   \
  template void launch_scale_dev<R>(hipStream_t, int64_t, const cx<R>*, cx<R>*, const double*, int);              \
  template void launch_smooth2<R>(hipStream_t, const cx<R>*, const cx<R>*, const cx<R>*, int64_t, double2*, cx<R>*, \
                                  cx<R>*, double2*, unsigned*);                                                    \
  template void launch_axpbyz<R>(hipStream_t, int64_t, double, const cx<R>*, double, const cx<R>*, cx<R>*);
INST(double)
INST(float)
#undef INST

}  // namespace dmg
