// Multi-right-hand-side kernels of the lockstep solver (layout and state in mrhs.h).
// Every reduction is deterministic and runs in two launches: each workgroup reduces
// its threads in a fixed order into partials, then one workgroup per right-hand side
// adds the partials in a fixed order and applies the small-dense step for that
// right-hand side.  Right-hand sides never mix: a thread owns one right-hand side
// r = threadIdx.x mod nb throughout a kernel.
#include <algorithm>
#include <array>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>

#include "mrhs.h"

namespace dmg {

constexpr int BT = 256;      // threads of the vector and reduction kernels
constexpr int BMAXBLK = 512; // most workgroups of a reduction

int bred_blocks(int64_t N) {
  int64_t b = (N + BT * 2 - 1) / (BT * 2);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, BMAXBLK));
}
size_t bred_partials(int nb) { return (size_t)BMAXBLK * MQ * nb; }


static inline int vec_blocks(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>((N + BT - 1) / BT, 4096)); }

__device__ inline double2 bcdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Block partials of the per-thread accumulators acc[q], q < nq, into
// part[(r * nq + q) * G + block] (G workgroups, so that the second phase reads each
// right-hand side's partials contiguously); threads with the same r are added in thread order.
template <int NQ>
__device__ void b_publish(const double2 (&acc)[NQ], int nq, int nb, double2* part) {
  __shared__ double2 red[4][BT];
  const int t = threadIdx.x;
  const int per = BT / nb;
#pragma unroll
  for (int q0 = 0; q0 < NQ; q0 += 4) {
    if (q0 < nq) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q0 + u < NQ) red[u][t] = acc[q0 + u];
      __syncthreads();
      if (t < 4 * nb) {
        const int u = t / nb, r = t % nb;
        if (q0 + u < nq) {
          double2 s = red[u][r];
          for (int k = 1; k < per; ++k) s = cadd(s, red[u][k * nb + r]);
          part[((int64_t)r * nq + q0 + u) * gridDim.x + blockIdx.x] = s;
        }
      }
      __syncthreads();
    }
  }
}

// Second phase of every batched reduction: one workgroup per right-hand side adds the
// workgroups' partials of each quantity (4 lanes per quantity, then the lanes in
// order) and applies the step's small-dense epilogue to that right-hand side.
enum FinMode { FIN_NORM0, FIN_NORM3, FIN_START, FIN_ARN1, FIN_ARN2, FIN_SMOOTH2, FIN_PROJ };

struct FinArgs {
  int mode, nq, nblk, nb, j, k;
  double tol_rel;
  int bnorm_too;  // FIN_START: also record bnorm = beta
  double* out;
  double2* coef;
  const double2* M;
  const double2* Pi;
  double eta;     // FIN_ARN1: cancellation threshold of the one-pass norm
  int* anyp2;     // FIN_ARN1: set when some right-hand side needs a second pass
};

constexpr int LDH = MB + 1;

__device__ void fin_start(BS& b, double s2, const FinArgs& a) {
  const double beta = sqrt(s2);
  if (a.bnorm_too) b.bnorm = beta;
  b.steps = 0;
  b.brk = 0;
  b.pass2 = 0;
  b.tol_abs = a.tol_rel * b.bnorm;
  if (!b.active) {
    b.beta = 0.0;
    b.est = 0.0;
    b.done = 1;
  } else {
    b.beta = beta;
    b.est = beta;
    b.done = (beta == 0.0 || beta <= b.tol_abs || b.cap < 1) ? 1 : 0;
  }
}

// Per right-hand-side state the Givens epilogue reads, staged in LDS at the start of the
// second phase so that its loads overlap those of the partials.
struct FinStage {
  double rc[MB];
  double2 rs[MB];
  double2 g[2];   // g[j], g[j + 1]
  double tol_abs, wn0;
  int cap, done, pass2;
};

// column j: rotate by the cycle's rotations, annihilate the subdiagonal, update g.  Called by
// every thread of the workgroup with the same arguments; the column (col[i], i <= j) is in
// LDS and one thread runs the serial rotation chain.
__device__ void fin_givens(BS& b, int j, double hn_sq, double wn0, double2* col, const FinStage& st) {
  const int t = threadIdx.x;
  if (t == 0) {
    double hn = sqrt(hn_sq);
    const bool brk = !(hn > 1e-12 * wn0);
    if (brk) hn = 0.0;
    b.H[LDH * j + j + 1] = mk(hn, 0.0);
    col[j + 1] = mk(hn, 0.0);
    for (int q = 0; q < j; ++q) {
      const double c = st.rc[q];
      const double2 sn = st.rs[q];
      const double2 x = col[q], y = col[q + 1];
      col[q] = cadd(cscale(x, c), cmul(sn, y));
      col[q + 1] = csub(cscale(y, c), cmul(cconj(sn), x));
    }
    const double2 x = col[j], y = col[j + 1];
    const double na = sqrt(cabs2(x)), ny = sqrt(cabs2(y));
    double c;
    double2 sn;
    if (ny == 0.0) {
      c = 1.0;
      sn = mk(0.0, 0.0);
    } else if (na == 0.0) {
      c = 0.0;
      sn = cscale(cconj(y), 1.0 / ny);
    } else {
      const double nr = sqrt(na * na + ny * ny);
      c = na / nr;
      sn = cscale(cmul(cconj(y), x), 1.0 / (na * nr));
    }
    col[j] = cadd(cscale(x, c), cmul(sn, y));
    col[j + 1] = mk(0.0, 0.0);
    const double2 gj = st.g[0], gj1 = st.g[1];
    b.g[j] = cadd(cscale(gj, c), cmul(sn, gj1));
    const double2 ng1 = csub(cscale(gj1, c), cmul(cconj(sn), gj));
    b.g[j + 1] = ng1;
    b.rc[j] = c;
    b.rs[j] = sn;
    double est = sqrt(cabs2(ng1));
    b.steps = j + 1;
    if (brk) {
      b.brk = 1;
      est = 0.0;
    }
    b.est = est;
    if (brk || est <= st.tol_abs || j + 1 >= st.cap) b.done = 1;
  }
  __syncthreads();
  for (int i = t; i <= j + 1; i += BT) b.Rm[LDH * j + i] = col[i];
}

__global__ void __launch_bounds__(BT) kb_final(const double2* __restrict__ part, BS* bs, FinArgs a) {
  static_assert(BMAXBLK <= 2 * BT, "at most two partials per thread and quantity");
  const int r = blockIdx.x, t = threadIdx.x;
  const bool skip = a.mode == FIN_ARN1                           ? lanes_all_done(bs, a.nb)
                    : a.mode == FIN_ARN2                         ? !*a.anyp2
                                                                 : false;
  if (skip) return;  // the same for every thread (no barrier has been passed yet)
  // Each thread adds the partials t and t + BT of every quantity (contiguous per quantity, so
  // a wavefront's loads coalesce; all loads are issued before the first add); a fixed shuffle
  // tree adds the 64 lanes of a wavefront and the wavefronts' sums are added in order.
  __shared__ double2 wsum[BT / 64][MQ];
  __shared__ double2 tot[64];
  __shared__ FinStage st;
  const double2* pr = part + (int64_t)r * a.nq * a.nblk;
  const bool h0 = t < a.nblk, h1 = t + BT < a.nblk;
  double2 sq[MQ];
#pragma unroll
  for (int q = 0; q < MQ; ++q) {
    double2 v0 = mk(0.0, 0.0), v1 = mk(0.0, 0.0);
    if (q < a.nq) {
      if (h0) v0 = pr[(int64_t)q * a.nblk + t];
      if (h1) v1 = pr[(int64_t)q * a.nblk + t + BT];
    }
    sq[q] = cadd(v0, v1);
  }
  BS& b = bs[r];
  const int j = a.j;
  if (a.mode == FIN_ARN1 || a.mode == FIN_ARN2) {
    if (t < j) {
      st.rc[t] = b.rc[t];
      st.rs[t] = b.rs[t];
    } else if (t == MB) {
      st.g[0] = b.g[j];
      st.g[1] = b.g[j + 1];
    } else if (t == MB + 1) {
      st.tol_abs = b.tol_abs;
      st.wn0 = b.wn0;
      st.cap = b.cap;
      st.done = b.done;
      st.pass2 = b.pass2;
    }
  }
#pragma unroll
  for (int q = 0; q < MQ; ++q) {
    if (q < a.nq) {
      double2 v = sq[q];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        v.x += __shfl_down(v.x, off);
        v.y += __shfl_down(v.y, off);
      }
      if ((t & 63) == 0) wsum[t >> 6][q] = v;
    }
  }
  __syncthreads();
  if (t < a.nq) {
    double2 v = wsum[0][t];
#pragma unroll
    for (int w = 1; w < BT / 64; ++w) v = cadd(v, wsum[w][t]);
    tot[t] = v;
  }
  __syncthreads();
  if (a.mode == FIN_SMOOTH2) {
    // two-step smoother: least-squares fit of v by [w1, w2] from the Gram entries
    if (t == 0) {
      const double g11 = tot[0].x, g22 = tot[2].x;
      const double2 g12 = tot[1], r1 = tot[3], r2 = tot[4];
      double2 c0 = mk(0.0, 0.0), c1 = mk(0.0, 0.0);
      const double det = g11 * g22 - cabs2(g12);  // Gram determinant (>= 0)
      if (g11 > 0.0 && det > 1e-13 * g11 * g22) {
        const double inv = 1.0 / det;
        c0 = cscale(csub(cscale(r1, g22), cmul(g12, r2)), inv);
        c1 = cscale(csub(cscale(r2, g11), cmul(cconj(g12), r1)), inv);
      } else if (g11 > 0.0) {
        c0 = cscale(r1, 1.0 / g11);
      }
      a.coef[2 * r] = c0;
      a.coef[2 * r + 1] = c1;
    }
    return;
  }
  switch (a.mode) {
    case FIN_NORM0:
      if (t == 0) a.out[r] = tot[0].x;
      break;
    case FIN_NORM3:
      if (t == 0) b.bnorm = sqrt(tot[0].x);
      break;
    case FIN_START:
      for (int i = t; i <= MB; i += BT) b.g[i] = b.c[i] = (i == 0) ? mk(sqrt(tot[0].x), 0.0) : mk(0.0, 0.0);
      if (t == 0) fin_start(b, tot[0].x, a);
      break;
    case FIN_ARN1: {
      // h = V^H w and ||w||^2: keep h as column j; one-pass norm ||w||^2 - ||h||^2 unless it
      // cancels, then the Givens update at once, else flag a second pass
      __shared__ double2 col[MB + 2];
      __shared__ double rest_s, wn0_s;
      __shared__ int one_s;
      if (!st.done) {
        for (int i = t; i <= MB; i += BT) {
          if (i <= j) {
            b.H[LDH * j + i] = tot[i];
            col[i] = tot[i];
          } else if (i > j + 1) {
            b.H[LDH * j + i] = mk(0.0, 0.0);
          }
        }
        if (t == 0) {
          const double ww = tot[j + 1].x;
          double hh = 0.0;
          for (int i = 0; i <= j; ++i) hh += cabs2(tot[i]);
          const double wn0 = sqrt(ww);
          b.wn0 = wn0;
          wn0_s = wn0;
          const double rest = ww - hh;
          one_s = rest > a.eta * ww ? 1 : 0;
          rest_s = rest;
          if (one_s) {
            b.pass2 = 0;
          } else {
            b.pass2 = 1;
            atomicOr(a.anyp2, 1);
          }
        }
        __syncthreads();
        if (one_s) fin_givens(b, j, rest_s, wn0_s, col, st);
      }
      break;
    }
    case FIN_ARN2: {
      // second pass: H(:, j) += h2, norm ||w||^2 - ||h2||^2 (no cancellation after the first
      // pass), then the Givens update; the next kernel subtracts V h2 and normalises
      __shared__ double2 col2[MB + 2];
      __shared__ double rest2;
      if (st.pass2 == 1) {
        for (int i = t; i <= j; i += BT) {
          const double2 hij = cadd(b.H[LDH * j + i], tot[i]);
          b.h2[i] = tot[i];
          b.H[LDH * j + i] = hij;
          col2[i] = hij;
        }
        if (t == 0) {
          double hh = 0.0;
          for (int i = 0; i <= j; ++i) hh += cabs2(tot[i]);
          rest2 = tot[j + 1].x - hh;
          b.pass2 = 2;
        }
        __syncthreads();
        fin_givens(b, j, rest2 > 0.0 ? rest2 : 0.0, st.wn0, col2, st);
      }
      break;
    }
    case FIN_PROJ:
      if (b.active) {
        // y_i = sum_l M[i + k l] c_l (i < k), u_i = sum_l Pi[i + (k+1) l] c_l (i <= k)
        const int k = a.k;
        for (int i = t; i < 2 * k + 1; i += BT) {
          double2 acc = mk(0.0, 0.0);
          if (i < k) {
            for (int l = 0; l <= k; ++l) cfma(acc, a.M[i + (int64_t)k * l], tot[l]);
            b.y[i] = acc;
          } else {
            const int ii = i - k;
            for (int l = 0; l <= k; ++l) cfma(acc, a.Pi[ii + (int64_t)(k + 1) * l], tot[l]);
            b.u[ii] = acc;
          }
        }
      }
      break;
  }
}

static void launch_final(hipStream_t s, const double2* part, BS* bs, const FinArgs& a) {
  hipLaunchKernelGGL(kb_final, dim3(a.nb), dim3(BT), 0, s, part, bs, a);
  DMG_LAUNCH_CHECK();
}

static FinArgs fin(int mode, int nq, int nblk, int nb) {
  FinArgs a{};
  a.mode = mode;
  a.nq = nq;
  a.nblk = nblk;
  a.nb = nb;
  return a;
}

// ---------------------------------------------------------------- norms and cycle start
template <typename R>
__global__ void __launch_bounds__(BT) kb_norm(const cx<R>* __restrict__ x, int64_t n, int nb, double2* part) {
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  double2 acc[1] = {mk(0.0, 0.0)};
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < N; i += stride) acc[0].x += cabs2(to_d(x[i]));
  b_publish<1>(acc, 1, nb, part);
}

__global__ void __launch_bounds__(NBMAX) kb_all_done(const BS* bs, int nb, int* flag) {
  const bool all = lanes_all_done(bs, nb);
  if (threadIdx.x == 0) *flag = all ? 1 : 0;
}

void launch_b_all_done(hipStream_t s, const BS* bs, int nb, int* flag) {
  hipLaunchKernelGGL(kb_all_done, dim3(1), dim3(NBMAX), 0, s, bs, nb, flag);
  DMG_LAUNCH_CHECK();
}

template <typename R>
void launch_b_norm(hipStream_t s, const cx<R>* x, int64_t n, int nb, BS* bs, double tol_rel, int mode, double* out,
                   double2* part) {
  const int G = bred_blocks(n * nb);
  hipLaunchKernelGGL(kb_norm<R>, dim3(G), dim3(BT), 0, s, x, n, nb, part);
  FinArgs a = fin(mode == 0 ? FIN_NORM0 : mode == 3 ? FIN_NORM3 : FIN_START, 1, G, nb);
  a.tol_rel = tol_rel;
  a.bnorm_too = mode == 2 ? 1 : 0;
  a.out = out;
  launch_final(s, part, bs, a);
}

template <typename R>
__global__ void __launch_bounds__(BT) kb_scale_beta(const cx<R>* __restrict__ x, cx<R>* __restrict__ y, int64_t n,
                                                    int nb, const BS* bs) {
  const int r = threadIdx.x & (nb - 1);
  const double beta = bs[r].beta;
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < N; i += stride) y[i] = from_d<R>(cscale(to_d(x[i]), inv));
}

template <typename R>
void launch_b_scale_beta(hipStream_t s, const cx<R>* x, cx<R>* y, int64_t n, int nb, const BS* bs) {
  hipLaunchKernelGGL(kb_scale_beta<R>, dim3(vec_blocks(n * nb)), dim3(BT), 0, s, x, y, n, nb, bs);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- Arnoldi (CGS2)

// (a) h_i = V_i^H w (i <= j) and ||w||^2 with w = V_{j+1}
template <typename R>
__global__ void __launch_bounds__(BT) kb_arn_dots1(const cx<R>* __restrict__ V, int64_t ld, int64_t n, int nb, int j,
                                                   const BS* bs, int* anyp2, double2* part) {
  if (lanes_all_done(bs, nb)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) *anyp2 = 0;
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  const cx<R>* w = V + (int64_t)(j + 1) * ld;
  double2 acc[MB + 2];
#pragma unroll
  for (int q = 0; q < MB + 2; ++q) acc[q] = mk(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x; e < N; e += stride) {
    const double2 wv = to_d(w[e]);
#pragma unroll
    for (int i = 0; i < MB + 1; ++i)
      if (i <= j) cfmac(acc[i], to_d(V[(int64_t)i * ld + e]), wv);
#pragma unroll
    for (int i = 0; i < MB + 2; ++i)
      if (i == j + 1) acc[i].x += cabs2(wv);
  }
  b_publish<MB + 2>(acc, j + 2, nb, part);
}

// (b) w -= sum_i H[i, j] V_i for the right-hand sides that took step j in one pass (then
// normalised at once: v_{j+1} = (w - V h) / h_{j+1, j}) or that need a second pass
template <typename R>
__global__ void __launch_bounds__(BT) kb_arn_update(cx<R>* __restrict__ V, int64_t ld, int64_t n, int nb, int j,
                                                    const BS* bs) {
  const int r0 = threadIdx.x & (nb - 1);
  const BS& b = bs[r0];
  const bool one = b.steps == j + 1 && b.pass2 == 0;
  if (!(one || b.pass2 == 1)) return;
  double scale = 1.0;
  if (one && !b.brk) {
    const double hn = b.H[LDH * j + j + 1].x;
    if (hn != 0.0) scale = 1.0 / hn;
  }
  double2 cf[MB + 1];
#pragma unroll
  for (int i = 0; i < MB + 1; ++i) cf[i] = (i <= j) ? b.H[LDH * j + i] : mk(0.0, 0.0);
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  cx<R>* w = V + (int64_t)(j + 1) * ld;
  for (int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x; e < N; e += stride) {
    double2 wv = to_d(w[e]);
#pragma unroll
    for (int i = 0; i < MB + 1; ++i)
      if (i <= j) wv = csub(wv, cmul(cf[i], to_d(V[(int64_t)i * ld + e])));
    w[e] = from_d<R>(cscale(wv, scale));
  }
}

// (c) h2_i = V_i^H w and ||w||^2 of the updated w, for the right-hand sides that need a
// second pass (returns at once when none does)
template <typename R>
__global__ void __launch_bounds__(BT) kb_arn_dots2(const cx<R>* __restrict__ V, int64_t ld, int64_t n, int nb, int j,
                                                   const BS* bs, const int* anyp2, double2* part) {
  if (!*anyp2) return;
  const int r0 = threadIdx.x & (nb - 1);
  const bool act = bs[r0].pass2 == 1;
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  const cx<R>* w = V + (int64_t)(j + 1) * ld;
  double2 acc[MB + 2];
#pragma unroll
  for (int q = 0; q < MB + 2; ++q) acc[q] = mk(0.0, 0.0);
  if (act)
    for (int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x; e < N; e += stride) {
      const double2 wv = to_d(w[e]);
#pragma unroll
      for (int i = 0; i < MB + 1; ++i)
        if (i <= j) cfmac(acc[i], to_d(V[(int64_t)i * ld + e]), wv);
#pragma unroll
      for (int i = 0; i < MB + 2; ++i)
        if (i == j + 1) acc[i].x += cabs2(wv);
    }
  b_publish<MB + 2>(acc, j + 2, nb, part);
}

// (d) second pass: v_{j+1} = (w - sum_i h2_i V_i) / h_{j+1, j} for the right-hand sides that
// took it (their Givens update ran in the second phase of (c))
template <typename R>
__global__ void __launch_bounds__(BT) kb_arn_update2(cx<R>* __restrict__ V, int64_t ld, int64_t n, int nb, int j,
                                                     const BS* bs, const int* anyp2) {
  if (!*anyp2) return;
  const int r0 = threadIdx.x & (nb - 1);
  const BS& b = bs[r0];
  if (b.pass2 != 2 || b.steps != j + 1) return;
  double scale = 1.0;
  if (!b.brk) {
    const double hn = b.H[LDH * j + j + 1].x;
    if (hn != 0.0) scale = 1.0 / hn;
  }
  double2 cf[MB + 1];
#pragma unroll
  for (int i = 0; i < MB + 1; ++i) cf[i] = (i <= j) ? b.h2[i] : mk(0.0, 0.0);
  cx<R>* w = V + (int64_t)(j + 1) * ld;
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  for (int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x; e < N; e += stride) {
    double2 wv = to_d(w[e]);
#pragma unroll
    for (int i = 0; i < MB + 1; ++i)
      if (i <= j) wv = csub(wv, cmul(cf[i], to_d(V[(int64_t)i * ld + e])));
    w[e] = from_d<R>(cscale(wv, scale));
  }
}

template <typename R>
void launch_b_arnoldi(hipStream_t s, cx<R>* V, int64_t ld, int64_t n, int nb, int j, BS* bs, int* anyp2,
                      double2* part) {
  const int G = bred_blocks(n * nb);
  FinArgs a = fin(FIN_ARN1, j + 2, G, nb);
  a.j = j;
  a.anyp2 = anyp2;
  a.eta = sizeof(R) == sizeof(float) ? 1e-4 : 1e-8;
  hipLaunchKernelGGL(kb_arn_dots1<R>, dim3(G), dim3(BT), 0, s, (const cx<R>*)V, ld, n, nb, j, (const BS*)bs,
                     anyp2, part);
  launch_final(s, part, bs, a);
  hipLaunchKernelGGL(kb_arn_update<R>, dim3(vec_blocks(n * nb)), dim3(BT), 0, s, V, ld, n, nb, j, (const BS*)bs);
  hipLaunchKernelGGL(kb_arn_dots2<R>, dim3(G), dim3(BT), 0, s, (const cx<R>*)V, ld, n, nb, j, (const BS*)bs,
                     (const int*)anyp2, part);
  a.mode = FIN_ARN2;
  launch_final(s, part, bs, a);
  hipLaunchKernelGGL(kb_arn_update2<R>, dim3(vec_blocks(n * nb)), dim3(BT), 0, s, V, ld, n, nb, j, (const BS*)bs,
                     (const int*)anyp2);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- least squares, combinations
// One workgroup per right-hand side: y = Rm^{-1} g (steps terms), u = c - H y.
__global__ void __launch_bounds__(64) kb_ls_solve(BS* bs) {
  __shared__ double2 Rs[LDH * MB];
  __shared__ double2 ys[MB + 1];
  BS& b = bs[blockIdx.x];
  const int t = threadIdx.x;
  const int n = b.active ? b.steps : 0;
  for (int e = t; e < LDH * n; e += 64) Rs[e] = b.Rm[e];
  __syncthreads();
  if (t == 0) {
    for (int i = n - 1; i >= 0; --i) {
      double2 acc = b.g[i];
      for (int l = i + 1; l < n; ++l) acc = csub(acc, cmul(Rs[i + LDH * l], ys[l]));
      const double2 d = Rs[i + LDH * i];
      ys[i] = cabs2(d) > 0.0 ? bcdiv(acc, d) : mk(0.0, 0.0);
    }
  }
  __syncthreads();
  for (int i = t; i < n; i += 64) b.y[i] = ys[i];
  for (int i = t; i <= n; i += 64) {
    double2 acc = b.c[i];
    for (int l = 0; l < n; ++l) acc = csub(acc, cmul(b.H[i + LDH * l], ys[l]));
    b.u[i] = acc;
  }
}

void launch_b_ls_solve(hipStream_t s, BS* bs, int nb) {
  hipLaunchKernelGGL(kb_ls_solve, dim3(nb), dim3(64), 0, s, bs);
  DMG_LAUNCH_CHECK();
}

template <typename R>
__global__ void __launch_bounds__(BT) kb_combine(cx<R>* __restrict__ x, const cx<R>* __restrict__ V, int64_t ld,
                                                 int64_t n, int nb, const BS* bs, int use_u, int accumulate) {
  const int r0 = threadIdx.x & (nb - 1);
  const BS& b = bs[r0];
  if (!b.active) return;
  const int cntc = b.steps + (use_u ? 1 : 0);
  const double2* src = use_u ? b.u : b.y;
  double2 cf[MB + 1];
#pragma unroll
  for (int i = 0; i < MB + 1; ++i) cf[i] = (i < cntc) ? src[i] : mk(0.0, 0.0);
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  for (int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x; e < N; e += stride) {
    double2 acc = accumulate ? to_d(x[e]) : mk(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < MB + 1; ++i)
      if (i < cntc) cfma(acc, cf[i], to_d(V[(int64_t)i * ld + e]));
    x[e] = from_d<R>(acc);
  }
}

template <typename R>
void launch_b_combine(hipStream_t s, cx<R>* x, const cx<R>* V, int64_t ld, int64_t n, int nb, const BS* bs, int use_u,
                      int accumulate) {
  hipLaunchKernelGGL(kb_combine<R>, dim3(vec_blocks(n * nb)), dim3(BT), 0, s, x, V, ld, n, nb, bs, use_u, accumulate);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- two-step smoother
template <typename R>
__global__ void __launch_bounds__(BT) kb_smooth2_dots(const cx<R>* __restrict__ v, const cx<R>* __restrict__ w1,
                                                      const cx<R>* __restrict__ w2, int64_t n, int nb, double2* part) {
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  double2 acc[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) acc[q] = mk(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x; e < N; e += stride) {
    const double2 vv = to_d(v[e]), x1 = to_d(w1[e]), x2 = to_d(w2[e]);
    acc[0].x += cabs2(x1);
    cfmac(acc[1], x1, x2);
    acc[2].x += cabs2(x2);
    cfmac(acc[3], x1, vv);
    cfmac(acc[4], x2, vv);
  }
  b_publish<5>(acc, 5, nb, part);
}

template <typename R>
__global__ void __launch_bounds__(BT) kb_smooth2_combine(const cx<R>* __restrict__ v, const cx<R>* __restrict__ w1,
                                                         const cx<R>* __restrict__ w2, int64_t n, int nb,
                                                         const double2* coef, cx<R>* __restrict__ y,
                                                         cx<R>* __restrict__ rr) {
  const int r0 = threadIdx.x & (nb - 1);
  const double2 c0 = coef[2 * r0], c1 = coef[2 * r0 + 1];
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  for (int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x; e < N; e += stride) {
    const double2 vv = to_d(v[e]), x1 = to_d(w1[e]);
    double2 yv = mk(0.0, 0.0);
    cfma(yv, c0, vv);
    cfma(yv, c1, x1);
    y[e] = from_d<R>(yv);
    if (rr) {
      double2 rv = vv;
      rv = csub(rv, cmul(c0, x1));
      rv = csub(rv, cmul(c1, to_d(w2[e])));
      rr[e] = from_d<R>(rv);
    }
  }
}

template <typename R>
void launch_b_smooth2(hipStream_t s, const cx<R>* v, const cx<R>* w1, const cx<R>* w2, int64_t n, int nb,
                      double2* coef, cx<R>* y, cx<R>* r, double2* part) {
  const int G = bred_blocks(n * nb);
  hipLaunchKernelGGL(kb_smooth2_dots<R>, dim3(G), dim3(BT), 0, s, v, w1, w2, n, nb, part);
  FinArgs a = fin(FIN_SMOOTH2, 5, G, nb);
  a.coef = coef;
  launch_final(s, part, nullptr, a);
  hipLaunchKernelGGL(kb_smooth2_combine<R>, dim3(vec_blocks(n * nb)), dim3(BT), 0, s, v, w1, w2, n, nb,
                     (const double2*)coef, y, r);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- GMRES-Proj projection
// c_i = DV_i^H r (i <= k) per right-hand side (the final phase forms y = M c and u = Pi c)
template <typename R>
__global__ void __launch_bounds__(BT) kb_proj_dots(const cx<R>* __restrict__ DV, int k, const cx<R>* __restrict__ rr,
                                                   int64_t n, int nb, double2* part) {
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  const int lg = __ffs(nb) - 1;
  double2 acc[MQ];
#pragma unroll
  for (int q = 0; q < MQ; ++q) acc[q] = mk(0.0, 0.0);
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < N; i += stride) {
    const int64_t e = i >> lg;
    const double2 rv = to_d(rr[i]);
#pragma unroll
    for (int q = 0; q < MQ; ++q)
      if (q <= k) cfmac(acc[q], to_d(DV[(int64_t)q * n + e]), rv);
  }
  b_publish<MQ>(acc, k + 1, nb, part);
}

// x += sum_{i<k} y_i DV_i ; r -= sum_{i<=k} u_i DV_i (active right-hand sides)
template <typename R>
__global__ void __launch_bounds__(BT) kb_proj_apply(const cx<R>* __restrict__ DV, int k, cx<R>* __restrict__ x,
                                                    cx<R>* __restrict__ rr, int64_t n, int nb, const BS* bs) {
  __shared__ double2 cy[MQ][NBMAX];
  __shared__ double2 cu[MQ][NBMAX];
  for (int p = threadIdx.x; p < (k + 1) * nb; p += BT) {
    const int r = p % nb, q = p / nb;
    cy[q][r] = (q < k) ? bs[r].y[q] : mk(0.0, 0.0);
    cu[q][r] = bs[r].u[q];
  }
  __syncthreads();
  const int r0 = threadIdx.x & (nb - 1);
  if (!bs[r0].active) return;
  const int lg = __ffs(nb) - 1;
  const int64_t N = n * nb;
  const int64_t stride = (int64_t)gridDim.x * BT;
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < N; i += stride) {
    const int64_t e = i >> lg;
    double2 xv = to_d(x[i]), rv = to_d(rr[i]);
    for (int q = 0; q <= k; ++q) {
      const double2 dv = to_d(DV[(int64_t)q * n + e]);
      cfma(xv, cy[q][r0], dv);
      rv = csub(rv, cmul(cu[q][r0], dv));
    }
    x[i] = from_d<R>(xv);
    rr[i] = from_d<R>(rv);
  }
}

template <typename R>
void launch_b_project(hipStream_t s, const cx<R>* DV, int k, const double2* M, const double2* Pi, cx<R>* x, cx<R>* r,
                      int64_t n, int nb, BS* bs, double2* part) {
  const int G = bred_blocks(n * nb);
  hipLaunchKernelGGL(kb_proj_dots<R>, dim3(G), dim3(BT), 0, s, DV, k, (const cx<R>*)r, n, nb, part);
  FinArgs a = fin(FIN_PROJ, k + 1, G, nb);
  a.k = k;
  a.M = M;
  a.Pi = Pi;
  launch_final(s, part, bs, a);
  hipLaunchKernelGGL(kb_proj_apply<R>, dim3(vec_blocks(n * nb)), dim3(BT), 0, s, DV, k, x, r, n, nb, (const BS*)bs);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- stencils
template <typename T> __device__ inline T bmul_i(T z) { T r; r.x = -z.y; r.y = z.x; return r; }

// Wilson-Dirac operator on a batched field: one thread per (site, right-hand side),
// both spins (the spin-projected hops of the single-field stencil).
template <typename R>
__global__ void __launch_bounds__(BT) kb_wilson(const cx<R>* __restrict__ U, const cx<R>* __restrict__ in,
                                                cx<R>* __restrict__ out, R diag, int Nx, int Nt, int nb,
                                                const cx<R>* __restrict__ sub, const BS* skip) {
  if (skip && lanes_all_done(skip, nb)) return;
  using T = cx<R>;
  const int lg = __ffs(nb) - 1;
  const int64_t idx = (int64_t)blockIdx.x * BT + threadIdx.x;
  const int V = Nx * Nt;
  if (idx >= (int64_t)V * nb) return;
  const int s = (int)(idx >> lg), r = (int)(idx & (nb - 1));
  const int x = s % Nx, t = s / Nx;
  const int xp = (x + 1 == Nx) ? 0 : x + 1, xm = (x == 0) ? Nx - 1 : x - 1;
  const int tp = (t + 1 == Nt) ? 0 : t + 1, tm = (t == 0) ? Nt - 1 : t - 1;
  const int sxp = xp + Nx * t, sxm = xm + Nx * t, stp = x + Nx * tp, stm = x + Nx * tm;
  auto at = [&](int site, int spin) { return in[((int64_t)(2 * site + spin) << lg) + r]; };
  const R half = R(0.5);
  T acc0 = cscale(at(s, 0), diag), acc1 = cscale(at(s, 1), diag);
  {
    T h = csub(at(sxp, 0), at(sxp, 1));
    T w = cmul(U[2 * s + 0], h);
    acc0 = csub(acc0, cscale(w, half));
    acc1 = cadd(acc1, cscale(w, half));
  }
  {
    T h = cadd(at(sxm, 0), at(sxm, 1));
    T w = cmulc(U[2 * sxm + 0], h);
    acc0 = csub(acc0, cscale(w, half));
    acc1 = csub(acc1, cscale(w, half));
  }
  {
    T h = cadd(at(stp, 0), bmul_i(at(stp, 1)));
    T w = cmul(U[2 * s + 1], h);
    acc0 = csub(acc0, cscale(w, half));
    acc1 = cadd(acc1, cscale(bmul_i(w), half));
  }
  {
    T h = csub(at(stm, 0), bmul_i(at(stm, 1)));
    T w = cmulc(U[2 * stm + 1], h);
    acc0 = csub(acc0, cscale(w, half));
    acc1 = csub(acc1, cscale(bmul_i(w), half));
  }
  const int64_t o0 = ((int64_t)(2 * s) << lg) + r, o1 = o0 + nb;
  if (sub) {
    acc0 = csub(sub[o0], acc0);
    acc1 = csub(sub[o1], acc1);
  }
  out[o0] = acc0;
  out[o1] = acc1;
}

// FP32 form with two lanes per thread: each neighbour spin is one 16-byte load covering both lanes,
// and the output stores are nontemporal (the 2 x nb x 8 B written per site are not re-read by this
// kernel).  The per-lane arithmetic is the same sequence of operations as kb_wilson's.
__device__ inline float2 half2of(float4 v, int h) { return h ? make_float2(v.z, v.w) : make_float2(v.x, v.y); }

template <int TBW>
__global__ void __launch_bounds__(TBW) kb_wilson_pair_t(const float2* __restrict__ U, const float4* __restrict__ in,
                                                        float4* __restrict__ out, float diag, int Nx, int Nt, int nb,
                                                        const float4* __restrict__ sub, const BS* skip) {
  if (skip && lanes_all_done(skip, nb)) return;
  const int hb = nb >> 1;  // lane pairs = float4 per (site, spin); a power of two
  const int lg = __ffs(hb) - 1;
  // dispatch order (an XCD-aware order cut the fabric reads by 14 % but ran 8 % slower: the re-read
  // neighbour fields come from the Infinity Cache)
  const int64_t idx = (int64_t)blockIdx.x * TBW + threadIdx.x;
  const int V = Nx * Nt;
  if (idx >= (int64_t)V * hb) return;
  const int s = (int)(idx >> lg), rp = (int)(idx & (hb - 1));
  const int x = s % Nx, t = s / Nx;
  const int xp = (x + 1 == Nx) ? 0 : x + 1, xm = (x == 0) ? Nx - 1 : x - 1;
  const int tp = (t + 1 == Nt) ? 0 : t + 1, tm = (t == 0) ? Nt - 1 : t - 1;
  const int sxp = xp + Nx * t, sxm = xm + Nx * t, stp = x + Nx * tp, stm = x + Nx * tm;
  auto at = [&](int site, int spin) { return in[((int64_t)(2 * site + spin) << lg) + rp]; };
  const float4 a0 = at(s, 0), a1 = at(s, 1);
  const float4 p0 = at(sxp, 0), p1 = at(sxp, 1), m0 = at(sxm, 0), m1 = at(sxm, 1);
  const float4 u0 = at(stp, 0), u1 = at(stp, 1), n0 = at(stm, 0), n1 = at(stm, 1);
  const float2 ux = U[2 * s], uxm = U[2 * sxm], ut = U[2 * s + 1], utm = U[2 * stm + 1];
  float r0[4], r1[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float2 acc0 = cscale(half2of(a0, h), diag), acc1 = cscale(half2of(a1, h), diag);
    {
      const float2 z = cmul(ux, csub(half2of(p0, h), half2of(p1, h)));
      acc0 = csub(acc0, cscale(z, 0.5f));
      acc1 = cadd(acc1, cscale(z, 0.5f));
    }
    {
      const float2 z = cmulc(uxm, cadd(half2of(m0, h), half2of(m1, h)));
      acc0 = csub(acc0, cscale(z, 0.5f));
      acc1 = csub(acc1, cscale(z, 0.5f));
    }
    {
      const float2 z = cmul(ut, cadd(half2of(u0, h), bmul_i(half2of(u1, h))));
      acc0 = csub(acc0, cscale(z, 0.5f));
      acc1 = cadd(acc1, cscale(bmul_i(z), 0.5f));
    }
    {
      const float2 z = cmulc(utm, csub(half2of(n0, h), bmul_i(half2of(n1, h))));
      acc0 = csub(acc0, cscale(z, 0.5f));
      acc1 = csub(acc1, cscale(bmul_i(z), 0.5f));
    }
    r0[2 * h] = acc0.x; r0[2 * h + 1] = acc0.y;
    r1[2 * h] = acc1.x; r1[2 * h + 1] = acc1.y;
  }
  const int64_t i0 = ((int64_t)(2 * s) << lg) + rp, i1 = i0 + hb;
  if (sub) {
    const float4 s0 = sub[i0], s1 = sub[i1];
    r0[0] = s0.x - r0[0]; r0[1] = s0.y - r0[1]; r0[2] = s0.z - r0[2]; r0[3] = s0.w - r0[3];
    r1[0] = s1.x - r1[0]; r1[1] = s1.y - r1[1]; r1[2] = s1.z - r1[2]; r1[3] = s1.w - r1[3];
  }
  typedef float f4v __attribute__((ext_vector_type(4)));
  __builtin_nontemporal_store(f4v{r0[0], r0[1], r0[2], r0[3]}, reinterpret_cast<f4v*>(out + i0));
  __builtin_nontemporal_store(f4v{r1[0], r1[1], r1[2], r1[3]}, reinterpret_cast<f4v*>(out + i1));
}

static void launch_wilson_form(hipStream_t s, int form, const float2* U, const float4* in, float4* out, float diag,
                               int Nx, int Nt, int nb, const float4* sub, const BS* skip) {
  const int64_t N2 = (int64_t)Nx * Nt * (nb / 2);
  const int tb = form == 1 ? 128 : form == 2 ? 512 : form == 3 ? 64 : form == 4 ? 1024 : 256;
  const dim3 g((unsigned)((N2 + tb - 1) / tb));
  if (tb == 1024)
    hipLaunchKernelGGL(kb_wilson_pair_t<1024>, g, dim3(1024), 0, s, U, in, out, diag, Nx, Nt, nb, sub, skip);
  else if (tb == 128) hipLaunchKernelGGL(kb_wilson_pair_t<128>, g, dim3(128), 0, s, U, in, out, diag, Nx, Nt, nb, sub, skip);
  else if (tb == 512) hipLaunchKernelGGL(kb_wilson_pair_t<512>, g, dim3(512), 0, s, U, in, out, diag, Nx, Nt, nb, sub, skip);
  else if (tb == 64) hipLaunchKernelGGL(kb_wilson_pair_t<64>, g, dim3(64), 0, s, U, in, out, diag, Nx, Nt, nb, sub, skip);
  else hipLaunchKernelGGL(kb_wilson_pair_t<256>, g, dim3(256), 0, s, U, in, out, diag, Nx, Nt, nb, sub, skip);
  DMG_LAUNCH_CHECK();
}


template <typename R>
void launch_b_wilson(hipStream_t s, const cx<R>* U, const cx<R>* in, cx<R>* out, double m0, int Nx, int Nt, int nb,
                     const cx<R>* sub, const BS* skip) {
  if constexpr (sizeof(R) == sizeof(float)) {
    if (nb >= 2) {
      launch_wilson_form(s, tuned_form(TK_WILSON, sizeof(R), Nx * Nt, nb), (const float2*)U, (const float4*)in,
                         (float4*)out, (float)(m0 + 2.0), Nx, Nt, nb, (const float4*)sub, skip);
      return;
    }
  }
  const int64_t N = (int64_t)Nx * Nt * nb;
  hipLaunchKernelGGL(kb_wilson<R>, dim3((unsigned)((N + BT - 1) / BT)), dim3(BT), 0, s, U, in, out, (R)(m0 + 2.0), Nx,
                     Nt, nb, sub, skip);
  DMG_LAUNCH_CHECK();
}

// Blocked operator on a batched field, one site per workgroup: out(S) = sum_d A_d(S) in(S+d).
// The five neighbours' 24 x nb values are staged in LDS together when they fit in
// 64 KB (one round of global loads), else one direction at a time; thread o owns
// outputs (row i, right-hand side r) = (o / nb, o % nb), o = threadIdx.x + BT k.
template <typename R, typename B = cx<R>>
__global__ void __launch_bounds__(BT) kb_block(const B* __restrict__ A, const cx<R>* __restrict__ in,
                                               cx<R>* __restrict__ out, int Lx, int Lt, int nb,
                                               const cx<R>* __restrict__ sub, const BS* skip) {
  if (skip && lanes_all_done(skip, nb)) return;
  using T = cx<R>;
  constexpr int OPT = NC * NBMAX / BT;  // most outputs per thread
  extern __shared__ __align__(16) unsigned char kb_smem[];
  T* xs = (T*)kb_smem;
  const int S = blockIdx.x;
  const int X = S % Lx, Tt = S / Lx;
  const int tid = threadIdx.x;
  const int nout = NC * nb;
  const bool all5 = (size_t)5 * nout * sizeof(T) <= 65536;
  int nbS[5];
  nbS[0] = S;
  nbS[1] = ((X + 1 == Lx) ? 0 : X + 1) + Lx * Tt;
  nbS[2] = ((X == 0) ? Lx - 1 : X - 1) + Lx * Tt;
  nbS[3] = X + Lx * ((Tt + 1 == Lt) ? 0 : Tt + 1);
  nbS[4] = X + Lx * ((Tt == 0) ? Lt - 1 : Tt - 1);
  double2 acc[OPT];
#pragma unroll
  for (int k = 0; k < OPT; ++k) acc[k] = mk(0.0, 0.0);
  for (int d0 = 0; d0 < 5; d0 += all5 ? 5 : 1) {
    const int nd = all5 ? 5 : 1;
    __syncthreads();
    for (int dd = 0; dd < nd; ++dd)
      for (int p = tid; p < nout; p += BT) xs[dd * nout + p] = in[(int64_t)nbS[d0 + dd] * nout + p];
    __syncthreads();
    for (int dd = 0; dd < nd; ++dd) {
      const B* a = A + ((int64_t)S * 5 + d0 + dd) * NC * NC;
      const T* xd = xs + dd * nout;
#pragma unroll
      for (int k = 0; k < OPT; ++k) {
        const int o = tid + BT * k;
        if (o < nout) {
          const int i = o / nb, r = o % nb;
          T sacc = make_cx<R>(R(0), R(0));
#pragma unroll 8
          for (int c = 0; c < NC; ++c) cfma(sacc, ld_blk(a + c * NC + i), xd[c * nb + r]);
          acc[k] = cadd(acc[k], to_d(sacc));
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < OPT; ++k) {
    const int o = tid + BT * k;
    if (o < nout) {
      const int64_t g = (int64_t)S * nout + o;
      double2 y = acc[k];
      if (sub) y = csub(to_d(sub[g]), y);
      out[g] = from_d<R>(y);
    }
  }
}

// Blocked operator on the matrix cores (FP32 or FP64) for nb = 16, 32 or 64 right-hand sides.
// Per site and direction the complex product A_d (24 x 24) X_d (24 x nb) is the real
// product [[Ar, -Ai], [Ai, Ar]] (48 x 48) [Xr; Xi] (48 x nb), run as 16 x 16 x 4 MFMA
// tiles: 3 row tiles x nb/16 column tiles x 12 k-steps, accumulated over the five
// directions in the MFMA registers (direction, then k-step, for every tile).
typedef float v4f __attribute__((ext_vector_type(4)));

// nb / (16 NTW) workgroups per site, each with NTW wavefronts, one per 16-lane column tile.  The five hop directions are streamed through two LDS stages (block d as re / im
// planes, the neighbour field of direction d as re / im planes): while the matrix cores work on
// direction d, the loads of direction d + 1 are in flight.  Each wavefront keeps the three row
// tiles of its column tile in three independent accumulators, so every B fragment read from LDS
// feeds three MFMAs.  Results pass through LDS to be written as complex entries (row i: real
// part, row 24 + i: imaginary part).
typedef double v4d __attribute__((ext_vector_type(4)));
template <typename R> struct MfmaT;
// 16 x 16 x 4 tiles: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its four results
// are column l % 16 and rows 4 (l / 16) + v (FP32) or 4 v + l / 16 (FP64).
template <> struct MfmaT<float> {
  using acc = v4f;
  static __device__ inline acc step(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct MfmaT<double> {
  using acc = v4d;
  static __device__ inline acc step(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lk, int v) { return 4 * v + lk; }
};

template <typename R, int NTW, typename B = cx<R>>
__global__ void __launch_bounds__(64 * NTW) kb_block_mfma_p(const B* __restrict__ A, const cx<R>* __restrict__ in,
                                                            cx<R>* __restrict__ out, int Lx, int Lt, int nb,
                                                            const cx<R>* __restrict__ sub, const BS* skip) {
  using T = cx<R>;
  using M = MfmaT<R>;
  constexpr int TB = 64 * NTW;
  constexpr int NBW = 16 * NTW;                    // lanes (right-hand sides) of this workgroup
  constexpr int RA = (NC * NC + TB - 1) / TB;      // block entries staged per thread
  constexpr int RX = NC * NBW / TB;                // field entries staged per thread (= 6)
  if (skip && lanes_all_done(skip, nb)) return;
  __shared__ R sa[2][2][NC * NC];                  // [stage][re, im][c * NC + i]
  __shared__ R sx[2][2][NC * NBW];                 // [stage][re, im][c * nb + r]
  const int NG = nb / NBW;                         // workgroups per site
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int site = bid / NG, lb = (bid % NG) * NBW;
  const int X = site % Lx, Tt = site / Lx;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int nbS[5];
  nbS[0] = site;
  nbS[1] = ((X + 1 == Lx) ? 0 : X + 1) + Lx * Tt;
  nbS[2] = ((X == 0) ? Lx - 1 : X - 1) + Lx * Tt;
  nbS[3] = X + Lx * ((Tt + 1 == Lt) ? 0 : Tt + 1);
  nbS[4] = X + Lx * ((Tt == 0) ? Lt - 1 : Tt - 1);
  const int nout = NC * nb;
  T ra[RA], rx[RX];
  auto fetch = [&](int d) {
    const B* ad = A + ((int64_t)site * 5 + d) * NC * NC;
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int p = tid + q * TB;
      if (p < NC * NC) ra[q] = ld_blk(ad + p);
    }
    const T* xd = in + (int64_t)nbS[d] * nout;
#pragma unroll
    for (int q = 0; q < RX; ++q) {
      const int p = tid + q * TB, c = p / NBW, r = p % NBW;
      rx[q] = xd[c * nb + lb + r];
    }
  };
  auto stash = [&](int st) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int p = tid + q * TB;
      if (p < NC * NC) {
        sa[st][0][p] = ra[q].x;
        sa[st][1][p] = ra[q].y;
      }
    }
#pragma unroll
    for (int q = 0; q < RX; ++q) {
      sx[st][0][tid + q * TB] = rx[q].x;
      sx[st][1][tid + q * TB] = rx[q].y;
    }
  };
  const int li = lane & 15, lk = lane >> 4;
  const int j = 16 * w + li;  // column (right-hand side) of this lane's B fragment
  typename M::acc acc[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) acc[m] = typename M::acc{0, 0, 0, 0};
  fetch(0);
  stash(0);
  __syncthreads();
  for (int d = 0; d < 5; ++d) {
    const int st = d & 1;
    if (d + 1 < 5) fetch(d + 1);
    const R* are = sa[st][0];
    const R* aim = sa[st][1];
#pragma unroll
    for (int kk = 0; kk < 12; ++kk) {
      const int K = 4 * kk + lk;  // row of [Xr; Xi]
      const int c = K < NC ? K : K - NC;
      const R bval = sx[st][K < NC ? 0 : 1][c * NBW + j];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int I = 16 * m + li;  // row of the 48-row product
        const int i = I < NC ? I : I - NC;
        const R aval = (I < NC) ? (K < NC ? are[c * NC + i] : -aim[c * NC + i])
                                : (K < NC ? aim[c * NC + i] : are[c * NC + i]);
        acc[m] = M::step(aval, bval, acc[m]);
      }
    }
    if (d + 1 < 5) stash(st ^ 1);
    __syncthreads();
  }
  // result planes [48][nb] in the (now free) field stage 0
  R* res = &sx[0][0][0];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) res[(16 * m + M::row(lk, v)) * NBW + j] = acc[m][v];
  __syncthreads();
  for (int o = tid; o < NC * NBW; o += TB) {
    const int ii = o / NBW, r = o % NBW;
    T y = make_cx<R>(res[ii * NBW + r], res[(NC + ii) * NBW + r]);
    const int64_t g = (int64_t)site * nout + ii * nb + lb + r;
    if (sub) y = make_cx<R>(sub[g].x - y.x, sub[g].y - y.y);
    out[g] = y;
  }
}

// ---------------------------------------------------------------- autotuning
// Launch forms that compute the same bits, chosen per shape by timing each once (per process):
// block stencil on the matrix cores: 16 NTW lanes per workgroup, NTW in {4, 2, 1}; multi-RHS
// Wilson stencil (FP32): 64, 128, 256, 512 or 1024 threads per workgroup.
namespace {
constexpr int TUNE_FORMS = 5;
struct TuneEntry {
  int form;
  float us[TUNE_FORMS];
};
std::mutex g_tune_mu;
std::map<std::array<long long, 4>, TuneEntry> g_tune;
int g_tune_mode = 1;
int g_tune_force[TK_COUNT] = {-1, -1};
}  // namespace

static int block_forms(int nb) { return nb >= 64 ? 3 : nb >= 32 ? 2 : 1; }  // NTW = 4 >> form (capped by nb)
static int block_ntw(int nb, int form) {
  const int top = nb / 16;  // largest NTW for nb lanes
  int ntw = top >> form;
  return ntw < 1 ? 1 : ntw;
}

int tuned_form(int kernel, int prec, int sites, int nb) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune_force[kernel] >= 0) return g_tune_force[kernel];
  if (!g_tune_mode) return 0;
  auto it = g_tune.find({kernel, prec, sites, nb});
  return it == g_tune.end() ? 0 : it->second.form;
}

template <typename R, typename B>
static void launch_block_form(hipStream_t s, int form, const B* A, const cx<R>* in, cx<R>* out, int Lx, int Lt,
                              int nb, const cx<R>* sub, const BS* skip) {
  if (form < 0 || form >= block_forms(nb)) form = 0;
  const int ntw = block_ntw(nb, form);
  const dim3 g((unsigned)(Lx * Lt * (nb / (16 * ntw))));
  if (ntw == 4) hipLaunchKernelGGL((kb_block_mfma_p<R, 4, B>), g, dim3(256), 0, s, A, in, out, Lx, Lt, nb, sub, skip);
  else if (ntw == 2)
    hipLaunchKernelGGL((kb_block_mfma_p<R, 2, B>), g, dim3(128), 0, s, A, in, out, Lx, Lt, nb, sub, skip);
  else hipLaunchKernelGGL((kb_block_mfma_p<R, 1, B>), g, dim3(64), 0, s, A, in, out, Lx, Lt, nb, sub, skip);
  DMG_LAUNCH_CHECK();
}

// times nforms launch forms (three interleaved rounds of one warm-up and 5 timed launches each)
// and records the fastest
template <typename F>
static void tune_shape(hipStream_t s, int kernel, int prec, int sites, int nb, int nforms, F&& run) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_mode || g_tune.count({kernel, prec, sites, nb})) return;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return;
  }
  hipEvent_t a, b;
  DMG_HIP(hipEventCreate(&a));
  DMG_HIP(hipEventCreate(&b));
  TuneEntry e{0, {0.f, 0.f, 0.f, 0.f, 0.f}};
  // three rounds over the forms (interleaved, so that clock and cache states affect every form
  // alike), five timed launches each after one warm-up; each form keeps its fastest round
  for (int round = 0; round < 3; ++round)
    for (int f = 0; f < nforms && f < TUNE_FORMS; ++f) {
      run(f);
      DMG_HIP(hipEventRecord(a, s));
      for (int r = 0; r < 5; ++r) run(f);
      DMG_HIP(hipEventRecord(b, s));
      DMG_HIP(hipEventSynchronize(b));
      float ms = 0.f;
      DMG_HIP(hipEventElapsedTime(&ms, a, b));
      const float us = ms * 1e3f / 5.f;
      if (round == 0 || us < e.us[f]) e.us[f] = us;
    }
  for (int f = 1; f < nforms && f < TUNE_FORMS; ++f)
    if (e.us[f] < e.us[e.form]) e.form = f;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[{kernel, prec, sites, nb}] = e;
}

template <typename R>
void b_tune_block(hipStream_t s, const cx<R>* A, const cx<R>* in, cx<R>* out, int Lx, int Lt, int nb, bool mfma) {
  if (nb < 16 || !mfma) return;
  tune_shape(s, TK_BLOCK, sizeof(R), Lx * Lt, nb, block_forms(nb), [&](int f) {
    launch_block_form<R, cx<R>>(s, f, A, in, out, Lx, Lt, nb, nullptr, nullptr);
  });
}

void b_tune_block_bf16(hipStream_t s, const bf16c* A, const float2* in, float2* out, int Lx, int Lt, int nb,
                       bool mfma) {
  if (nb < 16 || !mfma) return;
  tune_shape(s, TK_BLOCK, 2, Lx * Lt, nb, block_forms(nb), [&](int f) {
    launch_block_form<float, bf16c>(s, f, A, in, out, Lx, Lt, nb, nullptr, nullptr);
  });
}

template <typename R>
void b_tune_wilson(hipStream_t s, const cx<R>* U, const cx<R>* in, cx<R>* out, double m0, int Nx, int Nt, int nb) {
  if constexpr (sizeof(R) == sizeof(float)) {
    if (nb < 2) return;
    tune_shape(s, TK_WILSON, sizeof(R), Nx * Nt, nb, 5, [&](int f) {
      launch_wilson_form(s, f, (const float2*)U, (const float4*)in, (float4*)out, (float)(m0 + 2.0), Nx, Nt, nb,
                         nullptr, nullptr);
    });
  }
}

void b_tune_mode(int mode) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_mode = mode ? 1 : 0;
  if (mode == 2) g_tune.clear();
}

void b_tune_force(int kernel, int form) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (kernel >= 0 && kernel < TK_COUNT) g_tune_force[kernel] = form;
}

std::string b_tune_report() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::string o;
  char line[256];
  for (const auto& kv : g_tune) {
    const auto& k = kv.first;
    const auto& e = kv.second;
    snprintf(line, sizeof(line), "%s fp%lld sites=%lld nb=%lld form=%d us=[%.1f %.1f %.1f %.1f %.1f]\n",
             k[0] == TK_BLOCK ? "block_mfma" : "wilson_pair", 8 * k[1], k[2], k[3], e.form, e.us[0], e.us[1], e.us[2],
             e.us[3], e.us[4]);
    o += line;
  }
  return o;
}

template <typename R>
void launch_b_block(hipStream_t s, const cx<R>* A, const cx<R>* in, cx<R>* out, int Lx, int Lt, int nb,
                    const cx<R>* sub, const BS* skip, bool mfma) {
  // blocks on the matrix cores from 16 lanes on; mfma = false forces the vector-FMA kernel
  if (nb >= 16 && mfma) {
    launch_block_form<R, cx<R>>(s, tuned_form(TK_BLOCK, sizeof(R), Lx * Lt, nb), A, in, out, Lx, Lt, nb, sub, skip);
    return;
  }
  const size_t one = (size_t)NC * nb * sizeof(cx<R>);
  const size_t lds = 5 * one <= 65536 ? 5 * one : one;
  hipLaunchKernelGGL(kb_block<R>, dim3(Lx * Lt), dim3(BT), lds, s, A, in, out, Lx, Lt, nb, sub, skip);
  DMG_LAUNCH_CHECK();
}

void launch_b_block_bf16(hipStream_t s, const bf16c* A, const float2* in, float2* out, int Lx, int Lt, int nb,
                         const float2* sub, const BS* skip, bool mfma) {
  if (nb >= 16 && mfma) {
    launch_block_form<float, bf16c>(s, tuned_form(TK_BLOCK, 2, Lx * Lt, nb), A, in, out, Lx, Lt, nb, sub, skip);
    return;
  }
  const size_t one = (size_t)NC * nb * sizeof(float2);
  const size_t lds = 5 * one <= 65536 ? 5 * one : one;
  hipLaunchKernelGGL((kb_block<float, bf16c>), dim3(Lx * Lt), dim3(BT), lds, s, A, in, out, Lx, Lt, nb, sub, skip);
  DMG_LAUNCH_CHECK();
}

// Restriction on batched fields, one workgroup per coarse site (see the single-field kernel).
template <typename R>
__global__ void __launch_bounds__(BT) kb_restrict(const cx<R>* __restrict__ P, const cx<R>* __restrict__ fine,
                                                  cx<R>* __restrict__ coarse, int Lx, int Lt, int dof, int nb) {
  using T = cx<R>;
  const int B = blockIdx.x;
  const int BX = Lx / BLK;
  const int X = B % BX, Tb = B / BX;
  const int h = dof / 2;
  const int nout = NC * nb;
  for (int o = threadIdx.x; o < nout; o += BT) {
    const int oo = o / nb, r = o % nb;
    const int c = oo / NV, k = oo % NV;
    double2 acc = mk(0.0, 0.0);
    for (int sl = 0; sl < BLK * BLK; ++sl) {
      const int s = (BLK * X + sl % BLK) + Lx * (BLK * Tb + sl / BLK);
      for (int ii = 0; ii < h; ++ii) {
        const int a = c * h + ii;
        const int64_t fe = (int64_t)s * dof + a;
        const T p = P[fe * NV + k];
        cfmac(acc, to_d(p), to_d(fine[fe * nb + r]));
      }
    }
    coarse[(int64_t)B * nout + o] = from_d<R>(acc);
  }
}

template <typename R>
void launch_b_restrict(hipStream_t s, const cx<R>* P, const cx<R>* fine, cx<R>* coarse, int Lx, int Lt, int dof,
                       int nb) {
  const int nbk = (Lx / BLK) * (Lt / BLK);
  hipLaunchKernelGGL(kb_restrict<R>, dim3(nbk), dim3(BT), 0, s, P, fine, coarse, Lx, Lt, dof, nb);
  DMG_LAUNCH_CHECK();
}

template <typename R>
__global__ void __launch_bounds__(BT) kb_prolong(const cx<R>* __restrict__ P, const cx<R>* __restrict__ coarse,
                                                 cx<R>* __restrict__ fine, int Lx, int Lt, int dof, int nb,
                                                 int accumulate) {
  using T = cx<R>;
  const int lg = __ffs(nb) - 1;
  const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
  const int64_t n = (int64_t)Lx * Lt * dof;
  if (i >= n * nb) return;
  const int64_t e = i >> lg;
  const int r = (int)(i & (nb - 1));
  const int s = (int)(e / dof), a = (int)(e % dof);
  const int x = s % Lx, t = s / Lx;
  const int B = x / BLK + (Lx / BLK) * (t / BLK);
  const int c = a / (dof / 2);
  const T* p = P + e * NV;
  const T* cv = coarse + ((int64_t)B * NC + c * NV) * nb + r;
  double2 acc = accumulate ? to_d(fine[i]) : mk(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < NV; ++k) cfma(acc, to_d(p[k]), to_d(cv[(int64_t)k * nb]));
  fine[i] = from_d<R>(acc);
}

template <typename R>
void launch_b_prolong(hipStream_t s, const cx<R>* P, const cx<R>* coarse, cx<R>* fine, int Lx, int Lt, int dof, int nb,
                      int accumulate) {
  const int64_t N = (int64_t)Lx * Lt * dof * nb;
  hipLaunchKernelGGL(kb_prolong<R>, dim3((unsigned)((N + BT - 1) / BT)), dim3(BT), 0, s, P, coarse, fine, Lx, Lt, dof,
                     nb, accumulate);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- layout changes, flags
template <typename T>
__global__ void kb_gather(const T* __restrict__ in, T* __restrict__ out, int64_t n, int nrhs, int nb) {
  const int lg = __ffs(nb) - 1;
  const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (i >= n * nb) return;
  const int64_t e = i >> lg;
  const int r = (int)(i & (nb - 1));
  T z;
  z.x = 0;
  z.y = 0;
  out[i] = (r < nrhs) ? in[(int64_t)r * n + e] : z;
}

template <typename T>
__global__ void kb_scatter(const T* __restrict__ in, T* __restrict__ out, int64_t n, int nrhs, int nb) {
  const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (i >= n * nrhs) return;
  const int64_t r = i / n, e = i % n;
  out[i] = in[e * nb + r];
}

template <typename T>
void launch_b_gather(hipStream_t s, const T* in, T* out, int64_t n, int nrhs, int nb) {
  hipLaunchKernelGGL(kb_gather<T>, dim3((unsigned)((n * nb + BT - 1) / BT)), dim3(BT), 0, s, in, out, n, nrhs, nb);
  DMG_LAUNCH_CHECK();
}

template <typename T>
void launch_b_scatter(hipStream_t s, const T* in, T* out, int64_t n, int nrhs, int nb) {
  hipLaunchKernelGGL(kb_scatter<T>, dim3((unsigned)((n * nrhs + BT - 1) / BT)), dim3(BT), 0, s, in, out, n, nrhs, nb);
  DMG_LAUNCH_CHECK();
}
template void launch_b_gather<double2>(hipStream_t, const double2*, double2*, int64_t, int, int);
template void launch_b_gather<float2>(hipStream_t, const float2*, float2*, int64_t, int, int);
template void launch_b_scatter<double2>(hipStream_t, const double2*, double2*, int64_t, int, int);
template void launch_b_scatter<float2>(hipStream_t, const float2*, float2*, int64_t, int, int);

// lane r of a batched field: dst[e][r] = src ? src[e][r] (batched) : 0
__global__ void kb_lane_copy(const double2* __restrict__ src, double2* __restrict__ dst, int64_t n, int nb, int r) {
  const int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (e >= n) return;
  dst[e * nb + r] = src ? src[e * nb + r] : mk(0.0, 0.0);
}

void launch_b_lane_copy(hipStream_t s, const double2* src, double2* dst, int64_t n, int nb, int r) {
  hipLaunchKernelGGL(kb_lane_copy, dim3((unsigned)((n + BT - 1) / BT)), dim3(BT), 0, s, src, dst, n, nb, r);
  DMG_LAUNCH_CHECK();
}

// single field <-> lane r of a batched field
__global__ void kb_lane_io(const double2* __restrict__ in, double2* __restrict__ out, int64_t n, int nb, int r,
                           int to_lane) {
  const int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (e >= n) return;
  if (to_lane) out[e * nb + r] = in[e];
  else out[e] = in[e * nb + r];
}

void launch_b_lane_io(hipStream_t s, const double2* in, double2* out, int64_t n, int nb, int r, int to_lane) {
  hipLaunchKernelGGL(kb_lane_io, dim3((unsigned)((n + BT - 1) / BT)), dim3(BT), 0, s, in, out, n, nb, r, to_lane);
  DMG_LAUNCH_CHECK();
}

struct StateArg {
  int v[2 * NBMAX];
};

__global__ void kb_set_state(BS* bs, StateArg st, int nb) {
  const int r = threadIdx.x;
  if (r >= nb) return;
  bs[r].active = st.v[2 * r];
  bs[r].cap = st.v[2 * r + 1];
}

void launch_b_set_state(hipStream_t s, BS* bs, const int* host_st, int nb) {
  StateArg a;
  for (int i = 0; i < 2 * nb; ++i) a.v[i] = host_st[i];
  hipLaunchKernelGGL(kb_set_state, dim3(1), dim3(NBMAX), 0, s, bs, a, nb);
  DMG_LAUNCH_CHECK();
}

#define INST(R)                                                                                                        \
  template void launch_b_norm<R>(hipStream_t, const cx<R>*, int64_t, int, BS*, double, int, double*, double2*);      \
  template void launch_b_scale_beta<R>(hipStream_t, const cx<R>*, cx<R>*, int64_t, int, const BS*);                   \
  template void launch_b_arnoldi<R>(hipStream_t, cx<R>*, int64_t, int64_t, int, int, BS*, int*, double2*);            \
  template void launch_b_combine<R>(hipStream_t, cx<R>*, const cx<R>*, int64_t, int64_t, int, const BS*, int, int);   \
  template void launch_b_smooth2<R>(hipStream_t, const cx<R>*, const cx<R>*, const cx<R>*, int64_t, int, double2*,    \
                                    cx<R>*, cx<R>*, double2*);                                                         \
  template void launch_b_project<R>(hipStream_t, const cx<R>*, int, const double2*, const double2*, cx<R>*, cx<R>*,   \
                                    int64_t, int, BS*, double2*);                                                      \
  template void launch_b_wilson<R>(hipStream_t, const cx<R>*, const cx<R>*, cx<R>*, double, int, int, int,            \
                                   const cx<R>*, const BS*);                                                           \
  template void launch_b_block<R>(hipStream_t, const cx<R>*, const cx<R>*, cx<R>*, int, int, int, const cx<R>*,       \
                                  const BS*, bool);                                                                        \
  template void launch_b_restrict<R>(hipStream_t, const cx<R>*, const cx<R>*, cx<R>*, int, int, int, int);            \
  template void launch_b_prolong<R>(hipStream_t, const cx<R>*, const cx<R>*, cx<R>*, int, int, int, int, int);
INST(double)
INST(float)
#undef INST
template void b_tune_block<float>(hipStream_t, const float2*, const float2*, float2*, int, int, int, bool);
template void b_tune_block<double>(hipStream_t, const double2*, const double2*, double2*, int, int, int, bool);
template void b_tune_wilson<float>(hipStream_t, const float2*, const float2*, float2*, double, int, int, int);
template void b_tune_wilson<double>(hipStream_t, const double2*, const double2*, double2*, double, int, int, int);

}  // namespace dmg
