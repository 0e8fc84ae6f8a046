// Small dense FP64 work of the Krylov solvers, done on the device by one
// workgroup per launch: least-squares back-substitution, the GMRES-DR deflated
// restart (harmonic Ritz eigenproblem on several wavefronts or by the QR
// algorithm, choice of the k smallest, new basis change and Hbar_k), Givens QR of
// a full (k+1) x k block, and the GMRES-Proj projection.
#include "kernels.h"

namespace dmg {

constexpr int LD = MMAX + 1;
constexpr int DW = 64;  // threads of the dense kernels (one wavefront)

__device__ inline double cabs_(double2 a) { return sqrt(cabs2(a)); }
__device__ inline double2 cdiv(double2 a, double2 b) {
  const double d = cabs2(b);
  return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }
// principal square root (real part >= 0) from sqrt((|z| +/- Re z) / 2)
__device__ inline double2 csqrt_(double2 z) {
  const double r = sqrt(cabs2(z));
  if (r == 0.0) return mk(0.0, 0.0);
  const double a = sqrt(0.5 * (r + fabs(z.x)));
  if (z.x >= 0.0) return mk(a, z.y / (2.0 * a));
  return mk(fabs(z.y) / (2.0 * a), copysign(a, z.y));
}
// value of lane l of a wavefront (scalar register read of both 32-bit halves)
__device__ inline double rd_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double2 rd_lane(double2 v, int l) { return mk(rd_lane(v.x, l), rd_lane(v.y, l)); }
// DPP lane permutation (quad_perm / row_ror control) on both 32-bit halves of a double
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum over the whole wavefront (all 64 lanes active): rows of 16 by DPP, then the four row
// sums read into scalar registers; every lane gets the same bits.
__device__ inline double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x124>(v);  // row_ror 4
  v += dpp_d<0x128>(v);  // row_ror 8
  return (rd_lane(v, 0) + rd_lane(v, 16)) + (rd_lane(v, 32) + rd_lane(v, 48));
}
__device__ inline double2 wave_sum(double2 v) { return mk(wave_sum(v.x), wave_sum(v.y)); }
// Largest value over the wavefront and the first lane holding it (-1 when no lane compares
// equal to the maximum, i.e. with NaN)
__device__ inline int wave_argmax(double v) {
  double m = v;
  m = fmax(m, dpp_d<0xB1>(m));
  m = fmax(m, dpp_d<0x4E>(m));
  m = fmax(m, dpp_d<0x124>(m));
  m = fmax(m, dpp_d<0x128>(m));
  m = fmax(fmax(rd_lane(m, 0), rd_lane(m, 16)), fmax(rd_lane(m, 32), rd_lane(m, 48)));
  const unsigned long long at = __ballot(v == m);
  return __ffsll((long long)at) - 1;
}

// Givens rotation G = [c s; -conj(s) c] (c real) with G [a; b] = [r; 0].
__device__ inline void make_givens(double2 a, double2 b, double& c, double2& s) {
  const double na = cabs_(a), nb = cabs_(b);
  if (nb == 0.0) { c = 1.0; s = mk(0.0, 0.0); return; }
  if (na == 0.0) { c = 0.0; s = cscale(cconj(b), 1.0 / nb); return; }
  const double nr = sqrt(na * na + nb * nb);
  c = na / nr;
  s = cscale(cmul(cconj(b), a), 1.0 / (na * nr));
}
// The same rotation with one square root and one division (as in LAPACK's zlartg):
// c = |a|^2 / d, s = conj(b) a / d, d = |a| r = sqrt(|a|^2 (|a|^2 + |b|^2)); the product is
// split into two roots only where it would leave the double range.
__device__ inline void make_givens_fast(double2 a, double2 b, double& c, double2& s) {
  const double na2 = cabs2(a), nb2 = cabs2(b);
  if (nb2 == 0.0) { c = 1.0; s = mk(0.0, 0.0); return; }
  if (na2 == 0.0) { c = 0.0; s = cscale(cconj(b), 1.0 / sqrt(nb2)); return; }
  const double h2 = na2 + nb2, pr = na2 * h2;
  double d;
  if (pr > 1e-290 && pr < 1e290) d = sqrt(pr);
  else d = sqrt(na2) * sqrt(h2);
  const double inv = 1.0 / d;
  c = na2 * inv;
  s = cscale(cmul(cconj(b), a), inv);
}

// ---------------------------------------------------------------- least squares
// y = R^{-1} g over the completed steps by columns on one wavefront (lane i holds the running
// g_i; column l gives y_l from lane l, then every lane above drops its term), R staged in LDS;
// then u = c - H y with one thread per row, H staged in the same LDS when it fits.  Each lane
// issues eight staging loads before it stores any (the loads are independent; one at a time,
// each would wait a full L2 round trip).
__device__ inline void ls_stage(double2* dst, const double2* src, int rows, int cols, bool upper) {
  const int t = threadIdx.x, ne = rows * cols;
  for (int e0 = t; e0 < ne; e0 += 8 * DW) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * DW, i = e % rows, l = e / rows;
      v[u] = (e < ne && (!upper || i <= l)) ? src[i + LD * l] : mk(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (e0 + u * DW < ne) dst[e0 + u * DW] = v[u];
  }
}
__global__ void __launch_bounds__(DW) k_ls_solve(KState* ks) {
  __shared__ double2 Rs[MMAX * MMAX];
  __shared__ double2 ys[MMAX + 1];
  const int t = threadIdx.x;
  const int n = ks->steps;
  ls_stage(Rs, ks->R, n, n, true);
  double2 acc = t < n ? ks->g[t] : mk(0.0, 0.0);
  __syncthreads();
  for (int l = n - 1; l >= 0; --l) {
    const double2 r = t < l ? Rs[t + n * l] : mk(0.0, 0.0);
    const double2 d = Rs[l + n * l];
    const double2 al = rd_lane(acc, l);
    const double2 yl = cabs2(d) > 0.0 ? cdiv(al, d) : mk(0.0, 0.0);
    if (t == l) ys[l] = yl;
    if (t < l) acc = csub(acc, cmul(r, yl));
  }
  __syncthreads();
  for (int i = t; i < n; i += DW) ks->y[i] = ys[i];
  const bool staged = (n + 1) * n <= MMAX * MMAX;
  if (staged) ls_stage(Rs, ks->H, n + 1, n, false);  // R is no longer read
  __syncthreads();
  for (int i = t; i <= n; i += DW) {
    double2 a2 = ks->c[i];
    if (staged)
      for (int l = 0; l < n; ++l) a2 = csub(a2, cmul(Rs[i + (n + 1) * l], ys[l]));
    else
      for (int l = 0; l < n; ++l) a2 = csub(a2, cmul(ks->H[i + LD * l], ys[l]));
    ks->u[i] = a2;
  }
}

void launch_ls_solve(hipStream_t s, KState* ks) {
  hipLaunchKernelGGL(k_ls_solve, dim3(1), dim3(DW), 0, s, ks);
  DMG_LAUNCH_CHECK();
}

// Givens QR of the leading (k+1) x k block of ks->H (full after a deflated restart):
// rotations on adjacent rows, bottom-up in each column; rotated copy to ks->R, c -> g.
__device__ void qr_block_serial(KState* ks, int k) {
  for (int jc = 0; jc < k; ++jc)
    for (int i = 0; i <= k; ++i) ks->R[i + LD * jc] = ks->H[i + LD * jc];
  for (int i = 0; i <= MMAX; ++i) ks->g[i] = (i <= k) ? ks->c[i] : mk(0.0, 0.0);
  ks->nrot = 0;
  for (int jc = 0; jc < k; ++jc) {
    for (int r = k; r > jc; --r) {
      double c;
      double2 s;
      make_givens(ks->R[r - 1 + LD * jc], ks->R[r + LD * jc], c, s);
      for (int q = jc; q < k; ++q) {
        const double2 a = ks->R[r - 1 + LD * q], b = ks->R[r + LD * q];
        ks->R[r - 1 + LD * q] = cadd(cscale(a, c), cmul(s, b));
        ks->R[r + LD * q] = csub(cscale(b, c), cmul(cconj(s), a));
      }
      ks->R[r + LD * jc] = mk(0.0, 0.0);
      const double2 a = ks->g[r - 1], b = ks->g[r];
      ks->g[r - 1] = cadd(cscale(a, c), cmul(s, b));
      ks->g[r] = csub(cscale(b, c), cmul(cconj(s), a));
      const int q = ks->nrot++;
      ks->rot_p[q] = r - 1;
      ks->rot_c[q] = c;
      ks->rot_s[q] = s;
    }
  }
  ks->est = cabs_(ks->g[k]);
}

// Same rotations as qr_block_serial, computed on an LDS copy (scratch: >= (k+1) * k
// double2) so the serial part never waits on global memory.
constexpr int QRL_MAXROT = 528;  // k <= 32
__device__ void qr_block_lds(KState* ks, int k, double2* scratch) {
  const int t = threadIdx.x;
  const int nr = k * (k + 1) / 2;
  __shared__ double2 gq[MMAX + 1];
  __shared__ double rcq[QRL_MAXROT];
  __shared__ double2 rsq[QRL_MAXROT];
  __shared__ int rpq[QRL_MAXROT];
  if (nr > QRL_MAXROT) {
    if (t == 0) qr_block_serial(ks, k);
    __syncthreads();
    return;
  }
  double2* Rq = scratch;
  for (int e = t; e < (k + 1) * k; e += blockDim.x) Rq[e] = ks->H[(e % (k + 1)) + LD * (e / (k + 1))];
  for (int i = t; i <= k; i += blockDim.x) gq[i] = ks->c[i];
  __syncthreads();
  if (t == 0) {
    int q = 0;
    for (int jc = 0; jc < k; ++jc)
      for (int r = k; r > jc; --r) {
        double c;
        double2 sg;
        make_givens(Rq[r - 1 + (k + 1) * jc], Rq[r + (k + 1) * jc], c, sg);
        for (int q2 = jc; q2 < k; ++q2) {
          const double2 a = Rq[r - 1 + (k + 1) * q2], b = Rq[r + (k + 1) * q2];
          Rq[r - 1 + (k + 1) * q2] = cadd(cscale(a, c), cmul(sg, b));
          Rq[r + (k + 1) * q2] = csub(cscale(b, c), cmul(cconj(sg), a));
        }
        Rq[r + (k + 1) * jc] = mk(0.0, 0.0);
        const double2 a = gq[r - 1], b = gq[r];
        gq[r - 1] = cadd(cscale(a, c), cmul(sg, b));
        gq[r] = csub(cscale(b, c), cmul(cconj(sg), a));
        rcq[q] = c;
        rsq[q] = sg;
        rpq[q] = r - 1;
        ++q;
      }
  }
  __syncthreads();
  for (int e = t; e < (k + 1) * k; e += blockDim.x) ks->R[(e % (k + 1)) + LD * (e / (k + 1))] = Rq[e];
  for (int i = t; i <= MMAX; i += blockDim.x) ks->g[i] = (i <= k) ? gq[i] : mk(0.0, 0.0);
  for (int q = t; q < nr; q += blockDim.x) {
    ks->rot_c[q] = rcq[q];
    ks->rot_s[q] = rsq[q];
    ks->rot_p[q] = rpq[q];
  }
  if (t == 0) {
    ks->nrot = nr;
    ks->est = cabs_(gq[k]);
  }
  __syncthreads();
}

// qr_block_serial's rotations with one lane per column of [R | g] ((k+1) x (k+1), k + 1 <= 64):
// for each rotation every lane updates rows p, p+1 of its own column, the rotation itself from
// column jc's entries (read by all lanes); the same rotations in the same order.
__device__ void qr_block_wave(KState* ks, int k, double2* Rq) {
  const int t = threadIdx.x;
  const int K1 = k + 1;
  for (int e = t; e < K1 * k; e += DW) Rq[e] = ks->H[(e % K1) + LD * (e / K1)];
  for (int i = t; i < K1; i += DW) Rq[K1 * k + i] = ks->c[i];  // column k: g
  __shared__ double rcq[QRL_MAXROT];
  __shared__ double2 rsq[QRL_MAXROT];
  __shared__ int rpq[QRL_MAXROT];
  __syncthreads();
  int q = 0;
  for (int jc = 0; jc < k; ++jc)
    for (int r = k; r > jc; --r) {
      double c;
      double2 sg;
      make_givens(Rq[r - 1 + K1 * jc], Rq[r + K1 * jc], c, sg);
      if (t >= jc && t <= k) {
        double2* col = Rq + K1 * t;
        const double2 a = col[r - 1], b = col[r];
        col[r - 1] = cadd(cscale(a, c), cmul(sg, b));
        col[r] = (t == jc) ? mk(0.0, 0.0) : csub(cscale(b, c), cmul(cconj(sg), a));
      }
      if (t == 0) {
        rcq[q] = c;
        rsq[q] = sg;
        rpq[q] = r - 1;
      }
      ++q;
    }
  __syncthreads();
  for (int e = t; e < K1 * k; e += DW) ks->R[(e % K1) + LD * (e / K1)] = Rq[e];
  for (int i = t; i <= MMAX; i += DW) ks->g[i] = (i <= k) ? Rq[K1 * k + i] : mk(0.0, 0.0);
  for (int i = t; i < q; i += DW) {
    ks->rot_c[i] = rcq[i];
    ks->rot_s[i] = rsq[i];
    ks->rot_p[i] = rpq[i];
  }
  if (t == 0) {
    ks->nrot = q;
    ks->est = cabs_(Rq[K1 * k + k]);
  }
  __syncthreads();
}

__global__ void k_qr_block(KState* ks, int k) {
  if (threadIdx.x == 0) qr_block_serial(ks, k);
}

void launch_qr_block(hipStream_t s, KState* ks, int k) {
  hipLaunchKernelGGL(k_qr_block, dim3(1), dim3(1), 0, s, ks, k);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- GMRES-Proj projection
// d = argmin || c - Hk d ||, Hk (k+1) x k column-major with ld k+1; y = d, u = Hk d.
__global__ void k_proj_solve(const double2* Hk, int k, KState* ks) {
  if (threadIdx.x != 0) return;
  // work copy into R/g using the block QR
  for (int jc = 0; jc < k; ++jc)
    for (int i = 0; i <= k; ++i) ks->H[i + LD * jc] = Hk[i + (k + 1) * jc];
  qr_block_serial(ks, k);
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = ks->g[i];
    for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(ks->R[i + LD * l], ks->y[l]));
    const double2 d = ks->R[i + LD * i];
    ks->y[i] = cabs2(d) > 0.0 ? cdiv(acc, d) : mk(0.0, 0.0);
  }
  for (int i = 0; i <= k; ++i) {
    double2 acc = mk(0.0, 0.0);
    for (int l = 0; l < k; ++l) acc = cadd(acc, cmul(Hk[i + (k + 1) * l], ks->y[l]));
    ks->u[i] = acc;
  }
  ks->steps = k;
}

void launch_proj_solve(hipStream_t s, const double2* Hk, int k, KState* ks) {
  hipLaunchKernelGGL(k_proj_solve, dim3(1), dim3(1), 0, s, Hk, k, ks);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- projection matrices of a deflation space
// For Hbar_k ((k+1) x k, column-major, ld k+1) with Givens QR Hbar_k = Q [R; 0]:
//   M  = R^{-1} [I_k 0] Q^H   (k x (k+1)): d = M c minimises || c - Hbar_k d ||
//   Pi = Hbar_k M             ((k+1) x (k+1)): the projector onto range(Hbar_k)
// Both column-major.  One workgroup; column i of M is formed by one thread.
constexpr int KDMAX = 32;  // largest deflation space handled here
__global__ void __launch_bounds__(DW) k_defl_prepare(const double2* Hk, int k, double2* M, double2* Pi) {
  __shared__ double2 Rs[(KDMAX + 1) * KDMAX];
  __shared__ double rc[KDMAX * (KDMAX + 1) / 2];
  __shared__ double2 rsn[KDMAX * (KDMAX + 1) / 2];
  __shared__ int rp[KDMAX * (KDMAX + 1) / 2];
  __shared__ double2 Ms[KDMAX * (KDMAX + 1)];
  const int t = threadIdx.x;
  const int K1 = k + 1;
  for (int e = t; e < K1 * k; e += DW) Rs[e] = Hk[e];
  __syncthreads();
  if (t == 0) {
    int q = 0;
    for (int jc = 0; jc < k; ++jc)
      for (int r = k; r > jc; --r) {
        double c;
        double2 sg;
        make_givens(Rs[r - 1 + K1 * jc], Rs[r + K1 * jc], c, sg);
        for (int q2 = jc; q2 < k; ++q2) {
          const double2 a = Rs[r - 1 + K1 * q2], b = Rs[r + K1 * q2];
          Rs[r - 1 + K1 * q2] = cadd(cscale(a, c), cmul(sg, b));
          Rs[r + K1 * q2] = csub(cscale(b, c), cmul(cconj(sg), a));
        }
        Rs[r + K1 * jc] = mk(0.0, 0.0);
        rc[q] = c;
        rsn[q] = sg;
        rp[q] = r - 1;
        ++q;
      }
  }
  __syncthreads();
  const int nr = k * (k + 1) / 2;
  for (int col = t; col < K1; col += DW) {
    double2 v[KDMAX + 1];
    for (int i = 0; i <= k; ++i) v[i] = mk(i == col ? 1.0 : 0.0, 0.0);
    for (int q = 0; q < nr; ++q) {
      const int p = rp[q];
      const double2 a = v[p], b = v[p + 1];
      v[p] = cadd(cscale(a, rc[q]), cmul(rsn[q], b));
      v[p + 1] = csub(cscale(b, rc[q]), cmul(cconj(rsn[q]), a));
    }
    for (int i = k - 1; i >= 0; --i) {
      double2 acc = v[i];
      for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(Rs[i + K1 * l], Ms[l + k * col]));
      const double2 d = Rs[i + K1 * i];
      Ms[i + k * col] = cabs2(d) > 0.0 ? cdiv(acc, d) : mk(0.0, 0.0);
    }
  }
  __syncthreads();
  for (int e = t; e < k * K1; e += DW) M[e] = Ms[e];
  for (int e = t; e < K1 * K1; e += DW) {
    const int i = e % K1, col = e / K1;
    double2 acc = mk(0.0, 0.0);
    for (int l = 0; l < k; ++l) cfma(acc, Hk[i + K1 * l], Ms[l + k * col]);
    Pi[e] = acc;
  }
}

void launch_defl_prepare(hipStream_t s, const double2* Hk, int k, double2* M, double2* Pi) {
  DMG_CHECK(k >= 1 && k <= KDMAX, DMG_E_INVALID, "deflation spaces above 32 vectors are not supported");
  hipLaunchKernelGGL(k_defl_prepare, dim3(1), dim3(DW), 0, s, Hk, k, M, Pi);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- eigenproblem helpers
// All routines run on one wavefront (DW threads) with matrices column-major in LDS:
// A[i + n * j].

// Hessenberg reduction by Householder reflections, accumulating X (A_orig = X A X^H).
// One wavefront (n < 64): the norms are wavefront sums over one row per lane, the reflector
// sits in LDS for broadcast reads, the left update has one lane per column and the right
// update one lane per row of A and of X; inner products use two accumulators so that the
// LDS loads of consecutive terms overlap.
__device__ void hessenberg(double2* A, double2* X, double2* v, int n) {
  const int t = threadIdx.x;
  for (int e = t; e < n * n; e += DW) X[e] = ((e % n) == (e / n)) ? mk(1.0, 0.0) : mk(0.0, 0.0);
  __syncthreads();
  for (int col = 0; col + 2 < n; ++col) {
    // x = A[col+1 .. n-1, col]
    const double2 xi = (t > col && t < n) ? A[t + n * col] : mk(0.0, 0.0);
    const double xn2 = wave_sum(t >= col + 2 ? cabs2(xi) : 0.0);
    if (xn2 == 0.0) continue;
    const double2 alpha = rd_lane(xi, col + 1);
    const double anorm = cabs_(alpha);
    const double xnorm = sqrt(xn2 + anorm * anorm);
    const double2 ph = anorm > 0.0 ? cscale(alpha, 1.0 / anorm) : mk(1.0, 0.0);
    const double2 beta = cscale(ph, -xnorm);
    // v = x - beta e1 (indices col+1 .. n-1 stored at v[0 .. n-col-2]); the reflector ends at the
    // column's last nonzero row (after a deflated restart the matrix is banded: a dense leading
    // block whose bulge each reflector moves one row down), and the zeros beyond it would add
    // exact zeros to every product below
    const unsigned long long nzr = __ballot(t > col && t < n && (xi.x != 0.0 || xi.y != 0.0));
    const int len = (63 - __clzll(nzr)) - col;
    const double2 vi = (t == col + 1) ? csub(alpha, beta) : xi;
    if (t > col && t < n) v[t - col - 1] = vi;
    const double f = 2.0 / wave_sum(cabs2(vi));
    __syncthreads();
    // left: A[col+1:, j] -= f v (v^H A[col+1:, j]) for the columns j >= col
    if (t >= col && t < n) {
      const double2* a = A + col + 1 + n * t;
      double2 d0 = mk(0.0, 0.0), d1 = mk(0.0, 0.0);
      int i = 0;
      for (; i + 1 < len; i += 2) {
        cfmac(d0, v[i], a[i]);
        cfmac(d1, v[i + 1], a[i + 1]);
      }
      if (i < len) cfmac(d0, v[i], a[i]);
      const double2 d = cscale(cadd(d0, d1), f);
      double2* aw = A + col + 1 + n * t;
      for (int l = 0; l < len; ++l) aw[l] = csub(aw[l], cmul(v[l], d));
    }
    __syncthreads();
    // right: A[i, col+1:] -= f (A[i, col+1:] v) v^H for all rows; same for X
    for (int r = t; r < 2 * n; r += DW) {
      double2* M = (r < n) ? A : X;
      const int i = (r < n) ? r : r - n;
      double2 d0 = mk(0.0, 0.0), d1 = mk(0.0, 0.0);
      int l = 0;
      for (; l + 1 < len; l += 2) {
        cfma(d0, M[i + n * (col + 1 + l)], v[l]);
        cfma(d1, M[i + n * (col + 2 + l)], v[l + 1]);
      }
      if (l < len) cfma(d0, M[i + n * (col + 1 + l)], v[l]);
      const double2 d = cscale(cadd(d0, d1), f);
      for (int l2 = 0; l2 < len; ++l2)
        M[i + n * (col + 1 + l2)] = csub(M[i + n * (col + 1 + l2)], cmul(d, cconj(v[l2])));
    }
    __syncthreads();
    if (t >= col + 2 && t < n) A[t + n * col] = mk(0.0, 0.0);
    __syncthreads();
  }
}

// Givens rotation as make_givens_fast with the reciprocal square root of |a|^2 (|a|^2 + |b|^2)
// taken directly (rsqrt, within an ulp or two) instead of a square root and a division.
__device__ inline void make_givens_rs(double2 a, double2 b, double& c, double2& s) {
  const double na2 = cabs2(a), nb2 = cabs2(b);
  if (nb2 == 0.0) { c = 1.0; s = mk(0.0, 0.0); return; }
  if (na2 == 0.0) { c = 0.0; s = cscale(cconj(b), rsqrt(nb2)); return; }
  const double h2 = na2 + nb2, pr = na2 * h2;
  const double inv = (pr > 1e-290 && pr < 1e290) ? rsqrt(pr) : 1.0 / (sqrt(na2) * sqrt(h2));
  c = na2 * inv;
  s = cscale(cmul(cconj(b), a), inv);
}

// Complex Schur form of the Hessenberg A by single-shift implicit QR (Wilkinson shifts,
// exceptional shifts every 10 iterations).  Returns 0 on success.  One wavefront (n <= 64);
// the deflation test is one ballot over the subdiagonal (|re| + |im| magnitudes, as in the
// reference QR codes).
//
// A sweep chases the bulge with its updates deferred, so that the chain of rotations never
// waits on the LDS and a rotation costs few instructions (one wavefront issues them one at a
// time).  Rotation k mixes rows and columns k, k+1 of the active block [lo, hi].  Every lane
// t plays two parts:
//  - column t (t >= k-1): it holds the current A[k, t] and A[k+1, t] and applies the left
//    rotation; its row-k result is final under the left rotations and the row-(k+1) result
//    is carried to the next rotation.  Lanes k-1, k, k+1 hold the bulge pair and the 2 x 2
//    diagonal block; lanes beyond read the untouched A[k+1, t] from the LDS.
//  - row t (t <= k+2): it holds A[t, k] and A[t, k+1] after the left rotation and applies the
//    right one; its column-k result is final and the column-(k+1) result is carried.  Rows
//    above k read A[t, k+1] as the column lane wrote it; rows k and k+1 take the block from
//    lanes k, k+1 (two lane reads), row k+2 has a zero in column k.
//  - row t of X in the same way against the untouched X[t, k+1].
// The next rotation's bulge pair and block come back from rows k+1, k+2 by lane reads.  Left
// and right rotations commute and each entry sees its rotations in the plain sweep's order,
// so the result equals that of applying every rotation to whole rows and columns in turn.
static_assert(MMAX <= DW, "one lane per row and column of the restart eigenproblem");
__device__ int schur_qr(double2* A, double2* X, int n) {
  const int t = threadIdx.x;
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, iter = 0, total = 0;
  __syncthreads();
  while (hi > 0) {
    // the active block [lo, hi]: lo is the last small subdiagonal at or above hi
    bool small = false;
    if (t >= 1 && t <= hi) {
      double sc = cabs1(A[t - 1 + n * (t - 1)]) + cabs1(A[t + n * t]);
      if (sc == 0.0) sc = 1.0;
      small = cabs1(A[t + n * (t - 1)]) <= eps * sc;
    }
    const unsigned long long msk = __ballot(small);
    const int lo = msk ? 63 - __clzll(msk) : 0;
    if (lo > 0 && t == 0) A[lo + n * (lo - 1)] = mk(0.0, 0.0);
    if (lo == hi) { --hi; iter = 0; continue; }
    if (++total > 60 * n) return 1;
    ++iter;
    // shift
    const double2 a = A[hi - 1 + n * (hi - 1)], b = A[hi - 1 + n * hi], c = A[hi + n * (hi - 1)], d = A[hi + n * hi];
    double2 mu;
    if (iter % 11 == 10) {
      mu = cadd(d, mk(cabs_(c), 0.0));
    } else {
      const double2 hm = cscale(csub(a, d), 0.5);
      const double2 disc = csqrt_(cadd(cmul(hm, hm), cmul(b, c)));
      const double2 m0 = cscale(cadd(a, d), 0.5);
      const double2 m1 = cadd(m0, disc), m2 = csub(m0, disc);
      mu = (cabs2(csub(m1, d)) <= cabs2(csub(m2, d))) ? m1 : m2;
    }
    const bool in = t < n;
    double2 P = (t >= lo && in) ? A[lo + n * t] : mk(0.0, 0.0);  // column part: A[k, t]
    double2 Q = mk(0.0, 0.0);                                    // column part: A[k+1, t]
    double2 RC = (t < lo) ? A[t + n * lo] : mk(0.0, 0.0);        // row part: A[t, k]
    double2 XC = in ? X[t + n * lo] : mk(0.0, 0.0);              // X[t, k]
    double2 x = csub(A[lo + n * lo], mu), y = A[lo + 1 + n * lo];
    for (int k = lo; k < hi; ++k) {
      // untouched operands first: their latency overlaps the rotation's coefficients
      if (t >= (k > lo ? k + 1 : lo) && in) Q = A[k + 1 + n * t];
      const bool rl = t <= k - 1 || (t == k + 2 && t <= hi);
      double2 RB = rl ? A[t + n * (k + 1)] : mk(0.0, 0.0);
      const double2 XB = in ? X[t + n * (k + 1)] : mk(0.0, 0.0);
      double cg;
      double2 sg;
      make_givens_rs(x, y, cg, sg);
      const double2 csg = cconj(sg);
      // left rotation (lanes k-1 .. n-1 are meaningful)
      const double2 PN = cadd(cscale(P, cg), cmul(sg, Q));
      const double2 QN = csub(cscale(Q, cg), cmul(csg, P));
      if ((k > lo && t == k - 1) || (t >= k + 2 && in)) A[k + n * t] = PN;
      if (k > lo && t == k - 1) A[k + 1 + n * t] = mk(0.0, 0.0);
      if (t >= k + 2) P = QN;
      // rows k, k+1 of the block; row k+2 has a zero in column k
      const double2 pk1 = rd_lane(PN, k + 1), qk = rd_lane(QN, k);
      double2 RA = RC;
      if (t == k) { RA = PN; RB = pk1; }
      if (t == k + 1) { RA = qk; RB = QN; }
      if (t == k + 2) RA = mk(0.0, 0.0);
      // right rotation (rows 0 .. k+2 are meaningful)
      const double2 RAN = cadd(cscale(RA, cg), cmul(RB, csg));
      const double2 RBN = csub(cscale(RB, cg), cmul(RA, sg));
      if (t <= k) {
        A[t + n * k] = RAN;
        RC = RBN;
      }
      const double2 XN = cadd(cscale(XC, cg), cmul(XB, csg));
      const double2 XCN = csub(cscale(XB, cg), cmul(XC, sg));
      if (in) {
        X[t + n * k] = XN;
        XC = XCN;
      }
      if (k + 1 < hi) {
        // the next bulge pair (rows k+1, k+2 of column k) into lane k, the block's first
        // column into lane k+1
        const double2 xn = rd_lane(RAN, k + 1), yn = rd_lane(RAN, k + 2), a21 = rd_lane(RBN, k + 2);
        if (t == k) {
          P = xn;
          Q = yn;
        }
        if (t == k + 1) {
          P = RBN;
          Q = a21;
        }
        x = xn;
        y = yn;
      } else {
        // last rotation: write back the block's last row and every carried entry
        if (t == hi) {
          A[hi + n * (hi - 1)] = RAN;
          A[hi + n * hi] = RBN;
        }
        if (t < hi) A[t + n * hi] = RC;
        if (t >= hi + 1 && in) A[hi + n * t] = P;
        if (in) X[t + n * hi] = XC;
      }
    }
  }
  __syncthreads();
  return 0;
}

// ---------------------------------------------------------------- harmonic Ritz eigenproblem on several wavefronts
// The eigenvalues of the restart's Hessenberg matrix, the choice of the k smallest and their
// eigenvectors, for orders up to EIG_NMAX, in one workgroup of EIG_WAVES wavefronts (the
// one-wavefront QR algorithm is a chain of dependent rotations; here the work of each step is
// spread over lanes and the steps of different eigenvalues run side by side).
constexpr int EIG_NMAX = 32;
constexpr int EIG_WAVES = 5;
constexpr int EIG_THREADS = 64 * EIG_WAVES;  // 32 roots x 2 chains x 4 lanes, then 10 inverse iterations
constexpr int EIG_HALVES = 2 * EIG_WAVES;
constexpr int EIG_MAXIT = 80;

__device__ inline int lane_id() { return threadIdx.x & 63; }
// DPP lane permutation of a double for controls under which every lane reads a valid lane
template <int CTRL>
__device__ inline double dpp_v(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// sum over each quad of lanes; the four lanes get the same bits
__device__ inline double2 quad_sum(double2 v) {
  v = cadd(v, mk(dpp_v<0xB1>(v.x), dpp_v<0xB1>(v.y)));  // quad_perm [1, 0, 3, 2]
  v = cadd(v, mk(dpp_v<0x4E>(v.x), dpp_v<0x4E>(v.y)));  // quad_perm [2, 3, 0, 1]
  return v;
}
// value of lane 7 - i of each group of eight lanes (row_half_mirror)
__device__ inline double2 half_mirror(double2 v) { return mk(dpp_v<0x141>(v.x), dpp_v<0x141>(v.y)); }
// value of lane p of this lane's half (32 lanes) of the wavefront
__device__ inline double2 rd_half(double2 v, int p) {
  const double2 lo = rd_lane(v, p), hi = rd_lane(v, 32 + p);
  return (lane_id() & 32) ? hi : lo;
}
// sum over this lane's half of the wavefront (all lanes active): rows of 16 by DPP, then the
// half's two row sums from scalar registers
__device__ inline double half_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x124>(v);
  v += dpp_d<0x128>(v);
  const double lo = rd_lane(v, 0) + rd_lane(v, 16), hi = rd_lane(v, 32) + rd_lane(v, 48);
  return (lane_id() & 32) ? hi : lo;
}
// 1 / b with one division
__device__ inline double2 crcp(double2 b) {
  const double d = 1.0 / cabs2(b);
  return mk(b.x * d, -b.y * d);
}
// packed upper triangle of an n x n matrix: row p holds columns p .. n-1
__device__ inline int upk_off(int p, int n) { return p * n - p * (p - 1) / 2; }

// Global scratch of the restart (double2 entries unless stated): the Hessenberg form A (m x m)
// and its basis X (m x m), f = H^{-H} e_m (m), the eigenvalues (m), the selected eigenvectors
// of A ((m+1) x k, rows < m used), the selected indices (k ints), the path flag (1 int: 0 when
// the several-wavefront step produced them, 1 when the QR algorithm must) and the order whose
// eigenvalues the several-wavefront step left in theta (1 int, 0 if none).
struct DrWork {
  double2* A;
  double2* X;
  double2* f;
  double2* theta;
  double2* Y;
  int* sel;
  int* flag;
  int* prev;
};
__host__ __device__ inline DrWork dr_layout(double2* w, int m, int k) {
  DrWork d;
  d.A = w;
  d.X = d.A + m * m;
  d.f = d.X + m * m;
  d.theta = d.f + m;
  d.Y = d.theta + m;
  d.sel = (int*)(d.Y + (m + 1) * k);
  d.flag = d.sel + k;
  d.prev = d.flag + 1;
  return d;
}

// Eigenvalues by the Aberth-Ehrlich iteration on p(z) = det(A - z I), all roots at once:
//   z_e <- z_e - N_e / (1 - N_e sum_{j != e} 1 / (z_e - z_j)),   N_e = p(z_e) / p'(z_e),
// which converges cubically to simple roots.  p is evaluated by Hyman's method: x_{n-1} = 1 and
// rows n-1, ..., 1 of (A - z I) x = 0 give x_{n-2}, ..., x_0 in turn through the subdiagonal;
// the residual of row 0 is then p(z) times a factor independent of z (the product of the
// subdiagonal entries), and the recurrence differentiated in z gives p'(z) with the same
// factor.  Hyman's evaluation has a backward error of the order of the QR algorithm's, so the
// roots are as accurate; subdiagonal entries below eps ||A||_F are raised to that size (a
// perturbation of the same order).  Lanes 8e .. 8e+7 own root e: the first four carry x(z_e),
// the last four x'(z_e), lane l of a chain holding the entries j = l, l + 4, ... in registers;
// a row's sum is a quad sum, the two chains meet through the half-row mirror.  Starting points
// lie on a circle about c = trace(A) / n of radius 0.7 ||A - c I||_F / sqrt(n) (the root mean
// square distance of the eigenvalues from c is at most ||A - c I||_F / sqrt(n)).  A root is
// settled once its correction is below 4 eps |z| or, having fallen below 1e-10 |z|, stops
// shrinking (the rounding level of an ill-conditioned root).  Without convergence within
// EIG_MAXIT steps or with a non-finite value (multiple or tightly clustered roots, where the
// iteration converges only linearly) the kernel leaves the flag at 1 and the QR algorithm runs.
// Then the k of smallest modulus are chosen (the restart's order) and their eigenvectors found
// by two steps of inverse iteration, as in the reference eigenvector codes for Hessenberg
// matrices: LU of A - lam I with partial pivoting between the two rows the Hessenberg structure
// leaves in a column, a first solve U y = (1, ..., 1)^T (an implicit right-hand side), then
// (A - lam I) y' = y / ||y||; pivots below eps ||A||_F are raised to that size, and a value
// within that distance of an earlier chosen one is moved by it.  Each half wavefront takes one
// eigenvalue (lane j holds column j in the factorisation, row j in the solves).
__global__ void __launch_bounds__(EIG_THREADS) k_dr_eig(double2* work, int n, int k, int warm, int maxit,
                                                         const int* status) {
  extern __shared__ double2 esh[];
  double2* Ar = esh;  // EIG_NMAX x EIG_NMAX, row-major, zero beyond n
  const int upk = n * (n + 1) / 2;
  double2* U = Ar + EIG_NMAX * EIG_NMAX;  // EIG_HALVES packed upper triangles
  double2* Lm = U + EIG_HALVES * upk;     // EIG_HALVES x 32 multipliers
  double2* rU = Lm + EIG_HALVES * 32;     // EIG_HALVES x 32 reciprocal pivots
  int* pv = (int*)(rU + EIG_HALVES * 32);  // EIG_HALVES x 32 row exchanges
  __shared__ double2 zs[EIG_NMAX], rs[EIG_NMAX], lam[EIG_NMAX];
  __shared__ double st0[EIG_NMAX + 1];
  __shared__ double2 c0s;
  __shared__ double nrm[2];
  __shared__ double keys[64];
  __shared__ int sel[EIG_NMAX];
  if (*status != 0) return;
  const DrWork d = dr_layout(work, n, k);
  const int t = threadIdx.x;
  const double eps = 2.220446049250313e-16;
  for (int e = t; e < EIG_NMAX * EIG_NMAX; e += EIG_THREADS) {
    const int r = e / EIG_NMAX, j = e % EIG_NMAX;
    Ar[e] = (r < n && j < n) ? d.A[r + n * j] : mk(0.0, 0.0);
  }
  __syncthreads();
  if (t < 64) {
    double fro2 = 0.0;
    double2 tr = mk(0.0, 0.0);
    for (int e = t; e < n * n; e += 64) fro2 += cabs2(Ar[(e / n) * EIG_NMAX + e % n]);
    if (t < n) tr = Ar[t * (EIG_NMAX + 1)];
    fro2 = wave_sum(fro2);
    tr = wave_sum(tr);
    const double2 c0 = cscale(tr, 1.0 / n);
    double d2 = 0.0;
    for (int e = t; e < n * n; e += 64) {
      const int r = e / n, j = e % n;
      const double2 a = Ar[r * EIG_NMAX + j];
      d2 += cabs2(r == j ? csub(a, c0) : a);
    }
    d2 = wave_sum(d2);
    if (t == 0) {
      c0s = c0;
      nrm[0] = fmax(sqrt(fro2), 1e-300);
      nrm[1] = 0.7 * sqrt(d2 / n);
    }
  }
  __syncthreads();
  const double small = eps * nrm[0];
  if (t < EIG_NMAX) {
    double2 sb = Ar[t * EIG_NMAX + max(t - 1, 0)];
    if (!(cabs_(sb) >= small)) sb = mk(small, 0.0);
    rs[t] = (t >= 1 && t < n) ? crcp(sb) : mk(0.0, 0.0);
    st0[t] = (t == n) ? 1.0 : 0.0;
  }
  if (t == EIG_NMAX) st0[t] = (n == EIG_NMAX) ? 1.0 : 0.0;
  // start from the previous restart's eigenvalues when it solved a problem of this order here
  // (the spectra of consecutive restarts are close: about half the steps), else from the circle
  const bool from_prev = warm && *d.prev == n;
  const int e = t >> 3, c = (t >> 2) & 1, l = t & 3, g8 = t & 7;
  const bool act = e < n;
  double2 zz = mk(0.0, 0.0);
  if (act) {
    if (from_prev) {
      zz = d.theta[e];
    } else {
      double sn, cs;
      sincos(6.283185307179586 * e / n + 0.4, &sn, &cs);
      zz = mk(c0s.x + nrm[1] * cs, c0s.y + nrm[1] * sn);
    }
    if (g8 == 0) zs[e] = zz;
  }
  __syncthreads();
  if (t == 0) *d.prev = 0;
  bool done = !act;
  double wprev = 1e300;
  int ok = 0;
  for (int it = 0; it < maxit; ++it) {
    double2 w = mk(0.0, 0.0);
    if (t < 4 * 64) {  // the fifth wavefront holds no root
      // Hyman's recurrence over the rows of the zero-padded EIG_NMAX x EIG_NMAX matrix, unrolled so
      // that every slot index is a constant.  Rows above n - 1 give zero (their reciprocal
      // subdiagonal is zero) and the row at n adds the start value (x_{n-1} = 1, x'_{n-1} = 0).
      // Slots below r / 4 hold only entries j < r - 1, still zero, and are left out of row r's
      // sum; the slot that holds the newest entry y_r is added last, after the older ones.
      const double cx = (c == 0) ? 1.0 : 0.0, cd = (c == 1) ? 1.0 : 0.0;
      double2 y[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) y[s] = mk(0.0, 0.0);
      double2 ycur = mk(0.0, 0.0);
#pragma unroll
      for (int r = EIG_NMAX; r >= 1; --r) {
        const int sr = r >> 2;
        double2 a0 = mk(0.0, 0.0), a1 = mk(0.0, 0.0);
#pragma unroll
        for (int s = sr + 1; s < 8; ++s) {
          if ((s & 1) == 0) cfma(a0, Ar[(r % EIG_NMAX) * EIG_NMAX + l + 4 * s], y[s]);
          else cfma(a1, Ar[(r % EIG_NMAX) * EIG_NMAX + l + 4 * s], y[s]);
        }
        double2 acc = cadd(a0, a1);
        if (sr < 8) cfma(acc, Ar[(r % EIG_NMAX) * EIG_NMAX + l + 4 * sr], y[sr]);
        double2 full = csub(quad_sum(acc), cmul(zz, ycur));
        const double2 py = half_mirror(ycur);  // x_r on the derivative chain
        full.x -= cd * py.x;
        full.y -= cd * py.y;
        double2 yn = cmul(full, cscale(rs[r % EIG_NMAX], -1.0));
        yn.x += cx * st0[r];
        if (l == ((r - 1) & 3)) y[(r - 1) >> 2] = yn;
        ycur = yn;
      }
      double2 a0 = mk(0.0, 0.0), a1 = mk(0.0, 0.0);
#pragma unroll
      for (int s = 0; s < 8; s += 2) {
        cfma(a0, Ar[l + 4 * s], y[s]);
        cfma(a1, Ar[l + 4 * s + 4], y[s + 1]);
      }
      double2 full = csub(quad_sum(cadd(a0, a1)), cmul(zz, ycur));
      const double2 py = half_mirror(ycur);
      full.x -= cd * py.x;
      full.y -= cd * py.y;
      const double2 other = half_mirror(full);  // p on the derivative chain, p' on the other
      const double2 N = (c == 0) ? cdiv(full, other) : cdiv(other, full);
      // sum over the other roots, two terms per lane, then over the eight lanes of the root
      double2 Sv = mk(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = g8 + 8 * u;
        const double2 term = crcp(csub(zz, zs[min(j, n - 1)]));
        if (j < n && j != e) Sv = cadd(Sv, term);
      }
      Sv = quad_sum(Sv);
      Sv = cadd(Sv, half_mirror(Sv));
      w = cdiv(N, csub(mk(1.0, 0.0), cmul(N, Sv)));
      if (done) w = mk(0.0, 0.0);
    }
    if (__syncthreads_or(act && !(isfinite(w.x) && isfinite(w.y)))) break;
    zz = csub(zz, w);
    if (!done) {
      const double aw = cabs_(w), az = cabs_(zz);
      done = aw <= 4.0 * eps * az || (wprev <= 1e-10 * az && aw >= 0.5 * wprev);
      wprev = aw;
    }
    if (act && g8 == 0) zs[e] = zz;
    if (!__syncthreads_or(act && !done)) {
      ok = 1;
      break;
    }
  }
  if (!ok) return;  // the flag stays 1
  if (act && g8 == 0) d.theta[e] = zz;
  // the k of smallest modulus: key (round(|theta| / max|theta|, 12), Im theta, index)
  if (t < 64) {
    const double2 th = t < n ? zs[t] : mk(0.0, 0.0);
    const double ab = t < n ? cabs_(th) : 0.0;
    double mx = ab;
    mx = fmax(mx, dpp_d<0xB1>(mx));
    mx = fmax(mx, dpp_d<0x4E>(mx));
    mx = fmax(mx, dpp_d<0x124>(mx));
    mx = fmax(mx, dpp_d<0x128>(mx));
    mx = fmax(fmax(rd_lane(mx, 0), rd_lane(mx, 16)), fmax(rd_lane(mx, 32), rd_lane(mx, 48)));
    if (mx == 0.0) mx = 1e-300;
    keys[t] = rint(ab / mx * 1e12);
  }
  __syncthreads();
  if (t < n) {
    const double ke = keys[t];
    int rank = 0;
    for (int o = 0; o < n; ++o) {
      if (o == t) continue;
      const double ko = keys[o];
      const bool less = (ko < ke) || (ko == ke && (zs[o].y < zs[t].y || (zs[o].y == zs[t].y && o < t)));
      rank += less ? 1 : 0;
    }
    if (rank < k) sel[rank] = t;
  }
  __syncthreads();
  if (t == 0) {
    for (int q = 0; q < k; ++q) {
      double2 lq = zs[sel[q]];
      for (int again = 1, guard = 0; again && guard < 4 * k; ++guard) {
        again = 0;
        for (int p = 0; p < q; ++p)
          if (cabs_(csub(lq, lam[p])) < small) {
            lq = cadd(lq, mk(small, 0.0));
            again = 1;
          }
      }
      lam[q] = lq;
      d.sel[q] = sel[q];
    }
  }
  __syncthreads();
  // inverse iteration, one eigenvalue per half wavefront
  const int hw = t >> 5, j = t & 31;
  const bool cj = j < n;
  double2* Uh = U + hw * upk;
  double2* Lh = Lm + hw * 32;
  double2* rh = rU + hw * 32;
  int* ph = pv + hw * 32;
  for (int q0 = 0; q0 < k; q0 += EIG_HALVES) {
    const int qq = q0 + hw, q = min(qq, k - 1);
    const double2 lm = lam[q];
    double2 cr = cj ? Ar[j] : mk(0.0, 0.0);
    if (j == 0) cr = csub(cr, lm);
    for (int p = 0; p + 1 < n; ++p) {
      double2 nr = (cj && j >= p) ? Ar[(p + 1) * EIG_NMAX + j] : mk(0.0, 0.0);
      if (j == p + 1) nr = csub(nr, lm);
      const double2 a = rd_half(cr, p), b = Ar[(p + 1) * EIG_NMAX + p];
      const bool sw = cabs2(b) > cabs2(a);
      double2 piv = sw ? b : a;
      const double2 oth = sw ? a : b;
      if (!(cabs_(piv) >= small)) piv = mk(small, 0.0);
      const double2 ip = crcp(piv), lf = cmul(oth, ip);
      const double2 urow = (j == p) ? piv : (sw ? nr : cr), orow = sw ? cr : nr;
      if (cj && j >= p) Uh[upk_off(p, n) + j - p] = urow;
      if (j == 0) {
        Lh[p] = lf;
        rh[p] = ip;
        ph[p] = sw ? 1 : 0;
      }
      cr = csub(orow, cmul(lf, urow));
    }
    {
      double2 piv = rd_half(cr, n - 1);
      if (!(cabs_(piv) >= small)) piv = mk(small, 0.0);
      if (j == 0) rh[n - 1] = crcp(piv);
    }
    __syncthreads();
    double2 v = mk(cj ? 1.0 : 0.0, 0.0), yv = mk(0.0, 0.0);
    for (int step = 0; step < 2; ++step) {
      if (step == 1) {
        // the factorisation's row operations on the normalised first solution
        v = yv;
        for (int p = 0; p + 1 < n; ++p) {
          const double2 a = rd_half(v, p), b = rd_half(v, p + 1);
          const bool sw = ph[p] != 0;
          const double2 top = sw ? b : a;
          const double2 bot = csub(sw ? a : b, cmul(Lh[p], top));
          if (j == p) v = top;
          if (j == p + 1) v = bot;
        }
      }
      for (int i = n - 1; i >= 0; --i) {
        const double2 yi = cmul(rd_half(v, i), rh[i]);
        if (j == i) yv = yi;
        if (j < i) v = csub(v, cmul(Uh[upk_off(j, n) + i - j], yi));
      }
      const double nn = half_sum(cj ? cabs2(yv) : 0.0);
      yv = cscale(yv, 1.0 / sqrt(nn));
    }
    if (cj && qq < k) d.Y[j + (n + 1) * qq] = yv;
    __syncthreads();
  }
  if (t == 0) {
    *d.flag = 0;
    *d.prev = n;
  }
}

static size_t dr_eig_lds_bytes(int n) {
  return sizeof(double2) * ((size_t)EIG_NMAX * EIG_NMAX + (size_t)EIG_HALVES * (n * (n + 1) / 2) + 2 * EIG_HALVES * 32 +
                            EIG_HALVES * 32 / 4);
}

// ---------------------------------------------------------------- GMRES-DR deflated restart
// Inputs in ks: H ((m+1) x m, unrotated), c, u = c - H d (the residual coordinates s).  Three
// launches on one stream: k_dr_pre forms the harmonic Ritz matrix H + |h|^2 f e_m^T and its
// Hessenberg form; k_dr_eig (orders up to EIG_NMAX) its eigenvalues, the choice of k and their
// eigenvectors; k_dr_post takes the QR algorithm where k_dr_eig did not run or did not settle,
// then forms the new basis change.  Scratch: work (global) of dr_work_elems(m, k) double2.
// Output: P ((m+1) x (k+1), ld m+1) in Pout; ks->H <- Hbar_k, ks->c <- P^H s, rotations reset
// for the full block (unless final_mode), steps = k.  status[0] becomes nonzero on failure
// (2: singular H, 3: no QR convergence, 4: dependent kept vectors); a launch that finds it
// nonzero does nothing.
__global__ void __launch_bounds__(DW) k_dr_pre(KState* ks, int m, int k, double2* work, int* status) {
  extern __shared__ double2 sh[];
  if (*status != 0) return;
  const int t = threadIdx.x;
  const DrWork d = dr_layout(work, m, k);
  double2* A = sh;            // m x m
  double2* X = A + m * m;     // m x m
  double2* v = X + m * m;     // m + 1
  double2* Hb = v + (m + 1);  // (m+1) x m copy of Hbar
  double2* f = Hb + (m + 1) * m;  // m
  __shared__ int fail;
  if (t == 0) fail = 0;
  for (int e = t; e < (m + 1) * m; e += DW) Hb[e] = ks->H[(e % (m + 1)) + LD * (e / (m + 1))];
  __syncthreads();
  const double h = Hb[m + (m + 1) * (m - 1)].x;  // h_{m+1,m}, real >= 0

  // f = H^{-H} e_m from the LU factors of H itself (P H = L U, partial pivoting).  H is upper
  // Hessenberg outside its leading restart block, so column p has nonzeros only in rows
  // p .. hi_p (hi_p = p + 1 past the block): the pivot is chosen among those rows and the
  // elimination updates only them.  With E_p the elimination of column p and P_p its row swap,
  // H^H f = e_m gives f = P_0 E_0^H P_1 E_1^H ... U^{-H} e_m, where U^{-H} e_m = e_m / conj(u_mm)
  // and E_p^H changes only entry p (by the multipliers of column p).
  __shared__ int hiv[MMAX], pvv[MMAX];
  for (int e = t; e < m * m; e += DW) A[e] = Hb[(e % m) + (m + 1) * (e / m)];
  __syncthreads();
  for (int p = 0; p < m; ++p) {
    const double2 ap = (t >= p && t < m) ? A[t + m * p] : mk(0.0, 0.0);
    const unsigned long long nz = __ballot(t >= p && t < m && (ap.x != 0.0 || ap.y != 0.0));
    const int hi = nz ? 63 - __clzll(nz) : p;  // last row with a nonzero in column p
    const double a2 = (t >= p && t <= hi) ? cabs2(ap) : -1.0;
    const int piv = wave_argmax(a2);  // the first row of largest modulus; -1 on NaN
    const double bv = piv >= 0 ? rd_lane(a2, piv) : 0.0;
    if (!(bv > 0.0)) {  // uniform: singular (or not finite)
      if (t == 0) fail = 1;
      break;
    }
    if (t == 0) {
      hiv[p] = hi;
      pvv[p] = piv;
    }
    if (piv != p && t >= p && t < m) {  // swap rows p and piv in columns p .. m-1
      const double2 x = A[p + m * t];
      A[p + m * t] = A[piv + m * t];
      A[piv + m * t] = x;
    }
    __syncthreads();
    const double2 dp = A[p + m * p];
    if (t > p && t <= hi) A[t + m * p] = cdiv(A[t + m * p], dp);  // multipliers, kept in place
    __syncthreads();
    if (t > p && t < m) {  // rows p+1 .. hi of column t
      const double2 up = A[p + m * t];
      for (int r = p + 1; r <= hi; ++r) A[r + m * t] = csub(A[r + m * t], cmul(A[r + m * p], up));
    }
    __syncthreads();
  }
  __syncthreads();
  if (fail) { if (t == 0) *status = 2; return; }
  if (t == 0) {
    for (int i = 0; i < m - 1; ++i) v[i] = mk(0.0, 0.0);
    v[m - 1] = cdiv(mk(1.0, 0.0), cconj(A[(m - 1) + m * (m - 1)]));
    for (int p = m - 2; p >= 0; --p) {
      double2 zp = v[p];
      for (int r = p + 1; r <= hiv[p]; ++r) zp = csub(zp, cmul(cconj(A[r + m * p]), v[r]));
      const int q = pvv[p];
      v[p] = v[q];
      v[q] = zp;
    }
    for (int i = 0; i < m; ++i) f[i] = v[i];
  }
  __syncthreads();
  // G = H + |h|^2 f e_m^T into A
  for (int e = t; e < m * m; e += DW) {
    const int i = e % m, j = e / m;
    double2 g = Hb[i + (m + 1) * j];
    if (j == m - 1) g = cadd(g, cscale(f[i], h * h));
    A[e] = g;
  }
  __syncthreads();
  hessenberg(A, X, v, m);
  __syncthreads();
  for (int e = t; e < m * m; e += DW) {
    d.A[e] = A[e];
    d.X[e] = X[e];
  }
  for (int i = t; i < m; i += DW) d.f[i] = f[i];
  if (t == 0) *d.flag = 1;
}

static size_t dr_pre_lds_bytes(int m) {
  return sizeof(double2) * ((size_t)2 * m * m + (m + 1) + (size_t)(m + 1) * m + m);
}

__global__ void __launch_bounds__(DW) k_dr_post(KState* ks, int m, int k, double2* Pout, int final_mode,
                                                double2* work, int* status) {
  extern __shared__ double2 sh[];
  if (*status != 0) return;
  const int t = threadIdx.x;
  const DrWork d = dr_layout(work, m, k);
  double2* A = sh;                           // m x m
  double2* X = A + m * m;                    // m x m
  double2* v = X + m * m;                    // m + 1
  double2* Hb = v + (m + 1);                 // (m+1) x m copy of Hbar
  double2* W = Hb + (m + 1) * m;             // (m+1) x (k+1)
  double2* T1 = W + (m + 1) * (k + 1);       // (m+1) x k
  double2* f = T1 + (m + 1) * k;             // m
  double2* s = f + m;                        // m + 1
  double2* theta = s + m + 1;                // m
  int* sel = (int*)(theta + m);              // k ints
  (void)v;
  const bool fast = *d.flag == 0;
  for (int e = t; e < (m + 1) * m; e += DW) Hb[e] = ks->H[(e % (m + 1)) + LD * (e / (m + 1))];
  for (int i = t; i <= m; i += DW) s[i] = ks->u[i];
  for (int e = t; e < m * m; e += DW) {
    X[e] = d.X[e];
    if (!fast) A[e] = d.A[e];
  }
  for (int i = t; i < m; i += DW) f[i] = d.f[i];
  if (fast) {
    for (int i = t; i < m; i += DW) theta[i] = d.theta[i];
    for (int q = t; q < k; q += DW) sel[q] = d.sel[q];
    for (int e = t; e < (m + 1) * k; e += DW) T1[e] = (e % (m + 1) < m) ? d.Y[e] : mk(0.0, 0.0);
  }
  __syncthreads();
  const double h = Hb[m + (m + 1) * (m - 1)].x;  // h_{m+1,m}, real >= 0
  if (!fast) {
    if (schur_qr(A, X, m)) { if (t == 0) *status = 3; return; }
    if (t < m) theta[t] = A[t + m * t];
    __syncthreads();
    // the order: key (round(|theta| / max|theta|, 12), Im theta, index); lane e forms its modulus
    // and key once (m <= 64), the maximum is a wavefront max
    __shared__ double keys[DW];
    {
      const double2 th = t < m ? theta[t] : mk(0.0, 0.0);
      const double ab = t < m ? cabs_(th) : 0.0;
      double mx = ab;
      mx = fmax(mx, dpp_d<0xB1>(mx));
      mx = fmax(mx, dpp_d<0x4E>(mx));
      mx = fmax(mx, dpp_d<0x124>(mx));
      mx = fmax(mx, dpp_d<0x128>(mx));
      mx = fmax(fmax(rd_lane(mx, 0), rd_lane(mx, 16)), fmax(rd_lane(mx, 32), rd_lane(mx, 48)));
      if (mx == 0.0) mx = 1e-300;
      keys[t] = rint(ab / mx * 1e12);
    }
    __syncthreads();
    for (int e = t; e < m; e += DW) {
      const double ke = keys[e];
      int rank = 0;
      for (int o = 0; o < m; ++o) {
        if (o == e) continue;
        const double ko = keys[o];
        const bool less = (ko < ke) || (ko == ke && (theta[o].y < theta[e].y || (theta[o].y == theta[e].y && o < e)));
        rank += less ? 1 : 0;
      }
      if (rank < k) sel[rank] = e;
    }
    __syncthreads();
    // eigenvectors of the triangular T = A for the selected values, into T1 columns (length m)
    double tn = 0.0;
    {
      double part = 0.0;
      for (int e = t; e < m * m; e += DW) part += cabs2(A[e]);
      tn = wave_sum(part);
    }
    const double smin = fmax(sqrt(tn) * 2.220446049250313e-16, 1e-300);
    for (int q = t; q < k; q += DW) {
      const int e = sel[q];
      double2* y = T1 + (m + 1) * q;
      for (int i = 0; i < m; ++i) y[i] = mk(0.0, 0.0);
      y[e] = mk(1.0, 0.0);
      const double2 lam = A[e + m * e];
      for (int i = e - 1; i >= 0; --i) {
        double2 acc = mk(0.0, 0.0);
        for (int l = i + 1; l <= e; ++l) cfma(acc, A[i + m * l], y[l]);
        double2 den = csub(A[i + m * i], lam);
        if (cabs_(den) < smin) den = mk(smin, 0.0);
        y[i] = cscale(cdiv(acc, den), -1.0);
      }
    }
  }
  __syncthreads();
  // W[:, q] = [X y_q ; 0]
  for (int e = t; e < (m + 1) * k; e += DW) {
    const int i = e % (m + 1), q = e / (m + 1);
    double2 acc = mk(0.0, 0.0);
    if (i < m)
      for (int l = 0; l < m; ++l) cfma(acc, X[i + m * l], T1[l + (m + 1) * q]);
    W[i + (m + 1) * q] = acc;
  }
  // last column: s (restart) or the harmonic residual direction [-|h|^2 f; h] (final)
  for (int i = t; i <= m; i += DW) {
    double2 w;
    if (final_mode) w = (i < m) ? cscale(f[i], -h * h) : mk(h, 0.0);
    else w = s[i];
    W[i + (m + 1) * k] = w;
  }
  __syncthreads();
  // orthonormalise the k+1 columns (modified Gram-Schmidt, two passes): lane i holds row i
  // (m + 1 <= 64) of the column being orthogonalised; dots are wavefront sums
  for (int q = 0; q <= k; ++q) {
    double2 wq = t <= m ? W[t + (m + 1) * q] : mk(0.0, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
      for (int p = 0; p < q; ++p) {
        const double2 wp = t <= m ? W[t + (m + 1) * p] : mk(0.0, 0.0);
        double2 pr = mk(0.0, 0.0);
        cfmac(pr, wp, wq);
        const double2 dot = wave_sum(pr);
        wq = csub(wq, cmul(dot, wp));
      }
    }
    const double tot = wave_sum(cabs2(wq));
    if (!(tot > 0.0)) { if (t == 0) *status = 4; return; }
    const double inv = 1.0 / sqrt(tot);
    if (t <= m) W[t + (m + 1) * q] = cscale(wq, inv);
  }
  __syncthreads();
  // T1 = Hbar P_k  ((m+1) x k); Hk = P^H T1 ((k+1) x k); c_new = P^H s
  for (int e = t; e < (m + 1) * k; e += DW) {
    const int i = e % (m + 1), q = e / (m + 1);
    double2 acc = mk(0.0, 0.0);
    for (int l = 0; l < m; ++l) cfma(acc, Hb[i + (m + 1) * l], W[l + (m + 1) * q]);
    T1[e] = acc;
  }
  __syncthreads();
  for (int e = t; e < LD * MMAX; e += DW) ks->H[e] = mk(0.0, 0.0);
  __syncthreads();
  for (int e = t; e < (k + 1) * k; e += DW) {
    const int i = e % (k + 1), q = e / (k + 1);
    double2 acc = mk(0.0, 0.0);
    for (int l = 0; l <= m; ++l) cfmac(acc, W[l + (m + 1) * i], T1[l + (m + 1) * q]);
    ks->H[i + LD * q] = acc;
  }
  for (int i = t; i <= MMAX; i += DW) {
    double2 acc = mk(0.0, 0.0);
    if (i <= k)
      for (int l = 0; l <= m; ++l) cfmac(acc, W[l + (m + 1) * i], s[l]);
    ks->c[i] = acc;
  }
  for (int e = t; e < (m + 1) * (k + 1); e += DW) Pout[e] = W[e];
  __syncthreads();
  __syncthreads();
  if (!final_mode) {  // A is free again: scratch for the block QR
    if (k + 1 <= DW && k * (k + 1) / 2 <= QRL_MAXROT) qr_block_wave(ks, k, A);
    else qr_block_lds(ks, k, A);
  }
  if (t == 0) {
    ks->steps = k;
    ks->done = 0;
    ks->breakdown = 0;
  }
}


size_t dr_work_elems(int m, int k) { return (size_t)2 * m * m + 2 * (size_t)m + (size_t)(m + 1) * k + (k + 3) / 2 + 2; }

static size_t dr_post_lds_bytes(int m, int k) {
  return sizeof(double2) * ((size_t)2 * m * m + (m + 1) + (size_t)(m + 1) * m + (size_t)(m + 1) * (k + 1) +
                            (size_t)(m + 1) * k + m + (m + 1) + m + (k + 1) / 2 + 2);
}

static size_t dr_post_static_lds() {
  static size_t bytes = 0;
  if (!bytes) {
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, (const void*)k_dr_post) != hipSuccess) return (size_t)1 << 30;
    bytes = fa.sharedSizeBytes + 1;
  }
  return bytes;
}

// DMG_RESTART_QR=1 sends every restart to the QR algorithm; DMG_RESTART_QR=2 runs the
// simultaneous iteration with no steps, so that it gives up and the QR algorithm takes over
// (read at each launch, so that one process can compare the eigenvalue paths).
static int dr_force_qr() {
  const char* e = getenv("DMG_RESTART_QR");
  return (e && *e) ? atoi(e) : 0;
}

bool dr_restart_fits(int m, int k) {
  return k >= 1 && m + 1 <= DW && (size_t)m * m >= (size_t)(k + 1) * k &&
         dr_post_lds_bytes(m, k) + dr_post_static_lds() <= 160 * 1024;
}

void launch_dr_restart(hipStream_t st, KState* ks, int m, int k, double2* Pout, int final_mode, double2* work,
                       int* status, int warm) {
  const size_t shp = dr_pre_lds_bytes(m), sho = dr_post_lds_bytes(m, k);
  DMG_CHECK(dr_restart_fits(m, k), DMG_E_INVALID, "GMRES-DR sizes too large for the one-workgroup restart");
  DMG_HIP(ensure_dyn_lds((const void*)k_dr_pre, shp));
  DMG_HIP(ensure_dyn_lds((const void*)k_dr_post, sho));
  hipLaunchKernelGGL(k_dr_pre, dim3(1), dim3(DW), shp, st, ks, m, k, work, status);
  DMG_LAUNCH_CHECK();
  const int force = dr_force_qr();
  if (m <= EIG_NMAX && force != 1) {
    const size_t she = dr_eig_lds_bytes(m);
    DMG_HIP(ensure_dyn_lds((const void*)k_dr_eig, she));
    hipLaunchKernelGGL(k_dr_eig, dim3(1), dim3(EIG_THREADS), she, st, work, m, k, warm, force == 2 ? 0 : EIG_MAXIT,
                       (const int*)status);
    DMG_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_dr_post, dim3(1), dim3(DW), sho, st, ks, m, k, Pout, final_mode, work, status);
  DMG_LAUNCH_CHECK();
}

}  // namespace dmg
