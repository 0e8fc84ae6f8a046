// Long-cycle GMRES-DR(m, k) and GMRES-Proj(m, k) (Methods section: the paper's coarse and
// fine-grid deflation uses m = 200, k = 40).  The small-dense state of the short-cycle solvers
// (KState, m <= 64, restart in one wavefront's LDS) does not hold such cycles, so these keep
// their Arnoldi matrix, rotations and right-hand side in device memory (KBig) and run the
// harmonic-Ritz restart in one workgroup with its matrices in device memory (L2 resident).
//
// The dense steps are written once for a "team" of threads: on the device the team is a
// workgroup (sync = __syncthreads), on the host a single thread (sync does nothing), so the
// same code can be checked on the CPU.  Parallel loops stride by the team size; sections
// guarded by `lead()` run on one thread.  Data that one team member writes and another reads
// is separated by a sync.
#pragma once

#include "common.h"

namespace dmg {

constexpr int MBIG = 256;                             // longest cycle
constexpr int KBIG = 64;                              // most kept vectors
constexpr int LDBIG = MBIG + 1;                         // leading dimension of (m + 1) x m matrices
constexpr int RBIG = MBIG * (MBIG + 1) / 2 + 2 * MBIG;    // Givens rotations held

// Small-dense state of one long Krylov cycle (FP64, device memory).
struct KBig {
  double2 H[LDBIG * MBIG];   // unrotated Arnoldi matrix Hbar, column-major
  double2 R[LDBIG * MBIG];   // its rotated (upper triangular) copy
  double2 c[LDBIG];        // unrotated right-hand side coordinates (beta e1 after a fresh start)
  double2 g[LDBIG];        // rotated right-hand side
  double2 y[LDBIG];        // least-squares solution
  double2 u[LDBIG];        // residual coordinates c - Hbar y
  double2 h1[LDBIG];       // Gram-Schmidt coefficients of the current column, first pass
  double2 h2[LDBIG];       // second pass
  double2 rs[RBIG];      // rotation q acts on rows (ri[q], rj[q]) as [c s; -conj(s) c]
  double rc[RBIG];
  int ri[RBIG], rj[RBIG];
  int nrot, steps, done, breakdown;
  double tol_abs;        // stop when |g[steps]| <= tol_abs
  double est;            // least-squares residual norm
  double beta;           // norm of the cycle's starting residual
  double bnorm;          // ||b|| of the enclosing solve
  double wn0;            // ||A v_j||^2 before orthogonalisation
  double wn;             // ||w||^2 after it
};

// status mirror read by the host (layout of KBig's tail)
struct KBigStatus {
  int nrot, steps, done, breakdown;
  double tol_abs, est, beta, bnorm;
};

// device-memory workspace of the restart (double2 entries)
inline size_t big_restart_work_elems() { return (size_t)6 * LDBIG * LDBIG + 4 * LDBIG; }

// ---------------------------------------------------------------- complex helpers
__host__ __device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }
__host__ __device__ inline double cabsd(double2 a) { return hypot(a.x, a.y); }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__host__ __device__ inline double2 csqrt_(double2 z) {
  const double r = cabsd(z);
  if (r == 0.0) return mk(0.0, 0.0);
  double re = sqrt(0.5 * (r + fabs(z.x)));
  double im = 0.5 * z.y / re;
  if (z.x < 0.0) {
    const double t = fabs(im);
    im = z.y >= 0.0 ? re : -re;
    re = t;
  }
  return mk(re, im);
}
// Givens rotation with real c >= 0: [c s; -conj(s) c] [a; b] = [r; 0]
__host__ __device__ inline void givens(double2 a, double2 b, double& c, double2& s, double2& r) {
  const double na = cabsd(a), nb = cabsd(b);
  if (nb == 0.0) {
    c = 1.0;
    s = mk(0.0, 0.0);
    r = a;
    return;
  }
  if (na == 0.0) {
    c = 0.0;
    s = cscale(cconj(b), 1.0 / nb);
    r = mk(nb, 0.0);
    return;
  }
  const double nu = hypot(na, nb);
  c = na / nu;
  const double2 ph = cscale(a, 1.0 / na);
  s = cscale(cmul(ph, cconj(b)), 1.0 / nu);
  r = cscale(ph, nu);
}
// rows: [x; y] <- [c x + s y; -conj(s) x + c y]
__host__ __device__ inline void rot_rows(double c, double2 s, double2& x, double2& y) {
  const double2 nx = cadd(cscale(x, c), cmul(s, y));
  const double2 ny = csub(cscale(y, c), cmul(cconj(s), x));
  x = nx;
  y = ny;
}
// columns (right multiplication by the adjoint): [p q] <- [p c + q conj(s), -p s + q c]
__host__ __device__ inline void rot_cols(double c, double2 s, double2& p, double2& q) {
  const double2 np = cadd(cscale(p, c), cmul(q, cconj(s)));
  const double2 nq = csub(cscale(q, c), cmul(p, s));
  p = np;
  q = nq;
}

// ---------------------------------------------------------------- teams
struct HostTeam {
  double2* shm;  // scratch standing in for LDS
  int tid() const { return 0; }
  int size() const { return 1; }
  bool lead() const { return true; }
  void sync() const {}
};

// Harmonic-Ritz restart of GMRES-DR on an (m+1) x m Arnoldi matrix (Methods: the deflated
// restart of GMRES-DR keeps the k harmonic Ritz vectors of smallest magnitude and the
// residual direction).  With Hm the leading m x m block and h = Hbar[m][m-1]:
//   f = Hm^{-H} e_m;  G = Hm + |h|^2 f e_m^T;  eigenpairs (theta, g) of G, the k smallest |theta|
//   (ties by Im theta, then index, magnitudes compared to 12 digits of the largest);
//   W = [g_1 .. g_k padded with a zero row | s], P = orthonormal basis of W (Gram-Schmidt
//   applied twice, columns in order);  Hbar_k = P^H Hbar P_k;  c_new = P^H s.
// s is the least-squares residual c - Hbar y (restart) or the harmonic residual direction
// [-|h|^2 f; h] (final compression).  Outputs: P ((m+1) x (k+1), ld m + 1), and, in the
// restart, KBig holding Hbar_k, c_new, its Givens QR (rotations, R, g) and steps = k.
// status: 0 ok; 1 singular Hm; 2 eigenvalue iteration did not converge.
// work: big_restart_work_elems() double2; shm: at least 2 * LDBIG + 16 double2.
template <class Team>
__host__ __device__ int big_restart_body(Team& tm, KBig* kb, int m, int k, double2* P, int final_mode,
                                         double2* work) {
  const int t = tm.tid(), nt = tm.size();
  double2* A = work;                  // LU of Hm^H, then reused
  double2* T = work + LDBIG * LDBIG;      // G, Hessenberg form, Schur form
  double2* Z = work + 2 * LDBIG * LDBIG;  // Schur vectors
  double2* X = work + 3 * LDBIG * LDBIG;  // eigenvectors of T (columns), then of G
  double2* W = work + 4 * LDBIG * LDBIG;  // [G_k | s], then P
  double2* T1 = work + 5 * LDBIG * LDBIG; // Hbar P_k
  double2* f = work + 6 * LDBIG * LDBIG;  // f, then s
  double2* lam = f + LDBIG;             // eigenvalues
  int* order = (int*)(lam + LDBIG);     // kept eigenvalue indices
  double2* sh = tm.shm;               // shared scalars and vectors
  int* shi = (int*)(sh + 2 * LDBIG);
  const double ulp = 2.220446049250313e-16;

  // ---- f = Hm^{-H} e_m : LU with partial pivoting of A = Hm^H
  for (int e = t; e < m * m; e += nt) {
    const int i = e % m, j = e / m;
    A[i + LDBIG * j] = cconj(kb->H[j + LDBIG * i]);
  }
  for (int i = t; i < m; i += nt) f[i] = mk(i == m - 1 ? 1.0 : 0.0, 0.0);
  tm.sync();
  for (int q = 0; q < m; ++q) {
    if (tm.lead()) {
      int p = q;
      double best = cabs1(A[q + LDBIG * q]);
      for (int i = q + 1; i < m; ++i) {
        const double v = cabs1(A[i + LDBIG * q]);
        if (v > best) {
          best = v;
          p = i;
        }
      }
      shi[0] = best == 0.0 ? -1 : p;
      if (p != q && best != 0.0) {
        for (int j = 0; j < m; ++j) {
          const double2 tmp = A[q + LDBIG * j];
          A[q + LDBIG * j] = A[p + LDBIG * j];
          A[p + LDBIG * j] = tmp;
        }
        const double2 tmp = f[q];
        f[q] = f[p];
        f[p] = tmp;
      }
    }
    tm.sync();
    if (shi[0] < 0) return 1;
    const double2 piv = A[q + LDBIG * q];
    for (int i = q + 1 + t; i < m; i += nt) {
      const double2 l = cdiv(A[i + LDBIG * q], piv);
      A[i + LDBIG * q] = l;
      for (int j = q + 1; j < m; ++j) A[i + LDBIG * j] = csub(A[i + LDBIG * j], cmul(l, A[q + LDBIG * j]));
      f[i] = csub(f[i], cmul(l, f[q]));
    }
    tm.sync();
  }
  // back substitution (column oriented)
  for (int q = m - 1; q >= 0; --q) {
    if (tm.lead()) f[q] = cdiv(f[q], A[q + LDBIG * q]);
    tm.sync();
    for (int i = t; i < q; i += nt) f[i] = csub(f[i], cmul(A[i + LDBIG * q], f[q]));
    tm.sync();
  }
  const double2 hlast = kb->H[m + LDBIG * (m - 1)];
  const double h2 = cabs2(hlast);
  // ---- G = Hm + |h|^2 f e_m^T ; Z = I
  for (int e = t; e < m * m; e += nt) {
    const int i = e % m, j = e / m;
    double2 v = kb->H[i + LDBIG * j];
    if (j == m - 1) v = cadd(v, cscale(f[i], h2));
    T[i + LDBIG * j] = v;
    Z[i + LDBIG * j] = mk(i == j ? 1.0 : 0.0, 0.0);
  }
  tm.sync();
  // ---- Householder reduction to upper Hessenberg form, T <- Q^H T Q, Z <- Z Q
  double2* v = sh;  // Householder vector (length <= m)
  for (int q = 0; q + 2 < m; ++q) {
    const int L = m - q - 1;  // rows q+1 .. m-1
    if (tm.lead()) {
      double xn2 = 0.0;
      for (int i = 0; i < L; ++i) xn2 += cabs2(T[q + 1 + i + LDBIG * q]);
      const double2 x0 = T[q + 1 + LDBIG * q];
      double tail = xn2 - cabs2(x0);
      const double xn = sqrt(xn2);
      int skip = (tail <= 0.0 || xn == 0.0) ? 1 : 0;
      if (!skip) {
        const double ax0 = cabsd(x0);
        const double2 ph = ax0 > 0.0 ? cscale(x0, 1.0 / ax0) : mk(1.0, 0.0);
        const double2 alpha = cscale(ph, -xn);  // -e^{i arg x0} ||x||
        v[0] = csub(x0, alpha);
        for (int i = 1; i < L; ++i) v[i] = T[q + 1 + i + LDBIG * q];
        double vn2 = cabs2(v[0]) + tail;
        const double inv = 1.0 / sqrt(vn2);
        for (int i = 0; i < L; ++i) v[i] = cscale(v[i], inv);
        sh[LDBIG] = alpha;
      }
      shi[0] = skip;
    }
    tm.sync();
    if (!shi[0]) {
      // rows q+1.. of T, columns q..m-1: T[:, c] -= 2 v (v^H T[:, c])
      for (int c = q + t; c < m; c += nt) {
        double2 d = mk(0.0, 0.0);
        for (int i = 0; i < L; ++i) cfmac(d, v[i], T[q + 1 + i + LDBIG * c]);
        d = cscale(d, 2.0);
        for (int i = 0; i < L; ++i) T[q + 1 + i + LDBIG * c] = csub(T[q + 1 + i + LDBIG * c], cmul(v[i], d));
      }
      tm.sync();
      // columns q+1.. of T (all rows) and of Z: row r: T[r, :] -= 2 (T[r, :] v) v^H
      for (int r = t; r < 2 * m; r += nt) {
        double2* M = r < m ? T : Z;
        const int rr = r < m ? r : r - m;
        double2 d = mk(0.0, 0.0);
        for (int i = 0; i < L; ++i) cfma(d, M[rr + LDBIG * (q + 1 + i)], v[i]);
        d = cscale(d, 2.0);
        for (int i = 0; i < L; ++i) M[rr + LDBIG * (q + 1 + i)] = csub(M[rr + LDBIG * (q + 1 + i)], cmul(d, cconj(v[i])));
      }
      tm.sync();
      if (tm.lead()) {
        T[q + 1 + LDBIG * q] = sh[LDBIG];
        for (int i = q + 2; i < m; ++i) T[i + LDBIG * q] = mk(0.0, 0.0);
      }
    }
    tm.sync();
  }
  // ---- complex Schur form by single-shift QR sweeps (bulge chasing with Givens rotations)
  // shared: sh[0..1] rotation (s) by parity, sh[2..3] rotation (c) as double, shi[1] lo, shi[2] status
  {
    int hi = m - 1, its = 0, total = 0;
    while (hi > 0) {
      // deflation search: largest l in [1, hi] with a negligible T[l][l-1]
      if (tm.lead()) {
        int lo = 0;
        for (int l = hi; l >= 1; --l) {
          const double sub = cabs1(T[l + LDBIG * (l - 1)]);
          double scale = cabs1(T[l - 1 + LDBIG * (l - 1)]) + cabs1(T[l + LDBIG * l]);
          if (scale == 0.0) scale = 1.0;
          if (sub <= ulp * scale) {
            T[l + LDBIG * (l - 1)] = mk(0.0, 0.0);
            lo = l;
            break;
          }
        }
        shi[1] = lo;
        shi[2] = 0;
        if (lo < hi) {
          if (total > 30 * m) {
            shi[2] = 1;
          } else {
            // shift: eigenvalue of the trailing 2 x 2 block closer to its last diagonal entry,
            // or an exceptional shift after 10 and 20 sweeps without deflation
            double2 mu;
            const double2 a = T[hi - 1 + LDBIG * (hi - 1)], b = T[hi - 1 + LDBIG * hi];
            const double2 cc = T[hi + LDBIG * (hi - 1)], d = T[hi + LDBIG * hi];
            if (its == 10 || its == 20) {
              mu = cadd(d, mk(0.75 * fabs(cc.x) + 0.75 * fabs(cc.y), 0.0));
            } else {
              const double2 half = cscale(csub(a, d), 0.5);
              const double2 disc = csqrt_(cadd(cmul(half, half), cmul(b, cc)));
              const double2 m1 = cadd(cadd(d, half), disc), m2 = csub(cadd(d, half), disc);
              mu = cabs1(csub(m1, d)) <= cabs1(csub(m2, d)) ? m1 : m2;
            }
            double cs;
            double2 sn, r;
            givens(csub(T[lo + LDBIG * lo], mu), T[lo + 1 + LDBIG * lo], cs, sn, r);
            sh[0] = sn;
            ((double*)(sh + 2))[0] = cs;
          }
        }
      }
      tm.sync();
      const int lo = shi[1];
      if (shi[2]) return 2;
      if (lo == hi) {
        --hi;
        its = 0;
        continue;
      }
      for (int i = lo; i < hi; ++i) {
        const int par = (i - lo) & 1;
        const double cs = ((double*)(sh + 2))[par];
        const double2 sn = sh[par];
        if (tm.lead()) {
          // corner rows/columns i, i+1: the left rotation, then the right one
          double2 a00 = T[i + LDBIG * i], a01 = T[i + LDBIG * (i + 1)];
          double2 a10 = T[i + 1 + LDBIG * i], a11 = T[i + 1 + LDBIG * (i + 1)];
          rot_rows(cs, sn, a00, a10);
          rot_rows(cs, sn, a01, a11);
          rot_cols(cs, sn, a00, a01);
          rot_cols(cs, sn, a10, a11);
          T[i + LDBIG * i] = a00;
          T[i + LDBIG * (i + 1)] = a01;
          T[i + 1 + LDBIG * i] = a10;
          T[i + 1 + LDBIG * (i + 1)] = a11;
          if (i + 2 <= hi) {
            // row i + 2 of columns i, i+1: the new bulge at (i + 2, i)
            double2 b0 = mk(0.0, 0.0), b1 = T[i + 2 + LDBIG * (i + 1)];
            rot_cols(cs, sn, b0, b1);
            T[i + 2 + LDBIG * (i + 1)] = b1;
            // the next rotation annihilates it against (i + 1, i)
            double c2;
            double2 s2, r2;
            givens(a10, b0, c2, s2, r2);
            T[i + 1 + LDBIG * i] = r2;
            T[i + 2 + LDBIG * i] = mk(0.0, 0.0);
            sh[par ^ 1] = s2;
            ((double*)(sh + 2))[par ^ 1] = c2;
          }
        }
        // the rest of rows i, i+1 (columns i+2 .. m-1), of columns i, i+1 (rows 0 .. i-1)
        // and of Z's columns i, i+1 (all rows)
        const int nr = m - (i + 2) > 0 ? m - (i + 2) : 0;
        for (int e = t; e < nr + i + m; e += nt) {
          if (e < nr) {
            const int c = i + 2 + e;
            double2 x = T[i + LDBIG * c], y = T[i + 1 + LDBIG * c];
            rot_rows(cs, sn, x, y);
            T[i + LDBIG * c] = x;
            T[i + 1 + LDBIG * c] = y;
          } else if (e < nr + i) {
            const int r = e - nr;
            double2 p = T[r + LDBIG * i], q = T[r + LDBIG * (i + 1)];
            rot_cols(cs, sn, p, q);
            T[r + LDBIG * i] = p;
            T[r + LDBIG * (i + 1)] = q;
          } else {
            const int r = e - nr - i;
            double2 p = Z[r + LDBIG * i], q = Z[r + LDBIG * (i + 1)];
            rot_cols(cs, sn, p, q);
            Z[r + LDBIG * i] = p;
            Z[r + LDBIG * (i + 1)] = q;
          }
        }
        tm.sync();
      }
      ++its;
      ++total;
    }
  }
  // ---- eigenvalues, the k smallest in magnitude (ties by imaginary part, then index)
  for (int i = t; i < m; i += nt) lam[i] = T[i + LDBIG * i];
  tm.sync();
  if (tm.lead()) {
    double mx = 0.0;
    for (int i = 0; i < m; ++i) mx = fmax(mx, cabsd(lam[i]));
    if (mx == 0.0) mx = 1.0;
    // selection of the k smallest keys (k passes over m entries)
    for (int q = 0; q < k; ++q) {
      int best = -1;
      double bm = 0.0, bi = 0.0;
      for (int i = 0; i < m; ++i) {
        bool used = false;
        for (int p = 0; p < q; ++p) used = used || order[p] == i;
        if (used) continue;
        const double key = rint(cabsd(lam[i]) / mx * 1e12);
        const double im = lam[i].y;
        if (best < 0 || key < bm || (key == bm && (im < bi || (im == bi && i < best)))) {
          best = i;
          bm = key;
          bi = im;
        }
      }
      order[q] = best;
    }
  }
  tm.sync();
  // ---- eigenvectors of T for the kept eigenvalues (back substitution), then g = Z x
  for (int q = t; q < k; q += nt) {
    const int i0 = order[q];
    const double2 l0 = lam[i0];
    double2* x = X + LDBIG * q;
    for (int r = 0; r < m; ++r) x[r] = mk(r == i0 ? 1.0 : 0.0, 0.0);
    double tnorm = 0.0;
    for (int r = 0; r <= i0; ++r) tnorm = fmax(tnorm, cabs1(T[r + LDBIG * r]));
    const double small = ulp * (tnorm > 0.0 ? tnorm : 1.0);
    for (int r = i0 - 1; r >= 0; --r) {
      double2 acc = mk(0.0, 0.0);
      for (int l = r + 1; l <= i0; ++l) cfma(acc, T[r + LDBIG * l], x[l]);
      double2 den = csub(T[r + LDBIG * r], l0);
      if (cabs1(den) < small) den = mk(small, 0.0);
      x[r] = cscale(cdiv(acc, den), -1.0);
    }
  }
  tm.sync();
  for (int e = t; e < m * k; e += nt) {
    const int r = e % m, q = e / m;
    const int i0 = order[q];
    double2 acc = mk(0.0, 0.0);
    for (int l = 0; l <= i0; ++l) cfma(acc, Z[r + LDBIG * l], X[l + LDBIG * q]);
    W[r + LDBIG * q] = acc;
  }
  tm.sync();
  // ---- s, the last column of W (kept in X's column k for c_new = P^H s): the least-squares
  // residual coordinates u = c - Hbar y of the cycle (restart), or [-|h|^2 f; h] (final)
  double2* sv = X + LDBIG * k;
  for (int r = t; r <= m; r += nt) {
    const double2 sr = final_mode ? (r < m ? cscale(f[r], -h2) : hlast) : kb->u[r];
    W[r + LDBIG * k] = sr;
    sv[r] = sr;
  }
  for (int q = t; q < k; q += nt) W[m + LDBIG * q] = mk(0.0, 0.0);
  tm.sync();
  // ---- P: Gram-Schmidt twice over the columns of W, in order
  for (int q = 0; q <= k; ++q) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int p = t; p < q; p += nt) {
        double2 d = mk(0.0, 0.0);
        for (int r = 0; r <= m; ++r) cfmac(d, W[r + LDBIG * p], W[r + LDBIG * q]);
        sh[p] = d;
      }
      tm.sync();
      for (int r = t; r <= m; r += nt) {
        double2 acc = W[r + LDBIG * q];
        for (int p = 0; p < q; ++p) acc = csub(acc, cmul(sh[p], W[r + LDBIG * p]));
        W[r + LDBIG * q] = acc;
      }
      tm.sync();
    }
    if (tm.lead()) {
      double n2 = 0.0;
      for (int r = 0; r <= m; ++r) n2 += cabs2(W[r + LDBIG * q]);
      ((double*)(sh + LDBIG))[0] = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
      shi[3] = n2 > 0.0 ? 0 : 1;
    }
    tm.sync();
    const double inv = ((double*)(sh + LDBIG))[0];
    for (int r = t; r <= m; r += nt) W[r + LDBIG * q] = cscale(W[r + LDBIG * q], inv);
    tm.sync();
  }
  for (int e = t; e < (m + 1) * (k + 1); e += nt) {
    const int r = e % (m + 1), q = e / (m + 1);
    P[r + (m + 1) * q] = W[r + LDBIG * q];
  }
  // ---- Hbar_k = P^H Hbar P_k  (T1 = Hbar P_k first)
  for (int e = t; e < (m + 1) * k; e += nt) {
    const int r = e % (m + 1), q = e / (m + 1);
    double2 acc = mk(0.0, 0.0);
    for (int j = 0; j < m; ++j) cfma(acc, kb->H[r + LDBIG * j], W[j + LDBIG * q]);
    T1[r + LDBIG * q] = acc;
  }
  tm.sync();
  // new state: Hbar_k in the leading (k+1) x k block, zero elsewhere; c = P^H s
  for (int e = t; e < LDBIG * MBIG; e += nt) {
    const int r = e % LDBIG, q = e / LDBIG;
    double2 acc = mk(0.0, 0.0);
    if (r <= k && q < k)
      for (int i = 0; i <= m; ++i) cfmac(acc, W[i + LDBIG * r], T1[i + LDBIG * q]);
    kb->R[e] = acc;  // staged; copied to H below
  }
  tm.sync();
  if (final_mode) {
    for (int e = t; e < LDBIG * MBIG; e += nt) kb->H[e] = kb->R[e];
    return 0;
  }
  for (int r = t; r < LDBIG; r += nt) {
    double2 acc = mk(0.0, 0.0);
    if (r <= k)
      for (int i = 0; i <= m; ++i) cfmac(acc, W[i + LDBIG * r], sv[i]);
    f[r] = acc;  // c_new (f is no longer needed)
  }
  tm.sync();
  for (int e = t; e < LDBIG * MBIG; e += nt) kb->H[e] = kb->R[e];
  for (int r = t; r < LDBIG; r += nt) {
    kb->c[r] = f[r];
    kb->g[r] = f[r];
  }
  tm.sync();
  // ---- Givens QR of the (k+1) x k block: column q, rows k .. q+1 from the bottom up
  if (tm.lead()) {
    int nrot = 0;
    for (int q = 0; q < k; ++q) {
      for (int i = k; i > q; --i) {
        double cs;
        double2 sn, r;
        givens(kb->R[i - 1 + LDBIG * q], kb->R[i + LDBIG * q], cs, sn, r);
        kb->R[i - 1 + LDBIG * q] = r;
        kb->R[i + LDBIG * q] = mk(0.0, 0.0);
        for (int j = q + 1; j < k; ++j) rot_rows(cs, sn, kb->R[i - 1 + LDBIG * j], kb->R[i + LDBIG * j]);
        rot_rows(cs, sn, kb->g[i - 1], kb->g[i]);
        kb->rc[nrot] = cs;
        kb->rs[nrot] = sn;
        kb->ri[nrot] = i - 1;
        kb->rj[nrot] = i;
        ++nrot;
      }
    }
    kb->nrot = nrot;
    kb->steps = k;
    kb->est = cabsd(kb->g[k]);
    kb->done = 0;
    kb->breakdown = 0;
  }
  tm.sync();
  return 0;
}

// One Arnoldi column j: H[:, j] = h1 + h2 (rows 0..j), H[j+1][j] = ||w|| (0 at a breakdown:
// ||w|| <= 1e-14 ||A v_j||), the held rotations and a new one on rows (j, j+1) applied to R's
// column j and to g; est = |g[j+1]|; done when est <= tol_abs or at a breakdown.
template <class Team>
__host__ __device__ void big_column_body(Team& tm, KBig* kb, int j) {
  const int t = tm.tid(), nt = tm.size();
  double2* col = tm.shm;
  for (int i = t; i <= j; i += nt) col[i] = cadd(kb->h1[i], kb->h2[i]);
  tm.sync();
  if (tm.lead()) {
    const double hn = sqrt(kb->wn > 0.0 ? kb->wn : 0.0);
    const bool bd = !(hn > 1e-14 * sqrt(kb->wn0 > 0.0 ? kb->wn0 : 0.0));
    col[j + 1] = mk(bd ? 0.0 : hn, 0.0);
    for (int i = 0; i <= j + 1; ++i) kb->H[i + LDBIG * j] = col[i];
    for (int q = 0; q < kb->nrot; ++q) rot_rows(kb->rc[q], kb->rs[q], col[kb->ri[q]], col[kb->rj[q]]);
    double cs;
    double2 sn, r;
    givens(col[j], col[j + 1], cs, sn, r);
    col[j] = r;
    col[j + 1] = mk(0.0, 0.0);
    const int q = kb->nrot;
    kb->rc[q] = cs;
    kb->rs[q] = sn;
    kb->ri[q] = j;
    kb->rj[q] = j + 1;
    kb->nrot = q + 1;
    rot_rows(cs, sn, kb->g[j], kb->g[j + 1]);
    for (int i = 0; i <= j + 1; ++i) kb->R[i + LDBIG * j] = col[i];
    kb->est = cabsd(kb->g[j + 1]);
    kb->steps = j + 1;
    kb->breakdown = bd ? 1 : 0;
    kb->done = (bd || kb->est <= kb->tol_abs) ? 1 : 0;
  }
  tm.sync();
}

// y = R^{-1} g over the first `steps` columns, then u = c - Hbar y (steps + 1 rows).
template <class Team>
__host__ __device__ void big_lssolve_body(Team& tm, KBig* kb) {
  const int t = tm.tid(), nt = tm.size();
  const int n = kb->steps;
  double2* acc = tm.shm;
  for (int i = t; i < n; i += nt) acc[i] = kb->g[i];
  tm.sync();
  for (int q = n - 1; q >= 0; --q) {
    if (tm.lead()) {
      const double2 d = kb->R[q + LDBIG * q];
      acc[q] = (d.x == 0.0 && d.y == 0.0) ? mk(0.0, 0.0) : cdiv(acc[q], d);
    }
    tm.sync();
    for (int i = t; i < q; i += nt) acc[i] = csub(acc[i], cmul(kb->R[i + LDBIG * q], acc[q]));
    tm.sync();
  }
  for (int i = t; i < LDBIG; i += nt) kb->y[i] = i < n ? acc[i] : mk(0.0, 0.0);
  tm.sync();
  for (int r = t; r <= n; r += nt) {
    double2 a = kb->c[r];
    for (int j = 0; j < n; ++j) a = csub(a, cmul(kb->H[r + LDBIG * j], kb->y[j]));
    kb->u[r] = a;
  }
  tm.sync();
}

}  // namespace dmg
