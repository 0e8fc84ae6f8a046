// Setup kernels of the multigrid hierarchy (Methods section): batched CG on the
// normal equations for the near-null vectors, the chiral split with local
// orthonormalisation that gives the prolongator, and the Galerkin product
// P^dagger A P assembled block by block.
#include "kernels.h"

namespace dmg {

constexpr int SB = 256;

__device__ inline double2 wsum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// ---------------------------------------------------------------- batched dots
// out[f] = a_f^H b_f (real and imaginary parts interleaved) for f < nvec; fields are
// consecutive with n complex entries each.  Grid (G, nvec); the last workgroup reduces.
__global__ void __launch_bounds__(SB) k_batched_dots(int64_t n, const double2* __restrict__ a,
                                                     const double2* __restrict__ b, double* out, double2* partials,
                                                     unsigned* counter) {
  __shared__ double2 red[SB / 64];
  __shared__ int am_last;
  const int f = blockIdx.y;
  const double2* af = a + (int64_t)f * n;
  const double2* bf = b + (int64_t)f * n;
  double2 acc = mk(0.0, 0.0);
  const int64_t stride = (int64_t)gridDim.x * SB;
  for (int64_t e = (int64_t)blockIdx.x * SB + threadIdx.x; e < n; e += stride) cfmac(acc, af[e], bf[e]);
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 r = red[0];
    for (int w = 1; w < SB / 64; ++w) r = cadd(r, red[w]);
    // device-scope atomic stores reach the coherence point: after the wait below no fence (and
    // so no L2 write-back) is needed before the ticket, nor an invalidation after it
    double2* pp = &partials[(int64_t)f * gridDim.x + blockIdx.x];
    __hip_atomic_store(&pp->x, r.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&pp->y, r.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    const unsigned t = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (t == gridDim.x * gridDim.y - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!am_last) return;
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int q = threadIdx.x; q < (int)gridDim.y; q += SB) {
    const double2* pq = partials + (int64_t)q * gridDim.x;
    double2 r = mk(0.0, 0.0);
    for (int b0 = 0; b0 < (int)gridDim.x; b0 += 8) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = b0 + u < (int)gridDim.x ? mk(__hip_atomic_load(&pq[b0 + u].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                            __hip_atomic_load(&pq[b0 + u].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                                       : mk(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (b0 + u < (int)gridDim.x) r = cadd(r, v[u]);
    }
    out[2 * q] = r.x;
    out[2 * q + 1] = r.y;
  }
}

void launch_batched_dots(hipStream_t s, int64_t n, int nvec, const double2* a, const double2* b, double* out,
                         double2* partials, unsigned* counter) {
  int G = (int)((n + SB - 1) / SB);
  if (G > 128) G = 128;
  hipLaunchKernelGGL(k_batched_dots, dim3(G, nvec), dim3(SB), 0, s, n, a, b, out, partials, counter);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- batched CG scalars
// phase 0: alpha_f = rr_f / Re(p_f^H q_f) for active fields (pq holds complex pairs).
// phase 1: after the x, r update and rr_new = ||r||^2: converged fields (rr_new <= tol^2 b2)
//          become inactive; beta_f = rr_new / rr, rr = rr_new.
__global__ void k_cg_scalars(int nvec, const double* pq, const double* rr_new, double* rr, double* alpha,
                             double* beta, int* active, const double* b2, double tol2, int* iters, int phase) {
  const int f = threadIdx.x;
  if (f >= nvec) return;
  if (!active[f]) { alpha[f] = 0.0; beta[f] = 0.0; return; }
  if (phase == 0) {
    alpha[f] = rr[f] / pq[2 * f];
  } else {
    const double rn = rr_new[2 * f];
    iters[f] += 1;
    if (rn <= tol2 * b2[f]) {
      active[f] = 0;
      beta[f] = 0.0;
    } else {
      beta[f] = rn / rr[f];
    }
    rr[f] = rn;
  }
}

void launch_cg_scalars(hipStream_t s, int nvec, const double* pq, const double* rr_new, double* rr, double* alpha,
                       double* beta, int* active, const double* b2, double tol2, int* iters, int phase) {
  hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(64), 0, s, nvec, pq, rr_new, rr, alpha, beta, active, b2, tol2,
                     iters, phase);
  DMG_LAUNCH_CHECK();
}

// phase 0: x += alpha p, r -= alpha q (fields that were active when alpha was formed)
// phase 1: p = r + beta p (fields still active)
template <typename R>
__global__ void k_cg_update(int64_t n, cx<R>* x, cx<R>* r, cx<R>* p, const cx<R>* q, const double* alpha,
                            const double* beta, const int* active, int phase) {
  const int f = blockIdx.y;
  const int64_t off = (int64_t)f * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (phase == 0) {
    const double a = alpha[f];
    if (a == 0.0) return;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
      const double2 pv = to_d(p[off + e]), qv = to_d(q[off + e]);
      x[off + e] = from_d<R>(cadd(to_d(x[off + e]), cscale(pv, a)));
      r[off + e] = from_d<R>(csub(to_d(r[off + e]), cscale(qv, a)));
    }
  } else {
    if (!active[f]) return;
    const double bt = beta[f];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
      p[off + e] = from_d<R>(cadd(to_d(r[off + e]), cscale(to_d(p[off + e]), bt)));
  }
}

template <typename R>
void launch_cg_update(hipStream_t s, int64_t n, int nvec, cx<R>* x, cx<R>* r, cx<R>* p, const cx<R>* q,
                      const double* alpha, const double* beta, const int* active, int phase) {
  int G = (int)((n + SB - 1) / SB);
  if (G > 256) G = 256;
  hipLaunchKernelGGL(k_cg_update<R>, dim3(G, nvec), dim3(SB), 0, s, n, x, r, p, q, alpha, beta, active, phase);
  DMG_LAUNCH_CHECK();
}
template void launch_cg_update<double>(hipStream_t, int64_t, int, double2*, double2*, double2*, const double2*,
                                       const double*, const double*, const int*, int);
template void launch_cg_update<float>(hipStream_t, int64_t, int, float2*, float2*, float2*, const float2*,
                                      const double*, const double*, const int*, int);

// ---------------------------------------------------------------- local orthonormalisation
// One workgroup (one wavefront) per (block, chirality).  Rows are the block's sites in
// order x_l + 4 t_l, each with the h = dof/2 components of that chirality; columns are
// the nvec (globally orthonormalised) near-null vectors.  Restricting to one chirality's
// components is the chiral doubling (1 +- gamma_5)/2 followed by blocking.  MGS applied
// twice per column in index order; P[s][c h + i][k] receives row (s, i) of column k.
constexpr int LO_MAXROWS = BLK * BLK * NV;  // 192

__global__ void __launch_bounds__(64) k_local_ortho(const double2* __restrict__ vecs, int64_t n, int nvec,
                                                    double2* __restrict__ P, int Lx, int Lt, int dof, int* status) {
  __shared__ double2 W[LO_MAXROWS * NV];
  const int t = threadIdx.x;
  const int B = blockIdx.x >> 1, c = blockIdx.x & 1;
  const int BX = Lx / BLK;
  const int X = B % BX, T = B / BX;
  const int h = dof / 2;
  const int rows = BLK * BLK * h;
  for (int e = t; e < rows * nvec; e += 64) {
    const int row = e % rows, k = e / rows;
    const int sl = row / h, i = row % h;
    const int s = (BLK * X + sl % BLK) + Lx * (BLK * T + sl / BLK);
    W[row + rows * k] = vecs[(int64_t)k * n + (int64_t)s * dof + c * h + i];
  }
  __syncthreads();
  for (int k = 0; k < nvec; ++k) {
    double n0 = 0.0;
    for (int row = t; row < rows; row += 64) n0 += cabs2(W[row + rows * k]);
    n0 = wsum(mk(n0, 0.0)).x;
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < k; ++j) {
        double2 d = mk(0.0, 0.0);
        for (int row = t; row < rows; row += 64) cfmac(d, W[row + rows * j], W[row + rows * k]);
        d = wsum(d);
        for (int row = t; row < rows; row += 64) W[row + rows * k] = csub(W[row + rows * k], cmul(d, W[row + rows * j]));
        __syncthreads();
      }
    }
    double nn = 0.0;
    for (int row = t; row < rows; row += 64) nn += cabs2(W[row + rows * k]);
    nn = wsum(mk(nn, 0.0)).x;
    if (!(nn > 1e-24 * n0) || !(nn > 0.0)) {
      if (t == 0) status[0] = 1;
      nn = 1.0;
    }
    const double inv = 1.0 / sqrt(nn);
    for (int row = t; row < rows; row += 64) W[row + rows * k] = cscale(W[row + rows * k], inv);
    __syncthreads();
  }
  for (int e = t; e < rows * nvec; e += 64) {
    const int row = e / nvec, k = e % nvec;
    const int sl = row / h, i = row % h;
    const int s = (BLK * X + sl % BLK) + Lx * (BLK * T + sl / BLK);
    P[((int64_t)s * dof + c * h + i) * NV + k] = W[row + rows * k];
  }
}

void launch_local_ortho(hipStream_t s, const double2* vecs, int64_t n, int nvec, double2* P, int Lx, int Lt, int dof,
                        int* status) {
  const int nb = (Lx / BLK) * (Lt / BLK);
  hipLaunchKernelGGL(k_local_ortho, dim3(2 * nb), dim3(64), 0, s, vecs, n, nvec, P, Lx, Lt, dof, status);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- Wilson operator as 2 x 2 blocks
// blocks[s][d][col][row], d = 0 self, 1 +x, 2 -x, 3 +t, 4 -t (coupling from s + d into s):
//   self (m0 + 2) I;  +mu: -1/2 (1 - g_mu) U_mu(s);  -mu: -1/2 (1 + g_mu) conj(U_mu(s - mu)).
__global__ void k_wilson_blocks(const double2* __restrict__ U, double m0, int Nx, int Nt, double2* blocks) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= Nx * Nt) return;
  const int x = s % Nx, t = s / Nx;
  const int sxm = ((x == 0) ? Nx - 1 : x - 1) + Nx * t;
  const int stm = x + Nx * ((t == 0) ? Nt - 1 : t - 1);
  double2* b = blocks + (int64_t)s * 5 * 4;
  // gamma matrices, row-major g[mu][row][col]
  const double2 g[2][2][2] = {{{mk(0, 0), mk(1, 0)}, {mk(1, 0), mk(0, 0)}},
                              {{mk(0, 0), mk(0, -1)}, {mk(0, 1), mk(0, 0)}}};
  for (int e = 0; e < 4; ++e) b[e] = mk(0.0, 0.0);
  b[0] = mk(m0 + 2.0, 0.0);
  b[3] = mk(m0 + 2.0, 0.0);
  for (int mu = 0; mu < 2; ++mu) {
    const double2 uf = U[2 * s + mu];
    const double2 ub = cconj(U[2 * (mu == 0 ? sxm : stm) + mu]);
    double2* bf = b + 4 * (1 + 2 * mu);
    double2* bb = b + 4 * (2 + 2 * mu);
    for (int row = 0; row < 2; ++row)
      for (int col = 0; col < 2; ++col) {
        const double2 id = mk(row == col ? 1.0 : 0.0, 0.0);
        const double2 pm = csub(id, g[mu][row][col]);  // 1 - g
        const double2 pp = cadd(id, g[mu][row][col]);  // 1 + g
        bf[col * 2 + row] = cscale(cmul(pm, uf), -0.5);
        bb[col * 2 + row] = cscale(cmul(pp, ub), -0.5);
      }
  }
}

void launch_wilson_blocks(hipStream_t s, const double2* U, double m0, int Nx, int Nt, double2* blocks) {
  const int V = Nx * Nt;
  hipLaunchKernelGGL(k_wilson_blocks, dim3((V + 255) / 256), dim3(256), 0, s, U, m0, Nx, Nt, blocks);
  DMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- Galerkin product
// coarse block d of coarse site B:
//   Ahat_d(B) = sum over fine sites s in B and fine directions d' whose hop s -> s + d' is
//   classified as d (self: diagonal term and hops inside B; +-mu: hops that leave B through
//   its +-mu face) of P(s)^H A_{d'}(s) P(s + d').
// P(s) is the dof x 24 slab of P at site s: entry (a, 12 c + k) = P[s][a][k] when a has
// chirality c, zero otherwise.  One workgroup of 576 threads per (B, d); thread (o, o')
// owns one entry; each term goes through LDS as T = A P(s') then P(s)^H T.
__global__ void __launch_bounds__(NC * NC) k_galerkin(const double2* __restrict__ fineA,
                                                      const double2* __restrict__ P, int Lx, int Lt, int dof,
                                                      double2* __restrict__ coarseA) {
  __shared__ double2 As[NC * NC];
  __shared__ double2 Ps[NC * NV];
  __shared__ double2 Pn[NC * NV];
  __shared__ double2 Ts[NC * NC];
  const int B = blockIdx.x / 5, d = blockIdx.x % 5;
  const int BX = Lx / BLK;
  const int X = B % BX, T = B / BX;
  const int tid = threadIdx.x;
  const int o = tid % NC, op = tid / NC;  // row (c, k) and column (c', k') of the output block
  const int h = dof / 2;
  double2 acc = mk(0.0, 0.0);
  for (int sl = 0; sl < BLK * BLK; ++sl) {
    const int xl = sl % BLK, tl = sl / BLK;
    const int x = BLK * X + xl, t = BLK * T + tl;
    const int s = x + Lx * t;
    for (int dp = 0; dp < 5; ++dp) {
      int cls, sn;
      switch (dp) {
        case 0: cls = 0; sn = s; break;
        case 1: cls = (xl == BLK - 1) ? 1 : 0; sn = ((x + 1 == Lx) ? 0 : x + 1) + Lx * t; break;
        case 2: cls = (xl == 0) ? 2 : 0; sn = ((x == 0) ? Lx - 1 : x - 1) + Lx * t; break;
        case 3: cls = (tl == BLK - 1) ? 3 : 0; sn = x + Lx * ((t + 1 == Lt) ? 0 : t + 1); break;
        default: cls = (tl == 0) ? 4 : 0; sn = x + Lx * ((t == 0) ? Lt - 1 : t - 1); break;
      }
      if (cls != d) continue;
      __syncthreads();
      const double2* a = fineA + ((int64_t)s * 5 + dp) * dof * dof;
      for (int e = tid; e < dof * dof; e += NC * NC) As[e] = a[e];
      for (int e = tid; e < dof * NV; e += NC * NC) {
        Ps[e] = P[(int64_t)s * dof * NV + e];
        Pn[e] = P[(int64_t)sn * dof * NV + e];
      }
      __syncthreads();
      // T[a][o'] = sum_{b in chirality c'} A[a][b] P(s')[b][k'],  o' = 12 c' + k'
      if (tid < dof * NC) {
        const int arow = tid % dof, col = tid / dof;
        const int cp = col / NV, kp = col % NV;
        double2 tv = mk(0.0, 0.0);
        for (int ib = 0; ib < h; ++ib) {
          const int bcol = cp * h + ib;
          cfma(tv, As[bcol * dof + arow], Pn[bcol * NV + kp]);
        }
        Ts[arow + dof * col] = tv;
      }
      __syncthreads();
      // out[o][o'] += sum_{a in chirality c} conj(P(s)[a][k]) T[a][o']
      {
        const int c = o / NV, k = o % NV;
        for (int ia = 0; ia < h; ++ia) {
          const int arow = c * h + ia;
          cfmac(acc, Ps[arow * NV + k], Ts[arow + dof * op]);
        }
      }
    }
  }
  coarseA[(((int64_t)B * 5 + d) * NC + op) * NC + o] = acc;
}

void launch_galerkin(hipStream_t s, const double2* fineA, const double2* P, int Lx, int Lt, int dof, double2* coarseA) {
  const int nb = (Lx / BLK) * (Lt / BLK);
  hipLaunchKernelGGL(k_galerkin, dim3(5 * nb), dim3(NC * NC), 0, s, fineA, P, Lx, Lt, dof, coarseA);
  DMG_LAUNCH_CHECK();
}

}  // namespace dmg
