// Stencil and transfer kernels: the fine Wilson-Dirac operator, the 24 x 24
// block nearest-neighbour operators of the Galerkin levels, and the 4 x 4-block
// restriction / prolongation (Methods section).
#include "kernels.h"

namespace dmg {

// i * z
template <typename T> __device__ inline T cmul_i(T z) { T r; r.x = -z.y; r.y = z.x; return r; }

// One thread per fine site; both spin components.  The projectors (1 -+ g_mu) have
// rank one, so each hop is one complex link multiply on a spin-projected value:
//   (1 - s sigma_1) psi = (psi0 - s psi1) [1, -s]     (1 + s sigma_1) psi = (psi0 + s psi1) [1,  s]
//   (1 - s sigma_2) psi = (psi0 + s i psi1) [1, -s i]  (1 + s sigma_2) psi = (psi0 - s i psi1) [1, s i]
// with s = +1 for D and s = -1 for D^dagger = sigma_3 D sigma_3.
template <typename R>
__global__ void __launch_bounds__(256) k_wilson(const cx<R>* __restrict__ U, const cx<R>* __restrict__ in,
                                                cx<R>* __restrict__ out, R diag, int Nx, int Nt, int dagger,
                                                const int* skip, const cx<R>* __restrict__ sub) {
  if (skip && *skip) return;
  using T = cx<R>;
  const int V = Nx * Nt;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  const int64_t off = (int64_t)blockIdx.y * 2 * V;
  in += off;
  out += off;
  const int x = s % Nx, t = s / Nx;
  const int xp = (x + 1 == Nx) ? 0 : x + 1, xm = (x == 0) ? Nx - 1 : x - 1;
  const int tp = (t + 1 == Nt) ? 0 : t + 1, tm = (t == 0) ? Nt - 1 : t - 1;
  const int sxp = xp + Nx * t, sxm = xm + Nx * t, stp = x + Nx * tp, stm = x + Nx * tm;
  const R sg = dagger ? R(-1) : R(1);
  const R half = R(0.5);

  T a0 = in[2 * s], a1 = in[2 * s + 1];
  T acc0 = cscale(a0, diag), acc1 = cscale(a1, diag);

  {  // forward x
    T p0 = in[2 * sxp], p1 = in[2 * sxp + 1];
    T h = csub(p0, cscale(p1, sg));
    T w = cmul(U[2 * s + 0], h);
    acc0 = csub(acc0, cscale(w, half));
    acc1 = cadd(acc1, cscale(w, half * sg));
  }
  {  // backward x
    T p0 = in[2 * sxm], p1 = in[2 * sxm + 1];
    T h = cadd(p0, cscale(p1, sg));
    T w = cmulc(U[2 * sxm + 0], h);
    acc0 = csub(acc0, cscale(w, half));
    acc1 = csub(acc1, cscale(w, half * sg));
  }
  {  // forward t
    T p0 = in[2 * stp], p1 = in[2 * stp + 1];
    T h = cadd(p0, cscale(cmul_i(p1), sg));
    T w = cmul(U[2 * s + 1], h);
    acc0 = csub(acc0, cscale(w, half));
    acc1 = cadd(acc1, cscale(cmul_i(w), half * sg));
  }
  {  // backward t
    T p0 = in[2 * stm], p1 = in[2 * stm + 1];
    T h = csub(p0, cscale(cmul_i(p1), sg));
    T w = cmulc(U[2 * stm + 1], h);
    acc0 = csub(acc0, cscale(w, half));
    acc1 = csub(acc1, cscale(cmul_i(w), half * sg));
  }
  if (sub) {
    acc0 = csub(sub[off + 2 * s], acc0);
    acc1 = csub(sub[off + 2 * s + 1], acc1);
  }
  out[2 * s] = acc0;
  out[2 * s + 1] = acc1;
}

template <typename R>
void launch_wilson(hipStream_t st, const cx<R>* U, const cx<R>* in, cx<R>* out, double m0, int Nx, int Nt,
                   int dagger, int nrhs, const int* skip, const cx<R>* sub) {
  const int V = Nx * Nt;
  dim3 grid((V + 255) / 256, nrhs);
  hipLaunchKernelGGL(k_wilson<R>, grid, dim3(256), 0, st, U, in, out, (R)(m0 + 2.0), Nx, Nt, dagger, skip, sub);
  DMG_LAUNCH_CHECK();
}

// Blocked operator y(S) = sum_d A_d(S) x(S + d).  Blocks are stored column-major
// ([S][d][col j][row i]) so that the 24 rows of one column are contiguous and the
// 24 threads that own the rows of a site read them in one coalesced sweep.
// Thread (site, d, row) forms one 24-term dot product; the five direction partials
// are summed through LDS.  D^dagger = Gamma_5 D Gamma_5: sign flips on x and y.
constexpr int BA_SITES = 4;  // sites per workgroup: 4 * 5 * 24 = 480 threads

template <typename R, typename B>
__global__ void __launch_bounds__(512) k_block_apply(const B* __restrict__ A, const cx<R>* __restrict__ in,
                                                     cx<R>* __restrict__ out, int Lx, int Lt, int dagger,
                                                     const int* skip, const cx<R>* __restrict__ sub) {
  if (skip && *skip) return;
  using T = cx<R>;
  __shared__ T xs[BA_SITES][5][NC];
  __shared__ T part[BA_SITES][5][NC];
  const int V = Lx * Lt;
  const int tid = threadIdx.x;
  const int ls = tid / (5 * NC);           // local site
  const int d = (tid / NC) % 5;            // direction
  const int i = tid % NC;                  // row
  const int S = blockIdx.x * BA_SITES + ls;
  const bool active = (ls < BA_SITES) && (S < V);
  int nb = 0;
  if (active) {
    const int X = S % Lx, Tt = S / Lx;
    switch (d) {
      case 0: nb = S; break;
      case 1: nb = ((X + 1 == Lx) ? 0 : X + 1) + Lx * Tt; break;
      case 2: nb = ((X == 0) ? Lx - 1 : X - 1) + Lx * Tt; break;
      case 3: nb = X + Lx * ((Tt + 1 == Lt) ? 0 : Tt + 1); break;
      default: nb = X + Lx * ((Tt == 0) ? Lt - 1 : Tt - 1); break;
    }
    T v = in[(int64_t)nb * NC + i];
    if (dagger && i >= NV) { v.x = -v.x; v.y = -v.y; }
    xs[ls][d][i] = v;
  }
  __syncthreads();
  if (active) {
    const auto* a = A + ((int64_t)S * 5 + d) * NC * NC + i;
    // all 24 block loads in flight at once; two accumulators halve the dependent chain
    T acc = make_cx<R>(R(0), R(0)), acc2 = make_cx<R>(R(0), R(0));
#pragma unroll
    for (int j = 0; j < NC; j += 2) {
      cfma(acc, ld_blk(a + j * NC), xs[ls][d][j]);
      cfma(acc2, ld_blk(a + (j + 1) * NC), xs[ls][d][j + 1]);
    }
    part[ls][d][i] = cadd(acc, acc2);
  }
  __syncthreads();
  if (active && d == 0) {
    T y = part[ls][0][i];
    y = cadd(y, part[ls][1][i]);
    y = cadd(y, part[ls][2][i]);
    y = cadd(y, part[ls][3][i]);
    y = cadd(y, part[ls][4][i]);
    if (dagger && i >= NV) { y.x = -y.x; y.y = -y.y; }
    if (sub) y = csub(sub[(int64_t)S * NC + i], y);
    out[(int64_t)S * NC + i] = y;
  }
}

template <typename R>
void launch_block_apply(hipStream_t st, const cx<R>* A, const cx<R>* in, cx<R>* out, int Lx, int Lt, int dagger,
                        const int* skip, const cx<R>* sub) {
  const int V = Lx * Lt;
  hipLaunchKernelGGL((k_block_apply<R, cx<R>>), dim3((V + BA_SITES - 1) / BA_SITES), dim3(BA_SITES * 5 * NC), 0, st,
                     A, in, out, Lx, Lt, dagger, skip, sub);
  DMG_LAUNCH_CHECK();
}

void launch_block_apply_bf16(hipStream_t st, const bf16c* A, const float2* in, float2* out, int Lx, int Lt,
                             int dagger, const int* skip, const float2* sub) {
  const int V = Lx * Lt;
  hipLaunchKernelGGL((k_block_apply<float, bf16c>), dim3((V + BA_SITES - 1) / BA_SITES), dim3(BA_SITES * 5 * NC), 0,
                     st, A, in, out, Lx, Lt, dagger, skip, sub);
  DMG_LAUNCH_CHECK();
}

// BF16 copy of FP64 blocks: each part rounded to FP32, then to bfloat16 (nearest, ties to even)
__global__ void k_d2bf16(int64_t n, const double2* __restrict__ x, bf16c* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto rnd = [](double v) {
    const unsigned u = __float_as_uint((float)v);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  };
  const double2 v = x[i];
  bf16c o;
  o.re = rnd(v.x);
  o.im = rnd(v.y);
  y[i] = o;
}

void launch_d2bf16(hipStream_t st, int64_t n, const double2* x, bf16c* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_d2bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, y);
  DMG_LAUNCH_CHECK();
}

// The same rounding to bfloat16, the result held as FP32 (the low 16 bits zero)
__global__ void k_d2bf16f(int64_t n, const double2* __restrict__ x, float2* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto rnd = [](double v) {
    const unsigned u = __float_as_uint((float)v);
    return __uint_as_float(((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16) << 16);
  };
  const double2 v = x[i];
  y[i] = make_float2(rnd(v.x), rnd(v.y));
}

void launch_d2bf16f(hipStream_t st, int64_t n, const double2* x, float2* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_d2bf16f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, y);
  DMG_LAUNCH_CHECK();
}

// Restriction: coarse(B, 12 c + k) = sum_{s in B} sum_{i < h} conj(P[s][c h + i][k]) fine[s][c h + i],
// h = dof / 2.  One workgroup per block; thread (g, o) sums the terms q = g, g + G, ... of
// output o, then the G partials are added through LDS in a fixed order.
constexpr int RG = 8;

template <typename R>
__global__ void __launch_bounds__(NC * RG) k_restrict(const cx<R>* __restrict__ P, const cx<R>* __restrict__ fine,
                                                      cx<R>* __restrict__ coarse, int Lx, int Lt, int dof) {
  using T = cx<R>;
  __shared__ double2 part[RG][NC];
  const int B = blockIdx.x;
  const int BX = Lx / BLK;
  const int X = B % BX, Tb = B / BX;
  const int o = threadIdx.x % NC, g = threadIdx.x / NC;
  const int c = o / NV, k = o % NV;
  const int h = dof / 2;
  const int nterms = BLK * BLK * h;
  double2 acc = make_double2(0.0, 0.0);
  for (int q = g; q < nterms; q += RG) {
    const int sl = q / h, ii = q % h;
    const int s = (BLK * X + sl % BLK) + Lx * (BLK * Tb + sl / BLK);
    const int a = c * h + ii;
    const T p = P[((int64_t)s * dof + a) * NV + k];
    const T v = fine[(int64_t)s * dof + a];
    cfmac(acc, to_d(p), to_d(v));
  }
  part[g][o] = acc;
  __syncthreads();
  if (g == 0) {
    double2 r = part[0][o];
    for (int q = 1; q < RG; ++q) r = cadd(r, part[q][o]);
    coarse[(int64_t)B * NC + o] = from_d<R>(r);
  }
}

template <typename R>
void launch_restrict(hipStream_t st, const cx<R>* P, const cx<R>* fine, cx<R>* coarse, int Lx, int Lt, int dof) {
  const int nb = (Lx / BLK) * (Lt / BLK);
  hipLaunchKernelGGL(k_restrict<R>, dim3(nb), dim3(NC * RG), 0, st, P, fine, coarse, Lx, Lt, dof);
  DMG_LAUNCH_CHECK();
}

// Prolongation: fine[s][a] (+)= sum_k P[s][a][k] coarse(B(s), 12 c(a) + k).  One thread per
// fine component.
template <typename R>
__global__ void __launch_bounds__(256) k_prolong(const cx<R>* __restrict__ P, const cx<R>* __restrict__ coarse,
                                                 cx<R>* __restrict__ fine, int Lx, int Lt, int dof, int accumulate) {
  using T = cx<R>;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)Lx * Lt * dof;
  if (e >= n) return;
  const int s = (int)(e / dof), a = (int)(e % dof);
  const int x = s % Lx, t = s / Lx;
  const int B = x / BLK + (Lx / BLK) * (t / BLK);
  const int c = a / (dof / 2);
  const T* p = P + e * NV;
  const T* cv = coarse + (int64_t)B * NC + c * NV;
  double2 acc = accumulate ? to_d(fine[e]) : make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < NV; ++k) cfma(acc, to_d(p[k]), to_d(cv[k]));
  fine[e] = from_d<R>(acc);
}

template <typename R>
void launch_prolong(hipStream_t st, const cx<R>* P, const cx<R>* coarse, cx<R>* fine, int Lx, int Lt, int dof,
                    int accumulate) {
  const int64_t n = (int64_t)Lx * Lt * dof;
  hipLaunchKernelGGL(k_prolong<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, coarse, fine, Lx, Lt,
                     dof, accumulate);
  DMG_LAUNCH_CHECK();
}

#define INST(R)                                                                                                   \
  template void launch_wilson<R>(hipStream_t, const cx<R>*, const cx<R>*, cx<R>*, double, int, int, int, int,     \
                                 const int*, const cx<R>*);                                                       \
  template void launch_block_apply<R>(hipStream_t, const cx<R>*, const cx<R>*, cx<R>*, int, int, int, const int*,  \
                                      const cx<R>*);                                                              \
  template void launch_restrict<R>(hipStream_t, const cx<R>*, const cx<R>*, cx<R>*, int, int, int);               \
  template void launch_prolong<R>(hipStream_t, const cx<R>*, const cx<R>*, cx<R>*, int, int, int, int);
INST(double)
INST(float)
#undef INST

}  // namespace dmg
