// Persistent coarse-grid GMRES-Proj(m, k) (Methods section: every coarse solve after
// the first is a projection over the GMRES-DR space followed by GMRES cycles).
//
// One launch runs a whole coarse solve.  About 64 workgroups each own
// `spw` consecutive coarse sites; a workgroup keeps its slices of the Krylov basis,
// of the deflation basis and of x and r in LDS for the whole solve (and its 24 x 24
// blocks too when they fit).  Neighbour values for the stencil travel through one
// global exchange vector; dot products are summed per workgroup, written to
// global memory, and after a grid barrier every workgroup adds the same partials
// in the same order, so all workgroups hold identical small-dense state and take
// identical control decisions without further communication.
//
// The grid barrier is a flag array: each workgroup publishes its barrier
// generation with one store and its first wavefront polls all flags (bounded
// spin).  The exchanged data itself is stored and loaded with device-scope atomic
// accesses, and every wavefront waits for its stores before the workgroup barrier
// that precedes the flag store, so the flags need no cache write-back or
// invalidation.  Its cost grows slowly with the number of
// workgroups, unlike a single atomic counter whose arrivals serialise; hence few,
// larger workgroups.  In the two-barrier form an Arnoldi step exchanges v_j for the
// stencil and then reduces the Gram-Schmidt dots; the halo form (k_coarse_proj's HALO)
// keeps the basis on each workgroup's halo sites as well and needs only the reduction
// barrier, and its 512-thread variant (REG) keeps the blocks in registers.  The
// orthogonalisation is classical Gram-Schmidt with the norm from ||w||^2 - ||h||^2; when
// that difference shows more than 99.99 % cancellation a second pass with an exact norm
// is taken (one more barrier).  The Givens rotations of each new Hessenberg column come
// from a lane scan (cp_rotation_scan), and each cycle's least-squares solve and residual
// coordinates run on one wavefront.  In exact arithmetic this is the Arnoldi process of
// GMRES; the oracle uses modified Gram-Schmidt twice.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "kernels.h"

namespace dmg {

constexpr int CP_THREADS = 1024;  // 16 wavefronts: enough loads in flight to stream the blocks
constexpr int CP_QMAX = 32;     // quantities per reduction

struct CPArgs {
  const void* A;          // coarse blocks [S][d][col][row]
  int Lx, Lt;
  const void* DV;         // deflation basis, k + 1 fields
  const double2* DM;      // Hbar_k^+, k x (k+1) column-major
  const double2* DP;      // Hbar_k Hbar_k^+, (k+1) x (k+1) column-major
  int k;
  const void* b;
  void* x;
  double tol;
  int mm;                 // GMRES cycle length m - k
  int max_iters;
  void* xchg;             // exchange field (n entries)
  double2* partials;      // 2 x CP_QMAX x G
  int* out_iters;
  double* out_relres;
  unsigned* flags;        // G barrier flags, CP_FLAGPAD apart, zero at launch
  int* err;               // set when a barrier wait exceeds its spin limit
  int spw;                // sites per workgroup
  int a_in_lds;
  int nl;                 // halo form: bound on own + halo sites of any workgroup (else spw)
};

constexpr int CP_FLAGPAD = 32;  // one flag per 128-byte line

// Data exchanged between workgroups inside one launch (the stencil exchange field and
// the per-workgroup partial sums) is written and read with device-scope atomic
// accesses, which go to the device's coherence point rather than a compute die's own
// L2.  A wavefront then only has to wait for its own stores to complete before the
// barrier; no cache write-back is needed.
__device__ inline void cp_store(double2* p, double2 v) {
  __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void cp_store(float2* p, float2 v) {
  unsigned long long u;
  __builtin_memcpy(&u, &v, sizeof(u));
  __hip_atomic_store((unsigned long long*)p, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double2 cp_load(const double2* p) {
  return mk(__hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
            __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ inline float2 cp_load(const float2* p) {
  const unsigned long long u =
      __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  float2 v;
  __builtin_memcpy(&v, &u, sizeof(v));
  return v;
}
// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima): this wavefront's
// outstanding vector-memory operations have completed.
__device__ inline void cp_wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Flag-array grid barrier (see the file comment).  `gen` counts this workgroup's
// barriers; a wait longer than the spin limit sets *err and gives up, so no wave
// can hang the device.
// Returns true when the grid must stop: some wait (here or in another workgroup) ran
// past its spin limit.  A workgroup that stops publishes no more flags, so a wait for one
// of its flags finds *err set (it is read every 64 spins) and stops too, and the callers
// leave their loops: the whole grid drains quickly.  *err is not read on the fast path,
// where its round trip would delay the flag store or the first poll.
// Every wavefront waits for its own exchange stores before the workgroup barrier: a
// wavefront's wait covers only its own outstanding stores, so the flag store of
// wavefront 0 alone would not order the other wavefronts' stores before it.
struct CpNoHook {
  __device__ void operator()() const {}
};
// `during` runs on the workgroup's last wavefront after the flag store, while wavefront 0 waits
// for the other workgroups' flags (work that does not feed this reduction).
template <typename Hook = CpNoHook>
__device__ inline bool cp_barrier(unsigned* flags, int G, unsigned gen, int* err, Hook during = Hook()) {
  __shared__ int aborted;
  cp_wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    // relaxed: every datum the flag publishes was stored with a device-scope atomic
    // that completed before the workgroup barrier above
    __hip_atomic_store(&flags[blockIdx.x * CP_FLAGPAD], gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    aborted = 0;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    bool stop = false, timed_out = false;
    for (int b = threadIdx.x; b < G && !stop; b += 64) {
      long spins = 0;
      // relaxed: the published data is read with device-scope atomics after this wait,
      // so no cache invalidation is needed (it would also evict the operator's blocks)
      while (__hip_atomic_load(&flags[b * CP_FLAGPAD], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
        __builtin_amdgcn_s_sleep(1);
        ++spins;
        if ((spins & 63) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          stop = true;  // some workgroup gave up: its flag may never come
          break;
        }
        if (spins > (1L << 22)) {
          stop = timed_out = true;
          break;
        }
      }
    }
    if (timed_out) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (stop) aborted = 1;
  }
  if (threadIdx.x >= blockDim.x - 64) during();
  __syncthreads();
  return aborted != 0;
}

__host__ __device__ inline size_t cp_align(size_t v) { return (v + 15) & ~(size_t)15; }

// Site reached from S in stencil direction d (0: S itself, 1/2: x +/- 1, 3/4: t +/- 1), periodic.
__host__ __device__ inline int cp_nbr(int S, int d, int Lx, int Lt) {
  const int X = S % Lx, Tt = S / Lx;
  switch (d) {
    case 0: return S;
    case 1: return ((X + 1 == Lx) ? 0 : X + 1) + Lx * Tt;
    case 2: return ((X == 0) ? Lx - 1 : X - 1) + Lx * Tt;
    case 3: return X + Lx * ((Tt + 1 == Lt) ? 0 : Tt + 1);
    default: return X + Lx * ((Tt == 0) ? Lt - 1 : Tt - 1);
  }
}

// Halo of the workgroup owning sites S0 .. S0 + nsl - 1: the other sites its stencil reads,
// numbered in first-use order (own site sl, direction d ascending).  loc[sl * 5 + d] receives
// the local index of the site read (own sites 0 .. nsl - 1, halo slots after them); hs the
// halo sites.  Returns the halo size.  The host uses the same routine to size the LDS.
__host__ __device__ inline int cp_halo(int S0, int nsl, int Lx, int Lt, int* loc, int* hs) {
  int nh = 0;
  for (int sl = 0; sl < nsl; ++sl)
    for (int d = 0; d < 5; ++d) {
      const int nb = cp_nbr(S0 + sl, d, Lx, Lt);
      int li;
      if (nb >= S0 && nb < S0 + nsl) {
        li = nb - S0;
      } else {
        int h = 0;
        while (h < nh && hs[h] != nb) ++h;
        if (h == nh) hs[nh++] = nb;
        li = nsl + h;
      }
      if (loc) loc[sl * 5 + d] = li;
    }
  return nh;
}

// LDS layout (bytes) shared by host sizing and the kernel.
// halo form (nl > 0): the basis vectors and w hold own + halo entries (nl sites), and there
// is no exchange staging area.
struct CPLayout {
  size_t A, Vb, DVb, xl, rl, wl, xs, part, Hr, rc, rs, g, y, u, Hk, Rk, kc, ks, kp, red, cs, res, loc, hs, tot;
  __host__ __device__ CPLayout(int spw, int mm, int k, size_t es, int a_in_lds, int nl = 0) {
    const size_t ne = (size_t)spw * NC;
    const size_t nle = (size_t)(nl > 0 ? nl : spw) * NC;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = cp_align(o + bytes); return at; };
    A = take(a_in_lds ? (size_t)spw * 5 * NC * NC * es : 0);
    Vb = take((size_t)(mm + 1) * nle * es);
    DVb = take((size_t)(k + 1) * ne * es);
    xl = take(ne * es);
    rl = take(ne * es);
    wl = take(nle * es);
    xs = take(nl > 0 ? 0 : (size_t)spw * 5 * NC * es);
    part = take((size_t)spw * 5 * NC * sizeof(double2));
    loc = take((size_t)spw * 5 * sizeof(int));
    hs = take((size_t)spw * 4 * sizeof(int));
    Hr = take((size_t)(mm + 1) * mm * sizeof(double2));
    rc = take((size_t)mm * sizeof(double));
    rs = take((size_t)mm * sizeof(double2));
    const size_t sv = (size_t)((mm > k ? mm : k) + 1) * sizeof(double2);  // also holds projection vectors
    g = take(sv);
    y = take(sv);
    u = take(sv);
    Hk = take((size_t)(k + 1) * k * sizeof(double2));        // M
    Rk = take((size_t)(k + 1) * (k + 1) * sizeof(double2));  // Pi
    kc = ks = kp = 0;
    red = take((size_t)CP_QMAX * sizeof(double2));
    cs = part;  // chunk sums reuse the stencil partials (never live at the same time)
    res = take((size_t)(CP_QMAX + 2) * sizeof(double2));
    tot = o;
  }
};

__device__ inline double2 cp_wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// Cross-lane moves without the LDS: a DPP lane permutation (quad_perm / row_ror control) and a
// read of one lane into a scalar register, on the two 32-bit halves of a double.
template <int CTRL>
__device__ inline double cp_dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// DPP move whose lanes without a source (row_shr past the row start) keep `keep`
template <int CTRL>
__device__ inline double cp_dpp_or(double v, double keep) {
  const long long b = __double_as_longlong(v), k = __double_as_longlong(keep);
  const int lo = __builtin_amdgcn_update_dpp((int)(k & 0xffffffff), (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(k >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double cp_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double2 cp_lane(double2 v, int l) { return mk(cp_lane(v.x, l), cp_lane(v.y, l)); }

// Sum over each 16-lane row (neighbour swaps within quads, then rotations by 4 and 8); lanes
// 0, 16, 32 and 48 hold their rows' sums, always added in the same order.
__device__ inline double cp_row_sum(double v) {
  v += cp_dpp<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += cp_dpp<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += cp_dpp<0x124>(v);  // row_ror 4
  v += cp_dpp<0x128>(v);  // row_ror 8
  return v;
}
// Sum over the 32 lanes of each half-wavefront; every lane of a half gets its half's total
// (rows 0 + 1, rows 2 + 3), the same bits in every workgroup.  Both rows of an active half
// must be active.
__device__ inline double2 cp_half_sum(double2 v) {
  v.x = cp_row_sum(v.x);
  v.y = cp_row_sum(v.y);
  const double2 lo = cadd(cp_lane(v, 0), cp_lane(v, 16));
  const double2 hi = cadd(cp_lane(v, 32), cp_lane(v, 48));
  return (threadIdx.x & 32) ? hi : lo;
}

constexpr int CP_GMAX = 128;  // workgroups of one persistent launch (at most one per compute unit)

// Sum of the G published per-workgroup partials of one quantity by the 32 lanes of a
// half-wavefront: lane c loads partials c, c + 32, ... (all loads issued before the first
// add, so the device-scope latency is paid once), adds them in that order, then the
// half-wavefront tree.  Every workgroup adds the same values in the same order.
__device__ inline double2 cp_gather_sum(const double2* P, int G, int c) {
  double2 v[CP_GMAX / 32];
#pragma unroll
  for (int u = 0; u < CP_GMAX / 32; ++u) {
    const int b = c + 32 * u;
    v[u] = b < G ? cp_load(&P[b]) : mk(0.0, 0.0);
  }
  double2 sm = v[0];
#pragma unroll
  for (int u = 1; u < CP_GMAX / 32; ++u) sm = cadd(sm, v[u]);
  return cp_half_sum(sm);
}

// cp_gather_sum for two quantities at once (loads of both issued before any add).
__device__ inline void cp_gather_sum2(const double2* P0, const double2* P1, int G, int c, double2& s0, double2& s1) {
  double2 v[CP_GMAX / 32], w[CP_GMAX / 32];
#pragma unroll
  for (int u = 0; u < CP_GMAX / 32; ++u) {
    const int b = c + 32 * u;
    v[u] = b < G ? cp_load(&P0[b]) : mk(0.0, 0.0);
    w[u] = b < G ? cp_load(&P1[b]) : mk(0.0, 0.0);
  }
  double2 a0 = v[0], a1 = w[0];
#pragma unroll
  for (int u = 1; u < CP_GMAX / 32; ++u) {
    a0 = cadd(a0, v[u]);
    a1 = cadd(a1, w[u]);
  }
  s0 = cp_half_sum(a0);
  s1 = cp_half_sum(a1);
}

// A chain of Givens rotations applied to one Hessenberg column by a wavefront.  Rotation l
// (lane l < cnt, coefficients cl, sl) maps the carried entry x_l and the column entry
// h_{l+1} (hnext) to out_l = c_l x_l + s_l h_{l+1} and x_{l+1} = c_l h_{l+1} - conj(s_l) x_l,
// an affine map of x_l.  The composed maps come from an inclusive scan over lanes (rows of 16
// by DPP shifts, then the second row composed with lane 15's), so the chain takes log2 steps
// instead of cnt.  Returns x_l (the carry entering rotation l; x_0 = h0) in each lane and the
// carry after all cnt rotations.  cnt <= 31; all lanes active.
__device__ inline double2 cp_rotation_scan(int lane, int cnt, double2 h0, double cl, double2 sl, double2 hnext,
                                           double2& xlast) {
  const bool live = lane < cnt;
  double2 A = live ? mk(-sl.x, sl.y) : mk(1.0, 0.0);  // -conj(s)
  double2 Bv = live ? cscale(hnext, cl) : mk(0.0, 0.0);
  auto step = [&](auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    const double2 Ap = mk(cp_dpp_or<C>(A.x, 1.0), cp_dpp_or<C>(A.y, 0.0));
    const double2 Bp = mk(cp_dpp_or<C>(Bv.x, 0.0), cp_dpp_or<C>(Bv.y, 0.0));
    Bv = cadd(cmul(A, Bp), Bv);
    A = cmul(A, Ap);
  };
  step(std::integral_constant<int, 0x111>{});  // row_shr 1
  step(std::integral_constant<int, 0x112>{});  // row_shr 2
  step(std::integral_constant<int, 0x114>{});  // row_shr 4
  step(std::integral_constant<int, 0x118>{});  // row_shr 8
  {
    const double2 A15 = cp_lane(A, 15), B15 = cp_lane(Bv, 15);
    if (lane >= 16) {
      Bv = cadd(cmul(A, B15), Bv);
      A = cmul(A, A15);
    }
  }
  const double2 xn = cadd(cmul(A, h0), Bv);  // x_{lane+1}
  double2 xq = mk(cp_dpp_or<0x111>(xn.x, h0.x), cp_dpp_or<0x111>(xn.y, h0.y));
  const double2 x16 = cp_lane(xn, 15);
  if (lane == 16) xq = x16;
  xlast = cnt > 0 ? cp_lane(xn, cnt - 1) : h0;
  return xq;
}

// Givens rotation [c s; -conj(s) c] with c real and [c s; -conj(s) c] [a; b] = [r; 0]:
// c = |a| / r, s = conj(b) a / (|a| r), r = sqrt(|a|^2 + |b|^2), both from the one reciprocal
// square root of |a|^2 r^2 (rsqrt, within an ulp or two; two roots and a division only where
// that product would leave the double range).  It sits on the serial path of every Arnoldi
// step, where square roots and divisions are long dependent instruction chains.
__device__ inline void cp_givens(double2 a, double2 b, double& c, double2& s) {
  const double na2 = cabs2(a), nb2 = cabs2(b);
  if (nb2 == 0.0) { c = 1.0; s = mk(0.0, 0.0); return; }
  if (na2 == 0.0) { c = 0.0; s = cscale(cconj(b), rsqrt(nb2)); return; }
  const double h2 = na2 + nb2, pr = na2 * h2;
  const double inv = (pr > 1e-290 && pr < 1e290) ? rsqrt(pr) : 1.0 / (sqrt(na2) * sqrt(h2));
  c = na2 * inv;
  s = cscale(cmul(cconj(b), a), inv);
}
__device__ inline double2 cp_div(double2 a, double2 b) {
  const double d = cabs2(b);
  return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// HALO: one grid barrier per Arnoldi step instead of two.  Each workgroup also keeps the
// basis vectors on its halo sites: w is published with the Gram-Schmidt partials (the
// exchange field alternates between two halves by step), and after that barrier every
// workgroup applies the same Gram-Schmidt update to its own and its halo entries, so the
// next stencil needs no exchange.  The halo values are bitwise the owners' (same inputs,
// same operations in the same loop).
// REG (halo form, at most 4 sites per workgroup): 512 threads, and thread t < 5 * 24 * spw keeps
// 24 entries of the 24 x 24 blocks in registers for the whole solve (96 VGPRs in FP64), so the
// stencil reads only v_j (LDS) instead of streaming the blocks from L2 every step.  Thread t
// serves block t / 24 (site-major, directions 0 .. 4): with u = t % 24 it holds rows u / 2 and
// u / 2 + 12 over the column half u % 2, so it reads only half of v_j's 24 entries (the LDS
// bandwidth bounds this phase: every thread of a block reads the same values), and the two
// threads of a pair (adjacent lanes) exchange one half-row sum by DPP.
template <typename R, bool ALDS, bool HALO, bool REG = false>
__global__ void __launch_bounds__(REG ? 512 : CP_THREADS) k_coarse_proj(CPArgs a) {
  static_assert(!REG || (HALO && !ALDS), "register blocks come with the halo form");
  constexpr int TPB = REG ? 512 : CP_THREADS;  // threads per workgroup
  constexpr int NHW = TPB / 32;                // half-wavefronts
  using T = cx<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned gen = 0;
  bool dead = false;  // a barrier wait timed out: stop everything
  const int G = gridDim.x, gi = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int V = a.Lx * a.Lt;
  const int S0 = gi * a.spw;
  const int nsl = min(a.spw, V - S0);
  const int ne = nsl * NC;
  const int mm = a.mm, k = a.k;
  const CPLayout L(a.spw, mm, k, sizeof(T), ALDS ? 1 : 0, HALO ? a.nl : 0);
  T* Ab = (T*)(smem + L.A);
  T* Vb = (T*)(smem + L.Vb);
  T* DVb = (T*)(smem + L.DVb);
  T* xl = (T*)(smem + L.xl);
  T* rl = (T*)(smem + L.rl);
  T* wl = (T*)(smem + L.wl);
  T* xs = (T*)(smem + L.xs);
  double2* part = (double2*)(smem + L.part);
  double2* Hr = (double2*)(smem + L.Hr);
  double* rc = (double*)(smem + L.rc);
  double2* rs = (double2*)(smem + L.rs);
  double2* gv = (double2*)(smem + L.g);
  double2* yv = (double2*)(smem + L.y);
  double2* uv = (double2*)(smem + L.u);
  double2* Mk = (double2*)(smem + L.Hk);
  double2* Pk = (double2*)(smem + L.Rk);
  double2* res = (double2*)(smem + L.res);
  int* loc = (int*)(smem + L.loc);
  int* hsite = (int*)(smem + L.hs);
  __shared__ double sh_scal[8];
  __shared__ int sh_flag[4];
  __shared__ double2 pg_hnext[64], pg_h0;  // a deferred Givens update's column (lane l: h_{l+1})
  __shared__ double pg_hn;
  __shared__ int pg_j;

  const T* Ag = (const T*)a.A;
  const T* DVg = (const T*)a.DV;
  const T* bg = (const T*)a.b;
  T* xg = (T*)a.x;
  T* xch = (T*)a.xchg;
  const int64_t n = (int64_t)V * NC;
  const int64_t e0 = (int64_t)S0 * NC;
  int rbuf = 0;
  // halo form: local sites (own, then halo) and the stride of the basis in LDS
  if (HALO && tid == 0) sh_flag[0] = cp_halo(S0, nsl, a.Lx, a.Lt, loc, hsite);
  __syncthreads();
  const int nh = HALO ? sh_flag[0] : 0;
  const int nle = (nsl + nh) * NC;  // entries of a basis vector in LDS
  const int vst = HALO ? a.nl * NC : ne;
  if (HALO && nsl + nh > a.nl) {
    // cannot happen (the host sized nl with the same routine); stop without touching LDS
    __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    dead = true;
  }
  // halo entries of exchange half `half` into wl[ne ..], right after a barrier: thread
  // TPB - 1 - t loads entry t (at most one per thread for every supported halo; the loop
  // covers the rest) and issues that load before the reduction's gather loads, so that both
  // device-scope round trips are in flight together
  auto halo_load1 = [&](int half, T& hv) {
    const int t = TPB - 1 - tid;
    if (t < nh * NC) hv = cp_load(&xch[(size_t)half * n + (int64_t)hsite[t / NC] * NC + t % NC]);
  };
  auto halo_store = [&](int half, const T& hv) {
    const T* src = xch + (size_t)half * n;
    int t = TPB - 1 - tid;
    if (t < nh * NC) wl[ne + t] = hv;
    for (t += TPB; t < nh * NC; t += TPB) wl[ne + t] = cp_load(&src[(int64_t)hsite[t / NC] * NC + t % NC]);
  };

  // ---------------------------------------------------------------- reduction helpers
  // wg_sums: per-workgroup sums of nq quantities, term(q, e) over the local entries e; the QL
  // lanes of group q (a 16-lane row with 512 threads, a half-wavefront with 1024, so all
  // CP_QMAX quantities are summed in one pass) add every QL-th entry, then a fixed DPP tree
  // (lane 0 of the group publishes the sum straight to this workgroup's slot of quantity q).
  // grid_reduce: barrier, then every workgroup adds all workgroups' sums in the same order into
  // res[q] (half-wavefront q mod NHW gathers one or two quantities).
  constexpr int QL = REG ? 16 : 32;
  static_assert(CP_QMAX * QL == TPB, "one lane group per summed quantity");
  auto group_sum = [](double2 v) {
    if constexpr (QL == 16) return mk(cp_row_sum(v.x), cp_row_sum(v.y));
    else return cp_half_sum(v);
  };
  auto publish = [&](int q, double2 v) { cp_store(&a.partials[((size_t)rbuf * CP_QMAX + q) * G + gi], v); };
  auto wg_sums = [&](int nq, auto&& term) {
    const int q = tid / QL, c = tid % QL;
    if (q < nq) {
      double2 sm = mk(0.0, 0.0);
      for (int e = c; e < ne; e += QL) sm = cadd(sm, term(q, e));
      sm = group_sum(sm);
      if (c == 0) publish(q, sm);
    }
  };
  // the barrier's own wait and workgroup barrier order every wavefront's published sums (and
  // exchange stores) before the flag store
  auto grid_reduce_h = [&](int nq, int halo_half, auto during) {
    double2* P = a.partials + (size_t)rbuf * CP_QMAX * G;
    dead = dead || cp_barrier(a.flags, G, ++gen, a.err, during);
    T hv = make_cx<R>(R(0), R(0));
    if (HALO && halo_half >= 0) halo_load1(halo_half, hv);
    const int q = tid >> 5, c = tid & 31;
    if (NHW < CP_QMAX && q + NHW < nq) {
      // two quantities per half-wavefront, all loads in flight together
      double2 s0, s1;
      cp_gather_sum2(P + (size_t)q * G, P + (size_t)(q + NHW) * G, G, c, s0, s1);
      if (c == 0) {
        res[q] = s0;
        res[q + NHW] = s1;
      }
    } else if (q < nq) {
      const double2 sm = cp_gather_sum(P + (size_t)q * G, G, c);
      if (c == 0) res[q] = sm;
    }
    if (HALO && halo_half >= 0) halo_store(halo_half, hv);
    __syncthreads();
    rbuf ^= 1;
  };
  auto grid_reduce = [&](int nq, int halo_half = -1) { grid_reduce_h(nq, halo_half, CpNoHook()); };
  auto sq = [&](const T* v) { return [=](int, int e) { return mk(cabs2(to_d(v[e])), 0.0); }; };

  // ---------------------------------------------------------------- load the resident data
  T areg[REG ? NC : 1];
  if constexpr (REG) {
    if (tid < nsl * 5 * NC) {
      const int u = tid % NC, r = u >> 1, c0 = (u & 1) * (NC / 2);
      const T* blk = Ag + ((int64_t)S0 * 5 + tid / NC) * NC * NC;  // block (site, direction) of t / 24
#pragma unroll
      for (int c = 0; c < NC / 2; ++c) {
        areg[c] = blk[(c0 + c) * NC + r];
        areg[NC / 2 + c] = blk[(c0 + c) * NC + r + NC / 2];
      }
    }
  }
  if (ALDS) {
    const T* src = Ag + (int64_t)S0 * 5 * NC * NC;
    for (int t = tid; t < nsl * 5 * NC * NC; t += TPB) Ab[t] = src[t];
  }
  for (int t = tid; t < (k + 1) * ne; t += TPB) {
    const int i = t / ne, e = t % ne;
    DVb[t] = DVg[(int64_t)i * n + e0 + e];
  }
  for (int t = tid; t < ne; t += TPB) {
    rl[t] = bg[e0 + t];
    xl[t] = make_cx<R>(R(0), R(0));
  }
  for (int t = tid; t < (k + 1) * k; t += TPB) Mk[t] = a.DM[t];
  for (int t = tid; t < (k + 1) * (k + 1); t += TPB) Pk[t] = a.DP[t];
  __syncthreads();
  // ||b||
  wg_sums(1, sq(rl));
  grid_reduce(1);
  const double bnorm = sqrt(res[0].x);
  const double tol_abs = a.tol * bnorm;
  int iters = 0;
  bool converged = bnorm == 0.0;
  double est = bnorm;

  while (!converged && !dead && iters < a.max_iters) {
    // ------------------------------------------------------------ projection over V_{k+1}
    wg_sums(k + 1, [&](int q, int e) {
      double2 v = mk(0.0, 0.0);
      cfmac(v, to_d(DVb[q * ne + e]), to_d(rl[e]));
      return v;
    });
    grid_reduce(k + 1);
    // d = M c minimises || c - Hbar_k d ||; u = Pi c = Hbar_k d
    if (tid < k) {
      double2 acc = mk(0.0, 0.0);
      for (int l = 0; l <= k; ++l) cfma(acc, Mk[tid + k * l], res[l]);
      yv[tid] = acc;
    } else if (tid >= 64 && tid <= 64 + k) {
      const int i = tid - 64;
      double2 acc = mk(0.0, 0.0);
      for (int l = 0; l <= k; ++l) cfma(acc, Pk[i + (k + 1) * l], res[l]);
      uv[i] = acc;
    }
    __syncthreads();
    for (int t = tid; t < ne; t += TPB) {
      double2 xv = to_d(xl[t]), rv = to_d(rl[t]);
      for (int i = 0; i < k; ++i) cfma(xv, yv[i], to_d(DVb[i * ne + t]));
      for (int i = 0; i <= k; ++i) rv = csub(rv, cmul(uv[i], to_d(DVb[i * ne + t])));
      xl[t] = from_d<R>(xv);
      rl[t] = from_d<R>(rv);
      cp_store(&xch[e0 + t], from_d<R>(rv));
    }
    // ------------------------------------------------------------ GMRES(mm) cycle from r
    __syncthreads();
    if (HALO)
      for (int t = tid; t < ne; t += TPB) wl[t] = rl[t];
    wg_sums(1, sq(rl));
    grid_reduce(1, 0);
    double hprev = sqrt(res[0].x);  // beta; xchg holds the unnormalised start vector
    est = hprev;
    if (dead) break;
    if (hprev <= tol_abs || hprev == 0.0) {
      converged = true;
      break;
    }
    if (tid == 0) {
      for (int i = 0; i <= mm; ++i) gv[i] = mk(0.0, 0.0);
      gv[0] = mk(hprev, 0.0);
    }
    // the rotation wavefront keeps this cycle's rotations (lane l: rotation l) and the last
    // entry of g in registers; the LDS copies serve the least-squares solve at the end
    double rot_c = 1.0;
    double2 rot_s = mk(0.0, 0.0), gcur = mk(hprev, 0.0);
    int steps = 0;
    bool brk = false, stop = false;
    // cancellation below which the Pythagorean norm is replaced by a second pass
    const double eta = sizeof(R) == sizeof(float) ? 1e-4 : 1e-8;
    // A column's Givens update needs only h and hn, so in the one-pass case the rotation wavefront
    // keeps them in registers and applies the rotation during the next grid barrier, while
    // wavefront 0 waits for the other workgroups; the residual test of column j then comes
    // after the next column's stencil and sums, and if it stops the solve, that column is
    // dropped (its v_{j+1} = Vb[j + 1] closes the cycle).  pend is uniform.
    // The rotation's inputs wait in LDS (pg_*), not in registers that every thread would hold.
    bool pend = false, vlast_in_vb = false;
    for (int j = 0; j < mm; ++j) {
      // xchg holds hprev * v_j (written before the last barrier); halo form: wl holds it
      // on the own and halo sites
      const double inv = 1.0 / hprev;
      for (int t = tid; t < (HALO ? nle : ne); t += TPB) {
        const T src = (!HALO && j == 0) ? rl[t] : wl[t];
        Vb[j * vst + t] = from_d<R>(cscale(to_d(src), inv));
      }
      for (int t = tid; t < (HALO ? 0 : nsl * 5 * NC); t += TPB) {
        const int sl = t / (5 * NC), d = (t / NC) % 5, jj = t % NC;
        const int S = S0 + sl, X = S % a.Lx, Tt = S / a.Lx;
        int nb;
        switch (d) {
          case 0: nb = S; break;
          case 1: nb = ((X + 1 == a.Lx) ? 0 : X + 1) + a.Lx * Tt; break;
          case 2: nb = ((X == 0) ? a.Lx - 1 : X - 1) + a.Lx * Tt; break;
          case 3: nb = X + a.Lx * ((Tt + 1 == a.Lt) ? 0 : Tt + 1); break;
          default: nb = X + a.Lx * ((Tt == 0) ? a.Lt - 1 : Tt - 1); break;
        }
        xs[t] = cp_load(&xch[(int64_t)nb * NC + jj]);
      }
      // the halo form's stencil reads w itself, not the scaled copy or an exchange load
      if (!HALO) __syncthreads();
      if (REG && tid < nsl * 5 * NC) {
        const int g = tid / NC, u = tid % NC, odd = u & 1;
        const T* xv = wl + loc[g] * NC + odd * (NC / 2);
        double2 a0 = mk(0.0, 0.0), a1 = mk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < NC / 2; ++c) {
          const double2 xc = to_d(xv[c]);
          cfma(a0, to_d(areg[c]), xc);
          cfma(a1, to_d(areg[NC / 2 + c]), xc);
        }
        // the even thread of the pair completes row u / 2, the odd one row u / 2 + 12 (first
        // column half first in both); a pair never straddles a block or a wavefront
        const double2 send = odd ? a0 : a1;
        const double2 recv = mk(cp_dpp<0xB1>(send.x), cp_dpp<0xB1>(send.y));  // quad_perm [1, 0, 3, 2]
        part[g * NC + (u >> 1) + odd * (NC / 2)] = odd ? cadd(recv, a1) : cadd(a0, recv);
      }
      for (int t = tid; t < (REG ? 0 : nsl * 5 * NC); t += TPB) {
        const int sl = t / (5 * NC), d = (t / NC) % 5, i = t % NC;
        const T* blk = ALDS ? (Ab + ((int64_t)sl * 5 + d) * NC * NC) : (Ag + ((int64_t)(S0 + sl) * 5 + d) * NC * NC);
        const T* xv = HALO ? wl + loc[sl * 5 + d] * NC : xs + (sl * 5 + d) * NC;
        T av[NC / 2];
        double2 acc = mk(0.0, 0.0);
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
#pragma unroll
          for (int jj = 0; jj < NC / 2; ++jj) av[jj] = blk[(h2 * (NC / 2) + jj) * NC + i];
#pragma unroll
          for (int jj = 0; jj < NC / 2; ++jj) cfma(acc, to_d(av[jj]), to_d(xv[h2 * (NC / 2) + jj]));
        }
        part[t] = acc;
      }
      __syncthreads();
      for (int t = tid; t < ne; t += TPB) {
        const int sl = t / NC, i = t % NC;
        double2 y = part[(sl * 5 + 0) * NC + i];
        for (int d = 1; d < 5; ++d) y = cadd(y, part[(sl * 5 + d) * NC + i]);
        const T wv = from_d<R>(cscale(y, inv));
        wl[t] = wv;
        if (HALO) cp_store(&xch[(size_t)((j + 1) & 1) * n + e0 + t], wv);
      }
      __syncthreads();
      // h_i = V_i^H w (i <= j) and ||w||^2 in one reduction: half-wavefront q pairs w with V_q
      // (q <= j) or with itself (q = j + 1; the real part is ||w||^2)
      auto arn_dots = [&]() {
        const int q = tid / QL, c = tid % QL;
        if (q < j + 2) {
          const T* vq = q <= j ? Vb + q * vst : wl;
          double2 sm = mk(0.0, 0.0);
          for (int e = c; e < ne; e += QL) cfmac(sm, to_d(vq[e]), to_d(wl[e]));
          sm = group_sum(sm);
          if (c == 0) publish(q, sm);
        }
      };
      // w -= sum_{i <= j} res_i V_i on the own (and halo) entries
      const int nup = HALO ? nle : ne;
      auto gs_update = [&]() {
        for (int t = tid; t < nup; t += TPB) {
          double2 w = to_d(wl[t]);
          for (int i = 0; i <= j; ++i) w = csub(w, cmul(res[i], to_d(Vb[i * vst + t])));
          const T ws = from_d<R>(w);
          wl[t] = ws;
          if (!HALO && j + 1 < mm) cp_store(&xch[e0 + t], ws);  // hn * v_{j+1} for the next stencil
        }
      };
      // Givens update of column j (h_0 .. h_j from src, then hn) on the last wavefront: lane l
      // loads entry l and rotation l, then the chain runs in every lane on values read from one
      // lane at a time (scalar registers, no LDS round trip per rotation); lane 0 stores
      auto givens_r = [&](int j, double2 h0, double2 hnext, double hn) {
        // rotations 0 .. j-1 on the column (h_0 .. h_j, hn) by a lane scan, then the new one
        double2* col = Hr + (mm + 1) * j;
        const double cl = lane < j ? rot_c : 1.0;
        const double2 sl = lane < j ? rot_s : mk(0.0, 0.0);
        double2 x0;
        const double2 xq = cp_rotation_scan(lane, j, h0, cl, sl, hnext, x0);
        if (lane < j) col[lane] = cadd(cscale(xq, cl), cmul(sl, hnext));
        const double2 x1 = mk(hn, 0.0);
        double c;
        double2 sg;
        cp_givens(x0, x1, c, sg);
        // g_j = c g_j + s g_{j+1} and g_{j+1} = -conj(s) g_j with g_{j+1} = 0 before this rotation
        const double2 gj = cscale(gcur, c), gn = csub(mk(0.0, 0.0), cmul(cconj(sg), gcur));
        if (lane == j) {
          rot_c = c;
          rot_s = sg;
        }
        gcur = gn;
        if (lane == 0) {
          col[j] = cadd(cscale(x0, c), cmul(sg, x1));
          col[j + 1] = mk(0.0, 0.0);
          rc[j] = c;
          rs[j] = sg;
          gv[j] = gj;
          gv[j + 1] = gn;
          sh_scal[0] = cabs2(gn);  // squared residual estimate
        }
      };
      auto givens = [&](const double2* src, double hn) {
        givens_r(j, src[0], lane + 1 <= j ? src[lane + 1] : mk(hn, 0.0), hn);  // lane l: h_{l+1}
      };
      auto run_pending = [&]() {
        if (wave == (TPB / 64) - 1) givens_r(pg_j, pg_h0, pg_hnext[lane], pg_hn);
      };
      arn_dots();
      const bool had_pend = pend;
      grid_reduce_h(j + 2, (j + 1) & 1, [&]() {
        if (had_pend) run_pending();
      });
      pend = false;
      if (had_pend && !dead && sh_scal[0] <= tol_abs * tol_abs) {
        // column j - 1 met the tolerance: drop column j
        est = sh_scal[0];
        steps = j;
        vlast_in_vb = true;
        stop = true;
        break;
      }
      const double ww = res[j + 1].x;
      if (wave == (TPB / 64) - 1) {
        // ||h||^2, the cancellation test and (without a second pass) the rotation's inputs,
        // while the other wavefronts apply the first pass
        const double rsum = cp_row_sum(lane <= j ? cabs2(res[lane]) : 0.0);
        const double hh = (cp_lane(rsum, 0) + cp_lane(rsum, 16)) + (cp_lane(rsum, 32) + cp_lane(rsum, 48));
        const double hn2 = ww - hh;
        const bool second = !(hn2 > eta * ww);
        if (second) {
          if (lane <= j) Hr[lane + (mm + 1) * j] = res[lane];  // first-pass coefficients
        } else {
          double hn1 = sqrt(fmax(hn2, 0.0));
          const bool b = !(hn2 > 1e-24 * ww);  // hn1 <= 1e-12 ||w|| without a second root
          if (b) hn1 = 0.0;
          pg_hnext[lane] = lane + 1 <= j ? res[lane + 1] : mk(hn1, 0.0);  // lane l: h_{l+1}
          if (lane == 0) {
            pg_j = j;
            pg_h0 = res[0];
            pg_hn = hn1;
            sh_scal[1] = hn1;
            sh_flag[2] = b ? 1 : 0;
          }
        }
        if (lane == 0) sh_flag[1] = second ? 1 : 0;
      }
      gs_update();
      __syncthreads();
      double hn;
      if (sh_flag[1]) {
        // heavy cancellation: a second pass with an exact norm
        arn_dots();
        grid_reduce(j + 2);
        double hh2 = 0.0;
        for (int i = 0; i <= j; ++i) hh2 += cabs2(res[i]);
        const double hn2 = res[j + 1].x - hh2;
        if (tid <= j) Hr[tid + (mm + 1) * j] = cadd(Hr[tid + (mm + 1) * j], res[tid]);
        gs_update();
        hn = sqrt(fmax(hn2, 0.0));
        if (!(hn > 1e-12 * sqrt(ww))) { hn = 0.0; brk = true; }
        __syncthreads();
        if (wave == (TPB / 64) - 1) givens(Hr + (mm + 1) * j, hn);
        __syncthreads();
      } else {
        hn = sh_scal[1];
        brk = sh_flag[2] != 0;
        pend = true;
      }
      if (!HALO && j + 1 < mm) {
        // the two-barrier form's second barrier carries the rotation
        const bool p2 = pend;
        dead = dead || cp_barrier(a.flags, G, ++gen, a.err, [&]() {
          if (p2) run_pending();
        });
        pend = false;
      }
      steps = j + 1;
      hprev = hn;
      const bool halt = dead || brk || iters + steps >= a.max_iters;
      if (pend && (halt || j + 1 == mm)) {
        run_pending();
        __syncthreads();
        pend = false;
      }
      if (!pend) {
        est = brk ? 0.0 : sh_scal[0];  // squared until the cycle ends
        if (halt || est <= tol_abs * tol_abs) { stop = true; break; }
      }
    }
    est = sqrt(est);  // every step above left the squared estimate
    // ------------------------------------------------------------ end of cycle: x += V y, r = V u
    if (wave == 0) {
      // y = R^{-1} g by columns on one wavefront: lane i carries g_i - sum_{l > i} R_il y_l;
      // y_l = carry_l / R_ll from lane l's carry and reciprocal (scalar reads; the reciprocals
      // are taken beforehand, one per lane), then every lane i < l drops its term, with its
      // entry of the next column already loaded
      double2 acc = lane < steps ? gv[lane] : mk(0.0, 0.0);
      const double2 dl = lane < steps ? Hr[lane + (mm + 1) * lane] : mk(1.0, 0.0);
      const double2 rdl = cabs2(dl) > 0.0 ? cp_div(mk(1.0, 0.0), dl) : mk(0.0, 0.0);
      double2 rcol = (steps > 0 && lane < steps) ? Hr[lane + (mm + 1) * (steps - 1)] : mk(0.0, 0.0);
      for (int l = steps - 1; l >= 0; --l) {
        const double2 rnx = (l > 0 && lane < l) ? Hr[lane + (mm + 1) * (l - 1)] : mk(0.0, 0.0);
        const double2 yl = cmul(cp_lane(acc, l), cp_lane(rdl, l));
        if (lane == l) yv[l] = yl;
        if (lane < l) acc = csub(acc, cmul(rcol, yl));
        rcol = rnx;
      }
      // residual coordinates u = Omega^H (g_steps e_steps), Omega^H applying the inverse
      // rotations [c -s; conj(s) c] from the last one down: with u_q = 0 on entry, rotation q
      // leaves u_{q+1} = c_q t and carries t <- -s_q t down to u_q (t = g_steps at first)
      const double cl = lane < steps ? rc[lane] : 1.0;
      const double2 sl = lane < steps ? rs[lane] : mk(0.0, 0.0);
      double2 tc = brk ? mk(0.0, 0.0) : gv[steps];
      for (int q = steps - 1; q >= 0; --q) {
        if (lane == q + 1) uv[q + 1] = cscale(tc, cp_lane(cl, q));
        tc = csub(mk(0.0, 0.0), cmul(cp_lane(sl, q), tc));
      }
      if (lane == 0) uv[0] = tc;
    }
    __syncthreads();
    // v_steps: hprev * v_steps is in wl, or v_steps itself in Vb when a column was dropped
    const double invn = vlast_in_vb ? 1.0 : (hprev > 0.0 ? 1.0 / hprev : 0.0);
    const T* vlast = vlast_in_vb ? Vb + steps * vst : wl;
    for (int t = tid; t < ne; t += TPB) {
      double2 xv = to_d(xl[t]);
      double2 rv = mk(0.0, 0.0);
      for (int i = 0; i < steps; ++i) {
        const double2 vi = to_d(Vb[i * vst + t]);
        cfma(xv, yv[i], vi);
        cfma(rv, uv[i], vi);
      }
      cfma(rv, uv[steps], cscale(to_d(vlast[t]), invn));
      xl[t] = from_d<R>(xv);
      rl[t] = from_d<R>(rv);
    }
    __syncthreads();
    iters += steps;
    if (brk || est <= tol_abs) converged = true;
    if (stop && !converged) break;  // iteration cap
  }
  for (int t = tid; t < ne; t += TPB) xg[e0 + t] = xl[t];
  if (gi == 0 && tid == 0) {
    a.out_iters[0] += iters;  // accumulated over the calls of one outer solve
    a.out_relres[0] = bnorm > 0.0 ? est / bnorm : 0.0;
  }
}

// ---------------------------------------------------------------- persistent GMRES-DR cycle
// The Arnoldi part of one GMRES-DR cycle (the first coarse solve) in one launch: starting from
// the j0 + 1 orthonormal columns in V and the cycle's small-dense state (after a deflated
// restart: the full (k+1) x k block, its rotations, g), the kernel extends the relation
// A V_j = V_{j+1} Hbar_j column by column up to m, or until the Givens residual reaches
// tol_abs or the process breaks down, with the same layout and helpers as k_coarse_proj:
// workgroups own consecutive coarse sites, keep their slices of V in LDS, exchange v_j for
// the stencil through one global field, and reduce dot products through per-workgroup
// partials and a flag-array grid barrier.  Gram-Schmidt is classical: one pass with the norm
// from ||w||^2 - ||h||^2, and a second, exact pass when that difference shows cancellation
// beyond eta (the Arnoldi relation holds to working accuracy either way, since H holds the
// coefficients actually subtracted).  Two barriers per column (exchange and reduction), three
// with a second pass.  Every workgroup holds the same small-dense state; workgroup 0 writes it
// back (H, R, g, rotations, steps, flags).
constexpr int CA_NROT = 256;  // rotations held in LDS (restart block plus this cycle's)

struct CAArgs {
  const double2* A;
  int Lx, Lt;
  double2* V;          // basis, ld n entries, columns 0 .. j0 valid on entry
  KState* ks;
  int j0, m;
  double2* xchg;       // exchange field (n entries)
  double2* partials;   // 2 x CP_QMAX x G
  unsigned* flags;     // G barrier flags, CP_FLAGPAD apart, zero at launch
  int* err;
  int spw;
  double eta;          // cancellation below which the Pythagorean norm gives way to a second pass
};

struct CALayout {
  size_t Vb, xs, part, wl, hcol, red, res, rc, rs, rp, g, q0, tot;
  __host__ __device__ CALayout(int spw, int m) {
    const size_t ne = (size_t)spw * NC;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = cp_align(o + bytes); return at; };
    Vb = take((size_t)(m + 1) * ne * sizeof(double2));
    xs = take((size_t)spw * 5 * NC * sizeof(double2));
    part = take((size_t)(spw * 5 * NC > CP_QMAX * 32 ? spw * 5 * NC : CP_QMAX * 32) * sizeof(double2));
    wl = take(ne * sizeof(double2));
    hcol = take((size_t)(m + 2) * sizeof(double2));
    red = take((size_t)CP_QMAX * sizeof(double2));
    res = take((size_t)(CP_QMAX + 2) * sizeof(double2));
    rc = take((size_t)CA_NROT * sizeof(double));
    rs = take((size_t)CA_NROT * sizeof(double2));
    rp = take((size_t)CA_NROT * sizeof(int));
    g = take((size_t)(m + 2) * sizeof(double2));
    q0 = take((size_t)m * m * sizeof(double2));  // product of the entry rotations, (j0 + 1)^2 <= m^2
    tot = o;
  }
};

__global__ void __launch_bounds__(CP_THREADS) k_coarse_arnoldi(CAArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int LDK = MMAX + 1;
  unsigned gen = 0;
  bool dead = false;
  const int G = gridDim.x, gi = blockIdx.x, tid = threadIdx.x;
  const int V = a.Lx * a.Lt;
  const int S0 = gi * a.spw;
  const int nsl = min(a.spw, V - S0);
  const int ne = nsl * NC;
  const int m = a.m, j0 = a.j0;
  const int64_t n = (int64_t)V * NC;
  const int64_t e0 = (int64_t)S0 * NC;
  const CALayout L(a.spw, m);
  double2* Vb = (double2*)(smem + L.Vb);
  double2* xs = (double2*)(smem + L.xs);
  double2* part = (double2*)(smem + L.part);
  double2* wl = (double2*)(smem + L.wl);
  double2* hcol = (double2*)(smem + L.hcol);
  double2* red = (double2*)(smem + L.red);
  double2* res = (double2*)(smem + L.res);
  double* rc = (double*)(smem + L.rc);
  double2* rs = (double2*)(smem + L.rs);
  int* rp = (int*)(smem + L.rp);
  double2* gl = (double2*)(smem + L.g);
  double2* Q0 = (double2*)(smem + L.q0);
  __shared__ double sh_est;
  KState* ks = a.ks;
  double2* xch = a.xchg;
  if (ks->done) return;  // the cycle start found nothing to do (uniform: read before any write)
  const int nrot0 = ks->nrot;
  const double tol_abs = ks->tol_abs;
  int rbuf = 0;

  // the reductions of k_coarse_proj (quantity q on threads 32 q .. 32 q + 31)
  auto wg_sums = [&](int nq, auto&& term) {
    const int q = tid >> 5, c = tid & 31;
    if (q < nq) {
      double2 sm = mk(0.0, 0.0);
      for (int e = c; e < ne; e += 32) sm = cadd(sm, term(q, e));
      sm = cp_half_sum(sm);
      if (c == 0) red[q] = sm;
    }
  };
  auto grid_reduce = [&](int nq) {
    __syncthreads();
    double2* P = a.partials + (size_t)rbuf * CP_QMAX * G;
    if (tid < nq) cp_store(&P[(size_t)tid * G + gi], red[tid]);
    dead = dead || cp_barrier(a.flags, G, ++gen, a.err);
    const int q = tid >> 5, c = tid & 31;
    if (q < nq) {
      const double2 sm = cp_gather_sum(P + (size_t)q * G, G, c);
      if (c == 0) res[q] = sm;
    }
    __syncthreads();
    rbuf ^= 1;
  };

  // ---------------------------------------------------------------- resident state
  for (int q = tid; q < nrot0; q += CP_THREADS) {
    rc[q] = ks->rot_c[q];
    rs[q] = ks->rot_s[q];
    rp[q] = ks->rot_p[q];
  }
  for (int i = tid; i <= m; i += CP_THREADS) gl[i] = ks->g[i];
  for (int t = tid; t < (j0 + 1) * ne; t += CP_THREADS) {
    const int i = t / ne, e = t % ne;
    Vb[t] = a.V[(int64_t)i * n + e0 + e];
  }
  __syncthreads();
  // Q0 = product of the rotations held on entry (they act on rows 0 .. j0 only): thread l
  // carries e_l through them, so every new column needs one (j0+1) x (j0+1) product instead of
  // a chain of nrot0 rotations
  const int n0 = j0 + 1;
  if (tid < n0) {
    for (int i = 0; i < n0; ++i) Q0[i + n0 * tid] = mk(i == tid ? 1.0 : 0.0, 0.0);
    for (int q = 0; q < nrot0; ++q) {
      const int p = rp[q];
      const double2 x0 = Q0[p + n0 * tid], x1 = Q0[p + 1 + n0 * tid];
      Q0[p + n0 * tid] = cadd(cscale(x0, rc[q]), cmul(rs[q], x1));
      Q0[p + 1 + n0 * tid] = csub(cscale(x1, rc[q]), cmul(cconj(rs[q]), x0));
    }
  }
  for (int t = tid; t < ne; t += CP_THREADS) cp_store(&xch[e0 + t], Vb[j0 * ne + t]);
  dead = dead || cp_barrier(a.flags, G, ++gen, a.err);

  int nrot = nrot0, steps = j0;
  bool brk = false;
  double est = ks->est, wn0 = 0.0;
  for (int j = j0; j < m && !dead; ++j) {
    // w = A v_j (neighbour values of v_j from the exchange field)
    for (int t = tid; t < nsl * 5 * NC; t += CP_THREADS) {
      const int sl = t / (5 * NC), d = (t / NC) % 5, jj = t % NC;
      const int S = S0 + sl, X = S % a.Lx, Tt = S / a.Lx;
      int nb;
      switch (d) {
        case 0: nb = S; break;
        case 1: nb = ((X + 1 == a.Lx) ? 0 : X + 1) + a.Lx * Tt; break;
        case 2: nb = ((X == 0) ? a.Lx - 1 : X - 1) + a.Lx * Tt; break;
        case 3: nb = X + a.Lx * ((Tt + 1 == a.Lt) ? 0 : Tt + 1); break;
        default: nb = X + a.Lx * ((Tt == 0) ? a.Lt - 1 : Tt - 1); break;
      }
      xs[t] = cp_load(&xch[(int64_t)nb * NC + jj]);
    }
    __syncthreads();
    for (int t = tid; t < nsl * 5 * NC; t += CP_THREADS) {
      const int sl = t / (5 * NC), d = (t / NC) % 5, i = t % NC;
      const double2* blk = a.A + ((int64_t)(S0 + sl) * 5 + d) * NC * NC;
      const double2* xv = xs + (sl * 5 + d) * NC;
      double2 av[NC / 2];
      double2 acc = mk(0.0, 0.0);
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
#pragma unroll
        for (int jj = 0; jj < NC / 2; ++jj) av[jj] = blk[(h2 * (NC / 2) + jj) * NC + i];
#pragma unroll
        for (int jj = 0; jj < NC / 2; ++jj) cfma(acc, av[jj], xv[h2 * (NC / 2) + jj]);
      }
      part[t] = acc;
    }
    __syncthreads();
    for (int t = tid; t < ne; t += CP_THREADS) {
      const int sl = t / NC, i = t % NC;
      double2 y = part[(sl * 5 + 0) * NC + i];
      for (int d = 1; d < 5; ++d) y = cadd(y, part[(sl * 5 + d) * NC + i]);
      wl[t] = y;
    }
    __syncthreads();
    auto dots = [&](int q, int e) {
      double2 v = mk(0.0, 0.0);
      if (q <= j) cfmac(v, Vb[q * ne + e], wl[e]);
      else v.x = cabs2(wl[e]);
      return v;
    };
    // h = V^H w and ||w||^2 in one reduction; the norm of w - V h from ||w||^2 - ||h||^2 unless
    // that difference shows cancellation beyond eta, in which case w - V h goes through an exact
    // second pass (H(:, j) = h + h2)
    wg_sums(j + 2, dots);
    grid_reduce(j + 2);
    const double ww = res[j + 1].x;
    wn0 = sqrt(ww);
    double hh = 0.0;
    for (int i = 0; i <= j; ++i) hh += cabs2(res[i]);
    double hn;
    if (tid <= j) hcol[tid] = res[tid];
    if (!(ww - hh > a.eta * ww)) {
      for (int t = tid; t < ne; t += CP_THREADS) {
        double2 w = wl[t];
        for (int i = 0; i <= j; ++i) w = csub(w, cmul(res[i], Vb[i * ne + t]));
        wl[t] = w;
      }
      __syncthreads();
      wg_sums(j + 2, dots);
      grid_reduce(j + 2);
      double hh2 = 0.0;
      for (int i = 0; i <= j; ++i) hh2 += cabs2(res[i]);
      hn = sqrt(fmax(res[j + 1].x - hh2, 0.0));
      if (!(hn > 1e-12 * wn0)) {
        hn = 0.0;
        brk = true;
      }
      if (tid <= j) hcol[tid] = cadd(hcol[tid], res[tid]);
    } else {
      hn = sqrt(ww - hh);  // above sqrt(eta) ||w||: no breakdown
    }
    __syncthreads();
    // Givens update on the last wavefront (overlaps the vector update below): rows 0 .. j0 of
    // the column through the entry rotations (Q0), then this cycle's rotations at positions
    // j0 .. j-1 by a lane scan, then the new rotation
    if (tid >= CP_THREADS - 64) {
      const int lane = tid & 63;
      double2* col = hcol;  // rotated in place (no other thread reads it until the next column)
      const double2 hl = lane <= j ? col[lane] : (lane == j + 1 ? mk(hn, 0.0) : mk(0.0, 0.0));
      if (gi == 0)
        for (int i = lane; i <= MMAX; i += 64) ks->H[LDK * j + i] = (i <= j) ? col[i] : (i == j + 1 ? mk(hn, 0.0) : mk(0.0, 0.0));
      double2 y = hl;
      if (lane < n0) {
        y = mk(0.0, 0.0);
        for (int l = 0; l < n0; ++l) cfma(y, Q0[lane + n0 * l], col[l]);
      }
      const int cnt = j - j0;  // this cycle's earlier rotations
      const int q = nrot0 + lane;
      const double cl = lane < cnt ? rc[q] : 1.0;
      const double2 sl = lane < cnt ? rs[q] : mk(0.0, 0.0);
      const double2 hnext = j0 + lane + 1 <= j ? col[j0 + lane + 1] : mk(hn, 0.0);
      double2 x0;
      const double2 xq = cp_rotation_scan(lane, cnt, cp_lane(y, j0), cl, sl, hnext, x0);
      const double2 x1 = mk(hn, 0.0);
      double c;
      double2 sg;
      cp_givens(x0, x1, c, sg);
      // the rotated column: rows < j0 from Q0, rows j0 .. j-1 from the scan (scan lane l holds
      // row j0 + l), row j from the new rotation; every lane read col above
      const double2 o = cadd(cscale(xq, cl), cmul(sl, hnext));
      const double2 rj = cadd(cscale(x0, c), cmul(sg, x1));
      if (lane < j0) col[lane] = y;
      if (lane < cnt) col[j0 + lane] = o;
      if (lane == 0) {
        col[j] = rj;
        col[j + 1] = mk(0.0, 0.0);
      }
      if (gi == 0) {
        if (lane < j0) ks->R[LDK * j + lane] = y;
        if (lane < cnt) ks->R[LDK * j + j0 + lane] = o;
        if (lane == 0) {
          ks->R[LDK * j + j] = rj;
          ks->R[LDK * j + j + 1] = mk(0.0, 0.0);
        }
      }
      if (lane == 0) {
        rc[nrot] = c;
        rs[nrot] = sg;
        rp[nrot] = j;
        const double2 g0 = gl[j], g1 = gl[j + 1];
        gl[j] = cadd(cscale(g0, c), cmul(sg, g1));
        gl[j + 1] = csub(cscale(g1, c), cmul(cconj(sg), g0));
        sh_est = sqrt(cabs2(gl[j + 1]));
        if (gi == 0) {
          ks->g[j] = gl[j];
          ks->g[j + 1] = gl[j + 1];
          ks->rot_c[nrot] = c;
          ks->rot_s[nrot] = sg;
          ks->rot_p[nrot] = j;
        }
      }
    }
    // v_{j+1} = (w - V h) / hn, h of the last pass
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    for (int t = tid; t < ne; t += CP_THREADS) {
      double2 w = wl[t];
      for (int i = 0; i <= j; ++i) w = csub(w, cmul(res[i], Vb[i * ne + t]));
      const double2 v = hn > 0.0 ? cscale(w, inv) : w;
      Vb[(j + 1) * ne + t] = v;
      a.V[(int64_t)(j + 1) * n + e0 + t] = v;
      cp_store(&xch[e0 + t], v);
    }
    __syncthreads();
    ++nrot;
    steps = j + 1;
    est = brk ? 0.0 : sh_est;
    if (brk || est <= tol_abs) break;
    if (j + 1 < m) dead = dead || cp_barrier(a.flags, G, ++gen, a.err);
  }
  if (gi == 0 && tid == 0) {
    ks->nrot = nrot;
    ks->steps = steps;
    ks->est = est;
    ks->wn0 = wn0;
    if (brk) ks->breakdown = 1;
    if (brk || est <= tol_abs) ks->done = 1;
  }
}

size_t coarse_arnoldi_lds(int spw, int m) { return CALayout(spw, m).tot; }

// Returns 1 if the persistent cycle ran (V columns j0+1 .. steps and ks updated), 0 if it
// cannot run co-resident or its state does not fit (the caller then takes the kernel-per-step
// path).  Cooperative launch.
int launch_coarse_arnoldi(hipStream_t st, const double2* A, int Lx, int Lt, double2* V, KState* ks, int nrot_bound,
                          int j0, int m, double2* xchg, double2* partials, size_t partials_elems, unsigned* flags,
                          size_t flag_words, int* err) {
  if (m + 2 > CP_QMAX || m > MMAX || j0 >= m || nrot_bound + (m - j0) > CA_NROT) return 0;
  const int Vs = Lx * Lt;
  int spw = (Vs + 63) / 64;  // about 64 workgroups (measured: 5 % faster per step than 32)
  if (spw > 10) spw = 10;
  const int G = (Vs + spw - 1) / spw;
  if (G > CP_GMAX || (size_t)2 * CP_QMAX * G > partials_elems || (size_t)CP_FLAGPAD * G > flag_words) return 0;
  const size_t lds = coarse_arnoldi_lds(spw, m);
  if (lds > 160 * 1024) return 0;
  const void* fn = (const void*)k_coarse_arnoldi;
  if (ensure_dyn_lds(fn, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  int per_cu = 0, ncu = 0;
  if (occupancy_cached(fn, CP_THREADS, lds, &per_cu, &ncu) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (per_cu < 1 || G > per_cu * ncu) return 0;
  if (hipMemsetAsync(flags, 0, sizeof(unsigned) * CP_FLAGPAD * G, st) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  // DMG_ARNOLDI_TWO_PASS=1 takes the second pass at every step (read at each call)
  const char* e2 = getenv("DMG_ARNOLDI_TWO_PASS");
  const double eta = (e2 && *e2 && *e2 != '0') ? 2.0 : 1e-8;
  CAArgs a{A, Lx, Lt, V, ks, j0, m, xchg, partials, flags, err, spw, eta};
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel(fn, dim3(G), dim3(CP_THREADS), args, (unsigned)lds, st) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return 1;
}

// DMG_COARSE_HALO=0 selects the two-barrier form (the same solve up to rounding order).
static bool cp_halo_enabled() {
  static const int on = [] {
    const char* e = getenv("DMG_COARSE_HALO");
    return (e && *e == '0') ? 0 : 1;
  }();
  return on != 0;
}

// Target number of workgroups of the persistent GMRES-Proj launch (DMG_COARSE_GROUPS, default 64).
static int cp_groups_default() {
  static const int g = [] {
    const char* e = getenv("DMG_COARSE_GROUPS");
    const int v = e ? atoi(e) : 0;
    return (v >= 1 && v <= CP_GMAX) ? v : 64;
  }();
  return g;
}

static bool cp_debug() {
  static const int on = [] {
    const char* e = getenv("DMG_DEBUG");
    return (e && *e && *e != '0') ? 1 : 0;
  }();
  return on != 0;
}

template <typename R>
static const void* proj_fn(bool alds, bool halo, bool reg) {
  if (reg) return (const void*)k_coarse_proj<R, false, true, true>;
  if (halo) return alds ? (const void*)k_coarse_proj<R, true, true> : (const void*)k_coarse_proj<R, false, true>;
  return alds ? (const void*)k_coarse_proj<R, true, false> : (const void*)k_coarse_proj<R, false, false>;
}

template <typename R>
static int try_launch(hipStream_t st, CPArgs& a, int G, size_t lds, bool alds, bool halo, bool reg, int coop) {
  void* args[] = {&a};
  const void* fn = proj_fn<R>(alds, halo, reg);
  const int threads = reg ? 512 : CP_THREADS;
  hipError_t e = ensure_dyn_lds(fn, lds);
  if (e != hipSuccess) {
    if (cp_debug()) fprintf(stderr, "[dmg] coarse kernel: set LDS %zu failed: %s\n", lds, hipGetErrorString(e));
    (void)hipGetLastError();
    return 0;
  }
  int per_cu = 0, ncu = 0;
  e = occupancy_cached(fn, threads, lds, &per_cu, &ncu);
  if (e != hipSuccess) {
    if (cp_debug()) fprintf(stderr, "[dmg] coarse kernel: occupancy query failed: %s\n", hipGetErrorString(e));
    (void)hipGetLastError();
    return 0;
  }
  if (per_cu < 1 || G > per_cu * ncu) {
    if (cp_debug())
      fprintf(stderr, "[dmg] coarse kernel: %d workgroups of %d threads, LDS %zu: %d per CU x %d CUs\n", G,
              threads, lds, per_cu, ncu);
    return 0;
  }
  if (hipMemsetAsync(a.flags, 0, sizeof(unsigned) * CP_FLAGPAD * G, st) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (coop) {
    e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(threads), args, (unsigned)lds, st);
  } else {
    // Plain launch: the grid (G <= 256 workgroups, one per CU) always fits the device,
    // so every workgroup is placed once earlier kernels drain; the barrier's spin limit
    // bounds any wait.
    if (reg) {
      hipLaunchKernelGGL((k_coarse_proj<R, false, true, true>), dim3(G), dim3(threads), lds, st, a);
    } else if (halo) {
      if (alds) hipLaunchKernelGGL((k_coarse_proj<R, true, true>), dim3(G), dim3(CP_THREADS), lds, st, a);
      else hipLaunchKernelGGL((k_coarse_proj<R, false, true>), dim3(G), dim3(CP_THREADS), lds, st, a);
    } else {
      if (alds) hipLaunchKernelGGL((k_coarse_proj<R, true, false>), dim3(G), dim3(CP_THREADS), lds, st, a);
      else hipLaunchKernelGGL((k_coarse_proj<R, false, false>), dim3(G), dim3(CP_THREADS), lds, st, a);
    }
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    if (cp_debug()) fprintf(stderr, "[dmg] coarse kernel: launch failed: %s\n", hipGetErrorString(e));
    (void)hipGetLastError();
    return 0;
  }
  return 1;
}

size_t coarse_proj_flag_words(int G) { return (size_t)CP_FLAGPAD * G; }

// Returns 1 if the persistent kernel was launched, 0 if it cannot run co-resident here
// (the caller then uses the multi-kernel path).  `groups` is the target number of
// workgroups (0: 64).
template <typename R>
int launch_coarse_proj(hipStream_t st, const cx<R>* A, int Lx, int Lt, const cx<R>* DV, const double2* DM,
                       const double2* DP, int k,
                       const cx<R>* b, cx<R>* x, double tol, int mm, int max_iters, cx<R>* xchg,
                       double2* partials, size_t partials_elems, int* out_iters, double* out_relres,
                       unsigned* flags, size_t flag_words, int* err, int groups, int coop) {
  if (mm + 2 > CP_QMAX || k + 1 > CP_QMAX || mm < 1) return 0;
  const int V = Lx * Lt;
  const size_t lds_max = 160 * 1024;
  if (groups <= 0) groups = cp_groups_default();
  int spw = (V + groups - 1) / groups;
  if (spw > 10) spw = 10;  // one thread per local entry
  const int G = (V + spw - 1) / spw;
  if (G > CP_GMAX || (size_t)2 * CP_QMAX * G > partials_elems || (size_t)CP_FLAGPAD * G > flag_words) return 0;
  static_assert(CP_QMAX * 32 == CP_THREADS, "one half-wavefront per reduced quantity");
  // own + halo sites of the largest halo (same routine as the kernel)
  int nl = 0;
  {
    std::vector<int> hs((size_t)4 * spw);
    for (int g = 0; g < G; ++g) {
      const int S0 = g * spw, nsl = std::min(spw, V - S0);
      nl = std::max(nl, nsl + cp_halo(S0, nsl, Lx, Lt, nullptr, hs.data()));
    }
  }
  // halo form (one barrier per Arnoldi step) first: with the blocks in registers (512 threads,
  // at most 4 sites per workgroup), then with the blocks in LDS where they fit, then from L2
  const int halo_ok = cp_halo_enabled() ? 1 : 0;
  if (halo_ok && spw * 5 * NC <= 512) {
    const size_t lds = CPLayout(spw, mm, k, sizeof(cx<R>), 0, nl).tot;
    if (lds <= lds_max) {
      CPArgs a{A, Lx, Lt, DV, DM, DP, k, b, x, tol, mm, max_iters, xchg, partials, out_iters, out_relres,
               flags, err, spw, 0, nl};
      if (try_launch<R>(st, a, G, lds, false, true, true, coop)) return 1;
    }
  }
  for (int halo = halo_ok; halo >= 0; --halo)
    for (int alds = 1; alds >= 0; --alds) {
      const size_t lds = CPLayout(spw, mm, k, sizeof(cx<R>), alds, halo ? nl : 0).tot;
      if (lds > lds_max) {
        if (cp_debug()) fprintf(stderr, "[dmg] coarse kernel (halo %d, blocks in LDS %d): LDS %zu exceeds %zu\n",
                                halo, alds, lds, lds_max);
        continue;
      }
      CPArgs a{A, Lx, Lt, DV, DM, DP, k, b, x, tol, mm, max_iters, xchg, partials, out_iters, out_relres,
               flags, err, spw, alds, halo ? nl : spw};
      if (try_launch<R>(st, a, G, lds, alds == 1, halo == 1, false, coop)) return 1;
    }
  return 0;
}

template int launch_coarse_proj<double>(hipStream_t, const double2*, int, int, const double2*, const double2*,
                                        const double2*, int,
                                        const double2*, double2*, double, int, int, double2*, double2*, size_t,
                                        int*, double*, unsigned*, size_t, int*, int, int);
template int launch_coarse_proj<float>(hipStream_t, const float2*, int, int, const float2*, const double2*,
                                       const double2*, int,
                                       const float2*, float2*, double, int, int, float2*, double2*, size_t, int*,
                                       double*, unsigned*, size_t, int*, int, int);

}  // namespace dmg
