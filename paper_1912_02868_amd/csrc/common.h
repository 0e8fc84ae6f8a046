// Internal declarations shared by the HIP sources of libdmg (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dmg.h"

namespace dmg {

// ---------------------------------------------------------------- complex types
template <typename R> struct C2;
template <> struct C2<double> { using T = double2; };
template <> struct C2<float> { using T = float2; };
template <typename R> using cx = typename C2<R>::T;

__host__ __device__ inline double2 mk(double a, double b) { return make_double2(a, b); }
__host__ __device__ inline float2 mkf(float a, float b) { return make_float2(a, b); }

template <typename R> __host__ __device__ inline cx<R> make_cx(R a, R b) { cx<R> z; z.x = a; z.y = b; return z; }

template <typename T> __host__ __device__ inline T cadd(T a, T b) { T z; z.x = a.x + b.x; z.y = a.y + b.y; return z; }
template <typename T> __host__ __device__ inline T csub(T a, T b) { T z; z.x = a.x - b.x; z.y = a.y - b.y; return z; }
template <typename T> __host__ __device__ inline T cmul(T a, T b) {
  T z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z;
}
// conj(a) * b
template <typename T> __host__ __device__ inline T cmulc(T a, T b) {
  T z; z.x = a.x * b.x + a.y * b.y; z.y = a.x * b.y - a.y * b.x; return z;
}
template <typename T> __host__ __device__ inline T cconj(T a) { T z; z.x = a.x; z.y = -a.y; return z; }
template <typename T, typename S> __host__ __device__ inline T cscale(T a, S s) { T z; z.x = a.x * s; z.y = a.y * s; return z; }
// acc += a * b
template <typename T> __host__ __device__ inline void cfma(T& acc, T a, T b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename T> __host__ __device__ inline void cfmac(T& acc, T a, T b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double2 to_d(double2 a) { return a; }
__host__ __device__ inline double2 to_d(float2 a) { return make_double2(a.x, a.y); }
template <typename R> __host__ __device__ inline cx<R> from_d(double2 a) { return make_cx<R>((R)a.x, (R)a.y); }

// A complex block entry stored as two bfloat16 (the high 16 bits of the FP32 value, rounded to
// nearest even); loaded as FP32, exactly.
struct bf16c {
  unsigned short re, im;
};
__host__ __device__ inline double2 ld_blk(const double2* p) { return *p; }
__host__ __device__ inline float2 ld_blk(const float2* p) { return *p; }
__device__ inline float2 ld_blk(const bf16c* p) {
  const bf16c v = *p;
  return make_float2(__uint_as_float((unsigned)v.re << 16), __uint_as_float((unsigned)v.im << 16));
}
// XCD-aware workgroup order.  The dispatcher hands workgroup b of a grid of G to compute die
// (XCD) b % 8, and each of the 8 XCDs has its own L2.  The logical block returned here gives each
// XCD one contiguous range of [0, G) (XCD x: blocks start_x .. start_x + count_x - 1, in dispatch
// order), so neighbouring sites of a stencil are worked on by the same XCD, close in time, and
// their shared neighbour fields come from that XCD's L2 instead of the fabric.  A bijection on
// [0, G) for any G.
__device__ inline int xcd_block(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// storage type of the blocks of a stencil computing in precision R
template <typename R, bool B16> struct BlkT { using T = cx<R>; };
template <> struct BlkT<float, true> { using T = bf16c; };

// ---------------------------------------------------------------- errors
struct Error {
  dmg_status code;
  std::string msg;
};

#define DMG_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::dmg::Error{DMG_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define DMG_CHECK(cond, code, msg)                          \
  do {                                                      \
    if (!(cond)) throw ::dmg::Error{(code), std::string(msg)}; \
  } while (0)

#define DMG_LAUNCH_CHECK() DMG_HIP(hipGetLastError())

// ---------------------------------------------------------------- lattice constants
constexpr int NC = 24;      // dof per blocked site
constexpr int NV = 12;      // near-null vectors (per chirality)
constexpr int BLK = 4;      // blocking factor per direction
constexpr int MMAX = 64;    // largest Krylov cycle held by the small-dense state
constexpr int ROTMAX = MMAX * (MMAX + 1) / 2 + 2 * MMAX;

// ---------------------------------------------------------------- launch attributes
// Raise fn's dynamic-LDS limit on the current device to at least `bytes`; the attribute call is
// made only when a launch needs more than this process last set for that function.
inline hipError_t ensure_dyn_lds(const void* fn, size_t bytes) {
  struct Set {
    int dev;
    const void* fn;
    size_t bytes;
  };
  static std::mutex mu;
  static std::vector<Set> done;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  Set* hit = nullptr;
  for (auto& e : done)
    if (e.dev == dev && e.fn == fn) hit = &e;
  if (hit && hit->bytes >= bytes) return hipSuccess;
  const hipError_t r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (r == hipSuccess) {
    if (hit) hit->bytes = bytes;
    else done.push_back({dev, fn, bytes});
  }
  return r;
}
// Workgroups of fn (threads, lds) that one compute unit holds, and the compute units of the
// current device, remembered per (device, fn, threads, lds).
inline hipError_t occupancy_cached(const void* fn, int threads, size_t lds, int* per_cu, int* ncu) {
  struct Fit {
    int dev;
    const void* fn;
    int threads;
    size_t lds;
    int per_cu, ncu;
  };
  static std::mutex mu;
  static std::vector<Fit> known;
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> lock(mu);
    for (const auto& e : known)
      if (e.dev == dev && e.fn == fn && e.threads == threads && e.lds == lds) {
        *per_cu = e.per_cu;
        *ncu = e.ncu;
        return hipSuccess;
      }
  }
  int pc = 0, nc = 0;
  hipError_t r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, fn, threads, lds);
  if (r != hipSuccess) return r;
  r = hipDeviceGetAttribute(&nc, hipDeviceAttributeMultiprocessorCount, dev);
  if (r != hipSuccess) return r;
  std::lock_guard<std::mutex> lock(mu);
  known.push_back({dev, fn, threads, lds, pc, nc});
  *per_cu = pc;
  *ncu = nc;
  return hipSuccess;
}

// Small-dense state of one Krylov cycle, resident in device memory (FP64).
// Column-major (m + 1) x m Hessenberg: H[i + (MMAX + 1) * j].
struct KState {
  double2 H[(MMAX + 1) * MMAX];   // unrotated Arnoldi matrix
  double2 R[(MMAX + 1) * MMAX];   // rotated (upper triangular) factor
  double2 g[MMAX + 1];            // rotated right-hand side
  double2 c[MMAX + 1];            // unrotated right-hand side
  double2 y[MMAX + 1];            // least-squares solution / small work vector
  double2 u[MMAX + 1];            // residual coordinates c - H y
  double2 h2[MMAX + 1];           // scratch (second Gram-Schmidt pass)
  double2 rot_s[ROTMAX];
  double rot_c[ROTMAX];
  int rot_p[ROTMAX];
  int nrot;
  int steps;                      // Arnoldi columns completed in this cycle
  int done;                       // 1: stop (converged, breakdown or cap)
  int breakdown;
  double tol_abs;                 // stop when |g_{j+1}| <= tol_abs
  double est;                     // current least-squares residual norm
  double beta;                    // norm of the starting residual
  double wn0;                     // ||A v_j|| before orthogonalisation
  double bnorm;                   // ||b|| of the enclosing solve
  int pass2;                      // one-pass Gram-Schmidt cancelled: the exact second pass is due
  double scratch[8];
};

}  // namespace dmg

struct dmg_context {
  int device = 0;
  hipStream_t stream = nullptr;
  dmg_allocator alloc{nullptr, nullptr, nullptr};
  size_t budget = 0;
  size_t in_use = 0;
  std::mutex mu;  // allocation accounting and the kernel timer (batch slots run on host threads)
  // kernel timer (dmg_kernel_timer): event pairs per timed kernel, work units per launch
  int timing = 0;  // bit mask of timed kernels
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Span { int kernel; hipEvent_t a, b; long long units; };
  std::vector<Span> spans;
  long long pending_units[4] = {0, 0, 0, 0};
  void* scratch = nullptr;  // this device's address of the static scratch array (api.hip)
  ~dmg_context();
};

namespace dmg {
// Records an event on `stream` when kernel `kernel` is timed (nullptr otherwise).
hipEvent_t timer_mark(dmg_context* c, int kernel, hipStream_t stream);
void timer_span(dmg_context* c, int kernel, hipEvent_t a, hipEvent_t b, long long units);
}  // namespace dmg

namespace dmg {
// Error text of the calling thread's last call on context c (calls on different lane
// batches may come from different host threads at once, so the text is kept per thread).
std::string& err_text(const dmg_context* c);
// Drops the calling thread's text of a context that is being destroyed.
void err_forget(const dmg_context* c);
// Runs an entry point's body: clears the calling thread's error text, turns an Error or a
// standard exception into its status code and text, so no exception crosses the C ABI.
template <typename F>
dmg_status guarded(dmg_context* c, F&& f) {
  try {
    if (c) err_text(c).clear();
    return f();
  } catch (const Error& e) {
    if (c) err_text(c) = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (c) err_text(c) = "host allocation failed";
    return DMG_E_NOMEM;
  } catch (const std::exception& e) {
    if (c) err_text(c) = e.what();
    return DMG_E_INVALID;
  }
}
// Device memory through the context's allocator hooks, charged against its budget.
void* dev_alloc(dmg_context* c, size_t bytes);
void dev_free(dmg_context* c, void* p, size_t bytes);
}  // namespace dmg

struct dmg_gauge {
  dmg_context* ctx = nullptr;
  int Nx = 0, Nt = 0;
  double2* U64 = nullptr;  // [t][x][mu], fermion sign folded in
  float2* U32 = nullptr;
};
