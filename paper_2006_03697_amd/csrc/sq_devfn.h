// sq_devfn.h -- device helpers and launcher declarations shared by the
// gfx950 kernel units of the infinite-cell Clenshaw-Curtis SQ hot path
// (arXiv 2006.03697, Sec. IV and App. A): sq_recur.hip (the recurrence
// kernels, one unit per cube width) and sq_misc.hip (width-independent
// kernels and the dispatch over widths).
#pragma once
#include "sq_dev.h"

#include <float.h>
#include <math.h>

#include <utility>

namespace {

// ---------------------------------------------------------------------------
// geometry helpers: the same IEEE operations as the oracle, no contraction
// ---------------------------------------------------------------------------

__device__ __forceinline__ double node_coord(long long i, double h, double R) {
#pragma clang fp contract(off)
  return (double)i * h - R;
}

__device__ __forceinline__ double sq_sum2(double a, double b) {
#pragma clang fp contract(off)
  return a * a + b * b;
}

__device__ __forceinline__ double sq_add(double s, double c) {
#pragma clang fp contract(off)
  return s + c * c;
}

__device__ __forceinline__ long long wrapll(long long i, long long n) {
  long long r = i % n;
  return r < 0 ? r + n : r;
}

// f(std::integral_constant<int, k>) for k = 0 .. N - 1, expanded in the
// front end: a loop of large bodies indexed into register arrays stays
// unrolled whatever the unroller's size limits.
template <class F, int... K>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, K...>) {
  (f(std::integral_constant<int, K>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// The projector-slot loop: expanded in the front end up to 16 slots; wider
// variants keep an unrolled loop (fully expanded, their register allocation
// measured worse).
template <int N, class F>
__device__ __forceinline__ void slot_for(F&& f) {
  if constexpr (N <= 16) {
    static_for<N>(f);
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) f(k);
  }
}

// Make a register value opaque to the optimiser (no hoisting of values
// derived from it); 64-bit values go through their two 32-bit halves.
#ifdef SQ_NO_OPAQUE
template <typename U>
__device__ __forceinline__ void opaque(U&) {}
#else
__device__ __forceinline__ void opaque(int& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void opaque(unsigned& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void opaque(float& x) {
  unsigned u = __float_as_uint(x);
  asm volatile("" : "+v"(u));
  x = __uint_as_float(u);
}
__device__ __forceinline__ void opaque(double& x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  asm volatile("" : "+v"(lo), "+v"(hi));
  x = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
#endif

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------------------
// Deterministic sums of FP64 terms: each term x is split into two integers,
// x = hi 2^-30 + lo 2^-80 (hi = x 2^30 rounded to an integer, lo = the
// remainder 2^50 rounded), and the integers are added with 64-bit integer
// atomics.  Integer addition is associative, so the sum does not depend on
// the order in which the terms arrive: a result is the same bit for bit on
// every run and in every batch.  Each term is rounded to 2^-81 (absolute);
// |x| < 2^20 is required (checked by the caller), and up to 2^13 terms of
// that size fit the integer range.  The rounding to integers uses the
// 1.5 2^52 shift: for |y| < 2^51, y + 1.5 2^52 carries y rounded to the
// nearest integer in its low mantissa bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long fx_round_bits(double y, double& yr) {
#pragma clang fp contract(off)
  const double M = 6755399441055744.0;   // 1.5 * 2^52
  const double t = y + M;
  yr = t - M;
  return (long long)(__double_as_longlong(t) - __double_as_longlong(M));
}

__device__ __forceinline__ void fx_split(double x, long long& hi, long long& lo) {
#pragma clang fp contract(off)
  const double xs = x * 0x1p30;
  double hr;
  hi = fx_round_bits(xs, hr);
  const double rem = xs - hr;              // exact, |rem| <= 1/2
  double lr;
  lo = fx_round_bits(rem * 0x1p50, lr);
}

__device__ __forceinline__ double fx_join(long long hi, long long lo) {
  return (double)hi * 0x1p-30 + (double)lo * 0x1p-80;
}

// Adds x to the two-word accumulator p[0..1] (LDS), without branches; a
// term with |x| >= 2^20 (or not a number) is replaced by zero and sets bad.
__device__ __forceinline__ void fx_add(unsigned long long* p, double x, bool& bad) {
  const bool ok = fabs(x) < 0x1p20;
  bad = bad || !ok;
  long long hi, lo;
  fx_split(ok ? x : 0.0, hi, lo);
  atomicAdd(&p[0], (unsigned long long)hi);
  atomicAdd(&p[1], (unsigned long long)lo);
}

__device__ __forceinline__ double fx_load(const unsigned long long* p) {
  return fx_join((long long)p[0], (long long)p[1]);
}

__device__ __forceinline__ int quad_points(double zeta, double kT, int npl) {
  double t = ceil(8.0 * zeta / kT);
  double tgt = fmax((double)(4 * (npl + 2)), t);
  int M = 1;
  while ((double)M < tgt) M <<= 1;
  return M;
}

}  // namespace

// ---------------------------------------------------------------------------
// Per-width launchers.  sq_recur.hip is compiled once per cube width
// (SQ_ONE_NC), so that the widths build in parallel; within a width the
// variant is picked from the slot capacity kc the cell needs (largest number
// of atom images crossing one z-column of a cube, measured at set-up).
// ---------------------------------------------------------------------------
#define SQ_NC_LIST(X) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25)

#define SQ_DECL_NC(N)                                                                          \
  hipError_t sq_launch_lanczos_##N(const RecLaunch& R, const PlanDev& P, const long long* items, \
                                   const int* ic, long long n, hipStream_t s);                \
  hipError_t sq_launch_moments_##N(const RecLaunch& R, bool fp64, const PlanDev& P,            \
                                   const long long* items, const int* ic, long long n,        \
                                   hipStream_t s);                                            \
  hipError_t sq_launch_stress_##N(const RecLaunch& R, bool fp64, const PlanDev& P,             \
                                  const long long* items, const int* ic, long long n,         \
                                  hipStream_t s);                                             \
  hipError_t sq_launch_gram_##N(const PlanDev& P, const long long* items, const int* ic,       \
                                long long n, hipStream_t s);                                  \
  hipError_t sq_launch_census_##N(const PlanDev& P, const long long* items, const int* ic,     \
                                  long long n, int* stats, long long* pairs, hipStream_t s);
SQ_NC_LIST(SQ_DECL_NC)

__host__ __device__ constexpr int sq_threads(int nc) { return ((nc * nc + 63) / 64) * 64; }

// Slot capacities compiled per single-sweep form: the smallest that holds
// kc (16 and 24: plane-0 weights kept in registers; 48: recomputed);
// two-sweep nodes: 48.  0: none.
__host__ __device__ constexpr int sq_kc_pick(bool fused, int kc) {
  return !fused ? (kc <= 48 ? 48 : 0) : (kc <= 16 ? 16 : (kc <= 24 ? 24 : (kc <= 48 ? 48 : 0)));
}

// Largest number of atom images one cube may see (the image index shares a
// 32-bit slot word with the chord bits of the planes of one thread).
__host__ __device__ constexpr int sq_img_max(int nc) { return (1 << (32 - nc)) < 160 ? (1 << (32 - nc)) : 160; }

// Gram entries a node may store for the single-sweep form: at most four
// per thread of the workgroup (each thread adds up to four Gram terms per
// step), and at most SQ_GRAM_MAX.
__host__ __device__ constexpr int sq_gram_cap(int nc) {
  return 4 * sq_threads(nc) < SQ_GRAM_MAX ? 4 * sq_threads(nc) : SQ_GRAM_MAX;
}
