// sq_devfn.h -- device helpers and launcher declarations shared by the
// gfx950 kernel units of the infinite-cell Clenshaw-Curtis SQ hot path
// (arXiv 2006.03697, Sec. IV and App. A): sq_recur.hip (the recurrence
// kernels, one unit per cube width) and sq_misc.hip (width-independent
// kernels and the dispatch over widths).
#pragma once
#include "sq_dev.h"

#include <float.h>
#include <math.h>

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
  hipError_t sq_launch_lanczos_##N(int kc, bool fused, const PlanDev& P, const long long* items, \
                                   const int* ic, long long n, hipStream_t s);                \
  hipError_t sq_launch_moments_##N(bool fp64, int kc, bool fused, const PlanDev& P,            \
                                   const long long* items, const int* ic, long long n,        \
                                   hipStream_t s);                                            \
  hipError_t sq_launch_stress_##N(bool fp64, int kc, bool fused, const PlanDev& P,             \
                                  const long long* items, const int* ic, long long n,         \
                                  hipStream_t s);                                             \
  hipError_t sq_launch_gram_##N(int kc, const PlanDev& P, const long long* items, const int* ic, \
                                long long n, hipStream_t s);                                  \
  hipError_t sq_launch_census_##N(const PlanDev& P, const long long* items, const int* ic,     \
                                  long long n, int* stats, long long* pairs, hipStream_t s);
SQ_NC_LIST(SQ_DECL_NC)

// Largest slot capacity per precision and width (0: unsupported).
__host__ __device__ constexpr int sq_kc_max(bool, int) { return 48; }

// Largest number of atom images one cube may see (the image index shares a
// 32-bit slot word with the chord bits of the NC planes).
__host__ __device__ constexpr int sq_img_max(int nc) { return (1 << (32 - nc)) < 160 ? (1 << (32 - nc)) : 160; }
