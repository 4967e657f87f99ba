// sq_probe.hip -- measured peaks for the rooflines of the SQ kernels on
// gfx950: LDS read bandwidth of conflict-free ds_read of 4, 8 and 16 bytes
// per lane.  The recurrence kernels are bound by the LDS reads of the x/y
// stencil neighbours and by the vector ALU, so their LDS fraction is taken
// against this measured rate rather than a nominal one.
#include <hip/hip_runtime.h>

#include "sq_probe.h"

namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_WORDS = 8192;   // 32-bit words of LDS per workgroup (32 KB)

using u64 = unsigned long long;
template <int W>
struct Vec;
template <>
struct Vec<4> {
  using T = unsigned;
  __device__ static u64 fold(u64 a, T v) { return a + v; }
};
template <>
struct Vec<8> {
  using T = u64;
  __device__ static u64 fold(u64 a, T v) { return a + v; }
};
template <>
struct Vec<16> {
  using T = ulonglong2;
  __device__ static u64 fold(u64 a, T v) { return a + (v.x ^ v.y); }
};

// Every lane reads W bytes per access; lane l of a wave reads element
// (base + l) so a wave's access covers 64 consecutive elements (distinct
// banks for every 128 bytes): conflict-free.  Eight independent 64-bit
// accumulators keep eight reads in flight per lane; each read is folded in
// with one 64-bit integer add (gfx950 has a single-instruction 64-bit add),
// so the vector ALU work stays below the LDS time.
template <int W>
__global__ void __launch_bounds__(PROBE_THREADS) k_lds_read(int iters, unsigned* sink) {
  using T = typename Vec<W>::T;
  constexpr int N = PROBE_WORDS * 4 / W;   // elements of T in the buffer
  static_assert((N & (N - 1)) == 0, "power of two");
  __shared__ T buf[N];
  unsigned* w = reinterpret_cast<unsigned*>(buf);
  for (int i = threadIdx.x; i < PROBE_WORDS; i += PROBE_THREADS) w[i] = (unsigned)i * 2654435761u;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  u64 acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int base = wave * 64 * 8;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = Vec<W>::fold(acc[u], buf[(base + u * 64 + lane) & (N - 1)]);
    base += 8 * 64;
  }
  u64 r = 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) r ^= acc[u];
  if (r == 0x9e3779b97f4a7c15ull) sink[0] = (unsigned)r;   // keeps the reads live; practically never taken
}

template <int W>
hipError_t run(int blocks, int iters, unsigned* sink, hipStream_t s, float* ms) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  // one warm-up launch, then the timed one
  hipLaunchKernelGGL(k_lds_read<W>, dim3(blocks), dim3(PROBE_THREADS), 0, s, iters, sink);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_lds_read<W>, dim3(blocks), dim3(PROBE_THREADS), 0, s, iters, sink);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

extern "C" int sq_probe_lds(int bytes_per_lane, void* hip_stream, double* tb_per_s,
                            double* bytes_per_clk_per_cu) {
  if (!tb_per_s || (bytes_per_lane != 4 && bytes_per_lane != 8 && bytes_per_lane != 16)) return 1;
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 3;
  const int cus = prop.multiProcessorCount;
  // 8 workgroups of 4 waves per CU (32 KB of LDS each), 4096 iterations of
  // 8 reads per lane
  const int blocks = cus * 8, iters = 4096;
  unsigned* sink = nullptr;
  if (hipMalloc(&sink, sizeof(unsigned)) != hipSuccess) return 2;
  float ms = 0.f;
  hipError_t e = bytes_per_lane == 4 ? run<4>(blocks, iters, sink, s, &ms)
                 : bytes_per_lane == 8 ? run<8>(blocks, iters, sink, s, &ms)
                                       : run<16>(blocks, iters, sink, s, &ms);
  (void)hipFree(sink);
  if (e != hipSuccess || !(ms > 0.f)) return 3;
  const double bytes = (double)blocks * PROBE_THREADS * iters * 8.0 * bytes_per_lane;
  *tb_per_s = bytes / (ms * 1e-3) / 1e12;
  if (bytes_per_clk_per_cu) {
    // clockRate is the peak shader clock in kHz
    const double clk = (double)prop.clockRate * 1e3;
    *bytes_per_clk_per_cu = clk > 0 ? bytes / (ms * 1e-3) / clk / cus : 0.0;
  }
  return 0;
}
