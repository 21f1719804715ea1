// Machine probes (STREAM triad, FP64 FMA throughput) for the achievable rooflines;
// declared in cosmos_probe.h. Measurement only: the evolution does not call them.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cosmos_probe.h"

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 16;

// Triad over 16-byte pairs: each thread loads kUnroll pairs of each input (strided by
// the workgroup width, so every load instruction is coalesced) before it stores any, so
// that enough loads are in flight per wave.
constexpr int kUnroll = 4;
__global__ __launch_bounds__(kThreads) void k_triad(double2* __restrict__ a, const double2* __restrict__ b,
                                                    const double2* __restrict__ c, double s, size_t npairs) {
  const size_t base = (size_t)blockIdx.x * kThreads * kUnroll + threadIdx.x;
  double2 x[kUnroll], y[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const size_t i = base + (size_t)u * kThreads;
    if (i < npairs) {
      x[u] = b[i];
      y[u] = c[i];
    }
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const size_t i = base + (size_t)u * kThreads;
    if (i < npairs) a[i] = make_double2(x[u].x + s * y[u].x, x[u].y + s * y[u].y);
  }
}

// 16 independent FMA chains per thread: enough independent work per wave to keep the
// FP64 pipeline busy at the occupancy this small register footprint allows.
__global__ __launch_bounds__(kThreads) void k_fma64(double* __restrict__ out, int iters) {
  const size_t t = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const double m = 0.999999940395355, k = 1.0e-7;
  double x[kChains];
#pragma unroll
  for (int r = 0; r < kChains; ++r) x[r] = 1.0 + 1.0e-3 * r + 1.0e-9 * (double)(t & 1023);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < kChains; ++r) x[r] = fma(x[r], m, k);
  }
  double sum = 0.0;
#pragma unroll
  for (int r = 0; r < kChains; ++r) sum += x[r];
  out[t] = sum;
}

bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

extern "C" {

int cosmos_probe_triad(double* a, const double* b, const double* c, double s, size_t n, void* stream) {
  if (!a || !b || !c || n == 0 || (n & 1) || !aligned(a, 16) || !aligned(b, 16) || !aligned(c, 16)) return -1;
  const char *pa = (const char*)a, *pb = (const char*)b, *pc = (const char*)c;
  const size_t nb = n * sizeof(double);
  if ((pa < pb + nb && pb < pa + nb) || (pa < pc + nb && pc < pa + nb)) return -1;
  const size_t npairs = n / 2;
  const size_t blocks = (npairs + (size_t)kThreads * kUnroll - 1) / ((size_t)kThreads * kUnroll);
  if (blocks > 0x7fffffffu) return -1;
  hipLaunchKernelGGL(k_triad, dim3((unsigned)blocks), dim3(kThreads), 0, (hipStream_t)stream, (double2*)a,
                     (const double2*)b, (const double2*)c, s, npairs);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int cosmos_probe_fma64(double* out, size_t nthreads, int iters, void* stream) {
  if (!out || !aligned(out, 8) || nthreads == 0 || nthreads % kThreads || iters <= 0 ||
      nthreads / kThreads > 0x7fffffffu)
    return -1;
  hipLaunchKernelGGL(k_fma64, dim3((unsigned)(nthreads / kThreads)), dim3(kThreads), 0, (hipStream_t)stream, out,
                     iters);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

double cosmos_probe_fma64_flops(size_t nthreads, int iters) {
  return 2.0 * kChains * (double)iters * (double)nthreads;
}

}  // extern "C"
