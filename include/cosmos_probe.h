/* Machine probes for the rooflines the evolution kernels are measured against: the
 * achievable HBM bandwidth of a STREAM triad and the achievable FP64 vector FMA rate
 * of the device. Measurement only: no entry point of cosmos.h calls them, and they
 * compute nothing of the method. Separate library: libcosmos_probe.so.
 *
 * Return codes are those of cosmos.h (0 = COSMOS_OK, -1 = COSMOS_EINVAL for invalid
 * arguments, detected on the host before any launch, -2 = COSMOS_EHIP for a failed
 * launch). Device pointers are caller-owned; `stream` is a hipStream_t (NULL = the
 * default stream); every call is asynchronous on that stream.
 */
#ifndef COSMOS_PROBE_H
#define COSMOS_PROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* a[i] = b[i] + s * c[i] for i < n (FP64, one multiply-add per element). a, b, c: device
 * arrays of n doubles, 16-byte aligned, n even and > 0; a must not overlap b or c. Moves
 * 24 n bytes (two reads and one write per element). */
int cosmos_probe_triad(double* a, const double* b, const double* c, double s, size_t n, void* stream);

/* FP64 FMA throughput: `nthreads` threads (a multiple of 256, > 0) each run `iters` (> 0)
 * rounds of 16 independent fused multiply-add chains, x <- x * m + k, and write the sum of
 * their 16 values to out[thread] (device, nthreads doubles, 8-byte aligned) so that no
 * chain is dead code. FP64 operations = cosmos_probe_fma64_flops(nthreads, iters). */
int cosmos_probe_fma64(double* out, size_t nthreads, int iters, void* stream);
double cosmos_probe_fma64_flops(size_t nthreads, int iters);

#ifdef __cplusplus
}
#endif

#endif
