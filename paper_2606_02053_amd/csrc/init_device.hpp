// Initial data on the device (paper, "Physical system settings", initial-data
// paragraph): leading-order long-wavelength growing mode of a curvature
// perturbation zeta(x) on the radiation FLRW background. gamma_ij =
// e^{2 zeta} delta_ij (chi = e^{-2 zeta}, gt = delta), K = -3 H0, At = 0,
// Gt = 0, alpha = 1, beta = 0, fluid at rest, and the energy density fixed by
// the Hamiltonian constraint, E = (R + 2/3 K^2) / 16 pi with
// R = -e^{-2 zeta} (4 lap zeta + 2 |grad zeta|^2) -- no elliptic solve.
//
// The same kernel also gives d u0 / d mu and d u0 / d sigma: it evaluates the
// closed form on value-tangent pairs (Tan) seeded in the chosen parameter.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bssn_device.hpp"

namespace cosmos {

struct InitArgs {
  int n[3];
  double L[3], h[3];
  double H0;
  double mu, sigma, center[3], noise;
  uint64_t seed;
  int profile, density_mode;
  double sc_mu, sc_sigma;  // iso-curvature mode of the scalar field (sc_mu = 0: none)
};

inline InitArgs make_init_args(const cosmos_grid* g, const cosmos_params* p, const cosmos_init* in) {
  InitArgs a;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = g->n[d];
    a.L[d] = g->L[d];
    a.h[d] = g->L[d] / g->n[d];
    a.center[d] = in->center[d];
  }
  a.H0 = p->H0;
  a.mu = in->mu;
  a.sigma = in->sigma;
  a.noise = in->noise_amp;
  a.seed = in->seed;
  a.profile = in->profile;
  a.density_mode = in->density_mode;
  a.sc_mu = 0.0;
  a.sc_sigma = 1.0;
  return a;
}

// value + tangent
struct Tan {
  double v, d;
};
__device__ __forceinline__ Tan operator+(Tan a, Tan b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Tan operator-(Tan a, Tan b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Tan operator*(Tan a, Tan b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Tan operator*(double s, Tan a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Tan operator/(Tan a, Tan b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Tan texp(Tan a) {
  const double e = exp(a.v);
  return {e, e * a.d};
}
__device__ __forceinline__ Tan tsqrt(Tan a) {
  const double r = sqrt(a.v);
  return {r, a.d / (2.0 * r)};
}
__device__ __forceinline__ Tan tc(double x) { return {x, 0.0}; }

// SplitMix64 (Steele, Lea & Flood 2014) used as a counter-based generator:
// the (p+1)-th output of the sequence started from `seed`.
__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t p) {
  uint64_t z = seed + (p + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// which = -1: write the initial data; 0 / 1: write its derivative in mu / sigma.
// Profile f = mu * shape(x) (x relative to the centre): value, Laplacian and
// |grad f|^2 in closed form. 0: Gaussian mu exp(-r^2 / 2 sigma^2); 1: single mode
// mu sin(2 pi x / L_x); 2: Gaussian in s_a = (L_a / pi) sin(pi x_a / L_a).
__device__ __forceinline__ void profile_tan(const InitArgs& a, int profile, Tan mu, Tan sg, const double x[3], Tan& val,
                                            Tan& lap, Tan& grad2) {
  if (profile == 0) {  // Gaussian
    const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    const Tan s2 = sg * sg;
    val = mu * texp(tc(-r2) / (2.0 * s2));
    lap = val * (tc(r2) / (s2 * s2) - tc(3.0) / s2);
    grad2 = val * val * tc(r2) / (s2 * s2);
  } else if (profile == 1) {  // single sinusoidal mode along x
    const double kx = 2.0 * PI_D / a.L[0];
    const double sn = sin(kx * x[0]), cs = cos(kx * x[0]);
    val = mu * tc(sn);
    lap = tc(-kx * kx) * val;
    grad2 = mu * mu * tc(kx * kx * cs * cs);
  } else {  // Gaussian in s_a = (L_a / pi) sin(pi x_a / L_a)
    const Tan s2 = sg * sg;
    double sa[3], ca[3], kk[3], q2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      kk[d] = PI_D / a.L[d];
      sa[d] = sin(kk[d] * x[d]) / kk[d];
      ca[d] = cos(kk[d] * x[d]);
      q2 += sa[d] * sa[d];
    }
    val = mu * texp(tc(-q2) / (2.0 * s2));
    Tan l = tc(0.0), gg = tc(0.0);
    for (int d = 0; d < 3; ++d) {
      // d_a f = -f s c / sigma^2;  d_a^2 f = f (s c)^2 / sigma^4 - f (c^2 - k^2 s^2) / sigma^2
      const double sc = sa[d] * ca[d];
      l = l + val * tc(sc * sc) / (s2 * s2) - val * tc(ca[d] * ca[d] - kk[d] * kk[d] * sa[d] * sa[d]) / s2;
      gg = gg + val * val * tc(sc * sc) / (s2 * s2);
    }
    lap = l;
    grad2 = gg;
  }
}

// Initial data at point p: out[NF] receives the state (which = -1) or its derivative with
// respect to mu / sigma (which = 0 / 1), ups the scalar field's iso-curvature mode (or its
// derivative). With a scalar field (a.sc_mu != 0) the mode Upsilon = sc_mu * profile(sc_sigma)
// sets phi = Upsilon, Pi = 0, and the fluid takes the rest of the Hamiltonian constraint's
// energy: E_fluid = E - 1/2 chi |grad Upsilon|^2.
__device__ __forceinline__ void init_point(const InitArgs& a, size_t p, int which, double out[NF], double& ups_out) {
  const int i = (int)(p % a.n[0]);
  const int j = (int)((p / a.n[0]) % a.n[1]);
  const int k = (int)(p / ((size_t)a.n[0] * a.n[1]));
  const double x[3] = {-0.5 * a.L[0] + i * a.h[0] - a.center[0], -0.5 * a.L[1] + j * a.h[1] - a.center[1],
                       -0.5 * a.L[2] + k * a.h[2] - a.center[2]};
  const Tan mu = {a.mu, which == 0 ? 1.0 : 0.0};
  const Tan sg = {a.sigma, which == 1 ? 1.0 : 0.0};
  Tan zeta, lap, grad2;
  profile_tan(a, a.profile, mu, sg, x, zeta, lap, grad2);
  const Tan chi = texp(-2.0 * zeta);
  const Tan R = tc(0.0) - chi * (4.0 * lap + 2.0 * grad2);
  const double K = -3.0 * a.H0;
  Tan E = (a.density_mode == 0) ? (R + tc((2.0 / 3.0) * K * K)) / tc(16.0 * PI_D)
                                : tc(3.0 * a.H0 * a.H0 / (8.0 * PI_D));
  Tan ups = tc(0.0);
  if (a.sc_mu != 0.0) {
    Tan ulap, ug2;
    profile_tan(a, a.profile, tc(a.sc_mu), tc(a.sc_sigma), x, ups, ulap, ug2);
    if (a.density_mode == 0) E = E - (0.5 * chi) * ug2;
  }
  if (a.noise != 0.0) {
    const double xi = 2.0 * ((double)(sm64(a.seed, p) >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
    E = E * tc(1.0 + a.noise * xi);
  }
  const Tan Et = E / (chi * tsqrt(chi));
  const bool tangent = which >= 0;
  for (int f = 0; f < NF; ++f) out[f] = 0.0;
  out[F_CHI] = tangent ? chi.d : chi.v;
  out[F_K] = tangent ? 0.0 : K;
  out[F_ALP] = tangent ? 0.0 : 1.0;
  if (!tangent) out[F_GT + 0] = out[F_GT + 3] = out[F_GT + 5] = 1.0;
  out[F_ET] = tangent ? Et.d : Et.v;
  ups_out = tangent ? ups.d : ups.v;
}

// which = -1: the state; 0 / 1: its derivative with respect to mu / sigma (and the
// scalar field's initial data when sc is non-null).
__global__ __launch_bounds__(256) void k_init(InitArgs a, double* __restrict__ u, int which,
                                              double* __restrict__ sc) {
  const size_t N3 = (size_t)a.n[0] * a.n[1] * a.n[2];
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= N3) return;
  double out[NF], ups;
  init_point(a, p, which, out, ups);
  for (int f = 0; f < NF; ++f) u[(size_t)f * N3 + p] = out[f];
  if (sc) {
    sc[p] = ups;
    sc[N3 + p] = 0.0;
  }
}

// Sum of (v0, v1) over the 256 threads of a workgroup in a fixed order: a butterfly
// within each wavefront (the same partner pattern every time), then the four wave
// results in wave order. The result is valid in thread 0. `red` holds 8 doubles of LDS.
__device__ __forceinline__ void block_sum2(double& v0, double& v1, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    v0 += __shfl_xor(v0, o);
    v1 += __shfl_xor(v1, o);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[2 * wv] = v0;
    red[2 * wv + 1] = v1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    v0 = ((red[0] + red[2]) + red[4]) + red[6];
    v1 = ((red[1] + red[3]) + red[5]) + red[7];
  }
}

// Gradient of an objective J(u_0(mu, sigma)) from its adjoint lam = dJ/du_0:
// part[2 b + w] = sum over the points of workgroup b of sum_f lam[f] d u_0[f] / d theta_w,
// theta = (mu, sigma), with the initial-data tangent formed at the point (the fields whose
// tangent is not identically zero: chi and Et). Workgroup b takes points b*256 + t +
// m * gridDim.x * 256; k_sum_partials2 folds the partials in workgroup order.
__global__ __launch_bounds__(256) void k_adjoint_gradient(InitArgs a, const double* __restrict__ lam,
                                                          double* __restrict__ part) {
  __shared__ double red[8];
  const size_t N3 = (size_t)a.n[0] * a.n[1] * a.n[2];
  double g0 = 0.0, g1 = 0.0;
  for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N3; p += (size_t)gridDim.x * 256) {
    const double lchi = lam[(size_t)F_CHI * N3 + p], let = lam[(size_t)F_ET * N3 + p];
    double out[NF], ups;
    init_point(a, p, 0, out, ups);
    g0 += lchi * out[F_CHI] + let * out[F_ET];
    init_point(a, p, 1, out, ups);
    g1 += lchi * out[F_CHI] + let * out[F_ET];
  }
  block_sum2(g0, g1, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = g0;
    part[2 * blockIdx.x + 1] = g1;
  }
}

// out[0..1] = sum over b < nparts of part[2 b + 0..1], in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_sum_partials2(const double* __restrict__ part, int nparts,
                                                       double* __restrict__ out) {
  __shared__ double red[8];
  double v0 = 0.0, v1 = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256) {
    v0 += part[2 * b];
    v1 += part[2 * b + 1];
  }
  block_sum2(v0, v1, red);
  if (threadIdx.x == 0) {
    out[0] = v0;
    out[1] = v1;
  }
}
}  // namespace cosmos
