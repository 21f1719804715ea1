// Massless scalar field (the second matter field of the paper's "Physical
// system settings": stress tensor d phi d phi - 1/2 g (d phi)^2 and wave
// equation box phi = 0), evolved as phi and Pi = n^mu d_mu phi in a separate
// 2-field state (field-major: phi, then Pi). The 3+1 form of box phi = 0:
//   d_t phi = alpha Pi + beta^k d_k phi,
//   d_t Pi  = beta^k d_k Pi + alpha K Pi + alpha chi (gt^ij d_i d_j phi - (Gd^k + gt^kl d_l chi / 2 chi) d_k phi)
//             + chi gt^ij d_i alpha d_j phi,
// Gd^k = gt^ij Gt^k_ij the contracted connection of the conformal metric, formed from its first
// derivatives (the evolved Gt^k enter the system only through their own derivatives, their
// advection and the shift condition), so the operator is the covariant Laplacian of gt_ij / chi,
// plus Kreiss-Oliger dissipation on both fields; its normal-frame densities,
// the sources it adds to the geometry:
//   E = 1/2 (Pi^2 + |D phi|^2), S = 3/2 Pi^2 - 1/2 |D phi|^2, S_j = -Pi d_j phi,
//   S_ij = d_i phi d_j phi - 1/2 (gt_ij / chi) (|D phi|^2 - Pi^2),  |D phi|^2 = chi gt^ij d_i phi d_j phi.
#pragma once
#include "bssn_device.hpp"

namespace cosmos {

// Derivative source of scalar_stage_point reading every stencil tap from global memory. Field q
// of the fixed request order: gt_ij (q = 0..5), chi, alpha, phi, Pi.
struct ScDirect {
  const double* U;
  const double* Sc;
  size_t fs;
  const Nbr& nb;
  const DevParams& P;
  __device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }
  template <bool SECOND, bool ADV, bool KO>
  __device__ __forceinline__ void get(int q, const double beta[3], FieldDerivs& d) {
    // a compiler-level fence per field: the stencil loads of later fields stay after it
    asm volatile("" ::: "memory");
    const double* F = q < 6 ? U + (size_t)(F_GT + q) * fs
                            : (q == 6 ? U + (size_t)F_CHI * fs : (q == 7 ? U + (size_t)F_ALP * fs : Sc + (size_t)(q - 8) * fs));
    field_derivs<SECOND, ADV, KO>(F, nb, P, beta, d);
  }
};

// One RK4 stage of the scalar field at the grid point with linear index c from the stage state
// (U, Sc); also writes the geometry's source arrays `src` (kScalarSrc x fs doubles, layout of
// DevParams::xsrc) for the stage kernel that follows. MODE as the stage kernel's epilogue:
// 0 sout = f; 1 sacc = Sc + ca f, sout = Sc + cn f; 2 sacc += ca f, sout = sun + cn f;
// 3 sout = sacc + ca f. Der supplies the fields' derivatives in the order gt_ij (6, first), chi
// and alpha (first), phi (second, with shift advection and dissipation), Pi (first, with
// advection and dissipation); der.pin(x) keeps a running value in a register where it is final
// for the current field (it changes no value). Nothing is stored unless `active`.
template <int MODE, class Der>
__device__ __forceinline__ void scalar_stage_point(const double* __restrict__ U, const double* __restrict__ Sc,
                                                   double* __restrict__ src, const double* __restrict__ sun,
                                                   double* __restrict__ sacc, double* __restrict__ sout, size_t fs,
                                                   const DevParams& P, int c, bool active, Der& der, double ca,
                                                   double cn) {
  const size_t p = (size_t)c;
  const double chi = ldq(U + F_CHI * fs, c), K = ldq(U + F_K * fs, c), alpha = ldq(U + F_ALP * fs, c);
  double gt[6], gi[6], beta[3];
#pragma unroll
  for (int s = 0; s < 6; ++s) gt[s] = ldq(U + (F_GT + s) * fs, c);
#pragma unroll
  for (int a = 0; a < 3; ++a) beta[a] = ldq(U + (F_BET + a) * fs, c);
  inv_sym(gt, gi);
  const double nob[3] = {0.0, 0.0, 0.0};
  // Contracted connection Gd^k = gt^ij Gt^k_ij = gt^kl (A_l - B_l / 2), A_l = gt^xy d_x gt_ly,
  // B_l = gt^xy d_l gt_xy, accumulated one metric component at a time (the 18 first
  // derivatives are never live together): component ab with derivative d_c adds
  // gt^cb d_c gt_ab to A_a (and gt^ca d_c gt_ab to A_b if a != b) and w gt^ab d_c gt_ab to B_c
  // (w = 2 off the diagonal).
  double Gd[3];
  {
    double A[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      FieldDerivs d;
      der.template get<false, false, false>(q, nob, d);
      const int a = SI(q), b = SJ(q);
      const double w = (a == b) ? 1.0 : 2.0;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        A[a] += gi[S(cc, b)] * d.d1[cc];
        if (a != b) A[b] += gi[S(cc, a)] * d.d1[cc];
        B[cc] += w * gi[q] * d.d1[cc];
      }
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        der.pin(A[cc]);
        der.pin(B[cc]);
      }
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) A[l] -= 0.5 * B[l];
#pragma unroll
    for (int k = 0; k < 3; ++k) Gd[k] = gi[S(k, 0)] * A[0] + gi[S(k, 1)] * A[1] + gi[S(k, 2)] * A[2];
  }
  double dchi[3], dal[3];
  {
    FieldDerivs d;
    der.template get<false, false, false>(6, nob, d);
#pragma unroll
    for (int a = 0; a < 3; ++a) dchi[a] = d.d1[a];
    der.template get<false, false, false>(7, nob, d);
#pragma unroll
    for (int a = 0; a < 3; ++a) dal[a] = d.d1[a];
  }
  FieldDerivs dphi;
  der.template get<true, true, true>(8, beta, dphi);  // d1, d2, upwind advection + KO of phi
  double advko_pi;
  {
    FieldDerivs d;
    der.template get<false, true, true>(9, beta, d);  // upwind advection + KO of Pi
    advko_pi = d.advko;
  }
  const double Pi = ldq(Sc + fs, c);

  // sources of the geometry
  double dd[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) dd[s] = dphi.d1[SI(s)] * dphi.d1[SJ(s)];
  const double g2 = chi * contract_sym(gi, dd);
  const double P2 = Pi * Pi;
  const double E = 0.5 * (P2 + g2);
  const double Str = 1.5 * P2 - 0.5 * g2;
  const double ichi = 1.0 / chi;
  if (active) {
    stq(src + SRC_EPS * fs, c, E + Str);
    stq(src + SRC_E * fs, c, E);
#pragma unroll
    for (int a = 0; a < 3; ++a) stq(src + (SRC_S + a) * fs, c, -Pi * dphi.d1[a]);
#pragma unroll
    for (int s = 0; s < 6; ++s) stq(src + (SRC_SIJ + s) * fs, c, dd[s] - 0.5 * (gt[s] * ichi) * (g2 - P2));
  }

  // right-hand side of (phi, Pi)
  double lap = contract_sym(gi, dphi.d2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double gk = Gd[a] + (gi[S(a, 0)] * dchi[0] + gi[S(a, 1)] * dchi[1] + gi[S(a, 2)] * dchi[2]) * (0.5 * ichi);
    lap -= gk * dphi.d1[a];
  }
  double dad = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    dad += dal[a] * (gi[S(a, 0)] * dphi.d1[0] + gi[S(a, 1)] * dphi.d1[1] + gi[S(a, 2)] * dphi.d1[2]);
  const double r[2] = {alpha * Pi + dphi.advko, ((alpha * K * Pi + alpha * chi * lap) + chi * dad) + advko_pi};
  if (!active) return;
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const size_t q = (size_t)f * fs + p;
    if constexpr (MODE == 0) {
      sout[q] = r[f];
    } else if constexpr (MODE == 1) {
      const double s0 = Sc[q];
      sacc[q] = s0 + ca * r[f];
      sout[q] = s0 + cn * r[f];
    } else if constexpr (MODE == 2) {
      sacc[q] = sacc[q] + ca * r[f];
      sout[q] = sun[q] + cn * r[f];
    } else {
      sout[q] = sacc[q] + ca * r[f];
    }
  }
}

// The same at grid point (i, j, k) with direct loads (the batched form and grids the LDS-staged
// kernel does not take).
template <int MODE>
__device__ __forceinline__ void scalar_point(const double* __restrict__ U, const double* __restrict__ Sc,
                                             double* __restrict__ src, const double* __restrict__ sun,
                                             double* __restrict__ sacc, double* __restrict__ sout, size_t fs,
                                             const DevParams& P, int i, int j, int k, double ca, double cn) {
  const int c = i + P.n[0] * (j + P.n[1] * k);
  Nbr nb;
  make_nbr(nb, i, j, k, P.n);
  ScDirect der{U, Sc, fs, nb, P};
  scalar_stage_point<MODE>(U, Sc, src, sun, sacc, sout, fs, P, c, true, der, ca, cn);
}

// The scalar stage of one grid: one thread per point of a 16x4x4 brick (bricks in XCD
// slabs, so the stencil halos of neighbouring bricks meet in one L2). The compiler's own
// register choice (2 waves per SIMD, no spills) is kept: a cap at 3 or 4 waves spills.
template <int MODE>
__global__ __launch_bounds__(256) void k_scalar_stage(
    const double* __restrict__ U, const double* __restrict__ Sc, double* __restrict__ src,
    const double* __restrict__ sun, double* __restrict__ sacc, double* __restrict__ sout, size_t fs, DevParams P,
    Tile T, double ca, double cn) {
  int i, j, k;
  if (!tile_point(T, P.n, i, j, k)) return;
  scalar_point<MODE>(U, Sc, src, sun, sacc, sout, fs, P, i, j, k, ca, cn);
}

}  // namespace cosmos
