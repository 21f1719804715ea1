// Hand-written reverse mode of the pointwise part of the right-hand side (and
// of the fluid fluxes), for the discrete adjoint of the RK4 step.
//
// pt_vjp forms the cotangents of every input of the pointwise algebra at one
// point -- point values, first and second finite differences -- from the
// cotangents of the 25 outputs: the same equations as the stage kernel
// (conformal connection and Ricci tensor, second covariant derivative of the
// lapse, perfect-fluid recovery and projections, the BSSN and fluid source
// terms) without the advection, dissipation and flux-divergence stencils.
// flux_forward / flux_reverse do the same for the fluxes of the densitised fluid
// variables along one axis. The building blocks (inverse metric, fluid recovery)
// come as forward/reverse pairs: dy = a dx gives xbar += a ybar. Branches
// (recovery clamps) are taken exactly as in the forward evaluation, so this is
// the derivative of the discrete map.
//
// __host__ __device__ so that the algebra can also be checked on the CPU.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "bssn_device.hpp"

namespace cosmos {

__host__ __device__ inline double wsym(int s) { return (s == 0 || s == 3 || s == 5) ? 1.0 : 2.0; }

// ---------------------------------------------------------------- inverse metric
struct InvTape {
  double c[6], det, id, gi[6];
};
__host__ __device__ inline void inv_forward(const double g[6], InvTape& T) {
  T.c[0] = g[3] * g[5] - g[4] * g[4];
  T.c[1] = g[2] * g[4] - g[1] * g[5];
  T.c[2] = g[1] * g[4] - g[2] * g[3];
  T.c[3] = g[0] * g[5] - g[2] * g[2];
  T.c[4] = g[1] * g[2] - g[0] * g[4];
  T.c[5] = g[0] * g[3] - g[1] * g[1];
  T.det = g[0] * T.c[0] + g[1] * T.c[1] + g[2] * T.c[2];
  T.id = 1.0 / T.det;
  for (int s = 0; s < 6; ++s) T.gi[s] = T.c[s] * T.id;
}
__host__ __device__ inline void inv_reverse(const double g[6], const InvTape& T, const double gib[6], double gb[6]) {
  double cb[6], idb = 0.0;
  for (int s = 0; s < 6; ++s) {
    cb[s] = gib[s] * T.id;
    idb += gib[s] * T.c[s];
  }
  const double detb = -idb * T.id * T.id;
  gb[0] += detb * T.c[0];
  gb[1] += detb * T.c[1];
  gb[2] += detb * T.c[2];
  cb[0] += detb * g[0];
  cb[1] += detb * g[1];
  cb[2] += detb * g[2];
  gb[3] += cb[0] * g[5];
  gb[5] += cb[0] * g[3];
  gb[4] -= 2.0 * cb[0] * g[4];
  gb[2] += cb[1] * g[4];
  gb[4] += cb[1] * g[2];
  gb[1] -= cb[1] * g[5];
  gb[5] -= cb[1] * g[1];
  gb[1] += cb[2] * g[4];
  gb[4] += cb[2] * g[1];
  gb[2] -= cb[2] * g[3];
  gb[3] -= cb[2] * g[2];
  gb[0] += cb[3] * g[5];
  gb[5] += cb[3] * g[0];
  gb[2] -= 2.0 * cb[3] * g[2];
  gb[1] += cb[4] * g[2];
  gb[2] += cb[4] * g[1];
  gb[0] -= cb[4] * g[4];
  gb[4] -= cb[4] * g[0];
  gb[0] += cb[5] * g[3];
  gb[3] += cb[5] * g[0];
  gb[1] -= 2.0 * cb[5] * g[1];
}

// ---------------------------------------------------------------- fluid recovery
struct RecTape {
  double sq, c32, E, S[3], Sup[3], S2, disc, sd, X, P, invX;
  bool Eok, dok;
};
__host__ __device__ inline bool rec_forward(double w, double chi, const double gi[6], double Et, const double St[3],
                                            RecTape& R) {
  R.sq = sqrt(chi);
  R.c32 = chi * R.sq;
  R.E = R.c32 * Et;
  for (int i = 0; i < 3; ++i) R.S[i] = R.c32 * St[i];
  for (int j = 0; j < 3; ++j) R.Sup[j] = chi * (gi[S(j, 0)] * R.S[0] + gi[S(j, 1)] * R.S[1] + gi[S(j, 2)] * R.S[2]);
  R.S2 = R.Sup[0] * R.S[0] + R.Sup[1] * R.S[1] + R.Sup[2] * R.S[2];
  R.Eok = R.E > 0.0;
  R.dok = true;
  if (!R.Eok) {
    R.P = 0.0;
    R.invX = 0.0;
    return true;
  }
  const double opw = 1.0 + w;
  R.disc = (opw * R.E) * (opw * R.E) - 4.0 * w * R.S2;
  if (!(R.disc >= 0.0)) {
    R.dok = false;
    R.disc = 0.0;
  }
  R.sd = sqrt(R.disc);
  R.X = 0.5 * (opw * R.E + R.sd);
  R.P = R.X - R.E;
  R.invX = 1.0 / R.X;
  return !R.dok;
}
// cotangents of (E, S[3], Sup[3], S2, P, invX) -> chi, gi, Et, St
struct RecBar {
  double E, S[3], Sup[3], S2, P, invX;
};
__host__ __device__ inline void rec_reverse(double w, double chi, const double gi[6], double Et, const double St[3],
                                            const RecTape& R, RecBar B, double& chib, double gib[6], double& Etb,
                                            double Stb[3]) {
  if (R.Eok) {
    const double opw = 1.0 + w;
    double Xb = -B.invX * R.invX * R.invX;
    Xb += B.P;
    B.E -= B.P;
    B.E += 0.5 * opw * Xb;
    const double sdb = 0.5 * Xb;
    if (R.dok && R.sd > 0.0) {
      const double discb = sdb * 0.5 / R.sd;
      B.E += discb * 2.0 * opw * opw * R.E;
      B.S2 -= 4.0 * w * discb;
    }
  }
  for (int j = 0; j < 3; ++j) {
    B.Sup[j] += B.S2 * R.S[j];
    B.S[j] += B.S2 * R.Sup[j];
  }
  for (int j = 0; j < 3; ++j) {
    const double U = gi[S(j, 0)] * R.S[0] + gi[S(j, 1)] * R.S[1] + gi[S(j, 2)] * R.S[2];
    chib += B.Sup[j] * U;
    for (int k = 0; k < 3; ++k) {
      gib[S(j, k)] += B.Sup[j] * chi * R.S[k];
      B.S[k] += B.Sup[j] * chi * gi[S(j, k)];
    }
  }
  double c32b = 0.0;
  for (int i = 0; i < 3; ++i) {
    c32b += B.S[i] * St[i];
    Stb[i] += B.S[i] * R.c32;
  }
  c32b += B.E * Et;
  Etb += B.E * R.c32;
  chib += c32b * R.sq;
  const double sqb = c32b * chi;
  chib += sqb * 0.5 / R.sq;
}

// ---------------------------------------------------------------- fluxes along one axis
// u15 = {chi, gt[6], alpha, beta_a, Et, St[3]} (beta_a: shift component along the axis)
struct FluxIn {
  double chi, gt[6], alpha, ba, Et, St[3];
};
__host__ __device__ inline void flux_forward(double w, int a, const FluxIn& in, double F[4]) {
  InvTape I;
  inv_forward(in.gt, I);
  RecTape R;
  rec_forward(w, in.chi, I.gi, in.Et, in.St, R);
  const double im32 = 1.0 / (in.chi * sqrt(in.chi));
  F[0] = im32 * (in.alpha * R.Sup[a] - in.ba * R.E);
  const double t = in.alpha * R.Sup[a] * R.invX;
  for (int i = 0; i < 3; ++i) F[1 + i] = im32 * ((t * R.S[i] + (i == a ? in.alpha * R.P : 0.0)) - in.ba * R.S[i]);
}
__host__ __device__ inline void flux_reverse(double w, int a, const FluxIn& in, const double Fb[4], FluxIn& b) {
  InvTape I;
  inv_forward(in.gt, I);
  RecTape R;
  rec_forward(w, in.chi, I.gi, in.Et, in.St, R);
  const double v = in.chi * sqrt(in.chi);
  const double im32 = 1.0 / v;
  const double t = in.alpha * R.Sup[a] * R.invX;
  RecBar B = {0.0, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, 0.0, 0.0, 0.0};
  double im32b = Fb[0] * (in.alpha * R.Sup[a] - in.ba * R.E);
  const double G0 = Fb[0] * im32;
  b.alpha += G0 * R.Sup[a];
  B.Sup[a] += G0 * in.alpha;
  b.ba -= G0 * R.E;
  B.E -= G0 * in.ba;
  double tb = 0.0;
  for (int i = 0; i < 3; ++i) {
    im32b += Fb[1 + i] * ((t * R.S[i] + (i == a ? in.alpha * R.P : 0.0)) - in.ba * R.S[i]);
    const double Gi = Fb[1 + i] * im32;
    tb += Gi * R.S[i];
    B.S[i] += Gi * (t - in.ba);
    if (i == a) {
      b.alpha += Gi * R.P;
      B.P += Gi * in.alpha;
    }
    b.ba -= Gi * R.S[i];
  }
  b.alpha += tb * R.Sup[a] * R.invX;
  B.Sup[a] += tb * in.alpha * R.invX;
  B.invX += tb * in.alpha * R.Sup[a];
  // im32 = 1 / (chi sqrt(chi))
  const double vb = -im32b * im32 * im32;
  const double sq = sqrt(in.chi);
  b.chi += vb * sq;
  b.chi += vb * in.chi * 0.5 / sq;
  double gib[6] = {0, 0, 0, 0, 0, 0};
  rec_reverse(w, in.chi, I.gi, in.Et, in.St, R, B, b.chi, gib, b.Et, b.St);
  inv_reverse(in.gt, I, gib, b.gt);
}

// ---------------------------------------------------------------- vector-Jacobian product at one point
// A reverse sweep taped in statement order would keep every forward
// intermediate and every input cotangent live at once (several hundred doubles
// per point, far beyond the registers of a wavefront). The algebra is only a few
// layers deep, though: the cotangent of every intermediate that feeds an output
// directly (the curvature source X_ij and its trace, the Ricci tensor, the
// Hessians of chi and alpha, the matter projections) is fixed by the output
// cotangents and the point values alone, and only the connection coefficients
// need a reverse of their own. So the sweep runs forwards through the inputs:
// metric and output cotangents first; then the first differences of chi, alpha
// and beta; then the connection (the metric's first differences) with its
// reverse; then the metric's second differences, d_a Gamma^k, the shift's second
// differences and d_a K, one field at a time; last the terms of the point values
// and the fluid. Forward values are formed where they are used (nothing is
// taped), and every cotangent is handed to `out` as soon as it is final (the
// shift's point values last, after every difference request, so that a source
// may fold other terms into them on the way):
//   out.val(f, v)    cotangent of the point value of field f,
//   out.d1(f, a, v)  of its first difference along a,
//   out.d2(f, q, v)  of its second difference, symmetric pair q.
// `src` provides the inputs where they are needed -- val(f) and cot(f), the point
// value and the output cotangent of field f; d1(f, d[3]), d12(f, d1[3], d2[6]) and
// d2(f, d2[6]), its differences -- fence(), a point across which device code is
// not to be reordered, and pin(x), which makes x be formed before the code goes on
// (both no-ops on the host).
template <class Src, class Sink>
__host__ __device__ inline void pt_vjp(const DevParams& P, double t, const Src& src, Sink& out) {
  const double third = 1.0 / 3.0;
  const double chi = src.val(F_CHI), alpha = src.val(F_ALP);
  double gt[6], gi[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) gt[s] = src.val(F_GT + s);
  {
    InvTape I;
    inv_forward(gt, I);
#pragma unroll
    for (int s = 0; s < 6; ++s) gi[s] = I.gi[s];
  }
  const double ichi = 1.0 / chi, ih = 0.5 / chi, iq = 0.25 / (chi * chi);

  // ---- cotangents fixed by the output cotangents: X_ij, Ricci, Hessians
  double X6b[6], DDab[6], DDchib[6], trDDb = 0.0, dc2b = 0.0, cdab = 0.0;
  {
    double rAt[6], trXb = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      rAt[s] = src.cot(F_AT + s);
      trXb -= rAt[s] * chi * gt[s] * third;
    }
#pragma unroll
    for (int s = 0; s < 6; ++s) X6b[s] = rAt[s] * chi + trXb * wsym(s) * gi[s];
  }
  const double Cg = -src.cot(F_K) * chi;  // cotangent of the lapse Laplacian, times chi
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    DDab[s] = -X6b[s] + Cg * wsym(s) * gi[s];
    const double r = X6b[s] * alpha;  // Ricci cotangent
    trDDb += r * ih * gt[s];
    dc2b -= r * iq * 3.0 * gt[s];
    cdab -= DDab[s] * (0.5 / chi) * gt[s];
  }
#pragma unroll
  for (int s = 0; s < 6; ++s) DDchib[s] = X6b[s] * alpha * ih + trDDb * wsym(s) * gi[s];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    out.d2(F_CHI, q, DDchib[q]);
    out.d2(F_ALP, q, DDab[q]);
  }
#pragma unroll
  for (int s = 0; s < 6; ++s)
#pragma unroll
    for (int q = 0; q < 6; ++q) out.d2(F_GT + s, q, -0.5 * X6b[s] * alpha * wsym(q) * gi[q]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double dGb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      const double r = X6b[s] * alpha;
      dGb[j] += 0.5 * r * gt[S(k, i)];
      dGb[i] += 0.5 * r * gt[S(k, j)];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) out.d1(F_GAM + k, a, dGb[a]);
  }
  src.fence();
  {  // connection-function and shift cotangents of the shift's second differences, d_a K, Gamma, beta
    double rGam[3], Yb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) rGam[i] = src.cot(F_GAM + i);
#pragma unroll
    for (int l = 0; l < 3; ++l) Yb[l] = (rGam[0] * gi[S(0, l)] + rGam[1] * gi[S(1, l)] + rGam[2] * gi[S(2, l)]) * third;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double d2b[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) d2b[q] = rGam[k] * wsym(q) * gi[q];
#pragma unroll
      for (int l = 0; l < 3; ++l) d2b[S(l, k)] += Yb[l];
#pragma unroll
      for (int q = 0; q < 6; ++q) out.d2(F_BET + k, q, d2b[q]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
      out.d1(F_K, j, -(2.0 / 3.0) * 2.0 * alpha * (rGam[0] * gi[S(0, j)] + rGam[1] * gi[S(1, j)] + rGam[2] * gi[S(2, j)]));
#pragma unroll
    for (int i = 0; i < 3; ++i) out.val(F_GAM + i, P.evolve_shift ? 0.75 * src.cot(F_BET + i) : 0.0);
  }
  src.fence();
  // fluid quantities the connection step needs: S^jk and the momentum-source cotangent
  double Sjk[6], Ttb[3];
  {
    const double St[3] = {src.val(F_ST), src.val(F_ST + 1), src.val(F_ST + 2)};
    RecTape R;
    rec_forward(P.w, chi, gi, src.val(F_ET), St, R);
#pragma unroll
    for (int s = 0; s < 6; ++s) Sjk[s] = R.Sup[SI(s)] * R.Sup[SJ(s)] * R.invX + R.P * chi * gi[s];
    const double im32 = 1.0 / (chi * sqrt(chi));
#pragma unroll
    for (int i = 0; i < 3; ++i) Ttb[i] = src.cot(F_ST + i) * im32 * 0.5 * alpha;
  }
  src.fence();

  // ---- first differences of chi, alpha, beta; the conformal-factor terms of the Hessians
  double dchi[3], dal[3], db[3][3], DDchi[6], DDa[6];  // DDchi, DDa: second differences for now
  src.d12(F_CHI, dchi, DDchi);
  src.d12(F_ALP, dal, DDa);
#pragma unroll
  for (int c = 0; c < 3; ++c) src.d1(F_BET + c, db[c]);
  const double divb = db[0][0] + db[1][1] + db[2][2];
  double bchi = 0.0, balpha = 0.0, bgt[6], gib[6], Xacc[6];  // Xacc: X_ij, summed as its terms appear
  double bdchi[3] = {0.0, 0.0, 0.0}, bdal[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 6; ++s) bgt[s] = gib[s] = Xacc[s] = 0.0;
  {
    double cda = 0.0, dc2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        cda += gi[S(k, l)] * dchi[k] * dal[l];
        dc2 += gi[S(k, l)] * dchi[k] * dchi[l];
      }
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      const double Wv = (dchi[i] * dal[j] + dchi[j] * dal[i]) - gt[s] * cda;
      DDa[s] += (0.5 / chi) * Wv;
      const double Wb = DDab[s] * (0.5 / chi);
      bchi -= DDab[s] * Wv * 0.5 / (chi * chi);
      bdchi[i] += Wb * dal[j];
      bdal[j] += Wb * dchi[i];
      bdchi[j] += Wb * dal[i];
      bdal[i] += Wb * dchi[j];
      bgt[s] -= Wb * cda;
      const double r = X6b[s] * alpha;
      const double dq = -iq * (dchi[i] * dchi[j] + 3.0 * gt[s] * dc2);
      Xacc[s] += alpha * dq;
      balpha += X6b[s] * dq;
      bdchi[i] -= r * iq * dchi[j];
      bdchi[j] -= r * iq * dchi[i];
      bgt[s] -= r * iq * 3.0 * dc2;
      bchi += r * (dchi[i] * dchi[j] + 3.0 * gt[s] * dc2) * 0.5 / (chi * chi * chi);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        gib[S(k, l)] += cdab * dchi[k] * dal[l] + dc2b * dchi[k] * dchi[l];
        bdchi[k] += cdab * gi[S(k, l)] * dal[l];
        bdal[l] += cdab * gi[S(k, l)] * dchi[k];
        bdchi[l] += dc2b * gi[S(k, l)] * dchi[k];
        bdchi[k] += dc2b * gi[S(k, l)] * dchi[l];
      }
  }
  src.fence();

  // ---- connection and its reverse
  double Gl[3][6], sg[3], SjkbD[6];  // SjkbD: the d gamma part of the S^jk cotangent
  {
    double dgt[6][3];
#pragma unroll
    for (int s = 0; s < 6; ++s) src.d1(F_GT + s, dgt[s]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), j = SJ(s);
        Gl[k][s] = 0.5 * ((dgt[S(k, j)][i] + dgt[S(k, i)][j]) - dgt[s][k]);
      }
#pragma unroll
    for (int s = 0; s < 6; ++s) SjkbD[s] = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sg[a] = 0.0;
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        sg[a] += wsym(s) * Sjk[s] * dgt[s][a];
        SjkbD[s] += Ttb[a] * ichi * wsym(s) * dgt[s][a];
      }
    }
  }
  double Gu[3][6], Gd[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int s = 0; s < 6; ++s) Gu[k][s] = gi[S(k, 0)] * Gl[0][s] + gi[S(k, 1)] * Gl[1][s] + gi[S(k, 2)] * Gl[2][s];
    Gd[k] = contract_sym(gi, Gu[k]);
  }
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    DDchi[s] -= Gu[0][s] * dchi[0] + Gu[1][s] * dchi[1] + Gu[2][s] * dchi[2];
    DDa[s] -= Gu[0][s] * dal[0] + Gu[1][s] * dal[1] + Gu[2][s] * dal[2];
  }
  {
    const double trDD = contract_sym(gi, DDchi);
    bchi += -src.cot(F_K) * contract_sym(gi, DDa);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const double r = X6b[s] * alpha;
      const double dr = ih * (DDchi[s] + gt[s] * trDD);
      Xacc[s] += alpha * dr - DDa[s];
      balpha += X6b[s] * dr;
      bgt[s] += r * ih * trDD;
      bchi -= r * (DDchi[s] + gt[s] * trDD) * 0.5 / (chi * chi);
      gib[s] += trDDb * wsym(s) * DDchi[s] + Cg * wsym(s) * DDa[s];
    }
  }
  double Gub[3][6], Glb[3][6], Gdb[3], AupbG[6];  // AupbG: the connection part of the A^ij cotangent
  {
    double Aup[6], innb[3];
    {
      double At[6], Amix[3][3];
#pragma unroll
      for (int s = 0; s < 6; ++s) At[s] = src.val(F_AT + s);
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          Amix[k][j] = gi[S(k, 0)] * At[S(0, j)] + gi[S(k, 1)] * At[S(1, j)] + gi[S(k, 2)] * At[S(2, j)];
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), j = SJ(s);
        Aup[s] = Amix[i][0] * gi[S(0, j)] + Amix[i][1] * gi[S(1, j)] + Amix[i][2] * gi[S(2, j)];
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double rG = src.cot(F_GAM + k);
      innb[k] = 2.0 * rG * alpha;
      Gdb[k] = (2.0 / 3.0) * rG * divb - (src.cot(F_GAM) * db[0][k] + src.cot(F_GAM + 1) * db[1][k] +
                                           src.cot(F_GAM + 2) * db[2][k]);
      balpha += 2.0 * rG * contract_sym(Gu[k], Aup);
    }
#pragma unroll
    for (int s = 0; s < 6; ++s) AupbG[s] = innb[0] * wsym(s) * Gu[0][s] + innb[1] * wsym(s) * Gu[1][s] +
                                           innb[2] * wsym(s) * Gu[2][s];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        Gub[k][s] = innb[k] * wsym(s) * Aup[s] - DDab[s] * dal[k] - DDchib[s] * dchi[k];
        Glb[k][s] = 0.0;
        bdal[k] -= DDab[s] * Gu[k][s];
        bdchi[k] -= DDchib[s] * Gu[k][s];
      }
  }
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    src.fence();
    const int i = SI(s), j = SJ(s);
    const double r = X6b[s] * alpha;
    double dr = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double gsum = Gl[i][S(j, k)] + Gl[j][S(i, k)];
      dr += 0.5 * Gd[k] * gsum;
      Gdb[k] += 0.5 * r * gsum;
      Glb[i][S(j, k)] += 0.5 * r * Gd[k];
      Glb[j][S(i, k)] += 0.5 * r * Gd[k];
    }
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        src.fence();
        const double g = gi[S(l, m)];
        double term = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          term += (Gu[k][S(l, i)] * Gl[j][S(k, m)] + Gu[k][S(l, j)] * Gl[i][S(k, m)]) + Gu[k][S(i, m)] * Gl[k][S(l, j)];
          Gub[k][S(l, i)] += r * g * Gl[j][S(k, m)];
          Glb[j][S(k, m)] += r * g * Gu[k][S(l, i)];
          Gub[k][S(l, j)] += r * g * Gl[i][S(k, m)];
          Glb[i][S(k, m)] += r * g * Gu[k][S(l, j)];
          Gub[k][S(i, m)] += r * g * Gl[k][S(l, j)];
          Glb[k][S(l, j)] += r * g * Gu[k][S(i, m)];
        }
        dr += g * term;
        gib[S(l, m)] += r * term;
      }
    Xacc[s] += alpha * dr;
    balpha += X6b[s] * dr;
  }
  src.fence();
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      gib[s] += Gdb[k] * wsym(s) * Gu[k][s];
      Gub[k][s] += Gdb[k] * wsym(s) * gi[s];
    }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int s = 0; s < 6; ++s)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        gib[S(k, l)] += Gub[k][s] * Gl[l][s];
        Glb[l][s] += Gub[k][s] * gi[S(k, l)];
      }
  {
    double bdgt[6][3];
#pragma unroll
    for (int s = 0; s < 6; ++s)
#pragma unroll
      for (int a = 0; a < 3; ++a) bdgt[s][a] = Ttb[a] * ichi * wsym(s) * Sjk[s];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), j = SJ(s);
        bdgt[S(k, j)][i] += 0.5 * Glb[k][s];
        bdgt[S(k, i)][j] += 0.5 * Glb[k][s];
        bdgt[s][k] -= 0.5 * Glb[k][s];
      }
#pragma unroll
    for (int s = 0; s < 6; ++s)
#pragma unroll
      for (int a = 0; a < 3; ++a) out.d1(F_GT + s, a, bdgt[s][a]);
  }
  src.fence();

  // ---- streamed: second differences of the metric, d_a Gamma^k, shift second differences, d_a K
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    double d2[6];
    src.d2(F_GT + s, d2);
    const double dr = -0.5 * contract_sym(gi, d2);
    Xacc[s] += alpha * dr;
    balpha += X6b[s] * dr;
#pragma unroll
    for (int q = 0; q < 6; ++q) gib[q] -= 0.5 * X6b[s] * alpha * wsym(q) * d2[q];
    src.pin(Xacc[s]);
    src.pin(balpha);
#pragma unroll
    for (int q = 0; q < 6; ++q) src.pin(gib[q]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double d[3];
    src.d1(F_GAM + k, d);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      const double dr = 0.5 * (gt[S(k, i)] * d[j] + gt[S(k, j)] * d[i]);
      Xacc[s] += alpha * dr;
      balpha += X6b[s] * dr;
      bgt[S(k, i)] += 0.5 * X6b[s] * alpha * d[j];
      bgt[S(k, j)] += 0.5 * X6b[s] * alpha * d[i];
    }
    src.pin(balpha);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      src.pin(Xacc[s]);
      src.pin(bgt[s]);
    }
  }
  {
    double Y[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double d2[6];
      src.d2(F_BET + k, d2);
      const double rG = src.cot(F_GAM + k);
#pragma unroll
      for (int q = 0; q < 6; ++q) gib[q] += rG * wsym(q) * d2[q];
#pragma unroll
      for (int l = 0; l < 3; ++l) Y[l] += d2[S(l, k)];
#pragma unroll
      for (int q = 0; q < 6; ++q) src.pin(gib[q]);
#pragma unroll
      for (int l = 0; l < 3; ++l) src.pin(Y[l]);
    }
    double dK[3];
    src.d1(F_K, dK);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double rG = src.cot(F_GAM + i);
      const double W = gi[S(i, 0)] * dK[0] + gi[S(i, 1)] * dK[1] + gi[S(i, 2)] * dK[2];
      balpha -= 2.0 * rG * (2.0 / 3.0) * W;
#pragma unroll
      for (int l = 0; l < 3; ++l) gib[S(i, l)] += rG * Y[l] * third - 2.0 * rG * alpha * (2.0 / 3.0) * dK[l];
    }
  }
  src.fence();

  // ---- terms of the point values, and the fluid
  const double K = src.val(F_K);
  double At[6], Amix[3][3], Aup[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) At[s] = src.val(F_AT + s);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Amix[k][j] = gi[S(k, 0)] * At[S(0, j)] + gi[S(k, 1)] * At[S(1, j)] + gi[S(k, 2)] * At[S(2, j)];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    Aup[s] = Amix[i][0] * gi[S(0, j)] + Amix[i][1] * gi[S(1, j)] + Amix[i][2] * gi[S(2, j)];
  }
  const double St[3] = {src.val(F_ST), src.val(F_ST + 1), src.val(F_ST + 2)};
  const double Et = src.val(F_ET);
  RecTape R;
  rec_forward(P.w, chi, gi, Et, St, R);
  const double im32 = 1.0 / (chi * sqrt(chi));
  const double rK = src.cot(F_K), rEt = src.cot(F_ET), rchi = src.cot(F_CHI);
  const double AAb = rK * alpha, KSb = rEt * im32 * alpha, Sdab = -rEt * im32;
  double bK = 0.0, bAt[6], Aupb[6], Amixb[3][3], ichib = 0.0, im32b = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    bAt[s] = AAb * wsym(s) * Aup[s];
    Aupb[s] = AAb * wsym(s) * At[s] + AupbG[s];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j) Amixb[k][j] = 0.0;
  RecBar B = {0.0, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, 0.0, 0.0, 0.0};
  double Kij[6], KS = 0.0, sgt = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    Kij[s] = (At[s] + gt[s] * K * third) / chi;
    KS += wsym(s) * Kij[s] * Sjk[s];
    sgt += wsym(s) * Sjk[s] * gt[s];
  }
  balpha += rEt * im32 * KS;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const double Kijb = KSb * wsym(s) * Sjk[s];
    bAt[s] += Kijb / chi;
    bgt[s] += Kijb * K / (3.0 * chi);
    bK += Kijb * gt[s] / (3.0 * chi);
    bchi -= Kijb * Kij[s] / chi;
  }
  {
    const double Kbg = P.lapse_bg ? -3.0 * P.H0 / (1.0 + 2.0 * P.H0 * t) : 0.0;
    const double ra = src.cot(F_ALP);
    balpha -= 2.0 * (K - Kbg) * ra;
    bK -= 2.0 * alpha * ra;
  }
  double divbb = -(2.0 / 3.0) * rchi * chi, bdb[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) bdb[c][a] = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    const double r = src.cot(F_AT + s), rg = src.cot(F_GT + s);
    double AAij = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) AAij += At[S(i, k)] * Amix[k][j];
    balpha += r * (K * At[s] - 2.0 * AAij);
    bK += r * alpha * At[s];
    bAt[s] += r * alpha * K;
    const double AAijb = -2.0 * r * alpha;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      bAt[S(i, k)] += AAijb * Amix[k][j];
      Amixb[k][j] += AAijb * At[S(i, k)];
      // Lie derivative along the shift
      bAt[S(i, k)] += r * db[k][j];
      bdb[k][j] += r * At[S(i, k)];
      bAt[S(j, k)] += r * db[k][i];
      bdb[k][i] += r * At[S(j, k)];
      bgt[S(i, k)] += rg * db[k][j];
      bdb[k][j] += rg * gt[S(i, k)];
      bgt[S(j, k)] += rg * db[k][i];
      bdb[k][i] += rg * gt[S(j, k)];
    }
    bAt[s] -= (2.0 / 3.0) * r * divb;
    bgt[s] -= (2.0 / 3.0) * rg * divb;
    divbb -= (2.0 / 3.0) * (r * At[s] + rg * gt[s]);
    balpha -= 2.0 * rg * At[s];
    bAt[s] -= 2.0 * rg * alpha;
  }
  {
    const double Str = R.S2 * R.invX + 3.0 * R.P;
    const double AA = contract_sym(At, Aup);
    const double Strb = rK * 4.0 * PI_D * alpha;
    balpha += rK * (AA + K * K * third + 4.0 * PI_D * (R.E + Str));
    bK += rK * alpha * 2.0 * K * third;
    B.E += rK * 4.0 * PI_D * alpha;
    B.S2 += Strb * R.invX;
    B.invX += Strb * R.S2;
    B.P += 3.0 * Strb;
  }
  balpha += rchi * (2.0 / 3.0) * chi * K;
  bK += rchi * (2.0 / 3.0) * chi * alpha;
  bchi += rchi * (2.0 / 3.0) * (alpha * K - divb);
  out.val(F_K, bK);
  // connection functions: the terms without the connection
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double r = src.cot(F_GAM + i);
    double V = 0.0, Z = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      V += gi[S(i, j)] * R.S[j];
      Z += Aup[S(i, j)] * dchi[j];
    }
    balpha -= 16.0 * PI_D * r * V;
    const double Vb = -16.0 * PI_D * r * alpha;
    balpha -= 2.0 * r * (1.5 / chi) * Z;
    const double innb = 2.0 * r * alpha, Zb = -innb * 1.5 / chi;
    bchi += innb * 1.5 * Z / (chi * chi);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      gib[S(i, j)] += Vb * R.S[j];
      B.S[j] += Vb * gi[S(i, j)];
      Aupb[S(i, j)] += Zb * dchi[j] - 2.0 * r * dal[j];
      bdchi[j] += Zb * Aup[S(i, j)];
      bdal[j] -= 2.0 * r * Aup[S(i, j)];
      bdb[i][j] -= r * Gd[j];
    }
    divbb += r * (2.0 / 3.0) * Gd[i];
  }
  bdb[0][0] += divbb;
  bdb[1][1] += divbb;
  bdb[2][2] += divbb;
  // matter: S_ij in the curvature source, the fluid sources
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    const double Sij = R.S[i] * R.S[j] * R.invX + R.P * gt[s] * ichi;
    Xacc[s] -= 8.0 * PI_D * alpha * Sij;
    balpha -= 8.0 * PI_D * X6b[s] * Sij;
    const double Sijb = -8.0 * PI_D * X6b[s] * alpha;
    B.S[i] += Sijb * R.S[j] * R.invX;
    B.S[j] += Sijb * R.S[i] * R.invX;
    B.invX += Sijb * R.S[i] * R.S[j];
    B.P += Sijb * gt[s] * ichi;
    bgt[s] += Sijb * R.P * ichi;
    ichib += Sijb * R.P * gt[s];
  }
  double sgtb = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double qb = src.cot(F_ST + i) * im32;
    sgtb -= Ttb[i] * dchi[i] * ichi * ichi;
    B.E -= qb * dal[i];
    bdal[i] -= qb * R.E;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      B.S[k] += qb * db[k][i];
      bdb[k][i] += qb * R.S[k];
    }
    bdchi[i] -= Ttb[i] * sgt * ichi * ichi;
    ichib -= Ttb[i] * sgt * dchi[i] * 2.0 * ichi;
    const double Tt = sg[i] * ichi - sgt * dchi[i] * (ichi * ichi);
    const double q = -R.E * dal[i] + (R.S[0] * db[0][i] + R.S[1] * db[1][i] + R.S[2] * db[2][i]) + 0.5 * alpha * Tt;
    im32b += src.cot(F_ST + i) * q;
    balpha += qb * 0.5 * Tt;
    ichib += Ttb[i] * sg[i];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) out.d1(F_BET + c, a, bdb[c][a]);
  {
    const double Sda = R.Sup[0] * dal[0] + R.Sup[1] * dal[1] + R.Sup[2] * dal[2];
    im32b += rEt * (alpha * KS - Sda);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      B.Sup[j] += Sdab * dal[j];
      bdal[j] += Sdab * R.Sup[j];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    out.d1(F_CHI, a, bdchi[a]);
    out.d1(F_ALP, a, bdal[a]);
  }
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    bgt[s] += sgtb * wsym(s) * Sjk[s];
    const double Sjkb = sgtb * wsym(s) * gt[s] + KSb * wsym(s) * Kij[s] + SjkbD[s];
    B.Sup[i] += Sjkb * R.Sup[j] * R.invX;
    B.Sup[j] += Sjkb * R.Sup[i] * R.invX;
    B.invX += Sjkb * R.Sup[i] * R.Sup[j];
    B.P += Sjkb * chi * gi[s];
    bchi += Sjkb * R.P * gi[s];
    gib[s] += Sjkb * R.P * chi;
  }
  {  // im32 = 1 / (chi sqrt(chi))
    const double vb = -im32b * im32 * im32;
    const double sq = sqrt(chi);
    bchi += vb * sq + vb * chi * 0.5 / sq;
  }
  bchi -= ichib * ichi * ichi;
  {
    double bEt = 0.0, bSt[3] = {0.0, 0.0, 0.0};
    rec_reverse(P.w, chi, gi, Et, St, R, B, bchi, gib, bEt, bSt);
    out.val(F_ET, bEt);
#pragma unroll
    for (int c = 0; c < 3; ++c) out.val(F_ST + c, bSt[c]);
  }
  // A^ij and A^i_j back to A_ij and the inverse metric
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      Amixb[i][l] += Aupb[s] * gi[S(l, j)];
      gib[S(l, j)] += Aupb[s] * Amix[i][l];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        gib[S(k, l)] += Amixb[k][j] * At[S(l, j)];
        bAt[S(l, j)] += Amixb[k][j] * gi[S(k, l)];
      }
#pragma unroll
  for (int s = 0; s < 6; ++s) out.val(F_AT + s, bAt[s]);
  // the curvature source X_ij is complete
  {
    double trXb = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) trXb -= src.cot(F_AT + s) * chi * gt[s] * third;
    const double trX = contract_sym(gi, Xacc);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const double r = src.cot(F_AT + s);
      bchi += r * (Xacc[s] - gt[s] * trX * third);
      bgt[s] -= r * chi * trX * third;
      gib[s] += trXb * wsym(s) * Xacc[s];
    }
  }
  {
    InvTape I;
    inv_forward(gt, I);
    inv_reverse(gt, I, gib, bgt);
  }
  out.val(F_CHI, bchi);
#pragma unroll
  for (int s = 0; s < 6; ++s) out.val(F_GT + s, bgt[s]);
  out.val(F_ALP, balpha);
#pragma unroll
  for (int i = 0; i < 3; ++i) out.val(F_BET + i, P.evolve_shift ? -P.eta * src.cot(F_BET + i) : 0.0);
}

}  // namespace cosmos
