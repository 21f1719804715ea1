// Hand-written reverse mode of the pointwise part of the right-hand side (and
// of the fluid fluxes), for the discrete adjoint of the RK4 step.
//
// pt_forward evaluates the pointwise algebra of one point -- everything except
// the advection, dissipation and flux-divergence stencils -- from the point
// values and the finite-difference derivatives (the same equations as the
// stage kernel: conformal connection and Ricci tensor, second covariant
// derivative of the lapse, perfect-fluid recovery and projections, the BSSN
// and fluid source terms), keeping its intermediates. pt_reverse then walks the
// same statements backwards: given the cotangent rbar of the 25 outputs it
// accumulates the cotangents of every input (dy = a dx  =>  xbar += a ybar).
// flux_forward / flux_reverse do the same for the fluxes of the densitised
// fluid variables along one axis. Branches (recovery clamps) are taken exactly
// as in the forward evaluation, so this is the derivative of the discrete map.
//
// __host__ __device__ so that the algebra can also be checked on the CPU.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "bssn_device.hpp"

namespace cosmos {

// Inputs of the pointwise algebra at one point. dX[c][a] = d_a X_c.
struct PtIn {
  double chi, gt[6], K, At[6], Gam[3], alpha, beta[3];
  double dchi[3], d2chi[6], dgt[6][3], d2gt[6][6], dGam[3][3], dalpha[3], d2alpha[6], dbeta[3][3], d2beta[3][6];
  double dK[3], dAt[6][3];  // dAt: constraint input, unused by the right-hand side
  double Et, St[3];
};

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

// ---------------------------------------------------------------- pointwise right-hand side
struct PtTape {
  InvTape I;
  RecTape R;
  double ichi, Sjk[6], Sij[6], Str;
  double Gl[3][6], Gu[3][6], Gd[3];
  double DDchi[6], trDD, dc2;
  double Ric[6];
  double cda, DDa[6], D2a;
  double Amix[3][3], Aup[6], AA, divb;
  double X6[6], trX;
  double Kij[6], KS, im32, sg[3], sgt, Sda;
  double Kbg;
};

__host__ __device__ inline void pt_forward(const DevParams& P, double t, const PtIn& in, PtTape& T, double r[NF],
                                           bool& fail) {
  const double* gt = in.gt;
  const double chi = in.chi, K = in.K, alpha = in.alpha;
  inv_forward(gt, T.I);
  const double* gi = T.I.gi;
  fail = rec_forward(P.w, chi, gi, in.Et, in.St, T.R);
  const RecTape& R = T.R;
  T.ichi = 1.0 / chi;
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    T.Sjk[s] = R.Sup[i] * R.Sup[j] * R.invX + R.P * chi * gi[s];
    T.Sij[s] = R.S[i] * R.S[j] * R.invX + R.P * gt[s] * T.ichi;
  }
  T.Str = R.S2 * R.invX + 3.0 * R.P;
  // connection
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      T.Gl[k][s] = 0.5 * ((in.dgt[S(k, j)][i] + in.dgt[S(k, i)][j]) - in.dgt[s][k]);
    }
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 6; ++s) T.Gu[k][s] = gi[S(k, 0)] * T.Gl[0][s] + gi[S(k, 1)] * T.Gl[1][s] + gi[S(k, 2)] * T.Gl[2][s];
  for (int k = 0; k < 3; ++k) T.Gd[k] = contract_sym(gi, T.Gu[k]);
  // Ricci
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    double rr = -0.5 * contract_sym(gi, in.d2gt[s]);
    for (int k = 0; k < 3; ++k) rr += 0.5 * (gt[S(k, i)] * in.dGam[k][j] + gt[S(k, j)] * in.dGam[k][i]);
    for (int k = 0; k < 3; ++k) rr += 0.5 * T.Gd[k] * (T.Gl[i][S(j, k)] + T.Gl[j][S(i, k)]);
    for (int l = 0; l < 3; ++l)
      for (int m = 0; m < 3; ++m) {
        const double g = gi[S(l, m)];
        for (int k = 0; k < 3; ++k)
          rr += g * ((T.Gu[k][S(l, i)] * T.Gl[j][S(k, m)] + T.Gu[k][S(l, j)] * T.Gl[i][S(k, m)]) +
                     T.Gu[k][S(i, m)] * T.Gl[k][S(l, j)]);
      }
    T.Ric[s] = rr;
  }
  for (int s = 0; s < 6; ++s)
    T.DDchi[s] = in.d2chi[s] - (T.Gu[0][s] * in.dchi[0] + T.Gu[1][s] * in.dchi[1] + T.Gu[2][s] * in.dchi[2]);
  T.trDD = contract_sym(gi, T.DDchi);
  T.dc2 = 0.0;
  for (int l = 0; l < 3; ++l)
    for (int m = 0; m < 3; ++m) T.dc2 += gi[S(l, m)] * in.dchi[l] * in.dchi[m];
  {
    const double ih = 0.5 / chi, iq = 0.25 / (chi * chi);
    for (int s = 0; s < 6; ++s)
      T.Ric[s] += ih * (T.DDchi[s] + gt[s] * T.trDD) - iq * (in.dchi[SI(s)] * in.dchi[SJ(s)] + 3.0 * gt[s] * T.dc2);
  }
  // lapse
  T.cda = 0.0;
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) T.cda += gi[S(k, l)] * in.dchi[k] * in.dalpha[l];
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    T.DDa[s] = (in.d2alpha[s] - (T.Gu[0][s] * in.dalpha[0] + T.Gu[1][s] * in.dalpha[1] + T.Gu[2][s] * in.dalpha[2])) +
               (0.5 / chi) * ((in.dchi[i] * in.dalpha[j] + in.dchi[j] * in.dalpha[i]) - gt[s] * T.cda);
  }
  T.D2a = chi * contract_sym(gi, T.DDa);
  // traceless curvature
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      T.Amix[k][j] = gi[S(k, 0)] * in.At[S(0, j)] + gi[S(k, 1)] * in.At[S(1, j)] + gi[S(k, 2)] * in.At[S(2, j)];
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    T.Aup[s] = T.Amix[i][0] * gi[S(0, j)] + T.Amix[i][1] * gi[S(1, j)] + T.Amix[i][2] * gi[S(2, j)];
  }
  T.AA = contract_sym(in.At, T.Aup);
  const double (*db)[3] = in.dbeta;
  T.divb = db[0][0] + db[1][1] + db[2][2];
  // outputs
  r[F_CHI] = (2.0 / 3.0) * chi * (alpha * K - T.divb);
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    double v = 0.0;
    for (int k = 0; k < 3; ++k) v += gt[S(i, k)] * db[k][j] + gt[S(j, k)] * db[k][i];
    r[F_GT + s] = v - (2.0 / 3.0) * gt[s] * T.divb - 2.0 * alpha * in.At[s];
  }
  r[F_K] = -T.D2a + alpha * (T.AA + K * K * (1.0 / 3.0)) + 4.0 * PI_D * alpha * (R.E + T.Str);
  for (int s = 0; s < 6; ++s) T.X6[s] = -T.DDa[s] + alpha * (T.Ric[s] - 8.0 * PI_D * T.Sij[s]);
  T.trX = contract_sym(gi, T.X6);
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    double v = 0.0;
    for (int k = 0; k < 3; ++k) v += in.At[S(i, k)] * db[k][j] + in.At[S(j, k)] * db[k][i];
    v -= (2.0 / 3.0) * in.At[s] * T.divb;
    v += chi * (T.X6[s] - gt[s] * T.trX * (1.0 / 3.0));
    double AAij = 0.0;
    for (int k = 0; k < 3; ++k) AAij += in.At[S(i, k)] * T.Amix[k][j];
    r[F_AT + s] = v + alpha * (K * in.At[s] - 2.0 * AAij);
  }
  for (int i = 0; i < 3; ++i) {
    double v = -(T.Gd[0] * db[i][0] + T.Gd[1] * db[i][1] + T.Gd[2] * db[i][2]);
    v += (2.0 / 3.0) * T.Gd[i] * T.divb;
    v += contract_sym(gi, in.d2beta[i]);
    for (int l = 0; l < 3; ++l) {
      const double Y = in.d2beta[0][S(l, 0)] + in.d2beta[1][S(l, 1)] + in.d2beta[2][S(l, 2)];
      v += gi[S(i, l)] * Y * (1.0 / 3.0);
    }
    v -= 2.0 * (T.Aup[S(i, 0)] * in.dalpha[0] + T.Aup[S(i, 1)] * in.dalpha[1] + T.Aup[S(i, 2)] * in.dalpha[2]);
    double inner = contract_sym(T.Gu[i], T.Aup);
    inner -= (1.5 / chi) * (T.Aup[S(i, 0)] * in.dchi[0] + T.Aup[S(i, 1)] * in.dchi[1] + T.Aup[S(i, 2)] * in.dchi[2]);
    inner -= (2.0 / 3.0) * (gi[S(i, 0)] * in.dK[0] + gi[S(i, 1)] * in.dK[1] + gi[S(i, 2)] * in.dK[2]);
    v += 2.0 * alpha * inner;
    v -= 16.0 * PI_D * alpha * (gi[S(i, 0)] * R.S[0] + gi[S(i, 1)] * R.S[1] + gi[S(i, 2)] * R.S[2]);
    r[F_GAM + i] = v;
  }
  T.Kbg = P.lapse_bg ? -3.0 * P.H0 / (1.0 + 2.0 * P.H0 * t) : 0.0;
  r[F_ALP] = -2.0 * alpha * (K - T.Kbg);
  for (int i = 0; i < 3; ++i) r[F_BET + i] = P.evolve_shift ? 0.75 * in.Gam[i] - P.eta * in.beta[i] : 0.0;
  T.im32 = 1.0 / (chi * sqrt(chi));
  T.KS = 0.0;
  for (int s = 0; s < 6; ++s) {
    T.Kij[s] = (in.At[s] + gt[s] * K * (1.0 / 3.0)) / chi;
    T.KS += wsym(s) * T.Kij[s] * T.Sjk[s];
  }
  T.Sda = R.Sup[0] * in.dalpha[0] + R.Sup[1] * in.dalpha[1] + R.Sup[2] * in.dalpha[2];
  r[F_ET] = T.im32 * (alpha * T.KS - T.Sda);
  T.sgt = 0.0;
  for (int s = 0; s < 6; ++s) T.sgt += wsym(s) * T.Sjk[s] * gt[s];
  for (int a = 0; a < 3; ++a) {
    T.sg[a] = 0.0;
    for (int s = 0; s < 6; ++s) T.sg[a] += wsym(s) * T.Sjk[s] * in.dgt[s][a];
  }
  for (int i = 0; i < 3; ++i) {
    double q = -R.E * in.dalpha[i] + (R.S[0] * db[0][i] + R.S[1] * db[1][i] + R.S[2] * db[2][i]);
    q += 0.5 * alpha * (T.sg[i] * T.ichi - T.sgt * in.dchi[i] * (T.ichi * T.ichi));
    r[F_ST + i] = T.im32 * q;
  }
}

// Reverse sweep: accumulates into b (which the caller zeroes) the cotangents of the inputs.
__host__ __device__ inline void pt_reverse(const DevParams& P, const PtIn& in, const PtTape& T, const double rb[NF],
                                           PtIn& b) {
  const double* gt = in.gt;
  const double chi = in.chi, K = in.K, alpha = in.alpha;
  const double* gi = T.I.gi;
  const RecTape& R = T.R;
  const double (*db)[3] = in.dbeta;
  double gib[6] = {0, 0, 0, 0, 0, 0};
  RecBar B = {0.0, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, 0.0, 0.0, 0.0};
  double Sjkb[6] = {0, 0, 0, 0, 0, 0}, Sijb[6] = {0, 0, 0, 0, 0, 0}, Strb = 0.0;
  double Glb[3][6] = {}, Gub[3][6] = {}, Gdb[3] = {0, 0, 0};
  double DDchib[6] = {}, trDDb = 0.0, dc2b = 0.0, Ricb[6] = {};
  double cdab = 0.0, DDab[6] = {}, D2ab = 0.0;
  double Amixb[3][3] = {}, Aupb[6] = {}, AAb = 0.0, divbb = 0.0;
  double X6b[6] = {}, trXb = 0.0;
  double Kijb[6] = {}, KSb = 0.0, im32b = 0.0, sgb[3] = {0, 0, 0}, sgtb = 0.0, Sdab = 0.0;
  double ichib = 0.0;

  // ---- fluid momentum
  for (int i = 0; i < 3; ++i) {
    const double q = -R.E * in.dalpha[i] + (R.S[0] * db[0][i] + R.S[1] * db[1][i] + R.S[2] * db[2][i]) +
                     0.5 * alpha * (T.sg[i] * T.ichi - T.sgt * in.dchi[i] * (T.ichi * T.ichi));
    im32b += rb[F_ST + i] * q;
    const double qb = rb[F_ST + i] * T.im32;
    B.E -= qb * in.dalpha[i];
    b.dalpha[i] -= qb * R.E;
    for (int k = 0; k < 3; ++k) {
      B.S[k] += qb * db[k][i];
      b.dbeta[k][i] += qb * R.S[k];
    }
    const double Tt = T.sg[i] * T.ichi - T.sgt * in.dchi[i] * (T.ichi * T.ichi);
    b.alpha += qb * 0.5 * Tt;
    const double Ttb = qb * 0.5 * alpha;
    sgb[i] += Ttb * T.ichi;
    ichib += Ttb * T.sg[i];
    sgtb -= Ttb * in.dchi[i] * T.ichi * T.ichi;
    b.dchi[i] -= Ttb * T.sgt * T.ichi * T.ichi;
    ichib -= Ttb * T.sgt * in.dchi[i] * 2.0 * T.ichi;
  }
  // ---- fluid energy
  im32b += rb[F_ET] * (alpha * T.KS - T.Sda);
  b.alpha += rb[F_ET] * T.im32 * T.KS;
  KSb += rb[F_ET] * T.im32 * alpha;
  Sdab -= rb[F_ET] * T.im32;
  for (int j = 0; j < 3; ++j) {
    B.Sup[j] += Sdab * in.dalpha[j];
    b.dalpha[j] += Sdab * R.Sup[j];
  }
  for (int s = 0; s < 6; ++s) {
    Sjkb[s] += sgtb * wsym(s) * gt[s];
    b.gt[s] += sgtb * wsym(s) * T.Sjk[s];
    for (int a = 0; a < 3; ++a) {
      Sjkb[s] += sgb[a] * wsym(s) * in.dgt[s][a];
      b.dgt[s][a] += sgb[a] * wsym(s) * T.Sjk[s];
    }
    Kijb[s] += KSb * wsym(s) * T.Sjk[s];
    Sjkb[s] += KSb * wsym(s) * T.Kij[s];
    b.At[s] += Kijb[s] / chi;
    b.gt[s] += Kijb[s] * K / (3.0 * chi);
    b.K += Kijb[s] * gt[s] / (3.0 * chi);
    b.chi -= Kijb[s] * T.Kij[s] / chi;
  }
  {  // im32 = 1 / (chi sqrt(chi))
    const double vb = -im32b * T.im32 * T.im32;
    const double sq = sqrt(chi);
    b.chi += vb * sq + vb * chi * 0.5 / sq;
  }
  // ---- gauge
  if (P.evolve_shift)
    for (int i = 0; i < 3; ++i) {
      b.Gam[i] += 0.75 * rb[F_BET + i];
      b.beta[i] -= P.eta * rb[F_BET + i];
    }
  b.alpha -= 2.0 * (K - T.Kbg) * rb[F_ALP];
  b.K -= 2.0 * alpha * rb[F_ALP];
  // ---- connection functions
  for (int i = 0; i < 3; ++i) {
    const double r = rb[F_GAM + i];
    for (int k = 0; k < 3; ++k) {
      Gdb[k] -= r * db[i][k];
      b.dbeta[i][k] -= r * T.Gd[k];
    }
    Gdb[i] += r * (2.0 / 3.0) * T.divb;
    divbb += r * (2.0 / 3.0) * T.Gd[i];
    for (int s = 0; s < 6; ++s) {
      gib[s] += r * wsym(s) * in.d2beta[i][s];
      b.d2beta[i][s] += r * wsym(s) * gi[s];
    }
    for (int l = 0; l < 3; ++l) {
      const double Y = in.d2beta[0][S(l, 0)] + in.d2beta[1][S(l, 1)] + in.d2beta[2][S(l, 2)];
      gib[S(i, l)] += r * Y * (1.0 / 3.0);
      for (int k = 0; k < 3; ++k) b.d2beta[k][S(l, k)] += r * gi[S(i, l)] * (1.0 / 3.0);
    }
    for (int j = 0; j < 3; ++j) {
      Aupb[S(i, j)] -= 2.0 * r * in.dalpha[j];
      b.dalpha[j] -= 2.0 * r * T.Aup[S(i, j)];
    }
    const double Z = T.Aup[S(i, 0)] * in.dchi[0] + T.Aup[S(i, 1)] * in.dchi[1] + T.Aup[S(i, 2)] * in.dchi[2];
    const double W = gi[S(i, 0)] * in.dK[0] + gi[S(i, 1)] * in.dK[1] + gi[S(i, 2)] * in.dK[2];
    const double inner = contract_sym(T.Gu[i], T.Aup) - (1.5 / chi) * Z - (2.0 / 3.0) * W;
    b.alpha += 2.0 * r * inner;
    const double innb = 2.0 * r * alpha;
    for (int s = 0; s < 6; ++s) {
      Gub[i][s] += innb * wsym(s) * T.Aup[s];
      Aupb[s] += innb * wsym(s) * T.Gu[i][s];
    }
    const double Zb = -innb * 1.5 / chi;
    b.chi += innb * 1.5 * Z / (chi * chi);
    for (int j = 0; j < 3; ++j) {
      Aupb[S(i, j)] += Zb * in.dchi[j];
      b.dchi[j] += Zb * T.Aup[S(i, j)];
      gib[S(i, j)] -= innb * (2.0 / 3.0) * in.dK[j];
      b.dK[j] -= innb * (2.0 / 3.0) * gi[S(i, j)];
    }
    const double V = gi[S(i, 0)] * R.S[0] + gi[S(i, 1)] * R.S[1] + gi[S(i, 2)] * R.S[2];
    b.alpha -= 16.0 * PI_D * r * V;
    const double Vb = -16.0 * PI_D * r * alpha;
    for (int j = 0; j < 3; ++j) {
      gib[S(i, j)] += Vb * R.S[j];
      B.S[j] += Vb * gi[S(i, j)];
    }
  }
  // ---- traceless curvature
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    const double r = rb[F_AT + s];
    for (int k = 0; k < 3; ++k) {
      b.At[S(i, k)] += r * db[k][j];
      b.dbeta[k][j] += r * in.At[S(i, k)];
      b.At[S(j, k)] += r * db[k][i];
      b.dbeta[k][i] += r * in.At[S(j, k)];
    }
    b.At[s] -= (2.0 / 3.0) * r * T.divb;
    divbb -= (2.0 / 3.0) * r * in.At[s];
    b.chi += r * (T.X6[s] - gt[s] * T.trX * (1.0 / 3.0));
    X6b[s] += r * chi;
    b.gt[s] -= r * chi * T.trX * (1.0 / 3.0);
    trXb -= r * chi * gt[s] * (1.0 / 3.0);
    double AAij = 0.0;
    for (int k = 0; k < 3; ++k) AAij += in.At[S(i, k)] * T.Amix[k][j];
    b.alpha += r * (K * in.At[s] - 2.0 * AAij);
    b.K += r * alpha * in.At[s];
    b.At[s] += r * alpha * K;
    const double AAb = -2.0 * r * alpha;
    for (int k = 0; k < 3; ++k) {
      b.At[S(i, k)] += AAb * T.Amix[k][j];
      Amixb[k][j] += AAb * in.At[S(i, k)];
    }
  }
  for (int s = 0; s < 6; ++s) {
    gib[s] += trXb * wsym(s) * T.X6[s];
    X6b[s] += trXb * wsym(s) * gi[s];
  }
  for (int s = 0; s < 6; ++s) {
    DDab[s] -= X6b[s];
    b.alpha += X6b[s] * (T.Ric[s] - 8.0 * PI_D * T.Sij[s]);
    Ricb[s] += X6b[s] * alpha;
    Sijb[s] -= 8.0 * PI_D * X6b[s] * alpha;
  }
  // ---- trace K
  {
    const double r = rb[F_K];
    D2ab -= r;
    b.alpha += r * (T.AA + K * K * (1.0 / 3.0) + 4.0 * PI_D * (R.E + T.Str));
    AAb += r * alpha;
    b.K += r * alpha * 2.0 * K * (1.0 / 3.0);
    B.E += r * 4.0 * PI_D * alpha;
    Strb += r * 4.0 * PI_D * alpha;
  }
  // ---- conformal metric
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    const double r = rb[F_GT + s];
    for (int k = 0; k < 3; ++k) {
      b.gt[S(i, k)] += r * db[k][j];
      b.dbeta[k][j] += r * gt[S(i, k)];
      b.gt[S(j, k)] += r * db[k][i];
      b.dbeta[k][i] += r * gt[S(j, k)];
    }
    b.gt[s] -= (2.0 / 3.0) * r * T.divb;
    divbb -= (2.0 / 3.0) * r * gt[s];
    b.alpha -= 2.0 * r * in.At[s];
    b.At[s] -= 2.0 * r * alpha;
  }
  // ---- conformal factor
  {
    const double r = rb[F_CHI];
    b.chi += r * (2.0 / 3.0) * (alpha * K - T.divb);
    b.alpha += r * (2.0 / 3.0) * chi * K;
    b.K += r * (2.0 / 3.0) * chi * alpha;
    divbb -= r * (2.0 / 3.0) * chi;
  }
  b.dbeta[0][0] += divbb;
  b.dbeta[1][1] += divbb;
  b.dbeta[2][2] += divbb;
  // ---- At contractions
  for (int s = 0; s < 6; ++s) {
    b.At[s] += AAb * wsym(s) * T.Aup[s];
    Aupb[s] += AAb * wsym(s) * in.At[s];
  }
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    for (int l = 0; l < 3; ++l) {
      Amixb[i][l] += Aupb[s] * gi[S(l, j)];
      gib[S(l, j)] += Aupb[s] * T.Amix[i][l];
    }
  }
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      for (int l = 0; l < 3; ++l) {
        gib[S(k, l)] += Amixb[k][j] * in.At[S(l, j)];
        b.At[S(l, j)] += Amixb[k][j] * gi[S(k, l)];
      }
  // ---- lapse Hessian
  {
    const double c2 = contract_sym(gi, T.DDa);
    b.chi += D2ab * c2;
    const double Cg = D2ab * chi;
    for (int s = 0; s < 6; ++s) {
      gib[s] += Cg * wsym(s) * T.DDa[s];
      DDab[s] += Cg * wsym(s) * gi[s];
    }
  }
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    b.d2alpha[s] += DDab[s];
    for (int k = 0; k < 3; ++k) {
      Gub[k][s] -= DDab[s] * in.dalpha[k];
      b.dalpha[k] -= DDab[s] * T.Gu[k][s];
    }
    const double Wv = (in.dchi[i] * in.dalpha[j] + in.dchi[j] * in.dalpha[i]) - gt[s] * T.cda;
    const double Wb = DDab[s] * (0.5 / chi);
    b.chi -= DDab[s] * Wv * 0.5 / (chi * chi);
    b.dchi[i] += Wb * in.dalpha[j];
    b.dalpha[j] += Wb * in.dchi[i];
    b.dchi[j] += Wb * in.dalpha[i];
    b.dalpha[i] += Wb * in.dchi[j];
    b.gt[s] -= Wb * T.cda;
    cdab -= Wb * gt[s];
  }
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      gib[S(k, l)] += cdab * in.dchi[k] * in.dalpha[l];
      b.dchi[k] += cdab * gi[S(k, l)] * in.dalpha[l];
      b.dalpha[l] += cdab * gi[S(k, l)] * in.dchi[k];
    }
  // ---- Ricci: conformal-factor part
  {
    const double ih = 0.5 / chi, iq = 0.25 / (chi * chi);
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      const double r = Ricb[s];
      DDchib[s] += r * ih;
      b.gt[s] += r * ih * T.trDD;
      trDDb += r * ih * gt[s];
      b.chi -= r * (T.DDchi[s] + gt[s] * T.trDD) * 0.5 / (chi * chi);
      b.dchi[i] -= r * iq * in.dchi[j];
      b.dchi[j] -= r * iq * in.dchi[i];
      b.gt[s] -= r * iq * 3.0 * T.dc2;
      dc2b -= r * iq * 3.0 * gt[s];
      b.chi += r * (in.dchi[i] * in.dchi[j] + 3.0 * gt[s] * T.dc2) * 0.5 / (chi * chi * chi);
    }
  }
  for (int l = 0; l < 3; ++l)
    for (int m = 0; m < 3; ++m) {
      gib[S(l, m)] += dc2b * in.dchi[l] * in.dchi[m];
      b.dchi[l] += dc2b * gi[S(l, m)] * in.dchi[m];
      b.dchi[m] += dc2b * gi[S(l, m)] * in.dchi[l];
    }
  for (int s = 0; s < 6; ++s) {
    gib[s] += trDDb * wsym(s) * T.DDchi[s];
    DDchib[s] += trDDb * wsym(s) * gi[s];
  }
  for (int s = 0; s < 6; ++s) {
    b.d2chi[s] += DDchib[s];
    for (int k = 0; k < 3; ++k) {
      Gub[k][s] -= DDchib[s] * in.dchi[k];
      b.dchi[k] -= DDchib[s] * T.Gu[k][s];
    }
  }
  // ---- Ricci: metric part
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    const double r = Ricb[s];
    for (int q = 0; q < 6; ++q) {
      gib[q] -= 0.5 * r * wsym(q) * in.d2gt[s][q];
      b.d2gt[s][q] -= 0.5 * r * wsym(q) * gi[q];
    }
    for (int k = 0; k < 3; ++k) {
      b.gt[S(k, i)] += 0.5 * r * in.dGam[k][j];
      b.dGam[k][j] += 0.5 * r * gt[S(k, i)];
      b.gt[S(k, j)] += 0.5 * r * in.dGam[k][i];
      b.dGam[k][i] += 0.5 * r * gt[S(k, j)];
      Gdb[k] += 0.5 * r * (T.Gl[i][S(j, k)] + T.Gl[j][S(i, k)]);
      Glb[i][S(j, k)] += 0.5 * r * T.Gd[k];
      Glb[j][S(i, k)] += 0.5 * r * T.Gd[k];
    }
    for (int l = 0; l < 3; ++l)
      for (int m = 0; m < 3; ++m) {
        const double g = gi[S(l, m)];
        for (int k = 0; k < 3; ++k) {
          const double term = (T.Gu[k][S(l, i)] * T.Gl[j][S(k, m)] + T.Gu[k][S(l, j)] * T.Gl[i][S(k, m)]) +
                              T.Gu[k][S(i, m)] * T.Gl[k][S(l, j)];
          gib[S(l, m)] += r * term;
          Gub[k][S(l, i)] += r * g * T.Gl[j][S(k, m)];
          Glb[j][S(k, m)] += r * g * T.Gu[k][S(l, i)];
          Gub[k][S(l, j)] += r * g * T.Gl[i][S(k, m)];
          Glb[i][S(k, m)] += r * g * T.Gu[k][S(l, j)];
          Gub[k][S(i, m)] += r * g * T.Gl[k][S(l, j)];
          Glb[k][S(l, j)] += r * g * T.Gu[k][S(i, m)];
        }
      }
  }
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 6; ++s) {
      gib[s] += Gdb[k] * wsym(s) * T.Gu[k][s];
      Gub[k][s] += Gdb[k] * wsym(s) * gi[s];
    }
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 6; ++s)
      for (int l = 0; l < 3; ++l) {
        gib[S(k, l)] += Gub[k][s] * T.Gl[l][s];
        Glb[l][s] += Gub[k][s] * gi[S(k, l)];
      }
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      b.dgt[S(k, j)][i] += 0.5 * Glb[k][s];
      b.dgt[S(k, i)][j] += 0.5 * Glb[k][s];
      b.dgt[s][k] -= 0.5 * Glb[k][s];
    }
  // ---- matter projections
  B.S2 += Strb * R.invX;
  B.invX += Strb * R.S2;
  B.P += 3.0 * Strb;
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    B.S[i] += Sijb[s] * R.S[j] * R.invX;
    B.S[j] += Sijb[s] * R.S[i] * R.invX;
    B.invX += Sijb[s] * R.S[i] * R.S[j];
    B.P += Sijb[s] * gt[s] * T.ichi;
    b.gt[s] += Sijb[s] * R.P * T.ichi;
    ichib += Sijb[s] * R.P * gt[s];
    B.Sup[i] += Sjkb[s] * R.Sup[j] * R.invX;
    B.Sup[j] += Sjkb[s] * R.Sup[i] * R.invX;
    B.invX += Sjkb[s] * R.Sup[i] * R.Sup[j];
    B.P += Sjkb[s] * chi * gi[s];
    b.chi += Sjkb[s] * R.P * gi[s];
    gib[s] += Sjkb[s] * R.P * chi;
  }
  b.chi -= ichib * T.ichi * T.ichi;
  rec_reverse(P.w, chi, gi, in.Et, in.St, R, B, b.chi, gib, b.Et, b.St);
  inv_reverse(gt, T.I, gib, b.gt);
}

}  // namespace cosmos
