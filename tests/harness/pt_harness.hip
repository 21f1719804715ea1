// Host-side harness (tests only): exposes the HIP path's pointwise reverse
// algebra, compiled for the CPU, so that the CPU tests can compare the
// hand-written vector-Jacobian products with the oracle's taped reverse mode.
#include "adjoint_point.hpp"

using namespace cosmos;

// Inputs of the pointwise algebra at one point, in the oracle's packed order.
// dX[c][a] = d_a X_c.
struct PtIn {
  double chi, gt[6], K, At[6], Gam[3], alpha, beta[3];
  double dchi[3], d2chi[6], dgt[6][3], d2gt[6][6], dGam[3][3], dalpha[3], d2alpha[6], dbeta[3][3], d2beta[3][6];
  double dK[3], dAt[6][3];  // dAt: constraint input, unused by the right-hand side
  double Et, St[3];
};

static void unpack(const double* a, double Et, const double* St, PtIn& in) {
  const double* q = a;
  in.chi = *q++;
  for (int s = 0; s < 6; ++s) in.gt[s] = *q++;
  in.K = *q++;
  for (int s = 0; s < 6; ++s) in.At[s] = *q++;
  for (int s = 0; s < 3; ++s) in.Gam[s] = *q++;
  in.alpha = *q++;
  for (int s = 0; s < 3; ++s) in.beta[s] = *q++;
  for (int s = 0; s < 3; ++s) in.dchi[s] = *q++;
  for (int s = 0; s < 6; ++s) in.d2chi[s] = *q++;
  for (int s = 0; s < 6; ++s)
    for (int a = 0; a < 3; ++a) in.dgt[s][a] = *q++;
  for (int s = 0; s < 6; ++s)
    for (int c = 0; c < 6; ++c) in.d2gt[s][c] = *q++;
  for (int s = 0; s < 3; ++s)
    for (int c = 0; c < 3; ++c) in.dGam[s][c] = *q++;
  for (int s = 0; s < 3; ++s) in.dalpha[s] = *q++;
  for (int s = 0; s < 6; ++s) in.d2alpha[s] = *q++;
  for (int s = 0; s < 3; ++s)
    for (int c = 0; c < 3; ++c) in.dbeta[s][c] = *q++;
  for (int s = 0; s < 3; ++s)
    for (int c = 0; c < 6; ++c) in.d2beta[s][c] = *q++;
  for (int s = 0; s < 3; ++s) in.dK[s] = *q++;
  for (int s = 0; s < 6; ++s)
    for (int c = 0; c < 3; ++c) in.dAt[s][c] = *q++;
  in.Et = Et;
  for (int c = 0; c < 3; ++c) in.St[c] = St[c];
}

static int pack(const PtIn& in, double* a) {
  double* q = a;
  *q++ = in.chi;
  for (int s = 0; s < 6; ++s) *q++ = in.gt[s];
  *q++ = in.K;
  for (int s = 0; s < 6; ++s) *q++ = in.At[s];
  for (int s = 0; s < 3; ++s) *q++ = in.Gam[s];
  *q++ = in.alpha;
  for (int s = 0; s < 3; ++s) *q++ = in.beta[s];
  for (int s = 0; s < 3; ++s) *q++ = in.dchi[s];
  for (int s = 0; s < 6; ++s) *q++ = in.d2chi[s];
  for (int s = 0; s < 6; ++s)
    for (int a2 = 0; a2 < 3; ++a2) *q++ = in.dgt[s][a2];
  for (int s = 0; s < 6; ++s)
    for (int c = 0; c < 6; ++c) *q++ = in.d2gt[s][c];
  for (int s = 0; s < 3; ++s)
    for (int c = 0; c < 3; ++c) *q++ = in.dGam[s][c];
  for (int s = 0; s < 3; ++s) *q++ = in.dalpha[s];
  for (int s = 0; s < 6; ++s) *q++ = in.d2alpha[s];
  for (int s = 0; s < 3; ++s)
    for (int c = 0; c < 3; ++c) *q++ = in.dbeta[s][c];
  for (int s = 0; s < 3; ++s)
    for (int c = 0; c < 6; ++c) *q++ = in.d2beta[s][c];
  for (int s = 0; s < 3; ++s) *q++ = in.dK[s];
  for (int s = 0; s < 6; ++s)
    for (int c = 0; c < 3; ++c) *q++ = in.dAt[s][c];
  *q++ = in.Et;
  for (int c = 0; c < 3; ++c) *q++ = in.St[c];
  return (int)(q - a);
}

static DevParams params(const double* prm, const int* iprm) {
  DevParams P = {};
  P.w = prm[0];
  P.H0 = prm[1];
  P.eta = prm[2];
  P.ko_eps = prm[3];
  P.lapse_bg = iprm[0];
  P.evolve_shift = iprm[1];
  return P;
}


// pt_vjp reading its differences from a PtIn and writing its cotangents into one
struct HostSrc {
  const PtIn& in;
  const double* rb;
  double cot(int f) const { return rb[f]; }
  double val(int f) const {
    if (f == F_CHI) return in.chi;
    if (f >= F_GT && f < F_GT + 6) return in.gt[f - F_GT];
    if (f == F_K) return in.K;
    if (f >= F_AT && f < F_AT + 6) return in.At[f - F_AT];
    if (f >= F_GAM && f < F_GAM + 3) return in.Gam[f - F_GAM];
    if (f == F_ALP) return in.alpha;
    if (f >= F_BET && f < F_BET + 3) return in.beta[f - F_BET];
    if (f == F_ET) return in.Et;
    return in.St[f - F_ST];
  }
  void copy3(const double* a, double d[3]) const {
    for (int c = 0; c < 3; ++c) d[c] = a[c];
  }
  void copy6(const double* a, double d[6]) const {
    for (int c = 0; c < 6; ++c) d[c] = a[c];
  }
  void d1(int f, double d[3]) const {
    if (f == F_CHI) copy3(in.dchi, d);
    else if (f >= F_GT && f < F_GT + 6) copy3(in.dgt[f - F_GT], d);
    else if (f == F_K) copy3(in.dK, d);
    else if (f >= F_GAM && f < F_GAM + 3) copy3(in.dGam[f - F_GAM], d);
    else if (f == F_ALP) copy3(in.dalpha, d);
    else copy3(in.dbeta[f - F_BET], d);
  }
  void d2(int f, double d[6]) const {
    if (f == F_CHI) copy6(in.d2chi, d);
    else if (f >= F_GT && f < F_GT + 6) copy6(in.d2gt[f - F_GT], d);
    else if (f == F_ALP) copy6(in.d2alpha, d);
    else copy6(in.d2beta[f - F_BET], d);
  }
  void d12(int f, double a[3], double b[6]) const {
    d1(f, a);
    d2(f, b);
  }
  void fence() const {}
  static void pin(double&) {}
};
struct HostSink {
  PtIn& b;
  int count = 0;
  double* val_slot(int f) {
    if (f == F_CHI) return &b.chi;
    if (f >= F_GT && f < F_GT + 6) return &b.gt[f - F_GT];
    if (f == F_K) return &b.K;
    if (f >= F_AT && f < F_AT + 6) return &b.At[f - F_AT];
    if (f >= F_GAM && f < F_GAM + 3) return &b.Gam[f - F_GAM];
    if (f == F_ALP) return &b.alpha;
    if (f >= F_BET && f < F_BET + 3) return &b.beta[f - F_BET];
    if (f == F_ET) return &b.Et;
    return &b.St[f - F_ST];
  }
  double* d1_slot(int f) {
    if (f == F_CHI) return b.dchi;
    if (f >= F_GT && f < F_GT + 6) return b.dgt[f - F_GT];
    if (f == F_K) return b.dK;
    if (f >= F_GAM && f < F_GAM + 3) return b.dGam[f - F_GAM];
    if (f == F_ALP) return b.dalpha;
    return b.dbeta[f - F_BET];
  }
  double* d2_slot(int f) {
    if (f == F_CHI) return b.d2chi;
    if (f >= F_GT && f < F_GT + 6) return b.d2gt[f - F_GT];
    if (f == F_ALP) return b.d2alpha;
    return b.d2beta[f - F_BET];
  }
  // every slot is written exactly once
  void val(int f, double v) {
    *val_slot(f) += v;
    ++count;
  }
  void d1(int f, int a, double v) {
    d1_slot(f)[a] += v;
    ++count;
  }
  void d2(int f, int q, double v) {
    d2_slot(f)[q] += v;
    ++count;
  }
};

extern "C" {
int harness_pt_vjp(const double* prm, const int* iprm, double t, const double* packed, double Et, const double* St,
                   const double* rbar, double* out) {
  PtIn in;
  unpack(packed, Et, St, in);
  const DevParams P = params(prm, iprm);
  HostSrc src{in, rbar};
  PtIn b = {};
  HostSink sink{b};
  pt_vjp(P, t, src, sink);
  // 25 point values, 45 first and 66 second differences
  if (sink.count != 136) return -sink.count;
  return pack(b, out);
}
// u15 = chi, gt[6], alpha, beta_a, Et, St[3]
int harness_flux(double w, int a, const double* u15, const double* Fb, double* F, double* ub) {
  FluxIn in = {u15[0], {u15[1], u15[2], u15[3], u15[4], u15[5], u15[6]}, u15[7], u15[8], u15[9],
               {u15[10], u15[11], u15[12]}};
  flux_forward(w, a, in, F);
  FluxIn b = {};
  flux_reverse(w, a, in, Fb, b);
  ub[0] = b.chi;
  for (int s = 0; s < 6; ++s) ub[1 + s] = b.gt[s];
  ub[7] = b.alpha;
  ub[8] = b.ba;
  ub[9] = b.Et;
  for (int c = 0; c < 3; ++c) ub[10 + c] = b.St[c];
  return 0;
}
}
