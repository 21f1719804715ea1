// Host-side harness (tests only): exposes the HIP path's pointwise forward and
// reverse algebra, compiled for the CPU, so that the CPU tests can compare the
// hand-written reverse sweep with the oracle's taped reverse mode.
#include "adjoint_point.hpp"

using namespace cosmos;

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

extern "C" {
int harness_pt_forward(const double* prm, const int* iprm, double t, const double* packed, double Et,
                       const double* St, double* r) {
  PtIn in;
  unpack(packed, Et, St, in);
  PtTape T;
  bool fail;
  pt_forward(params(prm, iprm), t, in, T, r, fail);
  return fail ? 1 : 0;
}
int harness_pt_vjp(const double* prm, const int* iprm, double t, const double* packed, double Et, const double* St,
                   const double* rbar, double* out) {
  PtIn in;
  unpack(packed, Et, St, in);
  PtTape T;
  double r[NF];
  bool fail;
  const DevParams P = params(prm, iprm);
  pt_forward(P, t, in, T, r, fail);
  PtIn b = {};
  pt_reverse(P, in, T, rbar, b);
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
