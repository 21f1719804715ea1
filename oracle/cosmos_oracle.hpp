// CPU oracle for the COSMOS evolution hot path -- TEST INFRASTRUCTURE ONLY.
//
// This is the plain, slow, serial FP64 statement of what the GPU path computes.
// It is used by tests/, by the smoke check and by the benchmark's CPU-baseline
// leg, never by the product path. It shares no source with the HIP library.
//
// What it computes (paper: "Physical system settings"):
//   * the Einstein equations with a perfect-fluid stress tensor T = (rho+P) u u + P g,
//     linear equation of state P = w rho, and the fluid equation of motion
//     div T = 0, rewritten in a 3+1 form "suitable for numerical integration";
//     the paper defers that rewrite to the standard numerical-relativity
//     textbooks, and this oracle uses the chi-form of the BSSN system (conformal
//     factor chi, conformal metric gt_ij, trace K, traceless At_ij, conformal
//     connection functions Gt^i) with densitised fluid variables;
//   * initial data of the paper's "Physical system settings" initial-data
//     paragraph: a curvature perturbation zeta(x) on a radiation FLRW background,
//     with the fluid energy density chosen so that the Hamiltonian constraint
//     holds at t = 0 (no elliptic solve);
//   * the discretisation the paper leaves open: 4th-order centred differences,
//     lopsided (upwinded) shift advection, 6th-difference Kreiss-Oliger
//     dissipation, periodic ghost zones of width 3, classic RK4 in time;
//   * the Hamiltonian and momentum constraints and their grid norms.
//
// Every function is a template over the scalar type T (double, or the Dual /
// Rev / Cnt types of ad.hpp). Branches test value(), so all scalars follow the
// branch the double evaluation takes.
//
// Layout of a state: SoA, u[f][k][j][i] with i (x) fastest, 25 fields in the
// order of enum Field below, no ghost points stored.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "ad.hpp"

namespace oracle {

using std::sqrt;
using std::exp;
using std::sin;
using std::cos;

// ------------------------------------------------------------------ fields
constexpr int NF = 25;
enum Field : int {
  CHI = 0,   // conformal factor chi = (det gamma)^(-1/3)
  GT = 1,    // gt_xx, gt_xy, gt_xz, gt_yy, gt_yz, gt_zz  (1..6)
  TRK = 7,   // K, trace of the extrinsic curvature
  AT = 8,    // At_xx .. At_zz  (8..13)
  GAM = 14,  // Gt^x, Gt^y, Gt^z  (14..16)
  ALP = 17,  // lapse alpha
  BET = 18,  // shift beta^x, beta^y, beta^z  (18..20)
  ET = 21,   // densitised energy density Et = chi^(-3/2) E
  ST = 22    // densitised momentum density St_i = chi^(-3/2) S_i  (22..24)
};
// symmetric 3x3 <-> 6-vector (xx, xy, xz, yy, yz, zz)
constexpr int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
constexpr int SI[6] = {0, 0, 0, 1, 1, 2};
constexpr int SJ[6] = {0, 1, 2, 1, 2, 2};
constexpr double PI = 3.14159265358979323846;

// ------------------------------------------------------------------ setup
// Periodic vertex-centred grid: x_i = -L/2 + i*h, h = L/n, point n/2 is the centre.
struct Grid {
  int n[3];
  double L[3];
  double h(int a) const { return L[a] / n[a]; }
  int64_t npts() const { return (int64_t)n[0] * n[1] * n[2]; }
};

struct Params {
  double w = 1.0 / 3.0;  // P = w rho
  double H0 = 1.0;       // Hubble rate of the background at t = 0
  double eta = 1.0;      // Gamma-driver damping
  double ko_eps = 0.1;   // Kreiss-Oliger strength
  int lapse_bg = 1;      // 1: lapse source uses K - K_bg(t); 0: plain 1+log
  int evolve_shift = 1;  // 1: Gamma-driver shift; 0: shift frozen
  int fluid_scheme = 0;  // 0: centred 4th-order flux divergence + KO; 1: Kurganov-Tadmor interface fluxes
};

enum Profile : int { GAUSS = 0, SINE = 1, PGAUSS = 2 };
enum DensityMode : int { HAMILTONIAN = 0, LITERAL = 1 };
struct InitSpec {
  double mu = 0.1, sigma = 1.0;
  double center[3] = {0, 0, 0};
  double noise_amp = 0.0;
  uint64_t seed = 2606;
  int profile = GAUSS;
  int density_mode = HAMILTONIAN;
  // iso-curvature mode of the massless scalar field: Upsilon(x) = sc_mu * (profile
  // above with width sc_sigma) about the same centre (sc_mu = 0: no scalar field)
  double sc_mu = 0.0, sc_sigma = 1.0;
};

struct Status {
  int64_t prim_fail = 0;  // primitive-recovery failures (centre points only)
};

// ------------------------------------------------------------------ ghost zones
constexpr int NG = 3;  // stencil reach of the upwind and dissipation operators

// A window of m[0] x m[1] x m[2] points of all 25 fields, padded by NG ghost
// points on every side.
template <class T>
struct Padded {
  int m[3] = {0, 0, 0};
  int p[3] = {0, 0, 0};
  std::vector<T> a;
  void resize(const int mm[3]) {
    for (int d = 0; d < 3; ++d) {
      m[d] = mm[d];
      p[d] = mm[d] + 2 * NG;
    }
    a.assign((size_t)NF * p[0] * p[1] * p[2], T(0.0));
  }
  size_t idx(int f, int i, int j, int k) const {
    return (size_t)(i + NG) + (size_t)p[0] * ((size_t)(j + NG) + (size_t)p[1] * ((size_t)(k + NG) + (size_t)p[2] * f));
  }
  T& operator()(int f, int i, int j, int k) { return a[idx(f, i, j, k)]; }
  const T& operator()(int f, int i, int j, int k) const { return a[idx(f, i, j, k)]; }
};

inline int wrap(int i, int n) { return ((i % n) + n) % n; }

// Periodic ghost fill: copy the window starting at o[] (interior plus NG ghosts)
// out of the periodic state u. With o = 0 and m = n this is the ordinary
// periodic ghost-zone fill of the whole grid.
template <class T>
void pad_periodic(const Grid& g, const T* u, const int o[3], const int m[3], Padded<T>& P, int nfields = NF) {
  P.resize(m);
  const int64_t N3 = g.npts();
  for (int f = 0; f < nfields; ++f)
    for (int k = -NG; k < m[2] + NG; ++k)
      for (int j = -NG; j < m[1] + NG; ++j)
        for (int i = -NG; i < m[0] + NG; ++i) {
          int I = wrap(o[0] + i, g.n[0]), J = wrap(o[1] + j, g.n[1]), K = wrap(o[2] + k, g.n[2]);
          P(f, i, j, k) = u[f * N3 + I + (int64_t)g.n[0] * (J + (int64_t)g.n[1] * K)];
        }
}

// ------------------------------------------------------------------ stencils
// 4th-order centred first derivative along axis a:  (f[-2] - 8f[-1] + 8f[+1] - f[+2]) / 12h
// 4th-order centred second derivative:  (-f[-2] + 16f[-1] - 30f[0] + 16f[+1] - f[+2]) / 12h^2
// mixed second derivative: D1 along a of D1 along b
// lopsided advection:  U+ (beta > 0) = (-3f[-1] - 10f[0] + 18f[+1] - 6f[+2] + f[+3]) / 12h
//                      U- (beta <= 0) = (3f[+1] + 10f[0] - 18f[-1] + 6f[-2] - f[-3]) / 12h
// Kreiss-Oliger: (eps/64) sum_a (f[-3] - 6f[-2] + 15f[-1] - 20f[0] + 15f[+1] - 6f[+2] + f[+3]) / h_a
struct Stencil {
  const double* h;  // grid spacing per axis
  static constexpr double C1[4] = {1.0, -8.0, 8.0, -1.0};  // offsets -2,-1,+1,+2
  static constexpr int O1[4] = {-2, -1, 1, 2};
  static constexpr double C2[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};  // offsets -2..+2
  static constexpr double CUP[5] = {-3.0, -10.0, 18.0, -6.0, 1.0};  // offsets -1..+3
  static constexpr double CUM[5] = {-1.0, 6.0, -18.0, 10.0, 3.0};  // offsets -3..+1
  static constexpr double CKO[7] = {1.0, -6.0, 15.0, -20.0, 15.0, -6.0, 1.0};  // offsets -3..+3
};

template <class T>
inline T tap(const Padded<T>& P, int f, int i, int j, int k, int a, int off) {
  int d[3] = {0, 0, 0};
  d[a] = off;
  return P(f, i + d[0], j + d[1], k + d[2]);
}

template <class T>
T D1(const Padded<T>& P, const double* h, int f, int i, int j, int k, int a) {
  T v[4];
  for (int q = 0; q < 4; ++q) v[q] = tap(P, f, i, j, k, a, Stencil::O1[q]);
  return lincomb(v, Stencil::C1, 4) * T(1.0 / (12.0 * h[a]));
}

template <class T>
T D2(const Padded<T>& P, const double* h, int f, int i, int j, int k, int a) {
  T v[5];
  for (int q = 0; q < 5; ++q) v[q] = tap(P, f, i, j, k, a, q - 2);
  return lincomb(v, Stencil::C2, 5) * T(1.0 / (12.0 * h[a] * h[a]));
}

// D1_a (D1_b f), a != b
template <class T>
T Dmixed(const Padded<T>& P, const double* h, int f, int i, int j, int k, int a, int b) {
  T inner[4];
  for (int q = 0; q < 4; ++q) {
    int d[3] = {0, 0, 0};
    d[a] = Stencil::O1[q];
    inner[q] = D1(P, h, f, i + d[0], j + d[1], k + d[2], b);
  }
  return lincomb(inner, Stencil::C1, 4) * T(1.0 / (12.0 * h[a]));
}

// second derivative, symmetric component ab (a <= b)
template <class T>
T Dsecond(const Padded<T>& P, const double* h, int f, int i, int j, int k, int a, int b) {
  return a == b ? D2(P, h, f, i, j, k, a) : Dmixed(P, h, f, i, j, k, a, b);
}

// beta^a d_a f with the one-sided stencil chosen by the sign of beta^a at the point
template <class T>
T Advect(const Padded<T>& P, const double* h, int f, int i, int j, int k, const T beta[3]) {
  T s = T(0.0);
  for (int a = 0; a < 3; ++a) {
    T v[5];
    T d;
    if (value(beta[a]) > 0.0) {
      for (int q = 0; q < 5; ++q) v[q] = tap(P, f, i, j, k, a, q - 1);
      d = lincomb(v, Stencil::CUP, 5) * T(1.0 / (12.0 * h[a]));
    } else {
      for (int q = 0; q < 5; ++q) v[q] = tap(P, f, i, j, k, a, q - 3);
      d = lincomb(v, Stencil::CUM, 5) * T(1.0 / (12.0 * h[a]));
    }
    s = s + beta[a] * d;
  }
  return s;
}

template <class T>
T KO(const Padded<T>& P, const double* h, double eps, int f, int i, int j, int k) {
  T s = T(0.0);
  for (int a = 0; a < 3; ++a) {
    T v[7];
    for (int q = 0; q < 7; ++q) v[q] = tap(P, f, i, j, k, a, q - 3);
    s = s + lincomb(v, Stencil::CKO, 7) * T(1.0 / h[a]);
  }
  return T(eps / 64.0) * s;
}

// ------------------------------------------------------------------ geometry
// Conformal inverse metric (full inverse; det gt = 1 is not assumed).
template <class T>
void inverse_sym(const T g[6], T gi[6], T& det) {
  T c00 = g[3] * g[5] - g[4] * g[4];
  T c01 = g[2] * g[4] - g[1] * g[5];
  T c02 = g[1] * g[4] - g[2] * g[3];
  T c11 = g[0] * g[5] - g[2] * g[2];
  T c12 = g[1] * g[2] - g[0] * g[4];
  T c22 = g[0] * g[3] - g[1] * g[1];
  det = g[0] * c00 + g[1] * c01 + g[2] * c02;
  T id = T(1.0) / det;
  gi[0] = c00 * id;
  gi[1] = c01 * id;
  gi[2] = c02 * id;
  gi[3] = c11 * id;
  gi[4] = c12 * id;
  gi[5] = c22 * id;
}

// Derivatives of the geometric fields at one point, as inputs to the
// pointwise algebra. Index conventions: dX[c][a] = d_a X_c, with c a symmetric
// component (SYM) or a vector index.
template <class T>
struct GeomIn {
  T chi, gt[6], K, At[6], Gam[3], alpha, beta[3];
  T dchi[3], d2chi[6];
  T dgt[6][3], d2gt[6][6];
  T dGam[3][3];     // dGam[k][j] = d_j Gt^k (evolved)
  T dalpha[3], d2alpha[6];
  T dbeta[3][3];    // dbeta[i][j] = d_j beta^i
  T d2beta[3][6];
  T dK[3];
  T dAt[6][3];      // momentum constraint only
};

// Conformal connection, Ricci tensor and the related quantities.
template <class T>
struct Geom {
  T gi[6], det;
  T Gl[3][6];  // Gt_kij = 1/2 (d_i gt_kj + d_j gt_ki - d_k gt_ij)
  T Gu[3][6];  // Gt^k_ij = gt^kl Gt_lij
  T Gd[3];     // Gt^k computed from the metric: gt^ij Gt^k_ij
  T Ric[6];    // R_ij = Rt_ij + R^chi_ij
  T R;         // chi gt^ij R_ij
};

template <class T>
void geometry(const GeomIn<T>& in, Geom<T>& G) {
  inverse_sym(in.gt, G.gi, G.det);
  const T* gi = G.gi;
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 6; ++s) {
      int i = SI[s], j = SJ[s];
      G.Gl[k][s] = T(0.5) * (in.dgt[SYM[k][j]][i] + in.dgt[SYM[k][i]][j] - in.dgt[s][k]);
    }
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 6; ++s) {
      T acc = T(0.0);
      for (int l = 0; l < 3; ++l) acc = acc + gi[SYM[k][l]] * G.Gl[l][s];
      G.Gu[k][s] = acc;
    }
  for (int k = 0; k < 3; ++k) {
    T acc = T(0.0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) acc = acc + gi[SYM[i][j]] * G.Gu[k][SYM[i][j]];
    G.Gd[k] = acc;
  }
  // conformal Ricci tensor Rt_ij
  for (int s = 0; s < 6; ++s) {
    int i = SI[s], j = SJ[s];
    T r = T(0.0);
    for (int l = 0; l < 3; ++l)
      for (int m = 0; m < 3; ++m) r = r - T(0.5) * gi[SYM[l][m]] * in.d2gt[s][SYM[l][m]];
    for (int k = 0; k < 3; ++k)
      r = r + T(0.5) * (in.gt[SYM[k][i]] * in.dGam[k][j] + in.gt[SYM[k][j]] * in.dGam[k][i]);
    for (int k = 0; k < 3; ++k) r = r + T(0.5) * G.Gd[k] * (G.Gl[i][SYM[j][k]] + G.Gl[j][SYM[i][k]]);
    for (int l = 0; l < 3; ++l)
      for (int m = 0; m < 3; ++m) {
        T gl = gi[SYM[l][m]];
        for (int k = 0; k < 3; ++k) {
          r = r + gl * (G.Gu[k][SYM[l][i]] * G.Gl[j][SYM[k][m]] + G.Gu[k][SYM[l][j]] * G.Gl[i][SYM[k][m]] +
                        G.Gu[k][SYM[i][m]] * G.Gl[k][SYM[l][j]]);
        }
      }
    G.Ric[s] = r;
  }
  // conformal-factor part R^chi_ij
  T DDchi[6];
  for (int s = 0; s < 6; ++s) {
    T acc = in.d2chi[s];
    for (int k = 0; k < 3; ++k) acc = acc - G.Gu[k][s] * in.dchi[k];
    DDchi[s] = acc;
  }
  T trDD = T(0.0), dchi2 = T(0.0);
  for (int l = 0; l < 3; ++l)
    for (int m = 0; m < 3; ++m) {
      trDD = trDD + gi[SYM[l][m]] * DDchi[SYM[l][m]];
      dchi2 = dchi2 + gi[SYM[l][m]] * in.dchi[l] * in.dchi[m];
    }
  for (int s = 0; s < 6; ++s) {
    int i = SI[s], j = SJ[s];
    T rc = (DDchi[s] + in.gt[s] * trDD) / (T(2.0) * in.chi) -
           (in.dchi[i] * in.dchi[j] + T(3.0) * in.gt[s] * dchi2) / (T(4.0) * in.chi * in.chi);
    G.Ric[s] = G.Ric[s] + rc;
  }
  T R = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R = R + gi[SYM[i][j]] * G.Ric[SYM[i][j]];
  G.R = in.chi * R;
}

// Physical second covariant derivative of the lapse, D_i D_j alpha.
template <class T>
void ddalpha(const GeomIn<T>& in, const Geom<T>& G, T DDa[6]) {
  T dchida = T(0.0);
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) dchida = dchida + G.gi[SYM[k][l]] * in.dchi[k] * in.dalpha[l];
  for (int s = 0; s < 6; ++s) {
    int i = SI[s], j = SJ[s];
    T acc = in.d2alpha[s];
    for (int k = 0; k < 3; ++k) acc = acc - G.Gu[k][s] * in.dalpha[k];
    acc = acc + (in.dchi[i] * in.dalpha[j] + in.dchi[j] * in.dalpha[i] - in.gt[s] * dchida) / (T(2.0) * in.chi);
    DDa[s] = acc;
  }
}

// ------------------------------------------------------------------ matter
// Radiation fluid (perfect fluid, P = w rho). From the conserved energy and
// momentum densities E, S_i measured by the normal observer, X = (rho+P) W^2
// solves X^2 - (1+w) E X + w S^2 = 0 (larger root); then P = X - E.
template <class T>
struct Matter {
  T E, S[3];     // physical (not densitised) E and S_i
  T S2;          // gamma^ij S_i S_j
  T P, invX;     // pressure and 1/X (invX = 0 when the fluid state is invalid)
  T Sup[3];      // S^i = gamma^ij S_j
  T Sij[6];      // S_ij = S_i S_j / X + P gamma_ij
  T Strace;      // gamma^ij S_ij
  T Sjk[6];      // S^jk = S^j S^k / X + P gamma^jk
};

template <class T>
bool matter(const Params& p, T chi, const T gt[6], const T gi[6], T Et, const T St[3], Matter<T>& M,
            bool want_stress = true) {
  bool fail = false;
  T c32 = chi * sqrt(chi);
  M.E = c32 * Et;
  for (int i = 0; i < 3; ++i) M.S[i] = c32 * St[i];
  T s2 = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s2 = s2 + gi[SYM[i][j]] * M.S[i] * M.S[j];
  M.S2 = chi * s2;
  T X;
  if (!(value(M.E) > 0.0)) {
    fail = true;
    M.P = T(0.0);
    M.invX = T(0.0);
  } else {
    T opw = T(1.0 + p.w);
    T disc = opw * opw * M.E * M.E - T(4.0 * p.w) * M.S2;
    if (!(value(disc) >= 0.0)) {
      fail = true;
      disc = T(0.0);
    }
    X = T(0.5) * (opw * M.E + sqrt(disc));
    M.P = X - M.E;
    M.invX = T(1.0) / X;
  }
  for (int j = 0; j < 3; ++j) {
    T acc = T(0.0);
    for (int k = 0; k < 3; ++k) acc = acc + gi[SYM[j][k]] * M.S[k];
    M.Sup[j] = chi * acc;
  }
  if (!want_stress) return fail;  // fluxes and speeds need E, S_i, S^i, S^2, P, 1/X only
  for (int s = 0; s < 6; ++s) {
    int i = SI[s], j = SJ[s];
    M.Sij[s] = M.S[i] * M.S[j] * M.invX + M.P * gt[s] / chi;
    M.Sjk[s] = M.Sup[i] * M.Sup[j] * M.invX + M.P * chi * gi[s];
  }
  M.Strace = M.S2 * M.invX + T(3.0) * M.P;
  return fail;
}

// Fluxes of the densitised fluid variables along direction j:
//   F^j_E = chi^(-3/2) (alpha S^j - beta^j E)
//   F^j_i = chi^(-3/2) (alpha (S^j S_i / X + P delta^j_i) - beta^j S_i)
// out[4*j + 0] = F^j_E, out[4*j + 1 + i] = F^j_i
template <class T>
void fluid_flux(const Params& p, const T u[NF], T out[12]) {
  T gt[6], gi[6], det, St[3], beta[3];
  for (int s = 0; s < 6; ++s) gt[s] = u[GT + s];
  inverse_sym(gt, gi, det);
  for (int i = 0; i < 3; ++i) {
    St[i] = u[ST + i];
    beta[i] = u[BET + i];
  }
  Matter<T> M;
  matter(p, u[CHI], gt, gi, u[ET], St, M, false);
  T chi = u[CHI];
  T im32 = T(1.0) / (chi * sqrt(chi));
  T alpha = u[ALP];
  for (int j = 0; j < 3; ++j) {
    out[4 * j] = im32 * (alpha * M.Sup[j] - beta[j] * M.E);
    for (int i = 0; i < 3; ++i) {
      T pd = (i == j) ? M.P : T(0.0);
      out[4 * j + 1 + i] = im32 * (alpha * (M.Sup[j] * M.S[i] * M.invX + pd) - beta[j] * M.S[i]);
    }
  }
}

// ------------------------------------------------------------------ massless scalar field
// The second matter field of the paper ("Physical system settings": the scalar
// stress tensor T^SC = d phi d phi - 1/2 g (d phi)^2 and the wave equation
// box phi = 0). Evolved as phi and Pi = n^mu d_mu phi (n the unit normal of the
// slices), held in a separate 2-field state s[PHI], s[PIF]. The 3+1 form of
// box phi = 0:
//   d_t phi = alpha Pi + beta^k d_k phi,
//   d_t Pi  = beta^k d_k Pi + alpha K Pi + alpha gamma^ij (d_i d_j phi - Gamma^k_ij d_k phi)
//             + gamma^ij d_i alpha d_j phi,
// with gamma^ij = chi gt^ij and gamma^ij Gamma^k_ij = chi Gd^k + 1/2 gt^kl d_l chi, where
// Gd^k = gt^ij Gt^k_ij is formed from the conformal metric's first derivatives (the same
// rule as in the geometry: the evolved Gt^k enter only through their own derivatives, their
// advection and the shift condition). This makes the operator the covariant Laplacian of
// the physical metric gt_ij / chi whatever the evolved Gt^k hold.
// Projections of T^SC on the normal frame (the sources of the geometry):
//   E = 1/2 (Pi^2 + |D phi|^2),  S_i = -Pi d_i phi,
//   S_ij = d_i phi d_j phi - 1/2 gamma_ij (|D phi|^2 - Pi^2),  S = 3/2 Pi^2 - 1/2 |D phi|^2.
constexpr int NS = 2;
enum ScalarField : int { PHI = 0, PIF = 1 };

template <class T>
struct ScalarIn {
  T Pi, dphi[3], d2phi[6];
};

template <class T>
struct ScalarSrc {
  T E, S[3], Sij[6], Strace;  // physical (not densitised)
};

template <class T>
void scalar_matter(T chi, const T gt[6], const T gi[6], const ScalarIn<T>& sc, ScalarSrc<T>& M) {
  T g2 = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) g2 = g2 + gi[SYM[i][j]] * sc.dphi[i] * sc.dphi[j];
  g2 = chi * g2;  // |D phi|^2
  const T P2 = sc.Pi * sc.Pi;
  M.E = T(0.5) * (P2 + g2);
  for (int i = 0; i < 3; ++i) M.S[i] = -sc.Pi * sc.dphi[i];
  for (int s = 0; s < 6; ++s) M.Sij[s] = sc.dphi[SI[s]] * sc.dphi[SJ[s]] - T(0.5) * (gt[s] / chi) * (g2 - P2);
  M.Strace = T(1.5) * P2 - T(0.5) * g2;
}

// ------------------------------------------------------------------ Kurganov-Tadmor fluxes
// The paper's fluid scheme (section "Physical system settings" cites Kurganov &
// Tadmor 2000 and Shibata & Font 2005): a semi-discrete central scheme in
// conservation form, d q_i/dt = -sum_a (Fh^a_{i+1/2} - Fh^a_{i-1/2}) / h_a + sources,
// with the numerical flux at the interface i+1/2 along axis a
//   Fh = 1/2 (F^a(q_L) + F^a(q_R)) - 1/2 c (q_R - q_L),
// q = (Et, St_i) the densitised conserved variables reconstructed piecewise
// linearly with the minmod limiter,
//   q_L = q_i + s_i / 2,  q_R = q_{i+1} - s_{i+1} / 2,  s_i = minmod(q_i - q_{i-1}, q_{i+1} - q_i),
// and c the largest characteristic speed magnitude of the two interface states.
// The geometric fields at the interface are the average of the two neighbours.

// minmod(a, b): the argument of smaller magnitude when both have the same strict
// sign, else 0 (equal magnitudes give the same value either way).
template <class T>
T minmod(const T& a, const T& b) {
  if (value(a) > 0.0 && value(b) > 0.0) return value(a) < value(b) ? a : b;
  if (value(a) < 0.0 && value(b) < 0.0) return value(a) > value(b) ? a : b;
  return T(0.0);
}

// Characteristic speeds of the perfect fluid along axis a (the sound-wave pair
// of the relativistic Euler equations in 3+1 form, e.g. Banyuls et al. 1997;
// sound speed cs^2 = w for P = w rho):
//   lambda_pm = alpha / (1 - v^2 cs^2) [v^a (1 - cs^2)
//                 pm cs sqrt((1 - v^2)(gamma^aa (1 - v^2 cs^2) - (v^a)^2 (1 - cs^2)))] - beta^a
// with the Eulerian velocity v^i = S^i / X and v^2 = S^2 / X^2. A negative
// radicand (only possible at unphysical states) is taken as 0; a state whose
// recovery failed has invX = 0, hence v = 0.
template <class T>
void fluid_speeds(const Params& p, const T u[NF], int a, T& lm, T& lp) {
  T gt[6], gi[6], det, St[3];
  for (int s = 0; s < 6; ++s) gt[s] = u[GT + s];
  inverse_sym(gt, gi, det);
  for (int i = 0; i < 3; ++i) St[i] = u[ST + i];
  Matter<T> M;
  matter(p, u[CHI], gt, gi, u[ET], St, M, false);
  const T cs2 = T(p.w);
  const T cs = sqrt(cs2);
  const T va = M.Sup[a] * M.invX;
  const T v2 = M.S2 * M.invX * M.invX;
  const T gaa = u[CHI] * gi[SYM[a][a]];
  T rad = (T(1.0) - v2) * (gaa * (T(1.0) - v2 * cs2) - va * va * (T(1.0) - cs2));
  if (!(value(rad) > 0.0)) rad = T(0.0);
  const T root = value(rad) > 0.0 ? sqrt(rad) : T(0.0);
  const T f = u[ALP] / (T(1.0) - v2 * cs2);
  lp = f * (va * (T(1.0) - cs2) + cs * root) - u[BET + a];
  lm = f * (va * (T(1.0) - cs2) - cs * root) - u[BET + a];
}

template <class T>
T absval(const T& x) {
  return value(x) < 0.0 ? -x : x;
}

template <class T>
T maxval(const T& x, const T& y) {
  return value(y) > value(x) ? y : x;
}

// Numerical flux along axis a between the interface states uL and uR (25 values
// each): out[q] for q = Et, St_x, St_y, St_z.
template <class T>
void kt_flux(const Params& p, const T uL[NF], const T uR[NF], int a, T out[4]) {
  T FL[12], FR[12];
  fluid_flux(p, uL, FL);
  fluid_flux(p, uR, FR);
  T lmL, lpL, lmR, lpR;
  fluid_speeds(p, uL, a, lmL, lpL);
  fluid_speeds(p, uR, a, lmR, lpR);
  const T c = maxval(maxval(absval(lmL), absval(lpL)), maxval(absval(lmR), absval(lpR)));
  for (int q = 0; q < 4; ++q)
    out[q] = T(0.5) * (FL[4 * a + q] + FR[4 * a + q]) - T(0.5) * c * (uR[ET + q] - uL[ET + q]);
}

// Interface states at i+1/2 along axis a of the padded window, from the points
// i-1 .. i+2 along a: geometry averaged, fluid reconstructed.
template <class T, class Window>
void kt_interface_states(const Window& P, int i, int j, int k, int a, T uL[NF], T uR[NF]) {
  auto at = [&](int f, int o) {
    int d[3] = {0, 0, 0};
    d[a] = o;
    return P(f, i + d[0], j + d[1], k + d[2]);
  };
  for (int f = 0; f < ET; ++f) uL[f] = uR[f] = T(0.5) * (at(f, 0) + at(f, 1));
  for (int f = ET; f < NF; ++f) {
    const T qm = at(f, -1), q0 = at(f, 0), q1 = at(f, 1), q2 = at(f, 2);
    const T s0 = minmod(q0 - qm, q1 - q0);
    const T s1 = minmod(q1 - q0, q2 - q1);
    uL[f] = q0 + T(0.5) * s0;
    uR[f] = q1 - T(0.5) * s1;
  }
}

// ------------------------------------------------------------------ RHS
// Background trace K_bg(t) of the radiation FLRW universe with unit lapse:
// a(t) = (1 + 2 H0 t)^(1/2), H = H0 / (1 + 2 H0 t), K_bg = -3H.
inline double K_background(const Params& p, double t) {
  return p.lapse_bg ? -3.0 * p.H0 / (1.0 + 2.0 * p.H0 * t) : 0.0;
}

template <class T>
void gather_geom(const Padded<T>& P, const double* h, int i, int j, int k, GeomIn<T>& in, bool want_dAt) {
  in.chi = P(CHI, i, j, k);
  for (int s = 0; s < 6; ++s) in.gt[s] = P(GT + s, i, j, k);
  in.K = P(TRK, i, j, k);
  for (int s = 0; s < 6; ++s) in.At[s] = P(AT + s, i, j, k);
  for (int a = 0; a < 3; ++a) in.Gam[a] = P(GAM + a, i, j, k);
  in.alpha = P(ALP, i, j, k);
  for (int a = 0; a < 3; ++a) in.beta[a] = P(BET + a, i, j, k);
  for (int a = 0; a < 3; ++a) {
    in.dchi[a] = D1(P, h, CHI, i, j, k, a);
    in.dalpha[a] = D1(P, h, ALP, i, j, k, a);
    in.dK[a] = D1(P, h, TRK, i, j, k, a);
    for (int s = 0; s < 6; ++s) in.dgt[s][a] = D1(P, h, GT + s, i, j, k, a);
    for (int c = 0; c < 3; ++c) {
      in.dGam[c][a] = D1(P, h, GAM + c, i, j, k, a);
      in.dbeta[c][a] = D1(P, h, BET + c, i, j, k, a);
    }
    if (want_dAt)
      for (int s = 0; s < 6; ++s) in.dAt[s][a] = D1(P, h, AT + s, i, j, k, a);
  }
  for (int s = 0; s < 6; ++s) {
    int a = SI[s], b = SJ[s];
    in.d2chi[s] = Dsecond(P, h, CHI, i, j, k, a, b);
    in.d2alpha[s] = Dsecond(P, h, ALP, i, j, k, a, b);
    for (int q = 0; q < 6; ++q) in.d2gt[q][s] = Dsecond(P, h, GT + q, i, j, k, a, b);
    for (int c = 0; c < 3; ++c) in.d2beta[c][s] = Dsecond(P, h, BET + c, i, j, k, a, b);
  }
}

// Pointwise right-hand side of the BSSN + fluid system (without the advection,
// dissipation and flux-divergence terms, which rhs_padded adds).
// With a scalar field (sc non-null) its stress tensor adds to the sources of K,
// At and Gt, and sout[PHI], sout[PIF] receive its right-hand side (without the
// advection and dissipation terms, which the caller adds).
template <class T>
bool rhs_point(const Params& p, double t, const GeomIn<T>& in, T Et, const T St[3], T out[NF],
               const ScalarIn<T>* sc = nullptr, T* sout = nullptr) {
  Geom<T> G;
  geometry(in, G);
  const T* gi = G.gi;
  const T chi = in.chi, K = in.K, alpha = in.alpha;
  Matter<T> M;
  bool fail = matter(p, chi, in.gt, gi, Et, St, M);
  ScalarSrc<T> X;  // scalar-field sources (zero without a scalar field)
  X.E = X.Strace = T(0.0);
  for (int c = 0; c < 3; ++c) X.S[c] = T(0.0);
  for (int q = 0; q < 6; ++q) X.Sij[q] = T(0.0);
  if (sc) scalar_matter(chi, in.gt, gi, *sc, X);

  T DDa[6];
  ddalpha(in, G, DDa);
  T D2a = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D2a = D2a + gi[SYM[i][j]] * DDa[SYM[i][j]];
  D2a = chi * D2a;

  // raised / mixed At
  T Amix[3][3];  // Amix[k][j] = gt^kl At_lj
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) {
      T acc = T(0.0);
      for (int l = 0; l < 3; ++l) acc = acc + gi[SYM[k][l]] * in.At[SYM[l][j]];
      Amix[k][j] = acc;
    }
  T Aup[6];
  for (int s = 0; s < 6; ++s) {
    int i = SI[s], j = SJ[s];
    T acc = T(0.0);
    for (int l = 0; l < 3; ++l) acc = acc + Amix[i][l] * gi[SYM[l][j]];
    Aup[s] = acc;
  }
  T AA = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) AA = AA + in.At[SYM[i][j]] * Aup[SYM[i][j]];
  T divb = in.dbeta[0][0] + in.dbeta[1][1] + in.dbeta[2][2];
  const T pi4 = T(4.0 * PI), pi8 = T(8.0 * PI), pi16 = T(16.0 * PI);

  // chi
  out[CHI] = T(2.0 / 3.0) * chi * (alpha * K - divb);
  // gt_ij
  for (int s = 0; s < 6; ++s) {
    int i = SI[s], j = SJ[s];
    T acc = T(0.0);
    for (int k = 0; k < 3; ++k) acc = acc + in.gt[SYM[i][k]] * in.dbeta[k][j] + in.gt[SYM[j][k]] * in.dbeta[k][i];
    out[GT + s] = acc - T(2.0 / 3.0) * in.gt[s] * divb - T(2.0) * alpha * in.At[s];
  }
  // K
  T EpS = M.E + M.Strace;
  if (sc) EpS = EpS + (X.E + X.Strace);
  out[TRK] = -D2a + alpha * (AA + K * K / T(3.0)) + pi4 * alpha * EpS;
  // At_ij
  T Xs[6];
  for (int s = 0; s < 6; ++s) Xs[s] = -DDa[s] + alpha * (G.Ric[s] - pi8 * (sc ? M.Sij[s] + X.Sij[s] : M.Sij[s]));
  T trX = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) trX = trX + gi[SYM[i][j]] * Xs[SYM[i][j]];
  for (int s = 0; s < 6; ++s) {
    int i = SI[s], j = SJ[s];
    T acc = T(0.0);
    for (int k = 0; k < 3; ++k) acc = acc + in.At[SYM[i][k]] * in.dbeta[k][j] + in.At[SYM[j][k]] * in.dbeta[k][i];
    acc = acc - T(2.0 / 3.0) * in.At[s] * divb;
    acc = acc + chi * (Xs[s] - in.gt[s] * trX / T(3.0));
    T AAij = T(0.0);
    for (int k = 0; k < 3; ++k) AAij = AAij + in.At[SYM[i][k]] * Amix[k][j];
    out[AT + s] = acc + alpha * (K * in.At[s] - T(2.0) * AAij);
  }
  // Gt^i
  for (int i = 0; i < 3; ++i) {
    T acc = T(0.0);
    for (int k = 0; k < 3; ++k) acc = acc - G.Gd[k] * in.dbeta[i][k];
    acc = acc + T(2.0 / 3.0) * G.Gd[i] * divb;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) acc = acc + gi[SYM[j][k]] * in.d2beta[i][SYM[j][k]];
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) acc = acc + gi[SYM[i][j]] * in.d2beta[k][SYM[j][k]] / T(3.0);
    for (int j = 0; j < 3; ++j) acc = acc - T(2.0) * Aup[SYM[i][j]] * in.dalpha[j];
    T inner = T(0.0);
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) inner = inner + G.Gu[i][SYM[j][k]] * Aup[SYM[j][k]];
    for (int j = 0; j < 3; ++j) inner = inner - T(1.5) * Aup[SYM[i][j]] * in.dchi[j] / chi;
    for (int j = 0; j < 3; ++j) inner = inner - T(2.0 / 3.0) * gi[SYM[i][j]] * in.dK[j];
    acc = acc + T(2.0) * alpha * inner;
    T gS = T(0.0);
    for (int j = 0; j < 3; ++j) gS = gS + gi[SYM[i][j]] * (sc ? M.S[j] + X.S[j] : M.S[j]);
    out[GAM + i] = acc - pi16 * alpha * gS;
  }
  // gauge
  out[ALP] = T(-2.0) * alpha * (K - T(K_background(p, t)));
  for (int i = 0; i < 3; ++i)
    out[BET + i] = p.evolve_shift ? T(0.75) * in.Gam[i] - T(p.eta) * in.beta[i] : T(0.0);
  // fluid sources (the flux divergences are added by the caller)
  T im32 = T(1.0) / (chi * sqrt(chi));
  T KS = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T Kij = (in.At[SYM[i][j]] + in.gt[SYM[i][j]] * K / T(3.0)) / chi;
      KS = KS + Kij * M.Sjk[SYM[i][j]];
    }
  T Sda = T(0.0);
  for (int j = 0; j < 3; ++j) Sda = Sda + M.Sup[j] * in.dalpha[j];
  out[ET] = im32 * (alpha * KS - Sda);
  for (int i = 0; i < 3; ++i) {
    T acc = -M.E * in.dalpha[i];
    for (int k = 0; k < 3; ++k) acc = acc + M.S[k] * in.dbeta[k][i];
    T sg = T(0.0);
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        T dgam = in.dgt[SYM[j][k]][i] / chi - in.gt[SYM[j][k]] * in.dchi[i] / (chi * chi);
        sg = sg + M.Sjk[SYM[j][k]] * dgam;
      }
    out[ST + i] = im32 * (acc + alpha / T(2.0) * sg);
  }
  // scalar field
  if (sc && sout) {
    sout[PHI] = alpha * sc->Pi;
    T lap = T(0.0);  // gt^ij (d_i d_j phi) - (Gt^k + 1/(2 chi) gt^kl d_l chi) d_k phi, times chi below
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) lap = lap + gi[SYM[i][j]] * sc->d2phi[SYM[i][j]];
    for (int k = 0; k < 3; ++k) {
      T gk = G.Gd[k];  // contracted connection of the conformal metric (not the evolved Gt^k)
      for (int l = 0; l < 3; ++l) gk = gk + gi[SYM[k][l]] * in.dchi[l] / (T(2.0) * chi);
      lap = lap - gk * sc->dphi[k];
    }
    T dad = T(0.0);  // gt^ij d_i alpha d_j phi
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) dad = dad + gi[SYM[i][j]] * in.dalpha[i] * sc->dphi[j];
    sout[PIF] = alpha * K * sc->Pi + alpha * chi * lap + chi * dad;
  }
  return fail;
}

// Right-hand side on the interior of a padded window. out is SoA over the
// window: out[f*m0*m1*m2 + i + m0*(j + m1*k)].
// With a scalar field, Q is its padded window (fields PHI, PIF) and sout receives
// its right-hand side in the same layout as out (2 fields).
template <class T>
void rhs_padded(const Grid& g, const Params& p, double t, const Padded<T>& P, T* out, Status& st, bool parallel,
                const Padded<T>* Q = nullptr, T* sout = nullptr) {
  const double h[3] = {g.h(0), g.h(1), g.h(2)};
  const int* m = P.m;
  // fluxes at every padded point within reach 2 of the interior (pointwise)
  std::vector<T> F((size_t)12 * P.p[0] * P.p[1] * P.p[2]);
  auto fidx = [&](int c, int i, int j, int k) {
    return (size_t)c + 12 * ((size_t)(i + NG) + (size_t)P.p[0] * ((size_t)(j + NG) + (size_t)P.p[1] * (size_t)(k + NG)));
  };
  const bool par = parallel && std::is_same<T, double>::value;
  const bool kt = p.fluid_scheme == 1;
  if (!kt) {
#pragma omp parallel for schedule(static) if (par)
    for (int k = -2; k < m[2] + 2; ++k)
      for (int j = -2; j < m[1] + 2; ++j)
        for (int i = -2; i < m[0] + 2; ++i) {
          T u[NF];
          for (int f = 0; f < NF; ++f) u[f] = P(f, i, j, k);
          T fl[12];
          fluid_flux(p, u, fl);
          for (int c = 0; c < 12; ++c) F[fidx(c, i, j, k)] = fl[c];
        }
  } else {
    // F[4a + q] at (i, j, k) holds the KT flux through the interface at i+1/2 along a
#pragma omp parallel for schedule(static) if (par)
    for (int k = -1; k < m[2]; ++k)
      for (int j = -1; j < m[1]; ++j)
        for (int i = -1; i < m[0]; ++i)
          for (int a = 0; a < 3; ++a) {
            T uL[NF], uR[NF], fh[4];
            kt_interface_states<T>(P, i, j, k, a, uL, uR);
            kt_flux(p, uL, uR, a, fh);
            for (int q = 0; q < 4; ++q) F[fidx(4 * a + q, i, j, k)] = fh[q];
          }
  }
  const int64_t M3 = (int64_t)m[0] * m[1] * m[2];
  int64_t fails = 0;
#pragma omp parallel for schedule(static) reduction(+ : fails) if (par)
  for (int k = 0; k < m[2]; ++k)
    for (int j = 0; j < m[1]; ++j)
      for (int i = 0; i < m[0]; ++i) {
        GeomIn<T> in;
        gather_geom(P, h, i, j, k, in, false);
        T St[3] = {P(ST, i, j, k), P(ST + 1, i, j, k), P(ST + 2, i, j, k)};
        T r[NF], sr[NS];
        ScalarIn<T> sci;
        if (Q) {
          sci.Pi = (*Q)(PIF, i, j, k);
          for (int a = 0; a < 3; ++a) sci.dphi[a] = D1(*Q, h, PHI, i, j, k, a);
          for (int q = 0; q < 6; ++q) sci.d2phi[q] = Dsecond(*Q, h, PHI, i, j, k, SI[q], SJ[q]);
        }
        if (rhs_point(p, t, in, P(ET, i, j, k), St, r, Q ? &sci : nullptr, sr)) ++fails;
        // shift advection for the 21 geometric fields
        for (int f = 0; f < ET; ++f) {
          if (f >= BET && !p.evolve_shift) continue;
          r[f] = r[f] + Advect(P, h, f, i, j, k, in.beta);
        }
        // flux divergence for the fluid
        for (int c = 0; c < 4; ++c) {
          T div = T(0.0);
          for (int a = 0; a < 3; ++a) {
            if (kt) {
              int d[3] = {0, 0, 0};
              d[a] = -1;
              div = div + (F[fidx(4 * a + c, i, j, k)] - F[fidx(4 * a + c, i + d[0], j + d[1], k + d[2])]) *
                              T(1.0 / h[a]);
              continue;
            }
            T v[4];
            for (int q = 0; q < 4; ++q) {
              int d[3] = {0, 0, 0};
              d[a] = Stencil::O1[q];
              v[q] = F[fidx(4 * a + c, i + d[0], j + d[1], k + d[2])];
            }
            div = div + lincomb(v, Stencil::C1, 4) * T(1.0 / (12.0 * h[a]));
          }
          r[ET + c] = r[ET + c] - div;
        }
        // Kreiss-Oliger dissipation on every evolved field (with the KT scheme,
        // on the geometric fields only: the scheme carries its own dissipation)
        for (int f = 0; f < NF; ++f) {
          if (f >= BET && f < ET && !p.evolve_shift) continue;
          if (kt && f >= ET) continue;
          r[f] = r[f] + KO(P, h, p.ko_eps, f, i, j, k);
        }
        const int64_t q = i + (int64_t)m[0] * (j + (int64_t)m[1] * k);
        for (int f = 0; f < NF; ++f) out[f * M3 + q] = r[f];
        if (Q) {  // scalar field: shift advection and KO dissipation of phi and Pi
          for (int f = 0; f < NS; ++f) {
            sr[f] = sr[f] + Advect(*Q, h, f, i, j, k, in.beta);
            sr[f] = sr[f] + KO(*Q, h, p.ko_eps, f, i, j, k);
            sout[f * M3 + q] = sr[f];
          }
        }
      }
  st.prim_fail += fails;
}

// Right-hand side of the whole periodic grid (with the scalar field s, 2 x N3
// values, when s is non-null: its right-hand side goes to dsdt).
template <class T>
void rhs(const Grid& g, const Params& p, double t, const T* u, T* dudt, Status& st, bool parallel = false,
         const T* s = nullptr, T* dsdt = nullptr) {
  Padded<T> P, Q;
  const int o[3] = {0, 0, 0};
  pad_periodic(g, u, o, g.n, P);
  if (s) pad_periodic(g, s, o, g.n, Q, NS);
  rhs_padded(g, p, t, P, dudt, st, parallel, s ? &Q : nullptr, dsdt);
}

// Kurganov-Tadmor flux divergence alone on the whole periodic grid:
// div[q][p] = sum_a (Fh^a_q(p + 1/2) - Fh^a_q(p - 1/2)) / h_a, q = Et, St_x, St_y, St_z
// (the term the fluid right-hand side subtracts with fluid_scheme 1).
inline void kt_divergence(const Grid& g, const Params& p, const double* u, double* div) {
  Padded<double> P;
  const int o[3] = {0, 0, 0};
  pad_periodic(g, u, o, g.n, P);
  const int64_t N3 = g.npts();
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a) {
          int d[3] = {0, 0, 0};
          d[a] = -1;
          double uL[NF], uR[NF], fp[4], fm[4];
          kt_interface_states<double>(P, i, j, k, a, uL, uR);
          kt_flux(p, uL, uR, a, fp);
          kt_interface_states<double>(P, i + d[0], j + d[1], k + d[2], a, uL, uR);
          kt_flux(p, uL, uR, a, fm);
          for (int q = 0; q < 4; ++q) acc[q] = acc[q] + (fp[q] - fm[q]) * (1.0 / g.h(a));
        }
        const int64_t c = i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * k);
        for (int q = 0; q < 4; ++q) div[q * N3 + c] = acc[q];
      }
}

// ------------------------------------------------------------------ RK4
// Classic fourth-order Runge-Kutta:
//   k1 = f(t, u), k2 = f(t + dt/2, u + dt/2 k1), k3 = f(t + dt/2, u + dt/2 k2),
//   k4 = f(t + dt, u + dt k3),  u' = u + dt/6 (k1 + 2 k2 + 2 k3 + k4)
template <class T>
void rk4_step(const Grid& g, const Params& p, double t, double dt, T* u, Status& st, bool parallel = false,
              T* s = nullptr) {
  // with a scalar field the RK4 state is (u, s): both advance together
  const size_t n = (size_t)NF * g.npts(), ns = s ? (size_t)NS * g.npts() : 0;
  std::vector<T> k1(n + ns), k2(n + ns), k3(n + ns), k4(n + ns), U(n + ns);
  auto f = [&](double tt, const T* x, T* k) { rhs(g, p, tt, x, k, st, parallel, s ? x + n : nullptr, s ? k + n : nullptr); };
  std::vector<T> x0(n + ns);
  for (size_t q = 0; q < n; ++q) x0[q] = u[q];
  for (size_t q = 0; q < ns; ++q) x0[n + q] = s[q];
  f(t, x0.data(), k1.data());
  for (size_t q = 0; q < n + ns; ++q) U[q] = x0[q] + T(dt / 2.0) * k1[q];
  f(t + dt / 2.0, U.data(), k2.data());
  for (size_t q = 0; q < n + ns; ++q) U[q] = x0[q] + T(dt / 2.0) * k2[q];
  f(t + dt / 2.0, U.data(), k3.data());
  for (size_t q = 0; q < n + ns; ++q) U[q] = x0[q] + T(dt) * k3[q];
  f(t + dt, U.data(), k4.data());
  for (size_t q = 0; q < n + ns; ++q) {
    const T v = x0[q] + T(dt / 6.0) * (k1[q] + T(2.0) * k2[q] + T(2.0) * k3[q] + k4[q]);
    if (q < n) u[q] = v;
    else s[q - n] = v;
  }
}

// One RK4 step evaluated only at the listed points of a periodic grid, with
// the same arithmetic as rk4_step. The new value at a point depends on the
// state within 4*NG = 12 points along each axis, so stage s (s = 1..4) is
// formed on the window of radius 3*(4-s) around the point: k_s is evaluated on
// that window from the stage state on the window widened by NG.
inline void rk4_step_at_points(const Grid& g, const Params& p, double t, double dt, const double* u,
                               const int64_t* pts, int npts, double* out /* [npts][NF] */, Status& st,
                               const double* sc = nullptr, double* sout = nullptr /* [npts][NS] */) {
  // with the scalar field (sc non-null) its windows follow the same radii as u's
  const double tst[4] = {t, t + dt / 2.0, t + dt / 2.0, t + dt};
  const double cst[3] = {dt / 2.0, dt / 2.0, dt};  // U_{s+1} = u + cst[s] k_s
  for (int q = 0; q < npts; ++q) {
    const int64_t lin = pts[q];
    const int c[3] = {(int)(lin % g.n[0]), (int)((lin / g.n[0]) % g.n[1]), (int)(lin / ((int64_t)g.n[0] * g.n[1]))};
    int r = 3 * NG;  // interior radius of the first stage window
    const int o[3] = {c[0] - r, c[1] - r, c[2] - r};
    const int m[3] = {2 * r + 1, 2 * r + 1, 2 * r + 1};
    Padded<double> U0, S0;  // u (and the scalar) on the widest window (radius 12 with ghosts)
    pad_periodic(g, u, o, m, U0);
    if (sc) pad_periodic(g, sc, o, m, S0, NS);
    Padded<double> P = U0, Q = S0;
    double kc[4][NF], ks[4][NS];
    for (int s = 0; s < 4; ++s) {
      const int mw = 2 * r + 1;
      const int64_t M3 = (int64_t)mw * mw * mw;
      std::vector<double> k((size_t)NF * M3), kq(sc ? (size_t)NS * M3 : 0);
      rhs_padded(g, p, tst[s], P, k.data(), st, false, sc ? &Q : nullptr, sc ? kq.data() : nullptr);
      const int64_t mid = r + (int64_t)mw * (r + (int64_t)mw * r);
      for (int f = 0; f < NF; ++f) kc[s][f] = k[f * M3 + mid];
      if (sc)
        for (int f = 0; f < NS; ++f) ks[s][f] = kq[f * M3 + mid];
      if (s == 3) break;
      // next stage: interior radius r - NG; its padded points cover this window
      const int rn = r - NG;
      const int mn[3] = {2 * rn + 1, 2 * rn + 1, 2 * rn + 1};
      Padded<double> Pn, Qn;
      Pn.resize(mn);
      if (sc) Qn.resize(mn);
      for (int kk = -NG; kk < mn[2] + NG; ++kk)
        for (int jj = -NG; jj < mn[1] + NG; ++jj)
          for (int ii = -NG; ii < mn[0] + NG; ++ii) {
            // offsets from the point: (ii - rn, ...); index in this window: + r; in U0: + 3*NG
            const int I = ii - rn + r, J = jj - rn + r, K = kk - rn + r;
            const int64_t w = I + (int64_t)mw * (J + (int64_t)mw * K);
            for (int f = 0; f < NF; ++f)
              Pn(f, ii, jj, kk) = U0(f, ii - rn + 3 * NG, jj - rn + 3 * NG, kk - rn + 3 * NG) + cst[s] * k[f * M3 + w];
            if (sc)
              for (int f = 0; f < NS; ++f)
                Qn(f, ii, jj, kk) = S0(f, ii - rn + 3 * NG, jj - rn + 3 * NG, kk - rn + 3 * NG) + cst[s] * kq[f * M3 + w];
          }
      P = Pn;
      if (sc) Q = Qn;
      r = rn;
    }
    for (int f = 0; f < NF; ++f) {
      const double u0 = U0(f, 3 * NG, 3 * NG, 3 * NG);
      out[(size_t)q * NF + f] = u0 + (dt / 6.0) * (kc[0][f] + 2.0 * kc[1][f] + 2.0 * kc[2][f] + kc[3][f]);
    }
    if (sc)
      for (int f = 0; f < NS; ++f) {
        const double s0 = S0(f, 3 * NG, 3 * NG, 3 * NG);
        sout[(size_t)q * NS + f] = s0 + (dt / 6.0) * (ks[0][f] + 2.0 * ks[1][f] + 2.0 * ks[2][f] + ks[3][f]);
      }
  }
}

// Right-hand side evaluated only at the listed points of a periodic grid (with
// the scalar field's right-hand side in sout when sc is non-null).
inline void rhs_at_points(const Grid& g, const Params& p, double t, const double* u, const int64_t* pts, int npts,
                          double* out /* [npts][NF] */, Status& st, const double* sc = nullptr,
                          double* sout = nullptr /* [npts][NS] */) {
  for (int q = 0; q < npts; ++q) {
    const int64_t lin = pts[q];
    const int o[3] = {(int)(lin % g.n[0]), (int)((lin / g.n[0]) % g.n[1]), (int)(lin / ((int64_t)g.n[0] * g.n[1]))};
    const int m[3] = {1, 1, 1};
    Padded<double> P, Q;
    pad_periodic(g, u, o, m, P);
    if (sc) pad_periodic(g, sc, o, m, Q, NS);
    double r[NF], rs[NS];
    rhs_padded(g, p, t, P, r, st, false, sc ? &Q : nullptr, sc ? rs : nullptr);
    for (int f = 0; f < NF; ++f) out[(size_t)q * NF + f] = r[f];
    if (sc)
      for (int f = 0; f < NS; ++f) sout[(size_t)q * NS + f] = rs[f];
  }
}

// ------------------------------------------------------------------ constraints
// H   = R + 2/3 K^2 - At_ij At^ij - 16 pi E
// M_i = gt^jk (d_j At_ki - Gt^l_jk At_li - Gt^l_ji At_kl) - 3/(2 chi) At^j_i d_j chi - 2/3 d_i K - 8 pi S_i
// With a scalar field (sc non-null) E and S_i include its energy and momentum densities.
template <class T>
void constraints_point(const Params& p, const GeomIn<T>& in, T Et, const T St[3], T& H, T M[3], T& Hn,
                       const ScalarIn<T>* sc = nullptr) {
  Geom<T> G;
  geometry(in, G);
  const T* gi = G.gi;
  Matter<T> Mt;
  matter(p, in.chi, in.gt, gi, Et, St, Mt);
  if (sc) {
    ScalarSrc<T> X;
    scalar_matter(in.chi, in.gt, gi, *sc, X);
    Mt.E = Mt.E + X.E;
    for (int i = 0; i < 3; ++i) Mt.S[i] = Mt.S[i] + X.S[i];
  }
  T Amix[3][3];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) {
      T acc = T(0.0);
      for (int l = 0; l < 3; ++l) acc = acc + gi[SYM[k][l]] * in.At[SYM[l][j]];
      Amix[k][j] = acc;
    }
  T AA = T(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T aup = T(0.0);
      for (int l = 0; l < 3; ++l) aup = aup + Amix[i][l] * gi[SYM[l][j]];
      AA = AA + in.At[SYM[i][j]] * aup;
    }
  H = G.R + T(2.0 / 3.0) * in.K * in.K - AA - T(16.0 * PI) * Mt.E;
  for (int i = 0; i < 3; ++i) {
    T acc = T(0.0);
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        T term = in.dAt[SYM[k][i]][j];
        for (int l = 0; l < 3; ++l)
          term = term - G.Gu[l][SYM[j][k]] * in.At[SYM[l][i]] - G.Gu[l][SYM[j][i]] * in.At[SYM[k][l]];
        acc = acc + gi[SYM[j][k]] * term;
      }
    for (int j = 0; j < 3; ++j) acc = acc - T(1.5) * Amix[j][i] * in.dchi[j] / in.chi;
    acc = acc - T(2.0 / 3.0) * in.dK[i] - T(8.0 * PI) * Mt.S[i];
    M[i] = acc;
  }
  double Rabs = std::fabs(value(G.R)), Eabs = std::fabs(value(Mt.E));
  T den = T(Rabs) + T(2.0 / 3.0) * in.K * in.K + AA + T(16.0 * PI) * T(Eabs);
  Hn = (value(den) > 0.0) ? H / den : T(0.0);
}

// Neumaier (compensated) summation
struct NSum {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double get() const { return s + c; }
};

// norms[8] = { rms H, max|H|, rms |M|, max |M|, rms Hn, #non-finite points, min alpha, argmin alpha }
// A point is non-finite if any state value or H or a component of M is not finite.
// argmin alpha is the lowest linear index among the minima (NaN never compares less).
inline void constraints(const Grid& g, const Params& p, const double* u, double norms[8], double* Hout, double* Mout,
                        bool parallel = false, const double* s = nullptr) {
  Padded<double> P, Q;
  const int o[3] = {0, 0, 0};
  pad_periodic(g, u, o, g.n, P);
  if (s) pad_periodic(g, s, o, g.n, Q, NS);
  const double h[3] = {g.h(0), g.h(1), g.h(2)};
  const int64_t N3 = g.npts();
  std::vector<double> Hv(N3), Mv(N3), Hnv(N3), nonf(N3);
#pragma omp parallel for schedule(static) if (parallel)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        GeomIn<double> in;
        gather_geom(P, h, i, j, k, in, true);
        double St[3] = {P(ST, i, j, k), P(ST + 1, i, j, k), P(ST + 2, i, j, k)};
        double H, M[3], Hn;
        ScalarIn<double> sci;
        if (s) {
          sci.Pi = Q(PIF, i, j, k);
          for (int a = 0; a < 3; ++a) sci.dphi[a] = D1(Q, h, PHI, i, j, k, a);
          for (int c = 0; c < 6; ++c) sci.d2phi[c] = 0.0;  // not used by the constraints
        }
        constraints_point(p, in, P(ET, i, j, k), St, H, M, Hn, s ? &sci : nullptr);
        const int64_t q = i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * k);
        bool bad = !std::isfinite(H) || !std::isfinite(M[0]) || !std::isfinite(M[1]) || !std::isfinite(M[2]);
        for (int f = 0; f < NF; ++f) bad = bad || !std::isfinite(u[f * N3 + q]);
        if (s)
          for (int f = 0; f < NS; ++f) bad = bad || !std::isfinite(s[f * N3 + q]);
        Hv[q] = H;
        Mv[q] = std::sqrt(M[0] * M[0] + M[1] * M[1] + M[2] * M[2]);
        Hnv[q] = Hn;
        nonf[q] = bad ? 1.0 : 0.0;
        if (Hout) Hout[q] = H;
        if (Mout)
          for (int c = 0; c < 3; ++c) Mout[c * N3 + q] = M[c];
      }
  NSum sH, sM, sHn;
  double maxH = 0.0, maxM = 0.0, minA = INFINITY, arg = -1.0;
  int64_t bad = 0;
  for (int64_t q = 0; q < N3; ++q) {
    sH.add(Hv[q] * Hv[q]);
    sM.add(Mv[q] * Mv[q]);
    sHn.add(Hnv[q] * Hnv[q]);
    maxH = std::max(maxH, std::fabs(Hv[q]));
    maxM = std::max(maxM, Mv[q]);
    bad += (int64_t)nonf[q];
    double a = u[ALP * N3 + q];
    if (a < minA) {
      minA = a;
      arg = (double)q;
    }
  }
  norms[0] = std::sqrt(sH.get() / (double)N3);
  norms[1] = maxH;
  norms[2] = std::sqrt(sM.get() / (double)N3);
  norms[3] = maxM;
  norms[4] = std::sqrt(sHn.get() / (double)N3);
  norms[5] = (double)bad;
  norms[6] = minA;
  norms[7] = arg;
}

// ------------------------------------------------------------------ initial data
// Counter-based SplitMix64 (Steele, Lea & Flood 2014): the (p+1)-th output of
// the SplitMix64 sequence started from state `seed`.
inline uint64_t splitmix64_at(uint64_t seed, uint64_t p) {
  uint64_t z = seed + (p + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
// uniform in [-1, 1) from the top 53 bits
inline double noise_at(uint64_t seed, uint64_t p) {
  double u01 = (double)(splitmix64_at(seed, p) >> 11) * (1.0 / 9007199254740992.0);
  return 2.0 * u01 - 1.0;
}

// Profile f = mu * shape(x) of a perturbation about the box point x (x relative to
// the centre): value, Laplacian and |grad f|^2, in closed form.
//   GAUSS:  mu exp(-r^2 / 2 sigma^2);  SINE: mu sin(2 pi x_0 / L_0);
//   PGAUSS: Gaussian in s_a = (L_a / pi) sin(pi x_a / L_a) (smooth and periodic).
template <class T>
void profile_at(const Grid& g, int profile, T mu, T sigma, const double x[3], T& val, T& lap, T& grad2) {
  if (profile == GAUSS) {
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    T s2 = sigma * sigma;
    val = mu * exp(T(-r2) / (T(2.0) * s2));
    lap = val * (T(r2) / (s2 * s2) - T(3.0) / s2);
    grad2 = val * val * T(r2) / (s2 * s2);
  } else if (profile == SINE) {
    double kx = 2.0 * PI / g.L[0];
    T sn = T(std::sin(kx * x[0]));
    double cs = std::cos(kx * x[0]);
    val = mu * sn;
    lap = T(-kx * kx) * val;
    grad2 = mu * mu * T(kx * kx * cs * cs);
  } else {
    T s2 = sigma * sigma;
    double sa[3], ca[3], q2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      double kk = PI / g.L[a];
      sa[a] = std::sin(kk * x[a]) / kk;
      ca[a] = std::cos(kk * x[a]);
      q2 += sa[a] * sa[a];
    }
    val = mu * exp(T(-q2) / (T(2.0) * s2));
    T l = T(0.0), gg = T(0.0);
    for (int a = 0; a < 3; ++a) {
      double kk = PI / g.L[a];
      double sc = sa[a] * ca[a];
      // d_a f = -f s c / sigma^2 ; d_a^2 f = f (s c)^2/sigma^4 - f (c^2 - k^2 s^2)/sigma^2
      l = l + val * T(sc * sc) / (s2 * s2) - val * T(ca[a] * ca[a] - kk * kk * sa[a] * sa[a]) / s2;
      gg = gg + val * val * T(sc * sc) / (s2 * s2);
    }
    lap = l;
    grad2 = gg;
  }
}

// Leading-order long-wavelength growing mode for a curvature perturbation
// zeta(x) on the radiation FLRW background (paper: initial-data paragraph of
// "Physical system settings"): conformally flat metric gamma_ij = e^{2 zeta}
// delta_ij (chi = e^{-2 zeta}, gt_ij = delta_ij), K = -3 H0, At = 0, Gt = 0,
// alpha = 1, beta = 0, fluid at rest. The energy density is fixed by the
// Hamiltonian constraint with At = 0 and S = 0:  E = (R + 2/3 K^2) / 16 pi,
// R = -e^{-2 zeta} (4 lap(zeta) + 2 |grad zeta|^2).
// With an iso-curvature mode Upsilon(x) of the massless scalar field (paper:
// "Spherically symmetric iso-curvature" example; the field does not enter the
// background metric at leading order): phi = Upsilon, Pi = 0, and the fluid
// carries the rest of the constraint's energy, E_fluid = E - 1/2 chi |grad Upsilon|^2.
// Returns the 25 field values at grid point (i, j, k) (any integers; wrapped),
// and phi, Pi in sout when non-null.
template <class T>
void init_point(const Grid& g, const Params& p, const InitSpec& s, T mu, T sigma, int i, int j, int k, T out[NF],
                T* sout = nullptr) {
  int I[3] = {wrap(i, g.n[0]), wrap(j, g.n[1]), wrap(k, g.n[2])};
  double x[3];
  for (int a = 0; a < 3; ++a) x[a] = -0.5 * g.L[a] + I[a] * g.h(a) - s.center[a];
  T zeta, lap, grad2;
  profile_at(g, s.profile, mu, sigma, x, zeta, lap, grad2);
  T chi = exp(T(-2.0) * zeta);
  T R = -chi * (T(4.0) * lap + T(2.0) * grad2);
  T K = T(-3.0 * p.H0);
  T E;
  if (s.density_mode == HAMILTONIAN)
    E = (R + T(2.0 / 3.0) * K * K) / T(16.0 * PI);
  else
    E = T(3.0 * p.H0 * p.H0 / (8.0 * PI));
  T ups = T(0.0);
  if (s.sc_mu != 0.0) {
    T ulap, ug2;
    profile_at(g, s.profile, T(s.sc_mu), T(s.sc_sigma), x, ups, ulap, ug2);
    if (s.density_mode == HAMILTONIAN) E = E - T(0.5) * chi * ug2;
  }
  if (s.noise_amp != 0.0) {
    uint64_t lin = (uint64_t)I[0] + (uint64_t)g.n[0] * ((uint64_t)I[1] + (uint64_t)g.n[1] * (uint64_t)I[2]);
    E = E * T(1.0 + s.noise_amp * noise_at(s.seed, lin));
  }
  for (int f = 0; f < NF; ++f) out[f] = T(0.0);
  out[CHI] = chi;
  out[GT + 0] = T(1.0);
  out[GT + 3] = T(1.0);
  out[GT + 5] = T(1.0);
  out[TRK] = K;
  out[ALP] = T(1.0);
  out[ET] = E / (chi * sqrt(chi));
  if (sout) {
    sout[PHI] = ups;
    sout[PIF] = T(0.0);
  }
}

template <class T>
void init_fields(const Grid& g, const Params& p, const InitSpec& s, T mu, T sigma, T* u, T* sc = nullptr) {
  const int64_t N3 = g.npts();
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        T v[NF], w[NS];
        init_point(g, p, s, mu, sigma, i, j, k, v, w);
        const int64_t q = i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * k);
        for (int f = 0; f < NF; ++f) u[f * N3 + q] = v[f];
        if (sc)
          for (int f = 0; f < NS; ++f) sc[f * N3 + q] = w[f];
      }
}

}  // namespace oracle
