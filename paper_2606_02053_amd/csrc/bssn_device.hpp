// Device-side building blocks of the gfx950 COSMOS hot path (FP64 vector ALU).
//
// Physics (paper, "Physical system settings"): Einstein equations with a
// perfect fluid T = (rho + P) u u + P g, P = w rho, and div T = 0, in the
// chi-form BSSN 3+1 system (conformal factor chi, conformal metric gt_ij,
// trace K, traceless At_ij, connection functions Gt^i; 1+log lapse with the
// background trace subtracted, Gamma-driver shift) with the fluid in
// conservative densitised variables Et = chi^(-3/2) E, St_i = chi^(-3/2) S_i.
// Discretisation: 4th-order centred differences (mixed = D1 of D1), lopsided
// radius-3 shift advection, 6th-difference Kreiss-Oliger dissipation, periodic
// wrap of width 3 (the ghost-zone fill is the index wrap below).
//
// The right-hand side is evaluated by bssn_rhs_stream(): fields are visited in
// a fixed order and each field's derivatives are consumed into a small set of
// running accumulators (partial Ricci tensor, partial Gt^i source, ...) as soon
// as they are formed, and each output is handed to the sink the moment it is
// final. This keeps the live FP64 register set far below the ~190 derivative
// values a "gather everything, then do algebra" point evaluation holds.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cosmos {

constexpr int NF = 25;

// Scheduling fence between the per-field phases of a point evaluation: keeps
// the compiler from hoisting the stencil loads of later fields above the
// arithmetic of earlier ones (which would make every load live at once).
#define COSMOS_PHASE() do { asm volatile("" ::: "memory"); __builtin_amdgcn_sched_barrier(0); } while (0)

enum : int { F_CHI = 0, F_GT = 1, F_K = 7, F_AT = 8, F_GAM = 14, F_ALP = 17, F_BET = 18, F_ET = 21, F_ST = 22 };
constexpr double PI_D = 3.14159265358979323846;

// symmetric pair (i, j) -> component index xx, xy, xz, yy, yz, zz
__host__ __device__ constexpr int S(int i, int j) { return i <= j ? i * (5 - i) / 2 + j : j * (5 - j) / 2 + i; }
__host__ __device__ constexpr int SI(int s) { return s < 3 ? 0 : (s < 5 ? 1 : 2); }
__host__ __device__ constexpr int SJ(int s) { return s < 3 ? s : (s < 5 ? s - 2 : 2); }
// mixed-axis pair index: (0,1) -> 0, (0,2) -> 1, (1,2) -> 2
__host__ __device__ constexpr int PAIR(int a, int b) { return a + b - 1; }

struct DevParams {
  double w, H0, eta, ko_eps, alpha_collapse;
  int lapse_bg, evolve_shift;
  int n[3];
  double i12h[3];   // 1 / (12 h_a)
  double i12h2[3];  // 1 / (12 h_a^2)
  double i144[3];   // 1 / (144 h_a h_b) for pairs (0,1), (0,2), (1,2)
  double iko[3];    // ko_eps / (64 h_a)
};

// Linear neighbour offsets of one point on the periodic grid (the ghost-zone
// fill as an index wrap: valid for |offset| <= 3 < n).
struct Nbr {
  int base;
  int d[3][7];  // d[a][o + 3]: linear offset of the neighbour at offset o along axis a
};

__device__ __forceinline__ int wrap1(int i, int n) {
  i = (i < 0) ? i + n : i;
  return (i >= n) ? i - n : i;
}

__device__ __forceinline__ void make_nbr(Nbr& nb, int i, int j, int k, const int n[3]) {
  const int sy = n[0], sz = n[0] * n[1];
  nb.base = i + sy * j + sz * k;
#pragma unroll
  for (int o = -3; o <= 3; ++o) {
    nb.d[0][o + 3] = wrap1(i + o, n[0]) - i;
    nb.d[1][o + 3] = (wrap1(j + o, n[1]) - j) * sy;
    nb.d[2][o + 3] = (wrap1(k + o, n[2]) - k) * sz;
  }
}

// ---------------------------------------------------------------- 1D operators on a 7-point line
// v[0..6] = f at offsets -3..+3 along one axis
__device__ __forceinline__ double op_d1(const double v[7], double i12h) {
  return ((v[1] - v[5]) + 8.0 * (v[4] - v[2])) * i12h;
}
__device__ __forceinline__ double op_d2(const double v[7], double i12h2) {
  return ((16.0 * (v[2] + v[4]) - (v[1] + v[5])) - 30.0 * v[3]) * i12h2;
}
// beta * (one-sided derivative chosen by the sign of beta)
__device__ __forceinline__ double op_adv(const double v[7], double beta, double i12h) {
  double d = (beta > 0.0) ? (((v[6] - 3.0 * v[2]) - 10.0 * v[3]) + (18.0 * v[4] - 6.0 * v[5]))
                          : (((3.0 * v[4] - v[0]) + 10.0 * v[3]) + (6.0 * v[1] - 18.0 * v[2]));
  return beta * (d * i12h);
}
__device__ __forceinline__ double op_ko(const double v[7], double iko) {
  return (((v[0] + v[6]) - 6.0 * (v[1] + v[5])) + (15.0 * (v[2] + v[4]) - 20.0 * v[3])) * iko;
}

// Load f at linear index q: uniform base pointer + zero-extended 32-bit byte offset
// (selects the SGPR-base + 32-bit VGPR-offset form of the global load).
__device__ __forceinline__ double ldq(const double* F, int q) {
  return *(const double*)((const char*)F + (uint32_t)q * 8u);
}

__device__ __forceinline__ void stq(double* F, int q, double v) {
  *(double*)((char*)F + (uint32_t)q * 8u) = v;
}

// A per-phase copy of the neighbour offsets that the compiler cannot prove equal
// to the other phases' copies, so the address arithmetic is redone per field
// instead of being kept live across the whole point evaluation.
__device__ __forceinline__ Nbr opaque(const Nbr& nb) {
  Nbr r = nb;
  asm volatile("" : "+v"(r.base));
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < 7; ++o) asm volatile("" : "+v"(r.d[a][o]));
  return r;
}

__device__ __forceinline__ void load_line(const double* F, const Nbr& nb, int a, double v[7]) {
#pragma unroll
  for (int o = 0; o < 7; ++o) v[o] = ldq(F, nb.base + nb.d[a][o]);
}

// D1_a (D1_b f): 16-point tensor product of the centred first-derivative stencil
__device__ __forceinline__ double op_mixed(const double* F, const Nbr& nb, int a, int b, double i144) {
  double in[4];
  const int oa[4] = {1, 2, 4, 5};  // offsets -2, -1, +1, +2
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int base = nb.base + nb.d[a][oa[p]];
    const double m2 = ldq(F, base + nb.d[b][1]), m1 = ldq(F, base + nb.d[b][2]);
    const double p1 = ldq(F, base + nb.d[b][4]), p2 = ldq(F, base + nb.d[b][5]);
    in[p] = (m2 - p2) + 8.0 * (p1 - m1);
  }
  return ((in[0] - in[3]) + 8.0 * (in[2] - in[1])) * i144;
}

// All derivatives of one field used by the right-hand side: first, pure and
// mixed second derivatives, and the advection + dissipation contribution.
struct FieldDerivs {
  double d1[3];
  double d2[6];  // symmetric components (xx, xy, xz, yy, yz, zz)
  double advko;  // beta^a d_a f (upwinded) + KO f
};

template <bool SECOND, bool ADV, bool KO = true>
__device__ __forceinline__ void field_derivs(const double* F, const Nbr& nb0, const DevParams& P,
                                             const double beta[3], FieldDerivs& r) {
  const Nbr nb = opaque(nb0);
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v[7];
    load_line(F, nb, a, v);
    r.d1[a] = op_d1(v, P.i12h[a]);
    if (SECOND) r.d2[S(a, a)] = op_d2(v, P.i12h2[a]);
    if (ADV) acc += op_adv(v, beta[a], P.i12h[a]);
    if (KO) acc += op_ko(v, P.iko[a]);
  }
  r.advko = acc;
  if (SECOND) {
    r.d2[S(0, 1)] = op_mixed(F, nb, 0, 1, P.i144[0]);
    r.d2[S(0, 2)] = op_mixed(F, nb, 0, 2, P.i144[1]);
    r.d2[S(1, 2)] = op_mixed(F, nb, 1, 2, P.i144[2]);
  }
}

// Only the advection (optional) and dissipation of a field, plus its first derivatives.
template <bool ADV>
__device__ __forceinline__ double field_advko(const double* F, const Nbr& nb0, const DevParams& P,
                                              const double beta[3], double d1[3]) {
  const Nbr nb = opaque(nb0);
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v[7];
    load_line(F, nb, a, v);
    d1[a] = op_d1(v, P.i12h[a]);
    if (ADV) acc += op_adv(v, beta[a], P.i12h[a]);
    acc += op_ko(v, P.iko[a]);
  }
  return acc;
}

// Contraction g^{ab} X_{ab} of two symmetric tensors in 6-component storage.
__device__ __forceinline__ double contract_sym(const double gi[6], const double X[6]) {
  return (gi[0] * X[0] + gi[3] * X[3] + gi[5] * X[5]) + 2.0 * (gi[1] * X[1] + gi[2] * X[2] + gi[4] * X[4]);
}

__device__ __forceinline__ void inv_sym(const double g[6], double gi[6]) {
  const double c00 = g[3] * g[5] - g[4] * g[4];
  const double c01 = g[2] * g[4] - g[1] * g[5];
  const double c02 = g[1] * g[4] - g[2] * g[3];
  const double det = g[0] * c00 + g[1] * c01 + g[2] * c02;
  const double id = 1.0 / det;
  gi[0] = c00 * id;
  gi[1] = c01 * id;
  gi[2] = c02 * id;
  gi[3] = (g[0] * g[5] - g[2] * g[2]) * id;
  gi[4] = (g[1] * g[2] - g[0] * g[4]) * id;
  gi[5] = (g[0] * g[3] - g[1] * g[1]) * id;
}

// ---------------------------------------------------------------- radiation fluid
// Closed-form recovery for P = w rho: X = (rho + P) W^2 is the larger root of
// X^2 - (1 + w) E X + w S^2 = 0, P = X - E. Invalid states (E <= 0) use
// P = 0 and 1/X = 0 (fluid at rest); a negative discriminant is clamped to 0.
struct Fluid {
  double E, S[3], P, invX, Sup[3];
};

__device__ __forceinline__ bool recover(double w, double chi, const double gi[6], double Et, const double St[3],
                                        Fluid& fl) {
  const double c32 = chi * sqrt(chi);
  fl.E = c32 * Et;
#pragma unroll
  for (int i = 0; i < 3; ++i) fl.S[i] = c32 * St[i];
#pragma unroll
  for (int j = 0; j < 3; ++j) fl.Sup[j] = chi * (gi[S(j, 0)] * fl.S[0] + gi[S(j, 1)] * fl.S[1] + gi[S(j, 2)] * fl.S[2]);
  const double S2 = fl.Sup[0] * fl.S[0] + fl.Sup[1] * fl.S[1] + fl.Sup[2] * fl.S[2];
  bool fail = false;
  if (!(fl.E > 0.0)) {
    fail = true;
    fl.P = 0.0;
    fl.invX = 0.0;
  } else {
    const double opw = 1.0 + w;
    double disc = (opw * fl.E) * (opw * fl.E) - 4.0 * w * S2;
    if (!(disc >= 0.0)) {
      fail = true;
      disc = 0.0;
    }
    const double X = 0.5 * (opw * fl.E + sqrt(disc));
    fl.P = X - fl.E;
    fl.invX = 1.0 / X;
  }
  return fail;
}

// Flux of (Et, St_x, St_y, St_z) along axis a at a grid point given by linear index q:
//   F^a_E = chi^(-3/2) (alpha S^a - beta^a E),
//   F^a_i = chi^(-3/2) (alpha (S^a S_i / X + P delta^a_i) - beta^a S_i).
__device__ __forceinline__ void flux_at(const double* U, size_t fs, int q, int a, double w, double Fo[4]) {
  const double chi = ldq(U + F_CHI * fs, q);
  double g[6], gi[6], St[3];
#pragma unroll
  for (int s = 0; s < 6; ++s) g[s] = ldq(U + (F_GT + s) * fs, q);
#pragma unroll
  for (int i = 0; i < 3; ++i) St[i] = ldq(U + (F_ST + i) * fs, q);
  inv_sym(g, gi);
  Fluid fl;
  recover(w, chi, gi, ldq(U + F_ET * fs, q), St, fl);
  const double alpha = ldq(U + F_ALP * fs, q);
  const double ba = ldq(U + (F_BET + a) * fs, q);
  const double im32 = 1.0 / (chi * sqrt(chi));
  Fo[0] = im32 * (alpha * fl.Sup[a] - ba * fl.E);
  const double t = alpha * fl.Sup[a] * fl.invX;
#pragma unroll
  for (int i = 0; i < 3; ++i) Fo[1 + i] = im32 * ((t * fl.S[i] + (i == a ? alpha * fl.P : 0.0)) - ba * fl.S[i]);
}

// Conformal Christoffels from d gt: Gt_kij = 1/2 (d_i gt_kj + d_j gt_ki - d_k gt_ij)
// (first index lowered, local), Gu[k][ij] = Gt^k_ij, Gd^k = gt^ij Gt^k_ij; and
// adds to Ric the terms quadratic in the connection:
//   1/2 Gd^k (Gt_ijk + Gt_jik) + gt^lm (Gt^k_li Gt_jkm + Gt^k_lj Gt_ikm + Gt^k_im Gt_klj)
__device__ __forceinline__ void connection_and_quadratic_ricci(const double dgt[6][3], const double gi[6],
                                                               double Gu[3][6], double Gd[3], double Ric[6]) {
  double Gl[3][6];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      Gl[k][s] = 0.5 * ((dgt[S(k, j)][i] + dgt[S(k, i)][j]) - dgt[s][k]);
    }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int s = 0; s < 6; ++s) Gu[k][s] = gi[S(k, 0)] * Gl[0][s] + gi[S(k, 1)] * Gl[1][s] + gi[S(k, 2)] * Gl[2][s];
#pragma unroll
  for (int k = 0; k < 3; ++k) Gd[k] = contract_sym(gi, Gu[k]);
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) r += 0.5 * Gd[k] * (Gl[i][S(j, k)] + Gl[j][S(i, k)]);
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double g = gi[S(l, m)];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          r += g * ((Gu[k][S(l, i)] * Gl[j][S(k, m)] + Gu[k][S(l, j)] * Gl[i][S(k, m)]) + Gu[k][S(i, m)] * Gl[k][S(l, j)]);
      }
    Ric[s] += r;
  }
}

// Conformal-factor part of the Ricci tensor added to Ric:
//   (1/2chi)(DDchi_ij + gt_ij gt^lm DDchi_lm) - (1/4chi^2)(d_i chi d_j chi + 3 gt_ij gt^lm d_l chi d_m chi),
// DDchi_ij = d_i d_j chi - Gt^k_ij d_k chi.
__device__ __forceinline__ void ricci_conformal_factor(double chi, const double dchi[3], const double d2chi[6],
                                                       const double gt[6], const double gi[6], const double Gu[3][6],
                                                       double Ric[6]) {
  double DD[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) DD[s] = d2chi[s] - (Gu[0][s] * dchi[0] + Gu[1][s] * dchi[1] + Gu[2][s] * dchi[2]);
  const double trDD = contract_sym(gi, DD);
  double dc2 = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int m = 0; m < 3; ++m) dc2 += gi[S(l, m)] * dchi[l] * dchi[m];
  const double ih = 0.5 / chi, iq = 0.25 / (chi * chi);
#pragma unroll
  for (int s = 0; s < 6; ++s) Ric[s] += ih * (DD[s] + gt[s] * trDD) - iq * (dchi[SI(s)] * dchi[SJ(s)] + 3.0 * gt[s] * dc2);
}

// ---------------------------------------------------------------- streaming right-hand side
// Sink interface: put(f, value) receives the final right-hand side of field f at this point.
template <class Sink>
__device__ __forceinline__ void bssn_rhs_stream(const double* U, size_t fs, const Nbr& nb,
                                                const DevParams& P, double t, Sink& sink, bool& prim_fail) {
  const int c = nb.base;
  // ---- point values
  const double chi = ldq(U + F_CHI * fs, c);
  const double K = ldq(U + F_K * fs, c);
  const double alpha = ldq(U + F_ALP * fs, c);
  double gt[6], gi[6], beta[3];
#pragma unroll
  for (int s = 0; s < 6; ++s) gt[s] = ldq(U + (F_GT + s) * fs, c);
#pragma unroll
  for (int i = 0; i < 3; ++i) beta[i] = ldq(U + (F_BET + i) * fs, c);
  inv_sym(gt, gi);

  // ---- matter at the point
  Fluid fl;
  {
    double St[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) St[i] = ldq(U + (F_ST + i) * fs, c);
    prim_fail = recover(P.w, chi, gi, ldq(U + F_ET * fs, c), St, fl);
  }
  // S^jk = S^j S^k / X + P chi gt^jk
  double Sjk[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) Sjk[s] = fl.Sup[SI(s)] * fl.Sup[SJ(s)] * fl.invX + fl.P * chi * gi[s];

  COSMOS_PHASE();
  // ---- shift: first derivatives kept; second derivatives consumed into the Gt^i source
  double db[3][3];  // db[i][a] = d_a beta^i
  double rg[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    COSMOS_PHASE();
    FieldDerivs d;
    field_derivs<true, true>(U + (F_BET + i) * fs, nb, P, beta, d);
#pragma unroll
    for (int a = 0; a < 3; ++a) db[i][a] = d.d1[a];
    // gt^jk d_j d_k beta^i
    rg[i] += contract_sym(gi, d.d2);
    // 1/3 gt^lj d_j d_i beta^i (summed over i as the loop runs)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      rg[l] += (gi[S(l, 0)] * d.d2[S(0, i)] + gi[S(l, 1)] * d.d2[S(1, i)] + gi[S(l, 2)] * d.d2[S(2, i)]) * (1.0 / 3.0);
    double r = 0.0;
    if (P.evolve_shift) r = d.advko + (0.75 * ldq(U + (F_GAM + i) * fs, c) - P.eta * beta[i]);
    sink.put(F_BET + i, r);
  }
  const double divb = db[0][0] + db[1][1] + db[2][2];

  COSMOS_PHASE();
  // ---- conformal metric
  double dgt[6][3];
  double Ric[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    COSMOS_PHASE();
    FieldDerivs d;
    field_derivs<true, true>(U + (F_GT + s) * fs, nb, P, beta, d);
#pragma unroll
    for (int a = 0; a < 3; ++a) dgt[s][a] = d.d1[a];
    Ric[s] = -0.5 * contract_sym(gi, d.d2);
    const int i = SI(s), j = SJ(s);
    double r = d.advko;
#pragma unroll
    for (int k = 0; k < 3; ++k) r += gt[S(i, k)] * db[k][j] + gt[S(j, k)] * db[k][i];
    r -= (2.0 / 3.0) * gt[s] * divb;
    r -= 2.0 * alpha * ldq(U + (F_AT + s) * fs, c);
    sink.put(F_GT + s, r);
  }
  // fluid geometric source: sg_i = S^jk d_i gt_jk
  double sg[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double d[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) d[s] = dgt[s][a];
    sg[a] = (Sjk[0] * d[0] + Sjk[3] * d[3] + Sjk[5] * d[5]) + 2.0 * (Sjk[1] * d[1] + Sjk[2] * d[2] + Sjk[4] * d[4]);
  }
  COSMOS_PHASE();
  // conformal Christoffels and the Ricci terms quadratic in them
  double Gu[3][6], Gd[3];
  connection_and_quadratic_ricci(dgt, gi, Gu, Gd, Ric);

  COSMOS_PHASE();
  // ---- connection functions: d_j Gt^k into the Ricci tensor; advection kept for later
  double rgam_adv[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    COSMOS_PHASE();
    double d1[3];
    rgam_adv[k] = field_advko<true>(U + (F_GAM + k) * fs, nb, P, beta, d1);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      Ric[s] += 0.5 * (gt[S(k, i)] * d1[j] + gt[S(k, j)] * d1[i]);
    }
  }

  COSMOS_PHASE();
  // ---- conformal factor
  double dchi[3];
  {
    FieldDerivs d;
    field_derivs<true, true>(U + F_CHI * fs, nb, P, beta, d);
#pragma unroll
    for (int a = 0; a < 3; ++a) dchi[a] = d.d1[a];
    ricci_conformal_factor(chi, dchi, d.d2, gt, gi, Gu, Ric);
    sink.put(F_CHI, d.advko + (2.0 / 3.0) * chi * (alpha * K - divb));
  }

  COSMOS_PHASE();
  // ---- lapse
  double dal[3], D2a;
  double X[6];  // becomes -D_iD_j alpha + alpha (R_ij - 8 pi S_ij)
  {
    FieldDerivs d;
    field_derivs<true, true>(U + F_ALP * fs, nb, P, beta, d);
#pragma unroll
    for (int a = 0; a < 3; ++a) dal[a] = d.d1[a];
    double cda = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) cda += gi[S(k, l)] * dchi[k] * dal[l];
    const double ih = 0.5 / chi;
    double DDa[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      DDa[s] = (d.d2[s] - (Gu[0][s] * dal[0] + Gu[1][s] * dal[1] + Gu[2][s] * dal[2])) +
               ih * ((dchi[i] * dal[j] + dchi[j] * dal[i]) - gt[s] * cda);
    }
    D2a = chi * contract_sym(gi, DDa);
    const double Kbg = P.lapse_bg ? -3.0 * P.H0 / (1.0 + 2.0 * P.H0 * t) : 0.0;
    sink.put(F_ALP, d.advko - 2.0 * alpha * (K - Kbg));
    const double ichi = 1.0 / chi;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const double Sij = fl.S[SI(s)] * fl.S[SJ(s)] * fl.invX + fl.P * gt[s] * ichi;
      X[s] = -DDa[s] + alpha * (Ric[s] - 8.0 * PI_D * Sij);
    }
  }

  COSMOS_PHASE();
  // ---- trace K: its gradient feeds the Gt^i source
  {
    double dK[3];
    const double r_adv = field_advko<true>(U + F_K * fs, nb, P, beta, dK);
#pragma unroll
    for (int i = 0; i < 3; ++i)
      rg[i] -= (4.0 / 3.0) * alpha * (gi[S(i, 0)] * dK[0] + gi[S(i, 1)] * dK[1] + gi[S(i, 2)] * dK[2]);
    // traceless curvature and its contractions
    double At[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) At[s] = ldq(U + (F_AT + s) * fs, c);
    double Amix[3][3];  // Amix[k][j] = gt^kl At_lj
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < 3; ++j) Amix[k][j] = gi[S(k, 0)] * At[S(0, j)] + gi[S(k, 1)] * At[S(1, j)] + gi[S(k, 2)] * At[S(2, j)];
    double Aup[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      Aup[s] = Amix[i][0] * gi[S(0, j)] + Amix[i][1] * gi[S(1, j)] + Amix[i][2] * gi[S(2, j)];
    }
    const double AA = contract_sym(At, Aup);
    const double E = fl.E;
    const double Str = (fl.Sup[0] * fl.S[0] + fl.Sup[1] * fl.S[1] + fl.Sup[2] * fl.S[2]) * fl.invX + 3.0 * fl.P;
    sink.put(F_K, r_adv + (-D2a + alpha * (AA + K * K * (1.0 / 3.0)) + 4.0 * PI_D * alpha * (E + Str)));

  COSMOS_PHASE();
    // At_ij
    const double trX = contract_sym(gi, X);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      COSMOS_PHASE();
      const int i = SI(s), j = SJ(s);
      double d1[3];
      double r = field_advko<true>(U + (F_AT + s) * fs, nb, P, beta, d1);
#pragma unroll
      for (int k = 0; k < 3; ++k) r += At[S(i, k)] * db[k][j] + At[S(j, k)] * db[k][i];
      r -= (2.0 / 3.0) * At[s] * divb;
      r += chi * (X[s] - gt[s] * trX * (1.0 / 3.0));
      const double AAij = At[S(i, 0)] * Amix[0][j] + At[S(i, 1)] * Amix[1][j] + At[S(i, 2)] * Amix[2][j];
      r += alpha * (K * At[s] - 2.0 * AAij);
      sink.put(F_AT + s, r);
    }

  COSMOS_PHASE();
    // Gt^i
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double r = rgam_adv[i] + rg[i];
      r -= Gd[0] * db[i][0] + Gd[1] * db[i][1] + Gd[2] * db[i][2];
      r += (2.0 / 3.0) * Gd[i] * divb;
      r -= 2.0 * (Aup[S(i, 0)] * dal[0] + Aup[S(i, 1)] * dal[1] + Aup[S(i, 2)] * dal[2]);
      double inner = contract_sym(Gu[i], Aup);
      inner -= (1.5 / chi) * (Aup[S(i, 0)] * dchi[0] + Aup[S(i, 1)] * dchi[1] + Aup[S(i, 2)] * dchi[2]);
      r += 2.0 * alpha * inner;
      r -= 16.0 * PI_D * alpha * (gi[S(i, 0)] * fl.S[0] + gi[S(i, 1)] * fl.S[1] + gi[S(i, 2)] * fl.S[2]);
      sink.put(F_GAM + i, r);
    }

  COSMOS_PHASE();
    // ---- fluid: sources, flux divergence, dissipation
    const double im32 = 1.0 / (chi * sqrt(chi));
    double KS = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const double Kij = (At[s] + gt[s] * K * (1.0 / 3.0)) / chi;
      KS += (s == 0 || s == 3 || s == 5 ? 1.0 : 2.0) * Kij * Sjk[s];
    }
    double div[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double Fm2[4], Fm1[4], Fp1[4], Fp2[4];
      COSMOS_PHASE();
      flux_at(U, fs, c + nb.d[a][1], a, P.w, Fm2);
      COSMOS_PHASE();
      flux_at(U, fs, c + nb.d[a][2], a, P.w, Fm1);
      COSMOS_PHASE();
      flux_at(U, fs, c + nb.d[a][4], a, P.w, Fp1);
      COSMOS_PHASE();
      flux_at(U, fs, c + nb.d[a][5], a, P.w, Fp2);
#pragma unroll
      for (int q = 0; q < 4; ++q) div[q] += ((Fm2[q] - Fp2[q]) + 8.0 * (Fp1[q] - Fm1[q])) * P.i12h[a];
    }
    const double nbeta[3] = {0.0, 0.0, 0.0};
    double dummy[3];
    COSMOS_PHASE();
    {
      const double ko = field_advko<false>(U + F_ET * fs, nb, P, nbeta, dummy);
      const double Sda = fl.Sup[0] * dal[0] + fl.Sup[1] * dal[1] + fl.Sup[2] * dal[2];
      sink.put(F_ET, ko + (im32 * (alpha * KS - Sda) - div[0]));
    }
    const double sgt = contract_sym(Sjk, gt);
    const double ichi = 1.0 / chi, ichi2 = ichi * ichi;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      COSMOS_PHASE();
      const double ko = field_advko<false>(U + (F_ST + i) * fs, nb, P, nbeta, dummy);
      double src = -E * dal[i] + (fl.S[0] * db[0][i] + fl.S[1] * db[1][i] + fl.S[2] * db[2][i]);
      src += 0.5 * alpha * (sg[i] * ichi - sgt * dchi[i] * ichi2);
      sink.put(F_ST + i, ko + (im32 * src - div[1 + i]));
    }
  }
}

}  // namespace cosmos
