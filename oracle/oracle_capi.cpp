// C entry points of the CPU oracle (test infrastructure only), called from
// Python through ctypes by tests/, the smoke check and the CPU baseline.
//
// Conventions: n[3] grid points and L[3] box lengths per axis; prm = {w, H0,
// eta, ko_eps}; iprm = {lapse_bg, evolve_shift, fluid_scheme}; states are SoA float64 arrays
// of 25 * n0*n1*n2 values (x fastest). Every function returns 0 on success and
// a negative value on invalid arguments.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "cosmos_oracle.hpp"

namespace oracle {
Tape g_tape;
OpCount g_count;
}  // namespace oracle

using namespace oracle;

static bool make(const int* n, const double* L, const double* prm, const int* iprm, Grid& g, Params& p) {
  if (!n || !L || !prm || !iprm) return false;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 8 || !(L[a] > 0.0)) return false;
    g.n[a] = n[a];
    g.L[a] = L[a];
  }
  p.w = prm[0];
  p.H0 = prm[1];
  p.eta = prm[2];
  p.ko_eps = prm[3];
  p.lapse_bg = iprm[0];
  p.evolve_shift = iprm[1];
  p.fluid_scheme = iprm[2];
  if (p.fluid_scheme != 0 && p.fluid_scheme != 1) return false;
  return true;
}

static InitSpec make_init(const double* d, uint64_t seed, int profile, int density_mode) {
  InitSpec s;
  s.mu = d[0];
  s.sigma = d[1];
  s.center[0] = d[2];
  s.center[1] = d[3];
  s.center[2] = d[4];
  s.noise_amp = d[5];
  s.seed = seed;
  s.profile = profile;
  s.density_mode = density_mode;
  return s;
}

extern "C" {

int oracle_rhs(const int* n, const double* L, const double* prm, const int* iprm, double t, const double* u,
               double* dudt, int64_t* prim_fail, int parallel) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !dudt) return -1;
  Status st;
  rhs(g, p, t, u, dudt, st, parallel != 0);
  if (prim_fail) *prim_fail = st.prim_fail;
  return 0;
}

int oracle_kt_divergence(const int* n, const double* L, const double* prm, const int* iprm, const double* u,
                         double* div) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !div) return -1;
  kt_divergence(g, p, u, div);
  return 0;
}

// Operation count of one Kurganov-Tadmor interface flux (reconstruction, two flux and
// speed evaluations, combination) at the interface x+1/2 of point 0 of the state u.
int oracle_count_kt_flops(const int* n, const double* L, const double* prm, const int* iprm, const double* u,
                          double* out) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !out) return -1;
  const int64_t N3 = g.npts();
  Padded<Cnt> P;
  const int o[3] = {0, 0, 0}, m[3] = {1, 1, 1};
  std::vector<Cnt> x((size_t)NF * N3);
  for (size_t q = 0; q < x.size(); ++q) x[q] = Cnt(u[q]);
  pad_periodic(g, x.data(), o, m, P);
  g_count = OpCount();
  Cnt uL[NF], uR[NF], fh[4];
  kt_interface_states<Cnt>(P, 0, 0, 0, 0, uL, uR);
  kt_flux(p, uL, uR, 0, fh);
  const OpCount total = g_count;
  // the speed evaluation repeats the inverse metric and the recovery that the flux of
  // the same state has formed: counted once
  g_count = OpCount();
  {
    Cnt gt[6], gi[6], det, St[3];
    for (int s = 0; s < 6; ++s) gt[s] = uL[GT + s];
    inverse_sym(gt, gi, det);
    for (int i = 0; i < 3; ++i) St[i] = uL[ST + i];
    Matter<Cnt> M;
    matter(p, uL[CHI], gt, gi, uL[ET], St, M, false);
  }
  const OpCount dup = g_count;
  out[0] = (double)(total.flops() - 2 * dup.flops());
  out[1] = (double)(total.sqrt - 2 * dup.sqrt);
  out[2] = (double)total.flops();
  return 0;
}

int oracle_rk4_steps(const int* n, const double* L, const double* prm, const int* iprm, double t0, double dt,
                     int nsteps, double* u, int64_t* prim_fail, int parallel) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || nsteps < 0) return -1;
  Status st;
  for (int s = 0; s < nsteps; ++s) rk4_step(g, p, t0 + s * dt, dt, u, st, parallel != 0);
  if (prim_fail) *prim_fail = st.prim_fail;
  return 0;
}

// ---- with the massless scalar field: s holds phi and Pi (2 * N3 values, SoA)
int oracle_rhs_sc(const int* n, const double* L, const double* prm, const int* iprm, double t, const double* u,
                  const double* s, double* dudt, double* dsdt, int64_t* prim_fail, int parallel) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !s || !dudt || !dsdt) return -1;
  Status st;
  rhs(g, p, t, u, dudt, st, parallel != 0, s, dsdt);
  if (prim_fail) *prim_fail = st.prim_fail;
  return 0;
}

int oracle_rk4_steps_sc(const int* n, const double* L, const double* prm, const int* iprm, double t0, double dt,
                        int nsteps, double* u, double* s, int64_t* prim_fail, int parallel) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !s || nsteps < 0) return -1;
  Status st;
  for (int q = 0; q < nsteps; ++q) rk4_step(g, p, t0 + q * dt, dt, u, st, parallel != 0, s);
  if (prim_fail) *prim_fail = st.prim_fail;
  return 0;
}

int oracle_constraints_sc(const int* n, const double* L, const double* prm, const int* iprm, const double* u,
                          const double* s, double* norms, double* H, double* M, int parallel) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !s || !norms) return -1;
  constraints(g, p, u, norms, H, M, parallel != 0, s);
  return 0;
}

// init_d = {mu, sigma, cx, cy, cz, noise_amp}, sc_d = {sc_mu, sc_sigma}
int oracle_init_sc(const int* n, const double* L, const double* prm, const int* iprm, const double* init_d,
                   const double* sc_d, uint64_t seed, int profile, int density_mode, double* u, double* s) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !init_d || !sc_d || !u || !s) return -1;
  InitSpec spec = make_init(init_d, seed, profile, density_mode);
  spec.sc_mu = sc_d[0];
  spec.sc_sigma = sc_d[1];
  init_fields<double>(g, p, spec, spec.mu, spec.sigma, u, s);
  return 0;
}

int oracle_rhs_sc_at_points(const int* n, const double* L, const double* prm, const int* iprm, double t,
                            const double* u, const double* s, const int64_t* pts, int npts, double* out,
                            double* sout) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !s || !pts || !out || !sout) return -1;
  Status st;
  rhs_at_points(g, p, t, u, pts, npts, out, st, s, sout);
  return 0;
}

int oracle_rk4_sc_at_points(const int* n, const double* L, const double* prm, const int* iprm, double t, double dt,
                            const double* u, const double* s, const int64_t* pts, int npts, double* out,
                            double* sout) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !s || !pts || !out || !sout) return -1;
  Status st;
  rk4_step_at_points(g, p, t, dt, u, pts, npts, out, st, s, sout);
  return 0;
}

int oracle_rhs_at_points(const int* n, const double* L, const double* prm, const int* iprm, double t,
                         const double* u, const int64_t* pts, int npts, double* out) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !pts || !out) return -1;
  Status st;
  rhs_at_points(g, p, t, u, pts, npts, out, st);
  return 0;
}

int oracle_rk4_at_points(const int* n, const double* L, const double* prm, const int* iprm, double t, double dt,
                         const double* u, const int64_t* pts, int npts, double* out) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !pts || !out) return -1;
  Status st;
  rk4_step_at_points(g, p, t, dt, u, pts, npts, out, st);
  return 0;
}

int oracle_constraints(const int* n, const double* L, const double* prm, const int* iprm, const double* u,
                       double* norms, double* H, double* M, int parallel) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !norms) return -1;
  constraints(g, p, u, norms, H, M, parallel != 0);
  return 0;
}

// init_d = {mu, sigma, cx, cy, cz, noise_amp}
int oracle_init(const int* n, const double* L, const double* prm, const int* iprm, const double* init_d,
                uint64_t seed, int profile, int density_mode, double* u) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !init_d || !u) return -1;
  InitSpec s = make_init(init_d, seed, profile, density_mode);
  init_fields<double>(g, p, s, s.mu, s.sigma, u);
  return 0;
}

int oracle_init_at_points(const int* n, const double* L, const double* prm, const int* iprm, const double* init_d,
                          uint64_t seed, int profile, int density_mode, const int64_t* pts, int npts, double* out) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !init_d || !pts || !out) return -1;
  InitSpec s = make_init(init_d, seed, profile, density_mode);
  for (int q = 0; q < npts; ++q) {
    int64_t lin = pts[q];
    int i = (int)(lin % g.n[0]), j = (int)((lin / g.n[0]) % g.n[1]), k = (int)(lin / ((int64_t)g.n[0] * g.n[1]));
    init_point<double>(g, p, s, s.mu, s.sigma, i, j, k, out + (size_t)q * NF);
  }
  return 0;
}

// Tangent of the initial data with respect to mu (which = 0) or sigma (which = 1),
// by forward-mode differentiation of init_fields.
int oracle_init_tangent(const int* n, const double* L, const double* prm, const int* iprm, const double* init_d,
                        uint64_t seed, int profile, int density_mode, int which, double* du) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !init_d || !du || which < 0 || which > 1) return -1;
  InitSpec s = make_init(init_d, seed, profile, density_mode);
  const size_t N = (size_t)NF * g.npts();
  std::vector<Dual> u(N);
  Dual mu(s.mu, which == 0 ? 1.0 : 0.0), sigma(s.sigma, which == 1 ? 1.0 : 0.0);
  init_fields<Dual>(g, p, s, mu, sigma, u.data());
  for (size_t q = 0; q < N; ++q) du[q] = u[q].d;
  return 0;
}

// Jacobian-vector products of the discrete maps (forward mode):
// what = 0: Jv = (d rhs / d u) v at time t;  what = 1: Jv = (d step / d u) v for one RK4 step.
// fu receives the primal result (rhs or stepped state).
int oracle_jvp(const int* n, const double* L, const double* prm, const int* iprm, int what, double t, double dt,
               const double* u, const double* v, double* fu, double* Jv) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !v || !Jv) return -1;
  const size_t N = (size_t)NF * g.npts();
  std::vector<Dual> x(N), y(N);
  for (size_t q = 0; q < N; ++q) x[q] = Dual(u[q], v[q]);
  Status st;
  if (what == 0) {
    rhs(g, p, t, x.data(), y.data(), st);
  } else {
    y = x;
    rk4_step(g, p, t, dt, y.data(), st);
  }
  for (size_t q = 0; q < N; ++q) {
    if (fu) fu[q] = y[q].v;
    Jv[q] = y[q].d;
  }
  return 0;
}

// Vector-Jacobian products (reverse mode on a tape), the oracle's discrete adjoint:
// what = 0: lam_in = (d rhs / d u)^T lam_out;  what = 1: lam_in = (d step / d u)^T lam_out.
int oracle_vjp(const int* n, const double* L, const double* prm, const int* iprm, int what, double t, double dt,
               const double* u, const double* lam_out, double* lam_in) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !lam_out || !lam_in) return -1;
  const size_t N = (size_t)NF * g.npts();
  g_tape.clear();
  std::vector<Rev> x(N), y(N);
  for (size_t q = 0; q < N; ++q) x[q] = Rev::input(u[q]);
  Status st;
  if (what == 0) {
    rhs(g, p, t, x.data(), y.data(), st);
  } else {
    y = x;
    rk4_step(g, p, t, dt, y.data(), st);
  }
  g_tape.adj.assign((size_t)g_tape.size(), 0.0);
  for (size_t q = 0; q < N; ++q)
    if (y[q].id >= 0) g_tape.adj[(size_t)y[q].id] += lam_out[q];
  g_tape.sweep();
  for (size_t q = 0; q < N; ++q) lam_in[q] = g_tape.adj[(size_t)x[q].id];
  g_tape.clear();
  g_tape.adj.clear();
  g_tape.adj.shrink_to_fit();
  g_tape.parent.shrink_to_fit();
  g_tape.partial.shrink_to_fit();
  g_tape.start.shrink_to_fit();
  return 0;
}

// Arithmetic-operation counts of the method on the given state, per grid point:
// out[0] one right-hand-side evaluation excluding the fluid fluxes,
// out[1] one evaluation of the fluid fluxes at one point,
// out[2] the RK4 combinations of one step, out[3] FLOPs of one whole RK4 step
//        (4 * (out[0] + out[1]) + out[2]); out[4] sqrt count per RHS point.
int oracle_count_flops(const int* n, const double* L, const double* prm, const int* iprm, const double* u,
                       double* out) {
  Grid g;
  Params p;
  if (!make(n, L, prm, iprm, g, p) || !u || !out) return -1;
  const int64_t N3 = g.npts();
  const size_t N = (size_t)NF * N3;
  std::vector<Cnt> x(N), y(N);
  for (size_t q = 0; q < N; ++q) x[q] = Cnt(u[q]);
  // fluxes at one point
  Cnt uu[NF], fl[12];
  for (int f = 0; f < NF; ++f) uu[f] = x[f * N3];
  g_count = OpCount();
  fluid_flux(p, uu, fl);
  double flux = (double)g_count.flops();
  // whole RHS, minus the flux evaluations it makes on the window padded by 2
  g_count = OpCount();
  Status st;
  rhs(g, p, 0.0, x.data(), y.data(), st);
  double nflux = (double)(g.n[0] + 4) * (g.n[1] + 4) * (g.n[2] + 4);
  double rhs_total = (double)g_count.flops() - nflux * flux;
  double sq = (double)g_count.sqrt;
  // RK4 combinations: 3 stage states (2 ops per value) and the final update (7 ops)
  g_count = OpCount();
  Cnt a = x[0], b = x[1];
  Cnt U = a + Cnt(0.5) * b;
  double stage = (double)g_count.flops();
  g_count = OpCount();
  Cnt fin = a + Cnt(1.0 / 6.0) * (b + Cnt(2.0) * b + Cnt(2.0) * b + b);
  double final_ = (double)g_count.flops();
  (void)U;
  (void)fin;
  out[0] = rhs_total / (double)N3;
  out[1] = flux;
  out[2] = NF * (3.0 * stage + final_);
  out[3] = 4.0 * (out[0] + out[1]) + out[2];
  out[4] = sq / (double)N3;
  return 0;
}

// Pointwise pieces for the algebra tests. in = packed GeomIn<double> in the
// order: chi, gt[6], K, At[6], Gam[3], alpha, beta[3], dchi[3], d2chi[6],
// dgt[6][3], d2gt[6][6], dGam[3][3], dalpha[3], d2alpha[6], dbeta[3][3],
// d2beta[3][6], dK[3], dAt[6][3].
static void unpack(const double* a, GeomIn<double>& in) {
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
    for (int a2 = 0; a2 < 3; ++a2) in.dgt[s][a2] = *q++;
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
}
int oracle_geomin_size(void) { return 1 + 6 + 1 + 6 + 3 + 1 + 3 + 3 + 6 + 18 + 36 + 9 + 3 + 6 + 9 + 18 + 3 + 18; }

// out: Ric[6], R, DDalpha[6], Gd[3], det
int oracle_geometry_point(const double* packed, double* out) {
  GeomIn<double> in;
  unpack(packed, in);
  Geom<double> G;
  geometry(in, G);
  double DDa[6];
  ddalpha(in, G, DDa);
  for (int s = 0; s < 6; ++s) out[s] = G.Ric[s];
  out[6] = G.R;
  for (int s = 0; s < 6; ++s) out[7 + s] = DDa[s];
  for (int s = 0; s < 3; ++s) out[13 + s] = G.Gd[s];
  out[16] = G.det;
  return 0;
}

// Pointwise RHS (without advection, dissipation and flux divergence) and the
// constraints at one point. out: rhs[25], H, M[3], Hn; returns the recovery-failure flag.
int oracle_point_rhs(const double* prm, const int* iprm, double t, const double* packed, double Et, const double* St,
                     double* out) {
  Params p;
  p.w = prm[0];
  p.H0 = prm[1];
  p.eta = prm[2];
  p.ko_eps = prm[3];
  p.lapse_bg = iprm[0];
  p.evolve_shift = iprm[1];
  GeomIn<double> in;
  unpack(packed, in);
  bool fail = rhs_point(p, t, in, Et, St, out);
  double H, M[3], Hn;
  constraints_point(p, in, Et, St, H, M, Hn);
  out[25] = H;
  out[26] = M[0];
  out[27] = M[1];
  out[28] = M[2];
  out[29] = Hn;
  return fail ? 1 : 0;
}

// Reverse mode of the pointwise right-hand side (rhs_point) at one point:
// given rbar[25], returns the adjoints of the packed GeomIn inputs (size
// oracle_geomin_size()) followed by those of Et and St[3].
int oracle_point_rhs_vjp(const double* prm, const int* iprm, double t, const double* packed, double Et,
                         const double* St, const double* rbar, double* out) {
  Params p;
  p.w = prm[0];
  p.H0 = prm[1];
  p.eta = prm[2];
  p.ko_eps = prm[3];
  p.lapse_bg = iprm[0];
  p.evolve_shift = iprm[1];
  const int n = oracle_geomin_size();
  g_tape.clear();
  std::vector<Rev> x(n + 4);
  for (int q = 0; q < n; ++q) x[q] = Rev::input(packed[q]);
  x[n] = Rev::input(Et);
  for (int c = 0; c < 3; ++c) x[n + 1 + c] = Rev::input(St[c]);
  // unpack into a GeomIn<Rev> in the packed order
  std::vector<double> tmp(n);
  GeomIn<Rev> in;
  {
    const Rev* q = x.data();
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
  }
  Rev r[NF];
  Rev St3[3] = {x[n + 1], x[n + 2], x[n + 3]};
  rhs_point(p, t, in, x[n], St3, r);
  g_tape.adj.assign((size_t)g_tape.size(), 0.0);
  for (int f = 0; f < NF; ++f)
    if (r[f].id >= 0) g_tape.adj[(size_t)r[f].id] += rbar[f];
  g_tape.sweep();
  for (int q = 0; q < n + 4; ++q) out[q] = g_tape.adj[(size_t)x[q].id];
  g_tape.clear();
  return 0;
}

// Primitive recovery at one point. out: E, S[3], S2, P, invX, Sup[3], Strace
int oracle_matter_point(double w, double chi, const double* gt, double Et, const double* St, double* out) {
  Params p;
  p.w = w;
  double gi[6], det;
  inverse_sym(gt, gi, det);
  Matter<double> M;
  bool fail = matter(p, chi, gt, gi, Et, St, M);
  out[0] = M.E;
  for (int i = 0; i < 3; ++i) out[1 + i] = M.S[i];
  out[4] = M.S2;
  out[5] = M.P;
  out[6] = M.invX;
  for (int i = 0; i < 3; ++i) out[7 + i] = M.Sup[i];
  out[10] = M.Strace;
  return fail ? 1 : 0;
}

// Fluid fluxes at one point from the 25 state values.
int oracle_flux_point(const double* prm, const double* u, double* out) {
  Params p;
  p.w = prm[0];
  fluid_flux(p, u, out);
  return 0;
}

// Kurganov-Tadmor numerical flux along axis a between two interface states
// (25 values each): out[4] for Et, St_x, St_y, St_z.
int oracle_kt_flux(const double* prm, const double* uL, const double* uR, int a, double* out) {
  if (!prm || !uL || !uR || !out || a < 0 || a > 2) return -1;
  Params p;
  p.w = prm[0];
  kt_flux(p, uL, uR, a, out);
  return 0;
}

// Characteristic speeds (lambda_minus, lambda_plus) of the fluid along axis a at one state.
int oracle_fluid_speeds(const double* prm, const double* u, int a, double* out) {
  if (!prm || !u || !out || a < 0 || a > 2) return -1;
  Params p;
  p.w = prm[0];
  fluid_speeds(p, u, a, out[0], out[1]);
  return 0;
}

// Stencil operators applied at grid point (i, j, k) to a single periodic grid
// function f (n0*n1*n2 values): kind 0 = D1 along a, 1 = D2 along a,
// 2 = D1_a(D1_b f), 3 = advection with shift beta[3], 4 = Kreiss-Oliger (eps).
int oracle_stencil(const int* n, const double* L, const double* f, int i, int j, int k, int kind, int a, int b,
                   const double* beta, double eps, double* out) {
  Grid g;
  Params p;
  const double prm[4] = {1.0 / 3.0, 1.0, 1.0, 0.1};
  const int iprm[3] = {1, 1, 0};
  if (!make(n, L, prm, iprm, g, p) || !f || !out) return -1;
  const int64_t N3 = g.npts();
  std::vector<double> u((size_t)NF * N3, 0.0);
  for (int64_t q = 0; q < N3; ++q) u[q] = f[q];  // stored as field 0
  Padded<double> P;
  const int o[3] = {i, j, k};
  const int m[3] = {1, 1, 1};
  pad_periodic(g, u.data(), o, m, P);
  const double h[3] = {g.h(0), g.h(1), g.h(2)};
  switch (kind) {
    case 0: *out = D1(P, h, 0, 0, 0, 0, a); break;
    case 1: *out = D2(P, h, 0, 0, 0, 0, a); break;
    case 2: *out = Dmixed(P, h, 0, 0, 0, 0, a, b); break;
    case 3: *out = Advect(P, h, 0, 0, 0, 0, beta); break;
    case 4: *out = KO(P, h, eps, 0, 0, 0, 0); break;
    default: return -1;
  }
  return 0;
}

// Consistency of the evolved conformal connection with the metric:
// out[0] = rms over the grid of |Gt^i - gt^jk Gt^i_jk|, out[1] = its maximum.
int oracle_gamma_constraint(const int* n, const double* L, const double* u, double* out) {
  Grid g;
  Params p;
  const double prm[4] = {1.0 / 3.0, 1.0, 1.0, 0.1};
  const int iprm[3] = {1, 1, 0};
  if (!make(n, L, prm, iprm, g, p) || !u || !out) return -1;
  Padded<double> P;
  const int o[3] = {0, 0, 0};
  pad_periodic(g, u, o, g.n, P);
  const double h[3] = {g.h(0), g.h(1), g.h(2)};
  NSum s;
  double mx = 0.0;
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        GeomIn<double> in;
        gather_geom(P, h, i, j, k, in, false);
        Geom<double> G;
        geometry(in, G);
        double e2 = 0.0;
        for (int c = 0; c < 3; ++c) e2 += (in.Gam[c] - G.Gd[c]) * (in.Gam[c] - G.Gd[c]);
        s.add(e2);
        mx = std::max(mx, std::sqrt(e2));
      }
  out[0] = std::sqrt(s.get() / (double)g.npts());
  out[1] = mx;
  return 0;
}

uint64_t oracle_splitmix64(uint64_t seed, uint64_t p) { return splitmix64_at(seed, p); }

}  // extern "C"
