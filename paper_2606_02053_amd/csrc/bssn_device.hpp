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
  double i24h[3];   // 1 / (24 h_a)
  double ih[3];     // 1 / h_a
  int fluid_scheme; // 0: centred 4th-order flux divergence + KO; 1: Kurganov-Tadmor (divergence from its pre-pass)
  // scalar-field sources of the geometry (null without a scalar field): kScalarSrc arrays of fs
  // doubles, [SRC_EPS] E + S, [SRC_E] E, [SRC_S + j] S_j, [SRC_SIJ + s] S_ij (physical densities)
  const double* xsrc;
};

constexpr int SRC_EPS = 0, SRC_E = 1, SRC_S = 2, SRC_SIJ = 5, kScalarSrc = 11;

// Brick decomposition of the grid for the stage kernel: a workgroup of
// bx*by*bz (= 256) threads owns one bx x by x bz brick, one point per thread
// (x fastest within the brick, so a wave covers whole x-rows). With
// xcd_order the flat brick sequence is cut into 8 contiguous chunks, chunk q
// served by the workgroups with blockIdx % 8 == q: the hardware deals
// consecutive workgroups round-robin to the 8 XCDs, so each XCD then walks one
// contiguous slab and the stencil halos of a brick are found in its own L2.
struct Tile {
  int bx, by, bz;
  int nbx, nby, nbz;
  int nbricks, per, xcd_order;
  // brick order of the persistent LDS kernel: 0 XCD slabs, 1 linear, 2 XCD-blocked
  // (each XCD owns a slab of zr brick layers and its W = gx gy gz resident
  // workgroups process one gx x gy x gz block of bricks at a time, so that the
  // halos they share are read from that XCD's L2 once)
  int order, gx, gy, gz, zr, ngx, ngy, ngroups;
};

// Maps (blockIdx, threadIdx) to a grid point; false for padding workgroups
// and for threads beyond the edge of a partial brick.
__device__ __forceinline__ bool tile_point(const Tile& T, const int n[3], int& i, int& j, int& k) {
  int brick = blockIdx.x;
  if (T.xcd_order) brick = (blockIdx.x & 7) * T.per + (blockIdx.x >> 3);
  if (brick >= T.nbricks) return false;
  const int bxi = brick % T.nbx;
  const int byz = brick / T.nbx;
  const int byi = byz % T.nby;
  const int bzi = byz / T.nby;
  const int t = threadIdx.x;
  i = bxi * T.bx + t % T.bx;
  j = byi * T.by + (t / T.bx) % T.by;
  k = bzi * T.bz + t / (T.bx * T.by);
  return i < n[0] && j < n[1] && k < n[2];
}

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
__device__ __forceinline__ double op_ko(const double v[7], double iko) {
  return (((v[0] + v[6]) - 6.0 * (v[1] + v[5])) + (15.0 * (v[2] + v[4]) - 20.0 * v[3])) * iko;
}

// Every operator of one stencil line v[o] = f(x + (o - 3) h) in one pass, branch
// free. With t_k = f_k - f_-k and s_k = f_k + f_-k:
//   D1 = (8 t1 - t2) / 12h,   D2 = (16 s1 - s2 - 30 f0) / 12h^2,
// and the lopsided derivatives of the advection term split into a centred odd part
// and a multiple of the 6th difference D6 that the KO operator also uses,
//   U+ (beta > 0), U- (beta <= 0) = (t3 - 6 t2 + 21 t1) / 24h +/- D6 / 24h,
//   D6 = s3 - 6 s2 + 15 s1 - 20 f0,
// so beta U + KO = beta (t3 - 6 t2 + 21 t1) / 24h + (|beta| / 24h + eps / 64h) D6
// (equal to the textbook branch form up to rounding, also at beta = 0).
template <bool SECOND, bool ADV, bool KO>
__device__ __forceinline__ void op_line(const double v[7], double beta, double i12h, double i12h2, double i24h,
                                        double iko, double& d1, double& d2, double& advko) {
  const double t1 = v[4] - v[2], t2 = v[5] - v[1];
  d1 = (8.0 * t1 - t2) * i12h;
  const double s1 = v[4] + v[2], s2 = v[5] + v[1];
  if (SECOND) d2 = ((16.0 * s1 - s2) - 30.0 * v[3]) * i12h2;
  if (ADV || KO) {
    const double d6 = ((v[6] + v[0]) - 6.0 * s2) + (15.0 * s1 - 20.0 * v[3]);
    double cd6 = 0.0;
    if (ADV) {
      const double odd = ((v[6] - v[0]) - 6.0 * t2) + 21.0 * t1;
      advko += (beta * i24h) * odd;
      cd6 = fabs(beta) * i24h;
    }
    if (KO) cd6 += iko;
    advko += cd6 * d6;
  }
}

// Load f at linear index q: uniform base pointer + zero-extended 32-bit byte offset
// (selects the SGPR-base + 32-bit VGPR-offset form of the global load).
__device__ __forceinline__ double ldq(const double* F, int q) {
  return *(const double*)((const char*)F + (uint32_t)q * 8u);
}

__device__ __forceinline__ void stq(double* F, int q, double v) {
  *(double*)((char*)F + (uint32_t)q * 8u) = v;
}

// One field array as a raw buffer: the uniform base address sits in a buffer
// descriptor in SGPRs and each lane supplies only a 32-bit byte offset, so a load
// or store costs no vector address arithmetic (a plain pointer load makes the
// compiler form a 64-bit VGPR address per access). Descriptor word 3 = 0x00020000
// is the gfx9 raw-buffer format (32-bit data, no swizzle, no index stride). The
// record size bounds the access; grids keep 8 * points < 2^32 bytes per field.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const double* base, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, (int)nbytes, 0x00020000);
}
__device__ __forceinline__ double bld(const double* base, uint32_t nbytes, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(field_rsrc(base, nbytes), off, 0, 0));
}
__device__ __forceinline__ void bst(double* base, uint32_t nbytes, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), field_rsrc(base, nbytes), off, 0, 0);
}
// The same with the non-temporal hint (cache policy nt): for data used once per launch (the RK4
// epilogue operands and results), so that it is the first to leave L2 and the halo lines that
// neighbouring bricks share stay.
__device__ __forceinline__ double bld_nt(const double* base, uint32_t nbytes, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(field_rsrc(base, nbytes), off, 0, 2));
}
__device__ __forceinline__ void bst_nt(double* base, uint32_t nbytes, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), field_rsrc(base, nbytes), off, 0, 2);
}

// Base of field f of a field-major array. The field offset passes through an empty
// asm statement so the compiler recomputes it (two scalar ops) at each use instead
// of keeping one base per field live for the whole kernel, which would overflow the
// scalar registers and spill them.
__device__ __forceinline__ size_t field_off(int f, size_t fs) {
  size_t off = (size_t)f * fs;
  asm volatile("" : "+s"(off));
  return off;
}
template <class T>
__device__ __forceinline__ T* field_ptr(T* U, int f, size_t fs) {
  return U + field_off(f, fs);
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
    double d2 = 0.0;
    op_line<SECOND, ADV, KO>(v, beta[a], P.i12h[a], P.i12h2[a], P.i24h[a], P.iko[a], r.d1[a], d2, acc);
    if (SECOND) r.d2[S(a, a)] = d2;
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
    double d2 = 0.0;
    op_line<false, ADV, true>(v, beta[a], P.i12h[a], P.i12h2[a], P.i24h[a], P.iko[a], d1[a], d2, acc);
  }
  return acc;
}

// Contraction g^{ab} X_{ab} of two symmetric tensors in 6-component storage.
__host__ __device__ __forceinline__ double contract_sym(const double gi[6], const double X[6]) {
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

// Fluxes of (Et, St_x, St_y, St_z) along the three axes at grid point c, stored
// field-major as F[(4 a + q) fs + c] (12 arrays of fs doubles):
//   F^a_E = chi^(-3/2) (alpha S^a - beta^a E),
//   F^a_i = chi^(-3/2) (alpha (S^a S_i / X + P delta^a_i) - beta^a S_i).
// Formed once per point per stage (a pointwise pre-pass), so the stage kernel
// takes the divergence from 4 loads per flux component instead of recovering
// the primitives at all 12 axis neighbours.
// The same from the 15 values it depends on (chi, gt_ij, alpha, beta^a, Et, St_i), which the stage
// kernel holds at the end of a point's evaluation for the state it has just written.
__device__ __forceinline__ void fluid_flux_values(double chi, const double g[6], double alpha, const double beta[3],
                                                  double Et, const double St[3], double w, double* F, size_t fs,
                                                  int c) {
  double gi[6];
  inv_sym(g, gi);
  Fluid fl;
  recover(w, chi, gi, Et, St, fl);
  const double im32 = 1.0 / (chi * sqrt(chi));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ba = beta[a];
    stq(F + (4 * a) * fs, c, im32 * (alpha * fl.Sup[a] - ba * fl.E));
    const double t = alpha * fl.Sup[a] * fl.invX;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      stq(F + (4 * a + 1 + i) * fs, c, im32 * ((t * fl.S[i] + (i == a ? alpha * fl.P : 0.0)) - ba * fl.S[i]));
  }
}

__device__ __forceinline__ void fluid_flux_point(const double* U, size_t fs, int c, double w, double* F) {
  double g[6], St[3], beta[3];
#pragma unroll
  for (int s = 0; s < 6; ++s) g[s] = ldq(U + (F_GT + s) * fs, c);
#pragma unroll
  for (int i = 0; i < 3; ++i) St[i] = ldq(U + (F_ST + i) * fs, c);
#pragma unroll
  for (int a = 0; a < 3; ++a) beta[a] = ldq(U + (F_BET + a) * fs, c);
  fluid_flux_values(ldq(U + F_CHI * fs, c), g, ldq(U + F_ALP * fs, c), beta, ldq(U + F_ET * fs, c), St, w, F, fs, c);
}

// Divergence of the fluxes at point c, div[q] = sum_a D1_a F^a_q (4th-order centred),
// in two steps per axis so that callers can issue the loads early:
// flux_axis_load fetches F^a_q at the four axis neighbours, flux_axis_add
// accumulates their centred difference.
__device__ __forceinline__ void flux_axis_load(const double* F, size_t fs, int c, const Nbr& nb, int a,
                                               double v[4][4]) {
  const uint32_t nbytes = (uint32_t)(fs * 8);
  const uint32_t o0 = (uint32_t)(c + nb.d[a][1]) * 8u, o1 = (uint32_t)(c + nb.d[a][2]) * 8u;
  const uint32_t o2 = (uint32_t)(c + nb.d[a][4]) * 8u, o3 = (uint32_t)(c + nb.d[a][5]) * 8u;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double* Fa = field_ptr(F, 4 * a + q, fs);
    v[q][0] = bld(Fa, nbytes, o0);
    v[q][1] = bld(Fa, nbytes, o1);
    v[q][2] = bld(Fa, nbytes, o2);
    v[q][3] = bld(Fa, nbytes, o3);
  }
}

__device__ __forceinline__ void flux_axis_add(const double v[4][4], double i12h, double div[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) div[q] += ((v[q][0] - v[q][3]) + 8.0 * (v[q][2] - v[q][1])) * i12h;
}

// The same divergence for one conserved variable q: flux_var_load fetches F^a_q at
// the four neighbours along each axis a, flux_var_div sums the centred differences
// over a = 0, 1, 2 (the order flux_divergence uses). With the Kurganov-Tadmor
// scheme (kt) the pre-pass has stored the whole divergence of q at F[q fs + c]:
// one load, returned as it is.
__device__ __forceinline__ void flux_var_load(const double* F, size_t fs, int c, const Nbr& nb, int q,
                                              double v[3][4], bool kt) {
  const uint32_t nbytes = (uint32_t)(fs * 8);
  if (kt) {
    v[0][0] = bld(field_ptr(F, q, fs), nbytes, (uint32_t)c * 8u);
    return;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double* Fa = field_ptr(F, 4 * a + q, fs);
    v[a][0] = bld(Fa, nbytes, (uint32_t)(c + nb.d[a][1]) * 8u);
    v[a][1] = bld(Fa, nbytes, (uint32_t)(c + nb.d[a][2]) * 8u);
    v[a][2] = bld(Fa, nbytes, (uint32_t)(c + nb.d[a][4]) * 8u);
    v[a][3] = bld(Fa, nbytes, (uint32_t)(c + nb.d[a][5]) * 8u);
  }
}

__device__ __forceinline__ double flux_var_div(const double v[3][4], const DevParams& P, bool kt) {
  if (kt) return v[0][0];
  double div = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) div += ((v[a][0] - v[a][3]) + 8.0 * (v[a][2] - v[a][1])) * P.i12h[a];
  return div;
}

__device__ __forceinline__ void flux_divergence(const double* F, size_t fs, int c, const Nbr& nb, const DevParams& P,
                                                double div[4]) {
  if (P.fluid_scheme == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) div[q] = ldq(field_ptr(F, q, fs), c);
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) div[q] = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v[4][4];
    flux_axis_load(F, fs, c, nb, a, v);
    flux_axis_add(v, P.i12h[a], div);
  }
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
  // With Q[j][k][l] = gt^lm Gt_jkm (last index raised; 27 values), every gt^lm
  // contraction of the quadratic terms becomes a single sum over k, l:
  //   gt^lm Gt^k_li Gt_jkm = Gt^k_li Q[j][k][l],  gt^lm Gt^k_im Gt_klj = Gt^k_im Q[k][j][m].
  double Q[3][3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l)
        Q[j][k][l] = gi[S(l, 0)] * Gl[j][S(k, 0)] + gi[S(l, 1)] * Gl[j][S(k, 1)] + gi[S(l, 2)] * Gl[j][S(k, 2)];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) r += 0.5 * Gd[k] * (Gl[i][S(j, k)] + Gl[j][S(i, k)]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l)
        r += (Gu[k][S(l, i)] * Q[j][k][l] + Gu[k][S(l, j)] * Q[i][k][l]) + Gu[k][S(i, l)] * Q[k][j][l];
    Ric[s] += r;
  }
}

// Conformal-factor part of the Ricci tensor added to Ric:
//   (1/2chi)(DDchi_ij + gt_ij gt^lm DDchi_lm) - (1/4chi^2)(d_i chi d_j chi + 3 gt_ij gt^lm d_l chi d_m chi),
// DDchi_ij = d_i d_j chi - Gt^k_ij d_k chi.
__device__ __forceinline__ void ricci_conformal_factor(double ichi, const double dchi[3], const double d2chi[6],
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
  const double ih = 0.5 * ichi, iq = 0.25 * (ichi * ichi);  // ichi = 1 / chi
#pragma unroll
  for (int s = 0; s < 6; ++s) Ric[s] += ih * (DD[s] + gt[s] * trDD) - iq * (dchi[SI(s)] * dchi[SJ(s)] + 3.0 * gt[s] * dc2);
}

// ---------------------------------------------------------------- streaming right-hand side
// Long-lived per-point intermediates live in an LDS record (slot k of thread t
// at rec[k * stride + t]: consecutive lanes hit consecutive banks). Each phase
// reloads what it needs after the phase fence and writes back what later phases
// use, so the registers hold one phase's working set only.
enum : int {
  R_GI = 0,     // 6  conformal inverse metric gt^ij
  R_E = 6,      // 1  E (normal-observer energy density)
  R_S = 7,      // 3  S_i
  R_P = 10,     // 1  pressure
  R_IX = 11,    // 1  1 / X
  R_SUP = 12,   // 3  S^i
  R_DB = 15,    // 9  d_a beta^i at 3 i + a
  R_RG = 24,    // 3  accumulated Gt^i right-hand side
  R_RIC = 27,   // 6  R_ij (accumulated)
  R_SG = 33,    // 3  S^jk d_i gt_jk
  R_GU = 36,    // 18 Gt^k_ij at 6 k + ij (holds d_a gt_ij at 3 ij + a before the connection phase)
  R_GD = 54,    // 3  Gt^k computed from the metric
  R_DCHI = 57,  // 3  d_a chi
  R_DAL = 60,   // 3  d_a alpha
  R_X = 63,     // 6  -D_iD_j alpha + alpha (R_ij - 8 pi S_ij)
  R_D2A = 69,   // 1  D^i D_i alpha
  R_AUP = 70,   // 6  At^ij
  R_COUNT = 76
};

struct Rec {
  double* p;
  int stride;
  __device__ __forceinline__ double& operator[](int k) const { return p[k * stride]; }
};

// S^jk = S^j S^k / X + P chi gt^jk from the record
__device__ __forceinline__ double rec_Sjk(const Rec& R, double chi, int s) {
  return R[R_SUP + SI(s)] * R[R_SUP + SJ(s)] * R[R_IX] + R[R_P] * chi * R[R_GI + s];
}

// Sink interface: put(f, value) receives the final right-hand side of field f at this point.
// F holds the fluid fluxes of U (fluid_flux_point) at every grid point.
template <class Sink>
__device__ __forceinline__ void bssn_rhs_stream(const double* U, const double* F, size_t fs, const Nbr& nb,
                                                const DevParams& P, double t, const Rec& R, Sink& sink,
                                                bool& prim_fail) {
  const int c = nb.base;
  // centre values kept in registers for the whole evaluation
  const double chi = ldq(U + F_CHI * fs, c);
  const double K = ldq(U + F_K * fs, c);
  const double alpha = ldq(U + F_ALP * fs, c);
  double gt[6], beta[3];
#pragma unroll
  for (int s = 0; s < 6; ++s) gt[s] = ldq(U + (F_GT + s) * fs, c);
#pragma unroll
  for (int i = 0; i < 3; ++i) beta[i] = ldq(U + (F_BET + i) * fs, c);

  // ---- inverse metric and matter at the point
  {
    double gi[6], St[3];
    inv_sym(gt, gi);
#pragma unroll
    for (int i = 0; i < 3; ++i) St[i] = ldq(U + (F_ST + i) * fs, c);
    Fluid fl;
    prim_fail = recover(P.w, chi, gi, ldq(U + F_ET * fs, c), St, fl);
#pragma unroll
    for (int s = 0; s < 6; ++s) R[R_GI + s] = gi[s];
    R[R_E] = fl.E;
    R[R_P] = fl.P;
    R[R_IX] = fl.invX;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      R[R_S + i] = fl.S[i];
      R[R_SUP + i] = fl.Sup[i];
      R[R_RG + i] = 0.0;
      R[R_SG + i] = 0.0;
    }
  }

  // ---- shift: d beta kept; second derivatives consumed into the Gt^i source
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    COSMOS_PHASE();
    double gi[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) gi[s] = R[R_GI + s];
    FieldDerivs d;
    field_derivs<true, true>(U + (F_BET + i) * fs, nb, P, beta, d);
#pragma unroll
    for (int a = 0; a < 3; ++a) R[R_DB + 3 * i + a] = d.d1[a];
    // gt^jk d_j d_k beta^i  and  1/3 gt^lj d_j d_i beta^i (summed over i as the loop runs)
    R[R_RG + i] += contract_sym(gi, d.d2);
#pragma unroll
    for (int l = 0; l < 3; ++l)
      R[R_RG + l] += (gi[S(l, 0)] * d.d2[S(0, i)] + gi[S(l, 1)] * d.d2[S(1, i)] + gi[S(l, 2)] * d.d2[S(2, i)]) * (1.0 / 3.0);
    double r = 0.0;
    if (P.evolve_shift) r = d.advko + (0.75 * ldq(U + (F_GAM + i) * fs, c) - P.eta * beta[i]);
    sink.put(F_BET + i, r);
  }

  // ---- conformal metric: d gt parked in the connection slots, -1/2 gt^lm d_l d_m gt_ij into R_ij
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    COSMOS_PHASE();
    double gi[6], db[3][3];
#pragma unroll
    for (int q = 0; q < 6; ++q) gi[q] = R[R_GI + q];
#pragma unroll
    for (int q = 0; q < 9; ++q) db[q / 3][q % 3] = R[R_DB + q];
    FieldDerivs d;
    field_derivs<true, true>(U + (F_GT + s) * fs, nb, P, beta, d);
    const double wsym = (s == 0 || s == 3 || s == 5) ? 1.0 : 2.0;
    const double Sjk = rec_Sjk(R, chi, s);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R[R_GU + 3 * s + a] = d.d1[a];
      R[R_SG + a] += wsym * Sjk * d.d1[a];
    }
    R[R_RIC + s] = -0.5 * contract_sym(gi, d.d2);
    const int i = SI(s), j = SJ(s);
    const double divb = db[0][0] + db[1][1] + db[2][2];
    double r = d.advko;
#pragma unroll
    for (int k = 0; k < 3; ++k) r += gt[S(i, k)] * db[k][j] + gt[S(j, k)] * db[k][i];
    r -= (2.0 / 3.0) * gt[s] * divb;
    r -= 2.0 * alpha * ldq(U + (F_AT + s) * fs, c);
    sink.put(F_GT + s, r);
  }

  // ---- conformal Christoffels and the Ricci terms quadratic in them
  COSMOS_PHASE();
  {
    double gi[6], dgt[6][3], Gu[3][6], Gd[3], Ric[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      gi[q] = R[R_GI + q];
      Ric[q] = R[R_RIC + q];
#pragma unroll
      for (int a = 0; a < 3; ++a) dgt[q][a] = R[R_GU + 3 * q + a];
    }
    connection_and_quadratic_ricci(dgt, gi, Gu, Gd, Ric);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      R[R_RIC + q] = Ric[q];
#pragma unroll
      for (int k = 0; k < 3; ++k) R[R_GU + 6 * k + q] = Gu[k][q];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) R[R_GD + k] = Gd[k];
  }

  // ---- connection functions: d_j Gt^k into R_ij; advection + dissipation into the Gt^k accumulator
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    COSMOS_PHASE();
    double d1[3];
    R[R_RG + k] += field_advko<true>(U + (F_GAM + k) * fs, nb, P, beta, d1);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      R[R_RIC + s] += 0.5 * (gt[S(k, i)] * d1[j] + gt[S(k, j)] * d1[i]);
    }
  }

  // ---- conformal factor
  COSMOS_PHASE();
  {
    double gi[6], Gu[3][6], Ric[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      gi[q] = R[R_GI + q];
      Ric[q] = R[R_RIC + q];
#pragma unroll
      for (int k = 0; k < 3; ++k) Gu[k][q] = R[R_GU + 6 * k + q];
    }
    FieldDerivs d;
    field_derivs<true, true>(U + F_CHI * fs, nb, P, beta, d);
    ricci_conformal_factor(1.0 / chi, d.d1, d.d2, gt, gi, Gu, Ric);
#pragma unroll
    for (int q = 0; q < 6; ++q) R[R_RIC + q] = Ric[q];
#pragma unroll
    for (int a = 0; a < 3; ++a) R[R_DCHI + a] = d.d1[a];
    const double divb = R[R_DB + 0] + R[R_DB + 4] + R[R_DB + 8];
    sink.put(F_CHI, d.advko + (2.0 / 3.0) * chi * (alpha * K - divb));
  }

  // ---- lapse: D_iD_j alpha, its trace, and X_ij = -D_iD_j alpha + alpha (R_ij - 8 pi S_ij)
  COSMOS_PHASE();
  {
    double gi[6], Gu[3][6], dchi[3];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      gi[q] = R[R_GI + q];
#pragma unroll
      for (int k = 0; k < 3; ++k) Gu[k][q] = R[R_GU + 6 * k + q];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) dchi[a] = R[R_DCHI + a];
    FieldDerivs d;
    field_derivs<true, true>(U + F_ALP * fs, nb, P, beta, d);
    const double* dal = d.d1;
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
    R[R_D2A] = chi * contract_sym(gi, DDa);
    const double Kbg = P.lapse_bg ? -3.0 * P.H0 / (1.0 + 2.0 * P.H0 * t) : 0.0;
    sink.put(F_ALP, d.advko - 2.0 * alpha * (K - Kbg));
    const double ichi = 1.0 / chi;
    const double ix = R[R_IX], pr = R[R_P];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      double Sij = R[R_S + SI(s)] * R[R_S + SJ(s)] * ix + pr * gt[s] * ichi;
      if (P.xsrc) Sij += ldq(P.xsrc + (SRC_SIJ + s) * fs, c);
      R[R_X + s] = -DDa[s] + alpha * (R[R_RIC + s] - 8.0 * PI_D * Sij);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) R[R_DAL + a] = dal[a];
  }

  // ---- trace K: d K feeds the Gt^i source; At^ij, At.At and the K right-hand side
  COSMOS_PHASE();
  {
    double gi[6], At[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      gi[q] = R[R_GI + q];
      At[q] = ldq(U + (F_AT + q) * fs, c);
    }
    double dK[3];
    const double r_adv = field_advko<true>(U + F_K * fs, nb, P, beta, dK);
#pragma unroll
    for (int i = 0; i < 3; ++i)
      R[R_RG + i] -= (4.0 / 3.0) * alpha * (gi[S(i, 0)] * dK[0] + gi[S(i, 1)] * dK[1] + gi[S(i, 2)] * dK[2]);
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
      R[R_AUP + s] = Aup[s];
    }
    const double AA = contract_sym(At, Aup);
    const double Str = (R[R_SUP + 0] * R[R_S + 0] + R[R_SUP + 1] * R[R_S + 1] + R[R_SUP + 2] * R[R_S + 2]) * R[R_IX] +
                       3.0 * R[R_P];
    double EpS = R[R_E] + Str;
    if (P.xsrc) EpS += ldq(P.xsrc + SRC_EPS * fs, c);
    sink.put(F_K, r_adv + (-R[R_D2A] + alpha * (AA + K * K * (1.0 / 3.0)) + 4.0 * PI_D * alpha * EpS));
  }

  // ---- traceless extrinsic curvature
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    COSMOS_PHASE();
    double gi[6], At[6], X[6], db[3][3];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      gi[q] = R[R_GI + q];
      At[q] = ldq(U + (F_AT + q) * fs, c);
      X[q] = R[R_X + q];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) db[q / 3][q % 3] = R[R_DB + q];
    const int i = SI(s), j = SJ(s);
    double d1[3];
    double r = field_advko<true>(U + (F_AT + s) * fs, nb, P, beta, d1);
#pragma unroll
    for (int k = 0; k < 3; ++k) r += At[S(i, k)] * db[k][j] + At[S(j, k)] * db[k][i];
    r -= (2.0 / 3.0) * At[s] * (db[0][0] + db[1][1] + db[2][2]);
    r += chi * (X[s] - gt[s] * contract_sym(gi, X) * (1.0 / 3.0));
    double AAij = 0.0;  // At_ik gt^kl At_lj
#pragma unroll
    for (int k = 0; k < 3; ++k)
      AAij += At[S(i, k)] * (gi[S(k, 0)] * At[S(0, j)] + gi[S(k, 1)] * At[S(1, j)] + gi[S(k, 2)] * At[S(2, j)]);
    r += alpha * (K * At[s] - 2.0 * AAij);
    sink.put(F_AT + s, r);
  }

  // ---- connection functions: final right-hand side
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    COSMOS_PHASE();
    double Aup[6], Gu[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      Aup[q] = R[R_AUP + q];
      Gu[q] = R[R_GU + 6 * i + q];
    }
    const double divb = R[R_DB + 0] + R[R_DB + 4] + R[R_DB + 8];
    double r = R[R_RG + i];
    r -= R[R_GD + 0] * R[R_DB + 3 * i + 0] + R[R_GD + 1] * R[R_DB + 3 * i + 1] + R[R_GD + 2] * R[R_DB + 3 * i + 2];
    r += (2.0 / 3.0) * R[R_GD + i] * divb;
    r -= 2.0 * (Aup[S(i, 0)] * R[R_DAL + 0] + Aup[S(i, 1)] * R[R_DAL + 1] + Aup[S(i, 2)] * R[R_DAL + 2]);
    double inner = contract_sym(Gu, Aup);
    inner -= (1.5 / chi) * (Aup[S(i, 0)] * R[R_DCHI + 0] + Aup[S(i, 1)] * R[R_DCHI + 1] + Aup[S(i, 2)] * R[R_DCHI + 2]);
    r += 2.0 * alpha * inner;
    double Sj[3] = {R[R_S + 0], R[R_S + 1], R[R_S + 2]};
    if (P.xsrc)
#pragma unroll
      for (int j = 0; j < 3; ++j) Sj[j] += ldq(P.xsrc + (SRC_S + j) * fs, c);
    r -= 16.0 * PI_D * alpha * (R[R_GI + S(i, 0)] * Sj[0] + R[R_GI + S(i, 1)] * Sj[1] + R[R_GI + S(i, 2)] * Sj[2]);
    sink.put(F_GAM + i, r);
  }

  // ---- fluid: flux divergence, geometric sources, dissipation
  double div[4];
  COSMOS_PHASE();
  flux_divergence(F, fs, c, nb, P, div);
  const double nbeta[3] = {0.0, 0.0, 0.0};
  const double im32 = 1.0 / (chi * sqrt(chi));
  COSMOS_PHASE();
  {
    double KS = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const double Kij = (ldq(U + (F_AT + s) * fs, c) + gt[s] * K * (1.0 / 3.0)) / chi;
      KS += (s == 0 || s == 3 || s == 5 ? 1.0 : 2.0) * Kij * rec_Sjk(R, chi, s);
    }
    double dummy[3];
    // the Kurganov-Tadmor scheme carries its own dissipation: no KO on the fluid
    const double ko = P.fluid_scheme == 1 ? 0.0 : field_advko<false>(U + F_ET * fs, nb, P, nbeta, dummy);
    const double Sda = R[R_SUP + 0] * R[R_DAL + 0] + R[R_SUP + 1] * R[R_DAL + 1] + R[R_SUP + 2] * R[R_DAL + 2];
    sink.put(F_ET, ko + (im32 * (alpha * KS - Sda) - div[0]));
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    COSMOS_PHASE();
    double sgt = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) sgt += (s == 0 || s == 3 || s == 5 ? 1.0 : 2.0) * rec_Sjk(R, chi, s) * gt[s];
    double dummy[3];
    const double ko = P.fluid_scheme == 1 ? 0.0 : field_advko<false>(U + (F_ST + i) * fs, nb, P, nbeta, dummy);
    double src = -R[R_E] * R[R_DAL + i] +
                 (R[R_S + 0] * R[R_DB + 0 + i] + R[R_S + 1] * R[R_DB + 3 + i] + R[R_S + 2] * R[R_DB + 6 + i]);
    const double ichi = 1.0 / chi;
    src += 0.5 * alpha * (R[R_SG + i] * ichi - sgt * R[R_DCHI + i] * (ichi * ichi));
    sink.put(F_ST + i, ko + (im32 * src - div[1 + i]));
  }
}

}  // namespace cosmos
