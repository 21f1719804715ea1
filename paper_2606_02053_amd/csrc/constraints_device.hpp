// Hamiltonian and momentum constraints (paper, "Physical system settings":
// the constraint part of the Einstein equations, which the initial data
// satisfy) and their deterministic grid reductions.
//   H   = R + 2/3 K^2 - At_ij At^ij - 16 pi E
//   M_i = gt^jk (d_j At_ki - Gt^l_jk At_li - Gt^l_ji At_kl) - 3/(2 chi) At^j_i d_j chi - 2/3 d_i K - 8 pi S_i
// Reduction: per-block tree in LDS, then one block folds the block partials in
// a fixed order -- no floating-point atomics, bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "bssn_device.hpp"

namespace cosmos {

// partial record: sum H^2, sum |M|^2, sum Hn^2, max |H|, max |M|, #non-finite, min alpha, argmin alpha
constexpr int kRedRecord = 8;

// Derivatives from global memory: the centred stencils at the point, periodic wrap in the offsets.
struct DirectDerivs {
  const double* U;
  size_t fs;
  const Nbr& nb;
  const DevParams& P;
  // a value final for this field stays in a register here (as with the LDS source)
  __device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }
  template <bool SECOND>
  __device__ __forceinline__ void get(int f, FieldDerivs& d) {
    // a compiler-level fence per field: the stencil loads of later fields stay after it, so they
    // are not all hoisted to the start and kept live (no instruction is emitted)
    asm volatile("" ::: "memory");
    const double nob[3] = {0.0, 0.0, 0.0};
    field_derivs<SECOND, false, false>(U + (size_t)f * fs, nb, P, nob, d);
  }
};

// H, M_i and the normalised H at the point with linear index c. Der supplies the
// first (and, with SECOND, second) centred derivatives of a field; it is asked for
// them in a fixed order: gt_ij (6, with second), chi (with second), Gt^i (3), K, At_ij (6).
// Every field's derivatives are folded into running sums as they arrive (the Ricci tensor,
// then H; M_i term by term), so that few of them stay live at once.
// der.pin(x) marks a running value as final for the current field (a source with barriers
// between fields keeps it in a register there instead of recomputing it later from every
// field's derivatives); it changes no value.
template <class Der>
__device__ __forceinline__ void constraint_point(const double* __restrict__ U, size_t fs, int c, Der& der,
                                                 const DevParams& P, double& H, double M[3], double& Hn,
                                                 bool& nonfinite) {
  nonfinite = false;
  for (int f = 0; f < NF; ++f) nonfinite = nonfinite || !isfinite(ldq(U + (size_t)f * fs, c));
  // point values are loaded where they are needed (gt_ij twice: for its inverse, then for the
  // chi and Gt^i terms), so that they are not live across the connection
  double gi[6];
  {
    double gt[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) gt[s] = ldq(U + (F_GT + s) * fs, c);
    inv_sym(gt, gi);
  }
  // ---- conformal metric: second derivatives into the Ricci tensor, first into the connection
  double dgt[6][3], Ric[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    FieldDerivs d;
    der.template get<true>(F_GT + s, d);
#pragma unroll
    for (int a = 0; a < 3; ++a) dgt[s][a] = d.d1[a];
    Ric[s] = -0.5 * contract_sym(gi, d.d2);
    der.pin(Ric[s]);
  }
  double Gu[3][6], Gd[3];
  connection_and_quadratic_ricci(dgt, gi, Gu, Gd, Ric);
  double At[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) At[s] = ldq(U + (F_AT + s) * fs, c);
  // the connection's part of M_i: -gt^jk (Gt^l_jk At_li + Gt^l_ji At_kl)
  double Mc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double term = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) term -= Gu[l][S(j, k)] * At[S(l, i)] + Gu[l][S(j, i)] * At[S(k, l)];
        acc += gi[S(j, k)] * term;
      }
    Mc[i] = acc;
  }
  // ---- chi: its terms of the Ricci tensor (they need the connection, free after this) and of M_i
  double Amix[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j) Amix[k][j] = gi[S(k, 0)] * At[S(0, j)] + gi[S(k, 1)] * At[S(1, j)] + gi[S(k, 2)] * At[S(2, j)];
  double AA = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) AA += Amix[i][j] * Amix[j][i];
  const double chi = ldq(U + F_CHI * fs, c);
  double gt[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) gt[s] = ldq(U + (F_GT + s) * fs, c);
  {
    FieldDerivs d;
    der.template get<true>(F_CHI, d);
    ricci_conformal_factor(1.0 / chi, d.d1, d.d2, gt, gi, Gu, Ric);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Mc[i] -= (1.5 / chi) * (Amix[0][i] * d.d1[0] + Amix[1][i] * d.d1[1] + Amix[2][i] * d.d1[2]);
      der.pin(Mc[i]);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) der.pin(Ric[q]);
  }
  // ---- evolved connection functions: gt_k(i d_j) Gt^k
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    FieldDerivs d;
    der.template get<false>(F_GAM + k, d);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      Ric[s] += 0.5 * (gt[S(k, i)] * d.d1[j] + gt[S(k, j)] * d.d1[i]);
      der.pin(Ric[s]);
    }
  }
  const double R = chi * contract_sym(gi, Ric);
  const double K = ldq(U + F_K * fs, c);
  double St[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) St[i] = ldq(U + (F_ST + i) * fs, c);
  Fluid fl;
  recover(P.w, chi, gi, ldq(U + F_ET * fs, c), St, fl);
  if (P.xsrc) {  // scalar field: its energy and momentum densities join the fluid's
    fl.E += ldq(P.xsrc + SRC_E * fs, c);
#pragma unroll
    for (int i = 0; i < 3; ++i) fl.S[i] += ldq(P.xsrc + (SRC_S + i) * fs, c);
    nonfinite = nonfinite || !isfinite(fl.E);
  }
  H = R + (2.0 / 3.0) * K * K - AA - 16.0 * PI_D * fl.E;
  der.pin(H);
  const double den = fabs(R) + (2.0 / 3.0) * K * K + AA + 16.0 * PI_D * fabs(fl.E);
  Hn = (den > 0.0) ? H / den : 0.0;
  der.pin(Hn);
  // ---- trace K
  {
    FieldDerivs d;
    der.template get<false>(F_K, d);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Mc[i] -= (2.0 / 3.0) * d.d1[i];
      der.pin(Mc[i]);
    }
  }
  // ---- At_ab: d_j At_ab enters M_b with gt^ja and, off the diagonal, M_a with gt^jb
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    FieldDerivs d;
    der.template get<false>(F_AT + s, d);
    const int a = SI(s), b = SJ(s);
    Mc[b] += gi[S(0, a)] * d.d1[0] + gi[S(1, a)] * d.d1[1] + gi[S(2, a)] * d.d1[2];
    if (a != b) Mc[a] += gi[S(0, b)] * d.d1[0] + gi[S(1, b)] * d.d1[1] + gi[S(2, b)] * d.d1[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) der.pin(Mc[i]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) M[i] = Mc[i] - 8.0 * PI_D * fl.S[i];
  nonfinite = nonfinite || !isfinite(H) || !isfinite(M[0]) || !isfinite(M[1]) || !isfinite(M[2]);
}

struct Red {
  double sH2, sM2, sHn2, mH, mM, nbad, minA, arg;
};

__device__ __forceinline__ Red red_neutral() { return {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, 1e300}; }

// b follows a in index order; max ignores NaN (keeps the accumulated value);
// the argmin keeps the lowest index among equal minima.
__device__ __forceinline__ Red red_combine(const Red& a, const Red& b) {
  Red r;
  r.sH2 = a.sH2 + b.sH2;
  r.sM2 = a.sM2 + b.sM2;
  r.sHn2 = a.sHn2 + b.sHn2;
  r.mH = (a.mH < b.mH) ? b.mH : a.mH;
  r.mM = (a.mM < b.mM) ? b.mM : a.mM;
  r.nbad = a.nbad + b.nbad;
  const bool takeb = (b.minA < a.minA) || (b.minA == a.minA && b.arg < a.arg);
  r.minA = takeb ? b.minA : a.minA;
  r.arg = takeb ? b.arg : a.arg;
  return r;
}

__device__ __forceinline__ void red_store(double* p, const Red& r) {
  p[0] = r.sH2; p[1] = r.sM2; p[2] = r.sHn2; p[3] = r.mH; p[4] = r.mM; p[5] = r.nbad; p[6] = r.minA; p[7] = r.arg;
}
__device__ __forceinline__ Red red_load(const double* p) { return {p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]}; }

// Wavefront reduction, then one step across the block's four waves: lane l combines
// with lane l ^ m for m = 32, 16, ..., 1 (cross-lane moves, no LDS round trips), lane 0
// of each wave parks its wave's result in LDS, and thread 0 combines the four in a
// fixed order. The order never depends on timing, so the result is bitwise reproducible.
__device__ __forceinline__ Red red_shfl_xor(const Red& a, int m) {
  return {__shfl_xor(a.sH2, m), __shfl_xor(a.sM2, m),  __shfl_xor(a.sHn2, m), __shfl_xor(a.mH, m),
          __shfl_xor(a.mM, m),  __shfl_xor(a.nbad, m), __shfl_xor(a.minA, m), __shfl_xor(a.arg, m)};
}

__device__ __forceinline__ Red block_tree(Red mine, Red* sh) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const Red o = red_shfl_xor(mine, m);
    // the lower lane of each pair keeps the left operand, so both lanes hold the same value
    mine = ((threadIdx.x & m) == 0) ? red_combine(mine, o) : red_combine(o, mine);
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mine;
  __syncthreads();
  return red_combine(red_combine(sh[0], sh[1]), red_combine(sh[2], sh[3]));
}

// H and M_i of point p into the optional output fields.
__device__ __forceinline__ void store_hm(size_t fs, int p, double H, const double M[3], double* __restrict__ Hout,
                                         double* __restrict__ Mout) {
  if (Hout) Hout[p] = H;
  if (Mout)
    for (int q = 0; q < 3; ++q) Mout[(size_t)q * fs + p] = M[q];
}

// The reduction record of one point.
__device__ __forceinline__ Red point_record(const double* __restrict__ U, size_t fs, int p, double H, const double M[3],
                                            double Hn, bool bad) {
  Red mine = red_neutral();
  const double Mn = sqrt(M[0] * M[0] + M[1] * M[1] + M[2] * M[2]);
  const double aH = fabs(H);
  mine.sH2 = H * H;
  mine.sM2 = Mn * Mn;
  mine.sHn2 = Hn * Hn;
  mine.mH = (0.0 < aH) ? aH : 0.0;  // NaN never wins
  mine.mM = (0.0 < Mn) ? Mn : 0.0;
  mine.nbad = bad ? 1.0 : 0.0;
  const double a = ldq(U + F_ALP * fs, p);
  if (a < INFINITY) {
    mine.minA = a;
    mine.arg = (double)p;
  }
  return mine;
}

// Direct variant: one thread per point in linear order, stencils from global memory. Workgroup
// b takes the 256-point blocks b, b + gridDim.x, ... (one block each when launched with one
// workgroup per block) and folds them in that order into its partial record.
__global__ __launch_bounds__(256) void k_constraints(const double* __restrict__ U, size_t fs, DevParams P,
                                                      double* __restrict__ Hout, double* __restrict__ Mout,
                                                      double* __restrict__ part) {
  __shared__ Red sh[4];  // one entry per wave
  Red mine = red_neutral();
  const size_t nblk = (fs + 255) / 256;
  for (size_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int p = (int)(blk * 256 + threadIdx.x);
    if (p < (int)fs) {
      const int i = p % P.n[0];
      const int jk = p / P.n[0];
      const int j = jk % P.n[1];
      const int k = jk / P.n[1];
      Nbr nb;
      make_nbr(nb, i, j, k, P.n);
      DirectDerivs der{U, fs, nb, P};
      double H, M[3], Hn;
      bool bad;
      constraint_point(U, fs, p, der, P, H, M, Hn, bad);
      store_hm(fs, p, H, M, Hout, Mout);
      mine = red_combine(mine, point_record(U, fs, p, H, M, Hn, bad));
    }
  }
  const Red r = block_tree(mine, sh);
  if (threadIdx.x == 0) red_store(part + (size_t)blockIdx.x * kRedRecord, r);
}

__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ part, int nblocks, size_t N3,
                                                          double* __restrict__ norms) {
  __shared__ Red sh[4];  // one entry per wave
  Red acc = red_neutral();
  for (int b = threadIdx.x; b < nblocks; b += 256) acc = red_combine(acc, red_load(part + (size_t)b * kRedRecord));
  const Red r = block_tree(acc, sh);
  if (threadIdx.x == 0) {
    const double n = (double)N3;
    norms[0] = sqrt(r.sH2 / n);
    norms[1] = r.mH;
    norms[2] = sqrt(r.sM2 / n);
    norms[3] = r.mM;
    norms[4] = sqrt(r.sHn2 / n);
    norms[5] = r.nbad;
    norms[6] = r.minA;
    norms[7] = (r.arg < 1e300) ? r.arg : -1.0;
  }
}

}  // namespace cosmos
