// Kurganov-Tadmor fluid fluxes (fluid_scheme 1): the paper's fluid scheme
// (section "Physical system settings" cites Kurganov & Tadmor 2000 and Shibata &
// Font 2005). The fluid right-hand side takes the conservation form
//   d q/dt = -sum_a (Fh^a_{i+1/2} - Fh^a_{i-1/2}) / h_a + sources,
// q = (Et, St_x, St_y, St_z), with the central numerical flux at each interface
//   Fh = 1/2 (F^a(q_L) + F^a(q_R)) - 1/2 c (q_R - q_L),
// q_L, q_R the minmod-limited piecewise-linear reconstructions from the two
// sides, the geometric fields the average of the two neighbouring points, and c
// the largest characteristic-speed magnitude of the two interface states.
//
// One pre-pass kernel per stage forms the whole flux divergence: a workgroup owns
// an 8 x 8 x 4 brick, evaluates every interface flux of the brick once into LDS
// (9x8x4 + 8x9x4 + 8x8x5 = 896 interfaces for 256 points, in three wave-aligned
// segments of 320) and differences them.
// The stage kernel then reads the divergence at the point itself.
#pragma once
#include "bssn_device.hpp"

namespace cosmos {

// Interface bookkeeping of a BX x BY x BZ brick (one point per thread): the
// interfaces normal to each axis (the brick's own plus the one past its upper
// face) and their LDS segments, each padded to whole waves so that every wave
// works on one axis (a compile-time constant inside the interface evaluation).
template <int BX, int BY, int BZ>
struct KtBrick {
  static constexpr int threads = BX * BY * BZ;
  static constexpr int NX = (BX + 1) * BY * BZ, NY = BX * (BY + 1) * BZ, NZ = BX * BY * (BZ + 1);
  static constexpr int PX = (NX + 63) / 64 * 64, PY = (NY + 63) / 64 * 64, PZ = (NZ + 63) / 64 * 64;
  static constexpr int P = PX + PY + PZ;
};
constexpr int kKtBX = 8, kKtBY = 8, kKtBZ = 4;  // brick of k_fluid_kt
using KtB = KtBrick<kKtBX, kKtBY, kKtBZ>;
constexpr int kKtThreads = KtB::threads;
constexpr int kKtP = KtB::P;  // 960 interface slots (the 16 x 4 x 4 brick has as many)
static_assert(KtBrick<16, 4, 4>::P == kKtP, "both bricks use the same LDS segment sizes");

// Smaller-magnitude argument when both have the same strict sign, else 0.
__device__ __forceinline__ double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

// Flux along axis a of one interface state (geometry g, chi, alpha, beta^a;
// conserved q) into Fa[4]; returns the largest magnitude of the two sound-wave
// speeds along a,
//   lambda_pm = alpha / (1 - v^2 w) [v^a (1 - w) pm sqrt(w) sqrt((1 - v^2)(gamma^aa (1 - v^2 w)
//               - (v^a)^2 (1 - w)))] - beta^a,
// v^i = S^i / X, v^2 = S^2 / X^2 (a negative radicand counts as 0; a failed
// recovery has 1/X = 0, so v = 0 there).
template <int a>
__device__ __forceinline__ double kt_state(double w, double sw, double chi, const double gi[6], double alpha,
                                           double ba, const double q[4], double Fa[4]) {
  Fluid fl;
  recover(w, chi, gi, q[0], q + 1, fl);
  const double im32 = 1.0 / (chi * sqrt(chi));
  Fa[0] = im32 * (alpha * fl.Sup[a] - ba * fl.E);
  const double t = alpha * fl.Sup[a] * fl.invX;
#pragma unroll
  for (int i = 0; i < 3; ++i) Fa[1 + i] = im32 * ((t * fl.S[i] + (i == a ? alpha * fl.P : 0.0)) - ba * fl.S[i]);
  const double S2 = fl.Sup[0] * fl.S[0] + fl.Sup[1] * fl.S[1] + fl.Sup[2] * fl.S[2];
  const double va = fl.Sup[a] * fl.invX;
  const double v2 = S2 * fl.invX * fl.invX;
  const double gaa = chi * gi[S(a, a)];
  double rad = (1.0 - v2) * (gaa * (1.0 - v2 * w) - va * va * (1.0 - w));
  const double root = rad > 0.0 ? sqrt(rad) : 0.0;
  const double f = alpha / (1.0 - v2 * w);
  const double lp = f * (va * (1.0 - w) + sw * root) - ba;
  const double lm = f * (va * (1.0 - w) - sw * root) - ba;
  return fmax(fabs(lm), fabs(lp));
}

// Periodic wrap of a coordinate in [-2, 2n] (n >= 8, so one or two corrections).
__device__ __forceinline__ int kt_wrap(int x, int n) {
  x += x < 0 ? n : 0;
  x -= x >= n ? n : 0;
  x -= x >= n ? n : 0;
  return x;
}

// Numerical flux through the interface between points g - e_a and g (global
// coordinates gx, gy, gz of g, unwrapped) into fh[4].
template <int a>
__device__ __forceinline__ void kt_interface(const double* U, size_t fs, const DevParams& P, double sw, int gx, int gy,
                                             int gz, double fh[4]) {
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  int idx[4];  // points g-2, g-1, g, g+1 along a (no wrap needed away from the faces)
  if (gx >= 2 && gx + 1 < n0 && gy >= 2 && gy + 1 < n1 && gz >= 2 && gz + 1 < n2) {
    const int st = a == 0 ? 1 : (a == 1 ? n0 : n0 * n1);
    const int c0 = gx + n0 * (gy + n1 * gz);
#pragma unroll
    for (int o = 0; o < 4; ++o) idx[o] = c0 + (o - 2) * st;
  } else {
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const int x = kt_wrap(gx + (a == 0 ? o - 2 : 0), n0);
      const int y = kt_wrap(gy + (a == 1 ? o - 2 : 0), n1);
      const int z = kt_wrap(gz + (a == 2 ? o - 2 : 0), n2);
      idx[o] = x + n0 * (y + n1 * z);
    }
  }
  const uint32_t nbytes = (uint32_t)(fs * 8);
  auto ld = [&](int f, int o) { return bld(field_ptr(U, f, fs), nbytes, (uint32_t)idx[o] * 8u); };
  // geometry at the interface: average of the two neighbours
  double g[6], gi[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) g[s] = 0.5 * (ld(F_GT + s, 1) + ld(F_GT + s, 2));
  const double chi = 0.5 * (ld(F_CHI, 1) + ld(F_CHI, 2));
  const double alpha = 0.5 * (ld(F_ALP, 1) + ld(F_ALP, 2));
  const double ba = 0.5 * (ld(F_BET + a, 1) + ld(F_BET + a, 2));
  inv_sym(g, gi);
  // fluid: minmod-limited linear reconstruction from both sides
  double qL[4], qR[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double vm = ld(F_ET + q, 0), v0 = ld(F_ET + q, 1), v1 = ld(F_ET + q, 2), v2 = ld(F_ET + q, 3);
    qL[q] = v0 + 0.5 * minmod(v0 - vm, v1 - v0);
    qR[q] = v1 - 0.5 * minmod(v1 - v0, v2 - v1);
  }
  double FL[4], FR[4];
  const double cL = kt_state<a>(P.w, sw, chi, gi, alpha, ba, qL, FL);
  const double cR = kt_state<a>(P.w, sw, chi, gi, alpha, ba, qR, FR);
  const double c = fmax(cL, cR);
#pragma unroll
  for (int q = 0; q < 4; ++q) fh[q] = 0.5 * (FL[q] + FR[q]) - 0.5 * c * (qR[q] - qL[q]);
}

// Brick b of the 8 x 8 x 4 decomposition for workgroup v. Consecutive workgroups
// go round-robin to the 8 XCDs, so workgroups v % 8 == q share XCD q's L2. Where the
// brick grid allows, XCD q owns the q-th slab of brick layers along z and walks it in
// columns of 4 x 4 bricks, z fastest: the bricks resident together on an XCD (about
// 160) are neighbours along all three axes and read each other's halos from its L2.
// Otherwise the bricks are cut into 8 contiguous chunks (nbricks a multiple of 8) or
// taken in order.
__device__ __forceinline__ int kt_brick(int v, int nbricks, int nbx, int nby, int nbz) {
  constexpr int TX = 4, TY = 4;
  if (nbz % 8 == 0 && nbx % TX == 0 && nby % TY == 0) {
    const int zr = nbz / 8, l = v / 8, per = TX * TY * zr;
    const int tile = l / per, w = l % per;
    const int bzl = w % zr, col = w / zr;
    const int bx = (tile % (nbx / TX)) * TX + col % TX, by = (tile / (nbx / TX)) * TY + col / TX;
    return bx + nbx * (by + nby * ((v % 8) * zr + bzl));
  }
  if (nbricks % 8) return v;
  return (v % 8) * (nbricks / 8) + v / 8;
}

// Interface e of axis a's segment: the brick-local coordinates of the point on
// its + side (extent B_a + 1 along a), then the numerical flux into fh[q][slot].
template <int BX, int BY, int a>
__device__ __forceinline__ void kt_segment(const double* U, size_t fs, const DevParams& P, double sw, int e, int slot,
                                           int ox, int oy, int oz, double (*fh)[kKtP]) {
  constexpr int EX = BX + (a == 0), EY = BY + (a == 1);
  const int li = e % EX, lj = (e / EX) % EY, lk = e / (EX * EY);
  double f[4];
  kt_interface<a>(U, fs, P, sw, ox + li, oy + lj, oz + lk, f);
#pragma unroll
  for (int q = 0; q < 4; ++q) fh[q][slot] = f[q];
}

// The divergence for the brick with origin (ox, oy, oz): every interface flux of
// the brick once into LDS, then D[q fs + c] = sum_a (Fh^a_q(c + 1/2) - Fh^a_q(c - 1/2)) / h_a
// for its points inside the grid. All threads of the workgroup call it (it
// synchronises); fh is the workgroup's LDS.
template <int BX, int BY, int BZ>
__device__ __forceinline__ void kt_brick_divergence(const double* U, size_t fs, const DevParams& P, double* D, int ox,
                                                    int oy, int oz, double (*fh)[kKtP]) {
  using KB = KtBrick<BX, BY, BZ>;
  const double sw = sqrt(P.w);
  for (int t = threadIdx.x; t < KB::P; t += KB::threads) {
    // the segments are whole waves: the axis is uniform over the wave
    const int a = __builtin_amdgcn_readfirstlane(t < KB::PX ? 0 : (t < KB::PX + KB::PY ? 1 : 2));
    if (a == 0) {
      if (t < KB::NX) kt_segment<BX, BY, 0>(U, fs, P, sw, t, t, ox, oy, oz, fh);
    } else if (a == 1) {
      if (t - KB::PX < KB::NY) kt_segment<BX, BY, 1>(U, fs, P, sw, t - KB::PX, t, ox, oy, oz, fh);
    } else {
      if (t - KB::PX - KB::PY < KB::NZ) kt_segment<BX, BY, 2>(U, fs, P, sw, t - KB::PX - KB::PY, t, ox, oy, oz, fh);
    }
  }
  __syncthreads();
  const int li = threadIdx.x % BX, lj = (threadIdx.x / BX) % BY, lk = threadIdx.x / (BX * BY);
  const int x = ox + li, y = oy + lj, z = oz + lk;
  if (x < P.n[0] && y < P.n[1] && z < P.n[2]) {
    // interface slots: the one at the point's minus side and the next along each axis
    const int sx = li + (BX + 1) * (lj + BY * lk);
    const int sy = KB::PX + li + BX * (lj + (BY + 1) * lk);
    const int sz = KB::PX + KB::PY + li + BX * (lj + BY * lk);
    const size_t c = (size_t)x + (size_t)P.n[0] * ((size_t)y + (size_t)P.n[1] * z);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double div = (fh[q][sx + 1] - fh[q][sx]) * P.ih[0];
      div += (fh[q][sy + BX] - fh[q][sy]) * P.ih[1];
      div += (fh[q][sz + BX * BY] - fh[q][sz]) * P.ih[2];
      D[q * fs + c] = div;
    }
  }
  __syncthreads();  // fh may be refilled for another brick
}

// Workgroups of k_fluid_kt: one per 8 x 8 x 4 brick (partial bricks at the upper faces).
inline unsigned kt_bricks(const DevParams& P) {
  return (unsigned)(((P.n[0] + kKtBX - 1) / kKtBX) * ((P.n[1] + kKtBY - 1) / kKtBY) * ((P.n[2] + kKtBZ - 1) / kKtBZ));
}

// The Kurganov-Tadmor divergence of one grid, one 8 x 8 x 4 brick per workgroup.
__global__ __launch_bounds__(kKtThreads) void k_fluid_kt(const double* U, size_t fs, DevParams P, double* D) {
  __shared__ double fh[4][kKtP];
  const int nbx = (P.n[0] + kKtBX - 1) / kKtBX, nby = (P.n[1] + kKtBY - 1) / kKtBY;
  const int nbz = (P.n[2] + kKtBZ - 1) / kKtBZ;
  const int b = kt_brick(blockIdx.x, nbx * nby * nbz, nbx, nby, nbz);
  const int ox = (b % nbx) * kKtBX, oy = ((b / nbx) % nby) * kKtBY, oz = (b / (nbx * nby)) * kKtBZ;
  kt_brick_divergence<kKtBX, kKtBY, kKtBZ>(U, fs, P, D, ox, oy, oz, fh);
}

}  // namespace cosmos
