// LDS-staged stage kernel: one 256-thread workgroup owns a BX x BY x BZ brick
// (one point per thread). The 25 fields are visited in a fixed order; for each
// field the workgroup copies the brick plus its periodic halo of width 3 (the
// ghost-zone fill, done as an index wrap while loading) from HBM into an LDS
// buffer with ~NH/256 independent coalesced loads per thread, and every thread
// then forms that field's derivatives at its point from LDS with
// compile-time-offset reads. The copy of the next field is issued before the
// current field's arithmetic and written to the second LDS buffer after it, so
// its latency hides behind the FP64 work. A workgroup walks several bricks and
// loads the next brick's first fields, epilogue operands and point values during
// the last phases of the current one. Long-lived per-point intermediates
// (R3_* slots) stay in registers: one wave per SIMD is resident anyway (the
// fused point evaluation needs ~300 registers), so the VGPR + AGPR file holds
// them, and LDS only carries the two halo buffers. The fluid fluxes come from a
// pointwise pre-pass (fluid_flux_point) and are differentiated from global loads.
//
// The arithmetic is that of bssn_rhs_stream in bssn_device.hpp (same
// operations in the same order); only where the operands come from differs, so
// the two variants agree to rounding.
#pragma once
#include <type_traits>

#include "bssn_device.hpp"

namespace cosmos {

enum : int {
  R3_GI = 0,     // 6  gt^ij
  R3_E = 6,      // 1  E
  R3_S = 7,      // 3  S_i
  R3_P = 10,     // 1  P
  R3_IX = 11,    // 1  1 / X
  R3_DB = 12,    // 9  d_a beta^i at 3 i + a
  R3_RG = 21,    // 3  accumulated Gt^i right-hand side
  R3_RX = 24,    // 6  R_ij, then X_ij = -D_iD_j alpha + alpha (R_ij - 8 pi S_ij)
  R3_SG = 30,    // 3  S^jk d_i gt_jk
  R3_GU = 33,    // 18 d_a gt_ij at 3 ij + a, then Gt^k_ij at 6 k + ij
  R3_DCHI = 51,  // 3
  R3_DAL = 54,   // 3
  R3_D2A = 57,   // 1
  R3_COUNT = 58
};

template <int BX, int BY, int BZ>
struct Brick {
  static constexpr int X = BX, Y = BY, Z = BZ;   // brick (one point per thread)
  static constexpr int XO = 3;                  // x offset of the brick in its halo box
  static constexpr int HX = BX + 6, HY = BY + 6, HZ = BZ + 6;
  static constexpr int NH = HX * HY * HZ;       // halo-box points
  static constexpr int NQ = (NH + 255) / 256;   // loads per thread per field
  static constexpr int NP = NQ * 256;            // padded LDS buffer: every thread copies NQ points
  static constexpr int SY = HX, SZ = HX * HY;   // LDS strides
  static constexpr int NOFF = NQ;                // per-thread halo offsets
  static constexpr int LDS_DOUBLES = 2 * NP;       // two halo buffers
  static_assert(BX * BY * BZ == 256, "one point per thread");
  static_assert(LDS_DOUBLES * 8 <= 160 * 1024, "LDS budget");
};

// Workgroup barrier for LDS staging. __syncthreads() carries a workgroup-scope release fence,
// which waits for every outstanding global load and store of the wave (s_waitcnt vmcnt(0)) and so
// drains the prefetch of later fields and epilogue operands at every phase. Here only the wave's
// own LDS operations are completed (lgkmcnt 0: its halo writes are visible and its reads of a
// buffer about to be refilled have returned) before s_barrier; global memory is not ordered.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt not waited on
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Brick of round `it` for workgroup `blk` in the XCD-blocked order (T.order 2, set up by the
// launcher): XCD blk % 8 owns a slab of T.zr brick layers, and its workgroups take one
// T.gx x T.gy x T.gz block of bricks per round. False when the workgroup's slot lies outside the
// grid's bricks in this round.
__device__ __forceinline__ bool blocked_brick(const Tile& T, int it, int blk, int& bxi, int& byi, int& bzi) {
  const int l = blk >> 3, gxy = T.ngx * T.ngy;
  bxi = (it % T.ngx) * T.gx + l % T.gx;
  byi = ((it / T.ngx) % T.ngy) * T.gy + (l / T.gx) % T.gy;
  const int bzl = (it / gxy) * T.gz + l / (T.gx * T.gy);
  bzi = (blk & 7) * T.zr + bzl;
  return bxi < T.nbx && byi < T.nby && bzl < T.zr && bzi < T.nbz;
}

// Stencil taps read from the LDS halo box: c points at the thread's centre.
template <class B>
__device__ __forceinline__ void lds_line(const double* c, int a, double v[7]) {
  const int st = a == 0 ? 1 : (a == 1 ? B::SY : B::SZ);
#pragma unroll
  for (int o = 0; o < 7; ++o) v[o] = c[(o - 3) * st];
}

template <class B>
__device__ __forceinline__ double lds_mixed(const double* c, int a, int b, double i144) {
  const int sa = a == 0 ? 1 : (a == 1 ? B::SY : B::SZ);
  const int sb = b == 0 ? 1 : (b == 1 ? B::SY : B::SZ);
  const int oa[4] = {-2, -1, 1, 2};
  double in[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const double* r = c + oa[p] * sa;
    in[p] = (r[-2 * sb] - r[2 * sb]) + 8.0 * (r[sb] - r[-sb]);
  }
  return ((in[0] - in[3]) + 8.0 * (in[2] - in[1])) * i144;
}

template <class B, bool SECOND, bool ADV, bool KO = true>
__device__ __forceinline__ void lds_derivs(const double* c, const DevParams& P, const double beta[3], FieldDerivs& r) {
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v[7];
    lds_line<B>(c, a, v);
    double d2 = 0.0;
    op_line<SECOND, ADV, KO>(v, beta[a], P.i12h[a], P.i12h2[a], P.i24h[a], P.iko[a], r.d1[a], d2, acc);
    if (SECOND) r.d2[S(a, a)] = d2;
  }
  r.advko = acc;
  if (SECOND) {
    r.d2[S(0, 1)] = lds_mixed<B>(c, 0, 1, P.i144[0]);
    r.d2[S(0, 2)] = lds_mixed<B>(c, 0, 2, P.i144[1]);
    r.d2[S(1, 2)] = lds_mixed<B>(c, 1, 2, P.i144[2]);
  }
}

// Order in which the fields are staged (one per phase).
constexpr int kStageOrder[NF] = {F_BET,    F_BET + 1, F_BET + 2, F_GT,     F_GT + 1, F_GT + 2, F_GT + 3,
                                 F_GT + 4, F_GT + 5,  F_GAM,     F_GAM + 1, F_GAM + 2, F_CHI,   F_ALP,
                                 F_K,      F_AT,      F_AT + 1,  F_AT + 2, F_AT + 3, F_AT + 4, F_AT + 5,
                                 F_ET,     F_ST,      F_ST + 1,  F_ST + 2};
// Phases whose field is differentiated twice (second and mixed derivatives: the shift, the
// conformal metric, chi and the lapse); the others take first derivatives only.
constexpr bool kSecondDerivs[NF] = {true,  true,  true,  true,  true,  true,  true,  true,  true,
                                    false, false, false, true,  true,  false, false, false, false,
                                    false, false, false, false, false, false, false};
constexpr int kPrefetch = 2;  // fields in flight ahead of the one being processed

// Fields whose right-hand side becomes final in each phase, in the order they are
// handed to the sink (the Gt^i right-hand sides complete in the trace-K phase).
constexpr int kPutCount[NF] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0, 1, 1, 4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
constexpr int kPutField[NF][4] = {
    {F_BET}, {F_BET + 1}, {F_BET + 2}, {F_GT}, {F_GT + 1}, {F_GT + 2}, {F_GT + 3}, {F_GT + 4}, {F_GT + 5},
    {}, {}, {}, {F_CHI}, {F_ALP}, {F_K, F_GAM, F_GAM + 1, F_GAM + 2},
    {F_AT}, {F_AT + 1}, {F_AT + 2}, {F_AT + 3}, {F_AT + 4}, {F_AT + 5}, {F_ET}, {F_ST}, {F_ST + 1}, {F_ST + 2}};
// The RK4 epilogue operands of phase p's outputs (u_n and/or acc at the point) are
// loaded kEpiAhead phases earlier: they come from HBM, whose latency exceeds one phase.
constexpr int kEpiAhead = 3;

__device__ __forceinline__ int wrap_halo(int x, int n) {
  x = x < 0 ? x + n : x;
  x = x >= n ? x - n : x;
  return x >= n ? x - n : x;
}

// Cooperative copy of the fields' halo boxes: a ring of kPrefetch register
// sets (slot 0 = next field to commit to LDS), rotated with constant indices.
template <class B>
struct HaloCopy {
  uint32_t goffb[B::NQ];  // byte offset of this thread's halo-box points in a field (wrapped)
  double v[kPrefetch][B::NQ];
  __device__ __forceinline__ void init(int i0, int j0, int k0, const int n[3]) { offsets(i0, j0, k0, n, goffb); }
  static __device__ __forceinline__ void offsets(int i0, int j0, int k0, const int n[3], uint32_t goffb[B::NQ]) {
    // Most bricks' halo boxes lie inside the grid (82 % of the 16x4x4 bricks at 256^3): no
    // wrap is needed there, and the choice is uniform over the workgroup.
    const bool inside = i0 >= 3 && i0 + B::HX - 3 <= n[0] && j0 >= 3 && j0 + B::HY - 3 <= n[1] && k0 >= 3 &&
                        k0 + B::HZ - 3 <= n[2];
    if (inside) {
      const int base = (i0 - 3) + n[0] * ((j0 - 3) + n[1] * (k0 - 3));
#pragma unroll
      for (int q = 0; q < B::NQ; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int ee = e < B::NH ? e : 0;
        const int hx = ee % B::HX, hy = (ee / B::HX) % B::HY, hz = ee / (B::HX * B::HY);
        goffb[q] = 8u * (uint32_t)(base + hx + n[0] * (hy + n[1] * hz));
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < B::NQ; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int ee = e < B::NH ? e : 0;
      const int hx = ee % B::HX, hy = (ee / B::HX) % B::HY, hz = ee / (B::HX * B::HY);
      // Brick origins lie inside the grid and n >= 8, so a halo coordinate lies in
      // [-3, 3n): one conditional add and two conditional subtracts wrap it (cheaper
      // than an integer remainder by a run-time n).
      goffb[q] = 8u * (uint32_t)(wrap_halo(i0 + hx - 3, n[0]) +
                                 n[0] * (wrap_halo(j0 + hy - 3, n[1]) + n[1] * wrap_halo(k0 + hz - 3, n[2])));
    }
  }
  template <int SLOT>
  __device__ __forceinline__ void fetch(const double* F, uint32_t nbytes) {
    fetch_at<SLOT>(F, nbytes, goffb);
  }
  template <int SLOT>
  __device__ __forceinline__ void fetch_at(const double* F, uint32_t nbytes, const uint32_t off[B::NQ]) {
    static_assert(SLOT < kPrefetch, "ring slot");
#pragma unroll
    for (int q = 0; q < B::NQ; ++q)
      v[SLOT][q] = bld(F, nbytes, off[q]);
  }
  __device__ __forceinline__ void commit_and_rotate(double* buf) {
#pragma unroll
    for (int q = 0; q < B::NQ; ++q)
      buf[threadIdx.x + 256 * q] = v[0][q];
#pragma unroll
    for (int d = 0; d + 1 < kPrefetch; ++d)
#pragma unroll
      for (int q = 0; q < B::NQ; ++q) v[d][q] = v[d + 1][q];
  }
};

// Halo box for staging by LDS-direct loads: x runs from i0 - 4 to i0 + BX + 3 (BX + 8 points,
// one more on each side than the stencils need), so that with n0 even every aligned pair of
// x-neighbours (2m, 2m + 1) of the box is two consecutive doubles in memory, 16-byte aligned,
// also where the box wraps around the periodic boundary. One lane moves one such pair per load
// (buffer_load_dwordx4 into LDS), NR rounds of 256 pairs per field.
template <int BX, int BY, int BZ>
struct DBrick {
  static constexpr int X = BX, Y = BY, Z = BZ;
  static constexpr int XO = 4;
  static constexpr int HX = BX + 8, HY = BY + 6, HZ = BZ + 6;
  static constexpr int NPR = HX / 2;                 // pairs per row
  static constexpr int NPAIR = NPR * HY * HZ;
  static constexpr int NR = (NPAIR + 255) / 256;     // load rounds per field
  static constexpr int NP = NR * 512;                // doubles per LDS buffer (padded to whole rounds)
  static constexpr int SY = HX, SZ = HX * HY;
  static constexpr int NOFF = 2 * NR;  // two offset sets: fields with and without second derivatives
  static_assert(BX * BY * BZ == 256 && BX % 2 == 0, "one point per thread, even brick width");
};
constexpr int kRing = 5;      // LDS halo buffers of the direct-load ring (25 phases = 5 rounds of the ring)
constexpr int kDmaAhead = 4;  // fields whose loads are in flight ahead of the one being processed
// With the scalar field, its 10 source values at the point are loaded in phase kSrcPhase (the
// second connection-function phase), three phases before the first use.
constexpr int kSrcPhase = 10, kSrcLoads = 10;
static_assert(NF % kRing == 0 && kDmaAhead == kRing - 1, "ring slot = phase mod kRing, across bricks");

// Wait until at most n vector-memory operations of this wave are outstanding (expcnt and
// lgkmcnt not waited on). Loads complete in issue order, so a load is complete once n newer
// ones have been issued and the count drops to n.
__device__ __forceinline__ void wait_vm(int n) {
  switch (n) {  // the count is an instruction immediate
    case 0: __builtin_amdgcn_s_waitcnt(0x0F70); break;
    case 5: __builtin_amdgcn_s_waitcnt(0x0F75); break;
    case 6: __builtin_amdgcn_s_waitcnt(0x0F76); break;
    case 10: __builtin_amdgcn_s_waitcnt(0x0F7A); break;
    case 12: __builtin_amdgcn_s_waitcnt(0x0F7C); break;
    case 15: __builtin_amdgcn_s_waitcnt(0x0F7F); break;
    case 18: __builtin_amdgcn_s_waitcnt(0x4F72); break;
    case 25: __builtin_amdgcn_s_waitcnt(0x4F79); break;
    default: __builtin_amdgcn_s_waitcnt(0x0F70); break;  // any other count: wait for everything
  }
}

// LDS-direct halo staging: each lane holds the byte offsets of its pair in a field (one per
// round); a fetch issues NR loads that write the field's halo box straight into an LDS buffer,
// round q of wave w filling pairs [256 q + 64 w, 256 q + 64 w + 64). No registers hold the data.
template <class B>
struct HaloDma {
  uint32_t goffb[B::NOFF];
  __device__ __forceinline__ void init(int i0, int j0, int k0, const int n[3]) { offsets(i0, j0, k0, n, goffb); }
  // Box points that no stencil reads load a pair from a cache line the brick reads anyway, so
  // that only the lines the stencils use are requested. Offsets [0, NR): fields with second
  // derivatives -- x-halo reads come from rows within +-2 of the brick in y and z with the other
  // coordinate inside (mixed xy and xz derivatives; +-3 axial ones in rows inside in both), the
  // other rows are read only at the brick's x-range (y and z stencils, mixed yz ones within
  // +-2 in both), and the box's corner rows not at all. Offsets [NR, 2 NR): fields with first
  // derivatives only -- axial stencils: the x-halo in rows inside in y and z, the brick's
  // x-range in rows inside in one of them, nothing elsewhere.
  static __device__ __forceinline__ void offsets(int i0, int j0, int k0, const int n[3], uint32_t goffb[B::NOFF]) {
#pragma unroll
    for (int q = 0; q < B::NR; ++q) {
      const int m = threadIdx.x + 256 * q;
      const int mm = m < B::NPAIR ? m : 0;  // padding lanes load an in-box pair into the padding
      const int hx2 = mm % B::NPR, dy = (mm / B::NPR) % B::HY - 3, dz = mm / (B::NPR * B::HY) - 3;
      const bool yin = dy >= 0 && dy < B::Y, zin = dz >= 0 && dz < B::Z;
      const bool y2 = dy >= -2 && dy < B::Y + 2, z2 = dz >= -2 && dz < B::Z + 2;
      const int hxi = min(max(hx2, 2), B::NPR - 3);  // the pair moved into the brick's x-range
      const int x = wrap_halo(i0 - 4 + 2 * hx2, n[0]), xi = wrap_halo(i0 - 4 + 2 * hxi, n[0]);
      const int y = wrap_halo(j0 + dy, n[1]), z = wrap_halo(k0 + dz, n[2]);
      // a row that is read nowhere is replaced by the row with y moved inside the brick (read by
      // the z stencils of both sets at the brick's x-range)
      const int yc = wrap_halo(j0 + min(max(dy, 0), B::Y - 1), n[1]);
      const bool xh2 = (y2 && zin) || (yin && z2), row2 = yin || zin || (y2 && z2);
      goffb[q] = 8u * (uint32_t)((xh2 ? x : xi) + n[0] * ((row2 ? y : yc) + n[1] * z));
      // first derivatives: rows inside in y or z are read, the others replaced as above
      const bool xh1 = yin && zin, row1 = yin || zin;
      goffb[B::NR + q] = 8u * (uint32_t)((xh1 ? x : xi) + n[0] * ((row1 ? y : yc) + n[1] * z));
    }
  }
  // one field's halo box: SECOND selects the offset set of the fields with second derivatives
  __device__ __forceinline__ void fetch(const double* F, uint32_t nbytes, double* buf, bool second = true) const {
    fetch_at(F, nbytes, buf, second ? goffb : goffb + B::NR);
  }
  static __device__ __forceinline__ void fetch_at(const double* F, uint32_t nbytes, double* buf,
                                                  const uint32_t off[B::NR]) {
    const __amdgpu_buffer_rsrc_t r = field_rsrc(F, nbytes);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int q = 0; q < B::NR; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          r, (__attribute__((address_space(3))) void*)(buf + 2 * (256 * q + 64 * w)), 16, off[q], 0, 0, 0);
  }
};

// State carried from one brick to the next by a workgroup that walks several
// bricks: the halo ring (the next fields to commit), the epilogue-operand ring
// (slot d = phase + d) and the 25 values of the thread's point.
// Halo staging of a brick type: a register ring (Brick) or LDS-direct loads (DBrick).
template <class B> struct HaloOf { using type = HaloCopy<B>; static constexpr bool dma = false; };
template <int BX, int BY, int BZ> struct HaloOf<DBrick<BX, BY, BZ>> {
  using type = HaloDma<DBrick<BX, BY, BZ>>;
  static constexpr bool dma = true;
};

template <class B, class Pre>
struct LdsCarry {
  typename HaloOf<B>::type hc;
  Pre ep[kEpiAhead + 1][4];
  double cen[NF];
};

// The brick a workgroup processes next (valid is uniform): its halo offsets, this
// thread's point in it (0 for a thread outside the grid), and the arrays and field
// size of its grid (another run's in the batched form; the current ones otherwise).
template <class B>
struct NextBrick {
  bool valid;
  int c;
  uint32_t goffb[B::NOFF];
  const double* U;   // stage input
  const double* un;  // RK4 epilogue operands
  const double* acc;
  size_t fs;
};

// Loads of the first brick of a workgroup (later bricks are prefetched during the
// previous one): the epilogue operands of phases 0 .. kEpiAhead-1, the point's values, and
// the first fields -- 0 .. kPrefetch-1 into the register ring, or with LDS-direct staging
// 0 .. kDmaAhead-1 into ring slots 0 .. kDmaAhead-1 at `ring` (issued last, so that waiting
// for the other loads does not wait for them).
template <class B, class Sink, class Pre>
__device__ __forceinline__ void lds_carry_fill(LdsCarry<B, Pre>& cy, const double* U, size_t fs, const Sink& sink,
                                               int c, double* ring = nullptr) {
  static_assert(kPrefetch >= 1 && kPrefetch <= 3, "ring depth");
  const uint32_t nbytes = (uint32_t)(fs * 8);
  if constexpr (!HaloOf<B>::dma) {
    cy.hc.template fetch<0>(field_ptr(U, kStageOrder[0], fs), nbytes);
    if constexpr (kPrefetch > 1) cy.hc.template fetch<(kPrefetch > 1 ? 1 : 0)>(field_ptr(U, kStageOrder[1], fs), nbytes);
    if constexpr (kPrefetch > 2) cy.hc.template fetch<(kPrefetch > 2 ? 2 : 0)>(field_ptr(U, kStageOrder[2], fs), nbytes);
  }
#pragma unroll
  for (int d = 0; d < kEpiAhead; ++d)
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < kPutCount[d]) cy.ep[d][k] = sink.preload_at(kPutField[d][k], c);
#pragma unroll
  for (int f = 0; f < NF; ++f) cy.cen[f] = bld(field_ptr(U, f, fs), nbytes, (uint32_t)c * 8u);
  if constexpr (HaloOf<B>::dma) {
#pragma unroll
    for (int q = 0; q < kDmaAhead; ++q) cy.hc.fetch(field_ptr(U, kStageOrder[q], fs), nbytes, ring + q * B::NP);
  }
}

// The whole right-hand side of one point with LDS-staged stencils. All threads
// of the workgroup must call it (it contains barriers); `active` marks threads
// whose point lies inside the grid. On entry `cy` holds this brick's ring,
// epilogue operands and point values; if nx.valid, on return it holds those of
// the next brick (loaded during the last phases of this one).
// SC: the scalar field's source arrays (P.xsrc) are added in the K, At and Gt
// equations: 0 none, 1 read through buffer descriptors (P.xsrc uniform in scalar
// registers, a kernel argument), 2 read with plain loads (P.xsrc formed per work item).
template <class B, bool KT, int SC, class Sink, class Pre>
__device__ __forceinline__ void bssn_rhs_lds(const double* U, const double* F, size_t fs, const DevParams& P, double t,
                                             int c, bool active, LdsCarry<B, Pre>& cy, const NextBrick<B>& nx,
                                             double* buf0, double* buf1, Sink& sink, bool& prim_fail) {
  struct {  // the per-point record, indexed by compile-time constants only (kept in registers)
    double v[R3_COUNT];
    __device__ __forceinline__ double& operator[](int k) { return v[k]; }
  } R;
  const int lx = threadIdx.x % B::X, ly = (threadIdx.x / B::X) % B::Y, lz = threadIdx.x / (B::X * B::Y);
  const int cidx = (lx + B::XO) + B::SY * ((ly + 3) + B::HY * (lz + 3));
  constexpr bool dma = HaloOf<B>::dma;  // LDS-direct staging: buf0 is the ring of kRing buffers
  auto& hc = cy.hc;
  auto& ep = cy.ep;
  const uint32_t nbytes = (uint32_t)(fs * 8);
  auto xsrc = [&](int q) -> double {  // source array q at this point (SC != 0)
    if constexpr (SC == 1) return bld(field_ptr(P.xsrc, q, fs), nbytes, (uint32_t)c * 8u);
    return P.xsrc[(size_t)q * fs + c];
  };

  // centre values (registers); inactive threads hold a valid point's values and never store
  const double chi = cy.cen[F_CHI];
  const double ichi = 1.0 / chi;
  const double K = cy.cen[F_K];
  const double alpha = cy.cen[F_ALP];
  double gt[6], beta[3], At[6], Gam[3];
#pragma unroll
  for (int s = 0; s < 6; ++s) gt[s] = cy.cen[F_GT + s];
#pragma unroll
  for (int q = 0; q < 3; ++q) beta[q] = cy.cen[F_BET + q];
#pragma unroll
  for (int s = 0; s < 6; ++s) At[s] = cy.cen[F_AT + s];
#pragma unroll
  for (int q = 0; q < 3; ++q) Gam[q] = cy.cen[F_GAM + q];

  // epilogue operands of phase ph (of this brick, or of the next one when ph >= NF)
  auto epi_load = [&](int ph, auto slot) {
    if (ph < NF) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < kPutCount[ph]) ep[decltype(slot)::value][k] = sink.preload(kPutField[ph][k]);
    } else if (nx.valid) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < kPutCount[ph - NF])
          ep[decltype(slot)::value][k] = sink.preload_from(kPutField[ph - NF][k], nx.c, nx.un, nx.acc, nx.fs);
    }
  };
  {
    double gi[6], St[3];
    inv_sym(gt, gi);
#pragma unroll
    for (int q = 0; q < 3; ++q) St[q] = cy.cen[F_ST + q];
    Fluid fl;
    prim_fail = active && recover(P.w, chi, gi, cy.cen[F_ET], St, fl);
#pragma unroll
    for (int s = 0; s < 6; ++s) R[R3_GI + s] = gi[s];
    R[R3_E] = fl.E;
    R[R3_P] = fl.P;
    R[R3_IX] = fl.invX;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      R[R3_S + q] = fl.S[q];
      R[R3_RG + q] = 0.0;
      R[R3_SG + q] = 0.0;
    }
  }
  if constexpr (dma) {
    wait_vm(3 * B::NR);  // field 0 is in LDS once the loads of fields 1 .. 3, issued after it, remain
  } else {
    hc.commit_and_rotate(buf0);
  }
  lds_barrier();

  // Phase p processes field kStageOrder[p] from LDS buffer p & 1 (register ring: at its start
  // the field p + kPrefetch is fetched into the last register slot, at its end the field p + 1
  // is committed to the other buffer) or from ring slot p % kRing (LDS-direct: at its start the
  // loads of field p + kDmaAhead go to slot (p - 1) % kRing, free since the last barrier; at its
  // end the wave waits until field p + 1 has landed).
  int phase = 0;
  auto cur = [&]() -> const double* {
    if constexpr (dma) return buf0 + (phase % kRing) * B::NP + cidx;
    return ((phase & 1) ? buf1 : buf0) + cidx;
  };
  auto prefetch = [&]() {
    if constexpr (dma) {
      epi_load(phase + kEpiAhead, std::integral_constant<int, kEpiAhead>());
      double* slot = buf0 + ((phase + kDmaAhead) % kRing) * B::NP;
      if (phase + kDmaAhead < NF)
        hc.fetch(field_ptr(U, kStageOrder[phase + kDmaAhead], fs), nbytes, slot, kSecondDerivs[phase + kDmaAhead]);
      else if (nx.valid)
        hc.fetch_at(field_ptr(nx.U, kStageOrder[phase + kDmaAhead - NF], nx.fs), (uint32_t)(nx.fs * 8), slot, nx.goffb);
    } else {
      if (phase + kPrefetch < NF)
        hc.template fetch<kPrefetch - 1>(field_ptr(U, kStageOrder[phase + kPrefetch], fs), nbytes);
      else if (nx.valid)
        hc.template fetch_at<kPrefetch - 1>(field_ptr(nx.U, kStageOrder[phase + kPrefetch - NF], nx.fs),
                                            (uint32_t)(nx.fs * 8), nx.goffb);
      epi_load(phase + kEpiAhead, std::integral_constant<int, kEpiAhead>());
    }
  };
  auto advance = [&](int) {
#pragma unroll
    for (int d = 0; d < kEpiAhead; ++d)
#pragma unroll
      for (int k = 0; k < 4; ++k) ep[d][k] = ep[d + 1][k];
    if constexpr (dma) {
      // field phase + 1 was issued kDmaAhead - 1 phases ago; the phases since issued one field
      // each, except past the brick's last field when there is no next brick
      const int v = nx.valid ? 1 : 0;
      const int newer = phase <= NF - 1 - kDmaAhead ? 3 : (phase == NF - kDmaAhead ? 2 + v : (phase == NF - 3 ? 1 + 2 * v : 3 * v));
      // the scalar field's source loads, issued in phase kSrcPhase after that phase's halo
      // loads, are newer than the field awaited at the end of the phases kSrcPhase .. kSrcPhase + 2
      const int extra = (SC != 0 && phase >= kSrcPhase && phase < kSrcPhase + 3) ? kSrcLoads : 0;
      wait_vm(newer * B::NR + extra);
    } else {
      if (phase + 1 < NF) hc.commit_and_rotate((phase & 1) ? buf0 : buf1);
    }
    lds_barrier();
    ++phase;
  };
  double Sup[3];  // S^j = chi gt^jk S_k
#pragma unroll
  for (int j = 0; j < 3; ++j)
    Sup[j] = chi * (R[R3_GI + S(j, 0)] * R[R3_S + 0] + R[R3_GI + S(j, 1)] * R[R3_S + 1] + R[R3_GI + S(j, 2)] * R[R3_S + 2]);
  auto Sjk_at = [&](int s) { return Sup[SI(s)] * Sup[SJ(s)] * R[R3_IX] + R[R3_P] * chi * R[R3_GI + s]; };

  // ---- shift
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    prefetch();
    if (active) {
      double gi[6];
#pragma unroll
      for (int s = 0; s < 6; ++s) gi[s] = R[R3_GI + s];
      FieldDerivs d;
      lds_derivs<B, true, true>(cur(), P, beta, d);
#pragma unroll
      for (int a = 0; a < 3; ++a) R[R3_DB + 3 * i + a] = d.d1[a];
      R[R3_RG + i] += contract_sym(gi, d.d2);
#pragma unroll
      for (int l = 0; l < 3; ++l)
        R[R3_RG + l] +=
            (gi[S(l, 0)] * d.d2[S(0, i)] + gi[S(l, 1)] * d.d2[S(1, i)] + gi[S(l, 2)] * d.d2[S(2, i)]) * (1.0 / 3.0);
      double r = 0.0;
      if (P.evolve_shift) r = d.advko + (0.75 * Gam[i] - P.eta * beta[i]);
      sink.put(F_BET + i, r, ep[0][0]);
    }
    advance(0);
  }

  // ---- conformal metric
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    prefetch();
    if (active) {
      double gi[6], db[3][3];
#pragma unroll
      for (int q = 0; q < 6; ++q) gi[q] = R[R3_GI + q];
#pragma unroll
      for (int q = 0; q < 9; ++q) db[q / 3][q % 3] = R[R3_DB + q];
      FieldDerivs d;
      lds_derivs<B, true, true>(cur(), P, beta, d);
      const double wsym = (s == 0 || s == 3 || s == 5) ? 1.0 : 2.0;
      const double Sjk = Sjk_at(s);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        R[R3_GU + 3 * s + a] = d.d1[a];
        R[R3_SG + a] += wsym * Sjk * d.d1[a];
      }
      R[R3_RX + s] = -0.5 * contract_sym(gi, d.d2);
      const int i = SI(s), j = SJ(s);
      const double divb = db[0][0] + db[1][1] + db[2][2];
      double r = d.advko;
#pragma unroll
      for (int k = 0; k < 3; ++k) r += gt[S(i, k)] * db[k][j] + gt[S(j, k)] * db[k][i];
      r -= (2.0 / 3.0) * gt[s] * divb;
      r -= 2.0 * alpha * At[s];
      sink.put(F_GT + s, r, ep[0][0]);
    }
    if (s == 5 && active) {  // connection and the quadratic Ricci terms (pure algebra)
      COSMOS_PHASE();
      double gi[6], dgt[6][3], Gu[3][6], Gd[3], Ric[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        gi[q] = R[R3_GI + q];
        Ric[q] = R[R3_RX + q];
#pragma unroll
        for (int a = 0; a < 3; ++a) dgt[q][a] = R[R3_GU + 3 * q + a];
      }
      connection_and_quadratic_ricci(dgt, gi, Gu, Gd, Ric);
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        R[R3_RX + q] = Ric[q];
#pragma unroll
        for (int k = 0; k < 3; ++k) R[R3_GU + 6 * k + q] = Gu[k][q];
      }
    }
    advance(0);
  }

  // ---- connection functions
  double xs[kSrcLoads];  // the scalar field's sources at this point: E + S, S_j, S_ij
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    prefetch();
    if constexpr (SC != 0) {
      if (9 + k == kSrcPhase) {  // every thread of the wave issues them (inactive ones hold a valid point)
        xs[0] = xsrc(SRC_EPS);
#pragma unroll
        for (int j = 0; j < 3; ++j) xs[1 + j] = xsrc(SRC_S + j);
#pragma unroll
        for (int q = 0; q < 6; ++q) xs[4 + q] = xsrc(SRC_SIJ + q);
      }
    }
    if (active) {
      FieldDerivs d;
      lds_derivs<B, false, true>(cur(), P, beta, d);
      R[R3_RG + k] += d.advko;
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), j = SJ(s);
        R[R3_RX + s] += 0.5 * (gt[S(k, i)] * d.d1[j] + gt[S(k, j)] * d.d1[i]);
      }
    }
    advance(0);
  }

  // ---- conformal factor
  prefetch();
  if (active) {
    double gi[6], Gu[3][6], Ric[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      gi[q] = R[R3_GI + q];
      Ric[q] = R[R3_RX + q];
#pragma unroll
      for (int k = 0; k < 3; ++k) Gu[k][q] = R[R3_GU + 6 * k + q];
    }
    FieldDerivs d;
    lds_derivs<B, true, true>(cur(), P, beta, d);
    ricci_conformal_factor(ichi, d.d1, d.d2, gt, gi, Gu, Ric);
#pragma unroll
    for (int q = 0; q < 6; ++q) R[R3_RX + q] = Ric[q];
#pragma unroll
    for (int a = 0; a < 3; ++a) R[R3_DCHI + a] = d.d1[a];
    const double divb = R[R3_DB + 0] + R[R3_DB + 4] + R[R3_DB + 8];
    sink.put(F_CHI, d.advko + (2.0 / 3.0) * chi * (alpha * K - divb), ep[0][0]);
  }
  advance(0);

  // ---- lapse
  prefetch();
  if (active) {
    double gi[6], Gu[3][6], dchi[3];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      gi[q] = R[R3_GI + q];
#pragma unroll
      for (int k = 0; k < 3; ++k) Gu[k][q] = R[R3_GU + 6 * k + q];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) dchi[a] = R[R3_DCHI + a];
    FieldDerivs d;
    lds_derivs<B, true, true>(cur(), P, beta, d);
    const double* dal = d.d1;
    double cda = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) cda += gi[S(k, l)] * dchi[k] * dal[l];
    const double ih = 0.5 * ichi;
    double DDa[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      DDa[s] = (d.d2[s] - (Gu[0][s] * dal[0] + Gu[1][s] * dal[1] + Gu[2][s] * dal[2])) +
               ih * ((dchi[i] * dal[j] + dchi[j] * dal[i]) - gt[s] * cda);
    }
    R[R3_D2A] = chi * contract_sym(gi, DDa);
    const double Kbg = P.lapse_bg ? -3.0 * P.H0 / (1.0 + 2.0 * P.H0 * t) : 0.0;
    sink.put(F_ALP, d.advko - 2.0 * alpha * (K - Kbg), ep[0][0]);
    const double ix = R[R3_IX], pr = R[R3_P];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      double Sij = R[R3_S + SI(s)] * R[R3_S + SJ(s)] * ix + pr * gt[s] * ichi;
      if constexpr (SC != 0) Sij += xs[4 + s];
      R[R3_RX + s] = -DDa[s] + alpha * (R[R3_RX + s] - 8.0 * PI_D * Sij);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) R[R3_DAL + a] = dal[a];
  }
  advance(0);

  // ---- trace K, and the final Gt^i right-hand side. Amix = gt^kl At_lj and one third of
  // the trace gt^ij X_ij are kept for the At phases.
  double Amix[3][3], trX3 = 0.0;
  prefetch();
  if (active) {
    double gi[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) gi[q] = R[R3_GI + q];
    FieldDerivs d;
    lds_derivs<B, false, true>(cur(), P, beta, d);
    {
      double X[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) X[q] = R[R3_RX + q];
      trX3 = contract_sym(gi, X) * (1.0 / 3.0);
    }
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
    const double Str = (Sup[0] * R[R3_S + 0] + Sup[1] * R[R3_S + 1] + Sup[2] * R[R3_S + 2]) * R[R3_IX] + 3.0 * R[R3_P];
    double EpS = R[R3_E] + Str;
    if constexpr (SC != 0) EpS += xs[0];
    sink.put(F_K, d.advko + (-R[R3_D2A] + alpha * (AA + K * K * (1.0 / 3.0)) + 4.0 * PI_D * alpha * EpS), ep[0][0]);
    // Gt^i: every remaining term
    const double divb = R[R3_DB + 0] + R[R3_DB + 4] + R[R3_DB + 8];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double Gu[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) Gu[q] = R[R3_GU + 6 * i + q];
      double Gd[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double g[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) g[q] = R[R3_GU + 6 * k + q];
        Gd[k] = contract_sym(gi, g);
      }
      double r = R[R3_RG + i];
      r -= (4.0 / 3.0) * alpha * (gi[S(i, 0)] * d.d1[0] + gi[S(i, 1)] * d.d1[1] + gi[S(i, 2)] * d.d1[2]);
      r -= Gd[0] * R[R3_DB + 3 * i + 0] + Gd[1] * R[R3_DB + 3 * i + 1] + Gd[2] * R[R3_DB + 3 * i + 2];
      r += (2.0 / 3.0) * Gd[i] * divb;
      r -= 2.0 * (Aup[S(i, 0)] * R[R3_DAL + 0] + Aup[S(i, 1)] * R[R3_DAL + 1] + Aup[S(i, 2)] * R[R3_DAL + 2]);
      double inner = contract_sym(Gu, Aup);
      inner -= (1.5 * ichi) * (Aup[S(i, 0)] * R[R3_DCHI + 0] + Aup[S(i, 1)] * R[R3_DCHI + 1] + Aup[S(i, 2)] * R[R3_DCHI + 2]);
      r += 2.0 * alpha * inner;
      if constexpr (SC != 0) {
        double Sj[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) Sj[j] = R[R3_S + j] + xs[1 + j];
        r -= 16.0 * PI_D * alpha * (gi[S(i, 0)] * Sj[0] + gi[S(i, 1)] * Sj[1] + gi[S(i, 2)] * Sj[2]);
      } else {
        r -= 16.0 * PI_D * alpha * (gi[S(i, 0)] * R[R3_S + 0] + gi[S(i, 1)] * R[R3_S + 1] + gi[S(i, 2)] * R[R3_S + 2]);
      }
      sink.put(F_GAM + i, r, ep[0][1 + i]);
    }
  }
  advance(0);

  // ---- traceless extrinsic curvature. The flux-divergence loads of conserved
  // variable q (all three axes) are issued two phases before the phase that
  // completes its right-hand side (q = 0 in At phase 4, 1 in At phase 5, 2 in the
  // Et phase, 3 in the first St phase), so their latency overlaps the algebra.
  double fa[3][4], fb[3][4];
  constexpr bool kt = KT;  // divergence formed by the Kurganov-Tadmor pre-pass
  Nbr fnb;
  if (active) {
    const int i = c % P.n[0], jk = c / P.n[0], j = jk % P.n[1], k = jk / P.n[1];
    if (i >= 3 && i + 3 < P.n[0] && j >= 3 && j + 3 < P.n[1] && k >= 3 && k + 3 < P.n[2]) {
      // no wrap: uniform over the interior bricks, most of the grid
      const int sy = P.n[0], sz = P.n[0] * P.n[1];
      fnb.base = c;
#pragma unroll
      for (int o = -3; o <= 3; ++o) {
        fnb.d[0][o + 3] = o;
        fnb.d[1][o + 3] = o * sy;
        fnb.d[2][o + 3] = o * sz;
      }
    } else {
      make_nbr(fnb, i, j, k, P.n);
    }
  }
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    prefetch();
    if (active) {
      if (s == 4) flux_var_load(F, fs, c, fnb, 0, fa, kt);
      if (s == 5) flux_var_load(F, fs, c, fnb, 1, fb, kt);
      double db[3][3];
#pragma unroll
      for (int q = 0; q < 9; ++q) db[q / 3][q % 3] = R[R3_DB + q];
      const int i = SI(s), j = SJ(s);
      FieldDerivs d;
      lds_derivs<B, false, true>(cur(), P, beta, d);
      double r = d.advko;
#pragma unroll
      for (int k = 0; k < 3; ++k) r += At[S(i, k)] * db[k][j] + At[S(j, k)] * db[k][i];
      r -= (2.0 / 3.0) * At[s] * (db[0][0] + db[1][1] + db[2][2]);
      r += chi * (R[R3_RX + s] - gt[s] * trX3);
      double AAij = 0.0;  // At_ik gt^kl At_lj
#pragma unroll
      for (int k = 0; k < 3; ++k) AAij += At[S(i, k)] * Amix[k][j];
      r += alpha * (K * At[s] - 2.0 * AAij);
      sink.put(F_AT + s, r, ep[0][0]);
    }
    advance(0);
  }

  // ---- fluid: flux divergence (from the pre-pass), sources, dissipation (KO only
  // with the centred scheme: the Kurganov-Tadmor scheme carries its own)
  const double nbeta[3] = {0.0, 0.0, 0.0};
  const double im32 = 1.0 / (chi * sqrt(chi));
  double sgt = 0.0;  // S^jk gt_jk (formed in the Et phase, used by the St phases)
  prefetch();
  if (active) {
    const double div0 = flux_var_div(fa, P, kt);
    flux_var_load(F, fs, c, fnb, 2, fa, kt);
    double KS = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const double Sjk = Sjk_at(s), wS = (s == 0 || s == 3 || s == 5 ? 1.0 : 2.0) * Sjk;
      KS += wS * ((At[s] + gt[s] * K * (1.0 / 3.0)) * ichi);
      sgt += wS * gt[s];
    }
    FieldDerivs d;
    lds_derivs<B, false, false>(cur(), P, nbeta, d);
    const double Sda = Sup[0] * R[R3_DAL + 0] + Sup[1] * R[R3_DAL + 1] + Sup[2] * R[R3_DAL + 2];
    sink.put(F_ET, (kt ? 0.0 : d.advko) + (im32 * (alpha * KS - Sda) - div0), ep[0][0]);
  }
  advance(0);
  double cnext[NF];  // the next brick's point values, loaded during the St phases
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    prefetch();
    if (i == 0 && nx.valid) {
#pragma unroll
      for (int f = 0; f < NF; ++f) cnext[f] = bld(field_ptr(nx.U, f, nx.fs), (uint32_t)(nx.fs * 8), (uint32_t)nx.c * 8u);
    }
    if (active) {
      // St_0: q = 1 (loaded in At phase 5), then issue q = 3; St_1: q = 2; St_2: q = 3
      double divi;
      if (i == 0) {
        divi = flux_var_div(fb, P, kt);
        flux_var_load(F, fs, c, fnb, 3, fb, kt);
      } else {
        divi = flux_var_div(i == 1 ? fa : fb, P, kt);
      }
      FieldDerivs d;
      lds_derivs<B, false, false>(cur(), P, nbeta, d);
      double src = -R[R3_E] * R[R3_DAL + i] +
                   (R[R3_S + 0] * R[R3_DB + 0 + i] + R[R3_S + 1] * R[R3_DB + 3 + i] + R[R3_S + 2] * R[R3_DB + 6 + i]);
      src += 0.5 * alpha * (R[R3_SG + i] * ichi - sgt * R[R3_DCHI + i] * (ichi * ichi));
      sink.put(F_ST + i, (kt ? 0.0 : d.advko) + (im32 * src - divi), ep[0][0]);
    }
    if (i < 2) advance(0);
  }
  if (nx.valid) {  // hand over to the next brick: the halo ring already holds its first fields
#pragma unroll
    for (int f = 0; f < NF; ++f) cy.cen[f] = cnext[f];
#pragma unroll
    for (int q = 0; q < B::NOFF; ++q) hc.goffb[q] = nx.goffb[q];
#pragma unroll
    for (int d = 0; d < kEpiAhead; ++d)
#pragma unroll
      for (int k = 0; k < 4; ++k) ep[d][k] = ep[d + 1][k];
  }
}

}  // namespace cosmos
