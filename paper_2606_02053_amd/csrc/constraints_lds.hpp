// LDS-staged constraint kernel: one 256-thread workgroup per 16x4x4 brick (one point per
// thread), two workgroups per CU (two waves per SIMD: one works while the other waits). The 17
// fields whose derivatives H and M_i need are staged one at a time, in the order
// constraint_point asks for them, by LDS-direct loads of their halo boxes (HaloDma: no
// registers hold the halo, the periodic wrap is in each lane's load offsets, and box points that
// no stencil of the field reads load from a line the brick reads anyway) into a ring of 4 LDS
// buffers, 3 fields in flight, with one fence-free barrier per field. The point arithmetic is
// that of the direct kernel (same function, same operation order), so the two variants give
// identical H and M_i; only the order of the norm sums follows the brick walk.
#pragma once
#include "bssn_lds.hpp"
#include "constraints_device.hpp"

namespace cosmos {

using ConsBrick = DBrick<16, 4, 4>;
constexpr int kConsRing = 4;                 // LDS buffers: 4 x 20 KB, so two workgroups fit a CU
constexpr int kConsAhead = kConsRing - 1;    // fields in flight beyond the one being read

// Fields in the order constraint_point requests their derivatives, and which of them it
// differentiates twice (the halo offset set of their loads).
constexpr int kConsFields = 17;
constexpr int kConsOrder[kConsFields] = {F_GT,  F_GT + 1,  F_GT + 2, F_GT + 3, F_GT + 4, F_GT + 5,
                                         F_CHI, F_GAM,     F_GAM + 1, F_GAM + 2, F_K,    F_AT,
                                         F_AT + 1, F_AT + 2, F_AT + 3, F_AT + 4, F_AT + 5};
constexpr bool kConsSecond[kConsFields] = {true,  true,  true,  true,  true,  true,  true,  false, false,
                                           false, false, false, false, false, false, false, false};

// Derivatives of the staged fields from the LDS ring; call order = kConsOrder. All threads of the
// workgroup take part. Call p issues the loads of field p + 3 into the slot field p - 1 used
// (free: every wave read it before the previous call's barrier), reads field p from slot p % 4,
// then waits until field p + 1 has landed (its own loads; the loads complete in issue order, so
// a count of the newer ones suffices) and passes the barrier.
struct LdsDerivs {
  const HaloDma<ConsBrick>& hc;
  double* ring;
  const double* U;
  size_t fs;
  uint32_t nbytes;
  int cidx;
  const DevParams& P;
  int phase;
  // an empty register constraint: the value must exist here, so the algebra that forms it
  // stays in this field's phase
  __device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }
  // the first fields of a brick: 0 .. kConsAhead - 1 issued, field 0 landed everywhere
  __device__ __forceinline__ void start() {
#pragma unroll
    for (int q = 0; q < kConsAhead; ++q)
      hc.fetch(field_ptr(U, kConsOrder[q], fs), nbytes, ring + q * ConsBrick::NP, kConsSecond[q]);
    wait_vm((kConsAhead - 1) * ConsBrick::NR);
    lds_barrier();
  }
  template <bool SECOND>
  __device__ __forceinline__ void get(int /*f: equals kConsOrder[phase]*/, FieldDerivs& d) {
    if (phase + kConsAhead < kConsFields)
      hc.fetch(field_ptr(U, kConsOrder[phase + kConsAhead], fs), nbytes,
               ring + ((phase + kConsAhead) % kConsRing) * ConsBrick::NP, kConsSecond[phase + kConsAhead]);
    const double nob[3] = {0.0, 0.0, 0.0};
    lds_derivs<ConsBrick, SECOND, false, false>(ring + (phase % kConsRing) * ConsBrick::NP + cidx, P, nob, d);
    // Pin the results in registers here: the point algebra that consumes them is pure
    // arithmetic, and without the pins the compiler moves it (and keeps every phase's
    // stencil taps live) past all the barriers to the end of the brick.
#pragma unroll
    for (int a = 0; a < 3; ++a) asm volatile("" : "+v"(d.d1[a]));
    if constexpr (SECOND) {
#pragma unroll
      for (int s = 0; s < 6; ++s) asm volatile("" : "+v"(d.d2[s]));
    }
    if (phase + 1 < kConsFields) {
      const int newer = min(kConsAhead - 1, kConsFields - 2 - phase);  // fields issued after phase + 1
      wait_vm(newer * ConsBrick::NR);
    }
    lds_barrier();
    ++phase;
  }
};

// T: 16x4x4 bricks. T.order 2: the XCD-blocked order (a persistent grid of the resident
// workgroups; each round, an XCD's workgroups take one compact block of bricks, whose halos
// overlap in its L2); else with T.xcd_order, workgroup w takes brick (w mod 8) * T.per + w / 8,
// so each XCD walks its own slab of brick layers (launched with one workgroup per brick);
// otherwise workgroups stride over the bricks in linear order. One partial record per workgroup
// (its bricks folded in walk order). Two waves per SIMD: 256 registers.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_constraints_lds(
    const double* __restrict__ U, size_t fs, DevParams P, Tile T, double* __restrict__ Hout,
    double* __restrict__ Mout, double* __restrict__ part) {
  __shared__ double ring[kConsRing * ConsBrick::NP];
  const uint32_t nbytes = (uint32_t)(fs * 8);
  const int t = threadIdx.x;
  const int tx = t % 16, ty = (t / 16) % 4, tz = t / 64;
  const int cidx = (tx + ConsBrick::XO) + ConsBrick::SY * ((ty + 3) + ConsBrick::HY * (tz + 3));
  Red mine = red_neutral();
  HaloDma<ConsBrick> hc;
  // T.order 2: round w of the XCD-blocked order; else brick slot w of the slab or linear order
  const bool blocked = T.order == 2;
  const int nslots = blocked ? T.ngroups : (T.xcd_order ? 8 * T.per : T.nbricks);
  const int first = blocked ? 0 : (int)blockIdx.x, stride = blocked ? 1 : (int)gridDim.x;
  for (int w = first; w < nslots; w += stride) {
    int bxi, byi, bzi;
    if (blocked) {
      if (!blocked_brick(T, w, blockIdx.x, bxi, byi, bzi)) continue;  // uniform over the workgroup
    } else {
      const int brick = T.xcd_order ? (w & 7) * T.per + (w >> 3) : w;
      if (brick >= T.nbricks) continue;  // uniform over the workgroup
      bxi = brick % T.nbx, byi = (brick / T.nbx) % T.nby, bzi = brick / T.nbx / T.nby;
    }
    const int i0 = bxi * 16, j0 = byi * 4, k0 = bzi * 4;
    const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
    const bool active = i < P.n[0] && j < P.n[1] && k < P.n[2];
    const int p = active ? i + P.n[0] * (j + P.n[1] * k) : 0;
    hc.init(i0, j0, k0, P.n);
    LdsDerivs der{hc, ring, U, fs, nbytes, cidx, P, 0};
    der.start();
    double H, M[3], Hn;
    bool bad;
    constraint_point(U, fs, p, der, P, H, M, Hn, bad);
    // The record is formed for every thread and selected: were it formed only under
    // `active`, the compiler would sink the whole point algebra past the barriers into
    // that branch and keep every phase's derivatives live until the end.
    const Red rec = point_record(U, fs, p, H, M, Hn, bad);
    if (active) store_hm(fs, p, H, M, Hout, Mout);
    mine = red_combine(mine, active ? rec : red_neutral());
  }
  // the ring is free now (every wave passed the last field's barrier): it holds the four wave results
  const Red r = block_tree(mine, reinterpret_cast<Red*>(ring));
  if (threadIdx.x == 0) red_store(part + (size_t)blockIdx.x * kRedRecord, r);
}

}  // namespace cosmos
