// LDS-staged scalar-field stage: one 256-thread workgroup per 16x4x4 brick (one point per thread),
// two workgroups per CU. The 10 fields whose derivatives scalar_stage_point asks for (gt_ij, chi,
// alpha, phi, Pi) are staged one at a time, in that order, by LDS-direct loads of their halo
// boxes (HaloDma: the periodic wrap is in each lane's load offsets, and box points no stencil of
// the field reads load from a line the brick reads anyway) into a ring of 4 LDS buffers, 3 fields
// in flight, with one fence-free barrier per field. The point arithmetic is the direct kernel's
// (same function, same operation order), so both give the same values bitwise.
#pragma once
#include "bssn_lds.hpp"
#include "scalar_device.hpp"

namespace cosmos {

using ScBrick = DBrick<16, 4, 4>;
constexpr int kScRing = 4;               // LDS buffers: 4 x 20 KB, so two workgroups fit a CU
constexpr int kScAhead = kScRing - 1;    // fields in flight beyond the one being read
constexpr int kScFields = 10;            // gt_ij (6), chi, alpha, phi, Pi
// phi is differentiated twice (second and mixed derivatives: the offset set of its loads)
constexpr bool kScSecond[kScFields] = {false, false, false, false, false, false, false, false, true, false};

struct ScLds {
  const HaloDma<ScBrick>& hc;
  double* ring;
  const double* U;
  const double* Sc;
  size_t fs;
  uint32_t nbytes;
  int cidx;
  const DevParams& P;
  int phase;
  __device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }
  __device__ __forceinline__ const double* field(int q) const {
    return q < 6 ? U + (size_t)(F_GT + q) * fs
                 : (q == 6 ? U + (size_t)F_CHI * fs : (q == 7 ? U + (size_t)F_ALP * fs : Sc + (size_t)(q - 8) * fs));
  }
  // the first fields of a brick: 0 .. kScAhead - 1 issued, field 0 landed everywhere
  __device__ __forceinline__ void start() {
#pragma unroll
    for (int q = 0; q < kScAhead; ++q) hc.fetch(field(q), nbytes, ring + q * ScBrick::NP, kScSecond[q]);
    wait_vm((kScAhead - 1) * ScBrick::NR);
    lds_barrier();
  }
  // Call p (p = the field's place in the order) issues the loads of field p + 3 into the slot
  // field p - 1 used (every wave read it before the previous call's barrier), reads field p from
  // slot p % 4, then waits until field p + 1 has landed (the loads complete in issue order, so a
  // count of the newer ones suffices) and passes the barrier.
  template <bool SECOND, bool ADV, bool KO>
  __device__ __forceinline__ void get(int /*q: equals phase*/, const double beta[3], FieldDerivs& d) {
    if (phase + kScAhead < kScFields)
      hc.fetch(field(phase + kScAhead), nbytes, ring + ((phase + kScAhead) % kScRing) * ScBrick::NP,
               kScSecond[phase + kScAhead]);
    lds_derivs<ScBrick, SECOND, ADV, KO>(ring + (phase % kScRing) * ScBrick::NP + cidx, P, beta, d);
    // the results exist here, so the algebra that consumes them stays in this field's phase
#pragma unroll
    for (int a = 0; a < 3; ++a) asm volatile("" : "+v"(d.d1[a]));
    if constexpr (SECOND) {
#pragma unroll
      for (int s = 0; s < 6; ++s) asm volatile("" : "+v"(d.d2[s]));
    }
    if constexpr (ADV || KO) asm volatile("" : "+v"(d.advko));
    if (phase + 1 < kScFields) {
      const int newer = min(kScAhead - 1, kScFields - 2 - phase);  // fields issued after phase + 1
      wait_vm(newer * ScBrick::NR);
    }
    lds_barrier();
    ++phase;
  }
};

// T: 16x4x4 bricks. T.order 2: the XCD-blocked order (a persistent grid of the resident
// workgroups; each round, an XCD's workgroups take one compact block of bricks); else with
// T.xcd_order, slot w is brick (w mod 8) * T.per + w / 8, so each XCD walks its own slab of brick
// layers, and the workgroups stride over the slots. Needs n0 even and U, Sc 16-byte aligned
// (aligned pairs of x-neighbours).
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_scalar_stage_lds(
    const double* __restrict__ U, const double* __restrict__ Sc, double* __restrict__ src,
    const double* __restrict__ sun, double* __restrict__ sacc, double* __restrict__ sout, size_t fs, DevParams P,
    Tile T, double ca, double cn) {
  __shared__ double ring[kScRing * ScBrick::NP];
  const uint32_t nbytes = (uint32_t)(fs * 8);
  const int t = threadIdx.x;
  const int tx = t % 16, ty = (t / 16) % 4, tz = t / 64;
  const int cidx = (tx + ScBrick::XO) + ScBrick::SY * ((ty + 3) + ScBrick::HY * (tz + 3));
  HaloDma<ScBrick> hc;
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
    const int p = active ? i + P.n[0] * (j + P.n[1] * k) : 0;  // inactive threads evaluate point 0
    hc.init(i0, j0, k0, P.n);
    ScLds der{hc, ring, U, Sc, fs, nbytes, cidx, P, 0};
    der.start();
    scalar_stage_point<MODE>(U, Sc, src, sun, sacc, sout, fs, P, p, active, der, ca, cn);
  }
}

}  // namespace cosmos
