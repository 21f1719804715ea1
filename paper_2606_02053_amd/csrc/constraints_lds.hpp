// LDS-staged constraint kernel: one 256-thread workgroup per 16x4x4 brick (one
// point per thread). The 17 fields whose derivatives H and M_i need are copied,
// one at a time and in the order constraint_point asks for them, from HBM into
// LDS with the brick's periodic halo (the stage kernel's cooperative halo copy:
// coalesced loads, two fields in flight ahead in registers, two LDS buffers and
// one barrier per field), and each thread differentiates from LDS. The point
// arithmetic is that of the direct kernel (same function, same operation order),
// so the two variants give identical H and M_i; only the order of the norm sums
// follows the brick walk.
#pragma once
#include "bssn_lds.hpp"
#include "constraints_device.hpp"

namespace cosmos {

using ConsBrick = Brick<16, 4, 4>;
static_assert(kPrefetch == 2, "the first two fields are fetched into ring slots 0 and 1");

// Fields in the order constraint_point requests their derivatives.
constexpr int kConsFields = 17;
constexpr int kConsOrder[kConsFields] = {F_GT,  F_GT + 1,  F_GT + 2,  F_GT + 3, F_GT + 4, F_GT + 5,
                                         F_GAM, F_GAM + 1, F_GAM + 2, F_CHI,    F_K,      F_AT,
                                         F_AT + 1, F_AT + 2, F_AT + 3, F_AT + 4, F_AT + 5};

// Derivatives of the staged fields from the LDS halo box; call order = kConsOrder.
// All threads of the workgroup take part (each call holds one barrier). The two
// buffers alternate call by call across bricks (`odd`), so a buffer is rewritten one
// barrier after its last read; `phase` counts the calls within the brick.
struct LdsDerivs {
  HaloCopy<ConsBrick>& hc;
  double* buf0;
  double* buf1;
  const double* U;
  size_t fs;
  uint32_t nbytes;
  int cidx;
  const DevParams& P;
  bool& odd;
  int phase;
  // an empty register constraint: the value must exist here, so the algebra that forms it
  // stays in this field's phase
  __device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }
  template <bool SECOND>
  __device__ __forceinline__ void get(int /*f: equals kConsOrder[phase]*/, FieldDerivs& d) {
    double* buf = odd ? buf1 : buf0;
    hc.commit_and_rotate(buf);
    if (phase + kPrefetch < kConsFields)
      hc.template fetch<kPrefetch - 1>(field_ptr(U, kConsOrder[phase + kPrefetch], fs), nbytes);
    __syncthreads();
    const double nob[3] = {0.0, 0.0, 0.0};
    lds_derivs<ConsBrick, SECOND, false, false>(buf + cidx, P, nob, d);
    // Pin the results in registers here: the point algebra that consumes them is pure
    // arithmetic, and without the pins the compiler moves it (and keeps every phase's
    // stencil taps live) past all the barriers to the end of the brick.
#pragma unroll
    for (int a = 0; a < 3; ++a) asm volatile("" : "+v"(d.d1[a]));
    if constexpr (SECOND) {
#pragma unroll
      for (int s = 0; s < 6; ++s) asm volatile("" : "+v"(d.d2[s]));
    }
    odd = !odd;
    ++phase;
  }
};

// T: 16x4x4 bricks; with T.xcd_order, workgroup w takes brick (w mod 8) * T.per + w / 8,
// so each XCD walks its own slab of brick layers (launched with one workgroup per
// brick); otherwise workgroups stride over the bricks in linear order. One partial
// record per workgroup (its bricks folded in walk order). Two waves per SIMD (two
// workgroups per CU, so one works while the other waits at a field barrier): 256
// registers with about 100 spilled, faster than one wave per SIMD without spills.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_constraints_lds(
    const double* __restrict__ U, size_t fs, DevParams P, Tile T, double* __restrict__ Hout,
    double* __restrict__ Mout, double* __restrict__ part) {
  __shared__ double lds[ConsBrick::LDS_DOUBLES];
  __shared__ Red sh[4];
  double* buf0 = lds;
  double* buf1 = lds + ConsBrick::NP;
  const uint32_t nbytes = (uint32_t)(fs * 8);
  const int t = threadIdx.x;
  const int tx = t % 16, ty = (t / 16) % 4, tz = t / 64;
  const int cidx = (tz + 3) * ConsBrick::SZ + (ty + 3) * ConsBrick::SY + (tx + 3);
  const int nslots = T.xcd_order ? 8 * T.per : T.nbricks;
  Red mine = red_neutral();
  HaloCopy<ConsBrick> hc;
  bool odd = false;
  for (int w = blockIdx.x; w < nslots; w += gridDim.x) {
    const int brick = T.xcd_order ? (w & 7) * T.per + (w >> 3) : w;
    if (brick >= T.nbricks) continue;  // uniform over the workgroup
    const int i0 = (brick % T.nbx) * 16, j0 = ((brick / T.nbx) % T.nby) * 4, k0 = (brick / T.nbx / T.nby) * 4;
    const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
    const bool active = i < P.n[0] && j < P.n[1] && k < P.n[2];
    const int p = active ? i + P.n[0] * (j + P.n[1] * k) : 0;
    hc.init(i0, j0, k0, P.n);
    hc.template fetch<0>(field_ptr(U, kConsOrder[0], fs), nbytes);
    hc.template fetch<1>(field_ptr(U, kConsOrder[1], fs), nbytes);
    LdsDerivs der{hc, buf0, buf1, U, fs, nbytes, cidx, P, odd, 0};
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
  const Red r = block_tree(mine, sh);
  if (threadIdx.x == 0) red_store(part + (size_t)blockIdx.x * kRedRecord, r);
}

}  // namespace cosmos
