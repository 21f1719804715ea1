// libcosmos: C ABI and gfx950 kernels of the COSMOS evolution hot path.
// The ABI (argument meaning, layout, ownership, errors) is documented in
// include/cosmos.h; the physics and stencils in bssn_device.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>
#include <mutex>

#include "cosmos.h"
#include "bssn_device.hpp"
#include "init_device.hpp"
#include "constraints_device.hpp"
#include "bssn_lds.hpp"
#include "constraints_lds.hpp"
#include "kt_device.hpp"
#include "scalar_device.hpp"
#include "scalar_lds.hpp"
#include "adjoint_point.hpp"

using namespace cosmos;

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

static int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return set_error(COSMOS_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- workspace layout
// [status: 8 x int64 | reduction partials | acc | stage A | stage B | fluid fluxes (12 fields)]
namespace {
constexpr size_t kAlign = 256;
constexpr int kBlock = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t status, partials, acc, A, B, F, F2, total;
};
constexpr int kFluxFields = 12;  // F^a_q, a = axis, q = (Et, St_x, St_y, St_z)

bool grid_ok(const cosmos_grid* g) {
  if (!g) return false;
  for (int a = 0; a < 3; ++a)
    if (g->n[a] < 8 || g->n[a] > 2048 || !(g->L[a] > 0.0) || !std::isfinite(g->L[a])) return false;
  // per-field byte offsets are 32-bit in the kernels (8 * n0 n1 n2 < 2^32); 4 RK4 states of
  // that size are 430 GB, beyond one GPU's HBM anyway
  return (int64_t)g->n[0] * g->n[1] * g->n[2] < (int64_t)1 << 29;
}

size_t npts(const cosmos_grid* g) { return (size_t)g->n[0] * g->n[1] * g->n[2]; }
size_t nblocks(const cosmos_grid* g) { return (npts(g) + kBlock - 1) / kBlock; }

Layout layout(const cosmos_grid* g) {
  Layout L;
  const size_t state = (size_t)NF * npts(g) * sizeof(double);
  L.status = 0;
  L.partials = align_up(8 * sizeof(int64_t));
  L.acc = align_up(L.partials + nblocks(g) * kRedRecord * sizeof(double));
  L.A = align_up(L.acc + state);
  L.B = align_up(L.A + state);
  L.F = align_up(L.B + state);
  L.F2 = align_up(L.F + (size_t)kFluxFields * npts(g) * sizeof(double));  // the next stage's fluxes
  L.total = align_up(L.F2 + (size_t)kFluxFields * npts(g) * sizeof(double));
  return L;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int check_common(const cosmos_grid* g, const cosmos_params* p) {
  if (!grid_ok(g)) return set_error(COSMOS_EINVAL, "invalid grid (need 8 <= n <= 2048, L > 0, n0*n1*n2 < 2^29)");
  if (!p) return set_error(COSMOS_EINVAL, "params is NULL");
  if (!std::isfinite(p->w) || !std::isfinite(p->H0) || !std::isfinite(p->eta) || !std::isfinite(p->ko_eps) ||
      !(p->w > 0.0))
    return set_error(COSMOS_EINVAL, "invalid params (w must be > 0; all values finite)");
  if (p->fluid_scheme != 0 && p->fluid_scheme != 1)
    return set_error(COSMOS_EUNSUPPORTED, "fluid_scheme %d not implemented (0: centred, 1: Kurganov-Tadmor)",
                     p->fluid_scheme);
  if (p->variant != 0 && p->variant != 1) return set_error(COSMOS_EINVAL, "variant must be 0 (LDS-staged) or 1 (direct)");
  return COSMOS_OK;
}

// Entry points whose kernels implement the centred fluid scheme only (the batched
// form and the adjoint).
int check_centred(const cosmos_params* p, const char* what) {
  if (p->fluid_scheme != 0) return set_error(COSMOS_EUNSUPPORTED, "%s supports fluid_scheme 0 only", what);
  return COSMOS_OK;
}

int check_state(const void* ptr, const char* name) {
  if (!ptr) return set_error(COSMOS_EINVAL, "%s is NULL", name);
  if (!aligned(ptr, 8)) return set_error(COSMOS_EINVAL, "%s is not 8-byte aligned", name);
  return COSMOS_OK;
}

int check_ws(const cosmos_grid* g, const void* ws) {
  if (!ws) return set_error(COSMOS_EINVAL, "workspace is NULL");
  if (!aligned(ws, kAlign)) return set_error(COSMOS_EINVAL, "workspace is not 256-byte aligned");
  return COSMOS_OK;
}

// Brick shape from the params (0 = default 16 x 4 x 4, XCD-ordered).
int make_tile(const cosmos_grid* g, const cosmos_params* p, Tile& T) {
  T.bx = p->tile_x ? p->tile_x : 16;
  T.by = p->tile_y ? p->tile_y : 4;
  T.bz = p->tile_z ? p->tile_z : 4;
  T.order = p->tile_order;
  T.xcd_order = p->tile_order == 0 ? 1 : 0;  // the direct variant treats order 2 as linear
  if (T.bx < 1 || T.by < 1 || T.bz < 1 || T.bx * T.by * T.bz != kBlock || T.order < 0 || T.order > 2)
    return set_error(COSMOS_EINVAL,
                     "tile %dx%dx%d (order %d) invalid: need tile_x*tile_y*tile_z == %d, order 0, 1 or 2", T.bx, T.by,
                     T.bz, p->tile_order, kBlock);
  T.gx = T.gy = T.gz = T.zr = T.ngx = T.ngy = T.ngroups = 0;  // set at launch for order 2
  T.nbx = (g->n[0] + T.bx - 1) / T.bx;
  T.nby = (g->n[1] + T.by - 1) / T.by;
  T.nbz = (g->n[2] + T.bz - 1) / T.bz;
  T.nbricks = T.nbx * T.nby * T.nbz;
  T.per = (T.nbricks + 7) / 8;
  return COSMOS_OK;
}

unsigned tile_blocks(const Tile& T) { return T.xcd_order ? 8u * (unsigned)T.per : (unsigned)T.nbricks; }

DevParams dev_params(const cosmos_grid* g, const cosmos_params* p) {
  DevParams d;
  d.w = p->w;
  d.H0 = p->H0;
  d.eta = p->eta;
  d.ko_eps = p->ko_eps;
  d.alpha_collapse = p->alpha_collapse;
  d.lapse_bg = p->lapse_bg;
  d.evolve_shift = p->evolve_shift;
  double h[3];
  for (int a = 0; a < 3; ++a) {
    d.n[a] = g->n[a];
    h[a] = g->L[a] / g->n[a];
    d.i12h[a] = 1.0 / (12.0 * h[a]);
    d.i12h2[a] = 1.0 / (12.0 * h[a] * h[a]);
    d.iko[a] = p->ko_eps / (64.0 * h[a]);
    d.i24h[a] = 1.0 / (24.0 * h[a]);
    d.ih[a] = 1.0 / h[a];
  }
  d.fluid_scheme = p->fluid_scheme;
  d.xsrc = nullptr;
  d.i144[0] = 1.0 / (144.0 * h[0] * h[1]);
  d.i144[1] = 1.0 / (144.0 * h[0] * h[2]);
  d.i144[2] = 1.0 / (144.0 * h[1] * h[2]);
  return d;
}
}  // namespace

#include "stage.hip.inc"

namespace {
// The two flux arrays of an RK4 step: a stage reads `cur`; where its kernel also writes the next
// stage's fluxes (into `nxt`), the two swap and the next stage skips its pre-pass. The last stage
// of a step writes them only when `chain` is set: for the next step of the same call, whose u
// nobody else can have changed in between.
struct FluxPair {
  double* cur;
  double* nxt;
  bool ready = false;
  bool chain = false;
  int stage(const cosmos_params* p, const Tile& T, hipStream_t s, const double* U, const double* un, double* acc,
            double* out, size_t fs, const DevParams& P, double t, double ca, double cn, int mode,
            unsigned long long* status) {
    bool wrote = false;
    const int rc = launch_stage(p, T, s, U, cur, un, acc, out, fs, P, t, ca, cn, mode, status,
                                (mode == 1 || mode == 2 || (mode == 3 && chain)) ? nxt : nullptr, ready, &wrote);
    if (wrote) std::swap(cur, nxt);
    ready = wrote;
    return rc;
  }
};
}  // namespace

namespace {
// One RK4 step in place on u; the stage states go to U2, U3, U4 (U4 may be U2: it is
// written after U2 has been read for the last time). carry: the flux arrays carried from one step
// of a call to the next (see FluxPair); nullptr: a step of its own.
int rk4_step(const cosmos_grid* grid, const cosmos_params* params, double t, double dt, double* u, double* U2,
             double* U3, double* U4, void* ws, void* stream, FluxPair* carry = nullptr, double* unew = nullptr) {
  const Layout L = layout(grid);
  char* w = (char*)ws;
  double* acc = (double*)(w + L.acc);
  double* F = (double*)(w + L.F);
  auto* status = (unsigned long long*)(w + L.status);
  const DevParams P = dev_params(grid, params);
  Tile T;
  int rc;
  if ((rc = make_tile(grid, params, T))) return rc;
  const size_t fs = npts(grid);
  hipStream_t s = (hipStream_t)stream;
  FluxPair own{F, (double*)(w + L.F2)};
  FluxPair& fx = carry ? *carry : own;
  if ((rc = fx.stage(params, T, s, u, u, acc, U2, fs, P, t, dt / 6.0, dt / 2.0, 1, status))) return rc;
  fx.stage(params, T, s, U2, u, acc, U3, fs, P, t + dt / 2.0, dt / 3.0, dt / 2.0, 2, status);
  fx.stage(params, T, s, U3, u, acc, U4, fs, P, t + dt / 2.0, dt / 3.0, dt, 2, status);
  // the last stage writes u_{n+1} over u, or into unew (u itself then keeps u_n)
  fx.stage(params, T, s, U4, nullptr, acc, unew ? unew : u, fs, P, t + dt, dt / 6.0, 0.0, 3, status);
  HIP_TRY(hipGetLastError());
  return COSMOS_OK;
}

}  // namespace

// ---------------------------------------------------------------- ABI
extern "C" {

int cosmos_abi_version(void) { return COSMOS_ABI_VERSION; }

const char* cosmos_last_error(void) { return g_last_error.c_str(); }

size_t cosmos_workspace_bytes(const cosmos_grid* grid) {
  if (!grid_ok(grid)) return 0;
  return layout(grid).total;
}

int cosmos_status_reset(void* ws, void* stream) {
  if (!ws || !aligned(ws, kAlign)) return set_error(COSMOS_EINVAL, "invalid workspace");
  HIP_TRY(hipMemsetAsync(ws, 0, 8 * sizeof(int64_t), (hipStream_t)stream));
  return COSMOS_OK;
}

int cosmos_status(void* ws, void* stream, int64_t out[4]) {
  if (!ws || !aligned(ws, kAlign) || !out) return set_error(COSMOS_EINVAL, "invalid workspace or output");
  int64_t h[8];
  HIP_TRY(hipMemcpyAsync(h, ws, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  for (int q = 0; q < 4; ++q) out[q] = h[q];
  return COSMOS_OK;
}

int cosmos_init_fields(const cosmos_grid* grid, const cosmos_params* params, const cosmos_init* init, double* u,
                       void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u"))) return rc;
  if (!init) return set_error(COSMOS_EINVAL, "init is NULL");
  if (!(init->sigma > 0.0) || init->profile < 0 || init->profile > 2 || init->density_mode < 0 ||
      init->density_mode > 1)
    return set_error(COSMOS_EINVAL, "invalid init (sigma > 0, profile 0..2, density_mode 0..1)");
  InitArgs a = make_init_args(grid, params, init);
  hipLaunchKernelGGL(k_init, dim3(nblocks(grid)), dim3(kBlock), 0, (hipStream_t)stream, a, u, -1, nullptr);
  HIP_TRY(hipGetLastError());
  return COSMOS_OK;
}

int cosmos_init_tangent(const cosmos_grid* grid, const cosmos_params* params, const cosmos_init* init, int which,
                        double* du0, void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(du0, "du0"))) return rc;
  if (!init || which < 0 || which > 1) return set_error(COSMOS_EINVAL, "init is NULL or which not in {0, 1}");
  if (!(init->sigma > 0.0) || init->profile < 0 || init->profile > 2 || init->density_mode < 0 ||
      init->density_mode > 1)
    return set_error(COSMOS_EINVAL, "invalid init (sigma > 0, profile 0..2, density_mode 0..1)");
  InitArgs a = make_init_args(grid, params, init);
  hipLaunchKernelGGL(k_init, dim3(nblocks(grid)), dim3(kBlock), 0, (hipStream_t)stream, a, du0, which, nullptr);
  HIP_TRY(hipGetLastError());
  return COSMOS_OK;
}

int cosmos_rhs(const cosmos_grid* grid, const cosmos_params* params, double t, const double* u, double* dudt,
               void* ws, void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u")) || (rc = check_state(dudt, "dudt")) ||
      (rc = check_ws(grid, ws)))
    return rc;
  if (u == dudt) return set_error(COSMOS_EINVAL, "dudt must not alias u");
  if (!std::isfinite(t)) return set_error(COSMOS_EINVAL, "t is not finite");
  const DevParams P = dev_params(grid, params);
  Tile T;
  if ((rc = make_tile(grid, params, T))) return rc;
  auto* status = (unsigned long long*)ws;
  double* F = (double*)((char*)ws + layout(grid).F);
  if ((rc = launch_stage(params, T, (hipStream_t)stream, u, F, nullptr, nullptr, dudt, npts(grid), P, t, 0.0, 0.0, 0,
                         status)))
    return rc;
  HIP_TRY(hipGetLastError());
  return COSMOS_OK;
}


int cosmos_kt_divergence(const cosmos_grid* grid, const cosmos_params* params, const double* u, double* div,
                         void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u")) || (rc = check_state(div, "div"))) return rc;
  const size_t N = npts(grid);
  if (div < u + (size_t)NF * N && u < div + 4 * N) return set_error(COSMOS_EINVAL, "div must not overlap u");
  const DevParams P = dev_params(grid, params);
  hipLaunchKernelGGL(k_fluid_kt, dim3(kt_bricks(P)), dim3(kKtThreads), 0, (hipStream_t)stream, u, N, P, div);
  HIP_TRY(hipGetLastError());
  return COSMOS_OK;
}

int cosmos_rk4_step(const cosmos_grid* grid, const cosmos_params* params, double t, double dt, double* u, void* ws,
                    void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u")) || (rc = check_ws(grid, ws))) return rc;
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t)) return set_error(COSMOS_EINVAL, "dt must be > 0, t finite");
  const Layout L = layout(grid);
  double* A = (double*)((char*)ws + L.A);
  double* B = (double*)((char*)ws + L.B);
  return rk4_step(grid, params, t, dt, u, A, B, A, ws, stream);
}

int cosmos_rk4_steps(const cosmos_grid* grid, const cosmos_params* params, double t, double dt, int32_t nsteps,
                     double* u, void* ws, void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u")) || (rc = check_ws(grid, ws))) return rc;
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t)) return set_error(COSMOS_EINVAL, "dt must be > 0, t finite");
  if (nsteps < 0) return set_error(COSMOS_EINVAL, "nsteps %d < 0", (int)nsteps);
  const Layout L = layout(grid);
  char* w = (char*)ws;
  double* A = (double*)(w + L.A);
  double* B = (double*)(w + L.B);
  FluxPair fx{(double*)(w + L.F), (double*)(w + L.F2)};
  double tm = t;
  for (int32_t m = 0; m < nsteps; ++m) {
    fx.chain = m + 1 < nsteps;
    if ((rc = rk4_step(grid, params, tm, dt, u, A, B, A, ws, stream, &fx))) return rc;
    tm += dt;  // as a caller stepping one call at a time would advance it
  }
  return COSMOS_OK;
}

int cosmos_rk4_step_stages(const cosmos_grid* grid, const cosmos_params* params, double t, double dt, double* u,
                           double* stages, void* ws, void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u")) || (rc = check_state(stages, "stages")) ||
      (rc = check_ws(grid, ws)))
    return rc;
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t)) return set_error(COSMOS_EINVAL, "dt must be > 0, t finite");
  const size_t n = (size_t)NF * npts(grid);
  const char *a = (const char*)stages, *a1 = a + 3 * n * sizeof(double);
  const char *b = (const char*)u, *b1 = b + n * sizeof(double);
  const char *c = (const char*)ws, *c1 = c + cosmos_workspace_bytes(grid);
  if ((a < b1 && b < a1) || (a < c1 && c < a1)) return set_error(COSMOS_EINVAL, "stages overlaps u or ws");
  return rk4_step(grid, params, t, dt, u, stages, stages + n, stages + 2 * n, ws, stream);
}

int cosmos_rk4_step_stages_to(const cosmos_grid* grid, const cosmos_params* params, double t, double dt,
                              const double* u, double* u_next, double* stages, void* ws, void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u")) || (rc = check_state(u_next, "u_next")) ||
      (rc = check_state(stages, "stages")) || (rc = check_ws(grid, ws)))
    return rc;
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t)) return set_error(COSMOS_EINVAL, "dt must be > 0, t finite");
  const size_t n = (size_t)NF * npts(grid);
  const char *ua = (const char*)u, *ub = ua + n * sizeof(double);
  const char *va = (const char*)u_next, *vb = va + n * sizeof(double);
  const char *ga = (const char*)stages, *gb = ga + 3 * n * sizeof(double);
  const char *wa = (const char*)ws, *wb = wa + cosmos_workspace_bytes(grid);
  auto apart = [](const char* a0, const char* a1, const char* b0, const char* b1) { return a1 <= b0 || b1 <= a0; };
  if (!apart(ua, ub, va, vb) || !apart(ua, ub, ga, gb) || !apart(ua, ub, wa, wb) || !apart(va, vb, ga, gb) ||
      !apart(va, vb, wa, wb) || !apart(ga, gb, wa, wb))
    return set_error(COSMOS_EINVAL, "u, u_next, stages and ws must not overlap");
  // u is only read: every stage takes it as u_n, and the last one writes u_next
  double* U = const_cast<double*>(u);
  return rk4_step(grid, params, t, dt, U, stages, stages + n, stages + 2 * n, ws, stream, nullptr, u_next);
}

int cosmos_rk4_steps_stages(const cosmos_grid* grid, const cosmos_params* params, double t, double dt,
                            int32_t nsteps, double* u, double* states, double* stages, void* ws, void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u")) || (rc = check_state(states, "states")) ||
      (rc = check_state(stages, "stages")) || (rc = check_ws(grid, ws)))
    return rc;
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t)) return set_error(COSMOS_EINVAL, "dt must be > 0, t finite");
  if (nsteps < 0) return set_error(COSMOS_EINVAL, "nsteps %d < 0", (int)nsteps);
  const size_t n = (size_t)NF * npts(grid);
  const char *ua = (const char*)u, *ub = ua + n * sizeof(double);
  const char *wa = (const char*)ws, *wb = wa + cosmos_workspace_bytes(grid);
  const char *sa = (const char*)states, *sb = sa + (size_t)nsteps * n * sizeof(double);
  const char *ga = (const char*)stages, *gb = ga + (size_t)nsteps * 3 * n * sizeof(double);
  auto apart = [](const char* a0, const char* a1, const char* b0, const char* b1) { return a1 <= b0 || b1 <= a0; };
  if (!apart(sa, sb, ua, ub) || !apart(sa, sb, wa, wb) || !apart(ga, gb, ua, ub) || !apart(ga, gb, wa, wb) ||
      !apart(sa, sb, ga, gb))
    return set_error(COSMOS_EINVAL, "states, stages, u and ws must not overlap");
  const Layout L = layout(grid);
  char* w = (char*)ws;
  FluxPair fx{(double*)(w + L.F), (double*)(w + L.F2)};
  hipStream_t s = (hipStream_t)stream;
  double tm = t;
  for (int32_t m = 0; m < nsteps; ++m) {
    HIP_TRY(hipMemcpyAsync(states + (size_t)m * n, u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    double* st = stages + (size_t)m * 3 * n;
    fx.chain = m + 1 < nsteps;
    if ((rc = rk4_step(grid, params, tm, dt, u, st, st + n, st + 2 * n, ws, stream, &fx))) return rc;
    tm += dt;
  }
  return COSMOS_OK;
}

}  // extern "C"

namespace {

// Constraint norms of u: the LDS-staged kernel (variant 0 with n0 even; 16x4x4 bricks, a
// persistent grid in the XCD-blocked order where the resident workgroups split evenly into blocks
// and fit the `cap` partial records at `part`, else XCD slabs, workgroups striding over the
// bricks when there are more than `cap`) or the direct one (variant 1, and grids with odd n0: one workgroup per
// 256 points, or at most `cap` of them striding over the blocks), then the fixed-order fold of
// the per-workgroup partials.
void launch_constraints(const cosmos_grid* grid, const cosmos_params* params, const DevParams& P, const double* u,
                        double* H_out, double* M_out, double* part, size_t cap, double* norms_dev, hipStream_t s) {
  const size_t nb = std::min(nblocks(grid), cap);
  unsigned nparts = (unsigned)nb;
  // the LDS-staged kernel loads aligned pairs of x-neighbours: n0 even, u 16-byte aligned
  if (params->variant == 0 && grid->n[0] % 2 == 0 && aligned(u, 16)) {
    cosmos_params bp{};
    bp.tile_x = 16, bp.tile_y = 4, bp.tile_z = 4, bp.tile_order = 0;
    Tile T;
    make_tile(grid, &bp, T);
    // the XCD-blocked order where the resident workgroups split evenly into blocks (a persistent
    // grid of G workgroups, so G partial records); else one workgroup per brick in XCD slabs
    const unsigned G = resident_groups(k_constraints_lds);
    if (G <= nb && T.nbricks >= (int)G && blocked_order(T, G / 8)) {
      T.order = 2;
      nparts = G;
    } else {
      if (tile_blocks(T) > nb) T.xcd_order = 0;
      nparts = (unsigned)std::min<size_t>(T.xcd_order ? tile_blocks(T) : (size_t)T.nbricks, nb);
    }
    hipLaunchKernelGGL(k_constraints_lds, dim3(nparts), dim3(kBlock), 0, s, u, npts(grid), P, T, H_out, M_out, part);
  } else {
    hipLaunchKernelGGL(k_constraints, dim3(nparts), dim3(kBlock), 0, s, u, npts(grid), P, H_out, M_out, part);
  }
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, s, part, (int)nparts, npts(grid), norms_dev);
}

}  // namespace

extern "C" {

int cosmos_constraints(const cosmos_grid* grid, const cosmos_params* params, const double* u, double* norms_dev,
                       double* H_out, double* M_out, void* ws, void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u")) || (rc = check_state(norms_dev, "norms_dev")) ||
      (rc = check_ws(grid, ws)))
    return rc;
  if ((H_out && !aligned(H_out, 8)) || (M_out && !aligned(M_out, 8)))
    return set_error(COSMOS_EINVAL, "H_out / M_out not 8-byte aligned");
  const Layout L = layout(grid);
  double* part = (double*)((char*)ws + L.partials);
  const DevParams P = dev_params(grid, params);
  launch_constraints(grid, params, P, u, H_out, M_out, part, nblocks(grid), norms_dev, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return COSMOS_OK;
}

}  // extern "C"

#include "batch.hip.inc"
#include "adjoint.hip.inc"
#include "scalar.hip.inc"
#include "fmr.hip.inc"

// ---------------------------------------------------------------- allocation-free constraint norms
// For callers that cannot allocate (code under graph capture, tight monitoring loops): the
// constraint norms with the reduction partials in a fixed device array instead of a workspace.
namespace {
constexpr int kNoAllocParts = 4096;  // partial records of the array: 4096 x 8 doubles = 256 KiB
constexpr int kMaxDevices = 64;
}  // namespace

// One copy per GPU the library runs on, held until the process ends. Host code must not use
// this name as a device address: it takes the address that hipGetSymbolAddress returns.
static __device__ __align__(256) double scratch[kNoAllocParts * kRedRecord];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up on the first call on that device.
int scratch_for_current_device(double** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(COSMOS_EUNSUPPORTED, "device %d: the allocation-free entry points serve devices 0..%d", dev,
                     kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(COSMOS_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_dev[dev] = (double*)ptr;
  }
  *out = g_scratch_dev[dev];
  return COSMOS_OK;
}
}  // namespace

extern "C" {

int cosmos_constraints_noalloc(const cosmos_grid* grid, const cosmos_params* params, const double* u,
                               double* norms_dev, double* H_out, double* M_out, void* stream) {
  int rc;
  if ((rc = check_common(grid, params)) || (rc = check_state(u, "u")) || (rc = check_state(norms_dev, "norms_dev")))
    return rc;
  if ((H_out && !aligned(H_out, 8)) || (M_out && !aligned(M_out, 8)))
    return set_error(COSMOS_EINVAL, "H_out / M_out not 8-byte aligned");
  double* part = nullptr;
  if ((rc = scratch_for_current_device(&part))) return rc;
  // At most kNoAllocParts workgroups: the LDS-staged kernel's workgroups stride over the
  // bricks, so every grid the library accepts fits; each launched workgroup writes its record
  // and the fold reads exactly those, so nothing in the array needs clearing between calls.
  cosmos_params p = *params;
  p.variant = 0;
  const DevParams P = dev_params(grid, &p);
  launch_constraints(grid, &p, P, u, H_out, M_out, part, (size_t)kNoAllocParts, norms_dev, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return COSMOS_OK;
}

}  // extern "C"
