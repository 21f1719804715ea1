/*
 * cosmos.h -- C ABI of the MI355X (gfx950) library for the COSMOS evolution
 * hot path: the 3+1 Einstein equations in a BSSN (chi) form coupled to a
 * radiation fluid, on a periodic uniform Cartesian grid, in FP64.
 *
 * Paper passages the operations follow (the paper's sections; its displayed
 * equations are unnumbered):
 *   - "Physical system settings": Einstein equations G = 8 pi T with the
 *     perfect-fluid stress tensor T = (rho + P) u u + P g, linear equation of
 *     state P = w rho and the fluid equation of motion div T = 0, rewritten in
 *     the textbook 3+1 form; the initial-data paragraph (long-wavelength
 *     growing mode characterised by the curvature perturbation zeta(x), fluid
 *     distribution chosen so that the constraints hold, no elliptic solver);
 *   - "Statement of need" / "Examples": a box of size L.
 * The discretisation (4th-order centred differences, lopsided shift
 * advection, Kreiss-Oliger dissipation, periodic ghost zones of width 3,
 * classic RK4) is not fixed by the paper; see the per-function notes.
 *
 * Conventions shared by every entry point
 *   - State layout: 25 FP64 fields, structure of arrays, u[f][k][j][i] with
 *     i (x) fastest; field stride n0*n1*n2 values. Field order (enum
 *     cosmos_field): chi, gt_xx, gt_xy, gt_xz, gt_yy, gt_yz, gt_zz, K,
 *     At_xx..At_zz, Gt^x, Gt^y, Gt^z, alpha, beta^x, beta^y, beta^z,
 *     Et = chi^(-3/2) E, St_i = chi^(-3/2) S_i.
 *   - Grid: periodic, vertex centred, x_i = -L/2 + i*h with h = L/n per axis;
 *     point (n0/2, n1/2, n2/2) is the centre. n >= 8 on every axis.
 *   - Memory: every pointer argument named u, dudt, lam*, du0, norms_dev,
 *     H_out, M_out, ws or arena is DEVICE memory owned by the caller and must
 *     be 8-byte aligned (ws and arena 256-byte aligned). The library never
 *     allocates, frees or retains caller memory. Descriptor structs are HOST
 *     memory, read during the call only.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *     stream). Every call validates its arguments synchronously and returns a
 *     status; the work itself is enqueued asynchronously on `stream`.
 *   - Errors: a negative return value is a cosmos_status_code; the reason is
 *     available from cosmos_last_error() (thread local). Data-dependent
 *     failures found on the device (non-finite values, fluid-recovery
 *     failures, lapse collapse) are counted in the workspace and read with
 *     cosmos_status(), which synchronises the stream.
 *   - Threading: calls are re-entrant across host threads and streams as long
 *     as concurrent calls use distinct workspaces.
 */
#ifndef COSMOS_H
#define COSMOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COSMOS_NFIELDS 25
#define COSMOS_ABI_VERSION 1

enum cosmos_status_code {
  COSMOS_OK = 0,
  COSMOS_EINVAL = -1,      /* invalid argument (null/misaligned pointer, n < 8, L <= 0, dt <= 0, small workspace) */
  COSMOS_EHIP = -2,        /* a HIP runtime call failed */
  COSMOS_ENOMEM = -3,      /* size overflow */
  COSMOS_ENONFINITE = -4,  /* reserved: non-finite values are counted on the device (cosmos_status) */
  COSMOS_EPRIM = -5,       /* reserved: fluid-recovery failures are counted on the device (cosmos_status) */
  COSMOS_EUNSUPPORTED = -6 /* option not implemented (e.g. an unknown fluid scheme) */
};

enum cosmos_field {
  COSMOS_CHI = 0, COSMOS_GT = 1, COSMOS_TRK = 7, COSMOS_AT = 8, COSMOS_GAM = 14,
  COSMOS_ALPHA = 17, COSMOS_BETA = 18, COSMOS_ET = 21, COSMOS_ST = 22
};

/* Periodic box: n[a] points and length L[a] along axis a (x, y, z); 8 <= n[a] <= 2048 and
 * n[0] n[1] n[2] < 2^29 (the kernels address a field with 32-bit byte offsets). */
typedef struct {
  int32_t n[3];
  double L[3];
} cosmos_grid;

/* Evolution parameters.
 *   w        equation of state P = w rho ("Physical system settings"); 1/3 for radiation
 *   H0       Hubble rate of the background at t = 0 (units: lengths in 1/H0)
 *   eta      damping of the Gamma-driver shift condition
 *   ko_eps   Kreiss-Oliger dissipation strength (6th difference / 64 / h)
 *   lapse_bg 1: d_t alpha = beta.grad alpha - 2 alpha (K - K_bg(t)), K_bg = -3 H0 / (1 + 2 H0 t),
 *            which keeps alpha = 1 on the radiation background; 0: plain 1+log (K_bg = 0)
 *   evolve_shift 1: d_t beta^i = beta.grad beta^i + 3/4 Gt^i - eta beta^i; 0: shift frozen
 *   fluid_scheme 0: centred 4th-order flux divergence of the point fluxes, KO dissipation on every field;
 *            1: Kurganov-Tadmor central scheme ("Physical system settings" cites Kurganov & Tadmor 2000):
 *            conservation form with interface fluxes 1/2 (F(q_L) + F(q_R)) - 1/2 c (q_R - q_L), q_L, q_R
 *            minmod-limited linear reconstructions of (Et, St_i), the geometry averaged to the interface,
 *            c the largest characteristic speed of the two sides; no KO on the fluid fields. Supported by
 *            cosmos_rhs, cosmos_rk4_step(_stages), the batched form (cosmos_rk4_step_batched must then
 *            be given the fluid_scheme given to cosmos_batch_setup) and cosmos_constraints (which does
 *            not depend on it); the adjoint entry points return COSMOS_EUNSUPPORTED for it. Other
 *            values: COSMOS_EUNSUPPORTED
 *   variant  stage-kernel implementation: 0 = LDS-staged bricks (default; bricks 16x4x4, 16x8x2,
 *            8x8x4, 8x4x8), 1 = direct loads through the caches (any brick); same results
 *   alpha_collapse  a point with alpha below this value after a step counts as collapsed (0: off)
 *   tile_x, tile_y, tile_z  brick owned by one 256-thread workgroup of the stage kernel
 *            (tile_x * tile_y * tile_z must be 256; all 0 = default 16 x 4 x 4); results do not
 *            depend on the tile (bitwise), only the speed does
 *   tile_order brick order: 0 = XCD slabs (each of the 8 XCDs walks one contiguous slab of bricks),
 *            1 = linear, 2 = XCD-blocked (LDS-staged variant: each XCD owns a slab of brick layers and
 *            its resident workgroups process one compact block of bricks at a time, so shared halos
 *            are read into that XCD's L2 once; used where the brick grid splits evenly into such
 *            blocks -- brick layers a multiple of 8, blocks dividing each XCD's slab -- and linear
 *            otherwise; the direct variant treats 2 as linear) */
typedef struct {
  double w, H0, eta, ko_eps;
  int32_t lapse_bg, evolve_shift, fluid_scheme, variant;
  double alpha_collapse;
  int32_t tile_x, tile_y, tile_z, tile_order;
} cosmos_params;

/* Initial data (paper: "Physical system settings", initial-data paragraph).
 * zeta profile: 0 = Gaussian mu exp(-r^2 / 2 sigma^2) about `center`, 1 = single mode
 * mu sin(2 pi x / L_x), 2 = Gaussian in s_a = (L_a / pi) sin(pi x_a / L_a) (smooth, periodic).
 * density_mode: 0 = energy density from the Hamiltonian constraint, E = (R + 2/3 K^2) / 16 pi;
 *               1 = uniform E = 3 H0^2 / 8 pi (constraint violating; for experiments).
 * noise_amp A > 0 multiplies E by (1 + A xi_p), xi_p uniform in [-1, 1) from the counter-based
 * SplitMix64 generator (Steele, Lea & Flood 2014): xi_p = 2 (SM64(seed, p) >> 11) 2^-53 - 1,
 * SM64(seed, p) = the (p+1)-th output of SplitMix64 started at `seed`, p = i + n0 (j + n1 k). */
typedef struct {
  double mu, sigma, center[3], noise_amp;
  uint64_t seed;
  int32_t profile, density_mode;
} cosmos_init;

/* Bytes of device workspace needed by cosmos_rhs / cosmos_rk4_step / cosmos_constraints on this
 * grid: the status counters, the reduction partials, 3 state-sized RK4 buffers and two arrays of
 * 12 * N3 doubles for the fluid fluxes of a stage state (the point fluxes; with fluid_scheme 1
 * the first 4 * N3 hold the Kurganov-Tadmor flux divergence). A stage forms them in a pre-pass,
 * except where the previous stage's kernel wrote them into the other array beside its new state
 * (the LDS-staged 16x4x4 kernel of the centred scheme does). Returns 0 for an invalid grid. */
size_t cosmos_workspace_bytes(const cosmos_grid* grid);

/* Zero the status counters held in the workspace (asynchronous). */
int cosmos_status_reset(void* ws, void* stream);

/* Synchronise `stream` and copy the status counters to host out[4]:
 * out[0] points with a non-finite value seen after an RK4 step or in cosmos_constraints,
 * out[1] fluid-recovery failures (E <= 0 or negative discriminant; the recovery then uses
 *        P = 0, v = 0, respectively a clamped discriminant), out[2] points with
 *        alpha < alpha_collapse after a step, out[3] RK4 steps taken since the last reset. */
int cosmos_status(void* ws, void* stream, int64_t out[4]);

/* Initial data: fills u (25 * N3 values) with the leading-order long-wavelength growing mode of
 * a curvature perturbation zeta on the radiation FLRW background: chi = e^{-2 zeta}, gt = delta,
 * K = -3 H0, At = 0, Gt = 0, alpha = 1, beta = 0, fluid at rest, E from the Hamiltonian
 * constraint (no elliptic solve), Et = chi^(-3/2) E. */
int cosmos_init_fields(const cosmos_grid* grid, const cosmos_params* params, const cosmos_init* init,
                       double* u, void* stream);

/* d u0 / d theta for theta = mu (which = 0) or sigma (which = 1): derivative of the initial
 * data above with respect to the perturbation amplitude or width (du0: 25 * N3 values). */
int cosmos_init_tangent(const cosmos_grid* grid, const cosmos_params* params, const cosmos_init* init,
                        int which, double* du0, void* stream);

/* Discrete right-hand side du/dt at time t (dudt: 25 * N3 values, must not alias u):
 * BSSN chi-form evolution equations with 1+log lapse and Gamma-driver shift, perfect-fluid
 * sources and conservative fluid equations (Et, St_i) with a centred flux divergence (or the
 * Kurganov-Tadmor fluxes, fluid_scheme 1), all derivatives by 4th-order centred differences,
 * shift advection beta^k d_k by lopsided radius-3 stencils chosen by the sign of beta^k, plus
 * Kreiss-Oliger dissipation on every evolved field (on the geometric fields only with
 * fluid_scheme 1); periodic ghost zones of width 3. ws is used for the status counters. */
int cosmos_rhs(const cosmos_grid* grid, const cosmos_params* params, double t, const double* u,
               double* dudt, void* ws, void* stream);

/* Kurganov-Tadmor flux divergence of the fluid alone (the pre-pass of every stage with
 * fluid_scheme 1; "Physical system settings" names Kurganov & Tadmor 2000 for the fluid):
 * div[q * N3 + p] = sum_a (Fh^a_q(p + 1/2) - Fh^a_q(p - 1/2)) / h_a for q = Et, St_x, St_y, St_z,
 * Fh the numerical interface flux described under fluid_scheme above (params.fluid_scheme itself
 * is not consulted). u: 25 * N3 device values; div: 4 * N3 device values owned by the caller,
 * not overlapping u. Asynchronous on `stream`; no workspace. Errors: COSMOS_EINVAL for an invalid
 * grid, NULL, misaligned or overlapping pointers. */
int cosmos_kt_divergence(const cosmos_grid* grid, const cosmos_params* params, const double* u, double* div,
                         void* stream);

/* ---- Massless scalar field ("Physical system settings": the second matter field, stress tensor
 * d phi d phi - 1/2 g (d phi)^2 and wave equation box phi = 0; "Spherically symmetric
 * iso-curvature" example for its initial data). The field lives in a separate state s of
 * 2 * N3 doubles (phi, then Pi = n^mu d_mu phi, each x fastest), caller-owned device memory. Its
 * evolution: d_t phi = alpha Pi + beta.grad phi, d_t Pi = beta.grad Pi + alpha K Pi + alpha D^i D_i phi
 * + D^i alpha D_i phi, with KO dissipation on both; its energy E = (Pi^2 + |D phi|^2) / 2, momentum
 * S_i = -Pi d_i phi and stress S_ij = d_i phi d_j phi - gamma_ij (|D phi|^2 - Pi^2) / 2 join the fluid's
 * in the K, At and Gt equations and in the constraints (the fluid equations are unchanged).
 * sws: device workspace of cosmos_scalar_workspace_bytes(grid) bytes, 256-byte aligned (the
 * 11 source arrays and the scalar's RK4 buffers), used besides ws. With variant 0 the stage kernel
 * runs the 16x4x4 brick only (other bricks: COSMOS_EUNSUPPORTED); fluid_scheme 0 and 1 are both
 * supported; the batched form carries the field too (cosmos_rk4_step_batched_scalar), the adjoint
 * does not. The status counters do not look at s (cosmos_constraints_scalar flags non-finite
 * scalar energies). */
size_t cosmos_scalar_workspace_bytes(const cosmos_grid* grid);

/* cosmos_init_fields with an iso-curvature mode Upsilon = sc_mu * profile(x; sc_sigma) of the scalar
 * field (the same profile family and centre as zeta): phi = Upsilon, Pi = 0, and with density_mode 0
 * the fluid energy is the Hamiltonian constraint's remainder, E = (R + 2/3 K^2) / 16 pi -
 * chi |grad Upsilon|^2 / 2 (leading order: the field does not enter the background metric). sc_mu = 0
 * gives exactly cosmos_init_fields and s = 0. Errors: COSMOS_EINVAL (invalid init, sc_sigma <= 0, s
 * overlapping u). */
int cosmos_init_fields_scalar(const cosmos_grid* grid, const cosmos_params* params, const cosmos_init* init,
                              double sc_mu, double sc_sigma, double* u, double* s, void* stream);

/* Right-hand side of (u, s) at time t: dudt (25 * N3) and dsdt (2 * N3); neither may overlap u, s or
 * the other. */
int cosmos_rhs_scalar(const cosmos_grid* grid, const cosmos_params* params, double t, const double* u,
                      const double* s, double* dudt, double* dsdt, void* ws, void* sws, void* stream);

/* One classic RK4 step of (u, s) in place (both advance together). */
int cosmos_rk4_step_scalar(const cosmos_grid* grid, const cosmos_params* params, double t, double dt, double* u,
                           double* s, void* ws, void* sws, void* stream);

/* nsteps (>= 0) RK4 steps of (u, s) in one call: the same states bitwise as nsteps calls of
 * cosmos_rk4_step_scalar at t, t + dt, t + dt + dt, ..., the fluid fluxes carried from step to
 * step as in cosmos_rk4_steps. COSMOS_EINVAL for nsteps < 0. */
int cosmos_rk4_steps_scalar(const cosmos_grid* grid, const cosmos_params* params, double t, double dt, int32_t nsteps,
                            double* u, double* s, void* ws, void* sws, void* stream);

/* cosmos_constraints with the scalar field's energy and momentum in H and M_i. */
int cosmos_constraints_scalar(const cosmos_grid* grid, const cosmos_params* params, const double* u, const double* s,
                              double* norms_dev, double* H_out, double* M_out, void* ws, void* sws, void* stream);

/* One classic RK4 step of size dt from time t, in place on u:
 * u <- u + dt/6 (k1 + 2 k2 + 2 k3 + k4). The stage update is fused into the right-hand-side
 * kernels (k is never stored): 4 launches, 3 state-sized buffers in ws. */
int cosmos_rk4_step(const cosmos_grid* grid, const cosmos_params* params, double t, double dt,
                    double* u, void* ws, void* stream);

/* nsteps (>= 0) RK4 steps of size dt from time t, in place on u: the same u bitwise as nsteps calls
 * of cosmos_rk4_step at t, t + dt, t + dt + dt, ... (the time advanced by repeated addition).
 * Within the call the last stage of a step also writes the fluid fluxes of the new u for the next
 * step (the LDS-staged 16x4x4 kernel of the centred scheme; others run the pre-pass), which a
 * step of its own cannot do: its caller may change u before the next call. Errors as
 * cosmos_rk4_step, and COSMOS_EINVAL for nsteps < 0. */
int cosmos_rk4_steps(const cosmos_grid* grid, const cosmos_params* params, double t, double dt, int32_t nsteps,
                     double* u, void* ws, void* stream);

/* One RK4 step as cosmos_rk4_step (bitwise the same u), keeping the stage states for a reverse
 * sweep: stages (device, caller-owned, 3 * 25 * N3 doubles, must not overlap u or ws) receives
 * U2, U3, U4 in that order, each in the state layout, where U_{s+1} = u_n + c_s dt k_s
 * (c = 1/2, 1/2, 1) is the state the next stage's right-hand side is evaluated at. */
int cosmos_rk4_step_stages(const cosmos_grid* grid, const cosmos_params* params, double t, double dt,
                           double* u, double* stages, void* ws, void* stream);

/* One RK4 step as cosmos_rk4_step_stages, out of place: u (read only) keeps u_n and u_next
 * (device, caller-owned, 25 * N3 doubles) receives u_{n+1}, bitwise the state
 * cosmos_rk4_step_stages leaves in u; stages receives U2, U3, U4 as there. For drivers that need
 * the step's start state afterwards (the refined layers' interpolation in time below; the paper's
 * fixed mesh refinement, "Statement of need"): alternating two state arrays saves a copy of u.
 * u, u_next, stages and ws must not overlap (COSMOS_EINVAL); other errors as cosmos_rk4_step. */
int cosmos_rk4_step_stages_to(const cosmos_grid* grid, const cosmos_params* params, double t, double dt,
                              const double* u, double* u_next, double* stages, void* ws, void* stream);

/* nsteps (>= 0) RK4 steps as cosmos_rk4_steps (the same u bitwise as single steps at t, t + dt,
 * t + dt + dt, ...), keeping the whole trajectory for a reverse sweep: states (nsteps * 25 * N3
 * doubles) receives the start state of step m at offset m * 25 * N3, stages (nsteps * 3 * 25 * N3
 * doubles) the stage states of step m at offset m * 3 * 25 * N3, as cosmos_rk4_step_stages writes
 * them. Device, caller-owned; states, stages, u and ws must not overlap (COSMOS_EINVAL). */
int cosmos_rk4_steps_stages(const cosmos_grid* grid, const cosmos_params* params, double t, double dt,
                            int32_t nsteps, double* u, double* states, double* stages, void* ws, void* stream);

/* Hamiltonian and momentum constraints of u and their grid norms:
 *   H   = R + 2/3 K^2 - At_ij At^ij - 16 pi E
 *   M_i = gt^jk (d_j At_ki - Gt^l_jk At_li - Gt^l_ji At_kl) - 3/(2 chi) At^j_i d_j chi - 2/3 d_i K - 8 pi S_i
 * norms_dev[8] (device) = { sqrt(mean H^2), max |H|, sqrt(mean |M|^2), max |M|,
 *   sqrt(mean Hn^2) with Hn = H / (|R| + 2/3 K^2 + At.At + 16 pi |E|) (0 where that is 0),
 *   number of points with a non-finite state value, H or M, min alpha, argmin alpha (lowest
 *   linear index among ties) }. H_out (N3) and M_out (3 * N3, component-major) are optional
 *   (NULL to skip). The reduction is deterministic (fixed order, no floating-point atomics). */
int cosmos_constraints(const cosmos_grid* grid, const cosmos_params* params, const double* u,
                       double* norms_dev, double* H_out, double* M_out, void* ws, void* stream);

/* cosmos_constraints without a workspace, for callers that cannot allocate device memory (code
 * under graph capture, monitoring loops and harnesses that forbid allocation). Same arguments and
 * results as cosmos_constraints (the LDS-staged kernel, or the direct one on grids with odd n0 or u
 * not 16-byte aligned, as there; params->variant is not consulted), minus ws: the per-workgroup reduction partials go to a fixed device array inside the library,
 * 4096 records of 8 doubles (256 KiB) per GPU, held from the first call on that GPU until the
 * process ends. At most 4096 workgroups are launched and they stride over the grid's bricks, so
 * every grid the library accepts fits; grids beyond its limits (8 <= n <= 2048, n0 n1 n2 < 2^29)
 * are rejected with COSMOS_EINVAL as by every entry point. Every launched workgroup writes its own
 * record before the fold reads it, so no state carries over from one call to the next. All calls
 * on one GPU share the array: calls that overlap in time on one GPU (different streams or host
 * threads without ordering) race and give wrong norms. The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine). Errors: as cosmos_constraints; COSMOS_EHIP if the
 * array's device address cannot be obtained, COSMOS_EUNSUPPORTED on a device index above 63. */
int cosmos_constraints_noalloc(const cosmos_grid* grid, const cosmos_params* params, const double* u,
                               double* norms_dev, double* H_out, double* M_out, void* stream);

/* Bytes of device workspace for cosmos_rhs_vjp / cosmos_adjoint_step: status counters, the
 * recomputed stage states U2..U4 and the stage accumulator, two state-sized cotangent buffers and
 * 136 * N3 doubles of per-point cotangent scratch. 0 for an invalid grid. */
size_t cosmos_adjoint_workspace_bytes(const cosmos_grid* grid);

/* Transposed Jacobian of the discrete right-hand side at state u and time t applied to kbar:
 * ubar = (d rhs / d u)^T kbar (all three 25 * N3 values; ubar must not alias the others).
 * The upwind branches are frozen at the forward choice (sign of beta^a at each point). */
int cosmos_rhs_vjp(const cosmos_grid* grid, const cosmos_params* params, double t, const double* u,
                   const double* kbar, double* ubar, void* ws, void* stream);

/* Discrete adjoint of one RK4 step of cosmos_rk4_step: lam_n = (d u_{n+1} / d u_n)^T lam_np1 at
 * state u_n, time t, step dt. The stage states are recomputed from u_n; then, with
 * kb4 = dt/6 lam', ub_s = J_f(U_s)^T kb_s, kb3 = dt/3 lam' + dt ub4, kb2 = dt/3 lam' + dt/2 ub3,
 * kb1 = dt/6 lam' + dt/2 ub2:  lam_n = lam' + ub1 + ub2 + ub3 + ub4. ws: at least
 * cosmos_adjoint_workspace_bytes. lam_n must not alias u_n or lam_np1. */
int cosmos_adjoint_step(const cosmos_grid* grid, const cosmos_params* params, double t, double dt,
                        const double* u_n, const double* lam_np1, double* lam_n, void* ws, void* stream);

/* cosmos_adjoint_step with the step's stage states supplied instead of recomputed: stages holds
 * U2, U3, U4 as cosmos_rk4_step_stages wrote them when stepping from u_n (same params and dt).
 * Same lam_n bitwise, three stage launches fewer. stages must not overlap lam_n or ws. */
int cosmos_adjoint_step_stages(const cosmos_grid* grid, const cosmos_params* params, double t, double dt,
                               const double* u_n, const double* stages, const double* lam_np1, double* lam_n,
                               void* ws, void* stream);

/* Gradient of an objective J(u_0) with respect to the initial-data parameters theta = (mu, sigma)
 * of cosmos_init, given its adjoint lam0 = dJ/du_0 (25 * N3 device values, e.g. the result of the
 * reverse sweep of cosmos_adjoint_step down to step 0): the last step of the discrete adjoint,
 * dJ/dtheta_w = < lam0, d u_0 / d theta_w > = sum over points and fields of lam0 times the tangent of
 * cosmos_init_fields that cosmos_init_tangent(which = w) writes. The tangent is formed at each point
 * and contracted at once (never stored); the sums use a fixed order (a butterfly within each
 * wavefront, then workgroup partials folded in workgroup order), so the result is bitwise
 * reproducible. grad_dev: 2 device doubles (dJ/dmu, dJ/dsigma). ws: an adjoint workspace
 * (cosmos_adjoint_workspace_bytes); its contents are overwritten. Errors: COSMOS_EINVAL (invalid
 * grid or init, NULL or misaligned pointers, lam0 overlapping ws). */
int cosmos_adjoint_gradient(const cosmos_grid* grid, const cosmos_params* params, const cosmos_init* init,
                            const double* lam0, double* grad_dev, void* ws, void* stream);

/* Batched form: many independent runs advanced together, one persistent launch per RK4 stage
 * for all of them (work items = (run, brick)). Run r has a cubic periodic grid of n[r]^3
 * points (n[r] divisible by 16) and box L[r]; its state (25 * n[r]^3 doubles, layout as above)
 * starts at arena + state_off[r] (state_off[r] a multiple of 32). All runs share the params; their
 * tile fields choose the brick (0 = 16x4x4; 16x8x2, 8x8x4, 8x4x8; the Kurganov-Tadmor scheme and
 * the scalar field run 16x4x4 only; the order field is not used) and the results do not depend on
 * it (bitwise). Host arrays, read during the call only. */
typedef struct {
  int32_t nruns;
  const int32_t* n;
  const double* L;
  const int64_t* state_off;
} cosmos_batch;

/* Bytes of batch workspace: descriptor table, work list, per-run status counters and three
 * stage buffers matching the arena layout. 0 for an invalid batch. */
size_t cosmos_batch_workspace_bytes(const cosmos_batch* batch);

/* Upload the per-run descriptor table and the interleaved (run, brick) work list into bws and
 * zero the per-run status counters. Synchronises `stream`. Call once per batch (not inside a
 * graph capture). Errors: COSMOS_EINVAL for an invalid batch or brick, COSMOS_EUNSUPPORTED for a
 * brick other than 16x4x4 with fluid_scheme 1. */
int cosmos_batch_setup(const cosmos_batch* batch, const cosmos_params* params, void* bws, void* stream);

/* One classic RK4 step of every run: run r advances by dt_dev[r] from time t_dev[r]; t_dev is
 * advanced on the device (t_dev, dt_dev: device arrays of nruns doubles). Enqueues 4 stage
 * launches and one time update and nothing else, so it can be captured in a hipGraph and
 * replayed; the results equal those of cosmos_rk4_step on each run with the same brick. The
 * runs' parameters are those given to cosmos_batch_setup; params->fluid_scheme and the tile
 * fields select the kernels and must be the ones given there. */
int cosmos_rk4_step_batched(const cosmos_batch* batch, const cosmos_params* params, double* arena,
                            double* t_dev, const double* dt_dev, void* bws, void* stream);

/* nsteps (>= 1) batched steps in one call, graph-capturable as one step is: every run ends in the
 * same state bitwise as after nsteps calls of cosmos_rk4_step_batched. Within the call the last
 * stage of a step also writes the fluid fluxes of the new states for the next step (the 16x4x4
 * brick of the centred scheme; other bricks and schemes run the pre-pass every step). Errors as
 * cosmos_rk4_step_batched, and COSMOS_EINVAL for nsteps < 1. */
int cosmos_rk4_steps_batched(const cosmos_batch* batch, const cosmos_params* params, double* arena, double* t_dev,
                             const double* dt_dev, int32_t nsteps, void* bws, void* stream);

/* Bytes of the batch's scalar-field workspace (256-byte aligned device memory, used besides bws by
 * cosmos_rk4_step_batched_scalar): the field's RK4 buffers and source arrays of every run, laid out
 * like the state arena. 0 for an invalid batch. */
size_t cosmos_batch_scalar_workspace_bytes(const cosmos_batch* batch);

/* cosmos_rk4_step_batched with the massless scalar field (see cosmos_rk4_step_scalar) in every run:
 * sarena is laid out like the state arena, run r's (phi, Pi) (2 n^3 doubles) at sarena +
 * state_off[r]; both advance together; sbws holds cosmos_batch_scalar_workspace_bytes(batch)
 * bytes. Each run equals cosmos_rk4_step_scalar on its grid with a 16x4x4 brick. */
int cosmos_rk4_step_batched_scalar(const cosmos_batch* batch, const cosmos_params* params, double* arena,
                                   double* sarena, double* t_dev, const double* dt_dev, void* bws, void* sbws,
                                   void* stream);

/* Per-run outcome of a scan, on the device: out_dev[2 r] = alpha at run r's centre point
 * (n/2, n/2, n/2), out_dev[2 r + 1] = the minimum of alpha over run r's grid (order independent, so
 * exact and reproducible). arena: the batch's state arena; bws: the workspace given to
 * cosmos_batch_setup (its descriptor table); out_dev: 2 * nruns device doubles. Asynchronous. */
int cosmos_batch_outcomes(const cosmos_batch* batch, const double* arena, void* bws, double* out_dev, void* stream);

/* Synchronise and copy the per-run counters to host out[nruns][4] (as cosmos_status). */
int cosmos_batch_status(const cosmos_batch* batch, void* bws, void* stream, int64_t* out);

/* ---------------------------------------------------------------- fixed mesh refinement
 * Nested refinement layers ("Statement of need": the code resolves collapse with fixed mesh
 * refinement; the adiabatic-fluctuation example shows the lowest, 1st and 2nd layers). The paper
 * leaves the scheme to its references; this library's is Berger-Oliger sub-cycling with buffer
 * zones:
 *   - a layer ("child") refines a box of its parent ("parent": the periodic grid, or a child
 *     itself) by 2 per axis, vertex-aligned: the child's interior point i (per axis,
 *     0 <= i < 2 m) lies at parent index origin + i / 2;
 *   - the child's state is a 25-field SoA array on its padded grid (cosmos_fmr_child_grid:
 *     n = 2 m + 2 COSMOS_FMR_BUFFER per axis, spacing half the parent's) and is advanced with
 *     cosmos_rk4_step on that grid as if periodic: what the wrap-around spoils reaches at most 3
 *     points further inwards per RK4 stage, so the outer COSMOS_FMR_BUFFER layers go stale within
 *     a step and the interior stays exact;
 *   - per parent step dt the child takes two steps dt/2; before each, cosmos_fmr_prolong refills
 *     the buffer from the parent (6-point Lagrange in space; in time the continuous extension of
 *     the parent's RK4 step from its stage states), and after both cosmos_fmr_restrict copies the
 *     child's interior onto the parent points it covers.
 * The driver (paper_2606_02053_amd/fmr.py) sequences these calls; every value is computed here. */
#define COSMOS_FMR_BUFFER 12

typedef struct cosmos_box {
  int32_t origin[3]; /* parent array index (x, y, z) of the child's interior point 0; any integer:
                        indices wrap periodically on the parent */
  int32_t m[3];      /* parent cells covered per axis (>= 4); the child interior has 2 m points */
} cosmos_box;

/* The child's padded grid: n[a] = 2 m[a] + 2 COSMOS_FMR_BUFFER, L[a] = n[a] * h_parent[a] / 2.
 * Errors: COSMOS_EINVAL for an invalid parent grid or box, or a child beyond the grid limits. */
int cosmos_fmr_child_grid(const cosmos_grid* parent, const cosmos_box* box, cosmos_grid* child);

/* Device bytes of the workspace cosmos_fmr_prolong needs for this parent and box (its two
 * partially interpolated intermediates); 0 for invalid arguments. */
size_t cosmos_fmr_workspace_bytes(const cosmos_grid* parent, const cosmos_box* box);

/* Child values interpolated from the parent. The parent's values in time: theta == 0 takes u_n
 * (stages and u_np1 may be NULL); 0 < theta <= 1 takes the continuous extension of the parent's
 * RK4 step from u_n to u_np1 at t_n + theta dt, u_n + dt sum_i b_i(theta) k_i with
 * b = (theta - 3/2 theta^2 + 2/3 theta^3, theta^2 - 2/3 theta^3 (twice), -1/2 theta^2 + 2/3 theta^3),
 * the slopes k_i recovered from the step's stage states (stages: U2, U3, U4 as
 * cosmos_rk4_step_stages or cosmos_rk4_step_stages_to keeps them, 3 x 25 x N3(parent) doubles);
 * at theta = 1/2 this is
 * (2 U2 + 2 U3 + U4 - u_np1) / 4. In space, per axis: a child point that coincides with a parent
 * point copies it, a midpoint takes (3, -25, 150, 150, -25, 3)/256 of the 6 parent points around
 * it (exact for quintics), applied along x, then y, then z. buffer_only != 0 writes only the child
 * points within COSMOS_FMR_BUFFER of a face; 0 writes the whole padded child (initial data).
 * Parent arrays: device, 25 x N3(parent) doubles each; child_u: device, 25 x N3(child) doubles,
 * not overlapping them; ws: cosmos_fmr_workspace_bytes, 256-byte aligned. Asynchronous on
 * `stream`. Errors: COSMOS_EINVAL (invalid grid/box/pointers, theta outside [0, 1], theta > 0
 * without stages or u_np1). */
int cosmos_fmr_prolong(const cosmos_grid* parent, const cosmos_box* box, const double* u_n, const double* stages,
                       const double* u_np1, double theta, int32_t buffer_only, double* child_u, void* ws,
                       void* stream);

/* Injection: parent points origin + j (0 <= j < m per axis, wrapped) take the child's values at
 * its interior points 2 j (padded index COSMOS_FMR_BUFFER + 2 j). child_u and parent_u: device,
 * 25-field SoA on their grids, not overlapping. Asynchronous. Errors: COSMOS_EINVAL. */
int cosmos_fmr_restrict(const cosmos_grid* parent, const cosmos_box* box, const double* child_u, double* parent_u,
                        void* stream);

/* Human-readable reason for the last error on this thread ("" if none). */
const char* cosmos_last_error(void);

/* COSMOS_ABI_VERSION of the loaded library. */
int cosmos_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* COSMOS_H */
