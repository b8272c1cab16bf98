/*
 * tclbm.h -- C ABI of the MI355X (gfx950) thermal cascaded lattice Boltzmann
 * library libtclbm.so.
 *
 * The library advances the two D2Q9 distribution functions of the thermal
 * cascaded lattice Boltzmann method of Fei & Luo (arXiv:1610.07114): the
 * density DF f, relaxed by the cascaded (central-moment) collision with
 * central-moment forcing (Sections 2-3) and the third-moment correction term
 * C (Section 4), and the total-energy DF h, relaxed towards its equilibrium
 * with the coupling source K (Section 4) -- or, for the Rayleigh-Benard runs
 * of Section 5D, an internal-energy DF (tclbm_params.energy_df).  Both are
 * pull-streamed.  Every step is one fused HIP kernel launch on the handle's
 * stream.
 *
 * Conventions
 *   - Lattice units: R*T0 must be 1/3 (c_s^2); the default R = 1/3, T0 = 1.
 *   - Host fields are float64 arrays of nx*ny values, index y*nx + x.
 *   - D2Q9 order (Section 2): 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
 *   - No C++ types or exceptions cross this interface.  Every function returns
 *     a tclbm_status (or a size / string); nothing aborts the process.
 *   - A handle may be used from one host thread at a time.  Work is enqueued
 *     on the stream given at creation; functions that return host data
 *     (tclbm_moments, tclbm_step_timed) synchronise that stream.
 *
 * Ownership
 *   - dev_buf passed to tclbm_create is caller-owned device memory (for
 *     example a torch tensor's storage) of at least tclbm_state_bytes() bytes;
 *     the library borrows it until tclbm_destroy and never frees it.
 *   - The stream is borrowed.  Host arrays are read (copied) during the call.
 *   - The handle owns a small device buffer for macroscopic output fields,
 *     allocated on the first tclbm_moments call that asks for fields.
 */
#ifndef TCLBM_H
#define TCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tclbm_ctx *tclbm_handle;

typedef enum {
  TCLBM_OK = 0,
  TCLBM_E_INVALID = 1,  /* bad argument or parameter; nothing was changed   */
  TCLBM_E_NOMEM = 2,    /* dev_bytes too small or an internal allocation failed */
  TCLBM_E_DEVICE = 3,   /* a HIP runtime call failed (message: tclbm_last_error) */
  TCLBM_E_STATE = 4,    /* handle unusable (failed create or earlier instability) */
  TCLBM_E_UNSTABLE = 5  /* non-finite or non-positive density/temperature found */
} tclbm_status;

/* Storage of f and h in device memory.  Arithmetic is FP32 for the first
 * three and FP64 for the last.  Every form stores each population as its
 * deviation from a per-row rest-state equilibrium (fixed at create time from
 * the row means of the initial density and temperature), and the arithmetic
 * runs on those deviations.  F16_DEV keeps the deviation times 2^10 as an
 * IEEE half: deviations from 6.0e-8 up to 64 are normal numbers; a larger one
 * overflows and is reported as unstable.  BF16_DEV keeps the deviation as a
 * bfloat16.  Both 16-bit forms round stochastically and without bias: random
 * bits below the target's last place are added to the FP32 value, which is
 * then truncated.  The bits come from a counter-based generator keyed by
 * (lattice step, node, population), so results are deterministic and do not
 * depend on the launch shape or on the other members of a batch.  (Rounding
 * to nearest would freeze a stored value whose change per step is below half
 * a unit in the last place.) */
typedef enum {
  TCLBM_STORE_F32 = 0,
  TCLBM_STORE_F16_DEV = 1,
  TCLBM_STORE_BF16_DEV = 2,
  TCLBM_STORE_F64 = 3
} tclbm_storage;

typedef enum { TCLBM_XLO = 0, TCLBM_XHI = 1, TCLBM_YLO = 2, TCLBM_YHI = 3 } tclbm_side;

/* Boundary kinds.  PERIODIC must be set on both sides of an axis or neither.
 * BOUNCEBACK: halfway bounce-back at rest (adiabatic for h), any side.
 * WALL: node wall on the boundary row (y sides only) imposing (ux_w, uy_w, T_w)
 * by non-equilibrium extrapolation of both DFs from the adjacent fluid node.
 * WALL_ADIABATIC: as WALL for the velocity; the wall temperature is the one
 * that makes the one-sided second-order normal derivative vanish,
 * T_w = (4 T_1 - T_2)/3 from the nodes one and two rows inside (the fixed
 * lower plate of the Couette test of Section 5B); needs ny >= 4. */
typedef enum {
  TCLBM_BC_PERIODIC = 0,
  TCLBM_BC_BOUNCEBACK = 1,
  TCLBM_BC_WALL = 2,
  TCLBM_BC_WALL_ADIABATIC = 3
} tclbm_bc_kind;

typedef struct {
  int32_t nx, ny;        /* lattice size, each >= 3; nx * ny <= 2^28 and
                            ceil(nx / w) * 64 * ny * planes < 2^32, where
                            w = 62 with periodic x, 61 otherwise (each x
                            tile of w columns owns a 64-slot block per row)
                            and planes = 18, or 9 when athermal (offsets
                            within a state buffer are 32-bit): up to about
                            230 M nodes */
  double R, T0;          /* gas constant and reference temperature, R*T0 = 1/3 */
  double gamma, Pr;      /* specific-heat ratio (> 1) and Prandtl number (> 0) */
  double tau_f;          /* 1/w1 (> 0.5): mu = p (tau_f - 1/2), Eq. (29) */
  double w2, w3, w4;     /* bulk, third- and fourth-order rates, in (0, 2) */
  double ax, ay;         /* uniform body acceleration (force density rho a) */
  int32_t thermal;       /* 1: TCLBM; 0: athermal cascaded LBM (T = T0, no h) */
  int32_t correction;    /* 1: include the correction term C_a (Section 4) */
  int32_t storage;       /* tclbm_storage */
  int32_t wall_rho;      /* wall-node density: 0 from the populations that reached
                            the wall node (default), 1 the fluid neighbour's,
                            2 the fluid neighbour's pressure plus rho a.n */
  int32_t heq_moments;   /* h^eq moments beyond second order: 0 continuous
                            Maxwellian values (default), 1 raw zero (Section 4's
                            explicit form) */
  int32_t h_collision;   /* energy DF update: 0 two-rate (energy flux at w_h,
                            other moments at 1; default), 1 BGK (Section 4) */
  int32_t h_force;       /* energy DF body-force source: 1 (default) adds the
                            change of the equilibrium energy flux (rho E + p) u
                            that the force makes within a step, first moment
                            (rho E + p) a with the (1 - w_h/2) factor; 0 none
                            (Section 4 as printed) */
  int32_t accel_field;   /* 1: tclbm_create receives per-node acceleration
                            arrays (space for them is part of the state) */
  int32_t bc[4];         /* tclbm_bc_kind per side (tclbm_side order); the
                            initial state is built for these boundaries */
  double wall_ux[4], wall_uy[4], wall_T[4];  /* WALL sides: imposed u and T */
  int32_t viscosity_mode; /* 0: w1 = 1/tau_f everywhere (default); 1: dynamic
                             viscosity mu = mu0 T/T0 (Section 5B): Eq. (29)
                             with p = rho R T gives, per node,
                             1/w1 = mu0/(rho R T0) + 1/2, and w_h, tau_hf follow
                             from that w1 at constant Pr (tau_f is then unused) */
  double mu0;             /* reference dynamic viscosity (> 0 when
                             viscosity_mode = 1) */
  int32_t energy_df;      /* 0: total-energy DF (Section 4; default); 1: the
                             internal-energy DF that Section 5D uses for
                             Rayleigh-Benard convection so that no viscous
                             heating enters (the paper cites it without stating
                             it).  Reading: the second DF carries rho e,
                             e = b R T/2, relaxes by BGK at w_h towards
                             e f^eq, and receives a body-force source of first
                             moment e rho a with the (1 - w_h/2) factor; then
                             T = 2 sum(g)/(rho b R), the diffusivity is
                             R T (1/w_h - 1/2) = nu/Pr, and neither viscous
                             dissipation nor pressure work enters.
                             heq_moments, h_collision and h_force are ignored;
                             the energy sum of tclbm_sums is then sum rho e */
} tclbm_params;

/* FP64 whole-lattice reductions of the state the next step would see
 * (Eq. (20) and the temperature of Section 4). */
typedef struct {
  double mass;       /* sum rho */
  double momx, momy; /* sum rho u */
  double energy;     /* sum of hbar = sum rho E (sum rho e with energy_df = 1) */
  double kinetic;    /* sum rho u^2 / 2 */
  double nu_num;     /* sum u_y (T - T0)  (Nusselt numerator, Section 5D) */
  double rho_min, T_min;
  int64_t nonfinite; /* nodes with non-finite rho, u or T */
} tclbm_sums;

/* Fill *p with defaults: R = 1/3, T0 = 1, gamma = 1.4, Pr = 0.71, tau_f = 0.8,
 * w2 = w3 = w4 = 1, no force, thermal with correction, FP32 storage, all
 * sides periodic. */
void tclbm_default_params(int32_t nx, int32_t ny, tclbm_params *p);

/* Exact device bytes tclbm_create needs in dev_buf for these parameters
 * (two ping-pong population buffers, per-row reference tables, force field
 * and reduction scratch), or 0 if the parameters are invalid. */
size_t tclbm_state_bytes(const tclbm_params *p);

/* Validate p, lay out dev_buf, upload the initial macroscopic fields and
 * initialise fbar = f^eq - S/2, hbar = h^eq (Sections 3-4; g^eq = e f^eq for
 * the internal-energy DF) on the stream.
 * rho, ux, uy, T: host, nx*ny each (T ignored when thermal = 0).
 * ax_field, ay_field: host per-node acceleration (nullable; when given they
 * replace the uniform ax, ay).  hip_stream: a hipStream_t (NULL: default).
 * Boundaries come from p->bc (E_INVALID if unpaired or WALL on an x side).
 * On error *out is NULL and nothing is kept. */
tclbm_status tclbm_create(const tclbm_params *p, void *dev_buf, size_t dev_bytes, void *hip_stream,
                          const double *rho, const double *ux, const double *uy, const double *T,
                          const double *ax_field, const double *ay_field, tclbm_handle *out);

/* Change the boundary kind of one side and, for WALL, its velocity and
 * temperature, from the next step on (the state is left as it is).  The kinds
 * are those of Section 5: periodic sides; node walls whose velocity and
 * temperature are imposed by non-equilibrium extrapolation of both DFs from
 * the adjacent fluid node (the wall treatment of Sections 5B and 5D, applied
 * before the collision of each step); halfway bounce-back ends (the closed
 * shock tube of Section 5C).  side: tclbm_side; kind: tclbm_bc_kind; ux_w,
 * uy_w, T_w: the imposed wall velocity and temperature (used by WALL; T_w > 0;
 * WALL_ADIABATIC takes its temperature from the fluid, BOUNCEBACK and
 * PERIODIC ignore all three).  E_INVALID for an unknown side or kind, a WALL
 * kind on an x side, an adiabatic wall with ny < 4, a non-finite value, or a
 * change of an x side to or from PERIODIC (the x tiling of the state, hence
 * its layout, is fixed by the x sides given at create) (nothing is changed
 * then); an unpaired periodic axis is refused at step
 * time (set both sides of an axis before stepping).  Does not touch the
 * device; a batch that holds the handle must be rebuilt. */
tclbm_status tclbm_set_bc(tclbm_handle h, int32_t side, int32_t kind, double ux_w, double uy_w, double T_w);

/* Enqueue nsteps time steps (asynchronous, on the handle's stream).  One time
 * step is the update of Sections 2-4 for every node: wall extrapolation
 * (Sections 5B/5D), the macroscopic variables of Eq. (20) and the temperature
 * of Section 4, the correction gradients of Section 4, the cascaded relaxation
 * of Eq. (8) towards the shifted equilibria of Section 4 with the force source
 * of Section 3, the post-collision raw moments of Eq. (18) mapped back by
 * Eq. (3), the energy-DF update of Section 4 with its coupling source K, and
 * pull streaming of both DFs: Eq. (27) for f and the time-discrete energy-DF
 * equation of Section 4 for h.  The reading of the energy-DF update
 * (heq_moments, h_collision, h_force, or the internal-energy DF of Section
 * 5D with energy_df = 1) follows the parameters.  Long runs replay
 * a captured HIP graph of a fixed chunk of steps (not on the NULL stream, which
 * cannot be captured).  nsteps >= 0.  E_INVALID for a NULL handle, nsteps < 0
 * or an unpaired periodic axis; E_STATE once the handle has reported an
 * unstable state; E_DEVICE when a HIP launch fails (the steps enqueued before
 * the failure are counted by tclbm_steps_done). */
tclbm_status tclbm_step(tclbm_handle h, int64_t nsteps);

/* As tclbm_step, then synchronise and report the elapsed device time of the
 * enqueued steps (HIP events recorded on the handle's stream). */
tclbm_status tclbm_step_timed(tclbm_handle h, int64_t nsteps, double *ms);

/* Macroscopic fields (host float64, nx*ny each; any pointer may be NULL) and
 * FP64 sums of the current state.  Synchronises.  Returns E_UNSTABLE (fields
 * and sums still written) when a node is non-finite or has rho <= 0 or
 * T <= 0; the handle then refuses further steps with E_STATE. */
tclbm_status tclbm_moments(tclbm_handle h, double *rho, double *ux, double *uy, double *T, tclbm_sums *sums);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * outputs as tclbm_moments, bitwise, without any allocation.  The per-block
 * FP64 partial sums and the staged fields go through a fixed device array of
 * 4 MiB that the library holds on every GPU it runs on until the process ends
 * (not through the handle's buffers); the lattice is reduced in chunks of at
 * most 512 blocks of 256 nodes, in the block order of tclbm_moments, so any
 * lattice size is accepted.  Works on the handle's device (made current for
 * the call).  Every call on one GPU shares that array: calls that overlap on
 * one GPU (other host threads, other handles) race and must be serialised by
 * the caller.  Nothing in the array has to start at zero: each chunk rewrites
 * what it reads.  Host outputs as in tclbm_moments (any pointer may be NULL);
 * synchronises the handle's stream once per chunk.  Status codes as
 * tclbm_moments, plus E_DEVICE when the array's address cannot be obtained. */
tclbm_status tclbm_moments_noalloc(tclbm_handle h, double *rho, double *ux, double *uy, double *T,
                                   tclbm_sums *sums);

/* Number of time steps taken so far. */
int64_t tclbm_steps_done(tclbm_handle h);

/* Copy the raw post-collision population planes of the current state to the
 * host, in storage order [2][9][ny][nx] (f then h; h planes omitted when
 * thermal = 0), converted to float64 with the row reference added back.
 * out must hold 18*nx*ny doubles (9*nx*ny when athermal).  Synchronises. */
tclbm_status tclbm_read_state(tclbm_handle h, double *out);

/* Launch shape of the step kernel: rows per wave strip (>= 1; 0 = automatic)
 * and steps per captured HIP graph (even, >= 2; 0 = no graphs).  Results do not
 * depend on either (every node runs the same arithmetic). */
tclbm_status tclbm_set_tuning(tclbm_handle h, int32_t strip_rows, int32_t graph_chunk);

/* Name of the kernel that one step of this lattice launches under its current
 * launch shape: "row_group_kernel" (FP32 storage, default scheme, single-row
 * strips), "step_kernel" (other FP32), "step_kernel_16" (FP16/BF16) or
 * "step_kernel_f64".  A static string owned by the library; NULL for a NULL
 * handle.  For profilers and reports: it matches the kernel-trace name. */
const char *tclbm_step_kernel(tclbm_handle h);

/* Release the handle (waits for its stream, frees the library's own field
 * buffer and captured graphs).  No passage of the paper defines it: resource
 * management only.  dev_buf and the stream are not freed.  E_INVALID for a
 * NULL handle. */
tclbm_status tclbm_destroy(tclbm_handle h);

/* Diagnostic: enqueue one streaming copy of `bytes` (multiple of 16, 16-byte
 * aligned device pointers, non-overlapping) on the stream, with the access
 * types of the step kernels (plain loads, non-temporal stores).  Used to
 * measure the achievable HBM bandwidth next to the step kernel and to scale
 * hardware byte counters. */
tclbm_status tclbm_hbm_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* ---- batches: many resident lattices advanced by one launch per step ----
 * A batch references existing handles (all with the same storage form and the
 * same stream) and owns a small device table of their launch descriptors,
 * ordered largest lattice first.  tclbm_batch_step advances every member by
 * nsteps with one kernel launch per step (HIP-graph chunks when the stream is
 * not NULL); results equal those of stepping each member alone, bitwise.
 * While a member belongs to a batch, step it only through the batch; other
 * calls on it (moments, read_state) are fine.  Changing a member's boundaries
 * or tuning requires a new batch: tclbm_batch_step returns TCLBM_E_STATE,
 * stepping nothing, when a member was stepped alone, re-tuned, given new
 * boundaries or found unstable since the batch was built (or last stepped).
 * Destroy the batch before its members. */
typedef struct tclbm_batch *tclbm_batch_handle;
tclbm_status tclbm_batch_create(tclbm_handle *members, int32_t n, tclbm_batch_handle *out);
tclbm_status tclbm_batch_step(tclbm_batch_handle b, int64_t nsteps);
tclbm_status tclbm_batch_step_timed(tclbm_batch_handle b, int64_t nsteps, double *ms);
int32_t tclbm_batch_size(tclbm_batch_handle b);
int64_t tclbm_batch_waves(tclbm_batch_handle b);  /* wave64 work items per step */
tclbm_status tclbm_batch_set_graph_chunk(tclbm_batch_handle b, int32_t chunk);
/* Strip height (rows per wave strip) used for every member inside the batch,
 * capped at each member's ny; 0 (the default) picks one from the batch's total
 * work.  Members' own tuning is not changed; results are identical for any
 * height.  Synchronizes the stream.  Returns TCLBM_E_INVALID for rows < 0. */
tclbm_status tclbm_batch_set_strip_rows(tclbm_batch_handle b, int32_t rows);
int32_t tclbm_batch_strip_rows(tclbm_batch_handle b);  /* height in use */
/* Persistent launches: with steps_per_launch > 0, tclbm_batch_step runs the
 * time steps of Sections 2-4 for every member in launches of up to that many
 * steps each, instead of one launch per step.  The launch is cooperative (the
 * runtime refuses a grid that cannot be resident at once); its blocks meet at
 * a grid barrier between steps.  Results are identical to the per-step path.
 * wait_us bounds a block's wait at a barrier (0: one second): a block that
 * waits longer flags the launch and every block leaves, so a launch always
 * ends; the steps it counted then leave the members' states undefined, the
 * members are marked unstable and the next tclbm_batch_step returns
 * TCLBM_E_STATE (tclbm_batch_step_timed reports TCLBM_E_DEVICE itself).
 * Under stream capture the batch records per-step launches.  steps_per_launch
 * = 0 returns to per-step launches.  TCLBM_E_INVALID for negative arguments,
 * FP64 storage, or a member off the default scheme or beyond buffer
 * addressing (4 GiB of state); TCLBM_E_DEVICE without cooperative launch. */
tclbm_status tclbm_batch_set_persistent(tclbm_batch_handle b, int32_t steps_per_launch, int32_t wait_us);
int32_t tclbm_batch_persistent(tclbm_batch_handle b);  /* steps per launch, 0: per-step launches */
/* Name of the kernel a batch step launches ("batch_step_kernel_f32",
 * "batch_step_kernel" for 16-bit storage, "batch_step_kernel_f64"; with
 * persistent launches "batch_persistent_kernel_f32" or
 * "batch_persistent_kernel"), as a kernel trace shows it; a static string,
 * NULL for a NULL batch. */
const char *tclbm_batch_step_kernel(tclbm_batch_handle b);
tclbm_status tclbm_batch_destroy(tclbm_batch_handle b);

/* Static string for a status code; last HIP/validation message of a handle. */
const char *tclbm_status_str(tclbm_status s);
const char *tclbm_last_error(tclbm_handle h);

#ifdef __cplusplus
}
#endif

#endif /* TCLBM_H */
