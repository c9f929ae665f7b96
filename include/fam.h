/*
 * fam.h - C ABI of the MI355X (gfx950) library for the compact
 * finite-average-moment (FAM) scheme with single-step oscillation elimination.
 *
 * Method (all section / equation / table labels refer to the FAM paper):
 *  - evolved state: cell average and scaled first moments of every conserved
 *    component (Sec. 2.1 for 1D, Sec. 2.2 for 2D);
 *  - each SSP-RK3 stage (eq. 3 / eq. 12) evaluates the semi-discrete operator
 *    of eq. (1dSemi) / eq. (11): componentwise compact linear reconstruction of
 *    order k = 3..6 (Sec. 2.4), Lax-Friedrichs (Rusanov) flux at 4 Gauss points
 *    per face, 4x4 Gauss quadrature of the first-moment volume term;
 *  - after the last stage one OE pass (Prop. 2.1; eqs. 1dOE_system,
 *    2dOE_system; Tables sigma1d / sigma2d) keeps the cell averages and damps
 *    the first moments by exp(-beta dt sigma / dx).
 *
 * Memory layout of a state U (all doubles, structure of arrays):
 *   U[((c * M) + m) * ny * nx + j * nx + i]
 * with component c (scalar laws: 1; 1D Euler: rho, rho u, E; 2D Euler: rho,
 * rho u, rho v, E), moment m (M = 2 in 1D: average, x-moment; M = 3 in 2D:
 * average, x-moment, y-moment), row j < ny (ny = 1 in 1D) and column i < nx.
 * A batched context stores its instances one after another in one buffer, each
 * in the layout above (fam_instance_offset gives the start of each).
 *
 * Ownership: every pointer to state data is a DEVICE pointer owned by the
 * caller.  The library owns its scratch (two stage buffers, reduction slots,
 * the adjoint's checkpoints and tapes), allocated in fam_init / fam_init_batched
 * / on the first fam_adjoint call and freed by fam_destroy.
 *
 * Clock: a context keeps the simulation time of every instance, 0 after
 * fam_init / fam_init_batched.  Every step advances it by its dt (fam_step,
 * fam_run, and fam_dt, which begins a step for fam_stage / fam_oe); fam_set_time
 * sets it.  The time enters the scheme only through time-dependent boundary data
 * (the dmr boundaries' moving shock, evaluated at each RK stage's time).  The
 * autotuner and the adjoint leave it unchanged.
 *
 * Streams: all work is enqueued on the stream given to fam_init (NULL: the
 * default stream).  fam_step and fam_stage / fam_oe / fam_dt are asynchronous;
 * fam_run, fam_check and fam_adjoint synchronise the stream before returning.
 * Calls on one context must not overlap.
 *
 * Errors: functions return a fam_status and never throw.  A non-physical state
 * (a cell average used for a wave speed with rho <= 0, p <= 0 or not finite)
 * raises a device flag; fam_run and fam_check report it as FAM_ERR_NONPHYSICAL.
 */
#ifndef FAM_H
#define FAM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FAM_OK = 0,
  FAM_ERR_ARG = -1,          /* invalid argument or configuration            */
  FAM_ERR_DEVICE = -2,       /* a HIP call failed                            */
  FAM_ERR_NOMEM = -3,        /* device allocation failed                     */
  FAM_ERR_NONPHYSICAL = -4,  /* inadmissible cell average met (device flag)  */
  FAM_ERR_STATE = -5,        /* call not valid for this context              */
  FAM_ERR_SIZE = -6          /* problem larger than fam_step_static's scratch */
} fam_status;

typedef enum { FAM_ADVECTION = 0, FAM_BURGERS = 1, FAM_EULER = 2 } fam_system;
typedef enum { FAM_BC_PERIODIC = 0, FAM_BC_TRANSMISSIVE = 1 } fam_bc;
typedef enum { FAM_OE_OFF = 0, FAM_OE_TYPE1 = 1, FAM_OE_TYPE2 = 2 } fam_oe_type;

typedef struct {
  int dim;                /* 1 or 2                                               */
  int nx, ny;             /* cells; ny is ignored (1) when dim == 1               */
  double x0, x1, y0, y1;  /* domain [x0,x1] x [y0,y1]                             */
  int k;                  /* order 3..6 (Sec. 2.4)                                */
  int system;             /* fam_system                                           */
  double gamma;           /* ratio of specific heats (Euler)                      */
  double ax, ay;          /* advection velocity                                   */
  int bc_x, bc_y;         /* fam_bc: periodic, or transmissive (two ghost layers
                             copying every moment of the nearest interior cell;
                             Remark after Algorithm 1)                            */
  int oe;                 /* fam_oe_type                                          */
  double oe_gamma_k;      /* <= 0: the paper's gamma_k (1D 25/25/12.5/12.5,
                             2D 25/25/15/15 for k = 3..6; Secs. 2.1, 2.2)         */
  double cfl;             /* C of the time step dt = C dx/alpha_x (1D) or
                             C/(alpha_x/dx + alpha_y/dy) (2D) (Sec. 4)            */
  int k6_jump_from_table; /* k = 6, 2D: 0 = OE jumps of p_6 (the text's u_h^*),
                             1 = jumps of the full auxiliary Q_6, which is what
                             the printed matrices A_6, B_6, C_6 encode           */
  int pp;                 /* 2D Euler only: positivity safeguard applied to each
                             stage's reconstruction (the paper's auxiliary BP/PP
                             limiter is cited, not specified; this is the scaling
                             limiter toward the cell average that keeps density
                             and pressure >= min(1e-13, rho_avg, p_avg) at all 32
                             flux points of every cell).  0 = off.               */
  int dt_rule;            /* time step without dt_fixed (Sec. 4): 0 = C dx/alpha_x
                             (2D: C/(alpha_x/dx + alpha_y/dy)), the rule of the
                             discontinuous problems; 1 = the same with dx^{k/3},
                             dy^{k/3} in place of dx, dy, the rule of the smooth
                             accuracy tests.                                      */
  int dmr;                /* 2D Euler only: the boundaries of the double Mach
                             reflection example (Sec. 4): post-shock inflow on the
                             left, outflow (copy) on the right, on the bottom the
                             post-shock state for x < 1/6 and a reflecting wall
                             beyond, on the top the exact moving shock (post-shock
                             state for cell centres x < 1/6 + (y1 + 20 t)/sqrt 3,
                             pre-shock state beyond); states (rho, u, v, p) =
                             (8, 8.25 cos 30deg, -8.25 sin 30deg, 116.5) and
                             (1.4, 0, 0, 1).  bc_x, bc_y are ignored.  0 = off.  */
  int char_vars;          /* Euler with k = 5 only: every RK stage reconstructs in
                             the local characteristic variables of each cell's
                             average (textbook eigenvectors of the x-direction flux
                             Jacobian; L on the stencil moments, R on the
                             coefficients), the FAM5 variant timed in Sec. 4.3
                             (Table runtime-main, Panel B).  The reconstruction is
                             linear, so the result is the conservative one up to
                             rounding (Sec. 2.3); OE and the limiter are unchanged.
                             0 = off.                                             */
} fam_config;

typedef struct fam_ctx fam_ctx;

/* Validate cfg, allocate scratch, bind the HIP stream (hipStream_t or NULL). */
fam_status fam_init(const fam_config* cfg, void* hip_stream, fam_ctx** out);

/* A context advancing n_inst independent 2D instances together (one launch per
 * RK stage and one OE launch for all of them).  All instances share dim = 2,
 * k, system, gamma, oe, cfl and the boundary conditions; sizes and domains may
 * differ.  Every instance uses its own time step.  FAM_ERR_ARG for OE Type I,
 * the dmr boundaries or char_vars (single contexts only). */
fam_status fam_init_batched(const fam_config* per_instance, int n_inst, void* hip_stream,
                            fam_ctx** out);

/* Number of doubles in a state (sum over instances for a batched context). */
size_t fam_state_len(const fam_ctx* ctx);
/* Offset (in doubles) of instance i inside a batched state; 0 for i = 0. */
size_t fam_instance_offset(const fam_ctx* ctx, int i);
int fam_num_instances(const fam_ctx* ctx);

/* One full step in place on U: CFL time step (unless dt_fixed > 0), three
 * SSP-RK3 stages, OE; from the context clock's time t to t + dt (the clock
 * advances).  If dt_used_dev is not NULL the time step used is stored
 * there (device memory; one double per instance).  Asynchronous.  Allocates
 * nothing and enqueues only kernels and device-to-device copies on the
 * context's stream, so it may be captured in a HIP graph and replayed. */
fam_status fam_step(fam_ctx* ctx, double* U, double dt_fixed, double* dt_used_dev);

/* Advance U in place until the context clock reaches t_final (the last step
 * clipped to land on it; nothing is done if the clock is already there) or
 * until max_steps steps, whichever comes first (t_final <= 0: max_steps steps).
 * dt_fixed > 0 replaces the CFL rule.  Steps are enqueued in chunks replayed
 * from a captured HIP graph; the stream is synchronised between chunks to test
 * for termination and non-physical states.  For a batched context every
 * instance runs to t_final (each with its own dt), and steps_done is the
 * largest per-instance count of this call.  t_done (host, may be NULL): the
 * clock at return (the smallest over instances). */
fam_status fam_run(fam_ctx* ctx, double* U, double t_final, int max_steps, double dt_fixed,
                   int* steps_done, double* t_done);

/* Set the context clock of every instance to t (for example back to 0 before
 * running again from an initial state).  Asynchronous, on the context's stream
 * (a kernel, so it may be captured too).  FAM_ERR_ARG for a NULL context or a
 * t that is not finite. */
fam_status fam_set_time(fam_ctx* ctx, double t);

/* Building blocks of one step, for tests and profiling (asynchronous):
 * fam_dt:    dt_dev[inst] = CFL time step of U (or dt_fixed if > 0); also primes
 *            the wave-speed reduction used by the next fam_stage(s = 0).
 * fam_stage: Uout = a_s U0 + b_s (Us + dt R(Us)) with (a_s, b_s) = (0, 1),
 *            (3/4, 1/4), (1/3, 2/3) for s = 0, 1, 2 (eq. 12).  Uout must not
 *            alias Us.  Call in order s = 0, 1, 2 after fam_dt.  With the limiter's
 *            segment list, the s = 0 launch also re-cuts the list from its row
 *            costs for the following launches, as a step does.
 * fam_oe:    Uout = OE(Un) with the time step in dt_dev (Uout must not alias Un). */
fam_status fam_dt(fam_ctx* ctx, const double* U, double dt_fixed, double* dt_dev);
fam_status fam_stage(fam_ctx* ctx, int s, const double* U0, const double* Us, double* Uout,
                     const double* dt_dev);
fam_status fam_oe(fam_ctx* ctx, const double* Un, double* Uout, const double* dt_dev);

/* Synchronise and report the device flag (FAM_OK or FAM_ERR_NONPHYSICAL);
 * clears the flag. */
fam_status fam_check(fam_ctx* ctx);

/* Launch-shape autotuner (not part of the method: it only picks how the same
 * arithmetic is tiled).  Times candidate shapes on the state U (device, read
 * only) with reps timed launches each and keeps the fastest for this context:
 * a single 2D instance tunes the strip-tile height of the RK stage kernel and of
 * the OE kernel separately; a batch tunes the tile height of its work list and
 * the persistent grid size.  Results are unchanged by the choice (bitwise).
 * The context's stage buffers are overwritten, captured step graphs are
 * dropped, and the device flag is cleared.  choice (host, may be NULL, 2 ints)
 * receives (stage H, OE H) or (batch H, persistent blocks); stage H = 0 is the
 * segment list of a limiter-on context (fam_set_tiling).  Synchronous.
 * FAM_ERR_ARG for a NULL context / state or reps < 1; 1D contexts: no-op. */
fam_status fam_autotune(fam_ctx* ctx, const double* U, int reps, int* choice);

/* Set the launch shapes of a single 2D instance directly (for example a choice
 * that fam_autotune returned earlier): stage_H = strip-tile height of the RK
 * stage kernel, or 0 for the segment list of a limiter-on context (each strip
 * cut into segments of equal cost, recorded per row by the previous stage
 * launch; one round of waves); oe_H = tile height of the OE kernel.  Results
 * are unchanged by the choice (bitwise).  Captured step graphs are dropped.
 * FAM_ERR_ARG for a NULL context, heights outside [8, ny] (or [1, ny] when ny <
 * 8) or stage_H = 0 without the limiter (or with more strips than wave slots);
 * FAM_ERR_STATE for 1D or batched contexts.  Asynchronous. */
fam_status fam_set_tiling(fam_ctx* ctx, int stage_H, int oe_H);

/* Gradient of a final-time functional J(U_T) with respect to the initial state
 * U0 after nsteps steps with the fixed time step dt (not differentiated), by
 * hand-written adjoint kernels of the OE, the three RK stages and R(U), with a
 * checkpoint every checkpoint_every steps and recomputation of each segment.
 * dJdUT: device pointer to dJ/dU_T, or NULL for the built-in functional
 * J = integral over [1/4,3/4]^2 of rho_h(T)^2 = sum over cells with centres in
 * the window of dx dy (rho0^2 + 12 rho1^2 + 12 rho2^2) (2D only).
 * dJdU0: device output, same layout as U0.  J_out (host, may be NULL) receives
 * J for the built-in functional.  Non-smooth points use one-sided choices:
 * |x|' = sign(x) with sign(0) = 0, maxima pass the derivative to their first
 * maximal entry, the zero-denominator branch of the OE coefficient has zero
 * derivative.  Synchronous.  Supported contexts: one 2D Euler instance,
 * periodic in x and y (no dmr boundaries, no char_vars), OE off or Type II, no positivity limiter, k = 6 with the
 * jumps of p_6; any other context returns FAM_ERR_STATE.  FAM_ERR_ARG for NULL
 * pointers, nsteps < 1, dt <= 0 or checkpoint_every < 1; FAM_ERR_NOMEM when the
 * checkpoints (ceil(nsteps / checkpoint_every) states) and the segment tape
 * (4 checkpoint_every states) do not fit (checkpoint_every >= nsteps records
 * the whole run as one segment: no recomputation, a tape of 4 nsteps states); FAM_ERR_NONPHYSICAL if the forward
 * run meets an inadmissible state.  The scratch is kept for later calls and
 * freed by fam_destroy. */
fam_status fam_adjoint(fam_ctx* ctx, const double* U0, int nsteps, double dt,
                       int checkpoint_every, const double* dJdUT, double* dJdU0, double* J_out);

/* Test-only exports (single-instance contexts; FAM_ERR_STATE otherwise, and for
 * fam_dbg_recon also with the dmr boundaries; FAM_ERR_ARG
 * for NULL pointers).  Asynchronous.
 *
 * fam_dbg_recon: point values of the stage reconstruction p_k of U (Sec. 2.4;
 *   eqs. 5 / 6, appendix coefficients; ghost cells per the boundary conditions;
 *   no positivity limiter; conservative variables also with char_vars, which
 *   gives the same polynomial up to rounding) at every cell's flux points.  2D: NP = 32 points per
 *   cell and component: right face (1/2, eta_g), left face (-1/2, eta_g), top
 *   face (xi_g, 1/2), bottom face (xi_g, -1/2) for g = 0..3, then the volume
 *   nodes (xi_a, eta_b) at 16 + 4b + a; 1D: NP = 6: right face, left face, volume
 *   node xi_a at 2 + a.  Gauss nodes ascending in [-1/2, 1/2].  vals (device,
 *   caller-owned, nc * NP * cells doubles): vals[((c * NP) + q) * cells + cell].
 * fam_dbg_oe_factors: the OE damping factor delta = exp(-beta^x dt sigma^x / dx
 *   - beta^y dt sigma^y / dy) of every cell (Prop. 2.1; eq. 2dOE_system, in 1D
 *   eq. 1dOE_system), as computed by the OE launch of fam_oe on Un with the time
 *   step in dt_dev; delta (device, caller-owned, cells doubles) in cell order.
 *   The launch's state output goes to the context's own scratch.  Un must be a
 *   caller buffer.  FAM_ERR_STATE with OE off. */
fam_status fam_dbg_recon(fam_ctx* ctx, const double* U, double* vals);
fam_status fam_dbg_oe_factors(fam_ctx* ctx, const double* Un, const double* dt_dev, double* delta);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): one full step in place
 * on U, as fam_step on a fresh context for cfg (same kernels and launch shapes,
 * the same result bit for bit), without a context and without allocating.
 * cfg: as for fam_init (single instance).  hip_stream: hipStream_t or NULL.
 * U: device state in the layout above (caller-owned).  t: the time at the start
 * of the step (it enters only through time-dependent boundary data: the dmr
 * boundaries).  dt_fixed > 0 replaces the CFL rule.  dt_used_dev (device, may be
 * NULL): receives the step's dt.  flag_dev (device int, may be NULL): 1 is ORed
 * into it when a non-physical cell average is met (the caller clears it; NULL:
 * the condition is not reported).  Asynchronous; enqueues only kernels and one
 * device-to-device copy of dt.
 * Scratch: a device array of FAM_STATIC_SCRATCH_BYTES on each GPU the library
 * runs on, held until the process ends (the two SSP-RK3 stage states and the
 * step's reduction slots): states of at most (FAM_STATIC_SCRATCH_BYTES -
 * 256 KiB) / 16 doubles, e.g. a 2D Euler mesh of 512 x 512 cells; larger ones
 * return FAM_ERR_SIZE before anything is enqueued.  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller.  FAM_ERR_ARG for a NULL
 * cfg or U, an invalid cfg, a t that is not finite or a NaN dt_fixed. */
#define FAM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
fam_status fam_step_static(const fam_config* cfg, void* hip_stream, double* U, double t, double dt_fixed,
                           double* dt_used_dev, int* flag_dev);

void fam_destroy(fam_ctx* ctx);
const char* fam_status_str(fam_status s);

#ifdef __cplusplus
}
#endif

#endif /* FAM_H */
