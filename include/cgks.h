/*
 * cgks.h -- C ABI of the compact 8th-order gas-kinetic scheme on MI355X.
 *
 * The library advances the Euler equations (with a viscosity mu > 0 in the
 * configuration, the Navier-Stokes equations of the BGK model) on structured
 * 1D and 2D grids by the compact gas-kinetic scheme of Zhao, Ji, Shyy, Xu
 * (arXiv 2001.01570):
 * given cell averages W and cell-averaged gradients W' (Sec. 3.1, eqs.
 * compact-deriv-1 / compact-deriv), one step performs the compact linear and
 * WENO-Z reconstruction (Sec. 3.2-3.3), the gas-kinetic interface evolution
 * (Sec. 2.1, eq. 3rd-simplify-flux) and the two-stage fourth-order update of
 * both W and W' (Sec. 2.2, eq. step-hyper-1 and the interface-state update).
 * Every step runs in HIP kernels on the device; all arithmetic is FP64.
 *
 * Field layout (structure of arrays, x fastest, row-major in y):
 *   1D: 6 fields  [rho, rhoU, rhoE, (rho)_x, (rhoU)_x, (rhoE)_x], each nx
 *   2D: 12 fields [W(4), W_x(4), W_y(4)], W = (rho, rhoU, rhoV, rhoE), each ny*nx
 * Field f, cell (i, j) lives at fields[(f*ny + j)*nx + i].
 *
 * Error behaviour: every call returns CGKS_OK (0) or a negative code; nothing
 * aborts.  A step that produces a non-physical cell (rho <= 0, p <= 0 or
 * NaN) is not committed: the state stays at the last good step and the call
 * returns CGKS_ENONPHYS (cgks_last_bad_cell names the first bad cell).
 * Threading: one host thread per context at a time.
 */
#ifndef CGKS_H
#define CGKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGKS_OK 0
#define CGKS_EINVAL (-1)     /* bad argument or configuration                      */
#define CGKS_ENOMEM (-2)     /* device or host allocation failed                    */
#define CGKS_EDEVICE (-3)    /* a HIP call failed                                   */
#define CGKS_ENONPHYS (-4)   /* non-physical state; step not committed              */
#define CGKS_EBUSY (-5)      /* batch: no free slot or memory budget exhausted      */
#define CGKS_ESTATE (-6)     /* call not valid in the current state (e.g. no state) */

/* Boundary conditions (two ghost layers, mirrored or copied cells): periodic;
 * free (copy of the edge cell, zero gradients); slip wall (mirror, normal
 * momentum odd); inflow (the side's fixed state, zero gradients); no-slip
 * wall (mirror with every momentum odd: zero velocity and, the temperature
 * being even, zero heat flux at the wall; for viscous flow). */
enum { CGKS_PERIODIC = 0, CGKS_FREE = 1, CGKS_WALL = 2, CGKS_INFLOW = 3, CGKS_NOSLIP = 4 };
/* Storage of the state fields.  CGKS_FP32_STORAGE (2D only): the 8 cell-
 * averaged gradient fields of the state and of the stage buffers are kept in
 * FP32; cell averages, all arithmetic, the conservative accumulation and the
 * tau/exp evaluation stay FP64.  Fields cross the boundary in FP64 either way
 * (the gradients are rounded to FP32 on set_state). */
enum { CGKS_FP64 = 0, CGKS_FP32_STORAGE = 1 };
/* Variables of the nonlinear reconstruction (Sec. 3.2: the compact
 * reconstruction acts on conservative or characteristic variables).
 * CGKS_CHARACTERISTIC: on every stencil line the WENO-Z left and right
 * states are reconstructed in the coordinates of the right eigenvectors of
 * the Euler flux Jacobian normal to the face, at the mean of the two cells
 * beside the face (eigenvectors scaled to a first entry of 1), and projected
 * back; a line whose mean state is not admissible keeps the conservative
 * variables.  The linear reconstruction is the same either way. */
enum { CGKS_CONSERVATIVE = 0, CGKS_CHARACTERISTIC = 1 };

typedef struct cgks_ctx cgks_ctx;

typedef struct {
  int dim;                   /* 1 or 2                                                  */
  int nx, ny;                /* cells; ny ignored in 1D; wall sides need >= 2 cells      */
  double x0, x1, y0, y1;     /* domain                                                   */
  double gamma;              /* ratio of specific heats (> 1)                            */
  double cfl;                /* CFL number of the time step rule (Sec. 4)                */
  int bc[4];                 /* xlo, xhi, ylo, yhi: CGKS_PERIODIC|FREE|WALL|INFLOW|NOSLIP;
                                periodic must be paired on both sides of an axis         */
  double inflow_prim[4][4];  /* (rho, U, V, p) of each CGKS_INFLOW side                  */
  double weno_eps;           /* epsilon of the WENO-Z weights (eq. WENO-Z-w), e.g. 1e-6  */
  double tau_eps, tau_C;     /* collision time eps*dt + C|dp/sum p|*dt (Sec. 4): 0.01, 1 */
  double fixed_dt;           /* 0: CFL rule; > 0: fixed step (accuracy tests, Sec. 4.1) */
  int storage;               /* CGKS_FP64 or CGKS_FP32_STORAGE (2D)                      */
  double mu;                 /* dynamic viscosity (>= 0).  0: Euler equations.  > 0:
                                Navier-Stokes with the BGK Prandtl number 1; the
                                collision time is mu/p + C|dp/sum p|*dt in both of
                                its roles (Sec. 4, viscous form) and tau_eps is
                                unused; CGKS_NOSLIP gives viscous walls              */
  int gauss_points;          /* 2D: Gauss-Legendre points per face segment (the
                                quadrature points along the interface of Sec. 2,
                                their number not given there).  0 or 2: the
                                quartic through 5 segment averages, two points
                                (fourth order in space in 2D; the default).  4:
                                the sextic through 7 segment averages, four
                                points (eighth order in 2D; walls need 3 cells
                                across; tile shape fixed)                            */
  int recon_vars;            /* CGKS_CONSERVATIVE (0, the default) or
                                CGKS_CHARACTERISTIC, for the WENO-Z states           */
  int side_slopes;           /* normal slopes of the two non-equilibrium sides in the
                                kinetic evolution (Sec. 2.1).  0 (the default): the
                                linear reconstruction's derivative at the face for
                                both sides.  1 (an evaluated variant; 1D or 2D, two
                                or four Gauss points; conservative variables;
                                contexts, the batch and cgks_step_noalloc): each side
                                takes the derivative of its WENO-Z combination (the
                                candidates' slopes with the same nonlinear weights),
                                in 2D per stencil line, taken to the Gauss point
                                like the normal derivative; a side that falls back
                                to its cell average takes the linear one.  Other
                                values and combinations: CGKS_EINVAL               */
  int tang_weno;             /* tangential assembly of the two WENO-Z states in 2D.
                                0 (the default): the quintic of the three nearest
                                face segments, as for the linear quantities.  1 (an
                                evaluated variant; two or four Gauss points,
                                conservative variables, side_slopes 0; contexts,
                                the batch and cgks_step_noalloc): a WENO-Z of the
                                three quadratics on the five nearest segments'
                                averages.  Other values and combinations:
                                CGKS_EINVAL                                          */
} cgks_config;

typedef struct {
  long steps;                /* committed steps since set_state                         */
  long guard_w0;             /* points where the linear equilibrium state was replaced  */
  long guard_weno;           /* points where a WENO state fell back to a cell average   */
  double last_dt;            /* step size of the last committed step                    */
  double t;                  /* current time                                            */
} cgks_counters_t;

/* Create a solver context.  hip_stream (a hipStream_t, may be NULL for the
 * null stream) is borrowed: all work is queued on it and it must outlive the
 * context.  The context owns every device buffer it allocates. */
int cgks_create(const cgks_config *cfg, void *hip_stream, cgks_ctx **out);

/* Load a state (layout above).  fields is a host pointer (on_device = 0) or a
 * device pointer (on_device = 1); it is copied, never retained.  Rejects a
 * non-physical cell with CGKS_ENONPHYS. */
int cgks_set_state(cgks_ctx *ctx, const double *fields, int on_device, double t0);

/* One step of the rule in the configuration (CFL or fixed_dt). */
int cgks_step(cgks_ctx *ctx, double *dt_used);

/* One step of the given size dt > 0 (dt <= 0 falls back to the rule). */
int cgks_step_dt(cgks_ctx *ctx, double dt, double *dt_used);

/* Advance until t_end: every step uses the rule; the step that reaches t_end
 * to within (1 + 1e-9) of its size is the last and lands on t_end exactly.
 * max_steps > 0 bounds the number of steps of this call. */
int cgks_advance_to(cgks_ctx *ctx, double t_end, long max_steps, long *steps_taken);

/* Exactly n steps of the rule (no end time); used to time fixed step counts.
 * On a capturable stream (not the legacy null stream) and with profiling
 * off, runs of 25 steps replay one captured HIP graph.
 * 1D grids of at most 255 cells (with profiling off) run whole steps in one
 * single-block launch instead, in cgks_step, cgks_step_dt, cgks_advance_to
 * and cgks_run_steps alike: the same arithmetic, with results that agree with
 * the separate launches to rounding. */
int cgks_run_steps(cgks_ctx *ctx, long n);

/* Copy the current state out (host or device pointer); t and step may be NULL. */
int cgks_get_state(cgks_ctx *ctx, double *fields_out, int on_device, double *t, long *step);

int cgks_last_bad_cell(const cgks_ctx *ctx, long *cell);

/* Measurement: kernel kind k (2D: xfaces1, yfaces1, update1, xfaces2,
 * yfaces2, update2; 1D: faces1, update1, faces2, update2) is bracketed by HIP
 * events on the context's stream at every launch while bit k of the
 * profiling mask is set (mask -1: all kinds; 0: off; fewer kinds, fewer
 * events in the stream).  cgks_kernel_times fills ms[k] (accumulated device
 * milliseconds) and calls[k] and returns the number of kinds, or an error.
 * Setting a nonzero mask clears the accumulators.  While profiling is on,
 * cgks_run_steps launches step by step instead of replaying its graph,
 * and small 1D grids use the separate kernels, so that each can be timed. */
int cgks_set_profiling(cgks_ctx *ctx, int mask);
int cgks_kernel_times(cgks_ctx *ctx, double *ms, long *calls, int n);
int cgks_counters(cgks_ctx *ctx, cgks_counters_t *out);

/* Tile shape of the face kernels per direction: 0 = 8 faces x 16 segments,
 * 1 = 4 x 32, 2 = 2 x 64 (faces along the normal x segments along the face).
 * Results do not depend on the shape (each face is computed alike); the
 * choice only changes speed and is made by the autotuner's table.  It
 * applies to two-point FP64 and FP32 configurations with conservative
 * variables; four points and characteristic variables use one fixed shape
 * per direction. */
int cgks_set_tiles(cgks_ctx *ctx, int x_shape, int y_shape);
void cgks_destroy(cgks_ctx *ctx);
const char *cgks_strerror(int code);

/* ---- One step without allocation ------------------------------------------
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One step of
 * the configuration's problem (as cgks_step / cgks_step_dt on a context with
 * that configuration and state) from the device state `in` to the device
 * state `out`: both device pointers of nf * nx * ny doubles in the layout
 * above, distinct buffers; `in` is only read.  dt > 0: a step of that size;
 * otherwise the configuration's rule (CFL or fixed_dt).  The intermediate
 * buffers of the step live in a static device array of the library, one per
 * GPU for the life of the process, sized for CGKS_NOALLOC_MAX_CELLS cells:
 * larger grids, FP32 storage or in == out return CGKS_EINVAL.  The call
 * allocates nothing; it runs on the current device, and hip_stream (NULL: the
 * null stream) must belong to it.  Every call on one GPU uses that GPU's one
 * array: calls that overlap on a GPU (other streams or host threads) race and
 * must be serialised by the caller.
 * dt_used == NULL: the work is only queued on hip_stream (no host
 * synchronisation, so the call can be captured into a graph), and a
 * non-physical result is not reported.  Otherwise the call waits for the step
 * and returns CGKS_ENONPHYS if the input or the result has a non-physical
 * cell (out then holds no valid state), else stores the step size. */
#define CGKS_NOALLOC_MAX_CELLS 65536
int cgks_step_noalloc(const cgks_config *cfg, const double *in, double *out, double dt, void *hip_stream,
                      double *dt_used);

/* ---- Batch: many independent 2D problems advanced together (serving) ------
 *
 * Same scheme and kernels as a context; the requests of a serving workload
 * are independent solves of the problem statement above.  A batch owns one
 * device arena of hbm_budget_bytes (first-fit with coalescing) from which each
 * admitted problem, a "slot", takes its buffers (about 130 bytes per cell:
 * 4 x 12 fields plus the face results).  cgks_batch_run advances every running
 * slot together: each of the 8 kernels of a step is one launch covering the
 * blocks of all running slots (a work list in device memory, rewritten on
 * admission and release), and the requested number of steps is one HIP graph,
 * captured again only when a work list leaves the power-of-two bucket its
 * launch grid was sized for, or the step count changes.  A slot stops by
 * itself at its end time or step bound; its state
 * stays readable until it is released.  All calls are synchronous with
 * respect to the host and not thread-safe. */
typedef struct cgks_batch cgks_batch;

enum { CGKS_SLOT_FREE = 0, CGKS_SLOT_RUNNING = 1, CGKS_SLOT_DONE = 2, CGKS_SLOT_FAILED = 3 };

/* max_slots in [1, 1024].  hip_stream NULL: the batch creates its own stream;
 * otherwise the given stream is used and must be capturable (not the legacy
 * null stream).  CGKS_ENOMEM if the arena cannot be allocated. */
int cgks_batch_create(size_t hbm_budget_bytes, int max_slots, void *hip_stream, cgks_batch **out);

/* Admit a 2D problem (configuration and initial state as for a context; the
 * state is copied, host or device pointer) that runs until t_end (> 0) or for
 * max_steps (> 0) steps, whichever comes first (one of them must be given).
 * Any configuration a 2D context accepts is admitted: two or four Gauss
 * points, FP64 or FP32 gradient storage, conservative or characteristic
 * variables, the side-slope and tangential-WENO variants; slots of each such kind share their own
 * face launches, so a mix
 * of kinds runs in one step.  Returns its slot.
 * CGKS_EBUSY: no free slot or no room in the arena; CGKS_ENONPHYS:
 * non-physical initial state; CGKS_EINVAL: bad configuration or dim != 2.  A
 * device pointer must be ready (its producer synchronized). */
int cgks_batch_admit(cgks_batch *b, const cgks_config *cfg, const double *fields, int on_device,
                     double t_end, long max_steps, int *slot);

/* Advance every running slot by up to `steps` (>= 1) steps. */
int cgks_batch_run(cgks_batch *b, int steps);

/* Slot state after the last run or admit: CGKS_SLOT_*; t and step may be NULL. */
int cgks_batch_poll(cgks_batch *b, int slot, int *state, double *t, long *step);

/* Copy a slot's current state out (layout as for a context). */
int cgks_batch_read(cgks_batch *b, int slot, double *fields_out, int on_device);

/* Face tile shapes (as for cgks_set_tiles) of the two-point FP64 slots;
 * only while no slot is admitted (CGKS_ESTATE otherwise).  A new batch takes
 * the autotuner's shapes.  Results do not depend on the shapes. */
int cgks_batch_set_tiles(cgks_batch *b, int x_shape, int y_shape);

/* The autotuner's batch entry: tile shapes of the two-point FP64 slots and
 * the steps per cgks_batch_run that gave the serving mix its highest rate
 * (any pointer may be NULL). */
int cgks_batch_tuning(int *x_shape, int *y_shape, int *steps_per_run);

/* Free a slot and return its memory to the arena. */
int cgks_batch_release(cgks_batch *b, int slot);
void cgks_batch_destroy(cgks_batch *b);

#ifdef __cplusplus
}
#endif
#endif
