/*
 * hweno.h -- C ABI of the MI355X (gfx950) L-HWENO hot path.
 *
 * Method: Zhang & Zhao, "A fifth-order finite difference HWENO scheme combined
 * with limiter for hyperbolic conservation laws" (arXiv 2207.05258), Section 2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is DEVICE memory owned by the caller
 * (e.g. torch tensors); the library allocates no device memory and keeps no
 * device state, apart from the fixed static array of hweno_rk3_step_static.
 * Pointers are borrowed until the enqueued work has completed.
 *
 * State layout.  One contiguous buffer of nf fields, each ny * nx values of the
 * problem's dtype, x fastest ("SoA [nf][ny][nx]", ny == 1 when dim == 1):
 * the m conserved components U, then their x-derivatives U_x, then (2D) their
 * y-derivatives U_y, nf = m * (1 + dim), with m = 1 for the scalar
 * equations, 3 for 1D Euler and 4 for 2D Euler (rho, rho u, [rho v,] E).
 * Values are point values at cell centres x_i = x_lo + (i + 1/2) dx.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default stream).
 * Every call only enqueues work on it, never synchronises, and never copies
 * between host and device, so the calls may be captured in a hipGraph.
 *
 * Errors.  Argument errors are detected on the host before any HIP call and
 * returned as a status code; hweno_last_error() then gives a thread-local
 * message.  Launch failures return HWENO_ERR_LAUNCH.  Numerical failure
 * (non-finite values, rho <= 0, p <= 0) is not an error code: it is recorded
 * in the device status word of the step control block (see below).  Nothing
 * aborts and nothing throws across this ABI.  A grid with nx == 0 or ny == 0 is
 * a valid, empty problem: calls return HWENO_OK and enqueue nothing.
 */
#ifndef HWENO_H
#define HWENO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HWENO_OK = 0,
  HWENO_ERR_INVALID_ARG = 1,
  HWENO_ERR_UNSUPPORTED = 2,
  HWENO_ERR_WORKSPACE = 3,
  HWENO_ERR_LAUNCH = 4
} hweno_status;

typedef enum { HWENO_F32 = 0, HWENO_F64 = 1 } hweno_dtype;
typedef enum { HWENO_LINADV = 0, HWENO_BURGERS = 1, HWENO_EULER = 2 } hweno_physics;
typedef enum {
  HWENO_BC_PERIODIC = 0,
  HWENO_BC_OUTFLOW = 1,
  HWENO_BC_REFLECT = 2,
  HWENO_BC_EDGES = 3
} hweno_bc;

/* Segment kinds of an edge-described side (HWENO_BC_EDGES). */
typedef enum { HWENO_SEG_OUTFLOW = 0, HWENO_SEG_REFLECT = 1, HWENO_SEG_STATE = 2 } hweno_seg;

/* One side of the domain under HWENO_BC_EDGES (the boundaries of the double
 * Mach reflection problem, Example 3.11: an inflow stretch followed by a
 * wall on the bottom, the exact motion of an oblique shock on the top).
 * The side is cut in two segments at the position, measured along the side
 * from the domain's low corner (cell centres at (i + 1/2) dx, (j + 1/2) dy),
 *     split = split[0] + split[1] * t + split[2] * d,
 * where t is the time of the state being read and d the distance of the
 * ghost cell's centre beyond the side ((k - 1/2) h for ghost layer k = 1, 2).
 * Ghost cells before the split take segment 0, the others segment 1:
 *   HWENO_SEG_OUTFLOW  copy of the nearest interior cell (all fields);
 *   HWENO_SEG_REFLECT  solid wall, as HWENO_BC_REFLECT;
 *   HWENO_SEG_STATE    the conserved state `state[s]` (rho, rho u, rho v, E)
 *                      with every derivative field zero (an inflow).
 * A side may not combine OUTFLOW with REFLECT. */
typedef struct {
  int32_t kind[2];
  double split[3];
  double state[2][4];
} hweno_edge;

/* Problem description (host memory, read during the call only).
 *  dim            1 or 2.
 *  nx, ny         cells per direction (ny must be 1 when dim == 1); >= 0.
 *  physics        hweno_physics: u_t + f(u)_x [+ g(u)_y] = 0 with
 *                 f = a_x u, g = a_y u (LINADV), f = g = u^2/2 (BURGERS), or
 *                 the Euler equations with E = p/(gamma-1) + rho|vel|^2/2.
 *  dtype          hweno_dtype of every array (FP32 or FP64).
 *  bc_x, bc_y     hweno_bc: periodic wrap; outflow = copy of the nearest
 *                 interior value of every field into the two ghost cells;
 *                 reflect = solid wall: ghost k mirrors interior cell k
 *                 (k = 1, 2 from the wall) with the wall-normal momentum and
 *                 every derivative across the wall negated (signs multiply:
 *                 the normal derivative of the normal momentum is kept).
 *                 Euler only (HWENO_ERR_UNSUPPORTED for scalar laws, which
 *                 have no mirror symmetry with the same flux); at least 2
 *                 cells across the wall's direction.
 *                 edges = each side of the direction described by `edges`
 *                 (2D Euler, single-grid forward entry points only: the
 *                 batched and adjoint entry points return
 *                 HWENO_ERR_UNSUPPORTED).
 *  characteristic Euler only: 1 = nonlinear flux reconstruction in local
 *                 characteristic fields (Remarks 2.1/2.2; Roe average),
 *                 0 = component by component.  Ignored for scalars.
 *  limiter_on     1 = HWENO limiter on the derivatives in the time update
 *                 (Section 2.2), 0 = no limiter (ablation of Table 5).
 *  limiter_characteristic
 *                 Euler only, 0 or 1: 0 = the limiter acts component by
 *                 component on the conserved variables; 1 = a variant (the
 *                 paper does not say how its limiter treats systems): the
 *                 stencil of each cell is projected on the characteristic
 *                 fields of the cell's own state, limited field by field and
 *                 mapped back (the adjoint entry points differentiate
 *                 it too).  Ignored for scalars.
 *  dx, dy         cell sizes (> 0; dy ignored in 1D).
 *  gamma_gas      ratio of specific heats (> 1; Euler only).
 *  adv_speed      (a_x, a_y) for LINADV.
 *  lin_w          gamma_0..2 of the reconstruction; lim_w: d_0..2 of the
 *                 limiter.  Each must be > 0 and sum to 1 within 1e-12.
 *  eps            epsilon of the nonlinear weights (> 0; paper: 1e-6).
 *  cfl            CFL number for the device-side time step (> 0; paper: 0.6).
 *  edges          sides x_lo, x_hi, y_lo, y_hi, read when that direction's
 *                 bc is HWENO_BC_EDGES.  The stages of hweno_rk3_step(s)
 *                 read them at their own times t_n, t_n + dt, t_n + dt/2
 *                 (t_n = simulated time in the control block);
 *                 hweno_rhs and hweno_limit read them at t = 0.
 *  obstacle       {i_s, j_s}: the cells i >= i_s, j < j_s are solid (the
 *                 step of Example 3.12, against the bottom-right corner),
 *                 {0, 0} = none.  Needs bc_x == HWENO_BC_EDGES, 2 <= i_s <= nx
 *                 and 1 <= j_s <= ny - 2.  Its faces x = i_s dx and
 *                 y = j_s dy are walls: along x a solid cell holds the mirror
 *                 image of the fluid across the front face, along y the
 *                 mirror image across the top face (each with the wall
 *                 signs).  Solid cells keep their values, enter no wave speed
 *                 and have a zero right-hand side; the limiter leaves their
 *                 derivatives as they are.
 */
typedef struct {
  int32_t dim, nx, ny;
  int32_t physics, dtype, bc_x, bc_y;
  int32_t characteristic, limiter_on;
  int32_t limiter_characteristic;
  double dx, dy;
  double gamma_gas;
  double adv_speed[2];
  double lin_w[3], lim_w[3];
  double eps, cfl;
  hweno_edge edges[4];
  int32_t obstacle[2];
} hweno_problem;

/* Step control block: HWENO_CTRL_LEN doubles of device memory at the start of
 * the workspace (and the layout of one tape record).
 *   [0..1] alpha_x, alpha_y of stage 1 (global Lax-Friedrichs speeds of U^n)
 *   [2..3] alpha of stage 2, [4..5] alpha of stage 3
 *   [6]    dt of the last step (0 when the step was skipped)
 *   [7]    simulated time t (accumulates over steps; caller sets the start)
 *   [8]    status word (uint64 bit pattern): bit 0 non-finite value produced,
 *          bit 1 rho <= 0, bit 2 p <= 0, bit 3 step skipped (non-finite or
 *          non-positive dt).  Bits accumulate until the caller clears them.
 *   [9]    number of steps taken
 * Wave speeds are stored as IEEE doubles and reduced with an integer atomic
 * max on their bit pattern (exact, order independent; NaN propagates). */
#define HWENO_CTRL_LEN 16
#define HWENO_ST_NONFINITE 1u
#define HWENO_ST_RHO 2u
#define HWENO_ST_PRESSURE 4u
#define HWENO_ST_SKIPPED 8u

/* Host-side validation of a problem (no HIP call).  Returns HWENO_OK, or
 * HWENO_ERR_INVALID_ARG / HWENO_ERR_UNSUPPORTED (reflecting walls for a scalar
 * law) with hweno_last_error() set. */
hweno_status hweno_validate(const hweno_problem* prob);

/* Bytes of device workspace hweno_rk3_step needs for `prob`
 * (control block, two stage states and the limited base derivatives).
 * Returns 0 for an invalid problem. */
size_t hweno_workspace_bytes(const hweno_problem* prob);

/* Global Lax-Friedrichs speeds alpha_d = max over the grid of |f_d'(u)|
 * (Section 2.1; Euler: |u_d| + c).  alpha: device double[2], overwritten
 * (alpha[1] = 0 in 1D). */
hweno_status hweno_alpha(const hweno_problem* prob, const void* state,
                         double* alpha, void* stream);

/* Semi-discrete right-hand side (eqs. odeH and ode2H):
 *   rhs = (L_U, L_Ux[, L_Uy]) in the state layout, with the flux f-hat from
 *   the nonlinear HWENO reconstruction (Section 2.1), h-hat / theta-hat from
 *   p_0' and the mixed eta-hat / xi-hat from the four-point formula (eq. mixed).
 * alpha: device double[2]; if compute_alpha != 0 it is first overwritten with
 *   the speeds of `state` (as hweno_alpha), else it is read as given.
 * state, rhs: device, nf * ny * nx values; must not overlap. */
hweno_status hweno_rhs(const hweno_problem* prob, const void* state, void* rhs,
                       double* alpha, int32_t compute_alpha, void* stream);

/* HWENO limiter (Section 2.2), component by component on the conserved
 * variables, or on the characteristic fields of each cell when the problem's
 * limiter_characteristic is set (Euler):
 *   dlim = (U_x limited along x [, U_y limited along y]), m * dim fields in
 *   the state layout.  The centre derivative is not an input of the limiter. */
hweno_status hweno_limit(const hweno_problem* prob, const void* state,
                         void* dlim, void* stream);

/* One SSP-RK3 step (Section 2.2, eqs. for u^(1), u^(2), u^(n+1)), in place:
 *   S1 = S^ + dt L(S0); S2 = 3/4 S^ + 1/4 (S1^ + dt L(S1));
 *   S^{n+1} = 1/3 S^ + 2/3 (S2^ + dt L(S2)), with S^ = (U, limited
 *   derivatives) used in the update only and L always evaluated on the
 *   unlimited state.  Each stage recomputes the wave speeds of its own input.
 * state: device, in/out.
 * ws: device workspace of at least hweno_workspace_bytes(prob) bytes, 256-byte
 *   aligned; its first HWENO_CTRL_LEN doubles are the step control block.
 *   Zero the control block before the first step of a run (t and the status
 *   word accumulate there across calls).
 * dt_fixed: > 0 uses this time step; otherwise dt = cfl dx / alpha_x (1D) or
 *   cfl / (alpha_x/dx + alpha_y/dy) (2D) from the stage-1 speeds, on device.
 * t_end: > 0 clips dt to t_end - t (a step at t >= t_end is skipped).
 * tape: device double[HWENO_CTRL_LEN] or NULL; receives the control block
 *   after the step (speeds of all three stages, dt, t, status).
 * replay: device double[HWENO_CTRL_LEN] or NULL; when given, the stage speeds
 *   [0..5] and dt [6] are taken from it instead of being computed (used to
 *   recompute a taped forward pass exactly). */
hweno_status hweno_rk3_step(const hweno_problem* prob, void* state, void* ws,
                            size_t ws_bytes, double dt_fixed, double t_end,
                            double* tape, const double* replay, void* stream);

/* n_steps consecutive SSP-RK3 steps of `state` in one call, each exactly as
 * hweno_rk3_step with the same dt_fixed and t_end (no replay).  Between the
 * steps of one call nothing else touches the state, so the stage-1 speeds of
 * step k+1 are folded by step k's third stage (which already evaluates every
 * new cell) instead of by a separate pass over the state: the results, the
 * control block and the tapes are bitwise those of n_steps single calls.
 * Uses control-block entries [10..11] as scratch.  tapes: device
 * double[n_steps][HWENO_CTRL_LEN] (one record per step, as `tape` of
 * hweno_rk3_step) or NULL.  n_steps >= 0. */
hweno_status hweno_rk3_steps(const hweno_problem* prob, void* state, void* ws, size_t ws_bytes,
                             int32_t n_steps, double dt_fixed, double t_end, double* tapes,
                             void* stream);

/* Allocation-free variant of hweno_rk3_step, for callers that cannot
 * allocate device memory (code under hipGraph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The step is exactly that of
 * hweno_rk3_step (same kernels, bitwise the same results, control block and
 * tape); only the stage states S1, S2 and the limited base derivatives live
 * in a static device array of the library, HWENO_STATIC_SCRATCH_BYTES per GPU,
 * held by every GPU the library runs on until the process ends.  Nothing is
 * allocated or freed by the call, and nothing must start at zero in that
 * array: every step writes each stage state before reading it.
 * ctrl: device double[HWENO_CTRL_LEN], the step control block (as the first
 *   HWENO_CTRL_LEN doubles of a hweno_rk3_step workspace: zero it before the
 *   first step of a run; t and the status word accumulate there).
 * dt_fixed, t_end, tape, replay, stream: as for hweno_rk3_step.  The stream's
 *   device must be the current device.
 * Size limit: 2 * align256(cells * nf * elem) + align256(cells * m * dim * elem)
 *   bytes must not exceed HWENO_STATIC_SCRATCH_BYTES (64 MiB: 2D Euler up to
 *   262144 cells in FP64, e.g. 512 x 512, and 524288 in FP32); a larger grid
 *   returns HWENO_ERR_WORKSPACE before any HIP call.
 * Concurrency: all calls on one GPU share its array, so calls that overlap in
 *   time on one GPU (other streams, other host threads) race and corrupt
 *   each other's stages; serialise them on one stream. */
#define HWENO_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
hweno_status hweno_rk3_step_static(const hweno_problem* prob, void* state, double* ctrl,
                                   double dt_fixed, double t_end, double* tape,
                                   const double* replay, void* stream);

/* Bytes of device workspace the adjoint entry points need for `prob`
 * (a ghost-padded adjoint buffer and three stage adjoints).  0 if invalid. */
size_t hweno_adjoint_workspace_bytes(const hweno_problem* prob);

/* Vector-Jacobian product of the right-hand side and the limiter with frozen
 * wave speeds (discrete adjoint of eqs. odeH / ode2H with the reconstruction
 * of Section 2.1, and of the limiter of Section 2.2):
 *   lam_state += (dL/dS)^T lam_rhs + (dLim/dS)^T lam_lim
 * evaluated at `state`.  The absolute values in tau are differentiated as
 * sign(x) with sign(0) = 0; ghost cells are differentiated through the
 * boundary index maps (periodic wrap, outflow copy, reflection with the
 * wall's sign flips).
 * alpha: device double[2], the speeds of the forward evaluation (replayed).
 * lam_rhs: nf fields; lam_lim: m * dim fields (limited-derivative layout of
 * hweno_limit) or NULL; lam_state: nf fields, accumulated into.  lam_state
 * may overlap lam_rhs or lam_lim (the result is folded in a separate pass).
 * ws: device workspace of >= hweno_adjoint_workspace_bytes(prob) bytes. */
hweno_status hweno_rhs_adjoint(const hweno_problem* prob, const void* state,
                               const double* alpha, const void* lam_rhs,
                               const void* lam_lim, void* lam_state, void* ws,
                               size_t ws_bytes, void* stream);

/* Discrete adjoint of one hweno_rk3_step taken with `tape` (speeds of the
 * three stages and dt held fixed):
 *   lam <- (d S^{n+1} / d S^n)^T lam        (in place)
 * state0: S^n, the step's input; step_ws: the workspace of a forward step
 * from state0 taken with that tape (it holds the stage states S1, S2 until
 * the next step on it); tape: device double[HWENO_CTRL_LEN] (as written by
 * hweno_rk3_step); ws: >= hweno_adjoint_workspace_bytes(prob) bytes.
 * lam, state0, step_ws and ws must not overlap (2D grids finish most cells
 * of each stage's adjoint in the kernel that reads the stage's inputs). */
hweno_status hweno_rk3_step_adjoint(const hweno_problem* prob, const void* state0,
                                    const void* step_ws, size_t step_ws_bytes,
                                    const double* tape, void* lam, void* ws,
                                    size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Batched 2D Euler: many independent grids advanced by one persistent launch
 * per Runge-Kutta stage (the same stage computation as hweno_rk3_step, per
 * instance: own speeds, own dt, own boundary conditions).
 *
 * Descriptor of one instance.  Fields marked (caller) are set by the caller
 * before hweno_batch_prepare; fields marked (prepare) are filled by it.  The
 * kernels read an array of these from DEVICE memory (the caller copies the
 * host array there after filling state/ws pointers).
 * --------------------------------------------------------------------------- */
#define HWENO_BATCH_VARIANTS 2   /* tile shapes: 0 = 16 x 15 cells, 1 = 32 x 7 cells */
typedef struct {
  void* state;             /* (caller) device state of this instance, [12][ny][nx]  */
  void* ws;                /* (caller) device workspace, >= ws_bytes, 256-B aligned */
  int32_t nx, ny;          /* (caller) grid, each >= 1                              */
  int32_t bc_x, bc_y;      /* (caller) hweno_bc                                     */
  double dx, dy;           /* (caller) cell sizes                                   */
  double dt_fixed, t_end;  /* (caller) as in hweno_rk3_step                         */
  int64_t ws_bytes;        /* (prepare) workspace bytes this instance needs          */
  int64_t off_s1, off_s2, off_base;            /* (prepare) workspace layout        */
  int32_t tile_begin[HWENO_BATCH_VARIANTS];    /* (prepare) first global tile index */
  int32_t n_tiles[HWENO_BATCH_VARIANTS];       /* (prepare) tiles of this instance  */
} hweno_instance;

/* Host only: validates every instance against `common` (dim must be 2,
 * physics Euler; nx, ny, bc, dx, dy, dt_fixed, t_end taken from the instance),
 * fills the (prepare) fields and writes the total tile count of each variant
 * to total_tiles[HWENO_BATCH_VARIANTS].  The control block at the start of
 * every workspace follows the hweno_rk3_step rules (zero it before the first
 * step). */
hweno_status hweno_batch_prepare(const hweno_problem* common, hweno_instance* inst,
                                 int32_t n_inst, int32_t* total_tiles);

/* Host only: fills map[0..total_tiles) with the instance index of every
 * global tile of `variant` (from the prepared tile_begin / n_tiles). */
hweno_status hweno_batch_tile_map(const hweno_instance* inst, int32_t n_inst, int32_t variant,
                                  int32_t* map, int32_t total_tiles);

/* One SSP-RK3 step of every instance: wave speeds, three persistent stage
 * launches striding over the flattened tile list, and the per-instance time
 * update.  Enqueues six kernels and nothing else, so it can be captured in a
 * hipGraph.  inst_dev: device copy of the prepared descriptors; tile_map_dev:
 * device copy of the tile map of `variant`; total_tiles: the prepared count
 * for `variant`; blocks: persistent grid size (0 = up to 8 workgroups per
 * compute unit). */
hweno_status hweno_rk3_step_batched(const hweno_problem* common, const hweno_instance* inst_dev,
                                    const int32_t* tile_map_dev, int32_t n_inst,
                                    int32_t total_tiles, int32_t variant, int32_t blocks,
                                    void* stream);

/* Autotuner of the batched stepper: the tile variant and the persistent grid
 * size of hweno_rk3_step_batched for one batch, chosen by measurement.  For
 * every tile variant (0 = 16 x 15 cells, 1 = 32 x 7 cells) and every grid
 * candidate -- the stage kernel's resident capacity (blocks = 0), 2 and 4
 * workgroups per compute unit, and one workgroup per tile -- it runs one
 * warm-up step and then `trials` steps between two hipEvents on `stream`,
 * and returns the fastest pair in *variant, *blocks (pass them to
 * hweno_rk3_step_batched; *blocks is the workgroup count the fastest
 * candidate launched, the resident capacity resolved, never 0).  The steps are real steps of the instances that
 * inst_dev describes, so give it descriptors of scratch copies (states and
 * workspaces) of the batch to tune; their control blocks follow the usual
 * rules.  tile_maps_dev: host array of HWENO_BATCH_VARIANTS device tile maps;
 * total_tiles: host int32[HWENO_BATCH_VARIANTS], the prepared tile counts.
 * times_ms (may be NULL): host double[HWENO_BATCH_VARIANTS *
 * HWENO_AUTOTUNE_CANDIDATES], the mean step time of each (variant, candidate),
 * variant-major; grid_sizes (may be NULL): host int32[same], the workgroups
 * each candidate launched.  Unlike the other entry points this one
 * synchronises on its events (and creates and destroys two of them); it
 * allocates no device memory, and the stage timer does not see its launches.
 * trials in [1, 1000]. */
#define HWENO_AUTOTUNE_CANDIDATES 4
hweno_status hweno_autotune(const hweno_problem* common, const hweno_instance* inst_dev,
                            const int32_t* const* tile_maps_dev, int32_t n_inst,
                            const int32_t* total_tiles, int32_t trials, void* stream,
                            int32_t* variant, int32_t* blocks, double* times_ms,
                            int32_t* grid_sizes);

/* Diagnostics: kernel timing of the Runge-Kutta stage kernels.
 * hweno_timing_begin(1) makes subsequent hweno_rk3_step calls (on this
 * thread) record a hipEvent pair around every stage-kernel launch on the
 * call's stream; hweno_timing_end() synchronises on the recorded events, adds
 * up the elapsed times and returns the number of timed launches and their
 * total duration in milliseconds (either pointer may be NULL), then stops
 * timing and releases the events.  hweno_timing_begin(0) stops without
 * reporting.  Timing adds two event records per stage launch. */
hweno_status hweno_timing_begin(int32_t enable);
hweno_status hweno_timing_end(int64_t* launches, double* total_ms);

/* Human-readable name of a status code (static string). */
const char* hweno_status_string(int32_t status);

/* Thread-local detail of the last non-OK return on this thread ("" if none). */
const char* hweno_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HWENO_H */
