/*
 * mmk - micro-step library for the microscale kinetic theory of a gliding motility assay
 * (S. Cook and T. Shinar, "Enabling Simulation of High-Dimensional Micro-Macro Biophysical
 * Models through Hybrid CPU and Multi-GPU Parallelism").  MI355X (gfx950), HIP.
 *
 * One micro-step, at every configuration point (x, y, th) of a periodic nx x ny box with
 * ntheta orientations and ns arclength cells per filament:
 *   1. bound-motor density M(s) walks towards the plus end at speed v0, attaches at k_on and
 *      detaches at k_off M (Sec. 2, Eq. (4)), superbee-limited flux (Sec. 2), two-stage
 *      midpoint Runge-Kutta (Sec. 3.1, Alg. 2);
 *   2. s-moments m0 = sum M ds and m1 = sum (s - L/2) M ds (Eq. (5) reduced to one filament);
 *   3. conservative donor-cell update of the filament density Psi(x, y, th) with velocity
 *      u - F m0 p and rotation rate p_perp . grad(u) . p (Sec. 2, Eqs. (1)-(3));
 *   4. on the last micro-step of a call: theta-moments of Psi and the extra stress
 *      sigma = sigma_f (D - c I / 2) + F sum Psi m1 p p dth (extra-stress step of Alg. 1).
 *
 * Conventions for every function below:
 *  - Arrays are DEVICE pointers on the context's device, C-contiguous, in the context's
 *    precision (double for MMK_FP64, float for MMK_FP32), with layouts
 *      psi [nx][ny][ntheta], M [nx][ny][ntheta][ns] (s fastest),
 *      u [2][nx][ny] = (u_x, u_y), gradu [4][nx][ny] = (dux/dx, dux/dy, duy/dx, duy/dy),
 *      sigma [3][nx][ny] = (xx, xy, yy), moments [7][nx][ny] = (c, n_x, n_y, Dxx, Dxy, Dyy, B),
 *      m0 / m1 [nx][ny][ntheta].
 *    Host arguments are marked "host".
 *  - The caller owns every buffer it passes, including the workspace.  The library never
 *    allocates device memory; it only reads and writes inside the workspace and the
 *    arguments during calls.  Input pointers are not retained after a call returns.
 *  - All device work is ordered on the HIP stream given to mmk_create.  Functions return
 *    once the work is enqueued, except those marked "synchronizes".
 *  - Every function returns an mmk_status and never aborts; mmk_last_error() gives the text.
 *    A context is not thread-safe; separate contexts are independent.
 */
#ifndef MMK_H
#define MMK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mmk_ctx mmk_ctx;

typedef enum {
    MMK_OK = 0,
    MMK_ERR_ARG = -1,          /* bad sizes, null pointers, non-finite or <= 0 dt, ... */
    MMK_ERR_NOMEM = -2,        /* workspace smaller than mmk_workspace_bytes() */
    MMK_ERR_HIP = -3,          /* a HIP runtime call failed (message says which) */
    MMK_ERR_STATE = -4,        /* call order: step before set_state/set_fluid, ... */
    MMK_ERR_UNSUPPORTED = -5   /* sizes the kernels are not built for */
} mmk_status;

typedef enum { MMK_FP64 = 0, MMK_FP32 = 1 } mmk_precision;
typedef enum { MMK_SUPERBEE = 0, MMK_UPWIND1 = 1 } mmk_limiter;

typedef struct {
    int32_t nx, ny;        /* periodic grid, >= 1 each */
    int32_t ntheta;        /* orientations th_k = 2 pi k / ntheta, 1 .. 4096 */
    int32_t ns;            /* arclength cells s_l = (l + 1/2) L / ns, 1 .. 512 */
    double lx, ly;         /* box size (> 0) */
    double L;              /* filament length (> 0) */
    double k_on, k_off;    /* attachment rate (per free motor) and detachment rate */
    double v0;             /* motor walking speed along +s, >= 0 */
    double F;              /* motor force coefficient: gliding speed F m0 along -p */
    double sigma_f;        /* filament extra-stress coefficient */
    int32_t precision;     /* mmk_precision: storage AND arithmetic of every field */
    int32_t limiter;       /* mmk_limiter; MMK_UPWIND1 sets the superbee slope to 0 */
    double m_total;        /* total motors per unit area, >= 0.  0: the free-motor pool is 1
                            * everywhere (linear attachment).  > 0: free-motor depletion
                            * (Eqs. (5)-(6)) and the over-binding clamp of Alg. 2: each
                            * micro-step starts from B(x, y) = sum_th psi m0 dth of the
                            * current state; where B > m_total every motor column at (x, y)
                            * is scaled by m_total / B and none attach, elsewhere they
                            * attach at rate k_on (m_total - B).  Not supported by the tape. */
    double motor_cfl;      /* >= 0.  0: one motor step per micro-step.  > 0: the motor step
                            * sub-cycles (Alg. 2, local dt*): a micro-step of length dt
                            * advances M by n = ceil(dt (v0 / ds + k_off) / motor_cfl)
                            * steps of dt / n inside one launch (M is read and written once),
                            * the s-moments taken after the last; n <= 4096.  The stability
                            * limit is the same at every point here, so one n serves all.
                            * With m_total > 0 each sub-step is preceded by the clamp and the
                            * free pool of the current sub-state (Alg. 2 clamps inside its
                            * inner loop), psi held at its start-of-step value: all sub-steps
                            * in one launch with one block per (x, y) point where the column
                            * tiling allows it (FP32 ns = 32, 64, 128; FP64 ns = 16, 32, 64;
                            * ntheta times the lanes per column a multiple of 64, at most
                            * 1024), else one launch per sub-step.  Not supported by the
                            * tape. */
    double rc;             /* >= 0.  0: the anchor-marginal model above.  > 0: anchor-resolved
                            * bound motors M_b(r0, x, th, s) (Sec. 2, Eqs. (4)-(6), Alg. 2) with
                            * capture radius rc; needs rc + L/2 < lx/2 and < ly/2 (else
                            * MMK_ERR_ARG).  Anchors r0 sit on the cell centres; the tracked
                            * cells are listed by mmk_r0_cells.  M (set_state / get_state) is
                            * then Mb [ncell][nx][ny]: cell c = (a, b, k, l) of the filament
                            * centred at cell (i, j) with angle th_k, arclength cell l, bound to
                            * the anchor at cell (i - a, j - b) (periodic).  Along a filament the
                            * tracked cells form runs; each run walks as its own column (no
                            * influx at its first cell, free outflow at its last: motors leave
                            * the capture ball).  The attachment source of a run is k_on times
                            * its anchor's free pool: 1 with m_total = 0, else m_total minus the
                            * anchor's coarse density coarse(r0) = sum over its tracked cells of
                            * M_b psi ds dx dy dth, with the clamp of Alg. 2 per anchor at the
                            * start of each micro-step (where coarse > m_total the anchor's cells
                            * are scaled by m_total / coarse and the pool is 0).  Psi is driven by,
                            * and m0 / m1 / the moments report, the anchor marginals
                            * m0(x, th) = sum over anchors and s of M_b ds dx dy (m1 with the lever
                            * arm s - L/2); mmk_get_force spreads the anchor-marginal field
                            * sum over anchors of M_b dx dy.  With motor_cfl > 0 the runs
                            * sub-cycle as above, n steps of dt / n, and with m_total > 0 every
                            * sub-step starts with the clamp and the pool of the current
                            * sub-state (psi of the step's start).  Runs longer than 32 cells
                            * and the tape give MMK_ERR_UNSUPPORTED.  Launches per micro-step:
                            * n (coarse + pool, motor) + 1 (psi) with m_total > 0, n + 1 with
                            * m_total = 0. */
} mmk_params;

/* Tracked cells of the anchor-resolved model (p->rc > 0), host: returns their number ncell
 * (0 is possible for a tiny rc) and, when cells is not NULL, writes cells[4 c + 0..3] =
 * (a, b, k, l) for c < ncell in lexicographic order of (a, b, k, l).  The motor point of the
 * cell, relative to its anchor, is (a lx/nx, b ly/ny) + ((l + 1/2) L/ns - L/2) p_k, and the cell
 * is tracked when its squared length (FP64, in that order) is at most rc^2.  Returns -1 on
 * invalid params or an unusable rc (<= 0, or rc + L/2 not below lx/2 and ly/2). */
int64_t mmk_r0_cells(const mmk_params *p, int32_t *cells);

/* Bytes of device workspace a context needs (the fields of one micro-step, Sec. 3.1: the whole
 * state stays resident on the device between steps).  ckpt_every > 0 reserves the adjoint tape:
 * checkpoints of (Psi, M) every ckpt_every steps for up to max_tape_steps taped steps, a
 * ckpt_every-step recompute buffer, adjoint fields and one fluid slot per taped step.
 * ckpt_every = 0 (max_tape_steps ignored) gives the forward-only size.  Returns 0 on
 * invalid params. */
size_t mmk_workspace_bytes(const mmk_params *p, int32_t ckpt_every, int32_t max_tape_steps);

/* Creates a context on the current HIP device: the grid and model of Sec. 2 (Eqs. (1)-(6))
 * with the discretisation of its Sec. 3.1 (uniform theta and s, superbee, two-stage RK).
 * workspace: device pointer, 256-byte aligned, ws_bytes >= mmk_workspace_bytes(p, ckpt_every,
 * max_tape_steps); the caller keeps it alive until mmk_destroy.  hip_stream: a hipStream_t
 * (NULL = the null stream).  *out receives the context (host memory owned by the library,
 * freed by mmk_destroy).  Fills the angle tables in the workspace and synchronizes once.
 * MMK_ERR_ARG: invalid params, NULL or misaligned workspace; MMK_ERR_NOMEM: ws_bytes too small;
 * MMK_ERR_UNSUPPORTED: sizes beyond the kernels (message says which). */
mmk_status mmk_create(const mmk_params *p, void *workspace, size_t ws_bytes, void *hip_stream,
                      int32_t ckpt_every, int32_t max_tape_steps, mmk_ctx **out);
mmk_status mmk_destroy(mmk_ctx *ctx);

/* Replaces the rates of Eq. (4), k_on, k_off, and the walking speed v0 (host values) for the
 * following steps (for finite-difference and gradient runs).  MMK_ERR_ARG: non-finite values or
 * v0 < 0; MMK_ERR_STATE: inside a taped run that has steps. */
mmk_status mmk_set_params(mmk_ctx *ctx, double k_on, double k_off, double v0);

/* Copies the state in (device to device, stream-ordered; the sources may be freed once the
 * stream has passed the call): the filament density psi [nx][ny][ntheta] of Eq. (1) and the
 * bound-motor density M [nx][ny][ntheta][ns] of Eq. (4), or NULL for M = 0.  Drops the outputs
 * of earlier steps.  MMK_ERR_ARG: psi NULL; MMK_ERR_STATE: during a taped run. */
mmk_status mmk_set_state(mmk_ctx *ctx, const void *psi, const void *M);

/* Copies the fluid velocity u [2][nx][ny] and its gradient gradu [4][nx][ny] in (device to
 * device, stream-ordered); they act on every following micro-step until replaced.  This is the
 * exchange with the macroscale Stokes solve of Eqs. (7)-(9) in Alg. 1: the velocity enters the
 * translational velocity of Eq. (2), its gradient the rotation rate of Eq. (3).  Recorded by an
 * active tape.  MMK_ERR_ARG: NULL pointer. */
mmk_status mmk_set_fluid(mmk_ctx *ctx, const void *u, const void *gradu);

/* Runs K >= 0 micro-steps of size dt (finite, > 0), each the bound-motor update of Eq. (4)
 * (Alg. 2: two-stage RK per column, with the clamp and the free pool of Eqs. (5)-(6) under
 * m_total > 0, sub-cycled under motor_cfl > 0) followed by the conservative update of psi,
 * Eq. (1), with the velocities of Eqs. (2)-(3) driven by the new m0.  The last micro-step also
 * forms the theta-moments and the extra stress (the stress step of Alg. 1) and the FP64 global
 * sums.  No host sync.  Launches: for the linear model one motor launch per up to 16 micro-steps
 * (MMK_OPT_MOTOR_BLOCK) and one psi launch per micro-step; see mmk_params for the others.
 * MMK_ERR_ARG: K < 0, dt not finite or <= 0, more than 4096 motor sub-steps, or a taped run past
 * max_tape_steps; MMK_ERR_STATE: no state or no fluid set. */
mmk_status mmk_step(mmk_ctx *ctx, int32_t K, double dt);

/* The same K micro-steps as mmk_step, replayed as one HIP graph launch on the context's stream
 * (for launch-bound small grids, where the host's launch overhead exceeds the kernels' time;
 * Sec. 3.1 puts the micro-step loop on the GPU with no host work between steps).  The first call
 * for a (K, dt) from a given state buffer captures the launches mmk_step(K, dt) would enqueue
 * into a graph held by the context (on a capture stream of the library's own; nothing runs
 * during the capture), later calls replay it: the same kernels with the same arguments, so the
 * results are bitwise those of mmk_step.  Fields are read and written in place, so set_state and
 * set_fluid between calls take effect.  mmk_set_params and mmk_set_option drop the captured
 * graphs; at most 8 are held.  Launches are not timed by mmk_profile.  MMK_ERR_STATE during a
 * taped run (use mmk_step); otherwise errors as mmk_step.  No host sync. */
mmk_status mmk_step_graph(mmk_ctx *ctx, int32_t K, double dt);

/* Copies the current state (psi, M as in mmk_set_state) out, device to device, stream-ordered
 * (either pointer may be NULL).  MMK_ERR_STATE: no state set. */
mmk_status mmk_get_state(mmk_ctx *ctx, void *psi, void *M);
/* Outputs of the last micro-step of the last mmk_step with K > 0 (the extra-stress step of
 * Alg. 1, from Psi of Eq. (1) and the s-moments of Eq. (5)): sigma [3][nx][ny] =
 * sigma_f (D - c I/2) + F sum_th psi m1 p p dth, and moments [7][nx][ny] = (c, n_x, n_y, D_xx,
 * D_xy, D_yy, B) with c = sum psi dth, n = sum psi p dth, D = sum psi p p dth and the coarse
 * bound density B = sum psi m0 dth (Eq. (5) reduced to one filament).  Device to device,
 * stream-ordered.  MMK_ERR_ARG: NULL pointer; MMK_ERR_STATE: no step has produced outputs. */
mmk_status mmk_get_stress(mmk_ctx *ctx, void *sigma);
mmk_status mmk_get_moments(mmk_ctx *ctx, void *moments);
/* s-moments of the current M (Eq. (5) per filament, and the lever-arm moment that enters the
 * stress): m0 = sum M ds always, m1 = sum (s - L/2) M ds as of the last step that produced
 * outputs; [nx][ny][ntheta] each, either pointer may be NULL.  MMK_ERR_STATE: no outputs yet. */
mmk_status mmk_get_motor_moments(mmk_ctx *ctx, void *m0, void *m1);
/* Motor force density of the current state (Eq. (10)), force [2][nx][ny] = (f_x, f_y): every
 * bound-motor cell l of a filament at (x_i, y_j) with orientation p_k adds F p_k psi M_l ds dth
 * (with rc > 0, M is the anchor marginal sum over anchors of M_b dx dy, the r0 integral of
 * Eq. (10), formed first; its kernel needs ns * 65 * sizeof(value) <= 160 KB of LDS, else
 * MMK_ERR_UNSUPPORTED)
 * at its head (x_i, y_j) + (s_l - L/2) p_k, spread onto the cell centres with the two-point
 * hat (bilinear) in x and y, periodic.  The filament length L is in the units of lx, ly.
 * Same bits on every run (each spreading window is private to one wave and summed in a fixed
 * order).  Needs state; MMK_ERR_UNSUPPORTED if the filament's reach makes the spreading window
 * ((8 + 2 r)^2 cells for a reach of r = L nx / (2 lx) cells, 8 bytes each, plus 18 KB of
 * staging) larger than the device's LDS per block; windows beyond 3072 cells cost one more
 * read of M per 3072 cells.  Leaves the state as it is (with rc > 0 it may use the second state
 * buffer of the workspace as scratch).  No host sync. */
mmk_status mmk_get_force(mmk_ctx *ctx, void *force);
/* Anchor-resolved model only (rc > 0; else MMK_ERR_STATE): coarse [nx][ny] = the coarse density
 * of Eq. (5) at every anchor of the current state, and free_pool [nx][ny] = its free motors of
 * Eq. (6) before the next step's clamp, m_total - min(coarse, m_total) (1 with m_total = 0).
 * Either pointer may be NULL.  Needs state.  No host sync. */
mmk_status mmk_get_anchors(mmk_ctx *ctx, void *coarse, void *free_pool);
/* Global sums of the last outputs (the total filament count that Eq. (1) conserves, and the
 * domain integral of the extra stress of Alg. 1), host outputs, synchronizes: mass =
 * sum Psi dx dy dth and sum_sigma[c] = sum sigma_c dx dy, accumulated in FP64 (compensated) in a
 * fixed order (bitwise reproducible).  The output psi step of each mmk_step call leaves FP64
 * block partials; their reduction runs here, on the context's stream, the first time the sums
 * of those outputs are asked for.  Either pointer may be NULL.  MMK_ERR_STATE: no outputs. */
mmk_status mmk_get_sums(mmk_ctx *ctx, double *mass, double sum_sigma[3]);

/* Adjoint tape (a project extra: the paper has no adjoint; it differentiates the micro-step of
 * mmk_step).  mmk_tape_begin records the current state as checkpoint 0 and the current
 * fluid; later set_fluid/step calls are recorded (at most max_tape_steps steps).
 * mmk_tape_backward (synchronizes) returns the gradient of
 *     L = <g_sigma, sigma(T)> + <g_moments, moments(T)>
 * (either cotangent may be NULL = 0) with respect to the taped initial Psi (g_psi0, device,
 * [nx][ny][ntheta]) and to k_on, k_off, v0 (g_params, host double[3]).  dt is held fixed.
 * It recomputes each checkpoint segment forward, then runs the hand-written reverse
 * kernels.  The forward state is left as it was.  mmk_tape_end drops the tape. */
mmk_status mmk_tape_begin(mmk_ctx *ctx, int32_t ckpt_every);
mmk_status mmk_tape_backward(mmk_ctx *ctx, const void *g_sigma, const void *g_moments,
                             void *g_psi0, double g_params[3]);
mmk_status mmk_tape_end(mmk_ctx *ctx);

/* Implementation options of a context (project extras, not in the paper).  Each selects
 * between kernels or launch shapes that compute the same micro-step; the defaults are the
 * ones measured fastest on MI355X.  Results under any setting agree with the defaults up to the
 * association of the s- and theta-sums (the lane tiling, the psi kernel) and are bitwise equal
 * where those are the same.  An option may be set at any time between calls and applies from the next call on.
 * MMK_ERR_ARG for an unknown option or a value outside its range.  No device work. */
typedef enum {
    MMK_OPT_MOTOR_BLOCK = 0,   /* 1 (default): with m_total = 0, rc = 0 and no tape, one motor
                                * launch advances M through up to 16 micro-steps of a call (the
                                * column stays in registers; m0 of every micro-step is kept for
                                * its psi step); 0: one motor launch per micro-step */
    MMK_OPT_PSI_KERNEL = 1,    /* 0 (default): the LDS-free walking psi kernel for ntheta = 64
                                * or 128 in FP32, and in FP64 where nx is a multiple of 8 (the
                                * walk with a ring of register sets), the LDS-tiled one
                                * otherwise; 1: LDS-tiled; 2: walking where ntheta allows it,
                                * else LDS-tiled */
    MMK_OPT_DEPL_FUSED = 2,    /* 1 (default): depletion with motor sub-cycling runs all
                                * sub-steps of a micro-step in one launch where the tiling allows
                                * it; 0: one launch per sub-step */
    MMK_OPT_MOTOR_LANES = 3,   /* 0 (default: from ns, the precision and whether a launch takes
                                * several steps per load); else lanes per motor column, a power
                                * of two 2 .. 64; a value without a compiled tiling for ns and the
                                * precision leaves the default */
    MMK_OPT_MOTOR_CHUNKS = 4,  /* 0 (default): each lane holds consecutive cells; 2 or 4: each
                                * lane holds that many 16-byte chunks spaced a lane group apart
                                * (no depletion; a value without a tiling for ns leaves 0) */
    MMK_OPT_MOTOR_NT = 5,      /* -1 (default): in FP32 nontemporal loads and stores of M for a
                                * launch of one step, plain accesses for launches of several
                                * micro-steps or sub-steps; plain in FP64; 0: plain; 1: nontemporal
                                * loads and stores; 2: nontemporal loads only */
    MMK_OPT_PSI_DEPTH = 6,     /* walking psi kernel: pencils of a walk of 8 whose loads are in
                                * flight together, where nx is a multiple of 8 (else always two
                                * alternating register sets); 0 (default): 8 at ntheta = 64, 4
                                * at 128; 2: two alternating sets; 4, 8: a ring of that many
                                * sets (4 at ntheta = 128) */
    MMK_OPT_R0_ONEPASS = 7     /* anchor-resolved model with depletion and motor sub-cycling:
                                * 1 (default): where one anchor's tracked cells fit one block
                                * (1024 threads of 24 register slots in FP32, 16 in FP64), one
                                * launch per micro-step holds each anchor's cells and runs all
                                * its sub-steps, re-forming the clamp before each (the state
                                * is then kept in an anchor-major layout, converted back where
                                * needed); 0: one coarse pass and one motor launch per sub-step */
} mmk_option;
mmk_status mmk_set_option(mmk_ctx *ctx, int32_t option, int32_t value);

/* Kernel timing (a measurement extra, in the spirit of the profiler-driven analysis of
 * Sec. 3.2): with enable = N > 0 every N-th launch of each kernel is bracketed by HIP
 * events on the context's stream (enable = 0 turns timing off, < 0 is MMK_ERR_ARG).
 * mmk_profile_read (synchronizes) sums the elapsed times of the timed launches of `kernel_id`
 * (0 motor step, 1 psi step, 2 global sums, 3 reverse psi step, 4 reverse motor step, 5 motor
 * force: spreading and merge, 6 anchor-resolved motor step, 7 anchor coarse density and pool,
 * 8 anchor-resolved sub-steps of a micro-step with one anchor per block, 9 anchor marginals
 * from its run totals)
 * since profiling was enabled; up to 65536 launches per id are timed. */
mmk_status mmk_profile(mmk_ctx *ctx, int32_t enable);
mmk_status mmk_profile_read(mmk_ctx *ctx, int32_t kernel_id, double *total_ms, int64_t *launches);
/* After mmk_profile: time every `every`-th launch of kernel_id from here on (0: none of them),
 * restarting its count; the other ids keep theirs.  Synchronizes. */
mmk_status mmk_profile_every(mmk_ctx *ctx, int32_t kernel_id, int32_t every);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the global sums of mmk_get_sums computed without a
 * context or a workspace, from caller-given device arrays psi [nx][ny][ntheta] and sigma
 * [3][nx][ny] in the precision p->precision (only nx, ny, ntheta, lx, ly and precision of *p are
 * read): mass = sum psi dx dy dth and sum_sigma[c] = sum sigma_c dx dy (host outputs),
 * accumulated in FP64 (compensated) in a fixed order, bitwise reproducible.  Its block partials
 * live in a static device array of the library (4096 rows of 4 doubles and the 4 totals,
 * 131104 bytes; one copy per device, held until the process ends); nothing is allocated, and
 * every row it reads is written first in the same call.  Calls that overlap on one device race
 * for that array: serialise them (one stream, or host synchronisation).  Work is ordered on
 * hip_stream (NULL = the null stream) and the call synchronizes it.  MMK_ERR_ARG: NULL pointers,
 * sizes < 1, bad precision or box; MMK_ERR_UNSUPPORTED: more than 2^36 psi cells (the scratch
 * holds 4096 partial rows of at most 2^24 cells) or a device index beyond 63; MMK_ERR_HIP: a
 * HIP call failed.  The message is given by mmk_last_error(NULL). */
mmk_status mmk_sums_static(const mmk_params *p, const void *psi, const void *sigma, void *hip_stream,
                           double *mass, double sum_sigma[3]);

/* Message of the last failure on ctx; with ctx == NULL, of the last failed mmk_create,
 * mmk_workspace_bytes or mmk_sums_static on this thread. */
const char *mmk_last_error(const mmk_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
