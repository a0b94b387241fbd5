/*
 * tenom: TENO-M per-face high-order reconstruction on AMD Instinct MI355X
 * (gfx950), after Li, Fu & Adams, "A low-dissipation shock-capturing
 * framework with flexible nonlinear dissipation control" (arXiv 2010.13289).
 *
 * C ABI of libtenom.so.  Plain pointers and sizes only.
 *
 * Data layout (all calls):
 *   - Every array pointer is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *     tensor's storage), FP64, C-contiguous, structure of arrays
 *     [field][z][y][x] with x fastest.  Grids carry no ghost cells: the
 *     boundary rule of each axis (periodic wrap or transmissive clamp,
 *     i.e. zero-gradient ghosts) is applied inside the kernels.
 *   - Fields: scalar system 1 field (u); Euler ndim+2 fields
 *     (rho, rho*u, [rho*v], [rho*w], E), ideal gas with ratio `gamma`.
 *   - Points are cell-centre point values of a finite-difference scheme
 *     (Sec. 2): du_i/dt = -(F_{i+1/2} - F_{i-1/2})/dx along each axis.
 *
 * Ownership: the caller allocates and frees everything.  The library never
 * allocates device memory on the compute path; only tenom_max_wave_speed
 * and tenom_check_finite keep one small (16-byte) device buffer per device,
 * allocated on first use and held until the process ends.  All compute
 * calls enqueue asynchronously on `stream` (a hipStream_t passed as void*;
 * NULL = the default stream) and do not synchronise, except where stated.
 * Calls on different streams are independent; concurrent calls that write
 * the same buffers race.
 *
 * Errors: every int-returning call returns TENOM_OK (0) or a negative code;
 * no call aborts or throws across the ABI.  tenom_last_error() gives a
 * message for the last failure on the calling thread.
 */
#ifndef TENOM_H
#define TENOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ----------------------------------------------------- */
#define TENOM_OK 0
#define TENOM_EINVAL (-1)      /* null pointer, ndim not in {1,2,3}, a used
                                  axis with fewer than K cells, axis >= ndim,
                                  C_T < 0 or NaN (or > 1/(K-2) for classic
                                  TENO), gamma <= 1 (Euler), dt <= 0 or
                                  non-finite, dx <= 0                      */
#define TENOM_EUNSUPPORTED (-2) /* unknown scheme, limiter or system ID     */
#define TENOM_EWORKSPACE (-3)  /* workspace smaller than
                                  tenom_workspace_bytes()                   */
#define TENOM_EHIP (-4)        /* HIP launch or runtime error              */
#define TENOM_ENONFINITE (-5)  /* tenom_check_finite found NaN or Inf      */

/* ---- identifiers -------------------------------------------------------- */
/* Boundary rule per axis. */
#define TENOM_BC_PERIODIC 0
#define TENOM_BC_TRANSMISSIVE 1 /* zero-gradient: cell indices clamped    */

/* Conservation law. */
#define TENOM_SYS_SCALAR 0 /* u_t + a . grad u = 0, a = grid.adv            */
#define TENOM_SYS_EULER 1  /* compressible Euler, ideal gas                 */

/* Scheme: number of points K of the full stencil (Sec. 2.1, Table 1).
 * K = 6: candidates S0..S3 on i-2..i+3; K = 8: S0..S5 on i-3..i+4.  The
 * optimal weights d_k are the maximum-order ones (Sec. 3.3), so with every
 * candidate smooth the scheme is the K-point linear scheme.
 * TENOM_SCHEME_8A is the eight-point scheme with the adaptive cutoff of
 * Sec. 2.4 (Eqs. shock_indicator, cut-off_adjust; xi = 1e-3, C_r = 0.23,
 * alpha_1 = 10.5, alpha_2 = 3.5): each reconstruction takes
 * C_T = 10^-floor(beta) in {1e-7 .. 1e-10} from its own stencil values and
 * the C_T argument of the calls is ignored. */
#define TENOM_SCHEME_6 6
#define TENOM_SCHEME_8 8
#define TENOM_SCHEME_ADAPTIVE 0x100
#define TENOM_SCHEME_8A (TENOM_SCHEME_8 | TENOM_SCHEME_ADAPTIVE)

/* Filter applied to the candidates the cutoff marks nonsmooth (Sec. 3.2,
 * Eq. mp_flux).  MP: Suresh-Huynh bounds with alpha = 1.25 and the given
 * curvature measure and beta (Eqs. upper_limiter .. value_monotonicity_
 * preserving), computed once per face and applied to each nonsmooth
 * candidate.  TVD-type: one limited flux on the fixed stencil centred at i
 * replaces every nonsmooth candidate (Sec. 3.2.3). */
#define TENOM_LIM_TENO 0       /* none: classic TENO, nonsmooth candidates
                                  dropped and the weights renormalised
                                  (Eq. weight_renormalize); needs
                                  C_T <= 1/(K-2)                           */
#define TENOM_LIM_MP 1         /* MP, d^M4, beta = 4 (the paper's default) */
#define TENOM_LIM_TVD_MINMOD 2 /* f_i + minmod(f_i - f_{i-1}, f_{i+1} - f_i)/2 */
#define TENOM_LIM_TVD5 3       /* Kim & Kim fifth-order TVD, alpha = 2      */
#define TENOM_LIM_VA 4         /* Van Albada, kappa = 1/3 (Eq. vAflux)     */
#define TENOM_LIM_MP_M4_B2 5   /* MP, d^M4, beta = 2 (Sec. 4.2.5)          */
#define TENOM_LIM_MP_MM_B4 6   /* MP, d^MM (Eq. maximal_curvature1), beta 4 */
#define TENOM_LIM_MP_MM_B2 7   /* MP, d^MM, beta = 2 (Sec. 4.2.5)          */
#define TENOM_LIM_MP_MM_B1 8   /* MP, d^MM, beta = 1 (Sec. 4.4)            */

/* ---- grid descriptor ---------------------------------------------------- */
typedef struct tenom_grid {
    int32_t ndim;   /* 1, 2 or 3                                            */
    int32_t n[3];   /* cells along x, y, z (entries >= ndim are ignored)     */
    double dx[3];   /* cell size along x, y, z (> 0 for used axes)           */
    int32_t bc[3];  /* TENOM_BC_* per axis                                   */
    int32_t system; /* TENOM_SYS_*                                           */
    double adv[3];  /* advection velocity (scalar system only)               */
} tenom_grid;

/* Number of fields of the grid's system (1, or ndim + 2), 0 if invalid. */
int tenom_num_fields(const tenom_grid* grid);

/* ---- compute calls ------------------------------------------------------ */

/*
 * Numerical fluxes at every face of one axis (Sec. 2-3 and 4).
 *
 * For each face i+1/2 the K cells i-K/2+1 .. i+K/2 along `axis` are read;
 * for the Euler system they are projected on the left eigenvectors of the
 * flux Jacobian at the Roe average of cells i and i+1 and split by the
 * Rusanov (local Lax-Friedrichs) rule f+- = (F +- alpha U)/2, alpha = the
 * largest |u_n| + c over the K cells (scalar system: f = a u, alpha = |a|).
 * Each split component is reconstructed by TENO-M: candidate fluxes
 * (Table 1), smoothness indicators and tau_K (Eqs. measureTENO, taukTENO),
 * the sharp cutoff chi_k < C_T -> nonsmooth (Eqs. normalize, cut-off), the
 * limiter on the nonsmooth candidates (Eq. mp_flux) and assembly with the
 * optimal weights, no renormalisation (Eq. reconstuction).  The f- side is
 * the mirror image about the face.  The two sides are summed and projected
 * back with the right eigenvectors.
 *
 *   U     : [nf][z][y][x] input state (device).
 *   Fhat  : [nf][...] output with the `axis` extent n_axis + 1; face j lies
 *           between cells j-1 and j (for periodic axes face n_axis equals
 *           face 0 and both are written).
 *   flags : nullable; [2][nf][faces] uint8 (side 0 = f+, 1 = f-), bit k set
 *           iff candidate S_k was classified smooth (delta_k = 1).
 *   C_T   : cutoff, >= 0 (C_T = 0 makes every candidate smooth).
 *   gamma : ratio of specific heats (> 1; ignored by the scalar system).
 */
int tenom_reconstruct_faces(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma,
                            int axis, const double* U, double* Fhat, uint8_t* flags, void* stream);

/*
 * Semi-discrete right-hand side (Eq. approximateEq, dimension by dimension):
 *   dUdt = -sum_axis (Fhat_{i+1/2} - Fhat_{i-1/2}) / dx_axis
 * accumulated in the axis order x, y, z.  Needs no workspace.
 *   U    : [nf][z][y][x] input (device);  dUdt : same shape, output.
 */
int tenom_flux_divergence(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma,
                          const double* U, double* dUdt, void* stream);

/*
 * One third-order SSP Runge-Kutta step of size dt, in place (Sec. 4, after
 * Gottlieb & Shu):
 *   U1 = U + dt L(U);  U2 = 3/4 U + 1/4 (U1 + dt L(U1));
 *   U <- 1/3 U + 2/3 (U2 + dt L(U2)),
 * with L = tenom_flux_divergence.  The stage states and the right-hand-side
 * accumulator live in the caller's workspace `ws` (device memory of at
 * least tenom_workspace_bytes(grid, scheme) bytes, 256-byte aligned).
 */
int tenom_rk3_step(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                   double* U, void* ws, size_t ws_bytes, void* stream);

/*
 * tenom_rk3_step that also writes its stage states: U1 = U + dt L(U) and
 * U2 = 3/4 U + 1/4 (U1 + dt L(U1)) into the caller's device arrays U1, U2
 * (the state's shape, distinct from U and from each other), e.g. to hand
 * them to tenom_rk3_step_vjp_stages.  Same workspace as tenom_rk3_step;
 * the same kernels, so U is updated to the same bits.
 */
int tenom_rk3_step_stages(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                          double* U, double* U1, double* U2, void* ws, size_t ws_bytes, void* stream);

/*
 * One SSP-RK3 step whose size comes from the CFL condition on the device
 * (Sec. 4): dt = cfl / R with R = max_cells sum_d (|u_d| + c) / dx_d (scalar
 * system: sum_d |a_d| / dx_d), the rate tenom_max_wave_speed returns; then
 * the step of tenom_rk3_step with that dt, to the same bits.  Nothing is
 * synchronised, copied to the host or allocated, so the call can be captured
 * in a HIP graph and replayed.
 *   cfl    : CFL number, finite and > 0 (else TENOM_EINVAL).
 *   ws     : the workspace of tenom_rk3_step (tenom_workspace_bytes; its
 *            tail holds the per-block maxima of R and dt).
 *   dt_out : device address that receives the dt used, or NULL.
 * A state whose R is NaN, zero or infinite gives a non-finite dt, and the
 * step then writes non-finite values (tenom_check_finite finds them).
 */
int tenom_rk3_step_cfl(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double cfl,
                       double* U, void* ws, size_t ws_bytes, double* dt_out, void* stream);

/* Workspace bytes tenom_rk3_step, tenom_rk3_step_stages and tenom_rk3_step_cfl
 * need for this grid (0 if invalid). */
size_t tenom_workspace_bytes(const tenom_grid* grid, int scheme);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step
 * of tenom_rk3_step_cfl, same kernels and the same bits, with its scratch
 * (divergence accumulator, stage states, per-block rate maxima and dt) in a
 * library-held static device array of TENOM_STATIC_SCRATCH_BYTES instead of
 * a caller workspace.  The caller still passes U (in/out) and dt_out.
 *   - Grids whose tenom_workspace_bytes exceeds TENOM_STATIC_SCRATCH_BYTES
 *     are rejected with TENOM_EWORKSPACE (128 MiB holds a 2D Euler grid of
 *     1024^2 or a 3D one of 100^3).
 *   - Each device the call runs on holds its own copy of the array from the
 *     first call on that device until the process ends; the call looks its
 *     address up once per device (nothing is allocated by the call itself).
 *   - Every call on one device shares that device's array, and the array
 *     keeps the last call's contents; each step writes every part it reads
 *     first, so nothing needs clearing.  Calls that overlap on one device
 *     (other streams, other threads) race on the array.
 * Errors as tenom_rk3_step_cfl.
 */
#define TENOM_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
size_t tenom_static_scratch_bytes(void);
int tenom_rk3_step_cfl_noalloc(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma,
                               double cfl, double* U, double* dt_out, void* stream);

/*
 * Largest signal rate over the cells: max_cells sum_d (|u_d| + c) / dx_d
 * (scalar system: sum_d |a_d| / dx_d).  A step at CFL number sigma is
 * dt = sigma / *out_host.  Synchronises `stream`; a NaN in U yields NaN.
 */
int tenom_max_wave_speed(const tenom_grid* grid, double gamma, const double* U, double* out_host,
                         void* stream);

/* TENOM_OK if every value of U is finite, else TENOM_ENONFINITE.
 * Synchronises `stream`. */
int tenom_check_finite(const tenom_grid* grid, const double* U, void* stream);

/* ---- adjoint ------------------------------------------------------------- */
/*
 * Vector-Jacobian products of the flux divergence and of one SSP-RK3 step,
 * for gradients through rollouts (loss functions of the final state).
 * Each is the exact derivative of the forward map with every
 * piecewise choice frozen at the state it is evaluated on:
 *   - the smoothness decisions delta_k (the cutoff, Eq. cut-off; adaptive
 *     C_T of Sec. 2.4);
 *   - the limiter branches (min/max, minmod and median selections of
 *     Secs. 3.2.1-3.2.2);
 *   - the cell attaining the Rusanov alpha.
 * With these frozen, the reconstruction with optimal weights (Eq.
 * reconstuction) is linear in the split fluxes.  Van Albada's slope function
 * (Eq. van_Albada_limiter) is differentiated as it stands.  Ties go to the
 * first argument of a min/max; a minmod passes the derivative to its
 * smallest-magnitude argument only when all arguments share a strict sign;
 * alpha's derivative goes to its first maximising cell, and |u_n| in the
 * signal speed passes sgn(u_n) (0 at u_n = 0).  dt is a parameter (not
 * differentiated).
 */

/* Workspace bytes tenom_flux_divergence_vjp needs (0 if invalid): one
 * contribution per face, stencil slot and field of the largest axis. */
size_t tenom_vjp_workspace_bytes(const tenom_grid* grid, int scheme);

/*
 * Ubar = (accumulate ? Ubar : 0) + scale * (d L / d U)^T Lbar, where
 * L(U) = tenom_flux_divergence(U).  U, Lbar, Ubar: device arrays of the
 * state's shape; Ubar must not alias U or Lbar.  ws: device workspace of
 * tenom_vjp_workspace_bytes.  Deterministic (no atomics).
 */
int tenom_flux_divergence_vjp(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma,
                              const double* U, const double* Lbar, double scale, double* Ubar, int accumulate,
                              void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes tenom_rk3_step_vjp needs: five states plus the above. */
size_t tenom_rk3_vjp_workspace_bytes(const tenom_grid* grid, int scheme);

/*
 * Adjoint of one tenom_rk3_step from the state U (the step's input, not
 * modified) with step dt: on entry Ubar holds the cotangent of the step's
 * output, on return that of its input.  The stage states are recomputed by
 * the forward sweeps into the workspace (256-byte aligned, at least
 * tenom_rk3_vjp_workspace_bytes), so every decision is the one the forward
 * step took.
 */
int tenom_rk3_step_vjp(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                       const double* U, double* Ubar, void* ws, size_t ws_bytes, void* stream);

/*
 * tenom_rk3_step_vjp with the step's stage states given (U1, U2 as written
 * by tenom_rk3_step_stages from the same U, dt and scheme) instead of
 * recomputed.  U, U1, U2 are not modified; Ubar must not alias any of them.
 * Same workspace as tenom_rk3_step_vjp.  The stage states are not checked
 * against U: the caller guarantees they are the ones the step from U made
 * (otherwise the result is the adjoint of no step).
 */
int tenom_rk3_step_vjp_stages(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                              const double* U, const double* U1, const double* U2, double* Ubar, void* ws,
                              size_t ws_bytes, void* stream);

/* ---- batched independent 1D problems ------------------------------------ */
/*
 * Many independent 1D Euler problems of uneven size (the shock tubes of
 * Sec. 4.2, one per problem) advanced together: each problem p has n[p]
 * cells of size dx[p], the same boundary rule at both of its ends, and its
 * own SSP-RK3 step dt_p = cfl / max_cells (|u| + c) / dx[p], computed on the
 * device at the start of every step from the problem's current state.
 *
 * State layout: one device array [3][total] (rho, rho*u, E), the problems
 * packed end to end in order: problem p occupies cells
 * off[p] .. off[p] + n[p] - 1 of every field, off[p] = n[0] + ... + n[p-1],
 * and total = off[count] (tenom_batch_cells).
 *
 * The plan holds everything the calls need on the device: the problem
 * offsets, 1/dx, each problem's last dt and its clock (the sum of its
 * steps), two stage states of 3 * total doubles (the RK3 intermediates), a
 * segment table per tile shape, and the captured graph.  A plan belongs to
 * the device that was current at tenom_batch_create; every call needs that
 * device current.  Calls on one plan must not run concurrently.
 */
typedef struct tenom_batch_plan tenom_batch_plan;

/* Tile shapes of the batched sweep: a workgroup of `threads` threads
 * computes threads * faces_per_thread faces of one problem. */
#define TENOM_BATCH_TILES 6
int tenom_batch_tile_shape(int tile, int* threads, int* faces_per_thread);

/*
 * Create a plan for `count` problems (count >= 0; 0 makes every call a
 * no-op).  n, dx: HOST arrays of count entries, n[p] >= 6, dx[p] > 0.
 * bc: TENOM_BC_PERIODIC or TENOM_BC_TRANSMISSIVE for every problem.
 * Allocates the plan's device memory (about 48 * total bytes plus small
 * tables); clocks start at 0; the tile is 3 until set or autotuned.
 * Errors: EINVAL for bad arguments (no allocation), EHIP if an allocation
 * fails.
 */
int tenom_batch_create(int count, const int64_t* n, const double* dx, int bc, tenom_batch_plan** plan);
/* Synchronise the device and free the plan (NULL is a no-op). */
int tenom_batch_destroy(tenom_batch_plan* plan);
/* Total cells of the batch (the field pitch of U), -1 for NULL. */
int64_t tenom_batch_cells(const tenom_batch_plan* plan);
/* Select the tile shape of later calls (0 .. TENOM_BATCH_TILES-1). */
int tenom_batch_set_tile(tenom_batch_plan* plan, int tile);
int tenom_batch_get_tile(const tenom_batch_plan* plan);

/*
 * Enqueue `steps` SSP-RK3 steps (Sec. 4) of problems first .. first+count-1
 * on `stream`, in place on U (device, [3][total]).  Per step: one kernel for
 * the step sizes of the selected problems, then three stage sweeps, each
 * one launch over all selected problems (reconstruction as in
 * tenom_reconstruct_faces, divergence and the stage update fused).  Other
 * problems' cells are not touched.  No allocation, no synchronisation.
 * Every problem needs n >= K.  Euler system only (gamma > 1).
 */
int tenom_batch_rk3(tenom_batch_plan* plan, int scheme, int limiter, double C_T, double gamma, double cfl, int steps,
                    int first, int count, double* U, void* stream);

/*
 * The same for all problems as one HIP graph launch on `stream`: the first
 * call captures the `steps` steps (4 * steps kernels) into a graph the
 * plan keeps; later calls with the same arguments, U and tile replay it.
 * Other arguments recapture.  Equal in every bit to tenom_batch_rk3.
 */
int tenom_batch_rk3_graph(tenom_batch_plan* plan, int scheme, int limiter, double C_T, double gamma, double cfl,
                          int steps, double* U, void* stream);

/*
 * The same `steps` steps of all problems as ONE kernel launch on `stream`
 * (persistent: each workgroup advances its share of the problems through
 * every step and stage on its own, with the step sizes and stage states of
 * tenom_batch_rk3; problems are independent, so no workgroup waits for
 * another).  Three 256-thread workgroups per compute unit take the problems
 * from a queue in the plan, longest first, each whole; the plan's queue is
 * clear again when the launch ends, so launches on one plan must not
 * overlap (calls on a plan never may).  Equal in every bit to tenom_batch_rk3 (the
 * tile shape does not matter); updates the clocks and last steps the same
 * way.  No allocation, no synchronisation; the launch can be captured in a
 * HIP graph.
 */
int tenom_batch_rk3_persistent(tenom_batch_plan* plan, int scheme, int limiter, double C_T, double gamma, double cfl,
                               int steps, double* U, void* stream);

/*
 * Autotuner of the tile shape: time `steps` steps (after one untimed step)
 * of every tile on a copy of U, for this scheme and limiter, select the
 * fastest for later calls and return it in *best (nullable).
 * ms_per_step: nullable HOST array of TENOM_BATCH_TILES entries.  U and the
 * plan's clocks are left as they were.  Allocates one temporary state copy
 * and synchronises `stream`.  Every tile gives the same bits, so the choice
 * changes only the speed.
 */
int tenom_batch_autotune(tenom_batch_plan* plan, int scheme, int limiter, double C_T, double gamma, double cfl,
                         const double* U, int steps, float* ms_per_step, int* best, void* stream);

/* Each problem's clock (sum of its steps) and last step into HOST arrays of
 * count entries (either nullable); synchronises `stream`. */
int tenom_batch_times(const tenom_batch_plan* plan, double* t, double* dt, void* stream);
/* Set every clock and last step to 0 (enqueued on `stream`). */
int tenom_batch_reset_times(tenom_batch_plan* plan, void* stream);

/* ---- diagnostics -------------------------------------------------------- */

/* Static text for a return code. */
const char* tenom_strerror(int code);
/* Message of the last failure on the calling thread ("" if none). */
const char* tenom_last_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int tenom_version(void);

/*
 * Kernel of the sweeps, for every later call in the process (a test and
 * tuning aid; the kernels compute the same face fluxes and cell updates,
 * operation for operation, so the results are identical bit for bit).
 * TENOM_SWEEP_MARCH: the line kernels; x rows are staged in LDS by
 * segments of 256 cells, and along y and z each lane marches one x column
 * along a segment of the line with its stencil in an LDS ring.
 * TENOM_SWEEP_TILE: a workgroup stages tiles of 8 adjacent lines (x columns
 * for y and z, y rows for x) by a chunk of the line in LDS and walks the
 * lines whole.  TENOM_SWEEP_AUTO (the default): per axis, the tile kernel
 * when the lines alone give at least 512 workgroups (along x only for the
 * six-point schemes), else the line kernel.
 * Returns TENOM_EINVAL for any other value.  The setting is process-wide;
 * calls made while another thread changes it may use either kernel.
 */
#define TENOM_SWEEP_AUTO 0
#define TENOM_SWEEP_MARCH 1
#define TENOM_SWEEP_TILE 2
int tenom_set_sweep_kernel(int kind);

/*
 * Kernel timing: while enabled, every kernel the compute calls launch is
 * bracketed by HIP events recorded on the same stream.  tenom_profile_read
 * synchronises those events and returns, per kernel kind, the number of
 * launches and their summed duration in milliseconds since the last reset.
 * Kinds: 0 face fluxes (reconstruct_faces), 1 x-sweep, 2 y-sweep,
 * 3 z-sweep, 4 batched sweep, 5 batched step size, 6 one replay of a batched
 * graph (kernels inside a graph are not bracketed one by one), 7 one axis of
 * an adjoint (face kernel + gather), 8 one persistent batched launch.  At
 * most 4096 launches are recorded between reads.
 */
#define TENOM_KERNEL_KINDS 9
int tenom_profile_enable(int on);
int tenom_profile_read(int64_t* counts, double* total_ms, int nkinds);

#ifdef __cplusplus
}
#endif

#endif /* TENOM_H */
