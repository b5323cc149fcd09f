/*
 * bn2d.h -- C ABI of the MI355X (gfx950) library for the explicit time step of the
 * second-order, well-balanced, path-conservative finite-volume scheme for the reduced
 * three-equation Baer-Nunziato free-surface model (Gaburro, Castro, Dumbser,
 * arXiv:1806.04960).
 *
 * State.  Q = (alpha rho, alpha rho u, alpha rho v, alpha) of the reduced model (Sec. 2,
 * conservative variables of the non-conservative form; the gravity potential y of Sec. 2.1 is
 * implicit: cell-centre and edge heights are computed from the grid).  A state buffer is
 * 4 * nx * ny FP64 values in structure-of-arrays order: plane k (k = 0..3) then row j
 * (0..ny-1, bottom to top) then column i (0..nx-1, x fastest).  Cell (i, j) covers
 * [x0 + i dx, x0 + (i+1) dx] x [y0 + j dy, y0 + (j+1) dy], dx = (x1-x0)/nx, dy = (y1-y0)/ny
 * (Sec. 3, Cartesian mesh).
 *
 * Ownership.  The context owns every device buffer it uses: two state buffers (ping-pong),
 * the solid mask, the per-column free-surface integrals (64-bit fixed point), the step kernel's
 * work lists, the CFL maximum, dt and the elapsed time.
 * State crosses the boundary only through bn_set_state / bn_get_state, which copy from / to
 * a caller-owned device buffer.  All work is enqueued on the HIP stream given at creation
 * (NULL = the legacy default stream); a context is used by one host thread at a time.
 *
 * Errors.  Every call returns BN_OK (0) or a negative BN_E* code; bn_strerror names it.
 * Nothing is thrown across the ABI.  Asynchronous calls (bn_step, bn_run) report HIP launch
 * errors immediately; non-physical states found on the device (a fluid cell with
 * alpha rho <= 0, alpha <= 0 or a non-finite value) are reported by the next synchronising
 * call (bn_compute_dt, bn_get_time, bn_status).  The product path has no CPU fallback.
 */
#ifndef BN2D_H
#define BN2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BN_OK 0
#define BN_EINVAL (-1)        /* bad argument: null pointer, size, parameter out of range */
#define BN_EHIP (-2)          /* a HIP runtime call failed (text via bn_strerror) */
#define BN_ENONPHYS (-3)      /* a fluid cell left the admissible set */
#define BN_EUNSUPPORTED (-4)  /* a solid cell above a fluid cell in one column */
#define BN_ENOMEM (-5)        /* device allocation failed */
#define BN_EINTERNAL (-6)     /* the step kernel's work distribution failed (a bug, never expected) */

/* Cartesian grid of nx x ny cells on [x0, x1] x [y0, y1] (Sec. 3). */
typedef struct {
    int32_t nx, ny;
    double x0, x1, y0, y1;
} bn_grid;

/* Model constants: gravity g (Sec. 2), Tait constants k0, rho0 with gamma = 1 (Sec. 2, all
 * tests of Sec. 5), two-level volume fractions alpha_liq (liquid, 1 - eps or 1) and
 * alpha_gas (eps) of the equilibrium profile and of the second-order switch alpha > 10 eps
 * (Sec. 3.4), the CFL number, and the boundary condition of each side (W, E, S, N):
 * 0 = reflective wall (mirror state with negated normal velocity, Sec. 5), 1 = transmissive.
 * Requires k0 > 0, rho0 > 0, 0 < alpha_gas < alpha_liq <= 1, 0 < cfl <= 1, g >= 0. */
typedef struct {
    double g, k0, rho0, alpha_liq, alpha_gas, cfl;
    int32_t bc[4];
} bn_params;

typedef struct bn_ctx bn_ctx;

/* Create a context.  solid: host array of nx*ny bytes (row-major, 1 = solid cell removed from
 * the domain, Sec. 5.1) or NULL; each column's solid cells must form one run attached to the
 * bottom (else BN_EUNSUPPORTED), as the free-surface detector of Sec. 3.5 integrates alpha
 * from the top of that run.  hip_stream: a hipStream_t or NULL.  Synchronous.  Sizes: at most
 * 32767 column strips of 60 (nx <= 1966020) and ny <= 16711680 (0xFF0000), the fields of the
 * step kernel's range descriptors; larger grids give BN_EINVAL. */
int bn_create(const bn_grid *grid, const bn_params *params, const uint8_t *solid, void *hip_stream,
              bn_ctx **out);

/* Copy a state from the caller's device buffer q_dev (4*nx*ny doubles, layout above) and
 * compute its free-surface heights (Sec. 3.5) and CFL time step.  Stream-ordered. */
int bn_set_state(bn_ctx *ctx, const double *q_dev);

/* Copy the current state into the caller's device buffer q_dev.  Stream-ordered. */
int bn_get_state(bn_ctx *ctx, double *q_dev);

/* dt = CFL / max over fluid cells of ((|u|+c)/dx + (|v|+c)/dy) for the current state.
 * Synchronises the stream; BN_ENONPHYS if the state is not admissible. */
int bn_compute_dt(bn_ctx *ctx, double *dt_host);

/* One explicit step of the scheme (Sec. 3, eq. Scheme) with the given dt > 0: free-surface
 * detection, well-balanced reconstruction with Hancock predictor (Sec. 3.4), Osher edge
 * fluctuations in x (Sec. 3.2), well-balanced Osher-Romberg fluctuations in y (Sec. 3.3), cell
 * update.  Asynchronous on the context's stream; adds dt to the elapsed time. */
int bn_step(bn_ctx *ctx, double dt);

/* n_steps >= 0 steps, each with the CFL time step of the state it starts from, computed and
 * kept on the device.  Asynchronous. */
int bn_run(bn_ctx *ctx, int32_t n_steps);

/* Elapsed simulated time since bn_set_state and the dt the next bn_run step will use.
 * Synchronises; BN_ENONPHYS if a non-physical state was met. */
int bn_get_time(bn_ctx *ctx, double *t_host, double *next_dt_host);

/* Free-surface height of every column of the current state (nx doubles, host).  Synchronises. */
int bn_get_y0(bn_ctx *ctx, double *y0_host);

/* Synchronise and report BN_ENONPHYS if any step met a non-physical state. */
int bn_status(bn_ctx *ctx);

/* Bottom height y_L of each column for the free-surface detector (Sec. 3.5: y0 = y_L + the integral
 * of the normalised volume fraction from y_L up), e.g. the top of an obstacle that does not lie on a
 * grid line (the wall of Sec. 5.7).  y_bottom_host: nx doubles (host), each within half a cell of the
 * top of its column's solid run: -dy/2 <= y_L - (y0 + jb dy) < dy/2 with jb the column's solid cells
 * (else BN_EINVAL, nothing changed); NULL restores the default, the top of each solid run.  The
 * cells stay whole; the detector takes the column's first fluid cell to cover the interval from y_L
 * to its top edge:  y0 = (y0 + jb dy) + dy sum_j a_j + (y_L - y0 - jb dy)(1 - a_jb),
 * a = (alpha - alpha_gas)/(alpha_liq - alpha_gas), so a full first cell gives the grid-aligned value
 * exactly.  Applies from the next step on; synchronises the stream. */
int bn_set_bottom(bn_ctx *ctx, const double *y_bottom_host);

/* Launch shape of the step kernel.  Wavefronts march strips of 60 columns and claim rows in blocks
 * of rows_per_block (1..4096, 0 = default 4); the launch is persistent with `wavefronts`
 * wavefronts (1..65536, 0 = default: as many as the device holds at once, or fewer for a small grid,
 * about one per 4.5 rows of 60-column strips, a power of two, at least 256).  Results are bitwise the same
 * for every shape: each cell is computed by the same arithmetic whatever wavefront does it, and
 * the free-surface integral is summed exactly (64-bit fixed point).  Synchronises the stream. */
int bn_set_launch(bn_ctx *ctx, int32_t rows_per_block, int32_t wavefronts);

/* The current launch shape (defaults resolved); either pointer may be NULL. */
int bn_get_launch(bn_ctx *ctx, int32_t *rows_per_block, int32_t *wavefronts);

void bn_destroy(bn_ctx *ctx);
const char *bn_strerror(int code);

/* Discrete adjoint of one step with time step dt (the step of bn_step, Sec. 3 eq. Scheme with
 * Sec. 3.1-3.5, differentiated in reverse mode with respect to the state at t^n):
 *   lam_dev = (d Q^{n+1} / d Q^n)^T lam_next_dev,   Q^{n+1} = step(q_dev, dt).
 * q_dev, lam_next_dev: caller-owned device buffers, 4 planes x nx*ny FP64 (the state layout);
 * lam_dev receives the adjoint of the state at t^n in the same layout and must not overlap
 * either input.  The context's own state, time and schedule are not touched; q_dev need not be
 * the context's state.  dt is held fixed (the CFL maximum is not differentiated); the free-surface
 * height is differentiated as the real column sum of Sec. 3.5; at the scheme's non-smooth points
 * (limiter min/max, |u|, sign, the second-order and liquid switches, walls) the branch the step
 * takes is differentiated.  grad_bottom_dev: NULL, or a caller-owned device buffer of nx doubles
 * that receives the model-parameter gradient (d Q^{n+1} / d y_L)^T lam_next_dev of the columns'
 * bottom heights y_L (bn_set_bottom; e.g. an obstacle's height): y_L enters the step only through
 * its column's free surface, dy0/dy_L = 1 - a of the column's first fluid cell (0 for a fully solid
 * column).  src_dev: NULL, or a caller-owned device buffer in the state layout added to the result
 * (lam_dev = (d Q^{n+1} / d Q^n)^T lam_next_dev + src_dev): the per-step term dJ/dQ^n of a loss summed
 * over a trajectory, so that a reverse sweep needs no separate addition; it may be lam_next_dev
 * itself but must not overlap lam_dev.  The library allocates its scratch (about 6.5 doubles per cell) on the first call and keeps
 * it until bn_destroy.  Asynchronous on the context's stream.  Errors: BN_EINVAL (null pointer, dt <= 0
 * or not finite), BN_ENOMEM, BN_EHIP.  A non-physical q_dev gives non-finite values. */
int bn_adjoint_step(bn_ctx *ctx, const double *q_dev, const double *lam_next_dev, double dt, double *lam_dev,
                    double *grad_bottom_dev, const double *src_dev);

/* The free-surface column integrals of the context's current state (Sec. 3.5: per column the sum
 * over its fluid cells of (alpha - alpha_g) / (alpha_l - alpha_g)), in the library's 64-bit fixed
 * point (exact, independent of the order of summation): nx words into the caller-owned device
 * buffer sums_dev, the values a step from that state uses.  The step that produced the state (or
 * bn_set_state) computed them, so this is a copy of nx words.  For bn_adjoint_step_sums.
 * Asynchronous on the context's stream.  Errors: BN_EINVAL (null pointer), BN_EHIP. */
int bn_get_column_sums(bn_ctx *ctx, int64_t *sums_dev);

/* bn_adjoint_step with the free-surface column integrals of q_dev given instead of computed from
 * q_dev again: sums_dev, nx words, is what bn_get_column_sums returned for a context of the same
 * grid, model and bottoms whose state was q_dev (e.g. the context that recomputed q_dev on another
 * stream).  Bitwise the same lambda as bn_adjoint_step, one kernel fewer on the context's stream.
 * Other values in sums_dev give a wrong result, not an error.  Other arguments, ownership, scratch,
 * stream and errors as bn_adjoint_step (BN_EINVAL also for a null sums_dev). */
int bn_adjoint_step_sums(bn_ctx *ctx, const double *q_dev, const int64_t *sums_dev, const double *lam_next_dev,
                         double dt, double *lam_dev, double *grad_bottom_dev, const double *src_dev);

/* bn_adjoint_step without any allocation, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc).  Same arguments, result
 * and errors as bn_adjoint_step (bitwise the same lambda: the same kernels), but the scratch is a
 * fixed library array of 2^24 doubles (128 MiB) per GPU, reserved when the library's device code is
 * loaded and held until the process ends, instead of memory allocated on the first call.  The grid
 * must fit: 4 nx ny + 560 ceil(nx / 64) ceil(ny / 4) + nx (ceil(ny / 4) + ceil(ny / 16) + 1) <= 2^24
 * (about 2.5 million cells, e.g. 2048 x 1024; not 2048 x 2048), else BN_EINVAL before any work is
 * enqueued.  The first call on a device resolves the
 * array's address on that device (the current device must be the context's).  Every call on a GPU
 * uses that GPU's one array: calls that overlap in time on one GPU (other streams, other contexts,
 * other threads) race and give wrong results; calls ordered on one stream, or synchronised, do not.
 * Calls no hipMalloc, hipFree or allocating library routine. */
int bn_adjoint_step_noalloc(bn_ctx *ctx, const double *q_dev, const double *lam_next_dev, double dt, double *lam_dev,
                            double *grad_bottom_dev, const double *src_dev);

/* ---- Batches: many grids advanced by one launch per step -------------------------------------
 * A batch holds `count` independent grids (members) of any sizes, parameters and masks, e.g. an
 * ensemble of scenarios too small to fill the device one by one.  Every bn_batch_run step advances
 * each member by one explicit step of the scheme (the same step as bn_step) with its own CFL time
 * step, in one launch of the step kernel whose work list spans all members.  Each member's results
 * are bitwise those of a single-grid context on the same input.  A single-grid context is a batch
 * of one.  Members are numbered 0..count-1.  Same ownership, error and stream rules as above. */
typedef struct bn_batch bn_batch;

/* grids[count], params[count]; solids: NULL or an array of count host masks (each NULL or nx*ny
 * bytes, as for bn_create).  count in 1..32767, at most 32767 column strips of 60 in total. */
int bn_batch_create(int32_t count, const bn_grid *grids, const bn_params *params, const uint8_t *const *solids,
                    void *hip_stream, bn_batch **out);

/* Set / read member `member`'s state (device buffers as for bn_set_state / bn_get_state).  Every
 * member needs a state before bn_batch_run.  Setting a state resets that member's time. */
int bn_batch_set_state(bn_batch *batch, int32_t member, const double *q_dev);
int bn_batch_get_state(bn_batch *batch, int32_t member, double *q_dev);

/* n_steps >= 0 steps of every member, each with its own CFL time step.  Asynchronous. */
int bn_batch_run(bn_batch *batch, int32_t n_steps);

/* Elapsed time of a member and the dt its next step will use; free-surface heights of a member
 * (nx doubles, host).  Synchronise. */
int bn_batch_get_time(bn_batch *batch, int32_t member, double *t_host, double *next_dt_host);
int bn_batch_get_y0(bn_batch *batch, int32_t member, double *y0_host);

/* Synchronise; BN_ENONPHYS with *member set to the first member that met a non-physical state
 * (member may be NULL; -1 when all are fine). */
int bn_batch_status(bn_batch *batch, int32_t *member);

/* Bottom heights of member `member`, as bn_set_bottom. */
int bn_batch_set_bottom(bn_batch *batch, int32_t member, const double *y_bottom_host);

/* Launch shape, as bn_set_launch / bn_get_launch. */
int bn_batch_set_launch(bn_batch *batch, int32_t rows_per_block, int32_t wavefronts);
int bn_batch_get_launch(bn_batch *batch, int32_t *rows_per_block, int32_t *wavefronts);

void bn_batch_destroy(bn_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* BN2D_H */
