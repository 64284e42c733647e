/*
 * igr.h -- C ABI of libigr, the MI355X (gfx950) implementation of the hot
 * path of the information-geometric-regularisation (IGR) compressible Euler
 * solver of "Simulating many-engine spacecraft: Exceeding 1 quadrillion
 * degrees of freedom via information geometric regularization"
 * (arXiv 2505.07392).
 *
 * The problem is the IGR-modified Euler system, eqs. (6)-(8) of the paper
 * with the viscous stress set to zero, closed by the ideal-gas law, eq. (4),
 * and the entropic-pressure equation, eq. (9):
 *
 *   alpha [tr((grad u)^2) + tr^2(grad u)] = Sigma/rho - alpha div(grad Sigma / rho)
 *
 * discretised as in the "Discretization" subsection and Algorithm 1 ("The
 * algorithm"): fifth-order linear reconstruction of the conserved variables
 * and of Sigma, local Lax-Friedrichs fluxes with p + Sigma, second-order
 * central velocity gradients for the left side of eq. (9), a 7-point stencil
 * for its operator solved by a fixed number of Jacobi sweeps warm-started
 * from the previous Sigma, and third-order SSP Runge-Kutta in time.
 *
 * Data layout (every array argument)
 * ----------------------------------
 * Cell arrays are padded with G = 3 ghost layers on every side and stored
 * x fastest: one field holds (nz+6)*(ny+6)*(nx+6) elements, element
 * (i, j, k) of the interior (0 <= i < nx, ...) at offset
 * ((k+3)*(ny+6) + (j+3))*(nx+6) + (i+3).  A state U is five consecutive
 * fields (rho, rho*u, rho*v, rho*w, E); Sigma and scalar outputs are one
 * field.  The element type follows the context precision: double
 * (IGR_F64), float (IGR_F32), uint16_t holding bfloat16 (IGR_BF16_F32:
 * bfloat16 storage, float arithmetic) or IEEE binary16 (IGR_F16_F32: half
 * storage, float arithmetic -- the storage form of the paper's "Mixed
 * Precision" section).  Every stored value is rounded to nearest even once;
 * dt, the conservation sums and the Jacobi residual are FP64 in every form.
 *
 * Ownership and streams
 * ---------------------
 * All array pointers are device pointers owned by the caller; the library
 * never frees them.  Interior cells are inputs/outputs as documented per
 * call; ghost layers of U and Sigma are library-written scratch.  Internal
 * scratch (two more states, a second Sigma, the Sigma source, reduction
 * buffers, the error flag) is allocated by igr_init on the device current
 * at that time and released by igr_finalize.  `stream` is a hipStream_t
 * passed as void* (NULL = the default stream); all work is enqueued on it.
 * Calls that return host values (dt, residual, sums) synchronise that
 * stream.  A context may be used by one host thread at a time; calls on
 * one context must not overlap.
 *
 * Errors
 * ------
 * Every call returns IGR_OK (0) or an error code; no C++ exception crosses
 * the ABI.  igr_last_error() returns a thread-local message for the last
 * failing call.  IGR_ENONFINITE reports a face or cell state with
 * rho <= 0, p <= 0 or a non-finite value seen by a kernel since the last
 * check; the arrays are left as computed.  Asynchronous calls (igr_step
 * with dt_used == NULL) record such states in a device flag that the next
 * synchronising call (or igr_check) reports.
 */
#ifndef IGR_H
#define IGR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    IGR_OK = 0,
    IGR_EINVAL = 1,        /* bad argument: null pointer, size, gamma <= 1, alpha < 0, ... */
    IGR_ENOMEM = 2,        /* device allocation failed */
    IGR_EHIP = 3,          /* HIP runtime error (message in igr_last_error) */
    IGR_ENONFINITE = 4,    /* rho <= 0, p <= 0 or NaN/Inf seen by a kernel */
    IGR_EUNSUPPORTED = 5   /* valid but unimplemented option */
};

enum { IGR_BC_PERIODIC = 0, IGR_BC_EXTRAP = 1 };

enum { IGR_F64 = 0, IGR_F32 = 1, IGR_BF16_F32 = 2, IGR_F16_F32 = 3, IGR_F32_BF16D = 4 };

enum { IGR_SMOOTH_JACOBI = 0, IGR_SMOOTH_RBGS = 1 };

/* Uniform rectilinear grid of nx*ny*nz interior cells with spacings dx, dy,
 * dz (paper, "Example simulation result": rectilinear grid).  Each extent
 * must be >= 1; ghost indices wrap modulo the extent on periodic axes. */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
} igr_grid;

/* Inflow disc on the x-min face (engines are modelled by inflow boundary
 * conditions: paper, "Example simulation result").  Centre (yc, zc),
 * radius r and edge width `width` in physical units; primitive jet state
 * (rho, ux, uy, uz, p).  Each x-min ghost column takes the disc whose
 * centre is nearest to the column's cell centre ((j+1/2)dy, (k+1/2)dz)
 * (lowest index on ties) and sets all three ghost layers to
 * chi*U_jet + (1-chi)*U_extrap, chi = (1 - tanh((s - r)/width))/2 at
 * distance s (chi = [s <= r] when width == 0), U_extrap being the first
 * interior cell of that column. */
typedef struct {
    double yc, zc, r, width;
    double rho, ux, uy, uz, p;
} igr_patch;

/* Boundary description: face kinds in the order -x, +x, -y, +y, -z, +z
 * (IGR_BC_PERIODIC must come in pairs; IGR_BC_EXTRAP copies the first
 * interior cell into all three ghost layers), plus optional inflow discs
 * (require a non-periodic x axis).  Sigma uses periodic wrap on periodic
 * faces and zero gradient on every other face.  The patch array is copied
 * by igr_init. */
typedef struct {
    int32_t face[6];
    int32_t npatch;
    const igr_patch *patch;
} igr_bc;

/* Options: storage/arithmetic precision, reconstruction order (5, or 3:
 * the paper's third- or fifth-order finite volume method, "Discretization";
 * the adjoint entry points need 5), Jacobi
 * sweeps per right-hand side (the paper uses up to 5: "Shock treatment with
 * information geometric regularization"), and sigma_block, how the sweeps
 * are grouped into passes over memory: 1 runs one z-marching sweep per
 * pass (the first also forms the source); 2 runs that first pass and then
 * two sweeps per pass (temporally blocked, reusing the stored source);
 * 3..5 run passes of up to that many sweeps of a kernel that forms the
 * source itself.  0 selects the default: 2 for IGR_F64; for the forms
 * with FP32 arithmetic, 1 while one sweep's working set (padded field
 * elements x (3 x storage bytes + 4)) fits the 256 MiB last-level cache,
 * else 2 (igr_get_opts reports the choice).  Results agree to rounding.  smoother selects the
 * sweep: IGR_SMOOTH_JACOBI (default), or IGR_SMOOTH_RBGS, red-black
 * Gauss-Seidel (the paper's alternative, "Discretization"): each sweep
 * updates the cells with i + j + k even, then the others, each colour from
 * the values at the start of its half-sweep (with sigma_block 2 one pass
 * per sweep forms both halves; otherwise each half is a launch of its own,
 * in place; periodic axes need even extents, else IGR_EUNSUPPORTED;
 * the adjoint entry points need Jacobi). */
typedef struct {
    int32_t precision;
    int32_t order;
    int32_t nsweeps;
    int32_t sigma_block;
    int32_t smoother;
    double mu;     /* shear viscosity of eq. (5), >= 0 (0: the Euler system) */
    double zeta;   /* bulk viscosity of eq. (5), >= 0 */
} igr_opts;

typedef struct igr_ctx igr_ctx;

/* Create a context for one grid on the current device.  gamma > 1,
 * alpha >= 0 (the paper takes alpha proportional to dx^2); a padded x-y
 * plane, (nx+6)*(ny+6), below 2^29 elements (the kernels address a plane
 * with 32-bit byte offsets), else IGR_EINVAL.  On success *out owns the
 * scratch memory; release it with igr_finalize. */
int igr_init(const igr_grid *grid, double gamma, double alpha, const igr_bc *bc,
             const igr_opts *opts, igr_ctx **out);

/* Release a context and its scratch (NULL is accepted). */
int igr_finalize(igr_ctx *ctx);

/* Thread-local message of the last failing call on this thread. */
const char *igr_last_error(void);

/* Elements per padded field, (nz+6)*(ny+6)*(nx+6), and bytes per element. */
int igr_field_size(const igr_ctx *ctx, int64_t *elems, int32_t *elem_bytes);

/* The options a context runs with, defaults resolved (sigma_block is never
 * 0 here). */
int igr_get_opts(const igr_ctx *ctx, igr_opts *out);

/* Replace the primitive state (rho, ux, uy, uz, p) of inflow disc `index`
 * (geometry unchanged).  The update is enqueued on `stream`: work queued
 * before it on that stream uses the old state, work queued after it the
 * new one (other streams order themselves with events).  Asynchronous. */
int igr_set_patch_state(igr_ctx *ctx, int32_t index, const double prim[5], void *stream);

/* Entropic pressure: fill U's ghosts, form the source
 * b = alpha [tr((grad u)^2) + tr^2(grad u)] with central differences, and
 * run `nsweeps` Jacobi sweeps of eq. (9)'s 7-point discretisation
 * (face coefficient (1/rho_c + 1/rho_nb)/2) starting from sigma's interior
 * (warm start; paper: "Discretization" and "Shock treatment ...").
 * On return sigma's interior holds the last iterate and its ghosts are
 * filled.  If resid_l2 is not NULL it receives the FP64 l2 norm (no volume
 * weight) of b - A sigma over interior cells (synchronises). */
int igr_sigma_solve(igr_ctx *ctx, void *U, void *sigma, int32_t nsweeps, double *resid_l2,
                    void *stream);

/* One right-hand-side evaluation L(U) (Algorithm 1): ghosts, Sigma solve
 * with the context's sweep count warm-started from sigma (in: previous
 * Sigma, out: new Sigma), reconstruction, local Lax-Friedrichs fluxes
 * with p + Sigma, divergence.  rhs's interior receives L(U); its ghosts
 * are not written. */
int igr_rhs(igr_ctx *ctx, void *U, void *sigma, void *rhs, void *stream);

/* One SSP-RK3 step (Gottlieb & Shu; paper "Discretization") in place on U
 * and sigma, one Sigma solve per stage warm-started from the previous
 * stage.  dt = dt_fixed if dt_fixed > 0, else
 * cfl / max_cells sum_d (|u_d| + c)/dx_d computed on the device in FP64.
 * If dt_used is not NULL the stream is synchronised, *dt_used receives dt
 * and the error flag is checked. */
int igr_step(igr_ctx *ctx, void *U, void *sigma, double cfl, double dt_fixed, double *dt_used,
             void *stream);

/* nsteps igr_step calls in one: the same states and time steps.  With a
 * CFL time step (dt_fixed <= 0) the maximum speed for step n+1 is formed
 * by step n's last stage as it writes the new state (the same FP64
 * expression as the standalone reduction, on the values as stored; with
 * viscous terms by their kernel, which completes the new state), so the
 * separate pass over U runs only before the first step.  Between steps
 * Sigma may live in the context's scratch copy (a step starts from where
 * the previous one's solve left it); sigma holds the last step's Sigma on
 * return, as after nsteps igr_step calls (if a call fails part-way,
 * sigma's contents are unspecified).  If dt_last is not NULL the stream
 * is synchronised, *dt_last receives the last step's dt and the error
 * flag is checked.  nsteps >= 0. */
int igr_advance(igr_ctx *ctx, void *U, void *sigma, int32_t nsteps, double cfl, double dt_fixed, double *dt_last,
                void *stream);

/* Discrete adjoint of igr_rhs (FP64 contexts with Jacobi sweeps, either
 * reconstruction order, with or without the viscous terms, else
 * IGR_EUNSUPPORTED; vector-Jacobian product of
 * the map (U, sigma_prev) -> (L(U), sigma_new) and of the jet-disc
 * states).  Given rhs_bar (5 fields) and sigma_bar (cotangent of the new
 * Sigma), writes U_bar (5 fields) and sigma_prev_bar; only interiors are
 * read, outputs have zero ghosts.  patch_bar (nullable, host, npatch*5)
 * receives the cotangents of the primitive jet states (rho, ux, uy, uz, p).
 * The LLF maximum passes its cotangent to the larger wave speed (half to
 * each on a tie) and |u_n| uses sign(u_n).  U's ghosts are rewritten.
 * Inputs may alias outputs.  Scratch (about 70 + nsweeps FP64 fields) is
 * allocated on the first call and kept by the context.  Synchronises. */
int igr_rhs_adjoint(igr_ctx *ctx, void *U, const void *sigma_prev, const void *rhs_bar, const void *sigma_bar,
                    void *U_bar, void *sigma_prev_bar, double *patch_bar, void *stream);

/* Discrete adjoint of one igr_step with a fixed time step dt > 0 (the
 * contexts igr_rhs_adjoint accepts):
 * given the step's input (U_n, sigma_n) and the cotangents of its output
 * (U_bar_np1, sigma_bar_np1), writes the cotangents of its input (U_bar_n,
 * sigma_bar_n) and, if patch_bar is not NULL, of the primitive jet states
 * (npatch*5, host).  The three stage states and Sigma iterates are
 * recomputed from U_n inside the call (no storage between calls), so a
 * multi-step gradient needs only the per-step inputs (checkpointing).
 * Conventions, aliasing and scratch as igr_rhs_adjoint.  Synchronises. */
int igr_step_adjoint(igr_ctx *ctx, void *U_n, const void *sigma_n, double dt, const void *U_bar_np1,
                     const void *sigma_bar_np1, void *U_bar_n, void *sigma_bar_n, double *patch_bar,
                     void *stream);

/* FP64 CFL time step of state U (rule as in igr_step; synchronises). */
int igr_compute_dt(igr_ctx *ctx, const void *U, double cfl, double *dt, void *stream);

/* igr_compute_dt without a context, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same FP64 CFL time step as
 * igr_compute_dt for a state U of the padded layout above, described by
 * grid, gamma (> 1) and precision (one of the IGR_* storage forms); U is
 * only read and may hold any ghost values.  The call allocates nothing:
 * its reduction partials, result and non-finite flag live in a fixed
 * 16 KiB device array of the library (one per device, held until the
 * process ends), located once per device on the first call with that
 * device current.  The reduction runs on a fixed grid of 1024 blocks, so
 * every grid whose x-y plane fits 32-bit offsets fits the array (larger
 * planes: IGR_EINVAL).  The flag is cleared by a kernel at the start of
 * each call; the stream is synchronised and *dt receives the step;
 * IGR_ENONFINITE reports rho <= 0, p <= 0 or a non-finite value.  All
 * calls on one device share the array: calls that overlap on one device
 * (on different streams or host threads) race and must not be issued. */
int igr_compute_dt_noalloc(const igr_grid *grid, double gamma, int32_t precision, const void *U, double cfl,
                           double *dt, void *stream);

/* FP64 totals sum_cells U dV of the five conserved variables in a fixed
 * reduction order (synchronises). */
int igr_sums(igr_ctx *ctx, const void *U, double out[5], void *stream);

/* Synchronise the stream and report (and clear) the non-finite flag. */
int igr_check(igr_ctx *ctx, void *stream);

/* Per-kernel timing with HIP events on the call's stream (for measurement
 * only).  igr_timing(ctx, 1) starts recording every launch; 0 stops.
 * igr_kernel_time(ctx, name, &ms, &count) returns the summed duration in
 * milliseconds and the launch count of kernel `name` since recording
 * started (synchronises; names are listed by igr_kernel_name). */
int igr_timing(igr_ctx *ctx, int32_t enable);
int igr_kernel_time(igr_ctx *ctx, const char *name, double *ms, int64_t *count);
const char *igr_kernel_name(int32_t index);

#ifdef __cplusplus
}
#endif

#endif /* IGR_H */
