/*
 * adg.h -- C ABI of libadg, an ADER-DG step engine for AMD Instinct MI355X
 * (gfx950).  The operations follow the ExaHyPE paper (Reinarz et al.,
 * "ExaHyPE: An Engine for Parallel Dynamically Adaptive Simulations of Wave
 * Problems"), Sec. 2-3: the balance law of Eq. (1) with flux,
 * non-conservative product, source and point sources, discretised by
 * ADER-DG (Sec. 3.3: element-local space-time predictor solved by a Picard
 * iteration, Rusanov face flux, corrector Eq. (6) with a diagonal mass
 * matrix) under the time step restriction of Eq. (7) (Sec. 3.4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Mesh: uniform Cartesian, dim = 2 or 3, cells[d] cells on [lo[d], hi[d]],
 *    periodic in every direction.  Cell index c = cx + Cx*(cy + Cy*cz).
 *  - Basis: tensor-product Lagrange polynomials of degree N on the n = N+1
 *    Gauss-Legendre points of each axis (Sec. 3.3).  Node index
 *    k = kx + n*(ky + n*kz), x fastest; S = n^dim nodes per cell.
 *  - State Q: float64 device array [C][nvar][S] (per-cell structure of
 *    arrays).  Material parameters: float64 device array [C][nparam]
 *    (constant per cell; may be NULL when nparam == 0).
 *  - Clock: float64 device array of 2 entries {t, dt}.  Entry points read
 *    and write it on the device, so a sequence of steps needs no host
 *    synchronisation.
 *  - Ownership: every Q / params / clock / flags / output pointer belongs to
 *    the caller, must be device memory of the current HIP device, and is not
 *    retained after the call returns.  The context owns its tables, source
 *    and receiver descriptors and its workspace (face traces, reduction
 *    slots).
 *  - Streams: every device entry point only enqueues work on `stream` (a
 *    hipStream_t; NULL is the null stream) and returns without waiting.
 *    Calls on one context must be ordered (one context per concurrent
 *    stream): the context's workspace is shared by its calls.
 *  - Errors: every entry point returns adg_status.  Arguments are checked
 *    before anything is enqueued; on error nothing is enqueued and
 *    adg_last_error() (thread-local) describes the problem.  Nothing aborts
 *    or throws across the ABI.  Device-side faults surface as ADG_ERR_HIP
 *    from a later call, as with any HIP work.
 */
#ifndef ADG_H
#define ADG_H

#if !defined(__HIPCC_RTC__)
#include <stddef.h>
#include <stdint.h>
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int adg_status;
#define ADG_OK 0
#define ADG_ERR_INVALID_ARG (-1) /* bad pointer, size or configuration value */
#define ADG_ERR_HIP (-2)         /* a HIP runtime call failed (message has the hipError_t) */
#define ADG_ERR_NOMEM (-3)       /* device or host allocation failed */
#define ADG_ERR_UNSUPPORTED (-4) /* valid but not built: order, PDE/dim pair, precision */
#define ADG_ERR_COMPILE (-5)     /* a run-time PDE failed to compile (hiprtc log in the message) */
#define ADG_ERR_STATE (-6)       /* call out of order, e.g. sampling with no receivers set */

/* Built-in PDEs (Sec. 2 and Sec. 6).  Their pointwise terms follow the
 * paper's user-function convention (Sec. 4.1, Table 2): flux(Q, direction),
 * nonConservativeProduct(Q, gradQ), source(Q, x, t), eigenvalues(Q,
 * direction) (the kernels use the largest absolute value) and
 * isPhysicallyAdmissible(Q).
 *  ADG_PDE_EULER      compressible Euler, Eqs. (8) and (10):
 *                     Q = (rho, j_1..j_dim, E), nvar = dim + 2, nparam = 0,
 *                     p = (gamma - 1)(E - |j|^2 / (2 rho)); admissible iff
 *                     rho > 0, p > 0 and finite.
 *  ADG_PDE_ELASTIC    linear elasticity in velocity-stress form (Sec. 2.1),
 *                     dim = 3 only: Q = (sxx, syy, szz, sxy, sxz, syz,
 *                     rho vx, rho vy, rho vz), nvar = 9; params per cell
 *                     (rho, cp, cs), nparam = 3; flux F = (0, sigma),
 *                     non-conservative product E(lambda, mu) grad v with
 *                     lambda = rho (cp^2 - 2 cs^2), mu = rho cs^2.
 *  ADG_PDE_ADVECTION  scalar test PDE: F_d = a_d q, S(q) = -kappa q,
 *                     nvar = 1, nparam = 0. */
#define ADG_PDE_EULER 1
#define ADG_PDE_ELASTIC 2
#define ADG_PDE_ADVECTION 3
#define ADG_PDE_USER 4 /* the PDE of adg_create_user's source text */

/* Arithmetic of the predictor (space-time predictor, time averages, face
 * projection and volume integral).  The time step, the Rusanov face flux,
 * the surface integral and the solution update are always float64, and the
 * state, traces and clock are always stored in float64. */
#define ADG_FP64 0
#define ADG_MIXED_FP32 1
/* FP32 predictor whose derivative contractions of the Picard passes run in
 * split BF16 on the matrix cores: each float operand is the exact sum of
 * three BF16 terms, the six partial products of size >= 2^-16 are
 * accumulated in FP32 (v_mfma_f32_16x16x32_bf16).  Built for the
 * built-in Euler PDEs; elsewhere UNSUPPORTED.  Its error is that of
 * ADG_MIXED_FP32, and on MI355X it runs about 5x slower than ADG_MIXED_FP32
 * (a 6-point contraction fills a 16x16x32 tile poorly and the splits cost
 * as much vector work as the FP32 contraction): a measured alternative, not
 * the recommended mixed-precision form. */
#define ADG_MIXED_BF16X3 2

/* Initial guess of the predictor's Picard iteration (Sec. 3.3; Sec. 5.2 names
 * a continuous extension Runge-Kutta (CERK) guess as the alternative).
 *  ADG_GUESS_CONSTANT  q^0 = u^n at every time node (the default; with
 *                      N + 1 passes the predictor is of order N + 1).
 *  ADG_GUESS_CERK      q^0 = the classical four-stage Runge-Kutta method's
 *                      continuous extension of uniform order three on the
 *                      cell-local ODE dq/dt = R(q, t) of the predictor (the
 *                      cell's derivatives, non-conservative product, sources
 *                      and point sources; no face terms), taken at the time
 *                      nodes; its error is O(dt^4) instead of O(dt), so
 *                      N - 2 passes reach the order of N + 1 passes from the
 *                      constant guess.  Built for the FP64 predictor of the
 *                      built-in PDEs that are not linear in Q (Euler);
 *                      elsewhere UNSUPPORTED. */
#define ADG_GUESS_CONSTANT 0
#define ADG_GUESS_CERK 1

typedef struct {
  int dim;          /* 2 or 3 */
  int order;        /* polynomial degree N >= 1 (built range: adg_max_order) */
  int pde;          /* ADG_PDE_* */
  int precision;    /* ADG_FP64, ADG_MIXED_FP32 or ADG_MIXED_BF16X3 */
  int cells[3];     /* cells per axis (cells[2] ignored for dim 2) */
  double lo[3];     /* domain lower corner */
  double hi[3];     /* domain upper corner */
  double cfl;       /* CFL_N of Eq. (7), 0 < cfl; the paper requires < 1 */
  int picard_iters; /* fixed number of Picard iterations; 0 selects N+1
                       (ADG_GUESS_CONSTANT) or max(1, N-2) (ADG_GUESS_CERK) */
  int initial_guess; /* ADG_GUESS_* (the first Picard iterate) */
  double gamma;     /* Euler ratio of specific heats (> 1) */
  double adv[3];    /* advection velocity */
  double kappa;     /* advection decay rate */
  int bc[6];        /* ADG_BC_* of face 2 d + side (side 1 at the high end of
                       axis d); all ADG_BC_PERIODIC (0) by default */
  double bc_state[6][16]; /* ADG_BC_INFLOW: the outside state of face
                             2 d + side (its first nvar entries) */
} adg_config;

/* Boundary conditions (the boundaryValues user function of the paper's
 * Table 2 supplies the state and normal flux outside a boundary face).
 * Both faces of an axis are periodic, or neither is.  Outside a boundary
 * face the corrector uses, per face node, a state and normal flux built
 * from the cell's own time-averaged traces (qin, Fin):
 *  ADG_BC_OUTFLOW  (qin, Fin): transmissive, no jump across the face;
 *  ADG_BC_WALL     the mirror image: Euler, the normal momentum reversed
 *                  (qout = R qin, Fout = -R Fin, as F_d(R q) = -R F_d(q)):
 *                  a reflecting wall, no mass or energy crosses it;
 *                  elasticity, the traction sigma_{i d} reversed and the
 *                  velocity kept (Fout = -Fin): a traction-free surface.
 *                  Not defined for ADG_PDE_ADVECTION (INVALID_ARG).
 *  ADG_BC_INFLOW   a prescribed outside state, cfg.bc_state of the face
 *                  (constant in time, material parameters the cell's own),
 *                  and its normal flux F_d(qout).
 *  ADG_BC_USER     run-time PDEs only (adg_create_user): the struct's
 *                  boundary_values(x, t, dt, face, Qin, Fin, Qout, Fout),
 *                  the paper's boundaryValues user function, called at every
 *                  node x of the face with the step's start time t and size
 *                  dt and the cell's own trace (Qin with the parameters
 *                  appended, Fin); it returns the outside state and normal
 *                  flux.  The struct declares HAS_BOUNDARY = true.
 * Walls and inflow faces are not offered for run-time PDEs (INVALID_ARG).
 * The adjoint entry points need a periodic mesh; the subcell limiter has no
 * inflow faces (UNSUPPORTED). */
#define ADG_BC_PERIODIC 0
#define ADG_BC_OUTFLOW 1
#define ADG_BC_WALL 2
#define ADG_BC_INFLOW 3
#define ADG_BC_USER 4

/* Sizes derived from a configuration (adg_query). */
typedef struct {
  int nvar, nparam;
  int nodes_per_cell;    /* S = n^dim */
  int face_nodes;        /* n^(dim-1) */
  long long ncells;      /* C */
  long long state_elems; /* C * nvar * S */
  size_t workspace_bytes; /* device bytes the context holds: face traces
                            (each trace array also holding C * nparam
                            doubles for the adjoint where it is built; the
                            second array once adg_run_reserve has run),
                            reduction slots, and the limiter workspace once
                            adg_limiter_reserve has run */
  size_t trace_elems;    /* C * 2 dim * 2 * nvar * face_nodes */
} adg_info;

/* A point source of Eq. (1): delta(x - x_s) * s(t) * weight[v], with s the
 * Ricker wavelet s(t) = amp (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2).
 * The source belongs to the cell whose half-open box [lo, lo + h) holds x. */
typedef struct {
  double x[3];
  double weight[16]; /* per evolved quantity (first nvar entries used) */
  double f0, t0, amp;
} adg_point_source;

typedef struct adg_ctx adg_ctx;

/* Thread-local description of the last error on this thread ("" if none). */
const char* adg_last_error(void);

/* Largest polynomial degree N built for a (pde, dim) pair, 0 if none. */
int adg_max_order(int pde, int dim);

/* Host-only: the one-dimensional tables on [0, 1] for n = order + 1 points:
 * Gauss-Legendre nodes xi[n] and weights w[n] (sum 1), D[n*n] with
 * D[i*n + j] = phi_j'(xi_i), boundary values l0[n] = phi(0), l1[n] = phi(1),
 * and K1inv[n*n], the inverse of the predictor's time matrix
 * K1_ij = phi_i(1) phi_j(1) - int_0^1 phi_i' phi_j (Sec. 3.3, Eq. (5)
 * integrated by parts in time with upwinding from the old time level).
 * Any output pointer may be NULL.  Needs no GPU. */
adg_status adg_basis_tables(int order, double* xi, double* w, double* D, double* l0,
                            double* l1, double* K1inv);

/* Host-only: the tables of the a-posteriori subcell limiter (Sec. 3.5; the
 * projectOnFVLimiterSpace / projectOnDGSpace kernels of Table 1) for
 * n = order + 1 nodes and m = 2 order + 1 equal subcells of [0, 1]:
 * A[s*n + k], the average of phi_k over subcell s; B[k*m + s], the
 * least-squares inverse (A^T A)^{-1} A^T (so B A = I); Qf[k*m + s] =
 * A[s*n + k] / (m w_k), which maps piecewise constant face data to face-node
 * values with the same integral against every basis function.  Needs no
 * GPU. */
adg_status adg_limiter_tables(int order, double* A, double* B, double* Qf);

/* Validate cfg, build the tables, and allocate the workspace on the current
 * HIP device.  *out receives a context owned by the caller, released with
 * adg_destroy.  Errors: INVALID_ARG (bad values), UNSUPPORTED (order or
 * PDE/dim not built), NOMEM, HIP. */
adg_status adg_create(const adg_config* cfg, adg_ctx** out);

/* A context for a PDE given as HIP source text (cfg->pde == ADG_PDE_USER),
 * the run-time counterpart of the user functions of the paper's Table 2
 * (flux, eigenvalues, nonConservativeProduct, algebraicSource,
 * isPhysicallyAdmissible) with the (Q, direction, out) convention of its
 * printed eigenvalues signature.  source (NUL-terminated, not retained)
 * defines
 *
 *   struct AdgUserPDE {
 *     static constexpr int DIM = 2 or 3 (== cfg->dim), NV, NP;  // NV + NP <= 16
 *     static constexpr bool LINEAR, HAS_NCP, HAS_SOURCE;
 *     template <class R> __device__ static void flux(const R* Q, int d, R* F);
 *     template <class R> __device__ static void eigenvalues(const R* Q, int d, R* lam);
 *     template <class R> __device__ static void ncp(const R* Q, const R* gradQ, R* BgradQ);
 *     template <class R> __device__ static void source(const R* Q, R* S);
 *     template <class R> __device__ static bool admissible(const R* Q);
 *   };
 *
 * Q = NV evolved quantities then the cell's NP parameters; F, lam, BgradQ,
 * S: NV entries; gradQ [DIM][NV]; R = double (float in the MIXED_FP32
 * predictor).  The kernels use the largest |lam|.  LINEAR declares flux, ncp
 * and source linear and homogeneous in the evolved quantities (the
 * polynomial form of the predictor is then used).  The library's kernels are
 * compiled for the struct with hiprtc for the current device, once, here
 * (seconds).  Everything else is as for built-in PDEs (nvar, nparam come
 * from the struct, see adg_query), except: no wall boundaries
 * (INVALID_ARG) and no adjoint (UNSUPPORTED).  Errors as adg_create, plus
 * COMPILE with the compiler log in adg_last_error(). */
adg_status adg_create_user(const adg_config* cfg, const char* source, adg_ctx** out);

/* Release the context and its device memory (waits for the device). */
adg_status adg_destroy(adg_ctx* ctx);

/* Sizes of a context's problem. */
adg_status adg_query(const adg_ctx* ctx, adg_info* info);

/* Host-only: physical coordinates of every node, xyz[C][S][dim] (host
 * memory, float64), for pointwise initial data as the paper's
 * adjustPointSolution (Table 2). */
adg_status adg_node_coords(const adg_ctx* ctx, double* xyz);

/* Eq. (7): clock[1] <- cfl / (dim (2N + 1)) * min_d h_d / lambda_max, with
 * lambda_max the largest absolute eigenvalue over all cells, nodes and
 * directions of Q.  clock[0] is not touched.  A NaN eigenvalue bound at any
 * node is not skipped: lambda_max and dt become NaN.  For Euler that is any
 * NaN in Q and any state whose sound speed is the square root of a negative
 * number (e.g. a negative pressure at positive density); the speeds of
 * elasticity (cp of the cell) and advection (|a_d|) do not depend on Q, so a
 * non-finite Q leaves their dt finite: adg_check_admissible detects it. */
adg_status adg_stable_dt(adg_ctx* ctx, const double* Q, const double* params, double* clock,
                         void* stream);

/* Host copy of a device clock {t, dt} (2 doubles): waits for the work
 * queued on stream, then copies (the step path itself never synchronises;
 * this getter does). */
adg_status adg_read_clock_host(const double* clock, double* host, void* stream);

/* One ADER-DG step (Sec. 3.3, three phases) in place: Q <- u^{n+1} with
 * dt = clock[1] and t^n = clock[0]; afterwards clock[0] <- t^n + dt.
 * flags: ADG_STEP_NEXT_DT also evaluates Eq. (7) on u^{n+1} during the
 * update and stores it in clock[1] (bitwise the value adg_stable_dt would
 * give, NaN included); without it clock[1] is left unchanged (a frozen step
 * size).
 * Does not test for non-finite values: that is adg_check_admissible. */
#define ADG_STEP_NEXT_DT 1
#define ADG_STEP_REUSE_RANGES 2  /* adg_step_limited only (see there) */
adg_status adg_step(adg_ctx* ctx, double* Q, const double* params, double* clock, int flags,
                    void* stream);

/* For callers that cannot allocate device memory or use a context's
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the step of adg_step, same kernels, same result
 * bit for bit, with its face traces and reduction slots in the library's
 * static device scratch array (32 MiB of traces plus 16 KiB of slots, held
 * by every GPU the library runs on until the process ends) instead of the
 * context's workspace.  Allocates nothing and does not synchronise; the
 * context's own workspace is not touched.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (several streams, several
 * contexts) race and must be ordered by the caller.  The slots are cleared
 * by a kernel at the start of every call.  Errors: as adg_step, plus
 * UNSUPPORTED when the mesh's face traces (adg_query trace_elems * 8 bytes)
 * exceed 32 MiB. */
adg_status adg_step_noalloc(adg_ctx* ctx, double* Q, const double* params, double* clock, int flags,
                            void* stream);

/* Allocates the second face-trace array that fused runs of adg_run swap
 * with the workspace (trace_elems doubles, see adg_query), once, on the
 * context's device; later calls, and contexts whose runs do not fuse
 * (PDEs not linear in Q, picard_iters > 16, run-time PDEs), do nothing.
 * Synchronous.  Errors: INVALID_ARG (null), STATE (another current device),
 * NOMEM. */
adg_status adg_run_reserve(adg_ctx* ctx);

/* nsteps steps in place with the step size clock[1] held fixed (as in
 * adg_step without ADG_STEP_NEXT_DT; clock[0] advances by dt each step), in
 * the context's precision.  rec_out (device [nsteps][nrec][nvar], or NULL)
 * receives the receiver samples after every step.  For the built-in PDEs
 * linear in Q (elasticity, advection; picard_iters <= 16) the corrector of
 * each step and the predictor of the next run as one kernel (the step
 * fusion of Sec. 5.1: one pass over the state per step instead of two),
 * alternating between the trace workspace and the array of adg_run_reserve
 * (STATE if that was not called); otherwise the steps run one by one.  No
 * allocation and no host synchronisation.  The states are those of nsteps
 * adg_step calls; samples agree with adg_sample_receivers to rounding.
 * Leaves the trace workspace unusable for adg_correct.  Errors:
 * INVALID_ARG (null Q or clock, nsteps < 0, missing params), STATE (no
 * receivers set with rec_out, fused run without adg_run_reserve, another
 * current device), HIP. */
adg_status adg_run(adg_ctx* ctx, double* Q, const double* params, double* clock, int nsteps,
                   double* rec_out, void* stream);

/* The predictor phase alone (Sec. 3.3 phase 1 with the projection onto the
 * faces of Sec. 5.1): Qvol <- u^n + dt (-div Fbar - Nbar + Sbar) per node
 * ([C][nvar][S], may equal Q) and, if traces is not NULL, the face traces
 * traces[C][2 dim][2][nvar][F] with face = 2 d + side (side 0 at the low
 * end of axis d), [0] = time-averaged state, [1] = time-averaged normal
 * flux.  With traces NULL the context's workspace receives what adg_correct
 * reads (for the PDEs with a linear flux, elasticity and advection, only the
 * state traces).  For tests and instrumentation; adg_step is the production
 * path. */
adg_status adg_predict(adg_ctx* ctx, const double* Q, const double* params, const double* clock,
                       double* Qvol, double* traces, void* stream);

/* The corrector phase alone (Sec. 3.3 phases 2 and 3): Rusanov fluxes from
 * the face traces the last adg_predict call on this context left in its
 * workspace, then Q <- Q - dt * (surface integral) and the clock update of
 * adg_step (same flags).  adg_predict(ctx, Q, params, clock, Q, NULL, s)
 * followed by adg_correct(ctx, Q, params, clock, flags, s) is exactly
 * adg_step; the split lets callers time or interleave the two kernels.
 * STATE error if no adg_predict with workspace traces preceded it. */
adg_status adg_correct(adg_ctx* ctx, double* Q, const double* params, double* clock, int flags,
                       void* stream);

/* Allocates the workspace of adg_step_limited on the context's device (a
 * copy of u^n and the FV face fluxes, 1 + 2 dim / (order + 1) state arrays,
 * plus 32 nvar + 10 bytes per cell, and the limiter tables), once; later
 * calls do nothing.  Synchronous; the step itself then allocates nothing.
 * Errors: INVALID_ARG (null context; limiter tables not constructible),
 * UNSUPPORTED where adg_step_limited is not built (not Euler, an order
 * above the limit, inflow faces, run-time PDEs, more than 2^31 - 1 cells),
 * NOMEM, HIP, STATE (another current device). */
adg_status adg_limiter_reserve(adg_ctx* ctx);

/* One step with the a-posteriori subcell limiter (Sec. 3.5, the hybrid
 * ADER-DG/FV method with the status stencil of Fig. 2), in place, for the
 * Euler equations (2-D N <= 7, 3-D N <= 3; else ADG_ERR_UNSUPPORTED):
 *   1. the unlimited step of adg_step gives a candidate in every cell;
 *   2. a cell is troubled if the candidate fails the physical admissibility
 *      test at a node or a subcell average, or the relaxed discrete maximum
 *      principle: its subcell averages must lie within the range of the
 *      subcell averages at t^n of the cell and its face neighbours, widened
 *      by max(1e-4, 1e-3 * range) per variable;
 *   3. troubled cells and their face neighbours take a MUSCL-Hancock step
 *      (minmod slopes, Rusanov fluxes) on their m^dim subcells, m =
 *      2 order + 1, from the subcell averages at t^n (for a cell that was
 *      FV already, its FV data; else the averages of its polynomial), and
 *      their DG polynomial becomes the least-squares fit of the result;
 *   4. DG cells that share a face with an FV cell take the FV flux through
 *      that face in place of the Rusanov flux of step 1, so the step
 *      conserves what the PDE conserves.
 * Q [C][nvar][S] device, in/out.  clock as for adg_step (t advances by dt;
 * flags ADG_STEP_NEXT_DT evaluates Eq. (7) on the limited u^{n+1}, the
 * signal speed of an FV cell taken over its subcell averages, of a DG cell
 * over its nodes).
 * status [C] uint8 device, in/out: 0 DG, 1 DG with an FV face, 2 FV as a
 * neighbour of a troubled cell, 3 troubled (FV); zero it before the first
 * step (or mark cells that start on FV with 3 and give their data in
 * sub_in).  sub_in, sub_out [C][nvar][m^dim] device, x fastest: the FV
 * subcell averages at t^n and t^{n+1}; only the entries of cells with
 * status >= 2 are read (sub_in, status before the step) or written
 * (sub_out, status after it); they must be distinct arrays, and a run
 * swaps them every step.  counts: device int32[3] (troubled cells, FV
 * cells, DG cells with an FV face), or NULL.  The context's limiter
 * workspace comes from adg_limiter_reserve (STATE without it).  Calls on
 * one context must not overlap.  No allocation and no host synchronisation,
 * so the status values are not checked: the caller keeps them in 0..3.
 * flags ADG_STEP_REUSE_RANGES: the caller's Q, status and sub_in are
 * exactly what the previous adg_step_limited on this context left in Q,
 * status and sub_out (a run of limited steps with nothing else touching
 * them).  The call then takes the t^n range of every cell with status 0
 * from the subcell averages the previous call computed for its candidate
 * (which is that cell's u^n) instead of projecting u^n again, and stores
 * its own candidate's ranges for the next call; results are bitwise those
 * without the flag.  The stored ranges are used only if the previous call
 * on the context set the flag too; a state changed in between with the
 * flag set gives wrong ranges.
 * Errors: INVALID_ARG (null arrays, sub_in == sub_out, unknown flags),
 * UNSUPPORTED (not Euler, an order above the limit, inflow faces, run-time
 * PDEs), STATE (no workspace reserved), HIP (launches). */
adg_status adg_step_limited(adg_ctx* ctx, double* Q, double* clock, const double* sub_in, double* sub_out,
                            uint8_t* status, int32_t* counts, int flags, void* stream);

/* A-posteriori physical admissibility (Sec. 3.5): troubled[c] <- 1 if any
 * node of cell c is non-finite or fails the PDE's admissibility test, else
 * 0; *count <- number of troubled cells (device int32). */
adg_status adg_check_admissible(adg_ctx* ctx, const double* Q, const double* params,
                                uint8_t* troubled, int32_t* count, void* stream);

/* Replace the context's point sources (host array of n <= 16 entries;
 * n = 0 clears).  Synchronous upload. */
adg_status adg_set_point_sources(adg_ctx* ctx, int n, const adg_point_source* src);

/* Replace the receiver set: n points xyz[n][3] (host), each inside the
 * domain.  Synchronous upload of per-receiver interpolation weights. */
adg_status adg_set_receivers(adg_ctx* ctx, int n, const double* xyz);

/* out[r][v] <- sum_k Phi_k(xi_r) Q[c_r][v][k]: the degree-N polynomial of
 * the receiver's cell evaluated at the receiver (device output [n][nvar]). */
adg_status adg_sample_receivers(adg_ctx* ctx, const double* Q, double* out, void* stream);

/* ---- Discrete adjoint (for gradients of functionals of the solution) ----
 *
 * The FP64 step of adg_step with the step size held fixed is, for PDEs
 * linear in Q, an affine map u^{n+1} = A(m) u^n + b(t) of the state, m the
 * per-cell material parameters (point sources make up b).  These two calls
 * are the exact transposes (up to rounding) of that map and of receiver
 * sampling, so that a caller can run a reverse sweep: with
 * lam = dJ/du^{n+1}, adg_step_adjoint gives dJ/du^n and dJ/dm.  The inner
 * products are the plain Euclidean ones over the nodal arrays (a discrete
 * adjoint, not a discretised continuous adjoint).  Reading: where the two
 * cells of a face have the same largest eigenvalue, the derivative of the
 * Rusanov speed max() is split half and half between them. */

/* One adjoint step, reverse of the step that took Q = u^n to u^{n+1} with
 * the clock {t^n, dt} (device, read only; the same values the forward step
 * used).
 *   Q        [C][nvar][S] device, the forward state u^n (read only)
 *   params   [C][nparam] device (NULL iff nparam == 0)
 *   lam      [C][nvar][S] device, in: dJ/du^{n+1}, out: dJ/du^n (in place)
 *   gparams  [C][nparam] device, dJ/dm of this step is ADDED (NULL iff
 *            nparam == 0)
 * Available for ADG_PDE_ELASTIC and ADG_PDE_ADVECTION at every built order
 * with picard_iters <= order + 1 on a periodic mesh; otherwise
 * (ADG_PDE_EULER, more Picard iterations, boundaries) ADG_ERR_UNSUPPORTED.  Deterministic (no atomics).  Uses the context's
 * trace workspace: a following adg_correct needs a new adg_predict. */
adg_status adg_step_adjoint(adg_ctx* ctx, const double* Q, const double* params,
                            const double* clock, double* lam, double* gparams, void* stream);

/* The same adjoint step without recomputing the forward predictor: a
 * reverse sweep that keeps, per step, what the step's adjoint reads of the
 * forward predictor (the Horner iterates of the linear predictor's time
 * average, Sec. 3.3 / Eq. 5 in its polynomial form, in the channels whose
 * gradient the non-conservative product reads, and the time average itself)
 * needs neither u^n nor the forward sweep inside the adjoint step.
 *
 * adg_keep_size: *n <- doubles of one step's keep buffer ([C][slots][S]
 *   per-node quantities, then the step's face traces in the layout of
 *   adg_predict's traces, trace_elems of adg_info).
 * adg_step_keep: one FP64 step of adg_step (flags 0: the step size in clock
 *   is kept) that also writes the step's keep buffer (device, caller-owned,
 *   *n doubles; overwritten).  Its face traces go to the keep buffer, not
 *   to the context's workspace (a following adg_correct needs a new
 *   adg_predict).
 * adg_run_keep: adg_run of nsteps steps (rec_out as there; fused
 *   corrector/predictor kernels where built, after adg_run_reserve) that
 *   writes step n's keep buffer at keeps + n *n (device, caller-owned,
 *   nsteps *n doubles); the states and buffers equal those of nsteps
 *   adg_step_keep, the samples those of adg_run.
 * adg_step_adjoint_kept: adg_step_adjoint of that step from its keep buffer
 *   (device, read only) instead of Q; lam, gparams, clock as there.  lam
 *   equals adg_step_adjoint's (the same arithmetic on the same values);
 *   gparams equals it to rounding (the Rusanov flux's two transposes run
 *   as one pass over the faces, on the kept traces, and its compiled
 *   products may round differently).
 * Available where adg_step_adjoint is, for ADG_FP64 contexts; otherwise
 * ADG_ERR_UNSUPPORTED; a NULL buffer is ADG_ERR_INVALID_ARG. */
adg_status adg_keep_size(const adg_ctx* ctx, long long* n);
adg_status adg_step_keep(adg_ctx* ctx, double* Q, const double* params, double* clock, double* keep,
                         void* stream);
adg_status adg_run_keep(adg_ctx* ctx, double* Q, const double* params, double* clock, int nsteps,
                        double* rec_out, double* keeps, void* stream);
adg_status adg_step_adjoint_kept(adg_ctx* ctx, const double* params, const double* clock,
                                 const double* keep, double* lam, double* gparams, void* stream);

/* Transpose of adg_sample_receivers: lam[c_r][v][k] += Phi_k(xi_r) lamrec[r][v]
 * for every receiver r (device lamrec [n][nvar], lam [C][nvar][S]).
 * Receivers in the same cell add in receiver order (deterministic). */
adg_status adg_sample_receivers_adjoint(adg_ctx* ctx, const double* lamrec, double* lam,
                                        void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ADG_H */
