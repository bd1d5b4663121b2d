/*
 * fld.h - C ABI of the MI355X implicit flux-limited-diffusion (FLD) radiation step.
 *
 * One call of fld_step advances the radiation energy density E_r and the gas
 * temperature T_g of a 2D finite-volume grid by one backward-Euler step of the
 * coupled system of Chen et al. ("Guangqi"), Section 3.2.1:
 *
 *   radiation row : phi_1..phi_11 (5-point stencil in E, local T coupling),
 *   gas row       : psi_5, psi_6, psi_11 (local),
 *   with the FLD closure F = -D grad E, D = c lambda(R) / (kappa_R rho)
 *   (Section 2) and (T^{n+1})^4 linearised about T^n.
 *
 * The library eliminates T exactly, solves the resulting symmetric positive
 * definite E system (volume-weighted rows) with matrix-free conjugate gradients
 * preconditioned by a geometric-multigrid V-cycle, optionally in FP32 inside
 * an FP64 iterative-refinement loop, and recovers T^{n+1} from the psi row.
 *
 * Conventions (all entry points):
 *  - Cell arrays are row-major [ny][nx] (x or r fastest), IEEE binary64,
 *    DEVICE pointers owned by the caller.  They must stay valid until the work
 *    queued on the context's stream has finished.
 *  - Every call is queued on the stream given to fld_create (a hipStream_t;
 *    NULL = the default stream).  A call that returns a fld_solve_info, or
 *    that must test convergence, synchronises that stream.
 *  - The context owns all workspace; it is allocated in fld_create /
 *    fld_batch_create.  Only these other entry points allocate device
 *    memory: fld_set_cv_law (one array of nx*ny doubles, on the first call
 *    with p != 0, kept until fld_destroy) and the tuners fld_tune /
 *    fld_batch_tune (a context per candidate and scratch copies of E and T,
 *    freed before they return).  Assembly, solve, step, multi-step and
 *    sub-step calls allocate nothing.
 *  - Errors are returned as fld_status, never thrown; fld_last_error gives a
 *    human-readable message.  Contexts are not thread-safe: use one per stream.
 *  - Units are cgs.  The azimuthal factor 2 pi of spherical-polar volumes and
 *    areas is dropped throughout (it cancels).
 */
#ifndef FLD_H
#define FLD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fld_ctx fld_ctx;

typedef enum {
    FLD_OK = 0,
    FLD_EINVAL = 1,        /* bad argument: sizes, pointers, dt <= 0, unknown enum value     */
    FLD_ENOMEM = 2,        /* device or pinned allocation failed (create, set_cv_law, tuners) */
    FLD_EHIP = 3,          /* a HIP runtime call failed                                        */
    FLD_ENOCONV = 4,       /* tolerance not reached within max_inner iterations (or stalled)   */
    FLD_EBREAKDOWN = 5,    /* CG breakdown: p.Ap <= 0 or non-finite scalar                     */
    FLD_ENONFINITE = 6,    /* an input field is non-finite or outside its domain (E,T,rho,    */
                           /* kappa_R > 0; kappa_P, c_v >= 0), detected on the device          */
    FLD_ENOTREADY = 7      /* fld_solve / fld_get_operator called before fld_assemble          */
} fld_status;

/* Grid geometry: Cartesian (x, y) or spherical-polar (r, theta), Section 3.2. */
typedef enum { FLD_CARTESIAN = 0, FLD_SPHERICAL_POLAR = 1 } fld_geom;

/* Boundary condition of one side.  Interior faces follow the paper's
 * interface coefficient (Section 3.2.1); the paper prints only zero-gradient
 * and Milne boundaries, so the kinds below are this library's readings:
 *   REFLECT         zero flux (zero-gradient radiation boundary, Section 5.2.2).
 *   DIRICHLET_FACE  E = a_R value^4 on the face (value = boundary temperature, K);
 *                   face opacity = first cell's, distance = centre to face.
 *   DIRICHLET_GHOST ghost cell mirrored across the face holding E from the
 *                   ghost_E array passed to fld_assemble / fld_step.
 *   FLUX_IN         fixed inward flux, value = F_in [erg cm^-2 s^-1].
 *   FREE_STREAM     outward flux c E of the first cell.
 *   AXIS            theta = 0 or pi of a spherical-polar grid: zero area, zero flux.
 *   MILNE           the paper's blackbody-absorber condition E = -2/(3 rho kappa_R)
 *                   dE/dn on the face (Section 5.2, radiative shock with the
 *                   hydrogen EoS), first cell's opacity, dE/dn = (E_b - E_1)/h1
 *                   (h1: centre to face): outward flux D E_1/(h1 (1 + a)),
 *                   a = 2/(3 sigma_1 h1), D = c lambda(3/2)/sigma_1 (R is 3/2
 *                   on such a face); value unused.  Single grids only. */
typedef enum {
    FLD_BC_REFLECT = 0, FLD_BC_DIRICHLET_FACE = 1, FLD_BC_DIRICHLET_GHOST = 2,
    FLD_BC_FLUX_IN = 3, FLD_BC_FREE_STREAM = 4, FLD_BC_AXIS = 5, FLD_BC_MILNE = 6
} fld_bc_kind;

/* Side order in fld_grid.bc and in the packed ghost array:
 *   0 = x_lo (ny values), 1 = x_hi (ny), 2 = y_lo (nx), 3 = y_hi (nx). */
typedef struct { int32_t kind; double value; } fld_bc;

typedef struct {
    int32_t nx, ny;            /* cells; 1 <= nx, ny; nx * ny <= 2^28                       */
    int32_t geom;              /* fld_geom                                                   */
    const double* x_faces;     /* HOST array of nx+1 increasing face coordinates (cm; r > 0) */
    const double* y_faces;     /* HOST array of ny+1 increasing faces (cm, or radians in [0, pi]) */
    fld_bc bc[4];
} fld_grid;

/* Inner (Krylov / multigrid) precision.
 *   FP64  : all arithmetic and storage in binary64.
 *   FP32  : one binary32 solve of the correction equation, no refinement.
 *   MIXED : binary32 storage and arithmetic inside CG and the V-cycle; residuals,
 *           norms, dot-product accumulation, the T^4 linearisation and the
 *           solution update in binary64 (iterative refinement). */
typedef enum { FLD_FP64 = 0, FLD_FP32 = 1, FLD_MIXED = 2 } fld_precision;

/* Flux limiter lambda(R), Section 2: Levermore-Pomraning (coth R - 1/R)/R
 * (default), the paper's Minerbo-type piecewise form, or the pure-diffusion
 * value 1/3. */
typedef enum { FLD_LIMITER_LP = 0, FLD_LIMITER_MINERBO = 1, FLD_LIMITER_DIFFUSION = 2 } fld_limiter;

/* Stopping norm (Section 3.2.1 stop rule ||b - A x|| < eps ||b||):
 *   ROW    : per-volume rows, ||(rhs - M E)/dV||_2 <= eps ||rhs/dV||_2 (the phi rows);
 *   SCALED : Jacobi-scaled rows, ||S (rhs - M E)||_2 <= eps ||S rhs||_2, S = diag(M)^-1/2. */
typedef enum { FLD_NORM_ROW = 0, FLD_NORM_SCALED = 1 } fld_norm;

/* Multigrid coarse operator: GALERKIN = P^T A P with 2x2 piecewise-constant
 * aggregation; HALVED = same aggregation with the coarse face conductances
 * halved (rescaled to the coarse spacing; masses still summed). */
typedef enum { FLD_MG_GALERKIN = 0, FLD_MG_HALVED = 1 } fld_mg_coarse;

/* Multigrid smoother: alternating zebra line Gauss-Seidel (x lines then y
 * lines; robust to the strong anisotropy of optically thin spherical shells),
 * or point red-black Gauss-Seidel.  LINE runs both zebra half-sweeps of one
 * direction in a single launch where a band of rows fits in LDS (same result
 * as LINE_SPLIT up to the summation order of r.z); LINE_SPLIT launches every
 * half-sweep separately. */
typedef enum { FLD_SMOOTH_LINE = 0, FLD_SMOOTH_POINT = 1, FLD_SMOOTH_LINE_SPLIT = 2 } fld_smoother;

/* Multigrid cycle.  V: one pass down and up.  K: as V, but the coarse problem
 * of the last launched grid level (the first level of the one-workgroup LDS
 * sub-cycle) is solved by two steps of flexible CG, each preconditioned by the
 * sub-cycle's V-cycle (the Krylov-accelerated K-cycle of Notay and
 * Vassilevski, 2008).  With piecewise-constant aggregation the V-cycle loses
 * convergence as levels are added; the K-cycle restores most of it at the cost
 * of a second pass through the LDS levels only.  W2: the same two passes with
 * fixed coefficients, x = c1 + V(b - A c1) (a linear, symmetric
 * preconditioner; measured better than K on the 1e8-contrast spherical
 * stress grid, worse on the stretched Cartesian one).  W2 is positive
 * definite only where the V-cycle converges as a stationary iteration
 * (spectral radius of I - V A below one): on thin theta slabs of the stress
 * grid (4096 x 64 .. 128 rows about the equator) it is not, and CG then
 * stops with FLD_EBREAKDOWN; K and V have no such condition.  K and W2 act
 * as V where a line smoother has no LDS sub-cycle (fewer than three levels,
 * point smoothing, or a coarsest level above 256 cells, which is solved
 * exactly).  KL_K and KL_W2 make every second launched level (levels 1, 3,
 * 5, ... above the coarse solve) Krylov-accelerated: its coarse problem is
 * solved by two flexible-CG steps, each preconditioned by the cycle from
 * that level down (the sub-cycle entered as K or W2; the two are the same
 * above an exact coarsest solve), so that the coarse correction takes its
 * A-norm best scale instead of the aggregated operator's (a K-cycle over the
 * launched levels; each such level doubles the work below it; acts as K or
 * W2 where fewer than three levels are launched). */
typedef enum { FLD_MG_CYCLE_V = 0, FLD_MG_CYCLE_K = 1, FLD_MG_CYCLE_W2 = 2, FLD_MG_CYCLE_KL_K = 3,
               FLD_MG_CYCLE_KL_W2 = 4 } fld_mg_cycle;

typedef struct {
    int32_t precision;      /* fld_precision (default MIXED)                                 */
    int32_t limiter;        /* fld_limiter (default LP)                                      */
    int32_t norm;           /* fld_norm (default ROW)                                        */
    double  rel_tol;        /* eps of the stop rule (default 1e-10)                          */
    int32_t max_outer;      /* unused, kept for layout; must be >= 1 (default 8): the FP64   */
                            /* residual checks of the reliable-update solver are triggered   */
                            /* by the inner residual, not counted                            */
    int32_t max_inner;      /* CG iterations per solve, all checks included (default 2000)   */
    double  inner_rtol;     /* FP32 mode only: stop once the inner (FP32) residual has       */
                            /* dropped by this factor (default 1e-5)                         */
    int32_t mg_coarse_max;  /* coarsest level size in cells, solved exactly (1..4096, def 64): up to
                               256 cells by one workgroup (inside the LDS sub-cycle with a line
                               smoother), above that by its dense inverse, formed on the GPU at each
                               assembly (block cyclic reduction over the lines along the shorter
                               grid direction) and applied by a multi-workgroup product; the LDS
                               sub-cycle is then not used (inverse: nc^2 inner-precision words,
                               nc = the level's cells, plus (11 min(nx, ny) + 3) nc doubles of
                               set-up workspace, and nc^2 more doubles when the inner precision
                               is FP32)                                                       */
    int32_t mg_coarse_op;   /* fld_mg_coarse (default HALVED)                                */
    int32_t smoother;       /* fld_smoother (default LINE); LINE* need nx, ny <= 4096        */
    int32_t chunk;          /* CG iterations queued between host convergence checks (def 8) */
    int32_t use_graph;      /* capture each chunk as a hipGraph (default 1)                  */
    int32_t mg_cycle;       /* fld_mg_cycle (default K; the batch runs V)                    */
} fld_options;

typedef struct {
    int32_t status;         /* fld_status of the solve                                       */
    int32_t outer_iters;    /* refinement steps taken                                        */
    int32_t inner_iters;    /* CG iterations summed over refinement steps                    */
    int32_t mg_levels;      /* multigrid levels (fine level included)                        */
    double  rel_resid;      /* final relative residual in the selected norm (FP64)           */
    double  rel_resid_row;  /* final relative residual in the ROW norm                       */
    double  rel_resid_scaled; /* final relative residual in the SCALED norm                 */
    float   ms;             /* wall time of the call, host clock, ms                         */
} fld_solve_info;

/* Fills *opt with the defaults listed above. */
void fld_default_options(fld_options* opt);

/* Creates a context for one grid.  Computes the grid metrics (cell volumes,
 * face areas, volume-centre distances; Section 3.2.1 g = dS/dV and alpha) on
 * the device and allocates all workspace.  grid->x_faces / y_faces are read
 * during the call only.  stream: hipStream_t (NULL = default stream).
 * opt may be NULL (defaults).  Returns EINVAL for bad sizes / enums / faces,
 * ENOMEM, EHIP. */
fld_status fld_create(fld_ctx** out, const fld_grid* grid, const fld_options* opt, void* stream);

/* Assembles the system of one step (Section 3.2.1 coefficient list, eliminated
 * T; Section 3.2.1 steps 2-5): face conductances W = dt dS D / h, the diagonal
 * dV (1 + beta f) + sum W + boundary terms, the right-hand side
 * dV (E^n + beta f a_R T^4) + boundary terms, the Jacobi scaling and the
 * multigrid hierarchy.  beta = kappa_P rho c dt, f = C_V / (C_V + 4 beta a_R T^3),
 * C_V = rho c_v.  Inputs are device arrays of nx*ny doubles; ghost_E (device,
 * 2 ny + 2 nx doubles, side order as above) is read only for DIRICHLET_GHOST
 * sides and may be NULL otherwise.  The context keeps the T, rho, kappa_P, c_v
 * pointers for the gas update of fld_step; they must not change before it.
 * Asynchronous; invalid field values are reported by the next fld_solve. */
fld_status fld_assemble(fld_ctx* ctx, const double* E_r, const double* T_g, const double* rho,
                        const double* kappa_R, const double* kappa_P, const double* c_v,
                        const double* ghost_E, double dt);

/* Solves the assembled system (Section 3.2.1 step 6).  E_new (device, nx*ny):
 * on entry the initial guess (e.g. E^n), on return E^{n+1}.  info (host) may be
 * NULL.  Synchronises the context's stream.  Returns ENOCONV / EBREAKDOWN /
 * ENONFINITE as described above (E_new then holds the last iterate), EINVAL
 * on a context that has replayed fld_steps_graph. */
fld_status fld_solve(fld_ctx* ctx, double* E_new, fld_solve_info* info);

/* Gas update from the psi row (Section 3.2.1 psi_5, psi_6, psi_11):
 * T^{n+1} = (C_V T^n + 3 beta a_R T^4 + beta E^{n+1}) / (C_V + 4 beta a_R T^3),
 * using the T^n, rho, kappa_P, c_v pointers of the last fld_assemble and
 * writing T^{n+1} to T_out (device, may alias that T^n).  Asynchronous. */
fld_status fld_gas_update(fld_ctx* ctx, const double* E_new, double* T_out);

/* One implicit radiation step = assemble + solve + gas update.  E_r and T_g
 * are updated in place (device).  info may be NULL.  EINVAL on a context that
 * has replayed fld_steps_graph. */
fld_status fld_step(fld_ctx* ctx, double* E_r, double* T_g, const double* rho, const double* kappa_R,
                    const double* kappa_P, const double* c_v, const double* ghost_E, double dt,
                    fld_solve_info* info);

/* nsteps consecutive steps with (E, T) <- (E^{n+1}, T^{n+1}) and the opacities,
 * rho and c_v held fixed (Section 3.2.1 sub-step loop, one sub-step per step).
 * Every step queues the kernels of fld_step (assembly, hierarchy, solve
 * prologue, CG iterations, final correction, gas update) and a device-side
 * status record, without fld_step's blocking synchronisations: the CG
 * iterations run as a captured graph of two iteration slots with device-side
 * early exit, launched repeatedly; after each launch the solver flags are
 * copied to one of two pinned host mirrors, and the host reads a chunk's
 * flags while the next chunk already runs, so the GPU never waits for the
 * host and at most one chunk of early-exit slots follows convergence (the
 * iteration limit is max_inner).  The host reads the step records once per 8
 * steps.  Results equal those of nsteps fld_step calls bit for bit.  A step
 * that fails (no convergence within max_inner, stagnation, breakdown,
 * non-finite input) is recorded and, unlike fld_step, its gas update and the
 * following steps still run.  With profiling on or use_graph = 0 the steps
 * run as fld_step calls and stop at the first failure.  The pinned mirrors
 * and the device step records belong to the context (allocated by
 * fld_create); the call allocates no device memory.  per_step (host, nsteps
 * entries) may be NULL; each step's ms is the mean over the call.  Returns
 * the first non-OK step status; EINVAL on a context that has replayed
 * fld_steps_graph (below). */
fld_status fld_steps(fld_ctx* ctx, int32_t nsteps, double* E_r, double* T_g, const double* rho,
                     const double* kappa_R, const double* kappa_P, const double* c_v,
                     const double* ghost_E, double dt, fld_solve_info* per_step);

/* The same steps with one whole step captured as a hipGraph.  The first step
 * runs as fld_step; its CG iteration count k1 fixes a budget
 * S = min(max_inner, even(2 k1 + 16)) iterations.  One whole step (assembly,
 * hierarchy, S iteration slots with device-side early exit, gas update, a
 * device-side status record) is then captured once and replayed for the
 * remaining steps in segments of 1, 2, 4, then 8 launches, with no host
 * work inside a segment; the host reads the records once per segment.  If a
 * step used up the budget, the budget grows by half (up to max_inner), the
 * step is re-captured and the segment replays from the (E, T) saved at its
 * start, segments restarting at one step; if the budget exceeds
 * 1.5 x even(k + max(4, k/4) + 2), k the most iterations a step of the last
 * segment took, it is cut to that value and the step re-captured.  Unused
 * slots cost their early-exit launches, so on grids whose iterations are
 * expensive fld_steps is faster (4096 x 2048 stress steps: 24.6 against
 * 32.6 ms); results are the same bit for bit.  The saved copy of E and T
 * belongs to the context.  Once a captured step has been replayed, the
 * context serves only further fld_steps_graph calls: fld_step, fld_solve,
 * fld_steps and fld_substep return EINVAL on it (runs of single steps on such
 * a context ended in a host heap-corruption abort whose cause is not
 * established).  Other arguments, records and return values as fld_steps. */
fld_status fld_steps_graph(fld_ctx* ctx, int32_t nsteps, double* E_r, double* T_g, const double* rho,
                           const double* kappa_R, const double* kappa_P, const double* c_v,
                           const double* ghost_E, double dt, fld_solve_info* per_step);

/* One radiation step of length dt taken as sub-steps, in the order of the
 * radiation-subsystem algorithm of Section 3.2.1: the advection term S_adv
 * (step 1) and the face coefficients D of every interior and boundary face
 * (step 2) are evaluated once, from the E^n passed in (the context keeps a
 * copy); every sub-step then recomputes C_V (step 3, see fld_set_cv_law),
 * builds the coefficients for its own length dt_k (alpha = dt_k / h,
 * beta = kappa_P rho c dt_k, the conductances dt_k dS D^n / h, the boundary
 * terms and dt_k dV S_adv), solves, and updates T (steps 4-6), E and T
 * advancing in place, opacities and rho held fixed (step 7 returns to step 3).
 * Sub-step lengths:
 *   dbar == 0: the prescribed geometric series dt_i = dt_0 q^(i-1),
 *              i = 1..n_sub, dt_0 = dt (1 - q) / (1 - q^n_sub) (the paper asks
 *              for 1 < q < 2; any q > 0 is accepted, q = 1 giving n_sub equal
 *              sub-steps and n_sub = 1 the step itself);
 *   dbar > 0:  coupling-limited sub-steps dt_k = min(dt_remaining,
 *              min over cells of dbar T C_V / |G0|), G0 = kappa_P rho c
 *              (a_R T^4 - E), C_V = rho c_v, from the state at the start of
 *              each sub-step (a cell with G0 = 0 does not limit; the paper
 *              suggests dbar < 0.1); the loop ends once the remaining time is
 *              at most 1e-12 dt.  Each sub-step's limit is a device reduction
 *              read back by the host.
 * dts, per_sub (host arrays of max_sub entries, may be NULL) receive each
 * sub-step's length and solve record; *n_done (may be NULL) the number of
 * sub-steps taken.  Fx, Fy (device, layouts of fld_face_flux, may be NULL)
 * receive the face fluxes averaged over the sub-steps, sum_k (dt_k / dt) F_k
 * with F_k = -D^n (E_hi^k - E_lo^k) / h (the paper's flux formula, D^n
 * outside the sum over the sub-cycle; boundary faces from their fixed terms).
 * With one sub-step the result equals fld_step's bit for bit.  Returns EINVAL for bad parameters (max_sub < 1, dbar < 0,
 * geometric with n_sub outside 1..max_sub or q <= 0) or fields, ENOCONV if the
 * coupling-limited loop needs more than max_sub sub-steps (E, T then hold the
 * state after max_sub of them), ENONFINITE if a limit is not positive, else
 * the first failing sub-step's status (the later ones are not taken). */
fld_status fld_substep(fld_ctx* ctx, double* E_r, double* T_g, const double* rho, const double* kappa_R,
                       const double* kappa_P, const double* c_v, const double* ghost_E, double dt, int32_t n_sub,
                       double q, double dbar, int32_t max_sub, double* dts, fld_solve_info* per_sub,
                       int32_t* n_done, double* Fx, double* Fy);

/* Radiative flux F through every face after a step (Section 3.2.1 flux
 * formula), from the context's last assembly and E (device, the step's
 * E^{n+1}), positive along +x / +y: Fx [ny][nx+1] (face i below cell i along
 * x), Fy [ny+1][nx] (device arrays, either may be NULL).  An interior face
 * carries W (E_lo - E_hi) / (dt dS) = -D (E_hi - E_lo) / h with the step's
 * conductance; a boundary face the outward flux that its side's boundary terms
 * put into the rows, negated on the lower sides; faces of zero area (the axis)
 * carry none.  Without gas coupling these fluxes close each cell's balance,
 * dV (E^{n+1} - E^n) = -dt sum over faces of F dS outward.  Writes w F
 * (accumulate == 0) or adds it (accumulate != 0), so a caller can average over
 * sub-steps (fld_substep does this itself).  Queued on the context's stream.
 * Returns ENOTREADY before an assembly, EINVAL for a NULL ctx or E. */
fld_status fld_face_flux(fld_ctx* ctx, const double* E_r, double* Fx, double* Fy, double w, int32_t accumulate);

/* Face mass fluxes f = rho v of the explicit radiation advection term
 * (Section 3.2.1 advection equation; the mass fluxes come from the hydro
 * step's Riemann solutions): every later assembly of this context (fld_assemble,
 * fld_step, fld_steps, fld_substep) adds dt dV S_adv to its right-hand side,
 * dV S_adv = sum over the cell's faces of +-dS f e_r (inflow through the
 * lower x / y face positive), e_r = E / rho taken from the upwind cell and,
 * at a boundary face, from the boundary cell itself (zero-gradient e_r).
 * fx: device array [ny][nx+1], the flux through x face i of row j (face i
 * lies below cell i along x; positive along +x); fy: [ny+1][nx], through y
 * face j below cell row j (positive along +y).  Either may be NULL (no flux
 * in that direction); both NULL turns advection off (the default).  The
 * arrays stay owned by the caller and are read at each assembly, so they
 * must stay valid (and hold finite values: else the assembly reports
 * ENONFINITE) while set; a multi-step graph reads the arrays set when
 * fld_steps was called.  Returns EINVAL for a NULL ctx. */
fld_status fld_set_mass_flux(fld_ctx* ctx, const double* fx, const double* fy);

/* Temperature-dependent heat capacity (Section 3.2.1: the radiation-subsystem
 * algorithm recomputes C_V before every sub-step; Section 5.1.2: a nonlinear
 * gas energy enters linearised, C_V = de_g/dT).  With p != 0 every later
 * assembly of this context (fld_assemble, fld_step, fld_steps, each sub-step
 * of fld_substep and its coupling limit) uses, instead of the c_v array it is
 * given, the power law
 *     c_v(T) = c_v[c] (T[c] / T_ref)^p
 * evaluated from that step's T^n (the c_v array then holds each cell's value
 * at T_ref), and the gas update uses the same values: an analytic stand-in for
 * a nonlinear equation of state.  p == 0 turns the law off (the default).
 * The first call with p != 0 allocates one array of nx*ny doubles, kept
 * until fld_destroy.  The batched blocks do not use the law.  Returns EINVAL
 * for a NULL ctx, T_ref <= 0 or a non-finite T_ref or p, ENOMEM if that array
 * cannot be allocated. */
fld_status fld_set_cv_law(fld_ctx* ctx, double T_ref, double p);

/* Copies the assembled FP64 operator of the last fld_assemble to caller device
 * arrays of nx*ny doubles (any may be NULL): W_e[j][i] = conductance of the
 * face between cells i and i+1 (0 in the last column), W_n[j][i] = face between
 * rows j and j+1 (0 in the last row), diag = full diagonal, rhs.  For tests. */
fld_status fld_get_operator(fld_ctx* ctx, double* W_e, double* W_n, double* diag, double* rhs);

/* Number of multigrid levels built by the last fld_assemble (fine included). */
int32_t fld_mg_levels(const fld_ctx* ctx);

/* Measurement of the dominant kernel family (the multigrid line-sweep
 * kernels).  While enabled, every such launch is bracketed by HIP events on
 * the context's stream (CG chunks then run as plain launches, not graphs).
 * fld_profile_read synchronises, and returns the number of timed launches that
 * did work (launches that exited early after convergence are excluded), their
 * summed duration in ms, and their summed algorithmic bytes (compulsory reads
 * and writes of each launch).  Enabling resets the totals. */
fld_status fld_profile(fld_ctx* ctx, int32_t enable);
fld_status fld_profile_read(fld_ctx* ctx, int64_t* launches, double* total_ms, double* bytes);
/* Mean elapsed time (us) of the same event pair around an empty one-wave
 * kernel on the context's stream, over `reps` launches: the timing cost that
 * every event-bracketed launch above carries. */
fld_status fld_profile_overhead(fld_ctx* ctx, int32_t reps, double* us_per_launch);
/* Replay measurement of the same kernel family without per-launch events:
 * the line-sweep launches of one V-cycle (every grid level, in V-cycle order,
 * on the current operator; the LDS sub-cycle, restrictions and transposes
 * left out) are captured once as a hipGraph on a private solver state that
 * never reports convergence, then replayed `reps` times on the context's
 * stream between two HIP events.  Returns the mean time per launch (us, the
 * replay's elapsed time over reps x launches), the same for a graph of as
 * many empty one-wave launches (floor_us: what each dependent launch costs
 * by itself), the mean algorithmic bytes per launch and the number of
 * launches per V-cycle.  Needs fld_assemble and a line smoother (EINVAL
 * otherwise, ENOTREADY before assembly).  The multigrid work vectors are
 * overwritten (the next solve starts afresh). */
fld_status fld_profile_sweeps(fld_ctx* ctx, int32_t reps, double* us_per_launch, double* floor_us,
                              double* bytes_per_launch, int32_t* launches);
/* The same replay limited to the line-sweep launches of the finest `levels`
 * grid levels (levels = 1: the fine grid's half-sweeps alone; 0: every
 * level, as fld_profile_sweeps). */
fld_status fld_profile_sweeps_levels(fld_ctx* ctx, int32_t levels, int32_t reps, double* us_per_launch,
                                     double* floor_us, double* bytes_per_launch, int32_t* launches);
/* The same replay limited to grid levels first .. first + levels - 1
 * (levels = 0: to the last launched level; first = 1: the coarse levels'
 * band sweeps without the fine grid).  EINVAL if the range holds no
 * line-sweep launch. */
fld_status fld_profile_sweeps_range(fld_ctx* ctx, int32_t first, int32_t levels, int32_t reps,
                                    double* us_per_launch, double* floor_us, double* bytes_per_launch,
                                    int32_t* launches);

const char* fld_status_string(fld_status s);
const char* fld_last_error(const fld_ctx* ctx);
const char* fld_version(void);

/* Releases the context and all its device memory.  NULL is accepted. */
void fld_destroy(fld_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batched blocks (Section 3.2.2, static mesh refinement: every block is an
 * independent grid whose boundaries are ghost cells filled from its parent
 * or neighbours).  A batch holds nblocks Cartesian blocks of nx[b] x ny[b]
 * cells (1 .. 512 per side) with uniform spacing dx[b], dy[b] (cm; faces at
 * i dx[b], j dy[b]).  Fields are packed block after block, each block
 * row-major [ny][nx] (device doubles, sum nx ny in total); ghost_E packs
 * 2 ny + 2 nx values per block in the side order of fld_bc, block after
 * block.  One step of the whole batch is one kernel launch: one workgroup per
 * block runs the block's assembly, multigrid hierarchy, reliable-update
 * MG-preconditioned CG solve (line smoothing) and gas update; blocks are
 * launched largest first.  Every block solves the system fld_step would solve
 * for the same grid, boundaries and options.
 * ------------------------------------------------------------------------ */
typedef struct fld_batch fld_batch;

/* Creates a batch.  nx, ny, dx, dy: host arrays of nblocks entries, read
 * during the call.  bc: host array of 4 sides applied to every block (NULL =
 * DIRICHLET_GHOST on all sides; AXIS is not allowed).  opt may be NULL; the
 * batch needs smoother = LINE; mg_coarse_max above 64 acts as 64; chunk and
 * mg_cycle are unused (V-cycles); use_graph selects graph capture in fld_batch_steps.  stream: hipStream_t.
 * Returns EINVAL (sizes, spacing, options), ENOMEM, EHIP. */
fld_status fld_batch_create(fld_batch** out, int32_t nblocks, const int32_t* nx, const int32_t* ny,
                            const double* dx, const double* dy, const fld_bc* bc,
                            const fld_options* opt, void* stream);

/* One implicit step of every block, E_r and T_g updated in place (packed
 * device arrays).  per_block (host, nblocks entries, caller's block order)
 * may be NULL: then the call is asynchronous and returns OK once launched;
 * otherwise it synchronises, fills the records (ms = device time of the
 * block's workgroup, from the GPU wall clock) and returns the first non-OK
 * block status.  A block that fails
 * keeps its last iterate in E_r and its T_g unchanged; the others are not
 * affected. */
fld_status fld_batch_step(fld_batch* b, double* E_r, double* T_g, const double* rho,
                          const double* kappa_R, const double* kappa_P, const double* c_v,
                          const double* ghost_E, double dt, fld_solve_info* per_block);

/* nsteps consecutive batch steps (fields other than E_r, T_g held fixed),
 * captured as one hipGraph of nsteps kernel nodes when use_graph is set;
 * synchronises once; allocates no device memory (each block's first failure
 * is kept on the device between steps).  per_block receives the records of
 * the last step; returns the first failure over all steps of the first
 * failing block in the caller's order (failed blocks continue with the next
 * step). */
fld_status fld_batch_steps(fld_batch* b, int32_t nsteps, double* E_r, double* T_g, const double* rho,
                           const double* kappa_R, const double* kappa_P, const double* c_v,
                           const double* ghost_E, double dt, fld_solve_info* per_block);

/* Workgroup size of the batch kernel (256, 512 or 1024; default 512).  Any
 * value gives results that agree to rounding; the tuner picks the fastest. */
fld_status fld_batch_set_threads(fld_batch* b, int32_t threads);
fld_status fld_batch_get_threads(const fld_batch* b, int32_t* threads);

/* Packed sizes: cells (sum nx ny) and ghost values (sum 2 nx + 2 ny). */
fld_status fld_batch_sizes(const fld_batch* b, int64_t* cells, int64_t* ghosts);

/* Reason of the last error of b; with b = NULL, of the last failed
 * fld_batch_create or fld_block_step_noalloc on the calling thread. */
const char* fld_batch_last_error(const fld_batch* b);

/* Releases the batch and its device memory.  NULL is accepted. */
void fld_batch_destroy(fld_batch* b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one block
 * stepped exactly as one block of fld_batch_step with the same sides,
 * spacing, boundaries and options (same kernel, same result bit for bit), but
 * with no handle and no allocation.  Every byte of device workspace (block
 * table, metrics, FP64 operator, hierarchy, CG vectors, the record) lives in
 * a static array of 4 MiB per device, which each GPU the library runs on
 * holds until the process ends; it is set up on the first call on a device
 * (the caller's current device).  Only kernels are queued on `stream`
 * (hipStream_t, NULL = default), so the call can be captured into a graph;
 * with info == NULL it is asynchronous, otherwise it synchronises the stream
 * and returns the block's status.  Workspace need (bytes, each piece rounded
 * up to 256): about 6 n x 8 + 8 n x s + 5 x (4/3) n x s + 88 (nx + ny) with
 * n = nx ny and s = 4 (FP32, MIXED) or 8 (FP64): e.g. square blocks up to
 * 158 x 158 in FP64, 197 x 197 in FP32 and MIXED.  A block that does not fit is
 * rejected with FLD_EINVAL (the reason, as every other argument error, is
 * given by fld_batch_last_error(NULL) on the calling thread).  All calls on
 * one GPU share its array and the array keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other threads) race, so they
 * must be serialised by the caller.  Fields as for a one-block batch. */
fld_status fld_block_step_noalloc(int32_t nx, int32_t ny, double dx, double dy, const fld_bc* bc,
                                  const fld_options* opt, double* E_r, double* T_g, const double* rho,
                                  const double* kappa_R, const double* kappa_P, const double* c_v,
                                  const double* ghost_E, double dt, void* stream, fld_solve_info* info);

/* ------------------------------------------------------------------------
 * Block forest (Section 3.2.2, multilevel implicit radiation transport in a
 * single matrix; Section 4, radiation communications): a 2D Cartesian domain
 * of nx0 x ny0 level-0 cells (spacing dx0, dy0; faces at i dx0, j dy0) covered
 * exactly by leaf blocks of any level L (spacing dx0 / 2^L, dy0 / 2^L).
 * Neighbouring leaf cells may differ by one level at most (2:1 balance).  One
 * step assembles and solves one linear system over every leaf cell of every
 * level: a face between two leaf cells carries one conductance, used by both
 * rows, so a coarse cell beside a finer block couples directly to the two
 * fine cells of that side, each through the fine face's own D, and the flux
 * through the coarse side equals the sum of the two fine faces' fluxes.  A
 * level-jump face is the uniform grid's face (sigma and E interpolated
 * linearly along the normal between the two centres, R from their
 * difference, D = c lambda(R) / sigma_f) with the fine face's area and the
 * normal distance dx_fine/2 + dx_coarse/2 of the centres (the coarse centre's
 * lateral offset is neglected).  Cells: the single grid's T elimination and
 * gas update.  Solver: Jacobi-preconditioned CG in FP64 over ELL neighbour
 * lists (up to eight neighbours per cell), true-residual restarts.
 * ------------------------------------------------------------------------ */
typedef struct fld_forest fld_forest;

/* A leaf block: nx x ny cells of level `level` (0 .. 16) whose lower-left cell
 * is (i0, j0) in that level's index space (0 <= i0, i0 + nx <= nx0 2^level). */
typedef struct { int32_t level, i0, j0, nx, ny; } fld_forest_block;

/* Creates a forest: checks that the blocks cover the domain exactly (no
 * overlap, no leaf inside a coarser leaf, areas adding up) and are 2:1
 * balanced, numbers the leaf cells block after block (each block row-major:
 * the layout of every field array), and builds the face and neighbour tables
 * on the device.  bc: the four domain sides (side order of fld_bc; NULL =
 * reflecting): REFLECT, DIRICHLET_FACE, FLUX_IN or FREE_STREAM.  opt: FP64
 * only (precision = FLD_FP64); limiter, norm, rel_tol and max_inner apply.
 * Host arrays are read during the call.  Returns EINVAL with the reason in
 * fld_forest_last_error(NULL), ENOMEM, EHIP. */
fld_status fld_forest_create(fld_forest** out, int32_t nblocks, const fld_forest_block* blocks, int32_t nx0,
                             int32_t ny0, double dx0, double dy0, const fld_bc* bc, const fld_options* opt,
                             void* stream);

/* Numbers of leaf cells, interior faces and domain-boundary faces. */
fld_status fld_forest_sizes(const fld_forest* f, int64_t* cells, int64_t* faces, int64_t* boundary_faces);

/* Cell centres (cm) and levels in cell order (host arrays of `cells`
 * entries, any may be NULL). */
fld_status fld_forest_cells(const fld_forest* f, double* xc, double* yc, int32_t* level);

/* One implicit radiation step on every leaf cell (E_r, T_g updated in place;
 * device arrays of `cells` doubles in cell order).  Synchronises the stream
 * while solving.  info may be NULL.  Returns ENOCONV (E_r then holds the last
 * iterate and T_g is unchanged), EBREAKDOWN, ENONFINITE. */
fld_status fld_forest_step(fld_forest* f, double* E_r, double* T_g, const double* rho, const double* kappa_R,
                           const double* kappa_P, const double* c_v, double dt, fld_solve_info* info);

/* Reason of the last error of f; with f = NULL, of the last failed
 * fld_forest_create on the calling thread. */
const char* fld_forest_last_error(const fld_forest* f);

void fld_forest_destroy(fld_forest* f);

/* ------------------------------------------------------------------------
 * Autotuning: the method leaves the preconditioner's schedule open, and its
 * cost depends on the grid and the fields (launch latency on small levels,
 * line versus point smoothing under anisotropy, band fusion, multigrid depth).
 * The tuner times candidate configurations on the caller's own fields and
 * keeps the fastest whose steps converge.
 * ------------------------------------------------------------------------ */
typedef struct {
    fld_options opt;        /* the candidate                                              */
    int32_t threads;        /* batch workgroup size (0 for single-grid candidates)        */
    int32_t status;         /* status of the last timed step                             */
    int32_t inner_iters;    /* CG iterations of the last timed step (batch: max over blocks) */
    float   ms;             /* mean wall time of one step (assembly, solve, gas update)   */
} fld_tune_entry;

/* Single grid: candidates are base with smoother in {LINE, LINE_SPLIT, POINT},
 * mg_cycle in {K, V, W2, KL_K, KL_W2} (line smoothers; POINT keeps base's),
 * mg_coarse_max in {64, 256, 1024, 4096} and chunk in {8, 16, 4} (132 candidates);
 * precision, limiter,
 * norm and tolerances are those of base (NULL = defaults).  Each candidate
 * gets its own context and runs reps + 1 steps (the first untimed) from the
 * given E, T (device arrays, not modified; the trials run on scratch copies).
 * *best receives the fastest candidate with every step OK; entries (host,
 * max_entries, may be NULL) the whole table, *n_entries its length.  Returns
 * ENOCONV if no candidate converged, EINVAL / ENOMEM / EHIP. */
fld_status fld_tune(const fld_grid* grid, const fld_options* base, const double* E_r, const double* T_g,
                    const double* rho, const double* kappa_R, const double* kappa_P, const double* c_v,
                    const double* ghost_E, double dt, int32_t reps, fld_options* best,
                    fld_tune_entry* entries, int32_t max_entries, int32_t* n_entries, void* stream);

/* Batch: candidates are mg_coarse_max in {64, 32, 16} (multigrid depth) times
 * workgroup size in {512, 256, 1024}, timed as whole batch steps
 * (fld_batch_step) on scratch copies of the packed E, T.  Arguments as
 * fld_batch_create and fld_batch_step; *best and *best_threads receive the
 * fastest converging configuration. */
fld_status fld_batch_tune(int32_t nblocks, const int32_t* nx, const int32_t* ny, const double* dx,
                          const double* dy, const fld_bc* bc, const fld_options* base, const double* E_r,
                          const double* T_g, const double* rho, const double* kappa_R,
                          const double* kappa_P, const double* c_v, const double* ghost_E, double dt,
                          int32_t reps, fld_options* best, int32_t* best_threads, fld_tune_entry* entries,
                          int32_t max_entries, int32_t* n_entries, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FLD_H */
