/*
 * libdvm -- discrete-velocity BGK primal / adjoint solver and wall shape
 * sensitivity for AMD Instinct MI355X (gfx950).
 *
 * Method: Yuan & Wu, "Adjoint shape optimization from the continuum to
 * free-molecular gas flows" (arXiv 2501.00923).  The calls follow the
 * paper's statement of the problem:
 *   mesh and velocity grid ........ Sec. 3.1 (cells i, faces A_ij n_ij, volumes V_i;
 *                                   discrete velocities v_k with weights dXi_k)
 *   flow state and objective ...... Sec. 2.3 (far field f_d, diffuse wall at T_w),
 *                                   Sec. 2.4 eq. (formula_opt) (m_J = v1 drag, v^2/2 heat)
 *   primal solve .................. Sec. 3.1 eq. (numerpr_gov) with the BCs of Sec. 2.3
 *   adjoint solve ................. Sec. 2.5 eq. (formula_adjointbgk), Sec. 3.1 eq. (numerad_gov)
 *   objective ..................... Sec. 3.2 eq. (numer_J)
 *   wall sensitivity .............. Sec. 3.2 eqs. (sens_J_itf), (gaussgrad), (sens_B_itf), (sens_nod)
 *   volume constraint ............. Sec. 2.4 eq. (formula_opt), Sec. 3.2 eq. (sens_con_nod)
 *   CST design, initial fit ....... Sec. 3.3 eqs. (cstsuf), (cst_classfunc), (cst_shapefunc), (cstini)
 *   bulk-mesh deformation ......... Sec. 3.4 Step 2 (RBF, Wendland C0)
 *
 * Discretisation (the paper omits its scheme): first-order upwind finite
 * volume, Jacobi point-implicit iteration; the adjoint is the exact
 * transpose of the discrete primal map.  Units: rho_inf = 1, theta = RT with
 * theta_inf = 1/2, gamma = 5/3, u_inf = Ma sqrt(5/6) along +x,
 * tau_inf = (5 sqrt(pi) / 8) Kn (Kn = +inf gives collisionless flow).
 *
 * Conventions
 *   - Host arrays are FP64 or int32, row-major, 0-based; the caller owns
 *     every array and every device buffer it passes in.  The library owns
 *     only its opaque handles; destroy(NULL) is a no-op.
 *   - No exception or exit() crosses this boundary.  Every int-returning
 *     call returns a DVM_* status; on failure dvm_last_error() returns a
 *     thread-local message.
 *   - Device work is enqueued on the HIP stream given to dvm_solver_bind
 *     (or to a batch call).  Calls that return host values synchronise that
 *     stream.
 *   - Call order is enforced: solve calls before bind, adjoint before a
 *     primal state exists, sensitivity before an adjoint state exists
 *     return DVM_ESTATE.
 *   - Limits: 2 <= n1, n2 <= 128 velocity nodes per direction.
 */
#ifndef DVM_H
#define DVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dvm_mesh dvm_mesh;
typedef struct dvm_vgrid dvm_vgrid;
typedef struct dvm_solver dvm_solver;

enum {
    DVM_OK = 0,
    DVM_EINVAL = -1,    /* bad argument (sizes, pointers, geometry) */
    DVM_ENOMEM = -2,    /* host allocation failed or device buffer too small */
    DVM_EHIP = -3,      /* a HIP runtime call failed */
    DVM_ENOTCONV = -4,  /* iteration cap reached above tolerance; state stays valid */
    DVM_ENAN = -5,      /* NaN / Inf / non-positive density or temperature detected */
    DVM_ESTATE = -6     /* call out of order */
};
enum { DVM_TOPO_O = 0, DVM_TOPO_C = 1 };
enum { DVM_FP64 = 0, DVM_MIXED = 1 };   /* MIXED: f, phi and per-pair arithmetic in FP32;
                                           moments, Maxwellian parameters, residuals,
                                           wall fluxes, J and sensitivities in FP64 */
enum { DVM_OBJ_DRAG = 0, DVM_OBJ_HEAT = 1 };
enum { DVM_VG_MIDPOINT = 0, DVM_VG_NEWTON_COTES = 1, DVM_VG_SINH = 2 };
enum { DVM_STATE_F = 0, DVM_STATE_PHI = 1, DVM_STATE_PHI_ROWS = 2 };
enum { DVM_LIMITER_NONE = 0, DVM_LIMITER_VENKAT = 1 };   /* second-order slope limiter */
enum { DVM_EQ_POINTWISE = 0, DVM_EQ_CONSERVATIVE = 1 };   /* equilibrium on the velocity grid */
#define DVM_MAX_PARAMS 64

typedef struct {
    double Kn;       /* Knudsen number on l_ref = 1 (eq. kndefine); +inf allowed */
    double Ma;       /* free-stream Mach number, flow along +x */
    double Tw;       /* wall temperature / free-stream temperature */
    int objective;   /* DVM_OBJ_DRAG (m_J = v1) or DVM_OBJ_HEAT (m_J = |v|^2/2) */
} dvm_flow;

/* ---- mesh (Sec. 3.1) ------------------------------------------------
 * Structured body-fitted grid given by its nodes: nodes_xy[(j*(ni+1)+i)*2+{0,1}]
 * for i in [0, ni], j in [0, nj]; j = 0 is the wall (and the wake cut of a
 * C-grid), j = nj the far field.  The wall is walked clockwise as i grows so
 * that every cell (i,j),(i+1,j),(i+1,j+1),(i,j+1) is counter-clockwise; a
 * cell with non-positive area gives DVM_EINVAL.  O-grid: periodic in i,
 * column ni repeats column 0, n_wake = 0.  C-grid: cells i < n_wake and
 * i >= ni - n_wake of row 0 face each other across the wake cut (cell i
 * pairs with ni - 1 - i); faces i = 0 and i = ni are far field.
 * Cell c = i + ni*j; faces per cell in the order (j-, i+, j+, i-).  The mesh
 * copies nodes_xy. */
int dvm_mesh_create(int topology, int ni, int nj, int n_wake, const double *nodes_xy,
                    dvm_mesh **out);
int dvm_mesh_info(const dvm_mesh *m, int32_t *n_cells, int32_t *n_wall);
/* Exports (any pointer may be NULL): nbr[nc][4] (>= 0 neighbour cell, -1 far
 * field, -2-l wall element l), wall_cell[nw], face vectors S[nc][4][2] =
 * A_ij n_ij (outward of the cell), vol[nc], wall_A[nw], wall_n[nw][2] (unit
 * normal into the solid, Sec. 3.2), wall_x[nw][2] (element midpoint).
 * Wall element l joins wall nodes l (x_{l,1}) and (l+1) mod nw (x_{l,2}). */
int dvm_mesh_export(const dvm_mesh *m, int32_t *nbr, int32_t *wall_cell, double *S, double *vol,
                    double *wall_A, double *wall_n, double *wall_x);
void dvm_mesh_destroy(dvm_mesh *m);

/* ---- velocity grid (Sec. 2.2, d Xi = dv1 dv2) ------------------------
 * Tensor product of two 1-D rules on [-vmax, vmax]; velocity k = a + n1*b has
 * v = (x_a, y_b), weight w_a w_b.  MIDPOINT: n cells; NEWTON_COTES: n nodes,
 * n % 4 == 0, composite Simpson either side of one centred 3/8 panel;
 * SINH: x = vmax sinh(p s)/sinh(p) at the n cell midpoints s of (-1, 1),
 * weight = mapped cell width (param p > 0, default 2). */
int dvm_vgrid_create(int kind, int n1, int n2, double vmax, double param, dvm_vgrid **out);
int dvm_vgrid_info(const dvm_vgrid *g, int32_t *nv);
int dvm_vgrid_export(const dvm_vgrid *g, double *v /*[nv][2]*/, double *w /*[nv]*/);
void dvm_vgrid_destroy(dvm_vgrid *g);

/* ---- solver ----------------------------------------------------------
 * The solver copies what it needs from mesh and vgrid (both may be
 * destroyed afterwards).  precision: DVM_FP64 or DVM_MIXED.  want_adjoint
 * = 0 leaves the adjoint buffers out of the workspace. */
int dvm_solver_create(const dvm_mesh *m, const dvm_vgrid *g, const dvm_flow *flow, int precision,
                      int want_adjoint, dvm_solver **out);
/* Spatial scheme of the solve, set before dvm_solver_bind (the workspace
 * grows with order 2; DVM_ESTATE once bound).  Sec. 3.1 states second-order
 * accuracy in physical space for eqs. (numerpr_gov) and (numerad_gov) and
 * defers the scheme; order 1 (the default) takes face values from the
 * upwind cell.  order 2: cell values at the area centroids, Green-Gauss
 * slopes (face mean of the two cell values; the cell value on boundary
 * faces), limiter DVM_LIMITER_VENKAT (Venkatakrishnan, per cell, velocity
 * and component, smoothing e = 1e-3 |f_c|) or DVM_LIMITER_NONE, face values
 * reconstructed on the upwind side; far-field and wall inflow are not
 * reconstructed and the wall flux F_l sums the reconstructed outgoing
 * values; the drag uses the same wall values.  It is iterated by defect
 * correction: every correction_interval (K >= 1) sweeps the difference
 * between the second- and first-order face fluxes is evaluated from the
 * current state and held, and the sweeps between are the first-order Jacobi
 * sweep with that difference moved to the right-hand side; a fixed point
 * solves the second-order balance.  K must be large enough for the
 * first-order sweeps to approximate the first-order inverse, more so the
 * larger the grid and the Knudsen number: K = 1 is unstable where transport
 * dominates; on a 256x128 C-grid K = 5 diverged at Kn 0.1 (Ma 0.8), K = 10
 * at Kn 1 and K = 20 at Kn 10, where K = 40 converges (small grids converge
 * with K = 3).  Default K = 40.  The adjoint
 * freezes the limiter factors of the converged f (at dvm_adjoint_init) and
 * solves the transpose of that linearisation the same way.  Loading a state
 * re-evaluates the correction at the next sweep.  The wall sensitivity
 * (and its chain to shape parameters) evaluates the paper's formulas with
 * the second-order values: reconstructed wall and face values, F_l + dF_l.
 * The exact mesh sensitivity differentiates the second-order balance with
 * the limiter factors of f held fixed (exact with DVM_LIMITER_NONE). */
int dvm_solver_set_scheme(dvm_solver *s, int order, int limiter, int correction_interval);
/* Equilibrium of the BGK relaxation on the discrete velocity grid (Sec.
 * 2.1, eqs. maxwell_reduce, kndefine), set before dvm_solver_bind
 * (DVM_ESTATE once bound).  DVM_EQ_POINTWISE (the default): the reduced
 * Maxwellian of the cell's primitive variables at each grid velocity; its
 * grid moments differ from W by the grid's quadrature error, so the
 * discrete collision term does not conserve exactly.  DVM_EQ_CONSERVATIVE:
 * the reduced Maxwellian whose grid moments equal W exactly (its
 * parameters rho', u', theta' found by Newton's method from the primitive
 * variables, a fixed six steps, per cell and sweep); tau keeps the cell's
 * own rho and theta; the adjoint differentiates through the parameters
 * (dP'/dW = (dm/dP')^{-1}).  On grids whose quadrature of the Maxwellian
 * is off (Newton-Cotes, sinh-stretched) the pointwise iteration can diverge
 * in the near-continuum regime, where collisions amplify the moment error
 * every sweep; the conservative one does not. */
int dvm_solver_set_equilibrium(dvm_solver *s, int kind);
/* Macroscopic prediction of the primal and adjoint iterations (Sec. 3.1:
 * approximate macroscopic equations from the continuum limit provide
 * prediction solutions that accelerate the kinetic iteration), first-order
 * scheme and conservative equilibrium (the macroscopic equations are
 * conservation laws; DVM_EINVAL with order 2 or the pointwise Maxwellian),
 * set before dvm_solver_bind (the workspace grows by 108 doubles per cell;
 * DVM_ESTATE once bound).  every > 0: after every
 * `every`-th primal sweep (counted from dvm_primal_init, a loaded or
 * copied f), the moments r of the kinetic residual of eq. (numerpr_gov)
 * drive the linearised macroscopic system (A + Lambda) dW = -r, A being
 * the moments of the scheme's upwind transport of equilibrium perturbations
 * (each face's upwind cell's dg/dW; the diffuse wall's response through
 * F_l) and Lambda the pseudo-time term (|u| + c) sum_q |S_q| / 1000 per
 * cell, solved by `inner` red-black block Gauss-Seidel steps from dW = 0;
 * W + dW, limited so that rho and theta change by at most 20% per cell, is
 * the state the next sweep relaxes towards.  Every `every`-th adjoint sweep
 * (counted from dvm_adjoint_init or a loaded phi) is corrected by the
 * transpose of that step, -Psi L^T (H^T dphi) with L the Gauss-Seidel map,
 * H the sweep's response to the predicted moments and dphi the sweep's
 * change, so the accelerated adjoint iteration converges like the
 * accelerated primal one.  Both corrections vanish at the discrete
 * solutions, so the converged states are the plain iterations'; the
 * residual reported is the plain sweep's change.  In batches the
 * prediction runs on each member's own cadence, with the same kernels.
 * every = 0: off. */
int dvm_solver_set_acceleration(dvm_solver *s, int every, int inner);
/* Exact device bytes the solver needs (used for admission by footprint). */
size_t dvm_solver_workspace_bytes(const dvm_solver *s);
/* Bind a caller-owned device buffer (>= workspace bytes, 256-byte aligned)
 * and a HIP stream (NULL = default stream) on the current device; uploads
 * the geometry and velocity tables.  May be called again to move the solver
 * to another buffer (state is not carried over; call *_init again). */
int dvm_solver_bind(dvm_solver *s, void *dev_ptr, size_t bytes, void *hip_stream);
int dvm_solver_set_stream(dvm_solver *s, void *hip_stream);

/* f = far-field Maxwellian in every cell (Sec. 2.3); moments and wall
 * fluxes of it. */
int dvm_primal_init(dvm_solver *s);
/* Up to max_iter Jacobi sweeps of eq. (numerpr_gov).  Every check_every
 * sweeps (and after the last) the relative change of the moments
 * r = ||W^{n+1} - W^n||_2 / ||W^n||_2 is read back; stops when r < tol
 * (tol <= 0: run exactly max_iter sweeps).  *iters / *resid (may be NULL)
 * receive the sweeps done and the last r.  DVM_ENOTCONV if tol > 0 was not
 * reached, DVM_ENAN on NaN/Inf. */
int dvm_primal_iterate(dvm_solver *s, int max_iter, double tol, int check_every, int *iters,
                       double *resid);
/* Enqueue exactly n sweeps with no read-back (for timing and graphs). */
int dvm_primal_sweeps(dvm_solver *s, int n);
/* J of eq. (numer_J) for the current f, FP64; C_d = J / (u_inf^2 L / 2) with
 * L = 2 (O-grid: circle diameter) or 1 (C-grid: chord).  Synchronises. */
int dvm_objective(dvm_solver *s, double *J, double *Cd);
/* Conservative moments W[nc][4] of the current f (FP64), cells in mesh
 * order (c = i + ni*j).  Synchronises. */
int dvm_read_moments(dvm_solver *s, double *W);

/* Freeze the current f as the primal solution and set phi = 0. */
int dvm_adjoint_init(dvm_solver *s);
/* Jacobi sweeps of eq. (numerad_gov); r = ||phi^{n+1} - phi^n||_w / ||phi^{n+1}||_w
 * with weights w_k.  Same stopping contract as dvm_primal_iterate. */
int dvm_adjoint_iterate(dvm_solver *s, int max_iter, double tol, int check_every, int *iters,
                        double *resid);
int dvm_adjoint_sweeps(dvm_solver *s, int n);

/* Per wall element l: S_A[l] = dL/dA_l, S_x[l][2] = dL/dx_l, S_n[l][2] = dL/dn_l
 * (eqs. sens_J_itf + sens_B_itf, Green-Gauss gradient of eq. gaussgrad with
 * the scheme's upwind face values, dB/dn carrying A_l), and dJ_dnodes[nw][2]
 * through eq. (sens_nod) (wall node m = x_{m,1} of element m and x_{m,2} of
 * element m-1).  Any output may be NULL.  Synchronises. */
int dvm_wall_sensitivity(dvm_solver *s, double *S_A, double *S_x, double *S_n, double *dJ_dnodes);
/* dJ/dalpha_p = sum_m dJ/dx_m . dx_m/dalpha_p for a wall-node Jacobian
 * wall_jac[nw][2][n_params] (host, FP64), n_params <= DVM_MAX_PARAMS.  Runs
 * the sensitivity kernels first.  Synchronises. */
int dvm_param_sensitivity(dvm_solver *s, int n_params, const double *wall_jac, double *dJ_dalpha);
/* Exact discrete shape derivative: dJ_dx[(nj+1)(ni+1)][2] (mesh node order,
 * node (i, j) at index j*(ni+1)+i as in dvm_mesh_create) receives dL/dx for
 * every node coordinate, L = J + sum_{c,k} w_k phi_c,k . R_c,k the discrete
 * Lagrangian of Sec. 2.5 (R the residual of eq. numerpr_gov, J of eq.
 * numer_J) with the current f and phi held fixed: face vectors, volumes,
 * and the wall element normals and lengths (through F_l, D_l and J_l) all
 * move with the nodes.  With converged primal and adjoint states this is
 * the derivative of the discrete drag under mesh motion, including the
 * volume-mesh terms that the wall-only form (dvm_wall_sensitivity) leaves
 * out; chain it through the caller's d(nodes)/d(alpha).  The two copies of
 * a periodic O-grid column (i = 0 and i = ni) are separate entries.
 * Second-order scheme: the slopes, centroids and face midpoints move with
 * the nodes too; the limiter factors of f are held fixed, so the result is
 * the exact derivative with DVM_LIMITER_NONE and the frozen-limiter one
 * otherwise.  Requires the adjoint phase (DVM_ESTATE otherwise).
 * Synchronises. */
int dvm_mesh_sensitivity(dvm_solver *s, double *dJ_dx);

/* Checkpoint / restore as raw bytes, cells in mesh order (c = i + ni*j)
 * whatever the library's internal cell numbering.  DVM_STATE_F: f in the
 * storage precision ([nc][nv][2]); loading it recomputes its moments and
 * wall fluxes (bitwise as the sweep computes them) and starts a primal
 * phase.  DVM_STATE_PHI: phi followed by its FP64 adjoint moments ([nc][8])
 * and wall multipliers ([nw]); needs an adjoint phase.  Resuming from a
 * snapshot reproduces the iterates bitwise.  DVM_STATE_PHI_ROWS: phi alone
 * ([nc][nv][2], storage precision); loading it computes its adjoint moments
 * (eq. adjoint_macdefines, with the frozen f) and wall multipliers (eq.
 * formula_adjointbgk) on the device, with the arithmetic and summation order
 * of the adjoint sweep, so any phi (e.g. one from another solver) can start
 * an adjoint iteration; needs an adjoint phase.  Both synchronise. */
size_t dvm_state_bytes(const dvm_solver *s, int which);
int dvm_state_save(dvm_solver *s, int which, void *host_dst, size_t bytes);
int dvm_state_load(dvm_solver *s, int which, const void *host_src, size_t bytes);

/* Device-to-device copy of a state between two bound solvers of the same
 * grid size, topology, velocity count and precision (their geometry may
 * differ: a warm start for the solve of a nearby shape).  DVM_STATE_F:
 * src's f (its frozen primal solution in the adjoint phase) becomes dst's
 * f, with its moments and wall fluxes recomputed; dst starts a primal phase.
 * DVM_STATE_PHI: both in the adjoint phase; src's phi, adjoint moments and
 * wall multipliers replace dst's.  Synchronises both streams. */
int dvm_state_copy(dvm_solver *dst, const dvm_solver *src, int which);

/* ---- batched serving --------------------------------------------------
 * A batch groups n bound solvers of one precision.  Each member takes part
 * in the phase it is in when the batch is created: primal (after
 * dvm_primal_init) or adjoint (after dvm_adjoint_init).  dvm_batch_run
 * advances every member by `iters` Jacobi sweeps with up to four kernel
 * launches per sweep (over the cells of the primal-phase members of the
 * first- and of the second-order scheme, then those of the adjoint-phase
 * members), on the batch's stream; a second-order member's held correction
 * is re-evaluated before the sweep on its own cadence, with the kernels of
 * a single solve.  Each launch gives
 * every one of the 8 XCDs one eighth of every member, so a mix of mesh and
 * velocity-grid sizes keeps all XCDs equally loaded.  A member's sweep
 * computes exactly what its own dvm_*_sweeps computes alone (same kernels,
 * same reduction order, no floating-point atomics).  work_dev is a
 * caller-owned device buffer of at least dvm_batch_work_bytes(n, total
 * cells of the n members) bytes, 256-byte aligned, holding the launch
 * tables, written once at create (which
 * synchronises the stream).  While a batch exists its members must not be
 * re-initialised, re-bound, destroyed or swept outside the batch; destroy
 * the batch first.  Admission (which solves share a batch) is the caller's
 * policy; dvm_solver_workspace_bytes gives each solve's exact footprint. */
typedef struct dvm_batch dvm_batch;
size_t dvm_batch_work_bytes(int n, int64_t total_cells);
int dvm_batch_create(dvm_solver *const *solvers, int n, void *work_dev, size_t work_bytes,
                     void *hip_stream, dvm_batch **out);
/* Allocation-free variant of dvm_batch_create, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same batch, whose launch tables
 * live in a fixed device array the library holds on each GPU it runs on
 * (8 MiB, until the process ends) instead of a caller-owned work buffer;
 * they are built there by a kernel on hip_stream, with no device or host
 * allocation.  At most 64 members, and tables of at most 8 MiB (about 2 M
 * patches, i.e. some 8 M cells over all members); larger batches give
 * DVM_EINVAL.  One such batch may exist per device at a time: a second
 * create on the same device gives DVM_ESTATE until dvm_batch_destroy of the
 * first.  All calls on one device share the array, so concurrent use from
 * several host threads on one device races.  run, residual and destroy as
 * for dvm_batch_create; results are bitwise those of dvm_batch_create. */
int dvm_batch_create_static(dvm_solver *const *solvers, int n, void *hip_stream, dvm_batch **out);
int dvm_batch_run(dvm_batch *b, int iters);
/* Residual (as in *_iterate) of each member's last sweep into resid[n].
 * Synchronises the batch's stream. */
int dvm_batch_residual(dvm_batch *b, double *resid);
void dvm_batch_destroy(dvm_batch *b);
/* Sweeps done so far in the solver's current phase (0 primal, 1 adjoint). */
int dvm_solver_iterations(const dvm_solver *s, int phase);
/* Current phase: -1 no state, 0 primal, 1 adjoint. */
int dvm_solver_phase(const dvm_solver *s);

/* ---- outer loop of the optimisation (Sec. 3.3, Sec. 3.4) -------------
 * CST parameterisation, the volume constraint and the bulk-mesh deformation
 * that turn a design vector into a mesh for the next solve, and chain the
 * solve's node sensitivities back to the design vector. */
#define DVM_CST_MAX_NB 20
/* CST surface (Sec. 3.3, eqs. cstsuf, cst_classfunc, cst_shapefunc).
 * alpha[2 nb + 6] = {N1, N2, A_u[0..nb], A_l[0..nb], eta_T,u, eta_T,l},
 * 1 <= nb <= DVM_CST_MAX_NB, N1 > 0, N2 > 0.  For n stations xi[m] in [0, 1]
 * (chord-normalised abscissa) on the upper (upper[m] != 0) or lower surface:
 *   eta[m] = xi^N1 (1 - xi)^N2 sum_b A_b binom(nb, b) xi^b (1 - xi)^(nb - b)
 *            + xi eta_T
 * with the A's and eta_T of that surface.  jac (may be NULL) receives
 * d eta_m / d alpha as jac[m][2 nb + 6].  Host computation. */
int dvm_cst_eval(int nb, const double *alpha, int n, const double *xi, const int32_t *upper,
                 double *eta, double *jac);
/* Initial design (Sec. 3.3, eq. cstini): least-squares fit of the CST
 * surface to eta[n] at the stations xi[n], over the design variables p with
 * fixed[p] == 0 (fixed == NULL: all but the two trailing-edge offsets);
 * fixed variables keep their values from alpha.  Damped Gauss-Newton from
 * N1 = 0.5, N2 = 1 (where free) with the free A's and eta_T's first fitted
 * linearly at that class.  alpha[2 nb + 6] is in/out; *rms (may be NULL)
 * receives sqrt(sum of squared residuals / n).  DVM_EINVAL if the free
 * variables are not determined by the stations (e.g. n too small). */
int dvm_cst_fit(int nb, int n, const double *xi, const int32_t *upper, const double *eta,
                const int32_t *fixed, double *alpha, double *rms);
/* Volume constraint (Sec. 2.4, eq. formula_opt, D = 2) of the closed wall
 * loop wall_xy[nw][2] (wall node l starts wall element l, as in a mesh's
 * row j = 0): Q = (1/2) sum_l A_l n_l . x_l + v_min, n_l the unit normal
 * into the solid, x_l the element midpoint, so Q = v_min - (area of the
 * body) for the clockwise walls of dvm_mesh_create.  dQ_dx (may be NULL)
 * receives dQ/dx[nw][2] by eq. (sens_con_nod): half the sum of A n over the
 * two elements that share the node. */
int dvm_volume_constraint(int nw, const double *wall_xy, double v_min, double *Q, double *dQ_dx);

/* Bulk-mesh motion by radial-basis-function interpolation with the
 * Wendland C0 function (Sec. 3.4, Step 2): phi(r) = (1 - r/R)^2 for r < R,
 * else 0, R = radius.  Centres c_w are the nw wall nodes of the reference
 * mesh m (row j = 0; the two copies of the trailing-edge node of a C-grid
 * and of the periodic column of an O-grid are one centre).  For new wall
 * positions the weights solve M gamma = (new - c), M[w][v] = phi(|c_w - c_v|);
 * every other node moves to x0_n + sum_w gamma_w phi(|x0_n - c_w|) from its
 * reference position x0_n, and wall nodes take the new positions exactly.
 * The nodes are therefore linear in the wall displacement.  create factors
 * M (Cholesky, O(nw^3) host work on up to 16 threads, a few seconds at the
 * limit nw <= 8192, nw > 8192 is DVM_EINVAL; DVM_EINVAL if M is not
 * positive definite, e.g. two coincident wall nodes) and copies the
 * reference nodes. */
typedef struct dvm_deform dvm_deform;
int dvm_deform_create(const dvm_mesh *m, double radius, dvm_deform **out);
/* Device bytes the deformer needs; bind a caller-owned buffer (256-byte
 * aligned, >= that size) and a HIP stream (NULL: default stream) on the
 * current device, uploading the reference nodes. */
size_t dvm_deform_workspace_bytes(const dvm_deform *d);
int dvm_deform_bind(dvm_deform *d, void *dev_ptr, size_t bytes, void *hip_stream);
/* wall_xy[nw][2] (host) new wall node positions -> nodes_xy (host), every
 * node of the mesh in dvm_mesh_create's layout.  Synchronises. */
int dvm_deform_apply(dvm_deform *d, const double *wall_xy, double *nodes_xy);
/* Transpose: from dJ_dx (host, every node coordinate in dvm_mesh_create's
 * layout, e.g. dvm_mesh_sensitivity's output) to dJ_dwall[nw][2] (host),
 * the derivative with respect to the wall node positions through
 * dvm_deform_apply (the wall nodes' own entries plus the interpolated
 * motion of all others).  Synchronises. */
int dvm_deform_chain(dvm_deform *d, const double *dJ_dx, double *dJ_dwall);
void dvm_deform_destroy(dvm_deform *d);

const char *dvm_last_error(void);
void dvm_solver_destroy(dvm_solver *s);

#ifdef __cplusplus
}
#endif
#endif /* DVM_H */
