/*
 * gdg.h -- C-ABI of libgdg, the MI355X (gfx950) implementation of the
 * per-stage algebraic sweep of the graph-based discontinuous Galerkin scheme
 * for the compressible Euler equations of Kronbichler, Maier & Tomas,
 * "Graph-based methods for hyperbolic systems of conservation laws using
 * discontinuous space discretizations" (arXiv 2402.04514).
 *
 * The problem these calls solve (Sec. 3.1, eq. cijdijscheme): given nodal
 * states U_i^n in the admissible set A (rho > 0, eps > 0, eq. AddSet) of a
 * DG Q_k space on a mesh, and boundary data built from them (Sec. 4), produce
 * U^{n+1} with a time step from the CFL rule (eq. MaxCFLdt), using the
 * low-order update, the entropy-viscosity high-order update and convex
 * limiting (Sec. 5) inside SSP-RK3 or SSPRK(5,4) (Sec. 6.2).
 *
 * Conventions
 *  - dofs: cell-major.  Cells lexicographic with x fastest; inside a cell the
 *    (k+1)^d Gauss-Lobatto nodes lexicographic with x fastest.  Face nodes of
 *    neighbouring cells are distinct dofs at the same point (Sec. 2.3).
 *  - states: SoA double arrays of (dim+2) planes of ndofs values,
 *    plane 0 = rho, planes 1..dim = momentum, plane dim+1 = total energy E.
 *  - box faces: f = 2*axis + side, side 0 = low end.
 *  - memory: the caller owns every host buffer and the device workspace;
 *    the library allocates no device memory.  All device work is enqueued on
 *    the HIP stream given at creation.
 *  - errors: every call returns a gdg_status; gdg_last_error() gives text.
 *    No exception crosses this interface.  Calls on one context are not
 *    thread-safe.
 */
#ifndef GDG_H
#define GDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gdg_ctx gdg_ctx;

typedef enum {
  GDG_OK = 0,
  GDG_E_INVALID = -1,      /* bad argument or mesh description */
  GDG_E_INADMISSIBLE = -2, /* a state left A: rho <= 0, eps <= 0 or NaN (eq. AddSet) */
  GDG_E_CFL = -3,          /* the CFL condition eq. CFLcond failed after all restarts */
  GDG_E_NOMEM = -4,        /* workspace smaller than gdg_workspace_bytes() */
  GDG_E_DEVICE = -5,       /* a HIP runtime call failed */
  GDG_E_BUDGET = -6,       /* a request can never fit the server's memory pool */
  GDG_E_BOUNDARY = -7      /* no boundary state: subsonic normal flow at a GDG_BC_SUPERSONIC face,
                              or no admissible characteristic state at a GDG_BC_INOUTFLOW face */
} gdg_status;

/* Boundary kinds per box face (Sec. 4.1), with n the outward unit normal
 * c_i^{d}/|c_i^{d}| of the boundary part:
 *  - OUTFLOW: the supersonic-outflow branch U^d := U_i of
 *    eq. supersonic_inoutflow ("do nothing");
 *  - SLIP: eq. slip_boundary, the normal momentum reflected;
 *  - DIRICHLET: U^d := the face's data (Sec. 4.1, Dirichlet boundary
 *    conditions): bc_state[f], or the isentropic vortex at the node and the
 *    stage time (gdg_mesh_desc.data_kind);
 *  - SUPERSONIC: eq. supersonic_inoutflow, U^d := the data where
 *    u_i.n < -a_i (inflow) and U^d := U_i where u_i.n >= a_i (outflow); a
 *    step that meets subsonic normal flow fails with GDG_E_BOUNDARY;
 *  - INOUTFLOW: sub- and supersonic in/outflow: eq. supersonic_inoutflow
 *    where |u_i.n| >= a_i, and in the subsonic range the state whose
 *    characteristic variables of eq. characteristics are those of the data for
 *    the incoming characteristics (speed <= 0 at U_i) and those of U_i for
 *    the others; if that state has no positive sound speed the step fails
 *    with GDG_E_BOUNDARY;
 *  - PERIODIC: must be set on both faces of an axis. */
typedef enum {
  GDG_BC_PERIODIC = 0,
  GDG_BC_OUTFLOW = 1,
  GDG_BC_SLIP = 2,
  GDG_BC_DIRICHLET = 3,
  GDG_BC_SUPERSONIC = 4,
  GDG_BC_INOUTFLOW = 5
} gdg_bc;

/* Source of the data U^d of the DIRICHLET, SUPERSONIC and INOUTFLOW faces. */
typedef enum {
  GDG_DATA_CONSTANT = 0, /* bc_state[f], constant in space and time */
  GDG_DATA_VORTEX = 1,   /* the isentropic vortex of Sec. 6.2 at the node and
                            the stage time (2D): vortex[] = beta, x0 (2),
                            u_inf (2), gamma of the data; free space (no
                            periodic images).  The SSP-RK3 stages take their
                            data at t, t + tau and t + tau / 2; those of
                            SSPRK(5,4) at t + c_k tau (gdg_integrator). */
  GDG_DATA_STEP_START = 2 /* U^d_i = U^n_i, the node's own state at the start
                            of the step, in every stage (strategy (d) of
                            Sec. 6.3, for flows without known boundary
                            data); bc_state is not read.  Lattice, general
                            and unstructured meshes; not continuous
                            elements, not served. */
} gdg_data_kind;

/* GDG_LOW_ORDER: eq. cijdijscheme only.  GDG_HIGH_ORDER: eq. HighScheme
 * unlimited.  GDG_LIMITED: eq. LimitedScheme with the bounds of
 * eq. local_bounds (the paper's method). */
typedef enum { GDG_LOW_ORDER = 0, GDG_HIGH_ORDER = 1, GDG_LIMITED = 2 } gdg_scheme;

/* GDG_FP64: every operation in double precision.
 * GDG_MIXED: the stencil coefficients c_ij are stored in single precision and
 * the flux sums sum_j (f(U_j) - f(U_i)) c_ij of the low- and high-order
 * updates and the sums of the entropy residual (Sec. 5.2) are accumulated in
 * single precision (each term rounded once from the double-precision flux
 * difference that the bar state needs); the state and its updates,
 * the wave-speed bound and d_ij (eq. dij_low_order), the bar states and local
 * bounds (eq. local_bounds) and the limiter line search (Sec. 5.4) stay in
 * double precision, so every stage output is still checked against A.  The
 * boundary parts use the double-precision flux that their bar state needs. */
typedef enum { GDG_FP64 = 0, GDG_MIXED = 1 } gdg_precision;

/* Time integration of gdg_step() and gdg_run_to().
 * GDG_SSPRK3: the three-stage, third-order SSP Runge-Kutta method in
 * Shu-Osher form (Sec. 6): stages at t, t + tau, t + tau / 2, each a
 * forward-Euler stage of size tau; tau = Cr min_i (-m_i / (2 d_ii)) of U^n
 * (eq. MaxCFLdt).
 * GDG_SSPRK54: the five-stage, fourth-order SSP method of Spiteri and Ruuth
 * that Sec. 6.2 uses for the isentropic vortex, in its Shu-Osher form with
 * non-negative coefficients.  Stage k is the forward-Euler stage of size
 * r_k tau (r_k = beta_{k+1,k} / alpha_{k+1,k}: 0.3918, 0.6631, 0.6631,
 * 0.6631, 0.5844) at time t + c_k tau (c = 0, 0.3918, 0.5861, 0.4745,
 * 0.9350), and the new state is the convex combination of the method.
 * tau = Cr tau_max(U^n) / max_k r_k, so that every stage is an Euler step
 * within Cr of the CFL bound of U^n (about 1.51 times the SSP-RK3 step, for
 * 5/3 of its stages).  Either method restarts a step whose stage k finds
 * r_k tau above its own bound tau_max(u_k), with tau = Cr tau_max(u_k) / r_k. */
typedef enum { GDG_SSPRK3 = 0, GDG_SSPRK54 = 1 } gdg_integrator;

/* Cartesian mesh of cells[0] x cells[1] x cells[2] cells over the box
 * [lo, hi] (only the first dim entries are read), Q_degree elements with
 * degree 1 or 2 in dim 1..3 and degree 3 in dim 1 and 2, bc[2*dim] boundary
 * kinds.  With data_kind GDG_DATA_CONSTANT, bc_state[f] holds the conserved
 * data (rho, momentum, E: the first dim+2 entries) of face f for the
 * DIRICHLET, SUPERSONIC and INOUTFLOW kinds; it must be admissible (rho > 0,
 * eps > 0) on those faces and is ignored elsewhere.  With GDG_DATA_VORTEX
 * the data of those faces come from the vortex (vortex[]).
 *
 * General cells (Sec. 2.3): with vertices non-NULL the cells keep the
 * lattice's connectivity but each one is the multilinear image of the unit
 * square or cube through its own 2^dim corners.  vertices holds
 * (cells[0]+1) x .. x (cells[dim-1]+1) points of dim coordinates each
 * (interleaved per point, the first axis fastest: point (p0, p1, p2) at
 * index p0 + (cells[0]+1) (p1 + (cells[1]+1) p2)); cell (k0, k1, k2) takes the
 * points (k0 + b0, k1 + b1, k2 + b2), b in {0, 1}^dim.  lo and hi are not
 * read.  m_ij, c_ij and the boundary parts c_i^d are integrated through the
 * map, so every Jacobian determinant must be positive (else GDG_E_INVALID).
 * A periodic axis identifies the lattice's first and last layers of cells
 * across it; the caller keeps the two boundary layers of points congruent.
 * The pointer is read during gdg_create() only (the context keeps a copy for
 * gdg_node_coords()).  Not combined with GDG_DATA_VORTEX.
 *
 * Curved cells: with map_degree 2 each cell is the image of the reference
 * cell under the tensor-product quadratic map through its 3^dim points
 * (corners, edge and face midpoints, centre), and vertices holds the lattice
 * of (2 cells[0]+1) x .. points, same order; cell (k0, k1, k2) takes the
 * points (2 k0 + q0, 2 k1 + q1, 2 k2 + q2), q in {0, 1, 2}^dim.  The integrals
 * stay exact (Gauss rules of degree + 2 points per direction, degree + 3 for
 * the 3D masses).
 *
 * Boundary parts (Sec. 4.1 applies its conditions part by part): with
 * bc_cells non-NULL each cell face on the boundary has its own kind.  For each
 * box face f = 0 .. 2 dim - 1 whose bc[f] is not PERIODIC, in order of f, one
 * entry per cell face on it, those cells taken lexicographically over the
 * other axes with the lowest axis fastest; each entry is a gdg_bc other than
 * PERIODIC.  The DIRICHLET, SUPERSONIC and INOUTFLOW parts of face f take
 * face f's data (bc_state[f], or the vortex), which must then be admissible.
 * bc[f] still decides which axes are periodic.  Read during gdg_create()
 * only.
 *
 * Unstructured meshes (dim 2 or 3): with ucells > 0 the mesh is ucells cells
 * of any connectivity.  Cell q is the image of the reference cell under its
 * map of degree map_degree (multilinear or quadratic) through the points
 * vertices[ucell_points[q (g+1)^dim + v]] (npoints points of dim coordinates;
 * v: the digits q_e of v in base g + 1, the first axis lowest).  Two cells
 * are neighbours across faces with the same corner points (in any relative
 * orientation; with map_degree 2 all the face's points must agree); a face
 * may be shared by two cells at most.  A face of no other cell is a boundary
 * part: uface_bc[q 2 dim + f] (local face f = 2 axis + side) is its kind (a
 * gdg_bc other than PERIODIC) + 8 * the box-face slot (< 2 dim) whose data
 * (bc_state) it takes; entries of interior faces must be 0.  cells, lo, hi,
 * bc and bc_cells are not read; cells connect through shared points only, so
 * an O-grid's seam is periodic by construction and a translated periodic
 * image is not expressible.  The arrays are read during gdg_create() only.
 *
 * Continuous elements (App. B): with continuous = 1 the dofs are the nodes of
 * the continuous Q_degree space on the box (degree * cells[e] + 1 per axis,
 * degree * cells[e] on a periodic axis, which needs at least 2 degree + 1 of
 * them; node (I_0, I_1, I_2) at index I_0 + n_0 (I_1 + n_1 I_2)), the graph
 * of a node is every node of the cells around it, and c_ij and the boundary
 * parts c_i^d (one per box face the node lies on) are those of
 * eq. cijcidefCg.  The scheme must be GDG_LOW_ORDER: the high-order update
 * of continuous elements needs a global mass solve, which the paper does not
 * give.  Not with vertices, bc_cells, unstructured meshes or vortex data. */
typedef struct {
  int32_t dim;
  int32_t degree;
  int64_t cells[3];
  double lo[3];
  double hi[3];
  int32_t bc[6];
  double bc_state[6][5];
  int32_t data_kind;  /* gdg_data_kind */
  int32_t map_degree; /* general cells: 0 or 1 multilinear, 2 quadratic (curved); see above */
  double vortex[6];
  const double *vertices; /* NULL: the uniform box [lo, hi]; else host memory, see above */
  const int8_t *bc_cells; /* NULL: kind bc[f] on all of box face f; else host memory, see above */
  /* unstructured meshes (see above); ucells = 0: the lattice of cells[] */
  int64_t ucells;
  int64_t npoints;
  const int64_t *ucell_points;
  const int8_t *uface_bc;
  int32_t continuous; /* 1: continuous Q_degree elements on the box (App. B), see above */
  int32_t reserved;   /* 0 */
} gdg_mesh_desc;

/* Scheme constants.  gdg_default_params() gives the paper's values:
 * gamma 1.4, Cr 0.5 (eq. MaxCFLdt), c_ev 1 / 0.5 / 0.25 for k = 1 / 2 / 3 (Sec. 5.2),
 * c_k 1 (eq. ViscMin), c_r 4 and p_r 1.5 (eq. ViscMinConst2), two limiter
 * passes (Sec. 6.1), the limited scheme, FP64, SSP-RK3. */
typedef struct {
  double gamma;
  double cfl;
  double c_ev;
  double c_k;
  double c_r;
  double p_r;
  int32_t limiter_passes; /* 0, 1 or 2 */
  int32_t scheme;         /* gdg_scheme */
  int32_t precision;      /* gdg_precision */
  int32_t flags;          /* 0, or GDG_FLAG_NO_QUIET_ROWS */
  int32_t integrator;     /* gdg_integrator */
  int32_t reserved;       /* 0 */
} gdg_params;

/* gdg_params.flags.  GDG_FLAG_NO_QUIET_ROWS: the first limiter pass visits
 * the pairs of every row, also of rows whose whole stencil holds one state bit
 * for bit (their antidiffusive fluxes are exactly zero, so by default the pass
 * accepts them without a visit).  The results are the same; the flag exists to
 * check that. */
enum { GDG_FLAG_NO_QUIET_ROWS = 1 };

/* Counters and measures of a run (Sec. 3 and 5: the properties the scheme
 * guarantees, so that a caller can check them without downloading the state).
 * The state measures are reduced on the device in a fixed order (the same
 * state gives the same bits); the counters are integer totals since the last
 * gdg_upload_state(), and include the stages of steps that a CFL violation
 * restarted. */
typedef struct {
  double t;          /* simulated time */
  int64_t steps;     /* time steps taken */
  int64_t restarts;  /* steps restarted after a CFL violation in stage 2 or 3 */
  double last_dt;    /* tau of the last step */
  double min_rho;    /* min_i rho_i of the current state (eq. AddSet: > 0) */
  double min_eps;    /* min_i eps_i = E_i - |m_i|^2 / (2 rho_i) (eq. AddSet: > 0) */
  double total[5];   /* sum_i m_i U_i per component (rho, momentum, E; dim + 2
                        entries): conserved on periodic meshes (Sec. 3.2,
                        Lemma TotBalLemma),
                        mass and energy also in slip boxes */
  int64_t bound_violations; /* limiter-pass outputs outside their relaxed bounds
                               of eq. local_bounds (beyond 1e-12 relative on rho,
                               1e-11 on the rescaled entropy); 0 by Lemma
                               ConsInvariants */
  int64_t limited_pairs;    /* pairs (i, j) that limiter pass 1 cut, l_ij < 1,
                               summed over stages */
  int64_t quiet_rows;       /* rows of cells whose whole stencil held one state
                               (every flux exactly zero), summed over stages */
} gdg_stats;

/* Intermediate fields of the last forward-Euler stage, for inspection. */
typedef enum {
  GDG_FIELD_STATE = 0,  /* current state U, (dim+2) planes */
  GDG_FIELD_EV_N = 1,   /* normalized entropy residual N_i (Sec. 5.2), 1 plane */
  GDG_FIELD_BOUNDS = 2, /* rho_min, rho_max, s~_min of eq. local_bounds, 3 planes */
  GDG_FIELD_UL = 3,     /* low-order update U^L, eq. cijdijscheme, (dim+2) planes */
  GDG_FIELD_DUH = 4,    /* high-order increment U^H - U, eq. HighScheme, (dim+2) planes */
  GDG_FIELD_U1 = 5      /* state after limiter pass 1, eq. LimitedScheme, (dim+2) planes */
} gdg_field;

/* Fills *out with the paper's constants for Q_degree. */
gdg_status gdg_default_params(int32_t degree, gdg_params *out);

/* Device workspace, in bytes, that gdg_create() needs for this mesh. */
gdg_status gdg_workspace_bytes(const gdg_mesh_desc *mesh, const gdg_params *prm, size_t *bytes);

/* Builds the stencil of Sec. 2.3 (m_i, m_ij, c_ij, c_i^{d,k} of
 * eq. mass_matrices, cij_def1, cij_def2 and Sec. 4.2) on the host and copies
 * it into dev_workspace (caller-owned device memory of ws_bytes bytes, 256-byte
 * aligned, alive until gdg_destroy).  hip_stream is a hipStream_t (NULL: the
 * null stream).  *out receives the context; GDG_E_NOMEM if ws_bytes is too
 * small, GDG_E_INVALID for a bad description. */
gdg_status gdg_create(const gdg_mesh_desc *mesh, const gdg_params *prm, void *dev_workspace,
                      size_t ws_bytes, void *hip_stream, gdg_ctx **out);

/* Releases the context (not the workspace).  Synchronizes the stream. */
void gdg_destroy(gdg_ctx *ctx);

/* Number of dofs N (per component). */
int64_t gdg_num_dofs(const gdg_ctx *ctx);

/* Collocation points x_i into host_xyz[N * dim] (interleaved per dof). */
gdg_status gdg_node_coords(const gdg_ctx *ctx, double *host_xyz);

/* Copies a state (SoA, (dim+2) * N doubles) into the context.  U may be host
 * or device memory: the copy uses unified addressing (hipMemcpyDefault), so
 * is_device_ptr only documents the caller's intent and is not needed for the
 * copy (the same holds for gdg_download_state and gdg_read_field).  Resets t
 * and the step counters.  Returns
 * GDG_E_INADMISSIBLE if some U_i is outside A (the paper's guarantees assume
 * admissible data, Sec. 3.1).  Synchronizes the stream. */
gdg_status gdg_upload_state(gdg_ctx *ctx, const double *U, int32_t is_device_ptr);

/* Copies the current state out (same layout).  Synchronizes the stream. */
gdg_status gdg_download_state(gdg_ctx *ctx, double *U, int32_t is_device_ptr);

/* One step of the params' integrator (gdg_integrator).  tau from the first
 * stage's bound (eq. MaxCFLdt; divided by max_k r_k for GDG_SSPRK54), or
 * dt_fixed if dt_fixed > 0; then capped by dt_cap if dt_cap > 0.  Every later
 * stage re-checks eq. CFLcond for its own Euler step on its own state; on
 * violation the step restarts with the tau of gdg_integrator's rule (at most
 * 8 times, then GDG_E_CFL).  *dt_taken (may be NULL) receives tau.
 * Returns GDG_E_INADMISSIBLE if a stage output left A, GDG_E_BOUNDARY if a
 * node of a GDG_BC_SUPERSONIC face saw subsonic normal flow; after either
 * error the context's state is not a valid step result: upload a state
 * before stepping again. */
gdg_status gdg_step(gdg_ctx *ctx, double dt_cap, double dt_fixed, double *dt_taken);

/* Steps until t = t_final (last step capped) or max_steps steps.  The time
 * loop runs on the device: captured HIP graphs of several steps, the host
 * synchronizing once per graph; a step whose stage 2 or 3 violates the CFL
 * condition is redone host-driven with the restart rule of gdg_step().  With
 * kernel timing on (gdg_profile) every step runs host-driven.  Errors as for
 * gdg_step(); stats (may be NULL) receives the counters. */
gdg_status gdg_run_to(gdg_ctx *ctx, double t_final, int64_t max_steps, gdg_stats *stats);

/* One forward-Euler stage U <- Phi(U; tau) of the selected scheme (tau <= 0:
 * the CFL rule), keeping its intermediates for gdg_read_field().  Returns
 * GDG_E_INADMISSIBLE or GDG_E_BOUNDARY as gdg_step() does. */
gdg_status gdg_stage(gdg_ctx *ctx, double tau, double *tau_used);

/* Copies a field of the last stage (gdg_field) to dst in dof order, one plane
 * of N doubles after the other. */
gdg_status gdg_read_field(gdg_ctx *ctx, int32_t field, double *dst, int32_t is_device_ptr);

/* Time, counters and the measures of the current state (gdg_stats).  Enqueues
 * the state reduction on the context's stream and synchronizes it. */
gdg_status gdg_get_stats(gdg_ctx *ctx, gdg_stats *stats);

/* Kernel timing.  gdg_profile(ctx, 1) starts bracketing every sweep launch
 * with HIP events on the context's stream (and clears the sums); 0 stops.
 * gdg_profile_read() returns, per kernel, the summed device time in ms and
 * the number of launches since the last gdg_profile() call, in the order
 * GDG_KERNEL_*. */
typedef enum {
  GDG_KERNEL_PRIM = 0,   /* per-node primitives */
  GDG_KERNEL_SWEEP1 = 1, /* d^L, CFL bound, entropy-viscosity ratio, ring-1 bounds */
  GDG_KERNEL_SWEEP2 = 2, /* U^L, bounds, d^H, high-order residual, cell solve */
  GDG_KERNEL_LIMIT1 = 3, /* limiter pass 1 */
  GDG_KERNEL_LIMIT2 = 4, /* limiter pass 2 and the SSP combination */
  GDG_KERNEL_COUNT = 5
} gdg_kernel;
gdg_status gdg_profile(gdg_ctx *ctx, int32_t enable);
gdg_status gdg_profile_read(const gdg_ctx *ctx, double *ms_total, int64_t *launches);

/* Text of the last error on this context ("" if none); with ctx == NULL, the
 * reason of the last failed gdg_create() or gdg_solve_noalloc() on the
 * calling thread. */
const char *gdg_last_error(const gdg_ctx *ctx);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture of their own, tight serving loops, harnesses that forbid hipMalloc):
 * gdg_create() + gdg_upload_state() + gdg_run_to() + gdg_download_state() in
 * one call, with the workspace taken from a static device array of the
 * library instead of the caller.  The array holds GDG_NOALLOC_MAX_BYTES on
 * every GPU the library runs on, from the library's load until the process
 * ends; meshes whose gdg_workspace_bytes() exceed it are refused with
 * GDG_E_NOMEM.  The call allocates no device memory and captures no graph
 * (its device-driven steps are launched directly on hip_stream); it
 * synchronizes the stream before it returns.
 *
 * U0 (initial state) and U (final state) are SoA, (dim+2) * N doubles, host or
 * device memory, owned by the caller; t_final, max_steps and stats as for
 * gdg_run_to().  Every call on one GPU uses that GPU's one array: calls that
 * overlap on one GPU (other threads, other streams) race and corrupt each
 * other; calls in sequence are independent (the array's contents are
 * rewritten by each call before they are read).  Errors as for gdg_create()
 * and gdg_run_to(); the text is in gdg_last_error(NULL). */
#define GDG_NOALLOC_MAX_BYTES ((size_t)64 << 20)
gdg_status gdg_solve_noalloc(const gdg_mesh_desc *mesh, const gdg_params *prm, const double *U0, double *U,
                             double t_final, int64_t max_steps, void *hip_stream, gdg_stats *stats);

/* ---------------------------------------------------------------------------
 * Serving: many independent simulations on one GPU with continuous batching.
 *
 * A server owns a caller-provided device memory pool (its HBM budget) and a
 * stream.  gdg_server_submit() queues a request (mesh, scheme constants,
 * initial state, final time) without touching the GPU.  Each
 * gdg_server_pump() call
 *   1. waits for the previous batched launch and reads every resident
 *      request's time and flags (one small copy),
 *   2. retires finished requests: their state is copied to host memory held
 *      by the server and their workspace returns to the pool,
 *   3. redoes, host-driven, a step that a CFL violation halted (the restart
 *      rule of gdg_step),
 *   4. admits queued requests in arrival order while a slot is free and the
 *      pool has room for the request's workspace (gdg_workspace_bytes), and
 *   5. launches one captured graph of steps_per_graph SSP-RK3 steps of all
 *      resident requests and returns without waiting.
 * The graph's kernels are persistent: one grid walks the row blocks of every
 * resident request from a work list in device memory, so requests admitted
 * later join the next launch without a new capture.  Each request steps with
 * its own time step and stops at its own final time, as gdg_run_to() on a
 * context of its own would (same steps; results equal to rounding, since the
 * batched kernels are compiled apart and may contract other multiply-adds),
 * and its result does not depend on the other requests: it is bit-identical
 * alone and in any mix.  All requests of a server share one class: dim,
 * degree and precision (gdg_server_desc); the scheme constants may differ.
 * Calls on one server are not thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct gdg_server gdg_server;

typedef struct {
  int32_t dim, degree, precision; /* the request class */
  int32_t max_slots;              /* resident requests at most, 1 .. 256 */
  int32_t steps_per_graph;        /* SSP-RK3 steps per batched launch, >= 1 */
  int32_t solo_dofs;              /* > 0: a request of at least this many dofs is not batched; each
                                     launch replays its own single-mesh graph of 8 steps after the
                                     batched graph (large meshes fill the chip alone, and the
                                     single-mesh kernels run them faster); 0: every request is
                                     batched */
} gdg_server_desc;

typedef enum { GDG_REQ_PENDING = 0, GDG_REQ_RUNNING = 1, GDG_REQ_DONE = 2, GDG_REQ_FAILED = 3 } gdg_req_state;

typedef struct {
  int32_t state;    /* gdg_req_state */
  int32_t status;   /* gdg_status of a failed request, else GDG_OK */
  double t;         /* simulated time reached */
  int64_t steps;    /* SSP-RK3 steps taken */
  int64_t restarts; /* CFL restarts */
  int64_t ndofs;
  double submit_s;  /* host clock of submission, admission and completion, */
  double admit_s;   /* seconds since the server's creation (0 if not yet) */
  double done_s;
} gdg_request_info;

/* Device bytes of the pool that the server keeps for its work list; a pool
 * must be larger than this by at least one request's workspace. */
gdg_status gdg_server_overhead_bytes(const gdg_server_desc *desc, size_t *bytes);

/* Creates a server over dev_pool (caller-owned device memory of pool_bytes,
 * 256-byte aligned, alive until gdg_server_destroy) and hip_stream. */
gdg_status gdg_server_create(const gdg_server_desc *desc, void *dev_pool, size_t pool_bytes, void *hip_stream,
                             gdg_server **out);

/* Queues a request; U0 is a host state (SoA, (dim+2) * N doubles), copied,
 * as are the mesh's vertices (general cells) and boundary parts.
 * Unstructured meshes, continuous elements and GDG_SSPRK54 are not served
 * (GDG_E_INVALID).
 * GDG_E_INVALID for a description outside the server's class or bad
 * constants, GDG_E_BUDGET if its workspace exceeds the whole pool. */
gdg_status gdg_server_submit(gdg_server *srv, const gdg_mesh_desc *mesh, const gdg_params *prm, const double *U0,
                             double t_final, uint64_t *ticket);

/* One round of the serving loop (above).  *resident and *pending (may be
 * NULL) receive the requests on the GPU and still queued after the call. */
gdg_status gdg_server_pump(gdg_server *srv, int32_t *resident, int32_t *pending);

/* Waits for the launch in flight and processes it (steps 1-3 of a pump), without admitting or launching. */
gdg_status gdg_server_sync(gdg_server *srv);

/* State, counters and host timestamps of a request. */
gdg_status gdg_server_poll(const gdg_server *srv, uint64_t ticket, gdg_request_info *info);

/* Copies a finished request's final state to U (host, SoA) and forgets the
 * request.  GDG_E_INVALID if the ticket is unknown or not finished. */
gdg_status gdg_server_result(gdg_server *srv, uint64_t ticket, double *U);

/* Waits for the stream, releases every context and the server (not the pool). */
void gdg_server_destroy(gdg_server *srv);

const char *gdg_server_last_error(const gdg_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* GDG_H */
