/*
 * accfem.h - C ABI of the MI355X (gfx950) contact-FEM library.
 *
 * The library solves the quasi-static equilibrium of cable-driven continuum
 * robots discretised into co-rotational beam elements (Sec. II-B, eq. 1) under
 * cable actuation carried to the tip (Sec. II-E, eq. 16-18), a clamped and
 * inserted base (fixed-node constraints, eq. 14-15) and frictionless contacts
 * with a triangulated lumen wall (Sec. II-C, eq. 3-13).  Every load step runs a
 * Newton iteration whose linear steps are the quadratic programs of eq. 23,
 * solved exactly with a block-tridiagonal Cholesky factorisation, a
 * contact-space Schur complement and a finite active-set method, followed by
 * the step-size limit of eq. 25-27.  Many independent robots ("a batch")
 * are solved together on one GPU.
 *
 * Conventions
 *  - Units are SI.  Nodes of robot b are numbered 0..n_elem[b] from the base;
 *    node state arrays concatenate robots in order, 7 doubles per node:
 *    (px, py, pz, qw, qx, qy, qz) = position and unit quaternion of the node
 *    triad (columns: tangent, section y, section z).
 *  - Ownership: the caller owns every array.  Inputs are copied during the
 *    call; nothing is retained.  Outputs are written into caller buffers.
 *    When fem_params.io_on_device is 1, every array argument of the calls
 *    below is a device pointer on the context's device; otherwise host memory.
 *  - A context is not thread-safe.  Separate contexts are independent.
 *  - Errors: a negative fem_status and a message from fem_last_error().
 *    Invalid sizes, NULL pointers or non-positive material give FEM_E_INVAL
 *    and leave the context unchanged.
 */
#ifndef ACCFEM_H
#define ACCFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fem_ctx fem_ctx;

typedef enum {
  FEM_OK = 0,
  FEM_E_INVAL = -1,    /* bad argument */
  FEM_E_NOMEM = -2,    /* device allocation failed */
  FEM_E_HIP = -3,      /* HIP runtime error */
  FEM_E_STATE = -4,    /* call out of order (lumen / actuation not set) */
  FEM_E_NOCONV = -5    /* results written, some robots did not converge: see info */
} fem_status;

/* Arithmetic of the Newton loop.  FEM_FP64: everything in FP64.  FEM_MIXED: while a
 * robot's residual is above 1e-4 (N, N m) its element forces are evaluated in FP32
 * with FP32 accumulation (chord, stretch and relative rotations formed in FP64, then
 * cast), below it in FP64: the convergence decision is always taken on an FP64
 * residual (FP64 refinement of the Newton iteration); the element chord directions
 * that carry the QP tangent are stored in FP32 (the tangent blocks are regenerated
 * from them in FP64, so K stays positive definite) and contact detection screens
 * triangles in FP32 before deciding in FP64; the factorisation, the LCP and the state
 * stay FP64, so both precisions converge to the same equilibrium. */
typedef enum { FEM_FP64 = 0, FEM_MIXED = 1 } fem_precision;

/* Actuation kinds (Sec. II-E, eq. 16-18).  Cable j is attached at radius
 * cable_radius and angle cable_angle[j] in the tip section,
 * d_j = r (0, cos a_j, sin a_j), and pulls toward the base, F_j = -T_j e_x, both in
 * the tip frame T_M, which turns them into global axes (a follower load).
 *   CABLES: values[b*n_cables + j] = tension T_j (N); the tip node receives the
 *     moments sum_j d_j x F_j of eq. 16 only (the pull is carried inside the
 *     cable-tube pair, so it adds no net axial force).  Default of the workloads.
 *   CABLE_WRENCH: values as CABLES; the tip node receives eq. 17 as printed, the
 *     summed cable force sum_j F_j and the moments sum_j d_j x F_j.  The axial
 *     follower compression makes the QP-tangent iteration of eq. 20-23 converge only
 *     at small tensions (a few Euler loads of the robot).
 *   TIP_WRENCH_LOCAL: values[b*6..] = (F, M) in the tip frame (follower).
 *   TIP_WRENCH_GLOBAL: values[b*6..] = (F, M) in global axes (dead load). */
typedef enum {
  FEM_ACT_CABLES = 0,
  FEM_ACT_TIP_WRENCH_LOCAL = 1,
  FEM_ACT_TIP_WRENCH_GLOBAL = 2,
  FEM_ACT_CABLE_WRENCH = 3
} fem_act_kind;

/* QP method of the Newton iteration's linear step (eq. 23, Sec. III-B).
 *   FEM_QP_EXACT: block-tridiagonal Cholesky, contact-space Schur complement and a finite
 *     active-set LCP method (the exact QP solution).
 *   FEM_QP_ADMM: the operator-splitting iteration of OSQP, the solver the paper uses
 *     (Stellato et al. 2020, Algorithm 1, without problem scaling, fixed penalty admm_rho,
 *     sigma 1e-6, relaxation 1.6) on the same QP, with the block-tridiagonal factor of
 *     K + sigma I + rho A^T A (every contact row lies on one node) and one forward and
 *     backward sweep per iteration, until the primal and dual residuals are below
 *     admm_eps (absolute and relative) or admm_max_iter iterations. */
typedef enum { FEM_QP_EXACT = 0, FEM_QP_ADMM = 1 } fem_qp_solver;

/* Per-robot status in fem_solve_info.status */
enum {
  FEM_ROBOT_OK = 0,        /* last load step converged */
  FEM_ROBOT_NOCONV = 1,    /* max_newton iterations without convergence */
  FEM_ROBOT_LCPFAIL = 2,   /* the contact active-set method did not terminate */
  FEM_ROBOT_NONSPD = 3,    /* a Cholesky pivot was not positive */
  FEM_ROBOT_OVERFLOW = 4   /* more contacts than contact_capacity, or more than 48 at a node */
};

typedef struct {
  int32_t n_robots;           /* B >= 1 */
  const int32_t* n_elem;      /* [B] elements per robot, >= 1 (host) */
  const double* length;       /* [B] centreline length (host) */
  const double* base_pos;     /* [B*3] base node position before insertion (host) */
  const double* base_dir;     /* [B*3] centreline direction at the base (host) */
  const double* base_up;      /* [B*3] section y-axis at the base, not parallel to base_dir (host) */
  double r_out, r_in, E, nu;  /* tube section and material */
  double tip_len;             /* > 0: only the distal tip_len uses (r_out, r_in, E); */
  double shaft_E, shaft_A, shaft_I; /* elements proximal to it use this shaft */
  int32_t n_cables;           /* 1..8 */
  double cable_radius;        /* r of the cable attachment in the tip section */
  const double* cable_angle;  /* [n_cables] angles in the tip section (host) */
  double contact_radius;      /* r_c: robot radius offset of the wall constraint */
  double contact_margin;      /* delta: detection band beyond r_c */
  double beta0;               /* step-size limit (max node translation per step) */
  double guide_len;           /* straight insertion guide from the initial base; 0 = none.
                                 Requires base_dir along a coordinate axis. */
  double newton_tol;          /* residual 2-norm over free DOFs (N, N m) */
  double stag_tol;            /* accept a stagnating residual below this */
  int32_t max_newton;         /* Newton iterations per load step */
  int32_t contact_capacity;   /* max contacts per robot (<= 1024) */
  double grid_cell;           /* uniform-grid cell size for the lumen, 0 = automatic */
  fem_precision precision;    /* FEM_FP64 or FEM_MIXED */
  void* hip_stream;           /* hipStream_t to run on, or NULL: the null stream for copies
                                 and a stream of the context's own for the load-step loop */
  int32_t io_on_device;       /* 1: array arguments of later calls are device pointers */
  int32_t profile;            /* 1: time every kernel launch with HIP events (fem_profile) */
  int32_t autotune;           /* 1: the launch shapes of the element update and contact
                                 detection are picked by timing during the first solve
                                 (fem_tuning) */
  int32_t qp_solver;          /* fem_qp_solver; FEM_QP_EXACT = 0 */
  double admm_rho;            /* FEM_QP_ADMM penalty (N/m); 0 = 1 */
  double admm_eps;            /* FEM_QP_ADMM tolerance; 0 = 1e-11 */
  int32_t admm_max_iter;      /* FEM_QP_ADMM iteration limit per linear step; 0 = 20000 */
  int32_t contact_along_elements; /* 1: contacts anywhere along an element as well (eq. 3-7
                                 with 0 < xi < l0): the chord of every element whose two
                                 nodes are contact nodes against the edges and vertices of
                                 the wall, kind 2; needs FEM_QP_EXACT */
} fem_params;

typedef struct {
  int32_t status;           /* FEM_ROBOT_* of the last load step */
  int32_t iters;            /* Newton iterations of the last load step */
  int32_t n_contacts;       /* contacts of the last iterate */
  int32_t n_limited;        /* step-limited iterations in the last load step */
  double res_norm;          /* residual norm at the last check */
  int32_t steps_converged;  /* converged load steps since fem_create / fem_set_state */
  int32_t steps_total;      /* load steps since fem_create / fem_set_state */
  int64_t iters_total;      /* Newton iterations since fem_create / fem_set_state */
  int64_t rhs_total;        /* right-hand sides solved (1 + contacts per Newton step), same span */
  int64_t rhs_fused;        /* of those, swept forward inside the factorisation (the first 64
                               of each Newton step), same span */
  int64_t sweep_passes;     /* substitution passes of 64 right-hand sides (none for a Newton
                               step without contacts), same span */
  int64_t qp_iters_total;   /* FEM_QP_ADMM iterations, same span (0 for FEM_QP_EXACT) */
  int64_t products_total;   /* contact products n_i . x formed by the substitution, (1 +
                               contacts) x contacts per Newton step, same span */
  int64_t contact_steps_total; /* Newton steps with at least one contact, same span */
} fem_solve_info;

typedef struct {
  int32_t robot, node, tri; /* node index within its robot; triangle index of the lumen */
  int32_t kind;             /* 0 = face contact, 1 = edge/vertex contact (at the node),
                               2 = contact along the element from node to node + 1 */
  double n[3];              /* unit normal pointing from the wall into the lumen */
  double gap;               /* gap at the last iterate (m) */
  double force;             /* contact force magnitude y >= 0 (N) of the last linear step */
  double s;                 /* kind 2: the contact point's position xi / l0 along the element
                               (0 < s < 1; row (1 - s) n^T on node, s n^T on node + 1);
                               0 for the other kinds */
} fem_contact;

/* Create a context for a batch of robots (Sec. II-B: each robot is split into
 * n_elem equal beam elements of length l0 = length / n_elem along its centreline,
 * six DOF per node; section and material as in Table I).  Allocates device memory
 * for all of them and places every robot in its straight reference configuration
 * S_0 of eq. 3 (node i at base_pos + i l0 base_dir, triads [base_dir, base_up, x]).
 * p and its arrays are host memory, read during the call.  *out receives the
 * context (the caller frees it with fem_destroy), or NULL on error; FEM_E_INVAL for
 * out-of-range sizes or material (message from fem_last_error(NULL)), FEM_E_NOMEM,
 * FEM_E_HIP. */
fem_status fem_create(const fem_params* p, fem_ctx** out);

/* Free the context and all its device memory (library bookkeeping, no passage of
 * the method).  Waits for the context's stream first.  NULL is ignored. */
void fem_destroy(fem_ctx* c);

/* Message of the last error on this context, or of the last failed fem_create for
 * NULL (library bookkeeping, no passage of the method).  The string is owned by the
 * library and valid until the next call on c. */
const char* fem_last_error(const fem_ctx* c);

/* Upload the lumen mesh, the triangulated cavity wall whose planes bound the nodes
 * in the contact constraint of eq. 3 (Sec. II-C) and that detection matches nodes
 * against (Sec. III-C): verts [n_verts*3] (x y z per vertex), tris [n_tris*3] vertex
 * indices with winding (v1-v0)x(v2-v0) pointing into the lumen.  Both follow
 * io_on_device and are copied.  Builds the triangle planes and the uniform grid used
 * by contact detection.  n_tris may be 0 (no wall).  FEM_E_INVAL: negative sizes,
 * NULL arrays, an index out of range or a degenerate triangle (the previous mesh is
 * then dropped). */
fem_status fem_set_lumen(fem_ctx* c, const double* verts, int64_t n_verts,
                         const int32_t* tris, int64_t n_tris);

/* Set the actuation (Sec. II-E, eq. 16-18) and the insertion depth reached at the
 * end of the next fem_solve call.  The depth moves the clamped base node along
 * base_dir: the prescribed displacement b_fn of the fixed-node constraint (Sec. II-D,
 * eq. 14-15), the insertion of Sec. IV-B.  values: [B*n_cables] (CABLES,
 * CABLE_WRENCH) or [B*6] (tip wrench kinds); insertion_depth: [B] or NULL (= 0); both
 * follow io_on_device and are copied.  The kind must not change between calls
 * (FEM_E_INVAL). */
fem_status fem_set_actuation(fem_ctx* c, fem_act_kind kind, const double* values,
                             const double* insertion_depth);

/* Run n_load_steps quasi-static load steps, each solved to the equilibrium of the
 * complementarity problem of eq. 19 by a Newton iteration whose linear steps are
 * the quadratic programs of eq. 23 (Sec. III-A, III-B) with the step-size limit of
 * eq. 25-27 (Sec. III-D).  Load step j applies
 * prev + (target - prev) * j / n_load_steps of the actuation and depth, where
 * prev is what the previous call reached (0 initially) and target the values
 * of fem_set_actuation.  Each load step starts from the previous state.
 * n_load_steps = 0 solves nothing and takes the target as reached, so that it
 * starts the next ramp (e.g. after fem_set_state with a state at that load).  Every robot
 * advances through the load steps on its own (see fem_solve_schedule).
 * node_state [total_nodes*7] and info [B] may be NULL.  Returns FEM_E_NOCONV
 * if any robot's last load step did not converge (outputs still written). */
fem_status fem_solve(fem_ctx* c, int32_t n_load_steps, double* node_state,
                     fem_solve_info* info);

/* Run an explicit schedule of quasi-static load steps (Sec. III-A: each time step of the
 * insertion solves the equilibrium of eq. 19 with the QP of eq. 23 and the step-size
 * limit of eq. 25-27), e.g. tensions ramped over the first load steps and the insertion
 * depth over all of them.  Step k (1-based) of robot b applies the actuation values
 * values[((k-1)*B + b)*n_values ..] of `kind` (n_values = n_cables for the cable kinds,
 * 6 for the tip wrenches) and the insertion depth insertion_depth[(k-1)*B + b] (NULL:
 * the depth stays where the previous call left it).  Every robot advances through the
 * steps on its own: a robot whose load step has ended starts its next one while other
 * robots are still iterating, so the results equal those of n_load_steps calls of
 * fem_set_actuation + fem_solve(1) with the same values.  The last step's values become
 * the target reached (a later fem_solve ramps from them).  Optional per-step records
 * (NULL to skip): rec_tip [n_load_steps*B*3] tip-node position at the end of each load
 * step, rec_status [n_load_steps*B] its FEM_ROBOT_* status, rec_iters [n_load_steps*B]
 * its Newton iterations, step-major like the inputs.  values, insertion_depth and the
 * records follow io_on_device; node_state and info as in fem_solve.  FEM_E_INVAL:
 * n_load_steps < 1, NULL values or a kind different from the context's.  FEM_E_STATE: no
 * lumen set.  Returns FEM_E_NOCONV if any robot's last load step did not converge. */
fem_status fem_solve_schedule(fem_ctx* c, fem_act_kind kind, int32_t n_load_steps,
                              const double* values, const double* insertion_depth,
                              double* node_state, fem_solve_info* info, double* rec_tip,
                              int32_t* rec_status, int32_t* rec_iters);

/* Contacts of the last iterate of robot `robot` (-1 = all robots, in order): the
 * rows of A_c (normal n_i, eq. 9), the gaps b_c (eq. 10) and the contact forces y_c
 * (eq. 11), i.e. the collision positions that detection returns (Sec. III-C).
 * out [capacity] follows io_on_device.  Writes min(total, capacity) entries;
 * *n_out (host) = total even if larger.  FEM_E_INVAL: robot out of range, NULL
 * n_out, or capacity > 0 with NULL out. */
fem_status fem_contacts(const fem_ctx* c, int32_t robot, fem_contact* out,
                        int32_t capacity, int32_t* n_out);

/* Adjoint gradient at the converged state of the last load step (equilibrium of
 * eq. 19 with the contact conditions of eq. 12-13 and the fixed-node constraints of
 * eq. 14-15; the adjoint is an addition to the method).  For a loss L on node positions, given dL/dp of n_sensors sensor
 * nodes per robot, writes dL/du for the actuation values u of the last
 * fem_set_actuation kind: the cable tensions [B*n_cables] for FEM_ACT_CABLES and
 * FEM_ACT_CABLE_WRENCH, else the tip wrench [B*6].  It solves J^T lam + A_act^T mu = dL/dx,
 * A_act lam = 0 with the exact Jacobian J of the out-of-balance force (element
 * material and geometric stiffness plus the follower-load stiffness), the active
 * contacts (force > 0) held as planes at their normals and the base and guided
 * lateral DOFs fixed, then dL/du_j = lam . dF_a/du_j.  Always FP64.  A robot with an
 * active contact along an element (kind 2) is not supported: its entries are NaN and the
 * call returns FEM_E_NOCONV.
 *   sensor_nodes [n_sensors] host memory: node index i >= 0 counts from the base,
 *                i < 0 from the tip (-1 = tip), the same for every robot
 *   dL_dp        [B*n_sensors*3] robot-major, then sensor, then x y z
 *   dL_du        [B*n_cables] or [B*6] output
 * dL_dp and dL_du follow io_on_device.  The device workspace (about 1 KB per node)
 * is allocated on the first call and kept by the context.  FEM_E_INVAL: NULL
 * pointers, n_sensors < 1 or a sensor index outside some robot.  FEM_E_STATE: no
 * converged-or-not load step solved since creation or the last fem_set_state.
 * FEM_E_NOCONV: some robot's last load step did not converge, or its adjoint
 * system was singular; its entries are NaN, the others are valid. */
fem_status fem_grad(fem_ctx* c, const int32_t* sensor_nodes, int32_t n_sensors,
                    const double* dL_dp, double* dL_du);

/* Copy the nodal configuration x_t of eq. 1 (Sec. II-B), node state
 * [total_nodes*7] in the layout above, out of / into the context; node_state
 * follows io_on_device.  fem_set_state also resets the per-robot statistics;
 * quaternions are renormalised.  FEM_E_INVAL for NULL. */
fem_status fem_get_state(const fem_ctx* c, double* node_state);
fem_status fem_set_state(fem_ctx* c, const double* node_state);

/* Evaluate the out-of-balance force F(x) - F_a of eq. 1 and 18, the tangent
 * K(x) of eq. 20 and contact detection (Sec. III-C) at the current state under
 * the actuation and depth set by the last fem_set_actuation (no Newton step):
 * F [total_nodes*6] = internal force minus actuation per node, KD and KS
 * [total_nodes*36] = row-major 6x6 diagonal block of each node and its
 * coupling block K[i, i+1] of the QP tangent (eq. 20-23).  Any output may be
 * NULL.  Afterwards fem_contacts returns the detected contacts (force 0).
 * Intended for verification of the element and detection kernels. */
fem_status fem_eval(fem_ctx* c, double* F, double* KD, double* KS);

/* Measurement, not part of the method.  Kernel timing of a context created with
 * profile = 1: for kernel class k
 * (0 = element update, 1 = contact detection, 2..6 = the Newton step's phases:
 * convergence test + right-hand sides, block Cholesky, substitutions (contact
 * products), contact forces (LCP), step solve + state update) the
 * accumulated device time in ms measured with HIP events on the context's
 * stream, and the number of launches, since the last call with reset = 1. */
fem_status fem_profile(fem_ctx* c, int32_t kernel, double* total_ms, int64_t* launches,
                       int32_t reset);

/* Solve one linear complementarity problem  w = W y + q >= 0, y >= 0, y . w = 0
 * (the contact conditions of eq. 12 for the contact forces y, with W = A_c K^-1 A_c^T
 * the contact-space Schur complement) with the device routines that fem_solve applies
 * to a robot's contact set; no context.  Intended for verification of those routines.
 *   W [m*m] symmetric positive semidefinite, column-major; q [m]; y [m] output; host memory
 *   *path: the routine taken, 0 = active set with W packed in LDS (m <= 64),
 *          1 = wavefront active set with W columns in device memory and the Cholesky
 *          factor of the active block in LDS (m > 64), 2 = that routine's single-lane
 *          fallback once the active set outgrows 128 positions
 * Runs on the null stream of the current device and allocates and frees its own device
 * buffers.  FEM_E_INVAL: NULL pointers or m outside 1..1024.  FEM_E_NOCONV: a
 * non-positive pivot, a dependent constraint that no active one can give way to (no
 * solution), or the iteration limit (y not written).  FEM_E_NOMEM, FEM_E_HIP. */
fem_status fem_lcp(const double* W, const double* q, int32_t m, double* y, int32_t* path);

/* Largest m accepted by fem_lcp_noalloc. */
#define FEM_LCP_NOALLOC_MAX_M 512

/* fem_lcp without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same device
 * routines and results as fem_lcp, with the caller's device buffers and a workspace held in
 * a fixed device array of the library (about 1.1 MB: the HBM factor of up to
 * FEM_LCP_NOALLOC_MAX_M positions and a result code), one per GPU, kept until the process
 * ends.  No hipMalloc, hipFree or other allocating call is made.
 *   W [m*m] column-major, q [m], y [m] output: device pointers on the current device
 *   path: host pointer, the routine taken (as fem_lcp)
 *   hip_stream: hipStream_t the routines run on (NULL = the null stream); the call waits
 *     for it before returning
 * Every call on one GPU uses that GPU's workspace, which keeps the last call's contents;
 * calls that overlap on one GPU (other threads, other streams) race and must be
 * serialised by the caller.  FEM_E_INVAL: NULL pointers or m outside
 * 1..FEM_LCP_NOALLOC_MAX_M.  FEM_E_NOCONV as fem_lcp (y then undefined).  FEM_E_HIP. */
fem_status fem_lcp_noalloc(const double* W, const double* q, int32_t m, double* y,
                           int32_t* path, void* hip_stream);

/* Launch shapes of the context (a measurement aid, no passage of the method): threads per
 * block of the element update and lanes per node of contact detection, as picked by the
 * autotuner of a context created with autotune = 1, once, after 512 Newton passes of its
 * first fem_solve / fem_solve_schedule call (or at the end of that call if it is shorter),
 * each candidate timed with HIP events on the state reached (64, 128, 256 threads; 4, 8, 16
 * lanes); else the defaults 256 and 8.  times_us [6] (or NULL) receives
 * the measured median launch times in that order (NaN before tuning).  The results of the
 * method do not depend on the shapes.  Any output may be NULL. */
fem_status fem_tuning(const fem_ctx* c, int32_t* elem_block, int32_t* detect_lanes,
                      double* times_us);

/* Total number of nodes over the batch (Sec. II-B: n_elem + 1 per robot, summed),
 * or -1 for NULL. */
int64_t fem_total_nodes(const fem_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* ACCFEM_H */
