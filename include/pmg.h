/*
 * pmg: MI355X-native DGSEM compressible Navier-Stokes residual, FAS p-multigrid and in-cycle anisotropic
 * truncation-error estimation, behind a plain C ABI.
 *
 * Method: Rueda-Ramirez, Manzanero, Ferrer, Rubio, Valero, "A p-Multigrid Strategy with Anisotropic
 * p-Adaptation Based on Truncation Errors for High-Order Discontinuous Galerkin Methods" (J. Comput.
 * Phys.), cited below by section and equation.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Problem (Sec. 3.1, eq. NonLinFAS): find the nodal solution Q of A(Q) = S, where A = [M]^{-1} F is the
 *   DGSEM spatial operator (Sec. 2, eqs. DiscretNSElem/DiscretNS) of the non-dimensional compressible
 *   Navier-Stokes equations (Appendix A) and S the nodal source.  The residual is r = S - A(Q)
 *   (eq. nonlinRes).
 * - Elements are hexahedra with reference coordinates (xi, eta, zeta) in [-1,1]^3 and per-element,
 *   per-direction orders (N1, N2, N3), 1 <= N_d <= 7.  Element e holds (N1+1)(N2+1)(N3+1) nodes numbered
 *   i + (N1+1)(j + (N2+1) k), xi fastest.  Node family: Legendre-Gauss (the paper's) or Gauss-Lobatto.
 * - State arrays are FP64, variable-major "[5][n_nodes]": all rho values, then rho u, rho v, rho w,
 *   rho e; nodes of element 0 first, then element 1, ...  pmg_state_layout gives n_nodes and offsets.
 * - Faces are numbered 0..5 = xi-, xi+, eta-, eta+, zeta-, zeta+.  Face-local coordinates (s, t) are the two
 *   tangential reference coordinates in increasing axis order.  Orientation code o (0..7) of face f of
 *   element e towards its neighbour face f' maps (s, t) on e's face to (s', t') on the neighbour's face:
 *   (u, v) = (t, s) if (o & 4) else (s, t); s' = -u if (o & 1) else u; t' = -v if (o & 2) else v.
 * - Boundary tags: 0 interior or periodic (has a neighbour), 1 no-slip adiabatic wall, 2 far field (also
 *   the uniform inflow), 3 free-slip wall, 4 subsonic outflow with only the far-field pressure imposed (the
 *   flat-plate case of Sec. 4.1).  Far field is rho = 1, v = (1, 0, 0), p = 1 / (gamma M^2); the outflow
 *   ghost state keeps the interior density and velocity with that pressure.  The viscous flux on far field
 *   and outflow faces is the interior one.
 * - Pointers named *_dev are device pointers on the solver's GPU; the caller owns them (for example the
 *   data_ptr() of torch tensors) and keeps them alive until the stream has consumed them.  Host arrays
 *   are copied during the call and may be freed afterwards.  The library owns its handles and every
 *   internal device buffer (metrics, level states, face arrays).
 * - stream is a hipStream_t (NULL = the default stream).  Every call is asynchronous on it, except that a
 *   non-NULL host out-pointer (res_inf_host, dt_host, ...) makes the call wait for its result.
 * - Every call returns a pmg_status; on failure pmg_last_error() describes it (thread-local text, valid
 *   until the next call on the same thread).  No C++ exception crosses the ABI.  Handles are not
 *   thread-safe: use one handle per thread, or serialise.
 */
#ifndef PMG_H
#define PMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PMG_OK = 0,
  PMG_ERR_INVALID_ARG = 1,   /* a size, order, table entry or pointer is out of range */
  PMG_ERR_OOM = 2,           /* device allocation failed */
  PMG_ERR_HIP = 3,           /* a HIP runtime call failed */
  PMG_ERR_NONPHYSICAL = 4,   /* non-finite residual, or rho <= 0 / p <= 0 detected at a sync point */
  PMG_ERR_NOT_CONVERGED = 5, /* pmg_solve reached max_cycles */
  PMG_ERR_BUSY = 6,
  PMG_ERR_UNIMPLEMENTED = 7
} pmg_status;

typedef struct pmg_ctx_s* pmg_ctx;       /* one GPU */
typedef struct pmg_mesh_s* pmg_mesh;     /* geometry + connectivity, copied to the GPU */
typedef struct pmg_solver_s* pmg_solver; /* mesh + order tensor + physics + multigrid hierarchy */
typedef struct pmg_server_s* pmg_server; /* continuous-batching solve server on one GPU */

/* Physics (Appendix A; CFL constants of Sec. 2). */
typedef struct {
  double mach;        /* far-field Mach number M */
  double reynolds;    /* far-field Reynolds number Re */
  double prandtl;     /* 0.72 */
  double gamma;       /* 1.4 */
  double sutherland;  /* Sutherland constant over the reference temperature, 110.4 / 288.15 */
  double cfl_adv;     /* C^a of the advective step limit */
  double cfl_visc;    /* C^nu of the diffusive step limit */
  int32_t node_family;     /* 0 Legendre-Gauss, 1 Legendre-Gauss-Lobatto */
  int32_t viscosity_model; /* 0 Sutherland's law, 1 constant viscosity */
} pmg_physics;

/* FAS p-multigrid (Sec. 3.1, Algorithm "FAS: V-Cycle"; Secs. 3.1.1-3.1.2; Sec. 3.3.3). */
typedef struct {
  int32_t n_levels;          /* number of isotropic levels; 0 = max order (Delta N = 1 down to order 1) */
  const int32_t* level_caps; /* host, n_levels entries finest first, e.g. {3, 1}; NULL = max, max-1, ..., 1.
                                Level with cap c holds min(N_d, c) in every direction (high-order coarsening). */
  int32_t beta_pre;          /* pre-smoothing RK3 sweeps (beta_1, or beta_1^0 with tuning) */
  int32_t beta_post;         /* post-smoothing sweeps (beta_2, or beta_2^0 with tuning) */
  int32_t beta_coarse;       /* sweeps on the coarsest level (replace pre + post there) */
  int32_t tuning;            /* 0 fixed sweeps; 1 residual-based tuning of Sec. 3.1.2 */
  double eta;                /* pre-smoothing tuning factor (1.1) */
  int32_t max_repeats;       /* cap on tuning repetitions per smoothing phase */
  int32_t fmg;               /* 1: pmg_solve starts with a full-multigrid ramp */
  double fmg_threshold;      /* residual that raises the FMG level (1e-1 plate, 1.0 sphere) */
  int32_t precision;         /* 0: every level in FP64.  1: mixed precision, with the isotropic levels below the
                                finest smoothed in FP32.  Their state Q~ is the FP64 restriction rounded once;
                                their FAS source is A(Q~) + r formed by the same FP32 operator, so Q~ = Q~0
                                leaves exactly r.  Their correction Q~ - Q~0 is taken in FP32 and added in FP64.
                                The finest level, its residual, the stopping test and the truncation-error
                                hierarchies stay FP64.  pmg_solve / pmg_batch_solve switch a problem to FP64
                                coarse levels once its FP64 residual stops reaching new minima (the round-off
                                floor of the FP32 correction), so the converged solution is an FP64 solution. */
  int32_t mixed_patience;    /* precision 1: stalled cycles before the switch (0 = 4).  A cycle is stalled when
                                the residual reaches no new minimum, has fallen below its first value of the
                                call, stays within twice its best and did not rise over the cycle (a floor
                                hovers; a start-up transient rises cycle after cycle); a cycle the divergence
                                guard rolled back restarts the count. */
  int32_t guard;             /* divergence guard of pmg_solve / pmg_batch_solve: 0 off; n > 0: a problem whose
                                residual check is non-finite or grew more than 1e4-fold over one cycle gets
                                back its state of the previous check (of the start of the call if it fails
                                again before an accepted check) and both explicit step constants halved, at
                                most n times.  A problem that still fails keeps its last accepted state:
                                pmg_solve returns PMG_ERR_NONPHYSICAL; pmg_batch_solve freezes it, finishes
                                the others, reports its residual as NaN and returns PMG_ERR_NONPHYSICAL (its
                                outputs filled).  The halved constants stay with the solver
                                (pmg_guard_stats).  Device memory: two copies of the finest state. */
} pmg_mg_params;

const char* pmg_last_error(void);

pmg_status pmg_ctx_create(int hip_device, pmg_ctx* out);
void pmg_ctx_destroy(pmg_ctx ctx);

/*
 * Mesh (Sec. 2, eq. mapping): K hexahedra with a tensor-product Lagrange mapping of degree M = (M1,M2,M3)
 * (1 <= M_d <= 4), given by its values at equispaced reference nodes.
 *   geom_nodes: host, K*(M1+1)*(M2+1)*(M3+1)*3 doubles, [e][k][j][i][xyz] (xi index i fastest).
 *   nbr_elem:   host, K*6, neighbour element of each face, -1 on a boundary face.
 *   nbr_face:   host, K*6, the neighbour's face number.
 *   orient:     host, K*6, orientation code towards the neighbour (see above).
 *   bc:         host, K*6, boundary tag (0 where a neighbour exists).
 * Errors: PMG_ERR_INVALID_ARG for inconsistent connectivity (neighbour not pointing back, codes out of
 * range, boundary face tagged 0).
 */
pmg_status pmg_mesh_create(pmg_ctx ctx, int64_t K, const int32_t M[3], const double* geom_nodes,
                           const int64_t* nbr_elem, const int32_t* nbr_face, const int32_t* orient,
                           const int32_t* bc, pmg_mesh* out);
void pmg_mesh_destroy(pmg_mesh mesh);

/*
 * Solver: mesh + order tensor (host, K*3 int32, each 1..7) + physics + multigrid parameters.  Builds the
 * isotropic level hierarchy (high-order coarsening, Sec. 3.3.3) and, lazily, the three one-direction
 * hierarchies of the anisotropic cycle (Sec. 3.3.1).  Metric terms are computed on the GPU for every
 * level's own orders (curl form, Sec. 2).  The mesh must outlive the solver.
 */
pmg_status pmg_solver_create(pmg_ctx ctx, pmg_mesh mesh, const int32_t* orders, const pmg_physics* phys,
                             const pmg_mg_params* mg, pmg_solver* out);
void pmg_solver_destroy(pmg_solver s);

/* n_nodes = sum_e (N1+1)(N2+1)(N3+1) (the paper's DOF count); elem_node_offset (host, K+1, nullable). */
pmg_status pmg_state_layout(pmg_solver s, int64_t* n_nodes, int64_t* elem_node_offset);

/* Q_dev[5][n_nodes] <- the far-field state. */
pmg_status pmg_init_freestream(pmg_solver s, double* Q_dev, void* stream);

/*
 * Residual r = S - A(Q) on the finest level (eq. nonlinRes).  op = 0: DGSEM operator with Roe advective
 * and Bassi-Rebay 1 viscous numerical fluxes, mortars on p-nonconforming faces (Sec. 2, eq. weak2);
 * op = 1: isolated operator, every numerical flux replaced by the element's own physical flux
 * (Sec. 3.2.1, eq. IsolTruncErrorSteady).  S_dev may be NULL (S = 0).  R_dev[5][n_nodes] is written.
 * res_inf_host (nullable) receives max |r| over nodes and variables (waits for the stream).
 */
pmg_status pmg_residual(pmg_solver s, int op, const double* Q_dev, const double* S_dev, double* R_dev,
                        double* res_inf_host, void* stream);

/* CFL step of Sec. 2 for Q on the finest level: min over nodes and directions of
 * min(C^a h_d / ((|v| + c) N_d^2), C^nu h_d^2 / (nu N_d^4)), h_d = 2 J / |J a^d|, nu = mu / (rho Re). */
pmg_status pmg_timestep(pmg_solver s, const double* Q_dev, double* dt_host, void* stream);

/* 'sweeps' sweeps of Williamson's low-storage RK3 (Sec. 3.1) on the finest level, the step recomputed
 * from Q at the start of each sweep: G <- a_s G + dt r(Q); Q <- Q + b_s G. */
pmg_status pmg_smooth(pmg_solver s, double* Q_dev, const double* S_dev, int sweeps, void* stream);

/*
 * Level hierarchy.  hierarchy = -1 for the isotropic one, 0/1/2 for the one that coarsens only xi/eta/zeta.
 * Level index 0 is the coarsest; the last is the finest (the solver's orders).  pmg_level_info returns the
 * number of levels when level < 0, else that level's node count and (nullable) its orders (host K*3).
 */
pmg_status pmg_level_info(pmg_solver s, int hierarchy, int level, int32_t* n_levels, int64_t* n_nodes,
                          int32_t* orders);
/* L2 projection (restriction, eqs. FASCoarseSol/FASCoarseRes) of U from level 'level' to level-1, and
 * exact interpolation (prolongation, eq. FASCorrectSol) from 'level' to level+1; [5][n] arrays. */
pmg_status pmg_restrict(pmg_solver s, int hierarchy, int level, const double* Ufine_dev, double* Ucoarse_dev,
                        void* stream);
pmg_status pmg_prolong(pmg_solver s, int hierarchy, int level, const double* Ucoarse_dev, double* Ufine_dev,
                       void* stream);

/*
 * n_cycles isotropic FAS V-cycles (Algorithm "FAS: V-Cycle" with iteration error eps = Q~ - Q~_0,
 * eq. FASIterError) on Q_dev (in/out) with physical source S_dev (nullable).  res_inf_host (nullable)
 * receives max |S - A(Q)| after the last cycle.
 */
pmg_status pmg_vcycle(pmg_solver s, double* Q_dev, const double* S_dev, int n_cycles, double* res_inf_host,
                      void* stream);

/* Steady solve: optional FMG start, then V-cycles until max |r| < tol (checked on the host after every
 * cycle).  Returns PMG_ERR_NOT_CONVERGED when max_cycles is reached first. */
pmg_status pmg_solve(pmg_solver s, double* Q_dev, const double* S_dev, double tol, int max_cycles, int* cycles_out,
                     double* res_inf_out, void* stream);

/*
 * Anisotropic truncation-error estimate inside the multigrid cycle (Secs. 3.2.1 and 3.3.1, eqs. TruncError!
 * and AnisTruncError): one V-cycle per direction d, coarsening only d ("3V" cycle), each starting from the
 * previous one's result; Q_dev is smoothed in place by the three cycles.  At the entry of each coarse level
 * with cap n, tau = S_phys - A^n(I Q~) (isolated = 0, reusing the coarse-source operator evaluation) or
 * tau^ = S_phys - A^^n(I Q~) (isolated = 1), S_phys the physical source restricted level by level.
 * tau_map_dev: device, K*3*nt doubles with nt = (max order) - 1, [e][d][n-1] = max over the element's nodes
 * and variables of |tau| for n < N_d^e, NaN otherwise.  Sweeps per level come from the solver's params.
 */
pmg_status pmg_tau_estimate(pmg_solver s, double* Q_dev, const double* S_dev, int isolated, double* tau_map_dev,
                            void* stream);
/* Residual history of the last pmg_solve: ||r||_inf at every check (the start and after each cycle).  n
 * receives the number of entries; at most 'capacity' are copied to out (host). */
pmg_status pmg_solve_history(pmg_solver s, double* out, int32_t capacity, int32_t* n);
/* V-cycles run on the solver's state since creation or the last restore (pmg_vcycle, pmg_solve). */
pmg_status pmg_cycle_count(pmg_solver s, int64_t* cycles);
/*
 * Checkpoint / resume.  pmg_checkpoint writes to 'path' (through 'path'.tmp and a rename) the fine state
 * Q_dev, the orders, the cycle counter and the residual history, with a checksum; every coarse level is
 * rebuilt from the fine state by each cycle, so nothing else carries over.  pmg_restore checks the file
 * (checksum, same mesh size, orders and problem count, else PMG_ERR_INVALID_ARG) and writes the state into
 * Q_dev: cycles run from it reproduce, bitwise, those run from the state that was saved.
 */
pmg_status pmg_checkpoint(pmg_solver s, const char* path, const double* Q_dev, void* stream);
pmg_status pmg_restore(pmg_solver s, const char* path, double* Q_dev, void* stream);

/*
 * Pointwise truncation error of one anisotropic level (Sec. 3.3.1; the quantity the tau map reduces): runs
 * the anisotropic V-cycle of direction dir on Q_dev (as pmg_tau_estimate does for that direction, so Q_dev
 * is updated by that one cycle) and writes tau = S_phys - A(Q~0) (isolated = 0) or S_phys - A^(Q~0)
 * (isolated = 1) of the level whose order in dir is capped at 'order' (1 <= order < max order in dir) into
 * tau_dev, layout [5][n_nodes of that level] (pmg_level_info(dir, level) gives the level's orders; elements
 * in user order).  Elements whose order in dir is at most 'order' are not coarsened there and hold the
 * residual of the restricted state.
 */
pmg_status pmg_tau_nodal(pmg_solver s, int dir, int order, double* Q_dev, const double* S_dev, int isolated,
                         double* tau_dev, void* stream);

/*
 * Batches of independent steady problems (many solves advanced together by the same V-cycle).  The n
 * problems become one solver over the union of their elements (no faces between problems): every kernel
 * launch covers all problems, elements are bucketed per (problem, order triple), and the explicit step and
 * the residual norms are reduced per problem, so each problem's arithmetic is the same as in its own solve.
 * Requirements: one node family and the same maximum order for all problems (their level sequences then
 * coincide), fixed sweep counts (no residual-based tuning).  Mapping orders may differ (lower ones are
 * raised exactly).  The batch state is the concatenation of the problems' states in problem order
 * ([5][total nodes]); pmg_batch_layout gives the n+1 node offsets.  All single-problem entry points
 * accept a batch handle and act on every problem at once.
 */
pmg_status pmg_batch_create(pmg_ctx ctx, int n, const pmg_mesh* meshes, const int32_t* const* orders,
                            const pmg_physics* phys /* n entries */, const pmg_mg_params* mg, pmg_solver* out);
pmg_status pmg_batch_layout(pmg_solver s, int* n_problems, int64_t* problem_node_offset /* n+1, nullable */);
/* res_inf_host: host, n entries, max |S - A(Q)| of each problem (waits for the stream). */
pmg_status pmg_batch_norms(pmg_solver s, const double* Q_dev, const double* S_dev, double* res_inf_host,
                           void* stream);
/* V-cycles until every problem is below tol; a converged problem is frozen (the tiles of its elements and
 * faces skip the cycle's work, so its state no longer changes) while the others continue.  With mixed
 * precision, problems on FP32 coarse levels and problems already switched to FP64 ones advance in two
 * cycles per iteration, each skipping the other set.  cycles_out / res_inf_out: n entries. */
pmg_status pmg_batch_solve(pmg_solver s, double* Q_dev, const double* S_dev, double tol, int max_cycles,
                           int32_t* cycles_out, double* res_inf_out, void* stream);
/*
 * Device footprint of a single-problem solver for (mesh, orders, mg) as pmg_solver_create builds it,
 * counted on the host from the connectivity and the orders: every level's geometry, face and work arrays,
 * the multigrid arrays of the isotropic hierarchy and the solver's own arrays; not the mesh's geometry
 * nodes.  Built later, on first use, and reported apart: transient_bytes (nullable), the extra memory held
 * while a level's geometry is computed during construction; switch_bytes (nullable), the FP64 coarse
 * hierarchy a mixed-precision solver builds when it switches precision (0 with precision 0).  The
 * anisotropic truncation-error hierarchies of pmg_tau_estimate are not counted.
 */
pmg_status pmg_footprint(pmg_mesh mesh, const int32_t* orders, const pmg_mg_params* mg, int64_t* bytes,
                         int64_t* transient_bytes, int64_t* switch_bytes);
/* Device bytes currently allocated by the library (every handle, every device). */
pmg_status pmg_device_bytes(int64_t* bytes);

/*
 * Serving (steady solves of independent problems arriving over time).  A request is a problem (mesh,
 * orders, physics, multigrid parameters without tuning or FMG), a caller-owned state Q_dev holding the
 * initial state (its producing work complete when submitted; solved in place) and a stopping test
 * (fine-level FP64 ||r||_inf < tol, at most max_cycles V-cycles, as pmg_solve).  The mesh and Q_dev must
 * stay alive until the request is done.
 * - Admission: requests are admitted first come, first served, when the sum of the footprints (pmg_footprint
 *   with its construction transient and precision-switch hierarchy) of the resident requests and of the next one fits hbm_budget_bytes.
 *   Its solver (all levels) stays resident until the request retires.  A request larger than the whole
 *   budget is refused at submission with PMG_ERR_OOM.
 * - Continuous batching at V-cycle granularity: a worker thread repeatedly runs one V-cycle of every
 *   resident unfinished request, spread over n_streams HIP streams (captured graphs when use_graph = 1),
 *   then every request's residual norm, then waits once; new arrivals join at the next iteration, converged
 *   or failed requests retire and release their memory.
 * - batched = 0: each request runs exactly the launch sequence of pmg_solve on its own solver (mixed-precision
 *   switch included), one stream per request in turn.
 * - batched = 1: resident requests with the same multigrid parameters, node family and maximum order share
 *   one union solver (as pmg_batch_create) on one stream: each iteration is one batched V-cycle for the members
 *   on FP32 coarse levels and one for those on FP64 ones (members not advanced skip their tiles), then one
 *   residual launch with every member's norm.  The union holds the members' states and is rebuilt when its
 *   membership changes (states copied back to the members and in again); a retiring member's state is
 *   copied back before it is reported done.
 * - Either way each request's arithmetic is that of its own solve, so its result is bitwise the result of
 *   solving it alone.
 * The server's functions may be called from any thread.  Destroying the server stops the worker after its
 * current iteration; requests still resident or queued are abandoned (their state is left as it is).
 */
pmg_status pmg_server_create(pmg_ctx ctx, int64_t hbm_budget_bytes, int n_streams, int use_graph, int batched,
                             pmg_server* out);
pmg_status pmg_server_submit(pmg_server sv, pmg_mesh mesh, const int32_t* orders, const pmg_physics* phys,
                             const pmg_mg_params* mg, double* Q_dev, double tol, int max_cycles, uint64_t* ticket);
/* done = 0 while queued or resident.  When done: status (PMG_OK converged, PMG_ERR_NOT_CONVERGED,
 * PMG_ERR_NONPHYSICAL, ...), cycles run, of which fp32_cycles on FP32 coarse levels, the final residual,
 * latency = submission to retirement and queue_s = submission to admission, in seconds (all nullable). */
pmg_status pmg_server_poll(pmg_server sv, uint64_t ticket, int* done, int* status, int* cycles, int* fp32_cycles,
                           double* res_inf, double* latency_s, double* queue_s);
pmg_status pmg_server_stats(pmg_server sv, int* resident, int* queued, int64_t* completed, int64_t* iterations,
                            int64_t* bytes_in_use, int64_t* peak_bytes, int* max_resident);
void pmg_server_destroy(pmg_server sv);

/*
 * Per problem: the step-constant halvings the divergence guard (pmg_mg_params.guard) made since the solver
 * was created (halvings[n_problems], host, out) and, if cfl_host is not NULL, the current constants
 * (cfl_host[2 n_problems]: C^a, C^nu of each problem; the step limits of Sec. 2).
 */
pmg_status pmg_guard_stats(pmg_solver s, int32_t* halvings, double* cfl_host);

/* Mixed precision (pmg_mg_params.precision = 1, Sec. 3.1 cycle with FP32 coarse levels): fp32_cycles (host,
 * one entry per problem) receives the number of cycles of the last pmg_solve / pmg_batch_solve that ran
 * with FP32 coarse levels before the switch to FP64 ones (0 for an FP64 solver). */
pmg_status pmg_solve_stats(pmg_solver s, int32_t* fp32_cycles);

/*
 * Graph mode: with enable = 1, pmg_vcycle, pmg_batch_solve (cycles) and pmg_tau_estimate replay a HIP graph
 * captured once per (state, source, tau map) pointers on the first call, instead of launching every kernel
 * from the host (only for fixed sweep counts).  Results are identical to the eager launches.
 */
pmg_status pmg_set_graph(pmg_solver s, int enable);
/* Tile autotuner: times the operator on every built level for element tiles of about 32, 64, 128, 256 and 512
 * nodes and, for each, the gradient and the divergence kernels launched either as one grid over every tile
 * or once per class of tiles by size (at most 64, 128, 256 nodes, larger) with a block size per class (split
 * bit 0: gradient, bit 1: divergence), and keeps the fastest (cached per context by the level's order-bucket
 * histogram).  Results do not depend on the choice.  pmg_level_tiles returns a level's node target and
 * (split, nullable) its split bits. */
pmg_status pmg_autotune(pmg_solver s, void* stream);
pmg_status pmg_level_tiles(pmg_solver s, int hierarchy, int level, int32_t* tile_target, int32_t* split);
/* Sets one level's element tiles by hand (tile_target 32, 64, 128, 256 or 512 nodes; split 0..3, as above):
 * waits for the device, rebuilds the level's tile arrays and drops the solver's captured graphs.  Results do
 * not change.  PMG_ERR_INVALID_ARG for other values or a level out of range. */
pmg_status pmg_set_tiles(pmg_solver s, int hierarchy, int level, int tile_target, int split);

/*
 * Kernel timing with HIP events (diagnostics).  mask selects kernel kinds (bit k = kind k):
 * 0 face traces, 1 interface state + Roe flux, 2 BR1 gradient, 3 viscous numerical flux, 4 divergence
 * and epilogue, 5 CFL step, 6 transfers.  While enabled, every launch of a selected kind is bracketed by
 * two events on its stream.  pmg_profile_read waits for the recorded events and returns, for one kind,
 * the summed event-to-event time, the number of launches and the summed compulsory bytes of those launches
 * (every input array read once, every output written once, at the launched level's sizes) since the last
 * read of that kind; alg_bytes may be NULL.
 */
pmg_status pmg_profile_enable(pmg_solver s, uint32_t mask);
pmg_status pmg_profile_read(pmg_solver s, int kind, double* total_ms, int64_t* launches, double* alg_bytes);
/*
 * Sample the timing: bracket only every stride-th launch of each selected kind (1, the default: every
 * launch), counting from this call.  A stride coprime with the number of launches of a kind per repeated
 * step samples every launch position of the step over `stride` steps, at 1/stride of the timing overhead.
 * PMG_ERR_INVALID_ARG for stride < 1.
 */
pmg_status pmg_profile_stride(pmg_solver s, int32_t stride);

/*
 * Truncation-error-driven anisotropic p-adaptation (paper, Sec. 3.3.2; eq. AnisTruncError of Sec. 3.2.1; order
 * jumps: eq. poljump2D of Sec. 4.1.2 and Sec. 4.2.1).  Host function: every pointer is a host pointer, no
 * device or solver is needed.
 *
 * Inputs: the mesh connectivity as given to pmg_mesh_create (K elements; nbr_elem[K*6], nbr_face[K*6],
 * orient[K*6], bc[K*6]); the reference orders P[K*3] (each 1..7) on which the map was estimated; the
 * directional truncation-error map tau_map[K][3][nt] of pmg_tau_estimate (entry (e, d, n-1): the element's
 * infinity norm of the truncation error with order n < P_d in direction d; NaN where not estimated).
 *
 * Per element: the inner map (orders n_min <= N_d < P_d, tau(N) = tau_1(N_1) + tau_2(N_2) + tau_3(N_3)) is
 * searched for tau(N) < tau_max; failing that, each direction's values are extrapolated to
 * P_d <= N_d <= n_max[d] by a least-squares fit of log tau_d(n) = a + b n over its measured orders (at least two
 * positive values) and the full map is searched; among the combinations found, the fewest degrees of freedom
 * (N1+1)(N2+1)(N3+1), ties broken by the lexicographically smallest triple; none: N_d = n_max[d].  A direction
 * without estimates (P_d = 1) keeps P_d and adds nothing.  Then, with jump_rule 1 (|N_i+ - N_i-| <= 1) or 2
 * (N_i+ >= floor(2 N_i- / 3)) and/or wall_conforming (elements that both touch a no-slip wall have equal orders
 * across their common face), the lower side is raised, direction by direction through the face orientation,
 * until every constraint holds (the least such orders).  The comparisons are taken in FP64 without fused
 * multiply-adds.  With n_cap > 0 (a multi-stage adaptation's next stage order, Sec. 3.3.4) every selected order
 * above n_cap becomes n_cap before the jump rule is enforced.
 *
 * Output: new_orders[K*3] (caller-owned); max_required (nullable): the largest selected order before the cap.
 * PMG_ERR_INVALID_ARG for NULL pointers, orders outside 1..7, n_max outside n_min..7, tau_max <= 0, an unknown
 * jump rule, 0 < n_cap < n_min.
 */
typedef struct {
  double tau_max;
  int32_t n_max[3];
  int32_t n_min;
  int32_t jump_rule;       /* 0 none, 1 |N+ - N-| <= 1, 2 N+ >= floor(2 N- / 3) */
  int32_t wall_conforming; /* 1: equal orders across faces between elements that both touch a no-slip wall */
  int32_t n_cap;           /* > 0: upper bound on the selected orders (the next stage's order); 0: none */
} pmg_adapt_params;

pmg_status pmg_adapt_orders(int64_t K, const int64_t* nbr_elem, const int32_t* nbr_face, const int32_t* orient,
                            const int32_t* bc, const int32_t* orders, const double* tau_map, int32_t nt,
                            const pmg_adapt_params* prm, int32_t* new_orders, int32_t* max_required);

/*
 * State carried over to new orders after an adaptation (Sec. 3.3.4: the solution continues on the adapted
 * orders).  Per element and direction: exact interpolation where the order rises (the prolongation of
 * eq. FASCorrectSol), the L2 projection of the restriction (eq. FASCoarseSol, Sec. 3.1) where it falls, the
 * identity where it is unchanged;
 * tensor product over the three directions.  Both solvers hold one problem each, on the same mesh (one handle,
 * or two handles created from identical mesh data) and node family.  Q_from_dev [5][nn_from] and Q_to_dev [5][nn_to]: device, FP64, caller-owned, layouts of
 * pmg_state_layout.  Enqueued on 'stream'; returns once it has completed.
 */
pmg_status pmg_remap_state(pmg_solver from, const double* Q_from_dev, pmg_solver to, double* Q_to_dev,
                           void* stream);

/*
 * Multi-stage adaptation inside the FMG cycle (Sec. 3.3.4; each stage as in Sec. 3.3.2).  From free stream on
 * the first stage's orders 'orders' [K*3] (host): for each stage i the problem (no physical source) is solved
 * to max |r| < conv * tau_max (FMG start on the first stage if mg->fmg, V-cycles from the carried-over state
 * afterwards; at most max_cycles), the isolated truncation-error map is estimated by the anisotropic 3V cycle
 * and the orders are selected by pmg_adapt_orders with n_cap = stages[i+1] (none on the last stage); the state
 * is carried over (pmg_remap_state).  The adaptation ends at the last stage or at the first one whose largest
 * required order does not exceed stages[i+1]; the adapted problem is then solved to max |r| < final_tol.
 * Every solver and buffer of the stages is the library's and is freed before the call returns.  The work runs
 * on 'stream'; the call returns once it has completed.
 *
 * mg: multigrid parameters of every stage's solver (level_caps must be NULL: the levels follow the orders,
 * from the solver's largest order down to n_coarse with Delta N = 1).
 * Outputs (caller-owned): Q_out_dev (device) receives the final state as [5][nn] in its first 5*nn doubles,
 * with nn <= capacity_nodes; out_orders[K*3], out_nodes (= nn), reports[n_stages] of which *n_reports are
 * written, final_cycles and final_res (nullable).  PMG_ERR_NOT_CONVERGED when the final solve stops at
 * max_cycles (every output written); a stage that stops there is reported (converged = 0) and the adaptation
 * continues.  PMG_ERR_INVALID_ARG for bad parameters or a capacity below the adapted node count (out_nodes
 * then holds the count needed).
 */
typedef struct {
  const int32_t* stages;   /* host, n_stages increasing orders P_1 < P_2 < ... */
  int32_t n_stages;
  pmg_adapt_params adapt;  /* tau_max, n_max, n_min, jump rule, wall conformity; n_cap is set per stage */
  double conv;             /* each stage is converged to conv * tau_max before its estimate (0.1) */
  double final_tol;        /* tolerance of the final solve on the adapted orders */
  int32_t max_cycles;      /* cap on the V-cycles of each solve */
  int32_t n_coarse;        /* coarsest multigrid order of every stage's solver (the paper's N_coarse; <= 1: 1) */
} pmg_multistage_params;

typedef struct {
  int32_t stage_order;     /* P_i */
  int32_t cycles;          /* V-cycles of the solve before the estimate */
  double res_inf;          /* max |r| when the estimate was taken */
  int32_t converged;       /* 1: res_inf < conv * tau_max */
  int32_t max_required;    /* largest selected order before the stage cap */
  int32_t last;            /* 1: this stage ended the adaptation */
  int32_t pad;
  int64_t nodes_before;    /* nodes (degrees of freedom per variable) before and after the stage's adaptation */
  int64_t nodes_after;
} pmg_stage_report;

pmg_status pmg_adapt_multistage(pmg_ctx ctx, pmg_mesh mesh, const int32_t* orders, const pmg_physics* phys,
                                const pmg_mg_params* mg, const pmg_multistage_params* prm, double* Q_out_dev,
                                int64_t capacity_nodes, int32_t* out_orders, int64_t* out_nodes,
                                pmg_stage_report* reports, int32_t* n_reports, int32_t* final_cycles,
                                double* final_res, void* stream);

/*
 * Force of the fluid on the no-slip walls (tag 1); its components over the dynamic pressure and a reference
 * area are the drag and lift coefficients of Secs. 4.1 and 4.2 (with rho_inf = |v_inf| = 1: C = 2 F / A_ref,
 * drag along v_inf = (1, 0, 0)).  F = the Gauss quadrature over every wall face of (p n - tau . n) dS, n the
 * element's outward unit normal (into the wall), p from the element's trace of Q and tau . n the viscous
 * traction of its BR1 gradient trace, tau = (mu / Re)(grad v + grad v^T - 2/3 div v I): the traces the
 * residual's wall flux uses.  Q_dev [5][nn] (device, FP64) on the solver's finest level; force_host[6] (host):
 * pressure part x, y, z, then viscous part x, y, z (zeros without wall faces).  Single-problem solvers only
 * (PMG_ERR_INVALID_ARG otherwise); returns once the stream has completed.
 */
pmg_status pmg_wall_force(pmg_solver s, const double* Q_dev, double* force_host, void* stream);

/*
 * pmg_wall_force for callers that cannot allocate device memory (code under stream or graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same force, bit for bit, computed without any
 * hipMalloc / hipFree or allocating library call.  Its block partials and their sum live in a static device
 * array of the library (one per GPU, 384 KiB, held until the process ends); the caller passes the solver,
 * Q_dev and force_host exactly as for pmg_wall_force.  At most 8192 x 256 = 2,097,152 wall nodes on the
 * finest level (PMG_ERR_INVALID_ARG beyond).  Every call on one GPU shares that array: calls that overlap on
 * one GPU (other threads, other streams) race and must be serialised by the caller.  Returns once the stream
 * has completed.
 */
pmg_status pmg_wall_force_noalloc(pmg_solver s, const double* Q_dev, double* force_host, void* stream);

/*
 * Drag and lift coefficients of a wall force (Secs. 4.1 and 4.2): with the non-dimensional far field
 * rho_inf = 1, |v_inf| = 1 the dynamic pressure is 1/2, so C = 2 F / A_ref; drag along v_inf = (1, 0, 0),
 * lift along y.  force_host[6] (host): the output of pmg_wall_force (pressure part x, y, z, then viscous
 * part x, y, z; each coefficient takes the sum of both parts).  area_ref > 0 (for the unit sphere pi).
 * coef_host[4] (host, out): C_d, C_l, then the pressure part of C_d and its viscous part.  Host arithmetic
 * only; PMG_ERR_INVALID_ARG for NULL pointers or a non-positive area.
 */
pmg_status pmg_force_coefficients(const double* force_host, double area_ref, double* coef_host);

#ifdef __cplusplus
}
#endif

#endif /* PMG_H */
