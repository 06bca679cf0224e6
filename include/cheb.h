/*
 * cheb.h - C ABI of the MI355X (gfx950) Chebyshev-collocation diffusion solver.
 *
 * Problem (Section 2, 3-D extension; Section 3.3 flux form):
 *     div(K(x) grad u) = f   in the box  prod_a [lo_a, hi_a],
 *     per face either u = g (Dirichlet) or du/dn + sigma u = g (Neumann,
 *     outward normal; sigma = 0 unless a Robin coefficient is given),
 * discretised by collocation at the tensor Chebyshev-Gauss-Lobatto (CGL) nodes:
 * the PDE holds at interior nodes, one boundary-condition row holds at every
 * boundary node (Section 2.3.1).  The discrete operator is applied matrix-free
 * (Algorithm 3): per axis a DCT-I of every pencil (the FFT of its even
 * extension), the derivative-coefficient recurrence, the back-transform, the
 * pointwise flux K * du/dx_a, and the same three steps again for the
 * divergence.  Boundary conditions are eliminated (Section 2.3.1) and the
 * reduced system is solved by LGMRES (Algorithm 2); hierarchical refinement
 * prolongs a coarse solution by zero-padding its Chebyshev coefficients
 * (Section 2.3.3, Algorithm 4).
 *
 * Conventions for every call:
 *   - Field arrays are device pointers to C-contiguous [i][j][k] arrays of
 *     n[0] x n[1] x n[2] values (i along x, slowest; k along z, fastest), in the
 *     plan's precision (double for CHEB_F64 and CHEB_MIXED, float for CHEB_F32).
 *   - Node coordinates along axis a are ascending:
 *         x_j = (lo+hi)/2 - (hi-lo)/2 * cos(pi j / N_a),  N_a = n[a] - 1.
 *   - Faces are numbered 0..5 = x_lo, x_hi, y_lo, y_hi, z_lo, z_hi.  Face data
 *     (g_faces) are packed face after face; the array of face f on axis a has
 *     shape (n[b], n[c]) with b < c the two other axes.
 *   - Neumann data are the outward normal derivative du/dn (not the flux),
 *     plus sigma u on faces with a Robin coefficient (cheb_grid.robin).
 *   - Edge and corner nodes (on several faces) carry exactly one equation: the
 *     Dirichlet face of lowest axis if one contains the node, otherwise the
 *     Neumann face of lowest axis.  (The paper is silent on this; the interior
 *     solution does not depend on the choice.)
 *   - All calls are asynchronous on the plan's HIP stream unless stated; the
 *     caller keeps every buffer alive until the stream has finished with it.
 *   - The caller owns all field buffers and the workspace.  The plan owns its
 *     device constants and tables (allocated at creation, see
 *     cheb_plan_create), the preconditioner's factors (allocated when a call
 *     first needs them) and per-node Robin coefficients (when set).
 *   - Errors are return codes, never exceptions.  0 = success; negative = hard
 *     error, outputs untouched; positive = soft status with valid outputs.
 *     cheb_last_error() gives a thread-local message for the last failure.
 *   - A plan is not re-entrant: use it from one host thread at a time.
 */
#ifndef CHEB_H_
#define CHEB_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CHEB_OK 0
#define CHEB_NOT_CONVERGED 1     /* iterative solve stopped at maxiter; best iterate returned */
#define CHEB_STAGNATED 2         /* refinement stopped contracting; best iterate returned */
#define CHEB_ERR_INVALID_ARG (-1)
#define CHEB_ERR_SINGULAR_BC (-2) /* all six faces Neumann: solution defined up to a constant */
#define CHEB_ERR_BAD_INPUT (-3)   /* NaN/Inf or non-positive conductivity */
#define CHEB_ERR_DEVICE (-4)      /* HIP runtime error */
#define CHEB_ERR_WORKSPACE (-5)   /* workspace missing or too small */
#define CHEB_ERR_UNSUPPORTED (-6)

/* precision */
#define CHEB_F64 0   /* everything in FP64 */
#define CHEB_F32 1   /* everything in FP32 (fields are float) */
#define CHEB_MIXED 2 /* FP64 fields and outer refinement, FP32 transforms and inner Krylov */

/* face types */
#define CHEB_DIRICHLET 0
#define CHEB_NEUMANN 1

/* cheb_apply flags */
#define CHEB_APPLY_FULL 0u      /* y = A u: interior rows sum_a D_a(K D_a u), boundary rows B u */
#define CHEB_APPLY_REDUCED 1u   /* y = (A_kk + A_kr G) u_k on interior nodes, 0 on boundary nodes */
#define CHEB_APPLY_TRANSPOSE 2u /* with REDUCED: y = (A_kk + A_kr G)^T u_k */

/* operator route of the reduced apply and its transpose (cheb_plan_set_route) */
#define CHEB_ROUTE_AUTO 0   /* matrix-core route on axes with N in {16,32,48,64,96,128}, FFT route elsewhere */
#define CHEB_ROUTE_FFT 1    /* DCT-I through the FFT of the even extension on every axis */
#define CHEB_ROUTE_MATRIX 2 /* matrix-core route wherever N allows it (as AUTO) */

typedef struct cheb_grid {
  int32_t n[3];  /* nodes per axis, 3 <= n <= 513 */
  double lo[3];  /* box lower corner */
  double hi[3];  /* box upper corner, hi > lo */
  int32_t bc[6]; /* CHEB_DIRICHLET or CHEB_NEUMANN per face */
  /* Robin coefficient sigma per face (Section 2.3.1, general linear boundary
   * operator): a Neumann face's row becomes du/dn + sigma u = g (outward
   * normal derivative).  A row a u + b du/dn = g with b != 0 is sigma = a / b
   * with data g / b.  0 gives the plain Neumann row; must be 0 on Dirichlet
   * faces.  A plan rejects (CHEB_ERR_INVALID_ARG) coefficients that make an
   * end-value elimination block singular, and accepts six Neumann faces only
   * when some sigma is nonzero.  Batches take sigma = 0 only. */
  double robin[6];
} cheb_grid;

typedef struct cheb_solve_opts {
  double rtol;           /* stop when ||r|| <= max(rtol * ||b||, atol) (reduced system) */
  double atol;
  int32_t maxiter;       /* maximum operator applications (0 = 10000) */
  int32_t inner_m;       /* LGMRES Krylov dimension per restart cycle (0 = 30) */
  int32_t outer_k;       /* LGMRES augmentation vectors (0 = 3, negative = none, max 6) */
  double ir_inner_rtol;  /* MIXED: smallest relative tolerance of an FP32 inner solve (0 = 1e-3);
                            each inner solve targets max(ir_inner_rtol, 0.3 x the reduction the
                            outer residual still needs) and also stops when a restart cycle gains
                            less than 10% (the FP32 operator's floor) */
  int32_t ir_max_outer;  /* MIXED: maximum FP64 refinement steps (0 = 50) */
  int32_t flags;         /* bit 0: use the initial guess in u_inout (else start from 0);
                            bit 1: right-precondition LGMRES by fast diagonalisation of the
                            constant-coefficient operator (mean K) -- an extension, off in the
                            paper's plain method */
  double* history;       /* optional host array receiving the relative residual per restart / IR step */
  int32_t history_len;
  int32_t reserved[3];
} cheb_solve_opts;

typedef struct cheb_solve_info {
  int32_t status;        /* CHEB_OK / CHEB_NOT_CONVERGED / CHEB_STAGNATED */
  int32_t matvecs;       /* operator applications, FP64 + FP32 */
  int32_t matvecs_f32;   /* of which in FP32 */
  int32_t restarts;      /* LGMRES restart cycles */
  int32_t ir_steps;      /* refinement steps (MIXED) */
  int32_t history_used;
  double relres_final;   /* ||b - A x|| / ||b||, recomputed in FP64 at the end */
  double seconds;        /* host wall time of the call */
} cheb_solve_info;

typedef struct cheb_plan cheb_plan;

/* Create a plan for one grid.  Validates n (3..513), lo < hi, bc values and
 * Robin coefficients, and rejects all-Neumann problems without a Robin
 * coefficient with CHEB_ERR_SINGULAR_BC.  `stream` is a
 * hipStream_t (NULL = default stream).  Allocates a few KB of device constants
 * (boundary rows of the differentiation matrix), the matrix-core route's
 * fragment tables when an axis has N <= 128, and, when all three axes can take
 * that route and axes x and y have the same N, one field-sized buffer
 * (n0*n1*n2 values, 4 bytes each for CHEB_F32 plans, 8 otherwise) that holds
 * the second partial sum of an apply whose x and y passes share one launch
 * (if that allocation fails, applies take three launches instead).
 * Nothing is allocated after creation except where a call says so. */
int cheb_plan_create(const cheb_grid* grid, int32_t precision, void* stream, cheb_plan** out);

/* Bytes of device workspace needed by cheb_solve / cheb_adjoint / cheb_picard
 * with these options (opts may be NULL for defaults). */
int cheb_plan_workspace_bytes(const cheb_plan* plan, const cheb_solve_opts* opts, size_t* bytes);

/* Give the plan a caller-owned device workspace (256-byte aligned).  The plan
 * never allocates device memory on the solve path. */
int cheb_plan_set_workspace(cheb_plan* plan, void* dev_ptr, size_t bytes);

/* Change the stream subsequent calls enqueue on. */
int cheb_plan_set_stream(cheb_plan* plan, void* stream);

/* Robin coefficients that vary along a face (Section 2.3.1's general linear
 * row with node-dependent coefficients; the flux condition k(T) dT/dn = h of
 * Section 3.4 with k = K0 / (1 + alpha T) is the row
 * dT/dn - (alpha h / K0) T = h / K0, i.e. sigma = -alpha h / K0 at each node and
 * data h / K0).  sigma_faces: FP64, the packed face layout of g_faces (faces
 * x_lo .. z_hi, each n_b x n_c in the order of the two other axes); entry i of
 * face f is added to grid.robin[f] at that node.  Entries on Dirichlet faces
 * must be 0.  The library copies the array (device or host memory; the caller
 * keeps ownership) into plan-owned device memory (FP64 and FP32 copies, one
 * packed-face array each, with each pencil's end-block inverse) and
 * synchronises the plan's stream.  Every operator, lift, solve, adjoint and
 * Newton call of the plan then uses the node's own row, on either derivative
 * route; the preconditioner, rebuilt on its next use, uses each face's mean
 * coefficient.  NULL removes the per-node part.
 * Returns CHEB_ERR_INVALID_ARG for a null plan, a non-finite entry, a nonzero
 * entry on a Dirichlet face, or coefficients that make some pencil's
 * end-value elimination block singular (the plan is then unchanged), and
 * CHEB_ERR_DEVICE on a HIP failure (the plan then has no per-node part). */
int cheb_plan_set_robin_nodes(cheb_plan* plan, const double* sigma_faces);

/* Choose how the reduced operator and its transpose evaluate the per-axis
 * derivatives (Section 2.2 defines the derivative; both routes compute it):
 *   CHEB_ROUTE_FFT    -- the DCT-I of each pencil through the FFT of its even
 *                        extension, coefficient recurrence, back-transform
 *                        (Algorithm 1 / Section 2.2), any N;
 *   CHEB_ROUTE_MATRIX -- for N in {16, 32, 48, 64, 96, 128}: the derivative as a
 *                        dense contraction with the collocation matrix on the
 *                        matrix cores (even-odd split), other axes use the FFT;
 *   CHEB_ROUTE_AUTO   -- the default; currently identical to CHEB_ROUTE_MATRIX.
 * The two routes agree to rounding.  FULL applies, derivatives and the adjoint
 * gradient always use the FFT route; the Newton Jacobian's derivative term
 * follows the plan's route like the reduced operator.  Returns
 * CHEB_ERR_INVALID_ARG for an unknown route. */
int cheb_plan_set_route(cheb_plan* plan, int32_t route);

/* Autotuner of the reduced operator: times the FFT route and the two tile
 * shapes of the matrix-core route (12 reduced applies each, HIP events on the
 * plan's stream) on the caller's fields and keeps the fastest for
 * CHEB_ROUTE_AUTO in that precision.  field_precision selects which passes are
 * tuned and the type of K, u, y (device, n0*n1*n2 each, y distinct from u and
 * K; y is overwritten): CHEB_F64 (F64 or MIXED plans) or CHEB_F32 (F32 or MIXED
 * plans).  report (host, may be NULL when report_len is 0) receives up to 4
 * values: microseconds per apply for [FFT route, matrix tile shape 0, matrix
 * tile shape 1] (-1 where not applicable) and the index chosen.  Synchronises
 * the plan's stream.  Without this call AUTO uses tile shape 1 (the faster one
 * at every N measured, both precisions). */
int cheb_plan_autotune(cheb_plan* plan, int32_t field_precision, const void* K, const void* u, void* y,
                       double* report, int32_t report_len);

/* Tile shape of the matrix-core route for one precision, on every axis:
 * 0 = 8-wave workgroups with the derivative's fragment table in LDS, 1 = 4-wave
 * workgroups with each wave's fragments in registers (the two shapes the
 * autotuner times).  field_precision: CHEB_F64 or CHEB_F32 (the passes that run
 * in that type).  Returns CHEB_ERR_INVALID_ARG for another precision or shape;
 * affects only the matrix-core route. */
int cheb_plan_set_tile_shape(cheb_plan* plan, int32_t field_precision, int32_t shape);

int cheb_plan_destroy(cheb_plan* plan);

/* Operator application (Algorithm 3 with the rows of Section 2.3.1).
 *   K : coefficient at every node (the solves require K > 0; the apply is
 *   linear in K and evaluates any finite values), u : input field, y : output field
 *   (y must not alias u or K).  flags: CHEB_APPLY_FULL, CHEB_APPLY_REDUCED or
 *   CHEB_APPLY_REDUCED|CHEB_APPLY_TRANSPOSE.  In REDUCED modes boundary entries
 *   of u are ignored and boundary entries of y are set to 0.  Asynchronous.
 *   Needs no workspace. */
int cheb_apply(cheb_plan* plan, const void* K, const void* u, void* y, uint32_t flags);

/* Solve div(K grad u) = f with face data g (Algorithm 2): build the reduced
 * right-hand side f_k - A_kr H g, run LGMRES on the reduced operator (MIXED:
 * FP32 LGMRES inside FP64 iterative refinement), reconstruct the boundary
 * values x_r = G x_k + H g.  u_inout: on entry the initial guess if opts->flags
 * bit 0 is set (its boundary values are ignored), on exit the full nodal
 * solution.  g_faces: device array of packed face data (double; float for
 * CHEB_F32).  f: source at every node (boundary entries ignored).  Requires the
 * workspace.  Synchronises the plan's stream before returning. */
int cheb_solve(cheb_plan* plan, const void* K, const void* f, const void* g_faces, void* u_inout,
               const cheb_solve_opts* opts, cheb_solve_info* info);

/* Modal prolongation (Section 2.3.3): u_f = the coarse interpolant evaluated at
 * the fine CGL nodes, i.e. DCT-I of u_c along each axis, zero-padding of the
 * coefficients to the fine size, back-transform.  Fine sizes must be >= coarse
 * sizes and both plans must describe the same box and precision.  If
 * u_f_solved is not NULL, also returns e_ref = ||u_f_solved - u_f|| / ||u_f_solved||
 * (Section 2.3.3 refinement indicator) in *e_ref (synchronises the stream).
 * Uses the fine plan's stream and workspace. */
int cheb_prolong(const cheb_plan* coarse, const cheb_plan* fine, const void* u_c, void* u_f,
                 const void* u_f_solved, double* e_ref);

/* Allocation-free prolongation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same result as cheb_prolong(coarse, fine, u_c, u_f,
 * NULL, NULL), bit for bit, with the two intermediate fields of its three axis
 * passes held in the library's file-scope device scratch array (128 MiB per
 * GPU, allocated with the library's code object and held until the process
 * ends) instead of the fine plan's workspace.  Needs no workspace, calls no
 * allocating routine and does not synchronise: asynchronous on the fine plan's
 * stream.  The intermediates take round_up(nc0*nc1*nf2*e, 256) +
 * round_up(nc0*nf1*nf2*e, 256) bytes (e = 8 for FP64, 4 for FP32; nc = coarse,
 * nf = fine sizes); larger requests fail with CHEB_ERR_WORKSPACE before any
 * work is enqueued (FP64 129^3 -> 257^3 fits).  Both plans must live on the
 * same device.  Every call on a GPU shares that GPU's scratch array: calls
 * that overlap in time on one GPU (other streams, other host threads) race on
 * it and must be serialised by the caller.  Other errors as cheb_prolong. */
int cheb_prolong_noalloc(const cheb_plan* coarse, const cheb_plan* fine, const void* u_c, void* u_f);

/* Hierarchical refinement with its stopping rule (Section 2.3.3, Algorithm 4):
 * levels l = 0 .. nlev-1 on plans[l] (same box, face types and precision;
 * sizes non-decreasing; the last level the largest), each with its own data
 * K[l], f[l], g_faces[l] (device fields of that level, as in cheb_solve) and
 * output u[l].  Level 0 is solved by cheb_solve with opts (bit 0 of
 * opts->flags: u[0] holds the initial guess).  Every later level starts from
 * the modal prolongation of the previous level's result into u[l].  While the
 * refinement has not converged the level is solved from that start and
 * e_ref[l] = ||U_l - P U_{l-1}||_2 / ||U_l||_2 (the refinement indicator) is
 * recorded; once some e_ref[l] <= tol the refinement has converged and every
 * finer level is the prolongation alone, with no solve (solved[l] = 0,
 * e_ref[l] = NaN).  tmp: device scratch field of the last level's size.  Each
 * plan needs the workspace of cheb_solve with these opts.  e_ref, solved (nlev
 * entries each) and infos (per level; zeroed for levels not solved) are host
 * arrays and may be NULL.  Returns the worst soft status of the solves, or a
 * negative error.  Synchronises. */
int cheb_refine(cheb_plan* const* plans, int32_t nlev, const void* const* K, const void* const* f,
                const void* const* g_faces, void* const* u, void* tmp, const cheb_solve_opts* opts, double tol,
                double* e_ref, int32_t* solved, cheb_solve_info* infos);

/* Adjoint sensitivity: given the converged state u of cheb_solve for K and
 * dL/du at every node, solves A^T lambda = dL/du through the reduced transpose
 * (interior rows: (A_kk + A_kr G)^T lambda_k = r_k + G^T r_r) and writes
 *   dLdlogK_j = -K_j sum_a (D_a u)_j (D_a^T lambda~)_j,
 * lambda~ = lambda on interior rows and 0 on boundary rows.  lambda receives
 * lambda~.  FP64 or MIXED plans only.  Requires the workspace; synchronises. */
int cheb_adjoint(cheb_plan* plan, const void* K, const void* u, const void* dLdu, void* lambda,
                 void* dLdlogK, const cheb_solve_opts* opts, cheb_solve_info* info);

/* Lagged-coefficient (Picard) iteration for K(x,u) = K0(x) (1 + u^2/2)
 * (Section 2.3, Picard form): K_m = K0 (1 + u_m^2/2), solve, until
 * ||u_{m+1} - u_m|| / ||u_{m+1}|| <= picard_tol or max_steps.  u_inout as in
 * cheb_solve (bit 0 of opts->flags selects the warm start).  Kwork: caller
 * device array of one field for the current coefficient.  *steps receives the
 * number of Picard steps.  Synchronises. */
int cheb_picard(cheb_plan* plan, const void* K0, const void* f, const void* g_faces, void* u_inout,
                void* Kwork, double picard_tol, int32_t max_steps, const cheb_solve_opts* opts,
                cheb_solve_info* info, int32_t* steps);

/* Newton iteration for the conductivity law k(x, T) = K0(x) / (1 + alpha T)
 * (Section 3.4, reciprocal law, with alpha = 0.5 and K0 = 1 in the paper's
 * example; Section 2.3, Newton form).  All arrays are FP64 fields of the plan's
 * grid except g_faces (packed face data as in cheb_solve).  FP64 or MIXED plans
 * only (CHEB_ERR_UNSUPPORTED otherwise); the linear solves run in FP64.
 *
 * work: caller device buffer of cheb_newton_work_bytes() bytes, 256-byte
 * aligned, holding k(T), c_a = k'(T) D_a T (a = 0, 1, 2) and one scratch
 * field; its contents are not kept between calls.  Every call fails with
 * CHEB_ERR_BAD_INPUT when k(T) is not finite and positive at some node
 * (1 + alpha T <= 0, or K0 <= 0); cheb_newton checks this also at the cold
 * start lift(0, g), which sets its residual scale, when a warm start is given. */
int cheb_newton_work_bytes(const cheb_plan* plan, size_t* bytes);

/* r = R(T) = sum_a D_a (k(T) D_a T) - f on interior nodes, 0 on boundary nodes
 * (the Section 3.4 residual, written for div(k grad T) = f).  T is a full
 * nodal state; its boundary rows are taken as satisfied.  Synchronises. */
int cheb_newton_residual(cheb_plan* plan, const void* K0, double alpha, const void* T, const void* f, void* r,
                         void* work);

/* y = J(T) v, the reduced Jacobian of cheb_newton_residual at T applied to the
 * interior values of v (boundary values of v are ignored): with V the
 * homogeneous lift of v (Section 2.3.1),
 *   y = sum_a D_a (k(T) D_a V + k'(T) V D_a T)   on interior nodes, 0 elsewhere
 * (the Jacobian action of Section 3.4).  Synchronises. */
int cheb_newton_jacobian(cheb_plan* plan, const void* K0, double alpha, const void* T, const void* v, void* y,
                         void* work);

/* Newton-LGMRES solve of div(k(T) grad T) = f with the boundary rows of
 * cheb_solve (Dirichlet values; Neumann outward dT/dn plus the plan's Robin
 * coefficients, per face and per node: the flux condition k(T) dT/dn = h of
 * Section 3.4 is such a row, see cheb_plan_set_robin_nodes).  The state is
 * T_m = lift(x_m, g).  The scale is r_ref = ||R(lift(0, g))||, the residual of
 * the cold start, also when a warm start is given.  The iteration stops once
 * ||R(T_m)|| <= newton_tol r_ref (CHEB_OK) or after max_steps updates
 * (CHEB_NOT_CONVERGED); otherwise it solves J(T_m) dx = -R(T_m) by LGMRES to
 * max(opts->rtol ||R(T_m)||, opts->atol, newton_tol r_ref / 10) (an inexact
 * Newton step; fast-diagonalisation preconditioner at the mean of k(T_m) when
 * bit 1 of opts->flags is set) and sets x_{m+1} = x_m + dx.  u_inout: initial
 * state when bit 0 of opts->flags is set (its interior values are used), else
 * T_0 = lift(0, g); receives the final full state.  opts->history, if given,
 * receives ||R(T_m)|| / r_ref for m = 0, 1, ...  *steps receives the number of
 * updates; mv_per_step (host, max_steps entries, may be NULL) the LGMRES
 * matrix-vector products of each.  Needs the plan workspace of
 * cheb_plan_workspace_bytes(opts).  Synchronises. */
int cheb_newton(cheb_plan* plan, const void* K0, double alpha, const void* f, const void* g_faces, void* u_inout,
                void* work, double newton_tol, int32_t max_steps, const cheb_solve_opts* opts,
                cheb_solve_info* info, int32_t* steps, int32_t* mv_per_step);

/* Derivative along one axis, D_a u at every node (first half of an axis pass).
 * Asynchronous. */
int cheb_derivative(cheb_plan* plan, const void* u, void* du, int32_t axis);

/* Clenshaw-Curtis volume averages <K du/dx_b>, b = 0,1,2, written to host
 * out[3] (Section 3.3 effective conductivity: K_num = <K du/dx_a> / G).
 * Uses 4 fields of workspace.  Synchronises. */
int cheb_flux_average(cheb_plan* plan, const void* K, const void* u, double out[3]);

/* Apparent conductivity of one load case (Section 3.3): with u the solution
 * of a load case along `axis` whose faces impose a jump `jump` of u across the
 * box (mean gradient G = jump / (hi[axis] - lo[axis])), out[b] = <K du/dx_b>_CC
 * / G for b = 0, 1, 2 (host out[3]): column `axis` of the apparent
 * conductivity tensor.  Same workspace and synchronisation as
 * cheb_flux_average; CHEB_ERR_INVALID_ARG for an axis outside 0..2 or a zero
 * or non-finite jump. */
int cheb_apparent_conductivity(cheb_plan* plan, const void* K, const void* u, int32_t axis, double jump,
                               double out[3]);

/* Fast-diagonalisation preconditioner, the one the preconditioned solves use
 * (an addition to the paper's plain LGMRES).  With constant K = kc the reduced
 * operator of Section 2.3.1 is kc (A_x (+) A_y (+) A_z), a Kronecker sum of the
 * 1-D reduced second-derivative operators (boundary rows eliminated per axis);
 * this call applies its exact inverse,
 *     out = (V_x V_y V_z) diag(1 / (kc (lx_i + ly_j + lz_k))) (V_x V_y V_z)^{-1} in,
 * A_a = V_a diag(l_a) V_a^{-1}, as six axis contractions on the matrix cores
 * (even-odd split on axes with the same face type at both ends), or its
 * transpose with CHEB_APPLY_TRANSPOSE in flags (the adjoint solves use it).
 *   field_precision: CHEB_F64 or CHEB_F32, the type of in and out (any plan
 *     precision: the plan keeps the factors in both);
 *   in, out: device fields of n0 n1 n2 values; boundary values of in are
 *     ignored, those of out are set to 0; out may equal in;
 *   kc: positive and finite.
 * Needs two interior blocks of workspace (2 (n0-2)(n1-2)(n2-2) values of
 * field_precision, each rounded up to 256 bytes; a preconditioned solve's
 * workspace always holds them).  The first call on a plan computes the 1-D
 * eigen-decompositions on the host and synchronises; later calls are
 * asynchronous.  Errors: CHEB_ERR_INVALID_ARG (null pointer, precision, flags,
 * kc), CHEB_ERR_WORKSPACE, CHEB_ERR_UNSUPPORTED (an eigen-decomposition
 * failed). */
int cheb_precond_apply(cheb_plan* plan, int32_t field_precision, double kc, const void* in, void* out,
                       uint32_t flags);

const char* cheb_status_string(int status);
const char* cheb_last_error(void);

/* ---- batched solves (many independent systems in lockstep) --------------
 * For studies that solve many small problems at once, e.g. the homogenisation
 * of a set of microstructures under three load cases each (Section 3.3 defines
 * the effective conductivity from such solves).  Every Krylov step of all
 * systems is a few launches: one matrix-core operator pass per group of
 * identical grids and axis, over a tile queue spanning the group, one
 * fast-diagonalisation contraction per group of identical grids and face types,
 * and segmented vector kernels.  Systems that converge drop out of the queues.
 */
typedef struct cheb_batch cheb_batch;

/* nprob systems, system s on grids[s] (any sizes and face types; systems with
 * the same n, lo, hi share operator launches).  precision: CHEB_F64 or
 * CHEB_MIXED (FP64 fields at the ABI).  Allocates the per-system plans and a few
 * KB of device tables. */
int cheb_batch_create(const cheb_grid* grids, int32_t nprob, int32_t precision, void* stream, cheb_batch** out);

/* Device workspace of cheb_batch_solve (all systems' fields packed back to back). */
int cheb_batch_workspace_bytes(const cheb_batch* batch, const cheb_solve_opts* opts, size_t* bytes);
int cheb_batch_set_workspace(cheb_batch* batch, void* dev_ptr, size_t bytes);
int cheb_batch_set_stream(cheb_batch* batch, void* stream);

/* Solve all systems.  K, f, g_faces, u_inout: host arrays of nprob device
 * pointers (FP64, each system's own layout as in cheb_solve; systems may share
 * a K pointer, e.g. the load cases of one microstructure).  opts apply to every
 * system (rtol relative to each system's own right-hand side; flags bit 0 warm
 * start, bit 1 preconditioner).  infos (host, nprob entries, may be NULL)
 * receive the per-system results.  Returns the worst per-system status, or a
 * negative error (outputs untouched on CHEB_ERR_BAD_INPUT).  Synchronises the
 * stream. */
int cheb_batch_solve(cheb_batch* batch, const void* const* K, const void* const* f, const void* const* g_faces,
                     void* const* u_inout, const cheb_solve_opts* opts, cheb_solve_info* infos);

/* Tile shapes the batch's autotuner chose.  On its first solve in each field
 * precision a batch times the three-pass matrix-core apply of every size group
 * over all the group's members with both tile shapes (see
 * cheb_plan_set_tile_shape; 4 applies each, HIP events on the batch's stream)
 * and keeps the faster one for that group.  out (host) receives 4 values per
 * matrix-core group, up to len entries: nodes per axis, chosen shape (-1 if
 * not tuned yet), nanoseconds per apply with shape 0 and with shape 1.
 * field_precision: CHEB_F64 (FP64 passes) or CHEB_F32 (the FP32 passes of
 * MIXED batches).  Returns the number of groups written, or a negative error. */
int cheb_batch_tile_shapes(const cheb_batch* batch, int32_t field_precision, int32_t* out, int32_t len);

int cheb_batch_destroy(cheb_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* CHEB_H_ */
