/*
 * hdg.h -- C ABI of the entropy-variable hybridized DG hot path on MI355X (gfx950).
 *
 * Method: Fernandez, Nguyen & Peraire, "Entropy-stable hybridized discontinuous
 * Galerkin methods for the compressible Euler and Navier-Stokes equations".
 * For every element the library evaluates, at volume and face quadrature points,
 * the residual of the hybridized DG weak forms in entropy variables (section on
 * the Euler discretization: element and trace equations; section on the
 * Navier-Stokes discretization: gradient, element and trace equations) and its
 * exact Newton Jacobian, factors the dense local block and forms the Schur
 * complement onto the trace unknowns (the local elimination noted after both
 * weak forms: only v_hat is globally coupled).  Numerical flux: the inviscid
 * trace flux f_hat = 1/2 (F(v_hat) + F(v)).n + 1/2 sigma (v - v_hat) with the
 * symmetric Lax-Friedrichs matrix sigma = lambda_max(v_hat) A0(v_hat), and the
 * viscous trace flux g_hat = G(v_hat, q).n -- the choices of the paper's
 * numerical examples.
 *
 * Conventions (all arrays are plain contiguous memory):
 *   m = dim + 2 components.  Element e has Np nodes, nf faces, Nfp nodes per face.
 *   Local unknowns x_K (length n):  v at [c*Np + a], then q at
 *     [m*Np + (c*dim + j)*Np + a]          (n = m*Np Euler, m*Np*(1+dim) NS)
 *   Element trace unknowns (length k = nf*m*Nfp): [f*(m*Nfp) + c*Nfp + b].
 *   Global fields are structure-of-arrays:
 *     v     [m][E*Np]       entropy variables at element nodes, node e*Np + a
 *     q     [m*dim][E*Np]   gradient unknowns, row c*dim + j
 *     vhat  [m][n_trace]    trace unknowns at global trace nodes
 *   Per-element matrices are column-major and element-major:
 *     S [E][k][k], g [E][k], Y [E][k][n] (n x k column-major), z [E][n].
 *   Element node order: tensor Gauss-Lobatto lattice, x fastest (quad/hex);
 *   equispaced barycentric lattice, k outer / j / i inner (tri/tet).  Local face
 *   f: xi=-1,+1, eta=-1,+1, zeta=-1,+1 (quad/hex); opposite vertex f (tri/tet).
 *   Face node b is the b-th element node (ascending) on that face.
 *   Quadrature: Gauss-Legendre with p+2 points per direction (collapsed on
 *   simplices).  Gas constant R = 1, c_v = 1/(gamma-1), s0 = 0, beta = 0.
 *
 * Memory: every device buffer is owned by the caller.  The plan keeps host
 * copies of the mesh tables; after hdg_plan_bind_workspace it also uses the
 * caller's workspace (tables at its start, per-element scratch after).
 * Calls are asynchronous on the given stream; errors detected on the host are
 * returned immediately, errors detected on the device land in the per-element
 * status array (HDG_ENONPHYS, HDG_ESINGULAR).
 * Thread safety: one plan must not be used by overlapping calls (the bound
 * workspace is shared scratch).
 */
#ifndef HDG_H_
#define HDG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HDG_OK = 0,
  HDG_EINVAL = -1,        /* bad argument: null pointer, size mismatch, det J <= 0 */
  HDG_EUNSUPPORTED = -2,  /* element type / order / dimension not built */
  HDG_ENONPHYS = -3,      /* v_m >= 0 or non-finite state at a quadrature point */
  HDG_ESINGULAR = -4,     /* zero pivot in the local LU */
  HDG_EHIP = -5,          /* HIP runtime error (see hdg_last_error) */
  HDG_ENOMEM = -6         /* workspace smaller than hdg_plan_workspace_bytes */
};

enum { HDG_TRI = 0, HDG_QUAD = 1, HDG_TET = 2, HDG_HEX = 3 };
enum { HDG_FP64 = 0, HDG_FP32 = 1, HDG_BF16 = 2 };

typedef struct hdg_plan hdg_plan;

/* Physical parameters (Euler / Navier-Stokes sections; numerical examples for
 * beta = 0).  alpha is the mass coefficient of a backward-Euler / DIRK stage:
 * the element equation gets alpha (u(v_h) - u*, w); alpha = 0 is steady. */
typedef struct {
  int viscous;     /* 0 Euler, 1 Navier-Stokes */
  double gamma;
  double mu;       /* constant dynamic viscosity */
  double Pr;
  double alpha;
} hdg_phys;

/* Mesh description, host memory, read once by hdg_plan_create. */
typedef struct {
  int elem_type;           /* HDG_TRI .. HDG_HEX */
  int order;               /* polynomial degree p (1..4) */
  int n_elem;
  const double *elem_xyz;  /* [n_elem][n_vertices][dim]: straight-sided or multilinear */
  const int32_t *face_bc;  /* [n_elem][nf]: 0 flux face, 1 Dirichlet-trace face; NULL: all 0.
                              The trace rows of a Dirichlet-trace face are <v_hat - v_bc, mu>
                              (the boundary operator of the trace equation, left open by the
                              paper); a trace node that a Dirichlet face shares with flux faces
                              (a continuous, EDG trace) keeps only those rows: the flux faces'
                              rows at that node are dropped, so the node takes the boundary value */
  const int32_t *trace_map;/* [n_elem][nf][Nfp] global trace node; encodes HDG/EDG/IEDG */
  int n_trace;             /* number of global trace nodes */
} hdg_mesh;

enum { HDG_FLAG_SPLIT_DENSE = 1, HDG_FLAG_NARROW_BLOCK = 2, HDG_FLAG_ELIMINATE_Q = 4, HDG_FLAG_GHAT_INTERIOR = 8,
       HDG_FLAG_SIGMA_S = 16, HDG_FLAG_SIGMA_MV = 32, HDG_FLAG_GHAT_PROJ = 64 };

typedef struct {
  int chunk_elems;         /* elements per internal wave (0: all) */
  int precision;           /* HDG_FP64; the FP32 path has its own entry points below */
  int flags;               /* HDG_FLAG_SPLIT_DENSE: the reference kernel variants (VALU
                              block contraction; separate LU / solve / Schur kernels)
                              instead of the matrix-core contraction and the fused
                              left-looking condensation used by default when their LDS
                              working sets fit.
                              HDG_FLAG_ELIMINATE_Q (Navier-Stokes): hdg_assemble_condense
                              first eliminates the gradient unknowns q element by element
                              (their block is the mass matrix times the identity), then
                              condenses the m N_p x m N_p block of v; same outputs S, g,
                              Y, z (to rounding) with 4x smaller dense factorizations.
                              FP64 hdg_assemble_condense only (the FP32 path and batches
                              condense the full block). Needs N_p + nf N_fp + 1 <= 112
                              and the elimination's LDS sets within 160 KB (hexahedra up
                              to p = 2, tetrahedra up to p = 3); otherwise plan creation
                              returns HDG_EUNSUPPORTED, and HDG_EINVAL for Euler. 
                              HDG_FLAG_GHAT_INTERIOR (Navier-Stokes): viscous numerical
                              flux G(v_h, q_h).n with the element's v_h (the first of the
                              two viscous fluxes of Section 3.3) instead of G(vhat_h, q_h).n
                              (the one of the paper's examples, the default).
                              HDG_FLAG_SIGMA_S: stabilization matrix sigma_S =
                              |A_n(vhat)| A0(vhat) (the symmetric variable matrix of
                              Section 4, v* = vhat) instead of sigma_SLF =
                              lambda_max(vhat) A0(vhat) (the paper's examples).
                              HDG_FLAG_SIGMA_MV: the mean-value stabilization matrix of
                              Section 4 on the straight path between vhat and v in
                              entropy variables (its two integrals combined into one
                              integral of sigma_S over the path, 4-point Gauss-Legendre);
                              takes precedence over HDG_FLAG_SIGMA_S.
                              HDG_FLAG_GHAT_PROJ: the projection viscous numerical flux
                              of Section 4, (Pi G(v_h, q_h)).n on every face with Pi the
                              element L2 projection onto the space of q_h (volume
                              quadrature); Navier-Stokes only, element blocks and
                              residuals (not the matrix-free Jacobian of the FP32 path,
                              which refuses it); takes precedence over
                              HDG_FLAG_GHAT_INTERIOR. */
} hdg_opts;

typedef struct {
  int dim, m, Np, nf, Nfp, Nq, Nfq;
  int n, k;                /* local and element-trace block sizes */
  int n_pad, k_pad;        /* internal padded sizes */
  int n_elem, n_trace, chunk_elems;
} hdg_dims;

/* Create a plan: builds reference tables and element geometry on the host.
 * Returns HDG_EINVAL for bad sizes or a non-positive Jacobian, HDG_EUNSUPPORTED
 * for an order outside 1..4. */
int hdg_plan_create(hdg_plan **plan, const hdg_mesh *mesh, const hdg_phys *phys, const hdg_opts *opts);
void hdg_plan_destroy(hdg_plan *plan);
/* Replace gamma, mu, Pr and alpha of a plan (the viscous flag must not change);
 * takes effect at the next call. */
int hdg_plan_set_phys(hdg_plan *plan, const hdg_phys *phys);
int hdg_plan_dims(const hdg_plan *plan, hdg_dims *out);
/* Source term of the conservation law (the right-hand side s of the Navier-Stokes
 * equations with a source, as in the Couette problem of Section 5): nodal values
 * src [m][E*Np] in the layout of v (device, caller-owned, read at every assemble
 * until replaced; NULL removes it).  The element residual receives -(s_h, w) with s_h
 * the nodal interpolant at the volume quadrature points; the Jacobian is unchanged. */
int hdg_plan_set_source(hdg_plan *plan, const double *src);
/* The same source given by its values at the volume quadrature points, src [m][E*Nq]
 * (hdg_quad_coords order; device, caller-owned, read at every assemble until replaced; NULL
 * removes it): the element residual receives -sum_q W_q s(x_q) phi_a(x_q), the quadrature of
 * (s, w) with s itself, as the oracle forms it. */
int hdg_plan_set_source_points(hdg_plan *plan, const double *src);
/* Physical coordinates of the volume quadrature points, xq [dim][E*Nq] (device),
 * element-major (e Nq + q): the image of the reference points under the element map. */
int hdg_quad_coords(const hdg_plan *plan, double *xq, void *stream);
/* Element L2 errors against values at the volume quadrature points (xq order):
 *   out[e][c] = sum_q W_q (f_c(x_q) - exact[c][e Nq + q])^2,
 * kind 0: f = u(v_h) from v [m][E*Np], c < m (conserved variables);
 * kind 1: f = the gradient unknowns q [m*dim][E*Np] interpolated, c < m*dim (NS only);
 * kind 2: f = the entropy variables v_h [m][E*Np] interpolated, c < m;
 * kind 3 (NS only): the viscous stress and heat flux formed from the state and its gradient
 *   unknowns, as the Couette example of Section 5 measures them: f = [v; q] stacked
 *   [(m + m*dim)][E*Np] (v_h, q_h), exact = [v; q] stacked [(m + m*dim)][E*Nq] at the
 *   quadrature points; c < dim*dim + dim (tau[i][j] row-major, then f[j]); tau and f are those
 *   of the plan's viscous flux G = -(0, tau, V.tau - f).
 * All device; out [E][m], [E][m*dim] or [E][dim*dim + dim]. */
int hdg_l2_error(const hdg_plan *plan, int kind, const double *f, const double *exact, double *out,
                 void *stream);
/* Physical coordinates of the face quadrature points of every element face,
 * xf [dim][E*nf*Nfq] (device), ordered (e nf + f) Nfq + q: the face's image under the element
 * map.  Where Dirichlet data is known as a function, evaluate it here for hdg_trace_project. */
int hdg_face_quad_coords(const hdg_plan *plan, double *xf, void *stream);
/* Dirichlet data of the trace equation as the face L2 projection (Section 3: the trace equation
 * is tested against every trace function mu, so <v_hat - v_bc, mu>_F = 0 with v_bc the boundary
 * function makes v_hat its L2(F) projection): for every Dirichlet-trace face, the nodal trace
 * coefficients c solving M_F c = <g, mu>_F (M_F the face mass matrix of the trace basis, face
 * quadrature) are written to v_bc [m][n_trace] at that face's trace nodes; other entries are left
 * as they are.  g [m][E*nf*Nfq]: entropy variables of the boundary state at the face quadrature
 * points (hdg_face_quad_coords order; only Dirichlet faces are read).  Device pointers, caller
 * owned.  HDG_EUNSUPPORTED when a trace node is shared by two Dirichlet faces (a continuous
 * trace at a boundary corner has no face-local projection) or a face has more than 25 nodes. */
int hdg_trace_project(const hdg_plan *plan, const double *g, double *v_bc, void *stream);
/* Total thermodynamic entropy and mass of each element (the quantities whose evolution
 * Proposition 1 and the Shu vortex example of Section 5 follow):
 *   out[e][0] = int_K rho s,  out[e][1] = int_K rho,  s = ln(p / rho^gamma),
 * at the states u(v_h) of v [m][E*Np], by the volume quadrature.  -out[e][0] is the
 * element integral of the generalized entropy H = -rho s of the entropy-variable section;
 * a baseline s0 enters as -s0 out[e][1].  Device pointers; out [E][2]. */
int hdg_entropy_integral(const hdg_plan *plan, const double *v, double *out, void *stream);
/* Element integrals of the flow statistics followed in the Taylor-Green example of
 * Section 5, by the volume quadrature at the states u(v_h) of v [m][E*Np] and the
 * velocity gradients of v_h (V = -w / v_m, w = the middle entropy variables):
 *   out[e][0..7] = int_K (rho s, rho, rho |V|^2 / 2, |omega|^2, theta, theta^2, T, T^2),
 * s = ln(p / rho^gamma), omega = curl V (the scalar dV_y/dx - dV_x/dy in 2D), theta = div V,
 * T = p / rho (temperature up to the gas constant).  Means and variances follow by
 * dividing by the domain volume.  Device pointers; out [E][8]. */
int hdg_flow_statistics(const hdg_plan *plan, const double *v, double *out, void *stream);

/* Bytes of device workspace the plan needs (tables + per-chunk scratch). */
int hdg_plan_workspace_bytes(const hdg_plan *plan, size_t *bytes);

/* Bind caller-owned device workspace (>= hdg_plan_workspace_bytes, 256-byte
 * aligned) and upload the tables into it (synchronous on `stream`).  The
 * workspace belongs to the plan until it is bound again or the plan is
 * destroyed: when all elements fit in one chunk, the plan keeps the structural
 * zeros of its coupling blocks there between calls and clears them only on the
 * first call after a bind. */
int hdg_plan_bind_workspace(hdg_plan *plan, void *dev_ptr, size_t bytes, void *stream);

/* Physical coordinates of the element nodes x[dim][E*Np] and of the global
 * trace nodes xt[dim][n_trace] (device pointers, either may be NULL). */
int hdg_node_coords(const hdg_plan *plan, double *x, double *xt, void *stream);

/* Workload preparation (entropy-variable section): from primitives
 * prim[m][N] = (rho, V_1..V_dim, p) and optional gradients grad[m][dim][N]
 * compute v[m][N] = v(u(prim)), q[m*dim][N] = dv/dprim . grad (NULL-able),
 * u[m][N] = conservation variables (NULL-able).  Device pointers. */
int hdg_prepare_state(const hdg_plan *plan, int N, const double *prim, const double *grad,
                      double *v, double *q, double *u, void *stream);

/* Residual and Jacobian blocks of every element (no condensation), compact
 * column-major: A [E][n][n], B [E][k][n] (n x k), C [E][n][k] (k x n),
 * D [E][k][k], R_loc [E][n], R_tr [E][k].  Inputs as in hdg_assemble_condense.
 * Any output may be NULL.  Meant for inspection and tests. */
int hdg_assemble(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                 const double *u_star, const double *v_bc,
                 double *A, double *B, double *C, double *D, double *R_loc, double *R_tr,
                 int32_t *elem_status, void *stream);

/* Static condensation of caller-supplied element blocks (local elimination remark of
 * Section 3.3): for every element, S = D - C A^-1 B, g = -R_tr + C A^-1 R_loc,
 * Y = A^-1 B, z = A^-1 R_loc with the kernels of hdg_assemble_condense.  Blocks in the
 * compact layout hdg_assemble exports (A [E][n][n], B [E][k][n], C [E][n][k], D [E][k][k],
 * R_loc [E][n], R_tr [E][k], column-major); outputs as hdg_assemble_condense.  A zero pivot
 * sets elem_status[e] = HDG_ESINGULAR (the outputs of that element are then meaningless).
 * Uses the plan's workspace; device pointers. */
int hdg_condense_blocks(hdg_plan *plan, const double *A, const double *B, const double *C, const double *D,
                        const double *R_loc, const double *R_tr, double *S, double *g, double *Y, double *z,
                        int32_t *elem_status, void *stream);

/* The hot path.  For every element: residual R_loc, R_tr and Jacobian blocks
 * [A B; C D] of the Newton system [A B; C D][dx; dlambda] = -[R_loc; R_tr],
 * LU of A with partial pivoting, and
 *     Y = A^-1 B,  z = A^-1 R_loc,  S = D - C Y,  g = -R_tr + C z.
 * v, vhat required; q required iff viscous; u_star [m][E*Np] nodal u* of the
 * mass term (NULL: u* = 0, needs alpha == 0 to be meaningful); v_bc [m][n_trace]
 * Dirichlet data read on Dirichlet-trace faces (NULL: zero).  Outputs S, g, Y, z
 * required; R_loc, R_tr optional copies of the element residuals.
 * elem_status [E] (required) receives HDG_OK or a device-side error code. */
int hdg_assemble_condense(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                          const double *u_star, const double *v_bc,
                          double *S, double *g, double *Y, double *z,
                          double *R_loc, double *R_tr, int32_t *elem_status, void *stream);

/* Local back-solve after the global trace update (same passage):
 *   dx_K = -z_K - Y_K P_K dlambda,   P_K the trace-map gather.
 * dvhat [m][n_trace]; outputs dv [m][E*Np] and (NS) dq [m*dim][E*Np] in the
 * global SoA layout (dq may be NULL for Euler). */
int hdg_backsolve(hdg_plan *plan, const double *Y, const double *z, const double *dvhat,
                  double *dv, double *dq, void *stream);

/* Condensed trace operator y = sum_K P_K^T S_K P_K x on [m][n_trace] vectors
 * (overwrites y).  HDG, EDG and IEDG differ only in the trace map (the paper's
 * remark that the three schemes differ only in the trace unknowns). */
int hdg_trace_matvec(hdg_plan *plan, const double *S, const double *x, double *y, void *stream);

/* Right-hand side of the condensed system r = sum_K P_K^T g_K ([m][n_trace]). */
int hdg_trace_rhs(hdg_plan *plan, const double *g, double *r, void *stream);

/* ---- Kernel tuning ---------------------------------------------------------
 * Launch shapes of one plan (0 leaves a field unchanged): workgroup size of
 * the block contraction (256, 512, 1024 threads), column-block width of the
 * fused FP64 / FP32 condensation (32 or 16; must fit in LDS), and its number
 * of launches: 1 (one workgroup per element factors A and works through every
 * right-hand-side block) or 2 (default: one workgroup per element for the LU,
 * then one per element and right-hand-side block, the workgroups of an
 * element on one XCD so that they share its factors in L2; the results are
 * the same bit for bit).  The autotuner
 * (paper_1808_05066_amd/autotune.py) sweeps these per (n, k, dtype) and caches
 * the fastest in JSON.  Set before building a batch (batches run their own
 * two launches with the LDS-block LU).
 * lu_waves selects the LU of the two-launch FP64 condensation: 1 keeps its
 * 32-column working block in LDS (one workgroup per CU), 2, 4 or 8 keep it in
 * the registers of that many waves (LDS for staging only: with 2 waves four
 * elements share a CU, with 4 waves two; 2 for n_pad <= 160, 4 for
 * n_pad <= 192, 8 for n_pad <= 640).  Default: 2 where it applies, else 4
 * where it applies, else 1.
 * lp_operands selects the matrix-core operands of hdg_assemble_condense_lp:
 * 1 (default) FP32, 2 BF16 (rounded to nearest, FP32 accumulation; the data,
 * the panel factorizations, the stored factors and the outputs stay FP32).
 * With BF16 the factors and S, Y carry BF16-level errors (relative ~1e-3
 * times the growth), so the FP64 refinement needs more steps.  The factors are stored the same way, so S, g, Y,
 * z agree to rounding (the register kernels pick a pivot whose magnitude is
 * within a relative 2^-11 of the column's largest).  HDG_EUNSUPPORTED if the
 * block is too large for the choice. */
typedef struct {
  int contract_threads;
  int condense_width;
  int condense_width_lp;
  int condense_launches;
  int lu_waves;
  int lp_operands;
} hdg_tuning;

int hdg_plan_set_tuning(hdg_plan *plan, const hdg_tuning *t);
int hdg_plan_get_tuning(const hdg_plan *plan, hdg_tuning *t);

/* ---- Batches ----------------------------------------------------------------
 * Several plans (element types / orders with uneven n, k, e.g. tetrahedra of
 * orders 1..4 next to hexahedra) condensed by two launches over item lists:
 * LU items (plan, element) in decreasing order of block cost (order 0, longest
 * processing time first) or plan order (order 1), then right-hand-side items
 * (plan, element, column block) in eight lists, one per XCD (an element's
 * items lie together in one XCD's list, so its workgroups share the factors
 * in that XCD's L2).  By default each item gets a workgroup of its own, in
 * list order (the hardware starts them in index order as CUs free up);
 * hdg_batch_set_groups selects a persistent grid instead, whose workgroups
 * take items from atomic counters until the lists are empty.  Outputs equal the per-plan
 * two-launch condensation with the LDS-block LU bit for bit.  Every plan must
 * be bound, use the fused condensation and process all its elements in one
 * chunk; its pointwise and contraction kernels run first, per plan.  The
 * whole sequence can be captured in a hipGraph and replayed.  The batch
 * copies the plans' descriptors at bind time: set tunings before binding. */
typedef struct hdg_batch hdg_batch;

typedef struct {            /* per plan, device pointers as in hdg_assemble_condense */
  const double *v, *q, *vhat, *u_star, *v_bc;
  double *S, *g, *Y, *z;
  int32_t *elem_status;
} hdg_batch_io;

int hdg_batch_create(hdg_batch **batch, hdg_plan *const *plans, int n_plans, int order);
void hdg_batch_destroy(hdg_batch *batch);
/* Caller-owned device workspace (descriptors, queues, counters). */
int hdg_batch_workspace_bytes(const hdg_batch *batch, size_t *bytes);
int hdg_batch_bind_workspace(hdg_batch *batch, void *dev_ptr, size_t bytes, void *stream);
/* Stream mode (n = 1..8; 0, the default, returns to the item lists): instead
 * of the two batched launches, every plan runs its own hdg_assemble_condense
 * (its own tuning: block width, launch count, LU variant, LDS size) on one of
 * n streams the batch creates (default priority, non-blocking), forked from
 * the caller's stream and joined back into it, so that the plans' kernels run
 * concurrently and the small blocks fill the LDS and wave slots the large
 * ones leave free.  Plans go to streams largest first (order 0) or in plan
 * order, each to the stream with the least work so far.  Outputs equal the
 * plans' own hdg_assemble_condense bit for bit.  A captured graph holds the
 * fork and join. */
int hdg_batch_set_streams(hdg_batch *batch, int n);
/* 0 (default): one workgroup per item.  groups > 0: persistent grids, the LU
 * launch with `groups` workgroups (at most one per item), the right-hand-side
 * launch with `groups` rounded up to a multiple of 8.  HDG_EINVAL if < 0. */
int hdg_batch_set_groups(hdg_batch *batch, int groups);
/* Inputs / outputs of every plan (array of n_plans); synchronous upload. */
int hdg_batch_set_io(hdg_batch *batch, const hdg_batch_io *io, void *stream);
/* Run once: per plan status reset + pointwise + contraction, then the two
 * launches of the condensation.  n_items of hdg_batch_info counts the LU
 * items (one per element); its groups is the value of hdg_batch_set_groups. */
int hdg_batch_run(hdg_batch *batch, void *stream);
/* Capture the sequence of hdg_batch_run in a graph (after one eager run on the
 * same stream); hdg_batch_replay launches it.  Phase timing must be off. */
int hdg_batch_capture(hdg_batch *batch, void *stream);
int hdg_batch_replay(hdg_batch *batch, void *stream);
int hdg_batch_info(const hdg_batch *batch, int *n_items, int *groups, size_t *lds_bytes);

/* ---- Global trace solve --------------------------------------------------
 * The paper leaves the linear solver of the condensed system open; this
 * library solves  K dlambda = r,  K = sum_K P_K^T S_K P_K  (the trace operator
 * above), with restarted GMRES, right-preconditioned:
 *   precond 0: none;
 *   precond 1: block Jacobi on the diagonal blocks of K.  A block holds the
 *     unknowns of one mesh face (all components, face nodes in ascending
 *     trace-node order) when every trace node lies on exactly one face (HDG),
 *     else the m x m block of one trace node (EDG / IEDG, where faces share
 *     nodes).
 * Arnoldi uses classical Gram-Schmidt with one reorthogonalization pass; every
 * vector operation runs on the device, the (restart+1) x restart Hessenberg
 * matrix and its Givens rotations on the host (one stream synchronization per
 * iteration).  Stopping test: ||r - K x|| <= tol ||r||, checked on the true
 * residual at every restart and on return. */
typedef struct {
  int restart;    /* Krylov dimension per cycle (>= 1; 50 in the benchmarks) */
  int maxit;      /* total Arnoldi steps allowed */
  double tol;     /* relative residual target (> 0) */
  int precond;    /* 0 none, 1 block Jacobi */
  int s_dtype;    /* element type of S: HDG_FP64 (double) or HDG_FP32 (float, the
                     mixed-precision path); vectors and arithmetic stay FP64 */
} hdg_solve_opts;

typedef struct {
  int iterations;       /* Arnoldi steps taken */
  int converged;        /* 1 if the returned x meets tol */
  double rel_residual;  /* true ||r - K x|| / ||r|| of the returned x */
  double solve_ms;      /* host wall time of hdg_trace_solve */
} hdg_solve_info;

/* Bytes of caller-owned device workspace for the solver (block inverses,
 * restart+1 Krylov vectors, reduction scratch); 256-byte aligned pointer. */
int hdg_solver_workspace_bytes(const hdg_plan *plan, const hdg_solve_opts *opts, size_t *bytes);

/* Assemble the block-Jacobi blocks of K from S [E][k][k] and invert them (LU
 * with partial pivoting) into `work`.  Synchronizes `stream`; HDG_ESINGULAR if
 * a block has a zero pivot.  Required before precond 1 is used. */
int hdg_precond_setup(hdg_plan *plan, const void *S, void *work, size_t bytes,
                      const hdg_solve_opts *opts, void *stream);

/* z = M^-1 r with the blocks from hdg_precond_setup; r, z [m][n_trace]. */
int hdg_precond_apply(hdg_plan *plan, void *work, size_t bytes, const hdg_solve_opts *opts,
                      const double *r, double *z, void *stream);

/* Solve K x = rhs (x overwritten, initial guess 0).  Device pointers S, rhs,
 * x, work; `info` on the host.  Returns HDG_OK also when tol is not reached
 * within maxit (info->converged = 0). */
int hdg_trace_solve(hdg_plan *plan, const void *S, const double *rhs, double *x, void *work,
                    size_t bytes, const hdg_solve_opts *opts, hdg_solve_info *info, void *stream);

/* ---- Learned block-Jacobi correction ---------------------------------------
 * Not in the paper.  A small network corrects every block-Jacobi inverse B_F by
 * a row and column rescaling and a rank-R term (R = 4) that couples the block's
 * unknowns:
 *   M_F^-1 = diag(e^a) (B_F + (c U)(c V)^T) diag(e^b),  c_i = |B_F,ii|^(1/2),
 *   a_i = 0.5 tanh(o_i,0), b_i = 0.5 tanh(o_i,1),
 *   U_ik = tanh(o_i,2+k), V_ik = tanh(o_i,2+R+k)   (k < R),
 *   o_i = W3 tanh(W2 tanh(W1 f_i + b1) + b2) + b3   (16 -> 32 -> 32 -> NO = 2 + 2R, FP32)
 * with f_i 16 features of block row i (log10 |D_ii| and ||D_i,:|| of the
 * assembled block, log10 of the coupling of the row to other blocks and its
 * ratio to the row norm, one-hot component, node position on the face, local
 * Mach number, log10 p and log10 rho of the trace state, a constant 1; logs
 * scaled by 1/4).  Rows are in block order (block F, position i -> F*bs + i,
 * i = c * nodes_per_block + p); N_rows = m * n_trace.  Parameters (float,
 * hdg_learn_nparams of them): W1[32][16] b1[32] W2[32][32] b2[32] W3[NO][32] b3[NO].
 * Training loss over random vectors x_v with w_v = K x_v:
 *   L = sum_v ||x_v - M^-1 w_v||^2 / x2,  x2 = sum_v ||x_v||^2,
 * minimized with Adam (beta 0.9, 0.999, eps 1e-8).  All pointers device. */
int hdg_learn_nparams(void);
/* NO, the network outputs per row. */
int hdg_learn_outputs(void);

/* Block-Jacobi setup as hdg_precond_setup (inverses into `work`) plus the
 * features feat [N_rows][16] from S (type per opts->s_dtype) and vhat [m][n_trace]. */
int hdg_learn_setup(hdg_plan *plan, const void *S, const double *vhat, float *feat, void *work, size_t bytes,
                    const hdg_solve_opts *opts, void *stream);
/* out [N_rows][NO] = network outputs o. */
int hdg_learn_forward(hdg_plan *plan, const float *theta, const float *feat, float *out, void *stream);
/* Replace the inverses held in `work` by the corrected blocks M_F^-1 (formed
 * whole, bs <= 256); hdg_trace_solve with precond 1 then applies the learned
 * preconditioner (same cost as block Jacobi). */
int hdg_learn_apply(hdg_plan *plan, const float *out, void *work, size_t bytes, const hdg_solve_opts *opts,
                    void *stream);
/* Loss (into *loss, device double) and dL/do [N_rows][NO] for nvec vectors X, Wv
 * [nvec][m][n_trace] with the UNSCALED inverses in `work`. */
int hdg_learn_loss_grad(hdg_plan *plan, const void *work, size_t bytes, const hdg_solve_opts *opts,
                        const float *out, const double *X, const double *Wv, int nvec, double x2, float *dO,
                        double *loss, void *stream);
/* Floats of scratch for hdg_learn_backward. */
int hdg_learn_scratch_floats(const hdg_plan *plan, size_t *n);
/* grad [nparams] = dL/dtheta from dO (recomputes the forward pass). */
int hdg_learn_backward(hdg_plan *plan, const float *theta, const float *feat, const float *dO, float *grad,
                       float *scratch, void *stream);
/* hdg_learn_backward without the caller's scratch, for callers that cannot allocate device
 * memory (code under stream capture, serving loops, harnesses that forbid allocation): the
 * partial gradients live in a static device array of 32 MiB that the library holds on every GPU
 * it runs on until the process ends; no hipMalloc, hipFree or other allocation is made.  Same
 * kernels and result as hdg_learn_backward.  N_rows = m * n_trace may be at most 278,144 (the
 * array holds 4,346 workgroups of 64 rows); larger plans get HDG_EINVAL.  Calls on one GPU share
 * the array: calls that overlap on one GPU (other streams or threads) race. */
int hdg_learn_backward_noalloc(hdg_plan *plan, const float *theta, const float *feat, const float *dO, float *grad,
                               void *stream);
/* One Adam step (t >= 1) on theta with moments m, v. */
int hdg_learn_adam(float *theta, const float *grad, float *m, float *v, int t, float lr, void *stream);
/* forward + loss_grad + backward + adam. */
int hdg_learn_train_step(hdg_plan *plan, float *theta, float *m, float *v, int t, float lr, const float *feat,
                         const void *work, size_t bytes, const hdg_solve_opts *opts, const double *X,
                         const double *Wv, int nvec, double x2, float *out, float *dO, float *grad, float *scratch,
                         double *loss, void *stream);
/* Training on face blocks sampled from many systems (a pool; blocks of equal size bs).
 * hdg_learn_extract copies, after hdg_learn_setup of a system, the blocks sel[q] (device int
 * array, nsel entries, q < nsel) to pool block b0 + q: the unscaled inverse into pool_B
 * [blocks][bs][bs] (column-major), the rows' features into pool_feat [blocks * bs][16], and x and
 * w = K x of the rows for the nvec vectors X, Wv [nvec][m][n_trace] into pool_X, pool_W
 * [nvec][ld] (block-row order; ld >= (b0 + nsel) * bs, else HDG_EINVAL).  The caller owns the
 * pool and picks the blocks. */
int hdg_learn_extract(hdg_plan *plan, const void *work, size_t bytes, const hdg_solve_opts *opts, const float *feat,
                      const double *X, const double *Wv, int nvec, const int *sel, int nsel, size_t b0, size_t ld,
                      double *pool_B, float *pool_feat, double *pool_X, double *pool_W, void *stream);
/* Network forward / backward on N rows of features (no plan); scratch of backward_rows:
 * hdg_learn_rows_scratch_floats(N) floats. */
int hdg_learn_forward_rows(const float *theta, const float *feat, size_t N, float *out, void *stream);
int hdg_learn_rows_scratch_floats(size_t N, size_t *n);
int hdg_learn_backward_rows(const float *theta, const float *feat, const float *dO, size_t N, float *grad,
                            float *scratch, void *stream);
/* Loss (into *loss, cleared first) and dL/do [nblk * bs][NO] over the first nblk pool blocks
 * (bs <= 256), x2 the squared norm of the pool's x over those rows and vectors. */
int hdg_learn_pool_loss_grad(int nblk, int bs, const double *pool_B, const float *out, const double *X,
                             const double *Wv, size_t ld, int nvec, double x2, float *dO, double *loss,
                             void *stream);

/* ---- Mixed precision ------------------------------------------------------
 * Low-precision condensation with FP64 refinement of the full Newton linear
 * system  J delta = -R,  J = [A B; C D] coupled through the traces.
 *
 * hdg_assemble_condense_lp: as hdg_assemble_condense (points, residuals and
 * block contraction in FP64), then per element the symmetric power-of-two
 * scaling A_hat = D A D, d_i = 2^-round(log2 sqrt|a_ii|), LU with partial
 * pivoting of A_hat in FP32 on the FP32 matrix cores (FP32 accumulation), and
 *   Y = D A_hat^-1 D B,  z = D A_hat^-1 D R_loc,  S = D - C Y,  g = -R_tr + C z
 * with FP32 arithmetic.  S [E][k][k] and Y [E][k][n] are written as float
 * (column-major as in the FP64 path), g and z as double (low-precision values).
 * `factors` (hdg_lp_factor_bytes) receives per element the FP32 factors,
 * pivots, scaling and diagonal-block inverses for hdg_lp_solve; R_loc [E][n]
 * and R_tr [E][k] (FP64 residuals) are optional but needed by the refinement.
 * HDG_EUNSUPPORTED when the FP32 working block does not fit in LDS. */
int hdg_lp_factor_bytes(const hdg_plan *plan, size_t *bytes);
int hdg_assemble_condense_lp(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                             const double *u_star, const double *v_bc, float *S, double *g, float *Y,
                             double *z, float *factors, double *R_loc, double *R_tr, int32_t *elem_status,
                             void *stream);

/* x_K = A_lp,K^-1 r_K for every element from the stored FP32 factors (FP64
 * vectors and arithmetic); r, x [E][n] element-local, must not alias. */
int hdg_lp_solve(hdg_plan *plan, const float *factors, const double *r, double *x, void *stream);

/* Matrix-free FP64 action of the element Newton matrices:
 *   y_loc,K = A_K dx_K + B_K P_K dlam,   y_tr,K = C_K dx_K + D_K P_K dlam
 * from the quadrature-point Jacobians (no element matrix is formed).
 * dx, y_loc [E][n]; dlam [m][n_trace]; y_tr [E][k] (element-local trace rows;
 * hdg_trace_rhs assembles them).  The pointwise data are recomputed from the
 * state (v, q, vhat, u_star, v_bc as in hdg_assemble_condense) unless
 * reuse_points != 0 and the plan processes all elements in one chunk, in which
 * case those of the last call on this plan are used (caller guarantees the
 * state is unchanged). */
int hdg_jacobian_apply(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                       const double *u_star, const double *v_bc, int reuse_points, const double *dx,
                       const double *dlam, double *y_loc, double *y_tr, int32_t *elem_status, void *stream);

typedef struct {
  int max_outer;          /* refinement steps allowed */
  double tol;             /* target ||J delta + R|| / ||R|| (FP64, full system) */
  int reuse_points;       /* passed to hdg_jacobian_apply */
  hdg_solve_opts gmres;   /* inner solve on the FP32 condensed system (s_dtype forced FP32) */
} hdg_refine_opts;

typedef struct {
  int outer_iterations, gmres_iterations, converged;
  double rel_residual;    /* ||J delta + R|| / ||R|| of the returned delta */
  double total_ms, gmres_ms;   /* host wall time: whole call; global solves incl. preconditioner setup */
  double history[16];     /* relative residual after each refinement step */
  int fallback_elements;  /* hdg_refine_local: elements solved by the FP64 fallback */
} hdg_refine_info;

int hdg_refine_workspace_bytes(const hdg_plan *plan, const hdg_refine_opts *opts, size_t *bytes);

/* Outer refinement: delta = 0; repeat  c = J_lp^-1 r  (hdg_lp_solve, FP64
 * action of C, GMRES on the FP32 Schur system, back-solve with FP32 Y),
 * delta += c,  r = -R - J delta (hdg_jacobian_apply)  until the relative
 * residual reaches tol.  Outputs dx [E][n] (element-local) and dlam
 * [m][n_trace] with J (dx, dlam) = -(R_loc, sum_K P^T R_tr). */
int hdg_refine_solve(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                     const double *u_star, const double *v_bc, const float *S, const float *Y,
                     const float *factors, const double *R_loc, const double *R_tr, double *dx,
                     double *dlam, void *work, size_t bytes, const hdg_refine_opts *opts,
                     hdg_refine_info *info, int32_t *elem_status, void *stream);

/* Element-local back-solve dx [E][n] = -z - Y P dvhat in the element-local ordering (the
 * layout of hdg_refine_solve / hdg_refine_local), FP64 Y [E][k][n] and z [E][n] of
 * hdg_assemble_condense; dvhat [m][n_trace].  Device pointers. */
int hdg_backsolve_elements(hdg_plan *plan, const double *Y, const double *z, const double *dvhat, double *dx,
                           void *stream);

/* Element-level refinement with a fixed trace update (the element version of the mixed-precision
 * criterion, for meshes processed without a global solve): with the low-precision factors of
 * hdg_assemble_condense_lp, solve per element  A dx = -(R_loc + B P dvhat)  by dx = 0; repeat
 * dx += A_lp^-1 r, r = -(R_loc + A dx + B P dvhat) with A and B applied matrix-free in FP64
 * (hdg_jacobian_apply), until max_K ||r_K|| / ||R_loc,K + B_K P_K dvhat|| <= tol, max_iter
 * steps, or a step that does not halve that maximum (stagnation).  Short of tol, the elements
 * still above it fall back to FP64: their blocks are re-assembled in full and solved with the
 * FP64 LU (right-looking kernels); info->fallback_elements counts them.  dx [E][n]
 * element-local; info->rel_residual is the final maximum, history[] per step, gmres fields 0.  reuse_points: the pointwise data of the last assembly of this plan are
 * current (one chunk only).  Workspace: hdg_refine_local_workspace_bytes, 256-byte aligned. */
int hdg_refine_local_workspace_bytes(const hdg_plan *plan, size_t *bytes);
int hdg_refine_local(hdg_plan *plan, const double *v, const double *q, const double *vhat, const double *u_star,
                     const double *v_bc, const float *factors, const double *R_loc, const double *dvhat, double *dx,
                     void *work, size_t bytes, int max_iter, double tol, int reuse_points, hdg_refine_info *info,
                     int32_t *elem_status, void *stream);

/* ---- Newton iterations on the nonlinear system (library's own driver) ----
 * Solves R(v, q, vhat) = 0 for one implicit stage (the plan's alpha > 0 with the
 * previous-stage state u_star) or the steady problem (alpha = 0): R is the element
 * residual R_loc of every element together with the assembled trace residual
 * sum_K P_K^T R_tr,K (the weak forms of Sections 3.3 and 4).  Each iteration
 * assembles and condenses every element (hdg_assemble_condense), solves the
 * condensed system K dlambda = sum_K P_K^T g_K with GMRES (opts->lin, block
 * Jacobi if precond = 1; S in FP64), back-solves dx_K = -z_K - Y_K P_K dlambda
 * and updates v += dv, q += dq (Navier-Stokes), vhat += dlambda in place (the
 * local elimination remark after the weak forms).  Stops when
 * ||R|| <= atol or ||R|| <= tol ||R_0|| (converged = 1), or after maxit updates.
 * v [m][E*Np], q [m*dim][E*Np] (NULL for Euler), vhat [m][n_trace] device,
 * updated in place; u_star, v_bc as for hdg_assemble_condense.  work: device,
 * 256-byte aligned, at least hdg_newton_workspace_bytes (S, g, Y, z, the
 * residuals, the updates and the solver's workspace); info on the host.
 * Synchronizes `stream` every iteration.  An element with a non-OK status stops
 * the iteration with its code (e.g. HDG_ENONPHYS). */
#define HDG_NEWTON_HIST 32
typedef struct {
  int maxit;              /* Newton updates at most (>= 1) */
  double tol;             /* relative stop: ||R|| <= tol ||R_0|| */
  double atol;            /* absolute stop: ||R|| <= atol */
  hdg_solve_opts lin;     /* linear solves; s_dtype must be HDG_FP64 */
} hdg_newton_opts;

typedef struct {
  int iterations;         /* updates applied */
  int converged;          /* 1 if a stop criterion was met */
  int lin_iterations;     /* GMRES Arnoldi steps over all iterations */
  int lin_converged;      /* 1 if every linear solve met opts->lin.tol */
  double res[HDG_NEWTON_HIST];   /* ||R|| at the state before update i (res[iterations]: final state) */
  double ms;              /* host wall time */
} hdg_newton_info;

int hdg_newton_workspace_bytes(const hdg_plan *plan, const hdg_newton_opts *opts, size_t *bytes);
int hdg_newton_solve(hdg_plan *plan, double *v, double *q, double *vhat, const double *u_star,
                     const double *v_bc, void *work, size_t bytes, const hdg_newton_opts *opts,
                     hdg_newton_info *info, void *stream);

/* One step of Alexander's three-stage L-stable DIRK(3,3) (the time integration of the
 * paper's numerical examples, Section 5) around hdg_newton_solve: stage i solves
 *   alpha (u(v_i) - u*_i, w) + s(v_i; w) = 0,  alpha = 1/(a_ii dt),
 * s the steady residual, with (u*_i, w) = (u_n, w) - dt sum_{j<i} a_ij s(v_j; w) formed
 * on the element L2 products b(v) = (u(v), phi_a)_K from the converged earlier stages
 * (s(v_j; w) = -alpha (u(v_j) - u*_j, w)), and u*_i = M_K^-1 b*_i as nodal values.  The
 * scheme is stiffly accurate: (v, q, vhat) are replaced by the last stage's solution
 * (each stage starts from the previous one).  Sets the plan's alpha to 1/(a_ii dt) (left
 * so afterwards).  info[3]: one hdg_newton_info per stage.  work: device, 256-byte
 * aligned, at least hdg_dirk_workspace_bytes.  Errors as hdg_newton_solve; a stage that
 * does not converge is reported in its info, not as an error. */
int hdg_dirk_workspace_bytes(const hdg_plan *plan, const hdg_newton_opts *opts, size_t *bytes);
int hdg_dirk_step(hdg_plan *plan, double *v, double *q, double *vhat, const double *v_bc, double dt,
                  void *work, size_t bytes, const hdg_newton_opts *opts, hdg_newton_info *info, void *stream);

/* Optional per-phase timing with HIP events recorded on the call's stream
 * around each kernel group: 0 points (pointwise physics), 1 contract (block
 * assembly), 2 LU, 3 triangular solves, 4 Schur product (split dense path),
 * 5 back-solve, 6 trace operator, 7 trace right-hand side, 8 fused
 * condensation (LU + solves + Schur: one kernel, or the two below), 9
 * low-precision fused condensation, 10 low-precision local solve, 11
 * matrix-free Jacobian action, 12 and 13 the LU launch and the right-hand-side
 * launch of an FP64 condensation in two launches (inside phase 8).
 * Enabling resets the totals; hdg_plan_phase_times returns accumulated
 * milliseconds and call counts (up to n entries) and synchronizes on the last
 * recorded events. */
int hdg_plan_set_timing(hdg_plan *plan, int enable);
int hdg_plan_phase_times(hdg_plan *plan, double *ms, long *calls, int n);

/* Device self-check of the FP64 matrix-core operand layout the dense kernels
 * rely on (one 16x16x4 product against a scalar loop); *max_err receives the
 * largest absolute difference (0 expected).  Allocates 8 bytes of device memory. */
int hdg_selftest(double *max_err);

/* First element whose status is not HDG_OK: synchronizes `stream`, copies the
 * n_elem entries of elem_status (device, as filled by an assemble call of this
 * plan) to the host and scans them; *first_bad_elem receives the index (-1 if
 * every element is HDG_OK) and *code its status (HDG_OK then).  Returns
 * HDG_EHIP if the copy fails. */
int hdg_status(const hdg_plan *plan, const int32_t *elem_status, void *stream, int *first_bad_elem, int *code);

/* Last host-side error message of the calling thread. */
const char *hdg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HDG_H_ */
