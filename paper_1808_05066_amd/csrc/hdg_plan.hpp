// Plan: host-built tables, device descriptor passed to the kernels, launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "hdg.h"
#include "hdg_tables.hpp"

namespace hdg {

// Offsets (in doubles) of the pointwise data written per volume / face point.
struct PointLayout {
  int Mv, Kv, Kq, Fr, Wu, Wq, v, WJ, W, size;       // volume
  int fFv, fFq, fFh, fFf, fWn, fvh, fFd, fW, fsize;   // face
};

// Everything a kernel needs; passed by value.
struct DevPlan {
  int dim, m, Np, nf, Nfp, Nq, Nfq, n, k, n_pad, k_pad, kx, viscous, n_elem, n_trace;
  int cw, cw_lp;           // column-block width of the fused FP64 / FP32 condensation (0: not available)
  int contract_threads;    // workgroup size of the block contraction (256, 512, 1024)
  int zero_xcd;            // 1: the contraction clears X, C and D first (0: they hold the zeros already)
  int a_qmin;              // 1: of the q rows of A only M and G_j of the first component are formed
  int ghat_v;              // 1: viscous numerical flux G(v, q).n with the element's v (else G(v_hat, q).n)
  int ghat_proj;           // 1: projection viscous numerical flux (Pi G(v, q)).n, added by the projection kernels
  int sigma_s;             // stabilization: 0 sigma_SLF = lambda_max A0, 1 sigma_S = |A_n| A0 (both at v_hat),
                           // 2 sigma_MV (mean value between v_hat and v)
  int condense_launches;   // 1: fused condensation; 2: LU, then one workgroup per right-hand-side block
  int lu_waves;            // LU of the two-launch FP64 condensation: 0 working block in LDS (k_lu_f64_w32),
                           // 2, 4 or 8: in the registers of that many waves (k_lu_reg)
  int lu_waves_set;        // 1: lu_waves chosen by hdg_plan_set_tuning (else the default per block size)
  int lp_bf16;             // low-precision condensation: 0 FP32 operands, 1 BF16 operands (FP32 accumulation)
  double gamma, mu, Pr, alpha;
  const double *src;       // source of the conservation law (device, caller-owned) or null: nodal [m][E*Np],
  int src_qp;              // or (src_qp = 1) its values at the volume quadrature points [m][E*Nq]
  PointLayout L;
  // tables (device)
  const double *phi;       // [Nq][Np]
  const double *dphi;      // [dim][Nq][Np]
  const double *fphi;      // [nf][Nfq][Nfp]
  const int *fnodes;       // [nf][Nfp]
  const int *node_face;    // [Np][nf]: position of the node on face f, or -1
  const double *geo_vol;   // [E][Nq][1 + dim*dim]: W, dxi_r/dx_j
  const double *geo_face;  // [E][nf][Nfq][1 + dim]: W_f, n
  const int *tmap;         // [E][nf][Nfp]
  const int *face_bc;      // [E][nf]
  const int *row_drop;     // [E][nf][Nfp] 1: the trace rows of this face node are dropped (a continuous
                           // trace node of a Dirichlet face seen from another face), or null when none is
  const double *node_x;    // [dim][E*Np]
  const double *trace_x;   // [dim][n_trace]
  // per-chunk scratch (device)
  double *pv;              // [chunk][Nq][L.size]
  double *pf;              // [chunk][nf][Nfq][L.fsize]
  double *A;               // [chunk][n_pad][n_pad]       column-major
  double *X;               // [chunk][kx][n_pad]          [B | R_loc | 0] then [Y | z]
  double *C;               // [chunk][n_pad][k_pad]       column-major k_pad x n_pad
  double *D;               // [chunk][k_pad][k_pad]
  double *Rt;              // [chunk][k_pad]
  int *ipiv;               // [chunk][n_pad]
  double *inv;             // [chunk][n_pad/32][2][32][32] inverses of diagonal factor blocks
  // q rows of A in compact form (Navier-Stokes with the matrix-core contraction, else null):
  // the condensation forms the q rows and the padding of A from these instead of reading them
  double *mg;              // [chunk][1 + dim][Np][Np]: G_j[a][b] (j < dim), M[a][b] (j = dim)
  const int *uinfo;        // [n_pad]: node | direction << 8 | component << 12 of each local unknown
  // projection viscous flux scratch (null unless ghat_proj): W (G, dG/dv, dG/dq) at the volume
  // points [chunk][Nq][MD + MD M + MD MD], and the face lift Z [chunk][nf][dim][Nfp][Nq]
  double *gp;
  double *gz;
  // block-Jacobi structure of the condensed operator
  int bj_face;             // 1: one block per mesh face (HDG), 0: one m x m block per trace node
  int bj_nblk, bj_bs;
  const int *bj_nodes;     // [nblk][nodes per block] global trace nodes (sorted)
  const int *bj_ce;        // [nblk][2] contributing elements (-1: none)   (face blocks)
  const int *bj_cf;        // [nblk][2] their local faces
  const int *bj_loc;       // [nblk][2][Nfp] local face node of each block position
  const int *bj_tpos;      // [n_trace] block * (nodes per block) + position of each trace node
};

// Phases timed with HIP events when phase timing is enabled.
enum Phase {
  PH_POINTS = 0, PH_CONTRACT, PH_LU, PH_SOLVE, PH_SCHUR, PH_BACKSOLVE, PH_MATVEC, PH_RHS, PH_CONDENSE,
  PH_CONDENSE_LP, PH_LP_SOLVE, PH_JVP, PH_CONDENSE_LU, PH_CONDENSE_RHS, PH_COUNT
};

// Buffers of the q elimination, per chunk slot: the reduced block (n_r = m N_p,
// padded to nr_pad) in the layout of the condensation, M^-1 and H_j, and the v
// rows of Y and z from the reduced condensation.
struct QElimArgs {
  int nr_pad;
  double *A;    // [chunk][nr_pad][nr_pad]
  double *X;    // [chunk][kx][nr_pad]
  double *C;    // [chunk][nr_pad][k_pad]
  double *D;    // [chunk][k_pad][k_pad]
  double *Rt;   // [chunk][k_pad]
  double *MH;   // [chunk][1 + dim][Np][Np]
  double *Yv;   // [chunk][k][m Np]
  double *zv;   // [chunk][m Np]
};

struct Plan {
  RefTables ref;
  bool timing = false;
  bool fused = true;
  bool split_ok = true;     // separate LU / solve / Schur kernels fit (LDS of the LU panel)
  bool contract_mfma = true;
  hipEvent_t ev[PH_COUNT][2] = {};
  bool ev_pending[PH_COUNT] = {};
  double phase_ms[PH_COUNT] = {};
  long phase_calls[PH_COUNT] = {};
  DevPlan dp{};
  hdg_phys phys{};
  int n_elem = 0, n_trace = 0, chunk = 0;
  // host copies
  std::vector<double> geo_vol, geo_face, node_x, trace_x;
  std::vector<int> tmap, face_bc, node_face;
  std::vector<int> row_drop;  // see DevPlan::row_drop (empty: no row is dropped)
  std::vector<int> bj_nodes, bj_ce, bj_cf, bj_loc, bj_tpos;
  std::vector<int> uinfo;   // see DevPlan::uinfo (empty: the q rows of A are read, not formed)
  // workspace
  void *ws = nullptr;
  size_t ws_bytes = 0;
  size_t off_tables_end = 0;
  bool bound = false;
  bool xcd_clean = false;   // workspace X, C, D hold this plan's structural zeros (one chunk)
  // element-local elimination of q (HDG_FLAG_ELIMINATE_Q): reduced condensation plan and buffers
  bool qelim = false;
  DevPlan rp{};
  QElimArgs qa{};
};

// q elimination (hdg_qelim.hip)
size_t qelim_lds_bytes(const DevPlan &P);
hipError_t launch_qelim(const DevPlan &P, const QElimArgs &Q, int ec, hipStream_t s);
hipError_t launch_qrecover(const DevPlan &P, const QElimArgs &Q, int e0, int ec, double *Y, double *z,
                           hipStream_t s);

// plan helpers shared by the entry-point sources (hdg_plan.cpp)
Plan *checked(hdg_plan *plan);   // null or unbound plan -> nullptr with the error recorded
hipError_t phase_begin(Plan *P, int ph, hipStream_t s);
hipError_t phase_end(Plan *P, int ph, hipStream_t s);
int run_front(Plan *P, const double *v, const double *q, const double *vhat, const double *ustar,
              const double *vbc, int32_t *status, int e0, int ec, hipStream_t s, bool q_only = false);
int check_inputs(const Plan *P, const double *v, const double *q, const double *vhat, const double *ustar,
                 int32_t *status);

// learned block-Jacobi correction (hdg_learn.hip)
int learn_nparams();
int learn_outputs();
hipError_t launch_pool_grad(int nblk, int bs, const double *Binv, const float *o, const double *X, const double *Wv,
                            size_t ld, int nvec, double x2, float *dO, double *loss, hipStream_t s);
hipError_t launch_pool_extract(const DevPlan &P, const double *Binv, const float *feat, const double *X,
                               const double *Wv, int nvec, const int *sel, int nsel, size_t b0, size_t ld,
                               double *pB, float *pfeat, double *pX, double *pW, hipStream_t s);
size_t learn_partial_floats(size_t N);
hipError_t launch_feat(const DevPlan &P, const double *Bd, const void *S, int s_f32, const double *vhat,
                       const int *tpos, double *coup, float *feat, hipStream_t s);
hipError_t launch_mlp_fwd(const float *theta, const float *feat, size_t N, float *out, hipStream_t s);
hipError_t launch_precond_grad(const DevPlan &P, const double *Binv, const float *o, const double *X,
                               const double *Wv, int nvec, double x2, float *dO, double *loss, hipStream_t s);
hipError_t launch_mlp_bwd(const float *theta, const float *feat, const float *dO, size_t N, float *partial,
                          float *grad, hipStream_t s);
hipError_t launch_adam(float *theta, const float *g, float *m, float *v, int t, float lr, hipStream_t s);
size_t learn_noalloc_max_rows();
hipError_t launch_mlp_bwd_noalloc(const float *theta, const float *feat, const float *dO, size_t N, float *grad,
                                  hipStream_t s);
hipError_t launch_scale_blocks(const DevPlan &P, double *B, const float *o, hipStream_t s);

// Raise a kernel's dynamic-LDS limit once (cached per kernel): the attribute
// call is not repeated inside stream capture.
hipError_t set_dyn_lds(const void *kernel, size_t bytes);

// The thread index, read through an empty volatile asm.  The compiler can neither hoist what
// is derived from it out of a loop nor merge two reads: a kernel that re-reads it at the top of
// a long loop body (or in every helper such a loop calls) keeps its index arithmetic inside
// the body, where it is cheap to recompute, instead of holding it live across the loop, where
// it spills to scratch memory.
__device__ __forceinline__ int cur_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// error channel of hdg_last_error(): records the message, returns the code
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *where);

// kernel launchers (hdg_assemble.hip / hdg_dense.hip / hdg_trace.hip)
hipError_t launch_fill_int(int32_t *p, int n, int val, hipStream_t s);
hipError_t launch_fill_double(double *p, size_t n, double val, hipStream_t s);
hipError_t launch_points(const DevPlan &P, int e0, int ec, const double *v, const double *q,
                         const double *vhat, const double *ustar, const double *vbc,
                         int32_t *status, hipStream_t s);
hipError_t launch_contract(const DevPlan &P, int e0, int ec, hipStream_t s);
hipError_t launch_lu(const DevPlan &P, int ec, int32_t *status, hipStream_t s);
size_t lu_lds_bytes(int np);
hipError_t launch_solve(const DevPlan &P, int ec, hipStream_t s);
hipError_t launch_schur(const DevPlan &P, int e0, int ec, double *S, double *g, double *Y,
                        double *z, double *Rloc, double *Rtr, hipStream_t s);
hipError_t launch_copy_resid(const DevPlan &P, int e0, int ec, double *Rloc, double *Rtr, hipStream_t s);
hipError_t launch_mfma_selftest(double *out, hipStream_t s);
int condense_width(int np, bool lp);
size_t condense_lds_bytes(int np, int w);
size_t condense_lds_bytes_lp(int np, int w);
size_t lp_record_bytes(int np);
hipError_t launch_condense_lp(const DevPlan &P, int e0, int ec, int32_t *status, float *S, double *g, float *Y,
                              double *z, float *fac, hipStream_t s);
hipError_t launch_lp_solve(const DevPlan &P, const float *fac, const double *r, double *x, hipStream_t s);
hipError_t launch_jvp(const DevPlan &P, int e0, int ec, const double *dx, const double *dlam, double *yloc,
                      double *ytr, hipStream_t s);
hipError_t launch_trace_matvec_f32(const DevPlan &P, const float *S, const double *x, double *y, hipStream_t s);
hipError_t launch_backsolve_local_f32(const DevPlan &P, const float *Y, const double *a, const double *dvhat,
                                      double *out, hipStream_t s);
hipError_t launch_backsolve_elements(const DevPlan &P, const double *Y, const double *z, const double *dvhat,
                                     double *dx, hipStream_t s);
hipError_t launch_elem_ratio_max(const double *r, const double *b, int E, int n, unsigned long long *out,
                                 double *per, hipStream_t s);
hipError_t launch_fallback_rhs(const DevPlan &P, int e0, int ec, const double *b, hipStream_t s);
hipError_t launch_fallback_take(const DevPlan &P, int e0, int ec, const double *ratio, double tol, double *dx,
                                int *count, hipStream_t s);
hipError_t launch_bj_assemble_f32(const DevPlan &P, const float *S, double *B, hipStream_t s);
size_t condense_inv_doubles(int np);
bool contract_mfma_supported(const DevPlan &P);
hipError_t launch_contract_mfma(const DevPlan &P, int e0, int ec, hipStream_t s);
hipError_t launch_condense(const DevPlan &P, int e0, int ec, int32_t *status, double *S, double *g, double *Y,
                           double *z, hipStream_t s);
// FP64 condensation in two launches (condense_launches == 2): the LU, then the right-hand sides
bool condense_two_launches(const DevPlan &P);
hipError_t launch_condense_lu(const DevPlan &P, int e0, int ec, int32_t *status, hipStream_t s);
bool lu_reg_supported(int np, int nwv);
int default_lu_waves(int np);
size_t lu_reg_lds_bytes(int np, int nwv);
hipError_t launch_condense_rhs(const DevPlan &P, int e0, int ec, double *S, double *g, double *Y, double *z,
                               hipStream_t s);
hipError_t launch_bj_assemble(const DevPlan &P, const double *S, double *B, hipStream_t s);
hipError_t launch_block_invert(const DevPlan &P, double *B, int32_t *bad, hipStream_t s);
hipError_t launch_block_apply(const DevPlan &P, const double *Binv, const double *r, double *z, hipStream_t s);
hipError_t launch_multidot(const double *V, size_t ldv, int nv, const double *w, size_t N, double *partial, int nb,
                           double *out, hipStream_t s);
hipError_t launch_multiaxpy(const double *V, size_t ldv, int nv, const double *h, double *w, size_t N,
                            hipStream_t s);
hipError_t launch_lincomb(const double *V, size_t ldv, int nv, const double *y, double *out, size_t N,
                          hipStream_t s);
hipError_t launch_axpby(double alpha, const double *x, double beta, const double *y, double *out, size_t N,
                        hipStream_t s);
hipError_t launch_scale_by(const double *x, const double *sc, double *out, size_t N, hipStream_t s);
hipError_t launch_export_blocks(const DevPlan &P, int e0, int ec, double *A, double *B, double *C,
                                double *D, double *Rloc, double *Rtr, hipStream_t s);
hipError_t launch_backsolve(const DevPlan &P, const double *Y, const double *z, const double *dvhat,
                            double *dv, double *dq, hipStream_t s);
hipError_t launch_trace_matvec(const DevPlan &P, const double *S, const double *x, double *y,
                               hipStream_t s);
hipError_t launch_trace_rhs(const DevPlan &P, const double *g, double *r, hipStream_t s);
// element L2 products of the DIRK stage combination (hdg_stage.hip)
hipError_t launch_weak_u(const DevPlan &P, const double *v, double *b, hipStream_t s);
hipError_t launch_mass_solve(const DevPlan &P, const double *b, double *u, hipStream_t s);
hipError_t launch_quad_coords(const DevPlan &P, double *xq, hipStream_t s);
hipError_t launch_import_blocks(const DevPlan &P, int e0, int ec, const double *A, const double *B, const double *C,
                                const double *D, const double *Rloc, const double *Rtr, hipStream_t s);
hipError_t launch_l2_error_visc(const DevPlan &P, const double *f, const double *ex, double *out, hipStream_t s);
hipError_t launch_face_quad_coords(const DevPlan &P, double *xf, hipStream_t s);
hipError_t launch_trace_project(const DevPlan &P, const double *g, double *vbc, hipStream_t s);
hipError_t launch_l2_error(const DevPlan &P, int kind, const double *f, const double *ex, double *out,
                           hipStream_t s);
hipError_t launch_drop_rows(const DevPlan &P, int e0, int ec, hipStream_t s);
hipError_t launch_flow_stats(const DevPlan &P, const double *v, double *out, hipStream_t s);
hipError_t launch_gproj(const DevPlan &P, int e0, int ec, const double *v, const double *q, hipStream_t s);
size_t gproj_lift_lds(const DevPlan &P);
hipError_t launch_entropy(const DevPlan &P, const double *v, double *out, hipStream_t s);
hipError_t launch_prepare_state(const DevPlan &P, int N, const double *prim, const double *grad,
                                double *v, double *q, double *u, hipStream_t s);

}  // namespace hdg
