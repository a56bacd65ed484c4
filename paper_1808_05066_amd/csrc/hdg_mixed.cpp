// Mixed-precision Newton linear solve: low-precision condensation, FP64
// matrix-free residuals, outer iterative refinement of the full system
//   J delta = -R,   J = [A B; C D] (element blocks coupled through the traces).
//
// One refinement step with the low-precision factorization (A_lp = L U of the
// scaled FP32 A, Y_lp, S_lp from the same kernel) solves J_lp c = r by static
// condensation:
//   z_hat = A_lp^-1 r_loc;  K_lp c_lambda = r_tr - sum_K P^T C z_hat  (GMRES);
//   c_x = z_hat - Y_lp P c_lambda,
// then delta += c and r = -R - J delta with J applied matrix-free in FP64.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "hdg_plan.hpp"

using namespace hdg;

namespace {

constexpr int NB_RED = 256;

struct RefineLayout {
  size_t rloc, rtr_e, rtr, zh, cl, cx, ytr, R0, solver, partial, scal, total;
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

RefineLayout refine_layout(const Plan *P, size_t solver_bytes) {
  const size_t E = P->n_elem, n = P->dp.n, k = P->dp.k;
  const size_t NT = (size_t)P->dp.m * P->n_trace;
  RefineLayout l{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o = a256(o + b);
    return r;
  };
  l.rloc = take(E * n * 8);
  l.rtr_e = take(E * k * 8);
  l.rtr = take(NT * 8);
  l.zh = take(E * n * 8);
  l.cl = take(NT * 8);
  l.cx = take(E * n * 8);
  l.ytr = take(NT * 8);
  l.R0 = take(NT * 8);
  l.partial = take((size_t)NB_RED * 8);
  l.scal = take(64);
  l.solver = take(solver_bytes);
  l.total = o;
  return l;
}

bool lp_supported(const Plan *P) { return P->dp.cw_lp != 0; }

}  // namespace

extern "C" int hdg_solver_workspace_bytes(const hdg_plan *plan, const hdg_solve_opts *opts, size_t *bytes);
extern "C" int hdg_precond_setup(hdg_plan *plan, const void *S, void *work, size_t bytes, const hdg_solve_opts *opts,
                                 void *stream);
extern "C" int hdg_trace_solve(hdg_plan *plan, const void *S, const double *rhs, double *x, void *work,
                               size_t bytes, const hdg_solve_opts *opts, hdg_solve_info *info, void *stream);

extern "C" int hdg_lp_factor_bytes(const hdg_plan *plan, size_t *bytes) {
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  if (!P || !bytes) return fail(HDG_EINVAL, "bad argument");
  *bytes = (size_t)P->n_elem * lp_record_bytes(P->dp.n_pad);
  return HDG_OK;
}

extern "C" int hdg_assemble_condense_lp(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                                        const double *ustar, const double *vbc, float *S, double *g, float *Y,
                                        double *z, float *factors, double *Rloc, double *Rtr, int32_t *status,
                                        void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  int rc = check_inputs(P, v, q, vhat, ustar, status);
  if (rc) return rc;
  if (!S || !g || !Y || !z || !factors) return fail(HDG_EINVAL, "S, g, Y, z and factors are required");
  if (!lp_supported(P)) return fail(HDG_EUNSUPPORTED, "local block too large for the low-precision kernel");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_fill_int(status, P->n_elem, HDG_OK, s);
  if (e) return hip_fail(e, "status init");
  for (int e0 = 0; e0 < P->n_elem; e0 += P->chunk) {
    const int ec = std::min(P->chunk, P->n_elem - e0);
    rc = run_front(P, v, q, vhat, ustar, vbc, status, e0, ec, s, P->dp.mg != nullptr);
    if (rc) return rc;
    e = launch_copy_resid(P->dp, e0, ec, Rloc, Rtr, s);
    if (!e) e = phase_begin(P, PH_CONDENSE_LP, s);
    if (!e) e = launch_condense_lp(P->dp, e0, ec, status + e0, S, g, Y, z, factors, s);
    if (!e) e = phase_end(P, PH_CONDENSE_LP, s);
    if (e) return hip_fail(e, "condense_lp");
  }
  return HDG_OK;
}

extern "C" int hdg_lp_solve(hdg_plan *plan, const float *factors, const double *r, double *x, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!factors || !r || !x) return fail(HDG_EINVAL, "factors, r and x are required");
  if (r == x) return fail(HDG_EINVAL, "r and x must not alias");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = phase_begin(P, PH_LP_SOLVE, s);
  if (!e) e = launch_lp_solve(P->dp, factors, r, x, s);
  if (!e) e = phase_end(P, PH_LP_SOLVE, s);
  if (e) return hip_fail(e, "lp_solve");
  return HDG_OK;
}

extern "C" int hdg_jacobian_apply(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                                  const double *ustar, const double *vbc, int reuse_points, const double *dx,
                                  const double *dlam, double *y_loc, double *y_tr, int32_t *status, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!dx || !dlam || !y_loc || !y_tr) return fail(HDG_EINVAL, "dx, dlam, y_loc and y_tr are required");
  if (P->dp.ghat_proj) return fail(HDG_EUNSUPPORTED, "the matrix-free Jacobian has no projection viscous flux");
  const bool reuse = reuse_points && P->chunk >= P->n_elem;
  if (!reuse) {
    int rc = check_inputs(P, v, q, vhat, ustar, status);
    if (rc) return rc;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  for (int e0 = 0; e0 < P->n_elem && !e; e0 += P->chunk) {
    const int ec = std::min(P->chunk, P->n_elem - e0);
    if (!reuse) {
      e = phase_begin(P, PH_POINTS, s);
      if (!e) e = launch_points(P->dp, e0, ec, v, q, vhat, ustar, vbc, status, s);
      if (!e) e = phase_end(P, PH_POINTS, s);
    }
    if (!e) e = phase_begin(P, PH_JVP, s);
    if (!e) e = launch_jvp(P->dp, e0, ec, dx, dlam, y_loc, y_tr, s);
    if (!e) e = phase_end(P, PH_JVP, s);
  }
  if (e) return hip_fail(e, "jacobian_apply");
  return HDG_OK;
}

extern "C" int hdg_refine_workspace_bytes(const hdg_plan *plan, const hdg_refine_opts *opts, size_t *bytes) {
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  if (!P || !opts || !bytes) return fail(HDG_EINVAL, "bad argument");
  size_t sb = 0;
  int rc = hdg_solver_workspace_bytes(plan, &opts->gmres, &sb);
  if (rc) return rc;
  *bytes = refine_layout(P, sb).total;
  return HDG_OK;
}

extern "C" int hdg_refine_solve(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                                const double *ustar, const double *vbc, const float *S, const float *Y,
                                const float *factors, const double *Rloc, const double *Rtr, double *dx,
                                double *dlam, void *work, size_t bytes, const hdg_refine_opts *opts,
                                hdg_refine_info *info, int32_t *status, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!S || !Y || !factors || !Rloc || !Rtr || !dx || !dlam || !work || !opts || !info || !status)
    return fail(HDG_EINVAL, "null argument");
  if (opts->max_outer < 1 || !(opts->tol > 0.0)) return fail(HDG_EINVAL, "bad refinement options");
  if (P->dp.ghat_proj) return fail(HDG_EUNSUPPORTED, "the matrix-free Jacobian has no projection viscous flux");
  hdg_solve_opts go = opts->gmres;
  go.s_dtype = HDG_FP32;
  size_t sb = 0;
  int rc = hdg_solver_workspace_bytes(plan, &go, &sb);
  if (rc) return rc;
  const RefineLayout l = refine_layout(P, sb);
  if (bytes < l.total) return fail(HDG_ENOMEM, "refinement workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(work);
  const size_t E = P->n_elem, n = P->dp.n;
  const size_t NL = E * n, NT = (size_t)P->dp.m * P->n_trace;
  double *rloc = reinterpret_cast<double *>(base + l.rloc);
  double *rtr_e = reinterpret_cast<double *>(base + l.rtr_e);
  double *rtr = reinterpret_cast<double *>(base + l.rtr);
  double *zh = reinterpret_cast<double *>(base + l.zh);
  double *cl = reinterpret_cast<double *>(base + l.cl);
  double *cx = reinterpret_cast<double *>(base + l.cx);
  double *ytr = reinterpret_cast<double *>(base + l.ytr);
  double *R0 = reinterpret_cast<double *>(base + l.R0);
  double *partial = reinterpret_cast<double *>(base + l.partial);
  double *dn = reinterpret_cast<double *>(base + l.scal);
  void *swork = base + l.solver;
  const bool reuse = opts->reuse_points != 0;

  auto t0 = std::chrono::steady_clock::now();
  double gmres_ms = 0.0;
  hipError_t e = hipSuccess;
  auto sumsq = [&](const double *x, size_t N, double &out) -> hipError_t {
    hipError_t ee = launch_multidot(x, N, 1, x, N, partial, NB_RED, dn, s);
    double h = 0.0;
    if (!ee) ee = hipMemcpyAsync(&h, dn, 8, hipMemcpyDeviceToHost, s);
    if (!ee) ee = hipStreamSynchronize(s);
    out = h;
    return ee;
  };
  // residual r = -R - J delta  (delta = (dx, dlam)); returns ||r||^2
  auto residual = [&](double &nrm2) -> int {
    int rc2 = hdg_jacobian_apply(plan, v, q, vhat, ustar, vbc, reuse ? 1 : 0, dx, dlam, rloc, rtr_e, status, stream);
    if (rc2) return rc2;
    hipError_t ee = launch_axpby(-1.0, Rloc, -1.0, rloc, rloc, NL, s);
    if (!ee) ee = launch_trace_rhs(P->dp, rtr_e, ytr, s);
    if (!ee) ee = launch_axpby(-1.0, R0, -1.0, ytr, rtr, NT, s);
    double a = 0.0, b = 0.0;
    if (!ee) ee = sumsq(rloc, NL, a);
    if (!ee) ee = sumsq(rtr, NT, b);
    if (ee) return hip_fail(ee, "refine residual");
    nrm2 = a + b;
    return HDG_OK;
  };

  // R0 = sum_K P^T R_tr;  ||R||
  e = launch_trace_rhs(P->dp, Rtr, R0, s);
  double a = 0.0, b = 0.0;
  if (!e) e = sumsq(Rloc, NL, a);
  if (!e) e = sumsq(R0, NT, b);
  if (!e) e = launch_fill_double(dx, NL, 0.0, s);
  if (!e) e = launch_fill_double(dlam, NT, 0.0, s);
  if (!e) e = launch_axpby(-1.0, Rloc, 0.0, nullptr, rloc, NL, s);
  if (!e) e = launch_axpby(-1.0, R0, 0.0, nullptr, rtr, NT, s);
  if (e) return hip_fail(e, "refine init");
  const double Rn = std::sqrt(a + b);
  info->outer_iterations = 0;
  info->gmres_iterations = 0;
  info->fallback_elements = 0;
  info->rel_residual = Rn > 0.0 ? 1.0 : 0.0;
  info->converged = Rn == 0.0 ? 1 : 0;
  for (int i = 0; i < 16; ++i) info->history[i] = 0.0;
  if (Rn == 0.0) return HDG_OK;

  {
    auto g0 = std::chrono::steady_clock::now();
    rc = hdg_precond_setup(plan, S, swork, sb, &go, stream);
    if (rc) return rc;
    gmres_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - g0).count();
  }
  for (int it = 0; it < opts->max_outer; ++it) {
    // low-precision correction
    rc = hdg_lp_solve(plan, factors, rloc, zh, stream);
    if (rc) return rc;
    e = launch_fill_double(cl, NT, 0.0, s);
    if (e) return hip_fail(e, "refine");
    rc = hdg_jacobian_apply(plan, v, q, vhat, ustar, vbc, reuse ? 1 : 0, zh, cl, cx, rtr_e, status, stream);
    if (rc) return rc;
    e = launch_trace_rhs(P->dp, rtr_e, ytr, s);
    if (!e) e = launch_axpby(1.0, rtr, -1.0, ytr, ytr, NT, s);   // ytr = r_tr - sum P^T C z_hat
    if (e) return hip_fail(e, "refine rhs");
    hdg_solve_info gi{};
    auto g0 = std::chrono::steady_clock::now();
    rc = hdg_trace_solve(plan, S, ytr, cl, swork, sb, &go, &gi, stream);
    if (rc) return rc;
    gmres_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - g0).count();
    info->gmres_iterations += gi.iterations;
    e = launch_backsolve_local_f32(P->dp, Y, zh, cl, cx, s);   // c_x = z_hat - Y P c_lambda
    if (!e) e = launch_axpby(1.0, dx, 1.0, cx, dx, NL, s);
    if (!e) e = launch_axpby(1.0, dlam, 1.0, cl, dlam, NT, s);
    if (e) return hip_fail(e, "refine update");
    double nrm2 = 0.0;
    rc = residual(nrm2);
    if (rc) return rc;
    const double rel = std::sqrt(nrm2) / Rn;
    if (it < 16) info->history[it] = rel;
    info->outer_iterations = it + 1;
    info->rel_residual = rel;
    if (rel <= opts->tol) {
      info->converged = 1;
      break;
    }
  }
  info->total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  info->gmres_ms = gmres_ms;
  return HDG_OK;
}

// ---- element-level refinement with a fixed trace update -------------------------------------
namespace {

struct LocalLayout {
  size_t b, r, c, y, ytr, zero, ratio, per, count, total;
};

LocalLayout local_layout(const Plan *P) {
  const size_t E = P->n_elem, n = P->dp.n, k = P->dp.k;
  LocalLayout l{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = a256(o + bytes);
    return r;
  };
  l.b = take(E * n * 8);
  l.r = take(E * n * 8);
  l.c = take(E * n * 8);
  l.y = take(E * n * 8);
  l.ytr = take(E * k * 8);
  l.zero = take(E * n * 8);
  l.ratio = take(64);
  l.per = take(E * 8);
  l.count = take(64);
  l.total = o;
  return l;
}

}  // namespace

extern "C" int hdg_backsolve_elements(hdg_plan *plan, const double *Y, const double *z, const double *dvhat,
                                      double *dx, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!Y || !z || !dvhat || !dx) return fail(HDG_EINVAL, "Y, z, dvhat and dx are required");
  hipError_t e = launch_backsolve_elements(P->dp, Y, z, dvhat, dx, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "backsolve_elements");
  return HDG_OK;
}

extern "C" int hdg_refine_local_workspace_bytes(const hdg_plan *plan, size_t *bytes) {
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  if (!P || !bytes) return fail(HDG_EINVAL, "bad argument");
  *bytes = local_layout(P).total;
  return HDG_OK;
}

extern "C" int hdg_refine_local(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                                const double *ustar, const double *vbc, const float *factors, const double *Rloc,
                                const double *dvhat, double *dx, void *work, size_t bytes, int max_iter, double tol,
                                int reuse_points, hdg_refine_info *info, int32_t *status, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!factors || !Rloc || !dvhat || !dx || !work || !info || !status) return fail(HDG_EINVAL, "null argument");
  if (max_iter < 1 || !(tol > 0.0)) return fail(HDG_EINVAL, "bad refinement options");
  if (P->dp.ghat_proj) return fail(HDG_EUNSUPPORTED, "the matrix-free Jacobian has no projection viscous flux");
  const LocalLayout l = local_layout(P);
  if (bytes < l.total) return fail(HDG_ENOMEM, "local refinement workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(work);
  double *b = reinterpret_cast<double *>(base + l.b);
  double *r = reinterpret_cast<double *>(base + l.r);
  double *c = reinterpret_cast<double *>(base + l.c);
  double *y = reinterpret_cast<double *>(base + l.y);
  double *ytr = reinterpret_cast<double *>(base + l.ytr);
  double *zero = reinterpret_cast<double *>(base + l.zero);
  unsigned long long *ratio = reinterpret_cast<unsigned long long *>(base + l.ratio);
  const size_t E = P->n_elem, n = P->dp.n, NL = E * n;
  const int reuse = reuse_points ? 1 : 0;
  auto t0 = std::chrono::steady_clock::now();
  // b = -(R_loc + B P dvhat)
  hipError_t e = launch_fill_double(zero, NL, 0.0, s);
  if (e) return hip_fail(e, "refine_local init");
  int rc = hdg_jacobian_apply(plan, v, q, vhat, ustar, vbc, reuse, zero, dvhat, y, ytr, status, stream);
  if (rc) return rc;
  e = launch_axpby(-1.0, Rloc, -1.0, y, b, NL, s);
  if (!e) e = launch_fill_double(dx, NL, 0.0, s);
  if (!e) e = launch_axpby(1.0, b, 0.0, nullptr, r, NL, s);
  if (e) return hip_fail(e, "refine_local init");
  info->outer_iterations = 0;
  info->gmres_iterations = 0;
  info->converged = 0;
  info->rel_residual = 1.0;
  info->gmres_ms = 0.0;
  for (int i = 0; i < 16; ++i) info->history[i] = 0.0;
  double* per = reinterpret_cast<double *>(base + l.per);
  int *count = reinterpret_cast<int *>(base + l.count);
  // max_K ||r_K|| / ||b_K|| of the current r (and per element into `per`)
  auto ratio_of = [&](double &rel) -> hipError_t {
    hipError_t ee = launch_fill_double(reinterpret_cast<double *>(ratio), 1, 0.0, s);
    if (!ee) ee = launch_elem_ratio_max(r, b, (int)E, (int)n, ratio, per, s);
    unsigned long long hb = 0;
    if (!ee) ee = hipMemcpyAsync(&hb, ratio, 8, hipMemcpyDeviceToHost, s);
    if (!ee) ee = hipStreamSynchronize(s);
    std::memcpy(&rel, &hb, 8);
    return ee;
  };
  info->fallback_elements = 0;
  double prev = 1.0;
  for (int it = 0; it < max_iter; ++it) {
    rc = hdg_lp_solve(plan, factors, r, c, stream);   // c = A_lp^-1 r
    if (rc) return rc;
    e = launch_axpby(1.0, dx, 1.0, c, dx, NL, s);
    if (e) return hip_fail(e, "refine_local update");
    rc = hdg_jacobian_apply(plan, v, q, vhat, ustar, vbc, 1, dx, dvhat, y, ytr, status, stream);
    if (rc) return rc;
    e = launch_axpby(-1.0, Rloc, -1.0, y, r, NL, s);   // r = -R_loc - (A dx + B P dvhat)
    double rel = 0.0;
    if (!e) e = ratio_of(rel);
    if (e) return hip_fail(e, "refine_local residual");
    if (it < 16) info->history[it] = rel;
    info->outer_iterations = it + 1;
    info->rel_residual = rel;
    if (rel <= tol) {
      info->converged = 1;
      break;
    }
    if (rel > 0.5 * prev) break;   // stagnating: the low-precision factors cannot reach tol
    prev = rel;
  }
  if (!info->converged) {
    // per-element FP64 fallback: the elements still above tol are solved with the FP64 LU of their
    // block (re-assembled in full, right-looking kernels); the others keep the refined dx
    DevPlan Dp = P->dp;
    Dp.mg = nullptr;
    Dp.uinfo = nullptr;
    e = launch_fill_int(count, 1, 0, s);
    if (e) return hip_fail(e, "refine_local fallback");
    for (int e0 = 0; e0 < P->n_elem; e0 += P->chunk) {
      const int ec = std::min(P->chunk, P->n_elem - e0);
      rc = run_front(P, v, q, vhat, ustar, vbc, status, e0, ec, s, false);
      if (rc) return rc;
      P->xcd_clean = false;   // X is overwritten below
      e = launch_fallback_rhs(Dp, e0, ec, b, s);
      if (!e) e = launch_lu(Dp, ec, status + e0, s);
      if (!e) e = launch_solve(Dp, ec, s);
      if (!e) e = launch_fallback_take(Dp, e0, ec, per, tol, dx, count, s);
      if (e) return hip_fail(e, "refine_local fallback");
    }
    int hc = 0;
    e = hipMemcpyAsync(&hc, count, 4, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return hip_fail(e, "refine_local fallback");
    info->fallback_elements = hc;
    rc = hdg_jacobian_apply(plan, v, q, vhat, ustar, vbc, 0, dx, dvhat, y, ytr, status, stream);
    if (rc) return rc;
    e = launch_axpby(-1.0, Rloc, -1.0, y, r, NL, s);
    double rel = 0.0;
    if (!e) e = ratio_of(rel);
    if (e) return hip_fail(e, "refine_local fallback residual");
    info->rel_residual = rel;
    info->converged = rel <= tol ? 1 : 0;
  }
  info->total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return HDG_OK;
}
