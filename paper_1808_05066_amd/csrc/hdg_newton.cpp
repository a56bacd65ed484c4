// Newton iterations on the nonlinear HDG system of one implicit stage (alpha > 0,
// u* given) or of the steady problem (alpha = 0), with the linearization solved by
// static condensation (the local elimination remark after the weak forms of
// Sections 3.3 and 4):
//   assemble and condense every element at the current (v, q, vhat),
//   ||R|| = ||(R_loc, sum_K P_K^T R_tr,K)||_2,
//   K dlambda = sum_K P_K^T g_K   (GMRES, block Jacobi),
//   dx_K = -z_K - Y_K P_K dlambda,
//   v += dv, q += dq, vhat += dlambda.
// Host loop in C++; every step runs in the library's kernels.
#include <chrono>
#include <cmath>

#include "hdg_plan.hpp"

using namespace hdg;

namespace {

constexpr int NB_RED = 256;

struct NewtonLayout {
  size_t S, g, Y, z, rloc, rtr, rasm, rhs, dl, dv, dq, status, partial, scal, solver, total;
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

NewtonLayout newton_layout(const Plan *P, size_t solver_bytes) {
  const DevPlan &D = P->dp;
  const size_t E = P->n_elem, n = D.n, k = D.k, NT = (size_t)D.m * P->n_trace;
  const size_t NN = (size_t)E * D.Np;
  NewtonLayout l{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o = a256(o + b);
    return r;
  };
  l.S = take(E * k * k * 8);
  l.g = take(E * k * 8);
  l.Y = take(E * n * k * 8);
  l.z = take(E * n * 8);
  l.rloc = take(E * n * 8);
  l.rtr = take(E * k * 8);
  l.rasm = take(NT * 8);
  l.rhs = take(NT * 8);
  l.dl = take(NT * 8);
  l.dv = take((size_t)D.m * NN * 8);
  l.dq = take(D.viscous ? (size_t)D.m * D.dim * NN * 8 : 0);
  l.status = take(E * 4);
  l.partial = take((size_t)NB_RED * 8);
  l.scal = take(64);
  l.solver = take(solver_bytes);
  l.total = o;
  return l;
}

bool check_opts(const hdg_newton_opts *o) {
  return o && o->maxit >= 1 && o->tol >= 0.0 && o->atol >= 0.0 && o->lin.s_dtype == HDG_FP64;
}

}  // namespace

extern "C" int hdg_newton_workspace_bytes(const hdg_plan *plan, const hdg_newton_opts *opts, size_t *bytes) {
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  if (!P || !bytes || !check_opts(opts)) return fail(HDG_EINVAL, "bad argument");
  size_t sb = 0;
  int rc = hdg_solver_workspace_bytes(plan, &opts->lin, &sb);
  if (rc) return rc;
  *bytes = newton_layout(P, sb).total;
  return HDG_OK;
}

extern "C" int hdg_newton_solve(hdg_plan *plan, double *v, double *q, double *vhat, const double *u_star,
                                const double *v_bc, void *work, size_t bytes, const hdg_newton_opts *opts,
                                hdg_newton_info *info, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!v || !vhat || !work || !info || !check_opts(opts)) return fail(HDG_EINVAL, "bad argument");
  if (P->dp.viscous && !q) return fail(HDG_EINVAL, "q is required for Navier-Stokes");
  size_t sb = 0;
  int rc = hdg_solver_workspace_bytes(plan, &opts->lin, &sb);
  if (rc) return rc;
  const NewtonLayout l = newton_layout(P, sb);
  if (bytes < l.total) return fail(HDG_ENOMEM, "Newton workspace smaller than hdg_newton_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(HDG_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(work);
  auto ptr = [&](size_t off) { return reinterpret_cast<double *>(base + off); };
  double *S = ptr(l.S), *g = ptr(l.g), *Y = ptr(l.Y), *z = ptr(l.z), *rloc = ptr(l.rloc), *rtr = ptr(l.rtr);
  double *rasm = ptr(l.rasm), *rhs = ptr(l.rhs), *dl = ptr(l.dl), *dv = ptr(l.dv);
  double *dq = P->dp.viscous ? ptr(l.dq) : nullptr;
  int32_t *status = reinterpret_cast<int32_t *>(base + l.status);
  double *partial = ptr(l.partial), *dn = ptr(l.scal);
  void *swork = base + l.solver;
  const size_t E = P->n_elem, NL = E * P->dp.n, NT = (size_t)P->dp.m * P->n_trace;
  const size_t NN = E * P->dp.Np;

  auto sumsq = [&](const double *x, size_t N, double &out) -> hipError_t {
    hipError_t ee = launch_multidot(x, N, 1, x, N, partial, NB_RED, dn, s);
    double h = 0.0;
    if (!ee) ee = hipMemcpyAsync(&h, dn, 8, hipMemcpyDeviceToHost, s);
    if (!ee) ee = hipStreamSynchronize(s);
    out = h;
    return ee;
  };

  const auto t0 = std::chrono::steady_clock::now();
  info->iterations = 0;
  info->converged = 0;
  info->lin_iterations = 0;
  info->lin_converged = 1;
  for (int i = 0; i < HDG_NEWTON_HIST; ++i) info->res[i] = 0.0;
  double r0 = 0.0;
  for (int it = 0;; ++it) {
    rc = hdg_assemble_condense(plan, v, q, vhat, u_star, v_bc, S, g, Y, z, rloc, rtr, status, stream);
    if (rc) return rc;
    int bad = -1, code = HDG_OK;
    rc = hdg_status(plan, status, stream, &bad, &code);
    if (rc) return rc;
    if (bad >= 0) return fail(code, "Newton: an element reported a non-OK status");
    hipError_t e = launch_trace_rhs(P->dp, rtr, rasm, s);
    double a = 0.0, b = 0.0;
    if (!e) e = sumsq(rloc, NL, a);
    if (!e) e = sumsq(rasm, NT, b);
    if (e) return hip_fail(e, "Newton residual");
    const double res = std::sqrt(a + b);
    if (it == 0) r0 = res;
    if (it < HDG_NEWTON_HIST) info->res[it] = res;
    if (res <= opts->atol || res <= opts->tol * r0) {
      info->converged = 1;
      break;
    }
    if (it == opts->maxit) break;
    // condensed system and its solve
    e = launch_trace_rhs(P->dp, g, rhs, s);
    if (e) return hip_fail(e, "Newton trace right-hand side");
    if (opts->lin.precond) {
      rc = hdg_precond_setup(plan, S, swork, sb, &opts->lin, stream);
      if (rc) return rc;
    }
    hdg_solve_info si{};
    rc = hdg_trace_solve(plan, S, rhs, dl, swork, sb, &opts->lin, &si, stream);
    if (rc) return rc;
    info->lin_iterations += si.iterations;
    if (!si.converged) info->lin_converged = 0;
    // local back-solve and update
    rc = hdg_backsolve(plan, Y, z, dl, dv, dq, stream);
    if (rc) return rc;
    e = launch_axpby(1.0, v, 1.0, dv, v, (size_t)P->dp.m * NN, s);
    if (!e && dq) e = launch_axpby(1.0, q, 1.0, dq, q, (size_t)P->dp.m * P->dp.dim * NN, s);
    if (!e) e = launch_axpby(1.0, vhat, 1.0, dl, vhat, NT, s);
    if (e) return hip_fail(e, "Newton update");
    info->iterations = it + 1;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "Newton");
  info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return HDG_OK;
}

// ---- DIRK(3,3) step (Alexander's three-stage, L-stable, stiffly accurate scheme)
//
// Stage i solves  alpha (u(v_i) - u*_i, w) + s(v_i; w) = 0,  alpha = 1/(a_ii dt), with the
// steady residual s and (u*_i, w) = (u_n, w) - dt sum_{j<i} a_ij s(v_j; w).  The converged
// stage j gives s(v_j; w) = -alpha (u(v_j) - u*_j, w), so on the element L2 products
// b(v) = (u(v), phi_a)_K:   b*_i = b(v_n) + sum_{j<i} (a_ij / a_jj) (b(v_j) - b*_j),  and the
// nodal u*_i = M_K^-1 b*_i makes the stage's mass term exact.  The new state is the last
// stage's (stiffly accurate).  The plan's alpha is set to 1/(a_ii dt) and left there.
namespace {

constexpr double DIRK_G = 0.435866521508459;   // a_ii, root of x^3 - 3x^2 + 3x/2 - 1/6 in (1/6, 1/2)

struct DirkLayout {
  size_t bn, bs, d0, d1, us, newton, total;
};

DirkLayout dirk_layout(const Plan *P, size_t newton_bytes) {
  const size_t NM = (size_t)P->dp.m * P->n_elem * P->dp.Np * 8;
  DirkLayout l{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o = a256(o + b);
    return r;
  };
  l.bn = take(NM);
  l.bs = take(NM);
  l.d0 = take(NM);
  l.d1 = take(NM);
  l.us = take(NM);
  l.newton = take(newton_bytes);
  l.total = o;
  return l;
}

}  // namespace

extern "C" int hdg_dirk_workspace_bytes(const hdg_plan *plan, const hdg_newton_opts *opts, size_t *bytes) {
  size_t nb = 0;
  int rc = hdg_newton_workspace_bytes(plan, opts, &nb);
  if (rc) return rc;
  *bytes = dirk_layout(reinterpret_cast<const Plan *>(plan), nb).total;
  return HDG_OK;
}

extern "C" int hdg_dirk_step(hdg_plan *plan, double *v, double *q, double *vhat, const double *v_bc, double dt,
                             void *work, size_t bytes, const hdg_newton_opts *opts, hdg_newton_info *info,
                             void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!v || !vhat || !work || !info || !check_opts(opts) || !(dt > 0.0)) return fail(HDG_EINVAL, "bad argument");
  size_t nb = 0;
  int rc = hdg_newton_workspace_bytes(plan, opts, &nb);
  if (rc) return rc;
  const DirkLayout l = dirk_layout(P, nb);
  if (bytes < l.total) return fail(HDG_ENOMEM, "DIRK workspace smaller than hdg_dirk_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(HDG_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(work);
  auto ptr = [&](size_t off) { return reinterpret_cast<double *>(base + off); };
  double *bn = ptr(l.bn), *bs = ptr(l.bs), *us = ptr(l.us);
  double *d[2] = {ptr(l.d0), ptr(l.d1)};
  const size_t NM = (size_t)P->dp.m * P->n_elem * P->dp.Np;
  const double g = DIRK_G;
  const double a[3][3] = {{g, 0.0, 0.0},
                          {0.5 * (1.0 - g), g, 0.0},
                          {-0.25 * (6.0 * g * g - 16.0 * g + 1.0), 0.25 * (6.0 * g * g - 20.0 * g + 5.0), g}};
  hdg_phys ph = P->phys;
  ph.alpha = 1.0 / (g * dt);
  rc = hdg_plan_set_phys(plan, &ph);
  if (rc) return rc;
  hipError_t e = launch_weak_u(P->dp, v, bn, s);
  if (e) return hip_fail(e, "DIRK stage products");
  for (int i = 0; i < 3; ++i) {
    // b*_i = b_n + sum_{j<i} (a_ij / a_jj) d_j,  d_j = b(v_j) - b*_j
    e = launch_axpby(1.0, bn, 0.0, nullptr, bs, NM, s);
    for (int j = 0; j < i && !e; ++j) e = launch_axpby(1.0, bs, a[i][j] / a[j][j], d[j], bs, NM, s);
    if (!e) e = launch_mass_solve(P->dp, bs, us, s);
    if (e) return hip_fail(e, "DIRK stage state");
    rc = hdg_newton_solve(plan, v, q, vhat, us, v_bc, base + l.newton, nb, opts, info + i, stream);
    if (rc) return rc;
    if (i < 2) {
      e = launch_weak_u(P->dp, v, d[i], s);
      if (!e) e = launch_axpby(1.0, d[i], -1.0, bs, d[i], NM, s);
      if (e) return hip_fail(e, "DIRK stage products");
    }
  }
  e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "DIRK step");
  return HDG_OK;
}
