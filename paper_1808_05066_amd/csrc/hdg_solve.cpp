// Global trace solve: restarted GMRES with right preconditioning on the
// condensed operator sum_K P_K^T S_K P_K, driven from the host.  Every vector
// operation runs on the device; only the Hessenberg column crosses to the host
// (one synchronization per Arnoldi step).  Arnoldi uses classical Gram-Schmidt
// with one reorthogonalization pass.  The block-Jacobi inverses live at the
// start of the solver workspace, written by hdg_precond_setup.
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "hdg_plan.hpp"

using namespace hdg;

namespace {

constexpr int NB_RED = 256;

struct SolveLayout {
  size_t binv, V, w, z, u, partial, scal, bad, total;
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

SolveLayout solve_layout(const Plan *P, int restart) {
  const size_t N = (size_t)P->dp.m * P->n_trace;
  SolveLayout l{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o = a256(o + b);
    return r;
  };
  l.binv = take((size_t)P->dp.bj_nblk * P->dp.bj_bs * P->dp.bj_bs * 8);
  l.V = take((size_t)(restart + 1) * N * 8);
  l.w = take(N * 8);
  l.z = take(N * 8);
  l.u = take(N * 8);
  l.partial = take((size_t)NB_RED * (restart + 2) * 8);
  l.scal = take((size_t)(3 * (restart + 2) + 8) * 8);
  l.bad = take(64);
  l.total = o;
  return l;
}

}  // namespace

extern "C" int hdg_solver_workspace_bytes(const hdg_plan *plan, const hdg_solve_opts *opts, size_t *bytes) {
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  if (!P || !opts || !bytes || opts->restart < 1) return fail(HDG_EINVAL, "bad argument");
  *bytes = solve_layout(P, opts->restart).total;
  return HDG_OK;
}

extern "C" int hdg_precond_setup(hdg_plan *plan, const void *S, void *work, size_t bytes,
                                 const hdg_solve_opts *opts, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !S || !work || !opts) return fail(HDG_EINVAL, "bad argument or unbound plan");
  if (opts->s_dtype != HDG_FP64 && opts->s_dtype != HDG_FP32) return fail(HDG_EINVAL, "s_dtype must be FP64 or FP32");
  SolveLayout l = solve_layout(P, opts->restart);
  if (bytes < l.total) return fail(HDG_ENOMEM, "solver workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(work);
  double *B = reinterpret_cast<double *>(base + l.binv);
  int32_t *bad = reinterpret_cast<int32_t *>(base + l.bad);
  hipError_t e = launch_fill_int(bad, 1, 0, s);
  if (!e)
    e = opts->s_dtype == HDG_FP32 ? launch_bj_assemble_f32(P->dp, static_cast<const float *>(S), B, s)
                                  : launch_bj_assemble(P->dp, static_cast<const double *>(S), B, s);
  if (!e) e = launch_block_invert(P->dp, B, bad, s);
  int32_t hbad = 0;
  if (!e) e = hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "precond_setup");
  if (hbad) return fail(HDG_ESINGULAR, "singular block-Jacobi block");
  return HDG_OK;
}

extern "C" int hdg_precond_apply(hdg_plan *plan, void *work, size_t bytes, const hdg_solve_opts *opts,
                                 const double *r, double *z, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !work || !opts || !r || !z) return fail(HDG_EINVAL, "bad argument");
  SolveLayout l = solve_layout(P, opts->restart);
  if (bytes < l.total) return fail(HDG_ENOMEM, "solver workspace too small");
  const double *B = reinterpret_cast<const double *>(static_cast<char *>(work) + l.binv);
  hipError_t e = launch_block_apply(P->dp, B, r, z, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "precond_apply");
  return HDG_OK;
}

extern "C" int hdg_trace_solve(hdg_plan *plan, const void *S, const double *rhs, double *x, void *work,
                               size_t bytes, const hdg_solve_opts *opts, hdg_solve_info *info, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !S || !rhs || !x || !work || !opts || !info) return fail(HDG_EINVAL, "bad argument");
  const int m = opts->restart;
  if (m < 1 || opts->maxit < 1 || !(opts->tol > 0.0) || (opts->s_dtype != HDG_FP64 && opts->s_dtype != HDG_FP32))
    return fail(HDG_EINVAL, "bad solver options");
  SolveLayout l = solve_layout(P, m);
  if (bytes < l.total) return fail(HDG_ENOMEM, "solver workspace too small");
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(work);
  const size_t N = (size_t)P->dp.m * P->n_trace;
  const double *B = reinterpret_cast<const double *>(base + l.binv);
  double *V = reinterpret_cast<double *>(base + l.V);
  double *w = reinterpret_cast<double *>(base + l.w);
  double *z = reinterpret_cast<double *>(base + l.z);
  double *u = reinterpret_cast<double *>(base + l.u);
  double *partial = reinterpret_cast<double *>(base + l.partial);
  double *dh = reinterpret_cast<double *>(base + l.scal);
  double *dh2 = dh + (m + 2);
  double *dy = dh2 + (m + 2);
  double *dn = dy + (m + 2);
  const bool pre = opts->precond != 0;
  hipError_t e = hipSuccess;

  auto prec = [&](const double *in, double *out) -> hipError_t {
    if (pre) return launch_block_apply(P->dp, B, in, out, s);
    return hipMemcpyAsync(out, in, N * 8, hipMemcpyDeviceToDevice, s);
  };
  auto matvec = [&](const double *in, double *out) -> hipError_t {
    if (opts->s_dtype == HDG_FP32) return launch_trace_matvec_f32(P->dp, static_cast<const float *>(S), in, out, s);
    return launch_trace_matvec(P->dp, static_cast<const double *>(S), in, out, s);
  };
  auto norm = [&](const double *v, double &out) -> hipError_t {
    hipError_t ee = launch_multidot(v, N, 1, v, N, partial, NB_RED, dn, s);
    double h = 0.0;
    if (!ee) ee = hipMemcpyAsync(&h, dn, 8, hipMemcpyDeviceToHost, s);
    if (!ee) ee = hipStreamSynchronize(s);
    out = std::sqrt(h);
    return ee;
  };

  double bnorm = 0.0;
  e = launch_fill_double(x, N, 0.0, s);
  if (!e) e = norm(rhs, bnorm);
  if (e) return hip_fail(e, "trace_solve");
  info->iterations = 0;
  info->converged = 0;
  info->rel_residual = 0.0;
  info->solve_ms = 0.0;
  if (bnorm == 0.0) {
    info->converged = 1;
    return HDG_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hh(m + 2), hh2(m + 2), y(m);
  int it = 0;
  double relres = 1.0;
  while (it < opts->maxit) {
    // r = rhs - K x  -> V0
    e = matvec(x, w);
    if (!e) e = launch_axpby(1.0, rhs, -1.0, w, V, N, s);
    double beta = 0.0;
    if (!e) e = norm(V, beta);
    if (e) return hip_fail(e, "trace_solve");
    relres = beta / bnorm;
    if (relres <= opts->tol) break;
    e = launch_axpby(1.0 / beta, V, 0.0, nullptr, V, N, s);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double *Vj = V + (size_t)j * N;
      if (!e) e = prec(Vj, z);
      if (!e) e = matvec(z, w);
      if (!e) e = launch_multidot(V, N, j + 1, w, N, partial, NB_RED, dh, s);
      if (!e) e = launch_multiaxpy(V, N, j + 1, dh, w, N, s);
      if (!e) e = launch_multidot(V, N, j + 1, w, N, partial, NB_RED, dh2, s);
      if (!e) e = launch_multiaxpy(V, N, j + 1, dh2, w, N, s);
      if (!e) e = launch_multidot(w, N, 1, w, N, partial, NB_RED, dn, s);
      if (!e) e = hipMemcpyAsync(hh.data(), dh, (j + 1) * 8, hipMemcpyDeviceToHost, s);
      if (!e) e = hipMemcpyAsync(hh2.data(), dh2, (j + 1) * 8, hipMemcpyDeviceToHost, s);
      double nrm2 = 0.0;
      if (!e) e = hipMemcpyAsync(&nrm2, dn, 8, hipMemcpyDeviceToHost, s);
      if (!e) e = hipStreamSynchronize(s);
      if (e) return hip_fail(e, "trace_solve");
      const double hn = std::sqrt(nrm2);
      double *col = &H[(size_t)j * (m + 1)];
      for (int i = 0; i <= j; ++i) col[i] = hh[i] + hh2[i];
      col[j + 1] = hn;
      if (hn > 0.0) e = launch_axpby(1.0 / hn, w, 0.0, nullptr, V + (size_t)(j + 1) * N, N, s);
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
      }
      const double den = std::hypot(col[j], col[j + 1]);
      cs[j] = col[j] / den;
      sn[j] = col[j + 1] / den;
      col[j] = den;
      col[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      jend = j + 1;
      relres = std::fabs(g[j + 1]) / bnorm;
      if (relres <= opts->tol || it >= opts->maxit || hn == 0.0) break;
    }
    // y = H^-1 g (upper triangular), x += M^-1 V y
    for (int i = jend - 1; i >= 0; --i) {
      double acc = g[i];
      for (int k2 = i + 1; k2 < jend; ++k2) acc -= H[(size_t)k2 * (m + 1) + i] * y[k2];
      y[i] = acc / H[(size_t)i * (m + 1) + i];
    }
    if (!e) e = hipMemcpyAsync(dy, y.data(), jend * 8, hipMemcpyHostToDevice, s);
    if (!e) e = launch_lincomb(V, N, jend, dy, u, N, s);
    if (!e) e = prec(u, z);
    if (!e) e = launch_axpby(1.0, x, 1.0, z, x, N, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return hip_fail(e, "trace_solve");
    // the next cycle starts from the true residual, which confirms convergence
  }
  // true residual
  double rn = 0.0;
  e = matvec(x, w);
  if (!e) e = launch_axpby(1.0, rhs, -1.0, w, w, N, s);
  if (!e) e = norm(w, rn);
  if (e) return hip_fail(e, "trace_solve");
  info->iterations = it;
  info->rel_residual = rn / bnorm;
  info->converged = info->rel_residual <= opts->tol ? 1 : 0;
  info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return HDG_OK;
}

// ---- learned block-Jacobi correction ---------------------------------------

extern "C" int hdg_learn_nparams(void) { return learn_nparams(); }

extern "C" int hdg_learn_outputs(void) { return learn_outputs(); }

extern "C" int hdg_learn_extract(hdg_plan *plan, const void *work, size_t bytes, const hdg_solve_opts *opts,
                                 const float *feat, const double *X, const double *Wv, int nvec, const int *sel,
                                 int nsel, size_t b0, size_t ld, double *pool_B, float *pool_feat, double *pool_X,
                                 double *pool_W, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !work || !opts || !feat || !X || !Wv || nvec < 1 || !sel || nsel < 1 || !pool_B ||
      !pool_feat || !pool_X || !pool_W)
    return fail(HDG_EINVAL, "bad argument");
  if ((b0 + (size_t)nsel) * P->dp.bj_bs > ld) return fail(HDG_EINVAL, "pool rows (ld) too small for b0 + nsel blocks");
  SolveLayout l = solve_layout(P, opts->restart);
  if (bytes < l.total) return fail(HDG_ENOMEM, "solver workspace too small");
  const double *B = reinterpret_cast<const double *>(static_cast<const char *>(work) + l.binv);
  hipError_t e = launch_pool_extract(P->dp, B, feat, X, Wv, nvec, sel, nsel, b0, ld, pool_B, pool_feat, pool_X,
                                     pool_W, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "learn_extract");
  return HDG_OK;
}

extern "C" int hdg_learn_forward_rows(const float *theta, const float *feat, size_t N, float *out, void *stream) {
  if (!theta || !feat || !out || N == 0) return fail(HDG_EINVAL, "bad argument");
  hipError_t e = launch_mlp_fwd(theta, feat, N, out, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "learn_forward_rows");
  return HDG_OK;
}

extern "C" int hdg_learn_rows_scratch_floats(size_t N, size_t *n) {
  if (!n) return fail(HDG_EINVAL, "bad argument");
  *n = learn_partial_floats(N);
  return HDG_OK;
}

extern "C" int hdg_learn_backward_rows(const float *theta, const float *feat, const float *dO, size_t N, float *grad,
                                       float *scratch, void *stream) {
  if (!theta || !feat || !dO || !grad || !scratch || N == 0) return fail(HDG_EINVAL, "bad argument");
  hipError_t e = launch_mlp_bwd(theta, feat, dO, N, scratch, grad, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "learn_backward_rows");
  return HDG_OK;
}

extern "C" int hdg_learn_pool_loss_grad(int nblk, int bs, const double *pool_B, const float *out, const double *X,
                                        const double *Wv, size_t ld, int nvec, double x2, float *dO, double *loss,
                                        void *stream) {
  if (nblk < 1 || bs < 1 || bs > 256 || !pool_B || !out || !X || !Wv || nvec < 1 || !(x2 > 0.0) || !dO || !loss ||
      ld < (size_t)nblk * bs)
    return fail(HDG_EINVAL, "bad argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_fill_double(loss, 1, 0.0, s);
  if (!e) e = launch_pool_grad(nblk, bs, pool_B, out, X, Wv, ld, nvec, x2, dO, loss, s);
  if (e) return hip_fail(e, "learn_pool_loss_grad");
  return HDG_OK;
}

extern "C" int hdg_learn_setup(hdg_plan *plan, const void *S, const double *vhat, float *feat, void *work,
                               size_t bytes, const hdg_solve_opts *opts, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !S || !vhat || !feat || !work || !opts) return fail(HDG_EINVAL, "bad argument");
  if (opts->s_dtype != HDG_FP64 && opts->s_dtype != HDG_FP32) return fail(HDG_EINVAL, "s_dtype must be FP64 or FP32");
  SolveLayout l = solve_layout(P, opts->restart);
  if (bytes < l.total) return fail(HDG_ENOMEM, "solver workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(work);
  double *B = reinterpret_cast<double *>(base + l.binv);
  double *coup = reinterpret_cast<double *>(base + l.V);   // Krylov space reused as scratch
  int32_t *bad = reinterpret_cast<int32_t *>(base + l.bad);
  const bool f32 = opts->s_dtype == HDG_FP32;
  hipError_t e = launch_fill_int(bad, 1, 0, s);
  if (!e)
    e = f32 ? launch_bj_assemble_f32(P->dp, static_cast<const float *>(S), B, s)
            : launch_bj_assemble(P->dp, static_cast<const double *>(S), B, s);
  if (!e) e = launch_feat(P->dp, B, S, f32 ? 1 : 0, vhat, P->dp.bj_tpos, coup, feat, s);
  if (!e) e = launch_block_invert(P->dp, B, bad, s);
  int32_t hbad = 0;
  if (!e) e = hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "learn_setup");
  if (hbad) return fail(HDG_ESINGULAR, "singular block-Jacobi block");
  return HDG_OK;
}

extern "C" int hdg_learn_forward(hdg_plan *plan, const float *theta, const float *feat, float *out, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !theta || !feat || !out) return fail(HDG_EINVAL, "bad argument");
  const size_t N = (size_t)P->dp.bj_nblk * P->dp.bj_bs;
  hipError_t e = launch_mlp_fwd(theta, feat, N, out, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "learn_forward");
  return HDG_OK;
}

extern "C" int hdg_learn_apply(hdg_plan *plan, const float *out, void *work, size_t bytes,
                               const hdg_solve_opts *opts, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !out || !work || !opts) return fail(HDG_EINVAL, "bad argument");
  SolveLayout l = solve_layout(P, opts->restart);
  if (bytes < l.total) return fail(HDG_ENOMEM, "solver workspace too small");
  double *B = reinterpret_cast<double *>(static_cast<char *>(work) + l.binv);
  hipError_t e = launch_scale_blocks(P->dp, B, out, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "learn_apply");
  return HDG_OK;
}

extern "C" int hdg_learn_loss_grad(hdg_plan *plan, const void *work, size_t bytes, const hdg_solve_opts *opts,
                                   const float *out, const double *X, const double *Wv, int nvec, double x2,
                                   float *dO, double *loss, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !work || !opts || !out || !X || !Wv || !dO || !loss || nvec < 1 || !(x2 > 0.0))
    return fail(HDG_EINVAL, "bad argument");
  SolveLayout l = solve_layout(P, opts->restart);
  if (bytes < l.total) return fail(HDG_ENOMEM, "solver workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const double *B = reinterpret_cast<const double *>(static_cast<const char *>(work) + l.binv);
  hipError_t e = launch_fill_double(loss, 1, 0.0, s);
  if (!e) e = launch_precond_grad(P->dp, B, out, X, Wv, nvec, x2, dO, loss, s);
  if (e) return hip_fail(e, "learn_loss_grad");
  return HDG_OK;
}

extern "C" int hdg_learn_scratch_floats(const hdg_plan *plan, size_t *n) {
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  if (!P || !n) return fail(HDG_EINVAL, "bad argument");
  *n = learn_partial_floats((size_t)P->dp.bj_nblk * P->dp.bj_bs);
  return HDG_OK;
}

extern "C" int hdg_learn_backward(hdg_plan *plan, const float *theta, const float *feat, const float *dO,
                                  float *grad, float *scratch, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !theta || !feat || !dO || !grad || !scratch) return fail(HDG_EINVAL, "bad argument");
  const size_t N = (size_t)P->dp.bj_nblk * P->dp.bj_bs;
  hipError_t e = launch_mlp_bwd(theta, feat, dO, N, scratch, grad, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "learn_backward");
  return HDG_OK;
}

extern "C" int hdg_learn_backward_noalloc(hdg_plan *plan, const float *theta, const float *feat, const float *dO,
                                          float *grad, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !P->bound || !theta || !feat || !dO || !grad) return fail(HDG_EINVAL, "bad argument");
  const size_t N = (size_t)P->dp.bj_nblk * P->dp.bj_bs;
  if (N > learn_noalloc_max_rows())
    return fail(HDG_EINVAL, "hdg_learn_backward_noalloc: " + std::to_string(N) + " rows exceed the static scratch (" +
                                std::to_string(learn_noalloc_max_rows()) + " rows); use hdg_learn_backward");
  hipError_t e = launch_mlp_bwd_noalloc(theta, feat, dO, N, grad, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "learn_backward_noalloc");
  return HDG_OK;
}

extern "C" int hdg_learn_adam(float *theta, const float *grad, float *m, float *v, int t, float lr, void *stream) {
  if (!theta || !grad || !m || !v || t < 1) return fail(HDG_EINVAL, "bad argument");
  hipError_t e = launch_adam(theta, grad, m, v, t, lr, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "learn_adam");
  return HDG_OK;
}

extern "C" int hdg_learn_train_step(hdg_plan *plan, float *theta, float *m, float *v, int t, float lr,
                                    const float *feat, const void *work, size_t bytes, const hdg_solve_opts *opts,
                                    const double *X, const double *Wv, int nvec, double x2, float *out, float *dO,
                                    float *grad, float *scratch, double *loss, void *stream) {
  int rc = hdg_learn_forward(plan, theta, feat, out, stream);
  if (!rc) rc = hdg_learn_loss_grad(plan, work, bytes, opts, out, X, Wv, nvec, x2, dO, loss, stream);
  if (!rc) rc = hdg_learn_backward(plan, theta, feat, dO, grad, scratch, stream);
  if (!rc) rc = hdg_learn_adam(theta, grad, m, v, t, lr, stream);
  return rc;
}
