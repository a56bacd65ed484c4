// Trace-side operations: local back-solve, condensed trace operator, condensed
// right-hand side, and workload state preparation.
//
// Back-solve (local elimination after the global trace update):
//   dx_K = -z_K - Y_K P_K dlambda.
// Condensed operator: y = sum_K P_K^T S_K P_K x, with P_K the gather through the
// trace map (HDG / EDG / IEDG differ only in that map).  Scatter-adds use FP64
// atomics on the [m][n_trace] vector.
#include "hdg_physics.hpp"
#include "hdg_plan.hpp"

namespace hdg {

namespace {

constexpr int BLK = 256;

// one row per thread in a single pass: whole waves covering the rows (at most 1024; more rows loop)
inline int matvec_threads(int k) { return k >= 1024 ? 1024 : ((k + 63) / 64) * 64; }

// gather the element trace vector (k) of a [m][n_trace] field into LDS
__device__ inline void gather_trace(const DevPlan &P, int e, const double *x, double *xl) {
  const int Nfp = P.Nfp, M = P.m, nf = P.nf;
  const int *tm = P.tmap + (size_t)e * nf * Nfp;
  for (int i = threadIdx.x; i < P.k; i += blockDim.x) {
    const int b = i % Nfp, c = (i / Nfp) % M, f = i / (Nfp * M);
    xl[i] = x[(size_t)c * P.n_trace + tm[f * Nfp + b]];
  }
}

__global__ __launch_bounds__(1024) void k_backsolve(DevPlan P, const double *__restrict__ Y,
                                                    const double *__restrict__ z,
                                                    const double *__restrict__ dvhat, double *dv, double *dq) {
  extern __shared__ double xl[];
  const int e = blockIdx.x;
  const int n = P.n, k = P.k, Np = P.Np, M = P.m;
  gather_trace(P, e, dvhat, xl);
  __syncthreads();
  const double *Ye = Y + (size_t)e * n * k;
  const size_t NN = (size_t)P.n_elem * Np;
  for (int row = threadIdx.x; row < n; row += blockDim.x) {
    double acc = -z[(size_t)e * n + row];
    for (int col = 0; col < k; ++col) acc -= Ye[(size_t)col * n + row] * xl[col];
    const int a = row % Np, cs = row / Np;
    if (cs < M) dv[(size_t)cs * NN + (size_t)e * Np + a] = acc;
    else if (dq) dq[(size_t)(cs - M) * NN + (size_t)e * Np + a] = acc;
  }
}

// out[e] = sa a[e] - Y_e P_e dlambda on element-local vectors [E][n] (refinement
// loop of the mixed-precision path with sa = 1; the back-solve dx = -z - Y P dlambda in the
// element-local ordering with sa = -1; Y in FP64 or FP32, arithmetic in FP64).
template <typename T>
__global__ __launch_bounds__(1024) void k_backsolve_local(DevPlan P, const T *__restrict__ Y,
                                                          const double *__restrict__ a,
                                                          const double *__restrict__ dvhat, double *out,
                                                          double sa) {
  extern __shared__ double xl[];
  const int e = blockIdx.x;
  const int n = P.n, k = P.k;
  gather_trace(P, e, dvhat, xl);
  __syncthreads();
  const T *Ye = Y + (size_t)e * n * k;
  for (int row = threadIdx.x; row < n; row += blockDim.x) {
    double acc = sa * a[(size_t)e * n + row];
    for (int col = 0; col < k; ++col) acc -= (double)Ye[(size_t)col * n + row] * xl[col];
    out[(size_t)e * n + row] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_trace_matvec(DevPlan P, const T *__restrict__ S,
                                                        const double *__restrict__ x, double *y) {
  extern __shared__ double xl[];
  const int e = blockIdx.x;
  const int k = P.k, Nfp = P.Nfp, M = P.m, nf = P.nf;
  gather_trace(P, e, x, xl);
  __syncthreads();
  const T *Se = S + (size_t)e * k * k;
  const int *tm = P.tmap + (size_t)e * nf * Nfp;
  for (int row = threadIdx.x; row < k; row += blockDim.x) {
    double acc = 0.0;
    for (int col = 0; col < k; ++col) acc += (double)Se[(size_t)col * k + row] * xl[col];
    const int b = row % Nfp, c = (row / Nfp) % M, f = row / (Nfp * M);
    atomicAdd(&y[(size_t)c * P.n_trace + tm[f * Nfp + b]], acc);
  }
}

__global__ void k_trace_rhs(DevPlan P, const double *__restrict__ g, double *r) {
  const int e = blockIdx.x;
  const int k = P.k, Nfp = P.Nfp, M = P.m, nf = P.nf;
  const int *tm = P.tmap + (size_t)e * nf * Nfp;
  for (int row = threadIdx.x; row < k; row += blockDim.x) {
    const int b = row % Nfp, c = (row / Nfp) % M, f = row / (Nfp * M);
    atomicAdd(&r[(size_t)c * P.n_trace + tm[f * Nfp + b]], g[(size_t)e * k + row]);
  }
}

// v(u(prim)) and the chain-rule gradient q = dv/dprim . grad prim (one forward
// pass per direction), u = conservation variables.  Entropy variables of
// H = -rho s with s = log(p / rho^gamma):
//   v_1 = gamma - s - (gamma-1) rho |V|^2 / (2 p),  v_{1+i} = (gamma-1) rho V_i / p,
//   v_m = -(gamma-1) rho / p.
template <int D, typename T>
__device__ inline void v_of_prim(const T *pr, double gam, T *v) {
  const T rho = pr[0], p = pr[D + 1];
  T kin = cst<T>(0.0);
  for (int i = 0; i < D; ++i) kin = kin + pr[1 + i] * pr[1 + i];
  // log(p / rho^gamma) written with exp/log-free pieces through dpow and the identity
  // s = log(p) - gamma log(rho)
  const T s = dlog(p) - gam * dlog(rho);
  const T rp = rho / p;
  v[0] = gam - s - 0.5 * (gam - 1.0) * rp * kin;
  for (int i = 0; i < D; ++i) v[1 + i] = (gam - 1.0) * rp * pr[1 + i];
  v[D + 1] = -(gam - 1.0) * rp;
}

template <int D>
__global__ void k_prepare(int N, double gam, const double *__restrict__ prim, const double *__restrict__ grad,
                          double *v, double *q, double *u) {
  constexpr int M = D + 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double pr[M];
  for (int c = 0; c < M; ++c) pr[c] = prim[(size_t)c * N + i];
  double vv[M];
  v_of_prim<D, double>(pr, gam, vv);
  for (int c = 0; c < M; ++c) v[(size_t)c * N + i] = vv[c];
  if (q) {
    for (int kd = 0; kd < D; ++kd) {
      Dual pd[M], vd[M];
      for (int c = 0; c < M; ++c) pd[c] = Dual{pr[c], grad[((size_t)c * D + kd) * N + i]};
      v_of_prim<D, Dual>(pd, gam, vd);
      for (int c = 0; c < M; ++c) q[((size_t)c * D + kd) * N + i] = vd[c].d;
    }
  }
  if (u) {
    double kin = 0.0;
    for (int j = 0; j < D; ++j) kin += pr[1 + j] * pr[1 + j];
    u[i] = pr[0];
    for (int j = 0; j < D; ++j) u[(size_t)(1 + j) * N + i] = pr[0] * pr[1 + j];
    u[(size_t)(D + 1) * N + i] = pr[D + 1] / (gam - 1.0) + 0.5 * pr[0] * kin;
  }
}

}  // namespace

hipError_t launch_backsolve(const DevPlan &P, const double *Y, const double *z, const double *dvhat, double *dv,
                            double *dq, hipStream_t s) {
  hipLaunchKernelGGL(k_backsolve, dim3(P.n_elem), dim3(matvec_threads(P.n)), P.k * sizeof(double), s, P, Y, z, dvhat,
                     dv, dq);
  return hipGetLastError();
}

hipError_t launch_trace_matvec(const DevPlan &P, const double *S, const double *x, double *y, hipStream_t s) {
  hipError_t e = launch_fill_double(y, (size_t)P.m * P.n_trace, 0.0, s);
  if (e) return e;
  hipLaunchKernelGGL(k_trace_matvec<double>, dim3(P.n_elem), dim3(matvec_threads(P.k)), P.k * sizeof(double), s, P, S,
                     x, y);
  return hipGetLastError();
}

hipError_t launch_trace_matvec_f32(const DevPlan &P, const float *S, const double *x, double *y, hipStream_t s) {
  hipError_t e = launch_fill_double(y, (size_t)P.m * P.n_trace, 0.0, s);
  if (e) return e;
  hipLaunchKernelGGL(k_trace_matvec<float>, dim3(P.n_elem), dim3(matvec_threads(P.k)), P.k * sizeof(double), s, P, S,
                     x, y);
  return hipGetLastError();
}

hipError_t launch_backsolve_local_f32(const DevPlan &P, const float *Y, const double *a, const double *dvhat,
                                      double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_backsolve_local<float>, dim3(P.n_elem), dim3(matvec_threads(P.n)), P.k * sizeof(double), s, P,
                     Y, a, dvhat, out, 1.0);
  return hipGetLastError();
}

hipError_t launch_backsolve_elements(const DevPlan &P, const double *Y, const double *z, const double *dvhat,
                                     double *dx, hipStream_t s) {
  hipLaunchKernelGGL(k_backsolve_local<double>, dim3(P.n_elem), dim3(matvec_threads(P.n)), P.k * sizeof(double), s,
                     P, Y, z, dvhat, dx, -1.0);
  return hipGetLastError();
}

hipError_t launch_trace_rhs(const DevPlan &P, const double *g, double *r, hipStream_t s) {
  hipError_t e = launch_fill_double(r, (size_t)P.m * P.n_trace, 0.0, s);
  if (e) return e;
  hipLaunchKernelGGL(k_trace_rhs, dim3(P.n_elem), dim3(BLK), 0, s, P, g, r);
  return hipGetLastError();
}

hipError_t launch_prepare_state(const DevPlan &P, int N, const double *prim, const double *grad, double *v,
                                double *q, double *u, hipStream_t s) {
  if (N == 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_prepare<2>, dim3((N + 255) / 256), dim3(256), 0, s, N, P.gamma, prim, grad, v, q, u);
  else
    hipLaunchKernelGGL(k_prepare<3>, dim3((N + 255) / 256), dim3(256), 0, s, N, P.gamma, prim, grad, v, q, u);
  return hipGetLastError();
}

}  // namespace hdg
