// Element L2 products for the stage combination of a DIRK step, quadrature-point
// coordinates and element L2 errors against values at the quadrature points:
//   b_K = (u(v_h), phi_a)_K        (weak form of the conserved state, quadrature)
//   u*  = M_K^-1 b_K               (the nodal state whose L2 products are b_K)
// so that the mass term alpha (u(v) - u*, w) of a stage sees exactly the
// combination of previous stages formed on the b vectors.  Layouts: v, b, u
// [m][E*Np] (structure of arrays, element-major nodes).
#include "hdg_physics.hpp"
#include "hdg_plan.hpp"

namespace hdg {

namespace {

constexpr int SB = 128;

// b[c][e Np + a] = sum_q W_q u_c(v(x_q)) phi_a(x_q)
template <int D>
__global__ __launch_bounds__(SB) void k_weak_u(DevPlan P, const double *__restrict__ v, double *b) {
  constexpr int M = D + 2;
  extern __shared__ double sm[];
  const int e = blockIdx.x, tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq;
  const size_t NN = (size_t)P.n_elem * Np;
  double *vs = sm;              // [M][Np]
  double *uq = vs + M * Np;     // [Nq][M] W_q u(v(x_q))
  for (int t = tid; t < M * Np; t += SB) vs[t] = v[(size_t)(t / Np) * NN + (size_t)e * Np + t % Np];
  __syncthreads();
  const int gs = 1 + D * D;
  for (int q = tid; q < Nq; q += SB) {
    double vq[M];
    for (int c = 0; c < M; ++c) {
      double acc = 0.0;
      for (int a = 0; a < Np; ++a) acc += P.phi[(size_t)q * Np + a] * vs[c * Np + a];
      vq[c] = acc;
    }
    const Prim<D, double> s = prim_of_v<D, double>(vq, P.gamma);
    double u[M];
    u_of_prim<D, double>(s, P.gamma, u);
    const double W = P.geo_vol[((size_t)e * Nq + q) * gs];
    for (int c = 0; c < M; ++c) uq[q * M + c] = W * u[c];
  }
  __syncthreads();
  for (int t = tid; t < M * Np; t += SB) {
    const int c = t / Np, a = t % Np;
    double acc = 0.0;
    for (int q = 0; q < Nq; ++q) acc += uq[q * M + c] * P.phi[(size_t)q * Np + a];
    b[(size_t)c * NN + (size_t)e * Np + a] = acc;
  }
}

// u[c][e Np + :] = M_K^-1 b[c][e Np + :],  M_K[a][a'] = sum_q W_q phi_a phi_a'
// (Cholesky in LDS: M_K is symmetric positive definite)
template <int D>
__global__ __launch_bounds__(SB) void k_mass_solve(DevPlan P, const double *__restrict__ b, double *u) {
  constexpr int M = D + 2;
  extern __shared__ double sm[];
  const int e = blockIdx.x, tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq;
  const size_t NN = (size_t)P.n_elem * Np;
  double *L = sm;              // [Np][Np], lower triangle
  double *x = L + Np * Np;     // [M][Np]
  double *W = x + M * Np;      // [Nq]
  const int gs = 1 + D * D;
  for (int q = tid; q < Nq; q += SB) W[q] = P.geo_vol[((size_t)e * Nq + q) * gs];
  for (int t = tid; t < M * Np; t += SB) x[t] = b[(size_t)(t / Np) * NN + (size_t)e * Np + t % Np];
  __syncthreads();
  for (int t = tid; t < Np * Np; t += SB) {
    const int i = t / Np, j = t % Np;
    double acc = 0.0;
    if (j <= i)
      for (int q = 0; q < Nq; ++q) acc += W[q] * P.phi[(size_t)q * Np + i] * P.phi[(size_t)q * Np + j];
    L[t] = acc;
  }
  __syncthreads();
  // right-looking Cholesky, column k per pass
  for (int k = 0; k < Np; ++k) {
    if (tid == 0) L[k * Np + k] = sqrt(L[k * Np + k]);
    __syncthreads();
    const double d = L[k * Np + k];
    for (int i = k + 1 + tid; i < Np; i += SB) L[i * Np + k] /= d;
    __syncthreads();
    for (int t = tid; t < (Np - k - 1) * (Np - k - 1); t += SB) {
      const int i = k + 1 + t / (Np - k - 1), j = k + 1 + t % (Np - k - 1);
      if (j <= i) L[i * Np + j] -= L[i * Np + k] * L[j * Np + k];
    }
    __syncthreads();
  }
  // L L^T x = b for the M components, one thread per component
  for (int c = tid; c < M; c += SB) {
    double *xc = x + c * Np;
    for (int i = 0; i < Np; ++i) {
      double s = xc[i];
      for (int j = 0; j < i; ++j) s -= L[i * Np + j] * xc[j];
      xc[i] = s / L[i * Np + i];
    }
    for (int i = Np - 1; i >= 0; --i) {
      double s = xc[i];
      for (int j = i + 1; j < Np; ++j) s -= L[j * Np + i] * xc[j];
      xc[i] = s / L[i * Np + i];
    }
  }
  __syncthreads();
  for (int t = tid; t < M * Np; t += SB) u[(size_t)(t / Np) * NN + (size_t)e * Np + t % Np] = x[t];
}

// x_q = sum_a phi_a(x_q) x_a (exact for straight-sided simplices and multilinear quads/hexes)
__global__ void k_quad_coords(DevPlan P, double *xq) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t NQ = (size_t)P.n_elem * P.Nq, NN = (size_t)P.n_elem * P.Np;
  if (t >= NQ) return;
  const int e = (int)(t / P.Nq), q = (int)(t % P.Nq);
  for (int d = 0; d < P.dim; ++d) {
    double acc = 0.0;
    for (int a = 0; a < P.Np; ++a) acc += P.phi[(size_t)q * P.Np + a] * P.node_x[(size_t)d * NN + (size_t)e * P.Np + a];
    xq[(size_t)d * NQ + t] = acc;
  }
}

// out[e][c] = sum_q W_q (f_c(x_q) - ex[c][e Nq + q])^2 with f_c = u_c(v_h) (kind 0, f = v),
// the interpolated gradient unknowns (kind 1, f = q) or the interpolated entropy variables
// (kind 2, f = v)
template <int D>
__global__ __launch_bounds__(64) void k_l2_error(DevPlan P, int kind, const double *__restrict__ f,
                                                 const double *__restrict__ ex, double *out) {
  constexpr int M = D + 2, NC = M * D;
  __shared__ double red[64][NC];
  const int e = blockIdx.x, tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq, nc = kind == 1 ? NC : M;
  const size_t NN = (size_t)P.n_elem * Np, NQ = (size_t)P.n_elem * Nq;
  double acc[NC];
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  for (int q = tid; q < Nq; q += 64) {
    const double *phi = P.phi + (size_t)q * Np;
    double val[NC];
    for (int c = 0; c < nc; ++c) {
      double s = 0.0;
      for (int a = 0; a < Np; ++a) s += phi[a] * f[(size_t)c * NN + (size_t)e * Np + a];
      val[c] = s;
    }
    if (kind == 0) {
      const Prim<D, double> st = prim_of_v<D, double>(val, P.gamma);
      u_of_prim<D, double>(st, P.gamma, val);
    }
    const double W = P.geo_vol[((size_t)e * Nq + q) * (1 + D * D)];
    for (int c = 0; c < nc; ++c) {
      const double d = val[c] - ex[(size_t)c * NQ + (size_t)e * Nq + q];
      acc[c] += W * d * d;
    }
  }
  for (int c = 0; c < nc; ++c) red[tid][c] = acc[c];
  __syncthreads();
  if (tid < nc) {
    double s = 0.0;
    for (int t = 0; t < 64; ++t) s += red[t][tid];
    out[(size_t)e * nc + tid] = s;
  }
}

// Viscous stress tau[i][j] and heat flux f[j] of the state with entropy variables v[M] and
// gradient unknowns q[c D + k] (G = -(0, tau, V.tau - f) of the viscous flux), into out[D D + D].
template <int D>
__device__ inline void stress_heat(const double *v, const double *q, const DevPlan &P, double *out) {
  constexpr int M = D + 2;
  const Prim<D, double> st = prim_of_v<D, double>(v, P.gamma);
  double G[M * D];
  flux_G<D, double, double>(st, q, P.gamma, P.mu, P.Pr, G);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) out[i * D + j] = -G[(1 + i) * D + j];
  for (int j = 0; j < D; ++j) {
    double vt = 0.0;
    for (int i = 0; i < D; ++i) vt += st.V[i] * out[i * D + j];
    out[D * D + j] = G[(D + 1) * D + j] + vt;
  }
}

// out[e][c] = sum_q W_q (s_c(v_h, q_h)(x_q) - s_c(v, q)(x_q))^2 for the stress and heat flux s of
// the viscous flux: f = [v; q] stacked [(M + M D)][E*Np] (nodal, interpolated), ex the same
// stacked [(M + M D)][E*Nq] at the volume quadrature points; c < D D + D
template <int D>
__global__ __launch_bounds__(64) void k_l2_error_visc(DevPlan P, const double *__restrict__ f,
                                                      const double *__restrict__ ex, double *out) {
  constexpr int M = D + 2, NV = M + M * D, NS = D * D + D;
  __shared__ double red[64][NS];
  const int e = blockIdx.x, tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq;
  const size_t NN = (size_t)P.n_elem * Np, NQ = (size_t)P.n_elem * Nq;
  double acc[NS];
  for (int c = 0; c < NS; ++c) acc[c] = 0.0;
  for (int q = tid; q < Nq; q += 64) {
    const double *phi = P.phi + (size_t)q * Np;
    double h[NV], x[NV];
    for (int c = 0; c < NV; ++c) {
      double s = 0.0;
      for (int a = 0; a < Np; ++a) s += phi[a] * f[(size_t)c * NN + (size_t)e * Np + a];
      h[c] = s;
      x[c] = ex[(size_t)c * NQ + (size_t)e * Nq + q];
    }
    double sh[NS], sx[NS];
    stress_heat<D>(h, h + M, P, sh);
    stress_heat<D>(x, x + M, P, sx);
    const double W = P.geo_vol[((size_t)e * Nq + q) * (1 + D * D)];
    for (int c = 0; c < NS; ++c) acc[c] += W * (sh[c] - sx[c]) * (sh[c] - sx[c]);
  }
  for (int c = 0; c < NS; ++c) red[tid][c] = acc[c];
  __syncthreads();
  if (tid < NS) {
    double s = 0.0;
    for (int t = 0; t < 64; ++t) s += red[t][tid];
    out[(size_t)e * NS + tid] = s;
  }
}

// Physical coordinates of the face quadrature points, xf[c][(e nf + f) Nfq + q] =
// sum_b psi_b(x_q) x_c(face node b): the face's image under the element map (affine and
// multilinear faces are reproduced by the face-node interpolant)
__global__ void k_face_quad_coords(DevPlan P, double *xf) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t NF = (size_t)P.n_elem * P.nf * P.Nfq, NN = (size_t)P.n_elem * P.Np;
  if (t >= NF) return;
  const int q = (int)(t % P.Nfq);
  const size_t ef = t / P.Nfq;
  const int f = (int)(ef % P.nf), e = (int)(ef / P.nf);
  const double *psi = P.fphi + ((size_t)f * P.Nfq + q) * P.Nfp;
  for (int d = 0; d < P.dim; ++d) {
    double acc = 0.0;
    for (int b = 0; b < P.Nfp; ++b)
      acc += psi[b] * P.node_x[(size_t)d * NN + (size_t)e * P.Np + P.fnodes[f * P.Nfp + b]];
    xf[(size_t)d * NF + t] = acc;
  }
}

// Face L2 projection of Dirichlet data: for every Dirichlet-trace face, M_F c = <g, mu>_F with
// M_F[b][b'] = sum_q W_q psi_b psi_b' and g given at the face quadrature points,
// g[c][(e nf + f) Nfq + q]; c (Nfp x m) written to the face's trace nodes of vbc [m][n_trace].
// One 64-thread workgroup per element face; Gauss-Jordan on the SPD face mass matrix in LDS.
constexpr int PJ_NFP = 25;   // face nodes of a p = 4 quadrilateral face
__global__ __launch_bounds__(64) void k_trace_project(DevPlan P, const double *__restrict__ g, double *vbc) {
  __shared__ double Mf[PJ_NFP][PJ_NFP];
  __shared__ double R[PJ_NFP][8];
  const int ef = blockIdx.x, tid = threadIdx.x;
  if (P.face_bc[ef] != 1) return;   // whole workgroup
  const int f = ef % P.nf, m = P.m, Nfp = P.Nfp, Nfq = P.Nfq;
  const size_t NF = (size_t)P.n_elem * P.nf * Nfq;
  const double *psi = P.fphi + (size_t)f * Nfq * Nfp;
  const double *gf = P.geo_face + (size_t)ef * Nfq * (1 + P.dim);
  for (int t = tid; t < Nfp * Nfp; t += 64) {
    const int b = t / Nfp, c = t % Nfp;
    double s = 0.0;
    for (int q = 0; q < Nfq; ++q) s += gf[(size_t)q * (1 + P.dim)] * psi[q * Nfp + b] * psi[q * Nfp + c];
    Mf[b][c] = s;
  }
  for (int t = tid; t < Nfp * m; t += 64) {
    const int b = t / m, c = t % m;
    double s = 0.0;
    for (int q = 0; q < Nfq; ++q)
      s += gf[(size_t)q * (1 + P.dim)] * psi[q * Nfp + b] * g[(size_t)c * NF + (size_t)ef * Nfq + q];
    R[b][c] = s;
  }
  __syncthreads();
  for (int i = 0; i < Nfp; ++i) {
    const double inv = 1.0 / Mf[i][i];
    __syncthreads();
    // rows other than i: subtract their multiple of row i (row i itself is scaled after)
    for (int t = tid; t < Nfp * (Nfp + m); t += 64) {
      const int r = t / (Nfp + m), c = t % (Nfp + m);
      if (r == i) continue;
      const double l = Mf[r][i] * inv;
      if (c < Nfp) {
        if (c != i) Mf[r][c] -= l * Mf[i][c];
      } else {
        R[r][c - Nfp] -= l * R[i][c - Nfp];
      }
    }
    __syncthreads();
    for (int r = tid; r < Nfp; r += 64)
      if (r != i) Mf[r][i] = 0.0;
    __syncthreads();
  }
  for (int t = tid; t < Nfp * m; t += 64) {
    const int b = t / m, c = t % m;
    vbc[(size_t)c * P.n_trace + P.tmap[(size_t)ef * Nfp + b]] = R[b][c] / Mf[b][b];
  }
}

// out[e] = (sum_q W_q rho s, sum_q W_q rho) at the states v_h(x_q), s = ln(p / rho^gamma):
// the element's total thermodynamic entropy (minus the generalized entropy H = -rho s of the
// entropy-variable section) and its mass
template <int D>
__global__ __launch_bounds__(64) void k_entropy(DevPlan P, const double *__restrict__ v, double *out) {
  constexpr int M = D + 2;
  __shared__ double red[2][64];
  const int e = blockIdx.x, tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq;
  const size_t NN = (size_t)P.n_elem * Np;
  double rs = 0.0, rm = 0.0;
  for (int q = tid; q < Nq; q += 64) {
    const double *phi = P.phi + (size_t)q * Np;
    double val[M];
    for (int c = 0; c < M; ++c) {
      double s = 0.0;
      for (int a = 0; a < Np; ++a) s += phi[a] * v[(size_t)c * NN + (size_t)e * Np + a];
      val[c] = s;
    }
    const Prim<D, double> st = prim_of_v<D, double>(val, P.gamma);
    const double W = P.geo_vol[((size_t)e * Nq + q) * (1 + D * D)];
    rs += W * st.rho * (log(st.p) - P.gamma * log(st.rho));
    rm += W * st.rho;
  }
  red[0][tid] = rs;
  red[1][tid] = rm;
  __syncthreads();
  if (tid < 2) {
    double s = 0.0;
    for (int t = 0; t < 64; ++t) s += red[tid][t];
    out[(size_t)e * 2 + tid] = s;
  }
}

// Element integrals of the flow statistics of the Taylor-Green example (Section 5) at the
// states u(v_h) and velocity gradients of v_h by the volume quadrature:
//   out[e] = (rho s, rho, rho |V|^2 / 2, |omega|^2, theta, theta^2, T, T^2),
// s = ln(p / rho^gamma), omega = curl V (scalar in 2D), theta = div V, T = p / rho (the
// temperature up to the gas constant).  V = -w / v_m with w = v_2..v_{d+1}, so
// dV_i = -(dw_i + V_i dv_m) / v_m.
template <int D>
__global__ __launch_bounds__(64) void k_flow_stats(DevPlan P, const double *__restrict__ v, double *out) {
  constexpr int M = D + 2, NS = 8;
  __shared__ double red[NS][64];
  const int e = blockIdx.x, tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq;
  const size_t NN = (size_t)P.n_elem * Np;
  double acc[NS];
  for (int i = 0; i < NS; ++i) acc[i] = 0.0;
  for (int q = tid; q < Nq; q += 64) {
    const double *phi = P.phi + (size_t)q * Np;
    const double *g = P.geo_vol + ((size_t)e * Nq + q) * (1 + D * D);
    double val[M], gr[M][D];
    for (int c = 0; c < M; ++c) {
      double s = 0.0, dr[D];
      for (int r = 0; r < D; ++r) dr[r] = 0.0;
      const double *vc = v + (size_t)c * NN + (size_t)e * Np;
      for (int a = 0; a < Np; ++a) {
        const double va = vc[a];
        s += phi[a] * va;
        for (int r = 0; r < D; ++r) dr[r] += P.dphi[((size_t)r * Nq + q) * Np + a] * va;
      }
      val[c] = s;
      for (int j = 0; j < D; ++j) {
        double t = 0.0;
        for (int r = 0; r < D; ++r) t += dr[r] * g[1 + r * D + j];
        gr[c][j] = t;
      }
    }
    const Prim<D, double> st = prim_of_v<D, double>(val, P.gamma);
    const double vm = val[M - 1];
    double dV[D][D];   // dV[i][j] = dV_i / dx_j
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) dV[i][j] = -(gr[1 + i][j] + st.V[i] * gr[M - 1][j]) / vm;
    double ke = 0.0, th = 0.0, om2 = 0.0;
    for (int i = 0; i < D; ++i) {
      ke += st.V[i] * st.V[i];
      th += dV[i][i];
    }
    if constexpr (D == 2) {
      const double w3 = dV[1][0] - dV[0][1];
      om2 = w3 * w3;
    } else {
      const double w1 = dV[2][1] - dV[1][2], w2 = dV[0][2] - dV[2][0], w3 = dV[1][0] - dV[0][1];
      om2 = w1 * w1 + w2 * w2 + w3 * w3;
    }
    const double W = g[0], T = st.p / st.rho;
    acc[0] += W * st.rho * (log(st.p) - P.gamma * log(st.rho));
    acc[1] += W * st.rho;
    acc[2] += W * 0.5 * st.rho * ke;
    acc[3] += W * om2;
    acc[4] += W * th;
    acc[5] += W * th * th;
    acc[6] += W * T;
    acc[7] += W * T * T;
  }
  for (int i = 0; i < NS; ++i) red[i][tid] = acc[i];
  __syncthreads();
  if (tid < NS) {
    double s = 0.0;
    for (int t = 0; t < 64; ++t) s += red[tid][t];
    out[(size_t)e * NS + tid] = s;
  }
}

}  // namespace

hipError_t launch_flow_stats(const DevPlan &P, const double *v, double *out, hipStream_t s) {
  if (P.dim == 2)
    hipLaunchKernelGGL(k_flow_stats<2>, dim3(P.n_elem), dim3(64), 0, s, P, v, out);
  else
    hipLaunchKernelGGL(k_flow_stats<3>, dim3(P.n_elem), dim3(64), 0, s, P, v, out);
  return hipGetLastError();
}

hipError_t launch_entropy(const DevPlan &P, const double *v, double *out, hipStream_t s) {
  if (P.dim == 2)
    hipLaunchKernelGGL(k_entropy<2>, dim3(P.n_elem), dim3(64), 0, s, P, v, out);
  else
    hipLaunchKernelGGL(k_entropy<3>, dim3(P.n_elem), dim3(64), 0, s, P, v, out);
  return hipGetLastError();
}

hipError_t launch_quad_coords(const DevPlan &P, double *xq, hipStream_t s) {
  const size_t NQ = (size_t)P.n_elem * P.Nq;
  hipLaunchKernelGGL(k_quad_coords, dim3((unsigned)((NQ + 255) / 256)), dim3(256), 0, s, P, xq);
  return hipGetLastError();
}

hipError_t launch_l2_error(const DevPlan &P, int kind, const double *f, const double *ex, double *out,
                           hipStream_t s) {
  if (P.dim == 2)
    hipLaunchKernelGGL(k_l2_error<2>, dim3(P.n_elem), dim3(64), 0, s, P, kind, f, ex, out);
  else
    hipLaunchKernelGGL(k_l2_error<3>, dim3(P.n_elem), dim3(64), 0, s, P, kind, f, ex, out);
  return hipGetLastError();
}

hipError_t launch_l2_error_visc(const DevPlan &P, const double *f, const double *ex, double *out, hipStream_t s) {
  if (P.dim == 2)
    hipLaunchKernelGGL(k_l2_error_visc<2>, dim3(P.n_elem), dim3(64), 0, s, P, f, ex, out);
  else
    hipLaunchKernelGGL(k_l2_error_visc<3>, dim3(P.n_elem), dim3(64), 0, s, P, f, ex, out);
  return hipGetLastError();
}

hipError_t launch_face_quad_coords(const DevPlan &P, double *xf, hipStream_t s) {
  const size_t NF = (size_t)P.n_elem * P.nf * P.Nfq;
  hipLaunchKernelGGL(k_face_quad_coords, dim3((unsigned)((NF + 255) / 256)), dim3(256), 0, s, P, xf);
  return hipGetLastError();
}

hipError_t launch_trace_project(const DevPlan &P, const double *g, double *vbc, hipStream_t s) {
  if (P.Nfp > PJ_NFP || P.m > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trace_project, dim3((unsigned)((size_t)P.n_elem * P.nf)), dim3(64), 0, s, P, g, vbc);
  return hipGetLastError();
}

hipError_t launch_weak_u(const DevPlan &P, const double *v, double *b, hipStream_t s) {
  const size_t lds = (size_t)((P.dim + 2) * P.Np + P.Nq * (P.dim + 2)) * sizeof(double);
  if (P.dim == 2)
    hipLaunchKernelGGL(k_weak_u<2>, dim3(P.n_elem), dim3(SB), lds, s, P, v, b);
  else
    hipLaunchKernelGGL(k_weak_u<3>, dim3(P.n_elem), dim3(SB), lds, s, P, v, b);
  return hipGetLastError();
}

hipError_t launch_mass_solve(const DevPlan &P, const double *b, double *u, hipStream_t s) {
  const size_t lds = (size_t)(P.Np * P.Np + (P.dim + 2) * P.Np + P.Nq) * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_mass_solve<2>, dim3(P.n_elem), dim3(SB), lds, s, P, b, u);
  else
    hipLaunchKernelGGL(k_mass_solve<3>, dim3(P.n_elem), dim3(SB), lds, s, P, b, u);
  return hipGetLastError();
}

}  // namespace hdg
