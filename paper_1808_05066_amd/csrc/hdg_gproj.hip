// Projection viscous numerical flux (Section 4):  g_hat = (Pi G(v_h, q_h)) . n on every face,
// Pi the element L2 projection onto the polynomial space of q_h.  It depends on the whole
// element, so it is not a face-point quantity: the face points carry no viscous flux when it
// is selected, and these kernels add its terms to the blocks after the contraction.
//
// With H = M_K^-1 Phi^T (Np x Nq, M_K the element mass matrix), the projected flux at a face
// point x is sum_a phi_a(x) sum_q H[a][q] W_q G(x_q), so every face term becomes a sum over the
// volume points:
//   <g_hat, phi_i>_F = sum_j sum_q Z_f^j[b][q] W_q G_{.j}(x_q),   i = fnodes[f][b],
//   Z_f^j[b][q] = sum_{x in F} W_x n_j(x) mu_b(x) sum_b' mu_b'(x) H[fnodes[f][b']][q]
// (the volume functions of a nodal basis restricted to a face are the face's own nodal
// functions, and vanish there for nodes off the face).  The same Z gives the trace rows
// <g_hat, mu_b>_F.  Derivatives: G is differentiated at the volume points with respect to v
// (dual numbers) and q (G is linear in q: the columns are G(v, e_s)).
//
// Scratch (per chunk slot): gp [Nq][MD + MD*M + MD*MD] = W_q (G, dG/dv, dG/dq) at the volume
// points; gz [nf][dim][Nfp][Nq] = Z.
#include "hdg_physics.hpp"
#include "hdg_plan.hpp"

namespace hdg {

namespace {

constexpr int GB = 256;

template <int D>
__global__ __launch_bounds__(GB) void k_gproj_points(DevPlan P, int e0, int ec, const double *__restrict__ v,
                                                      const double *__restrict__ q) {
  constexpr int M = D + 2, MD = M * D, PS = MD + MD * M + MD * MD;
  const int t = blockIdx.x * GB + threadIdx.x;
  if (t >= ec * P.Nq) return;
  const int el = t / P.Nq, qp = t % P.Nq, e = e0 + el;
  const int Np = P.Np;
  const size_t NN = (size_t)P.n_elem * Np;
  const double *phi = P.phi + (size_t)qp * Np;
  double vq[M], qq[MD];
  for (int c = 0; c < M; ++c) {
    double acc = 0.0;
    for (int a = 0; a < Np; ++a) acc += phi[a] * v[(size_t)c * NN + (size_t)e * Np + a];
    vq[c] = acc;
  }
  for (int s = 0; s < MD; ++s) {
    double acc = 0.0;
    for (int a = 0; a < Np; ++a) acc += phi[a] * q[(size_t)s * NN + (size_t)e * Np + a];
    qq[s] = acc;
  }
  const double W = P.geo_vol[((size_t)e * P.Nq + qp) * (1 + D * D)];
  const double gam = P.gamma;
  double *o = P.gp + ((size_t)el * P.Nq + qp) * PS;
  const Prim<D, double> sv = prim_of_v<D, double>(vq, gam);
  double G[MD];
  flux_G<D, double, double>(sv, qq, gam, P.mu, P.Pr, G);
  for (int i = 0; i < MD; ++i) o[i] = W * G[i];
  for (int tt = 0; tt < M; ++tt) {
    Dual vd[M];
    for (int c = 0; c < M; ++c) vd[c] = Dual{vq[c], c == tt ? 1.0 : 0.0};
    Dual Gd[MD];
    flux_G<D, Dual, double>(prim_of_v<D, Dual>(vd, gam), qq, gam, P.mu, P.Pr, Gd);
    for (int i = 0; i < MD; ++i) o[MD + i * M + tt] = W * Gd[i].d;
  }
  for (int si = 0; si < MD; ++si) {
    double es[MD];
    for (int i = 0; i < MD; ++i) es[i] = (i == si) ? 1.0 : 0.0;
    flux_G<D, double, double>(sv, es, gam, P.mu, P.Pr, G);
    for (int i = 0; i < MD; ++i) o[MD + MD * M + i * MD + si] = W * G[i];
  }
}

// M_K^-1 by Gauss-Jordan in LDS (symmetric positive definite: no pivoting), H = M_K^-1 Phi^T,
// then Z for every face and direction.  One workgroup per element of the chunk.
template <int D>
__global__ __launch_bounds__(GB) void k_gproj_lift(DevPlan P, int e0) {
  extern __shared__ double sm[];
  const int el = blockIdx.x, e = e0 + el, tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq, nf = P.nf, Nfp = P.Nfp, Nfq = P.Nfq, N2 = 2 * Np;
  double *Mi = sm;                     // [Np][2 Np]: [M | I] -> [I | M^-1]
  double *fac = Mi + (size_t)Np * N2;  // [Np]
  double *H = fac + Np;                // [Np][Nq]
  const int gs = 1 + D * D;
  for (int t = tid; t < Np * Np; t += GB) {
    const int a = t / Np, b = t % Np;
    double acc = 0.0;
    for (int qp = 0; qp < Nq; ++qp)
      acc += P.geo_vol[((size_t)e * Nq + qp) * gs] * P.phi[(size_t)qp * Np + a] * P.phi[(size_t)qp * Np + b];
    Mi[a * N2 + b] = acc;
    Mi[a * N2 + Np + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < Np; ++k) {
    const double inv = 1.0 / Mi[k * N2 + k];
    __syncthreads();
    for (int t = tid; t < N2; t += GB) Mi[k * N2 + t] *= inv;
    __syncthreads();
    for (int r = tid; r < Np; r += GB) fac[r] = (r == k) ? 0.0 : Mi[r * N2 + k];
    __syncthreads();
    for (int t = tid; t < Np * N2; t += GB) {
      const int r = t / N2, c = t % N2;
      if (r != k) Mi[t] -= fac[r] * Mi[k * N2 + c];
    }
    __syncthreads();
  }
  for (int t = tid; t < Np * Nq; t += GB) {
    const int a = t / Nq, qp = t % Nq;
    double acc = 0.0;
    for (int b = 0; b < Np; ++b) acc += Mi[a * N2 + Np + b] * P.phi[(size_t)qp * Np + b];
    H[t] = acc;
  }
  __syncthreads();
  double *Z = P.gz + (size_t)el * nf * D * Nfp * Nq;
  for (int t = tid; t < nf * D * Nfp * Nq; t += GB) {
    const int qp = t % Nq, b = (t / Nq) % Nfp, j = (t / (Nq * Nfp)) % D, f = t / (Nq * Nfp * D);
    const int *fn = P.fnodes + f * Nfp;
    double acc = 0.0;
    for (int x = 0; x < Nfq; ++x) {
      const double *g = P.geo_face + (((size_t)e * nf + f) * Nfq + x) * (1 + D);
      const double *mu = P.fphi + ((size_t)f * Nfq + x) * Nfp;
      double h = 0.0;
      for (int b2 = 0; b2 < Nfp; ++b2) h += mu[b2] * H[fn[b2] * Nq + qp];
      acc += g[0] * g[1 + j] * mu[b] * h;
    }
    Z[t] = acc;
  }
}

// Add the projected flux terms: v rows of A and R_loc (every face of the element), trace rows
// of C and R_tr (flux faces).  One workgroup per element of the chunk, one output entry per
// thread pass.
template <int D>
__global__ __launch_bounds__(GB) void k_gproj_add(DevPlan P, int e0) {
  constexpr int M = D + 2, MD = M * D, PS = MD + MD * M + MD * MD;
  const int el = blockIdx.x, e = e0 + el, tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq, nf = P.nf, Nfp = P.Nfp, n = P.n, np = P.n_pad, kp = P.k_pad;
  const int MF = M * Nfp;
  const double *gp = P.gp + (size_t)el * Nq * PS;
  const double *Z = P.gz + (size_t)el * nf * D * Nfp * Nq;
  double *A = P.A + (size_t)el * np * np;
  double *R = P.X + (size_t)el * P.kx * np + (size_t)kp * np;
  double *C = P.C + (size_t)el * np * kp;
  double *Rt = P.Rt + (size_t)el * kp;
  const int *fbc = P.face_bc + (size_t)e * nf;
  // sum_j sum_q Z_f^j[b][q] J(q, c, j, col) phi_a(q) for one face row (f, b), component c and
  // column col (v columns c' Np + a, q columns M Np + s Np + a, or -1 for the residual)
  auto term = [&](int f, int b, int c, int col) {
    int off, a = 0;
    if (col < 0) {
      off = 0;
    } else if (col < M * Np) {
      off = MD + (col / Np);                 // + (c D + j) M
      a = col % Np;
    } else {
      off = MD + MD * M + (col - M * Np) / Np;   // + (c D + j) MD
      a = (col - M * Np) % Np;
    }
    const int stride = col < 0 ? 1 : (col < M * Np ? M : MD);
    double acc = 0.0;
    for (int j = 0; j < D; ++j) {
      const double *z = Z + ((size_t)(f * D + j) * Nfp + b) * Nq;
      const int o = off + (c * D + j) * stride;
      for (int qp = 0; qp < Nq; ++qp) {
        const double w = gp[(size_t)qp * PS + o];
        acc += z[qp] * (col < 0 ? w : w * P.phi[(size_t)qp * Np + a]);
      }
    }
    return acc;
  };
  // element rows (c, i) of the v equation
  for (int t = tid; t < M * Np * (n + 1); t += GB) {
    const int row = t % (M * Np), col = t / (M * Np) - 1;   // col -1: residual
    const int c = row / Np, i = row % Np;
    double acc = 0.0;
    for (int f = 0; f < nf; ++f) {
      const int b = P.node_face[i * nf + f];
      if (b >= 0) acc += term(f, b, c, col);
    }
    if (acc == 0.0) continue;
    if (col < 0)
      R[row] += acc;
    else
      A[(size_t)col * np + row] += acc;
  }
  // trace rows (f, c, b) of flux faces
  for (int t = tid; t < nf * MF * (n + 1); t += GB) {
    const int row = t % (nf * MF), col = t / (nf * MF) - 1;
    const int f = row / MF, c = (row % MF) / Nfp, b = row % Nfp;
    if (fbc[f]) continue;
    const double acc = term(f, b, c, col);
    if (col < 0)
      Rt[row] += acc;
    else
      C[(size_t)col * kp + row] += acc;
  }
}

}  // namespace

size_t gproj_lift_lds(const DevPlan &P) {
  return ((size_t)P.Np * 2 * P.Np + P.Np + (size_t)P.Np * P.Nq) * sizeof(double);
}

hipError_t launch_gproj(const DevPlan &P, int e0, int ec, const double *v, const double *q, hipStream_t s) {
  if (!P.ghat_proj || !P.gp || !P.gz || !q) return hipErrorInvalidValue;
  const size_t lds = gproj_lift_lds(P);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)(((size_t)ec * P.Nq + GB - 1) / GB);
  if (P.dim == 2) {
    hipLaunchKernelGGL(k_gproj_points<2>, dim3(nb), dim3(GB), 0, s, P, e0, ec, v, q);
    hipLaunchKernelGGL(k_gproj_lift<2>, dim3(ec), dim3(GB), lds, s, P, e0);
    hipLaunchKernelGGL(k_gproj_add<2>, dim3(ec), dim3(GB), 0, s, P, e0);
  } else {
    hipLaunchKernelGGL(k_gproj_points<3>, dim3(nb), dim3(GB), 0, s, P, e0, ec, v, q);
    hipLaunchKernelGGL(k_gproj_lift<3>, dim3(ec), dim3(GB), lds, s, P, e0);
    hipLaunchKernelGGL(k_gproj_add<3>, dim3(ec), dim3(GB), 0, s, P, e0);
  }
  return hipGetLastError();
}

}  // namespace hdg
