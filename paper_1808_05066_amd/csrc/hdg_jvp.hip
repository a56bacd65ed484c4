// Matrix-free FP64 action of the element Newton matrix,
//   [y_loc; y_tr] = [A B; C D] [dx; P_K dlambda]   for every element,
// from the quadrature-point Jacobians that the point kernels store (the same
// coefficients the block contraction turns into A, B, C, D).  It is the FP64
// residual of the refinement loop of the mixed-precision path: nothing of the
// element matrices is formed, so its cost is that of one residual evaluation.
//
// Rows follow the weak forms of the element, gradient and trace equations:
//   v rows (c,a):   sum_q phi_a (Mv dv_q)_c + sum_q grad phi_a . (Kv dv_q + Kq dq_q)_c
//                   + sum_faces phi_a (Fv dv_f + Fq dq_f + Fh dlam_f)_c
//   q rows (c,j,a): sum_q d_j phi_a dv_q,c + sum_q W phi_a dq_q,cj - sum_faces phi_a n_j dlam_f,c
//   trace (f,c,b):  sum_fq mu_b (Fv dv_f + Fq dq_f + Fh dlam_f)_c,  or mu_b W dlam_f,c on
//                   Dirichlet-trace faces.
#include "hdg_plan.hpp"

namespace hdg {

namespace {

constexpr int JB = 256;

template <int D, bool VISC>
__global__ __launch_bounds__(JB) void k_jvp(DevPlan P, int e0, const double *__restrict__ dx,
                                            const double *__restrict__ dlam, double *yloc, double *ytr) {
  constexpr int M = D + 2;
  constexpr int MD = M * D;
  constexpr int PV = M + MD + (VISC ? MD * D + MD : 0);   // per volume point
  constexpr int PF = 2 * M;                                // per face point
  extern __shared__ double sm[];
  const int el = blockIdx.x, e = e0 + el, tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq, nf = P.nf, Nfp = P.Nfp, Nfq = P.Nfq, n = P.n, k = P.k;
  const int MF = M * Nfp;
  const PointLayout L = P.L;
  double *xv = sm;              // [n]
  double *lam = xv + n;         // [k]
  double *pq = lam + k;         // [Nq][PV]
  double *pfq = pq + (size_t)Nq * PV;   // [nf][Nfq][PF]
  const double *xe = dx + (size_t)e * n;
  for (int i = tid; i < n; i += JB) xv[i] = xe[i];
  const int *tm = P.tmap + (size_t)e * nf * Nfp;
  for (int i = tid; i < k; i += JB) {
    const int b = i % Nfp, c = (i / Nfp) % M, f = i / MF;
    lam[i] = dlam[(size_t)c * P.n_trace + tm[f * Nfp + b]];
  }
  __syncthreads();

  // volume points
  for (int qp = tid; qp < Nq; qp += JB) {
    const double *phi = P.phi + (size_t)qp * Np;
    const double *w = P.pv + ((size_t)el * Nq + qp) * L.size;
    double dv[M], dq[VISC ? MD : 1];
    for (int c = 0; c < M; ++c) {
      double a = 0.0;
      for (int b = 0; b < Np; ++b) a += phi[b] * xv[c * Np + b];
      dv[c] = a;
    }
    if (VISC)
      for (int s = 0; s < MD; ++s) {
        double a = 0.0;
        for (int b = 0; b < Np; ++b) a += phi[b] * xv[M * Np + s * Np + b];
        dq[s] = a;
      }
    double *o = pq + (size_t)qp * PV;
    for (int c = 0; c < M; ++c) {
      double a = 0.0;
      for (int cp = 0; cp < M; ++cp) a += w[L.Mv + c * M + cp] * dv[cp];
      o[c] = a;
      for (int r = 0; r < D; ++r) {
        double t = 0.0;
        for (int cp = 0; cp < M; ++cp) t += w[L.Kv + (c * D + r) * M + cp] * dv[cp];
        if (VISC)
          for (int s = 0; s < MD; ++s) t += w[L.Kq + (c * D + r) * MD + s] * dq[s];
        o[M + c * D + r] = t;
      }
    }
    if (VISC) {
      const double W = w[L.W];
      for (int c = 0; c < M; ++c)
        for (int j = 0; j < D; ++j) {
          for (int r = 0; r < D; ++r) o[M + MD + (c * D + j) * D + r] = w[L.WJ + r * D + j] * dv[c];
          o[M + MD + MD * D + c * D + j] = W * dq[c * D + j];
        }
    }
  }
  // face points
  for (int t = tid; t < nf * Nfq; t += JB) {
    const int f = t / Nfq, fq = t % Nfq;
    const double *fp = P.fphi + ((size_t)f * Nfq + fq) * Nfp;
    const int *fn = P.fnodes + f * Nfp;
    const double *w = P.pf + (((size_t)el * nf + f) * Nfq + fq) * L.fsize;
    double dv[M], dl[M], dq[VISC ? MD : 1];
    for (int c = 0; c < M; ++c) {
      double a = 0.0, h = 0.0;
      for (int b = 0; b < Nfp; ++b) {
        a += fp[b] * xv[c * Np + fn[b]];
        h += fp[b] * lam[f * MF + c * Nfp + b];
      }
      dv[c] = a;
      dl[c] = h;
    }
    if (VISC)
      for (int s = 0; s < MD; ++s) {
        double a = 0.0;
        for (int b = 0; b < Nfp; ++b) a += fp[b] * xv[M * Np + s * Np + fn[b]];
        dq[s] = a;
      }
    double *o = pfq + (size_t)t * PF;
    for (int c = 0; c < M; ++c) {
      double a = 0.0;
      for (int cp = 0; cp < M; ++cp) a += w[L.fFv + c * M + cp] * dv[cp] + w[L.fFh + c * M + cp] * dl[cp];
      if (VISC)
        for (int s = 0; s < MD; ++s) a += w[L.fFq + c * MD + s] * dq[s];
      o[c] = a;
      o[M + c] = dl[c];
    }
  }
  __syncthreads();

  // element rows
  double *ye = yloc + (size_t)e * n;
  for (int row = tid; row < n; row += JB) {
    const int a = row % Np, cs = row / Np;
    double acc = 0.0;
    if (cs < M) {
      const int c = cs;
      for (int qp = 0; qp < Nq; ++qp) {
        const double *o = pq + (size_t)qp * PV;
        acc += P.phi[(size_t)qp * Np + a] * o[c];
        for (int r = 0; r < D; ++r) acc += P.dphi[((size_t)r * Nq + qp) * Np + a] * o[M + c * D + r];
      }
      for (int f = 0; f < nf; ++f) {
        const int ia = P.node_face[a * nf + f];
        if (ia < 0) continue;
        for (int fq = 0; fq < Nfq; ++fq)
          acc += P.fphi[((size_t)f * Nfq + fq) * Nfp + ia] * pfq[((size_t)f * Nfq + fq) * PF + c];
      }
    } else if (VISC) {
      const int cj = cs - M, c = cj / D, j = cj % D;
      for (int qp = 0; qp < Nq; ++qp) {
        const double *o = pq + (size_t)qp * PV;
        for (int r = 0; r < D; ++r) acc += P.dphi[((size_t)r * Nq + qp) * Np + a] * o[M + MD + cj * D + r];
        acc += P.phi[(size_t)qp * Np + a] * o[M + MD + MD * D + cj];
      }
      for (int f = 0; f < nf; ++f) {
        const int ia = P.node_face[a * nf + f];
        if (ia < 0) continue;
        for (int fq = 0; fq < Nfq; ++fq) {
          const double *w = P.pf + (((size_t)el * nf + f) * Nfq + fq) * L.fsize;
          acc -= P.fphi[((size_t)f * Nfq + fq) * Nfp + ia] * w[L.fWn + j] * pfq[((size_t)f * Nfq + fq) * PF + M + c];
        }
      }
    }
    ye[row] = acc;
  }
  // trace rows
  double *yt = ytr + (size_t)e * k;
  const int *fbc = P.face_bc + (size_t)e * nf;
  for (int row = tid; row < k; row += JB) {
    const int ib = row % Nfp, c = (row / Nfp) % M, f = row / MF;
    const bool dir = fbc[f] != 0;
    double acc = 0.0;
    for (int fq = 0; fq < Nfq; ++fq) {
      const double mu = P.fphi[((size_t)f * Nfq + fq) * Nfp + ib];
      const double *o = pfq + ((size_t)f * Nfq + fq) * PF;
      if (dir) {
        const double *w = P.pf + (((size_t)el * nf + f) * Nfq + fq) * L.fsize;
        acc += mu * w[L.fW] * o[M + c];
      } else {
        acc += mu * o[c];
      }
    }
    yt[row] = (P.row_drop && P.row_drop[((size_t)e * nf + f) * Nfp + ib]) ? 0.0 : acc;
  }
}

template <int D, bool VISC>
hipError_t launch_jvp_t(const DevPlan &P, int e0, int ec, const double *dx, const double *dlam, double *yloc,
                        double *ytr, hipStream_t s) {
  constexpr int M = D + 2, MD = M * D;
  constexpr int PV = M + MD + (VISC ? MD * D + MD : 0);
  const size_t lds = ((size_t)P.n + P.k + (size_t)P.Nq * PV + (size_t)P.nf * P.Nfq * 2 * M) * sizeof(double);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = set_dyn_lds((const void *)k_jvp<D, VISC>, lds);
  if (e) return e;
  hipLaunchKernelGGL((k_jvp<D, VISC>), dim3(ec), dim3(JB), lds, s, P, e0, dx, dlam, yloc, ytr);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_jvp(const DevPlan &P, int e0, int ec, const double *dx, const double *dlam, double *yloc,
                      double *ytr, hipStream_t s) {
  if (P.dim == 2) return P.viscous ? launch_jvp_t<2, true>(P, e0, ec, dx, dlam, yloc, ytr, s)
                                   : launch_jvp_t<2, false>(P, e0, ec, dx, dlam, yloc, ytr, s);
  return P.viscous ? launch_jvp_t<3, true>(P, e0, ec, dx, dlam, yloc, ytr, s)
                   : launch_jvp_t<3, false>(P, e0, ec, dx, dlam, yloc, ytr, s);
}

}  // namespace hdg
