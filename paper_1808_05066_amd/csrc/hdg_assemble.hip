// Element residual and Jacobian blocks (volume and face integrals).
//
// Stage 1 (k_vol_points / k_face_points): one thread per quadrature point
// evaluates the pointwise physics and, by forward-mode passes seeded along each
// input direction, the pointwise Jacobians; it stores them pre-multiplied by
// the quadrature weight and, for volume points, already contracted with the
// inverse metric so the contraction stage only sees reference-element tables.
// Stage 2 (k_contract): one workgroup per element contracts the pointwise data
// against the basis tables into the padded dense blocks
//   A (n_pad x n_pad), [B | R_loc] (n_pad x kx), C (k_pad x n_pad), D, R_tr
// of the element Newton system (weak forms of the gradient, element and trace
// equations of the hybridized DG methods in entropy variables).
#include "hdg_physics.hpp"
#include "hdg_plan.hpp"

namespace hdg {

namespace {

constexpr int BLK = 256;

__device__ inline bool bad_state(double vm, double x) { return !(vm < 0.0) || !isfinite(x); }

template <int D, bool VISC>
__global__ __launch_bounds__(128) void k_vol_points(DevPlan P, int e0, int ec, const double *__restrict__ v,
                                                     const double *__restrict__ q,
                                                     const double *__restrict__ ustar, int32_t *status) {
  constexpr int M = D + 2;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= ec * P.Nq) return;
  const int el = tid / P.Nq, qp = tid % P.Nq, e = e0 + el;
  const int Np = P.Np;
  const size_t NN = (size_t)P.n_elem * Np;
  const double *phi = P.phi + (size_t)qp * Np;
  const size_t nb = (size_t)e * Np;
  double vq[M], qq[VISC ? M * D : 1], us[M], sq[M];
  for (int c = 0; c < M; ++c) {
    double s = 0.0, t = 0.0, f = 0.0;
    for (int a = 0; a < Np; ++a) {
      s += phi[a] * v[c * NN + nb + a];
      if (ustar) t += phi[a] * ustar[c * NN + nb + a];
      if (P.src && !P.src_qp) f += phi[a] * P.src[c * NN + nb + a];
    }
    vq[c] = s;
    us[c] = t;
    sq[c] = (P.src && P.src_qp) ? P.src[c * (size_t)P.n_elem * P.Nq + (size_t)e * P.Nq + qp] : f;
  }
  if (VISC)
    for (int s = 0; s < M * D; ++s) {
      double acc = 0.0;
      for (int a = 0; a < Np; ++a) acc += phi[a] * q[s * NN + nb + a];
      qq[s] = acc;
    }
  const double *g = P.geo_vol + ((size_t)e * P.Nq + qp) * (1 + D * D);
  const double W = g[0];
  double Ji[D * D];
  for (int i = 0; i < D * D; ++i) Ji[i] = g[1 + i];
  double *out = P.pv + ((size_t)el * P.Nq + qp) * P.L.size;
  const PointLayout &L = P.L;
  double chk = 0.0;
  for (int c = 0; c < M; ++c) chk += vq[c];
  if (VISC)
    for (int s = 0; s < M * D; ++s) chk += qq[s];
  if (bad_state(vq[M - 1], chk)) {
    status[e] = HDG_ENONPHYS;
    for (int i = 0; i < L.size; ++i) out[i] = 0.0;
    return;
  }
  const double gam = P.gamma, alpha = P.alpha;
  for (int t = 0; t < M; ++t) {
    Dual vd[M];
    for (int c = 0; c < M; ++c) vd[c] = Dual{vq[c], c == t ? 1.0 : 0.0};
    Prim<D, Dual> s = prim_of_v<D, Dual>(vd, gam);
    Dual u[M];
    u_of_prim<D, Dual>(s, gam, u);
    Dual F[M * D];
    flux_F<D, Dual>(s, gam, F);
    if (VISC) {
      Dual G[M * D];
      flux_G<D, Dual, double>(s, qq, gam, P.mu, P.Pr, G);
      for (int i = 0; i < M * D; ++i) F[i] = F[i] + G[i];
    }
    for (int c = 0; c < M; ++c) out[L.Mv + c * M + t] = W * alpha * u[c].d;
    for (int c = 0; c < M; ++c)
      for (int r = 0; r < D; ++r) {
        double acc = 0.0;
        for (int j = 0; j < D; ++j) acc += F[c * D + j].d * Ji[r * D + j];
        out[L.Kv + (c * D + r) * M + t] = -W * acc;
      }
    if (t == 0) {
      for (int c = 0; c < M; ++c) {
        out[L.Wu + c] = W * (alpha * (u[c].v - us[c]) - sq[c]);
        for (int r = 0; r < D; ++r) {
          double acc = 0.0;
          for (int j = 0; j < D; ++j) acc += F[c * D + j].v * Ji[r * D + j];
          out[L.Fr + c * D + r] = -W * acc;
        }
      }
    }
  }
  if (VISC) {
    Prim<D, double> s = prim_of_v<D, double>(vq, gam);
    for (int si = 0; si < M * D; ++si) {
      double es[M * D];
      for (int i = 0; i < M * D; ++i) es[i] = (i == si) ? 1.0 : 0.0;
      double G[M * D];
      flux_G<D, double, double>(s, es, gam, P.mu, P.Pr, G);
      for (int c = 0; c < M; ++c)
        for (int r = 0; r < D; ++r) {
          double acc = 0.0;
          for (int j = 0; j < D; ++j) acc += G[c * D + j] * Ji[r * D + j];
          out[L.Kq + (c * D + r) * (M * D) + si] = -W * acc;
        }
    }
    for (int i = 0; i < M * D; ++i) out[L.Wq + i] = W * qq[i];
  }
  for (int c = 0; c < M; ++c) out[L.v + c] = vq[c];
  for (int i = 0; i < D * D; ++i) out[L.WJ + i] = W * Ji[i];
  out[L.W] = W;
}

// MV: the mean-value stabilization (its own instantiation: its path integral needs many
// registers, which the other stabilizations should not pay for)
template <int D, bool VISC, bool MV>
__global__ __launch_bounds__(128) void k_face_points(DevPlan P, int e0, int ec, const double *__restrict__ v,
                                                      const double *__restrict__ q,
                                                      const double *__restrict__ vhat,
                                                      const double *__restrict__ vbc, int32_t *status) {
  constexpr int M = D + 2;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int Nfq = P.Nfq, nf = P.nf, Nfp = P.Nfp, Np = P.Np;
  if (tid >= ec * nf * Nfq) return;
  const int fq = tid % Nfq, f = (tid / Nfq) % nf, el = tid / (Nfq * nf), e = e0 + el;
  const size_t NN = (size_t)P.n_elem * Np, NT = (size_t)P.n_trace;
  const double *fp = P.fphi + ((size_t)f * Nfq + fq) * Nfp;
  const int *fn = P.fnodes + f * Nfp;
  const int *tm = P.tmap + ((size_t)e * nf + f) * Nfp;
  const int bc = P.face_bc[(size_t)e * nf + f];
  double vv[M], vh[M], vb[M], qq[VISC ? M * D : 1];
  for (int c = 0; c < M; ++c) {
    double a = 0.0, h = 0.0, bb = 0.0;
    for (int b = 0; b < Nfp; ++b) {
      a += fp[b] * v[c * NN + (size_t)e * Np + fn[b]];
      h += fp[b] * vhat[c * NT + tm[b]];
      if (bc && vbc) bb += fp[b] * vbc[c * NT + tm[b]];
    }
    vv[c] = a;
    vh[c] = h;
    vb[c] = bb;
  }
  if (VISC)
    for (int s = 0; s < M * D; ++s) {
      double a = 0.0;
      for (int b = 0; b < Nfp; ++b) a += fp[b] * q[s * NN + (size_t)e * Np + fn[b]];
      qq[s] = a;
    }
  const double *g = P.geo_face + (((size_t)e * nf + f) * Nfq + fq) * (1 + D);
  const double W = g[0];
  double n[D];
  for (int j = 0; j < D; ++j) n[j] = g[1 + j];
  const PointLayout &L = P.L;
  double *out = P.pf + (((size_t)el * nf + f) * Nfq + fq) * L.fsize;
  double chk = 0.0;
  for (int c = 0; c < M; ++c) chk += vv[c] + vh[c];
  if (bad_state(vv[M - 1], chk) || bad_state(vh[M - 1], chk)) {
    status[e] = HDG_ENONPHYS;
    for (int i = 0; i < L.fsize; ++i) out[i] = 0.0;
    return;
  }
  const double gam = P.gamma;
  // element state: normal flux and (below) its Jacobian columns
  Prim<D, double> sv = prim_of_v<D, double>(vv, gam);
  double Fv[M * D], Fnv[M];
  flux_F<D, double>(sv, gam, Fv);
  for (int c = 0; c < M; ++c) {
    double a = 0.0;
    for (int j = 0; j < D; ++j) a += Fv[c * D + j] * n[j];
    Fnv[c] = a;
  }
  // sigma = lambda_max(v_hat) A0(v_hat)
  Prim<D, double> sh = prim_of_v<D, double>(vh, gam);
  double A0h[M * M];
  A0_of_prim<D, double>(sh, gam, A0h);
  double vn = 0.0;
  for (int j = 0; j < D; ++j) vn += sh.V[j] * n[j];
  const double lam = dabs(vn) + sqrt(gam * sh.p / sh.rho);
  // trace-state directions: d(f_hat + g_hat)/d v_hat and the flux value
  // (with ghat_v the viscous numerical flux does not depend on v_hat: it is added below)
  // with the projection viscous flux the face points carry no viscous flux: it is added from
  // the volume points by the projection kernels
  const bool gface = VISC && !P.ghat_proj;
  const bool gh_trace = gface && !P.ghat_v;
  for (int t = 0; t < M; ++t) {
    Dual vd[M], o[M];
    for (int c = 0; c < M; ++c) vd[c] = Dual{vh[c], c == t ? 1.0 : 0.0};
    trace_flux<D, Dual, double>(vd, vv, Fnv, qq, n, gam, P.mu, P.Pr, gh_trace, o, P.sigma_s == 1);
    for (int c = 0; c < M; ++c) out[L.fFh + c * M + t] = W * o[c].d;
    if (t == 0)
      for (int c = 0; c < M; ++c) out[L.fFf + c] = W * o[c].v;
  }
  if (gface && P.ghat_v) {
    double G[M * D];
    flux_G<D, double, double>(sv, qq, gam, P.mu, P.Pr, G);
    for (int c = 0; c < M; ++c) {
      double a = 0.0;
      for (int j = 0; j < D; ++j) a += G[c * D + j] * n[j];
      out[L.fFf + c] += W * a;
    }
  }
  // element-state directions: d f_hat / d v = 1/2 (A_n(v) + sigma)
  double sig[M * M];   // sigma(v_hat), column t = sigma e_t
  if (P.sigma_s == 1) {
    for (int t = 0; t < M; ++t) {
      double et[M], col[M];
      for (int c = 0; c < M; ++c) et[c] = c == t ? 1.0 : 0.0;
      sigma_s_apply<D, double, double>(sh, A0h, n, gam, et, col);
      for (int c = 0; c < M; ++c) sig[c * M + t] = col[c];
    }
  } else {
    for (int i = 0; i < M * M; ++i) sig[i] = lam * A0h[i];
  }
  for (int t = 0; t < M; ++t) {
    Dual vd[M];
    for (int c = 0; c < M; ++c) vd[c] = Dual{vv[c], c == t ? 1.0 : 0.0};
    Prim<D, Dual> s = prim_of_v<D, Dual>(vd, gam);
    Dual F[M * D];
    flux_F<D, Dual>(s, gam, F);
    for (int c = 0; c < M; ++c) {
      double an = 0.0;
      for (int j = 0; j < D; ++j) an += F[c * D + j].d * n[j];
      out[L.fFv + c * M + t] = W * 0.5 * (an + sig[c * M + t]);
    }
    if (gface && P.ghat_v) {
      // d g_hat / d v with g_hat = G(v, q).n
      Dual G[M * D];
      flux_G<D, Dual, double>(s, qq, gam, P.mu, P.Pr, G);
      for (int c = 0; c < M; ++c) {
        double gn = 0.0;
        for (int j = 0; j < D; ++j) gn += G[c * D + j].d * n[j];
        out[L.fFv + c * M + t] += W * gn;
      }
    }
  }
  if (MV) {
    // mean-value stabilization: sigma depends on both states, so f_hat is differentiated with
    // respect to v_hat and to v in full (the values above are replaced)
    double gval[M];
    for (int c = 0; c < M; ++c) gval[c] = 0.0;
    if (gface) {
      double G[M * D];
      flux_G<D, double, double>(P.ghat_v ? sv : sh, qq, gam, P.mu, P.Pr, G);
      for (int c = 0; c < M; ++c)
        for (int j = 0; j < D; ++j) gval[c] += G[c * D + j] * n[j];
    }
    for (int t = 0; t < M; ++t) {
      Dual a[M], b[M], o[M];
      for (int c = 0; c < M; ++c) {
        a[c] = Dual{vh[c], c == t ? 1.0 : 0.0};
        b[c] = Dual{vv[c], 0.0};
      }
      fhat_mv<D, Dual>(a, b, n, gam, o);
      double gd[M];
      for (int c = 0; c < M; ++c) gd[c] = 0.0;
      if (gface && !P.ghat_v) {
        Dual G[M * D];
        flux_G<D, Dual, double>(prim_of_v<D, Dual>(a, gam), qq, gam, P.mu, P.Pr, G);
        for (int c = 0; c < M; ++c)
          for (int j = 0; j < D; ++j) gd[c] += G[c * D + j].d * n[j];
      }
      for (int c = 0; c < M; ++c) out[L.fFh + c * M + t] = W * (o[c].d + gd[c]);
      if (t == 0)
        for (int c = 0; c < M; ++c) out[L.fFf + c] = W * (o[c].v + gval[c]);
      for (int c = 0; c < M; ++c) {
        a[c] = Dual{vh[c], 0.0};
        b[c] = Dual{vv[c], c == t ? 1.0 : 0.0};
      }
      fhat_mv<D, Dual>(a, b, n, gam, o);
      for (int c = 0; c < M; ++c) gd[c] = 0.0;
      if (gface && P.ghat_v) {
        Dual G[M * D];
        flux_G<D, Dual, double>(prim_of_v<D, Dual>(b, gam), qq, gam, P.mu, P.Pr, G);
        for (int c = 0; c < M; ++c)
          for (int j = 0; j < D; ++j) gd[c] += G[c * D + j].d * n[j];
      }
      for (int c = 0; c < M; ++c) out[L.fFv + c * M + t] = W * (o[c].d + gd[c]);
    }
  }
  if (VISC) {
    // d g_hat / d q: g_hat is linear in q
    for (int si = 0; si < M * D; ++si) {
      double es[M * D], G[M * D];
      for (int i = 0; i < M * D; ++i) es[i] = (i == si) ? 1.0 : 0.0;
      if (gface) flux_G<D, double, double>(P.ghat_v ? sv : sh, es, gam, P.mu, P.Pr, G);
      for (int c = 0; c < M; ++c) {
        double a = 0.0;
        if (gface)
          for (int j = 0; j < D; ++j) a += G[c * D + j] * n[j];
        out[L.fFq + c * (M * D) + si] = W * a;
      }
    }
  }
  for (int j = 0; j < D; ++j) out[L.fWn + j] = W * n[j];
  for (int c = 0; c < M; ++c) {
    out[L.fvh + c] = vh[c];
    out[L.fFd + c] = W * (vh[c] - vb[c]);
  }
  out[L.fW] = W;
}

// Accumulate acc[bb] += t * tab[b0 + bb] for the face node b = fnodes[ib] when it
// falls in the current column chunk [b0, b0 + 16).
__device__ inline void face_scatter(double (&acc)[16], int b, int b0, double val) {
#pragma unroll
  for (int bb = 0; bb < 16; ++bb)
    if (b == b0 + bb) acc[bb] += val;
}

template <int D, bool VISC>
__global__ __launch_bounds__(BLK) void k_contract(DevPlan P, int e0, int ec) {
  constexpr int M = D + 2;
  const int el = blockIdx.x;
  const int e = e0 + el;
  const int tid = threadIdx.x;
  const int Np = P.Np, Nq = P.Nq, nf = P.nf, Nfp = P.Nfp, Nfq = P.Nfq;
  const int np = P.n_pad, kp = P.k_pad, kx = P.kx;
  const PointLayout L = P.L;
  double *A = P.A + (size_t)el * np * np;
  double *X = P.X + (size_t)el * kx * np;
  double *C = P.C + (size_t)el * np * kp;
  double *Dm = P.D + (size_t)el * kp * kp;
  double *Rt = P.Rt + (size_t)el * kp;
  const double *pv = P.pv + (size_t)el * Nq * L.size;
  const double *pf = P.pf + (size_t)el * nf * Nfq * L.fsize;
  const double *phi = P.phi, *dphi = P.dphi, *fphi = P.fphi;
  const int *fnodes = P.fnodes, *node_face = P.node_face;
  const int *fbc = P.face_bc + (size_t)e * nf;

  // zero the blocks; identity on the padding of A
  for (size_t i = tid; i < (size_t)np * np; i += BLK) {
    int col = (int)(i / np), row = (int)(i % np);
    A[i] = (row == col && row >= P.n) ? 1.0 : 0.0;
  }
  for (size_t i = tid; i < (size_t)kx * np; i += BLK) X[i] = 0.0;
  for (size_t i = tid; i < (size_t)np * kp; i += BLK) C[i] = 0.0;
  for (size_t i = tid; i < (size_t)kp * kp; i += BLK) Dm[i] = 0.0;
  for (int i = tid; i < kp; i += BLK) Rt[i] = 0.0;
  __syncthreads();

  // A_vv: row (c, a), columns (cp, b)
  for (int t = tid; t < M * M * Np; t += BLK) {
    const int a = t % Np, c = (t / Np) % M, cp = t / (Np * M);
    const int row = c * Np + a;
    for (int b0 = 0; b0 < Np; b0 += 16) {
      double acc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = 0.0;
      for (int qp = 0; qp < Nq; ++qp) {
        const double *w = pv + (size_t)qp * L.size;
        double ta = w[L.Mv + c * M + cp] * phi[qp * Np + a];
        for (int r = 0; r < D; ++r) ta += w[L.Kv + (c * D + r) * M + cp] * dphi[((size_t)r * Nq + qp) * Np + a];
#pragma unroll
        for (int bb = 0; bb < 16; ++bb)
          if (b0 + bb < Np) acc[bb] += ta * phi[qp * Np + b0 + bb];
      }
      for (int f = 0; f < nf; ++f) {
        const int ia = node_face[a * nf + f];
        if (ia < 0) continue;
        for (int fq = 0; fq < Nfq; ++fq) {
          const double *w = pf + ((size_t)f * Nfq + fq) * L.fsize;
          const double *fpr = fphi + ((size_t)f * Nfq + fq) * Nfp;
          const double tf = w[L.fFv + c * M + cp] * fpr[ia];
          for (int ib = 0; ib < Nfp; ++ib) face_scatter(acc, fnodes[f * Nfp + ib], b0, tf * fpr[ib]);
        }
      }
      for (int bb = 0; bb < 16 && b0 + bb < Np; ++bb) A[(size_t)(cp * Np + b0 + bb) * np + row] = acc[bb];
    }
  }
  if (VISC) {
    // A_vq: row (c, a), columns (s, b)
    for (int t = tid; t < M * M * D * Np; t += BLK) {
      const int a = t % Np, c = (t / Np) % M, s = t / (Np * M);
      const int row = c * Np + a;
      for (int b0 = 0; b0 < Np; b0 += 16) {
        double acc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.0;
        for (int qp = 0; qp < Nq; ++qp) {
          const double *w = pv + (size_t)qp * L.size;
          double ta = 0.0;
          for (int r = 0; r < D; ++r)
            ta += w[L.Kq + (c * D + r) * (M * D) + s] * dphi[((size_t)r * Nq + qp) * Np + a];
#pragma unroll
          for (int bb = 0; bb < 16; ++bb)
            if (b0 + bb < Np) acc[bb] += ta * phi[qp * Np + b0 + bb];
        }
        for (int f = 0; f < nf; ++f) {
          const int ia = node_face[a * nf + f];
          if (ia < 0) continue;
          for (int fq = 0; fq < Nfq; ++fq) {
            const double *w = pf + ((size_t)f * Nfq + fq) * L.fsize;
            const double *fpr = fphi + ((size_t)f * Nfq + fq) * Nfp;
            const double tf = w[L.fFq + c * (M * D) + s] * fpr[ia];
            for (int ib = 0; ib < Nfp; ++ib) face_scatter(acc, fnodes[f * Nfp + ib], b0, tf * fpr[ib]);
          }
        }
        for (int bb = 0; bb < 16 && b0 + bb < Np; ++bb)
          A[(size_t)(M * Np + s * Np + b0 + bb) * np + row] = acc[bb];
      }
    }
    // gradient rows (c, j, a): A_qv (columns (c, b)) and A_qq (columns (c, j, b))
    for (int t = tid; t < M * D * Np; t += BLK) {
      const int a = t % Np, cj = t / Np, c = cj / D, j = cj % D;
      const int row = M * Np + cj * Np + a;
      for (int b0 = 0; b0 < Np; b0 += 16) {
        double av[16], aq[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) av[i] = aq[i] = 0.0;
        for (int qp = 0; qp < Nq; ++qp) {
          const double *w = pv + (size_t)qp * L.size;
          double ta = 0.0;
          for (int r = 0; r < D; ++r) ta += w[L.WJ + r * D + j] * dphi[((size_t)r * Nq + qp) * Np + a];
          const double tm = w[L.W] * phi[qp * Np + a];
#pragma unroll
          for (int bb = 0; bb < 16; ++bb)
            if (b0 + bb < Np) {
              av[bb] += ta * phi[qp * Np + b0 + bb];
              aq[bb] += tm * phi[qp * Np + b0 + bb];
            }
        }
        for (int bb = 0; bb < 16 && b0 + bb < Np; ++bb) {
          A[(size_t)(c * Np + b0 + bb) * np + row] = av[bb];
          A[(size_t)(M * Np + cj * Np + b0 + bb) * np + row] = aq[bb];
        }
      }
    }
  }
  // element residual rows -> column k_pad of X
  double *R = X + (size_t)kp * np;
  for (int t = tid; t < M * Np; t += BLK) {
    const int a = t % Np, c = t / Np;
    double acc = 0.0;
    for (int qp = 0; qp < Nq; ++qp) {
      const double *w = pv + (size_t)qp * L.size;
      double ta = w[L.Wu + c] * phi[qp * Np + a];
      for (int r = 0; r < D; ++r) ta += w[L.Fr + c * D + r] * dphi[((size_t)r * Nq + qp) * Np + a];
      acc += ta;
    }
    for (int f = 0; f < nf; ++f) {
      const int ia = node_face[a * nf + f];
      if (ia < 0) continue;
      for (int fq = 0; fq < Nfq; ++fq)
        acc += pf[((size_t)f * Nfq + fq) * L.fsize + L.fFf + c] * fphi[((size_t)f * Nfq + fq) * Nfp + ia];
    }
    R[c * Np + a] = acc;
  }
  if (VISC) {
    for (int t = tid; t < M * D * Np; t += BLK) {
      const int a = t % Np, cj = t / Np, c = cj / D, j = cj % D;
      double acc = 0.0;
      for (int qp = 0; qp < Nq; ++qp) {
        const double *w = pv + (size_t)qp * L.size;
        double ta = 0.0;
        for (int r = 0; r < D; ++r) ta += w[L.WJ + r * D + j] * dphi[((size_t)r * Nq + qp) * Np + a];
        acc += w[L.Wq + c * D + j] * phi[qp * Np + a] + w[L.v + c] * ta;
      }
      for (int f = 0; f < nf; ++f) {
        const int ia = node_face[a * nf + f];
        if (ia < 0) continue;
        for (int fq = 0; fq < Nfq; ++fq) {
          const double *w = pf + ((size_t)f * Nfq + fq) * L.fsize;
          acc -= w[L.fWn + j] * w[L.fvh + c] * fphi[((size_t)f * Nfq + fq) * Nfp + ia];
        }
      }
      R[M * Np + cj * Np + a] = acc;
    }
  }
  // B (columns 0..k-1 of X): element rows of face-f nodes against trace block f
  const int MF = M * Nfp;
  for (int t = tid; t < nf * M * Nfp; t += BLK) {
    const int ia = t % Nfp, c = (t / Nfp) % M, f = t / (Nfp * M);
    const int row = c * Np + fnodes[f * Nfp + ia];
    for (int cp = 0; cp < M; ++cp)
      for (int ib = 0; ib < Nfp; ++ib) {
        double acc = 0.0;
        for (int fq = 0; fq < Nfq; ++fq) {
          const double *fpr = fphi + ((size_t)f * Nfq + fq) * Nfp;
          acc += pf[((size_t)f * Nfq + fq) * L.fsize + L.fFh + c * M + cp] * fpr[ia] * fpr[ib];
        }
        X[(size_t)(f * MF + cp * Nfp + ib) * np + row] = acc;
      }
  }
  if (VISC) {
    for (int t = tid; t < nf * M * D * Nfp; t += BLK) {
      const int ia = t % Nfp, cj = (t / Nfp) % (M * D), f = t / (Nfp * M * D);
      const int c = cj / D, j = cj % D;
      const int row = M * Np + cj * Np + fnodes[f * Nfp + ia];
      for (int ib = 0; ib < Nfp; ++ib) {
        double acc = 0.0;
        for (int fq = 0; fq < Nfq; ++fq) {
          const double *fpr = fphi + ((size_t)f * Nfq + fq) * Nfp;
          acc -= pf[((size_t)f * Nfq + fq) * L.fsize + L.fWn + j] * fpr[ia] * fpr[ib];
        }
        X[(size_t)(f * MF + c * Nfp + ib) * np + row] = acc;
      }
    }
  }
  // trace rows (f, c, b): C, D and R_tr
  for (int t = tid; t < nf * M * Nfp; t += BLK) {
    const int ib = t % Nfp, c = (t / Nfp) % M, f = t / (Nfp * M);
    const int row = f * MF + c * Nfp + ib;
    const bool dir = fbc[f] != 0;
    double rt = 0.0;
    for (int fq = 0; fq < Nfq; ++fq) {
      const double *w = pf + ((size_t)f * Nfq + fq) * L.fsize;
      rt += (dir ? w[L.fFd + c] : w[L.fFf + c]) * fphi[((size_t)f * Nfq + fq) * Nfp + ib];
    }
    Rt[row] = rt;
    for (int cp = 0; cp < M; ++cp)
      for (int i2 = 0; i2 < Nfp; ++i2) {
        double dd = 0.0, cv = 0.0;
        for (int fq = 0; fq < Nfq; ++fq) {
          const double *w = pf + ((size_t)f * Nfq + fq) * L.fsize;
          const double *fpr = fphi + ((size_t)f * Nfq + fq) * Nfp;
          const double bb = fpr[ib] * fpr[i2];
          if (dir) {
            if (cp == c) dd += w[L.fW] * bb;
          } else {
            dd += w[L.fFh + c * M + cp] * bb;
            cv += w[L.fFv + c * M + cp] * bb;
          }
        }
        Dm[(size_t)(f * MF + cp * Nfp + i2) * kp + row] = dd;
        C[(size_t)(cp * Np + fnodes[f * Nfp + i2]) * kp + row] = cv;
      }
    if (VISC && !dir)
      for (int s = 0; s < M * D; ++s)
        for (int i2 = 0; i2 < Nfp; ++i2) {
          double cq = 0.0;
          for (int fq = 0; fq < Nfq; ++fq) {
            const double *w = pf + ((size_t)f * Nfq + fq) * L.fsize;
            const double *fpr = fphi + ((size_t)f * Nfq + fq) * Nfp;
            cq += w[L.fFq + c * (M * D) + s] * fpr[ib] * fpr[i2];
          }
          C[(size_t)(M * Np + s * Np + fnodes[f * Nfp + i2]) * kp + row] = cq;
        }
  }
}

// Zero the trace rows (f, c, b) of C, D and R_tr of the face nodes marked in row_drop, one
// workgroup per element of the chunk; index i runs over (row, column) with the row fastest
// (columns n of C, then k of D, then R_tr), matching the column-major blocks.
__global__ __launch_bounds__(256) void k_drop_rows(DevPlan P, int e0) {
  const int el = blockIdx.x, e = e0 + el;
  const int n = P.n, k = P.k, kp = P.k_pad, Nfp = P.Nfp, MF = P.m * P.Nfp;
  const int *drop = P.row_drop + (size_t)e * P.nf * Nfp;
  double *C = P.C + (size_t)el * P.n_pad * kp;
  double *Dm = P.D + (size_t)el * kp * kp;
  double *Rt = P.Rt + (size_t)el * kp;
  const size_t total = (size_t)k * (n + k + 1);
  for (size_t i = threadIdx.x; i < total; i += 256) {
    const int row = (int)(i % k), col = (int)(i / k);
    if (!drop[(row / MF) * Nfp + row % Nfp]) continue;
    if (col < n)
      C[(size_t)col * kp + row] = 0.0;
    else if (col < n + k)
      Dm[(size_t)(col - n) * kp + row] = 0.0;
    else
      Rt[row] = 0.0;
  }
}

__global__ void k_export(DevPlan P, int e0, int ec, double *A, double *B, double *C, double *Dm, double *Rl,
                         double *Rtr) {
  const int el = blockIdx.x, e = e0 + el;
  const int n = P.n, k = P.k, np = P.n_pad, kp = P.k_pad, kx = P.kx;
  const double *Ai = P.A + (size_t)el * np * np;
  const double *Xi = P.X + (size_t)el * kx * np;
  const double *Ci = P.C + (size_t)el * np * kp;
  const double *Di = P.D + (size_t)el * kp * kp;
  const double *Ri = P.Rt + (size_t)el * kp;
  for (size_t i = threadIdx.x; i < (size_t)n * n; i += blockDim.x) {
    size_t col = i / n, row = i % n;
    if (A) A[(size_t)e * n * n + i] = Ai[col * np + row];
  }
  for (size_t i = threadIdx.x; i < (size_t)n * k; i += blockDim.x) {
    size_t col = i / n, row = i % n;
    if (B) B[(size_t)e * n * k + i] = Xi[col * np + row];
  }
  for (size_t i = threadIdx.x; i < (size_t)n * k; i += blockDim.x) {
    size_t col = i / k, row = i % k;
    if (C) C[(size_t)e * n * k + i] = Ci[col * kp + row];
  }
  for (size_t i = threadIdx.x; i < (size_t)k * k; i += blockDim.x) {
    size_t col = i / k, row = i % k;
    if (Dm) Dm[(size_t)e * k * k + i] = Di[col * kp + row];
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (Rl) Rl[(size_t)e * n + i] = Xi[(size_t)kp * np + i];
  for (int i = threadIdx.x; i < k; i += blockDim.x)
    if (Rtr) Rtr[(size_t)e * k + i] = Ri[i];
}

// The inverse of k_export: caller blocks (compact, column-major) into the workspace of the
// condensation, with the padding of A set to the identity and every other padding entry zero.
__global__ void k_import(DevPlan P, int e0, const double *A, const double *B, const double *C, const double *Dm,
                         const double *Rl, const double *Rtr) {
  const int el = blockIdx.x, e = e0 + el;
  const int n = P.n, k = P.k, np = P.n_pad, kp = P.k_pad, kx = P.kx;
  double *Ai = P.A + (size_t)el * np * np;
  double *Xi = P.X + (size_t)el * kx * np;
  double *Ci = P.C + (size_t)el * np * kp;
  double *Di = P.D + (size_t)el * kp * kp;
  double *Ri = P.Rt + (size_t)el * kp;
  for (size_t i = threadIdx.x; i < (size_t)np * np; i += blockDim.x) {
    const size_t col = i / np, row = i % np;
    Ai[i] = (row < (size_t)n && col < (size_t)n) ? A[(size_t)e * n * n + col * n + row] : (row == col ? 1.0 : 0.0);
  }
  for (size_t i = threadIdx.x; i < (size_t)kx * np; i += blockDim.x) {
    const size_t col = i / np, row = i % np;
    double v = 0.0;
    if (row < (size_t)n) {
      if (col < (size_t)k) v = B[(size_t)e * n * k + col * n + row];
      else if (col == (size_t)kp) v = Rl[(size_t)e * n + row];
    }
    Xi[i] = v;
  }
  for (size_t i = threadIdx.x; i < (size_t)np * kp; i += blockDim.x) {
    const size_t col = i / kp, row = i % kp;
    Ci[i] = (row < (size_t)k && col < (size_t)n) ? C[(size_t)e * n * k + col * k + row] : 0.0;
  }
  for (size_t i = threadIdx.x; i < (size_t)kp * kp; i += blockDim.x) {
    const size_t col = i / kp, row = i % kp;
    Di[i] = (row < (size_t)k && col < (size_t)k) ? Dm[(size_t)e * k * k + col * k + row] : 0.0;
  }
  for (int i = threadIdx.x; i < kp; i += blockDim.x) Ri[i] = i < k ? Rtr[(size_t)e * k + i] : 0.0;
}

// FP64 fallback of the element-level refinement: column 0 of X <- b (rows of the element, zero
// padding), so the right-looking solve leaves A^-1 b there ...
__global__ void k_fallback_rhs(DevPlan P, int e0, const double *b) {
  const int el = blockIdx.x, e = e0 + el;
  double *X0 = P.X + (size_t)el * P.kx * P.n_pad;
  for (int i = threadIdx.x; i < P.n_pad; i += blockDim.x) X0[i] = i < P.n ? b[(size_t)e * P.n + i] : 0.0;
}

// ... and dx[e] <- that column for the elements whose refinement ratio exceeds tol (counted).
__global__ void k_fallback_take(DevPlan P, int e0, const double *ratio, double tol, double *dx, int *count) {
  const int el = blockIdx.x, e = e0 + el;
  if (!(ratio[e] > tol)) return;   // whole workgroup
  const double *X0 = P.X + (size_t)el * P.kx * P.n_pad;
  for (int i = threadIdx.x; i < P.n; i += blockDim.x) dx[(size_t)e * P.n + i] = X0[i];
  if (threadIdx.x == 0) atomicAdd(count, 1);
}

__global__ void k_fill_int(int32_t *p, int n, int val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}
__global__ void k_fill_double(double *p, size_t n, double val) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}

template <int D, bool VISC>
hipError_t points_t(const DevPlan &P, int e0, int ec, const double *v, const double *q, const double *vhat,
                    const double *ustar, const double *vbc, int32_t *status, hipStream_t s) {
  int nv = ec * P.Nq;
  hipLaunchKernelGGL((k_vol_points<D, VISC>), dim3((nv + 127) / 128), dim3(128), 0, s, P, e0, ec, v, q, ustar,
                     status);
  hipError_t e = hipGetLastError();
  if (e) return e;
  int nfp = ec * P.nf * P.Nfq;
  if (P.sigma_s == 2)
    hipLaunchKernelGGL((k_face_points<D, VISC, true>), dim3((nfp + 127) / 128), dim3(128), 0, s, P, e0, ec, v, q,
                       vhat, vbc, status);
  else
    hipLaunchKernelGGL((k_face_points<D, VISC, false>), dim3((nfp + 127) / 128), dim3(128), 0, s, P, e0, ec, v, q,
                       vhat, vbc, status);
  return hipGetLastError();
}

template <int D, bool VISC>
hipError_t contract_t(const DevPlan &P, int e0, int ec, hipStream_t s) {
  hipLaunchKernelGGL((k_contract<D, VISC>), dim3(ec), dim3(BLK), 0, s, P, e0, ec);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_int(int32_t *p, int n, int val, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n, val);
  return hipGetLastError();
}

hipError_t launch_fill_double(double *p, size_t n, double val, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_double, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, val);
  return hipGetLastError();
}

hipError_t launch_points(const DevPlan &P, int e0, int ec, const double *v, const double *q, const double *vhat,
                         const double *ustar, const double *vbc, int32_t *status, hipStream_t s) {
  if (P.dim == 2) {
    return P.viscous ? points_t<2, true>(P, e0, ec, v, q, vhat, ustar, vbc, status, s)
                     : points_t<2, false>(P, e0, ec, v, q, vhat, ustar, vbc, status, s);
  }
  return P.viscous ? points_t<3, true>(P, e0, ec, v, q, vhat, ustar, vbc, status, s)
                   : points_t<3, false>(P, e0, ec, v, q, vhat, ustar, vbc, status, s);
}

hipError_t launch_contract(const DevPlan &P, int e0, int ec, hipStream_t s) {
  if (P.dim == 2) return P.viscous ? contract_t<2, true>(P, e0, ec, s) : contract_t<2, false>(P, e0, ec, s);
  return P.viscous ? contract_t<3, true>(P, e0, ec, s) : contract_t<3, false>(P, e0, ec, s);
}

hipError_t launch_export_blocks(const DevPlan &P, int e0, int ec, double *A, double *B, double *C, double *D,
                                double *Rloc, double *Rtr, hipStream_t s) {
  hipLaunchKernelGGL(k_export, dim3(ec), dim3(256), 0, s, P, e0, ec, A, B, C, D, Rloc, Rtr);
  return hipGetLastError();
}

hipError_t launch_import_blocks(const DevPlan &P, int e0, int ec, const double *A, const double *B, const double *C,
                                const double *D, const double *Rloc, const double *Rtr, hipStream_t s) {
  hipLaunchKernelGGL(k_import, dim3(ec), dim3(256), 0, s, P, e0, A, B, C, D, Rloc, Rtr);
  return hipGetLastError();
}

hipError_t launch_fallback_rhs(const DevPlan &P, int e0, int ec, const double *b, hipStream_t s) {
  hipLaunchKernelGGL(k_fallback_rhs, dim3(ec), dim3(256), 0, s, P, e0, b);
  return hipGetLastError();
}

hipError_t launch_fallback_take(const DevPlan &P, int e0, int ec, const double *ratio, double tol, double *dx,
                                int *count, hipStream_t s) {
  hipLaunchKernelGGL(k_fallback_take, dim3(ec), dim3(256), 0, s, P, e0, ratio, tol, dx, count);
  return hipGetLastError();
}

hipError_t launch_drop_rows(const DevPlan &P, int e0, int ec, hipStream_t s) {
  if (!P.row_drop) return hipSuccess;
  hipLaunchKernelGGL(k_drop_rows, dim3(ec), dim3(256), 0, s, P, e0);
  return hipGetLastError();
}

}  // namespace hdg
