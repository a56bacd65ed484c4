// Learned correction of the block-Jacobi preconditioner (not in the paper).
//
// Every block-Jacobi inverse B_F of the condensed operator is corrected as
//   M_F^-1 = diag(e^a) (B_F + (c U)(c V)^T) diag(e^b),
//   a_i = 0.5 tanh(o_i0), b_i = 0.5 tanh(o_i1), U_ik = tanh(o_i,2+k), V_ik = tanh(o_i,2+R+k),
//   c_i = |B_F,ii|^(1/2),
// o_i = MLP(features of unknown i): 16 -> 32 (tanh) -> 32 (tanh) -> 2 + 2R, FP32, R = 4: a
// rescaling of rows and columns and a rank-R term that couples the unknowns of the block.
// Training minimizes L = sum_v ||x_v - M^-1 K x_v||^2 / sum_v ||x_v||^2 over random vectors
// with Adam, either on a whole system or on a pool of face blocks sampled from many systems;
// these kernels are the features, the network's forward and backward passes, the loss
// gradient, the Adam update, the sampling into a pool and the correction of the inverses.
//
// Parameter vector (float): W1[32][16] b1[32] W2[32][32] b2[32] W3[NO][32] b3[NO], NO = 2 + 2R.
// Rows are block rows: block F, position i -> F*bs + i, i = c*npb + p.
#include <mutex>

#include "hdg_physics.hpp"
#include "hdg_plan.hpp"

namespace hdg {

namespace {

constexpr int NF = 16, NH = 32, RK = 4, NO = 2 + 2 * RK;
constexpr int OW1 = 0, OB1 = OW1 + NH * NF, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NO * NH, NPAR = OB3 + NO;
constexpr float LOGS = 0.25f;   // scale of log10 features

__device__ inline int npb_of(const DevPlan &P) { return P.bj_face ? P.Nfp : 1; }

// features of every row from the assembled (not yet inverted) diagonal blocks
// and the trace state; columns 2 and 3 are completed by k_feat_finish.
template <int D>
__global__ void k_feat_block(DevPlan P, const double *__restrict__ Bd, const double *__restrict__ vhat,
                             float *feat) {
  constexpr int M = D + 2;
  const int blk = blockIdx.x;
  const int bs = P.bj_bs, npb = npb_of(P);
  const double *Bb = Bd + (size_t)blk * bs * bs;
  for (int i = threadIdx.x; i < bs; i += blockDim.x) {
    const int c = i / npb, p = i % npb;
    const int t = P.bj_nodes[(size_t)blk * npb + p];
    double rn = 0.0;
    for (int j = 0; j < bs; ++j) rn += Bb[(size_t)j * bs + i] * Bb[(size_t)j * bs + i];
    float f[NF];
    for (int q = 0; q < NF; ++q) f[q] = 0.f;
    f[0] = LOGS * (float)log10(fabs(Bb[(size_t)i * bs + i]) + 1e-300);
    f[1] = LOGS * (float)log10(sqrt(rn) + 1e-300);
    if (c < 5) f[4 + c] = 1.f;
    if (P.bj_face) {
      const int e = P.bj_ce[blk * 2], fc = P.bj_cf[blk * 2];
      const int bb = P.bj_loc[((size_t)blk * 2) * P.Nfp + p];
      const int a = P.fnodes[fc * P.Nfp + bb];
      int nfc = 0;
      for (int ff = 0; ff < P.nf; ++ff) nfc += P.node_face[a * P.nf + ff] >= 0;
      f[9 + (nfc >= 3 ? 2 : nfc - 1)] = 1.f;
      (void)e;
    }
    double vv[M];
    for (int cc = 0; cc < M; ++cc) vv[cc] = vhat[(size_t)cc * P.n_trace + t];
    if (vv[M - 1] < 0.0) {
      Prim<D, double> s = prim_of_v<D, double>(vv, P.gamma);
      double v2 = 0.0;
      for (int j = 0; j < D; ++j) v2 += s.V[j] * s.V[j];
      f[12] = (float)sqrt(v2 / (P.gamma * s.p / s.rho));
      f[13] = LOGS * (float)log10(s.p);
      f[14] = LOGS * (float)log10(s.rho);
    }
    f[15] = 1.f;
    float *o = feat + ((size_t)blk * bs + i) * NF;
    for (int q = 0; q < NF; ++q) o[q] = f[q];
  }
}

// coupling^2 of every global row: squared entries of the element Schur rows in
// columns whose trace node lies outside the row's block
template <typename T>
__global__ void k_feat_coupling(DevPlan P, const T *__restrict__ S, const int *__restrict__ tpos, double *coup) {
  const int e = blockIdx.x;
  const int k = P.k, Nfp = P.Nfp, M = P.m, nf = P.nf, npb = npb_of(P), bs = P.bj_bs;
  const int *tm = P.tmap + (size_t)e * nf * Nfp;
  const T *Se = S + (size_t)e * k * k;
  for (int l = threadIdx.x; l < k; l += blockDim.x) {
    const int b = l % Nfp, c = (l / Nfp) % M, f = l / (Nfp * M);
    const int tp = tpos[tm[f * Nfp + b]];
    const int blk = tp / npb, p = tp % npb;
    double acc = 0.0;
    for (int j = 0; j < k; ++j) {
      const int bj = j % Nfp, fj = j / (Nfp * M);
      if (tpos[tm[fj * Nfp + bj]] / npb == blk) continue;
      const double s = (double)Se[(size_t)j * k + l];
      acc += s * s;
    }
    atomicAdd(&coup[(size_t)blk * bs + c * npb + p], acc);
  }
}

__global__ void k_feat_finish(const double *__restrict__ coup, float *feat, size_t N) {
  const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const float lc = LOGS * (float)log10(sqrt(coup[r]) + 1e-300);
  feat[r * NF + 2] = lc;
  feat[r * NF + 3] = lc - feat[r * NF + 1];
}

__device__ inline void mlp_fwd_row(const float *th, const float *x, float *h1, float *h2, float *o) {
  for (int j = 0; j < NH; ++j) {
    float s = th[OB1 + j];
#pragma unroll
    for (int i = 0; i < NF; ++i) s += th[OW1 + j * NF + i] * x[i];
    h1[j] = tanhf(s);
  }
  for (int j = 0; j < NH; ++j) {
    float s = th[OB2 + j];
#pragma unroll 8
    for (int i = 0; i < NH; ++i) s += th[OW2 + j * NH + i] * h1[i];
    h2[j] = tanhf(s);
  }
  for (int j = 0; j < NO; ++j) {
    float s = th[OB3 + j];
#pragma unroll 8
    for (int i = 0; i < NH; ++i) s += th[OW3 + j * NH + i] * h2[i];
    o[j] = s;
  }
}

__global__ __launch_bounds__(256) void k_mlp_fwd(const float *__restrict__ theta, const float *__restrict__ feat,
                                                 size_t N, float *out) {
  __shared__ float th[NPAR];
  for (int i = threadIdx.x; i < NPAR; i += blockDim.x) th[i] = theta[i];
  __syncthreads();
  const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  float x[NF], h1[NH], h2[NH], o[NO];
  for (int i = 0; i < NF; ++i) x[i] = feat[r * NF + i];
  mlp_fwd_row(th, x, h1, h2, o);
  for (int j = 0; j < NO; ++j) out[r * NO + j] = o[j];
}

// Loss and dL/do of one block (bs <= blockDim.x <= 256, thread i = row i): per vector, with
// e = e^b w, t = (cV)^T e, u = B e + (cU) t, y = e^a u, r = x - y, dL/dy = -2 r / x2, then
// du = e^a dy, dt = (cU)^T du, de = B^T du + (cV) dt and dL/da = dy y, dL/dU = du t^T c,
// dL/dV = e dt^T c, dL/db = de e.  xw(v, i) returns (x, w) of row i for vector v.
template <typename XW>
__device__ inline void precond_grad_block(const double *__restrict__ Bb, int bs, const float *__restrict__ ob,
                                          int nvec, double x2, XW xw, float *dOb, double *loss, double *sm) {
  double *ea = sm, *eb = ea + bs, *ew = eb + bs, *du = ew + bs, *c = du + bs, *cU = c + bs, *cV = cU + bs * RK,
         *tt = cV + bs * RK, *dt = tt + RK, *red = dt + RK;
  const int tid = threadIdx.x;
  double ga = 0.0, gb = 0.0, lsum = 0.0, gU[RK], gV[RK], th[NO];
  for (int k = 0; k < RK; ++k) gU[k] = gV[k] = 0.0;
  if (tid < bs) {
    for (int j = 0; j < NO; ++j) th[j] = tanh((double)ob[tid * NO + j]);
    ea[tid] = exp(0.5 * th[0]);
    eb[tid] = exp(0.5 * th[1]);
    c[tid] = sqrt(fabs(Bb[(size_t)tid * bs + tid]));
    for (int k = 0; k < RK; ++k) {
      cU[tid * RK + k] = c[tid] * th[2 + k];
      cV[tid * RK + k] = c[tid] * th[2 + RK + k];
    }
  }
  for (int v = 0; v < nvec; ++v) {
    __syncthreads();
    double xv = 0.0;
    if (tid < bs) {
      const double2 q = xw(v, tid);
      xv = q.x;
      ew[tid] = eb[tid] * q.y;
    }
    __syncthreads();
    if (tid < RK) {
      double t = 0.0;
      for (int j = 0; j < bs; ++j) t += cV[j * RK + tid] * ew[j];
      tt[tid] = t;
    }
    __syncthreads();
    if (tid < bs) {
      double u = 0.0;
      for (int j = 0; j < bs; ++j) u += Bb[(size_t)j * bs + tid] * ew[j];
      for (int k = 0; k < RK; ++k) u += cU[tid * RK + k] * tt[k];
      const double y = ea[tid] * u;
      const double r = xv - y;
      lsum += r * r;
      const double d = -2.0 * r / x2;
      ga += d * y;
      du[tid] = ea[tid] * d;
      for (int k = 0; k < RK; ++k) gU[k] += du[tid] * tt[k] * c[tid];
    }
    __syncthreads();
    if (tid < RK) {
      double t = 0.0;
      for (int i = 0; i < bs; ++i) t += cU[i * RK + tid] * du[i];
      dt[tid] = t;
    }
    __syncthreads();
    if (tid < bs) {
      double de = 0.0;
      for (int i = 0; i < bs; ++i) de += Bb[(size_t)tid * bs + i] * du[i];
      for (int k = 0; k < RK; ++k) {
        de += cV[tid * RK + k] * dt[k];
        gV[k] += ew[tid] * dt[k] * c[tid];
      }
      gb += de * ew[tid];
    }
  }
  if (tid < bs) {
    float *o = dOb + (size_t)tid * NO;
    o[0] = (float)(ga * 0.5 * (1.0 - th[0] * th[0]));
    o[1] = (float)(gb * 0.5 * (1.0 - th[1] * th[1]));
    for (int k = 0; k < RK; ++k) {
      o[2 + k] = (float)(gU[k] * (1.0 - th[2 + k] * th[2 + k]));
      o[2 + RK + k] = (float)(gV[k] * (1.0 - th[2 + RK + k] * th[2 + RK + k]));
    }
  }
  // block sum of the loss
  red[tid] = lsum;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) atomicAdd(loss, red[0] / x2);
}

__host__ __device__ inline size_t precond_grad_lds(int bs, int nt) {
  return ((size_t)5 * bs + 2 * (size_t)bs * RK + 2 * RK + nt) * sizeof(double);
}

// whole system: x and w of a row through its global trace unknown
__global__ void k_precond_grad(DevPlan P, const double *__restrict__ Binv, const float *__restrict__ o,
                               const double *__restrict__ X, const double *__restrict__ Wv, int nvec, double x2,
                               float *dO, double *loss) {
  extern __shared__ double sm[];
  const int blk = blockIdx.x, bs = P.bj_bs, npb = npb_of(P);
  const size_t NT = (size_t)P.n_trace, NV = (size_t)P.m * NT;
  int gidx = 0;
  if ((int)threadIdx.x < bs) {
    const int c = threadIdx.x / npb, p = threadIdx.x % npb;
    gidx = (int)(c * NT) + P.bj_nodes[(size_t)blk * npb + p];
  }
  const auto xw = [&](int v, int) { return make_double2(X[(size_t)v * NV + gidx], Wv[(size_t)v * NV + gidx]); };
  precond_grad_block(Binv + (size_t)blk * bs * bs, bs, o + (size_t)blk * bs * NO, nvec, x2, xw,
                     dO + (size_t)blk * bs * NO, loss, sm);
}

// pool of sampled blocks: x and w in block-row order, vector v at v * ld
__global__ void k_pool_grad(int bs, const double *__restrict__ Binv, const float *__restrict__ o,
                            const double *__restrict__ X, const double *__restrict__ Wv, size_t ld, int nvec,
                            double x2, float *dO, double *loss) {
  extern __shared__ double sm[];
  const size_t blk = blockIdx.x;
  const auto xw = [&](int v, int i) {
    const size_t r = (size_t)v * ld + blk * bs + i;
    return make_double2(X[r], Wv[r]);
  };
  precond_grad_block(Binv + blk * bs * bs, bs, o + blk * bs * NO, nvec, x2, xw, dO + blk * bs * NO, loss, sm);
}

// sampled blocks of a system into a pool (block q of the sample -> pool block b0 + q): the
// block inverse, the rows' features, and x and w of its rows for every vector
__global__ void k_pool_extract(DevPlan P, const double *__restrict__ Binv, const float *__restrict__ feat,
                               const double *__restrict__ X, const double *__restrict__ Wv, int nvec,
                               const int *__restrict__ sel, size_t b0, size_t ld, double *pB, float *pfeat,
                               double *pX, double *pW) {
  const int q = blockIdx.x, blk = sel[q], bs = P.bj_bs, npb = npb_of(P);
  const size_t NT = (size_t)P.n_trace, NV = (size_t)P.m * NT, dstb = b0 + q;
  for (int t = threadIdx.x; t < bs * bs; t += blockDim.x)
    pB[dstb * bs * bs + t] = Binv[(size_t)blk * bs * bs + t];
  for (int t = threadIdx.x; t < bs * NF; t += blockDim.x)
    pfeat[dstb * bs * NF + t] = feat[(size_t)blk * bs * NF + t];
  for (int t = threadIdx.x; t < bs * nvec; t += blockDim.x) {
    const int i = t % bs, v = t / bs;
    const int c = i / npb, p = i % npb;
    const size_t g = c * NT + P.bj_nodes[(size_t)blk * npb + p];
    pX[(size_t)v * ld + dstb * bs + i] = X[(size_t)v * NV + g];
    pW[(size_t)v * ld + dstb * bs + i] = Wv[(size_t)v * NV + g];
  }
}

// Backward: 64 rows per workgroup; activations and deltas in LDS, then every
// thread accumulates its share of the parameters over the rows.
constexpr int BR = 64;

__global__ __launch_bounds__(BR) void k_mlp_bwd(const float *__restrict__ theta, const float *__restrict__ feat,
                                                const float *__restrict__ dO, size_t N, float *partial) {
  __shared__ float th[NPAR];
  __shared__ float sx[BR][NF + 1], sh1[BR][NH + 1], sh2[BR][NH + 1], sd1[BR][NH + 1], sd2[BR][NH + 1],
      so[BR][NO];
  const int tid = threadIdx.x;
  for (int i = tid; i < NPAR; i += BR) th[i] = theta[i];
  __syncthreads();
  const size_t r = (size_t)blockIdx.x * BR + tid;
  float x[NF], h1[NH], h2[NH], o[NO], g[NO];
  if (r < N) {
    for (int i = 0; i < NF; ++i) x[i] = feat[r * NF + i];
    for (int q = 0; q < NO; ++q) g[q] = dO[r * NO + q];
  } else {
    for (int i = 0; i < NF; ++i) x[i] = 0.f;
    for (int q = 0; q < NO; ++q) g[q] = 0.f;
  }
  mlp_fwd_row(th, x, h1, h2, o);
  float d2[NH], d1[NH];
  for (int j = 0; j < NH; ++j) {
    float s = 0.f;
    for (int q = 0; q < NO; ++q) s += g[q] * th[OW3 + q * NH + j];
    d2[j] = s * (1.f - h2[j] * h2[j]);
  }
  for (int j = 0; j < NH; ++j) {
    float s = 0.f;
    for (int q = 0; q < NH; ++q) s += d2[q] * th[OW2 + q * NH + j];
    d1[j] = s * (1.f - h1[j] * h1[j]);
  }
  for (int i = 0; i < NF; ++i) sx[tid][i] = x[i];
  for (int j = 0; j < NH; ++j) {
    sh1[tid][j] = h1[j];
    sh2[tid][j] = h2[j];
    sd1[tid][j] = d1[j];
    sd2[tid][j] = d2[j];
  }
  for (int q = 0; q < NO; ++q) so[tid][q] = g[q];
  __syncthreads();
  float *out = partial + (size_t)blockIdx.x * NPAR;
  for (int p = tid; p < NPAR; p += BR) {
    float acc = 0.f;
    if (p < OB1) {
      const int j = (p - OW1) / NF, i = (p - OW1) % NF;
      for (int q = 0; q < BR; ++q) acc += sd1[q][j] * sx[q][i];
    } else if (p < OW2) {
      const int j = p - OB1;
      for (int q = 0; q < BR; ++q) acc += sd1[q][j];
    } else if (p < OB2) {
      const int j = (p - OW2) / NH, i = (p - OW2) % NH;
      for (int q = 0; q < BR; ++q) acc += sd2[q][j] * sh1[q][i];
    } else if (p < OW3) {
      const int j = p - OB2;
      for (int q = 0; q < BR; ++q) acc += sd2[q][j];
    } else if (p < OB3) {
      const int j = (p - OW3) / NH, i = (p - OW3) % NH;
      for (int q = 0; q < BR; ++q) acc += so[q][j] * sh2[q][i];
    } else {
      const int j = p - OB3;
      for (int q = 0; q < BR; ++q) acc += so[q][j];
    }
    out[p] = acc;
  }
}

// out[p] = sum_b partial[b][p]  (FP64 accumulation)
__global__ void k_reduce_cols(const float *__restrict__ partial, int nb, float *out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) acc += partial[(size_t)b * NPAR + p];
  out[p] = (float)acc;
}

__global__ void k_adam(float *theta, const float *__restrict__ g, float *m, float *v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  const float mm = b1 * m[p] + (1.f - b1) * g[p];
  const float vv = b2 * v[p] + (1.f - b2) * g[p] * g[p];
  m[p] = mm;
  v[p] = vv;
  theta[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// M_F^-1 in place of B_F: entry (i, j) <- e^(a_i) (B_ij + c_i c_j sum_k U_ik V_jk) e^(b_j)
// (column-major blocks; the diagonal, for c, is read before any entry changes)
__global__ void k_correct_blocks(DevPlan P, double *B, const float *__restrict__ o) {
  __shared__ double c[256], ea[256], eb[256], cu[256 * RK], cv[256 * RK];
  const int blk = blockIdx.x, bs = P.bj_bs;
  double *Bb = B + (size_t)blk * bs * bs;
  const float *ob = o + (size_t)blk * bs * NO;
  for (int i = threadIdx.x; i < bs; i += blockDim.x) {
    c[i] = sqrt(fabs(Bb[(size_t)i * bs + i]));
    ea[i] = exp(0.5 * tanh((double)ob[i * NO]));
    eb[i] = exp(0.5 * tanh((double)ob[i * NO + 1]));
    for (int k = 0; k < RK; ++k) {
      cu[i * RK + k] = c[i] * tanh((double)ob[i * NO + 2 + k]);
      cv[i * RK + k] = c[i] * tanh((double)ob[i * NO + 2 + RK + k]);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < bs * bs; t += blockDim.x) {
    const int i = t % bs, j = t / bs;
    double corr = 0.0;
    for (int k = 0; k < RK; ++k) corr += cu[i * RK + k] * cv[j * RK + k];
    Bb[t] = ea[i] * (Bb[t] + corr) * eb[j];
  }
}

}  // namespace

int learn_nparams() { return NPAR; }

int learn_outputs() { return NO; }

hipError_t launch_feat(const DevPlan &P, const double *Bd, const void *S, int s_f32, const double *vhat,
                       const int *tpos, double *coup, float *feat, hipStream_t s) {
  const size_t N = (size_t)P.bj_nblk * P.bj_bs;
  if (P.dim == 2) hipLaunchKernelGGL(k_feat_block<2>, dim3(P.bj_nblk), dim3(64), 0, s, P, Bd, vhat, feat);
  else hipLaunchKernelGGL(k_feat_block<3>, dim3(P.bj_nblk), dim3(64), 0, s, P, Bd, vhat, feat);
  hipError_t e = hipGetLastError();
  if (!e) e = launch_fill_double(coup, N, 0.0, s);
  if (e) return e;
  if (s_f32)
    hipLaunchKernelGGL(k_feat_coupling<float>, dim3(P.n_elem), dim3(256), 0, s, P, static_cast<const float *>(S),
                       tpos, coup);
  else
    hipLaunchKernelGGL(k_feat_coupling<double>, dim3(P.n_elem), dim3(256), 0, s, P,
                       static_cast<const double *>(S), tpos, coup);
  e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_feat_finish, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, coup, feat, N);
  return hipGetLastError();
}

hipError_t launch_mlp_fwd(const float *theta, const float *feat, size_t N, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, theta, feat, N, out);
  return hipGetLastError();
}

static int grad_threads(int bs) { return bs <= 64 ? 64 : (bs <= 128 ? 128 : 256); }

hipError_t launch_precond_grad(const DevPlan &P, const double *Binv, const float *o, const double *X,
                               const double *Wv, int nvec, double x2, float *dO, double *loss, hipStream_t s) {
  const int bs = P.bj_bs, nt = grad_threads(bs);
  if (bs > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_precond_grad, dim3(P.bj_nblk), dim3(nt), precond_grad_lds(bs, nt), s, P, Binv, o, X, Wv,
                     nvec, x2, dO, loss);
  return hipGetLastError();
}

hipError_t launch_pool_grad(int nblk, int bs, const double *Binv, const float *o, const double *X, const double *Wv,
                            size_t ld, int nvec, double x2, float *dO, double *loss, hipStream_t s) {
  const int nt = grad_threads(bs);
  if (bs > 256 || nblk < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pool_grad, dim3(nblk), dim3(nt), precond_grad_lds(bs, nt), s, bs, Binv, o, X, Wv, ld, nvec,
                     x2, dO, loss);
  return hipGetLastError();
}

hipError_t launch_pool_extract(const DevPlan &P, const double *Binv, const float *feat, const double *X,
                               const double *Wv, int nvec, const int *sel, int nsel, size_t b0, size_t ld,
                               double *pB, float *pfeat, double *pX, double *pW, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_extract, dim3(nsel), dim3(256), 0, s, P, Binv, feat, X, Wv, nvec, sel, b0, ld, pB, pfeat,
                     pX, pW);
  return hipGetLastError();
}

size_t learn_partial_floats(size_t N) { return ((N + BR - 1) / BR) * NPAR; }

hipError_t launch_mlp_bwd(const float *theta, const float *feat, const float *dO, size_t N, float *partial,
                          float *grad, hipStream_t s) {
  const unsigned nb = (unsigned)((N + BR - 1) / BR);
  hipLaunchKernelGGL(k_mlp_bwd, dim3(nb), dim3(BR), 0, s, theta, feat, dO, N, partial);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_reduce_cols, dim3((NPAR + 255) / 256), dim3(256), 0, s, partial, (int)nb, grad);
  return hipGetLastError();
}

// Scratch of hdg_learn_backward_noalloc: the per-workgroup partial gradients of k_mlp_bwd in a
// file-scope device array (each GPU the library runs on holds its own copy until the process
// ends).  In host code `scratch` names a host-side stand-in; its device address is resolved once
// per device with hipGetSymbolAddress (with that device current) and only that address is used.
constexpr size_t NOALLOC_SCRATCH_FLOATS = size_t(8) << 20;   // 32 MiB
static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];
constexpr int NOALLOC_MAX_DEV = 64;
static float *g_scratch_ptr[NOALLOC_MAX_DEV];
static std::mutex g_scratch_mu;

static hipError_t noalloc_scratch(float **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<float *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

size_t learn_noalloc_max_rows() { return NOALLOC_SCRATCH_FLOATS / NPAR * BR; }

hipError_t launch_mlp_bwd_noalloc(const float *theta, const float *feat, const float *dO, size_t N, float *grad,
                                  hipStream_t s) {
  if (learn_partial_floats(N) > NOALLOC_SCRATCH_FLOATS) return hipErrorInvalidValue;
  float *ptr = nullptr;
  hipError_t e = noalloc_scratch(&ptr);
  if (e) return e;
  // every partial the reduction reads is written by this call's k_mlp_bwd (one row of NPAR per
  // workgroup), so nothing left by an earlier call is read and nothing needs clearing
  return launch_mlp_bwd(theta, feat, dO, N, ptr, grad, s);
}

hipError_t launch_adam(float *theta, const float *g, float *m, float *v, int t, float lr, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((NPAR + 255) / 256), dim3(256), 0, s, theta, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_scale_blocks(const DevPlan &P, double *B, const float *o, hipStream_t s) {
  if (P.bj_bs > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_correct_blocks, dim3(P.bj_nblk), dim3(256), 0, s, P, B, o);
  return hipGetLastError();
}

}  // namespace hdg
