// Element-local elimination of the gradient unknowns q before the dense
// condensation (Navier-Stokes only).
//
// The q rows of the element block are the weak gradient equations (Sec. 3,
// the equation of the auxiliary variable): A_qq = I_{m d} (x) M with M the
// element mass matrix, and A_qv holds, in the (c, j) row block and the c column
// block, the same weak-derivative matrix G_j for every component c.  With
// H_j = M^-1 G_j and W = A_qq^-1 [B_q | R_q]:
//   A^ = A_vv - A_vq A_qq^-1 A_qv     (column block c: A_vv - sum_j A_vq(c, j) H_j)
//   B^ = B_v  - A_vq W_B,  r^ = R_v - A_vq W_R
//   C^ = C_v  - C_q A_qq^-1 A_qv,  D^ = D - C_q W_B,  R^_tr = R_tr - C_q W_R
// and the condensation of (A^, [B^ r^], C^, D^, R^_tr) gives the same S, g and
// v rows of Y, z as the full block; the q rows follow from
//   Y_q = W_B - A_qq^-1 A_qv Y_v,   z_q = W_R - A_qq^-1 A_qv z_v.
// A column of B_q (trace unknown (f, c, b)) only touches the q rows of its own
// component c, so W_B has D N_p nonzeros per column.
#include "hdg_plan.hpp"

namespace hdg {

namespace {

constexpr int QT = 512;   // threads per workgroup
constexpr int QCB = 16;   // right-hand-side columns per pass

// LDS carve-up (doubles): mass matrix inverse, H_j, and a region shared by the
// Gauss-Jordan work array and the W columns of a pass.
struct QLds {
  int mi, hh, w, xs, total;
};

__host__ __device__ inline QLds q_lds(int Np, int D, int M, int ntc) {
  QLds L;
  L.mi = 0;
  L.hh = Np * Np;
  L.w = L.hh + D * Np * Np;
  const int gj = Np * 2 * Np;
  const int wc = QCB * D * Np + (M * D * Np > QCB * M * Np ? M * D * Np : QCB * M * Np);
  const int rcb = ((D * Np + 3) & ~3) * 7 * 16;   // R_c of the q elimination (QCT column tiles)
  int w = gj > wc ? gj : wc;
  if (rcb > w) w = rcb;
  L.xs = L.w + w;
  // staged q rows of X: the residual (M D Np), a component's trace columns (ntc x D Np)
  // or the columns of a recovery pass (QCB x D Np)
  int nq = M * D * Np;
  if (ntc * D * Np > nq) nq = ntc * D * Np;
  if (QCB * D * Np > nq) nq = QCB * D * Np;
  L.total = L.xs + nq;
  return L;
}

// component of trace column col (trace order f (m Nfp) + c Nfp + b)
__device__ inline int trace_comp(int col, int M, int Nfp) { return (col % (M * Nfp)) / Nfp; }

// M^-1 (Gauss-Jordan on [M | I], no pivoting: M is symmetric positive definite)
// and H_j = M^-1 G_j into LDS; both also stored per element for the recovery.
__device__ void mass_and_h(const DevPlan &P, const double *A, double *mi, double *hh, double *aug, double *MH) {
  const int Np = P.Np, D = P.dim, np = P.n_pad, nv = P.m * Np;
  const int tid = threadIdx.x;
  const int w2 = 2 * Np;
  // aug[a][0..Np) = M[a][:], aug[a][Np..2Np) = I; M[a][b] = A(q row (0,0,a), q col (0,0,b))
  for (int t = tid; t < Np * w2; t += QT) {
    const int a = t / w2, b = t % w2;
    aug[t] = b < Np ? A[(size_t)(nv + b) * np + nv + a] : (b - Np == a ? 1.0 : 0.0);
  }
  __syncthreads();
  double *fcol = mi;   // [Np] column factors (mi is written after the elimination)
  for (int p = 0; p < Np; ++p) {
    const double piv = aug[p * w2 + p];
    __syncthreads();
    for (int b = tid; b < w2; b += QT) aug[p * w2 + b] /= piv;
    for (int a = tid; a < Np; a += QT) fcol[a] = aug[a * w2 + p];
    __syncthreads();
    for (int t = tid; t < Np * w2; t += QT) {
      const int a = t / w2, b = t % w2;
      if (a != p) aug[t] -= fcol[a] * aug[p * w2 + b];
    }
    __syncthreads();
  }
  for (int t = tid; t < Np * Np; t += QT) {
    const int a = t % Np, b = t / Np;   // column-major mi[b * Np + a] = M^-1[a][b]
    mi[t] = aug[a * w2 + Np + b];
  }
  __syncthreads();
  // H_j[a][b] = sum_a' M^-1[a][a'] G_j[a'][b], G_j[a'][b] = A(q row (0, j, a'), v col (0, b))
  for (int t = tid; t < D * Np * Np; t += QT) {
    const int a = t % Np, b = (t / Np) % Np, j = t / (Np * Np);
    const double *g = A + (size_t)b * np + nv + j * Np;
    double acc = 0.0;
    for (int q = 0; q < Np; ++q) acc += mi[q * Np + a] * g[q];
    hh[t] = acc;
  }
  __syncthreads();
  for (int t = tid; t < (1 + D) * Np * Np; t += QT) MH[t] = t < Np * Np ? mi[t] : hh[t - Np * Np];
}

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma4(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Per element; for each component c the products of the q columns of c with
// R_c = [H (v columns of c) | W_B (trace columns of c)] form one GEMM on the
// FP64 matrix cores: rows = the v rows of A (A_vq) followed by the trace rows
// of C (C_q), K = D N_p, N = N_p + nf N_fp.  Lane l supplies the operand row
// tile*16 + l%16 at k = k0 + l/16 (A operand, streamed from the column-major
// blocks) and R_c[k0 + l/16][ct*16 + l%16] (B operand, LDS); accumulator r of
// lane l is the output (row tile*16 + l/16 + 4r, column ct*16 + l%16).
constexpr int QCT = 7;   // column tiles of R_c (N_p + nf N_fp <= 112)

__global__ __launch_bounds__(QT) void k_qelim(DevPlan P, QElimArgs Q) {
  extern __shared__ double sm[];
  const int el = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int Np = P.Np, D = P.dim, M = P.m, np = P.n_pad, kp = P.k_pad, kx = P.kx, k = P.k, Nfp = P.Nfp, nf = P.nf;
  const int nv = M * Np, nr = Q.nr_pad, DN = D * Np, MF = M * Nfp;
  const double *A = P.A + (size_t)el * np * np;
  const double *X = P.X + (size_t)el * kx * np;
  const double *C = P.C + (size_t)el * np * kp;
  const double *Dm = P.D + (size_t)el * kp * kp;
  const double *Rt = P.Rt + (size_t)el * kp;
  double *Ar = Q.A + (size_t)el * nr * nr;
  double *Xr = Q.X + (size_t)el * kx * nr;
  double *Cr = Q.C + (size_t)el * nr * kp;
  double *Dr = Q.D + (size_t)el * kp * kp;
  double *Rtr = Q.Rt + (size_t)el * kp;
  double *MH = Q.MH + (size_t)el * (1 + D) * Np * Np;
  const QLds L = q_lds(Np, D, M, nf * Nfp);
  double *mi = sm + L.mi, *hh = sm + L.hh, *rc = sm + L.w, *xs = sm + L.xs;
  mass_and_h(P, A, mi, hh, rc, MH);

  const int ncol = Np + nf * Nfp;          // columns of R_c
  const int nrow = nv + kp;                // operand rows: A_vq then C_q
  const int nrt = (nrow + 15) / 16;
  const int K4 = (DN + 3) & ~3;
  const int ntc = nf * Nfp;                // trace columns of one component
  for (int c = 0; c < M; ++c) {
    __syncthreads();
    // B_q rows of component c of its trace columns, xs[fi][ja] (contiguous in the column)
    for (int t = tid; t < ntc * DN; t += QT) {
      const int fi = t / DN, ja = t % DN;
      xs[t] = X[(size_t)((fi / Nfp) * MF + c * Nfp + fi % Nfp) * np + nv + c * DN + ja];
    }
    __syncthreads();
    // R_c[(j, a)][col]: H_j[a][b] for col = b < Np; W_B for trace column f Nfp + ib of component c
    for (int t = tid; t < K4 * QCT * 16; t += QT) {
      const int col = t % (QCT * 16), ja = t / (QCT * 16);
      double val = 0.0;
      if (ja < DN && col < ncol) {
        const int j = ja / Np, a = ja % Np;
        if (col < Np) {
          val = hh[(j * Np + col) * Np + a];
        } else {
          const double *xq = xs + (col - Np) * DN + j * Np;
          for (int q = 0; q < Np; ++q) val += mi[q * Np + a] * xq[q];
        }
      }
      rc[t] = val;   // rc[ja][col], row stride QCT * 16
    }
    __syncthreads();
    for (int rt = wave; rt < nrt; rt += QT / 64) {
      const int row = rt * 16 + li;   // operand row of this lane
      const double *src = nullptr;    // column (nv + c DN + ja) of A or C at this row
      size_t ld = 0;
      if (row < nv) {
        src = A + (size_t)(nv + c * DN) * np + row;
        ld = np;
      } else if (row < nrow) {
        src = C + (size_t)(nv + c * DN) * kp + (row - nv);
        ld = kp;
      }
      d4 acc[QCT];
#pragma unroll
      for (int ct = 0; ct < QCT; ++ct) acc[ct] = d4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < K4; k0 += 4) {
        const int ja = k0 + lk;
        const double av = (src && ja < DN) ? src[(size_t)ja * ld] : 0.0;
        const double *rr = rc + ja * (QCT * 16) + li;
#pragma unroll
        for (int ct = 0; ct < QCT; ++ct) acc[ct] = mfma4(av, rr[ct * 16], acc[ct]);
      }
      // outputs: original entry minus the product
#pragma unroll
      for (int ct = 0; ct < QCT; ++ct) {
        const int col = ct * 16 + li;
        if (col >= ncol) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int orow = rt * 16 + lk + 4 * r;
          if (orow >= nrow) continue;
          const double v = acc[ct][r];
          if (col < Np) {
            const int cv = c * Np + col;
            if (orow < nv) Ar[(size_t)cv * nr + orow] = A[(size_t)cv * np + orow] - v;
            else Cr[(size_t)cv * kp + orow - nv] = C[(size_t)cv * kp + orow - nv] - v;
          } else {
            const int fi = col - Np, tc = (fi / Nfp) * MF + c * Nfp + fi % Nfp;
            if (orow < nv) Xr[(size_t)tc * nr + orow] = X[(size_t)tc * np + orow] - v;
            else Dr[(size_t)tc * kp + orow - nv] = Dm[(size_t)tc * kp + orow - nv] - v;
          }
        }
      }
    }
  }
  // the residual column (all components): W_R = A_qq^-1 R_q
  __syncthreads();
  double *wr = rc;   // [M D Np]
  for (int t = tid; t < M * DN; t += QT) xs[t] = X[(size_t)kp * np + nv + t];
  __syncthreads();
  for (int t = tid; t < M * DN; t += QT) {
    const int a = t % Np, cj = t / Np;
    const double *xq = xs + cj * Np;
    double acc = 0.0;
    for (int q = 0; q < Np; ++q) acc += mi[q * Np + a] * xq[q];
    wr[t] = acc;
  }
  __syncthreads();
  for (int row = tid; row < nr; row += QT) {
    double val = 0.0;
    if (row < nv) {
      val = X[(size_t)kp * np + row];
      for (int q = 0; q < M * DN; ++q) val -= A[(size_t)(nv + q) * np + row] * wr[q];
    }
    Xr[(size_t)kp * nr + row] = val;
  }
  for (int trow = tid; trow < kp; trow += QT) {
    double val = Rt[trow];
    for (int q = 0; q < M * DN; ++q) val -= C[(size_t)(nv + q) * kp + trow] * wr[q];
    Rtr[trow] = val;
  }
  // padding: identity of A^ beyond n_r, zero rows of B^ and columns of C^ beyond n_r, the zero
  // columns of [B^ r^ | 0], the padding columns of D
  for (size_t t = tid; t < (size_t)nr * nr; t += QT) {
    const int col = (int)(t / nr), row = (int)(t % nr);
    if (col >= nv || row >= nv) Ar[t] = (row == col) ? 1.0 : 0.0;
  }
  for (size_t t = tid; t < (size_t)(nr - nv) * kp; t += QT) Cr[(size_t)nv * kp + t] = 0.0;
  for (size_t t = tid; t < (size_t)k * (nr - nv); t += QT) {
    const int col = (int)(t / (nr - nv)), row = nv + (int)(t % (nr - nv));
    Xr[(size_t)col * nr + row] = 0.0;
  }
  for (size_t t = tid; t < (size_t)(kx - k) * nr; t += QT) {
    const int col = k + (int)(t / nr);
    if (col != kp) Xr[(size_t)col * nr + t % nr] = 0.0;
  }
  for (size_t t = tid; t < (size_t)(kp - k) * kp; t += QT) {
    const int col = k + (int)(t / kp);
    Dr[(size_t)col * kp + t % kp] = Dm[(size_t)col * kp + t % kp];
  }
}

// Y = [Y_v; Y_q], z = [z_v; z_q] from the condensation of the reduced block.
__global__ __launch_bounds__(QT) void k_qrecover(DevPlan P, QElimArgs Q, int e0, double *Y, double *z) {
  extern __shared__ double sm[];
  const int el = blockIdx.x, tid = threadIdx.x, e = e0 + el;
  const int Np = P.Np, D = P.dim, M = P.m, np = P.n_pad, kp = P.k_pad, kx = P.kx, k = P.k, n = P.n, Nfp = P.Nfp;
  const int nv = M * Np, DN = D * Np;
  const double *X = P.X + (size_t)el * kx * np;
  const double *MH = Q.MH + (size_t)el * (1 + D) * Np * Np;
  const double *Yv = Q.Yv + (size_t)el * nv * k;
  const double *zv = Q.zv + (size_t)el * nv;
  double *Ye = Y + (size_t)e * n * k;
  double *ze = z + (size_t)e * n;
  double *mi = sm, *hh = sm + Np * Np, *wb = hh + D * Np * Np;   // wb [QCB][DN] or [M D Np]
  double *ys = wb + QCB * DN;                                       // [QCB][nv] Y_v of the pass
  double *xs = sm + q_lds(Np, D, M, P.nf * Nfp).xs;                             // [QCB][DN] B_q rows of the pass
  for (int t = tid; t < (1 + D) * Np * Np; t += QT) sm[t] = MH[t];
  for (int c0 = 0; c0 < k; c0 += QCB) {
    const int nc = (k - c0) < QCB ? (k - c0) : QCB;
    __syncthreads();
    for (int t = tid; t < nc * nv; t += QT) ys[t] = Yv[(size_t)c0 * nv + t];
    for (int t = tid; t < nc * DN; t += QT) {
      const int cl = t / DN, ja = t % DN, col = c0 + cl;
      xs[t] = X[(size_t)col * np + nv + trace_comp(col, M, Nfp) * DN + ja];
    }
    __syncthreads();
    for (int t = tid; t < nc * DN; t += QT) {
      const int cl = t / DN, ja = t % DN, j = ja / Np, a = ja % Np;
      const double *xq = xs + cl * DN + j * Np;
      double acc = 0.0;
      for (int q = 0; q < Np; ++q) acc += mi[q * Np + a] * xq[q];
      wb[t] = acc;
    }
    __syncthreads();
    for (int t = tid; t < nc * n; t += QT) {
      const int cl = t / n, row = t % n, col = c0 + cl;
      double val;
      if (row < nv) {
        val = ys[cl * nv + row];
      } else {
        const int cja = row - nv, cc = cja / DN, ja = cja % DN, j = ja / Np, a = ja % Np;
        val = (cc == trace_comp(col, M, Nfp)) ? wb[cl * DN + ja] : 0.0;
        const double *yv = ys + cl * nv + cc * Np;
        const double *h = hh + j * Np * Np + a;   // H_j[a][b] at h[b * Np]
        for (int b = 0; b < Np; ++b) val -= h[b * Np] * yv[b];
      }
      Ye[(size_t)col * n + row] = val;
    }
  }
  __syncthreads();
  for (int t = tid; t < M * DN; t += QT) {
    const int a = t % Np, cj = t / Np;
    const double *xq = X + (size_t)kp * np + nv + cj * Np;
    double acc = 0.0;
    for (int q = 0; q < Np; ++q) acc += mi[q * Np + a] * xq[q];
    wb[t] = acc;
  }
  __syncthreads();
  for (int row = tid; row < n; row += QT) {
    double val;
    if (row < nv) {
      val = zv[row];
    } else {
      const int cja = row - nv, cc = cja / DN, ja = cja % DN, j = ja / Np, a = ja % Np;
      val = wb[cja];
      const double *h = hh + j * Np * Np + a;
      for (int b = 0; b < Np; ++b) val -= h[b * Np] * zv[cc * Np + b];
    }
    ze[row] = val;
  }
}

}  // namespace

size_t qelim_lds_bytes(const DevPlan &P) {
  return (size_t)q_lds(P.Np, P.dim, P.m, P.nf * P.Nfp).total * sizeof(double);
}

hipError_t launch_qelim(const DevPlan &P, const QElimArgs &Q, int ec, hipStream_t s) {
  const size_t lds = qelim_lds_bytes(P);
  hipError_t e = set_dyn_lds((const void *)k_qelim, lds);
  if (e) return e;
  hipLaunchKernelGGL(k_qelim, dim3(ec), dim3(QT), lds, s, P, Q);
  return hipGetLastError();
}

hipError_t launch_qrecover(const DevPlan &P, const QElimArgs &Q, int e0, int ec, double *Y, double *z,
                           hipStream_t s) {
  const size_t lds = qelim_lds_bytes(P);
  hipError_t e = set_dyn_lds((const void *)k_qrecover, lds);
  if (e) return e;
  hipLaunchKernelGGL(k_qrecover, dim3(ec), dim3(QT), lds, s, P, Q, e0, Y, z);
  return hipGetLastError();
}

}  // namespace hdg
