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
constexpr int QCB = 16;   // right-hand-side columns per recovery pass

// LDS carve-up (doubles): mass matrix inverse, H_j, and a region shared by the
// Gauss-Jordan work array and the W columns of a pass.
struct QLds {
  int mi, hh, w, xs, ti, total;
};

__host__ __device__ inline QLds q_lds(int Np, int D, int M, int ntc) {
  QLds L;
  L.mi = 0;
  L.hh = Np * Np;
  L.w = L.hh + D * Np * Np;
  const int gj = Np * 2 * Np;
  const int wc = QCB * D * Np + (M * D * Np > QCB * M * Np ? M * D * Np : QCB * M * Np);
  const int rcb = ((D * Np + 15) & ~15) * 7 * 16;   // R_c of the q elimination (up to 7 column tiles)
  int w = gj > wc ? gj : wc;
  if (rcb > w) w = rcb;
  L.xs = L.w + w;
  // staged q rows of X: the residual (M D Np), a component's trace columns and residual ((ntc + 1) x D Np)
  // or the columns of a recovery pass (QCB x D Np)
  int nq = M * D * Np;
  if ((ntc + 1) * D * Np > nq) nq = (ntc + 1) * D * Np;
  if (QCB * D * Np > nq) nq = QCB * D * Np;
  L.ti = L.xs + nq;
  L.total = L.ti + 56;   // int table of up to 112 trace columns
  return L;
}

// LDS of the recovery, in doubles: M^-1, H_j, W_B of a pass (or of the residual), the pass's
// Y_v columns and B_q rows; small enough for two workgroups per CU at N_p = 27.
struct QRecLds {
  int hh, wb, ys, xs, total;
};
__host__ __device__ inline QRecLds qrec_lds(int Np, int D, int M) {
  QRecLds L;
  L.hh = Np * Np;
  L.wb = L.hh + D * Np * Np;
  L.ys = L.wb + (QCB * D * Np > M * D * Np ? QCB * D * Np : M * D * Np);
  L.xs = L.ys + QCB * M * Np;
  L.total = L.xs + QCB * D * Np;
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
// of C (C_q), K = D N_p, N = N_p + nf N_fp + 1 (the last column is the
// residual).  The product is formed transposed so that outputs leave in
// column-major runs: lane l supplies R_c[k0 + l/16][ct*16 + l%16] (MFMA A
// operand, LDS) and the operand row tile*16 + l%16 at k = k0 + l/16 (MFMA B
// operand, streamed from the column-major blocks); accumulator r of lane l is
// the output (row tile*16 + l%16, column ct*16 + l/16 + 4r).
// NCT column tiles of R_c (N_p + nf N_fp + 1 <= 16 NCT <= 112); at most QKS k-steps (D N_p <= 4 QKS)
constexpr int QKS = 28;

template <int NCT>
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

  int *tcb = reinterpret_cast<int *>(sm + L.ti);   // trace column of R_c column Np + fi, less c Nfp
  for (int fi = tid; fi < nf * Nfp; fi += QT) tcb[fi] = (fi / Nfp) * MF + fi % Nfp;
  const int ntc = nf * Nfp;                // trace columns of one component
  const int ncr = Np + ntc;                // column of R_c holding the residual
  const int nrow = nv + kp;                // operand rows: A_vq then C_q
  const int nrt = (nrow + 15) / 16;
  const int K16 = (DN + 15) & ~15, KS = (DN + 3) / 4;
  for (int c = 0; c < M; ++c) {
    __syncthreads();
    // B_q rows of component c of its trace columns, xs[fi][ja] (contiguous in the column), then
    // the R_q rows of component c
    for (int t = tid; t < (ntc + 1) * DN; t += QT) {
      const int fi = t / DN, ja = t % DN;
      const int col = fi < ntc ? (fi / Nfp) * MF + c * Nfp + fi % Nfp : kp;
      xs[t] = X[(size_t)col * np + nv + c * DN + ja];
    }
    __syncthreads();
    // R_c[(j, a)][col]: H_j[a][b] for col = b < Np; W_B for trace column f Nfp + ib of component c;
    // W_R (component c) in column ncr
    for (int t = tid; t < K16 * NCT * 16; t += QT) {
      const int col = t % (NCT * 16), ja = t / (NCT * 16);
      double val = 0.0;
      if (ja < DN && col <= ncr) {
        const int j = ja / Np, a = ja % Np;
        if (col < Np) {
          val = hh[(j * Np + col) * Np + a];
        } else {
          const double *xq = xs + (col - Np) * DN + j * Np;
          for (int q = 0; q < Np; ++q) val += mi[q * Np + a] * xq[q];
        }
      }
      rc[t] = -val;   // -R_c[ja][col], row stride NCT * 16
    }
    __syncthreads();
    // the operands of a row tile (all k-steps) are loaded one row tile ahead of the MFMAs
    auto load_ops = [&](double (&ob)[QKS], int rt) {
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
#pragma unroll
      for (int ks = 0; ks < QKS; ++ks) {
        const int ja = 4 * ks + lk;
        ob[ks] = (ks < KS && src && ja < DN) ? src[(size_t)ja * ld] : 0.0;
      }
    };
    // outputs: original entry minus the product.  The accumulators start from the original
    // entries (the residual column accumulates over c; the same lane owns an output entry for
    // every c) and the MFMAs add the operand times -R_c, so the results are stored as they are.
    // (The column offset is made opaque per row tile so that the column address arithmetic is
    // not hoisted out of the row-tile loop into registers.)
    auto src_of = [&](int col, int orow) -> const double * {
      const bool vrow = orow < nv;
      const int trow = orow - nv;
      if (col < Np) {
        const size_t cv = c * Np + col;
        return vrow ? A + cv * np + orow : C + cv * kp + trow;
      }
      if (col < ncr) {
        const size_t tc = tcb[col - Np] + c * Nfp;
        return vrow ? X + tc * np + orow : Dm + tc * kp + trow;
      }
      if (vrow) return c == 0 ? X + (size_t)kp * np + orow : Xr + (size_t)kp * nr + orow;
      return c == 0 ? Rt + trow : Rtr + trow;
    };
    auto dst_of = [&](int col, int orow) -> double * {
      const bool vrow = orow < nv;
      const int trow = orow - nv;
      if (col < Np) {
        const size_t cv = c * Np + col;
        return vrow ? Ar + cv * nr + orow : Cr + cv * kp + trow;
      }
      if (col < ncr) {
        const size_t tc = tcb[col - Np] + c * Nfp;
        return vrow ? Xr + tc * nr + orow : Dr + tc * kp + trow;
      }
      return vrow ? Xr + (size_t)kp * nr + orow : Rtr + trow;
    };
    auto init = [&](d4 (&acc)[NCT], int rt) {
      const int orow = rt * 16 + li;
      int cb = lk;
      asm volatile("" : "+v"(cb));
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = ct * 16 + cb + 4 * r;
          acc[ct][r] = (orow < nrow && col <= ncr) ? *src_of(col, orow) : 0.0;
        }
    };
    auto mma = [&](d4 (&acc)[NCT], const double (&ob)[QKS]) {
#pragma unroll
      for (int ks = 0; ks < QKS; ++ks) {
        if (ks >= KS) break;
        const double *rr = rc + (4 * ks + lk) * (NCT * 16) + li;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct] = mfma4(rr[ct * 16], ob[ks], acc[ct]);
      }
    };
    auto store = [&](const d4 (&acc)[NCT], int rt) {
      const int orow = rt * 16 + li;
      if (orow >= nrow) return;
      int cb = lk;
      asm volatile("" : "+v"(cb));
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = ct * 16 + cb + 4 * r;
          if (col <= ncr) *dst_of(col, orow) = acc[ct][r];
        }
    };
    constexpr int NW = QT / 64;
    double o0[QKS], o1[QKS];
    d4 acc[NCT];
    if (wave < nrt) load_ops(o0, wave);
    for (int rt = wave; rt < nrt; rt += 2 * NW) {
      init(acc, rt);
      if (rt + NW < nrt) load_ops(o1, rt + NW);
      mma(acc, o0);
      store(acc, rt);
      if (rt + NW >= nrt) break;
      init(acc, rt + NW);
      if (rt + 2 * NW < nrt) load_ops(o0, rt + 2 * NW);
      mma(acc, o1);
      store(acc, rt + NW);
    }
  }
  for (int row = nv + tid; row < nr; row += QT) Xr[(size_t)kp * nr + row] = 0.0;
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
  const QRecLds L = qrec_lds(Np, D, M);
  double *mi = sm, *hh = sm + L.hh;
  double *wb = sm + L.wb;   // [QCB][DN] or [M D Np]
  double *ys = sm + L.ys;   // [QCB][nv] Y_v of the pass
  double *xs = sm + L.xs;   // [QCB][DN] B_q rows of the pass
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
    // W_B of the pass (M^-1 per direction block) and the v rows of Y
    for (int t = tid; t < nc * DN; t += QT) {
      const int cl = t / DN, ja = t % DN, j = ja / Np, a = ja % Np;
      const double *xq = xs + cl * DN + j * Np;
      double acc = 0.0;
      for (int q = 0; q < Np; ++q) acc += mi[q * Np + a] * xq[q];
      wb[t] = acc;
    }
    for (int t = tid; t < nc * nv; t += QT) Ye[(size_t)(c0 + t / nv) * n + t % nv] = ys[t];
    __syncthreads();
    // q rows of component cc: Y_q = [cc == comp(col)] W_B - H_j Y_v(cc), one FP64 MFMA tile per
    // (column tile, (j, a) tile, cc) with the columns as MFMA rows: lane l supplies
    // Y_v(cc, b = k0 + l/16)[col l%16] and H_j[a][b] for (j, a) = tile + l%16; accumulator r of
    // lane l is column l/16 + 4r, (j, a) = tile + l%16, so 16 lanes store 16 consecutive rows.
    const int nct = (nc + 15) / 16, njt = (DN + 15) / 16;
    for (int task = tid >> 6; task < nct * njt * M; task += QT / 64) {
      const int ct = task % nct, jt = (task / nct) % njt, cc = task / (nct * njt);
      const int li = tid & 15, lk = (tid >> 4) & 3;
      const int cl = ct * 16 + li, ja = jt * 16 + li, j = ja / Np, a = ja % Np;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < Np; k0 += 4) {
        const int b = k0 + lk;
        const double av = (b < Np && cl < nc) ? ys[cl * nv + cc * Np + b] : 0.0;
        const double bv = (b < Np && ja < DN) ? hh[(j * Np + b) * Np + a] : 0.0;
        acc = mfma4(av, bv, acc);
      }
      if (ja < DN) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int cr = ct * 16 + lk + 4 * r;
          if (cr >= nc) continue;
          const int col = c0 + cr;
          const double w = (cc == trace_comp(col, M, Nfp)) ? wb[cr * DN + ja] : 0.0;
          Ye[(size_t)col * n + nv + cc * DN + ja] = w - acc[r];
        }
      }
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
  const int a = q_lds(P.Np, P.dim, P.m, P.nf * P.Nfp).total, r = qrec_lds(P.Np, P.dim, P.m).total;
  return (size_t)(a > r ? a : r) * sizeof(double);
}

hipError_t launch_qelim(const DevPlan &P, const QElimArgs &Q, int ec, hipStream_t s) {
  const size_t lds = qelim_lds_bytes(P);
  const int nct = (P.Np + P.nf * P.Nfp + 16) / 16;
  auto go = [&](auto kern) -> hipError_t {
    hipError_t e = set_dyn_lds((const void *)kern, lds);
    if (e) return e;
    hipLaunchKernelGGL(kern, dim3(ec), dim3(QT), lds, s, P, Q);
    return hipGetLastError();
  };
  switch (nct) {
    case 1: return go(k_qelim<1>);
    case 2: return go(k_qelim<2>);
    case 3: return go(k_qelim<3>);
    case 4: return go(k_qelim<4>);
    case 5: return go(k_qelim<5>);
    case 6: return go(k_qelim<6>);
    case 7: return go(k_qelim<7>);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_qrecover(const DevPlan &P, const QElimArgs &Q, int e0, int ec, double *Y, double *z,
                           hipStream_t s) {
  const size_t lds = (size_t)qrec_lds(P.Np, P.dim, P.m).total * sizeof(double);
  hipError_t e = set_dyn_lds((const void *)k_qrecover, lds);
  if (e) return e;
  hipLaunchKernelGGL(k_qrecover, dim3(ec), dim3(QT), lds, s, P, Q, e0, Y, z);
  return hipGetLastError();
}

}  // namespace hdg
