// Element block assembly on matrix cores (volume) plus face-local products.
//
// Volume part of the element rows (weak forms of the element equation):
//   A[(c,a),(g,b)] = sum_qp T[(g,c,a), qp] phi_b(qp),  column group g = c' (v columns)
//   or g = m + s (q columns), with
//   T = W alpha A0_{c c'} phi_a + sum_r Kv_{c r c'} dphi_{r a}     (g < m)
//   T = sum_r Kq_{c r s} dphi_{r a}                                 (g >= m)
// is a GEMM with M = (groups x m x Np) rows, K = N_q, N = Np, run on FP64 MFMA
// with the basis tables and a 4-point slice of the pointwise coefficients
// staged in LDS.  Face f contributes small products
//   T_f[(.,.), ia, ib] = sum_fq coef(fq) psi_ia(fq) psi_ib(fq)
// that are formed once and scattered into A (added), B, C and D; the gradient
// rows (mass and divergence matrices) are formed once and copied per component.
#include "hdg_plan.hpp"

namespace hdg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));


__device__ inline d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Quadrature points per staged chunk of the basis tables: all of them when the
// (1 + D) tables of NB columns fit in 64 KB, else the largest multiple of 4 that does.
template <int D, int NCT>
__host__ __device__ inline int table_chunk(int Nq4) {
  const int per_point = (1 + D) * 16 * NCT * 8;
  int qc = (64 * 1024 / per_point) & ~3;
  return qc >= Nq4 ? Nq4 : qc;
}

// Dynamic LDS of the kernel in doubles: the larger of the volume phase (staged
// tables + a 4-point coefficient slice), the gradient phase (tables if resident +
// a group of Np x Np matrices) and the face phase.
template <int D, bool VISC, int NCT>
__host__ __device__ inline size_t contract_lds_doubles(int Np, int Nq, int Nfq, int Nfp, int fsize) {
  constexpr int M = D + 2;
  const int Nq4 = (Nq + 3) & ~3;
  const int QC = table_chunk<D, NCT>(Nq4);
  const size_t tables = (size_t)(1 + D) * QC * 16 * NCT;
  const size_t cs = (size_t)(M * M + M * D * M + (VISC ? M * D * M * D : 0));
  size_t total = tables + 4 * cs;
  const size_t facew = (size_t)Nfq * fsize + (size_t)Nfq * Nfp * Nfp + (size_t)Nfq * Nfp;
  if (facew > total) total = facew;
  if (VISC) {
    // all D + 1 gradient/mass matrices at once when they fit in 160 KB beside
    // resident tables and the per-point W J, W (register use keeps the kernel at
    // one workgroup per CU, so the LDS costs no occupancy), else as many as fit,
    // at least one
    const size_t held = (QC >= Nq4 ? tables : 0) + (size_t)Nq * (D * D + 1);
    const size_t nn = (size_t)Np * Np;
    size_t jg = (20480 > held + nn) ? (20480 - held) / nn : 1;
    if (jg > (size_t)(D + 1)) jg = D + 1;
    if (held + jg * nn > total) total = held + jg * nn;
  }
  return total;
}

// Gradient and mass matrices formed per pass (as many as fit in the LDS beside
// resident tables).
template <int D, bool VISC, int NCT>
__host__ __device__ inline int grad_group(int Np, int Nq, int Nfq, int Nfp, int fsize) {
  const int Nq4 = (Nq + 3) & ~3;
  const int QC = table_chunk<D, NCT>(Nq4);
  const size_t held = (QC >= Nq4 ? (size_t)(1 + D) * QC * 16 * NCT : 0) + (size_t)Nq * (D * D + 1);
  const size_t avail = contract_lds_doubles<D, VISC, NCT>(Np, Nq, Nfq, Nfp, fsize) - held;
  const size_t jg = avail / ((size_t)Np * Np);
  return jg > (size_t)(D + 1) ? D + 1 : (int)jg;
}

// NTH threads per workgroup (256, 512 or 1024; chosen per plan, default 1024).
template <int D, bool VISC, int NCT, int NTH>
__global__ __launch_bounds__(NTH) void k_contract_mfma(DevPlan P, int e0, int ec) {
  constexpr int NT = NTH;
  constexpr int M = D + 2;
  constexpr int G = VISC ? M + M * D : M;   // column groups
  constexpr int RT = (NCT == 1) ? (NTH >= 1024 ? 8 : 16) : (NCT == 2 ? (NTH >= 1024 ? 4 : 8) : (NTH >= 1024 ? 2 : 4));
  extern __shared__ double lds[];
  const int el = blockIdx.x, e = e0 + el;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int Np = P.Np, Nq = P.Nq, nf = P.nf, Nfp = P.Nfp, Nfq = P.Nfq;
  const int Nq4 = (Nq + 3) & ~3;
  const int np = P.n_pad, kp = P.k_pad, kx = P.kx;
  const PointLayout L = P.L;
  double *A = P.A + (size_t)el * np * np;
  double *X = P.X + (size_t)el * kx * np;
  double *Cm = P.C + (size_t)el * np * kp;
  double *Dm = P.D + (size_t)el * kp * kp;
  double *Rt = P.Rt + (size_t)el * kp;
  const double *pv = P.pv + (size_t)el * Nq * L.size;
  const double *pf = P.pf + (size_t)el * nf * Nfq * L.fsize;
  const int *fnodes = P.fnodes;
  const int *fbc = P.face_bc + (size_t)e * nf;

  // LDS: basis tables of QC quadrature points at a time (zero-padded, 16*NCT basis
  // functions).  When all Nq4 points fit (QC == Nq4) the tables stay resident for
  // the later phases; otherwise those phases read the global tables.
  const int NB = 16 * NCT;
  const int QC = table_chunk<D, NCT>(Nq4);
  const bool resident = QC >= Nq4;
  double *sphi = lds;                          // [QC][NB]
  double *sdphi = sphi + QC * NB;              // [D][QC][NB]
  double *work = sdphi + D * QC * NB;          // shared scratch
  auto stage = [&](int qc) {
    for (int t = tid; t < (1 + D) * QC * NB; t += NT) {
      const int b = t % NB, qq = (t / NB) % QC, r = t / (NB * QC), qp = qc + qq;
      double val = 0.0;
      if (b < Np && qp < Nq) val = (r == 0) ? P.phi[qp * Np + b] : P.dphi[((size_t)(r - 1) * Nq + qp) * Np + b];
      sphi[t] = val;
    }
  };
  auto PHI = [&](int qp, int a) { return resident ? sphi[qp * NB + a] : P.phi[qp * Np + a]; };
  auto DPHI = [&](int r, int qp, int a) {
    return resident ? sdphi[(r * QC + qp) * NB + a] : P.dphi[((size_t)r * Nq + qp) * Np + a];
  };
  if (resident) stage(0);
  // zero fill: q rows and padding of A, X, C, D, R_tr
  const int nv = M * Np;
  // (a wave per column, lanes along the rows: no index division).  With a_qmin the q rows
  // and the padding of A are left unwritten: the condensation forms them from the compact
  // M and G_j, the q elimination reads M and G_j of the first component.
  for (int col = P.a_qmin ? np : wave; col < np; col += NT / 64) {
    double *Ac = A + (size_t)col * np;
    for (int row = (col < P.n ? nv : 0) + lane; row < np; row += 64) Ac[row] = (row == col && row >= P.n) ? 1.0 : 0.0;
  }
  if (P.zero_xcd) {
    for (size_t i = tid; i < (size_t)kx * np; i += NT) X[i] = 0.0;
    for (size_t i = tid; i < (size_t)np * kp; i += NT) Cm[i] = 0.0;
    for (size_t i = tid; i < (size_t)kp * kp; i += NT) Dm[i] = 0.0;
  }
  for (int i = tid; i < kp; i += NT) Rt[i] = 0.0;
  __syncthreads();

  // ---- volume GEMM on MFMA
  const int nrows = G * M * Np;
  const int ntiles = (nrows + 15) / 16;
  constexpr int CS = M * M + M * D * M + (VISC ? M * D * M * D : 0);  // coefficients per point
  constexpr int CR = (4 * CS + NT - 1) / NT;                          // slice values per thread
  double *coef = work;                                                // [4][CS]
  // the coefficient slice of points q0..q0+3, fetched into registers one slice
  // ahead of its use so that the loads overlap the previous slice's MFMAs
  auto fetch = [&](int q0, double (&cv)[CR]) {
    const int ft = cur_tid();
#pragma unroll
    for (int u = 0; u < CR; ++u) {
      const int t = ft + u * NT;
      double val = 0.0;
      if (t < 4 * CS) {
        const int j = t % CS, qq = t / CS;
        if (q0 + qq < Nq) val = pv[(size_t)(q0 + qq) * L.size + L.Mv + j];   // Mv, Kv, Kq are contiguous
      }
      cv[u] = val;
    }
  };
  for (int base = 0; base < ntiles; base += (NT / 64) * RT) {
    // thread indices re-read per pass (cur_tid): derived offsets stay inside the loop body
    const int tid = cur_tid(), lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    d4 acc[RT][NCT];
#pragma unroll
    for (int u = 0; u < RT; ++u)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[u][ct] = d4{0.0, 0.0, 0.0, 0.0};
    // per row tile: basis function a and the coefficient offsets of row rho = (g, c, a):
    // T = [g < M] cq[o1] phi_a + sum_r cq[o2 + r * st] dphi_{r,a}, packed in one word
    // per tile (a: bits 0-6, o2: bits 7-18, g < M: bit 19; o1 = o2 - M * M - c * D * M
    // + c * M is kept as the difference o2 - o1 = M * M + c * (D - 1) * M in bits 20-30)
    int pk[RT];
#pragma unroll
    for (int u = 0; u < RT; ++u) {
      const int tile = base + wave * RT + u;
      const int rho = tile * 16 + li;
      pk[u] = -1;
      if (tile < ntiles && rho < nrows) {
        const int a = rho % Np, c = (rho / Np) % M, g = rho / (Np * M);
        if (g < M) pk[u] = a | ((M * M + c * D * M + g) << 7) | (1 << 19) | ((M * M + c * (D - 1) * M) << 20);
        else pk[u] = a | ((M * M + M * D * M + c * D * (M * D) + (g - M)) << 7);
      }
    }
    double cv[CR];
    fetch(0, cv);
    for (int q0 = 0; q0 < Nq4; q0 += 4) {
      if (!resident && q0 % QC == 0) {
        __syncthreads();
        stage(q0);
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < CR; ++u)
        if (tid + u * NT < 4 * CS) coef[tid + u * NT] = cv[u];
      if (q0 + 4 < Nq4) fetch(q0 + 4, cv);
      __syncthreads();
      const int lk = (cur_tid() & 63) >> 4, li = cur_tid() & 15;
      const int qp = q0 + lk;
      const int ql = resident ? qp : qp % QC;   // row of the staged tables
      const double *cq = coef + lk * CS;
#pragma unroll
      for (int u = 0; u < RT; ++u) {
        double tval = 0.0;
        if (pk[u] >= 0) {
          const int a = pk[u] & 127, o2 = (pk[u] >> 7) & 4095;
          const bool vcol = (pk[u] >> 19) & 1;
          const int st = vcol ? M : M * D;
          if (vcol) tval = cq[o2 - (pk[u] >> 20)] * sphi[ql * NB + a];
#pragma unroll
          for (int r = 0; r < D; ++r) tval += cq[o2 + r * st] * sdphi[(r * QC + ql) * NB + a];
        }
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[u][ct] = mfma4(sphi[ql * NB + ct * 16 + li], tval, acc[u][ct]);
      }
    }
    // write the tiles.  The products are formed transposed (phi as the first operand), so
    // that lane l holds row rho = tile * 16 + l % 16 and columns b = ct * 16 + l / 16 + 4 r:
    // neighbouring lanes write neighbouring rows of A
#pragma unroll
    for (int u = 0; u < RT; ++u) {
      const int tile = base + wave * RT + u;
      const int rho = tile * 16 + li;
      if (tile >= ntiles || rho >= nrows) continue;
      const int a = rho % Np, c = (rho / Np) % M, g = rho / (Np * M);
      double *Ac = A + (size_t)(g * Np) * np + c * Np + a;
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int b = ct * 16 + lk + 4 * r;
          if (b < Np) Ac[(size_t)b * np] = acc[u][ct][r];
        }
    }
  }
  __syncthreads();

  // ---- gradient rows: G_j[a][b] = sum W dphi_j,a phi_b (physical), M[a][b] = sum W phi_a phi_b,
  // one matrix at a time (j = 0..D-1 gradients, j = D mass)
  if (VISC) {
    constexpr int DW = D * D + 1;   // W J (D x D) and W per point
    const int JG = grad_group<D, VISC, NCT>(Np, Nq, Nfq, Nfp, L.fsize);
    double *swj = resident ? work : lds;   // [Nq][DW]
    double *gm = swj + Nq * DW;            // [JG][Np][Np]
    for (int t = tid; t < Nq * DW; t += NT) {
      const int qp = t / DW, i = t % DW;
      swj[t] = pv[(size_t)qp * L.size + (i < D * D ? L.WJ + i : L.W)];
    }
    __syncthreads();
    for (int j0 = 0; j0 <= D; j0 += JG) {
      const int nj = (D + 1 - j0) < JG ? (D + 1 - j0) : JG;
      // G_j = U_j Phi on the matrix cores, U_j[a][qp] = sum_r W J_rj dphi_r,a(qp) (j < D) or
      // W phi_a(qp) (the mass matrix, j = D), Phi[qp][b] = phi_b(qp): one 16 x 16 output tile
      // (a, b) per wave, K = N_q in steps of 4 points; lane (li, lk) forms the A operand
      // U_j[16 ta + li][q0 + lk] and reads the B operand phi_{16 tb + li}(q0 + lk), and holds
      // rows 16 ta + lk + 4 r of the result (padding rows, columns and points are zero)
      for (int tt = wave; tt < nj * NCT * NCT; tt += NT / 64) {
        const int jl = tt / (NCT * NCT), ta = (tt / NCT) % NCT, tb = tt % NCT;
        const int j = j0 + jl, a = 16 * ta + li, b = 16 * tb + li;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < Nq; q0 += 4) {
          const int qp = q0 + lk;
          double u = 0.0, v = 0.0;
          if (qp < Nq) {
            if (a < Np) {
              if (j < D) {
#pragma unroll
                for (int r = 0; r < D; ++r) u += swj[qp * DW + r * D + j] * DPHI(r, qp, a);
              } else {
                u = swj[qp * DW + D * D] * PHI(qp, a);
              }
            }
            if (b < Np) v = PHI(qp, b);
          }
          acc = mfma4(u, v, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ar = 16 * ta + lk + 4 * r;
          if (ar < Np && b < Np) gm[(jl * Np + ar) * Np + b] = acc[r];
        }
      }
      __syncthreads();
      // the compact copy the condensation forms the q rows of A from
      if (P.mg) {
        double *mg = P.mg + (size_t)el * (D + 1) * Np * Np + (size_t)j0 * Np * Np;
        for (int t = tid; t < nj * Np * Np; t += NT) mg[t] = gm[t];
      }
      // G_j into the (q_j, v) block, the mass matrix into every (q_j, q_j) block (with a_qmin
      // into those of the first component and its first direction only)
      const int mc = P.a_qmin ? 1 : M, mj = P.a_qmin ? 1 : D;
      for (int t = tid; t < mc * nj * Np * Np; t += NT) {
        const int a = t % Np, b = (t / Np) % Np, jl = (t / (Np * Np)) % nj, c = t / (nj * Np * Np);
        const int j = j0 + jl;
        const double val = gm[(jl * Np + a) * Np + b];
        if (j < D) {
          A[(size_t)(c * Np + b) * np + nv + (c * D + j) * Np + a] = val;
        } else {
          for (int jj = 0; jj < mj; ++jj) {
            const int cj = c * D + jj;
            A[(size_t)(nv + cj * Np + b) * np + nv + cj * Np + a] = val;
          }
        }
      }
      __syncthreads();
    }
  }

  // ---- element residual rows (column k_pad of X): volume parts
  double *R = X + (size_t)kp * np;
  for (int t = tid; t < M * Np; t += NT) {
    const int a = t % Np, c = t / Np;
    double acc = 0.0;
#pragma unroll 4
    for (int qp = 0; qp < Nq; ++qp) {
      const double *w = pv + (size_t)qp * L.size;
      double ta = w[L.Wu + c] * PHI(qp, a);
#pragma unroll
      for (int r = 0; r < D; ++r) ta += w[L.Fr + c * D + r] * DPHI(r, qp, a);
      acc += ta;
    }
    R[c * Np + a] = acc;
  }
  if (VISC) {
    for (int t = tid; t < M * D * Np; t += NT) {
      const int a = t % Np, cj = t / Np, c = cj / D, j = cj % D;
      double acc = 0.0;
#pragma unroll 4
      for (int qp = 0; qp < Nq; ++qp) {
        const double *w = pv + (size_t)qp * L.size;
        double ta = 0.0;
#pragma unroll
        for (int r = 0; r < D; ++r) ta += w[L.WJ + r * D + j] * DPHI(r, qp, a);
        acc += w[L.Wq + c * D + j] * PHI(qp, a) + w[L.v + c] * ta;
      }
      R[nv + cj * Np + a] = acc;
    }
  }
  __syncthreads();

  // ---- faces, one at a time (A entries of edge nodes receive several faces)
  const int MF = M * Nfp;
  const int NP2 = Nfp * Nfp;
  double *spf = lds;                            // [Nfq][fsize] (tables no longer needed)
  double *spp = spf + Nfq * L.fsize;            // [Nfq][Nfp][Nfp]
  double *sps = spp + Nfq * NP2;                // [Nfq][Nfp]
  for (int f = 0; f < nf; ++f) {
    const int tid = cur_tid(), lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const double *pff = pf + (size_t)f * Nfq * L.fsize;
    for (int t = tid; t < Nfq * L.fsize; t += NT) spf[t] = pff[t];
    const double *fp = P.fphi + (size_t)f * Nfq * Nfp;
    for (int t = tid; t < Nfq * NP2; t += NT) {
      const int ib = t % Nfp, ia = (t / Nfp) % Nfp, fq = t / NP2;
      spp[t] = fp[fq * Nfp + ia] * fp[fq * Nfp + ib];
    }
    for (int t = tid; t < Nfq * Nfp; t += NT) sps[t] = fp[t];
    __syncthreads();
    const bool dir = fbc[f] != 0;
    const int *fn = fnodes + f * Nfp;
    // face products on MFMA: T[rho][(ia, ib)] = sum_fq coef_rho(fq) psi_ia(fq) psi_ib(fq), with
    // rows rho: Tv (c, c') | Th (c, c') | mass | Tq (c, s) | B_q (j) (the last two viscous only)
    {
      constexpr int MM = M * M, RV = 2 * MM + 1;
      constexpr int NR = RV + (VISC ? MM * D + D : 0);
      constexpr int RTL = (NR + 15) / 16;
      const int nct = (NP2 + 15) / 16;
      const int Nfq4 = (Nfq + 3) & ~3;
      for (int tt = wave; tt < RTL * nct; tt += NT / 64) {
        const int lane = cur_tid() & 63, li = lane & 15, lk = lane >> 4;
        const int rt = tt / nct, ct = tt % nct;
        const int ra = rt * 16 + li;   // A-operand row of this lane
        int off = -1;
        if (ra < MM) off = L.fFv + ra;
        else if (ra < 2 * MM) off = L.fFh + (ra - MM);
        else if (ra == 2 * MM) off = L.fW;
        else if (VISC && ra < RV + MM * D) off = L.fFq + (ra - RV);
        else if (VISC && ra < NR) off = L.fWn + (ra - RV - MM * D);
        const int nb = ct * 16 + li;   // B-operand column of this lane
        // output column of this lane, n = ib * Nfp + ia (the product table is symmetric in
        // ia, ib; with ia fastest the lanes write neighbouring rows of A, B and D), and
        // the A entries it will add to, read before the products so that the loads overlap them
        const int n = nb;
        const int ib = n < NP2 ? n / Nfp : 0, ia = n < NP2 ? n % Nfp : 0;
        const int a = fn[ia], b = fn[ib];
        double *ap[4];
        double aold[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rho = rt * 16 + lk + 4 * r;
          ap[r] = nullptr;
          if (n < NP2) {
            if (rho < MM) ap[r] = A + (size_t)((rho % M) * Np + b) * np + (rho / M) * Np + a;
            else if (VISC && rho >= RV && rho < RV + MM * D)
              ap[r] = A + (size_t)(nv + ((rho - RV) % (M * D)) * Np + b) * np + ((rho - RV) / (M * D)) * Np + a;
          }
          aold[r] = ap[r] ? *ap[r] : 0.0;
        }
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < Nfq4; k0 += 4) {
          const int fq = k0 + lk;
          const double av = (off >= 0 && fq < Nfq) ? spf[fq * L.fsize + off] : 0.0;
          const double bv = (nb < NP2 && fq < Nfq) ? spp[fq * NP2 + nb] : 0.0;
          acc = mfma4(av, bv, acc);
        }
        if (n >= NP2) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rho = rt * 16 + lk + 4 * r;
          const double v = acc[r];
          if (ap[r]) *ap[r] = aold[r] + v;   // A_vv += Tv, A_vq += Tq
          // (C entries use T[.][ia][ib] = T[.][ib][ia]: column from node ib, row from ia, so
          // that neighbouring lanes write neighbouring rows of C as well)
          if (rho < MM) {                 // C_v = Tv (flux faces)
            const int c = rho / M, cp = rho % M;
            if (!dir) Cm[(size_t)(cp * Np + b) * kp + f * MF + c * Nfp + ia] = v;
          } else if (rho < 2 * MM) {      // B_v = Th, D = Th (flux faces)
            const int c = (rho - MM) / M, cp = (rho - MM) % M;
            X[(size_t)(f * MF + cp * Nfp + ib) * np + c * Np + a] = v;
            if (!dir) Dm[(size_t)(f * MF + cp * Nfp + ib) * kp + f * MF + c * Nfp + ia] = v;
          } else if (rho == 2 * MM) {     // D = mass on Dirichlet faces
            if (dir)
              for (int c = 0; c < M; ++c) Dm[(size_t)(f * MF + c * Nfp + ib) * kp + f * MF + c * Nfp + ia] = v;
          } else if (VISC && rho < RV + MM * D) {   // C_q = Tq (flux faces)
            const int q = rho - RV, c = q / (M * D), sq = q % (M * D);
            if (!dir) Cm[(size_t)(nv + sq * Np + b) * kp + f * MF + c * Nfp + ia] = v;
          } else if (VISC && rho < NR) {  // B_q[(c, j, a), (f, c, b)] = -sum W n_j psi_a psi_b
            const int j = rho - RV - MM * D;
            for (int c = 0; c < M; ++c) X[(size_t)(f * MF + c * Nfp + ib) * np + nv + (c * D + j) * Np + a] = -v;
          }
        }
      }
    }
    // residual face terms
    for (int t = tid; t < M * Nfp; t += NT) {
      const int ia = t % Nfp, c = t / Nfp;
      double rv = 0.0, rt = 0.0;
      for (int fq = 0; fq < Nfq; ++fq) {
        const double *w = spf + fq * L.fsize;
        const double ps = sps[fq * Nfp + ia];
        rv += w[L.fFf + c] * ps;
        rt += (dir ? w[L.fFd + c] : w[L.fFf + c]) * ps;
      }
      R[c * Np + fn[ia]] += rv;
      Rt[f * MF + c * Nfp + ia] = rt;
    }
    if (VISC) {
      for (int t = tid; t < M * D * Nfp; t += NT) {
        const int ia = t % Nfp, cj = t / Nfp, c = cj / D, j = cj % D;
        double rq = 0.0;
        for (int fq = 0; fq < Nfq; ++fq) {
          const double *w = spf + fq * L.fsize;
          rq += w[L.fWn + j] * w[L.fvh + c] * sps[fq * Nfp + ia];
        }
        R[nv + cj * Np + fn[ia]] -= rq;
      }
    }
    __syncthreads();
  }
}

template <int D, bool VISC, int NCT>
size_t lds_bytes_t(const DevPlan &P) {
  return contract_lds_doubles<D, VISC, NCT>(P.Np, P.Nq, P.Nfq, P.Nfp, P.L.fsize) * sizeof(double);
}

template <int D, bool VISC, int NCT, int NTH>
hipError_t launch_nt(const DevPlan &P, int e0, int ec, hipStream_t s) {
  const size_t lds = lds_bytes_t<D, VISC, NCT>(P);
  hipError_t e = set_dyn_lds((const void *)k_contract_mfma<D, VISC, NCT, NTH>, lds);
  if (e) return e;
  hipLaunchKernelGGL((k_contract_mfma<D, VISC, NCT, NTH>), dim3(ec), dim3(NTH), lds, s, P, e0, ec);
  return hipGetLastError();
}

template <int D, bool VISC, int NCT>
hipError_t launch_t(const DevPlan &P, int e0, int ec, hipStream_t s) {
  if (P.contract_threads == 256) return launch_nt<D, VISC, NCT, 256>(P, e0, ec, s);
  if (P.contract_threads == 512) return launch_nt<D, VISC, NCT, 512>(P, e0, ec, s);
  return launch_nt<D, VISC, NCT, 1024>(P, e0, ec, s);
}

template <int D, bool VISC>
size_t lds_for(const DevPlan &P) {
  if (P.Np <= 16) return lds_bytes_t<D, VISC, 1>(P);
  if (P.Np <= 32) return lds_bytes_t<D, VISC, 2>(P);
  if (P.Np <= 48) return lds_bytes_t<D, VISC, 3>(P);
  return lds_bytes_t<D, VISC, 4>(P);
}

template <int D, bool VISC>
hipError_t launch_dv(const DevPlan &P, int e0, int ec, hipStream_t s) {
  if (P.Np <= 16) return launch_t<D, VISC, 1>(P, e0, ec, s);
  if (P.Np <= 32) return launch_t<D, VISC, 2>(P, e0, ec, s);
  if (P.Np <= 48) return launch_t<D, VISC, 3>(P, e0, ec, s);
  return launch_t<D, VISC, 4>(P, e0, ec, s);
}

}  // namespace

bool contract_mfma_supported(const DevPlan &P) {
  if (P.Np > 64) return false;
  size_t lds = 0;
  if (P.dim == 2) lds = P.viscous ? lds_for<2, true>(P) : lds_for<2, false>(P);
  else lds = P.viscous ? lds_for<3, true>(P) : lds_for<3, false>(P);
  return lds <= 160 * 1024;
}

hipError_t launch_contract_mfma(const DevPlan &P, int e0, int ec, hipStream_t s) {
  if (P.dim == 2) return P.viscous ? launch_dv<2, true>(P, e0, ec, s) : launch_dv<2, false>(P, e0, ec, s);
  return P.viscous ? launch_dv<3, true>(P, e0, ec, s) : launch_dv<3, false>(P, e0, ec, s);
}

}  // namespace hdg
