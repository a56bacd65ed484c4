// Static condensation of every element (the local elimination that leaves only
// v_hat globally coupled):  A = P L U,  [Y z] = A^-1 [B R_loc],
// S = D - C Y,  g = -R_tr + C z.
//
// One workgroup (4 wave64s) per element.  A is column-major with leading
// dimension n_pad (a multiple of 16; the padding is the identity).  The LU is a
// right-looking blocked factorization with 16-column panels factored in LDS
// with partial pivoting; trailing updates, the blocked triangular solves and
// the Schur product run on FP64 MFMA 16x16x4 tiles.
#include "hdg_plan.hpp"

namespace hdg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BLK = 256;
constexpr int PS = 17;   // LDS row stride of a 16-column panel

// MFMA f64 16x16x4 operand layout (checked on gfx950 by hdg_selftest): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element r of
// lane l is C[l / 16 + 4 r][l % 16].
__device__ inline d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Rows of a 16-column panel held in LDS (the rest of a taller panel stays in A itself).
constexpr int LU_LDS_CAP = 160 * 1024 - 4 * 1024;
constexpr int LU_RL = (LU_LDS_CAP / (PS * (int)sizeof(double))) / 16 * 16;   // 1168

// BIG: panels taller than LU_RL rows keep their rows from LU_RL on in A (global memory, in
// place): every panel access then goes through a generic pointer, which the LDS-only
// instantiation avoids.
template <bool BIG>
__global__ __launch_bounds__(BLK) void k_lu(DevPlan P, int32_t *status) {
  extern __shared__ double sm[];
  __shared__ double redv[BLK];
  __shared__ int redi[BLK];
  const int el = blockIdx.x;
  const int np = P.n_pad;
  double *A = P.A + (size_t)el * np * np;
  int *ipiv = P.ipiv + (size_t)el * np;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  bool singular = false;
  for (int j0 = 0; j0 < np; j0 += 16) {
    const int rows = np - j0;
    const int rl = BIG ? (rows < LU_RL ? rows : LU_RL) : rows;   // rows of the panel in LDS
    // entry (i, jj) of the panel: LDS below rl, A itself from rl on
    const auto pe = [&](int i, int jj) -> double & {
      if (BIG && i >= rl) return A[(size_t)(j0 + jj) * np + j0 + i];
      return sm[i * PS + jj];
    };
    for (int t = tid; t < rl * 16; t += BLK) {
      const int i = t % rl, jj = t / rl;
      sm[i * PS + jj] = A[(size_t)(j0 + jj) * np + j0 + i];
    }
    __syncthreads();
    for (int jj = 0; jj < 16; ++jj) {
      double best = -1.0;
      int bi = jj;
      for (int i = jj + tid; i < rows; i += BLK) {
        const double a = fabs(pe(i, jj));
        if (a > best) {
          best = a;
          bi = i;
        }
      }
      redv[tid] = best;
      redi[tid] = bi;
      __syncthreads();
      for (int s = BLK / 2; s > 0; s >>= 1) {
        if (tid < s) {
          const double o = redv[tid + s];
          const int oi = redi[tid + s];
          if (o > redv[tid] || (o == redv[tid] && oi < redi[tid])) {
            redv[tid] = o;
            redi[tid] = oi;
          }
        }
        __syncthreads();
      }
      const int piv = redi[0];
      const bool zero = !(redv[0] > 0.0);
      if (zero) singular = true;
      if (!zero && piv != jj && tid < 16) {
        const double t0 = sm[jj * PS + tid];
        sm[jj * PS + tid] = pe(piv, tid);
        pe(piv, tid) = t0;
      }
      if (tid == 0) ipiv[j0 + jj] = zero ? j0 + jj : j0 + piv;
      __syncthreads();
      if (!zero) {
        const double inv = 1.0 / sm[jj * PS + jj];
        for (int i = jj + 1 + tid; i < rows; i += BLK) {
          const double l = pe(i, jj) * inv;
          pe(i, jj) = l;
          for (int c = jj + 1; c < 16; ++c) pe(i, c) -= l * sm[jj * PS + c];
        }
      }
      __syncthreads();
    }
    for (int t = tid; t < rl * 16; t += BLK) {
      const int i = t % rl, jj = t / rl;
      A[(size_t)(j0 + jj) * np + j0 + i] = sm[i * PS + jj];
    }
    // row interchanges on the columns outside the panel
    for (int c = tid; c < np - 16; c += BLK) {
      const int col = c < j0 ? c : c + 16;
      double *Ac = A + (size_t)col * np;
      for (int jj = 0; jj < 16; ++jj) {
        const int r1 = j0 + jj, r2 = ipiv[j0 + jj];
        if (r2 != r1) {
          const double t0 = Ac[r1];
          Ac[r1] = Ac[r2];
          Ac[r2] = t0;
        }
      }
    }
    __syncthreads();
    // U12 = L11^-1 A12
    for (int col = j0 + 16 + tid; col < np; col += BLK) {
      double *Ac = A + (size_t)col * np + j0;
      double x[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) x[jj] = Ac[jj];
#pragma unroll
      for (int jj = 1; jj < 16; ++jj)
#pragma unroll
        for (int ii = 0; ii < jj; ++ii) x[jj] -= sm[jj * PS + ii] * x[ii];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) Ac[jj] = x[jj];
    }
    __syncthreads();
    // A22 -= L21 U12
    const int r0 = j0 + 16;
    const int nt = (np - r0) / 16;
    const int li = lane & 15, lk = lane >> 4;
    for (int t = wave; t < nt * nt; t += 4) {
      const int ti = t % nt, tj = t / nt;
      const int row0 = r0 + ti * 16, col0 = r0 + tj * 16;
      double *Ct = A + (size_t)(col0 + li) * np + row0 + lk;
      d4 acc;
      acc[0] = Ct[0];
      acc[1] = Ct[4];
      acc[2] = Ct[8];
      acc[3] = Ct[12];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int pr = 16 + ti * 16 + li;   // panel row of the L21 entry
        const double a = -(BIG && pr >= rl ? A[(size_t)(j0 + 4 * kk + lk) * np + j0 + pr] : sm[pr * PS + 4 * kk + lk]);
        const double b = A[(size_t)(col0 + li) * np + j0 + 4 * kk + lk];
        acc = mfma4(a, b, acc);
      }
      Ct[0] = acc[0];
      Ct[4] = acc[1];
      Ct[8] = acc[2];
      Ct[12] = acc[3];
    }
    __syncthreads();
  }
  if (singular && tid == 0 && status[el] == HDG_OK) status[el] = HDG_ESINGULAR;
}

// [Y z] = U^-1 L^-1 P [B R] in place in X (n_pad x kx, column-major).
__global__ __launch_bounds__(BLK) void k_solve(DevPlan P) {
  __shared__ double T[16 * PS];
  const int el = blockIdx.x;
  const int np = P.n_pad, kx = P.kx;
  const double *A = P.A + (size_t)el * np * np;
  const int *ipiv = P.ipiv + (size_t)el * np;
  double *X = P.X + (size_t)el * kx * np;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int col = tid; col < kx; col += BLK) {
    double *Xc = X + (size_t)col * np;
    for (int i = 0; i < np; ++i) {
      const int r = ipiv[i];
      if (r != i) {
        const double t0 = Xc[i];
        Xc[i] = Xc[r];
        Xc[r] = t0;
      }
    }
  }
  __syncthreads();
  const int ntc = kx / 16;
  // forward substitution with unit lower L
  for (int j0 = 0; j0 < np; j0 += 16) {
    for (int t = tid; t < 256; t += BLK) T[(t % 16) * PS + t / 16] = A[(size_t)(j0 + t / 16) * np + j0 + t % 16];
    __syncthreads();
    for (int col = tid; col < kx; col += BLK) {
      double *Xc = X + (size_t)col * np + j0;
      double x[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) x[jj] = Xc[jj];
#pragma unroll
      for (int jj = 1; jj < 16; ++jj)
#pragma unroll
        for (int ii = 0; ii < jj; ++ii) x[jj] -= T[jj * PS + ii] * x[ii];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) Xc[jj] = x[jj];
    }
    __syncthreads();
    const int r0 = j0 + 16, ntr = (np - r0) / 16;
    for (int t = wave; t < ntr * ntc; t += 4) {
      const int ti = t % ntr, tj = t / ntr;
      const int row0 = r0 + ti * 16, col0 = tj * 16;
      double *Ct = X + (size_t)(col0 + li) * np + row0 + lk;
      d4 acc;
      acc[0] = Ct[0];
      acc[1] = Ct[4];
      acc[2] = Ct[8];
      acc[3] = Ct[12];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double a = -A[(size_t)(j0 + 4 * kk + lk) * np + row0 + li];
        const double b = X[(size_t)(col0 + li) * np + j0 + 4 * kk + lk];
        acc = mfma4(a, b, acc);
      }
      Ct[0] = acc[0];
      Ct[4] = acc[1];
      Ct[8] = acc[2];
      Ct[12] = acc[3];
    }
    __syncthreads();
  }
  // backward substitution with U
  for (int j0 = np - 16; j0 >= 0; j0 -= 16) {
    for (int t = tid; t < 256; t += BLK) T[(t % 16) * PS + t / 16] = A[(size_t)(j0 + t / 16) * np + j0 + t % 16];
    __syncthreads();
    for (int col = tid; col < kx; col += BLK) {
      double *Xc = X + (size_t)col * np + j0;
      double x[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) x[jj] = Xc[jj];
#pragma unroll
      for (int jj = 15; jj >= 0; --jj) {
#pragma unroll
        for (int ii = jj + 1; ii < 16; ++ii) x[jj] -= T[jj * PS + ii] * x[ii];
        x[jj] /= T[jj * PS + jj];
      }
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) Xc[jj] = x[jj];
    }
    __syncthreads();
    const int ntr = j0 / 16;
    for (int t = wave; t < ntr * ntc; t += 4) {
      const int ti = t % ntr, tj = t / ntr;
      const int row0 = ti * 16, col0 = tj * 16;
      double *Ct = X + (size_t)(col0 + li) * np + row0 + lk;
      d4 acc;
      acc[0] = Ct[0];
      acc[1] = Ct[4];
      acc[2] = Ct[8];
      acc[3] = Ct[12];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double a = -A[(size_t)(j0 + 4 * kk + lk) * np + row0 + li];
        const double b = X[(size_t)(col0 + li) * np + j0 + 4 * kk + lk];
        acc = mfma4(a, b, acc);
      }
      Ct[0] = acc[0];
      Ct[4] = acc[1];
      Ct[8] = acc[2];
      Ct[12] = acc[3];
    }
    __syncthreads();
  }
}

// T = C X; S = D - T[:, :k], g = -R_tr + T[:, k_pad]; compact copies of Y and z.
__global__ __launch_bounds__(BLK) void k_schur(DevPlan P, int e0, double *S, double *g, double *Y, double *z) {
  const int el = blockIdx.x, e = e0 + el;
  const int np = P.n_pad, kp = P.k_pad, kx = P.kx, n = P.n, k = P.k;
  const double *X = P.X + (size_t)el * kx * np;
  const double *C = P.C + (size_t)el * np * kp;
  const double *Dm = P.D + (size_t)el * kp * kp;
  const double *Rt = P.Rt + (size_t)el * kp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ntr = kp / 16, ntc = kx / 16;
  double *Se = S + (size_t)e * k * k;
  double *ge = g + (size_t)e * k;
  for (int t = wave; t < ntr * ntc; t += 4) {
    const int ti = t % ntr, tj = t / ntr;
    const int row0 = ti * 16, col0 = tj * 16;
    if (col0 > kp) continue;   // columns after the z column are padding
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < np; kk += 4) {
      const double a = C[(size_t)(kk + lk) * kp + row0 + li];
      const double b = X[(size_t)(col0 + li) * np + kk + lk];
      acc = mfma4(a, b, acc);
    }
    const int col = col0 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + lk + 4 * r;
      if (row >= k) continue;
      if (col < k) Se[(size_t)col * k + row] = Dm[(size_t)col * kp + row] - acc[r];
      else if (col == kp) ge[row] = -Rt[row] + acc[r];
    }
  }
  double *Ye = Y + (size_t)e * n * k;
  for (size_t i = tid; i < (size_t)n * k; i += BLK) {
    const size_t col = i / n, row = i % n;
    Ye[i] = X[col * np + row];
  }
  for (int i = tid; i < n; i += BLK) z[(size_t)e * n + i] = X[(size_t)kp * np + i];
}

__global__ void k_copy_resid(DevPlan P, int e0, double *Rl, double *Rtr) {
  const int el = blockIdx.x, e = e0 + el;
  const int np = P.n_pad, kp = P.k_pad, kx = P.kx;
  const double *X = P.X + (size_t)el * kx * np;
  for (int i = threadIdx.x; i < P.n; i += blockDim.x)
    if (Rl) Rl[(size_t)e * P.n + i] = X[(size_t)kp * np + i];
  for (int i = threadIdx.x; i < P.k; i += blockDim.x)
    if (Rtr) Rtr[(size_t)e * P.k + i] = P.Rt[(size_t)el * kp + i];
}

}  // namespace

// LDS of the split LU: the whole first panel where it fits, else LU_RL of its rows
size_t lu_lds_bytes(int np) { return (size_t)(np < LU_RL ? np : LU_RL) * PS * sizeof(double); }

hipError_t launch_lu(const DevPlan &P, int ec, int32_t *status, hipStream_t s) {
  const size_t lds = lu_lds_bytes(P.n_pad);
  const bool big = P.n_pad > LU_RL;
  hipError_t e = set_dyn_lds(big ? (const void *)k_lu<true> : (const void *)k_lu<false>, lds);
  if (e) return e;
  if (big)
    hipLaunchKernelGGL(k_lu<true>, dim3(ec), dim3(BLK), lds, s, P, status);
  else
    hipLaunchKernelGGL(k_lu<false>, dim3(ec), dim3(BLK), lds, s, P, status);
  return hipGetLastError();
}

hipError_t launch_solve(const DevPlan &P, int ec, hipStream_t s) {
  hipLaunchKernelGGL(k_solve, dim3(ec), dim3(BLK), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_schur(const DevPlan &P, int e0, int ec, double *S, double *g, double *Y, double *z,
                        double *Rloc, double *Rtr, hipStream_t s) {
  (void)Rloc;
  (void)Rtr;
  hipLaunchKernelGGL(k_schur, dim3(ec), dim3(BLK), 0, s, P, e0, S, g, Y, z);
  return hipGetLastError();
}

hipError_t launch_copy_resid(const DevPlan &P, int e0, int ec, double *Rloc, double *Rtr, hipStream_t s) {
  if (!Rloc && !Rtr) return hipSuccess;
  hipLaunchKernelGGL(k_copy_resid, dim3(ec), dim3(256), 0, s, P, e0, Rloc, Rtr);
  return hipGetLastError();
}

// Device self-check of the MFMA operand layout assumed above: one 16x16x4
// product of known matrices compared with a scalar loop.  Returns max |err|.
__global__ void k_mfma_selftest(double *out) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  __shared__ double Am[16 * 4], Bm[4 * 16];
  for (int t = threadIdx.x; t < 64; t += 64) {
    Am[t] = 1.0 + (t % 7) * 0.25 - (t / 7) * 0.125;   // A[i][k] at i*4 + k
    Bm[t] = 0.5 - (t % 5) * 0.375 + (t / 11) * 0.0625; // B[k][j] at k*16 + j
  }
  __syncthreads();
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  acc = mfma4(Am[li * 4 + lk], Bm[lk * 16 + li], acc);
  double err = 0.0;
  for (int r = 0; r < 4; ++r) {
    const int i = lk + 4 * r, j = li;
    double ref = 0.0;
    for (int kk = 0; kk < 4; ++kk) ref += Am[i * 4 + kk] * Bm[kk * 16 + j];
    err = fmax(err, fabs(ref - acc[r]));
  }
  __shared__ double red[64];
  red[lane] = err;
  __syncthreads();
  if (lane == 0) {
    double m = 0.0;
    for (int i = 0; i < 64; ++i) m = fmax(m, red[i]);
    out[0] = m;
  }
}

hipError_t launch_mfma_selftest(double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_mfma_selftest, dim3(1), dim3(64), 0, s, out);
  return hipGetLastError();
}

}  // namespace hdg
