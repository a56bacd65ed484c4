// Fused static condensation of one element per workgroup, left-looking.
//
// The local elimination of the hybridized DG methods (only v_hat stays globally
// coupled) needs, per element,  A = P L U,  [Y z] = A^-1 [B R_loc],
// S = D - C Y,  g = -R_tr + C z.  Every step here works on a 32-column block
// of the matrix held in LDS (n_pad x 32 doubles) while the factors and the
// coupling blocks are streamed from HBM once per block: each streamed double
// feeds 32 FMAs, which keeps the FP64 matrix cores ahead of the memory system.
//
// * LU (left-looking): block J is gathered through the current row permutation,
//   updated by all previous blocks (unit-lower triangle solves and MFMA
//   updates), then factored in LDS with partial pivoting.  Factored columns are
//   stored at their ORIGINAL row index, so later row interchanges only touch the
//   permutation vector, never stored columns.
// * Right-hand sides [B | R_loc] in blocks of 32 columns: permutation gather,
//   forward and backward substitution against the stored factors, then the
//   Schur product C * Y_block straight from LDS into S and g.
#include "hdg_plan.hpp"

namespace hdg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int W = 32;        // block width
constexpr int BS = W + 1;    // LDS row stride of the block (doubles)
constexpr int NT = 512;      // threads per workgroup (8 wave64)
constexpr int NW = NT / 64;

__device__ inline d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct Lds {
  double *blk;   // [np][BS]
  double *tri;   // [W][BS]
  int *perm;     // [np]
  double *redv;  // [NW]
  int *redi;     // [NW]
};

// blk[i][c] = M[(c0 + c) * ld + perm[i]]  (gathered through the permutation)
__device__ inline void load_block(const Lds &s, const double *M, int ld, int c0, int np) {
  for (int t = threadIdx.x; t < np * W; t += NT) {
    const int c = t / np, i = t - c * np;
    s.blk[i * BS + c] = M[(size_t)(c0 + c) * ld + s.perm[i]];
  }
}

__device__ inline void store_block(const Lds &s, double *M, int ld, int c0, int np) {
  for (int t = threadIdx.x; t < np * W; t += NT) {
    const int c = t / np, i = t - c * np;
    M[(size_t)(c0 + c) * ld + s.perm[i]] = s.blk[i * BS + c];
  }
}

// Stage the 32 x 32 diagonal block of the stored factors at rows / columns p0.
__device__ inline void stage_tri(const Lds &s, const double *A, int ld, int p0) {
  for (int t = threadIdx.x; t < W * W; t += NT) {
    const int kk = t / W, i = t - kk * W;
    s.tri[i * BS + kk] = A[(size_t)(p0 + kk) * ld + s.perm[p0 + i]];
  }
}

// Rows p0..p0+31 of the block <- L_pp^-1 (unit lower) or U_pp^-1 (upper) times them.
template <bool LOWER>
__device__ inline void tri_solve(const Lds &s, int p0) {
  const int tid = threadIdx.x;
  if (tid < W) {
    double x[W];
#pragma unroll
    for (int i = 0; i < W; ++i) x[i] = s.blk[(p0 + i) * BS + tid];
    if (LOWER) {
#pragma unroll
      for (int kk = 0; kk < W; ++kk)
#pragma unroll
        for (int i = kk + 1; i < W; ++i) x[i] -= s.tri[i * BS + kk] * x[kk];
    } else {
#pragma unroll
      for (int kk = W - 1; kk >= 0; --kk) {
        x[kk] /= s.tri[kk * BS + kk];
#pragma unroll
        for (int i = 0; i < kk; ++i) x[i] -= s.tri[i * BS + kk] * x[kk];
      }
    }
#pragma unroll
    for (int i = 0; i < W; ++i) s.blk[(p0 + i) * BS + tid] = x[i];
  }
}

// blk[r][:] -= sum_kk M[(p0+kk) * ld + perm[r]] * blk[p0+kk][:]  for rows r in [r_lo, r_hi)
// (r_lo, r_hi multiples of 16, disjoint from p0..p0+31).
__device__ inline void gemm_update(const Lds &s, const double *M, int ld, int p0, int r_lo, int r_hi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ntile = (r_hi - r_lo) / 16;
  for (int t = wave; t < ntile; t += NW) {
    const int r0 = r_lo + t * 16;
    const size_t grow = (size_t)s.perm[r0 + li];
    double a[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) a[kk] = -M[(size_t)(p0 + 4 * kk + lk) * ld + grow];
    d4 c0, c1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      c0[r] = s.blk[(r0 + lk + 4 * r) * BS + li];
      c1[r] = s.blk[(r0 + lk + 4 * r) * BS + 16 + li];
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const double *brow = s.blk + (p0 + 4 * kk + lk) * BS;
      c0 = mfma4(a[kk], brow[li], c0);
      c1 = mfma4(a[kk], brow[16 + li], c1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      s.blk[(r0 + lk + 4 * r) * BS + li] = c0[r];
      s.blk[(r0 + lk + 4 * r) * BS + 16 + li] = c1[r];
    }
  }
}

// Unblocked LU with partial pivoting of block rows j0..np-1 (block columns 0..31).
__device__ inline bool panel_factor(const Lds &s, int j0, int np) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  bool singular = false;
  for (int jj = 0; jj < W; ++jj) {
    const int r = j0 + jj;
    double best = -1.0;
    int bi = r;
    for (int i = r + tid; i < np; i += NT) {
      const double a = fabs(s.blk[i * BS + jj]);
      if (a > best) {
        best = a;
        bi = i;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      s.redv[wave] = best;
      s.redi[wave] = bi;
    }
    __syncthreads();
    best = s.redv[0];
    bi = s.redi[0];
    for (int w2 = 1; w2 < NW; ++w2) {
      const double ob = s.redv[w2];
      const int oi = s.redi[w2];
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const bool zero = !(best > 0.0);
    singular |= zero;
    if (!zero && bi != r) {
      if (tid < W) {
        const double t0 = s.blk[r * BS + tid];
        s.blk[r * BS + tid] = s.blk[bi * BS + tid];
        s.blk[bi * BS + tid] = t0;
      } else if (tid == W) {
        const int t0 = s.perm[r];
        s.perm[r] = s.perm[bi];
        s.perm[bi] = t0;
      }
    }
    __syncthreads();
    if (!zero) {
      const double inv = 1.0 / s.blk[r * BS + jj];
      for (int i = r + 1 + tid; i < np; i += NT) {
        const double l = s.blk[i * BS + jj] * inv;
        s.blk[i * BS + jj] = l;
        for (int c = jj + 1; c < W; ++c) s.blk[i * BS + c] -= l * s.blk[r * BS + c];
      }
    }
    __syncthreads();
  }
  return singular;
}

__global__ __launch_bounds__(NT) void k_condense(DevPlan P, int e0, int32_t *status, double *S, double *g,
                                                 double *Y, double *z) {
  extern __shared__ double smem[];
  const int el = blockIdx.x, e = e0 + el;
  const int np = P.n_pad, kp = P.k_pad, kx = P.kx, n = P.n, k = P.k;
  double *A = P.A + (size_t)el * np * np;
  const double *X = P.X + (size_t)el * kx * np;
  const double *C = P.C + (size_t)el * np * kp;
  const double *Dm = P.D + (size_t)el * kp * kp;
  const double *Rt = P.Rt + (size_t)el * kp;
  Lds s;
  s.blk = smem;
  s.tri = s.blk + (size_t)np * BS;
  s.perm = reinterpret_cast<int *>(s.tri + W * BS);
  s.redv = reinterpret_cast<double *>(s.perm + np);
  s.redi = reinterpret_cast<int *>(s.redv + NW);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nJ = np / W;

  for (int i = tid; i < np; i += NT) s.perm[i] = i;
  __syncthreads();
  bool singular = false;

  // ---- LU, left-looking over 32-column blocks
  for (int J = 0; J < nJ; ++J) {
    const int j0 = J * W;
    load_block(s, A, np, j0, np);
    __syncthreads();
    for (int Pp = 0; Pp < J; ++Pp) {
      const int p0 = Pp * W;
      stage_tri(s, A, np, p0);
      __syncthreads();
      tri_solve<true>(s, p0);
      __syncthreads();
      gemm_update(s, A, np, p0, p0 + W, np);
      __syncthreads();
    }
    singular |= panel_factor(s, j0, np);
    store_block(s, A, np, j0, np);
    __syncthreads();
  }

  // ---- right-hand sides, 32 columns at a time, then the Schur product
  double *Se = S + (size_t)e * k * k;
  double *ge = g + (size_t)e * k;
  double *Ye = Y + (size_t)e * n * k;
  const int ntr = kp / 16;
  for (int c0 = 0; c0 < kx; c0 += W) {
    load_block(s, X, np, c0, np);
    __syncthreads();
    for (int Pp = 0; Pp < nJ; ++Pp) {
      const int p0 = Pp * W;
      stage_tri(s, A, np, p0);
      __syncthreads();
      tri_solve<true>(s, p0);
      __syncthreads();
      if (p0 + W < np) gemm_update(s, A, np, p0, p0 + W, np);
      __syncthreads();
    }
    for (int Pp = nJ - 1; Pp >= 0; --Pp) {
      const int p0 = Pp * W;
      stage_tri(s, A, np, p0);
      __syncthreads();
      tri_solve<false>(s, p0);
      __syncthreads();
      if (p0 > 0) gemm_update(s, A, np, p0, 0, p0);
      __syncthreads();
    }
    // outputs Y, z (compact)
    for (int t = tid; t < n * W; t += NT) {
      const int c = t / n, i = t - c * n;
      const int col = c0 + c;
      if (col < k) Ye[(size_t)col * n + i] = s.blk[i * BS + c];
      else if (col == kp) z[(size_t)e * n + i] = s.blk[i * BS + c];
    }
    // T = C * block (k_pad x 32): S = D - T, g = -R_tr + T
    for (int t = wave; t < ntr; t += NW) {
      const int r0 = t * 16;
      d4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
      for (int kb = 0; kb < np; kb += 32) {
        double a[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) a[kk] = C[(size_t)(kb + 4 * kk + lk) * kp + r0 + li];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const double *brow = s.blk + (kb + 4 * kk + lk) * BS;
          a0 = mfma4(a[kk], brow[li], a0);
          a1 = mfma4(a[kk], brow[16 + li], a1);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + lk + 4 * r;
        if (row >= k) continue;
        const int col0 = c0 + li, col1 = c0 + 16 + li;
        if (col0 < k) Se[(size_t)col0 * k + row] = Dm[(size_t)col0 * kp + row] - a0[r];
        else if (col0 == kp) ge[row] = -Rt[row] + a0[r];
        if (col1 < k) Se[(size_t)col1 * k + row] = Dm[(size_t)col1 * kp + row] - a1[r];
        else if (col1 == kp) ge[row] = -Rt[row] + a1[r];
      }
    }
    __syncthreads();
  }
  if (singular && tid == 0 && status[el] == HDG_OK) status[el] = HDG_ESINGULAR;
}

}  // namespace

size_t condense_lds_bytes(int np) {
  return ((size_t)np * BS + (size_t)W * BS) * sizeof(double) + (size_t)np * sizeof(int) +
         NW * (sizeof(double) + sizeof(int));
}

hipError_t launch_condense(const DevPlan &P, int e0, int ec, int32_t *status, double *S, double *g, double *Y,
                           double *z, hipStream_t s) {
  const size_t lds = condense_lds_bytes(P.n_pad);
  hipError_t e = hipFuncSetAttribute((const void *)k_condense, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e) return e;
  hipLaunchKernelGGL(k_condense, dim3(ec), dim3(NT), lds, s, P, e0, status, S, g, Y, z);
  return hipGetLastError();
}

}  // namespace hdg
