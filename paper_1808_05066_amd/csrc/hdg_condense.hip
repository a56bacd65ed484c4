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
  double *prow;  // [W] pivot row
  double *tmp;   // [W] displaced row
  int *perm;     // [np]
  double *redv;  // [2][NW]
  int *redi;     // [2][NW]
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

// Rows p0..p0+31 of the block <- Inv * rows, Inv the stored inverse of the unit-lower
// (L) or upper (U) 32 x 32 diagonal block of the factors; four waves each form one
// 16 x 16 tile on MFMA, then write back after a barrier.
__device__ inline void inv_apply(const Lds &s, const double *Inv, int p0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  const int ti = wave & 1, tj = (wave >> 1) & 1;
  if (wave < 4) {
    double a[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) a[kk] = Inv[(4 * kk + lk) * W + ti * 16 + li];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) acc = mfma4(a[kk], s.blk[(p0 + 4 * kk + lk) * BS + tj * 16 + li], acc);
  }
  __syncthreads();
  if (wave < 4) {
#pragma unroll
    for (int r = 0; r < 4; ++r) s.blk[(p0 + ti * 16 + lk + 4 * r) * BS + tj * 16 + li] = acc[r];
  }
}

// Inverses of the diagonal 32 x 32 blocks of the freshly factored panel (block rows
// j0..j0+31): wave 0 inverts the unit-lower part, wave 1 the upper part; column c
// of each inverse is solved by lane c.  Stored column-major (32 x 32) in Linv / Uinv.
__device__ inline void invert_diag(const Lds &s, int j0, double *Linv, double *Uinv) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane >= W || wave > 1) return;
  const int c = lane;
  double x[W];
  if (wave == 0) {
#pragma unroll
    for (int i = 0; i < W; ++i) x[i] = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int kk = 0; kk < W; ++kk)
#pragma unroll
      for (int i = kk + 1; i < W; ++i) x[i] -= s.blk[(j0 + i) * BS + kk] * x[kk];
#pragma unroll
    for (int i = 0; i < W; ++i) Linv[c * W + i] = x[i];
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) x[i] = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int kk = W - 1; kk >= 0; --kk) {
      x[kk] /= s.blk[(j0 + kk) * BS + kk];
#pragma unroll
      for (int i = 0; i < kk; ++i) x[i] -= s.blk[(j0 + i) * BS + kk] * x[kk];
    }
#pragma unroll
    for (int i = 0; i < W; ++i) Uinv[c * W + i] = x[i];
  }
}

// blk[r][:] -= sum_kk M[(p0+kk) * ld + perm[r]] * blk[p0+kk][:]  for rows r in [r_lo, r_hi)
// (r_lo, r_hi multiples of 16, disjoint from p0..p0+31).
__device__ inline void gemm_update(const Lds &s, const double *M, int ld, int p0, int r_lo, int r_hi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ntile = (r_hi - r_lo) / 16;
  const double *Mp = M + (size_t)(p0 + lk) * ld;
  double a[8], an[8];
  int t = wave;
  if (t < ntile) {
    const size_t grow = (size_t)s.perm[r_lo + t * 16 + li];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) a[kk] = -Mp[(size_t)(4 * kk) * ld + grow];
  }
  for (; t < ntile; t += NW) {
    const int r0 = r_lo + t * 16;
    const int tn = t + NW;
    if (tn < ntile) {
      const size_t grow = (size_t)s.perm[r_lo + tn * 16 + li];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) an[kk] = -Mp[(size_t)(4 * kk) * ld + grow];
    }
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
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) a[kk] = an[kk];
  }
}

// LU with partial pivoting of block rows j0..np-1 (block columns 0..31), in four
// sub-panels of 8 columns.  Inside a sub-panel thread t keeps the 8 entries of
// row j0+t in registers (rows beyond j0+NT, present only when np - j0 > NT,
// stay in LDS); per column the pivot is found by wave shuffles plus one
// exchange through LDS, the pivot row is published and whole rows are swapped
// in LDS: two barriers per column.  After a sub-panel, its 8 pivot rows are
// solved against the remaining columns (unit-lower 8 x 8) and the rows below
// receive the rank-8 update.
constexpr int SPW = 8;   // sub-panel width

__device__ inline bool panel_factor(const Lds &s, int j0, int np, double *prow, double *tmprow) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = j0 + tid, r1 = j0 + tid + NT;
  const bool has0 = r0 < np, has1 = r1 < np;
  double *y0 = s.blk + (size_t)r0 * BS;
  double *y1 = s.blk + (size_t)r1 * BS;
  bool singular = false;
  for (int cs = 0; cs < W; cs += SPW) {
    double x0[SPW];
#pragma unroll
    for (int c = 0; c < SPW; ++c) x0[c] = has0 ? y0[cs + c] : 0.0;
    for (int jj = 0; jj < SPW; ++jj) {
      const int col = cs + jj;
      const int r = j0 + col;
      double v0 = 0.0;
#pragma unroll
      for (int c = 0; c < SPW; ++c)
        if (c == jj) v0 = x0[c];
      double best = -1.0;
      int bi = np;
      if (has0 && r0 >= r) {
        best = fabs(v0);
        bi = r0;
      }
      if (has1) {
        const double v1 = fabs(y1[col]);
        if (v1 > best) {
          best = v1;
          bi = r1;
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
      double *rv = s.redv + (col & 1) * NW;
      int *ri = s.redi + (col & 1) * NW;
      if (lane == 0) {
        rv[wave] = best;
        ri[wave] = bi;
      }
      __syncthreads();
      best = rv[0];
      bi = ri[0];
#pragma unroll
      for (int w2 = 1; w2 < NW; ++w2) {
        const double ob = rv[w2];
        const int oi = ri[w2];
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      const bool zero = !(best > 0.0);
      singular |= zero;
      const int piv = zero ? r : bi;
      // pivot row entries of this sub-panel -> prow; if rows move, the register
      // part of row r -> tmprow and the LDS columns outside the sub-panel swap.
      if (has0 && r0 == piv) {
#pragma unroll
        for (int c = 0; c < SPW; ++c) prow[c] = x0[c];
      }
      if (has1 && r1 == piv) {
#pragma unroll
        for (int c = 0; c < SPW; ++c) prow[c] = y1[cs + c];
      }
      if (piv != r) {
        if (has0 && r0 == r) {
#pragma unroll
          for (int c = 0; c < SPW; ++c) tmprow[c] = x0[c];
        }
        if (tid < W && (tid < cs || tid >= cs + SPW)) {
          const double t0 = s.blk[r * BS + tid];
          s.blk[r * BS + tid] = s.blk[piv * BS + tid];
          s.blk[piv * BS + tid] = t0;
        }
        if (tid == W) {
          const int t0 = s.perm[r];
          s.perm[r] = s.perm[piv];
          s.perm[piv] = t0;
        }
      }
      __syncthreads();
      if (piv != r) {
        if (has0 && r0 == piv) {
#pragma unroll
          for (int c = 0; c < SPW; ++c) x0[c] = tmprow[c];
        } else if (has0 && r0 == r) {
#pragma unroll
          for (int c = 0; c < SPW; ++c) x0[c] = prow[c];
        }
        if (has1 && r1 == piv) {
#pragma unroll
          for (int c = 0; c < SPW; ++c) y1[cs + c] = tmprow[c];
        }
      }
      if (!zero) {
        const double inv = 1.0 / prow[jj];
        if (has0 && r0 > r) {
          double l0 = 0.0;
#pragma unroll
          for (int c = 0; c < SPW; ++c)
            if (c == jj) l0 = x0[c] * inv;
#pragma unroll
          for (int c = 0; c < SPW; ++c) {
            if (c == jj) x0[c] = l0;
            else if (c > jj) x0[c] -= l0 * prow[c];
          }
        }
        if (has1) {
          const double l1 = y1[col] * inv;
          y1[col] = l1;
          for (int c = jj + 1; c < SPW; ++c) y1[cs + c] -= l1 * prow[c];
        }
      }
    }
    if (has0) {
#pragma unroll
      for (int c = 0; c < SPW; ++c) y0[cs + c] = x0[c];
    }
    __syncthreads();
    if (cs + SPW < W) {
      // pivot rows j0+cs..j0+cs+7 of the remaining columns: unit-lower 8 x 8 solve
      const int rp = j0 + cs;
      if (tid < W - cs - SPW) {
        const int c = cs + SPW + tid;
        double u[SPW];
#pragma unroll
        for (int i = 0; i < SPW; ++i) u[i] = s.blk[(rp + i) * BS + c];
#pragma unroll
        for (int k = 0; k < SPW; ++k)
#pragma unroll
          for (int i = k + 1; i < SPW; ++i) u[i] -= s.blk[(rp + i) * BS + cs + k] * u[k];
#pragma unroll
        for (int i = 0; i < SPW; ++i) s.blk[(rp + i) * BS + c] = u[i];
      }
      __syncthreads();
      // rank-8 update of the rows below
      for (int i = rp + SPW + tid; i < np; i += NT) {
        double l[SPW];
#pragma unroll
        for (int k = 0; k < SPW; ++k) l[k] = s.blk[i * BS + cs + k];
        for (int c = cs + SPW; c < W; ++c) {
          double acc = s.blk[i * BS + c];
#pragma unroll
          for (int k = 0; k < SPW; ++k) acc -= l[k] * s.blk[(rp + k) * BS + c];
          s.blk[i * BS + c] = acc;
        }
      }
      __syncthreads();
    }
  }
  return singular;
}

__global__ __launch_bounds__(NT) void k_condense(DevPlan P, int e0, int32_t *status, double *S, double *g,
                                                 double *Y, double *z, double *inv) {
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
  s.prow = s.blk + (size_t)np * BS;
  s.tmp = s.prow + W;
  s.perm = reinterpret_cast<int *>(s.tmp + W);
  s.redv = reinterpret_cast<double *>(s.perm + np);
  s.redi = reinterpret_cast<int *>(s.redv + 2 * NW);
  // inverses of the diagonal blocks: [nJ][2][W][W] per element
  double *Ie = inv + (size_t)el * (np / W) * 2 * W * W;
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
      inv_apply(s, Ie + (size_t)Pp * 2 * W * W, p0);
      __syncthreads();
      gemm_update(s, A, np, p0, p0 + W, np);
      __syncthreads();
    }
    singular |= panel_factor(s, j0, np, s.prow, s.tmp);
    __syncthreads();
    invert_diag(s, j0, Ie + (size_t)J * 2 * W * W, Ie + (size_t)J * 2 * W * W + W * W);
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
      inv_apply(s, Ie + (size_t)Pp * 2 * W * W, p0);
      __syncthreads();
      if (p0 + W < np) gemm_update(s, A, np, p0, p0 + W, np);
      __syncthreads();
    }
    for (int Pp = nJ - 1; Pp >= 0; --Pp) {
      const int p0 = Pp * W;
      inv_apply(s, Ie + (size_t)Pp * 2 * W * W + W * W, p0);
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
      const double *Cr = C + (size_t)lk * kp + r0 + li;
      double a[8], an[8];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) a[kk] = Cr[(size_t)(4 * kk) * kp];
      for (int kb = 0; kb < np; kb += 32) {
        if (kb + 32 < np) {
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) an[kk] = Cr[(size_t)(kb + 32 + 4 * kk) * kp];
        }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const double *brow = s.blk + (kb + 4 * kk + lk) * BS;
          a0 = mfma4(a[kk], brow[li], a0);
          a1 = mfma4(a[kk], brow[16 + li], a1);
        }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) a[kk] = an[kk];
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
  return ((size_t)np * BS + 2 * W) * sizeof(double) + (size_t)np * sizeof(int) +
         2 * NW * (sizeof(double) + sizeof(int));
}

size_t condense_inv_doubles(int np) { return (size_t)(np / W) * 2 * W * W; }

hipError_t launch_condense(const DevPlan &P, int e0, int ec, int32_t *status, double *S, double *g, double *Y,
                           double *z, hipStream_t s) {
  double *inv = P.inv;
  const size_t lds = condense_lds_bytes(P.n_pad);
  hipError_t e = hipFuncSetAttribute((const void *)k_condense, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e) return e;
  hipLaunchKernelGGL(k_condense, dim3(ec), dim3(NT), lds, s, P, e0, status, S, g, Y, z, inv);
  return hipGetLastError();
}

}  // namespace hdg
