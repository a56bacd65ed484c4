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
//   stored in pivot-position order; the row interchanges of a later panel are
//   also applied to the stored columns of the earlier panels (as LAPACK's laswp,
//   once per panel as one row movement), which keeps every later read of the
//   factors contiguous.
// * Right-hand sides [B | R_loc] in blocks of 32 columns: permutation gather,
//   forward and backward substitution against the stored factors, then the
//   Schur product C * Y_block straight from LDS into S and g.
//
// The same kernel, instantiated for FP32, is the low-precision factorization of
// the mixed-precision path: the FP64 blocks are symmetrically scaled by powers
// of two, D A D with d_i = 2^-round(log2 sqrt|a_ii|) (exact in binary), rounded
// to FP32 on their way into LDS, factored and solved on the FP32 matrix cores
// (FP32 accumulation); Y = D Y_hat and z = D z_hat are unscaled on output and
// the factors, pivots, scales and diagonal-block inverses are kept for the
// refinement solves.
#include <utility>

#include "hdg_plan.hpp"

namespace hdg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Block width W (32, or 16 where a 32-column block does not fit in LDS); the
// LDS row stride of the block is W + 1 elements.
constexpr int WMAX = 32;
constexpr int NT = 512;      // threads per workgroup (8 wave64)
constexpr int NW = NT / 64;

// Matrix-core tile 16 x 16 x 4 per element type.  Operands: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator r of lane l holds
// C[row(l / 16, r)][l % 16] with the row map below (measured on gfx950: the
// FP64 and FP32 instructions distribute rows differently).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc;
  __device__ static inline acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma<float> {
  typedef f4 acc;
  __device__ static inline acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int r) { return 4 * lk + r; }
};

// BF16 operands, FP32 accumulation (the low-precision path with LP == 2).  A panel of 4 KS
// k values is held as the 16x16x4 instructions take it: lane (li, lk) has a[kk] = A[li][lk + 4 kk]
// and b[kk] = B[lk + 4 kk][li], kk < KS.  The 16x16x(4 KS) BF16 instruction sums, for every
// lane group g = lk, over its KS slots i the products of slot i of the A lane (row li, group g)
// and slot i of the B lane (column li, group g): putting the lane's own kk into slot i = kk gives
// every k of the panel exactly once, the panel's product summed in another order.  The
// accumulators keep the FP32 16x16 layout.  Operands are rounded to BF16 (nearest, ties even).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
template <int KS>
struct BfPanel;
template <>
struct BfPanel<8> {
  typedef bf16x8 op;
  template <typename F>
  __device__ static inline op pack(F f) {
    op v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (__bf16)f(i);
    return v;
  }
  __device__ static inline f4 mma(op a, op b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <>
struct BfPanel<4> {
  typedef bf16x4 op;
  template <typename F>
  __device__ static inline op pack(F f) {
    op v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (__bf16)f(i);
    return v;
  }
  __device__ static inline f4 mma(op a, op b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(i16x4, a), __builtin_bit_cast(i16x4, b), c,
                                                     0, 0, 0);
  }
};

// acc + sum over the panel's k of a[k] b[k] for this lane's operands (see above): KS 16x16x4
// instructions in the operands' precision, or with BF one BF16 instruction
template <typename T, bool BF, int KS, typename Fb>
__device__ __forceinline__ typename Mfma<T>::acc mma_panel(const T (&a)[KS], Fb b, typename Mfma<T>::acc c) {
  if constexpr (BF) {
    typedef BfPanel<KS> BP;
    return BP::mma(BP::pack([&](int i) { return a[i]; }), BP::pack(b), c);
  } else {
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) c = Mfma<T>::op(a[kk], b(kk), c);
    return c;
  }
}

template <typename T>
struct Lds {
  T *blk;        // [np][BS]
  T *crow;       // [2][NW + 1][8] pivot candidate rows and diagonal row, by column parity
  int *perm;     // [np]
  int *redi;     // [2][NW] pivot keys of the waves
  double *dsc;   // [np] symmetric scaling (low-precision path only)
  int *invb;     // [np] original row -> position before the current panel
  int *mvx;      // [2W] positions changed by the panel's interchanges
  int *mvy;      // [2W] position each of them takes its value from
  int *mvn;      // [1] number of changed positions
};

// Thread index of the helpers below, by workgroup size.  The 256-thread kernels run the LU's
// loop over column blocks (and the batch's loop over elements) with a large live state: they
// read it through cur_tid, so that index arithmetic is recomputed inside each helper instead of
// being held, and spilled, across the loop.  The 1024-thread right-hand-side kernels hold few
// registers per thread and read threadIdx.x directly: cur_tid's volatile asm also fixes the
// order of the loads around it, which these load-bound kernels pay for.
template <int NTT>
__device__ __forceinline__ int tid_of() {
  if constexpr (NTT >= 1024) return (int)threadIdx.x;
  else return cur_tid();
}

// blk[i][c] = M[(c0 + c) * ld + perm[i]]  (gathered through the permutation;
// each thread keeps LU loads in flight before writing them to LDS)
constexpr int LU = 8;

template <typename T, int W, int NTT = NT, typename Fetch>
__device__ inline void load_block_f(const Lds<T> &s, int np, Fetch fetch) {
  constexpr int BS = W + 1;
  const int total = np * W;
  for (int t0 = tid_of<NTT>(); t0 < total; t0 += LU * NTT) {
    T v[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int t = t0 + u * NTT;
      if (t < total) {
        const int c = t / np, i = t - c * np;
        v[u] = fetch(c, s.perm[i]);
      }
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int t = t0 + u * NTT;
      if (t < total) {
        const int c = t / np, i = t - c * np;
        s.blk[i * BS + c] = v[u];
      }
    }
  }
}

template <typename T, int W, int NTT = NT>
__device__ inline void load_block(const Lds<T> &s, const T *M, int ld, int c0, int np) {
  load_block_f<T, W, NTT>(s, np, [&](int c, int o) { return M[(size_t)(c0 + c) * ld + o]; });
}

// Same with the symmetric scaling of the low-precision path (rows always, columns
// if colscale), converting to T; fetch(c, o) returns the FP64 entry.
template <typename T, int W, int NTT = NT, typename Fetch>
__device__ inline void load_block_scaled_f(const Lds<T> &s, int c0, int np, bool colscale, Fetch fetch) {
  constexpr int BS = W + 1;
  const int total = np * W;
  for (int t0 = tid_of<NTT>(); t0 < total; t0 += LU * NTT) {
    double v[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int t = t0 + u * NTT;
      if (t < total) {
        const int c = t / np, i = t - c * np;
        v[u] = fetch(c, s.perm[i]);
      }
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int t = t0 + u * NTT;
      if (t < total) {
        const int c = t / np, i = t - c * np;
        double x = v[u] * s.dsc[s.perm[i]];
        if (colscale) x *= s.dsc[c0 + c];
        s.blk[i * BS + c] = (T)x;
      }
    }
  }
}

template <typename T, int W, int NTT = NT>
__device__ inline void load_block_scaled(const Lds<T> &s, const double *M, int ld, int c0, int np, bool colscale) {
  load_block_scaled_f<T, W, NTT>(s, c0, np, colscale, [&](int c, int o) { return M[(size_t)(c0 + c) * ld + o]; });
}

// Entry (o, col) of the local block A of an element (A64: its stored block, mg: its compact
// M and G_j).  Without the compact copy every entry is stored; with it only the v rows are
// (the contraction leaves the q rows and the padding unwritten), and the rest follows from
// the block structure: the q row (c, j, a) holds G_j[a][b] in the v column (c, b) and
// M[a][b] in the q column (c, j, b), zero elsewhere; the padding is the identity.
__device__ inline double a_entry(const DevPlan &P, const double *A64, const double *mg, int o, int col) {
  const int nv = P.m * P.Np;
  if (!mg || (o < nv && col < P.n)) return A64[(size_t)col * P.n_pad + o];
  if (o < nv) return 0.0;
  if (o >= P.n || col >= P.n) return o == col ? 1.0 : 0.0;
  const int ro = P.uinfo[o], rc = P.uinfo[col];
  if ((ro >> 12) != (rc >> 12)) return 0.0;
  const int a = ro & 255, b = rc & 255, j = (ro >> 8) & 15;
  if (col < nv) return mg[(j * P.Np + a) * P.Np + b];
  return j == ((rc >> 8) & 15) ? mg[(P.dim * P.Np + a) * P.Np + b] : 0.0;
}

// Block j0 of A (gathered through perm, scaled in the low-precision path) when only its v rows
// are stored: the v rows are read, the q rows and the padding start as zero / identity, and
// after a barrier the nonzeros of the q rows in these columns are placed through the inverse
// permutation (invb, formed here in full) -- at most d N_p per column.  The caller's barrier
// follows.
template <typename T, int LP, int W>
__device__ inline void load_block_formed(const Lds<T> &s, const DevPlan &P, const double *A64, const double *mg,
                                         int j0) {
  constexpr int BS = W + 1;
  const int np = P.n_pad, n = P.n, Np = P.Np, D = P.dim, nv = P.m * Np, DN = D * Np;
  for (int x = cur_tid(); x < np; x += NT) s.invb[s.perm[x]] = x;
  const auto fetch = [&](int c, int o) {
    const int col = j0 + c;
    if (o < nv) return col < n ? A64[(size_t)col * np + o] : 0.0;
    return (o == col && o >= n) ? 1.0 : 0.0;
  };
  if constexpr (LP) load_block_scaled_f<T, W>(s, j0, np, true, fetch);
  else load_block_f<T, W>(s, np, fetch);
  __syncthreads();
  for (int t = cur_tid(); t < W * DN; t += NT) {
    const int c = t / DN, r = t - c * DN, col = j0 + c;
    if (col >= n) continue;
    int o;
    double val;
    if (col < nv) {
      // v column (cc, b): G_j[a][b] in the q rows (cc, j, a)
      const int cc = col / Np, b = col - cc * Np, j = r / Np, a = r - j * Np;
      o = nv + (cc * D + j) * Np + a;
      val = mg[(j * Np + a) * Np + b];
    } else {
      // q column (cc, jj, b): M[a][b] in the q rows (cc, jj, a)
      if (r >= Np) continue;
      const int qc = col - nv, cj = qc / Np, b = qc - cj * Np;
      o = nv + cj * Np + r;
      val = mg[(D * Np + r) * Np + b];
    }
    if constexpr (LP) val *= s.dsc[o] * s.dsc[col];
    s.blk[s.invb[o] * BS + c] = (T)val;
  }
}

// factored block -> M at pivot position (row i of the block is position i)
template <typename T, int W>
__device__ inline void store_block(const Lds<T> &s, T *M, int ld, int c0, int np) {
  constexpr int BS = W + 1;
  for (int t = cur_tid(); t < np * W; t += NT) {
    const int c = t / np, i = t - c * np;
    M[(size_t)(c0 + c) * ld + i] = s.blk[i * BS + c];
  }
}

// Barrier for exchanges through LDS only: waits for this wave's LDS operations, not for its
// global loads.  __syncthreads() also waits for every outstanding global load, which in the
// blocked sweeps below would expose the full memory latency of the operands prefetched for
// the next step at every step; here those loads stay in flight across the barrier (each
// wave consumes only its own loads, and the compiler waits for them where they are used).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// One step "apply diagonal-block inverse, then update the other rows" of a
// blocked triangular sweep.  Both global operands of a step (the W x W inverse
// and the first row tile of the factor panel) are loaded one step ahead into
// registers, so their latency overlaps the previous step.
struct Step {
  int inv;          // offset of the W x W inverse in the inverse table (-1: no step)
  int p0;           // first row / factor column of the diagonal block
  int r_lo, r_hi;   // rows updated by the panel p0..p0+W-1 (empty if r_lo >= r_hi)
};

template <typename T, int W, int NTT = NT>
__device__ inline void load_inv(T (&ia)[W / 4], const T *Ie, const Step &st) {
  constexpr int TW = W / 16;
  const int tid = tid_of<NTT>(), lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (st.inv < 0 || wave >= TW * TW) return;
  const T *Inv = Ie + st.inv;
  const int ti = wave % TW;
#pragma unroll
  for (int kk = 0; kk < W / 4; ++kk) ia[kk] = Inv[(4 * kk + lk) * W + ti * 16 + li];
}

template <typename T, int W, int NTT = NT>
__device__ inline void load_tile(T (&a)[W / 4], const T *M, int ld, const Step &st) {
  const int tid = tid_of<NTT>(), lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (st.inv < 0 || st.r_lo + wave * 16 >= st.r_hi) return;
  const T *Mb = M + (size_t)st.p0 * ld;
  const int o0 = lk * ld + st.r_lo + wave * 16 + li;
#pragma unroll
  for (int kk = 0; kk < W / 4; ++kk) a[kk] = -Mb[o0 + 4 * kk * ld];
}

// Rows p0..p0+W-1 of the block <- Inv * rows, Inv (preloaded in ia) the stored
// inverse of the unit-lower (L) or upper (U) W x W diagonal block of the factors;
// (W/16)^2 waves each form one 16 x 16 tile on MFMA, then write back after a
// barrier.  The inverse of the next step is loaded into ia meanwhile.
template <typename T, int W, int NTT = NT, bool BF = false>
__device__ inline void inv_apply(const Lds<T> &s, T (&ia)[W / 4], int p0, const T *Ie, const Step &next) {
  typedef Mfma<T> MF;
  constexpr int BS = W + 1, TW = W / 16;
  const int tid = tid_of<NTT>(), lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  typename MF::acc acc = {0, 0, 0, 0};
  const int ti = wave % TW, tj = wave / TW;
  if (wave < TW * TW)
    acc = mma_panel<T, BF, W / 4>(ia, [&](int kk) { return s.blk[(p0 + 4 * kk + lk) * BS + tj * 16 + li]; }, acc);
  load_inv<T, W, NTT>(ia, Ie, next);
  lds_barrier();
  if (wave < TW * TW) {
#pragma unroll
    for (int r = 0; r < 4; ++r) s.blk[(p0 + ti * 16 + MF::row(lk, r)) * BS + tj * 16 + li] = acc[r];
  }
}

// Wave-wide reductions on the DPP network: within each row of 16 lanes by quad
// permutations and row rotations (every lane ends with its row's result), then
// across the four rows by reading lanes 0, 16, 32, 48.  All 64 lanes must be active.
template <int CTRL>
__device__ inline int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
__device__ inline double lane_val(double v, int l) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ inline float lane_val(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
constexpr int DPP_QUAD_1032 = 0xB1, DPP_QUAD_2301 = 0x4E, DPP_ROW_ROR4 = 0x124, DPP_ROW_ROR8 = 0x128;

__device__ inline unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)dpp_i32<DPP_QUAD_1032>((int)v));
  v = max(v, (unsigned)dpp_i32<DPP_QUAD_2301>((int)v));
  v = max(v, (unsigned)dpp_i32<DPP_ROW_ROR4>((int)v));
  v = max(v, (unsigned)dpp_i32<DPP_ROW_ROR8>((int)v));
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0), b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32), d = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(a, b), max(c, d));
}

// Pivot key of row `row` (< 2048) in the LDS kernels: the magnitude's exponent and leading
// mantissa bits (10 of FP64, 13 of FP32), then the lower row; exact partial pivoting up to a
// relative 2^-10 (FP64) / 2^-13 (FP32) between near-equal candidates.  One wave maximum and one
// maximum over the waves' winners replace a maximum of the value and a minimum of the row.
__device__ inline unsigned mag_key(double a, int row) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, fabs(a));
  return ((unsigned)(b >> 42) << 11) | (unsigned)(2047 - row);
}
__device__ inline unsigned mag_key(float a, int row) {
  const unsigned b = __builtin_bit_cast(unsigned, fabsf(a));
  return ((b >> 10) << 11) | (unsigned)(2047 - row);
}
// 1 / x from the hardware estimate and Newton steps (two in FP64, one in FP32)
__device__ inline double rcp_newton(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ inline float rcp_newton(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Inverses of the diagonal W x W blocks of the freshly factored panel (block rows
// j0..j0+W-1): wave 0 inverts the unit-lower part, wave 1 the upper part; column c
// of each inverse is solved by lane c.  Stored column-major (W x W) in Linv / Uinv.
template <typename T, int W>
__device__ inline void invert_diag(const Lds<T> &s, int j0, T *Linv, T *Uinv) {
  constexpr int BS = W + 1;
  const int tid = cur_tid(), lane = tid & 63, wave = tid >> 6;
  if (lane >= W || wave > 1) return;
  // c is made opaque to the optimizer: otherwise the identity columns below are hoisted
  // out of the caller's block loop and stay live (2W registers) through every phase
  int c = lane;
  asm volatile("" : "+v"(c));
  T x[W];
  if (wave == 0) {
#pragma unroll
    for (int i = 0; i < W; ++i) x[i] = (i == c) ? T(1) : T(0);
#pragma unroll
    for (int kk = 0; kk < W; ++kk)
#pragma unroll
      for (int i = kk + 1; i < W; ++i) x[i] -= s.blk[(j0 + i) * BS + kk] * x[kk];
#pragma unroll
    for (int i = 0; i < W; ++i) Linv[c * W + i] = x[i];
  } else {
    // reciprocal of the diagonal entry of column c, one division per lane; lane kk's
    // reciprocal is read by every lane in the sweep (no division in the dependent chain)
    const T rc = T(1) / s.blk[(j0 + c) * BS + c];
#pragma unroll
    for (int i = 0; i < W; ++i) x[i] = (i == c) ? T(1) : T(0);
#pragma unroll
    for (int kk = W - 1; kk >= 0; --kk) {
      x[kk] *= lane_val(rc, kk);
#pragma unroll
      for (int i = 0; i < kk; ++i) x[i] -= s.blk[(j0 + i) * BS + kk] * x[kk];
    }
#pragma unroll
    for (int i = 0; i < W; ++i) Uinv[c * W + i] = x[i];
  }
}

// blk[r][:] -= sum_kk M[(p0+kk) * ld + r] * blk[p0+kk][:]  for rows r in [r_lo, r_hi)
// (stored factors are in pivot-position order, so the loads are contiguous;
// r_lo, r_hi multiples of 16, disjoint from p0..p0+W-1).  Wave w updates the row
// tiles w, w + NWT, ...; its first tile arrives preloaded in a, and the factor
// tiles of its next MT - 1 tiles and the first tile of the next step are all
// requested before the first MFMA, so one memory latency is exposed per step
// rather than one per tile (a step is short next to a load from memory).  Tiles
// beyond the first MT of a wave (large blocks) are fetched one tile ahead.
template <typename T, int W, int NTT = NT, int MT = 5, bool BF = false>
__device__ inline void gemm_update(const Lds<T> &s, T (&a)[W / 4], const T *M, int ld, const Step &st,
                                   const Step &next) {
  constexpr int NWT = NTT / 64;
  typedef Mfma<T> MF;
  constexpr int BS = W + 1, TW = W / 16, KS = W / 4;
  const int tid = tid_of<NTT>(), lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int p0 = st.p0, r_lo = st.r_lo;
  const int ntile = st.r_hi > r_lo ? (st.r_hi - r_lo) / 16 : 0;
  // uniform base, 32-bit lane offsets (a block has fewer than 2^31 entries)
  const T *Mb = M + (size_t)p0 * ld;
  const int o0 = lk * ld + r_lo + li;
  T ab[MT][KS];
#pragma unroll
  for (int u = 1; u < MT; ++u) {
    const int t = wave + u * NWT;
    if (t < ntile) {
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) ab[u][kk] = -Mb[o0 + 4 * kk * ld + t * 16];
    }
  }
  T an[KS];
  load_tile<T, W, NTT>(an, M, ld, next);
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) ab[0][kk] = a[kk];
  const auto tile = [&](int t, const T (&op)[KS]) {
    const int r0 = r_lo + t * 16;
    typename MF::acc c[TW];
#pragma unroll
    for (int q = 0; q < TW; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) c[q][r] = s.blk[(r0 + MF::row(lk, r)) * BS + q * 16 + li];
#pragma unroll
    for (int q = 0; q < TW; ++q)
      c[q] = mma_panel<T, BF, KS>(op, [&](int kk) { return s.blk[(p0 + 4 * kk + lk) * BS + q * 16 + li]; }, c[q]);
#pragma unroll
    for (int q = 0; q < TW; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.blk[(r0 + MF::row(lk, r)) * BS + q * 16 + li] = c[q][r];
  };
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int t = wave + u * NWT;
    if (t < ntile) tile(t, ab[u]);
  }
  // remaining tiles of the wave, one tile ahead
  int t = wave + MT * NWT;
  if (t < ntile) {
    T cur[KS], nx[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) cur[kk] = -Mb[o0 + 4 * kk * ld + t * 16];
    for (; t < ntile; t += NWT) {
      const int tn = t + NWT;
      if (tn < ntile) {
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) nx[kk] = -Mb[o0 + 4 * kk * ld + tn * 16];
      }
      tile(t, cur);
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) cur[kk] = nx[kk];
    }
  }
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) a[kk] = an[kk];
}

// A sequence of steps: spec(i) for i in [0, count), each applied with its
// operands loaded one step ahead.
template <typename T, int W, typename Spec, int NTT = NT, int MT = 5, bool BF = false>
__device__ inline void run_steps(const Lds<T> &s, const T *Ie, const T *Fm, int ld, int count, Spec spec) {
  T ia[W / 4], a[W / 4];
  Step cur = spec(0);
  load_inv<T, W, NTT>(ia, Ie, cur);
  load_tile<T, W, NTT>(a, Fm, ld, cur);
  for (int i = 0; i < count; ++i) {
    const Step nxt = (i + 1 < count) ? spec(i + 1) : Step{-1, 0, 0, 0};
    inv_apply<T, W, NTT, BF>(s, ia, cur.p0, Ie, nxt);
    lds_barrier();
    gemm_update<T, W, NTT, MT, BF>(s, a, Fm, ld, cur, nxt);
    lds_barrier();
    cur = nxt;
  }
}

// LU with partial pivoting of block rows j0..np-1 (block columns 0..W-1), in
// sub-panels of 8 columns.  Inside a sub-panel thread t keeps the 8 entries of
// row j0+t in registers (its rows j0+t+NT, j0+t+2NT, ... stay in LDS).  One
// barrier per column: each wave takes the maximum of its candidates' pivot keys
// (magnitude, then the lowest row; mag_key) on the DPP network and the winning
// lane publishes the key with its row's 8 sub-panel entries, next to the entries
// of the diagonal row; after the barrier every wave takes the largest of the NW
// keys and applies the interchange and the rank-1 update to its own rows (the
// interchanges of the columns outside the sub-panel and of perm wait for the
// sub-panel's end, where they are applied as one row movement).  The publication
// slots are double-buffered by column parity, so the next column's writes cannot
// overtake this column's reads.  After a sub-panel, its 8 pivot rows are solved
// against the remaining columns (unit-lower 8 x 8) and the rows below receive
// the rank-8 update.
constexpr int SPW = 8;   // sub-panel width

template <typename T, int W>
__device__ inline bool panel_factor(const Lds<T> &s, int j0, int np) {
  constexpr int BS = W + 1;
  const int tid = cur_tid(), lane = tid & 63, wave = tid >> 6;
  const int r0 = j0 + tid, r1 = j0 + tid + NT;   // rows r1, r1 + NT, ... stay in LDS
  const bool has0 = r0 < np;
  T *y0 = s.blk + (size_t)r0 * BS;
  bool singular = false;
  for (int cs = 0; cs < W; cs += SPW) {
    T x0[SPW];
    int pivs[SPW];
#pragma unroll
    for (int c = 0; c < SPW; ++c) x0[c] = has0 ? y0[cs + c] : T(0);
#pragma unroll
    for (int jj = 0; jj < SPW; ++jj) {
      const int col = cs + jj;
      const int r = j0 + col;   // diagonal row, always thread col's register row
      const int b = jj & 1;
      T *crow = s.crow + b * (NW + 1) * SPW;   // [NW candidate rows | diagonal row][SPW]
      // this thread's candidate key (0: none)
      unsigned best = 0;
      if (has0 && r0 >= r) best = mag_key(x0[jj], r0);
      for (int rr = r1; rr < np; rr += NT) {
        const unsigned k1 = mag_key(s.blk[(size_t)rr * BS + col], rr);
        if (k1 > best) best = k1;
      }
      const unsigned wb = wave_max_u32(best);
      if (best != 0 && best == wb) {   // one lane: keys differ by row
        const int bi = 2047 - (int)(best & 2047u);
        T v[SPW];
#pragma unroll
        for (int c = 0; c < SPW; ++c) v[c] = (bi == r0) ? x0[c] : s.blk[(size_t)bi * BS + cs + c];
        T *dst = crow + wave * SPW;
#pragma unroll
        for (int c = 0; c < SPW; ++c) dst[c] = v[c];
      }
      if (lane == 0) s.redi[b * NW + wave] = (int)wb;
      if (tid == col) {
#pragma unroll
        for (int c = 0; c < SPW; ++c) crow[NW * SPW + c] = x0[c];
      }
      __syncthreads();
      // global pivot: the largest of the waves' keys
      unsigned kb = 0;
      int wv = 0;
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        const unsigned kv = (unsigned)s.redi[b * NW + v];
        if (kv > kb) {
          kb = kv;
          wv = v;
        }
      }
      const T *pr = crow + wv * SPW;
      const T *dr = crow + NW * SPW;
      T prow[SPW], drow[SPW];
#pragma unroll
      for (int c = 0; c < SPW; ++c) {
        prow[c] = pr[c];
        drow[c] = dr[c];
      }
      const bool zero = kb == 0 || !(fabs(prow[jj]) > T(0));
      singular |= zero;
      const int piv = zero ? r : 2047 - (int)(kb & 2047u);
      pivs[jj] = piv;
      if (piv != r) {
        if (has0 && r0 == piv) {
#pragma unroll
          for (int c = 0; c < SPW; ++c) x0[c] = drow[c];
        } else if (has0 && r0 == r) {
#pragma unroll
          for (int c = 0; c < SPW; ++c) x0[c] = prow[c];
        }
        if (piv >= r1 && (piv - r1) % NT == 0) {   // this thread's LDS row
#pragma unroll
          for (int c = 0; c < SPW; ++c) s.blk[(size_t)piv * BS + cs + c] = drow[c];
        }
      }
      if (!zero) {
        const T inv = rcp_newton(prow[jj]);
        if (has0 && r0 > r) {
          const T l0 = x0[jj] * inv;
          x0[jj] = l0;
#pragma unroll
          for (int c = jj + 1; c < SPW; ++c) x0[c] -= l0 * prow[c];
        }
        for (int rr = r1; rr < np; rr += NT) {
          T *y1 = s.blk + (size_t)rr * BS;
          const T l1 = y1[col] * inv;
          y1[col] = l1;
#pragma unroll
          for (int c = jj + 1; c < SPW; ++c) y1[cs + c] -= l1 * prow[c];
        }
      }
    }
    // the sub-panel's interchanges on the block columns outside it and on perm:
    // position x receives the row of position t_0(t_1(...t_7(x))) (t_jj the
    // transposition of rows j0+cs+jj and pivs[jj]); all reads before the writes
    {
      constexpr int NOUT = W - SPW;
      const int m = tid / (NOUT + 1), cc = tid % (NOUT + 1);
      int x = -1, y = -1, c = 0;
      T val = T(0);
      int pval = 0;
      if (m < 2 * SPW) {
        x = j0 + cs + m;
#pragma unroll
        for (int q = 0; q < SPW; ++q)
          if (m == SPW + q) x = pivs[q];
        y = x;
#pragma unroll
        for (int q = SPW - 1; q >= 0; --q) {
          const int rq = j0 + cs + q;
          y = (y == rq) ? pivs[q] : (y == pivs[q] ? rq : y);
        }
        c = cc < cs ? cc : cc + SPW;
        if (y != x) {
          if (cc < NOUT) val = s.blk[(size_t)y * BS + c];
          else pval = s.perm[y];
        }
      }
      __syncthreads();
      if (y != x) {
        if (cc < NOUT) s.blk[(size_t)x * BS + c] = val;
        else s.perm[x] = pval;
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
        T u[SPW];
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
      // rank-8 update of the rows below, 4 columns at a time
      for (int i = rp + SPW + tid; i < np; i += NT) {
        T l[SPW];
#pragma unroll
        for (int k = 0; k < SPW; ++k) l[k] = s.blk[i * BS + cs + k];
        for (int c = cs + SPW; c < W; c += 4) {
          T acc[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = s.blk[i * BS + c + q];
#pragma unroll
          for (int k = 0; k < SPW; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] -= l[k] * s.blk[(rp + k) * BS + c + q];
#pragma unroll
          for (int q = 0; q < 4; ++q) s.blk[i * BS + c + q] = acc[q];
        }
      }
      __syncthreads();
    }
  }
  return singular;
}

// Positions x >= j0 whose row changed in the panel just factored, with the
// position y the row came from (perm after the panel vs. invb, the inverse of perm
// before it); at most 2W of them.
template <typename T>
__device__ inline void moved_rows(const Lds<T> &s, int j0, int np) {
  for (int x = j0 + cur_tid(); x < np; x += NT) {
    const int y = s.invb[s.perm[x]];
    if (y != x) {
      const int k = atomicAdd(s.mvn, 1);
      s.mvx[k] = x;
      s.mvy[k] = y;
    }
  }
}


// The row movement of one block's pivots on the stored factor columns 0..j0-1:
// col[mvx[i]] <- col[mvy[i]] for the m (<= 64) moved positions.  Each wave moves whole columns,
// lane i the position i: the lane's read precedes its write, and the reads of a column are
// the same wave's, so no barrier is needed between them.  Four columns per wave in flight.
template <int NWV, typename T>
__device__ inline void move_rows_waves(const int *mvx, const int *mvy, int m, T *Fm, int ld, int j0) {
  if (m == 0) return;
  const int tid = cur_tid(), lane = tid & 63, w = tid >> 6;
  const bool act = lane < m;
  const int y = act ? mvy[lane] : 0, x = act ? mvx[lane] : 0;
  constexpr int CU = 4;
  for (int c0 = w * CU; c0 < j0; c0 += NWV * CU) {
    T v[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u)
      if (act && c0 + u < j0) v[u] = Fm[(size_t)(c0 + u) * ld + y];
#pragma unroll
    for (int u = 0; u < CU; ++u)
      if (act && c0 + u < j0) Fm[(size_t)(c0 + u) * ld + x] = v[u];
  }
}

// LDS carve-up of k_condense_t (byte offsets, 16-byte aligned parts).
struct LdsLayout {
  size_t blk, crow, perm, redi, dsc, invb, mv, total;
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline LdsLayout lds_layout(int np, size_t tsize, bool lp, int W) {
  LdsLayout L;
  size_t o = 0;
  L.blk = o;
  o = al16(o + (size_t)np * (W + 1) * tsize);
  L.crow = o;
  o = al16(o + 2 * (NW + 1) * 8 * tsize);
  L.perm = o;
  o = al16(o + (size_t)np * sizeof(int));
  L.redi = o;
  o = al16(o + 2 * NW * sizeof(int));
  L.dsc = o;
  o = al16(o + (lp ? (size_t)np * sizeof(double) : 0));
  L.invb = o;
  o = al16(o + (size_t)np * sizeof(int));
  L.mv = o;
  o = al16(o + (4 * WMAX + 1) * sizeof(int));
  L.total = o;
  return L;
}

// Per-element record of the low-precision factorization (floats):
//   F [np][np] factors in pivot-position order | Inv [np/W][2][W][W] (space for
//   W = 32) | perm [np] (int) | dsc [np] (symmetric scaling, powers of two)
__host__ __device__ inline size_t rec_perm_off(int np) { return (size_t)np * np + 2 * (size_t)np * WMAX; }
__host__ __device__ inline size_t lp_rec_floats(int np) { return rec_perm_off(np) + 2 * (size_t)np; }

// LDS of the condensation kernels, carved as lds_layout describes.
template <typename T, int LP, int W>
__device__ __forceinline__ Lds<T> carve_lds(int np) {
  extern __shared__ double smem[];
  char *sm = reinterpret_cast<char *>(smem);
  const LdsLayout Lo = lds_layout(np, sizeof(T), LP, W);
  Lds<T> s;
  s.blk = reinterpret_cast<T *>(sm + Lo.blk);
  s.crow = reinterpret_cast<T *>(sm + Lo.crow);
  s.perm = reinterpret_cast<int *>(sm + Lo.perm);
  s.redi = reinterpret_cast<int *>(sm + Lo.redi);
  s.dsc = LP ? reinterpret_cast<double *>(sm + Lo.dsc) : nullptr;
  s.invb = reinterpret_cast<int *>(sm + Lo.invb);
  s.mvx = reinterpret_cast<int *>(sm + Lo.mv);
  s.mvy = s.mvx + 2 * WMAX;
  s.mvn = s.mvy + 2 * WMAX;
  return s;
}

// Factor storage of element el (chunk slot) / e (global index): FP64 factors
// overwrite the A scratch, FP32 factors go to the record.
template <typename T, int LP>
struct FactorPtrs {
  T *F;     // [np][np] factors in pivot-position order
  T *Inv;   // [np/W][2][W][W] inverses of the diagonal blocks
  float *rec;
};

template <typename T, int LP>
__device__ __forceinline__ FactorPtrs<T, LP> factor_ptrs(const DevPlan &P, int e, int el, T *inv, float *fac) {
  const int np = P.n_pad;
  FactorPtrs<T, LP> f;
  if constexpr (LP) {
    f.rec = fac + (size_t)e * lp_rec_floats(np);
    f.F = f.rec;
    f.Inv = f.rec + (size_t)np * np;
  } else {
    f.rec = nullptr;
    f.F = P.A + (size_t)el * np * np;
    f.Inv = inv + (size_t)el * 2 * np * WMAX;
  }
  return f;
}

// Symmetric power-of-two scaling of the low-precision path from the diagonal of A.
__device__ inline double diag_scale(const DevPlan &P, const double *A64, const double *mg, int i) {
  const double a = fabs(a_entry(P, A64, mg, i, i));
  return (a > 0.0 && a < 1e300) ? exp2(-rint(0.5 * log2(a))) : 1.0;
}

// Update steps of the left-looking LU: step i applies factor block i to the rows below it.
struct StepSpec {
  int W, np;
  __device__ Step operator()(int i) const { return Step{i * 2 * W * W, i * W, i * W + W, np}; }
};

// Factor tiles a wave requests ahead per update step: five where the kernel runs at two
// waves per SIMD (FP64, 32 columns; the register file has room), two or three in the kernels
// whose registers are capped for four waves per SIMD.
template <typename T, int W>
__host__ __device__ constexpr int lu_prefetch_tiles() {
  return (sizeof(T) == 8 && W == 32) ? 5 : (sizeof(T) == 4 ? 3 : 2);
}

// LU of element el, left-looking over W-column blocks; leaves perm (and the
// scaling) in LDS and stores the permutation (P.ipiv, or the record).
// Returns whether a zero pivot occurred.
template <typename T, int LP, int W>
__device__ __forceinline__ bool lu_part(const DevPlan &P, int el, const Lds<T> &s, const FactorPtrs<T, LP> &f) {
  const int np = P.n_pad;
  const double *A64 = P.A + (size_t)el * np * np;
  const double *mg = P.mg ? P.mg + (size_t)el * (P.dim + 1) * P.Np * P.Np : nullptr;
  T *Fm = f.F;
  T *Ie = f.Inv;
  const int tid = cur_tid();
  const int nJ = np / W;
  for (int i = tid; i < np; i += NT) {
    s.perm[i] = i;
    if constexpr (LP) s.dsc[i] = diag_scale(P, A64, mg, i);
  }
  __syncthreads();
  bool singular = false;
  for (int J = 0; J < nJ; ++J) {
    const int j0 = J * W;
    if (mg) load_block_formed<T, LP, W>(s, P, A64, mg, j0);
    else if constexpr (LP) load_block_scaled<T, W>(s, A64, np, j0, np, true);
    else load_block<T, W>(s, A64, np, j0, np);
    __syncthreads();
    if (J > 0)
      run_steps<T, W, StepSpec, NT, lu_prefetch_tiles<T, W>(), LP == 2>(s, Ie, Fm, np, J, StepSpec{W, np});
    if (J > 0) {
      for (int x = j0 + tid; x < np; x += NT) s.invb[s.perm[x]] = x;
      if (tid == 0) *s.mvn = 0;
    }
    singular |= panel_factor<T, W>(s, j0, np);
    __syncthreads();
    if (J > 0) {
      moved_rows<T>(s, j0, np);
      __syncthreads();
    }
    invert_diag<T, W>(s, j0, Ie + (size_t)J * 2 * W * W, Ie + (size_t)J * 2 * W * W + W * W);
    store_block<T, W>(s, Fm, np, j0, np);
    if (J > 0) move_rows_waves<NW>(s.mvx, s.mvy, *s.mvn, Fm, np, j0);
    __syncthreads();
  }
  if constexpr (LP) {
    int *rp = reinterpret_cast<int *>(f.rec + rec_perm_off(np));
    float *rd = reinterpret_cast<float *>(rp + np);
    for (int i = tid; i < np; i += NT) {
      rp[i] = s.perm[i];
      rd[i] = (float)s.dsc[i];
    }
  } else {
    int *ip = P.ipiv + (size_t)el * np;
    for (int i = tid; i < np; i += NT) ip[i] = s.perm[i];
  }
  return singular;
}

// Right-hand-side block c0..c0+W-1 of [B | R_loc] for element e (slot el), with
// perm (and the scaling) in LDS: permutation gather, forward and backward
// sweeps against the stored factors, outputs Y, z, then the Schur product
// C * Y_block straight from LDS into S and g.
template <typename T, int LP, int W, int NTT = NT>
__device__ __forceinline__ void rhs_block(const DevPlan &P, int e, int el, int c0, const Lds<T> &s,
                                          const FactorPtrs<T, LP> &f, T *S, double *g, T *Y, double *z) {
  typedef Mfma<T> MF;
  constexpr int BS = W + 1, TW = W / 16;
  const int np = P.n_pad, kp = P.k_pad, kx = P.kx, n = P.n, k = P.k;
  const double *X = P.X + (size_t)el * kx * np;
  const double *C = P.C + (size_t)el * np * kp;
  const double *Dm = P.D + (size_t)el * kp * kp;
  const double *Rt = P.Rt + (size_t)el * kp;
  const int tid = tid_of<NTT>(), lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nJ = np / W;
  T *Se = S + (size_t)e * k * k;
  double *ge = g + (size_t)e * k;
  T *Ye = Y + (size_t)e * n * k;
  const int ntr = kp / 16;
  if constexpr (LP) load_block_scaled<T, W, NTT>(s, X, np, c0, np, false);
  else load_block<T, W, NTT>(s, X, np, c0, np);
  __syncthreads();
  // forward (unit lower) then backward (upper) sweep as one pipelined sequence
  const auto rhs_spec = [&](int i) {
    if (i < nJ) return Step{i * 2 * W * W, i * W, i * W + W, np};
    const int Pb = 2 * nJ - 1 - i;
    return Step{Pb * 2 * W * W + W * W, Pb * W, 0, Pb * W};
  };
  run_steps<T, W, decltype(rhs_spec), NTT, (NTT >= 1024 ? 1 : lu_prefetch_tiles<T, W>()), LP == 2>(s, f.Inv, f.F, np,
                                                                                               2 * nJ, rhs_spec);

  if constexpr (LP) {
    // undo the column scaling: Y = D Y_hat, z = D z_hat
    for (int t = tid; t < np * W; t += NTT) {
      const int c = t / np, i = t - c * np;
      s.blk[i * BS + c] = (T)((double)s.blk[i * BS + c] * s.dsc[i]);
    }
    __syncthreads();
  }
  // outputs Y, z (compact)
  for (int t = tid; t < n * W; t += NTT) {
    const int c = t / n, i = t - c * n;
    const int col = c0 + c;
    if (col < k) Ye[(size_t)col * n + i] = s.blk[i * BS + c];
    else if (col == kp) z[(size_t)e * n + i] = (double)s.blk[i * BS + c];
  }
  // T = C * block (k_pad x W): S = D - T, g = -R_tr + T
  for (int t = wave; t < ntr; t += NTT / 64) {
    const int r0 = t * 16;
    typename MF::acc acc[TW];
#pragma unroll
    for (int q = 0; q < TW; ++q) acc[q] = typename MF::acc{0, 0, 0, 0};
    const double *Cr = C + (size_t)lk * kp + r0 + li;
    T a[8], an[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) a[kk] = (T)Cr[(size_t)(4 * kk) * kp];
    for (int kb = 0; kb < np; kb += 32) {
      if (kb + 32 < np) {
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) an[kk] = (T)Cr[(size_t)(kb + 32 + 4 * kk) * kp];
      }
#pragma unroll
      for (int q = 0; q < TW; ++q)
        acc[q] = mma_panel<T, LP == 2, 8>(a, [&](int kk) { return s.blk[(kb + 4 * kk + lk) * BS + q * 16 + li]; },
                                          acc[q]);
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) a[kk] = an[kk];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + MF::row(lk, r);
      if (row >= k) continue;
#pragma unroll
      for (int q = 0; q < TW; ++q) {
        const int col = c0 + q * 16 + li;
        if (col < k) Se[(size_t)col * k + row] = (T)(Dm[(size_t)col * kp + row] - (double)acc[q][r]);
        else if (col == kp) ge[row] = -Rt[row] + (double)acc[q][r];
      }
    }
  }
  __syncthreads();
}

// T = double, LP = false: FP64 condensation, factors overwrite the A scratch.
// T = float,  LP = true : scaled FP32 condensation, factors to the record `fac`.
// One workgroup per element (the LU, then every right-hand-side block).
template <typename T, int LP, int W>
__device__ __forceinline__ void condense_body(const DevPlan &P, int e0, int el, int32_t *status, T *S, double *g,
                                              T *Y, double *z, T *inv, float *fac) {
  const int e = e0 + el;
  const Lds<T> s = carve_lds<T, LP, W>(P.n_pad);
  const FactorPtrs<T, LP> f = factor_ptrs<T, LP>(P, e, el, inv, fac);
  const bool singular = lu_part<T, LP, W>(P, el, s, f);
  for (int c0 = 0; c0 < P.kx; c0 += W) rhs_block<T, LP, W>(P, e, el, c0, s, f, S, g, Y, z);
  if (singular && cur_tid() == 0 && status[el] == HDG_OK) status[el] = HDG_ESINGULAR;
}

// Split condensation: the LU of one element per workgroup, then one workgroup
// per (element, right-hand-side block).  The nRB workgroups of an element read
// the same factors and C, so they are placed on one XCD (workgroups are handed
// to the 8 XCDs round-robin by index: element slot el runs as indices
// (el / 8 * nRB + j) * 8 + el % 8) and share its L2.
template <typename T, int LP, int W>
__device__ __forceinline__ void lu_body(const DevPlan &P, int e0, int el, int32_t *status, T *inv, float *fac) {
  const int e = e0 + el;
  const Lds<T> s = carve_lds<T, LP, W>(P.n_pad);
  const FactorPtrs<T, LP> f = factor_ptrs<T, LP>(P, e, el, inv, fac);
  const bool singular = lu_part<T, LP, W>(P, el, s, f);
  if (singular && cur_tid() == 0 && status[el] == HDG_OK) status[el] = HDG_ESINGULAR;
}

constexpr int NXCD = 8;

template <typename T, int LP, int W, int NTT = NT>
__device__ __forceinline__ void rhs_body(const DevPlan &P, int e0, int ec, T *S, double *g, T *Y, double *z, T *inv,
                                         float *fac) {
  const int nrb = P.kx / W;
  const int b = blockIdx.x, xcd = b % NXCD, slot = b / NXCD;
  const int el = (slot / nrb) * NXCD + xcd, j = slot % nrb;
  if (el >= ec) return;   // whole workgroup
  const int e = e0 + el;
  const int np = P.n_pad;
  const Lds<T> s = carve_lds<T, LP, W>(np);
  const FactorPtrs<T, LP> f = factor_ptrs<T, LP>(P, e, el, inv, fac);
  const int *perm = LP ? reinterpret_cast<const int *>(f.rec + rec_perm_off(np)) : P.ipiv + (size_t)el * np;
  const double *A64 = P.A + (size_t)el * np * np;
  const double *mg = P.mg ? P.mg + (size_t)el * (P.dim + 1) * P.Np * P.Np : nullptr;
  for (int i = tid_of<NTT>(); i < np; i += NTT) {
    s.perm[i] = perm[i];
    if constexpr (LP) s.dsc[i] = diag_scale(P, A64, mg, i);
  }
  __syncthreads();
  rhs_block<T, LP, W, NTT>(P, e, el, j * W, s, f, S, g, Y, z);
}

__global__ __launch_bounds__(NT) void k_lu_f64_w32(DevPlan P, int e0, int32_t *status, double *inv) {
  lu_body<double, false, 32>(P, e0, blockIdx.x, status, inv, nullptr);
}

// right-hand sides: one workgroup per CU (LDS) with few registers, so 16 waves
constexpr int NT_RHS = 1024;

__global__ __launch_bounds__(NT_RHS) void k_rhs_f64_w32(DevPlan P, int e0, int ec, double *S, double *g, double *Y,
                                                        double *z, double *inv) {
  rhs_body<double, false, 32, NT_RHS>(P, e0, ec, S, g, Y, z, inv, nullptr);
}

// Small blocks (two or more working blocks fit in a CU's LDS): 4 waves per workgroup, so that
// the workgroups of several (element, block) items share a CU instead of one item's 16 waves
// outnumbering its row tiles.  Same arithmetic in the same order as k_rhs_f64_w32.
constexpr int NT_RHS_SMALL = 256;
__global__ __launch_bounds__(NT_RHS_SMALL) void k_rhs_f64_w32_small(DevPlan P, int e0, int ec, double *S, double *g,
                                                                    double *Y, double *z, double *inv) {
  rhs_body<double, false, 32, NT_RHS_SMALL>(P, e0, ec, S, g, Y, z, inv, nullptr);
}

// 16-column blocks (a 32-column block of n_pad > 704 rows does not fit in LDS): the LU, then one
// workgroup per (element, 16-column block), the blocks of an element on one XCD
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_lu_f64_w16(DevPlan P, int e0,
                                                                                            int32_t *status,
                                                                                            double *inv) {
  lu_body<double, false, 16>(P, e0, blockIdx.x, status, inv, nullptr);
}

__global__ __launch_bounds__(NT_RHS) void k_rhs_f64_w16(DevPlan P, int e0, int ec, double *S, double *g, double *Y,
                                                        double *z, double *inv) {
  rhs_body<double, false, 16, NT_RHS>(P, e0, ec, S, g, Y, z, inv, nullptr);
}

// LPM: 1 FP32 operands, 2 BF16 operands (FP32 data and accumulation either way)
template <int W, int LPM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_lu_f32(DevPlan P, int e0,
                                                                                        int32_t *status,
                                                                                        float *fac) {
  lu_body<float, LPM, W>(P, e0, blockIdx.x, status, nullptr, fac);
}

template <int W, int LPM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_rhs_f32(DevPlan P, int e0, int ec,
                                                                                         float *S, double *g,
                                                                                         float *Y, double *z,
                                                                                         float *fac) {
  rhs_body<float, LPM, W>(P, e0, ec, S, g, Y, z, nullptr, fac);
}

__global__ __launch_bounds__(NT) void k_condense_f64_w32(DevPlan P, int e0, int32_t *status, double *S, double *g,
                                                         double *Y, double *z, double *inv) {
  condense_body<double, false, 32>(P, e0, blockIdx.x, status, S, g, Y, z, inv, nullptr);
}

// 16-column blocks take half the LDS: two workgroups per CU with capped registers.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_condense_f64_w16(
    DevPlan P, int e0, int32_t *status, double *S, double *g, double *Y, double *z, double *inv) {
  condense_body<double, false, 16>(P, e0, blockIdx.x, status, S, g, Y, z, inv, nullptr);
}

// Two workgroups per CU where the FP32 working block fits twice in LDS:
// registers are capped so that 16 waves fit.
template <int W, int LPM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_condense_f32(
    DevPlan P, int e0, int32_t *status, float *S, double *g, float *Y, double *z, float *fac) {
  condense_body<float, LPM, W>(P, e0, blockIdx.x, status, S, g, Y, z, nullptr, fac);
}

// Condensation of a batch of plans (element types / orders with uneven n, k), in two launches
// as the per-plan path, over two item lists:
// * LU items (plan << 24 | element), longest processing time first: the LU of the element.
// * Right-hand-side items (plan << 24 | element, block j): one 32- (or 16-) column block of
//   [B | R_loc] against the element's factors.  Eight lists, one per XCD: the items of an
//   element sit together in the list of one XCD, and run on workgroups of that XCD
//   (workgroups are handed to the XCDs round-robin by index), so the workgroups working on an
//   element share its factors and C in that XCD's L2.
// Default: one workgroup per item (workgroup b of the right-hand-side launch takes item b / 8
// of XCD b % 8's list); the hardware dispatches workgroups in index order as slots free up,
// which is the longest-processing-time list schedule.  Persistent (a fixed grid of workgroups
// taking items from atomic counters until the lists are empty) is kept as an option.
struct BatchItemArgs {
  double *S, *g, *Y, *z;
  int32_t *status;
};

__device__ __forceinline__ void lu_item(const DevPlan *__restrict__ plans, const BatchItemArgs *__restrict__ io,
                                        int code) {
  const int pi = code >> 24, el = code & 0xFFFFFF;
  const DevPlan &P = plans[pi];
  if (P.cw == 32) lu_body<double, false, 32>(P, 0, el, io[pi].status, P.inv, nullptr);
  else lu_body<double, false, 16>(P, 0, el, io[pi].status, P.inv, nullptr);
}

__global__ __launch_bounds__(NT) void k_lu_batch(const DevPlan *__restrict__ plans,
                                                 const BatchItemArgs *__restrict__ io,
                                                 const int *__restrict__ queue, int n_items) {
  if ((int)blockIdx.x >= n_items) return;   // whole workgroup
  lu_item(plans, io, __builtin_amdgcn_readfirstlane(queue[blockIdx.x]));
}

__global__ __launch_bounds__(NT) void k_lu_batch_persistent(const DevPlan *__restrict__ plans,
                                                            const BatchItemArgs *__restrict__ io,
                                                            const int *__restrict__ queue, int n_items,
                                                            int *counter) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    // the item is the same for the whole workgroup: keep it (and the plan fields read through
    // it) in scalar registers
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n_items) break;
    lu_item(plans, io, __builtin_amdgcn_readfirstlane(queue[it]));
    __syncthreads();
  }
}

__device__ __forceinline__ void rhs_item(const DevPlan *__restrict__ plans, const BatchItemArgs *__restrict__ io,
                                         int code, int j) {
  const int pi = code >> 24, el = code & 0xFFFFFF;
  const DevPlan &P = plans[pi];
  const int np = P.n_pad;
  const int *perm = P.ipiv + (size_t)el * np;
  const FactorPtrs<double, false> f = factor_ptrs<double, false>(P, el, el, P.inv, nullptr);
  const BatchItemArgs &a = io[pi];
  if (P.cw == 32) {
    const Lds<double> s = carve_lds<double, false, 32>(np);
    for (int i = tid_of<NT_RHS>(); i < np; i += NT_RHS) s.perm[i] = perm[i];
    __syncthreads();
    rhs_block<double, false, 32, NT_RHS>(P, el, el, j * 32, s, f, a.S, a.g, a.Y, a.z);
  } else {
    const Lds<double> s = carve_lds<double, false, 16>(np);
    for (int i = tid_of<NT_RHS>(); i < np; i += NT_RHS) s.perm[i] = perm[i];
    __syncthreads();
    rhs_block<double, false, 16, NT_RHS>(P, el, el, j * 16, s, f, a.S, a.g, a.Y, a.z);
  }
}

__global__ __launch_bounds__(NT_RHS) void k_rhs_batch(const DevPlan *__restrict__ plans,
                                                      const BatchItemArgs *__restrict__ io,
                                                      const int2 *__restrict__ queue, const int *__restrict__ xoff) {
  const int x = blockIdx.x % NXCD, it = blockIdx.x / NXCD;
  if (it >= xoff[x + 1] - xoff[x]) return;   // whole workgroup
  const int2 c = queue[xoff[x] + it];
  rhs_item(plans, io, __builtin_amdgcn_readfirstlane(c.x), __builtin_amdgcn_readfirstlane(c.y));
}

__global__ __launch_bounds__(NT_RHS) void k_rhs_batch_persistent(const DevPlan *__restrict__ plans,
                                                                 const BatchItemArgs *__restrict__ io,
                                                                 const int2 *__restrict__ queue,
                                                                 const int *__restrict__ xoff, int *counters) {
  __shared__ int s_item;
  const int x = blockIdx.x % NXCD;
  const int n_items = xoff[x + 1] - xoff[x];
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&counters[x], 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n_items) break;
    const int2 c = queue[xoff[x] + it];
    rhs_item(plans, io, __builtin_amdgcn_readfirstlane(c.x), __builtin_amdgcn_readfirstlane(c.y));
    __syncthreads();
  }
}

// x = A_lp^-1 r per element from the low-precision record: y = P D r, forward
// substitution (unit L) and backward substitution (U) over W-column blocks
// with the stored diagonal-block inverses, x = D y.  Vectors and arithmetic in
// FP64, factors read as FP32 (stored in pivot-position order, so every factor
// column is read contiguously).  One workgroup per element.
constexpr int SB = 256;

__global__ __launch_bounds__(SB) void k_lp_solve(int n, int np, int W, const float *__restrict__ fac,
                                                 const double *__restrict__ r, double *x) {
  extern __shared__ double sm2[];
  const int e = blockIdx.x, tid = threadIdx.x;
  const int nJ = np / W;
  double *y = sm2;                                   // [np] by pivot position
  double *t32 = y + np;                              // [W]
  const float *rec = fac + (size_t)e * lp_rec_floats(np);
  const float *F = rec;
  const float *Inv = rec + (size_t)np * np;
  const int *perm = reinterpret_cast<const int *>(rec + rec_perm_off(np));
  const float *dsc = reinterpret_cast<const float *>(perm + np);
  const double *re = r + (size_t)e * n;
  for (int i = tid; i < np; i += SB) {
    const int o = perm[i];
    y[i] = o < n ? (double)dsc[o] * re[o] : 0.0;
  }
  __syncthreads();
  // forward: unit lower
  for (int J = 0; J < nJ; ++J) {
    const int j0 = J * W;
    const float *Li = Inv + (size_t)J * 2 * W * W;
    if (tid < W) {
      double acc = 0.0;
      for (int c = 0; c < W; ++c) acc += (double)Li[c * W + tid] * y[j0 + c];
      t32[tid] = acc;
    }
    __syncthreads();
    if (tid < W) y[j0 + tid] = t32[tid];
    __syncthreads();
    for (int i = j0 + W + tid; i < np; i += SB) {
      double acc = 0.0;
#pragma unroll 8
      for (int c = 0; c < W; ++c) acc += (double)F[(size_t)(j0 + c) * np + i] * y[j0 + c];
      y[i] -= acc;
    }
    __syncthreads();
  }
  // backward: upper
  for (int J = nJ - 1; J >= 0; --J) {
    const int j0 = J * W;
    const float *Ui = Inv + (size_t)J * 2 * W * W + W * W;
    if (tid < W) {
      double acc = 0.0;
      for (int c = 0; c < W; ++c) acc += (double)Ui[c * W + tid] * y[j0 + c];
      t32[tid] = acc;
    }
    __syncthreads();
    if (tid < W) y[j0 + tid] = t32[tid];
    __syncthreads();
    for (int i = tid; i < j0; i += SB) {
      double acc = 0.0;
#pragma unroll 8
      for (int c = 0; c < W; ++c) acc += (double)F[(size_t)(j0 + c) * np + i] * y[j0 + c];
      y[i] -= acc;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += SB) x[(size_t)e * n + i] = (double)dsc[i] * y[i];
}


// ---------------------------------------------------------------------------
// LU with the working block in registers (two elements per CU).
//
// The left-looking LU above keeps its 32-column working block in LDS
// (n_pad x 33 doubles, 143 KB at n_pad = 544), which leaves room for one
// workgroup per CU: the latency of the pivot searches and barriers then has
// nothing to hide behind.  Here the 32 columns live in the registers of NWV
// waves as matrix-core accumulators: row tile t (16 rows) belongs to wave
// t % NWV, whose lane (li, lk) holds rows lk + 4r (r = 0..3) of columns li and
// 16 + li.  LDS holds only staging (an 8-column sub-panel, the rows that feed a
// step, the permutations), about 66 KB at n_pad = 544, so with four waves two
// elements share a CU and one's panel factorization overlaps the other's
// updates.  The factors, their ordering and the diagonal-block inverses are
// stored exactly as the LDS kernel stores them, so the right-hand-side launch
// is the same.
//
// * Update of block J by the stored factors, in steps of 16 columns: the wave
//   that owns tile s applies the inverse of the unit-lower 16 x 16 diagonal
//   block to it on the matrix cores, its own accumulators serving as the B
//   operand (the accumulator layout of a 16-row tile is the B layout of its
//   four 4-row k-steps), and writes the result to LDS; after one barrier every
//   wave subtracts F(tile rows, step columns) times those rows from its tiles
//   below.  The owner of the next step's tile updates that tile first and
//   applies the next inverse before its other tiles, so one barrier per step
//   suffices (the staging is double-buffered).
// * Panel factorization of block J in four 8-column sub-panels with partial
//   pivoting: the sub-panel's rows are copied to LDS and each thread keeps up
//   to MR of them in registers; per column one wave-wide maximum of a 32-bit
//   key (the magnitude's exponent and leading 11 mantissa bits, then the lowest
//   row; pivot_key32) and one barrier.
//   Rows are not moved in the registers: sig[p] records the position that the
//   row held in physical slot p has reached, and every access goes through it.
//   After a sub-panel its 8 pivot rows are solved against the remaining
//   columns (unit-lower 8 x 8, per wave) and the rows below receive the rank-8
//   update on the matrix cores.
// ---------------------------------------------------------------------------

typedef unsigned long long u64;

// 32-bit pivot key of relative row i (< 1024): the magnitude's exponent and leading 11
// mantissa bits, then the lower row (the choice is that of exact partial pivoting up to a
// relative 2^-11, which keeps the multipliers below 1 + 2^-10 in magnitude); 0 marks "no
// candidate"
__device__ inline unsigned pivot_key32(double x, int i) {
  const u64 b = __builtin_bit_cast(u64, fabs(x));
  return ((unsigned)(b >> 41) << 10) | (unsigned)(1023 - i);
}

constexpr int RG_SS = 9;     // LDS row stride of the 8-column sub-panel
constexpr int RG_ST = 34;    // LDS row stride of the 16 x 32 / 8 x 32 staging

struct RegLayout {
  size_t sub, stage, ust, wst, crow, redk, perm, sig, invb, mv, total;
};

__host__ __device__ inline RegLayout reg_layout(int np, int nwv) {
  RegLayout L;
  size_t o = 0;
  const size_t subd = (size_t)np * RG_SS > 32 * 33 ? (size_t)np * RG_SS : 32 * 33;
  L.sub = o;   o = al16(o + subd * 8);
  L.stage = o; o = al16(o + 2 * 16 * RG_ST * 8);
  L.ust = o;   o = al16(o + 8 * RG_ST * 8);
  L.wst = o;   o = al16(o + (size_t)nwv * 8 * RG_ST * 8);
  L.crow = o;  o = al16(o + 2 * (size_t)(nwv + 1) * 8 * 8);
  L.redk = o;  o = al16(o + (2 * (size_t)nwv + 8) * 4);
  L.perm = o;  o = al16(o + (size_t)np * 4);
  L.sig = o;   o = al16(o + (size_t)np * 4);
  L.invb = o;  o = al16(o + (size_t)np * 4);
  L.mv = o;    o = al16(o + (4 * WMAX + 1) * 4);
  L.total = o;
  return L;
}

template <typename F, int... I>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

template <int NWV, int TPW>
__device__ __forceinline__ void lu_reg_body(const DevPlan &P, int el, int32_t *status, double *inv) {
  constexpr int NTR = 64 * NWV;
  constexpr int MR = (TPW + 3) / 4;   // sub-panel rows per thread: ceil(16 TPW NWV / NTR)
  extern __shared__ double smem[];
  char *sm = reinterpret_cast<char *>(smem);
  const int np = P.n_pad, NTILE = np / 16, nJ = np / 32;
  const int n = P.n, Np = P.Np, Dm = P.dim, nv = P.m * Np, DN = Dm * Np;
  const RegLayout Lo = reg_layout(np, NWV);
  double *sub = reinterpret_cast<double *>(sm + Lo.sub);
  double *stage = reinterpret_cast<double *>(sm + Lo.stage);
  double *ust = reinterpret_cast<double *>(sm + Lo.ust);
  double *crow = reinterpret_cast<double *>(sm + Lo.crow);
  unsigned *redk = reinterpret_cast<unsigned *>(sm + Lo.redk);
  int *pivl = reinterpret_cast<int *>(sm + Lo.redk) + 2 * NWV;
  int *perm = reinterpret_cast<int *>(sm + Lo.perm);
  int *sig = reinterpret_cast<int *>(sm + Lo.sig);
  int *invb = reinterpret_cast<int *>(sm + Lo.invb);
  int *mvx = reinterpret_cast<int *>(sm + Lo.mv);
  int *mvy = mvx + 2 * WMAX;
  int *mvn = mvy + 2 * WMAX;
  double *Fm = P.A + (size_t)el * np * np;   // factors overwrite A (columns of block J are read before)
  const double *mg = P.mg ? P.mg + (size_t)el * (P.dim + 1) * P.Np * P.Np : nullptr;
  double *Ie = inv + (size_t)el * 2 * np * WMAX;
  typedef Mfma<double> MF;

  for (int i = threadIdx.x; i < np; i += NTR) perm[i] = i;
  bool singular = false;
  d4 acc[TPW][2];
  __syncthreads();

  for (int J = 0; J < nJ; ++J) {
    const int j0 = J * 32;
    // Thread coordinates are redefined opaquely in every block: whatever is formed from them
    // (addresses, lane predicates) is recomputed inside the block loop instead of being hoisted
    // out of it and held in (spilled) registers.  The wave index is made uniform again.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    double *wst = reinterpret_cast<double *>(sm + Lo.wst) + (size_t)w * 8 * RG_ST;

  // operands of the update steps: F(tile t rows, step s columns), negated (uniform base,
  // 32-bit lane offset made opaque: otherwise the compiler hoists a 64-bit address per tile
  // and k-step out of the block loop and spills them), and the inverse of step s's 16 x 16
  // unit-lower diagonal block
  const auto load_f = [&](int s, int t, double (&f)[4]) {
    const double *base = Fm + (size_t)(16 * s) * np;
    unsigned o = lk * np + 16 * t + li;
    asm volatile("" : "+v"(o));
    sfor<4>([&](auto kk) { f[kk] = -base[o + 4u * kk * np]; });
  };
  const auto load_la = [&](int s, double (&la)[4]) {
    const int off = 16 * (s & 1);
    const double *Li = Ie + (size_t)(s >> 1) * 2 * WMAX * WMAX;
    sfor<4>([&](auto kk) { la[kk] = Li[(off + 4 * kk + lk) * WMAX + off + li]; });
  };
  // rows <- (16 x 16 inverse, operands la) x rows for the tile in at; result to the staging
  const auto inv_rows = [&](d4 (&at)[2], const double (&la)[4], double *stn) {
    d4 nw[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    sfor<2>([&](auto q) { sfor<4>([&](auto kk) { nw[q] = MF::op(la[kk], at[q][(int)kk], nw[q]); }); });
    sfor<2>([&](auto q) {
      at[q] = nw[q];
      sfor<4>([&](auto r) { stn[(lk + 4 * r) * RG_ST + 16 * q + li] = nw[q][(int)r]; });
    });
  };
  // the accumulator column half q (0 or 1, uniform) of slot (u, r), as selects of values (a
  // select of the two addresses would keep acc out of the registers)
  const auto acc_get = [&](auto u, auto r, int q) {
    const double v0 = acc[u][0][(int)r], v1 = acc[u][1][(int)r];
    return q ? v1 : v0;
  };
  const auto acc_set = [&](auto u, auto r, int q, double v) {
    const double v0 = acc[u][0][(int)r], v1 = acc[u][1][(int)r];
    acc[u][0][(int)r] = q ? v0 : v;
    acc[u][1][(int)r] = q ? v : v1;
  };

    for (int x = tid; x < np; x += NTR) {
      sig[x] = x;
      invb[perm[x]] = x;
    }
    if (tid == 0) *mvn = 0;
    __syncthreads();
    // gather block J through the permutation, 8 columns at a time through LDS: the stored
    // rows directly (all of A, or only its v rows when the q rows are formed from the compact
    // M and G_j), then the nonzeros of the formed q rows placed through the inverse permutation
    for (int h = 0; h < 4; ++h) {
      const int c0 = j0 + 8 * h;
      constexpr int GU = 4;   // entries per thread with their loads in flight together
      for (int x0 = tid; x0 < np * 8; x0 += GU * NTR) {
        double v[GU];
        sfor<GU>([&](auto g) {
          const int x = x0 + g * NTR;
          v[g] = 0.0;
          if (x < np * 8) {
            const int c = x / np, o = perm[x - c * np], col = c0 + c;
            if (!mg) v[g] = Fm[(size_t)col * np + o];
            else if (o < nv) v[g] = col < n ? Fm[(size_t)col * np + o] : 0.0;
            else v[g] = (o == col && o >= n) ? 1.0 : 0.0;
          }
        });
        sfor<GU>([&](auto g) {
          const int x = x0 + g * NTR;
          if (x < np * 8) {
            const int c = x / np;
            sub[(x - c * np) * RG_SS + c] = v[g];
          }
        });
      }
      if (mg) {
        __syncthreads();
        // v column (cc, b): G_j[a][b] in the q rows (cc, j, a); q column (cc, jj, b): M[a][b]
        // in the q rows (cc, jj, a)
        for (int x = tid; x < 8 * DN; x += NTR) {
          const int c = x / DN, r = x - c * DN, col = c0 + c;
          if (col >= n) continue;
          int o;
          double val;
          if (col < nv) {
            const int cc = col / Np, bb = col - cc * Np, j = r / Np, aa = r - j * Np;
            o = nv + (cc * Dm + j) * Np + aa;
            val = mg[(j * Np + aa) * Np + bb];
          } else {
            if (r >= Np) continue;
            const int qc = col - nv, cj = qc / Np, bb = qc - cj * Np;
            o = nv + cj * Np + r;
            val = mg[(Dm * Np + r) * Np + bb];
          }
          sub[invb[o] * RG_SS + c] = val;
        }
      }
      __syncthreads();
      const int qh = h >> 1, lo = 8 * (h & 1);
      if (li >= lo && li < lo + 8) {
        sfor<TPW>([&](auto u) {
          const int t = w + NWV * u;
          if (t < NTILE) sfor<4>([&](auto r) { acc_set(u, r, qh, sub[(16 * t + lk + 4 * r) * RG_SS + li - lo]); });
        });
      }
      __syncthreads();
    }

    // ---- update by the stored factors, 16 columns per step ----
    // Every register that carries an operand into a later step is loaded unconditionally
    // (inactive slots re-read an active tile's address, a cache hit): a conditional load into
    // a loop-carried register becomes a load into a temporary and a copy, and the copy waits
    // for the load at once.  Loads complete in issue order, so the inverse operands of a step
    // are requested before the operand ring.
    const int ns = 2 * J;
    if (ns > 0) {
      double fr[TPW][4], L0[4], L1[4];
      // operand ring: fr[u] holds F(tile of slot u, columns of the coming step)
      const auto ring = [&](int s2) {
        const int tmin = s2 + 1 < NTILE ? s2 + 1 : NTILE - 1;
        sfor<TPW>([&](auto u) {
          int t = w + NWV * u;
          t = t < tmin ? tmin : (t > NTILE - 1 ? NTILE - 1 : t);
          load_f(s2, t, fr[u]);
        });
      };
      if (w == 0) {
        // step 0: rows 0..15 (tile 0 of wave 0) <- inverse of the first diagonal block times them
        load_la(0, L0);
        inv_rows(acc[0], L0, stage);
      }
      load_la(ns > 1 ? 1 : 0, L1);
      ring(0);
      // step s: the owner of tile s + 1 applies the inverse of step s + 1 (operands Ln); the
      // inverse of step s + 2 is requested into Lq (free: its last use was in step s - 1)
      const auto step = [&](int s, double (&Ln)[4], double (&Lq)[4]) {
        lds_barrier();
        const double *stg = stage + (s & 1) * 16 * RG_ST;
        double b[4][2];
        sfor<4>([&](auto kk) { sfor<2>([&](auto q) { b[kk][q] = stg[(4 * kk + lk) * RG_ST + 16 * q + li]; }); });
        load_la(s + 2 < ns ? s + 2 : ns - 1, Lq);
        const bool own = s + 1 < ns && w == (s + 1) % NWV;
        const auto update = [&](auto u) {
          sfor<4>([&](auto kk) { sfor<2>([&](auto q) { acc[u][q] = MF::op(fr[u][kk], b[kk][q], acc[u][q]); }); });
        };
        if (own) {
          // tile s + 1: its last update, then the inverse of step s + 1; rows to the staging
          const int us = (s + 1) / NWV;
          double *stn = stage + ((s + 1) & 1) * 16 * RG_ST;
          sfor<TPW>([&](auto u) {
            if (u == us) {
              update(u);
              inv_rows(acc[u], Ln, stn);
            }
          });
        }
        // the wave's other tiles below the step
        sfor<TPW>([&](auto u) {
          const int t = w + NWV * u;
          if (t > s + (own ? 1 : 0) && t < NTILE) update(u);
        });
        ring(s + 1 < ns ? s + 1 : s);
      };
      for (int s = 0; s < ns; s += 2) {
        step(s, L1, L0);
        if (s + 1 < ns) step(s + 1, L0, L1);
      }
    }
    __syncthreads();

    // ---- panel factorization of block J: four 8-column sub-panels ----
    for (int sp = 0; sp < 4; ++sp) {
      const int cs = 8 * sp, qs = sp >> 1, lo = 8 * (sp & 1);
      const int P0 = j0 + cs, R = np - P0;
      const bool mine = li >= lo && li < lo + 8;
      // (a) the sub-panel's rows from position P0 on into LDS
      if (mine) {
        sfor<TPW>([&](auto u) {
          const int t = w + NWV * u;
          if (t < NTILE) {
            sfor<4>([&](auto r) {
              const int sg = sig[16 * t + lk + 4 * r];
              if (sg >= P0) sub[(sg - P0) * RG_SS + li - lo] = acc_get(u, r, qs);
            });
          }
        });
      }
      __syncthreads();
      // (b) partial pivoting over the 8 columns; thread rows i = tid + NTR m.  The columns
      // are kept rotated so that the current one is x[m][0] (one copy of the column code):
      // at column jj, x[m][c] holds column jj + c for c < 8 - jj and the finished column
      // jj + c - 8 after that; after 8 rotations the order is the original one.
      double x[MR][8];
      int sgl[MR];   // positions reached by the rows of this thread's physical slots
      sfor<MR>([&](auto m) {
        const int i = tid + NTR * m;
        sfor<8>([&](auto c) { x[m][c] = i < R ? sub[i * RG_SS + c] : 0.0; });
        sgl[m] = tid + NTR * m < np ? sig[tid + NTR * m] : -1;
      });
      for (int jj = 0; jj < 8; ++jj) {
        unsigned best = 0;
        int bm = -1;
        sfor<MR>([&](auto m) {
          const int i = tid + NTR * m;
          if (i < R && i >= jj) {
            const unsigned kx = pivot_key32(x[m][0], i);
            if (kx > best) {
              best = kx;
              bm = m;
            }
          }
        });
        const unsigned wb = wave_max_u32(best);
        const int bs = jj & 1;
        double *cr = crow + (size_t)bs * (NWV + 1) * 8;
        if (bm >= 0 && best == wb) {
          sfor<MR>([&](auto m) {
            if (m == bm) sfor<8>([&](auto c) { cr[w * 8 + c] = x[m][c]; });
          });
        }
        if (lane == 0) redk[bs * NWV + w] = wb;
        if (tid == jj) sfor<8>([&](auto c) { cr[NWV * 8 + c] = x[0][c]; });
        lds_barrier();
        unsigned kb = 0;
        int wv = 0;
        sfor<NWV>([&](auto v) {
          const unsigned kv = redk[bs * NWV + v];
          if (kv > kb) {
            kb = kv;
            wv = v;
          }
        });
        double prow[8];
        sfor<8>([&](auto c) { prow[c] = cr[wv * 8 + c]; });
        const bool zero = kb == 0 || !(fabs(prow[0]) > 0.0);
        singular |= zero;
        const int piv = zero ? jj : 1023 - (int)(kb & 1023u);
        if (tid == 0) pivl[jj] = piv;
        if (piv != jj) {
          sfor<MR>([&](auto m) {
            if (tid + NTR * m == piv) sfor<8>([&](auto c) { x[m][c] = cr[NWV * 8 + c]; });
          });
          if (tid == jj) sfor<8>([&](auto c) { x[0][c] = prow[c]; });
          const int a = P0 + jj, bp = P0 + piv;
          sfor<MR>([&](auto m) { sgl[m] = sgl[m] == a ? bp : (sgl[m] == bp ? a : sgl[m]); });
        }
        // reciprocal of the pivot: hardware estimate and two Newton steps
        double rinv = 0.0;
        if (!zero) {
          rinv = __builtin_amdgcn_rcp(prow[0]);
          rinv = fma(rinv, fma(-prow[0], rinv, 1.0), rinv);
          rinv = fma(rinv, fma(-prow[0], rinv, 1.0), rinv);
        }
        sfor<MR>([&](auto m) {
          const int i = tid + NTR * m;
          if (!zero && i < R && i > jj) {
            const double l = x[m][0] * rinv;
            x[m][0] = l;
            sfor<7>([&](auto cm) {
              constexpr int c = cm + 1;
              if (c < 8 - jj) x[m][c] -= l * prow[c];
            });
          }
          const double t0 = x[m][0];
          sfor<7>([&](auto c) { x[m][c] = x[m][c + 1]; });
          x[m][7] = t0;
        });
      }
      sfor<MR>([&](auto m) {
        const int i = tid + NTR * m;
        if (i < R) sfor<8>([&](auto c) { sub[i * RG_SS + c] = x[m][c]; });
        if (tid + NTR * m < np) sig[tid + NTR * m] = sgl[m];
      });
      if (tid == 0) {
        // the sub-panel's interchanges on the permutation, in order
        for (int jj = 0; jj < 8; ++jj) {
          const int a = P0 + jj, bp = P0 + pivl[jj];
          if (a != bp) {
            const int tmp = perm[a];
            perm[a] = perm[bp];
            perm[bp] = tmp;
          }
        }
      }
      __syncthreads();
      // (d) factored sub-panel back into the registers; the 8 pivot rows to the staging
      // (their columns from cs + 8 on; zero before, so that they leave those columns unchanged)
      sfor<TPW>([&](auto u) {
        const int t = w + NWV * u;
        if (t < NTILE) {
          sfor<4>([&](auto r) {
            const int sg = sig[16 * t + lk + 4 * r];
            if (mine && sg >= P0) acc_set(u, r, qs, sub[(sg - P0) * RG_SS + li - lo]);
            if (sg >= P0 && sg < P0 + 8) {
              sfor<2>([&](auto q) {
                const int c = 16 * q + li;
                ust[(sg - P0) * RG_ST + c] = c >= cs + 8 ? acc[u][q][(int)r] : 0.0;
              });
            }
          });
        }
      });
      __syncthreads();
      // (e) pivot rows against the unit-lower 8 x 8 block (every wave, lane = column), into
      // the wave's own staging
      if (lane < 32) {
        double uu[8];
        sfor<8>([&](auto i) { uu[i] = ust[i * RG_ST + lane]; });
        sfor<8>([&](auto i) {
          sfor<8>([&](auto k2) {
            if constexpr (k2 < i) uu[i] -= sub[i * RG_SS + k2] * uu[k2];
          });
        });
        sfor<8>([&](auto i) { wst[i * RG_ST + lane] = uu[i]; });
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // (f) holders of the pivot rows take the solved values; rank-8 update of the rows below
      double bw[2][2];
      sfor<2>([&](auto kk) { sfor<2>([&](auto q) { bw[kk][q] = wst[(4 * kk + lk) * RG_ST + 16 * q + li]; }); });
      sfor<TPW>([&](auto u) {
        const int t = w + NWV * u;
        if (t < NTILE) {
          sfor<4>([&](auto r) {
            const int sg = sig[16 * t + lk + 4 * r];
            if (sg >= P0 && sg < P0 + 8) {
              sfor<2>([&](auto q) {
                const int c = 16 * q + li;
                if (c >= cs + 8) acc[u][q][(int)r] = wst[(sg - P0) * RG_ST + c];
              });
            }
          });
          const int sa = sig[16 * t + li];
          sfor<2>([&](auto kk) {
            const double a = sa >= P0 + 8 ? -sub[(sa - P0) * RG_SS + 4 * kk + lk] : 0.0;
            sfor<2>([&](auto q) { acc[u][q] = MF::op(a, bw[kk][q], acc[u][q]); });
          });
        }
      });
      __syncthreads();
    }

    // ---- store block J (pivot-position order), diagonal-block inverses, row movement ----
    double *dst = sub;   // 32 x 33 diagonal block
    sfor<TPW>([&](auto u) {
      const int t = w + NWV * u;
      if (t < NTILE) {
        sfor<4>([&](auto r) {
          const int sg = sig[16 * t + lk + 4 * r];
          sfor<2>([&](auto q) {
            Fm[(size_t)(j0 + 16 * q + li) * np + sg] = acc[u][q][(int)r];
            if (sg >= j0 && sg < j0 + 32) dst[(sg - j0) * 33 + 16 * q + li] = acc[u][q][(int)r];
          });
        });
      }
    });
    __syncthreads();
    {
      Lds<double> sd;
      sd.blk = dst;
      invert_diag<double, 32>(sd, 0, Ie + (size_t)J * 2 * WMAX * WMAX, Ie + (size_t)J * 2 * WMAX * WMAX + WMAX * WMAX);
    }
    if (J > 0) {
      for (int xp = j0 + tid; xp < np; xp += NTR) {
        const int y = invb[perm[xp]];
        if (y != xp) {
          const int kq = atomicAdd(mvn, 1);
          mvx[kq] = xp;
          mvy[kq] = y;
        }
      }
    }
    __syncthreads();
    if (J > 0) move_rows_waves<NWV>(mvx, mvy, *mvn, Fm, np, j0);
    __syncthreads();
  }
  int *ip = P.ipiv + (size_t)el * np;
  for (int i = threadIdx.x; i < np; i += NTR) ip[i] = perm[i];
  if (singular && threadIdx.x == 0 && status[el] == HDG_OK) status[el] = HDG_ESINGULAR;
}

template <int NWV, int TPW>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_lu_reg(DevPlan P,
                                                                                               int32_t *status,
                                                                                               double *inv) {
  lu_reg_body<NWV, TPW>(P, blockIdx.x, status, inv);
}

}  // namespace

int condense_width(int np, bool lp) {
  const size_t cap = 160 * 1024;
  const size_t ts = lp ? sizeof(float) : sizeof(double);
  if (lds_layout(np, ts, lp, 32).total <= cap) return 32;
  if (lds_layout(np, ts, lp, 16).total <= cap) return 16;
  return 0;
}

size_t condense_lds_bytes(int np, int w) { return lds_layout(np, sizeof(double), false, w).total; }

size_t condense_lds_bytes_lp(int np, int w) { return lds_layout(np, sizeof(float), true, w).total; }

size_t condense_inv_doubles(int np) { return 2 * (size_t)np * WMAX; }

size_t lp_record_bytes(int np) { return lp_rec_floats(np) * sizeof(float); }

template <typename K, typename... Args>
hipError_t launch_dyn_t(K kern, int ec, int nt, size_t lds, hipStream_t s, Args... args) {
  hipError_t e = set_dyn_lds((const void *)kern, lds);
  if (e) return e;
  hipLaunchKernelGGL(kern, dim3(ec), dim3(nt), lds, s, args...);
  return hipGetLastError();
}

template <typename K, typename... Args>
hipError_t launch_dyn(K kern, int ec, size_t lds, hipStream_t s, Args... args) {
  return launch_dyn_t(kern, ec, NT, lds, s, args...);
}

// grid of the right-hand-side launch: element slots rounded up to the XCD count, times the blocks
static int rhs_grid(const DevPlan &P, int ec, int W) { return (ec + NXCD - 1) / NXCD * NXCD * (P.kx / W); }

bool condense_two_launches(const DevPlan &P) { return (P.cw == 32 || P.cw == 16) && P.condense_launches == 2; }

size_t lu_reg_lds_bytes(int np, int nwv) { return reg_layout(np, nwv).total; }

// Register-resident LU (P.lu_waves waves per workgroup): 2 waves (four elements per CU) for
// n_pad <= 160, 4 waves (two elements per CU, all registers of a wave within 256) for
// n_pad <= 192, 8 waves for n_pad <= 640.
bool lu_reg_supported(int np, int nwv) {
  const int tpw = (np / 16 + nwv - 1) / nwv;
  if (nwv == 2) return tpw <= 5 && reg_layout(np, 2).total <= 40 * 1024;
  if (nwv == 4) return tpw <= 3 && reg_layout(np, 4).total <= 80 * 1024;
  if (nwv == 8) return tpw <= 5 && reg_layout(np, 8).total <= 160 * 1024;
  return false;
}

// Default LU of the two-launch FP64 condensation: the register-resident kernel with the most
// elements per CU that applies (at n_pad = 160, 32,768 elements: LDS kernel 28.0 ms, 4 waves
// 23.3 ms, 2 waves 17.5 ms), else the LDS kernel (at n_pad = 544 the register kernel streams
// the same factors and is slower).
int default_lu_waves(int np) {
  if (lu_reg_supported(np, 2)) return 2;
  return lu_reg_supported(np, 4) ? 4 : 0;
}

hipError_t launch_condense_lu_reg(const DevPlan &P, int ec, int32_t *status, hipStream_t s) {
  const int np = P.n_pad, nwv = P.lu_waves, tpw = (np / 16 + nwv - 1) / nwv;
  const size_t lds = reg_layout(np, nwv).total;
  if (nwv == 2) {
    if (tpw <= 3) return launch_dyn_t(k_lu_reg<2, 3>, ec, 128, lds, s, P, status, P.inv);
    if (tpw <= 5) return launch_dyn_t(k_lu_reg<2, 5>, ec, 128, lds, s, P, status, P.inv);
  }
  if (nwv == 4 && tpw <= 3) return launch_dyn_t(k_lu_reg<4, 3>, ec, 256, lds, s, P, status, P.inv);
  if (nwv == 8) {
    if (tpw <= 2) return launch_dyn_t(k_lu_reg<8, 2>, ec, 512, lds, s, P, status, P.inv);
    if (tpw <= 3) return launch_dyn_t(k_lu_reg<8, 3>, ec, 512, lds, s, P, status, P.inv);
    if (tpw <= 5) return launch_dyn_t(k_lu_reg<8, 5>, ec, 512, lds, s, P, status, P.inv);
  }
  return hipErrorInvalidValue;
}

// (the register-resident LU stores 32 x 32 diagonal-block inverses: 32-column plans only)
hipError_t launch_condense_lu(const DevPlan &P, int e0, int ec, int32_t *status, hipStream_t s) {
  if (P.cw == 16) return launch_dyn(k_lu_f64_w16, ec, condense_lds_bytes(P.n_pad, 16), s, P, e0, status, P.inv);
  if (P.lu_waves) return launch_condense_lu_reg(P, ec, status, s);
  return launch_dyn(k_lu_f64_w32, ec, condense_lds_bytes(P.n_pad, 32), s, P, e0, status, P.inv);
}

// 32-column right-hand sides with 4-wave workgroups where at least two working blocks fit in a
// CU's 160 KB of LDS (at n_pad = 160, 32,768 elements: 39.9 ms against 47.8 ms with 16 waves;
// at n_pad = 96: 0.68 against 1.10 ms per 5,062 elements; 8 waves were slower than either)
static bool rhs_small(const DevPlan &P) { return 2 * condense_lds_bytes(P.n_pad, 32) <= 160 * 1024; }

hipError_t launch_condense_rhs(const DevPlan &P, int e0, int ec, double *S, double *g, double *Y, double *z,
                               hipStream_t s) {
  if (P.cw == 32 && rhs_small(P))
    return launch_dyn_t(k_rhs_f64_w32_small, rhs_grid(P, ec, 32), NT_RHS_SMALL, condense_lds_bytes(P.n_pad, 32), s, P,
                        e0, ec, S, g, Y, z, P.inv);
  if (P.cw == 16)
    return launch_dyn_t(k_rhs_f64_w16, rhs_grid(P, ec, 16), NT_RHS, condense_lds_bytes(P.n_pad, 16), s, P, e0, ec, S,
                        g, Y, z, P.inv);
  return launch_dyn_t(k_rhs_f64_w32, rhs_grid(P, ec, 32), NT_RHS, condense_lds_bytes(P.n_pad, 32), s, P, e0, ec, S,
                      g, Y, z, P.inv);
}

hipError_t launch_condense(const DevPlan &P, int e0, int ec, int32_t *status, double *S, double *g, double *Y,
                           double *z, hipStream_t s) {
  const size_t lds = condense_lds_bytes(P.n_pad, P.cw);
  if (condense_two_launches(P)) {
    hipError_t e = launch_condense_lu(P, e0, ec, status, s);
    if (!e) e = launch_condense_rhs(P, e0, ec, S, g, Y, z, s);
    return e;
  }
  if (P.cw == 32) return launch_dyn(k_condense_f64_w32, ec, lds, s, P, e0, status, S, g, Y, z, P.inv);
  if (P.cw == 16) return launch_dyn(k_condense_f64_w16, ec, lds, s, P, e0, status, S, g, Y, z, P.inv);
  return hipErrorInvalidValue;
}

template <int LPM>
hipError_t launch_condense_lp_t(const DevPlan &P, int e0, int ec, int32_t *status, float *S, double *g, float *Y,
                                double *z, float *fac, hipStream_t s) {
  const size_t lds = condense_lds_bytes_lp(P.n_pad, P.cw_lp);
  if (P.condense_launches == 2 && (P.cw_lp == 32 || P.cw_lp == 16)) {
    hipError_t e;
    if (P.cw_lp == 32) {
      e = launch_dyn(k_lu_f32<32, LPM>, ec, lds, s, P, e0, status, fac);
      if (!e) e = launch_dyn(k_rhs_f32<32, LPM>, rhs_grid(P, ec, 32), lds, s, P, e0, ec, S, g, Y, z, fac);
    } else {
      e = launch_dyn(k_lu_f32<16, LPM>, ec, lds, s, P, e0, status, fac);
      if (!e) e = launch_dyn(k_rhs_f32<16, LPM>, rhs_grid(P, ec, 16), lds, s, P, e0, ec, S, g, Y, z, fac);
    }
    return e;
  }
  if (P.cw_lp == 32) return launch_dyn(k_condense_f32<32, LPM>, ec, lds, s, P, e0, status, S, g, Y, z, fac);
  if (P.cw_lp == 16) return launch_dyn(k_condense_f32<16, LPM>, ec, lds, s, P, e0, status, S, g, Y, z, fac);
  return hipErrorInvalidValue;
}

// FP32 or (P.lp_bf16) BF16 operands on the matrix cores
hipError_t launch_condense_lp(const DevPlan &P, int e0, int ec, int32_t *status, float *S, double *g, float *Y,
                              double *z, float *fac, hipStream_t s) {
  if (P.lp_bf16) return launch_condense_lp_t<2>(P, e0, ec, status, S, g, Y, z, fac, s);
  return launch_condense_lp_t<1>(P, e0, ec, status, S, g, Y, z, fac, s);
}

size_t batch_item_args_bytes() { return sizeof(BatchItemArgs); }

hipError_t launch_condense_batch(const DevPlan *plans_dev, const void *io_dev, const int *lu_queue, int n_lu,
                                 const void *rhs_queue, const int *rhs_xoff, int *counters, int lu_groups,
                                 int rhs_groups, bool persistent, size_t lds, hipStream_t s) {
  const BatchItemArgs *io = static_cast<const BatchItemArgs *>(io_dev);
  const int2 *rq = static_cast<const int2 *>(rhs_queue);
  hipError_t e;
  if (persistent) {
    e = set_dyn_lds((const void *)k_lu_batch_persistent, lds);
    if (!e) e = set_dyn_lds((const void *)k_rhs_batch_persistent, lds);
    if (e) return e;
    hipLaunchKernelGGL(k_lu_batch_persistent, dim3(lu_groups), dim3(NT), lds, s, plans_dev, io, lu_queue, n_lu,
                       counters);
    e = hipGetLastError();
    if (e) return e;
    hipLaunchKernelGGL(k_rhs_batch_persistent, dim3(rhs_groups), dim3(NT_RHS), lds, s, plans_dev, io, rq, rhs_xoff,
                       counters + 1);
    return hipGetLastError();
  }
  e = set_dyn_lds((const void *)k_lu_batch, lds);
  if (!e) e = set_dyn_lds((const void *)k_rhs_batch, lds);
  if (e) return e;
  hipLaunchKernelGGL(k_lu_batch, dim3(lu_groups), dim3(NT), lds, s, plans_dev, io, lu_queue, n_lu);
  e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_rhs_batch, dim3(rhs_groups), dim3(NT_RHS), lds, s, plans_dev, io, rq, rhs_xoff);
  return hipGetLastError();
}

hipError_t launch_lp_solve(const DevPlan &P, const float *fac, const double *r, double *x, hipStream_t s) {
  const int w = P.cw_lp;
  const size_t lds = (size_t)(P.n_pad + w) * sizeof(double) + (size_t)P.n_pad * sizeof(int);
  hipLaunchKernelGGL(k_lp_solve, dim3(P.n_elem), dim3(SB), lds, s, P.n, P.n_pad, w, fac, r, x);
  return hipGetLastError();
}

}  // namespace hdg
