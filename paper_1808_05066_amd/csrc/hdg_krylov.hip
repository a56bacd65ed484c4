// Kernels of the global trace solve: block-Jacobi assembly, inversion and
// application on the condensed operator sum_K P_K^T S_K P_K, and the vector
// kernels of restarted GMRES (multi-dot with a two-stage reduction,
// multi-AXPY, scaling, linear combinations).  The paper does not describe its
// linear solver; GMRES with a block-Jacobi preconditioner is this library's.
#include "hdg_plan.hpp"

namespace hdg {

namespace {

constexpr int RB = 256;   // reduction block size

// Face blocks: unknowns of one mesh face (HDG), ordered (c, p) -> c*Nfp + p with p
// the position of the trace node in the block's node list.  Each block sums the
// face-diagonal part of S of its (at most two) adjacent elements.
template <typename T>
__global__ void k_bj_assemble_face(DevPlan P, const T *__restrict__ S, double *B) {
  const int blk = blockIdx.x;
  const int M = P.m, Nfp = P.Nfp, k = P.k, bs = M * Nfp;
  double *Bb = B + (size_t)blk * bs * bs;
  for (int t = threadIdx.x; t < bs * bs; t += blockDim.x) {
    const int row = t % bs, col = t / bs;
    const int c = row / Nfp, p = row % Nfp, c2 = col / Nfp, p2 = col % Nfp;
    double acc = 0.0;
    for (int q = 0; q < 2; ++q) {
      const int e = P.bj_ce[blk * 2 + q];
      if (e < 0) continue;
      const int f = P.bj_cf[blk * 2 + q];
      const int *loc = P.bj_loc + ((size_t)blk * 2 + q) * Nfp;
      const int i = f * M * Nfp + c * Nfp + loc[p];
      const int j = f * M * Nfp + c2 * Nfp + loc[p2];
      acc += (double)S[(size_t)e * k * k + (size_t)j * k + i];
    }
    Bb[(size_t)col * bs + row] = acc;
  }
}

// Point blocks (m x m per trace node): every pair of element trace rows that map
// to the same node adds its entry (FP64 atomics; used when faces share nodes).
template <typename T>
__global__ void k_bj_assemble_point(DevPlan P, const T *__restrict__ S, double *B) {
  const int e = blockIdx.x;
  const int M = P.m, Nfp = P.Nfp, k = P.k;
  const int *tm = P.tmap + (size_t)e * P.nf * Nfp;
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    const int i = t % k, j = t / k;
    const int bi = i % Nfp, fi = i / (M * Nfp), ci = (i / Nfp) % M;
    const int bj = j % Nfp, fj = j / (M * Nfp), cj = (j / Nfp) % M;
    const int ni = tm[fi * Nfp + bi], nj = tm[fj * Nfp + bj];
    if (ni != nj) continue;
    atomicAdd(&B[(size_t)ni * M * M + cj * M + ci], (double)S[(size_t)e * k * k + (size_t)j * k + i]);
  }
}

// In-place inverse of each bs x bs block (column-major): Gauss-Jordan with
// partial pivoting on [B | I] held in LDS, every thread of the workgroup
// updating entries of the augmented matrix at each elimination step.
constexpr int BI = 256;

__global__ __launch_bounds__(BI) void k_block_invert(double *B, int bs, int32_t *bad) {
  extern __shared__ double aug[];   // [2 bs][bs + 1] column-major, then the multiplier column [bs]
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int ld = bs + 1, nc = 2 * bs;
  double *Bb = B + (size_t)blk * bs * bs;
  double *mul = aug + (size_t)nc * ld;
  __shared__ int s_p;
  __shared__ int s_zero;
  for (int t = tid; t < nc * bs; t += BI) {
    const int c = t / bs, i = t - c * bs;
    aug[c * ld + i] = c < bs ? Bb[(size_t)c * bs + i] : (c - bs == i ? 1.0 : 0.0);
  }
  if (tid == 0) s_zero = 0;
  __syncthreads();
  for (int j = 0; j < bs; ++j) {
    if (tid < 64) {
      double best = -1.0;
      int bi = j;
      for (int i = j + tid; i < bs; i += 64) {
        const double v = fabs(aug[j * ld + i]);
        if (v > best) {
          best = v;
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
      if (tid == 0) {
        s_p = bi;
        if (!(best > 0.0)) s_zero = 1;
      }
    }
    __syncthreads();
    const int p = s_p;
    if (p != j)
      for (int c = tid; c < nc; c += BI) {
        const double t0 = aug[c * ld + j];
        aug[c * ld + j] = aug[c * ld + p];
        aug[c * ld + p] = t0;
      }
    __syncthreads();
    const double d = aug[j * ld + j];
    const double inv = d != 0.0 ? 1.0 / d : 0.0;
    for (int i = tid; i < bs; i += BI) mul[i] = (i == j) ? 0.0 : aug[j * ld + i];
    __syncthreads();
    for (int c = tid; c < nc; c += BI) aug[c * ld + j] *= inv;
    __syncthreads();
    for (int t = tid; t < nc * bs; t += BI) {
      const int c = t / bs, i = t - c * bs;
      if (i != j) aug[c * ld + i] -= mul[i] * aug[c * ld + j];
    }
    __syncthreads();
  }
  for (int t = tid; t < bs * bs; t += BI) {
    const int c = t / bs, i = t - c * bs;
    Bb[(size_t)c * bs + i] = aug[(bs + c) * ld + i];
  }
  if (tid == 0 && s_zero) atomicAdd(bad, 1);
}

// z = blockdiag(Binv) r on [m][n_trace] vectors.
__global__ void k_block_apply(DevPlan P, const double *__restrict__ Binv, const double *__restrict__ r, double *z,
                              int bs, int nodes_per_blk) {
  extern __shared__ double rv[];
  const int blk = blockIdx.x;
  const int *nodes = P.bj_nodes + (size_t)blk * nodes_per_blk;
  const size_t NT_ = (size_t)P.n_trace;
  for (int i = threadIdx.x; i < bs; i += blockDim.x) {
    const int c = i / nodes_per_blk, p = i % nodes_per_blk;
    rv[i] = r[c * NT_ + nodes[p]];
  }
  __syncthreads();
  const double *Bb = Binv + (size_t)blk * bs * bs;
  for (int i = threadIdx.x; i < bs; i += blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < bs; ++j) acc += Bb[(size_t)j * bs + i] * rv[j];
    const int c = i / nodes_per_blk, p = i % nodes_per_blk;
    z[c * NT_ + nodes[p]] = acc;
  }
}

// partial[b][i] = sum over this block's slice of V[i][:] * w[:], i < nv
__global__ void k_multidot(const double *__restrict__ V, size_t ldv, int nv, const double *__restrict__ w, size_t N,
                           double *partial) {
  __shared__ double red[RB];
  const size_t per = (N + gridDim.x - 1) / gridDim.x;
  const size_t lo = blockIdx.x * per, hi = lo + per < N ? lo + per : N;
  for (int i = 0; i < nv; ++i) {
    double acc = 0.0;
    const double *Vi = V + (size_t)i * ldv;
    for (size_t t = lo + threadIdx.x; t < hi; t += RB) acc += Vi[t] * w[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * nv + i] = red[0];
    __syncthreads();
  }
}

__global__ void k_reduce_partial(const double *__restrict__ partial, int nb, int nv, double *out) {
  const int i = blockIdx.x;
  __shared__ double red[RB];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += RB) acc += partial[(size_t)b * nv + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// w -= sum_i h[i] V[i], and accumulate h into hacc (if given)
__global__ void k_multiaxpy(const double *__restrict__ V, size_t ldv, int nv, const double *__restrict__ h, double *w,
                            size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  double acc = w[t];
  for (int i = 0; i < nv; ++i) acc -= h[i] * V[(size_t)i * ldv + t];
  w[t] = acc;
}

// out = sum_i y[i] V[i]
__global__ void k_lincomb(const double *__restrict__ V, size_t ldv, int nv, const double *__restrict__ y, double *out,
                          size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  double acc = 0.0;
  for (int i = 0; i < nv; ++i) acc += y[i] * V[(size_t)i * ldv + t];
  out[t] = acc;
}

// out = alpha * x + beta * y  (y may be null for beta = 0)
__global__ void k_axpby(double alpha, const double *__restrict__ x, double beta, const double *__restrict__ y,
                        double *out, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  out[t] = alpha * x[t] + (y ? beta * y[t] : 0.0);
}

// out = x / s[0]   (s on the device)
__global__ void k_scale_by(const double *__restrict__ x, const double *__restrict__ s, double *out, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  out[t] = x[t] / s[0];
}

// Largest per-element ratio ||r_e|| / ||b_e|| over elements (r, b element-local [E][n]): one
// workgroup per element, the ratio (non-negative, so its bits order as unsigned integers) merged
// into *out by an atomic maximum (*out must start at 0); per[e] the ratio itself, if per is given.
__global__ __launch_bounds__(RB) void k_elem_ratio_max(const double *__restrict__ r, const double *__restrict__ b, int n,
                                                       unsigned long long *out, double *per) {
  __shared__ double sr[RB], sb[RB];
  const int e = blockIdx.x, tid = threadIdx.x;
  double ar = 0.0, ab = 0.0;
  for (int i = tid; i < n; i += RB) {
    const double x = r[(size_t)e * n + i], y = b[(size_t)e * n + i];
    ar += x * x;
    ab += y * y;
  }
  sr[tid] = ar;
  sb[tid] = ab;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if (tid < w) {
      sr[tid] += sr[tid + w];
      sb[tid] += sb[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double ratio = sb[0] > 0.0 ? sqrt(sr[0] / sb[0]) : (sr[0] > 0.0 ? INFINITY : 0.0);
    atomicMax(out, (unsigned long long)__double_as_longlong(ratio));
    if (per) per[e] = ratio;
  }
}

}  // namespace

template <typename T>
hipError_t launch_bj_assemble_t(const DevPlan &P, const T *S, double *B, hipStream_t s) {
  if (P.bj_face) {
    hipLaunchKernelGGL(k_bj_assemble_face<T>, dim3(P.bj_nblk), dim3(256), 0, s, P, S, B);
  } else {
    hipError_t e = launch_fill_double(B, (size_t)P.bj_nblk * P.m * P.m, 0.0, s);
    if (e) return e;
    hipLaunchKernelGGL(k_bj_assemble_point<T>, dim3(P.n_elem), dim3(256), 0, s, P, S, B);
  }
  return hipGetLastError();
}

hipError_t launch_bj_assemble(const DevPlan &P, const double *S, double *B, hipStream_t s) {
  return launch_bj_assemble_t<double>(P, S, B, s);
}

hipError_t launch_bj_assemble_f32(const DevPlan &P, const float *S, double *B, hipStream_t s) {
  return launch_bj_assemble_t<float>(P, S, B, s);
}

hipError_t launch_block_invert(const DevPlan &P, double *B, int32_t *bad, hipStream_t s) {
  const int bs = P.bj_bs;
  const size_t lds = ((size_t)2 * bs * (bs + 1) + bs) * sizeof(double);
  hipError_t e = set_dyn_lds((const void *)k_block_invert, lds);
  if (e) return e;
  hipLaunchKernelGGL(k_block_invert, dim3(P.bj_nblk), dim3(BI), lds, s, B, bs, bad);
  return hipGetLastError();
}

hipError_t launch_block_apply(const DevPlan &P, const double *Binv, const double *r, double *z, hipStream_t s) {
  const int bs = P.bj_bs;
  const int npb = P.bj_face ? P.Nfp : 1;
  hipLaunchKernelGGL(k_block_apply, dim3(P.bj_nblk), dim3(bs <= 64 ? 64 : 128), bs * sizeof(double), s, P, Binv, r,
                     z, bs, npb);
  return hipGetLastError();
}

hipError_t launch_elem_ratio_max(const double *r, const double *b, int E, int n, unsigned long long *out,
                                 double *per, hipStream_t s) {
  hipLaunchKernelGGL(k_elem_ratio_max, dim3(E), dim3(RB), 0, s, r, b, n, out, per);
  return hipGetLastError();
}

hipError_t launch_multidot(const double *V, size_t ldv, int nv, const double *w, size_t N, double *partial, int nb,
                           double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_multidot, dim3(nb), dim3(RB), 0, s, V, ldv, nv, w, N, partial);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_reduce_partial, dim3(nv), dim3(RB), 0, s, partial, nb, nv, out);
  return hipGetLastError();
}

hipError_t launch_multiaxpy(const double *V, size_t ldv, int nv, const double *h, double *w, size_t N,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_multiaxpy, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, V, ldv, nv, h, w, N);
  return hipGetLastError();
}

hipError_t launch_lincomb(const double *V, size_t ldv, int nv, const double *y, double *out, size_t N,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, V, ldv, nv, y, out, N);
  return hipGetLastError();
}

hipError_t launch_axpby(double alpha, const double *x, double beta, const double *y, double *out, size_t N,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, alpha, x, beta, y, out, N);
  return hipGetLastError();
}

hipError_t launch_scale_by(const double *x, const double *sc, double *out, size_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, x, sc, out, N);
  return hipGetLastError();
}

}  // namespace hdg
