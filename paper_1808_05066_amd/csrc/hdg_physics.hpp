// Pointwise physics in entropy variables, device side.
//
// Written once over a scalar type T that is either double or Dual (value plus
// one directional derivative): a pass with Dual seeded along one input
// direction yields that column of the pointwise Jacobian exactly (forward-mode
// differentiation), so the element Jacobian needs no hand-derived second
// derivatives of u(v).
//
// Paper sections used: perfect-gas Euler flux and pressure (Euler section);
// Newtonian stress with beta = 0 and Fourier heat flux, kappa = c_p mu / Pr
// (Navier-Stokes section); entropy variables of H = -rho s (entropy pairs
// section); inviscid trace flux and the symmetric Lax-Friedrichs matrix with
// v* = v_hat (numerical-flux equation and its definition in the stability
// section, choice stated in the numerical examples); viscous trace flux
// G(v_hat, q).n.  R = 1 so T = p / rho = -(gamma-1)/v_m, c_v = 1/(gamma-1).
// Viscous gradients are taken straight from q ~ grad v:
//   grad T = (gamma-1) grad v_m / v_m^2,  grad V_i = -grad w_i / v_m + w_i grad v_m / v_m^2.
#pragma once
#include <hip/hip_runtime.h>

namespace hdg {

struct Dual {
  double v, d;
};

__host__ __device__ inline Dual mk(double v, double d) { return Dual{v, d}; }
__host__ __device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__host__ __device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__host__ __device__ inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
__host__ __device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__host__ __device__ inline Dual operator/(Dual a, Dual b) {
  double r = 1.0 / b.v;
  double q = a.v * r;
  return {q, (a.d - q * b.d) * r};
}
__host__ __device__ inline Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__host__ __device__ inline Dual operator+(double b, Dual a) { return {a.v + b, a.d}; }
__host__ __device__ inline Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
__host__ __device__ inline Dual operator-(double b, Dual a) { return {b - a.v, -a.d}; }
__host__ __device__ inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__host__ __device__ inline Dual operator*(double b, Dual a) { return {a.v * b, a.d * b}; }
__host__ __device__ inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
__host__ __device__ inline Dual operator/(double a, Dual b) {
  double q = a / b.v;
  return {q, -q * b.d / b.v};
}

__device__ inline double dexp(double x) { return exp(x); }
__device__ inline Dual dexp(Dual x) {
  double e = exp(x.v);
  return {e, e * x.d};
}
__device__ inline double dpow(double x, double a) { return pow(x, a); }
__device__ inline Dual dpow(Dual x, double a) {
  double y = pow(x.v, a);
  return {y, a * y / x.v * x.d};
}
__device__ inline double dlog(double x) { return log(x); }
__device__ inline Dual dlog(Dual x) { return {log(x.v), x.d / x.v}; }
__device__ inline double dsqrt(double x) { return sqrt(x); }
__device__ inline Dual dsqrt(Dual x) {
  double s = sqrt(x.v);
  return {s, 0.5 * x.d / s};
}
// |x| with derivative +1 at x = 0
__device__ inline double dabs(double x) { return x >= 0.0 ? x : -x; }
__device__ inline Dual dabs(Dual x) { return x.v >= 0.0 ? x : -x; }
__device__ inline double val(double x) { return x; }
__device__ inline double val(Dual x) { return x.v; }
__device__ inline double der(double) { return 0.0; }
__device__ inline double der(Dual x) { return x.d; }

template <typename T>
__device__ inline T cst(double x) { return T(x); }
template <>
__device__ inline Dual cst<Dual>(double x) { return Dual{x, 0.0}; }

// Primitive state from entropy variables (inverse of the entropy-variable map).
template <int D, typename T>
struct Prim {
  T rho, p, V[D], vm, w[D];
};

template <int D, typename T>
__device__ inline Prim<D, T> prim_of_v(const T *v, double gam) {
  Prim<D, T> s;
  const T vm = v[D + 1];
  T ww = cst<T>(0.0);
  for (int i = 0; i < D; ++i) {
    s.w[i] = v[1 + i];
    ww = ww + v[1 + i] * v[1 + i];
  }
  s.vm = vm;
  // physical entropy s = gamma - v1 + |w|^2 / (2 v_m); rho^(gamma-1) = (gamma-1)/(-v_m) e^{-s}
  T sent = gam - v[0] + ww / (2.0 * vm);
  s.rho = dpow((gam - 1.0) / (-vm) * dexp(-sent), 1.0 / (gam - 1.0));
  s.p = (gam - 1.0) * s.rho / (-vm);
  for (int i = 0; i < D; ++i) s.V[i] = -s.w[i] / vm;
  return s;
}

template <int D, typename T>
__device__ inline void u_of_prim(const Prim<D, T> &s, double gam, T *u) {
  T kin = cst<T>(0.0);
  for (int i = 0; i < D; ++i) kin = kin + s.V[i] * s.V[i];
  u[0] = s.rho;
  for (int i = 0; i < D; ++i) u[1 + i] = s.rho * s.V[i];
  u[D + 1] = s.p / (gam - 1.0) + 0.5 * s.rho * kin;
}

// Inviscid flux along n (n == nullptr: all directions into F[c*D + j]).
template <int D, typename T>
__device__ inline void flux_F(const Prim<D, T> &s, double gam, T *F) {
  T kin = cst<T>(0.0);
  for (int i = 0; i < D; ++i) kin = kin + s.V[i] * s.V[i];
  T H = s.p / (gam - 1.0) + 0.5 * s.rho * kin + s.p;   // rho E + p
  for (int j = 0; j < D; ++j) {
    F[0 * D + j] = s.rho * s.V[j];
    for (int i = 0; i < D; ++i) F[(1 + i) * D + j] = s.rho * s.V[i] * s.V[j] + (i == j ? s.p : cst<T>(0.0));
    F[(D + 1) * D + j] = s.V[j] * H;
  }
}

// Viscous flux G[c*D + j] from the state and q[c*D + k] (q of scalar type Q).
template <int D, typename T, typename Q>
__device__ inline void flux_G(const Prim<D, T> &s, const Q *q, double gam, double mu, double Pr, T *G) {
  const T vm2 = s.vm * s.vm;
  T gT[D], gV[D][D];
  for (int k = 0; k < D; ++k) gT[k] = (gam - 1.0) * q[(D + 1) * D + k] / vm2;
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k) gV[i][k] = s.w[i] * q[(D + 1) * D + k] / vm2 - q[(1 + i) * D + k] / s.vm;
  T div = cst<T>(0.0);
  for (int i = 0; i < D; ++i) div = div + gV[i][i];
  const double kappa = gam / (gam - 1.0) * mu / Pr;
  for (int j = 0; j < D; ++j) {
    G[0 * D + j] = cst<T>(0.0);
    T vt = cst<T>(0.0);
    for (int i = 0; i < D; ++i) {
      T tau = mu * (gV[i][j] + gV[j][i]);
      if (i == j) tau = tau - (2.0 / 3.0) * mu * div;
      G[(1 + i) * D + j] = -tau;
      vt = vt + s.V[i] * tau;
    }
    G[(D + 1) * D + j] = -vt - kappa * gT[j];
  }
}

// dU/dV in closed form (symmetric), from the primitive state.
template <int D, typename T>
__device__ inline void A0_of_prim(const Prim<D, T> &s, double gam, T *A) {
  const int M = D + 2;
  T kin = cst<T>(0.0);
  for (int i = 0; i < D; ++i) kin = kin + s.V[i] * s.V[i];
  const double g1 = 1.0 / (gam - 1.0);
  T E = s.p / ((gam - 1.0) * s.rho) + 0.5 * kin;
  T Ht = E + s.p / s.rho;
  T c2 = gam * s.p / s.rho;
  A[0] = s.rho * g1;
  for (int i = 0; i < D; ++i) {
    A[0 * M + 1 + i] = s.rho * s.V[i] * g1;
    A[(1 + i) * M + 0] = A[0 * M + 1 + i];
    for (int k = 0; k < D; ++k)
      A[(1 + i) * M + 1 + k] = (s.rho * s.V[i] * s.V[k] + (i == k ? s.p : cst<T>(0.0))) * g1;
    A[(1 + i) * M + M - 1] = s.rho * Ht * s.V[i] * g1;
    A[(M - 1) * M + 1 + i] = A[(1 + i) * M + M - 1];
  }
  A[0 * M + M - 1] = s.rho * E * g1;
  A[(M - 1) * M + 0] = A[0 * M + M - 1];
  A[(M - 1) * M + M - 1] = (s.rho * Ht * Ht - c2 * s.p * g1) * g1;
}

// Symmetric variable stabilization sigma_S dv = |A_n(v*)| A0(v*) dv (Section 4): du = A0 dv, its
// primitive perturbation (linearized), then the wave decomposition of the Euler flux Jacobian
// along the unit normal n -- acoustic speeds u_n -/+ c with strengths (dp -/+ rho c du_n)/(2c^2)
// on (1, V -/+ c n, H -/+ c u_n), entropy (speed u_n, strength drho - dp/c^2) on (1, V, |V|^2/2)
// and shear (speed u_n) rho (0, dV_t, V . dV_t) -- each scaled by |speed|.
template <int D, typename T, typename U>
__device__ inline void sigma_s_apply(const Prim<D, T> &s, const T *A0, const double *n, double gam, const U *dv,
                                     T *out) {
  const int M = D + 2;
  T du[M];
  for (int c = 0; c < M; ++c) {
    T a = cst<T>(0.0);
    for (int e = 0; e < M; ++e) a = a + A0[c * M + e] * dv[e];
    du[c] = a;
  }
  T kin = cst<T>(0.0);
  for (int i = 0; i < D; ++i) kin = kin + s.V[i] * s.V[i];
  T dV[D], vdV = cst<T>(0.0), un = cst<T>(0.0), dun = cst<T>(0.0);
  for (int i = 0; i < D; ++i) {
    dV[i] = (du[1 + i] - s.V[i] * du[0]) / s.rho;
    vdV = vdV + s.V[i] * dV[i];
    un = un + s.V[i] * n[i];
    dun = dun + dV[i] * n[i];
  }
  const T dp = (gam - 1.0) * (du[M - 1] - 0.5 * kin * du[0] - s.rho * vdV);
  const T c2 = gam * s.p / s.rho, c = dsqrt(c2);
  const T H = c2 / (gam - 1.0) + 0.5 * kin;
  const T a1 = (dp - s.rho * c * dun) / (2.0 * c2), a4 = (dp + s.rho * c * dun) / (2.0 * c2);
  const T a2 = du[0] - dp / c2;
  const T l1 = dabs(un - c), l2 = dabs(un), l4 = dabs(un + c);
  T vdVt = cst<T>(0.0);
  for (int i = 0; i < D; ++i) vdVt = vdVt + s.V[i] * (dV[i] - dun * n[i]);
  out[0] = l1 * a1 + l2 * a2 + l4 * a4;
  for (int i = 0; i < D; ++i)
    out[1 + i] = l1 * a1 * (s.V[i] - c * n[i]) + l2 * (a2 * s.V[i] + s.rho * (dV[i] - dun * n[i])) +
                 l4 * a4 * (s.V[i] + c * n[i]);
  out[M - 1] = l1 * a1 * (H - c * un) + l2 * (a2 * 0.5 * kin + s.rho * vdVt) + l4 * a4 * (H + c * un);
}

// Wave speeds u_n - c, u_n, u_n + c at the state va + th (vb - va) (real values).
template <int D>
__device__ inline void path_speeds(const double *va, const double *vb, double th, const double *n, double gam,
                                   double *g) {
  const int M = D + 2;
  double vt[M];
  for (int c = 0; c < M; ++c) vt[c] = va[c] + th * (vb[c] - va[c]);
  const Prim<D, double> st = prim_of_v<D, double>(vt, gam);
  double un = 0.0;
  for (int j = 0; j < D; ++j) un += st.V[j] * n[j];
  const double c = sqrt(gam * st.p / st.rho);
  g[0] = un - c;
  g[1] = un;
  g[2] = un + c;
}

// Breakpoints of the mean-value integrand along the straight path va + th (vb - va): 0, 1 and
// the roots in between of the three wave speeds (kinks of |A_n|), located by sign changes over
// MV_NS equal sub-intervals and bisection; sorted into br, returns their number (2..5).
constexpr int MV_NS = 16;
template <int D>
__device__ inline int mv_breakpoints(const double *va, const double *vb, const double *n, double gam, double *br) {
  int nb = 0;
  double roots[3];
  double ga[3], gb[3];
  path_speeds<D>(va, vb, 0.0, n, gam, ga);
  for (int j = 0; j < MV_NS; ++j) {
    const double t0 = (double)j / MV_NS, t1 = (double)(j + 1) / MV_NS;
    path_speeds<D>(va, vb, t1, n, gam, gb);
    for (int k = 0; k < 3; ++k) {
      if (!((ga[k] < 0.0 && gb[k] > 0.0) || (ga[k] > 0.0 && gb[k] < 0.0) || (gb[k] == 0.0 && ga[k] != 0.0))) continue;
      double lo = t0, hi = t1, flo = ga[k];
      for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        double gm[3];
        path_speeds<D>(va, vb, mid, n, gam, gm);
        if ((gm[k] > 0.0) == (flo > 0.0) && gm[k] != 0.0) {
          lo = mid;
          flo = gm[k];
        } else {
          hi = mid;
        }
      }
      if (nb < 3) roots[nb++] = 0.5 * (lo + hi);
    }
    for (int k = 0; k < 3; ++k) ga[k] = gb[k];
  }
  br[0] = 0.0;
  for (int i = 0; i < nb; ++i) {   // insertion into the sorted list
    int p = i + 1;
    while (p > 1 && br[p - 1] > roots[i]) {
      br[p] = br[p - 1];
      --p;
    }
    br[p] = roots[i];
  }
  br[nb + 1] = 1.0;
  return nb + 2;
}

// Mean-value stabilization (Section 4) on the straight path in entropy variables:
// sigma_MV(vh, v) dv = int_0^1 sigma_S(vh + th (v - vh)) dv dth (the definition's two (1 - th)
// weighted integrals add up to this).  The integrand is smooth except where a wave speed changes
// sign along the path; the integral is split there (breakpoints from the values of the states)
// and each piece integrated with 8-point Gauss-Legendre.  Derivatives (T = Dual) need no term
// for the moving breakpoints: the integrand is continuous across them.
template <int D, typename T>
__device__ inline void sigma_mv_apply(const T *vh, const T *v, const double *n, double gam, const T *dv, T *out) {
  const int M = D + 2;
  // Gauss-Legendre, 8 points on [-1, 1] (nodes +-x_i, weights w_i)
  const double gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
  const double gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
  double va[M], vb[M], br[5];
  for (int c = 0; c < M; ++c) {
    va[c] = val(vh[c]);
    vb[c] = val(v[c]);
  }
  const int nb = mv_breakpoints<D>(va, vb, n, gam, br);
  for (int c = 0; c < M; ++c) out[c] = cst<T>(0.0);
  for (int i = 0; i + 1 < nb; ++i) {
    const double a = br[i], h = br[i + 1] - br[i];
    if (!(h > 0.0)) continue;
    for (int g = 0; g < 8; ++g) {
      const double x = (g < 4) ? -gx[3 - g] : gx[g - 4];
      const double wq = 0.5 * h * ((g < 4) ? gw[3 - g] : gw[g - 4]);
      const double th = a + 0.5 * h * (1.0 + x);
      T vt[M];
      for (int c = 0; c < M; ++c) vt[c] = vh[c] + th * (v[c] - vh[c]);
      const Prim<D, T> st = prim_of_v<D, T>(vt, gam);
      T A[M * M], o[M];
      A0_of_prim<D, T>(st, gam, A);
      sigma_s_apply<D, T, T>(st, A, n, gam, dv, o);
      for (int c = 0; c < M; ++c) out[c] = out[c] + wq * o[c];
    }
  }
}

// Inviscid trace flux with the mean-value stabilization: 1/2 (F_n(vh) + F_n(v)) + 1/2 sigma_MV (v - vh),
// both states of type T (derivatives with respect to either).
template <int D, typename T>
__device__ inline void fhat_mv(const T *vh, const T *v, const double *n, double gam, T *out) {
  const int M = D + 2;
  T Fh[M * D], Fv[M * D], dv[M], sd[M];
  flux_F<D, T>(prim_of_v<D, T>(vh, gam), gam, Fh);
  flux_F<D, T>(prim_of_v<D, T>(v, gam), gam, Fv);
  for (int c = 0; c < M; ++c) dv[c] = v[c] - vh[c];
  sigma_mv_apply<D, T>(vh, v, n, gam, dv, sd);
  for (int c = 0; c < M; ++c) {
    T fn = cst<T>(0.0);
    for (int j = 0; j < D; ++j) fn = fn + (Fh[c * D + j] + Fv[c * D + j]) * n[j];
    out[c] = 0.5 * fn + 0.5 * sd[c];
  }
}

// Trace flux f_hat + g_hat at one face point (stabilization sigma_SLF = lambda_max A0, or
// sigma_S with sym_s, both at v* = v_hat).  vh: trace state (type T),
// F_n(v) of the element state precomputed (double), dv = v - v_hat evaluated
// inside, q (type Q) the element gradient unknowns (ignored if !visc).
template <int D, typename T, typename Q>
__device__ inline void trace_flux(const T *vh, const double *v, const double *Fnv, const Q *q,
                                  const double *n, double gam, double mu, double Pr, bool visc,
                                  T *out, bool sym_s = false) {
  const int M = D + 2;
  Prim<D, T> s = prim_of_v<D, T>(vh, gam);
  T F[M * D];
  flux_F<D, T>(s, gam, F);
  T A[M * M];
  A0_of_prim<D, T>(s, gam, A);
  T vn = cst<T>(0.0);
  for (int j = 0; j < D; ++j) vn = vn + s.V[j] * n[j];
  T lam = dabs(vn) + dsqrt(gam * s.p / s.rho);
  T dv[M], ss[M];
  for (int c = 0; c < M; ++c) dv[c] = v[c] - vh[c];
  if (sym_s) sigma_s_apply<D, T, T>(s, A, n, gam, dv, ss);
  for (int c = 0; c < M; ++c) {
    T fn = cst<T>(0.0);
    for (int j = 0; j < D; ++j) fn = fn + F[c * D + j] * n[j];
    T sd = cst<T>(0.0);
    if (sym_s) {
      sd = ss[c];
    } else {
      for (int e = 0; e < M; ++e) sd = sd + A[c * M + e] * dv[e];
      sd = lam * sd;
    }
    out[c] = 0.5 * (fn + Fnv[c]) + 0.5 * sd;
  }
  if (visc) {
    T G[M * D];
    flux_G<D, T, Q>(s, q, gam, mu, Pr, G);
    for (int c = 0; c < M; ++c) {
      T gn = cst<T>(0.0);
      for (int j = 0; j < D; ++j) gn = gn + G[c * D + j] * n[j];
      out[c] = out[c] + gn;
    }
  }
}

}  // namespace hdg
