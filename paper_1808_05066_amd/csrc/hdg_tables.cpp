// Reference-element tables (host).  See hdg_tables.hpp.
#include "hdg_tables.hpp"

#include <cmath>
#include <cstring>

namespace hdg {

namespace {

// Legendre P_n and its derivative at x (three-term recurrence).
void legendre(int n, double x, double &P, double &dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // derivative from P_n and P_{n-1}; away from +-1 only
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

int n_nodes(int etype, int p) {
  switch (etype) {
    case TRI: return (p + 1) * (p + 2) / 2;
    case QUAD: return (p + 1) * (p + 1);
    case TET: return (p + 1) * (p + 2) * (p + 3) / 6;
    default: return (p + 1) * (p + 1) * (p + 1);
  }
}

// R_i(lambda) = prod_{s<i} (p lambda - s)/(s+1) and its derivative.
void silvester(int i, int p, double lam, double &R, double &dR) {
  R = 1.0;
  dR = 0.0;
  for (int s = 0; s < i; ++s) {
    double f = (p * lam - s) / (s + 1.0);
    double df = p / (s + 1.0);
    dR = dR * f + R * df;
    R = R * f;
  }
}

// 1D Lagrange polynomial i on nodes r[0..p] and its derivative at x.
void lagrange1d(const double *r, int p, int i, double x, double &l, double &dl) {
  l = 1.0;
  dl = 0.0;
  for (int k = 0; k <= p; ++k) {
    if (k == i) continue;
    double f = (x - r[k]) / (r[i] - r[k]);
    double df = 1.0 / (r[i] - r[k]);
    dl = dl * f + l * df;
    l = l * f;
  }
}

void tri_rule(int n, std::vector<double> &pts, std::vector<double> &w) {
  std::vector<double> g(n), gw(n);
  gauss_legendre(n, g.data(), gw.data());
  pts.clear();
  w.clear();
  for (int ib = 0; ib < n; ++ib)
    for (int ia = 0; ia < n; ++ia) {
      double a = 0.5 * (g[ia] + 1.0), b = 0.5 * (g[ib] + 1.0);
      pts.push_back(a * (1.0 - b));
      pts.push_back(b);
      w.push_back(0.25 * gw[ia] * gw[ib] * (1.0 - b));
    }
}

void tet_rule(int n, std::vector<double> &pts, std::vector<double> &w) {
  std::vector<double> g(n), gw(n);
  gauss_legendre(n, g.data(), gw.data());
  pts.clear();
  w.clear();
  for (int ic = 0; ic < n; ++ic)
    for (int ib = 0; ib < n; ++ib)
      for (int ia = 0; ia < n; ++ia) {
        double a = 0.5 * (g[ia] + 1.0), b = 0.5 * (g[ib] + 1.0), c = 0.5 * (g[ic] + 1.0);
        pts.push_back(a * (1.0 - b) * (1.0 - c));
        pts.push_back(b * (1.0 - c));
        pts.push_back(c);
        w.push_back(0.125 * gw[ia] * gw[ib] * gw[ic] * (1.0 - b) * (1.0 - c) * (1.0 - c));
      }
}

void tensor_rule(int d, int n, std::vector<double> &pts, std::vector<double> &w) {
  std::vector<double> g(n), gw(n);
  gauss_legendre(n, g.data(), gw.data());
  pts.clear();
  w.clear();
  int tot = 1;
  for (int a = 0; a < d; ++a) tot *= n;
  for (int t = 0; t < tot; ++t) {
    int r = t;
    double ww = 1.0;
    for (int a = 0; a < d; ++a) {
      int i = r % n;
      r /= n;
      pts.push_back(g[i]);
      ww *= gw[i];
    }
    w.push_back(ww);
  }
}

}  // namespace

void gauss_legendre(int n, double *x, double *w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double P, dP;
    for (int it = 0; it < 100; ++it) {
      legendre(n, z, P, dP);
      double dz = P / dP;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    legendre(n, z, P, dP);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
}

void gll_points(int p, double *x) {
  const double pi = 3.14159265358979323846;
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double z = -std::cos(pi * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, z, P, dP);
      double d2P = (2.0 * z * dP - p * (p + 1.0) * P) / (1.0 - z * z);
      double dz = dP / d2P;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
}

void vertex_shape(int etype, int dim, const double *xi, double *N, double *dN) {
  if (etype == TRI || etype == TET) {
    double s = 0.0;
    for (int a = 0; a < dim; ++a) s += xi[a];
    N[0] = 1.0 - s;
    for (int a = 0; a < dim; ++a) {
      N[a + 1] = xi[a];
      dN[0 * dim + a] = -1.0;
      for (int r = 0; r < dim; ++r) dN[(r + 1) * dim + a] = (r == a) ? 1.0 : 0.0;
    }
    return;
  }
  int nv = 1 << dim;
  for (int c = 0; c < nv; ++c) {
    double f[3], df[3];
    for (int a = 0; a < dim; ++a) {
      double sg = ((c >> a) & 1) ? 1.0 : -1.0;
      f[a] = 0.5 * (1.0 + sg * xi[a]);
      df[a] = 0.5 * sg;
    }
    double v = 1.0;
    for (int a = 0; a < dim; ++a) v *= f[a];
    N[c] = v;
    for (int a = 0; a < dim; ++a) {
      double g = df[a];
      for (int b = 0; b < dim; ++b)
        if (b != a) g *= f[b];
      dN[c * dim + a] = g;
    }
  }
}

void eval_basis(const RefTables &t, const double *x, int N, double *val, double *grad) {
  const int d = t.dim, Np = t.Np, p = t.p;
  if (t.etype == QUAD || t.etype == HEX) {
    std::vector<double> r(p + 1);
    gll_points(p, r.data());
    for (int n = 0; n < N; ++n) {
      std::vector<double> l(d * (p + 1)), dl(d * (p + 1));
      for (int a = 0; a < d; ++a)
        for (int i = 0; i <= p; ++i) lagrange1d(r.data(), p, i, x[n * d + a], l[a * (p + 1) + i], dl[a * (p + 1) + i]);
      for (int node = 0; node < Np; ++node) {
        double v = 1.0;
        for (int a = 0; a < d; ++a) v *= l[a * (p + 1) + t.mi[node * d + a]];
        val[n * Np + node] = v;
        for (int a = 0; a < d; ++a) {
          double g = 1.0;
          for (int b = 0; b < d; ++b) {
            int i = t.mi[node * d + b];
            g *= (b == a) ? dl[b * (p + 1) + i] : l[b * (p + 1) + i];
          }
          grad[(a * N + n) * Np + node] = g;
        }
      }
    }
    return;
  }
  for (int n = 0; n < N; ++n) {
    double lam[4];
    double s = 0.0;
    for (int a = 0; a < d; ++a) {
      lam[a + 1] = x[n * d + a];
      s += x[n * d + a];
    }
    lam[0] = 1.0 - s;
    for (int node = 0; node < Np; ++node) {
      int idx[4];
      int tot = 0;
      for (int a = 0; a < d; ++a) {
        idx[a + 1] = t.mi[node * d + a];
        tot += idx[a + 1];
      }
      idx[0] = p - tot;
      double R[4], dR[4];
      for (int r = 0; r <= d; ++r) silvester(idx[r], p, lam[r], R[r], dR[r]);
      double v = 1.0;
      for (int r = 0; r <= d; ++r) v *= R[r];
      val[n * Np + node] = v;
      // d phi / d lambda_r
      double dl[4];
      for (int r = 0; r <= d; ++r) {
        double g = dR[r];
        for (int q = 0; q <= d; ++q)
          if (q != r) g *= R[q];
        dl[r] = g;
      }
      for (int a = 0; a < d; ++a) grad[(a * N + n) * Np + node] = dl[a + 1] - dl[0];
    }
  }
}

std::string build_ref_tables(int etype, int p, RefTables &t) {
  if (etype < 0 || etype > 3) return "unknown element type";
  if (p < 1 || p > 4) return "polynomial order must be 1..4";
  t.etype = etype;
  t.p = p;
  t.dim = (etype == TRI || etype == QUAD) ? 2 : 3;
  const int d = t.dim;
  t.m = d + 2;
  t.Np = n_nodes(etype, p);
  t.nv = (etype == TRI) ? 3 : (etype == TET ? 4 : (1 << d));
  t.nf = (etype == TRI) ? 3 : (etype == TET ? 4 : 2 * d);
  const int nq1 = p + 2;
  // node multi-indices (see header for the order)
  t.mi.clear();
  if (etype == QUAD || etype == HEX) {
    if (d == 2) {
      for (int j = 0; j <= p; ++j)
        for (int i = 0; i <= p; ++i) { t.mi.push_back(i); t.mi.push_back(j); }
    } else {
      for (int k = 0; k <= p; ++k)
        for (int j = 0; j <= p; ++j)
          for (int i = 0; i <= p; ++i) { t.mi.push_back(i); t.mi.push_back(j); t.mi.push_back(k); }
    }
  } else if (d == 2) {
    for (int j = 0; j <= p; ++j)
      for (int i = 0; i <= p - j; ++i) { t.mi.push_back(i); t.mi.push_back(j); }
  } else {
    for (int k = 0; k <= p; ++k)
      for (int j = 0; j <= p - k; ++j)
        for (int i = 0; i <= p - j - k; ++i) { t.mi.push_back(i); t.mi.push_back(j); t.mi.push_back(k); }
  }
  // reference nodes and vertices
  t.nodes.assign(t.Np * d, 0.0);
  if (etype == QUAD || etype == HEX) {
    std::vector<double> r(p + 1);
    gll_points(p, r.data());
    for (int n = 0; n < t.Np; ++n)
      for (int a = 0; a < d; ++a) t.nodes[n * d + a] = r[t.mi[n * d + a]];
    t.vref.assign(t.nv * d, 0.0);
    for (int c = 0; c < t.nv; ++c)
      for (int a = 0; a < d; ++a) t.vref[c * d + a] = ((c >> a) & 1) ? 1.0 : -1.0;
  } else {
    for (int n = 0; n < t.Np; ++n)
      for (int a = 0; a < d; ++a) t.nodes[n * d + a] = double(t.mi[n * d + a]) / p;
    t.vref.assign(t.nv * d, 0.0);
    for (int a = 0; a < d; ++a) t.vref[(a + 1) * d + a] = 1.0;
  }
  // volume rule and basis
  if (etype == QUAD || etype == HEX) tensor_rule(d, nq1, t.xq, t.wq);
  else if (d == 2) tri_rule(nq1, t.xq, t.wq);
  else tet_rule(nq1, t.xq, t.wq);
  t.Nq = (int)t.wq.size();
  t.phi.assign(t.Nq * t.Np, 0.0);
  t.dphi.assign(d * t.Nq * t.Np, 0.0);
  eval_basis(t, t.xq.data(), t.Nq, t.phi.data(), t.dphi.data());
  // faces
  std::vector<double> fs, fws;   // face rule in d-1 dims
  if (etype == QUAD || etype == HEX) tensor_rule(d - 1, nq1, fs, fws);
  else if (d == 2) {
    std::vector<double> g(nq1), gw(nq1);
    gauss_legendre(nq1, g.data(), gw.data());
    for (int i = 0; i < nq1; ++i) { fs.push_back(0.5 * (g[i] + 1.0)); fws.push_back(0.5 * gw[i]); }
  } else tri_rule(nq1, fs, fws);
  t.Nfq = (int)fws.size();
  t.fnodes.clear();
  t.fxi.assign(t.nf * t.Nfq * d, 0.0);
  t.fw.assign(t.nf * t.Nfq, 0.0);
  t.fnref.assign(t.nf * d, 0.0);
  for (int f = 0; f < t.nf; ++f) {
    std::vector<int> fn;
    for (int n = 0; n < t.Np; ++n) {
      const int *mi = &t.mi[n * d];
      bool on = false;
      if (etype == QUAD || etype == HEX) {
        int ax = f / 2, side = f % 2;
        on = mi[ax] == (side ? p : 0);
      } else if (f == 0) {
        int s = 0;
        for (int a = 0; a < d; ++a) s += mi[a];
        on = (s == p);
      } else {
        on = (mi[f - 1] == 0);
      }
      if (on) fn.push_back(n);
    }
    if (f == 0) t.Nfp = (int)fn.size();
    if ((int)fn.size() != t.Nfp) return "inconsistent face node count";
    t.fnodes.insert(t.fnodes.end(), fn.begin(), fn.end());
    // parametrization xi = o + sum_r s_r T_r, area factor, reference normal
    double o[3] = {0, 0, 0}, T[3][2] = {{0, 0}, {0, 0}, {0, 0}}, area = 1.0;
    if (etype == QUAD || etype == HEX) {
      int ax = f / 2, side = f % 2;
      o[ax] = side ? 1.0 : -1.0;
      int r = 0;
      for (int a = 0; a < d; ++a)
        if (a != ax) T[a][r++] = 1.0;
      t.fnref[f * d + ax] = side ? 1.0 : -1.0;
    } else {
      int vs[3], nvs = 0;
      for (int r = 0; r <= d; ++r)
        if (r != f) vs[nvs++] = r;
      for (int a = 0; a < d; ++a) o[a] = t.vref[vs[0] * d + a];
      for (int r = 1; r < d; ++r)
        for (int a = 0; a < d; ++a) T[a][r - 1] = t.vref[vs[r] * d + a] - t.vref[vs[0] * d + a];
      if (d == 2) {
        area = std::sqrt(T[0][0] * T[0][0] + T[1][0] * T[1][0]);
      } else {
        double cx = T[1][0] * T[2][1] - T[2][0] * T[1][1];
        double cy = T[2][0] * T[0][1] - T[0][0] * T[2][1];
        double cz = T[0][0] * T[1][1] - T[1][0] * T[0][1];
        area = std::sqrt(cx * cx + cy * cy + cz * cz);
      }
      if (f == 0) {
        for (int a = 0; a < d; ++a) t.fnref[f * d + a] = 1.0 / std::sqrt((double)d);
      } else {
        t.fnref[f * d + (f - 1)] = -1.0;
      }
    }
    for (int q = 0; q < t.Nfq; ++q) {
      for (int a = 0; a < d; ++a) {
        double x = o[a];
        for (int r = 0; r < d - 1; ++r) x += T[a][r] * fs[q * (d - 1) + r];
        t.fxi[(f * t.Nfq + q) * d + a] = x;
      }
      t.fw[f * t.Nfq + q] = fws[q] * area;
    }
  }
  // face-node basis at the face points
  t.fphi.assign(t.nf * t.Nfq * t.Nfp, 0.0);
  std::vector<double> val(t.Nfq * t.Np), grad(d * t.Nfq * t.Np);
  for (int f = 0; f < t.nf; ++f) {
    eval_basis(t, &t.fxi[f * t.Nfq * d], t.Nfq, val.data(), grad.data());
    for (int q = 0; q < t.Nfq; ++q) {
      double off = 0.0;
      for (int n = 0; n < t.Np; ++n) {
        bool on = false;
        for (int b = 0; b < t.Nfp; ++b)
          if (t.fnodes[f * t.Nfp + b] == n) on = true;
        if (!on) off = std::fmax(off, std::fabs(val[q * t.Np + n]));
      }
      if (off > 1e-10) return "basis does not vanish off the face";
      for (int b = 0; b < t.Nfp; ++b) t.fphi[(f * t.Nfq + q) * t.Nfp + b] = val[q * t.Np + t.fnodes[f * t.Nfp + b]];
    }
  }
  return std::string();
}

}  // namespace hdg
