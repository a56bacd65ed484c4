// C ABI: plan creation, workspace binding and the entry points of hdg.h.
#include "hdg_plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>
#include <cstdio>
#include <cstring>

namespace {
thread_local std::string g_err;
}  // namespace

namespace hdg {

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return HDG_EHIP;
}

}  // namespace hdg

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int roundup(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

using namespace hdg;

extern "C" const char *hdg_last_error(void) { return g_err.c_str(); }

extern "C" int hdg_status(const hdg_plan *plan, const int32_t *elem_status, void *stream, int *first_bad_elem,
                          int *code) {
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  if (!P || !elem_status || !first_bad_elem || !code) return fail(HDG_EINVAL, "null argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<int32_t> h(P->n_elem);
  hipError_t e = hipMemcpyAsync(h.data(), elem_status, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "status copy");
  *first_bad_elem = -1;
  *code = HDG_OK;
  for (size_t i = 0; i < h.size(); ++i)
    if (h[i] != HDG_OK) {
      *first_bad_elem = (int)i;
      *code = h[i];
      break;
    }
  return HDG_OK;
}

extern "C" int hdg_plan_create(hdg_plan **out, const hdg_mesh *mesh, const hdg_phys *phys,
                               const hdg_opts *opts) {
  if (!out || !mesh || !phys) return fail(HDG_EINVAL, "null argument");
  *out = nullptr;
  if (mesh->n_elem <= 0 || !mesh->elem_xyz || !mesh->trace_map || mesh->n_trace <= 0)
    return fail(HDG_EINVAL, "mesh: n_elem, elem_xyz, trace_map and n_trace are required");
  if (mesh->order < 1 || mesh->order > 4) return fail(HDG_EUNSUPPORTED, "order must be 1..4");
  if (mesh->elem_type < 0 || mesh->elem_type > 3) return fail(HDG_EUNSUPPORTED, "unknown element type");
  if (!(phys->gamma > 1.0) || phys->mu < 0.0 || (phys->viscous && !(phys->Pr > 0.0)) || phys->alpha < 0.0)
    return fail(HDG_EINVAL, "physical parameters out of range");
  if (opts && opts->precision != HDG_FP64) return fail(HDG_EUNSUPPORTED, "only HDG_FP64 is built");

  Plan *P = new Plan();
  std::string err = build_ref_tables(mesh->elem_type, mesh->order, P->ref);
  if (!err.empty()) {
    delete P;
    return fail(HDG_EUNSUPPORTED, err);
  }
  const RefTables &R = P->ref;
  const int d = R.dim, E = mesh->n_elem, M = R.m;
  P->phys = *phys;
  P->n_elem = E;
  P->n_trace = mesh->n_trace;
  P->chunk = (opts && opts->chunk_elems > 0) ? std::min(opts->chunk_elems, E) : E;

  // trace map / face flags
  P->tmap.assign(mesh->trace_map, mesh->trace_map + (size_t)E * R.nf * R.Nfp);
  for (int t : P->tmap)
    if (t < 0 || t >= mesh->n_trace) {
      delete P;
      return fail(HDG_EINVAL, "trace_map entry out of range");
    }
  P->face_bc.assign((size_t)E * R.nf, 0);
  if (mesh->face_bc)
    for (size_t i = 0; i < P->face_bc.size(); ++i) P->face_bc[i] = mesh->face_bc[i] ? 1 : 0;
  // A continuous (EDG) trace node on a Dirichlet face keeps the Dirichlet condition alone: the
  // flux rows that other faces contribute at that node are dropped.
  {
    std::vector<char> dir_node(mesh->n_trace, 0);
    for (size_t ef = 0; ef < P->face_bc.size(); ++ef)
      if (P->face_bc[ef])
        for (int b = 0; b < R.Nfp; ++b) dir_node[P->tmap[ef * R.Nfp + b]] = 1;
    std::vector<int> drop(P->tmap.size(), 0);
    bool any = false;
    for (size_t ef = 0; ef < P->face_bc.size(); ++ef)
      if (!P->face_bc[ef])
        for (int b = 0; b < R.Nfp; ++b)
          if (dir_node[P->tmap[ef * R.Nfp + b]]) drop[ef * R.Nfp + b] = 1, any = true;
    if (any) P->row_drop.swap(drop);
  }
  P->node_face.assign(R.Np * R.nf, -1);
  for (int f = 0; f < R.nf; ++f)
    for (int b = 0; b < R.Nfp; ++b) P->node_face[R.fnodes[f * R.Nfp + b] * R.nf + f] = b;

  // geometry at quadrature points and node coordinates
  P->geo_vol.assign((size_t)E * R.Nq * (1 + d * d), 0.0);
  P->geo_face.assign((size_t)E * R.nf * R.Nfq * (1 + d), 0.0);
  P->node_x.assign((size_t)d * E * R.Np, 0.0);
  P->trace_x.assign((size_t)d * mesh->n_trace, 0.0);
  std::vector<double> Nv(R.nv), dNv(R.nv * d);
  for (int e = 0; e < E; ++e) {
    const double *X = mesh->elem_xyz + (size_t)e * R.nv * d;
    auto jac = [&](const double *xi, double J[3][3], double *x) {
      vertex_shape(R.etype, d, xi, Nv.data(), dNv.data());
      for (int i = 0; i < d; ++i) {
        if (x) x[i] = 0.0;
        for (int r = 0; r < d; ++r) J[i][r] = 0.0;
      }
      for (int v = 0; v < R.nv; ++v)
        for (int i = 0; i < d; ++i) {
          if (x) x[i] += Nv[v] * X[v * d + i];
          for (int r = 0; r < d; ++r) J[i][r] += dNv[v * d + r] * X[v * d + i];
        }
    };
    auto inv = [&](double J[3][3], double Ji[3][3]) -> double {
      if (d == 2) {
        double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Ji[0][0] = J[1][1] / det;
        Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det;
        Ji[1][1] = J[0][0] / det;
        return det;
      }
      double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
      Ji[0][0] = c00 / det;
      Ji[1][0] = c01 / det;
      Ji[2][0] = c02 / det;
      Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
      return det;
    };
    double J[3][3], Ji[3][3];
    for (int q = 0; q < R.Nq; ++q) {
      jac(&R.xq[q * d], J, nullptr);
      double det = inv(J, Ji);  // Ji[r][i] = dxi_r / dx_i
      if (!(det > 0.0)) {
        delete P;
        return fail(HDG_EINVAL, "element with non-positive Jacobian determinant");
      }
      double *g = &P->geo_vol[((size_t)e * R.Nq + q) * (1 + d * d)];
      g[0] = R.wq[q] * det;
      for (int r = 0; r < d; ++r)
        for (int j = 0; j < d; ++j) g[1 + r * d + j] = Ji[r][j];
    }
    for (int f = 0; f < R.nf; ++f)
      for (int q = 0; q < R.Nfq; ++q) {
        jac(&R.fxi[(f * R.Nfq + q) * d], J, nullptr);
        double det = inv(J, Ji);
        if (!(det > 0.0)) {
          delete P;
          return fail(HDG_EINVAL, "element with non-positive Jacobian determinant");
        }
        // Nanson: n dS = det J  J^-T n_ref dS_ref
        double a[3] = {0, 0, 0}, nrm = 0.0;
        for (int i = 0; i < d; ++i) {
          for (int r = 0; r < d; ++r) a[i] += Ji[r][i] * R.fnref[f * d + r];
          a[i] *= det;
          nrm += a[i] * a[i];
        }
        nrm = std::sqrt(nrm);
        double *g = &P->geo_face[(((size_t)e * R.nf + f) * R.Nfq + q) * (1 + d)];
        g[0] = R.fw[f * R.Nfq + q] * nrm;
        for (int i = 0; i < d; ++i) g[1 + i] = a[i] / nrm;
      }
    for (int a = 0; a < R.Np; ++a) {
      double x[3];
      jac(&R.nodes[a * d], J, x);
      for (int i = 0; i < d; ++i) P->node_x[(size_t)i * E * R.Np + (size_t)e * R.Np + a] = x[i];
    }
    for (int f = 0; f < R.nf; ++f)
      for (int b = 0; b < R.Nfp; ++b) {
        int a = R.fnodes[f * R.Nfp + b];
        int t = P->tmap[((size_t)e * R.nf + f) * R.Nfp + b];
        for (int i = 0; i < d; ++i)
          P->trace_x[(size_t)i * mesh->n_trace + t] = P->node_x[(size_t)i * E * R.Np + (size_t)e * R.Np + a];
      }
  }

  // block-Jacobi structure: one block per face when every trace node lies on
  // exactly one face (HDG), otherwise one m x m block per trace node
  {
    std::map<std::vector<int>, int> keys;
    std::vector<std::vector<int>> nodes_of;
    std::vector<std::vector<std::pair<int, int>>> contrib;
    std::vector<int> owner(mesh->n_trace, -1);
    bool face_ok = true;
    for (int e = 0; e < E && face_ok; ++e)
      for (int f = 0; f < R.nf && face_ok; ++f) {
        std::vector<int> key(&P->tmap[((size_t)e * R.nf + f) * R.Nfp], &P->tmap[((size_t)e * R.nf + f) * R.Nfp] + R.Nfp);
        std::sort(key.begin(), key.end());
        if (std::adjacent_find(key.begin(), key.end()) != key.end()) face_ok = false;
        auto it = keys.find(key);
        int id;
        if (it == keys.end()) {
          id = (int)nodes_of.size();
          keys[key] = id;
          nodes_of.push_back(key);
          contrib.emplace_back();
          for (int t : key) {
            if (owner[t] >= 0) face_ok = false;
            owner[t] = id;
          }
        } else {
          id = it->second;
        }
        contrib[id].push_back({e, f});
        if (contrib[id].size() > 2) face_ok = false;
      }
    for (int t = 0; t < mesh->n_trace && face_ok; ++t)
      if (owner[t] < 0) face_ok = false;
    P->dp.bj_face = face_ok ? 1 : 0;
    P->bj_tpos.assign(mesh->n_trace, 0);
    if (face_ok) {
      const int nb = (int)nodes_of.size();
      P->dp.bj_nblk = nb;
      P->dp.bj_bs = M * R.Nfp;
      P->bj_nodes.resize((size_t)nb * R.Nfp);
      P->bj_ce.assign((size_t)nb * 2, -1);
      P->bj_cf.assign((size_t)nb * 2, -1);
      P->bj_loc.assign((size_t)nb * 2 * R.Nfp, 0);
      for (int b = 0; b < nb; ++b) {
        for (int p = 0; p < R.Nfp; ++p) {
          P->bj_nodes[(size_t)b * R.Nfp + p] = nodes_of[b][p];
          P->bj_tpos[nodes_of[b][p]] = b * R.Nfp + p;
        }
        for (size_t q = 0; q < contrib[b].size(); ++q) {
          const int e = contrib[b][q].first, f = contrib[b][q].second;
          P->bj_ce[b * 2 + q] = e;
          P->bj_cf[b * 2 + q] = f;
          for (int p = 0; p < R.Nfp; ++p)
            for (int bb = 0; bb < R.Nfp; ++bb)
              if (P->tmap[((size_t)e * R.nf + f) * R.Nfp + bb] == nodes_of[b][p])
                P->bj_loc[((size_t)b * 2 + q) * R.Nfp + p] = bb;
        }
      }
    } else {
      P->dp.bj_nblk = mesh->n_trace;
      P->dp.bj_bs = M;
      P->bj_nodes.resize(mesh->n_trace);
      for (int t = 0; t < mesh->n_trace; ++t) P->bj_nodes[t] = P->bj_tpos[t] = t;
      P->bj_ce.assign(2, -1);
      P->bj_cf.assign(2, -1);
      P->bj_loc.assign(2, 0);
    }
  }

  // descriptor
  DevPlan &D = P->dp;
  D.dim = d;
  D.m = M;
  D.Np = R.Np;
  D.nf = R.nf;
  D.Nfp = R.Nfp;
  D.Nq = R.Nq;
  D.Nfq = R.Nfq;
  D.viscous = phys->viscous ? 1 : 0;
  D.n = M * R.Np * (D.viscous ? (1 + d) : 1);
  D.k = R.nf * M * R.Nfp;
  D.n_pad = roundup(D.n, 32);
  D.k_pad = roundup(D.k, 16);
  D.kx = roundup(D.k_pad + 1, 32);
  D.n_elem = E;
  D.n_trace = mesh->n_trace;
  D.gamma = phys->gamma;
  D.mu = phys->mu;
  D.Pr = phys->Pr;
  D.alpha = phys->alpha;
  // fused left-looking condensation when its 32- or 16-column LDS block fits
  D.cw = condense_width(D.n_pad, false);
  D.cw_lp = condense_width(D.n_pad, true);
  if (opts && (opts->flags & HDG_FLAG_NARROW_BLOCK)) {
    if (D.cw) D.cw = 16;
    if (D.cw_lp) D.cw_lp = 16;
  }
  D.contract_threads = 1024;
  D.zero_xcd = 1;
  D.src = nullptr;
  D.src_qp = 0;
  D.row_drop = nullptr;
  D.ghat_v = (opts && (opts->flags & HDG_FLAG_GHAT_INTERIOR)) ? 1 : 0;
  D.ghat_proj = (opts && (opts->flags & HDG_FLAG_GHAT_PROJ)) ? 1 : 0;
  D.gp = D.gz = nullptr;
  if (D.ghat_proj && (!D.viscous || gproj_lift_lds(D) > 64 * 1024)) {
    delete P;
    return fail(D.viscous ? HDG_EUNSUPPORTED : HDG_EINVAL,
                "projection viscous flux: Navier-Stokes only, element mass inverse and lift within 64 KB of LDS");
  }
  D.sigma_s = (opts && (opts->flags & HDG_FLAG_SIGMA_MV)) ? 2 : (opts && (opts->flags & HDG_FLAG_SIGMA_S)) ? 1 : 0;
  D.a_qmin = 0;
  D.condense_launches = 2;
  D.lu_waves = default_lu_waves(D.n_pad);
  D.lu_waves_set = 0;
  D.lp_bf16 = 0;
  P->fused = D.cw != 0;
  if (opts && (opts->flags & HDG_FLAG_SPLIT_DENSE)) P->fused = false;
  P->split_ok = lu_lds_bytes(D.n_pad) <= 160 * 1024;
  if (!P->fused && !P->split_ok && !D.cw_lp) {
    delete P;
    return fail(HDG_EUNSUPPORTED, "local block too large for every condensation kernel");
  }
  PointLayout &L = D.L;
  int o = 0;
  L.Mv = o; o += M * M;
  L.Kv = o; o += M * d * M;
  L.Kq = o; o += D.viscous ? M * d * M * d : 0;
  L.Fr = o; o += M * d;
  L.Wu = o; o += M;
  L.Wq = o; o += D.viscous ? M * d : 0;
  L.v = o; o += M;
  L.WJ = o; o += d * d;
  L.W = o; o += 1;
  L.size = o;
  o = 0;
  L.fFv = o; o += M * M;
  L.fFq = o; o += D.viscous ? M * M * d : 0;
  L.fFh = o; o += M * M;
  L.fFf = o; o += M;
  L.fWn = o; o += d;
  L.fvh = o; o += M;
  L.fFd = o; o += M;
  L.fW = o; o += 1;
  L.fsize = o;
  P->contract_mfma = contract_mfma_supported(D) && !(opts && (opts->flags & HDG_FLAG_SPLIT_DENSE));
  if (D.viscous && P->contract_mfma) {
    // local unknown x: v (c, a) at c Np + a, q (c, j, a) at m Np + (c d + j) Np + a, padding beyond n
    P->uinfo.assign(D.n_pad, 0);
    const int nv = D.m * D.Np;
    for (int x = 0; x < D.n; ++x) {
      const int c = x < nv ? x / D.Np : (x - nv) / (D.dim * D.Np);
      const int j = x < nv ? 0 : ((x - nv) / D.Np) % D.dim;
      P->uinfo[x] = x % D.Np | j << 8 | c << 12;
    }
  }
  if (opts && (opts->flags & HDG_FLAG_ELIMINATE_Q)) {
    const int nv = D.m * D.Np;
    P->qa.nr_pad = roundup(nv, 32);
    if (!D.viscous) {
      delete P;
      return fail(HDG_EINVAL, "HDG_FLAG_ELIMINATE_Q needs a Navier-Stokes plan (gradient unknowns)");
    }
    if (qelim_lds_bytes(D) > 160 * 1024 || D.Np + D.nf * D.Nfp + 1 > 112 || !condense_width(P->qa.nr_pad, false) ||
        !P->fused) {
      delete P;
      return fail(HDG_EUNSUPPORTED, "q elimination: element too large for its LDS working sets");
    }
    P->qelim = true;
  }
  *out = reinterpret_cast<hdg_plan *>(P);
  return HDG_OK;
}

extern "C" int hdg_plan_set_phys(hdg_plan *plan, const hdg_phys *phys) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !phys) return fail(HDG_EINVAL, "null argument");
  if ((phys->viscous != 0) != (P->dp.viscous != 0)) return fail(HDG_EINVAL, "viscous flag cannot change");
  if (!(phys->gamma > 1.0) || phys->mu < 0.0 || (phys->viscous && !(phys->Pr > 0.0)) || phys->alpha < 0.0)
    return fail(HDG_EINVAL, "physical parameters out of range");
  P->phys = *phys;
  P->dp.gamma = phys->gamma;
  P->dp.mu = phys->mu;
  P->dp.Pr = phys->Pr;
  P->dp.alpha = phys->alpha;
  return HDG_OK;
}

extern "C" int hdg_plan_set_source(hdg_plan *plan, const double *src) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P) return fail(HDG_EINVAL, "null plan");
  P->dp.src = src;
  P->dp.src_qp = 0;
  return HDG_OK;
}

extern "C" int hdg_plan_set_source_points(hdg_plan *plan, const double *src) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P) return fail(HDG_EINVAL, "null plan");
  P->dp.src = src;
  P->dp.src_qp = src ? 1 : 0;
  return HDG_OK;
}

extern "C" int hdg_quad_coords(const hdg_plan *plan, double *xq, void *stream) {
  const Plan *P = checked(const_cast<hdg_plan *>(plan));
  if (!P) return HDG_EINVAL;
  if (!xq) return fail(HDG_EINVAL, "null argument");
  hipError_t e = launch_quad_coords(P->dp, xq, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "quad_coords");
  return HDG_OK;
}

extern "C" int hdg_l2_error(const hdg_plan *plan, int kind, const double *f, const double *exact, double *out,
                            void *stream) {
  const Plan *P = checked(const_cast<hdg_plan *>(plan));
  if (!P) return HDG_EINVAL;
  if (!f || !exact || !out || kind < 0 || kind > 3 || (kind >= 1 && kind != 2 && !P->dp.viscous))
    return fail(HDG_EINVAL, "bad argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = kind == 3 ? launch_l2_error_visc(P->dp, f, exact, out, s) : launch_l2_error(P->dp, kind, f, exact, out, s);
  if (e) return hip_fail(e, "l2_error");
  return HDG_OK;
}

extern "C" int hdg_face_quad_coords(const hdg_plan *plan, double *xf, void *stream) {
  const Plan *P = checked(const_cast<hdg_plan *>(plan));
  if (!P) return HDG_EINVAL;
  if (!xf) return fail(HDG_EINVAL, "null argument");
  hipError_t e = launch_face_quad_coords(P->dp, xf, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "face_quad_coords");
  return HDG_OK;
}

extern "C" int hdg_trace_project(const hdg_plan *plan, const double *g, double *vbc, void *stream) {
  const Plan *P = checked(const_cast<hdg_plan *>(plan));
  if (!P) return HDG_EINVAL;
  if (!g || !vbc) return fail(HDG_EINVAL, "null argument");
  // every trace node of a Dirichlet face must belong to that face alone
  const int nf = P->dp.nf, Nfp = P->dp.Nfp;
  std::vector<char> seen(P->n_trace, 0);
  for (int ef = 0; ef < P->n_elem * nf; ++ef) {
    if (P->face_bc[ef] != 1) continue;
    for (int b = 0; b < Nfp; ++b) {
      const int t = P->tmap[(size_t)ef * Nfp + b];
      if (seen[t]) return fail(HDG_EUNSUPPORTED, "trace node shared by two Dirichlet faces (continuous trace)");
      seen[t] = 1;
    }
  }
  hipError_t e = launch_trace_project(P->dp, g, vbc, reinterpret_cast<hipStream_t>(stream));
  if (e == hipErrorInvalidValue) return fail(HDG_EUNSUPPORTED, "face too large for the projection kernel");
  if (e) return hip_fail(e, "trace_project");
  return HDG_OK;
}

extern "C" int hdg_entropy_integral(const hdg_plan *plan, const double *v, double *out, void *stream) {
  const Plan *P = checked(const_cast<hdg_plan *>(plan));
  if (!P) return HDG_EINVAL;
  if (!v || !out) return fail(HDG_EINVAL, "null argument");
  hipError_t e = launch_entropy(P->dp, v, out, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "entropy_integral");
  return HDG_OK;
}

extern "C" int hdg_flow_statistics(const hdg_plan *plan, const double *v, double *out, void *stream) {
  const Plan *P = checked(const_cast<hdg_plan *>(plan));
  if (!P) return HDG_EINVAL;
  if (!v || !out) return fail(HDG_EINVAL, "null argument");
  hipError_t e = launch_flow_stats(P->dp, v, out, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "flow_statistics");
  return HDG_OK;
}

extern "C" void hdg_plan_destroy(hdg_plan *plan) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P) return;
  for (int i = 0; i < PH_COUNT; ++i)
    for (int j = 0; j < 2; ++j)
      if (P->ev[i][j]) (void)hipEventDestroy(P->ev[i][j]);
  delete P;
}

extern "C" int hdg_plan_set_timing(hdg_plan *plan, int enable) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P) return fail(HDG_EINVAL, "null plan");
  P->timing = enable != 0;
  for (int i = 0; i < PH_COUNT; ++i) {
    P->phase_ms[i] = 0.0;
    P->phase_calls[i] = 0;
    P->ev_pending[i] = false;
  }
  return HDG_OK;
}

extern "C" int hdg_plan_phase_times(hdg_plan *plan, double *ms, long *calls, int n) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !ms || n < PH_COUNT) return fail(HDG_EINVAL, "null argument or n < phase count");
  for (int i = 0; i < PH_COUNT; ++i) {
    if (P->ev_pending[i]) {
      hipError_t e = hipEventSynchronize(P->ev[i][1]);
      float t = 0.f;
      if (!e) e = hipEventElapsedTime(&t, P->ev[i][0], P->ev[i][1]);
      if (e) return hip_fail(e, "phase_times");
      P->phase_ms[i] += t;
      P->phase_calls[i] += 1;
      P->ev_pending[i] = false;
    }
    ms[i] = P->phase_ms[i];
    if (calls) calls[i] = P->phase_calls[i];
  }
  return HDG_OK;
}

extern "C" int hdg_plan_dims(const hdg_plan *plan, hdg_dims *o) {
  if (!plan || !o) return fail(HDG_EINVAL, "null argument");
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  const DevPlan &D = P->dp;
  o->dim = D.dim; o->m = D.m; o->Np = D.Np; o->nf = D.nf; o->Nfp = D.Nfp; o->Nq = D.Nq; o->Nfq = D.Nfq;
  o->n = D.n; o->k = D.k; o->n_pad = D.n_pad; o->k_pad = D.k_pad;
  o->n_elem = P->n_elem; o->n_trace = P->n_trace; o->chunk_elems = P->chunk;
  return HDG_OK;
}

namespace {

struct Layout {
  size_t phi, dphi, fphi, fnodes, node_face, geo_vol, geo_face, tmap, face_bc, node_x, trace_x;
  size_t bj_nodes, bj_ce, bj_cf, bj_loc, bj_tpos, uinfo, row_drop, tables_end;
  size_t pv, pf, A, X, C, D, Rt, ipiv, inv, mg, gp, gz;
  size_t rA, rX, rC, rD, rRt, rMH, rYv, rzv, ripiv, rinv, total;
};

Layout layout(const Plan *P) {
  const RefTables &R = P->ref;
  const DevPlan &D = P->dp;
  const size_t E = P->n_elem, ch = P->chunk;
  Layout l{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  l.phi = take(R.phi.size() * 8);
  l.dphi = take(R.dphi.size() * 8);
  l.fphi = take(R.fphi.size() * 8);
  l.fnodes = take(R.fnodes.size() * 4);
  l.node_face = take(P->node_face.size() * 4);
  l.geo_vol = take(P->geo_vol.size() * 8);
  l.geo_face = take(P->geo_face.size() * 8);
  l.tmap = take(P->tmap.size() * 4);
  l.face_bc = take(E * R.nf * 4);
  l.node_x = take(P->node_x.size() * 8);
  l.trace_x = take(P->trace_x.size() * 8);
  l.bj_nodes = take(P->bj_nodes.size() * 4);
  l.bj_ce = take(P->bj_ce.size() * 4);
  l.bj_cf = take(P->bj_cf.size() * 4);
  l.bj_loc = take(P->bj_loc.size() * 4);
  l.bj_tpos = take(P->bj_tpos.size() * 4);
  l.uinfo = take(P->uinfo.size() * 4);
  l.row_drop = take(P->row_drop.size() * 4);
  l.tables_end = o;
  l.pv = take(ch * D.Nq * D.L.size * 8);
  l.pf = take(ch * D.nf * D.Nfq * D.L.fsize * 8);
  l.A = take(ch * (size_t)D.n_pad * D.n_pad * 8);
  l.X = take(ch * (size_t)D.kx * D.n_pad * 8);
  l.C = take(ch * (size_t)D.n_pad * D.k_pad * 8);
  l.D = take(ch * (size_t)D.k_pad * D.k_pad * 8);
  l.Rt = take(ch * (size_t)D.k_pad * 8);
  l.ipiv = take(ch * (size_t)D.n_pad * 4);
  l.inv = take(P->fused ? ch * condense_inv_doubles(D.n_pad) * 8 : 0);
  l.mg = take(P->uinfo.empty() ? 0 : ch * (size_t)(1 + D.dim) * D.Np * D.Np * 8);
  {
    const size_t MD = (size_t)D.m * D.dim;
    l.gp = take(D.ghat_proj ? ch * D.Nq * (MD + MD * D.m + MD * MD) * 8 : 0);
    l.gz = take(D.ghat_proj ? ch * (size_t)D.nf * D.dim * D.Nfp * D.Nq * 8 : 0);
  }
  if (P->qelim) {
    const size_t nr = P->qa.nr_pad, nv = (size_t)D.m * D.Np;
    l.rA = take(ch * nr * nr * 8);
    l.rX = take(ch * (size_t)D.kx * nr * 8);
    l.rC = take(ch * nr * D.k_pad * 8);
    l.rD = take(ch * (size_t)D.k_pad * D.k_pad * 8);
    l.rRt = take(ch * (size_t)D.k_pad * 8);
    l.rMH = take(ch * (size_t)(1 + D.dim) * D.Np * D.Np * 8);
    l.rYv = take(ch * (size_t)D.k * nv * 8);
    l.rzv = take(ch * nv * 8);
    l.ripiv = take(ch * nr * 4);
    l.rinv = take(ch * condense_inv_doubles((int)nr) * 8);
  }
  l.total = o;
  return l;
}

}  // namespace

namespace hdg {

hipError_t set_dyn_lds(const void *kernel, size_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void *>, size_t> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e) return e;
  std::lock_guard<std::mutex> lock(mu);
  size_t &have = done[{dev, kernel}];
  if (bytes <= have) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (!e) have = bytes;
  return e;
}

Plan *checked(hdg_plan *plan) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P) {
    g_err = "null plan";
    return nullptr;
  }
  if (!P->bound) {
    g_err = "workspace not bound";
    return nullptr;
  }
  return P;
}

}  // namespace hdg

namespace {

}  // namespace

extern "C" int hdg_plan_workspace_bytes(const hdg_plan *plan, size_t *bytes) {
  if (!plan || !bytes) return fail(HDG_EINVAL, "null argument");
  *bytes = layout(reinterpret_cast<const Plan *>(plan)).total;
  return HDG_OK;
}

extern "C" int hdg_plan_bind_workspace(hdg_plan *plan, void *dev, size_t bytes, void *stream) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !dev) return fail(HDG_EINVAL, "null argument");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(HDG_EINVAL, "workspace must be 256-byte aligned");
  Layout l = layout(P);
  if (bytes < l.total) return fail(HDG_ENOMEM, "workspace smaller than hdg_plan_workspace_bytes");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(dev);
  const RefTables &R = P->ref;
  auto up = [&](size_t off, const void *src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, s);
  };
  hipError_t e = hipSuccess;
  if (!e) e = up(l.phi, R.phi.data(), R.phi.size() * 8);
  if (!e) e = up(l.dphi, R.dphi.data(), R.dphi.size() * 8);
  if (!e) e = up(l.fphi, R.fphi.data(), R.fphi.size() * 8);
  if (!e) e = up(l.fnodes, R.fnodes.data(), R.fnodes.size() * 4);
  if (!e) e = up(l.node_face, P->node_face.data(), P->node_face.size() * 4);
  if (!e) e = up(l.geo_vol, P->geo_vol.data(), P->geo_vol.size() * 8);
  if (!e) e = up(l.geo_face, P->geo_face.data(), P->geo_face.size() * 8);
  if (!e) e = up(l.tmap, P->tmap.data(), P->tmap.size() * 4);
  if (!e) e = up(l.face_bc, P->face_bc.data(), P->face_bc.size() * 4);
  if (!e) e = up(l.node_x, P->node_x.data(), P->node_x.size() * 8);
  if (!e) e = up(l.trace_x, P->trace_x.data(), P->trace_x.size() * 8);
  if (!e) e = up(l.bj_nodes, P->bj_nodes.data(), P->bj_nodes.size() * 4);
  if (!e) e = up(l.bj_ce, P->bj_ce.data(), P->bj_ce.size() * 4);
  if (!e) e = up(l.bj_cf, P->bj_cf.data(), P->bj_cf.size() * 4);
  if (!e) e = up(l.bj_loc, P->bj_loc.data(), P->bj_loc.size() * 4);
  if (!e) e = up(l.bj_tpos, P->bj_tpos.data(), P->bj_tpos.size() * 4);
  if (!e) e = up(l.uinfo, P->uinfo.data(), P->uinfo.size() * 4);
  if (!e) e = up(l.row_drop, P->row_drop.data(), P->row_drop.size() * 4);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "bind_workspace upload");
  P->xcd_clean = false;
  DevPlan &D = P->dp;
  D.phi = reinterpret_cast<const double *>(base + l.phi);
  D.dphi = reinterpret_cast<const double *>(base + l.dphi);
  D.fphi = reinterpret_cast<const double *>(base + l.fphi);
  D.fnodes = reinterpret_cast<const int *>(base + l.fnodes);
  D.node_face = reinterpret_cast<const int *>(base + l.node_face);
  D.geo_vol = reinterpret_cast<const double *>(base + l.geo_vol);
  D.geo_face = reinterpret_cast<const double *>(base + l.geo_face);
  D.tmap = reinterpret_cast<const int *>(base + l.tmap);
  D.face_bc = reinterpret_cast<const int *>(base + l.face_bc);
  D.node_x = reinterpret_cast<const double *>(base + l.node_x);
  D.trace_x = reinterpret_cast<const double *>(base + l.trace_x);
  D.bj_nodes = reinterpret_cast<const int *>(base + l.bj_nodes);
  D.bj_ce = reinterpret_cast<const int *>(base + l.bj_ce);
  D.bj_cf = reinterpret_cast<const int *>(base + l.bj_cf);
  D.bj_loc = reinterpret_cast<const int *>(base + l.bj_loc);
  D.bj_tpos = reinterpret_cast<const int *>(base + l.bj_tpos);
  D.pv = reinterpret_cast<double *>(base + l.pv);
  D.pf = reinterpret_cast<double *>(base + l.pf);
  D.A = reinterpret_cast<double *>(base + l.A);
  D.X = reinterpret_cast<double *>(base + l.X);
  D.C = reinterpret_cast<double *>(base + l.C);
  D.D = reinterpret_cast<double *>(base + l.D);
  D.Rt = reinterpret_cast<double *>(base + l.Rt);
  D.ipiv = reinterpret_cast<int *>(base + l.ipiv);
  D.inv = reinterpret_cast<double *>(base + l.inv);
  D.mg = P->uinfo.empty() ? nullptr : reinterpret_cast<double *>(base + l.mg);
  D.gp = D.ghat_proj ? reinterpret_cast<double *>(base + l.gp) : nullptr;
  D.gz = D.ghat_proj ? reinterpret_cast<double *>(base + l.gz) : nullptr;
  D.uinfo = P->uinfo.empty() ? nullptr : reinterpret_cast<const int *>(base + l.uinfo);
  D.row_drop = P->row_drop.empty() ? nullptr : reinterpret_cast<const int *>(base + l.row_drop);
  if (P->qelim) {
    QElimArgs &Q = P->qa;
    Q.A = reinterpret_cast<double *>(base + l.rA);
    Q.X = reinterpret_cast<double *>(base + l.rX);
    Q.C = reinterpret_cast<double *>(base + l.rC);
    Q.D = reinterpret_cast<double *>(base + l.rD);
    Q.Rt = reinterpret_cast<double *>(base + l.rRt);
    Q.MH = reinterpret_cast<double *>(base + l.rMH);
    Q.Yv = reinterpret_cast<double *>(base + l.rYv);
    Q.zv = reinterpret_cast<double *>(base + l.rzv);
    P->rp.ipiv = reinterpret_cast<int *>(base + l.ripiv);
    P->rp.inv = reinterpret_cast<double *>(base + l.rinv);
  }
  P->ws = dev;
  P->ws_bytes = bytes;
  P->bound = true;
  return HDG_OK;
}

extern "C" int hdg_node_coords(const hdg_plan *plan, double *x, double *xt, void *stream) {
  const Plan *P = checked(const_cast<hdg_plan *>(plan));
  if (!P) return HDG_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (x) e = hipMemcpyAsync(x, P->dp.node_x, P->node_x.size() * 8, hipMemcpyDeviceToDevice, s);
  if (!e && xt) e = hipMemcpyAsync(xt, P->dp.trace_x, P->trace_x.size() * 8, hipMemcpyDeviceToDevice, s);
  if (e) return hip_fail(e, "node_coords");
  return HDG_OK;
}

extern "C" int hdg_prepare_state(const hdg_plan *plan, int N, const double *prim, const double *grad,
                                 double *v, double *q, double *u, void *stream) {
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  if (!P || !prim || !v || N < 0) return fail(HDG_EINVAL, "null argument");
  if (q && !grad) return fail(HDG_EINVAL, "q requested without gradients");
  hipError_t e = launch_prepare_state(P->dp, N, prim, grad, v, q, u, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "prepare_state");
  return HDG_OK;
}

namespace hdg {

// Accumulate the elapsed time of the previous launch of a phase (events are
// reused, so the previous interval is read before recording a new one).
hipError_t phase_begin(Plan *P, int ph, hipStream_t s) {
  if (!P->timing) return hipSuccess;
  hipError_t e = hipSuccess;
  if (!P->ev[ph][0]) {
    e = hipEventCreate(&P->ev[ph][0]);
    if (!e) e = hipEventCreate(&P->ev[ph][1]);
    if (e) return e;
  }
  if (P->ev_pending[ph]) {
    e = hipEventSynchronize(P->ev[ph][1]);
    float ms = 0.f;
    if (!e) e = hipEventElapsedTime(&ms, P->ev[ph][0], P->ev[ph][1]);
    if (e) return e;
    P->phase_ms[ph] += ms;
    P->phase_calls[ph] += 1;
    P->ev_pending[ph] = false;
  }
  return hipEventRecord(P->ev[ph][0], s);
}

hipError_t phase_end(Plan *P, int ph, hipStream_t s) {
  if (!P->timing) return hipSuccess;
  P->ev_pending[ph] = true;
  return hipEventRecord(P->ev[ph][1], s);
}

int run_front(Plan *P, const double *v, const double *q, const double *vhat, const double *ustar,
              const double *vbc, int32_t *status, int e0, int ec, hipStream_t s, bool q_only) {
  P->dp.a_qmin = q_only ? 1 : 0;
  hipError_t e = phase_begin(P, PH_POINTS, s);
  if (!e) e = launch_points(P->dp, e0, ec, v, q, vhat, ustar, vbc, status, s);
  if (!e) e = phase_end(P, PH_POINTS, s);
  if (!e) e = phase_begin(P, PH_CONTRACT, s);
  // With one chunk every element keeps its workspace slot, so the zeros of X, C and D
  // (a fixed pattern per element: face nodes and face boundary types do not change)
  // survive from the previous call; only the split solve overwrites X.
  const bool one_chunk = P->chunk >= P->n_elem;
  P->dp.zero_xcd = (one_chunk && P->xcd_clean) ? 0 : 1;
  if (!e) e = P->contract_mfma ? launch_contract_mfma(P->dp, e0, ec, s) : launch_contract(P->dp, e0, ec, s);
  if (!e && P->dp.ghat_proj) e = launch_gproj(P->dp, e0, ec, v, q, s);
  if (!e && P->dp.row_drop) e = launch_drop_rows(P->dp, e0, ec, s);
  if (!e) e = phase_end(P, PH_CONTRACT, s);
  if (e) {
    P->xcd_clean = false;
    return hip_fail(e, "assemble");
  }
  // the projection terms fill entries of C outside the contraction's pattern: clear every call
  P->xcd_clean = one_chunk && !P->dp.ghat_proj;
  return HDG_OK;
}

// FP64 condensation of one chunk with descriptor Dp (the plan's, or the reduced one of the q
// elimination); outputs indexed from element e0 of Dp's numbering
hipError_t condense_chunk(Plan *P, const DevPlan &Dp, int e0, int ec, int32_t *status, double *S, double *g,
                          double *Y, double *z, hipStream_t s) {
  if (!condense_two_launches(Dp)) return launch_condense(Dp, e0, ec, status, S, g, Y, z, s);
  hipError_t e = phase_begin(P, PH_CONDENSE_LU, s);
  if (!e) e = launch_condense_lu(Dp, e0, ec, status, s);
  if (!e) e = phase_end(P, PH_CONDENSE_LU, s);
  if (!e) e = phase_begin(P, PH_CONDENSE_RHS, s);
  if (!e) e = launch_condense_rhs(Dp, e0, ec, S, g, Y, z, s);
  if (!e) e = phase_end(P, PH_CONDENSE_RHS, s);
  return e;
}

int check_inputs(const Plan *P, const double *v, const double *q, const double *vhat,
                 const double *ustar, int32_t *status) {
  if (!v || !vhat || !status) return fail(HDG_EINVAL, "v, vhat and elem_status are required");
  if (P->dp.viscous && !q) return fail(HDG_EINVAL, "q is required for Navier-Stokes");
  (void)ustar;
  return HDG_OK;
}

}  // namespace hdg

extern "C" int hdg_assemble(hdg_plan *plan, const double *v, const double *q, const double *vhat,
                            const double *ustar, const double *vbc, double *A, double *B, double *C,
                            double *D, double *Rloc, double *Rtr, int32_t *status, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  int rc = check_inputs(P, v, q, vhat, ustar, status);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_fill_int(status, P->n_elem, HDG_OK, s);
  if (e) return hip_fail(e, "status init");
  for (int e0 = 0; e0 < P->n_elem; e0 += P->chunk) {
    int ec = std::min(P->chunk, P->n_elem - e0);
    rc = run_front(P, v, q, vhat, ustar, vbc, status, e0, ec, s);
    if (rc) return rc;
    e = launch_export_blocks(P->dp, e0, ec, A, B, C, D, Rloc, Rtr, s);
    if (e) return hip_fail(e, "export");
  }
  return HDG_OK;
}

extern "C" int hdg_condense_blocks(hdg_plan *plan, const double *A, const double *B, const double *C,
                                   const double *D, const double *Rloc, const double *Rtr, double *S, double *g,
                                   double *Y, double *z, int32_t *status, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!A || !B || !C || !D || !Rloc || !Rtr || !S || !g || !Y || !z || !status)
    return fail(HDG_EINVAL, "every block, output and elem_status is required");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_fill_int(status, P->n_elem, HDG_OK, s);
  if (e) return hip_fail(e, "status init");
  DevPlan Dp = P->dp;
  Dp.mg = nullptr;       // A is stored whole
  Dp.uinfo = nullptr;
  P->xcd_clean = false;  // X, C and D now hold the caller's blocks
  for (int e0 = 0; e0 < P->n_elem; e0 += P->chunk) {
    const int ec = std::min(P->chunk, P->n_elem - e0);
    e = launch_import_blocks(Dp, e0, ec, A, B, C, D, Rloc, Rtr, s);
    if (!e && P->fused) {
      e = condense_chunk(P, Dp, e0, ec, status + e0, S, g, Y, z, s);
    } else if (!e) {
      e = launch_lu(Dp, ec, status + e0, s);
      if (!e) e = launch_solve(Dp, ec, s);
      if (!e) e = launch_schur(Dp, e0, ec, S, g, Y, z, nullptr, nullptr, s);
    }
    if (e) return hip_fail(e, "condense_blocks");
  }
  return HDG_OK;
}

extern "C" int hdg_assemble_condense(hdg_plan *plan, const double *v, const double *q,
                                     const double *vhat, const double *ustar, const double *vbc,
                                     double *S, double *g, double *Y, double *z, double *Rloc,
                                     double *Rtr, int32_t *status, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  int rc = check_inputs(P, v, q, vhat, ustar, status);
  if (rc) return rc;
  if (!S || !g || !Y || !z) return fail(HDG_EINVAL, "S, g, Y and z are required");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_fill_int(status, P->n_elem, HDG_OK, s);
  if (e) return hip_fail(e, "status init");
  for (int e0 = 0; e0 < P->n_elem; e0 += P->chunk) {
    int ec = std::min(P->chunk, P->n_elem - e0);
    rc = run_front(P, v, q, vhat, ustar, vbc, status, e0, ec, s, (P->qelim || P->dp.mg) && P->fused);
    if (rc) return rc;
    e = launch_copy_resid(P->dp, e0, ec, Rloc, Rtr, s);
    if (!e && !P->fused && !P->split_ok) return fail(HDG_EUNSUPPORTED, "FP64 condensation: local block too large");
    if (!e && P->fused) {
      e = phase_begin(P, PH_CONDENSE, s);
      if (!e && P->qelim) {
        // eliminate q, condense the m N_p block of v (outputs of the slots 0..ec-1), recover the q rows
        DevPlan r = P->dp;
        r.n = P->dp.m * P->dp.Np;
        r.n_pad = P->qa.nr_pad;
        r.cw = condense_width(r.n_pad, false);
        if (!r.lu_waves_set) r.lu_waves = default_lu_waves(r.n_pad);
        if (r.lu_waves && !lu_reg_supported(r.n_pad, r.lu_waves)) r.lu_waves = 0;
        r.A = P->qa.A;
        r.X = P->qa.X;
        r.C = P->qa.C;
        r.D = P->qa.D;
        r.Rt = P->qa.Rt;
        r.ipiv = P->rp.ipiv;
        r.inv = P->rp.inv;
        r.mg = nullptr;   // the reduced block is stored whole
        r.uinfo = nullptr;
        const size_t k = P->dp.k;
        e = launch_qelim(P->dp, P->qa, ec, s);
        if (!e) e = condense_chunk(P, r, 0, ec, status + e0, S + (size_t)e0 * k * k, g + (size_t)e0 * k, P->qa.Yv,
                                   P->qa.zv, s);
        if (!e) e = launch_qrecover(P->dp, P->qa, e0, ec, Y, z, s);
      } else if (!e) {
        e = condense_chunk(P, P->dp, e0, ec, status + e0, S, g, Y, z, s);
      }
      if (!e) e = phase_end(P, PH_CONDENSE, s);
      if (e) return hip_fail(e, "condense");
      continue;
    }
    if (!e) e = phase_begin(P, PH_LU, s);
    if (!e) e = launch_lu(P->dp, ec, status + e0, s);
    if (!e) e = phase_end(P, PH_LU, s);
    if (!e) e = phase_begin(P, PH_SOLVE, s);
    P->xcd_clean = false;   // the split solve writes [Y z] over X
    if (!e) e = launch_solve(P->dp, ec, s);
    if (!e) e = phase_end(P, PH_SOLVE, s);
    if (!e) e = phase_begin(P, PH_SCHUR, s);
    if (!e) e = launch_schur(P->dp, e0, ec, S, g, Y, z, Rloc, Rtr, s);
    if (!e) e = phase_end(P, PH_SCHUR, s);
    if (e) return hip_fail(e, "condense");
  }
  return HDG_OK;
}

extern "C" int hdg_backsolve(hdg_plan *plan, const double *Y, const double *z, const double *dvhat,
                             double *dv, double *dq, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!Y || !z || !dvhat || !dv) return fail(HDG_EINVAL, "Y, z, dvhat and dv are required");
  if (P->dp.viscous && !dq) return fail(HDG_EINVAL, "dq is required for Navier-Stokes");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = phase_begin(P, PH_BACKSOLVE, s);
  if (!e) e = launch_backsolve(P->dp, Y, z, dvhat, dv, dq, s);
  if (!e) e = phase_end(P, PH_BACKSOLVE, s);
  if (e) return hip_fail(e, "backsolve");
  return HDG_OK;
}

extern "C" int hdg_trace_matvec(hdg_plan *plan, const double *S, const double *x, double *y, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!S || !x || !y) return fail(HDG_EINVAL, "S, x and y are required");
  if (x == y) return fail(HDG_EINVAL, "x and y must not alias");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = phase_begin(P, PH_MATVEC, s);
  if (!e) e = launch_trace_matvec(P->dp, S, x, y, s);
  if (!e) e = phase_end(P, PH_MATVEC, s);
  if (e) return hip_fail(e, "trace_matvec");
  return HDG_OK;
}

extern "C" int hdg_trace_rhs(hdg_plan *plan, const double *g, double *r, void *stream) {
  Plan *P = checked(plan);
  if (!P) return HDG_EINVAL;
  if (!g || !r) return fail(HDG_EINVAL, "g and r are required");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = phase_begin(P, PH_RHS, s);
  if (!e) e = launch_trace_rhs(P->dp, g, r, s);
  if (!e) e = phase_end(P, PH_RHS, s);
  if (e) return hip_fail(e, "trace_rhs");
  return HDG_OK;
}

extern "C" int hdg_selftest(double *max_err) {
  if (!max_err) return fail(HDG_EINVAL, "null argument");
  double *d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(double));
  if (!e) e = launch_mfma_selftest(d, nullptr);
  if (!e) e = hipMemcpy(max_err, d, sizeof(double), hipMemcpyDeviceToHost);
  if (d) (void)hipFree(d);
  if (e) return hip_fail(e, "selftest");
  return HDG_OK;
}
