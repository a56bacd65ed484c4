// Batches of plans (element types and orders with uneven block sizes)
// condensed by two launches (the LU items, then the right-hand-side items in
// per-XCD lists; one workgroup per item, or a persistent grid), and hipGraph
// capture of the whole assemble + condense sequence of a batch.
#include <algorithm>
#include <numeric>
#include <vector>

#include "hdg_plan.hpp"

using namespace hdg;

namespace hdg {
size_t batch_item_args_bytes();
hipError_t launch_condense_batch(const DevPlan *plans_dev, const void *io_dev, const int *lu_queue, int n_lu,
                                 const void *rhs_queue, const int *rhs_xoff, int *counters, int lu_groups,
                                 int rhs_groups, bool persistent, size_t lds, hipStream_t s);
}  // namespace hdg

namespace {

struct ItemArgs {   // device layout of the per-plan outputs read by the batch kernels
  double *S, *g, *Y, *z;
  int32_t *status;
};

constexpr int NXCD = 8;

struct Batch {
  std::vector<Plan *> plans;
  std::vector<int> queue;       // LU items: plan << 24 | element
  std::vector<int> rhs;         // right-hand-side items: (plan << 24 | element, block), by XCD
  int xoff[NXCD + 1] = {0};     // start of each XCD's items in rhs (in items)
  size_t lds = 0;
  int groups = 0, rhs_groups = 0;   // persistent grid sizes; groups == 0: one workgroup per item
  int rhs_max = 0;                  // longest per-XCD right-hand-side list
  bool bound = false;
  DevPlan *d_plans = nullptr;
  ItemArgs *d_io = nullptr;
  int *d_queue = nullptr;
  int *d_rhs = nullptr;
  int *d_xoff = nullptr;
  int *d_counter = nullptr;     // [1 + NXCD]
  std::vector<hdg_batch_io> io;
  bool io_set = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // stream mode (nstreams > 0): every plan's own condensation on one of nstreams streams
  int nstreams = 0;
  std::vector<double> cost;          // per plan: n_elem * (LU + solves + Schur) work
  int order = 0;
  std::vector<hipStream_t> side;     // created on first use, default priority
  std::vector<hipEvent_t> ev;        // [0] fork, [1 + t] join of stream t
  std::vector<int> stream_of;        // per plan
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct BatchLayout {
  size_t plans, io, queue, rhs, xoff, counter, total;
};

BatchLayout batch_layout(const Batch *B) {
  BatchLayout l{};
  size_t o = 0;
  l.plans = o;
  o = a256(o + B->plans.size() * sizeof(DevPlan));
  l.io = o;
  o = a256(o + B->plans.size() * sizeof(ItemArgs));
  l.queue = o;
  o = a256(o + B->queue.size() * sizeof(int));
  l.rhs = o;
  o = a256(o + B->rhs.size() * sizeof(int));
  l.xoff = o;
  o = a256(o + (NXCD + 1) * sizeof(int));
  l.counter = o;
  o = a256(o + 64);
  l.total = o;
  return l;
}

void drop_graph(Batch *B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
}

void drop_streams(Batch *B) {
  for (hipEvent_t e : B->ev) (void)hipEventDestroy(e);
  for (hipStream_t s : B->side) (void)hipStreamDestroy(s);
  B->ev.clear();
  B->side.clear();
}

}  // namespace

extern "C" int hdg_batch_create(hdg_batch **out, hdg_plan *const *plans, int n_plans, int order) {
  if (!out || !plans || n_plans < 1 || n_plans > 127) return fail(HDG_EINVAL, "need 1..127 plans");
  if (batch_item_args_bytes() != sizeof(ItemArgs)) return fail(HDG_EINVAL, "internal layout mismatch");
  *out = nullptr;
  Batch *B = new Batch;
  struct Item {
    double cost;
    int plan, el;
  };
  std::vector<Item> items, ritems;
  for (int i = 0; i < n_plans; ++i) {
    Plan *P = reinterpret_cast<Plan *>(plans[i]);
    if (!P || !P->bound || !P->fused || P->chunk < P->n_elem || P->n_elem >= (1 << 24)) {
      delete B;
      return fail(HDG_EINVAL, "batch plans must be bound, fused and process all elements in one chunk");
    }
    B->plans.push_back(P);
    B->lds = std::max(B->lds, condense_lds_bytes(P->dp.n_pad, P->dp.cw));
    const double np = P->dp.n_pad, kp = P->dp.k_pad;
    const double lu = np * np * np / 3.0, rhs = np * np * kp + np * kp * kp;   // LU; solves + Schur
    B->cost.push_back((lu + rhs) * P->n_elem);
    for (int e = 0; e < P->n_elem; ++e) {
      items.push_back({lu, i, e});
      ritems.push_back({rhs, i, e});
    }
  }
  B->order = order;
  const auto by_cost = [](const Item &a, const Item &b) { return a.cost > b.cost; };
  if (order == 0) {   // longest processing time first
    std::stable_sort(items.begin(), items.end(), by_cost);
    std::stable_sort(ritems.begin(), ritems.end(), by_cost);
  }
  for (const Item &it : items) B->queue.push_back((it.plan << 24) | it.el);
  // right-hand-side items: the k-th element (in queue order) to XCD k mod 8, its blocks together
  std::vector<std::vector<int>> xq(NXCD);
  for (size_t k = 0; k < ritems.size(); ++k) {
    const Item &it = ritems[k];
    const DevPlan &D = B->plans[it.plan]->dp;
    for (int j = 0; j < D.kx / D.cw; ++j) {
      xq[k % NXCD].push_back((it.plan << 24) | it.el);
      xq[k % NXCD].push_back(j);
    }
  }
  for (int x = 0; x < NXCD; ++x) {
    B->xoff[x + 1] = B->xoff[x] + (int)xq[x].size() / 2;
    B->rhs.insert(B->rhs.end(), xq[x].begin(), xq[x].end());
  }
  for (int x = 0; x < NXCD; ++x) B->rhs_max = std::max(B->rhs_max, B->xoff[x + 1] - B->xoff[x]);
  *out = reinterpret_cast<hdg_batch *>(B);
  return HDG_OK;
}

extern "C" void hdg_batch_destroy(hdg_batch *batch) {
  Batch *B = reinterpret_cast<Batch *>(batch);
  if (!B) return;
  drop_graph(B);
  drop_streams(B);
  delete B;
}

extern "C" int hdg_batch_workspace_bytes(const hdg_batch *batch, size_t *bytes) {
  const Batch *B = reinterpret_cast<const Batch *>(batch);
  if (!B || !bytes) return fail(HDG_EINVAL, "bad argument");
  *bytes = batch_layout(B).total;
  return HDG_OK;
}

extern "C" int hdg_batch_bind_workspace(hdg_batch *batch, void *ptr, size_t bytes, void *stream) {
  Batch *B = reinterpret_cast<Batch *>(batch);
  if (!B || !ptr) return fail(HDG_EINVAL, "bad argument");
  const BatchLayout l = batch_layout(B);
  if (bytes < l.total) return fail(HDG_ENOMEM, "batch workspace too small");
  char *base = static_cast<char *>(ptr);
  B->d_plans = reinterpret_cast<DevPlan *>(base + l.plans);
  B->d_io = reinterpret_cast<ItemArgs *>(base + l.io);
  B->d_queue = reinterpret_cast<int *>(base + l.queue);
  B->d_rhs = reinterpret_cast<int *>(base + l.rhs);
  B->d_xoff = reinterpret_cast<int *>(base + l.xoff);
  B->d_counter = reinterpret_cast<int *>(base + l.counter);
  std::vector<DevPlan> dp;
  for (Plan *P : B->plans) dp.push_back(P->dp);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(B->d_plans, dp.data(), dp.size() * sizeof(DevPlan), hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(B->d_queue, B->queue.data(), B->queue.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(B->d_rhs, B->rhs.data(), B->rhs.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(B->d_xoff, B->xoff, sizeof(B->xoff), hipMemcpyHostToDevice, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "batch_bind");
  B->bound = true;
  drop_graph(B);
  return HDG_OK;
}

extern "C" int hdg_batch_set_groups(hdg_batch *batch, int groups) {
  Batch *B = reinterpret_cast<Batch *>(batch);
  if (!B || groups < 0) return fail(HDG_EINVAL, "bad argument");
  B->groups = std::min<int>(groups, (int)B->queue.size());
  B->rhs_groups = NXCD * ((groups + NXCD - 1) / NXCD);
  drop_graph(B);
  return HDG_OK;
}

extern "C" int hdg_batch_set_streams(hdg_batch *batch, int n) {
  Batch *B = reinterpret_cast<Batch *>(batch);
  if (!B || n < 0 || n > 8) return fail(HDG_EINVAL, "streams: 0 (item lists) or 1..8");
  drop_graph(B);
  drop_streams(B);
  B->nstreams = n;
  if (n == 0) return HDG_OK;
  for (int t = 0; t < n; ++t) {
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e) {
      drop_streams(B);
      B->nstreams = 0;
      return hip_fail(e, "batch stream");
    }
    B->side.push_back(st);
  }
  for (int t = 0; t <= n; ++t) {
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e) {
      drop_streams(B);
      B->nstreams = 0;
      return hip_fail(e, "batch event");
    }
    B->ev.push_back(ev);
  }
  // plans to streams: largest first (order 0) or in plan order, each to the stream with the
  // least work so far
  std::vector<int> idx(B->plans.size());
  std::iota(idx.begin(), idx.end(), 0);
  if (B->order == 0) std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return B->cost[a] > B->cost[b]; });
  std::vector<double> load(n, 0.0);
  B->stream_of.assign(B->plans.size(), 0);
  for (int i : idx) {
    const int t = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    B->stream_of[i] = t;
    load[t] += B->cost[i];
  }
  return HDG_OK;
}

extern "C" int hdg_batch_set_io(hdg_batch *batch, const hdg_batch_io *io, void *stream) {
  Batch *B = reinterpret_cast<Batch *>(batch);
  if (!B || !B->bound || !io) return fail(HDG_EINVAL, "bad argument or unbound batch");
  std::vector<ItemArgs> args;
  for (size_t i = 0; i < B->plans.size(); ++i) {
    const hdg_batch_io &a = io[i];
    if (!a.v || !a.vhat || !a.S || !a.g || !a.Y || !a.z || !a.elem_status || (B->plans[i]->dp.viscous && !a.q))
      return fail(HDG_EINVAL, "batch io: v, vhat, S, g, Y, z, elem_status (and q for Navier-Stokes) required");
    args.push_back({a.S, a.g, a.Y, a.z, a.elem_status});
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(B->d_io, args.data(), args.size() * sizeof(ItemArgs), hipMemcpyHostToDevice, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "batch_set_io");
  B->io.assign(io, io + B->plans.size());
  B->io_set = true;
  drop_graph(B);
  return HDG_OK;
}

namespace {
// Stream mode: fork the side streams from s, run every plan's own assemble + condense on its
// stream (in the assignment order, so a stream runs its plans largest first), join back into s.
int batch_streams(Batch *B, hipStream_t s) {
  const int n = B->nstreams;
  hipError_t e = hipEventRecord(B->ev[0], s);
  for (int t = 0; t < n && !e; ++t) e = hipStreamWaitEvent(B->side[t], B->ev[0], 0);
  if (e) return hip_fail(e, "batch fork");
  std::vector<int> idx(B->plans.size());
  std::iota(idx.begin(), idx.end(), 0);
  if (B->order == 0) std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return B->cost[a] > B->cost[b]; });
  int rc = HDG_OK;
  for (int i : idx) {
    const hdg_batch_io &a = B->io[i];
    rc = hdg_assemble_condense(reinterpret_cast<hdg_plan *>(B->plans[i]), a.v, a.q, a.vhat, a.u_star, a.v_bc, a.S,
                               a.g, a.Y, a.z, nullptr, nullptr, a.elem_status, B->side[B->stream_of[i]]);
    if (rc) break;
  }
  // join every side stream, also after an error, so that none is left forked
  for (int t = 0; t < n; ++t) {
    hipError_t ej = hipEventRecord(B->ev[1 + t], B->side[t]);
    if (!ej) ej = hipStreamWaitEvent(s, B->ev[1 + t], 0);
    if (ej && !rc) rc = hip_fail(ej, "batch join");
  }
  return rc;
}

int batch_sequence(Batch *B, hipStream_t s) {
  if (B->nstreams > 0) return batch_streams(B, s);
  for (size_t i = 0; i < B->plans.size(); ++i) {
    Plan *P = B->plans[i];
    const hdg_batch_io &a = B->io[i];
    hipError_t e = launch_fill_int(a.elem_status, P->n_elem, HDG_OK, s);
    if (e) return hip_fail(e, "batch status init");
    int rc = run_front(P, a.v, a.q, a.vhat, a.u_star, a.v_bc, a.elem_status, 0, P->n_elem, s, P->dp.mg != nullptr);
    if (rc) return rc;
  }
  const bool persistent = B->groups > 0;
  hipError_t e = persistent ? launch_fill_int(B->d_counter, 1 + NXCD, 0, s) : hipSuccess;
  if (!e)
    e = launch_condense_batch(B->d_plans, B->d_io, B->d_queue, (int)B->queue.size(), B->d_rhs, B->d_xoff,
                              B->d_counter, persistent ? B->groups : (int)B->queue.size(),
                              persistent ? B->rhs_groups : NXCD * B->rhs_max, persistent, B->lds, s);
  if (e) return hip_fail(e, "batch condense");
  return HDG_OK;
}
}  // namespace

extern "C" int hdg_batch_run(hdg_batch *batch, void *stream) {
  Batch *B = reinterpret_cast<Batch *>(batch);
  if (!B || !B->bound || !B->io_set) return fail(HDG_EINVAL, "batch not bound or io not set");
  return batch_sequence(B, reinterpret_cast<hipStream_t>(stream));
}

extern "C" int hdg_batch_capture(hdg_batch *batch, void *stream) {
  Batch *B = reinterpret_cast<Batch *>(batch);
  if (!B || !B->bound || !B->io_set) return fail(HDG_EINVAL, "batch not bound or io not set");
  for (Plan *P : B->plans)
    if (P->timing) return fail(HDG_EINVAL, "disable phase timing before capturing a graph");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // one eager pass sets every kernel attribute outside the capture
  int rc = batch_sequence(B, s);
  if (rc) return rc;
  drop_graph(B);
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e) return hip_fail(e, "begin capture");
  rc = batch_sequence(B, s);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e) return hip_fail(e, "end capture");
  B->graph = g;
  e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
  if (e) {
    drop_graph(B);
    return hip_fail(e, "graph instantiate");
  }
  return HDG_OK;
}

extern "C" int hdg_batch_replay(hdg_batch *batch, void *stream) {
  Batch *B = reinterpret_cast<Batch *>(batch);
  if (!B || !B->exec) return fail(HDG_EINVAL, "no captured graph");
  hipError_t e = hipGraphLaunch(B->exec, reinterpret_cast<hipStream_t>(stream));
  if (e) return hip_fail(e, "graph launch");
  return HDG_OK;
}

extern "C" int hdg_batch_info(const hdg_batch *batch, int *n_items, int *groups, size_t *lds) {
  const Batch *B = reinterpret_cast<const Batch *>(batch);
  if (!B) return fail(HDG_EINVAL, "bad argument");
  if (n_items) *n_items = (int)B->queue.size();
  if (groups) *groups = B->groups;
  if (lds) *lds = B->lds;
  return HDG_OK;
}

extern "C" int hdg_plan_set_tuning(hdg_plan *plan, const hdg_tuning *t) {
  Plan *P = reinterpret_cast<Plan *>(plan);
  if (!P || !t) return fail(HDG_EINVAL, "bad argument");
  if (t->contract_threads) {
    if (t->contract_threads != 256 && t->contract_threads != 512 && t->contract_threads != 1024)
      return fail(HDG_EINVAL, "contract_threads must be 256, 512 or 1024");
    P->dp.contract_threads = t->contract_threads;
  }
  if (t->condense_width) {
    if (t->condense_width != 16 && t->condense_width != 32) return fail(HDG_EINVAL, "condense_width must be 16 or 32");
    if (condense_lds_bytes(P->dp.n_pad, t->condense_width) > 160 * 1024)
      return fail(HDG_EUNSUPPORTED, "condense_width does not fit in LDS for this block size");
    if (!P->fused) return fail(HDG_EINVAL, "plan uses the separate LU / solve / Schur kernels");
    P->dp.cw = t->condense_width;
  }
  if (t->condense_width_lp) {
    if (t->condense_width_lp != 16 && t->condense_width_lp != 32)
      return fail(HDG_EINVAL, "condense_width_lp must be 16 or 32");
    if (condense_lds_bytes_lp(P->dp.n_pad, t->condense_width_lp) > 160 * 1024)
      return fail(HDG_EUNSUPPORTED, "condense_width_lp does not fit in LDS for this block size");
    P->dp.cw_lp = t->condense_width_lp;
  }
  if (t->condense_launches) {
    if (t->condense_launches != 1 && t->condense_launches != 2)
      return fail(HDG_EINVAL, "condense_launches must be 1 or 2");
    P->dp.condense_launches = t->condense_launches;
  }
  if (t->lu_waves) {
    if (t->lu_waves == 1) {
      P->dp.lu_waves = 0;
    } else {
      if (t->lu_waves != 2 && t->lu_waves != 4 && t->lu_waves != 8)
        return fail(HDG_EINVAL, "lu_waves must be 1, 2, 4 or 8");
      if (!lu_reg_supported(P->dp.n_pad, t->lu_waves))
        return fail(HDG_EUNSUPPORTED, "register-resident LU not available for this block size");
      P->dp.lu_waves = t->lu_waves;
    }
    P->dp.lu_waves_set = 1;
  }
  if (t->lp_operands) {
    if (t->lp_operands != 1 && t->lp_operands != 2) return fail(HDG_EINVAL, "lp_operands must be 1 (FP32) or 2 (BF16)");
    P->dp.lp_bf16 = t->lp_operands == 2;
  }
  return HDG_OK;
}

extern "C" int hdg_plan_get_tuning(const hdg_plan *plan, hdg_tuning *t) {
  const Plan *P = reinterpret_cast<const Plan *>(plan);
  if (!P || !t) return fail(HDG_EINVAL, "bad argument");
  t->contract_threads = P->dp.contract_threads;
  t->condense_width = P->fused ? P->dp.cw : 0;
  t->condense_width_lp = P->dp.cw_lp;
  t->condense_launches = P->dp.condense_launches;
  t->lu_waves = P->dp.lu_waves ? P->dp.lu_waves : 1;
  t->lp_operands = P->dp.lp_bf16 ? 2 : 1;
  return HDG_OK;
}
