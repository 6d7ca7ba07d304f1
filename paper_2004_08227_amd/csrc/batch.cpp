// Host runtime of the batched solver: many independent FP32 models (each a
// pairwise MRF of Sec. 3 solved by MPLP++ iterations, Sec. 4-6) in one
// persistent launch, optionally replayed from a captured hipGraph.
//
// Planning.  The work of model b per iteration is modelled as
//   t_b(T) = S_b * (t_hand + t_edge(LT_b) / 2) + (m_b / T) * t_edge(LT_b)
// for a team of T workgroups (S_b matchings, each needing one cross-workgroup
// handoff; m_b / T edge updates per member, one after another), as
//   t_b = m_b * t_edge(LT_b)
// for a model on one workgroup with its unaries in LDS (no handoffs), and
// never less than the member's share of HBM traffic.  The planner
// binary-searches a makespan tau: every model gets the smallest team with
// t_b(T) <= tau (at most one member per edge of its largest matching), teams
// take the first workgroups, and single-workgroup models are packed, longest
// first, onto the least-loaded workgroups (which tau is feasible).  By default
// the single-workgroup models then go, longest first, to a shared queue from
// which every workgroup takes the next model once its own tasks are done, so
// errors in the time estimates do not unbalance the launch.  The time
// constants are options, so a tuner can calibrate them; they change only the
// assignment, never the results.
//
// Engines.  With every L <= 64 the launch runs the wave engine (one edge
// update per wavefront, twelve workers per workgroup; wave_engine.h), whose
// time model is in wave_model_time; otherwise the workgroup engine (the
// mailbox engine's kernel code, one update at a time per workgroup).  Both
// give every model bitwise the results of the single-model engine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <queue>
#include <vector>

#include "common.h"
#include "host_util.h"
#include "schedule.h"
#include "wave_batch.h"

using namespace mplpxx;

struct ModelHost {
  int n, L, m, S, lt;
  int potts = 0;                   // structured cost kind (MPLPXX_COST_*; parameters per edge), 0 dense
  int max_step;                    // edges of the largest matching
  std::vector<int> slot_of_edge;   // for state export
};

struct mplpxx_batch {
  int count = 0;
  std::vector<ModelHost> mh;
  std::vector<BatchModel> md;
  long long total_tables = 0, total_phi = 0, total_u = 0;
  int total_slots = 0, total_nodes = 0, total_csr = 0, total_inc = 0;
  int max_lt = 16;
  // device
  float* d_tables = nullptr;
  float* d_phi = nullptr;
  float* d_U = nullptr;
  float* d_Ulo = nullptr;  // bf16 corrections of U (compensated FP32 unaries)
  float* d_unaries = nullptr;
  unsigned long long* d_mb = nullptr;
  SlotInfo* d_slots = nullptr;
  int* d_deg = nullptr;
  BatchModel* d_models = nullptr;
  BatchTask* d_tasks = nullptr;
  int* d_task_ptr = nullptr;
  int* d_err = nullptr;
  int* d_ticket = nullptr;
  unsigned long long* d_sink = nullptr;  // scratch words of the workgroups
  long long* d_wg_time = nullptr;        // [grid][2] clocks of the last launch
  int* d_node_model = nullptr;
  int* d_slot_model = nullptr;
  int* d_node_ptr = nullptr;
  int* d_inc = nullptr;
  double* d_node_min = nullptr;
  double* d_edge_min = nullptr;
  double* d_duals = nullptr;
  // plan
  int grid = 0;
  int grid_opt = 0;
  int num_cus = 0;
  int ntasks = 0, nteams = 0, max_team = 1;
  double plan_us = 0.0;
  double t_hand_us = 0.7;
  double t_edge_us[4] = {0.30, 0.45, 0.85, 2.0};  // LT 16, 32, 64, 128
  int one_per_model = 0;
  int use_queue = 1;           // single-workgroup models from a shared queue (else statically packed)
  int qbegin = 0, qlen = 0;
  std::vector<int> wg_team_model;  // model of each workgroup's own task, -1 none
  int use_lds = 1;             // LDS-resident unaries for models on one workgroup
  size_t lds_limit = 0;        // dynamic LDS a workgroup can have
  size_t lds_bytes = 0;        // dynamic LDS of the launch
  int lds_tasks = 0;
  // wave engine (one wave per edge update; models with L <= 64)
  int engine_opt = 0;          // 0 auto, 1 workgroup (mailbox) engine, 2 wave engine
  bool wave = false;           // the plan runs the wave engine
  double wv_edge_us[3] = {0.05, 0.08, 0.13};  // workgroup time per edge update besides its bytes, LT 16, 32, 64
  double wv_lat_lds_us = 2.4;  // latency of one update, unaries in LDS
  double wv_lat_mb_us = 2.0;   // latency of one update through the mailboxes
  size_t wv_static = 0;        // static LDS of the wave kernel
  size_t wv_lds_limit = 0;     // dynamic LDS a workgroup of the wave kernel can have
  size_t wv_lds_cap = 0;       // dynamic LDS that keeps the kernel's register-limited occupancy
  int wv_waves = 8;
  int potts = 0;               // a batch of structured-cost models (MPLPXX_COST_*), 0 dense
  bool plan_dirty = true;
  // execution
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool use_graph = true;
  hipGraphExec_t gexec = nullptr;
  int graph_k = -1;
  long long spin_limit = 1ll << 22;
  double last_ms = 0.0;
  long long iterations = 0;
};

namespace {

int lt_index(int lt) { return lt == 16 ? 0 : lt == 32 ? 1 : lt == 64 ? 2 : 3; }

bool lds_fits(const mplpxx_batch* b, int i) {
  if (!b->use_lds) return false;
  if (b->wave) return wv_lds_bytes(b->mh[i].n, b->mh[i].L) <= b->wv_lds_cap;
  return lds_model_bytes(b->mh[i].n, b->mh[i].L) <= b->lds_limit;
}

// Wave engine: a team of T workgroups is T * NW workers.  Per iteration a
// model needs m / T edge updates of workgroup time, each t_w(LT) plus its
// bytes at the workgroup's share of the achievable HBM bandwidth (about 3/4
// of the nominal 8 TB/s), and S matchings one after another, each of
// ceil(max_step / (T NW)) rounds of one update latency.
double wave_model_time(const mplpxx_batch* b, int i, int T, double bw_per_wg_bytes_us) {
  const ModelHost& h = b->mh[i];
  const double tw = b->wv_edge_us[std::min(2, lt_index(h.lt))];
  const double lat = (T == 1 && lds_fits(b, i)) ? b->wv_lat_lds_us : b->wv_lat_mb_us;
  const double workers = (double)T * b->wv_waves;
  const double chain = h.S * std::ceil(h.max_step / workers) * lat;
  const double bytes = (h.potts ? 4.0 * cost_params(h.potts) : 4.0 * h.L * h.L) + 16.0 * h.L;
  const double work = (double)h.m / T * (tw + bytes / (0.75 * bw_per_wg_bytes_us));
  return std::max(chain, work);
}

double model_time(const mplpxx_batch* b, int i, int T, double bw_per_wg_bytes_us) {
  const ModelHost& h = b->mh[i];
  if (h.m == 0) return 0.0;
  if (b->wave) return wave_model_time(b, i, T, bw_per_wg_bytes_us);
  const double te = b->t_edge_us[lt_index(h.lt)];
  const double lat = (T == 1 && lds_fits(b, i)) ? h.m * te : h.S * (b->t_hand_us + 0.5 * te) + (double)h.m / T * te;
  const double bytes = (double)h.m * (4.0 * h.L * h.L + 16.0 * h.L) / T;
  return std::max(lat, bytes / bw_per_wg_bytes_us);
}

// tasks for makespan tau; returns the resulting max workgroup load
double assign(const mplpxx_batch* b, double tau, int G, int team_cap, double bw,
              std::vector<std::vector<BatchTask>>& wg_tasks, int* nteams, int* max_team) {
  wg_tasks.assign(G, {});
  std::vector<double> load(G, 0.0);
  std::vector<int> team(b->count, 1);
  int used = 0;
  *nteams = 0;
  *max_team = 1;
  for (int i = 0; i < b->count; ++i) {
    const ModelHost& h = b->mh[i];
    if (h.m == 0) continue;
    int tmax = std::max(1, std::min(h.max_step, team_cap));
    int T = 1;
    if (!b->one_per_model) {
      // smallest team meeting tau (model_time decreases with T)
      const double target = tau;
      int lo = 1, hi = tmax;
      if (model_time(b, i, tmax, bw) > target) {
        T = tmax;
      } else {
        while (lo < hi) {
          const int mid = (lo + hi) / 2;
          if (model_time(b, i, mid, bw) <= target) hi = mid; else lo = mid + 1;
        }
        T = lo;
      }
    }
    team[i] = T;
  }
  // teams first: each member's first task, consecutive workgroups
  for (int i = 0; i < b->count; ++i) {
    if (team[i] < 2) continue;
    if (used + team[i] > team_cap) return INFINITY;
    const double t = model_time(b, i, team[i], bw);
    for (int r = 0; r < team[i]; ++r) {
      wg_tasks[used + r].push_back(BatchTask{i, r, team[i], 0});
      load[used + r] += t;
    }
    used += team[i];
    ++*nteams;
    *max_team = std::max(*max_team, team[i]);
  }
  // single-workgroup models, longest first, onto the least-loaded workgroup
  std::vector<int> singles;
  for (int i = 0; i < b->count; ++i)
    if (team[i] < 2 && b->mh[i].m > 0) singles.push_back(i);
  std::sort(singles.begin(), singles.end(), [&](int x, int y) {
    const double tx = model_time(b, x, 1, bw), ty = model_time(b, y, 1, bw);
    return tx != ty ? tx > ty : x < y;
  });
  using Item = std::pair<double, int>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> pq;
  for (int w = 0; w < G; ++w) pq.push({load[w], w});
  for (int i : singles) {
    Item it = pq.top();
    pq.pop();
    wg_tasks[it.second].push_back(BatchTask{i, 0, 1, lds_fits(b, i) ? 1 : 0});
    it.first += model_time(b, i, 1, bw);
    load[it.second] = it.first;
    pq.push(it);
  }
  return *std::max_element(load.begin(), load.end());
}

int plan(mplpxx_batch* b) {
  if (b->engine_opt == 2 && b->max_lt > 64) return fail(MPLPXX_EINVAL, "the wave engine takes models with L <= 64");
  bool any_potts = false;
  for (const ModelHost& h : b->mh) any_potts = any_potts || h.potts;
  if (any_potts && b->engine_opt == 1) return fail(MPLPXX_EINVAL, "structured costs run on the wave engine only");
  b->wave = b->engine_opt == 2 || (b->engine_opt == 0 && b->max_lt <= 64);
  if (b->wave) {
    // LDS-resident models only as large as keeps the register-limited
    // number of workgroups per compute unit
    int dev = 0, cu_lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
      return fail(MPLPXX_EDEVICE, "device query failed");
    const int o = std::max(1, wbatch_blocks_per_cu(0, b->potts));
    const size_t share = (size_t)cu_lds / o;
    b->wv_lds_cap = share > b->wv_static + 256 ? std::min(b->wv_lds_limit, share - b->wv_static - 256) : 0;
  }
  // dynamic LDS: enough for the largest model that could keep its unaries there
  size_t dyn = 0;
  for (int i = 0; i < b->count; ++i)
    if (b->mh[i].m > 0 && lds_fits(b, i))
      dyn = std::max(dyn, b->wave ? wv_lds_bytes(b->mh[i].n, b->mh[i].L) : lds_model_bytes(b->mh[i].n, b->mh[i].L));
  const int per_cu = b->wave ? wbatch_blocks_per_cu(dyn, b->potts) : batch_blocks_per_cu(b->max_lt, dyn);
  if (per_cu < 1) return fail(MPLPXX_EDEVICE, "batched kernel does not fit on a compute unit");
  const int gmax = per_cu * b->num_cus;
  int G = b->grid_opt > 0 ? std::min(b->grid_opt, gmax) : gmax;
  G = std::max(1, G);
  // HBM share of one workgroup in bytes per microsecond (8 TB/s nominal)
  const double bw = 8.0e12 / 1e6 / G;
  // teams wait on each other, so they only use the first num_cus logical
  // workgroups: one per compute unit always fits
  const int team_cap = std::min(G, b->num_cus);
  double lo = 0.0, hi = 0.0;
  for (int i = 0; i < b->count; ++i) {
    const int tmax = std::max(1, std::min(b->mh[i].max_step, team_cap));
    lo = std::max(lo, model_time(b, i, tmax, bw));
    hi += model_time(b, i, 1, bw);
  }
  hi = std::max(hi, lo);
  std::vector<std::vector<BatchTask>> best, cur;
  int nteams = 0, max_team = 1, bt = 0, bm = 1;
  double best_load = assign(b, hi, G, team_cap, bw, best, &bt, &bm);
  for (int rep = 0; rep < 40 && hi - lo > 1e-3 * hi; ++rep) {
    const double mid = 0.5 * (lo + hi);
    const double l = assign(b, mid, G, team_cap, bw, cur, &nteams, &max_team);
    if (l <= mid * 1.05) {
      hi = mid;
      if (l < best_load) {
        best_load = l;
        best.swap(cur);
        bt = nteams;
        bm = max_team;
      }
    } else {
      lo = mid;
    }
  }
  // each workgroup's own tasks; with the queue, the single-workgroup tasks
  // (stride 1) go, longest first as packed, to the shared queue instead
  std::vector<BatchTask> tasks, queued;
  std::vector<int> ptr(G + 1, 0);
  for (int w = 0; w < G; ++w) {
    for (const BatchTask& t : best[w]) {
      if (b->use_queue && t.stride == 1) queued.push_back(t);
      else tasks.push_back(t);
    }
    ptr[w + 1] = (int)tasks.size();
  }
  if (b->use_queue) {
    std::stable_sort(queued.begin(), queued.end(), [&](const BatchTask& x, const BatchTask& y) {
      return model_time(b, x.model, 1, bw) > model_time(b, y.model, 1, bw);
    });
  }
  b->wg_team_model.assign(G, -1);
  for (int w = 0; w < G; ++w)
    if (ptr[w + 1] > ptr[w]) b->wg_team_model[w] = tasks[ptr[w]].model;
  b->qbegin = (int)tasks.size();
  b->qlen = (int)queued.size();
  tasks.insert(tasks.end(), queued.begin(), queued.end());
  if (b->d_tasks) (void)hipFree(b->d_tasks);
  if (b->d_task_ptr) (void)hipFree(b->d_task_ptr);
  if (b->d_sink) (void)hipFree(b->d_sink);
  if (b->d_wg_time) (void)hipFree(b->d_wg_time);
  b->d_tasks = nullptr;
  b->d_task_ptr = nullptr;
  b->d_sink = nullptr;
  b->d_wg_time = nullptr;
  const size_t sink_words = b->wave ? wbatch_sink_words() : (size_t)(256 + 128);
  HIP_TRY(hipMalloc(&b->d_sink, (size_t)G * sink_words * sizeof(unsigned long long)));
  HIP_TRY(hipMalloc(&b->d_wg_time, (size_t)G * 2 * sizeof(long long)));
  HIP_TRY(hipMemsetAsync(b->d_wg_time, 0, (size_t)G * 2 * sizeof(long long), b->stream));
  HIP_TRY(hipMalloc(&b->d_tasks, std::max<size_t>(1, tasks.size()) * sizeof(BatchTask)));
  HIP_TRY(hipMalloc(&b->d_task_ptr, (G + 1) * sizeof(int)));
  // every copy and fill goes through the batch's own (non-blocking) stream, so
  // that it is ordered before the kernels that read it
  if (!tasks.empty())
    HIP_TRY(hipMemcpyAsync(b->d_tasks, tasks.data(), tasks.size() * sizeof(BatchTask), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_task_ptr, ptr.data(), (G + 1) * sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->grid = G;
  b->lds_bytes = dyn;
  b->lds_tasks = 0;
  for (const BatchTask& t : tasks) b->lds_tasks += t.lds;
  b->ntasks = (int)tasks.size();
  b->nteams = bt;
  b->max_team = bm;
  b->plan_us = best_load;
  b->plan_dirty = false;
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->graph_k = -1;
  }
  return MPLPXX_OK;
}

void free_batch(mplpxx_batch* b) {
  void* ptrs[] = {b->d_tables, b->d_phi, b->d_U, b->d_Ulo, b->d_unaries, b->d_mb, b->d_slots, b->d_deg, b->d_models,
                  b->d_tasks, b->d_task_ptr, b->d_err, b->d_ticket, b->d_sink, b->d_wg_time, b->d_node_model,
                  b->d_slot_model, b->d_node_ptr, b->d_inc, b->d_node_min, b->d_edge_min, b->d_duals};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->stream) (void)hipStreamDestroy(b->stream);
}

hipError_t enqueue(mplpxx_batch* b, int k) {
  BatchArgs a{};
  a.tables = b->d_tables;
  a.phi = b->d_phi;
  a.mb = b->d_mb;
  a.slots = b->d_slots;
  a.deg = b->d_deg;
  a.models = b->d_models;
  a.tasks = b->d_tasks;
  a.task_ptr = b->d_task_ptr;
  a.ticket = b->d_ticket;
  a.sink = b->d_sink;
  a.wg_time = b->d_wg_time;
  a.err = b->d_err;
  a.spin_limit = b->spin_limit;
  a.qbegin = b->qbegin;
  a.qlen = b->qlen;
  hipError_t e = launch_fill_int(b->d_ticket, 0, 2, b->stream);
  if (e != hipSuccess) return e;
  e = launch_u_to_mb(b->d_U, b->d_Ulo, b->d_mb, (size_t)b->total_u, b->stream);
  if (e != hipSuccess) return e;
  e = b->wave ? launch_wbatch(a, b->grid, k, b->lds_bytes, b->potts, b->stream)
              : launch_batch(a, b->max_lt, b->grid, k, b->lds_bytes, b->stream);
  if (e != hipSuccess) return e;
  return launch_mb_to_u(b->d_U, b->d_Ulo, b->d_mb, (size_t)b->total_u, b->stream);
}

}  // namespace

extern "C" {

static int create_batch(int32_t count, const int32_t* n, const int32_t* L, const int64_t* m,
                        const int32_t* const* edges, const float* const* unaries, const float* const* pairwise,
                        int potts, mplpxx_batch** out) {
  if (!out) return fail(MPLPXX_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1) return fail(MPLPXX_EINVAL, "count must be >= 1");
  if (!n || !L || !m || !unaries) return fail(MPLPXX_EINVAL, "NULL size or unary array");
  mplpxx_batch* b = new (std::nothrow) mplpxx_batch();
  if (!b) return fail(MPLPXX_ENOMEM, "host allocation failed");
  auto bail = [&](int code) {
    free_batch(b);
    delete b;
    return code;
  };
  b->count = count;
  b->potts = potts;
  b->mh.resize(count);
  b->md.resize(count);
  std::vector<GraphPrep> preps(count);
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1) return bail(fail(MPLPXX_EINVAL, "model %d: n must be >= 1", i));
    if (L[i] < 1 || L[i] > MPLPXX_MAX_LABELS) return bail(fail(MPLPXX_EINVAL, "model %d: L out of range", i));
    if (m[i] < 0 || m[i] > (int64_t)n[i] * (n[i] - 1) / 2) return bail(fail(MPLPXX_EINVAL, "model %d: bad m", i));
    if (m[i] > 0 && (!edges || !pairwise || !edges[i] || !pairwise[i]))
      return bail(fail(MPLPXX_EINVAL, "model %d: NULL edges or pairwise", i));
    if (!unaries[i]) return bail(fail(MPLPXX_EINVAL, "model %d: NULL unaries", i));
    if (potts && L[i] > 64) return bail(fail(MPLPXX_EINVAL, "model %d: structured costs take L <= 64", i));
    for (size_t k = 0; k < (size_t)n[i] * L[i]; ++k)
      if (!(std::fabs(unaries[i][k]) <= (float)MPLPXX_F32_MAX_COST))
        return bail(fail(MPLPXX_EINVAL, "model %d: non-finite or too large unary", i));
    for (size_t k = 0; k < (size_t)m[i] * (potts ? (size_t)cost_params(potts) : (size_t)L[i] * L[i]); ++k)
      if (!(std::fabs(pairwise[i][k]) <= (float)MPLPXX_F32_MAX_COST))
        return bail(fail(MPLPXX_EINVAL, "model %d: non-finite or too large pairwise", i));
    if (potts && m[i] > 0 && check_structured_params(potts, pairwise[i], m[i]) != MPLPXX_OK) {
      const std::string msg = g_last_error;
      return bail(fail(MPLPXX_EINVAL, "model %d: %s", i, msg.c_str()));
    }
    const int rc = prepare_graph(n[i], (int)m[i], m[i] ? edges[i] : nullptr, preps[i]);
    if (rc != MPLPXX_OK) {
      const std::string msg = g_last_error;
      return bail(fail(rc, "model %d: %s", i, msg.c_str()));
    }
    ModelHost& h = b->mh[i];
    h.n = n[i];
    h.L = L[i];
    h.m = (int)m[i];
    h.potts = potts;
    h.S = preps[i].S;
    h.lt = next_tile(L[i]);
    h.max_step = 1;
    for (int s = 0; s < h.S; ++s) h.max_step = std::max(h.max_step, preps[i].step_ptr[s + 1] - preps[i].step_ptr[s]);
    for (int d : preps[i].deg)
      if (d >= 65536) return bail(fail(MPLPXX_EINVAL, "model %d: a node has degree >= 65536", i));
    h.slot_of_edge = preps[i].slot_of_edge;
    b->max_lt = std::max(b->max_lt, h.lt);
    BatchModel& d = b->md[i];
    d.table_off = b->total_tables;
    d.phi_off = b->total_phi;
    d.u_off = b->total_u;
    d.slot_off = b->total_slots;
    d.node_off = b->total_nodes;
    d.n = h.n;
    d.L = h.L;
    d.m = h.m;
    d.lt = h.lt;
    d.csr_off = b->total_csr;
    d.inc_off = b->total_inc;
    d.potts = h.potts;
    b->total_tables += (long long)h.m * (potts ? (long long)cost_params(potts) : (long long)h.L * h.L);
    b->total_phi += (long long)h.m * 2 * h.L;
    b->total_u += (long long)h.n * h.L;
    b->total_slots += h.m;
    b->total_nodes += h.n;
    b->total_csr += h.n + 1;
    b->total_inc += 2 * h.m;
  }
#define TRY(expr)                                                               \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      const int c_ = e_ == hipErrorOutOfMemory ? MPLPXX_ENOMEM : MPLPXX_EDEVICE; \
      return bail(fail(c_, "%s: %s", #expr, hipGetErrorString(e_)));            \
    }                                                                           \
  } while (0)
  int dev = 0;
  TRY(hipGetDevice(&dev));
  TRY(hipDeviceGetAttribute(&b->num_cus, hipDeviceAttributeMultiprocessorCount, dev));
  b->lds_limit = batch_lds_limit(b->max_lt);
  b->wv_lds_limit = wbatch_lds_limit(&b->wv_static, b->potts);
  b->wv_waves = wbatch_waves();
  TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  TRY(hipEventCreate(&b->ev0));
  TRY(hipEventCreate(&b->ev1));
  auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, bytes > 0 ? bytes : 16); };
  TRY(alloc((void**)&b->d_tables, ((size_t)b->total_tables + kTailPad) * sizeof(float)));
  TRY(alloc((void**)&b->d_phi, ((size_t)b->total_phi + kTailPad) * sizeof(float)));
  TRY(alloc((void**)&b->d_U, (size_t)b->total_u * sizeof(float)));
  TRY(alloc((void**)&b->d_Ulo, (size_t)b->total_u * sizeof(float)));
  TRY(alloc((void**)&b->d_unaries, (size_t)b->total_u * sizeof(float)));
  TRY(alloc((void**)&b->d_mb, (size_t)b->total_u * sizeof(unsigned long long)));
  TRY(alloc((void**)&b->d_slots, (size_t)b->total_slots * sizeof(SlotInfo)));
  TRY(alloc((void**)&b->d_deg, (size_t)b->total_nodes * sizeof(int)));
  TRY(alloc((void**)&b->d_models, (size_t)count * sizeof(BatchModel)));
  TRY(alloc((void**)&b->d_err, 8 * sizeof(int)));
  TRY(alloc((void**)&b->d_ticket, 2 * sizeof(int)));
  TRY(alloc((void**)&b->d_node_model, (size_t)b->total_nodes * sizeof(int)));
  TRY(alloc((void**)&b->d_slot_model, (size_t)b->total_slots * sizeof(int)));
  TRY(alloc((void**)&b->d_node_ptr, (size_t)b->total_csr * sizeof(int)));
  TRY(alloc((void**)&b->d_inc, (size_t)b->total_inc * sizeof(int)));
  TRY(alloc((void**)&b->d_node_min, (size_t)b->total_nodes * sizeof(double)));
  TRY(alloc((void**)&b->d_edge_min, (size_t)b->total_slots * sizeof(double)));
  TRY(alloc((void**)&b->d_duals, (size_t)count * sizeof(double)));
  hipStream_t cs = b->stream;
  TRY(hipMemsetAsync(b->d_phi, 0, ((size_t)b->total_phi + kTailPad) * sizeof(float), cs));
  TRY(hipMemsetAsync(b->d_tables + b->total_tables, 0, kTailPad * sizeof(float), cs));
  TRY(hipMemsetAsync(b->d_err, 0, 8 * sizeof(int), cs));
  // per model: packed tables (slot order, transposed where given as (v, u)),
  // unaries, slot metadata, degrees, incidence lists, node/slot maps
  std::vector<float> packed;
  std::vector<int> node_model(b->total_nodes), slot_model(b->total_slots);
  for (int i = 0; i < count; ++i) {
    const ModelHost& h = b->mh[i];
    const BatchModel& d = b->md[i];
    const GraphPrep& g = preps[i];
    const size_t tl = potts ? (size_t)cost_params(potts) : (size_t)h.L * h.L;
    packed.resize((size_t)h.m * tl);
    for (int s = 0; s < h.m; ++s) {
      const int e = g.order[s];
      const float* src = pairwise[i] + (size_t)e * tl;
      float* dst = packed.data() + (size_t)s * tl;
      if (potts == MPLPXX_COST_POTTS) {
        *dst = src[0] + 0.0f;  // (a weight of -0 is stored as +0: the table it stands for is the same)
      } else if (potts == MPLPXX_COST_TRUNC_QUAD || potts == MPLPXX_COST_TRUNC_LINEAR) {
        dst[0] = src[0] + 0.0f;  // (w and tau of -0 as +0: every cost is then +0 or positive)
        dst[1] = src[1] + 0.0f;
      } else if (potts || !g.flip[e]) {   // (structured costs are symmetric in s, t)
        std::memcpy(dst, src, tl * sizeof(float));
      } else {
        for (int r = 0; r < h.L; ++r)
          for (int c = 0; c < h.L; ++c) dst[(size_t)r * h.L + c] = src[(size_t)c * h.L + r];
      }
    }
    if (h.m) {
      TRY(hipMemcpyAsync(b->d_tables + d.table_off, packed.data(), packed.size() * sizeof(float), hipMemcpyHostToDevice, cs));
      TRY(hipStreamSynchronize(cs));  // `packed` is reused for the next model
    }
    TRY(hipMemcpyAsync(b->d_unaries + d.u_off, unaries[i], (size_t)h.n * h.L * sizeof(float), hipMemcpyHostToDevice, cs));
    if (h.m) TRY(hipMemcpyAsync(b->d_slots + d.slot_off, g.slots.data(), (size_t)h.m * sizeof(SlotInfo), hipMemcpyHostToDevice, cs));
    TRY(hipMemcpyAsync(b->d_deg + d.node_off, g.deg.data(), (size_t)h.n * sizeof(int), hipMemcpyHostToDevice, cs));
    std::vector<int> node_ptr(h.n + 1, 0), inc(2 * (size_t)h.m);
    for (int s = 0; s < h.m; ++s) {
      node_ptr[g.slots[s].u + 1]++;
      node_ptr[g.slots[s].v + 1]++;
    }
    for (int u = 0; u < h.n; ++u) node_ptr[u + 1] += node_ptr[u];
    std::vector<int> fillp(node_ptr.begin(), node_ptr.end() - 1);
    for (int s = 0; s < h.m; ++s) {
      inc[fillp[g.slots[s].u]++] = 2 * s;
      inc[fillp[g.slots[s].v]++] = 2 * s + 1;
    }
    TRY(hipMemcpyAsync(b->d_node_ptr + d.csr_off, node_ptr.data(), node_ptr.size() * sizeof(int), hipMemcpyHostToDevice, cs));
    if (h.m) TRY(hipMemcpyAsync(b->d_inc + d.inc_off, inc.data(), inc.size() * sizeof(int), hipMemcpyHostToDevice, cs));
    TRY(hipStreamSynchronize(cs));  // host vectors of this model go out of scope
    for (int u = 0; u < h.n; ++u) node_model[d.node_off + u] = i;
    for (int s = 0; s < h.m; ++s) slot_model[d.slot_off + s] = i;
  }
  TRY(hipMemcpyAsync(b->d_models, b->md.data(), (size_t)count * sizeof(BatchModel), hipMemcpyHostToDevice, cs));
  TRY(hipMemcpyAsync(b->d_node_model, node_model.data(), node_model.size() * sizeof(int), hipMemcpyHostToDevice, cs));
  if (b->total_slots)
    TRY(hipMemcpyAsync(b->d_slot_model, slot_model.data(), slot_model.size() * sizeof(int), hipMemcpyHostToDevice, cs));
  TRY(hipMemcpyAsync(b->d_U, b->d_unaries, (size_t)b->total_u * sizeof(float), hipMemcpyDeviceToDevice, cs));
  TRY(hipMemsetAsync(b->d_Ulo, 0, (size_t)b->total_u * sizeof(float), cs));
  TRY(hipStreamSynchronize(cs));
#undef TRY
  const int rc = plan(b);
  if (rc != MPLPXX_OK) return bail(rc);
  *out = b;
  return MPLPXX_OK;
}

int mplpxx_batch_create(int32_t count, const int32_t* n, const int32_t* L, const int64_t* m,
                        const int32_t* const* edges, const float* const* unaries, const float* const* pairwise,
                        mplpxx_batch** out) {
  return create_batch(count, n, L, m, edges, unaries, pairwise, 0, out);
}

int mplpxx_batch_create_potts(int32_t count, const int32_t* n, const int32_t* L, const int64_t* m,
                              const int32_t* const* edges, const float* const* unaries, const float* const* weights,
                              mplpxx_batch** out) {
  return create_batch(count, n, L, m, edges, unaries, weights, MPLPXX_COST_POTTS, out);
}

int mplpxx_batch_create_structured(int32_t count, const int32_t* n, const int32_t* L, const int64_t* m,
                                   const int32_t* const* edges, const float* const* unaries, int32_t kind,
                                   const float* const* params, mplpxx_batch** out) {
  if (out) *out = nullptr;
  if (!known_cost_kind(kind)) return fail(MPLPXX_EINVAL, "unknown cost kind %d", kind);
  return create_batch(count, n, L, m, edges, unaries, params, kind, out);
}

int mplpxx_batch_iterate(mplpxx_batch* b, int32_t k) {
  if (!b) return fail(MPLPXX_EINVAL, "handle is NULL");
  if (k < 0) return fail(MPLPXX_EINVAL, "k must be >= 0");
  if (b->plan_dirty) {
    const int rc = plan(b);
    if (rc != MPLPXX_OK) return rc;
  }
  HIP_TRY(hipEventRecord(b->ev0, b->stream));
  if (k > 0) {
    if (b->use_graph) {
      if (!b->gexec || b->graph_k != k) {
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        const hipError_t e = enqueue(b, k);
        const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        if (e != hipSuccess) return fail(MPLPXX_EDEVICE, "capture: %s", hipGetErrorString(e));
        if (e2 != hipSuccess) return fail(MPLPXX_EDEVICE, "end capture: %s", hipGetErrorString(e2));
        const hipError_t e3 = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) return fail(MPLPXX_EDEVICE, "instantiate: %s", hipGetErrorString(e3));
        b->graph_k = k;
      }
      HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
    } else {
      HIP_TRY(enqueue(b, k));
    }
  }
  HIP_TRY(hipEventRecord(b->ev1, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  int err[8] = {0};
  HIP_TRY(hipMemcpy(err, b->d_err, 8 * sizeof(int), hipMemcpyDeviceToHost));
  if (err[0]) {
    (void)hipMemsetAsync(b->d_err, 0, 8 * sizeof(int), b->stream);
    (void)hipStreamSynchronize(b->stream);
    return fail(err[0], "device wait exceeded its bound (workgroup %d, slot %d, node %d, expected version %d, seen %d)",
                err[1], err[2], err[3], err[4], err[5]);
  }
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  b->last_ms = ms;
  b->iterations += k;
  return MPLPXX_OK;
}

int mplpxx_batch_dual_bounds(mplpxx_batch* b, double* out) {
  if (!b || !out) return fail(MPLPXX_EINVAL, "NULL argument");
  HIP_TRY(launch_batch_dual(b->d_unaries, b->d_tables, b->d_phi, b->d_models, b->d_node_model, b->d_slot_model,
                            b->d_node_ptr, b->d_inc, b->total_nodes, b->total_slots, b->count, b->d_node_min,
                            b->d_edge_min, b->d_duals, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(hipMemcpy(out, b->d_duals, (size_t)b->count * sizeof(double), hipMemcpyDeviceToHost));
  return MPLPXX_OK;
}

int mplpxx_batch_get_state(mplpxx_batch* b, int32_t model, float* U, float* phi, float* U_comp) {
  if (!b) return fail(MPLPXX_EINVAL, "handle is NULL");
  if (model < 0 || model >= b->count) return fail(MPLPXX_EINVAL, "model index out of range");
  HIP_TRY(hipStreamSynchronize(b->stream));
  const ModelHost& h = b->mh[model];
  const BatchModel& d = b->md[model];
  if (U) HIP_TRY(hipMemcpy(U, b->d_U + d.u_off, (size_t)h.n * h.L * sizeof(float), hipMemcpyDeviceToHost));
  if (U_comp)
    HIP_TRY(hipMemcpy(U_comp, b->d_Ulo + d.u_off, (size_t)h.n * h.L * sizeof(float), hipMemcpyDeviceToHost));
  if (phi && h.m) {
    std::vector<float> tmp((size_t)h.m * 2 * h.L);
    HIP_TRY(hipMemcpy(tmp.data(), b->d_phi + d.phi_off, tmp.size() * sizeof(float), hipMemcpyDeviceToHost));
    const size_t row = 2 * (size_t)h.L;
    for (int e = 0; e < h.m; ++e)
      std::memcpy(phi + (size_t)e * row, tmp.data() + (size_t)h.slot_of_edge[e] * row, row * sizeof(float));
  }
  return MPLPXX_OK;
}

int mplpxx_batch_reset(mplpxx_batch* b) {
  if (!b) return fail(MPLPXX_EINVAL, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(hipMemsetAsync(b->d_phi, 0, (size_t)b->total_phi * sizeof(float), b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_U, b->d_unaries, (size_t)b->total_u * sizeof(float), hipMemcpyDeviceToDevice, b->stream));
  HIP_TRY(hipMemsetAsync(b->d_Ulo, 0, (size_t)b->total_u * sizeof(float), b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->iterations = 0;
  return MPLPXX_OK;
}

int mplpxx_batch_set_option(mplpxx_batch* b, int32_t key, double value) {
  if (!b) return fail(MPLPXX_EINVAL, "handle is NULL");
  switch (key) {
    case MPLPXX_BOPT_GRID:
      if (value < 0) return fail(MPLPXX_EINVAL, "grid must be >= 0");
      b->grid_opt = (int)value;
      b->plan_dirty = true;
      return MPLPXX_OK;
    case MPLPXX_BOPT_GRAPH:
      b->use_graph = value != 0;
      return MPLPXX_OK;
    case MPLPXX_BOPT_SPIN_LIMIT:
      if (value < 0) return fail(MPLPXX_EINVAL, "spin limit must be >= 0");
      b->spin_limit = value ? (long long)value : (1ll << 22);
      if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
        b->graph_k = -1;
      }
      return MPLPXX_OK;
    case MPLPXX_BOPT_ONE_PER_MODEL:
      b->one_per_model = value != 0;
      b->plan_dirty = true;
      return MPLPXX_OK;
    case MPLPXX_BOPT_LDS:
      b->use_lds = value != 0;
      b->plan_dirty = true;
      return MPLPXX_OK;
    case MPLPXX_BOPT_HANDOFF_US:
      if (!(value > 0)) return fail(MPLPXX_EINVAL, "handoff time must be > 0");
      b->t_hand_us = value;
      b->plan_dirty = true;
      return MPLPXX_OK;
    case MPLPXX_BOPT_EDGE16_US:
    case MPLPXX_BOPT_EDGE32_US:
    case MPLPXX_BOPT_EDGE64_US:
    case MPLPXX_BOPT_EDGE128_US:
      if (!(value > 0)) return fail(MPLPXX_EINVAL, "edge time must be > 0");
      b->t_edge_us[key - MPLPXX_BOPT_EDGE16_US] = value;
      b->plan_dirty = true;
      return MPLPXX_OK;
    case MPLPXX_BOPT_QUEUE:
      b->use_queue = value != 0;
      b->plan_dirty = true;
      return MPLPXX_OK;
    case MPLPXX_BOPT_ENGINE:
      if (value != 0 && value != 1 && value != 2) return fail(MPLPXX_EINVAL, "engine must be 0, 1 or 2");
      b->engine_opt = (int)value;
      b->plan_dirty = true;
      return MPLPXX_OK;
    case MPLPXX_BOPT_WAVE_EDGE16_US:
    case MPLPXX_BOPT_WAVE_EDGE32_US:
    case MPLPXX_BOPT_WAVE_EDGE64_US:
      if (!(value > 0)) return fail(MPLPXX_EINVAL, "edge time must be > 0");
      b->wv_edge_us[key - MPLPXX_BOPT_WAVE_EDGE16_US] = value;
      b->plan_dirty = true;
      return MPLPXX_OK;
    case MPLPXX_BOPT_WAVE_LAT_LDS_US:
      if (!(value > 0)) return fail(MPLPXX_EINVAL, "latency must be > 0");
      b->wv_lat_lds_us = value;
      b->plan_dirty = true;
      return MPLPXX_OK;
    case MPLPXX_BOPT_WAVE_LAT_MB_US:
      if (!(value > 0)) return fail(MPLPXX_EINVAL, "latency must be > 0");
      b->wv_lat_mb_us = value;
      b->plan_dirty = true;
      return MPLPXX_OK;
    default:
      return fail(MPLPXX_EINVAL, "unknown batch option %d", key);
  }
}

int mplpxx_batch_wg_profile(mplpxx_batch* b, double* start_end_us, int32_t* team_model) {
  if (!b || !start_end_us) return fail(MPLPXX_EINVAL, "NULL argument");
  if (b->plan_dirty) {
    const int rc = plan(b);
    if (rc != MPLPXX_OK) return rc;
  }
  std::vector<long long> t((size_t)b->grid * 2);
  HIP_TRY(hipMemcpyAsync(t.data(), b->d_wg_time, t.size() * sizeof(long long), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  long long t0 = t.empty() ? 0 : t[0];
  for (int w = 0; w < b->grid; ++w) t0 = std::min(t0, t[2 * w]);
  for (int w = 0; w < b->grid; ++w) {
    start_end_us[2 * w] = (double)(t[2 * w] - t0) / 100.0;
    start_end_us[2 * w + 1] = (double)(t[2 * w + 1] - t0) / 100.0;
    if (team_model) team_model[w] = b->wg_team_model[w];
  }
  return MPLPXX_OK;
}

int mplpxx_batch_get_info(mplpxx_batch* b, int32_t key, double* value) {
  if (!b || !value) return fail(MPLPXX_EINVAL, "NULL argument");
  if (b->plan_dirty) {
    const int rc = plan(b);
    if (rc != MPLPXX_OK) return rc;
  }
  switch (key) {
    case MPLPXX_BINFO_COUNT: *value = b->count; return MPLPXX_OK;
    case MPLPXX_BINFO_GRID: *value = b->grid; return MPLPXX_OK;
    case MPLPXX_BINFO_TASKS: *value = b->ntasks; return MPLPXX_OK;
    case MPLPXX_BINFO_TEAMS: *value = b->nteams; return MPLPXX_OK;
    case MPLPXX_BINFO_MAX_TEAM: *value = b->max_team; return MPLPXX_OK;
    case MPLPXX_BINFO_PLAN_US: *value = b->plan_us; return MPLPXX_OK;
    case MPLPXX_BINFO_EDGES: *value = b->total_slots; return MPLPXX_OK;
    case MPLPXX_BINFO_LAST_MS: *value = b->last_ms; return MPLPXX_OK;
    case MPLPXX_BINFO_TABLE_BYTES: *value = (double)b->total_tables * sizeof(float); return MPLPXX_OK;
    case MPLPXX_BINFO_LDS_TASKS: *value = b->lds_tasks; return MPLPXX_OK;
    case MPLPXX_BINFO_LDS_BYTES: *value = (double)b->lds_bytes; return MPLPXX_OK;
    case MPLPXX_BINFO_ENGINE: *value = b->wave ? 2 : 1; return MPLPXX_OK;
    case MPLPXX_BINFO_WAVES: *value = b->wave ? b->wv_waves : 4; return MPLPXX_OK;
    case MPLPXX_BINFO_WG_MAX_US:
    case MPLPXX_BINFO_WG_MEAN_US: {
      // start-to-end time of the workgroups in the last launch (100 MHz clock)
      std::vector<long long> t((size_t)b->grid * 2);
      HIP_TRY(hipMemcpyAsync(t.data(), b->d_wg_time, t.size() * sizeof(long long), hipMemcpyDeviceToHost, b->stream));
      HIP_TRY(hipStreamSynchronize(b->stream));
      double mx = 0.0, sum = 0.0;
      for (int w = 0; w < b->grid; ++w) {
        const double d = (double)(t[2 * w + 1] - t[2 * w]) / 100.0;
        mx = std::max(mx, d);
        sum += d;
      }
      *value = key == MPLPXX_BINFO_WG_MAX_US ? mx : sum / std::max(1, b->grid);
      return MPLPXX_OK;
    }
    default: return fail(MPLPXX_EINVAL, "unknown batch info key %d", key);
  }
}

void mplpxx_batch_destroy(mplpxx_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  free_batch(b);
  delete b;
}

}  // extern "C"
