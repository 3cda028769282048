// C ABI of the batched form (declared in include/pedsim.h).
//
// A batch holds up to `capacity` independent scenarios, each with its own
// caller-owned planes and scratch. A step call advances each scenario by its
// own number of steps in shared launches of the persistent batch kernel: the
// host writes the per-scenario descriptors and the per-launch work tables
// into a pinned staging buffer, copies them into the caller-owned device
// workspace with one asynchronous copy, and replays a captured hipGraph of
// the launch sequence (one graph per launch count, instantiated on first
// use). Calls with more launches than one graph holds are split.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "pedsim.h"
#include "pedsim_internal.hpp"

using namespace pedsim;

namespace {

struct HostSlot {
  bool used = false;
  sim_params p;
  int mode = 0;
  Planes user{}, shadow{};
  ScratchLayout L{};
  Scenario S{};
  uint32_t* stats = nullptr;
  unsigned long long* totals = nullptr;
  int stats_entries = 0;
  uint64_t t = 0;
  uint64_t agents = 0;
};

// Byte offsets of the tables inside the workspace (and the staging copy).
struct BatchLayout {
  size_t slots, entries, counts, totals, counters, upload, total;
};

BatchLayout batch_layout(int capacity) {
  BatchLayout L;
  L.slots = 0;
  L.entries = L.slots + round_up((size_t)capacity * sizeof(BatchSlot));
  L.counts = L.entries + round_up((size_t)kBatchMaxLaunches * capacity * sizeof(BatchEntry));
  L.totals = L.counts + round_up((size_t)kBatchMaxLaunches * sizeof(int));
  L.upload = L.totals + round_up((size_t)kBatchMaxLaunches * sizeof(int));  // bytes copied per call
  L.counters = L.upload;
  L.total = L.counters + round_up((size_t)kBatchMaxLaunches * sizeof(unsigned));
  return L;
}

}  // namespace

struct sim_batch {
  int capacity;
  uint8_t* ws;
  BatchLayout L;
  uint8_t* staging;  // pinned host copy of the uploaded tables
  hipEvent_t uploaded;
  bool upload_pending;
  hipStream_t capture;  // private stream the launch sequences are captured on
  std::vector<HostSlot> slots;
  std::vector<int> order;  // slots in the order their tiles are claimed
  Tiling tl;
  int wgs_per_cu;
  int use_graph;
  bool nb8;   // every scenario uses the eight-neighbour candidate set
  bool tour;  // a tour-variant scenario has been added (the LDS layout holds tour lengths)
  hipGraphExec_t graphs[kBatchMaxLaunches + 1];

  BatchPlan plan() const {
    BatchPlan P;
    P.slots = (const BatchSlot*)(ws + L.slots);
    P.entries = (const BatchEntry*)(ws + L.entries);
    P.counts = (const int*)(ws + L.counts);
    P.totals = (const int*)(ws + L.totals);
    P.counters = (unsigned*)(ws + L.counters);
    P.capacity = capacity;
    P.k = tl.steps;
    P.rows = tl.rows;
    P.nb8 = nb8 ? 1 : 0;
    P.tour = tour ? 1 : 0;
    return P;
  }
  void drop_graphs() {
    for (int i = 0; i <= kBatchMaxLaunches; ++i)
      if (graphs[i]) {
        (void)hipGraphExecDestroy(graphs[i]);
        graphs[i] = nullptr;
      }
  }
};

namespace {

// The eight-neighbour set runs on the row-lane engine with the pheromone in
// LDS: two 512-thread workgroups per compute unit.
Tiling default_batch_tiling(bool lds_form = false) {
  static const Tiling opts[] = {{3, 62, 4, 256}, {3, 62, 3, 256}, {1, 32, 1, 256}};
  static const Tiling opts8[] = {{0, 48, 3, 512}, {0, 40, 2, 512}, {0, 32, 1, 256}};
  const Tiling* o = lds_form ? opts8 : opts;
  for (int i = 0; i < 3; ++i)
    if (tiling_valid(o[i], lds_form ? kModeAcoTour : kModeAco, max_dynamic_lds() - kBatchItemBytes, lds_form))
      return o[i];
  return o[2];
}

bool slot_geometry(const Tiling& tl, HostSlot& hs, bool nb8) {
  Scenario S = base_scenario(&hs.p);
  S.neighbours = nb8 ? 8 : 5;
  set_geometry(S, tl);
  if (S.tiles_x * S.tiles_y > hs.L.stats_cap) return false;
  S.tile_stats = hs.stats;
  hs.S = S;
  return true;
}

// Enqueue one call's launch sequence on stream s: replay a cached graph
// (captured once on the batch's private stream; the caller's stream may be
// the null stream, which cannot be captured) or launch directly.
int enqueue_sequence(sim_batch* b, int launches, hipStream_t s) {
  const BatchPlan P = b->plan();
  const int grid = device_cu_count() * b->wgs_per_cu;
  auto issue = [&](hipStream_t on) -> hipError_t {
    hipError_t e = launch_batch_reset(P, launches, on);
    for (int j = 0; e == hipSuccess && j < launches; ++j) e = launch_batch(P, b->tl, j, grid, on);
    if (e == hipSuccess) e = launch_batch_copyback(P, b->capacity, on);
    return e;
  };
  if (!b->use_graph) {
    PEDSIM_HIP(issue(s));
    return SIM_OK;
  }
  if (!b->graphs[launches]) {
    hipGraph_t g = nullptr;
    PEDSIM_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    const hipError_t e = issue(b->capture);
    const hipError_t e2 = hipStreamEndCapture(b->capture, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(e != hipSuccess ? e : e2, "capture of the batch launch sequence", __LINE__);
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    PEDSIM_HIP(e3);
    b->graphs[launches] = exec;
  }
  PEDSIM_HIP(hipGraphLaunch(b->graphs[launches], s));
  return SIM_OK;
}

// One call of at most kBatchMaxLaunches launches; steps[i] per slot.
int run_chunk(sim_batch* b, const std::vector<int>& steps, hipStream_t s) {
  const int k = b->tl.steps;
  int launches = 0;
  for (int i = 0; i < b->capacity; ++i)
    if (steps[i] > 0) {
      const int l = (steps[i] + k - 1) / k;
      launches = l > launches ? l : launches;
    }
  if (launches == 0) return SIM_OK;
  // the previous upload must have left the staging buffer
  if (b->upload_pending) PEDSIM_HIP(hipEventSynchronize(b->uploaded));
  BatchSlot* hs = (BatchSlot*)(b->staging + b->L.slots);
  BatchEntry* he = (BatchEntry*)(b->staging + b->L.entries);
  int* hc = (int*)(b->staging + b->L.counts);
  int* ht = (int*)(b->staging + b->L.totals);
  memset(hs, 0, (size_t)b->capacity * sizeof(BatchSlot));
  for (int i = 0; i < b->capacity; ++i) {
    const HostSlot& x = b->slots[i];
    if (!x.used || steps[i] <= 0) continue;
    BatchSlot& d = hs[i];
    d.S = x.S;
    d.code[0] = x.user.code;
    d.code[1] = x.shadow.code;
    d.id[0] = x.user.id;
    d.id[1] = x.shadow.id;
    d.tau[0] = x.user.tau;
    d.tau[1] = x.shadow.tau;
    d.tour[0] = x.user.tour;
    d.tour[1] = x.shadow.tour;
    d.agents = (uint32_t)x.agents;
    d.t0 = x.t;
    d.steps = steps[i];
    d.mode = x.mode;
  }
  // Workgroups claim tiles in entry order: the scenarios with the most agents
  // per tile (the costliest tiles) first, so the last tiles claimed in a
  // launch are cheap ones and its tail is short. The order decides only who
  // takes which tile, never a result.
  int* order = b->order.data();
  int nused = 0;
  for (int i = 0; i < b->capacity; ++i)
    if (b->slots[i].used && steps[i] > 0) order[nused++] = i;
  std::stable_sort(order, order + nused, [&](int u, int v) {
    const HostSlot& a = b->slots[u];
    const HostSlot& c = b->slots[v];
    return (double)a.agents * (double)(c.S.tiles_x * c.S.tiles_y) >
           (double)c.agents * (double)(a.S.tiles_x * a.S.tiles_y);
  });
  for (int j = 0; j < launches; ++j) {
    int n = 0, first = 0;
    for (int o = 0; o < nused; ++o) {
      const int i = order[o];
      if (steps[i] <= j * k) continue;
      he[(size_t)j * b->capacity + n] = BatchEntry{i, first};
      first += b->slots[i].S.tiles_x * b->slots[i].S.tiles_y;
      ++n;
    }
    hc[j] = n;
    ht[j] = first;
  }
  PEDSIM_HIP(hipMemcpyAsync(b->ws, b->staging, b->L.upload, hipMemcpyHostToDevice, s));
  PEDSIM_HIP(hipEventRecord(b->uploaded, s));
  b->upload_pending = true;
  const int rc = enqueue_sequence(b, launches, s);
  if (rc) return rc;
  for (int i = 0; i < b->capacity; ++i) {
    HostSlot& x = b->slots[i];
    if (!x.used || steps[i] <= 0) continue;
    x.t += (uint64_t)steps[i];
    x.stats_entries = x.S.tiles_x * x.S.tiles_y;
  }
  return SIM_OK;
}

}  // namespace

extern "C" {

int sim_batch_workspace_bytes(int32_t capacity, size_t* out) {
  if (capacity < 1 || capacity > 65535 || !out) return SIM_EINVAL;
  *out = batch_layout(capacity).total;
  return SIM_OK;
}

int sim_batch_create(int32_t capacity, void* d_workspace, size_t workspace_bytes, sim_batch** out) {
  if (!out || capacity < 1 || capacity > 65535) return SIM_EINVAL;
  *out = nullptr;
  const BatchLayout L = batch_layout(capacity);
  if (!d_workspace || workspace_bytes < L.total) return SIM_ESCRATCH;
  prepare_batch_kernels();
  sim_batch* b = new (std::nothrow) sim_batch;
  if (!b) return SIM_EINVAL;
  b->capacity = capacity;
  b->ws = (uint8_t*)d_workspace;
  b->L = L;
  b->staging = nullptr;
  b->upload_pending = false;
  b->tl = default_batch_tiling();
  b->wgs_per_cu = 4;  // the default streaming tiling needs ~40 KB of LDS: four workgroups fit a CU
  b->use_graph = 1;
  b->nb8 = false;
  b->tour = false;
  for (int i = 0; i <= kBatchMaxLaunches; ++i) b->graphs[i] = nullptr;
  b->slots.resize(capacity);
  b->order.resize(capacity);
  hipError_t e = hipHostMalloc((void**)&b->staging, L.upload, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipHostMalloc(staging)", __LINE__);
  }
  e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipHostFree(b->staging);
    delete b;
    return hip_fail(e, "hipEventCreateWithFlags", __LINE__);
  }
  e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
  if (e != hipSuccess) {
    (void)hipEventDestroy(b->uploaded);
    (void)hipHostFree(b->staging);
    delete b;
    return hip_fail(e, "hipStreamCreateWithFlags", __LINE__);
  }
  *out = b;
  return SIM_OK;
}

int sim_batch_add(sim_batch* b, const sim_params* p, int32_t mode, uint8_t* d_code, uint32_t* d_id, float* d_tau,
                  void* d_scratch, size_t scratch_bytes, void* stream, int32_t* slot) {
  if (!b || !slot) return SIM_EINVAL;
  int e = check_params(p);
  if (e) return e;
  if (mode != kModeLem && mode != kModeAco && mode != kModeAcoTour) return SIM_EINVAL;
  if (!d_code || !d_id) return SIM_EINVAL;
  if (mode != kModeLem && !d_tau) return SIM_ENOTAU;
  if (mode == kModeAcoTour) {  // the row-lane engine with the pheromone and tour lengths in LDS
    if (b->tl.nw != 0 || !tiling_valid(b->tl, kModeAcoTour, max_dynamic_lds() - kBatchItemBytes, b->nb8))
      return SIM_EINVAL;
  }
  const ScratchLayout L = layout_of(p);
  if (!d_scratch || scratch_bytes < L.total) return SIM_ESCRATCH;
  int free_slot = -1;
  for (int i = 0; i < b->capacity; ++i)
    if (!b->slots[i].used) {
      free_slot = i;
      break;
    }
  if (free_slot < 0) return SIM_EFULL;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* scratch = (uint8_t*)d_scratch;
  uint64_t agents = 0;
  e = validate_state(p, d_code, d_id, d_tau, scratch, L, s, &agents);
  if (e) return e;
  HostSlot hs;
  hs.agents = agents;
  hs.p = *p;
  hs.mode = mode;
  hs.user = Planes{d_code, d_id, d_tau};
  hs.shadow = Planes{scratch + L.code2, (uint32_t*)(scratch + L.id2), d_tau ? (float*)(scratch + L.tau2) : nullptr};
  hs.L = L;
  hs.stats = (uint32_t*)(scratch + L.stats);
  hs.totals = (unsigned long long*)(scratch + L.totals);
  hs.t = p->step0;
  if (!slot_geometry(b->tl, hs, b->nb8)) return SIM_EINVAL;
  PEDSIM_HIP(launch_count(d_code, p->W, p->H, p->cross_a, p->cross_b, hs.stats, &hs.stats_entries, s));
  // the slot's counters are complete once the call returns, so a step call on
  // another stream may follow without an event
  PEDSIM_HIP(hipStreamSynchronize(s));
  hs.used = true;
  b->slots[free_slot] = hs;
  if (mode == kModeAcoTour && !b->tour) {
    b->tour = true;
    b->drop_graphs();  // the launches now reserve LDS for tour lengths
  }
  *slot = free_slot;
  return SIM_OK;
}

int sim_batch_remove(sim_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->capacity || !b->slots[slot].used) return SIM_EINVAL;
  b->slots[slot] = HostSlot();
  return SIM_OK;
}

int sim_batch_step_slots(sim_batch* b, const int32_t* steps, int32_t n, void* stream) {
  if (!b || !steps || n < 0 || n > b->capacity) return SIM_EINVAL;
  std::vector<int> remaining(b->capacity, 0);
  for (int i = 0; i < n; ++i) {
    if (steps[i] < 0) return SIM_EINVAL;
    if (steps[i] > 0 && !b->slots[i].used) return SIM_EINVAL;
    if (steps[i] > 0 && b->slots[i].mode == kModeAcoTour && b->slots[i].agents > 0 && !b->slots[i].user.tour)
      return SIM_ENOTOUR;
    remaining[i] = steps[i];
  }
  hipStream_t s = (hipStream_t)stream;
  const int per_call = kBatchMaxLaunches * b->tl.steps;
  for (;;) {
    std::vector<int> now(b->capacity, 0);
    bool any = false;
    for (int i = 0; i < b->capacity; ++i) {
      now[i] = remaining[i] < per_call ? remaining[i] : per_call;
      remaining[i] -= now[i];
      any = any || now[i] > 0;
    }
    if (!any) break;
    const int rc = run_chunk(b, now, s);
    if (rc) return rc;
  }
  return SIM_OK;
}

int sim_batch_step(sim_batch* b, int32_t nsteps, void* stream) {
  if (!b || nsteps < 0) return SIM_EINVAL;
  std::vector<int32_t> steps(b->capacity, 0);
  for (int i = 0; i < b->capacity; ++i)
    if (b->slots[i].used) steps[i] = nsteps;
  return sim_batch_step_slots(b, steps.data(), b->capacity, stream);
}

int sim_batch_stats(sim_batch* b, int32_t slot, sim_stats_t* out, void* stream) {
  if (!b || !out || slot < 0 || slot >= b->capacity || !b->slots[slot].used) return SIM_EINVAL;
  const HostSlot& x = b->slots[slot];
  hipStream_t s = (hipStream_t)stream;
  unsigned long long v[kTileStatFields];
  PEDSIM_HIP(launch_reduce_counts(x.stats, x.stats_entries, x.totals, s));
  PEDSIM_HIP(hipMemcpyAsync(v, x.totals, sizeof(v), hipMemcpyDeviceToHost, s));
  PEDSIM_HIP(hipStreamSynchronize(s));
  out->step = x.t;
  out->agents_a = v[0];
  out->agents_b = v[1];
  out->crossed_a = v[2];
  out->crossed_b = v[3];
  out->moved_last = v[4];
  return SIM_OK;
}

int sim_batch_set_tuning(sim_batch* b, int32_t nw, int32_t rows, int32_t steps_per_launch, int32_t threads,
                         int32_t wgs_per_cu, int32_t use_graph) {
  if (!b || wgs_per_cu < 1 || wgs_per_cu > 32) return SIM_EINVAL;
  const Tiling tl{nw, rows, steps_per_launch, threads};
  if (!tiling_valid(tl, b->tour ? kModeAcoTour : kModeAco, max_dynamic_lds() - kBatchItemBytes, b->nb8))
    return SIM_EINVAL;
  for (int i = 0; i < b->capacity; ++i) {
    if (!b->slots[i].used) continue;
    HostSlot probe = b->slots[i];
    if (!slot_geometry(tl, probe, b->nb8)) return SIM_EINVAL;
  }
  b->tl = tl;
  for (int i = 0; i < b->capacity; ++i)
    if (b->slots[i].used) slot_geometry(tl, b->slots[i], b->nb8);
  b->wgs_per_cu = wgs_per_cu;
  b->use_graph = use_graph ? 1 : 0;
  b->drop_graphs();
  return SIM_OK;
}

int sim_batch_attach_tour(sim_batch* b, int32_t slot, float* d_tour, float* d_tour_shadow, void* stream) {
  if (!b || slot < 0 || slot >= b->capacity || !b->slots[slot].used) return SIM_EINVAL;
  HostSlot& x = b->slots[slot];
  if (x.mode != kModeAcoTour) return SIM_EINVAL;
  if (x.agents > 0 && (!d_tour || !d_tour_shadow || d_tour == d_tour_shadow)) return SIM_EINVAL;
  if (x.agents > 0) {
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* counters = x.totals + kTileStatFields;
    unsigned long long host_counters[3];
    PEDSIM_HIP(launch_zero_words(counters, 3 * sizeof(unsigned long long) / 4, s));
    PEDSIM_HIP(launch_validate_values(d_tour, (size_t)x.agents, counters, s));
    PEDSIM_HIP(hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, s));
    PEDSIM_HIP(hipStreamSynchronize(s));
    if (host_counters[2]) return SIM_ESTATE;
  }
  x.user.tour = d_tour;
  x.shadow.tour = d_tour_shadow;
  return SIM_OK;
}

int sim_batch_set_neighbours(sim_batch* b, int32_t n) {
  if (!b || (n != 5 && n != 8)) return SIM_EINVAL;
  const bool nb8 = n == 8;
  const Tiling tl = default_batch_tiling(nb8 || b->tour);
  for (int i = 0; i < b->capacity; ++i) {
    if (!b->slots[i].used) continue;
    HostSlot probe = b->slots[i];
    if (!slot_geometry(tl, probe, nb8)) return SIM_EINVAL;
  }
  b->nb8 = nb8;
  b->tl = tl;
  b->wgs_per_cu = (nb8 || b->tour) ? 2 : 4;
  for (int i = 0; i < b->capacity; ++i)
    if (b->slots[i].used) slot_geometry(tl, b->slots[i], nb8);
  b->drop_graphs();
  return SIM_OK;
}

int sim_batch_get_tuning(sim_batch* b, int32_t out[6]) {
  if (!b || !out) return SIM_EINVAL;
  out[0] = b->tl.nw;
  out[1] = b->tl.rows;
  out[2] = b->tl.steps;
  out[3] = b->tl.threads;
  out[4] = b->wgs_per_cu;
  out[5] = b->use_graph;
  return SIM_OK;
}

void sim_batch_destroy(sim_batch* b) {
  if (!b) return;
  if (b->upload_pending) (void)hipEventSynchronize(b->uploaded);
  b->drop_graphs();
  (void)hipStreamDestroy(b->capture);
  (void)hipEventDestroy(b->uploaded);
  (void)hipHostFree(b->staging);
  delete b;
}

}  // extern "C"
