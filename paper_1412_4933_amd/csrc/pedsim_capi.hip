// C ABI of the single-scenario step (declared in include/pedsim.h).
//
// The state lives in the caller's planes between calls. Within a call the
// tile engine ping-pongs between the caller's planes and a copy in the
// scratch buffer (every launch reads one set and writes the other, because a
// tile's halo is its neighbours' interior); the call ends with the state back
// in the caller's planes.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "pedsim.h"
#include "pedsim_internal.hpp"
#include "range_step.hpp"

namespace pedsim {

static thread_local char g_last_error[256] = "";

int hip_fail(hipError_t e, const char* what, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s (%d) from %.150s at line %d", hipGetErrorString(e), (int)e,
           what, line);
  return SIM_EHIP;
}

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

static int count_entries(int W, int H) { return ((W + 63) / 64) * ((H + 3) / 4); }

ScratchLayout layout_of(const sim_params* p) {
  ScratchLayout L;
  const size_t cells = (size_t)p->W * (size_t)p->H;
  const int max_tiles = ((p->W + kMinInteriorX - 1) / kMinInteriorX) * ((p->H + kMinInteriorY - 1) / kMinInteriorY);
  const int ce = count_entries(p->W, p->H);
  L.stats_cap = max_tiles > ce ? max_tiles : ce;
  L.code2 = 0;
  L.id2 = L.code2 + round_up(cells);
  L.tau2 = L.id2 + round_up(cells * 4);
  L.stats = L.tau2 + round_up(cells * 8);
  L.totals = L.stats + round_up((size_t)L.stats_cap * kTileStatFields * 4);
  L.order = L.totals + round_up(8 * sizeof(unsigned long long));
  L.total = L.order + round_up((size_t)3 * (16 + L.stats_cap) * 4);
  return L;
}

int check_params(const sim_params* p) {
  if (!p) return SIM_EINVAL;
  if (p->W < 1 || p->H < 1) return SIM_EINVAL;
  if ((int64_t)p->W * (int64_t)p->H >= ((int64_t)1 << 31)) return SIM_EINVAL;
  if ((p->H + 3) / 4 > 65535) return SIM_EINVAL;  // count-kernel grid rows
  if (!(p->rho > 0.0f && p->rho <= 1.0f)) return SIM_EINVAL;
  if (!(p->dtau >= 0.0f && p->dtau <= 3.402823466e38f)) return SIM_EINVAL;
  if (p->alpha < 0 || p->alpha > 8 || p->beta < 0 || p->beta > 8) return SIM_EINVAL;
  if (p->cross_a < 0 || p->cross_a > p->W || p->cross_b < 0 || p->cross_b > p->W) return SIM_EINVAL;
  return SIM_OK;
}

// eta^beta = D2^(-beta/2) for the squared distance D2 from a candidate to the
// point two cells ahead (diagonal 2, lateral 5), rounded to float.
static float heuristic(double d2, int beta) { return (float)pow(d2, -0.5 * (double)beta); }

Scenario base_scenario(const sim_params* p) {
  Scenario S;
  memset(&S, 0, sizeof(S));
  S.W = p->W;
  S.H = p->H;
  S.key0 = (uint32_t)p->seed;
  S.key1 = (uint32_t)(p->seed >> 32);
  const float rho = p->rho;
  S.keep = 1.0f - rho;
  S.dtau = p->dtau;
  S.eta_diag = heuristic(2.0, p->beta);
  S.eta_lat = heuristic(5.0, p->beta);
  S.step_diag = sqrtf(2.0f);
  S.eta_back = heuristic(9.0, p->beta);
  S.eta_back_diag = heuristic(10.0, p->beta);
  S.neighbours = 5;
  S.alpha = p->alpha;
  S.cross_a = p->cross_a;
  S.cross_b = p->cross_b;
  return S;
}

void set_geometry(Scenario& S, const Tiling& tl) {
  S.halo = 3 * tl.steps;
  S.IX = region_cols(tl) - 2 * S.halo;
  S.IY = tl.rows - 2 * S.halo;
  S.tiles_x = (S.W + S.IX - 1) / S.IX;
  S.tiles_y = (S.H + S.IY - 1) / S.IY;
}

// Validate caller planes on the device (codes, id/code consistency, ids
// exactly 1..N, pheromone finite and >= 0); synchronises the stream.
int validate_state(const sim_params* p, const uint8_t* d_code, const uint32_t* d_id, const float* d_tau,
                   uint8_t* scratch, const ScratchLayout& L, hipStream_t s, uint64_t* agents) {
  const size_t cells = (size_t)p->W * (size_t)p->H;
  unsigned long long* counters = (unsigned long long*)(scratch + L.totals) + kTileStatFields;
  unsigned long long host_counters[3];
  PEDSIM_HIP(launch_zero_words(counters, 3 * sizeof(unsigned long long) / 4, s));
  PEDSIM_HIP(launch_validate(d_code, d_id, d_tau, cells, counters, s));
  PEDSIM_HIP(hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, s));
  PEDSIM_HIP(hipStreamSynchronize(s));
  if (host_counters[2]) return SIM_ESTATE;
  const unsigned long long n = host_counters[0] + host_counters[1];
  if (agents) *agents = n;
  if (n > 0) {
    uint32_t* bitmap = (uint32_t*)(scratch + L.id2);
    PEDSIM_HIP(launch_zero_words(bitmap, (n + 31) / 32, s));
    PEDSIM_HIP(launch_validate_ids(d_id, cells, (uint32_t)n, bitmap, counters, s));
    PEDSIM_HIP(hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, s));
    PEDSIM_HIP(hipStreamSynchronize(s));
    if (host_counters[2]) return SIM_ESTATE;
  }
  return SIM_OK;
}

}  // namespace pedsim

using namespace pedsim;

namespace {

// Default tiling by grid size (measured on MI355X): the row-lane engine,
// with more steps per launch on smaller grids (their launches are short, so
// the fixed cost of a launch weighs more than the wider halo), and its
// streaming form on large grids (many tiles per compute unit: the smaller
// LDS footprint lets four or five workgroups overlap). The first shape that
// fits the device's LDS is used.
// The tour variant runs on the row-lane engine with the pheromone in LDS
// (its deposits depend on per-move tour lengths, so they are applied in LDS
// as they happen; its per-cell tour lengths take the LDS of the contest
// tickets, which it draws again instead). The eight-neighbour set (LEM, ACO)
// also needs the pheromone in LDS.
Tiling default_tiling(int mode, size_t cells, bool nb8 = false) {
  static const Tiling tiny_opts[] = {{0, 48, 6, 512}, {0, 32, 4, 256}, {1, 32, 1, 256}};
  static const Tiling small_opts[] = {{0, 52, 5, 512}, {0, 52, 4, 512}, {1, 32, 1, 256}};
  static const Tiling large_opts[] = {{3, 62, 3, 256}, {0, 48, 2, 512}, {1, 32, 1, 256}};
  static const Tiling tour_tiny[] = {{0, 48, 6, 512}, {0, 32, 4, 256}, {0, 32, 1, 256}};
  static const Tiling tour_small[] = {{0, 52, 5, 512}, {0, 52, 4, 512}, {0, 32, 1, 256}};
  static const Tiling tour_large[] = {{0, 56, 3, 512}, {0, 56, 2, 512}, {0, 32, 1, 256}};
  static const Tiling nb8_tiny[] = {{0, 48, 6, 512}, {0, 32, 4, 256}, {0, 32, 1, 256}};
  static const Tiling nb8_small[] = {{0, 52, 5, 512}, {0, 52, 4, 512}, {0, 32, 1, 256}};
  static const Tiling nb8_large[] = {{0, 64, 3, 512}, {0, 64, 2, 512}, {0, 32, 1, 256}};
  const int size = cells < ((size_t)1 << 18) ? 0 : (cells < ((size_t)2 << 20) ? 1 : 2);
  const Tiling* const plain[3] = {tiny_opts, small_opts, large_opts};
  const Tiling* const tour[3] = {tour_tiny, tour_small, tour_large};
  const Tiling* const eight[3] = {nb8_tiny, nb8_small, nb8_large};
  const Tiling* opts = mode == kModeAcoTour ? tour[size] : (nb8 ? eight[size] : plain[size]);
  for (int i = 0; i < 3; ++i)
    if (tiling_valid(opts[i], mode, max_dynamic_lds(), nb8)) return opts[i];
  return opts[2];
}

}  // namespace

struct sim_handle {
  sim_params p;
  Planes user;     // caller-owned state
  Planes shadow;   // copy in scratch
  uint32_t* stats;
  int stats_cap;
  int stats_entries;
  unsigned long long* totals;
  Scenario base;   // parameters shared by every launch
  Tiling tiling[3];
  uint64_t t;      // index of the next step
  uint64_t agents; // number of agents (ids 1..agents)
  // Larger scanning and moving ranges: scan = 0 runs the base engines;
  // otherwise LEM and ACO steps run the range kernel with these ranges on
  // tiles of range_cols x range_rows cells, range_threads per workgroup.
  int scan, move;
  int range_cols, range_rows, range_steps, range_threads;
  float range_eta[2][kRangeMax];
  // tile order of the row-lane launches (see Scenario::order): the tiling
  // the rotations were written for, the rotation the next launch takes and
  // whether it holds a complete order
  uint32_t* order;
  Tiling order_tl;
  int order_mode;
  int order_rot;
  bool order_valid;
  bool order_on;  // the tile grid has more tiles than the device runs at once
};

namespace {

hipError_t copy_planes(const Planes& dst, const Planes& src, size_t cells, bool tau, size_t tour, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(dst.code, src.code, cells, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dst.id, src.id, cells * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && tau) e = hipMemcpyAsync(dst.tau, src.tau, cells * 8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && tour) e = hipMemcpyAsync(dst.tour, src.tour, tour * 4, hipMemcpyDeviceToDevice, s);
  return e;
}

// Launch plan for n steps: chunks of at most tl.steps, with an even number of
// launches when possible so the state ends in the caller's planes.
int plan(int nsteps, int per, int* chunks, int cap) {
  int n = 0;
  for (int done = 0; done < nsteps && n < cap; ++n) {
    chunks[n] = nsteps - done < per ? nsteps - done : per;
    done += chunks[n];
  }
  if ((n & 1) && n < cap) {
    for (int j = n - 1; j >= 0; --j)
      if (chunks[j] >= 2) {
        for (int m = n; m > j + 1; --m) chunks[m] = chunks[m - 1];
        chunks[j + 1] = chunks[j] / 2;
        chunks[j] -= chunks[j + 1];
        ++n;
        break;
      }
  }
  return n;
}

// eta^beta of a side ray with ranges (S, M): the float nearest to
// (f/S)^beta D2^(-beta/2), D2 the squared distance from the landing cell
// (k = min(f, M) cells along the ray; a = 1 for a diagonal, 0 for a lateral)
// to the point M+1 cells ahead. Evaluated in long double, then rounded once.
static float range_eta(int a, int f, int S, int M, int beta) {
  const int k = f < M ? f : M;
  const long double dx = (long double)(M + 1 - a * k);
  const long double d2 = dx * dx + (long double)k * (long double)k;
  const long double v = powl((long double)f / (long double)S, (long double)beta) * powl(d2, -0.5L * (long double)beta);
  return (float)v;
}

static void fill_range_eta(int S, int M, int beta, float out[2][kRangeMax]) {
  for (int f = 1; f <= kRangeMax; ++f) {
    out[0][f - 1] = f <= S ? range_eta(0, f, S, M, beta) : 0.0f;
    out[1][f - 1] = f <= S ? range_eta(1, f, S, M, beta) : 0.0f;
  }
}

// Range tiling is valid when the interior is at least 16 x 8 (bounds the
// per-tile counters), the steps per launch are 1..4 and the workgroup's LDS
// fits.
static bool range_tiling_valid(int cols, int rows, int steps, int threads, int S, int M) {
  if (cols < kMinInteriorX || cols > 256 || rows < kMinInteriorY || rows > 256) return false;
  if (steps < 1 || steps > kRangeMaxSteps) return false;
  if (threads < 64 || threads > kRangeMaxThreads || threads % 64) return false;
  return RangeLayout{cols, rows, S, M, steps, true}.bytes() <= (size_t)max_dynamic_lds();
}

// Default range tiling: 64 x 32 interiors, two steps per launch where the
// LDS allows, 512 threads per workgroup; smaller shapes for long ranges.
static bool default_range_tiling(sim_handle* h) {
  static const int shapes[][3] = {{64, 32, 2}, {64, 16, 2}, {64, 32, 1}, {64, 16, 1}, {64, 8, 1},
                                  {32, 16, 1}, {32, 8, 1},  {16, 8, 1}};
  for (const auto& sh : shapes)
    if (range_tiling_valid(sh[0], sh[1], sh[2], 512, h->scan, h->move)) {
      h->range_cols = sh[0];
      h->range_rows = sh[1];
      h->range_steps = sh[2];
      h->range_threads = 512;
      return true;
    }
  return false;
}

// Range launches of up to range_steps steps each, ping-ponging between the
// caller's planes and the shadow copy like the tile engines.
int run_range_steps(sim_handle* h, int mode, int32_t nsteps, hipStream_t s, hipEvent_t* ev, double* ms,
                    int64_t* launches) {
  const size_t cells = (size_t)h->p.W * (size_t)h->p.H;
  const bool aco = mode != kModeLem;
  RangeScenario P;
  memset(&P, 0, sizeof(P));
  P.W = h->p.W;
  P.H = h->p.H;
  P.TX = h->range_cols;
  P.TY = h->range_rows;
  P.tiles_x = (P.W + P.TX - 1) / P.TX;
  P.tiles_y = (P.H + P.TY - 1) / P.TY;
  P.S = h->scan;
  P.M = h->move;
  P.key0 = h->base.key0;
  P.key1 = h->base.key1;
  P.keep = h->base.keep;
  P.dtau = h->base.dtau;
  P.alpha = h->base.alpha;
  P.cross_a = h->base.cross_a;
  P.cross_b = h->base.cross_b;
  P.tile_stats = h->stats;
  memcpy(P.eta, h->range_eta, sizeof(P.eta));
  Planes src = h->user, dst = h->shadow;
  int chunk[64];
  int done = 0;
  while (done < nsteps) {
    const int remain = nsteps - done;
    const int span = remain < 62 * h->range_steps ? remain : 62 * h->range_steps;
    const int n = plan(span, h->range_steps, chunk, 64);
    for (int j = 0; j < n; ++j) {
      P.code_in = src.code;
      P.id_in = src.id;
      P.tau_in = aco ? src.tau : nullptr;
      P.code_out = dst.code;
      P.id_out = dst.id;
      P.tau_out = aco ? dst.tau : nullptr;
      P.quads = P.W % 4 == 0 && (uintptr_t)P.code_in % 4 == 0 && (uintptr_t)P.id_in % 16 == 0 &&
                (!aco || (uintptr_t)P.tau_in % 16 == 0);
      P.t = h->t;
      const bool last = done + chunk[j] == nsteps;
      if (ev) (void)hipEventRecord(ev[0], s);
      PEDSIM_HIP(launch_range(P, mode, h->range_threads, chunk[j], last, s));
      if (ev) {
        (void)hipEventRecord(ev[1], s);
        PEDSIM_HIP(hipEventSynchronize(ev[1]));
        float f = 0.0f;
        (void)hipEventElapsedTime(&f, ev[0], ev[1]);
        ms[0] += f;
        launches[0] += 1;
      }
      h->t += (uint64_t)chunk[j];
      done += chunk[j];
      const Planes tmp = src;
      src = dst;
      dst = tmp;
    }
  }
  if (src.code != h->user.code) {  // odd number of launches: state is in the shadow planes
    if (ev) (void)hipEventRecord(ev[0], s);
    PEDSIM_HIP(copy_planes(h->user, src, cells, aco, 0, s));
    if (ev) {
      (void)hipEventRecord(ev[1], s);
      PEDSIM_HIP(hipEventSynchronize(ev[1]));
      float f = 0.0f;
      (void)hipEventElapsedTime(&f, ev[0], ev[1]);
      ms[1] += f;
      launches[1] += 1;
    }
  }
  h->stats_entries = P.tiles_x * P.tiles_y;
  return SIM_OK;
}

// Run nsteps steps; ev (optional, 2 events) brackets each tile launch, and
// its elapsed time is added into ms[0] (launches[0]); a copy-back is timed
// into ms[1] (launches[1]).
int run_steps(sim_handle* h, int mode, int32_t nsteps, hipStream_t s, hipEvent_t* ev, double* ms,
              int64_t* launches) {
  if (nsteps == 0) return SIM_OK;
  if (h->scan) return run_range_steps(h, mode, nsteps, s, ev, ms, launches);
  const Tiling& tl = h->tiling[mode];
  Scenario S = h->base;
  set_geometry(S, tl);
  if (rows_engine(tl) && (h->order_tl.nw != tl.nw || h->order_tl.rows != tl.rows || h->order_tl.steps != tl.steps ||
                          h->order_tl.threads != tl.threads || h->order_mode != mode)) {
    // another tile grid or kernel: start from row-major order
    PEDSIM_HIP(launch_zero_words(h->order, (size_t)3 * (16 + h->stats_cap), s));
    h->order_tl = tl;
    h->order_mode = mode;
    h->order_rot = 0;
    h->order_valid = false;
    h->order_on = rows_order_pays(S, tl, mode);
  }
  const bool ordered = rows_engine(tl) && h->order_on;
  const size_t cells = (size_t)S.W * (size_t)S.H;
  const bool aco = mode != kModeLem;
  const bool tour = mode == kModeAcoTour;
  Planes src = h->user, dst = h->shadow;
  int chunk[64];
  int done = 0;
  while (done < nsteps) {
    // plan at most 64 launches at a time (keeps the parity logic simple)
    const int remain = nsteps - done;
    const int span = remain < 62 * tl.steps ? remain : 62 * tl.steps;
    const int n = plan(span, tl.steps, chunk, 64);
    for (int j = 0; j < n; ++j) {
      S.code_in = src.code;
      S.id_in = src.id;
      S.tau_in = aco ? src.tau : nullptr;
      S.code_out = dst.code;
      S.id_out = dst.id;
      S.tau_out = aco ? dst.tau : nullptr;
      S.tour_in = tour ? src.tour : nullptr;
      S.tour_out = tour ? dst.tour : nullptr;
      S.tile_stats = h->stats;
      S.order = ordered ? h->order : nullptr;
      S.order_cap = h->stats_cap;
      S.order_rot = h->order_rot;
      S.order_valid = h->order_valid ? 1 : 0;
      const bool last = done + chunk[j] == nsteps;
      if (ev) (void)hipEventRecord(ev[0], s);
      PEDSIM_HIP(launch_tiles(S, tl, mode, h->t, chunk[j], last, s));
      if (ordered) {
        h->order_rot = (h->order_rot + 1) % 3;
        h->order_valid = true;
      }
      if (ev) {
        (void)hipEventRecord(ev[1], s);
        PEDSIM_HIP(hipEventSynchronize(ev[1]));
        float f = 0.0f;
        (void)hipEventElapsedTime(&f, ev[0], ev[1]);
        ms[0] += f;
        launches[0] += 1;
      }
      h->t += (uint64_t)chunk[j];
      done += chunk[j];
      const Planes tmp = src;
      src = dst;
      dst = tmp;
    }
  }
  if (src.code != h->user.code) {  // odd number of launches: state is in the shadow planes
    if (ev) (void)hipEventRecord(ev[0], s);
    PEDSIM_HIP(copy_planes(h->user, src, cells, aco, tour ? (size_t)h->agents : 0, s));
    if (ev) {
      (void)hipEventRecord(ev[1], s);
      PEDSIM_HIP(hipEventSynchronize(ev[1]));
      float f = 0.0f;
      (void)hipEventElapsedTime(&f, ev[0], ev[1]);
      ms[1] += f;
      launches[1] += 1;
    }
  }
  h->stats_entries = S.tiles_x * S.tiles_y;
  return SIM_OK;
}

// Set up *h over the caller's planes and a scratch area laid out as L:
// validate the state, then count the initial state; synchronises s, so the
// handle's counters are complete (and the caller's planes no longer read)
// whichever stream the next call uses.
int init_handle(sim_handle* h, const sim_params* p, uint8_t* d_code, uint32_t* d_id, float* d_tau,
                uint8_t* scratch, const ScratchLayout& L, hipStream_t s) {
  const size_t cells = (size_t)p->W * (size_t)p->H;
  uint64_t agents = 0;
  const int e = validate_state(p, d_code, d_id, d_tau, scratch, L, s, &agents);
  if (e) return e;
  h->p = *p;
  h->user = Planes{d_code, d_id, d_tau};
  h->shadow = Planes{scratch + L.code2, (uint32_t*)(scratch + L.id2), d_tau ? (float*)(scratch + L.tau2) : nullptr};
  h->stats = (uint32_t*)(scratch + L.stats);
  h->stats_cap = L.stats_cap;
  h->totals = (unsigned long long*)(scratch + L.totals);
  h->t = p->step0;
  h->agents = agents;
  h->base = base_scenario(p);
  h->tiling[kModeLem] = default_tiling(kModeLem, cells);
  h->tiling[kModeAco] = default_tiling(kModeAco, cells);
  h->tiling[kModeAcoTour] = default_tiling(kModeAcoTour, cells);
  h->scan = h->move = 0;
  h->range_cols = h->range_rows = h->range_steps = h->range_threads = 0;
  memset(h->range_eta, 0, sizeof(h->range_eta));
  h->order = (uint32_t*)(scratch + L.order);
  h->order_tl = Tiling{-1, 0, 0, 0};  // no order yet: the first row-lane launch clears the rotations
  h->order_mode = -1;
  h->order_on = false;
  PEDSIM_HIP(launch_count(d_code, p->W, p->H, p->cross_a, p->cross_b, h->stats, &h->stats_entries, s));
  PEDSIM_HIP(hipStreamSynchronize(s));
  return SIM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch for callers that cannot allocate (sim_run_noalloc): one static
// device array per GPU, held until the process ends. Host code must never
// pass `scratch` itself to a kernel or a copy (in host code the name is a
// host-side stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device and kept in g_noalloc_ptr.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)SIM_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu[kNoAllocMaxDevices];  // one call at a time per device
uint8_t* g_noalloc_ptr[kNoAllocMaxDevices];   // device address of `scratch` per device

}  // namespace

extern "C" {

const char* sim_strerror(int code) {
  switch (code) {
    case SIM_OK: return "ok";
    case SIM_EINVAL: return "invalid argument";
    case SIM_ESTATE: return "invalid initial state";
    case SIM_ESCRATCH: return "scratch buffer missing or too small";
    case SIM_EHIP: return "HIP runtime error";
    case SIM_ENOTAU: return "ACO step needs pheromone planes";
    case SIM_EFULL: return "no free batch slot";
    case SIM_ENOTOUR: return "tour step needs an attached tour array";
    default: return "unknown error";
  }
}

int sim_scratch_bytes(const sim_params* p, size_t* out) {
  int e = check_params(p);
  if (e) return e;
  if (!out) return SIM_EINVAL;
  *out = layout_of(p).total;
  return SIM_OK;
}

int sim_create(const sim_params* p, uint8_t* d_code, uint32_t* d_id, float* d_tau, void* d_scratch,
               size_t scratch_bytes, void* stream, sim_handle** out) {
  int e = check_params(p);
  if (e) return e;
  if (!d_code || !d_id || !out) return SIM_EINVAL;
  *out = nullptr;
  const ScratchLayout L = layout_of(p);
  if (!d_scratch || scratch_bytes < L.total) return SIM_ESCRATCH;
  sim_handle* h = new (std::nothrow) sim_handle;
  if (!h) return SIM_EINVAL;
  e = init_handle(h, p, d_code, d_id, d_tau, (uint8_t*)d_scratch, L, (hipStream_t)stream);
  if (e) {
    delete h;
    return e;
  }
  *out = h;
  return SIM_OK;
}

// SIM_OK if `mode` can step on h now.
static int mode_ready(sim_handle* h, int mode) {
  if (mode != kModeLem && mode != kModeAco && mode != kModeAcoTour) return SIM_EINVAL;
  if (mode != kModeLem && !h->user.tau) return SIM_ENOTAU;
  if (mode == kModeAcoTour && h->agents > 0 && !h->user.tour) return SIM_ENOTOUR;
  if (mode == kModeAcoTour && h->scan) return SIM_EINVAL;  // ranges are not combined with the tour variant
  return SIM_OK;
}

static int step_mode(sim_handle* h, int mode, int32_t nsteps, void* stream) {
  if (!h || nsteps < 0) return SIM_EINVAL;
  const int e = mode_ready(h, mode);
  if (e) return e;
  return run_steps(h, mode, nsteps, (hipStream_t)stream, nullptr, nullptr, nullptr);
}

int sim_step_lem(sim_handle* h, int32_t nsteps, void* stream) { return step_mode(h, kModeLem, nsteps, stream); }

int sim_step_aco(sim_handle* h, int32_t nsteps, void* stream) { return step_mode(h, kModeAco, nsteps, stream); }

int sim_step_aco_tour(sim_handle* h, int32_t nsteps, void* stream) {
  return step_mode(h, kModeAcoTour, nsteps, stream);
}

int sim_attach_tour(sim_handle* h, float* d_tour, float* d_tour_shadow, void* stream) {
  if (!h) return SIM_EINVAL;
  if (h->agents > 0 && (!d_tour || !d_tour_shadow || d_tour == d_tour_shadow)) return SIM_EINVAL;
  if (h->agents > 0) {
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* counters = h->totals + kTileStatFields;
    unsigned long long host_counters[3];
    PEDSIM_HIP(launch_zero_words(counters, 3 * sizeof(unsigned long long) / 4, s));
    PEDSIM_HIP(launch_validate_values(d_tour, (size_t)h->agents, counters, s));
    PEDSIM_HIP(hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, s));
    PEDSIM_HIP(hipStreamSynchronize(s));
    if (host_counters[2]) return SIM_ESTATE;
  }
  h->user.tour = d_tour;
  h->shadow.tour = d_tour_shadow;
  return SIM_OK;
}

int sim_set_neighbours(sim_handle* h, int32_t n) {
  if (!h || (n != 5 && n != 8)) return SIM_EINVAL;
  if (n == 8 && h->scan) return SIM_EINVAL;  // ranges are not combined with the eight-neighbour set
  h->base.neighbours = n;
  const size_t cells = (size_t)h->p.W * (size_t)h->p.H;
  for (int m = 0; m < 3; ++m) h->tiling[m] = default_tiling(m, cells, n == 8);
  return SIM_OK;
}

int sim_set_ranges(sim_handle* h, int32_t scan, int32_t move) {
  if (!h) return SIM_EINVAL;
  if (scan == 0 && move == 0) {
    h->scan = h->move = 0;
    return SIM_OK;
  }
  if (scan < 1 || scan > kRangeMax || move < 1 || move > scan) return SIM_EINVAL;
  if (h->base.neighbours == 8) return SIM_EINVAL;
  const int old_scan = h->scan, old_move = h->move;
  h->scan = scan;
  h->move = move;
  if (!default_range_tiling(h)) {  // no launch shape fits this device's LDS
    h->scan = old_scan;
    h->move = old_move;
    return SIM_EINVAL;
  }
  fill_range_eta(scan, move, h->p.beta, h->range_eta);
  return SIM_OK;
}

int sim_set_range_tiling(sim_handle* h, int32_t cols, int32_t rows, int32_t steps_per_launch, int32_t threads) {
  if (!h || !h->scan) return SIM_EINVAL;
  if (!range_tiling_valid(cols, rows, steps_per_launch, threads, h->scan, h->move)) return SIM_EINVAL;
  h->range_cols = cols;
  h->range_rows = rows;
  h->range_steps = steps_per_launch;
  h->range_threads = threads;
  return SIM_OK;
}

int sim_get_range_tiling(sim_handle* h, int32_t out[4]) {
  if (!h || !out || !h->scan) return SIM_EINVAL;
  out[0] = h->range_cols;
  out[1] = h->range_rows;
  out[2] = h->range_steps;
  out[3] = h->range_threads;
  return SIM_OK;
}

int sim_range_weights(int32_t scan, int32_t move, int32_t beta, float diagonal[8], float lateral[8]) {
  if (scan < 1 || scan > kRangeMax || move < 1 || move > scan || beta < 0 || beta > 8 || !diagonal || !lateral)
    return SIM_EINVAL;
  float t[2][kRangeMax];
  fill_range_eta(scan, move, beta, t);
  for (int f = 0; f < kRangeMax; ++f) {
    diagonal[f] = t[1][f];
    lateral[f] = t[0][f];
  }
  return SIM_OK;
}

int sim_set_tiling(sim_handle* h, int32_t mode, int32_t nw, int32_t rows, int32_t steps_per_launch,
                   int32_t threads) {
  if (!h || (mode != kModeLem && mode != kModeAco && mode != kModeAcoTour)) return SIM_EINVAL;
  const Tiling tl{nw, rows, steps_per_launch, threads};
  if (!tiling_valid(tl, mode, max_dynamic_lds(), h->base.neighbours == 8)) return SIM_EINVAL;
  Scenario S = h->base;
  set_geometry(S, tl);
  if (S.tiles_x * S.tiles_y > h->stats_cap) return SIM_EINVAL;
  h->tiling[mode] = tl;
  return SIM_OK;
}

int sim_get_tiling(sim_handle* h, int32_t mode, int32_t out[4]) {
  if (!h || !out || (mode != kModeLem && mode != kModeAco && mode != kModeAcoTour)) return SIM_EINVAL;
  const Tiling& tl = h->tiling[mode];
  out[0] = tl.nw;
  out[1] = tl.rows;
  out[2] = tl.steps;
  out[3] = tl.threads;
  return SIM_OK;
}

int sim_stats(sim_handle* h, sim_stats_t* out, void* stream) {
  if (!h || !out) return SIM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long v[kTileStatFields];
  PEDSIM_HIP(launch_reduce_counts(h->stats, h->stats_entries, h->totals, s));
  PEDSIM_HIP(hipMemcpyAsync(v, h->totals, sizeof(v), hipMemcpyDeviceToHost, s));
  PEDSIM_HIP(hipStreamSynchronize(s));
  out->step = h->t;
  out->agents_a = v[0];
  out->agents_b = v[1];
  out->crossed_a = v[2];
  out->crossed_b = v[3];
  out->moved_last = v[4];
  return SIM_OK;
}

int sim_read_state(sim_handle* h, uint8_t* code, uint32_t* id, float* tau, void* stream) {
  if (!h) return SIM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const size_t cells = (size_t)h->p.W * (size_t)h->p.H;
  if (code) PEDSIM_HIP(hipMemcpyAsync(code, h->user.code, cells, hipMemcpyDefault, s));
  if (id) PEDSIM_HIP(hipMemcpyAsync(id, h->user.id, cells * sizeof(uint32_t), hipMemcpyDefault, s));
  if (tau && h->user.tau) PEDSIM_HIP(hipMemcpyAsync(tau, h->user.tau, 2 * cells * sizeof(float), hipMemcpyDefault, s));
  PEDSIM_HIP(hipStreamSynchronize(s));
  return SIM_OK;
}

int sim_step_timed(sim_handle* h, int32_t mode, int32_t nsteps, void* stream, double* kernel_ms,
                   int64_t* launches, int32_t max_kinds) {
  if (!h || nsteps < 0 || !kernel_ms || !launches || max_kinds < 2) return SIM_EINVAL;
  const int ready = mode_ready(h, mode);
  if (ready) return ready;
  hipEvent_t ev[2];
  PEDSIM_HIP(hipEventCreate(&ev[0]));
  const hipError_t e1 = hipEventCreate(&ev[1]);
  if (e1 != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return hip_fail(e1, "hipEventCreate", __LINE__);
  }
  const int rc = run_steps(h, mode, nsteps, (hipStream_t)stream, ev, kernel_ms, launches);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  return rc == SIM_OK ? 2 : rc;
}

const char* sim_last_error(void) { return g_last_error; }

const char* sim_kernel_name(int32_t kind) {
  switch (kind) {
    case 0: return "tile_kernel";
    case 1: return "copy_back";
    default: return "";
  }
}

int sim_run_noalloc(const sim_params* p, int32_t mode, uint8_t* d_code, uint32_t* d_id, float* d_tau,
                    int32_t nsteps, void* stream, sim_stats_t* out) {
  int e = check_params(p);
  if (e) return e;
  if (!d_code || !d_id || !out || nsteps < 0 || (mode != kModeLem && mode != kModeAco)) return SIM_EINVAL;
  if (mode == kModeAco && !d_tau) return SIM_ENOTAU;
  const ScratchLayout L = layout_of(p);
  if (L.total > kNoAllocScratchBytes) return SIM_ESCRATCH;
  int dev = 0;
  PEDSIM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return SIM_EINVAL;
  std::lock_guard<std::mutex> lock(g_noalloc_mu[dev]);
  if (!g_noalloc_ptr[dev]) {  // first call on this device (it is current)
    void* ptr = nullptr;
    PEDSIM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return SIM_EHIP;
    g_noalloc_ptr[dev] = (uint8_t*)ptr;
  }
  hipStream_t s = (hipStream_t)stream;
  sim_handle h;  // on the stack: this call allocates nothing, host or device
  e = init_handle(&h, p, d_code, d_id, d_tau, g_noalloc_ptr[dev], L, s);
  if (e) return e;
  e = run_steps(&h, mode, nsteps, s, nullptr, nullptr, nullptr);
  if (e) return e;
  return sim_stats(&h, out, stream);  // synchronises: the array is free for the next call
}

void sim_destroy(sim_handle* h) { delete h; }

}  // extern "C"
