// Internal declarations shared by the kernels and the C ABI implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rules.hpp"
#include "tile_engine.hpp"
#include "tile_rows.hpp"

namespace pedsim {

constexpr int kModeLem = 0;
constexpr int kModeAco = 1;
constexpr int kModeAcoTour = 2;  // ACO with the tour matrix and eq. 5's deposit

// Tiling of one scenario: regions of `rows` rows advanced `steps` steps per
// launch (halo 3*steps), `threads` per workgroup. nw = 1 or 2 selects the
// multi-wave engine on regions of 64*nw columns; nw = 0 selects the row-lane
// engine on regions of 64 columns and at most 64 rows, and nw = 3 its
// streaming form (pheromone read from HBM, tickets recomputed, less LDS).
struct Tiling {
  int nw;       // 0 / 3 (row-lane engine / streaming), 1 or 2 (multi-wave engine, words per row)
  int rows;     // region rows
  int steps;    // steps per launch (>= 1)
  int threads;  // workgroup size, multiple of 64, <= 1024
};

// Smallest tile interior the host accepts (bounds the per-tile counter array).
constexpr int kMinInteriorX = 16;
constexpr int kMinInteriorY = 8;

inline bool rows_engine(const Tiling& tl) { return tl.nw == 0 || tl.nw == 3; }
inline bool rows_stream(const Tiling& tl) { return tl.nw == 3; }
inline int region_cols(const Tiling& tl) { return rows_engine(tl) ? 64 : 64 * tl.nw; }
// LDS of one workgroup for `mode` (nb8: the eight-neighbour candidate set);
// a tiling is valid for a mode when its shape is allowed, fits max_lds, and
// (tour variant, eight neighbours) uses the row-lane engine with the
// pheromone staged in LDS (nw = 0).
size_t tile_lds_bytes(const Tiling& tl, int mode, bool nb8 = false);
bool tiling_valid(const Tiling& tl, int mode, int max_lds, bool nb8 = false);

// Whether the row-lane launches of S with tiling tl run more workgroups than
// the device holds at once, so that the order in which tiles are dealt out
// matters (see Scenario::order).
bool rows_order_pays(const Scenario& S, const Tiling& tl, int mode);

// One launch of the tile engine over every tile of S.
hipError_t launch_tiles(const Scenario& S, const Tiling& tl, int mode, uint64_t t0, int steps, int last,
                        hipStream_t s);

// Counters of the current planes without stepping: kTileStatFields per
// workgroup of the count kernel; returns the number of entries written.
hipError_t launch_count(const uint8_t* code, int W, int H, int cross_a, int cross_b, uint32_t* stats,
                        int* entries, hipStream_t s);

hipError_t launch_reduce_counts(const uint32_t* stats, int entries, unsigned long long* out, hipStream_t s);
hipError_t launch_validate(const uint8_t* code, const uint32_t* id, const float* tau, size_t cells,
                           unsigned long long* counters, hipStream_t s);
hipError_t launch_validate_ids(const uint32_t* id, size_t cells, uint32_t n, uint32_t* bitmap,
                               unsigned long long* counters, hipStream_t s);
// Zero `words` 32-bit words at p with a kernel.
hipError_t launch_zero_words(void* p, size_t words, hipStream_t s);
// counters[2] |= 1 if any of the n values is negative, NaN or infinite.
hipError_t launch_validate_values(const float* v, size_t n, unsigned long long* counters, hipStream_t s);

int max_dynamic_lds();

}  // namespace pedsim

#include "pedsim.h"

namespace pedsim {

// Host-side helpers shared by the single-scenario and batch C ABIs.
constexpr size_t kAlign = 256;
size_t round_up(size_t v);

struct Planes {
  uint8_t* code;
  uint32_t* id;
  float* tau;
  float* tour = nullptr;  // tour variant: one float per agent
};

// Per-scenario scratch: shadow planes (code, id, both pheromone planes),
// per-tile counters, totals and validation counters.
struct ScratchLayout {
  size_t code2, id2, tau2, stats, totals, order, total;
  int stats_cap;
};

// Record a failed HIP call for sim_last_error() (per thread) and return
// SIM_EHIP.
int hip_fail(hipError_t e, const char* what, int line);
#define PEDSIM_HIP(expr)                                                         \
  do {                                                                           \
    const hipError_t pedsim_e_ = (expr);                                         \
    if (pedsim_e_ != hipSuccess) return ::pedsim::hip_fail(pedsim_e_, #expr, __LINE__); \
  } while (0)

ScratchLayout layout_of(const sim_params* p);
int check_params(const sim_params* p);
Scenario base_scenario(const sim_params* p);
void set_geometry(Scenario& S, const Tiling& tl);
int validate_state(const sim_params* p, const uint8_t* d_code, const uint32_t* d_id, const float* d_tau,
                   uint8_t* scratch, const ScratchLayout& L, hipStream_t s, uint64_t* agents = nullptr);

}  // namespace pedsim

namespace pedsim {

// ---------------------------------------------------------------------------
// Batched form: many independent scenarios advanced together.
// ---------------------------------------------------------------------------

// One scenario of a batch as the device sees it during one call.
struct BatchSlot {
  Scenario S;         // parameters and tile geometry; plane pointers set per launch
  uint8_t* code[2];   // [0] caller planes, [1] shadow planes in the slot's scratch
  uint32_t* id[2];
  float* tau[2];
  float* tour[2];     // tour variant: tour matrices (caller's, shadow), one float per agent
  uint64_t t0;        // index of the slot's first step in this call
  int steps;          // steps the slot runs in this call (0: idle)
  int mode;           // kModeLem, kModeAco or kModeAcoTour
  uint32_t agents;    // number of agents (tour matrix entries)
};

// Launch j of a call processes, in order, the tiles of every slot with
// steps > j * k: entries[j * capacity + e] = {slot, index of its first tile
// among the launch's work items}.
struct BatchEntry {
  int slot;
  int first;
};

struct BatchPlan {
  const BatchSlot* slots;
  const BatchEntry* entries;  // [launch][capacity]
  const int* counts;          // [launch] number of entries
  const int* totals;          // [launch] number of work items (tiles)
  unsigned* counters;         // [launch] work-claim counters
  int capacity;
  int k;                      // steps per launch
  int rows;                   // region rows
  int nb8;                    // every scenario uses the eight-neighbour set (row-lane engine, nw = 0)
  int tour;                   // the batch holds tour-variant scenarios (row-lane engine, nw = 0)
};

constexpr int kBatchMaxLaunches = 128;  // launches per captured graph
constexpr int kBatchItemBytes = 16;     // LDS the batch kernel needs beyond the tile layout

hipError_t launch_batch_reset(const BatchPlan& P, int launches, hipStream_t s);
hipError_t launch_batch(const BatchPlan& P, const Tiling& tl, int j, int grid, hipStream_t s);
hipError_t launch_batch_copyback(const BatchPlan& P, int capacity, hipStream_t s);
int device_cu_count();
void prepare_batch_kernels();  // sets the batch kernels' LDS limit once (outside any capture)

}  // namespace pedsim
