// Internal declarations shared by the kernels and the C ABI implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rules.hpp"
#include "tile_engine.hpp"

namespace pedsim {

constexpr int kModeLem = 0;
constexpr int kModeAco = 1;

// Tiling of one scenario for the tile engine: regions of 64*nw columns x
// rows, advanced `steps` steps per launch (halo 3*steps), `threads` per
// workgroup.
struct Tiling {
  int nw;       // 1 or 2 words per row
  int rows;     // region rows, <= threads
  int steps;    // steps per launch (>= 1)
  int threads;  // workgroup size, multiple of 64, <= 1024
};

// Smallest tile interior the host accepts (bounds the per-tile counter array).
constexpr int kMinInteriorX = 16;
constexpr int kMinInteriorY = 8;

size_t tile_lds_bytes(const Tiling& tl, bool aco);
bool tiling_valid(const Tiling& tl, bool aco, int max_lds);

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

int max_dynamic_lds();

}  // namespace pedsim
