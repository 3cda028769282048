// Internal declarations shared by the kernels and the C ABI implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rules.hpp"

namespace pedsim {

constexpr int kModeLem = 0;
constexpr int kModeAco = 1;

// decide: a workgroup owns a kDecideTX x kDecideTY tile.
constexpr int kDecideTX = 64;
constexpr int kDecideTY = 8;
constexpr int kDecideThreads = 256;

// commit: a workgroup owns a kCommitTX x kCommitTY block, one cell per lane.
constexpr int kCommitTX = 64;
constexpr int kCommitTY = 4;
constexpr int kCommitThreads = kCommitTX * kCommitTY;

// per-workgroup counters: agents A, agents B, crossed A, crossed B, moved
constexpr int kStatFields = 5;

struct StepArgs {
  uint8_t* code;
  uint32_t* id;
  float* tau_a;
  float* tau_b;
  uint8_t* dec;           // one decision byte per cell (scratch)
  uint32_t* block_stats;  // kStatFields per commit workgroup (scratch)
  int W, H;
  int tiles_x, tiles_y;   // decide tiles
  int commit_bx, commit_by;
  uint64_t t;             // index of the step being run
  uint32_t key0, key1;    // Philox key (seed)
  float keep;             // fl(1 - rho)
  float dtau;
  float eta_diag, eta_lat;  // eta^beta of the diagonal and lateral candidates
  int alpha;
  int cross_a, cross_b;
};

// Kernel kinds of one step, in launch order.
constexpr int kKernelKinds = 2;
extern const char* const kKernelNames[kKernelKinds];

// Launch one step. With `ev` non-null (kKernelKinds + 1 events), event i is
// recorded before kernel i and the last one after the final kernel.
hipError_t launch_step(const StepArgs& a, int mode, int write_stats, hipStream_t s,
                       hipEvent_t* ev = nullptr);
hipError_t launch_count(const StepArgs& a, hipStream_t s);
hipError_t launch_reduce_counts(const uint32_t* block_stats, int nblocks, unsigned long long* out,
                                hipStream_t s);
hipError_t launch_validate(const uint8_t* code, const uint32_t* id, const float* tau, size_t cells,
                           unsigned long long* counters, hipStream_t s);
hipError_t launch_validate_ids(const uint32_t* id, size_t cells, uint32_t n, uint32_t* bitmap,
                               unsigned long long* counters, hipStream_t s);

}  // namespace pedsim
