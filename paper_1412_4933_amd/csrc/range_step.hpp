// Step with larger scanning and moving ranges (the paper's future work,
// Sec. VII): parameters, LDS layout and the launch entry of the range kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pedsim {

constexpr int kRangeMax = 8;           // largest scanning range
constexpr int kRangeMaxThreads = 512;  // workgroup size limit of the range kernel

// One launch (one step) of the range kernel over a scenario.
struct RangeScenario {
  const uint8_t* code_in;
  const uint32_t* id_in;
  const float* tau_in;  // 2 planes (A then B) or nullptr for LEM
  uint8_t* code_out;
  uint32_t* id_out;
  float* tau_out;
  uint32_t* tile_stats;  // 5 counters per tile (agents A, B, crossed A, B, moved)
  uint64_t t;            // index of the step
  int W, H;
  int TX, TY;            // tile interior
  int tiles_x, tiles_y;
  int S, M;              // scanning and moving range, 1 <= M <= S <= kRangeMax
  uint32_t key0, key1;   // Philox key (seed)
  float keep, dtau;      // 1 - rho, deposit
  int alpha;
  int cross_a, cross_b;
  float eta[2][kRangeMax];  // eta^beta of a side ray: [0 lateral, 1 diagonal][free run - 1]
};

// LDS of one workgroup: codes of the interior plus a 2M + S halo; ids, request
// bytes and the compacted agent list of the request region (the interior plus
// a 2M halo); claim keys and claim counts of the interior plus an M halo;
// counters and the heuristic table; for ACO, both pheromone planes of the
// interior plus a 3M halo.
struct RangeLayout {
  int TX, TY, S, M;
  bool aco;
  __host__ __device__ static size_t up16(size_t v) { return (v + 15) / 16 * 16; }
  __host__ __device__ size_t rcells() const { return (size_t)(TX + 4 * M) * (TY + 4 * M); }
  __host__ __device__ size_t kcells() const { return (size_t)(TX + 2 * M) * (TY + 2 * M); }
  __host__ __device__ size_t code() const { return 0; }
  __host__ __device__ size_t ids() const {
    return up16((size_t)(TX + 2 * (2 * M + S)) * (size_t)(TY + 2 * (2 * M + S)));
  }
  __host__ __device__ size_t req() const { return ids() + rcells() * 4; }
  __host__ __device__ size_t list() const { return up16(req() + rcells()); }
  __host__ __device__ size_t keys() const { return up16(list() + rcells() * 2); }
  __host__ __device__ size_t claims() const { return keys() + kcells() * 8; }
  __host__ __device__ size_t ctl() const { return up16(claims() + kcells() * 4); }
  __host__ __device__ size_t tau() const { return ctl() + 32 * 4; }  // ctl: 8 counters, 16 eta, pad
  __host__ __device__ size_t bytes() const {
    return tau() + (aco ? (size_t)2 * (TX + 6 * M) * (TY + 6 * M) * 4 : 0);
  }
};

hipError_t launch_range(const RangeScenario& P, int mode, int threads, int last, hipStream_t s);

}  // namespace pedsim
