// Step with larger scanning and moving ranges (the paper's future work,
// Sec. VII): parameters, LDS layout and the launch entry of the range kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pedsim {

constexpr int kRangeMax = 8;           // largest scanning range
constexpr int kRangeMaxThreads = 512;  // workgroup size limit of the range kernel
constexpr int kRangeMaxSteps = 4;      // steps per launch of the range kernel

// One launch (one step) of the range kernel over a scenario.
struct RangeScenario {
  const uint8_t* code_in;
  const uint32_t* id_in;
  const float* tau_in;  // 2 planes (A then B) or nullptr for LEM
  uint8_t* code_out;
  uint32_t* id_out;
  float* tau_out;
  uint32_t* tile_stats;  // 5 counters per tile (agents A, B, crossed A, B, moved)
  uint64_t t;            // index of the launch's first step
  int W, H;
  int TX, TY;            // tile interior
  int tiles_x, tiles_y;
  int S, M;              // scanning and moving range, 1 <= M <= S <= kRangeMax
  uint32_t key0, key1;   // Philox key (seed)
  float keep, dtau;      // 1 - rho, deposit
  int alpha;
  int cross_a, cross_b;
  float eta[2][kRangeMax];  // eta^beta of a side ray: [0 lateral, 1 diagonal][free run - 1]
  int quads;  // W % 4 == 0, codes 4-byte and ids / pheromone 16-byte aligned: stage 4 cells per load
};

// LDS of one workgroup for k steps per launch (R1 = 2M + S, the reach of one
// step): codes of the interior plus k R1 (1 B/cell); ids and, for ACO, both
// pheromone planes of the interior plus (k-1) R1 + 3M; request bytes and the
// compacted agent list of the interior plus (k-1) R1 + 2M; claim keys and
// counts of the interior plus (k-1) R1 + M; counters and the heuristic table;
// for ACO with k > 1 an occupancy history byte per pheromone cell.
struct RangeLayout {
  int TX, TY, S, M, K;
  bool aco;
  __host__ __device__ static size_t up16(size_t v) { return (v + 15) / 16 * 16; }
  __host__ __device__ size_t cells(int halo) const { return (size_t)(TX + 2 * halo) * (size_t)(TY + 2 * halo); }
  __host__ __device__ int r1() const { return 2 * M + S; }
  __host__ __device__ size_t code() const { return 0; }
  __host__ __device__ size_t ids() const { return up16(cells(K * r1())); }
  __host__ __device__ size_t req() const { return ids() + cells((K - 1) * r1() + 3 * M) * 4; }
  __host__ __device__ size_t list() const { return up16(req() + cells((K - 1) * r1() + 2 * M)); }
  __host__ __device__ size_t keys() const { return up16(list() + cells((K - 1) * r1() + 2 * M) * 2); }
  __host__ __device__ size_t claims() const { return keys() + cells((K - 1) * r1() + M) * 8; }
  __host__ __device__ size_t ctl() const { return up16(claims() + cells((K - 1) * r1() + M) * 4); }
  __host__ __device__ size_t tau() const { return ctl() + 32 * 4; }  // ctl: 8 counters, 16 eta, pad
  // ACO with k > 1: the occupancy after each of the launch's first k - 1
  // steps, 2 bits per step, per cell of the pheromone array
  __host__ __device__ size_t hist() const { return tau() + (aco ? (size_t)2 * cells((K - 1) * r1() + 3 * M) * 4 : 0); }
  __host__ __device__ size_t bytes() const {
    return hist() + (aco && K > 1 ? up16(cells((K - 1) * r1() + 3 * M)) : 0);
  }
};

hipError_t launch_range(const RangeScenario& P, int mode, int threads, int steps, int last, hipStream_t s);

}  // namespace pedsim
