// Single-scenario kernels for gfx950: the tile-engine launch (k steps per
// launch, one workgroup per tile), plus counting, reduction and create-time
// validation.
#include "pedsim_internal.hpp"

namespace pedsim {

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD one
// contiguous run of row-major tiles so shared halo lines stay in its L2.
__device__ __forceinline__ int tile_of_block(int bid, int ntiles) {
  const int per = (ntiles + 7) >> 3;
  return (bid & 7) * per + (bid >> 3);
}

template <int NW, int MODE>
__global__ __launch_bounds__(1024) void tile_kernel(Scenario S, int R, uint64_t t0, int steps, int last) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int ntiles = S.tiles_x * S.tiles_y;
  const int tile = tile_of_block(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  advance_tile<NW, MODE>(S, smem, R, tile % S.tiles_x, tile / S.tiles_x, tile, t0, steps, last != 0);
}

// The tile a workgroup takes (-1: none): the XCD's run of tiles in the order
// the previous launch recorded, or in row-major order.
__device__ __forceinline__ int pick_tile(const Scenario& S) {
  const int ntiles = S.tiles_x * S.tiles_y;
  const int per = (ntiles + 7) >> 3;
  const int x = blockIdx.x & 7, j = blockIdx.x >> 3;  // XCD, and the workgroup's place in its run
  const int run = ntiles - x * per < per ? ntiles - x * per : per;
  if (j >= run) return -1;
  if (S.order) {
    const size_t stride = 16 + (size_t)S.order_cap;
    if (blockIdx.x == 0 && threadIdx.x < 16) S.order[(size_t)((S.order_rot + 2) % 3) * stride + threadIdx.x] = 0u;
    if (S.order_valid) {
      const uint32_t t = S.order[(size_t)S.order_rot * stride + 16 + x * per + j];
      if (t < (uint32_t)ntiles) return (int)t;  // (always, when the previous launch recorded the order)
    }
  }
  return x * per + j;
}

// Records `tile` in the next launch's order: from the front of its XCD's run
// if it held agents, from the back otherwise.
__device__ __forceinline__ void record_tile(const Scenario& S, int tile, bool busy) {
  const int ntiles = S.tiles_x * S.tiles_y;
  const int per = (ntiles + 7) >> 3;
  const int x = blockIdx.x & 7;
  const int run = ntiles - x * per < per ? ntiles - x * per : per;
  uint32_t* wr = S.order + (size_t)((S.order_rot + 1) % 3) * (16 + (size_t)S.order_cap);
  const uint32_t slot = atomicAdd(&wr[2 * x + (busy ? 0 : 1)], 1u);
  if (slot < (uint32_t)run) wr[16 + x * per + (busy ? (int)slot : run - 1 - (int)slot)] = (uint32_t)tile;
}

// On grids with more tiles than the device runs at once, the tiles that hold
// agents take several times longer than the empty ones, and a busy tile
// dealt out late extends the launch. Each XCD therefore deals its tiles in the
// order the previous launch recorded: the tiles that had agents first. The
// order only changes which workgroup takes which tile, never the result.
// ORDERED: S.order is set. Without it the kernel is the plain row-major one
// (no order state kept live through the step phases).
template <int MODE, bool STREAM, bool NB8 = false, bool ORDERED = false>
__global__ __launch_bounds__(kRowsMaxThreads, kRowsMinWavesPerSimd) void tile_rows_kernel(Scenario S, int R, int k_max, uint64_t t0,
                                                                    int steps, int last) {
  extern __shared__ __align__(16) uint8_t smem[];
  if (!ORDERED) {
    const int ntiles = S.tiles_x * S.tiles_y;
    const int tile = tile_of_block(blockIdx.x, ntiles);
    if (tile >= ntiles) return;
    advance_tile_rows<MODE, STREAM, NB8>(S, smem, R, k_max, tile % S.tiles_x, tile / S.tiles_x, tile, t0, steps,
                                         last != 0);
    return;
  }
  const int tile = pick_tile(S);
  if (tile < 0) return;
  const bool busy = advance_tile_rows<MODE, STREAM, NB8>(S, smem, R, k_max, tile % S.tiles_x, tile / S.tiles_x,
                                                         tile, t0, steps, last != 0);
  if (threadIdx.x == 0) record_tile(S, tile, busy);
}

size_t tile_lds_bytes(const Tiling& tl, int mode, bool nb8) {
  const bool aco = mode != kModeLem;
  if (rows_engine(tl)) return RowsLayout{tl.rows, tl.steps, aco, rows_stream(tl), mode == kModeAcoTour, nb8}.bytes();
  return tl.nw == 1 ? Layout<1>{tl.rows, aco}.bytes() : Layout<2>{tl.rows, aco}.bytes();
}

bool tiling_valid(const Tiling& tl, int mode, int max_lds, bool nb8) {
  if (tl.nw < 0 || tl.nw > 3) return false;
  if ((mode == kModeAcoTour || nb8) && tl.nw != 0) return false;
  if (rows_engine(tl) && (tl.rows > kRowsMaxRows || tl.steps > kRowsMaxSteps || tl.threads > kRowsMaxThreads))
    return false;
  if (tl.steps < 1 || tl.threads < 64 || tl.threads > 1024 || tl.threads % 64) return false;
  if (tl.rows < 1 || tl.rows > 1023) return false;
  if (region_cols(tl) - 6 * tl.steps < kMinInteriorX || tl.rows - 6 * tl.steps < kMinInteriorY) return false;
  return tile_lds_bytes(tl, mode, nb8) <= (size_t)max_lds;
}

int max_dynamic_lds() {
  static int cached = -1;
  if (cached < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
    cached = v;
  }
  return cached;
}

template <int NW, int MODE>
static hipError_t launch_one(const Scenario& S, const Tiling& tl, uint64_t t0, int steps, int last, hipStream_t s) {
  const size_t lds = Layout<NW>{tl.rows, MODE == kModeAco}.bytes();
  static bool attr_done = false;
  if (!attr_done) {
    (void)hipFuncSetAttribute((const void*)tile_kernel<NW, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              max_dynamic_lds());
    (void)hipGetLastError();  // an unsupported attribute value must not linger as the last error
    attr_done = true;
  }
  const int ntiles = S.tiles_x * S.tiles_y;
  const int blocks = ((ntiles + 7) / 8) * 8;
  tile_kernel<NW, MODE><<<blocks, tl.threads, lds, s>>>(S, tl.rows, t0, steps, last);
  return hipGetLastError();
}

template <int MODE, bool STREAM, bool NB8 = false>
static size_t rows_prepare(const Tiling& tl) {
  static bool attr_done = false;
  if (!attr_done) {
    (void)hipFuncSetAttribute((const void*)tile_rows_kernel<MODE, STREAM, NB8, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, max_dynamic_lds());
    (void)hipFuncSetAttribute((const void*)tile_rows_kernel<MODE, STREAM, NB8, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, max_dynamic_lds());
    (void)hipGetLastError();  // an unsupported attribute value must not linger as the last error
    attr_done = true;
  }
  return RowsLayout{tl.rows, tl.steps, MODE != kModeLem, STREAM, MODE == kModeAcoTour, NB8}.bytes();
}

// Workgroups of this kernel the whole device runs at once (0 if unknown).
template <int MODE, bool STREAM, bool NB8 = false>
static long rows_resident(const Tiling& tl) {
  const size_t lds = rows_prepare<MODE, STREAM, NB8>(tl);
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)tile_rows_kernel<MODE, STREAM, NB8, true>,
                                                   tl.threads, lds) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return (long)per_cu * cus;
}

template <int MODE, bool STREAM, bool NB8 = false>
static hipError_t launch_rows(const Scenario& S, const Tiling& tl, uint64_t t0, int steps, int last, hipStream_t s) {
  const size_t lds = rows_prepare<MODE, STREAM, NB8>(tl);
  const int ntiles = S.tiles_x * S.tiles_y;
  const int blocks = ((ntiles + 7) / 8) * 8;
  if (S.order)
    tile_rows_kernel<MODE, STREAM, NB8, true><<<blocks, tl.threads, lds, s>>>(S, tl.rows, tl.steps, t0, steps, last);
  else
    tile_rows_kernel<MODE, STREAM, NB8, false><<<blocks, tl.threads, lds, s>>>(S, tl.rows, tl.steps, t0, steps, last);
  return hipGetLastError();
}

bool rows_order_pays(const Scenario& S, const Tiling& tl, int mode) {
  if (!rows_engine(tl)) return false;
  long resident = 0;
  if (S.neighbours == 8)
    resident = mode == kModeLem ? rows_resident<kModeLem, false, true>(tl)
                                : (mode == kModeAco ? rows_resident<kModeAco, false, true>(tl)
                                                    : rows_resident<kModeAcoTour, false, true>(tl));
  else if (mode == kModeAcoTour)
    resident = rows_resident<kModeAcoTour, false>(tl);
  else if (rows_stream(tl))
    resident = mode == kModeLem ? rows_resident<kModeLem, true>(tl) : rows_resident<kModeAco, true>(tl);
  else
    resident = mode == kModeLem ? rows_resident<kModeLem, false>(tl) : rows_resident<kModeAco, false>(tl);
  return resident > 0 && (long)S.tiles_x * S.tiles_y > resident;
}

hipError_t launch_tiles(const Scenario& S, const Tiling& tl, int mode, uint64_t t0, int steps, int last,
                        hipStream_t s) {
  if (S.neighbours == 8) {  // the eight-neighbour set: row-lane engine, pheromone in LDS
    if (tl.nw != 0) return hipErrorInvalidValue;
    if (mode == kModeLem) return launch_rows<kModeLem, false, true>(S, tl, t0, steps, last, s);
    if (mode == kModeAco) return launch_rows<kModeAco, false, true>(S, tl, t0, steps, last, s);
    return launch_rows<kModeAcoTour, false, true>(S, tl, t0, steps, last, s);
  }
  if (mode == kModeAcoTour) {
    if (tl.nw != 0) return hipErrorInvalidValue;
    return launch_rows<kModeAcoTour, false>(S, tl, t0, steps, last, s);
  }
  if (rows_stream(tl))
    return mode == kModeLem ? launch_rows<kModeLem, true>(S, tl, t0, steps, last, s)
                            : launch_rows<kModeAco, true>(S, tl, t0, steps, last, s);
  if (rows_engine(tl))
    return mode == kModeLem ? launch_rows<kModeLem, false>(S, tl, t0, steps, last, s)
                            : launch_rows<kModeAco, false>(S, tl, t0, steps, last, s);
  if (tl.nw == 1)
    return mode == kModeLem ? launch_one<1, kModeLem>(S, tl, t0, steps, last, s)
                            : launch_one<1, kModeAco>(S, tl, t0, steps, last, s);
  return mode == kModeLem ? launch_one<2, kModeLem>(S, tl, t0, steps, last, s)
                          : launch_one<2, kModeAco>(S, tl, t0, steps, last, s);
}

// ---------------------------------------------------------------------------
// counters without stepping
// ---------------------------------------------------------------------------
constexpr int kCountTX = 64, kCountTY = 4;

__global__ __launch_bounds__(256) void count_kernel(const uint8_t* code, int W, int H, int cross_a, int cross_b,
                                                    uint32_t* stats) {
  __shared__ uint32_t s_cnt[kTileStatFields];
  const int x = blockIdx.x * kCountTX + (threadIdx.x % kCountTX);
  const int y = blockIdx.y * kCountTY + (threadIdx.x / kCountTX);
  int g = kWall;
  if (x < W && y < H) g = code[(size_t)y * W + x];
  if (threadIdx.x < kTileStatFields) s_cnt[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t v[kTileStatFields] = {(uint32_t)__popcll(__ballot(g == kGroupA)),
                                       (uint32_t)__popcll(__ballot(g == kGroupB)),
                                       (uint32_t)__popcll(__ballot(g == kGroupA && x >= W - cross_b)),
                                       (uint32_t)__popcll(__ballot(g == kGroupB && x < cross_a)), 0u};
  if ((threadIdx.x & 63) == 0)
    for (int f = 0; f < kTileStatFields; ++f) atomicAdd(&s_cnt[f], v[f]);
  __syncthreads();
  const int blin = blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x < kTileStatFields) stats[(size_t)blin * kTileStatFields + threadIdx.x] = s_cnt[threadIdx.x];
}

hipError_t launch_count(const uint8_t* code, int W, int H, int cross_a, int cross_b, uint32_t* stats, int* entries,
                        hipStream_t s) {
  const dim3 grid((W + kCountTX - 1) / kCountTX, (H + kCountTY - 1) / kCountTY);
  *entries = (int)(grid.x * grid.y);
  count_kernel<<<grid, kCountTX * kCountTY, 0, s>>>(code, W, H, cross_a, cross_b, stats);
  return hipGetLastError();
}

// Sum per-tile counters into kTileStatFields 64-bit totals.
__global__ __launch_bounds__(256) void reduce_counts_kernel(const uint32_t* stats, int entries,
                                                            unsigned long long* out) {
  __shared__ unsigned long long s[256];
  for (int f = 0; f < kTileStatFields; ++f) {
    unsigned long long acc = 0;
    for (int b = threadIdx.x; b < entries; b += 256) acc += stats[(size_t)b * kTileStatFields + f];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[f] = s[0];
    __syncthreads();
  }
}

hipError_t launch_reduce_counts(const uint32_t* stats, int entries, unsigned long long* out, hipStream_t s) {
  reduce_counts_kernel<<<1, 256, 0, s>>>(stats, entries, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// create-time validation
// ---------------------------------------------------------------------------
// counters: [0] agents A, [1] agents B, [2] bad-state flag
__global__ __launch_bounds__(256) void validate_cells_kernel(const uint8_t* code, const uint32_t* id,
                                                             const float* tau, size_t cells,
                                                             unsigned long long* counters) {
  unsigned long long na = 0, nb = 0;
  unsigned bad = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < cells; i += (size_t)gridDim.x * 256) {
    const int g = code[i];
    const uint32_t k = id[i];
    const bool agent = g == kGroupA || g == kGroupB;
    if (g > kWall) bad = 1;
    if (agent != (k != 0u)) bad = 1;
    na += g == kGroupA;
    nb += g == kGroupB;
    if (tau) {
      const float ta = tau[i], tb = tau[cells + i];
      if (!(ta >= 0.0f && ta <= 3.402823466e38f)) bad = 1;
      if (!(tb >= 0.0f && tb <= 3.402823466e38f)) bad = 1;
    }
  }
  // one atomic per wave: sum the lanes' counts with cross-lane shuffles first
  for (int off = 32; off > 0; off >>= 1) {
    na += __shfl_down(na, off, 64);
    nb += __shfl_down(nb, off, 64);
  }
  const bool any_bad = __ballot(bad != 0u) != 0ull;
  if ((threadIdx.x & 63) == 0) {
    if (na) atomicAdd(&counters[0], na);
    if (nb) atomicAdd(&counters[1], nb);
    if (any_bad) atomicOr(&counters[2], 1ull);
  }
}

// Each agent id must be in 1..n and appear once: mark a bitmap.
__global__ __launch_bounds__(256) void validate_ids_kernel(const uint32_t* id, size_t cells, uint32_t n,
                                                           uint32_t* bitmap, unsigned long long* counters) {
  unsigned bad = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < cells; i += (size_t)gridDim.x * 256) {
    const uint32_t k = id[i];
    if (k == 0u) continue;
    if (k > n) {
      bad = 1;
      continue;
    }
    const uint32_t bit = 1u << ((k - 1u) & 31u);
    const uint32_t old = atomicOr(&bitmap[(k - 1u) >> 5], bit);
    if (old & bit) bad = 1;
  }
  if (bad) atomicOr(&counters[2], 1ull);
}

hipError_t launch_validate(const uint8_t* code, const uint32_t* id, const float* tau, size_t cells,
                           unsigned long long* counters, hipStream_t s) {
  int blocks = (int)((cells + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  validate_cells_kernel<<<blocks, 256, 0, s>>>(code, id, tau, cells, counters);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void validate_values_kernel(const float* v, size_t n,
                                                              unsigned long long* counters) {
  unsigned bad = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float x = v[i];
    if (!(x >= 0.0f && x <= 3.402823466e38f)) bad = 1;
  }
  if (bad) atomicOr(&counters[2], 1ull);
}

// Clear `words` 32-bit words with stores from a kernel (not a memset node:
// the calls that clear counters may be recorded into a graph by a caller).
__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t* p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

hipError_t launch_zero_words(void* p, size_t words, hipStream_t s) {
  if (words == 0) return hipSuccess;
  int blocks = (int)((words + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  zero_words_kernel<<<blocks, 256, 0, s>>>((uint32_t*)p, words);
  return hipGetLastError();
}

hipError_t launch_validate_values(const float* v, size_t n, unsigned long long* counters, hipStream_t s) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  validate_values_kernel<<<blocks, 256, 0, s>>>(v, n, counters);
  return hipGetLastError();
}

hipError_t launch_validate_ids(const uint32_t* id, size_t cells, uint32_t n, uint32_t* bitmap,
                               unsigned long long* counters, hipStream_t s) {
  int blocks = (int)((cells + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  validate_ids_kernel<<<blocks, 256, 0, s>>>(id, cells, n, bitmap, counters);
  return hipGetLastError();
}

}  // namespace pedsim
