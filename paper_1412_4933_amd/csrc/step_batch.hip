// Batched form: one persistent kernel launch advances every active scenario
// of a batch by up to k steps. Workgroups claim (scenario, tile) work items
// from a per-launch counter; each item runs the tile engine with the
// scenario's own parameters and mode (LEM or ACO), so scenarios of any size
// and mode share the launch. A call is a fixed sequence (counter reset, one
// launch per k steps, copy back of scenarios whose state ended in their
// shadow planes) that the host captures once in a hipGraph and replays with
// new tables.
#include "pedsim_internal.hpp"

namespace pedsim {

// readfirstlane returns a signed int: widen through uint32_t so that the low
// word is not sign-extended into the high one.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  return ((uint64_t)uniform_u32((uint32_t)(v >> 32)) << 32) | (uint64_t)uniform_u32((uint32_t)v);
}

// A workgroup-uniform copy of a scenario read from global memory: every word
// goes through readfirstlane, so the copy (and everything derived from it)
// lives in scalar registers.
__device__ __forceinline__ Scenario uniform_scenario(const Scenario* src) {
  static_assert(sizeof(Scenario) % 4 == 0, "Scenario must be a whole number of words");
  Scenario out;
  const uint32_t* w = (const uint32_t*)src;
  uint32_t* o = (uint32_t*)&out;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(Scenario) / 4); ++i) o[i] = uniform_u32(w[i]);
  return out;
}

// The work item's scenario for launch j, with the planes it reads and writes.
struct ItemView {
  Scenario S;
  uint64_t t0;
  int steps, mode, tile;
  bool last;
};

__device__ __forceinline__ ItemView item_view(const BatchPlan& P, const BatchEntry* E, int lo, int item, int j) {
  ItemView v;
  const int slot = __builtin_amdgcn_readfirstlane(E[lo].slot);
  const int first = __builtin_amdgcn_readfirstlane(E[lo].first);
  const BatchSlot& B = P.slots[slot];
  v.S = uniform_scenario(&B.S);
  const int par = j & 1;
  v.S.code_in = (const uint8_t*)uniform_u64((uint64_t)B.code[par]);
  v.S.id_in = (const uint32_t*)uniform_u64((uint64_t)B.id[par]);
  v.S.tau_in = (const float*)uniform_u64((uint64_t)B.tau[par]);
  v.S.code_out = (uint8_t*)uniform_u64((uint64_t)B.code[par ^ 1]);
  v.S.id_out = (uint32_t*)uniform_u64((uint64_t)B.id[par ^ 1]);
  v.S.tau_out = (float*)uniform_u64((uint64_t)B.tau[par ^ 1]);
  v.S.tour_in = (const float*)uniform_u64((uint64_t)B.tour[par]);
  v.S.tour_out = (float*)uniform_u64((uint64_t)B.tour[par ^ 1]);
  const int bsteps = __builtin_amdgcn_readfirstlane(B.steps);
  v.mode = __builtin_amdgcn_readfirstlane(B.mode);
  const int done = j * P.k;
  v.steps = bsteps - done < P.k ? bsteps - done : P.k;
  v.last = done + v.steps == bsteps;
  v.t0 = uniform_u64(B.t0) + (uint64_t)done;
  v.tile = item - first;
  return v;
}

template <int NW>
__global__ __launch_bounds__(1024) void batch_kernel(BatchPlan P, int j) {
  extern __shared__ __align__(16) uint8_t smem[];
  // the claimed item is passed through the word after the tile's LDS layout
  int& s_item = *(int*)(smem + Layout<NW>{P.rows, true}.bytes());
  const int count = P.counts[j];
  const int total = P.totals[j];
  const BatchEntry* E = P.entries + (size_t)j * P.capacity;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&P.counters[j], 1u);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= total) break;
    int lo = 0, hi = count - 1;  // last entry whose first item is <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (E[mid].first <= item) lo = mid; else hi = mid - 1;
    }
    const ItemView v = item_view(P, E, lo, item, j);
    const int tx = v.tile % v.S.tiles_x, ty = v.tile / v.S.tiles_x;
    if (v.mode == kModeAco)
      advance_tile<NW, kModeAco>(v.S, smem, P.rows, tx, ty, v.tile, v.t0, v.steps, v.last);
    else
      advance_tile<NW, kModeLem>(v.S, smem, P.rows, tx, ty, v.tile, v.t0, v.steps, v.last);
  }
}

// The same with the row-lane engine (regions of 64 columns).
template <bool STREAM, bool NB8 = false>
__global__ __launch_bounds__(kRowsMaxThreads, kRowsMinWavesPerSimd) void batch_rows_kernel(BatchPlan P, int j) {
  extern __shared__ __align__(16) uint8_t smem[];
  int& s_item = *(int*)(smem + RowsLayout{P.rows, P.k, true, STREAM, !STREAM && P.tour != 0, NB8}.bytes());
  const int count = P.counts[j];
  const int total = P.totals[j];
  const BatchEntry* E = P.entries + (size_t)j * P.capacity;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&P.counters[j], 1u);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= total) break;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (E[mid].first <= item) lo = mid; else hi = mid - 1;
    }
    const ItemView v = item_view(P, E, lo, item, j);
    const int tx = v.tile % v.S.tiles_x, ty = v.tile / v.S.tiles_x;
    if constexpr (!STREAM) {
      if (v.mode == kModeAcoTour) {
        advance_tile_rows<kModeAcoTour, false, NB8>(v.S, smem, P.rows, P.k, tx, ty, v.tile, v.t0, v.steps, v.last);
        continue;
      }
    }
    if (v.mode == kModeAco)
      advance_tile_rows<kModeAco, STREAM, NB8>(v.S, smem, P.rows, P.k, tx, ty, v.tile, v.t0, v.steps, v.last);
    else
      advance_tile_rows<kModeLem, STREAM, NB8>(v.S, smem, P.rows, P.k, tx, ty, v.tile, v.t0, v.steps, v.last);
  }
}

__global__ void batch_reset_kernel(unsigned* counters, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0u;
}

// A slot that ran an odd number of launches has its state in the shadow
// planes: copy it back (blockIdx.y = slot).
__global__ __launch_bounds__(256) void batch_copyback_kernel(BatchPlan P) {
  const BatchSlot& B = P.slots[blockIdx.y];
  if (B.steps <= 0) return;
  const int launches = (B.steps + P.k - 1) / P.k;
  if ((launches & 1) == 0) return;
  const size_t cells = (size_t)B.S.W * (size_t)B.S.H;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += stride) {
    B.code[0][i] = B.code[1][i];
    B.id[0][i] = B.id[1][i];
    if (B.mode != kModeLem) {
      B.tau[0][i] = B.tau[1][i];
      B.tau[0][cells + i] = B.tau[1][cells + i];
    }
  }
  if (B.mode == kModeAcoTour)
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < B.agents; i += stride) B.tour[0][i] = B.tour[1][i];
}

hipError_t launch_batch_reset(const BatchPlan& P, int launches, hipStream_t s) {
  batch_reset_kernel<<<1, 256, 0, s>>>(P.counters, launches);
  return hipGetLastError();
}

void prepare_batch_kernels() {
  static bool done = false;
  if (done) return;
  (void)hipFuncSetAttribute((const void*)batch_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_dynamic_lds());
  (void)hipFuncSetAttribute((const void*)batch_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_dynamic_lds());
  (void)hipFuncSetAttribute((const void*)batch_rows_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_dynamic_lds());
  (void)hipFuncSetAttribute((const void*)batch_rows_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_dynamic_lds());
  (void)hipFuncSetAttribute((const void*)batch_rows_kernel<false, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_dynamic_lds());
  (void)hipGetLastError();  // an unsupported attribute value must not linger as the last error
  done = true;
}

template <int NW>
static hipError_t launch_batch_nw(const BatchPlan& P, const Tiling& tl, int j, int grid, hipStream_t s) {
  const size_t lds = Layout<NW>{tl.rows, true}.bytes() + kBatchItemBytes;
  batch_kernel<NW><<<grid, tl.threads, lds, s>>>(P, j);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchPlan& P, const Tiling& tl, int j, int grid, hipStream_t s) {
  if (P.nb8) {
    if (tl.nw != 0) return hipErrorInvalidValue;
    const size_t lds = RowsLayout{tl.rows, tl.steps, true, false, P.tour != 0, true}.bytes() + kBatchItemBytes;
    batch_rows_kernel<false, true><<<grid, tl.threads, lds, s>>>(P, j);
    return hipGetLastError();
  }
  if (P.tour && tl.nw != 0) return hipErrorInvalidValue;
  if (rows_engine(tl)) {
    const size_t lds =
        RowsLayout{tl.rows, tl.steps, true, rows_stream(tl), P.tour != 0 && !rows_stream(tl)}.bytes() + kBatchItemBytes;
    if (rows_stream(tl))
      batch_rows_kernel<true><<<grid, tl.threads, lds, s>>>(P, j);
    else
      batch_rows_kernel<false><<<grid, tl.threads, lds, s>>>(P, j);
    return hipGetLastError();
  }
  return tl.nw == 1 ? launch_batch_nw<1>(P, tl, j, grid, s) : launch_batch_nw<2>(P, tl, j, grid, s);
}

hipError_t launch_batch_copyback(const BatchPlan& P, int capacity, hipStream_t s) {
  batch_copyback_kernel<<<dim3(64, capacity), 256, 0, s>>>(P);
  return hipGetLastError();
}

int device_cu_count() {
  static int cached = -1;
  if (cached < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cached = v;
  }
  return cached;
}

}  // namespace pedsim
