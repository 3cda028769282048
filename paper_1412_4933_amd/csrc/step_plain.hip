// Single-scenario step kernels for gfx950.
//
// One step of the paper's update (Sec. IV.b-d) runs as two kernels:
//
//   decide  (request + resolve, the paper's initial-calculation and
//            tour-construction phases plus the gather half of its movement
//            phase): a workgroup stages the code plane of its tile plus a
//            2-cell halo in LDS, computes the request of every agent of the
//            tile plus a 1-cell ring, then every empty cell of the tile
//            gathers the neighbours whose request points at it and keeps the
//            lowest (Philox word 0, agent number). It writes one decision byte
//            per cell (request code on agent cells; winner slot and group on
//            empty cells) and the winner's id into the receiving cell.
//   commit  (the rest of the movement phase + pheromone update): each cell
//            reads its own code and decision byte; a receiving cell takes the
//            winner's group, a winning agent's cell empties (it checks its
//            target's winner slot), then both pheromone planes evaporate and
//            receive the deposit (eq. 3 then eq. 4), and wave64 ballots count
//            agents, crossings and moves per workgroup.
//
// Both kernels update the caller's planes in place without races: decide
// reads codes everywhere and ids only on agent cells, and writes ids only on
// cells that are empty at t; commit touches only its own cell's code, id and
// pheromone and reads decision bytes, which nobody writes during commit.
#include "pedsim_internal.hpp"

namespace pedsim {

// ---------------------------------------------------------------------------
// decide
// ---------------------------------------------------------------------------
constexpr int kHX = kDecideTX + 4;  // staged code region (2-cell halo)
constexpr int kHY = kDecideTY + 4;
constexpr int kRX = kDecideTX + 2;  // request ring (1-cell halo)
constexpr int kRY = kDecideTY + 2;

__device__ __forceinline__ int tile_of_block(int bid, int ntiles) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD one
  // contiguous run of row-major tiles so halo lines are reused in its L2.
  const int per = (ntiles + 7) >> 3;
  return (bid & 7) * per + (bid >> 3);
}

template <int MODE>
__global__ __launch_bounds__(kDecideThreads) void decide_kernel(StepArgs a) {
  __shared__ uint8_t s_code[kHY * kHX];
  __shared__ uint8_t s_req[kRY * kRX];

  const int tile = tile_of_block(blockIdx.x, a.tiles_x * a.tiles_y);
  if (tile >= a.tiles_x * a.tiles_y) return;
  const int x0 = (tile % a.tiles_x) * kDecideTX;
  const int y0 = (tile / a.tiles_x) * kDecideTY;
  const int W = a.W, H = a.H;

  for (int i = threadIdx.x; i < kHY * kHX; i += kDecideThreads) {
    const int gx = x0 + (i % kHX) - 2;
    const int gy = y0 + (i / kHX) - 2;
    uint8_t v = kWall;
    if (gx >= 0 && gx < W && gy >= 0 && gy < H) v = a.code[(size_t)gy * W + gx];
    s_code[i] = v;
  }
  __syncthreads();

  // Requests on the tile plus a 1-cell ring, from the snapshot of time t.
  for (int i = threadIdx.x; i < kRY * kRX; i += kDecideThreads) {
    const int rx = i % kRX, ry = i / kRX;
    const int c = (ry + 1) * kHX + (rx + 1);
    const int g = s_code[c];
    int req = kReqNone;
    if (g == kGroupA || g == kGroupB) {
      const int d = g == kGroupA ? 1 : -1;
      if (s_code[c + d] == kEmpty) {
        req = kReqF;
      } else {
        const unsigned avail = (unsigned)(s_code[c - kHX + d] == kEmpty) |
                               ((unsigned)(s_code[c + kHX + d] == kEmpty) << 1) |
                               ((unsigned)(s_code[c - kHX] == kEmpty) << 2) |
                               ((unsigned)(s_code[c + kHX] == kEmpty) << 3);
        if (avail) {
          const int gx = x0 + rx - 1, gy = y0 + ry - 1;
          const size_t gi = (size_t)gy * W + gx;
          const Words w = agent_words(a.id[gi] - 1u, a.t, a.key0, a.key1);
          if (MODE == kModeLem) {
            req = lem_choose(avail, w.w1, w.w2);
          } else {
            const float* plane = g == kGroupA ? a.tau_a : a.tau_b;
            float tau[4];
            tau[0] = (avail & 1u) ? plane[gi - W + d] : 0.0f;
            tau[1] = (avail & 2u) ? plane[gi + W + d] : 0.0f;
            tau[2] = (avail & 4u) ? plane[gi - W] : 0.0f;
            tau[3] = (avail & 8u) ? plane[gi + W] : 0.0f;
            req = aco_choose(avail, tau, a.alpha, a.eta_diag, a.eta_lat, w.w1, w.w2);
          }
        }
      }
    }
    s_req[i] = (uint8_t)req;
  }
  __syncthreads();

  // Resolve: every cell of the tile that is empty at t gathers its requesters.
  for (int i = threadIdx.x; i < kDecideTY * kDecideTX; i += kDecideThreads) {
    const int lx = i % kDecideTX, ly = i / kDecideTX;
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx >= W || gy >= H) continue;
    const size_t gi = (size_t)gy * W + gx;
    const int c = (ly + 2) * kHX + (lx + 2);
    const int g = s_code[c];
    uint8_t dec = 0;
    if (g == kGroupA || g == kGroupB) {
      dec = s_req[(ly + 1) * kRX + (lx + 1)];
    } else if (g == kEmpty) {
      int count = 0, win_dx = 0, win_dy = 0;
      unsigned cand = 0;  // bit (slot-1) set for each requester
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (dx == 0 && dy == 0) continue;
          const int ng = s_code[c + dy * kHX + dx];
          if (ng != kGroupA && ng != kGroupB) continue;
          const int r = s_req[(ly + 1 + dy) * kRX + (lx + 1 + dx)];
          if (r == kReqNone) continue;
          const int d = ng == kGroupA ? 1 : -1;
          if (dx + req_dx(r, d) == 0 && dy + req_dy(r) == 0) {
            count += 1;
            cand |= 1u << (slot_of(dx, dy) - 1);
            win_dx = dx;
            win_dy = dy;
          }
        }
      }
      if (count > 1) {
        // Several requesters: lowest (word 0, agent number) wins.
        uint32_t best_t = 0xFFFFFFFFu, best_k = 0xFFFFFFFFu;
        bool have = false;
        while (cand) {
          const int s = __ffs(cand) - 1;
          cand &= cand - 1;
          const int dx = s % 3 - 1, dy = s / 3 - 1;
          const uint32_t k = a.id[gi + (ptrdiff_t)dy * W + dx] - 1u;
          const uint32_t tk = agent_words(k, a.t, a.key0, a.key1).w0;
          if (!have || tk < best_t || (tk == best_t && k < best_k)) {
            have = true;
            best_t = tk;
            best_k = k;
            win_dx = dx;
            win_dy = dy;
          }
        }
      }
      if (count > 0) {
        const size_t src = gi + (ptrdiff_t)win_dy * W + win_dx;
        const int wg = s_code[c + win_dy * kHX + win_dx];
        dec = (uint8_t)((wg << 4) | slot_of(win_dx, win_dy));
        a.id[gi] = a.id[src];
      }
    }
    a.dec[gi] = dec;
  }
}

// ---------------------------------------------------------------------------
// commit + pheromone + counters
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_counts(bool agent_a, bool agent_b, bool cross_a, bool cross_b,
                                             bool moved, uint32_t* out) {
  __shared__ uint32_t s_cnt[kCommitThreads / 64][kStatFields];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t v[kStatFields] = {
      (uint32_t)__popcll(__ballot(agent_a)), (uint32_t)__popcll(__ballot(agent_b)),
      (uint32_t)__popcll(__ballot(cross_a)), (uint32_t)__popcll(__ballot(cross_b)),
      (uint32_t)__popcll(__ballot(moved))};
  if (lane == 0) {
#pragma unroll
    for (int f = 0; f < kStatFields; ++f) s_cnt[wave][f] = v[f];
  }
  __syncthreads();
  if (threadIdx.x < kStatFields) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kCommitThreads / 64; ++w) s += s_cnt[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

template <int MODE>
__global__ __launch_bounds__(kCommitThreads) void commit_kernel(StepArgs a, int write_stats) {
  const int x = blockIdx.x * kCommitTX + (threadIdx.x % kCommitTX);
  const int y = blockIdx.y * kCommitTY + (threadIdx.x / kCommitTX);
  const int W = a.W, H = a.H;
  const bool in = x < W && y < H;
  int g_new = kWall;
  bool moved_in = false;
  if (in) {
    const size_t gi = (size_t)y * W + x;
    const int g = a.code[gi];
    const int dec = a.dec[gi];
    g_new = g;
    if (g == kEmpty) {
      if (dec & 0xF) {
        g_new = dec >> 4;
        moved_in = true;
      }
    } else if ((g == kGroupA || g == kGroupB) && dec != kReqNone) {
      const int d = g == kGroupA ? 1 : -1;
      const int dx = req_dx(dec, d), dy = req_dy(dec);
      const int back = a.dec[gi + (ptrdiff_t)dy * W + dx] & 0xF;
      if (back == slot_of(-dx, -dy)) {
        g_new = kEmpty;
        a.id[gi] = 0u;
      }
    }
    if (g_new != g) a.code[gi] = (uint8_t)g_new;
    if (MODE == kModeAco) {
      float va = a.keep * a.tau_a[gi];
      float vb = a.keep * a.tau_b[gi];
      if (g_new == kGroupA) va = va + a.dtau;
      if (g_new == kGroupB) vb = vb + a.dtau;
      a.tau_a[gi] = va;
      a.tau_b[gi] = vb;
    }
  }
  if (write_stats) {
    const int blin = blockIdx.y * gridDim.x + blockIdx.x;
    block_counts(g_new == kGroupA, g_new == kGroupB, g_new == kGroupA && x >= W - a.cross_b,
                 g_new == kGroupB && x < a.cross_a, moved_in, a.block_stats + (size_t)blin * kStatFields);
  }
}

// Counters of the current planes without stepping (used after create).
__global__ __launch_bounds__(kCommitThreads) void count_kernel(StepArgs a) {
  const int x = blockIdx.x * kCommitTX + (threadIdx.x % kCommitTX);
  const int y = blockIdx.y * kCommitTY + (threadIdx.x / kCommitTX);
  int g = kWall;
  if (x < a.W && y < a.H) g = a.code[(size_t)y * a.W + x];
  const int blin = blockIdx.y * gridDim.x + blockIdx.x;
  block_counts(g == kGroupA, g == kGroupB, g == kGroupA && x >= a.W - a.cross_b,
               g == kGroupB && x < a.cross_a, false, a.block_stats + (size_t)blin * kStatFields);
}

// Sum the per-workgroup counters into kStatFields 64-bit totals.
__global__ __launch_bounds__(256) void reduce_counts_kernel(const uint32_t* block_stats, int nblocks,
                                                            unsigned long long* out) {
  __shared__ unsigned long long s[256];
  for (int f = 0; f < kStatFields; ++f) {
    unsigned long long acc = 0;
    for (int b = threadIdx.x; b < nblocks; b += 256) acc += block_stats[(size_t)b * kStatFields + f];
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
  atomicAdd(&counters[0], na);
  atomicAdd(&counters[1], nb);
  if (bad) atomicOr(&counters[2], 1ull);
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

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
const char* const kKernelNames[kKernelKinds] = {"decide", "commit"};

hipError_t launch_step(const StepArgs& a, int mode, int write_stats, hipStream_t s, hipEvent_t* ev) {
  const int ntiles = a.tiles_x * a.tiles_y;
  const int nblocks = ((ntiles + 7) / 8) * 8;
  const dim3 cgrid(a.commit_bx, a.commit_by);
  if (ev) (void)hipEventRecord(ev[0], s);
  if (mode == kModeLem)
    decide_kernel<kModeLem><<<nblocks, kDecideThreads, 0, s>>>(a);
  else
    decide_kernel<kModeAco><<<nblocks, kDecideThreads, 0, s>>>(a);
  if (ev) (void)hipEventRecord(ev[1], s);
  if (mode == kModeLem)
    commit_kernel<kModeLem><<<cgrid, kCommitThreads, 0, s>>>(a, write_stats);
  else
    commit_kernel<kModeAco><<<cgrid, kCommitThreads, 0, s>>>(a, write_stats);
  if (ev) (void)hipEventRecord(ev[2], s);
  return hipGetLastError();
}

hipError_t launch_count(const StepArgs& a, hipStream_t s) {
  count_kernel<<<dim3(a.commit_bx, a.commit_by), kCommitThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_reduce_counts(const uint32_t* block_stats, int nblocks, unsigned long long* out,
                                hipStream_t s) {
  reduce_counts_kernel<<<1, 256, 0, s>>>(block_stats, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_validate(const uint8_t* code, const uint32_t* id, const float* tau, size_t cells,
                           unsigned long long* counters, hipStream_t s) {
  int blocks = (int)((cells + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  validate_cells_kernel<<<blocks, 256, 0, s>>>(code, id, tau, cells, counters);
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
