// Row-lane tile engine: one workgroup advances one tile of a scenario by k
// steps of the bi-directional pedestrian update (Sec. III, Sec. IV.b-d).
//
// The region is 64 columns x R rows (R <= 64) around the tile: the interior
// plus a halo of 3k cells on every side, as in the multi-wave engine (after
// k steps the cells at least 3k from the region border are exact). Outside
// the region counts as wall.
//
// Wave 0 is the mask wave: lane r owns row r, whose A, B and wall masks (one
// bit per cell) stay in its registers for the whole launch; rows r-1 and r+1
// are read with full-wave DPP shifts. Every decision that follows from
// occupancy alone is mask arithmetic in that wave: forward requests, side
// requests of agents with exactly one empty side candidate (LEM and ACO both
// take the only candidate), the cells that can possibly be contested, and the
// commit. Only agents that draw a choice (two or more empty side candidates)
// or that may meet a contest need their Philox words; they are queued and
// all waves draw them together, so a step has one Philox pass, and its word
// 0 is kept as the agent's ticket for the resolution (the streaming form, the
// tour variant and the eight-neighbour form keep no tickets: only choices are
// queued, and a contested cell draws its contenders' words again).
//
// Per step (B = workgroup barrier):
//   1. masks     (wave 0) forward requests, single-candidate side requests,
//                possibly contested cells; queue the agents that draw   B
//   2. draw      (all) Philox words, tickets, LEM (eq. 1) / ACO (eq. 2)
//                choices or-ed into side-request masks                  B
//   3. gather    (wave 0) requester masks per target, in eight
//                directions; queue every requested cell                 B
//   4. resolve   (all) contested cells keep the lowest (ticket, agent
//                number) (Sec. IV.d); every winner's id moves to its
//                target (targets were empty and sources occupied at the
//                start of the step, so the moves never overlap)         B
//   5. commit    (wave 0) new occupancy, recorded in an LDS history.
// Ids live in LDS; the pheromone planes are staged in LDS and never rewritten
// during the launch: a cell's value after s steps is fl(keep * v) (+ dtau when
// the group occupies it) applied s times, using the recorded occupancy,
// exactly the per-step update of eq. 3 then eq. 4; it is evaluated where
// needed (ACO candidates in step 2, every interior cell at write-back).
//
// Tour variant (MODE 2, eq. 5): a per-cell LDS copy of the tour length of the
// agent standing there moves with the agent, grown by each move's length in
// step 4. Deposits land only on entered cells, so step 4 also brings the
// entered cell's value up to date (the evaporations since its last deposit in
// this launch, then fl(dtau / L)) and stores it; every other evaluation only
// owes the evaporations since a cell's last deposit, read off the history
// (an agent of group g entered cell c in step u iff c was empty before step u
// and holds g after it).
#pragma once

#include "rules.hpp"
#include "tile_engine.hpp"

namespace pedsim {

constexpr int kRowsMaxRows = 64;
constexpr int kRowsMaxSteps = 8;
constexpr int kRowsMaxThreads = 512;  // workgroup size limit
// Register budget: at least 4 waves per SIMD (<= 128 VGPRs), so that two
// 512-thread workgroups share a compute unit.
constexpr int kRowsMinWavesPerSimd = 4;

// LDS layout of a row-lane region of R rows x 64 columns, k steps per launch.
struct RowsLayout {
  int R, k;
  bool aco;
  bool stream;        // pheromone read from HBM, tickets recomputed: no tick or tau arrays
  bool tour = false;  // tour variant: tour lengths per cell
  bool nb8 = false;   // eight-neighbour candidates: side requests kept per move direction (8 masks)
  __host__ __device__ size_t hist() const { return 0; }                                  // [k+1][2][R] u64
  __host__ __device__ size_t wall() const { return hist() + (size_t)(k + 1) * 2 * R * 8; }  // [R] u64
  __host__ __device__ size_t side() const { return wall() + (size_t)R * 8; }             // [6][R] u64
  __host__ __device__ size_t reqm() const { return side() + (size_t)(nb8 ? 8 : 6) * R * 8; }  // [8][R] u64
  __host__ __device__ size_t cwin() const { return reqm() + (size_t)8 * R * 8; }         // [8][R] u64
  __host__ __device__ size_t moved() const { return cwin() + (size_t)8 * R * 8; }        // [R] u64
  __host__ __device__ size_t ctl() const { return moved() + (size_t)R * 8; }             // 16 u32
  __host__ __device__ size_t ids() const { return ctl() + 64; }                         // [R][64] u32
  __host__ __device__ size_t tick() const { return ids() + (size_t)R * 256; }           // [R][64] u32
  __host__ __device__ size_t queue() const { return tick() + (stream || tour || nb8 ? 0 : (size_t)R * 256); }  // [R*64] u16
  __host__ __device__ size_t tau() const { return queue() + (size_t)R * 128; }          // [2][R][64] f32
  __host__ __device__ size_t tour_len() const { return tau() + (aco && !stream ? (size_t)R * 512 : 0); }  // [R][64] f32
  __host__ __device__ size_t bytes() const { return tour_len() + (tour ? (size_t)R * 256 : 0); }
};

// Row r-1's value in lane r (0 in lane 0) / row r+1's value in lane r (0 in lane 63).
__device__ __forceinline__ uint64_t from_up(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)v, 0x138, 0xF, 0xF, false);  // wave_shr:1
  const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(v >> 32), 0x138, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t from_down(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)v, 0x130, 0xF, 0xF, false);  // wave_shl:1
  const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(v >> 32), 0x130, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

// Number of lanes below this one whose bit is set in `bal`.
__device__ __forceinline__ int lanes_below(uint64_t bal) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}

// Wave 0: append (row = lane, column) of every set bit of `bits` to `queue`
// as row | column << 6; returns the number appended (wave-uniform). Lanes
// take turns bit by bit, so the loop runs as many times as the fullest row
// has bits.
__device__ __forceinline__ int enqueue_row_bits(uint16_t* queue, uint64_t bits, int lane) {
  int base = 0;
  for (;;) {
    const bool has = bits != 0ull;
    const uint64_t bal = __ballot(has);
    if (bal == 0ull) break;
    if (has) {
      const int c = __ffsll((unsigned long long)bits) - 1;
      bits &= bits - 1ull;
      queue[base + lanes_below(bal)] = (uint16_t)(lane | (c << 6));
    }
    base += __popcll(bal);
  }
  return base;
}

// Row `lane` of the cells that step s of a launch must still get right.
// After the launch only the interior (the region minus a halo of h cells)
// must be exact, and a cell's new state reaches 3 cells back (its own or its
// agent's target's contest, whose requesters chose on their neighbours), so
// step s must commit exactly the interior grown by m = 3 (steps - 1 - s)
// cells, resolve the contests up to m + 1 cells out and draw for the agents
// up to m + 2 cells out; work farther out only feeds cells that are never
// read again. Returns the bits of the interior grown by `grow` cells (all of
// the region when that covers it).
__device__ __forceinline__ uint64_t live_window(int grow, int h, int R, int lane) {
  const int lo = h - grow;
  if (lo <= 0) return ~0ull;
  if (lane < lo || lane >= R - lo) return 0ull;
  const int hi = 64 - lo;  // exclusive, > lo because the interior is at least 16 wide
  return (~0ull << lo) & ((1ull << hi) - 1ull);
}

// Staging: a thread loads the cells of column `lane` in rows wave + j * nwaves
// (j < kStageRows per batch) into registers, all loads in flight together,
// then converts them into the region's LDS form.
constexpr int kStageRows = 8;

struct StageRegs {
  int g[kStageRows];
  uint32_t id[kStageRows];
  float ta[kStageRows], tb[kStageRows];
};

// Rows row0 + j * nwaves (j < kStageRows) of the region at (x0, y0).
template <int MODE>
__device__ __forceinline__ void stage_issue(const Scenario& S, int R, int x0, int y0, int row0, int nwaves, int lane,
                                            StageRegs& q) {
  const size_t plane = (size_t)S.W * (size_t)S.H;
#pragma unroll
  for (int j = 0; j < kStageRows; ++j) {
    const int r = row0 + j * nwaves;
    const int gx = x0 + lane, gy = y0 + r;
    const bool in = r < R && gx >= 0 && gx < S.W && gy >= 0 && gy < S.H;
    const size_t gi = in ? (size_t)gy * S.W + gx : 0;
    q.g[j] = in ? S.code_in[gi] : kWall;
    q.id[j] = in ? S.id_in[gi] : 0u;
    if (MODE != 0) {
      q.ta[j] = in ? S.tau_in[gi] : 0.0f;
      q.tb[j] = in ? S.tau_in[plane + gi] : 0.0f;
    }
  }
}

// STREAM: the pheromone planes are not staged (the draw and the write-back read
// them from HBM and bring them up to date from the recorded occupancy) and
// contest tickets are recomputed instead of kept per cell, which leaves ids,
// masks and the queue as the region's only LDS and lets more workgroups share
// a compute unit on large grids.
// NB8: the paper's full neighbourhood (Sec. III), backward cells ranked last.
// Side requests are then kept by move direction rather than by kind and
// group: direction q moves an agent from the neighbour at (dir_dc(q),
// dir_dr(q)) of a cell into the cell, i.e. by the vector (-dir_dc(q),
// -dir_dr(q)); forward moves are directions 0 (A) and 1 (B), and every
// direction may carry either group.
// Returns whether the region held agents at the start of the launch.
template <int MODE, bool STREAM = false, bool NB8 = false>
__device__ bool advance_tile_rows(const Scenario& S, uint8_t* smem, int R, int k_max, int tx, int ty, int tile_index,
                                  uint64_t t0, int steps, bool last) {
  static_assert(!(NB8 && STREAM), "the eight-neighbour set runs on the LDS form only");
  // Contest tickets are kept per cell from the draw, except in the streaming
  // form, the tour variant and the eight-neighbour form, which draw a
  // contested cell's contenders again instead: that queues only the agents
  // that choose (with backward cells open, far more agents could meet a
  // contest than end up in one) and frees the LDS of the tickets.
  constexpr bool kTicks = !STREAM && MODE != 2 && !NB8;
  const RowsLayout L{R, k_max, MODE != 0, STREAM, MODE == 2, NB8};
  uint64_t* hist = (uint64_t*)(smem + L.hist());
  uint64_t* wall_m = (uint64_t*)(smem + L.wall());
  uint64_t* side = (uint64_t*)(smem + L.side());
  uint64_t* reqm = (uint64_t*)(smem + L.reqm());
  uint64_t* cwin = (uint64_t*)(smem + L.cwin());
  uint64_t* moved_m = (uint64_t*)(smem + L.moved());
  uint32_t* ctl = (uint32_t*)(smem + L.ctl());
  uint32_t* ids = (uint32_t*)(smem + L.ids());
  uint32_t* tick = (uint32_t*)(smem + L.tick());
  uint16_t* queue = (uint16_t*)(smem + L.queue());
  float* tau_a = (float*)(smem + L.tau());
  float* tau_b = tau_a + (size_t)R * 64;
  float* tlen = (float*)(smem + L.tour_len());  // tour variant only
  // occupancy of group g (0 = A, 1 = B) at step s of the launch, row r
  auto H = [&](int s, int g, int r) -> uint64_t& { return hist[((size_t)s * 2 + g) * R + r]; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: row loops and addresses stay scalar
  const int nthreads = blockDim.x;
  const int nwaves = nthreads >> 6;
  const bool mask_wave = wave == 0;
  const bool row_lane = lane < R;
  // The mask wave's phases (and the draws and contests of small queues,
  // which also land in wave 0) are the serial part of every step: let it
  // win instruction arbitration over the throughput phases of a workgroup
  // sharing its compute unit, and let every wave's step work go before
  // such a workgroup's write-back, which drops back to the base priority
  // (measured: 1024x512 ACO 7.18 -> 6.82 us/step, eight neighbours
  // 9.92 -> 9.53). The streaming form, four or five workgroups to a compute
  // unit, loses from it (256-scenario batch 8.5e9 -> 8.3e9 agent-steps/s).
  if (!STREAM) {
    if (mask_wave)
      __builtin_amdgcn_s_setprio(2);
    else
      __builtin_amdgcn_s_setprio(1);
  }
  const int h = S.halo;
  const int x0 = tx * S.IX - h;  // region origin in grid coordinates
  const int y0 = ty * S.IY - h;
  const size_t plane = (size_t)S.W * (size_t)S.H;
  const uint64_t lane_bit = 1ull << lane;

  // ---- stage: rows dealt round-robin to the waves, all loads in flight --
  for (int r0 = wave; r0 < R; r0 += nwaves * kStageRows) {
    StageRegs q;
    stage_issue<(STREAM ? 0 : MODE)>(S, R, x0, y0, r0, nwaves, lane, q);
#pragma unroll
    for (int j = 0; j < kStageRows; ++j) {
      const int r = r0 + j * nwaves;
      if (r >= R) break;
      const uint64_t ba = __ballot(q.g[j] == kGroupA), bb = __ballot(q.g[j] == kGroupB);
      const uint64_t bw = __ballot(q.g[j] == kWall);
      if (lane == 0) {
        H(0, 0, r) = ba;
        H(0, 1, r) = bb;
        wall_m[r] = bw;
      }
      ids[r * 64 + lane] = q.id[j];
      if (MODE != 0 && !STREAM) {
        tau_a[r * 64 + lane] = q.ta[j];
        tau_b[r * 64 + lane] = q.tb[j];
      }
    }
    if (MODE == 2) {  // the agents' tour lengths, gathered by agent number
      float len[kStageRows];
#pragma unroll
      for (int j = 0; j < kStageRows; ++j) {
        const int r = r0 + j * nwaves;
        len[j] = (r < R && q.id[j] != 0u) ? S.tour_in[q.id[j] - 1u] : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < kStageRows; ++j) {
        const int r = r0 + j * nwaves;
        if (r < R) tlen[r * 64 + lane] = len[j];
      }
    }
  }
  if (tid < 16) ctl[tid] = 0u;
  __syncthreads();

  // the mask wave's registers: row `lane` of the region (rows >= R: all wall)
  uint64_t A = 0ull, B = 0ull, Wl = ~0ull;
  if (mask_wave && row_lane) {
    A = H(0, 0, lane);
    B = H(0, 1, lane);
    Wl = wall_m[lane];
  }
  uint64_t moved_in = 0ull;
  uint64_t fA = 0ull, fB = 0ull;
  uint64_t rq[8];  // single-candidate side requests (six kinds, or eight move directions with NB8)
#pragma unroll
  for (int q = 0; q < 8; ++q) rq[q] = 0ull;
  uint64_t Wt[8];

  // A region without agents stays without agents in the interior for the
  // whole launch (an agent moves at most one cell per step and the halo is
  // 3 cells per step): its interior only evaporates, so the steps are skipped
  // and the write-back applies `steps` evaporations with no deposit. Every
  // wave reads the staged occupancy itself (no extra barrier).
  const bool empty_region = __ballot(row_lane && ((H(0, 0, lane) | H(0, 1, lane)) != 0ull)) == 0ull;
  const int run_steps = empty_region ? 0 : steps;

  for (int s = 0; s < run_steps; ++s) {
    const uint64_t t = t0 + (uint64_t)s;

    // ---- 1. masks: requests that need no random word; who must draw -------
    if (NB8 && mask_wave) {
      const uint64_t E = ~(A | B | Wl);
      const uint64_t Eu = from_up(E), Ed = from_down(E);
      const uint64_t e_r = E >> 1, e_l = E << 1;  // cell to the right / left is empty
      fA = A & e_r;
      fB = B & e_l;
      const uint64_t bl = (A & ~e_r) | (B & ~e_l);  // agents whose forward cell is blocked
      // their empty side candidates by move vector (dx, dy) of direction q
      uint64_t Sq[8];
      Sq[0] = B & ~e_l & e_r;  // (+1, 0): B backward
      Sq[1] = A & ~e_r & e_l;  // (-1, 0): A backward
      Sq[2] = bl & (Eu >> 1);  // (+1, -1)
      Sq[3] = bl & (Ed >> 1);  // (+1, +1)
      Sq[4] = bl & (Eu << 1);  // (-1, -1)
      Sq[5] = bl & (Ed << 1);  // (-1, +1)
      Sq[6] = bl & Eu;         // (0, -1)
      Sq[7] = bl & Ed;         // (0, +1)
      uint64_t ones = 0ull, multi = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        multi |= ones & Sq[q];
        ones |= Sq[q];
      }
      const uint64_t single = ones & ~multi;
#pragma unroll
      for (int q = 0; q < 8; ++q) rq[q] = single & Sq[q];
      // possible requesters of each cell, by direction; two or more: contestable
      const uint64_t Pv0 = Sq[0] | fA, Pv1 = Sq[1] | fB;
      const uint64_t P[8] = {Pv0 << 1,           Pv1 >> 1,           from_down(Sq[2]) << 1, from_up(Sq[3]) << 1,
                             from_down(Sq[4]) >> 1, from_up(Sq[5]) >> 1, from_down(Sq[6]),       from_up(Sq[7])};
      uint64_t pones = 0ull, twos = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        twos |= pones & P[q];
        pones |= P[q];
      }
      const uint64_t pu = from_up(twos), pd = from_down(twos);
      const uint64_t need =
          kTicks ? ((Pv0 & (twos >> 1)) | (Pv1 & (twos << 1)) | (Sq[2] & (pu >> 1)) | (Sq[3] & (pd >> 1)) |
                    (Sq[4] & (pu << 1)) | (Sq[5] & (pd << 1)) | (Sq[6] & pu) | (Sq[7] & pd))
                 : 0ull;
      if (row_lane) {
#pragma unroll
        for (int q = 0; q < 8; ++q) side[q * R + lane] = 0ull;
#pragma unroll
        for (int q = 0; q < 8; ++q) cwin[q * R + lane] = 0ull;
      }
      const int nq = enqueue_row_bits(queue, (multi | need) & live_window(3 * (steps - 1 - s) + 2, h, R, lane), lane);
      if (lane == 0) ctl[0] = (uint32_t)nq;
    }
    if (!NB8 && mask_wave) {
      const uint64_t E = ~(A | B | Wl);
      const uint64_t Eu = from_up(E), Ed = from_down(E);
      const uint64_t e_r = E >> 1, e_l = E << 1;  // cell to the right / left is empty
      fA = A & e_r;
      fB = B & e_l;
      const uint64_t bA = A & ~e_r, bB = B & ~e_l;  // forward cell blocked
      // blocked agents' empty side candidates: 0 FD-, 1 FD+, 2 L-, 3 L+
      const uint64_t oA0 = bA & (Eu >> 1), oA1 = bA & (Ed >> 1);
      const uint64_t oB0 = bB & (Eu << 1), oB1 = bB & (Ed << 1);
      const uint64_t o2 = (bA | bB) & Eu, o3 = (bA | bB) & Ed;
      const uint64_t o0 = oA0 | oB0, o1 = oA1 | oB1;
      const uint64_t multi = (o0 & (o1 | o2 | o3)) | (o1 & (o2 | o3)) | (o2 & o3);
      const uint64_t single = (o0 | o1 | o2 | o3) & ~multi;
      // side requests by requester row: 0 FD-A, 1 FD-B, 2 FD+A, 3 FD+B, 4 L-, 5 L+
      rq[0] = single & oA0;
      rq[1] = single & oB0;
      rq[2] = single & oA1;
      rq[3] = single & oB1;
      rq[4] = single & o2;
      rq[5] = single & o3;
      // possible requesters of each cell, by direction; two or more: contestable
      const uint64_t P[8] = {fA << 1,           fB >> 1,           from_down(oA0) << 1, from_up(oA1) << 1,
                             from_down(oB0) >> 1, from_up(oB1) >> 1, from_down(o2),       from_up(o3)};
      uint64_t ones = 0ull, twos = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        twos |= ones & P[q];
        ones |= P[q];
      }
      uint64_t need = 0ull;  // with recomputed tickets only the choices are queued
      if (kTicks) {
        const uint64_t pu = from_up(twos), pd = from_down(twos);
        need = (fA & (twos >> 1)) | (fB & (twos << 1)) | (oA0 & (pu >> 1)) | (oA1 & (pd >> 1)) |
               (oB0 & (pu << 1)) | (oB1 & (pd << 1)) | (o2 & pu) | (o3 & pd);
      }
      if (row_lane) {
#pragma unroll
        for (int q = 0; q < 6; ++q) side[q * R + lane] = 0ull;
#pragma unroll
        for (int q = 0; q < 8; ++q) cwin[q * R + lane] = 0ull;
      }
      const int nq = enqueue_row_bits(queue, (multi | need) & live_window(3 * (steps - 1 - s) + 2, h, R, lane), lane);
      if (lane == 0) ctl[0] = (uint32_t)nq;
    }
    __syncthreads();

    // ---- 2. draw: tickets for all queued agents, choices where needed -----
    const int nq = (int)ctl[0];
    if (nq > 0) {
      for (int qi = tid; qi < nq; qi += nthreads) {
        const uint32_t e = queue[qi];
        const int r = (int)(e & 63u), c = (int)((e >> 6) & 63u);
        // One round of LDS reads: rows r-1, r, r+1 (clamped; rows outside the
        // region count as wall) and the agent's id.
        const int ru = r > 0 ? r - 1 : r, rd = r + 1 < R ? r + 1 : r;
        const uint64_t a0 = H(s, 0, r), b0 = H(s, 1, r), w0m = wall_m[r];
        const uint64_t au = H(s, 0, ru), bu = H(s, 1, ru), wu = wall_m[ru];
        const uint64_t ad = H(s, 0, rd), bd = H(s, 1, rd), wd = wall_m[rd];
        const uint32_t id = ids[r * 64 + c];
        const uint64_t e0 = ~(a0 | b0 | w0m);
        const uint64_t eu = r > 0 ? ~(au | bu | wu) : 0ull;
        const uint64_t ed = r + 1 < R ? ~(ad | bd | wd) : 0ull;
        const bool is_a = (a0 >> c) & 1ull;
        const int d = is_a ? 1 : -1;
        const int cf = c + d;  // forward column; outside the region when -1 or 64
        const bool cf_in = cf >= 0 && cf < 64;
        const int cfc = cf_in ? cf : c;
        const unsigned bf = cf_in ? 1u : 0u;
        const bool fwd = bf & (unsigned)(e0 >> cfc);
        const unsigned avail = (bf & (unsigned)(eu >> cfc)) | ((bf & (unsigned)(ed >> cfc)) << 1) |
                               (((unsigned)(eu >> c) & 1u) << 2) | (((unsigned)(ed >> c) & 1u) << 3);
        const Words w = agent_words(id - 1u, t, S.key0, S.key1);
        if (kTicks) tick[r * 64 + c] = w.w0;
        if constexpr (NB8) {
          // backward column; candidates 4 B (r, cbc), 5 BD- (ru, cbc), 6 BD+ (rd, cbc)
          const int cb = c - d;
          const bool cb_in = cb >= 0 && cb < 64;
          const int cbc = cb_in ? cb : c;
          const unsigned bk = cb_in ? 1u : 0u;
          const unsigned avail7 = avail | ((bk & (unsigned)(e0 >> cbc)) << 4) | ((bk & (unsigned)(eu >> cbc)) << 5) |
                                  ((bk & (unsigned)(ed >> cbc)) << 6);
          if (!fwd && (avail7 & (avail7 - 1u)) != 0u) {  // two or more side candidates: a choice
            int j;
            if (MODE == 0) {
              j = lem_choose7(avail7, w.w1, w.w2);
            } else {
              const int gp = is_a ? 0 : 1;
              const float* tp = is_a ? tau_a : tau_b;
              // candidate rows: 0 = ru, 1 = rd, 2 = r
              const int rsel[7] = {0, 1, 0, 1, 2, 0, 1};
              const int cc[7] = {cfc, cfc, c, c, cbc, cbc, cbc};
              const int rows3[3] = {ru, rd, r};
              float tau[7];
#pragma unroll
              for (int k = 0; k < 7; ++k) tau[k] = tp[rows3[rsel[k]] * 64 + cc[k]];
              if (MODE == 1) {
                for (int u = 1; u <= s; ++u) {
                  const uint64_t hv[3] = {H(u, gp, ru), H(u, gp, rd), H(u, gp, r)};
#pragma unroll
                  for (int k = 0; k < 7; ++k) {
                    tau[k] = S.keep * tau[k];
                    if ((hv[rsel[k]] >> cc[k]) & 1ull) tau[k] = tau[k] + S.dtau;
                  }
                }
              } else {  // the LDS value is current through the cell's last deposit
                int owed[7];
#pragma unroll
                for (int k = 0; k < 7; ++k) owed[k] = s;
                for (int u = 0; u < s; ++u) {
                  const uint64_t nv[3] = {H(u + 1, gp, ru) & ~(H(u, 0, ru) | H(u, 1, ru)),
                                          H(u + 1, gp, rd) & ~(H(u, 0, rd) | H(u, 1, rd)),
                                          H(u + 1, gp, r) & ~(H(u, 0, r) | H(u, 1, r))};
#pragma unroll
                  for (int k = 0; k < 7; ++k)
                    if ((nv[rsel[k]] >> cc[k]) & 1ull) owed[k] = s - 1 - u;
                }
                for (int u = 0; u < s; ++u) {
#pragma unroll
                  for (int k = 0; k < 7; ++k)
                    if (u >= s - owed[k]) tau[k] = S.keep * tau[k];
                }
              }
#pragma unroll
              for (int k = 0; k < 7; ++k)
                if (!((avail7 >> k) & 1u)) tau[k] = 0.0f;
              const float eta[7] = {S.eta_diag, S.eta_diag, S.eta_lat,      S.eta_lat,
                                    S.eta_back, S.eta_back_diag, S.eta_back_diag};
              j = aco_choose7(avail7, tau, S.alpha, eta, w.w1, w.w2);
            }
            // candidate j -> move direction: A (+x) 2 3 6 7 1 4 5, B (-x) 4 5 6 7 0 2 3
            const int q = (int)(((is_a ? 0x5417632u : 0x3207654u) >> (4 * j)) & 0xFu);
            atomicOr((unsigned long long*)&side[q * R + r], 1ull << c);
          }
        } else if (!fwd && (avail & (avail - 1u)) != 0u) {  // two or more side candidates: a choice
          int req;
          if (MODE == 0) {
            req = lem_choose(avail, w.w1, w.w2);
          } else {
            const int gp = is_a ? 0 : 1;
            // candidates 0 FD- (ru, cfc), 1 FD+ (rd, cfc), 2 L- (ru, c), 3 L+ (rd, c):
            // their values at the launch start, advanced to step s with the
            // occupancy of their two rows after each step
            float tau[4];
            if (STREAM) {  // from HBM; a candidate outside the grid is never empty, index 0 stands in
              const float* tp = S.tau_in + (is_a ? 0 : plane);
              const int cr[4] = {ru, rd, ru, rd}, cc[4] = {cfc, cfc, c, c};
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const int gx = x0 + cc[j], gy = y0 + cr[j];
                const bool in = ((avail >> j) & 1u) && gx >= 0 && gx < S.W && gy >= 0 && gy < S.H;
                tau[j] = tp[in ? (size_t)gy * S.W + gx : 0];
              }
            } else {
              const float* tp = is_a ? tau_a : tau_b;
              tau[0] = tp[ru * 64 + cfc];
              tau[1] = tp[rd * 64 + cfc];
              tau[2] = tp[ru * 64 + c];
              tau[3] = tp[rd * 64 + c];
            }
            if (MODE == 1) {
              for (int u = 1; u <= s; ++u) {
                const uint64_t hu = H(u, gp, ru), hd = H(u, gp, rd);
                const unsigned ob = ((unsigned)(hu >> cfc) & 1u) | (((unsigned)(hd >> cfc) & 1u) << 1) |
                                    (((unsigned)(hu >> c) & 1u) << 2) | (((unsigned)(hd >> c) & 1u) << 3);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  tau[j] = S.keep * tau[j];
                  if ((ob >> j) & 1u) tau[j] = tau[j] + S.dtau;
                }
              }
            } else {  // the LDS value is current through the cell's last deposit
              int owed[4] = {s, s, s, s};
              for (int u = 0; u < s; ++u) {
                const uint64_t nu = H(u + 1, gp, ru) & ~(H(u, 0, ru) | H(u, 1, ru));
                const uint64_t nd = H(u + 1, gp, rd) & ~(H(u, 0, rd) | H(u, 1, rd));
                const unsigned ob = ((unsigned)(nu >> cfc) & 1u) | (((unsigned)(nd >> cfc) & 1u) << 1) |
                                    (((unsigned)(nu >> c) & 1u) << 2) | (((unsigned)(nd >> c) & 1u) << 3);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                  if ((ob >> j) & 1u) owed[j] = s - 1 - u;
              }
              for (int u = 0; u < s; ++u) {  // the owed evaporations are the last ones
#pragma unroll
                for (int j = 0; j < 4; ++j)
                  if (u >= s - owed[j]) tau[j] = S.keep * tau[j];
              }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (!((avail >> j) & 1u)) tau[j] = 0.0f;
            req = aco_choose(avail, tau, S.alpha, S.eta_diag, S.eta_lat, w.w1, w.w2);
          }
          const int which = req == kReqFDm ? (is_a ? 0 : 1)
                                           : (req == kReqFDp ? (is_a ? 2 : 3) : (req == kReqLm ? 4 : 5));
          atomicOr((unsigned long long*)&side[which * R + r], 1ull << c);
        }
      }
      __syncthreads();
    }

    // ---- 3. gather: requesters of every cell, by direction -----------------
    if (NB8 && mask_wave) {
      uint64_t own[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) own[q] = rq[q] | ((nq > 0 && row_lane) ? side[q * R + lane] : 0ull);
      own[0] |= fA;  // forward moves: A by (+1, 0), B by (-1, 0)
      own[1] |= fB;
      Wt[0] = own[0] << 1;
      Wt[1] = own[1] >> 1;
      Wt[2] = from_down(own[2]) << 1;
      Wt[3] = from_up(own[3]) << 1;
      Wt[4] = from_down(own[4]) >> 1;
      Wt[5] = from_up(own[5]) >> 1;
      Wt[6] = from_down(own[6]);
      Wt[7] = from_up(own[7]);
      uint64_t ones = 0ull, twos = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        twos |= ones & Wt[q];
        ones |= Wt[q];
      }
      if (row_lane) {
#pragma unroll
        for (int q = 0; q < 8; ++q) reqm[q * R + lane] = Wt[q];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) Wt[q] &= ~twos;  // uncontested winners
      const int na = enqueue_row_bits(queue, ones & live_window(3 * (steps - 1 - s) + 1, h, R, lane), lane);
      if (lane == 0) ctl[1] = (uint32_t)na;
    }
    if (!NB8 && mask_wave) {
      uint64_t own[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) own[q] = rq[q] | ((nq > 0 && row_lane) ? side[q * R + lane] : 0ull);
      Wt[0] = fA << 1;                 // A from the left (F)
      Wt[1] = fB >> 1;                 // B from the right (F)
      Wt[2] = from_down(own[0]) << 1;  // A from below-left (FD-)
      Wt[3] = from_up(own[2]) << 1;    // A from above-left (FD+)
      Wt[4] = from_down(own[1]) >> 1;  // B from below-right (FD-)
      Wt[5] = from_up(own[3]) >> 1;    // B from above-right (FD+)
      Wt[6] = from_down(own[4]);       // from below (L-)
      Wt[7] = from_up(own[5]);         // from above (L+)
      uint64_t ones = 0ull, twos = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        twos |= ones & Wt[q];
        ones |= Wt[q];
      }
      if (row_lane) {
#pragma unroll
        for (int q = 0; q < 8; ++q) reqm[q * R + lane] = Wt[q];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) Wt[q] &= ~twos;  // uncontested winners
      const int na = enqueue_row_bits(queue, ones & live_window(3 * (steps - 1 - s) + 1, h, R, lane), lane);
      if (lane == 0) ctl[1] = (uint32_t)na;
    }
    __syncthreads();

    // ---- 4. resolve contests; every winner's id moves to its target --------
    const int na = (int)ctl[1];
    if (na > 0) {
      for (int qi = tid; qi < na; qi += nthreads) {
        const uint32_t e = queue[qi];
        const int r = (int)(e & 63u), c = (int)((e >> 6) & 63u);
        uint32_t dirs = 0u;
#pragma unroll
        for (int q = 0; q < 8; ++q) dirs |= (uint32_t)((reqm[q * R + r] >> c) & 1ull) << q;
        int best = __ffs(dirs) - 1;
        uint32_t src_id;
        if (dirs & (dirs - 1u)) {  // contested: lowest (ticket, agent number)
          // every direction's ticket and id in one round (clamped addresses;
          // directions without a requester are ignored)
          uint32_t tk[8], kk[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            int sr = r + dir_dr(q), sc = c + dir_dc(q);
            sr = sr < 0 ? 0 : (sr >= R ? R - 1 : sr);
            sc = sc < 0 ? 0 : (sc > 63 ? 63 : sc);
            kk[q] = ids[sr * 64 + sc];
            if (kTicks) tk[q] = tick[sr * 64 + sc];
          }
          if (!kTicks) {  // the contenders' tickets, drawn again (independent chains)
#pragma unroll
            for (int q = 0; q < 8; ++q)
              tk[q] = ((dirs >> q) & 1u) ? agent_words(kk[q] - 1u, t, S.key0, S.key1).w0 : 0xFFFFFFFFu;
          }
          uint32_t best_t = 0xFFFFFFFFu;
          src_id = 0xFFFFFFFFu;
          best = -1;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            if (((dirs >> q) & 1u) &&
                (best < 0 || tk[q] < best_t || (tk[q] == best_t && kk[q] < src_id))) {
              best = q;
              best_t = tk[q];
              src_id = kk[q];
            }
          }
          atomicOr((unsigned long long*)&cwin[best * R + r], 1ull << c);
        } else {
          src_id = ids[(r + dir_dr(best)) * 64 + c + dir_dc(best)];
        }
        ids[r * 64 + c] = src_id;
        if (MODE == 2) {  // the tour grows by the move's length; eq. 5's deposit on the entered cell
          const int sr = r + dir_dr(best), sc = c + dir_dc(best);
          const bool diagonal = best >= 2 && best <= 5;
          const float len = tlen[sr * 64 + sc] + (diagonal ? S.step_diag : 1.0f);
          tlen[r * 64 + c] = len;
          const bool ga = NB8 ? (bool)((H(s, 0, sr) >> sc) & 1ull)
                              : (best == 0 || best == 2 || best == 3 || (best >= 6 && ((H(s, 0, sr) >> sc) & 1ull)));
          const int gp = ga ? 0 : 1;
          float* tp = ga ? tau_a : tau_b;
          int owed = s + 1;  // evaporations since the cell's last deposit, this step's included
          for (int u = 0; u < s; ++u) {
            const uint64_t entered = H(u + 1, gp, r) & ~(H(u, 0, r) | H(u, 1, r));
            if ((entered >> c) & 1ull) owed = s - u;
          }
          float v = tp[r * 64 + c];
          for (int u = 0; u <= s; ++u)
            if (u > s - owed) v = S.keep * v;
          tp[r * 64 + c] = v + S.dtau / len;
        }
      }
      __syncthreads();
    }

    // ---- 5. commit: next occupancy, recorded in the history ---------------
    if (NB8 && mask_wave) {
      if (na > 0 && row_lane) {
#pragma unroll
        for (int q = 0; q < 8; ++q) Wt[q] |= cwin[q * R + lane];
      }
      const uint64_t Au = from_up(A), Ad = from_down(A);
      const uint64_t in_all = Wt[0] | Wt[1] | Wt[2] | Wt[3] | Wt[4] | Wt[5] | Wt[6] | Wt[7];
      const uint64_t in_a = (Wt[0] & (A << 1)) | (Wt[1] & (A >> 1)) | (Wt[2] & (Ad << 1)) | (Wt[3] & (Au << 1)) |
                            (Wt[4] & (Ad >> 1)) | (Wt[5] & (Au >> 1)) | (Wt[6] & Ad) | (Wt[7] & Au);
      const uint64_t out = (Wt[0] >> 1) | (Wt[1] << 1) | (from_up(Wt[2]) >> 1) | (from_down(Wt[3]) >> 1) |
                           (from_up(Wt[4]) << 1) | (from_down(Wt[5]) << 1) | from_up(Wt[6]) | from_down(Wt[7]);
      A = (A & ~out) | in_a;
      B = (B & ~out) | (in_all & ~in_a);
      moved_in = in_all;
      if (row_lane) {
        H(s + 1, 0, lane) = A;
        H(s + 1, 1, lane) = B;
      }
    }
    if (!NB8 && mask_wave) {
      if (na > 0 && row_lane) {
#pragma unroll
        for (int q = 0; q < 8; ++q) Wt[q] |= cwin[q * R + lane];
      }
      const uint64_t in_a = Wt[0] | Wt[2] | Wt[3] | (Wt[6] & from_down(A)) | (Wt[7] & from_up(A));
      const uint64_t in_b = Wt[1] | Wt[4] | Wt[5] | (Wt[6] & from_down(B)) | (Wt[7] & from_up(B));
      const uint64_t out = (Wt[0] >> 1) | (Wt[1] << 1) | (from_up(Wt[2]) >> 1) | (from_down(Wt[3]) >> 1) |
                           (from_up(Wt[4]) << 1) | (from_down(Wt[5]) << 1) | from_up(Wt[6]) | from_down(Wt[7]);
      A = (A & ~out) | in_a;
      B = (B & ~out) | in_b;
      moved_in = in_a | in_b;
      if (row_lane) {
        H(s + 1, 0, lane) = A;
        H(s + 1, 1, lane) = B;
      }
    }
  }
  if (mask_wave && row_lane) moved_m[lane] = moved_in;
  __syncthreads();

  if (!STREAM) __builtin_amdgcn_s_setprio(0);

  // ---- write the interior back; pheromone applied step by step ------------
  // Interior rows are dealt round-robin to the waves, kWriteRows at a time;
  // every LDS read of a block is issued before its arithmetic, and each
  // cell's occupancy history is packed into bit vectors (bit u: occupied
  // after step u).
  constexpr int kWriteRows = 3;
  uint32_t cnt[kTileStatFields] = {0, 0, 0, 0, 0};
  const int c = lane;
  const int gx = x0 + c;
  for (int r0 = h + wave; r0 < R - h; r0 += nwaves * kWriteRows) {
    uint64_t ra[kWriteRows], rb[kWriteRows], rw[kWriteRows], rm[kWriteRows];
    uint32_t idv[kWriteRows], hist_a[kWriteRows], hist_b[kWriteRows];
    float va[kWriteRows], vb[kWriteRows], tl[kWriteRows];
    int rr[kWriteRows];
#pragma unroll
    for (int j = 0; j < kWriteRows; ++j) {
      const int r = r0 + j * nwaves;
      rr[j] = r < R - h ? r : R - h - 1;  // rows past the interior repeat the last one, unused
      ra[j] = H(run_steps, 0, rr[j]);
      rb[j] = H(run_steps, 1, rr[j]);
      rw[j] = wall_m[rr[j]];
      rm[j] = moved_m[rr[j]];
      idv[j] = ids[rr[j] * 64 + c];
      hist_a[j] = 0u;
      hist_b[j] = 0u;
      if (MODE == 2) {
        va[j] = tau_a[rr[j] * 64 + c];
        vb[j] = tau_b[rr[j] * 64 + c];
        tl[j] = tlen[rr[j] * 64 + c];
      }
      if (MODE == 1) {
        if (STREAM) {  // from HBM (interior cells only; index 0 stands in for the rest)
          const int gy = y0 + rr[j];
          const bool in = c >= h && c < h + S.IX && gx < S.W && gy < S.H;
          const size_t gi = in ? (size_t)gy * S.W + gx : 0;
          va[j] = S.tau_in[gi];
          vb[j] = S.tau_in[plane + gi];
        } else {
          va[j] = tau_a[rr[j] * 64 + c];
          vb[j] = tau_b[rr[j] * 64 + c];
        }
      }
    }
    if (MODE == 1) {
      for (int u = 1; u <= run_steps; ++u) {
#pragma unroll
        for (int j = 0; j < kWriteRows; ++j) {
          hist_a[j] |= (uint32_t)((H(u, 0, rr[j]) >> c) & 1ull) << u;
          hist_b[j] |= (uint32_t)((H(u, 1, rr[j]) >> c) & 1ull) << u;
        }
      }
    }
    if (MODE == 2) {  // bit u: an agent of the group entered the cell in step u
      for (int u = 0; u < run_steps; ++u) {
#pragma unroll
        for (int j = 0; j < kWriteRows; ++j) {
          const uint64_t before = H(u, 0, rr[j]) | H(u, 1, rr[j]);
          hist_a[j] |= (uint32_t)(((H(u + 1, 0, rr[j]) & ~before) >> c) & 1ull) << u;
          hist_b[j] |= (uint32_t)(((H(u + 1, 1, rr[j]) & ~before) >> c) & 1ull) << u;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kWriteRows; ++j) {
      const int r = r0 + j * nwaves;
      if (r >= R - h) break;  // wave-uniform
      const int gy = y0 + r;
      const bool interior = c >= h && c < h + S.IX && gx < S.W && gy < S.H;
      const int g = !interior ? kEmpty
                              : ((ra[j] & lane_bit) ? kGroupA
                                                    : ((rb[j] & lane_bit) ? kGroupB
                                                                          : ((rw[j] & lane_bit) ? kWall : kEmpty)));
      if (interior) {
        const size_t gi = (size_t)gy * S.W + gx;
        S.code_out[gi] = (uint8_t)g;
        S.id_out[gi] = (g == kGroupA || g == kGroupB) ? idv[j] : 0u;
        if (MODE == 1) {
          float a = va[j], b = vb[j];
          for (int u = 1; u <= steps; ++u) {
            a = S.keep * a;
            b = S.keep * b;
            if ((hist_a[j] >> u) & 1u) a = a + S.dtau;
            if ((hist_b[j] >> u) & 1u) b = b + S.dtau;
          }
          S.tau_out[gi] = a;
          S.tau_out[plane + gi] = b;
        }
        if (MODE == 2) {  // evaporations owed since each plane's last deposit
          const int oa = hist_a[j] ? steps - 1 - (31 - __clz((int)hist_a[j])) : steps;
          const int ob = hist_b[j] ? steps - 1 - (31 - __clz((int)hist_b[j])) : steps;
          float a = va[j], b = vb[j];
          for (int u = 0; u < steps; ++u) {  // the owed evaporations are the last ones
            if (u >= steps - oa) a = S.keep * a;
            if (u >= steps - ob) b = S.keep * b;
          }
          S.tau_out[gi] = a;
          S.tau_out[plane + gi] = b;
          if (g == kGroupA || g == kGroupB) S.tour_out[idv[j] - 1u] = tl[j];
        }
      }
      if (last) {
        const bool moved = interior && steps > 0 && ((rm[j] >> c) & 1ull);
        cnt[0] += __popcll(__ballot(g == kGroupA));
        cnt[1] += __popcll(__ballot(g == kGroupB));
        cnt[2] += __popcll(__ballot(g == kGroupA && gx >= S.W - S.cross_b));
        cnt[3] += __popcll(__ballot(g == kGroupB && gx < S.cross_a));
        cnt[4] += __popcll(__ballot(moved));
      }
    }
  }
  if (last) {
    if (lane == 0) {
#pragma unroll
      for (int f = 0; f < kTileStatFields; ++f) atomicAdd(&ctl[8 + f], cnt[f]);
    }
    __syncthreads();
    if (tid < kTileStatFields) S.tile_stats[(size_t)tile_index * kTileStatFields + tid] = ctl[8 + tid];
  }
  return !empty_region;
}

}  // namespace pedsim
