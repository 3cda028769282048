// LDS-resident tile engine: advance one tile of a scenario by k steps of the
// bi-directional pedestrian update (Sec. III, Sec. IV.b-d) inside one
// workgroup.
//
// The workgroup stages a region of RX = 64*NW columns x R rows around its
// tile (the tile interior plus a halo of 3k cells on every side) in LDS, runs
// k steps on the region, and writes the interior back. One step depends on
// cells at most 3 away (a cell's new content depends on the resolution at its
// target, which depends on the requests of the target's neighbours, which
// depend on their neighbours), so after k steps the cells at least 3k from
// the region border are exact; the rest of the region is scratch. Outside the
// region counts as wall.
//
// Occupancy is kept as 64-bit masks, one bit per cell and one word per 64
// cells of a row, built with wave64 ballots. The mask passes (1, 3, 5) give
// each lane one row-word, so one wave64 instruction advances 64 x 64 cells;
// the cell passes (staging, 6, write-back) give each wave one word and each
// lane one cell of it:
//   1. forward   an agent whose forward cell is empty requests it; agents
//                whose forward cell is blocked but have an empty side
//                candidate are appended to an LDS queue;
//   2. draw      each queued agent draws its Philox words and picks a side
//                candidate by the LEM (eq. 1) or ACO (eq. 2) rule; the pick
//                is or-ed into a request mask;
//   3. gather    for every empty cell, eight requester masks (one per
//                direction a requester can come from); cells with exactly one
//                requester get it as winner, contested cells are queued with
//                the set of directions they are requested from;
//   4. resolve   contested cells keep the requester with the lowest
//                (Philox word 0, agent number) (Sec. IV.d);
//   5. commit    new occupancy masks: winners leave their cells and enter
//                their targets;
//   6. cells     ids follow their agents; both pheromone planes evaporate and
//                receive the deposit (eq. 3 then eq. 4, ACO only).
#pragma once

#include "rules.hpp"

namespace pedsim {

// Masks kept per row-word (index into the mask block).
enum : int {
  kMWall = 0,   // walls and cells outside the grid
  kMOcc = 1,    // 2 sets x (A agents, B agents, empty): current and next step
  kMIn = 7,     // cells that received an agent in the last step
  kMReq = 8,    // 8 request masks
  kMWin = 16,   // 8 winner masks
  kMaskCount = 24
};

// Request masks (indexed by the requester's row), offsets from kMReq.
enum : int { kRqFA = 0, kRqFB = 1, kRqFDmA = 2, kRqFDmB = 3, kRqFDpA = 4, kRqFDpB = 5, kRqLm = 6, kRqLp = 7 };

// Winner directions (indexed by the target's row): where the winner comes
// from, as (column offset, row offset) of its old cell.
//   0 A from the left (F)          1 B from the right (F)
//   2 A from below-left (FD-)      3 A from above-left (FD+)
//   4 B from below-right (FD-)     5 B from above-right (FD+)
//   6 from below (L-)              7 from above (L+)
__host__ __device__ constexpr int dir_dc(int i) {
  return (i == 0 || i == 2 || i == 3) ? -1 : ((i == 1 || i == 4 || i == 5) ? 1 : 0);
}
__host__ __device__ constexpr int dir_dr(int i) {
  return (i == 2 || i == 4 || i == 6) ? 1 : ((i == 3 || i == 5 || i == 7) ? -1 : 0);
}

// Counters in the control block.
enum : int { kCtlQueue = 0, kCtlConflicts = 1, kCtlWords = 16 };

// Per-tile counters written at the end of a call's last launch.
constexpr int kTileStatFields = 5;  // agents A, agents B, crossed A, crossed B, moved

// One scenario as the engine sees it.
struct Scenario {
  const uint8_t* code_in;
  const uint32_t* id_in;
  const float* tau_in;  // 2 planes (A then B) or nullptr for LEM
  uint8_t* code_out;
  uint32_t* id_out;
  float* tau_out;
  const float* tour_in;  // tour variant: tour length per agent (index = agent number), else nullptr
  float* tour_out;
  uint32_t* tile_stats;  // kTileStatFields per tile
  int W, H;
  int tiles_x, tiles_y;  // tile grid
  int IX, IY;            // tile interior
  int halo;              // 3 * steps per launch
  uint32_t key0, key1;
  float keep, dtau, eta_diag, eta_lat;
  float step_diag;  // tour variant: length of a diagonal move, fl(sqrt 2)
  float eta_back, eta_back_diag;  // eight neighbours: eta^beta of B (D2 = 9) and BD (D2 = 10)
  int neighbours;                 // 5 (no backward cells) or 8
  int alpha;
  int cross_a, cross_b;
  // Row-lane launches of one scenario: the order in which each XCD's
  // workgroups take its tiles. Three rotations of [16 counters][order_cap
  // entries]: a launch takes rotation order_rot (if order_valid; else the
  // tiles in row-major order), writes the next one (per XCD, the tiles that
  // had agents from the front, the others from the back) and clears the
  // counters of the one after. nullptr: row-major order, nothing written.
  uint32_t* order;
  int order_cap, order_rot, order_valid;
};

// LDS layout of a region of R rows x 64*NW columns.
template <int NW>
struct Layout {
  int R;
  bool aco;
  __host__ __device__ static constexpr int RX() { return 64 * NW; }
  __host__ __device__ size_t masks() const { return 0; }
  __host__ __device__ size_t ids() const { return (size_t)kMaskCount * R * NW * 8; }
  __host__ __device__ size_t tau() const { return ids() + (size_t)R * RX() * 4; }
  __host__ __device__ size_t queue() const { return tau() + (aco ? (size_t)2 * R * RX() * 4 : 0); }
  __host__ __device__ size_t ctl() const { return queue() + (size_t)R * RX() * 4; }
  __host__ __device__ size_t bytes() const { return ctl() + kCtlWords * 4; }
};

template <int NW>
struct Tile {
  uint64_t* mask;  // [kMaskCount][R][NW]
  uint32_t* id;    // [R][RX]
  float* tau_a;    // [R][RX]
  float* tau_b;
  uint32_t* queue;
  uint32_t* ctl;
  int R;
  int occ;  // mask index of the current occupancy set (A, B, empty)

  __device__ __forceinline__ uint64_t* m(int which, int r) const { return mask + ((size_t)which * R + r) * NW; }
  // Word w of row r of mask `which`; 0 outside the region.
  __device__ __forceinline__ uint64_t word(int which, int r, int w) const {
    return (r < 0 || r >= R || w < 0 || w >= NW) ? 0ull : m(which, r)[w];
  }
  // Word w of the row shifted so that bit c holds cell c+1 (cell to the right).
  __device__ __forceinline__ uint64_t right(int which, int r, int w) const {
    return (word(which, r, w) >> 1) | (word(which, r, w + 1) << 63);
  }
  // Word w of the row shifted so that bit c holds cell c-1 (cell to the left).
  __device__ __forceinline__ uint64_t left(int which, int r, int w) const {
    return (word(which, r, w) << 1) | (word(which, r, w - 1) >> 63);
  }
  __device__ __forceinline__ bool bit(int which, int r, int c) const {
    if (r < 0 || r >= R || c < 0 || c >= 64 * NW) return false;
    return (m(which, r)[c >> 6] >> (c & 63)) & 1ull;
  }
  __device__ __forceinline__ void or_bit(int which, int r, int c) const {
    atomicOr((unsigned long long*)(m(which, r) + (c >> 6)), 1ull << (c & 63));
  }
  // Append the cells of row r whose bits are set in `bits` (columns c0 + bit)
  // to queue `counter`; with `q` (the eight requester masks of the word) each
  // entry also records the directions its cell is requested from.
  __device__ __forceinline__ void append_bits(int counter, uint64_t bits, uint32_t r, int c0,
                                              const uint64_t* q) const {
    if (bits == 0ull) return;
    uint32_t pos = atomicAdd(&ctl[counter], (uint32_t)__popcll(bits));
    while (bits) {
      const int b = __ffsll((unsigned long long)bits) - 1;
      bits &= bits - 1;
      uint32_t dirs = 0;
      if (q) {
#pragma unroll
        for (int k = 0; k < 8; ++k) dirs |= (uint32_t)((q[k] >> b) & 1ull) << k;
      }
      queue[pos++] = r | ((uint32_t)(c0 + b) << 10) | (dirs << 18);
    }
  }
};

template <int NW>
__device__ __forceinline__ Tile<NW> tile_view(uint8_t* smem, const Layout<NW>& L) {
  Tile<NW> T;
  T.mask = (uint64_t*)(smem + L.masks());
  T.id = (uint32_t*)(smem + L.ids());
  T.tau_a = (float*)(smem + L.tau());
  T.tau_b = T.tau_a + (size_t)L.R * Layout<NW>::RX();
  T.queue = (uint32_t*)(smem + L.queue());
  T.ctl = (uint32_t*)(smem + L.ctl());
  T.R = L.R;
  T.occ = kMOcc;
  return T;
}

// Advance the tile (tx, ty) of scenario S by `steps` steps starting at step t0.
// Must be called by every thread of the workgroup (blockDim.x a multiple of
// 64). last: write the tile's counters.
template <int NW, int MODE>
__device__ void advance_tile(const Scenario& S, uint8_t* smem, int R, int tx, int ty, int tile_index, uint64_t t0,
                             int steps, bool last) {
  constexpr int RX = 64 * NW;
  constexpr int kStage = 4;  // words staged per wave batch, all loads issued first
  const Layout<NW> L{R, MODE == 1};
  Tile<NW> T = tile_view<NW>(smem, L);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: row loops and addresses stay scalar
  const int nthreads = blockDim.x;
  const int nwaves = blockDim.x >> 6;
  const int nwords = R * NW;
  const int h = S.halo;
  const int x0 = tx * S.IX - h;  // region origin in grid coordinates
  const int y0 = ty * S.IY - h;
  const size_t plane = (size_t)S.W * (size_t)S.H;
  const uint64_t lane_bit = 1ull << lane;

  // ---- stage the region ------------------------------------------------------
  for (int wd0 = wave * kStage; wd0 < nwords; wd0 += nwaves * kStage) {
    int g[kStage];
    uint32_t idv[kStage];
    float ta[kStage], tb[kStage];
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
      const int wd = wd0 + j;
      const int r = wd / NW, c = (wd % NW) * 64 + lane;
      const int gx = x0 + c, gy = y0 + r;
      const bool in = wd < nwords && gx >= 0 && gx < S.W && gy >= 0 && gy < S.H;
      const size_t gi = in ? (size_t)gy * S.W + gx : 0;
      g[j] = in ? S.code_in[gi] : kWall;
      idv[j] = in ? S.id_in[gi] : 0u;
      if (MODE == 1) {
        ta[j] = in ? S.tau_in[gi] : 0.0f;
        tb[j] = in ? S.tau_in[plane + gi] : 0.0f;
      }
    }
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
      const int wd = wd0 + j;
      if (wd >= nwords) break;
      const int r = wd / NW, w = wd % NW;
      const uint64_t ba = __ballot(g[j] == kGroupA), bb = __ballot(g[j] == kGroupB);
      const uint64_t bw = __ballot(g[j] == kWall);
      if (lane < 5) {
        const uint64_t v = lane == 0 ? ba : (lane == 1 ? bb : (lane == 2 ? ~(ba | bb | bw) : (lane == 3 ? bw : 0ull)));
        T.m(lane < 3 ? kMOcc + lane : (lane == 3 ? kMWall : kMIn), r)[w] = v;
      }
      const int i = r * RX + w * 64 + lane;
      T.id[i] = idv[j];
      if (MODE == 1) {
        T.tau_a[i] = ta[j];
        T.tau_b[i] = tb[j];
      }
    }
  }
  if (tid < kCtlWords) T.ctl[tid] = 0u;
  __syncthreads();

  for (int s = 0; s < steps; ++s) {
    const uint64_t t = t0 + (uint64_t)s;
    const int mA = T.occ, mB = T.occ + 1, mE = T.occ + 2;
    const int nxt = T.occ == kMOcc ? kMOcc + 3 : kMOcc;

    // ---- 1. forward requests; queue blocked agents with an empty side cell ----
    for (int wd = tid; wd < nwords; wd += nthreads) {  // one lane per row-word
      const int r = wd / NW, w = wd % NW;
      const uint64_t a = T.word(mA, r, w), b = T.word(mB, r, w);
      const uint64_t e_r = T.right(mE, r, w), e_l = T.left(mE, r, w);
      const uint64_t eu = T.word(mE, r - 1, w), ed = T.word(mE, r + 1, w);
      const uint64_t side_a = T.right(mE, r - 1, w) | T.right(mE, r + 1, w) | eu | ed;
      const uint64_t side_b = T.left(mE, r - 1, w) | T.left(mE, r + 1, w) | eu | ed;
      const uint64_t act = (a & ~e_r & side_a) | (b & ~e_l & side_b);
      uint64_t* req = T.m(kMReq, r) + w;
      const size_t stride = (size_t)R * NW;
      req[kRqFA * stride] = a & e_r;
      req[kRqFB * stride] = b & e_l;
#pragma unroll
      for (int k = kRqFDmA; k <= kRqLp; ++k) req[k * stride] = 0ull;
      T.append_bits(kCtlQueue, act, (uint32_t)r, w * 64, nullptr);
    }
    __syncthreads();

    // ---- 2. queued agents pick a side candidate --------------------------------
    {
      const int nq = (int)T.ctl[kCtlQueue];
      for (int q = tid; q < nq; q += blockDim.x) {
        const uint32_t e = T.queue[q];
        const int r = (int)(e & 1023u), c = (int)((e >> 10) & 255u);
        const bool is_a = T.bit(mA, r, c);
        const int d = is_a ? 1 : -1;
        const unsigned avail = (unsigned)T.bit(mE, r - 1, c + d) | ((unsigned)T.bit(mE, r + 1, c + d) << 1) |
                               ((unsigned)T.bit(mE, r - 1, c) << 2) | ((unsigned)T.bit(mE, r + 1, c) << 3);
        const Words wds = agent_words(T.id[r * RX + c] - 1u, t, S.key0, S.key1);
        int req;
        if (MODE == 0) {
          req = lem_choose(avail, wds.w1, wds.w2);
        } else {
          const float* tp = is_a ? T.tau_a : T.tau_b;
          float tau[4];
          tau[0] = (avail & 1u) ? tp[(r - 1) * RX + c + d] : 0.0f;
          tau[1] = (avail & 2u) ? tp[(r + 1) * RX + c + d] : 0.0f;
          tau[2] = (avail & 4u) ? tp[(r - 1) * RX + c] : 0.0f;
          tau[3] = (avail & 8u) ? tp[(r + 1) * RX + c] : 0.0f;
          req = aco_choose(avail, tau, S.alpha, S.eta_diag, S.eta_lat, wds.w1, wds.w2);
        }
        int which = -1;
        if (req == kReqFDm) which = is_a ? kRqFDmA : kRqFDmB;
        if (req == kReqFDp) which = is_a ? kRqFDpA : kRqFDpB;
        if (req == kReqLm) which = kRqLm;
        if (req == kReqLp) which = kRqLp;
        if (which >= 0) T.or_bit(kMReq + which, r, c);
      }
    }
    __syncthreads();

    // ---- 3. requesters per empty cell: single ones win, contested are queued ---
    if (tid == 0) T.ctl[kCtlQueue] = 0u;  // the agent queue has been consumed
    for (int wd = tid; wd < nwords; wd += nthreads) {  // one lane per row-word
      const int r = wd / NW, w = wd % NW;
      uint64_t q[8];
      q[0] = T.left(kMReq + kRqFA, r, w);
      q[1] = T.right(kMReq + kRqFB, r, w);
      q[2] = T.left(kMReq + kRqFDmA, r + 1, w);
      q[3] = T.left(kMReq + kRqFDpA, r - 1, w);
      q[4] = T.right(kMReq + kRqFDmB, r + 1, w);
      q[5] = T.right(kMReq + kRqFDpB, r - 1, w);
      q[6] = T.word(kMReq + kRqLm, r + 1, w);
      q[7] = T.word(kMReq + kRqLp, r - 1, w);
      uint64_t ones = 0ull, twos = 0ull;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        twos |= ones & q[k];
        ones |= q[k];
      }
      uint64_t* win = T.m(kMWin, r) + w;
      const size_t stride = (size_t)R * NW;
#pragma unroll
      for (int k = 0; k < 8; ++k) win[k * stride] = q[k] & ~twos;
      T.append_bits(kCtlConflicts, twos, (uint32_t)r, w * 64, q);
    }
    __syncthreads();

    // ---- 4. contested cells: lowest (word 0, agent number) wins ----------------
    {
      const int nc = (int)T.ctl[kCtlConflicts];
      for (int q = tid; q < nc; q += blockDim.x) {
        const uint32_t e = T.queue[q];
        const int r = (int)(e & 1023u), c = (int)((e >> 10) & 255u);
        uint32_t dirs = e >> 18;
        uint32_t best_t = 0xFFFFFFFFu, best_k = 0xFFFFFFFFu;
        int best = -1;
        while (dirs) {
          const int k = __ffs(dirs) - 1;
          dirs &= dirs - 1;
          const uint32_t agent = T.id[(r + dir_dr(k)) * RX + c + dir_dc(k)] - 1u;
          const uint32_t tk = agent_words(agent, t, S.key0, S.key1).w0;
          if (best < 0 || tk < best_t || (tk == best_t && agent < best_k)) {
            best = k;
            best_t = tk;
            best_k = agent;
          }
        }
        T.or_bit(kMWin + best, r, c);
      }
    }
    __syncthreads();

    // ---- 5. next occupancy: winners leave their cells and enter their targets --
    if (tid == 0) T.ctl[kCtlConflicts] = 0u;  // the conflict queue has been consumed
    for (int wd = tid; wd < nwords; wd += nthreads) {  // one lane per row-word
      const int r = wd / NW, w = wd % NW;
      uint64_t win[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) win[k] = T.word(kMWin + k, r, w);
      const uint64_t in_a = win[0] | win[2] | win[3] | (win[6] & T.word(mA, r + 1, w)) |
                            (win[7] & T.word(mA, r - 1, w));
      const uint64_t in_b = win[1] | win[4] | win[5] | (win[6] & T.word(mB, r + 1, w)) |
                            (win[7] & T.word(mB, r - 1, w));
      const uint64_t out = T.right(kMWin + 0, r, w) | T.left(kMWin + 1, r, w) | T.right(kMWin + 2, r - 1, w) |
                           T.right(kMWin + 3, r + 1, w) | T.left(kMWin + 4, r - 1, w) |
                           T.left(kMWin + 5, r + 1, w) | T.word(kMWin + 6, r - 1, w) | T.word(kMWin + 7, r + 1, w);
      const uint64_t na = (T.word(mA, r, w) & ~out) | in_a;
      const uint64_t nb = (T.word(mB, r, w) & ~out) | in_b;
      T.m(nxt, r)[w] = na;
      T.m(nxt + 1, r)[w] = nb;
      T.m(nxt + 2, r)[w] = ~(T.word(kMWall, r, w) | na | nb);
      T.m(kMIn, r)[w] = in_a | in_b;
    }
    __syncthreads();

    // ---- 6. ids follow their agents; pheromone evaporates and is deposited -----
    for (int wd = wave; wd < nwords; wd += nwaves) {  // one wave per word, one lane per cell
      const int r = wd / NW, w = wd % NW;
      const int i = r * RX + w * 64 + lane;
      const uint64_t in_w = T.word(kMIn, r, w);
      if (in_w & lane_bit) {
        int k = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (T.word(kMWin + j, r, w) & lane_bit) k = j;
        T.id[i] = T.id[i + dir_dr(k) * RX + dir_dc(k)];
      }
      if (MODE == 1) {
        const bool ga = (T.word(nxt, r, w) & lane_bit) != 0ull;
        const bool gb = (T.word(nxt + 1, r, w) & lane_bit) != 0ull;
        float va = S.keep * T.tau_a[i];
        float vb = S.keep * T.tau_b[i];
        if (ga) va = va + S.dtau;
        if (gb) vb = vb + S.dtau;
        T.tau_a[i] = va;
        T.tau_b[i] = vb;
      }
    }
    __syncthreads();
    T.occ = nxt;
  }

  // ---- write the interior back; count agents, crossings and moves ------------
  const int mA = T.occ, mB = T.occ + 1;
  uint32_t cnt[kTileStatFields] = {0, 0, 0, 0, 0};
  for (int wd = wave; wd < nwords; wd += nwaves) {
    const int r = wd / NW, w = wd % NW;
    const int c = w * 64 + lane;
    const int gx = x0 + c, gy = y0 + r;
    const bool interior = r >= h && r < h + S.IY && c >= h && c < h + S.IX && gx < S.W && gy < S.H;
    const uint64_t wa = T.word(mA, r, w), wb = T.word(mB, r, w), ww = T.word(kMWall, r, w);
    const uint64_t win_mask = T.word(kMIn, r, w);
    const int g = !interior ? kEmpty
                            : ((wa & lane_bit) ? kGroupA
                                               : ((wb & lane_bit) ? kGroupB : ((ww & lane_bit) ? kWall : kEmpty)));
    if (interior) {
      const int i = r * RX + c;
      const size_t gi = (size_t)gy * S.W + gx;
      S.code_out[gi] = (uint8_t)g;
      S.id_out[gi] = (g == kGroupA || g == kGroupB) ? T.id[i] : 0u;
      if (MODE == 1) {
        S.tau_out[gi] = T.tau_a[i];
        S.tau_out[plane + gi] = T.tau_b[i];
      }
    }
    if (last) {
      const bool moved = interior && (win_mask & lane_bit) != 0ull;
      cnt[0] += __popcll(__ballot(g == kGroupA));
      cnt[1] += __popcll(__ballot(g == kGroupB));
      cnt[2] += __popcll(__ballot(g == kGroupA && gx >= S.W - S.cross_b));
      cnt[3] += __popcll(__ballot(g == kGroupB && gx < S.cross_a));
      cnt[4] += __popcll(__ballot(moved));
    }
  }
  if (last) {
    __syncthreads();  // queue space is free now: reuse it for the reduction
    if (tid < kTileStatFields) T.queue[tid] = 0u;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
      for (int f = 0; f < kTileStatFields; ++f) atomicAdd(&T.queue[f], cnt[f]);
    }
    __syncthreads();
    if (tid < kTileStatFields) S.tile_stats[(size_t)tile_index * kTileStatFields + tid] = T.queue[tid];
  }
}

}  // namespace pedsim
