// One-wave tile engine: a single wavefront advances one tile of a scenario by
// k steps of the bi-directional pedestrian update (Sec. III, Sec. IV.b-d).
//
// The region is 64 columns x R rows (R <= 64) around the tile (interior plus
// a 3k-cell halo, as in the multi-wave engine). Lane r owns row r: its A, B
// and wall masks (one bit per cell) live in registers, and the rows above and
// below are read with full-wave DPP shifts, so the mask passes touch no LDS
// and need no workgroup barrier. LDS holds the agent ids, the per-step
// occupancy history, the side-request and contested-winner masks, and one
// work queue. Per step:
//   1. forward   F requests of every agent (mask arithmetic); blocked agents
//                with an empty side candidate are queued;
//   2. draw      queued agents draw Philox words and pick a side candidate
//                (LEM eq. 1 / ACO eq. 2); picks are or-ed into LDS masks;
//   3. gather    eight requester masks per row: single requesters win,
//                contested cells are queued with their requester directions;
//   4. resolve   contested cells keep the lowest (Philox word 0, agent
//                number) (Sec. IV.d);
//   5. commit    new occupancy (recorded in the history) and id moves.
// The pheromone planes are not kept in LDS: a cell's value after s steps is
// fl(keep * v) (+ dtau when occupied) applied s times to its value at the
// launch start, using the recorded occupancy, exactly the per-step update of
// eq. 3 then eq. 4. It is evaluated where needed: at ACO candidates during
// step 2 and for every interior cell at write-back.
#pragma once

#include "rules.hpp"
#include "tile_engine.hpp"

namespace pedsim {

constexpr int kWaveMaxRows = 64;
constexpr int kWaveMaxSteps = 8;

// LDS layout of a one-wave region of R rows (64 columns).
struct WaveLayout {
  int R, k;
  __host__ __device__ size_t ids() const { return 0; }
  __host__ __device__ size_t hist() const { return ids() + (size_t)R * 64 * 4; }       // [k+1][2][R] u64
  __host__ __device__ size_t wall() const { return hist() + (size_t)(k + 1) * 2 * R * 8; }  // [R] u64
  __host__ __device__ size_t side() const { return wall() + (size_t)R * 8; }           // [6][R] u64
  __host__ __device__ size_t cwin() const { return side() + (size_t)6 * R * 8; }       // [8][R] u64
  __host__ __device__ size_t queue() const { return cwin() + (size_t)8 * R * 8; }      // [R*64] u32
  __host__ __device__ size_t ctl() const { return queue() + (size_t)R * 64 * 4; }
  __host__ __device__ size_t bytes() const { return ctl() + 16; }
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
// Row r's value broadcast to every lane (r wave-uniform).
__device__ __forceinline__ uint64_t row_of(uint64_t v, int r) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, r);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), r);
  return ((uint64_t)hi << 32) | lo;
}

template <int MODE>
__device__ void advance_tile_wave(const Scenario& S, uint8_t* smem, int R, int k_max, int tx, int ty, int tile_index,
                                  uint64_t t0, int steps, bool last) {
  const WaveLayout L{R, k_max};
  uint32_t* ids = (uint32_t*)(smem + L.ids());
  uint64_t* hist = (uint64_t*)(smem + L.hist());
  uint64_t* wall_m = (uint64_t*)(smem + L.wall());
  uint64_t* side = (uint64_t*)(smem + L.side());
  uint64_t* cwin = (uint64_t*)(smem + L.cwin());
  uint32_t* queue = (uint32_t*)(smem + L.queue());
  uint32_t* ctl = (uint32_t*)(smem + L.ctl());
  auto H = [&](int s, int g, int r) -> uint64_t& { return hist[((size_t)s * 2 + g) * R + r]; };

  const int lane = threadIdx.x & 63;
  const int h = S.halo;
  const int x0 = tx * S.IX - h;
  const int y0 = ty * S.IY - h;
  const size_t plane = (size_t)S.W * (size_t)S.H;
  const uint64_t lane_bit = 1ull << lane;
  const bool row_lane = lane < R;

  // ---- stage: row r's masks end in lane r; ids in LDS ------------------------
  uint64_t A = 0ull, B = 0ull, Wl = ~0ull;  // lanes >= R: all wall, never empty
  constexpr int kBatch = 4;
  for (int r0 = 0; r0 < R; r0 += kBatch) {
    int g[kBatch];
    uint32_t idv[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int gx = x0 + lane, gy = y0 + r0 + j;
      const bool in = r0 + j < R && gx >= 0 && gx < S.W && gy >= 0 && gy < S.H;
      const size_t gi = in ? (size_t)gy * S.W + gx : 0;
      g[j] = in ? S.code_in[gi] : kWall;
      idv[j] = in ? S.id_in[gi] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int r = r0 + j;
      if (r >= R) break;
      const uint64_t ba = __ballot(g[j] == kGroupA), bb = __ballot(g[j] == kGroupB), bw = __ballot(g[j] == kWall);
      if (lane == r) {
        A = ba;
        B = bb;
        Wl = bw;
      }
      ids[r * 64 + lane] = idv[j];
    }
  }
  if (row_lane) {
    H(0, 0, lane) = A;
    H(0, 1, lane) = B;
    wall_m[lane] = Wl;
  }
  __syncthreads();

  uint64_t moved_in = 0ull;  // this lane's row: cells entered in the last step
  for (int s = 0; s < steps; ++s) {
    const uint64_t t = t0 + (uint64_t)s;

    // ---- 1. forward requests; queue blocked agents with an empty side cell ----
    const uint64_t E = ~(A | B | Wl);
    const uint64_t Eu = from_up(E), Ed = from_down(E);
    const uint64_t e_r = E >> 1, e_l = E << 1;
    const uint64_t fA = A & e_r, fB = B & e_l;
    const uint64_t side_a = (Eu >> 1) | (Ed >> 1) | Eu | Ed;
    const uint64_t side_b = (Eu << 1) | (Ed << 1) | Eu | Ed;
    uint64_t act = (A & ~e_r & side_a) | (B & ~e_l & side_b);
    if (lane == 0) {
      ctl[0] = 0u;
      ctl[1] = 0u;
    }
    __syncthreads();
    if (row_lane) {
#pragma unroll
      for (int q = 0; q < 6; ++q) side[q * R + lane] = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) cwin[q * R + lane] = 0ull;
      if (act) {
        uint32_t pos = atomicAdd(&ctl[0], (uint32_t)__popcll(act));
        while (act) {
          const int c = __ffsll((unsigned long long)act) - 1;
          act &= act - 1;
          queue[pos++] = (uint32_t)lane | ((uint32_t)c << 10);
        }
      }
    }
    __syncthreads();

    // ---- 2. queued agents pick a side candidate -------------------------------
    {
      const int nq = (int)ctl[0];
      for (int q = lane; q < nq; q += 64) {
        const uint32_t e = queue[q];
        const int r = (int)(e & 1023u), c = (int)((e >> 10) & 255u);
        const bool is_a = (H(s, 0, r) >> c) & 1ull;
        const int d = is_a ? 1 : -1;
        auto empty_at = [&](int rr, int cc) -> bool {
          if (rr < 0 || rr >= R || cc < 0 || cc >= 64) return false;
          const uint64_t occ = H(s, 0, rr) | H(s, 1, rr) | wall_m[rr];
          return !((occ >> cc) & 1ull);
        };
        const unsigned avail = (unsigned)empty_at(r - 1, c + d) | ((unsigned)empty_at(r + 1, c + d) << 1) |
                               ((unsigned)empty_at(r - 1, c) << 2) | ((unsigned)empty_at(r + 1, c) << 3);
        const Words w = agent_words(ids[r * 64 + c] - 1u, t, S.key0, S.key1);
        int req;
        if (MODE == 0) {
          req = lem_choose(avail, w.w1, w.w2);
        } else {
          const int gp = is_a ? 0 : 1;
          const float* tp = S.tau_in + (is_a ? 0 : plane);
          float tau[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            tau[j] = 0.0f;
            if ((avail >> j) & 1u) {
              const int rr = r + ((j & 1) ? 1 : -1);
              const int cc = c + (j < 2 ? d : 0);
              float v = tp[(size_t)(y0 + rr) * S.W + (x0 + cc)];
              for (int u = 1; u <= s; ++u) {  // the cell's value at step s
                v = S.keep * v;
                if ((H(u, gp, rr) >> cc) & 1ull) v = v + S.dtau;
              }
              tau[j] = v;
            }
          }
          req = aco_choose(avail, tau, S.alpha, S.eta_diag, S.eta_lat, w.w1, w.w2);
        }
        int which = -1;  // 0 FD-A, 1 FD-B, 2 FD+A, 3 FD+B, 4 L-, 5 L+
        if (req == kReqFDm) which = is_a ? 0 : 1;
        if (req == kReqFDp) which = is_a ? 2 : 3;
        if (req == kReqLm) which = 4;
        if (req == kReqLp) which = 5;
        if (which >= 0) atomicOr((unsigned long long*)&side[which * R + r], 1ull << c);
      }
    }
    __syncthreads();

    // ---- 3. requesters per empty cell: single ones win, contested are queued ---
    uint64_t W[8];
    {
      uint64_t own[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) own[q] = row_lane ? side[q * R + lane] : 0ull;
      W[0] = fA << 1;                   // A from the left
      W[1] = fB >> 1;                   // B from the right
      W[2] = from_down(own[0]) << 1;    // A from below-left (FD-)
      W[3] = from_up(own[2]) << 1;      // A from above-left (FD+)
      W[4] = from_down(own[1]) >> 1;    // B from below-right (FD-)
      W[5] = from_up(own[3]) >> 1;      // B from above-right (FD+)
      W[6] = from_down(own[4]);         // from below (L-)
      W[7] = from_up(own[5]);           // from above (L+)
      uint64_t ones = 0ull, twos = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        twos |= ones & W[q];
        ones |= W[q];
      }
      if (lane == 0) ctl[1] = 0u;
      __syncthreads();
      if (row_lane && twos) {
        uint32_t pos = atomicAdd(&ctl[1], (uint32_t)__popcll(twos));
        uint64_t bits = twos;
        while (bits) {
          const int c = __ffsll((unsigned long long)bits) - 1;
          bits &= bits - 1;
          uint32_t dirs = 0;
#pragma unroll
          for (int q = 0; q < 8; ++q) dirs |= (uint32_t)((W[q] >> c) & 1ull) << q;
          queue[pos++] = (uint32_t)lane | ((uint32_t)c << 10) | (dirs << 18);
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) W[q] &= ~twos;
    }
    __syncthreads();

    // ---- 4. contested cells: lowest (word 0, agent number) wins ----------------
    {
      const int nc = (int)ctl[1];
      for (int q = lane; q < nc; q += 64) {
        const uint32_t e = queue[q];
        const int r = (int)(e & 1023u), c = (int)((e >> 10) & 255u);
        uint32_t dirs = e >> 18;
        uint32_t best_t = 0xFFFFFFFFu, best_k = 0xFFFFFFFFu;
        int best = -1;
        while (dirs) {
          const int kk = __ffs(dirs) - 1;
          dirs &= dirs - 1;
          const uint32_t agent = ids[(r + dir_dr(kk)) * 64 + c + dir_dc(kk)] - 1u;
          const uint32_t tk = agent_words(agent, t, S.key0, S.key1).w0;
          if (best < 0 || tk < best_t || (tk == best_t && agent < best_k)) {
            best = kk;
            best_t = tk;
            best_k = agent;
          }
        }
        atomicOr((unsigned long long*)&cwin[best * R + r], 1ull << c);
      }
    }
    __syncthreads();

    // ---- 5. commit: next occupancy, history, ids follow their agents ----------
    {
#pragma unroll
      for (int q = 0; q < 8; ++q) W[q] |= row_lane ? cwin[q * R + lane] : 0ull;
      const uint64_t in_a = W[0] | W[2] | W[3] | (W[6] & from_down(A)) | (W[7] & from_up(A));
      const uint64_t in_b = W[1] | W[4] | W[5] | (W[6] & from_down(B)) | (W[7] & from_up(B));
      const uint64_t out = (W[0] >> 1) | (W[1] << 1) | (from_up(W[2]) >> 1) | (from_down(W[3]) >> 1) |
                           (from_up(W[4]) << 1) | (from_down(W[5]) << 1) | from_up(W[6]) | from_down(W[7]);
      A = (A & ~out) | in_a;
      B = (B & ~out) | in_b;
      moved_in = in_a | in_b;
      if (row_lane) {
        H(s + 1, 0, lane) = A;
        H(s + 1, 1, lane) = B;
        uint64_t bits = moved_in;  // a target was empty at t and a source occupied: no overlap
        while (bits) {
          const int c = __ffsll((unsigned long long)bits) - 1;
          bits &= bits - 1;
          int kk = 0;
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if ((W[q] >> c) & 1ull) kk = q;
          ids[lane * 64 + c] = ids[(lane + dir_dr(kk)) * 64 + c + dir_dc(kk)];
        }
      }
    }
    __syncthreads();
  }

  // ---- write the interior back; pheromone applied step by step from history --
  uint32_t cnt[kTileStatFields] = {0, 0, 0, 0, 0};
  for (int r = h; r < h + S.IY && r < R; ++r) {
    const int gy = y0 + r;
    const int c = lane;
    const int gx = x0 + c;
    const bool interior = c >= h && c < h + S.IX && gx < S.W && gy < S.H;
    const uint64_t ra = row_of(A, r), rb = row_of(B, r), rw = row_of(Wl, r), rin = row_of(moved_in, r);
    int g = kEmpty;
    if (interior) {
      const size_t gi = (size_t)gy * S.W + gx;
      g = (ra & lane_bit) ? kGroupA : ((rb & lane_bit) ? kGroupB : ((rw & lane_bit) ? kWall : kEmpty));
      S.code_out[gi] = (uint8_t)g;
      S.id_out[gi] = (g == kGroupA || g == kGroupB) ? ids[r * 64 + c] : 0u;
      if (MODE == 1) {
        float va = S.tau_in[gi], vb = S.tau_in[plane + gi];
        for (int u = 1; u <= steps; ++u) {
          va = S.keep * va;
          vb = S.keep * vb;
          if ((H(u, 0, r) >> c) & 1ull) va = va + S.dtau;
          if ((H(u, 1, r) >> c) & 1ull) vb = vb + S.dtau;
        }
        S.tau_out[gi] = va;
        S.tau_out[plane + gi] = vb;
      }
    }
    if (last) {
      cnt[0] += __popcll(__ballot(g == kGroupA));
      cnt[1] += __popcll(__ballot(g == kGroupB));
      cnt[2] += __popcll(__ballot(g == kGroupA && gx >= S.W - S.cross_b));
      cnt[3] += __popcll(__ballot(g == kGroupB && gx < S.cross_a));
      cnt[4] += __popcll(__ballot(interior && steps > 0 && (rin & lane_bit)));
    }
  }
  if (last && lane < kTileStatFields) {
    uint32_t v = cnt[0];
#pragma unroll
    for (int f = 1; f < kTileStatFields; ++f)
      if (lane == f) v = cnt[f];
    S.tile_stats[(size_t)tile_index * kTileStatFields + lane] = v;
  }
}

}  // namespace pedsim
