// Larger scanning and moving ranges (the paper's future work, Sec. VII) for
// gfx950: one launch per step, one workgroup per tile.
//
// Rules (the base step of Sec. IV.b-d widened to a scanning range S and a
// moving range M, 1 <= M <= S <= 8):
//   * the five candidates F, FD-, FD+, L-, L+ become rays; along each ray an
//     agent sees the free run f (consecutive cells next to it that are inside
//     the grid and empty at t, at most S); an open ray (f >= 1) is travelled
//     k = min(f, M) cells;
//   * forward first: an open forward ray is taken without a draw; otherwise
//     LEM (eq. 1) ranks the open side rays by (f/S)(Dmin/D), D the distance
//     from the landing cell to the point M+1 cells ahead, and ACO (eq. 2)
//     weighs them by tau(landing cell)^alpha (f/S)^beta D^-beta;
//   * every cell empty at t goes to the lowest (Philox word 0, agent number)
//     among the agents landing on it; eq. 3 then eq. 4 on every cell.
// With S = M = 1 this is the base step bit for bit.
//
// A tile is an interior of TX x TY cells advanced k steps per launch. The new
// state of a cell depends on cells up to R1 = 2M + S away (the contest at its
// own cell, or at the landing cell of its agent, up to M away, among
// claimants up to M from that cell, whose rays reach S further), so after
// step j of a launch the state is needed exactly on the interior grown by
// (k-1-j) R1 cells, and the workgroup stages the codes of the interior grown
// by k R1 (ids and pheromone by (k-1) R1 + 3M, all it will read). Each step:
//   1. list the agents up to (k-1-j) R1 + 2M from the interior (a wave ballot
//      and one LDS atomic per wave);
//   2. requests: every listed agent scans its rays in LDS and chooses (the
//      forward ray without a draw; a side ray by eq. 1 or eq. 2 with its
//      Philox words 1 and 2); every landing cell counts its claims;
//   3. resolve: a landing cell with one claim goes to its claimant, one with
//      several to the lowest (Philox word 0, agent number), by a 64-bit LDS
//      atomic min of (word 0 << 32 | agent number << 1 | group - 1) -- min is
//      commutative, so the winner never depends on thread order;
//   4. commit on the interior grown by (k-1-j) R1: an empty cell with a claim
//      takes the winner's group and id from its key, an agent whose landing
//      cell's key names it leaves, both planes evaporate and gain the deposit
//      where their group stands after the step. A cell's new value depends
//      only on its own old value and the keys, so the commit is done in place
//      in LDS; after the last step the interior goes to the output planes.
// Reads one copy of the planes and writes the other (the caller's planes and
// the scratch shadow ping-pong), since a tile's halo is its neighbours'
// interior.
#include "range_step.hpp"

#include "pedsim_internal.hpp"

namespace pedsim {

namespace {

// Ray r (0 F, 1 FD-, 2 FD+, 3 L-, 4 L+) of an agent heading d.
__device__ __forceinline__ int ray_dx(int r, int d) { return r <= 2 ? d : 0; }
__device__ __forceinline__ int ray_dy(int r) { return (r == 1 || r == 3) ? -1 : ((r == 2 || r == 4) ? 1 : 0); }

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD one
// contiguous run of row-major tiles so shared halo lines stay in its L2.
__device__ __forceinline__ int range_tile_of_block(int bid, int ntiles) {
  const int per = (ntiles + 7) >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// LEM over the open side rays 1..4 (f[r] >= 1): a stable sort by descending
// score C_r = f_r / D_r in the order [FD_s, FD_-s, L_s, L_-s] (s = +1 when
// bit 0 of w2 is set), then the rank index of the normal draw (as in the base
// rule), clamped to the last open ray. Returns the ray, or 0 if none is open.
__device__ __forceinline__ int range_lem(const int f[5], const int d2[5], uint32_t w1, uint32_t w2) {
  const int flip = (int)(w2 & 1u);
  int n = 0;
#pragma unroll
  for (int r = 1; r <= 4; ++r) n += f[r] >= 1;
  if (n == 0) return 0;
  int idx = (w1 >= kNormalCut0) + (w1 >= kNormalCut1) + (w1 >= kNormalCut2);
  idx = idx < n - 1 ? idx : n - 1;
  int pick = 0;
#pragma unroll
  for (int r = 1; r <= 4; ++r) {
    if (f[r] < 1) continue;
    const int pos_r = (r - 1) ^ flip;
    int rank = 0;
#pragma unroll
    for (int q = 1; q <= 4; ++q) {
      if (q == r || f[q] < 1) continue;
      // C_q > C_r  <=>  f_q^2 D2_r > f_r^2 D2_q (all small integers)
      const int lhs = f[q] * f[q] * d2[r];
      const int rhs = f[r] * f[r] * d2[q];
      rank += (lhs > rhs) || (lhs == rhs && ((q - 1) ^ flip) < pos_r);
    }
    if (rank == idx) pick = r;
  }
  return pick;
}

// ACO over the open side rays: weights tau^alpha * eta summed left to right
// over FD-, FD+, L-, L+; u = (w1 >> 8) 2^-24; the first ray whose running sum
// exceeds fl(u * sum), else the last positive one; all-zero weights fall back
// to the LEM rule with the same words. One binary32 rounding per operation.
__device__ __forceinline__ int range_aco(const int f[5], const int d2[5], const float tau[5], const float eta[5],
                                         int alpha, uint32_t w1, uint32_t w2) {
  float w[5];
#pragma unroll
  for (int r = 1; r <= 4; ++r) {
    float p = 1.0f;
    if (alpha > 0) {
      p = tau[r];
      for (int a = 1; a < alpha; ++a) p = p * tau[r];
    }
    w[r] = f[r] >= 1 ? p * eta[r] : 0.0f;
  }
  float sum = w[1];
  sum = sum + w[2];
  sum = sum + w[3];
  sum = sum + w[4];
  if (sum == 0.0f) return range_lem(f, d2, w1, w2);
  const float u = (float)(w1 >> 8) * 0x1p-24f;
  const float target = u * sum;
  float running = 0.0f;
  int last = 0, pick = 0;
#pragma unroll
  for (int r = 1; r <= 4; ++r) {
    running = running + w[r];
    if (w[r] > 0.0f) {
      last = r;
      if (pick == 0 && target < running) pick = r;
    }
  }
  return pick ? pick : last;
}

constexpr unsigned long long kNoClaim = ~0ull;
constexpr int kStageBatch = 4;  // cells whose global loads a thread keeps in flight while staging
constexpr int kCellBatch = 2;   // cells a thread takes at a time in the list and commit phases

// q = i / d for i * d < 2^32, with m = ceil(2^32 / d): one multiply-high.
__device__ __forceinline__ uint32_t div_magic(uint32_t d) {
  return (uint32_t)((0x100000000ull + d - 1) / d);
}
__device__ __forceinline__ int fast_div(int i, uint32_t m) { return (int)__umulhi((uint32_t)i, m); }

// Number of lanes below this one whose bit is set in `bal`.
__device__ __forceinline__ int lanes_below_range(uint64_t bal) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}

template <int MODE, int S>
__global__ __launch_bounds__(kRangeMaxThreads) void range_kernel(RangeScenario P, int steps, int last) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int ntiles = P.tiles_x * P.tiles_y;
  const int tile = range_tile_of_block(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  const int TX = P.TX, TY = P.TY, M = P.M;
  const int R1 = 2 * M + S;  // reach of one step
  // halos of the arrays (cells beyond the interior), fixed for the launch
  const int hc = steps * R1;            // codes
  const int hp = (steps - 1) * R1 + 3 * M;  // ids and pheromone
  const int hr = (steps - 1) * R1 + 2 * M;  // request bytes
  const int hk = (steps - 1) * R1 + M;      // claim keys and counts
  const int CW = TX + 2 * hc, CH = TY + 2 * hc;
  const int PW = TX + 2 * hp, PH = TY + 2 * hp;
  const int RW = TX + 2 * hr, RH = TY + 2 * hr;
  const int KW = TX + 2 * hk, KH = TY + 2 * hk;
  const RangeLayout L{TX, TY, S, M, steps, MODE != kModeLem};
  uint8_t* code = smem + L.code();
  uint32_t* ids = (uint32_t*)(smem + L.ids());
  uint8_t* rq = smem + L.req();
  uint16_t* list = (uint16_t*)(smem + L.list());
  unsigned long long* keys = (unsigned long long*)(smem + L.keys());
  uint32_t* claims = (uint32_t*)(smem + L.claims());
  uint32_t* cnt = (uint32_t*)(smem + L.ctl());  // [0..4] counters, [5] agents in the list
  float* eta_s = (float*)(cnt + 8);             // eta^beta: [0 lateral, 1 diagonal][free run - 1]
  float* tau_a = (float*)(smem + L.tau());      // ACO: [PH][PW] per plane
  float* tau_b = tau_a + (size_t)PW * PH;
  // ACO, k > 1: the pheromone arrays keep their staged values for the whole
  // launch; a cell's value after step u is evaluated when needed from the
  // occupancy it had after each step v <= u (2 bits per step: 0 empty or
  // wall, 1 A, 2 B), with the operations of the per-step update in its order
  uint8_t* hist = smem + L.hist();
  constexpr bool kAco = MODE != kModeLem;
  const bool lazy = kAco && steps > 1;

  const int x0 = (tile % P.tiles_x) * TX, y0 = (tile / P.tiles_x) * TY;
  const int W = P.W, H = P.H;
  const int lane = threadIdx.x & 63;
  const int nthreads = blockDim.x;

  // this step's windows, as [lo, lo + width) in each array's coordinates:
  // step j leaves the state exact on the interior grown by (steps - 1 - j) R1
  auto req_window = [&](int j, int& lo, int& w, int& h) {
    const int grow = (steps - 1 - j) * R1;
    lo = hr - (grow + 2 * M);
    w = TX + 2 * (grow + 2 * M);
    h = TY + 2 * (grow + 2 * M);
  };
  auto key_window = [&](int j, int& lo, int& w, int& h) {
    const int grow = (steps - 1 - j) * R1;
    lo = hk - (grow + M);
    w = TX + 2 * (grow + M);
    h = TY + 2 * (grow + M);
  };

  // clear the claims of step j's key window
  auto clear_claims = [&](int j) {
    int klo, kw, kh;
    key_window(j, klo, kw, kh);
    const uint32_t mkw = div_magic((uint32_t)kw);
    for (int i = threadIdx.x; i < kw * kh; i += nthreads) {
      const int r = fast_div(i, mkw), c = i - r * kw;
      const int ki = (r + klo) * KW + c + klo;
      keys[ki] = kNoClaim;
      claims[ki] = 0u;
    }
  };

  // 2. list the agents of step j's request window that have an empty cell
  //    next to them on one of their five rays (the others make no request);
  //    clear every cell's request. A wave takes kCellBatch runs of 64 cells
  //    at a time, their LDS reads in flight together, and reserves the list
  //    entries of all of them with one LDS atomic. Reads the codes only.
  auto list_agents = [&](int j) {
    int rlo, rw, rh;
    req_window(j, rlo, rw, rh);
    const uint32_t mrw = div_magic((uint32_t)rw);
    for (int i0 = threadIdx.x - lane; i0 < rw * rh; i0 += nthreads * kCellBatch) {
      int ri[kCellBatch], at[kCellBatch], g[kCellBatch];
      bool valid[kCellBatch], agent[kCellBatch];
#pragma unroll
      for (int u = 0; u < kCellBatch; ++u) {
        const int i = i0 + u * nthreads + lane;
        valid[u] = i < rw * rh;
        const int ii = valid[u] ? i : 0;
        const int r = fast_div(ii, mrw) + rlo, c = ii - fast_div(ii, mrw) * rw + rlo;
        ri[u] = r * RW + c;
        at[u] = (r + hc - hr) * CW + c + hc - hr;
        g[u] = code[at[u]];
      }
#pragma unroll
      for (int u = 0; u < kCellBatch; ++u) {
        // the window lies 2 cells or more inside the code array: every
        // neighbour read is in range, agent or not
        const int d = g[u] == kGroupB ? -1 : 1;
        const bool open = (code[at[u] + d] == kEmpty) | (code[at[u] - CW + d] == kEmpty) |
                          (code[at[u] + CW + d] == kEmpty) | (code[at[u] - CW] == kEmpty) |
                          (code[at[u] + CW] == kEmpty);
        agent[u] = valid[u] && (g[u] == kGroupA || g[u] == kGroupB) && open;
        if (valid[u]) rq[ri[u]] = 0u;
      }
      uint64_t bal[kCellBatch];
      uint32_t total = 0u;
#pragma unroll
      for (int u = 0; u < kCellBatch; ++u) {
        bal[u] = __ballot(agent[u]);
        total += (uint32_t)__popcll(bal[u]);
      }
      if (total) {
        uint32_t base = 0u;
        if (lane == 0) base = atomicAdd(&cnt[5], total);
        base = __shfl(base, 0);
#pragma unroll
        for (int u = 0; u < kCellBatch; ++u) {
          if (agent[u]) list[base + lanes_below_range(bal[u])] = (uint16_t)ri[u];
          base += (uint32_t)__popcll(bal[u]);
        }
      }
    }
  };

  // 1. stage the codes (outside the grid reads as wall), the ids and, for
  //    ACO, both pheromone planes (whose array is a sub-rectangle of the code
  //    array). With aligned rows (P.quads) a load brings 4 cells: the aligned
  //    quads of columns covering each array's rows are dealt to the threads,
  //    kStageBatch quads of each array in flight before their LDS stores, and
  //    only the cells inside an array are stored. The first step's list reads
  //    only the codes, so the ids and pheromone of a thread's first batch stay
  //    in its registers, their loads in flight, until that list is built.
  //    Without aligned rows cells are dealt one by one in row-major order,
  //    kStageBatch cells' loads in flight.
  const int W4 = W >> 2;
  const size_t plane4 = ((size_t)W * H) >> 2;
  const int cx0 = x0 - hc, cy0 = y0 - hc, px0 = x0 - hp, py0 = y0 - hp;
  const int qc0 = cx0 >> 2, qp0 = px0 >> 2;  // floor: the origins may be negative
  const int nqc = ((cx0 + CW - 1) >> 2) - qc0 + 1, nqp = ((px0 + PW - 1) >> 2) - qp0 + 1;
  const int NC = CH * nqc, NP = PH * nqp;
  const uint32_t mqc = div_magic((uint32_t)nqc), mqp = div_magic((uint32_t)nqp);
  const uint32_t* code4 = (const uint32_t*)P.code_in;
  const uint4* id4 = (const uint4*)P.id_in;
  const uint4* tau4 = (const uint4*)P.tau_in;
  auto load_code_quad = [&](int i) -> uint32_t {
    const int r = fast_div(i, mqc), q = qc0 + i - r * nqc;
    const int gy = cy0 + r;
    const bool in = i < NC && gy >= 0 && gy < H && q >= 0 && q < W4;
    return in ? code4[(size_t)gy * W4 + q] : 0x01010101u * (uint32_t)kWall;
  };
  auto store_code_quad = [&](int i, uint32_t v) {
    if (i >= NC) return;
    const int r = fast_div(i, mqc), c = 4 * (qc0 + i - r * nqc) - cx0;  // the quad's first column
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (c + e >= 0 && c + e < CW) code[r * CW + c + e] = (uint8_t)(v >> (8 * e));
  };
  // the id, pheromone A and pheromone B quads of p-array quad i
  auto load_p_quad = [&](int i, uint4& vi, uint4& va, uint4& vb) {
    const int pr = fast_div(i, mqp), pq = qp0 + i - pr * nqp;
    const int py = py0 + pr;
    const bool pin = i < NP && py >= 0 && py < H && pq >= 0 && pq < W4;
    const size_t gi = pin ? (size_t)py * W4 + pq : 0;
    // (a zero written as a value: a captured constant would turn the select
    // into a generic-address load)
    vi = pin ? id4[gi] : make_uint4(0u, 0u, 0u, 0u);
    if (MODE != kModeLem) {
      va = pin ? tau4[gi] : make_uint4(0u, 0u, 0u, 0u);
      vb = pin ? tau4[plane4 + gi] : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store_p_quad = [&](int i, const uint4& vi, const uint4& va, const uint4& vb) {
    if (i >= NP) return;
    const int pr = fast_div(i, mqp), c = 4 * (qp0 + i - pr * nqp) - px0;
    const uint32_t ev[4] = {vi.x, vi.y, vi.z, vi.w};
    const uint32_t ea[4] = {va.x, va.y, va.z, va.w};
    const uint32_t eb[4] = {vb.x, vb.y, vb.z, vb.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (c + e >= 0 && c + e < PW) {
        ids[pr * PW + c + e] = ev[e];
        if (MODE != kModeLem) {
          tau_a[pr * PW + c + e] = __uint_as_float(ea[e]);
          tau_b[pr * PW + c + e] = __uint_as_float(eb[e]);
        }
      }
    }
  };
  uint4 held_i[kStageBatch], held_a[kStageBatch], held_b[kStageBatch];
  if (P.quads) {
    // the first batch's codes are stored before its other loads are issued:
    // a wait for a load also waits for every load issued before it
    uint32_t vc[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) vc[u] = load_code_quad(threadIdx.x + u * nthreads);
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) store_code_quad(threadIdx.x + u * nthreads, vc[u]);
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) load_p_quad(threadIdx.x + u * nthreads, held_i[u], held_a[u], held_b[u]);
    // later batches (regions larger than one batch per thread) go straight to LDS
    for (int i0 = threadIdx.x + nthreads * kStageBatch; i0 < (NC > NP ? NC : NP); i0 += nthreads * kStageBatch) {
      uint4 vi[kStageBatch], va[kStageBatch], vb[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        load_p_quad(i0 + u * nthreads, vi[u], va[u], vb[u]);
        vc[u] = load_code_quad(i0 + u * nthreads);
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        store_code_quad(i0 + u * nthreads, vc[u]);
        store_p_quad(i0 + u * nthreads, vi[u], va[u], vb[u]);
      }
    }
  } else {
    const int off = hc - hp;  // the pheromone array's origin in code-array coordinates
    const size_t plane = (size_t)W * H;
    const uint32_t mc = div_magic((uint32_t)CW);
    for (int i0 = threadIdx.x; i0 < CW * CH; i0 += nthreads * kStageBatch) {
      uint32_t vc[kStageBatch], vi[kStageBatch];
      float va[kStageBatch], vb[kStageBatch];
      int pi[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int i = i0 + u * nthreads;
        const int r = fast_div(i, mc), c = i - r * CW;
        const int gx = x0 - hc + c, gy = y0 - hc + r;
        const bool in = i < CW * CH && gx >= 0 && gx < W && gy >= 0 && gy < H;
        const int pr = r - off, pc = c - off;
        const bool pin = pr >= 0 && pr < PH && pc >= 0 && pc < PW;  // (i < CW * CH follows)
        pi[u] = pin ? pr * PW + pc : -1;
        const size_t gi = in ? (size_t)gy * W + gx : 0;
        vc[u] = in ? P.code_in[gi] : (uint32_t)kWall;
        vi[u] = in && pin ? P.id_in[gi] : 0u;
        if (MODE != kModeLem) {
          va[u] = in && pin ? P.tau_in[gi] : 0.0f;
          vb[u] = in && pin ? P.tau_in[plane + gi] : 0.0f;
        }
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int i = i0 + u * nthreads;
        if (i < CW * CH) code[i] = (uint8_t)vc[u];
        if (pi[u] >= 0) {
          ids[pi[u]] = vi[u];
          if (MODE != kModeLem) {
            tau_a[pi[u]] = va[u];
            tau_b[pi[u]] = vb[u];
          }
        }
      }
    }
  }
  if (threadIdx.x < 2 * kRangeMax) eta_s[threadIdx.x] = P.eta[threadIdx.x / kRangeMax][threadIdx.x % kRangeMax];
  if (threadIdx.x < 8) cnt[threadIdx.x] = 0u;
  clear_claims(0);
  __syncthreads();  // codes staged, counters and the first step's claims cleared
  list_agents(0);
  if (lazy) {  // every slot holds the staged occupancy, on the cells whose value is read later
    const int g0w = (steps - 1) * R1;
    const int ew = TX + 2 * g0w, eh = TY + 2 * g0w;
    const uint32_t mew = div_magic((uint32_t)ew);
    for (int i = threadIdx.x; i < ew * eh; i += nthreads) {
      const int er = fast_div(i, mew), ec = i - er * ew;
      const int g = code[(er - g0w + hc) * CW + ec - g0w + hc];
      hist[(er - g0w + hp) * PW + ec - g0w + hp] = (uint8_t)(g == kGroupA ? 0x55u : (g == kGroupB ? 0xAAu : 0u));
    }
  }
  if (P.quads) {
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) store_p_quad(threadIdx.x + u * nthreads, held_i[u], held_a[u], held_b[u]);
  }
  __syncthreads();  // ids, pheromone and the first step's list in place

  uint32_t n_a = 0, n_b = 0, c_a = 0, c_b = 0, moved = 0;
  for (int j = 0; j < steps; ++j) {
    const uint64_t t = P.t + (uint64_t)j;
    const int grow = (steps - 1 - j) * R1;  // the state after this step is needed on the interior grown by it
    int klo, kw, kh;
    key_window(j, klo, kw, kh);
    const int n_agents = (int)cnt[5];

    // 3. requests of the listed agents; every landing cell counts its claims
    const uint32_t mRW = div_magic((uint32_t)RW);
    for (int q = threadIdx.x; q < n_agents; q += nthreads) {
      const int ri = list[q];
      const int r = fast_div(ri, mRW), c = ri - r * RW;  // request-array coordinates
      const int cx = c + hc - hr, cy = r + hc - hr;     // code-array coordinates
      const int at = cy * CW + cx;
      const int g = code[at];
      const int d = g == kGroupA ? 1 : -1;
      // (listed agents have at least one ray open)
      uint32_t first[5];
#pragma unroll
      for (int ray = 0; ray < 5; ++ray) first[ray] = code[at + ray_dy(ray) * CW + ray_dx(ray, d)];
      int f[5], d2[5];
      bool side = false;
#pragma unroll
      for (int ray = 0; ray < 5; ++ray) {
        const int ux = ray_dx(ray, d), uy = ray_dy(ray);
        // the rest of the ray read at once (independent LDS loads), the free
        // run counted afterwards
        const int step = uy * CW + ux;
        uint32_t v[S];
        v[0] = first[ray];
#pragma unroll
        for (int jj = 1; jj < S; ++jj) v[jj] = code[at + (jj + 1) * step];
        int run = 0;
        bool open = true;
#pragma unroll
        for (int qq = 0; qq < S; ++qq) {
          open = open && v[qq] == kEmpty;
          run += open ? 1 : 0;
        }
        f[ray] = run;
        const int k = run < M ? run : M;
        const int a = ray <= 2 ? 1 : 0;
        const int b = ray == 0 ? 0 : 1;
        const int dx = M + 1 - a * k;
        d2[ray] = dx * dx + b * k * k;
        side |= ray > 0 && run >= 1;
      }
      const int px = c + hp - hr, py = r + hp - hr;  // id / pheromone-array coordinates
      int choice = -1;
      if (f[0] >= 1) {
        choice = 0;
      } else if (side) {
        const Words w = agent_words(ids[py * PW + px] - 1u, t, P.key0, P.key1);
        if (MODE == kModeLem) {
          choice = range_lem(f, d2, w.w1, w.w2);
        } else {
          const float* tp = g == kGroupA ? tau_a : tau_b;
          float tau[5], eta[5];
#pragma unroll
          for (int ray = 1; ray <= 4; ++ray) {
            tau[ray] = 0.0f;
            eta[ray] = 0.0f;
            if (f[ray] >= 1) {
              const int k = f[ray] < M ? f[ray] : M;
              eta[ray] = eta_s[(ray <= 2 ? kRangeMax : 0) + f[ray] - 1];
              const int li = (py + k * ray_dy(ray)) * PW + px + k * ray_dx(ray, d);
              float x = tp[li];
              if (lazy && j > 0) {  // the updates of steps 0 .. j-1
                const uint32_t hc_ = hist[li];
                for (int v = 0; v < j; ++v) {
                  x = P.keep * x;
                  if ((int)((hc_ >> (2 * v)) & 3u) == g) x = x + P.dtau;
                }
              }
              tau[ray] = x;
            }
          }
          choice = range_aco(f, d2, tau, eta, P.alpha, w.w1, w.w2);
        }
      }
      if (choice >= 0) {
        const int len = f[choice] < M ? f[choice] : M;
        rq[ri] = (uint8_t)((choice + 1) | (len << 3));
        // landing cell in key-array coordinates; outside this step's key window
        // it is not needed
        const int kx = c + hk - hr + len * ray_dx(choice, d), ky = r + hk - hr + len * ray_dy(choice);
        if (kx >= klo && kx < klo + kw && ky >= klo && ky < klo + kh) atomicAdd(&claims[ky * KW + kx], 1u);
      }
    }
    __syncthreads();

    // 4. resolve: one claim goes to its claimant; several to the lowest
    //    (Philox word 0, agent number)
    for (int q = threadIdx.x; q < n_agents; q += nthreads) {
      const int ri = list[q];
      const int code_req = rq[ri];
      if (!code_req) continue;
      const int r = fast_div(ri, mRW), c = ri - r * RW;
      const int g = code[(r + hc - hr) * CW + c + hc - hr];
      const int ray = (code_req & 7) - 1, len = code_req >> 3;
      const int d = g == kGroupA ? 1 : -1;
      const int kx = c + hk - hr + len * ray_dx(ray, d), ky = r + hk - hr + len * ray_dy(ray);
      if (kx < klo || kx >= klo + kw || ky < klo || ky >= klo + kh) continue;
      const int ki = ky * KW + kx;
      const uint32_t k_agent = ids[(r + hp - hr) * PW + c + hp - hr] - 1u;
      const unsigned long long who = ((unsigned long long)k_agent << 1) | (unsigned long long)(g - 1);
      if (claims[ki] == 1u) {
        keys[ki] = who;
      } else {
        const uint32_t w0 = agent_words(k_agent, t, P.key0, P.key1).w0;
        atomicMin(&keys[ki], ((unsigned long long)w0 << 32) | who);
      }
    }
    __syncthreads();

    // 5. commit on the interior grown by `grow`. Before the last step, in
    //    place in LDS and only where something moves: every listed agent that
    //    won its landing cell leaves its cell and enters the landing cell
    //    (each inside the window); nothing else changes but the pheromone,
    //    which is evaluated lazily from the occupancy history. The last step
    //    writes the interior to the output planes, with pheromone and counters.
    const bool final_step = j == steps - 1;
    if (!final_step) {
      const uint32_t slots = (0x3Fu << (2 * j)) & 0x3Fu;  // history slots of steps j .. k-2
      for (int q = threadIdx.x; q < n_agents; q += nthreads) {
        const int ri = list[q];
        const int code_req = rq[ri];
        if (!code_req) continue;
        const int r = fast_div(ri, mRW), c = ri - r * RW;
        const int ix = c - hr, iy = r - hr;  // interior coordinates of the agent's cell
        const int ci = (iy + hc) * CW + ix + hc, pi = (iy + hp) * PW + ix + hp;
        const int g = code[ci];
        const int ray = (code_req & 7) - 1, len = code_req >> 3;
        const int d = g == kGroupA ? 1 : -1;
        const int tx_ = ix + len * ray_dx(ray, d), ty_ = iy + len * ray_dy(ray);
        if (tx_ + hk < klo || tx_ + hk >= klo + kw || ty_ + hk < klo || ty_ + hk >= klo + kh) continue;
        const uint32_t nid = ids[pi];
        const unsigned long long key = keys[(ty_ + hk) * KW + tx_ + hk];
        if ((uint32_t)((key >> 1) & 0x7fffffffull) != nid - 1u) continue;  // lost its contest
        if (ix >= -grow && ix < TX + grow && iy >= -grow && iy < TY + grow) {
          code[ci] = (uint8_t)kEmpty;
          ids[pi] = 0u;
          if (lazy) hist[pi] = (uint8_t)(hist[pi] & ~slots);
        }
        if (tx_ >= -grow && tx_ < TX + grow && ty_ >= -grow && ty_ < TY + grow) {
          const int ti = (ty_ + hp) * PW + tx_ + hp;
          code[(ty_ + hc) * CW + tx_ + hc] = (uint8_t)g;
          ids[ti] = nid;
          if (lazy) hist[ti] = (uint8_t)((hist[ti] & ~slots) | ((g == kGroupA ? 0x55u : 0xAAu) & slots));
        }
      }
    } else {
    const int ew = TX + 2 * grow, eh = TY + 2 * grow;
    const uint32_t mew = div_magic((uint32_t)ew);
    const size_t plane = (size_t)W * H;
    // kCellBatch cells per thread at a time: first every cell's own LDS
    // values, then the landing cells' keys of its movers, then the stores
    for (int i0 = threadIdx.x; i0 < ew * eh; i0 += nthreads * kCellBatch) {
      int ix[kCellBatch], iy[kCellBatch], g0[kCellBatch], req[kCellBatch], kl[kCellBatch];
      bool valid[kCellBatch];
      uint32_t id0[kCellBatch], h0[kCellBatch];
      unsigned long long kown[kCellBatch], kmv[kCellBatch];
      float ta[kCellBatch], tb[kCellBatch];
#pragma unroll
      for (int u = 0; u < kCellBatch; ++u) {
        const int i = i0 + u * nthreads;
        const int ii = i < ew * eh ? i : 0;
        const int er = fast_div(ii, mew), ec = ii - er * ew;
        ix[u] = ec - grow;  // interior coordinates
        iy[u] = er - grow;
        valid[u] = i < ew * eh && x0 + ix[u] < W && y0 + iy[u] < H;
        const int pi = (iy[u] + hp) * PW + ix[u] + hp;
        g0[u] = code[(iy[u] + hc) * CW + ix[u] + hc];
        kown[u] = keys[(iy[u] + hk) * KW + ix[u] + hk];
        id0[u] = ids[pi];
        req[u] = rq[(iy[u] + hr) * RW + ix[u] + hr];
        if (MODE != kModeLem) {
          ta[u] = tau_a[pi];
          tb[u] = tau_b[pi];
          h0[u] = lazy ? hist[pi] : 0u;
        }
      }
#pragma unroll
      for (int u = 0; u < kCellBatch; ++u) {
        kl[u] = -1;
        if ((g0[u] == kGroupA || g0[u] == kGroupB) && req[u]) {
          const int ray = (req[u] & 7) - 1, len = req[u] >> 3;
          const int d = g0[u] == kGroupA ? 1 : -1;
          kl[u] = (iy[u] + hk + len * ray_dy(ray)) * KW + ix[u] + hk + len * ray_dx(ray, d);
        }
        kmv[u] = kl[u] >= 0 ? keys[kl[u]] : kNoClaim;
      }
#pragma unroll
      for (int u = 0; u < kCellBatch; ++u) {
        if (!valid[u]) continue;
        const int g = g0[u];
        int nc = g;
        uint32_t nid = 0u;
        if (g == kEmpty) {
          if (kown[u] != kNoClaim) {
            nc = (int)(kown[u] & 1ull) + 1;
            nid = (uint32_t)((kown[u] >> 1) & 0x7fffffffull) + 1u;
            moved += final_step ? 1u : 0u;
          }
        } else if (g == kGroupA || g == kGroupB) {
          nid = id0[u];
          if (kl[u] >= 0 && (uint32_t)((kmv[u] >> 1) & 0x7fffffffull) == nid - 1u) {
            nc = kEmpty;
            nid = 0u;
          }
        }
        float va = 0.0f, vb = 0.0f;
        if (MODE != kModeLem) {
          va = ta[u];
          vb = tb[u];
          if (lazy) {  // the updates of steps 0 .. k-2
            for (int v = 0; v < steps - 1; ++v) {
              const uint32_t o = (h0[u] >> (2 * v)) & 3u;
              va = P.keep * va;
              vb = P.keep * vb;
              if (o == (uint32_t)kGroupA) va = va + P.dtau;
              if (o == (uint32_t)kGroupB) vb = vb + P.dtau;
            }
          }
          va = P.keep * va;
          vb = P.keep * vb;
          if (nc == kGroupA) va = va + P.dtau;
          if (nc == kGroupB) vb = vb + P.dtau;
        }
        {
          const int gx = x0 + ix[u], gy = y0 + iy[u];
          const size_t gi = (size_t)gy * W + gx;
          P.code_out[gi] = (uint8_t)nc;
          P.id_out[gi] = nid;
          if (MODE != kModeLem) {
            P.tau_out[gi] = va;
            P.tau_out[plane + gi] = vb;
          }
          n_a += nc == kGroupA;
          n_b += nc == kGroupB;
          c_a += nc == kGroupA && gx >= W - P.cross_b;
          c_b += nc == kGroupB && gx < P.cross_a;
        }
      }
    }
    }
    if (threadIdx.x == 0) cnt[5] = 0u;  // the next step's list (read by everyone before the resolve barrier)
    if (!final_step) {
      __syncthreads();  // the commit's key reads and LDS writes before the next step's clear and list
      clear_claims(j + 1);
      list_agents(j + 1);
      __syncthreads();
    }
  }

  if (last) {
    // one LDS atomic per wave after a cross-lane sum
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      n_a += __shfl_xor(n_a, off);
      n_b += __shfl_xor(n_b, off);
      c_a += __shfl_xor(c_a, off);
      c_b += __shfl_xor(c_b, off);
      moved += __shfl_xor(moved, off);
    }
    if (lane == 0) {
      atomicAdd(&cnt[0], n_a);
      atomicAdd(&cnt[1], n_b);
      atomicAdd(&cnt[2], c_a);
      atomicAdd(&cnt[3], c_b);
      atomicAdd(&cnt[4], moved);
    }
    __syncthreads();
    if (threadIdx.x < kTileStatFields) P.tile_stats[(size_t)tile * kTileStatFields + threadIdx.x] = cnt[threadIdx.x];
  }
}

template <int MODE, int S>
hipError_t launch_range_mode(const RangeScenario& P, int threads, int steps, int last, hipStream_t s) {
  const size_t lds = RangeLayout{P.TX, P.TY, P.S, P.M, steps, MODE != kModeLem}.bytes();
  static bool attr_done = false;
  if (!attr_done) {
    (void)hipFuncSetAttribute((const void*)range_kernel<MODE, S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              max_dynamic_lds());
    (void)hipGetLastError();  // an unsupported attribute value must not linger as the last error
    attr_done = true;
  }
  const int ntiles = P.tiles_x * P.tiles_y;
  const int blocks = ((ntiles + 7) / 8) * 8;
  range_kernel<MODE, S><<<blocks, threads, lds, s>>>(P, steps, last);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_range_scan(const RangeScenario& P, int threads, int steps, int last, hipStream_t s) {
  switch (P.S) {
    case 1: return launch_range_mode<MODE, 1>(P, threads, steps, last, s);
    case 2: return launch_range_mode<MODE, 2>(P, threads, steps, last, s);
    case 3: return launch_range_mode<MODE, 3>(P, threads, steps, last, s);
    case 4: return launch_range_mode<MODE, 4>(P, threads, steps, last, s);
    case 5: return launch_range_mode<MODE, 5>(P, threads, steps, last, s);
    case 6: return launch_range_mode<MODE, 6>(P, threads, steps, last, s);
    case 7: return launch_range_mode<MODE, 7>(P, threads, steps, last, s);
    default: return launch_range_mode<MODE, 8>(P, threads, steps, last, s);
  }
}

}  // namespace

hipError_t launch_range(const RangeScenario& P, int mode, int threads, int steps, int last, hipStream_t s) {
  if (threads < 64 || threads > kRangeMaxThreads || threads % 64) return hipErrorInvalidValue;
  if (P.S < 1 || P.S > kRangeMax || P.M < 1 || P.M > P.S || steps < 1) return hipErrorInvalidValue;
  return mode == kModeLem ? launch_range_scan<kModeLem>(P, threads, steps, last, s)
                          : launch_range_scan<kModeAco>(P, threads, steps, last, s);
}

}  // namespace pedsim
