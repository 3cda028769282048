// Device-side rules of one step of the bi-directional pedestrian update
// (Dutta, McLeod, Friesen, arXiv 1412.4933): the counter-based random words,
// the Least Effort Model choice (eq. 1) and the ACO random-proportional choice
// (eq. 2). Shared by the single-scenario and the batched kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pedsim {

enum : uint8_t { kEmpty = 0, kGroupA = 1, kGroupB = 2, kWall = 3 };

// Request codes. Side candidates are numbered j = code - kReqFDm:
// j = 0 FD- (x+d, y-1), 1 FD+ (x+d, y+1), 2 L- (x, y-1), 3 L+ (x, y+1).
enum : uint8_t { kReqNone = 0, kReqF = 1, kReqFDm = 2, kReqFDp = 3, kReqLm = 4, kReqLp = 5 };

// Position of a neighbour (dx, dy) as seen from a cell, 1..9 (5 = itself).
__host__ __device__ constexpr int slot_of(int dx, int dy) { return 1 + (dy + 1) * 3 + (dx + 1); }

// Offset of request r for heading d (+1 group A, -1 group B).
__device__ __forceinline__ int req_dx(int r, int d) { return (r >= kReqF && r <= kReqFDp) ? d : 0; }
__device__ __forceinline__ int req_dy(int r) {
  return (r == kReqFDm || r == kReqLm) ? -1 : ((r == kReqFDp || r == kReqLp) ? 1 : 0);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies by fixed odd constants, high halves xored with the
// other words and the round key, the key advanced by two Weyl increments
// between rounds.
struct Words {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // one 32x32->64 product each (a single v_mad_u64_u32): high and low halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words{c0, c1, c2, c3};
}

// The words agent k draws at step t: counter (k, t lo, t hi, 0), key = seed.
__device__ __forceinline__ Words agent_words(uint32_t k, uint64_t t, uint32_t key0, uint32_t key1) {
  return philox4x32_10(k, (uint32_t)t, (uint32_t)(t >> 32), 0u, key0, key1);
}

// z ~ N(0,1) drawn from word w1: z >= j + 1/2 exactly when w1 >= T_j with
// T_j = ceil(2^32 Phi(j + 1/2)) (Phi(0.5) = 0.691462461..., Phi(1.5) =
// 0.933192798..., Phi(2.5) = 0.993790334...).
constexpr uint32_t kNormalCut0 = 2969808658u;
constexpr uint32_t kNormalCut1 = 4008032552u;
constexpr uint32_t kNormalCut2 = 4268296987u;

// LEM (eq. 1): the empty side candidates ranked by distance to the target
// (diagonals before laterals; within each symmetric pair the +y member first
// when bit 0 of w2 is set), index = round-half-up(max(z, 0)) clamped to the
// last one. avail: bit j set when side candidate j is empty. Returns a
// request code (kReqNone when avail == 0).
__device__ __forceinline__ int lem_choose(unsigned avail, uint32_t w1, uint32_t w2) {
  const unsigned flip = w2 & 1u;  // 1: visit j ^ 1 (pair members swapped)
  const int n = __popc(avail);
  int idx = (w1 >= kNormalCut0) + (w1 >= kNormalCut1) + (w1 >= kNormalCut2);
  idx = idx < n - 1 ? idx : n - 1;
  int pick = -1;
#pragma unroll
  for (int rank = 0; rank < 4; ++rank) {
    const int j = rank ^ (int)flip;
    if ((avail >> j) & 1u) {
      if (idx == 0 && pick < 0) pick = j;
      idx -= 1;
    }
  }
  return pick < 0 ? kReqNone : kReqFDm + pick;
}

// ACO (eq. 2): weights tau^alpha * eta^beta on the empty side candidates in
// the order FD-, FD+, L-, L+, summed left to right; u = (w1 >> 8) 2^-24 and
// the first candidate whose running sum exceeds u * sum is taken (the last
// positive one if rounding leaves none). All-zero weights fall back to the
// LEM rule with the same words. Every operation is one binary32 rounding.
__device__ __forceinline__ int aco_choose(unsigned avail, const float tau[4], int alpha,
                                          float eta_diag, float eta_lat, uint32_t w1, uint32_t w2) {
  float w[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float p = 1.0f;
    if (alpha > 0) {
      p = tau[j];
      for (int a = 1; a < alpha; ++a) p = p * tau[j];
    }
    w[j] = ((avail >> j) & 1u) ? p * (j < 2 ? eta_diag : eta_lat) : 0.0f;
  }
  float sum = w[0] + w[1];
  sum = sum + w[2];
  sum = sum + w[3];
  if (sum == 0.0f) return lem_choose(avail, w1, w2);
  const float u = (float)(w1 >> 8) * 0x1p-24f;
  const float target = u * sum;
  float running = 0.0f;
  int last = -1, pick = -1;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    running = running + w[j];
    if (w[j] > 0.0f) {
      last = j;
      if (pick < 0 && target < running) pick = j;
    }
  }
  return kReqFDm + (pick >= 0 ? pick : last);
}

// Eight-neighbour candidate set (Sec. III): side candidates numbered
// j = 0 FD- (x+d, y-1), 1 FD+ (x+d, y+1), 2 L- (x, y-1), 3 L+ (x, y+1),
// 4 B (x-d, y), 5 BD- (x-d, y-1), 6 BD+ (x-d, y+1); the backward cells are
// ranked after the laterals (Sec. IV.b-c). Thresholds T_3..T_5 continue the
// ones above (Phi(3.5) = 0.999767370..., Phi(4.5) = 0.999996602...,
// Phi(5.5) = 0.999999981...).
constexpr uint32_t kNormalCut3 = 4293968162u;
constexpr uint32_t kNormalCut4 = 4294952704u;
constexpr uint32_t kNormalCut5 = 4294967215u;

// LEM over the seven side candidates: ranks [FD_s, FD_-s, L_s, L_-s, B,
// BD_s, BD_-s] (s from bit 0 of w2 as above). Returns the candidate j, or -1
// when avail == 0.
__device__ __forceinline__ int lem_choose7(unsigned avail, uint32_t w1, uint32_t w2) {
  const unsigned flip = w2 & 1u;
  const int n = __popc(avail);
  int idx = (w1 >= kNormalCut0) + (w1 >= kNormalCut1) + (w1 >= kNormalCut2) + (w1 >= kNormalCut3) +
            (w1 >= kNormalCut4) + (w1 >= kNormalCut5);
  idx = idx < n - 1 ? idx : n - 1;
  int pick = -1;
#pragma unroll
  for (int rank = 0; rank < 7; ++rank) {
    const int j = rank < 4 ? (rank ^ (int)flip) : (rank == 4 ? 4 : 5 + ((rank - 5) ^ (int)flip));
    if ((avail >> j) & 1u) {
      if (idx == 0 && pick < 0) pick = j;
      idx -= 1;
    }
  }
  return pick;
}

// ACO over the seven side candidates: weights tau^alpha * eta^beta in the
// order FD-, FD+, L-, L+, B, BD-, BD+ (eta[j] per candidate), summed left to
// right, roulette as in aco_choose; all-zero weights fall back to
// lem_choose7 with the same words. Returns the candidate j.
__device__ __forceinline__ int aco_choose7(unsigned avail, const float tau[7], int alpha, const float eta[7],
                                           uint32_t w1, uint32_t w2) {
  float w[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    float p = 1.0f;
    if (alpha > 0) {
      p = tau[j];
      for (int a = 1; a < alpha; ++a) p = p * tau[j];
    }
    w[j] = ((avail >> j) & 1u) ? p * eta[j] : 0.0f;
  }
  float sum = w[0];
#pragma unroll
  for (int j = 1; j < 7; ++j) sum = sum + w[j];
  if (sum == 0.0f) return lem_choose7(avail, w1, w2);
  const float u = (float)(w1 >> 8) * 0x1p-24f;
  const float target = u * sum;
  float running = 0.0f;
  int last = -1, pick = -1;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    running = running + w[j];
    if (w[j] > 0.0f) {
      last = j;
      if (pick < 0 && target < running) pick = j;
    }
  }
  return pick >= 0 ? pick : last;
}

}  // namespace pedsim
