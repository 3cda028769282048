/*
 * Plain CPU oracle for the bi-directional pedestrian update of Dutta, McLeod
 * and Friesen, "GPU accelerated Nature Inspired Methods for Modelling Large
 * Scale Bi-Directional Pedestrian Movement" (arXiv 1412.4933).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct reference
 * that the HIP library is checked against. Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load it. It shares no code, header,
 * table or constant with the HIP library.
 *
 * Every step follows the paper's order on the snapshot of time t:
 *   1. request  (tour construction, Sec. III and Sec. IV.b-c): every agent
 *      picks one target cell;
 *   2. resolve  (scatter-to-gather, Sec. IV.d): every cell that is empty at t
 *      looks at the neighbours that picked it and keeps exactly one;
 *   3. commit   (Sec. IV.d): winners move, everyone else stays;
 *   4. pheromone (ACO only; eq. 3 then eq. 4, Sec. IV.d): every cell of both
 *      planes evaporates, then gains the deposit if its group stands on it.
 * A second ACO variant (mode 2) keeps the paper's tour matrix (Sec. IV.a):
 * every move adds its length to the agent's tour length L_k, and the deposit
 * of eq. 4 becomes eq. 5's amount, dtau / L_k, on the cell the agent entered.
 *
 * Readings taken where the paper is silent (each listed in the design notes):
 *   - frame: x = column, y = row; group A (code 1) heads +x, group B (code 2)
 *     heads -x; code 3 is a wall; outside the grid counts as wall.
 *   - candidates: forward F=(x+d,y), forward diagonals FD-=(x+d,y-1) and
 *     FD+=(x+d,y+1), laterals L-=(x,y-1) and L+=(x,y+1); staying is implicit.
 *     With neighbours = 8 (the paper's full neighbourhood, Sec. III) also
 *     backward B=(x-d,y) and the backward diagonals BD-=(x-d,y-1) and
 *     BD+=(x-d,y+1), ranked after the laterals (Sec. IV.b-c); otherwise the
 *     backward cells are left out.
 *   - "empty" means code 0 in the snapshot of time t: a cell vacated in step
 *     t can only be entered in step t+1.
 *   - forward first: an empty F is taken without further calculation
 *     (Sec. III, Sec. IV.c).
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 *     counter (agent k, t low word, t high word, 0) and key (seed low word,
 *     seed high word); words r0 = conflict ticket, r1 = choice, r2 = side bit.
 *   - distance table (constant, Sec. IV.a-b): squared distance from each
 *     candidate to the point two cells ahead: F 1, FD 2, L 5, B 9, BD 10, so
 *     that F is nearest, the two diagonals tie (Sec. IV.b) and the backward
 *     cells come last. eta = 1/D, and the heuristic weight eta^beta is the
 *     correctly rounded float of D2^(-beta/2).
 *   - LEM (eq. 1, Sec. II.A and IV.c): the empty candidates are ranked by
 *     distance, the two members of a symmetric pair in an order drawn from
 *     bit 0 of r2 (set: the +y side first). z ~ N(0,1) from r1, negatives go
 *     to 0, the index is round-half-up(z) clamped to the last candidate:
 *     index = #{j : r1 >= T_j}, T_j = ceil(2^32 * Phi(j + 1/2)).
 *   - ACO (eq. 2 with alpha, beta, Sec. II.B and IV.c): weights
 *     w_i = tau_g(c_i)^alpha * eta_i^beta over [FD-, FD+, L-, L+] (then
 *     [B, BD-, BD+] with eight neighbours; 0 when the candidate is not
 *     empty), tau_g the agent's own group's plane, summed left to right;
 *     roulette with u = (r1 >> 8) * 2^-24 against running float sums; when
 *     every weight is 0 the LEM rule is used with the same words.
 *   - conflict winner (Sec. IV.d picks one requester uniformly): the lowest
 *     (r0, k) among the requesters.
 *   - deposit (eq. 4 with a constant amount): dtau on every cell occupied by
 *     the group after the commit; keep = fl(1 - rho).
 *   - tour variant (eq. 5, Sec. IV.a and IV.d): the tour matrix holds one
 *     float per agent (index k); a move adds the distance between the two
 *     cell centres, 1 for F and L-/L+ and fl(sqrt 2) for FD-/FD+, by one
 *     float addition; the cell the agent enters gains fl(dtau / L_k) with the
 *     increased L_k (dtau = 1 gives eq. 5's 1/L_k), after its evaporation;
 *     agents that stay deposit nothing.
 *   - larger scanning and moving ranges (oracle_step_range): see the block
 *     before that function.
 * All float arithmetic is IEEE binary32, one operation at a time, without
 * contraction into fused multiply-adds (built with -ffp-contract=off) and
 * with subnormals kept.
 *
 * Threads: the same source builds twice, plainly (one thread; the OpenMP
 * pragmas are ignored) and with -fopenmp. Every parallel loop below runs over
 * cells whose iterations write disjoint entries: a request is written only at
 * its agent's cell; a cell that is empty at t is the only one that writes
 * itself and the source cell of its winner (a source is never empty at t and
 * is won by at most one cell, since its agent made one request); the
 * pheromone update and the counts touch one cell each. Integer sums are
 * exact in any order. So both builds give identical results.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O_EMPTY 0
#define O_A 1
#define O_B 2
#define O_WALL 3

/* request codes: which candidate an agent picked */
#define O_REQ_NONE 0
#define O_REQ_F 1
#define O_REQ_FDM 2
#define O_REQ_FDP 3
#define O_REQ_LM 4
#define O_REQ_LP 5
#define O_REQ_B 6
#define O_REQ_BDM 7
#define O_REQ_BDP 8

typedef struct {
  int32_t W, H;
  uint64_t seed;
  float rho, dtau;
  int32_t alpha, beta;
  int32_t cross_a, cross_b;
  int32_t neighbours; /* 8: all eight neighbours; anything else: no backward cells */
} oracle_params;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 from its published definition: a 4-word counter block goes */
/* through 10 rounds; each round multiplies words 0 and 2 by two fixed odd   */
/* constants, the high halves are xored with the other two words and the     */
/* round key, and the words are permuted; the 2-word key is advanced by two  */
/* Weyl constants between rounds.                                            */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t mul0 = 0xD2511F53u, mul1 = 0xCD9E8D57u;
  const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  int round;
  for (round = 0; round < 10; ++round) {
    uint64_t p0, p1;
    uint32_t hi0, lo0, hi1, lo1;
    if (round > 0) {
      k0 += weyl0;
      k1 += weyl1;
    }
    p0 = (uint64_t)mul0 * (uint64_t)x0;
    p1 = (uint64_t)mul1 * (uint64_t)x2;
    hi0 = (uint32_t)(p0 >> 32);
    lo0 = (uint32_t)p0;
    hi1 = (uint32_t)(p1 >> 32);
    lo1 = (uint32_t)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* The four words an agent draws in step t. */
static void agent_words(uint64_t seed, uint64_t t, uint32_t k, uint32_t w[4]) {
  uint32_t ctr[4], key[2];
  ctr[0] = k;
  ctr[1] = (uint32_t)t;
  ctr[2] = (uint32_t)(t >> 32);
  ctr[3] = 0;
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  oracle_philox4x32_10(ctr, key, w);
}

/* LEM thresholds T_j = ceil(2^32 * Phi(j + 1/2)), j = 0..5, with Phi the
 * standard normal CDF: Phi(0.5) = 0.69146246127..., Phi(1.5) = 0.93319279873...,
 * Phi(2.5) = 0.99379033467..., Phi(3.5) = 0.99976737092..., Phi(4.5) =
 * 0.99999660232..., Phi(5.5) = 0.99999998101... */
static const uint32_t lem_threshold[6] = {2969808658u, 4008032552u, 4268296987u,
                                          4293968162u, 4294952704u, 4294967215u};

void oracle_lem_thresholds(uint32_t out[6]) {
  int j;
  for (j = 0; j < 6; ++j) out[j] = lem_threshold[j];
}

/* Squared distances from a candidate to the point two cells ahead. */
#define D2_FORWARD 1.0
#define D2_DIAGONAL 2.0
#define D2_LATERAL 5.0
#define D2_BACKWARD 9.0
#define D2_BACK_DIAGONAL 10.0

/* eta^beta = D2^(-beta/2), rounded to float. */
static float heuristic_weight(double d2, int beta) {
  return (float)pow(d2, -0.5 * (double)beta);
}

void oracle_heuristic_weights(int32_t beta, float out[5]) {
  out[0] = heuristic_weight(D2_FORWARD, beta);
  out[1] = heuristic_weight(D2_DIAGONAL, beta);
  out[2] = heuristic_weight(D2_LATERAL, beta);
  out[3] = heuristic_weight(D2_BACKWARD, beta);
  out[4] = heuristic_weight(D2_BACK_DIAGONAL, beta);
}

/* Number of side candidates (all but F): 4, or 7 with eight neighbours. */
static int side_count(const oracle_params *p) { return p->neighbours == 8 ? 7 : 4; }

static int inside(const oracle_params *p, int x, int y) {
  return x >= 0 && x < p->W && y >= 0 && y < p->H;
}

static int free_cell(const oracle_params *p, const uint8_t *code, int x, int y) {
  if (!inside(p, x, y)) return 0;
  return code[(size_t)y * (size_t)p->W + (size_t)x] == O_EMPTY;
}

static int heading(int group) { return group == O_A ? 1 : -1; }

/* Target of request `r` for an agent at (x, y) heading d. */
static void target_of(int r, int x, int y, int d, int *tx, int *ty) {
  *tx = x;
  *ty = y;
  switch (r) {
    case O_REQ_F: *tx = x + d; break;
    case O_REQ_FDM: *tx = x + d; *ty = y - 1; break;
    case O_REQ_FDP: *tx = x + d; *ty = y + 1; break;
    case O_REQ_LM: *ty = y - 1; break;
    case O_REQ_LP: *ty = y + 1; break;
    case O_REQ_B: *tx = x - d; break;
    case O_REQ_BDM: *tx = x - d; *ty = y - 1; break;
    case O_REQ_BDP: *tx = x - d; *ty = y + 1; break;
    default: break;
  }
}

/* LEM choice among the side candidates, eq. (1) with the normal draw.
 * avail[i] refers to request O_REQ_FDM + i (FD-, FD+, L-, L+, B, BD-, BD+);
 * the first `sides` of them exist. */
static int lem_choice(const int avail[7], int sides, uint32_t r1, uint32_t r2) {
  static const int minus_first[7] = {O_REQ_FDM, O_REQ_FDP, O_REQ_LM, O_REQ_LP,
                                     O_REQ_B, O_REQ_BDM, O_REQ_BDP};
  static const int plus_first[7] = {O_REQ_FDP, O_REQ_FDM, O_REQ_LP, O_REQ_LM,
                                    O_REQ_B, O_REQ_BDP, O_REQ_BDM};
  const int *order = (r2 & 1u) ? plus_first : minus_first;
  int ranked[7];
  int n = 0, i, index;
  for (i = 0; i < sides; ++i) {
    int r = order[i];
    if (avail[r - O_REQ_FDM]) ranked[n++] = r;
  }
  if (n == 0) return O_REQ_NONE;
  index = 0;
  for (i = 0; i < sides - 1; ++i)
    if (r1 >= lem_threshold[i]) index += 1;
  if (index > n - 1) index = n - 1;
  return ranked[index];
}

/* ACO choice among the side candidates, eq. (2): roulette on
 * tau^alpha * eta^beta. tau[i] is the group's pheromone on candidate i
 * (FD-, FD+, L-, L+, B, BD-, BD+), eta[i] its heuristic weight. */
static int aco_choice(const int avail[7], int sides, const float tau[7], const float eta[7],
                      int alpha, uint32_t r1, uint32_t r2) {
  float w[7];
  float sum, u, target, running;
  int i, last;
  for (i = 0; i < sides; ++i) {
    if (avail[i]) {
      float power = 1.0f;
      int a;
      if (alpha > 0) {
        power = tau[i];
        for (a = 1; a < alpha; ++a) power = power * tau[i];
      }
      w[i] = power * eta[i];
    } else {
      w[i] = 0.0f;
    }
  }
  sum = w[0];
  for (i = 1; i < sides; ++i) sum = sum + w[i];
  if (sum == 0.0f) return lem_choice(avail, sides, r1, r2);
  u = (float)(r1 >> 8) * 0x1p-24f;
  target = u * sum;
  running = 0.0f;
  last = -1;
  for (i = 0; i < sides; ++i) {
    running = running + w[i];
    if (w[i] > 0.0f) {
      last = i;
      if (target < running) return O_REQ_FDM + i;
    }
  }
  return O_REQ_FDM + last;
}

/* Request of the agent standing on (x, y) at step t. */
static int request_of(const oracle_params *p, int mode, uint64_t t, const uint8_t *code,
                      const uint32_t *id, const float *tau_a, const float *tau_b,
                      const float eta[7], int x, int y) {
  size_t c = (size_t)y * (size_t)p->W + (size_t)x;
  int g = code[c];
  int d = heading(g);
  int sides = side_count(p);
  int avail[7];
  int side_x[7], side_y[7];
  uint32_t w[4];
  int i, any = 0;
  if (free_cell(p, code, x + d, y)) return O_REQ_F;
  for (i = 0; i < sides; ++i) {
    target_of(O_REQ_FDM + i, x, y, d, &side_x[i], &side_y[i]);
    avail[i] = free_cell(p, code, side_x[i], side_y[i]);
    any = any || avail[i];
  }
  if (!any) return O_REQ_NONE;
  agent_words(p->seed, t, id[c] - 1u, w);
  if (mode == 0) return lem_choice(avail, sides, w[1], w[2]);
  {
    const float *plane = (g == O_A) ? tau_a : tau_b;
    float tau[7];
    for (i = 0; i < sides; ++i)
      tau[i] = avail[i] ? plane[(size_t)side_y[i] * (size_t)p->W + (size_t)side_x[i]] : 0.0f;
    return aco_choice(avail, sides, tau, eta, p->alpha, w[1], w[2]);
  }
}

/*
 * One step in place. mode 0 = LEM, 1 = ACO, 2 = ACO with the tour matrix
 * (tau planes required for 1 and 2, tour[N] for 2).
 * req_out (optional, H*W bytes): each agent's request code, 0 elsewhere.
 * win_out (optional, H*W bytes): for each cell empty at t that received an
 *   agent, 1 + (dy+1)*3 + (dx+1) where (dx, dy) points from the cell to the
 *   winner's old cell; 0 elsewhere.
 * Returns the number of agents that moved, or -1 on allocation failure.
 */
static int64_t step_any(const oracle_params *p, int32_t mode, uint64_t t, uint8_t *code,
                        uint32_t *id, float *tau_a, float *tau_b, float *tour,
                        uint8_t *req_out, uint8_t *win_out) {
  const int W = p->W, H = p->H;
  const size_t cells = (size_t)W * (size_t)H;
  uint8_t *req = (uint8_t *)calloc(cells, 1);
  uint8_t *new_code = (uint8_t *)malloc(cells);
  uint32_t *new_id = (uint32_t *)malloc(cells * sizeof(uint32_t));
  uint8_t *entered = (uint8_t *)calloc(cells, 1); /* mode 2: group that entered the cell */
  float eta[7];
  const float diagonal_step = (float)sqrt(2.0);
  int64_t moved = 0;
  int x, y;
  if (!req || !new_code || !new_id || !entered) {
    free(req);
    free(new_code);
    free(new_id);
    free(entered);
    return -1;
  }
  eta[0] = eta[1] = heuristic_weight(D2_DIAGONAL, p->beta);
  eta[2] = eta[3] = heuristic_weight(D2_LATERAL, p->beta);
  eta[4] = heuristic_weight(D2_BACKWARD, p->beta);
  eta[5] = eta[6] = heuristic_weight(D2_BACK_DIAGONAL, p->beta);
  if (win_out) memset(win_out, 0, cells);

  /* 1. request, every agent on the snapshot of time t */
#pragma omp parallel for private(x) schedule(static)
  for (y = 0; y < H; ++y)
    for (x = 0; x < W; ++x) {
      size_t c = (size_t)y * W + x;
      if (code[c] == O_A || code[c] == O_B)
        req[c] = (uint8_t)request_of(p, mode, t, code, id, tau_a, tau_b, eta, x, y);
    }

  /* 2.+3. resolve every cell empty at t, then commit into fresh planes */
  memcpy(new_code, code, cells);
  memcpy(new_id, id, cells * sizeof(uint32_t));
#pragma omp parallel for private(x) reduction(+ : moved) schedule(static)
  for (y = 0; y < H; ++y)
    for (x = 0; x < W; ++x) {
      size_t c = (size_t)y * W + x;
      int dx, dy, have = 0, best_dx = 0, best_dy = 0;
      uint32_t best_ticket = 0, best_k = 0;
      if (code[c] != O_EMPTY) continue;
      for (dy = -1; dy <= 1; ++dy)
        for (dx = -1; dx <= 1; ++dx) {
          int nx = x + dx, ny = y + dy, tx, ty;
          size_t n;
          if ((dx == 0 && dy == 0) || !inside(p, nx, ny)) continue;
          n = (size_t)ny * W + nx;
          if (code[n] != O_A && code[n] != O_B) continue;
          if (req[n] == O_REQ_NONE) continue;
          target_of(req[n], nx, ny, heading(code[n]), &tx, &ty);
          if (tx != x || ty != y) continue;
          {
            uint32_t w[4];
            uint32_t k = id[n] - 1u;
            agent_words(p->seed, t, k, w);
            if (!have || w[0] < best_ticket || (w[0] == best_ticket && k < best_k)) {
              have = 1;
              best_ticket = w[0];
              best_k = k;
              best_dx = dx;
              best_dy = dy;
            }
          }
        }
      if (have) {
        size_t n = (size_t)(y + best_dy) * W + (x + best_dx);
        new_code[c] = code[n];
        new_id[c] = id[n];
        new_code[n] = O_EMPTY;
        new_id[n] = 0;
        moved += 1;
        if (mode == 2) {
          /* the tour grows by the length of this move */
          const float len = (best_dx != 0 && best_dy != 0) ? diagonal_step : 1.0f;
          tour[best_k] = tour[best_k] + len;
          entered[c] = code[n];
        }
        if (win_out) win_out[c] = (uint8_t)(1 + (best_dy + 1) * 3 + (best_dx + 1));
      }
    }
  if (req_out) memcpy(req_out, req, cells);
  memcpy(code, new_code, cells);
  memcpy(id, new_id, cells * sizeof(uint32_t));

  /* 4. pheromone: evaporation (eq. 3) then deposit (eq. 4), both planes */
  if (mode == 1) {
    float rho = p->rho;
    float keep = 1.0f - rho;
    size_t c;
#pragma omp parallel for schedule(static)
    for (c = 0; c < cells; ++c) {
      float va = keep * tau_a[c];
      float vb = keep * tau_b[c];
      if (code[c] == O_A) va = va + p->dtau;
      if (code[c] == O_B) vb = vb + p->dtau;
      tau_a[c] = va;
      tau_b[c] = vb;
    }
  }

  /* 4'. tour variant: evaporation (eq. 3), then eq. 5's deposit on entered cells */
  if (mode == 2) {
    float rho = p->rho;
    float keep = 1.0f - rho;
    size_t c;
#pragma omp parallel for schedule(static)
    for (c = 0; c < cells; ++c) {
      float evaporated_a = keep * tau_a[c];
      float evaporated_b = keep * tau_b[c];
      if (entered[c] == O_A) evaporated_a = evaporated_a + p->dtau / tour[id[c] - 1u];
      if (entered[c] == O_B) evaporated_b = evaporated_b + p->dtau / tour[id[c] - 1u];
      tau_a[c] = evaporated_a;
      tau_b[c] = evaporated_b;
    }
  }
  free(req);
  free(new_code);
  free(new_id);
  free(entered);
  return moved;
}

/* ------------------------------------------------------------------------ */
/* Larger scanning and moving ranges (the paper's future work, Sec. VII).     */
/* Scanning range S and moving range M (1 <= M <= S): the five candidate      */
/* directions become rays. Along each ray the agent sees the free run f, the  */
/* number of consecutive cells next to it that are inside the grid and empty  */
/* at t (at most S); an open ray (f >= 1) is travelled k = min(f, M) cells.   */
/* The distance of Sec. IV.a-b is taken from the landing cell to the point    */
/* M+1 cells ahead; LEM (eq. 1) reads the occupancy of a candidate as the     */
/* blocked share of its scanned ray, 1 - f/S, and ACO (eq. 2) weighs the      */
/* pheromone of the landing cell with the heuristic (f/S)/D. With S = M = 1   */
/* every rule reduces to the steps above.                                     */
/* ------------------------------------------------------------------------ */

/* Ray r (0 F, 1 FD-, 2 FD+, 3 L-, 4 L+) of an agent heading d: its forward
 * component a (1 or 0), lateral component b, and unit step (ux, uy). */
static void range_ray(int r, int d, int *a, int *b, int *ux, int *uy) {
  static const int fwd[5] = {1, 1, 1, 0, 0};
  static const int lat[5] = {0, -1, 1, -1, 1};
  *a = fwd[r];
  *b = lat[r];
  *ux = d * fwd[r];
  *uy = lat[r];
}

/* Free run along the unit step (ux, uy) from (x, y), at most S cells. */
static int free_run(const oracle_params *p, const uint8_t *code, int x, int y, int ux, int uy,
                    int S) {
  int j = 0;
  while (j < S && free_cell(p, code, x + (j + 1) * ux, y + (j + 1) * uy)) j += 1;
  return j;
}

/* Squared distance from the cell k steps along a ray with components (a, b)
 * to the point M+1 cells ahead of the agent. */
static int64_t range_d2(int a, int b, int k, int M) {
  int64_t dx = (int64_t)(M + 1) - (int64_t)a * k;
  int64_t dy = (int64_t)b * k;
  return dx * dx + dy * dy;
}

/* eta^beta of a side ray with forward component a and free run f >= 1:
 * (f/S)^beta * D2^(-beta/2), rounded to float. */
static float range_weight(int a, int f, int S, int M, int beta) {
  int k = f < M ? f : M;
  double d2 = (double)range_d2(a, 1, k, M);
  return (float)(pow((double)f / (double)S, (double)beta) * pow(d2, -0.5 * (double)beta));
}

void oracle_range_weights(int32_t S, int32_t M, int32_t beta, float out_diagonal[8],
                          float out_lateral[8]) {
  int f;
  for (f = 1; f <= 8; ++f) {
    out_diagonal[f - 1] = f <= S ? range_weight(1, f, S, M, beta) : 0.0f;
    out_lateral[f - 1] = f <= S ? range_weight(0, f, S, M, beta) : 0.0f;
  }
}

/* LEM with ranges: open side rays (f[i] >= 1 for side ray i = 1..4) ranked by
 * C = (f/S)(Dmin/D), highest first, ties in the order [FD_s, FD_-s, L_s, L_-s];
 * returns the chosen ray (1..4), or 0 if none is open. */
static int range_lem_choice(const int f[5], const int64_t d2[5], uint32_t r1, uint32_t r2) {
  const int minus_first[4] = {1, 2, 3, 4};
  const int plus_first[4] = {2, 1, 4, 3};
  const int *order = (r2 & 1u) ? plus_first : minus_first;
  int ranked[4];
  int n = 0, i, j, index;
  for (i = 0; i < 4; ++i) {
    int r = order[i];
    if (f[r] < 1) continue;
    /* insertion: move past every ranked ray with a strictly higher score */
    j = n;
    while (j > 0) {
      int q = ranked[j - 1];
      /* C_q < C_r  <=>  f_q^2 D2_r < f_r^2 D2_q */
      if ((int64_t)f[q] * f[q] * d2[r] < (int64_t)f[r] * f[r] * d2[q]) {
        ranked[j] = q;
        j -= 1;
      } else {
        break;
      }
    }
    ranked[j] = r;
    n += 1;
  }
  if (n == 0) return 0;
  index = 0;
  for (i = 0; i < 3; ++i)
    if (r1 >= lem_threshold[i]) index += 1;
  if (index > n - 1) index = n - 1;
  return ranked[index];
}

/* ACO with ranges: roulette over the side rays 1..4 with weights
 * tau(landing cell)^alpha * eta^beta; all-zero weights fall back to LEM. */
static int range_aco_choice(const int f[5], const int64_t d2[5], const float tau[5],
                            const float eta[5], int alpha, uint32_t r1, uint32_t r2) {
  float w[5];
  float sum, u, target, running;
  int i, last;
  for (i = 1; i <= 4; ++i) {
    if (f[i] >= 1) {
      float power = 1.0f;
      int a;
      if (alpha > 0) {
        power = tau[i];
        for (a = 1; a < alpha; ++a) power = power * tau[i];
      }
      w[i] = power * eta[i];
    } else {
      w[i] = 0.0f;
    }
  }
  sum = w[1];
  for (i = 2; i <= 4; ++i) sum = sum + w[i];
  if (sum == 0.0f) return range_lem_choice(f, d2, r1, r2);
  u = (float)(r1 >> 8) * 0x1p-24f;
  target = u * sum;
  running = 0.0f;
  last = -1;
  for (i = 1; i <= 4; ++i) {
    running = running + w[i];
    if (w[i] > 0.0f) {
      last = i;
      if (target < running) return i;
    }
  }
  return last;
}

/*
 * One step with scanning range S and moving range M, in place; mode 0 = LEM,
 * 1 = ACO (tau planes required). req_out (optional, H*W bytes): each agent's
 * ray + 1 (1 F, 2 FD-, 3 FD+, 4 L-, 5 L+) or 0; len_out (optional, H*W
 * bytes): the cells it asked to travel. Returns the number of agents that
 * moved, -1 on allocation failure, -2 on bad ranges.
 */
int64_t oracle_step_range(const oracle_params *p, int32_t mode, uint64_t t, int32_t S, int32_t M,
                          uint8_t *code, uint32_t *id, float *tau_a, float *tau_b,
                          uint8_t *req_out, uint8_t *len_out) {
  const int W = p->W, H = p->H;
  const size_t cells = (size_t)W * (size_t)H;
  uint8_t *ray, *len, *new_code;
  uint32_t *new_id;
  int64_t moved = 0;
  int x, y;
  if (S < 1 || S > 8 || M < 1 || M > S || (mode != 0 && mode != 1)) return -2;
  ray = (uint8_t *)calloc(cells, 1);
  len = (uint8_t *)calloc(cells, 1);
  new_code = (uint8_t *)malloc(cells);
  new_id = (uint32_t *)malloc(cells * sizeof(uint32_t));
  if (!ray || !len || !new_code || !new_id) {
    free(ray);
    free(len);
    free(new_code);
    free(new_id);
    return -1;
  }

  /* 1. request: every agent on the snapshot of time t */
#pragma omp parallel for private(x) schedule(static)
  for (y = 0; y < H; ++y)
    for (x = 0; x < W; ++x) {
      size_t c = (size_t)y * W + x;
      int g = code[c], d, r, choice, any = 0;
      int f[5], a[5], b[5], ux[5], uy[5];
      int64_t d2[5];
      float eta[5], tau[5];
      uint32_t w[4];
      if (g != O_A && g != O_B) continue;
      d = heading(g);
      for (r = 0; r < 5; ++r) {
        range_ray(r, d, &a[r], &b[r], &ux[r], &uy[r]);
        f[r] = free_run(p, code, x, y, ux[r], uy[r], S);
        d2[r] = range_d2(a[r], b[r], f[r] < M ? f[r] : M, M);
        if (r > 0 && f[r] >= 1) any = 1;
      }
      if (f[0] >= 1) {
        choice = 0; /* forward first */
      } else {
        if (!any) continue;
        agent_words(p->seed, t, id[c] - 1u, w);
        if (mode == 0) {
          choice = range_lem_choice(f, d2, w[1], w[2]);
        } else {
          const float *plane = (g == O_A) ? tau_a : tau_b;
          for (r = 1; r <= 4; ++r) {
            eta[r] = 0.0f;
            tau[r] = 0.0f;
            if (f[r] >= 1) {
              int k = f[r] < M ? f[r] : M;
              eta[r] = range_weight(a[r], f[r], S, M, p->beta);
              tau[r] = plane[(size_t)(y + k * uy[r]) * W + (size_t)(x + k * ux[r])];
            }
          }
          choice = range_aco_choice(f, d2, tau, eta, p->alpha, w[1], w[2]);
        }
      }
      ray[c] = (uint8_t)(choice + 1);
      len[c] = (uint8_t)(f[choice] < M ? f[choice] : M);
    }

  /* 2.+3. resolve every cell empty at t among the agents (up to M cells
   * away) landing on it, then commit into fresh planes */
  memcpy(new_code, code, cells);
  memcpy(new_id, id, cells * sizeof(uint32_t));
#pragma omp parallel for private(x) reduction(+ : moved) schedule(static)
  for (y = 0; y < H; ++y)
    for (x = 0; x < W; ++x) {
      size_t c = (size_t)y * W + x;
      int dx, dy, have = 0;
      size_t best_n = 0;
      uint32_t best_ticket = 0, best_k = 0;
      if (code[c] != O_EMPTY) continue;
      for (dy = -M; dy <= M; ++dy)
        for (dx = -M; dx <= M; ++dx) {
          int nx = x + dx, ny = y + dy, a, b, ux, uy, k;
          size_t n;
          if ((dx == 0 && dy == 0) || !inside(p, nx, ny)) continue;
          n = (size_t)ny * W + nx;
          if (code[n] != O_A && code[n] != O_B) continue;
          if (ray[n] == 0) continue;
          range_ray(ray[n] - 1, heading(code[n]), &a, &b, &ux, &uy);
          k = len[n];
          if (nx + k * ux != x || ny + k * uy != y) continue;
          {
            uint32_t w[4];
            uint32_t kk = id[n] - 1u;
            agent_words(p->seed, t, kk, w);
            if (!have || w[0] < best_ticket || (w[0] == best_ticket && kk < best_k)) {
              have = 1;
              best_ticket = w[0];
              best_k = kk;
              best_n = n;
            }
          }
        }
      if (have) {
        new_code[c] = code[best_n];
        new_id[c] = id[best_n];
        new_code[best_n] = O_EMPTY;
        new_id[best_n] = 0;
        moved += 1;
      }
    }
  if (req_out) memcpy(req_out, ray, cells);
  if (len_out) memcpy(len_out, len, cells);
  memcpy(code, new_code, cells);
  memcpy(id, new_id, cells * sizeof(uint32_t));

  /* 4. pheromone: evaporation (eq. 3) then deposit (eq. 4), both planes */
  if (mode == 1) {
    float rho = p->rho;
    float keep = 1.0f - rho;
    size_t c;
#pragma omp parallel for schedule(static)
    for (c = 0; c < cells; ++c) {
      float va = keep * tau_a[c];
      float vb = keep * tau_b[c];
      if (code[c] == O_A) va = va + p->dtau;
      if (code[c] == O_B) vb = vb + p->dtau;
      tau_a[c] = va;
      tau_b[c] = vb;
    }
  }
  free(ray);
  free(len);
  free(new_code);
  free(new_id);
  return moved;
}

int64_t oracle_run_range(const oracle_params *p, int32_t mode, uint64_t t0, int64_t nsteps,
                         int32_t S, int32_t M, uint8_t *code, uint32_t *id, float *tau_a,
                         float *tau_b) {
  int64_t s, moved = 0;
  for (s = 0; s < nsteps; ++s) {
    moved = oracle_step_range(p, mode, t0 + (uint64_t)s, S, M, code, id, tau_a, tau_b, NULL, NULL);
    if (moved < 0) return moved;
  }
  return moved;
}

int64_t oracle_step(const oracle_params *p, int32_t mode, uint64_t t, uint8_t *code,
                    uint32_t *id, float *tau_a, float *tau_b, uint8_t *req_out,
                    uint8_t *win_out) {
  if (mode != 0 && mode != 1) return -1;
  return step_any(p, mode, t, code, id, tau_a, tau_b, NULL, req_out, win_out);
}

/* One step of the tour variant (mode 2); tour[k] is agent k's tour length. */
int64_t oracle_step_tour(const oracle_params *p, uint64_t t, uint8_t *code, uint32_t *id,
                         float *tau_a, float *tau_b, float *tour, uint8_t *req_out,
                         uint8_t *win_out) {
  return step_any(p, 2, t, code, id, tau_a, tau_b, tour, req_out, win_out);
}

/* Crossing and population counts of the current state:
 * out[0] agents in A, out[1] agents in B, out[2] A at x >= W - cross_b,
 * out[3] B at x < cross_a. */
void oracle_counts(const oracle_params *p, const uint8_t *code, uint64_t out[4]) {
  int x, y;
  uint64_t n_a = 0, n_b = 0, crossed_a = 0, crossed_b = 0;
#pragma omp parallel for private(x) reduction(+ : n_a, n_b, crossed_a, crossed_b) schedule(static)
  for (y = 0; y < p->H; ++y)
    for (x = 0; x < p->W; ++x) {
      int g = code[(size_t)y * p->W + x];
      if (g == O_A) {
        n_a += 1;
        if (x >= p->W - p->cross_b) crossed_a += 1;
      } else if (g == O_B) {
        n_b += 1;
        if (x < p->cross_a) crossed_b += 1;
      }
    }
  out[0] = n_a;
  out[1] = n_b;
  out[2] = crossed_a;
  out[3] = crossed_b;
}

/* Threads the OpenMP build uses from now on (n >= 1); returns the number it
 * will use, 1 in the plain build. */
int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* nsteps steps from step t0; returns the moves of the last step (or -1). */
int64_t oracle_run(const oracle_params *p, int32_t mode, uint64_t t0, int64_t nsteps,
                   uint8_t *code, uint32_t *id, float *tau_a, float *tau_b) {
  int64_t s, moved = 0;
  for (s = 0; s < nsteps; ++s) {
    moved = oracle_step(p, mode, t0 + (uint64_t)s, code, id, tau_a, tau_b, NULL, NULL);
    if (moved < 0) return -1;
  }
  return moved;
}

int64_t oracle_run_tour(const oracle_params *p, uint64_t t0, int64_t nsteps, uint8_t *code,
                        uint32_t *id, float *tau_a, float *tau_b, float *tour) {
  int64_t s, moved = 0;
  for (s = 0; s < nsteps; ++s) {
    moved = oracle_step_tour(p, t0 + (uint64_t)s, code, id, tau_a, tau_b, tour, NULL, NULL);
    if (moved < 0) return -1;
  }
  return moved;
}
