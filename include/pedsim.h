/*
 * pedsim: the per-time-step bi-directional pedestrian update of Dutta, McLeod
 * and Friesen (arXiv 1412.4933) on one MI355X (gfx950), as a C ABI.
 *
 * Two groups walk toward opposite sides of a 2D grid (Sec. III). Each step
 * (Sec. IV.b-d):
 *   request   every agent picks a target: the forward cell if it is empty,
 *             otherwise one empty forward-diagonal or lateral cell chosen by
 *             the Least Effort Model (eq. 1) or by the ACO random-proportional
 *             rule on its group's pheromone (eq. 2);
 *   resolve   every empty cell gathers the neighbours that picked it and
 *             keeps one (scatter-to-gather, Sec. IV.d);
 *   commit    winners move, everybody else stays;
 *   pheromone (ACO) both planes evaporate (eq. 3) and gain a deposit on the
 *             cells their group occupies (eq. 4).
 * A second ACO variant keeps the tour matrix of Sec. IV.a (one tour length
 * per agent, grown by every move) and deposits eq. 5's amount dtau / L_k on
 * the cell an agent enters (sim_attach_tour, sim_step_aco_tour).
 *
 * Frame and encoding
 *   Cell (x, y), x = column 0..W-1, y = row 0..H-1, flat index y*W + x
 *   (row-major, pitch W). Planes:
 *     code  uint8  [H*W]   0 empty, 1 group A (heads +x), 2 group B (heads -x),
 *                          3 wall. Outside the grid counts as wall.
 *     id    uint32 [H*W]   agent number + 1 on cells with code 1 or 2, else 0.
 *                          The agents' ids must be exactly 1..N.
 *     tau   float  [2*H*W] pheromone, plane 0 for group A then plane 1 for B
 *                          (only needed for ACO steps; may be NULL).
 *   Candidates of an agent at (x, y) heading d: F (x+d, y), FD- (x+d, y-1),
 *   FD+ (x+d, y+1), L- (x, y-1), L+ (x, y+1); staying is implicit.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with counter
 * (agent number, step low word, step high word, 0) and key (seed low word,
 * seed high word), so results do not depend on thread order, tile shape or
 * launch configuration. Conflicts go to the lowest (word 0, agent number).
 * Pheromone arithmetic is IEEE binary32 with no fused multiply-add and with
 * subnormals kept, so results are bit-identical to a plain sequential
 * evaluation of the same rules.
 *
 * Ownership: the caller allocates every device buffer (planes and scratch)
 * and keeps it alive while a handle uses it. The library allocates no device
 * memory. A handle is not thread-safe; distinct handles are independent.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream). Step calls are asynchronous and stream-ordered; once the stream
 * has reached the end of a call, the caller's planes hold the state after
 * its last step.
 *
 * Errors: every call returns SIM_OK (0) or a negative SIM_E* code; nothing
 * is thrown or aborted across the ABI. sim_strerror() names a code.
 */
#ifndef PEDSIM_H
#define PEDSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_OK 0
#define SIM_EINVAL (-1)   /* bad argument or parameter */
#define SIM_ESTATE (-2)   /* initial planes are not a valid state */
#define SIM_ESCRATCH (-3) /* scratch buffer missing or too small */
#define SIM_EHIP (-4)     /* a HIP runtime call failed */
#define SIM_ENOTAU (-5)   /* ACO step on a handle created without pheromone */
#define SIM_EFULL (-6)    /* batch has no free slot */
#define SIM_ENOTOUR (-7)  /* tour step on a handle without a tour array */

#define SIM_MODE_LEM 0
#define SIM_MODE_ACO 1
#define SIM_MODE_ACO_TOUR 2

typedef struct sim_handle sim_handle;

/* Parameters of one scenario. */
typedef struct {
  int32_t W, H;      /* grid columns and rows, 1 <= W, H; W*H < 2^31 */
  uint64_t seed;     /* Philox key */
  uint64_t step0;    /* index of the first step to run (0 for a fresh start;
                        the saved step counter when resuming a checkpoint) */
  float rho;         /* evaporation rate, 0 < rho <= 1 (eq. 3) */
  float dtau;        /* deposit per occupied cell per step, finite, >= 0 (eq. 4) */
  int32_t alpha;     /* pheromone exponent of eq. 2, 0..8 */
  int32_t beta;      /* heuristic exponent of eq. 2, 0..8 */
  int32_t cross_a;   /* B has crossed once x <  cross_a, 0..W */
  int32_t cross_b;   /* A has crossed once x >= W - cross_b, 0..W */
} sim_params;

/* Counters of a scenario after its last completed step. */
typedef struct {
  uint64_t step;       /* steps run so far, counting step0 */
  uint64_t agents_a;   /* agents of group A (constant) */
  uint64_t agents_b;   /* agents of group B (constant) */
  uint64_t crossed_a;  /* A agents with x >= W - cross_b (throughput, Sec. VI) */
  uint64_t crossed_b;  /* B agents with x <  cross_a */
  uint64_t moved_last; /* agents that moved in the last step */
} sim_stats_t;

/* Bytes of device scratch a scenario with these parameters needs: a shadow
 * copy of the planes the step kernels ping-pong with (13 bytes per cell:
 * code 1, id 4, both pheromone planes 8) plus per-tile counters, a few
 * 64-bit totals and the order in which the row-lane launches deal out their
 * tiles (three rotations of one word per tile; it changes no result). */
int sim_scratch_bytes(const sim_params* p, size_t* out);

/*
 * Create a handle over caller-owned device planes that hold the initial
 * state (layout above) and a device scratch buffer of at least
 * sim_scratch_bytes(). This is the paper's data-preparation stage
 * (Sec. IV.a): the grid, the agents' groups and positions and the initial
 * pheromone become the state every later step updates. d_tau may be NULL
 * (then only LEM steps are allowed). The planes are validated on the
 * device: codes in 0..3, ids consistent with codes and exactly 1..N,
 * pheromone finite and >= 0; a bad state returns SIM_ESTATE. The initial
 * counters are computed before the call returns. Synchronises `stream`.
 */
int sim_create(const sim_params* p, uint8_t* d_code, uint32_t* d_id, float* d_tau,
               void* d_scratch, size_t scratch_bytes, void* stream, sim_handle** out);

/* Run nsteps (>= 0) Least Effort Model steps (eq. 1), asynchronously. */
int sim_step_lem(sim_handle* h, int32_t nsteps, void* stream);

/* Run nsteps (>= 0) ACO steps (eq. 2 choice, eq. 3 and 4 update),
 * asynchronously; SIM_ENOTAU if the handle has no pheromone planes. */
int sim_step_aco(sim_handle* h, int32_t nsteps, void* stream);

/*
 * Tour variant (eq. 5 with the tour matrix of Sec. IV.a and IV.d). Attach the
 * caller-owned tour array d_tour: float [N], entry k = the tour length of
 * agent k (id k + 1), finite and >= 0 (0 for a fresh start), plus a second
 * caller-owned float [N] buffer d_tour_shadow that the library uses as the
 * other half of its ping-pong. N is the number of agents of the state given
 * to sim_create; with N = 0 both may be NULL. The values are validated on the
 * device (SIM_ESTATE if one is negative or not finite); synchronises
 * `stream`. Attaching again replaces the arrays.
 */
int sim_attach_tour(sim_handle* h, float* d_tour, float* d_tour_shadow, void* stream);

/*
 * Run nsteps (>= 0) steps of the tour variant, asynchronously: requests,
 * resolution and evaporation as in sim_step_aco; a winner's tour length
 * grows by the length of its move (1 for F and L-/L+, fl(sqrt 2) for FD-/FD+,
 * one float addition), and only the cell it enters gains fl(dtau / L_k) with
 * the grown L_k, on its group's plane, after that cell's evaporation
 * (dtau = 1 gives eq. 5's 1/L_k). Once the stream has reached the end of the
 * call, d_tour holds the tour lengths after the last step. SIM_ENOTAU
 * without pheromone planes, SIM_ENOTOUR without an attached tour array.
 */
int sim_step_aco_tour(sim_handle* h, int32_t nsteps, void* stream);

/*
 * Candidate set of every later step on h: n = 5 (F, FD-, FD+, L-, L+; the
 * default) or n = 8, the paper's full neighbourhood (Sec. III) with the
 * backward cells B (x-d, y), BD- (x-d, y-1) and BD+ (x-d, y+1) ranked after
 * the laterals (Sec. IV.b-c): squared distances 9 and 10 to the point two
 * cells ahead give their heuristic weights, the LEM rank order is
 * [FD_s, FD_-s, L_s, L_-s, B, BD_s, BD_-s] with six normal thresholds, and
 * the ACO roulette sums seven weights in the order FD-, FD+, L-, L+, B, BD-,
 * BD+. A tour-variant move to a backward diagonal adds fl(sqrt 2), to B 1.
 * With n = 8 every mode runs on the row-lane engine with the pheromone in
 * LDS (nw = 0). Resets every mode's tiling to that set's default. SIM_EINVAL
 * for other n. Not available in batches.
 */
int sim_set_neighbours(sim_handle* h, int32_t n);

/*
 * Larger scanning and moving ranges (the paper's future work, Sec. VII, which
 * names them without a rule; the rule below widens Sec. III and IV.b-d).
 * Every later sim_step_lem / sim_step_aco on h uses a scanning range
 * `scan` and a moving range `move`, 1 <= move <= scan <= 8:
 *   - the candidates F, FD-, FD+, L-, L+ become rays; along each ray the
 *     agent sees its free run f, the number of consecutive cells next to it
 *     that are inside the grid and empty at the start of the step, at most
 *     `scan`; a ray with f >= 1 is open and is travelled k = min(f, move)
 *     cells; paths may cross, only landing cells are contested;
 *   - an open forward ray is taken without a draw. Otherwise LEM (eq. 1)
 *     scores an open side ray by (f/scan)(Dmin/D), where D is the distance
 *     from its landing cell to the point move+1 cells ahead of the agent
 *     (D^2 = (move+1 - a k)^2 + k^2, a = 1 for a diagonal, 0 for a lateral),
 *     ranks the open side rays by score, highest first, ties in the order
 *     [FD_s, FD_-s, L_s, L_-s], and takes the rank index of the normal draw
 *     of the base rule. ACO (eq. 2) weighs an open side ray by
 *     tau_g(landing cell)^alpha * eta, eta = the float nearest to
 *     (f/scan)^beta D^-beta (sim_range_weights), with the base rule's
 *     roulette, order and all-zero fallback;
 *   - every cell empty at the start of the step goes to the lowest
 *     (Philox word 0, agent number) among the agents landing on it; then
 *     eq. 3 and eq. 4 on every cell, as in the base step.
 * With scan = move = 1 every rule is the base step's, and the results are
 * identical to it. scan = move = 0 returns h to the base step. A step's
 * dependence reaches 2*move + scan cells, so a launch of k steps stages a halo
 * of k times that (sim_set_range_tiling). SIM_EINVAL for other values, on a
 * handle with the eight-neighbour set, and for sim_step_aco_tour while
 * ranges are set (not combined).
 */
int sim_set_ranges(sim_handle* h, int32_t scan, int32_t move);

/* Launch shape of the range step (results never depend on it): tile
 * interiors of cols (16..256) x rows (8..256) cells advanced steps_per_launch
 * (1..4) steps per launch, `threads` per workgroup (multiple of 64, <= 512).
 * With R1 = 2*move + scan (the reach of one step) and k steps per launch, the
 * workgroup keeps in LDS the codes of the interior plus k*R1 cells, the ids
 * (and for ACO both pheromone planes) of the interior plus (k-1)*R1 + 3*move,
 * a request byte and an agent list entry per cell of the interior plus
 * (k-1)*R1 + 2*move, and a 64-bit claim key and a claim count per cell of the
 * interior plus (k-1)*R1 + move. SIM_EINVAL if ranges are not set or the
 * shape does not fit. sim_get_range_tiling writes {cols, rows,
 * steps_per_launch, threads}. */
int sim_set_range_tiling(sim_handle* h, int32_t cols, int32_t rows, int32_t steps_per_launch, int32_t threads);
int sim_get_range_tiling(sim_handle* h, int32_t out[4]);

/* Host-only: the ACO heuristic weights eta of sim_set_ranges for free runs
 * f = 1..8 (entry f-1; 0 for f > scan): diagonal[] for FD rays, lateral[]
 * for L rays. SIM_EINVAL for ranges or beta (0..8) out of bounds. */
int sim_range_weights(int32_t scan, int32_t move, int32_t beta, float diagonal[8], float lateral[8]);

/* Counters after the last completed step; synchronises `stream`. */
int sim_stats(sim_handle* h, sim_stats_t* out, void* stream);

/* Copy the current state (a checkpoint, with the step counter from
 * sim_stats) into caller buffers, device or host: code [H*W], id [H*W],
 * tau [2*H*W] (ignored when NULL or when the handle has no pheromone).
 * Synchronises `stream`. */
int sim_read_state(sim_handle* h, uint8_t* code, uint32_t* id, float* tau, void* stream);

/*
 * Tiling of the step kernel for `mode` (SIM_MODE_*; results never depend on
 * it; the tour variant and the eight-neighbour set accept nw = 0 only): each
 * workgroup of `threads` lanes (multiple of 64, <= 1024) stages a region of
 * `rows` rows in LDS and advances it `steps_per_launch` steps per launch; the
 * tile interior is the region minus 3*steps_per_launch cells on every side
 * and must be at least 16 x 8.
 *   nw = 1 or 2: multi-wave engine, regions of 64*nw columns (rows <= 1023);
 *   nw = 0:      row-lane engine, regions of 64 columns, rows <= 64,
 *                steps_per_launch <= 8, threads <= 512;
 *   nw = 3:      the same engine streaming the pheromone from HBM and
 *                recomputing contest tickets (less LDS per workgroup, so more
 *                workgroups per compute unit on large grids).
 * SIM_EINVAL if the shape is not allowed or does not fit the LDS.
 * sim_get_tiling writes {nw, rows, steps_per_launch, threads} into out[4].
 */
int sim_set_tiling(sim_handle* h, int32_t mode, int32_t nw, int32_t rows, int32_t steps_per_launch,
                   int32_t threads);
int sim_get_tiling(sim_handle* h, int32_t mode, int32_t out[4]);

/*
 * Instrumentation: run nsteps steps of `mode` (a SIM_MODE_* value)
 * exactly as sim_step_* does, but bracket every kernel launch with HIP events
 * recorded on `stream`, and add each kernel kind's elapsed milliseconds into
 * kernel_ms[kind] and its launch count into launches[kind] (arrays of
 * max_kinds >= 2 entries, not cleared): kind 0 is the step kernel, kind 1 the
 * copy back into the caller's planes after an odd number of launches. Kind
 * names come from sim_kernel_name(). Returns the number of kernel kinds or a
 * SIM_E* code. Synchronises.
 */
int sim_step_timed(sim_handle* h, int32_t mode, int32_t nsteps, void* stream, double* kernel_ms,
                   int64_t* launches, int32_t max_kinds);

/* Static name of kernel kind `kind` reported by sim_step_timed ("" if none). */
const char* sim_kernel_name(int32_t kind);

/* Release a handle (not the caller's buffers). NULL is ignored. */
void sim_destroy(sim_handle* h);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): create +
 * nsteps steps of `mode` (SIM_MODE_LEM or SIM_MODE_ACO) + stats in one call,
 * with results identical to sim_create / sim_step_lem or sim_step_aco /
 * sim_stats on the same planes. The caller passes the state planes (layout,
 * validation and errors as sim_create; they hold the state after the last
 * step when the call returns) and a host sim_stats_t; no scratch argument:
 * the shadow planes and counters live in a static device array of the
 * library, SIM_NOALLOC_SCRATCH_BYTES per GPU (allocated when the library is
 * loaded and held until the process ends), so the call makes no hipMalloc,
 * hipFree or other allocation, host or device. SIM_ESCRATCH when the
 * scenario's scratch (sim_scratch_bytes) exceeds that size: about 2.5M cells.
 * Every call on a GPU shares that GPU's array: calls within one process are
 * serialised per device by a lock, and the array keeps the last call's
 * contents (each call clears what it needs at zero itself). Synchronises
 * `stream`.
 */
#define SIM_NOALLOC_SCRATCH_BYTES (32u << 20)
int sim_run_noalloc(const sim_params* p, int32_t mode, uint8_t* d_code, uint32_t* d_id, float* d_tau,
                    int32_t nsteps, void* stream, sim_stats_t* out);

/*
 * Batched form: many independent scenarios (any sizes; LEM, ACO or the tour
 * variant each)
 * advanced together by one persistent kernel per launch, whose work items are
 * (scenario, tile) pairs claimed from a counter; a call's launch sequence is
 * captured once in a hipGraph and replayed. Every scenario's results are
 * bit-identical to running it alone through sim_step_lem / sim_step_aco /
 * sim_step_aco_tour.
 */
typedef struct sim_batch sim_batch;

/* Bytes of device workspace a batch of `capacity` (1..65535) scenarios needs. */
int sim_batch_workspace_bytes(int32_t capacity, size_t* out);

/* Create an empty batch over a caller-owned device workspace. The batch
 * also holds a small pinned host staging buffer of its own. */
int sim_batch_create(int32_t capacity, void* d_workspace, size_t workspace_bytes, sim_batch** out);

/* Add a scenario: same planes, scratch (sim_scratch_bytes) and validation as
 * sim_create; mode (SIM_MODE_LEM / SIM_MODE_ACO / SIM_MODE_ACO_TOUR) is fixed
 * for the scenario.
 * Writes its slot index. SIM_EFULL when no slot is free. Synchronises. */
int sim_batch_add(sim_batch* b, const sim_params* p, int32_t mode, uint8_t* d_code, uint32_t* d_id, float* d_tau,
                  void* d_scratch, size_t scratch_bytes, void* stream, int32_t* slot);

/* Free a slot; the scenario's buffers are the caller's again once the stream
 * has passed the calls that used them. */
int sim_batch_remove(sim_batch* b, int32_t slot);

/* Advance slot i by steps[i] >= 0 steps, i < n (0 leaves it idle), in shared
 * launches; asynchronous. Every stepped slot's planes hold its new state once
 * the stream has reached the end of the call. */
int sim_batch_step_slots(sim_batch* b, const int32_t* steps, int32_t n, void* stream);

/* Advance every scenario of the batch by nsteps. */
int sim_batch_step(sim_batch* b, int32_t nsteps, void* stream);

/* Counters of one scenario after its last completed step; synchronises. */
int sim_batch_stats(sim_batch* b, int32_t slot, sim_stats_t* out, void* stream);

/* Launch shape (results never depend on it): tiling as for sim_set_tiling,
 * wgs_per_cu persistent workgroups per compute unit (1..32), and whether
 * calls replay captured hipGraphs (1) or launch directly (0).
 * sim_batch_get_tuning writes {nw, rows, steps_per_launch, threads,
 * wgs_per_cu, use_graph}. */
int sim_batch_set_tuning(sim_batch* b, int32_t nw, int32_t rows, int32_t steps_per_launch, int32_t threads,
                         int32_t wgs_per_cu, int32_t use_graph);
int sim_batch_get_tuning(sim_batch* b, int32_t out[6]);

/* Tour arrays of a tour-variant slot (added with mode SIM_MODE_ACO_TOUR),
 * with the meaning, validation and errors of sim_attach_tour. A batch takes
 * tour-variant scenarios only with a tuning of nw = 0 (sim_batch_add returns
 * SIM_EINVAL otherwise), and its later tunings must leave room for the tour
 * lengths in LDS (once a tour-variant scenario has been added, the batch
 * keeps that room for its lifetime). */
int sim_batch_attach_tour(sim_batch* b, int32_t slot, float* d_tour, float* d_tour_shadow, void* stream);

/* Candidate set of every scenario of the batch (see sim_set_neighbours):
 * n = 5 (default) or 8. With 8 the batch runs the row-lane engine with the
 * pheromone in LDS (nw = 0); the call resets the tuning to that set's
 * default. SIM_EINVAL for other n or a resident scenario whose geometry
 * does not fit. */
int sim_batch_set_neighbours(sim_batch* b, int32_t n);

/* Release the batch (not the caller's buffers). NULL is ignored. */
void sim_batch_destroy(sim_batch* b);

/* Static text for a SIM_* code. */
const char* sim_strerror(int code);

/* Details of the most recent SIM_EHIP on the calling thread: the failing HIP
 * call, its error string and code ("" if none yet). Valid until the next
 * failing call on the same thread. */
const char* sim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PEDSIM_H */
