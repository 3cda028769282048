// C ABI of the single-scenario step (declared in include/pedsim.h).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "pedsim.h"
#include "pedsim_internal.hpp"

using namespace pedsim;

struct sim_handle {
  sim_params p;
  uint8_t* code;
  uint32_t* id;
  float* tau;  // 2*H*W or nullptr
  StepArgs args;
  unsigned long long* totals;  // kStatFields device totals (scratch)
  int commit_blocks;
  uint64_t t;  // index of the next step
};

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t dec, block_stats, totals, total;
  int commit_bx, commit_by;
};

Layout layout_of(const sim_params* p) {
  Layout L;
  const size_t cells = (size_t)p->W * (size_t)p->H;
  L.commit_bx = (p->W + kCommitTX - 1) / kCommitTX;
  L.commit_by = (p->H + kCommitTY - 1) / kCommitTY;
  L.dec = 0;
  L.block_stats = round_up(cells);
  L.totals = L.block_stats + round_up((size_t)L.commit_bx * L.commit_by * kStatFields * sizeof(uint32_t));
  L.total = L.totals + round_up(8 * sizeof(unsigned long long));
  return L;
}

int check_params(const sim_params* p) {
  if (!p) return SIM_EINVAL;
  if (p->W < 1 || p->H < 1) return SIM_EINVAL;
  if ((int64_t)p->W * (int64_t)p->H >= ((int64_t)1 << 31)) return SIM_EINVAL;
  if ((p->H + kCommitTY - 1) / kCommitTY > 65535) return SIM_EINVAL;  // commit grid rows
  if (!(p->rho > 0.0f && p->rho <= 1.0f)) return SIM_EINVAL;
  if (!(p->dtau >= 0.0f && p->dtau <= 3.402823466e38f)) return SIM_EINVAL;
  if (p->alpha < 0 || p->alpha > 8 || p->beta < 0 || p->beta > 8) return SIM_EINVAL;
  if (p->cross_a < 0 || p->cross_a > p->W || p->cross_b < 0 || p->cross_b > p->W) return SIM_EINVAL;
  return SIM_OK;
}

// eta^beta = D2^(-beta/2) for the squared distance D2 from a candidate to the
// point two cells ahead (diagonal 2, lateral 5), rounded to float.
float heuristic(double d2, int beta) { return (float)pow(d2, -0.5 * (double)beta); }

}  // namespace

extern "C" {

const char* sim_strerror(int code) {
  switch (code) {
    case SIM_OK: return "ok";
    case SIM_EINVAL: return "invalid argument";
    case SIM_ESTATE: return "invalid initial state";
    case SIM_ESCRATCH: return "scratch buffer missing or too small";
    case SIM_EHIP: return "HIP runtime error";
    case SIM_ENOTAU: return "ACO step needs pheromone planes";
    case SIM_EFULL: return "no free batch slot";
    default: return "unknown error";
  }
}

int sim_scratch_bytes(const sim_params* p, size_t* out) {
  int e = check_params(p);
  if (e) return e;
  if (!out) return SIM_EINVAL;
  *out = layout_of(p).total;
  return SIM_OK;
}

int sim_create(const sim_params* p, uint8_t* d_code, uint32_t* d_id, float* d_tau, void* d_scratch,
               size_t scratch_bytes, void* stream, sim_handle** out) {
  int e = check_params(p);
  if (e) return e;
  if (!d_code || !d_id || !out) return SIM_EINVAL;
  *out = nullptr;
  const Layout L = layout_of(p);
  if (!d_scratch || scratch_bytes < L.total) return SIM_ESCRATCH;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* scratch = (uint8_t*)d_scratch;
  const size_t cells = (size_t)p->W * (size_t)p->H;
  unsigned long long* totals = (unsigned long long*)(scratch + L.totals);
  unsigned long long* counters = totals + kStatFields;  // 3 validation counters

  // Validate the initial state on the device.
  unsigned long long host_counters[3];
  if (hipMemsetAsync(counters, 0, 3 * sizeof(unsigned long long), s) != hipSuccess) return SIM_EHIP;
  if (launch_validate(d_code, d_id, d_tau, cells, counters, s) != hipSuccess) return SIM_EHIP;
  if (hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, s) != hipSuccess)
    return SIM_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return SIM_EHIP;
  if (host_counters[2]) return SIM_ESTATE;
  const unsigned long long n = host_counters[0] + host_counters[1];
  if (n > 0) {
    uint32_t* bitmap = (uint32_t*)(scratch + L.dec);
    if (hipMemsetAsync(bitmap, 0, (n + 31) / 32 * sizeof(uint32_t), s) != hipSuccess) return SIM_EHIP;
    if (launch_validate_ids(d_id, cells, (uint32_t)n, bitmap, counters, s) != hipSuccess) return SIM_EHIP;
    if (hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, s) != hipSuccess)
      return SIM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SIM_EHIP;
    if (host_counters[2]) return SIM_ESTATE;
  }

  sim_handle* h = new (std::nothrow) sim_handle;
  if (!h) return SIM_EINVAL;
  h->p = *p;
  h->code = d_code;
  h->id = d_id;
  h->tau = d_tau;
  h->totals = totals;
  h->commit_blocks = L.commit_bx * L.commit_by;
  h->t = p->step0;
  StepArgs& a = h->args;
  a.code = d_code;
  a.id = d_id;
  a.tau_a = d_tau;
  a.tau_b = d_tau ? d_tau + cells : nullptr;
  a.dec = scratch + L.dec;
  a.block_stats = (uint32_t*)(scratch + L.block_stats);
  a.W = p->W;
  a.H = p->H;
  a.tiles_x = (p->W + kDecideTX - 1) / kDecideTX;
  a.tiles_y = (p->H + kDecideTY - 1) / kDecideTY;
  a.commit_bx = L.commit_bx;
  a.commit_by = L.commit_by;
  a.t = p->step0;
  a.key0 = (uint32_t)p->seed;
  a.key1 = (uint32_t)(p->seed >> 32);
  const float rho = p->rho;
  a.keep = 1.0f - rho;
  a.dtau = p->dtau;
  a.eta_diag = heuristic(2.0, p->beta);
  a.eta_lat = heuristic(5.0, p->beta);
  a.alpha = p->alpha;
  a.cross_a = p->cross_a;
  a.cross_b = p->cross_b;
  if (launch_count(a, s) != hipSuccess) {
    delete h;
    return SIM_EHIP;
  }
  *out = h;
  return SIM_OK;
}

static int step_n(sim_handle* h, int mode, int32_t nsteps, void* stream) {
  if (!h || nsteps < 0) return SIM_EINVAL;
  if (mode == kModeAco && !h->tau) return SIM_ENOTAU;
  hipStream_t s = (hipStream_t)stream;
  for (int32_t i = 0; i < nsteps; ++i) {
    h->args.t = h->t + (uint64_t)i;
    if (launch_step(h->args, mode, i == nsteps - 1, s) != hipSuccess) return SIM_EHIP;
  }
  h->t += (uint64_t)nsteps;
  return SIM_OK;
}

int sim_step_lem(sim_handle* h, int32_t nsteps, void* stream) { return step_n(h, kModeLem, nsteps, stream); }

int sim_step_aco(sim_handle* h, int32_t nsteps, void* stream) { return step_n(h, kModeAco, nsteps, stream); }

int sim_stats(sim_handle* h, sim_stats_t* out, void* stream) {
  if (!h || !out) return SIM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long v[kStatFields];
  if (launch_reduce_counts(h->args.block_stats, h->commit_blocks, h->totals, s) != hipSuccess) return SIM_EHIP;
  if (hipMemcpyAsync(v, h->totals, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess) return SIM_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return SIM_EHIP;
  out->step = h->t;
  out->agents_a = v[0];
  out->agents_b = v[1];
  out->crossed_a = v[2];
  out->crossed_b = v[3];
  out->moved_last = v[4];
  return SIM_OK;
}

int sim_read_state(sim_handle* h, uint8_t* code, uint32_t* id, float* tau, void* stream) {
  if (!h) return SIM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const size_t cells = (size_t)h->p.W * (size_t)h->p.H;
  if (code && hipMemcpyAsync(code, h->code, cells, hipMemcpyDefault, s) != hipSuccess) return SIM_EHIP;
  if (id && hipMemcpyAsync(id, h->id, cells * sizeof(uint32_t), hipMemcpyDefault, s) != hipSuccess)
    return SIM_EHIP;
  if (tau && h->tau &&
      hipMemcpyAsync(tau, h->tau, 2 * cells * sizeof(float), hipMemcpyDefault, s) != hipSuccess)
    return SIM_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return SIM_EHIP;
  return SIM_OK;
}

int sim_step_timed(sim_handle* h, int32_t mode, int32_t nsteps, void* stream, double* kernel_ms,
                   int64_t* launches, int32_t max_kinds) {
  if (!h || nsteps < 0 || !kernel_ms || !launches || max_kinds < kKernelKinds) return SIM_EINVAL;
  if (mode != kModeLem && mode != kModeAco) return SIM_EINVAL;
  if (mode == kModeAco && !h->tau) return SIM_ENOTAU;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev[kKernelKinds + 1];
  int made = 0;
  int rc = SIM_OK;
  for (; made < kKernelKinds + 1; ++made)
    if (hipEventCreate(&ev[made]) != hipSuccess) {
      rc = SIM_EHIP;
      break;
    }
  for (int32_t i = 0; rc == SIM_OK && i < nsteps; ++i) {
    h->args.t = h->t;
    if (launch_step(h->args, mode, i == nsteps - 1, s, ev) != hipSuccess ||
        hipEventSynchronize(ev[kKernelKinds]) != hipSuccess) {
      rc = SIM_EHIP;
      break;
    }
    h->t += 1;
    for (int k = 0; k < kKernelKinds; ++k) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) rc = SIM_EHIP;
      kernel_ms[k] += ms;
      launches[k] += 1;
    }
  }
  for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
  return rc == SIM_OK ? kKernelKinds : rc;
}

const char* sim_kernel_name(int32_t kind) {
  return (kind >= 0 && kind < kKernelKinds) ? kKernelNames[kind] : "";
}

void sim_destroy(sim_handle* h) { delete h; }

}  // extern "C"
