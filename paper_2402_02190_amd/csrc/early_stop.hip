// Early stopping on the device (Sec. 4.1 Implementation; training-setting
// appendix): the summed head loss L_t = sum_s l_s and the annealing term
// Phi_t = gamma_t * sum (1 - (2P - 1)^alpha) are monitored with a tolerance
// (absolute, or relative to the previous value) and a patience; the rule and the state layout are stated with
// cpra_early_stop_cfg in cpra.h.
//
// One block runs after the per-graph loss terms of the step are complete.  It
// sums them in a fixed order (FP64), updates the state, and advances the step
// counter unless the rule has fired, so that gamma and Adam's t stop with the
// training.  Adam reads `stopped` and skips the update of a stopped step.
#include <cmath>

#include "common.hpp"

namespace cpra {

namespace {

__global__ __launch_bounds__(256) void k_early_stop(int n_graphs, int S, const double* __restrict__ terms,
                                                    cpra_early_stop_state* st, double tol, int relative,
                                                    int patience, int32_t* counter, double g0, double g1,
                                                    int T) {
  if (st->stopped) return;  // uniform: every thread reads the same flag
  double head = 0.0, ent = 0.0;
  for (int g = threadIdx.x; g < n_graphs; g += 256) {
    const double* row = terms + (int64_t)g * (S + 2);
    double h = 0.0;
    for (int s = 0; s < S; ++s) h += row[s];
    head += h;
    ent += row[S];
  }
  __shared__ double sh[2][256];
  sh[0][threadIdx.x] = head;
  sh[1][threadIdx.x] = ent;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const int t = *counter;
  // gamma of this step exactly as the loss kernel formed it
  const double frac = T > 1 ? (double)min(t, T - 1) / (double)(T - 1) : 1.0;
  const float gamma = (float)(g0 + (g1 - g0) * frac);
  const double L = sh[0][0];
  const double phi = (double)gamma * sh[1][0];
  if (st->seen > 0) {
    const double tol_l = relative ? tol * fabs(st->prev_head) : tol;
    const double tol_p = relative ? tol * fabs(st->prev_phi) : tol;
    const bool stalled = (L - st->prev_head >= -tol_l) && (phi - st->prev_phi >= -tol_p);
    st->stalled = stalled ? st->stalled + 1 : 0;
    if (st->stalled >= patience) {
      st->stopped = 1;
      st->stop_step = t;
    }
  }
  st->prev_head = L;
  st->prev_phi = phi;
  st->seen = st->seen + 1;
  if (!st->stopped) counter[0] = t + 1;
}

__global__ void k_early_stop_reset(cpra_early_stop_state* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->prev_head = 0.0;
    st->prev_phi = 0.0;
    st->stalled = 0;
    st->stopped = 0;
    st->stop_step = -1;
    st->seen = 0;
  }
}

}  // namespace

cpra_status check_early_stop_cfg(const cpra_early_stop_cfg* es) {
  if (es->state == nullptr) return CPRA_OK;
  if (!(es->tol >= 0.0) || !std::isfinite(es->tol))
    CPRA_FAIL(CPRA_ERR_PARAM, "early_stop: tol must be finite and >= 0");
  if (es->patience < 1) CPRA_FAIL(CPRA_ERR_PARAM, "early_stop: patience must be >= 1");
  if (es->relative != 0 && es->relative != 1)
    CPRA_FAIL(CPRA_ERR_PARAM, "early_stop: relative must be 0 or 1");
  return CPRA_OK;
}

cpra_status early_stop_update(const cpra_csr* g, const cpra_loss_cfg* lc, const double* terms,
                              const cpra_early_stop_cfg* es, int32_t* counter, hipStream_t stream) {
  hipLaunchKernelGGL(k_early_stop, dim3(1), dim3(256), 0, stream, g->n_graphs, lc->S, terms, es->state,
                     es->tol, es->relative, es->patience, counter, (double)lc->gamma_start, (double)lc->gamma_end,
                     lc->T);
  CPRA_CHECK_LAUNCH("early_stop");
  return CPRA_OK;
}

}  // namespace cpra

extern "C" cpra_status cpra_early_stop_reset(cpra_early_stop_state* state, cpra_stream_t stream) {
  if (state == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "early_stop_reset: state is NULL");
  hipLaunchKernelGGL(cpra::k_early_stop_reset, dim3(1), dim3(64), 0, cpra::as_stream(stream), state);
  CPRA_CHECK_LAUNCH("early_stop_reset");
  return CPRA_OK;
}
