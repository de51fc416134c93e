// Fused relaxed CPRA objective and its gradient dR/dZ (Sec. 3.1-3.3; objective
// table of the problem-specification appendix).
//
// For node i and head s with P = sigmoid(Z) and (AP)_is = sum_{j in N(i)} A_ij P_js:
//   MIS:    l_is = P_is (-w_is + lambda_s/2 (AP)_is), dl/dP_is = -w_is + lambda_s (AP)_is
//           (node weights w, 1 by default)
//   MaxCut: l_is = P_is ((AP)_is - wdeg_i),          dl/dP_is = 2 (AP)_is - wdeg_i
// so that sum_i l_is equals the per-head objective with every edge counted once.
// With one instance per head (per-head edge weights A_ijs, template flag PH)
// the gathers read A_ijs beside P_js, and MaxCut's wdeg_is = sum_j A_ijs is
// summed in the same pass.
//   annealing: phi_is = 1 - t^alpha, t = 2P - 1 = P - Q (Q = sigmoid(-Z)),
//              evaluated as 4 P Q sum_{k<alpha/2} t^(2k); d(gamma phi)/dP = -2 alpha gamma t^(alpha-1)
//   diversity: Psi_i = -S sigma_i over the heads of node i,
//              dPsi/dP_is = -S (P_is - mu_i) / ((S - ddof) sigma_i), 0 where sigma_i = 0
//   dZ_is = dR/dP_is * P_is * Q_is.
//
// Layout: a wavefront holds 64/LPR nodes, the LPR lanes of a node cover its
// heads (NC heads per lane).  Row gathers of P are contiguous per neighbour.
// Per-head and scalar sums go through a fixed butterfly within the wavefront,
// a fixed-order sum across the block's 4 wavefronts, one FP32 partial per
// (column, item) and a fixed-order FP64 reduction per graph: deterministic.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace cpra {

namespace {

struct LossArgs {
  int n, S, problem, alpha, ddof, lpr_log2, iters, want_psi;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* weight;
  const float* wdeg;
  const float* Z;
  int64_t ldz;
  const float* P;
  int64_t ldp;
  float* dZ;
  int64_t lddz;
  const float* lambda;
  float gamma, nu;
  const int32_t* step_counter;
  double g0, g1;
  int T;
  int n_graphs;
  const int32_t* graph_ptr;
  const int32_t* item_ptr;
  int R;
  float* part;
  int64_t items_cap;
  const float* node_w;  // MIS node weights or null
  int64_t ld_nw;        // 0: one weight per node
  const float* edge_w;  // per-head edge weights [nnz, ld_ew] (PH) or null
  int64_t ld_ew;
};

__device__ inline float wave_sum_xor(float v, int from_mask, int to_mask) {
  for (int m = from_mask; m < to_mask; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <int NC, bool PH>
__global__ __launch_bounds__(256) void k_loss(LossArgs a) {
  int g, r0, r1;
  const int item = xcd_unit(blockIdx.x, gridDim.x);
  if (!item_rows(item, a.n_graphs, a.n, a.graph_ptr, a.item_ptr, a.R, &g, &r0, &r1)) return;

  float gamma = a.gamma;
  if (a.step_counter) {
    int t = *a.step_counter;
    double frac = a.T > 1 ? (double)min(t, a.T - 1) / (double)(a.T - 1) : 1.0;
    gamma = (float)(a.g0 + (a.g1 - a.g0) * frac);
  }

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lpr = 1 << a.lpr_log2;
  const int rpw = 64 >> a.lpr_log2;
  const int sub = lane >> a.lpr_log2;
  const int cl = lane & (lpr - 1);
  const int S = a.S;
  const bool mis = a.problem == CPRA_MIS;
  const int half_alpha = a.alpha >> 1;
  const float two_alpha_gamma = 2.0f * (float)a.alpha * gamma;
  const bool diverse = a.nu != 0.0f && S > 1;          // gradient of Psi needed
  const bool stats = S > 1 && (diverse || a.want_psi);  // Psi itself needed

  float lam_h[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int s = c * lpr + cl;
    lam_h[c] = (mis && s < S) ? a.lambda[s] : 0.0f;
  }

  float hl[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) hl[c] = 0.0f;
  float ent = 0.0f, psi = 0.0f;

  const int rows_per_iter = 4 * rpw;
  for (int base = r0; base < r1; base += rows_per_iter) {
    const int row = base + wave * rpw + sub;
    const bool active = row < r1;
    float z[NC], ap[NC], wdh[NC];  // wdh: per-head weighted degree (PH)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int s = c * lpr + cl;
      z[c] = (active && s < S) ? a.Z[(int64_t)row * a.ldz + s] : 0.0f;
      ap[c] = 0.0f;
      wdh[c] = 0.0f;
    }
    if (active) {
      // Neighbours in full chunks of 4 (index and weight loads, then the four
      // gathers, then the adds in CSR order), and the remaining 1-3 as one
      // predicated chunk, so that the tail costs one round trip, not one each.
      const int beg = a.row_ptr[row], end = a.row_ptr[row + 1];
      int k = beg;
      for (; k + 4 <= end; k += 4) {
        const int j0 = a.col_idx[k], j1 = a.col_idx[k + 1], j2 = a.col_idx[k + 2], j3 = a.col_idx[k + 3];
        float w0 = 1.f, w1 = 1.f, w2 = 1.f, w3 = 1.f;
        if (a.weight) { w0 = a.weight[k]; w1 = a.weight[k + 1]; w2 = a.weight[k + 2]; w3 = a.weight[k + 3]; }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int s = c * lpr + cl;
          if (s < S) {
            const float p0 = a.P[(int64_t)j0 * a.ldp + s];
            const float p1 = a.P[(int64_t)j1 * a.ldp + s];
            const float p2 = a.P[(int64_t)j2 * a.ldp + s];
            const float p3 = a.P[(int64_t)j3 * a.ldp + s];
            if constexpr (PH) {
              const float* e = a.edge_w + (int64_t)k * a.ld_ew + s;
              const float v0 = e[0], v1 = e[a.ld_ew], v2 = e[2 * a.ld_ew], v3 = e[3 * a.ld_ew];
              ap[c] += v0 * p0;
              ap[c] += v1 * p1;
              ap[c] += v2 * p2;
              ap[c] += v3 * p3;
              wdh[c] += v0;
              wdh[c] += v1;
              wdh[c] += v2;
              wdh[c] += v3;
            } else {
              ap[c] += w0 * p0;
              ap[c] += w1 * p1;
              ap[c] += w2 * p2;
              ap[c] += w3 * p3;
            }
          }
        }
      }
      if (k < end) {  // 1-3 left
        // entries past the end re-read the row's last neighbour (and add 0)
        const int n_left = end - k;
        const int j0 = a.col_idx[k];
        const int j1 = a.col_idx[min(k + 1, end - 1)];
        const int j2 = a.col_idx[min(k + 2, end - 1)];
        float w0 = 1.f, w1 = 1.f, w2 = 1.f;
        if (a.weight) {
          w0 = a.weight[k];
          w1 = a.weight[min(k + 1, end - 1)];
          w2 = a.weight[min(k + 2, end - 1)];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int s = c * lpr + cl;
          if (s < S) {
            const float p0 = a.P[(int64_t)j0 * a.ldp + s];
            const float p1 = a.P[(int64_t)j1 * a.ldp + s];
            const float p2 = a.P[(int64_t)j2 * a.ldp + s];
            // padded entries add an exact zero (weight 0 by a select, no branch)
            if constexpr (PH) {
              const float* e = a.edge_w + s;
              const float v0 = e[(int64_t)k * a.ld_ew];
              const float v1 = n_left > 1 ? e[(int64_t)min(k + 1, end - 1) * a.ld_ew] : 0.f;
              const float v2 = n_left > 2 ? e[(int64_t)min(k + 2, end - 1) * a.ld_ew] : 0.f;
              ap[c] += v0 * p0;
              ap[c] += v1 * p1;
              ap[c] += v2 * p2;
              wdh[c] += v0;
              wdh[c] += v1;
              wdh[c] += v2;
            } else {
              ap[c] += w0 * p0;
              ap[c] += (n_left > 1 ? w1 : 0.f) * p1;
              ap[c] += (n_left > 2 ? w2 : 0.f) * p2;
            }
          }
        }
      }
    }
    const float wd = (!PH && active && !mis) ? a.wdeg[row] : 0.0f;

    float p[NC], q[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const float e = expf(-fabsf(z[c]));
      const float r = 1.0f / (1.0f + e);
      p[c] = z[c] >= 0.0f ? r : e * r;
      q[c] = z[c] >= 0.0f ? e * r : r;
    }

    // Diversity statistics of the node across its heads (two passes).
    float mu = 0.0f, sig = 0.0f, inv_dev_scale = 0.0f;
    if (stats) {
      float sp = 0.0f;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c * lpr + cl < S) sp += p[c];
      sp = wave_sum_xor(sp, 1, lpr);
      mu = sp / (float)S;
      float sd = 0.0f;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c * lpr + cl < S) {
          const float d = p[c] - mu;
          sd += d * d;
        }
      sd = wave_sum_xor(sd, 1, lpr);
      sig = sqrtf(sd / (float)(S - a.ddof));
      inv_dev_scale = sig > 0.0f ? -(float)S / ((float)(S - a.ddof) * sig) : 0.0f;
      if (active && cl == 0) psi += -(float)S * sig;
    }

#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int s = c * lpr + cl;
      if (!active || s >= S) continue;
      const float t = p[c] - q[c];
      const float t2 = t * t;
      float series = 1.0f, tp = 1.0f;
      for (int kk = 1; kk < half_alpha; ++kk) {
        tp *= t2;
        series += tp;
      }
      const float phi = 4.0f * p[c] * q[c] * series;
      const float t_am1 = t * tp;  // t^(alpha-1)
      float l, gr;
      if (mis) {
        const float u = a.node_w ? -a.node_w[a.ld_nw ? (int64_t)row * a.ld_nw + s : (int64_t)row]
                                 : -1.0f;
        l = p[c] * (u + 0.5f * lam_h[c] * ap[c]);
        gr = u + lam_h[c] * ap[c];
      } else {
        const float wdc = PH ? wdh[c] : wd;
        l = p[c] * (ap[c] - wdc);
        gr = 2.0f * ap[c] - wdc;
      }
      gr -= two_alpha_gamma * t_am1;
      if (diverse) gr += a.nu * inv_dev_scale * (p[c] - mu);
      hl[c] += l;
      ent += phi;
      if (a.dZ) a.dZ[(int64_t)row * a.lddz + s] = gr * p[c] * q[c];
    }
  }

  // ---- block reduction into this item's partial column entries ----------
  __shared__ float sh_head[4][NC * 64];
  __shared__ float sh_scal[4][2];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const float v = wave_sum_xor(hl[c], lpr, 64);
    if (sub == 0) sh_head[wave][c * lpr + cl] = v;
  }
  {
    const float e = wave_sum_xor(ent, 1, 64);
    const float ps = wave_sum_xor(psi, 1, 64);
    if (lane == 0) {
      sh_scal[wave][0] = e;
      sh_scal[wave][1] = ps;
    }
  }
  __syncthreads();
  const int slots = NC * lpr;
  for (int s = threadIdx.x; s < slots; s += 256) {
    if (s < S) {
      const float v = ((sh_head[0][s] + sh_head[1][s]) + sh_head[2][s]) + sh_head[3][s];
      a.part[(int64_t)s * a.items_cap + item] = v;
    }
  }
  if (threadIdx.x == 0) {
    a.part[(int64_t)S * a.items_cap + item] =
        ((sh_scal[0][0] + sh_scal[1][0]) + sh_scal[2][0]) + sh_scal[3][0];
    a.part[(int64_t)(S + 1) * a.items_cap + item] =
        ((sh_scal[0][1] + sh_scal[1][1]) + sh_scal[2][1]) + sh_scal[3][1];
  }
}

struct LossGeom {
  int lpr, lpr_log2, nc, R, iters;
  int64_t items_cap;
};

LossGeom loss_geom(const cpra_csr* g, int S) {
  LossGeom G{};
  G.lpr = 1;
  while (G.lpr < S && G.lpr < 64) G.lpr <<= 1;
  G.lpr_log2 = 0;
  while ((1 << G.lpr_log2) < G.lpr) ++G.lpr_log2;
  int need = (int)ceil_div(S, G.lpr);
  G.nc = 1;
  while (G.nc < need) G.nc <<= 1;
  const int rows_per_iter = 4 * (64 / G.lpr);
  // Enough items to fill the GPU several times over, at most 8 row groups each.
  int64_t it = g->n_nodes / ((int64_t)rows_per_iter * 2048);
  G.iters = (int)std::max<int64_t>(1, std::min<int64_t>(8, it));
  G.R = rows_per_iter * G.iters;
  G.items_cap = max_items(g, G.R);
  return G;
}

struct LossWs {
  size_t p_off, item_off, part_off, total;
};

// Workspace: [item table][partials][P = sigmoid(Z) when the caller passes none].
LossWs loss_ws_layout(const cpra_csr* g, int S, bool need_p) {
  LossGeom G = loss_geom(g, S);
  LossWs w{};
  size_t off = 0;
  w.item_off = off;
  off += align_up((size_t)(g->n_graphs + 1) * sizeof(int32_t), 256);
  w.part_off = off;
  off += align_up((size_t)(S + 2) * G.items_cap * sizeof(float), 256);
  w.p_off = off;
  if (need_p) off += align_up((size_t)g->n_nodes * S * sizeof(float), 256);
  w.total = off;
  return w;
}

cpra_status check_loss_cfg(const cpra_csr* g, const cpra_loss_cfg* cfg) {
  if (cfg == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "loss: cfg is NULL");
  if (cfg->problem != CPRA_MIS && cfg->problem != CPRA_MAXCUT)
    CPRA_FAIL(CPRA_ERR_PARAM, "loss: unknown problem %d", cfg->problem);
  if (cfg->S < 1 || cfg->S > 1024) CPRA_FAIL(CPRA_ERR_PARAM, "loss: S = %d outside 1..1024", cfg->S);
  if (cfg->alpha < 2 || cfg->alpha > 64 || (cfg->alpha & 1))
    CPRA_FAIL(CPRA_ERR_PARAM, "loss: alpha = %d must be even in 2..64", cfg->alpha);
  if (cfg->std_ddof != 0 && cfg->std_ddof != 1)
    CPRA_FAIL(CPRA_ERR_PARAM, "loss: std_ddof must be 0 or 1");
  if (cfg->nu != 0.0f && cfg->S <= cfg->std_ddof)
    CPRA_FAIL(CPRA_ERR_PARAM, "loss: S must exceed std_ddof when nu != 0");
  if (!std::isfinite(cfg->gamma) || !std::isfinite(cfg->nu))
    CPRA_FAIL(CPRA_ERR_NONFINITE, "loss: gamma or nu is not finite");
  if (cfg->step_counter && (!std::isfinite(cfg->gamma_start) || !std::isfinite(cfg->gamma_end) || cfg->T < 1))
    CPRA_FAIL(CPRA_ERR_PARAM, "loss: bad device schedule (gamma endpoints finite, T >= 1)");
  if (cfg->problem == CPRA_MIS && g->n_nodes > 0 && cfg->lambda == nullptr)
    CPRA_FAIL(CPRA_ERR_NULL, "loss: lambda is NULL for MIS");
  if (cfg->node_weight && cfg->problem != CPRA_MIS)
    CPRA_FAIL(CPRA_ERR_PARAM, "loss: node weights are defined for MIS only");
  if (cfg->node_weight && cfg->ld_node_weight != 0 && cfg->ld_node_weight < cfg->S)
    CPRA_FAIL(CPRA_ERR_SHAPE, "loss: ld_node_weight must be 0 or >= S");
  if (cfg->edge_weight && cfg->ld_edge_weight < cfg->S)
    CPRA_FAIL(CPRA_ERR_SHAPE, "loss: ld_edge_weight must be >= S");
  return CPRA_OK;
}

}  // namespace

size_t loss_workspace_bytes(const cpra_csr* g, int S, bool need_p) {
  return loss_ws_layout(g, S, need_p).total;
}

cpra_status loss_fwd_bwd(const cpra_csr* g, const cpra_loss_cfg* cfg, const float* Z, int64_t ldz,
                         const float* P, int64_t ldp, float* dZ, int64_t lddz, double* terms,
                         void* ws, size_t ws_bytes, hipStream_t stream, bool want_terms) {
  want_terms = want_terms || terms != nullptr;
  const int S = cfg->S;
  LossWs L = loss_ws_layout(g, S, P == nullptr);
  if (ws == nullptr || ws_bytes < L.total)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "loss: workspace %zu < %zu bytes", ws_bytes, L.total);
  char* base = static_cast<char*>(ws);
  if (P == nullptr) {
    float* Pw = reinterpret_cast<float*>(base + L.p_off);
    CPRA_CHECK(sigmoid(g->n_nodes, S, Z, ldz, Pw, S, stream));
    P = Pw;
    ldp = S;
  }
  LossGeom G = loss_geom(g, S);
  int32_t* item_ptr = reinterpret_cast<int32_t*>(base + L.item_off);
  float* part = reinterpret_cast<float*>(base + L.part_off);
  CPRA_CHECK(launch_item_ptr(g, G.R, item_ptr, stream));
  LossArgs a{};
  a.n = g->n_nodes;
  a.S = S;
  a.problem = cfg->problem;
  a.alpha = cfg->alpha;
  a.ddof = cfg->std_ddof;
  a.lpr_log2 = G.lpr_log2;
  a.iters = G.iters;
  a.want_psi = want_terms ? 1 : 0;
  a.row_ptr = g->row_ptr;
  a.col_idx = g->col_idx;
  a.weight = g->weight;
  a.wdeg = g->wdeg;
  a.Z = Z;
  a.ldz = ldz;
  a.P = P;
  a.ldp = ldp;
  a.dZ = dZ;
  a.lddz = lddz;
  a.lambda = cfg->lambda;
  a.gamma = cfg->gamma;
  a.nu = cfg->nu;
  a.step_counter = cfg->step_counter;
  a.g0 = cfg->gamma_start;
  a.g1 = cfg->gamma_end;
  a.T = cfg->T;
  a.n_graphs = g->n_graphs;
  a.graph_ptr = g->n_graphs > 1 ? g->graph_ptr : nullptr;
  a.item_ptr = item_ptr;
  a.R = G.R;
  a.part = part;
  a.items_cap = G.items_cap;
  a.node_w = cfg->node_weight;
  a.ld_nw = cfg->ld_node_weight;
  a.edge_w = cfg->edge_weight;
  a.ld_ew = cfg->ld_edge_weight;
  const bool ph = cfg->edge_weight != nullptr;
  const int blocks = (int)xcd_grid(G.items_cap);
  // compulsory bytes: Z and P read once, dZ written, CSR (+weights), wdeg, partials
  const double ns4 = 4.0 * (double)g->n_nodes * S;
  const double loss_bytes = ns4 * (dZ ? 3.0 : 2.0) +
                            4.0 * (double)g->nnz * (g->weight && !ph ? 2.0 : 1.0) +
                            4.0 * (double)g->n_nodes * (cfg->problem == CPRA_MAXCUT && !ph ? 2.0 : 1.0) +
                            (cfg->node_weight ? 4.0 * (double)g->n_nodes *
                                                    (cfg->ld_node_weight ? S : 1) : 0.0) +
                            (ph ? 4.0 * (double)g->nnz * S : 0.0) +
                            4.0 * (double)(S + 2) * G.items_cap;
  ProfScope ps("loss_fwd_bwd", stream, 0.0, loss_bytes);
  switch (G.nc) {
#define CPRA_LOSS_CASE(NCV)                                                             \
  case NCV:                                                                             \
    if (ph) hipLaunchKernelGGL((k_loss<NCV, true>), dim3(blocks), dim3(256), 0, stream, a); \
    else hipLaunchKernelGGL((k_loss<NCV, false>), dim3(blocks), dim3(256), 0, stream, a);   \
    break;
    CPRA_LOSS_CASE(1)
    CPRA_LOSS_CASE(2)
    CPRA_LOSS_CASE(4)
    CPRA_LOSS_CASE(8)
    CPRA_LOSS_CASE(16)
#undef CPRA_LOSS_CASE
    default:
      CPRA_FAIL(CPRA_ERR_PARAM, "loss: S too large");
  }
  CPRA_CHECK_LAUNCH("loss");
  if (terms) CPRA_CHECK(loss_terms_reduce(g, cfg, terms, ws, stream));
  return CPRA_OK;
}

// Reduce the partials left in `ws` by the last loss launch on the same graph/config.
cpra_status loss_terms_reduce(const cpra_csr* g, const cpra_loss_cfg* cfg, double* terms, void* ws,
                              hipStream_t stream, int32_t* advance) {
  const int S = cfg->S;
  const LossWs L = loss_ws_layout(g, S, false);
  const LossGeom G = loss_geom(g, S);
  char* base = static_cast<char*>(ws);
  const int32_t* item_ptr = reinterpret_cast<const int32_t*>(base + L.item_off);
  const float* part = reinterpret_cast<const float*>(base + L.part_off);
  return launch_segment_reduce(g, G.R, item_ptr, part, nullptr, G.items_cap, S + 2, terms, stream,
                               advance);
}

}  // namespace cpra

extern "C" {

size_t cpra_loss_workspace_bytes(const cpra_csr* g, const cpra_loss_cfg* cfg) {
  if (g == nullptr || cfg == nullptr || cfg->S < 1) return 0;
  return cpra::loss_workspace_bytes(g, cfg->S, true);
}

cpra_status cpra_loss_fwd_bwd(const cpra_csr* g, const cpra_loss_cfg* cfg, const float* Z,
                              int64_t ldz, const float* P, int64_t ldp, float* dZ, int64_t lddz,
                              double* terms, void* ws, size_t ws_bytes, cpra_stream_t stream) {
  CPRA_CHECK(cpra::check_csr(g, "loss_fwd_bwd", false,
                             cfg && cfg->problem == CPRA_MAXCUT && cfg->edge_weight == nullptr));
  CPRA_CHECK(cpra::check_loss_cfg(g, cfg));
  if (g->n_nodes > 0) {
    if (Z == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "loss_fwd_bwd: Z is NULL");
    if (ldz < cfg->S || (P && ldp < cfg->S) || (dZ && lddz < cfg->S))
      CPRA_FAIL(CPRA_ERR_SHAPE, "loss_fwd_bwd: leading dimension < S");
  }
  return cpra::loss_fwd_bwd(g, cfg, Z, ldz, P, ldp, dZ, lddz, terms, ws, ws_bytes,
                            cpra::as_stream(stream));
}

}  // extern "C"

namespace cpra {
cpra_status check_loss_cfg_public(const cpra_csr* g, const cpra_loss_cfg* cfg) {
  return check_loss_cfg(g, cfg);
}
}  // namespace cpra
