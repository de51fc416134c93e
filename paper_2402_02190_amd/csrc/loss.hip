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
//              (exactly where all heads of node i are equal)
//   dZ_is = dR/dP_is * P_is * Q_is.
//
// Layout: a wavefront holds 64/LPR nodes, the LPR lanes of a node cover its
// heads (NC heads per lane).  Row gathers of P are contiguous per neighbour.
// Per-head and scalar sums go through a fixed butterfly within the wavefront,
// a fixed-order sum across the block's 4 wavefronts, one FP32 partial per
// (column, item) and a fixed-order FP64 reduction per graph: deterministic.
#include <algorithm>
#include <cmath>
#include <mutex>

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
  int32_t* queue;  // persistent launches: the work queue (kQueueInts counters)
  int chunk;       // persistent launches: items per dequeue
};

__device__ inline float wave_sum_xor(float v, int from_mask, int to_mask) {
  for (int m = from_mask; m < to_mask; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Per-lane vectors of VEC consecutive heads (float4 when VEC = 4).
template <int VEC>
struct HV {
  float v[VEC];
  __device__ inline void load(const float* p) {
    if constexpr (VEC == 4) {
      const float4 x = *reinterpret_cast<const float4*>(p);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else {
      v[0] = *p;
    }
  }
  __device__ inline void store(float* p) const {
    if constexpr (VEC == 4) *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    else *p = v[0];
  }
  __device__ inline void zero() {
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[e] = 0.0f;
  }
};

// Lane layout: a wavefront holds 64/LPR nodes; lane cl of a node owns NC units
// of VEC consecutive heads, unit c covering heads (c * LPR + cl) * VEC + e.
// Item `item` (a block of rows inside one graph) and its partial sums.
template <int NC, int VEC, bool PH>
__device__ __forceinline__ void loss_item(const LossArgs& a, int item) {
  int g, r0, r1;
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

  int h0[NC];      // first head of each unit
  bool uok[NC];    // unit inside [0, S) (S is a multiple of VEC)
  HV<VEC> lam_h[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    h0[c] = (c * lpr + cl) * VEC;
    uok[c] = h0[c] < S;
    if (mis && uok[c]) lam_h[c].load(a.lambda + h0[c]); else lam_h[c].zero();
  }

  HV<VEC> hl[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) hl[c].zero();
  float ent = 0.0f, psi = 0.0f;

  const int rows_per_iter = 4 * rpw;
  for (int base = r0; base < r1; base += rows_per_iter) {
    const int row = base + wave * rpw + sub;
    const bool active = row < r1;
    HV<VEC> z[NC], ap[NC], wdh[NC];  // wdh: per-head weighted degree (PH)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (active && uok[c]) z[c].load(a.Z + (int64_t)row * a.ldz + h0[c]); else z[c].zero();
      ap[c].zero();
      wdh[c].zero();
    }
    if (active) {
      // Neighbours in full chunks of 4 (index and weight loads, then the four
      // gathers, then the adds in CSR order), and the remaining 1-3 as one
      // padded chunk, so that the tail costs one round trip, not one each.
      const int beg = a.row_ptr[row], end = a.row_ptr[row + 1];
      int k = beg;
      for (; k + 4 <= end; k += 4) {
        const int j0 = a.col_idx[k], j1 = a.col_idx[k + 1], j2 = a.col_idx[k + 2], j3 = a.col_idx[k + 3];
        float w0 = 1.f, w1 = 1.f, w2 = 1.f, w3 = 1.f;
        if (!PH && a.weight) { w0 = a.weight[k]; w1 = a.weight[k + 1]; w2 = a.weight[k + 2]; w3 = a.weight[k + 3]; }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (!uok[c]) continue;
          HV<VEC> p0, p1, p2, p3;
          p0.load(a.P + (int64_t)j0 * a.ldp + h0[c]);
          p1.load(a.P + (int64_t)j1 * a.ldp + h0[c]);
          p2.load(a.P + (int64_t)j2 * a.ldp + h0[c]);
          p3.load(a.P + (int64_t)j3 * a.ldp + h0[c]);
          if constexpr (PH) {
            HV<VEC> v0, v1, v2, v3;
            const float* e = a.edge_w + (int64_t)k * a.ld_ew + h0[c];
            v0.load(e);
            v1.load(e + a.ld_ew);
            v2.load(e + 2 * a.ld_ew);
            v3.load(e + 3 * a.ld_ew);
#pragma unroll
            for (int x = 0; x < VEC; ++x) {
              ap[c].v[x] += v0.v[x] * p0.v[x];
              ap[c].v[x] += v1.v[x] * p1.v[x];
              ap[c].v[x] += v2.v[x] * p2.v[x];
              ap[c].v[x] += v3.v[x] * p3.v[x];
              wdh[c].v[x] += v0.v[x];
              wdh[c].v[x] += v1.v[x];
              wdh[c].v[x] += v2.v[x];
              wdh[c].v[x] += v3.v[x];
            }
          } else {
#pragma unroll
            for (int x = 0; x < VEC; ++x) {
              ap[c].v[x] += w0 * p0.v[x];
              ap[c].v[x] += w1 * p1.v[x];
              ap[c].v[x] += w2 * p2.v[x];
              ap[c].v[x] += w3 * p3.v[x];
            }
          }
        }
      }
      if (k < end) {  // 1-3 left
        // entries past the end re-read the row's last neighbour (and add 0)
        const int n_left = end - k;
        const int k1 = min(k + 1, end - 1), k2 = min(k + 2, end - 1);
        const int j0 = a.col_idx[k], j1 = a.col_idx[k1], j2 = a.col_idx[k2];
        float w0 = 1.f, w1 = 1.f, w2 = 1.f;
        if (!PH && a.weight) {
          w0 = a.weight[k];
          w1 = a.weight[k1];
          w2 = a.weight[k2];
        }
        w1 = n_left > 1 ? w1 : 0.f;  // padded entries add an exact zero (by a select, no branch)
        w2 = n_left > 2 ? w2 : 0.f;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (!uok[c]) continue;
          HV<VEC> p0, p1, p2;
          p0.load(a.P + (int64_t)j0 * a.ldp + h0[c]);
          p1.load(a.P + (int64_t)j1 * a.ldp + h0[c]);
          p2.load(a.P + (int64_t)j2 * a.ldp + h0[c]);
          if constexpr (PH) {
            HV<VEC> v0, v1, v2;
            v0.load(a.edge_w + (int64_t)k * a.ld_ew + h0[c]);
            v1.load(a.edge_w + (int64_t)k1 * a.ld_ew + h0[c]);
            v2.load(a.edge_w + (int64_t)k2 * a.ld_ew + h0[c]);
#pragma unroll
            for (int x = 0; x < VEC; ++x) {
              const float u1 = n_left > 1 ? v1.v[x] : 0.f, u2 = n_left > 2 ? v2.v[x] : 0.f;
              ap[c].v[x] += v0.v[x] * p0.v[x];
              ap[c].v[x] += u1 * p1.v[x];
              ap[c].v[x] += u2 * p2.v[x];
              wdh[c].v[x] += v0.v[x];
              wdh[c].v[x] += u1;
              wdh[c].v[x] += u2;
            }
          } else {
#pragma unroll
            for (int x = 0; x < VEC; ++x) {
              ap[c].v[x] += w0 * p0.v[x];
              ap[c].v[x] += w1 * p1.v[x];
              ap[c].v[x] += w2 * p2.v[x];
            }
          }
        }
      }
    }
    const float wd = (!PH && active && !mis) ? a.wdeg[row] : 0.0f;

    HV<VEC> p[NC], q[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int x = 0; x < VEC; ++x) {
        const float zz = z[c].v[x];
        const float e = expf(-fabsf(zz));
        const float r = 1.0f / (1.0f + e);
        p[c].v[x] = zz >= 0.0f ? r : e * r;
        q[c].v[x] = zz >= 0.0f ? e * r : r;
      }

    // Diversity statistics of the node across its heads: mean, then deviations
    // corrected by their own mean (the corrected two-pass variance of Chan, Golub
    // and LeVeque), so that a deviation keeps its relative accuracy when sigma is
    // far below the mean.  A node whose heads are all equal has sigma = 0 (and a
    // zero gradient) by definition: the rounded mean of equal values need not
    // equal them, which would leave a spurious sigma of a few ulps.
    float mu = 0.0f, dmu = 0.0f, sig = 0.0f, inv_dev_scale = 0.0f;
    if (stats) {
      float sp = 0.0f;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (uok[c])
#pragma unroll
          for (int x = 0; x < VEC; ++x) sp += p[c].v[x];
      sp = wave_sum_xor(sp, 1, lpr);
      mu = sp / (float)S;
      const float first = __shfl(p[0].v[0], lane & ~(lpr - 1), 64);  // head 0 of the node
      float sd = 0.0f, s1 = 0.0f;
      int differ = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (uok[c])
#pragma unroll
          for (int x = 0; x < VEC; ++x) {
            const float d = p[c].v[x] - mu;
            s1 += d;
            sd += d * d;
            differ |= p[c].v[x] != first;
          }
      for (int m = 1; m < lpr; m <<= 1) {
        s1 += __shfl_xor(s1, m, 64);
        sd += __shfl_xor(sd, m, 64);
        differ |= __shfl_xor(differ, m, 64);
      }
      dmu = s1 / (float)S;
      sd = fmaxf(sd - s1 * dmu, 0.0f);
      sig = differ ? sqrtf(sd / (float)(S - a.ddof)) : 0.0f;
      inv_dev_scale = sig > 0.0f ? -(float)S / ((float)(S - a.ddof) * sig) : 0.0f;
      if (active && cl == 0) psi += -(float)S * sig;
    }

#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!active || !uok[c]) continue;
      HV<VEC> u, dz;
      if (mis) {
        if (a.node_w && a.ld_nw) {
          u.load(a.node_w + (int64_t)row * a.ld_nw + h0[c]);
        } else {
          const float w = a.node_w ? a.node_w[row] : 1.0f;
#pragma unroll
          for (int x = 0; x < VEC; ++x) u.v[x] = w;
        }
      }
#pragma unroll
      for (int x = 0; x < VEC; ++x) {
        const float pp = p[c].v[x], qq = q[c].v[x], aa = ap[c].v[x];
        const float t = pp - qq;
        const float t2 = t * t;
        float series = 1.0f, tp = 1.0f;
        for (int kk = 1; kk < half_alpha; ++kk) {
          tp *= t2;
          series += tp;
        }
        const float phi = 4.0f * pp * qq * series;
        const float t_am1 = t * tp;  // t^(alpha-1)
        float l, gr;
        if (mis) {
          const float un = -u.v[x];
          l = pp * (un + 0.5f * lam_h[c].v[x] * aa);
          gr = un + lam_h[c].v[x] * aa;
        } else {
          const float wdc = PH ? wdh[c].v[x] : wd;
          l = pp * (aa - wdc);
          gr = 2.0f * aa - wdc;
        }
        gr -= two_alpha_gamma * t_am1;
        if (diverse) gr += a.nu * inv_dev_scale * ((pp - mu) - dmu);
        hl[c].v[x] += l;
        ent += phi;
        dz.v[x] = gr * pp * qq;
      }
      if (a.dZ) dz.store(a.dZ + (int64_t)row * a.lddz + h0[c]);
    }
  }

  // ---- block reduction into this item's partial column entries ----------
  __shared__ float sh_head[4][NC * 64 * VEC];
  __shared__ float sh_scal[4][2];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int x = 0; x < VEC; ++x) {
      const float v = wave_sum_xor(hl[c].v[x], lpr, 64);
      if (sub == 0) sh_head[wave][h0[c] + x] = v;
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
  const int slots = NC * lpr * VEC;
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

// One block per item, in XCD order.
template <int NC, int VEC, bool PH>
__global__ __launch_bounds__(256) void k_loss(LossArgs a) {
  loss_item<NC, VEC, PH>(a, xcd_unit(blockIdx.x, gridDim.x));
}

// Persistent: at most the resident blocks, each taking items from the queue.  An
// item's partials do not depend on the block that computes it.
template <int NC, int VEC, bool PH>
__global__ __launch_bounds__(256) void k_loss_persistent(LossArgs a) {
  __shared__ int s_chunk;
  const int items = (int)a.items_cap;
  const int chunks = (items + a.chunk - 1) / a.chunk;
  for (bool first = true;; first = false) {
    if (threadIdx.x == 0) s_chunk = queue_next(a.queue, chunks, first);
    __syncthreads();
    const int c = s_chunk;
    if (c < 0) break;  // uniform across the block
    const int i1 = min(items, (c + 1) * a.chunk);
    for (int it = c * a.chunk; it < i1; ++it) {
      loss_item<NC, VEC, PH>(a, it);
      __syncthreads();  // the reduction's LDS is rewritten by the next item
    }
  }
}

// Lanes per node (LPR), units per lane (NC) for VEC heads per unit.
struct LossLanes {
  int lpr, lpr_log2, nc;
};

LossLanes loss_lanes(int S, int vec) {
  LossLanes L{};
  const int units = (int)ceil_div(S, vec);
  L.lpr = 1;
  while (L.lpr < units && L.lpr < 64) L.lpr <<= 1;
  L.lpr_log2 = 0;
  while ((1 << L.lpr_log2) < L.lpr) ++L.lpr_log2;
  const int need = (int)ceil_div(units, L.lpr);
  L.nc = 1;
  while (L.nc < need) L.nc <<= 1;
  return L;
}

// Item geometry (rows per item R, items) depends on the graph and S only, not on
// the lane layout a launch picks, so the partials of any launch are summed by
// the same segmented reduction: R is a multiple of the rows per iteration of
// every layout S admits.
struct LossGeom {
  int R, iters;
  int64_t items_cap;
};

LossGeom loss_geom(const cpra_csr* g, int S) {
  LossGeom G{};
  int rows_per_iter = 4 * (64 / loss_lanes(S, 1).lpr);
  if (S % 4 == 0) rows_per_iter = std::max(rows_per_iter, 4 * (64 / loss_lanes(S, 4).lpr));
  // Enough items to give every CU about 16, at most 8 row groups each.
  const int64_t it = g->n_nodes / ((int64_t)rows_per_iter * 4096);
  G.iters = (int)std::max<int64_t>(1, std::min<int64_t>(8, it));
  G.R = rows_per_iter * G.iters;
  G.items_cap = max_items(g, G.R);
  return G;
}

inline bool al16(const void* p) { return p == nullptr || reinterpret_cast<uintptr_t>(p) % 16 == 0; }

struct LossWs {
  size_t p_off, item_off, part_off, queue_off, total;
};

// Workspace: [work queue][item table][partials][P = sigmoid(Z) when the caller passes none].
LossWs loss_ws_layout(const cpra_csr* g, int S, bool need_p) {
  LossGeom G = loss_geom(g, S);
  LossWs w{};
  size_t off = 0;
  w.queue_off = off;
  off += align_up((size_t)kQueueInts * sizeof(int32_t), 256);
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
  // Four consecutive heads per lane (float4 rows) when every per-head operand allows it.
  const bool vec4 = S % 4 == 0 && ldz % 4 == 0 && ldp % 4 == 0 && (dZ == nullptr || lddz % 4 == 0) &&
                    al16(Z) && al16(P) && al16(dZ) && al16(cfg->lambda) &&
                    (cfg->edge_weight == nullptr || (cfg->ld_edge_weight % 4 == 0 && al16(cfg->edge_weight))) &&
                    (cfg->node_weight == nullptr || cfg->ld_node_weight == 0 ||
                     (cfg->ld_node_weight % 4 == 0 && al16(cfg->node_weight)));
  const LossLanes LN = loss_lanes(S, vec4 ? 4 : 1);
  int32_t* item_ptr = reinterpret_cast<int32_t*>(base + L.item_off);
  float* part = reinterpret_cast<float*>(base + L.part_off);
  CPRA_CHECK(launch_item_ptr(g, G.R, item_ptr, stream));
  LossArgs a{};
  a.n = g->n_nodes;
  a.S = S;
  a.problem = cfg->problem;
  a.alpha = cfg->alpha;
  a.ddof = cfg->std_ddof;
  a.lpr_log2 = LN.lpr_log2;
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
  a.queue = persistent_enabled() ? reinterpret_cast<int32_t*>(base + L.queue_off) : nullptr;
  const bool ph = cfg->edge_weight != nullptr;
  const int blocks = (int)xcd_grid(G.items_cap);
  // compulsory bytes: Z read once, dZ written, CSR (+weights), wdeg, partials.  The
  // node's own row of P is a second read of what Z already holds (it saves the
  // sigmoid), so it is not counted; the neighbour rows of P are gathers.
  const double ns4 = 4.0 * (double)g->n_nodes * S;
  const double loss_bytes = ns4 * (dZ ? 2.0 : 1.0) +
                            4.0 * (double)g->nnz * (g->weight && !ph ? 2.0 : 1.0) +
                            4.0 * (double)g->n_nodes * (cfg->problem == CPRA_MAXCUT && !ph ? 2.0 : 1.0) +
                            (cfg->node_weight ? 4.0 * (double)g->n_nodes *
                                                    (cfg->ld_node_weight ? S : 1) : 0.0) +
                            (ph ? 4.0 * (double)g->nnz * S : 0.0) +
                            4.0 * (double)(S + 2) * G.items_cap;
  ProfScope ps("loss_fwd_bwd", stream, 0.0, loss_bytes, 4.0 * (double)g->nnz * S);
  bool launched = true;
  if (a.queue) CPRA_CHECK(zero_queue(a.queue, stream));
  // a persistent launch runs min(items, resident blocks) blocks
  auto pgrid = [&](const void* k) {
    const int grid = (int)std::min<int64_t>(G.items_cap, resident_blocks(k, 256));
    a.chunk = queue_chunk((int)G.items_cap, grid);
    return dim3((unsigned)grid);
  };
#define CPRA_LOSS_ONE(NCV, VECV, PHV)                                                               \
  if (a.queue) {                                                                                    \
    const dim3 grid = pgrid(reinterpret_cast<const void*>(&k_loss_persistent<NCV, VECV, PHV>));     \
    hipLaunchKernelGGL((k_loss_persistent<NCV, VECV, PHV>), grid, dim3(256), 0, stream, a);         \
  } else {                                                                                          \
    hipLaunchKernelGGL((k_loss<NCV, VECV, PHV>), dim3(blocks), dim3(256), 0, stream, a);            \
  }
#define CPRA_LOSS_LAUNCH(NCV, VECV)    \
  if (ph) {                            \
    CPRA_LOSS_ONE(NCV, VECV, true)     \
  } else {                             \
    CPRA_LOSS_ONE(NCV, VECV, false)    \
  }
  if (vec4) {
    switch (LN.nc) {
      case 1: CPRA_LOSS_LAUNCH(1, 4) break;
      case 2: CPRA_LOSS_LAUNCH(2, 4) break;
      case 4: CPRA_LOSS_LAUNCH(4, 4) break;
      default: launched = false;
    }
  } else {
    switch (LN.nc) {
      case 1: CPRA_LOSS_LAUNCH(1, 1) break;
      case 2: CPRA_LOSS_LAUNCH(2, 1) break;
      case 4: CPRA_LOSS_LAUNCH(4, 1) break;
      case 8: CPRA_LOSS_LAUNCH(8, 1) break;
      case 16: CPRA_LOSS_LAUNCH(16, 1) break;
      default: launched = false;
    }
  }
#undef CPRA_LOSS_LAUNCH
#undef CPRA_LOSS_ONE
  if (!launched) CPRA_FAIL(CPRA_ERR_PARAM, "loss: S too large");
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

// ---- the workspace of cpra_loss_fwd_bwd_noalloc: one static array per GPU --
// Host code never passes `scratch` itself (on the host it only names the
// symbol): the device address comes from hipGetSymbolAddress, looked up once
// per device with that device current and kept in scratch_addr.
static __device__ __align__(256) unsigned char scratch[CPRA_LOSS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

cpra_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "loss_fwd_bwd_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    CPRA_FAIL(CPRA_ERR_PARAM, "loss_fwd_bwd_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      CPRA_FAIL(CPRA_ERR_HIP, "loss_fwd_bwd_noalloc: hipGetSymbolAddress on device %d: %s", dev,
                hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return CPRA_OK;
}
}  // namespace

// R = sum_g (sum_s t[g][s] + gamma t[g][S] + nu t[g][S+1]): thread i sums the
// graphs i, i + 256, ... in order, then a fixed tree over the threads.
__global__ __launch_bounds__(256) void k_loss_total(int n_graphs, int S, const double* __restrict__ t,
                                                    double gamma, double nu, double* R) {
  double acc = 0.0;
  for (int g = threadIdx.x; g < n_graphs; g += 256) {
    const double* row = t + (int64_t)g * (S + 2);
    double h = 0.0;
    for (int s = 0; s < S; ++s) h += row[s];
    acc += h + gamma * row[S] + nu * row[S + 1];
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) R[0] = sh[0];
}

}  // namespace cpra

extern "C" {

cpra_status cpra_loss_total(int32_t n_graphs, int32_t S, const double* terms, double gamma,
                            double nu, double* R, cpra_stream_t stream) {
  if (terms == nullptr || R == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "loss_total: NULL pointer");
  if (n_graphs < 1 || S < 1) CPRA_FAIL(CPRA_ERR_PARAM, "loss_total: n_graphs and S must be >= 1");
  if (!std::isfinite(gamma) || !std::isfinite(nu))
    CPRA_FAIL(CPRA_ERR_NONFINITE, "loss_total: gamma or nu is not finite");
  hipLaunchKernelGGL(cpra::k_loss_total, dim3(1), dim3(256), 0, cpra::as_stream(stream), n_graphs, S,
                     terms, gamma, nu, R);
  CPRA_CHECK_LAUNCH("loss_total");
  return CPRA_OK;
}

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

cpra_status cpra_loss_fwd_bwd_noalloc(const cpra_csr* g, const cpra_loss_cfg* cfg, const float* Z,
                                      int64_t ldz, const float* P, int64_t ldp, float* dZ,
                                      int64_t lddz, double* terms, cpra_stream_t stream) {
  CPRA_CHECK(cpra::check_csr(g, "loss_fwd_bwd_noalloc", false,
                             cfg && cfg->problem == CPRA_MAXCUT && cfg->edge_weight == nullptr));
  CPRA_CHECK(cpra::check_loss_cfg(g, cfg));
  if (g->n_nodes > 0) {
    if (Z == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "loss_fwd_bwd_noalloc: Z is NULL");
    if (ldz < cfg->S || (P && ldp < cfg->S) || (dZ && lddz < cfg->S))
      CPRA_FAIL(CPRA_ERR_SHAPE, "loss_fwd_bwd_noalloc: leading dimension < S");
  }
  const size_t need = cpra::loss_workspace_bytes(g, cfg->S, P == nullptr);
  if (need > CPRA_LOSS_NOALLOC_SCRATCH_BYTES)
    CPRA_FAIL(CPRA_ERR_WORKSPACE,
              "loss_fwd_bwd_noalloc: this graph and S need %zu bytes of scratch, the static array "
              "holds %zu (pass P, or use cpra_loss_fwd_bwd with a workspace)",
              need, (size_t)CPRA_LOSS_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  CPRA_CHECK(cpra::scratch_address(&ws));
  cpra::ProfSuspend no_events;  // the profiler would create events
  return cpra::loss_fwd_bwd(g, cfg, Z, ldz, P, ldp, dZ, lddz, terms, ws,
                            CPRA_LOSS_NOALLOC_SCRATCH_BYTES, cpra::as_stream(stream));
}

}  // extern "C"

namespace cpra {
cpra_status check_loss_cfg_public(const cpra_csr* g, const cpra_loss_cfg* cfg) {
  return check_loss_cfg(g, cfg);
}
}  // namespace cpra
