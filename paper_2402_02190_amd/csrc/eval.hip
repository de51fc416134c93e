// Threshold rounding and exact integer evaluation of the S solutions
// (training-setting appendix: P <= 0.5 -> 0, P > 0.5 -> 1, i.e. x = [Z > 0];
// objective table; Sec. 4.1 Evaluation Metrics; Proposition 3.2).
//
// Same lane layout as the loss kernel: 64/LPR nodes per wavefront, the LPR
// lanes of a node cover its heads.  Each edge {i, j} is visited from its
// smaller endpoint only.  Integer counts are summed per block and added with
// 64-bit integer atomics (exact, so order does not matter); weighted values
// (the cut weight of MaxCut, the set weight of weighted MIS) go through
// per-item FP64 partials and the fixed-order segmented reduction.  With
// per-head edge weights head s is evaluated on its own instance: only edges
// with a nonzero weight in head s count, with that weight.
#include "common.hpp"

namespace cpra {

namespace {

// x = [Z > 0] decided on the bit pattern: +0 and negatives (sign bit set) give
// 0, every positive value from the smallest subnormal to +inf gives 1, NaN 0.
// The result does not depend on the wavefront's denormal mode.
__device__ inline bool rounds_to_one(float z) {
  const int32_t b = __float_as_int(z);
  return b > 0 && b <= 0x7f800000;
}

struct EvalArgs {
  int n, S, problem, lpr_log2;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* weight;
  const float* Z;
  int64_t ldz;
  uint8_t* X;
  int64_t ldx;
  int64_t* value;
  int64_t* viol;
  int64_t* pairham;
  double* wpart;
  int64_t items_cap;
  int n_graphs;
  const int32_t* graph_ptr;
  const int32_t* item_ptr;
  int R;
  const float* node_w;  // MIS node weights or null (weight 1)
  int64_t ld_nw;        // 0: one weight per node
  const float* edge_w;  // per-head edge weights [nnz, ld_ew] or null
  int64_t ld_ew;
};

template <typename T>
__device__ inline T xor_sum(T v, int from_mask, int to_mask) {
  for (int m = from_mask; m < to_mask; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <int NC>
__global__ __launch_bounds__(256) void k_round_eval(EvalArgs a) {
  int g, r0, r1;
  if (!item_rows(blockIdx.x, a.n_graphs, a.n, a.graph_ptr, a.item_ptr, a.R, &g, &r0, &r1)) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lpr = 1 << a.lpr_log2;
  const int rpw = 64 >> a.lpr_log2;
  const int sub = lane >> a.lpr_log2;
  const int cl = lane & (lpr - 1);
  const int S = a.S;
  const bool mis = a.problem == CPRA_MIS;

  int c_val[NC], c_vio[NC];
  double c_w[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    c_val[c] = 0;
    c_vio[c] = 0;
    c_w[c] = 0.0;
  }
  long long pair = 0;

  for (int base = r0; base < r1; base += 4 * rpw) {
    const int row = base + wave * rpw + sub;
    const bool active = row < r1;
    int x[NC];
    int k_row = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int s = c * lpr + cl;
      x[c] = (active && s < S && rounds_to_one(a.Z[(int64_t)row * a.ldz + s])) ? 1 : 0;
      k_row += x[c];
      if (active && s < S && a.X) a.X[(int64_t)row * a.ldx + s] = (uint8_t)x[c];
    }
    if (active) {
      if (mis) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int s = c * lpr + cl;
          c_val[c] += x[c];
          if (x[c] && s < S)
            c_w[c] += a.node_w ? (double)a.node_w[a.ld_nw ? (int64_t)row * a.ld_nw + s
                                                            : (int64_t)row]
                               : 1.0;
        }
      }
      const int beg = a.row_ptr[row], end = a.row_ptr[row + 1];
      for (int k = beg; k < end; ++k) {
        const int j = a.col_idx[k];
        if (j <= row) continue;
        const float w0 = a.weight ? a.weight[k] : 1.0f;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int s = c * lpr + cl;
          if (s >= S) continue;
          const float w = a.edge_w ? a.edge_w[(int64_t)k * a.ld_ew + s] : w0;
          if (a.edge_w && w == 0.0f) continue;  // not an edge of head s's instance
          const int xj = rounds_to_one(a.Z[(int64_t)j * a.ldz + s]) ? 1 : 0;
          if (mis) {
            c_vio[c] += x[c] & xj;
          } else if (x[c] != xj) {
            c_val[c] += 1;
            c_w[c] += (double)w;
          }
        }
      }
    }
    k_row = xor_sum<int>(k_row, 1, lpr);
    if (active && cl == 0) pair += (long long)k_row * (long long)(S - k_row);
  }

  __shared__ int sh_val[4][NC * 64];
  __shared__ int sh_vio[4][NC * 64];
  __shared__ double sh_w[4][NC * 64];
  __shared__ long long sh_pair[4];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int v1 = xor_sum<int>(c_val[c], lpr, 64);
    const int v2 = xor_sum<int>(c_vio[c], lpr, 64);
    const double v3 = xor_sum<double>(c_w[c], lpr, 64);
    if (sub == 0) {
      sh_val[wave][c * lpr + cl] = v1;
      sh_vio[wave][c * lpr + cl] = v2;
      sh_w[wave][c * lpr + cl] = v3;
    }
  }
  const long long pr = xor_sum<long long>(pair, 1, 64);
  if (lane == 0) sh_pair[wave] = pr;
  __syncthreads();
  for (int s = threadIdx.x; s < NC * lpr; s += 256) {
    if (s >= S) continue;
    const long long v1 = (long long)sh_val[0][s] + sh_val[1][s] + sh_val[2][s] + sh_val[3][s];
    const long long v2 = (long long)sh_vio[0][s] + sh_vio[1][s] + sh_vio[2][s] + sh_vio[3][s];
    if (a.value && v1) atomicAdd(reinterpret_cast<unsigned long long*>(a.value + (int64_t)g * S + s),
                                 (unsigned long long)v1);
    if (a.viol && v2) atomicAdd(reinterpret_cast<unsigned long long*>(a.viol + (int64_t)g * S + s),
                                (unsigned long long)v2);
    if (a.wpart)
      a.wpart[(int64_t)s * a.items_cap + blockIdx.x] =
          ((sh_w[0][s] + sh_w[1][s]) + sh_w[2][s]) + sh_w[3][s];
  }
  if (threadIdx.x == 0 && a.pairham) {
    const long long t = sh_pair[0] + sh_pair[1] + sh_pair[2] + sh_pair[3];
    if (t) atomicAdd(reinterpret_cast<unsigned long long*>(a.pairham + g), (unsigned long long)t);
  }
}

struct EvalGeom {
  int lpr, lpr_log2, nc, R;
  int64_t items_cap;
};

EvalGeom eval_geom(const cpra_csr* g, int S) {
  EvalGeom G{};
  G.lpr = 1;
  while (G.lpr < S && G.lpr < 64) G.lpr <<= 1;
  while ((1 << G.lpr_log2) < G.lpr) ++G.lpr_log2;
  int need = (int)ceil_div(S, G.lpr);
  G.nc = 1;
  while (G.nc < need) G.nc <<= 1;
  G.R = 4 * (64 / G.lpr) * 2;
  G.items_cap = max_items(g, G.R);
  return G;
}

size_t eval_ws(const cpra_csr* g, int S, size_t* item_off, size_t* part_off) {
  EvalGeom G = eval_geom(g, S);
  size_t off = 0;
  *item_off = off;
  off += align_up((size_t)(g->n_graphs + 1) * sizeof(int32_t), 256);
  *part_off = off;
  off += align_up((size_t)S * G.items_cap * sizeof(double), 256);
  return off;
}

}  // namespace

}  // namespace cpra

extern "C" {

size_t cpra_round_eval_workspace_bytes(const cpra_csr* g, int32_t S) {
  if (g == nullptr || S < 1) return 0;
  size_t a, b;
  return cpra::eval_ws(g, S, &a, &b);
}

cpra_status cpra_round_eval(const cpra_csr* g, int32_t problem, int32_t S, const float* Z,
                            int64_t ldz, uint8_t* X, int64_t ldx, int64_t* value,
                            int64_t* violations, double* wvalue, int64_t* pair_hamming,
                            const float* node_weight, int64_t ld_node_weight,
                            const float* edge_weight, int64_t ld_edge_weight, void* ws,
                            size_t ws_bytes, cpra_stream_t stream) {
  using namespace cpra;
  CPRA_CHECK(check_csr(g, "round_eval", false, false));
  if (problem != CPRA_MIS && problem != CPRA_MAXCUT)
    CPRA_FAIL(CPRA_ERR_PARAM, "round_eval: unknown problem %d", problem);
  if (S < 1 || S > 1024) CPRA_FAIL(CPRA_ERR_PARAM, "round_eval: S = %d outside 1..1024", S);
  if (g->n_nodes > 0 && Z == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "round_eval: Z is NULL");
  if (ldz < S || (X && ldx < S)) CPRA_FAIL(CPRA_ERR_SHAPE, "round_eval: leading dimension < S");
  if (node_weight && problem != CPRA_MIS)
    CPRA_FAIL(CPRA_ERR_PARAM, "round_eval: node weights are defined for MIS only");
  if (node_weight && ld_node_weight != 0 && ld_node_weight < S)
    CPRA_FAIL(CPRA_ERR_SHAPE, "round_eval: ld_node_weight must be 0 or >= S");
  if (edge_weight && ld_edge_weight < S)
    CPRA_FAIL(CPRA_ERR_SHAPE, "round_eval: ld_edge_weight must be >= S");
  size_t item_off, part_off;
  size_t need = eval_ws(g, S, &item_off, &part_off);
  if (ws == nullptr || ws_bytes < need)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "round_eval: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = as_stream(stream);
  EvalGeom G = eval_geom(g, S);
  char* base = static_cast<char*>(ws);
  int32_t* item_ptr = reinterpret_cast<int32_t*>(base + item_off);
  double* wpart = wvalue ? reinterpret_cast<double*>(base + part_off) : nullptr;
  CPRA_CHECK(launch_item_ptr(g, G.R, item_ptr, st));
  CPRA_CHECK(fill_i64(value, (int64_t)g->n_graphs * S, 0, st));
  CPRA_CHECK(fill_i64(violations, (int64_t)g->n_graphs * S, 0, st));
  CPRA_CHECK(fill_i64(pair_hamming, g->n_graphs, 0, st));
  EvalArgs a{};
  a.n = g->n_nodes;
  a.S = S;
  a.problem = problem;
  a.lpr_log2 = G.lpr_log2;
  a.row_ptr = g->row_ptr;
  a.col_idx = g->col_idx;
  a.weight = g->weight;
  a.Z = Z;
  a.ldz = ldz;
  a.X = X;
  a.ldx = ldx;
  a.value = value;
  a.viol = violations;
  a.pairham = pair_hamming;
  a.wpart = wpart;
  a.items_cap = G.items_cap;
  a.n_graphs = g->n_graphs;
  a.graph_ptr = g->n_graphs > 1 ? g->graph_ptr : nullptr;
  a.item_ptr = item_ptr;
  a.R = G.R;
  a.node_w = node_weight;
  a.ld_nw = ld_node_weight;
  a.edge_w = edge_weight;
  a.ld_ew = ld_edge_weight;
  const int blocks = (int)G.items_cap;
  ProfScope ps("round_eval", st, 0.0,
               4.0 * (double)g->n_nodes * S + (X ? (double)g->n_nodes * S : 0.0) +
                   4.0 * (double)g->nnz * (edge_weight ? 1.0 + S : 1.0) + 4.0 * g->n_nodes);
  switch (G.nc) {
#define CPRA_EVAL_CASE(NCV)                                                          \
  case NCV:                                                                          \
    hipLaunchKernelGGL(k_round_eval<NCV>, dim3(blocks), dim3(256), 0, st, a);        \
    break;
    CPRA_EVAL_CASE(1)
    CPRA_EVAL_CASE(2)
    CPRA_EVAL_CASE(4)
    CPRA_EVAL_CASE(8)
    CPRA_EVAL_CASE(16)
#undef CPRA_EVAL_CASE
    default:
      CPRA_FAIL(CPRA_ERR_PARAM, "round_eval: S too large");
  }
  CPRA_CHECK_LAUNCH("round_eval");
  if (wvalue)
    CPRA_CHECK(launch_segment_reduce(g, G.R, item_ptr, nullptr, wpart, G.items_cap, S, wvalue, st));
  return CPRA_OK;
}

}  // extern "C"
