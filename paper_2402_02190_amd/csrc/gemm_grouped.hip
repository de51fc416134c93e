// GEMMs over the graphs of a block-diagonal batch in which every graph has its
// own weights (batched CPRA with one network per instance): the group-mode
// instantiations of the MFMA GEMM kernel (gemm_kernel.hpp), the row-tile maps
// that keep every row tile inside one graph, and the public grouped entry
// point.  The planning, tuning and launch code is shared with the plain GEMM
// (gemm.hip, via gemm_batch).
#include "gemm_kernel.hpp"

namespace cpra {

namespace {

constexpr int kBm[3] = {32, 64, 128};  // row-tile heights of the GEMM configurations

// Exclusive scans of ceil(n_g / BM) over the graphs for the three heights at
// once, by one block of 256 threads in chunks of 256 graphs.
__global__ void k_row_tile_ptr(int n_graphs, const int32_t* __restrict__ graph_ptr,
                               int32_t* __restrict__ p32, int32_t* __restrict__ p64,
                               int32_t* __restrict__ p128) {
  __shared__ int32_t buf[3][256];
  int carry[3] = {0, 0, 0};
  int32_t* out[3] = {p32, p64, p128};
  for (int base = 0; base < n_graphs; base += 256) {
    const int g = base + threadIdx.x;
    const int ng = g < n_graphs ? graph_ptr[g + 1] - graph_ptr[g] : 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) buf[i][threadIdx.x] = (ng + kBm[i] - 1) / kBm[i];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // Hillis-Steele inclusive scans
      int v[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) v[i] = threadIdx.x >= off ? buf[i][threadIdx.x - off] : 0;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 3; ++i) buf[i][threadIdx.x] += v[i];
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (g < n_graphs) out[i][g + 1] = carry[i] + buf[i][threadIdx.x];
      carry[i] += buf[i][255];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) p32[0] = p64[0] = p128[0] = 0;
}

// map[t] = {graph, first row, end row, 0} of row tile t (height kBm[blockIdx.y]),
// or {-1, 0, 0, 0} past the last tile.
struct MapArgs {
  const int32_t* tile_ptr[3];
  int4* map[3];
  int count[3];
};

__global__ void k_row_tile_map(int n_graphs, int n_nodes, const int32_t* __restrict__ graph_ptr,
                               MapArgs a) {
  const int i = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count[i]) return;
  int g, r0, r1;
  a.map[i][t] = item_rows(t, n_graphs, n_nodes, graph_ptr, a.tile_ptr[i], kBm[i], &g, &r0, &r1)
                    ? make_int4(g, r0, r1, 0)
                    : make_int4(-1, 0, 0, 0);
}

inline size_t tile_ptr_bytes(const cpra_csr* g) {
  return align_up((size_t)(std::max(g->n_graphs, 1) + 1) * sizeof(int32_t), 256);
}

}  // namespace

size_t group_rows_bytes(const cpra_csr* g) {
  size_t b = 0;
  for (int i = 0; i < 3; ++i)
    b += tile_ptr_bytes(g) + align_up((size_t)max_items(g, kBm[i]) * sizeof(int4), 256);
  return b;
}

namespace {

void rows_layout(const cpra_csr* g, void* ws, MapArgs* a) {
  char* p = static_cast<char*>(ws);
  for (int i = 0; i < 3; ++i) {
    a->tile_ptr[i] = reinterpret_cast<int32_t*>(p);
    p += tile_ptr_bytes(g);
    a->map[i] = reinterpret_cast<int4*>(p);
    a->count[i] = (int)max_items(g, kBm[i]);
    p += align_up((size_t)a->count[i] * sizeof(int4), 256);
  }
}

}  // namespace

cpra_status group_rows_view(const cpra_csr* g, void* ws, GroupRows* out) {
  MapArgs a{};
  rows_layout(g, ws, &a);
  for (int i = 0; i < 3; ++i) {
    out->map[i] = a.map[i];
    out->count[i] = a.count[i];
  }
  return CPRA_OK;
}

cpra_status group_rows_build(const cpra_csr* g, void* ws, GroupRows* out, hipStream_t st) {
  const bool batch = g->n_graphs > 1;
  MapArgs a{};
  rows_layout(g, ws, &a);
  CPRA_CHECK(group_rows_view(g, ws, out));
  int max_count = 0;
  for (int i = 0; i < 3; ++i) max_count = std::max(max_count, a.count[i]);
  if (batch) {
    hipLaunchKernelGGL(k_row_tile_ptr, dim3(1), dim3(256), 0, st, g->n_graphs, g->graph_ptr,
                       const_cast<int32_t*>(a.tile_ptr[0]), const_cast<int32_t*>(a.tile_ptr[1]),
                       const_cast<int32_t*>(a.tile_ptr[2]));
    CPRA_CHECK_LAUNCH("row_tile_ptr");
  }
  if (max_count > 0) {
    hipLaunchKernelGGL(k_row_tile_map, dim3((unsigned)ceil_div(max_count, 256), 3), dim3(256), 0, st,
                       batch ? g->n_graphs : 1, g->n_nodes, batch ? g->graph_ptr : nullptr, a);
    CPRA_CHECK_LAUNCH("row_tile_map");
  }
  return CPRA_OK;
}

namespace gemmk {

void launch_grouped(int mode, bool a_t, bool b_t, int cfg, LaunchArgs& args, hipStream_t stream) {
  (void)a_t;  // checked by gemm_batch: mode 1 takes A [rows, K], mode 2 A^T B
  if (mode == 1) {
    if (b_t) launch_any<false, true, 1>(cfg, args, stream);
    else launch_any<false, false, 1>(cfg, args, stream);
  } else {
    launch_any<true, false, 2>(cfg, args, stream);
  }
}

}  // namespace gemmk

namespace {

cpra_status grouped_problem(const cpra_csr* g, int32_t mode, int32_t trans_b, int32_t M, int32_t N,
                            int32_t K, const float* A, int64_t lda, const float* B, int64_t ldb,
                            int64_t b_stride, float* C, int64_t ldc, int64_t c_stride,
                            const float* bias, int64_t bias_stride, float* bias_grad,
                            int64_t bg_stride, int32_t relu, GemmProblem* q) {
  CPRA_CHECK(check_csr(g, "gemm_grouped", false, false));
  const int G = std::max(g->n_graphs, 1);
  if (M < 0 || N < 0 || K < 0) CPRA_FAIL(CPRA_ERR_SHAPE, "gemm_grouped: negative size");
  *q = GemmProblem{};
  if (mode == CPRA_GROUP_ROWS) {
    if (M != g->n_nodes) CPRA_FAIL(CPRA_ERR_SHAPE, "gemm_grouped: rows mode needs M = n_nodes");
    if (bias_grad) CPRA_FAIL(CPRA_ERR_PARAM, "gemm_grouped: rows mode has no bias gradient");
    if (lda < K || ldc < N || ldb < (trans_b ? K : N))
      CPRA_FAIL(CPRA_ERR_SHAPE, "gemm_grouped: leading dimension too small");
    const int64_t b_span = trans_b ? (int64_t)(N > 0 ? N - 1 : 0) * ldb + K
                                   : (int64_t)(K > 0 ? K - 1 : 0) * ldb + N;
    if (G > 1 && (b_stride < b_span || (bias && bias_stride < N)))
      CPRA_FAIL(CPRA_ERR_SHAPE, "gemm_grouped: per-graph strides overlap");
  } else if (mode == CPRA_GROUP_K) {
    if (K != g->n_nodes) CPRA_FAIL(CPRA_ERR_SHAPE, "gemm_grouped: K mode needs K = n_nodes");
    if (trans_b || bias || relu) CPRA_FAIL(CPRA_ERR_PARAM, "gemm_grouped: K mode is a plain A^T B");
    if (lda < M || ldb < N || ldc < N) CPRA_FAIL(CPRA_ERR_SHAPE, "gemm_grouped: leading dimension too small");
    const int64_t c_span = (int64_t)(M > 0 ? M - 1 : 0) * ldc + N;
    if (G > 1 && (c_stride < c_span || (bias_grad && bg_stride < M)))
      CPRA_FAIL(CPRA_ERR_SHAPE, "gemm_grouped: per-graph strides overlap");
  } else {
    CPRA_FAIL(CPRA_ERR_PARAM, "gemm_grouped: unknown mode %d", mode);
  }
  if (M > 0 && N > 0) {
    if (C == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "gemm_grouped: C is NULL");
    if (K > 0 && (A == nullptr || B == nullptr)) CPRA_FAIL(CPRA_ERR_NULL, "gemm_grouped: A or B is NULL");
  }
  q->piece[0] = GemmPiece{A, B, lda, ldb, K};
  q->n_pieces = 1;
  q->C = C;
  q->ldc = ldc;
  q->M = M;
  q->N = N;
  q->bias = bias;
  q->relu = relu;
  q->bias_grad = bias_grad;
  q->group_mode = mode;
  q->n_groups = G;
  q->group_ptr = g->n_graphs > 1 ? g->graph_ptr : nullptr;
  q->b_stride = b_stride;
  q->c_stride = c_stride;
  q->bias_stride = bias_stride;
  q->bg_stride = bg_stride;
  return CPRA_OK;
}

}  // namespace

}  // namespace cpra

extern "C" {

size_t cpra_gemm_grouped_workspace_bytes(const cpra_csr* g, int32_t mode, int32_t M, int32_t N,
                                         int32_t with_bias_grad) {
  using namespace cpra;
  if (g == nullptr || g->n_nodes < 0) return 0;
  if (mode == CPRA_GROUP_ROWS) return group_rows_bytes(g);
  if (mode != CPRA_GROUP_K || M < 0 || N < 0) return 0;
  GemmProblem q{};
  q.piece[0].K = g->n_nodes;
  q.n_pieces = 1;
  q.M = M;
  q.N = N;
  q.bias_grad = with_bias_grad ? reinterpret_cast<float*>(1) : nullptr;  // shape only
  q.group_mode = CPRA_GROUP_K;
  q.n_groups = std::max(g->n_graphs, 1);
  return gemm_batch_workspace_bytes(true, false, &q, 1);
}

cpra_status cpra_gemm_grouped(const cpra_csr* g, int32_t mode, int32_t trans_b, int32_t M,
                              int32_t N, int32_t K, const float* A, int64_t lda, const float* B,
                              int64_t ldb, int64_t b_stride, float* C, int64_t ldc,
                              int64_t c_stride, const float* bias, int64_t bias_stride,
                              float* bias_grad, int64_t bg_stride, int32_t relu, void* ws,
                              size_t ws_bytes, cpra_stream_t stream) {
  using namespace cpra;
  if (g == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "gemm_grouped: graph is NULL");
  GemmProblem q;
  CPRA_CHECK(grouped_problem(g, mode, trans_b, M, N, K, A, lda, B, ldb, b_stride, C, ldc, c_stride,
                             bias, bias_stride, bias_grad, bg_stride, relu, &q));
  hipStream_t st = as_stream(stream);
  if (M == 0 || (N == 0 && bias_grad == nullptr)) return CPRA_OK;
  if (mode == CPRA_GROUP_ROWS) {
    const size_t need = group_rows_bytes(g);
    if (ws == nullptr || ws_bytes < need)
      CPRA_FAIL(CPRA_ERR_WORKSPACE, "gemm_grouped: workspace %zu < %zu bytes", ws_bytes, need);
    GroupRows rows;
    CPRA_CHECK(group_rows_build(g, ws, &rows, st));
    q.rows = &rows;
    return gemm_batch(false, trans_b != 0, &q, 1, nullptr, 0, st);
  }
  return gemm_batch(true, false, &q, 1, ws, ws_bytes, st);
}

}  // extern "C"
