// Graph preparation, graph-segmented fixed-order reductions and small utility kernels.
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>

#include "common.hpp"

namespace cpra {

// inv_deg[i] = 1/|N(i)| (0 if isolated); wdeg[i] = sum_j A_ij in CSR order.
__global__ void k_csr_prepare(int n, const int32_t* __restrict__ row_ptr,
                              const float* __restrict__ weight, float* __restrict__ inv_deg,
                              float* __restrict__ wdeg) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int a = row_ptr[i], b = row_ptr[i + 1];
  if (inv_deg) inv_deg[i] = b > a ? 1.0f / float(b - a) : 0.0f;
  if (wdeg) {
    float s;
    if (weight) {
      s = 0.0f;
      for (int k = a; k < b; ++k) s += weight[k];
    } else {
      s = float(b - a);
    }
    wdeg[i] = s;
  }
}

// col_inv_deg[e] = inv_deg[col_idx[e]]: the column scale of M^T = A D^-1 per CSR entry.
__global__ void k_csr_prepare_col(int64_t nnz, const int32_t* __restrict__ col_idx,
                                  const float* __restrict__ inv_deg, float* __restrict__ col_inv_deg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) col_inv_deg[e] = inv_deg[col_idx[e]];
}

// Exclusive scan of ceil(n_g / R) over graphs by one block, in chunks of blockDim.
__global__ void k_item_ptr(int n_graphs, const int32_t* __restrict__ graph_ptr, int R,
                           int32_t* __restrict__ item_ptr) {
  __shared__ int32_t buf[256];
  int carry = 0;
  for (int base = 0; base < n_graphs; base += 256) {
    int g = base + threadIdx.x;
    int cnt = 0;
    if (g < n_graphs) {
      int ng = graph_ptr[g + 1] - graph_ptr[g];
      cnt = (ng + R - 1) / R;
    }
    buf[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // Hillis-Steele inclusive scan
      int v = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += v;
      __syncthreads();
    }
    if (g < n_graphs) item_ptr[g + 1] = carry + buf[threadIdx.x];
    int total = buf[255];
    __syncthreads();
    carry += total;
  }
  if (threadIdx.x == 0) item_ptr[0] = 0;
}

int64_t max_items(const cpra_csr* g, int R) {
  return ceil_div(g->n_nodes, R) + (g->n_graphs > 1 ? g->n_graphs : 0) + 1;
}

cpra_status launch_item_ptr(const cpra_csr* g, int R, int32_t* item_ptr, hipStream_t stream) {
  if (g->n_graphs <= 1) return CPRA_OK;
  hipLaunchKernelGGL(k_item_ptr, dim3(1), dim3(256), 0, stream, g->n_graphs, g->graph_ptr, R,
                     item_ptr);
  CPRA_CHECK_LAUNCH("item_ptr");
  return CPRA_OK;
}

// One block per (graph, column): sum the graph's items in FP64, each thread a
// fixed strided subset, then a fixed-shape tree.
__global__ void k_segment_reduce(int n_graphs, int n_nodes, int R, const int32_t* __restrict__ item_ptr,
                                 const float* __restrict__ part, const double* __restrict__ part64,
                                 int64_t items_cap, int ncols, double* __restrict__ out,
                                 int32_t* advance) {
  int g = blockIdx.x;
  int c = blockIdx.y;
  if (advance && g == 0 && c == 0 && threadIdx.x == 0) advance[0] = advance[0] + 1;
  int b0, b1;
  if (item_ptr == nullptr) {
    b0 = 0;
    b1 = (n_nodes + R - 1) / R;
  } else {
    b0 = item_ptr[g];
    b1 = item_ptr[g + 1];
  }
  double acc = 0.0;
  if (part64) {
    const double* col = part64 + (int64_t)c * items_cap;
    for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) acc += col[b];
  } else {
    const float* col = part + (int64_t)c * items_cap;
    for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) acc += (double)col[b];
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)g * ncols + c] = sh[0];
}

cpra_status launch_segment_reduce(const cpra_csr* g, int R, const int32_t* item_ptr,
                                  const float* part, const double* part64, int64_t items_cap,
                                  int ncols, double* out, hipStream_t stream, int32_t* advance) {
  if (ncols <= 0) return CPRA_OK;
  dim3 grid(g->n_graphs, ncols);
  ProfScope ps("segment_reduce", stream, 0.0, (double)ncols * items_cap * (part64 ? 8.0 : 4.0));
  hipLaunchKernelGGL(k_segment_reduce, grid, dim3(256), 0, stream, g->n_graphs, g->n_nodes, R,
                     g->n_graphs > 1 ? item_ptr : nullptr, part, part64, items_cap, ncols, out,
                     advance);
  CPRA_CHECK_LAUNCH("segment_reduce");
  return CPRA_OK;
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

cpra_status fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t stream) {
  if (n <= 0 || p == nullptr) return CPRA_OK;
  hipLaunchKernelGGL(k_fill_i64, dim3(ceil_div(n, 256)), dim3(256), 0, stream, p, n, v);
  CPRA_CHECK_LAUNCH("fill_i64");
  return CPRA_OK;
}

__global__ void k_zero_i32(int32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

bool persistent_enabled() {
  const char* e = getenv("CPRA_PERSISTENT");
  return e != nullptr && e[0] == '1';
}

cpra_status zero_queue(int32_t* queue, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, stream, queue, kQueueInts);
  CPRA_CHECK_LAUNCH("zero_queue");
  return CPRA_OK;
}

int resident_blocks(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(dev, kernel);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int n = cus * per_cu;
  cache[key] = n;
  return n;
}

__global__ void k_increment(int32_t* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[0] = c[0] + 1;
}

cpra_status increment_counter(int32_t* counter, hipStream_t stream) {
  hipLaunchKernelGGL(k_increment, dim3(1), dim3(64), 0, stream, counter);
  CPRA_CHECK_LAUNCH("increment_counter");
  return CPRA_OK;
}

// sigmoid without cancellation: e = exp(-|z|); P = z >= 0 ? 1/(1+e) : e/(1+e).
__global__ void k_sigmoid(int n, int S, const float* __restrict__ Z, int64_t ldz,
                          float* __restrict__ P, int64_t ldp) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)n * S;
  if (idx >= total) return;
  int64_t i = idx / S;
  int s = (int)(idx - i * S);
  float z = Z[i * ldz + s];
  float e = expf(-fabsf(z));
  float r = 1.0f / (1.0f + e);
  P[i * ldp + s] = z >= 0.0f ? r : e * r;
}

cpra_status sigmoid(int N, int S, const float* Z, int64_t ldz, float* P, int64_t ldp,
                    hipStream_t stream) {
  int64_t total = (int64_t)N * S;
  if (total == 0) return CPRA_OK;
  {
    ProfScope ps("sigmoid", stream, 0.0, 8.0 * (double)total);
    hipLaunchKernelGGL(k_sigmoid, dim3(ceil_div(total, 256)), dim3(256), 0, stream, N, S, Z, ldz, P,
                       ldp);
  }
  CPRA_CHECK_LAUNCH("sigmoid");
  return CPRA_OK;
}

}  // namespace cpra

extern "C" {

cpra_status cpra_csr_prepare(const cpra_csr* g, float* inv_deg, float* wdeg, cpra_stream_t stream) {
  CPRA_CHECK(cpra::check_csr(g, "csr_prepare", false, false));
  if (g->n_nodes == 0) return CPRA_OK;
  hipLaunchKernelGGL(cpra::k_csr_prepare, dim3(cpra::ceil_div(g->n_nodes, 256)), dim3(256), 0,
                     cpra::as_stream(stream), g->n_nodes, g->row_ptr, g->weight, inv_deg, wdeg);
  CPRA_CHECK_LAUNCH("csr_prepare");
  return CPRA_OK;
}

cpra_status cpra_csr_prepare_col(const cpra_csr* g, float* col_inv_deg, cpra_stream_t stream) {
  CPRA_CHECK(cpra::check_csr(g, "csr_prepare_col", false, false));
  if (g->nnz == 0) return CPRA_OK;
  if (g->inv_deg == nullptr || col_inv_deg == nullptr)
    CPRA_FAIL(CPRA_ERR_NULL, "csr_prepare_col: g->inv_deg or col_inv_deg is NULL");
  hipLaunchKernelGGL(cpra::k_csr_prepare_col, dim3((unsigned)cpra::ceil_div(g->nnz, 256)), dim3(256),
                     0, cpra::as_stream(stream), g->nnz, g->col_idx, g->inv_deg, col_inv_deg);
  CPRA_CHECK_LAUNCH("csr_prepare_col");
  return CPRA_OK;
}

cpra_status cpra_sigmoid(int32_t N, int32_t S, const float* Z, int64_t ldz, float* P, int64_t ldp,
                         cpra_stream_t stream) {
  if (N < 0 || S < 1 || ldz < S || ldp < S) CPRA_FAIL(CPRA_ERR_SHAPE, "sigmoid: bad shape");
  if (N > 0 && (Z == nullptr || P == nullptr)) CPRA_FAIL(CPRA_ERR_NULL, "sigmoid: NULL pointer");
  return cpra::sigmoid(N, S, Z, ldz, P, ldp, cpra::as_stream(stream));
}

}  // extern "C"
