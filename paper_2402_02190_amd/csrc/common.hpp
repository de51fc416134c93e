// Internal declarations shared by the libcpra translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "cpra.h"

namespace cpra {

// ---- error reporting ------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

#define CPRA_FAIL(code, ...)         \
  do {                               \
    ::cpra::set_error(__VA_ARGS__);  \
    return (code);                   \
  } while (0)

#define CPRA_CHECK(expr)                   \
  do {                                     \
    cpra_status _s = (expr);               \
    if (_s != CPRA_OK) return _s;          \
  } while (0)

#define CPRA_CHECK_LAUNCH(name)                                                           \
  do {                                                                                    \
    hipError_t _e = hipGetLastError();                                                    \
    if (_e != hipSuccess)                                                                 \
      CPRA_FAIL(CPRA_ERR_HIP, "%s: kernel launch failed: %s", name, hipGetErrorString(_e)); \
  } while (0)

// Brackets one kernel launch with timing events while profiling is on
// (see profile.hip); `flops` / `bytes` are the launch's algorithmic work.
// While a ProfSuspend lives on a thread, ProfScope on that thread records
// nothing (creates no events): for entry points that must not allocate.
struct ProfSuspend {
  ProfSuspend();
  ~ProfSuspend();
  ProfSuspend(const ProfSuspend&) = delete;
  ProfSuspend& operator=(const ProfSuspend&) = delete;
};

class ProfScope {
 public:
  // gather: bytes of rows gathered through an index (a sparse product's neighbour
  // rows), which caches may serve; 0 for kernels without gathers
  ProfScope(const char* name, hipStream_t stream, double flops, double bytes, double gather = 0.0);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  bool active_;
  hipStream_t stream_;
  size_t idx_ = 0;
};

inline hipStream_t as_stream(cpra_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---- graph checks shared by entry points ----------------------------------
cpra_status check_csr(const cpra_csr* g, const char* who, bool need_inv_deg, bool need_wdeg);

// ---- row blocks ("items") that never cross a graph boundary ----------------
// A reduction over rows that must be segmented by graph assigns rows to items
// of at most `rows_per_item` consecutive rows inside one graph.  For a single
// graph item b covers rows [b*R, min(N, (b+1)*R)).  For a batch the item
// offsets per graph are an exclusive scan of ceil(n_g / R), computed on the
// device into `item_ptr` [n_graphs+1].
int64_t max_items(const cpra_csr* g, int rows_per_item);
cpra_status launch_item_ptr(const cpra_csr* g, int rows_per_item, int32_t* item_ptr,
                            hipStream_t stream);

// Device helper: the graph and row range of item b.  Returns false when b is
// past the last item.
// XCD-aware block order.  The hardware deals consecutive block ids round-robin
// to the 8 XCDs, each with its own L2.  With a grid of 8 * per blocks, block b
// takes work unit (b % 8) * per + b / 8, a bijection on [0, 8 * per): each XCD
// then works through one contiguous eighth of the units, so the rows of one
// graph of a batch (and their neighbours' rows) are gathered into one L2 instead
// of eight.
__device__ inline int xcd_unit(int b, int grid) { return (b & 7) * (grid >> 3) + (b >> 3); }
inline int64_t xcd_grid(int64_t units) { return (units + 7) / 8 * 8; }

// ---- persistent launches over a row-block work queue -----------------------
// A persistent launch runs at most as many blocks as the device holds at once
// (resident_blocks) over `chunks` chunks of work units (row blocks, or
// graph-segmented items).  The chunks form 8 queues, queue x holding the x-th
// contiguous eighth: the hardware deals block b to XCD b % 8, so block b takes
// the chunks of queue b % 8 -- an XCD works through its own eighth, as in the
// XCD-ordered launches.  Each block's first chunk is fixed (its rank among the
// blocks of its XCD), later ones come from the queue's counter, and a block
// whose queue is empty takes from the other queues, which balances uneven
// chunks.  A queue is kQueueInts int32 of device memory: 8 counters, each in
// its own 128-byte line, zeroed on the launch's stream right before the launch
// (zero_queue).  Every dequeue attempt advances a counter, so each block leaves
// after at most chunks + 8 attempts.
constexpr int kQueueStride = 32;  // ints between two counters (128 bytes)
constexpr int kQueueInts = 8 * kQueueStride;
bool persistent_enabled();  // CPRA_PERSISTENT=1 in the environment (read at every call)
cpra_status zero_queue(int32_t* queue, hipStream_t stream);
// Blocks of `threads` threads of `kernel` that the current device holds at once
// (compute units x blocks per unit; cached per device and kernel).
int resident_blocks(const void* kernel, int threads);

struct QueueRange {
  int lo, n, fixed;  // first chunk, chunks, chunks handed out without the counter
};
__device__ inline QueueRange queue_range(int x, int chunks) {
  const int per = (chunks + 7) >> 3;
  QueueRange r;
  r.lo = min(chunks, x * per);
  r.n = min(chunks, r.lo + per) - r.lo;
  r.fixed = ((int)gridDim.x - x + 7) >> 3;  // blocks dealt to XCD x
  return r;
}

// The calling block's next chunk, or -1 when every queue is empty (one thread
// of the block calls it; `first` is true on the block's first call).
__device__ inline int queue_next(int32_t* q, int chunks, bool first) {
  const int home = blockIdx.x & 7;
  if (first) {
    const QueueRange r = queue_range(home, chunks);
    const int rank = blockIdx.x >> 3;
    if (rank < r.n) return r.lo + rank;
  }
  for (int i = 0; i < 8; ++i) {
    const int x = (home + i) & 7;
    const QueueRange r = queue_range(x, chunks);
    if (r.n <= r.fixed) continue;  // all of it handed out as first chunks
    int32_t* c = q + x * kQueueStride;
    if (__atomic_load_n(c, __ATOMIC_RELAXED) >= r.n - r.fixed) continue;  // drained
    const int t = atomicAdd(c, 1);
    if (t < r.n - r.fixed) return r.lo + r.fixed + t;
  }
  return -1;
}

// Units per chunk: about four chunks per block of a grid of `grid`.
inline int queue_chunk(int units, int grid) {
  const int c = units / (4 * (grid > 0 ? grid : 1));
  return c > 1 ? c : 1;
}

__device__ inline bool item_rows(int b, int n_graphs, int n_nodes, const int32_t* graph_ptr,
                                 const int32_t* item_ptr, int R, int* g_out, int* r0, int* r1) {
  if (graph_ptr == nullptr) {
    int lo = b * R;
    if (lo >= n_nodes) return false;
    *g_out = 0;
    *r0 = lo;
    *r1 = min(n_nodes, lo + R);
    return true;
  }
  if (b >= item_ptr[n_graphs]) return false;
  int lo = 0, hi = n_graphs;  // find g with item_ptr[g] <= b < item_ptr[g+1]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (item_ptr[mid] <= b) lo = mid; else hi = mid;
  }
  int local = b - item_ptr[lo];
  int gs = graph_ptr[lo], ge = graph_ptr[lo + 1];
  *g_out = lo;
  *r0 = gs + local * R;
  *r1 = min(ge, *r0 + R);
  return true;
}

// Fixed-order FP64 reduction of per-item partial columns into per-graph sums:
// out[g*ncols + c] = sum over items of graph g of part[c*items_cap + item].
// advance (optional): block (0, 0) also increments *advance once.
cpra_status launch_segment_reduce(const cpra_csr* g, int rows_per_item, const int32_t* item_ptr,
                                  const float* part, const double* part64, int64_t items_cap,
                                  int ncols, double* out, hipStream_t stream,
                                  int32_t* advance = nullptr);

// ---- kernels used by the model orchestration ------------------------------
struct GemmPiece {
  const float* A;
  const float* B;
  int64_t lda, ldb;
  int K;
};

// Row tiles of a block-diagonal batch that never cross a graph boundary, for
// each row-tile height BM = 32, 64, 128: {graph, first row, end row, 0} per
// tile, graph -1 past the last tile.  Built on the device by group_rows_build.
struct GroupRows {
  const int4* map[3];
  int count[3];
};
size_t group_rows_bytes(const cpra_csr* g);
cpra_status group_rows_build(const cpra_csr* g, void* ws, GroupRows* out, hipStream_t stream);
// The maps that group_rows_build wrote into ws earlier (no launch).
cpra_status group_rows_view(const cpra_csr* g, void* ws, GroupRows* out);

struct GemmProblem {
  GemmPiece piece[2];  // the contraction runs over piece[0].K then piece[1].K
  int n_pieces;
  float* C;
  int64_t ldc;
  int M, N;
  const float* bias;   // [N] or null
  const float* mask;   // [M, N] (ld_mask): output zeroed where mask <= 0; or null
  int64_t ld_mask;
  float beta;
  int relu;
  float* bias_grad;  // [M]: also write sum_k op(A)[row, k], or null
  float* sig_out;    // [M, N] (ld_sig): also write sigmoid(C), or null
  int64_t ld_sig;
  const float* add;  // [M, N] (ld_add): added to the result after the bias, or null
  int64_t ld_add;
  // One weight set per graph of a block-diagonal batch (all problems of a
  // launch alike; n_groups <= 1 is the plain product):
  //  1 = by rows: rows of A and C split by graph (A [M, K] with M = batch rows),
  //      graph g's B and bias at g * b_stride / g * bias_stride floats;
  //  2 = by K: C_g = A[rows of g]^T B[rows of g] (A^T B with K = batch rows),
  //      graph g's C and bias_grad at g * c_stride / g * bg_stride floats.
  int group_mode;
  int n_groups;
  const int32_t* group_ptr;  // [n_groups + 1] graph row offsets (device; mode 2)
  const GroupRows* rows;     // row tiles (mode 1)
  int64_t b_stride, c_stride, bias_stride, bg_stride;
};

// Up to 4 independent problems in one launch, all with the same operand layout.
// a_t: A stored [K, M]; b_t: B stored [N, K].
size_t gemm_batch_workspace_bytes(bool a_t, bool b_t, const GemmProblem* probs, int n);
cpra_status gemm_batch(bool a_t, bool b_t, const GemmProblem* probs, int n, void* ws,
                       size_t ws_bytes, hipStream_t stream);

// sig_out (optional) receives sigmoid(Y) with leading dimension ld_sig.
// add2 (optional) is a second addend [N, width] (ld_add2), applied after add.
// queue (optional, kQueueInts ints of device memory used by this stream only):
// with persistent launches enabled, the aggregation runs as a persistent launch
// over that work queue.
cpra_status aggregate(const cpra_csr* g, bool transpose, int width, const float* X, int64_t ldx,
                      float* Y, int64_t ldy, const float* add, int64_t ld_add, const float* bias,
                      bool relu, const float* mask, int64_t ld_mask, hipStream_t stream,
                      float* sig_out = nullptr, int64_t ld_sig = 0, const float* add2 = nullptr,
                      int64_t ld_add2 = 0, int32_t* queue = nullptr);

cpra_status sigmoid(int N, int S, const float* Z, int64_t ldz, float* P, int64_t ldp,
                    hipStream_t stream);

size_t loss_workspace_bytes(const cpra_csr* g, int S, bool need_p);
// want_terms: the partials for the terms are needed (by a later loss_terms_reduce)
// even if `terms` itself is NULL here.
cpra_status loss_fwd_bwd(const cpra_csr* g, const cpra_loss_cfg* cfg, const float* Z, int64_t ldz,
                         const float* P, int64_t ldp, float* dZ, int64_t lddz, double* terms,
                         void* ws, size_t ws_bytes, hipStream_t stream, bool want_terms = false);
cpra_status check_loss_cfg_public(const cpra_csr* g, const cpra_loss_cfg* cfg);

// With step_counter, Adam's t = *step_counter + t_offset.  stop_flag (optional,
// device): the update is skipped while *stop_flag != 0.
cpra_status adam_step(int64_t n, float* params, const float* grads, float* m, float* v,
                      const cpra_adam_cfg* cfg, int32_t t, const int32_t* step_counter,
                      hipStream_t stream, int t_offset = 1, const int32_t* stop_flag = nullptr);

// Early stopping (early_stop.hip): checks of the config, and the per-step
// update of the device state from the step's complete per-graph terms, which
// also advances the step counter unless the rule has fired.
cpra_status check_early_stop_cfg(const cpra_early_stop_cfg* es);
cpra_status early_stop_update(const cpra_csr* g, const cpra_loss_cfg* lc, const double* terms,
                              const cpra_early_stop_cfg* es, int32_t* counter, hipStream_t stream);
cpra_status check_adam_cfg(const cpra_adam_cfg* cfg);

// Side stream of the current device (see streams.hip).  fork_to makes the side
// stream wait for everything enqueued so far on `main`; join_from makes `main`
// wait for everything enqueued so far on the side stream.  fork_mark +
// fork_wait is fork_to in two halves: the side stream waits for what `main` had
// enqueued at the mark, so main-stream work enqueued between the two is
// captured ahead of the side work (in a captured graph the main chain then
// keeps its hardware queue) without the side work waiting for it.
struct SideStream {
  hipStream_t stream;
  hipEvent_t ev[2];
};
bool overlap_enabled();  // unless CPRA_OVERLAP=0 in the environment
cpra_status get_side_stream(SideStream** out);
cpra_status fork_to(SideStream* s, hipStream_t main);
cpra_status fork_mark(SideStream* s, hipStream_t main);
cpra_status fork_wait(SideStream* s);
cpra_status join_from(SideStream* s, hipStream_t main);

// The loss in two launches: the fused per-node kernel (dZ + per-item partials
// in the workspace) and the per-graph FP64 reduction of the partials.
// advance (optional): one thread of the reduction increments *advance.
cpra_status loss_terms_reduce(const cpra_csr* g, const cpra_loss_cfg* cfg, double* terms, void* ws,
                              hipStream_t stream, int32_t* advance = nullptr);

cpra_status fill_i64(int64_t* p, int64_t n, int64_t value, hipStream_t stream);
cpra_status increment_counter(int32_t* counter, hipStream_t stream);

}  // namespace cpra
