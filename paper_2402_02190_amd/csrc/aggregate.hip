// Mean aggregation M X and its transpose M^T X over a CSR graph (GNN appendix:
// Aggregate step with the 1/|N(v)| normalisation).
//
// Layout: a 64-lane wavefront holds 64/LPR rows; the LPR lanes of one row
// cover its columns in VEC-float vectors, NC vectors per lane.  Each lane
// walks its row's neighbour list in chunks (the index loads are uniform across
// the row's lanes) and issues a chunk's row gathers together; every gathered
// row segment is read as contiguous, coalesced vectors.  Sums run in CSR
// order, so results are deterministic.
#include <algorithm>

#include "common.hpp"

namespace cpra {

namespace {

template <int VEC>
struct Vec;
template <>
struct Vec<1> {
  using T = float;
  __device__ static T zero() { return 0.0f; }
  __device__ static void axpy(T& acc, float s, const T& x) { acc += s * x; }
  __device__ static void add(T& acc, const T& x) { acc += x; }
  __device__ static void scale(T& acc, float s) { acc *= s; }
};
template <>
struct Vec<2> {
  using T = float2;
  __device__ static T zero() { return make_float2(0.f, 0.f); }
  __device__ static void axpy(T& acc, float s, const T& x) { acc.x += s * x.x; acc.y += s * x.y; }
  __device__ static void add(T& acc, const T& x) { acc.x += x.x; acc.y += x.y; }
  __device__ static void scale(T& acc, float s) { acc.x *= s; acc.y *= s; }
};
template <>
struct Vec<4> {
  using T = float4;
  __device__ static T zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  __device__ static void axpy(T& acc, float s, const T& x) {
    acc.x += s * x.x; acc.y += s * x.y; acc.z += s * x.z; acc.w += s * x.w;
  }
  __device__ static void add(T& acc, const T& x) {
    acc.x += x.x; acc.y += x.y; acc.z += x.z; acc.w += x.w;
  }
  __device__ static void scale(T& acc, float s) { acc.x *= s; acc.y *= s; acc.z *= s; acc.w *= s; }
};

template <int VEC>
__device__ inline float comp(const typename Vec<VEC>::T& v, int e) {
  if constexpr (VEC == 1) return v;
  else if constexpr (VEC == 2) return e == 0 ? v.x : v.y;
  else return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}
template <int VEC>
__device__ inline void set_comp(typename Vec<VEC>::T& v, int e, float x) {
  if constexpr (VEC == 1) v = x;
  else if constexpr (VEC == 2) { if (e == 0) v.x = x; else v.y = x; }
  else { if (e == 0) v.x = x; else if (e == 1) v.y = x; else if (e == 2) v.z = x; else v.w = x; }
}

constexpr double kStreamOutBytes = 32.0 * 1024 * 1024;

struct AggArgs {
  int n;
  int width;
  int lpr_log2;
  int relu;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* inv_deg;
  const float* col_inv_deg;  // inv_deg of each entry's column, or null (gathered instead)
  const float* X;
  int64_t ldx;
  float* Y;
  int64_t ldy;
  const float* add;
  int64_t ld_add;
  const float* bias;
  const float* mask;
  int64_t ld_mask;
  float* sig_out;  // optional sigmoid(Y) [N, width] (ld_sig)
  int64_t ld_sig;
  const float* add2;  // optional second addend [N, width] (ld_add2)
  int64_t ld_add2;
  int32_t* queue;  // persistent launches: the work queue (kQueueInts counters)
  int units;       // persistent launches: row blocks of 4 wavefronts
  int chunk;       // persistent launches: row blocks per dequeue
  int stream_out;  // streaming output stores and index loads (tables larger than L2)
};

// A streaming (nontemporal) store of one VEC-float vector.  Above kStreamOutBytes of
// output (more than the 8 XCDs' L2 together) the output rows, which this launch does
// not read again, are stored this way so that they take no L2 lines from the gathered
// table, and the index stream is read the same way: C3 (a 182 MB table) 1.775 ->
// 1.751 ms per step, C4 (51 MB) and C3s (22 MB) unchanged; on C2 (10 MB) it cost 0.8%.
template <int VEC>
__device__ inline void store_nt(const typename Vec<VEC>::T& v, float* p) {
  if constexpr (VEC == 1) {
    __builtin_nontemporal_store(v, p);
  } else {
    typedef float nv __attribute__((ext_vector_type(VEC)));
    nv x;
#pragma unroll
    for (int e = 0; e < VEC; ++e) x[e] = comp<VEC>(v, e);
    __builtin_nontemporal_store(x, reinterpret_cast<nv*>(p));
  }
}

__device__ inline float sigmoid_of(float z) {
  const float e = expf(-fabsf(z));
  const float r = 1.0f / (1.0f + e);
  return z >= 0.0f ? r : e * r;
}

// Row block `unit` (4 wavefronts of 64/LPR rows each).
template <int VEC, int NC, bool TRANS>
__device__ __forceinline__ void agg_unit(const AggArgs& a, int unit) {
  using V = typename Vec<VEC>::T;
  using O = Vec<VEC>;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lpr = 1 << a.lpr_log2;
  const int sub = lane >> a.lpr_log2;
  const int cl = lane & (lpr - 1);
  const int rpw = 64 >> a.lpr_log2;
  const int row = (unit * 4 + wave) * rpw + sub;
  if (row >= a.n) return;
  const int units = a.width / VEC;

  V acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = O::zero();

  // Neighbours in chunks of CH (all index loads, then all row gathers, then
  // the adds in CSR order); the entries of a last partial chunk past the
  // row's end are not gathered and add an exact zero instead (the sums never
  // hold -0, so x + 0 = x), so a row costs two dependent round trips per
  // chunk and there is no serial tail.
  constexpr int CH = NC <= 2 ? 8 : 4;
  const int beg = a.row_ptr[row];
  const int end = a.row_ptr[row + 1];
  for (int k = beg; k < end; k += CH) {
    const int n_in = min(CH, end - k);
    int j[CH];
    float s[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i)
      j[i] = a.stream_out ? __builtin_nontemporal_load(a.col_idx + min(k + i, end - 1))
                          : a.col_idx[min(k + i, end - 1)];
#pragma unroll
    for (int i = 0; i < CH; ++i)
      s[i] = !TRANS ? 1.f
                    : a.col_inv_deg ? a.col_inv_deg[min(k + i, end - 1)] : a.inv_deg[j[i]];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int u = c * lpr + cl;
      if (u < units) {
        V x[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i)  // padded entries are not gathered
          x[i] = i < n_in ? *reinterpret_cast<const V*>(a.X + (int64_t)j[i] * a.ldx + u * VEC)
                          : O::zero();
#pragma unroll
        for (int i = 0; i < CH; ++i) {  // and add an exact zero (no branch between the adds)
          if constexpr (TRANS) O::axpy(acc[c], s[i], x[i]); else O::add(acc[c], x[i]);
        }
      }
    }
  }
  const float rs = TRANS ? 1.f : a.inv_deg[row];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int u = c * lpr + cl;
    if (u >= units) continue;
    V r = acc[c];
    if constexpr (!TRANS) O::scale(r, rs);
    if (a.add) O::add(r, *reinterpret_cast<const V*>(a.add + (int64_t)row * a.ld_add + u * VEC));
    if (a.add2) O::add(r, *reinterpret_cast<const V*>(a.add2 + (int64_t)row * a.ld_add2 + u * VEC));
    if (a.bias) O::add(r, *reinterpret_cast<const V*>(a.bias + u * VEC));
    if (a.relu || a.mask) {
      V mk = O::zero();
      if (a.mask) mk = *reinterpret_cast<const V*>(a.mask + (int64_t)row * a.ld_mask + u * VEC);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        float x = comp<VEC>(r, e);
        if (a.relu) x = fmaxf(x, 0.0f);
        if (a.mask && !(comp<VEC>(mk, e) > 0.0f)) x = 0.0f;
        set_comp<VEC>(r, e, x);
      }
    }
    if (a.stream_out) store_nt<VEC>(r, a.Y + (int64_t)row * a.ldy + u * VEC);
    else *reinterpret_cast<V*>(a.Y + (int64_t)row * a.ldy + u * VEC) = r;
    if (a.sig_out) {
      V sg;
#pragma unroll
      for (int e = 0; e < VEC; ++e) set_comp<VEC>(sg, e, sigmoid_of(comp<VEC>(r, e)));
      *reinterpret_cast<V*>(a.sig_out + (int64_t)row * a.ld_sig + u * VEC) = sg;
    }
  }
}

// One block per row block, in XCD order.
template <int VEC, int NC, bool TRANS>
__global__ __launch_bounds__(256) void k_aggregate(AggArgs a) {
  agg_unit<VEC, NC, TRANS>(a, xcd_unit(blockIdx.x, gridDim.x));
}

// Persistent: at most the resident blocks, each taking row blocks from the queue.
template <int VEC, int NC, bool TRANS>
__global__ __launch_bounds__(256) void k_aggregate_persistent(AggArgs a) {
  __shared__ int s_chunk;
  const int chunks = (a.units + a.chunk - 1) / a.chunk;
  for (bool first = true;; first = false) {
    if (threadIdx.x == 0) s_chunk = queue_next(a.queue, chunks, first);
    __syncthreads();
    const int c = s_chunk;
    if (c < 0) break;  // uniform across the block
    const int u1 = min(a.units, (c + 1) * a.chunk);
    for (int u = c * a.chunk; u < u1; ++u) agg_unit<VEC, NC, TRANS>(a, u);
    __syncthreads();  // s_chunk is rewritten by the next dequeue
  }
}

inline bool aligned(const void* p, int bytes) {
  return p == nullptr || (reinterpret_cast<uintptr_t>(p) % bytes) == 0;
}

template <int VEC, bool TRANS>
cpra_status launch_nc(const AggArgs& a, int nc, int blocks, hipStream_t stream, int64_t nnz) {
  // compulsory bytes: X once, Y written, add/mask read, CSR, inv_deg
  const double nw = (double)a.n * a.width * 4.0;
  const double bytes = nw * (2.0 + (a.add ? 1.0 : 0.0) + (a.add2 ? 1.0 : 0.0) +
                             (a.mask ? 1.0 : 0.0) + (a.sig_out ? 1.0 : 0.0)) +
                       4.0 * (double)nnz * (TRANS && a.col_inv_deg ? 2.0 : 1.0) +
                       8.0 * (double)a.n + 4.0;
  ProfScope ps(TRANS ? "aggregate_transposed" : "aggregate", stream, 0.0, bytes,
               4.0 * (double)nnz * a.width);
  if (a.queue) CPRA_CHECK(zero_queue(a.queue, stream));
  switch (nc) {
#define CPRA_AGG_CASE(NCV)                                                                     \
  case NCV:                                                                                    \
    if (a.queue) {                                                                             \
      const int cap = resident_blocks(reinterpret_cast<const void*>(                           \
                                          &k_aggregate_persistent<VEC, NCV, TRANS>), 256);     \
      AggArgs ap = a;                                                                          \
      const int grid = std::min(a.units, cap);                                                 \
      ap.chunk = queue_chunk(a.units, grid);                                                   \
      hipLaunchKernelGGL((k_aggregate_persistent<VEC, NCV, TRANS>), dim3(grid), dim3(256), 0,  \
                         stream, ap);                                                          \
    } else {                                                                                   \
      hipLaunchKernelGGL((k_aggregate<VEC, NCV, TRANS>), dim3(blocks), dim3(256), 0, stream, a); \
    }                                                                                          \
    break;
    CPRA_AGG_CASE(1)
    CPRA_AGG_CASE(2)
    CPRA_AGG_CASE(4)
    CPRA_AGG_CASE(8)
    CPRA_AGG_CASE(16)
#undef CPRA_AGG_CASE
    default:
      CPRA_FAIL(CPRA_ERR_SHAPE, "aggregate: width too large");
  }
  CPRA_CHECK_LAUNCH("aggregate");
  return CPRA_OK;
}

}  // namespace

cpra_status aggregate(const cpra_csr* g, bool transpose, int width, const float* X, int64_t ldx,
                      float* Y, int64_t ldy, const float* add, int64_t ld_add, const float* bias,
                      bool relu, const float* mask, int64_t ld_mask, hipStream_t stream,
                      float* sig_out, int64_t ld_sig, const float* add2, int64_t ld_add2,
                      int32_t* queue) {
  if (g->n_nodes == 0 || width == 0) return CPRA_OK;
  int vec = 1;
  for (int v : {4, 2}) {
    int vb = v * 4;
    if (width % v == 0 && ldx % v == 0 && ldy % v == 0 && (add == nullptr || ld_add % v == 0) &&
        (mask == nullptr || ld_mask % v == 0) && (sig_out == nullptr || ld_sig % v == 0) &&
        (add2 == nullptr || ld_add2 % v == 0) && aligned(X, vb) && aligned(Y, vb) &&
        aligned(add, vb) && aligned(bias, vb) && aligned(mask, vb) && aligned(sig_out, vb) &&
        aligned(add2, vb)) {
      vec = v;
      break;
    }
  }
  int units = width / vec;
  // On graphs of mean degree >= 12, two vectors per lane (twice the rows, and
  // their independent gathers, in flight per wavefront) measured faster: the
  // 20-regular 100,000-node aggregation 167 -> 151 us.  On sparser graphs
  // (mean degree ~7) the one-vector layout was faster (150 vs 178 us).
  const int per_lane = g->nnz >= 12 * (int64_t)g->n_nodes ? 2 : 1;
  int lpr = 1;
  while (per_lane * lpr < units && lpr < 64) lpr <<= 1;
  int lpr_log2 = 0;
  while ((1 << lpr_log2) < lpr) ++lpr_log2;
  int need = (int)ceil_div(units, lpr);
  int nc = 1;
  while (nc < need) nc <<= 1;
  if (nc > 16) CPRA_FAIL(CPRA_ERR_SHAPE, "aggregate: width %d exceeds 4096", width);
  int rows_per_block = 4 * (64 / lpr);
  const int units_rb = (int)ceil_div(g->n_nodes, rows_per_block);
  int blocks = (int)xcd_grid(units_rb);
  AggArgs a{g->n_nodes, width, lpr_log2, relu ? 1 : 0, g->row_ptr, g->col_idx, g->inv_deg,
            g->col_inv_deg, X, ldx, Y, ldy, add, ld_add, bias, mask, ld_mask, sig_out, ld_sig, add2, ld_add2,
            (queue && persistent_enabled()) ? queue : nullptr, units_rb, 1,
            (double)g->n_nodes * width * 4.0 > kStreamOutBytes ? 1 : 0};
  if (transpose) {
    if (vec == 4) return launch_nc<4, true>(a, nc, blocks, stream, g->nnz);
    if (vec == 2) return launch_nc<2, true>(a, nc, blocks, stream, g->nnz);
    return launch_nc<1, true>(a, nc, blocks, stream, g->nnz);
  }
  if (vec == 4) return launch_nc<4, false>(a, nc, blocks, stream, g->nnz);
  if (vec == 2) return launch_nc<2, false>(a, nc, blocks, stream, g->nnz);
  return launch_nc<1, false>(a, nc, blocks, stream, g->nnz);
}

}  // namespace cpra

extern "C" cpra_status cpra_aggregate_mean(const cpra_csr* g, int32_t transpose, int32_t width,
                                           const float* X, int64_t ldx, float* Y, int64_t ldy,
                                           const float* add, int64_t ld_add, const float* bias,
                                           int32_t relu, const float* mask, int64_t ld_mask,
                                           cpra_stream_t stream) {
  CPRA_CHECK(cpra::check_csr(g, "aggregate_mean", true, false));
  if (width < 0) CPRA_FAIL(CPRA_ERR_SHAPE, "aggregate_mean: width < 0");
  if (g->n_nodes > 0 && width > 0) {
    if (X == nullptr || Y == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "aggregate_mean: X or Y is NULL");
    if (ldx < width || ldy < width || (add && ld_add < width) || (mask && ld_mask < width))
      CPRA_FAIL(CPRA_ERR_SHAPE, "aggregate_mean: leading dimension smaller than width");
    if (X == Y) CPRA_FAIL(CPRA_ERR_PARAM, "aggregate_mean: X must not alias Y");
  }
  return cpra::aggregate(g, transpose != 0, width, X, ldx, Y, ldy, add, ld_add, bias, relu != 0,
                         mask, ld_mask, cpra::as_stream(stream));
}
