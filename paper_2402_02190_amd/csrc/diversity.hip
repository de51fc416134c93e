// Solution-diversity analytics over the S rounded solutions: pairwise Hamming
// distances, their histogram over the S(S-1)/2 pairs and the number of distinct
// solutions (Sec. 4.1 Evaluation Metrics; the Hamming-distance and unique-
// solution analyses of the diversity appendix).  The pairwise distances are
// the O(N S^2) quantity that Proposition 3.2 lets the loss avoid; here they
// are computed once per evaluation, on bit-packed columns: each solution is
// packed into ceil(N/64) 64-bit words and d(s, l) is a sum of popcounts of
// XORed words.  Everything is integer and exact.
#include "common.hpp"

namespace cpra {

namespace {

// B[s * W + w] = bits of rows 64 w .. 64 w + 63 of column s (row r -> bit r % 64).
__global__ void k_pack_columns(int N, int S, int W, const uint8_t* __restrict__ X, int64_t ldx,
                               uint64_t* __restrict__ B) {
  const int s = blockIdx.y * blockDim.x + threadIdx.x;
  const int w = blockIdx.x;
  if (s >= S) return;
  uint64_t bits = 0;
  const int r0 = w * 64;
  const int rn = min(64, N - r0);
  for (int r = 0; r < rn; ++r)
    if (X[(int64_t)(r0 + r) * ldx + s]) bits |= (uint64_t)1 << r;
  B[(int64_t)s * W + w] = bits;
}

// One thread per ordered pair (s, l) of a 16 x 16 tile.
__global__ void k_pair_distances(int S, int W, const uint64_t* __restrict__ B, int32_t* __restrict__ D,
                                 int64_t ldd, int64_t* __restrict__ hist) {
  const int s = blockIdx.y * 16 + threadIdx.y;
  const int l = blockIdx.x * 16 + threadIdx.x;
  if (s >= S || l >= S) return;
  const uint64_t* bs = B + (int64_t)s * W;
  const uint64_t* bl = B + (int64_t)l * W;
  int d = 0;
  for (int w = 0; w < W; ++w) d += __popcll(bs[w] ^ bl[w]);
  D[(int64_t)s * ldd + l] = d;
  if (hist && s < l) atomicAdd(reinterpret_cast<unsigned long long*>(hist + d), 1ull);
}

// n_unique = number of heads s with no earlier head l < s at distance 0.
__global__ void k_count_unique(int S, const int32_t* __restrict__ D, int64_t ldd,
                               int32_t* __restrict__ n_unique) {
  __shared__ int cnt[1024];
  const int s = threadIdx.x;
  int first = 0;
  if (s < S) {
    first = 1;
    for (int l = 0; l < s; ++l)
      if (D[(int64_t)l * ldd + s] == 0) {
        first = 0;
        break;
      }
  }
  cnt[threadIdx.x] = first;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (threadIdx.x < off) cnt[threadIdx.x] += cnt[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_unique = cnt[0];
}

size_t div_ws(int N, int S, bool need_d, size_t* d_off) {
  const int W = (int)ceil_div(N, 64);
  size_t off = align_up((size_t)S * W * sizeof(uint64_t), 256);
  *d_off = off;
  if (need_d) off += align_up((size_t)S * S * sizeof(int32_t), 256);
  return std::max<size_t>(off, 256);
}

}  // namespace

}  // namespace cpra

extern "C" {

size_t cpra_pairwise_hamming_workspace_bytes(int32_t N, int32_t S) {
  if (N < 0 || S < 1 || S > 1024) return 0;
  size_t d;
  return cpra::div_ws(N, S, true, &d);
}

cpra_status cpra_pairwise_hamming(int32_t N, int32_t S, const uint8_t* X, int64_t ldx, int32_t* D,
                                  int64_t ldd, int64_t* hist, int32_t* n_unique, void* ws,
                                  size_t ws_bytes, cpra_stream_t stream) {
  using namespace cpra;
  if (N < 0) CPRA_FAIL(CPRA_ERR_SHAPE, "pairwise_hamming: N < 0");
  if (S < 1 || S > 1024) CPRA_FAIL(CPRA_ERR_PARAM, "pairwise_hamming: S = %d outside 1..1024", S);
  if (ldx < S || (D && ldd < S)) CPRA_FAIL(CPRA_ERR_SHAPE, "pairwise_hamming: leading dimension < S");
  if (N > 0 && X == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "pairwise_hamming: X is NULL");
  const bool need_d = D == nullptr && (hist || n_unique);
  size_t d_off;
  const size_t need = div_ws(N, S, need_d, &d_off);
  if (ws == nullptr || ws_bytes < need)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "pairwise_hamming: workspace %zu < %zu bytes", ws_bytes, need);
  if (!D && !hist && !n_unique) return CPRA_OK;
  hipStream_t st = as_stream(stream);
  const int W = (int)ceil_div(N, 64);
  uint64_t* B = reinterpret_cast<uint64_t*>(ws);
  int32_t* Dm = D ? D : reinterpret_cast<int32_t*>(static_cast<char*>(ws) + d_off);
  const int64_t ld = D ? ldd : S;
  if (hist) CPRA_CHECK(fill_i64(hist, (int64_t)N + 1, 0, st));
  {
    ProfScope ps("pack_columns", st, 0.0, (double)N * S + 8.0 * S * W);
    if (W > 0)
      hipLaunchKernelGGL(k_pack_columns, dim3(W, (unsigned)ceil_div(S, 256)), dim3(256), 0, st, N, S,
                         W, X, ldx, B);
    CPRA_CHECK_LAUNCH("pack_columns");
  }
  {
    ProfScope ps("pair_distances", st, 0.0, 4.0 * S * S + 8.0 * S * W);
    const unsigned t = (unsigned)ceil_div(S, 16);
    hipLaunchKernelGGL(k_pair_distances, dim3(t, t), dim3(16, 16), 0, st, S, W, B, Dm, ld, hist);
    CPRA_CHECK_LAUNCH("pair_distances");
  }
  if (n_unique) {
    hipLaunchKernelGGL(k_count_unique, dim3(1), dim3(1024), 0, st, S, Dm, ld, n_unique);
    CPRA_CHECK_LAUNCH("count_unique");
  }
  return CPRA_OK;
}

}  // extern "C"
