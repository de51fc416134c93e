// FP32 GEMM on the CDNA matrix cores (v_mfma_f32_32x32x2f32) for the GNN's
// dense weight products: forward X W^T, input gradient dY W and weight
// gradient dY^T X.
//
// Block tile BM x BN x 16 staged through LDS (double buffered, one barrier per
// K step), 4 wavefronts in a 2 x 2 grid, each owning (BM/64) x (BN/64) tiles
// of 32 x 32 accumulators.  Operands stored K-contiguous are transposed into
// the [k][mn] LDS layout while being written, so every MFMA operand read is
// one ds_read_b32 of 32 consecutive floats per half-wave.
//
// One launch runs up to four independent problems (grid.y = problem x split).
// A problem's contraction may be split in two K pieces with separate
// pointers, so [X | MX] [Ws | Wn]^T is a single GEMM without a concatenated
// copy.  Split-K writes FP32 partial tiles that a second kernel sums in a
// fixed order (deterministic), applying the epilogue.
#include "common.hpp"

namespace cpra {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BK = 16;
constexpr int kMaxProblems = 4;

struct ProbDev {
  const float* A[2];
  const float* B[2];
  int64_t lda[2], ldb[2];
  int K[2];
  int vecA[2], vecB[2];
  int n_pieces;
  float* C;
  int64_t ldc;
  int M, N;
  const float* bias;
  const float* mask;
  int64_t ld_mask;
  float beta;
  int relu;
  int tiles_m, tiles_n;
  int64_t part_off;  // float offset of this problem's split-K partials
};

struct LaunchArgs {
  ProbDev p[kMaxProblems];
  int n_prob;
  int splits;
  int grid_x;  // blocks per problem-split (a multiple of 8)
  float* partial;
};

template <int R, bool KCONTIG>
struct Tile {
  static constexpr int PAD = KCONTIG ? 2 : 4;
  static constexpr int LD = R + PAD;  // LDS row stride (floats) of the [BK][R] tile
  static constexpr int NV = R * BK / 4 / 256;
  static_assert(NV >= 1, "tile too small for 256 threads");
  float4 reg[NV];

  __device__ inline void load(const float* __restrict__ X, int64_t ld, int mn0, int mn_lim, int k0,
                              int k_lim, bool vec_ok, int tid) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = tid + v * 256;
      if constexpr (KCONTIG) {
        const int r = idx / (BK / 4);
        const int kq = (idx % (BK / 4)) * 4;
        const int gm = mn0 + r, gk = k0 + kq;
        if (vec_ok && gm < mn_lim && gk + 3 < k_lim) {
          reg[v] = *reinterpret_cast<const float4*>(X + (int64_t)gm * ld + gk);
        } else {
          const bool rok = gm < mn_lim;
          const float* p = X + (int64_t)(rok ? gm : 0) * ld;
          reg[v].x = (rok && gk + 0 < k_lim) ? p[gk + 0] : 0.f;
          reg[v].y = (rok && gk + 1 < k_lim) ? p[gk + 1] : 0.f;
          reg[v].z = (rok && gk + 2 < k_lim) ? p[gk + 2] : 0.f;
          reg[v].w = (rok && gk + 3 < k_lim) ? p[gk + 3] : 0.f;
        }
      } else {
        const int k = idx / (R / 4);
        const int rq = (idx % (R / 4)) * 4;
        const int gk = k0 + k, gm = mn0 + rq;
        if (vec_ok && gk < k_lim && gm + 3 < mn_lim) {
          reg[v] = *reinterpret_cast<const float4*>(X + (int64_t)gk * ld + gm);
        } else {
          const bool kok = gk < k_lim;
          const float* p = X + (int64_t)(kok ? gk : 0) * ld;
          reg[v].x = (kok && gm + 0 < mn_lim) ? p[gm + 0] : 0.f;
          reg[v].y = (kok && gm + 1 < mn_lim) ? p[gm + 1] : 0.f;
          reg[v].z = (kok && gm + 2 < mn_lim) ? p[gm + 2] : 0.f;
          reg[v].w = (kok && gm + 3 < mn_lim) ? p[gm + 3] : 0.f;
        }
      }
    }
  }

  __device__ inline void store(float* __restrict__ Xs, int tid) const {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = tid + v * 256;
      if constexpr (KCONTIG) {
        const int r = idx / (BK / 4);
        const int kq = (idx % (BK / 4)) * 4;
        Xs[(kq + 0) * LD + r] = reg[v].x;
        Xs[(kq + 1) * LD + r] = reg[v].y;
        Xs[(kq + 2) * LD + r] = reg[v].z;
        Xs[(kq + 3) * LD + r] = reg[v].w;
      } else {
        const int k = idx / (R / 4);
        const int rq = (idx % (R / 4)) * 4;
        *reinterpret_cast<float4*>(Xs + k * LD + rq) = reg[v];
      }
    }
  }
};

// A_T: A stored [K, M] (M contiguous); otherwise [M, K].
// B_T: B stored [N, K] (K contiguous); otherwise [K, N].
template <int BM, int BN, bool A_T, bool B_T>
__global__ __launch_bounds__(256) void k_gemm(LaunchArgs args) {
  constexpr int TM = BM / 64;  // 32x32 tiles per wave along M
  constexpr int TN = BN / 64;
  using TA = Tile<BM, !A_T>;
  using TB = Tile<BN, B_T>;
  __shared__ __attribute__((aligned(16))) float As[2][BK * TA::LD];
  __shared__ __attribute__((aligned(16))) float Bs[2][BK * TB::LD];

  const int prob = blockIdx.y / args.splits;
  const int split = blockIdx.y % args.splits;
  const ProbDev& P = args.p[prob];
  // XCD-aware order: hardware deals consecutive block ids round-robin to the 8
  // XCDs; give each XCD a contiguous run of tiles (neighbouring N tiles share
  // the A panel in that XCD's L2).
  const int per_xcd = args.grid_x / 8;
  const int tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (tile >= P.tiles_m * P.tiles_n) return;
  const int tm_idx = tile / P.tiles_n;
  const int tn_idx = tile % P.tiles_n;
  const int m0 = tm_idx * BM;
  const int n0 = tn_idx * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int half = lane >> 5, l32 = lane & 31;

  const int nt0 = (P.K[0] + BK - 1) / BK;
  const int nt1 = P.n_pieces > 1 ? (P.K[1] + BK - 1) / BK : 0;
  const int KT = nt0 + nt1;
  const int per_split = (KT + args.splits - 1) / args.splits;
  const int kt_begin = min(KT, split * per_split);
  const int kt_end = min(KT, kt_begin + per_split);

  floatx16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  TA ta;
  TB tb;
  auto load = [&](int kt) {
    const int pc = kt < nt0 ? 0 : 1;
    const int k0 = (kt - (pc ? nt0 : 0)) * BK;
    ta.load(P.A[pc], P.lda[pc], m0, P.M, k0, P.K[pc], P.vecA[pc] != 0, tid);
    tb.load(P.B[pc], P.ldb[pc], n0, P.N, k0, P.K[pc], P.vecB[pc] != 0, tid);
  };

  if (kt_begin < kt_end) {
    load(kt_begin);
    ta.store(As[0], tid);
    tb.store(Bs[0], tid);
    __syncthreads();
    for (int kt = kt_begin; kt < kt_end; ++kt) {
      const int cur = (kt - kt_begin) & 1;
      const bool more = kt + 1 < kt_end;
      if (more) load(kt + 1);
      const float* as = As[cur];
      const float* bs = Bs[cur];
#pragma unroll
      for (int kk = 0; kk < BK / 2; ++kk) {
        const int kr = 2 * kk + half;
        float a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = as[kr * TA::LD + (wm * TM + i) * 32 + l32];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = bs[kr * TB::LD + (wn * TN + j) * 32 + l32];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      if (more) {
        ta.store(As[cur ^ 1], tid);
        tb.store(Bs[cur ^ 1], tid);
      }
      __syncthreads();
    }
  }

  // Accumulator layout of the 32x32 MFMA: register r of lane l holds
  // D[8*(r/4) + 4*(l/32) + r%4][l%32].
  const bool partial = args.splits > 1;
  float* part = partial ? args.partial + P.part_off + (int64_t)split * P.M * P.N : nullptr;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + (wn * TN + j) * 32 + l32;
      if (col >= P.N) continue;
      const float bv = (!partial && P.bias) ? P.bias[col] : 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + (wm * TM + i) * 32 + (r >> 2) * 8 + half * 4 + (r & 3);
        if (row >= P.M) continue;
        float v = acc[i][j][r];
        if (partial) {
          part[(int64_t)row * P.N + col] = v;
        } else {
          float* cp = P.C + (int64_t)row * P.ldc + col;
          if (P.beta != 0.f) v += P.beta * *cp;
          v += bv;
          if (P.relu) v = fmaxf(v, 0.f);
          if (P.mask && !(P.mask[(int64_t)row * P.ld_mask + col] > 0.f)) v = 0.f;
          *cp = v;
        }
      }
    }
  }
}

// Sum split-K partials in split order and apply the epilogue.
__global__ void k_gemm_splitk_reduce(LaunchArgs args) {
  const int prob = blockIdx.y;
  const ProbDev& P = args.p[prob];
  const int64_t total = (int64_t)P.M * P.N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const float* part = args.partial + P.part_off;
  float v = 0.f;
  for (int s = 0; s < args.splits; ++s) v += part[(int64_t)s * total + idx];
  const int row = (int)(idx / P.N);
  const int col = (int)(idx - (int64_t)row * P.N);
  float* cp = P.C + (int64_t)row * P.ldc + col;
  if (P.beta != 0.f) v += P.beta * *cp;
  if (P.bias) v += P.bias[col];
  if (P.relu) v = fmaxf(v, 0.f);
  if (P.mask && !(P.mask[(int64_t)row * P.ld_mask + col] > 0.f)) v = 0.f;
  *cp = v;
}

inline bool vec_ok(const float* p, int64_t ld) {
  return (reinterpret_cast<uintptr_t>(p) % 16 == 0) && (ld % 4 == 0);
}

struct Plan {
  int bm, bn, splits;
};

int total_k_tiles(const GemmProblem& q) {
  int kt = (int)ceil_div(q.piece[0].K, BK);
  if (q.n_pieces > 1) kt += (int)ceil_div(q.piece[1].K, BK);
  return kt;
}

// Tile shape and split count: fill at least ~2 waves of 256 CUs.
Plan choose_plan(bool a_t, bool b_t, const GemmProblem* probs, int n, bool can_split) {
  (void)a_t;
  (void)b_t;
  int64_t tiles64 = 0, tiles128 = 0;
  int max_kt = 0;
  for (int i = 0; i < n; ++i) {
    tiles64 += ceil_div(probs[i].M, 64) * ceil_div(probs[i].N, 64);
    tiles128 += ceil_div(probs[i].M, 128) * ceil_div(probs[i].N, 128);
    max_kt = max(max_kt, total_k_tiles(probs[i]));
  }
  Plan p{64, 64, 1};
  if (tiles128 >= 1024) { p.bm = 128; p.bn = 128; }
  int64_t tiles = (p.bm == 128) ? tiles128 : tiles64;
  if (can_split && tiles < 512 && max_kt >= 16) {
    int s = (int)ceil_div(512, tiles);
    s = min(s, max(1, max_kt / 8));  // keep >= 8 K tiles per split
    p.splits = max(1, min(s, 64));
  }
  return p;
}

size_t partial_floats(const Plan& pl, const GemmProblem* probs, int n) {
  if (pl.splits <= 1) return 0;
  size_t f = 0;
  for (int i = 0; i < n; ++i) f += (size_t)pl.splits * probs[i].M * probs[i].N;
  return f;
}

template <bool A_T, bool B_T>
cpra_status launch(const Plan& pl, LaunchArgs& args, hipStream_t stream) {
  int max_tiles = 0;
  for (int i = 0; i < args.n_prob; ++i) {
    args.p[i].tiles_m = (int)ceil_div(args.p[i].M, pl.bm);
    args.p[i].tiles_n = (int)ceil_div(args.p[i].N, pl.bn);
    max_tiles = max(max_tiles, args.p[i].tiles_m * args.p[i].tiles_n);
  }
  args.grid_x = (int)ceil_div(max_tiles, 8) * 8;
  dim3 grid(args.grid_x, args.n_prob * args.splits);
  double flops = 0, red_bytes = 0;
  for (int i = 0; i < args.n_prob; ++i) {
    const double mn = (double)args.p[i].M * args.p[i].N;
    flops += 2.0 * mn * ((double)args.p[i].K[0] + (args.p[i].n_pieces > 1 ? args.p[i].K[1] : 0));
    red_bytes += 4.0 * mn * (args.splits + 1);
  }
  static const char* names[2][2][2] = {
      {{"gemm_nn_64x64", "gemm_nt_64x64"}, {"gemm_tn_64x64", "gemm_tt_64x64"}},
      {{"gemm_nn_128x128", "gemm_nt_128x128"}, {"gemm_tn_128x128", "gemm_tt_128x128"}}};
  {
    ProfScope ps(names[pl.bm == 128][A_T][B_T], stream, flops, 0.0);
    if (pl.bm == 128)
      hipLaunchKernelGGL((k_gemm<128, 128, A_T, B_T>), grid, dim3(256), 0, stream, args);
    else
      hipLaunchKernelGGL((k_gemm<64, 64, A_T, B_T>), grid, dim3(256), 0, stream, args);
  }
  CPRA_CHECK_LAUNCH("gemm");
  if (args.splits > 1) {
    int64_t maxel = 0;
    for (int i = 0; i < args.n_prob; ++i) maxel = max(maxel, (int64_t)args.p[i].M * args.p[i].N);
    {
      ProfScope ps("gemm_splitk_reduce", stream, 0.0, red_bytes);
      hipLaunchKernelGGL(k_gemm_splitk_reduce, dim3(ceil_div(maxel, 256), args.n_prob), dim3(256), 0,
                         stream, args);
    }
    CPRA_CHECK_LAUNCH("gemm_splitk_reduce");
  }
  return CPRA_OK;
}

}  // namespace

size_t gemm_batch_workspace_bytes(bool a_t, bool b_t, const GemmProblem* probs, int n) {
  Plan pl = choose_plan(a_t, b_t, probs, n, true);
  return partial_floats(pl, probs, n) * sizeof(float);
}

cpra_status gemm_batch(bool a_t, bool b_t, const GemmProblem* probs, int n, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
  if (n < 1 || n > kMaxProblems) CPRA_FAIL(CPRA_ERR_PARAM, "gemm: 1..4 problems per launch");
  int live = 0;
  for (int i = 0; i < n; ++i)
    if (probs[i].M > 0 && probs[i].N > 0) ++live;
  if (live == 0) return CPRA_OK;
  // Without a workspace the contraction is not split (correct, possibly slower).
  Plan pl = choose_plan(a_t, b_t, probs, n, ws != nullptr && ws_bytes > 0);
  size_t need = partial_floats(pl, probs, n) * sizeof(float);
  if (need > 0 && (ws == nullptr || ws_bytes < need))
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "gemm: workspace %zu < %zu bytes", ws_bytes, need);
  LaunchArgs args{};
  args.n_prob = n;
  args.splits = pl.splits;
  args.partial = static_cast<float*>(ws);
  int64_t off = 0;
  for (int i = 0; i < n; ++i) {
    const GemmProblem& q = probs[i];
    ProbDev& d = args.p[i];
    d.n_pieces = q.n_pieces;
    for (int pc = 0; pc < 2; ++pc) {
      const GemmPiece& g = q.piece[pc < q.n_pieces ? pc : 0];
      d.A[pc] = g.A;
      d.B[pc] = g.B;
      d.lda[pc] = g.lda;
      d.ldb[pc] = g.ldb;
      d.K[pc] = pc < q.n_pieces ? g.K : 0;
      d.vecA[pc] = vec_ok(g.A, g.lda);
      d.vecB[pc] = vec_ok(g.B, g.ldb);
    }
    d.C = q.C;
    d.ldc = q.ldc;
    d.M = q.M;
    d.N = q.N;
    d.bias = q.bias;
    d.mask = q.mask;
    d.ld_mask = q.ld_mask;
    d.beta = q.beta;
    d.relu = q.relu;
    d.part_off = off;
    off += (int64_t)pl.splits * q.M * q.N;
  }
  if (!a_t && b_t) return launch<false, true>(pl, args, stream);
  if (!a_t && !b_t) return launch<false, false>(pl, args, stream);
  if (a_t && !b_t) return launch<true, false>(pl, args, stream);
  return launch<true, true>(pl, args, stream);
}

}  // namespace cpra

extern "C" {

static cpra_status make_problem(int32_t ta, int32_t tb, int32_t M, int32_t N, int32_t K, const float* A,
                                int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                                int64_t ldc, const float* bias, int32_t relu,
                                cpra::GemmProblem* q) {
  if (M < 0 || N < 0 || K < 0) CPRA_FAIL(CPRA_ERR_SHAPE, "gemm: negative size");
  if (M > 0 && N > 0) {
    if (C == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "gemm: C is NULL");
    if (K > 0 && (A == nullptr || B == nullptr)) CPRA_FAIL(CPRA_ERR_NULL, "gemm: A or B is NULL");
    if (ldc < N) CPRA_FAIL(CPRA_ERR_SHAPE, "gemm: ldc < N");
    if (K > 0 && lda < (ta ? M : K)) CPRA_FAIL(CPRA_ERR_SHAPE, "gemm: lda too small");
    if (K > 0 && ldb < (tb ? K : N)) CPRA_FAIL(CPRA_ERR_SHAPE, "gemm: ldb too small");
  }
  *q = cpra::GemmProblem{};
  q->piece[0] = cpra::GemmPiece{A, B, lda, ldb, K};
  q->n_pieces = 1;
  q->C = C;
  q->ldc = ldc;
  q->M = M;
  q->N = N;
  q->bias = bias;
  q->beta = beta;
  q->relu = relu;
  return CPRA_OK;
}

size_t cpra_gemm_workspace_bytes(int32_t ta, int32_t tb, int32_t M, int32_t N, int32_t K) {
  cpra::GemmProblem q{};
  q.piece[0].K = K;
  q.n_pieces = 1;
  q.M = M;
  q.N = N;
  return cpra::gemm_batch_workspace_bytes(ta != 0, tb != 0, &q, 1);
}

cpra_status cpra_gemm(int32_t ta, int32_t tb, int32_t M, int32_t N, int32_t K, const float* A,
                      int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc,
                      const float* bias, int32_t relu, void* ws, size_t ws_bytes,
                      cpra_stream_t stream) {
  cpra::GemmProblem q;
  CPRA_CHECK(make_problem(ta, tb, M, N, K, A, lda, B, ldb, beta, C, ldc, bias, relu, &q));
  return cpra::gemm_batch(ta != 0, tb != 0, &q, 1, ws, ws_bytes, cpra::as_stream(stream));
}

}  // extern "C"
