// FP32 GEMM on the CDNA matrix cores (v_mfma_f32_32x32x2f32) for the GNN's
// dense weight products: forward X W^T, input gradient dY W and weight
// gradient dY^T X.  The kernel template is in gemm_kernel.hpp; this file
// holds the plain instantiations, planning, autotuning and the entry points.
//
// One launch runs up to four independent problems.
// A problem's contraction may be split in two K pieces with separate
// pointers, so [X | MX] [Ws | Wn]^T is a single GEMM without a concatenated
// copy.  Split-K writes FP32 partial tiles that a second kernel sums in a
// fixed order (deterministic), applying the epilogue.
//
// Weight-gradient problems may ask for the row sums of op(A) as well (the bias
// gradient sum_k dY[k, :]): the blocks of the first column tile add up the A
// tiles they stage in LDS (VALU adds beside the MFMAs, fixed order), so no
// extra output column of tiles is computed.
//
// Tile shape and split count come from a table filled by the autotuner
// (timed candidates per problem shape) or, for untuned shapes, a heuristic.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gemm_kernel.hpp"

namespace cpra {

namespace {

using namespace gemmk;

// Sum split-K partials and apply the epilogue.  A block covers 64 consecutive
// outputs with 4 groups of 64 threads; group g adds the g-th quarter of the
// splits in split order (loads issued eight at a time so their latencies
// overlap), and the four group sums are added in group order: a fixed order,
// so the result is deterministic.
constexpr int kRedElems = 64, kRedGroups = 4;
__global__ __launch_bounds__(kRedElems * kRedGroups) void k_gemm_splitk_reduce(LaunchArgs args) {
  __shared__ float red[kRedGroups][kRedElems];
  const int prob = blockIdx.y;
  const ProbDev& P = args.p[prob];
  const int64_t per_g = (int64_t)P.M * P.n_eff;  // one graph's outputs (mode 2), else all
  const int64_t total = per_g * args.G;
  const int e = threadIdx.x % kRedElems, grp = threadIdx.x / kRedElems;
  const int64_t idx = (int64_t)blockIdx.x * kRedElems + e;
  if ((int64_t)blockIdx.x * kRedElems >= total) return;  // uniform per block
  const float* part = args.partial + P.part_off;
  const int per = (args.splits + kRedGroups - 1) / kRedGroups;
  const int s0 = min(args.splits, grp * per), s1 = min(args.splits, s0 + per);
  float v = 0.f;
  if (idx < total) {
    int s = s0;
    for (; s + 8 <= s1; s += 8) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = part[(int64_t)(s + u) * total + idx];
#pragma unroll
      for (int u = 0; u < 8; ++u) v += x[u];
    }
    for (; s < s1; ++s) v += part[(int64_t)s * total + idx];
  }
  red[grp][e] = v;
  __syncthreads();
  if (grp != 0 || idx >= total) return;
  v = red[0][e];
#pragma unroll
  for (int g2 = 1; g2 < kRedGroups; ++g2) v += red[g2][e];
  const int g = (int)(idx / per_g);
  const int64_t rem = idx - (int64_t)g * per_g;
  const int row = (int)(rem / P.n_eff);
  const int col = (int)(rem - (int64_t)row * P.n_eff);
  if (col == P.N) {
    P.bias_grad[(int64_t)g * P.bg_stride + row] = v;
    return;
  }
  if (P.bias) v += P.bias[col];
  epilogue_store(P, P.C + (int64_t)g * P.c_stride, row, col, v);
}

inline bool vec_ok(const float* p, int64_t ld) {
  return (reinterpret_cast<uintptr_t>(p) % 16 == 0) && (ld % 4 == 0);
}

const char* kCfgNames[kNumCfgs] = {"64x64x32_w2x2",   "64x64x32_w2x1", "64x64x32_w1x1",
                                   "128x64x32_w2x2",  "64x128x32_w2x2", "128x128x32_w2x2",
                                   "64x64x16_w2x2",   "128x128x16_w2x2", "32x64x32_w1x1",
                                   "64x32x32_w1x1",   "64x64x16_w2x2_p2", "64x64x32_w2x2_p2",
                                   "128x64x16_w2x2_p2", "64x128x16_w2x2_p2",
                                   "128x128x16_w2x2_p2", "64x32x16_w1x1_p2",
                                   "32x64x16_w1x1_p2", "64x64x16_w1x1_p2",
                                   "64x64x16_w2x1_p2", "128x64x16_w2x1_p2",
                                   "64x64x16_w2x2_il", "128x128x16_w2x2_il",
                                   "128x64x16_w2x2_il", "256x128x16_w2x2_il",
                                   "64x128x16_w2x2_il", "64x64x32_w2x2_il",
                                   "64x128x32_w2x2_il", "64x64x16_w2x2_ring",
                                   "64x128x16_w2x2_ring", "128x64x16_w2x2_ring",
                                   "64x64x32_w2x2_ring", "128x128x16_w2x2_ring"};

struct Plan {
  int cfg, splits;
};

inline int n_eff_of(const GemmProblem& q) { return q.N + (q.bias_grad ? 1 : 0); }
// columns covered by output tiles: N (at least one tile when only the bias gradient is wanted)
inline int tile_cols_of(const GemmProblem& q) { return q.N > 0 ? q.N : (q.bias_grad ? 1 : 0); }

int total_k_tiles(const GemmProblem& q, int bk) {
  int kt = (int)ceil_div(q.piece[0].K, bk);
  if (q.n_pieces > 1) kt += (int)ceil_div(q.piece[1].K, bk);
  return kt;
}

// graphs of a grouped problem (1 when not grouped)
inline int groups_of(const GemmProblem& q) { return q.group_mode ? max(1, q.n_groups) : 1; }

int64_t tiles_of(const GemmProblem* probs, int n, const Cfg& c) {
  int64_t t = 0;
  for (int i = 0; i < n; ++i) {
    const GemmProblem& q = probs[i];
    const int64_t cols = ceil_div(tile_cols_of(q), c.bn);
    if (q.group_mode == 1) t += (ceil_div(q.M, c.bm) + groups_of(q)) * cols;  // row tiles (bound)
    else t += groups_of(q) * ceil_div(q.M, c.bm) * cols;
  }
  return t;
}

// K steps of the longest problem (mode 2: of a graph of average size)
int max_k_tiles(const GemmProblem* probs, int n, int bk) {
  int m = 0;
  for (int i = 0; i < n; ++i)
    m = max(m, (int)ceil_div(total_k_tiles(probs[i], bk), probs[i].group_mode == 2 ? groups_of(probs[i]) : 1));
  return m;
}

// Split count that brings the launch to ~512 blocks, keeping >= 4 K steps per split.
constexpr int kMaxSplits = 1024;

int heuristic_splits(const GemmProblem* probs, int n, const Cfg& c) {
  if (probs[0].group_mode == 1) return 1;  // row-grouped products are never split
  const int64_t tiles = tiles_of(probs, n, c);
  const int mkt = max_k_tiles(probs, n, c.bk);
  if (tiles >= 512 || mkt < 8) return 1;
  int s = (int)ceil_div(512, tiles);
  s = min(s, max(1, mkt / 4));
  return max(1, min(s, kMaxSplits));
}

Plan heuristic_plan(const GemmProblem* probs, int n, bool can_split) {
  Plan p{0, 1};
  if (tiles_of(probs, n, kCfgs[5]) >= 1024) p.cfg = 5;
  if (can_split) p.splits = heuristic_splits(probs, n, kCfgs[p.cfg]);
  return p;
}

size_t partial_floats(int splits, const GemmProblem* probs, int n);

// Split counts the tuner tries for a configuration: 1, the powers of two up to
// half the K steps, and the heuristic's count and its double, within a launch
// of at most 32768 blocks and 256 MiB of partial tiles.
constexpr int64_t kMaxTuneBlocks = 32768;
constexpr size_t kMaxPartialBytes = size_t(256) << 20;

std::vector<int> split_candidates(const GemmProblem* probs, int n, const Cfg& c) {
  std::vector<int> out = {1};
  if (probs[0].group_mode == 1) return out;
  const int64_t tiles = tiles_of(probs, n, c);
  const int cap = min(kMaxSplits, max(1, max_k_tiles(probs, n, c.bk) / 2));
  const int h = heuristic_splits(probs, n, c);
  std::vector<int> cand;
  for (int s = 2; s <= cap; s *= 2) cand.push_back(s);
  if (h > 1) {
    cand.push_back(h);
    if (2 * h <= kMaxSplits) cand.push_back(2 * h);
  }
  std::sort(cand.begin(), cand.end());
  for (int s : cand) {
    if (s == out.back()) continue;
    if (s != h && (tiles * s > kMaxTuneBlocks ||
                   partial_floats(s, probs, n) * sizeof(float) > kMaxPartialBytes))
      continue;
    out.push_back(s);
  }
  return out;
}

size_t partial_floats(int splits, const GemmProblem* probs, int n) {
  if (splits <= 1) return 0;
  size_t f = 0;
  for (int i = 0; i < n; ++i) f += (size_t)splits * groups_of(probs[i]) * probs[i].M * n_eff_of(probs[i]);
  return f;
}

// ---- tuning table -----------------------------------------------------------
struct TuneEntry {
  Plan plan;
  double us;
  double heuristic_us;
};

std::mutex g_tune_mu;
bool g_tuning = false;
std::map<std::string, TuneEntry> g_table;
std::vector<std::string> g_order;

std::string shape_key(bool a_t, bool b_t, const GemmProblem* probs, int n) {
  std::string k = a_t ? "T" : "N";
  k += b_t ? "T" : "N";
  char buf[96];
  if (probs[0].group_mode) {  // per-graph weights: mode and graph count
    snprintf(buf, sizeof(buf), "|g%d:%d", probs[0].group_mode, groups_of(probs[0]));
    k += buf;
  }
  for (int i = 0; i < n; ++i) {
    const GemmProblem& q = probs[i];
    snprintf(buf, sizeof(buf), "|%dx%dx%d", q.M, n_eff_of(q),
             q.piece[0].K + (q.n_pieces > 1 ? q.piece[1].K : 0));
    k += buf;
  }
  return k;
}

bool lookup(const std::string& key, Plan* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  *out = it->second.plan;
  return true;
}

void fill_args(const GemmProblem* probs, int n, int splits, void* ws, LaunchArgs* args) {
  *args = LaunchArgs{};
  const GemmProblem& q0 = probs[0];
  args->n_prob = n;
  args->splits = splits;
  args->partial = static_cast<float*>(ws);
  args->G = q0.group_mode == 2 ? groups_of(q0) : 1;
  args->n_vprob = n * args->G;
  args->gptr = q0.group_ptr;
  if (q0.group_mode == 1) {
    for (int b = 0; b < 3; ++b) {
      args->row_maps[b] = q0.rows->map[b];
      args->row_counts[b] = q0.rows->count[b];
    }
  }
  int64_t off = 0;
  for (int i = 0; i < n; ++i) {
    const GemmProblem& q = probs[i];
    ProbDev& d = args->p[i];
    d.n_pieces = q.n_pieces;
    for (int pc = 0; pc < 2; ++pc) {
      const GemmPiece& g = q.piece[pc < q.n_pieces ? pc : 0];
      d.A[pc] = g.A;
      d.B[pc] = g.B;
      d.lda[pc] = g.lda;
      d.ldb[pc] = g.ldb;
      d.K[pc] = pc < q.n_pieces ? g.K : 0;
      d.vecA[pc] = vec_ok(g.A, g.lda);
      d.vecB[pc] = vec_ok(g.B, g.ldb) && q.b_stride % 4 == 0;
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
    d.bias_grad = q.bias_grad;
    d.sig_out = q.sig_out;
    d.add = q.add;
    d.ld_add = q.ld_add;
    d.ld_sig = q.ld_sig;
    d.b_stride = q.b_stride;
    d.c_stride = q.c_stride;
    d.bias_stride = q.bias_stride;
    d.bg_stride = q.bg_stride;
    d.n_eff = n_eff_of(q);
    d.part_off = off;
    off += (int64_t)splits * args->G * q.M * d.n_eff;
  }
}

cpra_status run_plan(bool a_t, bool b_t, const GemmProblem* probs, int n, const Plan& pl, void* ws,
                     hipStream_t stream) {
  LaunchArgs args;
  fill_args(probs, n, pl.splits, ws, &args);
  // the configuration that runs (and names the profiler family)
  const int cfg = resolve_cfg(args, a_t, b_t, pl.cfg);
  double flops = 0, red_bytes = 0;
  for (int i = 0; i < n; ++i) {
    const double mn = (double)args.p[i].M * args.p[i].N;
    flops += 2.0 * mn * ((double)args.p[i].K[0] + (args.p[i].n_pieces > 1 ? args.p[i].K[1] : 0));
    red_bytes += 4.0 * (double)args.G * args.p[i].M * args.p[i].n_eff * (pl.splits + 1);
  }
  // profiler family = one kernel instantiation: layout + group mode + tile configuration
  static const char* layout[2][2] = {{"nn", "nt"}, {"tn", "tt"}};
  static const char* gmode[3] = {"", "_byrow", "_byk"};
  const int mode = probs[0].group_mode;
  char pname[64];
  snprintf(pname, sizeof(pname), "gemm_%s%s_%s", layout[a_t][b_t], gmode[mode], kCfgNames[cfg]);
  {
    ProfScope ps(pname, stream, flops, 0.0);
    if (mode) launch_grouped(mode, a_t, b_t, cfg, args, stream);
    else if (!a_t && b_t) launch_any<false, true, 0>(cfg, args, stream);
    else if (!a_t && !b_t) launch_any<false, false, 0>(cfg, args, stream);
    else if (a_t && !b_t) launch_any<true, false, 0>(cfg, args, stream);
    else launch_any<true, true, 0>(cfg, args, stream);
  }
  CPRA_CHECK_LAUNCH("gemm");
  if (pl.splits > 1) {
    int64_t maxel = 0;
    for (int i = 0; i < n; ++i) maxel = max(maxel, (int64_t)args.G * args.p[i].M * args.p[i].n_eff);
    {
      ProfScope ps("gemm_splitk_reduce", stream, 0.0, red_bytes);
      hipLaunchKernelGGL(k_gemm_splitk_reduce, dim3(ceil_div(maxel, kRedElems), n),
                         dim3(kRedElems * kRedGroups), 0, stream, args);
    }
    CPRA_CHECK_LAUNCH("gemm_splitk_reduce");
  }
  return CPRA_OK;
}

// Time every candidate (tile config x split count that fits the workspace) and
// keep the fastest.  Runs on `stream`, synchronising it; the candidates all
// compute the same C (overwritten each time), so re-running the chosen plan
// leaves its result.
cpra_status tune(bool a_t, bool b_t, const GemmProblem* probs, int n, void* ws, size_t ws_bytes,
                 hipStream_t stream, const std::string& key, Plan* best_out) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    CPRA_FAIL(CPRA_ERR_HIP, "gemm tune: event creation failed");
  const Plan heur = heuristic_plan(probs, n, ws != nullptr);
  const char* env = getenv("CPRA_AUTOTUNE_LOG");  // print every candidate's time
  const bool log_candidates = env != nullptr && env[0] == '1';
  TuneEntry entry{Plan{0, 1}, 1e30, -1.0};
  for (int c = 0; c < kNumCfgs; ++c) {
    std::vector<int> splits;
    for (int s : split_candidates(probs, n, kCfgs[c]))
      if (s == 1 || (ws != nullptr && partial_floats(s, probs, n) * sizeof(float) <= ws_bytes))
        splits.push_back(s);
    for (int s : splits) {
      Plan pl{c, s};
      CPRA_CHECK(run_plan(a_t, b_t, probs, n, pl, ws, stream));  // warm-up
      hipEventRecord(e0, stream);
      const int reps = 3;
      for (int r = 0; r < reps; ++r) CPRA_CHECK(run_plan(a_t, b_t, probs, n, pl, ws, stream));
      hipEventRecord(e1, stream);
      if (hipEventSynchronize(e1) != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "gemm tune: sync failed");
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      const double us = 1e3 * ms / reps;
      if (log_candidates)
        fprintf(stderr, "[cpra autotune] %s %s/split%d %.2f us\n", key.c_str(), kCfgNames[c], s, us);
      if (c == heur.cfg && s == heur.splits) entry.heuristic_us = us;
      if (us < entry.us) {
        entry.us = us;
        entry.plan = pl;
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_table.find(key) == g_table.end()) g_order.push_back(key);
    g_table[key] = entry;
  }
  *best_out = entry.plan;
  return run_plan(a_t, b_t, probs, n, entry.plan, ws, stream);
}

}  // namespace

size_t gemm_batch_workspace_bytes(bool a_t, bool b_t, const GemmProblem* probs, int n) {
  (void)a_t;
  (void)b_t;
  // Room for any candidate the tuner may pick.
  size_t best = 0;
  for (int c = 0; c < kNumCfgs; ++c)
    for (int s : split_candidates(probs, n, kCfgs[c]))
      if (s > 1) best = std::max(best, partial_floats(s, probs, n) * sizeof(float));
  return best;
}

cpra_status gemm_batch(bool a_t, bool b_t, const GemmProblem* probs_in, int n, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
  if (n < 1 || n > kMaxProblems) CPRA_FAIL(CPRA_ERR_PARAM, "gemm: 1..4 problems per launch");
  GemmProblem local[kMaxProblems];
  const GemmProblem* probs = probs_in;
  if (probs_in[0].group_mode) {
    const GemmProblem& q0 = probs_in[0];
    for (int i = 0; i < n; ++i) {
      const GemmProblem& q = probs_in[i];
      if (q.group_mode != q0.group_mode || q.n_groups != q0.n_groups || q.group_ptr != q0.group_ptr ||
          q.rows != q0.rows)
        CPRA_FAIL(CPRA_ERR_PARAM, "gemm: the problems of a launch must share their grouping");
      if (q.group_mode == 1 && (a_t || q.bias_grad || (q.n_groups > 1 && q.rows == nullptr)))
        CPRA_FAIL(CPRA_ERR_PARAM, "gemm: row-grouped products take A [rows, K], no bias gradient, a row map");
      if (q.group_mode == 2 && (!a_t || b_t || q.bias || q.mask || q.add || q.sig_out || q.beta != 0.f ||
                                q.relu || (q.n_groups > 1 && q.group_ptr == nullptr)))
        CPRA_FAIL(CPRA_ERR_PARAM, "gemm: K-grouped products are plain A^T B with a graph row map");
      if (q.group_mode != 1 && q.group_mode != 2)
        CPRA_FAIL(CPRA_ERR_PARAM, "gemm: group mode %d", q.group_mode);
    }
    if (q0.n_groups <= 1) {  // one graph: the plain product
      for (int i = 0; i < n; ++i) {
        local[i] = probs_in[i];
        local[i].group_mode = 0;
      }
      probs = local;
    }
  }
  for (int i = 0; i < n; ++i)
    if (probs[i].bias_grad && probs[i].bias)
      CPRA_FAIL(CPRA_ERR_PARAM, "gemm: bias_grad and bias are exclusive");
  int live = 0;
  for (int i = 0; i < n; ++i)
    if (probs[i].M > 0 && n_eff_of(probs[i]) > 0) ++live;
  if (live == 0) return CPRA_OK;
  const bool can_split = ws != nullptr && ws_bytes > 0;
  const std::string key = shape_key(a_t, b_t, probs, n);
  Plan pl;
  if (!lookup(key, &pl)) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing =
        hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
    bool overwrite_only = true;  // tuning re-runs the GEMM: only if C is overwritten
    for (int i = 0; i < n; ++i) overwrite_only = overwrite_only && probs[i].beta == 0.f;
    if (g_tuning && !capturing && overwrite_only)
      return tune(a_t, b_t, probs, n, can_split ? ws : nullptr, can_split ? ws_bytes : 0, stream,
                  key, &pl);
    pl = heuristic_plan(probs, n, can_split);
  }
  // A tuned plan may split more than this workspace allows: fall back to fewer splits.
  // Row-grouped products are never split (their reduction has no per-graph bias).
  if (!can_split || probs[0].group_mode == 1) pl.splits = 1;
  while (pl.splits > 1 && partial_floats(pl.splits, probs, n) * sizeof(float) > ws_bytes)
    pl.splits /= 2;
  return run_plan(a_t, b_t, probs, n, pl, ws, stream);
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

cpra_status cpra_autotune_begin(void) {
  std::lock_guard<std::mutex> lk(cpra::g_tune_mu);
  cpra::g_tuning = true;
  return CPRA_OK;
}

cpra_status cpra_autotune_end(int32_t* n_entries) {
  std::lock_guard<std::mutex> lk(cpra::g_tune_mu);
  cpra::g_tuning = false;
  if (n_entries) *n_entries = (int32_t)cpra::g_order.size();
  return CPRA_OK;
}

cpra_status cpra_autotune_reset(void) {
  std::lock_guard<std::mutex> lk(cpra::g_tune_mu);
  cpra::g_table.clear();
  cpra::g_order.clear();
  return CPRA_OK;
}

cpra_status cpra_autotune_get(int32_t i, char* key, size_t key_len, int32_t* cfg, int32_t* splits,
                              char* choice, size_t choice_len, double* us, double* heuristic_us) {
  using namespace cpra;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (i < 0 || i >= (int32_t)g_order.size())
    CPRA_FAIL(CPRA_ERR_PARAM, "autotune_get: index out of range");
  const TuneEntry& e = g_table[g_order[i]];
  if (key && key_len) snprintf(key, key_len, "%s", g_order[i].c_str());
  if (cfg) *cfg = e.plan.cfg;
  if (splits) *splits = e.plan.splits;
  if (choice && choice_len)
    snprintf(choice, choice_len, "%s/split%d", kCfgNames[e.plan.cfg], e.plan.splits);
  if (us) *us = e.us;
  if (heuristic_us) *heuristic_us = e.heuristic_us;
  return CPRA_OK;
}

cpra_status cpra_autotune_set(const char* key, int32_t cfg, int32_t splits) {
  using namespace cpra;
  if (key == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "autotune_set: key is NULL");
  if (cfg < 0 || cfg >= kNumCfgs || splits < 1 || splits > kMaxSplits)
    CPRA_FAIL(CPRA_ERR_PARAM, "autotune_set: config %d / splits %d out of range", cfg, splits);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_table.find(key) == g_table.end()) g_order.push_back(key);
  g_table[key] = TuneEntry{Plan{cfg, splits}, -1.0, -1.0};
  return CPRA_OK;
}

}  // extern "C"
