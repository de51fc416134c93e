// The GNN P_theta(G) of the GNN and architecture appendices, its hand-written
// backward, and the full CPRA training step (Sec. 3.1 loop).
//
// Layer k maps H [N, in] to act(M H Wn^T + H Ws^T (+ b)) [N, out].  Two
// evaluation orders, equal in exact arithmetic:
//  * aggregate-first (out >= in): AX = M H, then one GEMM over the K pieces
//    (H, Ws) and (AX, Wn) with bias/ReLU in the epilogue;
//  * linear-first (out < in, e.g. the S-wide output layer): [Ys | Yn] =
//    H [Ws; Wn]^T by two GEMMs in one launch, then Y = Ys + M Yn + b with
//    the ReLU in the aggregation epilogue -- the gather is out wide, not in.
// Backward (dY = upstream gradient, masked by the ReLU of the layer's output),
// in an order of its own (either one is valid whichever order the forward took):
//  * gradient-first (out > in): dWs = dY^T H, dWn = dY^T AX, G = dY [Ws | Wn],
//    dH = G_s + M^T G_n (masked by H > 0 in the same pass) -- the gather is in
//    wide;
//  * transpose-first (out <= in): T = M^T dY, dWs = dY^T H, dWn = T^T H,
//    dH = [dY | T] [Ws; Wn] (masked in the GEMM epilogue) -- the gather is out
//    wide, dH is written once instead of G [N, 2 in], and AX is not needed.
// A square layer (out = in) gathers as many columns either way, so it takes
// the transpose-first order.
// db = column sums of dY, added up by the dWs GEMM from the dY tiles it stages
// in LDS (no separate pass).  The output layer also writes P = sigmoid(Z) in
// its epilogue, for the loss.  M^T = A D^-1 is applied by the transposed
// aggregation (not M: the graph need not be regular).  With recompute set,
// AX is not kept from the forward and is rebuilt in the backward of the
// gradient-first layers.
//
// Per-graph weights (weight_groups = G > 1): every weight product becomes a
// grouped GEMM over the batch's graphs -- the forward and input-gradient
// products by rows (graph g's rows times graph g's weights), the weight
// gradients by K (graph g's weight gradient sums over graph g's rows only).
// The aggregations are unchanged (the batch is block-diagonal), and in the
// linear-first order the bias moves into the self-weight GEMM's epilogue
// (it is graph g's bias for graph g's rows).
#include <algorithm>
#include <cstdlib>
#include <functional>

#include "common.hpp"

namespace cpra {

cpra_status check_loss_cfg_public(const cpra_csr* g, const cpra_loss_cfg* cfg);
cpra_status check_adam_cfg(const cpra_adam_cfg* cfg);

namespace {

constexpr int kMaxLayers = 16;

struct Layer {
  int in, out;
  bool lf;  // linear-first forward (out < in)
  bool tf;  // transpose-first backward (out <= in)
  int64_t off_ws, off_wn, off_b;
};

struct Plan {
  int G;                  // weight sets (1: shared by all graphs)
  const float* z_offset;  // [N, S] added to the output layer, or null
  int train_from;         // first trained layer (0: all, embedding included)
  bool reuse_prefix;      // forward starts at train_from from saved activations
  int L;
  bool sage, recompute;
  int N;
  Layer layer[kMaxLayers];
  int64_t n_params;
  size_t h_off[kMaxLayers];   // saved input of layer k (k >= 1)
  size_t ax_off[kMaxLayers];  // saved M H of aggregate-first layers
  size_t ax_scratch_off;      // recompute buffer
  size_t yy_off, d_off[2], g_off, t_off[2], p_off, gemm_off, rows_off;
  size_t q_off;  // work queues of persistent aggregations: [main stream | side stream]
  size_t gemm_bytes;
  size_t total;
};

cpra_status check_model_cfg(const cpra_model_cfg* cfg) {
  if (cfg == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "model: cfg is NULL");
  if (cfg->layer_kind != CPRA_GCN && cfg->layer_kind != CPRA_SAGE)
    CPRA_FAIL(CPRA_ERR_PARAM, "model: unknown layer kind %d", cfg->layer_kind);
  if (cfg->n_layers < 1 || cfg->n_layers > kMaxLayers)
    CPRA_FAIL(CPRA_ERR_PARAM, "model: n_layers = %d outside 1..%d", cfg->n_layers, kMaxLayers);
  if (cfg->train_from_layer < 0 || cfg->train_from_layer >= cfg->n_layers)
    CPRA_FAIL(CPRA_ERR_PARAM, "model: train_from_layer = %d outside 0..%d", cfg->train_from_layer,
              cfg->n_layers - 1);
  if (cfg->reuse_frozen_prefix && cfg->train_from_layer < 1)
    CPRA_FAIL(CPRA_ERR_PARAM, "model: reuse_frozen_prefix needs train_from_layer >= 1");
  if (cfg->in_dim < 1 || cfg->hidden < 1 || cfg->S < 1 || cfg->S > 1024)
    CPRA_FAIL(CPRA_ERR_PARAM, "model: widths must be >= 1 and S <= 1024");
  if (cfg->in_dim > 4096 || cfg->hidden > 4096)
    CPRA_FAIL(CPRA_ERR_PARAM, "model: in_dim and hidden up to 4096 supported");
  if (cfg->weight_groups < 0) CPRA_FAIL(CPRA_ERR_PARAM, "model: weight_groups < 0");
  return CPRA_OK;
}

void make_layers(const cpra_model_cfg* cfg, int N, Plan* p) {
  p->G = std::max(cfg->weight_groups, 1);
  p->L = cfg->n_layers;
  p->sage = cfg->layer_kind == CPRA_SAGE;
  p->recompute = cfg->recompute != 0;
  p->N = N;
  int64_t off = (int64_t)N * cfg->in_dim;
  int d_in = cfg->in_dim;
  for (int k = 0; k < p->L; ++k) {
    Layer& l = p->layer[k];
    l.in = d_in;
    l.out = (k == p->L - 1) ? cfg->S : cfg->hidden;
    l.lf = l.out < l.in;
    l.tf = l.out <= l.in;
    l.off_ws = off;
    off += (int64_t)p->G * l.out * l.in;
    l.off_wn = off;
    off += (int64_t)p->G * l.out * l.in;
    if (p->sage) {
      l.off_b = off;
      off += (int64_t)p->G * l.out;
    } else {
      l.off_b = -1;
    }
    d_in = l.out;
  }
  p->n_params = off;
}

// Per-graph grouping of a GEMM (no-op with shared weights).
void set_groups(const Plan& p, const cpra_csr* g, const GroupRows* rows, int mode, GemmProblem* q,
                const Layer& l) {
  if (p.G <= 1) return;
  q->group_mode = mode;
  q->n_groups = p.G;
  q->group_ptr = g ? g->graph_ptr : nullptr;
  q->rows = rows;
  q->b_stride = (int64_t)l.out * l.in;  // one Ws / Wn copy
  q->c_stride = (int64_t)l.out * l.in;
  q->bias_stride = l.out;
  q->bg_stride = l.out;
}

// Weight-gradient GEMM shapes of layer k (for the workspace query).
void wgrad_problems(const Plan& p, int k, GemmProblem* q) {
  const Layer& l = p.layer[k];
  for (int i = 0; i < 2; ++i) {
    q[i] = GemmProblem{};
    q[i].n_pieces = 1;
    q[i].piece[0].K = p.N;
    q[i].M = l.out;
    q[i].N = l.in;
    set_groups(p, nullptr, nullptr, 2, &q[i], l);
  }
  if (p.sage) q[0].bias_grad = reinterpret_cast<float*>(1);  // shape only: one extra column
}

void make_plan(const cpra_model_cfg* cfg, const cpra_csr* g, Plan* p) {
  const int N = g->n_nodes;
  make_layers(cfg, N, p);
  p->z_offset = cfg->z_offset;
  p->train_from = cfg->train_from_layer;
  p->reuse_prefix = cfg->reuse_frozen_prefix != 0;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes, 256);
    return o;
  };
  const size_t f = sizeof(float);
  int max_in_after0 = 0, max_in_af = 0, max_out_lf = 0, max_in_gf = 0, max_out_tf = 0;
  for (int k = 0; k < p->L; ++k) {
    const Layer& l = p->layer[k];
    p->h_off[k] = (k >= 1) ? take((size_t)N * l.in * f) : 0;
    if (k >= 1) max_in_after0 = std::max(max_in_after0, l.in);
    if (l.tf) {
      max_out_tf = std::max(max_out_tf, l.out);
    } else {
      max_in_gf = std::max(max_in_gf, l.in);
    }
    if (!l.lf) {
      max_in_af = std::max(max_in_af, l.in);
      p->ax_off[k] = p->recompute ? 0 : take((size_t)N * l.in * f);
    } else {
      max_out_lf = std::max(max_out_lf, l.out);
      p->ax_off[k] = 0;
    }
  }
  p->ax_scratch_off = (p->recompute && max_in_af > 0) ? take((size_t)N * max_in_af * f) : 0;
  p->yy_off = max_out_lf ? take((size_t)N * 2 * max_out_lf * f) : 0;
  p->d_off[0] = max_in_after0 ? take((size_t)N * max_in_after0 * f) : 0;
  p->d_off[1] = max_in_after0 ? take((size_t)N * max_in_after0 * f) : 0;
  p->g_off = max_in_gf ? take((size_t)N * 2 * max_in_gf * f) : 0;
  // two T buffers, alternating between transpose-first layers, so that a layer's
  // T does not wait for the side stream to finish reading the previous one
  p->t_off[0] = max_out_tf ? take((size_t)N * max_out_tf * f) : 0;
  p->t_off[1] = max_out_tf ? take((size_t)N * max_out_tf * f) : 0;
  p->p_off = take((size_t)N * cfg->S * f);
  size_t gb = 0;
  for (int k = 0; k < p->L; ++k) {
    GemmProblem q[2];
    wgrad_problems(*p, k, q);
    gb = std::max(gb, gemm_batch_workspace_bytes(true, false, q, 2));
  }
  p->gemm_bytes = gb;
  p->gemm_off = gb ? take(gb) : 0;
  p->rows_off = p->G > 1 ? take(group_rows_bytes(g)) : 0;
  p->q_off = take(2 * kQueueInts * sizeof(int32_t));
  p->total = std::max<size_t>(off, 256);
}

inline float* fptr(void* ws, size_t off) {
  return reinterpret_cast<float*>(static_cast<char*>(ws) + off);
}

bool wgrad_late() {
  const char* e = getenv("CPRA_WGRAD_LATE");
  return e != nullptr && e[0] == '1';
}

bool side_first_order() {
  const char* e = getenv("CPRA_SIDE_FIRST");
  return e != nullptr && e[0] == '1';
}

// The work queue of the aggregations on the main (0) or side (1) stream.
inline int32_t* queue_of(void* ws, const Plan& p, int which) {
  return reinterpret_cast<int32_t*>(static_cast<char*>(ws) + p.q_off) + which * kQueueInts;
}


cpra_status forward_impl(const cpra_csr* g, const Plan& p, const float* params, float* Z,
                         int64_t ldz, void* ws, hipStream_t st) {
  const int N = g->n_nodes;
  GroupRows rows{};
  if (p.G > 1) CPRA_CHECK(group_rows_build(g, static_cast<char*>(ws) + p.rows_off, &rows, st));
  // With a reused frozen prefix the forward starts at the first trained layer,
  // from the input the previous forward saved.
  const int k0 = p.reuse_prefix ? p.train_from : 0;
  const float* H = k0 == 0 ? params : fptr(ws, p.h_off[k0]);  // embedding or saved input
  int64_t ldh = p.layer[k0].in;
  for (int k = k0; k < p.L; ++k) {
    const Layer& l = p.layer[k];
    const bool last = k == p.L - 1;
    float* dst = last ? Z : fptr(ws, p.h_off[k + 1]);
    const int64_t ldd = last ? ldz : l.out;
    const float* Ws = params + l.off_ws;
    const float* Wn = params + l.off_wn;
    const float* b = p.sage ? params + l.off_b : nullptr;
    float* P = last ? fptr(ws, p.p_off) : nullptr;  // sigmoid(Z) for the loss
    if (!l.lf) {
      float* AX = fptr(ws, p.recompute ? p.ax_scratch_off : p.ax_off[k]);
      const bool saved_ax = p.reuse_prefix && k == k0 && !p.recompute;  // M H of a frozen input
      if (!saved_ax)
        CPRA_CHECK(aggregate(g, false, l.in, H, ldh, AX, l.in, nullptr, 0, nullptr, false, nullptr, 0, st,
                             nullptr, 0, nullptr, 0, queue_of(ws, p, 0)));
      GemmProblem q{};
      q.piece[0] = GemmPiece{H, Ws, ldh, l.in, l.in};
      q.piece[1] = GemmPiece{AX, Wn, l.in, l.in, l.in};
      q.n_pieces = 2;
      q.C = dst;
      q.ldc = ldd;
      q.M = N;
      q.N = l.out;
      q.bias = b;
      q.relu = last ? 0 : 1;
      q.sig_out = P;
      q.ld_sig = l.out;
      if (last && p.z_offset) {
        q.add = p.z_offset;
        q.ld_add = l.out;
      }
      set_groups(p, g, &rows, 1, &q, l);
      CPRA_CHECK(gemm_batch(false, true, &q, 1, nullptr, 0, st));
    } else {
      float* YY = fptr(ws, p.yy_off);
      const int64_t ldyy = 2 * l.out;
      GemmProblem q[2] = {};
      for (int i = 0; i < 2; ++i) {
        q[i].piece[0] = GemmPiece{H, i == 0 ? Ws : Wn, ldh, l.in, l.in};
        q[i].n_pieces = 1;
        q[i].C = YY + (i == 0 ? 0 : l.out);
        q[i].ldc = ldyy;
        q[i].M = N;
        q[i].N = l.out;
        set_groups(p, g, &rows, 1, &q[i], l);
      }
      // per-graph biases are added by the self-weight GEMM (graph g's bias on graph g's rows)
      if (p.G > 1) q[0].bias = b;
      CPRA_CHECK(gemm_batch(false, true, q, 2, nullptr, 0, st));
      CPRA_CHECK(aggregate(g, false, l.out, YY + l.out, ldyy, dst, ldd, YY, ldyy, p.G > 1 ? nullptr : b,
                           !last, nullptr, 0, st, P, l.out, last ? p.z_offset : nullptr, l.out,
                           queue_of(ws, p, 0)));
    }
    H = dst;
    ldh = ldd;
  }
  return CPRA_OK;
}

// The weight-gradient GEMMs of a layer only feed the optimiser, so they run on
// the side stream (when `side` is given) while the main stream computes the
// input gradients.  The main stream waits for the side stream only before it
// overwrites a buffer that forked side work still reads (and the caller joins
// at the end).
struct PendingReads {
  const void* buf[4];
  int n = 0;
  bool full = false;  // more than fit: every write waits (safe, never seen at these depths)
  void add(const void* p) {
    if (n < 4) {
      buf[n++] = p;
    } else {
      full = true;
    }
  }
  bool has(const void* p) const {
    if (full) return true;
    for (int i = 0; i < n; ++i)
      if (buf[i] == p) return true;
    return false;
  }
  void clear() {
    n = 0;
    full = false;
  }
};

// rows_ready: the row-tile maps of per-graph weights are in ws already (built
// by the forward of the same step).  side_task (optional, with a side stream):
// work enqueued on the side stream right after the first fork -- the
// training step's loss-term reduction, so that it needs no fork of its own.
cpra_status backward_impl(const cpra_csr* g, const Plan& p, const float* params, const float* dZ,
                          int64_t lddz, float* grads, void* ws, hipStream_t st,
                          SideStream* side, bool rows_ready,
                          const std::function<cpra_status(hipStream_t)>* side_task = nullptr) {
  const int N = g->n_nodes;
  GroupRows rows{};
  if (p.G > 1) {
    void* rws = static_cast<char*>(ws) + p.rows_off;
    if (rows_ready) {
      CPRA_CHECK(group_rows_view(g, rws, &rows));
    } else {
      CPRA_CHECK(group_rows_build(g, rws, &rows, st));
    }
  }
  const hipStream_t wst = side ? side->stream : st;  // stream of the weight gradients
  PendingReads pending;
  auto forked = [&]() -> cpra_status {  // after each fork: the pending side task, once
    if (side_task && *side_task) {
      CPRA_CHECK((*side_task)(side->stream));
      side_task = nullptr;
    }
    return CPRA_OK;
  };
  auto before_write = [&](const void* buf) -> cpra_status {
    if (side && pending.has(buf)) {
      CPRA_CHECK(join_from(side, st));
      pending.clear();
    }
    return CPRA_OK;
  };
  // Order of a layer's two halves after its fork.  By default the fork is
  // marked, the input gradient (the main chain) enqueued, and only then the
  // side work: in a captured graph the input gradient is then the first
  // successor of the gather before it and keeps the main chain's hardware queue
  // (a hop to another queue costs a dependency wait of several microseconds).
  // CPRA_SIDE_FIRST=1 captures the side work first, which dispatches the weight
  // gradients ahead of the input gradient they run beside.  (Mixing the two
  // orders within one step let the graph launcher put independent kernels of
  // both halves on one queue, in series.)
  const bool side_first = side_first_order();
  auto main_first = [&](int) { return side != nullptr && !side_first; };
  const float* dY = dZ;
  int64_t lddy = lddz;
  int ping = 0, tping = 0;
  void* gemm_ws = p.gemm_bytes ? static_cast<char*>(ws) + p.gemm_off : nullptr;
  for (int k = p.L - 1; k >= p.train_from; --k) {
    const Layer& l = p.layer[k];
    // the input gradient is needed unless every layer below (and the embedding) is frozen
    const bool need_dx = k > p.train_from || p.train_from == 0;
    const float* Hk = (k == 0) ? params : fptr(ws, p.h_off[k]);
    const int64_t ldh = l.in;
    const float* Ws = params + l.off_ws;
    const float* Wn = params + l.off_wn;
    float* dWs = grads + l.off_ws;
    float* dWn = grads + l.off_wn;
    float* dX = (k == 0) ? grads : fptr(ws, p.d_off[ping]);
    const int64_t lddx = l.in;
    const float* mask = (k == 0) ? nullptr : Hk;  // H_k = ReLU output of layer k-1
    if (l.tf) {
      float* T = fptr(ws, p.t_off[tping]);
      tping ^= 1;
      CPRA_CHECK(before_write(T));
      CPRA_CHECK(aggregate(g, true, l.out, dY, lddy, T, l.out, nullptr, 0, nullptr, false, nullptr, 0, st,
                           nullptr, 0, nullptr, 0, queue_of(ws, p, 0)));
      // late: the weight gradients fork after dX, so that they run beside the next
      // layer's gather instead of beside dX's product
      const bool late = side && wgrad_late() && need_dx && k > p.train_from;
      if (late) {
        GemmProblem r{};
        r.piece[0] = GemmPiece{dY, Ws, lddy, l.in, l.out};
        r.piece[1] = GemmPiece{T, Wn, l.out, l.in, l.out};
        r.n_pieces = 2;
        r.C = dX;
        r.ldc = lddx;
        r.M = N;
        r.N = l.in;
        r.mask = mask;
        r.ld_mask = ldh;
        set_groups(p, g, &rows, 1, &r, l);
        CPRA_CHECK(before_write(dX));
        CPRA_CHECK(gemm_batch(false, false, &r, 1, nullptr, 0, st));
      }
      if (side) CPRA_CHECK(fork_mark(side, st));
      auto input_grad = [&]() -> cpra_status {
        if (!need_dx || late) return CPRA_OK;
        GemmProblem r{};
        r.piece[0] = GemmPiece{dY, Ws, lddy, l.in, l.out};
        r.piece[1] = GemmPiece{T, Wn, l.out, l.in, l.out};
        r.n_pieces = 2;
        r.C = dX;
        r.ldc = lddx;
        r.M = N;
        r.N = l.in;
        r.mask = mask;
        r.ld_mask = ldh;
        set_groups(p, g, &rows, 1, &r, l);
        CPRA_CHECK(before_write(dX));
        return gemm_batch(false, false, &r, 1, nullptr, 0, st);
      };
      auto weight_grads = [&]() -> cpra_status {
        if (side) {
          CPRA_CHECK(fork_wait(side));
          CPRA_CHECK(forked());
          pending.add(dY);
          pending.add(T);
        }
        GemmProblem q[2] = {};
        for (int i = 0; i < 2; ++i) {
          q[i].piece[0] = GemmPiece{i == 0 ? dY : T, Hk, i == 0 ? lddy : l.out, ldh, N};
          q[i].n_pieces = 1;
          q[i].C = i == 0 ? dWs : dWn;
          q[i].ldc = l.in;
          q[i].M = l.out;
          q[i].N = l.in;
          set_groups(p, g, &rows, 2, &q[i], l);
        }
        if (p.sage) q[0].bias_grad = grads + l.off_b;  // db = dY^T 1
        return gemm_batch(true, false, q, 2, gemm_ws, p.gemm_bytes, wst);
      };
      if (main_first(k)) {
        CPRA_CHECK(input_grad());
        CPRA_CHECK(weight_grads());
      } else {
        CPRA_CHECK(weight_grads());
        CPRA_CHECK(input_grad());
      }
      if (!need_dx) break;
    } else {
      float* G = fptr(ws, p.g_off);
      const int64_t ldg = 2 * l.in;
      if (side) CPRA_CHECK(fork_mark(side, st));
      auto input_grad = [&]() -> cpra_status {  // G = dY [Ws | Wn]; the gather follows below
        if (!need_dx) return CPRA_OK;
        GemmProblem r[2] = {};
        for (int i = 0; i < 2; ++i) {
          r[i].piece[0] = GemmPiece{dY, i == 0 ? Ws : Wn, lddy, l.in, l.out};
          r[i].n_pieces = 1;
          r[i].C = G + (i == 0 ? 0 : l.in);
          r[i].ldc = ldg;
          r[i].M = N;
          r[i].N = l.in;
          set_groups(p, g, &rows, 1, &r[i], l);
        }
        return gemm_batch(false, false, r, 2, nullptr, 0, st);
      };
      if (main_first(k)) CPRA_CHECK(input_grad());
      if (side) {
        CPRA_CHECK(fork_wait(side));
        CPRA_CHECK(forked());
        pending.add(dY);
      }
      const float* AX;
      if (p.recompute) {
        float* buf = fptr(ws, p.ax_scratch_off);
        CPRA_CHECK(aggregate(g, false, l.in, Hk, ldh, buf, l.in, nullptr, 0, nullptr, false, nullptr, 0, wst,
                             nullptr, 0, nullptr, 0, queue_of(ws, p, side ? 1 : 0)));
        AX = buf;
      } else {
        AX = fptr(ws, p.ax_off[k]);
      }
      GemmProblem q[2] = {};
      for (int i = 0; i < 2; ++i) {
        q[i].piece[0] = GemmPiece{dY, i == 0 ? Hk : AX, lddy, l.in, N};
        q[i].n_pieces = 1;
        q[i].C = i == 0 ? dWs : dWn;
        q[i].ldc = l.in;
        q[i].M = l.out;
        q[i].N = l.in;
        set_groups(p, g, &rows, 2, &q[i], l);
      }
      if (p.sage) q[0].bias_grad = grads + l.off_b;  // db = dY^T 1
      CPRA_CHECK(gemm_batch(true, false, q, 2, gemm_ws, p.gemm_bytes, wst));
      if (!need_dx) break;
      if (!main_first(k)) CPRA_CHECK(input_grad());
      CPRA_CHECK(before_write(dX));
      CPRA_CHECK(aggregate(g, true, l.in, G + l.in, ldg, dX, lddx, G, ldg, nullptr, false, mask, ldh, st,
                           nullptr, 0, nullptr, 0, queue_of(ws, p, 0)));
    }
    dY = dX;
    lddy = lddx;
    ping ^= 1;
  }
  return CPRA_OK;
}

cpra_status check_graph_and_model(const cpra_csr* g, const cpra_model_cfg* cfg, const char* who) {
  CPRA_CHECK(check_csr(g, who, true, false));
  CPRA_CHECK(check_model_cfg(cfg));
  if (cfg->weight_groups > 1 && cfg->weight_groups != g->n_graphs)
    CPRA_FAIL(CPRA_ERR_PARAM, "%s: weight_groups = %d but the graph has %d graphs", who,
              cfg->weight_groups, g->n_graphs);
  return CPRA_OK;
}

}  // namespace

}  // namespace cpra

extern "C" {

int64_t cpra_model_param_count(const cpra_model_cfg* cfg, int32_t n_nodes) {
  if (cpra::check_model_cfg(cfg) != CPRA_OK || n_nodes < 0) return -1;
  cpra::Plan p{};
  cpra::make_layers(cfg, n_nodes, &p);
  return p.n_params;
}

cpra_status cpra_model_param_offsets(const cpra_model_cfg* cfg, int32_t n_nodes, int64_t* offsets) {
  CPRA_CHECK(cpra::check_model_cfg(cfg));
  if (offsets == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "param_offsets: offsets is NULL");
  cpra::Plan p{};
  cpra::make_layers(cfg, n_nodes, &p);
  offsets[0] = 0;
  for (int k = 0; k < p.L; ++k) {
    offsets[1 + 3 * k] = p.layer[k].off_ws;
    offsets[2 + 3 * k] = p.layer[k].off_wn;
    offsets[3 + 3 * k] = p.layer[k].off_b;
  }
  return CPRA_OK;
}

size_t cpra_model_workspace_bytes(const cpra_csr* g, const cpra_model_cfg* cfg) {
  if (g == nullptr || cpra::check_model_cfg(cfg) != CPRA_OK) return 0;
  cpra::Plan p{};
  cpra::make_plan(cfg, g, &p);
  return p.total;
}

cpra_status cpra_model_forward(const cpra_csr* g, const cpra_model_cfg* cfg, const float* params,
                               float* Z, int64_t ldz, void* ws, size_t ws_bytes,
                               cpra_stream_t stream) {
  using namespace cpra;
  CPRA_CHECK(check_graph_and_model(g, cfg, "model_forward"));
  if (ldz < cfg->S) CPRA_FAIL(CPRA_ERR_SHAPE, "model_forward: ldz < S");
  if (g->n_nodes == 0) return CPRA_OK;
  if (params == nullptr || Z == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "model_forward: NULL buffer");
  Plan p{};
  make_plan(cfg, g, &p);
  if (ws == nullptr || ws_bytes < p.total)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "model_forward: workspace %zu < %zu bytes", ws_bytes, p.total);
  return forward_impl(g, p, params, Z, ldz, ws, as_stream(stream));
}

cpra_status cpra_model_backward(const cpra_csr* g, const cpra_model_cfg* cfg, const float* params,
                                const float* dZ, int64_t lddz, float* grads, void* ws,
                                size_t ws_bytes, cpra_stream_t stream) {
  using namespace cpra;
  CPRA_CHECK(check_graph_and_model(g, cfg, "model_backward"));
  if (lddz < cfg->S) CPRA_FAIL(CPRA_ERR_SHAPE, "model_backward: lddz < S");
  if (g->n_nodes == 0) return CPRA_OK;
  if (params == nullptr || dZ == nullptr || grads == nullptr)
    CPRA_FAIL(CPRA_ERR_NULL, "model_backward: NULL buffer");
  Plan p{};
  make_plan(cfg, g, &p);
  if (ws == nullptr || ws_bytes < p.total)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "model_backward: workspace %zu < %zu bytes", ws_bytes, p.total);
  SideStream* side = nullptr;
  if (overlap_enabled()) CPRA_CHECK(get_side_stream(&side));
  CPRA_CHECK(backward_impl(g, p, params, dZ, lddz, grads, ws, as_stream(stream), side, false));
  if (side) CPRA_CHECK(join_from(side, as_stream(stream)));
  return CPRA_OK;
}

cpra_status cpra_model_saved_activation(const cpra_csr* g, const cpra_model_cfg* cfg, void* ws,
                                        size_t ws_bytes, int32_t layer, const float** out,
                                        int64_t* ld) {
  using namespace cpra;
  CPRA_CHECK(check_graph_and_model(g, cfg, "model_saved_activation"));
  if (out == nullptr || ld == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "model_saved_activation: NULL output");
  if (layer < 1 || layer >= cfg->n_layers)
    CPRA_FAIL(CPRA_ERR_PARAM, "model_saved_activation: layer %d outside 1..%d", layer, cfg->n_layers - 1);
  Plan p{};
  make_plan(cfg, g, &p);
  if (ws == nullptr || ws_bytes < p.total)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "model_saved_activation: workspace %zu < %zu bytes", ws_bytes, p.total);
  *out = fptr(ws, p.h_off[layer]);
  *ld = p.layer[layer].in;
  return CPRA_OK;
}

size_t cpra_train_step_workspace_bytes(const cpra_csr* g, const cpra_step_cfg* cfg) {
  if (g == nullptr || cfg == nullptr || cpra::check_model_cfg(&cfg->model) != CPRA_OK) return 0;
  cpra::Plan p{};
  cpra::make_plan(&cfg->model, g, &p);
  return cpra::align_up(p.total, 256) + cpra::loss_workspace_bytes(g, cfg->model.S, false);
}

cpra_status cpra_train_step(const cpra_csr* g, const cpra_step_cfg* cfg, float* params,
                            float* grads, float* m, float* v, float* Z, float* dZ, double* terms,
                            int32_t t, int32_t* step_counter, void* ws, size_t ws_bytes,
                            cpra_stream_t stream) {
  using namespace cpra;
  if (cfg == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "train_step: cfg is NULL");
  CPRA_CHECK(check_graph_and_model(g, &cfg->model, "train_step"));
  if (cfg->loss.problem == CPRA_MAXCUT && cfg->loss.edge_weight == nullptr && g->n_nodes > 0 &&
      g->wdeg == nullptr)
    CPRA_FAIL(CPRA_ERR_NULL, "train_step: wdeg is NULL (run cpra_csr_prepare)");
  cpra_loss_cfg lc = cfg->loss;
  lc.step_counter = step_counter;
  CPRA_CHECK(check_loss_cfg_public(g, &lc));
  CPRA_CHECK(check_adam_cfg(&cfg->adam));
  CPRA_CHECK(check_early_stop_cfg(&cfg->early_stop));
  const bool es = cfg->early_stop.state != nullptr;
  if (es && (terms == nullptr || step_counter == nullptr))
    CPRA_FAIL(CPRA_ERR_PARAM, "train_step: early stopping needs terms and a step counter");
  if (cfg->loss.S != cfg->model.S) CPRA_FAIL(CPRA_ERR_PARAM, "train_step: loss.S != model.S");
  if (step_counter == nullptr && t < 1) CPRA_FAIL(CPRA_ERR_PARAM, "train_step: t must be >= 1");
  if (g->n_nodes == 0) return CPRA_OK;
  if (!params || !grads || !m || !v || !Z || !dZ) CPRA_FAIL(CPRA_ERR_NULL, "train_step: NULL buffer");
  Plan p{};
  make_plan(&cfg->model, g, &p);
  const size_t model_bytes = align_up(p.total, 256);
  const size_t need = model_bytes + loss_workspace_bytes(g, cfg->model.S, false);
  if (ws == nullptr || ws_bytes < need)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "train_step: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = as_stream(stream);
  const int S = cfg->model.S;
  SideStream* side = nullptr;
  if (overlap_enabled()) CPRA_CHECK(get_side_stream(&side));
  void* loss_ws = static_cast<char*>(ws) + model_bytes;
  CPRA_CHECK(forward_impl(g, p, params, Z, S, ws, st));
  CPRA_CHECK(loss_fwd_bwd(g, &lc, Z, S, fptr(ws, p.p_off), S, dZ, S, nullptr, loss_ws,
                          ws_bytes - model_bytes, st, terms != nullptr));
  // The step counter advances (t -> t + 1) after the loss has read t and before
  // Adam reads t + 1: done by one thread of the loss-term reduction, or by a
  // one-thread kernel when no terms are wanted.  With a side stream the
  // per-graph loss terms are reduced there, enqueued by the backward right
  // after its first fork (off the critical path, no fork of their own); Adam
  // runs after the join.  (Adam cannot be split across the streams: the side
  // stream's first-layer weight gradient reads the embedding, and the main
  // stream's last products read the layer weights.)
  // With early stopping the rule's update follows the reduction and advances
  // the counter itself (unless the rule has fired).
  std::function<cpra_status(hipStream_t)> terms_task = [&](hipStream_t s2) {
    CPRA_CHECK(loss_terms_reduce(g, &lc, terms, loss_ws, s2, es ? nullptr : step_counter));
    if (es) CPRA_CHECK(early_stop_update(g, &lc, terms, &cfg->early_stop, step_counter, s2));
    return CPRA_OK;
  };
  if (terms) {
    if (!side) CPRA_CHECK(terms_task(st));
  } else if (step_counter) {
    CPRA_CHECK(increment_counter(step_counter, st));
  }
  CPRA_CHECK(backward_impl(g, p, params, dZ, S, grads, ws, st, side, true,
                           side && terms ? &terms_task : nullptr));
  if (side) CPRA_CHECK(join_from(side, st));
  // only the trainable tail [first trained layer, end) when the encoder is frozen
  const int64_t a0 = p.train_from > 0 ? p.layer[p.train_from].off_ws : 0;
  CPRA_CHECK(adam_step(p.n_params - a0, params + a0, grads + a0, m + a0, v + a0, &cfg->adam, t,
                       step_counter, st, /*t_offset=*/0,
                       es ? &cfg->early_stop.state->stopped : nullptr));
  return CPRA_OK;
}

}  // extern "C"
