/*
 * cpra.h -- C ABI of libcpra, the MI355X (gfx950) implementation of the
 * CPRA training step: S relaxed solutions of one combinatorial problem
 * (or a block-diagonal batch of instances) trained at once by a GNN.
 *
 * Paper: Ichikawa & Iwashita, "Continuous Parallel Relaxation for Finding
 * Diverse Solutions in Combinatorial Optimization Problems", TMLR 2025.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrices are row-major float32 with an explicit leading dimension
 *   (elements between consecutive rows).  Node-by-head matrices are [N, S]
 *   with one node's S heads contiguous.
 * - Pointers documented as "device" must point to device memory owned by
 *   the caller; the library borrows them for the duration of the
 *   stream-ordered work it enqueues and never frees them.  "Host" pointers
 *   are read synchronously before the call returns.
 * - The library allocates no device memory.  Entry points that need
 *   scratch take a caller-owned workspace (ws, ws_bytes) sized by the
 *   matching *_workspace_bytes query; the workspace must stay untouched
 *   until the enqueued work completes.
 * - Every call is asynchronous with respect to the host and ordered on
 *   `stream` (a hipStream_t; NULL means the null stream).  Argument errors
 *   are detected on the host and returned synchronously, before any work is
 *   enqueued.  A launch failure returns CPRA_ERR_HIP; a device fault is
 *   reported by HIP on a later synchronisation.
 * - After a non-OK return, cpra_last_error_message() (thread-local) says
 *   what was wrong.
 * - Results are deterministic: no floating-point atomics; every reduction
 *   runs in a fixed order, so identical inputs give identical bits.
 */
#ifndef CPRA_H
#define CPRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPRA_ABI_VERSION 8

typedef void* cpra_stream_t; /* hipStream_t */

typedef enum {
  CPRA_OK = 0,
  CPRA_ERR_NULL = 1,       /* a required pointer is NULL */
  CPRA_ERR_SHAPE = 2,      /* a size or leading dimension is inconsistent */
  CPRA_ERR_CSR = 3,        /* the graph is not a valid symmetric simple CSR */
  CPRA_ERR_PARAM = 4,      /* a method parameter is out of its domain */
  CPRA_ERR_OVERFLOW = 5,   /* a size does not fit the int32 indexing used on device */
  CPRA_ERR_WORKSPACE = 6,  /* workspace missing or smaller than the query returned */
  CPRA_ERR_HIP = 7,        /* a HIP runtime call or kernel launch failed */
  CPRA_ERR_NONFINITE = 8   /* a host-side float parameter is NaN or infinite */
} cpra_status;

enum { CPRA_MIS = 0, CPRA_MAXCUT = 1 };   /* problems of the objective table */
enum { CPRA_GCN = 0, CPRA_SAGE = 1 };     /* layer forms of the GNN appendix */

/* Version of this ABI (CPRA_ABI_VERSION of the built library). */
int32_t cpra_abi_version(void);
/* Static name of a status code. */
const char* cpra_status_string(cpra_status status);
/* Message of the last failing call on this thread ("" if none). */
const char* cpra_last_error_message(void);

/* ------------------------------------------------------------------------
 * Graph.  Sec. 1 (Notation): an undirected graph G(V, E) with adjacency A,
 * A_ij > 0 on edges.  Stored as symmetric CSR: row i lists the neighbours
 * of node i in strictly increasing order, no self loops, j in row i iff i in
 * row j (with equal weight).  nnz = 2|E|.  A block-diagonal union of
 * n_graphs instances carries their node offsets in graph_ptr.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n_nodes;          /* N >= 0 */
  int32_t n_graphs;         /* >= 1 */
  int64_t nnz;              /* < 2^31 */
  const int32_t* row_ptr;   /* device [N+1] */
  const int32_t* col_idx;   /* device [nnz] */
  const int32_t* graph_ptr; /* device [n_graphs+1] node offsets; NULL iff n_graphs == 1 */
  const float* weight;      /* device [nnz] A_ij, or NULL for A_ij = 1 */
  const float* inv_deg;     /* device [N] 1/|N(i)| (0 for isolated nodes), from cpra_csr_prepare */
  const float* wdeg;        /* device [N] sum_j A_ij, from cpra_csr_prepare */
  const float* col_inv_deg; /* device [nnz] inv_deg[col_idx[e]] per CSR entry, from
                             * cpra_csr_prepare_col, or NULL: the scale of M^T = A D^-1 read
                             * in CSR order by the transposed aggregation instead of one
                             * gather of inv_deg per neighbour (same values, same result) */
} cpra_csr;

/* Host-side validation of a CSR (host pointers).  Checks row_ptr[0] = 0,
 * monotone rows, row_ptr[N] = nnz, indices in range, rows strictly
 * increasing, no self loop, symmetry of structure and weights, finite
 * weights.  O(nnz log d).  Returns CPRA_ERR_CSR (with the first offending
 * row in the message), CPRA_ERR_OVERFLOW or CPRA_ERR_NULL. */
cpra_status cpra_csr_validate_host(int32_t n_nodes, int64_t nnz, const int32_t* row_ptr,
                                   const int32_t* col_idx, const float* weight);

/* Fills inv_deg[N] = 1/|N(i)| (0 if isolated) -- the row scaling of the mean
 * aggregation in the GNN appendix -- and wdeg[N] = sum_j A_ij, the linear
 * coefficient of the MaxCut objective.  Reads g->row_ptr and g->weight only
 * (g->inv_deg / g->wdeg may still be NULL).  Either output may be NULL. */
cpra_status cpra_csr_prepare(const cpra_csr* g, float* inv_deg, float* wdeg, cpra_stream_t stream);

/* Fills col_inv_deg[e] = g->inv_deg[g->col_idx[e]] for every CSR entry e: the
 * factor D^-1 of M^T = A D^-1 (GNN appendix, mean aggregation, transposed for
 * the backward pass) laid out per entry.  Needs g->inv_deg (cpra_csr_prepare);
 * col_inv_deg [nnz] is caller-owned device memory.  CPRA_ERR_NULL when
 * g->inv_deg or col_inv_deg is NULL and nnz > 0. */
cpra_status cpra_csr_prepare_col(const cpra_csr* g, float* col_inv_deg, cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * Mean aggregation (GNN appendix: Aggregate step with the 1/|N(v)|
 * normalisation of the GCN equation).  M = D^-1 A over the neighbour set
 * (edge weights are not used here).
 *   transpose = 0:  Y[i,:] = add[i,:] + bias + inv_deg_i * sum_{j in N(i)} X[j,:]
 *   transpose = 1:  Y[j,:] = add[j,:] + bias + sum_{i in N(j)} inv_deg_i * X[i,:]   (M^T X)
 * then optionally ReLU (relu != 0), then optionally masked:
 *   Y[i,c] = 0 where mask[i,c] <= 0 (mask [N, width] with leading dim ld_mask).
 * X [N, width] (ldx), Y [N, width] (ldy); add (ld_add), bias [width] and
 * mask may be NULL.  add may equal Y (in place); X must not overlap Y.
 * Requires g->inv_deg. */
cpra_status cpra_aggregate_mean(const cpra_csr* g, int32_t transpose, int32_t width,
                                const float* X, int64_t ldx, float* Y, int64_t ldy,
                                const float* add, int64_t ld_add, const float* bias,
                                int32_t relu, const float* mask, int64_t ld_mask,
                                cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * Dense FP32 GEMM on the MFMA units (the GNN's weight products):
 *   C[M,N] = act( op(A) op(B) + beta * C + bias[N] )
 * op(A) is [M,K]: trans_a = 0 -> A stored [M,K] (lda >= K); 1 -> A stored [K,M].
 * op(B) is [K,N]: trans_b = 0 -> B stored [K,N] (ldb >= N); 1 -> B stored [N,K].
 * act = ReLU if relu != 0.  bias may be NULL.  FP32 inputs, FP32 accumulate.
 * Workspace: cpra_gemm_workspace_bytes (split-K partial tiles; may be 0). */
size_t cpra_gemm_workspace_bytes(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K);
cpra_status cpra_gemm(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                      const float* A, int64_t lda, const float* B, int64_t ldb, float beta,
                      float* C, int64_t ldc, const float* bias, int32_t relu,
                      void* ws, size_t ws_bytes, cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * Grouped FP32 GEMM over the graphs of a block-diagonal batch in which every
 * graph has its own weights (Sec. 3.1's multi-instance use of the heads, with
 * one network per instance).  Graph g owns rows graph_ptr[g] .. graph_ptr[g+1]-1
 * of g->graph_ptr (a single graph when g->n_graphs <= 1: the plain product).
 *  mode CPRA_GROUP_ROWS (M = n_nodes):
 *    C[rows of g, :N] = act( A[rows of g, :K] op(B_g) + bias_g ),
 *    B_g = B + g * b_stride: [N,K] (ldb >= K) if trans_b, else [K,N] (ldb >= N);
 *    bias_g = bias + g * bias_stride ([N], may be NULL); act = ReLU if relu;
 *    A [n_nodes, K] (lda >= K), C [n_nodes, N] (ldc >= N).
 *  mode CPRA_GROUP_K (K = n_nodes; trans_b = 0, no bias, no relu):
 *    C_g[:M, :N] = A[rows of g, :M]^T B[rows of g, :N] at C + g * c_stride (ldc >= N),
 *    and, when bias_grad is not NULL, bias_grad[g * bg_stride + m] = sum over
 *    the rows of g of A[r, m] (the bias gradient of graph g's layer);
 *    A [n_nodes, M] (lda >= M), B [n_nodes, N] (ldb >= N).
 * Per-graph blocks must not overlap (strides at least one block's span).
 * Workspace: cpra_gemm_grouped_workspace_bytes (rows: the row-tile maps, built
 * on every call; K: split-K partials, may be 0).  Borrowed, caller-owned. */
enum { CPRA_GROUP_ROWS = 1, CPRA_GROUP_K = 2 };
size_t cpra_gemm_grouped_workspace_bytes(const cpra_csr* g, int32_t mode, int32_t M, int32_t N,
                                         int32_t with_bias_grad);
cpra_status cpra_gemm_grouped(const cpra_csr* g, int32_t mode, int32_t trans_b, int32_t M,
                              int32_t N, int32_t K, const float* A, int64_t lda, const float* B,
                              int64_t ldb, int64_t b_stride, float* C, int64_t ldc,
                              int64_t c_stride, const float* bias, int64_t bias_stride,
                              float* bias_grad, int64_t bg_stride, int32_t relu, void* ws,
                              size_t ws_bytes, cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * Relaxed CPRA objective and its gradient (Sec. 3.1 Eq. CPRA-loss-function-GNN,
 * Sec. 3.2 penalty-diversified form, Sec. 3.3 Eq. CPRA-loss-function-GNN-variation,
 * objective table of the problem-specification appendix):
 *   P = sigmoid(Z),
 *   R = sum_s l_s(P[:,s]) + gamma * sum_{i,s} (1 - (2 P_is - 1)^alpha) + nu * Psi(P),
 *   MIS:    l_s = -sum_i w_is P_is + lambda_s * sum_{i<j} A_ij P_is P_js
 *           (w = 1 unless node weights are given: weighted MIS, one weight
 *           vector per head for the multi-task form of the two-stage appendix)
 *   MaxCut: l_s = sum_{i<j} A_ij (2 P_is P_js - P_is - P_js)
 *   with A_ij the graph's weight (1 when it has none) or, with per-head edge
 *   weights, A_ijs: one instance C_s per head on the graph's pattern (Sec. 3.1
 *   solves S instances at once; the multi-instance appendix, 27 instances of
 *   one structure), a zero leaving the edge out of head s's instance.
 *   Psi    = -S * sum_i STD_s[P_is]  (population STD, or sample STD if std_ddof = 1);
 *            STD_s[P_is] = 0 and dPsi/dP_i: = 0 exactly where all heads of node i
 *            are equal (0 is a subgradient of the norm there)
 * Output dZ = dR/dZ and, per graph g of the batch, terms[g*(S+2) + c]:
 *   c < S: l_c of graph g;  c = S: sum of (1-(2P-1)^alpha) over the graph;
 *   c = S+1: Psi of the graph.  R = sum_s terms[s] + gamma*terms[S] + nu*terms[S+1].
 * Per-node work is FP32; the cross-block sums of the terms are FP64.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t problem;        /* CPRA_MIS or CPRA_MAXCUT */
  int32_t S;              /* heads, 1 <= S <= 1024 */
  int32_t alpha;          /* even, 2 <= alpha <= 64 */
  int32_t std_ddof;       /* 0 or 1 (needs S > std_ddof) */
  float gamma;            /* annealing weight, used when step_counter is NULL */
  float nu;               /* diversity weight */
  const float* lambda;    /* device [S] penalty grid (MIS); ignored for MaxCut */
  /* Optional device-side schedule for captured graphs: when step_counter is
   * non-NULL, gamma = gamma_start + (gamma_end - gamma_start) * min(t, T-1)/(T-1)
   * with t = *step_counter, evaluated in FP64 on the device. */
  const int32_t* step_counter;
  float gamma_start, gamma_end;
  int32_t T;
  /* Optional MIS node weights (device): w_is = node_weight[i * ld_node_weight + s],
   * or node_weight[i] for every head when ld_node_weight = 0.  NULL: w = 1.
   * CPRA_ERR_PARAM for MaxCut. */
  const float* node_weight;
  int64_t ld_node_weight;
  /* Optional per-head edge weights (device), one instance per head:
   * A_ijs = edge_weight[e * ld_edge_weight + s] for CSR entry e = (i, j),
   * ld_edge_weight >= S.  They replace g->weight in the objective (the GNN's
   * mean aggregation is over the pattern either way) and must be symmetric
   * (entries (i, j) and (j, i) equal for every head; not checked on the
   * device).  MaxCut then uses each head's own weighted degree, summed in
   * the same pass, so g->wdeg is not read.  NULL: A_ijs = A_ij for every s. */
  const float* edge_weight;
  int64_t ld_edge_weight;
} cpra_loss_cfg;

size_t cpra_loss_workspace_bytes(const cpra_csr* g, const cpra_loss_cfg* cfg);
/* Z [N,S] (ldz >= S), P = sigmoid(Z) [N,S] (ldp) or NULL to have it computed
 * into the workspace, dZ [N,S] (lddz) or NULL for the forward terms only,
 * terms [n_graphs*(S+2)] doubles or NULL.  Requires g->wdeg for MaxCut. */
cpra_status cpra_loss_fwd_bwd(const cpra_csr* g, const cpra_loss_cfg* cfg,
                              const float* Z, int64_t ldz, const float* P, int64_t ldp,
                              float* dZ, int64_t lddz, double* terms,
                              void* ws, size_t ws_bytes, cpra_stream_t stream);

/* The fused loss that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): cpra_loss_fwd_bwd with its workspace (the item
 * table, the per-item partials and, when P is NULL, P = sigmoid(Z)) in a static
 * device array of CPRA_LOSS_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends.  Arguments, results and errors
 * as cpra_loss_fwd_bwd, plus CPRA_ERR_WORKSPACE when this graph and S need
 * more scratch than the array holds (cpra_loss_workspace_bytes with P NULL;
 * with P given the P area is not needed).  Every call on a GPU shares that
 * GPU's array and leaves its contents to the next call: calls ordered on one
 * stream are safe, calls that overlap in time on one GPU (other streams or
 * threads) race.  The first call on a device looks up the array's address
 * there (hipGetSymbolAddress; no allocation). */
#define CPRA_LOSS_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
cpra_status cpra_loss_fwd_bwd_noalloc(const cpra_csr* g, const cpra_loss_cfg* cfg,
                                      const float* Z, int64_t ldz, const float* P, int64_t ldp,
                                      float* dZ, int64_t lddz, double* terms,
                                      cpra_stream_t stream);

/* The total relaxed loss R of Sec. 3.1 / 3.3 from the per-graph terms that
 * cpra_loss_fwd_bwd writes: R = sum_g (sum_s terms[g][s] + gamma * terms[g][S]
 * + nu * terms[g][S+1]), summed in FP64 on the device in a fixed order (heads
 * in order within a graph, graphs in order), so it needs no host copy.
 * terms: device [n_graphs, S+2] doubles; R: device, one double.
 * CPRA_ERR_NULL / CPRA_ERR_PARAM for NULL pointers, n_graphs < 1 or S < 1. */
cpra_status cpra_loss_total(int32_t n_graphs, int32_t S, const double* terms, double gamma,
                            double nu, double* R, cpra_stream_t stream);

/* P[i,s] = sigmoid(Z[i,s]) (GNN appendix: sigmoid after the last layer). */
cpra_status cpra_sigmoid(int32_t N, int32_t S, const float* Z, int64_t ldz, float* P, int64_t ldp,
                         cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * The GNN P_theta(G) (GNN and architecture appendices):
 *   h^0 = trainable embedding [N, in_dim];
 *   h^k = act(Wn^k * mean_{u in N(v)} h_u^{k-1} + Ws^k h_v^{k-1} (+ b^k for SAGE));
 *   act = ReLU for every layer but the last; the last has S outputs (logits Z).
 * Widths: layer 1 maps in_dim -> hidden, middle layers hidden -> hidden,
 * the last maps to S (n_layers = 1 maps in_dim -> S).
 *
 * Flat parameter layout (float32), offsets from cpra_model_param_offsets:
 *   [embedding N*in_dim] then per layer k: Ws [out_k*in_k], Wn [out_k*in_k],
 *   b [out_k] (SAGE only; absent for GCN).  Each matrix row-major [out, in].
 * With weight_groups = G > 1 (one network per graph of a batch of G graphs)
 *   every layer block holds G copies back to back: Ws [G][out_k][in_k], then
 *   Wn [G][out_k][in_k], then b [G][out_k]; graph g's rows of the batch use
 *   copy g (the embedding is per node already).
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t layer_kind; /* CPRA_GCN (no bias) or CPRA_SAGE (one bias per layer) */
  int32_t n_layers;   /* >= 1 */
  int32_t in_dim;     /* embedding width (>= 1) */
  int32_t hidden;     /* hidden width (>= 1) */
  int32_t S;          /* output width = heads (>= 1) */
  int32_t recompute;  /* 1: backward recomputes neighbour aggregates instead of keeping them */
  /* Optional device [N, S] (contiguous) fixed logits added to the output layer:
   * Z = GNN(G) + z_offset, i.e. P = sigmoid(GNN(G) + z_offset).  This is how a
   * learned warm start (cpra_mpnn_forward) enters CPRA; the backward is
   * unchanged (dZ/d offset = 1, the offset is not trained).  NULL: none. */
  const float* z_offset;
  /* Frozen encoder (the two-stage scheme of Sec. 3.1's last paragraph and the
   * two-stage appendix): layers below train_from_layer, and the embedding when
   * train_from_layer > 0, are not trained -- the backward writes gradients only
   * for layers >= train_from_layer (the others are left untouched) and does not
   * propagate below that layer; cpra_train_step's Adam updates only the
   * trainable tail of the parameter vector.  0: everything is trained. */
  int32_t train_from_layer;
  /* 1: the forward starts at layer train_from_layer (>= 1) from the input that
   * the previous forward on the same workspace saved -- valid because the
   * layers below are frozen (and, unless recompute is set, that layer's saved
   * neighbour aggregate is reused too).  The caller guarantees that such a
   * forward ran on this workspace with the same frozen parameters. */
  int32_t reuse_frozen_prefix;
  /* 0 or 1: one set of layer weights shared by all graphs of a batch.
   * G > 1: one set per graph (the batch's graphs are then independent CPRA
   * problems trained in the same launches); G must equal the graph's
   * n_graphs at every call. */
  int32_t weight_groups;
} cpra_model_cfg;

/* Total float count including the embedding; -1 on invalid config. */
int64_t cpra_model_param_count(const cpra_model_cfg* cfg, int32_t n_nodes);
/* offsets[0] = embedding, then 3 per layer (Ws, Wn, b; b = -1 for GCN); host array
 * of 1 + 3*n_layers int64 entries. */
cpra_status cpra_model_param_offsets(const cpra_model_cfg* cfg, int32_t n_nodes, int64_t* offsets);
/* Bytes of activation storage kept from forward to backward plus backward scratch. */
size_t cpra_model_workspace_bytes(const cpra_csr* g, const cpra_model_cfg* cfg);
/* Z [N,S] (ldz >= S).  Saves the activations the backward needs in ws. */
cpra_status cpra_model_forward(const cpra_csr* g, const cpra_model_cfg* cfg, const float* params,
                               float* Z, int64_t ldz, void* ws, size_t ws_bytes,
                               cpra_stream_t stream);
/* Hand-written backward: grads (same layout as params, fully overwritten) of a
 * scalar loss whose gradient w.r.t. Z is dZ, using the activations that the
 * immediately preceding cpra_model_forward on the same ws saved. */
cpra_status cpra_model_backward(const cpra_csr* g, const cpra_model_cfg* cfg, const float* params,
                                const float* dZ, int64_t lddz, float* grads,
                                void* ws, size_t ws_bytes, cpra_stream_t stream);

/* The input of layer `layer` (1 <= layer < n_layers), i.e. the ReLU output of
 * layer - 1, as saved in ws by the last cpra_model_forward / cpra_train_step
 * on that workspace: a device pointer into ws ([N, hidden], leading dim *ld),
 * valid until the workspace is reused.  Its positive entries are the units
 * whose ReLU derivative the backward takes as 1. */
cpra_status cpra_model_saved_activation(const cpra_csr* g, const cpra_model_cfg* cfg, void* ws,
                                        size_t ws_bytes, int32_t layer, const float** out,
                                        int64_t* ld);

/* ------------------------------------------------------------------------
 * Adam / AdamW (Sec. 4.1 Implementation and the training-setting appendix;
 * Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 *   p = p (1 - lr wd) - lr * (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps),  t >= 1.
 * With step_counter non-NULL, t = *step_counter + 1 is read on the device.
 * ---------------------------------------------------------------------- */
typedef struct {
  double lr, beta1, beta2, eps, weight_decay; /* 1 - beta is formed in FP64 */
} cpra_adam_cfg;

cpra_status cpra_adam_step(int64_t n, float* params, const float* grads, float* m, float* v,
                           const cpra_adam_cfg* cfg, int32_t t, const int32_t* step_counter,
                           cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * One full CPRA training step (Sec. 3.1 loop): forward, sigmoid, loss and
 * dZ, hand-written backward, Adam over all parameters (embedding included).
 * With step_counter non-NULL (a device int32 holding the number of steps
 * done, t - 1), gamma and Adam's t come from the device and the step
 * increments the counter, so the same enqueued work can be captured once and
 * replayed for every step.  The weight-gradient GEMMs and the loss-term
 * reduction run on a library-owned second stream of the current device,
 * forked from and joined back into `stream` by events (also when captured);
 * CPRA_OVERLAP=0 in the environment (read at every call) keeps all work on
 * `stream`.
 * cpra_model_backward overlaps its weight gradients the same way.
 * ---------------------------------------------------------------------- */
/* ------------------------------------------------------------------------
 * Early stopping (Sec. 4.1 Implementation; training-setting appendix: the
 * summed head loss and the annealing term are monitored with a tolerance of
 * 1e-5 and a patience of 10^3 epochs).  Monitored per step t (summed over the
 * graphs of a batch):  L_t = sum_s l_s(P_t),  Phi_t = gamma_t * sum_{i,s}
 * (1 - (2 P_is - 1)^alpha).  Step t (t >= 1) is stalled when neither fell by
 * more than the tolerance (the paper's tolerance is absolute; relative = 1
 * scales it by the previous value's magnitude):
 *   L_t - L_{t-1} >= -tol_L  and  Phi_t - Phi_{t-1} >= -tol_Phi,
 *   tol_X = tol (absolute) or tol |X_{t-1}| (relative).
 * After `patience` consecutive stalled steps the rule fires at that step: its
 * parameter update is skipped, `stopped` is set and the step counter stops
 * advancing, so every later step (eager or replayed) leaves the parameters,
 * the Adam moments and the counter as they are.  The state lives on the
 * device and is updated inside the step, so a captured step carries the
 * rule; the host reads `stopped` whenever it likes (cpra_early_stop_reset
 * initialises it).  Needs terms and a step_counter in cpra_train_step.
 * ---------------------------------------------------------------------- */
typedef struct {
  double prev_head;  /* L of the last evaluated step */
  double prev_phi;   /* Phi of the last evaluated step */
  int32_t stalled;   /* consecutive stalled steps so far */
  int32_t stopped;   /* 1 once the rule fired */
  int32_t stop_step; /* 0-based index t of the step that fired it, -1 before */
  int32_t seen;      /* steps evaluated */
} cpra_early_stop_state;

typedef struct {
  double tol;                   /* tolerance, >= 0 (the paper: 1e-5) */
  int32_t patience;             /* stalled steps that stop training, >= 1 (the paper: 1000) */
  int32_t relative;             /* 0: absolute tolerance (the paper's); 1: relative */
  cpra_early_stop_state* state; /* device, caller-owned; NULL: no early stopping */
} cpra_early_stop_cfg;

/* state = {0, 0, 0, 0, -1, 0} by a kernel on `stream` (valid inside a capture). */
cpra_status cpra_early_stop_reset(cpra_early_stop_state* state, cpra_stream_t stream);

typedef struct {
  cpra_model_cfg model;
  cpra_loss_cfg loss;
  cpra_adam_cfg adam;
  cpra_early_stop_cfg early_stop; /* state == NULL: train every step */
} cpra_step_cfg;

size_t cpra_train_step_workspace_bytes(const cpra_csr* g, const cpra_step_cfg* cfg);
/* params, grads, m, v: flat [cpra_model_param_count]; Z, dZ: [N,S] contiguous;
 * terms: [n_graphs*(S+2)] doubles or NULL; t >= 1 used when step_counter is NULL
 * (then cfg->loss.gamma is this step's gamma). */
cpra_status cpra_train_step(const cpra_csr* g, const cpra_step_cfg* cfg, float* params,
                            float* grads, float* m, float* v, float* Z, float* dZ, double* terms,
                            int32_t t, int32_t* step_counter, void* ws, size_t ws_bytes,
                            cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * Rounding and evaluation (training-setting appendix: P <= 0.5 -> 0,
 * P > 0.5 -> 1, evaluated exactly as Z > 0; objective table; Sec. 4.1
 * Evaluation Metrics; Proposition 3.2).  Per graph g and head s:
 *   MIS:    value = |{i : x_is = 1}|,  violations = |{i<j in E : x_is = x_js = 1}|,
 *           wvalue = sum_i w_is x_is (node weights as in cpra_loss_cfg; 1 if NULL)
 *   MaxCut: value = |{i<j in E : x_is != x_js}| (cut edges), violations = 0,
 *           wvalue = sum of A_ij over cut edges (FP64, fixed-order sums)
 *   pair_hamming[g] = sum_{s<l} d_H(x_s, x_l) = sum_i k_i (S - k_i), k_i = sum_s x_is.
 * With per-head edge weights (edge_weight as in cpra_loss_cfg, or NULL) head s
 * is evaluated on its own instance: E is then the set of edges whose weight
 * in head s is nonzero, and A_ij is that weight.
 * X [N,S] uint8 (ldx), value/violations [n_graphs*S] int64, wvalue
 * [n_graphs*S] double, pair_hamming [n_graphs] int64: each may be NULL.
 * Integer results are exact.
 * ---------------------------------------------------------------------- */
size_t cpra_round_eval_workspace_bytes(const cpra_csr* g, int32_t S);
cpra_status cpra_round_eval(const cpra_csr* g, int32_t problem, int32_t S, const float* Z,
                            int64_t ldz, uint8_t* X, int64_t ldx, int64_t* value,
                            int64_t* violations, double* wvalue, int64_t* pair_hamming,
                            const float* node_weight, int64_t ld_node_weight,
                            const float* edge_weight, int64_t ld_edge_weight,
                            void* ws, size_t ws_bytes, cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * Solution diversity (Sec. 4.1 Evaluation Metrics; the Hamming-distance and
 * unique-solution analyses of the diversity appendix): for the S rounded
 * solutions X (uint8 {0,1} [N, S], ldx >= S; e.g. from cpra_round_eval),
 *   D[s * ldd + l] = d_H(x_s, x_l)        (int32 [S, S], ldd >= S) or NULL,
 *   hist[d] = #{s < l : d_H(x_s, x_l) = d} (int64 [N + 1]) or NULL,
 *   *n_unique = number of distinct solutions among the heads (int32) or NULL.
 * DScore = 2 / (N S (S-1)) * sum_d d hist[d].  Exact integers; S <= 1024.
 * ---------------------------------------------------------------------- */
size_t cpra_pairwise_hamming_workspace_bytes(int32_t N, int32_t S);
cpra_status cpra_pairwise_hamming(int32_t N, int32_t S, const uint8_t* X, int64_t ldx, int32_t* D,
                                  int64_t ldd, int64_t* hist, int32_t* n_unique, void* ws,
                                  size_t ws_bytes, cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * Learned warm start.  The background section's paragraph on learning
 * generalized heuristics from data describes networks trained over many
 * instances that propose a starting point (a meta-learned initialisation) for
 * a new one.  Here a small message-passing network maps per-node structural
 * features to S logits Z_w, and CPRA then trains on
 * P = sigmoid(GNN(G) + Z_w) (cpra_model_cfg.z_offset).
 *
 * bfloat16 tensors cross the ABI as uint16_t bit patterns, rounded to
 * nearest-even from float32 (finite values).
 * ---------------------------------------------------------------------- */

/* Features of every node, bf16 [N, in_dim] (ld_feat >= in_dim):
 *   column 0: d_i / 16;  column 1: local clustering 2 T_i / (d_i (d_i - 1))
 *   (0 if d_i < 2; formed in FP64, rounded to FP32, then to bf16);
 *   columns 2 .. 1 + n_rand: rand [N, n_rand] (ld_rand), caller-drawn;
 *   remaining columns: 0.
 * T_i = number of triangles through i, i.e. pairs of adjacent neighbours
 * (exact integers; written to triangles [N] when non-NULL).  Needs the
 * rows of the CSR sorted (cpra_csr_validate_host).  in_dim >= 2 + n_rand. */
cpra_status cpra_node_features(const cpra_csr* g, int32_t in_dim, int32_t n_rand,
                               const float* rand, int64_t ld_rand, uint16_t* feat, int64_t ld_feat,
                               int64_t* triangles, cpra_stream_t stream);

/* The network: n_layers layers of the GraphSAGE form (GNN appendix, with
 * one bias per layer), widths in_dim -> hidden -> ... -> S:
 *   A_k = bf16(M H_{k-1});  Y_k = H_{k-1} bf16(Ws_k)^T + A_k bf16(Wn_k)^T + b_k
 *   H_k = bf16(relu(Y_k)) (hidden layers);  Z_w = Y_L (float32)
 * with H_0 the features.  Products run on bf16 matrix cores with FP32
 * accumulation.  Parameters are float32 masters, per layer Ws [out, in],
 * Wn [out, in], b [out] (cpra_mpnn_param_offsets); they are rounded to bf16
 * inside every forward.  Limits: in_dim in {16, 32, 48, 64}; hidden in
 * {32, 64}; S a multiple of 32 up to 128. */
typedef struct {
  int32_t n_layers; /* 1..8 */
  int32_t in_dim;
  int32_t hidden;
  int32_t S;
} cpra_mpnn_cfg;

/* Float count of the parameter vector; -1 on an invalid config. */
int64_t cpra_mpnn_param_count(const cpra_mpnn_cfg* cfg);
/* offsets: host array of 3*n_layers entries (Ws, Wn, b per layer). */
cpra_status cpra_mpnn_param_offsets(const cpra_mpnn_cfg* cfg, int64_t* offsets);
size_t cpra_mpnn_workspace_bytes(const cpra_csr* g, const cpra_mpnn_cfg* cfg);
/* Z_w [N, S] contiguous.  feat: bf16 [N, in_dim] contiguous, 16-byte aligned.
 * Keeps the bf16 weights and activations the backward needs in ws. */
cpra_status cpra_mpnn_forward(const cpra_csr* g, const cpra_mpnn_cfg* cfg, const float* params,
                              const uint16_t* feat, float* Zw, void* ws, size_t ws_bytes,
                              cpra_stream_t stream);
/* Hand-written backward of the immediately preceding cpra_mpnn_forward on the
 * same ws: grads (param layout, fully overwritten) of a loss with gradient dZw
 * [N, S] (contiguous float32) w.r.t. Z_w.  Rounding points: dY_L = bf16(dZw);
 * dY_{k-1} = bf16((G_s + M^T G_n) * [H_{k-1} > 0]) with G = dY_k [bf16(Ws) |
 * bf16(Wn)] in FP32; weight and bias gradients in FP32, summed over fixed
 * row blocks in a fixed order (deterministic). */
cpra_status cpra_mpnn_backward(const cpra_csr* g, const cpra_mpnn_cfg* cfg, const uint16_t* feat,
                               const float* dZw, float* grads, void* ws, size_t ws_bytes,
                               cpra_stream_t stream);
/* A device pointer into ws to a tensor saved by the last forward: which = 0,
 * the bf16 input H of layer `layer` (layer >= 1); which = 1, its bf16
 * aggregate A = M H.  [N, in_layer] with leading dimension *ld. */
cpra_status cpra_mpnn_saved(const cpra_csr* g, const cpra_mpnn_cfg* cfg, void* ws, size_t ws_bytes,
                            int32_t layer, int32_t which, const uint16_t** out, int64_t* ld);
/* dZ += beta * (sigmoid(Z) - target): the gradient of beta * sum BCE(sigmoid(Z),
 * target) with logits Z.  target uint8 {0, 1} [n_rows, S] (ldt). */
cpra_status cpra_bce_grad(int32_t n_rows, int32_t S, const float* Z, int64_t ldz,
                          const uint8_t* target, int64_t ldt, float beta, float* dZ, int64_t lddz,
                          cpra_stream_t stream);

/* One training step of the network on a (batched) graph: forward; the CPRA
 * loss of P = sigmoid(Z_w) and its gradient (cpra_loss_fwd_bwd, per graph of
 * the batch); + beta * BCE towards target (converged CPRA solutions, uint8
 * [N, S] contiguous; skipped if NULL or beta = 0); backward; Adam.  Counter,
 * gamma and t semantics as cpra_train_step (loss.gamma_start = gamma_end for
 * a fixed gamma). */
typedef struct {
  cpra_mpnn_cfg net;
  cpra_loss_cfg loss;
  cpra_adam_cfg adam;
  float beta;
} cpra_mpnn_step_cfg;
size_t cpra_mpnn_train_step_workspace_bytes(const cpra_csr* g, const cpra_mpnn_step_cfg* cfg);
cpra_status cpra_mpnn_train_step(const cpra_csr* g, const cpra_mpnn_step_cfg* cfg, float* params,
                                 float* grads, float* m, float* v, const uint16_t* feat,
                                 const uint8_t* target, float* Zw, float* dZw, double* terms,
                                 int32_t t, int32_t* step_counter, void* ws, size_t ws_bytes,
                                 cpra_stream_t stream);

/* ------------------------------------------------------------------------
 * Captured step graphs: enqueue work between begin/end on a non-null stream
 * to record it once; launch replays it.  The only library-owned object.
 * ---------------------------------------------------------------------- */
typedef struct cpra_graph_s* cpra_graph;
cpra_status cpra_capture_begin(cpra_stream_t stream);
cpra_status cpra_capture_end(cpra_stream_t stream, cpra_graph* out);
cpra_status cpra_graph_launch(cpra_graph graph, cpra_stream_t stream);
cpra_status cpra_graph_destroy(cpra_graph graph);

/* ------------------------------------------------------------------------
 * GEMM autotuner.  Between autotune_begin and autotune_end, every GEMM the
 * library runs (cpra_gemm, or inside the model / train-step calls) whose
 * problem shape has no entry in the process-wide tuning table yet is timed
 * under each candidate tile configuration and split-K count that fits the
 * caller's workspace; the fastest is recorded and its result left in C.
 * Tuning synchronises the stream; launches on a stream being captured and
 * GEMMs with beta != 0 are never tuned.  Later calls with a tuned shape use
 * the recorded plan, others a fixed heuristic.  autotune_get reads entry i:
 * the shape key, the chosen configuration index and split count, their name
 * "config/splitN", its time and the time of the heuristic plan (microseconds).
 * ---------------------------------------------------------------------- */
cpra_status cpra_autotune_begin(void);
cpra_status cpra_autotune_end(int32_t* n_entries);
cpra_status cpra_autotune_reset(void);
cpra_status cpra_autotune_get(int32_t i, char* key, size_t key_len, int32_t* cfg, int32_t* splits,
                              char* choice, size_t choice_len, double* us, double* heuristic_us);
/* Insert or replace an entry (e.g. a table saved by an earlier run): shape key
 * as returned by autotune_get, configuration index (0..19) and split count
 * (1..1024; reduced to what the call's workspace holds).  CPRA_ERR_PARAM
 * outside those ranges. */
cpra_status cpra_autotune_set(const char* key, int32_t cfg, int32_t splits);

/* ------------------------------------------------------------------------
 * Per-kernel timing for roofline measurement.  Between profile_begin and
 * profile_end every kernel the library launches on a stream that is not
 * being captured is bracketed by two HIP events on that stream and tagged
 * with a kernel-family name and its algorithmic work (FLOPs for the GEMMs,
 * compulsory HBM bytes for the memory-bound kernels); launches on a stream
 * being captured are not recorded.  profile_collect waits for the recorded
 * events and adds their times to the per-family summary; profile_end frees
 * the events and returns the number of families; profile_get reads family i:
 * launches, summed event time (ms), summed FLOPs, compulsory bytes, and the
 * bytes of rows gathered through an index (neighbour rows of the sparse
 * products, which caches may serve; 0 for other kernels).  Profiling adds
 * two event records per launch: measurement runs only.  An event pair times
 * the kernel plus any wait for the host to launch it, so keep the GPU queue
 * ahead of the host (e.g. start with a sleep on the stream).
 * ---------------------------------------------------------------------- */
cpra_status cpra_profile_begin(void);
cpra_status cpra_profile_stop(void);     /* stop recording new launches, keep the events */
cpra_status cpra_profile_collect(void);  /* add the recorded events' times to the summary */
cpra_status cpra_profile_end(int32_t* n_kernels);
cpra_status cpra_profile_get(int32_t i, char* name, size_t name_len, int64_t* launches,
                             double* total_ms, double* flops, double* bytes, double* gather);

#ifdef __cplusplus
}
#endif
#endif /* CPRA_H */
