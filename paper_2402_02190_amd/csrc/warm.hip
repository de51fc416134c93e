// Learned warm start: per-node structural features and a small message-passing
// network (GraphSAGE form of the GNN appendix, with bias) in bfloat16 on the
// gfx950 matrix cores, with float32 accumulation, plus its backward and
// training step.  The network's output Z_w enters CPRA as fixed logits added
// to the GNN's output (cpra_model_cfg.z_offset).  The idea of a network
// trained across instances that proposes a starting point for a new instance
// is the background section's paragraph on learning generalized heuristics
// from data (meta-learned initialisation).
//
// Storage: bfloat16 activations [N, width] row-major (raw uint16 bit
// patterns, round-to-nearest-even from float32), float32 master weights and
// gradients, float32 output logits.  Kernels:
//  * k_node_features -- one wavefront per node: triangle count by binary
//    search of every neighbour's list in the node's own sorted list (integer,
//    exact), then the feature row [d/16, clustering, random channels, 0...];
//  * k_agg_bf16 -- mean over neighbours of bf16 rows (or, transposed, the
//    M^T gather of float32 rows with an addend and a ReLU mask), float32 sums
//    in CSR order, bf16 result;
//  * k_rows_mfma -- C[N, n_out] = [A_0 | A_1] B: each wavefront streams
//    32-row tiles of A straight from memory into v_mfma_f32_32x32x16_bf16
//    operands while B (the weights, at most 128 x 128) sits in LDS for the
//    whole launch; bias / ReLU / bf16 or float32 store in the epilogue;
//  * k_wgrad_mfma -- per block of rows, the partial dY^T [X_0 | X_1] and the
//    column sums of dY (bias gradient) through LDS-staged 64-row chunks; a
//    second kernel adds the partials in block order (deterministic).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.hpp"

namespace cpra {

cpra_status check_loss_cfg_public(const cpra_csr* g, const cpra_loss_cfg* cfg);
cpra_status check_adam_cfg(const cpra_adam_cfg* cfg);

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxLayers = 8;
constexpr int kMaxWidth = 128;    // n_out and k_total limit of the row GEMM
constexpr int kMaxWgBlocks = 1024;

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline float sigmoid_of(float z) {
  const float e = expf(-fabsf(z));
  const float r = 1.0f / (1.0f + e);
  return z >= 0.0f ? r : e * r;
}

// ------------------------------------------------------------------ features
__global__ __launch_bounds__(256) void k_node_features(int n, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx,
                                                       int in_dim, int n_rand,
                                                       const float* __restrict__ rand,
                                                       int64_t ld_rand, uint16_t* __restrict__ feat,
                                                       int64_t ld_feat, int64_t* __restrict__ tri) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;  // uniform per wavefront
  const int b = row_ptr[i], e = row_ptr[i + 1];
  const int d = e - b;
  long long cnt = 0;  // sum over neighbours j of |N(i) n N(j)| = 2 T_i
  for (int k = b + lane; k < e; k += 64) {
    const int j = col_idx[k];
    const int bj = row_ptr[j], ej = row_ptr[j + 1];
    for (int q = bj; q < ej; ++q) {
      const int x = col_idx[q];
      int lo = b, hi = e;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col_idx[mid] < x) lo = mid + 1; else hi = mid;
      }
      cnt += (lo < e && col_idx[lo] == x) ? 1 : 0;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
  const long long T = cnt / 2;
  if (lane == 0 && tri) tri[i] = T;
  for (int c = lane; c < in_dim; c += 64) {
    float v = 0.0f;
    if (c == 0) {
      v = (float)d * 0.0625f;
    } else if (c == 1) {
      v = d >= 2 ? (float)((2.0 * (double)T) / ((double)d * (double)(d - 1))) : 0.0f;
    } else if (c - 2 < n_rand) {
      v = rand[(int64_t)i * ld_rand + (c - 2)];
    }
    feat[(int64_t)i * ld_feat + c] = f2bf(v);
  }
}

// ------------------------------------------------------------------ casts
__global__ void k_cast_bf16(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

__global__ void k_zero(int64_t n, float* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0f;
}

__global__ void k_cast_rows_bf16(int rows, int cols, const float* __restrict__ x, int64_t ldx,
                                 uint16_t* __restrict__ y, int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * cols) return;
  const int64_t r = i / cols, c = i - r * cols;
  y[r * ldy + c] = f2bf(x[r * ldx + c]);
}

__global__ void k_bce_grad(int rows, int S, const float* __restrict__ Z, int64_t ldz,
                           const uint8_t* __restrict__ target, int64_t ldt, float beta,
                           float* __restrict__ dZ, int64_t lddz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * S) return;
  const int64_t r = i / S, s = i - r * S;
  const float p = sigmoid_of(Z[r * ldz + s]);
  dZ[r * lddz + s] += beta * (p - (float)target[r * ldt + s]);
}

// ------------------------------------------------------------------ aggregation
struct AggBfArgs {
  int n, units, lpr_log2;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* inv_deg;
  const float* col_inv_deg;  // inv_deg of each entry's column, or null (gathered instead)
  const void* X;  // bf16 rows (forward) or float rows (transposed)
  int64_t ldx;
  uint16_t* Y;
  int64_t ldy;
  const float* add;  // transposed only: [N, width] float addend
  int64_t ld_add;
  const uint16_t* mask;  // transposed only: output zeroed where mask <= 0
  int64_t ld_mask;
};

__device__ inline void load8(const uint16_t* p, float* v) {
  const u16x8 w = *reinterpret_cast<const u16x8*>(p);
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = bf2f(w[e]);
}
__device__ inline void load8(const float* p, float* v) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// Each lane owns 8 consecutive columns; the 2^lpr_log2 lanes of a row cover
// its units = width / 8 column groups (NC groups per lane).
template <bool TRANS, int NC>
__global__ __launch_bounds__(256) void k_agg_bf16(AggBfArgs a) {
  using In = typename std::conditional<TRANS, float, uint16_t>::type;
  const In* X = static_cast<const In*>(a.X);
  const int lane = threadIdx.x & 63;
  const int lpr = 1 << a.lpr_log2;
  const int sub = lane >> a.lpr_log2;
  const int cl = lane & (lpr - 1);
  const int row = (blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 >> a.lpr_log2) + sub;
  if (row >= a.n) return;
  float acc[NC][8];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[c][e] = 0.0f;
  const int beg = a.row_ptr[row], end = a.row_ptr[row + 1];
  for (int k = beg; k < end; ++k) {
    const int j = a.col_idx[k];
    const float s = !TRANS ? 1.0f : a.col_inv_deg ? a.col_inv_deg[k] : a.inv_deg[j];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int u = c * lpr + cl;
      if (u < a.units) {
        float v[8];
        load8(X + (int64_t)j * a.ldx + u * 8, v);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (TRANS) acc[c][e] += s * v[e]; else acc[c][e] += v[e];
        }
      }
    }
  }
  const float rs = TRANS ? 1.0f : a.inv_deg[row];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int u = c * lpr + cl;
    if (u >= a.units) continue;
    float r[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = TRANS ? acc[c][e] : acc[c][e] * rs;
    if (TRANS) {
      float ad[8], mk[8];
      load8(a.add + (int64_t)row * a.ld_add + u * 8, ad);
      load8(a.mask + (int64_t)row * a.ld_mask + u * 8, mk);
#pragma unroll
      for (int e = 0; e < 8; ++e) r[e] = (mk[e] > 0.0f) ? r[e] + ad[e] : 0.0f;
    }
    u16x8 w;
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = f2bf(r[e]);
    *reinterpret_cast<u16x8*>(a.Y + (int64_t)row * a.ldy + u * 8) = w;
  }
}

// ------------------------------------------------------------------ row GEMM
struct RowsArgs {
  int M, n_out, k_total;
  const uint16_t* A[2];  // pieces along K, [M, ka[p]] with leading dimension lda[p]
  int64_t lda[2];
  int ka[2];
  const uint16_t* B[2];  // b_kn = 0: [n_out, ka[p]] row-major, pieces along K
  int nb[2];             // b_kn = 1: [k_total, nb[q]] row-major, pieces along N
  int b_kn;
  const float* bias;  // [n_out] or null
  int relu;
  uint16_t* Cb;  // bf16 output [M, n_out] (ldcb) or null
  int64_t ldcb;
  float* Cf;  // float output [M, n_out] (ldcf) or null
  int64_t ldcf;
  int tiles;  // ceil(M / 32)
};

template <int NT>  // n_out / 32 output tiles of 32 columns per wavefront
__global__ __launch_bounds__(256) void k_rows_mfma(RowsArgs a) {
  constexpr int KP = kMaxWidth + 8;  // LDS row pitch (bf16 elements) of B^T
  __shared__ __attribute__((aligned(16))) uint16_t Bt[NT * 32 * KP];
  // stage B^T [n][k] once per block
  const int kt = a.k_total;
  for (int idx = threadIdx.x; idx < NT * 32 * kt; idx += 256) {
    const int n = idx / kt, k = idx - n * kt;
    uint16_t v;
    if (!a.b_kn) {
      const int p = k < a.ka[0] ? 0 : 1;
      const int kk = p ? k - a.ka[0] : k;
      v = a.B[p][(int64_t)n * a.ka[p] + kk];
    } else {
      const int q = n < a.nb[0] ? 0 : 1;
      const int nn = q ? n - a.nb[0] : n;
      v = a.B[q][(int64_t)k * a.nb[q] + nn];
    }
    Bt[n * KP + k] = v;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int m = lane & 31;
  const int g = lane >> 5;
  for (int tile = blockIdx.x * 4 + wave; tile < a.tiles; tile += gridDim.x * 4) {
    const int row = tile * 32 + m;
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
    for (int k0 = 0; k0 < kt; k0 += 16) {
      const int p = k0 < a.ka[0] ? 0 : 1;
      const int kc = (p ? k0 - a.ka[0] : k0) + 8 * g;
      u32x4 av = {0u, 0u, 0u, 0u};
      if (row < a.M) av = *reinterpret_cast<const u32x4*>(a.A[p] + (int64_t)row * a.lda[p] + kc);
      const bf16x8 af = __builtin_bit_cast(bf16x8, av);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const u32x4 bv = *reinterpret_cast<const u32x4*>(&Bt[(t * 32 + m) * KP + k0 + 8 * g]);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, __builtin_bit_cast(bf16x8, bv), acc[t],
                                                         0, 0, 0);
      }
    }
    // acc[t][r] holds C[tile*32 + 8*(r/4) + 4*g + r%4][t*32 + m]
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = t * 32 + m;
      const float bv = a.bias ? a.bias[col] : 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = tile * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
        if (rr >= a.M) continue;
        float v = acc[t][r] + bv;
        if (a.relu) v = fmaxf(v, 0.0f);
        if (a.Cb) a.Cb[(int64_t)rr * a.ldcb + col] = f2bf(v);
        if (a.Cf) a.Cf[(int64_t)rr * a.ldcf + col] = v;
      }
    }
  }
}

// ------------------------------------------------------------------ weight gradient
struct WgArgs {
  int M, n_o, n_c, c0;
  const uint16_t* dY;  // [M, n_o] (lddy)
  int64_t lddy;
  const uint16_t* X0;  // [M, c0] (ldx0)
  int64_t ldx0;
  const uint16_t* X1;  // [M, n_c - c0] (ldx1)
  int64_t ldx1;
  int rows_per_block;
  float* partial;  // [gridDim.x][n_o][n_c + 1]
};

template <int TPW>  // output tiles (32 x 32) per wavefront
__global__ __launch_bounds__(256) void k_wgrad_mfma(WgArgs a) {
  constexpr int CH = 64;               // rows per LDS chunk
  constexpr int YP = kMaxWidth + 8;    // pitches (bf16 elements)
  constexpr int XP = 2 * 64 + 8;
  __shared__ __attribute__((aligned(16))) uint16_t Ys[CH * YP];
  __shared__ __attribute__((aligned(16))) uint16_t Xs[CH * XP];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int m = lane & 31;
  const int g = lane >> 5;
  const int tiles_c = a.n_c / 32;
  const int n_tiles = (a.n_o / 32) * tiles_c;
  f32x16 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.0f;
  float bsum = 0.0f;  // thread o < n_o: column sum of dY (bias gradient)

  const int r_beg = blockIdx.x * a.rows_per_block;
  const int r_end = min(a.M, r_beg + a.rows_per_block);
  const int uy = a.n_o / 8, ux = a.n_c / 8;  // 16-byte units per row
  for (int c0 = r_beg; c0 < r_end; c0 += CH) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < CH * uy; idx += 256) {
      const int r = idx / uy, u = idx - r * uy;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (c0 + r < r_end) v = *reinterpret_cast<const u32x4*>(a.dY + (int64_t)(c0 + r) * a.lddy + u * 8);
      *reinterpret_cast<u32x4*>(&Ys[r * YP + u * 8]) = v;
    }
    for (int idx = threadIdx.x; idx < CH * ux; idx += 256) {
      const int r = idx / ux, u = idx - r * ux;
      const int c = u * 8;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (c0 + r < r_end) {
        const uint16_t* src = c < a.c0 ? a.X0 + (int64_t)(c0 + r) * a.ldx0 + c
                                       : a.X1 + (int64_t)(c0 + r) * a.ldx1 + (c - a.c0);
        v = *reinterpret_cast<const u32x4*>(src);
      }
      *reinterpret_cast<u32x4*>(&Xs[r * XP + c]) = v;
    }
    __syncthreads();
    if (threadIdx.x < a.n_o) {
      for (int r = 0; r < CH; ++r) bsum += bf2f(Ys[r * YP + threadIdx.x]);
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int tile = wave + 4 * i;
      if (tile >= n_tiles) break;
      const int to = tile / tiles_c, tc = tile - to * tiles_c;
      const int o = to * 32 + m, c = tc * 32 + m;
#pragma unroll
      for (int ks = 0; ks < CH; ks += 16) {
        u16x8 av, bv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int r = ks + 8 * g + e;
          av[e] = Ys[r * YP + o];
          bv[e] = Xs[r * XP + c];
        }
        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                         __builtin_bit_cast(bf16x8, bv), acc[i], 0,
                                                         0, 0);
      }
    }
  }
  float* out = a.partial + (int64_t)blockIdx.x * a.n_o * (a.n_c + 1);
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int tile = wave + 4 * i;
    if (tile >= n_tiles) break;
    const int to = tile / tiles_c, tc = tile - to * tiles_c;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int o = to * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
      out[(int64_t)o * (a.n_c + 1) + tc * 32 + m] = acc[i][r];
    }
  }
  if (threadIdx.x < a.n_o) out[(int64_t)threadIdx.x * (a.n_c + 1) + a.n_c] = bsum;
}

// grads of one layer: Ws [n_o, c0], Wn [n_o, n_c - c0], b [n_o]
__global__ void k_wgrad_reduce(int blocks, int n_o, int n_c, int c0, const float* __restrict__ part,
                               float* __restrict__ dWs, float* __restrict__ dWn,
                               float* __restrict__ db) {
  const int per = n_o * (n_c + 1);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= per) return;
  float s = 0.0f;
  for (int b = 0; b < blocks; ++b) s += part[(int64_t)b * per + idx];
  const int o = idx / (n_c + 1), c = idx - o * (n_c + 1);
  if (c < c0) dWs[o * c0 + c] = s;
  else if (c < n_c) dWn[o * (n_c - c0) + (c - c0)] = s;
  else db[o] = s;
}

// ------------------------------------------------------------------ plan
struct MLayer {
  int in, out;
  int64_t off_ws, off_wn, off_b;  // float offsets in the parameter vector
};

struct MPlan {
  int L, N;
  MLayer layer[kMaxLayers];
  int64_t n_params;
  size_t wbf_off;               // bf16 shadow of the parameters
  size_t h_off[kMaxLayers];     // bf16 input of layer k (k >= 1)
  size_t a_off[kMaxLayers];     // bf16 M H of layer k
  size_t dy_off[2];             // bf16 [N, max_out] ping-pong
  size_t g_off;                 // float [N, 2 max_in] (layers k >= 1)
  size_t part_off;              // float [kMaxWgBlocks][max_out (2 max_in + 1)]
  size_t total;
};

cpra_status check_mpnn_cfg(const cpra_mpnn_cfg* cfg) {
  if (cfg == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "mpnn: cfg is NULL");
  if (cfg->n_layers < 1 || cfg->n_layers > kMaxLayers)
    CPRA_FAIL(CPRA_ERR_PARAM, "mpnn: n_layers = %d outside 1..%d", cfg->n_layers, kMaxLayers);
  if (cfg->in_dim < 16 || cfg->in_dim > 64 || cfg->in_dim % 16 != 0)
    CPRA_FAIL(CPRA_ERR_PARAM, "mpnn: in_dim = %d must be 16, 32, 48 or 64", cfg->in_dim);
  if (cfg->n_layers > 1 && (cfg->hidden < 32 || cfg->hidden > 64 || cfg->hidden % 32 != 0))
    CPRA_FAIL(CPRA_ERR_PARAM, "mpnn: hidden = %d must be 32 or 64", cfg->hidden);
  if (cfg->S < 32 || cfg->S > kMaxWidth || cfg->S % 32 != 0)
    CPRA_FAIL(CPRA_ERR_PARAM, "mpnn: S = %d must be a multiple of 32 up to %d", cfg->S, kMaxWidth);
  return CPRA_OK;
}

void make_mplan(const cpra_mpnn_cfg* cfg, int N, MPlan* p) {
  p->L = cfg->n_layers;
  p->N = N;
  int64_t off = 0;
  int d = cfg->in_dim, max_out = 0, max_in1 = 0;
  for (int k = 0; k < p->L; ++k) {
    MLayer& l = p->layer[k];
    l.in = d;
    l.out = (k == p->L - 1) ? cfg->S : cfg->hidden;
    l.off_ws = off;
    off += (int64_t)l.out * l.in;
    l.off_wn = off;
    off += (int64_t)l.out * l.in;
    l.off_b = off;
    off += l.out;
    max_out = std::max(max_out, l.out);
    if (k >= 1) max_in1 = std::max(max_in1, l.in);
    d = l.out;
  }
  p->n_params = off;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align_up(std::max<size_t>(bytes, 1), 256);
    return r;
  };
  p->wbf_off = take((size_t)p->n_params * 2);
  int max_in = 0;
  for (int k = 0; k < p->L; ++k) {
    const MLayer& l = p->layer[k];
    p->h_off[k] = k >= 1 ? take((size_t)N * l.in * 2) : 0;
    p->a_off[k] = take((size_t)N * l.in * 2);
    max_in = std::max(max_in, l.in);
  }
  p->dy_off[0] = take((size_t)N * max_out * 2);
  p->dy_off[1] = take((size_t)N * max_out * 2);
  p->g_off = take((size_t)N * 2 * std::max(max_in1, 1) * 4);
  p->part_off = take((size_t)kMaxWgBlocks * max_out * (2 * max_in + 1) * 4);
  p->total = o;
}

template <typename T>
inline T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

cpra_status agg_bf16(const cpra_csr* g, bool trans, int width, const void* X, int64_t ldx,
                     uint16_t* Y, int64_t ldy, const float* add, int64_t ld_add,
                     const uint16_t* mask, int64_t ld_mask, hipStream_t st) {
  const int units = width / 8;
  int lpr = 1;
  while (lpr < units) lpr <<= 1;
  int lpr_log2 = 0;
  while ((1 << lpr_log2) < lpr) ++lpr_log2;
  AggBfArgs a{g->n_nodes, units, lpr_log2, g->row_ptr, g->col_idx, g->inv_deg, g->col_inv_deg,
              X, ldx, Y, ldy, add, ld_add, mask, ld_mask};
  const int rows_per_block = 4 * (64 >> lpr_log2);
  const int blocks = (int)ceil_div(g->n_nodes, rows_per_block);
  const double in_b = trans ? 4.0 : 2.0;
  const double bytes = (double)g->n_nodes * width * (in_b + 2.0 + (trans ? 6.0 : 0.0)) +
                       4.0 * (double)g->nnz + 8.0 * g->n_nodes;
  ProfScope ps(trans ? "mpnn_aggregate_transposed" : "mpnn_aggregate", st, 0.0, bytes);
  if (trans) hipLaunchKernelGGL((k_agg_bf16<true, 1>), dim3(blocks), dim3(256), 0, st, a);
  else hipLaunchKernelGGL((k_agg_bf16<false, 1>), dim3(blocks), dim3(256), 0, st, a);
  CPRA_CHECK_LAUNCH("mpnn aggregate");
  return CPRA_OK;
}

cpra_status rows_gemm(const RowsArgs& a0, hipStream_t st) {
  RowsArgs a = a0;
  a.tiles = (int)ceil_div(a.M, 32);
  if (a.M == 0) return CPRA_OK;
  const int blocks = (int)std::min<int64_t>(ceil_div(a.tiles, 4), 2048);
  const double flops = 2.0 * a.M * (double)a.n_out * a.k_total;
  const double bytes = (double)a.M * (2.0 * a.k_total + (a.Cb ? 2.0 : 0.0) * a.n_out +
                                      (a.Cf ? 4.0 : 0.0) * a.n_out);
  ProfScope ps("mpnn_gemm_bf16", st, flops, bytes);
  switch (a.n_out / 32) {
    case 1: hipLaunchKernelGGL((k_rows_mfma<1>), dim3(blocks), dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_rows_mfma<2>), dim3(blocks), dim3(256), 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_rows_mfma<3>), dim3(blocks), dim3(256), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_rows_mfma<4>), dim3(blocks), dim3(256), 0, st, a); break;
    default: CPRA_FAIL(CPRA_ERR_SHAPE, "mpnn gemm: n_out %d", a.n_out);
  }
  CPRA_CHECK_LAUNCH("mpnn gemm");
  return CPRA_OK;
}

cpra_status wgrad(const MPlan& p, int k, const uint16_t* dY, const uint16_t* H, float* grads,
                  void* ws, hipStream_t st) {
  const MLayer& l = p.layer[k];
  WgArgs a{};
  a.M = p.N;
  a.n_o = l.out;
  a.n_c = 2 * l.in;
  a.c0 = l.in;
  a.dY = dY;
  a.lddy = l.out;
  a.X0 = H;
  a.ldx0 = l.in;
  a.X1 = at<uint16_t>(ws, p.a_off[k]);
  a.ldx1 = l.in;
  a.rows_per_block = (int)std::max<int64_t>(64, ceil_div(ceil_div(p.N, kMaxWgBlocks), 64) * 64);
  a.partial = at<float>(ws, p.part_off);
  const int blocks = std::max(1, (int)ceil_div(p.N, a.rows_per_block));
  const int n_tiles = (a.n_o / 32) * (a.n_c / 32);
  const int tpw = (n_tiles + 3) / 4;
  {
    const double flops = 2.0 * p.N * (double)a.n_o * a.n_c;
    const double bytes = (double)p.N * 2.0 * (a.n_o + a.n_c) + 4.0 * blocks * a.n_o * (a.n_c + 1);
    ProfScope ps("mpnn_wgrad_bf16", st, flops, bytes);
    switch (tpw) {
      case 1: hipLaunchKernelGGL((k_wgrad_mfma<1>), dim3(blocks), dim3(256), 0, st, a); break;
      case 2: hipLaunchKernelGGL((k_wgrad_mfma<2>), dim3(blocks), dim3(256), 0, st, a); break;
      case 3: hipLaunchKernelGGL((k_wgrad_mfma<3>), dim3(blocks), dim3(256), 0, st, a); break;
      case 4: hipLaunchKernelGGL((k_wgrad_mfma<4>), dim3(blocks), dim3(256), 0, st, a); break;
      default: CPRA_FAIL(CPRA_ERR_SHAPE, "mpnn wgrad: %d tiles", n_tiles);
    }
    CPRA_CHECK_LAUNCH("mpnn wgrad");
  }
  const int per = a.n_o * (a.n_c + 1);
  ProfScope ps("mpnn_wgrad_reduce", st, 0.0, 4.0 * (double)blocks * per + 4.0 * per);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)ceil_div(per, 256)), dim3(256), 0, st, blocks,
                     a.n_o, a.n_c, a.c0, a.partial, grads + l.off_ws, grads + l.off_wn,
                     grads + l.off_b);
  CPRA_CHECK_LAUNCH("mpnn wgrad reduce");
  return CPRA_OK;
}

cpra_status mpnn_forward_impl(const cpra_csr* g, const MPlan& p, const float* params,
                              const uint16_t* feat, float* Zw, void* ws, hipStream_t st) {
  uint16_t* wbf = at<uint16_t>(ws, p.wbf_off);
  {
    ProfScope ps("mpnn_cast", st, 0.0, 6.0 * (double)p.n_params);
    hipLaunchKernelGGL(k_cast_bf16, dim3((unsigned)ceil_div(p.n_params, 256)), dim3(256), 0, st,
                       p.n_params, params, wbf);
    CPRA_CHECK_LAUNCH("mpnn cast");
  }
  const uint16_t* H = feat;
  for (int k = 0; k < p.L; ++k) {
    const MLayer& l = p.layer[k];
    const bool last = k == p.L - 1;
    uint16_t* A = at<uint16_t>(ws, p.a_off[k]);
    CPRA_CHECK(agg_bf16(g, false, l.in, H, l.in, A, l.in, nullptr, 0, nullptr, 0, st));
    RowsArgs r{};
    r.M = p.N;
    r.n_out = l.out;
    r.k_total = 2 * l.in;
    r.A[0] = H;
    r.A[1] = A;
    r.lda[0] = r.lda[1] = l.in;
    r.ka[0] = r.ka[1] = l.in;
    r.B[0] = wbf + l.off_ws;
    r.B[1] = wbf + l.off_wn;
    r.b_kn = 0;
    r.bias = params + l.off_b;
    r.relu = last ? 0 : 1;
    if (last) {
      r.Cf = Zw;
      r.ldcf = l.out;
    } else {
      r.Cb = at<uint16_t>(ws, p.h_off[k + 1]);
      r.ldcb = l.out;
    }
    CPRA_CHECK(rows_gemm(r, st));
    if (!last) H = at<uint16_t>(ws, p.h_off[k + 1]);
  }
  return CPRA_OK;
}

cpra_status mpnn_backward_impl(const cpra_csr* g, const MPlan& p, const uint16_t* feat,
                               const float* dZw, float* grads, void* ws, hipStream_t st) {
  const uint16_t* wbf = at<uint16_t>(ws, p.wbf_off);
  const MLayer& lo = p.layer[p.L - 1];
  uint16_t* dY = at<uint16_t>(ws, p.dy_off[0]);
  {
    const int64_t total = (int64_t)p.N * lo.out;
    ProfScope ps("mpnn_cast", st, 0.0, 6.0 * (double)total);
    hipLaunchKernelGGL(k_cast_rows_bf16, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st,
                       p.N, lo.out, dZw, (int64_t)lo.out, dY, (int64_t)lo.out);
    CPRA_CHECK_LAUNCH("mpnn cast");
  }
  int cur = 0;
  for (int k = p.L - 1; k >= 0; --k) {
    const MLayer& l = p.layer[k];
    const uint16_t* H = k == 0 ? feat : at<uint16_t>(ws, p.h_off[k]);
    CPRA_CHECK(wgrad(p, k, dY, H, grads, ws, st));
    if (k == 0) break;
    float* G = at<float>(ws, p.g_off);
    RowsArgs r{};
    r.M = p.N;
    r.n_out = 2 * l.in;
    r.k_total = l.out;
    r.A[0] = r.A[1] = dY;
    r.lda[0] = r.lda[1] = l.out;
    r.ka[0] = l.out;
    r.ka[1] = 0;
    r.B[0] = wbf + l.off_ws;
    r.B[1] = wbf + l.off_wn;
    r.nb[0] = r.nb[1] = l.in;
    r.b_kn = 1;
    r.Cf = G;
    r.ldcf = 2 * l.in;
    CPRA_CHECK(rows_gemm(r, st));
    uint16_t* dYn = at<uint16_t>(ws, p.dy_off[cur ^ 1]);
    CPRA_CHECK(agg_bf16(g, true, l.in, G + l.in, 2 * l.in, dYn, l.in, G, 2 * l.in, H, l.in, st));
    dY = dYn;
    cur ^= 1;
  }
  return CPRA_OK;
}

cpra_status check_graph_mpnn(const cpra_csr* g, const cpra_mpnn_cfg* cfg, const char* who) {
  CPRA_CHECK(check_csr(g, who, true, false));
  CPRA_CHECK(check_mpnn_cfg(cfg));
  return CPRA_OK;
}

}  // namespace
}  // namespace cpra

extern "C" {

cpra_status cpra_node_features(const cpra_csr* g, int32_t in_dim, int32_t n_rand,
                               const float* rand, int64_t ld_rand, uint16_t* feat, int64_t ld_feat,
                               int64_t* triangles, cpra_stream_t stream) {
  using namespace cpra;
  CPRA_CHECK(check_csr(g, "node_features", false, false));
  if (n_rand < 0 || in_dim < 2 + n_rand)
    CPRA_FAIL(CPRA_ERR_SHAPE, "node_features: in_dim %d < 2 + n_rand %d", in_dim, n_rand);
  if (ld_feat < in_dim || (n_rand > 0 && ld_rand < n_rand))
    CPRA_FAIL(CPRA_ERR_SHAPE, "node_features: leading dimension smaller than the row");
  if (g->n_nodes == 0) return CPRA_OK;
  if (feat == nullptr || (n_rand > 0 && rand == nullptr))
    CPRA_FAIL(CPRA_ERR_NULL, "node_features: feat or rand is NULL");
  hipStream_t st = as_stream(stream);
  const double bytes = 2.0 * g->n_nodes * (double)in_dim + 4.0 * g->n_nodes * (double)n_rand +
                       (triangles ? 8.0 : 0.0) * g->n_nodes + 4.0 * (double)g->nnz +
                       4.0 * (g->n_nodes + 1.0);
  ProfScope ps("node_features", st, 0.0, bytes);
  hipLaunchKernelGGL(k_node_features, dim3((unsigned)ceil_div(g->n_nodes, 4)), dim3(256), 0, st,
                     g->n_nodes, g->row_ptr, g->col_idx, in_dim, n_rand, rand, ld_rand, feat,
                     ld_feat, triangles);
  CPRA_CHECK_LAUNCH("node_features");
  return CPRA_OK;
}

int64_t cpra_mpnn_param_count(const cpra_mpnn_cfg* cfg) {
  if (cpra::check_mpnn_cfg(cfg) != CPRA_OK) return -1;
  cpra::MPlan p{};
  cpra::make_mplan(cfg, 0, &p);
  return p.n_params;
}

cpra_status cpra_mpnn_param_offsets(const cpra_mpnn_cfg* cfg, int64_t* offsets) {
  using namespace cpra;
  CPRA_CHECK(check_mpnn_cfg(cfg));
  if (offsets == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "mpnn_param_offsets: offsets is NULL");
  MPlan p{};
  make_mplan(cfg, 0, &p);
  for (int k = 0; k < p.L; ++k) {
    offsets[3 * k] = p.layer[k].off_ws;
    offsets[3 * k + 1] = p.layer[k].off_wn;
    offsets[3 * k + 2] = p.layer[k].off_b;
  }
  return CPRA_OK;
}

size_t cpra_mpnn_workspace_bytes(const cpra_csr* g, const cpra_mpnn_cfg* cfg) {
  if (g == nullptr || cpra::check_mpnn_cfg(cfg) != CPRA_OK) return 0;
  cpra::MPlan p{};
  cpra::make_mplan(cfg, g->n_nodes, &p);
  return p.total;
}

cpra_status cpra_mpnn_forward(const cpra_csr* g, const cpra_mpnn_cfg* cfg, const float* params,
                              const uint16_t* feat, float* Zw, void* ws, size_t ws_bytes,
                              cpra_stream_t stream) {
  using namespace cpra;
  CPRA_CHECK(check_graph_mpnn(g, cfg, "mpnn_forward"));
  MPlan p{};
  make_mplan(cfg, g->n_nodes, &p);
  if (ws == nullptr || ws_bytes < p.total)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "mpnn_forward: workspace %zu < %zu bytes", ws_bytes, p.total);
  if (!params || !feat || (g->n_nodes > 0 && !Zw)) CPRA_FAIL(CPRA_ERR_NULL, "mpnn_forward: NULL buffer");
  if (reinterpret_cast<uintptr_t>(feat) % 16 != 0)
    CPRA_FAIL(CPRA_ERR_SHAPE, "mpnn_forward: feat must be 16-byte aligned");
  if (g->n_nodes == 0) return CPRA_OK;
  return mpnn_forward_impl(g, p, params, feat, Zw, ws, as_stream(stream));
}

cpra_status cpra_mpnn_backward(const cpra_csr* g, const cpra_mpnn_cfg* cfg, const uint16_t* feat,
                               const float* dZw, float* grads, void* ws, size_t ws_bytes,
                               cpra_stream_t stream) {
  using namespace cpra;
  CPRA_CHECK(check_graph_mpnn(g, cfg, "mpnn_backward"));
  MPlan p{};
  make_mplan(cfg, g->n_nodes, &p);
  if (ws == nullptr || ws_bytes < p.total)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "mpnn_backward: workspace %zu < %zu bytes", ws_bytes, p.total);
  if (!feat || !grads || (g->n_nodes > 0 && !dZw)) CPRA_FAIL(CPRA_ERR_NULL, "mpnn_backward: NULL buffer");
  if (reinterpret_cast<uintptr_t>(feat) % 16 != 0)
    CPRA_FAIL(CPRA_ERR_SHAPE, "mpnn_backward: feat must be 16-byte aligned");
  if (g->n_nodes == 0) {  // no rows: every gradient is an empty sum
    hipLaunchKernelGGL(k_zero, dim3((unsigned)ceil_div(p.n_params, 256)), dim3(256), 0,
                       as_stream(stream), p.n_params, grads);
    CPRA_CHECK_LAUNCH("mpnn_backward");
    return CPRA_OK;
  }
  return mpnn_backward_impl(g, p, feat, dZw, grads, ws, as_stream(stream));
}

cpra_status cpra_mpnn_saved(const cpra_csr* g, const cpra_mpnn_cfg* cfg, void* ws, size_t ws_bytes,
                            int32_t layer, int32_t which, const uint16_t** out, int64_t* ld) {
  using namespace cpra;
  CPRA_CHECK(check_graph_mpnn(g, cfg, "mpnn_saved"));
  if (out == nullptr || ld == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "mpnn_saved: NULL output");
  MPlan p{};
  make_mplan(cfg, g->n_nodes, &p);
  if (ws == nullptr || ws_bytes < p.total)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "mpnn_saved: workspace %zu < %zu bytes", ws_bytes, p.total);
  if (layer < 0 || layer >= p.L || which < 0 || which > 1 || (which == 0 && layer == 0))
    CPRA_FAIL(CPRA_ERR_PARAM, "mpnn_saved: no saved tensor (%d, %d)", layer, which);
  *out = at<uint16_t>(ws, which == 0 ? p.h_off[layer] : p.a_off[layer]);
  *ld = p.layer[layer].in;
  return CPRA_OK;
}

cpra_status cpra_bce_grad(int32_t n_rows, int32_t S, const float* Z, int64_t ldz,
                          const uint8_t* target, int64_t ldt, float beta, float* dZ, int64_t lddz,
                          cpra_stream_t stream) {
  using namespace cpra;
  if (n_rows < 0 || S < 0 || ldz < S || ldt < S || lddz < S)
    CPRA_FAIL(CPRA_ERR_SHAPE, "bce_grad: bad sizes");
  if (!std::isfinite(beta)) CPRA_FAIL(CPRA_ERR_NONFINITE, "bce_grad: beta is not finite");
  const int64_t total = (int64_t)n_rows * S;
  if (total == 0) return CPRA_OK;
  if (!Z || !target || !dZ) CPRA_FAIL(CPRA_ERR_NULL, "bce_grad: NULL buffer");
  hipStream_t st = as_stream(stream);
  ProfScope ps("bce_grad", st, 0.0, 13.0 * (double)total);
  hipLaunchKernelGGL(k_bce_grad, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, n_rows, S,
                     Z, ldz, target, ldt, beta, dZ, lddz);
  CPRA_CHECK_LAUNCH("bce_grad");
  return CPRA_OK;
}

size_t cpra_mpnn_train_step_workspace_bytes(const cpra_csr* g, const cpra_mpnn_step_cfg* cfg) {
  if (g == nullptr || cfg == nullptr || cpra::check_mpnn_cfg(&cfg->net) != CPRA_OK) return 0;
  cpra::MPlan p{};
  cpra::make_mplan(&cfg->net, g->n_nodes, &p);
  return cpra::align_up(p.total, 256) + cpra::loss_workspace_bytes(g, cfg->net.S, true);
}

cpra_status cpra_mpnn_train_step(const cpra_csr* g, const cpra_mpnn_step_cfg* cfg, float* params,
                                 float* grads, float* m, float* v, const uint16_t* feat,
                                 const uint8_t* target, float* Zw, float* dZw, double* terms,
                                 int32_t t, int32_t* step_counter, void* ws, size_t ws_bytes,
                                 cpra_stream_t stream) {
  using namespace cpra;
  if (cfg == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "mpnn_train_step: cfg is NULL");
  CPRA_CHECK(check_graph_mpnn(g, &cfg->net, "mpnn_train_step"));
  cpra_loss_cfg lc = cfg->loss;
  lc.step_counter = step_counter;
  if (lc.S != cfg->net.S) CPRA_FAIL(CPRA_ERR_PARAM, "mpnn_train_step: loss.S != net.S");
  CPRA_CHECK(check_loss_cfg_public(g, &lc));
  CPRA_CHECK(check_adam_cfg(&cfg->adam));
  if (!std::isfinite(cfg->beta)) CPRA_FAIL(CPRA_ERR_NONFINITE, "mpnn_train_step: beta is not finite");
  if (step_counter == nullptr && t < 1) CPRA_FAIL(CPRA_ERR_PARAM, "mpnn_train_step: t must be >= 1");
  if (g->n_nodes == 0) return CPRA_OK;
  if (!params || !grads || !m || !v || !feat || !Zw || !dZw)
    CPRA_FAIL(CPRA_ERR_NULL, "mpnn_train_step: NULL buffer");
  MPlan p{};
  make_mplan(&cfg->net, g->n_nodes, &p);
  const size_t net_bytes = align_up(p.total, 256);
  const size_t need = net_bytes + loss_workspace_bytes(g, cfg->net.S, true);
  if (ws == nullptr || ws_bytes < need)
    CPRA_FAIL(CPRA_ERR_WORKSPACE, "mpnn_train_step: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = as_stream(stream);
  const int S = cfg->net.S;
  void* loss_ws = static_cast<char*>(ws) + net_bytes;
  CPRA_CHECK(mpnn_forward_impl(g, p, params, feat, Zw, ws, st));
  CPRA_CHECK(loss_fwd_bwd(g, &lc, Zw, S, nullptr, 0, dZw, S, nullptr, loss_ws, ws_bytes - net_bytes,
                          st, terms != nullptr));
  if (terms) {
    CPRA_CHECK(loss_terms_reduce(g, &lc, terms, loss_ws, st, step_counter));
  } else if (step_counter) {
    CPRA_CHECK(increment_counter(step_counter, st));
  }
  if (target && cfg->beta != 0.0f) {
    const int64_t total = (int64_t)g->n_nodes * S;
    ProfScope ps("bce_grad", st, 0.0, 13.0 * (double)total);
    hipLaunchKernelGGL(k_bce_grad, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st,
                       g->n_nodes, S, Zw, (int64_t)S, target, (int64_t)S, cfg->beta, dZw, (int64_t)S);
    CPRA_CHECK_LAUNCH("bce_grad");
  }
  CPRA_CHECK(mpnn_backward_impl(g, p, feat, dZw, grads, ws, st));
  CPRA_CHECK(adam_step(p.n_params, params, grads, m, v, &cfg->adam, t, step_counter, st,
                       /*t_offset=*/0));
  return CPRA_OK;
}

}  // extern "C"
