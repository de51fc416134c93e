// The FP32 MFMA GEMM kernel template (v_mfma_f32_32x32x2f32), shared by the
// translation unit of the plain launches (gemm.hip) and that of the launches
// over the graphs of a block-diagonal batch (gemm_grouped.hip), so that the
// two sets of instantiations compile in parallel.  Not part of the ABI.
//
// A block computes a BM x BN tile with WM x WN wavefronts, each owning
// TM x TN = (BM/32/WM) x (BN/32/WN) accumulators of 32 x 32.  K advances in
// BK-deep steps staged through LDS (one barrier per step), in one of four
// loops (PF):
//  * one-deep (1): the next step's global loads are issued before the current
//    step's MFMAs; interior tiles take unguarded float4 loads (a uniform
//    branch), edge tiles guarded ones;
//  * two-deep (2): loads two steps ahead in two register sets, branch-free at
//    clamped addresses;
//  * interleaved (3): loads three steps ahead, the next tile's MFMA operands
//    read into a second register set during the current MFMAs, and every
//    MFMA of a step followed by a fixed share of the step's other work;
//  * LDS ring (4): buffer loads write the tiles straight into a ring of four
//    LDS stages (no registers, no LDS store instructions), three steps ahead,
//    with the interleaved loop's operand reads between the MFMAs (see DmaTile).
// In the first two, tiles are [k][mn] in LDS (K-contiguous operands transposed
// while stored, so an operand read is 32 consecutive floats per
// half-wavefront); the last two keep K-contiguous tiles [row][k] (see Tile).
//
// Group modes (GM) for batches with one weight set per graph, graph g owning
// rows gptr[g] .. gptr[g+1]-1 of the batch:
//  GM = 1 (by rows): C[rows of g] = A[rows of g] op(B_g) (+ bias_g) with
//         B_g = B + g * b_stride and bias_g = bias + g * bias_stride.  Row
//         tiles never cross a graph boundary: a precomputed map gives each
//         row tile's graph, first row and end row;
//  GM = 2 (by K): C_g = A[rows of g]^T B[rows of g] at C + g * c_stride (and
//         the bias gradient of graph g at bias_grad + g * bg_stride): the
//         contraction runs over the graph's rows only.
#pragma once

#include <utility>

#include "common.hpp"

namespace cpra {
namespace gemmk {

// f(integral_constant<int, 0>) ... f(integral_constant<int, N - 1>): a loop
// whose index is a compile-time constant in every copy of the body, so arrays
// it indexes stay in registers however large the body is (a #pragma unroll
// may be declined past the unroller's size limit).
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

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
  float* bias_grad;  // [M] row sums of op(A) over K (computed by the first column tile), or null
  float* sig_out;    // [M, N] (ld_sig): sigmoid of the result, or null
  int64_t ld_sig;
  const float* add;  // [M, N] (ld_add): extra addend, or null
  int64_t ld_add;
  int64_t b_stride, c_stride, bias_stride, bg_stride;  // per-graph offsets (group modes)
  int n_eff;         // N + 1 when bias_grad is set
  int tiles_m, tiles_n;
  int64_t part_off;  // float offset of this problem's split-K partials
};

struct LaunchArgs {
  ProbDev p[kMaxProblems];
  int n_prob;
  int n_vprob;  // problems x graphs in mode 2, else n_prob
  int splits;
  int grid_x;   // 2-D grid: blocks per problem (a multiple of 8); 1-D grid: tiles per group
  float* partial;
  int G;                   // graphs (mode 2: C / partial sets per problem); 1 otherwise
  const int32_t* gptr;     // [G + 1] graph row offsets (mode 2)
  const int4* row_map;     // mode 1: per row tile {graph, first row, end row, 0}; graph -1: none
  const int4* row_maps[3];  // the maps for BM = 32, 64, 128 (the launcher picks row_map)
  int row_counts[3];
};

// One operand tile (R rows or columns of the output by BK steps of K) in LDS,
// loaded by NT threads as float4 vectors.  Layout [BK][LD] (K-contiguous
// operands transposed while stored, LD = R + 1; others LD = R + 4), or with
// ROWK a K-contiguous tile kept [R][BK], stored in whole float4s.  In that
// layout the 16-byte chunks of row r are permuted, chunk c at c ^ swz(r) with
// swz(r) = (r / (64/BK)) mod (BK/4): the rows that share a 256-byte bank line
// keep their chunks in place, so a store's 16 lanes fill the 64 banks once, and
// a read of one chunk by 16 consecutive rows finds it at 16 different banks.
// The interleaved loop reads MFMA operands with k = h * BK/2 + kk for
// half-wavefront h and MFMA kk (any order of a tile's k works when both operands
// use it): in the [R][BK] layout a lane's operands of a tile are BK/2
// consecutive floats, read as float4s.
template <int R, int BK, int NT, bool KCONTIG, bool ROWK = false>
struct Tile {
  static constexpr bool RK = KCONTIG && ROWK;
  static constexpr int PAD = KCONTIG ? 1 : 4;
  static constexpr int LD = R + PAD;  // [BK][LD] layout: row stride (floats)
  static constexpr int LDK = BK;  // [R][BK] layout: row stride (floats)
  static constexpr int SIZE = RK ? R * LDK : BK * LD;  // floats of LDS
  static_assert(!RK || (BK >= 16 && 64 % BK == 0 && BK % 8 == 0), "[row][k] layout: BK 16 or 32");
  // physical 16-byte chunk of logical chunk c in row r of the [R][BK] layout
  __device__ static inline int chunk_at(int r, int c) { return c ^ ((r / (64 / BK)) % (BK / 4)); }
  static constexpr int NREAD = RK ? BK / 8 : BK / 2;   // operand reads per row, interleaved loop
  static constexpr int NV = R * BK / 4 / NT;
  static_assert(NV >= 1 && R * BK / 4 % NT == 0, "tile does not divide among the threads");
  float4 reg[NV];

  __device__ inline void load(const float* __restrict__ X, int64_t ld, int mn0, int mn_lim, int k0,
                              int k_lim, bool vec_ok, int tid) {
    const bool full = vec_ok && (mn0 + R <= mn_lim) && (k0 + BK <= k_lim);
    if (full) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int idx = tid + v * NT;
        if constexpr (KCONTIG) {
          const int r = idx / (BK / 4);
          const int kq = (idx % (BK / 4)) * 4;
          reg[v] = *reinterpret_cast<const float4*>(X + (int64_t)(mn0 + r) * ld + k0 + kq);
        } else {
          const int k = idx / (R / 4);
          const int rq = (idx % (R / 4)) * 4;
          reg[v] = *reinterpret_cast<const float4*>(X + (int64_t)(k0 + k) * ld + mn0 + rq);
        }
      }
      return;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = tid + v * NT;
      if constexpr (KCONTIG) {
        const int r = idx / (BK / 4);
        const int kq = (idx % (BK / 4)) * 4;
        const int gm = mn0 + r, gk = k0 + kq;
        const bool rok = gm < mn_lim;
        const float* p = X + (int64_t)(rok ? gm : 0) * ld;
        reg[v].x = (rok && gk + 0 < k_lim) ? p[gk + 0] : 0.f;
        reg[v].y = (rok && gk + 1 < k_lim) ? p[gk + 1] : 0.f;
        reg[v].z = (rok && gk + 2 < k_lim) ? p[gk + 2] : 0.f;
        reg[v].w = (rok && gk + 3 < k_lim) ? p[gk + 3] : 0.f;
      } else {
        const int k = idx / (R / 4);
        const int rq = (idx % (R / 4)) * 4;
        const int gk = k0 + k, gm = mn0 + rq;
        const bool kok = gk < k_lim;
        const float* p = X + (int64_t)(kok ? gk : 0) * ld;
        reg[v].x = (kok && gm + 0 < mn_lim) ? p[gm + 0] : 0.f;
        reg[v].y = (kok && gm + 1 < mn_lim) ? p[gm + 1] : 0.f;
        reg[v].z = (kok && gm + 2 < mn_lim) ? p[gm + 2] : 0.f;
        reg[v].w = (kok && gm + 3 < mn_lim) ? p[gm + 3] : 0.f;
      }
    }
  }

  // Branch-free load for the two-deep prefetch: every access is one float4 at
  // a clamped, in-bounds address.  Rows or columns past mn_lim only feed
  // outputs that are never stored; vectors past k_lim are flagged in `ok` and
  // zeroed by store_masked, so no loaded value is consumed before the LDS
  // store that has to wait for it anyway.  Requires float4-aligned operands,
  // mn_lim >= 4 when MN is the contiguous axis, and k_lim a multiple of 4
  // (relative to k0) when K is the contiguous axis (see pf2_ok).
  unsigned ok;
  __device__ inline void load_clamped(const float* __restrict__ X, int64_t ld, int mn0, int mn_lim,
                                      int k0, int k_lim, int tid) {
    ok = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = tid + v * NT;
      if constexpr (KCONTIG) {
        const int r = idx / (BK / 4);
        const int kq = (idx % (BK / 4)) * 4;
        const int gm = min(mn0 + r, mn_lim - 1);
        const bool val = k0 + kq < k_lim;
        const int gk = val ? k0 + kq : k_lim - 4;
        reg[v] = *reinterpret_cast<const float4*>(X + (int64_t)gm * ld + gk);
        ok |= (unsigned)val << v;
      } else {
        const int k = idx / (R / 4);
        const int rq = (idx % (R / 4)) * 4;
        const bool val = k0 + k < k_lim;
        const int gk = val ? k0 + k : k_lim - 1;
        const int gm = min(mn0 + rq, mn_lim - 4);
        reg[v] = *reinterpret_cast<const float4*>(X + (int64_t)gk * ld + gm);
        ok |= (unsigned)val << v;
      }
    }
  }

  __device__ inline void store_masked(float* __restrict__ Xs, int tid) const {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = tid + v * NT;
      const bool val = (ok >> v) & 1u;
      const float4 x = val ? reg[v] : make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (RK) {
        const int r = idx / (BK / 4);
        const int c = idx % (BK / 4);
        *reinterpret_cast<float4*>(Xs + r * LDK + 4 * chunk_at(r, c)) = x;
      } else if constexpr (KCONTIG) {
        const int r = idx / (BK / 4);
        const int kq = (idx % (BK / 4)) * 4;
        Xs[(kq + 0) * LD + r] = x.x;
        Xs[(kq + 1) * LD + r] = x.y;
        Xs[(kq + 2) * LD + r] = x.z;
        Xs[(kq + 3) * LD + r] = x.w;
      } else {
        const int k = idx / (R / 4);
        const int rq = (idx % (R / 4)) * 4;
        *reinterpret_cast<float4*>(Xs + k * LD + rq) = x;
      }
    }
  }

  // Vector v of load_clamped / store_masked alone (the interleaved loop spreads
  // them between MFMAs); load_one<0> starts a new `ok` mask.
  template <int v>
  __device__ inline void load_one(const float* __restrict__ X, int64_t ld, int mn0, int mn_lim, int k0,
                                  int k_lim, int tid) {
    const int idx = tid + v * NT;
    bool val;
    if constexpr (KCONTIG) {
      const int r = idx / (BK / 4);
      const int kq = (idx % (BK / 4)) * 4;
      const int gm = min(mn0 + r, mn_lim - 1);
      val = k0 + kq < k_lim;
      const int gk = val ? k0 + kq : k_lim - 4;
      reg[v] = *reinterpret_cast<const float4*>(X + (int64_t)gm * ld + gk);
    } else {
      const int k = idx / (R / 4);
      const int rq = (idx % (R / 4)) * 4;
      val = k0 + k < k_lim;
      const int gk = val ? k0 + k : k_lim - 1;
      const int gm = min(mn0 + rq, mn_lim - 4);
      reg[v] = *reinterpret_cast<const float4*>(X + (int64_t)gk * ld + gm);
    }
    if constexpr (v == 0) ok = (unsigned)val;
    else ok |= (unsigned)val << v;
  }
  template <int v>
  __device__ inline void store_one(float* __restrict__ Xs, int tid) const {
    const int idx = tid + v * NT;
    // vectors past K become +0 by clearing their bits: no select, so no branch
    // splits the MFMA slots around the store
    const unsigned keep = 0u - ((ok >> v) & 1u);
    const float4 x = make_float4(__uint_as_float(__float_as_uint(reg[v].x) & keep),
                                 __uint_as_float(__float_as_uint(reg[v].y) & keep),
                                 __uint_as_float(__float_as_uint(reg[v].z) & keep),
                                 __uint_as_float(__float_as_uint(reg[v].w) & keep));
    if constexpr (RK) {
      const int r = idx / (BK / 4);
      const int c = idx % (BK / 4);
      *reinterpret_cast<float4*>(Xs + r * LDK + 4 * chunk_at(r, c)) = x;
    } else if constexpr (KCONTIG) {
      const int r = idx / (BK / 4);
      const int kq = (idx % (BK / 4)) * 4;
      Xs[(kq + 0) * LD + r] = x.x;
      Xs[(kq + 1) * LD + r] = x.y;
      Xs[(kq + 2) * LD + r] = x.z;
      Xs[(kq + 3) * LD + r] = x.w;
    } else {
      const int k = idx / (R / 4);
      const int rq = (idx % (R / 4)) * 4;
      *reinterpret_cast<float4*>(Xs + k * LD + rq) = x;
    }
  }
  // Read q of the interleaved loop's operands of row or column mn for
  // half-wavefront h: v[kk] for k = h * BK/2 + kk.
  template <int q>
  __device__ static inline void read_part(const float* Xs, int mn, int h, float (&v)[BK / 2]) {
    if constexpr (RK) {
      const float4 x =
          *reinterpret_cast<const float4*>(Xs + mn * LDK + 4 * chunk_at(mn, h * (BK / 8) + q));
      v[4 * q + 0] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    } else {
      v[q] = Xs[(h * (BK / 2) + q) * LD + mn];
    }
  }

  __device__ inline void store(float* __restrict__ Xs, int tid) const {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = tid + v * NT;
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

// One operand tile of the LDS-ring loop: R rows or columns of the output by BK
// steps of K, R * BK floats per stage with no padding.  A buffer load with the
// LDS flag writes the 16 bytes of lane l of a wavefront to LDS at the
// instruction's base + 16 l, so a stage is filled in 16-byte slots, slot
// v * NT + tid by vector v of thread tid, and the layout is chosen through the
// global vector each thread fetches for its slot:
//  * K-contiguous operands: [R][BK] with the chunk permutation of Tile's
//    [row][k] layout (slot (r, c) holds logical chunk chunk_at(r, c), the
//    permutation being its own inverse), read as float4s like Tile::read_part;
//  * others: [BK][R] with the column index of the rows in the second half of
//    the tile (k >= BK/2) XOR-ed with 32, so that the two half-wavefronts,
//    which read k and k + BK/2 at the same 32 columns, meet different banks.
// A vector outside the matrix (rows or columns past the edge, k past the
// piece's end) is given a byte offset past the buffer's range (2^31 - 1
// bytes), and the hardware writes zeros for it; valid offsets are below 2^31
// bytes (the launcher checks the operands' extents).
template <int R, int BK, int NT, bool KCONTIG>
struct DmaTile {
  static constexpr int SIZE = R * BK;  // floats per stage
  static constexpr int NV = SIZE / 4 / NT;
  static constexpr int NREAD = KCONTIG ? BK / 8 : BK / 2;
  static_assert(NV >= 1 && (SIZE / 4) % NT == 0, "tile does not divide among the threads");
  static_assert(KCONTIG || R % 64 == 0, "[k][mn] stage: a multiple of 64 columns");
  using RowK = Tile<R, BK, NT, true, true>;
  unsigned off[2][NV];  // per K piece: float offset of vector v without the k0 term
  unsigned kq[NV];      // k of vector v within the tile
  unsigned mn_ok;       // bit v: the vector's row or columns lie inside the matrix

  __device__ inline void setup(int64_t ld0, int64_t ld1, int mn0, int mn_lim, int tid) {
    mn_ok = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int s = v * NT + tid;
      if constexpr (KCONTIG) {
        const int r = s / (BK / 4);
        const int c = RowK::chunk_at(r, s % (BK / 4));
        const unsigned row = (unsigned)(mn0 + r);
        off[0][v] = row * (unsigned)ld0 + 4u * c;
        off[1][v] = row * (unsigned)ld1 + 4u * c;
        kq[v] = 4u * c;
        mn_ok |= (unsigned)(mn0 + r < mn_lim) << v;
      } else {
        const int k = s / (R / 4);
        const int c = (s % (R / 4)) ^ (((k / (BK / 2)) & 1) * 8);
        const unsigned col = (unsigned)(mn0 + 4 * c);
        off[0][v] = (unsigned)k * (unsigned)ld0 + col;
        off[1][v] = (unsigned)k * (unsigned)ld1 + col;
        kq[v] = (unsigned)k;
        mn_ok |= (unsigned)(mn0 + 4 * c < mn_lim) << v;
      }
    }
  }
  // Byte offset of vector v for the tile starting at k0 of piece pc (k_lim: the
  // piece's end; ld: its leading dimension).  A vector outside the matrix gets
  // bit 31 set, which puts it past the buffer's range whatever the rest holds
  // (valid offsets stay below 2^31): no select, so no branch.
  template <int v>
  __device__ inline unsigned voffset(int pc, int k0, int k_lim, int64_t ld) const {
    const unsigned ok = ((mn_ok >> v) & 1u) & (unsigned)(k0 + (int)kq[v] < k_lim);
    const unsigned o = KCONTIG ? off[pc][v] + (unsigned)k0 : off[pc][v] + (unsigned)k0 * (unsigned)ld;
    return (4u * o) | ((ok ^ 1u) << 31);
  }
  // Element (row or column mn, k) of a stage.
  __device__ static inline float at(const float* Xs, int mn, int k) {
    if constexpr (KCONTIG) {
      return Xs[mn * BK + 4 * RowK::chunk_at(mn, k / 4) + k % 4];
    } else {
      return Xs[k * R + (mn ^ (32 * ((k / (BK / 2)) & 1)))];
    }
  }
  // Read q of the operands of row or column mn for half-wavefront h:
  // v[kk] for k = h * BK/2 + kk.
  template <int q>
  __device__ static inline void read_part(const float* Xs, int mn, int h, float (&v)[BK / 2]) {
    if constexpr (KCONTIG) {
      RowK::template read_part<q>(Xs, mn, h, v);
    } else {
      v[q] = Xs[(h * (BK / 2) + q) * R + (mn ^ (32 * h))];
    }
  }
};

// One 16-byte buffer load per lane of base[voff] (voff in bytes; past 2^31 - 1:
// zeros) into LDS at lds + 16 * lane (lds the same for the whole wavefront).
// The size check of the builtin knows gfx950 only in the device pass.
__device__ inline void load_lds16(const float* base, float* lds, unsigned voff) {
#if defined(__HIP_DEVICE_COMPILE__)
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7fffffff, 0x00020000);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)lds, 16, voff, 0, 0, 0);
#endif
}

// s_waitcnt operand: vector-memory count at most `vm`, LDS count zero, export
// count unchecked (vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
constexpr int waitcnt_vm_lgkm0(int vm) { return (vm & 15) | (7 << 4) | ((vm >> 4) << 14); }

// C[row, col] = mask(relu(v + add + beta C)) and optionally sigmoid(C) into sig_out.
__device__ inline void epilogue_store(const ProbDev& P, float* C, int row, int col, float v) {
  float* cp = C + (int64_t)row * P.ldc + col;
  if (P.add) v += P.add[(int64_t)row * P.ld_add + col];
  if (P.beta != 0.f) v += P.beta * *cp;
  if (P.relu) v = fmaxf(v, 0.f);
  if (P.mask && !(P.mask[(int64_t)row * P.ld_mask + col] > 0.f)) v = 0.f;
  *cp = v;
  if (P.sig_out) {
    const float e = expf(-fabsf(v));
    const float r = 1.0f / (1.0f + e);
    P.sig_out[(int64_t)row * P.ld_sig + col] = v >= 0.0f ? r : e * r;
  }
}

// A_T: A stored [K, M] (M contiguous); otherwise [M, K].
// B_T: B stored [N, K] (K contiguous); otherwise [K, N].
// PF: prefetch distance in K tiles (1: the next tile is loaded while the
// current one is multiplied; 2: two tiles ahead, in two register sets, so a
// load has two K steps of MFMA work to land; 3: the interleaved loop, loads
// three tiles ahead with the step's work spread between its MFMAs; 4: the
// LDS ring, tiles written to LDS by the loads themselves, three tiles ahead).
// GM: group mode (0 none, 1 by rows, 2 by K).
// Waves per SIMD the register allocation aims for: one where a wave holds
// eight or more 32x32 accumulators (the whole register file is then one
// wave's), else the compiler's default.
template <int BM, int BN, int WM, int WN>
constexpr int min_waves_per_eu() {
  return (BM / (32 * WM)) * (BN / (32 * WN)) >= 8 ? 1 : 0;
}

template <int BM, int BN, int BK, int WM, int WN, bool A_T, bool B_T, int PF, int GM>
__global__ __launch_bounds__(64 * WM * WN)
__attribute__((amdgpu_waves_per_eu(min_waves_per_eu<BM, BN, WM, WN>(), min_waves_per_eu<BM, BN, WM, WN>())))
void k_gemm(LaunchArgs args) {
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / (32 * WM);  // 32x32 accumulators per wave along M
  constexpr int TN = BN / (32 * WN);
  static_assert(TM >= 1 && TN >= 1 && TM * 32 * WM == BM && TN * 32 * WN == BN, "bad tiling");
  using TA = Tile<BM, BK, NT, !A_T, PF == 3>;
  using TB = Tile<BN, BK, NT, B_T, PF == 3>;
  __shared__ __attribute__((aligned(16))) float As[2][TA::SIZE];
  __shared__ __attribute__((aligned(16))) float Bs[2][TB::SIZE];

  // XCD-aware order: the hardware deals consecutive block ids round-robin to
  // the 8 XCDs, each with its own L2.
  //  * 2-D grid (tiles x problems; no split, modes 0 and 1): each XCD gets a
  //    contiguous run of tiles, so neighbouring N tiles share their A panel in
  //    that XCD's L2;
  //  * 1-D grid (split-K, or mode 2): all tiles of one (problem, graph, split)
  //    group -- which read the same K rows of A and B -- go to the same XCD.
  int vp, split, tile;
  if (GM != 2 && args.splits == 1) {
    vp = blockIdx.y;
    split = 0;
    const int per_xcd = args.grid_x / 8;
    tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  } else {
    const int x = blockIdx.x % 8, j = blockIdx.x / 8;
    const int group = x + 8 * (j / args.grid_x);  // grid_x = tiles per group here
    tile = j % args.grid_x;
    if (group >= args.n_vprob * args.splits) return;
    vp = group / args.splits;
    split = group % args.splits;
  }
  int prob = vp, grp = 0;
  if constexpr (GM == 2) {
    prob = vp / args.G;
    grp = vp - prob * args.G;
  }
  const ProbDev& P = args.p[prob];
  if (tile >= P.tiles_m * P.tiles_n) return;
  const int tm_idx = tile / P.tiles_n;
  const int tn_idx = tile % P.tiles_n;
  int m0 = tm_idx * BM;
  const int n0 = tn_idx * BN;

  // operands, limits and outputs of this block's (problem, graph)
  int m_lim = P.M;
  int kb = 0, kn0 = P.K[0], kn1 = P.K[1];
  int64_t b_off = 0;
  float* Cg = P.C;
  const float* bias_g = P.bias;
  float* bgrad_g = P.bias_grad;
  bool vA0 = P.vecA[0] != 0, vA1 = P.vecA[1] != 0, vB0 = P.vecB[0] != 0, vB1 = P.vecB[1] != 0;
  if constexpr (GM == 1) {
    const int4 e = args.row_map[tm_idx];
    if (e.x < 0) return;  // past the last row tile of the batch
    m0 = e.y;
    m_lim = e.z;
    b_off = (int64_t)e.x * P.b_stride;
    if (bias_g) bias_g += (int64_t)e.x * P.bias_stride;
  } else if constexpr (GM == 2) {
    kb = args.gptr[grp];
    const int kn = args.gptr[grp + 1] - kb;
    kn0 = kn;
    kn1 = P.n_pieces > 1 ? kn : 0;
    Cg += (int64_t)grp * P.c_stride;
    if (bgrad_g) bgrad_g += (int64_t)grp * P.bg_stride;
    if (kb & 3) {  // K-contiguous operands lose their float4 alignment at this offset
      if (!A_T) vA0 = vA1 = false;
      if (B_T) vB0 = vB1 = false;
    }
  }

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int half = lane >> 5, l32 = lane & 31;

  const int nt0 = (kn0 + BK - 1) / BK;
  const int nt1 = P.n_pieces > 1 ? (kn1 + BK - 1) / BK : 0;
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

  // the operands of both K pieces, read from the arguments once
  const float* const A0p = P.A[0];
  const float* const A1p = P.A[1];
  const float* const B0p = P.B[0] + b_off;
  const float* const B1p = P.B[1] + b_off;
  const int64_t lda0 = P.lda[0], lda1 = P.lda[1], ldb0 = P.ldb[0], ldb1 = P.ldb[1];
  const int n_lim = P.N;
  auto load_into = [&](TA& ta, TB& tb, int kt) {
    const int pc = kt < nt0 ? 0 : 1;
    const int k0 = kb + (kt - (pc ? nt0 : 0)) * BK;
    const int kl = kb + (pc ? kn1 : kn0);
    if constexpr (PF >= 2) {
      ta.load_clamped(P.A[pc], P.lda[pc], m0, m_lim, k0, kl, tid);
      tb.load_clamped(P.B[pc] + b_off, P.ldb[pc], n0, P.N, k0, kl, tid);
    } else {
      ta.load(P.A[pc], P.lda[pc], m0, m_lim, k0, kl, pc ? vA1 : vA0, tid);
      tb.load(P.B[pc] + b_off, P.ldb[pc], n0, P.N, k0, kl, pc ? vB1 : vB0, tid);
    }
  };
  // Bias gradient (row sums of op(A) over this block's K range): the blocks of
  // the first column tile add up the staged A tile with plain VALU adds, thread
  // t owning row t % BM and a fixed slice of each tile's BK rows (zero padding
  // outside the matrix is already in the tile).
  constexpr int BG = NT / BM > 0 ? NT / BM : 1;  // threads per row
  static_assert(BK % BG == 0, "bias slice");
  static_assert(NT >= BM, "every row of the A tile needs a thread for the bias slice");
  const bool do_bias = bgrad_g != nullptr && tn_idx == 0;
  const int b_row = tid % BM, b_grp = tid / BM;
  float bsum = 0.f;
  float* bias_red = nullptr;  // LDS for the bias sums' reduction (the ring loop's first stage)

  // multiply the tile staged in LDS buffer `cur` (and add its A rows for the bias)
  auto compute = [&](int cur) {
    const float* as = As[cur];
    const float* bs = Bs[cur];
    // b_grp < BG for every thread (NT >= BM), so the branch is uniform across the
    // block: a scalar branch, no exec mask, which keeps the accumulators in place
    if (do_bias) {
#pragma unroll
      for (int q = 0; q < BK / BG; ++q) bsum += as[(b_grp * (BK / BG) + q) * TA::LD + b_row];
    }
    float af[BK / 2][TM], bf[BK / 2][TN];
#pragma unroll
    for (int kk = 0; kk < BK / 2; ++kk) {
      const int kr = 2 * kk + half;
#pragma unroll
      for (int i = 0; i < TM; ++i) af[kk][i] = as[kr * TA::LD + (wm * TM + i) * 32 + l32];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[kk][j] = bs[kr * TB::LD + (wn * TN + j) * 32 + l32];
    }
#pragma unroll
    for (int kk = 0; kk < BK / 2; ++kk)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[kk][i], bf[kk][j], acc[i][j], 0, 0, 0);
  };

  if constexpr (PF == 1) {
    TA ta;
    TB tb;
    if (kt_begin < kt_end) {
      load_into(ta, tb, kt_begin);
      ta.store(As[0], tid);
      tb.store(Bs[0], tid);
      __syncthreads();
      for (int kt = kt_begin; kt < kt_end; ++kt) {
        const int cur = (kt - kt_begin) & 1;
        const bool more = kt + 1 < kt_end;
        if (more) load_into(ta, tb, kt + 1);
        compute(cur);
        if (more) {
          ta.store(As[cur ^ 1], tid);
          tb.store(Bs[cur ^ 1], tid);
        }
        __syncthreads();
      }
    }
  } else if constexpr (PF == 2) {
    // Two register sets; the loop is unrolled by two so that every set is
    // named statically.  In the body for tile kt: LDS[cur] holds tile kt, set
    // `nxt` holds tile kt + 1 (stored to LDS[cur ^ 1] at the end), and set
    // `fre` (whose tile kt is already in LDS) receives tile kt + 2.  The loads
    // are unconditional (past the last tile they re-read it, unused) and
    // branch-free, so the compiler can wait for set `nxt` alone while the
    // loads of set `fre` stay in flight.
    // Pairs of steps run with unconditional MFMAs (a conditional around them
    // made the compiler copy the accumulators out of and back into the matrix
    // registers every pair, waiting for the MFMA chain to drain each time); an
    // odd last step follows the loop.
    TA ta0, ta1;
    TB tb0, tb1;
    auto body = [&](int kt, int cur, TA& fre_a, TB& fre_b, TA& nxt_a, TB& nxt_b) {
      load_into(fre_a, fre_b, min(kt + 2, kt_end - 1));
      compute(cur);
      if (kt + 1 < kt_end) {
        nxt_a.store_masked(As[cur ^ 1], tid);
        nxt_b.store_masked(Bs[cur ^ 1], tid);
      }
      __syncthreads();
    };
    if (kt_begin < kt_end) {
      load_into(ta0, tb0, kt_begin);
      load_into(ta1, tb1, min(kt_begin + 1, kt_end - 1));
      ta0.store_masked(As[0], tid);
      tb0.store_masked(Bs[0], tid);
      __syncthreads();
      int kt = kt_begin;
      for (; kt + 1 < kt_end; kt += 2) {
        body(kt, 0, ta0, tb0, ta1, tb1);
        body(kt + 1, 1, ta1, tb1, ta0, tb0);
      }
      if (kt < kt_end) compute(0);  // odd count: the last tile is in LDS buffer 0
    }
  }

  if constexpr (PF == 3) {
    // Interleaved two-deep loop.  Two load register sets and two sets of MFMA
    // operands; at the start of step kt (parity p): operand set p holds tile kt,
    // LDS buffer p ^ 1 holds tile kt + 1, load set `nxt` holds tile kt + 2 (in
    // flight), load set `fre` is free.  The step's MFMAs on set p are issued in
    // slots; after each slot comes a fixed share of the step's other work, in
    // this order over the step: the loads of tile kt + 3 into `fre`, the LDS
    // stores of `nxt` into buffer p (whose operands every wave read in the
    // previous step), the operand reads of tile kt + 1 from buffer p ^ 1.  A
    // scheduling barrier after each slot keeps that order, so the work issues
    // while the MFMAs occupy the matrix pipe.  Past the last tile the loads
    // re-read it and the stores and reads move values that are never used.
    // No bias gradient here (the launcher gives such problems another loop).
    struct Frags {
      float a[TM][BK / 2];
      float b[TN][BK / 2];
    };
    constexpr int NL = TA::NV + TB::NV;           // loads, then as many stores
    constexpr int NRA = TM * TA::NREAD, NRB = TN * TB::NREAD;
    constexpr int NOPS = 2 * NL + NRA + NRB;
    constexpr int NSLOT = (BK / 2) * TM * TN;
    auto read_all = [&](int buf, Frags& f) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
        static_for<TA::NREAD>([&](auto q) { TA::template read_part<decltype(q)::value>(As[buf], (wm * TM + i) * 32 + l32, half, f.a[i]); });
#pragma unroll
      for (int j = 0; j < TN; ++j)
        static_for<TB::NREAD>([&](auto q) { TB::template read_part<decltype(q)::value>(Bs[buf], (wn * TN + j) * 32 + l32, half, f.b[j]); });
    };
    auto mfma_all = [&](const Frags& f) {
      static_for<NSLOT>([&](auto sc) {
        constexpr int sl = decltype(sc)::value;
        constexpr int kk = sl / (TM * TN), i = (sl / TN) % TM, j = sl % TN;
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[i][kk], f.b[j][kk], acc[i][j], 0, 0, 0);
      });
    };
    TA ta0, ta1;
    TB tb0, tb1;
    Frags f0, f1;
    auto step = [&](int kt, int p, const Frags& cur, Frags& nxf, TA& fre_a, TB& fre_b, TA& nxt_a,
                    TB& nxt_b) {
      const int ktl = min(kt + 3, kt_end - 1);
      const bool p1 = ktl >= nt0;
      const int k0 = kb + (ktl - (p1 ? nt0 : 0)) * BK;
      const int kl = kb + (p1 ? kn1 : kn0);
      const float* const Ap = p1 ? A1p : A0p;
      const float* const Bp = p1 ? B1p : B0p;
      const int64_t la = p1 ? lda1 : lda0, lb = p1 ? ldb1 : ldb0;
      float* const as_st = As[p];
      float* const bs_st = Bs[p];
      const float* const as_rd = As[p ^ 1];
      const float* const bs_rd = Bs[p ^ 1];
      static_for<NSLOT>([&](auto sc) {
        constexpr int sl = decltype(sc)::value;
        constexpr int kk = sl / (TM * TN), i = (sl / TN) % TM, j = sl % TN;
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(cur.a[i][kk], cur.b[j][kk], acc[i][j], 0, 0, 0);
        static_for<NOPS>([&](auto oc) {
          constexpr int o = decltype(oc)::value;
          if constexpr (o * NSLOT / NOPS == sl) {
            if constexpr (o < TA::NV) {
              fre_a.template load_one<o>(Ap, la, m0, m_lim, k0, kl, tid);
            } else if constexpr (o < NL) {
              fre_b.template load_one<o - TA::NV>(Bp, lb, n0, n_lim, k0, kl, tid);
            } else if constexpr (o < NL + TA::NV) {
              nxt_a.template store_one<o - NL>(as_st, tid);
            } else if constexpr (o < 2 * NL) {
              nxt_b.template store_one<o - NL - TA::NV>(bs_st, tid);
            } else if constexpr (o < 2 * NL + NRA) {
              constexpr int r = o - 2 * NL;
              TA::template read_part<r % TA::NREAD>(as_rd, (wm * TM + r / TA::NREAD) * 32 + l32, half,
                                                    nxf.a[r / TA::NREAD]);
            } else {
              constexpr int r = o - 2 * NL - NRA;
              TB::template read_part<r % TB::NREAD>(bs_rd, (wn * TN + r / TB::NREAD) * 32 + l32, half,
                                                    nxf.b[r / TB::NREAD]);
            }
          }
        });
        __builtin_amdgcn_sched_barrier(0);
      });
      __syncthreads();
    };
    if (kt_begin < kt_end) {
      load_into(ta0, tb0, kt_begin);
      load_into(ta1, tb1, min(kt_begin + 1, kt_end - 1));
      ta0.store_masked(As[0], tid);
      tb0.store_masked(Bs[0], tid);
      __syncthreads();
      read_all(0, f0);
      ta1.store_masked(As[1], tid);
      tb1.store_masked(Bs[1], tid);
      load_into(ta0, tb0, min(kt_begin + 2, kt_end - 1));
      __syncthreads();
      int kt = kt_begin;
      for (; kt + 1 < kt_end; kt += 2) {
        step(kt, 0, f0, f1, ta1, tb1, ta0, tb0);
        step(kt + 1, 1, f1, f0, ta0, tb0, ta1, tb1);
      }
      if (kt < kt_end) mfma_all(f0);  // odd count: the last tile's operands are in set 0
    }
  }

  if constexpr (PF == 4) {
    // LDS ring of D stages, tile kt in stage (kt - kt_begin) mod D.  At the start
    // of step kt: operand set `cur` holds tile kt (read from its stage in the
    // previous step) and the loads of tiles kt + 1 .. kt + D - 1 are issued.  The
    // step waits for this wave's loads of tile kt + 1 and its own LDS reads, then
    // the block barrier: tile kt + 1 is in LDS and no wave still reads the stage
    // of tile kt, which receives tile kt + D.  The MFMAs of tile kt then run in
    // slots, the loads of tile kt + D and the reads of tile kt + 1's operands
    // placed between them.  Every stage is its own LDS array and the loop is
    // unrolled by D, so the compiler tells the stages apart and never waits for
    // loads of a later tile before an operand read.  The barrier is a plain
    // s_barrier: a workgroup fence would wait for every load in flight.
    // Past the last tile the loads re-read it into stages never read again.
    // Bias gradient: in the blocks that store one (the first column tile of a
    // problem that wants it; a uniform branch), every thread adds its slice of
    // each A tile (row b_row, k rows b_grp * BK/BG ..) from the stage while it
    // reads the tile's operands, a tile past the last one contributing zeros
    // (bit mask).  Other blocks skip the reads, which on a K-contiguous A tile
    // would meet bank conflicts.
    using DA = DmaTile<BM, BK, NT, !A_T>;
    using DB = DmaTile<BN, BK, NT, B_T>;
    constexpr int D = 4;
    __shared__ __attribute__((aligned(16))) float Sa0[DA::SIZE], Sa1[DA::SIZE], Sa2[DA::SIZE], Sa3[DA::SIZE];
    __shared__ __attribute__((aligned(16))) float Sb0[DB::SIZE], Sb1[DB::SIZE], Sb2[DB::SIZE], Sb3[DB::SIZE];
    constexpr int NL = DA::NV + DB::NV;  // loads per thread and tile
    static_assert((D - 1) * NL <= 63, "vmcnt range");
    auto stage_a = [&](auto st) -> float* {
      constexpr int x = decltype(st)::value;
      if constexpr (x == 0) return Sa0;
      else if constexpr (x == 1) return Sa1;
      else if constexpr (x == 2) return Sa2;
      else return Sa3;
    };
    auto stage_b = [&](auto st) -> float* {
      constexpr int x = decltype(st)::value;
      if constexpr (x == 0) return Sb0;
      else if constexpr (x == 1) return Sb1;
      else if constexpr (x == 2) return Sb2;
      else return Sb3;
    };
    struct Frags {
      float a[TM][BK / 2];
      float b[TN][BK / 2];
    };
    constexpr int NRA = TM * DA::NREAD, NRB = TN * DB::NREAD;
    constexpr int NBIAS = BK / BG;  // bias reads per thread and tile
    constexpr int NOPS = NL + NRA + NRB + NBIAS;
    constexpr int NSLOT = (BK / 2) * TM * TN;
    auto bias_add = [&](const float* st, int q, unsigned keep) {
      const float x = DA::at(st, b_row, b_grp * NBIAS + q);
      bsum += __uint_as_float(__float_as_uint(x) & keep);
    };
    DA da;
    DB db;
    da.setup(lda0, lda1, m0, m_lim, tid);
    db.setup(ldb0, ldb1, n0, n_lim, tid);
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // operand o of the loads of tile kt into stage st (o < NL)
    struct TileRef {
      int pc, k0, kl;
    };
    auto tile_ref = [&](int kt) {
      TileRef t;
      t.pc = kt < nt0 ? 0 : 1;
      t.k0 = kb + (kt - (t.pc ? nt0 : 0)) * BK;
      t.kl = kb + (t.pc ? kn1 : kn0);
      return t;
    };
    auto load_one = [&](auto oc, auto st, const TileRef& t) {
      constexpr int o = decltype(oc)::value;
      if constexpr (o < DA::NV) {
        load_lds16(t.pc ? A1p : A0p, stage_a(st) + (o * NT + wv * 64) * 4,
                   da.template voffset<o>(t.pc, t.k0, t.kl, t.pc ? lda1 : lda0));
      } else {
        constexpr int v = o - DA::NV;
        load_lds16(t.pc ? B1p : B0p, stage_b(st) + (v * NT + wv * 64) * 4,
                   db.template voffset<v>(t.pc, t.k0, t.kl, t.pc ? ldb1 : ldb0));
      }
    };
    auto load_all = [&](auto st, int kt) {
      const TileRef t = tile_ref(kt);
      static_for<NL>([&](auto oc) { load_one(oc, st, t); });
    };
    auto read_all = [&](auto st, Frags& f) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
        static_for<DA::NREAD>([&](auto q) {
          DA::template read_part<decltype(q)::value>(stage_a(st), (wm * TM + i) * 32 + l32, half, f.a[i]);
        });
#pragma unroll
      for (int j = 0; j < TN; ++j)
        static_for<DB::NREAD>([&](auto q) {
          DB::template read_part<decltype(q)::value>(stage_b(st), (wn * TN + j) * 32 + l32, half, f.b[j]);
        });
    };
    auto sync = [&](auto vm) {
      __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(decltype(vm)::value));
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
    };
    // step kt in phase ph = (kt - kt_begin) mod D
    auto step = [&](auto phc, int kt, const Frags& cur, Frags& nxf) {
      constexpr int ph = decltype(phc)::value;
      using StNow = std::integral_constant<int, ph>;
      using StNext = std::integral_constant<int, (ph + 1) % D>;
      sync(std::integral_constant<int, (D - 2) * NL>{});
      const TileRef t = tile_ref(min(kt + D, kt_end - 1));
      const unsigned keep_next = 0u - (unsigned)(kt + 1 < kt_end);  // tile kt + 1 exists
      static_for<NSLOT>([&](auto sc) {
        constexpr int sl = decltype(sc)::value;
        constexpr int kk = sl / (TM * TN), i = (sl / TN) % TM, j = sl % TN;
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(cur.a[i][kk], cur.b[j][kk], acc[i][j], 0, 0, 0);
        static_for<NOPS>([&](auto oc) {
          constexpr int o = decltype(oc)::value;
          if constexpr (o * NSLOT / NOPS == sl) {
            if constexpr (o < NL) {
              load_one(oc, StNow{}, t);
            } else if constexpr (o < NL + NRA) {
              constexpr int r = o - NL;
              DA::template read_part<r % DA::NREAD>(stage_a(StNext{}), (wm * TM + r / DA::NREAD) * 32 + l32,
                                                    half, nxf.a[r / DA::NREAD]);
            } else if constexpr (o < NL + NRA + NRB) {
              constexpr int r = o - NL - NRA;
              DB::template read_part<r % DB::NREAD>(stage_b(StNext{}), (wn * TN + r / DB::NREAD) * 32 + l32,
                                                    half, nxf.b[r / DB::NREAD]);
            } else {
              if (do_bias) bias_add(stage_a(StNext{}), o - NL - NRA - NRB, keep_next);
            }
          }
        });
        __builtin_amdgcn_sched_barrier(0);
      });
    };
    if (kt_begin < kt_end) {
      Frags f0, f1;
      static_for<D>([&](auto st) { load_all(st, min(kt_begin + decltype(st)::value, kt_end - 1)); });
      sync(std::integral_constant<int, (D - 1) * NL>{});
      read_all(std::integral_constant<int, 0>{}, f0);
      if (do_bias)
        for (int q = 0; q < NBIAS; ++q) bias_add(Sa0, q, ~0u);
      int kt = kt_begin;
      for (; kt + D <= kt_end; kt += D) {
        static_for<D>([&](auto ph) {
          constexpr int x = decltype(ph)::value;
          if constexpr (x % 2 == 0) step(ph, kt + x, f0, f1);
          else step(ph, kt + x, f1, f0);
        });
      }
      static_for<D - 1>([&](auto ph) {
        constexpr int x = decltype(ph)::value;
        if (kt + x < kt_end) {
          if constexpr (x % 2 == 0) step(ph, kt + x, f0, f1);
          else step(ph, kt + x, f1, f0);
        }
      });
      // the loads past the last tile land before the block may leave its LDS
      __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
    }
    bias_red = Sa0;
  }

  // Accumulator layout of the 32x32 MFMA: register r of lane l holds
  // D[8*(r/4) + 4*(l/32) + r%4][l%32].
  const bool partial = args.splits > 1;
  const int GE = GM == 2 ? args.G : 1;
  float* part = partial
                    ? args.partial + P.part_off + ((int64_t)split * GE + grp) * P.M * P.n_eff
                    : nullptr;
  static_for<TM>([&](auto i) {
    static_for<TN>([&](auto j) {
      const int col = n0 + (wn * TN + j) * 32 + l32;
      if (col >= P.N) return;
      const float bv = (!partial && bias_g) ? bias_g[col] : 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + (wm * TM + i) * 32 + (r >> 2) * 8 + half * 4 + (r & 3);
        if (row >= m_lim) continue;
        const float v = acc[i][j][r];
        if (partial) {
          part[(int64_t)row * P.n_eff + col] = v;
        } else {
          epilogue_store(P, Cg, row, col, v + bv);
        }
      }
    });
  });
  if (do_bias) {  // fixed-order sum of the BG slices of each row
    float* red;
    if constexpr (PF == 4) {
      red = bias_red;
      __syncthreads();  // every wave is past its last read of the ring and its loads have landed
    } else {
      red = As[0];  // free after the loop
    }
    if (b_grp < BG) red[b_grp * BM + b_row] = bsum;
    __syncthreads();
    if (tid < BM && m0 + tid < m_lim) {
      float v = 0.f;
      for (int g2 = 0; g2 < BG; ++g2) v += red[g2 * BM + tid];
      if (partial) part[(int64_t)(m0 + tid) * P.n_eff + P.N] = v;
      else bgrad_g[m0 + tid] = v;
    }
  }
}

// ---- configurations -------------------------------------------------------
struct Cfg {
  int bm, bn, bk, wm, wn;
};
constexpr Cfg kCfgs[] = {
    {64, 64, 32, 2, 2},    // 0: 256 threads, one 32x32 accumulator per wave
    {64, 64, 32, 2, 1},    // 1: 128 threads, 32x64 per wave
    {64, 64, 32, 1, 1},    // 2: 64 threads, 64x64 per wave
    {128, 64, 32, 2, 2},   // 3: 256 threads, 64x32 per wave
    {64, 128, 32, 2, 2},   // 4: 256 threads, 32x64 per wave
    {128, 128, 32, 2, 2},  // 5: 256 threads, 64x64 per wave
    {64, 64, 16, 2, 2},    // 6
    {128, 128, 16, 2, 2},  // 7
    {32, 64, 32, 1, 1},    // 8: 64 threads, 32x64 per wave
    {64, 32, 32, 1, 1},    // 9: 64 threads, 64x32 per wave
    // prefetch distance 2 (tiles loaded two K steps ahead)
    {64, 64, 16, 2, 2},    // 10
    {64, 64, 32, 2, 2},    // 11
    {128, 64, 16, 2, 2},   // 12
    {64, 128, 16, 2, 2},   // 13
    {128, 128, 16, 2, 2},  // 14
    // prefetch distance 2 with more than one accumulator per wave (fewer, busier waves)
    {64, 32, 16, 1, 1},    // 15: 64 threads, 64x32 per wave
    {32, 64, 16, 1, 1},    // 16: 64 threads, 32x64 per wave
    {64, 64, 16, 1, 1},    // 17: 64 threads, 64x64 per wave
    {64, 64, 16, 2, 1},    // 18: 128 threads, 32x64 per wave
    {128, 64, 16, 2, 1},   // 19: 128 threads, 64x64 per wave
    // interleaved two-deep loop (MFMA slots with the step's loads, stores and
    // operand reads between them); not for products with a bias gradient
    {64, 64, 16, 2, 2},    // 20
    {128, 128, 16, 2, 2},  // 21
    {128, 64, 16, 2, 2},   // 22
    {256, 128, 16, 2, 2},  // 23: 128x64 per wave, one wave per SIMD
    {64, 128, 16, 2, 2},   // 24
    {64, 64, 32, 2, 2},    // 25
    {64, 128, 32, 2, 2},   // 26
    // LDS ring (tiles written to LDS by the loads, three steps ahead)
    {64, 64, 16, 2, 2},    // 27
    {64, 128, 16, 2, 2},   // 28
    {128, 64, 16, 2, 2},   // 29
    {64, 64, 32, 2, 2},    // 30
    {128, 128, 16, 2, 2},  // 31
};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);

// index of a row-tile height in LaunchArgs::row_maps
constexpr int bm_index(int bm) { return bm == 32 ? 0 : bm == 64 ? 1 : 2; }

// ---- launching ---------------------------------------------------------------
template <int BM, int BN, int BK, int WM, int WN, bool A_T, bool B_T, int PF, int GM>
void launch_tiles(LaunchArgs& args, hipStream_t stream) {
  int max_tiles = 0;
  for (int i = 0; i < args.n_prob; ++i) {
    ProbDev& d = args.p[i];
    d.tiles_m = GM == 1 ? args.row_counts[bm_index(BM)] : (int)ceil_div(d.M, BM);
    d.tiles_n = (int)ceil_div(d.N > 0 ? d.N : (d.bias_grad ? 1 : 0), BN);
    max_tiles = max(max_tiles, d.tiles_m * d.tiles_n);
  }
  if (GM == 1) args.row_map = args.row_maps[bm_index(BM)];
  dim3 grid;
  if (GM != 2 && args.splits == 1) {
    args.grid_x = (int)ceil_div(max_tiles, 8) * 8;
    grid = dim3(args.grid_x, args.n_prob);
  } else {
    args.grid_x = max_tiles;  // tiles per (problem, graph, split) group
    const int64_t groups = (int64_t)args.n_vprob * args.splits;
    grid = dim3((unsigned)(ceil_div(groups, 8) * 8 * max_tiles));
  }
  hipLaunchKernelGGL((k_gemm<BM, BN, BK, WM, WN, A_T, B_T, PF, GM>), grid, dim3(64 * WM * WN), 0,
                     stream, args);
}

template <int BM, int BN, int BK, int WM, int WN, bool A_T, bool B_T, int PF, int GM>
void launch_cfg(LaunchArgs& args, hipStream_t stream) {
  if constexpr (GM == 1 && BM > 128)  // row-tile maps exist for heights up to 128
    launch_tiles<128, BN, BK, WM, WN, A_T, B_T, PF, GM>(args, stream);
  else
    launch_tiles<BM, BN, BK, WM, WN, A_T, B_T, PF, GM>(args, stream);
}

// Whether the branch-free loads of the two-deep-prefetch configurations may
// run on these operands: every piece float4-aligned, K a multiple of 4 where K
// is the contiguous axis, and M, N multiples of 4 (hence >= 4) where they are.
// Otherwise the launcher runs the configuration's one-deep twin.
inline bool pf2_ok(const LaunchArgs& args, bool a_t, bool b_t) {
  for (int i = 0; i < args.n_prob; ++i) {
    const ProbDev& d = args.p[i];
    if (d.M <= 0) continue;  // no tiles
    if (d.N <= 0) return false;
    if (a_t && d.M % 4 != 0) return false;
    if (!b_t && d.N % 4 != 0) return false;
    for (int pc = 0; pc < d.n_pieces; ++pc) {
      if (!d.vecA[pc] || !d.vecB[pc]) return false;
      if ((!a_t || b_t) && d.K[pc] % 4 != 0) return false;
    }
  }
  return true;
}

// one-deep configuration standing in for a two-deep one (similar tile shape)
constexpr int kPf1Twin[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 6, 0, 3, 4, 7, 9, 8, 2, 1, 3,
                            6, 7, 3, 7, 4, 0, 4, 6, 4, 3, 0, 7};
// two-deep configuration standing in for an interleaved one where a problem
// wants a bias gradient (the LDS-ring ones compute it themselves)
constexpr int kIlTwin[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19,
                           10, 14, 12, 14, 13, 11, 13, 27, 28, 29, 30, 31};
// interleaved configuration standing in for an LDS-ring one whose operands
// reach past the 2^31-byte offsets of its buffer loads
constexpr int kRingTwin[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19,
                             20, 21, 22, 23, 24, 25, 26, 20, 24, 22, 25, 21};
static_assert(sizeof(kIlTwin) / sizeof(kIlTwin[0]) == kNumCfgs, "one twin per configuration");
static_assert(sizeof(kRingTwin) / sizeof(kRingTwin[0]) == kNumCfgs, "one twin per configuration");

inline bool wants_bias_grad(const LaunchArgs& args) {
  for (int i = 0; i < args.n_prob; ++i)
    if (args.p[i].bias_grad) return true;
  return false;
}
static_assert(sizeof(kPf1Twin) / sizeof(kPf1Twin[0]) == kNumCfgs, "one twin per configuration");

// Whether every operand of the launch lies within 2^31 bytes of its base, as
// the 32-bit byte offsets of the LDS-ring loop's buffer loads need.
inline bool ring_ok(const LaunchArgs& args, bool a_t, bool b_t) {
  const double lim = 2147483648.0 - 64.0;
  for (int i = 0; i < args.n_prob; ++i) {
    const ProbDev& d = args.p[i];
    if (d.M <= 0) continue;
    for (int pc = 0; pc < d.n_pieces; ++pc) {
      const double ra = a_t ? d.K[pc] : d.M, ca = a_t ? d.M : d.K[pc];
      const double rb = b_t ? d.N : d.K[pc], cb = b_t ? d.K[pc] : d.N;
      if (4.0 * (ra * (double)d.lda[pc] + ca) >= lim) return false;
      if (4.0 * (rb * (double)d.ldb[pc] + cb) >= lim) return false;
    }
  }
  return true;
}

// The configuration that runs for a requested one: the one-deep twin where the
// branch-free loads may not run, the two-deep twin where the interleaved or
// ring loop would need a bias gradient, the interleaved twin where the ring's
// offsets would not reach.
inline int resolve_cfg(const LaunchArgs& args, bool a_t, bool b_t, int cfg) {
  if (cfg < 0 || cfg >= kNumCfgs) return cfg;
  if (!pf2_ok(args, a_t, b_t)) cfg = kPf1Twin[cfg];
  if (wants_bias_grad(args)) cfg = kIlTwin[cfg];
  if (!ring_ok(args, a_t, b_t)) cfg = kRingTwin[cfg];
  return cfg;
}

template <bool A_T, bool B_T, int GM>
void launch_any(int cfg, LaunchArgs& args, hipStream_t stream) {
  cfg = resolve_cfg(args, A_T, B_T, cfg);
  switch (cfg) {
#define CPRA_GEMM_CFG(I, BM, BN, BK, WM, WN, PF) \
  case I: launch_cfg<BM, BN, BK, WM, WN, A_T, B_T, PF, GM>(args, stream); break;
    CPRA_GEMM_CFG(0, 64, 64, 32, 2, 2, 1)
    CPRA_GEMM_CFG(1, 64, 64, 32, 2, 1, 1)
    CPRA_GEMM_CFG(2, 64, 64, 32, 1, 1, 1)
    CPRA_GEMM_CFG(3, 128, 64, 32, 2, 2, 1)
    CPRA_GEMM_CFG(4, 64, 128, 32, 2, 2, 1)
    CPRA_GEMM_CFG(5, 128, 128, 32, 2, 2, 1)
    CPRA_GEMM_CFG(6, 64, 64, 16, 2, 2, 1)
    CPRA_GEMM_CFG(7, 128, 128, 16, 2, 2, 1)
    CPRA_GEMM_CFG(8, 32, 64, 32, 1, 1, 1)
    CPRA_GEMM_CFG(9, 64, 32, 32, 1, 1, 1)
    CPRA_GEMM_CFG(10, 64, 64, 16, 2, 2, 2)
    CPRA_GEMM_CFG(11, 64, 64, 32, 2, 2, 2)
    CPRA_GEMM_CFG(12, 128, 64, 16, 2, 2, 2)
    CPRA_GEMM_CFG(13, 64, 128, 16, 2, 2, 2)
    CPRA_GEMM_CFG(14, 128, 128, 16, 2, 2, 2)
    CPRA_GEMM_CFG(15, 64, 32, 16, 1, 1, 2)
    CPRA_GEMM_CFG(16, 32, 64, 16, 1, 1, 2)
    CPRA_GEMM_CFG(17, 64, 64, 16, 1, 1, 2)
    CPRA_GEMM_CFG(18, 64, 64, 16, 2, 1, 2)
    CPRA_GEMM_CFG(19, 128, 64, 16, 2, 1, 2)
    CPRA_GEMM_CFG(20, 64, 64, 16, 2, 2, 3)
    CPRA_GEMM_CFG(21, 128, 128, 16, 2, 2, 3)
    CPRA_GEMM_CFG(22, 128, 64, 16, 2, 2, 3)
    CPRA_GEMM_CFG(23, 256, 128, 16, 2, 2, 3)
    CPRA_GEMM_CFG(24, 64, 128, 16, 2, 2, 3)
    CPRA_GEMM_CFG(25, 64, 64, 32, 2, 2, 3)
    CPRA_GEMM_CFG(26, 64, 128, 32, 2, 2, 3)
    CPRA_GEMM_CFG(27, 64, 64, 16, 2, 2, 4)
    CPRA_GEMM_CFG(28, 64, 128, 16, 2, 2, 4)
    CPRA_GEMM_CFG(29, 128, 64, 16, 2, 2, 4)
    CPRA_GEMM_CFG(30, 64, 64, 32, 2, 2, 4)
    CPRA_GEMM_CFG(31, 128, 128, 16, 2, 2, 4)
#undef CPRA_GEMM_CFG
    default: break;
  }
}

// Launchers of the group modes (defined in gemm_grouped.hip): mode 1 for the
// NN and NT layouts, mode 2 for TN.
void launch_grouped(int mode, bool a_t, bool b_t, int cfg, LaunchArgs& args, hipStream_t stream);

}  // namespace gemmk
}  // namespace cpra
