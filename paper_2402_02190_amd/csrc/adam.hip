// Adam / AdamW update over a flat parameter vector (Sec. 4.1 Implementation;
// Kingma & Ba, with decoupled weight decay for AdamW).  FP32 state and math;
// the bias corrections 1 - beta^t are formed in FP64 once per launch.
#include <cmath>

#include "common.hpp"

namespace cpra {

namespace {

// Hyperparameters arrive in double; 1 - beta and the decay factor are formed
// in double before rounding, so that beta = 0.999 gives 1 - beta = 0.001 to
// FP32 precision rather than 1 - float(0.999).
struct AdamArgs {
  int64_t n;
  float* p;
  const float* g;
  float* m;
  float* v;
  float lr, b1, omb1, b2, omb2, eps, decay;
  double b1d, b2d;
  int t;
  const int32_t* step_counter;
  int t_offset;  // t = *step_counter + t_offset when step_counter is given
  const int32_t* stop_flag;  // optional: no update while *stop_flag != 0 (early stopping)
};

struct AdamCoef {
  float lr, b1, omb1, b2, omb2, eps, decay;
};

__device__ inline void adam_one(float& p, float g, float& m, float& v, const AdamCoef& c,
                                float inv_bc1, float inv_sqrt_bc2) {
  m = c.b1 * m + c.omb1 * g;
  v = c.b2 * v + c.omb2 * g * g;
  const float mhat = m * inv_bc1;
  const float denom = sqrtf(v) * inv_sqrt_bc2 + c.eps;  // sqrt(v / bc2) + eps
  p = p * c.decay - c.lr * mhat / denom;
}

typedef float f4v __attribute__((ext_vector_type(4)));

// float4 load / store, streaming (nontemporal) when NT: the gradient and the
// moments are read and written once per step and need not stay in the caches;
// the parameters take ordinary accesses, since the next forward reads them
// again (its first aggregation gathers the embedding).
template <bool NT>
__device__ inline float4 ld4(const float4* p) {
  if constexpr (NT) {
    const f4v x = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    return make_float4(x.x, x.y, x.z, x.w);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ inline void st4(float4* p, const float4& v) {
  if constexpr (NT) {
    f4v x;
    x.x = v.x;
    x.y = v.y;
    x.z = v.z;
    x.w = v.w;
    __builtin_nontemporal_store(x, reinterpret_cast<f4v*>(p));
  } else {
    *p = v;
  }
}

template <bool VEC4, bool NT = false>
__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  if (a.stop_flag && *a.stop_flag) return;  // uniform across the grid
  __shared__ float s_bc[2];
  if (threadIdx.x == 0) {
    int t = a.step_counter ? (*a.step_counter + a.t_offset) : a.t;
    double bc1 = 1.0 - pow(a.b1d, (double)t);
    double bc2 = 1.0 - pow(a.b2d, (double)t);
    s_bc[0] = (float)(1.0 / bc1);
    s_bc[1] = (float)(1.0 / sqrt(bc2));
  }
  __syncthreads();
  const float inv_bc1 = s_bc[0], inv_sqrt_bc2 = s_bc[1];
  const AdamCoef c{a.lr, a.b1, a.omb1, a.b2, a.omb2, a.eps, a.decay};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if constexpr (VEC4) {
    const int64_t n4 = a.n / 4;
    float4* p4 = reinterpret_cast<float4*>(a.p);
    const float4* g4 = reinterpret_cast<const float4*>(a.g);
    float4* m4 = reinterpret_cast<float4*>(a.m);
    float4* v4 = reinterpret_cast<float4*>(a.v);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
      float4 p = p4[i], m = ld4<NT>(m4 + i), v = ld4<NT>(v4 + i);
      const float4 g = ld4<NT>(g4 + i);
      adam_one(p.x, g.x, m.x, v.x, c, inv_bc1, inv_sqrt_bc2);
      adam_one(p.y, g.y, m.y, v.y, c, inv_bc1, inv_sqrt_bc2);
      adam_one(p.z, g.z, m.z, v.z, c, inv_bc1, inv_sqrt_bc2);
      adam_one(p.w, g.w, m.w, v.w, c, inv_bc1, inv_sqrt_bc2);
      p4[i] = p;  // the next forward gathers the parameters (the embedding) again
      st4<NT>(m4 + i, m);
      st4<NT>(v4 + i, v);
    }
    for (int64_t i = n4 * 4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride)
      adam_one(a.p[i], a.g[i], a.m[i], a.v[i], c, inv_bc1, inv_sqrt_bc2);
  } else {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride)
      adam_one(a.p[i], a.g[i], a.m[i], a.v[i], c, inv_bc1, inv_sqrt_bc2);
  }
}

inline bool al16(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

}  // namespace

cpra_status adam_step(int64_t n, float* params, const float* grads, float* m, float* v,
                      const cpra_adam_cfg* cfg, int32_t t, const int32_t* step_counter,
                      hipStream_t stream, int t_offset, const int32_t* stop_flag) {
  if (n == 0) return CPRA_OK;
  AdamArgs a{n, params, grads, m, v,
             (float)cfg->lr, (float)cfg->beta1, (float)(1.0 - cfg->beta1),
             (float)cfg->beta2, (float)(1.0 - cfg->beta2), (float)cfg->eps,
             (float)(1.0 - cfg->lr * cfg->weight_decay), cfg->beta1, cfg->beta2,
             t, step_counter, t_offset, stop_flag};
  const bool vec = al16(params) && al16(grads) && al16(m) && al16(v);
  const int64_t work = vec ? (n + 3) / 4 : n;
  const int blocks = (int)std::min<int64_t>(ceil_div(work, 256), 256 * 8);
  ProfScope ps("adam", stream, 0.0, 28.0 * (double)n);
  // streaming accesses once the four arrays pass 64 MB (measured: 44 MB slower,
  // 88 MB and above faster)
  const bool nt = 16.0 * (double)n > 64.0 * 1024 * 1024;
  if (vec && nt)
    hipLaunchKernelGGL((k_adam<true, true>), dim3(blocks), dim3(256), 0, stream, a);
  else if (vec)
    hipLaunchKernelGGL(k_adam<true>, dim3(blocks), dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(k_adam<false>, dim3(blocks), dim3(256), 0, stream, a);
  CPRA_CHECK_LAUNCH("adam");
  return CPRA_OK;
}

cpra_status check_adam_cfg(const cpra_adam_cfg* cfg) {
  if (cfg == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "adam: cfg is NULL");
  const double vals[5] = {cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, cfg->weight_decay};
  for (double x : vals)
    if (!std::isfinite(x)) CPRA_FAIL(CPRA_ERR_NONFINITE, "adam: non-finite hyperparameter");
  if (cfg->lr < 0 || cfg->beta1 < 0 || cfg->beta1 >= 1 || cfg->beta2 < 0 || cfg->beta2 >= 1 ||
      cfg->eps <= 0 || cfg->weight_decay < 0)
    CPRA_FAIL(CPRA_ERR_PARAM, "adam: hyperparameter out of range");
  return CPRA_OK;
}

}  // namespace cpra

extern "C" cpra_status cpra_adam_step(int64_t n, float* params, const float* grads, float* m,
                                      float* v, const cpra_adam_cfg* cfg, int32_t t,
                                      const int32_t* step_counter, cpra_stream_t stream) {
  CPRA_CHECK(cpra::check_adam_cfg(cfg));
  if (n < 0) CPRA_FAIL(CPRA_ERR_SHAPE, "adam: n < 0");
  if (n > 0 && (!params || !grads || !m || !v)) CPRA_FAIL(CPRA_ERR_NULL, "adam: NULL buffer");
  if (step_counter == nullptr && t < 1) CPRA_FAIL(CPRA_ERR_PARAM, "adam: t must be >= 1");
  return cpra::adam_step(n, params, grads, m, v, cfg, t, step_counter, cpra::as_stream(stream));
}
