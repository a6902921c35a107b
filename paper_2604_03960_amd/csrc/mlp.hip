// Learned bond-dimension scheduler: a 25 -> 64 -> 64 -> 1 perceptron (tanh
// hidden units, linear output) trained by mean-squared error with Adam, all in
// hand-written FP32 kernels.  It predicts log2 of the bond dimension a bond
// needs at its next visit (the learned stand-in for the predictive scheduler
// of Sec. 7).  Parameter layout (5889 floats): W1[64][25] b1[64] W2[64][64]
// b2[64] W3[64] b3.
//
// Training step = fwdbwd_kernel (one 256-thread block per 64 samples: the
// forward pass, the backward pass and the block's gradient sum, all in LDS) ->
// grad_reduce_kernel (fixed-order sum of the block partials) -> adam_kernel.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace tna {
namespace {

constexpr int IN = 25, H = 64, NP = H * IN + H + H * H + H + H + 1;
constexpr int OW1 = 0, OB1 = H * IN, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
constexpr int SB = 64;  // samples per block

struct MlpIn {
  const float *mean, *inv_std;  // input standardisation (IN each), may be null
};

__device__ inline void load_params(const float *p, float *Ps) {
  for (int i = threadIdx.x; i < NP; i += 256) Ps[i] = p[i];
}

__device__ inline void load_x(const float *X, const int *idx, int B, int s0, MlpIn st, float (*Xs)[IN + 1]) {
  for (int e = threadIdx.x; e < SB * IN; e += 256) {
    const int s = e / IN, k = e % IN;
    float v = 0.f;
    if (s0 + s < B) {
      const int row = idx ? idx[s0 + s] : s0 + s;
      v = X[(int64_t)row * IN + k];
      if (st.mean) v = (v - st.mean[k]) * st.inv_std[k];
    }
    Xs[s][k] = v;
  }
}

// forward of SB samples: H1, H2 (pre-computed tanh), y
__device__ inline void forward_block(const float *Ps, float (*Xs)[IN + 1], float (*H1)[H + 1], float (*H2)[H + 1],
                                     float *ys) {
  for (int e = threadIdx.x; e < SB * H; e += 256) {
    const int s = e / H, i = e % H;
    float a = Ps[OB1 + i];
#pragma unroll 5
    for (int k = 0; k < IN; ++k) a += Ps[OW1 + i * IN + k] * Xs[s][k];
    H1[s][i] = tanhf(a);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < SB * H; e += 256) {
    const int s = e / H, i = e % H;
    float a = Ps[OB2 + i];
#pragma unroll 8
    for (int k = 0; k < H; ++k) a += Ps[OW2 + i * H + k] * H1[s][k];
    H2[s][i] = tanhf(a);
  }
  __syncthreads();
  if (threadIdx.x < SB) {
    const int s = threadIdx.x;
    float a = Ps[OB3];
    for (int k = 0; k < H; ++k) a += Ps[OW3 + k] * H2[s][k];
    ys[s] = a;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void forward_kernel(const float *p, const float *X, int B, MlpIn st, float *y) {
  __shared__ float Ps[NP];
  __shared__ float Xs[SB][IN + 1];
  __shared__ float H1[SB][H + 1], H2[SB][H + 1];
  __shared__ float ys[SB];
  const int s0 = blockIdx.x * SB;
  load_params(p, Ps);
  load_x(X, nullptr, B, s0, st, Xs);
  __syncthreads();
  forward_block(Ps, Xs, H1, H2, ys);
  if (threadIdx.x < SB && s0 + threadIdx.x < B) y[s0 + threadIdx.x] = ys[threadIdx.x];
}

// part[blk][NP] = gradient of (1/Btot) sum (y - t)^2 over this block's samples;
// lpart[blk] = sum of squared residuals of the block
__global__ __launch_bounds__(256) void fwdbwd_kernel(const float *p, const float *X, const float *T, const int *idx,
                                                     int B, int Btot, MlpIn st, float *part, float *lpart) {
  __shared__ float Ps[NP];
  __shared__ float Xs[SB][IN + 1];
  __shared__ float H1[SB][H + 1], H2[SB][H + 1], D1[SB][H + 1], D2[SB][H + 1];
  __shared__ float ys[SB], dy[SB];
  const int s0 = blockIdx.x * SB;
  load_params(p, Ps);
  load_x(X, idx, B, s0, st, Xs);
  __syncthreads();
  forward_block(Ps, Xs, H1, H2, ys);
  if (threadIdx.x < SB) {
    const int s = threadIdx.x;
    float r = 0.f;
    if (s0 + s < B) {
      const int row = idx ? idx[s0 + s] : s0 + s;
      r = ys[s] - T[row];
    }
    dy[s] = 2.f * r / (float)Btot;
    ys[s] = r * r;  // residual^2 for the loss
  }
  __syncthreads();
  // delta at the second hidden layer
  for (int e = threadIdx.x; e < SB * H; e += 256) {
    const int s = e / H, i = e % H;
    const float h = H2[s][i];
    D2[s][i] = dy[s] * Ps[OW3 + i] * (1.f - h * h);
  }
  __syncthreads();
  // delta at the first hidden layer
  for (int e = threadIdx.x; e < SB * H; e += 256) {
    const int s = e / H, k = e % H;
    float a = 0.f;
    for (int i = 0; i < H; ++i) a += Ps[OW2 + i * H + k] * D2[s][i];
    const float h = H1[s][k];
    D1[s][k] = a * (1.f - h * h);
  }
  __syncthreads();
  float *g = part + (int64_t)blockIdx.x * NP;
  // W2, b2
  for (int e = threadIdx.x; e < H * H; e += 256) {
    const int i = e / H, k = e % H;
    float a = 0.f;
    for (int s = 0; s < SB; ++s) a += D2[s][i] * H1[s][k];
    g[OW2 + e] = a;
  }
  // W1, b1
  for (int e = threadIdx.x; e < H * IN; e += 256) {
    const int i = e / IN, k = e % IN;
    float a = 0.f;
    for (int s = 0; s < SB; ++s) a += D1[s][i] * Xs[s][k];
    g[OW1 + e] = a;
  }
  if (threadIdx.x < H) {
    const int i = threadIdx.x;
    float a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int s = 0; s < SB; ++s) {
      a1 += D1[s][i];
      a2 += D2[s][i];
      a3 += dy[s] * H2[s][i];
    }
    g[OB1 + i] = a1;
    g[OB2 + i] = a2;
    g[OW3 + i] = a3;
  }
  if (threadIdx.x == 64) {
    float a = 0.f, l = 0.f;
    for (int s = 0; s < SB; ++s) {
      a += dy[s];
      l += ys[s];
    }
    g[OB3] = a;
    lpart[blockIdx.x] = l;
  }
}

// grad[i] = sum_b part[b][i] (fixed order); loss = sum_b lpart[b] / Btot
__global__ __launch_bounds__(256) void grad_reduce_kernel(const float *part, const float *lpart, int nblk, int Btot,
                                                          float *grad, float *loss) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < NP) {
    float a = 0.f;
    for (int b = 0; b < nblk; ++b) a += part[(int64_t)b * NP + i];
    grad[i] = a;
  }
  if (i == 0 && loss) {
    float l = 0.f;
    for (int b = 0; b < nblk; ++b) l += lpart[b];
    *loss = l / (float)Btot;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float *p, const float *g, float *m, float *v, float c1, float c2,
                                                   float lr, float b1, float b2, float eps) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= NP) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace
}  // namespace tna

using namespace tna;

struct tna_mlp_s {
  tna_ctx ctx;
  DevBuf p, m, v, g, part, lpart, mean, istd, scratch;
  int step = 0;
  int has_norm = 0;
};

static MlpIn norm_of(tna_mlp n) {
  MlpIn st{nullptr, nullptr};
  if (n->has_norm) {
    st.mean = n->mean.as<float>();
    st.inv_std = n->istd.as<float>();
  }
  return st;
}

static tna_status mlp_lossgrad(tna_mlp n, int B, const float *X, const float *T, const int *idx, float *grad,
                               float *loss) {
  hipStream_t s = n->ctx->stream;
  const int nblk = (B + SB - 1) / SB;
  TNA_TRY(n->part.ensure(sizeof(float) * (size_t)nblk * NP));
  TNA_TRY(n->lpart.ensure(sizeof(float) * (size_t)nblk));
  hipLaunchKernelGGL(fwdbwd_kernel, dim3(nblk), dim3(256), 0, s, n->p.as<float>(), X, T, idx, B, B, norm_of(n),
                     n->part.as<float>(), n->lpart.as<float>());
  hipLaunchKernelGGL(grad_reduce_kernel, dim3((NP + 255) / 256), dim3(256), 0, s, n->part.as<float>(),
                     n->lpart.as<float>(), nblk, B, grad, loss);
  TNA_LAUNCHED("mlp.lossgrad");
  return TNA_OK;
}

static tna_status mlp_adam(tna_mlp n, const float *grad, float lr) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  n->step += 1;
  const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
  hipLaunchKernelGGL(adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, n->ctx->stream, n->p.as<float>(), grad,
                     n->m.as<float>(), n->v.as<float>(), c1, c2, lr, b1, b2, eps);
  TNA_LAUNCHED("mlp.adam");
  return TNA_OK;
}

namespace tna {
// forward of B samples already on the device (used by the DMRG scheduler)
tna_status mlp_forward_dev(tna_mlp n, int B, const float *X, float *y, hipStream_t s) {
  hipLaunchKernelGGL(forward_kernel, dim3((B + SB - 1) / SB), dim3(256), 0, s, n->p.as<float>(), X, B, norm_of(n), y);
  TNA_LAUNCHED("mlp.forward");
  return TNA_OK;
}
}  // namespace tna

extern "C" {

tna_status tna_mlp_create(tna_ctx c, const float *params_host, tna_mlp *out) {
  if (!c || !params_host || !out) {
    set_error("mlp_create: null argument");
    return TNA_ERR_ARG;
  }
  auto n = new tna_mlp_s();
  n->ctx = c;
  tna_status st = TNA_OK;
  for (DevBuf *b : {&n->p, &n->m, &n->v, &n->g})
    if ((st = b->ensure(sizeof(float) * NP)) != TNA_OK) {
      delete n;
      return st;
    }
  if (hipMemcpy(n->p.ptr, params_host, sizeof(float) * NP, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(n->m.ptr, 0, sizeof(float) * NP) != hipSuccess || hipMemset(n->v.ptr, 0, sizeof(float) * NP) != hipSuccess) {
    set_error("mlp_create: copy failed");
    delete n;
    return TNA_ERR_DEVICE;
  }
  c->children += 1;
  *out = n;
  return TNA_OK;
}

tna_status tna_mlp_set_normalization(tna_mlp n, const float *mean_host, const float *std_host) {
  if (!n) {
    set_error("mlp: null handle");
    return TNA_ERR_ARG;
  }
  if (!mean_host || !std_host) {
    n->has_norm = 0;
    return TNA_OK;
  }
  float inv[IN];
  for (int k = 0; k < IN; ++k) {
    if (!(std_host[k] > 0.f)) {
      set_error("mlp: std must be positive");
      return TNA_ERR_ARG;
    }
    inv[k] = 1.f / std_host[k];
  }
  TNA_TRY(n->mean.ensure(sizeof(float) * IN));
  TNA_TRY(n->istd.ensure(sizeof(float) * IN));
  TNA_HIP(hipMemcpy(n->mean.ptr, mean_host, sizeof(float) * IN, hipMemcpyHostToDevice));
  TNA_HIP(hipMemcpy(n->istd.ptr, inv, sizeof(float) * IN, hipMemcpyHostToDevice));
  n->has_norm = 1;
  return TNA_OK;
}

tna_status tna_mlp_get_params(tna_mlp n, float *params_host) {
  if (!n || !params_host) {
    set_error("mlp: null argument");
    return TNA_ERR_ARG;
  }
  TNA_HIP(hipStreamSynchronize(n->ctx->stream));
  TNA_HIP(hipMemcpy(params_host, n->p.ptr, sizeof(float) * NP, hipMemcpyDeviceToHost));
  return TNA_OK;
}

tna_status tna_mlp_forward(tna_mlp n, int B, const float *X, float *y) {
  if (!n || !X || !y || B < 1) {
    set_error("mlp_forward: bad argument");
    return TNA_ERR_ARG;
  }
  return mlp_forward_dev(n, B, X, y, n->ctx->stream);
}

tna_status tna_mlp_loss_grad(tna_mlp n, int B, const float *X, const float *T, float *grad, float *loss) {
  if (!n || !X || !T || !grad || B < 1) {
    set_error("mlp_loss_grad: bad argument");
    return TNA_ERR_ARG;
  }
  return mlp_lossgrad(n, B, X, T, nullptr, grad, loss);
}

tna_status tna_mlp_adam_step(tna_mlp n, const float *grad, float lr) {
  if (!n || !grad || !(lr > 0.f)) {
    set_error("mlp_adam_step: bad argument");
    return TNA_ERR_ARG;
  }
  return mlp_adam(n, grad, lr);
}

tna_status tna_mlp_train(tna_mlp n, int nsamp, const float *X, const float *T, const int *perm, int epochs,
                         int batch, float lr, float *loss_per_epoch) {
  if (!n || !X || !T || !perm || nsamp < 1 || epochs < 1 || batch < 1 || !(lr > 0.f)) {
    set_error("mlp_train: bad argument");
    return TNA_ERR_ARG;
  }
  TNA_TRY(n->scratch.ensure(sizeof(float) * 8));
  float *dloss = n->scratch.as<float>();
  for (int e = 0; e < epochs; ++e) {
    const int *pe = perm + (int64_t)e * nsamp;
    for (int b0 = 0; b0 < nsamp; b0 += batch) {
      const int B = std::min(batch, nsamp - b0);
      TNA_TRY(mlp_lossgrad(n, B, X, T, pe + b0, n->g.as<float>(), dloss));
      TNA_TRY(mlp_adam(n, n->g.as<float>(), lr));
    }
    if (loss_per_epoch) {
      // full-data loss after the epoch
      TNA_TRY(mlp_lossgrad(n, nsamp, X, T, nullptr, n->g.as<float>(), dloss));
      TNA_HIP(hipMemcpyAsync(loss_per_epoch + e, dloss, sizeof(float), hipMemcpyDeviceToHost, n->ctx->stream));
    }
  }
  TNA_HIP(hipStreamSynchronize(n->ctx->stream));
  return TNA_OK;
}

void tna_mlp_destroy(tna_mlp n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->ctx->stream);
  for (DevBuf *b : {&n->p, &n->m, &n->v, &n->g, &n->part, &n->lpart, &n->mean, &n->istd, &n->scratch}) b->release();
  n->ctx->children -= 1;
  delete n;
}

}  // extern "C"
