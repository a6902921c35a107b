// Bandwidth-bound kernels of the path: the MPO mixing stage of H_eff and of
// the environment updates, and the Lanczos vector operations (dot products,
// classical Gram-Schmidt updates, norms) with fixed-order reductions so that
// every result is bitwise reproducible from run to run.
#include "internal.h"

namespace tna {
namespace {

constexpr int NT = 256;
constexpr int MAXPART = 512;  // partial sums per reduction

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum over the 256 threads of a block, fixed order; result valid in thread 0
__device__ inline double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

int n_parts(int64_t n) {
  int64_t g = (n + 4095) / 4096;
  if (g < 1) g = 1;
  if (g > MAXPART) g = MAXPART;
  return (int)g;
}

// ------------------------------------------------------------------ mixing
struct MixDev {
  int n0, n1, I, J;
  int64_t is0, is1, os0, os1;
  int ioff[32];
  int ooff[32];
  const void *in;
  void *out;
  const double *M;
};

template <typename TI, typename TO>
__global__ __launch_bounds__(NT) void mix_kernel(MixDev a) {
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t total = (int64_t)a.n0 * a.n1;
  if (idx >= total) return;
  const int64_t o0 = idx / a.n1, o1 = idx - o0 * a.n1;
  const TI *in = static_cast<const TI *>(a.in) + o0 * a.is0 + o1 * a.is1;
  TO *out = static_cast<TO *>(a.out) + o0 * a.os0 + o1 * a.os1;
  typedef typename std::conditional<sizeof(TI) == 8 || sizeof(TO) == 8, double, float>::type T;
  T x[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) x[i] = (i < a.I) ? (T)in[a.ioff[i]] : T(0);
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    if (j < a.J) {
      T acc = T(0);
      const double *Mj = a.M + j * a.I;
#pragma unroll
      for (int i = 0; i < 32; ++i)
        if (i < a.I) acc += (T)Mj[i] * x[i];
      out[a.ooff[j]] = (TO)acc;
    }
  }
}

__global__ void build_mix_kernel(int mode, int d, int D, const double *W1, const double *W2, double *M) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (mode == 0) {
    const int I = D * d * d, J = d * d * D;
    if (t >= I * J) return;
    const int j = t / I, i = t % I;
    const int s = j / (d * D), tt = (j / D) % d, wq = j % D;
    const int w = i / (d * d), sp = (i / d) % d, tp = i % d;
    double acc = 0.0;
    for (int wp = 0; wp < D; ++wp)
      acc += W1[((w * D + wp) * d + s) * d + sp] * W2[((wp * D + wq) * d + tt) * d + tp];
    M[t] = acc;
  } else {
    const int I = D * d, J = d * D;
    if (t >= I * J) return;
    const int j = t / I, i = t % I;
    const int s = j / D, wo = j % D;  // output (s, w') or (t, w)
    const int wi = i / d, sp = i % d;  // input (w, s') or (w'', t')
    // mode 1: W[w_in][w_out][s][s']   mode 2: W[w_out][w_in][t][t']
    M[t] = (mode == 1) ? W1[((wi * D + wo) * d + s) * d + sp] : W1[((wo * D + wi) * d + s) * d + sp];
  }
}

// ------------------------------------------------------------------ reductions
__global__ __launch_bounds__(NT) void multidot_kernel(const double *V, int64_t ldv, int nv, const double *w,
                                                      int64_t n, double *part) {
  __shared__ double sh[4];
  const int G = gridDim.x;
  const int64_t chunk = (n + G - 1) / G;
  const int64_t beg = chunk * blockIdx.x;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  for (int i0 = 0; i0 < nv; i0 += 8) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t e = beg + threadIdx.x; e < end; e += NT) {
      const double wv = w[e];
#pragma unroll
      for (int g = 0; g < 8; ++g)
        if (i0 + g < nv) acc[g] += V[(int64_t)(i0 + g) * ldv + e] * wv;
    }
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      if (i0 + g < nv) {  // uniform
        double r = block_sum(acc[g], sh);
        if (threadIdx.x == 0) part[(int64_t)(i0 + g) * G + blockIdx.x] = r;
      }
    }
  }
}

// h[i] = <V_i, w> with one block per vector (short vectors), fixed order
__global__ __launch_bounds__(NT) void multidot_small_kernel(const double *V, int64_t ldv, const double *w, int64_t n,
                                                            double *h) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  const double *v = V + (int64_t)i * ldv;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += NT) acc += v[e] * w[e];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) h[i] = acc;
}

// out[i] = sum_b part[i*G + b], one block per i, fixed tree
__global__ __launch_bounds__(NT) void reduce_parts_kernel(const double *part, int G, double *out) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < G; b += NT) v += part[(int64_t)i * G + b];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) out[i] = v;
}

__global__ __launch_bounds__(NT) void axpy_multi_kernel(const double *V, int64_t ldv, int nv, const double *h,
                                                        double *w, int64_t n, double *part) {
  __shared__ double sh[4];
  const int G = gridDim.x;
  const int64_t chunk = (n + G - 1) / G;
  const int64_t beg = chunk * blockIdx.x;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double loc = 0.0;
  for (int64_t e = beg + threadIdx.x; e < end; e += NT) {
    double acc = 0.0;
    for (int i = 0; i < nv; ++i) acc += h[i] * V[(int64_t)i * ldv + e];
    const double v = w[e] - acc;
    w[e] = v;
    loc += v * v;
  }
  if (part) {
    double r = block_sum(loc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
  }
}

__global__ __launch_bounds__(NT) void combine_kernel(const double *V, int64_t ldv, int nv, const double *c,
                                                     double *y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    double acc = 0.0;
    for (int i = 0; i < nv; ++i) acc += c[i] * V[(int64_t)i * ldv + e];
    y[e] = acc;
  }
}

__global__ __launch_bounds__(NT) void norm2_kernel(const double *x, int64_t n, double *part) {
  __shared__ double sh[4];
  const int G = gridDim.x;
  const int64_t chunk = (n + G - 1) / G;
  const int64_t beg = chunk * blockIdx.x;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double loc = 0.0;
  for (int64_t e = beg + threadIdx.x; e < end; e += NT) loc += x[e] * x[e];
  double r = block_sum(loc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(NT) void scale_kernel(const double *x, double *y, int64_t n, const double *nrm2,
                                                   double scal) {
  const double f = nrm2 ? 1.0 / sqrt(*nrm2) : scal;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) y[e] = x[e] * f;
}

__global__ __launch_bounds__(NT) void finite_kernel(const double *x, int64_t n, int *flag) {
  int bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT)
    bad |= !isfinite(x[e]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicAdd(flag, 1);
}

__global__ __launch_bounds__(NT) void cvt_kernel(const double *x, float *y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) y[e] = (float)x[e];
}

__global__ __launch_bounds__(NT) void fill_kernel(double *x, int64_t n, double v) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) x[e] = v;
}

__global__ __launch_bounds__(NT) void fill_int_kernel(int *x, int64_t n, int v) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) x[e] = v;
}

template <typename T>
__global__ __launch_bounds__(NT) void transpose_kernel(const T *A, int m, int n, double *B) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // bx over n, by over m
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int i = by + r, j = bx + tx;
    tile[r][tx] = (i < m && j < n) ? (double)A[(int64_t)i * n + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int j = bx + r, i = by + tx;
    if (j < n && i < m) B[(int64_t)j * m + i] = tile[tx][r];
  }
}

__global__ __launch_bounds__(NT) void identity_kernel(double *J, int n, int ld, int64_t stride) {
  double *Jb = J + stride * blockIdx.y;
  const int64_t total = (int64_t)n * ld;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    int64_t r = e / ld, c = e - r * ld;
    Jb[e] = (r == c) ? 1.0 : 0.0;
  }
}

int grid_for(int64_t n) {
  int64_t g = (n + NT - 1) / NT;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

}  // namespace

// ---------------------------------------------------------------------- API
tna_status mix(const MixArgs &a, hipStream_t s) {
  if (a.I < 1 || a.I > 32 || a.J < 1 || a.J > 32 || a.n0 < 0 || a.n1 < 0) {
    set_error("mix: bad channel count");
    return TNA_ERR_ARG;
  }
  int64_t total = (int64_t)a.n0 * a.n1;
  if (total == 0) return TNA_OK;
  MixDev d;
  d.n0 = a.n0; d.n1 = a.n1; d.I = a.I; d.J = a.J;
  d.is0 = a.is0; d.is1 = a.is1; d.os0 = a.os0; d.os1 = a.os1;
  for (int i = 0; i < 32; ++i) { d.ioff[i] = a.ioff[i]; d.ooff[i] = a.ooff[i]; }
  d.in = a.in; d.out = a.out; d.M = a.M;
  dim3 grid((unsigned)((total + NT - 1) / NT));
  const char *name = a.type_in == G_F64 ? "mix.f64" : "mix.f32";
  timer_begin(name, s);
  if (a.type_in == G_F64 && a.type_out == G_F64)
    hipLaunchKernelGGL((mix_kernel<double, double>), grid, dim3(NT), 0, s, d);
  else if (a.type_in == G_F32 && a.type_out == G_F32)
    hipLaunchKernelGGL((mix_kernel<float, float>), grid, dim3(NT), 0, s, d);
  else {
    set_error("mix: type combination not built");
    return TNA_ERR_UNSUPPORTED;
  }
  const int es = a.type_in == G_F64 ? 8 : 4;
  timer_end(name, 2.0 * a.I * a.J * (double)total, (double)total * (a.I + a.J) * es, s);
  TNA_LAUNCHED("vec.hip:1");
  return TNA_OK;
}

tna_status build_mix_matrix(int mode, int d, int D, const double *W1, const double *W2, double *M, hipStream_t s) {
  int n = (mode == 0) ? (D * d * d) * (D * d * d) : (D * d) * (D * d);
  hipLaunchKernelGGL(build_mix_kernel, dim3((n + 255) / 256), dim3(256), 0, s, mode, d, D, W1, W2, M);
  TNA_LAUNCHED("vec.hip:2");
  return TNA_OK;
}

tna_status multidot(const double *V, int64_t ldv, int nv, const double *w, int64_t n, double *h, double *part,
                    hipStream_t s) {
  if (nv <= 0) return TNA_OK;
  int G = n_parts(n);
  if (n <= 65536) {  // short vectors: a block per vector, no second pass
    timer_begin("vec.multidot", s);
    hipLaunchKernelGGL(multidot_small_kernel, dim3(nv), dim3(NT), 0, s, V, ldv, w, n, h);
    timer_end("vec.multidot", 2.0 * nv * (double)n, 8.0 * (nv + 1) * (double)n, s);
    TNA_LAUNCHED("vec.multidot");
    return TNA_OK;
  }
  timer_begin("vec.multidot", s);
  hipLaunchKernelGGL(multidot_kernel, dim3(G), dim3(NT), 0, s, V, ldv, nv, w, n, part);
  timer_end("vec.multidot", 2.0 * nv * (double)n, 8.0 * (nv + 1) * (double)n, s);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(nv), dim3(NT), 0, s, part, G, h);
  TNA_LAUNCHED("vec.hip:3");
  return TNA_OK;
}

tna_status axpy_multi(const double *V, int64_t ldv, int nv, const double *h, double *w, int64_t n, double *nrm2,
                      double *part, hipStream_t s) {
  int G = n_parts(n);
  timer_begin("vec.axpy", s);
  hipLaunchKernelGGL(axpy_multi_kernel, dim3(G), dim3(NT), 0, s, V, ldv, nv, h, w, n, nrm2 ? part : nullptr);
  timer_end("vec.axpy", 2.0 * nv * (double)n, 8.0 * (nv + 2) * (double)n, s);
  if (nrm2) hipLaunchKernelGGL(reduce_parts_kernel, dim3(1), dim3(NT), 0, s, part, G, nrm2);
  TNA_LAUNCHED("vec.hip:4");
  return TNA_OK;
}

tna_status combine(const double *V, int64_t ldv, int nv, const double *c, double *y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3(grid_for(n)), dim3(NT), 0, s, V, ldv, nv, c, y, n);
  TNA_LAUNCHED("vec.hip:5");
  return TNA_OK;
}

tna_status norm2(const double *x, int64_t n, double *out, double *part, hipStream_t s) {
  int G = n_parts(n);
  hipLaunchKernelGGL(norm2_kernel, dim3(G), dim3(NT), 0, s, x, n, part);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(1), dim3(NT), 0, s, part, G, out);
  TNA_LAUNCHED("vec.hip:6");
  return TNA_OK;
}

tna_status scale(const double *x, double *y, int64_t n, const double *nrm2, double scal, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(NT), 0, s, x, y, n, nrm2, scal);
  TNA_LAUNCHED("vec.hip:7");
  return TNA_OK;
}

tna_status check_finite(const double *x, int64_t n, int *flag, hipStream_t s) {
  hipLaunchKernelGGL(finite_kernel, dim3(grid_for(n)), dim3(NT), 0, s, x, n, flag);
  TNA_LAUNCHED("vec.hip:8");
  return TNA_OK;
}

tna_status convert_f64_f32(const double *x, float *y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(cvt_kernel, dim3(grid_for(n)), dim3(NT), 0, s, x, y, n);
  TNA_LAUNCHED("vec.hip:9");
  return TNA_OK;
}

tna_status fill(double *x, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return TNA_OK;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(NT), 0, s, x, n, v);
  TNA_LAUNCHED("vec.hip:10");
  return TNA_OK;
}

tna_status fill_int(int *x, int64_t n, int v, hipStream_t s) {
  if (n <= 0) return TNA_OK;
  hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(n)), dim3(NT), 0, s, x, n, v);
  TNA_LAUNCHED("vec.hip:11");
  return TNA_OK;
}

tna_status copy_transpose(const void *A, int m, int n, int type, double *B, hipStream_t s) {
  dim3 grid((n + 31) / 32, (m + 31) / 32);
  if (type == G_F64)
    hipLaunchKernelGGL(transpose_kernel<double>, grid, dim3(NT), 0, s, static_cast<const double *>(A), m, n, B);
  else
    hipLaunchKernelGGL(transpose_kernel<float>, grid, dim3(NT), 0, s, static_cast<const float *>(A), m, n, B);
  TNA_LAUNCHED("vec.hip:12");
  return TNA_OK;
}

tna_status set_identity(double *J, int n, int ld, int batch, int64_t stride, hipStream_t s) {
  int64_t total = (int64_t)n * ld;
  dim3 grid((unsigned)grid_for(total), batch);
  hipLaunchKernelGGL(identity_kernel, grid, dim3(NT), 0, s, J, n, ld, stride);
  TNA_LAUNCHED("vec.hip:13");
  return TNA_OK;
}

}  // namespace tna
