// Grouped kernels of the batched-chain sweep: many independent chains, each
// at its own bond and with its own bond dimensions, advance through one set
// of launches per step.  One grid y-slice per chain; a chain whose device
// `active` flag is zero (converged, or finished with its sweep) returns at
// once.  Each chain's Lanczos iteration index j lives in device memory, so the
// launch sequence of one iteration does not change from one iteration to the
// next and is captured once per sweep step as a HIP graph.
#include "dev_reduce.h"
#include "internal.h"

namespace tna {
namespace {

constexpr int NT = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double block_sum(double v, double *sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ mixing
// Pointers read from a descriptor in memory are generic to the compiler, which then uses flat
// accesses (counted against both memory and LDS waits); the mixing's operands live in device
// memory, so they are cast to the global address space.
template <typename T> using gptr = T __attribute__((address_space(1))) *;

// One thread per (o0, o1): the J outputs from the I inputs with the J x I matrix M, which every thread
// of the launch reads at the same addresses: through the constant address space those reads become
// scalar loads shared by the wave.  The channel counts are template constants for the MPOs and
// physical dimensions in use (CI1 = 0: runtime counts, at most 32 channels).
template <typename T, int CI1, int CI2, int CJ1, int CJ2>
__global__ __launch_bounds__(NT) void mix_grouped_kernel(const MixProb *probs, int rI1, int rI2, int rJ1, int rJ2) {
  constexpr bool fixed = CI1 > 0;
  const int I1 = fixed ? CI1 : rI1, I2 = fixed ? CI2 : rI2, J1 = fixed ? CJ1 : rJ1, J2 = fixed ? CJ2 : rJ2;
  constexpr int IM = fixed ? CI1 * CI2 : 32, JM = fixed ? CJ1 * CJ2 : 32;
  const MixProb &p = probs[blockIdx.y];
  if (p.active && !*p.active) return;
  const int I = I1 * I2, J = J1 * J2;
  const double __attribute__((address_space(4))) *Ms = (const double __attribute__((address_space(4))) *)p.M;
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t total = (int64_t)p.n0 * p.n1;
  if (idx >= total) return;
  const int64_t o0 = idx / p.n1, o1 = idx - o0 * p.n1;
  const gptr<const T> in = (gptr<const T>)(static_cast<const T *>(p.in) + o0 * p.is0 + o1 * p.is1);
  const gptr<T> out = (gptr<T>)(static_cast<T *>(p.out) + o0 * p.os0 + o1 * p.os1);
  const gptr<const double> inl =
      p.in_last ? (gptr<const double>)(p.in_last + (p.jin ? (int64_t)(*p.jin) * p.jin_stride : 0) + o0 * p.is0_last +
                                       o1 * p.is1)
                : nullptr;
  const gptr<double> outf =
      p.out_first ? (gptr<double>)(p.out_first + (p.jout ? (int64_t)(*p.jout) * p.jout_stride : 0) + o0 * p.os0_first +
                                   o1 * p.os1)
                  : nullptr;
  T x[IM];
#pragma unroll
  for (int i = 0; i < IM; ++i) {
    T v = T(0);
    if (i < I) v = (inl && i / I2 == I1 - 1) ? (T)inl[(i % I2) * p.ich2] : in[(i / I2) * p.ich1 + (i % I2) * p.ich2];
    x[i] = v;
  }
#pragma unroll
  for (int j = 0; j < JM; ++j) {
    if (j < J) {
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < IM; ++i)
        if (i < I) acc += (T)Ms[j * I + i] * x[i];
      if (outf && j % J2 == 0) outf[(j / J2) * p.och1_first] = (double)acc;
      else out[(j / J2) * p.och1 + (j % J2) * p.och2] = acc;
    }
  }
}

__global__ __launch_bounds__(NT) void ident_dev_kernel(const double *E, int chi, int D, int w, double *out) {
  double m = 0.0;
  const int64_t n = (int64_t)chi * chi;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const int64_t a = e / chi, b = e - a * chi;
    m = fmax(m, fabs(E[(a * D + w) * chi + b] - (a == b ? 1.0 : 0.0)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0)
    atomicMax(reinterpret_cast<unsigned long long *>(out), (unsigned long long)__double_as_longlong(m));
}

// ------------------------------------------------------------------ Lanczos
// Block b of a chain's G covers elements [beg, end) of the length-n vectors.  For even n (rows
// 16-byte aligned) the chunks are whole groups of four elements and every thread keeps two
// 16-byte loads per vector in flight, which the streaming passes need to approach the HBM
// rate; odd n takes one element per thread and step.
__device__ inline void lz_range(const LzProb &p, bool vec, int64_t &beg, int64_t &end) {
  int64_t chunk = (p.n + p.G - 1) / p.G;
  if (vec) chunk = (chunk + 3) & ~(int64_t)3;
  beg = chunk * blockIdx.x;
  if (beg > p.n) beg = p.n;
  end = beg + chunk < p.n ? beg + chunk : p.n;
}

// 16-byte load and store of two elements in device memory
typedef double v2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld2(gptr<const double> a) {
  const v2d t = *(gptr<const v2d>)a;
  return make_double2(t.x, t.y);
}
__device__ __forceinline__ void st2(gptr<double> a, double2 v) { *(gptr<v2d>)a = v2d{v.x, v.y}; }

// h[i] partials of <V_i, w> for i <= j, w = V_{j+1}, over block b's range
__device__ __forceinline__ void lz_dot_body(const LzProb &p, double *part, double *sh) {
  const int nv = *p.j + 1;
  const int64_t n = p.n;
  const int G = p.G;
  const gptr<const double> V = (gptr<const double>)p.V, w = V + (int64_t)nv * n;
  const bool vec = (n & 1) == 0;
  int64_t beg, end;
  lz_range(p, vec, beg, end);
  for (int i0 = 0; i0 < nv; i0 += 8) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (vec) {
      for (int64_t e = beg + 4 * threadIdx.x; e < end; e += 4 * NT) {
        const bool two = e + 2 < end;
        const double2 w0 = ld2(w + e);
        const double2 w1 = two ? ld2(w + e + 2) : make_double2(0.0, 0.0);
#pragma unroll
        for (int g = 0; g < 8; ++g)
          if (i0 + g < nv) {
            const gptr<const double> vr = V + (int64_t)(i0 + g) * n + e;
            const double2 a0 = ld2(vr);
            const double2 a1 = two ? ld2(vr + 2) : make_double2(0.0, 0.0);
            acc[g] += (a0.x * w0.x + a0.y * w0.y) + (a1.x * w1.x + a1.y * w1.y);
          }
      }
    } else {
      for (int64_t e = beg + threadIdx.x; e < end; e += NT) {
        const double wv = w[e];
#pragma unroll
        for (int g = 0; g < 8; ++g)
          if (i0 + g < nv) acc[g] += V[(int64_t)(i0 + g) * n + e] * wv;
      }
    }
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      if (i0 + g < nv) {
        const double r = block_sum(acc[g], sh);
        if (threadIdx.x == 0) part[(int64_t)(i0 + g) * G + blockIdx.x] = r;
      }
    }
  }
}


// h[i] = sum_b part[i][b]; grid (kmax+1, chains)
__global__ __launch_bounds__(NT) void lz_reduce_kernel(const LzProb *probs, int which) {
  __shared__ double sh[4];
  const LzProb &p = probs[blockIdx.y];
  const int i = blockIdx.x;
  if (!*p.active || i > *p.j) return;
  const double *part = which ? p.part2 : p.part1;
  double v = 0.0;
  for (int b = threadIdx.x; b < p.G; b += NT) v += part[(int64_t)i * p.G + b];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) (which ? p.h2 : p.h1)[i] = v;
}

// Coefficients that every thread of the launch reads at the same address (written by an earlier
// launch): through the constant address space these are scalar loads.
template <typename T> using cptr = const T __attribute__((address_space(4))) *;

// w -= sum_{i<=j} h[i] V_i over block b's range; with norm: partial |w|^2 into part1[b]
__device__ __forceinline__ void lz_axpy_body(const LzProb &p, const double *hg, int with_norm, double *sh) {
  const cptr<double> h = (cptr<double>)hg;
  const int nv = *p.j + 1;
  const int64_t n = p.n;
  const gptr<const double> V = (gptr<const double>)p.V;
  const gptr<double> w = (gptr<double>)p.V + (int64_t)nv * n;
  const bool vec = (n & 1) == 0;
  int64_t beg, end;
  lz_range(p, vec, beg, end);
  double loc = 0.0;
  if (vec) {
    for (int64_t e = beg + 4 * threadIdx.x; e < end; e += 4 * NT) {
      const bool two = e + 2 < end;
      double s0x = 0.0, s0y = 0.0, s1x = 0.0, s1y = 0.0;
      for (int i = 0; i < nv; ++i) {
        const double hi = h[i];
        const gptr<const double> vr = V + (int64_t)i * n + e;
        const double2 a0 = ld2(vr);
        const double2 a1 = two ? ld2(vr + 2) : make_double2(0.0, 0.0);
        s0x += hi * a0.x;
        s0y += hi * a0.y;
        s1x += hi * a1.x;
        s1y += hi * a1.y;
      }
      const double2 w0 = ld2(w + e);
      const double2 v0 = make_double2(w0.x - s0x, w0.y - s0y);
      st2(w + e, v0);
      loc += v0.x * v0.x + v0.y * v0.y;
      if (two) {
        const double2 w1 = ld2(w + e + 2);
        const double2 v1 = make_double2(w1.x - s1x, w1.y - s1y);
        st2(w + e + 2, v1);
        loc += v1.x * v1.x + v1.y * v1.y;
      }
    }
  } else {
    for (int64_t e = beg + threadIdx.x; e < end; e += NT) {
      double acc = 0.0;
      for (int i = 0; i < nv; ++i) acc += h[i] * V[(int64_t)i * n + e];
      const double v = w[e] - acc;
      w[e] = v;
      loc += v * v;
    }
  }
  if (with_norm) {
    const double r = block_sum(loc, sh);
    if (threadIdx.x == 0) p.part1[blockIdx.x] = r;
  }
}


// Passes over one chain's range with a basis of NV vectors, w = V_NV.  NV is a compile-time constant
// of each case (no guarded loads; all NV loads of an element pair are in flight at once):
//   LZ_DOT:    partials of <V_i, w>;
//   LZ_UPDOT:  w -= sum_i h[i] V_i, then partials of <V_i, w> from the same loads: the first CGS
//              pass's update fused with the second pass's projections, one read of the basis for both;
//   LZ_UPNORM: w -= sum_i h[i] V_i and the partial of |w|^2.
// Per-wave partials go to sw[i][wave] (the norm's to sw[0][wave]).  Bases longer than LZ_FIXED_MAX
// vectors take lz_dot_body / lz_axpy_body.
enum { LZ_DOT = 0, LZ_UPDOT = 1, LZ_UPNORM = 2 };
constexpr int LZ_FIXED_MAX = 24;
template <int NV, int MODE>
__device__ __forceinline__ void lz_fixed(gptr<const double> V, gptr<double> w, cptr<double> h, int64_t n,
                                         int64_t beg, int64_t end, bool vec, double (*sw)[NT / 64]) {
  constexpr bool upd = MODE != LZ_DOT, dots = MODE != LZ_UPNORM;
  constexpr int NA = dots ? NV : 1;
  double hv[NV], acc[NA];
#pragma unroll
  for (int i = 0; i < NV; ++i) hv[i] = upd ? h[i] : 0.0;
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = 0.0;
  if (vec) {  // beg and end even: whole 16-byte pairs
    for (int64_t e = beg + 2 * threadIdx.x; e < end; e += 2 * NT) {
      double2 v[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = ld2(V + (int64_t)i * n + e);
      double2 wv = ld2(w + e);
      if (upd) {
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          sx += hv[i] * v[i].x;
          sy += hv[i] * v[i].y;
        }
        wv.x -= sx;
        wv.y -= sy;
        st2(w + e, wv);
      }
      if (dots) {
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += v[i].x * wv.x + v[i].y * wv.y;
      } else {
        acc[0] += wv.x * wv.x + wv.y * wv.y;
      }
    }
  } else {
    for (int64_t e = beg + threadIdx.x; e < end; e += NT) {
      double v[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = V[(int64_t)i * n + e];
      double wv = w[e];
      if (upd) {
        double sx = 0.0;
#pragma unroll
        for (int i = 0; i < NV; ++i) sx += hv[i] * v[i];
        wv -= sx;
        w[e] = wv;
      }
      if (dots) {
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += v[i] * wv;
      } else {
        acc[0] += wv * wv;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const double r = wave_sum(acc[i]);
    if ((threadIdx.x & 63) == 0) sw[i][threadIdx.x >> 6] = r;
  }
}

// One pass of block b over chain p's range for nv <= LZ_FIXED_MAX; partials into part[i * G + b].
template <int MODE>
__device__ __forceinline__ void lz_pass(const LzProb &p, int nv, const double *hg, double *part,
                                        double (*sw)[NT / 64]) {
  const int64_t n = p.n;
  const int G = p.G;
  const gptr<const double> V = (gptr<const double>)p.V;
  const gptr<double> w = (gptr<double>)p.V + (int64_t)nv * n;
  const cptr<double> h = (cptr<double>)hg;
  const bool vec = (n & 1) == 0;
  int64_t beg, end;
  lz_range(p, vec, beg, end);
  switch (nv) {
#define LZ_F(k) \
  case k: lz_fixed<k, MODE>(V, w, h, n, beg, end, vec, sw); break;
    LZ_F(1) LZ_F(2) LZ_F(3) LZ_F(4) LZ_F(5) LZ_F(6) LZ_F(7) LZ_F(8) LZ_F(9) LZ_F(10) LZ_F(11) LZ_F(12) LZ_F(13) LZ_F(14) LZ_F(15) LZ_F(16) LZ_F(17) LZ_F(18) LZ_F(19) LZ_F(20) LZ_F(21) LZ_F(22) LZ_F(23) LZ_F(24)
#undef LZ_F
  }
  __syncthreads();
  const int nout = MODE == LZ_UPNORM ? 1 : nv;
  if ((int)threadIdx.x < nout) {
    const double *q = sw[threadIdx.x];
    part[(int64_t)threadIdx.x * G + blockIdx.x] = (q[0] + q[1]) + (q[2] + q[3]);
  }
}

// CGS projections: h[i] partials of <V_i, w> into part1 (which = 0) or part2; grid (G, chains)
__global__ __launch_bounds__(NT) void lz_dot_kernel(const LzProb *probs, int which) {
  __shared__ double sh[4];
  __shared__ double sw[LZ_FIXED_MAX][NT / 64];
  const LzProb &p = probs[blockIdx.y];
  if (!*p.active || (int)blockIdx.x >= p.G) return;
  const int nv = *p.j + 1;
  double *part = which ? p.part2 : p.part1;
  if (nv > LZ_FIXED_MAX) lz_dot_body(p, part, sh);
  else lz_pass<LZ_DOT>(p, nv, nullptr, part, sw);
}

// CGS update with h1 (which = 0) or h2; with norm: partial |w|^2 into part1[b]; grid (G, chains)
__global__ __launch_bounds__(NT) void lz_axpy_kernel(const LzProb *probs, int which, int with_norm) {
  __shared__ double sh[4];
  __shared__ double sw[LZ_FIXED_MAX][NT / 64];
  const LzProb &p = probs[blockIdx.y];
  if (!*p.active || (int)blockIdx.x >= p.G) return;
  const int nv = *p.j + 1;
  const double *h = which ? p.h2 : p.h1;
  if (nv > LZ_FIXED_MAX || !with_norm) lz_axpy_body(p, h, with_norm, sh);
  else lz_pass<LZ_UPNORM>(p, nv, h, p.part1, sw);
}

// First-pass update with h1 fused with the second-pass projections into part2; grid (G, chains)
__global__ __launch_bounds__(NT) void lz_axpy_dot_kernel(const LzProb *probs) {
  __shared__ double sh[4];
  __shared__ double sw[LZ_FIXED_MAX][NT / 64];
  const LzProb &p = probs[blockIdx.y];
  if (!*p.active || (int)blockIdx.x >= p.G) return;
  const int nv = *p.j + 1;
  if (nv > LZ_FIXED_MAX) {
    lz_axpy_body(p, p.h1, 0, sh);
    __syncthreads();
    lz_dot_body(p, p.part2, sh);
    return;
  }
  lz_pass<LZ_UPDOT>(p, nv, p.h1, p.part2, sw);
}

// beta^2 = sum of the norm partials; records alpha_j, beta_j^2; grid (1, chains)
__global__ __launch_bounds__(NT) void lz_record_kernel(const LzProb *probs) {
  __shared__ double sh[4];
  const LzProb &p = probs[blockIdx.y];
  if (!*p.active) return;
  double v = 0.0;
  for (int b = threadIdx.x; b < p.G; b += NT) v += p.part1[b];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) {
    const int j = *p.j;
    *p.nrm2 = v;
    p.rec[0] = p.h1[j];  // alpha_j
    p.rec[1] = v;        // beta_j^2
  }
}

// V_{j+1} /= beta_j (if beta_j is not negligible); grid (G, chains)
__global__ __launch_bounds__(NT) void lz_normalize_kernel(const LzProb *probs) {
  const LzProb &p = probs[blockIdx.y];
  if (!*p.active || (int)blockIdx.x >= p.G) return;
  const double b2 = *p.nrm2;
  if (!(b2 > 1e-28)) return;
  const double f = 1.0 / sqrt(b2);
  double *w = p.V + (int64_t)(*p.j + 1) * p.n;
  const int64_t chunk = (p.n + p.G - 1) / p.G;
  const int64_t beg = chunk * blockIdx.x, end = beg + chunk < p.n ? beg + chunk : p.n;
  for (int64_t e = beg + threadIdx.x; e < end; e += NT) w[e] *= f;
}

__global__ void lz_advance_kernel(const LzProb *probs, int nch) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nch && *probs[c].active) *probs[c].j += 1;
}

// Normalisation of theta; grid (G, chains) or (1, chains) for mode 1.
// mode 0: partials of |theta|^2 into part1; mode 1: reduce into nrm2;
// mode 2: V_0 = theta / |theta|; mode 3: theta /= |theta|.
__global__ __launch_bounds__(NT) void lz_norm_kernel(const LzProb *probs, int mode, int src_theta) {
  __shared__ double sh[4];
  const LzProb &p = probs[blockIdx.y];
  if (!*p.active) return;
  const double *src = src_theta ? p.theta : p.V;
  if (mode == 1) {
    double v = 0.0;
    for (int b = threadIdx.x; b < p.G; b += NT) v += p.part1[b];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) *p.nrm2 = v;
    return;
  }
  if (mode == 3) {  // theta /= |theta| in place
    if ((int)blockIdx.x >= p.G) return;
    const double f = 1.0 / sqrt(*p.nrm2);
    const int64_t chunk = (p.n + p.G - 1) / p.G;
    const int64_t beg = chunk * blockIdx.x, end = beg + chunk < p.n ? beg + chunk : p.n;
    for (int64_t e = beg + threadIdx.x; e < end; e += NT) p.theta[e] *= f;
    return;
  }
  if ((int)blockIdx.x >= p.G) return;
  const int64_t chunk = (p.n + p.G - 1) / p.G;
  const int64_t beg = chunk * blockIdx.x, end = beg + chunk < p.n ? beg + chunk : p.n;
  if (mode == 0) {
    double loc = 0.0;
    for (int64_t e = beg + threadIdx.x; e < end; e += NT) loc += src[e] * src[e];
    const double r = block_sum(loc, sh);
    if (threadIdx.x == 0) p.part1[blockIdx.x] = r;
  } else {
    const double f = 1.0 / sqrt(*p.nrm2);  // mode 2: V_0 = theta / |theta|
    for (int64_t e = beg + threadIdx.x; e < end; e += NT) p.V[e] = src[e] * f;
  }
}

// theta = sum_{i < nkeep} y_i V_i (the Ritz vector, unnormalised); grid (G, chains)
__global__ __launch_bounds__(NT) void lz_combine_kernel(const LzProb *probs) {
  const LzProb &p = probs[blockIdx.y];
  if (!*p.active || (int)blockIdx.x >= p.G) return;
  const int nv = p.nkeep;
  const int64_t chunk = (p.n + p.G - 1) / p.G;
  const int64_t beg = chunk * blockIdx.x, end = beg + chunk < p.n ? beg + chunk : p.n;
  for (int64_t e = beg + threadIdx.x; e < end; e += NT) {
    double acc = 0.0;
    for (int i = 0; i < nv; ++i) acc += p.y[i] * p.V[(int64_t)i * p.n + e];
    p.theta[e] = acc;
  }
}

// Start and Ritz steps of a chain whose vectors fit one partition (G == 1), one workgroup each:
// V_0 = theta / |theta|, and theta = sum_i y_i V_i normalised in place.
__global__ __launch_bounds__(NT) void lz_start1_kernel(const LzProb *probs) {
  __shared__ double sh[4];
  const LzProb &p = probs[blockIdx.x];
  if (!*p.active) return;
  double loc = 0.0;
  for (int64_t e = threadIdx.x; e < p.n; e += NT) loc += p.theta[e] * p.theta[e];
  const double f = 1.0 / sqrt(block_sum(loc, sh));
  for (int64_t e = threadIdx.x; e < p.n; e += NT) p.V[e] = p.theta[e] * f;
}

__global__ __launch_bounds__(NT) void lz_ritz1_kernel(const LzProb *probs) {
  __shared__ double sh[4];
  const LzProb &p = probs[blockIdx.x];
  if (!*p.active) return;
  const int nv = p.nkeep;
  double loc = 0.0;
  for (int64_t e = threadIdx.x; e < p.n; e += NT) {
    double acc = 0.0;
    int i = 0;
    for (; i + 8 <= nv; i += 8) {
      double x[8];
#pragma unroll
      for (int g = 0; g < 8; ++g) x[g] = p.V[(int64_t)(i + g) * p.n + e];
#pragma unroll
      for (int g = 0; g < 8; ++g) acc += p.y[i + g] * x[g];
    }
    for (; i < nv; ++i) acc += p.y[i] * p.V[(int64_t)i * p.n + e];
    p.theta[e] = acc;
    loc += acc * acc;
  }
  const double f = 1.0 / sqrt(block_sum(loc, sh));
  for (int64_t e = threadIdx.x; e < p.n; e += NT) p.theta[e] *= f;
}

// ------------------------------------------------------------------ single-workgroup Lanczos
// Whole Lanczos iterations of one short theta inside one workgroup (grid x =
// chain).  H_eff (Eq. 18's contraction in the order L, W_i W_{i+1}, R) runs as
// three small MFMA products on LDS-resident operands, a chunk of `ac` left
// indices at a time:
//   X[(a,w)][(s',t',c')] = sum_a' L[(a,w)][a'] theta[a'][(s',t',c')]
//   Z[o=(s,t,w'')][(a,c')] = sum_i M[o][i=(w,s',t')] X[a][i][c']
//   out[(a,s,t)][c] = sum_{(w'',c')} Z[a][(s,t,w'')][c'] R[c][(w'',c')]
// The operand type T is double (v_mfma_f64_16x16x4_f64) or float (the
// mixed-precision form: L, R, M and theta rounded to FP32 in LDS, products on
// v_mfma_f32_16x16x4_f32 with FP32 accumulation, the result stored as FP64).
// CGS2 against the FP64 basis in global memory follows (dot products eight at
// a time); alpha_j, beta_j^2 of every iteration go to rec[2j], rec[2j+1].  A
// workgroup stops at kmax, after `iters` iterations, or when beta_j is
// negligible.
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int NTS = 512;  // threads of the single-workgroup Lanczos (8 waves)

// x / d for 0 <= x < 2^16 and 1 <= d < 2^16 with one multiply-high by ceil(2^32 / d) (exact in
// that range: the rounding error of the reciprocal, times x, stays below 1 / d).
struct FastDiv {
  unsigned m;
  int d;
  __device__ explicit FastDiv(int d_) : m(d_ > 1 ? (unsigned)(((1ull << 32) + d_ - 1) / d_) : 0u), d(d_) {}
  __device__ int div(int x) const { return d > 1 ? (int)__umulhi((unsigned)x, m) : x; }
};

// 16 x 16 x 4 MFMA step and result layout per operand type.  Operands: A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k.  Result register r of lane group lk = lane / 16 holds row 4r + lk
// (f64) or 4lk + r (f32), column lane % 16.
template <class T> struct Mf;
template <> struct Mf<double> {
  typedef v4d acc;
  __device__ static acc step(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int r) { return 4 * r + lk; }
};
template <> struct Mf<float> {
  typedef v4f acc;
  __device__ static acc step(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int r) { return 4 * lk + r; }
};

// One 16 x 16 output tile, C(i, j) = sum_{kb <= k < ke} A(i, k) B(k, j).  Rows and columns past
// the matrix edge read the last valid row/column (their results are discarded by the caller), so
// only a final partial k-step needs a guard.  The operands of four k-steps are read together and
// fed to two independent accumulator chains.
template <class T, class FA, class FB>
__device__ inline typename Mf<T>::acc tile_mfma(int kb, int ke, int ia, int jb, int lk, FA a_at, FB b_at) {
  typedef typename Mf<T>::acc A4;
  A4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
  const int k16 = kb + ((ke - kb) & ~15), k4 = kb + ((ke - kb) & ~3);
  int k0 = kb;
  for (; k0 < k16; k0 += 16) {
    T av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = a_at(ia, k0 + 4 * u + lk);
      bv[u] = b_at(k0 + 4 * u + lk, jb);
    }
    c0 = Mf<T>::step(av[0], bv[0], c0);
    c1 = Mf<T>::step(av[1], bv[1], c1);
    c0 = Mf<T>::step(av[2], bv[2], c0);
    c1 = Mf<T>::step(av[3], bv[3], c1);
  }
  for (; k0 < k4; k0 += 4) c0 = Mf<T>::step(a_at(ia, k0 + lk), b_at(k0 + lk, jb), c0);
  if (k0 < ke) {
    const bool in = k0 + lk < ke;
    const T av = in ? a_at(ia, k0 + lk) : T(0), bv = in ? b_at(k0 + lk, jb) : T(0);
    c1 = Mf<T>::step(av, bv, c1);
  }
  return c0 + c1;
}

// C = A B over the whole workgroup, the waves taking 16 x 16 tiles in turn.  With no more than
// half as many tiles as waves (and `part` holding tiles x 256 values within part_cap), each
// tile's k range is split between two waves and the second half's partial sums pass through
// `part` in LDS.
template <class T, class FA, class FB, class FC>
__device__ inline void block_gemm(int M, int N, int K, FA a_at, FB b_at, FC c_put, T *part = nullptr,
                                  int part_cap = 0) {
  typedef typename Mf<T>::acc A4;
  const int lane = threadIdx.x & 63, nw = NTS / 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int tn = (N + 15) >> 4, tiles = ((M + 15) >> 4) * tn;
  if (part != nullptr && 2 * tiles <= nw && K >= 32 && tiles * 256 <= part_cap) {
    const int kh = ((K >> 1) + 3) & ~3;
    const bool have = wave < 2 * tiles, second = wave >= tiles;
    const int t = second ? wave - tiles : wave;
    const int i0 = (t / tn) << 4, j0 = (t - (t / tn) * tn) << 4;
    const int ia = min(i0 + lr, M - 1), jb = j0 + lr, jc = min(jb, N - 1);
    A4 acc = {0, 0, 0, 0};
    if (have) acc = tile_mfma<T>(second ? kh : 0, second ? K : kh, ia, jc, lk, a_at, b_at);
    if (have && second)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[(t * 64 + lane) * 4 + r] = acc[r];
    __syncthreads();
    if (have && !second)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + Mf<T>::row(lk, r);
        if (i < M && jb < N) c_put(i, jb, acc[r] + part[(t * 64 + lane) * 4 + r]);
      }
    return;
  }
  for (int t = wave; t < tiles; t += nw) {
    const int i0 = (t / tn) << 4, j0 = (t - (t / tn) * tn) << 4;
    const int ia = min(i0 + lr, M - 1), jb = j0 + lr, jc = min(jb, N - 1);
    const A4 acc = tile_mfma<T>(0, K, ia, jc, lk, a_at, b_at);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + Mf<T>::row(lk, r);
      if (i < M && jb < N) c_put(i, jb, acc[r]);
    }
  }
}

// NB independent products C_b = A B_b (one shared A), the tiles of all products dealt to the
// waves in turn.
template <class T, class FA, class FB, class FC>
__device__ inline void block_gemm_nb(int NB, int M, int N, int K, FA a_at, FB b_at, FC c_put) {
  typedef typename Mf<T>::acc A4;
  const int lane = threadIdx.x & 63, nw = NTS / 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int tn = (N + 15) >> 4, tpb = ((M + 15) >> 4) * tn;
  for (int t = wave; t < NB * tpb; t += nw) {
    const int b = t / tpb, tt = t - b * tpb;
    const int i0 = (tt / tn) << 4, j0 = (tt - (tt / tn) * tn) << 4;
    const int ia = min(i0 + lr, M - 1), jb = j0 + lr, jc = min(jb, N - 1);
    const A4 acc = tile_mfma<T>(0, K, ia, jc, lk, a_at, [&](int k, int j) { return b_at(b, k, j); });
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + Mf<T>::row(lk, r);
      if (i < M && jb < N) c_put(b, i, jb, acc[r]);
    }
  }
}

// Workgroup sum (fixed order), returned to every thread.
__device__ inline double block_total(double v, double *sh) {
  v = wave_total(v);
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < NTS / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

template <class T>
__global__ __launch_bounds__(NTS) void lz_small_kernel(const LzSmall *probs, int iters) {
  extern __shared__ double lds[];
  const LzSmall &p = probs[blockIdx.x];
  if (!*p.active) return;
  constexpr int dd = 4;  // d^2, d = 2
  constexpr int NW = NTS / 64;
  const int D = p.D, DD = D * dd;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int chl = p.chl, chr = p.chr, ac = p.ac, kmax = p.kmax;
  // descriptor fields in registers: the stores into the basis below could alias the descriptor for
  // the compiler, which would otherwise reload them from memory inside the iteration loop
  double *const V = p.V;
  double *const rec = p.rec;
  const int n = chl * dd * chr, nr = dd * chr;
  // Rows that the MFMA operand reads walk down (sixteen lanes, one row each) are stored with an
  // odd stride in elements, so those lanes fall on distinct LDS banks.
  const int ldl = chl | 1, ldr = (D * chr) | 1, ldm = DD | 1, ldz = (D * chr) | 1;
  const FastDiv divD(D), divC(chr);
  double *wv = lds;                                  // n: H V_j, then orthogonalised (FP64)
  double *hb = wv + n;                               // h of the two CGS passes
  double *red = hb + 2 * LZ_HMAX;                    // per-wave partial sums
  T *th = reinterpret_cast<T *>(red + 16 * NW);      // n: V_j in the operand type
  T *Ls = th + n;                                    // L[a][w][a'], rows (a, w) of stride ldl
  T *Rs = Ls + (size_t)chl * D * ldl;                // R[c][w''][c'], rows c of stride ldr
  T *Ms = Rs + (size_t)chr * ldr;                    // M[o][i], rows o of stride ldm
  T *Xc = Ms + DD * ldm;                             // X[al][i][c'] of a chunk
  T *Zc = Xc + (size_t)ac * DD * chr;                // Z[al][s t][w''][c'], rows (al, s t) of stride ldz
  for (int e = tid; e < chl * D * chl; e += NTS) Ls[(e / chl) * ldl + e % chl] = (T)p.L[e];
  for (int e = tid; e < chr * D * chr; e += NTS) Rs[(e / (D * chr)) * ldr + e % (D * chr)] = (T)p.R[e];
  for (int e = tid; e < DD * DD; e += NTS) Ms[(e / DD) * ldm + e % DD] = (T)p.M[e];
  int j = *p.j;
  for (int it = 0; it < iters && j < kmax; ++it) {
    const double *vj = V + (int64_t)j * n;
    double *vn = V + (int64_t)(j + 1) * n;
    __syncthreads();  // previous iteration done with th, wv and hb
    for (int e = tid; e < n; e += NTS) th[e] = (T)vj[e];
    __syncthreads();
    for (int a0 = 0; a0 < chl; a0 += ac) {
      const int na = chl - a0 < ac ? chl - a0 : ac;
      block_gemm<T>(na * D, nr, chl, [&](int i, int k) { return Ls[(a0 * D + i) * ldl + k]; },
                    [&](int k, int c) { return th[k * nr + c]; },
                    [&](int i, int c, T v) { Xc[i * nr + c] = v; });
      __syncthreads();
      // output row o = (s t, w'') goes to Zc row (al, s t) at column w'' chr + c'
      if (chr >= 16)  // one product per row index al: no division in the operand addressing
        block_gemm_nb<T>(na, DD, chr, DD, [&](int o, int i) { return Ms[o * ldm + i]; },
                         [&](int al, int i, int c) { return Xc[(al * DD + i) * chr + c]; },
                         [&](int al, int o, int c, T v) {
                           const int st = divD.div(o);
                           Zc[(al * dd + st) * ldz + (o - st * D) * chr + c] = v;
                         });
      else  // narrow right bond: the al blocks side by side in one product, so tiles stay full
        block_gemm<T>(DD, na * chr, DD, [&](int o, int i) { return Ms[o * ldm + i]; },
                      [&](int i, int c) {
                        const int al = divC.div(c);
                        return Xc[(al * DD + i) * chr + (c - al * chr)];
                      },
                      [&](int o, int c, T v) {
                        const int al = divC.div(c), st = divD.div(o);
                        Zc[(al * dd + st) * ldz + (o - st * D) * chr + (c - al * chr)] = v;
                      });
      __syncthreads();
      block_gemm<T>(na * dd, chr, D * chr, [&](int i, int q) { return Zc[i * ldz + q]; },
                    [&](int q, int c) { return Rs[c * ldr + q]; },
                    [&](int i, int c, T v) { wv[(a0 * dd + i) * chr + c] = (double)v; }, Xc, ac * DD * chr);
      __syncthreads();
    }
    // CGS2 against V_0..V_j (n is a multiple of 4: element pairs, 16-byte accesses).  Dot
    // products: one wave per basis vector (vectors wave, wave + 8, ..., two at a time), lanes over
    // the element pairs, a DPP reduction; updates: one thread per element pair, sixteen vectors
    // per batch of loads.
    const int n2 = n >> 1;
    const double2 *W2 = reinterpret_cast<const double2 *>(wv);
    double b2 = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      double *h = hb + pass * LZ_HMAX;
      for (int i = wave; i <= j; i += 2 * NW) {
        const bool two = i + NW <= j;
        const double2 *va = reinterpret_cast<const double2 *>(V + (int64_t)i * n);
        const double2 *vb = reinterpret_cast<const double2 *>(V + (int64_t)(two ? i + NW : i) * n);
        double a0 = 0.0, a1 = 0.0, c0 = 0.0, c1 = 0.0;
        int e = lane;
        for (; e + 192 < n2; e += 256) {
          double2 x[4], y[4], w[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            x[u] = va[e + 64 * u];
            y[u] = vb[e + 64 * u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) w[u] = W2[e + 64 * u];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a0 += x[u].x * w[u].x;
            a1 += x[u].y * w[u].y;
            c0 += y[u].x * w[u].x;
            c1 += y[u].y * w[u].y;
          }
        }
        for (; e < n2; e += 64) {
          const double2 x = va[e], y = vb[e], w = W2[e];
          a0 += x.x * w.x;
          a1 += x.y * w.y;
          c0 += y.x * w.x;
          c1 += y.y * w.y;
        }
        const double sa = wave_total(a0 + a1), sc = wave_total(c0 + c1);
        if (lane == 63) {
          h[i] = sa;
          if (two) h[i + NW] = sc;
        }
      }
      __syncthreads();
      double loc = 0.0;
      for (int e = tid; e < n2; e += NTS) {
        const double2 *ve = reinterpret_cast<const double2 *>(V) + e;
        double2 acc = {0.0, 0.0};
        int i = 0;
        for (; i + 16 <= j + 1; i += 16) {
          double2 x[16];
#pragma unroll
          for (int g = 0; g < 16; ++g) x[g] = ve[(int64_t)(i + g) * n2];
#pragma unroll
          for (int g = 0; g < 16; ++g) {
            acc.x += h[i + g] * x[g].x;
            acc.y += h[i + g] * x[g].y;
          }
        }
        for (; i + 4 <= j + 1; i += 4) {
          double2 x[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) x[g] = ve[(int64_t)(i + g) * n2];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            acc.x += h[i + g] * x[g].x;
            acc.y += h[i + g] * x[g].y;
          }
        }
        for (; i <= j; ++i) {
          const double2 x = ve[(int64_t)i * n2];
          acc.x += h[i] * x.x;
          acc.y += h[i] * x.y;
        }
        const double v0 = wv[2 * e] - acc.x, v1 = wv[2 * e + 1] - acc.y;
        wv[2 * e] = v0;
        wv[2 * e + 1] = v1;
        loc += v0 * v0 + v1 * v1;
      }
      if (pass == 1) b2 = block_total(loc, red);
      else __syncthreads();
    }
    if (tid == 0) {
      rec[2 * j] = hb[j];  // alpha_j from the first pass
      rec[2 * j + 1] = b2;
    }
    // the host stops a chain at beta_j < 1e-14 (or a non-finite record): same predicate here
    const double beta = sqrt(b2);
    const bool stop = !(beta >= 1e-14);
    const double f = stop ? 1.0 : 1.0 / beta;
    for (int e = tid; e < n; e += NTS) vn[e] = wv[e] * f;
    ++j;
    if (stop) break;
  }
  if (tid == 0) {
    *p.j = j;
    rec[2 * LZ_HMAX - 1] = (double)j;  // read back with the records (they end below 2 LZ_HMAX - 2)
  }
}

__global__ __launch_bounds__(NT) void convert_grouped_kernel(const CvtProb *probs) {
  const CvtProb &p = probs[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < p.n; e += (int64_t)gridDim.x * NT) p.dst[e] = (float)p.src[e];
}

}  // namespace

tna_status ident_deviation(const double *E, int chi, int D, int w, double *out, hipStream_t s) {
  const int64_t n = (int64_t)chi * chi;
  const unsigned grid = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 1024);
  hipLaunchKernelGGL(ident_dev_kernel, dim3(grid), dim3(NT), 0, s, E, chi, D, w, out);
  TNA_LAUNCHED("ident.check");
  return TNA_OK;
}

tna_status mix_grouped(const MixProb *d, int nprob, int64_t max_elems, int I1, int I2, int J1, int J2, int f32,
                       hipStream_t s) {
  if (nprob < 1 || max_elems < 1) return TNA_OK;
  if (I1 * I2 > 32 || J1 * J2 > 32) {
    set_error("mix_grouped: at most 32 channels");
    return TNA_ERR_ARG;
  }
  dim3 grid((unsigned)((max_elems + NT - 1) / NT), nprob);
  const char *name = f32 ? "mixg.f32" : "mixg.f64";
  timer_begin(name, s);
  // compile-time channel counts for the H_eff mixing (D, d^2, d^2, D) and the environment mixing
  // (D, d, d, D) of the MPOs here (d = 2; D = 3, 5, 8)
  auto launch = [&](auto kf, auto kd) {
    if (f32) hipLaunchKernelGGL(kf, grid, dim3(NT), 0, s, d, I1, I2, J1, J2);
    else hipLaunchKernelGGL(kd, grid, dim3(NT), 0, s, d, I1, I2, J1, J2);
  };
#define TNA_MIX_CASE(a, b, c, e)                                                                       \
  if (I1 == a && I2 == b && J1 == c && J2 == e) {                                                   \
    launch(mix_grouped_kernel<float, a, b, c, e>, mix_grouped_kernel<double, a, b, c, e>);          \
  } else
  TNA_MIX_CASE(5, 4, 4, 5)
  TNA_MIX_CASE(5, 2, 2, 5)
  TNA_MIX_CASE(8, 4, 4, 8)
  TNA_MIX_CASE(8, 2, 2, 8)
  TNA_MIX_CASE(3, 4, 4, 3)
  TNA_MIX_CASE(3, 2, 2, 3)
  launch(mix_grouped_kernel<float, 0, 0, 0, 0>, mix_grouped_kernel<double, 0, 0, 0, 0>);
#undef TNA_MIX_CASE
  timer_end(name, 2.0 * I1 * I2 * J1 * J2 * (double)max_elems * nprob,
            (double)(f32 ? 4 : 8) * (I1 * I2 + J1 * J2) * (double)max_elems * nprob, s);
  TNA_LAUNCHED("mix.grouped");
  return TNA_OK;
}

tna_status lz_iteration(const LzProb *d, int nch, int maxG, int kmax, double bytes_hint, hipStream_t s) {
  const dim3 g(maxG, nch), r(kmax + 1, nch), one(1, nch);
  // CGS2: projections h1, update with h1 fused with the projections h2, update with h2 and |w|^2
  timer_begin("lz.dot", s);
  hipLaunchKernelGGL(lz_dot_kernel, g, dim3(NT), 0, s, d, 0);
  timer_end("lz.dot", bytes_hint / 4.0, bytes_hint, s);
  hipLaunchKernelGGL(lz_reduce_kernel, r, dim3(NT), 0, s, d, 0);
  timer_begin("lz.axpy_dot", s);
  hipLaunchKernelGGL(lz_axpy_dot_kernel, g, dim3(NT), 0, s, d);
  timer_end("lz.axpy_dot", bytes_hint / 2.0, bytes_hint, s);
  hipLaunchKernelGGL(lz_reduce_kernel, r, dim3(NT), 0, s, d, 1);
  timer_begin("lz.axpy", s);
  hipLaunchKernelGGL(lz_axpy_kernel, g, dim3(NT), 0, s, d, 1, 1);
  timer_end("lz.axpy", bytes_hint / 4.0, bytes_hint, s);
  hipLaunchKernelGGL(lz_record_kernel, one, dim3(NT), 0, s, d);
  hipLaunchKernelGGL(lz_normalize_kernel, g, dim3(NT), 0, s, d);
  hipLaunchKernelGGL(lz_advance_kernel, dim3((nch + 63) / 64), dim3(64), 0, s, d, nch);
  TNA_LAUNCHED("lanczos.grouped");
  return TNA_OK;
}

tna_status lz_start(const LzProb *d, int nch, int maxG, hipStream_t s) {
  // V_0 = theta / |theta|
  if (maxG == 1) {
    hipLaunchKernelGGL(lz_start1_kernel, dim3(nch), dim3(NT), 0, s, d);
    TNA_LAUNCHED("lanczos.start");
    return TNA_OK;
  }
  hipLaunchKernelGGL(lz_norm_kernel, dim3(maxG, nch), dim3(NT), 0, s, d, 0, 1);
  hipLaunchKernelGGL(lz_norm_kernel, dim3(1, nch), dim3(NT), 0, s, d, 1, 1);
  hipLaunchKernelGGL(lz_norm_kernel, dim3(maxG, nch), dim3(NT), 0, s, d, 2, 1);
  TNA_LAUNCHED("lanczos.start");
  return TNA_OK;
}

tna_status lz_ritz(const LzProb *d, int nch, int maxG, hipStream_t s) {
  // theta = sum y_i V_i, then normalised in place
  if (maxG == 1) {
    hipLaunchKernelGGL(lz_ritz1_kernel, dim3(nch), dim3(NT), 0, s, d);
    TNA_LAUNCHED("lanczos.ritz");
    return TNA_OK;
  }
  hipLaunchKernelGGL(lz_combine_kernel, dim3(maxG, nch), dim3(NT), 0, s, d);
  hipLaunchKernelGGL(lz_norm_kernel, dim3(maxG, nch), dim3(NT), 0, s, d, 0, 1);
  hipLaunchKernelGGL(lz_norm_kernel, dim3(1, nch), dim3(NT), 0, s, d, 1, 1);
  hipLaunchKernelGGL(lz_norm_kernel, dim3(maxG, nch), dim3(NT), 0, s, d, 3, 1);
  TNA_LAUNCHED("lanczos.ritz");
  return TNA_OK;
}

size_t lz_small_lds(int chl, int chr, int d, int D, int ac, int f32) {
  const size_t n = (size_t)chl * d * d * chr, DD = (size_t)D * d * d;
  const size_t ldl = chl | 1, ldr = (D * chr) | 1, ldm = DD | 1, ldz = ldr;
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  return sizeof(double) * (n + 2 * LZ_HMAX + 16 * (NTS / 64)) +
         es * (n + (size_t)chl * D * ldl + (size_t)chr * ldr + DD * ldm + (size_t)ac * DD * chr +
               (size_t)ac * d * d * ldz);
}

tna_status lz_small(const LzSmall *d, int nch, int D, int dsq, int iters, size_t lds, int f32, hipStream_t s) {
  if (nch < 1) return TNA_OK;
  if (dsq != 4) {
    set_error("lz_small: physical dimension 2 only");
    return TNA_ERR_UNSUPPORTED;
  }
  if (D * dsq > 64) {
    set_error("lz_small: MPO bond dimension above 16");
    return TNA_ERR_UNSUPPORTED;
  }
  static bool attr_set[2] = {false, false};
  const void *fn = f32 ? reinterpret_cast<const void *>(lz_small_kernel<float>)
                       : reinterpret_cast<const void *>(lz_small_kernel<double>);
  if (!attr_set[f32 ? 1 : 0]) {
    TNA_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LZ_SMALL_LDS_MAX));
    attr_set[f32 ? 1 : 0] = true;
  }
  if (lds > LZ_SMALL_LDS_MAX) {
    set_error("lz_small: LDS need above the limit");
    return TNA_ERR_ARG;
  }
  const char *name = f32 ? "lz.small.f32" : "lz.small";
  timer_begin(name, s);
  if (f32) hipLaunchKernelGGL(lz_small_kernel<float>, dim3(nch), dim3(NTS), lds, s, d, iters);
  else hipLaunchKernelGGL(lz_small_kernel<double>, dim3(nch), dim3(NTS), lds, s, d, iters);
  timer_end(name, 0.0, 0.0, s);
  TNA_LAUNCHED("lanczos.small");
  return TNA_OK;
}

tna_status convert_grouped(const CvtProb *d, int nprob, hipStream_t s) {
  if (nprob < 1) return TNA_OK;
  hipLaunchKernelGGL(convert_grouped_kernel, dim3(64, nprob), dim3(NT), 0, s, d);
  TNA_LAUNCHED("convert.grouped");
  return TNA_OK;
}

}  // namespace tna
