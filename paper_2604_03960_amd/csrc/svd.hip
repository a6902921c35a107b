// Truncated SVD (Eq. 3 / Eq. 19) by blocked one-sided Jacobi on gfx950, and
// the spectrum sums of Eq. (4)-(5).
//
// The R = min(m,n) rows of length C = max(m,n) of A (or of A^T when m > n)
// are orthogonalised; the product of the rotations is accumulated in Jt
// (R x R, starts at I).  Rows are grouped in blocks of 32; one Jacobi sweep
// visits every pair of blocks once in round-robin order (nb-1 steps of nb/2
// disjoint pairs).  Per step three launches:
//   gram   G = [B_p; B_q][B_p; B_q]^T (64 x 64) on the FP64 MFMA, K split
//          across workgroups, partial sums in fixed order;
//   eigen  the 64 x 64 symmetric G is diagonalised in LDS by cyclic two-sided
//          Jacobi with a parallel (round-robin) pair order, eigenvectors sorted
//          by eigenvalue (larger rows to the lower block); skipped when every
//          off-diagonal already satisfies |g_ij| <= tol sqrt(g_ii g_jj);
//   apply  [B_p; B_q] <- Q^T [B_p; B_q] and [J_p; J_q] <- Q^T [J_p; J_q] on the
//          MFMA, column slab by column slab, in place.
// A sweep with no rotating pair ends the iteration (one 4-byte host read per
// sweep).  Afterwards sigma_r = |row r|, a bitonic sort orders them, and the
// factors are written with the sign gauge (largest-magnitude entry of each
// left vector positive) and Gram-Schmidt completion of null vectors.
#include "internal.h"

namespace tna {

tna_status DevBuf::ensure(size_t need) {
  if (need <= bytes) return TNA_OK;
  release();
  size_t want = need + need / 4;
  if (hipMalloc(&ptr, want) != hipSuccess) {
    ptr = nullptr;
    bytes = 0;
    set_error("device allocation failed");
    return TNA_ERR_NOMEM;
  }
  bytes = want;
  return TNA_OK;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr double EPS53 = 1.1102230246251565e-16;
constexpr int BS = 32;  // rows per block

// v_mfma_f64_16x16x4_f64: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
// result D[i][j] in lane j + 16(i%4), register i/4.
__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// round-robin pairing of nb blocks (nb even): step s in [0, nb-1), pair t in [0, nb/2)
__device__ inline void rr_pair(int nb, int s, int t, int &p, int &q) {
  const int n1 = nb - 1;
  int a, b;
  if (t == 0) { a = s % n1; b = n1; }
  else { a = (s + t) % n1; b = (s - t + n1) % n1; }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

__device__ inline int block_rows(int R, int blk) {
  int r = R - blk * BS;
  return r < 0 ? 0 : (r > BS ? BS : r);
}

struct SvdDev {
  int R, C, nb, ksplit, step;
  double *bw;   // batch x R x C
  double *jt;   // batch x R x R
  double *gram; // batch x npairs x ksplit x 64 x 64
  double *qt;   // batch x npairs x 64 x 64
  int *skip;    // batch x npairs
  int *ctr;
  double tol;
};

// -------------------------------------------------------------- gram
__global__ __launch_bounds__(256) void gram_kernel(SvdDev a) {
  constexpr int BK = 32;
  __shared__ double Ts[BK][64 + 1];
  const int pair = blockIdx.x, ks = blockIdx.y, z = blockIdx.z;
  const int npairs = a.nb / 2;
  int p, q;
  rr_pair(a.nb, a.step, pair, p, q);
  const int np = block_rows(a.R, p), nq = block_rows(a.R, q);
  const double *B = a.bw + (int64_t)z * a.R * a.C;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int qi = wave >> 1, qj = wave & 1;
  int64_t chunk = (a.C + a.ksplit - 1) / a.ksplit;
  chunk = (chunk + BK - 1) / BK * BK;
  const int64_t kb = chunk * ks;
  const int64_t ke = kb + chunk < a.C ? kb + chunk : a.C;
  v4d acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0, 0, 0, 0};
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int col = tid % BK, r = tid / BK + 8 * u;
      const bool valid = r < 32 ? (r < np) : (r - 32 < nq);
      const int grow = r < 32 ? p * BS + r : q * BS + (r - 32);
      const int64_t gc = k0 + col;
      Ts[col][r] = (valid && gc < ke) ? B[(int64_t)grow * a.C + gc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = Ts[kk + lk][32 * qi + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Ts[kk + lk][32 * qj + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  double *G = a.gram + (((int64_t)z * npairs + pair) * a.ksplit + ks) * 4096;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 32 * qi + 16 * i + 4 * r + lk, col = 32 * qj + 16 * j + lr;  // f64 result layout
        G[row * 64 + col] = acc[i][j][r];
      }
}

// -------------------------------------------------------------- eigen
__global__ __launch_bounds__(256) void eigen_kernel(SvdDev a) {
  __shared__ double Gs[64][65];
  __shared__ double Qs[64][65];
  __shared__ double cs_[32], sn_[32];
  __shared__ int pi_[32], pj_[32];
  __shared__ int rot_any, need;
  __shared__ int slot_of[64];
  const int pair = blockIdx.x, z = blockIdx.y;
  const int npairs = a.nb / 2;
  const int tid = threadIdx.x;
  int p, q;
  rr_pair(a.nb, a.step, pair, p, q);
  const int np = block_rows(a.R, p), nq = block_rows(a.R, q);
  int *skip = a.skip + (int64_t)z * npairs + pair;
  if (np + nq == 0) {
    if (tid == 0) *skip = 1;
    return;
  }
  auto valid = [&](int r) { return r < 32 ? (r < np) : (r - 32 < nq); };
  const double *Gp = a.gram + ((int64_t)z * npairs + pair) * a.ksplit * 4096;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e >> 6, j = e & 63;
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    double v = 0.0;
    for (int ks = 0; ks < a.ksplit; ++ks) v += Gp[(int64_t)ks * 4096 + lo * 64 + hi];
    Gs[i][j] = (valid(i) && valid(j)) ? v : 0.0;
    Qs[i][j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) need = 0;
  __syncthreads();
  // outer test on the fresh Gram
  {
    int loc = 0;
    for (int e = tid; e < 4096; e += 256) {
      const int i = e >> 6, j = e & 63;
      if (i < j) {
        const double gii = Gs[i][i], gjj = Gs[j][j], gij = Gs[i][j];
        if (gii > 0.0 && gjj > 0.0 && fabs(gij) > a.tol * sqrt(gii * gjj)) loc = 1;
      }
    }
    if (__any(loc) && (tid & 63) == 0) atomicOr(&need, 1);
  }
  __syncthreads();
  if (!need) {
    if (tid == 0) *skip = 1;
    return;
  }
  if (tid == 0) atomicAdd(a.ctr, 1);
  const double tol_in = 4.0 * EPS53;
  for (int sweep = 0; sweep < 40; ++sweep) {
    __syncthreads();  // every thread has read rot_any of the previous sweep
    if (tid == 0) rot_any = 0;
    __syncthreads();
    for (int rr = 0; rr < 63; ++rr) {
      if (tid < 32) {
        int i, j;
        if (tid == 0) { i = rr % 63; j = 63; }
        else { i = (rr + tid) % 63; j = (rr - tid + 63) % 63; }
        if (i > j) { const int t = i; i = j; j = t; }
        const double gii = Gs[i][i], gjj = Gs[j][j], gij = Gs[i][j];
        double c = 1.0, s = 0.0;
        if (gij != 0.0 && fabs(gij) > tol_in * sqrt(fabs(gii * gjj))) {
          const double zeta = (gjj - gii) / (2.0 * gij);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + t * t);
          s = c * t;
          rot_any = 1;
        }
        cs_[tid] = c; sn_[tid] = s; pi_[tid] = i; pj_[tid] = j;
      }
      __syncthreads();
      // rows i, j of G
      for (int e = tid; e < 32 * 64; e += 256) {
        const int t = e >> 6, k = e & 63;
        const double s = sn_[t];
        if (s != 0.0) {
          const double c = cs_[t];
          const int i = pi_[t], j = pj_[t];
          const double gi = Gs[i][k], gj = Gs[j][k];
          Gs[i][k] = c * gi - s * gj;
          Gs[j][k] = s * gi + c * gj;
        }
      }
      __syncthreads();
      // columns i, j of G and of Q
      for (int e = tid; e < 32 * 64; e += 256) {
        const int t = e >> 6, k = e & 63;
        const double s = sn_[t];
        if (s != 0.0) {
          const double c = cs_[t];
          const int i = pi_[t], j = pj_[t];
          const double gi = Gs[k][i], gj = Gs[k][j];
          double ni = c * gi - s * gj, nj = s * gi + c * gj;
          if (k == i) nj = 0.0;
          if (k == j) ni = 0.0;
          Gs[k][i] = ni;
          Gs[k][j] = nj;
          const double qi_ = Qs[k][i], qj_ = Qs[k][j];
          Qs[k][i] = c * qi_ - s * qj_;
          Qs[k][j] = s * qi_ + c * qj_;
        }
      }
      __syncthreads();
    }
    const int any = rot_any;
    if (!any) break;
  }
  // order eigenvalues descending (ties: lower slot first); invalid slots last
  if (tid < 64) {
    const int r = tid;
    int slot = -1;
    if (valid(r)) {
      const double lr_ = Gs[r][r];
      int rank = 0;
      for (int o = 0; o < 64; ++o) {
        if (o == r || !valid(o)) continue;
        const double lo = Gs[o][o];
        if (lo > lr_ || (lo == lr_ && o < r)) ++rank;
      }
      slot = rank < np ? rank : 32 + (rank - np);
    }
    if (slot >= 0) slot_of[slot] = r;
  }
  __syncthreads();
  double *Qt = a.qt + ((int64_t)z * npairs + pair) * 4096;
  for (int e = tid; e < 4096; e += 256) {
    const int so = e >> 6, ri = e & 63;
    double v = 0.0;
    if (valid(so) && valid(ri)) v = Qs[ri][slot_of[so]];
    Qt[e] = v;
  }
  if (tid == 0) *skip = 0;
}

// -------------------------------------------------------------- apply
__global__ __launch_bounds__(256) void apply_kernel(SvdDev a, int ntile_b) {
  __shared__ double As[64][65];  // As[k][i] = Qt[i][k]
  __shared__ double Xs[64][65];  // Xs[k][j] = X[row(k)][c0 + j]
  const int pair = blockIdx.x, tile = blockIdx.y, z = blockIdx.z;
  const int npairs = a.nb / 2;
  if (a.skip[(int64_t)z * npairs + pair]) return;
  int p, q;
  rr_pair(a.nb, a.step, pair, p, q);
  const int np = block_rows(a.R, p), nq = block_rows(a.R, q);
  auto valid = [&](int r) { return r < 32 ? (r < np) : (r - 32 < nq); };
  auto grow = [&](int r) { return r < 32 ? p * BS + r : q * BS + (r - 32); };
  double *X;
  int ld, c0;
  if (tile < ntile_b) { X = a.bw + (int64_t)z * a.R * a.C; ld = a.C; c0 = tile * 64; }
  else { X = a.jt + (int64_t)z * a.R * a.R; ld = a.R; c0 = (tile - ntile_b) * 64; }
  const double *Qt = a.qt + ((int64_t)z * npairs + pair) * 4096;
  const int tid = threadIdx.x;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e >> 6, k = e & 63;
    As[k][i] = Qt[e];
    const int r = e >> 6, c = e & 63;
    Xs[r][c] = (valid(r) && c0 + c < ld) ? X[(int64_t)grow(r) * ld + c0 + c] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  v4d acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = v4d{0, 0, 0, 0};
#pragma unroll 4
  for (int kk = 0; kk < 64; kk += 4) {
    const double av = As[kk + lk][16 * wave + lr];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = mfma16(av, Xs[kk + lk][16 * t + lr], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int so = 16 * wave + 4 * r + lk, col = 16 * t + lr;  // f64 result layout
      if (valid(so) && c0 + col < ld) X[(int64_t)grow(so) * ld + c0 + col] = acc[t][r];
    }
}

// -------------------------------------------------------------- finish
__global__ __launch_bounds__(256) void norms_kernel(const double *bw, int R, int C, double *sig) {
  const int z = blockIdx.y;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= R) return;
  const double *row = bw + ((int64_t)z * R + r) * C;
  double s = 0.0;
  for (int c = lane; c < C; c += 64) s += row[c] * row[c];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) sig[(int64_t)z * R + r] = sqrt(s);
}

// bitonic sort of (sigma desc, index asc); P = power of two >= R, P <= 4096
__global__ __launch_bounds__(1024) void sort_kernel(const double *sig, int R, int P, int *perm, double *S_out,
                                                    int64_t strideS) {
  __shared__ double key[4096];
  __shared__ int idx[4096];
  const int z = blockIdx.x;
  for (int i = threadIdx.x; i < P; i += 1024) {
    key[i] = i < R ? sig[(int64_t)z * R + i] : -1.0;
    idx[i] = i;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += 1024) {
        const int l = i ^ j;
        if (l > i) {
          // "before(x, y)": x sorts ahead of y
          const bool i_before_l = key[i] > key[l] || (key[i] == key[l] && idx[i] < idx[l]);
          const bool up = (i & k) == 0;
          if (up ? !i_before_l : i_before_l) {
            const double tk = key[i]; key[i] = key[l]; key[l] = tk;
            const int ti = idx[i]; idx[i] = idx[l]; idx[l] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < R; i += 1024) {
    perm[(int64_t)z * R + i] = idx[i];
    S_out[(int64_t)z * strideS + i] = key[i];
  }
}

struct OutDev {
  int R, C, m, n, k, trans;
  const double *bw, *jt, *S;  // S: sorted spectrum (stride strideS)
  int64_t strideS;
  const int *perm;
  void *U; int64_t strideU;
  void *Vt; int64_t strideVt;
};

// U (m x k) and Vt (k x n), unscaled; null Bw-derived vectors are zeroed
template <typename T>
__global__ __launch_bounds__(256) void write_u_kernel(OutDev o) {
  const int z = blockIdx.y;
  const int64_t total = (int64_t)o.m * o.k;
  const double *S = o.S + (int64_t)z * o.strideS;
  const double thr = EPS53 * S[0] * (o.m > o.n ? o.m : o.n);
  T *U = static_cast<T *>(o.U) + (int64_t)z * o.strideU;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / o.k), j = (int)(e % o.k);
    const int r = o.perm[(int64_t)z * o.R + j];
    double v;
    if (!o.trans) v = o.jt[((int64_t)z * o.R + r) * o.R + i];
    else v = (S[j] > thr && S[j] > 0.0) ? o.bw[((int64_t)z * o.R + r) * o.C + i] / S[j] : 0.0;
    U[e] = (T)v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void write_vt_kernel(OutDev o) {
  const int z = blockIdx.y;
  const int64_t total = (int64_t)o.k * o.n;
  const double *S = o.S + (int64_t)z * o.strideS;
  const double thr = EPS53 * S[0] * (o.m > o.n ? o.m : o.n);
  T *Vt = static_cast<T *>(o.Vt) + (int64_t)z * o.strideVt;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int j = (int)(e / o.n), c = (int)(e % o.n);
    const int r = o.perm[(int64_t)z * o.R + j];
    double v;
    if (o.trans) v = o.jt[((int64_t)z * o.R + r) * o.R + c];
    else v = (S[j] > thr && S[j] > 0.0) ? o.bw[((int64_t)z * o.R + r) * o.C + c] / S[j] : 0.0;
    Vt[e] = (T)v;
  }
}

// Gram-Schmidt completion of kept null vectors with unit vectors e_0, e_1, ...
// The completed factor is Vt (rows) when trans == 0, U (columns) when trans == 1.
template <typename T>
__global__ __launch_bounds__(256) void complete_kernel(OutDev o) {
  __shared__ double vec[4096];
  __shared__ double red[4];
  __shared__ int ok;
  const int z = blockIdx.x;
  const double *S = o.S + (int64_t)z * o.strideS;
  const double thr = EPS53 * S[0] * (o.m > o.n ? o.m : o.n);
  const int L = o.trans ? o.m : o.n;  // vector length
  T *base;
  int64_t es, vs;  // element stride, vector stride
  if (o.trans) { base = static_cast<T *>(o.U) + (int64_t)z * o.strideU; es = o.k; vs = 1; }
  else { base = static_cast<T *>(o.Vt) + (int64_t)z * o.strideVt; es = 1; vs = o.n; }
  const int tid = threadIdx.x;
  auto bsum = [&](double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
  };
  int e = 0;
  for (int j = 0; j < o.k; ++j) {
    if (S[j] > thr && S[j] > 0.0) continue;
    for (; e < L; ++e) {
      for (int i = tid; i < L; i += 256) vec[i] = (i == e) ? 1.0 : 0.0;
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass)
        for (int qv = 0; qv < o.k; ++qv) {
          if (qv == j) continue;
          if (!((S[qv] > thr && S[qv] > 0.0) || qv < j)) continue;
          double h = 0.0;
          for (int i = tid; i < L; i += 256) h += (double)base[qv * vs + (int64_t)i * es] * vec[i];
          h = bsum(h);
          for (int i = tid; i < L; i += 256) vec[i] -= h * (double)base[qv * vs + (int64_t)i * es];
          __syncthreads();
        }
      double nr = 0.0;
      for (int i = tid; i < L; i += 256) nr += vec[i] * vec[i];
      nr = sqrt(bsum(nr));
      if (tid == 0) ok = nr > 0.5;
      __syncthreads();
      if (ok) {
        for (int i = tid; i < L; i += 256) base[j * vs + (int64_t)i * es] = (T)(vec[i] / nr);
        __syncthreads();
        ++e;
        break;
      }
      __syncthreads();
    }
  }
}

// sign gauge: largest-|.| entry of U[:, j] positive (ties: lowest row); then scaling
template <typename T>
__global__ __launch_bounds__(256) void gauge_kernel(OutDev o, int scale_mode, const double *spec) {
  __shared__ double bv[4];
  __shared__ int bi[4];
  __shared__ double sgn;
  const int j = blockIdx.x, z = blockIdx.y, tid = threadIdx.x;
  T *U = static_cast<T *>(o.U) + (int64_t)z * o.strideU;
  T *Vt = static_cast<T *>(o.Vt) + (int64_t)z * o.strideVt;
  double best = -1.0;
  int bidx = 0x7fffffff;
  for (int i = tid; i < o.m; i += 256) {
    const double v = fabs((double)U[(int64_t)i * o.k + j]);
    if (v > best) { best = v; bidx = i; }  // ascending i: first max kept
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bidx, off, 64);
    if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
  }
  if ((tid & 63) == 0) { bv[tid >> 6] = best; bi[tid >> 6] = bidx; }
  __syncthreads();
  if (tid == 0) {
    double b = bv[0];
    int ii = bi[0];
    for (int w = 1; w < 4; ++w)
      if (bv[w] > b || (bv[w] == b && bi[w] < ii)) { b = bv[w]; ii = bi[w]; }
    sgn = ((double)U[(int64_t)ii * o.k + j] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  const double *S = o.S + (int64_t)z * o.strideS;
  const double nk = spec ? spec[(int64_t)z * 6 + 4] : 1.0;
  const double f = (scale_mode != 0 && nk > 0.0) ? S[j] / nk : 1.0;
  const double fu = sgn * (scale_mode == 2 ? f : 1.0);
  const double fv = sgn * (scale_mode == 1 ? f : 1.0);
  if (fu != 1.0)
    for (int i = tid; i < o.m; i += 256) U[(int64_t)i * o.k + j] = (T)((double)U[(int64_t)i * o.k + j] * fu);
  if (fv != 1.0)
    for (int c = tid; c < o.n; c += 256) Vt[(int64_t)j * o.n + c] = (T)((double)Vt[(int64_t)j * o.n + c] * fv);
}

// -------------------------------------------------------------- spectrum sums
__device__ inline double bsum256(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// spec[0] = Z = sum S^2, spec[1] = -sum p ln p
__global__ __launch_bounds__(256) void entropy_kernel(const double *S, int R, int64_t strideS, double *spec) {
  __shared__ double red[4];
  const int z = blockIdx.x;
  const double *s = S + (int64_t)z * strideS;
  double a = 0.0;
  for (int i = threadIdx.x; i < R; i += 256) a += s[i] * s[i];
  const double Z = bsum256(a, red);
  double e = 0.0;
  for (int i = threadIdx.x; i < R; i += 256) {
    const double p = s[i] * s[i] / Z;
    if (p > 0.0) e -= p * log(p);
  }
  const double ent = bsum256(e, red);
  if (threadIdx.x == 0) {
    spec[(int64_t)z * 6 + 0] = Z;
    spec[(int64_t)z * 6 + 1] = ent;
  }
}

// spec[2] = eps = sqrt(sum_{j>=k} S^2), spec[3] = eps^2/Z, spec[4] = |S_0..k-1|, spec[5] = gap
__global__ __launch_bounds__(256) void trunc_kernel(const double *S, int R, int k, int64_t strideS, double *spec) {
  __shared__ double red[4];
  const int z = blockIdx.x;
  const double *s = S + (int64_t)z * strideS;
  double t = 0.0, h = 0.0;
  for (int i = threadIdx.x; i < R; i += 256) {
    if (i >= k) t += s[i] * s[i];
    else h += s[i] * s[i];
  }
  const double tail = bsum256(t, red);
  const double head = bsum256(h, red);
  if (threadIdx.x == 0) {
    const double Z = spec[(int64_t)z * 6 + 0];
    spec[(int64_t)z * 6 + 2] = sqrt(tail);
    spec[(int64_t)z * 6 + 3] = tail / Z;
    spec[(int64_t)z * 6 + 4] = sqrt(head);
    spec[(int64_t)z * 6 + 5] = (k < R && s[0] > 0.0) ? (s[k - 1] - s[k]) / s[0] : 1.0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void load_rows_kernel(const T *A, int64_t strideA, double *bw, int64_t n) {
  const int z = blockIdx.y;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    bw[(int64_t)z * n + e] = (double)A[(int64_t)z * strideA + e];
}

template <typename T>
__global__ __launch_bounds__(256) void load_trans_kernel(const T *A, int64_t strideA, int m, int n, double *bw) {
  __shared__ double tile[32][33];
  const int z = blockIdx.z;
  const T *Az = A + (int64_t)z * strideA;
  double *B = bw + (int64_t)z * m * n;
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;
    tile[r][tx] = (i < m && j < n) ? (double)Az[(int64_t)i * n + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = bx + r, i = by + tx;
    if (j < n && i < m) B[(int64_t)j * m + i] = tile[tx][r];
  }
}

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace

// ====================================================================== host
tna_status svd_plan(int batch, int m, int n, int dtype, SvdPlan *p) {
  if (batch < 1 || m < 1 || n < 1) {
    set_error("svd: dimensions must be positive");
    return TNA_ERR_ARG;
  }
  p->batch = batch;
  p->m = m;
  p->n = n;
  p->trans = m > n;
  p->R = m < n ? m : n;
  p->C = m < n ? n : m;
  if (p->C > 4096) {
    set_error("svd: max(m,n) > 4096 is not supported");
    return TNA_ERR_UNSUPPORTED;
  }
  int nb = (p->R + BS - 1) / BS;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  p->nb = nb;
  const int npairs = nb / 2;
  int ks = ceil_div(1024, (int64_t)npairs * batch);
  const int kmax = ceil_div(p->C, 256);
  if (ks > kmax) ks = kmax;
  if (ks < 1) ks = 1;
  p->ksplit = ks;
  p->dtype = dtype;
  return TNA_OK;
}

static SvdDev make_dev(const SvdPlan &p, SvdBuffers &wb, double tol) {
  SvdDev d;
  d.R = p.R; d.C = p.C; d.nb = p.nb; d.ksplit = p.ksplit; d.step = 0;
  d.bw = wb.bw.as<double>(); d.jt = wb.jt.as<double>(); d.gram = wb.gram.as<double>();
  d.qt = wb.qt.as<double>(); d.skip = wb.flags.as<int>(); d.ctr = wb.ctr.as<int>();
  d.tol = tol;
  return d;
}

tna_status svd_run(const SvdPlan &p, SvdBuffers &wb, const void *A, int64_t strideA, int max_sweeps, int *sweeps,
                   hipStream_t s, int *host_ctr) {
  const int B = p.batch, npairs = p.nb / 2;
  TNA_TRY(wb.bw.ensure(sizeof(double) * (size_t)B * p.R * p.C));
  TNA_TRY(wb.jt.ensure(sizeof(double) * (size_t)B * p.R * p.R));
  TNA_TRY(wb.gram.ensure(sizeof(double) * (size_t)B * npairs * p.ksplit * 4096));
  TNA_TRY(wb.qt.ensure(sizeof(double) * (size_t)B * npairs * 4096));
  TNA_TRY(wb.flags.ensure(sizeof(int) * (size_t)B * npairs));
  TNA_TRY(wb.sig.ensure(sizeof(double) * (size_t)B * p.R));
  TNA_TRY(wb.perm.ensure(sizeof(int) * (size_t)B * p.R));
  TNA_TRY(wb.ctr.ensure(sizeof(int) * 4));
  // working rows
  const int64_t rc = (int64_t)p.R * p.C;
  if (!p.trans) {
    dim3 g((unsigned)std::min<int64_t>(ceil_div(rc, 256), 4096), B);
    if (p.dtype == TNA_F64)
      hipLaunchKernelGGL(load_rows_kernel<double>, g, dim3(256), 0, s, static_cast<const double *>(A), strideA,
                         wb.bw.as<double>(), rc);
    else
      hipLaunchKernelGGL(load_rows_kernel<float>, g, dim3(256), 0, s, static_cast<const float *>(A), strideA,
                         wb.bw.as<double>(), rc);
  } else {
    dim3 g(ceil_div(p.n, 32), ceil_div(p.m, 32), B);
    if (p.dtype == TNA_F64)
      hipLaunchKernelGGL(load_trans_kernel<double>, g, dim3(256), 0, s, static_cast<const double *>(A), strideA, p.m,
                         p.n, wb.bw.as<double>());
    else
      hipLaunchKernelGGL(load_trans_kernel<float>, g, dim3(256), 0, s, static_cast<const float *>(A), strideA, p.m,
                         p.n, wb.bw.as<double>());
  }
  TNA_LAUNCHED("svd.hip:1");
  TNA_TRY(set_identity(wb.jt.as<double>(), p.R, p.R, B, (int64_t)p.R * p.R, s));
  SvdDev d = make_dev(p, wb, (double)p.C * EPS53);
  const int ntile_b = ceil_div(p.C, 64), ntile_j = ceil_div(p.R, 64);
  // algorithmic work of one step: every row of B meets its partner block once
  // (Gram: 2 (2b)^2 C per pair), then [B;J] rows are rotated (2 (2b)^2 (C+R) per pair)
  const double pairs = (double)npairs * B, b2 = 64.0 * 64.0;
  const double gram_flops = 2.0 * b2 * p.C * pairs, gram_bytes = 8.0 * (double)p.R * p.C * B;
  const double eig_bytes = 8.0 * b2 * pairs * (p.ksplit + 1);
  const double apply_flops = 2.0 * b2 * (double)(p.C + p.R) * pairs;
  const double apply_bytes = 16.0 * ((double)p.R * p.C + (double)p.R * p.R) * B;
  int sw = 0;
  bool conv = false;
  for (sw = 1; sw <= max_sweeps; ++sw) {
    TNA_TRY(fill_int(wb.ctr.as<int>(), 1, 0, s));
    for (int step = 0; step < p.nb - 1; ++step) {
      d.step = step;
      timer_begin("svd.gram", s);
      hipLaunchKernelGGL(gram_kernel, dim3(npairs, p.ksplit, B), dim3(256), 0, s, d);
      timer_end("svd.gram", gram_flops, gram_bytes, s);
      timer_begin("svd.eigen", s);
      hipLaunchKernelGGL(eigen_kernel, dim3(npairs, B), dim3(256), 0, s, d);
      timer_end("svd.eigen", 0.0, eig_bytes, s);
      timer_begin("svd.apply", s);
      hipLaunchKernelGGL(apply_kernel, dim3(npairs, ntile_b + ntile_j, B), dim3(256), 0, s, d, ntile_b);
      timer_end("svd.apply", apply_flops, apply_bytes, s);
    }
    TNA_LAUNCHED("svd.hip:2");
    TNA_HIP(hipMemcpyAsync(host_ctr, wb.ctr.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    TNA_HIP(hipStreamSynchronize(s));
    if (*host_ctr == 0) {
      conv = true;
      break;
    }
  }
  if (sweeps) *sweeps = conv ? sw : max_sweeps;
  hipLaunchKernelGGL(norms_kernel, dim3(ceil_div(p.R, 4), B), dim3(256), 0, s, wb.bw.as<double>(), p.R, p.C,
                     wb.sig.as<double>());
  TNA_LAUNCHED("svd.hip:3");
  if (!conv) {
    set_error("svd: Jacobi sweep cap reached");
    return TNA_ERR_NOCONV;
  }
  return TNA_OK;
}

tna_status svd_spectrum(const SvdPlan &p, SvdBuffers &wb, double *S_out, int64_t strideS, double *spec,
                        hipStream_t s) {
  int P = 1;
  while (P < p.R) P <<= 1;
  hipLaunchKernelGGL(sort_kernel, dim3(p.batch), dim3(1024), 0, s, wb.sig.as<double>(), p.R, P, wb.perm.as<int>(),
                     S_out, strideS);
  hipLaunchKernelGGL(entropy_kernel, dim3(p.batch), dim3(256), 0, s, S_out, p.R, strideS, spec);
  TNA_LAUNCHED("svd.hip:4");
  return TNA_OK;
}

tna_status svd_trunc_S(const SvdPlan &p, const double *S, int64_t strideS, int k, double *spec, hipStream_t s) {
  hipLaunchKernelGGL(trunc_kernel, dim3(p.batch), dim3(256), 0, s, S, p.R, k, strideS, spec);
  TNA_LAUNCHED("svd.hip:5");
  return TNA_OK;
}

tna_status svd_outputs_S(const SvdPlan &p, SvdBuffers &wb, const double *S, int64_t strideS, int k, void *U,
                         int64_t strideU, void *Vt, int64_t strideVt, int out_type, int scale_mode,
                         const double *spec, hipStream_t s) {
  OutDev o;
  o.R = p.R; o.C = p.C; o.m = p.m; o.n = p.n; o.k = k; o.trans = p.trans;
  o.bw = wb.bw.as<double>(); o.jt = wb.jt.as<double>(); o.S = S; o.strideS = strideS;
  o.perm = wb.perm.as<int>(); o.U = U; o.strideU = strideU; o.Vt = Vt; o.strideVt = strideVt;
  const int B = p.batch;
  dim3 gu((unsigned)std::min<int64_t>(ceil_div((int64_t)p.m * k, 256), 4096), B);
  dim3 gv((unsigned)std::min<int64_t>(ceil_div((int64_t)k * p.n, 256), 4096), B);
  if (out_type == TNA_F64) {
    hipLaunchKernelGGL(write_u_kernel<double>, gu, dim3(256), 0, s, o);
    hipLaunchKernelGGL(write_vt_kernel<double>, gv, dim3(256), 0, s, o);
    hipLaunchKernelGGL(complete_kernel<double>, dim3(B), dim3(256), 0, s, o);
    hipLaunchKernelGGL(gauge_kernel<double>, dim3(k, B), dim3(256), 0, s, o, scale_mode, spec);
  } else {
    hipLaunchKernelGGL(write_u_kernel<float>, gu, dim3(256), 0, s, o);
    hipLaunchKernelGGL(write_vt_kernel<float>, gv, dim3(256), 0, s, o);
    hipLaunchKernelGGL(complete_kernel<float>, dim3(B), dim3(256), 0, s, o);
    hipLaunchKernelGGL(gauge_kernel<float>, dim3(k, B), dim3(256), 0, s, o, scale_mode, spec);
  }
  TNA_LAUNCHED("svd.hip:6");
  return TNA_OK;
}

tna_status spectrum_entropy(const double *S, int R, double *spec, int batch, int64_t strideS, hipStream_t s) {
  hipLaunchKernelGGL(entropy_kernel, dim3(batch), dim3(256), 0, s, S, R, strideS, spec);
  TNA_LAUNCHED("svd.hip:7");
  return TNA_OK;
}

tna_status spectrum_trunc(const double *S, int R, int k, double *spec, int batch, int64_t strideS, hipStream_t s) {
  hipLaunchKernelGGL(trunc_kernel, dim3(batch), dim3(256), 0, s, S, R, k, strideS, spec);
  TNA_LAUNCHED("svd.hip:8");
  return TNA_OK;
}

}  // namespace tna
