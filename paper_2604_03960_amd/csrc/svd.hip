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
#include <hip/hip_cooperative_groups.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "dev_reduce.h"
#include "internal.h"

namespace tna {

tna_status DevBuf::ensure(size_t need) {
  if (need <= bytes) return TNA_OK;
  if (borrowed) {
    set_error("workspace too small for this call");
    return TNA_ERR_NOMEM;
  }
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
  if (ptr && !borrowed) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
  borrowed = false;
}

namespace {

// Jacobi rotation zeroing the off-diagonal g of a symmetric 2 x 2 block [[a, g], [g, b]] (g != 0):
// t = sign(b - a) 2 g / (|b - a| + sqrt((b - a)^2 + 4 g^2)), c = 1 / sqrt(1 + t^2), s = c t.  The
// square roots and the quotient come from the hardware reciprocal and reciprocal-square-root
// estimates refined by two Newton steps each (the relative error squares per step), which keeps
// c^2 + s^2 = 1 to a few ulp while avoiding the long correctly rounded division and square-root
// sequences.
__device__ inline double rsqrt_nr(double x) {  // x > 0, finite
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
__device__ inline double rcp_nr(double x) {  // x > 0, finite
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ inline void jacobi_rot(double a, double b, double g, double &c, double &s) {
  const double dl = b - a, q = fma(dl, dl, 4.0 * g * g);
  const double t = (dl >= 0.0 ? 2.0 : -2.0) * g * rcp_nr(fabs(dl) + q * rsqrt_nr(q));
  c = rsqrt_nr(fma(t, t, 1.0));
  s = c * t;
}

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

__device__ inline double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double bsum256(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// -------------------------------------------------------------- gram
// 64 x 64 Gram of the rows of blocks p and q over columns [kb, ke) on MFMA:
// wave (qi, qj) holds the 32 x 32 quadrant (qi, qj) as 2 x 2 16 x 16 tiles.
constexpr int GBK = 64;
// The next 64-column slab (32 KB of the pair's rows) is loaded into registers while the current
// one is multiplied.
__device__ inline void gram_acc(const SvdMat &a, int p, int q, int np, int nq, int64_t kb, int64_t ke,
                                double (*Ts)[65], v4d acc[2][2]) {
  constexpr int RS = 256 / GBK, NU = 64 / RS;  // row stride of a thread's loads, rows per thread
  const double *B = a.bw;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int qi = wave >> 1, qj = wave & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0, 0, 0, 0};
  // thread tid loads column tid % GBK of rows tid / GBK + RS u, u < NU
  const int col = tid % GBK, r0 = tid / GBK;
  const double *rowp[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int r = r0 + RS * u;
    const bool valid = r < 32 ? (r < np) : (r - 32 < nq);
    const int grow = r < 32 ? p * BS + r : q * BS + (r - 32);
    rowp[u] = valid ? B + (int64_t)grow * a.C : nullptr;
  }
  double nx[NU];
  auto load = [&](int64_t k0) {
    const int64_t gc = k0 + col;
#pragma unroll
    for (int u = 0; u < NU; ++u) nx[u] = (rowp[u] && gc < ke) ? rowp[u][gc] : 0.0;
  };
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += GBK) {
#pragma unroll
    for (int u = 0; u < NU; ++u) Ts[col][r0 + RS * u] = nx[u];
    __syncthreads();
    if (k0 + GBK < ke) load(k0 + GBK);  // in flight during the products below
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 4) {
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
}

// G[row * 64 + col] = acc (f64 result layout)
__device__ inline void gram_store(const v4d acc[2][2], double *G, int ldg) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int qi = wave >> 1, qj = wave & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 32 * qi + 16 * i + 4 * r + lk, col = 32 * qj + 16 * j + lr;
        G[row * ldg + col] = acc[i][j][r];
      }
}

// grid (pairs, ksplit, matrices)
__global__ __launch_bounds__(256) void gram_kernel(const SvdMat *mats, int step) {
  __shared__ double Ts[GBK][64 + 1];
  const SvdMat &a = mats[blockIdx.z];
  const int pair = blockIdx.x, ks = blockIdx.y;
  if (!a.active || a.fused || step >= a.nb - 1 || pair >= a.nb / 2 || ks >= a.ksplit) return;
  int p, q;
  rr_pair(a.nb, step, pair, p, q);
  const int np = block_rows(a.Ra, p), nq = block_rows(a.Ra, q);
  int64_t chunk = (a.C + a.ksplit - 1) / a.ksplit;
  chunk = (chunk + GBK - 1) / GBK * GBK;
  const int64_t kb = chunk * ks;
  const int64_t ke = kb + chunk < a.C ? kb + chunk : a.C;
  v4d acc[2][2];
  gram_acc(a, p, q, np, nq, kb, ke, Ts, acc);
  gram_store(acc, a.gram + ((int64_t)pair * a.ksplit + ks) * 4096, 64);
}

// -------------------------------------------------------------- eigen
// Two-sided cyclic Jacobi on the 64 x 64 Gram of a block pair, in LDS.
struct EigLds {
  double G[64][65];
  double Q[64][65];
  double cs[32], sn[32];
  int pi[32], pj[32];
  int rot_any, need;
  int slot_of[64];
  int vs[64];                   // valid slots in order
  unsigned short sched[63][32]; // round-robin pairs (i | j << 8) of one sweep
  unsigned short pcol[63][64];  // per round and column: partner | pair << 6 | (first of its pair) << 11
  double rc[63][32], rs[63][32];  // the rotations of one inner sweep, applied to Q after it
};

// Rows whose squared norm is at or below row_floor2 = (0.1 eps C)^2 |A|_F^2 are at the
// rounding level of the rotations: their directions are noise, so pairs with such a
// row are neither tested nor rotated (the relative test could never settle on them).
// Skipping a coupling g_ij <= sigma_i sigma_floor moves sigma_i by at most
// sigma_floor^2 / sigma_i; kept vectors below the floor are completed afterwards.
// After the QR start such rows do settle under the relative test, but only after many
// more sweeps (a numerically low-rank matrix can need twice as many), so the floor is
// used there only when the factor built from the rows leaves scaled by the singular
// values (rows_scaled): then nothing needs their directions.  An input that carries
// noise of noise_rel |A|_F (rows_scaled only) raises the floor to that level.
__device__ inline double row_floor2(const SvdMat &a, double fro2) {
  if (a.precond && !a.rows_scaled) return 0.0;
  const double f = fmax(0.1 * EPS53 * (double)a.C, a.rows_scaled ? a.noise_rel : 0.0);
  return f * f * fro2;
}

// Outer test: does any pair of rows above the floor fail |g_ij| <= tol sqrt(g_ii g_jj)?
template <int NTE>
__device__ inline bool eig_needs_rotation(EigLds &L, double tol, double floor2) {
  const int tid = threadIdx.x;
  if (tid == 0) L.need = 0;
  __syncthreads();
  int loc = 0;
  for (int e = tid; e < 4096; e += NTE) {
    const int i = e >> 6, j = e & 63;
    if (i < j) {
      const double gii = L.G[i][i], gjj = L.G[j][j], gij = L.G[i][j];
      if (gii > floor2 && gjj > floor2 && gii > 0.0 && gjj > 0.0 && fabs(gij) > tol * sqrt(gii * gjj)) loc = 1;
    }
  }
  if (__any(loc) && (tid & 63) == 0) atomicOr(&L.need, 1);
  __syncthreads();
  return L.need != 0;
}

// Q <- Q J_1 ... J_nr for the rotations logged over one inner sweep: each wave holds 64 / waves rows
// of Q in registers, lane l column l; a rotation on columns (i, j) takes Q[k][i] <- c Q[k][i] - s Q[k][j]
// and Q[k][j] <- s Q[k][i] + c Q[k][j], the partner's value arriving by a lane shuffle.
template <int NTE>
__device__ inline void eig_apply_log(EigLds &L, int nr) {
  constexpr int RPW = 64 / (NTE / 64);  // rows per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double q[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) q[r] = L.Q[wave * RPW + r][lane];
  for (int rr = 0; rr < nr; ++rr) {
    const unsigned pc = L.pcol[rr][lane];
    const int partner = pc & 63, t = (pc >> 6) & 31;
    const bool first = (pc >> 11) & 1;
    const double c = L.rc[rr][t], sn = partner == lane ? 0.0 : L.rs[rr][t];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const double pv = __shfl(q[r], partner, 64);
      if (sn != 0.0) q[r] = first ? c * q[r] - sn * pv : sn * pv + c * q[r];
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) L.Q[wave * RPW + r][lane] = q[r];
  __syncthreads();
}

// Q <- Q J over sweeps of a round-robin ordering of the nv valid slots (np of block p at
// 0.., nq of block q at 32..) until a sweep rotates nothing (or inner_max sweeps); the
// diagonal of G ends as the eigenvalues.  With nv odd a dummy index sits out each round.
// The slot pairs of every round are tabulated in LDS once per call.
template <int NTE>
__device__ inline void eig_inner(EigLds &L, int inner_max, double floor2, int np, int nq) {
  const int tid = threadIdx.x;
  const int nv = np + nq, nvp = nv + (nv & 1), P = nvp / 2;
  if (tid < 64) L.vs[tid] = tid < np ? tid : 32 + (tid - np);  // entries >= nv unused
  __syncthreads();
  // pair table: (i, j) with i <= j; a pair with the dummy becomes (x, x) and rotates nothing,
  // but its row still takes the partner pairs' column rotations
  for (int e = tid; e < (nvp - 1) * P; e += NTE) {
    const int rr = e / P, t = e - rr * P;
    int ia, ib;
    if (t == 0) { ia = rr % (nvp - 1); ib = nvp - 1; }
    else { ia = (rr + t) % (nvp - 1); ib = (rr - t + nvp - 1) % (nvp - 1); }
    int i = ia < nv ? L.vs[ia] : -1, j = ib < nv ? L.vs[ib] : -1;
    if (i < 0) i = j;
    if (j < 0) j = i;
    L.sched[rr][t] = (unsigned short)((i < j ? i : j) | ((i < j ? j : i) << 8));
  }
  // column view of the same table (columns outside the valid slots are their own partner)
  for (int e = tid; e < (nvp - 1) * 64; e += NTE) L.pcol[e >> 6][e & 63] = (unsigned short)(e & 63);
  __syncthreads();
  for (int e = tid; e < (nvp - 1) * P; e += NTE) {
    const int rr = e / P, t = e - rr * P;
    const unsigned pr = L.sched[rr][t];
    const int i = pr & 0xff, j = pr >> 8;
    if (i != j) {
      L.pcol[rr][i] = (unsigned short)(j | (t << 6) | (1 << 11));
      L.pcol[rr][j] = (unsigned short)(i | (t << 6));
    }
  }
  const double tol_in = 4.0 * EPS53;
  for (int sweep = 0; sweep < inner_max; ++sweep) {
    __syncthreads();  // every thread has read rot_any of the previous sweep (and the table is set)
    if (tid == 0) L.rot_any = 0;
    __syncthreads();
    for (int rr = 0; rr < nvp - 1; ++rr) {
      // rotation J = [[c, s], [-s, c]] on (i, j), i < j, zeroing g_ij:
      // t = sign(d) 2 g_ij / (|d| + sqrt(d^2 + 4 g_ij^2)), d = g_jj - g_ii; c = 1 / sqrt(1 + t^2)
      if (tid < P) {
        const unsigned pr = L.sched[rr][tid];
        const int i = pr & 0xff, j = pr >> 8;
        double c = 1.0, s = 0.0;
        if (i != j) {
          const double gii = L.G[i][i], gjj = L.G[j][j], gij = L.G[i][j];
          if (gii > floor2 && gjj > floor2 && gij * gij > tol_in * tol_in * fabs(gii * gjj)) {
            jacobi_rot(gii, gjj, gij, c, s);
            L.rot_any = 1;
          }
        }
        L.cs[tid] = c; L.sn[tid] = s; L.pi[tid] = i; L.pj[tid] = j;
        L.rc[rr][tid] = c; L.rs[rr][tid] = s;
      }
      __syncthreads();
      // G <- J^T G J one 2 x 2 block (pair t rows, pair u columns) at a time, t <= u, and
      // the mirror block written from the same values so G stays exactly symmetric.  For
      // even P, rows t and P - 1 - t of the block triangle go together (P + 1 blocks per
      // row pair); for odd P the square is walked and its lower half skipped.
      const int nblk = (P & 1) ? P * P : (P / 2) * (P + 1);
      for (int e = tid; e < nblk; e += NTE) {
        int t, u;
        if (P & 1) {
          t = e / P;
          u = e - t * P;
          if (u < t) continue;
        } else {
          const int rp = e / (P + 1), off = e - rp * (P + 1);
          if (off < P - rp) { t = rp; u = rp + off; }
          else { t = P - 1 - rp; u = t + (off - (P - rp)); }
        }
        const double st = L.sn[t], su = L.sn[u];
        if (st == 0.0 && su == 0.0) continue;
        const double ct = L.cs[t], cu = L.cs[u];
        const int a0 = L.pi[t], a1 = L.pj[t], b0 = L.pi[u], b1 = L.pj[u];
        const double x00 = L.G[a0][b0], x01 = L.G[a0][b1], x10 = L.G[a1][b0], x11 = L.G[a1][b1];
        const double y00 = ct * x00 - st * x10, y01 = ct * x01 - st * x11;
        const double y10 = st * x00 + ct * x10, y11 = st * x01 + ct * x11;
        const double z00 = cu * y00 - su * y01, z01 = su * y00 + cu * y01;
        const double z10 = cu * y10 - su * y11, z11 = su * y10 + cu * y11;
        if (t == u) {
          L.G[a0][a0] = z00; L.G[a1][a1] = z11; L.G[a0][a1] = 0.0; L.G[a1][a0] = 0.0;
        } else {
          // a dummy pair has a0 == a1 (identity rotation): both writes carry the same value
          L.G[a0][b0] = z00; L.G[a0][b1] = z01; L.G[a1][b0] = z10; L.G[a1][b1] = z11;
          L.G[b0][a0] = z00; L.G[b1][a0] = z01; L.G[b0][a1] = z10; L.G[b1][a1] = z11;
        }
      }
      __syncthreads();
    }
    eig_apply_log<NTE>(L, nvp - 1);
    const int any = L.rot_any;
    if (!any) break;
  }
}

// slot_of[so] = eigen-slot whose vector becomes output row so: eigenvalues descending
// (ties: lower slot first), the np largest to block p, the rest to block q
__device__ inline void eig_order(EigLds &L, int np, int nq) {
  const int r = threadIdx.x;
  if (r < 64) {
    const bool vr = r < 32 ? (r < np) : (r - 32 < nq);
    if (vr) {
      const double lr_ = L.G[r][r];
      int rank = 0;
      for (int o = 0; o < 64; ++o) {
        const bool vo = o < 32 ? (o < np) : (o - 32 < nq);
        if (o == r || !vo) continue;
        const double lo = L.G[o][o];
        if (lo > lr_ || (lo == lr_ && o < r)) ++rank;
      }
      L.slot_of[rank < np ? rank : 32 + (rank - np)] = r;
    }
  }
  __syncthreads();
}

// ---- the eigen step of the blocked method: a tournament on moving slots
// The elements of the 64 x 64 Gram move between slots so that the pairs of every round are the
// slot pairs (2t, 2t+1): each round reads its 2 x 2 blocks as contiguous 16-byte pairs, rotates,
// and writes them to the slots of the next round in a second buffer (one barrier for the
// rotations, one for the round).  The move is the circle method on 64 slots with slot 0 fixed:
// every other element advances one place along 1 -> 2 -> 4 -> ... -> 62 -> 63 -> 61 -> ... -> 3
// -> 1, which brings every pair of elements together once in 63 rounds and restores the starting
// placement after the 63rd.  The eigenvector columns move with their elements, in registers.
__device__ inline int tour_next(int s) {
  if (s == 0) return 0;
  if (s == 1) return 2;
  if (s == 62) return 63;
  return (s & 1) ? s - 2 : s + 2;
}
__device__ inline int tour_prev(int m) {
  if (m == 0) return 0;
  if (m == 2) return 1;
  if (m == 63) return 62;
  return (m & 1) ? m + 2 : m - 2;
}

struct EigTour {
  double G[2][64][66];  // the matrix of the current round and of the next (rows 16-byte aligned)
  double cs[32], sn[32];
  int rot_any, need;
  int slot_of[64];
  int rank[64];
};

// Outer test on G[0] (rows above the floor only), as eig_needs_rotation
template <int NTE>
__device__ inline bool tour_needs_rotation(EigTour &L, double tol, double floor2) {
  const int tid = threadIdx.x;
  if (tid == 0) L.need = 0;
  __syncthreads();
  // the test squared (no square root on the path): g_ij^2 > tol^2 g_ii g_jj
  const double tol2 = tol * tol;
  int loc = 0;
#pragma unroll
  for (int m = 0; m < 4096 / NTE; ++m) {
    const int e = tid + m * NTE, i = e >> 6, j = e & 63;
    if (i < j) {
      const double gii = L.G[0][i][i], gjj = L.G[0][j][j], gij = L.G[0][i][j];
      if (gii > floor2 && gjj > floor2 && gii > 0.0 && gjj > 0.0 && gij * gij > tol2 * (gii * gjj)) loc = 1;
    }
  }
  if (__any(loc) && (tid & 63) == 0) atomicOr(&L.need, 1);
  __syncthreads();
  return L.need != 0;
}

// Sweeps of 63 rounds until one rotates nothing (or inner_max).  Returns the buffer holding the
// rotated matrix (eigenvalues on its diagonal, every element back on its starting slot); the
// eigenvector matrix Q (column s for slot s) is left in the other buffer.  Rotation and tests as
// in eig_inner; the 2 x 2 block (t, u) and its mirror (u, t) are computed by the same operations
// on the same values, so the matrix stays exactly symmetric.
template <int NTE>
__device__ inline int eig_tour(EigTour &L, int inner_max, double floor2) {
  constexpr int RPW = 64 / (NTE / 64);  // rows of Q per wave
  constexpr int BPT = 1024 / NTE;       // 2 x 2 blocks per thread
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double q[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) q[r] = (wave * RPW + r == lane) ? 1.0 : 0.0;
  const double tol_in = 4.0 * EPS53;
  const int qsrc = tour_prev(lane), qpair = lane >> 1;
  int cur = 0;
  for (int sweep = 0; sweep < inner_max; ++sweep) {
    __syncthreads();  // every thread has read rot_any of the previous sweep
    if (tid == 0) L.rot_any = 0;
    __syncthreads();
    for (int rr = 0; rr < 63; ++rr) {
      double (*Gi)[66] = L.G[cur];
      double (*Go)[66] = L.G[cur ^ 1];
      double x[BPT][4];
#pragma unroll
      for (int b = 0; b < BPT; ++b) {  // Gi does not change during the round: read before the rotations
        const int e = tid + b * NTE, t = e >> 5, u = e & 31;
        const double2 r0 = *reinterpret_cast<const double2 *>(&Gi[2 * t][2 * u]);
        const double2 r1 = *reinterpret_cast<const double2 *>(&Gi[2 * t + 1][2 * u]);
        x[b][0] = r0.x;
        x[b][1] = r0.y;
        x[b][2] = r1.x;
        x[b][3] = r1.y;
      }
      if (tid < 32) {
        // J = [[c, s], [-s, c]] on the slots (2t, 2t+1), zeroing their coupling
        const int t = tid;
        const double a = Gi[2 * t][2 * t], bb = Gi[2 * t + 1][2 * t + 1], g = Gi[2 * t][2 * t + 1];
        double c = 1.0, sn = 0.0;
        if (a > floor2 && bb > floor2 && g * g > tol_in * tol_in * fabs(a * bb)) {
          jacobi_rot(a, bb, g, c, sn);
          L.rot_any = 1;
        }
        L.cs[t] = c;
        L.sn[t] = sn;
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const int e = tid + b * NTE, t = e >> 5, u = e & 31;
        const bool up = t <= u;  // Z = J_lo^T X(lo, hi) J_hi, lo = min(t, u)
        const int lo = up ? t : u, hi = up ? u : t;
        const double cl = L.cs[lo], sl = L.sn[lo], ch = L.cs[hi], sh = L.sn[hi];
        const double x00 = x[b][0], x01 = up ? x[b][1] : x[b][2], x10 = up ? x[b][2] : x[b][1], x11 = x[b][3];
        const double y00 = cl * x00 - sl * x10, y01 = cl * x01 - sl * x11;
        const double y10 = sl * x00 + cl * x10, y11 = sl * x01 + cl * x11;
        double z00 = ch * y00 - sh * y01, z01 = sh * y00 + ch * y01;
        double z10 = ch * y10 - sh * y11, z11 = sh * y10 + ch * y11;
        if (t == u && sl != 0.0) {
          z01 = 0.0;
          z10 = 0.0;
        }
        const int r0 = tour_next(2 * t), r1 = tour_next(2 * t + 1);
        const int c0 = tour_next(2 * u), c1 = tour_next(2 * u + 1);
        Go[r0][c0] = z00;
        Go[r0][c1] = up ? z01 : z10;
        Go[r1][c0] = up ? z10 : z01;
        Go[r1][c1] = z11;
      }
      {  // Q <- Q J on the lane's column, then the column moves with its element
        const double c = L.cs[qpair], sn = L.sn[qpair];
        const bool first = (lane & 1) == 0;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          const double pv = dpp_d<0xB1, 0xf>(q[r]);  // the pair partner's value (quad_perm [1,0,3,2])
          const double nv = first ? c * q[r] - sn * pv : sn * pv + c * q[r];
          q[r] = __shfl(nv, qsrc, 64);
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    const int any = L.rot_any;
    if (!any) break;
  }
  double (*Qb)[66] = L.G[cur ^ 1];
#pragma unroll
  for (int r = 0; r < RPW; ++r) Qb[wave * RPW + r][lane] = q[r];
  __syncthreads();
  return cur;
}

// slot_of as eig_order, from the diagonal of G: the rank of slot r (eigenvalues descending, ties
// by slot) counted by NTE / 64 thread groups over slices of the other slots
template <int NTE>
__device__ inline void tour_order(const double (*G)[66], int *slot_of, int *rank, int np, int nq) {
  constexpr int NG = NTE / 64, PER = 64 / NG;
  const int r = threadIdx.x & 63, grp = threadIdx.x >> 6;
  auto valid = [&](int x) { return x < 32 ? (x < np) : (x - 32 < nq); };
  if (threadIdx.x < 64) rank[r] = 0;
  __syncthreads();
  if (valid(r)) {
    const double lr_ = G[r][r];
    int cnt = 0;
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int o = grp * PER + m;
      if (o != r && valid(o)) {
        const double lo = G[o][o];
        cnt += (lo > lr_ || (lo == lr_ && o < r)) ? 1 : 0;
      }
    }
    if (cnt) atomicAdd(&rank[r], cnt);
  }
  __syncthreads();
  if (threadIdx.x < 64 && valid(r)) {
    const int k = rank[r];
    slot_of[k < np ? k : 32 + (k - np)] = r;
  }
  __syncthreads();
}

// grid (pairs, matrices)
constexpr int EIG_NT = 512;
constexpr int KS_MAX = 16;  // K splits of the Gram: at most ceil(4096 / 256)
__global__ __launch_bounds__(EIG_NT) void eigen_kernel(const SvdMat *mats, int step) {
  __shared__ EigTour L;
  const SvdMat &a = mats[blockIdx.y];
  const int pair = blockIdx.x;
  if (!a.active || a.fused || step >= a.nb - 1 || pair >= a.nb / 2) return;
  const int tid = threadIdx.x;
  int p, q;
  rr_pair(a.nb, step, pair, p, q);
  const int np = block_rows(a.Ra, p), nq = block_rows(a.Ra, q);
  int *skip = a.skip + pair;
  if (np + nq == 0) {
    if (tid == 0) *skip = 1;
    return;
  }
  auto valid = [&](int r) { return r < 32 ? (r < np) : (r - 32 < nq); };
  // the K-split partial Grams (at most KS_MAX), summed in split order; only the upper triangle
  // is read (rows along the lanes, so every load is one contiguous segment) and mirrored, and
  // all partials of a thread's elements are loaded before the first sum
  const double *Gp = a.gram + (int64_t)pair * a.ksplit * 4096;
  const int nks = a.ksplit;
  constexpr int EPP = 4;  // elements per thread and pass: EPP x KS_MAX loads in flight
  for (int e0 = tid; e0 < 4096; e0 += EPP * EIG_NT) {
    double part[EPP][KS_MAX];
#pragma unroll
    for (int h = 0; h < EPP; ++h) {
      const int e = e0 + h * EIG_NT, i = e >> 6, j = e & 63;
#pragma unroll
      for (int ks = 0; ks < KS_MAX; ++ks) part[h][ks] = (ks < nks && i <= j) ? Gp[(int64_t)ks * 4096 + e] : 0.0;
    }
#pragma unroll
    for (int h = 0; h < EPP; ++h) {
      const int e = e0 + h * EIG_NT, i = e >> 6, j = e & 63;
      if (i > j) continue;
      double v = 0.0;
#pragma unroll
      for (int ks = 0; ks < KS_MAX; ++ks)
        if (ks < nks) v += part[h][ks];
      v = (valid(i) && valid(j)) ? v : 0.0;
      L.G[0][i][j] = v;
      L.G[0][j][i] = v;
    }
  }
  const double floor2 = row_floor2(a, *a.fro2);
  if (!tour_needs_rotation<EIG_NT>(L, a.tol, floor2)) {
    if (tid == 0) *skip = 1;
    return;
  }
  if (tid == 0) atomicAdd(a.ctr, 1);
  const int cur = eig_tour<EIG_NT>(L, a.inner_max, floor2);
  tour_order<EIG_NT>(L.G[cur], L.slot_of, L.rank, np, nq);
  const double(*Q)[66] = L.G[cur ^ 1];
  double *Qt = a.qt + (int64_t)pair * 4096;
  for (int e = tid; e < 4096; e += EIG_NT) {
    const int so = e >> 6, ri = e & 63;
    Qt[e] = (valid(so) && valid(ri)) ? Q[ri][L.slot_of[so]] : 0.0;
  }
  if (tid == 0) *skip = 0;
}

// -------------------------------------------------------------- apply
// rows of X (valid slots, row grow(slot)) columns [c0, c0 + 64) <- Qt X, with
// As[k][i] = Qt[i][k] in LDS; Xs is the staging tile
template <class Valid, class Grow>
__device__ inline void apply_tile(double *X, int ld, int c0, double (*As)[65], double (*Xs)[65], Valid valid,
                                  Grow grow) {
  const int tid = threadIdx.x;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e >> 6, k = e & 63;
    Xs[i][k] = (valid(i) && c0 + k < ld) ? X[(int64_t)grow(i) * ld + c0 + k] : 0.0;
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

// grid (pairs, groups of APPLY_TPW column tiles of B then of Jt, matrices).  Each wave
// keeps its 16 rows of the pair's rotation Qt as MFMA A-operands in registers (read once);
// the 64 x 64 tile of X passes through LDS, and the next tile of the group is loaded into
// registers while the current one is multiplied and written back, so one workgroup keeps
// a tile's loads in flight at all times.  33 KB of LDS: four workgroups per CU.
constexpr int APPLY_TPW = 4;
__global__ __launch_bounds__(256) void apply_kernel(const SvdMat *mats, int step) {
  __shared__ double Xs[64][65];  // Xs[k][j] = X[row(k)][c0 + j]
  const SvdMat &a = mats[blockIdx.z];
  const int pair = blockIdx.x;
  const int ntile_b = (a.C + 63) / 64, ntile_j = (a.R + 63) / 64;
  const int t0 = blockIdx.y * APPLY_TPW;
  if (!a.active || a.fused || step >= a.nb - 1 || pair >= a.nb / 2 || t0 >= ntile_b + ntile_j) return;
  if (a.skip[pair]) return;
  int p, q;
  rr_pair(a.nb, step, pair, p, q);
  const int np = block_rows(a.Ra, p), nq = block_rows(a.Ra, q);
  auto valid = [&](int r) { return r < 32 ? (r < np) : (r - 32 < nq); };
  auto grow = [&](int r) { return r < 32 ? p * BS + r : q * BS + (r - 32); };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // A(i, k) = Qt[i][k] for the wave's output rows i = 16 wave + lr, k = 4 kk + lk
  const double *Qt = a.qt + (int64_t)pair * 4096 + (16 * wave + lr) * 64 + lk;
  double aq[16];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) aq[kk] = Qt[4 * kk];
  const int t1 = t0 + APPLY_TPW < ntile_b + ntile_j ? t0 + APPLY_TPW : ntile_b + ntile_j;
  // thread tid loads rows (tid >> 6) + 4u, u < 16, at column tid & 63 of a tile
  const int lrow = tid >> 6, lcol = tid & 63;
  auto tile_of = [&](int tile, double *&X, int &ld, int &c0) {
    if (tile < ntile_b) { X = a.bw; ld = a.C; c0 = tile * 64; }
    else { X = a.jt; ld = a.R; c0 = (tile - ntile_b) * 64; }
  };
  double nx[16];
  auto load = [&](int tile) {
    double *X;
    int ld, c0;
    tile_of(tile, X, ld, c0);
    const bool colok = c0 + lcol < ld;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = lrow + 4 * u;
      nx[u] = (colok && valid(k)) ? X[(int64_t)grow(k) * ld + c0 + lcol] : 0.0;
    }
  };
  load(t0);
  for (int tile = t0; tile < t1; ++tile) {
    __syncthreads();  // the previous tile's products have read Xs
#pragma unroll
    for (int u = 0; u < 16; ++u) Xs[lrow + 4 * u][lcol] = nx[u];
    __syncthreads();
    if (tile + 1 < t1) load(tile + 1);  // in flight during the products below
    v4d acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = v4d{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = mfma16(aq[kk], Xs[4 * kk + lk][16 * t + lr], acc[t]);
    double *X;
    int ld, c0;
    tile_of(tile, X, ld, c0);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int so = 16 * wave + 4 * r + lk, col = 16 * t + lr;  // f64 result layout
        if (valid(so) && c0 + col < ld) X[(int64_t)grow(so) * ld + c0 + col] = acc[t][r];
      }
  }
}

// -------------------------------------------------------------- whole Jacobi, one workgroup
// Matrices with at most 64 rows to orthogonalise (one block pair) run every
// sweep inside one workgroup: Gram on MFMA into LDS, the outer test, the inner
// Jacobi, then the rotation of B and Jt, until a sweep needs no rotation.
// ctr[0] = 0 when converged (1 otherwise), ctr[1] = sweeps.  grid (matrices)
__global__ __launch_bounds__(256) void jacobi_fused_kernel(const SvdMat *mats, int max_sweeps) {
  __shared__ EigLds L;
  __shared__ double Xs[64][65];  // Gram staging, then apply tiles
  const SvdMat &a = mats[blockIdx.x];
  if (!a.active || a.fused != 1) return;
  const int tid = threadIdx.x;
  const int np = block_rows(a.R, 0), nq = block_rows(a.R, 1);
  auto valid = [&](int r) { return r < 32 ? (r < np) : (r - 32 < nq); };
  auto grow = [](int r) { return r; };  // blocks 0 and 1: slot r is row r
  const double floor2 = row_floor2(a, *a.fro2);
  int sw = 0, conv = 0;
  while (sw < max_sweeps) {
    ++sw;
    v4d acc[2][2];
    gram_acc(a, 0, 1, np, nq, 0, a.C, reinterpret_cast<double (*)[65]>(&Xs[0][0]), acc);
    gram_store(acc, &L.Q[0][0], 65);  // raw Gram, then the symmetric copy below
    __syncthreads();
    for (int e = tid; e < 4096; e += 256) {
      const int i = e >> 6, j = e & 63;
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      L.G[i][j] = (valid(i) && valid(j)) ? L.Q[lo][hi] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < 4096; e += 256) L.Q[e >> 6][e & 63] = ((e >> 6) == (e & 63)) ? 1.0 : 0.0;
    if (!eig_needs_rotation<256>(L, a.tol, floor2)) {
      conv = 1;
      break;
    }
    eig_inner<256>(L, a.inner_max, floor2, np, nq);
    eig_order(L, np, nq);
    // As[k][i] = Qt[i][k] = Q[k][slot_of[i]], written over G
    for (int e = tid; e < 4096; e += 256) {
      const int k = e >> 6, i = e & 63;
      L.G[k][i] = (valid(i) && valid(k)) ? L.Q[k][L.slot_of[i]] : 0.0;
    }
    __syncthreads();
    const int ntile_b = (a.C + 63) / 64;
    for (int t = 0; t < ntile_b; ++t) {
      apply_tile(a.bw, a.C, 64 * t, L.G, Xs, valid, grow);
      __syncthreads();
    }
    apply_tile(a.jt, a.R, 0, L.G, Xs, valid, grow);
    __syncthreads();
  }
  if (tid == 0) {
    a.ctr[0] = conv ? 0 : 1;
    a.ctr[1] = sw;
  }
}

// -------------------------------------------------------------- one-sided Jacobi, tiny matrices
// At most 32 rows of at most 64 columns: the cyclic one-sided (Hestenes) method directly on
// the rows, held in LDS with Jt.  Round-robin rounds of at most 16 disjoint row pairs; the 16
// lanes of a pair's lane group each hold 4 columns of B and 2 of Jt, the three dot products
// are reduced with shuffles inside the group, and every round ends with one barrier.
// Rotation and tests as in the blocked method: J = [[c, s], [-s, c]] on rows (i, j), i < j,
// outer tolerance a.tol, rows at the rounding floor left alone.  ctr[0] = 0 when converged,
// ctr[1] = sweeps.  grid (matrices), 256 threads.
__global__ __launch_bounds__(256) void jacobi_tiny_kernel(const SvdMat *mats, int max_sweeps) {
  __shared__ double Bs[32][65];
  __shared__ double Js[32][33];
  __shared__ int vs_dummy;
  const SvdMat &a = mats[blockIdx.x];
  if (!a.active || a.fused != 2) return;
  const int tid = threadIdx.x, t = tid >> 4, l = tid & 15;
  const int R = a.R, C = a.C;
  for (int e = tid; e < 32 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    Bs[r][c] = (r < R && c < C) ? a.bw[(int64_t)r * C + c] : 0.0;
  }
  for (int e = tid; e < 32 * 32; e += 256) {
    const int r = e >> 5, c = e & 31;
    Js[r][c] = (r < R && c < R) ? a.jt[(int64_t)r * R + c] : 0.0;
  }
  (void)vs_dummy;
  const double floor2 = row_floor2(a, *a.fro2);
  const double tol2 = a.tol * a.tol;  // read once: inside the rounds a descriptor load is a memory round trip
  const int nvp = R + (R & 1), P = nvp / 2;
  int sw = 0, conv = 0;
  __syncthreads();
  while (sw < max_sweeps) {
    ++sw;
    int rot = 0;
    for (int rr = 0; rr < nvp - 1; ++rr) {
      int i = -1, j = -1;
      if (t < P) {  // round rr of the round-robin: 0 <= rr + t, rr - t + nvp - 1 < 2 (nvp - 1)
        const int m1 = nvp - 1;
        if (t == 0) { i = rr; j = m1; }
        else {
          i = rr + t >= m1 ? rr + t - m1 : rr + t;
          j = rr - t + m1 >= m1 ? rr - t : rr - t + m1;
        }
        if (i > j) { const int q = i; i = j; j = q; }
        if (j >= R) i = -1;  // the dummy of an odd R
      }
      double xa[4], ya[4], xj[2], yj[2];
      double al = 0.0, be = 0.0, ga = 0.0;
      if (i >= 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xa[u] = Bs[i][l + 16 * u];
          ya[u] = Bs[j][l + 16 * u];
          al += xa[u] * xa[u];
          be += ya[u] * ya[u];
          ga += xa[u] * ya[u];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          xj[u] = Js[i][l + 16 * u];
          yj[u] = Js[j][l + 16 * u];
        }
      }
      // the 16 lanes of a pair are one DPP row
      al = row16_sum(al);
      be = row16_sum(be);
      ga = row16_sum(ga);
      if (i >= 0 && al > floor2 && be > floor2 && al > 0.0 && be > 0.0 && ga * ga > tol2 * (al * be)) {
        double c, s;
        jacobi_rot(al, be, ga, c, s);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          Bs[i][l + 16 * u] = c * xa[u] - s * ya[u];
          Bs[j][l + 16 * u] = s * xa[u] + c * ya[u];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          Js[i][l + 16 * u] = c * xj[u] - s * yj[u];
          Js[j][l + 16 * u] = s * xj[u] + c * yj[u];
        }
        rot = 1;
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rot)) {
      conv = 1;
      break;
    }
  }
  for (int e = tid; e < R * C; e += 256) a.bw[e] = Bs[e / C][e % C];
  for (int e = tid; e < R * R; e += 256) a.jt[e] = Js[e / R][e % R];
  if (tid == 0) {
    a.ctr[0] = conv ? 0 : 1;
    a.ctr[1] = sw;
  }
}

// -------------------------------------------------------------- load / init
// grid (tiles, 1, matrices): rows of A (or of A^T) into bw as double; Jt = I
__global__ __launch_bounds__(256) void load_kernel(const SvdMat *mats) {
  __shared__ double tile[32][33];
  const SvdMat &a = mats[blockIdx.z];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int ntj = (a.n + 31) / 32, nti = (a.m + 31) / 32;
  const int t = blockIdx.x;
  if (t < nti * ntj) {
    const int by = (t / ntj) * 32, bx = (t % ntj) * 32;  // by over m, bx over n
    for (int r = ty; r < 32; r += 8) {
      const int i = by + r, j = bx + tx;
      double v = 0.0;
      if (i < a.m && j < a.n)
        v = a.dtype == TNA_F64 ? static_cast<const double *>(a.A)[(int64_t)i * a.n + j]
                               : (double)static_cast<const float *>(a.A)[(int64_t)i * a.n + j];
      tile[r][tx] = v;
    }
    __syncthreads();
    if (!a.trans) {
      for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        if (i < a.m && j < a.n) a.bw[(int64_t)i * a.n + j] = tile[r][tx];
      }
    } else {
      for (int r = ty; r < 32; r += 8) {
        const int j = bx + r, i = by + tx;
        if (j < a.n && i < a.m) a.bw[(int64_t)j * a.m + i] = tile[tx][r];
      }
    }
  } else {
    const int64_t e0 = (int64_t)(t - nti * ntj) * 1024, tot = (int64_t)a.R * a.R;
    for (int64_t e = e0 + threadIdx.x; e < e0 + 1024 && e < tot; e += 256) {
      const int64_t r = e / a.R, c = e - r * a.R;
      a.jt[e] = (r == c) ? 1.0 : 0.0;
    }
  }
}

// |A|_F^2 of the loaded rows in two fixed-order stages: block partials into the Gram
// area (free until the first sweep), then one block per matrix sums them
constexpr int FRO_BLOCKS = 256;
__global__ __launch_bounds__(256) void fro_partial_kernel(const SvdMat *mats) {
  __shared__ double red[4];
  const SvdMat &a = mats[blockIdx.z];
  const int64_t tot = (int64_t)a.R * a.C;
  const int64_t chunk = (tot + FRO_BLOCKS - 1) / FRO_BLOCKS;
  const int64_t beg = chunk * blockIdx.x, end = beg + chunk < tot ? beg + chunk : tot;
  double v = 0.0;
  for (int64_t e = beg + threadIdx.x; e < end; e += 256) v += a.bw[e] * a.bw[e];
  v = bsum256(v, red);
  if (threadIdx.x == 0) a.gram[blockIdx.x] = v;
}
__global__ __launch_bounds__(256) void fro_kernel(const SvdMat *mats) {
  __shared__ double red[4];
  const SvdMat &a = mats[blockIdx.x];
  double v = threadIdx.x < FRO_BLOCKS ? a.gram[threadIdx.x] : 0.0;
  v = bsum256(v, red);
  if (threadIdx.x == 0) *a.fro2 = v;
}

__global__ void zero_ctr_kernel(const SvdMat *mats, int nmat) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < nmat && mats[z].active && !mats[z].fused) *mats[z].ctr = 0;
}

// -------------------------------------------------------------- QR start
// A Householder QR of the loaded rows, B = Q Rf, turns the start state (B, Jt) =
// (A, I) into (Rf, Q^T): B = Jt A still holds, and the one-sided Jacobi needs far
// fewer sweeps on the rows of Rf than on A itself.  Blocked: each panel of 32
// columns is factored by one workgroup, the trailing columns take the panel's
// block reflector as three GEMMs, and Q^T is formed from the stored reflectors the
// same way.  No column pivoting: on the prescribed-spectrum matrices it did not
// lower the sweep count; cperm / pinv keep the (identity) column order explicit.
constexpr int QR_MIN_ROWS_DEV = 256;
// The products of a block reflector with 32 rows (S = V V^T and W = V X) are long in K and short
// in M: K is cut into QR_SPLIT pieces that run as one batched launch, and the pieces are summed in
// order afterwards.
constexpr int QR_SPLIT = 8;

// grid (column blocks, 1, matrices): the identity column order
__global__ __launch_bounds__(256) void qr_init_kernel(const SvdMat *mats) {
  const SvdMat &a = mats[blockIdx.z];
  if (!a.active || !a.precond) return;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < a.C) a.cperm[j] = j;
  if (j == 0) a.ctr[2] = 0;  // arrival counter of qr_col_kernel
}

// A rows_scaled matrix whose QR start may stop early takes its columns in order of decreasing
// norm (ties: lower index first), decided once before the factorisation: the panels then meet
// the heavy columns first, so the rows below the factored panels fall to the rounding level at
// about the numerical rank whatever the input's column order (a two-site matrix is ordered
// physical index first, so half of its columns by weight sit at the end).
__device__ inline bool qr_sorts_columns(const SvdMat &a) { return a.active && a.precond && a.rows_scaled; }

// grid (column blocks, 1, matrices): squared column norms of B into qws[2048 ..) (free until the QR)
__global__ __launch_bounds__(256) void colnorm_kernel(const SvdMat *mats) {
  const SvdMat &a = mats[blockIdx.z];
  if (!qr_sorts_columns(a)) return;
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= a.C) return;
  double ss = 0.0;
  for (int r = 0; r < a.R; ++r) {
    const double v = a.bw[(int64_t)r * a.C + c];
    ss += v * v;
  }
  a.qws[2048 + c] = ss;
}

// one block per matrix: cperm <- columns by decreasing norm (bitonic sort of (norm, index))
__global__ __launch_bounds__(1024) void colsort_kernel(const SvdMat *mats) {
  __shared__ double key[4096];
  __shared__ int idx[4096];
  const SvdMat &a = mats[blockIdx.x];
  if (!qr_sorts_columns(a)) return;
  int P = 1;
  while (P < a.C) P <<= 1;
  for (int i = threadIdx.x; i < P; i += 1024) {
    key[i] = i < a.C ? a.qws[2048 + i] : -1.0;
    idx[i] = i;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += 1024) {
        const int l = i ^ j;
        if (l > i) {
          const bool i_before_l = key[i] > key[l] || (key[i] == key[l] && idx[i] < idx[l]);
          if ((i & k) == 0 ? !i_before_l : i_before_l) {
            const double tk = key[i]; key[i] = key[l]; key[l] = tk;
            const int ti = idx[i]; idx[i] = idx[l]; idx[l] = ti;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < a.C; i += 1024) a.cperm[i] = idx[i];
}

// grid (tiles, 1, matrices): B[r][c] <- row r of A (A^T when trans) at column cperm[c], read again
// from the input (the natural-order load served the norms)
__global__ __launch_bounds__(256) void permute_load_kernel(const SvdMat *mats) {
  __shared__ double tile[32][33];
  const SvdMat &a = mats[blockIdx.z];
  if (!qr_sorts_columns(a)) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int ntc = (a.C + 31) / 32, ntr = (a.R + 31) / 32;
  const int t = blockIdx.x;
  if (t >= ntr * ntc) return;
  const int r0 = (t / ntc) * 32, c0 = (t % ntc) * 32;
  auto in = [&](int64_t e) {
    return a.dtype == TNA_F64 ? static_cast<const double *>(a.A)[e] : (double)static_cast<const float *>(a.A)[e];
  };
  if (!a.trans) {  // B row r = A row r (length n = C): gather along the row
    for (int rr = ty; rr < 32; rr += 8) {
      const int r = r0 + rr, c = c0 + tx;
      if (r < a.R && c < a.C) a.bw[(int64_t)r * a.C + c] = in((int64_t)r * a.n + a.cperm[c]);
    }
  } else {  // B row r = A column r; B column c = A row cperm[c]: read A rows along r, write through LDS
    for (int cc = ty; cc < 32; cc += 8) {
      const int c = c0 + cc, r = r0 + tx;
      tile[cc][tx] = (c < a.C && r < a.R) ? in((int64_t)a.cperm[c] * a.n + r) : 0.0;
    }
    __syncthreads();
    for (int rr = ty; rr < 32; rr += 8) {
      const int r = r0 + rr, c = c0 + tx;
      if (r < a.R && c < a.C) a.bw[(int64_t)r * a.C + c] = tile[tx][rr];
    }
  }
}

// Householder QR of the panel of columns k0 .. k0+31 of B (rows k0..), one column after the
// other: x = B[k:R, k], alpha = -sign(x_0) |x|, v = x - alpha e_0 (stored as row k of qv),
// beta = 2 / v^T v = 1 / (|x| (|x| + |x_0|)) (stored in qws); B[k:, k] <- (alpha, 0, ...); then
// every later column c of the panel: B[k:, c] -= beta (v^T B[k:, c]) v.  The trailing columns are
// updated afterwards with the block reflector (qr_block_apply).
//
// Spread over row chunks of QC_ROWS rows, one launch per column: launch k applies reflector k to
// the panel columns right of it and forms the chunk partials that reflector k+1 needs
// (|B[k+1:, k+1]|^2 and the dots B[k+2:, k+1] . B[k+2:, c]); the last chunk to arrive (arrival
// counter, device-scope fences, no waiting) sums the partials in chunk order and writes alpha, beta,
// v_{k+1,k+1} = x0 - alpha and w_c = beta (v . B[:, c]) for the next launch.  The start launch
// (k = k0 - 1) forms the partials of column k0 only.  Scratch: chunk partials (33 per chunk) at
// qws[2048 ..), the scalars at qws[2048 + 64 C + R ..).  grid (chunks, 1, matrices), 256 threads.
constexpr int QC_ROWS = 128;
__global__ __launch_bounds__(256) void qr_col_kernel(const SvdMat *mats, int k0, int k) {
  __shared__ double red[8][33];
  __shared__ int last;
  const SvdMat &a = mats[blockIdx.z];
  if (!a.active || !a.precond || k0 >= a.Ra) return;
  const int R = a.R, C = a.C;
  const int kend = k0 + 32 < R ? k0 + 32 : R, cend = k0 + 32 < C ? k0 + 32 : C;
  if (k >= kend) return;
  const int G = (R - k0 + QC_ROWS - 1) / QC_ROWS, blk = blockIdx.x;
  if (blk >= G) return;
  const int tid = threadIdx.x, lane = tid & 63, cl = tid & 31, rsub = tid >> 5;
  const int c = k0 + cl;
  const bool colok = c < cend;
  double *B = a.bw;
  double *part = a.qws + 2048, *betas = a.qws + 2048 + 64 * (int64_t)C, *sc = betas + R;
  const bool start = k < k0;
  if (start) {
    // reflector rows k0 .. kend-1 start as zero (launch k writes its entries from row k on)
    const int64_t tot = (int64_t)(kend - k0) * R;
    for (int64_t e = (int64_t)blk * 256 + tid; e < tot; e += (int64_t)G * 256) a.qv[(int64_t)k0 * R + e] = 0.0;
    if (blk == 0 && tid == 0) a.fro2[1] = 0.0;  // trailing-row maximum of this panel (qr_tail_kernel)
  }
  double alpha = 0.0, beta = 0.0, vk = 0.0, x0 = 0.0, wc = 0.0;
  const int kc = k - k0;
  if (!start) {
    alpha = sc[0];
    beta = sc[1];
    vk = sc[2];
    x0 = sc[3];
    wc = (cl > kc && colok) ? sc[4 + cl] : 0.0;
  }
  double val[QC_ROWS / 8];
#pragma unroll
  for (int m = 0; m < QC_ROWS / 8; ++m) {
    const int i = k0 + blk * QC_ROWS + rsub + 8 * m;
    double x = (i < R && colok) ? B[(int64_t)i * C + c] : 0.0;
    if (!start) {
      const double bk = __shfl(x, (lane & 32) | kc, 64);  // this row's column-k entry
      if (i < R && i >= k && colok && cl >= kc) {
        const double vi = (i == k) ? vk : bk;
        if (cl > kc) {
          x -= wc * vi;
        } else {
          x = (i == k) ? (beta != 0.0 ? alpha : x0) : 0.0;
          a.qv[(int64_t)k * R + i] = vi;
        }
        B[(int64_t)i * C + c] = x;
      }
    }
    val[m] = x;
  }
  const int nk = k + 1, nc = nk - k0;
  if (nk >= kend) return;
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < QC_ROWS / 8; ++m) {
    const int i = k0 + blk * QC_ROWS + rsub + 8 * m;
    const double y = val[m];
    const double ynk = __shfl(y, (lane & 32) | nc, 64);
    if (i < R && i >= nk) {
      if (cl == nc) acc += y * y;                    // |B[nk:, nk]|^2
      else if (cl > nc && i > nk) acc += ynk * y;    // B[nk+1:, nk] . B[nk+1:, c]
    }
  }
  red[rsub][cl] = acc;
  __syncthreads();
  if (tid < 32 && cl >= nc) {
    double t = 0.0;
#pragma unroll
    for (int g = 0; g < 8; ++g) t += red[g][cl];
    part[(int64_t)blk * 33 + 1 + cl] = t;
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) last = atomicAdd(&a.ctr[2], 1) == G - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (tid < 32 && cl >= nc) {
    double t = 0.0;
    for (int b = 0; b < G; ++b) t += part[(int64_t)b * 33 + 1 + cl];
    red[0][cl] = t;
  }
  __syncthreads();
  if (tid < 32) {
    const double nx = sqrt(red[0][nc]);
    const double xn = B[(int64_t)nk * C + nk];
    const double al = xn >= 0.0 ? -nx : nx;
    const double be = nx > 0.0 ? 1.0 / (nx * (nx + fabs(xn))) : 0.0;
    const double v0 = xn - al;
    if (cl > nc && colok) sc[4 + cl] = be * (red[0][cl] + v0 * B[(int64_t)nk * C + c]);
    if (cl == 0) {
      sc[0] = al;
      sc[1] = be;
      sc[2] = v0;
      sc[3] = xn;
      betas[nk] = be;
      a.ctr[2] = 0;
    }
  }
}

// The same panel factorisation as qr_col_kernel in one cooperative launch per panel: each
// workgroup keeps its QC_ROWS-row chunk of the panel in registers for all 32 columns, and one grid
// barrier per column replaces a launch.  Per column every workgroup writes its chunk partials
// (|B[k+1:, k+1]|^2, the dots B[k+2:, k+1] . B[k+2:, c], and, for the chunk holding row k+1,
// that row's entries) into one of two alternating buffers, passes the barrier, and sums all
// chunks' partials in chunk order itself, so every workgroup forms the same reflector scalars
// with the additions of the per-launch path (row k+1's entries come from one chunk, the other
// chunks add exact zeros).  The chunk is written back to B after the last column.  Must be
// launched with hipLaunchCooperativeKernel (all workgroups resident); every workgroup of the
// grid passes the same 33 barriers whatever its matrix.  Scratch: 2 x 65 partials per chunk at
// qws[2048 ..).  grid (chunks, 1, matrices), 256 threads.
constexpr int QC_GROUP = 64;
__global__ __launch_bounds__(256) void qr_panel_coop_kernel(const SvdMat *mats, int k0) {
  __shared__ double pl[QC_GROUP * 64];
  __shared__ double red[8][33];
  __shared__ double rowv[32];
  __shared__ double scs[4 + 32];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const SvdMat &a = mats[blockIdx.z];
  const int R = a.R, C = a.C;
  const bool on = a.active && a.precond && k0 < a.Ra && k0 < R;
  const int kend = k0 + 32 < R ? k0 + 32 : R, cend = k0 + 32 < C ? k0 + 32 : C;
  const int G = on ? (R - k0 + QC_ROWS - 1) / QC_ROWS : 0, blk = blockIdx.x;
  const bool mine = blk < G;
  const int tid = threadIdx.x, lane = tid & 63, cl = tid & 31, rsub = tid >> 5;
  const int c = k0 + cl;
  const bool colok = c < cend;
  double *B = a.bw;
  double *part = a.qws + 2048, *betas = a.qws + 2048 + 64 * (int64_t)C;
  double val[QC_ROWS / 8];
  if (mine) {
    // reflector rows k0 .. kend-1 start as zero (column k writes its entries from row k on)
    const int64_t tot = (int64_t)(kend - k0) * R;
    for (int64_t e = (int64_t)blk * 256 + tid; e < tot; e += (int64_t)G * 256) a.qv[(int64_t)k0 * R + e] = 0.0;
    if (blk == 0 && tid == 0) a.fro2[1] = 0.0;  // trailing-row maximum of this panel (qr_tail_kernel)
  }
#pragma unroll
  for (int m = 0; m < QC_ROWS / 8; ++m) {
    const int i = k0 + blk * QC_ROWS + rsub + 8 * m;
    val[m] = (mine && i < R && colok) ? B[(int64_t)i * C + c] : 0.0;
  }
  for (int it = 0; it <= 32; ++it) {
    const int k = k0 - 1 + it;
    if (mine && it > 0 && k < kend) {  // apply reflector k to the chunk
      const int kc = k - k0;
      const double alpha = scs[0], beta = scs[1], vk = scs[2], x0 = scs[3];
      const double wc = (cl > kc && colok) ? scs[4 + cl] : 0.0;
#pragma unroll
      for (int m = 0; m < QC_ROWS / 8; ++m) {
        const int i = k0 + blk * QC_ROWS + rsub + 8 * m;
        double x = val[m];
        const double bk = __shfl(x, (lane & 32) | kc, 64);  // this row's column-k entry
        if (i < R && i >= k && colok && cl >= kc) {
          const double vi = (i == k) ? vk : bk;
          if (cl > kc) {
            x -= wc * vi;
          } else {
            x = (i == k) ? (beta != 0.0 ? alpha : x0) : 0.0;
            a.qv[(int64_t)k * R + i] = vi;
          }
        }
        val[m] = x;
      }
    }
    const int nk = k + 1, nc = nk - k0;
    const bool more = mine && nk < kend;
    double *pp = part + (int64_t)(it & 1) * G * 65;
    if (more) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < QC_ROWS / 8; ++m) {
        const int i = k0 + blk * QC_ROWS + rsub + 8 * m;
        const double y = val[m];
        const double ynk = __shfl(y, (lane & 32) | nc, 64);
        if (i < R && i >= nk) {
          if (cl == nc) acc += y * y;                    // |B[nk:, nk]|^2
          else if (cl > nc && i > nk) acc += ynk * y;    // B[nk+1:, nk] . B[nk+1:, c]
        }
      }
      red[rsub][cl] = acc;
      __syncthreads();
      if (tid < 32) {
        double t = 0.0;
#pragma unroll
        for (int g = 0; g < 8; ++g) t += red[g][cl];
        pp[(int64_t)blk * 65 + 1 + cl] = cl >= nc ? t : 0.0;
      }
      // row nk's entries from the chunk that holds the row, exact zeros from the others
      const int own = (nk - k0) / QC_ROWS, ro = (nk - k0) % QC_ROWS;
      if (blk != own) {
        if (tid < 32) pp[(int64_t)blk * 65 + 33 + cl] = 0.0;
      } else if (rsub == ro % 8) {
#pragma unroll
        for (int m = 0; m < QC_ROWS / 8; ++m)
          if (m == ro / 8) pp[(int64_t)blk * 65 + 33 + cl] = colok ? val[m] : 0.0;
      }
    }
    grid.sync();  // device-scope release and acquire: the partials written above are visible after it
    if (more) {
      // the chunks' partials come in through LDS, QC_GROUP chunks at a time with every thread
      // loading (the far-memory latency paid once per group), and are summed in chunk order
      double t = 0.0;
      for (int b0 = 0; b0 < G; b0 += QC_GROUP) {
        const int nb = G - b0 < QC_GROUP ? G - b0 : QC_GROUP;
        for (int e = tid; e < nb * 64; e += 256) pl[e] = pp[(int64_t)(b0 + (e >> 6)) * 65 + 1 + (e & 63)];
        __syncthreads();
        if (tid < 64)
          for (int b = 0; b < nb; ++b) t += pl[b * 64 + tid];
        __syncthreads();
      }
      if (tid < 64) {
        if (tid < 32) red[0][tid] = t;
        else rowv[tid - 32] = t;
      }
      __syncthreads();
      if (tid < 32) {
        const double nx = sqrt(red[0][nc]);
        const double xn = rowv[nc];
        const double al = xn >= 0.0 ? -nx : nx;
        const double be = nx > 0.0 ? 1.0 / (nx * (nx + fabs(xn))) : 0.0;
        const double v0 = xn - al;
        if (cl > nc && colok) scs[4 + cl] = be * (red[0][cl] + v0 * rowv[cl]);
        if (cl == 0) {
          scs[0] = al;
          scs[1] = be;
          scs[2] = v0;
          scs[3] = xn;
          if (blk == 0) betas[nk] = be;
        }
      }
      __syncthreads();
    }
  }
  if (mine) {
#pragma unroll
    for (int m = 0; m < QC_ROWS / 8; ++m) {
      const int i = k0 + blk * QC_ROWS + rsub + 8 * m;
      if (i < R && colok) B[(int64_t)i * C + c] = val[m];
    }
  }
}

// T of the compact form H_k0 ... H_k0+nb-1 = I - V T V^T (T upper triangular) from
// S = V^T V and the betas: T_ii = beta_i, T[0:i, i] = -beta_i T[0:i, 0:i] S[0:i, i].
// One workgroup per matrix; S at qws[0..1024), T at qws[1024..2048), 32 x 32 row-major.
__global__ __launch_bounds__(64) void qr_tfactor_kernel(const SvdMat *mats, int k0) {
  const SvdMat &a = mats[blockIdx.x];
  if (!a.active || !a.precond || k0 >= a.Ra) return;
  __shared__ double Ss[32][33], Ts[32][33], bs[32];
  const int nb = a.R - k0 < 32 ? a.R - k0 : 32;
  const double *S = a.qws;
  double *T = a.qws + 1024;
  const double *beta = a.qws + 2048 + 64 * (int64_t)a.C + k0;
  const int r = threadIdx.x;
  // S, beta into LDS once; the recurrence runs in LDS and T goes out at the end
  for (int e = r; e < 1024; e += 64) {
    Ss[e >> 5][e & 31] = S[e];
    Ts[e >> 5][e & 31] = 0.0;
  }
  if (r < 32) bs[r] = r < nb ? beta[r] : 0.0;
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    if (r < i) {
      double acc = 0.0;
      for (int c = r; c < i; ++c) acc += Ts[r][c] * Ss[c][i];
      Ts[r][i] = -bs[i] * acc;
    } else if (r == i) {
      Ts[i][i] = bs[i];
    }
    __syncthreads();
  }
  for (int e = r; e < 1024; e += 64) T[e] = Ts[e >> 5][e & 31];
}

// grid (ceil((R - k1) / 4), 1, matrices): fro2[1] <- the largest squared norm of the rows k1.. of B
// after the panels before k1 (their entries left of column k1 are zero), one wave per row.  Run
// only while the QR start of a rows_scaled matrix is still going; the maximum is taken on the bit
// patterns of the non-negative sums, which order like the values.
__global__ __launch_bounds__(256) void qr_tail_kernel(const SvdMat *mats, int k1) {
  const SvdMat &a = mats[blockIdx.z];
  if (!a.active || !a.precond || !a.rows_scaled || k1 >= a.Ra) return;
  const int r = k1 + blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= a.R) return;
  const double *row = a.bw + (int64_t)r * a.C;
  double ss = 0.0;
  for (int c = k1 + lane; c < a.C; c += 64) ss += row[c] * row[c];
  ss = wave_sum_d(ss);
  if (lane == 0)
    atomicMax(reinterpret_cast<unsigned long long *>(a.fro2 + 1), (unsigned long long)__double_as_longlong(ss));
}

// out[r * ldo + c] = sum over p < np of part[p * M N + r N + c] (split order), r < M, c < N; grid-stride
__global__ __launch_bounds__(256) void splitk_sum_kernel(const double *part, int np, int M, int N, double *out,
                                                         int ldo) {
  const int64_t n = (int64_t)M * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    for (int p = 0; p < np; ++p) v += part[(int64_t)p * n + e];
    out[(e / N) * ldo + e % N] = v;
  }
}

// grid (column blocks, 1, matrices)
__global__ __launch_bounds__(256) void qr_pinv_kernel(const SvdMat *mats) {
  const SvdMat &a = mats[blockIdx.z];
  if (!a.active || !a.precond) return;
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c < a.C) a.pinv[a.cperm[c]] = c;
}

// -------------------------------------------------------------- finish
// grid (ceil(R/4), 1, matrices): sigma_r = |row r|, one wave per row
__global__ __launch_bounds__(256) void norms_kernel(const SvdMat *mats) {
  const SvdMat &a = mats[blockIdx.z];
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= a.R) return;
  const double *row = a.bw + (int64_t)r * a.C;
  double s = 0.0;
  for (int c = lane; c < a.C; c += 64) s += row[c] * row[c];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) a.sig[r] = sqrt(s);
}

// one block per matrix: bitonic sort of (sigma desc, index asc), then Z and the entropy
__global__ __launch_bounds__(1024) void sort_kernel(const SvdMat *mats) {
  __shared__ double key[4096];
  __shared__ int idx[4096];
  __shared__ double red[16];
  const SvdMat &a = mats[blockIdx.x];
  int P = 1;
  while (P < a.R) P <<= 1;
  for (int i = threadIdx.x; i < P; i += 1024) {
    key[i] = i < a.R ? a.sig[i] : -1.0;
    idx[i] = i;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += 1024) {
        const int l = i ^ j;
        if (l > i) {
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
  for (int i = threadIdx.x; i < a.R; i += 1024) {
    a.perm[i] = idx[i];
    a.S[i] = key[i];
  }
  // Z = sum S^2 and S_vN = -sum p ln p (p = S^2 / Z), fixed-order block sums
  double z2 = 0.0;
  for (int i = threadIdx.x; i < a.R; i += 1024) z2 += key[i] * key[i];
  for (int off = 32; off > 0; off >>= 1) z2 += __shfl_xor(z2, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = z2;
  __syncthreads();
  double Z = 0.0;
  for (int w = 0; w < 16; ++w) Z += red[w];
  __syncthreads();
  double e = 0.0;
  for (int i = threadIdx.x; i < a.R; i += 1024) {
    const double p = key[i] * key[i] / Z;
    if (p > 0.0) e -= p * log(p);
  }
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ent = 0.0;
    for (int w = 0; w < 16; ++w) ent += red[w];
    a.spec[0] = Z;
    a.spec[1] = ent;
  }
  if (threadIdx.x < 16) a.spec[8 + threadIdx.x] = (int)threadIdx.x < a.R ? key[threadIdx.x] : 0.0;
  // spec[7]: sweeps of the single-workgroup Jacobi paths, negative when not converged (0 otherwise)
  if (threadIdx.x == 0) a.spec[7] = a.fused ? (a.ctr[0] ? -(double)a.ctr[1] : (double)a.ctr[1]) : 0.0;
  // spec[24] (thr > 0 only): how many values exceed thr, for threshold truncation
  if (a.thr > 0.0) {
    __shared__ int cnt_w[16];
    int cnt = 0;
    for (int i = threadIdx.x; i < a.R; i += 1024) cnt += key[i] > a.thr;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) cnt_w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      int c = 0;
      for (int w = 0; w < 16; ++w) c += cnt_w[w];
      a.spec[24] = (double)c;
    }
  }
  // spec[25]: numerical rank, the number of values above 1e-12 S_0
  {
    __shared__ int nr_w[16];
    const double cut = (a.noise_rel > 0.0 ? a.noise_rel : 1e-12) * key[0];
    int cnt = 0;
    for (int i = threadIdx.x; i < a.R; i += 1024) cnt += key[i] > cut;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) nr_w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      int c = 0;
      for (int w = 0; w < 16; ++w) c += nr_w[w];
      a.spec[25] = (double)c;
    }
  }
  // spec[6]: smallest k >= 1 with sqrt(sum_{j>=k} S_j^2) <= eps_target (k = R always qualifies)
  if (a.eps_target > 0.0) {
    __shared__ double csum[1024];
    __shared__ int best[16];
    const int t = threadIdx.x, R = a.R;
    const double eps2 = a.eps_target * a.eps_target;
    const int L = (R + 1023) / 1024;
    const int beg = t * L, end = beg + L < R ? beg + L : R;
    double c = 0.0;
    for (int j = beg; j < end; ++j) c += key[j] * key[j];
    // sums over the chunks after this one: inclusive suffix scan in a fixed tree order
    double v = c;
    for (int off = 1; off < 1024; off <<= 1) {
      csum[t] = v;
      __syncthreads();
      if (t + off < 1024) v += csum[t + off];
      __syncthreads();
    }
    csum[t] = v;
    __syncthreads();
    const double after = t + 1 < 1024 ? csum[t + 1] : 0.0;
    int kmin = R;
    double tsum = after;
    for (int j = end - 1; j >= beg; --j) {
      tsum += key[j] * key[j];
      if (tsum <= eps2) kmin = j;
    }
    if (kmin < 1) kmin = 1;
    for (int off = 32; off > 0; off >>= 1) kmin = min(kmin, __shfl_xor(kmin, off, 64));
    if ((t & 63) == 0) best[t >> 6] = kmin;
    __syncthreads();
    if (t == 0) {
      int b = best[0];
      for (int w = 1; w < 16; ++w) b = min(b, best[w]);
      a.spec[6] = (double)b;
    }
  }
}

// one block per matrix: spec[2..5] for the kept rank k
__global__ __launch_bounds__(256) void trunc_kernel(const SvdMat *mats) {
  __shared__ double red[4];
  const SvdMat &a = mats[blockIdx.x];
  if (a.k < 1) return;
  const double *s = a.S;
  const int R = a.R, k = a.k, t = threadIdx.x;
  double tl = 0.0, hd = 0.0;
  for (int i = t; i < R; i += 256) {
    if (i >= k) tl += s[i] * s[i];
    else hd += s[i] * s[i];
  }
  const double tail = bsum256(tl, red);
  const double head = bsum256(hd, red);
  if (t == 0) {
    const double Z = a.spec[0];
    a.spec[2] = sqrt(tail);
    a.spec[3] = tail / Z;
    a.spec[4] = sqrt(head);
    a.spec[5] = (k < R && s[0] > 0.0) ? (s[k - 1] - s[k]) / s[0] : 1.0;
  }
}

// Kept values at or below this are null: at the rounding level of sigma_0 or under the
// Jacobi row floor (whose rows were never orthogonalised against the others).  With the
// QR start and no floor (rows_scaled off) every row with a nonzero norm was
// orthogonalised, so only rows whose squares underflow count as null there.
__device__ inline double null_threshold(const SvdMat &a) {
  if (a.precond && !a.rows_scaled) return 1e-150 * a.S[0];
  const double C = (double)(a.m > a.n ? a.m : a.n);
  return EPS53 * C * fmax(a.S[0], 0.1 * sqrt(*a.fro2));
}

// U (m x k) and Vt (k x n), unscaled; null Bw-derived vectors are zeroed.
// grid (chunks, 2, matrices): y = 0 writes U, y = 1 writes Vt
template <typename T>
__device__ inline void write_factors(const SvdMat &a, int which, int64_t e0, int64_t stride) {
  const double thr = null_threshold(a);
  if (which == 0) {
    T *U = static_cast<T *>(a.U);
    const int64_t total = (int64_t)a.m * a.k;
    for (int64_t e = e0; e < total; e += stride) {
      const int i = (int)(e / a.k), j = (int)(e % a.k);
      const int r = a.perm[j];
      double v;
      if (!a.trans) v = a.jt[(int64_t)r * a.R + i];
      else v = (a.S[j] > thr && a.S[j] > 0.0) ? a.bw[(int64_t)r * a.C + (a.pinv ? a.pinv[i] : i)] / a.S[j] : 0.0;
      U[e] = (T)v;
    }
  } else {
    T *Vt = static_cast<T *>(a.Vt);
    const int64_t total = (int64_t)a.k * a.n;
    for (int64_t e = e0; e < total; e += stride) {
      const int j = (int)(e / a.n), c = (int)(e % a.n);
      const int r = a.perm[j];
      double v;
      if (a.trans) v = a.jt[(int64_t)r * a.R + c];
      else v = (a.S[j] > thr && a.S[j] > 0.0) ? a.bw[(int64_t)r * a.C + (a.pinv ? a.pinv[c] : c)] / a.S[j] : 0.0;
      Vt[e] = (T)v;
    }
  }
}

__global__ __launch_bounds__(256) void write_kernel(const SvdMat *mats) {
  const SvdMat &a = mats[blockIdx.z];
  if (a.k < 1) return;
  const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
  if (a.out_type == TNA_F64) write_factors<double>(a, blockIdx.y, e0, stride);
  else write_factors<float>(a, blockIdx.y, e0, stride);
}

// Gram-Schmidt completion of kept null vectors with unit vectors e_0, e_1, ...
// (Vt rows when rows of A were orthogonalised, U columns otherwise); one block per matrix
template <typename T>
__device__ void complete_one(const SvdMat &a, double *vec, double *red, int *ok) {
  const double thr = null_threshold(a);
  const int L = a.trans ? a.m : a.n;
  T *base;
  int64_t es, vs;
  if (a.trans) { base = static_cast<T *>(a.U); es = a.k; vs = 1; }
  else { base = static_cast<T *>(a.Vt); es = 1; vs = a.n; }
  const int tid = threadIdx.x;
  int e = 0;
  for (int j = 0; j < a.k; ++j) {
    if (a.S[j] > thr && a.S[j] > 0.0) continue;
    for (; e < L; ++e) {
      for (int i = tid; i < L; i += 256) vec[i] = (i == e) ? 1.0 : 0.0;
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass)
        for (int qv = 0; qv < a.k; ++qv) {
          if (qv == j) continue;
          if (!((a.S[qv] > thr && a.S[qv] > 0.0) || qv < j)) continue;
          double h = 0.0;
          for (int i = tid; i < L; i += 256) h += (double)base[qv * vs + (int64_t)i * es] * vec[i];
          h = bsum256(h, red);
          for (int i = tid; i < L; i += 256) vec[i] -= h * (double)base[qv * vs + (int64_t)i * es];
          __syncthreads();
        }
      double nr = 0.0;
      for (int i = tid; i < L; i += 256) nr += vec[i] * vec[i];
      nr = sqrt(bsum256(nr, red));
      if (tid == 0) *ok = nr > 0.5;
      __syncthreads();
      const int good = *ok;
      __syncthreads();
      if (good) {
        for (int i = tid; i < L; i += 256) base[j * vs + (int64_t)i * es] = (T)(vec[i] / nr);
        __syncthreads();
        ++e;
        break;
      }
    }
  }
}

__global__ __launch_bounds__(256) void complete_kernel(const SvdMat *mats) {
  __shared__ double vec[4096];
  __shared__ double red[4];
  __shared__ int ok;
  const SvdMat &a = mats[blockIdx.x];
  if (a.k < 1 || a.rows_scaled) return;  // the factor to complete leaves scaled by (near-)zero values
  // only matrices with a kept null vector do any work
  const double thr = null_threshold(a);
  if (a.S[a.k - 1] > thr && a.S[a.k - 1] > 0.0) return;
  if (a.out_type == TNA_F64) complete_one<double>(a, vec, red, &ok);
  else complete_one<float>(a, vec, red, &ok);
}

// sign gauge (largest-|.| entry of U[:, j] positive, ties: lowest row), then
// scaling by S_j/|S_k| of Vt rows (scale_mode 1) or U columns (scale_mode 2)
template <typename T>
__device__ void gauge_one(const SvdMat &a, int j, double *bv, int *bi, double *sgn) {
  const int tid = threadIdx.x;
  T *U = static_cast<T *>(a.U);
  T *Vt = static_cast<T *>(a.Vt);
  double best = -1.0;
  int bidx = 0x7fffffff;
  for (int i = tid; i < a.m; i += 256) {
    const double v = fabs((double)U[(int64_t)i * a.k + j]);
    if (v > best) { best = v; bidx = i; }
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
    *sgn = ((double)U[(int64_t)ii * a.k + j] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  const double nk = a.spec[4];
  const double f = (a.scale_mode != 0 && nk > 0.0) ? a.S[j] / nk : 1.0;
  const double fu = *sgn * (a.scale_mode == 2 ? f : 1.0);
  const double fv = *sgn * (a.scale_mode == 1 ? f : 1.0);
  if (fu != 1.0)
    for (int i = tid; i < a.m; i += 256) U[(int64_t)i * a.k + j] = (T)((double)U[(int64_t)i * a.k + j] * fu);
  if (fv != 1.0)
    for (int c = tid; c < a.n; c += 256) Vt[(int64_t)j * a.n + c] = (T)((double)Vt[(int64_t)j * a.n + c] * fv);
}

// grid (max k, 1, matrices)
__global__ __launch_bounds__(256) void gauge_kernel(const SvdMat *mats) {
  __shared__ double bv[4];
  __shared__ int bi[4];
  __shared__ double sgn;
  const SvdMat &a = mats[blockIdx.z];
  const int j = blockIdx.x;
  if (j >= a.k) return;
  if (a.out_type == TNA_F64) gauge_one<double>(a, j, bv, bi, &sgn);
  else gauge_one<float>(a, j, bv, bi, &sgn);
}

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
constexpr int QR_MIN_ROWS = QR_MIN_ROWS_DEV;

}  // namespace

// ====================================================================== host
tna_status svd_plan_mat(int m, int n, int dtype, int batch_hint, SvdMat *a, int orient) {
  if (m < 1 || n < 1) {
    set_error("svd: dimensions must be positive");
    return TNA_ERR_ARG;
  }
  *a = SvdMat{};
  a->m = m;
  a->n = n;
  a->trans = m > n || (m == n && orient == 2);
  a->R = m < n ? m : n;
  a->C = m < n ? n : m;
  a->Ra = a->R;
  a->dtype = dtype;
  if (a->C > 4096) {
    set_error("svd: max(m,n) > 4096 is not supported");
    return TNA_ERR_UNSUPPORTED;
  }
  int nb = (a->R + BS - 1) / BS;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  a->nb = nb;
  const int npairs = nb / 2;
  int ks = ceil_div(1024, (int64_t)npairs * (batch_hint > 0 ? batch_hint : 1));
  const int kmax = ceil_div(a->C, 256);
  if (ks > kmax) ks = kmax;
  if (ks < 1) ks = 1;
  a->ksplit = ks;
  // Outer convergence: every off-diagonal |g_ij| <= tol sqrt(g_ii g_jj).  Applying a
  // 64-row block rotation and re-forming the Gram leave a rounding floor of about
  // (64 + C) ulps whatever C is, so the bound sits at twice that floor.
  a->tol = 2.0 * (64.0 + (double)a->C) * EPS53;
  static const int inner_env = [] {
    const char *e = std::getenv("TNA_SVD_INNER");
    return e ? std::atoi(e) : 0;
  }();
  a->fused = (a->R <= 32 && a->C <= 64) ? 2 : ((nb == 2 && a->C <= 1024) ? 1 : 0);
  a->precond = (!a->fused && a->R >= QR_MIN_ROWS) ? 1 : 0;
  // Two inner sweeps per block pair (one after the QR start and in the
  // single-workgroup form) cost few extra outer sweeps and far less than diagonalising
  // each pair
  a->inner_max = inner_env > 0 ? inner_env : ((a->fused || a->precond) ? 1 : 2);
  a->active = 1;
  return TNA_OK;
}

size_t svd_work_doubles(const SvdMat &a) {
  const size_t npairs = a.nb / 2;
  return (size_t)a.R * a.C + (size_t)a.R * a.R + npairs * a.ksplit * 4096 + npairs * 4096 + a.R + 8 +
         (a.precond ? (size_t)a.R * a.R + 2048 + 64 * (size_t)a.C + 2 * (size_t)a.R + QR_SPLIT * 32 * (size_t)a.C : 0);
}
size_t svd_work_ints(const SvdMat &a) { return (size_t)a.nb / 2 + a.R + 4 + (a.precond ? 2 * (size_t)a.C : 0); }

void svd_bind_work(SvdMat *a, double *dw, int *iw) {
  const size_t npairs = a->nb / 2;
  a->bw = dw;
  dw += (size_t)a->R * a->C;
  a->jt = dw;
  dw += (size_t)a->R * a->R;
  a->gram = dw;
  dw += npairs * a->ksplit * 4096;
  a->qt = dw;
  dw += npairs * 4096;
  a->sig = dw;
  dw += a->R;
  a->fro2 = dw;
  dw += 8;
  a->skip = iw;
  iw += npairs;
  a->perm = iw;
  iw += a->R;
  a->ctr = iw;
  iw += 4;
  if (a->precond) {
    a->qv = dw;
    dw += (size_t)a->R * a->R;
    a->qws = dw;  // S (32 x 32), T (32 x 32), W and W2 (32 x C each), betas (R), spare (R), then the
                  // split-K partial products (QR_SPLIT x 32 x C)
    a->cperm = iw;
    iw += a->C;
    a->pinv = iw;
  } else {
    a->qv = a->qws = nullptr;
    a->cperm = a->pinv = nullptr;
  }
}

static tna_status upload(const std::vector<SvdMat> &mats, SvdGroup &g, hipStream_t s) {
  const size_t bytes = sizeof(SvdMat) * mats.size();
  TNA_TRY(g.desc.ensure(bytes));
  if (g.host_cap < bytes) {
    if (g.host) (void)hipHostFree(g.host);
    g.host = nullptr;
    g.host_cap = 0;
    TNA_HIP(hipHostMalloc(&g.host, bytes * 2, hipHostMallocDefault));
    g.host_cap = bytes * 2;
  }
  // the previous upload may still be in flight from this staging buffer
  TNA_HIP(hipStreamSynchronize(s));
  std::memcpy(g.host, mats.data(), bytes);
  TNA_HIP(hipMemcpyAsync(g.desc.ptr, g.host, bytes, hipMemcpyHostToDevice, s));
  return TNA_OK;
}

// C (M x N, row stride ldc) = A B over K cut into up to QR_SPLIT pieces: A is M x K (rows, lda; transA 0),
// B is K x N (transB 0: rows of ldb) or N x K (transB 1); pieces go to `part` (one M x N block
// each), then are summed into C in piece order.
static tna_status splitk_gemm(int M, int N, int K, const double *A, int lda, const double *B, int ldb, int transB,
                              double *C, int ldc, double *part, hipStream_t s) {
  const int kc = std::max(32, ceil_div(ceil_div(K, QR_SPLIT), 16) * 16);
  const int full = K / kc, rem = K - full * kc;
  const int64_t mn = (int64_t)M * N;
  if (full > 0)
    TNA_TRY(gemm(GemmArgs{M, N, kc, A, lda, 0, G_F64, B, ldb, transB, G_F64, part, N, G_F64, 1.0, 0.0, full, kc,
                          transB ? (int64_t)kc : (int64_t)kc * ldb, mn, G_F64, 0}, s));
  if (rem > 0)
    TNA_TRY(gemm(GemmArgs{M, N, rem, A + (int64_t)full * kc, lda, 0, G_F64,
                          B + (transB ? (int64_t)full * kc : (int64_t)full * kc * ldb), ldb, transB, G_F64,
                          part + (int64_t)full * mn, N, G_F64, 1.0, 0.0, 1, 0, 0, 0, G_F64, 0}, s));
  const int np = full + (rem > 0 ? 1 : 0);
  hipLaunchKernelGGL(splitk_sum_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(mn, 256), 1024)), dim3(256), 0, s,
                     part, np, M, N, C, ldc);
  TNA_LAUNCHED("svd.splitk");
  return TNA_OK;
}

// X[k0:, :] <- (I - V T^T V^T) X[k0:, :] for the 32 reflectors k0.. of every QR-started
// matrix, X the trailing columns of B (on_b) or all of Jt; V as rows in qv, T from
// S = V^T V by qr_tfactor_kernel; scratch in qws.
static tna_status qr_block_apply(const std::vector<SvdMat> &mats, const SvdMat *d, int nm, int k0, bool on_b,
                                 hipStream_t s) {
  bool any = false;
  for (auto &a : mats) {
    if (!a.precond || k0 >= a.Ra) continue;
    if (on_b && k0 + 32 >= a.C) continue;
    any = true;
    const int R = a.R, nbk = std::min(32, R - k0), K = R - k0;
    const double *Vb = a.qv + (int64_t)k0 * R + k0;
    double *part = a.qws + 2048 + 64 * (int64_t)a.C + 2 * (int64_t)R;
    TNA_TRY(splitk_gemm(nbk, nbk, K, Vb, R, Vb, R, 1, a.qws, 32, part, s));  // S = V V^T, row stride 32
  }
  if (!any) return TNA_OK;
  hipLaunchKernelGGL(qr_tfactor_kernel, dim3(nm), dim3(64), 0, s, d, k0);
  TNA_LAUNCHED("svd.qr_tfactor");
  for (auto &a : mats) {
    if (!a.precond || k0 >= a.Ra) continue;
    if (on_b && k0 + 32 >= a.C) continue;
    const int R = a.R, nbk = std::min(32, R - k0), K = R - k0;
    const double *Vb = a.qv + (int64_t)k0 * R + k0;
    double *T = a.qws + 1024, *W = a.qws + 2048, *W2 = a.qws + 2048 + 32 * (int64_t)a.C;
    double *X = on_b ? a.bw + (int64_t)k0 * a.C + k0 + 32 : a.jt + (int64_t)k0 * R;
    const int ldx = on_b ? a.C : R, N = on_b ? a.C - k0 - 32 : R;
    TNA_TRY(splitk_gemm(nbk, N, K, Vb, R, X, ldx, 0, W, N, a.qws + 2048 + 64 * (int64_t)a.C + 2 * (int64_t)R, s));
    TNA_TRY(gemm(GemmArgs{nbk, N, nbk, T, 32, 1, G_F64, W, N, 0, G_F64, W2, N, G_F64, 1.0, 0.0, 1, 0, 0, 0, G_F64, 0},
                 s));
    TNA_TRY(gemm(GemmArgs{K, N, nbk, Vb, R, 1, G_F64, W2, N, 0, G_F64, X, ldx, G_F64, -1.0, 1.0, 1, 0, 0, 0, G_F64,
                          0}, s));
  }
  return TNA_OK;
}

tna_status svd_group_run(std::vector<SvdMat> &mats, SvdGroup &g, int max_sweeps, std::vector<int> &sweeps,
                         hipStream_t s, bool defer_fused) {
  const int nm = (int)mats.size();
  if (nm == 0) return TNA_OK;
  sweeps.assign(nm, 0);
  int max_tiles_load = 0, max_pairs = 0, max_ks = 0, max_tiles = 0, max_steps = 0, max_r4 = 0;
  for (auto &a : mats) {
    a.active = 1;
    max_tiles_load = std::max(max_tiles_load, ceil_div(a.m, 32) * ceil_div(a.n, 32) + ceil_div((int64_t)a.R * a.R, 1024));
    max_pairs = std::max(max_pairs, a.nb / 2);
    max_ks = std::max(max_ks, a.ksplit);
    max_tiles = std::max(max_tiles, ceil_div(a.C, 64) + ceil_div(a.R, 64));
    max_steps = std::max(max_steps, a.nb - 1);
    max_r4 = std::max(max_r4, ceil_div(a.R, 4));
  }
  TNA_TRY(upload(mats, g, s));
  const SvdMat *d = g.desc.as<SvdMat>();
  hipLaunchKernelGGL(load_kernel, dim3(max_tiles_load, 1, nm), dim3(256), 0, s, d);
  hipLaunchKernelGGL(fro_partial_kernel, dim3(FRO_BLOCKS, 1, nm), dim3(256), 0, s, d);
  hipLaunchKernelGGL(fro_kernel, dim3(nm), dim3(256), 0, s, d);
  TNA_LAUNCHED("svd.load");
  if (!g.host_ctr) TNA_HIP(hipHostMalloc((void **)&g.host_ctr, sizeof(int) * 8192, hipHostMallocDefault));
  if (nm > 4096) {
    set_error("svd: at most 4096 matrices per group");
    return TNA_ERR_ARG;
  }
  // a NaN or Inf anywhere in an input shows in its squared Frobenius norm; the callers that defer
  // their reads (the sweep engine) check the spectrum sums they read anyway
  if (!defer_fused) {
    if (!g.host_fro) TNA_HIP(hipHostMalloc((void **)&g.host_fro, sizeof(double) * 3 * 4096, hipHostMallocDefault));
    for (int z = 0; z < nm; ++z)
      TNA_HIP(hipMemcpyAsync(g.host_fro + z, mats[z].fro2, sizeof(double), hipMemcpyDeviceToHost, s));
    TNA_HIP(hipStreamSynchronize(s));
    for (int z = 0; z < nm; ++z)
      if (!std::isfinite(g.host_fro[z])) {
        set_error("svd: non-finite entry in input matrix " + std::to_string(z));
        return TNA_ERR_NONFINITE;
      }
  }
  // QR start for the larger matrices
  int qr_rows = 0, qr_cblk = 0;
  for (auto &a : mats)
    if (a.precond) {
      qr_rows = std::max(qr_rows, a.R);
      qr_cblk = std::max(qr_cblk, ceil_div(a.C, 256));
    }
  if (qr_rows > 0) {
    hipLaunchKernelGGL(qr_init_kernel, dim3(qr_cblk, 1, nm), dim3(256), 0, s, d);
    int sorted = 0, ptiles = 0;
    for (auto &a : mats)
      if (a.precond && a.rows_scaled) {
        ++sorted;
        ptiles = std::max(ptiles, ceil_div(a.R, 32) * ceil_div(a.C, 32));
      }
    if (sorted > 0) {
      hipLaunchKernelGGL(colnorm_kernel, dim3(qr_cblk, 1, nm), dim3(256), 0, s, d);
      hipLaunchKernelGGL(colsort_kernel, dim3(nm), dim3(1024), 0, s, d);
      hipLaunchKernelGGL(permute_load_kernel, dim3(ptiles, 1, nm), dim3(256), 0, s, d);
      TNA_LAUNCHED("svd.qr_order");
    }
    double qr_bytes = 0.0;
    for (auto &a : mats)
      if (a.precond) qr_bytes += 16.0 * ((double)a.R * a.C / 3.0 + (double)a.R * a.R / 2.0);
    // Blocked Householder QR (no column pivoting: the start it gives converges as fast on
    // these matrices, and the trailing update becomes GEMMs): each 32-column panel is
    // factored column by column, then B[k0:, k0+32:] <- (I - V T^T V^T) B[k0:, k0+32:].
    // A rows_scaled matrix stops its QR start once every row below the factored panels is at the
    // rounding level (row_floor2): such rows are never rotated, so the sweeps run on the rows
    // above (Ra), and a numerically low-rank matrix pays for the panels of its rank only.
    std::vector<int> watch(nm, 0);
    int nwatch = 0;
    for (int z = 0; z < nm; ++z)
      if (mats[z].precond && mats[z].rows_scaled) {
        watch[z] = 1;
        ++nwatch;
      }
    if (nwatch > 0 && !g.host_fro)
      TNA_HIP(hipHostMalloc((void **)&g.host_fro, sizeof(double) * 3 * 4096, hipHostMallocDefault));
    // the panel factorisation: one cooperative launch per panel where the runtime admits the
    // grid (all workgroups resident), else one launch per column.  TNA_QR_PANEL=col forces the
    // per-column launches; TNA_QR_PANEL=coop makes a refused cooperative launch an error.
    const char *qp = std::getenv("TNA_QR_PANEL");
    const bool force_coop = qp && std::strcmp(qp, "coop") == 0;
    bool coop = !(qp && std::strcmp(qp, "col") == 0);
    timer_begin("svd.qr", s);
    for (int k0 = 0; k0 < qr_rows; k0 += 32) {
      const int chunks = ceil_div(qr_rows - k0, QC_ROWS);
      bool panel_done = false;
      if (coop) {
        int kk0 = k0;
        void *args[] = {(void *)&d, (void *)&kk0};
        const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(qr_panel_coop_kernel),
                                                        dim3(chunks, 1, nm), dim3(256), args, 0, s);
        if (e == hipSuccess) {
          panel_done = true;
        } else {
          (void)hipGetLastError();  // not admitted: the per-column launches from here on
          if (force_coop) {
            set_error("svd: cooperative QR panel launch not admitted");
            return TNA_ERR_UNSUPPORTED;
          }
          coop = false;
        }
      }
      if (!panel_done)
        for (int k = k0 - 1; k < k0 + 32 && k < qr_rows; ++k)
          hipLaunchKernelGGL(qr_col_kernel, dim3(chunks, 1, nm), dim3(256), 0, s, d, k0, k);
      TNA_TRY(qr_block_apply(mats, d, nm, k0, true, s));
      const int k1 = k0 + 32;
      int tail = 0;
      for (int z = 0; z < nm; ++z)
        if (watch[z] && k1 < mats[z].R) tail = std::max(tail, mats[z].R - k1);
      if (tail == 0) continue;
      hipLaunchKernelGGL(qr_tail_kernel, dim3(ceil_div(tail, 4), 1, nm), dim3(256), 0, s, d, k1);
      for (int z = 0; z < nm; ++z)
        if (watch[z])
          TNA_HIP(hipMemcpyAsync(g.host_fro + 4096 + 2 * z, mats[z].fro2, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                 s));
      TNA_HIP(hipStreamSynchronize(s));
      bool stopped = false;
      for (int z = 0; z < nm; ++z) {
        if (!watch[z]) continue;
        SvdMat &a = mats[z];
        const double f = std::fmax(0.1 * EPS53 * (double)a.C, a.noise_rel);
        const double floor2 = f * f * g.host_fro[4096 + 2 * z];
        if (g.host_fro[4096 + 2 * z + 1] <= floor2) {
          a.Ra = k1;
          stopped = true;
        }
        if (a.Ra < a.R || k1 + 32 >= a.R) {
          watch[z] = 0;
          --nwatch;
        }
      }
      if (stopped) TNA_TRY(upload(mats, g, s));
      if (nwatch == 0 && std::all_of(mats.begin(), mats.end(), [&](const SvdMat &a) {
            return !a.precond || a.Ra < a.R || k1 >= a.R;
          }))
        break;
    }
    timer_end("svd.qr", 0.0, qr_bytes, s);
    hipLaunchKernelGGL(qr_pinv_kernel, dim3(qr_cblk, 1, nm), dim3(256), 0, s, d);
    // Jt = Q^T = H_{R-1} ... H_0: 32 reflectors at a time, Jt <- (I - V T^T V^T) Jt
    timer_begin("svd.qr_form", s);
    for (int k0 = 0; k0 < qr_rows; k0 += 32) TNA_TRY(qr_block_apply(mats, d, nm, k0, false, s));
    timer_end("svd.qr_form", 0.0, 0.0, s);
    TNA_LAUNCHED("svd.qr");
    // the sweeps of a stopped matrix pair blocks of its Ra rows; the Gram partial sums keep
    // within the slots planned for all R rows
    bool replan = false;
    for (auto &a : mats) {
      if (!a.precond || a.Ra >= a.R) continue;
      const int slots = (a.nb / 2) * a.ksplit;
      int nb = ceil_div(a.Ra, BS);
      if (nb < 2) nb = 2;
      if (nb & 1) ++nb;
      a.nb = nb;
      int ks = ceil_div(1024, (int64_t)(nb / 2) * nm);
      ks = std::min(ks, ceil_div(a.C, 256));
      ks = std::min(ks, slots / (nb / 2));
      a.ksplit = std::max(ks, 1);
      replan = true;
    }
    if (replan) TNA_TRY(upload(mats, g, s));
  }
  max_pairs = max_ks = 0;
  double gram_flops = 0, gram_bytes = 0, apply_flops = 0, apply_bytes = 0;
  for (auto &a : mats) {
    max_pairs = std::max(max_pairs, a.nb / 2);
    max_ks = std::max(max_ks, a.ksplit);
    const double pairs = a.nb / 2, b2 = 4096.0;
    gram_flops += 2.0 * b2 * a.C * pairs;
    gram_bytes += 8.0 * (double)a.Ra * a.C;
    apply_flops += 2.0 * b2 * (double)(a.C + a.R) * pairs;
    apply_bytes += 16.0 * ((double)a.Ra * a.C + (double)a.Ra * a.R);
  }
  // one block pair: every sweep inside one workgroup, no host round trip per sweep
  int nfused = 0, n_two = 0, n_tiny = 0;
  for (auto &a : mats) {
    nfused += a.fused != 0;
    n_two += a.fused == 1;
    n_tiny += a.fused == 2;
  }
  if (nfused > 0) {
    timer_begin("svd.fused", s);
    if (n_two) hipLaunchKernelGGL(jacobi_fused_kernel, dim3(nm), dim3(256), 0, s, d, max_sweeps);
    if (n_tiny) hipLaunchKernelGGL(jacobi_tiny_kernel, dim3(nm), dim3(256), 0, s, d, max_sweeps);
    timer_end("svd.fused", 0.0, 0.0, s);
    TNA_LAUNCHED("svd.fused");
  }
  std::vector<int> live(nm);
  int active = 0;
  max_steps = 0;
  for (int z = 0; z < nm; ++z) {
    live[z] = !mats[z].fused;
    active += live[z];
    if (live[z]) max_steps = std::max(max_steps, mats[z].nb - 1);
  }
  for (int sw = 1; sw <= max_sweeps && active > 0; ++sw) {
    hipLaunchKernelGGL(zero_ctr_kernel, dim3(ceil_div(nm, 64)), dim3(64), 0, s, d, nm);
    for (int step = 0; step < max_steps; ++step) {
      timer_begin("svd.gram", s);
      hipLaunchKernelGGL(gram_kernel, dim3(max_pairs, max_ks, nm), dim3(256), 0, s, d, step);
      timer_end("svd.gram", gram_flops, gram_bytes, s);
      timer_begin("svd.eigen", s);
      hipLaunchKernelGGL(eigen_kernel, dim3(max_pairs, nm), dim3(EIG_NT), 0, s, d, step);
      timer_end("svd.eigen", 0.0, 0.0, s);
      timer_begin("svd.apply", s);
      hipLaunchKernelGGL(apply_kernel, dim3(max_pairs, ceil_div(max_tiles, APPLY_TPW), nm), dim3(256), 0, s, d,
                         step);
      timer_end("svd.apply", apply_flops, apply_bytes, s);
    }
    TNA_LAUNCHED("svd.sweep");
    for (int z = 0; z < nm; ++z)
      if (live[z]) TNA_HIP(hipMemcpyAsync(g.host_ctr + z, mats[z].ctr, sizeof(int), hipMemcpyDeviceToHost, s));
    TNA_HIP(hipStreamSynchronize(s));
    static const int dbg = [] {
      const char *e = std::getenv("TNA_DEBUG_SVD");
      return e && e[0] == '1';
    }();
    if (dbg) std::fprintf(stderr, "svd sweep %d: rotating pairs of matrix 0 = %d\n", sw, g.host_ctr[0]);
    bool changed = false;
    for (int z = 0; z < nm; ++z) {
      if (!live[z]) continue;
      sweeps[z] = sw;
      if (g.host_ctr[z] == 0) {
        mats[z].active = 0;
        live[z] = 0;
        --active;
        changed = true;
      }
    }
    if (changed && active > 0) {
      TNA_TRY(upload(mats, g, s));
      max_steps = 0;
      for (int z = 0; z < nm; ++z)
        if (live[z]) max_steps = std::max(max_steps, mats[z].nb - 1);
    }
  }
  // with defer_fused the caller takes the sweep counts and convergence of the single-workgroup
  // paths from spec[7] after its own read of the spectra (no synchronisation here)
  if (nfused > 0 && !defer_fused) {
    for (int z = 0; z < nm; ++z)
      if (mats[z].fused)
        TNA_HIP(hipMemcpyAsync(g.host_ctr + 2 * z, mats[z].ctr, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    TNA_HIP(hipStreamSynchronize(s));
    double fl = 0.0, by = 0.0;
    for (int z = 0; z < nm; ++z)
      if (mats[z].fused) {
        sweeps[z] = g.host_ctr[2 * z + 1];
        if (g.host_ctr[2 * z] != 0) ++active;  // not converged within max_sweeps
        // per sweep: Gram 2 R^2 C, rotation of B and Jt 2 R^2 (C + R); B read for the Gram,
        // B and Jt read and written by the rotation
        const double R = mats[z].R, C = mats[z].C, sw = sweeps[z];
        fl += sw * (2.0 * R * R * C + 2.0 * R * R * (C + R));
        by += sw * 8.0 * (R * C + 2.0 * (R * C + R * R));
      }
    timer_add_work("svd.fused", fl, by);
  }
  bool reup = false;  // finishing kernels run on every matrix
  for (auto &a : mats) {
    reup = reup || !a.active;
    a.active = 1;
  }
  if (reup) TNA_TRY(upload(mats, g, s));
  hipLaunchKernelGGL(norms_kernel, dim3(max_r4, 1, nm), dim3(256), 0, s, d);
  hipLaunchKernelGGL(sort_kernel, dim3(nm), dim3(1024), 0, s, d);
  TNA_LAUNCHED("svd.finish");
  return active > 0 ? TNA_ERR_NOCONV : TNA_OK;
}

tna_status svd_group_outputs(std::vector<SvdMat> &mats, SvdGroup &g, hipStream_t s) {
  const int nm = (int)mats.size();
  if (nm == 0) return TNA_OK;
  int max_k = 1;
  int64_t max_el = 1;
  for (auto &a : mats) {
    max_k = std::max(max_k, a.k);
    max_el = std::max<int64_t>(max_el, std::max<int64_t>((int64_t)a.m * a.k, (int64_t)a.k * a.n));
  }
  TNA_TRY(upload(mats, g, s));
  const SvdMat *d = g.desc.as<SvdMat>();
  hipLaunchKernelGGL(trunc_kernel, dim3(nm), dim3(256), 0, s, d);
  hipLaunchKernelGGL(write_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(max_el, 256), 2048), 2, nm), dim3(256),
                     0, s, d);
  hipLaunchKernelGGL(complete_kernel, dim3(nm), dim3(256), 0, s, d);
  hipLaunchKernelGGL(gauge_kernel, dim3(max_k, 1, nm), dim3(256), 0, s, d);
  TNA_LAUNCHED("svd.outputs");
  return TNA_OK;
}

void SvdGroup::release() {
  desc.release();
  work_d.release();
  work_i.release();
  if (host) (void)hipHostFree(host);
  if (host_ctr) (void)hipHostFree(host_ctr);
  if (host_fro) (void)hipHostFree(host_fro);
  host = nullptr;
  host_ctr = nullptr;
  host_fro = nullptr;
  host_cap = 0;
}

}  // namespace tna
