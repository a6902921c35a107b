// Dense contractions of the two-site DMRG step on the gfx950 matrix cores.
//
// One kernel template serves every GEMM of the path: H_eff stages S1 (L x theta)
// and S4 (Z x R^T), the environment updates, theta formation.  A workgroup owns
// a BM x BN tile of C: 64 x 64 with 256 threads (four wave64s in a 2 x 2
// arrangement), or 128 x 128 with 512 threads (eight wave64s, 4 x 2; half the
// operand traffic per flop of the small tile at the same registers per wave, and
// two workgroups per compute unit).  K advances in steps of 16 through two LDS
// buffers (the next slab is fetched into registers while the current one feeds
// the MFMAs).  Each wave accumulates its share of the tile as 16 x 16 MFMA tiles:
//   FP64: v_mfma_f64_16x16x4_f64, FP32: v_mfma_f32_16x16x4_f32.
// Operand layout of the 16x16x4 MFMAs (lane l, result register r = 0..3):
//   A[i][k]: lane i + 16k      B[k][j]: lane j + 16k
//   D[i][j]: lane j + 16(i%4), reg i/4 for f64;  lane j + 16(i/4), reg i%4 for f32.
#include <cstdint>
#include <cstdio>
#include <type_traits>

#include "internal.h"

namespace tna {
namespace {

typedef double v2d __attribute__((ext_vector_type(2)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { typedef v4d type; };
template <> struct Acc<float> { typedef v4f type; };

__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// row of result register r held by lane group lk (= lane / 16)
__device__ inline int mfma_row(double, int lk, int r) { return 4 * r + lk; }
__device__ inline int mfma_row(float, int lk, int r) { return 4 * lk + r; }

struct GemmDev {
  int M, N, K, lda, ldb, ldc;
  const void *A;
  const void *B;
  void *C;
  double alpha, beta;
  int64_t sA, sB, sC;
};

constexpr int BK = 16;

template <typename T, int BM, int BN> struct TileLds {
  T As[2][BK][BM + 1];
  T Bs[2][BK][BN + 1];
};

// threads of the workgroup that owns a BM x BN tile, and its waves along M
template <int BM> struct TileShape;
// (MINW: waves per SIMD the register allocation must leave room for; two 128 x 128
// workgroups per compute unit need four)
template <> struct TileShape<64> { static constexpr int NT = 256, WR = 2, MINW = 4; };
template <> struct TileShape<128> { static constexpr int NT = 512, WR = 4, MINW = 4; };

// Device-memory pointers in the global address space: operand pointers read from a descriptor in
// memory are generic to the compiler, whose flat accesses count against the LDS waits as well and so
// tie the operand prefetch to the LDS reads of the products.
template <typename X> using gp = X __attribute__((address_space(1))) *;

// One BM x BN tile of C = alpha op(A) op(B) + beta C at (m0, n0).
template <typename T, typename TA, typename TB, typename TC, int BM, int BN, bool TRA, bool TRB, bool PAIRS>
__device__ __forceinline__ void gemm_tile(gp<const TA> __restrict__ A, int lda, gp<const TB> __restrict__ B, int ldb,
                                          gp<TC> __restrict__ C, int ldc, int M, int N, int K, double alpha,
                                          double beta, int m0, int n0, TileLds<T, BM, BN> &L) {
  constexpr int NT = TileShape<BM>::NT, WR = TileShape<BM>::WR, WC = NT / 64 / WR;
  constexpr int WM = BM / WR, WN = BN / WC;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int LA = BM * BK / NT;  // A elements per thread per slab
  constexpr int LB = BN * BK / NT;
  static_assert(BM % WR == 0 && BN % WC == 0 && WM % 16 == 0 && WN % 16 == 0 && LA >= 2 && LB >= 2 &&
                    LA % 2 == 0 && LB % 2 == 0, "tile shape");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int lr = lane & 15, lk = lane >> 4;

  // element coordinates this thread loads (tile-local)
  auto a_coord = [&](int p, int &i, int &k) {
    if (!TRA) { k = tid % BK; i = tid / BK + (NT / BK) * p; }
    else { i = tid % BM; k = tid / BM + (NT / BM) * p; }
  };
  auto b_coord = [&](int p, int &k, int &j) {
    if (!TRB) { j = tid % BN; k = tid / BN + (NT / BN) * p; }
    else { k = tid % BK; j = tid / BK + (NT / BK) * p; }
  };

  T ra[LA], rb[LB];
  // PAIRS (FP64 operands with even sizes and leading dimensions and 16-byte aligned bases, checked on
  // the host for the whole launch): two consecutive elements per 16-byte load, half the load
  // instructions of the element-wise form that serves every other case.
  constexpr bool pairs = PAIRS && std::is_same<T, double>::value && std::is_same<TA, double>::value &&
                         std::is_same<TB, double>::value;
  // pair p of a thread: A rows/columns (i, k) and B (k, j) of its first element; the second element
  // follows along the contiguous index (k for A, i for A^T; j for B, k for B^T)
  auto a_pair = [&](int p, int &i, int &k) {
    if (!TRA) { k = (tid % (BK / 2)) * 2; i = tid / (BK / 2) + (NT / (BK / 2)) * p; }
    else { i = (tid % (BM / 2)) * 2; k = tid / (BM / 2) + (NT / (BM / 2)) * p; }
  };
  auto b_pair = [&](int p, int &k, int &j) {
    if (!TRB) { j = (tid % (BN / 2)) * 2; k = tid / (BN / 2) + (NT / (BN / 2)) * p; }
    else { k = (tid % (BK / 2)) * 2; j = tid / (BK / 2) + (NT / (BK / 2)) * p; }
  };
  auto load_pairs = [&](int k0) {
#pragma unroll
    for (int p = 0; p < LA / 2; ++p) {
      int i, k;
      a_pair(p, i, k);
      const int gi = m0 + i, gk = k0 + k;
      v2d v = {0.0, 0.0};
      if (gi < M && gk < K)
        v = *(gp<const v2d>)((gp<const double>)A + (TRA ? (int64_t)gk * lda + gi : (int64_t)gi * lda + gk));
      ra[2 * p] = v.x;
      ra[2 * p + 1] = v.y;
    }
#pragma unroll
    for (int p = 0; p < LB / 2; ++p) {
      int k, j;
      b_pair(p, k, j);
      const int gk = k0 + k, gj = n0 + j;
      v2d v = {0.0, 0.0};
      if (gj < N && gk < K)
        v = *(gp<const v2d>)((gp<const double>)B + (TRB ? (int64_t)gj * ldb + gk : (int64_t)gk * ldb + gj));
      rb[2 * p] = v.x;
      rb[2 * p + 1] = v.y;
    }
  };
  auto store_pairs = [&](int buf) {
#pragma unroll
    for (int p = 0; p < LA / 2; ++p) {
      int i, k;
      a_pair(p, i, k);
      L.As[buf][k][i] = ra[2 * p];
      L.As[buf][k + (TRA ? 0 : 1)][i + (TRA ? 1 : 0)] = ra[2 * p + 1];
    }
#pragma unroll
    for (int p = 0; p < LB / 2; ++p) {
      int k, j;
      b_pair(p, k, j);
      L.Bs[buf][k][j] = rb[2 * p];
      L.Bs[buf][k + (TRB ? 1 : 0)][j + (TRB ? 0 : 1)] = rb[2 * p + 1];
    }
  };
  auto load = [&](int k0) {
    if constexpr (pairs) {
      load_pairs(k0);
      return;
    }
#pragma unroll
    for (int p = 0; p < LA; ++p) {
      int i, k;
      a_coord(p, i, k);
      int gi = m0 + i, gk = k0 + k;
      T v = T(0);
      if (gi < M && gk < K) v = T(TRA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk]);
      ra[p] = v;
    }
#pragma unroll
    for (int p = 0; p < LB; ++p) {
      int k, j;
      b_coord(p, k, j);
      int gk = k0 + k, gj = n0 + j;
      T v = T(0);
      if (gj < N && gk < K) v = T(TRB ? B[(int64_t)gj * ldb + gk] : B[(int64_t)gk * ldb + gj]);
      rb[p] = v;
    }
  };
  auto store = [&](int buf) {
    if constexpr (pairs) {
      store_pairs(buf);
      return;
    }
#pragma unroll
    for (int p = 0; p < LA; ++p) {
      int i, k;
      a_coord(p, i, k);
      L.As[buf][k][i] = ra[p];
    }
#pragma unroll
    for (int p = 0; p < LB; ++p) {
      int k, j;
      b_coord(p, k, j);
      L.Bs[buf][k][j] = rb[p];
    }
  };

  typename Acc<T>::type acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = typename Acc<T>::type{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
    // this wave's MFMA block at raised issue priority (the next slab's loads are out; the LDS store
    // and the barrier follow it), with the compiler's MFMA / LDS-read interleaving strategy 0
    __builtin_amdgcn_s_setprio(1);
    __builtin_amdgcn_iglp_opt(0);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = L.As[buf][kk + lk][wr * WM + a * 16 + lr];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = L.Bs[buf][kk + lk][wc * WN + b * 16 + lr];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
    }
    __builtin_amdgcn_s_setprio(0);
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wr * WM + a * 16 + mfma_row(T(0), lk, r);
        int col = n0 + wc * WN + b * 16 + lr;
        if (row < M && col < N) {
          double v = alpha * (double)acc[a][b][r];
          int64_t idx = (int64_t)row * ldc + col;
          if (beta != 0.0) v += beta * (double)C[idx];
          C[idx] = (TC)v;
        }
      }
}

template <typename T, typename TA, typename TB, typename TC, int BM, int BN, bool TRA, bool TRB, bool PAIRS>
__global__ __launch_bounds__(TileShape<BM>::NT, TileShape<BM>::MINW) void gemm_kernel(GemmDev g) {
  __shared__ TileLds<T, BM, BN> L;
  const int z = blockIdx.z;
  gemm_tile<T, TA, TB, TC, BM, BN, TRA, TRB, PAIRS>((gp<const TA>)(static_cast<const TA *>(g.A) + g.sA * z), g.lda,
                                             (gp<const TB>)(static_cast<const TB *>(g.B) + g.sB * z), g.ldb,
                                             (gp<TC>)(static_cast<TC *>(g.C) + g.sC * z), g.ldc, g.M, g.N, g.K,
                                             g.alpha, g.beta, blockIdx.y * BM, blockIdx.x * BN, L);
}

// Persistent grouped GEMM: the grid walks a static work list of tiles that
// spans every problem of the group (problem p owns tiles [tile0, tile0 +
// tiles_m * tiles_n)); operand pointers may carry a device-side element offset
// (*jB) * jB_stride / (*jC) * jC_stride, read at run time, so a captured
// launch serves every Lanczos iteration.
template <typename T, typename TA, typename TB, typename TC, int BM, int BN, bool TRA, bool TRB, bool PAIRS>
__global__ __launch_bounds__(TileShape<BM>::NT, TileShape<BM>::MINW) void gemm_grouped_kernel(
    const GemmProb *probs, int nprob, int total, double alpha, double beta) {
  __shared__ TileLds<T, BM, BN> L;
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (probs[mid].tile0 <= t) lo = mid;
      else hi = mid - 1;
    }
    const GemmProb &p = probs[lo];
    if (p.active && !*p.active) continue;
    const int local = t - p.tile0;
    const int tm = local / p.tiles_n, tn = local - tm * p.tiles_n;
    const TB *B = static_cast<const TB *>(p.B) + (p.jB ? (int64_t)(*p.jB) * p.jB_stride : 0);
    TC *C = static_cast<TC *>(p.C) + (p.jC ? (int64_t)(*p.jC) * p.jC_stride : 0);
    gemm_tile<T, TA, TB, TC, BM, BN, TRA, TRB, PAIRS>((gp<const TA>)static_cast<const TA *>(p.A), p.lda, (gp<const TB>)B,
                                               p.ldb, (gp<TC>)C, p.ldc, p.M, p.N,
                                               p.K, alpha, beta, tm * BM, tn * BN, L);
    __syncthreads();
  }
}

template <typename T, typename TA, typename TB>
constexpr bool all_f64() {
  return std::is_same<T, double>::value && std::is_same<TA, double>::value && std::is_same<TB, double>::value;
}
inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <typename T, typename TA, typename TB, typename TC, int BM, int BN>
tna_status launch_tile(const GemmArgs &a, const GemmDev &d, hipStream_t s) {
  constexpr int NT = TileShape<BM>::NT;
  dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM, a.batch);
  if (grid.y > 65535 || grid.z > 65535) {
    set_error("gemm: grid too large");
    return TNA_ERR_ARG;
  }
  char name[64] = "";
  if (timing_on()) {
    std::snprintf(name, sizeof name, "gemm.%s.%dx%d.%c%c", sizeof(T) == 8 ? "f64" : "f32", BM, BN,
                  a.transA ? 'T' : 'N', a.transB ? 'T' : 'N');
    timer_begin(name, s);
  }
  if (a.transA && a.transB) {
    set_error("gemm: transA && transB not built");
    return TNA_ERR_UNSUPPORTED;
  }
  auto go = [&](auto pairs_c) {
    constexpr bool P = decltype(pairs_c)::value;
    if (!a.transA && !a.transB)
      hipLaunchKernelGGL((gemm_kernel<T, TA, TB, TC, BM, BN, false, false, P>), grid, dim3(NT), 0, s, d);
    else if (!a.transA)
      hipLaunchKernelGGL((gemm_kernel<T, TA, TB, TC, BM, BN, false, true, P>), grid, dim3(NT), 0, s, d);
    else
      hipLaunchKernelGGL((gemm_kernel<T, TA, TB, TC, BM, BN, true, false, P>), grid, dim3(NT), 0, s, d);
  };
  if constexpr (all_f64<T, TA, TB>()) {
    const bool pairs = ((a.lda | a.ldb | a.M | a.N | a.K) & 1) == 0 && aligned16(a.A) && aligned16(a.B) &&
                       (a.batch == 1 || ((a.sA | a.sB) & 1) == 0);
    if (pairs) go(std::true_type{});
    else go(std::false_type{});
  } else {
    go(std::false_type{});
  }
  if (name[0]) {
    const double mnk = (double)a.M * a.N * a.K * a.batch;
    const double by = ((double)a.M * a.K * sizeof(TA) + (double)a.K * a.N * sizeof(TB) + (double)a.M * a.N * sizeof(TC)) *
                      a.batch;
    timer_end(name, 2.0 * mnk, by, s);
  }
  TNA_LAUNCHED("gemm.hip:1");
  return TNA_OK;
}

// Tile choice: the 128 x 128 tile when the grid still has >= 2 waves of
// workgroups on 256 CUs, else 64 x 64 to spread small problems.
template <typename T, typename TA, typename TB, typename TC>
tna_status launch_types(const GemmArgs &a, const GemmDev &d, hipStream_t s) {
  int64_t big = (int64_t)((a.M + 127) / 128) * ((a.N + 127) / 128) * a.batch;
  if (big >= 512) return launch_tile<T, TA, TB, TC, 128, 128>(a, d, s);
  return launch_tile<T, TA, TB, TC, 64, 64>(a, d, s);
}

template <typename T, typename TA, typename TB, typename TC, int BM, int BN>
tna_status launch_grouped(const GemmGroup &g, const GemmProb *d, int nprob, int total, hipStream_t s) {
  constexpr int NT = TileShape<BM>::NT;
  int grid = total < 2048 ? total : 2048;
  if (grid < 1) return TNA_OK;
  char name[64] = "";
  if (timing_on()) {
    std::snprintf(name, sizeof name, "%s.%s.%dx%d.%c%c", g.tag ? g.tag : "gemmg", sizeof(T) == 8 ? "f64" : "f32", BM,
                  BN, g.transA ? 'T' : 'N', g.transB ? 'T' : 'N');
    timer_begin(name, s);
  }
  if (g.transA && g.transB) {
    set_error("gemm_grouped: transA && transB not built");
    return TNA_ERR_UNSUPPORTED;
  }
  auto go = [&](auto pairs_c) {
    constexpr bool P = decltype(pairs_c)::value;
    if (!g.transA && !g.transB)
      hipLaunchKernelGGL((gemm_grouped_kernel<T, TA, TB, TC, BM, BN, false, false, P>), dim3(grid), dim3(NT), 0, s,
                         d, nprob, total, g.alpha, g.beta);
    else if (!g.transA)
      hipLaunchKernelGGL((gemm_grouped_kernel<T, TA, TB, TC, BM, BN, false, true, P>), dim3(grid), dim3(NT), 0, s,
                         d, nprob, total, g.alpha, g.beta);
    else
      hipLaunchKernelGGL((gemm_grouped_kernel<T, TA, TB, TC, BM, BN, true, false, P>), dim3(grid), dim3(NT), 0, s,
                         d, nprob, total, g.alpha, g.beta);
  };
  if constexpr (all_f64<T, TA, TB>()) {
    if (g.pairs) go(std::true_type{});
    else go(std::false_type{});
  } else {
    go(std::false_type{});
  }
  if (name[0]) timer_end(name, g.flops, g.bytes, s);
  TNA_LAUNCHED("gemm.grouped");
  return TNA_OK;
}

template <typename T, typename TA, typename TB, typename TC>
tna_status grouped_types(const GemmGroup &g, const GemmProb *d, int nprob, int total, hipStream_t s) {
  if (g.tile == 128) return launch_grouped<T, TA, TB, TC, 128, 128>(g, d, nprob, total, s);
  return launch_grouped<T, TA, TB, TC, 64, 64>(g, d, nprob, total, s);
}

}  // namespace

int gemm_group_tiles(std::vector<GemmProb> &probs, int tile, int *pairs) {
  int total = 0;
  bool all_pairs = true;
  for (auto &p : probs) {
    p.tile0 = total;
    p.tiles_n = (p.N + tile - 1) / tile;
    const int tm = (p.M + tile - 1) / tile;
    total += (p.M > 0 && p.N > 0) ? tm * p.tiles_n : 0;
    all_pairs = all_pairs && ((p.lda | p.ldb | p.M | p.N | p.K) & 1) == 0 && aligned16(p.A) && aligned16(p.B) &&
                (!p.jB || (p.jB_stride & 1) == 0);
  }
  if (pairs) *pairs = all_pairs ? 1 : 0;
  return total;
}

tna_status gemm_grouped(const GemmGroup &g, const GemmProb *d, int nprob, int total, hipStream_t s) {
  if (nprob < 1 || total < 1) return TNA_OK;
  const int code = g.typeA * 4 + g.typeB * 2 + g.typeC;
  if (g.compute == G_F64) {
    if (code != 0) {
      set_error("gemm_grouped: FP64 compute takes double operands");
      return TNA_ERR_UNSUPPORTED;
    }
    return grouped_types<double, double, double, double>(g, d, nprob, total, s);
  }
  switch (code) {
    case 0: return grouped_types<float, double, double, double>(g, d, nprob, total, s);
    case 5: return grouped_types<float, float, double, float>(g, d, nprob, total, s);
    case 6: return grouped_types<float, float, float, double>(g, d, nprob, total, s);
    case 7: return grouped_types<float, float, float, float>(g, d, nprob, total, s);
  }
  set_error("gemm_grouped: FP32 operand combination not built");
  return TNA_ERR_UNSUPPORTED;
}

tna_status gemm(const GemmArgs &a, hipStream_t s) {
  if (a.M < 0 || a.N < 0 || a.K < 0 || a.batch < 1) {
    set_error("gemm: negative size");
    return TNA_ERR_ARG;
  }
  if (a.M == 0 || a.N == 0) return TNA_OK;
  GemmDev d{a.M, a.N, a.K, a.lda, a.ldb, a.ldc, a.A, a.B, a.C, a.alpha, a.beta, a.sA, a.sB, a.sC};
  if (a.K == 0) d.alpha = 0.0;
  const int code = a.typeA * 4 + a.typeB * 2 + a.typeC;  // 0 = all double
  if (a.compute == G_F64) {
    if (code != 0) {
      set_error("gemm: FP64 compute takes double operands");
      return TNA_ERR_UNSUPPORTED;
    }
    return launch_types<double, double, double, double>(a, d, s);
  }
  switch (code) {
    case 0: return launch_types<float, double, double, double>(a, d, s);
    case 1: return launch_types<float, double, double, float>(a, d, s);
    case 5: return launch_types<float, float, double, float>(a, d, s);
    case 6: return launch_types<float, float, float, double>(a, d, s);
    case 7: return launch_types<float, float, float, float>(a, d, s);
  }
  set_error("gemm: FP32 operand combination not built");
  return TNA_ERR_UNSUPPORTED;
}

}  // namespace tna
