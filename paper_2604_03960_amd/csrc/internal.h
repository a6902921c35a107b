// Internal declarations of the gfx950 library: kernel launchers and the
// context object.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tna.h"

struct tna_engine_s;

namespace tna {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
#define TNA_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::tna::set_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
      return TNA_ERR_DEVICE;                                                           \
    }                                                                                  \
  } while (0)
// After a launch: report launch errors; with TNA_DEBUG_SYNC=1 in the
// environment also synchronise the device and report execution errors.
tna_status post_launch(const char *what);
#define TNA_LAUNCHED(what) TNA_TRY(::tna::post_launch(what))
#define TNA_TRY(st)                      \
  do {                                   \
    tna_status s_ = (st);                \
    if (s_ != TNA_OK) return s_;         \
  } while (0)

// ------------------------------------------------------------------ kernel timing
// When enabled (tna_set_timing), launches whose name starts with the filter
// prefix are bracketed by HIP events on their stream; tna_kernel_stats()
// reports per-name launch count, total milliseconds and the algorithmic
// flops and bytes the launch sites declare.
bool timing_on();
// true when timing is on and its filter could match a kernel whose name starts with name_prefix
bool timing_may_match(const char *name_prefix);
bool timing_wanted(const char *name);
void timer_begin(const char *name, hipStream_t s);
void timer_end(const char *name, double flops, double bytes, hipStream_t s);
// adds work known only after the launch (e.g. iterations run) to the last record of `name`
void timer_add_work(const char *name, double flops, double bytes);

// ------------------------------------------------------------------ device buffer
// Grow-only device allocation; contents are not preserved across growth.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  bool borrowed = false;  // a view into a caller-owned workspace: never freed or grown here
  tna_status ensure(size_t need);
  void release();
  template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// ------------------------------------------------------------------ GEMM
// C[M][N] = alpha * op(A) op(B) + beta * C, row-major.  op(A)(i,k) is
// A[i*lda+k] (transA = 0) or A[k*lda+i] (transA = 1); op(B)(k,j) is
// B[k*ldb+j] (transB = 0) or B[j*ldb+k] (transB = 1).  batch copies at
// element strides sA, sB, sC.  Types: A/B/C each double or float; the
// product runs on FP64 MFMA when `f64` is set, otherwise FP32 MFMA.
enum GemmType { G_F64 = 0, G_F32 = 1 };
struct GemmArgs {
  int M, N, K;
  const void *A; int lda; int transA; int typeA;
  const void *B; int ldb; int transB; int typeB;
  void *C; int ldc; int typeC;
  double alpha, beta;
  int batch; int64_t sA, sB, sC;
  int compute;  // G_F64 or G_F32
  int bf16x3;   // compute == G_F32 only: split-bf16 x3 products
};
tna_status gemm(const GemmArgs &g, hipStream_t s);

// Grouped GEMM: one persistent launch for problems of different shapes that
// share transposes, operand types and alpha/beta.  Descriptors live in device
// memory; jB / jC (device ints, may be null) add (*jB) * jB_stride elements to
// B and (*jC) * jC_stride to C at run time; active (device int, may be null)
// skips the problem when zero.
struct GemmProb {
  int M, N, K, lda, ldb, ldc;
  const void *A;
  const void *B;
  void *C;
  const int *jB;
  const int *jC;
  const int *active;
  int64_t jB_stride, jC_stride;
  int tile0, tiles_n;  // filled by gemm_group_tiles
};
struct GemmGroup {
  int transA, transB, typeA, typeB, typeC, compute, tile;
  double alpha, beta;
  double flops, bytes;  // algorithmic work of the whole launch (timing only)
  const char *tag = nullptr;  // timer name prefix (default "gemmg")
  int pairs = 0;              // every problem takes 16-byte operand loads (set by gemm_group_tiles)
};
// Assigns tile ranges for a square tile of the given size; returns the total.  With pairs given,
// *pairs = 1 when every problem's operands can move two elements per 16-byte load (even sizes and
// leading dimensions, 16-byte aligned bases, even device-offset strides), else 0.
int gemm_group_tiles(std::vector<GemmProb> &probs, int tile, int *pairs = nullptr);
tna_status gemm_grouped(const GemmGroup &g, const GemmProb *d, int nprob, int total, hipStream_t s);

// ------------------------------------------------------------------ MPO mixing
// out[o0*os0 + o1*os1 + ooff[j]] = sum_i M[j*I + i] * in[o0*is0 + o1*is1 + ioff[i]]
// for o0 < n0, o1 < n1.  I, J <= 32.  in/out double or float.
struct MixArgs {
  int n0, n1;
  int64_t is0, is1, os0, os1;
  int I, J;
  int ioff[32];
  int ooff[32];
  const void *in; int type_in;
  void *out; int type_out;
  const double *M;  // device, J x I
};
tna_status mix(const MixArgs &a, hipStream_t s);
// Builds mixing matrices from MPO tensors on the device.
//  mode 0 (two-site): M[(s,t,w'')][(w,s',t')] = sum_w' W1[w][w'][s][s'] W2[w'][w''][t][t']
//  mode 1 (left env): M[(s,w')][(w,s')] = W1[w][w'][s][s']
//  mode 2 (right env): M[(t,w)][(w'',t')] = W1[w][w''][t][t']
tna_status build_mix_matrix(int mode, int d, int D, const double *W1, const double *W2, double *M, hipStream_t s);

// ------------------------------------------------------------------ vector kernels
// partial dot products of nv vectors V_i (stride ldv) with w over n
// elements; the fixed-order reduction writes h[i].  part >= nv * 512.
tna_status multidot(const double *V, int64_t ldv, int nv, const double *w, int64_t n, double *h, double *part,
                    hipStream_t s);
// w -= sum_i h[i] V_i ; optionally partial |w|^2 into part and the reduced
// value into *nrm2 (if nrm2 != nullptr).
tna_status axpy_multi(const double *V, int64_t ldv, int nv, const double *h, double *w, int64_t n, double *nrm2,
                      double *part, hipStream_t s);
// y = sum_i c[i] V_i (c device)
tna_status combine(const double *V, int64_t ldv, int nv, const double *c, double *y, int64_t n, hipStream_t s);
// |x|^2 into *out (device), fixed order.
tna_status norm2(const double *x, int64_t n, double *out, double *part, hipStream_t s);
// y = x * (1/sqrt(*nrm2)) if scale_from_nrm2, else y = x * scal
tna_status scale(const double *x, double *y, int64_t n, const double *nrm2, double scal, hipStream_t s);
// counts non-finite entries of x into *flag (int, device; not cleared here)
tna_status check_finite(const double *x, int64_t n, int *flag, hipStream_t s);
tna_status convert_f64_f32(const double *x, float *y, int64_t n, hipStream_t s);
tna_status fill(double *x, int64_t n, double v, hipStream_t s);
tna_status fill_int(int *x, int64_t n, int v, hipStream_t s);
tna_status copy_transpose(const void *A, int m, int n, int type, double *B, hipStream_t s);  // B = A^T as double
tna_status set_identity(double *J, int n, int ld, int batch, int64_t stride, hipStream_t s);

// ------------------------------------------------------------------ SVD
// One truncated SVD (blocked one-sided Jacobi): shape, plan, work buffers,
// input and outputs.  A group of them (one matrix, a uniform batch or
// matrices of different shapes) runs through the same launches, one grid
// z-slice per matrix.
struct SvdMat {
  int m, n, R, C, trans, nb, ksplit, active;  // R = min(m,n) rows of length C are orthogonalised
  int k, dtype, out_type, scale_mode;         // kept rank; scale 0 none, 1 Vt rows, 2 U columns by S_j/|S_k|
  int inner_max, fused;                        // cap on inner Jacobi sweeps; whole Jacobi in one workgroup
  double tol, eps_target;
  double thr;                                  // > 0: spec[24] = number of values above thr (spec holds 32)
  const void *A;                               // m x n (dtype)
  double *bw, *jt, *gram, *qt, *sig;           // work
  double *S;                                   // R sorted values (output)
  double *spec;                                // 32 doubles: Z, S_vN, eps, eps^2/Z, |S_k|, gap, k_needed, sweeps,
                                               // S_0..S_15, [24] values above thr, [25] values above 1e-12 S_0
  int *skip, *perm, *ctr;                      // work
  void *U, *Vt;                                // m x k, k x n (out_type)
  double *fro2;                                // work: [0] |A|_F^2, [1] largest squared row norm below a QR stop
  int precond;                                 // 1: rows start from the R factor of a Householder QR
  int Ra;  // rows [0, Ra) take part in the sweeps: R, or the point where a QR start stopped because every later
           // row was at the rounding level (rows_scaled only; such rows are never rotated)
  int *cperm, *pinv;                           // work: original column at position c, and its inverse (C each)
  double *qv, *qws;                            // work: reflectors as rows (R x R), blocked-product scratch
  double noise_rel;  // > 0: the input carries noise of about noise_rel |A|_F (an FP32 operator upstream); rows
                     // below it count as rounding-level rows, and the numerical rank spec[25] counts values above
                     // noise_rel S_0 (default: 1e-12 S_0)
  int rows_scaled;  // 1: the factor built from the orthogonalised rows (Vt, or U when trans) leaves the call
                    // multiplied by the singular values or unused, so it need not be orthonormal: rows at the
                    // rounding level stay unrotated after the QR start too, and null vectors are not completed
  int pad4_;
};
struct SvdGroup {
  DevBuf desc, work_d, work_i;
  void *host = nullptr;
  size_t host_cap = 0;
  int *host_ctr = nullptr;
  double *host_fro = nullptr;  // pinned: squared Frobenius norms of the inputs (finiteness check), then
                               // (|A|_F^2, largest trailing row norm^2) pairs during a QR start
  void release();
};
// orient (square matrices only): 0 by shape (rows of A), 1 rows of A, 2 rows of A^T (columns of A)
tna_status svd_plan_mat(int m, int n, int dtype, int batch_hint, SvdMat *a, int orient = 0);
size_t svd_work_doubles(const SvdMat &a);
size_t svd_work_ints(const SvdMat &a);
void svd_bind_work(SvdMat *a, double *dw, int *iw);
// Loads every A, runs Jacobi sweeps until a matrix's sweep rotates nothing
// (one host read per sweep), then sorts and writes S, spec[0,1,6,7,8..23].
// A rows_scaled matrix whose QR start stops early leaves with Ra < R and nb, ksplit
// re-planned for its Ra rows (plan every call afresh).
// Returns TNA_ERR_NOCONV if any matrix hit max_sweeps.  With defer_fused, the
// matrices on the single-workgroup Jacobi paths are not read back here: their
// sweep counts (negative when not converged) are in spec[7].
tna_status svd_group_run(std::vector<SvdMat> &mats, SvdGroup &g, int max_sweeps, std::vector<int> &sweeps,
                         hipStream_t s,
                         bool defer_fused = false);
// For each matrix's k: spec[2..5], U and Vt (completion of null vectors,
// sign gauge, scaling).
tna_status svd_group_outputs(std::vector<SvdMat> &mats, SvdGroup &g, hipStream_t s);

// ------------------------------------------------------------------ grouped (batched-chain) kernels
struct MixProb {
  int n0, n1;
  const void *in;
  void *out;
  int64_t is0, is1, os0, os1;
  int ich1, ich2, och1, och2;  // channel i = (i1, i2) sits at i1*ich1 + i2*ich2
  const double *M;             // J x I
  const int *active;           // device flag, may be null
  // optional (null = off): the input channels i1 = I1-1 read from in_last (FP64) at
  // o0*is0_last + o1*is1 + i2*ich2 plus (*jin)*jin_stride, and the output channels j2 = 0 go to
  // out_first (FP64) at o0*os0_first + o1*os1 + j1*och1_first plus (*jout)*jout_stride
  const double *in_last;
  int64_t is0_last;
  const int *jin;
  int64_t jin_stride;
  double *out_first;
  int64_t os0_first;
  int och1_first;
  const int *jout;
  int64_t jout_stride;
};
// max |E[a][w][a'] - delta(a, a')| over a, a' < chi into *out as the bit pattern of a non-negative
// double (*out zeroed beforehand); E is chi x D x chi.  grid-stride.
tna_status ident_deviation(const double *E, int chi, int D, int w, double *out, hipStream_t s);
tna_status mix_grouped(const MixProb *d, int nprob, int64_t max_elems, int I1, int I2, int J1, int J2, int f32,
                       hipStream_t s);
// One chain's Lanczos state for the current sweep step (device pointers).
struct LzProb {
  int64_t n;      // vector length
  int G, nkeep;   // partial-sum blocks; Ritz vector length
  double *V;      // (kmax+1) x n Krylov basis (V_{j+1} doubles as w)
  double *theta;  // start vector in, normalised Ritz vector out
  int *j, *active;
  double *h1, *h2, *part1, *part2, *nrm2, *rec, *y;  // rec: {alpha_j, beta_j^2}
};
// bytes_hint: algorithmic bytes of one dot (or update) pass, for kernel timing
tna_status lz_iteration(const LzProb *d, int nch, int maxG, int kmax, double bytes_hint, hipStream_t s);
tna_status lz_start(const LzProb *d, int nch, int maxG, hipStream_t s);
tna_status lz_ritz(const LzProb *d, int nch, int maxG, hipStream_t s);
// Single-workgroup Lanczos for short vectors (all of H_eff's operands in LDS).
constexpr int LZ_HMAX = 128;                       // >= kmax + 1
constexpr size_t LZ_SMALL_LDS_MAX = 160 * 1024;    // LDS of one gfx950 workgroup
struct LzSmall {
  int chl, chr, kmax, ac;  // ac: left indices per chunk of the three H_eff products
  int D, pad_;
  const double *L, *R, *M; // L[a][w][a'], R[c][w''][c'], mixing matrix (D d^2)^2
  double *V;               // Krylov basis, V_0 set
  int *j;
  const int *active;
  double *rec;             // 2 (kmax + 1): alpha_j, beta_j^2
};
// LDS bytes of one workgroup; f32: the H_eff operands are held and multiplied in FP32
size_t lz_small_lds(int chl, int chr, int d, int D, int ac, int f32);
// Runs up to `iters` iterations for every active chain; lds = max over chains.
tna_status lz_small(const LzSmall *d, int nch, int D, int dsq, int iters, size_t lds, int f32, hipStream_t s);
struct CvtProb {
  const double *src;
  float *dst;
  int64_t n;
};
tna_status convert_grouped(const CvtProb *d, int nprob, hipStream_t s);

// ------------------------------------------------------------------ step engine (batch.cpp)
// One lockstep bond visit of a set of chains (a single chain is a set of one).
typedef ::tna_engine_s *tna_engine;
tna_status engine_create(int nslot, tna_engine *out);
void engine_destroy(tna_engine e);
hipStream_t engine_stream(tna_engine e);
void engine_stats(tna_engine e, tna_batch_stats *st);
tna_status engine_step(tna_engine en, const std::vector<tna_dmrg> &ch, const std::vector<int> &slot,
                       const std::vector<int> &bond, const std::vector<int> &half, std::vector<double> &E_out,
                       std::vector<tna_visit_log *> &logs, tna_status *worst);
double tridiag_lowest_host(int n, const double *a, const double *b, double *y);

// ------------------------------------------------------------------ stand-alone H_eff (api.cpp)
struct HeffOp {
  int chl, chr, d, D;
  const void *L;  // double or float (prec)
  const void *R;
  const double *M12;
  void *X, *Z;    // scratch, D d^2 chl chr elements each
  int prec;
};
tna_status heff_device(const HeffOp &h, const double *x, double *out, hipStream_t s);
tna_status heff_check_args(tna_ctx c, int chi_l, int chi_r, int d, int D, const double *L, const double *W1,
                           const double *W2, const double *R, const double *theta, double *out, int prec);
// noalloc.cpp: records the calling device's address of the fixed scratch array (device current)
tna_status noalloc_init(int device);

// ------------------------------------------------------------------ host-side steps (api.cpp)
tna_status env_left(int chl, int k, int d, int D, const double *L, const double *Ml, const double *A, double *T1,
                    double *T2, double *Ln, hipStream_t s);
tna_status env_right(int k, int chr, int d, int D, const double *R, const double *Mr, const double *B, double *T1,
                     double *T2, double *Rn, hipStream_t s);
tna_status pid_update(const tna_pid_params *p, tna_pid_state *st, double s_raw, int *chi_next, double *terms);
tna_status entropy_update(const tna_pid_params *p, double gamma, tna_pid_state *st, double s_raw, int *chi_next,
                          double *terms);
// forward pass on stream s (the caller's stream: the sweep engine passes its own, so the inputs it
// uploaded and the outputs it reads back stay ordered with the launch)
tna_status mlp_forward_dev(tna_mlp n, int B, const float *X, float *y, hipStream_t s);

}  // namespace tna

// ------------------------------------------------------------------ context
struct tna_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int timing = 0;
  void *ws = nullptr;  // caller-owned device workspace (tna_set_workspace), or null
  size_t ws_bytes = 0;
  tna::DevBuf x, z, lf, rf, m12, part, misc, spec;
  tna::SvdGroup svd;
  int *host_ctr = nullptr;     // pinned
  double *host_scal = nullptr; // pinned, 64 doubles
  int children = 0;            // live DMRG runs and networks made from this context
};

// ------------------------------------------------------------------ DMRG chain state
struct tna_dmrg_s {
  tna_ctx ctx;
  int N, d, D;
  tna_pid_params pid;
  tna_dmrg_opts opts;
  std::vector<int> chi;                 // N-1 realised bond dims
  std::vector<tna_pid_state> st;        // N-1 controllers
  std::vector<tna::DevBuf> A, Le, Re;   // site tensors, left envs (site i), right envs (site i)
  tna::DevBuf W, M12, Ml, Mr;           // MPO tensors and mixing matrices (device)
  tna::DevBuf V, T1, T2, spec, S;       // Lanczos basis, env scratch, spectrum
  int sweeps_done = 0;
  int centre = 0;                       // site of the orthogonality centre (0 after create and after a sweep)
  double *host_stage = nullptr;         // pinned: per-visit readbacks
  // learned scheduler
  tna_mlp sched = nullptr;
  std::vector<std::array<double, 8>> hist;  // last EMA entropies per bond (oldest first)
  std::vector<int> nhist, pred;             // history length, pending proposal (0 = none)
  tna::tna_engine engine = nullptr;          // the step engine this chain's sweeps run on
  int CL(int i) const { return i == 0 ? 1 : chi[i - 1]; }
  int CR(int i) const { return i == N - 1 ? 1 : chi[i]; }
};
