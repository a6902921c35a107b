// Internal declarations of the gfx950 library: kernel launchers and the
// context object.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tna.h"

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
bool timing_wanted(const char *name);
void timer_begin(const char *name, hipStream_t s);
void timer_end(const char *name, double flops, double bytes, hipStream_t s);

// ------------------------------------------------------------------ device buffer
// Grow-only device allocation; contents are not preserved across growth.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
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
struct SvdWork;
struct SvdPlan {
  int batch, m, n;
  int R, C;       // working rows / row length (R = min(m,n))
  int trans;      // 1 when m > n (rows of A^T are orthogonalised)
  int nb;         // number of 32-row blocks (even)
  int ksplit;     // Gram K split
  int dtype;      // TNA_F64 / TNA_F32 of the working matrix
};
// Working storage for a batch of SVDs.
struct SvdBuffers {
  DevBuf bw, jt, gram, qt, flags, sig, perm, ctr, scratch;
};
tna_status svd_plan(int batch, int m, int n, int dtype, SvdPlan *p);
// Loads A (or A^T) into the working buffers, runs Jacobi sweeps until none
// rotates (one host read per sweep) or max_sweeps, then sorts the row norms.
// Returns TNA_ERR_NOCONV on the cap.
tna_status svd_run(const SvdPlan &p, SvdBuffers &wb, const void *A, int64_t strideA, int max_sweeps, int *sweeps,
                   hipStream_t s, int *host_ctr);
// Spectrum S (sorted) into S_out (stride), entropy/Z into spec (stride 6).
tna_status svd_spectrum(const SvdPlan &p, SvdBuffers &wb, double *S_out, int64_t strideS, double *spec,
                        hipStream_t s);
// Truncation sums for k from the sorted spectrum S (device spec[2..5]).
tna_status svd_trunc_S(const SvdPlan &p, const double *S, int64_t strideS, int k, double *spec, hipStream_t s);
// Writes U (m x k) and Vt (k x n) from the working buffers, completes null
// vectors, applies the sign gauge, then scale_mode 0 none, 1 scales Vt rows
// by S_j/|S_k|, 2 scales U columns by S_j/|S_k| (|S_k| = spec[4]).
tna_status svd_outputs_S(const SvdPlan &p, SvdBuffers &wb, const double *S, int64_t strideS, int k, void *U,
                         int64_t strideU, void *Vt, int64_t strideVt, int out_type, int scale_mode,
                         const double *spec, hipStream_t s);

// ------------------------------------------------------------------ spectrum
tna_status spectrum_entropy(const double *S, int R, double *spec, int batch, int64_t strideS, hipStream_t s);
tna_status spectrum_trunc(const double *S, int R, int k, double *spec, int batch, int64_t strideS, hipStream_t s);

// ------------------------------------------------------------------ host-side steps (api.cpp)
struct LanczosResult {
  double E = 0.0;
  int iters = 0;
  int converged = 0;
};
// Lowest eigenpair of H_eff (FP64 Lanczos, full CGS2 reorthogonalisation)
// starting from theta (overwritten by the normalised Ritz vector).
tna_status heff_lanczos(tna_ctx c, int chl, int chr, int d, int D, const double *L, const double *R,
                        const double *M12, int prec, double *theta, double *V, double tol, int kmax, int restarts,
                        int fixed_iters, LanczosResult *res);
tna_status env_left(int chl, int k, int d, int D, const double *L, const double *Ml, const double *A, double *T1,
                    double *T2, double *Ln, hipStream_t s);
tna_status env_right(int k, int chr, int d, int D, const double *R, const double *Mr, const double *B, double *T1,
                     double *T2, double *Rn, hipStream_t s);
tna_status pid_update(const tna_pid_params *p, tna_pid_state *st, double s_raw, int *chi_next, double *terms);
tna_status mlp_forward_dev(tna_mlp n, int B, const float *X, float *y);

}  // namespace tna

// ------------------------------------------------------------------ context
struct tna_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int timing = 0;
  tna::DevBuf x, z, lf, rf, m12, part, misc;
  tna::SvdBuffers svd;
  int *host_ctr = nullptr;     // pinned
  double *host_scal = nullptr; // pinned, 64 doubles
};
