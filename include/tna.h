/*
 * tna.h -- C ABI of the MI355X (gfx950) two-site DMRG hot path with an
 * entropy-EMA-PID bond-dimension controller (arXiv 2604.03960).
 *
 * Conventions shared by every entry point
 *  - All arrays are row-major.  Tensors named "device" live in device memory
 *    owned by the caller (e.g. PyTorch tensors passed as data pointers); the
 *    library never frees them.  "host" arrays are ordinary CPU memory.
 *  - site tensor  A_i[a][s][b]        (chi_{i-1}, d, chi_i)
 *    MPO tensor   W_i[wl][wr][s][s']  (D, D, d, d), s = output/bra, s' = input/ket
 *    left env     L[a][w][a']         (chi_l, D, chi_l)   bra, MPO, ket
 *    right env    R[b][w][b']         (chi_r, D, chi_r)   bra, MPO, ket
 *    two-site     theta[a][s][t][b]   (chi_l, d, d, chi_r) = matrix (chi_l d) x (d chi_r)
 *    The left boundary selects MPO row D-1 and the right boundary column 0.
 *  - Work is enqueued on the context's stream and is asynchronous unless the
 *    comment says the call synchronises.  Every call returns a tna_status;
 *    nothing throws across the ABI.  On TNA_ERR_ARG nothing has been launched.
 *    tna_last_error() returns a thread-local message for the last failure.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef TNA_H
#define TNA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TNA_OK = 0,
  TNA_ERR_ARG = 1,         /* bad dimension, pointer or parameter */
  TNA_ERR_NOMEM = 2,       /* device or pinned-host allocation failed */
  TNA_ERR_DEVICE = 3,      /* a HIP runtime call failed */
  TNA_ERR_NOCONV = 4,      /* iteration cap reached; the best result so far is written */
  TNA_ERR_NONFINITE = 5,   /* NaN or Inf met in the input or in an intermediate */
  TNA_ERR_UNSUPPORTED = 6  /* valid request this build does not implement */
} tna_status;

typedef enum { TNA_F64 = 0, TNA_F32 = 1 } tna_dtype;

/* Arithmetic of the effective-Hamiltonian matvec.  theta and the result are
 * always FP64; F32 converts the operands to FP32, accumulates in FP32 on the
 * matrix cores and stores FP64.  BF16X3 splits each FP32 operand x into
 * hi = bf16(x), lo = bf16(x - hi) and forms hi*hi + hi*lo + lo*hi in FP32. */
typedef enum { TNA_HEFF_F64 = 0, TNA_HEFF_F32 = 1, TNA_HEFF_BF16X3 = 2 } tna_prec;

typedef struct tna_ctx_s *tna_ctx;

/* ---------------------------------------------------------------- context */
/* Creates a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
tna_status tna_create(tna_ctx *out, int device, void *hip_stream);
/* Destroys the context.  Objects made from it (DMRG runs, batches, networks) must
 * be destroyed first: while any is alive the call returns TNA_ERR_ARG and frees
 * nothing (a host-side count, no HIP call).  NULL is a no-op. */
tna_status tna_destroy(tna_ctx ctx);
tna_status tna_set_stream(tna_ctx ctx, void *hip_stream);
/* Waits for all work the context enqueued.  Synchronises. */
tna_status tna_synchronize(tna_ctx ctx);
const char *tna_last_error(void);
/* Kernel timing.  With enable != 0, every launch whose kernel name starts
 * with `prefix` (NULL or "" = all) is bracketed by HIP events on its stream;
 * this perturbs the timing of small launches, so filter to the kernel of
 * interest.  tna_kernel_stats() synchronises, then writes a JSON array of
 * {name, count, ms, flops, bytes} (flops and bytes: the algorithmic amounts
 * the launch sites declare, summed over launches) into out (cap bytes) and
 * clears the counters if reset != 0. */
/* Caller-owned scratch.  tna_workspace_size: device bytes one call needs, for
 * op "heff_apply" with dims {chi_l, chi_r, d, D, prec} or "svd_truncate" with dims
 * {m, n, dtype, batch} (batch 1 for tna_svd_truncate).  tna_set_workspace: from
 * then on tna_heff_apply and tna_svd_truncate(_batched) on ctx take their scratch
 * from [dev_ptr, dev_ptr + bytes) (caller-owned device memory, e.g. a torch uint8
 * tensor) instead of context-owned buffers; a call needing more returns
 * TNA_ERR_NOMEM and launches nothing.  NULL (or 0 bytes) returns to context-owned
 * scratch.  The workspace must stay valid while calls on ctx are in flight; calls on
 * one ctx share it (they are ordered on the ctx stream).  Waits for the ctx stream. */
tna_status tna_workspace_size(tna_ctx ctx, const char *op, const int64_t *dims, size_t *bytes);
tna_status tna_set_workspace(tna_ctx ctx, void *dev_ptr, size_t bytes);
tna_status tna_set_timing(tna_ctx ctx, int enable, const char *prefix);
tna_status tna_kernel_stats(tna_ctx ctx, char *out, size_t cap, int reset);

/* ---------------------------------------------------------------- models */
/* Bulk MPO tensors of an open chain (host).  model 0: XXZ,
 * H = J sum[(S+S- + S-S+)/2 + Delta Sz Sz] - hz sum Sz, params {J, Delta, hz}
 * (Eq. 20 is J=1, Delta=1, hz=0), D = 5.  model 1: J1-J2 Heisenberg, params
 * {J1, J2}, D = 8.  model 2: transverse-field Ising in Pauli units,
 * H = -J sum sz sz - h sum sx, params {J, h}, D = 3.  W receives N copies of
 * the D x D x 2 x 2 tensor; *D_out the bond dimension.  Host only. */
tna_status tna_mpo_build(int model, int N, const double *params, double *W, int *D_out);

/* ---------------------------------------------------------------- H_eff */
/* Two-site effective Hamiltonian of Eq. (18) applied to theta:
 *   out[a][s][t][b] = sum L[a][w][a'] W1[w][w'][s][s'] W2[w'][w''][t][t']
 *                         R[b][w''][b'] theta[a'][s'][t'][b']
 * L (chi_l,D,chi_l), W1 and W2 (D,D,d,d), R (chi_r,D,chi_r), theta and out
 * (chi_l,d,d,chi_r): all device, FP64, caller-owned; out must not alias
 * theta.  prec is a tna_prec.  Scratch comes from the context. */
tna_status tna_heff_apply(tna_ctx ctx, int chi_l, int chi_r, int d, int D, const double *L, const double *W1,
                          const double *W2, const double *R, const double *theta, double *out, int prec);

/* Allocation-free form of tna_heff_apply, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as tna_heff_apply, and the same
 * kernels; the intermediates live in one fixed device array of
 * TNA_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends, instead of
 * context or workspace memory, and the call makes no allocation of any kind.  A
 * shape whose scratch (tna_heff_apply_noalloc_bytes) exceeds the array returns
 * TNA_ERR_ARG with nothing launched.  Every call on one GPU uses the same array:
 * calls that overlap on a GPU (other streams, other contexts, other host threads)
 * race, so the caller orders them (one stream, or events).  Nothing in the array
 * needs clearing: each call overwrites what it reads. */
#define TNA_NOALLOC_SCRATCH_BYTES (64u << 20)
tna_status tna_heff_apply_noalloc(tna_ctx ctx, int chi_l, int chi_r, int d, int D, const double *L, const double *W1,
                                  const double *W2, const double *R, const double *theta, double *out, int prec);
/* Scratch bytes tna_heff_apply_noalloc needs for a shape (host only). */
tna_status tna_heff_apply_noalloc_bytes(int chi_l, int chi_r, int d, int D, int prec, size_t *bytes);

/* ---------------------------------------------------------------- SVD */
/* Truncated SVD of Eq. (3)/(19), A = U diag(S) Vt, by blocked one-sided
 * Jacobi, plus the spectrum sums of Eq. (4)-(5).
 *  A       device, m x n, dtype (TNA_F64: double, TNA_F32: float; an F32
 *          input is widened to FP64 on load, the whole Jacobi runs in FP64
 *          and U, Vt are rounded to FP32 on output, so the F32 error is the
 *          rounding of the input and of the outputs)
 *  chi_keep  k = min(chi_keep, m, n) vectors are returned (chi_keep >= 1)
 *  S       device double[min(m,n)]: full spectrum, descending
 *  U       device, m x k (same dtype as A);  Vt device, k x n
 *  spec    device double[6]: {Z = sum S^2, entropy -sum p ln p (p = S^2/Z),
 *          eps = sqrt(sum_{j>=k} S_j^2), eps^2/Z, |S_0..k-1|, gap
 *          (S_{k-1}-S_k)/S_0 (1 if k = min(m,n))}
 *  k_out, sweeps_out  host, may be NULL; filling them synchronises.
 * Gauge: the largest-magnitude entry of each column of U is positive (ties:
 * lowest row).  Returns TNA_ERR_NOCONV if the Jacobi sweeps hit the cap. */
tna_status tna_svd_truncate(tna_ctx ctx, int m, int n, int dtype, const void *A, int chi_keep, double *S, void *U,
                            void *Vt, double *spec, int *k_out, int *sweeps_out);

/* The same for `batch` independent m x n matrices at element strides
 * strideA (A), strideS (S), strideU (U), strideVt (Vt); spec is batch x 6.
 * The batch runs through the same launches (one grid dimension per member). */
tna_status tna_svd_truncate_batched(tna_ctx ctx, int batch, int m, int n, int dtype, const void *A, int64_t strideA,
                                    int chi_keep, double *S, int64_t strideS, void *U, int64_t strideU, void *Vt,
                                    int64_t strideVt, double *spec, int *sweeps_out);

/* ---------------------------------------------------------------- controller */
/* EMA (Eq. 8), optional linear predictor (Eq. 16, beta > 0) and its second-order
 * extension (Sec. 7, beta2 > 0), then PID with
 * anti-windup (Eq. 9-11, Algorithm 2), one call per bond visit.
 * First visit: the EMA starts at S (or at 0 with ema_init_zero) and the
 * previous error equals the current one.  Rounding is to nearest, ties to
 * even.  The stored controller chi (not the realised rank) enters the
 * update.  Host only, pure: the result depends only on (params, state, s_raw).
 * terms (may be NULL) receives {P, I, D, u, Sbar, e}. */
typedef struct {
  double kp, ki, kd, s_target, alpha, beta;
  int chi_min, chi_max, ema_init_zero, pad;
  double beta2; /* second-order predictor (Sec. 7): adds beta2 (S(t) - 2 S(t-1) + S(t-2)) of the EMA
                   to the predicted entropy from a bond's third visit on; 0 = off */
} tna_pid_params;

typedef struct {
  double s_ema, s_ema_prev, e_prev, integ;
  int chi, visits;
} tna_pid_state;

tna_status tna_pid_chi_update(const tna_pid_params *p, tna_pid_state *st, double s_raw, int *chi_next,
                              double *terms);

/* Entropy-margin bond dimension (Sec. 4, Eq. 6-8 and Algorithm 1): the same EMA of the bond entropy
 * as the PID (p->alpha; seeded with the first entropy unless p->ema_init_zero), then
 * chi_next = clamp(ceil(gamma * exp(S_ema)), p->chi_min, p->chi_max).  gamma >= 1 is the margin.
 * Updates st->s_ema, st->s_ema_prev, st->visits and st->chi (the PID fields stay untouched).
 * Host arithmetic.  TNA_ERR_ARG on a null pointer, gamma < 1 or bad bounds; TNA_ERR_NONFINITE on a
 * non-finite entropy. */
tna_status tna_entropy_chi_update(const tna_pid_params *p, double gamma, tna_pid_state *st, double s_raw,
                                  int *chi_next);

/* ---------------------------------------------------------------- DMRG */
typedef struct {
  double lanczos_tol;     /* residual |beta_j y_j| <= tol*max(1,|E|); default 1e-12 */
  int lanczos_kmax;       /* Krylov vectors before a restart; default 100 */
  int lanczos_restarts;   /* default 5 */
  int lanczos_fixed_iters;/* >0: exactly this many matvecs per visit (throughput mode) */
  int heff_prec;          /* tna_prec */
  int fixed_chi;          /* >0: keep min(fixed_chi, m, n) regardless of the controller */
  int svd_max_sweeps;     /* default 60.  A visit whose Jacobi stops at this cap makes the sweep return
                             TNA_ERR_NOCONV; the truncation then uses the stopped iteration's factors (the
                             accumulated rotations stay orthonormal, the other factor does not), so the MPS
                             is no longer in canonical form after it: a diagnostic setting */
  double eps_target;      /* truncation-error target that is reported (and used by schedulers) */
  int chi_rule;           /* rank rule: TNA_CHI_PID (Algorithm 2, default), TNA_CHI_THRESHOLD,
                             TNA_CHI_ENTROPY (Algorithm 1); fixed_chi > 0 overrides all three */
  int pad_;
  double rule_param;      /* TNA_CHI_THRESHOLD: eps_trunc (keep the singular values above it, at most
                             pid.chi_max and at least one); TNA_CHI_ENTROPY: the margin gamma >= 1 */
} tna_dmrg_opts;

/* chi_rule values.  The PID runs and is logged under every rule; under TNA_CHI_ENTROPY the per-bond
 * state is advanced by tna_entropy_chi_update instead. */
enum { TNA_CHI_PID = 0, TNA_CHI_THRESHOLD = 1, TNA_CHI_ENTROPY = 2 };

/* One record per bond visit (host).  k_needed: smallest rank whose
 * truncation error meets opts.eps_target on this visit's spectrum;
 * chi_sched: the learned scheduler's proposal (0 if none); fallback: 1 when
 * the proposal would have missed eps_target and the controller's chi was
 * used; feat: the scheduler's 25 inputs for this visit. */
typedef struct {
  int sweep, dir, bond, m, n, k, chi_ctrl, lanczos_iters, svd_sweeps, lanczos_ok;
  double E, S, S_ema, eps, wdisc, gap, P, I, D, u, sigma0, sigma_last;
  double ms_lanczos, ms_svd, ms_other;
  int k_needed, chi_sched, fallback, pad;
  float feat[25];
} tna_visit_log;

typedef struct tna_dmrg_s *tna_dmrg;
typedef struct tna_mlp_s *tna_mlp;

/* Device-resident two-site DMRG (Sec. 10) with one controller per bond.
 * W_host: N MPO tensors (N, D, D, d, d).  A_host: the initial MPS packed site
 * after site (site tensor shapes from chi_init: chi_init[b] = dim of bond b,
 * N-1 values; boundary dims 1).  The library right-canonicalises it on the
 * device.  The controller starts every bond at chi_min.  Allocates device
 * memory owned by the returned object.  Synchronises. */
tna_status tna_dmrg_create(tna_ctx ctx, int N, int d, int D, const double *W_host, const double *A_host,
                           const int *chi_init, const tna_pid_params *pid, const tna_dmrg_opts *opts, tna_dmrg *out);
/* One full sweep: bonds 0..N-2 left to right, then N-2..0 right to left.
 * Per visit: theta = A_b A_{b+1}; Lanczos (FP64) on H_eff; SVD of theta;
 * entropy of the full spectrum; controller -> chi; keep k = min(chi, m, n);
 * renormalise the kept values; move the orthogonality centre; grow the
 * environment.  E_out (host) receives the last Ritz value; log (host, may be
 * NULL) receives 2*(N-1) records.  Synchronises. */
tna_status tna_dmrg_sweep(tna_dmrg dm, double *E_out, tna_visit_log *log);
/* One bond visit (Sec. 10, Eq. 18-19): the same steps as one visit of a sweep, on
 * bond `bond` (sites bond, bond+1) in direction dir (0: left to right, leaving the
 * orthogonality centre on site bond+1 and growing the left environment; 1: right to
 * left, leaving it on site bond and growing the right environment).  The centre
 * must be on site bond (dir 0) or bond+1 (dir 1); it is on site 0 after create and
 * after every sweep, and tna_dmrg_sweep needs it there.  A visit back and forth on
 * one bond repeats the same-shape step with unchanged environments.  E_out and log
 * (host, may be NULL) as for one record of a sweep; log->sweep is the number of
 * sweeps done.  TNA_ERR_ARG (nothing launched) on a bad bond, direction or centre.
 * Synchronises. */
tna_status tna_dmrg_visit(tna_dmrg dm, int bond, int dir, double *E_out, tna_visit_log *log);
/* Site of the orthogonality centre (-1 for a null handle).  Host only. */
int tna_dmrg_centre(tna_dmrg dm);
/* Counters of the run's step engine since create (tna_batch_stats below; ms_total stays 0 and
 * steps is the number of sweeps done).  Host only. */
typedef struct tna_batch_stats_s tna_batch_stats;
tna_status tna_dmrg_get_stats(tna_dmrg dm, tna_batch_stats *out);
/* Copies one environment tensor into dst (device or host memory, capacity in doubles):
 * side 0 the left environment of `site` (sites 0..site-1, layout L[a][w][a'], current
 * for site <= centre), side 1 the right environment of `site` (sites site+1..N-1,
 * R[b][w][b'], current for site >= centre).  *count receives chi*D*chi; dst NULL only
 * queries it.  TNA_ERR_ARG for an environment that is not current.  Synchronises. */
tna_status tna_dmrg_get_env(tna_dmrg dm, int side, int site, double *dst, size_t capacity, size_t *count);
/* Current realised bond dims (N-1) and controller states (N-1), host. */
tna_status tna_dmrg_get_state(tna_dmrg dm, int *chi, tna_pid_state *pid);
/* Copies the MPS packed site after site into A_host (capacity given in
 * doubles); *count receives the number of doubles.  Synchronises. */
tna_status tna_dmrg_get_mps(tna_dmrg dm, double *A_host, size_t capacity, size_t *count);
/* Checkpoint / resume: writes the MPO, controller parameters and options, bond
 * dimensions, site tensors, per-bond controller states (Alg. 2 state) and the
 * scheduler history to `path` (binary, this library's own format); load recreates
 * the run on ctx from them (right-canonicalisation and environments as in
 * tna_dmrg_create) and restores the controller state, so the next sweep continues
 * the saved run.  A learned scheduler is not saved: attach it again, and the
 * proposals it had pending at the save are used as if it had never left.  Errors:
 * TNA_ERR_ARG on a file that cannot be opened, is not a checkpoint or is truncated. */
tna_status tna_dmrg_save(tna_dmrg dm, const char *path);
tna_status tna_dmrg_load(tna_ctx ctx, const char *path, tna_dmrg *out);
void tna_dmrg_destroy(tna_dmrg dm);

/* ---------------------------------------------------------------- many chains */
/* Independent chains (own N, MPO, initial MPS) swept together: all chains
 * advance one bond visit per step and every stage of the visit is one grouped
 * launch over the chains (persistent grouped GEMM over a tile work list,
 * grouped mixing and Lanczos vector kernels, one group of Jacobi SVDs of
 * different shapes); the launch sequence of a Lanczos iteration is captured
 * as a HIP graph once per step and replayed.  Controllers, Lanczos options
 * and precision as for tna_dmrg_create (pid and opts are shared by all
 * chains; opts.heff_prec F32 runs the H_eff contractions in FP32).  The work
 * runs on the context's stream; a context created on the null stream (which
 * cannot be captured into a graph) gets a private non-blocking stream of
 * default priority instead.  Either way the call waits for the context
 * stream's earlier work first and synchronises before returning.  The same
 * holds for tna_dmrg_sweep and tna_dmrg_visit.  Synchronises. */
typedef struct tna_dmrg_batch_s *tna_dmrg_batch;
struct tna_batch_stats_s {
  double ms_total, ms_lanczos, ms_svd, ms_env;
  long lanczos_iters, graph_launches;
  long small_launches;   /* launches of the single-workgroup Lanczos path (short theta) */
  long heff_f32_iters;   /* Lanczos iterations the FP32 H_eff kernels executed (counted per launch on the
                            device side, so at least lanczos_iters under heff_prec F32; 0 under F64) */
  long svd_rows, svd_rows_swept; /* rows (min(m, n)) of the visits' SVDs, and the rows their Jacobi sweeps
                            worked on: fewer where a QR start stopped because every later row was at the
                            rounding level (those rows are never rotated) */
  long heff_ident_steps; /* steps whose H_eff products left out the MPO's identity channels (the left
                            environment's last channel and the right environment's first channel equal
                            the identity to 1e-10, as they do for canonical tensors) */
  double heff_ident_dev;  /* largest deviation of those channels from the identity at the last step */
  int autotune_entries, steps;
};
tna_status tna_dmrg_batch_create(tna_ctx ctx, int nchains, const int *N, int d, int D, const double *const *W_host,
                                 const double *const *A_host, const int *const *chi_init, const tna_pid_params *pid,
                                 const tna_dmrg_opts *opts, tna_dmrg_batch *out);
/* One sweep of every chain.  E_out (host, nchains): last Ritz value per
 * chain.  logs (host, may be NULL): records of chain c start at
 * log_offsets[c] (2*(N_c-1) records each).  stats (host, may be NULL). */
tna_status tna_dmrg_batch_sweep(tna_dmrg_batch b, double *E_out, tna_visit_log *logs, const int64_t *log_offsets,
                                tna_batch_stats *stats);
tna_status tna_dmrg_batch_get_state(tna_dmrg_batch b, int chain, int *chi, tna_pid_state *pid);
void tna_dmrg_batch_destroy(tna_dmrg_batch b);
/* GEMM tile autotuner of the grouped launches: the table maps (operation,
 * log2 flops) to the faster of the 64x64 and 128x128 tiles, measured the
 * first time a bucket is met; it can be saved and reloaded (text). */
tna_status tna_autotune_save(const char *path);
tna_status tna_autotune_load(const char *path);
int tna_autotune_entries(void);
/* Empties the table (the next launches measure again). */
void tna_autotune_clear(void);

/* ---------------------------------------------------------------- circuits */
/* Circuit simulation with adaptive bond dimensions (Sec. 8, circuit-level bond
 * dimension maps; the TEBD scheme of Sec. 2).  An MPS of N qubits (d = 2) starts
 * in |0...0>.  tna_circuit_layer applies one layer of real two-qubit gates to the
 * disjoint pairs (b, b+1) with b = parity, parity + 2, ..., b <= N - 2 (gates_host:
 * one row-major 4 x 4 matrix G[2s+t][2s'+t'] per pair in increasing b, s on qubit
 * b; qubit 0 is the most significant bit of a basis state).  At every gate bond:
 * the two-site tensor B_b B_{b+1}, the gate, the Schmidt-value scaling of the left
 * bond, the Jacobi SVD (Eq. 3) of the full two-site matrix, its entropy (Eq. 5),
 * the bond's EMA + PID (Eq. 8-11, Algorithm 2; the DMRG controller) or the fixed
 * chi, truncation to k = min(chi, rank) with the kept values renormalised, then
 * B_{b+1} <- Y_k^T and B_b <- (G B_b B_{b+1}) Y_k / |S_k|, so the MPS stays
 * right-canonical with the Schmidt values of every bond and no division by one.
 * All gates of a layer go through the same grouped launches (one group of SVDs);
 * controllers of bonds the layer does not touch are left alone.  chi_row (host,
 * N-1, may be NULL) receives the bond dimensions after the layer: one row of the
 * bond-dimension map.  log (host, one record per gate, may be NULL).  Runs on the
 * context stream (a private one when that is the null stream).  Synchronises. */
typedef struct tna_circuit_s *tna_circuit;
typedef struct {
  int fixed_chi;       /* > 0: keep min(fixed_chi, rank) regardless of the controller */
  int one_at_a_time;   /* 1: the gates of a layer run one after another (the unbatched form) */
  int svd_max_sweeps;  /* default 60 */
  int pad;
} tna_circuit_opts;
typedef struct {
  int layer, bond, m, n, k, chi_ctrl, svd_sweeps, pad;
  double S, S_ema, eps, wdisc, gap, sigma0, sigma_last, u;
} tna_gate_log;
tna_status tna_circuit_create(tna_ctx ctx, int N, const tna_pid_params *pid, const tna_circuit_opts *opts,
                              tna_circuit *out);
tna_status tna_circuit_layer(tna_circuit c, int parity, const double *gates_host, tna_gate_log *log, int *chi_row);
/* Site tensors packed site after site (B_i: chi_{i-1} x 2 x chi_i) and the bond dimensions (N-1, may be
 * NULL); B_host NULL only queries *count (doubles).  Synchronises. */
tna_status tna_circuit_get_mps(tna_circuit c, double *B_host, size_t capacity, size_t *count, int *chi);
void tna_circuit_destroy(tna_circuit c);

/* ---------------------------------------------------------------- learned scheduler */
/* A 25 -> 64 -> 64 -> 1 perceptron (tanh hidden units, linear output), the
 * learned stand-in for the predictive scheduler of Sec. 7, trained and run
 * in FP32 by the library's own kernels.  Inputs per bond visit: the last 8
 * EMA entropies (oldest first, missing history repeats the oldest), the 16
 * largest log singular values (floored at ln 1e-16) and the relative bond
 * position; output: log2 of the bond dimension the bond needs at its next
 * visit.  Parameter layout (5889 floats): W1[64][25] b1[64] W2[64][64] b2[64]
 * W3[64] b3.  Inputs are standardised by (x - mean)/std when a normalisation
 * is set. */
#define TNA_MLP_IN 25
#define TNA_MLP_NPARAM 5889
/* params_host: initial parameters (host, 5889 floats; the caller draws them). */
tna_status tna_mlp_create(tna_ctx ctx, const float *params_host, tna_mlp *out);
tna_status tna_mlp_set_normalization(tna_mlp n, const float *mean_host, const float *std_host);
tna_status tna_mlp_get_params(tna_mlp n, float *params_host);
/* y[b] (device, B floats) for X (device, B x 25 floats). */
tna_status tna_mlp_forward(tna_mlp n, int B, const float *X, float *y);
/* grad (device, 5889 floats) and loss (device, 1 float, may be NULL) of
 * (1/B) sum_b (y_b - T_b)^2. */
tna_status tna_mlp_loss_grad(tna_mlp n, int B, const float *X, const float *T, float *grad, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr. */
tna_status tna_mlp_adam_step(tna_mlp n, const float *grad, float lr);
/* epochs of mini-batch Adam over (X, T) (device, nsamp samples); perm (device,
 * epochs x nsamp ints) gives the sample order of every epoch; loss_per_epoch
 * (host, may be NULL) receives the full-data loss after each epoch.
 * Synchronises. */
tna_status tna_mlp_train(tna_mlp n, int nsamp, const float *X, const float *T, const int *perm, int epochs,
                         int batch, float lr, float *loss_per_epoch);
void tna_mlp_destroy(tna_mlp n);
/* Attaches a trained network to a DMRG run (NULL detaches).  From each bond's
 * second visit on, the bond keeps k = clamp(round(2^y), chi_min, chi_max)
 * predicted at its previous visit, unless that k would leave a truncation
 * error above opts.eps_target, in which case the controller's chi is used
 * (fallback).  The controller keeps running either way.  Replacing or detaching a
 * network drops its pending proposals. */
tna_status tna_dmrg_set_scheduler(tna_dmrg dm, tna_mlp net);

#ifdef __cplusplus
}
#endif
#endif /* TNA_H */
