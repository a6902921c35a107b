/*
 * circuit.c -- plain FP64 oracle for circuit simulation with adaptive bond
 * dimensions (Sec. 8 of arXiv 2604.03960, "circuit-level bond dimension maps";
 * the TEBD scheme of Sec. 2).  TEST INFRASTRUCTURE: only the tests, the smoke
 * check and the benchmark's CPU baseline use it; the GPU library neither links
 * nor calls it.  No BLAS, no LAPACK, no code shared with the GPU path.
 *
 * Conventions.  Qubits 0..N-1 on an open chain, d = 2.  A gate layer ("op")
 * acts on the disjoint pairs (b, b+1) of one parity p: b = p, p + 2, ...,
 * b <= N - 2.  A two-qubit gate is a real 4 x 4 matrix G[st][s't'] (row-major,
 * index 2 s + t, s on qubit b, t on qubit b + 1).  The gates of op l are packed
 * one after the other, 16 doubles each, in increasing b.  A state vector is
 * indexed by sum_i s_i 2^(N-1-i) (qubit 0 the most significant bit), which is
 * also the row-major order of the MPS amplitudes psi(s_0, ..., s_{N-1}).
 *
 * MPS form.  Right-canonical site tensors B_i[a][s][b] (chi_{i-1}, 2, chi_i)
 * plus the Schmidt values lam_i of every bond (Vidal's form in the variant of
 * Hastings, which never divides by Schmidt values); the state is B_0 ... B_{N-1}.
 * One gate on bond (i, i+1), in the method's order:
 *   C      = B_i B_{i+1}                         (chi_{i-1}, 2, 2, chi_{i+1})
 *   C'     = G applied to the physical pair of C
 *   Theta  = lam_{i-1}[a] C'[a][s][t][b]          (lam_{-1} = 1)
 *   Theta  = X diag(S) Y^T, full spectrum S (Eq. 3, Jacobi SVD)
 *   entropy of the full spectrum (Eq. 5) -> the bond's EMA + PID (Alg. 2)
 *   keep k = min(chi_next, rank) (or the fixed chi); |S_k| = norm of the kept values
 *   B_{i+1} <- Y_k^T,   B_i <- C' Y_k / |S_k|,   lam_i <- S_k / |S_k|
 * Controllers are updated at the bonds a layer touches only; the map records
 * every bond's dimension after each layer.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* from oracle.c */
int or_svd_jacobi(int m, int n, const double *A, double *S, double *U, double *V, int *info);
void or_spectrum(int R, const double *S, int k, double *out);
typedef struct {
  double kp, ki, kd, s_target, alpha, beta;
  int chi_min, chi_max, ema_init_zero, pad;
  double beta2;
} or_pid_params;
typedef struct {
  double s_ema, s_ema_prev, e_prev, integ;
  int chi, visits;
} or_pid_state;
int or_pid_update(const or_pid_params *p, or_pid_state *st, double s_raw, int *chi_next, double *terms);

static double *cdalloc(size_t n) {
  double *p = (double *)calloc(n ? n : 1, sizeof(double));
  if (!p) abort();
  return p;
}

/* number of gates of an op of parity p on N qubits */
int or_circuit_gates(int N, int parity) { return parity > N - 2 ? 0 : (N - 2 - parity) / 2 + 1; }

/* ------------------------------------------------------------------------ */
/* Exact state-vector simulation of the same ops (the reference amplitudes). */
/* psi: in = initial state (2^N), out = final state.                          */
/* ------------------------------------------------------------------------ */
void or_circuit_statevector(int N, int nops, const int *parity, const double *gates, double *psi) {
  const size_t dim = (size_t)1 << N;
  const double *g = gates;
  for (int l = 0; l < nops; ++l) {
    for (int b = parity[l]; b <= N - 2; b += 2, g += 16) {
      const size_t sb = (size_t)1 << (N - 1 - b), tb = (size_t)1 << (N - 2 - b);
      for (size_t x = 0; x < dim; ++x) {
        if ((x & sb) || (x & tb)) continue; /* x: both qubits 0; visit each group of four once */
        const size_t idx[4] = {x, x | tb, x | sb, x | sb | tb}; /* st = 00, 01, 10, 11 */
        double in[4], out[4];
        for (int q = 0; q < 4; ++q) in[q] = psi[idx[q]];
        for (int r = 0; r < 4; ++r) {
          double acc = 0.0;
          for (int q = 0; q < 4; ++q) acc += g[r * 4 + q] * in[q];
          out[r] = acc;
        }
        for (int q = 0; q < 4; ++q) psi[idx[q]] = out[q];
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Adaptive-chi circuit simulation on the MPS (the method).                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int fixed_chi;     /* > 0: keep min(fixed_chi, rank) instead of the controller's chi */
  int pad;
} or_circuit_opts;

#define OR_CIRC_LOG 16
/* per-gate record: 0 op, 1 bond, 2 m, 3 n, 4 k, 5 chi_ctrl, 6 S, 7 S_ema, 8 eps (Eq. 4, absolute),
 * 9 discarded weight eps^2 / Z, 10 gap (S_{k-1} - S_k) / S_0 (1 if nothing discarded), 11 sigma_0,
 * 12 last kept sigma, 13 u (PID output), 14 svd sweeps, 15 Z */

/* Runs nops layers from |0...0>.  log: one record per gate (may be NULL); chimap: nops x (N-1) bond
 * dimensions after each op (may be NULL); B_out: final site tensors packed (capacity cap doubles,
 * may be NULL), chi_out (N-1), lam_out: Schmidt values packed bond after bond (capacity lcap).
 * Returns 0, or -1 when an output capacity is too small. */
int or_circuit_run(int N, int nops, const int *parity, const double *gates, const or_pid_params *pp,
                   const or_circuit_opts *op, double *log, int *chimap, double *B_out, size_t cap, int *chi_out,
                   double *lam_out, size_t lcap) {
  const int d = 2;
  int *chi = (int *)calloc((size_t)N, sizeof(int));
  double **B = (double **)calloc((size_t)N, sizeof(double *));
  double **lam = (double **)calloc((size_t)N, sizeof(double *));
  or_pid_state *ps = (or_pid_state *)calloc((size_t)N, sizeof(or_pid_state));
  for (int b = 0; b < N - 1; ++b) {
    chi[b] = 1;
    lam[b] = cdalloc(1);
    lam[b][0] = 1.0;
    ps[b].chi = pp->chi_min;
  }
  for (int i = 0; i < N; ++i) { /* |0>: B_i[0][0][0] = 1 */
    B[i] = cdalloc(2);
    B[i][0] = 1.0;
  }
  const double *g = gates;
  int rec = 0, rc = 0;
  for (int l = 0; l < nops; ++l) {
    for (int b = parity[l]; b <= N - 2; b += 2, g += 16) {
      const int cl = b == 0 ? 1 : chi[b - 1], cm = chi[b], cr = b + 1 == N - 1 ? 1 : chi[b + 1];
      const int m = cl * d, n = d * cr, R = m < n ? m : n;
      /* C = B_b B_{b+1}: (cl d) x cm times cm x (d cr) */
      double *Cm = cdalloc((size_t)m * n);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
          double acc = 0.0;
          for (int q = 0; q < cm; ++q) acc += B[b][(size_t)i * cm + q] * B[b + 1][(size_t)q * n + j];
          Cm[(size_t)i * n + j] = acc;
        }
      /* C' = G on the physical pair: C'[a][s][t][c] = sum G[st][s't'] C[a][s'][t'][c] */
      double *Cp = cdalloc((size_t)m * n);
      for (int a = 0; a < cl; ++a)
        for (int c = 0; c < cr; ++c)
          for (int st = 0; st < 4; ++st) {
            double acc = 0.0;
            for (int q = 0; q < 4; ++q)
              acc += g[st * 4 + q] * Cm[((size_t)a * d + q / 2) * n + (size_t)(q % 2) * cr + c];
            Cp[((size_t)a * d + st / 2) * n + (size_t)(st % 2) * cr + c] = acc;
          }
      /* Theta = lam_{b-1}[a] C' */
      double *Th = cdalloc((size_t)m * n);
      for (int a = 0; a < cl; ++a) {
        const double la = b == 0 ? 1.0 : lam[b - 1][a];
        for (size_t e = 0; e < (size_t)d * n; ++e) Th[(size_t)a * d * n + e] = la * Cp[(size_t)a * d * n + e];
      }
      double *S = cdalloc(R), *U = cdalloc((size_t)m * R), *V = cdalloc((size_t)n * R);
      int info = 0;
      or_svd_jacobi(m, n, Th, S, U, V, &info);
      double sp[4];
      or_spectrum(R, S, R, sp); /* Z, entropy of the full spectrum */
      double terms[6] = {0};
      int chi_next = 0;
      or_pid_update(pp, &ps[b], sp[1], &chi_next, terms);
      const int keep = op && op->fixed_chi > 0 ? op->fixed_chi : chi_next;
      const int k = keep < R ? keep : R;
      or_spectrum(R, S, k, sp);
      double nk = 0.0;
      for (int j = k - 1; j >= 0; --j) nk += S[j] * S[j];
      nk = sqrt(nk);
      /* B_{b+1} <- Y_k^T (k x n), B_b <- C' Y_k / |S_k| (m x k), lam_b <- S_k / |S_k| */
      double *Bn1 = cdalloc((size_t)k * n), *Bn0 = cdalloc((size_t)m * k), *ln = cdalloc(k);
      for (int j = 0; j < k; ++j)
        for (int c = 0; c < n; ++c) Bn1[(size_t)j * n + c] = V[(size_t)c * R + j];
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < k; ++j) {
          double acc = 0.0;
          for (int c = 0; c < n; ++c) acc += Cp[(size_t)i * n + c] * V[(size_t)c * R + j];
          Bn0[(size_t)i * k + j] = acc / nk;
        }
      for (int j = 0; j < k; ++j) ln[j] = S[j] / nk;
      if (log) {
        double *r = log + (size_t)rec * OR_CIRC_LOG;
        r[0] = l; r[1] = b; r[2] = m; r[3] = n; r[4] = k; r[5] = chi_next; r[6] = sp[1]; r[7] = terms[4];
        r[8] = sp[2]; r[9] = sp[3]; r[10] = k < R ? (S[k - 1] - S[k]) / S[0] : 1.0; r[11] = S[0];
        r[12] = S[k - 1]; r[13] = terms[3]; r[14] = info; r[15] = sp[0];
      }
      ++rec;
      free(B[b]); free(B[b + 1]); free(lam[b]);
      B[b] = Bn0; B[b + 1] = Bn1; lam[b] = ln;
      chi[b] = k;
      free(Cm); free(Cp); free(Th); free(S); free(U); free(V);
    }
    if (chimap)
      for (int b = 0; b < N - 1; ++b) chimap[(size_t)l * (N - 1) + b] = chi[b];
  }
  if (B_out) {
    size_t off = 0;
    for (int i = 0; i < N; ++i) {
      const size_t cl = i == 0 ? 1 : chi[i - 1], cr = i == N - 1 ? 1 : chi[i];
      if (off + cl * d * cr > cap) { rc = -1; break; }
      memcpy(B_out + off, B[i], sizeof(double) * cl * d * cr);
      off += cl * d * cr;
    }
  }
  if (lam_out) {
    size_t off = 0;
    for (int b = 0; b < N - 1 && rc == 0; ++b) {
      if (off + (size_t)chi[b] > lcap) { rc = -1; break; }
      memcpy(lam_out + off, lam[b], sizeof(double) * chi[b]);
      off += chi[b];
    }
  }
  if (chi_out) memcpy(chi_out, chi, sizeof(int) * (N - 1));
  for (int i = 0; i < N; ++i) { free(B[i]); free(lam[i]); }
  free(B); free(lam); free(chi); free(ps);
  return rc;
}

/* Amplitudes psi(s_0..s_{N-1}) of packed site tensors (N <= 24): contraction left to right. */
void or_mps_amplitudes(int N, const double *A_packed, const int *chi, double *psi) {
  const int d = 2;
  size_t rows = 1;
  int cprev = 1;
  double *cur = cdalloc(1);
  cur[0] = 1.0;
  size_t off = 0;
  for (int i = 0; i < N; ++i) {
    const int cr = i == N - 1 ? 1 : chi[i];
    const double *A = A_packed + off;
    double *nxt = cdalloc(rows * d * (size_t)cr);
    for (size_t r = 0; r < rows; ++r)
      for (int s = 0; s < d; ++s)
        for (int c = 0; c < cr; ++c) {
          double acc = 0.0;
          for (int a = 0; a < cprev; ++a) acc += cur[r * cprev + a] * A[((size_t)a * d + s) * cr + c];
          nxt[(r * d + s) * cr + c] = acc;
        }
    free(cur);
    cur = nxt;
    off += (size_t)cprev * d * cr;
    rows *= d;
    cprev = cr;
  }
  memcpy(psi, cur, sizeof(double) * rows);
  free(cur);
}
