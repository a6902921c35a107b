/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the two-site DMRG step with an
 * entropy-EMA-PID bond-dimension controller (arXiv 2604.03960).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library.  It shares no
 * code, header, table or helper with the GPU library; it uses no BLAS, LAPACK
 * or threading inside the math.  Every loop is written out so that it can be
 * checked against the paper by eye.
 *
 * Conventions (row-major everywhere):
 *   site tensor  A_i[a][s][b]        a < chi_{i-1}, s < d, b < chi_i
 *   MPO tensor   W_i[wl][wr][s][s']  s = output (bra) index, s' = input (ket)
 *   left env     L[a][w][a']         bra, MPO, ket
 *   right env    R[b][w][b']         bra, MPO, ket
 *   two-site     theta[a][s][t][b]
 * The left boundary selects MPO row D-1, the right boundary MPO column 0.
 * Local basis: s = 0 is spin up (S^z = +1/2), s = 1 spin down.
 *
 * Pinned functions and their pins live in tests/test_oracle_*.py.  Functions
 * whose results have no pin independent of this file are marked
 * "parity unpinned" below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_NOMEM 2
#define OR_ERR_NOCONV 4

static const double EPS53 = 1.1102230246251565e-16; /* 2^-53 */

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */
static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

static double dot(size_t n, const double *x, const double *y) {
  double s = 0.0;
  for (size_t i = 0; i < n; ++i) s += x[i] * y[i];
  return s;
}

/* plain triple-loop product C[m][n] = A[m][k] * B[k][n] (row-major) */
static void matmul(int m, int n, int k, const double *A, const double *B, double *C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += A[(size_t)i * k + l] * B[(size_t)l * n + j];
      C[(size_t)i * n + j] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Spin operators and MPOs (the Hamiltonians of Eq. (20) and Table 5)        */
/* ------------------------------------------------------------------------ */
/* op index: 0 I, 1 S+, 2 S-, 3 Sz, 4 sigma_x, 5 sigma_z */
static double op_elem(int op, int so, int si) {
  switch (op) {
    case 0: return so == si ? 1.0 : 0.0;
    case 1: return (so == 0 && si == 1) ? 1.0 : 0.0;  /* |up><down| */
    case 2: return (so == 1 && si == 0) ? 1.0 : 0.0;  /* |down><up| */
    case 3: return so == si ? (so == 0 ? 0.5 : -0.5) : 0.0;
    case 4: return so != si ? 1.0 : 0.0;
    case 5: return so == si ? (so == 0 ? 1.0 : -1.0) : 0.0;
  }
  return 0.0;
}

static void put(double *W, int D, int wl, int wr, int op, double coef) {
  for (int so = 0; so < 2; ++so)
    for (int si = 0; si < 2; ++si)
      W[(((size_t)wl * D + wr) * 2 + so) * 2 + si] += coef * op_elem(op, so, si);
}

/* model 0: XXZ  H = J sum [ (S+S- + S-S+)/2 + Delta Sz Sz ] - hz sum Sz   (D=5)
 *   params = {J, Delta, hz}
 * model 1: J1-J2 Heisenberg  H = J1 sum S_i.S_{i+1} + J2 sum S_i.S_{i+2}   (D=8)
 *   params = {J1, J2}
 * model 2: transverse-field Ising (Pauli) H = -J sum sz sz - h sum sx       (D=3)
 *   params = {J, h}
 * Output W: N identical bulk tensors [D][D][2][2]; returns D (or <0 on error). */
int or_mpo_build(int model, int N, const double *p, double *W) {
  int D = model == 0 ? 5 : model == 1 ? 8 : model == 2 ? 3 : -1;
  if (D < 0 || N < 2) return -1;
  size_t sz = (size_t)D * D * 4;
  double *w = dalloc(sz);
  if (model == 0) {
    double J = p[0], Dz = p[1], hz = p[2];
    put(w, D, 0, 0, 0, 1.0);
    put(w, D, 4, 4, 0, 1.0);
    put(w, D, 4, 1, 1, 0.5 * J); put(w, D, 1, 0, 2, 1.0);
    put(w, D, 4, 2, 2, 0.5 * J); put(w, D, 2, 0, 1, 1.0);
    put(w, D, 4, 3, 3, J * Dz);  put(w, D, 3, 0, 3, 1.0);
    if (hz != 0.0) put(w, D, 4, 0, 3, -hz);
  } else if (model == 1) {
    double J1 = p[0], J2 = p[1];
    put(w, D, 0, 0, 0, 1.0);
    put(w, D, 7, 7, 0, 1.0);
    put(w, D, 7, 1, 1, 0.5 * J1); put(w, D, 1, 0, 2, 1.0);
    put(w, D, 7, 2, 2, 0.5 * J1); put(w, D, 2, 0, 1, 1.0);
    put(w, D, 7, 3, 3, J1);       put(w, D, 3, 0, 3, 1.0);
    /* next-nearest: place the operator, carry an identity, close with the partner */
    put(w, D, 7, 4, 1, 0.5 * J2); put(w, D, 4, 1, 0, 1.0);
    put(w, D, 7, 5, 2, 0.5 * J2); put(w, D, 5, 2, 0, 1.0);
    put(w, D, 7, 6, 3, J2);       put(w, D, 6, 3, 0, 1.0);
  } else {
    double J = p[0], h = p[1];
    put(w, D, 0, 0, 0, 1.0);
    put(w, D, 2, 2, 0, 1.0);
    put(w, D, 2, 1, 5, -J); put(w, D, 1, 0, 5, 1.0);
    put(w, D, 2, 0, 4, -h);
  }
  for (int i = 0; i < N; ++i) memcpy(W + (size_t)i * sz, w, sz * sizeof(double));
  free(w);
  return D;
}

/* Dense 2^N x 2^N matrix of the MPO (N <= 10): contract l^T W_0 ... W_{N-1} r.
 * Basis index x = sum_i s_i 2^(N-1-i). */
int or_mpo_dense(int N, int D, const double *W, double *H) {
  if (N < 1 || N > 10) return OR_ERR_ARG;
  size_t dim = (size_t)1 << N;
  size_t sz = (size_t)D * D * 4;
  /* T[w][x_out][x_in] over the sites processed so far */
  size_t cur = 1;
  double *T = dalloc((size_t)D);
  T[D - 1] = 1.0; /* left boundary, dims: T[w][1][1] */
  for (int i = 0; i < N; ++i) {
    size_t nxt = cur * 2;
    double *Tn = dalloc((size_t)D * nxt * nxt);
    const double *Wi = W + (size_t)i * sz;
    for (int wl = 0; wl < D; ++wl)
      for (int wr = 0; wr < D; ++wr)
        for (int so = 0; so < 2; ++so)
          for (int si = 0; si < 2; ++si) {
            double c = Wi[(((size_t)wl * D + wr) * 2 + so) * 2 + si];
            if (c == 0.0) continue;
            for (size_t xo = 0; xo < cur; ++xo)
              for (size_t xi = 0; xi < cur; ++xi)
                Tn[((size_t)wr * nxt + xo * 2 + so) * nxt + xi * 2 + si] +=
                    c * T[((size_t)wl * cur + xo) * cur + xi];
          }
    free(T);
    T = Tn;
    cur = nxt;
  }
  for (size_t xo = 0; xo < dim; ++xo)
    for (size_t xi = 0; xi < dim; ++xi) H[xo * dim + xi] = T[(0 * dim + xo) * dim + xi];
  free(T);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact diagonalisation: matrix-free H.v on the 2^N spin basis              */
/* ------------------------------------------------------------------------ */
static int bit(uint64_t x, int N, int i) { return (int)((x >> (N - 1 - i)) & 1u); }

static void heis_bond(int N, int i, int j, double Jxy, double Jz, const double *x, double *y, size_t dim) {
  uint64_t mi = 1ull << (N - 1 - i), mj = 1ull << (N - 1 - j);
  for (size_t s = 0; s < dim; ++s) {
    int bi = bit(s, N, i), bj = bit(s, N, j);
    double zz = (bi == bj) ? 0.25 : -0.25;
    y[s] += Jz * zz * x[s];
    if (bi != bj) y[s ^ mi ^ mj] += 0.5 * Jxy * x[s];
  }
}

/* y = H x for the models of or_mpo_build (open chain) */
int or_ed_apply(int model, int N, const double *p, const double *x, double *y) {
  if (N < 2 || N > 24) return OR_ERR_ARG;
  size_t dim = (size_t)1 << N;
  memset(y, 0, dim * sizeof(double));
  if (model == 0) {
    for (int i = 0; i + 1 < N; ++i) heis_bond(N, i, i + 1, p[0], p[0] * p[1], x, y, dim);
    if (p[2] != 0.0)
      for (size_t s = 0; s < dim; ++s)
        for (int i = 0; i < N; ++i) y[s] += -p[2] * (bit(s, N, i) ? -0.5 : 0.5) * x[s];
  } else if (model == 1) {
    for (int i = 0; i + 1 < N; ++i) heis_bond(N, i, i + 1, p[0], p[0], x, y, dim);
    for (int i = 0; i + 2 < N; ++i) heis_bond(N, i, i + 2, p[1], p[1], x, y, dim);
  } else if (model == 2) {
    for (size_t s = 0; s < dim; ++s) {
      double zz = 0.0;
      for (int i = 0; i + 1 < N; ++i) zz += (bit(s, N, i) == bit(s, N, i + 1)) ? 1.0 : -1.0;
      y[s] += -p[0] * zz * x[s];
      for (int i = 0; i < N; ++i) y[s ^ (1ull << (N - 1 - i))] += -p[1] * x[s];
    }
  } else {
    return OR_ERR_ARG;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Dense symmetric eigensolver: cyclic two-sided Jacobi (Golub & Van Loan,   */
/* Matrix Computations, sec. 8.5).  A is overwritten; V receives the         */
/* eigenvectors as columns; evals in w (unsorted, diagonal order).           */
/* ------------------------------------------------------------------------ */
int or_sym_eig_jacobi(int n, double *A, double *w, double *V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
  double fro = 0.0;
  for (size_t i = 0; i < (size_t)n * n; ++i) fro += A[i] * A[i];
  fro = sqrt(fro);
  double thr = fro * 1e-18;
  int sweep;
  for (sweep = 0; sweep < 100; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(size_t)p * n + q];
        if (fabs(apq) <= thr) continue;
        double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) { /* columns p, q */
          double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) { /* rows p, q */
          double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        A[(size_t)p * n + q] = 0.0;
        A[(size_t)q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {
          double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
        rotated = 1;
      }
    if (!rotated) break;
  }
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
  return sweep < 100 ? OR_OK : OR_ERR_NOCONV;
}

/* ------------------------------------------------------------------------ */
/* One-sided Jacobi SVD (Hestenes 1958; Golub & Van Loan sec. 8.6.3),        */
/* the truncated-SVD step of Eq. (3) and Eq. (19).                           */
/*   A: m x n row-major.  R = min(m,n).                                      */
/*   S[R] descending; U[m][R] and V[n][R] with singular vectors as columns.  */
/*   Columns are orthogonalised cyclically by rows of the pair order (i<j);  */
/*   a pair is rotated when |gamma| > tol*sqrt(alpha*beta), tol = rows*2^-53.*/
/*   Sign gauge: the largest-magnitude entry of each u_j is positive (ties:  */
/*   lowest row); v_j follows.  Null columns (sigma_j <= 2^-53 sigma_0       */
/*   max(m,n)) of U are completed by Gram-Schmidt on e_0, e_1, ...           */
/*   info[0] = sweeps used.  Returns OR_ERR_NOCONV after 60 sweeps.           */
/* ------------------------------------------------------------------------ */
int or_svd_jacobi(int m, int n, const double *A, double *S, double *U, double *V, int *info) {
  if (m < 1 || n < 1) return OR_ERR_ARG;
  int tr = m < n;               /* work on A^T so that rows >= cols */
  int rows = tr ? n : m, cols = tr ? m : n;
  int R = cols;
  double *B = dalloc((size_t)rows * cols);  /* working matrix, column j = B[.][j] */
  double *Q = dalloc((size_t)cols * cols);  /* accumulated rotations */
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) B[(size_t)i * cols + j] = tr ? A[(size_t)j * n + i] : A[(size_t)i * n + j];
  for (int i = 0; i < cols; ++i) Q[(size_t)i * cols + i] = 1.0;
  double tol = rows * EPS53;
  int sweep, conv = 0;
  for (sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int i = 0; i < cols - 1; ++i)
      for (int j = i + 1; j < cols; ++j) {
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int r = 0; r < rows; ++r) {
          double bi = B[(size_t)r * cols + i], bj = B[(size_t)r * cols + j];
          al += bi * bi;
          be += bj * bj;
          ga += bi * bj;
        }
        if (al == 0.0 || be == 0.0) continue;
        if (!(fabs(ga) > tol * sqrt(al * be))) continue;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int r = 0; r < rows; ++r) {
          double bi = B[(size_t)r * cols + i], bj = B[(size_t)r * cols + j];
          B[(size_t)r * cols + i] = c * bi - s * bj;
          B[(size_t)r * cols + j] = s * bi + c * bj;
        }
        for (int r = 0; r < cols; ++r) {
          double qi = Q[(size_t)r * cols + i], qj = Q[(size_t)r * cols + j];
          Q[(size_t)r * cols + i] = c * qi - s * qj;
          Q[(size_t)r * cols + j] = s * qi + c * qj;
        }
        rotated = 1;
      }
    if (!rotated) { conv = 1; break; }
  }
  if (info) info[0] = sweep + (conv ? 1 : 0);
  /* singular values = column norms, stable sort descending */
  double *sig = dalloc(cols);
  int *ord = (int *)malloc(sizeof(int) * (size_t)cols);
  for (int j = 0; j < cols; ++j) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += B[(size_t)r * cols + j] * B[(size_t)r * cols + j];
    sig[j] = sqrt(s);
    ord[j] = j;
  }
  for (int a = 1; a < cols; ++a) { /* insertion sort: stable */
    int x = ord[a], b = a - 1;
    while (b >= 0 && sig[ord[b]] < sig[x]) { ord[b + 1] = ord[b]; --b; }
    ord[b + 1] = x;
  }
  /* left vectors of the working problem (rows x R) and right vectors (cols x R) */
  double *Lw = dalloc((size_t)rows * R), *Rw = dalloc((size_t)cols * R);
  double smax = sig[ord[0]];
  double null_thr = EPS53 * smax * (m > n ? m : n);
  for (int k = 0; k < R; ++k) {
    int j = ord[k];
    S[k] = sig[j];
    for (int r = 0; r < cols; ++r) Rw[(size_t)r * R + k] = Q[(size_t)r * cols + j];
    if (sig[j] > null_thr && sig[j] > 0.0)
      for (int r = 0; r < rows; ++r) Lw[(size_t)r * R + k] = B[(size_t)r * cols + j] / sig[j];
  }
  /* Gram-Schmidt completion of null columns with unit vectors e_0, e_1, ... */
  int e = 0;
  for (int k = 0; k < R; ++k) {
    if (S[k] > null_thr && S[k] > 0.0) continue;
    for (; e < rows; ++e) {
      double *col = dalloc(rows);
      col[e] = 1.0;
      for (int pass = 0; pass < 2; ++pass)
        for (int q = 0; q < R; ++q) {
          if (q == k) continue;
          int filled = (S[q] > null_thr && S[q] > 0.0) || q < k;
          if (!filled) continue;
          double h = 0.0;
          for (int r = 0; r < rows; ++r) h += Lw[(size_t)r * R + q] * col[r];
          for (int r = 0; r < rows; ++r) col[r] -= h * Lw[(size_t)r * R + q];
        }
      double nr = sqrt(dot(rows, col, col));
      if (nr > 0.5) {
        for (int r = 0; r < rows; ++r) Lw[(size_t)r * R + k] = col[r] / nr;
        free(col);
        ++e;
        break;
      }
      free(col);
    }
  }
  /* map back: A = Lw diag(S) Rw^T (not transposed) or A^T = Lw S Rw^T */
  double *Uo = tr ? Rw : Lw;
  double *Vo = tr ? Lw : Rw;
  for (int i = 0; i < m; ++i)
    for (int k = 0; k < R; ++k) U[(size_t)i * R + k] = Uo[(size_t)i * R + k];
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < R; ++k) V[(size_t)i * R + k] = Vo[(size_t)i * R + k];
  /* sign gauge on the final U */
  for (int k = 0; k < R; ++k) {
    int imax = 0;
    double amax = -1.0;
    for (int i = 0; i < m; ++i) {
      double a = fabs(U[(size_t)i * R + k]);
      if (a > amax) { amax = a; imax = i; }
    }
    if (U[(size_t)imax * R + k] < 0.0) {
      for (int i = 0; i < m; ++i) U[(size_t)i * R + k] = -U[(size_t)i * R + k];
      for (int i = 0; i < n; ++i) V[(size_t)i * R + k] = -V[(size_t)i * R + k];
    }
  }
  free(B); free(Q); free(sig); free(ord); free(Lw); free(Rw);
  return conv ? OR_OK : OR_ERR_NOCONV;
}

/* ------------------------------------------------------------------------ */
/* Spectrum sums: Eq. (4) truncation error and Eq. (5) entropy.              */
/* Sums run smallest-first.  out = {Z, S, eps, w}:                            */
/*   Z = sum sigma^2, p = sigma^2/Z, S = -sum_{p>0} p ln p,                   */
/*   eps = sqrt(sum_{j>=k} sigma_j^2), w = eps^2 / Z.                         */
/* ------------------------------------------------------------------------ */
void or_spectrum(int R, const double *S, int k, double *out) {
  double Z = 0.0;
  for (int j = R - 1; j >= 0; --j) Z += S[j] * S[j];
  double ent = 0.0;
  for (int j = R - 1; j >= 0; --j) {
    double p = S[j] * S[j] / Z;
    if (p > 0.0) ent -= p * log(p);
  }
  double tail = 0.0;
  for (int j = R - 1; j >= k; --j) tail += S[j] * S[j];
  out[0] = Z;
  out[1] = ent;
  out[2] = sqrt(tail);
  out[3] = tail / Z;
}

/* ------------------------------------------------------------------------ */
/* EMA (Eq. 8) + optional linear predictor (Eq. 16) + PID with anti-windup   */
/* (Eq. 9-11, Algorithm 2), one call per bond visit.                          */
/* Readings: first visit seeds the EMA with S (or 0 with ema_init_zero);     */
/* e = Sbar - S_target; the first visit uses e_prev = e; rounding is to      */
/* nearest, ties to even; the stored controller chi enters the update.        */
/* ------------------------------------------------------------------------ */
typedef struct {
  double kp, ki, kd, s_target, alpha, beta;
  int chi_min, chi_max, ema_init_zero, pad;
  double beta2; /* weight of the curvature term of the second-order predictor (Sec. 7) */
} or_pid_params;

typedef struct {
  double s_ema, s_ema_prev, e_prev, integ;
  int chi, visits;
} or_pid_state;

int or_pid_update(const or_pid_params *pp, or_pid_state *st, double s_raw, int *chi_next, double *terms) {
  if (pp->chi_min < 1 || pp->chi_max < pp->chi_min) return OR_ERR_ARG;
  double a = pp->alpha, one_minus_a = 1.0 - pp->alpha;
  int first = st->visits == 0;
  double sbar_prev = first ? (pp->ema_init_zero ? 0.0 : s_raw) : st->s_ema;
  double sbar;
  if (first && !pp->ema_init_zero) {
    sbar = s_raw;
  } else {
    double t1 = a * s_raw;
    double t2 = one_minus_a * sbar_prev;
    sbar = t1 + t2;
  }
  double sig = sbar;
  if (pp->beta > 0.0) {
    double trend = sbar - sbar_prev;
    double ext = pp->beta * trend;
    sig = sbar + ext;
  }
  /* second-order predictor (Sec. 7): + beta2 (Sbar(t) - 2 Sbar(t-1) + Sbar(t-2)), from the
   * third visit on (s_ema_prev holds Sbar(t-2) before this update) */
  if (pp->beta2 > 0.0 && st->visits >= 2) {
    double curv = (sbar - 2.0 * sbar_prev) + st->s_ema_prev;
    double ext2 = pp->beta2 * curv;
    sig = sig + ext2;
  }
  double e = sig - pp->s_target;
  double e_prev = first ? e : st->e_prev;
  double P = pp->kp * e;
  double di = pp->ki * e;
  double I = st->integ + di;
  double de = e - e_prev;
  double Dt = pp->kd * de;
  double pi = P + I;
  double u = pi + Dt;
  double delta = nearbyint(u);
  long raw = (long)st->chi + (long)delta;
  long c = raw;
  if (c < pp->chi_min) c = pp->chi_min;
  if (c > pp->chi_max) c = pp->chi_max;
  if (c != raw) I = I - di; /* anti-windup: undo this step's integral update */
  st->s_ema_prev = first ? sbar : st->s_ema;
  st->s_ema = sbar;
  st->e_prev = e;
  st->integ = I;
  st->chi = (int)c;
  st->visits += 1;
  if (chi_next) *chi_next = (int)c;
  if (terms) { terms[0] = P; terms[1] = I; terms[2] = Dt; terms[3] = u; terms[4] = sbar; terms[5] = e; }
  return OR_OK;
}

/* Algorithm 1 (Sec. 4): entropy -> EMA (Eq. 8, seeded with the first entropy unless
 * ema_init_zero) -> chi_target = ceil(gamma exp(S_ema)) (Eq. 7) -> clamp to
 * [chi_min, chi_max].  Shares the per-bond state with the PID (EMA fields,
 * chi, visits); terms[4] = S_ema, the PID terms are zero. */
int or_entropy_chi_update(const or_pid_params *pp, double gamma, or_pid_state *st, double s_raw, int *chi_next,
                          double *terms) {
  if (pp->chi_min < 1 || pp->chi_max < pp->chi_min || !(gamma >= 1.0)) return OR_ERR_ARG;
  int first = st->visits == 0;
  double sbar_prev = first ? (pp->ema_init_zero ? 0.0 : s_raw) : st->s_ema;
  double sbar;
  if (first && !pp->ema_init_zero) {
    sbar = s_raw;
  } else {
    double t1 = pp->alpha * s_raw;
    double t2 = (1.0 - pp->alpha) * sbar_prev;
    sbar = t1 + t2;
  }
  double target = ceil(gamma * exp(sbar));
  long c;
  if (target < pp->chi_min) c = pp->chi_min;
  else if (target > pp->chi_max) c = pp->chi_max;
  else c = (long)target;
  st->s_ema_prev = first ? sbar : st->s_ema;
  st->s_ema = sbar;
  st->chi = (int)c;
  st->visits += 1;
  if (chi_next) *chi_next = (int)c;
  if (terms) { terms[0] = terms[1] = terms[2] = terms[3] = terms[5] = 0.0; terms[4] = sbar; }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* One element out[a][s][t][c] of H_eff theta (Eq. 18), straight from the     */
/* definition: the left block first (sum over a'), then the right block       */
/* (sum over c'), then the two MPO tensors.  For sizes whose full product is  */
/* too slow here; the result must equal or_heff_apply's element.              */
/* ------------------------------------------------------------------------ */
double or_heff_element(int chl, int chr, int d, int D, const double *L, const double *W1, const double *W2,
                       const double *R, const double *th, int a, int s, int t, int c) {
  const size_t nq = (size_t)D * d * d * chr;
  double *T1 = dalloc(nq);                 /* T1[w][s'][t'][c'] = sum_a' L[a][w][a'] th[a'][s'][t'][c'] */
  for (int w = 0; w < D; ++w)
    for (size_t q = 0; q < (size_t)d * d * chr; ++q) {
      double acc = 0.0;
      for (int ap = 0; ap < chl; ++ap)
        acc += L[((size_t)a * D + w) * chl + ap] * th[(size_t)ap * d * d * chr + q];
      T1[(size_t)w * d * d * chr + q] = acc;
    }
  double *T2 = dalloc((size_t)D * D * d * d); /* T2[w][w''][s'][t'] = sum_c' R[c][w''][c'] T1[w][s'][t'][c'] */
  for (int w = 0; w < D; ++w)
    for (int wq = 0; wq < D; ++wq)
      for (int sp = 0; sp < d; ++sp)
        for (int tp = 0; tp < d; ++tp) {
          double acc = 0.0;
          for (int cp = 0; cp < chr; ++cp)
            acc += R[((size_t)c * D + wq) * chr + cp] * T1[(((size_t)w * d + sp) * d + tp) * chr + cp];
          T2[(((size_t)w * D + wq) * d + sp) * d + tp] = acc;
        }
  double out = 0.0;                         /* sum W1[w][w'][s][s'] W2[w'][w''][t][t'] T2[w][w''][s'][t'] */
  for (int w = 0; w < D; ++w)
    for (int wp = 0; wp < D; ++wp)
      for (int wq = 0; wq < D; ++wq)
        for (int sp = 0; sp < d; ++sp)
          for (int tp = 0; tp < d; ++tp)
            out += W1[(((size_t)w * D + wp) * d + s) * d + sp] * W2[(((size_t)wp * D + wq) * d + t) * d + tp] *
                   T2[(((size_t)w * D + wq) * d + sp) * d + tp];
  free(T1);
  free(T2);
  return out;
}

/* ------------------------------------------------------------------------ */
/* Two-site effective Hamiltonian applied to theta (Eq. 18), contracted in   */
/* the textbook order: L, then W_b, then W_{b+1}, then R.                     */
/* out[a][s][t][c] = sum L[a][w][a'] W1[w][w'][s][s'] W2[w'][w''][t][t']      */
/*                       R[c][w''][c'] theta[a'][s'][t'][c']                 */
/* ------------------------------------------------------------------------ */
int or_heff_apply(int chl, int chr, int d, int D, const double *L, const double *W1, const double *W2,
                  const double *R, const double *th, double *out) {
  size_t n_x = (size_t)chl * D * d * d * chr;
  double *X1 = dalloc(n_x), *X2 = dalloc(n_x), *X3 = dalloc(n_x);
  /* X1[a][w][s'][t'][c'] = sum_a' L[a][w][a'] th[a'][s'][t'][c'] */
  for (int a = 0; a < chl; ++a)
    for (int w = 0; w < D; ++w)
      for (int sp = 0; sp < d; ++sp)
        for (int tp = 0; tp < d; ++tp)
          for (int cp = 0; cp < chr; ++cp) {
            double s = 0.0;
            for (int ap = 0; ap < chl; ++ap)
              s += L[((size_t)a * D + w) * chl + ap] * th[(((size_t)ap * d + sp) * d + tp) * chr + cp];
            X1[((((size_t)a * D + w) * d + sp) * d + tp) * chr + cp] = s;
          }
  /* X2[a][w'][s][t'][c'] = sum_{w,s'} W1[w][w'][s][s'] X1[a][w][s'][t'][c'] */
  for (int a = 0; a < chl; ++a)
    for (int wp = 0; wp < D; ++wp)
      for (int s = 0; s < d; ++s)
        for (int tp = 0; tp < d; ++tp)
          for (int cp = 0; cp < chr; ++cp) {
            double acc = 0.0;
            for (int w = 0; w < D; ++w)
              for (int sp = 0; sp < d; ++sp)
                acc += W1[(((size_t)w * D + wp) * d + s) * d + sp] *
                       X1[((((size_t)a * D + w) * d + sp) * d + tp) * chr + cp];
            X2[((((size_t)a * D + wp) * d + s) * d + tp) * chr + cp] = acc;
          }
  /* X3[a][s][w''][t][c'] = sum_{w',t'} W2[w'][w''][t][t'] X2[a][w'][s][t'][c'] */
  for (int a = 0; a < chl; ++a)
    for (int s = 0; s < d; ++s)
      for (int wq = 0; wq < D; ++wq)
        for (int t = 0; t < d; ++t)
          for (int cp = 0; cp < chr; ++cp) {
            double acc = 0.0;
            for (int wp = 0; wp < D; ++wp)
              for (int tp = 0; tp < d; ++tp)
                acc += W2[(((size_t)wp * D + wq) * d + t) * d + tp] *
                       X2[((((size_t)a * D + wp) * d + s) * d + tp) * chr + cp];
            X3[((((size_t)a * d + s) * D + wq) * d + t) * chr + cp] = acc;
          }
  /* out[a][s][t][c] = sum_{w'',c'} X3[a][s][w''][t][c'] R[c][w''][c'] */
  for (int a = 0; a < chl; ++a)
    for (int s = 0; s < d; ++s)
      for (int t = 0; t < d; ++t)
        for (int c = 0; c < chr; ++c) {
          double acc = 0.0;
          for (int wq = 0; wq < D; ++wq)
            for (int cp = 0; cp < chr; ++cp)
              acc += X3[((((size_t)a * d + s) * D + wq) * d + t) * chr + cp] * R[((size_t)c * D + wq) * chr + cp];
          out[(((size_t)a * d + s) * d + t) * chr + c] = acc;
        }
  free(X1); free(X2); free(X3);
  return OR_OK;
}

/* Left environment grown by one left-canonical site A[a][s][b]:
 * Ln[b][w'][b'] = sum A[a][s][b] L[a][w][a'] W[w][w'][s][s'] A[a'][s'][b'] */
int or_env_left(int chl, int chn, int d, int D, const double *L, const double *W, const double *A, double *Ln) {
  double *T1 = dalloc((size_t)chl * D * d * chn), *T2 = dalloc((size_t)chl * D * d * chn);
  for (int a = 0; a < chl; ++a)
    for (int w = 0; w < D; ++w)
      for (int sp = 0; sp < d; ++sp)
        for (int bp = 0; bp < chn; ++bp) {
          double s = 0.0;
          for (int ap = 0; ap < chl; ++ap) s += L[((size_t)a * D + w) * chl + ap] * A[((size_t)ap * d + sp) * chn + bp];
          T1[(((size_t)a * D + w) * d + sp) * chn + bp] = s;
        }
  for (int a = 0; a < chl; ++a)
    for (int wp = 0; wp < D; ++wp)
      for (int s = 0; s < d; ++s)
        for (int bp = 0; bp < chn; ++bp) {
          double acc = 0.0;
          for (int w = 0; w < D; ++w)
            for (int sp = 0; sp < d; ++sp)
              acc += W[(((size_t)w * D + wp) * d + s) * d + sp] * T1[(((size_t)a * D + w) * d + sp) * chn + bp];
          T2[(((size_t)a * D + wp) * d + s) * chn + bp] = acc;
        }
  for (int b = 0; b < chn; ++b)
    for (int wp = 0; wp < D; ++wp)
      for (int bp = 0; bp < chn; ++bp) {
        double acc = 0.0;
        for (int a = 0; a < chl; ++a)
          for (int s = 0; s < d; ++s)
            acc += A[((size_t)a * d + s) * chn + b] * T2[(((size_t)a * D + wp) * d + s) * chn + bp];
        Ln[((size_t)b * D + wp) * chn + bp] = acc;
      }
  free(T1); free(T2);
  return OR_OK;
}

/* Right environment grown by one right-canonical site B[a][t][c]:
 * Rn[a][w][a'] = sum B[a][t][c] W[w][w''][t][t'] R[c][w''][c'] B[a'][t'][c'] */
int or_env_right(int chn, int chr, int d, int D, const double *R, const double *W, const double *B, double *Rn) {
  double *T1 = dalloc((size_t)chn * d * chr * D), *T2 = dalloc((size_t)chn * d * chr * D);
  /* T1[a'][t'][c][w''] = sum_c' B[a'][t'][c'] R[c][w''][c'] */
  for (int ap = 0; ap < chn; ++ap)
    for (int tp = 0; tp < d; ++tp)
      for (int c = 0; c < chr; ++c)
        for (int wq = 0; wq < D; ++wq) {
          double s = 0.0;
          for (int cp = 0; cp < chr; ++cp) s += B[((size_t)ap * d + tp) * chr + cp] * R[((size_t)c * D + wq) * chr + cp];
          T1[(((size_t)ap * d + tp) * chr + c) * D + wq] = s;
        }
  /* T2[a'][t][c][w] = sum_{w'',t'} W[w][w''][t][t'] T1[a'][t'][c][w''] */
  for (int ap = 0; ap < chn; ++ap)
    for (int t = 0; t < d; ++t)
      for (int c = 0; c < chr; ++c)
        for (int w = 0; w < D; ++w) {
          double acc = 0.0;
          for (int wq = 0; wq < D; ++wq)
            for (int tp = 0; tp < d; ++tp)
              acc += W[(((size_t)w * D + wq) * d + t) * d + tp] * T1[(((size_t)ap * d + tp) * chr + c) * D + wq];
          T2[(((size_t)ap * d + t) * chr + c) * D + w] = acc;
        }
  /* Rn[a][w][a'] = sum_{t,c} B[a][t][c] T2[a'][t][c][w] */
  for (int a = 0; a < chn; ++a)
    for (int w = 0; w < D; ++w)
      for (int ap = 0; ap < chn; ++ap) {
        double acc = 0.0;
        for (int t = 0; t < d; ++t)
          for (int c = 0; c < chr; ++c)
            acc += B[((size_t)a * d + t) * chr + c] * T2[(((size_t)ap * d + t) * chr + c) * D + w];
        Rn[((size_t)a * D + w) * chn + ap] = acc;
      }
  free(T1); free(T2);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Lanczos for the lowest eigenpair with full reorthogonalisation (CGS2).     */
/* The paper names no eigensolver for Eq. (18); this is the standard choice.  */
/* Per iteration: w = H v_j; h = V^T w (alpha_j = h_j); w -= V h; again;      */
/* beta_j = |w|; lowest eigenpair (theta, y) of T_j by Jacobi; stop when      */
/* |beta_j y_j| <= tol*max(1,|theta|) or beta_j < 1e-14.  At most kmax        */
/* vectors, then up to `restarts` restarts from the Ritz vector.              */
/* x: in = start vector, out = normalised Ritz vector.                        */
/* ------------------------------------------------------------------------ */
typedef void (*or_matvec_fn)(void *ctx, const double *x, double *y);

static int lanczos(size_t dim, or_matvec_fn mv, void *ctx, double *x, double tol, int kmax_in, int restarts,
                   int fixed_iters, double *E_out, int *iters_out) {
  int kmax = kmax_in;
  if ((size_t)kmax > dim) kmax = (int)dim;
  if (fixed_iters > 0) kmax = fixed_iters < (int)dim ? fixed_iters : (int)dim;
  double *V = dalloc((size_t)(kmax + 1) * dim);
  double *w = dalloc(dim), *h = dalloc(kmax + 1);
  double *al = dalloc(kmax + 1), *be = dalloc(kmax + 1);
  double *T = dalloc((size_t)(kmax + 1) * (kmax + 1)), *Y = dalloc((size_t)(kmax + 1) * (kmax + 1));
  double *ev = dalloc(kmax + 1), *y = dalloc(kmax + 1);
  int total = 0, conv = 0;
  double E = 0.0;
  double nx = sqrt(dot(dim, x, x));
  for (size_t i = 0; i < dim; ++i) x[i] /= nx;
  for (int rs = 0; rs <= restarts && !conv; ++rs) {
    memcpy(V, x, dim * sizeof(double));
    int j = 0, nkeep = 0;
    for (;;) {
      mv(ctx, V + (size_t)j * dim, w);
      ++total;
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i <= j; ++i) h[i] = dot(dim, V + (size_t)i * dim, w);
        if (pass == 0) al[j] = h[j];
        for (int i = 0; i <= j; ++i)
          for (size_t r = 0; r < dim; ++r) w[r] -= h[i] * V[(size_t)i * dim + r];
      }
      be[j] = sqrt(dot(dim, w, w));
      int n = j + 1;
      memset(T, 0, sizeof(double) * (size_t)n * n);
      for (int i = 0; i < n; ++i) T[(size_t)i * n + i] = al[i];
      for (int i = 0; i + 1 < n; ++i) { T[(size_t)i * n + i + 1] = be[i]; T[(size_t)(i + 1) * n + i] = be[i]; }
      or_sym_eig_jacobi(n, T, ev, Y);
      int imin = 0;
      for (int i = 1; i < n; ++i) if (ev[i] < ev[imin]) imin = i;
      E = ev[imin];
      for (int i = 0; i < n; ++i) y[i] = Y[(size_t)i * n + imin];
      double res = fabs(be[j] * y[j]);
      nkeep = n;
      if (fixed_iters > 0) {
        if (n >= kmax || be[j] < 1e-14) { conv = 1; break; }
      } else {
        if (res <= tol * (fabs(E) > 1.0 ? fabs(E) : 1.0) || be[j] < 1e-14) { conv = 1; break; }
        if (n >= kmax) break;
      }
      for (size_t r = 0; r < dim; ++r) V[(size_t)(j + 1) * dim + r] = w[r] / be[j];
      ++j;
    }
    memset(x, 0, dim * sizeof(double));
    for (int i = 0; i < nkeep; ++i)
      for (size_t r = 0; r < dim; ++r) x[r] += y[i] * V[(size_t)i * dim + r];
    nx = sqrt(dot(dim, x, x));
    for (size_t r = 0; r < dim; ++r) x[r] /= nx;
  }
  free(V); free(w); free(h); free(al); free(be); free(T); free(Y); free(ev); free(y);
  *E_out = E;
  *iters_out = total;
  return conv ? OR_OK : OR_ERR_NOCONV;
}

typedef struct { int model, N; const double *p; } ed_ctx;
static void ed_mv(void *c, const double *x, double *y) {
  ed_ctx *e = (ed_ctx *)c;
  or_ed_apply(e->model, e->N, e->p, x, y);
}

/* Ground state of H by the Lanczos above.  psi: in = start vector (or NULL
 * for a fixed deterministic start), out = ground vector (if non-NULL). */
int or_ed_ground(int model, int N, const double *p, double tol, double *E0, double *psi, int *iters) {
  size_t dim = (size_t)1 << N;
  double *x = dalloc(dim);
  if (psi) memcpy(x, psi, dim * sizeof(double));
  else
    for (size_t i = 0; i < dim; ++i) x[i] = 1.0 + 0.37 * sin(1.7 * (double)i + 0.3) + 1e-3 * (double)(i % 7);
  ed_ctx c = {model, N, p};
  int it = 0;
  int rc = lanczos(dim, ed_mv, &c, x, tol, 120, 8, 0, E0, &it);
  if (psi) memcpy(psi, x, dim * sizeof(double));
  if (iters) *iters = it;
  free(x);
  return rc;
}

typedef struct { int chl, chr, d, D; const double *L, *W1, *W2, *R; } heff_ctx;
static void heff_mv(void *c, const double *x, double *y) {
  heff_ctx *h = (heff_ctx *)c;
  or_heff_apply(h->chl, h->chr, h->d, h->D, h->L, h->W1, h->W2, h->R, x, y);
}

int or_lanczos_heff(int chl, int chr, int d, int D, const double *L, const double *W1, const double *W2,
                    const double *R, double *theta, double tol, int kmax, int restarts, int fixed_iters,
                    double *E, int *iters) {
  heff_ctx c = {chl, chr, d, D, L, W1, W2, R};
  return lanczos((size_t)chl * d * d * chr, heff_mv, &c, theta, tol, kmax, restarts, fixed_iters, E, iters);
}

/* ------------------------------------------------------------------------ */
/* Two-site DMRG with per-bond PID bond dimensions (Sec. 10, Eq. 18-19,      */
/* Algorithm 2).  A full sweep visits bonds 0..N-2 left to right, then       */
/* N-2..0 right to left.  Per visit: theta = A_b A_{b+1}; Lanczos; SVD;      */
/* entropy of the full spectrum; PID -> chi; keep k = min(chi, m, n);        */
/* renormalise sigma_k; move the centre; grow the environment.               */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n_sweeps, lanczos_kmax, lanczos_restarts, fixed_iters;
  double lanczos_tol;
  int fixed_chi; /* >0: keep min(fixed_chi, m, n), controller still logged */
  int pad;
  int chi_rule;  /* 0: PID (Algorithm 2); 1: standard threshold rule, keep min(chi_max, r) with
                    r = #{sigma > rule_param} (at least 1; Sec. 10); 2: Algorithm 1, gamma = rule_param */
  int pad2;
  double rule_param;
  double eps_target;      /* truncation-error target of the learned scheduler's rule (> 0) */
  const int *sched_pred;  /* NULL, or one rank proposal per visit in run order (0 = none): the
                             scheduler's proposals are inputs here, the network is not run */
} or_dmrg_opts;

#define OR_LOG_FIELDS 50
/* log record per visit (doubles):
 * 0 sweep, 1 dir (0 L->R, 1 R->L), 2 bond, 3 m, 4 n, 5 k, 6 chi_ctrl, 7 E,
 * 8 S, 9 S_ema, 10 eps, 11 wdisc, 12 gap, 13 lanczos_iters, 14 svd_sweeps,
 * 15 P, 16 I, 17 D, 18 u, 19 lanczos_ok, 20 sigma_0, 21 sigma_last_kept,
 * 22 k_needed, 23 proposal used (0 = none), 24 fallback, 25..49 scheduler inputs */

/* ------------------------------------------------------------------------ */
/* Learned-scheduler inputs, labels and fallback rule.  The network stands   */
/* in for the predictive scheduler of Sec. 7 (Eq. 16-17): it sees the bond's */
/* recent entropy history and its singular-value tail.  Definitions:        */
/*  - inputs (25): the last 8 EMA entropies of the bond (Eq. 8), oldest      */
/*    first; with fewer than 8 visits so far the oldest one fills the front;  */
/*    then ln sigma_j of the 16 largest singular values of the full spectrum */
/*    (descending), floored at ln 1e-16, a missing value counting as the     */
/*    floor; then the relative bond position (b + 1) / N.                    */
/*  - label: the smallest k >= 1 whose truncation error of Eq. (4),          */
/*    sqrt(sum_{j>=k} sigma_j^2), is at most eps_target (k = R always is).   */
/*  - rule: a proposal k_p is used unless the truncation error it would      */
/*    leave, Eq. (4) at min(k_p, R), exceeds eps_target; then the controller */
/*    decides (fallback).                                                    */
/* ------------------------------------------------------------------------ */
void or_sched_features(const double *ema_hist, int nhist, const double *S, int R, int bond, int N, double *f) {
  /* ema_hist: the bond's EMA entropies of all its visits so far, oldest first (nhist >= 1) */
  int have = nhist < 8 ? nhist : 8;
  const double *last = ema_hist + (nhist - have);
  for (int r = 0; r < 8; ++r) {
    int src = r - (8 - have);
    f[r] = last[src < 0 ? 0 : src];
  }
  const double lnfloor = log(1e-16);
  for (int r = 0; r < 16; ++r) {
    double v = lnfloor;
    if (r < R && S[r] > 0.0) {
      double l = log(S[r]);
      v = l > lnfloor ? l : lnfloor;
    }
    f[8 + r] = v;
  }
  f[24] = (double)(bond + 1) / (double)N;
}

/* truncation error of Eq. (4) when k values are kept (tail summed smallest-first) */
double or_trunc_error(int R, const double *S, int k) {
  double tail = 0.0;
  for (int j = R - 1; j >= k; --j) tail += S[j] * S[j];
  return sqrt(tail);
}

int or_k_needed(int R, const double *S, double eps_target) {
  for (int k = 1; k < R; ++k)
    if (or_trunc_error(R, S, k) <= eps_target) return k;
  return R;
}

static void right_canonicalize(int N, int d, int *chi, double **A) {
  for (int b = N - 1; b >= 1; --b) {
    int cl = chi[b - 1], cr = (b == N - 1) ? 1 : chi[b];
    int m = cl, n = d * cr, Rk = m < n ? m : n;
    double *S = dalloc(Rk), *U = dalloc((size_t)m * Rk), *V = dalloc((size_t)n * Rk);
    int info = 0;
    or_svd_jacobi(m, n, A[b], S, U, V, &info);
    /* A_b <- V^T (Rk x n), A_{b-1} <- A_{b-1} U S */
    double *Ab = dalloc((size_t)Rk * n);
    for (int k = 0; k < Rk; ++k)
      for (int j = 0; j < n; ++j) Ab[(size_t)k * n + j] = V[(size_t)j * Rk + k];
    int cll = (b - 1 == 0) ? 1 : chi[b - 2];
    int mrows = cll * d;
    double *US = dalloc((size_t)m * Rk);
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < Rk; ++k) US[(size_t)i * Rk + k] = U[(size_t)i * Rk + k] * S[k];
    double *Ap = dalloc((size_t)mrows * Rk);
    matmul(mrows, Rk, m, A[b - 1], US, Ap);
    free(A[b]); free(A[b - 1]);
    A[b] = Ab;
    A[b - 1] = Ap;
    chi[b - 1] = Rk;
    free(S); free(U); free(V); free(US);
  }
  int n0 = d * chi[0];
  double nrm = sqrt(dot(n0, A[0], A[0]));
  for (int i = 0; i < n0; ++i) A[0][i] /= nrm;
}

/* Inputs: W (N bulk MPO tensors, D x D x d x d), A_init packed (site-major),
 * chi_init (N-1 bond dims of A_init), pid params, opts.
 * Outputs: log (n_sweeps * 2*(N-1) * OR_LOG_FIELDS), E_sweep (n_sweeps),
 * chi_final (N-1), pid_final (N-1 states, may be NULL). */
int or_dmrg_run(int N, int d, int D, const double *W, const double *A_init, const int *chi_init,
                const or_pid_params *pp, const or_dmrg_opts *op, double *log, double *E_sweep, int *chi_final,
                or_pid_state *pid_final) {
  if (N < 2 || d < 1 || D < 1 || pp->chi_min < 1 || pp->chi_max < pp->chi_min) return OR_ERR_ARG;
  size_t wsz = (size_t)D * D * d * d;
  int *chi = (int *)malloc(sizeof(int) * (size_t)(N - 1));
  memcpy(chi, chi_init, sizeof(int) * (size_t)(N - 1));
  double **A = (double **)calloc((size_t)N, sizeof(double *));
  size_t off = 0;
  for (int i = 0; i < N; ++i) {
    int cl = i == 0 ? 1 : chi[i - 1], cr = i == N - 1 ? 1 : chi[i];
    size_t n = (size_t)cl * d * cr;
    A[i] = dalloc(n);
    memcpy(A[i], A_init + off, n * sizeof(double));
    off += n;
  }
  right_canonicalize(N, d, chi, A);
#define CL(i) ((i) == 0 ? 1 : chi[(i)-1])
#define CR(i) ((i) == N - 1 ? 1 : chi[(i)])
  double **Le = (double **)calloc((size_t)N, sizeof(double *));
  double **Re = (double **)calloc((size_t)N, sizeof(double *));
  Le[0] = dalloc(D); Le[0][D - 1] = 1.0;
  Re[N - 1] = dalloc(D); Re[N - 1][0] = 1.0;
  for (int i = N - 1; i >= 2; --i) {
    Re[i - 1] = dalloc((size_t)CL(i) * D * CL(i));
    or_env_right(CL(i), CR(i), d, D, Re[i], W + (size_t)i * wsz, A[i], Re[i - 1]);
  }
  or_pid_state *ps = (or_pid_state *)calloc((size_t)(N - 1), sizeof(or_pid_state));
  for (int b = 0; b < N - 1; ++b) ps[b].chi = pp->chi_min;
  /* every visit's EMA entropy per bond (two visits per bond and sweep) */
  const size_t hist_cap = 2 * (size_t)(op->n_sweeps > 0 ? op->n_sweeps : 1);
  double *hist = dalloc(hist_cap * (size_t)(N - 1));
  int *nhist = (int *)calloc((size_t)(N - 1), sizeof(int));
  int rc_all = OR_OK;
  size_t rec = 0;
  for (int sw = 0; sw < op->n_sweeps; ++sw) {
    double E = 0.0;
    for (int half = 0; half < 2; ++half)
      for (int step = 0; step < N - 1; ++step) {
        int b = half == 0 ? step : N - 2 - step;
        int chl = CL(b), chm = chi[b], chr = CR(b + 1);
        int m = chl * d, n = d * chr;
        double *th = dalloc((size_t)m * n);
        matmul(m, n, chm, A[b], A[b + 1], th);
        int iters = 0;
        int rc = or_lanczos_heff(chl, chr, d, D, Le[b], W + (size_t)b * wsz, W + (size_t)(b + 1) * wsz, Re[b + 1], th,
                                 op->lanczos_tol, op->lanczos_kmax, op->lanczos_restarts, op->fixed_iters, &E, &iters);
        if (rc != OR_OK) rc_all = rc;
        int Rk = m < n ? m : n;
        double *S = dalloc(Rk), *U = dalloc((size_t)m * Rk), *V = dalloc((size_t)n * Rk);
        int sinfo = 0;
        or_svd_jacobi(m, n, th, S, U, V, &sinfo);
        double sp[4];
        or_spectrum(Rk, S, Rk, sp);
        double terms[6] = {0};
        int chi_next = 0;
        if (op->chi_rule == 2) or_entropy_chi_update(pp, op->rule_param, &ps[b], sp[1], &chi_next, terms);
        else or_pid_update(pp, &ps[b], sp[1], &chi_next, terms);
        int keep = op->fixed_chi > 0 ? op->fixed_chi : chi_next;
        if (op->fixed_chi <= 0 && op->chi_rule == 1) {
          int r = 0;
          for (int j = 0; j < Rk; ++j) r += S[j] > op->rule_param;
          if (r < 1) r = 1;
          keep = r < pp->chi_max ? r : pp->chi_max;
        }
        /* scheduler inputs and label of this visit; the bond's EMA history grows by one */
        double epst = op->eps_target > 0.0 ? op->eps_target : 1e-8;
        hist[(size_t)b * hist_cap + nhist[b]] = terms[4];
        nhist[b] += 1;
        double feat[25];
        or_sched_features(hist + (size_t)b * hist_cap, nhist[b], S, Rk, b, N, feat);
        int kneed = or_k_needed(Rk, S, epst);
        int prop = 0, fallback = 0;
        if (op->sched_pred && op->fixed_chi <= 0 && op->chi_rule == 0 && op->sched_pred[rec] > 0) {
          prop = op->sched_pred[rec];
          int kp = prop < Rk ? prop : Rk;
          if (or_trunc_error(Rk, S, kp) > epst) fallback = 1;
          else keep = prop;
        }
        int k = keep < Rk ? keep : Rk;
        or_spectrum(Rk, S, k, sp);
        double nk = 0.0;
        for (int j = k - 1; j >= 0; --j) nk += S[j] * S[j];
        nk = sqrt(nk);
        double gap = k < Rk ? (S[k - 1] - S[k]) / S[0] : 1.0;
        if (log) {
          double *r = log + rec * OR_LOG_FIELDS;
          r[0] = sw; r[1] = half; r[2] = b; r[3] = m; r[4] = n; r[5] = k; r[6] = chi_next; r[7] = E;
          r[8] = sp[1]; r[9] = terms[4]; r[10] = sp[2]; r[11] = sp[3]; r[12] = gap; r[13] = iters;
          r[14] = sinfo; r[15] = terms[0]; r[16] = terms[1]; r[17] = terms[2]; r[18] = terms[3];
          r[19] = rc == OR_OK; r[20] = S[0]; r[21] = S[k - 1];
          r[22] = kneed; r[23] = prop; r[24] = fallback;
          for (int q = 0; q < 25; ++q) r[25 + q] = feat[q];
        }
        ++rec;
        double *Ab = dalloc((size_t)m * k), *Ab1 = dalloc((size_t)k * n);
        for (int i = 0; i < m; ++i)
          for (int j = 0; j < k; ++j)
            Ab[(size_t)i * k + j] = U[(size_t)i * Rk + j] * (half == 1 ? S[j] / nk : 1.0);
        for (int j = 0; j < k; ++j)
          for (int c = 0; c < n; ++c)
            Ab1[(size_t)j * n + c] = V[(size_t)c * Rk + j] * (half == 0 ? S[j] / nk : 1.0);
        free(A[b]); free(A[b + 1]);
        A[b] = Ab; A[b + 1] = Ab1;
        chi[b] = k;
        if (half == 0) {
          free(Le[b + 1]);
          Le[b + 1] = dalloc((size_t)k * D * k);
          or_env_left(chl, k, d, D, Le[b], W + (size_t)b * wsz, A[b], Le[b + 1]);
        } else {
          free(Re[b]);
          Re[b] = dalloc((size_t)k * D * k);
          or_env_right(k, chr, d, D, Re[b + 1], W + (size_t)(b + 1) * wsz, A[b + 1], Re[b]);
        }
        free(th); free(S); free(U); free(V);
      }
    if (E_sweep) E_sweep[sw] = E;
  }
  if (chi_final) memcpy(chi_final, chi, sizeof(int) * (size_t)(N - 1));
  if (pid_final) memcpy(pid_final, ps, sizeof(or_pid_state) * (size_t)(N - 1));
  for (int i = 0; i < N; ++i) { free(A[i]); free(Le[i]); free(Re[i]); }
  free(A); free(Le); free(Re); free(chi); free(ps); free(hist); free(nhist);
#undef CL
#undef CR
  return rc_all;
}

/* Right-canonical form of a packed MPS (for tests): writes the canonical
 * tensors packed into A_out (same capacity as A_in) and the bond dims. */
int or_right_canonical(int N, int d, const double *A_in, const int *chi_in, double *A_out, int *chi_out) {
  int *chi = (int *)malloc(sizeof(int) * (size_t)(N - 1));
  memcpy(chi, chi_in, sizeof(int) * (size_t)(N - 1));
  double **A = (double **)calloc((size_t)N, sizeof(double *));
  size_t off = 0;
  for (int i = 0; i < N; ++i) {
    int cl = i == 0 ? 1 : chi[i - 1], cr = i == N - 1 ? 1 : chi[i];
    size_t n = (size_t)cl * d * cr;
    A[i] = dalloc(n);
    memcpy(A[i], A_in + off, n * sizeof(double));
    off += n;
  }
  right_canonicalize(N, d, chi, A);
  off = 0;
  for (int i = 0; i < N; ++i) {
    int cl = i == 0 ? 1 : chi[i - 1], cr = i == N - 1 ? 1 : chi[i];
    size_t n = (size_t)cl * d * cr;
    memcpy(A_out + off, A[i], n * sizeof(double));
    off += n;
    free(A[i]);
  }
  memcpy(chi_out, chi, sizeof(int) * (size_t)(N - 1));
  free(A); free(chi);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Learned bond-dimension scheduler (the learned stand-in for the predictive */
/* scheduler of Sec. 7): a multilayer perceptron 25 -> 64 -> 64 -> 1 with    */
/* tanh hidden units and a linear output, trained by mean-squared error with */
/* Adam (Kingma & Ba 2015).  Parameter layout (5889 values):                  */
/*   W1[64][25] b1[64] W2[64][64] b2[64] W3[64] b3                            */
/* ------------------------------------------------------------------------ */
#define MLP_IN 25
#define MLP_H 64
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)

int or_mlp_nparam(void) { return MLP_NPARAM; }

/* y[b] = W3 . tanh(W2 tanh(W1 x_b + b1) + b2) + b3 */
void or_mlp_forward(const double *p, int B, const double *x, double *y) {
  const double *W1 = p, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
  const double *W3 = b2 + MLP_H, *b3 = W3 + MLP_H;
  for (int b = 0; b < B; ++b) {
    double h1[MLP_H], h2[MLP_H];
    for (int i = 0; i < MLP_H; ++i) {
      double s = b1[i];
      for (int k = 0; k < MLP_IN; ++k) s += W1[i * MLP_IN + k] * x[(size_t)b * MLP_IN + k];
      h1[i] = tanh(s);
    }
    for (int i = 0; i < MLP_H; ++i) {
      double s = b2[i];
      for (int k = 0; k < MLP_H; ++k) s += W2[i * MLP_H + k] * h1[k];
      h2[i] = tanh(s);
    }
    double s = b3[0];
    for (int k = 0; k < MLP_H; ++k) s += W3[k] * h2[k];
    y[b] = s;
  }
}

/* loss = (1/B) sum_b (y_b - t_b)^2 and its gradient with respect to p
 * (chain rule through the three layers; d tanh(s)/ds = 1 - tanh(s)^2). */
double or_mlp_loss_grad(const double *p, int B, const double *x, const double *t, double *g) {
  const double *W1 = p, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
  const double *W3 = b2 + MLP_H, *b3 = W3 + MLP_H;
  double *gW1 = g, *gb1 = gW1 + MLP_H * MLP_IN, *gW2 = gb1 + MLP_H, *gb2 = gW2 + MLP_H * MLP_H;
  double *gW3 = gb2 + MLP_H, *gb3 = gW3 + MLP_H;
  memset(g, 0, sizeof(double) * MLP_NPARAM);
  double loss = 0.0;
  for (int b = 0; b < B; ++b) {
    const double *xb = x + (size_t)b * MLP_IN;
    double h1[MLP_H], h2[MLP_H], d2[MLP_H], d1[MLP_H];
    for (int i = 0; i < MLP_H; ++i) {
      double s = b1[i];
      for (int k = 0; k < MLP_IN; ++k) s += W1[i * MLP_IN + k] * xb[k];
      h1[i] = tanh(s);
    }
    for (int i = 0; i < MLP_H; ++i) {
      double s = b2[i];
      for (int k = 0; k < MLP_H; ++k) s += W2[i * MLP_H + k] * h1[k];
      h2[i] = tanh(s);
    }
    double y = b3[0];
    for (int k = 0; k < MLP_H; ++k) y += W3[k] * h2[k];
    const double r = y - t[b];
    loss += r * r;
    const double dy = 2.0 * r / B;
    gb3[0] += dy;
    for (int k = 0; k < MLP_H; ++k) {
      gW3[k] += dy * h2[k];
      d2[k] = dy * W3[k] * (1.0 - h2[k] * h2[k]);
    }
    for (int i = 0; i < MLP_H; ++i) {
      gb2[i] += d2[i];
      for (int k = 0; k < MLP_H; ++k) gW2[i * MLP_H + k] += d2[i] * h1[k];
    }
    for (int k = 0; k < MLP_H; ++k) {
      double s = 0.0;
      for (int i = 0; i < MLP_H; ++i) s += W2[i * MLP_H + k] * d2[i];
      d1[k] = s * (1.0 - h1[k] * h1[k]);
    }
    for (int i = 0; i < MLP_H; ++i) {
      gb1[i] += d1[i];
      for (int k = 0; k < MLP_IN; ++k) gW1[i * MLP_IN + k] += d1[i] * xb[k];
    }
  }
  return loss / B;
}

/* One Adam step at step count t (1-based): m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, p -= lr * (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps). */
void or_adam_step(int n, double *p, const double *g, double *m, double *v, int t, double lr, double b1, double b2,
                  double eps) {
  const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (int i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}
