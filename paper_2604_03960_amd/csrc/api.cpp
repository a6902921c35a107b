// Host side of the C ABI: context, H_eff application, truncated SVD, the
// EMA/PID controller, MPO builders and the device-resident two-site DMRG
// sweep.  Every numerical step runs in the kernels of gemm.hip, vec.hip and
// svd.hip; the host only sequences launches, reads back the Lanczos
// coefficients and the entropy, and runs O(1) controller arithmetic and the
// O(j) tridiagonal eigensolve of the Lanczos recurrence.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

namespace tna {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

// ---------------------------------------------------------------- kernel timing
namespace {
struct KStat {
  long count = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
};
struct Pending {
  std::string name;
  hipEvent_t a, b;
  double flops, bytes;
};
struct Timing {
  std::mutex mu;
  bool on = false;
  std::string prefix;
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  std::map<std::string, KStat> stats;
  hipEvent_t open_a = nullptr;
  std::string open_name;
} g_tm;

hipEvent_t take_event() {
  if (!g_tm.pool.empty()) {
    hipEvent_t e = g_tm.pool.back();
    g_tm.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void drain_pending() {
  for (auto &p : g_tm.pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    KStat &k = g_tm.stats[p.name];
    k.count += 1;
    k.ms += ms;
    k.flops += p.flops;
    k.bytes += p.bytes;
    g_tm.pool.push_back(p.a);
    g_tm.pool.push_back(p.b);
  }
  g_tm.pending.clear();
}
}  // namespace

bool timing_on() { return g_tm.on; }

bool timing_may_match(const char *name_prefix) {
  if (!g_tm.on) return false;
  const size_t a = g_tm.prefix.size(), b = std::strlen(name_prefix);
  return a == 0 || std::strncmp(g_tm.prefix.c_str(), name_prefix, a < b ? a : b) == 0;
}

bool timing_wanted(const char *name) {
  if (!g_tm.on) return false;
  return g_tm.prefix.empty() || std::strncmp(name, g_tm.prefix.c_str(), g_tm.prefix.size()) == 0;
}

void timer_begin(const char *name, hipStream_t s) {
  if (!timing_wanted(name)) return;
  std::lock_guard<std::mutex> lk(g_tm.mu);
  g_tm.open_a = take_event();
  g_tm.open_name = name;
  (void)hipEventRecord(g_tm.open_a, s);
}

void timer_end(const char *name, double flops, double bytes, hipStream_t s) {
  if (!timing_wanted(name)) return;
  std::lock_guard<std::mutex> lk(g_tm.mu);
  if (!g_tm.open_a || g_tm.open_name != name) return;
  hipEvent_t b = take_event();
  (void)hipEventRecord(b, s);
  g_tm.pending.push_back(Pending{name, g_tm.open_a, b, flops, bytes});
  g_tm.open_a = nullptr;
  if (g_tm.pending.size() > 8192) drain_pending();
}

void timer_add_work(const char *name, double flops, double bytes) {
  if (!timing_wanted(name)) return;
  std::lock_guard<std::mutex> lk(g_tm.mu);
  for (auto it = g_tm.pending.rbegin(); it != g_tm.pending.rend(); ++it)
    if (it->name == name) {
      it->flops += flops;
      it->bytes += bytes;
      return;
    }
}

tna_status post_launch(const char *what) {
  static const int dbg = [] {
    const char *e = std::getenv("TNA_DEBUG_SYNC");
    return e && e[0] == '1';
  }();
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && dbg) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return TNA_ERR_DEVICE;
  }
  return TNA_OK;
}

// ---------------------------------------------------------------- contraction recipes
// out = H_eff x (Eq. 18): S1 X = L x; S2 Z = W12-mix(X); S4 out = Z R^T.
tna_status heff_device(const HeffOp &h, const double *x, double *out, hipStream_t s) {
  const int chl = h.chl, chr = h.chr, d = h.d, D = h.D;
  const bool f32 = h.prec != TNA_HEFF_F64;
  const int tc = f32 ? G_F32 : G_F64;
  GemmArgs g{};
  // S1: X[(a,w)][(s',t',c')] = sum_a' L[(a,w)][a'] theta[a'][(s',t',c')]
  g.M = chl * D; g.N = d * d * chr; g.K = chl;
  g.A = h.L; g.lda = chl; g.transA = 0; g.typeA = tc;
  g.B = x; g.ldb = d * d * chr; g.transB = 0; g.typeB = G_F64;
  g.C = h.X; g.ldc = d * d * chr; g.typeC = tc;
  g.alpha = 1.0; g.beta = 0.0; g.batch = 1; g.compute = tc; g.bf16x3 = h.prec == TNA_HEFF_BF16X3;
  TNA_TRY(gemm(g, s));
  // S2: Z[a][s][t][w''][c'] = sum W12[(s,t,w'')][(w,s',t')] X[a][w][s'][t'][c']
  MixArgs m{};
  m.n0 = chl; m.n1 = chr;
  m.is0 = (int64_t)D * d * d * chr; m.is1 = 1;
  m.os0 = (int64_t)d * d * D * chr; m.os1 = 1;
  m.I = D * d * d; m.J = d * d * D;
  for (int w = 0; w < D; ++w)
    for (int sp = 0; sp < d; ++sp)
      for (int tp = 0; tp < d; ++tp) m.ioff[(w * d + sp) * d + tp] = w * d * d * chr + sp * d * chr + tp * chr;
  for (int s_ = 0; s_ < d; ++s_)
    for (int t = 0; t < d; ++t)
      for (int wq = 0; wq < D; ++wq) m.ooff[(s_ * d + t) * D + wq] = s_ * d * D * chr + t * D * chr + wq * chr;
  m.in = h.X; m.type_in = tc; m.out = h.Z; m.type_out = tc; m.M = h.M12;
  TNA_TRY(mix(m, s));
  // S4: out[(a,s,t)][c] = sum_{(w'',c')} Z[(a,s,t)][(w'',c')] R[c][(w'',c')]
  g = GemmArgs{};
  g.M = chl * d * d; g.N = chr; g.K = D * chr;
  g.A = h.Z; g.lda = D * chr; g.transA = 0; g.typeA = tc;
  g.B = h.R; g.ldb = D * chr; g.transB = 1; g.typeB = tc;
  g.C = out; g.ldc = chr; g.typeC = G_F64;
  g.alpha = 1.0; g.beta = 0.0; g.batch = 1; g.compute = tc; g.bf16x3 = h.prec == TNA_HEFF_BF16X3;
  return gemm(g, s);
}

// Ln[b][w'][b'] = sum A[a][s][b] L[a][w][a'] W[w][w'][s][s'] A[a'][s'][b']
tna_status env_left(int chl, int k, int d, int D, const double *L, const double *Ml, const double *A,
                           double *T1, double *T2, double *Ln, hipStream_t s) {
  GemmArgs g{};
  g.M = chl * D; g.N = d * k; g.K = chl;
  g.A = L; g.lda = chl; g.B = A; g.ldb = d * k; g.C = T1; g.ldc = d * k;
  g.alpha = 1.0; g.batch = 1; g.compute = G_F64;
  TNA_TRY(gemm(g, s));
  MixArgs m{};
  m.n0 = chl; m.n1 = k;
  m.is0 = (int64_t)D * d * k; m.is1 = 1;
  m.os0 = (int64_t)d * D * k; m.os1 = 1;
  m.I = D * d; m.J = d * D;
  for (int w = 0; w < D; ++w)
    for (int sp = 0; sp < d; ++sp) m.ioff[w * d + sp] = w * d * k + sp * k;
  for (int s_ = 0; s_ < d; ++s_)
    for (int wp = 0; wp < D; ++wp) m.ooff[s_ * D + wp] = s_ * D * k + wp * k;
  m.in = T1; m.type_in = G_F64; m.out = T2; m.type_out = G_F64; m.M = Ml;
  TNA_TRY(mix(m, s));
  g = GemmArgs{};
  g.M = k; g.N = D * k; g.K = chl * d;
  g.A = A; g.lda = k; g.transA = 1; g.B = T2; g.ldb = D * k; g.C = Ln; g.ldc = D * k;
  g.alpha = 1.0; g.batch = 1; g.compute = G_F64;
  return gemm(g, s);
}

// Rn[a][w][a'] = sum B[a][t][c] W[w][w''][t][t'] R[c][w''][c'] B[a'][t'][c']
tna_status env_right(int k, int chr, int d, int D, const double *R, const double *Mr, const double *B,
                            double *T1, double *T2, double *Rn, hipStream_t s) {
  GemmArgs g{};
  g.M = chr * D; g.N = k * d; g.K = chr;
  g.A = R; g.lda = chr; g.B = B; g.ldb = chr; g.transB = 1; g.C = T1; g.ldc = k * d;
  g.alpha = 1.0; g.batch = 1; g.compute = G_F64;
  TNA_TRY(gemm(g, s));
  MixArgs m{};
  m.n0 = chr; m.n1 = k;
  m.is0 = (int64_t)D * k * d; m.is1 = d;
  m.os0 = (int64_t)D * k; m.os1 = 1;
  m.I = D * d; m.J = d * D;
  for (int wq = 0; wq < D; ++wq)
    for (int tp = 0; tp < d; ++tp) m.ioff[wq * d + tp] = wq * k * d + tp;
  for (int t = 0; t < d; ++t)
    for (int w = 0; w < D; ++w) m.ooff[t * D + w] = t * chr * D * k + w * k;
  m.in = T1; m.type_in = G_F64; m.out = T2; m.type_out = G_F64; m.M = Mr;
  TNA_TRY(mix(m, s));
  g = GemmArgs{};
  g.M = k; g.N = D * k; g.K = d * chr;
  g.A = B; g.lda = d * chr; g.B = T2; g.ldb = D * k; g.C = Rn; g.ldc = D * k;
  g.alpha = 1.0; g.batch = 1; g.compute = G_F64;
  return gemm(g, s);
}

// ---------------------------------------------------------------- tridiagonal eigenpair
// Lowest eigenvalue of the symmetric tridiagonal (a, b) by Sturm-count
// bisection, eigenvector by two steps of inverse iteration (Gaussian
// elimination with partial pivoting on T - lambda I).
double tridiag_lowest_host(int n, const double *a, const double *b, double *y) {
  if (n == 1) {
    y[0] = 1.0;
    return a[0];
  }
  double lo = std::numeric_limits<double>::infinity(), hi = -lo, amax = 0.0;
  for (int i = 0; i < n; ++i) {
    double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < n - 1 ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
    amax = std::max(amax, std::fabs(a[i]) + r);
  }
  const double tiny = std::numeric_limits<double>::min() / std::numeric_limits<double>::epsilon();
  auto count_below = [&](double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < n; ++i) {
      if (q == 0.0) q = -tiny;
      q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  const double lam = 0.5 * (lo + hi);
  // inverse iteration
  std::vector<double> dl(n), dd(n), du(n), du2(n), x(n, 1.0);
  const double shift = lam - 4.0 * std::numeric_limits<double>::epsilon() * std::max(amax, 1.0);
  for (int rep = 0; rep < 3; ++rep) {
    for (int i = 0; i < n; ++i) {
      dd[i] = a[i] - shift;
      if (i < n - 1) { du[i] = b[i]; dl[i] = b[i]; }
    }
    // LU with partial pivoting of a tridiagonal matrix (dgtsv-like), solving in place
    std::vector<double> rhs = x;
    std::vector<int> swp(n, 0);
    for (int i = 0; i < n; ++i) du2[i] = 0.0;
    for (int i = 0; i < n - 1; ++i) {
      if (std::fabs(dd[i]) >= std::fabs(dl[i])) {
        if (dd[i] == 0.0) dd[i] = tiny;
        const double f = dl[i] / dd[i];
        dd[i + 1] -= f * du[i];
        rhs[i + 1] -= f * rhs[i];
        dl[i] = 0.0;
      } else {
        const double f = dd[i] / dl[i];
        dd[i] = dl[i];
        double t = dd[i + 1];
        dd[i + 1] = du[i] - f * t;
        du[i] = t;
        if (i < n - 2) {
          du2[i] = du[i + 1];
          du[i + 1] = -f * du[i + 1];
        }
        std::swap(rhs[i], rhs[i + 1]);
        rhs[i + 1] -= f * rhs[i];
      }
    }
    if (dd[n - 1] == 0.0) dd[n - 1] = tiny;
    x[n - 1] = rhs[n - 1] / dd[n - 1];
    if (n > 1) x[n - 2] = (rhs[n - 2] - du[n - 2] * x[n - 1]) / dd[n - 2];
    for (int i = n - 3; i >= 0; --i) x[i] = (rhs[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / dd[i];
    double nr = 0.0;
    for (int i = 0; i < n; ++i) nr += x[i] * x[i];
    nr = std::sqrt(nr);
    for (int i = 0; i < n; ++i) x[i] /= nr;
  }
  // sign convention: first component non-negative
  const double sg = x[0] < 0 ? -1.0 : 1.0;
  for (int i = 0; i < n; ++i) y[i] = sg * x[i];
  return lam;
}

// ---------------------------------------------------------------- controller
#pragma clang fp contract(off)
tna_status pid_update(const tna_pid_params *p, tna_pid_state *st, double s_raw, int *chi_next,
                             double *terms) {
  if (!p || !st) {
    set_error("pid: null argument");
    return TNA_ERR_ARG;
  }
  if (p->chi_min < 1 || p->chi_max < p->chi_min) {
    set_error("pid: need 1 <= chi_min <= chi_max");
    return TNA_ERR_ARG;
  }
  if (!std::isfinite(s_raw)) {
    set_error("pid: non-finite entropy");
    return TNA_ERR_NONFINITE;
  }
  const bool first = st->visits == 0;
  const double a = p->alpha;
  const double keep = 1.0 - p->alpha;
  // Eq. (8) EMA, seeded on the first visit
  const double prev = first ? (p->ema_init_zero ? 0.0 : s_raw) : st->s_ema;
  double sbar;
  if (first && !p->ema_init_zero) sbar = s_raw;
  else {
    const double fresh = a * s_raw;
    const double old = keep * prev;
    sbar = fresh + old;
  }
  // Eq. (16) predictor (beta > 0), then Eq. (9) error
  double signal = sbar;
  if (p->beta > 0.0) {
    const double slope = sbar - prev;
    const double ahead = p->beta * slope;
    signal = sbar + ahead;
  }
  // second-order predictor (Sec. 7): the EMA's curvature, from the third visit on (s_ema_prev
  // holds the EMA two visits back until this update)
  if (p->beta2 > 0.0 && st->visits >= 2) {
    const double curv = (sbar - 2.0 * prev) + st->s_ema_prev;
    const double extra = p->beta2 * curv;
    signal = signal + extra;
  }
  const double e = signal - p->s_target;
  const double e_last = first ? e : st->e_prev;
  // Algorithm 2
  const double P = p->kp * e;
  const double dI = p->ki * e;
  double I = st->integ + dI;
  const double de = e - e_last;
  const double Dd = p->kd * de;
  const double pi = P + I;
  const double u = pi + Dd;
  const double step = std::nearbyint(u);
  const long raw = (long)st->chi + (long)step;
  long chi = raw < p->chi_min ? p->chi_min : raw;
  if (chi > p->chi_max) chi = p->chi_max;
  if (chi != raw) I = I - dI;  // anti-windup: the integral step is undone
  st->s_ema_prev = first ? sbar : st->s_ema;
  st->s_ema = sbar;
  st->e_prev = e;
  st->integ = I;
  st->chi = (int)chi;
  st->visits += 1;
  if (chi_next) *chi_next = (int)chi;
  if (terms) {
    terms[0] = P; terms[1] = I; terms[2] = Dd; terms[3] = u; terms[4] = sbar; terms[5] = e;
  }
  return TNA_OK;
}

// Algorithm 1 (Eq. 6-8): the EMA as in pid_update, then clamp(ceil(gamma exp(S_ema)), chi_min, chi_max)
tna_status entropy_update(const tna_pid_params *p, double gamma, tna_pid_state *st, double s_raw, int *chi_next,
                          double *terms) {
  if (!p || !st) {
    set_error("entropy rule: null argument");
    return TNA_ERR_ARG;
  }
  if (p->chi_min < 1 || p->chi_max < p->chi_min || !(gamma >= 1.0) || !std::isfinite(gamma)) {
    set_error("entropy rule: need 1 <= chi_min <= chi_max and a finite gamma >= 1");
    return TNA_ERR_ARG;
  }
  if (!std::isfinite(s_raw)) {
    set_error("entropy rule: non-finite entropy");
    return TNA_ERR_NONFINITE;
  }
  const bool first = st->visits == 0;
  const double prev = first ? (p->ema_init_zero ? 0.0 : s_raw) : st->s_ema;
  double sbar;
  if (first && !p->ema_init_zero) sbar = s_raw;
  else {
    const double fresh = p->alpha * s_raw;
    const double old = (1.0 - p->alpha) * prev;
    sbar = fresh + old;
  }
  const double target = std::ceil(gamma * std::exp(sbar));
  long chi = target < (double)p->chi_min ? p->chi_min : target > (double)p->chi_max ? p->chi_max : (long)target;
  st->s_ema_prev = first ? sbar : st->s_ema;
  st->s_ema = sbar;
  st->chi = (int)chi;
  st->visits += 1;
  if (chi_next) *chi_next = (int)chi;
  if (terms) {
    terms[0] = terms[1] = terms[2] = terms[3] = terms[5] = 0.0;
    terms[4] = sbar;
  }
  return TNA_OK;
}
#pragma clang fp contract(on)

}  // namespace tna

using namespace tna;

namespace tna {
tna_status heff_check_args(tna_ctx c, int chi_l, int chi_r, int d, int D, const double *L, const double *W1,
                           const double *W2, const double *R, const double *theta, double *out, int prec) {
  if (!c || !L || !W1 || !W2 || !R || !theta || !out) {
    set_error("heff_apply: null argument");
    return TNA_ERR_ARG;
  }
  if (chi_l < 1 || chi_r < 1 || d < 1 || D < 1 || D * d * d > 32) {
    set_error("heff_apply: need chi >= 1 and D*d*d <= 32");
    return TNA_ERR_ARG;
  }
  if (prec < 0 || prec > 2) {
    set_error("heff_apply: bad precision");
    return TNA_ERR_ARG;
  }
  if (theta == out) {
    set_error("heff_apply: out must not alias theta");
    return TNA_ERR_ARG;
  }
  if (prec == TNA_HEFF_BF16X3) {
    set_error("heff_apply: BF16x3 not built");
    return TNA_ERR_UNSUPPORTED;
  }
  return TNA_OK;
}
}  // namespace tna

// ====================================================================== ABI
extern "C" {

const char *tna_last_error(void) { return g_err.c_str(); }

tna_status tna_create(tna_ctx *out, int device, void *hip_stream) {
  if (!out) {
    set_error("tna_create: null out");
    return TNA_ERR_ARG;
  }
  int n = 0;
  TNA_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) {
    set_error("tna_create: no such device");
    return TNA_ERR_ARG;
  }
  TNA_HIP(hipSetDevice(device));
  TNA_TRY(noalloc_init(device));  // device address of the fixed scratch of tna_heff_apply_noalloc
  auto c = std::make_unique<tna_ctx_s>();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  TNA_HIP(hipHostMalloc((void **)&c->host_ctr, sizeof(int) * 16, hipHostMallocDefault));
  TNA_HIP(hipHostMalloc((void **)&c->host_scal, sizeof(double) * 64, hipHostMallocDefault));
  TNA_TRY(c->misc.ensure(sizeof(double) * 1024));
  TNA_TRY(c->part.ensure(sizeof(double) * 512 * 128));
  *out = c.release();
  return TNA_OK;
}

tna_status tna_destroy(tna_ctx c) {
  if (!c) return TNA_OK;
  if (c->children > 0) {
    set_error("tna_destroy: " + std::to_string(c->children) +
              " DMRG run(s) or network(s) made from this context are still alive; destroy them first");
    return TNA_ERR_ARG;
  }
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (DevBuf *b : {&c->x, &c->z, &c->lf, &c->rf, &c->m12, &c->part, &c->misc, &c->spec}) b->release();
  c->svd.release();
  if (c->host_ctr) (void)hipHostFree(c->host_ctr);
  if (c->host_scal) (void)hipHostFree(c->host_scal);
  delete c;
  return TNA_OK;
}

tna_status tna_set_stream(tna_ctx c, void *hip_stream) {
  if (!c) {
    set_error("null context");
    return TNA_ERR_ARG;
  }
  c->stream = static_cast<hipStream_t>(hip_stream);
  return TNA_OK;
}

tna_status tna_synchronize(tna_ctx c) {
  if (!c) {
    set_error("null context");
    return TNA_ERR_ARG;
  }
  TNA_HIP(hipStreamSynchronize(c->stream));
  return TNA_OK;
}

tna_status tna_set_timing(tna_ctx c, int enable, const char *prefix) {
  if (!c) {
    set_error("null context");
    return TNA_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_tm.mu);
  c->timing = enable;
  g_tm.on = enable != 0;
  g_tm.prefix = prefix ? prefix : "";
  return TNA_OK;
}

tna_status tna_kernel_stats(tna_ctx c, char *out, size_t cap, int reset) {
  if (!c || !out || cap == 0) {
    set_error("kernel_stats: null argument");
    return TNA_ERR_ARG;
  }
  TNA_HIP(hipStreamSynchronize(c->stream));
  std::lock_guard<std::mutex> lk(g_tm.mu);
  drain_pending();
  std::string js = "[";
  bool first = true;
  for (auto &kv : g_tm.stats) {
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s{\"name\":\"%s\",\"count\":%ld,\"ms\":%.6f,\"flops\":%.6e,\"bytes\":%.6e}",
                  first ? "" : ",", kv.first.c_str(), kv.second.count, kv.second.ms, kv.second.flops,
                  kv.second.bytes);
    js += buf;
    first = false;
  }
  js += "]";
  if (reset) g_tm.stats.clear();
  if (js.size() + 1 > cap) {
    set_error("kernel_stats: buffer too small");
    return TNA_ERR_ARG;
  }
  std::memcpy(out, js.c_str(), js.size() + 1);
  return TNA_OK;
}

tna_status tna_mpo_build(int model, int N, const double *p, double *W, int *D_out) {
  if (N < 2 || !p || !W) {
    set_error("mpo: need N >= 2 and non-null params/W");
    return TNA_ERR_ARG;
  }
  const int D = model == 0 ? 5 : model == 1 ? 8 : model == 2 ? 3 : -1;
  if (D < 0) {
    set_error("mpo: unknown model");
    return TNA_ERR_ARG;
  }
  const size_t sz = (size_t)D * D * 4;
  std::vector<double> w(sz, 0.0);
  // local operators [s_out][s_in], s = 0 up, 1 down
  const double I2[4] = {1, 0, 0, 1}, Sp[4] = {0, 1, 0, 0}, Sm[4] = {0, 0, 1, 0}, Sz[4] = {0.5, 0, 0, -0.5};
  const double X2[4] = {0, 1, 1, 0}, Z2[4] = {1, 0, 0, -1};
  auto set = [&](int l, int r, const double *op, double f) {
    for (int q = 0; q < 4; ++q) w[((size_t)l * D + r) * 4 + q] += f * op[q];
  };
  if (model == 0) {  // XXZ: last row opens a term, first column closes it
    const double J = p[0], Dz = p[1], hz = p[2];
    set(0, 0, I2, 1.0); set(4, 4, I2, 1.0);
    set(4, 1, Sp, 0.5 * J); set(1, 0, Sm, 1.0);
    set(4, 2, Sm, 0.5 * J); set(2, 0, Sp, 1.0);
    set(4, 3, Sz, J * Dz);  set(3, 0, Sz, 1.0);
    if (hz != 0.0) set(4, 0, Sz, -hz);
  } else if (model == 1) {  // J1-J2: channels 4..6 carry an identity for the next-nearest term
    const double J1 = p[0], J2 = p[1];
    set(0, 0, I2, 1.0); set(7, 7, I2, 1.0);
    set(7, 1, Sp, 0.5 * J1); set(1, 0, Sm, 1.0);
    set(7, 2, Sm, 0.5 * J1); set(2, 0, Sp, 1.0);
    set(7, 3, Sz, J1);       set(3, 0, Sz, 1.0);
    set(7, 4, Sp, 0.5 * J2); set(4, 1, I2, 1.0);
    set(7, 5, Sm, 0.5 * J2); set(5, 2, I2, 1.0);
    set(7, 6, Sz, J2);       set(6, 3, I2, 1.0);
  } else {  // transverse-field Ising (Pauli)
    const double J = p[0], h = p[1];
    set(0, 0, I2, 1.0); set(2, 2, I2, 1.0);
    set(2, 1, Z2, -J); set(1, 0, Z2, 1.0);
    set(2, 0, X2, -h);
  }
  for (int i = 0; i < N; ++i) std::memcpy(W + (size_t)i * sz, w.data(), sz * sizeof(double));
  if (D_out) *D_out = D;
  return TNA_OK;
}

// Scratch of one call: with a caller workspace set, each buffer becomes a view into it
// (256-byte aligned, in list order); otherwise the context's own buffers grow as needed.
typedef std::vector<std::pair<DevBuf *, size_t>> ScratchList;
static size_t scratch_bytes(const ScratchList &l) {
  size_t off = 0;
  for (auto &e : l) off = ((off + 255) & ~(size_t)255) + e.second;
  return off;
}
static tna_status bind_scratch(tna_ctx c, const ScratchList &l) {
  if (c->ws) {
    const size_t need = scratch_bytes(l);
    if (need > c->ws_bytes) {
      set_error("workspace too small: this call needs " + std::to_string(need) + " bytes");
      return TNA_ERR_NOMEM;
    }
    size_t off = 0;
    for (auto &e : l) {
      off = (off + 255) & ~(size_t)255;
      e.first->release();
      e.first->ptr = static_cast<char *>(c->ws) + off;
      e.first->bytes = e.second;
      e.first->borrowed = true;
      off += e.second;
    }
    return TNA_OK;
  }
  for (auto &e : l) {
    if (e.first->borrowed) e.first->release();
    TNA_TRY(e.first->ensure(e.second));
  }
  return TNA_OK;
}

static ScratchList heff_scratch(tna_ctx c, int chi_l, int chi_r, int d, int D, int prec) {
  const int64_t nx = (int64_t)D * d * d * chi_l * chi_r;
  const size_t el = prec == TNA_HEFF_F64 ? sizeof(double) : sizeof(float);
  ScratchList l{{&c->x, el * nx}, {&c->z, el * nx}, {&c->m12, sizeof(double) * 32 * 32}};
  if (prec != TNA_HEFF_F64) {
    l.push_back({&c->lf, sizeof(float) * (size_t)chi_l * D * chi_l});
    l.push_back({&c->rf, sizeof(float) * (size_t)chi_r * D * chi_r});
  }
  return l;
}

static tna_status svd_scratch(tna_ctx c, int batch, int m, int n, int dtype, ScratchList *out, SvdMat *proto) {
  TNA_TRY(svd_plan_mat(m, n, dtype, batch, proto));
  const size_t nd = svd_work_doubles(*proto), ni = svd_work_ints(*proto);
  *out = ScratchList{{&c->svd.work_d, sizeof(double) * nd * batch},
                     {&c->svd.work_i, sizeof(int) * ni * batch},
                     {&c->spec, sizeof(double) * 32 * batch},
                     {&c->svd.desc, sizeof(SvdMat) * batch}};
  return TNA_OK;
}


tna_status tna_heff_apply(tna_ctx c, int chi_l, int chi_r, int d, int D, const double *L, const double *W1,
                          const double *W2, const double *R, const double *theta, double *out, int prec) {
  TNA_TRY(heff_check_args(c, chi_l, chi_r, d, D, L, W1, W2, R, theta, out, prec));
  hipStream_t s = c->stream;
  TNA_TRY(bind_scratch(c, heff_scratch(c, chi_l, chi_r, d, D, prec)));
  TNA_TRY(build_mix_matrix(0, d, D, W1, W2, c->m12.as<double>(), s));
  HeffOp op{chi_l, chi_r, d, D, L, R, c->m12.as<double>(), c->x.ptr, c->z.ptr, prec};
  if (prec != TNA_HEFF_F64) {
    const int64_t nl = (int64_t)chi_l * D * chi_l, nr = (int64_t)chi_r * D * chi_r;
    TNA_TRY(convert_f64_f32(L, c->lf.as<float>(), nl, s));
    TNA_TRY(convert_f64_f32(R, c->rf.as<float>(), nr, s));
    op.L = c->lf.ptr;
    op.R = c->rf.ptr;
  }
  return heff_device(op, theta, out, s);
}

static tna_status svd_common(tna_ctx c, int batch, int m, int n, int dtype, const void *A, int64_t strideA,
                             int chi_keep, double *S, int64_t strideS, void *U, int64_t strideU, void *Vt,
                             int64_t strideVt, double *spec, int *k_out, int *sweeps_out) {
  if (!c || !A || !S || !U || !Vt || !spec) {
    set_error("svd_truncate: null argument");
    return TNA_ERR_ARG;
  }
  if (dtype != TNA_F64 && dtype != TNA_F32) {
    set_error("svd_truncate: bad dtype");
    return TNA_ERR_ARG;
  }
  if (chi_keep < 1 || batch < 1) {
    set_error("svd_truncate: chi_keep and batch must be >= 1");
    return TNA_ERR_ARG;
  }
  SvdMat proto;
  ScratchList scr;
  TNA_TRY(svd_scratch(c, batch, m, n, dtype, &scr, &proto));
  TNA_TRY(bind_scratch(c, scr));
  const int k = std::min(chi_keep, proto.R);
  const size_t nd = svd_work_doubles(proto), ni = svd_work_ints(proto);
  const size_t el = dtype == TNA_F64 ? sizeof(double) : sizeof(float);
  std::vector<SvdMat> mats(batch, proto);
  for (int z = 0; z < batch; ++z) {
    SvdMat &a = mats[z];
    svd_bind_work(&a, c->svd.work_d.as<double>() + nd * z, c->svd.work_i.as<int>() + ni * z);
    a.A = static_cast<const char *>(A) + el * strideA * z;
    a.S = S + strideS * z;
    a.spec = c->spec.as<double>() + 32 * z;
    a.U = static_cast<char *>(U) + el * strideU * z;
    a.Vt = static_cast<char *>(Vt) + el * strideVt * z;
    a.k = k;
    a.out_type = dtype;
    a.scale_mode = 0;
    a.eps_target = 0.0;
  }
  hipStream_t s = c->stream;
  std::vector<int> sweeps;
  tna_status st = svd_group_run(mats, c->svd, 60, sweeps, s);
  if (st != TNA_OK && st != TNA_ERR_NOCONV) return st;
  TNA_TRY(svd_group_outputs(mats, c->svd, s));
  TNA_HIP(hipMemcpy2DAsync(spec, 6 * sizeof(double), c->spec.ptr, 32 * sizeof(double), 6 * sizeof(double), batch,
                           hipMemcpyDeviceToDevice, s));
  if (k_out) *k_out = k;
  if (sweeps_out) *sweeps_out = sweeps.empty() ? 0 : *std::max_element(sweeps.begin(), sweeps.end());
  return st;
}

tna_status tna_svd_truncate(tna_ctx c, int m, int n, int dtype, const void *A, int chi_keep, double *S, void *U,
                            void *Vt, double *spec, int *k_out, int *sweeps_out) {
  const int k = std::min(chi_keep, std::min(m, n));
  return svd_common(c, 1, m, n, dtype, A, (int64_t)m * n, chi_keep, S, std::min(m, n), U, (int64_t)m * k, Vt,
                    (int64_t)k * n, spec, k_out, sweeps_out);
}

tna_status tna_svd_truncate_batched(tna_ctx c, int batch, int m, int n, int dtype, const void *A, int64_t strideA,
                                    int chi_keep, double *S, int64_t strideS, void *U, int64_t strideU, void *Vt,
                                    int64_t strideVt, double *spec, int *sweeps_out) {
  return svd_common(c, batch, m, n, dtype, A, strideA, chi_keep, S, strideS, U, strideU, Vt, strideVt, spec,
                    nullptr, sweeps_out);
}

tna_status tna_workspace_size(tna_ctx c, const char *op, const int64_t *dims, size_t *bytes) {
  if (!c || !op || !dims || !bytes) {
    set_error("workspace_size: null argument");
    return TNA_ERR_ARG;
  }
  if (std::strcmp(op, "heff_apply") == 0) {
    *bytes = scratch_bytes(heff_scratch(c, (int)dims[0], (int)dims[1], (int)dims[2], (int)dims[3], (int)dims[4]));
    return TNA_OK;
  }
  if (std::strcmp(op, "svd_truncate") == 0) {
    ScratchList l;
    SvdMat proto;
    TNA_TRY(svd_scratch(c, dims[3] > 0 ? (int)dims[3] : 1, (int)dims[0], (int)dims[1], (int)dims[2], &l, &proto));
    *bytes = scratch_bytes(l);
    return TNA_OK;
  }
  set_error(std::string("workspace_size: unknown op ") + op);
  return TNA_ERR_ARG;
}

tna_status tna_set_workspace(tna_ctx c, void *dev_ptr, size_t bytes) {
  if (!c) {
    set_error("set_workspace: null context");
    return TNA_ERR_ARG;
  }
  TNA_HIP(hipStreamSynchronize(c->stream));  // calls in flight may still use the previous scratch
  for (DevBuf *b : {&c->x, &c->z, &c->lf, &c->rf, &c->m12, &c->spec, &c->svd.work_d, &c->svd.work_i, &c->svd.desc})
    if (b->borrowed) b->release();
  c->ws = (dev_ptr && bytes) ? dev_ptr : nullptr;
  c->ws_bytes = c->ws ? bytes : 0;
  return TNA_OK;
}

tna_status tna_pid_chi_update(const tna_pid_params *p, tna_pid_state *st, double s_raw, int *chi_next,
                              double *terms) {
  return pid_update(p, st, s_raw, chi_next, terms);
}

tna_status tna_entropy_chi_update(const tna_pid_params *p, double gamma, tna_pid_state *st, double s_raw,
                                  int *chi_next) {
  return entropy_update(p, gamma, st, s_raw, chi_next, nullptr);
}

}  // extern "C"
