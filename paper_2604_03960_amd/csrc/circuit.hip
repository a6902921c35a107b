// Circuit simulation with adaptive bond dimensions (Sec. 8 of the paper, "circuit-level bond
// dimension maps"; the TEBD scheme of Sec. 2).  An MPS of N qubits starts in |0...0>.  A layer applies
// real two-qubit gates to the disjoint pairs (b, b+1) of one parity; the gates of a layer are
// independent, so every stage runs as one grouped launch over all of them:
//   C = B_b B_{b+1}                 grouped GEMM (MFMA)
//   C' = G C, Theta = lam_{b-1} C'  gate_layer_kernel (4 x 4 mixing on the physical pair, row scaling)
//   Theta = X S Y^T                 one group of Jacobi SVDs of different shapes (full spectrum)
//   entropy -> EMA + PID            host, per bond (the DMRG controller)
//   B_{b+1} <- Y_k^T                written by the SVD output pass
//   B_b <- C' Y_k / |S_k|           grouped GEMM (NT) then gate_finish_kernel (scaling, new lam_b)
// The MPS stays right-canonical with the Schmidt values of every bond (Vidal's form in the variant
// that never divides by a Schmidt value).  Each layer's bond dimensions are one row of the map.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "internal.h"

using namespace tna;

namespace {

constexpr int NT = 256;
constexpr int SPEC = 32;  // doubles per spectrum record

struct GateProb {
  int cl, cr;          // left and right bond dimensions of the pair; the two-site matrix is (2 cl) x (2 cr)
  const double *C;     // B_b B_{b+1}
  double *Cp, *Th;     // G C, and lam_{b-1}-scaled G C
  const double *G;     // 16 doubles, G[2s+t][2s'+t']
  const double *lam;   // cl Schmidt values of bond b-1, or null (left edge: 1)
};

// grid (element blocks, gates): thread e handles the four physical entries of (a, c) = e
__global__ __launch_bounds__(NT) void gate_layer_kernel(const GateProb *probs) {
  const GateProb &p = probs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)p.cl * p.cr) return;
  const int a = (int)(e / p.cr), c = (int)(e - (int64_t)a * p.cr);
  const int64_t n = 2 * (int64_t)p.cr;  // row length of the two-site matrix
  const int64_t base = (int64_t)a * 2 * n + c;
  // (s, t) sits at row 2a + s, column t cr + c
  double x[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) x[q] = p.C[base + (q >> 1) * n + (q & 1) * p.cr];
  const double la = p.lam ? p.lam[a] : 1.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = fma(p.G[4 * r + q], x[q], acc);
    const int64_t o = base + (r >> 1) * n + (r & 1) * p.cr;
    p.Cp[o] = acc;
    p.Th[o] = la * acc;
  }
}

struct FinishProb {
  int64_t nb;          // elements of the new B_b
  int k;
  double *Bb;          // C' Y_k, scaled here by 1 / |S_k|
  double *lam;         // k new Schmidt values S_j / |S_k|
  const double *S;     // sorted spectrum
  const double *spec;  // spec[4] = |S_k|
};

__global__ __launch_bounds__(NT) void gate_finish_kernel(const FinishProb *probs) {
  const FinishProb &p = probs[blockIdx.y];
  const double inv = 1.0 / p.spec[4];
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < p.nb; e += (int64_t)gridDim.x * NT) p.Bb[e] *= inv;
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < p.k; j += NT) p.lam[j] = p.S[j] * inv;
}

int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

struct tna_circuit_s {
  tna_ctx ctx = nullptr;
  int N = 0;
  tna_pid_params pid{};
  tna_circuit_opts opts{};
  std::vector<int> chi;               // N-1 bond dimensions
  std::vector<tna_pid_state> st;      // N-1 controllers
  std::vector<DevBuf> B, Bn, lam;     // site tensors, the layer's new ones, Schmidt values per bond
  DevBuf C, Cp, Th, Uw, S, spec, gates, desc;
  DevBuf svd_wd, svd_wi;
  SvdGroup svd;
  char *stage = nullptr;              // pinned upload staging
  size_t stage_cap = 0;
  double *h_spec = nullptr;           // pinned spectrum read-back
  hipStream_t own = nullptr;
  int layers = 0;
  long gates_done = 0;
  int CL(int i) const { return i == 0 ? 1 : chi[i - 1]; }
  int CR(int i) const { return i == N - 1 ? 1 : chi[i]; }
};

namespace {

// host values -> device (offset `off` of the pinned staging, same offset of the device buffer), async
template <class T>
tna_status upload(tna_circuit c, DevBuf &dst, size_t &off, const std::vector<T> &v, const T **dev, hipStream_t s) {
  const size_t bytes = sizeof(T) * v.size(), need = (bytes + 255) & ~(size_t)255;
  if (off + need > c->stage_cap) {
    set_error("circuit: upload staging exhausted");
    return TNA_ERR_NOMEM;
  }
  std::memcpy(c->stage + off, v.data(), bytes);
  TNA_TRY(dst.bytes >= off + need ? TNA_OK : TNA_ERR_NOMEM);
  char *d = static_cast<char *>(dst.ptr) + off;
  if (bytes) TNA_HIP(hipMemcpyAsync(d, c->stage + off, bytes, hipMemcpyHostToDevice, s));
  *dev = reinterpret_cast<const T *>(d);
  off += need;
  return TNA_OK;
}

// One group of gates (bonds bs, gates G, 16 doubles each); records into log (may be null).
tna_status run_group(tna_circuit c, const std::vector<int> &bs, const double *G, tna_gate_log *log) {
  hipStream_t s = c->ctx->stream ? c->ctx->stream : c->own;
  const int ng = (int)bs.size();
  if (ng == 0) return TNA_OK;
  std::vector<int> m(ng), n(ng), cl(ng), cm(ng), cr(ng), R(ng);
  std::vector<size_t> off2(ng + 1, 0), offu(ng + 1, 0);
  for (int q = 0; q < ng; ++q) {
    const int b = bs[q];
    cl[q] = c->CL(b);
    cm[q] = c->chi[b];
    cr[q] = c->CR(b + 1);
    m[q] = 2 * cl[q];
    n[q] = 2 * cr[q];
    R[q] = std::min(m[q], n[q]);
    off2[q + 1] = off2[q] + (size_t)m[q] * n[q];
    offu[q + 1] = offu[q] + (size_t)m[q] * R[q];
  }
  TNA_TRY(c->C.ensure(sizeof(double) * off2[ng]));
  TNA_TRY(c->Cp.ensure(sizeof(double) * off2[ng]));
  TNA_TRY(c->Th.ensure(sizeof(double) * off2[ng]));
  TNA_TRY(c->Uw.ensure(sizeof(double) * offu[ng]));
  TNA_TRY(c->spec.ensure(sizeof(double) * SPEC * ng));
  TNA_TRY(c->gates.ensure(sizeof(double) * 16 * ng));
  TNA_TRY(c->desc.ensure(c->stage_cap));
  double *Cd = c->C.as<double>(), *Cpd = c->Cp.as<double>(), *Thd = c->Th.as<double>();
  TNA_HIP(hipMemcpyAsync(c->gates.ptr, G, sizeof(double) * 16 * ng, hipMemcpyHostToDevice, s));
  size_t so = 0;
  // ---- C = B_b B_{b+1}
  {
    std::vector<GemmProb> pr;
    for (int q = 0; q < ng; ++q) {
      const int b = bs[q];
      pr.push_back(GemmProb{m[q], n[q], cm[q], cm[q], n[q], n[q], c->B[b].ptr, c->B[b + 1].ptr, Cd + off2[q], nullptr,
                            nullptr, nullptr, 0, 0, 0, 0});
    }
    GemmGroup g{0, 0, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
    const int total = gemm_group_tiles(pr, 64, &g.pairs);
    const GemmProb *dp = nullptr;
    TNA_TRY(upload(c, c->desc, so, pr, &dp, s));
    TNA_TRY(gemm_grouped(g, dp, ng, total, s));
  }
  // ---- C' = G C, Theta = lam_{b-1} C'
  {
    std::vector<GateProb> gp;
    int64_t maxe = 1;
    for (int q = 0; q < ng; ++q) {
      const int b = bs[q];
      gp.push_back(GateProb{cl[q], cr[q], Cd + off2[q], Cpd + off2[q], Thd + off2[q], c->gates.as<double>() + 16 * q,
                            b == 0 ? nullptr : c->lam[b - 1].as<double>()});
      maxe = std::max<int64_t>(maxe, (int64_t)cl[q] * cr[q]);
    }
    const GateProb *dg = nullptr;
    TNA_TRY(upload(c, c->desc, so, gp, &dg, s));
    hipLaunchKernelGGL(gate_layer_kernel, dim3((unsigned)ceil_div64(maxe, NT), ng), dim3(NT), 0, s, dg);
    TNA_LAUNCHED("circuit.gate");
  }
  // ---- SVDs of every Theta (one group), spectra read back for the controllers
  std::vector<SvdMat> mats(ng);
  size_t nd = 0, ni = 0, ns = 0;
  for (int q = 0; q < ng; ++q) {
    // Vt becomes B_{b+1} (orthonormal rows needed): from the rotations when the shape allows; U is unused
    TNA_TRY(svd_plan_mat(m[q], n[q], TNA_F64, ng, &mats[q], 2));
    mats[q].rows_scaled = mats[q].trans;
    nd += svd_work_doubles(mats[q]);
    ni += svd_work_ints(mats[q]);
    ns += mats[q].R;
  }
  TNA_TRY(c->svd_wd.ensure(sizeof(double) * nd));
  TNA_TRY(c->svd_wi.ensure(sizeof(int) * ni));
  TNA_TRY(c->S.ensure(sizeof(double) * ns));
  std::vector<double *> Sq(ng);
  {
    double *dw = c->svd_wd.as<double>(), *sp = c->S.as<double>();
    int *iw = c->svd_wi.as<int>();
    for (int q = 0; q < ng; ++q) {
      SvdMat &a = mats[q];
      svd_bind_work(&a, dw, iw);
      dw += svd_work_doubles(a);
      iw += svd_work_ints(a);
      a.A = Thd + off2[q];
      a.S = sp;
      Sq[q] = sp;
      sp += a.R;
      a.spec = c->spec.as<double>() + SPEC * q;
      a.eps_target = 1e-8;
      a.thr = 0.0;
      a.out_type = TNA_F64;
    }
  }
  std::vector<int> sweeps;
  const int max_sw = c->opts.svd_max_sweeps > 0 ? c->opts.svd_max_sweeps : 60;
  tna_status worst = svd_group_run(mats, c->svd, max_sw, sweeps, s);
  if (worst != TNA_OK && worst != TNA_ERR_NOCONV) return worst;
  TNA_HIP(hipMemcpyAsync(c->h_spec, c->spec.ptr, sizeof(double) * SPEC * ng, hipMemcpyDeviceToHost, s));
  TNA_HIP(hipStreamSynchronize(s));
  std::vector<int> k(ng), chi_next(ng);
  std::vector<double> terms(6 * ng);
  for (int q = 0; q < ng; ++q) {
    const double *h = c->h_spec + SPEC * q;
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) {
      set_error("circuit: non-finite two-site spectrum");
      return TNA_ERR_NONFINITE;
    }
    TNA_TRY(pid_update(&c->pid, &c->st[bs[q]], h[1], &chi_next[q], &terms[6 * q]));
    const int keep = c->opts.fixed_chi > 0 ? c->opts.fixed_chi : chi_next[q];
    k[q] = std::min(keep, R[q]);
  }
  // ---- B_{b+1} <- Y_k^T (the SVD's Vt output), U into scratch; spectrum sums for k
  for (int q = 0; q < ng; ++q) {
    const int b = bs[q];
    TNA_TRY(c->Bn[b + 1].ensure(sizeof(double) * (size_t)k[q] * n[q]));
    TNA_TRY(c->Bn[b].ensure(sizeof(double) * (size_t)m[q] * k[q]));
    TNA_TRY(c->lam[b].ensure(sizeof(double) * k[q]));
    SvdMat &a = mats[q];
    a.k = k[q];
    a.U = c->Uw.as<double>() + offu[q];
    a.Vt = c->Bn[b + 1].ptr;
    a.scale_mode = 0;
  }
  TNA_TRY(svd_group_outputs(mats, c->svd, s));
  // ---- B_b <- C' Y_k (NT product), then / |S_k|, and the new Schmidt values
  {
    std::vector<GemmProb> pr;
    for (int q = 0; q < ng; ++q) {
      const int b = bs[q];
      pr.push_back(GemmProb{m[q], k[q], n[q], n[q], n[q], k[q], Cpd + off2[q], c->Bn[b + 1].ptr, c->Bn[b].ptr,
                            nullptr, nullptr, nullptr, 0, 0, 0, 0});
    }
    GemmGroup g{0, 1, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
    const int total = gemm_group_tiles(pr, 64, &g.pairs);
    const GemmProb *dp = nullptr;
    TNA_TRY(upload(c, c->desc, so, pr, &dp, s));
    TNA_TRY(gemm_grouped(g, dp, ng, total, s));
    std::vector<FinishProb> fp;
    int64_t maxe = 1;
    for (int q = 0; q < ng; ++q) {
      const int b = bs[q];
      fp.push_back(FinishProb{(int64_t)m[q] * k[q], k[q], c->Bn[b].as<double>(), c->lam[b].as<double>(), Sq[q],
                              c->spec.as<double>() + SPEC * q});
      maxe = std::max<int64_t>(maxe, (int64_t)m[q] * k[q]);
    }
    const FinishProb *df = nullptr;
    TNA_TRY(upload(c, c->desc, so, fp, &df, s));
    hipLaunchKernelGGL(gate_finish_kernel, dim3((unsigned)std::min<int64_t>(ceil_div64(maxe, NT), 1024), ng), dim3(NT),
                       0, s, df);
    TNA_LAUNCHED("circuit.finish");
  }
  // ---- records: truncation sums of the outputs pass, the last kept value
  TNA_HIP(hipMemcpyAsync(c->h_spec, c->spec.ptr, sizeof(double) * SPEC * ng, hipMemcpyDeviceToHost, s));
  std::vector<double> slast(ng);
  for (int q = 0; q < ng; ++q)
    TNA_HIP(hipMemcpyAsync(&slast[q], Sq[q] + (k[q] - 1), sizeof(double), hipMemcpyDeviceToHost, s));
  TNA_HIP(hipStreamSynchronize(s));
  for (int q = 0; q < ng; ++q) {
    const int b = bs[q];
    std::swap(c->B[b], c->Bn[b]);
    std::swap(c->B[b + 1], c->Bn[b + 1]);
    c->chi[b] = k[q];
    if (!log) continue;
    const double *h = c->h_spec + SPEC * q;
    const double *tm = &terms[6 * q];
    tna_gate_log &r = log[q];
    std::memset(&r, 0, sizeof r);
    r.layer = c->layers; r.bond = b; r.m = m[q]; r.n = n[q]; r.k = k[q]; r.chi_ctrl = chi_next[q];
    r.svd_sweeps = mats[q].fused ? (int)std::fabs(h[7]) : sweeps[q];
    r.S = h[1]; r.S_ema = tm[4]; r.eps = h[2]; r.wdisc = h[3]; r.gap = h[5]; r.sigma0 = h[8];
    r.sigma_last = slast[q]; r.u = tm[3];
  }
  c->gates_done += ng;
  return worst;
}

}  // namespace

extern "C" {

tna_status tna_circuit_create(tna_ctx ctx, int N, const tna_pid_params *pid, const tna_circuit_opts *opts,
                              tna_circuit *out) {
  if (!ctx || !pid || !out || N < 2) {
    set_error("circuit_create: bad arguments");
    return TNA_ERR_ARG;
  }
  if (pid->chi_min < 1 || pid->chi_max < pid->chi_min) {
    set_error("circuit_create: need 1 <= chi_min <= chi_max");
    return TNA_ERR_ARG;
  }
  auto c = std::make_unique<tna_circuit_s>();
  c->ctx = ctx;
  c->N = N;
  c->pid = *pid;
  if (opts) c->opts = *opts;
  c->chi.assign(N - 1, 1);
  c->st.assign(N - 1, tna_pid_state{0, 0, 0, 0, pid->chi_min, 0});
  c->B.resize(N);
  c->Bn.resize(N);
  c->lam.resize(N);
  if (!ctx->stream) TNA_HIP(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));  // default priority
  hipStream_t s = ctx->stream ? ctx->stream : c->own;
  const double zero_state[2] = {1.0, 0.0}, one = 1.0;
  for (int i = 0; i < N; ++i) {  // |0>: B_i[0][0][0] = 1, B_i[0][1][0] = 0
    TNA_TRY(c->B[i].ensure(sizeof(double) * 2));
    TNA_HIP(hipMemcpyAsync(c->B[i].ptr, zero_state, sizeof(double) * 2, hipMemcpyHostToDevice, s));
  }
  for (int b = 0; b < N - 1; ++b) {
    TNA_TRY(c->lam[b].ensure(sizeof(double)));
    TNA_HIP(hipMemcpyAsync(c->lam[b].ptr, &one, sizeof(double), hipMemcpyHostToDevice, s));
  }
  c->stage_cap = (size_t)1 << 20;
  TNA_HIP(hipHostMalloc((void **)&c->stage, c->stage_cap, hipHostMallocDefault));
  TNA_HIP(hipHostMalloc((void **)&c->h_spec, sizeof(double) * SPEC * (N / 2 + 1), hipHostMallocDefault));
  TNA_HIP(hipStreamSynchronize(s));
  ctx->children += 1;
  *out = c.release();
  return TNA_OK;
}

tna_status tna_circuit_layer(tna_circuit c, int parity, const double *gates_host, tna_gate_log *log, int *chi_row) {
  if (!c || !gates_host || (parity != 0 && parity != 1)) {
    set_error("circuit_layer: bad handle, gates or parity");
    return TNA_ERR_ARG;
  }
  hipStream_t s = c->ctx->stream ? c->ctx->stream : c->own;
  TNA_HIP(hipStreamSynchronize(c->ctx->stream));  // work the caller queued on the context stream
  std::vector<int> bs;
  for (int b = parity; b <= c->N - 2; b += 2) bs.push_back(b);
  tna_status worst = TNA_OK;
  if (c->opts.one_at_a_time) {
    for (size_t q = 0; q < bs.size(); ++q) {
      const tna_status st = run_group(c, std::vector<int>{bs[q]}, gates_host + 16 * q, log ? log + q : nullptr);
      if (st != TNA_OK && st != TNA_ERR_NOCONV) return st;
      if (st == TNA_ERR_NOCONV) worst = st;
    }
  } else {
    worst = run_group(c, bs, gates_host, log);
    if (worst != TNA_OK && worst != TNA_ERR_NOCONV) return worst;
  }
  TNA_HIP(hipStreamSynchronize(s));
  c->layers += 1;
  if (chi_row) std::memcpy(chi_row, c->chi.data(), sizeof(int) * (c->N - 1));
  return worst;
}

tna_status tna_circuit_get_mps(tna_circuit c, double *B_host, size_t capacity, size_t *count, int *chi) {
  if (!c) {
    set_error("circuit_get_mps: null handle");
    return TNA_ERR_ARG;
  }
  size_t total = 0;
  for (int i = 0; i < c->N; ++i) total += (size_t)c->CL(i) * 2 * c->CR(i);
  if (count) *count = total;
  if (chi) std::memcpy(chi, c->chi.data(), sizeof(int) * (c->N - 1));
  if (!B_host) return TNA_OK;
  if (capacity < total) {
    set_error("circuit_get_mps: capacity too small");
    return TNA_ERR_ARG;
  }
  hipStream_t s = c->ctx->stream ? c->ctx->stream : c->own;
  TNA_HIP(hipStreamSynchronize(s));
  size_t off = 0;
  for (int i = 0; i < c->N; ++i) {
    const size_t nb = (size_t)c->CL(i) * 2 * c->CR(i);
    TNA_HIP(hipMemcpy(B_host + off, c->B[i].ptr, sizeof(double) * nb, hipMemcpyDeviceToHost));
    off += nb;
  }
  return TNA_OK;
}

void tna_circuit_destroy(tna_circuit c) {
  if (!c) return;
  hipStream_t s = c->ctx->stream ? c->ctx->stream : c->own;
  (void)hipStreamSynchronize(s);
  for (auto *v : {&c->B, &c->Bn, &c->lam})
    for (auto &b : *v) b.release();
  for (DevBuf *b : {&c->C, &c->Cp, &c->Th, &c->Uw, &c->S, &c->spec, &c->gates, &c->desc, &c->svd_wd, &c->svd_wi})
    b->release();
  c->svd.release();
  if (c->stage) (void)hipHostFree(c->stage);
  if (c->h_spec) (void)hipHostFree(c->h_spec);
  if (c->own) (void)hipStreamDestroy(c->own);
  c->ctx->children -= 1;
  delete c;
}

}  // extern "C"
