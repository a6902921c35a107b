// Many independent chains swept together (the batching form of the two-site
// DMRG step).  Each chain keeps its own MPS, environments and per-bond
// controllers (the tna_dmrg_s state); all chains advance one bond visit per
// step in lockstep, and every stage of a visit is one grouped launch over
// the chains:
//   theta formation  persistent grouped GEMM over a tile work list
//   Lanczos          grouped H_eff (GEMM, mixing, GEMM) + grouped CGS2; the
//                    launch sequence of one iteration is captured once per
//                    step as a HIP graph and replayed every iteration; chains
//                    drop out through device flags as they converge
//   SVD              one group of Jacobi SVDs of different shapes
//   controller       host, per chain
//   truncation/env   grouped outputs, grouped GEMM + mixing + GEMM
// Tile shapes of the grouped GEMMs are chosen by a measuring autotuner.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

using namespace tna;

namespace tna {
double tridiag_lowest_host(int n, const double *a, const double *b, double *y);
}

namespace {

// ------------------------------------------------------------------ autotuner
// Picks the GEMM tile (64 or 128) per (operation, log2 flops) bucket by
// timing both candidates on the live operands the first time a bucket is met.
struct Autotune {
  std::map<std::pair<int, int>, int> table;
  int measured = 0;
};
Autotune g_tune;

int flop_bucket(double f) { return f < 1.0 ? 0 : (int)std::floor(std::log2(f)); }

struct Staging {
  char *host = nullptr;
  size_t cap = 0;
  DevBuf dev;
};

tna_status stage_upload(Staging &st, const void *src, size_t bytes, hipStream_t s) {
  TNA_TRY(st.dev.ensure(bytes));
  if (st.cap < bytes) {
    TNA_HIP(hipStreamSynchronize(s));
    if (st.host) (void)hipHostFree(st.host);
    st.host = nullptr;
    TNA_HIP(hipHostMalloc((void **)&st.host, bytes * 2, hipHostMallocDefault));
    st.cap = bytes * 2;
  }
  TNA_HIP(hipStreamSynchronize(s));  // staging buffer may still feed an earlier copy
  std::memcpy(st.host, src, bytes);
  TNA_HIP(hipMemcpyAsync(st.dev.ptr, st.host, bytes, hipMemcpyHostToDevice, s));
  return TNA_OK;
}

void stage_release(Staging &st) {
  st.dev.release();
  if (st.host) (void)hipHostFree(st.host);
  st.host = nullptr;
  st.cap = 0;
}

// grouped GEMM with tile choice by the autotuner (kind identifies the operation)
tna_status tuned_gemm(int kind, GemmGroup g, std::vector<GemmProb> probs, Staging &st, hipStream_t s,
                      bool allow_measure) {
  if (probs.empty()) return TNA_OK;
  double fl = 0.0, by = 0.0;
  const int es = g.compute == G_F64 ? 8 : 4;
  for (auto &p : probs) {
    fl += 2.0 * p.M * (double)p.N * p.K;
    by += (double)es * ((double)p.M * p.K + (double)p.K * p.N + (double)p.M * p.N);
  }
  g.flops = fl;
  g.bytes = by;
  const auto key = std::make_pair(kind, flop_bucket(fl));
  auto it = g_tune.table.find(key);
  int tile = 64;
  if (it != g_tune.table.end()) tile = it->second;
  else if (allow_measure) {
    float best = 1e30f;
    for (int cand : {64, 128}) {
      std::vector<GemmProb> pr = probs;
      const int total = gemm_group_tiles(pr, cand);
      TNA_TRY(stage_upload(st, pr.data(), sizeof(GemmProb) * pr.size(), s));
      g.tile = cand;
      hipEvent_t a, b;
      TNA_HIP(hipEventCreate(&a));
      TNA_HIP(hipEventCreate(&b));
      TNA_TRY(gemm_grouped(g, st.dev.as<GemmProb>(), (int)pr.size(), total, s));  // warm
      TNA_HIP(hipEventRecord(a, s));
      TNA_TRY(gemm_grouped(g, st.dev.as<GemmProb>(), (int)pr.size(), total, s));
      TNA_HIP(hipEventRecord(b, s));
      TNA_HIP(hipEventSynchronize(b));
      float ms = 0.f;
      TNA_HIP(hipEventElapsedTime(&ms, a, b));
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      if (ms < best) {
        best = ms;
        tile = cand;
      }
    }
    g_tune.table[key] = tile;
    g_tune.measured += 1;
  }
  g.tile = tile;
  const int total = gemm_group_tiles(probs, tile);
  TNA_TRY(stage_upload(st, probs.data(), sizeof(GemmProb) * probs.size(), s));
  return gemm_grouped(g, st.dev.as<GemmProb>(), (int)probs.size(), total, s);
}

int parts_for(int64_t n) {
  int64_t g = (n + 4095) / 4096;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 512));
}

}  // namespace

struct tna_dmrg_batch_s {
  tna_ctx ctx = nullptr;
  hipStream_t stream = nullptr;
  int nch = 0, d = 2, D = 5, prec = 0, kmax = 100, restarts = 5;
  double tol = 1e-12, eps_target = 1e-8;
  std::vector<tna_dmrg> ch;
  std::vector<int> nsteps;
  std::vector<DevBuf> V, X, Z, Lf, Rf, T1, T2;
  DevBuf ints, dbl, lzst;  // per-chain j/active; alpha/beta records; Lanczos scratch arena
  Staging st_lz, st_g1, st_g2, st_mix, st_cvt, st_misc;
  SvdGroup svd;
  DevBuf svd_wd, svd_wi, spec, S;
  int *h_ints = nullptr;
  double *h_dbl = nullptr;
  int sweeps_done = 0;
  long graph_launches = 0;
};

static const size_t LZ_SLOT = 128;              // per-chain h1/h2/y/nrm2 slots
static const size_t LZ_PER = 3 * LZ_SLOT + 8;   // doubles per chain before the partials
static const size_t LZ_PART = 128 * 512;        // partial-sum slots per chain and array

extern "C" {

tna_status tna_dmrg_batch_create(tna_ctx c, int nch, const int *N, int d, int D, const double *const *W_host,
                                 const double *const *A_host, const int *const *chi_init,
                                 const tna_pid_params *pid, const tna_dmrg_opts *opts, tna_dmrg_batch *out) {
  if (!c || !out || nch < 1 || !N || !W_host || !A_host || !chi_init || !pid) {
    set_error("dmrg_batch_create: bad arguments");
    return TNA_ERR_ARG;
  }
  auto b = std::make_unique<tna_dmrg_batch_s>();
  b->ctx = c;
  b->nch = nch;
  b->d = d;
  b->D = D;
  tna_dmrg_opts o{};
  if (opts) o = *opts;
  b->prec = o.heff_prec;
  b->tol = o.lanczos_tol > 0 ? o.lanczos_tol : 1e-12;
  b->kmax = o.lanczos_kmax > 0 ? std::min(o.lanczos_kmax, 120) : 100;
  b->restarts = o.lanczos_restarts >= 0 ? o.lanczos_restarts : 5;
  b->eps_target = o.eps_target > 0 ? o.eps_target : 1e-8;
  if (b->prec != TNA_HEFF_F64 && b->prec != TNA_HEFF_F32) {
    set_error("dmrg_batch_create: heff_prec must be F64 or F32");
    return TNA_ERR_ARG;
  }
  TNA_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));  // default priority
  for (int i = 0; i < nch; ++i) {
    tna_dmrg dm = nullptr;
    TNA_TRY(tna_dmrg_create(c, N[i], d, D, W_host[i], A_host[i], chi_init[i], pid, opts, &dm));
    b->ch.push_back(dm);
    b->nsteps.push_back(2 * (N[i] - 1));
  }
  b->V.resize(nch);
  b->X.resize(nch);
  b->Z.resize(nch);
  b->Lf.resize(nch);
  b->Rf.resize(nch);
  b->T1.resize(nch);
  b->T2.resize(nch);
  TNA_TRY(b->ints.ensure(sizeof(int) * 2 * nch));
  TNA_TRY(b->dbl.ensure(sizeof(double) * 2 * nch));
  TNA_TRY(b->lzst.ensure(sizeof(double) * (LZ_PER + 2 * LZ_PART) * nch));
  TNA_HIP(hipHostMalloc((void **)&b->h_ints, sizeof(int) * 2 * nch, hipHostMallocDefault));
  TNA_HIP(hipHostMalloc((void **)&b->h_dbl, sizeof(double) * (24 * nch + 2 * nch + 16), hipHostMallocDefault));
  TNA_TRY(b->spec.ensure(sizeof(double) * 24 * nch));
  *out = b.release();
  return TNA_OK;
}

tna_status tna_dmrg_batch_sweep(tna_dmrg_batch bt, double *E_out, tna_visit_log *logs, const int64_t *log_offsets,
                                tna_batch_stats *stats) {
  if (!bt) {
    set_error("dmrg_batch_sweep: null handle");
    return TNA_ERR_ARG;
  }
  hipStream_t s = bt->stream;
  const int nch = bt->nch, d = bt->d, D = bt->D;
  const bool f32 = bt->prec == TNA_HEFF_F32;
  const int I1 = D * d, I2 = D * d * d;
  int maxsteps = 0;
  for (int v : bt->nsteps) maxsteps = std::max(maxsteps, v);
  std::vector<double> E(nch, 0.0);
  tna_status worst = TNA_OK;
  int *j_dev = bt->ints.as<int>(), *act_dev = j_dev + nch;
  double *rec_dev = bt->dbl.as<double>();
  double *lz = bt->lzst.as<double>();
  auto t_start = std::chrono::steady_clock::now();
  double ms_lanczos = 0, ms_svd = 0, ms_env = 0;
  long iters_total = 0;
  for (int t = 0; t < maxsteps; ++t) {
    auto t0 = std::chrono::steady_clock::now();
    // ---- chains taking part in this step and their bond
    std::vector<int> cs;
    for (int i = 0; i < nch; ++i)
      if (t < bt->nsteps[i]) cs.push_back(i);
    const int nc = (int)cs.size();
    if (nc == 0) break;
    struct Visit {
      int b, half, chl, chm, chr, m, n, kmax;
      int64_t nv;
    };
    std::vector<Visit> vs(nc);
    for (int q = 0; q < nc; ++q) {
      tna_dmrg dm = bt->ch[cs[q]];
      const int N = dm->N;
      Visit &v = vs[q];
      v.half = t < N - 1 ? 0 : 1;
      v.b = v.half == 0 ? t : (N - 2) - (t - (N - 1));
      v.chl = dm->CL(v.b);
      v.chm = dm->chi[v.b];
      v.chr = dm->CR(v.b + 1);
      v.m = v.chl * d;
      v.n = d * v.chr;
      v.nv = (int64_t)v.m * v.n;
      v.kmax = (int)std::min<int64_t>(bt->kmax, v.nv);
      const size_t el = f32 ? sizeof(float) : sizeof(double);
      TNA_TRY(bt->V[q].ensure(sizeof(double) * (size_t)(v.kmax + 2) * v.nv));
      TNA_TRY(bt->X[q].ensure(el * (size_t)D * d * d * v.chl * v.chr));
      TNA_TRY(bt->Z[q].ensure(el * (size_t)D * d * d * v.chl * v.chr));
      if (f32) {
        TNA_TRY(bt->Lf[q].ensure(sizeof(float) * (size_t)v.chl * D * v.chl));
        TNA_TRY(bt->Rf[q].ensure(sizeof(float) * (size_t)v.chr * D * v.chr));
      }
    }
    auto theta_of = [&](int q) { return bt->V[q].as<double>() + (int64_t)(vs[q].kmax + 1) * vs[q].nv; };
    // ---- theta = A_b A_{b+1}
    {
      GemmGroup g{0, 0, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
      std::vector<GemmProb> pr;
      for (int q = 0; q < nc; ++q) {
        tna_dmrg dm = bt->ch[cs[q]];
        const Visit &v = vs[q];
        pr.push_back(GemmProb{v.m, v.n, v.chm, v.chm, v.n, v.n, dm->A[v.b].ptr, dm->A[v.b + 1].ptr, theta_of(q),
                              nullptr, nullptr, nullptr, 0, 0, 0, 0});
      }
      TNA_TRY(tuned_gemm(0, g, pr, bt->st_misc, s, true));
    }
    if (f32) {
      std::vector<CvtProb> cv;
      for (int q = 0; q < nc; ++q) {
        tna_dmrg dm = bt->ch[cs[q]];
        const Visit &v = vs[q];
        cv.push_back(CvtProb{dm->Le[v.b].as<double>(), bt->Lf[q].as<float>(), (int64_t)v.chl * D * v.chl});
        cv.push_back(CvtProb{dm->Re[v.b + 1].as<double>(), bt->Rf[q].as<float>(), (int64_t)v.chr * D * v.chr});
      }
      TNA_TRY(stage_upload(bt->st_cvt, cv.data(), sizeof(CvtProb) * cv.size(), s));
      TNA_TRY(convert_grouped(bt->st_cvt.dev.as<CvtProb>(), (int)cv.size(), s));
    }
    // ---- Lanczos descriptors
    std::vector<LzProb> lp(nc);
    int maxG = 1, maxk = 1;
    for (int q = 0; q < nc; ++q) {
      const Visit &v = vs[q];
      double *base = lz + (LZ_PER + 2 * LZ_PART) * q;
      LzProb &p = lp[q];
      p.n = v.nv;
      p.G = parts_for(v.nv);
      p.nkeep = 0;
      p.V = bt->V[q].as<double>();
      p.theta = theta_of(q);
      p.j = j_dev + q;
      p.active = act_dev + q;
      p.h1 = base;
      p.h2 = base + LZ_SLOT;
      p.y = base + 2 * LZ_SLOT;
      p.nrm2 = base + 3 * LZ_SLOT;
      p.part1 = base + LZ_PER;
      p.part2 = base + LZ_PER + LZ_PART;
      p.rec = rec_dev + 2 * q;
      maxG = std::max(maxG, p.G);
      maxk = std::max(maxk, v.kmax);
    }
    // H_eff group descriptors (operand offsets follow each chain's j on the device)
    std::vector<GemmProb> s1, s4;
    std::vector<MixProb> mx;
    int64_t max_mix = 1;
    for (int q = 0; q < nc; ++q) {
      tna_dmrg dm = bt->ch[cs[q]];
      const Visit &v = vs[q];
      const void *L = f32 ? (const void *)bt->Lf[q].ptr : dm->Le[v.b].ptr;
      const void *R = f32 ? (const void *)bt->Rf[q].ptr : dm->Re[v.b + 1].ptr;
      s1.push_back(GemmProb{v.chl * D, d * d * v.chr, v.chl, v.chl, d * d * v.chr, d * d * v.chr, L, lp[q].V,
                            bt->X[q].ptr, j_dev + q, nullptr, act_dev + q, v.nv, 0, 0, 0});
      mx.push_back(MixProb{v.chl, v.chr, bt->X[q].ptr, bt->Z[q].ptr, (int64_t)D * d * d * v.chr, 1,
                           (int64_t)d * d * D * v.chr, 1, d * d * v.chr, v.chr, d * D * v.chr, v.chr,
                           dm->M12.as<double>() + (size_t)I2 * I2 * v.b, act_dev + q});
      // Z channels: j = (s*d + t)*D + w''  -> offset (s*d + t)*D*chr + w''*chr; J1 = d*d, J2 = D
      mx.back().och1 = D * v.chr;
      mx.back().och2 = v.chr;
      s4.push_back(GemmProb{v.chl * d * d, v.chr, D * v.chr, D * v.chr, D * v.chr, v.chr, bt->Z[q].ptr, R,
                            lp[q].V + v.nv, nullptr, j_dev + q, act_dev + q, 0, v.nv, 0, 0});
      max_mix = std::max<int64_t>(max_mix, (int64_t)v.chl * v.chr);
    }
    // input channels of the two-site mixing: i = w*d^2 + (s'*d + t') -> w*d*d*chr + (s'*d+t')*chr
    for (auto &m : mx) {
      m.ich1 = d * d * m.n1;
      m.ich2 = m.n1;
    }
    const int tc = f32 ? G_F32 : G_F64;
    GemmGroup g1{0, 0, tc, G_F64, tc, tc, 64, 1.0, 0.0, 0.0, 0.0};
    GemmGroup g4{0, 1, tc, tc, G_F64, tc, 64, 1.0, 0.0, 0.0, 0.0};
    // ---- start: j = 0, every chain of the step active, V_0 = theta/|theta|
    for (int q = 0; q < nc; ++q) {
      bt->h_ints[q] = 0;
      bt->h_ints[nch + q] = 1;
    }
    TNA_HIP(hipMemcpyAsync(j_dev, bt->h_ints, sizeof(int) * 2 * nch, hipMemcpyHostToDevice, s));
    std::vector<int> h_act(nc, 1);
    TNA_TRY(stage_upload(bt->st_lz, lp.data(), sizeof(LzProb) * nc, s));
    const LzProb *dlp = bt->st_lz.dev.as<LzProb>();
    // tile choice for the two H_eff GEMMs (measured with j = 0 before capture)
    TNA_TRY(lz_start(dlp, nc, maxG, s));
    TNA_TRY(tuned_gemm(1, g1, s1, bt->st_g1, s, true));
    TNA_TRY(tuned_gemm(2, g4, s4, bt->st_g2, s, true));
    TNA_TRY(stage_upload(bt->st_mix, mx.data(), sizeof(MixProb) * nc, s));
    // capture one Lanczos iteration
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    {
      std::vector<GemmProb> p1 = s1, p4 = s4;
      double f1 = 0, f4 = 0;
      for (auto &p : s1) f1 += 2.0 * p.M * (double)p.N * p.K;
      for (auto &p : s4) f4 += 2.0 * p.M * (double)p.N * p.K;
      g1.tile = g_tune.table.count(std::make_pair(1, flop_bucket(f1))) ? g_tune.table[std::make_pair(1, flop_bucket(f1))] : 64;
      g4.tile = g_tune.table.count(std::make_pair(2, flop_bucket(f4))) ? g_tune.table[std::make_pair(2, flop_bucket(f4))] : 64;
      g1.flops = f1;
      g4.flops = f4;
      const int tot1 = gemm_group_tiles(p1, g1.tile), tot4 = gemm_group_tiles(p4, g4.tile);
      TNA_TRY(stage_upload(bt->st_g1, p1.data(), sizeof(GemmProb) * nc, s));
      TNA_TRY(stage_upload(bt->st_g2, p4.data(), sizeof(GemmProb) * nc, s));
      TNA_HIP(hipStreamSynchronize(s));
      TNA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      tna_status cs1 = gemm_grouped(g1, bt->st_g1.dev.as<GemmProb>(), nc, tot1, s);
      if (cs1 == TNA_OK) cs1 = mix_grouped(bt->st_mix.dev.as<MixProb>(), nc, max_mix, D, d * d, d * d, D, f32, s);
      if (cs1 == TNA_OK) cs1 = gemm_grouped(g4, bt->st_g2.dev.as<GemmProb>(), nc, tot4, s);
      if (cs1 == TNA_OK) cs1 = lz_iteration(dlp, nc, maxG, maxk, s);
      hipError_t ce = hipStreamEndCapture(s, &graph);
      if (cs1 != TNA_OK) return cs1;
      if (ce != hipSuccess) {
        set_error(std::string("graph capture: ") + hipGetErrorString(ce));
        return TNA_ERR_DEVICE;
      }
      TNA_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    }
    // ---- lockstep Lanczos
    std::vector<std::vector<double>> al(nc), be(nc), yv(nc);
    std::vector<int> conv(nc, 0), nkeep(nc, 0), iters(nc, 0), restart(nc, 0);
    std::vector<double> Ec(nc, 0.0);
    for (;;) {
      int live = 0;
      for (int q = 0; q < nc; ++q) live += h_act[q];
      if (live == 0) break;
      TNA_HIP(hipGraphLaunch(gexec, s));
      bt->graph_launches += 1;
      TNA_HIP(hipMemcpyAsync(bt->h_dbl, rec_dev, sizeof(double) * 2 * nc, hipMemcpyDeviceToHost, s));
      TNA_HIP(hipStreamSynchronize(s));
      bool act_changed = false;
      for (int q = 0; q < nc; ++q) {
        if (!h_act[q]) continue;
        const double a = bt->h_dbl[2 * q], b2 = bt->h_dbl[2 * q + 1];
        if (!std::isfinite(a) || !std::isfinite(b2)) {
          set_error("batch lanczos: non-finite coefficient");
          return TNA_ERR_NONFINITE;
        }
        al[q].push_back(a);
        be[q].push_back(std::sqrt(b2));
        iters[q] += 1;
        const int nn = (int)al[q].size();
        yv[q].assign(nn, 0.0);
        Ec[q] = tridiag_lowest_host(nn, al[q].data(), be[q].data(), yv[q].data());
        const double resid = std::fabs(be[q][nn - 1] * yv[q][nn - 1]);
        bool stop = false;
        if (resid <= bt->tol * std::max(1.0, std::fabs(Ec[q])) || be[q][nn - 1] < 1e-14) {
          conv[q] = 1;
          stop = true;
        } else if (nn >= vs[q].kmax) {
          stop = true;
        }
        if (stop) {
          nkeep[q] = nn;
          h_act[q] = 0;
          act_changed = true;
        }
      }
      if (!act_changed) continue;
      // chains that stopped at kmax unconverged restart from their Ritz vector
      std::vector<int> rs(nc, 0);
      bool any_restart = false;
      for (int q = 0; q < nc; ++q) {
        rs[q] = !h_act[q] && !conv[q] && nkeep[q] > 0 && restart[q] < bt->restarts;
        any_restart = any_restart || rs[q];
      }
      if (any_restart) {
        for (int q = 0; q < nc; ++q) {
          bt->h_ints[nch + q] = rs[q];  // only restarting chains take part in the Ritz step
          lp[q].nkeep = rs[q] ? nkeep[q] : 0;
          if (rs[q]) TNA_HIP(hipMemcpyAsync(lp[q].y, yv[q].data(), sizeof(double) * nkeep[q], hipMemcpyHostToDevice, s));
        }
        TNA_HIP(hipMemcpyAsync(act_dev, bt->h_ints + nch, sizeof(int) * nch, hipMemcpyHostToDevice, s));
        TNA_TRY(stage_upload(bt->st_lz, lp.data(), sizeof(LzProb) * nc, s));
        TNA_TRY(lz_ritz(dlp, nc, maxG, s));
        TNA_TRY(lz_start(dlp, nc, maxG, s));
        for (int q = 0; q < nc; ++q) {
          if (!rs[q]) continue;
          restart[q] += 1;
          al[q].clear();
          be[q].clear();
          nkeep[q] = 0;
          h_act[q] = 1;
          bt->h_ints[q] = 0;  // j = 0
          TNA_HIP(hipMemcpyAsync(j_dev + q, bt->h_ints + q, sizeof(int), hipMemcpyHostToDevice, s));
        }
      }
      for (int q = 0; q < nc; ++q) bt->h_ints[nch + q] = h_act[q];
      TNA_HIP(hipMemcpyAsync(act_dev, bt->h_ints + nch, sizeof(int) * nch, hipMemcpyHostToDevice, s));
      TNA_HIP(hipStreamSynchronize(s));
    }
    (void)hipGraphExecDestroy(gexec);
    (void)hipGraphDestroy(graph);
    // ---- Ritz vectors of every chain of the step
    for (int q = 0; q < nc; ++q) {
      lp[q].nkeep = nkeep[q];
      bt->h_ints[nch + q] = 1;
      iters_total += iters[q];
      if (!conv[q] && worst == TNA_OK) worst = TNA_ERR_NOCONV;
      TNA_HIP(hipMemcpyAsync(lp[q].y, yv[q].data(), sizeof(double) * nkeep[q], hipMemcpyHostToDevice, s));
    }
    TNA_HIP(hipMemcpyAsync(act_dev, bt->h_ints + nch, sizeof(int) * nch, hipMemcpyHostToDevice, s));
    TNA_TRY(stage_upload(bt->st_lz, lp.data(), sizeof(LzProb) * nc, s));
    TNA_TRY(lz_ritz(dlp, nc, maxG, s));
    auto t1 = std::chrono::steady_clock::now();
    // ---- SVD of every theta
    std::vector<SvdMat> mats(nc);
    size_t nd = 0, ni = 0, ns = 0;
    for (int q = 0; q < nc; ++q) {
      TNA_TRY(svd_plan_mat(vs[q].m, vs[q].n, TNA_F64, nc, &mats[q]));
      nd += svd_work_doubles(mats[q]);
      ni += svd_work_ints(mats[q]);
      ns += mats[q].R;
    }
    TNA_TRY(bt->svd_wd.ensure(sizeof(double) * nd));
    TNA_TRY(bt->svd_wi.ensure(sizeof(int) * ni));
    TNA_TRY(bt->S.ensure(sizeof(double) * ns));
    {
      double *dw = bt->svd_wd.as<double>(), *sp = bt->S.as<double>();
      int *iw = bt->svd_wi.as<int>();
      for (int q = 0; q < nc; ++q) {
        SvdMat &a = mats[q];
        svd_bind_work(&a, dw, iw);
        dw += svd_work_doubles(a);
        iw += svd_work_ints(a);
        a.A = lp[q].theta;
        a.S = sp;
        sp += a.R;
        a.spec = bt->spec.as<double>() + 24 * q;
        a.eps_target = bt->eps_target;
        a.out_type = TNA_F64;
      }
    }
    std::vector<int> sweeps;
    tna_status sst = svd_group_run(mats, bt->svd, 60, sweeps, s);
    if (sst != TNA_OK && sst != TNA_ERR_NOCONV) return sst;
    if (sst == TNA_ERR_NOCONV && worst == TNA_OK) worst = TNA_ERR_NOCONV;
    TNA_HIP(hipMemcpyAsync(bt->h_dbl, bt->spec.ptr, sizeof(double) * 24 * nc, hipMemcpyDeviceToHost, s));
    TNA_HIP(hipStreamSynchronize(s));
    std::vector<double> terms(6 * nc);
    std::vector<int> chi_next(nc), kk(nc);
    for (int q = 0; q < nc; ++q) {
      tna_dmrg dm = bt->ch[cs[q]];
      const double Sent = bt->h_dbl[24 * q + 1];
      TNA_TRY(pid_update(&dm->pid, &dm->st[vs[q].b], Sent, &chi_next[q], &terms[6 * q]));
      const int keep = dm->opts.fixed_chi > 0 ? dm->opts.fixed_chi : chi_next[q];
      kk[q] = std::min(keep, mats[q].R);
      SvdMat &a = mats[q];
      a.k = kk[q];
      TNA_TRY(dm->A[vs[q].b].ensure(sizeof(double) * (size_t)vs[q].m * kk[q]));
      TNA_TRY(dm->A[vs[q].b + 1].ensure(sizeof(double) * (size_t)kk[q] * vs[q].n));
      a.U = dm->A[vs[q].b].ptr;
      a.Vt = dm->A[vs[q].b + 1].ptr;
      a.scale_mode = vs[q].half == 0 ? 1 : 2;
    }
    TNA_TRY(svd_group_outputs(mats, bt->svd, s));
    auto t2 = std::chrono::steady_clock::now();
    // ---- environments: left grows for L->R chains, right for R->L chains
    {
      std::vector<GemmProb> l1, l3, r1, r3;
      std::vector<MixProb> lm, rm;
      int64_t maxl = 1, maxr = 1;
      for (int q = 0; q < nc; ++q) {
        tna_dmrg dm = bt->ch[cs[q]];
        const Visit &v = vs[q];
        const int k = kk[q];
        dm->chi[v.b] = k;
        if (v.half == 0) {
          const int chl = v.chl;
          TNA_TRY(bt->T1[q].ensure(sizeof(double) * (size_t)chl * D * d * k));
          TNA_TRY(bt->T2[q].ensure(sizeof(double) * (size_t)chl * D * d * k));
          TNA_TRY(dm->Le[v.b + 1].ensure(sizeof(double) * (size_t)k * D * k));
          l1.push_back(GemmProb{chl * D, d * k, chl, chl, d * k, d * k, dm->Le[v.b].ptr, dm->A[v.b].ptr, bt->T1[q].ptr,
                                nullptr, nullptr, nullptr, 0, 0, 0, 0});
          lm.push_back(MixProb{chl, k, bt->T1[q].ptr, bt->T2[q].ptr, (int64_t)D * d * k, 1, (int64_t)d * D * k, 1,
                               d * k, k, D * k, k, dm->Ml.as<double>() + (size_t)I1 * I1 * v.b, nullptr});
          l3.push_back(GemmProb{k, D * k, chl * d, k, D * k, D * k, dm->A[v.b].ptr, bt->T2[q].ptr,
                                dm->Le[v.b + 1].ptr, nullptr, nullptr, nullptr, 0, 0, 0, 0});
          maxl = std::max<int64_t>(maxl, (int64_t)chl * k);
        } else {
          const int chr = v.chr;
          TNA_TRY(bt->T1[q].ensure(sizeof(double) * (size_t)chr * D * k * d));
          TNA_TRY(bt->T2[q].ensure(sizeof(double) * (size_t)chr * D * k * d));
          TNA_TRY(dm->Re[v.b].ensure(sizeof(double) * (size_t)k * D * k));
          r1.push_back(GemmProb{chr * D, k * d, chr, chr, chr, k * d, dm->Re[v.b + 1].ptr, dm->A[v.b + 1].ptr,
                                bt->T1[q].ptr, nullptr, nullptr, nullptr, 0, 0, 0, 0});
          rm.push_back(MixProb{chr, k, bt->T1[q].ptr, bt->T2[q].ptr, (int64_t)D * k * d, d, (int64_t)D * k, 1, k * d,
                               1, chr * D * k, k, dm->Mr.as<double>() + (size_t)I1 * I1 * (v.b + 1), nullptr});
          r3.push_back(GemmProb{k, D * k, d * chr, d * chr, D * k, D * k, dm->A[v.b + 1].ptr, bt->T2[q].ptr,
                                dm->Re[v.b].ptr, nullptr, nullptr, nullptr, 0, 0, 0, 0});
          maxr = std::max<int64_t>(maxr, (int64_t)chr * k);
        }
      }
      GemmGroup nn{0, 0, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
      GemmGroup nt{0, 1, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
      GemmGroup tn{1, 0, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
      if (!l1.empty()) {
        TNA_TRY(tuned_gemm(3, nn, l1, bt->st_misc, s, true));
        TNA_TRY(stage_upload(bt->st_mix, lm.data(), sizeof(MixProb) * lm.size(), s));
        TNA_TRY(mix_grouped(bt->st_mix.dev.as<MixProb>(), (int)lm.size(), maxl, D, d, d, D, 0, s));
        TNA_TRY(tuned_gemm(4, tn, l3, bt->st_misc, s, true));
      }
      if (!r1.empty()) {
        TNA_TRY(tuned_gemm(5, nt, r1, bt->st_misc, s, true));
        TNA_TRY(stage_upload(bt->st_mix, rm.data(), sizeof(MixProb) * rm.size(), s));
        TNA_TRY(mix_grouped(bt->st_mix.dev.as<MixProb>(), (int)rm.size(), maxr, D, d, d, D, 0, s));
        TNA_TRY(tuned_gemm(6, nn, r3, bt->st_misc, s, true));
      }
    }
    // per-visit records (truncation sums of the outputs pass)
    TNA_HIP(hipMemcpyAsync(bt->h_dbl, bt->spec.ptr, sizeof(double) * 24 * nc, hipMemcpyDeviceToHost, s));
    TNA_HIP(hipStreamSynchronize(s));
    auto t3 = std::chrono::steady_clock::now();
    ms_lanczos += std::chrono::duration<double, std::milli>(t1 - t0).count();
    ms_svd += std::chrono::duration<double, std::milli>(t2 - t1).count();
    ms_env += std::chrono::duration<double, std::milli>(t3 - t2).count();
    for (int q = 0; q < nc; ++q) {
      const int cidx = cs[q];
      E[cidx] = Ec[q];
      if (logs && log_offsets) {
        tna_visit_log &r = logs[log_offsets[cidx] + t];
        const double *h = bt->h_dbl + 24 * q;
        const double *tm = &terms[6 * q];
        std::memset(&r, 0, sizeof r);
        r.sweep = bt->sweeps_done; r.dir = vs[q].half; r.bond = vs[q].b; r.m = vs[q].m; r.n = vs[q].n;
        r.k = kk[q]; r.chi_ctrl = chi_next[q]; r.lanczos_iters = iters[q]; r.svd_sweeps = sweeps[q];
        r.lanczos_ok = conv[q]; r.E = Ec[q]; r.S = h[1]; r.S_ema = tm[4]; r.eps = h[2]; r.wdisc = h[3];
        r.gap = h[5]; r.P = tm[0]; r.I = tm[1]; r.D = tm[2]; r.u = tm[3]; r.sigma0 = h[8];
        r.k_needed = (int)h[6];
      }
    }
  }
  for (tna_dmrg dm : bt->ch) dm->sweeps_done += 1;
  bt->sweeps_done += 1;
  if (E_out) std::memcpy(E_out, E.data(), sizeof(double) * nch);
  if (stats) {
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    stats->ms_lanczos = ms_lanczos;
    stats->ms_svd = ms_svd;
    stats->ms_env = ms_env;
    stats->lanczos_iters = iters_total;
    stats->graph_launches = bt->graph_launches;
    stats->autotune_entries = (int)g_tune.table.size();
    stats->steps = maxsteps;
  }
  return worst;
}

tna_status tna_dmrg_batch_get_state(tna_dmrg_batch bt, int chain, int *chi, tna_pid_state *pid) {
  if (!bt || chain < 0 || chain >= bt->nch) {
    set_error("dmrg_batch_get_state: bad chain");
    return TNA_ERR_ARG;
  }
  return tna_dmrg_get_state(bt->ch[chain], chi, pid);
}

void tna_dmrg_batch_destroy(tna_dmrg_batch bt) {
  if (!bt) return;
  (void)hipStreamSynchronize(bt->stream);
  for (tna_dmrg dm : bt->ch) tna_dmrg_destroy(dm);
  for (auto *vec : {&bt->V, &bt->X, &bt->Z, &bt->Lf, &bt->Rf, &bt->T1, &bt->T2})
    for (auto &b : *vec) b.release();
  for (DevBuf *b : {&bt->ints, &bt->dbl, &bt->lzst, &bt->svd_wd, &bt->svd_wi, &bt->spec, &bt->S}) b->release();
  for (Staging *st : {&bt->st_lz, &bt->st_g1, &bt->st_g2, &bt->st_mix, &bt->st_cvt, &bt->st_misc}) stage_release(*st);
  bt->svd.release();
  if (bt->h_ints) (void)hipHostFree(bt->h_ints);
  if (bt->h_dbl) (void)hipHostFree(bt->h_dbl);
  if (bt->stream) (void)hipStreamDestroy(bt->stream);
  delete bt;
}

tna_status tna_autotune_save(const char *path) {
  FILE *f = std::fopen(path, "w");
  if (!f) {
    set_error("autotune_save: cannot open file");
    return TNA_ERR_ARG;
  }
  for (auto &kv : g_tune.table) std::fprintf(f, "%d %d %d\n", kv.first.first, kv.first.second, kv.second);
  std::fclose(f);
  return TNA_OK;
}

tna_status tna_autotune_load(const char *path) {
  FILE *f = std::fopen(path, "r");
  if (!f) {
    set_error("autotune_load: cannot open file");
    return TNA_ERR_ARG;
  }
  int a, b, t;
  while (std::fscanf(f, "%d %d %d", &a, &b, &t) == 3)
    if (t == 64 || t == 128) g_tune.table[std::make_pair(a, b)] = t;
  std::fclose(f);
  return TNA_OK;
}

int tna_autotune_entries(void) { return (int)g_tune.table.size(); }

}  // extern "C"
