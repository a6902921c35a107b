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

#include <algorithm>
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


// ------------------------------------------------------------------ descriptor arena
// Everything a step uploads (descriptors, flags, small vectors) is copied into
// a fresh slice of a pinned host block and from there to the same offset of a
// device block.  Nothing is reused before the step's final synchronisation, so
// no host write can race a copy still in flight and every device pointer
// handed out stays valid for the whole step (a captured graph keeps using
// them); a full block is followed by a new one.
struct ArenaBlock {
  char *host = nullptr;
  void *dev = nullptr;
  size_t cap = 0;
};
struct Arena {
  std::vector<ArenaBlock> blocks;
  size_t cur = 0, off = 0;
};

void arena_begin(Arena &a) {
  a.cur = 0;
  a.off = 0;
}

// reserves `bytes` (256-byte aligned) in the current block, or in a new one
tna_status arena_reserve(Arena &a, size_t bytes, char **host, char **dev) {
  const size_t need = (bytes + 255) & ~(size_t)255;
  while (a.cur < a.blocks.size() && a.off + need > a.blocks[a.cur].cap) {
    ++a.cur;
    a.off = 0;
  }
  if (a.cur == a.blocks.size()) {
    ArenaBlock b;
    b.cap = std::max<size_t>((size_t)4 << 20, 2 * need);
    TNA_HIP(hipHostMalloc((void **)&b.host, b.cap, hipHostMallocDefault));
    if (hipMalloc(&b.dev, b.cap) != hipSuccess) {
      (void)hipHostFree(b.host);
      set_error("arena: device allocation failed");
      return TNA_ERR_NOMEM;
    }
    a.blocks.push_back(b);
    a.off = 0;
  }
  ArenaBlock &b = a.blocks[a.cur];
  *host = b.host + a.off;
  *dev = static_cast<char *>(b.dev) + a.off;
  a.off += need;
  return TNA_OK;
}

// host values -> the arena's device half (descriptors read by kernels)
template <class T>
tna_status arena_push(Arena &a, const T *src, size_t n, hipStream_t s, const T **dev_out) {
  const size_t bytes = sizeof(T) * n;
  char *h = nullptr, *d = nullptr;
  TNA_TRY(arena_reserve(a, bytes, &h, &d));
  if (bytes) std::memcpy(h, src, bytes);
  if (bytes) TNA_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
  *dev_out = reinterpret_cast<const T *>(d);
  return TNA_OK;
}

// host values -> a device location, uploaded in one transfer from the arena's pinned half (not
// reused before the step's final synchronisation)
template <class T>
tna_status put_dev(Arena &a, const T *src, size_t n, T *dst, hipStream_t s) {
  if (n == 0) return TNA_OK;
  const size_t bytes = sizeof(T) * n;
  char *h = nullptr, *d = nullptr;
  TNA_TRY(arena_reserve(a, bytes, &h, &d));
  std::memcpy(h, src, bytes);
  TNA_HIP(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s));
  return TNA_OK;
}

void arena_release(Arena &a) {
  for (auto &b : a.blocks) {
    if (b.dev) (void)hipFree(b.dev);
    if (b.host) (void)hipHostFree(b.host);
  }
  a.blocks.clear();
  a.cur = a.off = 0;
}

double group_flops(const std::vector<GemmProb> &probs) {
  double f = 0.0;
  for (auto &p : probs) f += 2.0 * p.M * (double)p.N * p.K;
  return f;
}
// algorithmic bytes of a group (each operand read once, C written once), es bytes per element
double group_bytes(const std::vector<GemmProb> &probs, int es) {
  double by = 0.0;
  for (auto &p : probs) by += (double)es * ((double)p.M * p.K + (double)p.K * p.N + (double)p.M * p.N);
  return by;
}

// grouped GEMM with its tile picked by the autotuner (kind names the operation)
tna_status tuned_gemm(int kind, GemmGroup g, std::vector<GemmProb> probs, Arena &ar, hipStream_t s, bool measure,
                      int *tile_out = nullptr) {
  if (probs.empty()) return TNA_OK;
  g.flops = group_flops(probs);
  g.bytes = group_bytes(probs, g.compute == G_F64 ? 8 : 4);
  const auto key = std::make_pair(kind, flop_bucket(g.flops));
  auto it = g_tune.table.find(key);
  int tile = 64;
  if (it != g_tune.table.end()) tile = it->second;
  else if (measure) {
    float best = 1e30f;
    for (int cand : {64, 128}) {
      std::vector<GemmProb> pr = probs;
      const int total = gemm_group_tiles(pr, cand, &g.pairs);
      const GemmProb *d = nullptr;
      TNA_TRY(arena_push(ar, pr.data(), pr.size(), s, &d));
      g.tile = cand;
      hipEvent_t a, b;
      TNA_HIP(hipEventCreate(&a));
      TNA_HIP(hipEventCreate(&b));
      TNA_TRY(gemm_grouped(g, d, (int)pr.size(), total, s));  // warm
      TNA_HIP(hipEventRecord(a, s));
      TNA_TRY(gemm_grouped(g, d, (int)pr.size(), total, s));
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
  if (tile_out) *tile_out = tile;
  g.tile = tile;
  const int total = gemm_group_tiles(probs, tile, &g.pairs);
  const GemmProb *d = nullptr;
  TNA_TRY(arena_push(ar, probs.data(), probs.size(), s, &d));
  return gemm_grouped(g, d, (int)probs.size(), total, s);
}

int parts_for(int64_t n) {
  int64_t g = (n + 4095) / 4096;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 512));
}

constexpr int SPEC = 32;                    // doubles per spectrum record (the SVD writes 0..24)
constexpr double IDENT_TOL = 1e-10;         // largest deviation of an identity channel that is used as one
constexpr int LZ_SMALL_N = 4096;            // longest theta of the single-workgroup Lanczos path
constexpr int NT_SMALL = 512;               // its workgroup size
constexpr size_t LZ_SLOT = 128;             // per-chain h1/h2/y/nrm2 slots
constexpr size_t LZ_PER = 3 * LZ_SLOT + 8;  // doubles per chain before the partials
constexpr size_t LZ_PART = 128 * 512;       // partial-sum slots per chain and array
constexpr double LZ_TOL_F32 = 1e-6;         // least Lanczos residual tolerance with the FP32 operator

}  // namespace

// ====================================================================== engine
// One lockstep step of a set of chains: every chain does one bond visit.
// Used with a single chain by tna_dmrg_sweep and with many by the batch.
struct tna_engine_s {
  hipStream_t stream = nullptr;
  int nslot = 0;
  std::vector<DevBuf> V, X, Z, Lf, Rf, T1, T2;
  DevBuf ints, dbl, lzst, feat_d, y_d, recs;
  Arena ar;
  SvdGroup svd;
  DevBuf svd_wd, svd_wi, spec, S;
  std::vector<int> hflags;  // j (nslot) then active (nslot) of the last upload
  double *h_dbl = nullptr;
  float *h_feat = nullptr;
  double *h_rec = nullptr;  // per slot 2 LZ_HMAX: alpha_j, beta_j^2 of the single-workgroup path
  int *h_j = nullptr;
  std::vector<int> lz_last;  // per slot: Lanczos iterations of the previous visit (launch sizing)
  long small_launches = 0;
  long graph_launches = 0, lanczos_iters = 0;
  long heff_f32_iters = 0;  // Lanczos iterations whose H_eff ran on FP32 operands
  long svd_rows = 0, svd_rows_swept = 0;
  long ident_steps = 0;  // steps whose H_eff products skipped the MPO's identity channels
  double ident_dev = 0.0;  // largest identity-channel deviation at the last step
  double ms_lanczos = 0, ms_svd = 0, ms_env = 0;
};

namespace tna {

tna_status engine_create(int nslot, tna_engine *out) {
  auto e = std::make_unique<tna_engine_s>();
  e->nslot = nslot;
  TNA_HIP(hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking));  // default priority
  e->V.resize(nslot);
  e->X.resize(nslot);
  e->Z.resize(nslot);
  e->Lf.resize(nslot);
  e->Rf.resize(nslot);
  e->T1.resize(nslot);
  e->T2.resize(nslot);
  TNA_TRY(e->ints.ensure(sizeof(int) * 2 * nslot));
  TNA_TRY(e->dbl.ensure(sizeof(double) * 4 * nslot));  // Lanczos records, then identity-channel deviations
  TNA_TRY(e->lzst.ensure(sizeof(double) * (LZ_PER + 2 * LZ_PART) * nslot));
  TNA_TRY(e->spec.ensure(sizeof(double) * SPEC * nslot));
  TNA_TRY(e->feat_d.ensure(sizeof(float) * 32 * nslot));
  TNA_TRY(e->y_d.ensure(sizeof(float) * 4 * nslot));
  e->hflags.assign(2 * (size_t)nslot, 0);
  e->lz_last.assign(nslot, 0);
  TNA_HIP(hipHostMalloc((void **)&e->h_dbl, sizeof(double) * (SPEC * nslot + 2 * nslot + 16), hipHostMallocDefault));
  TNA_HIP(hipHostMalloc((void **)&e->h_feat, sizeof(float) * 32 * nslot, hipHostMallocDefault));
  TNA_TRY(e->recs.ensure(sizeof(double) * 2 * LZ_HMAX * nslot));
  TNA_HIP(hipHostMalloc((void **)&e->h_rec, sizeof(double) * 2 * LZ_HMAX * nslot, hipHostMallocDefault));
  TNA_HIP(hipHostMalloc((void **)&e->h_j, sizeof(int) * nslot, hipHostMallocDefault));
  *out = e.release();
  return TNA_OK;
}

void engine_destroy(tna_engine e) {
  if (!e) return;
  (void)hipStreamSynchronize(e->stream);
  for (auto *vec : {&e->V, &e->X, &e->Z, &e->Lf, &e->Rf, &e->T1, &e->T2})
    for (auto &b : *vec) b.release();
  for (DevBuf *b : {&e->ints, &e->dbl, &e->lzst, &e->feat_d, &e->y_d, &e->recs, &e->svd_wd, &e->svd_wi, &e->spec,
                    &e->S})
    b->release();
  arena_release(e->ar);
  e->svd.release();
  if (e->h_dbl) (void)hipHostFree(e->h_dbl);
  if (e->h_feat) (void)hipHostFree(e->h_feat);
  if (e->h_rec) (void)hipHostFree(e->h_rec);
  if (e->h_j) (void)hipHostFree(e->h_j);
  if (e->stream) (void)hipStreamDestroy(e->stream);
  delete e;
}

hipStream_t engine_stream(tna_engine e) { return e->stream; }
void engine_stats(tna_engine e, tna_batch_stats *st) {
  st->ms_lanczos = e->ms_lanczos;
  st->ms_svd = e->ms_svd;
  st->ms_env = e->ms_env;
  st->lanczos_iters = e->lanczos_iters;
  st->graph_launches = e->graph_launches;
  st->small_launches = e->small_launches;
  st->heff_f32_iters = e->heff_f32_iters;
  st->svd_rows = e->svd_rows;
  st->svd_rows_swept = e->svd_rows_swept;
  st->heff_ident_steps = e->ident_steps;
  st->heff_ident_dev = e->ident_dev;
  st->autotune_entries = (int)g_tune.table.size();
}

// Chains ch[q] (slot slot[q]) each visit bond b[q] in direction half[q]
// (0: left to right, 1: right to left).  Records go to logs[q] (may be null).
tna_status engine_step(tna_engine en, const std::vector<tna_dmrg> &ch, const std::vector<int> &slot,
                       const std::vector<int> &bond, const std::vector<int> &half, std::vector<double> &E_out,
                       std::vector<tna_visit_log *> &logs, tna_status *worst) {
  const int nc = (int)ch.size();
  if (nc == 0) return TNA_OK;
  // the context's stream; a context on the null stream (which cannot be captured) uses the engine's own
  hipStream_t s = ch[0]->ctx->stream ? ch[0]->ctx->stream : en->stream;
  const int d = ch[0]->d, D = ch[0]->D;
  const int I1 = D * d, I2 = D * d * d;
  const int prec = ch[0]->opts.heff_prec;
  const bool f32 = prec == TNA_HEFF_F32;
  // residual tolerance of the Lanczos stop rule; with the FP32 operator its rounding (~1e-7 of the
  // operator norm) sets a floor on the residual estimate, so the test uses at least 1e-6 relative
  auto tol_of = [&](tna_dmrg dm) { return f32 ? std::max(dm->opts.lanczos_tol, LZ_TOL_F32) : dm->opts.lanczos_tol; };
  arena_begin(en->ar);  // the previous step ended with a synchronisation
  // the captured iteration is released, and the stream drained (the pinned arena of this step may
  // still feed copies), on every way out of the step, errors included
  struct StepGuard {
    hipStream_t s;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    ~StepGuard() {
      (void)hipStreamSynchronize(s);
      if (gexec) (void)hipGraphExecDestroy(gexec);
      if (graph) (void)hipGraphDestroy(graph);
    }
  } guard{s};
  hipGraph_t &graph = guard.graph;
  hipGraphExec_t &gexec = guard.gexec;
  auto t0 = std::chrono::steady_clock::now();
  struct Visit {
    int b, half, chl, chm, chr, m, n, kmax, fixed;
    int64_t nv;
  };
  std::vector<Visit> vs(nc);
  for (int q = 0; q < nc; ++q) {
    tna_dmrg dm = ch[q];
    Visit &v = vs[q];
    const int sl = slot[q];
    v.b = bond[q];
    v.half = half[q];
    v.chl = dm->CL(v.b);
    v.chm = dm->chi[v.b];
    v.chr = dm->CR(v.b + 1);
    v.m = v.chl * d;
    v.n = d * v.chr;
    v.nv = (int64_t)v.m * v.n;
    v.fixed = dm->opts.lanczos_fixed_iters;
    const int km = v.fixed > 0 ? v.fixed : dm->opts.lanczos_kmax;
    v.kmax = (int)std::min<int64_t>(std::min(km, 120), v.nv);
    const size_t el = f32 ? sizeof(float) : sizeof(double);
    TNA_TRY(en->V[sl].ensure(sizeof(double) * (size_t)(v.kmax + 2) * v.nv));
    TNA_TRY(en->X[sl].ensure(el * (size_t)D * d * d * v.chl * v.chr));
    TNA_TRY(en->Z[sl].ensure(el * (size_t)D * d * d * v.chl * v.chr));
    if (f32) {
      TNA_TRY(en->Lf[sl].ensure(sizeof(float) * (size_t)v.chl * D * v.chl));
      TNA_TRY(en->Rf[sl].ensure(sizeof(float) * (size_t)v.chr * D * v.chr));
    }
  }
  int *j_dev = en->ints.as<int>(), *act_dev = j_dev + en->nslot;
  double *rec_dev = en->dbl.as<double>();
  auto theta_of = [&](int q) { return en->V[slot[q]].as<double>() + (int64_t)(vs[q].kmax + 1) * vs[q].nv; };
  // ---- theta = A_b A_{b+1}
  {
    GemmGroup g{0, 0, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
    std::vector<GemmProb> pr;
    for (int q = 0; q < nc; ++q) {
      const Visit &v = vs[q];
      pr.push_back(GemmProb{v.m, v.n, v.chm, v.chm, v.n, v.n, ch[q]->A[v.b].ptr, ch[q]->A[v.b + 1].ptr, theta_of(q),
                            nullptr, nullptr, nullptr, 0, 0, 0, 0});
    }
    TNA_TRY(tuned_gemm(0, g, pr, en->ar, s, true));
  }
  if (f32) {
    std::vector<CvtProb> cv;
    for (int q = 0; q < nc; ++q) {
      const Visit &v = vs[q];
      cv.push_back(CvtProb{ch[q]->Le[v.b].as<double>(), en->Lf[slot[q]].as<float>(), (int64_t)v.chl * D * v.chl});
      cv.push_back(CvtProb{ch[q]->Re[v.b + 1].as<double>(), en->Rf[slot[q]].as<float>(), (int64_t)v.chr * D * v.chr});
    }
    const CvtProb *dc = nullptr;
    TNA_TRY(arena_push(en->ar, cv.data(), cv.size(), s, &dc));
    TNA_TRY(convert_grouped(dc, (int)cv.size(), s));
  }
  // ---- Lanczos descriptors (slot-indexed j/active flags)
  std::vector<LzProb> lp(nc);
  int maxG = 1, maxk = 1;
  for (int q = 0; q < nc; ++q) {
    const Visit &v = vs[q];
    const int sl = slot[q];
    double *base = en->lzst.as<double>() + (LZ_PER + 2 * LZ_PART) * sl;
    LzProb &p = lp[q];
    p.n = v.nv;
    p.G = parts_for(v.nv);
    p.nkeep = 0;
    p.V = en->V[sl].as<double>();
    p.theta = theta_of(q);
    p.j = j_dev + sl;
    p.active = act_dev + sl;
    p.h1 = base;
    p.h2 = base + LZ_SLOT;
    p.y = base + 2 * LZ_SLOT;
    p.nrm2 = base + 3 * LZ_SLOT;
    p.part1 = base + LZ_PER;
    p.part2 = base + LZ_PER + LZ_PART;
    p.rec = rec_dev + 2 * sl;
    maxG = std::max(maxG, p.G);
    maxk = std::max(maxk, v.kmax);
  }
  // ---- the MPO's identity channels.  Every MPO here keeps the not-yet-started state in the last
  // bond channel and the finished state in the first (W[D-1][D-1] = W[0][0] = 1 are the only ways
  // into them), so for left-canonical tensors the left environment's channel D-1 is the identity
  // matrix and for right-canonical ones the right environment's channel 0 is.  When both hold to
  // 1e-10 for every chain of the step (checked on the device), S1 skips the channel-(D-1) rows of L
  // (that part of X is theta itself, which the mixing reads directly) and S4 skips the channel-0
  // columns (the mixing writes that part of Z straight into the result, which S4 then adds to):
  // a fifth less of both products for D = 5.  Otherwise (a stopped SVD, a hand-made state) the
  // full products run.
  bool ident = true;
  {
    double *dev = rec_dev + 2 * en->nslot;
    TNA_HIP(hipMemsetAsync(dev, 0, sizeof(double) * 2 * en->nslot, s));
    for (int q = 0; q < nc; ++q) {
      const Visit &v = vs[q];
      const int sl = slot[q];
      TNA_TRY(ident_deviation(ch[q]->Le[v.b].as<double>(), v.chl, D, D - 1, dev + 2 * sl, s));
      TNA_TRY(ident_deviation(ch[q]->Re[v.b + 1].as<double>(), v.chr, D, 0, dev + 2 * sl + 1, s));
    }
    double *hd = en->h_dbl + SPEC * en->nslot;
    TNA_HIP(hipMemcpyAsync(hd, dev, sizeof(double) * 2 * en->nslot, hipMemcpyDeviceToHost, s));
    TNA_HIP(hipStreamSynchronize(s));
    en->ident_dev = 0.0;
    for (int q = 0; q < nc; ++q) {
      const int sl = slot[q];
      if (!(hd[2 * sl] <= IDENT_TOL && hd[2 * sl + 1] <= IDENT_TOL)) ident = false;
      en->ident_dev = std::max(en->ident_dev, std::max(hd[2 * sl], hd[2 * sl + 1]));
    }
  }
  en->ident_steps += ident ? 1 : 0;
  std::vector<GemmProb> s1, s4;
  std::vector<int> s1_chain, s4_chain;  // chain of each problem
  std::vector<MixProb> mx;
  int64_t max_mix = 1;
  const size_t el = f32 ? sizeof(float) : sizeof(double);
  for (int q = 0; q < nc; ++q) {
    tna_dmrg dm = ch[q];
    const Visit &v = vs[q];
    const int sl = slot[q];
    const char *L = static_cast<const char *>(f32 ? (const void *)en->Lf[sl].ptr : dm->Le[v.b].ptr);
    const char *R = static_cast<const char *>(f32 ? (const void *)en->Rf[sl].ptr : dm->Re[v.b + 1].ptr);
    char *X = static_cast<char *>(en->X[sl].ptr), *Z = static_cast<char *>(en->Z[sl].ptr);
    MixProb mp{v.chl, v.chr, X, Z, (int64_t)D * d * d * v.chr, 1, (int64_t)d * d * D * v.chr, 1, d * d * v.chr,
               v.chr, D * v.chr, v.chr, dm->M12.as<double>() + (size_t)I2 * I2 * v.b, act_dev + sl};
    if (!ident) {
      // S1: X[(a,w)][(s',t',c')] = L[(a,w)][a'] V_j[a'][(s',t',c')]
      s1.push_back(GemmProb{v.chl * D, d * d * v.chr, v.chl, v.chl, d * d * v.chr, d * d * v.chr, L, lp[q].V, X,
                            j_dev + sl, nullptr, act_dev + sl, v.nv, 0, 0, 0});
      s1_chain.push_back(q);
      // S4: V_{j+1}[(a,s,t)][c] = Z[(a,s,t)][(w'',c')] R[c][(w'',c')]
      s4.push_back(GemmProb{v.chl * d * d, v.chr, D * v.chr, D * v.chr, D * v.chr, v.chr, Z, R, lp[q].V + v.nv,
                            nullptr, j_dev + sl, act_dev + sl, 0, v.nv, 0, 0});
      s4_chain.push_back(q);
    } else {
      // S1 per channel w < D-1: X[(a,w)][.] = L[a][w][a'] V_j[a'][.]
      for (int w = 0; w < D - 1; ++w) {
        s1.push_back(GemmProb{v.chl, d * d * v.chr, v.chl, D * v.chl, d * d * v.chr, D * d * d * v.chr,
                              L + el * w * v.chl, lp[q].V, X + el * (size_t)w * d * d * v.chr, j_dev + sl, nullptr,
                              act_dev + sl, v.nv, 0, 0, 0});
        s1_chain.push_back(q);
      }
      mp.in_last = lp[q].V;  // channel D-1 of X is V_j
      mp.is0_last = (int64_t)d * d * v.chr;
      mp.jin = j_dev + sl;
      mp.jin_stride = v.nv;
      mp.out_first = lp[q].V + v.nv;  // channel 0 of Z goes to V_{j+1}
      mp.os0_first = (int64_t)d * d * v.chr;
      mp.och1_first = v.chr;
      mp.jout = j_dev + sl;
      mp.jout_stride = v.nv;
      // S4 over the channels w'' >= 1, added to V_{j+1}
      s4.push_back(GemmProb{v.chl * d * d, v.chr, (D - 1) * v.chr, D * v.chr, D * v.chr, v.chr, Z + el * v.chr,
                            R + el * v.chr, lp[q].V + v.nv, nullptr, j_dev + sl, act_dev + sl, 0, v.nv, 0, 0});
      s4_chain.push_back(q);
    }
    // S2: Z[a][(s,t)][w''][c'] = sum W12 X[a][w][(s',t')][c'];  channel strides per (a, c')
    mx.push_back(mp);
    max_mix = std::max<int64_t>(max_mix, (int64_t)v.chl * v.chr);
  }
  const int tc = f32 ? G_F32 : G_F64;
  GemmGroup g1{0, 0, tc, G_F64, tc, tc, 64, 1.0, 0.0, 0.0, 0.0, "heff"};  // the H_eff products S1 and S4
  GemmGroup g4{0, 1, tc, tc, G_F64, tc, 64, 1.0, ident ? 1.0 : 0.0, 0.0, 0.0, "heff"};
  const int n1 = (int)s1.size(), n4 = (int)s4.size();
  for (int q = 0; q < nc; ++q) {
    en->hflags[slot[q]] = 0;
    en->hflags[en->nslot + slot[q]] = 1;
  }
  // active flags: uploaded only when they differ from what the device holds (no kernel writes them)
  std::vector<int> act_up(en->hflags.begin() + en->nslot, en->hflags.end());
  auto push_act = [&]() -> tna_status {
    if (std::equal(act_up.begin(), act_up.end(), en->hflags.begin() + en->nslot)) return TNA_OK;
    act_up.assign(en->hflags.begin() + en->nslot, en->hflags.end());
    return put_dev(en->ar, en->hflags.data() + en->nslot, (size_t)en->nslot, act_dev, s);
  };
  TNA_TRY(put_dev(en->ar, en->hflags.data(), 2 * (size_t)en->nslot, j_dev, s));
  const LzProb *dlp = nullptr;
  TNA_TRY(arena_push(en->ar, lp.data(), nc, s, &dlp));
  TNA_TRY(lz_start(dlp, nc, maxG, s));
  // ---- which visits run whole Lanczos iterations inside one workgroup (short theta, all of
  // H_eff's operands in LDS); the rest go through the grouped GEMM/mixing/CGS2 launches
  std::vector<int> small(nc, 0), sm_ac(nc, 1);
  int nsmall = 0;
  size_t lds_small = 0;
  if (d == 2 && D * d * d <= 64) {
    for (int q = 0; q < nc; ++q) {
      const Visit &v = vs[q];
      if (v.nv > LZ_SMALL_N) continue;
      int ac = std::max(1, std::min(v.chl, NT_SMALL / std::max(1, v.chr)));
      while (ac > 1 && lz_small_lds(v.chl, v.chr, d, D, ac, f32) > LZ_SMALL_LDS_MAX) ac /= 2;
      const size_t need = lz_small_lds(v.chl, v.chr, d, D, ac, f32);
      if (need > LZ_SMALL_LDS_MAX) continue;
      small[q] = 1;
      sm_ac[q] = ac;
      lds_small = std::max(lds_small, need);
      ++nsmall;
    }
  }
  const int nbig = nc - nsmall;
  int tile1 = 64, tile4 = 64;
  const MixProb *dmx = nullptr;
  const GemmProb *dp1 = nullptr, *dp4 = nullptr;
  int tot1 = 0, tot4 = 0;
  const bool use_graph =
      !(timing_may_match("heff") || timing_may_match("gemmg") || timing_may_match("mixg") || timing_may_match("lz."));
  double lz_bytes = 0.0;  // one CGS pass at the current iteration, all chains (timing only)
  auto lz_hint = [&](int it) {
    double b = 0.0;
    for (int q = 0; q < nc; ++q) b += 8.0 * (double)(std::min(it, vs[q].kmax) + 2) * vs[q].nv;
    return b;
  };
  auto iterate_direct = [&]() -> tna_status {
    TNA_TRY(gemm_grouped(g1, dp1, n1, tot1, s));
    TNA_TRY(mix_grouped(dmx, nc, max_mix, D, d * d, d * d, D, f32, s));
    TNA_TRY(gemm_grouped(g4, dp4, n4, tot4, s));
    return lz_iteration(dlp, nc, maxG, maxk, lz_bytes, s);
  };
  if (nbig > 0) {
    // small visits take no part in the grouped launches (their active flag is off here)
    if (nsmall > 0) {
      for (int q = 0; q < nc; ++q) en->hflags[en->nslot + slot[q]] = !small[q];
      TNA_TRY(push_act());
    }
    // tile choice for the two H_eff GEMMs, measured before capture (j = 0)
    std::vector<GemmProb> b1, b4;
    for (int i = 0; i < n1; ++i)
      if (!small[s1_chain[i]]) b1.push_back(s1[i]);
    for (int i = 0; i < n4; ++i)
      if (!small[s4_chain[i]]) b4.push_back(s4[i]);
    TNA_TRY(tuned_gemm(1, g1, b1, en->ar, s, true, &tile1));
    TNA_TRY(tuned_gemm(2, g4, b4, en->ar, s, true, &tile4));
    TNA_TRY(arena_push(en->ar, mx.data(), nc, s, &dmx));
    std::vector<GemmProb> p1 = s1, p4 = s4;
    g1.tile = tile1;
    g4.tile = tile4;
    g1.flops = group_flops(b1);
    g4.flops = group_flops(b4);
    g1.bytes = group_bytes(b1, f32 ? 4 : 8);
    g4.bytes = group_bytes(b4, f32 ? 4 : 8);
    tot1 = gemm_group_tiles(p1, tile1, &g1.pairs);
    tot4 = gemm_group_tiles(p4, tile4, &g4.pairs);
    TNA_TRY(arena_push(en->ar, p1.data(), n1, s, &dp1));
    TNA_TRY(arena_push(en->ar, p4.data(), n4, s, &dp4));
    // capture one Lanczos iteration (H_eff + CGS2 + record + normalise + advance); with
    // kernel timing on, the iteration is launched directly so that events can bracket
    // single kernels
    if (use_graph) {
      TNA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      tna_status cs = gemm_grouped(g1, dp1, n1, tot1, s);
      if (cs == TNA_OK) cs = mix_grouped(dmx, nc, max_mix, D, d * d, d * d, D, f32, s);
      if (cs == TNA_OK) cs = gemm_grouped(g4, dp4, n4, tot4, s);
      if (cs == TNA_OK) cs = lz_iteration(dlp, nc, maxG, maxk, 0.0, s);
      hipError_t ce = hipStreamEndCapture(s, &graph);
      if (cs != TNA_OK) return cs;
      if (ce != hipSuccess) {
        set_error(std::string("graph capture: ") + hipGetErrorString(ce));
        return TNA_ERR_DEVICE;
      }
      hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        set_error(std::string("graph instantiate: ") + hipGetErrorString(ie));
        return TNA_ERR_DEVICE;
      }
    }
  }
  // ---- per-chain decisions on each new (alpha_j, beta_j^2), as in the single-chain method
  std::vector<std::vector<double>> al(nc), be(nc), yv(nc);
  std::vector<int> conv(nc, 0), nkeep(nc, 0), iters(nc, 0), restart(nc, 0), act(nc, 0);
  std::vector<double> Ec(nc, 0.0);
  tna_status lst = TNA_OK;
  // returns true when chain q stops (converged, breakdown or kmax)
  auto take = [&](int q, double a, double b2) -> bool {
    al[q].push_back(a);
    be[q].push_back(std::sqrt(b2));
    iters[q] += 1;
    const int nn = (int)al[q].size();
    yv[q].assign(nn, 0.0);
    Ec[q] = tridiag_lowest_host(nn, al[q].data(), be[q].data(), yv[q].data());
    const double resid = std::fabs(be[q][nn - 1] * yv[q][nn - 1]);
    bool stop = false;
    if (vs[q].fixed > 0) {
      if (nn >= vs[q].kmax || be[q][nn - 1] < 1e-14) stop = conv[q] = 1;
    } else if (resid <= tol_of(ch[q]) * std::max(1.0, std::fabs(Ec[q])) || be[q][nn - 1] < 1e-14) {
      stop = conv[q] = 1;
    } else if (nn >= vs[q].kmax) {
      stop = true;
    }
    if (stop) {
      nkeep[q] = nn;
      act[q] = 0;
    }
    return stop;
  };
  // records t0 .. jn-1 of chain q at once, from the single-workgroup path.  The stopping rule is
  // take()'s; the tridiagonal problem is solved for the newest record, and only when that one
  // meets the residual test are the earlier new records solved, in order, to find the first that
  // does (a record that met it and was followed by one that did not is not looked for).  Returns
  // true when the chain stops.
  auto take_batch = [&](int q, const double *r, int t0, int jn) -> bool {
    const int base = (int)al[q].size();
    const bool fixed = vs[q].fixed > 0;
    int last = jn, cheap = 0;  // cheap: breakdown or kmax at record `last`
    for (int t = t0; t < jn; ++t) {
      al[q].push_back(r[2 * t]);
      be[q].push_back(std::sqrt(r[2 * t + 1]));
      if (be[q].back() < 1e-14 || t + 1 >= vs[q].kmax) {
        last = t + 1;
        cheap = 1;
        break;
      }
    }
    auto solve = [&](int nn) {
      yv[q].assign(nn, 0.0);
      Ec[q] = tridiag_lowest_host(nn, al[q].data(), be[q].data(), yv[q].data());
      return std::fabs(be[q][nn - 1] * yv[q][nn - 1]) <= tol_of(ch[q]) * std::max(1.0, std::fabs(Ec[q]));
    };
    int stop_at = 0;
    bool converged = false;
    if (fixed) {
      solve(last);
      if (cheap) stop_at = last, converged = true;
    } else if (solve(last)) {
      stop_at = last;
      converged = true;
      for (int nn = base + 1; nn < last; ++nn)
        if (solve(nn)) {
          stop_at = nn;
          break;
        }
      if (stop_at == last) solve(last);  // the earlier trial solves overwrote Ec / yv
    } else if (cheap) {
      stop_at = last;
      converged = be[q][last - 1] < 1e-14;
    }
    const int nn = stop_at > 0 ? stop_at : last;
    al[q].resize(nn);
    be[q].resize(nn);
    iters[q] += nn - base;
    if (stop_at == 0) return false;
    conv[q] = converged;
    nkeep[q] = nn;
    act[q] = 0;
    return true;
  };
  // chains in `set` that stopped at kmax unconverged restart from their Ritz vector
  auto restart_stopped = [&](const std::vector<int> &set) -> tna_status {
    std::vector<int> rs(nc, 0);
    bool any = false;
    for (int q = 0; q < nc; ++q) {
      rs[q] = set[q] && !act[q] && !conv[q] && nkeep[q] > 0 && restart[q] < ch[q]->opts.lanczos_restarts;
      any = any || rs[q];
    }
    if (!any) return TNA_OK;
    for (int q = 0; q < nc; ++q) {
      en->hflags[en->nslot + slot[q]] = rs[q];
      lp[q].nkeep = rs[q] ? nkeep[q] : 0;
      if (rs[q]) TNA_TRY(put_dev(en->ar, yv[q].data(), (size_t)nkeep[q], lp[q].y, s));
    }
    TNA_TRY(push_act());
    const LzProb *dr = nullptr;
    TNA_TRY(arena_push(en->ar, lp.data(), nc, s, &dr));
    TNA_TRY(lz_ritz(dr, nc, maxG, s));
    TNA_TRY(lz_start(dr, nc, maxG, s));
    for (int q = 0; q < nc; ++q) {
      if (!rs[q]) continue;
      restart[q] += 1;
      al[q].clear();
      be[q].clear();
      nkeep[q] = 0;
      act[q] = 1;
      en->hflags[slot[q]] = 0;
      TNA_TRY(put_dev(en->ar, en->hflags.data() + slot[q], 1, j_dev + slot[q], s));
    }
    return TNA_OK;
  };
  // ---- single-workgroup path: launches of several iterations, then one read of the records
  if (nsmall > 0) {
    std::vector<LzSmall> sp;
    std::vector<int> sq;  // chain of each descriptor
    double *rec_small = en->recs.as<double>();
    for (int q = 0; q < nc; ++q) {
      if (!small[q]) continue;
      const Visit &v = vs[q];
      const int sl = slot[q];
      tna_dmrg dm = ch[q];
      sp.push_back(LzSmall{v.chl, v.chr, v.kmax, sm_ac[q], D, 0, dm->Le[v.b].as<double>(), dm->Re[v.b + 1].as<double>(),
                           dm->M12.as<double>() + (size_t)I2 * I2 * v.b, lp[q].V, j_dev + sl, act_dev + sl,
                           rec_small + (size_t)2 * LZ_HMAX * sl});
      sq.push_back(q);
      act[q] = 1;
    }
    const LzSmall *dsp = nullptr;
    TNA_TRY(arena_push(en->ar, sp.data(), sp.size(), s, &dsp));
    std::vector<int> start(nc, 0), jdev(nc, 0);
    // algorithmic work of one iteration at index t: H_eff products + CGS2 (two dot and two
    // update passes over V_0..V_t) ; bytes: theta in, V_{t+1} out, the four passes over V
    auto it_flops = [&](int q, int t) {
      const Visit &v = vs[q];
      const double cl = v.chl, cr = v.chr, dsq = (double)d * d;
      return 2.0 * D * dsq * cl * cr * (cl + cr) + 2.0 * (D * dsq) * (D * dsq) * cl * cr +
             8.0 * (t + 1) * (double)v.nv;
    };
    auto it_bytes = [&](int q, int t) { return 8.0 * (double)vs[q].nv * (2.0 + 4.0 * (t + 1)); };
    // the first launch runs about as many iterations as the chain's previous visit needed (the
    // sweep's neighbouring bonds converge alike), later launches a few at a time: fewer host
    // round trips and fewer iterations past convergence
    int chunk = 0;
    for (int q : sq) chunk = std::max(chunk, en->lz_last[slot[q]] - 2);
    chunk = chunk > 0 ? std::min(std::max(chunk, 4), 64) : 16;
    for (;;) {
      bool live = false;
      for (int q : sq) live = live || act[q];
      if (!live) break;
      for (int q = 0; q < nc; ++q) en->hflags[en->nslot + slot[q]] = small[q] && act[q];
      TNA_TRY(push_act());
      TNA_TRY(lz_small(dsp, (int)sp.size(), D, d * d, chunk, lds_small, f32, s));
      en->small_launches += 1;
      TNA_HIP(hipMemcpyAsync(en->h_rec, rec_small, sizeof(double) * 2 * LZ_HMAX * en->nslot, hipMemcpyDeviceToHost,
                             s));
      TNA_HIP(hipStreamSynchronize(s));
      for (int q : sq) en->h_j[slot[q]] = (int)en->h_rec[(size_t)2 * LZ_HMAX * slot[q] + 2 * LZ_HMAX - 1];
      const char *tname = f32 ? "lz.small.f32" : "lz.small";
      if (timing_wanted(tname)) {
        double fl = 0.0, by = 0.0;
        for (int q : sq)
          for (int t = jdev[q]; t < en->h_j[slot[q]]; ++t) {
            fl += it_flops(q, t);
            by += it_bytes(q, t);
          }
        timer_add_work(tname, fl, by);
      }
      if (f32)
        for (int q : sq) en->heff_f32_iters += en->h_j[slot[q]] - jdev[q];
      for (int q : sq) jdev[q] = en->h_j[slot[q]];
      for (int q : sq) {
        if (!act[q]) continue;
        start[q] = (int)al[q].size();
        const double *r = en->h_rec + (size_t)2 * LZ_HMAX * slot[q];
        const int jn = en->h_j[slot[q]];
        int jn_ok = jn;  // records past a non-finite one are not taken
        for (int t = start[q]; t < jn; ++t)
          if (!std::isfinite(r[2 * t]) || !std::isfinite(r[2 * t + 1])) {
            jn_ok = t;
            break;
          }
        if (jn_ok > start[q]) take_batch(q, r, start[q], jn_ok);
        if (act[q] && jn_ok < jn) {
          set_error("lanczos: non-finite coefficient");
          return TNA_ERR_NONFINITE;
        }
        if (act[q] && jn <= start[q]) {
          set_error("lanczos (single-workgroup path): no progress");
          return TNA_ERR_DEVICE;
        }
      }
      TNA_TRY(restart_stopped(small));
      for (int q : sq)
        if (act[q] && al[q].empty()) jdev[q] = 0;  // restarted: j reset on the device
      chunk = 4;
    }
    for (int q : sq) en->lz_last[slot[q]] = iters[q];
  }
  // ---- lockstep grouped path: replay, read every chain's (alpha_j, beta_j^2), decide on the host
  for (int q = 0; q < nc; ++q) act[q] = !small[q];
  std::vector<int> bigset(nc);
  for (int q = 0; q < nc; ++q) bigset[q] = !small[q];
  if (nbig > 0 && nsmall > 0) {
    for (int q = 0; q < nc; ++q) en->hflags[en->nslot + slot[q]] = act[q];
    TNA_TRY(push_act());
  }
  for (;;) {
    int live = 0;
    for (int q = 0; q < nc; ++q) live += act[q];
    if (live == 0) break;
    hipError_t le = hipSuccess;
    lz_bytes = lz_hint(iters.empty() ? 0 : *std::max_element(iters.begin(), iters.end()));
    if (use_graph) le = hipGraphLaunch(gexec, s);
    else if (iterate_direct() != TNA_OK) le = hipErrorLaunchFailure;
    if (le == hipSuccess) le = hipMemcpyAsync(en->h_dbl, rec_dev, sizeof(double) * 2 * en->nslot,
                                              hipMemcpyDeviceToHost, s);
    if (le == hipSuccess) le = hipStreamSynchronize(s);
    if (le != hipSuccess) {
      set_error(std::string("lanczos iteration: ") + hipGetErrorString(le));
      lst = TNA_ERR_DEVICE;
      break;
    }
    if (use_graph) en->graph_launches += 1;
    if (f32)
      for (int q = 0; q < nc; ++q) en->heff_f32_iters += act[q];
    bool changed = false;
    for (int q = 0; q < nc; ++q) {
      if (!act[q]) continue;
      const double a = en->h_dbl[2 * slot[q]], b2 = en->h_dbl[2 * slot[q] + 1];
      if (!std::isfinite(a) || !std::isfinite(b2)) {
        set_error("lanczos: non-finite coefficient");
        lst = TNA_ERR_NONFINITE;
        break;
      }
      changed = take(q, a, b2) || changed;
    }
    if (lst != TNA_OK) break;
    if (!changed) continue;
    lst = restart_stopped(bigset);
    if (lst != TNA_OK) break;
    for (int q = 0; q < nc; ++q) en->hflags[en->nslot + slot[q]] = act[q];
    TNA_TRY(push_act());
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  gexec = nullptr;
  graph = nullptr;
  if (lst != TNA_OK) return lst;
  // ---- Ritz vectors
  for (int q = 0; q < nc; ++q) {
    lp[q].nkeep = nkeep[q];
    en->hflags[en->nslot + slot[q]] = 1;
    en->lanczos_iters += iters[q];
    if (!conv[q] && *worst == TNA_OK) *worst = TNA_ERR_NOCONV;
    TNA_TRY(put_dev(en->ar, yv[q].data(), (size_t)nkeep[q], lp[q].y, s));
  }
  TNA_TRY(push_act());
  {
    const LzProb *dr = nullptr;
    TNA_TRY(arena_push(en->ar, lp.data(), nc, s, &dr));
    TNA_TRY(lz_ritz(dr, nc, maxG, s));
  }
  TNA_HIP(hipStreamSynchronize(s));  // yv (pageable) copies done
  auto t1 = std::chrono::steady_clock::now();
  // ---- SVD of every theta, entropy of the full spectra, needed ranks
  std::vector<SvdMat> mats(nc);
  size_t nd = 0, ni = 0, ns = 0;
  for (int q = 0; q < nc; ++q) {
    // the isometric factor comes from the accumulated rotations (orthonormal whatever the
    // convergence of rows at the rounding level): left to right the rows of theta are
    // orthogonalised (U isometric, Vt scaled), right to left its columns (Vt isometric, U scaled);
    // a rectangular theta keeps the orientation its shape needs
    TNA_TRY(svd_plan_mat(vs[q].m, vs[q].n, TNA_F64, nc, &mats[q], vs[q].half == 0 ? 1 : 2));
    mats[q].rows_scaled = vs[q].half == 0 ? !mats[q].trans : mats[q].trans;
    // with the FP32 operator theta carries noise of about 1e-7 of its norm: rows below it are
    // rounding-level rows for the Jacobi, and the numerical rank is counted above it
    if (f32) mats[q].noise_rel = 1e-7;
    nd += svd_work_doubles(mats[q]);
    ni += svd_work_ints(mats[q]);
    ns += mats[q].R;
  }
  TNA_TRY(en->svd_wd.ensure(sizeof(double) * nd));
  TNA_TRY(en->svd_wi.ensure(sizeof(int) * ni));
  TNA_TRY(en->S.ensure(sizeof(double) * ns));
  std::vector<double *> Sq(nc);
  {
    double *dw = en->svd_wd.as<double>(), *sp = en->S.as<double>();
    int *iw = en->svd_wi.as<int>();
    for (int q = 0; q < nc; ++q) {
      SvdMat &a = mats[q];
      svd_bind_work(&a, dw, iw);
      dw += svd_work_doubles(a);
      iw += svd_work_ints(a);
      a.A = lp[q].theta;
      a.S = sp;
      Sq[q] = sp;
      sp += a.R;
      a.spec = en->spec.as<double>() + SPEC * q;
      a.eps_target = ch[q]->opts.eps_target > 0 ? ch[q]->opts.eps_target : 1e-8;
      a.thr = ch[q]->opts.chi_rule == TNA_CHI_THRESHOLD ? ch[q]->opts.rule_param : 0.0;
      a.out_type = TNA_F64;
    }
  }
  std::vector<int> sweeps;
  tna_status sst = svd_group_run(mats, en->svd, ch[0]->opts.svd_max_sweeps, sweeps, s, true);
  if (sst != TNA_OK && sst != TNA_ERR_NOCONV) return sst;
  for (auto &a : mats) {
    en->svd_rows += a.R;
    en->svd_rows_swept += a.Ra;
  }
  if (sst == TNA_ERR_NOCONV && *worst == TNA_OK) *worst = TNA_ERR_NOCONV;
  TNA_HIP(hipMemcpyAsync(en->h_dbl, en->spec.ptr, sizeof(double) * SPEC * nc, hipMemcpyDeviceToHost, s));
  TNA_HIP(hipStreamSynchronize(s));
  for (int q = 0; q < nc; ++q)
    if (!std::isfinite(en->h_dbl[SPEC * q]) || !std::isfinite(en->h_dbl[SPEC * q + 1])) {
      set_error("dmrg visit: non-finite two-site spectrum");
      return TNA_ERR_NONFINITE;
    }
  for (int q = 0; q < nc; ++q)  // single-workgroup Jacobi paths: sweeps and convergence from spec[7]
    if (mats[q].fused) {
      const double f = en->h_dbl[SPEC * q + 7];
      sweeps[q] = (int)std::fabs(f);
      if (f < 0.0 && *worst == TNA_OK) *worst = TNA_ERR_NOCONV;
    }
  // ---- controllers, scheduler inputs, kept ranks
  std::vector<double> terms(6 * nc);
  std::vector<int> chi_next(nc), kk(nc), kneed(nc), chs(nc, 0), fb(nc, 0);
  std::vector<int> want_pred;
  for (int q = 0; q < nc; ++q) {
    tna_dmrg dm = ch[q];
    const Visit &v = vs[q];
    const double *h = en->h_dbl + SPEC * q;
    const double Sent = h[1];
    kneed[q] = (int)h[6];
    // rank rule: Algorithm 2 (PID, also run and logged under the threshold rule) or Algorithm 1
    if (dm->opts.chi_rule == TNA_CHI_ENTROPY)
      TNA_TRY(entropy_update(&dm->pid, dm->opts.rule_param, &dm->st[v.b], Sent, &chi_next[q], &terms[6 * q]));
    else
      TNA_TRY(pid_update(&dm->pid, &dm->st[v.b], Sent, &chi_next[q], &terms[6 * q]));
    // scheduler inputs: EMA history (oldest first, padded with the oldest),
    // 16 largest log sigma (floored at ln 1e-16), relative bond position
    auto &hb = dm->hist[v.b];
    if (dm->nhist[v.b] < 8) hb[dm->nhist[v.b]++] = terms[6 * q + 4];
    else {
      for (int r = 0; r < 7; ++r) hb[r] = hb[r + 1];
      hb[7] = terms[6 * q + 4];
    }
    const int nh = dm->nhist[v.b];
    float *f = en->h_feat + 32 * q;
    for (int r = 0; r < 8; ++r) f[r] = (float)hb[r < 8 - nh ? 0 : r - (8 - nh)];
    const double floor_ln = std::log(1e-16);
    for (int r = 0; r < 16; ++r) {
      const double sv = h[8 + r];
      f[8 + r] = (float)(sv > 0 ? std::max(std::log(sv), floor_ln) : floor_ln);
    }
    f[24] = (float)((v.b + 1.0) / dm->N);
    int keep = dm->opts.fixed_chi > 0 ? dm->opts.fixed_chi : chi_next[q];
    if (dm->opts.fixed_chi <= 0 && dm->opts.chi_rule == TNA_CHI_THRESHOLD)  // min(chi_max, r), r >= 1
      keep = std::min(dm->pid.chi_max, std::max(1, (int)h[24]));
    if (dm->sched && dm->opts.fixed_chi <= 0 && dm->opts.chi_rule == TNA_CHI_PID && dm->pred[v.b] > 0) {
      chs[q] = dm->pred[v.b];
      if (std::min(chs[q], mats[q].R) < std::min(kneed[q], mats[q].R)) fb[q] = 1;  // would miss eps_target
      else keep = chs[q];
    }
    if (dm->sched) want_pred.push_back(q);
    kk[q] = std::min(keep, mats[q].R);
  }
  // proposals for each bond's next visit (one forward per network)
  if (!want_pred.empty()) {
    TNA_TRY(put_dev(en->ar, en->h_feat, (size_t)32 * nc, en->feat_d.as<float>(), s));
    for (size_t i = 0; i < want_pred.size(); ++i) {
      const int q = want_pred[i];
      TNA_TRY(mlp_forward_dev(ch[q]->sched, 1, en->feat_d.as<float>() + 32 * q, en->y_d.as<float>() + 4 * q, s));
    }
    std::vector<float> yb(4 * nc);
    TNA_HIP(hipMemcpyAsync(yb.data(), en->y_d.ptr, sizeof(float) * 4 * nc, hipMemcpyDeviceToHost, s));
    TNA_HIP(hipStreamSynchronize(s));
    for (int q : want_pred) {
      tna_dmrg dm = ch[q];
      const double yv1 = yb[4 * q];
      double kp = std::isfinite(yv1) ? std::nearbyint(std::exp2(std::min(yv1, 30.0))) : dm->pid.chi_min;
      kp = std::min<double>(std::max<double>(kp, dm->pid.chi_min), dm->pid.chi_max);
      dm->pred[vs[q].b] = (int)kp;
    }
  }
  for (int q = 0; q < nc; ++q) {
    tna_dmrg dm = ch[q];
    const Visit &v = vs[q];
    SvdMat &a = mats[q];
    a.k = kk[q];
    TNA_TRY(dm->A[v.b].ensure(sizeof(double) * (size_t)v.m * kk[q]));
    TNA_TRY(dm->A[v.b + 1].ensure(sizeof(double) * (size_t)kk[q] * v.n));
    a.U = dm->A[v.b].ptr;
    a.Vt = dm->A[v.b + 1].ptr;
    a.scale_mode = v.half == 0 ? 1 : 2;
  }
  TNA_TRY(svd_group_outputs(mats, en->svd, s));
  auto t2 = std::chrono::steady_clock::now();
  // ---- environments: the left one grows on L->R visits, the right one on R->L
  {
    std::vector<GemmProb> l1, l3, r1, r3;
    std::vector<MixProb> lm, rm;
    int64_t maxl = 1, maxr = 1;
    for (int q = 0; q < nc; ++q) {
      tna_dmrg dm = ch[q];
      const Visit &v = vs[q];
      const int k = kk[q], sl = slot[q];
      dm->chi[v.b] = k;
      if (v.half == 0) {
        const int chl = v.chl;
        TNA_TRY(en->T1[sl].ensure(sizeof(double) * (size_t)chl * D * d * k));
        TNA_TRY(en->T2[sl].ensure(sizeof(double) * (size_t)chl * D * d * k));
        TNA_TRY(dm->Le[v.b + 1].ensure(sizeof(double) * (size_t)k * D * k));
        l1.push_back(GemmProb{chl * D, d * k, chl, chl, d * k, d * k, dm->Le[v.b].ptr, dm->A[v.b].ptr, en->T1[sl].ptr,
                              nullptr, nullptr, nullptr, 0, 0, 0, 0});
        lm.push_back(MixProb{chl, k, en->T1[sl].ptr, en->T2[sl].ptr, (int64_t)D * d * k, 1, (int64_t)d * D * k, 1,
                             d * k, k, D * k, k, dm->Ml.as<double>() + (size_t)I1 * I1 * v.b, nullptr});
        l3.push_back(GemmProb{k, D * k, chl * d, k, D * k, D * k, dm->A[v.b].ptr, en->T2[sl].ptr, dm->Le[v.b + 1].ptr,
                              nullptr, nullptr, nullptr, 0, 0, 0, 0});
        maxl = std::max<int64_t>(maxl, (int64_t)chl * k);
      } else {
        const int chr = v.chr;
        TNA_TRY(en->T1[sl].ensure(sizeof(double) * (size_t)chr * D * k * d));
        TNA_TRY(en->T2[sl].ensure(sizeof(double) * (size_t)chr * D * k * d));
        TNA_TRY(dm->Re[v.b].ensure(sizeof(double) * (size_t)k * D * k));
        r1.push_back(GemmProb{chr * D, k * d, chr, chr, chr, k * d, dm->Re[v.b + 1].ptr, dm->A[v.b + 1].ptr,
                              en->T1[sl].ptr, nullptr, nullptr, nullptr, 0, 0, 0, 0});
        rm.push_back(MixProb{chr, k, en->T1[sl].ptr, en->T2[sl].ptr, (int64_t)D * k * d, d, (int64_t)D * k, 1, k * d, 1,
                             chr * D * k, k, dm->Mr.as<double>() + (size_t)I1 * I1 * (v.b + 1), nullptr});
        r3.push_back(GemmProb{k, D * k, d * chr, d * chr, D * k, D * k, dm->A[v.b + 1].ptr, en->T2[sl].ptr,
                              dm->Re[v.b].ptr, nullptr, nullptr, nullptr, 0, 0, 0, 0});
        maxr = std::max<int64_t>(maxr, (int64_t)chr * k);
      }
    }
    GemmGroup nn{0, 0, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
    GemmGroup nt{0, 1, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
    GemmGroup tn{1, 0, G_F64, G_F64, G_F64, G_F64, 64, 1.0, 0.0, 0.0, 0.0};
    if (!l1.empty()) {
      TNA_TRY(tuned_gemm(3, nn, l1, en->ar, s, true));
      const MixProb *dm_ = nullptr;
      TNA_TRY(arena_push(en->ar, lm.data(), lm.size(), s, &dm_));
      TNA_TRY(mix_grouped(dm_, (int)lm.size(), maxl, D, d, d, D, 0, s));
      TNA_TRY(tuned_gemm(4, tn, l3, en->ar, s, true));
    }
    if (!r1.empty()) {
      TNA_TRY(tuned_gemm(5, nt, r1, en->ar, s, true));
      const MixProb *dm_ = nullptr;
      TNA_TRY(arena_push(en->ar, rm.data(), rm.size(), s, &dm_));
      TNA_TRY(mix_grouped(dm_, (int)rm.size(), maxr, D, d, d, D, 0, s));
      TNA_TRY(tuned_gemm(6, nn, r3, en->ar, s, true));
    }
  }
  // per-visit records: truncation sums of the outputs pass and the last kept value
  TNA_HIP(hipMemcpyAsync(en->h_dbl, en->spec.ptr, sizeof(double) * SPEC * nc, hipMemcpyDeviceToHost, s));
  std::vector<double> slast(nc, 0.0);
  for (int q = 0; q < nc; ++q)
    TNA_HIP(hipMemcpyAsync(en->h_dbl + SPEC * nc + q, Sq[q] + (kk[q] - 1), sizeof(double), hipMemcpyDeviceToHost, s));
  TNA_HIP(hipStreamSynchronize(s));
  auto t3 = std::chrono::steady_clock::now();
  const double mL = std::chrono::duration<double, std::milli>(t1 - t0).count();
  const double mS = std::chrono::duration<double, std::milli>(t2 - t1).count();
  const double mE = std::chrono::duration<double, std::milli>(t3 - t2).count();
  en->ms_lanczos += mL;
  en->ms_svd += mS;
  en->ms_env += mE;
  for (int q = 0; q < nc; ++q) {
    E_out[q] = Ec[q];
    tna_visit_log *rp = logs.empty() ? nullptr : logs[q];
    if (!rp) continue;
    tna_visit_log &r = *rp;
    const double *h = en->h_dbl + SPEC * q;
    const double *tm = &terms[6 * q];
    std::memset(&r, 0, sizeof r);
    r.sweep = ch[q]->sweeps_done; r.dir = vs[q].half; r.bond = vs[q].b; r.m = vs[q].m; r.n = vs[q].n;
    r.k = kk[q]; r.chi_ctrl = chi_next[q]; r.lanczos_iters = iters[q]; r.svd_sweeps = sweeps[q];
    r.lanczos_ok = conv[q]; r.E = Ec[q]; r.S = h[1]; r.S_ema = tm[4]; r.eps = h[2]; r.wdisc = h[3];
    r.gap = h[5]; r.P = tm[0]; r.I = tm[1]; r.D = tm[2]; r.u = tm[3]; r.sigma0 = h[8];
    r.sigma_last = en->h_dbl[SPEC * nc + q];
    r.ms_lanczos = mL; r.ms_svd = mS; r.ms_other = mE;
    r.k_needed = kneed[q]; r.chi_sched = chs[q]; r.fallback = fb[q];
    for (int i = 0; i < 25; ++i) r.feat[i] = en->h_feat[32 * q + i];
  }
  return TNA_OK;
}

}  // namespace tna

// ====================================================================== batch ABI
struct tna_dmrg_batch_s {
  tna_ctx ctx = nullptr;
  tna_engine en = nullptr;
  std::vector<tna_dmrg> ch;
  std::vector<int> nsteps;
  int sweeps_done = 0;
};

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
  for (int i = 0; i < nch; ++i) {
    tna_dmrg dm = nullptr;
    tna_status st = tna_dmrg_create(c, N[i], d, D, W_host[i], A_host[i], chi_init[i], pid, opts, &dm);
    if (st != TNA_OK) {
      for (tna_dmrg x : b->ch) tna_dmrg_destroy(x);
      return st;
    }
    b->ch.push_back(dm);
    b->nsteps.push_back(2 * (N[i] - 1));
  }
  tna_status st = engine_create(nch, &b->en);
  if (st != TNA_OK) {
    for (tna_dmrg x : b->ch) tna_dmrg_destroy(x);
    return st;
  }
  *out = b.release();
  return TNA_OK;
}

tna_status tna_dmrg_batch_sweep(tna_dmrg_batch bt, double *E_out, tna_visit_log *logs, const int64_t *log_offsets,
                                tna_batch_stats *stats) {
  if (!bt) {
    set_error("dmrg_batch_sweep: null handle");
    return TNA_ERR_ARG;
  }
  const int nch = (int)bt->ch.size();
  int maxsteps = 0;
  for (int v : bt->nsteps) maxsteps = std::max(maxsteps, v);
  std::vector<double> E(nch, 0.0);
  tna_status worst = TNA_OK;
  auto t_start = std::chrono::steady_clock::now();
  TNA_HIP(hipStreamSynchronize(bt->ctx->stream));  // work the caller queued on the context stream
  for (int t = 0; t < maxsteps; ++t) {
    std::vector<tna_dmrg> cs;
    std::vector<int> slot, bond, half;
    std::vector<tna_visit_log *> lg;
    for (int i = 0; i < nch; ++i) {
      if (t >= bt->nsteps[i]) continue;
      const int N = bt->ch[i]->N;
      const int h = t < N - 1 ? 0 : 1;
      cs.push_back(bt->ch[i]);
      slot.push_back(i);
      half.push_back(h);
      bond.push_back(h == 0 ? t : (N - 2) - (t - (N - 1)));
      if (logs && log_offsets) lg.push_back(logs + log_offsets[i] + t);
    }
    std::vector<double> Es(cs.size());
    TNA_TRY(engine_step(bt->en, cs, slot, bond, half, Es, lg, &worst));
    for (size_t q = 0; q < cs.size(); ++q) E[slot[q]] = Es[q];
  }
  for (tna_dmrg dm : bt->ch) dm->sweeps_done += 1;
  bt->sweeps_done += 1;
  if (E_out) std::memcpy(E_out, E.data(), sizeof(double) * nch);
  if (stats) {
    engine_stats(bt->en, stats);
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    stats->steps = maxsteps;
  }
  return worst;
}

tna_status tna_dmrg_batch_get_state(tna_dmrg_batch bt, int chain, int *chi, tna_pid_state *pid) {
  if (!bt || chain < 0 || chain >= (int)bt->ch.size()) {
    set_error("dmrg_batch_get_state: bad chain");
    return TNA_ERR_ARG;
  }
  return tna_dmrg_get_state(bt->ch[chain], chi, pid);
}

void tna_dmrg_batch_destroy(tna_dmrg_batch bt) {
  if (!bt) return;
  engine_destroy(bt->en);
  for (tna_dmrg dm : bt->ch) tna_dmrg_destroy(dm);
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

void tna_autotune_clear(void) {
  g_tune.table.clear();
  g_tune.measured = 0;
}

}  // extern "C"
