// Device-resident two-site DMRG (Sec. 10 of the paper) with one EMA+PID bond
// controller per bond (Algorithm 2, Sec. 6).  The MPS tensors, environments,
// Lanczos basis and SVD work buffers live in device memory for the whole run;
// per bond visit the host reads back only the Lanczos coefficients and the
// entropy of the two-site spectrum.
#include <hip/hip_runtime.h>

#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include "internal.h"

using namespace tna;

static tna_status check_dmrg_args(int N, int d, int D, const double *W, const double *A, const int *chi,
                                  const tna_pid_params *pid) {
  if (N < 2 || d < 1 || D < 1 || !W || !A || !chi || !pid) {
    set_error("dmrg_create: bad arguments");
    return TNA_ERR_ARG;
  }
  if (D * d * d > 32) {
    set_error("dmrg_create: D*d*d must be <= 32");
    return TNA_ERR_ARG;
  }
  if (pid->chi_min < 1 || pid->chi_max < pid->chi_min) {
    set_error("dmrg_create: need 1 <= chi_min <= chi_max");
    return TNA_ERR_ARG;
  }
  for (int b = 0; b < N - 1; ++b) {
    const int cl = b == 0 ? 1 : chi[b - 1];
    if (chi[b] < 1 || cl > d * chi[b] || chi[b] > d * cl) {
      set_error("dmrg_create: inconsistent initial bond dimensions");
      return TNA_ERR_ARG;
    }
  }
  return TNA_OK;
}

// Runs the Jacobi SVD of the m x n matrix src and sorts its spectrum into
// dm->S; *mat keeps the plan and work bindings for svd_finish.
static tna_status svd_start(tna_dmrg dm, int m, int n, const double *src, SvdMat *mat, int *sweeps) {
  tna_ctx c = dm->ctx;
  SvdMat a;
  // Vt becomes the right-canonical tensor (from the rotations when the shape allows), U S the left one
  TNA_TRY(svd_plan_mat(m, n, TNA_F64, 1, &a, 2));
  a.rows_scaled = a.trans;
  const size_t nd = svd_work_doubles(a), ni = svd_work_ints(a);
  TNA_TRY(c->svd.work_d.ensure(sizeof(double) * nd));
  TNA_TRY(c->svd.work_i.ensure(sizeof(int) * ni));
  TNA_TRY(dm->S.ensure(sizeof(double) * a.R));
  svd_bind_work(&a, c->svd.work_d.as<double>(), c->svd.work_i.as<int>());
  a.A = src;
  a.S = dm->S.as<double>();
  a.spec = dm->spec.as<double>();
  a.eps_target = dm->opts.eps_target > 0 ? dm->opts.eps_target : 1e-8;
  a.out_type = TNA_F64;
  std::vector<SvdMat> mats{a};
  std::vector<int> sw;
  tna_status st = svd_group_run(mats, c->svd, dm->opts.svd_max_sweeps, sw, c->stream);
  *mat = mats[0];
  if (sweeps) *sweeps = sw.empty() ? 0 : sw[0];
  return st;
}

// Writes the kept k vectors into U (m x k) and Vt (k x n) with scale_mode.
static tna_status svd_finish(tna_dmrg dm, SvdMat mat, int k, void *U, void *Vt, int scale_mode) {
  mat.k = k;
  mat.U = U;
  mat.Vt = Vt;
  mat.scale_mode = scale_mode;
  std::vector<SvdMat> mats{mat};
  return svd_group_outputs(mats, dm->ctx->svd, dm->ctx->stream);
}

extern "C" {

tna_status tna_dmrg_create(tna_ctx c, int N, int d, int D, const double *W_host, const double *A_host,
                           const int *chi_init, const tna_pid_params *pid, const tna_dmrg_opts *opts, tna_dmrg *out) {
  if (!c || !out) {
    set_error("dmrg_create: null context/out");
    return TNA_ERR_ARG;
  }
  TNA_TRY(check_dmrg_args(N, d, D, W_host, A_host, chi_init, pid));
  auto dm = std::make_unique<tna_dmrg_s>();
  dm->ctx = c;
  dm->N = N; dm->d = d; dm->D = D;
  dm->pid = *pid;
  tna_dmrg_opts o{};
  if (opts) o = *opts;
  if (!(o.lanczos_tol > 0)) o.lanczos_tol = 1e-12;
  if (o.lanczos_kmax <= 0) o.lanczos_kmax = 100;
  if (o.lanczos_restarts < 0) o.lanczos_restarts = 5;
  if (o.svd_max_sweeps <= 0) o.svd_max_sweeps = 60;
  if (o.heff_prec < 0 || o.heff_prec > 1) {
    set_error("dmrg_create: heff_prec must be F64 or F32");
    return TNA_ERR_ARG;
  }
  if (o.chi_rule < TNA_CHI_PID || o.chi_rule > TNA_CHI_ENTROPY ||
      (o.chi_rule == TNA_CHI_THRESHOLD && !(o.rule_param > 0.0)) ||
      (o.chi_rule == TNA_CHI_ENTROPY && !(o.rule_param >= 1.0))) {
    set_error("dmrg_create: chi_rule needs eps_trunc > 0 (threshold) or gamma >= 1 (entropy)");
    return TNA_ERR_ARG;
  }
  dm->opts = o;
  dm->chi.assign(chi_init, chi_init + N - 1);
  dm->st.assign(N - 1, tna_pid_state{0, 0, 0, 0, pid->chi_min, 0});
  dm->A.resize(N);
  dm->Le.resize(N);
  dm->Re.resize(N);
  hipStream_t s = c->stream;
  TNA_HIP(hipHostMalloc((void **)&dm->host_stage, sizeof(double) * 64, hipHostMallocDefault));
  dm->hist.assign(N - 1, std::array<double, 8>{});
  dm->nhist.assign(N - 1, 0);
  dm->pred.assign(N - 1, 0);
  // MPO and mixing matrices
  const size_t wsz = (size_t)D * D * d * d;
  TNA_TRY(dm->W.ensure(sizeof(double) * wsz * N));
  TNA_HIP(hipMemcpy(dm->W.ptr, W_host, sizeof(double) * wsz * N, hipMemcpyHostToDevice));
  const int I2 = D * d * d, I1 = D * d;
  TNA_TRY(dm->M12.ensure(sizeof(double) * I2 * I2 * (N - 1)));
  TNA_TRY(dm->Ml.ensure(sizeof(double) * I1 * I1 * N));
  TNA_TRY(dm->Mr.ensure(sizeof(double) * I1 * I1 * N));
  const double *Wd = dm->W.as<double>();
  for (int b = 0; b < N - 1; ++b)
    TNA_TRY(build_mix_matrix(0, d, D, Wd + wsz * b, Wd + wsz * (b + 1), dm->M12.as<double>() + (size_t)I2 * I2 * b, s));
  for (int i = 0; i < N; ++i) {
    TNA_TRY(build_mix_matrix(1, d, D, Wd + wsz * i, nullptr, dm->Ml.as<double>() + (size_t)I1 * I1 * i, s));
    TNA_TRY(build_mix_matrix(2, d, D, Wd + wsz * i, nullptr, dm->Mr.as<double>() + (size_t)I1 * I1 * i, s));
  }
  // site tensors
  size_t off = 0;
  for (int i = 0; i < N; ++i) {
    const size_t n = (size_t)dm->CL(i) * d * dm->CR(i);
    TNA_TRY(dm->A[i].ensure(sizeof(double) * n));
    TNA_HIP(hipMemcpy(dm->A[i].ptr, A_host + off, sizeof(double) * n, hipMemcpyHostToDevice));
    off += n;
  }
  TNA_TRY(dm->spec.ensure(sizeof(double) * 32));
  // right-canonicalise on the device: A_b = U S Vt -> A_b <- Vt, A_{b-1} <- A_{b-1} U S
  DevBuf Ub, Vb, Tb;
  for (int b = N - 1; b >= 1; --b) {
    const int m = dm->chi[b - 1], n = d * dm->CR(b);
    const int R = std::min(m, n);
    TNA_TRY(Ub.ensure(sizeof(double) * m * R));
    TNA_TRY(Vb.ensure(sizeof(double) * R * n));
    int sw = 0;
    SvdMat mat;
    tna_status st = svd_start(dm.get(), m, n, dm->A[b].as<double>(), &mat, &sw);
    if (st != TNA_OK && st != TNA_ERR_NOCONV) return st;  // a capped sweep count still gives a valid gauge
    const int k = R;
    TNA_TRY(svd_finish(dm.get(), mat, k, Ub.ptr, Vb.ptr, 2));
    const int ml = dm->CL(b - 1) * d;
    TNA_TRY(Tb.ensure(sizeof(double) * ml * k));
    GemmArgs g{};
    g.M = ml; g.N = k; g.K = m;
    g.A = dm->A[b - 1].ptr; g.lda = m; g.B = Ub.ptr; g.ldb = k; g.C = Tb.ptr; g.ldc = k;
    g.alpha = 1.0; g.batch = 1; g.compute = G_F64;
    TNA_TRY(gemm(g, s));
    TNA_TRY(dm->A[b - 1].ensure(sizeof(double) * ml * k));
    TNA_HIP(hipMemcpyAsync(dm->A[b - 1].ptr, Tb.ptr, sizeof(double) * ml * k, hipMemcpyDeviceToDevice, s));
    TNA_TRY(dm->A[b].ensure(sizeof(double) * k * n));
    TNA_HIP(hipMemcpyAsync(dm->A[b].ptr, Vb.ptr, sizeof(double) * k * n, hipMemcpyDeviceToDevice, s));
    dm->chi[b - 1] = k;
  }
  {
    const int64_t n0 = (int64_t)d * dm->CR(0);
    double *nr = c->misc.as<double>() + 512;
    TNA_TRY(norm2(dm->A[0].as<double>(), n0, nr, c->part.as<double>(), s));
    TNA_TRY(scale(dm->A[0].as<double>(), dm->A[0].as<double>(), n0, nr, 0.0, s));
  }
  Ub.release(); Vb.release(); Tb.release();
  // boundary environments and the right environments of the canonical MPS
  std::vector<double> bnd(D, 0.0);
  bnd[D - 1] = 1.0;
  TNA_TRY(dm->Le[0].ensure(sizeof(double) * D));
  TNA_HIP(hipMemcpy(dm->Le[0].ptr, bnd.data(), sizeof(double) * D, hipMemcpyHostToDevice));
  std::fill(bnd.begin(), bnd.end(), 0.0);
  bnd[0] = 1.0;
  TNA_TRY(dm->Re[N - 1].ensure(sizeof(double) * D));
  TNA_HIP(hipMemcpy(dm->Re[N - 1].ptr, bnd.data(), sizeof(double) * D, hipMemcpyHostToDevice));
  for (int i = N - 1; i >= 2; --i) {
    const int k = dm->CL(i), cr = dm->CR(i);
    TNA_TRY(dm->T1.ensure(sizeof(double) * (size_t)cr * D * k * d));
    TNA_TRY(dm->T2.ensure(sizeof(double) * (size_t)cr * D * k * d));
    TNA_TRY(dm->Re[i - 1].ensure(sizeof(double) * (size_t)k * D * k));
    TNA_TRY(env_right(k, cr, d, D, dm->Re[i].as<double>(), dm->Mr.as<double>() + (size_t)I1 * I1 * i,
                           dm->A[i].as<double>(), dm->T1.as<double>(), dm->T2.as<double>(), dm->Re[i - 1].as<double>(),
                           s));
  }
  TNA_HIP(hipStreamSynchronize(s));
  c->children += 1;
  *out = dm.release();
  return TNA_OK;
}

tna_status tna_dmrg_sweep(tna_dmrg dm, double *E_out, tna_visit_log *log) {
  if (!dm) {
    set_error("dmrg_sweep: null handle");
    return TNA_ERR_ARG;
  }
  if (dm->centre != 0) {
    set_error("dmrg_sweep: the orthogonality centre must be at site 0 (single visits moved it)");
    return TNA_ERR_ARG;
  }
  if (!dm->engine) TNA_TRY(engine_create(1, &dm->engine));
  TNA_HIP(hipStreamSynchronize(dm->ctx->stream));  // work the caller queued on the context stream
  const int N = dm->N;
  tna_status worst = TNA_OK;
  double E = 0.0;
  std::vector<tna_dmrg> cs{dm};
  std::vector<int> slot{0}, bond{0}, half{0};
  std::vector<double> Es(1, 0.0);
  std::vector<tna_visit_log *> lg(log ? 1 : 0, nullptr);
  // TNA_PROGRESS set: a line on stderr at most every 20 s, for long sweeps at large bond dimension
  const bool progress = std::getenv("TNA_PROGRESS") != nullptr;
  auto last = std::chrono::steady_clock::now();
  for (int h = 0; h < 2; ++h)
    for (int step = 0; step < N - 1; ++step) {
      bond[0] = h == 0 ? step : N - 2 - step;
      half[0] = h;
      if (log) lg[0] = log + h * (N - 1) + step;
      TNA_TRY(engine_step(dm->engine, cs, slot, bond, half, Es, lg, &worst));
      dm->centre = h == 0 ? bond[0] + 1 : bond[0];
      E = Es[0];
      if (progress) {
        const auto now = std::chrono::steady_clock::now();
        if (std::chrono::duration<double>(now - last).count() > 20.0) {
          std::fprintf(stderr, "[tna] sweep %d half %d bond %d chi %d E %.12f\n", dm->sweeps_done, h, bond[0],
                       dm->chi[bond[0]], E);
          std::fflush(stderr);
          last = now;
        }
      }
    }
  dm->sweeps_done += 1;
  if (E_out) *E_out = E;
  return worst;
}

tna_status tna_dmrg_visit(tna_dmrg dm, int bond, int dir, double *E_out, tna_visit_log *log) {
  if (!dm || bond < 0 || bond > dm->N - 2 || (dir != 0 && dir != 1)) {
    set_error("dmrg_visit: bad handle, bond or direction");
    return TNA_ERR_ARG;
  }
  if (dm->centre != (dir == 0 ? bond : bond + 1)) {
    set_error("dmrg_visit: a left-to-right visit of bond b needs the orthogonality centre on site b, a "
              "right-to-left one on site b+1");
    return TNA_ERR_ARG;
  }
  if (!dm->engine) TNA_TRY(engine_create(1, &dm->engine));
  TNA_HIP(hipStreamSynchronize(dm->ctx->stream));
  tna_status worst = TNA_OK;
  std::vector<tna_dmrg> cs{dm};
  std::vector<int> slot{0}, bd{bond}, half{dir};
  std::vector<double> Es(1, 0.0);
  std::vector<tna_visit_log *> lg(log ? 1 : 0, log);
  TNA_TRY(engine_step(dm->engine, cs, slot, bd, half, Es, lg, &worst));
  dm->centre = dir == 0 ? bond + 1 : bond;
  if (E_out) *E_out = Es[0];
  return worst;
}

int tna_dmrg_centre(tna_dmrg dm) { return dm ? dm->centre : -1; }

tna_status tna_dmrg_get_stats(tna_dmrg dm, tna_batch_stats *out) {
  if (!dm || !out) {
    set_error("dmrg_get_stats: null argument");
    return TNA_ERR_ARG;
  }
  std::memset(out, 0, sizeof *out);
  if (dm->engine) engine_stats(dm->engine, out);
  out->steps = dm->sweeps_done;
  return TNA_OK;
}

tna_status tna_dmrg_get_env(tna_dmrg dm, int side, int site, double *dst, size_t capacity, size_t *count) {
  if (!dm || (side != 0 && side != 1) || site < 0 || site >= dm->N) {
    set_error("dmrg_get_env: bad handle, side or site");
    return TNA_ERR_ARG;
  }
  // left environment of site i: sites 0..i-1, valid for i <= centre; right one: sites i+1..N-1, i >= centre
  if (side == 0 ? site > dm->centre : site < dm->centre) {
    set_error("dmrg_get_env: that environment is not current (wrong side of the orthogonality centre)");
    return TNA_ERR_ARG;
  }
  const size_t chi = side == 0 ? (size_t)dm->CL(site) : (size_t)dm->CR(site);
  const size_t n = chi * dm->D * chi;
  if (count) *count = n;
  if (!dst) return TNA_OK;
  if (capacity < n) {
    set_error("dmrg_get_env: capacity too small");
    return TNA_ERR_ARG;
  }
  if (dm->engine) TNA_HIP(hipStreamSynchronize(engine_stream(dm->engine)));
  const tna::DevBuf &src = side == 0 ? dm->Le[site] : dm->Re[site];
  TNA_HIP(hipMemcpyAsync(dst, src.ptr, sizeof(double) * n, hipMemcpyDefault, dm->ctx->stream));
  TNA_HIP(hipStreamSynchronize(dm->ctx->stream));
  return TNA_OK;
}

tna_status tna_dmrg_get_state(tna_dmrg dm, int *chi, tna_pid_state *pid) {
  if (!dm) {
    set_error("dmrg_get_state: null handle");
    return TNA_ERR_ARG;
  }
  if (chi) std::memcpy(chi, dm->chi.data(), sizeof(int) * (dm->N - 1));
  if (pid) std::memcpy(pid, dm->st.data(), sizeof(tna_pid_state) * (dm->N - 1));
  return TNA_OK;
}

tna_status tna_dmrg_get_mps(tna_dmrg dm, double *A_host, size_t capacity, size_t *count) {
  if (!dm) {
    set_error("dmrg_get_mps: null handle");
    return TNA_ERR_ARG;
  }
  size_t total = 0;
  for (int i = 0; i < dm->N; ++i) total += (size_t)dm->CL(i) * dm->d * dm->CR(i);
  if (count) *count = total;
  if (!A_host) return TNA_OK;
  if (capacity < total) {
    set_error("dmrg_get_mps: capacity too small");
    return TNA_ERR_ARG;
  }
  TNA_HIP(hipStreamSynchronize(dm->ctx->stream));
  size_t off = 0;
  for (int i = 0; i < dm->N; ++i) {
    const size_t n = (size_t)dm->CL(i) * dm->d * dm->CR(i);
    TNA_HIP(hipMemcpy(A_host + off, dm->A[i].ptr, sizeof(double) * n, hipMemcpyDeviceToHost));
    off += n;
  }
  return TNA_OK;
}

// Checkpoint: magic, sizes, MPO, controller parameters and options, bond dimensions,
// site tensors, per-bond controller states and scheduler history, sweeps done.  Loading
// recreates the run from the saved MPS (canonicalisation and environments as at create),
// then restores the controller and scheduler state, so a resumed run continues the same
// controller trajectory.
static const char kMagic[8] = {'T', 'N', 'A', 'D', 'M', 'R', 'G', '1'};

tna_status tna_dmrg_save(tna_dmrg dm, const char *path) {
  if (!dm || !path) {
    set_error("dmrg_save: null argument");
    return TNA_ERR_ARG;
  }
  size_t count = 0;
  TNA_TRY(tna_dmrg_get_mps(dm, nullptr, 0, &count));
  std::vector<double> A(count);
  TNA_TRY(tna_dmrg_get_mps(dm, A.data(), count, &count));
  const int N = dm->N, d = dm->d, D = dm->D;
  const size_t wsz = (size_t)D * D * d * d * N;
  std::vector<double> W(wsz);
  TNA_HIP(hipMemcpy(W.data(), dm->W.ptr, sizeof(double) * wsz, hipMemcpyDeviceToHost));
  FILE *f = std::fopen(path, "wb");
  if (!f) {
    set_error(std::string("dmrg_save: cannot open ") + path);
    return TNA_ERR_ARG;
  }
  const int32_t head[4] = {N, d, D, dm->sweeps_done};
  const uint64_t na = count;
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(head, sizeof(head), 1, f) == 1 &&
            std::fwrite(&na, sizeof(na), 1, f) == 1 && std::fwrite(W.data(), sizeof(double), wsz, f) == wsz &&
            std::fwrite(&dm->pid, sizeof(dm->pid), 1, f) == 1 && std::fwrite(&dm->opts, sizeof(dm->opts), 1, f) == 1 &&
            std::fwrite(dm->chi.data(), sizeof(int), N - 1, f) == (size_t)(N - 1) &&
            std::fwrite(A.data(), sizeof(double), count, f) == count &&
            std::fwrite(dm->st.data(), sizeof(tna_pid_state), N - 1, f) == (size_t)(N - 1) &&
            std::fwrite(dm->hist.data(), sizeof(double) * 8, N - 1, f) == (size_t)(N - 1) &&
            std::fwrite(dm->nhist.data(), sizeof(int), N - 1, f) == (size_t)(N - 1) &&
            std::fwrite(dm->pred.data(), sizeof(int), N - 1, f) == (size_t)(N - 1);
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) {
    set_error(std::string("dmrg_save: write failed on ") + path);
    return TNA_ERR_ARG;
  }
  return TNA_OK;
}

tna_status tna_dmrg_load(tna_ctx ctx, const char *path, tna_dmrg *out) {
  if (!ctx || !path || !out) {
    set_error("dmrg_load: null argument");
    return TNA_ERR_ARG;
  }
  FILE *f = std::fopen(path, "rb");
  if (!f) {
    set_error(std::string("dmrg_load: cannot open ") + path);
    return TNA_ERR_ARG;
  }
  auto fail = [&](const char *what) {
    std::fclose(f);
    set_error(std::string("dmrg_load: ") + what + " in " + path);
    return TNA_ERR_ARG;
  };
  char magic[8];
  int32_t head[4];
  uint64_t na = 0;
  if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, kMagic, 8) != 0) return fail("not a checkpoint");
  if (std::fread(head, sizeof(head), 1, f) != 1 || std::fread(&na, sizeof(na), 1, f) != 1) return fail("short header");
  const int N = head[0], d = head[1], D = head[2];
  if (N < 2 || N > 100000 || d < 1 || d > 16 || D < 1 || D > 64 || na > ((uint64_t)1 << 40)) return fail("bad sizes");
  const size_t wsz = (size_t)D * D * d * d * N;
  std::vector<double> W(wsz), A(na);
  tna_pid_params pid;
  tna_dmrg_opts opts;
  std::vector<int> chi(N - 1), nhist(N - 1), pred(N - 1);
  std::vector<tna_pid_state> st(N - 1);
  std::vector<std::array<double, 8>> hist(N - 1);
  if (std::fread(W.data(), sizeof(double), wsz, f) != wsz || std::fread(&pid, sizeof(pid), 1, f) != 1 ||
      std::fread(&opts, sizeof(opts), 1, f) != 1 || std::fread(chi.data(), sizeof(int), N - 1, f) != (size_t)(N - 1) ||
      std::fread(A.data(), sizeof(double), na, f) != na ||
      std::fread(st.data(), sizeof(tna_pid_state), N - 1, f) != (size_t)(N - 1) ||
      std::fread(hist.data(), sizeof(double) * 8, N - 1, f) != (size_t)(N - 1) ||
      std::fread(nhist.data(), sizeof(int), N - 1, f) != (size_t)(N - 1) ||
      std::fread(pred.data(), sizeof(int), N - 1, f) != (size_t)(N - 1))
    return fail("truncated file");
  std::fclose(f);
  size_t need = 0;
  for (int i = 0; i < N; ++i) {
    const size_t cl = i == 0 ? 1 : chi[i - 1], cr = i == N - 1 ? 1 : chi[i];
    need += cl * d * cr;
  }
  if (need != na) {
    set_error(std::string("dmrg_load: site tensors do not match the bond dimensions in ") + path);
    return TNA_ERR_ARG;
  }
  tna_dmrg dm = nullptr;
  TNA_TRY(tna_dmrg_create(ctx, N, d, D, W.data(), A.data(), chi.data(), &pid, &opts, &dm));
  dm->st = st;
  dm->hist = hist;
  dm->nhist = nhist;
  dm->pred = pred;
  dm->sweeps_done = head[3];
  *out = dm;
  return TNA_OK;
}

tna_status tna_dmrg_set_scheduler(tna_dmrg dm, tna_mlp net) {
  if (!dm) {
    set_error("dmrg_set_scheduler: null handle");
    return TNA_ERR_ARG;
  }
  // proposals pending from a previous network are dropped; a run fresh from a checkpoint keeps the
  // saved ones for the network that is attached again
  if (dm->sched) std::fill(dm->pred.begin(), dm->pred.end(), 0);
  dm->sched = net;
  return TNA_OK;
}

void tna_dmrg_destroy(tna_dmrg dm) {
  if (!dm) return;
  (void)hipStreamSynchronize(dm->ctx->stream);
  for (auto &b : dm->A) b.release();
  for (auto &b : dm->Le) b.release();
  for (auto &b : dm->Re) b.release();
  for (DevBuf *b : {&dm->W, &dm->M12, &dm->Ml, &dm->Mr, &dm->V, &dm->T1, &dm->T2, &dm->spec, &dm->S}) b->release();
  if (dm->host_stage) (void)hipHostFree(dm->host_stage);
  engine_destroy(dm->engine);
  dm->ctx->children -= 1;
  delete dm;
}

}  // extern "C"
