/* Drives the library's host-only code for the sanitizer build (no GPU is touched): the rank
 * controllers of Algorithm 2 and Algorithm 1 over long entropy sequences and every parameter form,
 * the MPO builder of every model, the autotuner table files, and the argument checks of the
 * device entry points (which must fail before any HIP call).  Exit status 0 on success; the
 * sanitizers abort on the first error they find. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tna.h"

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

static unsigned long long lcg = 88172645463325252ull;
static double uni(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static void controllers(void) {
  const double gains[3][3] = {{2.0, 0.1, 0.5}, {0.5, 0.05, 0.1}, {0.0, 0.0, 0.0}};
  for (int g = 0; g < 3; ++g)
    for (int form = 0; form < 4; ++form) {
      tna_pid_params p;
      memset(&p, 0, sizeof p);
      p.kp = gains[g][0];
      p.ki = gains[g][1];
      p.kd = gains[g][2];
      p.s_target = 1.0;
      p.alpha = 0.3;
      p.beta = form & 1 ? 0.4 : 0.0;
      p.beta2 = form & 2 ? 0.3 : 0.0;
      p.ema_init_zero = form == 3;
      p.chi_min = 4;
      p.chi_max = 512;
      tna_pid_state st, se;
      memset(&st, 0, sizeof st);
      memset(&se, 0, sizeof se);
      for (int t = 0; t < 20000; ++t) {
        const double s = 6.0 * uni();
        int chi = -1, che = -1;
        double terms[6];
        CHECK(tna_pid_chi_update(&p, &st, s, &chi, (t & 1) ? terms : NULL) == TNA_OK);
        CHECK(chi >= p.chi_min && chi <= p.chi_max);
        CHECK(tna_entropy_chi_update(&p, 1.0 + uni(), &se, s, &che) == TNA_OK);
        CHECK(che >= p.chi_min && che <= p.chi_max);
      }
      int chi = 0;
      CHECK(tna_pid_chi_update(&p, &st, NAN, &chi, NULL) != TNA_OK);
      CHECK(tna_pid_chi_update(&p, &st, INFINITY, &chi, NULL) != TNA_OK);
      CHECK(tna_entropy_chi_update(&p, 0.5, &se, 1.0, &chi) != TNA_OK);
      CHECK(tna_entropy_chi_update(&p, 1.5, &se, NAN, &chi) != TNA_OK);
      CHECK(strlen(tna_last_error()) > 0);
    }
  tna_pid_params bad;
  memset(&bad, 0, sizeof bad);
  bad.chi_min = 10;
  bad.chi_max = 2;
  tna_pid_state st;
  memset(&st, 0, sizeof st);
  int chi = 0;
  CHECK(tna_pid_chi_update(&bad, &st, 1.0, &chi, NULL) != TNA_OK);
  CHECK(tna_pid_chi_update(NULL, &st, 1.0, &chi, NULL) != TNA_OK);
  CHECK(tna_entropy_chi_update(&bad, 2.0, NULL, 1.0, &chi) != TNA_OK);
}

static void mpos(void) {
  const double prm[3][3] = {{1.0, 1.5, 0.2}, {1.0, 0.241, 0.0}, {1.0, 0.7, 0.0}};
  const int Ns[4] = {2, 3, 8, 33};
  for (int model = 0; model < 3; ++model)
    for (int i = 0; i < 4; ++i) {
      const int N = Ns[i], Dmax = 8;
      double *W = (double *)malloc(sizeof(double) * (size_t)N * Dmax * Dmax * 4);
      int D = 0;
      CHECK(tna_mpo_build(model, N, prm[model], W, &D) == TNA_OK);
      CHECK(D >= 3 && D <= Dmax);
      double s = 0.0;
      for (size_t e = 0; e < (size_t)N * D * D * 4; ++e) s += fabs(W[e]);
      CHECK(isfinite(s) && s > 0.0);
      free(W);
    }
  int D = 0;
  double W[64];
  CHECK(tna_mpo_build(7, 4, NULL, W, &D) != TNA_OK);
  CHECK(tna_mpo_build(0, 1, NULL, W, &D) != TNA_OK);
}

static void tables(const char *dir) {
  char path[4096];
  snprintf(path, sizeof path, "%s/tune.txt", dir);
  tna_autotune_clear();
  CHECK(tna_autotune_entries() == 0);
  CHECK(tna_autotune_save(path) == TNA_OK);
  CHECK(tna_autotune_load(path) == TNA_OK);
  FILE *f = fopen(path, "w");
  if (f) {
    fputs("garbage that is not a table\n\x01\x02 1 2 3\n", f);
    fclose(f);
  }
  (void)tna_autotune_load(path);  /* rejected or read as empty: no crash either way */
  snprintf(path, sizeof path, "%s/does/not/exist.txt", dir);
  CHECK(tna_autotune_load(path) != TNA_OK);
  tna_autotune_clear();
}

static void argument_checks(void) {
  double x[16] = {0};
  CHECK(tna_heff_apply(NULL, 4, 4, 2, 5, x, x, x, x, x, x, 0) != TNA_OK);
  double S[4], spec[32];
  int k = 0, sw = 0;
  CHECK(tna_svd_truncate(NULL, 4, 4, TNA_F64, x, 2, S, x, x, spec, &k, &sw) != TNA_OK);
  size_t bytes = 0;
  CHECK(tna_heff_apply_noalloc_bytes(64, 64, 2, 5, TNA_HEFF_F64, &bytes) == TNA_OK && bytes > 0);
  CHECK(tna_heff_apply_noalloc_bytes(-1, 64, 2, 5, TNA_HEFF_F64, &bytes) != TNA_OK);
  CHECK(tna_destroy(NULL) == TNA_OK);
  CHECK(strlen(tna_last_error()) > 0);
}

int main(int argc, char **argv) {
  controllers();
  mpos();
  tables(argc > 1 ? argv[1] : ".");
  argument_checks();
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("host driver: all checks passed\n");
  return 0;
}
