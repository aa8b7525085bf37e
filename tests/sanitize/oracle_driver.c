/* Sanitizer driver for the oracle (test infrastructure): parse a mechanism
 * file, evaluate the right-hand side and Jacobian, integrate a few cells in
 * every Jacobian mode, and feed malformed texts to the parser.  Built with
 * -fsanitize=address,undefined by tests/test_sanitizers.py. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_mech orc_mech;
typedef struct {
  int max_steps, q_max, fixed_T, fixed_step_n, jac_mode, jac_reuse;
} orc_opts;
typedef struct {
  int status, steps, attempts, n_rhs, n_jac, n_newton, n_etf, n_nnf, n_clip;
  double clip_mass;
} orc_cell_stats;

orc_mech *orc_load(const char *text, char *err, int errlen);
void orc_free(orc_mech *m);
int orc_info(const orc_mech *m, int *S, int *R, int *E);
int orc_rhs(const orc_mech *m, const double *y, double p, int fixed_T, double *f);
int orc_jac(const orc_mech *m, const double *y, double p, int fixed_T, double *J);
int64_t orc_integrate(const orc_mech *m, int64_t n, double *T, double *Y, double p, double dt, double rtol,
                      double atol, const orc_opts *o, orc_cell_stats *stats, int nthreads);

static char *slurp(const char *path) {
  FILE *f = fopen(path, "rb");
  if (!f) return NULL;
  fseek(f, 0, SEEK_END);
  long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  char *b = malloc((size_t)n + 1);
  if (fread(b, 1, (size_t)n, f) != (size_t)n) { fclose(f); free(b); return NULL; }
  b[n] = 0;
  fclose(f);
  return b;
}

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  char *text = slurp(argv[1]);
  if (!text) return 2;
  char err[256];
  orc_mech *m = orc_load(text, err, sizeof err);
  if (!m) { fprintf(stderr, "load failed: %s\n", err); return 1; }
  int S, R, E;
  orc_info(m, &S, &R, &E);
  const int N = S + 1, n = 6;
  double *y = malloc(sizeof(double) * N), *f = malloc(sizeof(double) * N), *J = malloc(sizeof(double) * N * N);
  for (int k = 0; k < S; ++k) y[k] = 1.0 / S;
  y[S] = 1500.0;
  orc_rhs(m, y, 101325.0, 0, f);
  orc_jac(m, y, 101325.0, 0, J);
  double *T = malloc(sizeof(double) * n), *Y = malloc(sizeof(double) * S * n);
  orc_cell_stats *st = malloc(sizeof(orc_cell_stats) * n);
  for (int mode = 0; mode < 3; ++mode)
    for (int reuse = 0; reuse < 2; ++reuse) {
      for (int i = 0; i < n; ++i) {
        T[i] = 1100.0 + 100.0 * i;
        for (int k = 0; k < S; ++k) Y[k * n + i] = 1.0 / S;
      }
      T[n - 1] = -1.0;   /* a bad cell: flagged, not integrated */
      orc_opts o = {100000, 5, 0, 0, mode, reuse};
      int64_t failed = orc_integrate(m, n, T, Y, 101325.0, 1e-7, 1e-8, 1e-12, &o, st, 1);
      if (failed != 1 || st[n - 1].status != 3) { fprintf(stderr, "unexpected failures\n"); return 1; }
    }
  const char *bad[] = {"", "chem-mech 2", "chem-mech 1\nELEMENTS 1\nH 1.008\nSPECIES 1\nA 9 9 9",
                       "chem-mech 1\nELEMENTS 0\n"};
  for (unsigned i = 0; i < sizeof bad / sizeof bad[0]; ++i) {
    orc_mech *b = orc_load(bad[i], err, sizeof err);
    if (b) { fprintf(stderr, "malformed text %u accepted\n", i); return 1; }
  }
  orc_free(m);
  free(text); free(y); free(f); free(J); free(T); free(Y); free(st);
  printf("oracle sanitizer run ok: S=%d R=%d\n", S, R);
  return 0;
}
