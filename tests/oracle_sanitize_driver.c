/* Test support: calls every entry point of the FP64 oracle once on a small system, so
 * that tests/test_oracle_sanitize.py can run the oracle built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (the oracle is otherwise loaded through ctypes, where the
 * sanitizers cannot be attached).
 *
 * argv[1]: model file; argv[2]: system file, little-endian
 *   int64 n, double coords[3 n], double box[9], int32 types[n], int64 nt, double mass[nt]
 * Prints the energy and a force checksum; exit status 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct or_model or_model;
or_model *or_load(const char *path);
void or_free(or_model *m);
void or_set_threads(int n);
int or_info(const or_model *m, int32_t *ntypes, int32_t *nm, int32_t *M, int32_t *m2, double *rc,
            int64_t *nparams);
int or_get_params(const or_model *m, double *out);
int or_set_params(or_model *m, const double *in);
int or_nlist(const or_model *m, int64_t n, const double *coords, const int32_t *types, const double *box,
             int64_t ncent, const int64_t *cent, int32_t *nlist, int32_t *img, int32_t *nnei, int32_t *overflow);
int or_eval(const or_model *m, int64_t n, const double *coords, const int32_t *types, const double *box, double *E,
            double *F, double *W, double *Ei, double *T, double *D, double *gT);
int or_eval_atomic(const or_model *m, int64_t n, const double *coords, const int32_t *types, const double *box,
                   double *E, double *F, double *W, double *Ei, double *Wi);
int or_eval_sampled(const or_model *m, int64_t n, const double *coords, const int32_t *types, const double *box,
                    int64_t ns, const int64_t *samp, double *Ei_out, double *F_out);
int or_md(const or_model *m, int64_t n, double *x, double *v, const int32_t *types, const double *mass,
          const double *box, double dt, int nsteps, int thermo_every, double *thermo);
int or_md_npt(const or_model *m, int64_t n, double *x, double *v, const int32_t *types, const double *mass,
              double *box, double pext_bar, double tau_p, double temp, double tau_t, double dt, int nsteps,
              int thermo_every, double *thermo, double *state);

static int rd(FILE *f, void *p, size_t bytes) { return fread(p, 1, bytes, f) == bytes ? 0 : -1; }

int main(int argc, char **argv) {
  if (argc < 3) return 2;
  or_model *m = or_load(argv[1]);
  if (!m) return 3;
  FILE *f = fopen(argv[2], "rb");
  if (!f) return 3;
  int64_t n = 0, nt = 0;
  if (rd(f, &n, 8) || n < 2) return 3;
  double *x = malloc(24 * n), box[9];
  int32_t *t = malloc(4 * n);
  if (rd(f, x, 24 * n) || rd(f, box, 72) || rd(f, t, 4 * n) || rd(f, &nt, 8) || nt < 1) return 3;
  double *mass = malloc(8 * nt);
  if (rd(f, mass, 8 * nt)) return 3;
  fclose(f);
  or_set_threads(2);

  int32_t ntypes, nm, M, m2;
  double rc;
  int64_t np;
  or_info(m, &ntypes, &nm, &M, &m2, &rc, &np);
  double *theta = malloc(8 * np);
  or_get_params(m, theta);
  or_set_params(m, theta);

  int64_t *cent = malloc(8 * n);
  for (int64_t i = 0; i < n; i++) cent[i] = i;
  int32_t *nl = malloc(4 * n * nm), *img = malloc(4 * n * nm), *nnei = malloc(4 * n * ntypes), ovf = 0;
  if (or_nlist(m, n, x, t, box, n, cent, nl, img, nnei, &ovf) < 0) return 4;

  double E = 0, E2 = 0, W[9];
  double *F = malloc(24 * n), *Ei = malloc(8 * n), *Wi = malloc(72 * n);
  double *T = malloc(8 * n * M * 4), *D = malloc(8 * n * M * m2), *gT = malloc(8 * n * M * 4);
  if (or_eval(m, n, x, t, box, &E, F, W, Ei, T, D, gT) < 0) return 5;
  if (or_eval_atomic(m, n, x, t, box, &E2, F, W, Ei, Wi) < 0) return 6;
  int64_t samp[2] = {0, n - 1};
  double Es[2], Fs[6];
  if (or_eval_sampled(m, n, x, t, box, 2, samp, Es, Fs) < 0) return 7;

  double *xx = malloc(24 * n), *v = calloc(3 * n, 8), th[2 * 6], thn[2 * 8], st[3] = {0, 0, 0}, box2[9];
  memcpy(xx, x, 24 * n);
  if (or_md(m, n, xx, v, t, mass, box, 0.5, 3, 3, th) < 0) return 8;
  memcpy(xx, x, 24 * n);
  memset(v, 0, 24 * n);
  memcpy(box2, box, 72);
  if (or_md_npt(m, n, xx, v, t, mass, box2, 1.0e4, 100.0, 300.0, 25.0, 0.5, 3, 3, thn, st) < 0) return 9;

  double fs = 0;
  for (int64_t i = 0; i < 3 * n; i++) fs += F[i] * (double)(i % 7 + 1);
  printf("E %.17g %.17g Fsum %.17g\n", E, E2, fs);
  free(x); free(t); free(mass); free(theta); free(cent); free(nl); free(img); free(nnei);
  free(F); free(Ei); free(Wi); free(T); free(D); free(gT); free(xx); free(v);
  or_free(m);
  return 0;
}
