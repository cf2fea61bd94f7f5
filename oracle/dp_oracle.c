/*
 * Plain FP64 CPU oracle for the Deep Potential smooth-edition (DP-SE) model of
 * "86 PFLOPS Deep Potential Molecular Dynamics simulation of 100 million atoms with
 * ab initio accuracy" (arXiv 2004.11658).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no code with the HIP library: it has its
 * own model-file parser, neighbour search, network code and adjoint.
 *
 * Everything is written the slow, obvious way: loops over atoms, over every periodic
 * image of every atom, over neighbour slots and over matrix entries, in double
 * precision, following the paper's definitions in order:
 *   Section 2, Eq. (1)   E = sum_i E_i,  E_i = N(D(R_i))
 *   Section 2, Eq. (2-3) fitting net with skip connections
 *   Section 2, Eq. (4)   descriptor  D = (G<)^T R R^T G   (stored as the M x M< transpose)
 *   Section 2, Eq. (5)   environment-matrix row s(r)(1, x/r, y/r, z/r), zero padding
 *   Section 2, Eq. (6-9) embedding net, first layer plain tanh, later layers (x,x)+tanh
 *   Section 2, Remark 1  one fitting net per species, one embedding net per species pair
 *   Section 2, Remark 2, Eq. (10)  F_i = -grad_{r_i} E, obtained by back propagation
 *   Section 3.2.2, Alg. 1 formatted neighbour list: sort by (neighbour type, distance,
 *                         index), pad every type block to its fixed width
 *   Section 3.2.2, Alg. 2 environment matrix from the formatted list, pads -> 0
 *   Section 3.1          ghost (image) atoms within rc; forces on images go to owners
 *   Section 4            velocity-Verlet integration
 *
 * Readings where the paper is silent (they bind the GPU library too):
 *   - normalisation T = G^T R / N_m (model flag desc_norm = 0; 1 disables it)
 *   - switch w(r): C2 quintic u^3(-6u^2+15u-10)+1 between rcs and rc (or cosine)
 *   - neighbours r < rc; every periodic image within rc, including self images
 *   - sort key (type, r^2 exactly, owner index, image code), no quantisation;
 *     image code ((n0+K0)(2K1+1) + n1+K1)(2K2+1) + n2+K2, K_k = ceil(rc / width_k)
 *   - a type block with more than sel neighbours keeps the nearest sel (flagged)
 *   - fitting layers: identity skip iff square, plain tanh otherwise; output affine
 *   - embedding layers k >= 1: concat skip iff width doubles, identity iff equal
 *   - virial W_ab = -sum_pairs d_a dE/dd_b  (= -dE/d(eps_ab) for x -> x (I + eps))
 *
 * Floating-point decisions that pick an integer (inside rc, order of neighbours) use
 * r^2 = (dx*dx + dy*dy) + dz*dz of d = (x_j,wrapped + n.B) - x_i,wrapped, evaluated in
 * exactly this order with contraction off (compile with -ffp-contract=off).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXL 8
#define OR_MAXT 8

typedef struct {
  int ntypes, n_emb, n_fit, m2, switch_kind, desc_norm;
  double rc, rcs;
  int emb_w[OR_MAXL], fit_w[OR_MAXL], sel[OR_MAXT];
  int64_t nparams;
  double *p;
  int nm, M;
  int sel_off[OR_MAXT + 1];
  int64_t eW[OR_MAXT * OR_MAXT][OR_MAXL], eB[OR_MAXT * OR_MAXT][OR_MAXL];
  int64_t fW[OR_MAXT][OR_MAXL + 1], fB[OR_MAXT][OR_MAXL + 1];
  char err[256];
} or_model;

static int g_threads = 1;
void or_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int or_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------------------------ */
/* model file                                                                            */
/* ------------------------------------------------------------------------------------ */

static int32_t rd_i32(const unsigned char *b) { int32_t v; memcpy(&v, b, 4); return v; }
static int64_t rd_i64(const unsigned char *b) { int64_t v; memcpy(&v, b, 8); return v; }
static double rd_f64(const unsigned char *b) { double v; memcpy(&v, b, 8); return v; }

static void layout(or_model *m) {
  int64_t off = 0;
  for (int a = 0; a < m->ntypes; a++)
    for (int b = 0; b < m->ntypes; b++) {
      int nin = 1;
      for (int k = 0; k < m->n_emb; k++) {
        m->eW[a * m->ntypes + b][k] = off; off += (int64_t)nin * m->emb_w[k];
        m->eB[a * m->ntypes + b][k] = off; off += m->emb_w[k];
        nin = m->emb_w[k];
      }
    }
  for (int a = 0; a < m->ntypes; a++) {
    int nin = m->M * m->m2;
    for (int k = 0; k < m->n_fit; k++) {
      m->fW[a][k] = off; off += (int64_t)nin * m->fit_w[k];
      m->fB[a][k] = off; off += m->fit_w[k];
      nin = m->fit_w[k];
    }
    m->fW[a][m->n_fit] = off; off += nin;
    m->fB[a][m->n_fit] = off; off += 1;
  }
  m->nparams = off;
}

or_model *or_load(const char *path) {
  FILE *f = fopen(path, "rb");
  if (!f) return NULL;
  fseek(f, 0, SEEK_END);
  long sz = ftell(f);
  fseek(f, 0, SEEK_SET);
  unsigned char *buf = (unsigned char *)malloc(sz);
  if (!buf || fread(buf, 1, sz, f) != (size_t)sz) { fclose(f); free(buf); return NULL; }
  fclose(f);
  or_model *m = (or_model *)calloc(1, sizeof(or_model));
  if (sz < 64 || memcmp(buf, "DPSEMDL1", 8) != 0 || rd_i32(buf + 8) != 1) goto bad;
  int hb = rd_i32(buf + 12);
  int64_t np = rd_i64(buf + 16);
  m->ntypes = rd_i32(buf + 24); m->n_emb = rd_i32(buf + 28); m->n_fit = rd_i32(buf + 32);
  m->m2 = rd_i32(buf + 36); m->switch_kind = rd_i32(buf + 40); m->desc_norm = rd_i32(buf + 44);
  m->rc = rd_f64(buf + 48); m->rcs = rd_f64(buf + 56);
  if (m->ntypes < 1 || m->ntypes > OR_MAXT || m->n_emb < 1 || m->n_emb > OR_MAXL ||
      m->n_fit < 1 || m->n_fit > OR_MAXL) goto bad;
  int nint = m->n_emb + m->n_fit + m->ntypes;
  if (64 + 4 * nint > hb || hb > sz) goto bad;
  for (int k = 0; k < m->n_emb; k++) m->emb_w[k] = rd_i32(buf + 64 + 4 * k);
  for (int k = 0; k < m->n_fit; k++) m->fit_w[k] = rd_i32(buf + 64 + 4 * (m->n_emb + k));
  m->nm = 0;
  for (int t = 0; t < m->ntypes; t++) {
    m->sel[t] = rd_i32(buf + 64 + 4 * (m->n_emb + m->n_fit + t));
    m->sel_off[t] = m->nm;
    m->nm += m->sel[t];
  }
  m->sel_off[m->ntypes] = m->nm;
  m->M = m->emb_w[m->n_emb - 1];
  if (m->m2 < 1 || m->m2 > m->M || !(m->rc > m->rcs) || m->rcs < 0) goto bad;
  layout(m);
  if (m->nparams != np || hb + 8 * np != sz) goto bad;
  m->p = (double *)malloc(8 * np);
  memcpy(m->p, buf + hb, 8 * np);
  free(buf);
  return m;
bad:
  free(buf);
  free(m);
  return NULL;
}

void or_free(or_model *m) { if (m) { free(m->p); free(m); } }

int or_info(const or_model *m, int32_t *ntypes, int32_t *nm, int32_t *M, int32_t *m2,
            double *rc, int64_t *nparams) {
  *ntypes = m->ntypes; *nm = m->nm; *M = m->M; *m2 = m->m2; *rc = m->rc;
  *nparams = m->nparams;
  return 0;
}
int or_get_params(const or_model *m, double *out) { memcpy(out, m->p, 8 * m->nparams); return 0; }
int or_set_params(or_model *m, const double *in) { memcpy(m->p, in, 8 * m->nparams); return 0; }

/* ------------------------------------------------------------------------------------ */
/* switch function and environment row (Section 2, Eq. 5)                                */
/* ------------------------------------------------------------------------------------ */

/* s(r) = w(r)/r and ds/dr */
void or_smooth(const or_model *m, double r, double *s, double *ds) {
  double w, dw;
  if (r < m->rcs) {
    w = 1.0; dw = 0.0;
  } else if (r < m->rc) {
    double h = m->rc - m->rcs;
    double u = (r - m->rcs) / h;
    if (m->switch_kind == 1) {
      w = 0.5 * cos(M_PI * u) + 0.5;
      dw = -0.5 * M_PI * sin(M_PI * u) / h;
    } else {
      w = u * u * u * (-6.0 * u * u + 15.0 * u - 10.0) + 1.0;
      dw = -30.0 * u * u * (u - 1.0) * (u - 1.0) / h;
    }
  } else {
    w = 0.0; dw = 0.0;
  }
  *s = w / r;
  *ds = dw / r - w / (r * r);
}

void or_smooth_vec(const or_model *m, int64_t n, const double *r, double *s, double *ds) {
  for (int64_t i = 0; i < n; i++) or_smooth(m, r[i], &s[i], &ds[i]);
}

/* R row and dR/dd (4 x 3) for displacement d (Eq. 5) */
static void env_row(const or_model *m, const double d[3], double R[4], double dR[4][3]) {
  double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  double s, ds;
  or_smooth(m, r, &s, &ds);
  R[0] = s;
  for (int e = 0; e < 3; e++) R[1 + e] = s * d[e] / r;
  double q = (ds / r - s / (r * r)) / r; /* d(s/r)/dd_b = q * d_b */
  for (int b = 0; b < 3; b++) {
    dR[0][b] = ds * d[b] / r;
    for (int e = 0; e < 3; e++) dR[1 + e][b] = q * d[e] * d[b] + (e == b ? s / r : 0.0);
  }
}

void or_env_row(const or_model *m, const double *d, double *R, double *dR) {
  double dd[4][3];
  env_row(m, d, R, dd);
  memcpy(dR, dd, sizeof(dd));
}

/* ------------------------------------------------------------------------------------ */
/* periodic box helpers                                                                  */
/* ------------------------------------------------------------------------------------ */

typedef struct {
  double B[3][3], Bi[3][3], width[3];
  int K[3];
} box_t;

/* B rows are the cell vectors; fractional f = x B^-1 (row vectors).  The inverse is
 * the adjugate over the determinant, evaluated in this order. */
static int box_setup(const double *b9, double rc, box_t *bx) {
  double (*B)[3] = bx->B;
  memcpy(B, b9, 9 * sizeof(double));
  double det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
               B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
               B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
  if (!(det > 0)) return -1;
  double C[3][3];
  C[0][0] = B[1][1] * B[2][2] - B[1][2] * B[2][1];
  C[0][1] = B[1][2] * B[2][0] - B[1][0] * B[2][2];
  C[0][2] = B[1][0] * B[2][1] - B[1][1] * B[2][0];
  C[1][0] = B[0][2] * B[2][1] - B[0][1] * B[2][2];
  C[1][1] = B[0][0] * B[2][2] - B[0][2] * B[2][0];
  C[1][2] = B[0][1] * B[2][0] - B[0][0] * B[2][1];
  C[2][0] = B[0][1] * B[1][2] - B[0][2] * B[1][1];
  C[2][1] = B[0][2] * B[1][0] - B[0][0] * B[1][2];
  C[2][2] = B[0][0] * B[1][1] - B[0][1] * B[1][0];
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) bx->Bi[r][c] = C[c][r] / det;
  /* perpendicular width along axis k = volume / |a_l x a_m| = 1 / |row k of B^-T| */
  for (int k = 0; k < 3; k++) {
    double n2 = bx->Bi[0][k] * bx->Bi[0][k] + bx->Bi[1][k] * bx->Bi[1][k] +
                bx->Bi[2][k] * bx->Bi[2][k];
    bx->width[k] = 1.0 / sqrt(n2);
    bx->K[k] = (int)ceil(rc / bx->width[k]);
  }
  return 0;
}

/* n . B, summed over rows in order */
static void shift_of(const box_t *bx, const int n[3], double s[3]) {
  for (int c = 0; c < 3; c++)
    s[c] = ((double)n[0] * bx->B[0][c] + (double)n[1] * bx->B[1][c]) + (double)n[2] * bx->B[2][c];
}

static void frac_of(const box_t *bx, const double x[3], double f[3]) {
  for (int k = 0; k < 3; k++)
    f[k] = (x[0] * bx->Bi[0][k] + x[1] * bx->Bi[1][k]) + x[2] * bx->Bi[2][k];
}

/* wrapped coordinates x_w = x - floor(f) . B and their fractional coordinates */
static void wrap_all(const box_t *bx, int64_t n, const double *x, double *xw, double *fw) {
  for (int64_t i = 0; i < n; i++) {
    double f[3], s[3];
    frac_of(bx, x + 3 * i, f);
    int mm[3] = {(int)floor(f[0]), (int)floor(f[1]), (int)floor(f[2])};
    shift_of(bx, mm, s);
    for (int c = 0; c < 3; c++) xw[3 * i + c] = x[3 * i + c] - s[c];
    frac_of(bx, xw + 3 * i, fw + 3 * i);
  }
}

static int img_code(const box_t *bx, const int n[3]) {
  return ((n[0] + bx->K[0]) * (2 * bx->K[1] + 1) + (n[1] + bx->K[1])) * (2 * bx->K[2] + 1) +
         (n[2] + bx->K[2]);
}

/* ------------------------------------------------------------------------------------ */
/* neighbour search and formatting (Alg. 1)                                              */
/* ------------------------------------------------------------------------------------ */

typedef struct {
  int type;
  double r2;
  int64_t j;
  int img;
  int n[3];
  double d[3];
} cand_t;

static int cand_less(const cand_t *a, const cand_t *b) {
  if (a->type != b->type) return a->type < b->type;
  if (a->r2 != b->r2) return a->r2 < b->r2;
  if (a->j != b->j) return a->j < b->j;
  return a->img < b->img;
}

static int cand_cmp(const void *pa, const void *pb) {
  const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
  if (cand_less(a, b)) return -1;
  if (cand_less(b, a)) return 1;
  return 0;
}

typedef struct { cand_t *v; int n, cap; } cvec;
static void cpush(cvec *c, const cand_t *x) {
  if (c->n == c->cap) { c->cap = c->cap ? 2 * c->cap : 256; c->v = (cand_t *)realloc(c->v, c->cap * sizeof(cand_t)); }
  c->v[c->n++] = *x;
}

/* Every (j, image n) with |(x_j,w + n.B) - p| < radius, relative image n - nc.
 * p = x_ic,w + nc.B is the centre position.  The image range per axis is the one
 * the fractional distance allows (a necessary condition), widened by one. */
static void gather(const box_t *bx, int64_t n, const double *xw,
                   const double *fw, const int32_t *types, int64_t ic, const int nc[3],
                   double radius, int exclude_self, cvec *out) {
  double fc[3], g[3];
  for (int k = 0; k < 3; k++) { fc[k] = fw[3 * ic + k] + nc[k]; g[k] = radius / bx->width[k]; }
  double r2max = radius * radius;
  for (int64_t j = 0; j < n; j++) {
    int lo[3], hi[3];
    for (int k = 0; k < 3; k++) {
      lo[k] = (int)ceil(fc[k] - fw[3 * j + k] - g[k]) - 1;
      hi[k] = (int)floor(fc[k] - fw[3 * j + k] + g[k]) + 1;
    }
    int nn[3];
    for (nn[0] = lo[0]; nn[0] <= hi[0]; nn[0]++)
      for (nn[1] = lo[1]; nn[1] <= hi[1]; nn[1]++)
        for (nn[2] = lo[2]; nn[2] <= hi[2]; nn[2]++) {
          int rel[3] = {nn[0] - nc[0], nn[1] - nc[1], nn[2] - nc[2]};
          if (exclude_self && j == ic && rel[0] == 0 && rel[1] == 0 && rel[2] == 0) continue;
          double s[3], d[3];
          shift_of(bx, rel, s);
          for (int c = 0; c < 3; c++) d[c] = (xw[3 * j + c] + s[c]) - xw[3 * ic + c];
          double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
          if (!(r2 < r2max)) continue;
          cand_t cd;
          cd.type = types[j]; cd.r2 = r2; cd.j = j;
          cd.img = (abs(rel[0]) <= bx->K[0] && abs(rel[1]) <= bx->K[1] && abs(rel[2]) <= bx->K[2])
                       ? img_code(bx, rel) : -1;
          memcpy(cd.n, rel, sizeof(rel));
          memcpy(cd.d, d, sizeof(d));
          cpush(out, &cd);
        }
  }
}

/* One formatted row: slots [sel_off[t], sel_off[t]+sel[t]) hold type-t neighbours sorted
 * by (r^2, j, image); pads are j = -1.  Returns 1 if a type block overflowed. */
static int format_row(const or_model *m, cand_t *c, int nc, int64_t *slot_j, int *slot_img,
                      double (*slot_d)[3], int32_t *nnei) {
  qsort(c, nc, sizeof(cand_t), cand_cmp);
  int ovf = 0;
  for (int k = 0; k < m->nm; k++) { slot_j[k] = -1; slot_img[k] = -1; }
  int cnt[OR_MAXT] = {0};
  for (int q = 0; q < nc; q++) {
    int t = c[q].type;
    if (cnt[t] < m->sel[t]) {
      int k = m->sel_off[t] + cnt[t];
      slot_j[k] = c[q].j; slot_img[k] = c[q].img;
      if (slot_d) memcpy(slot_d[k], c[q].d, sizeof(c[q].d));
      cnt[t]++;
    } else {
      ovf = 1;
    }
  }
  if (nnei)
    for (int t = 0; t < m->ntypes; t++) nnei[t] = cnt[t];
  return ovf;
}

/* Formatted neighbour list of the listed centres (all atoms if cent == NULL).
 * nlist/img: [ncent][nm] int32, nnei: [ncent][ntypes].  Returns 0, -1 bad box,
 * -2 bad type.  *overflow is set when a type block was truncated. */
int or_nlist(const or_model *m, int64_t n, const double *coords, const int32_t *types,
             const double *box, int64_t ncent, const int64_t *cent, int32_t *nlist,
             int32_t *img, int32_t *nnei, int32_t *overflow) {
  box_t bx;
  if (box_setup(box, m->rc, &bx)) return -1;
  for (int64_t i = 0; i < n; i++)
    if (types[i] < 0 || types[i] >= m->ntypes) return -2;
  double *xw = (double *)malloc(24 * n), *fw = (double *)malloc(24 * n);
  wrap_all(&bx, n, coords, xw, fw);
  if (!cent) ncent = n;
  int ovf = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(g_threads) reduction(| : ovf)
  for (int64_t q = 0; q < ncent; q++) {
    int64_t i = cent ? cent[q] : q;
    cvec cv = {0};
    int z[3] = {0, 0, 0};
    gather(&bx, n, xw, fw, types, i, z, m->rc, 1, &cv);
    int64_t *sj = (int64_t *)malloc(8 * m->nm);
    int *si = (int *)malloc(4 * m->nm);
    ovf |= format_row(m, cv.v, cv.n, sj, si, NULL, nnei ? nnei + q * m->ntypes : NULL);
    for (int k = 0; k < m->nm; k++) {
      nlist[q * m->nm + k] = (int32_t)sj[k];
      if (img) img[q * m->nm + k] = si[k];
    }
    free(sj); free(si); free(cv.v);
  }
  free(xw); free(fw);
  if (overflow) *overflow = ovf;
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* networks                                                                              */
/* ------------------------------------------------------------------------------------ */

/* embedding net (a, b) on scalar s (Eq. 7-9).  h[k], t[k]: layer outputs and their tanh
 * parts, each emb_w[k] long, stored consecutively in acts. */
static void emb_fwd(const or_model *m, int a, int b, double s, double *acts) {
  const double *p = m->p;
  int net = a * m->ntypes + b;
  double *hprev = NULL;
  int nin = 1;
  double *h = acts;
  for (int k = 0; k < m->n_emb; k++) {
    int nout = m->emb_w[k];
    double *t = h + nout;
    const double *W = p + m->eW[net][k], *bb = p + m->eB[net][k];
    for (int o = 0; o < nout; o++) {
      double z = bb[o];
      if (k == 0) z += s * W[o];
      else for (int i = 0; i < nin; i++) z += hprev[i] * W[i * nout + o];
      t[o] = tanh(z);
      if (k == 0) h[o] = t[o];
      else if (nout == 2 * nin) h[o] = hprev[o % nin] + t[o];
      else if (nout == nin) h[o] = hprev[o] + t[o];
      else h[o] = t[o];
    }
    hprev = h;
    nin = nout;
    h = t + nout;
  }
}

static int emb_acts_len(const or_model *m) {
  int n = 0;
  for (int k = 0; k < m->n_emb; k++) n += 2 * m->emb_w[k];
  return n;
}

static const double *emb_out(const or_model *m, const double *acts) {
  int off = 0;
  for (int k = 0; k < m->n_emb - 1; k++) off += 2 * m->emb_w[k];
  return acts + off;
}

/* back propagation of gG (length M) through the embedding net; returns ds */
static double emb_bwd(const or_model *m, int a, int b, const double *acts, const double *gG,
                      double *work) {
  const double *p = m->p;
  int net = a * m->ntypes + b;
  int offs[OR_MAXL];
  int off = 0;
  int maxw = 1;
  for (int k = 0; k < m->n_emb; k++) { offs[k] = off; off += 2 * m->emb_w[k]; if (m->emb_w[k] > maxw) maxw = m->emb_w[k]; }
  double *gh = work, *gprev = work + maxw;
  memcpy(gh, gG, sizeof(double) * m->M);
  double ds = 0.0;
  for (int k = m->n_emb - 1; k >= 0; k--) {
    int nout = m->emb_w[k];
    int nin = k == 0 ? 1 : m->emb_w[k - 1];
    const double *t = acts + offs[k] + nout;
    const double *W = p + m->eW[net][k];
    if (k == 0) {
      for (int o = 0; o < nout; o++) ds += gh[o] * (1.0 - t[o] * t[o]) * W[o];
      break;
    }
    for (int i = 0; i < nin; i++) {
      double v = 0.0;
      for (int o = 0; o < nout; o++) v += gh[o] * (1.0 - t[o] * t[o]) * W[i * nout + o];
      if (nout == 2 * nin) v += gh[i] + gh[i + nin];
      else if (nout == nin) v += gh[i];
      gprev[i] = v;
    }
    double *tmp = gh; gh = gprev; gprev = tmp;
  }
  return ds;
}

/* fitting net of type a on descriptor d (length M*m2) (Eq. 2-3); returns E_i and, if
 * gd != NULL, dE_i/dd. */
static double fit_eval(const or_model *m, int a, const double *d, double *gd, double *work) {
  const double *p = m->p;
  int maxw = m->M * m->m2;
  for (int k = 0; k < m->n_fit; k++) if (m->fit_w[k] > maxw) maxw = m->fit_w[k];
  /* per layer: input x_k and tanh t_k */
  double *xs = work;                            /* (n_fit+1) * maxw */
  double *ts = work + (m->n_fit + 1) * maxw;    /* n_fit * maxw */
  double *g0 = ts + m->n_fit * maxw, *g1 = g0 + maxw;
  int nin = m->M * m->m2;
  memcpy(xs, d, sizeof(double) * nin);
  for (int k = 0; k < m->n_fit; k++) {
    int nout = m->fit_w[k];
    const double *W = p + m->fW[a][k], *b = p + m->fB[a][k];
    double *x = xs + k * maxw, *y = xs + (k + 1) * maxw, *t = ts + k * maxw;
    for (int o = 0; o < nout; o++) {
      double z = b[o];
      for (int i = 0; i < nin; i++) z += x[i] * W[(int64_t)i * nout + o];
      t[o] = tanh(z);
      y[o] = (nout == nin ? x[o] : 0.0) + t[o];
    }
    nin = nout;
  }
  const double *wo = p + m->fW[a][m->n_fit];
  double E = p[m->fB[a][m->n_fit]];
  const double *xl = xs + m->n_fit * maxw;
  for (int i = 0; i < nin; i++) E += xl[i] * wo[i];
  if (!gd) return E;
  for (int i = 0; i < nin; i++) g0[i] = wo[i];
  for (int k = m->n_fit - 1; k >= 0; k--) {
    int nout = m->fit_w[k];
    int kin = k == 0 ? m->M * m->m2 : m->fit_w[k - 1];
    const double *W = p + m->fW[a][k];
    const double *t = ts + k * maxw;
    for (int i = 0; i < kin; i++) {
      double v = (nout == kin) ? g0[i] : 0.0;
      for (int o = 0; o < nout; o++) v += g0[o] * (1.0 - t[o] * t[o]) * W[(int64_t)i * nout + o];
      g1[i] = v;
    }
    double *tmp = g0; g0 = g1; g1 = tmp;
  }
  memcpy(gd, g0, sizeof(double) * m->M * m->m2);
  return E;
}

static int fit_work_len(const or_model *m) {
  int maxw = m->M * m->m2;
  for (int k = 0; k < m->n_fit; k++) if (m->fit_w[k] > maxw) maxw = m->fit_w[k];
  return (2 * m->n_fit + 3) * maxw;
}

/* ------------------------------------------------------------------------------------ */
/* one centre: E_i and dE_i/dd for every slot (Eq. 1, 4, 10)                             */
/* ------------------------------------------------------------------------------------ */

typedef struct {
  double *acts, *R, *dR, *T, *D, *gD, *gT, *fw, *ew, *gG;
} atom_ws;

static void ws_alloc(const or_model *m, atom_ws *w) {
  int al = emb_acts_len(m);
  w->acts = (double *)malloc(sizeof(double) * (size_t)m->nm * al);
  w->R = (double *)malloc(sizeof(double) * m->nm * 4);
  w->dR = (double *)malloc(sizeof(double) * m->nm * 12);
  w->T = (double *)malloc(sizeof(double) * m->M * 4);
  w->gT = (double *)malloc(sizeof(double) * m->M * 4);
  w->D = (double *)malloc(sizeof(double) * m->M * m->m2);
  w->gD = (double *)malloc(sizeof(double) * m->M * m->m2);
  w->fw = (double *)malloc(sizeof(double) * fit_work_len(m));
  int maxw = 1;
  for (int k = 0; k < m->n_emb; k++) if (m->emb_w[k] > maxw) maxw = m->emb_w[k];
  w->ew = (double *)malloc(sizeof(double) * 2 * maxw);
  w->gG = (double *)malloc(sizeof(double) * m->M);
}
static void ws_free(atom_ws *w) {
  free(w->acts); free(w->R); free(w->dR); free(w->T); free(w->gT); free(w->D); free(w->gD);
  free(w->fw); free(w->ew); free(w->gG);
}

/* slot_j[k] < 0 marks a pad; slot_d[k] is the displacement r_j - r_i of a real slot.
 * Outputs E_i, g[k][3] = dE_i/dd_k (zero for pads), and optional T, D, dE/dT dumps. */
static double center_eval(const or_model *m, int ti, const int64_t *slot_j,
                          const int32_t *slot_type, double (*slot_d)[3], double (*g)[3],
                          atom_ws *w, double *T_out, double *D_out, double *gT_out) {
  int M = m->M, m2 = m->m2, nm = m->nm, al = emb_acts_len(m);
  double norm = m->desc_norm == 0 ? (double)nm : 1.0;
  for (int q = 0; q < M * 4; q++) w->T[q] = 0.0;
  /* Alg. 2 + Eq. 6: environment rows and embedding rows, Eq. 4: T = G^T R / N_m */
  for (int k = 0; k < nm; k++) {
    double *R = w->R + 4 * k;
    if (slot_j[k] < 0) { R[0] = R[1] = R[2] = R[3] = 0.0; continue; }
    env_row(m, slot_d[k], R, (double (*)[3])(w->dR + 12 * k));
    double *acts = w->acts + (size_t)k * al;
    emb_fwd(m, ti, slot_type[k], R[0], acts);
    const double *G = emb_out(m, acts);
    for (int a = 0; a < M; a++)
      for (int c = 0; c < 4; c++) w->T[4 * a + c] += G[a] * R[c];
  }
  for (int q = 0; q < M * 4; q++) w->T[q] /= norm;
  /* Eq. 4: D[a][b] = sum_c T[a][c] T[b][c], b < M< */
  for (int a = 0; a < M; a++)
    for (int b = 0; b < m2; b++) {
      double v = 0.0;
      for (int c = 0; c < 4; c++) v += w->T[4 * a + c] * w->T[4 * b + c];
      w->D[a * m2 + b] = v;
    }
  double E = fit_eval(m, ti, w->D, w->gD, w->fw);
  /* dE/dT from dE/dD */
  for (int p = 0; p < M; p++)
    for (int c = 0; c < 4; c++) {
      double v = 0.0;
      for (int b = 0; b < m2; b++) v += w->gD[p * m2 + b] * w->T[4 * b + c];
      if (p < m2)
        for (int a = 0; a < M; a++) v += w->gD[a * m2 + p] * w->T[4 * a + c];
      w->gT[4 * p + c] = v;
    }
  if (T_out) memcpy(T_out, w->T, sizeof(double) * M * 4);
  if (D_out) memcpy(D_out, w->D, sizeof(double) * M * m2);
  if (gT_out) memcpy(gT_out, w->gT, sizeof(double) * M * 4);
  /* Eq. 10 by back propagation, slot by slot */
  for (int k = 0; k < nm; k++) {
    g[k][0] = g[k][1] = g[k][2] = 0.0;
    if (slot_j[k] < 0) continue;
    const double *R = w->R + 4 * k;
    const double *acts = w->acts + (size_t)k * al;
    const double *G = emb_out(m, acts);
    double gR[4];
    for (int a = 0; a < M; a++) {
      double v = 0.0;
      for (int c = 0; c < 4; c++) v += w->gT[4 * a + c] * R[c];
      w->gG[a] = v / norm;
    }
    for (int c = 0; c < 4; c++) {
      double v = 0.0;
      for (int a = 0; a < M; a++) v += G[a] * w->gT[4 * a + c];
      gR[c] = v / norm;
    }
    gR[0] += emb_bwd(m, ti, slot_type[k], acts, w->gG, w->ew);
    const double *dR = w->dR + 12 * k;
    for (int b = 0; b < 3; b++) {
      double v = 0.0;
      for (int c = 0; c < 4; c++) v += gR[c] * dR[3 * c + b];
      g[k][b] = v;
    }
  }
  return E;
}

/* ------------------------------------------------------------------------------------ */
/* full evaluation                                                                       */
/* ------------------------------------------------------------------------------------ */

/* E, F [n][3], W [9] (row major, W_ab = -sum d_a g_b), optional Ei [n], T [n][M][4],
 * D [n][M][m2], gT [n][M][4].  Returns 0; -1 bad box; -2 bad type; 1 sel overflow
 * (results valid, nearest neighbours kept). */
/* Wi (may be NULL): per-centre virial [n][9], W_i = -sum_j d_ij (x) dE_i/dd_ij over the
 * neighbours j of centre i (each pair term of W assigned to its centre; sum_i W_i = W) */
static int eval_core(const or_model *m, int64_t n, const double *coords, const int32_t *types,
                     const double *box, double *E, double *F, double *W, double *Ei, double *T,
                     double *D, double *gT, double *Wi) {
  box_t bx;
  if (box_setup(box, m->rc, &bx)) return -1;
  for (int64_t i = 0; i < n; i++)
    if (types[i] < 0 || types[i] >= m->ntypes) return -2;
  double *xw = (double *)malloc(24 * n), *fw = (double *)malloc(24 * n);
  wrap_all(&bx, n, coords, xw, fw);
  int nt = g_threads;
  /* per-thread partial sums, one slot per thread of the team */
  double *Fp = (double *)calloc((size_t)nt * n * 3, sizeof(double));
  double (*Wp)[9] = (double (*)[9])calloc((size_t)nt, sizeof(double[9]));
  double *Ep = (double *)calloc((size_t)nt, sizeof(double));
  int ovf = 0;
#pragma omp parallel num_threads(nt) reduction(| : ovf)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    atom_ws w;
    ws_alloc(m, &w);
    int64_t *sj = (int64_t *)malloc(8 * m->nm);
    int *si = (int *)malloc(4 * m->nm);
    int32_t *st = (int32_t *)malloc(4 * m->nm);
    double (*sd)[3] = (double (*)[3])malloc(24 * m->nm);
    double (*g)[3] = (double (*)[3])malloc(24 * m->nm);
    double *Fl = Fp + (size_t)tid * n * 3;
    for (int t = 0; t < m->ntypes; t++)
      for (int k = m->sel_off[t]; k < m->sel_off[t + 1]; k++) st[k] = t;
#pragma omp for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
      cvec cv = {0};
      int z[3] = {0, 0, 0};
      gather(&bx, n, xw, fw, types, i, z, m->rc, 1, &cv);
      ovf |= format_row(m, cv.v, cv.n, sj, si, sd, NULL);
      free(cv.v);
      double ei = center_eval(m, types[i], sj, st, sd, g, &w, T ? T + i * m->M * 4 : NULL,
                              D ? D + i * m->M * m->m2 : NULL, gT ? gT + i * m->M * 4 : NULL);
      if (Ei) Ei[i] = ei;
      Ep[tid] += ei;
      for (int k = 0; k < m->nm; k++) {
        if (sj[k] < 0) continue;
        int64_t j = sj[k];
        for (int b = 0; b < 3; b++) {
          Fl[3 * i + b] += g[k][b];
          Fl[3 * j + b] -= g[k][b];
        }
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) Wp[tid][3 * a + b] -= sd[k][a] * g[k][b];
      }
      if (Wi) {
        for (int q = 0; q < 9; q++) Wi[9 * i + q] = 0.0;
        for (int k = 0; k < m->nm; k++) {
          if (sj[k] < 0) continue;
          for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Wi[9 * i + 3 * a + b] -= sd[k][a] * g[k][b];
        }
      }
    }
    ws_free(&w);
    free(sj); free(si); free(st); free(sd); free(g);
  }
  double Et = 0.0;
  for (int t = 0; t < nt; t++) Et += Ep[t];
  *E = Et;
  for (int64_t q = 0; q < 3 * n; q++) {
    double v = 0.0;
    for (int t = 0; t < nt; t++) v += Fp[(size_t)t * n * 3 + q];
    F[q] = v;
  }
  if (W)
    for (int q = 0; q < 9; q++) {
      double v = 0.0;
      for (int t = 0; t < nt; t++) v += Wp[t][q];
      W[q] = v;
    }
  free(Fp); free(Wp); free(Ep); free(xw); free(fw);
  return ovf ? 1 : 0;
}

int or_eval(const or_model *m, int64_t n, const double *coords, const int32_t *types,
            const double *box, double *E, double *F, double *W, double *Ei, double *T,
            double *D, double *gT) {
  return eval_core(m, n, coords, types, box, E, F, W, Ei, T, D, gT, NULL);
}

/* or_eval with the per-atom energy Ei [n] and per-centre virial Wi [n][9] */
int or_eval_atomic(const or_model *m, int64_t n, const double *coords, const int32_t *types,
                   const double *box, double *E, double *F, double *W, double *Ei, double *Wi) {
  return eval_core(m, n, coords, types, box, E, F, W, Ei, NULL, NULL, NULL, Wi);
}

/* ------------------------------------------------------------------------------------ */
/* sampled evaluation: exact E_k and F_k for listed atoms k, from the centres that see k  */
/* ------------------------------------------------------------------------------------ */

int or_eval_sampled(const or_model *m, int64_t n, const double *coords, const int32_t *types,
                    const double *box, int64_t ns, const int64_t *samp, double *Ei_out,
                    double *F_out) {
  box_t bx;
  if (box_setup(box, m->rc, &bx)) return -1;
  for (int64_t i = 0; i < n; i++)
    if (types[i] < 0 || types[i] >= m->ntypes) return -2;
  double *xw = (double *)malloc(24 * n), *fw = (double *)malloc(24 * n);
  wrap_all(&bx, n, coords, xw, fw);
  int ovf = 0;
#pragma omp parallel num_threads(g_threads) reduction(| : ovf)
  {
    atom_ws w;
    ws_alloc(m, &w);
    int64_t *sj = (int64_t *)malloc(8 * m->nm);
    int *si = (int *)malloc(4 * m->nm);
    int32_t *st = (int32_t *)malloc(4 * m->nm);
    double (*sd)[3] = (double (*)[3])malloc(24 * m->nm);
    double (*g)[3] = (double (*)[3])malloc(24 * m->nm);
    for (int t = 0; t < m->ntypes; t++)
      for (int k = m->sel_off[t]; k < m->sel_off[t + 1]; k++) st[k] = t;
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < ns; q++) {
      int64_t kk = samp[q];
      int z[3] = {0, 0, 0};
      /* every image within 2 rc of atom kk: contains all centres that see kk and all
       * of their neighbours */
      cvec big = {0};
      gather(&bx, n, xw, fw, types, kk, z, 2.0 * m->rc, 0, &big);
      double Fk[3] = {0, 0, 0};
      /* distinct centre atoms: kk itself and every atom with an image within rc */
      int64_t *centres = (int64_t *)malloc(8 * (big.n + 1));
      int nce = 0;
      for (int a = 0; a < big.n; a++) {
        if (big.v[a].r2 >= m->rc * m->rc) continue;
        int dup = 0;
        for (int b = 0; b < nce; b++) if (centres[b] == big.v[a].j) { dup = 1; break; }
        if (!dup) centres[nce++] = big.v[a].j;
      }
      int has_self = 0;
      for (int b = 0; b < nce; b++) if (centres[b] == kk) has_self = 1;
      if (!has_self) centres[nce++] = kk;
      for (int b = 0; b < nce; b++) {
        int64_t ic = centres[b];
        /* the image of ic that lies within rc of kk (kk itself: image 0) */
        int nc[3] = {0, 0, 0};
        for (int a = 0; a < big.n; a++)
          if (big.v[a].j == ic && big.v[a].r2 < m->rc * m->rc) { memcpy(nc, big.v[a].n, sizeof(nc)); break; }
        /* neighbours of that image: candidates within rc of it, image relative to it */
        cvec cv = {0};
        for (int a = 0; a < big.n; a++) {
          int rel[3] = {big.v[a].n[0] - nc[0], big.v[a].n[1] - nc[1], big.v[a].n[2] - nc[2]};
          if (big.v[a].j == ic && rel[0] == 0 && rel[1] == 0 && rel[2] == 0) continue;
          double s[3], d[3];
          shift_of(&bx, rel, s);
          int64_t j = big.v[a].j;
          for (int c = 0; c < 3; c++) d[c] = (xw[3 * j + c] + s[c]) - xw[3 * ic + c];
          double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
          if (!(r2 < m->rc * m->rc)) continue;
          cand_t cd;
          cd.type = types[j]; cd.r2 = r2; cd.j = j; cd.img = img_code(&bx, rel);
          memcpy(cd.n, rel, sizeof(rel));
          memcpy(cd.d, d, sizeof(d));
          cpush(&cv, &cd);
        }
        ovf |= format_row(m, cv.v, cv.n, sj, si, sd, NULL);
        free(cv.v);
        double ei = center_eval(m, types[ic], sj, st, sd, g, &w, NULL, NULL, NULL);
        if (ic == kk) Ei_out[q] = ei;
        for (int k = 0; k < m->nm; k++) {
          if (sj[k] < 0) continue;
          for (int c = 0; c < 3; c++) {
            if (ic == kk) Fk[c] += g[k][c];
            if (sj[k] == kk) Fk[c] -= g[k][c];
          }
        }
      }
      memcpy(F_out + 3 * q, Fk, sizeof(Fk));
      free(centres);
      free(big.v);
    }
    ws_free(&w);
    free(sj); free(si); free(st); free(sd); free(g);
  }
  free(xw); free(fw);
  return ovf ? 1 : 0;
}

/* ------------------------------------------------------------------------------------ */
/* velocity Verlet (Section 4)                                                           */
/* ------------------------------------------------------------------------------------ */

#define OR_ACC 9.64853321e-3      /* eV / (A amu) in A / fs^2 */
#define OR_KB 8.617333262e-5      /* eV / K */
#define OR_EVA3_BAR 1.602176634e6 /* eV / A^3 in bar */

static void thermo_row(const or_model *m, int64_t n, const double *v, const int32_t *types,
                       const double *mass, const double *box, double E, const double *W,
                       int step, double *row) {
  (void)m;
  double ke = 0.0;
  for (int64_t i = 0; i < n; i++)
    for (int c = 0; c < 3; c++) ke += 0.5 * mass[types[i]] * v[3 * i + c] * v[3 * i + c];
  ke /= OR_ACC;
  double T = 2.0 * ke / ((3.0 * n - 3.0) * OR_KB);
  box_t bx;
  box_setup(box, 1.0, &bx);
  double V = bx.B[0][0] * (bx.B[1][1] * bx.B[2][2] - bx.B[1][2] * bx.B[2][1]) -
             bx.B[0][1] * (bx.B[1][0] * bx.B[2][2] - bx.B[1][2] * bx.B[2][0]) +
             bx.B[0][2] * (bx.B[1][0] * bx.B[2][1] - bx.B[1][1] * bx.B[2][0]);
  double P = (2.0 * ke + (W[0] + W[4] + W[8])) / (3.0 * V) * OR_EVA3_BAR;
  row[0] = step; row[1] = E; row[2] = ke; row[3] = T; row[4] = E + ke; row[5] = P;
}

/* nsteps of velocity Verlet with a fresh neighbour list at every force evaluation.
 * x, v updated in place; thermo rows [step, PE, KE, T, Etot, P(bar)] at step 0 and
 * every thermo_every steps. */
int or_md(const or_model *m, int64_t n, double *x, double *v, const int32_t *types,
          const double *mass, const double *box, double dt, int nsteps, int thermo_every,
          double *thermo) {
  double *F = (double *)malloc(24 * n);
  double E, W[9];
  int rc = or_eval(m, n, x, types, box, &E, F, W, NULL, NULL, NULL, NULL);
  if (rc < 0) { free(F); return rc; }
  int row = 0;
  if (thermo) thermo_row(m, n, v, types, mass, box, E, W, 0, thermo + 6 * row++);
  for (int s = 1; s <= nsteps; s++) {
    for (int64_t i = 0; i < n; i++)
      for (int c = 0; c < 3; c++) {
        v[3 * i + c] += 0.5 * dt * F[3 * i + c] / mass[types[i]] * OR_ACC;
        x[3 * i + c] += dt * v[3 * i + c];
      }
    rc = or_eval(m, n, x, types, box, &E, F, W, NULL, NULL, NULL, NULL);
    if (rc < 0) { free(F); return rc; }
    for (int64_t i = 0; i < n; i++)
      for (int c = 0; c < 3; c++) v[3 * i + c] += 0.5 * dt * F[3 * i + c] / mass[types[i]] * OR_ACC;
    if (thermo && thermo_every > 0 && s % thermo_every == 0)
      thermo_row(m, n, v, types, mass, box, E, W, s, thermo + 6 * row++);
  }
  free(F);
  return 0;
}

/* ---------------------------------------------------------------------------------
 * Isobaric MD (isotropic box scaling), an extension of Section 4's velocity Verlet in
 * which the pressure from the virial (the thermo quantity of Section 4) drives the box.
 * Equations of motion of Martyna, Tobias and Klein (1994) with a Nose-Hoover thermostat
 * on the particles (none when tau_t <= 0, i.e. isoenthalpic), N_f = 3N - 3 degrees of
 * freedom, alpha = 1 + 3 / N_f, v_eps = p_eps / W, v_xi = p_xi / Q:
 *   dx/dt = v + v_eps x
 *   dv/dt = F / m - alpha v_eps v - v_xi v
 *   dV/dt = 3 V v_eps,   dp_eps/dt = alpha 2 KE + tr(virial) - 3 V P_ext
 *   dxi/dt = v_xi,       dp_xi/dt = 2 KE - N_f kT
 * with W = (N_f + 3) kT tau_p^2 and Q = N_f kT tau_t^2.  Integrated by the symmetric
 * splitting T(dt/2) E(dt/2) P(dt/2) R(dt) [forces] P(dt/2) E(dt/2) T(dt/2), each part
 * solved exactly:
 *   E(h): p_eps += h G_eps
 *   P(h): v <- v exp(-alpha v_eps h) + h a exp(-alpha v_eps h / 2) sinhc(alpha v_eps h / 2)
 *   R(h): x <- x exp(v_eps h) + h v exp(v_eps h / 2) sinhc(v_eps h / 2),  B <- B exp(v_eps h)
 *   T(h): p_xi += h/2 G_xi;  v <- v exp(-h v_xi);  xi += h v_xi;  p_xi += h/2 G_xi
 * It conserves H = E_pot + KE + p_eps^2 / (2 W) + P_ext V + p_xi^2 / (2 Q) + N_f kT xi up
 * to O(dt^2).  box [9] is updated in place; thermo rows of 8:
 * [step, PE, KE, T, Etot, P(bar), V, H]; state [3] (may be NULL) receives p_eps, xi, p_xi.
 * --------------------------------------------------------------------------------- */
static double npt_sinhc(double y) {
  return fabs(y) < 1e-4 ? 1.0 + y * y / 6.0 * (1.0 + y * y / 20.0) : sinh(y) / y;
}

static double npt_ke(int64_t n, const double *v, const int32_t *types, const double *mass) {
  double ke = 0.0;
  for (int64_t i = 0; i < n; i++)
    for (int c = 0; c < 3; c++) ke += 0.5 * mass[types[i]] * v[3 * i + c] * v[3 * i + c];
  return ke / OR_ACC;
}

static double npt_volume(const double *B) {
  return B[0] * (B[4] * B[8] - B[5] * B[7]) - B[1] * (B[3] * B[8] - B[5] * B[6]) +
         B[2] * (B[3] * B[7] - B[4] * B[6]);
}

int or_md_npt(const or_model *m, int64_t n, double *x, double *v, const int32_t *types,
              const double *mass, double *box, double pext_bar, double tau_p, double temp,
              double tau_t, double dt, int nsteps, int thermo_every, double *thermo,
              double *state) {
  if (n < 2 || !(tau_p > 0) || !(temp > 0)) return -1;
  const double nf = 3.0 * (double)n - 3.0, alpha = 1.0 + 3.0 / nf, kT = OR_KB * temp;
  const double Wb = (nf + 3.0) * kT * tau_p * tau_p;
  const int thermostat = tau_t > 0;
  const double Q = thermostat ? nf * kT * tau_t * tau_t : 1.0;
  const double pext = pext_bar / OR_EVA3_BAR;
  double *F = (double *)malloc(24 * n);
  double E, W[9];
  int rc = or_eval(m, n, x, types, box, &E, F, W, NULL, NULL, NULL, NULL);
  if (rc < 0) { free(F); return rc; }
  double peps = 0.0, xi = 0.0, pxi = 0.0;
  const double h = 0.5 * dt;
  int row = 0;
  for (int s = 0; s <= nsteps; s++) {
    if (s > 0) {
      /* T(dt/2) */
      if (thermostat) {
        double ke = npt_ke(n, v, types, mass);
        pxi += 0.5 * h * (2.0 * ke - nf * kT);
        const double c = exp(-h * pxi / Q);
        for (int64_t q = 0; q < 3 * n; q++) v[q] *= c;
        xi += h * pxi / Q;
        ke = npt_ke(n, v, types, mass);
        pxi += 0.5 * h * (2.0 * ke - nf * kT);
      }
      /* E(dt/2) */
      {
        const double ke = npt_ke(n, v, types, mass);
        peps += h * (alpha * 2.0 * ke + (W[0] + W[4] + W[8]) - 3.0 * npt_volume(box) * pext);
      }
      /* P(dt/2) */
      {
        const double ve = peps / Wb, y = alpha * ve * h;
        const double a1 = exp(-y), b1 = h * exp(-0.5 * y) * npt_sinhc(0.5 * y);
        for (int64_t i = 0; i < n; i++)
          for (int c = 0; c < 3; c++)
            v[3 * i + c] = v[3 * i + c] * a1 + b1 * F[3 * i + c] / mass[types[i]] * OR_ACC;
      }
      /* R(dt) */
      {
        const double ve = peps / Wb, y = ve * dt;
        const double sx = exp(y), b2 = dt * exp(0.5 * y) * npt_sinhc(0.5 * y);
        for (int64_t q = 0; q < 3 * n; q++) x[q] = x[q] * sx + b2 * v[q];
        for (int q = 0; q < 9; q++) box[q] *= sx;
      }
      rc = or_eval(m, n, x, types, box, &E, F, W, NULL, NULL, NULL, NULL);
      if (rc < 0) { free(F); return rc; }
      /* P(dt/2) */
      {
        const double ve = peps / Wb, y = alpha * ve * h;
        const double a1 = exp(-y), b1 = h * exp(-0.5 * y) * npt_sinhc(0.5 * y);
        for (int64_t i = 0; i < n; i++)
          for (int c = 0; c < 3; c++)
            v[3 * i + c] = v[3 * i + c] * a1 + b1 * F[3 * i + c] / mass[types[i]] * OR_ACC;
      }
      /* E(dt/2) */
      {
        const double ke = npt_ke(n, v, types, mass);
        peps += h * (alpha * 2.0 * ke + (W[0] + W[4] + W[8]) - 3.0 * npt_volume(box) * pext);
      }
      /* T(dt/2) */
      if (thermostat) {
        double ke = npt_ke(n, v, types, mass);
        pxi += 0.5 * h * (2.0 * ke - nf * kT);
        const double c = exp(-h * pxi / Q);
        for (int64_t q = 0; q < 3 * n; q++) v[q] *= c;
        xi += h * pxi / Q;
        ke = npt_ke(n, v, types, mass);
        pxi += 0.5 * h * (2.0 * ke - nf * kT);
      }
    }
    if (thermo && (s == 0 || (thermo_every > 0 && s % thermo_every == 0))) {
      const double ke = npt_ke(n, v, types, mass), V = npt_volume(box);
      double *r = thermo + 8 * row++;
      r[0] = s;
      r[1] = E;
      r[2] = ke;
      r[3] = 2.0 * ke / (nf * OR_KB);
      r[4] = E + ke;
      r[5] = (2.0 * ke + (W[0] + W[4] + W[8])) / (3.0 * V) * OR_EVA3_BAR;
      r[6] = V;
      r[7] = E + ke + 0.5 * peps * peps / Wb + pext * V +
             (thermostat ? 0.5 * pxi * pxi / Q + nf * kT * xi : 0.0);
    }
  }
  if (state) {
    state[0] = peps;
    state[1] = xi;
    state[2] = pxi;
  }
  free(F);
  return 0;
}
