/*
 * FP64 CPU oracle for MRF dictionary generating and searching.
 *
 * TEST INFRASTRUCTURE ONLY (see mrf_oracle.h). Plain, sequential per entry
 * and per voxel; OpenMP only distributes independent entries or voxels.
 *
 * Parity status of each part:
 *   - simulator, CC, brute force: pinned by closed forms, exact symmetries,
 *     an independent matrix-exponential integration of Eq. A1 and a NumPy
 *     brute-force reduction (tests/test_oracle_*.py).
 *   - ZOOM engine mechanics: pinned on analytic objectives with known argmax
 *     and on the evaluation counts stated in the Theory section; an
 *     exhaustive unit-step scan equals brute force. Its agreement with the
 *     paper's own CC landscapes is parity unpinned (the figures carrying them
 *     are not available), and so are the B1 stages (the paper has no fourth
 *     parameter).
 *   - distance objective of the finest-resolution stages (phase-fitted
 *     residual of the non-normalised fingerprint): pinned by a numerical
 *     minimisation over the phase, exact matches and scalings, its relation
 *     to CC with the magnitude fitted, and a NumPy argmin over an
 *     independently integrated dictionary (tests/test_oracle_objective.py).
 */
#include "mrf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Step factors (Appendix A).                                                */
/* ------------------------------------------------------------------------ */

/* Longitudinal or transverse relaxation over t: exp(-t/T); T = inf gives 1. */
static double relax(double t, double T) { return exp(-t / T); }

/* Off-resonance precession angle over t ms at df Hz: 2*pi*df*t/1000 rad. */
static void precess(double t, double df, double* c, double* s) {
  double th = 2.0 * ORC_PI * df * t / 1000.0;
  *c = cos(th);
  *s = sin(th);
}

/* RF pulse factors: cos/sin of the phase and of the B1-scaled flip angle. */
static void rf_factors(double fa_deg, double phase_deg, double b1, double* f4) {
  double a = b1 * fa_deg * ORC_PI / 180.0;
  double p = phase_deg * ORC_PI / 180.0;
  f4[0] = cos(p);
  f4[1] = sin(p);
  f4[2] = cos(a);
  f4[3] = sin(a);
}

/* M <- Rz(phi) Rx(-alpha) Rz(-phi) M, with Rz, Rx counter-clockwise. */
static void apply_rf(double* M, const double* f4) {
  double cp = f4[0], sp = f4[1], ca = f4[2], sa = f4[3];
  /* Rz(-phi) */
  double x = cp * M[0] + sp * M[1];
  double y = -sp * M[0] + cp * M[1];
  double z = M[2];
  /* Rx(-alpha): y' = cos(a) y + sin(a) z, z' = -sin(a) y + cos(a) z */
  double y2 = ca * y + sa * z;
  double z2 = -sa * y + ca * z;
  /* Rz(phi) */
  M[0] = cp * x - sp * y2;
  M[1] = sp * x + cp * y2;
  M[2] = z2;
}

/* Free evolution: relaxation and precession about z, recovery toward M0 = 1. */
static void apply_free(double* M, double e1, double e2, double c, double s) {
  double x = M[0], y = M[1];
  M[0] = e2 * (c * x - s * y);
  M[1] = e2 * (s * x + c * y);
  M[2] = e1 * M[2] + (1.0 - e1);
}

/* Per-entry view of the step factors: each array has n_tr values. */
typedef struct {
  const double *e1a, *e1b;          /* T1 relaxation over TE and TR-TE */
  const double *e2a, *e2b;          /* T2 relaxation over TE and TR-TE */
  const double *ca, *sa, *cb, *sb;  /* precession over TE and TR-TE */
  const double* rf;                 /* [n_tr][4] */
  double e1_ti;                     /* T1 relaxation over TI */
} entry_factors;

/* The event model of the header comment; writes samples and/or states. */
static void run_entry(int32_t n_tr, int32_t inversion, const entry_factors* f,
                      double* re, double* im, double* states) {
  double M[3] = {0.0, 0.0, 1.0};
  if (inversion) M[2] = -M[2];
  M[2] = f->e1_ti * M[2] + (1.0 - f->e1_ti);  /* TI: transverse part is zero */
  for (int32_t j = 0; j < n_tr; ++j) {
    apply_rf(M, f->rf + 4 * (size_t)j);
    if (states) memcpy(states + 9 * (size_t)j, M, sizeof M);
    apply_free(M, f->e1a[j], f->e2a[j], f->ca[j], f->sa[j]);
    if (states) memcpy(states + 9 * (size_t)j + 3, M, sizeof M);
    if (re) re[j] = M[0];
    if (im) im[j] = M[1];
    apply_free(M, f->e1b[j], f->e2b[j], f->cb[j], f->sb[j]);
    if (states) memcpy(states + 9 * (size_t)j + 6, M, sizeof M);
  }
}

static int seq_ok(const orc_seq* seq, int32_t n_tr) {
  if (!seq || n_tr < 0 || n_tr > seq->n) return 0;
  for (int32_t j = 0; j < n_tr; ++j)
    if (!(seq->te_ms[j] > 0.0 && seq->te_ms[j] < seq->tr_ms[j])) return 0;
  return 1;
}

/* Direct factors for one parameter point (computed in the loop's order). */
static int direct_sim(const orc_seq* seq, int32_t n_tr, double t1, double t2,
                      double df, double b1, double* re, double* im,
                      double* states) {
  if (!seq_ok(seq, n_tr)) return 1;
  size_t n = (size_t)(n_tr > 0 ? n_tr : 1);
  double* buf = (double*)malloc(sizeof(double) * n * 12);
  if (!buf) return 2;
  entry_factors f;
  double *e1a = buf, *e1b = buf + n, *e2a = buf + 2 * n, *e2b = buf + 3 * n;
  double *ca = buf + 4 * n, *sa = buf + 5 * n, *cb = buf + 6 * n, *sb = buf + 7 * n;
  double* rf = buf + 8 * n;
  for (int32_t j = 0; j < n_tr; ++j) {
    double ta = seq->te_ms[j], tb = seq->tr_ms[j] - seq->te_ms[j];
    e1a[j] = relax(ta, t1);
    e1b[j] = relax(tb, t1);
    e2a[j] = relax(ta, t2);
    e2b[j] = relax(tb, t2);
    precess(ta, df, &ca[j], &sa[j]);
    precess(tb, df, &cb[j], &sb[j]);
    rf_factors(seq->fa_deg[j], seq->phase_deg[j], b1, rf + 4 * (size_t)j);
  }
  f.e1a = e1a; f.e1b = e1b; f.e2a = e2a; f.e2b = e2b;
  f.ca = ca; f.sa = sa; f.cb = cb; f.sb = sb; f.rf = rf;
  f.e1_ti = relax(seq->ti_ms, t1);
  run_entry(n_tr, seq->inversion, &f, re, im, states);
  free(buf);
  return 0;
}

int orc_simulate(const orc_seq* seq, int32_t n_tr, double t1, double t2,
                 double df, double b1, double* re, double* im) {
  return direct_sim(seq, n_tr, t1, t2, df, b1, re, im, NULL);
}

int orc_trajectory(const orc_seq* seq, int32_t n_tr, double t1, double t2,
                   double df, double b1, double* states) {
  return direct_sim(seq, n_tr, t1, t2, df, b1, NULL, NULL, states);
}

/* ------------------------------------------------------------------------ */
/* Per-axis factor tables: the same functions evaluated once per axis value. */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t n_tr, n1, n2, n3, n4;  /* n4 >= 1 */
  double* t1tab;  /* [n1][2][n_tr] */
  double* t1ti;   /* [n1] */
  double* t2tab;  /* [n2][2][n_tr] */
  double* dftab;  /* [n3][4][n_tr] */
  double* rftab;  /* [n4][n_tr][4] */
  int32_t inversion;
  int32_t smooth;  /* temporal smoothing of dictionary entries: 0, 3 or 5 taps */
  double* demod;   /* [2][n_tr] cos, sin of the RF phase (smoothing frame) */
} tables;

static void tables_free(tables* t) {
  free(t->t1tab); free(t->t1ti); free(t->t2tab); free(t->dftab); free(t->rftab);
  free(t->demod);
  memset(t, 0, sizeof *t);
}

static int tables_build(const orc_seq* seq, const orc_grid* g, int32_t n_tr,
                        tables* t) {
  memset(t, 0, sizeof *t);
  if (!seq_ok(seq, n_tr) || !g || g->n1 < 1 || g->n2 < 1 || g->n3 < 1 || g->n4 < 0)
    return 1;
  if (!(seq->smooth == 0 || seq->smooth == 1 || seq->smooth == 3 || seq->smooth == 5)) return 1;
  t->n_tr = n_tr; t->n1 = g->n1; t->n2 = g->n2; t->n3 = g->n3;
  t->n4 = g->n4 > 0 ? g->n4 : 1;
  t->inversion = seq->inversion;
  t->smooth = seq->smooth > 1 ? seq->smooth : 0;
  size_t n = (size_t)n_tr;
  t->demod = (double*)malloc(sizeof(double) * 2 * n + 8);
  if (!t->demod) return 2;
  for (size_t j = 0; j < n; ++j) {
    const double a = seq->phase_deg[j] * (ORC_PI / 180.0);
    t->demod[j] = cos(a);
    t->demod[n + j] = sin(a);
  }
  t->t1tab = (double*)malloc(sizeof(double) * (size_t)t->n1 * 2 * n + 8);
  t->t1ti = (double*)malloc(sizeof(double) * (size_t)t->n1);
  t->t2tab = (double*)malloc(sizeof(double) * (size_t)t->n2 * 2 * n + 8);
  t->dftab = (double*)malloc(sizeof(double) * (size_t)t->n3 * 4 * n + 8);
  t->rftab = (double*)malloc(sizeof(double) * (size_t)t->n4 * 4 * n + 8);
  if (!t->t1tab || !t->t1ti || !t->t2tab || !t->dftab || !t->rftab) {
    tables_free(t);
    return 2;
  }
  for (int32_t i = 0; i < t->n1; ++i) {
    for (int32_t j = 0; j < n_tr; ++j) {
      double ta = seq->te_ms[j], tb = seq->tr_ms[j] - seq->te_ms[j];
      t->t1tab[((size_t)i * 2 + 0) * n + j] = relax(ta, g->t1[i]);
      t->t1tab[((size_t)i * 2 + 1) * n + j] = relax(tb, g->t1[i]);
    }
    t->t1ti[i] = relax(seq->ti_ms, g->t1[i]);
  }
  for (int32_t i = 0; i < t->n2; ++i)
    for (int32_t j = 0; j < n_tr; ++j) {
      double ta = seq->te_ms[j], tb = seq->tr_ms[j] - seq->te_ms[j];
      t->t2tab[((size_t)i * 2 + 0) * n + j] = relax(ta, g->t2[i]);
      t->t2tab[((size_t)i * 2 + 1) * n + j] = relax(tb, g->t2[i]);
    }
  for (int32_t i = 0; i < t->n3; ++i)
    for (int32_t j = 0; j < n_tr; ++j) {
      double ta = seq->te_ms[j], tb = seq->tr_ms[j] - seq->te_ms[j];
      double* row = t->dftab + (size_t)i * 4 * n;
      precess(ta, g->df[i], &row[0 * n + j], &row[1 * n + j]);
      precess(tb, g->df[i], &row[2 * n + j], &row[3 * n + j]);
    }
  for (int32_t i = 0; i < t->n4; ++i) {
    double b1 = g->n4 > 0 ? g->b1[i] : 1.0;
    for (int32_t j = 0; j < n_tr; ++j)
      rf_factors(seq->fa_deg[j], seq->phase_deg[j], b1,
                 t->rftab + ((size_t)i * n + j) * 4);
  }
  return 0;
}

/* Temporal smoothing (Methods, Experiment 4; Results, Fig. 7B): a moving
 * Gaussian of 3 or 5 points applied along the readouts, here the binomial
 * weights (1, 2, 1) / 4 and (1, 4, 6, 4, 1) / 16; at the first and last
 * readouts the points that exist are used and their weights renormalised.
 * The smoothing acts on the signal as the receiver records it, demodulated
 * by each readout's RF phase (sample j times exp(-i phi_j)); the result is
 * modulated back, so it stays in the frame of the unsmoothed signals. With
 * c = s = NULL the phases are taken as zero. In place; taps 0 or 1 leave the
 * signal unchanged. */
static int smooth_in_frame(int32_t n, int32_t taps, const double* c, const double* s, double* re,
                           double* im) {
  static const double w3[3] = {1.0, 2.0, 1.0};
  static const double w5[5] = {1.0, 4.0, 6.0, 4.0, 1.0};
  if (taps == 0 || taps == 1) return 0;
  if (!(taps == 3 || taps == 5) || n < 0) return 1;
  const double* w = taps == 3 ? w3 : w5;
  const int32_t h = taps / 2;
  double* xr = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  double* xi = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  if (!xr || !xi) {
    free(xr);
    free(xi);
    return 2;
  }
  for (int32_t j = 0; j < n; ++j) {  /* demodulate: (re + i im)(c - i s) */
    const double cj = c ? c[j] : 1.0, sj = s ? s[j] : 0.0;
    xr[j] = re[j] * cj + im[j] * sj;
    xi[j] = im[j] * cj - re[j] * sj;
  }
  for (int32_t j = 0; j < n; ++j) {
    double sr = 0.0, si = 0.0, sw = 0.0;
    for (int32_t k = -h; k <= h; ++k) {
      const int32_t q = j + k;
      if (q < 0 || q >= n) continue;
      sr += w[k + h] * xr[q];
      si += w[k + h] * xi[q];
      sw += w[k + h];
    }
    sr /= sw;
    si /= sw;
    const double cj = c ? c[j] : 1.0, sj = s ? s[j] : 0.0;  /* modulate back: (sr + i si)(c + i s) */
    re[j] = sr * cj - si * sj;
    im[j] = sr * sj + si * cj;
  }
  free(xr);
  free(xi);
  return 0;
}

int orc_smooth(int32_t n, int32_t taps, const double* phase_deg, double* re, double* im) {
  if (!phase_deg || taps == 0 || taps == 1) return smooth_in_frame(n, taps, NULL, NULL, re, im);
  if (n < 0) return 1;
  double* cs = (double*)malloc(sizeof(double) * 2 * (size_t)(n + 1));
  if (!cs) return 2;
  for (int32_t j = 0; j < n; ++j) {
    const double a = phase_deg[j] * (ORC_PI / 180.0);
    cs[j] = cos(a);
    cs[n + j] = sin(a);
  }
  const int rc = smooth_in_frame(n, taps, cs, cs + n, re, im);
  free(cs);
  return rc;
}

/* The samples of dictionary entry f: the recursion, then the sequence's
 * temporal smoothing (if any). */
static void entry_samples(const tables* t, const entry_factors* f, double* re, double* im) {
  run_entry(t->n_tr, t->inversion, f, re, im, NULL);
  if (t->smooth)
    smooth_in_frame(t->n_tr, t->smooth, t->demod, t->demod + t->n_tr, re, im);
}

static void tables_view(const tables* t, int64_t k, entry_factors* f) {
  int32_t i4 = (int32_t)(k % t->n4);
  k /= t->n4;
  int32_t i3 = (int32_t)(k % t->n3);
  k /= t->n3;
  int32_t i2 = (int32_t)(k % t->n2);
  int32_t i1 = (int32_t)(k / t->n2);
  size_t n = (size_t)t->n_tr;
  f->e1a = t->t1tab + ((size_t)i1 * 2 + 0) * n;
  f->e1b = t->t1tab + ((size_t)i1 * 2 + 1) * n;
  f->e2a = t->t2tab + ((size_t)i2 * 2 + 0) * n;
  f->e2b = t->t2tab + ((size_t)i2 * 2 + 1) * n;
  const double* row = t->dftab + (size_t)i3 * 4 * n;
  f->ca = row; f->sa = row + n; f->cb = row + 2 * n; f->sb = row + 3 * n;
  f->rf = t->rftab + (size_t)i4 * n * 4;
  f->e1_ti = t->t1ti[i1];
}

static int64_t grid_size(const orc_grid* g) {
  return (int64_t)g->n1 * g->n2 * g->n3 * (g->n4 > 0 ? g->n4 : 1);
}

static double norm2(int32_t n, const double* re, const double* im) {
  double s = 0.0;
  for (int32_t j = 0; j < n; ++j) s += re[j] * re[j] + im[j] * im[j];
  return s;
}

int orc_simulate_grid(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
                      int64_t k0, int64_t count, double* re, double* im,
                      double* norm, int32_t n_threads) {
  tables t;
  if (!grid || k0 < 0 || count < 0 || k0 + count > grid_size(grid)) return 1;
  int rc = tables_build(seq, grid, n_tr, &t);
  if (rc) return rc;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t e = 0; e < count; ++e) {
    entry_factors f;
    tables_view(&t, k0 + e, &f);
    double* r = re + (size_t)e * n_tr;
    double* i = im + (size_t)e * n_tr;
    entry_samples(&t, &f, r, i);
    if (norm) norm[e] = sqrt(norm2(n_tr, r, i));
  }
  tables_free(&t);
  return 0;
}

/* Eq. 1: |sum_j v_j conj(d_j)| / (||v|| ||d||); 0 when a norm is 0. */
static void cdot(int32_t n, const double* vr, const double* vi, const double* dr,
                 const double* di, double* sr, double* si) {
  double a = 0.0, b = 0.0;
  for (int32_t j = 0; j < n; ++j) {
    /* (vr + i vi)(dr - i di) */
    a += vr[j] * dr[j] + vi[j] * di[j];
    b += vi[j] * dr[j] - vr[j] * di[j];
  }
  *sr = a;
  *si = b;
}

double orc_cc(int32_t n, const double* vr, const double* vi, const double* dr,
              const double* di) {
  double nv = sqrt(norm2(n, vr, vi)), nd = sqrt(norm2(n, dr, di));
  if (nv == 0.0 || nd == 0.0) return 0.0;
  double sr, si;
  cdot(n, vr, vi, dr, di, &sr, &si);
  return sqrt(sr * sr + si * si) / (nv * nd);
}

/* ------------------------------------------------------------------------ */
/* Brute force: every entry, every voxel; top lists ordered by (CC desc, k asc). */
/* ------------------------------------------------------------------------ */

static int better(double ca, int64_t ka, double cb, int64_t kb) {
  return ca > cb || (ca == cb && ka < kb);
}

/* insert (c, k) into a list of length L sorted best-first */
static void top_insert(double* lc, int64_t* lk, int32_t L, double c, int64_t k) {
  if (!better(c, k, lc[L - 1], lk[L - 1])) return;
  int32_t p = L - 1;
  while (p > 0 && better(c, k, lc[p - 1], lk[p - 1])) {
    lc[p] = lc[p - 1];
    lk[p] = lk[p - 1];
    --p;
  }
  lc[p] = c;
  lk[p] = k;
}

int orc_bruteforce(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
                   const double* vr, const double* vi, int32_t n_vox,
                   int32_t top_k, int64_t* idx, double* cc, double* margin,
                   double* pd_re, double* pd_im, int64_t* topk_idx,
                   double* topk_cc, int32_t n_threads) {
  if (!grid || n_vox < 0 || top_k < 1 || (n_vox > 0 && (!vr || !vi))) return 1;
  tables t;
  int rc = tables_build(seq, grid, n_tr, &t);
  if (rc) return rc;
  const int64_t E = grid_size(grid);
  const int32_t L = top_k > 2 ? top_k : 2;
  double* vnorm = (double*)malloc(sizeof(double) * (size_t)(n_vox + 1));
  for (int32_t v = 0; v < n_vox; ++v)
    vnorm[v] = sqrt(norm2(n_tr, vr + (size_t)v * n_tr, vi + (size_t)v * n_tr));
  int nth = 1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
  nth = omp_get_max_threads();
#endif
  size_t lsz = (size_t)nth * n_vox * L;
  double* allc = (double*)malloc(sizeof(double) * (lsz + 1));
  int64_t* allk = (int64_t*)malloc(sizeof(int64_t) * (lsz + 1));
  for (size_t i = 0; i < lsz; ++i) { allc[i] = -INFINITY; allk[i] = INT64_MAX; }
#ifdef _OPENMP
#pragma omp parallel
#endif
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* re = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
    double* im = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
    double* myc = allc + (size_t)tid * n_vox * L;
    int64_t* myk = allk + (size_t)tid * n_vox * L;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
    for (int64_t k = 0; k < E; ++k) {
      entry_factors f;
      tables_view(&t, k, &f);
      entry_samples(&t, &f, re, im);
      double nd = sqrt(norm2(n_tr, re, im));
      for (int32_t v = 0; v < n_vox; ++v) {
        double c = 0.0;
        if (nd != 0.0 && vnorm[v] != 0.0) {
          double sr, si;
          cdot(n_tr, vr + (size_t)v * n_tr, vi + (size_t)v * n_tr, re, im, &sr, &si);
          c = sqrt(sr * sr + si * si) / (vnorm[v] * nd);
        }
        top_insert(myc + (size_t)v * L, myk + (size_t)v * L, L, c, k);
      }
    }
    free(re);
    free(im);
  }
  /* merge the per-thread lists (the order is total, so the result does not
   * depend on how entries were split among threads) */
  double* re = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
  double* im = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
  double* lc = (double*)malloc(sizeof(double) * L);
  int64_t* lk = (int64_t*)malloc(sizeof(int64_t) * L);
  for (int32_t v = 0; v < n_vox; ++v) {
    for (int32_t i = 0; i < L; ++i) { lc[i] = -INFINITY; lk[i] = INT64_MAX; }
    for (int th = 0; th < nth; ++th)
      for (int32_t i = 0; i < L; ++i) {
        size_t o = ((size_t)th * n_vox + v) * L + i;
        if (allk[o] != INT64_MAX) top_insert(lc, lk, L, allc[o], allk[o]);
      }
    if (idx) idx[v] = lk[0];
    if (cc) cc[v] = lc[0];
    if (margin) margin[v] = (lk[1] == INT64_MAX) ? INFINITY : lc[0] - lc[1];
    for (int32_t i = 0; i < top_k; ++i) {
      if (topk_idx) topk_idx[(size_t)v * top_k + i] = lk[i] == INT64_MAX ? -1 : lk[i];
      if (topk_cc) topk_cc[(size_t)v * top_k + i] = lc[i];
    }
    if ((pd_re || pd_im) && lk[0] != INT64_MAX) {
      /* proton density from the scale: <v, d> / ||d||^2 (Theory section) */
      entry_factors f;
      tables_view(&t, lk[0], &f);
      entry_samples(&t, &f, re, im);
      double n2d = norm2(n_tr, re, im), sr = 0.0, si = 0.0;
      cdot(n_tr, vr + (size_t)v * n_tr, vi + (size_t)v * n_tr, re, im, &sr, &si);
      if (pd_re) pd_re[v] = n2d > 0.0 ? sr / n2d : 0.0;
      if (pd_im) pd_im[v] = n2d > 0.0 ? si / n2d : 0.0;
    }
  }
  free(re); free(im); free(lc); free(lk);
  free(allc); free(allk); free(vnorm);
  tables_free(&t);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* CC map (Methods and Results, Experiment 1): the CC of Eq. 1 between each   */
/* fingerprint and every entry of [k0, k0 + count), written out in full.      */
/* ------------------------------------------------------------------------ */

int orc_cc_map(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
               const double* vr, const double* vi, int32_t n_vox, int64_t k0,
               int64_t count, double* out, int32_t n_threads) {
  if (!grid || n_vox < 0 || count < 0 || k0 < 0 ||
      (n_vox > 0 && count > 0 && (!vr || !vi || !out)))
    return 1;
  tables t;
  int rc = tables_build(seq, grid, n_tr, &t);
  if (rc) return rc;
  if (k0 + count > grid_size(grid)) {
    tables_free(&t);
    return 1;
  }
  double* vnorm = (double*)malloc(sizeof(double) * (size_t)(n_vox + 1));
  for (int32_t v = 0; v < n_vox; ++v)
    vnorm[v] = sqrt(norm2(n_tr, vr + (size_t)v * n_tr, vi + (size_t)v * n_tr));
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
  {
    double* re = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
    double* im = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < count; ++i) {
      entry_factors f;
      tables_view(&t, k0 + i, &f);
      entry_samples(&t, &f, re, im);
      double nd = sqrt(norm2(n_tr, re, im));
      for (int32_t v = 0; v < n_vox; ++v) {
        double c = 0.0;
        if (nd != 0.0 && vnorm[v] != 0.0) {
          double sr, si;
          cdot(n_tr, vr + (size_t)v * n_tr, vi + (size_t)v * n_tr, re, im, &sr, &si);
          c = sqrt(sr * sr + si * si) / (vnorm[v] * nd);
        }
        out[(size_t)v * count + i] = c;
      }
    }
    free(re);
    free(im);
  }
  free(vnorm);
  tables_free(&t);
  return 0;
}

/* CC (Eq. 1) of voxel v against the listed entries idx[v*m + i] (a
 * negative index gives 0): the plain definition at chosen points, used to
 * check a search's answer where several answers are within tolerance. */
int orc_cc_at(const orc_seq* seq, const orc_grid* grid, int32_t n_tr, const double* vr,
              const double* vi, int32_t n_vox, int32_t m, const int64_t* idx, double* out,
              int32_t n_threads) {
  if (!grid || n_vox < 0 || m < 0 || (n_vox > 0 && m > 0 && (!vr || !vi || !idx || !out)))
    return 1;
  tables t;
  int rc = tables_build(seq, grid, n_tr, &t);
  if (rc) return rc;
  const int64_t E = grid_size(grid);
  for (int64_t q = 0; q < (int64_t)n_vox * m; ++q)
    if (idx[q] >= E) {
      tables_free(&t);
      return 1;
    }
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
  {
    double* re = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
    double* im = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
    for (int64_t q = 0; q < (int64_t)n_vox * m; ++q) {
      const int64_t v = q / m;
      if (idx[q] < 0) {
        out[q] = 0.0;
        continue;
      }
      entry_factors f;
      tables_view(&t, idx[q], &f);
      entry_samples(&t, &f, re, im);
      out[q] = orc_cc(n_tr, vr + (size_t)v * n_tr, vi + (size_t)v * n_tr, re, im);
    }
    free(re);
    free(im);
  }
  tables_free(&t);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* ZOOM (Theory: MRF ZOOM; Methods: Experiment 2 procedure).                 */
/* ------------------------------------------------------------------------ */

static int32_t round_half_away(double x) {
  return (int32_t)(x >= 0.0 ? floor(x + 0.5) : -floor(-x + 0.5));
}

/* physical step r on an axis -> index step, at least 1 */
static int32_t idx_step(double r, const double* ax, int32_t n) {
  if (n < 2) return 1;
  double d = (ax[n - 1] - ax[0]) / (double)(n - 1);
  int32_t s = round_half_away(r / d);
  return s < 1 ? 1 : s;
}

static int32_t nearest(const double* ax, int32_t n, double v) {
  int32_t b = 0;
  for (int32_t i = 1; i < n; ++i)
    if (fabs(ax[i] - v) < fabs(ax[b] - v)) b = i;
  return b;
}

static orc_stage mk(int32_t kind, int32_t a0, int32_t a1, int32_t s0, int32_t s1,
                    int32_t w, double hop) {
  orc_stage s;
  s.kind = kind; s.axis0 = a0; s.axis1 = a1; s.step0 = s0; s.step1 = s1;
  s.window = w; s.hop = hop;
  return s;
}

/* Methods, Experiment 2, zooming steps 1-5, converted to index steps. */
int orc_schedule_paper(const orc_grid* g, const orc_seq* seq, orc_schedule* o) {
  if (!g || !seq || !o || seq->n < 1) return 1;
  memset(o, 0, sizeof *o);
  double trmin = seq->tr_ms[0];
  for (int32_t j = 1; j < seq->n; ++j)
    if (seq->tr_ms[j] < trmin) trmin = seq->tr_ms[j];
  double omega = 1000.0 / trmin;  /* pseudo-period of CC in df (Property II) */
  const double *T1 = g->t1, *T2 = g->t2, *DF = g->df;
  int32_t n1 = g->n1, n2 = g->n2, n3 = g->n3;
  double ddf = n3 > 1 ? (DF[n3 - 1] - DF[0]) / (double)(n3 - 1) : 1.0;
  int32_t k = 0;
  /* step 1: df at the starting T1/T2 */
  o->stages[k++] = mk(ORC_SCAN_STRIDE, 2, 0, idx_step(60.0, DF, n3), 0, 0, 0.0);
  o->stages[k++] = mk(ORC_SCAN_WINDOW, 2, 0, idx_step(3.0, DF, n3), 0,
                      idx_step(75.0, DF, n3), 0.0);
  double hop = omega / ddf;
  o->stages[k++] = mk(ORC_SCAN_HOPS, 2, 0, 0, 0, 0, hop < 1.0 ? 1.0 : hop);
  /* step 2: 2-D zoom at 200 then 100 ms */
  o->stages[k++] = mk(ORC_ZOOM2, 0, 1, idx_step(200.0, T1, n1), idx_step(200.0, T2, n2), 0, 0.0);
  o->stages[k++] = mk(ORC_ZOOM2, 0, 1, idx_step(100.0, T1, n1), idx_step(100.0, T2, n2), 0, 0.0);
  /* step 3: finest df scan over +-omega/2 */
  o->stages[k++] = mk(ORC_SCAN_WINDOW, 2, 0, 1, 0, idx_step(0.5 * omega, DF, n3), 0.0);
  /* step 4: interleaved 1-D zooms */
  o->stages[k++] = mk(ORC_ZOOM1, 0, 0, idx_step(100.0, T1, n1), 0, 0, 0.0);
  o->stages[k++] = mk(ORC_ZOOM1, 1, 0, idx_step(100.0, T2, n2), 0, 0, 0.0);
  o->stages[k++] = mk(ORC_ZOOM1, 0, 0, idx_step(50.0, T1, n1), 0, 0, 0.0);
  o->stages[k++] = mk(ORC_ZOOM1, 0, 0, idx_step(20.0, T1, n1), 0, 0, 0.0);
  o->stages[k++] = mk(ORC_ZOOM1, 0, 0, idx_step(10.0, T1, n1), 0, 0, 0.0);
  o->stages[k++] = mk(ORC_ZOOM1, 1, 0, idx_step(50.0, T2, n2), 0, 0, 0.0);
  o->stages[k++] = mk(ORC_ZOOM1, 1, 0, idx_step(20.0, T2, n2), 0, 0, 0.0);
  o->stages[k++] = mk(ORC_ZOOM1, 1, 0, idx_step(10.0, T2, n2), 0, 0, 0.0);
  if (g->n4 > 1) {
    /* fourth parameter (extension; not in the paper's schedule) */
    const double steps[5] = {0.1, 0.05, 0.02, 0.01, 0.005};
    for (int i = 0; i < 5; ++i)
      o->stages[k++] = mk(ORC_ZOOM1, 3, 0, idx_step(steps[i], g->b1, g->n4), 0, 0, 0.0);
  }
  /* step 5: final 2-D zoom at the finest resolution */
  o->stages[k++] = mk(ORC_ZOOM2, 0, 1, 1, 1, 0, 0.0);
  o->n_stages = k;
  if (g->n4 > 1) {
    o->outer[0] = mk(ORC_ZOOM2, 0, 1, 1, 1, 0, 0.0);
    o->outer[1] = mk(ORC_ZOOM1, 3, 0, 1, 0, 0, 0.0);
    o->outer[2] = mk(ORC_SCAN_WINDOW, 2, 0, 1, 0, idx_step(0.5 * omega, DF, n3), 0.0);
    o->n_outer = 3;
    o->outer_max = 3;
  }
  o->n_starts = 1;
  o->starts[0][0] = nearest(T1, n1, 1000.0);
  o->starts[0][1] = nearest(T2, n2, 500.0);
  o->starts[0][2] = 0;
  o->starts[0][3] = g->n4 > 1 ? nearest(g->b1, g->n4, 1.0) : 0;
  o->pruned = 0;
  for (int a = 0; a < 4; ++a) o->prior_half[a] = -1;
  return 0;
}

/* The paper's stages from several initial values (Methods, Experiment 2;
 * Discussion: a second searching process after approximate T1 and T2):
 * k1 x k2 starts spread evenly over the T1 and T2 index ranges, ends
 * included, df index 0; afterwards the rounds [df scan of step 3 within the
 * 75 Hz window, finest df scan, 2-D zooms at 100, 50, 20, 10 ms and at unit
 * steps (+ unit B1 zoom)] repeat at most outer_max times while the centre
 * moves. */
int orc_schedule_multistart(const orc_grid* g, const orc_seq* seq, int32_t k1, int32_t k2,
                            int32_t outer_max, orc_schedule* o) {
  if (orc_schedule_paper(g, seq, o)) return 1;
  if (k1 < 1 || k2 < 1 || k1 * k2 > ORC_MAX_STARTS || outer_max < 0) return 1;
  int32_t b1 = o->starts[0][3];
  o->n_starts = 0;
  for (int32_t a = 0; a < k1; ++a) {
    for (int32_t b = 0; b < k2; ++b) {
      int32_t* st = o->starts[o->n_starts++];
      st[0] = k1 == 1 ? (g->n1 - 1) / 2 : round_half_away((double)a * (g->n1 - 1) / (k1 - 1));
      st[1] = k2 == 1 ? (g->n2 - 1) / 2 : round_half_away((double)b * (g->n2 - 1) / (k2 - 1));
      st[2] = 0;
      st[3] = b1;
    }
  }
  int32_t n = 0;
  o->outer[n++] = o->stages[1]; /* df window, step 3 Hz */
  o->outer[n++] = o->stages[5]; /* finest df scan */
  const double r[4] = {100.0, 50.0, 20.0, 10.0};
  for (int i = 0; i < 4; ++i)
    o->outer[n++] = mk(ORC_ZOOM2, 0, 1, idx_step(r[i], g->t1, g->n1), idx_step(r[i], g->t2, g->n2),
                       0, 0.0);
  o->outer[n++] = mk(ORC_ZOOM2, 0, 1, 1, 1, 0, 0.0);
  if (g->n4 > 1) o->outer[n++] = mk(ORC_ZOOM1, 3, 0, 1, 0, 0, 0.0);
  o->n_outer = n;
  o->outer_max = outer_max;
  return 0;
}

/* Neighbour prior (Methods, Experiment 3): the ranges T1p +- 3000 ms,
 * T2p +- 800 ms and dfp +- 150 Hz around a neighbour's result, intersected
 * with the search ranges. Here the half widths are given physically (B1 is
 * an extension; its default is +- 0.3) and converted to index steps like
 * every other physical step of the schedule: max(1, round_half_away(r /
 * ((max - min)/(n - 1)))). An axis of fewer than two values, or a negative
 * half width, gets -1 (the whole axis). */
int orc_prior_half(const orc_grid* g, const double* half, int32_t* out) {
  if (!g || !out) return 1;
  static const double dflt[4] = {3000.0, 800.0, 150.0, 0.3};
  const double* h = half ? half : dflt;
  const double* ax[4] = {g->t1, g->t2, g->df, g->b1};
  const int32_t n[4] = {g->n1, g->n2, g->n3, g->n4};
  for (int a = 0; a < 4; ++a) {
    if (n[a] < 2 || !(h[a] >= 0.0) || !ax[a]) {
      out[a] = -1;
      continue;
    }
    out[a] = idx_step(h[a], ax[a], n[a]);
  }
  return 0;
}

/* Finest resolution (Discussion): the stages at unit index steps get the
 * given objective. */
static int finest_stage(const orc_stage* st) {
  if (st->kind == ORC_ZOOM2) return st->step0 <= 1 && st->step1 <= 1;
  if (st->kind == ORC_ZOOM1 || st->kind == ORC_SCAN_WINDOW || st->kind == ORC_SCAN_STRIDE)
    return st->step0 <= 1;
  return 0;
}

int orc_schedule_finest_objective(orc_schedule* s, int32_t objective) {
  if (!s || (objective != ORC_OBJ_CC && objective != ORC_OBJ_DIST)) return 1;
  if (s->n_stages < 0 || s->n_stages > ORC_MAX_STAGES || s->n_outer < 0 ||
      s->n_outer > ORC_MAX_STAGES)
    return 1;
  for (int i = 0; i < s->n_stages; ++i)
    if (finest_stage(&s->stages[i])) s->stages[i].objective = objective;
  for (int i = 0; i < s->n_outer; ++i)
    if (finest_stage(&s->outer[i])) s->outer[i].objective = objective;
  return 0;
}

/* memo: open addressing, key = entry index, both objective values per key */
typedef struct {
  int64_t* keys;
  double* vals; /* [cap][2] */
  int64_t cap, count;
} memo_t;

static void memo_alloc(memo_t* m, int64_t cap) {
  m->cap = cap;
  m->count = 0;
  m->keys = (int64_t*)malloc(sizeof(int64_t) * m->cap);
  m->vals = (double*)malloc(sizeof(double) * 2 * m->cap);
  for (int64_t i = 0; i < m->cap; ++i) m->keys[i] = -1;
}
static void memo_init(memo_t* m) { memo_alloc(m, 1024); }
static void memo_free(memo_t* m) { free(m->keys); free(m->vals); }
static int64_t memo_slot(const memo_t* m, int64_t key) {
  uint64_t h = (uint64_t)key * 0x9E3779B97F4A7C15ull;
  int64_t s = (int64_t)(h >> 20) & (m->cap - 1);
  while (m->keys[s] != -1 && m->keys[s] != key) s = (s + 1) & (m->cap - 1);
  return s;
}
static void memo_put(memo_t* m, int64_t key, const double* v);
static void memo_grow(memo_t* m) {
  memo_t n;
  memo_alloc(&n, m->cap * 2);
  for (int64_t i = 0; i < m->cap; ++i)
    if (m->keys[i] != -1) memo_put(&n, m->keys[i], m->vals + 2 * i);
  memo_free(m);
  *m = n;
}
static void memo_put(memo_t* m, int64_t key, const double* v) {
  if (2 * (m->count + 1) > m->cap) memo_grow(m);
  int64_t s = memo_slot(m, key);
  if (m->keys[s] == -1) m->count++;
  m->keys[s] = key;
  m->vals[2 * s] = v[0];
  m->vals[2 * s + 1] = v[1];
}

typedef struct {
  const orc_schedule* sch;
  int32_t dims[4];
  int32_t lo[4], hi[4];
  orc_objective2 obj;
  void* ctx;
  int32_t cur_obj; /* objective of the stage being run */
  memo_t memo;
  double min_margin;
  int32_t n_eval;
  /* centre state */
  int32_t c[4];
  double cval;
  int cknown;
  /* optional move log: 5 ints per move (new centre, evaluations so far) */
  int32_t* path;
  int32_t path_cap, path_len;
} engine;

static int64_t key_of(const engine* e, const int32_t* i) {
  return (((int64_t)i[0] * e->dims[1] + i[1]) * e->dims[2] + i[2]) * e->dims[3] + i[3];
}

static double eval_at(engine* e, const int32_t* i) {
  for (int a = 0; a < 4; ++a)
    if (i[a] < e->lo[a] || i[a] > e->hi[a]) return -INFINITY;
  int64_t key = key_of(e, i);
  int64_t s = memo_slot(&e->memo, key);
  if (e->memo.keys[s] == key) return e->memo.vals[2 * s + e->cur_obj];
  double v[2];
  e->obj(e->ctx, i, v);
  memo_put(&e->memo, key, v);
  e->n_eval++;
  return v[e->cur_obj];
}

static void need_centre(engine* e) {
  if (!e->cknown) {
    e->cval = eval_at(e, e->c);
    e->cknown = 1;
  }
}

/* margin of one decision: best minus runner-up among finite compared values */
static void log_decision(engine* e, const double* v, int n) {
  double b1 = -INFINITY, b2 = -INFINITY;
  int nf = 0;
  for (int i = 0; i < n; ++i) {
    if (!isfinite(v[i])) continue;
    ++nf;
    if (v[i] > b1) { b2 = b1; b1 = v[i]; }
    else if (v[i] > b2) b2 = v[i];
  }
  if (nf >= 2 && b1 - b2 < e->min_margin) e->min_margin = b1 - b2;
}

static void log_pair(engine* e, double a, double b) {
  if (isfinite(a) && isfinite(b) && fabs(a - b) < e->min_margin) e->min_margin = fabs(a - b);
}

/* value list grown on the heap for scans */
typedef struct { double* v; int32_t n, cap; } vlist;
static void vl_push(vlist* l, double x) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 64;
    l->v = (double*)realloc(l->v, sizeof(double) * l->cap);
  }
  l->v[l->n++] = x;
}

static void stage_scan_stride(engine* e, const orc_stage* st) {
  int a = st->axis0, s = st->step0 > 0 ? st->step0 : 1;
  int32_t i[4];
  memcpy(i, e->c, sizeof i);
  double best = -INFINITY;
  int32_t bp = e->c[a];
  vlist l = {0, 0, 0};
  for (int32_t p = e->lo[a]; p <= e->hi[a]; p += s) {
    i[a] = p;
    double v = eval_at(e, i);
    vl_push(&l, v);
    if (v > best) { best = v; bp = p; }
  }
  log_decision(e, l.v, l.n);
  free(l.v);
  if (isfinite(best)) {
    e->c[a] = bp;
    e->cval = best;
    e->cknown = 1;
  }
}

/* scan over explicit points (increasing), the centre kept on ties */
static void scan_points(engine* e, int a, const int32_t* pts, int32_t np) {
  need_centre(e);
  int32_t i[4];
  memcpy(i, e->c, sizeof i);
  double best = e->cval;
  int32_t bp = e->c[a];
  vlist l = {0, 0, 0};
  vl_push(&l, e->cval);
  for (int32_t q = 0; q < np; ++q) {
    i[a] = pts[q];
    double v = eval_at(e, i);
    vl_push(&l, v);
    if (v > best) { best = v; bp = pts[q]; }
  }
  log_decision(e, l.v, l.n);
  free(l.v);
  e->c[a] = bp;
  e->cval = best;
}

static void stage_scan_window(engine* e, const orc_stage* st) {
  int a = st->axis0, s = st->step0 > 0 ? st->step0 : 1;
  int32_t m = st->window / s;
  int32_t* pts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  int32_t np = 0;
  for (int32_t q = -m; q <= m; ++q) {
    if (q == 0) continue;
    int32_t p = e->c[a] + q * s;
    if (p < e->lo[a] || p > e->hi[a]) continue;
    pts[np++] = p;
  }
  scan_points(e, a, pts, np);
  free(pts);
}

static void stage_scan_hops(engine* e, const orc_stage* st) {
  int a = st->axis0;
  double h = st->hop >= 1.0 ? st->hop : 1.0;
  int32_t c = e->c[a];
  int32_t span = e->hi[a] - e->lo[a] + 1;
  int32_t* neg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(span + 1));
  int32_t* pts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * span + 2));
  int32_t nn = 0, np = 0;
  for (int32_t k = 1;; ++k) {
    int32_t p = c + round_half_away(-(double)k * h);
    if (p < e->lo[a]) break;
    if (nn == 0 || neg[nn - 1] != p) neg[nn++] = p;
  }
  for (int32_t q = nn - 1; q >= 0; --q) pts[np++] = neg[q];
  for (int32_t k = 1;; ++k) {
    int32_t p = c + round_half_away((double)k * h);
    if (p > e->hi[a]) break;
    if (np == 0 || pts[np - 1] != p) pts[np++] = p;
  }
  scan_points(e, a, pts, np);
  free(neg);
  free(pts);
}

static void move_to(engine* e, const int32_t* i, double v) {
  memcpy(e->c, i, sizeof e->c);
  e->cval = v;
  if (e->path && e->path_len < e->path_cap) {
    int32_t* p = e->path + 5 * (size_t)e->path_len++;
    memcpy(p, i, sizeof(int32_t) * 4);
    p[4] = e->n_eval;
  }
}

static void stage_zoom1(engine* e, const orc_stage* st, int pruned) {
  int a = st->axis0, s = st->step0 > 0 ? st->step0 : 1;
  need_centre(e);
  for (;;) {
    int32_t L[4], R[4];
    memcpy(L, e->c, sizeof L);
    memcpy(R, e->c, sizeof R);
    L[a] -= s;
    R[a] += s;
    if (pruned) {
      double vr = eval_at(e, R);
      log_pair(e, vr, e->cval);
      if (vr > e->cval) { move_to(e, R, vr); continue; }
      double vl = eval_at(e, L);
      log_pair(e, vl, e->cval);
      if (vl > e->cval) { move_to(e, L, vl); continue; }
      break;
    }
    double vl = eval_at(e, L), vr = eval_at(e, R);
    double vals[3] = {e->cval, vl, vr};
    log_decision(e, vals, 3);
    const int32_t* bi = L;
    double bv = vl;
    if (vr > bv) { bv = vr; bi = R; }
    if (bv > e->cval) move_to(e, bi, bv);
    else break;
  }
}

/* neighbour offsets in the fixed order L, R, D, U, LD, LU, RD, RU */
static const int NB[8][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1},
                             {-1, -1}, {-1, 1}, {1, -1}, {1, 1}};
enum { NL = 0, NR, ND, NU, NLD, NLU, NRD, NRU };

static void nb_index(const engine* e, const orc_stage* st, int which, int32_t* out) {
  memcpy(out, e->c, sizeof(int32_t) * 4);
  out[st->axis0] += NB[which][0] * (st->step0 > 0 ? st->step0 : 1);
  out[st->axis1] += NB[which][1] * (st->step1 > 0 ? st->step1 : 1);
}

/* one pruned 2-D move; returns 1 if the centre moved */
static int zoom2_pruned_move(engine* e, const orc_stage* st) {
  int32_t p[8][4];
  double v[8];
  int have[8] = {0};
  for (int w = 0; w < 8; ++w) nb_index(e, st, w, p[w]);
#define EV(w) (have[w] ? v[w] : (have[w] = 1, v[w] = eval_at(e, p[w])))
#define UP(w) (EV(w) > e->cval)
  double C = e->cval;
  int upL = UP(NL), upD = UP(ND);
  log_pair(e, v[NL], C);
  log_pair(e, v[ND], C);
  int target = -1;
  int cand[3];
  int nc = 0;
  if (upL && upD) {
    cand[nc++] = NL; cand[nc++] = ND;
    EV(NLD); log_pair(e, v[NLD], C);
    if (v[NLD] > C) target = NLD;
  } else if (!upL && !upD) {
    int upR = UP(NR), upU = UP(NU);
    log_pair(e, v[NR], C);
    log_pair(e, v[NU], C);
    if (!upR && !upU) return 0;
    if (upR && upU) {
      cand[nc++] = NR; cand[nc++] = NU;
      EV(NRU); log_pair(e, v[NRU], C);
      if (v[NRU] > C) target = NRU;
    } else {
      target = upR ? NR : NU;
    }
  } else if (upL) { /* L > C, D not */
    cand[nc++] = NL;
    int upU = UP(NU);
    log_pair(e, v[NU], C);
    if (upU) {
      cand[nc++] = NU;
      EV(NLU); log_pair(e, v[NLU], C);
      if (v[NLU] > C) target = NLU;
    } else {
      target = NL;
    }
  } else { /* D > C, L not */
    cand[nc++] = ND;
    int upR = UP(NR);
    log_pair(e, v[NR], C);
    if (upR) {
      cand[nc++] = NR;
      EV(NRD); log_pair(e, v[NRD], C);
      if (v[NRD] > C) target = NRD;
    } else {
      target = ND;
    }
  }
#undef EV
#undef UP
  if (target < 0) {
    /* corner not better: best evaluated edge point that beats the centre,
     * ties broken by the fixed neighbour order */
    double bv = -INFINITY;
    for (int w = 0; w < 8; ++w) {
      int in = 0;
      for (int q = 0; q < nc; ++q) in |= cand[q] == w;
      if (in && v[w] > bv) { bv = v[w]; target = w; }
    }
    if (target < 0 || !(bv > C)) return 0;
  }
  move_to(e, p[target], v[target]);
  return 1;
}

static void stage_zoom2(engine* e, const orc_stage* st, int pruned) {
  need_centre(e);
  for (;;) {
    if (pruned) {
      if (!zoom2_pruned_move(e, st)) break;
      continue;
    }
    int32_t p[8][4];
    double vals[9];
    vals[0] = e->cval;
    int bw = -1;
    double bv = -INFINITY;
    for (int w = 0; w < 8; ++w) {
      nb_index(e, st, w, p[w]);
      vals[w + 1] = eval_at(e, p[w]);
      if (vals[w + 1] > bv) { bv = vals[w + 1]; bw = w; }
    }
    log_decision(e, vals, 9);
    if (bw >= 0 && bv > e->cval) move_to(e, p[bw], bv);
    else break;
  }
}

static void run_stage(engine* e, const orc_stage* st) {
  const int32_t obj = st->objective == ORC_OBJ_DIST ? ORC_OBJ_DIST : ORC_OBJ_CC;
  if (obj != e->cur_obj) {
    /* the centre's value under this stage's objective (a memo hit) */
    e->cur_obj = obj;
    e->cknown = 0;
  }
  switch (st->kind) {
    case ORC_SCAN_STRIDE: stage_scan_stride(e, st); break;
    case ORC_SCAN_WINDOW: stage_scan_window(e, st); break;
    case ORC_SCAN_HOPS: stage_scan_hops(e, st); break;
    case ORC_ZOOM1: stage_zoom1(e, st, e->sch->pruned); break;
    case ORC_ZOOM2: stage_zoom2(e, st, e->sch->pruned); break;
    default: break;
  }
}

static int sched_ok(const orc_schedule* s) {
  if (!s || s->n_stages < 0 || s->n_stages > ORC_MAX_STAGES || s->n_outer < 0 ||
      s->n_outer > ORC_MAX_STAGES || s->n_starts < 0 || s->n_starts > ORC_MAX_STARTS)
    return 0;
  return 1;
}

/* One voxel: every start runs the whole schedule; the best final value wins
 * (ties: lower entry index). The memo is shared across starts. */
static void engine_run(engine* e, const int32_t* init, int32_t* best_idx,
                       double* best_vals) {
  const orc_schedule* s = e->sch;
  for (int a = 0; a < 4; ++a) {
    e->lo[a] = 0;
    e->hi[a] = e->dims[a] - 1;
    if (init && s->prior_half[a] >= 0) {
      e->lo[a] = init[a] - s->prior_half[a] < 0 ? 0 : init[a] - s->prior_half[a];
      e->hi[a] = init[a] + s->prior_half[a] > e->dims[a] - 1 ? e->dims[a] - 1
                                                             : init[a] + s->prior_half[a];
    }
  }
  int nst = init ? 1 : s->n_starts;
  double bv = -INFINITY;
  int32_t bi[4] = {0, 0, 0, 0};
  int64_t bk = INT64_MAX;
  double* finals = (double*)malloc(sizeof(double) * (size_t)(nst + 1));
  int64_t* fkeys = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nst + 1));
  for (int q = 0; q < nst; ++q) {
    const int32_t* st = init ? init : s->starts[q];
    for (int a = 0; a < 4; ++a) {
      int32_t v = st[a];
      e->c[a] = v < e->lo[a] ? e->lo[a] : (v > e->hi[a] ? e->hi[a] : v);
    }
    e->cknown = 0;
    e->cur_obj = ORC_OBJ_CC;
    for (int i = 0; i < s->n_stages; ++i) run_stage(e, &s->stages[i]);
    for (int r = 0; r < s->outer_max && s->n_outer > 0; ++r) {
      int32_t before[4];
      memcpy(before, e->c, sizeof before);
      for (int i = 0; i < s->n_outer; ++i) run_stage(e, &s->outer[i]);
      if (memcmp(before, e->c, sizeof before) == 0) break;
    }
    need_centre(e);
    int64_t k = key_of(e, e->c);
    finals[q] = e->cval;
    fkeys[q] = k;
    if (e->cval > bv || (e->cval == bv && k < bk)) {
      bv = e->cval;
      bk = k;
      memcpy(bi, e->c, sizeof bi);
    }
  }
  /* cross-start decision margin among distinct final entries */
  for (int q = 0; q < nst; ++q)
    if (fkeys[q] != bk) log_pair(e, bv, finals[q]);
  free(finals);
  free(fkeys);
  memcpy(best_idx, bi, sizeof bi);
  /* both values of the entry returned (it is in the memo) */
  const int64_t sl = memo_slot(&e->memo, key_of(e, bi));
  best_vals[0] = e->memo.keys[sl] == key_of(e, bi) ? e->memo.vals[2 * sl] : bv;
  best_vals[1] = e->memo.keys[sl] == key_of(e, bi) ? e->memo.vals[2 * sl + 1] : bv;
}

int orc_zoom_generic2(const orc_schedule* sch, const int32_t* dims,
                      const int32_t* init, orc_objective2 obj, void* ctx,
                      int32_t* best_idx, double* best_vals, int32_t* n_eval,
                      double* min_margin, int32_t* path, int32_t path_cap,
                      int32_t* path_len) {
  if (!sched_ok(sch) || !dims || !obj) return 1;
  engine e;
  memset(&e, 0, sizeof e);
  e.sch = sch;
  for (int a = 0; a < 4; ++a) {
    if (dims[a] < 1) return 1;
    e.dims[a] = dims[a];
  }
  e.obj = obj;
  e.ctx = ctx;
  e.min_margin = INFINITY;
  e.path = path;
  e.path_cap = path ? path_cap : 0;
  memo_init(&e.memo);
  engine_run(&e, init, best_idx, best_vals);
  if (path_len) *path_len = e.path_len;
  if (n_eval) *n_eval = e.n_eval;
  if (min_margin) *min_margin = e.min_margin;
  memo_free(&e.memo);
  return 0;
}

/* a one-valued objective serving both objective kinds */
typedef struct {
  orc_objective f;
  void* ctx;
} one_valued;
static void one_valued_eval(void* p, const int32_t* i, double* out) {
  one_valued* o = (one_valued*)p;
  out[0] = out[1] = o->f(o->ctx, i);
}

int orc_zoom_generic(const orc_schedule* sch, const int32_t* dims,
                     const int32_t* init, orc_objective obj, void* ctx,
                     int32_t* best_idx, double* best_val, int32_t* n_eval,
                     double* min_margin, int32_t* path, int32_t path_cap,
                     int32_t* path_len) {
  if (!obj) return 1;
  one_valued o = {obj, ctx};
  double bv[2];
  int rc = orc_zoom_generic2(sch, dims, init, one_valued_eval, &o, best_idx, bv, n_eval,
                             min_margin, path, path_cap, path_len);
  if (rc == 0 && best_val) *best_val = bv[0];
  return rc;
}

typedef struct {
  const tables* t;
  const double *vr, *vi;
  double vnorm;
  double *re, *im;
  int32_t dims[4];
} phys_ctx;

/* The voxel against the simulated entry at idx: out[0] = CC (Eq. 1);
 * out[1] = the distance score, -min_phi ||v - exp(i phi) d||^2 / ||v||^2,
 * written out: the best phase makes the product <v, exp(i phi) d> real and
 * positive, exp(i phi) = <v, d> / |<v, d>| with <v, d> = sum v conj(d); then
 * the squared residual is summed readout by readout. */
static void phys_objective(void* p, const int32_t* i, double* out) {
  phys_ctx* c = (phys_ctx*)p;
  int64_t k = (((int64_t)i[0] * c->dims[1] + i[1]) * c->dims[2] + i[2]) * c->dims[3] + i[3];
  entry_factors f;
  tables_view(c->t, k, &f);
  entry_samples(c->t, &f, c->re, c->im);
  const int32_t n = c->t->n_tr;
  double nd2 = norm2(n, c->re, c->im);
  double nd = sqrt(nd2);
  double sr, si;
  cdot(n, c->vr, c->vi, c->re, c->im, &sr, &si);
  const double sabs = sqrt(sr * sr + si * si);
  out[0] = (nd == 0.0 || c->vnorm == 0.0) ? 0.0 : sabs / (c->vnorm * nd);
  /* exp(i phi); any phase when the product is 0 */
  const double pr = sabs > 0.0 ? sr / sabs : 1.0, pi = sabs > 0.0 ? si / sabs : 0.0;
  double e2 = 0.0;
  for (int32_t j = 0; j < n; ++j) {
    const double rr = c->vr[j] - (pr * c->re[j] - pi * c->im[j]);
    const double ri = c->vi[j] - (pr * c->im[j] + pi * c->re[j]);
    e2 += rr * rr + ri * ri;
  }
  out[1] = c->vnorm > 0.0 ? -e2 / (c->vnorm * c->vnorm) : -nd2;
}

int orc_zoom(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
             const orc_schedule* sch, const double* vr, const double* vi,
             int32_t n_vox, const int32_t* init, int64_t* idx, double* cc,
             double* score, int32_t* n_sim, double* min_margin, int32_t n_threads) {
  if (!sched_ok(sch) || !grid || n_vox < 0 || (n_vox > 0 && (!vr || !vi))) return 1;
  tables t;
  int rc = tables_build(seq, grid, n_tr, &t);
  if (rc) return rc;
  int32_t dims[4] = {t.n1, t.n2, t.n3, t.n4};
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
  {
    phys_ctx c;
    c.t = &t;
    memcpy(c.dims, dims, sizeof dims);
    c.re = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
    c.im = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int32_t v = 0; v < n_vox; ++v) {
      c.vr = vr + (size_t)v * n_tr;
      c.vi = vi + (size_t)v * n_tr;
      c.vnorm = sqrt(norm2(n_tr, c.vr, c.vi));
      int32_t bi[4];
      double bv[2];
      int32_t ne;
      double mm;
      orc_zoom_generic2(sch, dims, init ? init + 4 * (size_t)v : NULL, phys_objective,
                        &c, bi, bv, &ne, &mm, NULL, 0, NULL);
      if (idx) idx[v] = (((int64_t)bi[0] * dims[1] + bi[1]) * dims[2] + bi[2]) * dims[3] + bi[3];
      if (cc) cc[v] = bv[0];
      if (score) score[v] = bv[1];
      if (n_sim) n_sim[v] = ne;
      if (min_margin) min_margin[v] = mm;
    }
    free(c.re);
    free(c.im);
  }
  tables_free(&t);
  return 0;
}

/* Both objectives of the ZOOM engine (CC and the distance score, as
 * phys_objective computes them) at listed entries: cc/score[v*m + i] for
 * entry idx[v*m + i]; a negative index gives CC 0 and score -inf. */
int orc_objectives_at(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
                      const double* vr, const double* vi, int32_t n_vox, int32_t m,
                      const int64_t* idx, double* cc, double* score, int32_t n_threads) {
  if (!grid || n_vox < 0 || m < 0 ||
      (n_vox > 0 && m > 0 && (!vr || !vi || !idx || !cc || !score)))
    return 1;
  tables t;
  int rc = tables_build(seq, grid, n_tr, &t);
  if (rc) return rc;
  const int64_t E = grid_size(grid);
  for (int64_t q = 0; q < (int64_t)n_vox * m; ++q)
    if (idx[q] >= E) {
      tables_free(&t);
      return 1;
    }
  const int32_t dims[4] = {t.n1, t.n2, t.n3, t.n4};
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
  {
    phys_ctx c;
    c.t = &t;
    memcpy(c.dims, dims, sizeof dims);
    c.re = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
    c.im = (double*)malloc(sizeof(double) * (size_t)(n_tr + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
    for (int64_t q = 0; q < (int64_t)n_vox * m; ++q) {
      const int64_t v = q / m;
      if (idx[q] < 0) {
        cc[q] = 0.0;
        score[q] = -INFINITY;
        continue;
      }
      c.vr = vr + (size_t)v * n_tr;
      c.vi = vi + (size_t)v * n_tr;
      c.vnorm = sqrt(norm2(n_tr, c.vr, c.vi));
      int64_t k = idx[q];
      int32_t i[4];
      for (int a = 3; a >= 0; --a) {
        i[a] = (int32_t)(k % dims[a]);
        k /= dims[a];
      }
      double o[2];
      phys_objective(&c, i, o);
      cc[q] = o[0];
      score[q] = o[1];
    }
    free(c.re);
    free(c.im);
  }
  tables_free(&t);
  return 0;
}
