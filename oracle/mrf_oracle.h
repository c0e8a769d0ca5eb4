/*
 * FP64 CPU oracle for MRF dictionary generating and searching.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code with
 * the GPU library (no headers, helpers, tables or constants) and must never
 * be used by the product path.
 *
 * Conventions (all double precision, times in ms, frequencies in Hz):
 *   - Event model (Methods, IR-bSSFP; Appendix Eq. A2): equilibrium M = (0,0,1),
 *     ideal inversion Mz -> -Mz at t = 0, free evolution for TI, then for each
 *     readout j: hard RF pulse, free evolution for TE_j, sample
 *     s_j = Mx + i*My, free evolution for TR_j - TE_j.
 *   - RF pulse (Appendix, small-beta limit): Rz(phi) Rx(-B1*alpha) Rz(-phi),
 *     counter-clockwise rotation matrices as printed in the Appendix.
 *   - Free evolution over t (Appendix Eq. A1 solved exactly for constant field):
 *     transverse (Mx, My) <- exp(-t/T2) Rz(2*pi*df*t/1000) (Mx, My);
 *     Mz <- exp(-t/T1) Mz + (1 - exp(-t/T1)) with M0 = 1.
 *   - CC (Theory, Eq. 1): |sum_j v_j conj(d_j)| / (||v|| ||d||); 0 if a norm is 0.
 *   - Grid entry index k = ((i1*n2 + i2)*n3 + i3)*max(n4,1) + i4 over
 *     (T1, T2, df, B1); n4 = 0 means B1 = 1.
 */
#ifndef MRF_ORACLE_H
#define MRF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n;                 /* readouts available */
  const double* fa_deg;      /* [n] flip angles, degrees */
  const double* phase_deg;   /* [n] RF phases, degrees */
  const double* tr_ms;       /* [n] repetition times */
  const double* te_ms;       /* [n] echo times, 0 < te < tr */
  int32_t inversion;         /* 1: ideal inversion at t = 0 */
  double ti_ms;              /* inversion to first pulse */
  int32_t smooth;            /* dictionary entries smoothed over 3 or 5 readouts (0: none),
                                in the frame demodulated by the RF phases */
} orc_seq;

typedef struct {
  int32_t n1, n2, n3, n4;    /* axis lengths; n4 = 0 means B1 = 1 */
  const double *t1, *t2, *df, *b1;
} orc_grid;

/* ZOOM stage kinds (index space). */
enum {
  ORC_SCAN_STRIDE = 0, /* scan axis0 at lo, lo+s, lo+2s, ... (does not use the centre) */
  ORC_SCAN_WINDOW = 1, /* scan axis0 at c + m*s, 0 < |m*s| <= window (centre kept on ties) */
  ORC_SCAN_HOPS   = 2, /* scan axis0 at c + round_half_away(k*hop), k != 0 */
  ORC_ZOOM1       = 3, /* 1-D hill climb on axis0 with step s0 */
  ORC_ZOOM2       = 4  /* 2-D hill climb on (axis0, axis1) with steps (s0, s1) */
};

/* Objective of a stage: CC of Eq. 1, or the distance of the non-normalised
 * fingerprint from the raw entry (M0 = 1) with only a global phase fitted,
 * score = -min_phi ||v - exp(i phi) d||^2 / ||v||^2 (0 at a perfect match;
 * -||d||^2 for a zero fingerprint). The fingerprint must be in units of M0
 * (its proton density magnitude divided out). Each entry is simulated once;
 * both values are kept. */
enum { ORC_OBJ_CC = 0, ORC_OBJ_DIST = 1 };
typedef struct {
  int32_t kind, axis0, axis1, step0, step1, window;
  double hop;
  int32_t objective; /* ORC_OBJ_CC or ORC_OBJ_DIST */
} orc_stage;

#define ORC_MAX_STAGES 64
#define ORC_MAX_STARTS 16

typedef struct {
  int32_t n_stages;
  orc_stage stages[ORC_MAX_STAGES];
  int32_t n_outer;              /* stages repeated after the main list ... */
  orc_stage outer[ORC_MAX_STAGES];
  int32_t outer_max;            /* ... at most this many times, until the centre stops changing */
  int32_t n_starts;
  int32_t starts[ORC_MAX_STARTS][4];
  int32_t pruned;               /* 1: evaluation-saving move rules of the Theory section */
  int32_t prior_half[4];        /* neighbour-prior half widths in index steps (<0: whole axis) */
} orc_schedule;

/* Objective used by the generic engine: value at grid index i[4]. */
typedef double (*orc_objective)(void* ctx, const int32_t* idx);

/* ---- simulator ---- */
int orc_simulate(const orc_seq* seq, int32_t n_tr, double t1, double t2,
                 double df, double b1, double* re, double* im);
/* states[j*9 + 0..2] after the pulse, [3..5] at TE, [6..8] at the end of TR */
int orc_trajectory(const orc_seq* seq, int32_t n_tr, double t1, double t2,
                   double df, double b1, double* states);
/* entries [k0, k0+count) of the grid, entry-major re/im [count][n_tr], raw
 * (not normalised), norm [count] (may be NULL) */
int orc_simulate_grid(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
                      int64_t k0, int64_t count, double* re, double* im,
                      double* norm, int32_t n_threads);
double orc_cc(int32_t n, const double* vr, const double* vi, const double* dr,
              const double* di);

/* ---- brute-force search (streaming; the dictionary is never stored) ---- */
int orc_bruteforce(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
                   const double* vr, const double* vi, int32_t n_vox, /* [n_vox][n_tr] */
                   int32_t top_k, int64_t* idx, double* cc, double* margin,
                   double* pd_re, double* pd_im, int64_t* topk_idx,
                   double* topk_cc, int32_t n_threads);

/* ---- temporal smoothing (Experiment 4): binomial 3 / 5 points, in place,
 * in the frame demodulated by the RF phases phase_deg[0..n) (NULL: zero
 * phases); the result is modulated back ---- */
int orc_smooth(int32_t n, int32_t taps, const double* phase_deg, double* re, double* im);

/* ---- CC map (Experiment 1): out[v][i] = CC(v, entry k0 + i), Eq. 1 ---- */
int orc_cc_map(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
               const double* vr, const double* vi, int32_t n_vox, int64_t k0,
               int64_t count, double* out, int32_t n_threads);

/* ---- Eq. 1 at listed entries: out[v*m + i] = CC(v, entry idx[v*m + i]),
 * 0 for a negative index ---- */
int orc_cc_at(const orc_seq* seq, const orc_grid* grid, int32_t n_tr, const double* vr,
              const double* vi, int32_t n_vox, int32_t m, const int64_t* idx, double* out,
              int32_t n_threads);

/* ---- both ZOOM objectives at listed entries: cc/score[v*m + i] for entry
 * idx[v*m + i] (CC of Eq. 1 and the distance score of ORC_OBJ_DIST; a
 * negative index gives 0 and -inf) ---- */
int orc_objectives_at(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
                      const double* vr, const double* vi, int32_t n_vox, int32_t m,
                      const int64_t* idx, double* cc, double* score, int32_t n_threads);
/* ---- ZOOM ---- */
int orc_schedule_paper(const orc_grid* grid, const orc_seq* seq,
                       orc_schedule* out);
/* the paper's stages from a k1 x k2 lattice of starts over the T1/T2 index
 * ranges (ends included), then outer rounds [df window, fine df scan, 2-D
 * zooms at 100, 50, 20, 10 ms and unit steps (+ unit B1)] */
int orc_schedule_multistart(const orc_grid* grid, const orc_seq* seq, int32_t k1, int32_t k2,
                            int32_t outer_max, orc_schedule* out);
/* every stage at unit index steps (the finest resolution) gets `objective` */
int orc_schedule_finest_objective(orc_schedule* sched, int32_t objective);
/* neighbour-prior half widths (Experiment 3) in index steps from physical
 * half widths half[4] (T1 ms, T2 ms, df Hz, B1; NULL: 3000, 800, 150, 0.3) */
int orc_prior_half(const orc_grid* grid, const double* half, int32_t* out);
/* generic engine on a caller objective; the memo is per call. path (optional):
 * 5 ints per hill-climb move or scan update = new centre and the number of
 * evaluations made when it was reached. Every stage uses obj whatever its
 * objective field. best_val: the final value of the best start. */
int orc_zoom_generic(const orc_schedule* sch, const int32_t* dims,
                     const int32_t* init, orc_objective obj, void* ctx,
                     int32_t* best_idx, double* best_val, int32_t* n_eval,
                     double* min_margin, int32_t* path, int32_t path_cap,
                     int32_t* path_len);
/* the same engine on a two-valued objective: obj2 fills out[0] (used by
 * ORC_OBJ_CC stages) and out[1] (ORC_OBJ_DIST stages) for one entry, which
 * is evaluated once. best_vals[2]: both values of the entry returned. */
typedef void (*orc_objective2)(void* ctx, const int32_t* idx, double* out);
int orc_zoom_generic2(const orc_schedule* sch, const int32_t* dims,
                      const int32_t* init, orc_objective2 obj2, void* ctx,
                      int32_t* best_idx, double* best_vals, int32_t* n_eval,
                      double* min_margin, int32_t* path, int32_t path_cap,
                      int32_t* path_len);
/* physics objective: CC (Eq. 1) and the distance score of each voxel
 * against simulated entries. init: [n_vox][4] prior centres or NULL (then
 * the schedule's starts are used). cc: the CC of the entry returned; score
 * (may be NULL): its distance score. */
int orc_zoom(const orc_seq* seq, const orc_grid* grid, int32_t n_tr,
             const orc_schedule* sch, const double* vr, const double* vi,
             int32_t n_vox, const int32_t* init, int64_t* idx, double* cc,
             double* score, int32_t* n_sim, double* min_margin, int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
