/*
 * libmrf — MRF dictionary generating and searching on one MI355X (gfx950).
 *
 * C ABI. Every function returns an int status (MRF_OK = 0); no exception
 * crosses the boundary. mrf_last_error() returns a thread-local message for
 * the last failing call on the calling thread.
 *
 * Ownership: the caller owns every device array passed in (voxels,
 * dictionaries, outputs, workspaces) and libmrf never frees them. libmrf owns
 * the opaque handles (context, sequence with its resident step tables,
 * server). A ZOOM schedule is a plain struct (mrf_zoom_schedule) that the
 * caller allocates and the schedule builders fill in place: it holds no
 * pointers or resources, so there is no destroy call for it (a deviation
 * from an opaque-handle design with mrf_zoom_schedule_destroy). Device
 * pointers are plain hipMalloc'ed (or torch) device
 * memory on the context's device; host pointers are ordinary host memory.
 *
 * Streams: `void* stream` is a hipStream_t (NULL = the default stream). All
 * device work of a call is enqueued on it and is asynchronous unless stated;
 * outputs are valid after the stream has been synchronised. Calls on one
 * context are serialised by the caller.
 *
 * Method (arxiv 1506.05393):
 *   - signal model: inversion-recovery bSSFP train (Methods) simulated with
 *     the Bloch model of the Appendix (Eq. A1, A2; hard-pulse RF);
 *   - distance: |complex correlation| of Theory Eq. 1 (CC);
 *   - brute-force search: the entry of maximal CC over the whole grid
 *     (Introduction; Experiment 2);
 *   - MRF-ZOOM: parameter-separable coarse-to-fine search (Theory: MRF ZOOM;
 *     Methods: Experiment 2 steps 1-5; Experiment 3 neighbour prior).
 *
 * Units: times in ms, frequencies in Hz, angles in degrees.
 * Grid entry index: k = ((i_t1*n_t2 + i_t2)*n_df + i_df)*max(n_b1,1) + i_b1.
 */
#ifndef LIBMRF_H
#define LIBMRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MRF_OK = 0,
  MRF_ERR_INVALID = 1,     /* bad argument (null pointer, size, range, dtype) */
  MRF_ERR_OOM = 2,         /* device or host allocation failed */
  MRF_ERR_DEVICE = 3,      /* a HIP call failed */
  MRF_ERR_NOT_READY = 4,   /* result not available yet */
  MRF_ERR_REJECTED = 5,    /* request can never be admitted */
  MRF_ERR_UNSUPPORTED = 6, /* valid but not supported in this build */
  MRF_ERR_CANCELLED = 7
};

typedef enum { MRF_F32 = 0, MRF_BF16 = 1, MRF_F32_ROWS = 2 } mrf_dtype;

const char* mrf_status_str(int status);
const char* mrf_last_error(void);
/* library version string */
const char* mrf_version(void);

typedef struct mrf_context mrf_context;
typedef struct mrf_sequence mrf_sequence;

/* Bind a context to HIP device `device` (makes it current on this thread). */
int mrf_context_create(int device, mrf_context** out);
int mrf_context_destroy(mrf_context* ctx);

/* Acquisition sequence (Methods: IR-bSSFP; Theory: the same flip angles,
 * phases, TR and TE are used to acquire and to simulate). Host arrays of n
 * values, copied at creation. Requires 0 < te_ms[j] < tr_ms[j]. With
 * inversion = 1 the longitudinal magnetisation is ideally inverted at t = 0
 * and evolves freely for ti_ms >= 0 before the first pulse. */
typedef struct {
  int32_t n;
  const double* fa_deg;
  const double* phase_deg;
  const double* tr_ms;
  const double* te_ms;
  int32_t inversion;
  double ti_ms;
  /* Temporal smoothing of dictionary entries (Methods, Experiment 4): 0 or 1
   * none, 3 or 5 readouts (binomial weights (1, 2, 1) / 4 and
   * (1, 4, 6, 4, 1) / 16, renormalised over the readouts that exist at the
   * first and last readouts), applied to the samples demodulated by their RF
   * phase (times exp(-i phase_j)) and modulated back. Every dictionary entry the library simulates
   * for this sequence (dictionaries, CC maps, ZOOM candidates, BF16
   * re-scoring) is smoothed; fingerprints from mrf_simulate_signals are not:
   * smooth them with mrf_smooth_signals. Other values: MRF_ERR_INVALID. */
  int32_t smooth;
} mrf_sequence_desc;

int mrf_sequence_create(mrf_context* ctx, const mrf_sequence_desc* desc, mrf_sequence** out);
int mrf_sequence_destroy(mrf_sequence* seq);

/* Parameter grid: one strictly increasing host value list per axis
 * (T1 ms > 0, T2 ms > 0, df Hz, B1 scale of every flip angle). b1.n == 0
 * means B1 = 1. T1 or T2 may be +inf (no relaxation). At most 2^39 entries
 * (more -> MRF_ERR_INVALID). */
typedef struct {
  int32_t n;
  const double* v;
} mrf_axis;
typedef struct {
  mrf_axis t1_ms, t2_ms, df_hz, b1;
} mrf_grid;

/* Number of grid entries, or -1 if the grid is invalid. */
int64_t mrf_grid_size(const mrf_grid* grid);

/* ------------------------------------------------------------------------
 * Dictionary generation (Appendix Eq. A2 per entry; brute-force DGS).
 *
 * Simulates entries [entry_begin, entry_begin + entry_count) of `grid` over
 * the first n_tr readouts (n_tr <= sequence n). FP32 state; the relaxation
 * and precession factors are computed once per grid value in FP64 and
 * rounded to FP32; the norm accumulates FP32 partial sums of four readouts
 * in FP64.
 *
 * Layouts (entry e = k - entry_begin, 0 <= e < entry_count <= ld):
 *   MRF_F32  : planar, time-major. re[j*ld + e] = Re d_j, im[j*ld + e] = Im d_j,
 *              j < n_tr (re and im are separate [n_tr][ld] float arrays).
 *   MRF_BF16 : packed blocks of 4 readouts, re holds the whole dictionary:
 *              element ((b*ld + e)*4 + q)*2 + {0: Re, 1: Im} of readout
 *              j = 4b + q, bf16 round-to-nearest-even; im must be NULL.
 *              n_tr must be a multiple of 4.
 *   MRF_F32_ROWS: entry-major complex64 rows (the layout the resident-
 *              dictionary ZOOM gathers from): re[(e*ld + j)*2 + {0: Re, 1: Im}],
 *              j < n_tr; ld >= n_tr and even, re 16-byte aligned, im NULL;
 *              rows start on 128-byte lines when ld is a multiple of 16 and
 *              re is 128-byte aligned (each entry's readouts are written 16
 *              at a time, one line per burst). (Brute-force matching does
 *              not take this layout.)
 * Values are the raw signal (M0 = 1) unless unit_norm = 1, in which case each
 * entry is divided by its norm (two passes). norm (device, FP64
 * [entry_count], or NULL) receives, for MRF_F32, the raw norm ||d||; for
 * MRF_BF16, the norm of the stored (scaled, rounded) BF16 values, so that a
 * CC computed from the stored entries is normalised consistently (rounding
 * the entries but not their norm biases each entry's CC by up to ~2^-9).
 * ---------------------------------------------------------------------- */
int mrf_simulate_dictionary(mrf_context* ctx, const mrf_sequence* seq, const mrf_grid* grid,
                            int32_t n_tr, int64_t entry_begin, int64_t entry_count,
                            mrf_dtype dtype, void* re, void* im, int64_t ld,
                            double* norm, int32_t unit_norm, void* stream);

/* The FP32 planar (MRF_F32) and BF16 (MRF_BF16) dictionaries of one entry
 * range from one recursion pass (Appendix Eq. A2), raw values (M0 = 1):
 * re/im as MRF_F32 and packed as MRF_BF16 above, all with the same ld (in
 * entries); norm (FP64 [entry_count] or NULL) receives ||d|| of the FP32
 * values and norm_bf16 (or NULL) the norm of the stored BF16 values. Every
 * value and norm equals what mrf_simulate_dictionary writes for each dtype
 * with unit_norm = 0. Caller-owned device buffers; enqueued on `stream`.
 * Errors: as mrf_simulate_dictionary for both layouts (n_tr % 4 == 0, packed
 * 16-byte aligned, ld >= entry_count, NULL re/im/packed with entries). */
int mrf_simulate_dictionary_pair(mrf_context* ctx, const mrf_sequence* seq,
                                 const mrf_grid* grid, int32_t n_tr, int64_t entry_begin,
                                 int64_t entry_count, float* re, float* im, void* packed,
                                 int64_t ld, double* norm, double* norm_bf16, void* stream);

/* CC map (Methods and Results, Experiment 1): the CC of Eq. 1 between each
 * fingerprint and every entry of [entry_begin, entry_begin + entry_count) of
 * `grid`, written out in full:
 *   cc[v * ld_cc + i] = |<v, d_e>| / (||v|| ||d_e||),  e = entry_begin + i,
 * 0 where either norm is 0. The entries are simulated exactly as by
 * mrf_simulate_dictionary (FP32 recursion, the same step tables) and the CC
 * is accumulated on the fly (FP32 partial sums of four readouts added into
 * FP64), so no dictionary is stored and any grid size fits.
 *   vox: device complex64 [n_vox][ld_vox] (ld_vox >= n_tr; the first n_tr
 *        readouts are used), caller-owned, 8-byte aligned.
 *   cc:  device float32 [n_vox][ld_cc] (ld_cc >= entry_count), caller-owned.
 * One launch per fingerprint on `stream`; returns without waiting (profile
 * name "k_cc_map").
 * Errors: NULL pointers with work to do, n_tr outside [1, sequence length],
 * ld_vox < n_tr, ld_cc < entry_count, a range outside the grid, an invalid
 * grid -> MRF_ERR_INVALID (nothing launched). */
int mrf_cc_map(mrf_context* ctx, const mrf_sequence* seq, const mrf_grid* grid, int32_t n_tr,
               const void* vox, int32_t n_vox, int64_t ld_vox, int64_t entry_begin,
               int64_t entry_count, float* cc, int64_t ld_cc, void* stream);

/* Temporal smoothing of complex64 signals along their readouts (Methods,
 * Experiment 4: the fingerprints are smoothed like the dictionary). Row i of
 * n_sig: in[i*ld_in + j] -> out[i*ld_out + j], j < n_tr, device memory,
 * caller-owned. taps 3 or 5: the weights of mrf_sequence_desc.smooth, with
 * the same end renormalisation, in the frame demodulated by seq's RF phases
 * and modulated back (seq NULL: zero phases); taps 0 or 1: a copy. in == out
 * with ld_in == ld_out smooths in place; otherwise the two must not overlap.
 * Returns without waiting (profile name "k_smooth_signals").
 * Errors: other taps, n_tr above seq's length, ld < n_tr, NULL or misaligned
 * (8 B) pointers with work to do, partially overlapping rows ->
 * MRF_ERR_INVALID (nothing launched). */
int mrf_smooth_signals(mrf_context* ctx, const mrf_sequence* seq, const void* in, int64_t ld_in,
                       void* out, int64_t ld_out, int64_t n_sig, int32_t n_tr, int32_t taps,
                       void* stream);

/* Simulate fingerprints at arbitrary (not necessarily on-grid) parameter
 * values: params is a device FP64 array [count][4] = (T1 ms, T2 ms, df Hz,
 * B1). Output complex64 out[i*ld_out + j], j < n_tr (raw signal, M0 = 1). */
int mrf_simulate_signals(mrf_context* ctx, const mrf_sequence* seq, int32_t n_tr,
                         const double* params, int64_t count, void* out, int64_t ld_out,
                         void* stream);

/* ------------------------------------------------------------------------
 * Brute-force matching (Theory Eq. 1; Introduction: exhaustive search).
 *
 * For each voxel v (complex64 vox[v*ld_vox + j], j < n_tr) and every entry k
 * of the dictionary view, CC_vk = |sum_j v_j conj(d_kj)| / (||v|| ||d_k||).
 * The entry of maximal CC is returned (ties: lower k). Computed as a complex
 * GEMM on MFMA with the per-voxel running top-k fused into its epilogue; the
 * voxel x entry score matrix is never written.
 * ---------------------------------------------------------------------- */
typedef struct {
  mrf_dtype dtype;    /* layout as produced by mrf_simulate_dictionary */
  int32_t n_tr;       /* readouts used (<= readouts stored) */
  int64_t n_entries;  /* entries 0..n_entries-1 (global index = entry_base + e) */
  int64_t ld;
  const void* re;
  const void* im;     /* NULL for MRF_BF16 */
  const double* norm; /* raw norms [n_entries] (FP64), or NULL for unit-norm entries */
  int64_t entry_base; /* grid index of entry 0 */
} mrf_dict_view;

/* Per-voxel outputs (device arrays of n_vox; any but idx may be NULL).
 * idx: int64 grid index; cc: CC of that entry; margin: CC(best) - CC(runner-up)
 * (FP32 search) or of the rescored candidates (BF16 search); pd_re/pd_im:
 * proton density <v, d>/||d||^2 (Theory: PD from the signal scale);
 * n_sim: entries evaluated (ZOOM). */
typedef struct {
  int64_t* idx;
  float* cc;
  float* margin;
  float* pd_re;
  float* pd_im;
  int32_t* n_sim;
} mrf_result_view;

/* Workspace bytes needed by mrf_match_bruteforce for these sizes. */
int mrf_match_workspace(mrf_context* ctx, const mrf_dict_view* dict, int32_t n_vox,
                        int32_t top_k, size_t* bytes);

/* top_k: the kept candidate list per voxel (at least 2 internally for the
 * margin). FP32 dictionaries: top_k in [1, 64] (lists longer than 16 run a
 * GEMM instance with 64-entry lists in LDS, one workgroup per CU instead of
 * two). BF16 dictionaries: top_k in [2, 8] (the GEMM's four-stage LDS ring
 * leaves room for lists of 8) and seq/grid are required: the top_k BF16
 * candidates of each voxel are re-simulated in
 * FP32 (the values an FP32 dictionary stores) and re-scored with an FP32 dot
 * product under compensated summation (error ~1 FP32 ulp of the sum), and the
 * best of them is returned. topk_idx /
 * topk_cc (device [n_vox][top_k], optional) receive the candidate list
 * (FP32: exact scores; BF16: the BF16 GEMM's CC estimates). */
int mrf_match_bruteforce(mrf_context* ctx, const mrf_dict_view* dict, const void* vox,
                         int32_t n_vox, int64_t ld_vox, int32_t top_k,
                         const mrf_sequence* seq, const mrf_grid* grid, mrf_result_view out,
                         int64_t* topk_idx, float* topk_cc, void* workspace,
                         size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): FP32 brute
 * force exactly as mrf_match_bruteforce with an MRF_F32 dictionary (same
 * kernels, bitwise-equal outputs), with its workspace in a static device
 * array of mrf_static_scratch_bytes() bytes (64 MiB) that the library holds
 * on each GPU it runs on until the process ends. The call allocates nothing:
 * no hipMalloc/hipFree, no library allocation, no profiling events.
 * Arguments as mrf_match_bruteforce (vox, out, topk_idx/topk_cc device
 * memory, caller-owned). Every call on one GPU shares that GPU's array and
 * leaves its contents behind; nothing in it needs to start at zero (the
 * packing kernel writes every operand slot and the GEMM every candidate list
 * before they are read). Calls that overlap on one GPU (two streams, two
 * threads) race on the array: serialise them.
 * Errors: a BF16 or rows dictionary, or sizes whose workspace
 * (mrf_match_workspace) exceeds the array -> MRF_ERR_INVALID with the bytes
 * needed (a 64 x 64 slice at N = 1000 fits); otherwise as
 * mrf_match_bruteforce. */
size_t mrf_static_scratch_bytes(void);
int mrf_match_bruteforce_noalloc(mrf_context* ctx, const mrf_dict_view* dict, const void* vox,
                                 int32_t n_vox, int64_t ld_vox, int32_t top_k,
                                 mrf_result_view out, int64_t* topk_idx, float* topk_cc,
                                 void* stream);

/* ------------------------------------------------------------------------
 * MRF-ZOOM (Theory: MRF ZOOM; Methods: Experiment 2 zooming steps 1-5;
 * Experiment 3 neighbour prior).
 *
 * A per-voxel search in grid-index space that simulates candidate entries on
 * the fly (no stored dictionary) and maximises CC (Eq. 1). The schedule is a
 * list of stages applied to the current centre c (index tuple over T1, T2,
 * df, B1 = axes 0..3):
 *   SCAN_STRIDE(axis, s)     : evaluate lo, lo+s, lo+2s, ... <= hi on the axis;
 *                              the centre moves to the maximum (ties: lowest index)
 *   SCAN_WINDOW(axis, s, w)  : evaluate c + m s, 0 < |m s| <= w; move to the
 *                              maximum if it beats the centre (ties keep the centre,
 *                              then the lowest index)
 *   SCAN_HOPS(axis, hop)     : evaluate c + round_half_away(k hop), k != 0, in range
 *                              (the +-k*omega hops of the df search); as WINDOW
 *   ZOOM1(axis, s)           : hill climb: compare C with C-s, C+s, move to the
 *                              strictly larger (ties: the lower side), repeat
 *   ZOOM2(a0, a1, s0, s1)    : hill climb over the 8 neighbours in the order
 *                              L, R, D, U, LD, LU, RD, RU (first maximum wins)
 * With pruned = 1 the evaluation-saving move rules of the Theory section are
 * used (R first in 1-D; L, D first in 2-D). Each start in starts[] runs the
 * stage list, then the outer list is repeated (at most outer_max times) until
 * the centre no longer changes; the best final CC wins (ties: lower index).
 * Out-of-range points are skipped. Each distinct entry is simulated once per
 * voxel (n_sim counts them).
 * ---------------------------------------------------------------------- */
enum {
  MRF_SCAN_STRIDE = 0,
  MRF_SCAN_WINDOW = 1,
  MRF_SCAN_HOPS = 2,
  MRF_ZOOM1 = 3,
  MRF_ZOOM2 = 4
};
#define MRF_ZOOM_MAX_STAGES 32
#define MRF_ZOOM_MAX_STARTS 16

/* Objective of a stage (Discussion: at the finest resolution the paper
 * removed its errors at T1 > 2400 ms by matching the non-normalised
 * fingerprints and entries with the Euclidean distance instead of CC):
 *   MRF_OBJ_CC   the CC of Eq. 1 (every stage of the paper's schedule);
 *   MRF_OBJ_DIST the distance of the fingerprint, as given, from the raw
 *                entry (M0 = 1) with only a global phase fitted, scored as
 *                -min_phi ||v - exp(i phi) d||^2 / ||v||^2 (0 = perfect
 *                match). The fingerprint must be in units of M0, i.e. its
 *                proton-density magnitude divided out (the synthetic
 *                fingerprints of the paper's experiments have M0 = 1).
 * A schedule with MRF_OBJ_DIST stages runs a kernel that simulates every
 * candidate with a compensated FP32 dot product (as accurate as one in
 * twice the precision) and keeps both values per entry; the distance itself
 * is formed in FP64 from the two norms and that product. Not available
 * with smoothing sequences or the resident-dictionary search. */
enum { MRF_OBJ_CC = 0, MRF_OBJ_DIST = 1 };

typedef struct {
  int32_t kind, axis0, axis1, step0, step1, window;
  double hop;
  int32_t objective; /* MRF_OBJ_CC or MRF_OBJ_DIST */
} mrf_zoom_stage;

typedef struct {
  int32_t n_stages;
  mrf_zoom_stage stages[MRF_ZOOM_MAX_STAGES];
  int32_t n_outer;
  mrf_zoom_stage outer[MRF_ZOOM_MAX_STAGES];
  int32_t outer_max;
  int32_t n_starts;
  int32_t starts[MRF_ZOOM_MAX_STARTS][4];
  int32_t pruned;
  /* neighbour prior (Experiment 3): with init_idx given, each axis with
   * prior_half[a] >= 0 is restricted to init +- prior_half[a] index steps */
  int32_t prior_half[4];
} mrf_zoom_schedule;

/* The schedule of Methods, Experiment 2 (zooming steps 1-5) for `grid`, in
 * index steps: physical steps r become max(1, round_half_away(r / step)) with
 * step = (max - min)/(n - 1) per axis; omega = 1000 / min TR Hz; start at the
 * grid values nearest to T1 = 1000 ms, T2 = 500 ms. With a B1 axis, B1 zooms
 * at 0.1 ... 0.005 follow the interleaved 1-D zooms, and [2-D unit zoom, B1
 * unit zoom, fine df scan] is repeated up to 3 times. */
int mrf_zoom_schedule_paper(const mrf_grid* grid, const mrf_sequence* seq,
                            mrf_zoom_schedule* out);

/* Neighbour-prior ranges (Methods, Experiment 3: a neighbour's result
 * T1p/T2p/dfp opens the ranges T1p +- 3000 ms, T2p +- 800 ms, dfp +- 150 Hz,
 * intersected with the search ranges). Sets sched->prior_half (the only
 * field written) from physical half widths half[4] = (T1 ms, T2 ms, df Hz,
 * B1 scale), host memory, or NULL for the paper's ranges with +- 0.3 for a
 * B1 axis. Each becomes index steps like the schedule's other physical
 * steps, max(1, round_half_away(half / ((max - min)/(n - 1)))); an axis of
 * fewer than two values or a negative half width gets -1 (the whole axis).
 * The ranges apply to searches started from prior centres (init_idx,
 * mrf_zoom_search_from, the second lattice pass). Host only.
 * Errors: invalid grid, NULL sched, a NaN half width -> MRF_ERR_INVALID. */
int mrf_zoom_schedule_prior(const mrf_grid* grid, const double* half, mrf_zoom_schedule* sched);

/* Multi-start form of the paper's schedule (Methods, Experiment 2 steps
 * 1-5 from several initial values; Discussion: "a second searching process
 * can be used after finding an approximate value for T1 and T2"): the
 * stages of mrf_zoom_schedule_paper run from each of n_t1 x n_t2 starts, an
 * index lattice over the T1 and T2 axes from their first to their last
 * value (round_half_away(q (n - 1) / (k - 1)); one start per axis sits at
 * index (n - 1) / 2), df index 0; then an outer round [df window scan,
 * fine df scan, 2-D zooms at 100, 50, 20 and 10 ms, unit 2-D zoom (, unit
 * B1 zoom)] is repeated up to outer_max times until the centre stays; the
 * best final CC over the starts wins. 4 x 4 starts with outer_max 8 is the
 * cheapest lattice found to agree with brute force on every voxel whose
 * brute-force margin exceeds 1e-5 on the small workload (~970 entries per
 * voxel against 50,400). Host only.
 * Errors: as mrf_zoom_schedule_paper; n_t1 * n_t2 outside
 * [1, MRF_ZOOM_MAX_STARTS] or outer_max outside [0, 64] -> MRF_ERR_INVALID. */
int mrf_zoom_schedule_multistart(const mrf_grid* grid, const mrf_sequence* seq, int32_t n_t1,
                                 int32_t n_t2, int32_t outer_max, mrf_zoom_schedule* out);

/* Sets the objective of every stage of the finest resolution (unit index
 * steps: ZOOM1/ZOOM2 with steps 1, SCAN_WINDOW/SCAN_STRIDE with step 1;
 * both stage lists) to `objective` (MRF_OBJ_CC or MRF_OBJ_DIST). With
 * MRF_OBJ_DIST on the paper's schedule: the fine df scan and the final 2-D
 * zoom (and, with a B1 axis, the outer unit-step rounds). Host only.
 * Errors: NULL sched, another objective -> MRF_ERR_INVALID. */
int mrf_zoom_schedule_finest_objective(mrf_zoom_schedule* sched, int32_t objective);

/* Local refinement (not a schedule of the paper: its finest-resolution
 * steps, Methods Experiment 2 step 5, used alone): unit-step 2-D zoom on
 * (T1, T2), unit-step 1-D zoom on df (and on B1 with a B1 axis), repeated
 * while the centre moves, up to outer_max rounds. Run with init_idx = a
 * brute-force result it climbs to the local CC maximum next to it; without
 * init it starts at the grid centre. */
int mrf_zoom_schedule_local(const mrf_grid* grid, int32_t outer_max, mrf_zoom_schedule* out);

int mrf_zoom_workspace(mrf_context* ctx, const mrf_grid* grid, int32_t n_vox, int32_t n_tr,
                       size_t* bytes);

/* vox: complex64 [n_vox][ld_vox] (first n_tr readouts used). init_idx:
 * device int32 [n_vox][4] prior centres, or NULL (then the schedule's
 * starts are used). Outputs (out): idx, cc (the CC of the entry returned,
 * whatever objective its last stage used), margin (= the smallest decision
 * margin along the voxel's path: best minus runner-up among the values
 * compared by one decision, in the units of that stage's objective; across
 * starts, of the last stage's objective), pd_re/pd_im of the found entry,
 * n_sim. Errors: MRF_ERR_UNSUPPORTED for MRF_OBJ_DIST stages with a
 * smoothing sequence. */
int mrf_zoom_search(mrf_context* ctx, const mrf_sequence* seq, const mrf_grid* grid,
                    const mrf_zoom_schedule* sched, const void* vox, int32_t n_vox,
                    int64_t ld_vox, int32_t n_tr, const int32_t* init_idx,
                    mrf_result_view out, void* workspace, size_t ws_bytes, void* stream);

/* As mrf_zoom_search for a batch whose voxels use different readout counts
 * of the same sequence (prefixes, e.g. slices acquired with N = 500 and
 * N = 1000 searched in one launch): voxel v uses its first vox_n_tr[v]
 * readouts (device int32 [n_vox], each in [1, n_tr_max]); the step tables
 * of the first n_tr_max readouts serve every prefix, so each voxel's result
 * equals a search of that voxel alone with n_tr = vox_n_tr[v], bit for bit.
 * Workspace as mrf_zoom_workspace with n_tr_max. Counts outside
 * [1, n_tr_max] are clamped to it on the device. Errors: as
 * mrf_zoom_search, plus NULL vox_n_tr with voxels and a smoothing sequence
 * -> MRF_ERR_INVALID. */
int mrf_zoom_search_ragged(mrf_context* ctx, const mrf_sequence* seq, const mrf_grid* grid,
                           const mrf_zoom_schedule* sched, const void* vox, int32_t n_vox,
                           int64_t ld_vox, int32_t n_tr_max, const int32_t* vox_n_tr,
                           mrf_result_view out, void* workspace, size_t ws_bytes, void* stream);

/* MRF-ZOOM over a resident dictionary (Results: the MZfulldict variant, the
 * fastest of the paper's timings): the same search as mrf_zoom_search, but
 * each visited entry is read from `dict` instead of simulated. dict: an
 * MRF_F32_ROWS dictionary of the whole grid (entry_base 0, n_entries = grid
 * size, n_tr >= the n_tr searched, ld even), as mrf_simulate_dictionary
 * writes it; its norm may be NULL (norms are computed from the rows). A
 * group of lanes reads each entry's row together (coalesced 16-byte loads),
 * so the search is bound by HBM reads of ~8 B per readout per visited entry
 * instead of the simulation's ALU work. Outputs and errors as
 * mrf_zoom_search, plus MRF_ERR_INVALID for a dictionary of another layout,
 * another extent or a misaligned base. */
int mrf_zoom_search_dict(mrf_context* ctx, const mrf_dict_view* dict, const mrf_grid* grid,
                         const mrf_zoom_schedule* sched, const void* vox, int32_t n_vox,
                         int64_t ld_vox, int32_t n_tr, const int32_t* init_idx,
                         mrf_result_view out, void* workspace, size_t ws_bytes, void* stream);

/* As mrf_zoom_search, with each voxel's prior centre given as a flat grid
 * index (device int64 [n_vox], e.g. the idx output of mrf_match_bruteforce;
 * a negative index starts at the grid origin). With mrf_zoom_schedule_local
 * this refines a brute-force result to the local CC maximum next to it. */
int mrf_zoom_search_from(mrf_context* ctx, const mrf_sequence* seq, const mrf_grid* grid,
                         const mrf_zoom_schedule* sched, const void* vox, int32_t n_vox,
                         int64_t ld_vox, int32_t n_tr, const int64_t* start_idx,
                         mrf_result_view out, void* workspace, size_t ws_bytes, void* stream);

/* Neighbour prior (Methods, Experiment 3: each voxel starts from a
 * neighbour's result with narrowed ranges), as a two-pass lattice over a
 * volume of n_slices slices of width x height voxels stored slice-major in
 * raster order (voxel v = (s*height + y)*width + x): pass 1 searches the
 * voxels with x % stride == 0 and y % stride == 0 without a prior; pass 2
 * starts every other voxel at the result of the nearest pass-1 voxel of its
 * slice (Chebyshev distance, ties to the lower raster index), with each axis
 * restricted to that centre +- sched->prior_half (entries < 0: whole axis).
 * Workspace as mrf_zoom_workspace for width*height*n_slices voxels. */
int mrf_zoom_search_lattice(mrf_context* ctx, const mrf_sequence* seq, const mrf_grid* grid,
                            const mrf_zoom_schedule* sched, const void* vox, int32_t width,
                            int32_t height, int32_t n_slices, int64_t ld_vox, int32_t n_tr,
                            int32_t stride, mrf_result_view out, void* workspace,
                            size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop over resident dictionaries (not part of the paper,
 * whose searches are one slice at a time; it serves the same two searches,
 * brute force (Theory Eq. 1 over the whole grid) and MRF-ZOOM (Theory: MRF
 * ZOOM; Methods: Experiment 2), to many slices that arrive over time).
 *
 * The server owns one scheduler thread and n_streams device streams.
 *   - mrf_server_register builds a slot: the sequence's dictionary over a
 *     grid, simulated once at the longest registered readout count and kept
 *     in HBM, plus the per-entry norms of every registered shorter prefix
 *     (computed from the stored values, identical to the norms a dictionary
 *     of that length gets from mrf_simulate_dictionary).
 *   - mrf_serve_submit is non-blocking. A request whose buffers could never
 *     fit in the budget beside the resident dictionaries is rejected at once
 *     (MRF_ERR_REJECTED, no ticket).
 *   - Admission is first-in first-out by HBM footprint: the head request is
 *     admitted when the footprints of all admitted requests plus its own fit
 *     in hbm_budget_bytes minus the resident bytes and fewer than max_inflight
 *     requests are admitted; later requests never overtake it.
 *   - Continuous batching: whenever a stream is idle, the admitted requests
 *     that share the oldest one's (slot, mode, n_tr) form one batch (up to
 *     max_batch_vox voxels): their voxels are gathered into one matrix, one
 *     search runs over it, and the results are scattered to each request's
 *     outputs. Requests that arrive while others run join the next batch on
 *     the next free stream, so brute-force and ZOOM batches overlap on the
 *     device.
 *   - Brute force: FP32 slots search with top_k = 2 (the margin needs the
 *     runner-up); BF16 slots search with top_k = 8 and FP32 re-scoring.
 *     ZOOM: the slot's grid with mrf_zoom_schedule_paper, no prior.
 * Each voxel's result depends only on that voxel and the slot: a request's
 * outputs are the same alone and in any mix.
 *
 * Ownership: vox and the out arrays are caller device memory and must stay
 * valid until mrf_serve_poll reports DONE, FAILED or CANCELLED. Requests are
 * remembered for the server's lifetime (a few hundred bytes each).
 * ---------------------------------------------------------------------- */
typedef struct mrf_server mrf_server;

typedef enum { MRF_SERVE_BRUTE = 0, MRF_SERVE_ZOOM = 1 } mrf_serve_mode;
typedef enum {
  MRF_REQ_QUEUED = 0,    /* submitted, waiting for admission or a stream */
  MRF_REQ_RUNNING = 1,   /* its batch is on the device */
  MRF_REQ_DONE = 2,
  MRF_REQ_FAILED = 3,    /* the batch failed; mrf_serve_poll sets mrf_last_error */
  MRF_REQ_CANCELLED = 4
} mrf_request_state;

typedef struct {
  size_t hbm_budget_bytes;   /* resident dictionaries + buffers of admitted requests */
  int32_t max_inflight;      /* admitted requests (waiting for a stream or running), >= 1 */
  int32_t n_streams;         /* device streams, one batch in flight on each, >= 1 */
  int32_t max_batch_vox;     /* voxels per batch; 0 = 65536 */
  /* Host-simulated device for testing the scheduler without a GPU: no device
   * work at all and the outputs are never written; registration allocates
   * nothing; a batch takes fake_ns_per_byte x its buffer bytes of wall time;
   * the batch holding ticket fake_fail_ticket (0 = none) fails. ctx and the
   * sequence may be NULL. */
  int32_t fake_device;
  double fake_ns_per_byte;
  uint64_t fake_fail_ticket;
  /* 1: brute-force results of BF16 slots are refined after the FP32
   * re-scoring by the unit-step local search (mrf_zoom_schedule_local, 8
   * rounds) started at them, so that each is a maximum of its unit
   * neighbours in FP32 (the best entry can fall outside the BF16 top 8 when
   * its neighbours' BF16 scores are within the BF16 rounding of it); n_sim
   * then counts the entries the refinement simulated. 0: re-scored results
   * as mrf_match_bruteforce returns them. */
  int32_t refine_bf16;
  /* Batching window, ms (>= 0): a (slot, mode) batch is launched once its
   * oldest request has waited this long since submission, or once it is full
   * (max_batch_vox, or the next request does not fit its reservation), or
   * while the server drains at close; 0 launches on any idle stream at once.
   * Larger windows trade latency for larger batches. */
  double batch_window_ms;
} mrf_server_config;

typedef struct {
  int32_t mode;        /* mrf_serve_mode */
  int32_t slot;
  int32_t n_tr;        /* readouts used; brute force: one of the slot's lengths;
                          ZOOM: any value up to the longest. A batch holds
                          requests of one slot and mode, of any readout counts:
                          ZOOM voxels of different counts share one launch
                          (mrf_zoom_search_ragged); brute force runs one GEMM
                          per count within the batch (the GEMM's K is shared) */
  int32_t n_vox;       /* >= 0; 0 completes at submission */
  const void* vox;     /* complex64 [n_vox][ld_vox] device */
  int64_t ld_vox;      /* >= n_tr */
  mrf_result_view out; /* idx required; n_sim filled by ZOOM requests */
} mrf_request;

typedef struct {
  size_t budget_bytes, resident_bytes, reserved_bytes, peak_reserved_bytes, arena_peak_bytes;
  int64_t submitted, rejected, done, failed, cancelled, batches, max_batch_requests;
  int32_t peak_inflight;
  /* per mode (0 brute force, 1 ZOOM): batches launched, requests they held,
   * and batches holding more than one readout count */
  int64_t admitted;
  int64_t mode_batches[2], mode_requests[2], mixed_length_batches[2];
} mrf_server_stats;

int mrf_server_create(mrf_context* ctx, const mrf_server_config* cfg, mrf_server** out);
/* n_tr: n_lengths readout counts (each <= the sequence length; multiples of
 * 4 for BF16). Blocks until the dictionary is built. MRF_ERR_REJECTED if the
 * dictionary does not fit in the budget. A sequence with temporal smoothing
 * is MRF_ERR_INVALID (shorter readout counts are served from prefixes of one
 * dictionary, and a smoothed entry's prefix is not the smoothed prefix). */
int mrf_server_register(mrf_server* srv, const mrf_sequence* seq, const mrf_grid* grid,
                        mrf_dtype dtype, const int32_t* n_tr, int32_t n_lengths, int32_t* slot);
int mrf_serve_submit(mrf_server* srv, const mrf_request* req, uint64_t* ticket);
/* Non-blocking. Times in ms since the server was created (host clock);
 * t_start is when the request's batch was launched, t_done when its
 * completion was observed (-1 while unknown). Unknown ticket: MRF_ERR_INVALID. */
int mrf_serve_poll(mrf_server* srv, uint64_t ticket, int32_t* state, double* t_submit_ms,
                   double* t_start_ms, double* t_done_ms);
/* Cancels a QUEUED request (its state becomes CANCELLED and its admission
 * reservation is released). A RUNNING request cannot be cancelled
 * (MRF_ERR_NOT_READY); on a finished one this is a no-op (MRF_OK). */
int mrf_serve_cancel(mrf_server* srv, uint64_t ticket);
int mrf_server_stats_read(mrf_server* srv, mrf_server_stats* out);
/* Drains: waits for every submitted request to finish, then frees the slots. */
int mrf_server_destroy(mrf_server* srv);

/* ------------------------------------------------------------------------
 * Device peak probes (measurement aids; not steps of the method). They give
 * the rates this GPU sustains for the operations the matching GEMMs and the
 * dictionary generator are bound by, so that achieved rates can be quoted as
 * fractions of measured peaks beside the published ones. Both launch on
 * `stream` (a hipStream_t, NULL = default), return without waiting, and are
 * timed by mrf_profile_* under the names given below.
 *
 * mrf_probe_mfma ("k_probe_mfma_f32" / "k_probe_mfma_bf16"): out_len / 256
 * workgroups of 256 threads; every wave runs `iters` rounds of four
 * independent MFMAs on register operands (MRF_F32: v_mfma_f32_32x32x2_f32,
 * 4096 flop each; MRF_BF16: v_mfma_f32_32x32x16_bf16, 32768 flop each), all
 * operand elements 0.5 and 0.25. out (device float[out_len], caller-owned)
 * receives each lane's sum of its 64 accumulator values, exactly 16 * iters
 * (MRF_F32) or 128 * iters (MRF_BF16) while that stays below 2^24. *flops
 * (host, may be NULL) receives the flops the launch performs.
 * Errors: out_len not a positive multiple of 256, iters < 1, bad dtype ->
 * MRF_ERR_INVALID (nothing launched).
 *
 * mrf_probe_mfma_varied ("k_probe_mfma_bf16_varied"): the MRF_BF16 loop of
 * mrf_probe_mfma with operands that vary by lane and element: element e of
 * operand fragment f (8 per lane, two per accumulator) in lane l is
 * 0.375 * ((7 l + 13 f + 29 e) mod 61) - 11 rounded to BF16. The matrix
 * cores draw more power on such data and the clock drops, so this is the
 * BF16 rate a GEMM on real data can approach. out (device float[out_len],
 * caller-owned) receives each lane's sum of its 64 accumulator values; the
 * operands are multiples of 1/8 below 12 in magnitude, so for iters <= 7
 * every partial sum is a multiple of 1/64 below 2^18 and the result is exact.
 * *flops as above. Errors as for mrf_probe_mfma.
 *
 * mrf_probe_write ("k_probe_write"): fills `bytes` (a multiple of 16) at dst
 * (16-byte aligned device memory, caller-owned) with one 16 B store per
 * thread, each workgroup writing one contiguous 4 KB piece; 16-byte element
 * i holds the words (pattern, i, pattern, i), i taken modulo 2^32.
 * Errors: bad size or alignment -> MRF_ERR_INVALID.
 * ---------------------------------------------------------------------- */
int mrf_probe_mfma(mrf_context* ctx, mrf_dtype dtype, int64_t iters, float* out, int64_t out_len,
                   double* flops, void* stream);
int mrf_probe_mfma_varied(mrf_context* ctx, int64_t iters, float* out, int64_t out_len,
                          double* flops, void* stream);
int mrf_probe_write(mrf_context* ctx, void* dst, int64_t bytes, uint32_t pattern, void* stream);

/* ------------------------------------------------------------------------
 * Kernel timing. When enabled, every launch of a named kernel
 * ("k_sim_dict", "k_match_f32" (the three-product FP32 GEMM), "k_match_bf16",
 * "k_rescore", "k_zoom", ...)
 * is bracketed by HIP events recorded on the stream it is launched on.
 * mrf_profile_read waits for those events and returns the summed elapsed
 * time and launch count since the last reset (reset = 1 clears them).
 * ---------------------------------------------------------------------- */
int mrf_profile_enable(mrf_context* ctx, int32_t enable);
int mrf_profile_read(mrf_context* ctx, const char* kernel, int32_t reset, double* total_ms,
                     int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
