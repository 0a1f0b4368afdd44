/*
 * act.h -- C ABI of the MI355X (gfx950) residue-based Adaptive Chirplet
 * Transform library (libact.so).
 *
 * The library decomposes real signals as s ~ sum_k c_k g(theta_k*) by matching
 * pursuit on the residual (Sec. III-A, Eq. (3)-(4)): for every order it
 * correlates the residual with a unit-norm Gaussian chirplet dictionary
 * (Eq. (1), real part, sampled on a 4-D grid of t_c, f_c, c, log dt), takes
 * the arg-max of |<g_i, r_k>|, refines the winner's parameters by maximising
 * <g(theta), r_k>^2 / <g,g>, computes c_k = <g*, r_k> with the refined unit
 * atom, and subtracts the projection.  Several channels are batched in one
 * call, as in the paper's stacked projection P = D X^T (Sec. IV-A, Sec. V-A).
 *
 * Conventions
 *  - Units are SI: t_c in s, f_c in Hz, c in Hz/s (the coefficient of
 *    (t - t_c)^2 in Eq. (1)), logdt = ln(dt / 1 s).  Samples are at t_n = n/fs.
 *  - theta is stored as double[4] = (t_c, f_c, c, logdt).
 *  - An axis is (lo, hi, count, half_open); its j-th value is
 *    lo + j*((hi-lo)/d) with d = count (half_open != 0) or count-1 (the last
 *    value of a closed axis is hi exactly; a one-value axis is lo).
 *    A (start, stop, step) range as printed in the paper's parameter table is
 *    the half-open axis (start, start + count*step, ceil((stop-start)/step), 1).
 *  - Dictionary index i = ((i_tc*n_fc + i_fc)*n_c + i_c)*n_ld + i_ld; ties in
 *    the arg-max go to the lowest index.
 *  - Memory: every pointer argument named *_dev is device memory owned by the
 *    caller and must stay valid until the work enqueued on `stream` completes.
 *    The plan owns its tables and workspace.  `stream` is a hipStream_t (NULL
 *    = the null stream).  Calls other than act_plan / act_plan_destroy only
 *    enqueue work and return; errors found on the host are returned before
 *    anything is enqueued.  Device-side conditions are reported per channel in
 *    flags (ACT_FLAG_*), never by aborting.
 *  - A plan is not re-entrant: do not use one plan from two streams at once.
 *  - No function throws or aborts; on error the status says why and
 *    act_last_error() returns a message (thread-local).
 */
#ifndef ACT_H
#define ACT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ACT_OK = 0,
    ACT_ERR_INVALID = 1,     /* bad argument (message in act_last_error) */
    ACT_ERR_NOMEM = 2,       /* device allocation or byte budget exceeded */
    ACT_ERR_HIP = 3,         /* a HIP runtime call failed */
    ACT_ERR_UNSUPPORTED = 4  /* valid request this build does not implement */
} act_status;

typedef struct {
    double lo, hi;
    int32_t count, half_open;
} act_axis;

/* Sampling rate, signal length and the four parameter axes of a dictionary:
 * the grid of atom parameters the caller's ranges span (Sec. III-A; Table
 * "Parameter ranges"). */
typedef struct {
    double fs_hz;
    int32_t n_samples;
    int32_t reserved;
    act_axis tc_s, fc_hz, c_hz_per_s, logdt_ln_s;
} act_grid;

/* Dictionary source of the coarse search. */
enum {
    ACT_DICT_SYNTH = 0, /* atoms synthesised on the device inside the search */
    ACT_DICT_TABLE = 1, /* atoms streamed from an HBM-resident table built by act_plan */
    ACT_DICT_LAG = 2    /* one time centre's atoms over every lag in an HBM-resident FP16 table
                           (time centres on integer samples that are multiples of 8): the scores
                           of all (channel, time centre) rows are one dense matrix product with
                           the residual's shifted windows; ACT_PREC_F16: plain plans (real or
                           complex atoms) and ragged plans of real atoms (ragged_tc_div a
                           multiple of 8); ACT_PREC_BF16: the same table in BF16, plain plans of
                           real atoms */
};

/* Arithmetic of the coarse search (rescoring, refinement, coefficients and
 * updates are FP64 in every mode). */
enum {
    ACT_PREC_F64 = 0,  /* FP64 correlation (ACT_DICT_SYNTH only) */
    ACT_PREC_F32 = 1,  /* FP32 correlation, certified FP64 rescoring of the candidates */
    ACT_PREC_BF16 = 2, /* BF16 x BF16 -> FP32 MFMA correlation over the atom table
                          (ACT_DICT_TABLE) or the lag table (ACT_DICT_LAG), certified FP64
                          rescoring */
    ACT_PREC_F16 = 3   /* FP16 x FP16 -> FP32 MFMA correlation over factor tables
                          (ACT_DICT_SYNTH) or the lag table (ACT_DICT_LAG), certified FP64
                          rescoring */
};

/* Per-channel flags written by act_decompose / act_refine. */
enum {
    ACT_FLAG_NONFINITE = 1,       /* the input channel holds a NaN or an infinity */
    ACT_FLAG_REFINE_REJECTED = 2, /* refinement would lower J; the grid theta was kept */
    ACT_FLAG_CAND_OVERFLOW = 8,   /* more atoms than the candidate capacity lay inside the
                                     certified margin; the search was re-run once with the
                                     exact threshold (set only if even that overflowed) */
    ACT_FLAG_RAGGED_EMPTY = 16,   /* a ragged signal has no time centre (length < divisor) */
    ACT_FLAG_BAD_LENGTH = 32      /* a ragged length outside [0, n_samples]: channel skipped */
};

typedef struct {
    act_grid grid;          /* ragged plans: the t_c axis is ignored, see ragged_tc_div */
    int32_t dict;           /* ACT_DICT_* */
    int32_t prec;           /* ACT_PREC_* */
    int32_t max_batch;      /* most channels one call may pass (>= 1) */
    int32_t cand_cap;       /* candidate list capacity per channel; 0 = 4096 (16384 for BF16
                               and FP16-synthesis plans, 131072 for ragged plans, 524288
                               for ragged lag plans) */
    int32_t refine_steps;   /* L-BFGS iterations per order in act_decompose; 0 = none */
    int32_t ragged;         /* 1: channels have their own lengths (len_dev/off_dev) and
                               grids with floor(len/ragged_tc_div) time centres */
    int32_t ragged_tc_div;  /* samples per time centre of a ragged plan (e.g. 32) */
    int32_t support_cut;    /* ACT_PREC_F16 synthesis only. 0: dense correlation over every
                               sample. 1: each block of atoms skips the samples where the
                               Gaussian envelope of all its log-durations has tail energy
                               below 2^-48 (relative bound 2^-24 on the score, added to the
                               certified margin; the FP64 rescoring is unchanged, so the
                               selected atoms are the same) */
    int32_t prior_act;      /* 1: the prior ACT that Sec. III-A contrasts with (its table of
                               algorithmic properties), for stability comparisons: atoms keep
                               Eq. (1)'s prefactor (sqrt(pi) dt)^-1/2 instead of unit norm; the
                               exact FP64 search, the refinement of <s, g>^2 and the coefficient
                               <g*, s> all use the original signal s, repeated each order
                               (r_{k+1} = r_k - c g*). ACT_DICT_SYNTH + ACT_PREC_F64, not ragged;
                               coef_dev then multiplies these atoms (act_reconstruct uses them);
                               gap_dev is 0 */
    int32_t complex_atoms;  /* 1: complex (analytic) atoms g = E exp(i phi) of Eq. (1), E the
                               Gaussian envelope and phi = 2 pi (c tau^2 + f_c tau), scored by
                               |<g_hat, r>| = sqrt(<r, E cos phi>^2 + <r, E sin phi>^2) / |E|
                               (unit norm over the samples present), refined on its square,
                               and removed from the real residual by the least-squares fit of
                               amplitude and phase: r -= alpha E cos phi + beta E sin phi.
                               coef_dev then holds the pair (alpha, beta) per order
                               ([batch][order][2], amplitudes of the un-normalised parts), which
                               act_reconstruct takes in the same layout.  act_correlate returns
                               |<g_hat, r>|, act_refine maximises |<g_hat, r>|^2.
                               ACT_DICT_SYNTH with ACT_PREC_F64 or ACT_PREC_F32, not ragged,
                               not with prior_act or support_cut; act_value_and_grad and
                               act_lem_decompose return ACT_ERR_UNSUPPORTED */
} act_plan_desc;

typedef struct act_plan_s* act_plan_t;

/* Builds a plan: validates the grid, uploads the axis values, and for
 * ACT_DICT_TABLE synthesises every atom in FP64 on the device, scales it to
 * unit l2 norm over the n_samples present before any search (Sec. III-A) and
 * stores it as FP32 or BF16 rows; for
 * ACT_DICT_SYNTH it builds the small factor tables the search kernels combine.
 * Synchronises `stream` before returning.  On success *out owns all plan
 * memory until act_plan_destroy.  Errors: ACT_ERR_INVALID (counts < 1, n < 1,
 * fs <= 0, non-finite or reversed bounds, unknown dict/prec, F64 with a
 * table), ACT_ERR_NOMEM (a table, lag table or lag-energy table larger than
 * the free device memory: refused before it is allocated; or a failed
 * allocation), ACT_ERR_HIP. */
act_status act_plan(const act_plan_desc* desc, void* stream, act_plan_t* out);

/* Frees everything the plan owns (after synchronising its last stream).
 * NULL is ignored. */
void act_plan_destroy(act_plan_t plan);

/* Plan facts: ACT_Q_ATOMS (dictionary size), ACT_Q_TABLE_BYTES (table bytes,
 * 0 for synthesis), ACT_Q_N_PAD (padded row length of tables and shadows),
 * ACT_Q_CAND_CAP, ACT_Q_WORKSPACE_BYTES, ACT_Q_LAG_RESIDENT (1 when the
 * lag-table search of 32 or more channels can keep each group of 32
 * channels' residual copy resident in LDS: launch-shape form 0).  Returns -1
 * for an unknown key. */
enum { ACT_Q_ATOMS = 0, ACT_Q_TABLE_BYTES = 1, ACT_Q_N_PAD = 2, ACT_Q_CAND_CAP = 3,
       ACT_Q_WORKSPACE_BYTES = 4, ACT_Q_LAG_RESIDENT = 5 };
int64_t act_plan_query(act_plan_t plan, int32_t key);

/* Matrix-core work of one pass-0 coarse search of `batch` channels, in flops
 * (2 per multiply-add), with every channel taking part: for ACT_DICT_LAG
 * plans, the sum over the launch's tiles of their stages x 128 rows x the
 * tile's columns x 128 lags x 2.  Tiles run only the lags where their columns
 * hold nonzero FP16 (BF16) entries, so this is well below the dense count
 * 2 atoms n_samples batch (padding rows and columns included).  Diagnostic
 * for utilisation figures; host-only, no device work.  Errors:
 * ACT_ERR_INVALID (NULL plan or flops, batch outside [1, max_batch]),
 * ACT_ERR_UNSUPPORTED (plans of other dictionaries, and ragged plans, whose
 * tiles depend on the call's lengths). */
act_status act_search_flops(act_plan_t plan, int32_t batch, double* flops);

/* Matrix-core work the coarse searches of a lag-table or FP16-synthesis plan
 * actually executed, as counted by the device: every pass-0 search launch
 * (the first search of each order, in act_decompose, act_tune or their graph
 * replays; not the exact-threshold reruns, not act_correlate) adds the MFMA
 * instructions its waves issued (x 32 x 32 x 16 multiply-adds x 2 = flops)
 * and 1 to a launch count.  The counts cover every launch since the plan was
 * built or since the last call of this function, which returns them in
 * *flops and *launches and resets them.  For uneven batches, whose tiles
 * depend on the call's lengths, this is the executed work per call (the
 * launches of one act_decompose call are alike).  Synchronises the plan's
 * last stream.  Errors: ACT_ERR_INVALID (NULL argument),
 * ACT_ERR_UNSUPPORTED (other plans), ACT_ERR_HIP. */
act_status act_search_executed(act_plan_t plan, double* flops, int64_t* launches);

/* Residue-based matching pursuit of `batch` channels for `order` orders
 * (Sec. III-A, Fig. "simplified residue-driven ACT iteration"):
 *   resid_dev   in: the signals, out: the residuals r_P.  f64, channel b at
 *               [b*n_samples, (b+1)*n_samples) for a plain plan, at
 *               [off[b], off[b]+len[b]) for a ragged plan.
 *   approx_dev  out: a_P (same layout), or NULL.
 *   len_dev, off_dev  ragged plans only (int32 lengths, int64 offsets); NULL otherwise.
 *   theta_dev   out: [batch][order][4] refined parameters.
 *   coef_dev    out: [batch][order] coefficients c_k = <g*, r_k> ([batch][order][2]
 *               amplitude pairs for complex_atoms plans).
 *   index_dev   out: [batch][order] flat grid index of the coarse winner.
 *   energy_dev  out: [batch][order+1] |r_k|^2 (k = 0 is |s|^2); the normalised
 *               residue of Eq. (5) is energy[k]/energy[0].
 *   gap_dev     out: [batch][order] lower bound of (|p|_(1)-|p|_(2))/|p|_(1),
 *               the relative margin of the coarse winner, or NULL.
 *   flags_dev   out: [batch] ACT_FLAG_* bits.
 * The whole pass runs on the device; the host enqueues it and returns.  The
 * first call with a given set of (batch, order, pointer) arguments captures
 * the launch sequence into a HIP graph owned by the plan (at most 4 are kept);
 * later calls with the same arguments replay it as a single launch on
 * `stream`.  Phase timing (act_timing_enable) launches the kernels directly.
 * Errors: ACT_ERR_INVALID (batch outside [1, max_batch], order < 1, NULL
 * required pointer, ragged pointers missing or given to a plain plan). */
act_status act_decompose(act_plan_t plan, int32_t batch, const int32_t* len_dev,
                         const int64_t* off_dev, double* resid_dev, double* approx_dev,
                         int32_t order, double* theta_dev, double* coef_dev, int64_t* index_dev,
                         double* energy_dev, double* gap_dev, int32_t* flags_dev, void* stream);

/* LEM-inspired hierarchical coarse-to-fine search (Sec. VII, Fig.
 * "Hierarchical LEM-inspired coarse-to-fine search"): per order, Latin
 * hypercube samples of the parameter hull snapped to the level-0 steps, the
 * top-k distinct candidates by |<g_hat, r_k>|, then for each refinement level
 * the local families candidate + i * step_l (|i_d| <= radius_d, members
 * outside the hull dropped) pooled and re-ranked to the top-k; the best
 * candidate initialises the plan's refinement (scales capped by the finest
 * step), then c_k and the update.  No dictionary is evaluated beyond these
 * candidates. */
typedef struct {
    int32_t samples;        /* LHS samples per order (>= 1) */
    int32_t levels;         /* refinement levels, 0..7 */
    int32_t topk;           /* candidates kept per stage, 1..16 */
    int32_t reserved;
    int32_t radius[4];      /* neighbourhood half-width in steps (t_c, f_c, c, ln dt), >= 0 */
    double step[8][4];      /* step of level 0..levels per axis (t_c s, f_c Hz, c Hz/s, ln dt), > 0 */
} act_lem_desc;

/* Hierarchical decomposition of `batch` channels of a plain ACT_DICT_SYNTH +
 * ACT_PREC_F64 plan (the grid gives the parameter hull and the refinement box).
 *   lhs_dev   in: [batch][order][samples][4] Latin-hypercube uniforms in [0,1)
 *             (the random draws are the caller's, so runs are reproducible).
 *   resid_dev in/out as act_decompose; approx_dev optional.
 *   theta_dev [batch][order][4], coef_dev [batch][order],
 *   energy_dev [batch][order+1], flags_dev [batch] as act_decompose.
 * Candidates per stage: max(samples, topk * prod(2 radius_d + 1)) <= 8192;
 * the plan keeps a workspace of that many candidates per channel (allocated
 * on first use).  Errors: ACT_ERR_INVALID (bad settings or pointers),
 * ACT_ERR_UNSUPPORTED (plan not plain FP64 synthesised). */
act_status act_lem_decompose(act_plan_t plan, const act_lem_desc* cfg, int32_t batch,
                             const double* lhs_dev, double* resid_dev, double* approx_dev,
                             int32_t order, double* theta_dev, double* coef_dev, double* energy_dev,
                             int32_t* flags_dev, void* stream);

/* Bytes of the device array that act_lem_decompose_noalloc uses as its
 * workspace (one array per device, held until the process ends). */
#define ACT_LEM_SCRATCH_BYTES (16u << 20)

/* act_lem_decompose for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same settings, arguments, kernels and results, but the per-channel
 * candidate workspace (batch x cap x 41 bytes, cap = max(samples,
 * topk * prod(2 radius_d + 1))) lives in a fixed device array of
 * ACT_LEM_SCRATCH_BYTES per device instead of plan memory allocated on first
 * use.  The call allocates nothing (no hipMalloc, no events, no graphs); the
 * caller still owns every argument buffer.  Every call on one device shares
 * that array, so calls that overlap in time on one device (two streams, two
 * threads) race and must be serialised by the caller; the array keeps the
 * last call's contents, none of which a later call reads.  Phase timing does
 * not apply.  Errors: as act_lem_decompose, plus ACT_ERR_INVALID when
 * batch x cap x 41 exceeds ACT_LEM_SCRATCH_BYTES. */
act_status act_lem_decompose_noalloc(act_plan_t plan, const act_lem_desc* cfg, int32_t batch,
                                     const double* lhs_dev, double* resid_dev, double* approx_dev,
                                     int32_t order, double* theta_dev, double* coef_dev, double* energy_dev,
                                     int32_t* flags_dev, void* stream);

/* Continuous refinement alone (Sec. III-A "BFGS refinement"), for m
 * independent problems: from theta0 maximise J(theta) = <r, g(theta)>^2 /
 * <g(theta), g(theta)> with the plan's L-BFGS (box = the plan grid's hull,
 * coordinates scaled by the atom's resolution, at most `steps` iterations).
 *   resid_dev [m][n_samples] f64, theta0_dev [m][4], theta_dev [m][4] out,
 *   value_dev [m] out (J at theta), flags_dev [m] out or NULL.
 * Errors: ACT_ERR_INVALID (m < 1, steps < 0, NULL pointers, ragged plan). */
act_status act_refine(act_plan_t plan, int32_t m, const double* resid_dev,
                      const double* theta0_dev, int32_t steps, double* theta_dev,
                      double* value_dev, int32_t* flags_dev, void* stream);

/* act_refine with FP32 arithmetic (Sec. III-A refinement; real atoms of the
 * residue-based ACT): resid_dev is [m][n_samples] float; every objective
 * evaluation forms each sample's terms in FP32 (the phase reduced modulo one
 * cycle in FP64, then FP32 envelope, trigonometry, products and per-thread
 * sums; the block adds the threads' partial sums in FP64).  The coordinate
 * scales and the 4-parameter L-BFGS bookkeeping stay FP64.  The iteration
 * stops when the projected gradient is below 1e-6 max(1, J) (FP32 resolves J
 * to about 1e-7) and the line search's approximate-Wolfe test allows
 * f_new <= f + 1e-6 |f|; otherwise as act_refine.  value_dev holds J at
 * theta in the same FP32 arithmetic.  Errors: as act_refine, plus
 * ACT_ERR_UNSUPPORTED for complex_atoms and prior_act plans. */
act_status act_refine_f32(act_plan_t plan, int32_t m, const float* resid_dev, const double* theta0_dev,
                          int32_t steps, double* theta_dev, double* value_dev, int32_t* flags_dev, void* stream);

/* Forward and adjoint of the refinement objective for m (residual, theta)
 * pairs: value J = <r,g>^2/<g,g>, dtheta = dJ/d(t_c, f_c, c, logdt) and
 * optionally dr = dJ/dr = 2 <r, g_hat> g_hat.  dtype ACT_PREC_F64 (resid and
 * dr are double) or ACT_PREC_F32 (resid and dr are float; theta, value and
 * dtheta are double, the arithmetic is FP32).
 *   resid_dev [m][n_samples], theta_dev [m][4], value_dev [m],
 *   dtheta_dev [m][4], dr_dev [m][n_samples] or NULL.
 * Errors: ACT_ERR_INVALID. */
act_status act_value_and_grad(act_plan_t plan, int32_t m, int32_t dtype, const void* resid_dev,
                              const double* theta_dev, double* value_dev, double* dtheta_dev,
                              void* dr_dev, void* stream);

/* Approximation sum_k c_k g_hat(theta_k) per channel (Eq. (3)), FP64.
 * theta_dev [batch][order][4], coef_dev [batch][order]; out_dev has the
 * layout of resid_dev in act_decompose (len/off for ragged plans).
 * Errors: ACT_ERR_INVALID. */
act_status act_reconstruct(act_plan_t plan, int32_t batch, int32_t order, const double* theta_dev,
                           const double* coef_dev, const int32_t* len_dev, const int64_t* off_dev,
                           double* out_dev, void* stream);

/* Coarse-search scores in the plan's arithmetic, for checking: score[b][j] =
 * <g_hat_{atom_begin+j}, r_b> for j < atom_count, as the search computes it
 * (FP32 result for F32/BF16 plans, written as double).  resid_dev is
 * [batch][n_samples] f64 (plain plans only).
 * Errors: ACT_ERR_INVALID (range outside the dictionary, ragged plan). */
act_status act_correlate(act_plan_t plan, int32_t batch, const double* resid_dev,
                         int64_t atom_begin, int64_t atom_count, double* score_dev, void* stream);

/* Launch shape of the coarse search kernel (a tuning choice; results do not
 * depend on it: the certified selection is exact for every shape). */
typedef struct {
    int32_t grid_per_cu;    /* persistent search workgroups per compute unit */
    int32_t chan_per_fc;    /* FP16 synthesis of several channels: channels that share an f_c among a
                               tile's 128 columns (power of two <= 64); 0 for the other searches */
    int32_t from_cache;     /* 1: taken from the cache file without timing */
    int32_t form;           /* lag-table search of plain plans on >= 32 channels: 0 keeps each group of
                               32 channels' residual copy resident in LDS (where the grid allows it;
                               grid_per_cu is then unused), 1 stages the residual per tile */
    double ms;              /* mean search time per launch with this shape */
} act_launch_shape;

/* Autotuner of the batched search's tile and grid shapes (the stacked channels
 * of Sec. V-A and uneven batches): times the plan's pass-0 coarse search on
 * `batch` channels of resid_dev for every candidate shape -- workgroups per CU
 * of the persistent grid, the lag-table search's form and, for the FP16
 * synthesis of several channels, the channels per f_c of a tile -- `reps`
 * launches each, and keeps the fastest for
 * later act_decompose / act_correlate calls with this batch size (captured
 * graphs are rebuilt).
 *   resid_dev, len_dev, off_dev  as act_decompose; read only.  The plan's
 *               search copy of the residual and its candidate workspace are
 *               overwritten.
 *   reps        timed launches per candidate (1..100).
 *   cache_path  text file of earlier choices or NULL: a line for the same
 *               device, plan shape and batch is applied without timing; a new
 *               choice is appended (one line: device, CU count, dict, prec,
 *               n_samples, axis counts, ragged, divisor, support_cut,
 *               complex_atoms, batch, grid_per_cu, chan_per_fc, form, ms).
 *   out         the choice, or NULL.
 * Synchronises `stream`.  Errors: ACT_ERR_INVALID (batch outside
 * [1, max_batch], reps outside [1, 100], NULL residual, ragged pointers
 * missing), ACT_ERR_UNSUPPORTED (prior_act plans: their search has no tunable
 * shape), ACT_ERR_HIP. */
act_status act_tune(act_plan_t plan, int32_t batch, const int32_t* len_dev, const int64_t* off_dev,
                    const double* resid_dev, int32_t reps, const char* cache_path, act_launch_shape* out,
                    void* stream);

/* Applies `shape` (grid_per_cu in [1, 64], chan_per_fc in [0, 64], form 0 or
 * 1; from_cache and ms ignored) to later searches of `batch` channels, as an
 * act_tune choice would (captured graphs are rebuilt).  Results do not depend
 * on the shape.  Errors: ACT_ERR_INVALID (NULL plan or shape, batch outside
 * [1, max_batch], fields outside their ranges). */
act_status act_set_launch_shape(act_plan_t plan, int32_t batch, const act_launch_shape* shape);

/* Phase timing of act_decompose, for measurement.  While enabled, every
 * launch of each phase of an order -- 0: search, 1: exact-threshold rerun,
 * 2: FP64 rescoring, 3: select/refine/update -- is bracketed by HIP events on
 * the caller's stream.  act_timing_read synchronises on those events, writes
 * the summed milliseconds ms[4] and launch counts launches[4] since the last
 * read, and clears them.  Errors: ACT_ERR_INVALID (NULL plan or outputs). */
act_status act_timing_enable(act_plan_t plan, int32_t enable);
act_status act_timing_read(act_plan_t plan, double* ms, int64_t* launches);

/* Measurement probes (not part of the method), for reporting achievable peaks
 * beside the datasheet ones.  The caller times each launch on `stream`.
 * act_probe_read: one grid-stride streaming read of `bytes` (a multiple of
 *   16) from buf_dev (16-byte aligned device memory the caller owns; use a
 *   buffer well above the last-level cache), blocks_per_cu x CUs workgroups of
 *   256 threads, 8 16-byte non-temporal loads in flight per thread; nothing is
 *   written (sink_dev, one float, is written only for an impossible sum).
 * act_probe_mfma: blocks_per_cu x CUs workgroups of 4 waves, each wave
 *   `iters` rounds of 4 independent 32x32 MFMAs (prec ACT_PREC_BF16:
 *   v_mfma_f32_32x32x16_bf16, ACT_PREC_F16: _f16, ACT_PREC_F32:
 *   v_mfma_f32_32x32x2_f32) with no memory traffic; *flops = the flops the
 *   launch executes (2 per multiply-add).
 * Errors: ACT_ERR_INVALID (bad sizes, alignment or counts), ACT_ERR_HIP. */
act_status act_probe_read(const void* buf_dev, int64_t bytes, int32_t blocks_per_cu, float* sink_dev, void* stream);
act_status act_probe_mfma(int32_t prec, int32_t iters, int32_t blocks_per_cu, float* sink_dev, double* flops,
                          void* stream);

const char* act_status_string(act_status status);
const char* act_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ACT_H */
