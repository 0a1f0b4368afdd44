// act_common.h -- internal declarations of libact (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/act.h"

namespace act {

constexpr int kWave = 64;
constexpr double kTwoPi = 6.283185307179586476925286766559;

// --------------------------------------------------------------------------
// host-side error plumbing
// --------------------------------------------------------------------------
void set_error(const std::string& msg);

#define ACT_HIP(call)                                                               \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            ::act::set_error(std::string(#call) + ": " + hipGetErrorString(e_));    \
            return ACT_ERR_HIP;                                                     \
        }                                                                           \
    } while (0)

#define ACT_REQUIRE(cond, msg)                                                      \
    do {                                                                            \
        if (!(cond)) {                                                              \
            ::act::set_error(msg);                                                  \
            return ACT_ERR_INVALID;                                                 \
        }                                                                           \
    } while (0)

// --------------------------------------------------------------------------
// dictionary geometry passed to kernels by value
// --------------------------------------------------------------------------
struct GridDev {
    double fs;            // sampling rate [Hz]
    const double* axis;   // concatenated axis values: tc | fc | c | logdt
    int n;                // samples per signal (ragged plans: of this channel)
    int n_pad;            // padded row length (multiple of 256; ragged: of the longest)
    int cnt[4];           // n_tc, n_fc, n_c, n_ld
    int off[4];           // offsets of each axis inside `axis`
    long long atoms;      // n_tc*n_fc*n_c*n_ld
    int ragged_div;       // ragged plans: samples per time centre (0: plain plan)
    double tc_step;       // ragged channel: spacing of its time centres [s]
};

// grid-hull box and grid spacing used by the refinement
struct BoxDev {
    double step[4], lo[4], hi[4];
};

struct act_plan_impl;

// flat index -> parameter vector (t_c, f_c, c, logdt); order of Sec. III-A
__device__ __forceinline__ void grid_theta(const GridDev& g, long long i, double th[4]) {
    int id[4];
#pragma unroll
    for (int a = 3; a >= 0; --a) {
        id[a] = (int)(i % g.cnt[a]);
        i /= g.cnt[a];
    }
#pragma unroll
    for (int a = 1; a < 4; ++a) th[a] = g.axis[g.off[a] + id[a]];
    // a ragged channel's time centres form the half-open axis (0, n_tc div/fs,
    // n_tc): value j = 0 + j * step
    th[0] = g.ragged_div ? (double)id[0] * g.tc_step : g.axis[g.off[0] + id[0]];
}

// Geometry of channel b: its samples, offset in the packed residual, and its
// own dictionary (a ragged channel has floor(len/div) time centres, one every
// div samples; a plain channel uses the plan grid).
struct ChanGeom {
    GridDev g;          // the channel's grid
    long long off;      // first sample in the packed residual / approximation
    double box_step0, box_lo0, box_hi0;  // refinement box along t_c
};

__device__ __forceinline__ ChanGeom chan_geom(const GridDev& g, int b, const int* len,
                                              const long long* off) {
    ChanGeom c;
    c.g = g;
    if (g.ragged_div) {
        int n = len[b];
        if (n < 0 || n > g.n) n = 0;  // out-of-range lengths: no samples (flagged by the init pass)
        const int ntc = n / g.ragged_div;
        c.g.n = n;
        c.g.cnt[0] = ntc;
        c.g.tc_step = ntc > 0 ? ((double)(ntc * g.ragged_div) / g.fs) / (double)ntc : 1.0;
        c.g.atoms = (long long)ntc * g.cnt[1] * g.cnt[2] * g.cnt[3];
        c.off = off[b];
        c.box_step0 = ntc > 1 ? c.g.tc_step : 1.0;
        c.box_lo0 = 0.0;
        c.box_hi0 = ntc > 1 ? (double)(ntc - 1) * c.g.tc_step : 0.0;
    } else {
        c.off = (long long)b * g.n;
        c.box_step0 = c.box_lo0 = c.box_hi0 = 0.0;  // unused: the plan box applies
    }
    return c;
}

// One sample of the real Gaussian chirplet of Eq. (1) without its analytic
// prefactor: exp(-(1/2)(tau/dt)^2) cos(2 pi (c tau^2 + f_c tau)), tau = t - t_c.
// cospi keeps the phase reduction exact for the large phases of long signals.
__device__ __forceinline__ double atom_sample64(double t, double tc, double fc, double c,
                                                double inv_dt) {
    double tau = t - tc;
    double u = tau * inv_dt;
    double e = exp(-0.5 * u * u);
    double cyc = c * tau * tau + fc * tau;
    return e * cospi(2.0 * cyc);
}

// One sample of the complex chirplet E exp(i phi) (no prefactor): its real
// and imaginary parts and the envelope E.
__device__ __forceinline__ void atom_parts64(double t, double tc, double fc, double c, double inv_dt,
                                             double& re, double& im, double& env) {
    const double tau = t - tc;
    const double u = tau * inv_dt;
    env = exp(-0.5 * u * u);
    double si, co;
    sincospi(2.0 * (c * tau * tau + fc * tau), &si, &co);
    re = env * co;
    im = env * si;
}

// BF16 bits of an FP32 value, rounded to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// sample time of index k
__device__ __forceinline__ double sample_time(int k, double fs) { return (double)k / fs; }

// --------------------------------------------------------------------------
// reductions
// --------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        T w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

// v plus the value that DPP control CTRL moves into this lane; rows outside
// ROWS (and lanes without a source) add zero
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xf, false);
    return v + __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes of a wave with DPP row moves (no LDS traffic): lane
// pairs, quads, half rows, rows (mirrors); rows 1 and 3 then add rows 0 and 2
// (row_bcast15) and row 3 adds rows 0-1 (row_bcast31), so lane 63 holds the
// total, returned to every lane.  Fixed order: deterministic.
__device__ __forceinline__ double wave_total(double v) {
    v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xf>(v);  // row_mirror
    v = dpp_add<0x142, 0xa>(v);  // row_bcast15 into rows 1, 3
    v = dpp_add<0x143, 0xc>(v);  // row_bcast31 into rows 2, 3
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum NV doubles over a block of NT threads; every thread receives the totals.
// `lds` must hold block_sum_lds(NT, NV) doubles.  Deterministic: fixed order
// (the wave's DPP tree, then every thread adds the wave partials in order).
// Called by every thread of the block (it holds barriers).
constexpr int block_sum_lds(int nt, int nv) { return nv * (nt / kWave + 1); }

template <int NT, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_total(v[j]);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) lds[j * NW + w] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NW; ++k) s += lds[j * NW + k];
        v[j] = s;
    }
    __syncthreads();
}

// Sum NV doubles over a block of NT threads by transposition through LDS, for
// the wider reductions of the refinement (NV of 9 to 13): every thread stores
// its NV partial sums as one row; then P threads per value (P = 16, 8 or 4, as
// many as NV P <= NT allows) each add NT/P rows pairwise, and the P partials of
// a value, which sit in P adjacent lanes, are added by DPP moves within their
// row (each lane of the group then holds the same bits).  Two barriers, one
// LDS row write and NT/P reads per thread, against NV full wave trees for
// block_sum.  `lds` must hold block_sum_tr_lds(NT, NV) doubles; every thread
// receives the totals; deterministic (fixed order).  A block of several groups
// of NT threads sums each group apart (thread threadIdx.x mod NT of the group,
// each group with its own `lds`); all groups must call it together (it holds
// block-wide barriers).
constexpr int tr_stride(int nv) { return nv | 1; }   // odd row stride: rows start in different banks
constexpr int tr_parts(int nt, int nv) { return nv * 16 <= nt ? 16 : nv * 8 <= nt ? 8 : 4; }
constexpr int block_sum_tr_lds(int nt, int nv) { return nt * tr_stride(nv) + nv; }

template <int NT, int NV>
__device__ __forceinline__ void block_sum_tr(double (&v)[NV], double* lds) {
    constexpr int SP = tr_stride(NV), P = tr_parts(NT, NV), PER = NT / P;
    static_assert(NV * P <= NT && NT % P == 0, "block_sum_tr: too many values for the block");
    static_assert(NT % kWave == 0, "block_sum_tr: groups of whole waves");
    const int t = (int)(threadIdx.x % NT);
#pragma unroll
    for (int j = 0; j < NV; ++j) lds[t * SP + j] = v[j];
    __syncthreads();
    if (t < NV * P) {            // whole groups of P lanes: the DPP moves stay inside a group
        const int j = t / P, part = t % P;
        double x[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) x[i] = lds[(part + P * i) * SP + j];
#pragma unroll
        for (int w = PER / 2; w >= 1; w /= 2) {
#pragma unroll
            for (int i = 0; i < w; ++i) x[i] += x[i + w];
        }
        double s = x[0];
        s = dpp_add<0xB1, 0xf>(s);                      // quad_perm [1,0,3,2]
        s = dpp_add<0x4E, 0xf>(s);                      // quad_perm [2,3,0,1]
        if constexpr (P >= 8) s = dpp_add<0x141, 0xf>(s);  // row_half_mirror
        if constexpr (P >= 16) s = dpp_add<0x140, 0xf>(s); // row_mirror
        if (part == 0) lds[NT * SP + j] = s;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = lds[NT * SP + j];
}

// order-preserving bit patterns of non-negative floats / doubles
__device__ __forceinline__ unsigned fbits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ float bitsf(unsigned u) { return __uint_as_float(u); }

}  // namespace act

// --------------------------------------------------------------------------
// the plan (opaque to callers)
// --------------------------------------------------------------------------
struct act_plan_s {
    act_plan_desc desc;
    act::GridDev grid;        // grid of the plain plan (ragged: widest grid)
    act::BoxDev box;
    long long atoms = 0;
    int n = 0, n_pad = 0, cap = 0, max_batch = 0;
    double* axis_dev = nullptr;

    // dictionary table (ACT_DICT_TABLE)
    long long atoms_pad = 0;  // table rows (BF16: multiple of the 512-atom MFMA tile)
    double* inv_norm = nullptr;  // [atoms] 1/|g_i| in FP64 (tables only)
    void* table = nullptr;
    size_t table_bytes = 0;

    // synthesised dictionary (ACT_DICT_SYNTH with FP32): shift-invariant
    // factor tables [rows][fac_w], FP32 inverse norms, integer time centres
    void* fac_u = nullptr;
    void* fac_v = nullptr;
    void* fac_c = nullptr;
    void* fac_s = nullptr;
    int fac_w = 0, n_cl = 0;
    float* inv_norm32 = nullptr;
    int* tc_shift = nullptr;
    void* fac_u16 = nullptr;  // ACT_PREC_F16: FP16 copies of the four factor tables
    void* fac_v16 = nullptr;
    void* fac_c16 = nullptr;
    void* fac_s16 = nullptr;
    double* env_q = nullptr;  // ACT_PREC_F16: [n_ld][fac_w] prefix sums of the squared envelope
    float* rscale = nullptr;  // ACT_PREC_F16: [B] power-of-two scale of the FP16 search copy
    double* ebmul = nullptr;  // ACT_PREC_F16: [B] per-atom bound factor (times |E_w| / |g_w|)
    int* perm = nullptr;      // ACT_PREC_F16 ragged: [B] channels by decreasing length
    unsigned* tmax = nullptr; // ACT_PREC_F16: [B][n_tc] largest pass-0 upper bound per time centre
    int* ld_half = nullptr;   // ACT_PREC_F16: [n_ld] half-support in samples of each log-duration
    float* inv_full32 = nullptr;  // ACT_PREC_F16 ragged: [n_fc][n_cl] 1/|g| over all lags
    double* prior_s = nullptr;       // prior ACT: [B][n] original signals
    double* prior_part = nullptr;    // prior ACT: [B][search blocks] best |score| per block
    long long* prior_pidx = nullptr; // prior ACT: [B][search blocks] its atom index
    double* lem_cand = nullptr;      // LEM: [B][lem_cap][4] candidate parameters
    double* lem_score = nullptr;     // LEM: [B][lem_cap] candidate scores
    int lem_cap = 0;
    int lag_q_pad = 0;        // ACT_DICT_LAG: table columns (n_fc n_c n_ld padded to 256)
    float* lag_inv = nullptr; // ACT_DICT_LAG: [n_tc][lag_q_pad] FP32 1/|g| in the table's column order
    int* lag_span = nullptr;  // ACT_DICT_LAG: [lag_q_pad / 32] k-step range of each block's nonzero entries
    int* lag_order = nullptr; // ACT_DICT_LAG: tile column-block orders (128-column tiles, then 256)
    int lag_order_wide = 0;   // ACT_DICT_LAG: offset of the 256-column order in lag_order
    std::vector<int> lag_span_host;  // ACT_DICT_LAG: host copy of lag_span (lo, hi pairs)
    float* lag_rho = nullptr;  // ragged ACT_DICT_LAG: [256-column blocks][lag_rho_d] bound of |g_full| / |g_w|
    int lag_rho_d = 0;         // ragged ACT_DICT_LAG: distances to the signal end below which lag_rho applies
    int* lag_rows = nullptr;   // ragged ACT_DICT_LAG: per call, [channel groups + 1] prefix of time groups
    // ACT_DICT_LAG, real atoms of plain plans: the resident-residual search
    // (lag_rs_cp null when the grid does not allow it)
    int* lag_rs_cp = nullptr;     // [8][lag_rs_cp_per_x] column pairs per XCD, longest band first
    int* lag_rs_count = nullptr;  // [8] column pairs per XCD
    int lag_rs_cp_per_x = 0, lag_rs_ncg = 0;
    int lag_rs_glo = 0, lag_rs_len = 0, lag_rs_stride = 0;  // LDS copy: guard, samples, row stride
    int* lag_rs_units = nullptr;  // unit descriptors in list order (k_search_lag_rs)
    float* lag_rs_map = nullptr;  // [lag_rs_ncg][units][32] pass-0 largest |score| per channel and unit
    int* lag_rs_pairs = nullptr;  // pass 1: count, then the flagged (unit, channel) map entries
    long long lag_rs_mfma = 0;    // MFMA instructions of one channel group's units
    std::vector<int> tc_shift_host;  // host copy of tc_shift
    double shift_eps = 0.0;   // synthesised / lag searches: relative score error of rounding the
                              // time centres to integer samples
    double trunc_tail = 0.0;  // largest sqrt(envelope tail energy) outside the supports
    double rho_max = 0.0;     // max over atoms of |envelope|_2 / |g|_2
    double eg_max = 0.0;      // max over atoms of |fl(g_hat) - g_hat|_2 (table rounding)

    // per-channel workspace [max_batch]
    void* shadow = nullptr;   // [B][sh_stride] fp32 / bf16 / fp16 copy of the residual (row 0)
    void* shadow_alloc = nullptr;  // its allocation (lag-table plans: one zero guard row first)
    int sh_stride = 0;        // shadow row stride in elements: n_pad; lag-table plans 2 n_pad, the
                              // n_pad elements after each row zero, so window reads need no bounds
    unsigned* cand_idx = nullptr;   // [B][cap]
    float* cand_score = nullptr;    // [B][cap] search score
    double* cand_p64 = nullptr;     // [B][cap] FP64 rescore
    int* cand_count = nullptr;      // [B]
    unsigned* gmax = nullptr;       // [B] bits of max |score|
    double* ebound = nullptr;       // [B] certified score error bound
    double* rnorm = nullptr;        // [B] |r|
    int* need_rerun = nullptr;      // [B] candidate overflow -> exact-threshold search
    unsigned long long* exec_count = nullptr;  // [2] MFMA searches: executed MFMA instructions of the
                                               // pass-0 searches and their launches (act_search_executed)
    size_t workspace_bytes = 0;

    const double* search_resid = nullptr;  // FP64 residual the FP64 search reads
    const int* call_len = nullptr;          // ragged: lengths / offsets of the current call
    const long long* call_off = nullptr;
    double* lag_energy = nullptr;           // ragged synthesised: [n_fc][n_cl][fac_w] prefix sums of g^2
    int* items = nullptr;                   // ragged synthesised: [B + 1] item prefix, [B] order, counters
    int n_items_max = 0;
    int chain = 0;                          // FP32 score FMA-chain length (certified margin)

    hipStream_t last_stream = nullptr;

    // search launch shapes chosen by act_tune, per batch size; `shape` is the
    // one the launchers use (zeros: built-in defaults)
    std::vector<std::pair<int, act_launch_shape>> shapes;
    act_launch_shape shape{};

    // captured act_decompose sequences, keyed by every argument (small LRU)
    struct GraphEntry {
        std::vector<uintptr_t> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        unsigned long long last_use = 0;
    };
    std::vector<GraphEntry> graphs;
    unsigned long long graph_clock = 0;
    hipStream_t cap_stream = nullptr;
    bool use_graphs = true;

    // phase timing (act_timing_enable): event pairs recorded per launch
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    std::vector<int> ev_phase;
    size_t ev_used = 0;
};

namespace act {
// launch shapes (act_tune.hip): select the tuned shape of a batch size, and the
// persistent grid of a search kernel (workgroups per CU, default `def`)
void select_shape(act_plan_s* p, int batch);
long long grid_cap(const act_plan_s* p, int def);
int device_cus();
int device_lds_per_block();   // bytes of LDS one workgroup may hold
// search launchers (act_search.hip)
act_status launch_search(act_plan_s* p, int batch, int pass, hipStream_t s);
act_status launch_correlate(act_plan_s* p, int batch, const double* resid, long long begin,
                            long long count, double* out, hipStream_t s);
// plan-time builders (act_plan.hip)
act_status build_tables(act_plan_s* p, hipStream_t s);
act_status write_bf16_table(act_plan_s* p, hipStream_t s);
act_status build_synth(act_plan_s* p, hipStream_t s);
act_status launch_ragged_items(act_plan_s* p, int batch, hipStream_t s);
act_status build_h16_factors(act_plan_s* p, hipStream_t s);
act_status build_supports(act_plan_s* p, hipStream_t s);
act_status launch_h16_ragged_prep(act_plan_s* p, int batch, hipStream_t s);
act_status launch_lag_ragged_prep(act_plan_s* p, int batch, hipStream_t s);
act_status launch_prior_init(act_plan_s* p, int batch, const double* resid, hipStream_t s);
act_status launch_prior_order(act_plan_s* p, int batch, int k, int order, double* resid, double* approx,
                              double* theta, double* coef, long long* index, double* energy, double* gap,
                              int* flags, hipStream_t s);
size_t prior_workspace_blocks();
// LEM workspace per channel: cap candidates x (4 parameters + 1 score, FP64)
// and one mark byte, at cand_ws [B][cap][4], score_ws [B][cap], used_ws [B][cap]
act_status launch_lem_order(act_plan_s* p, const act_lem_desc* cfg, int cap, double* cand_ws, double* score_ws,
                            char* used_ws, int batch, int k, int order, const double* lhs, double* resid,
                            double* approx, double* theta, double* coef, double* energy, int* flags,
                            hipStream_t s);
// per-channel kernels (act_refine.hip)
act_status launch_init(act_plan_s* p, int batch, double* resid, double* approx, double* energy,
                       int* flags, int order, hipStream_t s);
act_status launch_rescore(act_plan_s* p, int batch, const double* resid, hipStream_t s);
act_status launch_select_refine_update(act_plan_s* p, int batch, int k, int order, double* resid,
                                       double* approx, double* theta, double* coef,
                                       long long* index, double* energy, double* gap, int* flags,
                                       hipStream_t s);
act_status launch_overflow_check(act_plan_s* p, int batch, hipStream_t s);
// True when a search of `batch` channels lists exactly the certified set in its
// second pass (the lag table's resident form): no overflow check or rerun
// applies to it.
bool search_emits_certified_set(const act_plan_s* p, int batch);
act_status launch_refine_many(act_plan_s* p, int m, const double* resid, const double* theta0,
                              int steps, double* theta, double* value, int* flags, hipStream_t s);
act_status launch_refine_many_f32(act_plan_s* p, int m, const float* resid, const double* theta0, int steps,
                                  double* theta, double* value, int* flags, hipStream_t s);
act_status launch_value_and_grad(act_plan_s* p, int m, int dtype, const void* resid,
                                 const double* theta, double* value, double* dtheta, void* dr,
                                 hipStream_t s);
act_status launch_to_shadow(act_plan_s* p, int batch, const double* resid, hipStream_t s);
int f32_chain_length(int n_pad);
int synth_chain_length(int n_pad);
int h16_chain_length(int n_pad);
int lag_chain_length(int n_pad);
act_status build_lag_table(act_plan_s* p, hipStream_t s);
double lag_search_flops(const act_plan_s* p, int batch);
struct SearchCtl;
act_status launch_search_lag(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s);
act_status launch_reconstruct(act_plan_s* p, int batch, int order, const double* theta,
                              const double* coef, const int* len, const long long* off, double* out,
                              hipStream_t s);
}  // namespace act
