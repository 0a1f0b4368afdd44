// act_plan.hip -- plan construction: grid validation, axis values, the HBM
// dictionary table (FP64 synthesis -> unit norm -> FP32 / BF16 rows), and the
// per-channel workspace.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "act_common.h"

namespace act {

// Axis value j: lo + j*((hi-lo)/d); d = count (half-open) or count-1 (closed,
// last value hi exactly); a one-value axis is lo.  No contraction, so the
// values are the IEEE results of exactly these operations.
#pragma clang fp contract(off)
static double axis_value(const act_axis& a, int j) {
    if (a.count <= 1) return a.lo;
    int d = a.half_open ? a.count : a.count - 1;
    if (!a.half_open && j == a.count - 1) return a.hi;
    double step = (a.hi - a.lo) / (double)d;
    return a.lo + (double)j * step;
}

static double axis_step(const act_axis& a) {
    if (a.count <= 1) return 1.0;
    int d = a.half_open ? a.count : a.count - 1;
    return (a.hi - a.lo) / (double)d;
}
#pragma clang fp contract(on)

__device__ __forceinline__ float d_bf16_to_f32(unsigned short h) {
    return __uint_as_float(((unsigned)h) << 16);
}

// One wave per atom: FP64 synthesis of Eq. (1) over the n samples present,
// unit l2 normalisation (Sec. III-A), the FP64 inverse norm, rounding to the
// table type (RNE; FP32 rows are written here, BF16 tiles by the swizzled
// writer), and the exact l2 norm of the rounding error, whose maximum over the
// dictionary enters the certified margin of the search.
template <typename TOut, bool WRITE>
__global__ void __launch_bounds__(256) k_build_table(GridDev g, TOut* __restrict__ table,
                                                     double* __restrict__ inv_norm,
                                                     unsigned long long* __restrict__ eg_bits) {
    const int lane = threadIdx.x & (kWave - 1);
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const long long nwaves = (long long)gridDim.x * blockDim.x / kWave;
    for (long long i = wave; i < g.atoms; i += nwaves) {
        double th[4];
        grid_theta(g, i, th);
        const double inv_dt = 1.0 / exp(th[3]);
        double q = 0.0;
        for (int k = lane; k < g.n; k += kWave) {
            double v = atom_sample64(sample_time(k, g.fs), th[0], th[1], th[2], inv_dt);
            q += v * v;
        }
        q = wave_sum(q);
        const double nrm = sqrt(q);
        const double sc = nrm >= 1e-300 ? 1.0 / nrm : 0.0;
        if (lane == 0) inv_norm[i] = sc;
        double e2 = 0.0;
        TOut* row = table + (size_t)i * g.n_pad;
        for (int k = lane; k < g.n_pad; k += kWave) {
            double v = 0.0;
            if (k < g.n) v = atom_sample64(sample_time(k, g.fs), th[0], th[1], th[2], inv_dt) * sc;
            float f = (float)v;
            double back;
            if constexpr (sizeof(TOut) == 4) {
                if (WRITE) row[k] = f;
                back = (double)f;
            } else {
                unsigned short h = bf16_rne(f);
                if (WRITE) row[k] = h;
                back = (double)d_bf16_to_f32(h);
            }
            double d = back - v;
            e2 += d * d;
        }
        e2 = wave_sum(e2);
        if (lane == 0) atomicMax(eg_bits, (unsigned long long)__double_as_longlong(sqrt(e2)));
    }
}

// Shift-invariant factor tables of the synthesised dictionary, FP64-evaluated
// and rounded to FP32 (RNE): for column e the lag is d = e - n_pad, tau = d/fs,
//   U_cl = E cos(2 pi c tau^2), V_cl = E sin(2 pi c tau^2), E = exp(-(tau/dt)^2/2),
//   C_fc = cos(2 pi f_c tau),   S_fc = sin(2 pi f_c tau).
__global__ void k_build_factors(GridDev g, int W, float* __restrict__ U, float* __restrict__ V,
                                float* __restrict__ C, float* __restrict__ S) {
    const int n_cl = g.cnt[2] * g.cnt[3], n_fc = g.cnt[1];
    const long long total = (long long)(n_cl + n_fc) * W;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int row = (int)(q / W), e = (int)(q % W);
        const double tau = (double)(e - g.n_pad) / g.fs;
        if (row < n_cl) {
            const int ic = row / g.cnt[3], il = row % g.cnt[3];
            const double c = g.axis[g.off[2] + ic];
            const double u = tau / exp(g.axis[g.off[3] + il]);
            const double env = exp(-0.5 * u * u);
            double si, co;
            sincospi(2.0 * (c * tau * tau), &si, &co);
            U[(size_t)row * W + e] = (float)(env * co);
            V[(size_t)row * W + e] = (float)(env * si);
        } else {
            const int fc = row - n_cl;
            double si, co;
            sincospi(2.0 * (g.axis[g.off[1] + fc] * tau), &si, &co);
            C[(size_t)fc * W + e] = (float)co;
            S[(size_t)fc * W + e] = (float)si;
        }
    }
}

// One wave per atom: FP64 norms of the atom and of its Gaussian envelope over
// the samples present; writes 1/|g| (FP64 and FP32) and the largest ratio
// |envelope| / |g| of the dictionary (it scales the synthesis error bound).
// Complex atoms E exp(i phi) have |g| = |E|: ratio 1.
__global__ void __launch_bounds__(256) k_norms_rho(GridDev g, double* __restrict__ inv_norm,
                                                   float* __restrict__ inv_norm32,
                                                   unsigned long long* __restrict__ rho_bits, int cplx) {
    const int lane = threadIdx.x & (kWave - 1);
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const long long nwaves = (long long)gridDim.x * blockDim.x / kWave;
    for (long long i = wave; i < g.atoms; i += nwaves) {
        double th[4];
        grid_theta(g, i, th);
        const double inv_dt = 1.0 / exp(th[3]);
        double q = 0.0, qe = 0.0;
        for (int k = lane; k < g.n; k += kWave) {
            const double tau = sample_time(k, g.fs) - th[0];
            const double u = tau * inv_dt;
            const double e = exp(-0.5 * u * u);
            const double v = e * cospi(2.0 * (th[2] * tau * tau + th[1] * tau));
            q += v * v;
            qe += e * e;
        }
        q = wave_sum(q);
        qe = wave_sum(qe);
        if (cplx) q = qe;
        const double nrm = sqrt(q);
        const double sc = nrm >= 1e-300 ? 1.0 / nrm : 0.0;
        if (lane == 0) {
            inv_norm[i] = sc;
            inv_norm32[i] = (float)sc;
            if (nrm >= 1e-300) atomicMax(rho_bits, (unsigned long long)__double_as_longlong(sqrt(qe) / nrm));
        }
    }
}

// Ragged synthesised plans: for every (f_c, cl) the inclusive prefix sums
// over lags d = e - n_pad of the squared atom, q[e] = sum_{e' <= e} g(d')^2,
// in FP64 and in a fixed order (each thread a contiguous run, then the runs'
// totals scanned by one thread).  The norm of the atom with time centre m on a
// channel of n samples is then q[n-1-m+n_pad] - q[-m+n_pad-1].
// Error-bound ratio: the synthesised score's rounding error scales with
// |E_w| / |g_w| over the channel's window w of lags.  Every time centre sits at
// least div samples before the channel's end, so w contains the lags 0..div-1
// and |g_w|^2 >= sum_{d<div} g(d)^2, while |E_w|^2 <= the envelope's energy
// over all lags: the ratio of the two bounds every window that occurs.
__global__ void __launch_bounds__(256) k_lag_energy(GridDev g, int n_cl, int W, int div,
                                                    double* __restrict__ q,
                                                    unsigned long long* __restrict__ rho_bits) {
    __shared__ double tot[256];
    __shared__ double tot_e[256];
    __shared__ double tot_h[256];
    const long long rows = (long long)g.cnt[1] * n_cl;
    const int per = (W + 255) / 256;
    for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
        const int fc = (int)(row / n_cl), cl = (int)(row % n_cl);
        const int ic = cl / g.cnt[3], il = cl % g.cnt[3];
        const double f = g.axis[g.off[1] + fc], c = g.axis[g.off[2] + ic];
        const double inv_dt = 1.0 / exp(g.axis[g.off[3] + il]);
        double* qr = q + (size_t)row * W;
        const int e0 = threadIdx.x * per, e1 = min(W, e0 + per);
        double acc = 0.0, acc_e = 0.0, acc_h = 0.0;
        for (int e = e0; e < e1; ++e) {
            const double tau = (double)(e - g.n_pad) / g.fs;
            const double u = tau * inv_dt;
            const double env = exp(-0.5 * u * u);
            const double v = env * cospi(2.0 * (c * tau * tau + f * tau));
            acc += v * v;
            acc_e += env * env;
            if (e >= g.n_pad && e < g.n_pad + div) acc_h += v * v;
            qr[e] = acc;
        }
        tot[threadIdx.x] = acc;
        tot_e[threadIdx.x] = acc_e;
        tot_h[threadIdx.x] = acc_h;
        __syncthreads();
        if (threadIdx.x == 0) {
            double run = 0.0, run_e = 0.0, head = 0.0;
            for (int t = 0; t < 256; ++t) {
                const double x = tot[t];
                tot[t] = run;
                run += x;
                run_e += tot_e[t];
                head += tot_h[t];
            }
            if (head > 0.0) atomicMax(rho_bits, (unsigned long long)__double_as_longlong(sqrt(run_e / head)));
        }
        __syncthreads();
        const double base = tot[threadIdx.x];
        for (int e = e0; e < e1; ++e) qr[e] += base;
        __syncthreads();
    }
}

// 1/|g| over every lag of the table, per (f_c, cl) row: the norm of an atom
// whose support lies inside its signal.
__global__ void k_inv_full(const double* __restrict__ q, long long rows, int W, float* __restrict__ inv) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < rows) {
        const double e2 = q[(size_t)r * W + (W - 1)];
        inv[r] = e2 > 0.0 ? (float)(1.0 / sqrt(e2)) : 0.0f;
    }
}

act_status build_synth(act_plan_s* p, hipStream_t s) {
    unsigned long long* rb = nullptr;
    ACT_HIP(hipMalloc((void**)&rb, sizeof(unsigned long long)));
    ACT_HIP(hipMemsetAsync(rb, 0, sizeof(unsigned long long), s));
    int dev = 0, cus = 0;
    ACT_HIP(hipGetDevice(&dev));
    ACT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const long long total = (long long)(p->n_cl + p->grid.cnt[1]) * p->fac_w;
    hipLaunchKernelGGL(k_build_factors, dim3((unsigned)std::min<long long>((total + 255) / 256, cus * 64LL)),
                       dim3(256), 0, s, p->grid, p->fac_w, (float*)p->fac_u, (float*)p->fac_v,
                       (float*)p->fac_c, (float*)p->fac_s);
    ACT_HIP(hipGetLastError());
    if (p->desc.ragged) {
        const long long rows = (long long)p->grid.cnt[1] * p->n_cl;
        hipLaunchKernelGGL(k_lag_energy, dim3((unsigned)std::min<long long>(rows, cus * 16LL)), dim3(256), 0, s,
                           p->grid, p->n_cl, p->fac_w, p->desc.ragged_tc_div, p->lag_energy, rb);
        if (p->inv_full32)
            hipLaunchKernelGGL(k_inv_full, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, p->lag_energy, rows,
                               p->fac_w, p->inv_full32);
    } else {
        hipLaunchKernelGGL(k_norms_rho, dim3((unsigned)std::min<long long>((p->atoms + 3) / 4, cus * 32LL)),
                           dim3(256), 0, s, p->grid, p->inv_norm, p->inv_norm32, rb, p->desc.complex_atoms);
    }
    ACT_HIP(hipGetLastError());
    unsigned long long bits = 0;
    ACT_HIP(hipMemcpyAsync(&bits, rb, sizeof bits, hipMemcpyDeviceToHost, s));
    ACT_HIP(hipStreamSynchronize(s));
    ACT_HIP(hipFree(rb));
    double v;
    memcpy(&v, &bits, sizeof v);
    p->rho_max = v;
    return ACT_OK;
}

// Lag-table plans: FP64 norms of every atom (FP32 copies for the search) and
// the FP16 lag table.
act_status build_lag(act_plan_s* p, hipStream_t s) {
    unsigned long long* rb = nullptr;
    ACT_HIP(hipMalloc((void**)&rb, sizeof(unsigned long long)));
    ACT_HIP(hipMemsetAsync(rb, 0, sizeof(unsigned long long), s));
    const int cus = device_cus();
    hipLaunchKernelGGL(k_norms_rho, dim3((unsigned)std::min<long long>((p->atoms + 3) / 4, cus * 32LL)), dim3(256),
                       0, s, p->grid, p->inv_norm, p->inv_norm32, rb, p->desc.complex_atoms);
    ACT_HIP(hipGetLastError());
    act_status st = build_lag_table(p, s);
    ACT_HIP(hipStreamSynchronize(s));
    ACT_HIP(hipFree(rb));
    return st;
}

// Half-supports of the FP16 search's envelopes: for each log-duration the
// smallest D (in samples) whose envelope tail energy over lags |d| > D (inside
// the table's lag range) is at most 2^-48, from the FP64 prefix sums.  They
// mark the atoms whose support lies inside their signal (full-window norm),
// and with support_cut the samples each block of atoms may skip (the tail then
// enters the certified bound).
act_status build_supports(act_plan_s* p, hipStream_t s) {
    const int n_ld = p->grid.cnt[3], W = p->fac_w, np = p->n_pad;
    std::vector<int> half(n_ld, np);
    double tail_max = 0.0;
    {
        std::vector<double> q((size_t)n_ld * W);
        ACT_HIP(hipMemcpyAsync(q.data(), p->env_q, q.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        ACT_HIP(hipStreamSynchronize(s));
        const double lim = 3.552713678800501e-15;  // 2^-48
        for (int il = 0; il < n_ld; ++il) {
            const double* qr = q.data() + (size_t)il * W;
            const double total = qr[W - 1];
            int D = np;
            double t_at = 0.0;
            for (int d = 0; d < np; ++d) {
                // lags <= -(d+1): columns [0, np-d-1); lags >= d+1: columns [np+d+1, W)
                const double left = np - d - 1 >= 0 ? qr[np - d - 1] : 0.0;
                const double right = total - qr[np + d];
                const double tail = left + right;
                if (tail <= lim) {
                    D = d;
                    t_at = tail > 0.0 ? tail : 0.0;
                    break;
                }
            }
            half[il] = D;
            tail_max = std::max(tail_max, std::sqrt(t_at) * (1.0 + 1e-9));
        }
    }
    ACT_HIP(hipMemcpyAsync(p->ld_half, half.data(), half.size() * sizeof(int), hipMemcpyHostToDevice, s));
    ACT_HIP(hipStreamSynchronize(s));
    p->trunc_tail = p->desc.support_cut ? tail_max : 0.0;
    return ACT_OK;
}

static act_status validate_axis(const act_axis& a, const char* name) {
    std::string n(name);
    ACT_REQUIRE(a.count >= 1, n + ": count must be >= 1");
    ACT_REQUIRE(std::isfinite(a.lo) && std::isfinite(a.hi), n + ": bounds must be finite");
    ACT_REQUIRE(a.count == 1 || a.hi >= a.lo, n + ": hi < lo");
    return ACT_OK;
}

act_status build_tables(act_plan_s* p, hipStream_t s) {
    if (p->desc.dict != ACT_DICT_TABLE) return ACT_OK;
    unsigned long long* eg = nullptr;
    ACT_HIP(hipMalloc((void**)&eg, sizeof(unsigned long long)));
    ACT_HIP(hipMemsetAsync(eg, 0, sizeof(unsigned long long), s));
    int dev = 0, cus = 0;
    ACT_HIP(hipGetDevice(&dev));
    ACT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    long long waves_needed = p->atoms;
    int blocks = (int)std::min<long long>((waves_needed + 3) / 4, (long long)cus * 32);
    if (p->desc.prec == ACT_PREC_F32) {
        hipLaunchKernelGGL((k_build_table<float, true>), dim3(blocks), dim3(256), 0, s, p->grid,
                           (float*)p->table, p->inv_norm, eg);
        ACT_HIP(hipGetLastError());
    } else {
        hipLaunchKernelGGL((k_build_table<unsigned short, false>), dim3(blocks), dim3(256), 0, s, p->grid,
                           (unsigned short*)nullptr, p->inv_norm, eg);
        ACT_HIP(hipGetLastError());
        act_status st = write_bf16_table(p, s);
        if (st != ACT_OK) return st;
    }
    unsigned long long bits = 0;
    ACT_HIP(hipMemcpyAsync(&bits, eg, sizeof bits, hipMemcpyDeviceToHost, s));
    ACT_HIP(hipStreamSynchronize(s));
    ACT_HIP(hipFree(eg));
    double v;
    memcpy(&v, &bits, sizeof v);
    p->eg_max = v;
    return ACT_OK;
}

static void free_plan(act_plan_s* p) {
    if (!p) return;
    if (p->last_stream) (void)hipStreamSynchronize(p->last_stream);
    void* ptrs[] = {p->axis_dev, p->inv_norm, p->table, p->fac_u, p->fac_v, p->fac_c, p->fac_s,
                    p->inv_norm32, p->tc_shift, p->lag_energy, p->items, p->fac_u16, p->fac_v16, p->fac_c16, p->fac_s16, p->env_q, p->rscale, p->ebmul, p->perm, p->tmax, p->ld_half, p->inv_full32, p->prior_s, p->prior_part, p->prior_pidx, p->lem_cand, p->lem_score, p->shadow_alloc, p->cand_idx, p->cand_score, p->cand_p64, p->exec_count,
                    p->cand_count, p->gmax, p->ebound, p->rnorm, p->need_rerun, p->lag_inv, p->lag_span, p->lag_order,
                    p->lag_rho, p->lag_rows, p->lag_rs_cp, p->lag_rs_count, p->lag_rs_units, p->lag_rs_map, p->lag_rs_pairs};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (auto& ge : p->graphs) {
        if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
        if (ge.graph) (void)hipGraphDestroy(ge.graph);
    }
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    for (auto& ev : p->ev_pool) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    delete p;
}

}  // namespace act

using namespace act;

extern "C" act_status act_plan(const act_plan_desc* desc, void* stream, act_plan_t* out) {
    ACT_REQUIRE(desc != nullptr && out != nullptr, "act_plan: desc and out must not be NULL");
    *out = nullptr;
    const act_grid& gr = desc->grid;
    ACT_REQUIRE(std::isfinite(gr.fs_hz) && gr.fs_hz > 0, "act_plan: fs_hz must be > 0");
    ACT_REQUIRE(gr.n_samples >= 1, "act_plan: n_samples must be >= 1");
    act_status st;
    if ((st = validate_axis(gr.tc_s, "tc_s")) != ACT_OK) return st;
    if ((st = validate_axis(gr.fc_hz, "fc_hz")) != ACT_OK) return st;
    if ((st = validate_axis(gr.c_hz_per_s, "c_hz_per_s")) != ACT_OK) return st;
    if ((st = validate_axis(gr.logdt_ln_s, "logdt_ln_s")) != ACT_OK) return st;
    ACT_REQUIRE(desc->dict == ACT_DICT_SYNTH || desc->dict == ACT_DICT_TABLE || desc->dict == ACT_DICT_LAG,
                "act_plan: unknown dict");
    ACT_REQUIRE(desc->prec == ACT_PREC_F64 || desc->prec == ACT_PREC_F32 || desc->prec == ACT_PREC_BF16 ||
                    desc->prec == ACT_PREC_F16,
                "act_plan: unknown prec");
    ACT_REQUIRE(!(desc->prec == ACT_PREC_F16 && desc->dict == ACT_DICT_TABLE),
                "act_plan: ACT_PREC_F16 is the synthesised factor-table search; use ACT_DICT_SYNTH");
    ACT_REQUIRE(desc->support_cut == 0 || desc->support_cut == 1, "act_plan: support_cut must be 0 or 1");
    ACT_REQUIRE(desc->prior_act == 0 || desc->prior_act == 1, "act_plan: prior_act must be 0 or 1");
    if (desc->prior_act && !(desc->dict == ACT_DICT_SYNTH && desc->prec == ACT_PREC_F64 && !desc->ragged)) {
        set_error("act_plan: prior_act needs a plain ACT_DICT_SYNTH + ACT_PREC_F64 plan");
        return ACT_ERR_UNSUPPORTED;
    }
    if (desc->support_cut && !(desc->prec == ACT_PREC_F16 && desc->dict == ACT_DICT_SYNTH)) {
        set_error("act_plan: support_cut applies to the FP16 synthesised search only");
        return ACT_ERR_UNSUPPORTED;
    }
    ACT_REQUIRE(desc->complex_atoms == 0 || desc->complex_atoms == 1, "act_plan: complex_atoms must be 0 or 1");
    if (desc->complex_atoms &&
        !(((desc->dict == ACT_DICT_SYNTH && (desc->prec == ACT_PREC_F64 || desc->prec == ACT_PREC_F32)) ||
           (desc->dict == ACT_DICT_LAG && desc->prec == ACT_PREC_F16)) &&
          !desc->ragged && !desc->prior_act && !desc->support_cut)) {
        set_error("act_plan: complex_atoms needs a plain ACT_DICT_SYNTH plan with ACT_PREC_F64 or ACT_PREC_F32, "
                  "or an ACT_DICT_LAG plan");
        return ACT_ERR_UNSUPPORTED;
    }
    ACT_REQUIRE(!(desc->prec == ACT_PREC_F64 && desc->dict == ACT_DICT_TABLE),
                "act_plan: ACT_PREC_F64 searches synthesise atoms; use ACT_DICT_SYNTH");
    ACT_REQUIRE(desc->max_batch >= 1, "act_plan: max_batch must be >= 1");
    ACT_REQUIRE(desc->cand_cap >= 0 && desc->refine_steps >= 0, "act_plan: negative cand_cap/refine_steps");
    if (desc->ragged) {
        ACT_REQUIRE(desc->ragged_tc_div >= 1, "act_plan: ragged plans need ragged_tc_div >= 1");
        if (!((desc->dict == ACT_DICT_SYNTH && desc->prec != ACT_PREC_BF16) ||
              (desc->dict == ACT_DICT_LAG && desc->prec == ACT_PREC_F16))) {
            set_error("act_plan: ragged plans support the synthesised FP64, FP32 and FP16 searches and the lag table");
            return ACT_ERR_UNSUPPORTED;
        }
        if (desc->dict == ACT_DICT_SYNTH && desc->prec != ACT_PREC_F64 && desc->ragged_tc_div % 16 != 0) {
            set_error("act_plan: the ragged MFMA synthesised searches need ragged_tc_div a multiple of 16");
            return ACT_ERR_UNSUPPORTED;
        }
        if (desc->dict == ACT_DICT_LAG && desc->ragged_tc_div % 8 != 0) {
            set_error("act_plan: the ragged lag-table search needs ragged_tc_div a multiple of 8");
            return ACT_ERR_UNSUPPORTED;
        }
    }
    if (desc->dict == ACT_DICT_LAG &&
        !(((desc->prec == ACT_PREC_F16 && !(desc->ragged && desc->complex_atoms)) ||
           (desc->prec == ACT_PREC_BF16 && !desc->ragged && !desc->complex_atoms)) &&
          !desc->prior_act && !desc->support_cut)) {
        set_error("act_plan: ACT_DICT_LAG is the FP16 lag-table search (complex atoms on plain plans only) "
                  "or its BF16 form (plain plans of real atoms)");
        return ACT_ERR_UNSUPPORTED;
    }
    if (desc->dict == ACT_DICT_SYNTH && desc->prec == ACT_PREC_BF16) {
        set_error("act_plan: this precision / dictionary pair is not implemented in this build");
        return ACT_ERR_UNSUPPORTED;
    }

    act_plan_s* p = new act_plan_s();
    p->desc = *desc;
    hipStream_t s = (hipStream_t)stream;
    p->n = gr.n_samples;
    p->n_pad = (gr.n_samples + 255) / 256 * 256;
    p->max_batch = desc->max_batch;
    {
        const char* ng = getenv("ACT_NO_GRAPH");
        p->use_graphs = !(ng && ng[0] == '1');
    }
    // longest FP32 accumulation chain of one search score (certified margin):
    // the FP32 GEMV's per-lane FMAs plus its reduction tree; the MFMA path is
    // bounded by one rounding per sample
    p->chain = desc->dict == ACT_DICT_LAG     ? lag_chain_length(p->n_pad)
               : desc->prec == ACT_PREC_BF16 ? p->n_pad
               : desc->prec == ACT_PREC_F16 ? h16_chain_length(p->n_pad)
               : desc->dict == ACT_DICT_SYNTH ? synth_chain_length(p->n_pad)
                                              : f32_chain_length(p->n_pad);
    // ragged batches hold long, densely sampled signals: a strong chirplet has
    // many grid neighbours inside the certified margin, and rescoring them
    // costs far less than a rerun of the search
    // (the ragged lag table's rows near a signal's end emit by a widened bound:
    // a longer list, 8 MiB per channel, spares the exact-threshold reruns, as
    // 2 MiB do for the ragged synthesis and its per-atom bounds; the
    // BF16 searches' margin (unit roundoff 2^-8) is 8x FP16's, and the FP16
    // synthesis' support cut widens its per-atom bounds)
    p->cap = desc->cand_cap > 0 ? desc->cand_cap
             : desc->ragged     ? (desc->dict == ACT_DICT_LAG ? 524288 : 131072)
             : (desc->prec == ACT_PREC_BF16 || (desc->prec == ACT_PREC_F16 && desc->dict == ACT_DICT_SYNTH))
                 ? 16384
                 : 4096;
    const act_axis* ax[4] = {&gr.tc_s, &gr.fc_hz, &gr.c_hz_per_s, &gr.logdt_ln_s};
    long long atoms = 1;
    int total = 0;
    for (int a = 0; a < 4; ++a) {
        atoms *= ax[a]->count;
        p->grid.cnt[a] = ax[a]->count;
        p->grid.off[a] = total;
        total += ax[a]->count;
        p->box.step[a] = axis_step(*ax[a]);
        p->box.lo[a] = axis_value(*ax[a], 0);
        p->box.hi[a] = axis_value(*ax[a], ax[a]->count - 1);
    }
    if (atoms >= (1LL << 32)) {
        free_plan(p);
        set_error("act_plan: more than 2^32 atoms");
        return ACT_ERR_INVALID;
    }
    p->atoms = atoms;
    std::vector<double> vals(total);
    for (int a = 0; a < 4; ++a)
        for (int j = 0; j < ax[a]->count; ++j) vals[p->grid.off[a] + j] = axis_value(*ax[a], j);

    auto fail = [&](act_status code) {
        free_plan(p);
        return code;
    };
#define PLAN_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));                \
            return fail(e_ == hipErrorOutOfMemory ? ACT_ERR_NOMEM : ACT_ERR_HIP);        \
        }                                                                                \
    } while (0)

    PLAN_HIP(hipMalloc((void**)&p->axis_dev, sizeof(double) * total));
    PLAN_HIP(hipMemcpyAsync(p->axis_dev, vals.data(), sizeof(double) * total, hipMemcpyHostToDevice, s));
    p->grid.fs = gr.fs_hz;
    p->grid.axis = p->axis_dev;
    p->grid.n = p->n;
    p->grid.n_pad = p->n_pad;
    p->grid.atoms = atoms;
    if (desc->ragged) {
        // a ragged channel has floor(len/div) time centres; the plan grid is the
        // widest channel's (n_samples long), used for sizing only
        p->grid.ragged_div = desc->ragged_tc_div;
        p->grid.cnt[0] = std::max(1, gr.n_samples / desc->ragged_tc_div);
        p->grid.atoms = (long long)p->grid.cnt[0] * p->grid.cnt[1] * p->grid.cnt[2] * p->grid.cnt[3];
        p->atoms = p->grid.atoms;
        // the widest channel's time-centre spacing, as a channel of that length computes it
        const int ntc = p->grid.cnt[0];
        p->grid.tc_step = ((double)(ntc * desc->ragged_tc_div) / gr.fs_hz) / (double)ntc;
    }

    const size_t B = (size_t)p->max_batch, cap = (size_t)p->cap;
    const size_t elt = (desc->prec == ACT_PREC_BF16 || desc->prec == ACT_PREC_F16) ? 2 : 4;
    p->atoms_pad = desc->prec == ACT_PREC_BF16 ? (atoms + 511) / 512 * 512 : atoms;
    if (desc->dict == ACT_DICT_TABLE) {
        p->table_bytes = (size_t)p->atoms_pad * p->n_pad * elt;
        size_t free_b = 0, total_b = 0;
        PLAN_HIP(hipMemGetInfo(&free_b, &total_b));
        if (p->table_bytes + (64ull << 20) > free_b) {
            set_error("act_plan: dictionary table of " + std::to_string(p->table_bytes) +
                      " bytes does not fit in free device memory");
            return fail(ACT_ERR_NOMEM);
        }
        PLAN_HIP(hipMalloc(&p->table, p->table_bytes));
        PLAN_HIP(hipMalloc((void**)&p->inv_norm, (size_t)atoms * sizeof(double)));
    }
    // MFMA synthesised searches (FP32, FP16) share the FP32 factor tables
    const bool synth32 = desc->dict == ACT_DICT_SYNTH && (desc->prec == ACT_PREC_F32 || desc->prec == ACT_PREC_F16);
    if (synth32 && desc->ragged) {
        p->n_cl = ax[2]->count * ax[3]->count;
        p->fac_w = 2 * p->n_pad;
        const size_t ucl = (size_t)p->n_cl * p->fac_w * sizeof(float);
        const size_t ufc = (size_t)ax[1]->count * p->fac_w * sizeof(float);
        const size_t qb = (size_t)ax[1]->count * p->n_cl * p->fac_w * sizeof(double);
        size_t free_b = 0, total_b = 0;
        PLAN_HIP(hipMemGetInfo(&free_b, &total_b));
        if (qb + 2 * ucl + 2 * ufc + (64ull << 20) > free_b) {
            set_error("act_plan: the lag-energy table of " + std::to_string(qb) + " bytes does not fit");
            return fail(ACT_ERR_NOMEM);
        }
        PLAN_HIP(hipMalloc(&p->fac_u, ucl));
        PLAN_HIP(hipMalloc(&p->fac_v, ucl));
        PLAN_HIP(hipMalloc(&p->fac_c, ufc));
        PLAN_HIP(hipMalloc(&p->fac_s, ufc));
        PLAN_HIP(hipMalloc((void**)&p->lag_energy, qb));
        // tile prefix [B + 1], pass-0 / pass-1 queue counters, any-rerun flag
        PLAN_HIP(hipMalloc((void**)&p->items, ((size_t)p->max_batch + 4) * sizeof(int)));
        p->table_bytes = 0;
        const long long tiles = (long long)p->max_batch * (gr.n_samples / desc->ragged_tc_div) *
                                ((p->n_cl + 127) / 128) * ((ax[1]->count + 63) / 64);
        if (tiles > 0x7fffffffLL) {
            set_error("act_plan: a ragged batch of max_batch signals has more than 2^31 search tiles");
            return fail(ACT_ERR_UNSUPPORTED);
        }
    } else if (synth32 || desc->dict == ACT_DICT_LAG) {
        // time centres must sit on integer samples (multiples of 16 for the
        // synthesised searches, of 8 for the lag table) inside the signal; the
        // residual distance to the integer enters the certified bound
        const int mult = desc->dict == ACT_DICT_LAG ? 8 : 16;
        const int n_tc = p->grid.cnt[0];
        std::vector<int> shift(n_tc);
        double delta = 0.0;
        for (int j = 0; j < n_tc && desc->ragged; ++j) {
            // ragged (lag table): centre j of a channel with ntc centres sits at
            // j ((ntc div / fs) / ntc) s; its sample is j div, at most delta away
            shift[j] = j * desc->ragged_tc_div;
            for (int ntc = j + 1; ntc <= n_tc; ++ntc) {
                const double step = ((double)(ntc * desc->ragged_tc_div) / gr.fs_hz) / (double)ntc;
                delta = std::max(delta, std::fabs((double)j * step * gr.fs_hz - (double)shift[j]));
            }
        }
        for (int j = 0; j < n_tc && !desc->ragged; ++j) {
            const double mv = vals[p->grid.off[0] + j] * gr.fs_hz;
            const double mr = std::nearbyint(mv);
            if (!(std::fabs(mv - mr) <= 1e-6 * std::max(1.0, std::fabs(mv))) || mr < 0 ||
                mr >= gr.n_samples || ((long long)mr % mult) != 0) {
                set_error(std::string("act_plan: the MFMA synthesised and lag-table searches need time centres "
                                      "on integer sample offsets that are multiples of ") +
                          std::to_string(mult) + " inside the signal");
                return fail(ACT_ERR_UNSUPPORTED);
            }
            shift[j] = (int)mr;
            delta = std::max(delta, std::fabs(mv - mr));
        }
        // |d g / d n| <= (2 pi (|f_c| + 2 |c| T) + T / dt^2) / fs over |tau| <= T = n / fs,
        // so shifting by delta samples moves a score by at most delta sqrt(2 n) times
        // that over |g_w| >= 1 (the centre sample, g(0) = 1, is present)
        {
            double fmax = 0.0, cmax = 0.0, dtmin = INFINITY;
            for (int j = 0; j < ax[1]->count; ++j) fmax = std::max(fmax, std::fabs(vals[p->grid.off[1] + j]));
            for (int j = 0; j < ax[2]->count; ++j) cmax = std::max(cmax, std::fabs(vals[p->grid.off[2] + j]));
            for (int j = 0; j < ax[3]->count; ++j) dtmin = std::min(dtmin, std::exp(vals[p->grid.off[3] + j]));
            const double T = gr.n_samples / gr.fs_hz;
            const double slope = (2.0 * M_PI * (fmax + 2.0 * cmax * T) + T / (dtmin * dtmin)) / gr.fs_hz;
            p->shift_eps = delta > 0.0 ? 1.01 * delta * std::sqrt(2.0 * gr.n_samples) * slope : 0.0;
        }
        p->n_cl = ax[2]->count * ax[3]->count;
        p->fac_w = 2 * p->n_pad;
        const size_t ucl = (size_t)p->n_cl * p->fac_w * sizeof(float);
        const size_t ufc = (size_t)ax[1]->count * p->fac_w * sizeof(float);
        if (synth32) {
            PLAN_HIP(hipMalloc(&p->fac_u, ucl));
            PLAN_HIP(hipMalloc(&p->fac_v, ucl));
            PLAN_HIP(hipMalloc(&p->fac_c, ufc));
            PLAN_HIP(hipMalloc(&p->fac_s, ufc));
        }
        PLAN_HIP(hipMalloc((void**)&p->inv_norm, (size_t)atoms * sizeof(double)));
        PLAN_HIP(hipMalloc((void**)&p->inv_norm32, (size_t)atoms * sizeof(float)));
        PLAN_HIP(hipMalloc((void**)&p->tc_shift, shift.size() * sizeof(int)));
        PLAN_HIP(hipMemcpyAsync(p->tc_shift, shift.data(), shift.size() * sizeof(int), hipMemcpyHostToDevice, s));
        p->tc_shift_host = shift;
        p->table_bytes = 0;
        if (desc->dict == ACT_DICT_LAG) {
            const long long Q = (long long)ax[1]->count * p->n_cl;
            // complex atoms: a 32-column block of cos parts, then the block of
            // their sin parts
            const long long cols = desc->complex_atoms ? 2 * ((Q + 31) / 32 * 32) : Q;
            p->lag_q_pad = (int)((cols + 255) / 256 * 256);
            p->table_bytes = (size_t)p->lag_q_pad * (2 * p->n_pad) * 2;
            if ((2.0 * p->max_batch + 1.0) * p->n_pad * 2.0 >= 2147483648.0) {
                set_error("act_plan: the lag-table search addresses its FP16 residual copy with 32-bit offsets; "
                          "max_batch x padded length is too large");
                return fail(ACT_ERR_INVALID);
            }
            size_t free_b = 0, total_b = 0;
            PLAN_HIP(hipMemGetInfo(&free_b, &total_b));
            if (p->table_bytes + (64ull << 20) > free_b) {
                set_error("act_plan: lag table of " + std::to_string(p->table_bytes) +
                          " bytes does not fit in free device memory");
                return fail(ACT_ERR_NOMEM);
            }
            PLAN_HIP(hipMalloc(&p->table, p->table_bytes));
            PLAN_HIP(hipMalloc((void**)&p->rscale, B * sizeof(float)));
            PLAN_HIP(hipMalloc((void**)&p->lag_inv, (size_t)p->grid.cnt[0] * p->lag_q_pad * sizeof(float)));
            if (desc->ragged) {
                PLAN_HIP(hipMalloc((void**)&p->perm, B * sizeof(int)));
                PLAN_HIP(hipMalloc((void**)&p->lag_rows, (B / 32 + 2) * sizeof(int)));
                // distances to the end below which an atom's tail beyond the end
                // can matter: 7 of the longest duration (tail energy < e^-49 dt fs)
                double ldmax = -INFINITY;
                for (int j = 0; j < ax[3]->count; ++j) ldmax = std::max(ldmax, vals[p->grid.off[3] + j]);
                p->lag_rho_d = (int)std::min<double>(p->n_pad, std::ceil(7.0 * std::exp(ldmax) * gr.fs_hz) + 2.0);
                PLAN_HIP(hipMalloc((void**)&p->lag_rho, (size_t)(p->lag_q_pad / 256) * p->lag_rho_d * sizeof(float)));
            }
            PLAN_HIP(hipMalloc((void**)&p->lag_span, (size_t)(p->lag_q_pad / 32) * 2 * sizeof(int)));
            PLAN_HIP(hipMalloc((void**)&p->lag_order, (size_t)(p->lag_q_pad / 128 + p->lag_q_pad / 256) * sizeof(int)));
        }
    }
    if (synth32 && desc->prec == ACT_PREC_F16) {
        const size_t u16b = (size_t)p->n_cl * p->fac_w * 2;
        const size_t c16b = (size_t)ax[1]->count * p->fac_w * 2;
        PLAN_HIP(hipMalloc(&p->fac_u16, u16b));
        PLAN_HIP(hipMalloc(&p->fac_v16, u16b));
        PLAN_HIP(hipMalloc(&p->fac_c16, c16b));
        PLAN_HIP(hipMalloc(&p->fac_s16, c16b));
        PLAN_HIP(hipMalloc((void**)&p->env_q, (size_t)ax[3]->count * p->fac_w * sizeof(double)));
        PLAN_HIP(hipMalloc((void**)&p->rscale, B * sizeof(float)));
        PLAN_HIP(hipMalloc((void**)&p->ebmul, B * sizeof(double)));
        if (desc->ragged) PLAN_HIP(hipMalloc((void**)&p->perm, B * sizeof(int)));
        PLAN_HIP(hipMalloc((void**)&p->tmax, B * p->grid.cnt[0] * sizeof(unsigned)));
        PLAN_HIP(hipMalloc((void**)&p->ld_half, ax[3]->count * sizeof(int)));
        if (desc->ragged)
            PLAN_HIP(hipMalloc((void**)&p->inv_full32, (size_t)ax[1]->count * p->n_cl * sizeof(float)));
    }
    if (desc->prior_act) {
        PLAN_HIP(hipMalloc((void**)&p->prior_s, B * p->n * sizeof(double)));
        PLAN_HIP(hipMalloc((void**)&p->prior_part, B * prior_workspace_blocks() * sizeof(double)));
        PLAN_HIP(hipMalloc((void**)&p->prior_pidx, B * prior_workspace_blocks() * sizeof(long long)));
    }
    {
        // lag-table plans: rows 2 n_pad apart after a zero guard of n_pad, so
        // every lag window of a row lies inside the allocation and reads zeros
        // outside the row's samples
        const bool guard = desc->dict == ACT_DICT_LAG;
        p->sh_stride = guard ? 2 * p->n_pad : p->n_pad;
        const size_t sh_elems = guard ? (2 * B + 1) * p->n_pad : B * p->n_pad;
        PLAN_HIP(hipMalloc(&p->shadow_alloc, sh_elems * elt));
        PLAN_HIP(hipMemsetAsync(p->shadow_alloc, 0, sh_elems * elt, s));
        p->shadow = (char*)p->shadow_alloc + (guard ? p->n_pad * elt : 0);
    }
    PLAN_HIP(hipMalloc((void**)&p->cand_idx, B * cap * sizeof(unsigned)));
    PLAN_HIP(hipMalloc((void**)&p->cand_score, B * cap * sizeof(float)));
    PLAN_HIP(hipMalloc((void**)&p->cand_p64, B * cap * sizeof(double)));
    PLAN_HIP(hipMalloc((void**)&p->cand_count, B * sizeof(int)));
    PLAN_HIP(hipMalloc((void**)&p->gmax, B * sizeof(unsigned)));
    PLAN_HIP(hipMalloc((void**)&p->ebound, B * sizeof(double)));
    PLAN_HIP(hipMalloc((void**)&p->rnorm, B * sizeof(double)));
    PLAN_HIP(hipMalloc((void**)&p->need_rerun, B * sizeof(int)));
    if (desc->dict == ACT_DICT_LAG || (desc->dict == ACT_DICT_SYNTH && desc->prec == ACT_PREC_F16)) {
        PLAN_HIP(hipMalloc((void**)&p->exec_count, 2 * sizeof(unsigned long long)));
        PLAN_HIP(hipMemsetAsync(p->exec_count, 0, 2 * sizeof(unsigned long long), s));
    }
    p->workspace_bytes = B * p->n_pad * elt + B * cap * 16 + B * 32;
#undef PLAN_HIP

    act_status bs = build_tables(p, s);
    if (bs != ACT_OK) return fail(bs);
    if (desc->dict == ACT_DICT_LAG) {
        if ((bs = build_lag(p, s)) != ACT_OK) return fail(bs);
    }
    if (synth32) {
        bs = build_synth(p, s);
        if (bs != ACT_OK) return fail(bs);
        if (desc->prec == ACT_PREC_F16 && (bs = build_h16_factors(p, s)) != ACT_OK) return fail(bs);
        if (desc->prec == ACT_PREC_F16 && (bs = build_supports(p, s)) != ACT_OK) return fail(bs);
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error(std::string("act_plan: ") + hipGetErrorString(e));
        return fail(ACT_ERR_HIP);
    }
    p->last_stream = s;
    *out = p;
    return ACT_OK;
}

extern "C" void act_plan_destroy(act_plan_t plan) { free_plan(plan); }

extern "C" int64_t act_plan_query(act_plan_t p, int32_t key) {
    if (!p) return -1;
    switch (key) {
        case ACT_Q_ATOMS: return p->atoms;
        case ACT_Q_TABLE_BYTES: return (int64_t)p->table_bytes;
        case ACT_Q_N_PAD: return p->n_pad;
        case ACT_Q_CAND_CAP: return p->cap;
        case ACT_Q_WORKSPACE_BYTES: return (int64_t)p->workspace_bytes;
        case ACT_Q_LAG_RESIDENT: return p->lag_rs_cp ? 1 : 0;
        default: return -1;
    }
}

extern "C" act_status act_search_executed(act_plan_t p, double* flops, int64_t* launches) {
    ACT_REQUIRE(p != nullptr && flops != nullptr && launches != nullptr,
                "act_search_executed: plan, flops or launches is NULL");
    if (!p->exec_count) {
        set_error("act_search_executed: only the lag-table and FP16 synthesised searches count their work");
        return ACT_ERR_UNSUPPORTED;
    }
    ACT_HIP(hipStreamSynchronize(p->last_stream));
    unsigned long long c[2] = {0, 0};
    ACT_HIP(hipMemcpy(c, p->exec_count, sizeof c, hipMemcpyDeviceToHost));
    const unsigned long long zero[2] = {0, 0};
    ACT_HIP(hipMemcpy(p->exec_count, zero, sizeof zero, hipMemcpyHostToDevice));
    // v_mfma_f32_32x32x16_{f16,bf16}: 32 x 32 x 16 multiply-adds
    *flops = (double)c[0] * (32.0 * 32.0 * 16.0 * 2.0);
    *launches = (int64_t)c[1];
    return ACT_OK;
}

extern "C" act_status act_search_flops(act_plan_t p, int32_t batch, double* flops) {
    ACT_REQUIRE(p != nullptr && flops != nullptr, "act_search_flops: plan or flops is NULL");
    ACT_REQUIRE(batch >= 1 && batch <= p->max_batch, "act_search_flops: batch outside [1, max_batch]");
    if (p->desc.dict != ACT_DICT_LAG || p->desc.ragged) {
        set_error("act_search_flops: only the lag-table search of plain plans has a counted matrix-core workload");
        return ACT_ERR_UNSUPPORTED;
    }
    select_shape(p, batch);  // the form of the lag-table search depends on the batch's shape
    *flops = lag_search_flops(p, batch);
    return ACT_OK;
}
