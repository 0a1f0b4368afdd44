// act_refine.hip -- per-channel FP64 work of every matching-pursuit order:
// certified FP64 rescoring of the search candidates, arg-max with the lowest
// index on ties, continuous refinement (Sec. III-A "BFGS refinement") by
// L-BFGS over the closed-form forward + adjoint of J(theta) = <r,g>^2/<g,g>,
// the coefficient c_k = <g*, r_k> with the refined unit atom, and the residual /
// approximation update of Eq. (4) with the energy |r_{k+1}|^2 (Eq. (5)).
#include <math.h>

#include <type_traits>

#include "act_common.h"

namespace act {

struct PlanDev {
    GridDev g;
    BoxDev box;
    int prec, dict, cap, chain;
    double eg_max, rho_max;
    void* shadow;
    int sh_stride;           // shadow row stride (elements)
    unsigned* cand_idx;
    float* cand_score;
    double* cand_p64;
    int* cand_count;
    unsigned* gmax;
    double* ebound;
    double* rnorm;
    int* need_rerun;
    const int* len;          // ragged plans: channel lengths and offsets
    const long long* off;
    int* items;              // ragged synthesised plans: tile queue (counters after [B])
    const int* by_length;    // ragged lag and FP16 plans: the call's channels by decreasing length
    int batch;
    float* rscale;           // ACT_PREC_F16: [B] power-of-two scale of the FP16 search copy
    double* ebmul;           // ACT_PREC_F16: [B] per-atom bound factor
    unsigned* tmax;          // ACT_PREC_F16: [B][n_tc] pass-0 upper bound per time centre
    double trunc_tail;       // ACT_PREC_F16 with support_cut: skipped envelope tail (relative)
    double shift_eps;        // synthesised / lag searches: time centres rounded to samples (relative)
    bool per_atom;           // gmax holds the max lower bound, cand_score upper bounds
    bool cplx;               // complex atoms: scores |<g_hat, r>|, two-part update
};

static PlanDev view(const act_plan_s* p) {
    PlanDev v;
    v.g = p->grid;
    v.box = p->box;
    v.prec = p->desc.prec;
    v.dict = p->desc.dict;
    v.rho_max = p->rho_max;
    v.cap = p->cap;
    v.chain = p->chain;
    v.eg_max = p->eg_max;
    v.shadow = p->shadow;
    v.sh_stride = p->sh_stride;
    v.cand_idx = p->cand_idx;
    v.cand_score = p->cand_score;
    v.cand_p64 = p->cand_p64;
    v.cand_count = p->cand_count;
    v.gmax = p->gmax;
    v.ebound = p->ebound;
    v.rnorm = p->rnorm;
    v.need_rerun = p->need_rerun;
    v.len = p->call_len;
    v.off = p->call_off;
    v.items = p->items;
    // filled by the call's ragged set-up for lag-table and FP16 plans only
    v.by_length = p->desc.ragged && (p->desc.dict == ACT_DICT_LAG || p->desc.prec == ACT_PREC_F16) ? p->perm
                                                                                                  : nullptr;
    v.batch = 0;
    v.rscale = p->rscale;
    v.ebmul = p->ebmul;
    v.tmax = p->tmax;
    v.trunc_tail = p->trunc_tail;
    v.shift_eps = p->shift_eps;
    v.per_atom = p->desc.prec == ACT_PREC_F16 && p->desc.dict == ACT_DICT_SYNTH;
    v.cplx = p->desc.complex_atoms != 0;
    return v;
}

constexpr int NT = 256;            // threads of every per-channel kernel
constexpr int NW = NT / kWave;

// Proven bound on |p~ - p| of one channel's search scores, where rn = |r|
// and er = |r - shadow(r)| (the rounding of the search copy of r):
//   p~ = fl( sum g~ r~ ),  g~ = g_hat + e_g (|e_g| <= eg_max),  r~ = r + e_r
//   |sum g~ r~ - p| <= eg_max |r~| + |e_r|
//   |fl(sum) - sum| <= gamma_m |g~| |r~|, gamma_m = m u / (1 - m u)   (chain m)
// FP64 searches round the score to FP32 when storing it: u32 |r| + FP64 sums.
//
// Complex atoms: a = <r, Re g_hat> and b = <r, Im g_hat> each obey the bound of
// the real score (|Re g_hat|, |Im g_hat| <= 1, and each factored product pair
// sums to at most |E| |r|), so |sqrt(a~^2 + b~^2) - sqrt(a^2 + b^2)| <= sqrt(2)
// times it; squaring, summing, the square root, the FP32 1/|E| and the scaling
// add <= 6 u |r~| (the score is at most |r~|).  FP64: two sums of n terms and
// the norm sum, <= 3 (n + 16) u64 |r| before the FP32 store.
__device__ double score_bound(const PlanDev& P, double rn, double er, double scale, int n) {
    const double u32 = 5.9604644775390625e-08;  // 2^-24
    if (P.prec == ACT_PREC_F64)
        return 1.01 * (u32 + (P.cplx ? 3.0 : 1.0) * (P.g.n + 16) * 2.220446049250313e-16) * rn;
    const double rt = rn + er;
    const double m = (double)P.chain;
    const double gam = m * u32 / (1.0 - m * u32);
    if (P.dict == ACT_DICT_LAG) {
        // FP16 lag table: |fl16(fl32(g)) - g| <= (u16 + u32) |g| + 2^-25 per
        // sample, so over the atom's window (|g_w| >= 1, at most 2N samples) the
        // table error is <= (u16 + u32 + 2^-25 sqrt(2N)) |r~| after 1/|g_w|; the
        // FP16 products are exact in FP32, their sum carries gamma_m; the FP32
        // 1/|g| and the scalings add <= 3 u |r~|; the search copy's error |e_r|.
        // BF16 table: u16 becomes 2^-8, with the same 2^-25 floor (entries
        // below it are zero); the copy's subnormal floor (at most 2^-126 per
        // sample of a copy whose channel maximum is scaled to >= 2^12) and the
        // second-order products of the two roundings lie inside the 1% margin
        const double u16 = P.prec == ACT_PREC_BF16 ? 3.90625e-03 : 4.8828125e-04;
        const double eg = u16 + u32 + 2.98023223876953125e-08 * sqrt(2.0 * n);
        (void)scale;
        if (P.cplx) {
            // complex atoms: each part a = <E cos phi, r>, b = <E sin phi, r>
            // carries the real bound with |E_w cos phi| <= |E_w| (|E_w| >= 1);
            // |sqrt(a~^2 + b~^2) - sqrt(a^2 + b^2)| <= |(da, db)| <= sqrt(2) x
            // that, and the squares, sum, root and the two scalings add 6 u |r~|
            const double part = eg * rt + er + gam * (1.0 + eg) * rt + P.shift_eps * rt;
            return 1.01 * (1.4142135623730951 * part + 6.0 * u32 * rt);
        }
        return 1.01 * (eg * rt + er + gam * (1.0 + eg) * rt + 3.0 * u32 * rt + P.shift_eps * rt);
    }
    if (P.prec == ACT_PREC_F16) {
        // additive part of the per-atom bound (the part that scales with
        // |E_w| / |g_w| is h16_bound_mul): the FP16 search copy's own error
        // |r - r~| (Cauchy-Schwarz), the FP32 1/|g| (<= 2.5 u when computed
        // from the prefix sums) and the scalings by 1/|g| and 1/s, and the FP16
        // subnormal floor 2^-25 of the A operand: sum_n 2^-25 |B_n|
        // <= 2^-25 sqrt(2N) |r~|, with |g_w| >= 1 (the centre sample is present).
        const double sub = 2.98023223876953125e-08 * sqrt(2.0 * n);  // 2^-25 sqrt(2N)
        (void)scale;
        // support cut: the skipped products sum to at most sqrt(tail) |r| / |g_w|
        // (|g| <= E and Cauchy-Schwarz), and |g_w| >= 1
        return 1.01 * (er + 6.0 * u32 * rt + sub * rt + P.trunc_tail * rt + P.shift_eps * rt);
    }
    if (P.dict == ACT_DICT_SYNTH && P.cplx) {
        const double part = (5.0 * u32 + gam) * 1.4142135623730951 * P.rho_max * rt + er + P.shift_eps * rt;
        return 1.01 * (1.4142135623730951 * part + 6.0 * u32 * rt);
    }
    if (P.dict == ACT_DICT_SYNTH) {
        // factored synthesis: each product U (C r) carries <= 5 FP32 roundings
        // (factors, r, the carrier product, the MFMA product) plus the chain,
        // against sum_n (|U C| + |V S|)|r_n| <= sqrt(2) |E| |r| = sqrt(2) rho |g| |r|;
        // the scaling by 1/|g| in FP32 adds 2 u |p|.
        return 1.01 * ((5.0 * u32 + gam) * 1.4142135623730951 * P.rho_max * rt + er + 3.0 * u32 * rn +
                       P.shift_eps * rt);
    }
    return 1.01 * (P.eg_max * rt + er + gam * (1.0 + P.eg_max) * rt);
}

// Factor of |E_w| / |g_w| in the per-atom bound of the FP16 synthesised search.
// Each product U (C r~ s) carries FP16 roundings of U and C (each after an
// FP32 one) and of the packed product: <= 3.01 u16 + 2 u32 relative, against
// sum_n (|U C| + |V S|)|r~_n| <= |E_w| |r~| (|cos a cos b| + |sin a sin b| is
// |cos(a - b)| or |cos(a + b)|, at most 1); plus the FP32 chain, the
// subnormal floor 2^-25 of C (times |r~ s| <= 2^13, i.e. 2^-25 max|r~| after
// 1/s) and of the product (2^-25 / s), each summed against |E_w| sqrt(2N).
__device__ double h16_bound_mul(double rn, double er, double scale, int n) {
    const double u32 = 5.9604644775390625e-08, u16 = 4.8828125e-04;
    // the channel's own chain: its 2N products (the zero samples past its end
    // add exactly), plus the final scalings
    const double m = 2.0 * n + 2.0;
    const double gam = m * u32 / (1.0 - m * u32);
    const double rt = rn + er;
    const double sub = 2.98023223876953125e-08 * sqrt(2.0 * n);
    return 1.01 * ((3.01 * u16 + 2.0 * u32 + gam) * rt + sub * (rt + 1.0 / scale));
}

// Largest |fl32(r_k)| of a channel (block-wide; every thread gets it).
template <int TB>
__device__ float block_absmax(const double* r, int n) {
    __shared__ unsigned s_mx;
    if (threadIdx.x == 0) s_mx = 0u;
    __syncthreads();
    float m = 0.0f;
    for (int k = threadIdx.x; k < n; k += TB) m = fmaxf(m, fabsf((float)r[k]));
    m = wave_max(m);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&s_mx, __float_as_uint(m));
    __syncthreads();
    const float v = __uint_as_float(s_mx);
    __syncthreads();
    return v;
}

// Power of two s with s max|r| in [2^12, 2^13): the FP16 operand C r s stays
// below 2^13 and its subnormal floor 2^-25 / s is at most 2^-37 max|r|.
// Clamped to [2^-100, 2^100] (the error bound uses the actual s).
__device__ __forceinline__ float f16_operand_scale(float absmax) {
    if (!(absmax > 0.0f) || !isfinite(absmax)) return 1.0f;
    int ex;
    (void)frexpf(absmax, &ex);  // absmax = f 2^ex, f in [0.5, 1)
    int k = 13 - ex;
    k = k < -100 ? -100 : (k > 100 ? 100 : k);
    return ldexpf(1.0f, k);
}

// E = |r|^2, the search copy of r (FP32 or BF16, zero padded) and its rounding
// error; resets the channel's search state.  Block-wide; returns E.
template <int TB>
__device__ double refresh_channel(const PlanDev& P, int b, const double* r, int n, double* red,
                                  bool bad) {
    double acc[2] = {0.0, 0.0};
    // power-of-two scale of the FP16 copy, and of the BF16 copy the lag table
    // multiplies (it keeps small residuals clear of the subnormal range)
    const bool scaled = P.prec == ACT_PREC_F16 || (P.prec == ACT_PREC_BF16 && P.dict == ACT_DICT_LAG);
    const float scale = scaled ? f16_operand_scale(block_absmax<TB>(r, n)) : 1.0f;
    for (int k = threadIdx.x; k < P.g.n_pad; k += TB) {
        const double v = k < n ? r[k] : 0.0;
        double back;
        if (P.prec == ACT_PREC_F16) {
            // search copy r~ = fl16(fl32(r) s) / s, stored scaled
            const _Float16 h = (_Float16)((float)v * scale);
            ((_Float16*)P.shadow)[(size_t)b * P.sh_stride + k] = h;
            back = (double)(float)h / (double)scale;
        } else if (P.prec == ACT_PREC_BF16) {
            unsigned short h = bf16_rne((float)v * scale);
            ((unsigned short*)P.shadow)[(size_t)b * P.sh_stride + k] = h;
            back = (double)__uint_as_float(((unsigned)h) << 16) / (double)scale;
        } else {
            const float f = (float)v;
            ((float*)P.shadow)[(size_t)b * P.sh_stride + k] = f;
            back = (double)f;
        }
        acc[0] += v * v;
        const double d = v - back;
        acc[1] += d * d;
    }
    if (P.tmax)
        for (int k = threadIdx.x; k < P.g.cnt[0]; k += TB) P.tmax[(size_t)b * P.g.cnt[0] + k] = 0u;
    block_sum<TB, 2>(acc, red);
    if (threadIdx.x == 0) {
        const double rn = sqrt(acc[0]);
        P.rnorm[b] = rn;
        if (P.rscale) P.rscale[b] = scale;
        if (P.ebmul) P.ebmul[b] = h16_bound_mul(rn, sqrt(acc[1]), scale, n);
        P.ebound[b] = (bad || !(acc[0] > 0.0) || !isfinite(acc[0])) ? -1.0
                                                                     : score_bound(P, rn, sqrt(acc[1]), scale, n);
        P.cand_count[b] = 0;
        P.gmax[b] = 0u;
        P.need_rerun[b] = 0;
    }
    return acc[0];
}

__global__ void __launch_bounds__(NT) k_init(PlanDev P, double* __restrict__ resid,
                                             double* __restrict__ approx,
                                             double* __restrict__ energy, int* __restrict__ flags,
                                             int order) {
    __shared__ double red[block_sum_lds(NT, 2)];
    const int b = blockIdx.x;
    const ChanGeom cg = chan_geom(P.g, b, P.len, P.off);
    const int n = cg.g.n;
    const double* r = resid + cg.off;
    int bad = 0;
    for (int k = threadIdx.x; k < n; k += NT) {
        if (!isfinite(r[k])) bad = 1;
        if (approx) approx[cg.off + k] = 0.0;
    }
    bad = __syncthreads_or(bad);
    const bool empty = cg.g.atoms == 0;
    const bool bad_len = P.len && (P.len[b] < 0 || P.len[b] > P.g.n);
    const double E = refresh_channel<NT>(P, b, r, n, red, bad != 0 || empty);
    if (threadIdx.x == 0) {
        energy[(size_t)b * (order + 1)] = E;
        flags[b] = (bad ? ACT_FLAG_NONFINITE : 0) | (empty ? ACT_FLAG_RAGGED_EMPTY : 0) |
                   (bad_len ? ACT_FLAG_BAD_LENGTH : 0);
    }
}

__global__ void __launch_bounds__(256) k_to_shadow(PlanDev P, const double* __restrict__ resid) {
    const int b = blockIdx.x;
    if (P.prec == ACT_PREC_F16 || (P.prec == ACT_PREC_BF16 && P.dict == ACT_DICT_LAG)) {
        const float sc = f16_operand_scale(block_absmax<256>(resid + (size_t)b * P.g.n, P.g.n));
        if (threadIdx.x == 0) P.rscale[b] = sc;
        for (int k = threadIdx.x; k < P.g.n_pad; k += blockDim.x) {
            const double v = k < P.g.n ? resid[(size_t)b * P.g.n + k] : 0.0;
            if (P.prec == ACT_PREC_F16)
                ((_Float16*)P.shadow)[(size_t)b * P.sh_stride + k] = (_Float16)((float)v * sc);
            else
                ((unsigned short*)P.shadow)[(size_t)b * P.sh_stride + k] = bf16_rne((float)v * sc);
        }
        return;
    }
    for (int k = threadIdx.x; k < P.g.n_pad; k += blockDim.x) {
        const double v = k < P.g.n ? resid[(size_t)b * P.g.n + k] : 0.0;
        if (P.prec == ACT_PREC_BF16)
            ((unsigned short*)P.shadow)[(size_t)b * P.sh_stride + k] = bf16_rne((float)v);
        else
            ((float*)P.shadow)[(size_t)b * P.sh_stride + k] = (float)v;
    }
}

// Candidate overflow: a channel whose list overflowed is searched again with
// the exact final threshold.
__global__ void k_overflow(PlanDev P, int batch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b == 0 && P.items) P.items[batch + 2] = 0;  // rerun-pass tile queue
    if (b >= batch) return;
    if (P.cand_count[b] > P.cap) {
        P.need_rerun[b] = 1;
        P.cand_count[b] = 0;
        if (P.items) atomicOr(&P.items[batch + 3], 1);  // the rerun queue has work
    } else {
        P.need_rerun[b] = 0;
    }
}

// Samples [k0, k1) within 9 durations of the centre.  Outside them the
// envelope is below e^-40.5 = 2.6e-18 (times at most 81 in a derivative term),
// so the refinement's sums over the window differ from the sums over all n
// samples by less than 1e-15 of their size (the rescore's, by less than FP64
// rounding).
__device__ __forceinline__ void support_window(int n, double fs, const double th[4], int& k0, int& k1) {
    const double half = 9.0 * exp(th[3]) * fs, c = th[0] * fs;
    k0 = (int)fmin((double)n, fmax(0.0, floor(c - half)));
    k1 = (int)fmax((double)k0, fmin((double)n, ceil(c + half) + 1.0));
}

// --------------------------------------------------------------------------
// refinement objective, block-wide
// --------------------------------------------------------------------------

// Per-sample terms of the refinement: g = E C and its partial derivatives
//   d_tc g = E[(tau/dt^2) C + 2 pi (2 c tau + f_c) S], d_fc g = -2 pi tau E S,
//   d_c g = -2 pi tau^2 E S, d_logdt g = (tau^2/dt^2) E C,
// from E and (C, S) = (cos, sin) of the phase.
__device__ __forceinline__ void terms_from(double tau, double fc, double c, double idt2, double e, double co,
                                           double si, double& gk, double d[4]) {
    gk = e * co;
    const double es = e * si;
    d[0] = e * (tau * idt2 * co) + kTwoPi * (2.0 * c * tau + fc) * es;
    d[1] = -kTwoPi * tau * es;
    d[2] = -kTwoPi * tau * tau * es;
    d[3] = tau * tau * idt2 * gk;
}

__device__ __forceinline__ void atom_terms64(double tau, double fc, double c, double inv_dt,
                                             double& gk, double d[4]) {
    const double u = tau * inv_dt;
    const double e = exp(-0.5 * u * u);
    double si, co;
    sincospi(2.0 * (c * tau * tau + fc * tau), &si, &co);
    terms_from(tau, fc, c, inv_dt * inv_dt, e, co, si, gk, d);
}

// FP32 forward/adjoint: the phase in cycles is formed and reduced modulo 1 in
// FP64 (an FP32 phase of a long chirp loses whole milliradians); the envelope,
// trigonometry, products and sums are FP32.
__device__ __forceinline__ void atom_terms_f32(double tau64, double c, double fc, float inv_dt,
                                               float& e, float& co, float& si, float& tau) {
    const double cyc = c * tau64 * tau64 + fc * tau64;
    const float red_c = (float)(cyc - rint(cyc));
    sincospif(2.0f * red_c, &si, &co);
    tau = (float)tau64;
    const float u = tau * inv_dt;
    e = expf(-0.5f * u * u);
}

// Visits this thread's samples k = k0 + (threadIdx.x mod TB) + TB j of [k0, k1) with
// (k, tau, E, cos phi, sin phi).  A window of at least 4 TB samples advances
// E and exp(i phi) from the thread's first sample by product recurrences over
// the step H = TB / fs:
//   E(tau + H) = E(tau) rho(tau),          rho(tau + H) = rho(tau) exp(-H^2/dt^2),
//   phi(tau + H) = phi(tau) + psi(tau),    psi(tau + H) = psi(tau) + 4 pi c H^2,
// with rho(tau) = exp(-(2 tau H + H^2)/(2 dt^2)), psi(tau) = 2 pi (c (2 tau H + H^2) + f_c H):
// three exp/sincospi pairs per thread instead of one per sample.  Inside such a
// window dt >= (4 TB - 1)/18 samples, so every factor lies in [e^-41, e^31].
// The rounding of the step angle psi accumulates over the steps: E cos phi and
// E sin phi agree with direct evaluation to about 3e-12 at N = 2048 (6e-12 at
// N = 16384).
template <int TB, typename F>
__device__ __forceinline__ void walk_atom(int k0, int k1, double fs, const double th[4], double inv_dt, F&& visit) {
    const double c = th[2], fc = th[1];
    const double ifs = 1.0 / fs;   // tau = k/fs - t_c as k (1/fs) - t_c: no division per sample
    const int k = k0 + (int)(threadIdx.x % TB);   // TB threads per group (the block may hold several)
    if (k1 - k0 >= 4 * TB) {
        const double H = (double)TB / fs, idt2 = inv_dt * inv_dt;
        const double tau0 = fma((double)k, ifs, -th[0]);
        const double u = tau0 * inv_dt;
        double e = exp(-0.5 * u * u);
        double rho = exp(-0.5 * (2.0 * tau0 * H + H * H) * idt2);
        const double q = exp(-H * H * idt2);
        double si, co, ws, wc, vs, vc;
        sincospi(2.0 * (c * tau0 * tau0 + fc * tau0), &si, &co);
        sincospi(2.0 * (c * (2.0 * tau0 * H + H * H) + fc * H), &ws, &wc);
        sincospi(4.0 * c * H * H, &vs, &vc);
#pragma unroll 1
        for (int kk = k; kk < k1; kk += TB) {
            visit(kk, fma((double)kk, ifs, -th[0]), e, co, si);
            e *= rho;
            rho *= q;
            const double co2 = co * wc - si * ws;
            si = si * wc + co * ws;
            co = co2;
            const double wc2 = wc * vc - ws * vs;
            ws = ws * vc + wc * vs;
            wc = wc2;
        }
    } else {
#pragma unroll 1
        for (int kk = k; kk < k1; kk += TB) {
            const double tau = fma((double)kk, ifs, -th[0]);
            const double u = tau * inv_dt;
            const double e = exp(-0.5 * u * u);
            double si, co;
            sincospi(2.0 * (c * tau * tau + fc * tau), &si, &co);
            visit(kk, tau, e, co, si);
        }
    }
}

// walk_atom for callers that need only g = E cos phi and E sin phi: the
// product z = E exp(i phi) = exp(a tau^2 + b tau), a = -1/(2 dt^2) + 2 pi i c,
// b = 2 pi i f_c, advances by complex factors,
//   z(tau + H) = z(tau) w(tau),  w(tau) = exp(a (2 tau H + H^2) + b H),
//   w(tau + H) = w(tau) v,       v = exp(2 a H^2),
// (|w| and arg w are the rho and psi of walk_atom, |v| and arg v its
// exp(-H^2/dt^2) and 4 pi c H^2): two complex products per sample, and no
// separate envelope.  Its steps cost less than walk_atom's, so the recurrence
// starts at 2 TB window samples (two per thread): inside such a window
// dt >= (2 TB - 1)/18 samples, so |w| lies in [e^-122, e^41] and |v| >= e^-81,
// far inside FP64's range; the rounding is walk_atom's.
// visit(k, tau, E cos phi, E sin phi).
template <int TB, typename F>
__device__ __forceinline__ void walk_chirp(int k0, int k1, double fs, const double th[4], double inv_dt,
                                           F&& visit) {
    const double c = th[2], fc = th[1];
    const double ifs = 1.0 / fs;
    const int k = k0 + (int)(threadIdx.x % TB);
    if (k1 - k0 >= 2 * TB) {
        const double H = (double)TB / fs, idt2 = inv_dt * inv_dt;
        const double tau0 = fma((double)k, ifs, -th[0]);
        const double u = tau0 * inv_dt;
        const double e = exp(-0.5 * u * u);
        const double rho = exp(-0.5 * (2.0 * tau0 * H + H * H) * idt2);
        const double q = exp(-H * H * idt2);
        double si, co, ws, wc, vs, vc;
        sincospi(2.0 * (c * tau0 * tau0 + fc * tau0), &si, &co);
        sincospi(2.0 * (c * (2.0 * tau0 * H + H * H) + fc * H), &ws, &wc);
        sincospi(4.0 * c * H * H, &vs, &vc);
        double zr = e * co, zi = e * si, wr = rho * wc, wi = rho * ws;
        const double vr = q * vc, vi = q * vs;
#pragma unroll 2   // two samples' independent products interleave
        for (int kk = k; kk < k1; kk += TB) {
            visit(kk, fma((double)kk, ifs, -th[0]), zr, zi);
            const double zr2 = zr * wr - zi * wi;
            zi = zr * wi + zi * wr;
            zr = zr2;
            const double wr2 = wr * vr - wi * vi;
            wi = wr * vi + wi * vr;
            wr = wr2;
        }
    } else {
#pragma unroll 1
        for (int kk = k; kk < k1; kk += TB) {
            const double tau = fma((double)kk, ifs, -th[0]);
            const double u = tau * inv_dt;
            const double e = exp(-0.5 * u * u);
            double si, co;
            sincospi(2.0 * (c * tau * tau + fc * tau), &si, &co);
            visit(kk, tau, e * co, e * si);
        }
    }
}

// FP64 rescoring: one wave per candidate whose search score lies inside the
// certified margin of the channel's final maximum; others are marked NaN.
// The atom's samples over its support window come from the chirp walk (the
// lanes' first samples direct, then complex-product recurrences; windows of
// fewer than two samples per lane are evaluated directly).  Each sample is
// then within about 2e-12 of direct evaluation (atom peak 1), so a score
// moves by at most 2e-12 sqrt(window) |r|: far inside every search form's
// certified margin, and below the 1e-6 relative gap at which selections are
// held to the exact arg-max.
__global__ void __launch_bounds__(256) k_rescore(PlanDev P, const double* __restrict__ resid) {
    const int b = P.by_length ? P.by_length[blockIdx.y] : (int)blockIdx.y;  // uneven batches: longest first
    const double eb = P.ebound[b];
    if (eb < 0.0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int cnt = min(P.cand_count[b], P.cap);
    // per-atom bounds: candidates carry upper bounds, gmax the largest lower bound
    const double T = P.per_atom ? (double)bitsf(P.gmax[b]) : (double)bitsf(P.gmax[b]) - 2.0 * eb;
    const ChanGeom cg = chan_geom(P.g, b, P.len, P.off);
    const double* r = resid + cg.off;
    const int wpb = blockDim.x / kWave, stride = gridDim.x * wpb;
    // wave w takes the list entries w, w + stride, ...: its lanes test the
    // next 64 of them against T at once (marking those below it), then the
    // wave rescores the ones that pass, in list order
    for (int j0 = blockIdx.x * wpb + threadIdx.x / kWave; j0 < cnt; j0 += stride * kWave) {
        const int jl = j0 + stride * lane;
        bool keep = false;
        if (jl < cnt) {
            const size_t sl = (size_t)b * P.cap + jl;
            keep = !((double)fabsf(P.cand_score[sl]) < T);
            if (!keep) P.cand_p64[sl] = __longlong_as_double(0x7ff8000000000000LL);
        }
        unsigned long long pend = __ballot(keep);
        while (pend) {
            const int l = __ffsll(pend) - 1;
            pend &= pend - 1ull;
            const size_t slot = (size_t)b * P.cap + (j0 + stride * l);
            double th[4];
            grid_theta(cg.g, (long long)P.cand_idx[slot], th);
            const double inv_dt = 1.0 / exp(th[3]);
            double s = 0.0, q = 0.0, sb = 0.0;
            // the atom's support window: the samples beyond it add below
            // 2.6e-18 sqrt(n) |r| to the score (|g| >= 1), under FP64 rounding
            int k0, k1;
            support_window(cg.g.n, cg.g.fs, th, k0, k1);
            if (P.cplx) {
                walk_chirp<kWave>(k0, k1, cg.g.fs, th, inv_dt, [&](int k, double, double re, double im) {
                    const double rk = r[k];
                    s += re * rk;
                    sb += im * rk;
                    q += re * re + im * im;
                });
                sb = wave_sum(sb);
            } else {
                walk_chirp<kWave>(k0, k1, cg.g.fs, th, inv_dt, [&](int k, double, double v, double) {
                    const double rk = r[k];
                    s += v * rk;
                    q += v * v;
                });
            }
            s = wave_sum(s);
            q = wave_sum(q);
            if (P.cplx) s = sqrt(s * s + sb * sb);
            if (lane == 0) P.cand_p64[slot] = q > 0.0 ? s / sqrt(q) : 0.0;
        }
    }
}

// Sums of the objective over every sample: {<r,g>, <g,g>, <r,d_j g> (4),
// <g,d_j g> (4)}.
template <int TB>
__device__ void sums_obj(const double* __restrict__ r, int n, double fs, const double th[4],
                         double (&acc)[10], double* red) {
    const double inv_dt = 1.0 / exp(th[3]);
#pragma unroll
    for (int j = 0; j < 10; ++j) acc[j] = 0.0;
#pragma unroll 1
    for (int k = threadIdx.x; k < n; k += TB) {
        double gk, d[4];
        atom_terms64(sample_time(k, fs) - th[0], th[1], th[2], inv_dt, gk, d);
        const double rk = r[k];
        acc[0] += rk * gk;
        acc[1] += gk * gk;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[2 + j] += rk * d[j];
            acc[6 + j] += gk * d[j];
        }
    }
    block_sum<TB, 10>(acc, red);
}

// The same ten sums over the support window, accumulated as moments in tau:
// with g = E C, the quadrature part E S, and x one of the products
// {r g, r E S, g g, g E S}, the twelve sums M_m(x) = sum x tau^m (m = 0, 1, 2)
// give
//   <r, d_tc g> = M_1(r g)/dt^2 + 2 pi (2 c M_1(r E S) + f_c M_0(r E S)),
//   <r, d_fc g> = -2 pi M_1(r E S),   <r, d_c g> = -2 pi M_2(r E S),
//   <r, d_logdt g> = M_2(r g)/dt^2,
// and <g, d_j g> alike from (g g, g E S): the per-sample terms of terms_from
// regrouped (three operations per product, tau^2 formed once), about half
// the operations per sample.  `red` must hold block_sum_tr_lds(TB, 12)
// doubles.
template <int TB>
__device__ void sums_obj_win(const double* __restrict__ r, int n, double fs, const double th[4],
                             double (&acc)[10], double* red) {
    const double inv_dt = 1.0 / exp(th[3]);
    int k0, k1;
    support_window(n, fs, th, k0, k1);
    double m[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) m[j] = 0.0;
    walk_chirp<TB>(k0, k1, fs, th, inv_dt, [&](int k, double tau, double gk, double es) {
        const double rk = r[k], t2 = tau * tau;
        const double x[4] = {rk * gk, rk * es, gk * gk, gk * es};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            m[3 * q] += x[q];
            m[3 * q + 1] = fma(x[q], tau, m[3 * q + 1]);
            m[3 * q + 2] = fma(x[q], t2, m[3 * q + 2]);
        }
    });
    block_sum_tr<TB, 12>(m, red);
    const double idt2 = inv_dt * inv_dt, c2 = 2.0 * th[2], fc = th[1];
    acc[0] = m[0];
    acc[1] = m[6];
    acc[2] = m[1] * idt2 + kTwoPi * (c2 * m[4] + fc * m[3]);
    acc[3] = -kTwoPi * m[4];
    acc[4] = -kTwoPi * m[5];
    acc[5] = m[2] * idt2;
    acc[6] = m[7] * idt2 + kTwoPi * (c2 * m[10] + fc * m[9]);
    acc[7] = -kTwoPi * m[10];
    acc[8] = -kTwoPi * m[11];
    acc[9] = m[8] * idt2;
}

// The same ten sums in FP32 arithmetic from an FP32 residual, over the
// support window: each sample's terms (phase reduced modulo one cycle in
// FP64, then FP32 envelope, trigonometry and products) and each thread's
// running sums are FP32; the block adds the threads' partial sums in FP64.
template <int TB>
__device__ void sums_obj32(const float* __restrict__ r, int n, double fs, const double th[4], double (&acc)[10],
                           double* red) {
    int k0, k1;
    support_window(n, fs, th, k0, k1);
    const double tc = th[0], fc = th[1], c = th[2];
    const float inv_dt = (float)(1.0 / exp(th[3]));
    const float idt2 = inv_dt * inv_dt;
    const float twopi = 6.2831853071795865f, fcf = (float)fc, cf = (float)c;
    const double ifs = 1.0 / fs;
    float a[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) a[j] = 0.0f;
#pragma unroll 1
    for (int k = k0 + (int)(threadIdx.x % TB); k < k1; k += TB) {
        float e, co, si, tau;
        atom_terms_f32(fma((double)k, ifs, -tc), c, fc, inv_dt, e, co, si, tau);
        const float gk = e * co, es = e * si;
        const float d0 = e * (tau * idt2 * co) + twopi * (2.0f * cf * tau + fcf) * es;
        const float d1 = -twopi * tau * es;
        const float d2 = -twopi * tau * tau * es;
        const float d3 = tau * tau * idt2 * gk;
        const float rk = r[k];
        a[0] += rk * gk;
        a[1] += gk * gk;
        a[2] += rk * d0;
        a[3] += rk * d1;
        a[4] += rk * d2;
        a[5] += rk * d3;
        a[6] += gk * d0;
        a[7] += gk * d1;
        a[8] += gk * d2;
        a[9] += gk * d3;
    }
#pragma unroll
    for (int j = 0; j < 10; ++j) acc[j] = (double)a[j];
    block_sum_tr<TB, 10>(acc, red);
}

// J = s^2/q and dJ/dtheta_j = 2 s <r, d_j g>/q - 2 s^2 <g, d_j g>/q^2.
__device__ __forceinline__ double obj_from_sums(const double acc[10], double grad[4]) {
    const double s = acc[0], q = acc[1];
    if (!(q > 0.0)) {
        grad[0] = grad[1] = grad[2] = grad[3] = 0.0;
        return 0.0;
    }
    const double sq = s * (1.0 / q);
#pragma unroll
    for (int j = 0; j < 4; ++j) grad[j] = 2.0 * sq * (acc[2 + j] - sq * acc[6 + j]);
    return s * sq;
}

template <int TB>
__device__ double eval_obj(const double* __restrict__ r, int n, double fs, const double th[4],
                           double grad[4], double* red) {
    double acc[10];
    sums_obj<TB>(r, n, fs, th, acc, red);
    return obj_from_sums(acc, grad);
}

// Sums of the coordinate scales: {<g,g>, <g,d_j g> (4), <d_j g,d_j g> (4)} over
// the support window (they set the refinement's coordinate scales).
template <int TB>
__device__ void sums_scales(int n, double fs, const double th[4], double (&acc)[9], double* red) {
    const double inv_dt = 1.0 / exp(th[3]);
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[j] = 0.0;
    int k0, k1;
    support_window(n, fs, th, k0, k1);
    const double idt2 = inv_dt * inv_dt;
    walk_atom<TB>(k0, k1, fs, th, inv_dt, [&](int, double tau, double e, double co, double si) {
        double gk, d[4];
        terms_from(tau, th[1], th[2], idt2, e, co, si, gk, d);
        acc[0] += gk * gk;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[1 + j] += gk * d[j];
            acc[5 + j] += d[j] * d[j];
        }
    });
    block_sum_tr<TB, 9>(acc, red);
}

__device__ __forceinline__ double dot4(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

// Complex atoms: J = (a^2 + b^2) / q with a = <r, E cos phi>, b = <r, E sin phi>,
// q = <E, E>.  With dE/dtheta = E (tau/dt^2, 0, 0, tau^2/dt^2) and dphi/dtheta =
// 2 pi (-(2 c tau + f_c), tau, tau^2, 0):
//   da_j = <r, cos phi dE_j - E sin phi dphi_j>, db_j = <r, sin phi dE_j + E cos phi dphi_j>,
//   dq_j = 2 <E, dE_j>,  dJ_j = (2 a da_j + 2 b db_j) / q - J dq_j / q.
// Sums: {a, b, q, da (4), db (4), dq_tc, dq_logdt}.
template <int TB>
__device__ void sums_obj_cplx(const double* __restrict__ r, int n, double fs, const double th[4],
                              double (&acc)[13], double* red) {
    // as for real atoms, the sums regroup into moments M_m(x) = sum x tau^m
    // (m = 0, 1, 2) of x in {r E cos phi, r E sin phi, E^2}, with E cos phi
    // and E sin phi from the chirp walk (E^2 = their squares' sum):
    //   da_tc = M_1(rC)/dt^2 + 2 pi (2 c M_1(rS) + f_c M_0(rS)),
    //   da_fc = -2 pi M_1(rS), da_c = -2 pi M_2(rS), da_logdt = M_2(rC)/dt^2,
    //   db_tc = M_1(rS)/dt^2 - 2 pi (2 c M_1(rC) + f_c M_0(rC)),
    //   db_fc = 2 pi M_1(rC), db_c = 2 pi M_2(rC), db_logdt = M_2(rS)/dt^2,
    //   dq_tc = 2 M_1(E^2)/dt^2, dq_logdt = 2 M_2(E^2)/dt^2.
    const double inv_dt = 1.0 / exp(th[3]);
    int k0, k1;
    support_window(n, fs, th, k0, k1);
    double m[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) m[j] = 0.0;
    walk_chirp<TB>(k0, k1, fs, th, inv_dt, [&](int k, double tau, double gc, double gs) {
        const double rk = r[k], t2 = tau * tau;
        const double x[3] = {rk * gc, rk * gs, gc * gc + gs * gs};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            m[3 * q] += x[q];
            m[3 * q + 1] = fma(x[q], tau, m[3 * q + 1]);
            m[3 * q + 2] = fma(x[q], t2, m[3 * q + 2]);
        }
    });
    block_sum_tr<TB, 9>(m, red);
    const double idt2 = inv_dt * inv_dt, c2 = 2.0 * th[2], fc = th[1];
    acc[0] = m[0];
    acc[1] = m[3];
    acc[2] = m[6];
    acc[3] = m[1] * idt2 + kTwoPi * (c2 * m[4] + fc * m[3]);
    acc[4] = -kTwoPi * m[4];
    acc[5] = -kTwoPi * m[5];
    acc[6] = m[2] * idt2;
    acc[7] = m[4] * idt2 - kTwoPi * (c2 * m[1] + fc * m[0]);
    acc[8] = kTwoPi * m[1];
    acc[9] = kTwoPi * m[2];
    acc[10] = m[5] * idt2;
    acc[11] = 2.0 * m[7] * idt2;
    acc[12] = 2.0 * m[8] * idt2;
}

// Coordinate scales for complex atoms: the metric of the unit complex atom
// modulo a global phase, G_jj = (|d_j g|^2 - |<g, d_j g>|^2 / q) / q with
// d_j g = (dE_j + i E dphi_j) exp(i phi).  Sums: {q, |d_j g|^2 (4),
// sum E dE_j (4), sum E^2 dphi_j (4)}.
template <int TB>
__device__ void sums_scales_cplx(int n, double fs, const double th[4], double (&acc)[13], double* red) {
    const double inv_dt = 1.0 / exp(th[3]);
    const double idt2 = inv_dt * inv_dt;
    const double fc = th[1], c = th[2];
#pragma unroll
    for (int j = 0; j < 13; ++j) acc[j] = 0.0;
    int k0, k1;
    support_window(n, fs, th, k0, k1);
    const double ifs = 1.0 / fs;
#pragma unroll 1
    for (int k = k0 + (int)(threadIdx.x % TB); k < k1; k += TB) {
        const double tau = fma((double)k, ifs, -th[0]);
        const double u = tau * inv_dt;
        const double e = exp(-0.5 * u * u);
        const double de[4] = {e * tau * idt2, 0.0, 0.0, e * tau * tau * idt2};
        const double dp[4] = {-kTwoPi * (2.0 * c * tau + fc), kTwoPi * tau, kTwoPi * tau * tau, 0.0};
        acc[0] += e * e;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[1 + j] += de[j] * de[j] + e * e * dp[j] * dp[j];
            acc[5 + j] += e * de[j];
            acc[9 + j] += e * e * dp[j];
        }
    }
    block_sum_tr<TB, 13>(acc, red);
}

__device__ __forceinline__ double obj_cplx_from_sums(const double acc[13], double grad[4]) {
    const double a = acc[0], b = acc[1], q = acc[2];
    if (!(q > 0.0)) {
        grad[0] = grad[1] = grad[2] = grad[3] = 0.0;
        return 0.0;
    }
    const double iq = 1.0 / q;
    const double J = (a * a + b * b) * iq;
    const double dq[4] = {acc[11], 0.0, 0.0, acc[12]};
#pragma unroll
    for (int j = 0; j < 4; ++j) grad[j] = (2.0 * a * acc[3 + j] + 2.0 * b * acc[7 + j] - J * dq[j]) * iq;
    return J;
}

// --------------------------------------------------------------------------
// Limited-memory BFGS refinement, block-wide.
//
// Every thread runs the same iteration on identical block-reduced values (so
// control flow is uniform and no thread waits for a controller); each lane
// keeps one component of the 4-vectors and of the pair memory in registers.
// Specification
// (identical to the oracle): coordinates u_j = (theta_j - theta0_j)/s_j with
// s_j = min(step_j, 1/sqrt(G_jj)), G_jj the Fisher metric of the unit atom
// along theta_j (axes with one grid value or G_jj <= 0 are frozen); minimise
// f(u) = -J on the grid-hull box; memory 8, H0 = gamma I with gamma = s'y/y'y
// of the newest pair; a pair is kept only if s'y > 1e-12|s||y|;
// projected-gradient stop max|pg| <= 1e-11 max(1, J); direction components
// pointing out of the box at active bounds are zeroed, steepest descent if the
// direction is not a descent direction; first step min(1, 1/max|d|) while the
// memory is empty, else 1; backtracking (halving, <= 30 trials) accepting a
// strict-descent trial by Armijo (c1 = 1e-4) or, once FP64 cannot resolve the
// change of J (f_new <= f + 1e-12|f|), by Hager and Zhang's approximate Wolfe
// slope test 0.9 dec <= dnew <= -0.8 dec; at most `steps` iterations; the
// result is kept only if J does not drop.
// --------------------------------------------------------------------------
// The prior ACT's objective (contrast mode): J = <s, g>^2 with the
// un-normalised atom P w (P^2 = 1/(sqrt(pi) dt), w the raw atom), so
// dJ/dtheta_j = 2 P^2 <s,w> <s, d_j w>, plus -J along ln dt.
__device__ __forceinline__ double obj_prior_from_sums(const double acc[10], double inv_dt, double grad[4]) {
    const double p2 = inv_dt * 0.56418958354775628694807945156077;  // 1/sqrt(pi)
    const double s = acc[0];
    const double J = p2 * s * s;
#pragma unroll
    for (int j = 0; j < 4; ++j) grad[j] = 2.0 * p2 * s * acc[2 + j];
    grad[3] -= J;
    return J;
}

// objective of the refinement: 0 = the residue-based ACT's J, 1 = the prior
// ACT's, 2 = complex atoms' |<g_hat, r>|^2 (the red buffer then holds 13 sums)
// 3 = the residue-based ACT's J with FP32 arithmetic (FP32 residual)
enum { kObjReal = 0, kObjPrior = 1, kObjComplex = 2, kObjReal32 = 3 };

// ---- the refinement's 4-parameter vectors, one component per lane: lane j
// of every quad holds component j = lane & 3 (every quad of the block holds
// the same vector, so control flow stays uniform).  A dot product is the
// quad's sum (x0 + x1) + (x2 + x3), which every lane of the quad computes
// with the same bits (IEEE addition commutes); maxima likewise.
__device__ __forceinline__ int qcomp() { return (int)(threadIdx.x & 3); }

template <int CTRL>
__device__ __forceinline__ double dpp_mov64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double quad_sum(double x) {
    x = x + dpp_mov64<0xB1>(x);     // quad_perm [1,0,3,2]
    return x + dpp_mov64<0x4E>(x);  // quad_perm [2,3,0,1]
}

__device__ __forceinline__ double quad_max(double x) {
    x = fmax(x, dpp_mov64<0xB1>(x));
    return fmax(x, dpp_mov64<0x4E>(x));
}

// component K of the quad's vector, in every lane
template <int K>
__device__ __forceinline__ double quad_get(double x) {
    return dpp_mov64<K | (K << 2) | (K << 4) | (K << 6)>(x);
}

__device__ __forceinline__ double sel4(const double* v, int j) {
    return j == 0 ? v[0] : j == 1 ? v[1] : j == 2 ? v[2] : v[3];
}

// f = -J at theta = theta0 + h u, and this lane's component of df/du
// (theta0, h and u given by this lane's components).
template <int TB, int MODE = kObjReal, typename RT = double>
__device__ __forceinline__ double refine_eval(const RT* r, const GridDev& g, double th0j, double hj, double uj,
                                              double& guj, double* red) {
    static_assert((MODE == kObjReal32) == std::is_same<RT, float>::value, "FP32 residuals go with kObjReal32");
    const double thj = th0j + hj * uj;
    const double th[4] = {quad_get<0>(thj), quad_get<1>(thj), quad_get<2>(thj), quad_get<3>(thj)};
    double gr[4];
    double J;
    if constexpr (MODE == kObjReal32) {
        double acc[10];
        sums_obj32<TB>(r, g.n, g.fs, th, acc, red);
        J = obj_from_sums(acc, gr);
    } else if constexpr (MODE == kObjComplex) {
        double acc[13];
        sums_obj_cplx<TB>(r, g.n, g.fs, th, acc, red);
        J = obj_cplx_from_sums(acc, gr);
    } else {
        double acc[10];
        sums_obj_win<TB>(r, g.n, g.fs, th, acc, red);
        J = MODE == kObjPrior ? obj_prior_from_sums(acc, 1.0 / exp(th[3]), gr) : obj_from_sums(acc, gr);
    }
    guj = -hj * sel4(gr, qcomp());
    return -J;
}

// FP32 objectives (kObjReal32) resolve J and its gradient to about 1e-7
// relative instead of 1e-16: the stopping gradient and the approximate-Wolfe
// tolerance on f follow that working precision.
// The L-BFGS state is per lane (component j): u, the gradient, the direction,
// the box in scaled coordinates, and the 8 newest (s, y) pairs in registers,
// newest first; 1/(s'y) is uniform.
// `red` must hold block_sum_tr_lds(TB, 13) doubles.
template <int TB, int MODE = kObjReal, typename RT = double>
__device__ int refine_block(const RT* __restrict__ r, const GridDev& g, const BoxDev& box,
                            const double th0[4], int steps, double th_out[4], double* J_out,
                            double* red) {
    constexpr double kStopTol = MODE == kObjReal32 ? 1e-6 : 1e-11;
    constexpr double kWolfeF = MODE == kObjReal32 ? 1e-6 : 1e-12;
    const int j = qcomp();
    const double th0j = sel4(th0, j);
    double hj, bloj, bhij;
    int flags = 0;
    {
        double Gd[4];
        if constexpr (MODE == kObjComplex) {
            double acc[13];
            sums_scales_cplx<TB>(g.n, g.fs, th0, acc, red);
            const double q = acc[0];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                Gd[k] = q > 0.0 ? (acc[1 + k] - (acc[5 + k] * acc[5 + k] + acc[9 + k] * acc[9 + k]) / q) / q : 0.0;
        } else {
            double acc[9];
            sums_scales<TB>(g.n, g.fs, th0, acc, red);
            const double q = acc[0];
#pragma unroll
            for (int k = 0; k < 4; ++k) Gd[k] = q > 0.0 ? (acc[5 + k] - acc[1 + k] * acc[1 + k] / q) / q : 0.0;
        }
        const double G = sel4(Gd, j), loj = sel4(box.lo, j), hij = sel4(box.hi, j), stj = sel4(box.step, j);
        if (!(hij > loj) || !(G > 0.0)) {
            hj = 0.0;
        } else {
            const double rr = 1.0 / sqrt(G);
            hj = rr < stj ? rr : stj;
        }
        bloj = hj == 0.0 ? 0.0 : (loj - th0j) / hj;
        bhij = hj == 0.0 ? 0.0 : (hij - th0j) / hj;
    }
    double uj = 0.0, gj;
    double f = refine_eval<TB, MODE, RT>(r, g, th0j, hj, uj, gj, red);
    const double f0 = f;
    double S[8], Y[8], RHO[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) S[t] = Y[t] = RHO[t] = 0.0;
    int nmem = 0;
    double gam = 1.0;  // H0 = gam I: s'y / y'y of the newest pair, formed when it is stored
    for (int it = 0; it < steps; ++it) {
        double pgj = gj;
        if (uj <= bloj && gj > 0.0) pgj = 0.0;
        if (uj >= bhij && gj < 0.0) pgj = 0.0;
        const double pgmax = quad_max(fabs(pgj));
        const double Jc = -f;
        if (pgmax <= kStopTol * (Jc > 1.0 ? Jc : 1.0)) break;
        // two-loop recursion, newest pair first
        double dj = -gj, al[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            al[t] = 0.0;
            if (t < nmem) {
                const double a = RHO[t] * quad_sum(S[t] * dj);
                al[t] = a;
                dj -= a * Y[t];
            }
        }
        if (nmem > 0) dj *= gam;
#pragma unroll
        for (int t = 7; t >= 0; --t) {
            if (t < nmem) {
                const double bb = RHO[t] * quad_sum(Y[t] * dj);
                dj += (al[t] - bb) * S[t];
            }
        }
        if (hj == 0.0) dj = 0.0;
        if (uj <= bloj && dj < 0.0) dj = 0.0;
        if (uj >= bhij && dj > 0.0) dj = 0.0;
        if (quad_sum(gj * dj) >= 0.0) dj = -pgj;
        const double dmax = quad_max(fabs(dj));
        double alpha = nmem > 0 ? 1.0 : (dmax > 1.0 ? 1.0 / dmax : 1.0);
        double unj = uj, gnj = gj, fn = 0.0;
        bool ok = false;
        for (int t = 0; t < 30; ++t) {
            double v = uj + alpha * dj;
            v = v < bloj ? bloj : v;
            v = v > bhij ? bhij : v;
            unj = v;
            fn = refine_eval<TB, MODE, RT>(r, g, th0j, hj, unj, gnj, red);
            const double dec = quad_sum(gj * (unj - uj));
            const double dnew = quad_sum(gnj * (unj - uj));
            const bool armijo = fn <= f + 1e-4 * dec;
            const bool approx_wolfe = fn <= f + kWolfeF * fabs(f) && dnew >= 0.9 * dec && dnew <= -0.8 * dec;
            if (dec < 0.0 && (armijo || approx_wolfe)) {
                ok = true;
                break;
            }
            alpha *= 0.5;
        }
        if (!ok) break;
        const double svj = unj - uj, yvj = gnj - gj;
        const double sy = quad_sum(svj * yvj), yy = quad_sum(yvj * yvj);
        if (sy > 1e-12 * sqrt(quad_sum(svj * svj)) * sqrt(yy)) {
#pragma unroll
            for (int t = 7; t > 0; --t) {
                S[t] = S[t - 1];
                Y[t] = Y[t - 1];
                RHO[t] = RHO[t - 1];
            }
            S[0] = svj;
            Y[0] = yvj;
            RHO[0] = 1.0 / sy;
            gam = sy / yy;
            if (nmem < 8) ++nmem;
        }
        uj = unj;
        gj = gnj;
        f = fn;
    }
    if (-f >= -f0) {
        const double thj = th0j + hj * uj;
        th_out[0] = quad_get<0>(thj);
        th_out[1] = quad_get<1>(thj);
        th_out[2] = quad_get<2>(thj);
        th_out[3] = quad_get<3>(thj);
        *J_out = -f;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) th_out[k] = th0[k];
        *J_out = -f0;
        flags |= ACT_FLAG_REFINE_REJECTED;
    }
    return flags;
}

// --------------------------------------------------------------------------
// select -> refine -> coefficient -> update, one block per channel
// --------------------------------------------------------------------------
constexpr int NTR = 256;            // threads of the refinement kernels at up to two blocks per CU
                                    // (fastest measured; larger batches use 128)
constexpr int NWR = NTR / kWave;

// CPLX: complex atoms (instantiated apart, so that each kernel carries only
// its own refinement: the two together exceed the instruction cache).
// STAGE: the refinement reads the channel's residual from a copy in dynamic
// LDS (n doubles; the launch passes that size) instead of global memory.
template <int TB, bool CPLX, bool STAGE>
__global__ void __launch_bounds__(TB) k_select_refine_update(
    PlanDev P, int k, int order, int steps, double* __restrict__ resid, double* __restrict__ approx,
    double* __restrict__ theta, double* __restrict__ coef, long long* __restrict__ index,
    double* __restrict__ energy, double* __restrict__ gap, int* __restrict__ flags) {
    constexpr int NWB = TB / kWave;
    extern __shared__ double s_dyn[];
    __shared__ double red[block_sum_tr_lds(TB, 13)];
    __shared__ double s_a1[NWB], s_a2[NWB];
    __shared__ unsigned s_i1[NWB];
    // uneven batches: the longest channels take the first blocks, so that each
    // starts at once and shares its compute unit with shorter ones
    const int b = P.by_length ? P.by_length[blockIdx.x] : (int)blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const ChanGeom cg = chan_geom(P.g, b, P.len, P.off);
    const GridDev& G = cg.g;
    double* r = resid + cg.off;
    int fl = flags[b];
    const double eb = P.ebound[b];
    const size_t o = (size_t)b * order + k;
    // the search of this order has drained its tile queue: reset it for the next
    if (blockIdx.x == 0 && threadIdx.x == 0 && P.items) {
        P.items[P.batch + 1] = 0;
        P.items[P.batch + 3] = 0;
    }

    if (fl & (ACT_FLAG_NONFINITE | ACT_FLAG_RAGGED_EMPTY)) {
        if (threadIdx.x == 0) {
            const double nan = __longlong_as_double(0x7ff8000000000000LL);
            for (int j = 0; j < 4; ++j) theta[o * 4 + j] = nan;
            if (CPLX) {
                coef[2 * o] = 0.0;
                coef[2 * o + 1] = 0.0;
            } else {
                coef[o] = 0.0;
            }
            index[o] = -1;
            if (gap) gap[o] = 0.0;
            energy[(size_t)b * (order + 1) + k + 1] = energy[(size_t)b * (order + 1) + k];
        }
        return;
    }

    // arg-max of |p64| over the rescored candidates; ties -> lowest atom index
    double a1 = -1.0, a2 = -1.0;
    unsigned i1 = 0xffffffffu;
    if (eb >= 0.0) {
        const int cnt_raw = P.cand_count[b];
        const int cnt = min(cnt_raw, P.cap);
        if (cnt_raw > P.cap) fl |= ACT_FLAG_CAND_OVERFLOW;
        // SU entries per thread and step requested together (long lists of
        // an uneven batch are mostly entries the rescoring marked NaN)
        constexpr int SU = 8;
        for (int j0 = threadIdx.x; j0 < cnt; j0 += SU * TB) {
            double vv[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int j = j0 + u * TB;
                vv[u] = j < cnt ? P.cand_p64[(size_t)b * P.cap + j] : __longlong_as_double(0x7ff8000000000000LL);
            }
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                if (isnan(vv[u])) continue;
                const double a = fabs(vv[u]);
                const unsigned id = P.cand_idx[(size_t)b * P.cap + j0 + u * TB];
                if (a > a1 || (a == a1 && id < i1)) {
                    a2 = a1;
                    a1 = a;
                    i1 = id;
                } else if (a > a2) {
                    a2 = a;
                }
            }
        }
    }
    // wave then block merge of (a1, i1, a2)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double oa1 = __shfl_xor(a1, off, kWave), oa2 = __shfl_xor(a2, off, kWave);
        const unsigned oi1 = __shfl_xor(i1, off, kWave);
        if (oa1 > a1 || (oa1 == a1 && oi1 < i1)) {
            a2 = fmax(a1, oa2);
            a1 = oa1;
            i1 = oi1;
        } else {
            a2 = fmax(a2, oa1);
        }
    }
    if (lane == 0) {
        s_a1[w] = a1;
        s_a2[w] = a2;
        s_i1[w] = i1;
    }
    __syncthreads();
    a1 = s_a1[0];
    a2 = s_a2[0];
    i1 = s_i1[0];
    for (int q = 1; q < NWB; ++q) {
        const double oa1 = s_a1[q], oa2 = s_a2[q];
        const unsigned oi1 = s_i1[q];
        if (oa1 > a1 || (oa1 == a1 && oi1 < i1)) {
            a2 = fmax(a1, oa2);
            a1 = oa1;
            i1 = oi1;
        } else {
            a2 = fmax(a2, oa1);
        }
    }
    __syncthreads();
    const long long best = (eb >= 0.0 && i1 != 0xffffffffu) ? (long long)i1 : 0;
    double g_gap = 0.0;
    if (eb >= 0.0 && a1 > 0.0) {
        // an atom outside the list has |p| < M - eb (its score was below M - 2 eb);
        // with per-atom bounds, |p| < L (its upper bound was below L)
        const double outside = P.per_atom ? (double)bitsf(P.gmax[b]) : (double)bitsf(P.gmax[b]) - eb;
        const double runner = fmax(a2, outside);
        g_gap = fmax(0.0, (a1 - runner) / a1);
    }

    double th0[4], th[4], J = 0.0;
    grid_theta(G, best, th0);
    BoxDev box = P.box;
    if (G.ragged_div) {
        box.step[0] = cg.box_step0;
        box.lo[0] = cg.box_lo0;
        box.hi[0] = cg.box_hi0;
    }
    if constexpr (STAGE) {  // the residual's LDS copy, read by the refinement (and the complex fit)
        for (int t = threadIdx.x; t < G.n; t += TB) s_dyn[t] = r[t];
        __syncthreads();
    }
    if (steps > 0) {
        if constexpr (STAGE) {
            if constexpr (CPLX)
                fl |= refine_block<TB, kObjComplex>(s_dyn, G, box, th0, steps, th, &J, red);
            else
                fl |= refine_block<TB>(s_dyn, G, box, th0, steps, th, &J, red);
        } else {
            if constexpr (CPLX)
                fl |= refine_block<TB, kObjComplex>(r, G, box, th0, steps, th, &J, red);
            else
                fl |= refine_block<TB>(r, G, box, th0, steps, th, &J, red);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) th[j] = th0[j];
    }

    const double inv_dt = 1.0 / exp(th[3]);
    if constexpr (CPLX) {
        // complex atom: amplitudes (alpha, beta) of u = E cos phi and v = E sin
        // phi by least squares, r -= alpha u + beta v (a pair that is singular
        // to working precision falls back to the fit on u alone).  Both
        // passes run over the atom's support window (E below 2.6e-18 of its
        // peak outside it) with u and v from the chirp walk.
        int k0, k1;
        support_window(G.n, G.fs, th, k0, k1);
        double acc5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        walk_chirp<TB>(k0, k1, G.fs, th, inv_dt, [&](int t, double, double re, double im) {
            double rt;
            if constexpr (STAGE) rt = s_dyn[t];
            else rt = r[t];
            acc5[0] += re * re;
            acc5[1] += im * im;
            acc5[2] += re * im;
            acc5[3] += re * rt;
            acc5[4] += im * rt;
        });
        block_sum<TB, 5>(acc5, red);
        const double uu = acc5[0], vv = acc5[1], uv = acc5[2], ur = acc5[3], vr = acc5[4];
        const double det = uu * vv - uv * uv;
        double al, be;
        if (!(det > 1e-300 * (uu * vv > 0.0 ? uu * vv : 1.0)) || !(uu > 0.0)) {
            al = uu > 0.0 ? ur / uu : 0.0;
            be = 0.0;
        } else {
            al = (vv * ur - uv * vr) / det;
            be = (uu * vr - uv * ur) / det;
        }
        walk_chirp<TB>(k0, k1, G.fs, th, inv_dt, [&](int t, double, double re, double im) {
            const double w = al * re + be * im;
            r[t] = r[t] - w;
            if (approx) approx[cg.off + t] = approx[cg.off + t] + w;
        });
        __syncthreads();
        const double E = refresh_channel<TB>(P, b, r, G.n, red, false);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) theta[o * 4 + j] = th[j];
            coef[2 * o] = al;
            coef[2 * o + 1] = be;
            index[o] = best;
            if (gap) gap[o] = g_gap;
            energy[(size_t)b * (order + 1) + k + 1] = E;
            flags[b] = fl;
        }
        return;
    }

    // unit atom at theta*, coefficient and update (Sec. III-A, Eq. (4)):
    // |w|^2 and <w, r> of the raw atom w in one pass, c = <w, r>/|w|,
    // r -= c w/|w|, over the atom's support window (w below 2.6e-18 of its
    // peak outside it, where the update would not move r beyond rounding), w
    // from the chirp walk.  A staged kernel keeps w in the LDS copy of the
    // residual (the refinement, which read it, has passed its last barrier;
    // each thread reads back only the samples it wrote: the walk's samples of
    // thread i are k0 + i + TB j).
    int k0, k1;
    support_window(G.n, G.fs, th, k0, k1);
    double acc[2] = {0.0, 0.0};
    walk_chirp<TB>(k0, k1, G.fs, th, inv_dt, [&](int t, double, double v, double) {
        if constexpr (STAGE) s_dyn[t] = v;
        acc[0] += v * v;
        acc[1] += v * r[t];
    });
    block_sum<TB, 2>(acc, red);
    const double nrm = sqrt(acc[0]);
    const double inrm = nrm >= 1e-300 ? 1.0 / nrm : 0.0;
    const double ck = acc[1] * inrm;
    if constexpr (STAGE) {
        for (int t = k0 + (int)threadIdx.x; t < k1; t += TB) {
            const double v = s_dyn[t] * inrm;
            r[t] = r[t] - ck * v;
            if (approx) approx[cg.off + t] = approx[cg.off + t] + ck * v;
        }
    } else {
        walk_chirp<TB>(k0, k1, G.fs, th, inv_dt, [&](int t, double, double w, double) {
            const double v = w * inrm;
            r[t] = r[t] - ck * v;
            if (approx) approx[cg.off + t] = approx[cg.off + t] + ck * v;
        });
    }
    __syncthreads();
    const double E = refresh_channel<TB>(P, b, r, G.n, red, false);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) theta[o * 4 + j] = th[j];
        coef[o] = ck;
        index[o] = best;
        if (gap) gap[o] = g_gap;
        energy[(size_t)b * (order + 1) + k + 1] = E;
        flags[b] = fl;
    }
}

// --------------------------------------------------------------------------
// refinement alone, forward/adjoint alone, reconstruction
// --------------------------------------------------------------------------
// STAGE: the pair's residual is read from a copy in dynamic LDS (n values of
// RT; the launch passes that size).
template <int MODE, int TB, typename RT, bool STAGE>
__global__ void __launch_bounds__(TB) k_refine_many(GridDev g, BoxDev box,
                                                     const RT* __restrict__ resid,
                                                     const double* __restrict__ theta0, int steps,
                                                     double* __restrict__ theta,
                                                     double* __restrict__ value,
                                                     int* __restrict__ flags) {
    extern __shared__ double s_dyn[];
    __shared__ double red[block_sum_tr_lds(TB, 13)];
    const int p = blockIdx.x;
    const RT* r = resid + (size_t)p * g.n;
    double th0[4], th[4], J;
#pragma unroll
    for (int j = 0; j < 4; ++j) th0[j] = theta0[p * 4 + j];
    int fl;
    if constexpr (STAGE) {
        RT* sr = reinterpret_cast<RT*>(s_dyn);
        for (int t = threadIdx.x; t < g.n; t += TB) sr[t] = r[t];
        __syncthreads();
        fl = refine_block<TB, MODE, RT>(sr, g, box, th0, steps, th, &J, red);
    } else {
        fl = refine_block<TB, MODE, RT>(r, g, box, th0, steps, th, &J, red);
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) theta[p * 4 + j] = th[j];
        value[p] = J;
        if (flags) flags[p] = fl;
    }
}

__global__ void __launch_bounds__(NT) k_vg_f64(GridDev g, const double* __restrict__ resid,
                                               const double* __restrict__ theta,
                                               double* __restrict__ value,
                                               double* __restrict__ dtheta, double* __restrict__ dr) {
    __shared__ double red[block_sum_lds(NT, 10)];
    const int p = blockIdx.x;
    const double* r = resid + (size_t)p * g.n;
    double th[4], gr[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) th[j] = theta[p * 4 + j];
    const double J = eval_obj<NT>(r, g.n, g.fs, th, gr, red);
    if (threadIdx.x == 0) {
        value[p] = J;
#pragma unroll
        for (int j = 0; j < 4; ++j) dtheta[p * 4 + j] = gr[j];
    }
    if (dr) {
        // dJ/dr = 2 (s/q) g = 2 <r, g_hat> g_hat
        const double inv_dt = 1.0 / exp(th[3]);
        double acc[2] = {0.0, 0.0};
        for (int k = threadIdx.x; k < g.n; k += NT) {
            const double v = atom_sample64(sample_time(k, g.fs), th[0], th[1], th[2], inv_dt);
            acc[0] += r[k] * v;
            acc[1] += v * v;
        }
        block_sum<NT, 2>(acc, red);
        const double f = acc[1] > 0.0 ? 2.0 * acc[0] / acc[1] : 0.0;
        for (int k = threadIdx.x; k < g.n; k += NT)
            dr[(size_t)p * g.n + k] = f * atom_sample64(sample_time(k, g.fs), th[0], th[1], th[2], inv_dt);
    }
}

__global__ void __launch_bounds__(NT) k_vg_f32(GridDev g, const float* __restrict__ resid,
                                               const double* __restrict__ theta,
                                               double* __restrict__ value,
                                               double* __restrict__ dtheta, float* __restrict__ dr) {
    __shared__ double red[block_sum_lds(NT, 10)];
    const int p = blockIdx.x;
    const float* r = resid + (size_t)p * g.n;
    const double tc = theta[p * 4 + 0], fc = theta[p * 4 + 1], c = theta[p * 4 + 2];
    const float inv_dt = (float)(1.0 / exp(theta[p * 4 + 3]));
    const float idt2 = inv_dt * inv_dt;
    const float twopi = 6.2831853071795865f, fcf = (float)fc, cf = (float)c;
    float acc[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) acc[j] = 0.0f;
    for (int k = threadIdx.x; k < g.n; k += NT) {
        float e, co, si, tau;
        atom_terms_f32(sample_time(k, g.fs) - tc, c, fc, inv_dt, e, co, si, tau);
        const float gk = e * co, es = e * si;
        const float d0 = e * (tau * idt2 * co) + twopi * (2.0f * cf * tau + fcf) * es;
        const float d1 = -twopi * tau * es;
        const float d2 = -twopi * tau * tau * es;
        const float d3 = tau * tau * idt2 * gk;
        const float rk = r[k];
        acc[0] += rk * gk;
        acc[1] += gk * gk;
        acc[2] += rk * d0;
        acc[3] += rk * d1;
        acc[4] += rk * d2;
        acc[5] += rk * d3;
        acc[6] += gk * d0;
        acc[7] += gk * d1;
        acc[8] += gk * d2;
        acc[9] += gk * d3;
    }
    // wave sums in FP32, the few cross-wave partials in FP64
    double accd[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) accd[j] = (double)wave_sum(acc[j]);
    {
        const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        if (lane == 0)
            for (int j = 0; j < 10; ++j) red[j * NW + w] = accd[j];
        __syncthreads();
        for (int j = 0; j < 10; ++j) {
            double s = 0.0;
            for (int q = 0; q < NW; ++q) s += red[j * NW + q];
            accd[j] = (double)(float)s;
        }
        __syncthreads();
    }
    const double s = accd[0], q = accd[1];
    const double J = q > 0.0 ? s * s / q : 0.0;
    if (threadIdx.x == 0) {
        value[p] = J;
        for (int j = 0; j < 4; ++j)
            dtheta[p * 4 + j] = q > 0.0 ? 2.0 * s * accd[2 + j] / q - 2.0 * s * s * accd[6 + j] / (q * q) : 0.0;
    }
    if (dr) {
        const float f = q > 0.0 ? (float)(2.0 * s / q) : 0.0f;
        for (int k = threadIdx.x; k < g.n; k += NT) {
            float e, co, si, tau;
            atom_terms_f32(sample_time(k, g.fs) - tc, c, fc, inv_dt, e, co, si, tau);
            dr[(size_t)p * g.n + k] = f * (e * co);
        }
    }
}

__global__ void __launch_bounds__(NT) k_reconstruct(GridDev g0, int order,
                                                    const double* __restrict__ theta,
                                                    const double* __restrict__ coef,
                                                    const int* __restrict__ len,
                                                    const long long* __restrict__ off,
                                                    double* __restrict__ out, int prior, int cplx) {
    __shared__ double red[block_sum_lds(NT, 1)];
    const int b = blockIdx.x;
    const ChanGeom cg = chan_geom(g0, b, len, off);
    const GridDev& g = cg.g;
    double* o = out + cg.off;
    for (int t = threadIdx.x; t < g.n; t += NT) o[t] = 0.0;
    for (int k = 0; k < order; ++k) {
        const double* th = theta + ((size_t)b * order + k) * 4;
        if (isnan(th[0])) continue;
        const double inv_dt = 1.0 / exp(th[3]);
        if (cplx) {  // amplitude pair of the raw parts E cos phi, E sin phi
            const double al = coef[2 * ((size_t)b * order + k)], be = coef[2 * ((size_t)b * order + k) + 1];
            for (int t = threadIdx.x; t < g.n; t += NT) {
                double re, im, e;
                atom_parts64(sample_time(t, g.fs), th[0], th[1], th[2], inv_dt, re, im, e);
                o[t] = o[t] + (al * re + be * im);
            }
            continue;
        }
        const double ck = coef[(size_t)b * order + k];
        double acc[1] = {0.0};
        for (int t = threadIdx.x; t < g.n; t += NT) {
            const double v = atom_sample64(sample_time(t, g.fs), th[0], th[1], th[2], inv_dt);
            acc[0] += v * v;
        }
        block_sum<NT, 1>(acc, red);
        // unit atoms; the prior ACT's atoms keep Eq. (1)'s prefactor instead
        const double nrm = prior ? 1.0 / sqrt(inv_dt * 0.56418958354775628694807945156077) : sqrt(acc[0]);
        if (!(nrm >= 1e-300)) continue;
        for (int t = threadIdx.x; t < g.n; t += NT)
            o[t] = o[t] + ck * (atom_sample64(sample_time(t, g.fs), th[0], th[1], th[2], inv_dt) / nrm);
    }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
act_status launch_init(act_plan_s* p, int batch, double* resid, double* approx, double* energy,
                       int* flags, int order, hipStream_t s) {
    hipLaunchKernelGGL(k_init, dim3(batch), dim3(NT), 0, s, view(p), resid, approx, energy, flags, order);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

act_status launch_to_shadow(act_plan_s* p, int batch, const double* resid, hipStream_t s) {
    hipLaunchKernelGGL(k_to_shadow, dim3(batch), dim3(256), 0, s, view(p), resid);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

act_status launch_overflow_check(act_plan_s* p, int batch, hipStream_t s) {
    hipLaunchKernelGGL(k_overflow, dim3((batch + 63) / 64), dim3(64), 0, s, view(p), batch);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

act_status launch_rescore(act_plan_s* p, int batch, const double* resid, hipStream_t s) {
    // 16 blocks of 4 waves per channel (measured at 64 channels: 8, 16, 32
    // and 128 blocks per channel took 29, 22, 23 and 26 us per BF16 order)
    const int bx = 16;
    hipLaunchKernelGGL(k_rescore, dim3(bx, batch), dim3(256), 0, s, view(p), resid);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

// Whether kernel `kern` with `dyn` bytes of dynamic LDS fits one workgroup.
static bool lds_fits(const void* kern, size_t dyn) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, kern) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.sharedSizeBytes + dyn <= (size_t)device_lds_per_block();
}

act_status launch_select_refine_update(act_plan_s* p, int batch, int k, int order, double* resid,
                                       double* approx, double* theta, double* coef,
                                       long long* index, double* energy, double* gap, int* flags,
                                       hipStream_t s) {
    PlanDev v = view(p);
    v.batch = batch;
    // more than two channels per CU: 128-thread blocks (several per CU keep its
    // FP64 units busy); otherwise NTR threads (each channel's latency sets the
    // time).  The refinement reads the residual from LDS when the longest
    // channel fits.
    const bool small = (long long)batch > 2LL * device_cus();
    const bool cx = p->desc.complex_atoms != 0;
    const size_t dyn = (size_t)p->grid.n * sizeof(double);
    using K = decltype(&k_select_refine_update<NTR, false, false>);
    static const K kerns[2][2][2] = {   // [small][complex][staged]
        {{k_select_refine_update<NTR, false, false>, k_select_refine_update<NTR, false, true>},
         {k_select_refine_update<NTR, true, false>, k_select_refine_update<NTR, true, true>}},
        {{k_select_refine_update<128, false, false>, k_select_refine_update<128, false, true>},
         {k_select_refine_update<128, true, false>, k_select_refine_update<128, true, true>}}};
    const bool stage = p->desc.refine_steps > 0 && lds_fits((const void*)kerns[small][cx][1], dyn);
    hipLaunchKernelGGL(kerns[small][cx][stage], dim3(batch), dim3(small ? 128 : NTR), stage ? dyn : 0, s, v, k,
                       order, p->desc.refine_steps, resid, approx, theta, coef, index, energy, gap, flags);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

template <int MODE, typename RT>
static act_status launch_refine_pairs(act_plan_s* p, int m, const RT* resid, const double* theta0, int steps,
                                      double* theta, double* value, int* flags, hipStream_t s) {
    // more than two pairs per CU: 128-thread blocks, several per CU, so that
    // the CU's FP64 units stay busy; otherwise NTR threads per pair (each
    // pair's own latency sets the time).  The residual is read from LDS when
    // it fits.
    const bool many = (long long)m > 2LL * device_cus();
    const size_t dyn = (size_t)p->grid.n * sizeof(RT);
    using K = decltype(&k_refine_many<MODE, NTR, RT, false>);
    K staged = many ? k_refine_many<MODE, 128, RT, true> : k_refine_many<MODE, NTR, RT, true>;
    K direct = many ? k_refine_many<MODE, 128, RT, false> : k_refine_many<MODE, NTR, RT, false>;
    const bool stage = lds_fits((const void*)staged, dyn);
    hipLaunchKernelGGL(stage ? staged : direct, dim3(m), dim3(many ? 128 : NTR), stage ? dyn : 0, s, p->grid,
                       p->box, resid, theta0, steps, theta, value, flags);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

act_status launch_refine_many(act_plan_s* p, int m, const double* resid, const double* theta0,
                              int steps, double* theta, double* value, int* flags, hipStream_t s) {
    return p->desc.complex_atoms != 0
               ? launch_refine_pairs<kObjComplex, double>(p, m, resid, theta0, steps, theta, value, flags, s)
               : launch_refine_pairs<kObjReal, double>(p, m, resid, theta0, steps, theta, value, flags, s);
}

act_status launch_refine_many_f32(act_plan_s* p, int m, const float* resid, const double* theta0, int steps,
                                  double* theta, double* value, int* flags, hipStream_t s) {
    return launch_refine_pairs<kObjReal32, float>(p, m, resid, theta0, steps, theta, value, flags, s);
}

act_status launch_value_and_grad(act_plan_s* p, int m, int dtype, const void* resid,
                                 const double* theta, double* value, double* dtheta, void* dr,
                                 hipStream_t s) {
    if (dtype == ACT_PREC_F64)
        hipLaunchKernelGGL(k_vg_f64, dim3(m), dim3(NT), 0, s, p->grid, (const double*)resid, theta,
                           value, dtheta, (double*)dr);
    else
        hipLaunchKernelGGL(k_vg_f32, dim3(m), dim3(NT), 0, s, p->grid, (const float*)resid, theta,
                           value, dtheta, (float*)dr);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

act_status launch_reconstruct(act_plan_s* p, int batch, int order, const double* theta,
                              const double* coef, const int* len, const long long* off, double* out,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_reconstruct, dim3(batch), dim3(NT), 0, s, p->grid, order, theta, coef, len, off,
                       out, p->desc.prior_act, p->desc.complex_atoms);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

// --------------------------------------------------------------------------
// The prior ACT (contrast mode, Sec. III-A and Table "Comparison of
// algorithmic properties"): atoms keep Eq. (1)'s prefactor (no unit-norm
// scaling); the search, the refinement and the coefficient all use the
// original signal, and each order repeats them: r_{k+1} = r_k - c g*.
// --------------------------------------------------------------------------
constexpr int kPriorBlocks = 512;  // search blocks per channel

// Exact FP64 scores |<g_i, s>| of every atom (one thread per atom, grid
// stride), arg-max per block with the lowest index on ties.
__global__ void __launch_bounds__(256) k_prior_search(GridDev g, const double* __restrict__ sorig,
                                                      double* __restrict__ part_score,
                                                      long long* __restrict__ part_idx) {
    __shared__ double bs[4];
    __shared__ long long bi[4];
    const int b = blockIdx.y;
    const double* sv = sorig + (size_t)b * g.n;
    double best = -1.0;
    long long bidx = -1;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < g.atoms; i += (long long)gridDim.x * 256) {
        double th[4];
        grid_theta(g, i, th);
        const double inv_dt = 1.0 / exp(th[3]);
        double acc = 0.0;
        for (int k = 0; k < g.n; ++k) acc += atom_sample64(sample_time(k, g.fs), th[0], th[1], th[2], inv_dt) * sv[k];
        const double p = fabs(acc) * sqrt(inv_dt * 0.56418958354775628694807945156077);
        if (p > best) {  // i grows along the thread's sequence: ties keep the lowest
            best = p;
            bidx = i;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const long long oi = __shfl_xor(bidx, o, 64);
        if (ob > best || (ob == best && oi >= 0 && (bidx < 0 || oi < bidx))) {
            best = ob;
            bidx = oi;
        }
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        bs[w] = best;
        bi[w] = bidx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 4; ++q)
            if (bs[q] > bs[0] || (bs[q] == bs[0] && bi[q] >= 0 && (bi[0] < 0 || bi[q] < bi[0]))) {
                bs[0] = bs[q];
                bi[0] = bi[q];
            }
        part_score[(size_t)b * gridDim.x + blockIdx.x] = bs[0];
        part_idx[(size_t)b * gridDim.x + blockIdx.x] = bi[0];
    }
}

__global__ void k_prior_copy(const double* __restrict__ src, double* __restrict__ dst, long long count) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Winner of the search blocks, refinement of J = <s, g>^2 on the original
// signal, c = <g*, s>, and the update of the residual and approximation.
__global__ void __launch_bounds__(NTR) k_prior_select_update(
    PlanDev P, int k, int order, int steps, const double* __restrict__ sorig, int nblk,
    const double* __restrict__ part_score, const long long* __restrict__ part_idx, double* __restrict__ resid,
    double* __restrict__ approx, double* __restrict__ theta, double* __restrict__ coef,
    long long* __restrict__ index, double* __restrict__ energy, double* __restrict__ gap,
    int* __restrict__ flags) {
    __shared__ double red[block_sum_tr_lds(NTR, 13)];
    __shared__ double s_best[NWR];
    __shared__ long long s_idx[NWR];
    const int b = blockIdx.x;
    const GridDev& G = P.g;
    const double* sv = sorig + (size_t)b * G.n;
    double* r = resid + (size_t)b * G.n;
    const size_t o = (size_t)b * order + k;
    int fl = flags[b];
    if (fl & ACT_FLAG_NONFINITE) {
        if (threadIdx.x == 0) {
            const double nan = __longlong_as_double(0x7ff8000000000000LL);
            for (int j = 0; j < 4; ++j) theta[o * 4 + j] = nan;
            coef[o] = 0.0;
            index[o] = -1;
            if (gap) gap[o] = 0.0;
            energy[(size_t)b * (order + 1) + k + 1] = energy[(size_t)b * (order + 1) + k];
        }
        return;
    }
    double best = -1.0;
    long long bidx = -1;
    for (int j = threadIdx.x; j < nblk; j += NTR) {
        const double v = part_score[(size_t)b * nblk + j];
        const long long id = part_idx[(size_t)b * nblk + j];
        if (id >= 0 && (v > best || (v == best && id < bidx))) {
            best = v;
            bidx = id;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, kWave);
        const long long oi = __shfl_xor(bidx, off, kWave);
        if (oi >= 0 && (ob > best || (ob == best && (bidx < 0 || oi < bidx)))) {
            best = ob;
            bidx = oi;
        }
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s_best[w] = best;
        s_idx[w] = bidx;
    }
    __syncthreads();
    best = s_best[0];
    bidx = s_idx[0];
    for (int q = 1; q < NWR; ++q)
        if (s_idx[q] >= 0 && (s_best[q] > best || (s_best[q] == best && (bidx < 0 || s_idx[q] < bidx)))) {
            best = s_best[q];
            bidx = s_idx[q];
        }
    __syncthreads();
    if (bidx < 0) bidx = 0;

    double th0[4], th[4], J = 0.0;
    grid_theta(G, bidx, th0);
    if (steps > 0) {
        fl |= refine_block<NTR, kObjPrior>(sv, G, P.box, th0, steps, th, &J, red);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) th[j] = th0[j];
    }
    const double inv_dt = 1.0 / exp(th[3]);
    const double pref = sqrt(inv_dt * 0.56418958354775628694807945156077);
    double acc[1] = {0.0};
    for (int t = threadIdx.x; t < G.n; t += NTR)
        acc[0] += pref * atom_sample64(sample_time(t, G.fs), th[0], th[1], th[2], inv_dt) * sv[t];
    block_sum<NTR, 1>(acc, red);
    const double ck = acc[0];
    acc[0] = 0.0;
    for (int t = threadIdx.x; t < G.n; t += NTR) {
        const double v = pref * atom_sample64(sample_time(t, G.fs), th[0], th[1], th[2], inv_dt);
        const double rn = r[t] - ck * v;
        r[t] = rn;
        if (approx) approx[(size_t)b * G.n + t] += ck * v;
        acc[0] += rn * rn;
    }
    block_sum<NTR, 1>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) theta[o * 4 + j] = th[j];
        coef[o] = ck;
        index[o] = bidx;
        if (gap) gap[o] = 0.0;
        energy[(size_t)b * (order + 1) + k + 1] = acc[0];
        flags[b] = fl;
    }
}

act_status launch_prior_init(act_plan_s* p, int batch, const double* resid, hipStream_t s) {
    const long long count = (long long)batch * p->n;
    hipLaunchKernelGGL(k_prior_copy, dim3((unsigned)std::min<long long>((count + 255) / 256, 4096)), dim3(256), 0,
                       s, resid, p->prior_s, count);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

act_status launch_prior_order(act_plan_s* p, int batch, int k, int order, double* resid, double* approx,
                              double* theta, double* coef, long long* index, double* energy, double* gap,
                              int* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_prior_search, dim3(kPriorBlocks, batch), dim3(256), 0, s, p->grid, p->prior_s,
                       p->prior_part, p->prior_pidx);
    ACT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_prior_select_update, dim3(batch), dim3(NTR), 0, s, view(p), k, order,
                       p->desc.refine_steps, p->prior_s, kPriorBlocks, p->prior_part, p->prior_pidx, resid, approx,
                       theta, coef, index, energy, gap, flags);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

size_t prior_workspace_blocks() { return kPriorBlocks; }

// --------------------------------------------------------------------------
// LEM-inspired hierarchical coarse-to-fine search (Sec. VII): one workgroup
// per channel runs every stage of one order on the device (LHS candidates,
// pooled top-k, local families per level, refinement, coefficient, update).
// --------------------------------------------------------------------------
struct LemDev {
    int samples, levels, topk, cap;
    int radius[4];
    double step[8][4];
};

// LHS sample x snapped to the level-0 grid anchored at lo (RN products and
// sums, no contraction, so candidates are bit-identical to a plain FP64 run)
__device__ __forceinline__ double lem_snap(double x, double lo, double hi, double st) {
    if (!(hi > lo) || !(st > 0.0)) return lo;
    double v = __dadd_rn(lo, __dmul_rn(floor(__dadd_rn(__ddiv_rn(__dadd_rn(x, -lo), st), 0.5)), st));
    if (v > hi) v = __dadd_rn(lo, __dmul_rn(floor(__ddiv_rn(__dadd_rn(hi, -lo), st)), st));
    return v < lo ? lo : v;
}

// Scores <g/|g|, r> of candidates [0, m) (one thread per candidate); a
// candidate marked invalid (first parameter NaN) scores NaN.
__device__ void lem_score_all(const GridDev& g, const double* r, const double* cand, double* sc, int m) {
    for (int j = threadIdx.x; j < m; j += NTR) {
        const double* th = cand + 4 * (size_t)j;
        if (isnan(th[0])) {
            sc[j] = __longlong_as_double(0x7ff8000000000000LL);
            continue;
        }
        const double inv_dt = 1.0 / exp(th[3]);
        double s = 0.0, q = 0.0;
        for (int k = 0; k < g.n; ++k) {
            const double v = atom_sample64(sample_time(k, g.fs), th[0], th[1], th[2], inv_dt);
            s += v * r[k];
            q += v * v;
        }
        sc[j] = q > 0.0 ? s / sqrt(q) : 0.0;
    }
}

// Top-k distinct candidates by |score| (ties: the earlier candidate), by one
// thread into kept[topk][4]; returns the count.
__device__ int lem_topk(const double* cand, const double* sc, int m, int k, double (*kept)[4], char* used) {
    for (int j = 0; j < m; ++j) used[j] = 0;
    int nk = 0;
    while (nk < k) {
        int best = -1;
        for (int j = 0; j < m; ++j)
            if (!used[j] && !isnan(sc[j]) && (best < 0 || fabs(sc[j]) > fabs(sc[best]))) best = j;
        if (best < 0) break;
        used[best] = 1;
        const double* c = cand + 4 * (size_t)best;
        bool dup = false;
        for (int a = 0; a < nk; ++a)
            if (kept[a][0] == c[0] && kept[a][1] == c[1] && kept[a][2] == c[2] && kept[a][3] == c[3]) dup = true;
        if (dup) continue;
        for (int d = 0; d < 4; ++d) kept[nk][d] = c[d];
        ++nk;
    }
    return nk;
}

__global__ void __launch_bounds__(NTR) k_lem_order(PlanDev P, LemDev cfg, int k, int order, int steps,
                                                   const double* __restrict__ lhs, double* __restrict__ cand_ws,
                                                   double* __restrict__ score_ws, char* __restrict__ used_ws,
                                                   double* __restrict__ resid, double* __restrict__ approx,
                                                   double* __restrict__ theta, double* __restrict__ coef,
                                                   double* __restrict__ energy, int* __restrict__ flags) {
    __shared__ double red[block_sum_tr_lds(NTR, 13)];
    __shared__ double kept[16][4];
    __shared__ int s_nk;
    const int b = blockIdx.x;
    const GridDev& G = P.g;
    double* r = resid + (size_t)b * G.n;
    const size_t o = (size_t)b * order + k;
    int fl = flags[b];
    if (fl & ACT_FLAG_NONFINITE) {
        if (threadIdx.x == 0) {
            const double nan = __longlong_as_double(0x7ff8000000000000LL);
            for (int j = 0; j < 4; ++j) theta[o * 4 + j] = nan;
            coef[o] = 0.0;
            energy[(size_t)b * (order + 1) + k + 1] = energy[(size_t)b * (order + 1) + k];
        }
        return;
    }
    double* cand = cand_ws + (size_t)b * cfg.cap * 4;
    double* sc = score_ws + (size_t)b * cfg.cap;
    char* used = used_ws + (size_t)b * cfg.cap;
    const double* lo = P.box.lo;
    const double* hi = P.box.hi;
    // level 0: Latin-hypercube samples snapped to the coarsest steps
    const double* u = lhs + ((size_t)b * order + k) * cfg.samples * 4;
    for (int j = threadIdx.x; j < cfg.samples; j += NTR)
        for (int d = 0; d < 4; ++d)
            cand[4 * (size_t)j + d] =
                lem_snap(__dadd_rn(lo[d], __dmul_rn(u[4 * (size_t)j + d], __dadd_rn(hi[d], -lo[d]))), lo[d], hi[d],
                         cfg.step[0][d]);
    __syncthreads();
    lem_score_all(G, r, cand, sc, cfg.samples);
    __syncthreads();
    if (threadIdx.x == 0) s_nk = lem_topk(cand, sc, cfg.samples, cfg.topk, kept, used);
    __syncthreads();
    int fam = 1;
    for (int d = 0; d < 4; ++d) fam *= 2 * cfg.radius[d] + 1;
    for (int lv = 1; lv <= cfg.levels; ++lv) {
        const int nk = s_nk, m = nk * fam;
        // families in parent order, offsets lexicographic (ln dt fastest)
        for (int q = threadIdx.x; q < m; q += NTR) {
            const int a = q / fam;
            int f = q % fam;
            int ii[4];
            for (int d = 3; d >= 0; --d) {
                const int w = 2 * cfg.radius[d] + 1;
                ii[d] = f % w - cfg.radius[d];
                f /= w;
            }
            double* c = cand + 4 * (size_t)q;
            bool in = true;
            for (int d = 0; d < 4; ++d) {
                c[d] = __dadd_rn(kept[a][d], __dmul_rn((double)ii[d], cfg.step[lv][d]));
                if (c[d] < lo[d] || c[d] > hi[d]) in = false;
            }
            if (!in) c[0] = __longlong_as_double(0x7ff8000000000000LL);
        }
        __syncthreads();
        lem_score_all(G, r, cand, sc, m);
        __syncthreads();
        if (threadIdx.x == 0) s_nk = lem_topk(cand, sc, m, cfg.topk, kept, used);
        __syncthreads();
    }
    double th0[4], th[4], J = 0.0;
    for (int d = 0; d < 4; ++d) th0[d] = kept[0][d];
    BoxDev box = P.box;
    for (int d = 0; d < 4; ++d) box.step[d] = cfg.step[cfg.levels][d];
    if (steps > 0) {
        fl |= refine_block<NTR>(r, G, box, th0, steps, th, &J, red);
    } else {
        for (int d = 0; d < 4; ++d) th[d] = th0[d];
    }
    // unit atom at theta*, coefficient and update (Sec. III-A, Eq. (4))
    const double inv_dt = 1.0 / exp(th[3]);
    double acc[1] = {0.0};
    for (int t = threadIdx.x; t < G.n; t += NTR) {
        const double v = atom_sample64(sample_time(t, G.fs), th[0], th[1], th[2], inv_dt);
        acc[0] += v * v;
    }
    block_sum<NTR, 1>(acc, red);
    const double nrm = sqrt(acc[0]);
    const bool ok = nrm >= 1e-300;
    acc[0] = 0.0;
    for (int t = threadIdx.x; t < G.n; t += NTR) {
        const double v = ok ? atom_sample64(sample_time(t, G.fs), th[0], th[1], th[2], inv_dt) / nrm : 0.0;
        acc[0] += v * r[t];
    }
    block_sum<NTR, 1>(acc, red);
    const double ck = acc[0];
    acc[0] = 0.0;
    for (int t = threadIdx.x; t < G.n; t += NTR) {
        const double v = ok ? atom_sample64(sample_time(t, G.fs), th[0], th[1], th[2], inv_dt) / nrm : 0.0;
        const double rn = r[t] - ck * v;
        r[t] = rn;
        if (approx) approx[(size_t)b * G.n + t] += ck * v;
        acc[0] += rn * rn;
    }
    block_sum<NTR, 1>(acc, red);
    if (threadIdx.x == 0) {
        for (int d = 0; d < 4; ++d) theta[o * 4 + d] = th[d];
        coef[o] = ck;
        energy[(size_t)b * (order + 1) + k + 1] = acc[0];
        flags[b] = fl;
    }
}

act_status launch_lem_order(act_plan_s* p, const act_lem_desc* cfg, int cap, double* cand_ws, double* score_ws,
                            char* used_ws, int batch, int k, int order, const double* lhs, double* resid,
                            double* approx, double* theta, double* coef, double* energy, int* flags,
                            hipStream_t s) {
    LemDev d;
    d.samples = cfg->samples;
    d.levels = cfg->levels;
    d.topk = cfg->topk;
    d.cap = cap;
    for (int a = 0; a < 4; ++a) d.radius[a] = cfg->radius[a];
    for (int l = 0; l < 8; ++l)
        for (int a = 0; a < 4; ++a) d.step[l][a] = cfg->step[l][a];
    hipLaunchKernelGGL(k_lem_order, dim3(batch), dim3(NTR), 0, s, view(p), d, k, order, p->desc.refine_steps, lhs,
                       cand_ws, score_ws, used_ws, resid, approx, theta, coef, energy, flags);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

}  // namespace act
