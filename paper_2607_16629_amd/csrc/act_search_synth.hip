// act_search_synth.hip -- coarse search with the dictionary synthesised on the
// device from shift-invariant factor tables (no HBM atom table).
//
// With time centres on integer samples t_c = m/fs, every atom of Eq. (1)
// (real part) factors through the angle-sum identity:
//   g(n) = E(d) cos(2 pi c tau^2 + 2 pi f_c tau)
//        = U_cl(d) C_fc(d) - V_cl(d) S_fc(d),   d = n - m, tau = d/fs,
//   U_cl = E cos(2 pi c tau^2), V_cl = E sin(2 pi c tau^2)  (cl = (c, logdt)),
//   C_fc = cos(2 pi f_c tau),   S_fc = sin(2 pi f_c tau).
// For one time centre the scores of all (f_c, cl) atoms are therefore one
// dense product with the carrier folded into the B operand:
//   P[cl][fc] = sum_n U_cl(n-m) (C_fc(n-m) r(n)) - V_cl(n-m) (S_fc(n-m) r(n)),
// i.e. A = [U | V] (rows cl), B = [C.r ; -S.r] (columns fc), K = 2N.  The
// tables hold only (n_c n_ld + n_fc) x 2N values, FP64-evaluated at plan time.
// The matrix cores run 2x the dense correlation's multiply-adds, with no
// per-element synthesis in the inner loop.
//
// FP32 form (this file): v_mfma_f32_32x32x2_f32, FP32 operands.  Workgroup =
// 4 waves = 128 cl rows x 64 f_c columns of one time centre; the B operand of a
// 128-sample stage is formed once per workgroup in LDS (64 KiB).  Within an
// MFMA the two k-slots carry samples j and 8+j of a 16-sample group, so every
// lane reads 8 contiguous values of A and of B.  Each stage is accumulated
// into fresh registers and then added to the total, so an FP32 score is a
// chain of at most 128 + N/128 roundings (certified margin).
//
// Complex atoms E exp(i phi) need both parts of the same product: with the
// B operand [C r ; -S r] unchanged, <r, E sin phi> = sum V (C r) + (-U)(-S r),
// a second accumulator fed by [V | -U]; the score is sqrt(a^2 + b^2) / |E|.
#include <type_traits>

#include "act_emit.h"

namespace act {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int SY_STAGE = 128;   // samples per LDS stage
constexpr int SY_ROWS = 128;    // cl rows per workgroup (32 per wave)
constexpr int SY_COLS = 64;     // f_c columns per workgroup

__device__ __forceinline__ int mfma32_row_s(int v, int lane) {
    return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}

struct SynthDev {
    const float* U;     // [n_cl][W] factor tables, W = 2 n_pad, column e = d + n_pad
    const float* V;
    const float* C;     // [n_fc][W]
    const float* S;
    const float* inv_norm;  // [atoms] FP32 copy of 1/|g| (plain plans)
    const int* tc_shift;    // [n_tc] integer sample of each time centre (plain plans)
    const double* lag_energy;  // [n_fc][n_cl][W] prefix sums of g(d)^2 (ragged plans)
    int W, n_cl;
};

// One workgroup tile: time centre tc (integer shift m) of channel b, 128 cl
// rows, 64 f_c columns; scores = P * 1/|g| (1/|g| read from inv_norm, or from
// the prefix sums of g^2 of a ragged channel), fused certified emission.
struct TileArgs {
    int b, tc, m, clb, fcc, n, n_pad_ch;  // n: samples of the channel
};

template <bool RERUN, bool DUMP, bool RAGGED, bool CPLX = false>
__device__ void synth_tile(const GridDev& g, const SynthDev& sy, const float* __restrict__ r,
                           const SearchCtl& ctl, const TileArgs& ta, f32x4 (*bl)[SY_COLS][SY_STAGE / 4 + 1],
                           float* s_red, float* s_M) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = ta.b, tc = ta.tc, m = ta.m, clb = ta.clb, fcc = ta.fcc;
    const int n_fc = g.cnt[1];
    {
        const int fc0 = fcc * SY_COLS;
        const int cl = clb * SY_ROWS + w * 32 + (lane & 31);   // this lane's A row
        const bool row_ok = cl < sy.n_cl;
        const float* urow = sy.U + (size_t)(row_ok ? cl : 0) * sy.W;
        const float* vrow = sy.V + (size_t)(row_ok ? cl : 0) * sy.W;
        const int h = lane >> 5;
        static_assert(!(CPLX && RAGGED), "complex atoms: plain plans only");
        f32x16 tot[2], acc[2], totb[2], accb[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                tot[cb][v] = 0.0f;
                if constexpr (CPLX) totb[cb][v] = 0.0f;
            }

        // A operands of one 16-sample group: rows past the dictionary read row
        // 0 (their scores are masked in the epilogue), so the loads need no branch
        auto load_a = [&](f32x4 (&a)[4], int n0, int s16) {
            const int e0 = n0 + s16 + 8 * h - m + g.n_pad;  // factor column of this lane's 8 samples
            a[0] = *reinterpret_cast<const f32x4*>(urow + e0);
            a[1] = *reinterpret_cast<const f32x4*>(urow + e0 + 4);
            a[2] = *reinterpret_cast<const f32x4*>(vrow + e0);
            a[3] = *reinterpret_cast<const f32x4*>(vrow + e0 + 4);
        };
        for (int n0 = 0; n0 < ta.n_pad_ch; n0 += SY_STAGE) {
            f32x4 abuf[2][4];
            load_a(abuf[0], n0, 0);  // in flight while B is formed
            __builtin_amdgcn_sched_barrier(0);
            __syncthreads();
            // B operand of this stage: C_fc(n-m) r(n) and -S_fc(n-m) r(n)
            for (int q = threadIdx.x; q < SY_COLS * SY_STAGE; q += 256) {
                const int fcl = q / SY_STAGE, sn = q % SY_STAGE;
                const int fc = fc0 + fcl, n = n0 + sn;
                float cv = 0.0f, sv = 0.0f;
                if (fc < n_fc && n < ta.n) {
                    const float rv = r[n];
                    const int e = n - m + g.n_pad;
                    cv = sy.C[(size_t)fc * sy.W + e] * rv;
                    sv = -(sy.S[(size_t)fc * sy.W + e] * rv);
                }
                reinterpret_cast<float*>(&bl[0][fcl][0])[sn] = cv;
                reinterpret_cast<float*>(&bl[1][fcl][0])[sn] = sv;
            }
            __syncthreads();
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    acc[cb][v] = 0.0f;
                    if constexpr (CPLX) accb[cb][v] = 0.0f;
                }
            // groups of 16 samples, the next group's A loaded while this one runs
            // (the scheduling barriers keep the loads ahead of the MFMAs)
#pragma unroll
            for (int s16 = 0; s16 < SY_STAGE; s16 += 16) {
                if (s16 + 16 < SY_STAGE) load_a(abuf[((s16 >> 4) + 1) & 1], n0, s16 + 16);
                __builtin_amdgcn_sched_barrier(0);
                const f32x4 ua = abuf[(s16 >> 4) & 1][0], ub = abuf[(s16 >> 4) & 1][1];
                const f32x4 va = abuf[(s16 >> 4) & 1][2], vb = abuf[(s16 >> 4) & 1][3];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const int col = cb * 32 + (lane & 31);
                    const f32x4 ca = bl[0][col][(s16 + 8 * h) / 4], cc = bl[0][col][(s16 + 8 * h) / 4 + 1];
                    const f32x4 sa = bl[1][col][(s16 + 8 * h) / 4], sc = bl[1][col][(s16 + 8 * h) / 4 + 1];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ua[j], ca[j], acc[cb], 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ub[j], cc[j], acc[cb], 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(va[j], sa[j], acc[cb], 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(vb[j], sc[j], acc[cb], 0, 0, 0);
                        if constexpr (CPLX) {
                            accb[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(va[j], ca[j], accb[cb], 0, 0, 0);
                            accb[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(vb[j], cc[j], accb[cb], 0, 0, 0);
                            accb[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ua[j], sa[j], accb[cb], 0, 0, 0);
                            accb[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ub[j], sc[j], accb[cb], 0, 0, 0);
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    tot[cb][v] += acc[cb][v];
                    if constexpr (CPLX) totb[cb][v] += accb[cb][v];
                }
        }
        if constexpr (CPLX) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    tot[cb][v] = sqrtf(tot[cb][v] * tot[cb][v] + totb[cb][v] * totb[cb][v]);
        }

        // ---- epilogue: rows = cl (A rows), columns = f_c; scale by 1/|g|
        const int clw = clb * SY_ROWS + w * 32;
        float lmax = 0.0f;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int fc = fc0 + cb * 32 + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int c2 = clw + mfma32_row_s(v, lane);
                const bool ok = fc < n_fc && c2 < sy.n_cl;
                const long long idx = ok ? ((long long)tc * n_fc + fc) * sy.n_cl + c2 : 0;
                float inv = 0.0f;
                if (ok) {
                    if (RAGGED) {
                        // |g|^2 over samples 0..n-1 of the channel = a window of the
                        // prefix sums of the squared lag atom (lags d = n - m)
                        const double* q = sy.lag_energy + ((size_t)fc * sy.n_cl + c2) * sy.W;
                        const int e_lo = g.n_pad - m, e_hi = ta.n - 1 - m + g.n_pad;
                        const double e2 = q[e_hi] - (e_lo > 0 ? q[e_lo - 1] : 0.0);
                        inv = e2 > 0.0 ? (float)(1.0 / sqrt(e2)) : 0.0f;
                    } else {
                        inv = sy.inv_norm[idx];
                    }
                }
                tot[cb][v] = ok ? tot[cb][v] * inv : 0.0f;
                lmax = fmaxf(lmax, fabsf(tot[cb][v]));
                if (DUMP && ok && idx >= ctl.dump_begin && idx < ctl.dump_begin + ctl.dump_count)
                    ctl.dump[(size_t)b * ctl.dump_count + (idx - ctl.dump_begin)] = tot[cb][v];
            }
        }
        if (DUMP) return;
        lmax = wave_max(lmax);
        if (lane == 0) s_red[w] = lmax;
        __syncthreads();
        if (threadIdx.x == 0) {
            const float wm = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
            const float cur = load_gmax(&ctl.gmax[b]);
            float M = cur;
            if (!RERUN && wm > cur) M = fmaxf(bitsf(atomicMax(&ctl.gmax[b], fbits(wm))), wm);
            *s_M = M;
        }
        __syncthreads();
        const double Td = (double)*s_M - 2.0 * ctl.ebound[b];
        float T = (float)Td;
        if ((double)T > Td) T = nextafterf(T, -INFINITY);
        if (lmax >= T) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int fc = fc0 + cb * 32 + (lane & 31);
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int c2 = clw + mfma32_row_s(v, lane);
                    if (fc < n_fc && c2 < sy.n_cl && fabsf(tot[cb][v]) >= T) {
                        const int j = atomicAdd(&ctl.cand_count[b], 1);
                        if (j < ctl.cap) {
                            ctl.cand_idx[(size_t)b * ctl.cap + j] =
                                (unsigned)(((long long)tc * n_fc + fc) * sy.n_cl + c2);
                            ctl.cand_score[(size_t)b * ctl.cap + j] = tot[cb][v];
                        }
                    }
                }
            }
        }
        __syncthreads();  // s_M is rewritten by the next tile
    }
}

// plain plans: grid x = (tc, cl block, f_c chunk) tiles, y = channel
template <bool RERUN, bool DUMP, bool CPLX>
__global__ void __launch_bounds__(256) k_search_synth_f32(GridDev g, SynthDev sy,
                                                          const float* __restrict__ shadow,
                                                          SearchCtl ctl, int n_clb, int n_fcc) {
    __shared__ f32x4 bl[2][SY_COLS][SY_STAGE / 4 + 1];
    __shared__ float s_red[4];
    __shared__ float s_M;
    const int b = blockIdx.y;
    if (RERUN && ctl.need_rerun[b] == 0) return;
    if (!DUMP && ctl.ebound[b] < 0.0) return;
    const long long tiles = (long long)g.cnt[0] * n_clb * n_fcc;
    const float* r = shadow + (size_t)b * g.n_pad;
    for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
        TileArgs ta;
        ta.b = b;
        ta.fcc = (int)(t % n_fcc);
        ta.clb = (int)((t / n_fcc) % n_clb);
        ta.tc = (int)(t / ((long long)n_fcc * n_clb));
        ta.m = sy.tc_shift[ta.tc];
        ta.n = g.n;
        ta.n_pad_ch = g.n_pad;
        synth_tile<RERUN, DUMP, false, CPLX>(g, sy, r, ctl, ta, bl, s_red, &s_M);
    }
}

// ragged plans: a persistent grid takes (channel, tc, cl block, f_c chunk)
// tiles from a queue (items[b] = first tile of channel b, items[B] = total,
// counters after it); every channel has floor(len/div) time centres.
template <bool RERUN>
__global__ void __launch_bounds__(256) k_search_synth_f32_ragged(GridDev g, SynthDev sy,
                                                                 const float* __restrict__ shadow,
                                                                 SearchCtl ctl, int batch, int n_clb,
                                                                 int n_fcc, int* __restrict__ items) {
    __shared__ f32x4 bl[2][SY_COLS][SY_STAGE / 4 + 1];
    __shared__ float s_red[4];
    __shared__ float s_M;
    __shared__ long long s_item;
    if (RERUN && items[batch + 3] == 0) return;  // no channel overflowed
    const long long total = items[batch];
    int* counter = items + batch + 1 + (RERUN ? 1 : 0);
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const long long it = s_item;
        if (it >= total) break;
        int lo = 0, hi = batch - 1;  // channel: last b with items[b] <= it
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid] <= it) lo = mid; else hi = mid - 1;
        }
        const int b = lo;
        if (RERUN && ctl.need_rerun[b] == 0) continue;
        if (ctl.ebound[b] < 0.0) continue;
        const long long t = it - items[b];
        TileArgs ta;
        ta.b = b;
        ta.fcc = (int)(t % n_fcc);
        ta.clb = (int)((t / n_fcc) % n_clb);
        ta.tc = (int)(t / ((long long)n_fcc * n_clb));
        ta.m = ta.tc * g.ragged_div;
        ta.n = ctl.len[b];  // in range: a channel with tiles has 0 < len <= n_samples
        ta.n_pad_ch = (ta.n + SY_STAGE - 1) / SY_STAGE * SY_STAGE;
        synth_tile<RERUN, false, true>(g, sy, shadow + (size_t)b * g.n_pad, ctl, ta, bl, s_red, &s_M);
    }
}

// Tile prefix of a ragged batch (one thread), and the queue counters reset.
__global__ void k_ragged_items(const int* __restrict__ len, int batch, int n_max, int div, int n_clb,
                               int n_fcc, int* __restrict__ items) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int acc = 0;
    for (int b = 0; b < batch; ++b) {
        items[b] = acc;
        const int n = (len[b] < 0 || len[b] > n_max) ? 0 : len[b];
        acc += (n / div) * n_clb * n_fcc;
    }
    items[batch] = acc;
    items[batch + 1] = 0;
    items[batch + 2] = 0;
    items[batch + 3] = 0;
}

// FP32 accumulation chain of one synthesised score: 2 roundings per MFMA over a
// stage (2 * SY_STAGE) plus one per stage added to the total.
int synth_chain_length(int n_pad) { return 2 * SY_STAGE + n_pad / SY_STAGE + 2; }

act_status launch_search_synth_f32(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s) {
    SynthDev sy{(const float*)p->fac_u, (const float*)p->fac_v, (const float*)p->fac_c,
                (const float*)p->fac_s, p->inv_norm32, p->tc_shift, p->lag_energy, p->fac_w, p->n_cl};
    const int n_clb = (p->n_cl + SY_ROWS - 1) / SY_ROWS;
    const int n_fcc = (p->grid.cnt[1] + SY_COLS - 1) / SY_COLS;
    const float* sh = (const float*)p->shadow;
    if (p->desc.ragged) {
        const unsigned blocks = (unsigned)grid_cap(p, 2);
        if (ctl.pass)
            hipLaunchKernelGGL((k_search_synth_f32_ragged<true>), dim3(blocks), dim3(256), 0, s, p->grid, sy,
                               sh, ctl, batch, n_clb, n_fcc, p->items);
        else
            hipLaunchKernelGGL((k_search_synth_f32_ragged<false>), dim3(blocks), dim3(256), 0, s, p->grid, sy,
                               sh, ctl, batch, n_clb, n_fcc, p->items);
        ACT_HIP(hipGetLastError());
        return ACT_OK;
    }
    const long long tiles = (long long)p->grid.cnt[0] * n_clb * n_fcc;
    long long blocks = tiles;
    const long long cap = grid_cap(p, 4);
    blocks = blocks < cap ? blocks : cap;
    auto go = [&](auto cplx) {
        constexpr bool C = decltype(cplx)::value;
        if (ctl.dump)
            hipLaunchKernelGGL((k_search_synth_f32<false, true, C>), dim3((unsigned)blocks, batch), dim3(256), 0, s,
                               p->grid, sy, sh, ctl, n_clb, n_fcc);
        else if (ctl.pass)
            hipLaunchKernelGGL((k_search_synth_f32<true, false, C>), dim3((unsigned)blocks, batch), dim3(256), 0, s,
                               p->grid, sy, sh, ctl, n_clb, n_fcc);
        else
            hipLaunchKernelGGL((k_search_synth_f32<false, false, C>), dim3((unsigned)blocks, batch), dim3(256), 0,
                               s, p->grid, sy, sh, ctl, n_clb, n_fcc);
    };
    if (p->desc.complex_atoms)
        go(std::true_type{});
    else
        go(std::false_type{});
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

act_status launch_ragged_items(act_plan_s* p, int batch, hipStream_t s) {
    if (p->desc.ragged && p->desc.dict == ACT_DICT_LAG) return launch_lag_ragged_prep(p, batch, s);
    if (!(p->desc.ragged && p->items)) return ACT_OK;
    if (p->desc.prec == ACT_PREC_F16) return launch_h16_ragged_prep(p, batch, s);
    const int n_clb = (p->n_cl + SY_ROWS - 1) / SY_ROWS;
    const int n_fcc = (p->grid.cnt[1] + SY_COLS - 1) / SY_COLS;
    hipLaunchKernelGGL(k_ragged_items, dim3(1), dim3(64), 0, s, p->call_len, batch, p->grid.n,
                       p->desc.ragged_tc_div, n_clb, n_fcc, p->items);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

}  // namespace act
