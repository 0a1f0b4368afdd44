// act_search_lag.hip -- coarse search as one dense FP16 matrix product over a
// lag-indexed table of the atoms of a single time centre.
//
// With time centres on integer samples m, the real atom of Eq. (1) at (m, q),
// q = (f_c, c, log dt), is the atom of lag 0 shifted by m:
//   <g_{m,q}, r> = sum_d G_q(d) r(d + m),
//   G_q(d) = E(d) cos(2 pi (c tau^2 + f_c tau)),  tau = d / fs.
// The scores of every (channel b, time centre m) row and every column q are
// therefore one product with K = the lags:
//   P[(b, m)][q] = sum_d R[(b, m)][d] G[d][q],   R[(b, m)][d] = r_b(d + m)
// (zero outside the signal).  The matrix cores execute the dense
// correlation's multiply-adds (plus a stage's span of lags), not the factored
// synthesis' two products per sample.
//
// G: FP16 (RNE of the FP64 value), columns padded to a multiple of 256, lags
// e = d + N_pad in [0, 2 N_pad), pre-swizzled in MFMA B-operand order: for 32
// columns and a k-step of 16 lags the 64 lanes' 16-byte operands are one
// contiguous KiB, so every wave streams its B fragments straight from L2.
// R: per 128-lag stage, 128 rows x 128 lags in LDS (two buffers), each row
// read from the FP16 search copy of its channel.
// Workgroup = 4 waves; tile = 128 rows x (128 or 256) columns; wave w owns
// every row (4 row blocks of 32) and 32 or 64 columns.  Tiles are dealt to the
// 8 XCDs in contiguous ranges with the row blocks of one column block adjacent,
// so the concurrent tiles of an XCD share their G columns in its L2.
//
// Certified emission with a uniform bound per channel (the FP16 table's
// rounding, the search copy's rounding, the FP32 accumulation): every atom
// with |p~| >= M - 2 E_b is emitted, M the running maximum.
#include <type_traits>

#include "act_emit.h"

namespace act {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int LG_S = 128;          // lags per stage
constexpr int LG_KS = LG_S / 16;   // MFMA k-steps per stage
constexpr int LG_ROWS = 128;       // (channel, time centre) rows per tile
constexpr int LG_RB = 4;           // 32-row blocks per wave (every row of the tile)
constexpr int LG_PAD = LG_S + 8;   // LDS row length in FP16 (272 B: conflict-free 16-byte reads)

__device__ __forceinline__ int lg_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// DPP step: max of x and the value of lane perm(lane) (row_mask selects the
// 16-lane rows that take part; the others keep x)
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_max(float x) {
    const int y = __builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), CTRL, ROWS, 0xf, false);
    return fmaxf(x, __int_as_float(y));
}

// Max over each 32-lane half of the wave, valid in lanes 16-31 and 48-63:
// quad xor 1, quad xor 2, half-row mirror, row mirror (max of each 16-lane
// row), then rows 1 and 3 take lane 15 of the row below.
__device__ __forceinline__ float half_wave_max(float x) {
    x = dpp_max<0xb1>(x);        // quad_perm [1,0,3,2]
    x = dpp_max<0x4e>(x);        // quad_perm [2,3,0,1]
    x = dpp_max<0x141>(x);       // row_half_mirror
    x = dpp_max<0x140>(x);       // row_mirror
    x = dpp_max<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    return x;
}

struct LagDev {
    const f16x8* G;          // [Q_pad/32][LS][64] pre-swizzled lag table
    const float* inv_norm;   // [atoms] FP32 1/|g|
    const int* tc_shift;     // [n_tc] integer sample of each time centre (increasing)
    const _Float16* shadow;  // [B][n_pad] fl16(fl32(r) s_b), zero past n
    const float* rscale;     // [B] s_b
    int LS;                  // k-steps of lags (2 N_pad / 16)
    int Q;                   // columns (n_fc n_c n_ld)
    int n_tc;
    int CB, TB;              // channels x time centres of a tile's 128 rows (CB TB = 128)
    int cb_log2;             // log2 CB (CB is a power of two): row = t CB + slot
};

struct LagLds {
    f16x8 a[2][LG_ROWS][LG_PAD / 8];  // R stages; after the main loop: the tile's 1/|g| [TB][cols]
    unsigned rmax[LG_ROWS];  // row maxima of |p~| (float bits)
    float M[LG_ROWS];        // emission threshold per channel slot
    float rinv[LG_ROWS];     // 1/s_b per channel slot
};
static_assert(sizeof(f16x8) * 2 * LG_ROWS * (LG_PAD / 8) >= 128 * 128 * sizeof(float), "1/|g| staging fits");

template <int WCB, bool RERUN, bool DUMP>
__global__ void __launch_bounds__(256, 1) k_search_lag(GridDev g, LagDev ld, SearchCtl ctl, int batch,
                                                       int n_cbk, int n_cg, int n_tg) {
    __shared__ LagLds L;
    constexpr int COLS = 4 * WCB * 32;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long n_rbk = (long long)n_cg * n_tg;
    const long long tiles = (long long)n_cbk * n_rbk;
    const long long chunk = (tiles + 7) / 8;
    for (long long x = blockIdx.x; x < 8 * chunk; x += gridDim.x) {
        const long long tid = (x % 8) * chunk + x / 8;
        if (tid >= tiles) continue;
        const int cbk = (int)(tid / n_rbk);
        const int rbk = (int)(tid % n_rbk);
        const int cg = rbk % n_cg, tg = rbk / n_cg;
        const int ch0 = cg * ld.CB, tc0 = tg * ld.TB;
        // skip tiles none of whose channels take part
        int live = 0;
        if (threadIdx.x < ld.CB && ch0 + (int)threadIdx.x < batch) {
            const int b = ch0 + threadIdx.x;
            live = DUMP || (ctl.ebound[b] >= 0.0 && (!RERUN || ctl.need_rerun[b]));
        }
        if (!__syncthreads_or(live)) continue;

        // lags that meet the tile's rows: e = d + N_pad with 0 <= d + m < n
        const int tc_last = min(tc0 + ld.TB, ld.n_tc) - 1;
        const int m_min = ld.tc_shift[tc0], m_max = ld.tc_shift[tc_last];
        const int e_first = (g.n_pad - m_max) / LG_S * LG_S;
        const int e_end = min(2 * g.n_pad, g.n_pad + g.n - m_min);
        const int ns = (e_end - e_first + LG_S - 1) / LG_S;

        // this thread's chunks of the R stages: chunk c = threadIdx.x + 256 i is
        // (row c / 16, lags 8 (c % 16) ..); a row past the batch or the time
        // centres reads nothing (zero)
        constexpr int NCH = LG_ROWS * (LG_S / 8) / 256;
        int rch[NCH], rm[NCH];
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int c = threadIdx.x + 256 * i, row = c / 16;
            const int b = ch0 + (row & (ld.CB - 1)), tc = tc0 + (row >> ld.cb_log2);
            const bool ok = b < batch && tc < ld.n_tc;
            rch[i] = ok ? b : -1;
            rm[i] = ok ? ld.tc_shift[tc] + 8 * (c % 16) - g.n_pad : 0;
        }
        f16x8 rst[NCH];
        auto load_R = [&](int s) {
            const int E0 = e_first + LG_S * s;
#pragma unroll
            for (int i = 0; i < NCH; ++i) {
                const int n0 = E0 + rm[i];  // first sample of the chunk (a multiple of 8)
                f16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
                if (rch[i] >= 0 && n0 >= 0 && n0 < g.n_pad)
                    v = *reinterpret_cast<const f16x8*>(ld.shadow + (size_t)rch[i] * g.n_pad + n0);
                rst[i] = v;
            }
        };
        auto store_R = [&](int buf) {
#pragma unroll
            for (int i = 0; i < NCH; ++i) {
                const int c = threadIdx.x + 256 * i;
                L.a[buf][c / 16][c % 16] = rst[i];
            }
        };

        f32x16 acc[LG_RB][WCB];
#pragma unroll
        for (int rb = 0; rb < LG_RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < WCB; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[rb][cb][v] = 0.0f;

        // B fragments of this wave's columns: k-step ls of column block qb at
        // G + (qb LS + ls) 64 + lane; loaded half a stage (4 k-steps) ahead
        const f16x8* gcol[WCB];
#pragma unroll
        for (int cb = 0; cb < WCB; ++cb)
            gcol[cb] = ld.G + ((size_t)(cbk * 4 * WCB + w * WCB + cb) * ld.LS) * 64 + lane;
        constexpr int HK = LG_KS / 2;
        f16x8 gh[2][HK][WCB];  // [half of the stage][k-step][column block]
        auto load_G = [&](f16x8 (&dst)[HK][WCB], int s, int half) {
            const int ls0 = (e_first + LG_S * s) / 16 + HK * half;
#pragma unroll
            for (int ks = 0; ks < HK; ++ks)
#pragma unroll
                for (int cb = 0; cb < WCB; ++cb) dst[ks][cb] = gcol[cb][(size_t)(ls0 + ks) * 64];
        };
        auto mfma_half = [&](const f16x8 (&src)[HK][WCB], int buf, int half) {
#pragma unroll
            for (int ks = 0; ks < HK; ++ks) {
                const int k8 = 2 * (HK * half + ks) + (lane >> 5);
                f16x8 af[LG_RB];
#pragma unroll
                for (int rb = 0; rb < LG_RB; ++rb) af[rb] = L.a[buf][rb * 32 + (lane & 31)][k8];
#pragma unroll
                for (int rb = 0; rb < LG_RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < WCB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[rb], src[ks][cb], acc[rb][cb], 0, 0, 0);
            }
        };

        // ---- software pipeline over stages: R of stage s+1 loads while stage
        // s runs (two LDS buffers, one barrier per stage: the other buffer was
        // last read before the previous barrier); G half-stages load one half
        // ahead (the scheduling barriers keep the loads ahead of the MFMAs)
        if (ns > 0) {
            load_R(0);
            load_G(gh[0], 0, 0);
            store_R(0);
        }
        __syncthreads();
        auto step = [&](int s, auto bufc) {
            constexpr int buf = decltype(bufc)::value;
            const int nxt = s + 1 < ns ? s + 1 : s;  // the last stage reloads itself: in range, unused
            load_R(nxt);
            load_G(gh[1], s, 1);
            __builtin_amdgcn_sched_barrier(0);
            mfma_half(gh[0], buf, 0);
            __builtin_amdgcn_sched_barrier(0);
            load_G(gh[0], nxt, 0);
            __builtin_amdgcn_sched_barrier(0);
            mfma_half(gh[1], buf, 1);
            store_R(buf ^ 1);
            __syncthreads();
        };
        for (int s = 0; s < ns; s += 2) {
            step(s, std::integral_constant<int, 0>{});
            if (s + 1 < ns) step(s + 1, std::integral_constant<int, 1>{});
        }

        // ---- epilogue: p = P inv_norm / s_b, row maxima, per-channel running
        // maximum, certified emission.  The tile's inverse norms (TB time
        // centres x cols, contiguous per time centre) are staged in the freed
        // R buffers with coalesced loads.
        float* invs = reinterpret_cast<float*>(&L.a[0][0][0]);
        const int n_fc_cl = ld.Q;
        // the epilogue's lane-dependent addresses are tile-invariant; an opaque
        // copy of the lane index keeps them from being hoisted out of the tile
        // loop (they would stay live across it and spill)
        int elane = lane;
        asm volatile("" : "+v"(elane));
        const int q0 = cbk * COLS;
        for (int idx = threadIdx.x; idx < ld.TB * COLS; idx += 256) {
            const int t = idx / COLS, c = idx % COLS;
            const int tc = tc0 + t, q = q0 + c;
            invs[idx] = (tc < ld.n_tc && q < n_fc_cl) ? ld.inv_norm[(long long)tc * n_fc_cl + q] : 0.0f;
        }
        if (threadIdx.x < LG_ROWS) {
            L.rmax[threadIdx.x] = 0u;
            const int b = ch0 + threadIdx.x;
            L.rinv[threadIdx.x] = (threadIdx.x < ld.CB && b < batch) ? 1.0f / ld.rscale[b] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int rb = 0; rb < LG_RB; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = rb * 32 + lg_row(v, elane);
                const int sl = row & (ld.CB - 1), t = row >> ld.cb_log2;
                const int b = ch0 + sl, tc = tc0 + t;
                const float rinv = L.rinv[sl];  // 0 past the batch
                float m = 0.0f;
#pragma unroll
                for (int cb = 0; cb < WCB; ++cb) {
                    const int c = (w * WCB + cb) * 32 + (elane & 31);
                    const float p = (acc[rb][cb][v] * invs[t * COLS + c]) * rinv;  // 0 past the dictionary
                    if (DUMP) {
                        const long long i = (long long)tc * n_fc_cl + q0 + c;
                        if (b < batch && tc < ld.n_tc && q0 + c < n_fc_cl && i >= ctl.dump_begin &&
                            i < ctl.dump_begin + ctl.dump_count)
                            ctl.dump[(size_t)b * ctl.dump_count + (i - ctl.dump_begin)] = p;
                    } else {
                        m = fmaxf(m, fabsf(p));
                    }
                }
                if (!DUMP) {
                    // lanes 0-31 share one row, lanes 32-63 another
                    m = half_wave_max(m);
                    if ((elane & 31) == 31) atomicMax(&L.rmax[row], fbits(m));
                }
                // bound the loads in flight (register pressure of the unrolled epilogue)
                __builtin_amdgcn_sched_barrier(0);
            }
        if (DUMP) {
            __syncthreads();
            continue;
        }
        __syncthreads();
        if (threadIdx.x < ld.CB) {
            const int sl = threadIdx.x, b = ch0 + sl;
            float M = INFINITY;
            if (b < batch && ctl.ebound[b] >= 0.0 && (!RERUN || ctl.need_rerun[b])) {
                float wm = 0.0f;
                for (int r = sl; r < LG_ROWS; r += ld.CB) wm = fmaxf(wm, bitsf(L.rmax[r]));
                const float cur = load_gmax(&ctl.gmax[b]);
                M = cur;
                if (!RERUN && wm > cur) M = fmaxf(bitsf(atomicMax(&ctl.gmax[b], fbits(wm))), wm);
                const double Td = (double)M - 2.0 * ctl.ebound[b];
                float T = (float)Td;
                if ((double)T > Td) T = nextafterf(T, -INFINITY);
                M = T;
            }
            L.M[sl] = M;
        }
        __syncthreads();
#pragma unroll
        for (int rb = 0; rb < LG_RB; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = rb * 32 + lg_row(v, elane);
                const int sl = row & (ld.CB - 1), t = row >> ld.cb_log2;
                const float T = L.M[sl];
                const int b = ch0 + sl, tc = tc0 + t;
                // rows whose largest |p~| misses the threshold emit nothing
                if (T == INFINITY || tc >= ld.n_tc || bitsf(L.rmax[row]) < T) continue;
                const float rinv = L.rinv[sl];
#pragma unroll
                for (int cb = 0; cb < WCB; ++cb) {
                    const int c = (w * WCB + cb) * 32 + (elane & 31);
                    // the same FP32 operations as the row maxima: the same p
                    const float p = (acc[rb][cb][v] * invs[t * COLS + c]) * rinv;
                    if (q0 + c < n_fc_cl && fabsf(p) >= T) {
                        const int j = atomicAdd(&ctl.cand_count[b], 1);
                        if (j < ctl.cap) {
                            ctl.cand_idx[(size_t)b * ctl.cap + j] = (unsigned)((long long)tc * n_fc_cl + q0 + c);
                            ctl.cand_score[(size_t)b * ctl.cap + j] = p;
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        __syncthreads();  // L.rmax / L.M / the R buffers are rewritten by the next tile
    }
}

// The lag table: G_q(d) in FP64, rounded to FP32 and then FP16 (RNE), written
// in MFMA B-operand order; columns past Q are zero.
__global__ void k_build_lag_table(GridDev g, int Q_pad, f16x8* __restrict__ G) {
    const int n_cl = g.cnt[2] * g.cnt[3];
    const int LS = 2 * g.n_pad / 16;
    const long long frags = (long long)(Q_pad / 32) * LS * 64;  // one f16x8 per (column block, k-step, lane)
    for (long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x; f < frags;
         f += (long long)gridDim.x * blockDim.x) {
        const int lane = (int)(f % 64);
        const long long qs = f / 64;
        const int ls = (int)(qs % LS);
        const int qb = (int)(qs / LS);
        const int q = qb * 32 + (lane & 31);
        f16x8 out;
        if (q >= g.cnt[1] * n_cl) {
#pragma unroll
            for (int j = 0; j < 8; ++j) out[j] = (_Float16)0.0f;
        } else {
            const int fc = q / n_cl, cl = q % n_cl;
            const double f0 = g.axis[g.off[1] + fc];
            const double c = g.axis[g.off[2] + cl / g.cnt[3]];
            const double inv_dt = 1.0 / exp(g.axis[g.off[3] + cl % g.cnt[3]]);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int e = 16 * ls + 8 * (lane >> 5) + j;
                const double tau = (double)(e - g.n_pad) / g.fs;
                const double u = tau * inv_dt;
                const double v = exp(-0.5 * u * u) * cospi(2.0 * (c * tau * tau + f0 * tau));
                out[j] = (_Float16)(float)v;
            }
        }
        G[f] = out;
    }
}

act_status build_lag_table(act_plan_s* p, hipStream_t s) {
    const int Q_pad = p->lag_q_pad;
    const long long frags = (long long)(Q_pad / 32) * (2 * p->n_pad / 16) * 64;
    const long long blocks = std::min<long long>((frags + 255) / 256, (long long)device_cus() * 64);
    hipLaunchKernelGGL(k_build_lag_table, dim3((unsigned)blocks), dim3(256), 0, s, p->grid, Q_pad,
                       (f16x8*)p->table);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

// FP32 accumulation chain of one score: at most one rounding per lag (2 N_pad)
// plus the scalings.
int lag_chain_length(int n_pad) { return 2 * n_pad + 2; }

act_status launch_search_lag(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s) {
    LagDev ld;
    ld.G = (const f16x8*)p->table;
    ld.inv_norm = p->inv_norm32;
    ld.tc_shift = p->tc_shift;
    ld.shadow = (const _Float16*)p->shadow;
    ld.rscale = p->rscale;
    ld.LS = 2 * p->n_pad / 16;
    ld.Q = p->grid.cnt[1] * p->n_cl;
    ld.n_tc = p->grid.cnt[0];
    // rows: the smallest power of two of channels covering the batch (at most
    // 32) times the time centres that fill 128 rows
    int CB = 1;
    while (CB < batch && CB < 32) CB *= 2;
    ld.CB = CB;
    ld.TB = LG_ROWS / CB;
    ld.cb_log2 = 0;
    while ((1 << ld.cb_log2) < CB) ++ld.cb_log2;
    const int n_cg = (batch + CB - 1) / CB;
    const int n_tg = (ld.n_tc + ld.TB - 1) / ld.TB;
    // one channel: 128 columns per tile (twice the tiles); several: 256
    const bool wide = batch > 1;
    const int cols = wide ? 256 : 128;
    const int n_cbk = (ld.Q + cols - 1) / cols;
    const long long tiles = (long long)n_cbk * n_cg * n_tg;
    long long blocks = (tiles + 7) / 8 * 8;
    const long long cap = grid_cap(p, 1);  // LDS: one workgroup per CU
    blocks = blocks < cap ? blocks : cap;
    const dim3 grid((unsigned)blocks), blk(256);
#define LAG_LAUNCH(WCB, RR, DD)                                                                       \
    hipLaunchKernelGGL((k_search_lag<WCB, RR, DD>), grid, blk, 0, s, p->grid, ld, ctl, batch, n_cbk, n_cg, \
                       n_tg)
    if (wide) {
        if (ctl.dump) LAG_LAUNCH(2, false, true);
        else if (ctl.pass) LAG_LAUNCH(2, true, false);
        else LAG_LAUNCH(2, false, false);
    } else {
        if (ctl.dump) LAG_LAUNCH(1, false, true);
        else if (ctl.pass) LAG_LAUNCH(1, true, false);
        else LAG_LAUNCH(1, false, false);
    }
#undef LAG_LAUNCH
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

}  // namespace act
