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
// correlation's multiply-adds (within each tile's nonzero lag band), not the
// factored synthesis' two products per sample.
//
// G: FP16 (RNE of the FP64 value), columns padded to a multiple of 256, lags
// e = d + N_pad in [0, 2 N_pad), pre-swizzled in MFMA B-operand order: for 32
// columns and a k-step of 16 lags the 64 lanes' 16-byte operands are one
// contiguous KiB, so every wave streams its B fragments straight from L2.
// Columns run log-duration major.  The envelope of a log-duration rounds to
// FP16 zero a few durations from its centre, so a tile's columns are zero
// outside a common band of lags; each tile runs only the k-steps inside the
// band of its columns (found from the table itself at plan time).  The
// skipped products are exact zeros: the scores are those of the full product.
// R: per 128-lag stage, 128 rows x 128 lags in LDS (two buffers), each row
// read from the FP16 search copy of its channel.
// Workgroup = 4 waves; tile = 128 rows x (128 or 256) columns; wave w owns
// every row (4 row blocks of 32) and 32 or 64 columns.  Tiles are dealt to the
// 8 XCDs in contiguous ranges with the row blocks of one column block adjacent,
// so the concurrent tiles of an XCD share their G columns in its L2; column
// blocks are ordered so that every XCD gets the same mix of band widths.
//
// Certified emission with a uniform bound per channel (the FP16 table's
// rounding, the search copy's rounding, the FP32 accumulation): every atom
// with |p~| >= M - 2 E_b is emitted, M the running maximum.
//
// Complex atoms (Eq. (1) as written) store each 32-atom block's cos and sin
// parts as two adjacent column blocks; uneven-length batches share the
// longest signal's table and bound each row's true score near its signal's
// end (see k_search_lag).
//
// BF16 form (plain plans of real atoms): the same table and search copy in
// BF16 (RNE) through v_mfma_f32_32x32x16_bf16; a wider per-channel bound
// (unit roundoff 2^-8), the same schedule and emission.
#include <algorithm>
#include <climits>
#include <type_traits>
#include <vector>

#include "act_emit.h"

namespace act {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));  // the BF16 form's operands, same storage
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
    const float* inv;        // [n_tc][Qp] FP32 1/|g| in the table's column order (0 past Q)
    const int2* span;        // [Q_pad/32] k-steps [lo, hi) holding the block's nonzero entries
    const int* order;        // [column blocks] tile column-block order (balanced over the XCDs)
    const int* tc_shift;     // [n_tc] integer sample of each time centre (increasing)
    const char* shadow;      // FP16 search copies fl16(fl32(r) s_b): allocation base; row b at
                             // element n_pad + b sh_stride, zero past n and in the n_pad-element guards
    int sh_stride;           // row stride (2 n_pad)
    const float* rscale;     // [B] s_b
    int LS;                  // k-steps of lags (2 N_pad / 16)
    int Q;                   // columns (n_fc n_c n_ld)
    int Qp;                  // padded columns (row stride of inv)
    int FC;                  // n_fc n_c: columns of one log-duration
    int n_ld;
    int n_tc;
    int CB, TB;              // channels x time centres of a tile's 128 rows (CB TB = 128)
    int cb_log2;             // log2 CB (CB is a power of two): row = t CB + slot
    // ragged batches: channels by decreasing length, per channel group the
    // prefix of its time groups, and the bound of |g_full| / |g_w| per
    // 256-column block and distance from the centre to the signal's end
    const int* perm;
    const int* rows;
    const float* rho;
    int rho_d, div;
    // pass-0 searches: [0] += MFMA instructions the launch executed (every
    // wave's), [1] += 1 per launch; NULL when not counting
    unsigned long long* exec;
    // resident-residual form (k_search_lag_rs): per XCD its column pairs,
    // longest band first ([8][rs_cp_per_x]) and their count; each channel's
    // copy in LDS holds samples [-rs_glo, rs_len - rs_glo) at a row stride of
    // rs_stride elements
    const int* rs_cp;
    const int* rs_cp_count;
    int rs_cp_per_x;
    float* rs_map;   // [channel groups][8 rs_cp_per_x n_tg units][32] the pass-0 max map
    int* rs_pairs;   // pass 1's count and list of flagged map entries; pass 0 clears the count
    int rs_glo, rs_len, rs_stride;
};

struct LagLds {
    f16x8 a[2][LG_ROWS][LG_PAD / 8];  // R stages; after the main loop: the tile's 1/|g| [TB][cols]
    float gm[4][32];         // per wave: max |p~| over the rows r = 32 rb + g of every rb, per g
    float M[LG_ROWS];        // emission threshold per channel slot
    float rinv[LG_ROWS];     // 1/s_b per channel slot
    float rrow[LG_ROWS];     // ragged: 1/s_b of the row's channel, 0 for a time centre past its end
    float rhor[LG_ROWS];     // ragged: the row's bound of |g_full| / |g_w| (1 away from the end)
    double ebs[32];          // ragged: E_b per channel slot
    unsigned emit;           // bit g: some row 32 rb + g reaches its channel's threshold
    unsigned cnt[32];        // per channel slot: the tile's candidates, then their running position
    int base[32];            // per channel slot: first list entry reserved for the tile
};
static_assert(sizeof(f16x8) * 2 * LG_ROWS * (LG_PAD / 8) >= 128 * 128 * sizeof(float), "1/|g| staging fits");

// flat atom index of table column qc (columns are ordered log-duration major:
// qc = ld FC + (f_c n_c + c); atoms are (f_c, c, ld) with ld fastest)
__device__ __forceinline__ long long lag_atom(const LagDev& ld, int tc, int qc) {
    const int l = qc / ld.FC, fcc = qc - l * ld.FC;
    return (long long)tc * ld.Q + (long long)fcc * ld.n_ld + l;
}

// CPLX: complex atoms.  A wave's two column blocks are the cos and sin parts
// of the same 32 atoms, so a lane's two accumulators are (a, b) of one atom and
// its score is sqrt(a^2 + b^2) / |E_w|.
//
// RAG: uneven-length batch.  Slots take channels in order of decreasing length
// (ld.perm), so a 32-channel group's longest signal comes first; only its time
// groups form tiles.  Every score is normalised by the atom's norm over the
// longest window [0, n_max) (the plan's 1/|g|).  The search copy is zero past
// a channel's end, so that score is the true one times |g_w| / |g_full| <= 1,
// and the true score is at most rho times it, rho <= sqrt(1 + tail energy of
// the atom beyond the end) (|g_w| >= 1).  A row of a channel emits its atoms
// by the upper bound (|p~| + E_b) rho - E_b against M - 2 E_b and stores that
// bound as the candidate's score; rho = 1 beyond ld.rho_d samples from the end.
template <int WCB, bool RERUN, bool DUMP, bool CPLX, bool RAG, bool BF>
__global__ void __launch_bounds__(256, 1) k_search_lag(GridDev g, LagDev ld, SearchCtl ctl, int batch,
                                                       int n_cbk, int n_cg, int n_tg) {
    static_assert(!CPLX || WCB == 2, "complex atoms pair two column blocks");
    static_assert(!RAG || (WCB == 2 && !CPLX && !DUMP), "ragged: real atoms, 256-column tiles, search only");
    static_assert(!BF || (!CPLX && !RAG), "BF16 table: plain plans of real atoms");
    __shared__ LagLds L;
    // the rerun pass: nothing to do unless some channel's list overflowed
    if (RERUN) {
        int any = 0;
        for (int b = threadIdx.x; b < batch; b += blockDim.x) any |= ctl.need_rerun[b];
        if (!__syncthreads_or(any)) return;
    }
    constexpr int COLS = 4 * WCB * 32;
    constexpr int ACOLS = CPLX ? COLS / 2 : COLS;  // atoms of a tile
    constexpr int NA = CPLX ? 1 : WCB;              // atoms of a lane per accumulator row
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long n_rbk = RAG ? (long long)ld.rows[n_cg] : (long long)n_cg * n_tg;
    const long long tiles = (long long)n_cbk * n_rbk;
    const long long chunk = (tiles + 7) / 8;
    unsigned long long stages_run = 0;  // the tiles' stages, counted for the executed-work report
    for (long long x = blockIdx.x; x < 8 * chunk; x += gridDim.x) {
        const long long tid = (x % 8) * chunk + x / 8;
        if (tid >= tiles) continue;
        const int cbk = ld.order[(int)(tid / n_rbk)];
        const int rbk = (int)(tid % n_rbk);
        int cg, tg;
        if (RAG) {
            cg = 0;
            while (cg + 1 < n_cg && ld.rows[cg + 1] <= rbk) ++cg;
            tg = rbk - ld.rows[cg];
        } else {
            cg = rbk % n_cg;
            tg = rbk / n_cg;
        }
        const int ch0 = cg * ld.CB, tc0 = tg * ld.TB;
        // the channel of slot sl (-1 past the batch); lengths outside [0, n] count as 0
        auto chan = [&](int sl) { const int k = ch0 + sl; return k < batch ? (RAG ? ld.perm[k] : k) : -1; };
        auto chan_len = [&](int b) {
            const int nb = RAG ? ctl.len[b] : g.n;
            return (nb < 0 || nb > g.n) ? 0 : nb;
        };
        const int n_long = RAG ? chan_len(chan(0)) : g.n;  // the group's longest signal
        const int n_tc_t = RAG ? n_long / ld.div : ld.n_tc;
        const int q0 = cbk * COLS;
        const int aq0 = cbk * ACOLS;  // first atom (in the table's order) of the tile

        // lags that meet the tile's rows, e = d + N_pad with 0 <= d + m < n,
        // cut to the k-steps where the tile's columns hold nonzero entries:
        // the skipped products are exact zeros, so every score is unchanged
        const int tc_last = min(tc0 + ld.TB, n_tc_t) - 1;
        const int m_min = ld.tc_shift[tc0], m_max = ld.tc_shift[tc_last];
        int klo = ld.LS, khi = 0;
#pragma unroll
        for (int j = 0; j < 4 * WCB; ++j) {
            const int2 sp = ld.span[cbk * 4 * WCB + j];
            klo = min(klo, sp.x);
            khi = max(khi, sp.y);
        }
        const int e_first = max((g.n_pad - m_max) / LG_S, 16 * klo / LG_S) * LG_S;
        const int e_end = min(min(2 * g.n_pad, g.n_pad + n_long - m_min), 16 * khi);
        const int ns = e_end > e_first ? (e_end - e_first + LG_S - 1) / LG_S : 0;
        stages_run += (unsigned long long)ns;

        // per channel slot: certified bound, running maximum, residual scale
        // (read now, used by the epilogue)
        int live = 0;
        double eb = -1.0;
        float pre_gmax = 0.0f, rsc = 0.0f;
        if (threadIdx.x < ld.CB && ch0 + (int)threadIdx.x < batch) {
            const int b = chan(threadIdx.x);
            eb = ctl.ebound[b];
            rsc = ld.rscale[b];
            if (!DUMP) pre_gmax = load_gmax(&ctl.gmax[b]);
            live = DUMP || (eb >= 0.0 && (!RERUN || ctl.need_rerun[b]));
        }
        // ragged: per row, 1/s_b (0 for a time centre past the channel's end) and rho
        float rrow_v = 0.0f, rhor_v = 1.0f;
        if (RAG && threadIdx.x < LG_ROWS) {
            const int sl = threadIdx.x & (ld.CB - 1), t = threadIdx.x >> ld.cb_log2;
            const int b = chan(sl);
            if (b >= 0) {
                const int nb = chan_len(b), tc = tc0 + t;
                if (tc < nb / ld.div) {
                    const float sc = ld.rscale[b];
                    rrow_v = sc > 0.0f ? 1.0f / sc : 0.0f;
                    const int dl = nb - ld.tc_shift[tc];
                    rhor_v = dl < ld.rho_d ? ld.rho[(size_t)cbk * ld.rho_d + dl] : 1.0f;
                }
            }
        }
        if (threadIdx.x == 0) L.emit = 0u;
        if (threadIdx.x < 32) L.cnt[threadIdx.x] = 0u;
        // the rerun pass skips most tiles: vote before any load
        if (RERUN && !__syncthreads_or(live)) continue;

        // this thread's chunks of the R stages: chunk c = threadIdx.x + 256 i is
        // (row c / 16, lags 8 (c % 16) ..).  The window of every lag lies in
        // the row's guarded slot of the search copy (zero outside the
        // signal), so the loads need no bounds; a row past the batch or the
        // time centres reads a valid row and scores zero (1/s_b or 1/|g| is 0).
        constexpr int NCH = LG_ROWS * (LG_S / 8) / 256;
        unsigned roff[NCH];  // byte offset of the chunk at e = 0
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int c = threadIdx.x + 256 * i, row = c / 16;
            const int bs = chan(row & (ld.CB - 1));
            const int b = RAG ? (bs >= 0 ? bs : chan(0)) : min(ch0 + (row & (ld.CB - 1)), batch - 1);
            const int tc = min(tc0 + (row >> ld.cb_log2), n_tc_t - 1);
            roff[i] = 2u * (unsigned)(b * ld.sh_stride + ld.tc_shift[tc] + 8 * (c % 16));
        }
        f16x8 rst[NCH];
        auto load_R = [&](int s) {
            const unsigned e0 = 2u * (unsigned)(e_first + LG_S * s);
#pragma unroll
            for (int i = 0; i < NCH; ++i) rst[i] = *reinterpret_cast<const f16x8*>(ld.shadow + (roff[i] + e0));
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
        // byte (qb LS + ls) 1 KiB + 16 lane; loaded half a stage (4 k-steps) ahead
        const char* gblk[WCB];
#pragma unroll
        for (int cb = 0; cb < WCB; ++cb)
            gblk[cb] = reinterpret_cast<const char*>(ld.G) + (size_t)(cbk * 4 * WCB + w * WCB + cb) * ld.LS * 1024;
        const unsigned glane = 16u * (unsigned)lane;
        constexpr int HK = LG_KS / 2;
        f16x8 gh[2][HK][WCB];  // [half of the stage][k-step][column block]
        auto load_G = [&](f16x8 (&dst)[HK][WCB], int s, int half) {
            const unsigned o = 1024u * (unsigned)((e_first + LG_S * s) / 16 + HK * half) + glane;
#pragma unroll
            for (int ks = 0; ks < HK; ++ks)
#pragma unroll
                for (int cb = 0; cb < WCB; ++cb)
                    dst[ks][cb] = *reinterpret_cast<const f16x8*>(gblk[cb] + (o + 1024u * ks));
        };
        // A fragments one k-step ahead of the MFMAs that use them
        auto mfma_half = [&](const f16x8 (&src)[HK][WCB], int buf, int half) {
            f16x8 af[2][LG_RB];
            auto load_A = [&](f16x8 (&dst)[LG_RB], int ks) {
                const int k8 = 2 * (HK * half + ks) + (lane >> 5);
#pragma unroll
                for (int rb = 0; rb < LG_RB; ++rb) dst[rb] = L.a[buf][rb * 32 + (lane & 31)][k8];
            };
            load_A(af[0], 0);
#pragma unroll
            for (int ks = 0; ks < HK; ++ks) {
                if (ks + 1 < HK) load_A(af[(ks + 1) & 1], ks + 1);
#pragma unroll
                for (int rb = 0; rb < LG_RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < WCB; ++cb)
                        if constexpr (BF)
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, af[ks & 1][rb]), __builtin_bit_cast(bf16x8, src[ks][cb]),
                                acc[rb][cb], 0, 0, 0);
                        else
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[ks & 1][rb], src[ks][cb],
                                                                                 acc[rb][cb], 0, 0, 0);
            }
            // order: the first k-step's A reads, then each k-step's MFMAs in
            // pairs with one A read of the next k-step between them
            __builtin_amdgcn_sched_group_barrier(0x100, LG_RB, 0);
#pragma unroll
            for (int ks = 0; ks < HK; ++ks)
#pragma unroll
                for (int rb = 0; rb < LG_RB; ++rb) {
                    __builtin_amdgcn_sched_group_barrier(0x008, WCB, 0);
                    if (ks + 1 < HK) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                }
        };

        // the first stage's loads and the first 1024 of the tile's inverse
        // norms (held until the epilogue) go out before the liveness vote
        if (ns > 0) {
            load_R(0);
            load_G(gh[0], 0, 0);
        }
        const int n_inv = ld.TB * ACOLS;
        float4 inv_pf = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        {
            const int idx = 4 * threadIdx.x, t = idx / ACOLS, c = idx % ACOLS;
            if (idx < n_inv && tc0 + t < ld.n_tc)
                inv_pf = *reinterpret_cast<const float4*>(ld.inv + (size_t)(tc0 + t) * ld.Qp + aq0 + c);
        }
        // skip tiles none of whose channels take part
        if (!RERUN && !__syncthreads_or(live)) continue;

        // ---- software pipeline over stages: R of stage s+1 loads while stage
        // s runs and is stored to the other LDS buffer after the first half
        // (one barrier per stage: that buffer was last read before the
        // previous barrier); G half-stages load one half ahead.  The
        // scheduling barriers keep the global loads ahead of the MFMAs and let
        // LDS reads move across.
        if (ns > 0) store_R(0);
        __syncthreads();
        auto step = [&](int s, auto bufc) {
            constexpr int buf = decltype(bufc)::value;
            const int nxt = s + 1 < ns ? s + 1 : s;  // the last stage reloads itself: in range, unused
            load_R(nxt);
            load_G(gh[1], s, 1);
            __builtin_amdgcn_sched_barrier(0x100);
            mfma_half(gh[0], buf, 0);
            __builtin_amdgcn_sched_barrier(0x100);
            store_R(buf ^ 1);
            load_G(gh[0], nxt, 0);
            __builtin_amdgcn_sched_barrier(0x100);
            mfma_half(gh[1], buf, 1);
            __syncthreads();
        };
        for (int s = 0; s < ns; s += 2) {
            step(s, std::integral_constant<int, 0>{});
            if (s + 1 < ns) step(s + 1, std::integral_constant<int, 1>{});
        }

        // ---- epilogue: p = P inv_norm / s_b (kept in acc), per-channel
        // maxima and running maximum, certified emission of the rows that
        // reach the threshold.  The tile's inverse norms (TB time centres x
        // cols, contiguous per time centre) are staged in the freed R buffers.
        float* invs = reinterpret_cast<float*>(&L.a[0][0][0]);
        if (4 * (int)threadIdx.x < n_inv) *reinterpret_cast<float4*>(invs + 4 * threadIdx.x) = inv_pf;
        for (int base = 1024; base < n_inv; base += 4096) {
            float4 vv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = base + 1024 * u + 4 * threadIdx.x, t = idx / ACOLS, c = idx % ACOLS;
                vv[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (idx < n_inv && tc0 + t < ld.n_tc)
                    vv[u] = *reinterpret_cast<const float4*>(ld.inv + (size_t)(tc0 + t) * ld.Qp + aq0 + c);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = base + 1024 * u + 4 * threadIdx.x;
                if (idx < n_inv) *reinterpret_cast<float4*>(invs + idx) = vv[u];
            }
        }
        if (threadIdx.x < LG_ROWS) L.rinv[threadIdx.x] = rsc > 0.0f ? 1.0f / rsc : 0.0f;
        if (RAG && threadIdx.x < LG_ROWS) {
            L.rrow[threadIdx.x] = rrow_v;
            L.rhor[threadIdx.x] = rhor_v;
        }
        if (RAG && threadIdx.x < ld.CB) L.ebs[threadIdx.x] = eb;
        // the epilogue's lane-dependent addresses are tile-invariant; an opaque
        // copy of the lane index keeps them from being hoisted out of the tile
        // loop (they would stay live across it and spill)
        int elane = lane;
        asm volatile("" : "+v"(elane));
        // the lane's atom of accumulator block cb (tile order) and its raw score
        auto acol = [&](int cb) { return CPLX ? w * 32 + (elane & 31) : (w * WCB + cb) * 32 + (elane & 31); };
        auto raw = [&](int rb, int cb, int v) {
            return CPLX ? sqrtf(acc[rb][0][v] * acc[rb][0][v] + acc[rb][1][v] * acc[rb][1][v]) : acc[rb][cb][v];
        };
        __syncthreads();
        // A lane's rows are r = 32 rb + g, g = lg_row(v, lane): the channel
        // slot g % CB does not depend on rb (CB divides 32), so a channel's
        // maximum takes the rb blocks in registers and one half-wave reduction
        // per v.
        if (DUMP) {
#pragma unroll
            for (int rb = 0; rb < LG_RB; ++rb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = rb * 32 + lg_row(v, elane);
                    const int sl = row & (ld.CB - 1), t = row >> ld.cb_log2;
                    const float rinv = L.rinv[sl];
                    const int b = ch0 + sl, tc = tc0 + t;
#pragma unroll
                    for (int cb = 0; cb < NA; ++cb) {
                        const int c = acol(cb);
                        const float p = (raw(rb, cb, v) * invs[t * ACOLS + c]) * rinv;
                        if (b < batch && tc < ld.n_tc && aq0 + c < ld.Q) {
                            const long long i = lag_atom(ld, tc, aq0 + c);
                            if (i >= ctl.dump_begin && i < ctl.dump_begin + ctl.dump_count)
                                ctl.dump[(size_t)b * ctl.dump_count + (i - ctl.dump_begin)] = p;
                        }
                    }
                }
            __syncthreads();
            continue;
        }
        // the scale factors of v + 1 load while v computes; the maxima are
        // stored after the loop (no store between the loads)
        float sc[2][LG_RB][WCB], ri[2][LG_RB], gmv[16];
        auto load_sc = [&](int v, float (&dst)[LG_RB][WCB], float (&r)[LG_RB]) {
            const int gr = lg_row(v, elane);
            const float r0 = RAG ? 0.0f : L.rinv[gr & (ld.CB - 1)];  // 0 past the batch
#pragma unroll
            for (int rb = 0; rb < LG_RB; ++rb) {
                r[rb] = RAG ? L.rrow[rb * 32 + gr] : r0;
                const int t = (rb * 32 + gr) >> ld.cb_log2;
#pragma unroll
                for (int cb = 0; cb < NA; ++cb) dst[rb][cb] = invs[t * ACOLS + acol(cb)];  // 0 past the dictionary
            }
        };
        load_sc(0, sc[0], ri[0]);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            if (v + 1 < 16) load_sc(v + 1, sc[(v + 1) & 1], ri[(v + 1) & 1]);
            float m = 0.0f;
#pragma unroll
            for (int rb = 0; rb < LG_RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < NA; ++cb) {
                    const float p = (raw(rb, cb, v) * sc[v & 1][rb][cb]) * ri[v & 1][rb];
                    acc[rb][cb][v] = p;
                    m = fmaxf(m, fabsf(p));
                }
            // lanes 0-31 share g, lanes 32-63 hold g + 4
            gmv[v] = half_wave_max(m);
        }
        if ((elane & 31) == 31) {
#pragma unroll
            for (int v = 0; v < 16; ++v) L.gm[w][lg_row(v, elane)] = gmv[v];
        }
        __syncthreads();
        // per channel slot: the threshold M - 2 E_b (M the running maximum,
        // raised by this tile's maximum), and the row groups that reach it
        if (threadIdx.x < ld.CB) {
            const int sl = threadIdx.x, b = chan(sl);
            float T = INFINITY;
            if (live) {
                float wm = 0.0f;
                for (int gr = sl; gr < 32; gr += ld.CB)
                    wm = fmaxf(wm, fmaxf(fmaxf(L.gm[0][gr], L.gm[1][gr]), fmaxf(L.gm[2][gr], L.gm[3][gr])));
                float M = pre_gmax;  // rerun: the final maximum of pass 0
                if (!RERUN && wm > M) {
                    atomicMax(&ctl.gmax[b], fbits(wm));
                    M = wm;
                }
                const double Td = (double)M - 2.0 * eb;
                T = (float)Td;
                if ((double)T > Td) T = nextafterf(T, -INFINITY);
                unsigned bits = 0u;
                for (int gr = sl; gr < 32; gr += ld.CB) {
                    const float gmg = fmaxf(fmaxf(L.gm[0][gr], L.gm[1][gr]), fmaxf(L.gm[2][gr], L.gm[3][gr]));
                    bool f = gmg >= T;
                    if (RAG) {
                        // the group's largest upper bound of a true score
                        const float rh = fmaxf(fmaxf(L.rhor[gr], L.rhor[32 + gr]), fmaxf(L.rhor[64 + gr], L.rhor[96 + gr]));
                        f = ((double)gmg + eb) * rh - eb >= (double)T;
                    }
                    if (f) bits |= 1u << gr;
                }
                if (bits) atomicOr(&L.emit, bits);
            }
            L.M[sl] = T;
        }
        __syncthreads();
        // Emission in two sweeps over the flagged row groups: count each
        // channel slot's candidates in LDS, reserve their list entries with
        // one device atomic per slot, then place them.
        const unsigned em = __builtin_amdgcn_readfirstlane(L.emit);
        if (em) {
            auto sweep = [&](bool place) {
#pragma unroll
                for (int rb = 0; rb < LG_RB; ++rb)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        // the wave's two row groups of v: g = 8 (v / 4) + v % 4 and g + 4
                        if (!((em >> (8 * (v >> 2) + (v & 3))) & 0x11u)) continue;
                        const int gr = lg_row(v, elane);
                        const int row = rb * 32 + gr, t = row >> ld.cb_log2, tc = tc0 + t;
                        if (((em >> gr) & 1u) && (RAG ? L.rrow[row] > 0.0f : tc < ld.n_tc)) {
                            const int sl = gr & (ld.CB - 1), b = chan(sl);
                            const float T = L.M[sl];
#pragma unroll
                            for (int cb = 0; cb < NA; ++cb) {
                                const int c = acol(cb);
                                float p = acc[rb][cb][v];
                                bool hit = fabsf(p) >= T;
                                if (RAG) {
                                    // upper bound of the true score, rounded up to FP32
                                    const float rh = L.rhor[row];
                                    const double e2 = L.ebs[sl];
                                    const double ub = rh == 1.0f ? (double)fabsf(p) : ((double)fabsf(p) + e2) * rh - e2;
                                    hit = ub >= (double)T;
                                    p = __double2float_ru(ub);
                                }
                                if (aq0 + c < ld.Q && hit) {
                                    if (!place) {
                                        atomicAdd(&L.cnt[sl], 1u);
                                    } else {
                                        const int j = L.base[sl] + (int)atomicAdd(&L.cnt[sl], 1u);
                                        if (j < ctl.cap) {
                                            ctl.cand_idx[(size_t)b * ctl.cap + j] = (unsigned)lag_atom(ld, tc, aq0 + c);
                                            ctl.cand_score[(size_t)b * ctl.cap + j] = p;
                                        }
                                    }
                                }
                            }
                        }
                    }
            };
            sweep(false);
            __syncthreads();
            if (threadIdx.x < ld.CB) {
                const unsigned n = L.cnt[threadIdx.x];
                L.base[threadIdx.x] = n ? atomicAdd(&ctl.cand_count[chan(threadIdx.x)], (int)n) : 0;
                L.cnt[threadIdx.x] = 0u;
            }
            __syncthreads();
            sweep(true);
        }
        __syncthreads();  // L.gm / L.M / L.emit / the R buffers are rewritten by the next tile
    }
    if (!RERUN && !DUMP && ld.exec && threadIdx.x == 0) {
        // every stage of a tile: 4 waves x 8 k-steps x 4 row blocks x WCB column blocks
        if (stages_run) atomicAdd(&ld.exec[0], stages_run * (4ull * LG_KS * LG_RB * WCB));
        if (blockIdx.x == 0) atomicAdd(&ld.exec[1], 1ull);
    }
}

// ---------------------------------------------------------------------------
// Resident-residual form: plain plans (real or complex atoms), at least 32
// channels.
//
// A workgroup of 8 waves holds the FP16/BF16 search copies of one group of 32
// channels in LDS, each with zero guards wide enough for every lag a unit
// reads, so that a row (channel, time centre m) of the Hankel operand at lag e
// is the channel's copy at sample e - N_pad + m and no stage is staged or
// synchronised.  A wave's unit of work is 128 rows (4 time centres x 32
// channels; row block rb = time centre, row in block = channel slot) x 64
// columns (two column blocks) over the k-steps where those columns' nonzero
// band meets the rows' lags, padded to a multiple of 4 k-steps (the products
// added by the padding are exact zeros: table entries outside the band, or
// residual samples outside the signal).  Each (channel group, XCD) pair has a
// list of units: the column pairs dealt to that XCD, longest band first, each
// with its time groups in a row, so that the units of a column pair run
// together and share its band in that XCD's L2.  The list is dealt to the
// pair's waves in a fixed schedule (no atomics).
//
// Selection in two launches.  Pass 0 (this kernel) computes every unit and
// keeps per (channel, unit) the unit's largest |p~| (the max map), raising
// each channel's running maximum M; it emits nothing.  Pass 1
// (k_lag_rs_emit) scores again, one (unit, channel) pair per workgroup, only
// the pairs whose map entry reaches M - 2 E_b, and emits every score that
// reaches that threshold.  The lists then hold the certified set and nothing
// else, whatever order the units ran in.
constexpr int RS_WAVES = 8;
constexpr int RS_CH = 32;   // channels per group (one per row of a 32-row block)
constexpr int RS_TB = 4;    // time centres per unit
constexpr int RS_U = 4;     // k-steps per loop trip; B fragments load one trip ahead

constexpr int RS_MAPB = 8;  // units whose map entries a wave holds in LDS before writing them out

struct RsScratch {
    float map[RS_WAVES][RS_MAPB][RS_CH];  // per wave: map entries of its last units
    float um[RS_WAVES][RS_CH];    // per wave: the unit's max |p| per channel slot (before 1/s_b)
    int mapu[RS_WAVES][RS_MAPB];  // per wave: the units of the entries in map
    float rinv[RS_CH];            // 1/s_b per channel slot (0 past the batch)
    unsigned wmax[RS_CH];         // the workgroup's maximum per channel slot (float bits)
};

// Unit descriptors, RS_UD ints per unit in list order ([8 XCDs][column pairs
// per XCD][time groups]): column pair, first time centre, first k-step, k-steps
// (a multiple of RS_U), and per row block the LDS element offset
// glo - N_pad + m_rb + 16 kb of its rows' first sample (lane part excluded).
// Read through the scalar cache: a kernel argument the kernel never writes.
constexpr int RS_UD = 8;

// DUMP: act_correlate's score dump instead of the max map.  CPLX: complex
// atoms; a unit's two column blocks are the cos and sin parts of the same 32
// atoms, so a lane's two accumulators are (a, b) of one atom and its score is
// sqrt(a^2 + b^2) / |E_w|, as in the staged tiles.
template <bool DUMP, bool BF, bool CPLX>
__global__ void __launch_bounds__(64 * RS_WAVES, 1) k_search_lag_rs(GridDev g, LagDev ld, SearchCtl ctl,
                                                                 const int* __restrict__ units, int batch,
                                                                 int n_cg, int n_tg) {
    extern __shared__ f16x8 rs_res[];  // [RS_CH][rs_stride / 8] copies, then RsScratch
    RsScratch& S = *reinterpret_cast<RsScratch*>(rs_res + RS_CH * (ld.rs_stride / 8));
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xcd = blockIdx.x & 7, cg = (int)(blockIdx.x >> 3) % n_cg;
    const int ch0 = cg * RS_CH;
    if (!DUMP && blockIdx.x == 0 && threadIdx.x == 0) ld.rs_pairs[0] = 0;  // pass 1's list, filled after this launch
    // per channel slot: 1/s_b
    if (threadIdx.x < RS_CH) {
        const int b = ch0 + (int)threadIdx.x;
        float ri = 0.0f;
        if (b < batch) {
            const float sc = ld.rscale[b];
            ri = sc > 0.0f ? 1.0f / sc : 0.0f;
        }
        S.rinv[threadIdx.x] = ri;
        S.wmax[threadIdx.x] = 0u;
    }
    const int total = ld.rs_cp_count[xcd] * n_tg;
    const int qbase = xcd * ld.rs_cp_per_x * n_tg;  // the pair's first unit in list order
    const int* qunits = units + (size_t)qbase * RS_UD;
    float* qmap = ld.rs_map + ((size_t)cg * 8 * ld.rs_cp_per_x * n_tg + qbase) * RS_CH;
    const char* lds_base = reinterpret_cast<const char*>(rs_res);
    const unsigned glane = 16u * (unsigned)lane;
    const unsigned alane = 2u * (unsigned)((lane & 31) * ld.rs_stride + 8 * (lane >> 5));
    unsigned long long mfma_run = 0;  // MFMA instructions this wave executed (pass 0)

    // The pair's units, longest band first, are dealt to its waves in rounds,
    // in snake order (round r gives unit r W + i for even r, r W + W - 1 - i
    // for odd r; W waves, i the wave's index); the second wave of each SIMD
    // (waves 4-7) starts half-way through the rounds, so that the two waves of
    // a SIMD reach their epilogues at different times.
    const int J = ((int)gridDim.x - xcd + 7) / 8;                  // workgroups on this XCD
    const int nwq = RS_WAVES * ((J - cg + n_cg - 1) / n_cg);       // waves of this (channel group, XCD)
    const int qi = RS_WAVES * ((int)(blockIdx.x >> 3) / n_cg) + w;
    const int rounds = (total + nwq - 1) / nwq;
    const int r0 = w >= RS_WAVES / 2 ? rounds / 2 : 0;
    auto unit_at = [&](int k) {  // the wave's k-th unit, or -1 (a partial last round)
        int r = k + r0;
        if (r >= rounds) r -= rounds;
        const int u = r * nwq + ((r & 1) ? nwq - 1 - qi : qi);
        return u < total ? u : -1;
    };
    auto next_k = [&](int k) {  // the wave's first position k' >= k with a unit (rounds if none)
        while (k < rounds && unit_at(k) < 0) ++k;
        return k;
    };
    struct Unit {
        int u, cp, tc0, kb, nk, a[RS_TB];
    };
    auto decode = [&](int u) {
        const int* d = qunits + (size_t)u * RS_UD;
        Unit x;
        x.u = u;
        x.cp = d[0];
        x.tc0 = d[1];
        x.kb = d[2];
        x.nk = d[3];
#pragma unroll
        for (int rb = 0; rb < RS_TB; ++rb) x.a[rb] = d[4 + rb];
        return x;
    };
    // B fragments of the current trip's RS_U k-steps.  Every trip issues
    // exactly 2 RS_U loads (the last trip's fetch the next unit's first
    // k-steps, or repeat a valid address).
    f16x8 ring[RS_U][2];
    // wave-uniform block addresses; a lane reads 16 bytes at glane past them
    auto gaddr = [&](const Unit& x, int cb) {
        return reinterpret_cast<const char*>(ld.G) + (size_t)(2 * x.cp + cb) * ld.LS * 1024;
    };
    // first k-steps of unit x (a unit without k-steps, or none: k-step 0 of block 0)
    auto first_addr = [&](bool has, const Unit& x, int cb) {
        return has && x.nk > 0 ? gaddr(x, cb) + 1024 * (size_t)x.kb : reinterpret_cast<const char*>(ld.G);
    };
    auto ldg = [&](const char* ub) { return *reinterpret_cast<const f16x8*>(ub + glane); };
    auto load_first = [&](const char* a0, const char* a1) {
#pragma unroll
        for (int j = 0; j < RS_U; ++j) {
            ring[j][0] = ldg(a0 + 1024 * j);
            ring[j][1] = ldg(a1 + 1024 * j);
        }
    };

    // One wait per unit.  A unit's B fragments of its first trip and its
    // epilogue inputs (the lane's 1/|g| per time centre and column) are issued
    // at the end of the previous unit's products, land during its epilogue,
    // and are taken together at the unit's start; the unit's descriptor comes
    // through the scalar cache.
    float sc[RS_TB][2];
    auto load_eps = [&](const Unit& x, float (&dsc)[RS_TB][2]) {
#pragma unroll
        for (int rb = 0; rb < RS_TB; ++rb) {
            const size_t row = (size_t)min(x.tc0 + rb, ld.n_tc - 1) * ld.Qp;
            if constexpr (CPLX) {  // one atom per lane: the same 1/|E_w| for its cos and sin columns
                dsc[rb][0] = dsc[rb][1] = ld.inv[row + x.cp * 32 + (lane & 31)];
            } else {
                const float* src = ld.inv + row + x.cp * 64 + (lane & 31);
                dsc[rb][0] = src[0];
                dsc[rb][1] = src[32];
            }
        }
    };
    // pass 0: the count of map entries held in LDS
    int nmap = 0;
    auto flush_map = [&]() {
        __builtin_amdgcn_wave_barrier();
        if (lane < RS_CH) {
#pragma unroll
            for (int i = 0; i < RS_MAPB; ++i)
                if (i < nmap) qmap[(size_t)S.mapu[w][i] * RS_CH + lane] = S.map[w][i][lane];
        }
        nmap = 0;
    };
    // the first unit's table fragments and epilogue inputs are requested
    // before the copies are filled, so that they arrive together
    int k = next_k(0);
    Unit cur;
    if (k < rounds) {
        cur = decode(unit_at(k));
        load_first(first_addr(true, cur, 0), first_addr(true, cur, 1));
        load_eps(cur, sc);
    }
    // the group's copies: samples [-glo, len - glo) of each channel (zero
    // outside the signal, also past the batch), 16 bytes per thread and step,
    // RS_FILL steps' loads in flight at a time
    {
        constexpr int RS_FILL = 10;
        const int per = ld.rs_len / 8, chunks = RS_CH * per;
        for (int c0 = threadIdx.x; c0 < chunks; c0 += RS_FILL * 64 * RS_WAVES) {
            f16x8 v[RS_FILL];
#pragma unroll
            for (int i = 0; i < RS_FILL; ++i) {
                const int c = c0 + i * 64 * RS_WAVES, sl = c / per, j = c - sl * per, b = ch0 + sl;
#pragma unroll
                for (int h = 0; h < 8; ++h) v[i][h] = (_Float16)0.0f;
                if (c < chunks && b < batch)
                    v[i] = *reinterpret_cast<const f16x8*>(
                        ld.shadow + 2 * ((size_t)g.n_pad + (size_t)b * ld.sh_stride + 8 * j - ld.rs_glo));
            }
#pragma unroll
            for (int i = 0; i < RS_FILL; ++i) {
                const int c = c0 + i * 64 * RS_WAVES, sl = c / per, j = c - sl * per;
                if (c < chunks) rs_res[sl * (ld.rs_stride / 8) + j] = v[i];
            }
        }
    }
    __syncthreads();
    while (k < rounds) {
        // everything issued for this unit has landed
#pragma unroll
        for (int rb = 0; rb < RS_TB; ++rb) asm volatile("" : "+v"(sc[rb][0]), "+v"(sc[rb][1]));
        const int k_next = next_k(k + 1);
        const int tc0 = cur.tc0;
        Unit nxt;
        const bool has_next = k_next < rounds;
        if (has_next) nxt = decode(unit_at(k_next));
        const char* n0 = first_addr(has_next, nxt, 0);
        const char* n1 = first_addr(has_next, nxt, 1);

        // A fragments: the lane's 8 lags of its channel's copy for row block rb
        // at k-step ks: element sl stride + glo - N_pad + m_rb + 16 ks + 8 (lane / 32)
        unsigned aoff[RS_TB];
#pragma unroll
        for (int rb = 0; rb < RS_TB; ++rb) aoff[rb] = alane + 2u * (unsigned)cur.a[rb];
        f32x16 acc[RS_TB][2];
#pragma unroll
        for (int rb = 0; rb < RS_TB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[rb][cb][v] = 0.0f;
        const char* g0 = gaddr(cur, 0);
        const char* g1 = gaddr(cur, 1);
        // each row block's next A fragment is read as soon as its two
        // products of this k-step have issued (across trips; the last trip's
        // look-ahead reads one k-step past the unit, inside the copy's guard)
        f16x8 af[RS_TB];
#pragma unroll
        for (int rb = 0; rb < RS_TB; ++rb) af[rb] = *reinterpret_cast<const f16x8*>(lds_base + aoff[rb]);
        for (int t = 0; t < cur.nk; t += RS_U) {
            const bool more = t + RS_U < cur.nk;
#pragma unroll
            for (int j = 0; j < RS_U; ++j) {
#pragma unroll
                for (int rb = 0; rb < RS_TB; ++rb) {
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        if constexpr (BF)
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, af[rb]), __builtin_bit_cast(bf16x8, ring[j][cb]),
                                acc[rb][cb], 0, 0, 0);
                        else
                            acc[rb][cb] =
                                __builtin_amdgcn_mfma_f32_32x32x16_f16(af[rb], ring[j][cb], acc[rb][cb], 0, 0, 0);
                    }
                    af[rb] = *reinterpret_cast<const f16x8*>(lds_base + aoff[rb] + 32u * (unsigned)(t + j + 1));
                }
                const size_t o = 1024 * (size_t)(cur.kb + t + RS_U + j);
                const char* a0 = more ? g0 + o : n0 + 1024 * j;
                const char* a1 = more ? g1 + o : n1 + 1024 * j;
                ring[j][0] = ldg(a0);
                ring[j][1] = ldg(a1);
            }
            // order: per k-step and row block its 2 MFMAs, then the read of the
            // row block's next A fragment; per k-step the 2 loads that refill
            // its B fragments
#pragma unroll
            for (int j = 0; j < RS_U; ++j) {
#pragma unroll
                for (int rb = 0; rb < RS_TB; ++rb) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);
            }
        }
        if (cur.nk == 0) load_first(n0, n1);
        mfma_run += (unsigned long long)cur.nk * (RS_TB * 2);
#pragma unroll
        for (int rb = 0; rb < RS_TB; ++rb)
            if (tc0 + rb >= ld.n_tc) sc[rb][0] = sc[rb][1] = 0.0f;
        // the next unit's epilogue inputs
        float sc_n[RS_TB][2];
        if (has_next) load_eps(nxt, sc_n);

        // ---- epilogue.  Lane holds column ecol0 + 32 cb of rows
        // (tc0 + rb, slot lg_row(v, lane)) (complex atoms: atom ecol0, its
        // cos and sin parts); p = (raw / |g|) / s_b.  Its lane-dependent
        // addresses use an opaque copy of the lane index, so that they are
        // formed here and not kept live across the unit loop.
        int elane = lane;
        asm volatile("" : "+v"(elane));
        const int ecol0 = cur.cp * (CPLX ? 32 : 64) + (elane & 31);
        // the raw score of accumulator block cb (complex: of the lane's atom)
        auto raw = [&](int rb, int cb, int v) {
            return CPLX ? sqrtf(acc[rb][0][v] * acc[rb][0][v] + acc[rb][1][v] * acc[rb][1][v]) : acc[rb][cb][v];
        };
        constexpr int NA = CPLX ? 1 : 2;  // atoms of a lane per row
        if (DUMP) {
#pragma unroll
            for (int rb = 0; rb < RS_TB; ++rb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int sl = lg_row(v, elane), b = ch0 + sl, tc = tc0 + rb;
                    const float ri = S.rinv[sl];
#pragma unroll
                    for (int cb = 0; cb < NA; ++cb) {
                        const int c = ecol0 + 32 * cb;
                        const float p = (raw(rb, cb, v) * sc[rb][cb]) * ri;
                        if (b < batch && tc < ld.n_tc && c < ld.Q) {
                            const long long i = lag_atom(ld, tc, c);
                            if (i >= ctl.dump_begin && i < ctl.dump_begin + ctl.dump_count)
                                ctl.dump[(size_t)b * ctl.dump_count + (i - ctl.dump_begin)] = p;
                        }
                    }
                }
        } else {
            // per row group v: max over the lane's rows and columns of |raw| / |g|,
            // then over the half-wave's 32 columns (the factor 1/s_b of a
            // channel is applied to its maximum: it is positive, and FP32
            // rounding is monotonic)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                float m = 0.0f;
#pragma unroll
                for (int rb = 0; rb < RS_TB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < NA; ++cb) m = fmaxf(m, fabsf(raw(rb, cb, v) * sc[rb][cb]));
                m = half_wave_max(m);
                if ((elane & 31) == 31) S.um[w][lg_row(v, elane)] = m;
            }
            __builtin_amdgcn_wave_barrier();
            // per channel slot (lane < 32): the unit's map entry, kept in LDS
            // with the wave's last RS_MAPB entries and written out with them,
            // and the workgroup's maximum (the running maxima are raised once,
            // when the workgroup ends: global writes here would hold up the
            // next unit's start, which waits for the memory operations issued
            // before its inputs)
            if (lane < RS_CH) {
                const float um = S.um[w][lane] * S.rinv[lane];
                S.map[w][nmap][lane] = um;
                atomicMax(&S.wmax[lane], fbits(um));
            }
            if (lane == 0) S.mapu[w][nmap] = cur.u;
            if (++nmap == RS_MAPB || !has_next) flush_map();
            __builtin_amdgcn_wave_barrier();
        }
        k = k_next;
        cur = nxt;
#pragma unroll
        for (int rb = 0; rb < RS_TB; ++rb) {
            sc[rb][0] = sc_n[rb][0];
            sc[rb][1] = sc_n[rb][1];
        }
    }
    if (!DUMP && ld.exec && lane == 0) {
        if (mfma_run) atomicAdd(&ld.exec[0], mfma_run);
        if (blockIdx.x == 0 && w == 0) atomicAdd(&ld.exec[1], 1ull);
    }
    if (!DUMP) {
        // the workgroup's maxima raise the channels' running maxima
        __syncthreads();
        if (threadIdx.x < RS_CH && ch0 + (int)threadIdx.x < batch && S.wmax[threadIdx.x])
            atomicMax(&ctl.gmax[ch0 + threadIdx.x], S.wmax[threadIdx.x]);
    }
}

// Pass 1 of the resident form, in two launches.  k_lag_rs_flag checks every
// (list slot, channel) map entry against its channel's threshold
// T = M - 2 E_b (rounded down to FP32; none without a bound) and appends the
// pairs that reach it to a list (pairs[0] counts them; pass 0 clears it).
// k_lag_rs_emit then takes the pairs one workgroup at a time and computes the
// unit's 4 x 64 scores of that channel again on the matrix cores: wave w
// runs every RS_EP-th k-step of the unit from w, as two MFMAs per k-step (the
// unit's two column blocks, the table fragments as the search reads them)
// whose A operand holds the four time centres' windows of the search copy in
// rows 0..3 and zeros below; the workgroup then adds the RS_EP partial sums
// of each score in a fixed order.
// The certified bound E_b holds for any order and grouping of these FP32
// sums.  Scores are scaled as the search scales them, and those that reach T
// are emitted (one device atomic per pair reserves the list entries).  A true
// arg-max atom has a pass-0 score of at least T, so its pair is flagged, and
// its pass-1 score, within E_b of its true score, reaches T too.
__device__ __forceinline__ float rs_threshold(const SearchCtl& ctl, int b) {
    const double eb = ctl.ebound[b];
    if (eb < 0.0) return INFINITY;
    const double Td = (double)load_gmax(&ctl.gmax[b]) - 2.0 * eb;
    float T = (float)Td;
    if ((double)T > Td) T = nextafterf(T, -INFINITY);
    return T;
}

constexpr int RS_FL_TB = 1024;                     // flag pass: threads per block
constexpr int RS_FL_PER = 2;                       // map entries per thread (channels of one slot)
constexpr int RS_FL_CHUNK = RS_FL_TB * RS_FL_PER;  // entries per block and step

__global__ void __launch_bounds__(RS_FL_TB) k_lag_rs_flag(LagDev ld, SearchCtl ctl, int batch, int n_cg,
                                                          int n_tg, int* __restrict__ pairs) {
    // a block gathers the flagged entries of its chunk in LDS and reserves
    // their list positions with one device atomic: flagged entries are
    // sparse, so per-entry or per-wave reservations on the one list counter
    // serialise
    __shared__ int s_list[RS_FL_CHUNK];
    __shared__ int s_n, s_base;
    const int perq = ld.rs_cp_per_x * n_tg, U = 8 * perq;
    const int n = n_cg * U * RS_CH;  // a multiple of RS_CH; the launch checks that it fits an int
    for (int c0 = blockIdx.x * RS_FL_CHUNK; c0 < n; c0 += gridDim.x * RS_FL_CHUNK) {
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
        const int e0 = c0 + RS_FL_PER * (int)threadIdx.x;  // RS_FL_PER divides RS_CH: one slot
        if (e0 < n) {
            const int sl = e0 / RS_CH, ch0 = e0 % RS_CH, cg = sl / U, us = sl - cg * U, x = us / perq;
            if (us - x * perq < ld.rs_cp_count[x] * n_tg) {
                const float2 m = *reinterpret_cast<const float2*>(ld.rs_map + e0);
                const float mv[RS_FL_PER] = {m.x, m.y};
#pragma unroll
                for (int j = 0; j < RS_FL_PER; ++j) {
                    const int b = cg * RS_CH + ch0 + j;
                    if (b < batch && mv[j] >= rs_threshold(ctl, b)) s_list[atomicAdd(&s_n, 1)] = e0 + j;
                }
            }
        }
        __syncthreads();
        const int cnt = s_n;
        if (threadIdx.x == 0 && cnt) s_base = atomicAdd(&pairs[0], cnt);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) pairs[1 + s_base + i] = s_list[i];
        __syncthreads();  // s_n and s_list are reused by the next chunk
    }
}

constexpr int RS_EP = 16;  // pass 1: k-step parts of a pair (one wave each, 64 columns)
constexpr int RS_EK = 2;   // pass 1: k-steps whose operands a wave loads before their MFMAs

template <bool BF, bool CPLX>
__global__ void __launch_bounds__(64 * RS_EP) k_lag_rs_emit(LagDev ld, SearchCtl ctl, const int* __restrict__ units,
                                                           int n_tg, const int* __restrict__ pairs) {
    __shared__ float part[RS_EP][RS_TB * 64];
    __shared__ unsigned s_cnt;
    __shared__ int s_base;
    const int U = 8 * ld.rs_cp_per_x * n_tg;
    const int lane = threadIdx.x & 63, part_i = threadIdx.x >> 6;
    // score (rb_t, c) of threads t < NS: 4 time centres x 64 columns, or x 32
    // complex atoms (their cos and sin columns c and 32 + c)
    constexpr int NS = RS_TB * (CPLX ? 32 : 64);
    const int t = threadIdx.x, rb_t = CPLX ? t >> 5 : t >> 6, c = CPLX ? t & 31 : t & 63;
    // A fragment: lane row lane % 32 (time centre rb of the unit when below
    // RS_TB, else a zero row), lags 8 (lane / 32) .. + 8 of each k-step
    const int arow = lane & 31, ahalf = lane >> 5;
    const f16x8 zero8 = {};
    const int np = pairs[0];
    // The flag pass lists each 2048-entry chunk of the map (four column pairs
    // of one channel group) as one run, and flagged pairs crowd onto few
    // column pairs (late BF16 orders: 3,919 pairs on 457).  Each XCD takes one
    // eighth of the list as a contiguous segment, its workgroups the
    // segment's pairs in turn, so the pairs of a column pair run together
    // and share its band in that XCD's L2.  (The grid is a multiple of 8:
    // workgroup w runs on XCD w mod 8.)
    const int xcd = blockIdx.x & 7, J = (int)gridDim.x >> 3;
    const int q_lo = (int)((long long)np * xcd / 8), q_hi = (int)((long long)np * (xcd + 1) / 8);
    const int q0 = q_lo + (int)(blockIdx.x >> 3);
    int e_next = q0 < q_hi ? pairs[1 + q0] : 0;
    for (int q = q0; q < q_hi; q += J) {
        const int e = e_next, ch = e % RS_CH, sl = e / RS_CH;
        if (q + J < q_hi) e_next = pairs[1 + q + J];  // the next pair's entry, early
        const int cg = sl / U, us = sl - cg * U, b = cg * RS_CH + ch;
        const int* d = units + (size_t)us * RS_UD;
        const int cp = d[0], tc0 = d[1], kb = d[2], nk = d[3];
        // what the epilogue needs, requested before the k-steps
        const float T = rs_threshold(ctl, b);
        const float rs = ld.rscale[b], ri = rs > 0.0f ? 1.0f / rs : 0.0f;
        const int tc = tc0 + rb_t, col = cp * (CPLX ? 32 : 64) + c;
        const float sc = t < NS && tc < ld.n_tc ? ld.inv[(size_t)tc * ld.Qp + col] : 0.0f;
        // time centre rb's window in the search copy's row b starts at
        // element b stride + 16 kb + m_rb (sample 16 kb - N_pad + m_rb); the
        // unit's descriptor holds glo - N_pad + m_rb + 16 kb (lag plans keep
        // N_pad guards: the row stride is 2 N_pad)
        const int arb = arow < RS_TB ? arow : 0;
        const char* ap = ld.shadow + 2 * ((size_t)b * ld.sh_stride + d[4 + arb] - ld.rs_glo + ld.sh_stride / 2) +
                         16 * ahalf;
        // B fragments: the two column blocks' k-step fragments, 16 bytes per lane
        const char* gp0 = reinterpret_cast<const char*>(ld.G) + ((size_t)(2 * cp) * ld.LS + kb) * 1024 + 16 * lane;
        const char* gp1 = gp0 + (size_t)ld.LS * 1024;
        f32x16 acc0 = {}, acc1 = {};
        // RS_EK k-steps' operands in flight per wave, then their MFMAs
        for (int k0 = part_i; k0 < nk; k0 += RS_EP * RS_EK) {
            f16x8 a[RS_EK], b0[RS_EK], b1[RS_EK];
#pragma unroll
            for (int i = 0; i < RS_EK; ++i) {
                const int ks = k0 + i * RS_EP;
                a[i] = b0[i] = b1[i] = zero8;
                if (ks < nk) {
                    if (arow < RS_TB) a[i] = *reinterpret_cast<const f16x8*>(ap + 32 * (size_t)ks);
                    b0[i] = *reinterpret_cast<const f16x8*>(gp0 + 1024 * (size_t)ks);
                    b1[i] = *reinterpret_cast<const f16x8*>(gp1 + 1024 * (size_t)ks);
                }
            }
#pragma unroll
            for (int i = 0; i < RS_EK; ++i) {
                if (k0 + i * RS_EP < nk) {
                    if constexpr (BF) {
                        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[i]),
                                                                       __builtin_bit_cast(bf16x8, b0[i]), acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[i]),
                                                                       __builtin_bit_cast(bf16x8, b1[i]), acc1, 0, 0, 0);
                    } else {
                        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[i], b0[i], acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[i], b1[i], acc1, 0, 0, 0);
                    }
                }
            }
        }
        // rows 0..3 (the unit's time centres) sit in accumulator slots 0..3
        // of lanes 0..31, column lane
        if (lane < 32) {
#pragma unroll
            for (int rb = 0; rb < RS_TB; ++rb) {
                part[part_i][rb * 64 + lane] = acc0[rb];
                part[part_i][rb * 64 + 32 + lane] = acc1[rb];
            }
        }
        if (threadIdx.x == 0) s_cnt = 0u;
        __syncthreads();
        bool hit = false;
        unsigned pos = 0u;
        float p = 0.0f;
        if (t < NS) {
            float raw;
            if constexpr (CPLX) {
                float a = part[0][rb_t * 64 + c], bq = part[0][rb_t * 64 + 32 + c];
#pragma unroll
                for (int i = 1; i < RS_EP; ++i) {
                    a += part[i][rb_t * 64 + c];
                    bq += part[i][rb_t * 64 + 32 + c];
                }
                raw = sqrtf(a * a + bq * bq);
            } else {
                raw = part[0][t];
#pragma unroll
                for (int i = 1; i < RS_EP; ++i) raw += part[i][t];
            }
            p = (raw * sc) * ri;
            hit = fabsf(p) >= T && tc < ld.n_tc && col < ld.Q;
            if (hit) pos = atomicAdd(&s_cnt, 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) s_base = s_cnt ? atomicAdd(&ctl.cand_count[b], (int)s_cnt) : 0;
        __syncthreads();
        const int j = s_base + (int)pos;
        if (hit && j < ctl.cap) {
            ctl.cand_idx[(size_t)b * ctl.cap + j] = (unsigned)lag_atom(ld, tc, col);
            ctl.cand_score[(size_t)b * ctl.cap + j] = p;
        }
        __syncthreads();
    }
}

// The lag table: G_q(d) in FP64, rounded to FP32 and then FP16 or BF16 (RNE;
// BF16 entries below 2^-25 are zero), written
// in MFMA B-operand order; columns past Q are zero.  Columns run log-duration
// major, qc = ld FC + (f_c n_c + c), so a tile's columns share an envelope and
// its nonzero lags.
__global__ void k_build_lag_table(GridDev g, int Q_pad, int cplx, int bf16, f16x8* __restrict__ G) {
    const int FC = g.cnt[1] * g.cnt[2];
    const int LS = 2 * g.n_pad / 16;
    const long long frags = (long long)(Q_pad / 32) * LS * 64;  // one f16x8 per (column block, k-step, lane)
    for (long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x; f < frags;
         f += (long long)gridDim.x * blockDim.x) {
        const int lane = (int)(f % 64);
        const long long qs = f / 64;
        const int ls = (int)(qs % LS);
        const int qb = (int)(qs / LS);
        // complex atoms: block 2 k holds the cos parts of atoms 32 k.., block
        // 2 k + 1 their sin parts
        const int qc = cplx ? (qb >> 1) * 32 + (lane & 31) : qb * 32 + (lane & 31);
        const bool sin_part = cplx && (qb & 1);
        f16x8 out;
        if (qc >= FC * g.cnt[3]) {
#pragma unroll
            for (int j = 0; j < 8; ++j) out[j] = (_Float16)0.0f;  // (also BF16 zero)
        } else {
            const int il = qc / FC, fcc = qc % FC;
            const double f0 = g.axis[g.off[1] + fcc / g.cnt[2]];
            const double c = g.axis[g.off[2] + fcc % g.cnt[2]];
            const double inv_dt = 1.0 / exp(g.axis[g.off[3] + il]);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int e = 16 * ls + 8 * (lane >> 5) + j;
                const double tau = (double)(e - g.n_pad) / g.fs;
                const double u = tau * inv_dt;
                const double ph = 2.0 * (c * tau * tau + f0 * tau);
                const double v = exp(-0.5 * u * u) * (sin_part ? sinpi(ph) : cospi(ph));
                // BF16 keeps FP16's floor: entries below 2^-25 are zero (error
                // <= 2^-25 per sample, as FP16's rounding), so both tables share
                // their nonzero bands
                out[j] = bf16 ? __builtin_bit_cast(_Float16, fabs(v) < 2.98023223876953125e-08
                                                                  ? (unsigned short)0
                                                                  : bf16_rne((float)v))
                              : (_Float16)(float)v;
            }
        }
        G[f] = out;
    }
}

// Per 32-column block: the first and one past the last k-step holding a
// nonzero entry (lo = LS, hi = 0 for an all-zero block).  One workgroup per block.
__global__ void __launch_bounds__(256) k_lag_span(const f16x8* __restrict__ G, int LS, int2* __restrict__ span) {
    __shared__ int lo, hi;
    if (threadIdx.x == 0) {
        lo = LS;
        hi = 0;
    }
    __syncthreads();
    const uint4* blk = reinterpret_cast<const uint4*>(G) + (size_t)blockIdx.x * LS * 64;
    int mlo = LS, mhi = 0;
    for (int f = threadIdx.x; f < LS * 64; f += 256) {
        const uint4 u = blk[f];
        // any half with a nonzero magnitude (the sign bit alone is a zero)
        if (((u.x | u.y | u.z | u.w) & 0x7fff7fffu) != 0u) {
            const int ks = f / 64;
            mlo = min(mlo, ks);
            mhi = max(mhi, ks + 1);
        }
    }
    atomicMin(&lo, mlo);
    atomicMax(&hi, mhi);
    __syncthreads();
    if (threadIdx.x == 0) span[blockIdx.x] = make_int2(lo, hi);
}

// 1/|g| in the table's atom order: inv[tc][qc] (zero past Q); Q_pad is the row
// length (the table's columns, or half of them for complex atoms)
__global__ void k_lag_inv(GridDev g, int Q_pad, const float* __restrict__ inv_norm32, float* __restrict__ inv) {
    const int FC = g.cnt[1] * g.cnt[2], n_ld = g.cnt[3];
    const int Q = FC * n_ld;
    const long long total = (long long)g.cnt[0] * Q_pad;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (long long)gridDim.x * blockDim.x) {
        const int tc = (int)(k / Q_pad), qc = (int)(k % Q_pad);
        float v = 0.0f;
        if (qc < Q) {
            const int il = qc / FC, fcc = qc % FC;
            v = inv_norm32[(long long)tc * Q + (long long)fcc * n_ld + il];
        }
        inv[k] = v;
    }
}

// Ragged plans: rho[cbk][dl] >= |g_full| / |g_w| for every atom of the
// 256-column block cbk whose window [-m, dl) ends dl lags after its centre,
// g_full its window over the longest signal.  |g_full|^2 - |g_w|^2 is at most
// the tail energy T(dl) = sum_{d >= dl} g(d)^2, and the window holds the lags
// [0, dl), so |g_w|^2 >= max(1, W(dl)), W(dl) = sum_{0 <= d < dl} g(d)^2
// (g(0) = 1): the ratio is <= sqrt(1 + T(dl) / max(1, W(dl))).  FP64 sums over
// d < D (the rest is below e^-49 dt fs); W is shrunk and the root widened by
// 1e-9 and rounded up to FP32.  One workgroup of 256 columns per block.
__global__ void __launch_bounds__(256) k_lag_rho(GridDev g, int D, float* __restrict__ rho) {
    __shared__ double wm[4];
    const int FC = g.cnt[1] * g.cnt[2], Q = FC * g.cnt[3];
    const int qc = blockIdx.x * 256 + threadIdx.x;
    const bool ok = qc < Q;
    double f0 = 0.0, c = 0.0, inv_dt = 0.0;
    if (ok) {
        const int il = qc / FC, fcc = qc % FC;
        f0 = g.axis[g.off[1] + fcc / g.cnt[2]];
        c = g.axis[g.off[2] + fcc % g.cnt[2]];
        inv_dt = 1.0 / exp(g.axis[g.off[3] + il]);
    }
    auto g2 = [&](int d) {
        const double tau = (double)d / g.fs, u = tau * inv_dt;
        const double v = exp(-0.5 * u * u) * cospi(2.0 * (c * tau * tau + f0 * tau));
        return v * v;
    };
    double tot = 0.0;  // sum_{0 <= d < D} g(d)^2
    if (ok)
        for (int d = 0; d < D; ++d) tot += g2(d);
    double T = 0.0;
    for (int d = D - 1; d >= 1; --d) {
        if (ok) T += g2(d);
        const double W = (tot - T) * (1.0 - 1e-9) - 1e-9 * tot;  // lower bound of sum_{0 <= d' < d}
        double r = sqrt(1.0 + T / fmax(1.0, W)) * (1.0 + 1e-9);
        r = wave_max(r);
        if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = r;
        __syncthreads();
        if (threadIdx.x == 0) {
            const double m = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
            rho[(size_t)blockIdx.x * D + d] = __double2float_ru(m);
            if (d == 1) rho[(size_t)blockIdx.x * D] = __double2float_ru(m);
        }
        __syncthreads();
    }
}

// Tile column-block order for tiles of `cols` columns: blocks sorted by their
// count of nonzero k-steps (longest first), dealt round-robin to the 8 XCDs'
// contiguous tile ranges so that each XCD gets the same mix.
static std::vector<int> lag_block_order(const std::vector<int2>& span, int Q, int cols) {
    const int n_cbk = (Q + cols - 1) / cols, per = cols / 32;
    std::vector<std::pair<int, int>> len(n_cbk);
    for (int k = 0; k < n_cbk; ++k) {
        int lo = 1 << 30, hi = 0;
        for (int j = 0; j < per; ++j) {
            lo = std::min(lo, span[(size_t)k * per + j].x);
            hi = std::max(hi, span[(size_t)k * per + j].y);
        }
        len[k] = {hi > lo ? hi - lo : 0, k};
    }
    std::stable_sort(len.begin(), len.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    std::vector<int> order;
    order.reserve(n_cbk);
    for (int bin = 0; bin < 8; ++bin)
        for (int s = bin; s < n_cbk; s += 8) order.push_back(len[s].second);
    return order;
}

// Resident-residual form, at plan time: the LDS copy's guards (every lag a
// unit reads, its k-steps padded to RS_U), and the column pairs by decreasing
// band dealt round-robin to the 8 XCDs (complex atoms: a column pair is the
// cos and sin blocks of 32 atoms).  The form is left out (lag_rs_cp null) for
// ragged plans, time centres off multiples of 8 samples (16-byte LDS reads)
// or copies that do not fit one workgroup's LDS.
static act_status prepare_lag_rs(act_plan_s* p, const std::vector<int2>& span, hipStream_t s) {
    if (p->desc.ragged) return ACT_OK;
    const int n_tc = p->grid.cnt[0], n = p->grid.n, n_pad = p->n_pad;
    const std::vector<int>& sh = p->tc_shift_host;
    int spread = 0;
    for (int m : sh)
        if (m % 8 != 0) return ACT_OK;
    for (int tc0 = 0; tc0 < n_tc; tc0 += RS_TB) spread = std::max(spread, sh[std::min(tc0 + RS_TB, n_tc) - 1] - sh[tc0]);
    // a unit's k-steps start at most 15 + 16 (RS_U - 1) lags before its
    // earliest row's first sample and end as far past its last row's, and
    // the A fragments look one k-step further ahead
    const int glo = (spread + 16 * RS_U - 1 + 7) / 8 * 8, ghi = (spread + 16 * RS_U + 15 + 7) / 8 * 8;
    if (glo > n_pad || (n + 7) / 8 * 8 + ghi > 2 * n_pad) return ACT_OK;
    const int len = glo + (n + 7) / 8 * 8 + ghi;
    const int stride = ((len / 8) & 1) ? len : len + 8;  // an odd count of 16-byte units per channel
    if ((size_t)RS_CH * stride * 2 + sizeof(RsScratch) > (size_t)device_lds_per_block()) return ACT_OK;
    const int n_cp = (int)span.size() / 2;
    std::vector<std::pair<int, int>> band(n_cp);
    for (int k = 0; k < n_cp; ++k) {
        const int lo = std::min(span[2 * k].x, span[2 * k + 1].x), hi = std::max(span[2 * k].y, span[2 * k + 1].y);
        band[k] = {hi > lo ? hi - lo : 0, k};
    }
    std::stable_sort(band.begin(), band.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    const int per_x = (n_cp + 7) / 8;
    std::vector<int> lists((size_t)8 * per_x, -1), counts(8, 0);
    for (int k = 0; k < n_cp; ++k) {
        const int x = k % 8;
        lists[(size_t)x * per_x + counts[x]++] = band[k].second;
    }
    // unit descriptors in list order (k-step ranges as the tiles' in
    // k_search_lag, cut to whole k-steps and padded to RS_U)
    const int n_tg = (n_tc + RS_TB - 1) / RS_TB, LS = 2 * n_pad / 16;
    std::vector<int> units((size_t)8 * per_x * n_tg * RS_UD, 0);
    long long mfma = 0;
    for (int x = 0; x < 8; ++x)
        for (int k = 0; k < counts[x]; ++k) {
            const int cp = lists[(size_t)x * per_x + k];
            const int lo = std::min(span[2 * cp].x, span[2 * cp + 1].x);
            const int hi = std::max(span[2 * cp].y, span[2 * cp + 1].y);
            for (int tg = 0; tg < n_tg; ++tg) {
                const int tc0 = tg * RS_TB, m_min = sh[tc0], m_max = sh[std::min(tc0 + RS_TB, n_tc) - 1];
                const int klo = std::max(lo, (n_pad - m_max) >> 4);
                const int khi = std::min(hi, (n_pad + n - m_min + 15) >> 4);
                const int nk = (std::max(khi - klo, 0) + RS_U - 1) / RS_U * RS_U;
                const int kb = std::min(klo + nk, LS) - nk;
                int* d = &units[(((size_t)x * per_x + k) * n_tg + tg) * RS_UD];
                d[0] = cp;
                d[1] = tc0;
                d[2] = kb;
                d[3] = nk;
                for (int rb = 0; rb < RS_TB; ++rb)
                    d[4 + rb] = glo - n_pad + sh[std::min(tc0 + rb, n_tc - 1)] + 16 * kb;
                mfma += (long long)nk * RS_TB * 2;
            }
        }
    const int ncg = (p->max_batch + RS_CH - 1) / RS_CH;
    ACT_HIP(hipMalloc((void**)&p->lag_rs_map, (size_t)ncg * 8 * per_x * n_tg * RS_CH * sizeof(float)));
    ACT_HIP(hipMalloc((void**)&p->lag_rs_pairs, (1 + (size_t)ncg * 8 * per_x * n_tg * RS_CH) * sizeof(int)));
    ACT_HIP(hipMalloc((void**)&p->lag_rs_units, units.size() * sizeof(int)));
    ACT_HIP(hipMemcpyAsync(p->lag_rs_units, units.data(), units.size() * sizeof(int), hipMemcpyHostToDevice, s));
    p->lag_rs_mfma = mfma;
    ACT_HIP(hipMalloc((void**)&p->lag_rs_cp, lists.size() * sizeof(int)));
    ACT_HIP(hipMalloc((void**)&p->lag_rs_count, 8 * sizeof(int)));
    ACT_HIP(hipMemcpyAsync(p->lag_rs_cp, lists.data(), lists.size() * sizeof(int), hipMemcpyHostToDevice, s));
    ACT_HIP(hipMemcpyAsync(p->lag_rs_count, counts.data(), 8 * sizeof(int), hipMemcpyHostToDevice, s));
    ACT_HIP(hipStreamSynchronize(s));
    p->lag_rs_cp_per_x = per_x;
    p->lag_rs_ncg = ncg;
    p->lag_rs_glo = glo;
    p->lag_rs_len = len;
    p->lag_rs_stride = stride;
    return ACT_OK;
}

// Whether a search of `batch` channels runs in the resident-residual form.
static bool lag_rs_use(const act_plan_s* p, int batch) {
    return p->lag_rs_cp && batch >= RS_CH && (batch + RS_CH - 1) / RS_CH <= p->lag_rs_ncg && p->shape.form == 0;
}

bool search_emits_certified_set(const act_plan_s* p, int batch) {
    return p->desc.dict == ACT_DICT_LAG && !p->desc.ragged && lag_rs_use(p, batch);
}

act_status build_lag_table(act_plan_s* p, hipStream_t s) {
    const int Q_pad = p->lag_q_pad;
    const int LS = 2 * p->n_pad / 16;
    const long long frags = (long long)(Q_pad / 32) * LS * 64;
    const long long blocks = std::min<long long>((frags + 255) / 256, (long long)device_cus() * 64);
    hipLaunchKernelGGL(k_build_lag_table, dim3((unsigned)blocks), dim3(256), 0, s, p->grid, Q_pad,
                       p->desc.complex_atoms, p->desc.prec == ACT_PREC_BF16 ? 1 : 0, (f16x8*)p->table);
    ACT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_lag_span, dim3((unsigned)(Q_pad / 32)), dim3(256), 0, s, (const f16x8*)p->table, LS,
                       (int2*)p->lag_span);
    ACT_HIP(hipGetLastError());
    if (p->desc.ragged) {
        hipLaunchKernelGGL(k_lag_rho, dim3((unsigned)(Q_pad / 256)), dim3(256), 0, s, p->grid, p->lag_rho_d,
                           p->lag_rho);
        ACT_HIP(hipGetLastError());
    }
    const int inv_row = p->desc.complex_atoms ? Q_pad / 2 : Q_pad;
    const long long inv_n = (long long)p->grid.cnt[0] * inv_row;
    hipLaunchKernelGGL(k_lag_inv, dim3((unsigned)std::min<long long>((inv_n + 255) / 256, device_cus() * 64LL)),
                       dim3(256), 0, s, p->grid, inv_row, p->inv_norm32, p->lag_inv);
    ACT_HIP(hipGetLastError());
    std::vector<int2> span(Q_pad / 32);
    ACT_HIP(hipMemcpyAsync(span.data(), p->lag_span, span.size() * sizeof(int2), hipMemcpyDeviceToHost, s));
    ACT_HIP(hipStreamSynchronize(s));
    const int Q = p->grid.cnt[1] * p->n_cl;
    const int ncols = p->desc.complex_atoms ? 2 * ((Q + 31) / 32 * 32) : Q;
    p->lag_span_host.resize(2 * span.size());
    for (size_t k = 0; k < span.size(); ++k) {
        p->lag_span_host[2 * k] = span[k].x;
        p->lag_span_host[2 * k + 1] = span[k].y;
    }
    std::vector<int> order = lag_block_order(span, ncols, 128);
    p->lag_order_wide = (int)order.size();
    const std::vector<int> wide = lag_block_order(span, ncols, 256);
    order.insert(order.end(), wide.begin(), wide.end());
    ACT_HIP(hipMemcpyAsync(p->lag_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, s));
    ACT_HIP(hipStreamSynchronize(s));
    return prepare_lag_rs(p, span, s);
}

// Flops one pass-0 launch executes on the matrix cores: every tile's stages
// (its rows' lag window cut to its columns' band) x 128 rows x the tile's
// columns x 128 lags x 2 -- the tiling of launch_search_lag and k_search_lag.
double lag_search_flops(const act_plan_s* p, int batch) {
    const int n_tc = p->grid.cnt[0], Q = p->grid.cnt[1] * p->n_cl, n_pad = p->n_pad, n = p->grid.n;
    if (lag_rs_use(p, batch)) {
        // resident-residual form: per (channel group, unit) its k-steps x 4
        // row blocks x 2 column blocks, counted when the units were laid out
        const int n_cg = (batch + RS_CH - 1) / RS_CH;
        return (double)p->lag_rs_mfma * n_cg * (32.0 * 32.0 * 16.0 * 2.0);
    }
    const bool cplx = p->desc.complex_atoms != 0;
    const int ncols = cplx ? 2 * ((Q + 31) / 32 * 32) : Q;
    int CB = 1;
    while (CB < batch && CB < 32) CB *= 2;
    const int TB = LG_ROWS / CB, n_cg = (batch + CB - 1) / CB, n_tg = (n_tc + TB - 1) / TB;
    const int cols = (batch > 1 || cplx) ? 256 : 128, per = cols / 32, n_cbk = (ncols + cols - 1) / cols;
    const int LS = 2 * n_pad / 16;
    long long stages = 0;
    for (int k = 0; k < n_cbk; ++k) {
        int klo = LS, khi = 0;
        for (int j = 0; j < per; ++j) {
            klo = std::min(klo, p->lag_span_host[2 * (k * per + j)]);
            khi = std::max(khi, p->lag_span_host[2 * (k * per + j) + 1]);
        }
        for (int tg = 0; tg < n_tg; ++tg) {
            const int tc0 = tg * TB, tc_last = std::min(tc0 + TB, n_tc) - 1;
            const int m_min = p->tc_shift_host[tc0], m_max = p->tc_shift_host[tc_last];
            const int e_first = std::max((n_pad - m_max) / LG_S, 16 * klo / LG_S) * LG_S;
            const int e_end = std::min(std::min(2 * n_pad, n_pad + n - m_min), 16 * khi);
            const int ns = e_end > e_first ? (e_end - e_first + LG_S - 1) / LG_S : 0;
            stages += (long long)ns * n_cg;
        }
    }
    return (double)stages * LG_ROWS * cols * LG_S * 2.0;
}

// FP32 accumulation chain of one score: at most one rounding per lag (2 N_pad)
// plus the scalings.
int lag_chain_length(int n_pad) { return 2 * n_pad + 2; }

// channels per tile: the smallest power of two covering the batch, at most 32
static int lag_channel_block(int batch) {
    int CB = 1;
    while (CB < batch && CB < 32) CB *= 2;
    return CB;
}

// Ragged batches, per call: channels by decreasing length (ties: lower index
// first) and, per group of CB channels, the prefix of the time groups of its
// longest signal.  Lengths outside [0, n_max] count as 0 (flagged elsewhere).
__global__ void __launch_bounds__(1024) k_lag_ragged_prep(const int* __restrict__ len, int batch, int n_max, int div,
                                                          int CB, int TB, int* __restrict__ perm,
                                                          int* __restrict__ rows) {
    for (int b = threadIdx.x; b < batch; b += blockDim.x) {
        int nb = len[b];
        nb = (nb < 0 || nb > n_max) ? 0 : nb;
        int rank = 0;
        for (int j = 0; j < batch; ++j) {
            int nj = len[j];
            nj = (nj < 0 || nj > n_max) ? 0 : nj;
            rank += (nj > nb || (nj == nb && j < b)) ? 1 : 0;
        }
        perm[rank] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int ncg = (batch + CB - 1) / CB;
        int acc = 0;
        for (int cg = 0; cg < ncg; ++cg) {
            rows[cg] = acc;
            int n = len[perm[cg * CB]];
            n = (n < 0 || n > n_max) ? 0 : n;
            acc += (n / div + TB - 1) / TB;
        }
        rows[ncg] = acc;
    }
}

act_status launch_lag_ragged_prep(act_plan_s* p, int batch, hipStream_t s) {
    const int CB = lag_channel_block(batch);
    hipLaunchKernelGGL(k_lag_ragged_prep, dim3(1), dim3(1024), 0, s, p->call_len, batch, p->grid.n,
                       p->desc.ragged_tc_div, CB, LG_ROWS / CB, p->perm, p->lag_rows);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

act_status launch_search_lag(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s) {
    LagDev ld{};
    ld.G = (const f16x8*)p->table;
    ld.inv = p->lag_inv;
    ld.span = (const int2*)p->lag_span;
    ld.tc_shift = p->tc_shift;
    ld.shadow = (const char*)p->shadow_alloc;
    ld.sh_stride = p->sh_stride;
    ld.rscale = p->rscale;
    ld.LS = 2 * p->n_pad / 16;
    ld.Q = p->grid.cnt[1] * p->n_cl;
    const bool cplx = p->desc.complex_atoms != 0;
    ld.Qp = cplx ? p->lag_q_pad / 2 : p->lag_q_pad;  // row length of the inverse norms (atoms)
    ld.FC = p->grid.cnt[1] * p->grid.cnt[2];
    ld.n_ld = p->grid.cnt[3];
    ld.n_tc = p->grid.cnt[0];
    const bool rag = p->desc.ragged != 0;
    ld.perm = p->perm;
    ld.rows = p->lag_rows;
    ld.rho = p->lag_rho;
    ld.rho_d = p->lag_rho_d;
    ld.div = rag ? p->desc.ragged_tc_div : 1;
    ld.exec = (ctl.pass == 0 && !ctl.dump) ? p->exec_count : nullptr;
    if (rag && ctl.dump) {
        set_error("act_correlate: the ragged lag-table search has no score dump");
        return ACT_ERR_UNSUPPORTED;
    }
    if (lag_rs_use(p, batch) && !rag) {
        ld.rs_cp = p->lag_rs_cp;
        ld.rs_cp_count = p->lag_rs_count;
        ld.rs_cp_per_x = p->lag_rs_cp_per_x;
        ld.rs_glo = p->lag_rs_glo;
        ld.rs_len = p->lag_rs_len;
        ld.rs_stride = p->lag_rs_stride;
        const int n_cg = (batch + RS_CH - 1) / RS_CH, n_tg = (ld.n_tc + RS_TB - 1) / RS_TB;
        // every (channel group, XCD) pair gets the same number of workgroups
        const int per = 8 * n_cg, cus = device_cus();
        const dim3 grid((unsigned)((cus + per - 1) / per * per)), blk(64 * RS_WAVES);
        const size_t dyn = (size_t)RS_CH * ld.rs_stride * 2 + sizeof(RsScratch);
        const bool bf = p->desc.prec == ACT_PREC_BF16, cx = p->desc.complex_atoms != 0;
        ld.rs_map = p->lag_rs_map;
        // pass 0 builds the max map (and clears pass 1's list), pass 1 lists
        // the flagged pairs and emits from them
        ld.rs_pairs = p->lag_rs_pairs;
        if (ctl.pass && !ctl.dump) {
            const long long n = (long long)n_cg * 8 * ld.rs_cp_per_x * n_tg * RS_CH;
            if (n > INT_MAX) {
                set_error("lag-table search: the resident form's map exceeds 2^31 entries");
                return ACT_ERR_UNSUPPORTED;
            }
            hipLaunchKernelGGL(k_lag_rs_flag, dim3((unsigned)std::min<long long>((n + RS_FL_CHUNK - 1) / RS_FL_CHUNK, cus)), dim3(RS_FL_TB),
                               0, s, ld, ctl, batch, n_cg, n_tg, p->lag_rs_pairs);
            ACT_HIP(hipGetLastError());
            // (BF16 lag tables hold real atoms only); the emission grid is a
            // multiple of 8: its workgroups split the list by XCD
            const unsigned emit_grid = (unsigned)((2 * cus + 7) / 8 * 8);
            if (bf)
                hipLaunchKernelGGL((k_lag_rs_emit<true, false>), dim3(emit_grid), dim3(64 * RS_EP), 0, s, ld, ctl,
                                   p->lag_rs_units, n_tg, p->lag_rs_pairs);
            else if (cx)
                hipLaunchKernelGGL((k_lag_rs_emit<false, true>), dim3(emit_grid), dim3(64 * RS_EP), 0, s, ld, ctl,
                                   p->lag_rs_units, n_tg, p->lag_rs_pairs);
            else
                hipLaunchKernelGGL((k_lag_rs_emit<false, false>), dim3(emit_grid), dim3(64 * RS_EP), 0, s, ld, ctl,
                                   p->lag_rs_units, n_tg, p->lag_rs_pairs);
            ACT_HIP(hipGetLastError());
            return ACT_OK;
        }
#define RS_LAUNCH(D, B, C)                                                                                        \
    hipLaunchKernelGGL((k_search_lag_rs<D, B, C>), grid, blk, dyn, s, p->grid, ld, ctl, p->lag_rs_units, batch, \
                       n_cg, n_tg)
        if (bf) {
            if (ctl.dump) RS_LAUNCH(true, true, false);
            else RS_LAUNCH(false, true, false);
        } else if (cx) {
            if (ctl.dump) RS_LAUNCH(true, false, true);
            else RS_LAUNCH(false, false, true);
        } else {
            if (ctl.dump) RS_LAUNCH(true, false, false);
            else RS_LAUNCH(false, false, false);
        }
#undef RS_LAUNCH
        ACT_HIP(hipGetLastError());
        return ACT_OK;
    }
    // rows: the smallest power of two of channels covering the batch (at most
    // 32) times the time centres that fill 128 rows
    int CB = lag_channel_block(batch);
    ld.CB = CB;
    ld.TB = LG_ROWS / CB;
    ld.cb_log2 = 0;
    while ((1 << ld.cb_log2) < CB) ++ld.cb_log2;
    const int n_cg = (batch + CB - 1) / CB;
    const int n_tg = (ld.n_tc + ld.TB - 1) / ld.TB;
    // one channel of real atoms: 128 columns per tile (twice the tiles);
    // otherwise 256 (complex atoms: 128 atoms, cos and sin blocks paired)
    const bool wide = batch > 1 || cplx || rag;
    const int cols = wide ? 256 : 128;
    const int ncols = cplx ? 2 * ((ld.Q + 31) / 32 * 32) : ld.Q;
    const int n_cbk = (ncols + cols - 1) / cols;
    ld.order = p->lag_order + (wide ? p->lag_order_wide : 0);
    // ragged: the tile count is known on the device only; a full persistent grid
    const long long tiles = rag ? LLONG_MAX / 2 : (long long)n_cbk * n_cg * n_tg;
    long long blocks = (tiles + 7) / 8 * 8;
    const long long cap = grid_cap(p, 1);  // LDS: one workgroup per CU
    blocks = blocks < cap ? blocks : cap;
    const dim3 grid((unsigned)blocks), blk(256);
#define LAG_LAUNCH(WCB, RR, DD, CX, RG)                                                                       \
    hipLaunchKernelGGL((k_search_lag<WCB, RR, DD, CX, RG, false>), grid, blk, 0, s, p->grid, ld, ctl, batch, n_cbk,  \
                       n_cg, n_tg)
#define LAG_LAUNCH_BF(WCB, RR, DD)                                                                            \
    hipLaunchKernelGGL((k_search_lag<WCB, RR, DD, false, false, true>), grid, blk, 0, s, p->grid, ld, ctl, batch,  \
                       n_cbk, n_cg, n_tg)
    if (p->desc.prec == ACT_PREC_BF16) {
        if (wide) {
            if (ctl.dump) LAG_LAUNCH_BF(2, false, true);
            else if (ctl.pass) LAG_LAUNCH_BF(2, true, false);
            else LAG_LAUNCH_BF(2, false, false);
        } else {
            if (ctl.dump) LAG_LAUNCH_BF(1, false, true);
            else if (ctl.pass) LAG_LAUNCH_BF(1, true, false);
            else LAG_LAUNCH_BF(1, false, false);
        }
    } else if (rag) {
        if (ctl.pass) LAG_LAUNCH(2, true, false, false, true);
        else LAG_LAUNCH(2, false, false, false, true);
    } else if (cplx) {
        if (ctl.dump) LAG_LAUNCH(2, false, true, true, false);
        else if (ctl.pass) LAG_LAUNCH(2, true, false, true, false);
        else LAG_LAUNCH(2, false, false, true, false);
    } else if (wide) {
        if (ctl.dump) LAG_LAUNCH(2, false, true, false, false);
        else if (ctl.pass) LAG_LAUNCH(2, true, false, false, false);
        else LAG_LAUNCH(2, false, false, false, false);
    } else {
        if (ctl.dump) LAG_LAUNCH(1, false, true, false, false);
        else if (ctl.pass) LAG_LAUNCH(1, true, false, false, false);
        else LAG_LAUNCH(1, false, false, false, false);
    }
#undef LAG_LAUNCH
#undef LAG_LAUNCH_BF
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

}  // namespace act
