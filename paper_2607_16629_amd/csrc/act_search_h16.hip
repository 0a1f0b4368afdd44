// act_search_h16.hip -- coarse search with the dictionary synthesised from
// shift-invariant factor tables on the FP16 matrix cores
// (v_mfma_f32_32x32x16_f16, FP32 accumulation).
//
// Same factorisation as the FP32 synthesised search (angle-sum identity on the
// real part of Eq. (1), time centres on integer samples m):
//   P[cl][(fc,b)] = sum_n U_cl(n-m) [C_fc(n-m) r_b(n)] - V_cl(n-m) [S_fc(n-m) r_b(n)]
// A = [U | V]: FP16 copies of the FP64-evaluated envelope-chirp factors (rows cl).
// B = the carrier-modulated residuals: the FP16 carrier table times the FP16
//     search copy of the residual (scaled by a power of two per channel), one
//     packed FP16 multiply per two samples, formed per stage in LDS.
// Columns are (f_c, channel) pairs, so up to 64 channels share every A
// fragment.  P is never written to memory.
//
// Workgroup = 4 waves stacked along the rows, each 32*WRB rows x 32*WCB columns:
//   WRB = 2, WCB = 4: 256 cl rows x 128 columns (channel groups of up to 64)
//   WRB = 2, WCB = 2: 256 cl rows x 64 columns (one channel, 64 f_c)
// The B operand of a 128-sample stage sits in LDS in MFMA operand order (each
// k-step and column block is one contiguous KiB: 16-byte conflict-free reads);
// A fragments stream from L2 in blocks of two k-steps, one block ahead.
//
// Certified emission with per-atom error bounds: every score p~_a carries a
// bound E_a = rho_a * mul_b + add_b on |p~_a - p_a|, where rho_a is the ratio
// |envelope| / |atom| over the atom's own window of samples.  The running
// maximum L of the lower bounds |p~| - E over the channel never exceeds the
// true maximum, so every atom with |p~_a| + E_a >= L is emitted (with its upper
// bound); the FP64 rescoring then decides among them exactly.
#include <type_traits>

#include "act_emit.h"

namespace act {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int H_KS = 128;             // samples per LDS stage
constexpr int H_KSTEPS = H_KS / 16;   // MFMA k-steps per stage
constexpr int H_WRB = 2;              // 32-row blocks per wave
constexpr int H_RW = 4 * 32 * H_WRB;  // rows per workgroup

__device__ __forceinline__ int h_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

struct H16Dev {
    const _Float16* U;       // [n_cl][W] envelope-chirp factors, column e = lag + n_pad
    const _Float16* V;
    const _Float16* C;       // [n_fc][W] carrier factors
    const _Float16* S;
    const float* inv_norm;   // plain plans: [atoms] FP32 1/|g|
    const int* tc_shift;     // plain plans: [n_tc] integer sample of each time centre
    const double* lag_energy;  // ragged plans: [n_fc][n_cl][W] prefix sums of g(d)^2
    const double* env_q;     // [n_ld][W] prefix sums of E(d)^2
    const _Float16* shadow;  // [B][n_pad] fl16(fl32(r) s_b), zero past each length
    const float* rscale;     // [B] s_b
    const double* ebmul;     // [B] per-atom bound factor (times rho_a)
    const int* perm;         // ragged plans: channels in order of decreasing length
    unsigned* tmax;          // [B][n_tc] largest upper bound of the pass-0 tiles (float bits)
    const int* ld_half;      // [n_ld] half-support (samples) of each log-duration's envelope
    const float* inv_full;   // ragged plans: [n_fc][n_cl] 1/|g| over all lags (interior atoms)
    int W, n_cl, n_ld, n_tc;
    int cut;                 // 1: skip samples outside the supports
    // pass-0 searches: [0] += MFMA instructions the launch executed (every
    // wave's), [1] += 1 per launch; NULL when not counting
    unsigned long long* exec;
};

// Rows are ordered log-duration major (row = il * n_c + ic), so a block of
// rows spans few envelope widths and can skip samples outside their support;
// the atom index keeps cl = ic * n_ld + il.
__device__ __forceinline__ int h_cl(int row, int n_c, int n_ld) { return (row % n_c) * n_ld + row / n_c; }

// Largest half-support over the rows [r0, r1] (clipped to the dictionary); -1 if none.
__device__ __forceinline__ int h_support(const H16Dev& hd, int n_c, int r0, int r1) {
    r1 = min(r1, hd.n_cl - 1);
    if (r0 > r1) return -1;
    int D = 0;
    for (int il = r0 / n_c; il <= r1 / n_c; ++il) D = max(D, hd.ld_half[il]);
    return D;
}

struct H16Tile {
    int tc, m;         // time centre index and its integer sample
    int row0;          // first cl row
    int fc0, cpf;      // first f_c; channels per f_c in the column set
    int slot0, nslot;  // first channel slot of the group, slots in the batch
    int n_pad_ch;      // samples covered by the stages (multiple of H_KS)
};

constexpr int H_NLD = 32;  // log-durations tabulated per tile for the ragged bounds

template <int WCB>
struct H16Lds {
    f16x8 bc[H_KSTEPS * WCB * 64];  // C-part of B, [k-step][column block][lane]
    f16x8 bs[H_KSTEPS * WCB * 64];  // (-S)-part of B
    unsigned cm[32 * WCB];          // column maxima of the lower bounds (float bits)
    unsigned cu[32 * WCB];          // column maxima of the upper bounds (float bits)
    float M[64];                    // per-slot running maximum used for emission
    float env[64 * H_NLD];          // |E_w| of the tile: per row (plain) or per (slot, ld) (ragged)
    int rowcl[H_RW];                // atom row cl of each tile row (-1 past the dictionary)
    int rowld[H_RW];                // log-duration index of each tile row
};

__device__ __forceinline__ double window_sum(const double* q, int e_lo, int e_hi) {
    return q[e_hi] - (e_lo > 0 ? q[e_lo - 1] : 0.0);
}

// Column c of a tile: its f_c and channel, the channel's length, and whether
// it takes part (exists, has this time centre, is searched in this pass).
struct H16Col {
    int fc, b, n;
    bool ok;
};

template <bool RERUN, bool DUMP, bool RAGGED>
__device__ __forceinline__ H16Col h16_col(const GridDev& g, const H16Dev& hd, const SearchCtl& ctl,
                                          const H16Tile& t, int c) {
    H16Col col;
    col.fc = t.fc0 + c / t.cpf;
    const int slot = t.slot0 + c % t.cpf;
    col.ok = col.fc < g.cnt[1] && slot < t.nslot;
    col.b = 0;
    col.n = g.n;
    if (col.ok) {
        col.b = RAGGED ? hd.perm[slot] : slot;
        if (RAGGED) {
            col.n = ctl.len[col.b];
            col.ok = col.n >= 0 && col.n <= g.n && t.tc < col.n / g.ragged_div;  // has this time centre
        }
        col.ok = col.ok && (DUMP || (ctl.ebound[col.b] >= 0.0 && (!RERUN || ctl.need_rerun[col.b])));
    }
    return col;
}

template <int WCB, bool RERUN, bool DUMP, bool RAGGED>
__device__ __forceinline__ void h16_tile(const GridDev& g, const H16Dev& hd, const SearchCtl& ctl, const H16Tile& t,
                         H16Lds<WCB>& L, unsigned& stages_run) {
    constexpr int TC = 32 * WCB;   // columns per workgroup
    // wave-uniform values live in scalar registers
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n_fc = g.cnt[1];
    const int W = hd.W;

    const int n_c = g.cnt[2];
    // row -> (cl, log-duration) of the tile, read by the epilogue; the previous
    // tile ended with a barrier and the first stage starts with one
    {
        const int row = t.row0 + (int)threadIdx.x;
        L.rowcl[threadIdx.x] = row < hd.n_cl ? h_cl(row, n_c, hd.n_ld) : -1;
        L.rowld[threadIdx.x] = row < hd.n_cl ? row / n_c : 0;
    }
    // A rows of this lane
    int arow[H_WRB];
#pragma unroll
    for (int rb = 0; rb < H_WRB; ++rb) {
        const int row = t.row0 + w * 32 * H_WRB + rb * 32 + (lane & 31);
        arow[rb] = row < hd.n_cl ? h_cl(row, n_c, hd.n_ld) : 0;
    }
    // samples that can matter: lags within the widest half-support of the
    // workgroup's rows (stages) and of this wave's rows (32-sample blocks)
    const int D_full = g.n_pad;  // dense: every lag
    int D_wg = h_support(hd, n_c, t.row0, t.row0 + H_RW - 1);
    int D_w = h_support(hd, n_c, t.row0 + w * 32 * H_WRB, t.row0 + (w + 1) * 32 * H_WRB - 1);
    if (!hd.cut) {
        D_wg = D_wg < 0 ? -1 : D_full;
        D_w = D_w < 0 ? -1 : D_full;
    }
    const int n_first = max(0, t.m - D_wg) / H_KS * H_KS;
    const int n_end = D_wg < 0 ? 0 : min(t.n_pad_ch, t.m + D_wg + 1);
    f32x16 acc[H_WRB][WCB];
#pragma unroll
    for (int rb = 0; rb < H_WRB; ++rb)
#pragma unroll
        for (int cb = 0; cb < WCB; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[rb][cb][v] = 0.0f;

    // this thread's B column for the whole tile (f_c, channel, row pointers)
    const int fm_c = threadIdx.x % TC;
    const _Float16 *fm_r, *fm_cs, *fm_ss;
    bool fm_ok;
    {
        const int fc = t.fc0 + fm_c / t.cpf, slot = t.slot0 + fm_c % t.cpf;
        fm_ok = fc < n_fc && slot < t.nslot;
        const int b = fm_ok ? (RAGGED ? hd.perm[slot] : slot) : 0;
        fm_r = hd.shadow + (size_t)b * g.n_pad;
        fm_cs = hd.C + (size_t)(fm_ok ? fc : 0) * W + (g.n_pad - t.m);
        fm_ss = hd.S + (size_t)(fm_ok ? fc : 0) * W + (g.n_pad - t.m);
    }
    for (int n0 = n_first; n0 < n_end; n0 += H_KS) {
        constexpr int KB = 2;
        static_assert(H_KSTEPS == 4 * KB, "four blocks per stage");
        const bool run = n0 + H_KS - 1 >= t.m - D_w && n0 <= t.m + D_w;
        stages_run += run ? 1u : 0u;
        f16x8 ua0[H_WRB][KB], va0[H_WRB][KB], ua1[H_WRB][KB], va1[H_WRB][KB];
        auto load_blk = [&](f16x8 (&ua)[H_WRB][KB], f16x8 (&va)[H_WRB][KB], int blk) {
            const int eb = n0 + 16 * KB * blk - t.m + g.n_pad + 8 * KB * (lane >> 5);
#pragma unroll
            for (int rb = 0; rb < H_WRB; ++rb) {
                const f16x8* up = reinterpret_cast<const f16x8*>(hd.U + (size_t)arow[rb] * W + eb);
                const f16x8* vp = reinterpret_cast<const f16x8*>(hd.V + (size_t)arow[rb] * W + eb);
#pragma unroll
                for (int j = 0; j < KB; ++j) {
                    ua[rb][j] = up[j];
                    va[rb][j] = vp[j];
                }
            }
        };
        // the first block's A fragments load while B is formed
        if (run) load_blk(ua0, va0, 0);
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
        // ---- B stage: each thread forms 8-sample chunks of its column; k-slot
        // order: in each 32-sample block, half h and k-step s' of a lane hold
        // samples 16 h + 8 s' + (0..7), so a lane's A operands of two k-steps
        // are 32 contiguous bytes (a lane pair reads 64 contiguous bytes)
        {
            constexpr int NQ = TC * H_KSTEPS * 2 / 256;  // chunks per thread
            constexpr int HALF = NQ / 2;
            const int c = fm_c;
            const bool ok = fm_ok;
            const _Float16* rp = fm_r + n0;
            const _Float16* cp = fm_cs + n0;
            const _Float16* sp = fm_ss + n0;
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                f16x8 r8[HALF], c8[HALF], s8[HALF];
#pragma unroll
                for (int i = 0; i < HALF; ++i) {  // loads first, then the products
                    const int no = 8 * ((hf * HALF + i) * (256 / TC) + threadIdx.x / TC);
                    r8[i] = *reinterpret_cast<const f16x8*>(rp + no);
                    c8[i] = *reinterpret_cast<const f16x8*>(cp + no);
                    s8[i] = *reinterpret_cast<const f16x8*>(sp + no);
                }
#pragma unroll
                for (int i = 0; i < HALF; ++i) {
                    const int no = 8 * ((hf * HALF + i) * (256 / TC) + threadIdx.x / TC);
                    const int s = 2 * (no >> 5) + ((no & 15) >> 3), h = (no >> 4) & 1;
                    f16x8 cv = c8[i] * r8[i], sv = -s8[i] * r8[i];
                    if (!ok) {
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            cv[j] = (_Float16)0.0f;
                            sv[j] = (_Float16)0.0f;
                        }
                    }
                    const int slot_lds = (s * WCB + (c >> 5)) * 64 + (c & 31) + 32 * h;
                    L.bc[slot_lds] = cv;
                    L.bs[slot_lds] = sv;
                }
            }
        }
        __syncthreads();

        // ---- MFMA over the stage: four blocks of two k-steps in two register
        // buffers, each block's A fragments loaded while the previous block
        // runs; a wave whose rows' supports miss the stage skips it.  The
        // scheduling barriers keep that order: at this register budget the
        // compiler would otherwise move each load next to its first use and
        // wait out the full L2 latency before every block.
        if (run) {
            auto run_blk = [&](const f16x8 (&ua)[H_WRB][KB], const f16x8 (&va)[H_WRB][KB], int blk) {
#pragma unroll
                for (int sp = 0; sp < KB; ++sp) {
                    const int s = KB * blk + sp;
#pragma unroll
                    for (int cb = 0; cb < WCB; ++cb) {
                        const f16x8 bC = L.bc[(s * WCB + cb) * 64 + lane];
                        const f16x8 bS = L.bs[(s * WCB + cb) * 64 + lane];
#pragma unroll
                        for (int rb = 0; rb < H_WRB; ++rb) {
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ua[rb][sp], bC, acc[rb][cb], 0, 0, 0);
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(va[rb][sp], bS, acc[rb][cb], 0, 0, 0);
                        }
                    }
                }
            };
            load_blk(ua1, va1, 1);
            __builtin_amdgcn_sched_barrier(0);
            run_blk(ua0, va0, 0);
            __builtin_amdgcn_sched_barrier(0);
            load_blk(ua0, va0, 2);
            __builtin_amdgcn_sched_barrier(0);
            run_blk(ua1, va1, 1);
            __builtin_amdgcn_sched_barrier(0);
            load_blk(ua1, va1, 3);
            __builtin_amdgcn_sched_barrier(0);
            run_blk(ua0, va0, 2);
            run_blk(ua1, va1, 3);
        }
    }

    // ---- epilogue: scores and per-atom bounds, one column block at a time
    const int e_lo = g.n_pad - t.m;
    // |E_w| (rounded up) of the envelope over each window of the tile: the
    // window depends on the log-duration and, for ragged plans, on the
    // signal's length (one entry per (slot, ld)); plain plans index by row.
    const bool env_tab = !DUMP && (!RAGGED || hd.n_ld <= H_NLD);
    if (env_tab) {
        if (RAGGED) {
            for (int q = threadIdx.x; q < t.cpf * hd.n_ld; q += 256) {
                const int sl = q / hd.n_ld, ld = q % hd.n_ld;
                float v = 0.0f;
                if (t.slot0 + sl < t.nslot) {
                    int n = ctl.len[hd.perm[t.slot0 + sl]];
                    n = (n < 0 || n > g.n) ? 0 : n;
                    if (t.tc < n / g.ragged_div)
                        v = (float)(sqrt(window_sum(hd.env_q + (size_t)ld * W, e_lo, n - 1 - t.m + g.n_pad)) *
                                    (1.0 + 1e-6));
                }
                L.env[sl * H_NLD + ld] = v;
            }
        } else {
            const int row = t.row0 + threadIdx.x;
            float v = 0.0f;
            if (row < hd.n_cl)
                v = (float)(sqrt(window_sum(hd.env_q + (size_t)(row / n_c) * W, e_lo, g.n - 1 - t.m + g.n_pad)) *
                            (1.0 + 1e-6));
            L.env[threadIdx.x] = v;
        }
    }
    __syncthreads();
    float emax[WCB];  // largest bound of this lane's atoms, per column block
    // column blocks unrolled by hand (compile-time cb): a rolled loop would
    // index the accumulators dynamically and move them to scratch memory
    auto for_cb = [&](auto f) {
        f(std::integral_constant<int, 0>{});
        f(std::integral_constant<int, 1>{});
        if constexpr (WCB > 2) {
            f(std::integral_constant<int, 2>{});
            f(std::integral_constant<int, 3>{});
        }
    };
    for_cb([&](auto cbc) {
        constexpr int cb = decltype(cbc)::value;
        const H16Col col = h16_col<RERUN, DUMP, RAGGED>(g, hd, ctl, t, cb * 32 + (lane & 31));
        const float rinv = col.ok ? 1.0f / hd.rscale[col.b] : 0.0f;
        // per-channel bound parts as FP32, rounded up
        const float mul = col.ok && !DUMP ? (float)(hd.ebmul[col.b] * (1.0 + 1e-6)) : 0.0f;
        const float add = col.ok && !DUMP ? (float)(ctl.ebound[col.b] * (1.0 + 1e-6)) : 0.0f;
        const int e_hi = col.n - 1 - t.m + g.n_pad;
        const int slot_l = (cb * 32 + (lane & 31)) % t.cpf;
        float em = 0.0f;
#pragma unroll
        for (int rb = 0; rb < H_WRB; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int rl = w * 32 * H_WRB + rb * 32 + h_row(v, lane);  // row in the tile
                const int cl = L.rowcl[rl];
                float p = 0.0f;
                if (col.ok && cl >= 0) {
                    float inv;
                    if (RAGGED) {
                        const int Dr = hd.ld_half[L.rowld[rl]];
                        if (t.m >= Dr && t.m + Dr <= col.n - 1) {
                            // the support lies inside the signal: the window misses
                            // at most 2^-48 of |g|^2 (>= 1), far inside the bound's slack
                            inv = hd.inv_full[(size_t)col.fc * hd.n_cl + cl];
                        } else {
                            // FP64 window of the prefix sums, then FP32 (correctly
                            // rounded) square root and division: <= 2.5 u relative
                            const double e2 = window_sum(hd.lag_energy + ((size_t)col.fc * hd.n_cl + cl) * W,
                                                         e_lo, e_hi);
                            inv = e2 > 0.0 ? 1.0f / sqrtf((float)e2) : 0.0f;
                        }
                    } else {
                        inv = hd.inv_norm[((size_t)t.tc * n_fc + col.fc) * hd.n_cl + cl];
                    }
                    p = (acc[rb][cb][v] * inv) * rinv;
                    if (DUMP) {
                        const long long idx = ((long long)t.tc * n_fc + col.fc) * hd.n_cl + cl;
                        if (idx >= ctl.dump_begin && idx < ctl.dump_begin + ctl.dump_count)
                            ctl.dump[(size_t)col.b * ctl.dump_count + (idx - ctl.dump_begin)] = p;
                    } else {
                        float envn;
                        if (!RAGGED) {
                            envn = L.env[rl];
                        } else if (env_tab) {
                            envn = L.env[slot_l * H_NLD + L.rowld[rl]];
                        } else {
                            envn = (float)(sqrt(window_sum(hd.env_q + (size_t)L.rowld[rl] * W, e_lo, e_hi)) *
                                           (1.0 + 1e-6));
                        }
                        // rho_a = |E_w| / |g_w| and E_a, rounded up (1 + 2^-20 covers
                        // the FP32 products), plus room for the rounding of |p| -+ E
                        const float ef = (envn * inv * mul + add) * 1.00000095f + 2.4e-7f * fabsf(p);
                        em = fmaxf(em, ef);
                    }
                }
                acc[rb][cb][v] = p;
                // bound the loads in flight (register pressure of the unrolled epilogue)
                if ((v & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
        emax[cb] = em;
    });
    if (DUMP) return;

    // column maxima of |p~| - E (E of the lane's atoms bounded by emax, which
    // only lowers the lower bounds: still valid)
    if (threadIdx.x < TC) {
        L.cm[threadIdx.x] = 0u;
        L.cu[threadIdx.x] = 0u;
    }
    __syncthreads();
    for_cb([&](auto cbc) {
        constexpr int cb = decltype(cbc)::value;
        float m = 0.0f;
#pragma unroll
        for (int rb = 0; rb < H_WRB; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) m = fmaxf(m, fabsf(acc[rb][cb][v]));
        float mu = m + emax[cb];
        m = fmaxf(m - emax[cb], 0.0f);
        m = fmaxf(m, __shfl_xor(m, 32, 64));
        mu = fmaxf(mu, __shfl_xor(mu, 32, 64));
        if (lane < 32) {
            atomicMax(&L.cm[cb * 32 + lane], fbits(m));
            atomicMax(&L.cu[cb * 32 + lane], fbits(mu));
        }
    });
    __syncthreads();
    const int nslots = min(t.cpf, t.nslot - t.slot0);
    if (threadIdx.x < nslots) {
        const int sl = threadIdx.x;
        const int b = RAGGED ? hd.perm[t.slot0 + sl] : t.slot0 + sl;
        float M = INFINITY;
        if (ctl.ebound[b] >= 0.0 && (!RERUN || ctl.need_rerun[b])) {
            float wm = 0.0f, wu = 0.0f;
            for (int c = sl; c < TC; c += t.cpf) {
                wm = fmaxf(wm, bitsf(L.cm[c]));
                wu = fmaxf(wu, bitsf(L.cu[c]));
            }
            const float cur = load_gmax(&ctl.gmax[b]);
            M = cur;
            if (!RERUN) {
                if (wm > cur) M = fmaxf(bitsf(atomicMax(&ctl.gmax[b], fbits(wm))), wm);
                // this time centre's largest upper bound: the rerun pass skips
                // time centres that cannot hold a candidate
                atomicMax(&hd.tmax[(size_t)b * hd.n_tc + t.tc], fbits(wu));
            }
        }
        L.M[sl] = M;
    }
    __syncthreads();
    // emission: every atom whose upper bound reaches the running maximum lower bound
    for_cb([&](auto cbc) {
        constexpr int cb = decltype(cbc)::value;
        const H16Col col = h16_col<RERUN, DUMP, RAGGED>(g, hd, ctl, t, cb * 32 + (lane & 31));
        if (!col.ok) return;
        const int b = col.b;
        const float T = L.M[(cb * 32 + (lane & 31)) % t.cpf];
        if (T == INFINITY) return;
#pragma unroll
        for (int rb = 0; rb < H_WRB; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int cl = L.rowcl[w * 32 * H_WRB + rb * 32 + h_row(v, lane)];
                const float up = fabsf(acc[rb][cb][v]) + emax[cb];
                if (cl >= 0 && up >= T) {
                    const int j = atomicAdd(&ctl.cand_count[b], 1);
                    if (j < ctl.cap) {
                        ctl.cand_idx[(size_t)b * ctl.cap + j] =
                            (unsigned)(((long long)t.tc * n_fc + col.fc) * hd.n_cl + cl);
                        ctl.cand_score[(size_t)b * ctl.cap + j] = up;
                    }
                }
            }
    });
    __syncthreads();  // L.M / L.cm are rewritten by the next tile
}

// Executed-work report of a pass-0 search: one atomic per wave; a stage a
// wave runs is 4 blocks x 2 k-steps x WCB column blocks x H_WRB row blocks x
// 2 MFMAs (C and S parts).
__device__ __forceinline__ void h16_count(const H16Dev& hd, bool skip, unsigned stages_run, int wcb) {
    if (skip || !hd.exec) return;
    if ((threadIdx.x & 63) == 0 && stages_run)
        atomicAdd(&hd.exec[0], (unsigned long long)stages_run * (unsigned long long)(4 * 2 * wcb * H_WRB * 2));
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&hd.exec[1], 1ull);
}

// Plain plans: tiles (row block, tc, f_c group, channel group), channel group
// fastest, so that concurrently running tiles read the A rows of one row block
// over overlapping windows (adjacent time centres); tile ids are dealt to the
// 8 XCDs in contiguous ranges (workgroup x runs on XCD x % 8, the grid is a
// multiple of 8) so those tiles share an L2.
template <int WCB, bool RERUN, bool DUMP>
__global__ void __launch_bounds__(256, 2) k_search_h16(GridDev g, H16Dev hd, SearchCtl ctl, int batch, int cpf,
                                                        int n_rb, int n_fg, int n_bg) {
    __shared__ H16Lds<WCB> L;
    constexpr int TC = 32 * WCB;
    const long long tiles = (long long)g.cnt[0] * n_rb * n_fg * n_bg;
    const long long chunk = (tiles + 7) / 8;
    unsigned stages_run = 0;  // this wave's stages, counted for the executed-work report
    for (long long x = blockIdx.x; x < 8 * chunk; x += gridDim.x) {
        const long long tid = (x % 8) * chunk + x / 8;
        if (tid >= tiles) continue;
        H16Tile t;
        const int bg = (int)(tid % n_bg);
        long long r = tid / n_bg;
        const int fg = (int)(r % n_fg);
        r /= n_fg;
        t.tc = (int)(r % g.cnt[0]);
        const int rb = (int)(r / g.cnt[0]);
        t.m = hd.tc_shift[t.tc];
        t.row0 = rb * H_RW;
        t.cpf = cpf;
        t.fc0 = fg * (TC / cpf);
        t.slot0 = bg * cpf;
        t.nslot = batch;
        t.n_pad_ch = g.n_pad;
        int live = 0;  // skip tiles none of whose channels take part
        if (threadIdx.x < cpf && t.slot0 + threadIdx.x < batch) {
            const int b = t.slot0 + threadIdx.x;
            live = DUMP || (ctl.ebound[b] >= 0.0 &&
                            (!RERUN || (ctl.need_rerun[b] && bitsf(hd.tmax[(size_t)b * hd.n_tc + t.tc]) >=
                                                                  bitsf(ctl.gmax[b]))));
        }
        if (!__syncthreads_or(live)) continue;
        h16_tile<WCB, RERUN, DUMP, false>(g, hd, ctl, t, L, stages_run);
    }
    h16_count(hd, RERUN || DUMP, stages_run, WCB);
}

// Ragged plans: channels sorted by decreasing length form groups of 64 (the
// columns of a tile: 2 f_c x 64 signals); a persistent grid takes (group, tc,
// row block, f_c group) tiles from a queue.  A group's stages cover its
// longest signal; shorter signals are zero past their end and their columns
// are masked for time centres they do not have.
template <bool RERUN>
__global__ void __launch_bounds__(256, 2) k_search_h16_ragged(GridDev g, H16Dev hd, SearchCtl ctl, int batch,
                                                               int n_rb, int n_fg, int* __restrict__ items) {
    __shared__ H16Lds<4> L;
    __shared__ int s_item;
    if (RERUN && items[batch + 3] == 0) return;  // no channel overflowed
    const int ng = (batch + 63) / 64;
    const int total = items[batch];
    int* counter = items + batch + 1 + (RERUN ? 1 : 0);
    unsigned stages_run = 0;  // this wave's stages, counted for the executed-work report
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);  // uniform: scalar registers
        if (it >= total) break;
        int lo = 0, hi = ng - 1;  // group: last j with items[j] <= it
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid] <= it) lo = mid; else hi = mid - 1;
        }
        const int grp = lo;
        const int q = it - items[grp];
        H16Tile t;
        t.slot0 = grp * 64;
        int nmax = ctl.len[hd.perm[t.slot0]];  // the group's longest signal comes first
        nmax = (nmax < 0 || nmax > g.n) ? 0 : nmax;
        const int n_tc = nmax / g.ragged_div;  // > 0: the group has tiles
        // row block outermost: concurrent tiles read one row block over
        // overlapping windows (adjacent time centres)
        const int fg = q % n_fg;
        t.tc = (q / n_fg) % n_tc;
        const int rb = q / (n_fg * n_tc);
        t.m = t.tc * g.ragged_div;
        t.row0 = rb * H_RW;
        t.cpf = 64;
        t.fc0 = fg * 2;
        t.nslot = batch;
        t.n_pad_ch = (nmax + H_KS - 1) / H_KS * H_KS;
        int live = 0;
        if (threadIdx.x < 64 && t.slot0 + threadIdx.x < batch) {
            const int b = hd.perm[t.slot0 + threadIdx.x];
            const int n = ctl.len[b];
            live = n >= 0 && n <= g.n && t.tc < n / g.ragged_div && ctl.ebound[b] >= 0.0 &&
                   (!RERUN || (ctl.need_rerun[b] &&
                               bitsf(hd.tmax[(size_t)b * hd.n_tc + t.tc]) >= bitsf(ctl.gmax[b])));
        }
        if (!__syncthreads_or(live)) continue;
        h16_tile<4, RERUN, false, true>(g, hd, ctl, t, L, stages_run);
    }
    h16_count(hd, RERUN, stages_run, 4);
}

// Ragged preparation, once per call: channels ranked by decreasing length
// (ties by index; out-of-range lengths count as 0), then the tile prefix of
// the groups of 64 (one thread) and the queue counters.
__global__ void __launch_bounds__(1024) k_h16_ragged_prep(const int* __restrict__ len, int batch, int n_max,
                                                          int div, int n_rb, int n_fg, int* __restrict__ perm,
                                                          int* __restrict__ items) {
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
        const int ng = (batch + 63) / 64;
        int acc = 0;
        for (int j = 0; j < ng; ++j) {
            items[j] = acc;
            int n = len[perm[j * 64]];
            n = (n < 0 || n > n_max) ? 0 : n;
            acc += (n / div) * n_rb * n_fg;
        }
        for (int j = ng; j <= batch; ++j) items[j] = acc;
        items[batch + 1] = 0;
        items[batch + 2] = 0;
        items[batch + 3] = 0;
    }
}

// FP32 accumulation chain of one score: one rounding per product (2 per
// sample) plus the final scaling.
int h16_chain_length(int n_pad) { return 2 * n_pad + 2; }

static H16Dev h16_dev(act_plan_s* p) {
    return H16Dev{(const _Float16*)p->fac_u16, (const _Float16*)p->fac_v16, (const _Float16*)p->fac_c16,
                  (const _Float16*)p->fac_s16, p->inv_norm32, p->tc_shift, p->lag_energy, p->env_q,
                  (const _Float16*)p->shadow, p->rscale, p->ebmul, p->perm, p->tmax, p->ld_half, p->inv_full32,
                  p->fac_w, p->n_cl, p->grid.cnt[3], p->grid.cnt[0], p->desc.support_cut};
}

act_status launch_h16_ragged_prep(act_plan_s* p, int batch, hipStream_t s) {
    const int n_rb = (p->n_cl + H_RW - 1) / H_RW, n_fg = (p->grid.cnt[1] + 1) / 2;
    hipLaunchKernelGGL(k_h16_ragged_prep, dim3(1), dim3(1024), 0, s, p->call_len, batch, p->grid.n,
                       p->desc.ragged_tc_div, n_rb, n_fg, p->perm, p->items);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

act_status launch_search_h16(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s) {
    H16Dev hd = h16_dev(p);
    hd.exec = (ctl.pass == 0 && !ctl.dump) ? p->exec_count : nullptr;
    const int n_fc = p->grid.cnt[1];
    const int n_rb = (p->n_cl + H_RW - 1) / H_RW;
    if (p->desc.ragged) {
        const int n_fg = (n_fc + 1) / 2;
        const unsigned blocks = (unsigned)grid_cap(p, 2);
        if (ctl.pass)
            hipLaunchKernelGGL((k_search_h16_ragged<true>), dim3(blocks), dim3(256), 0, s, p->grid, hd, ctl, batch,
                               n_rb, n_fg, p->items);
        else
            hipLaunchKernelGGL((k_search_h16_ragged<false>), dim3(blocks), dim3(256), 0, s, p->grid, hd, ctl, batch,
                               n_rb, n_fg, p->items);
        ACT_HIP(hipGetLastError());
        return ACT_OK;
    }
    // one channel: 64 f_c columns; several: cpf channels x 128/cpf f_c (by
    // default the smallest power of two covering the batch, at most 64)
    const bool multi = batch > 1;
    int cpf = 1;
    while (multi && cpf < batch && cpf < 64) cpf *= 2;
    if (multi && p->shape.chan_per_fc > 0) cpf = p->shape.chan_per_fc;
    const int TC = multi ? 128 : 64;
    const int n_fg = (n_fc + TC / cpf - 1) / (TC / cpf);
    const int n_bg = (batch + cpf - 1) / cpf;
    const long long tiles = (long long)p->grid.cnt[0] * n_rb * n_fg * n_bg;
    long long blocks = (tiles + 7) / 8 * 8;
    const long long cap = grid_cap(p, 2);  // a multiple of 8 (XCD dealing)
    blocks = blocks < cap ? blocks : cap;
    const dim3 grid((unsigned)blocks), blk(256);
#define H16_LAUNCH(WCB, RR, DD)                                                                      \
    hipLaunchKernelGGL((k_search_h16<WCB, RR, DD>), grid, blk, 0, s, p->grid, hd, ctl, batch, cpf, n_rb, \
                       n_fg, n_bg)
    if (multi) {
        if (ctl.dump) H16_LAUNCH(4, false, true);
        else if (ctl.pass) H16_LAUNCH(4, true, false);
        else H16_LAUNCH(4, false, false);
    } else {
        if (ctl.dump) H16_LAUNCH(2, false, true);
        else if (ctl.pass) H16_LAUNCH(2, true, false);
        else H16_LAUNCH(2, false, false);
    }
#undef H16_LAUNCH
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

// FP16 copies (RNE) of the FP32 factor tables, and the FP64 prefix sums of the
// squared Gaussian envelope over lags (one block per log-duration).
__global__ void k_factors_to_f16(const float* __restrict__ src, long long count, _Float16* __restrict__ dst) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = (_Float16)src[i];
}

__global__ void __launch_bounds__(256) k_env_prefix(GridDev g, int W, double* __restrict__ q) {
    __shared__ double tot[256];
    const int il = blockIdx.x;
    const double inv_dt = 1.0 / exp(g.axis[g.off[3] + il]);
    double* qr = q + (size_t)il * W;
    const int per = (W + 255) / 256;
    const int e0 = threadIdx.x * per, e1 = min(W, e0 + per);
    double acc = 0.0;
    for (int e = e0; e < e1; ++e) {
        const double u = (double)(e - g.n_pad) / g.fs * inv_dt;
        acc += exp(-u * u);  // E(d)^2
        qr[e] = acc;
    }
    tot[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int t = 0; t < 256; ++t) {
            const double x = tot[t];
            tot[t] = run;
            run += x;
        }
    }
    __syncthreads();
    const double base = tot[threadIdx.x];
    for (int e = e0; e < e1; ++e) qr[e] += base;
}

act_status build_h16_factors(act_plan_s* p, hipStream_t s) {
    const long long cl_count = (long long)p->n_cl * p->fac_w;
    const long long fc_count = (long long)p->grid.cnt[1] * p->fac_w;
    const long long cap = (long long)device_cus() * 64;
    const unsigned b1 = (unsigned)std::min<long long>((cl_count + 255) / 256, cap);
    const unsigned b2 = (unsigned)std::min<long long>((fc_count + 255) / 256, cap);
    hipLaunchKernelGGL(k_factors_to_f16, dim3(b1), dim3(256), 0, s, (const float*)p->fac_u, cl_count,
                       (_Float16*)p->fac_u16);
    hipLaunchKernelGGL(k_factors_to_f16, dim3(b1), dim3(256), 0, s, (const float*)p->fac_v, cl_count,
                       (_Float16*)p->fac_v16);
    hipLaunchKernelGGL(k_factors_to_f16, dim3(b2), dim3(256), 0, s, (const float*)p->fac_c, fc_count,
                       (_Float16*)p->fac_c16);
    hipLaunchKernelGGL(k_factors_to_f16, dim3(b2), dim3(256), 0, s, (const float*)p->fac_s, fc_count,
                       (_Float16*)p->fac_s16);
    hipLaunchKernelGGL(k_env_prefix, dim3(p->grid.cnt[3]), dim3(256), 0, s, p->grid, p->fac_w, p->env_q);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

}  // namespace act
