// act_search_h16.hip -- coarse search with the dictionary synthesised from
// shift-invariant factor tables on the FP16 matrix cores
// (v_mfma_f32_32x32x16_f16, FP32 accumulation).
//
// Same factorisation as the FP32 synthesised search (angle-sum identity on the
// real part of Eq. (1), time centres on integer samples m):
//   P[cl][(fc,b)] = sum_n U_cl(n-m) [C_fc(n-m) r_b(n)] - V_cl(n-m) [S_fc(n-m) r_b(n)]
// A = [U | V]: FP16 copies of the FP64-evaluated envelope-chirp factors, rows cl.
// B = the carrier-modulated residuals, formed per stage in FP32, scaled by a
//     power of two per channel (exact) and rounded to FP16.
// Columns are (f_c, channel) pairs, so a batch of channels shares every A
// fragment; P is never written to memory (fused certified emission).
//
// Workgroup = 4 waves, each 64 rows x 64 columns (2 x 2 MFMA tiles):
//   WGC = 1: 256 cl rows x 64 columns  (64 f_c of one channel)
//   WGC = 2: 128 cl rows x 128 columns (cpf channels for each of 128/cpf f_c)
// The B operand of a 128-sample stage sits in LDS in MFMA operand order (each
// k-step and column block is one contiguous KiB: 16-byte conflict-free reads);
// A fragments stream from L2 with one k-step of prefetch.  Every stage
// accumulates into fresh registers that are then added to the total, so the
// FP32 chain of one score is at most 2*128 + N/128 + 2 roundings.
#include "act_emit.h"

namespace act {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int H_KS = 128;             // samples per LDS stage
constexpr int H_KSTEPS = H_KS / 16;   // MFMA k-steps per stage

__device__ __forceinline__ int h_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

struct H16Dev {
    const _Float16* U;      // [n_cl][W] FP16 factor tables, column e = lag + n_pad
    const _Float16* V;
    const float* C;         // [n_fc][W] FP32 carrier tables
    const float* S;
    const float* inv_norm;  // plain plans: [atoms] FP32 1/|g|
    const int* tc_shift;    // plain plans: [n_tc] integer sample of each time centre
    const double* lag_energy;  // ragged plans: [n_fc][n_cl][W] prefix sums of g(d)^2
    const float* rscale;    // [B] power-of-two scale of each channel's FP16 operand
    int W, n_cl;
};

struct H16Tile {
    int tc, m;        // time centre index and its integer sample
    int row0;         // first cl row
    int fc0, b0, cpf; // first f_c, first channel, channels per f_c
    int nb;           // channels present in this tile's channel group
    int n_ch;         // samples of the channel (ragged) or of the plan
    int n_pad_ch;     // samples covered by the stages (multiple of H_KS)
};

template <int WGC>
struct H16Lds {
    f16x8 bc[H_KSTEPS * 2 * WGC * 64];  // C-part of B, [k-step][col block][lane]
    f16x8 bs[H_KSTEPS * 2 * WGC * 64];  // (-S)-part of B
    unsigned cm[64 * WGC];              // column maxima (float bits)
    float M[64];                        // per-channel running max used for emission
};

template <int WGC, bool RERUN, bool DUMP, bool RAGGED>
__device__ void h16_tile(const GridDev& g, const H16Dev& hd, const float* __restrict__ shadow,
                         const SearchCtl& ctl, const H16Tile& t, H16Lds<WGC>& L) {
    constexpr int TC = 64 * WGC;   // columns per workgroup
    constexpr int NCB = TC / 32;   // column blocks
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = w / WGC, wc = w % WGC;
    const int n_fc = g.cnt[1];
    const int W = hd.W;

    // A rows of this lane (two 32-row blocks)
    int arow[2];
    bool aok[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const int cl = t.row0 + wr * 64 + rb * 32 + (lane & 31);
        aok[rb] = cl < hd.n_cl;
        arow[rb] = aok[rb] ? cl : 0;
    }
    f32x16 tot[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) tot[rb][cb][v] = 0.0f;

    for (int n0 = 0; n0 < t.n_pad_ch; n0 += H_KS) {
        __syncthreads();
        // ---- B stage: chunk q = 8 samples of one column, column fastest
        for (int q = threadIdx.x; q < TC * H_KSTEPS * 2; q += 256) {
            const int c = q % TC, sh = q / TC, s = sh >> 1, h = sh & 1;
            const int fc = t.fc0 + c / t.cpf, bl = c % t.cpf;
            f16x8 cv, sv;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                cv[j] = (_Float16)0.0f;
                sv[j] = (_Float16)0.0f;
            }
            if (fc < n_fc && bl < t.nb) {
                const int b = t.b0 + bl;
                const int n = n0 + 16 * s + 8 * h;
                const float sc = hd.rscale[b];
                const float* rp = shadow + (size_t)b * g.n_pad + n;
                const size_t e = (size_t)fc * W + (n - t.m + g.n_pad);
                const f32x4 r0 = *reinterpret_cast<const f32x4*>(rp);
                const f32x4 r1 = *reinterpret_cast<const f32x4*>(rp + 4);
                const f32x4 c0 = *reinterpret_cast<const f32x4*>(hd.C + e);
                const f32x4 c1 = *reinterpret_cast<const f32x4*>(hd.C + e + 4);
                const f32x4 s0 = *reinterpret_cast<const f32x4*>(hd.S + e);
                const f32x4 s1 = *reinterpret_cast<const f32x4*>(hd.S + e + 4);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    cv[j] = (_Float16)((c0[j] * r0[j]) * sc);
                    cv[4 + j] = (_Float16)((c1[j] * r1[j]) * sc);
                    sv[j] = (_Float16)(-((s0[j] * r0[j]) * sc));
                    sv[4 + j] = (_Float16)(-((s1[j] * r1[j]) * sc));
                }
            }
            const int slot = (s * NCB + (c >> 5)) * 64 + (c & 31) + 32 * h;
            L.bc[slot] = cv;
            L.bs[slot] = sv;
        }
        __syncthreads();

        // ---- MFMA over the stage
        f32x16 acc[2][2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[rb][cb][v] = 0.0f;
        const int ebase = n0 - t.m + g.n_pad + 8 * (lane >> 5);
        f16x8 ua[2], va[2], un[2], vn[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const size_t o = (size_t)arow[rb] * W + ebase;
            ua[rb] = *reinterpret_cast<const f16x8*>(hd.U + o);
            va[rb] = *reinterpret_cast<const f16x8*>(hd.V + o);
        }
#pragma unroll 2
        for (int s = 0; s < H_KSTEPS; ++s) {
            if (s + 1 < H_KSTEPS) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const size_t o = (size_t)arow[rb] * W + ebase + 16 * (s + 1);
                    un[rb] = *reinterpret_cast<const f16x8*>(hd.U + o);
                    vn[rb] = *reinterpret_cast<const f16x8*>(hd.V + o);
                }
            }
            f16x8 bC[2], bS[2];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                bC[cb] = L.bc[(s * NCB + wc * 2 + cb) * 64 + lane];
                bS[cb] = L.bs[(s * NCB + wc * 2 + cb) * 64 + lane];
            }
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ua[rb], bC[cb], acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(va[rb], bS[cb], acc[rb][cb], 0, 0, 0);
                }
            if (s + 1 < H_KSTEPS) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    ua[rb] = un[rb];
                    va[rb] = vn[rb];
                }
            }
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) tot[rb][cb][v] += acc[rb][cb][v];
    }

    // ---- epilogue: scale to scores (1/|g| and the channel's 1/scale)
    int col_b[2], col_fc[2];
    bool col_ok[2];
    float col_rinv[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int c = wc * 64 + cb * 32 + (lane & 31);
        col_fc[cb] = t.fc0 + c / t.cpf;
        const int bl = c % t.cpf;
        col_b[cb] = t.b0 + bl;
        col_ok[cb] = col_fc[cb] < n_fc && bl < t.nb;
        col_rinv[cb] = col_ok[cb] ? 1.0f / hd.rscale[col_b[cb]] : 0.0f;
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int cl = t.row0 + wr * 64 + rb * 32 + h_row(v, lane);
                const bool ok = col_ok[cb] && cl < hd.n_cl;
                float inv = 0.0f;
                if (ok) {
                    if (RAGGED) {
                        const double* qr = hd.lag_energy + ((size_t)col_fc[cb] * hd.n_cl + cl) * W;
                        const int e_lo = g.n_pad - t.m, e_hi = t.n_ch - 1 - t.m + g.n_pad;
                        const double e2 = qr[e_hi] - (e_lo > 0 ? qr[e_lo - 1] : 0.0);
                        inv = e2 > 0.0 ? (float)(1.0 / sqrt(e2)) : 0.0f;
                    } else {
                        inv = hd.inv_norm[((size_t)t.tc * n_fc + col_fc[cb]) * hd.n_cl + cl];
                    }
                }
                tot[rb][cb][v] = ok ? (tot[rb][cb][v] * inv) * col_rinv[cb] : 0.0f;
                if (DUMP && ok) {
                    const long long idx = ((long long)t.tc * n_fc + col_fc[cb]) * hd.n_cl + cl;
                    if (idx >= ctl.dump_begin && idx < ctl.dump_begin + ctl.dump_count)
                        ctl.dump[(size_t)col_b[cb] * ctl.dump_count + (idx - ctl.dump_begin)] = tot[rb][cb][v];
                }
            }
    if (DUMP) return;

    // ---- certified emission: column maxima -> channel maxima -> threshold
    if (threadIdx.x < TC) L.cm[threadIdx.x] = 0u;
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        float m = 0.0f;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) m = fmaxf(m, fabsf(tot[rb][cb][v]));
        m = fmaxf(m, __shfl_xor(m, 32, 64));
        if (lane < 32) atomicMax(&L.cm[wc * 64 + cb * 32 + lane], fbits(m));
    }
    __syncthreads();
    const int nchan = t.cpf < t.nb ? t.cpf : t.nb;
    if (threadIdx.x < nchan) {
        const int bl = threadIdx.x, b = t.b0 + bl;
        float M = INFINITY;
        if (ctl.ebound[b] >= 0.0 && (!RERUN || ctl.need_rerun[b])) {
            float wm = 0.0f;
            for (int c = bl; c < TC; c += t.cpf) wm = fmaxf(wm, bitsf(L.cm[c]));
            const float cur = load_gmax(&ctl.gmax[b]);
            M = cur;
            if (!RERUN && wm > cur) M = fmaxf(bitsf(atomicMax(&ctl.gmax[b], fbits(wm))), wm);
        }
        L.M[bl] = M;
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        if (!col_ok[cb]) continue;
        const int b = col_b[cb];
        const float Mc = L.M[b - t.b0];
        if (Mc == INFINITY) continue;
        const double Td = (double)Mc - 2.0 * ctl.ebound[b];
        float T = (float)Td;
        if ((double)T > Td) T = nextafterf(T, -INFINITY);  // keep the test inclusive
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int cl = t.row0 + wr * 64 + rb * 32 + h_row(v, lane);
                if (cl < hd.n_cl && fabsf(tot[rb][cb][v]) >= T) {
                    const int j = atomicAdd(&ctl.cand_count[b], 1);
                    if (j < ctl.cap) {
                        ctl.cand_idx[(size_t)b * ctl.cap + j] =
                            (unsigned)(((long long)t.tc * n_fc + col_fc[cb]) * hd.n_cl + cl);
                        ctl.cand_score[(size_t)b * ctl.cap + j] = tot[rb][cb][v];
                    }
                }
            }
    }
    __syncthreads();  // L.M / L.cm are rewritten by the next tile
}

// Plain plans: tiles (tc, row block, f_c group, channel group), channel group
// fastest so that concurrently running tiles share the A window of one time
// centre; tile ids are dealt to the 8 XCDs in contiguous ranges (workgroup x
// runs on XCD x % 8) so that those tiles also share one L2.
template <int WGC, bool RERUN, bool DUMP>
__global__ void __launch_bounds__(256, 2) k_search_h16(GridDev g, H16Dev hd, const float* __restrict__ shadow,
                                                        SearchCtl ctl, int batch, int cpf, int n_rb, int n_fg,
                                                        int n_bg) {
    __shared__ H16Lds<WGC> L;
    constexpr int TC = 64 * WGC, RW = (4 / WGC) * 64;
    const long long tiles = (long long)g.cnt[0] * n_rb * n_fg * n_bg;
    const long long chunk = (tiles + 7) / 8;
    for (long long x = blockIdx.x; x < 8 * chunk; x += gridDim.x) {
        const long long tid = (x % 8) * chunk + x / 8;
        if (tid >= tiles) continue;
        H16Tile t;
        const int bg = (int)(tid % n_bg);
        long long r = tid / n_bg;
        const int fg = (int)(r % n_fg);
        r /= n_fg;
        const int rb = (int)(r % n_rb);
        t.tc = (int)(r / n_rb);
        t.m = hd.tc_shift[t.tc];
        t.row0 = rb * RW;
        t.cpf = cpf;
        t.fc0 = fg * (TC / cpf);
        t.b0 = bg * cpf;
        t.nb = min(cpf, batch - t.b0);
        t.n_ch = g.n;
        t.n_pad_ch = g.n_pad;
        // skip tiles none of whose channels take part
        int live = 0;
        if (threadIdx.x < t.nb) {
            const int b = t.b0 + threadIdx.x;
            live = DUMP || (ctl.ebound[b] >= 0.0 && (!RERUN || ctl.need_rerun[b]));
        }
        if (!__syncthreads_or(live)) continue;
        h16_tile<WGC, RERUN, DUMP, false>(g, hd, shadow, ctl, t, L);
    }
}

// Ragged plans: a persistent grid takes single-channel tiles (channel, tc, row
// block, f_c group) from a queue (items[b] = first tile of channel b,
// items[B] = total, the two pass counters after it).
template <bool RERUN>
__global__ void __launch_bounds__(256, 2) k_search_h16_ragged(GridDev g, H16Dev hd, const float* __restrict__ shadow,
                                                               SearchCtl ctl, int batch, int n_rb, int n_fg,
                                                               int* __restrict__ items) {
    __shared__ H16Lds<1> L;
    __shared__ int s_item;
    const int total = items[batch];
    int* counter = items + batch + 1 + (RERUN ? 1 : 0);
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= total) break;
        int lo = 0, hi = batch - 1;  // channel: last b with items[b] <= it
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid] <= it) lo = mid; else hi = mid - 1;
        }
        const int b = lo;
        if (RERUN && ctl.need_rerun[b] == 0) continue;
        if (ctl.ebound[b] < 0.0) continue;
        const int q = it - items[b];
        H16Tile t;
        const int fg = q % n_fg;
        const int rb = (q / n_fg) % n_rb;
        t.tc = q / (n_fg * n_rb);
        t.m = t.tc * g.ragged_div;
        t.row0 = rb * 256;
        t.cpf = 1;
        t.fc0 = fg * 64;
        t.b0 = b;
        t.nb = 1;
        t.n_ch = ctl.len[b];  // in range: a channel with tiles has 0 < len <= n_samples
        t.n_pad_ch = (t.n_ch + H_KS - 1) / H_KS * H_KS;
        h16_tile<1, RERUN, false, true>(g, hd, shadow, ctl, t, L);
    }
}

int h16_chain_length(int n_pad) { return 2 * H_KS + n_pad / H_KS + 2; }

static H16Dev h16_dev(act_plan_s* p) {
    return H16Dev{(const _Float16*)p->fac_u16, (const _Float16*)p->fac_v16, (const float*)p->fac_c,
                  (const float*)p->fac_s, p->inv_norm32, p->tc_shift, p->lag_energy, p->rscale,
                  p->fac_w, p->n_cl};
}

act_status launch_search_h16(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s) {
    const H16Dev hd = h16_dev(p);
    const float* sh = (const float*)p->shadow;
    const int n_fc = p->grid.cnt[1];
    if (p->desc.ragged) {
        const int n_rb = (p->n_cl + 255) / 256, n_fg = (n_fc + 63) / 64;
        const unsigned blocks = (unsigned)device_cus() * 2;
        if (ctl.pass)
            hipLaunchKernelGGL((k_search_h16_ragged<true>), dim3(blocks), dim3(256), 0, s, p->grid, hd, sh, ctl,
                               batch, n_rb, n_fg, p->items);
        else
            hipLaunchKernelGGL((k_search_h16_ragged<false>), dim3(blocks), dim3(256), 0, s, p->grid, hd, sh, ctl,
                               batch, n_rb, n_fg, p->items);
        ACT_HIP(hipGetLastError());
        return ACT_OK;
    }
    // one channel: 256 rows x 64 f_c tiles; several: 128 rows x (cpf channels x 128/cpf f_c)
    const bool multi = batch > 1;
    int cpf = 1;
    while (multi && cpf < batch && cpf < 64) cpf *= 2;
    const int TC = multi ? 128 : 64, RW = multi ? 128 : 256;
    const int n_rb = (p->n_cl + RW - 1) / RW;
    const int n_fg = (n_fc + TC / cpf - 1) / (TC / cpf);
    const int n_bg = (batch + cpf - 1) / cpf;
    const long long tiles = (long long)p->grid.cnt[0] * n_rb * n_fg * n_bg;
    long long blocks = (tiles + 7) / 8 * 8;
    const long long cap = (long long)device_cus() * 2;
    blocks = blocks < cap ? blocks : cap;
    const dim3 grid((unsigned)blocks), blk(256);
#define H16_LAUNCH(WGC, RR, DD)                                                                        \
    hipLaunchKernelGGL((k_search_h16<WGC, RR, DD>), grid, blk, 0, s, p->grid, hd, sh, ctl, batch, cpf, n_rb, \
                       n_fg, n_bg)
    if (multi) {
        if (ctl.dump) H16_LAUNCH(2, false, true);
        else if (ctl.pass) H16_LAUNCH(2, true, false);
        else H16_LAUNCH(2, false, false);
    } else {
        if (ctl.dump) H16_LAUNCH(1, false, true);
        else if (ctl.pass) H16_LAUNCH(1, true, false);
        else H16_LAUNCH(1, false, false);
    }
#undef H16_LAUNCH
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

// FP16 copies of the FP32 envelope-chirp factors (RNE).
__global__ void k_factors_to_f16(const float* __restrict__ U, const float* __restrict__ V, long long count,
                                 _Float16* __restrict__ U16, _Float16* __restrict__ V16) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        U16[i] = (_Float16)U[i];
        V16[i] = (_Float16)V[i];
    }
}

act_status build_h16_factors(act_plan_s* p, hipStream_t s) {
    const long long count = (long long)p->n_cl * p->fac_w;
    const long long blocks = std::min<long long>((count + 255) / 256, (long long)device_cus() * 64);
    hipLaunchKernelGGL(k_factors_to_f16, dim3((unsigned)blocks), dim3(256), 0, s, (const float*)p->fac_u,
                       (const float*)p->fac_v, count, (_Float16*)p->fac_u16, (_Float16*)p->fac_v16);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

}  // namespace act
