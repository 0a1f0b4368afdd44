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
    const float* inv_norm;  // [atoms] FP32 copy of 1/|g|
    const int* tc_shift;    // [n_tc] integer sample of each time centre
    int W, n_cl;
};

// grid: x = (tc, cl block, fc chunk) tiles, y = channel
template <bool RERUN, bool DUMP>
__global__ void __launch_bounds__(256) k_search_synth_f32(GridDev g, SynthDev sy,
                                                          const float* __restrict__ shadow,
                                                          SearchCtl ctl, int n_clb, int n_fcc) {
    // B operand [C|S part][fc][sample]; one f32x4 of padding per column keeps
    // the 16-byte column reads of 32 lanes on distinct LDS banks
    __shared__ f32x4 bl[2][SY_COLS][SY_STAGE / 4 + 1];
    __shared__ float s_red[4];
    __shared__ float s_M;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.y;
    if (RERUN && ctl.need_rerun[b] == 0) return;
    if (!DUMP && ctl.ebound[b] < 0.0) return;
    const int n_fc = g.cnt[1];
    const long long tiles = (long long)g.cnt[0] * n_clb * n_fcc;
    const float* r = shadow + (size_t)b * g.n_pad;
    for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int fcc = (int)(t % n_fcc);
        const int clb = (int)((t / n_fcc) % n_clb);
        const int tc = (int)(t / ((long long)n_fcc * n_clb));
        const int m = sy.tc_shift[tc];
        const int fc0 = fcc * SY_COLS;
        const int cl = clb * SY_ROWS + w * 32 + (lane & 31);   // this lane's A row
        const bool row_ok = cl < sy.n_cl;
        const float* urow = sy.U + (size_t)(row_ok ? cl : 0) * sy.W;
        const float* vrow = sy.V + (size_t)(row_ok ? cl : 0) * sy.W;
        const int h = lane >> 5;
        f32x16 tot[2], acc[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) tot[cb][v] = 0.0f;

        for (int n0 = 0; n0 < g.n_pad; n0 += SY_STAGE) {
            __syncthreads();
            // B operand of this stage: C_fc(n-m) r(n) and -S_fc(n-m) r(n)
            for (int q = threadIdx.x; q < SY_COLS * SY_STAGE; q += 256) {
                const int fcl = q / SY_STAGE, sn = q % SY_STAGE;
                const int fc = fc0 + fcl, n = n0 + sn;
                float cv = 0.0f, sv = 0.0f;
                if (fc < n_fc && n < g.n) {
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
                for (int v = 0; v < 16; ++v) acc[cb][v] = 0.0f;
            for (int s16 = 0; s16 < SY_STAGE; s16 += 16) {
                const int e0 = n0 + s16 + 8 * h - m + g.n_pad;  // factor column of this lane's 8 samples
                f32x4 ua = {0, 0, 0, 0}, ub = {0, 0, 0, 0}, va = {0, 0, 0, 0}, vb = {0, 0, 0, 0};
                if (row_ok) {
                    ua = *reinterpret_cast<const f32x4*>(urow + e0);
                    ub = *reinterpret_cast<const f32x4*>(urow + e0 + 4);
                    va = *reinterpret_cast<const f32x4*>(vrow + e0);
                    vb = *reinterpret_cast<const f32x4*>(vrow + e0 + 4);
                }
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
                    }
                }
            }
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) tot[cb][v] += acc[cb][v];
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
                tot[cb][v] = ok ? tot[cb][v] * sy.inv_norm[idx] : 0.0f;
                lmax = fmaxf(lmax, fabsf(tot[cb][v]));
                if (DUMP && ok && idx >= ctl.dump_begin && idx < ctl.dump_begin + ctl.dump_count)
                    ctl.dump[(size_t)b * ctl.dump_count + (idx - ctl.dump_begin)] = tot[cb][v];
            }
        }
        if (DUMP) continue;
        lmax = wave_max(lmax);
        if (lane == 0) s_red[w] = lmax;
        __syncthreads();
        if (threadIdx.x == 0) {
            const float wm = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
            const float cur = load_gmax(&ctl.gmax[b]);
            float M = cur;
            if (!RERUN && wm > cur) M = fmaxf(bitsf(atomicMax(&ctl.gmax[b], fbits(wm))), wm);
            s_M = M;
        }
        __syncthreads();
        const double Td = (double)s_M - 2.0 * ctl.ebound[b];
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

// FP32 accumulation chain of one synthesised score: 2 roundings per MFMA over a
// stage (2 * SY_STAGE) plus one per stage added to the total.
int synth_chain_length(int n_pad) { return 2 * SY_STAGE + n_pad / SY_STAGE + 2; }

act_status launch_search_synth_f32(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s) {
    SynthDev sy{(const float*)p->fac_u, (const float*)p->fac_v, (const float*)p->fac_c,
                (const float*)p->fac_s, p->inv_norm32, p->tc_shift, p->fac_w, p->n_cl};
    const int n_clb = (p->n_cl + SY_ROWS - 1) / SY_ROWS;
    const int n_fcc = (p->grid.cnt[1] + SY_COLS - 1) / SY_COLS;
    const long long tiles = (long long)p->grid.cnt[0] * n_clb * n_fcc;
    long long blocks = tiles;
    const long long cap = (long long)device_cus() * 4;
    blocks = blocks < cap ? blocks : cap;
    const float* sh = (const float*)p->shadow;
    if (ctl.dump)
        hipLaunchKernelGGL((k_search_synth_f32<false, true>), dim3((unsigned)blocks, batch), dim3(256), 0, s,
                           p->grid, sy, sh, ctl, n_clb, n_fcc);
    else if (ctl.pass)
        hipLaunchKernelGGL((k_search_synth_f32<true, false>), dim3((unsigned)blocks, batch), dim3(256), 0, s,
                           p->grid, sy, sh, ctl, n_clb, n_fcc);
    else
        hipLaunchKernelGGL((k_search_synth_f32<false, false>), dim3((unsigned)blocks, batch), dim3(256), 0, s,
                           p->grid, sy, sh, ctl, n_clb, n_fcc);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

}  // namespace act
