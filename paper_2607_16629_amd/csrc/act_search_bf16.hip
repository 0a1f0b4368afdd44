// act_search_bf16.hip -- multi-channel coarse search as a dense BF16 GEMM on
// the CDNA4 matrix cores: P[K x B] = D[K x N] R^T[N x B] (the paper's stacked
// projection P = D X^T, Sec. IV-A / Sec. V-A), FP32 accumulation, fused
// certified candidate emission, P never written to memory.
//
// Tiling (v_mfma_f32_32x32x16_bf16, 64-lane waves):
//   workgroup = 4 waves = 512 atoms x 64 channels; wave = 4 row blocks of 32
//   atoms x 2 column blocks of 32 channels (8 accumulator tiles, 128 FP32).
//   The dictionary table is stored pre-swizzled in MFMA operand order: for
//   row block rb and k-step s (16 samples) the 64 lanes' 16-byte A operands
//   are one contiguous KiB, so every wave load is a full-line streaming read.
//   The BF16 residuals of the 64 channels are staged through LDS 512 samples
//   at a time (64 KiB, already in B-operand order, bank-conflict-free 16-byte
//   reads), so two workgroups fit a CU.
// The sample order inside a k-step is a permutation applied identically to A
// and B, so it does not change the sum being computed.
#include "act_emit.h"

namespace act {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int BF_WAVES = 4;
constexpr int BF_RB = 4;                              // row blocks per wave
constexpr int BF_TILE = 32 * BF_RB * BF_WAVES;        // atoms per workgroup tile
constexpr int BF_STAGE = 32;                          // k-steps (16 samples) per LDS stage

// Row of accumulator register v of a 32x32 MFMA tile held by `lane`.
__device__ __forceinline__ int mfma32_row(int v, int lane) {
    return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}

template <bool RERUN, bool DUMP>
__global__ void __launch_bounds__(256, 2) k_search_bf16_table(const u16x8* __restrict__ table,
                                                              GridDev g,
                                                              const unsigned short* __restrict__ shadow,
                                                              int batch, SearchCtl ctl,
                                                              long long tile_begin,
                                                              long long tile_count) {
    __shared__ u16x8 lds_r[BF_STAGE * 2 * 64];
    __shared__ float s_red[BF_WAVES][64];
    __shared__ float s_M[64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int ch0 = blockIdx.y * 64;
    if (RERUN) {
        int any = 0;
        for (int c = 0; c < 64; ++c)
            if (ch0 + c < batch && ctl.need_rerun[ch0 + c]) any = 1;
        if (!any) return;
    }
    const int nsteps = g.n_pad / 16;
    for (long long t = blockIdx.x; t < tile_count; t += gridDim.x) {
        const long long tile = tile_begin + t;
        const long long rb0 = tile * (BF_TILE / 32) + (long long)w * BF_RB;
        f32x16 acc[BF_RB][2];
#pragma unroll
        for (int rb = 0; rb < BF_RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[rb][cb][v] = 0.0f;

        for (int q0 = 0; q0 < nsteps; q0 += BF_STAGE) {
            const int qs = min(BF_STAGE, nsteps - q0);
            __syncthreads();
            // residual stage -> LDS in B-operand order: chunk = 8 samples of one channel
            for (int c = threadIdx.x; c < 64 * qs * 2; c += 256) {
                const int chl = c / (qs * 2);
                const int nchunk = c - chl * (qs * 2);
                const int ch = ch0 + chl;
                u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
                if (ch < batch)
                    v = *reinterpret_cast<const u16x8*>(shadow + (size_t)ch * g.n_pad + (size_t)(q0 * 16 + nchunk * 8));
                const int s = nchunk >> 1, h = nchunk & 1;
                lds_r[(s * 2 + (chl >> 5)) * 64 + (chl & 31) + 32 * h] = v;
            }
            __syncthreads();
            const u16x8* ap = table + ((size_t)rb0 * nsteps + q0) * 64 + lane;
            u16x8 a_cur[BF_RB], a_nxt[BF_RB];
#pragma unroll
            for (int rb = 0; rb < BF_RB; ++rb)
                a_cur[rb] = __builtin_nontemporal_load(ap + (size_t)rb * nsteps * 64);
            for (int s = 0; s < qs; ++s) {
                if (s + 1 < qs) {
#pragma unroll
                    for (int rb = 0; rb < BF_RB; ++rb)
                        a_nxt[rb] = __builtin_nontemporal_load(ap + ((size_t)rb * nsteps + s + 1) * 64);
                }
                const u16x8 b0 = lds_r[(s * 2 + 0) * 64 + lane];
                const u16x8 b1 = lds_r[(s * 2 + 1) * 64 + lane];
#pragma unroll
                for (int rb = 0; rb < BF_RB; ++rb) {
                    const bf16x8 a = __builtin_bit_cast(bf16x8, a_cur[rb]);
                    acc[rb][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, b0),
                                                                         acc[rb][0], 0, 0, 0);
                    acc[rb][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, b1),
                                                                         acc[rb][1], 0, 0, 0);
                }
#pragma unroll
                for (int rb = 0; rb < BF_RB; ++rb) a_cur[rb] = a_nxt[rb];
            }
        }

        // ---- epilogue: scores of 512 atoms x 64 channels in registers
        const long long row_base = rb0 * 32;
        if (DUMP) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int ch = ch0 + cb * 32 + (lane & 31);
                if (ch >= batch) continue;
#pragma unroll
                for (int rb = 0; rb < BF_RB; ++rb)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const long long row = row_base + rb * 32 + mfma32_row(v, lane);
                        if (row >= ctl.dump_begin && row < ctl.dump_begin + ctl.dump_count)
                            ctl.dump[(size_t)ch * ctl.dump_count + (row - ctl.dump_begin)] = acc[rb][cb][v];
                    }
            }
            continue;
        }
        // rows of this tile that exist (the last tile may be padded)
        const int valid_rows = (int)min((long long)BF_TILE, g.atoms - tile * BF_TILE) - w * BF_RB * 32;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            float m = 0.0f;
#pragma unroll
            for (int rb = 0; rb < BF_RB; ++rb)
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    if (rb * 32 + mfma32_row(v, lane) < valid_rows) m = fmaxf(m, fabsf(acc[rb][cb][v]));
            m = fmaxf(m, __shfl_xor(m, 32, 64));
            if (lane < 32) s_red[w][cb * 32 + lane] = m;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int c = threadIdx.x, ch = ch0 + c;
            float M = INFINITY;
            if (ch < batch && ctl.ebound[ch] >= 0.0 && (!RERUN || ctl.need_rerun[ch])) {
                float wm = s_red[0][c];
#pragma unroll
                for (int q = 1; q < BF_WAVES; ++q) wm = fmaxf(wm, s_red[q][c]);
                const float cur = load_gmax(&ctl.gmax[ch]);
                if (RERUN) {
                    M = cur;
                } else if (wm > cur) {
                    const float old = bitsf(atomicMax(&ctl.gmax[ch], fbits(wm)));
                    M = fmaxf(old, wm);
                } else {
                    M = cur;
                }
            }
            s_M[c] = M;
        }
        __syncthreads();
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int c = cb * 32 + (lane & 31), ch = ch0 + c;
            const float Mc = s_M[c];
            if (Mc == INFINITY) continue;
            const double Td = (double)Mc - 2.0 * ctl.ebound[ch];
            float T = (float)Td;
            if ((double)T > Td) T = nextafterf(T, -INFINITY);  // keep the test inclusive
            // rare path: a score at or above the margin
#pragma unroll
            for (int rb = 0; rb < BF_RB; ++rb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int r = rb * 32 + mfma32_row(v, lane);
                    const float p = acc[rb][cb][v];
                    if (r < valid_rows && fabsf(p) >= T) {
                        const int j = atomicAdd(&ctl.cand_count[ch], 1);
                        if (j < ctl.cap) {
                            ctl.cand_idx[(size_t)ch * ctl.cap + j] = (unsigned)(row_base + r);
                            ctl.cand_score[(size_t)ch * ctl.cap + j] = p;
                        }
                    }
                }
        }
        __syncthreads();
    }
}

act_status launch_search_bf16t(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s) {
    const int ctiles = (batch + 63) / 64;
    long long tb = 0, tc = p->atoms_pad / BF_TILE;
    if (ctl.dump) {
        tb = ctl.dump_begin / BF_TILE;
        tc = (ctl.dump_begin + ctl.dump_count + BF_TILE - 1) / BF_TILE - tb;
    }
    long long blocks = tc;
    const long long cap = grid_cap(p, 2);
    blocks = blocks < cap ? blocks : cap;
    const u16x8* table = (const u16x8*)p->table;
    const unsigned short* sh = (const unsigned short*)p->shadow;
    if (ctl.dump)
        hipLaunchKernelGGL((k_search_bf16_table<false, true>), dim3((unsigned)blocks, ctiles), dim3(256), 0, s,
                           table, p->grid, sh, batch, ctl, tb, tc);
    else if (ctl.pass)
        hipLaunchKernelGGL((k_search_bf16_table<true, false>), dim3((unsigned)blocks, ctiles), dim3(256), 0, s,
                           table, p->grid, sh, batch, ctl, tb, tc);
    else
        hipLaunchKernelGGL((k_search_bf16_table<false, false>), dim3((unsigned)blocks, ctiles), dim3(256), 0, s,
                           table, p->grid, sh, batch, ctl, tb, tc);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

// Table layout: element (atom i, sample n) of the swizzled BF16 table.
__host__ __device__ inline size_t bf16_swz_offset(long long i, int n, int n_pad) {
    const long long rb = i >> 5;
    const int r = (int)(i & 31), s = n >> 4, o = n & 15;
    const int ln = r + 32 * (o >> 3);
    return (((size_t)rb * (n_pad >> 4) + s) * 64 + ln) * 8 + (o & 7);
}

// Plan-time writer of the swizzled BF16 table: one thread per 16-byte operand
// chunk (8 samples of one atom), FP64 synthesis scaled by the FP64 inverse
// norm, RNE to BF16.  Consecutive threads write consecutive 16 bytes.
__global__ void __launch_bounds__(256) k_write_bf16_swz(GridDev g, long long atoms_pad,
                                                        const double* __restrict__ inv_norm,
                                                        u16x8* __restrict__ table) {
    const int nsteps = g.n_pad / 16;
    const long long chunks = atoms_pad / 32 * nsteps * 64;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < chunks;
         c += (long long)gridDim.x * blockDim.x) {
        const int ln = (int)(c & 63);
        const long long rs = c >> 6;
        const int s = (int)(rs % nsteps);
        const long long rb = rs / nsteps;
        const long long i = rb * 32 + (ln & 31);
        const int n0 = s * 16 + 8 * (ln >> 5);
        u16x8 out = {0, 0, 0, 0, 0, 0, 0, 0};
        if (i < g.atoms) {
            double th[4];
            grid_theta(g, i, th);
            const double inv_dt = 1.0 / exp(th[3]);
            const double sc = inv_norm[i];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int n = n0 + j;
                const double v = n < g.n ? atom_sample64(sample_time(n, g.fs), th[0], th[1], th[2], inv_dt) * sc : 0.0;
                const unsigned u = __float_as_uint((float)v);
                out[j] = (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
            }
        }
        table[c] = out;
    }
}

act_status write_bf16_table(act_plan_s* p, hipStream_t s) {
    const int nsteps = p->n_pad / 16;
    const long long chunks = p->atoms_pad / 32 * nsteps * 64;
    long long blocks = (chunks + 255) / 256;
    const long long cap = (long long)device_cus() * 64;
    blocks = blocks < cap ? blocks : cap;
    hipLaunchKernelGGL(k_write_bf16_swz, dim3((unsigned)blocks), dim3(256), 0, s, p->grid, p->atoms_pad,
                       p->inv_norm, (u16x8*)p->table);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

}  // namespace act
