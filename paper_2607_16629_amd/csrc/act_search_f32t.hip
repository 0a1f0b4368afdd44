// act_search_f32t.hip -- coarse search streaming the FP32 dictionary table
// from HBM (GEMV-shaped for one channel; bound by HBM bandwidth).
#include "act_emit.h"

namespace act {

// --------------------------------------------------------------------------
// FP32 table GEMV (HBM-bound).  A wave owns a batch of R = 64/BT table rows
// and BT channels: every lane reads NCH float4 of each row (fully coalesced
// 1 KiB wave loads, non-temporal: the table is streamed once per order), does
// 4*NCH FMAs per (row, channel) against the residual held in registers, and a
// 63-shuffle reduce-scatter leaves slot l = row*BT + ch in lane l.  The FMA
// chain of one score is 4*NCH products plus 6 tree levels long.
// --------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int LVL>
__device__ __forceinline__ void rs_level(float (&v)[64], int lane) {
    const bool up = (lane & LVL) != 0;
#pragma unroll
    for (int s = 0; s < LVL; ++s) {
        const float send = up ? v[s] : v[s + LVL];
        const float keep = up ? v[s + LVL] : v[s];
        v[s] = keep + __shfl_xor(send, LVL, kWave);
    }
}

// After the six levels lane l holds the full sum of slot l in v[0].
__device__ __forceinline__ void reduce_scatter64(float (&v)[64], int lane) {
    rs_level<32>(v, lane);
    rs_level<16>(v, lane);
    rs_level<8>(v, lane);
    rs_level<4>(v, lane);
    rs_level<2>(v, lane);
    rs_level<1>(v, lane);
}

template <int NCH, int BT, bool RERUN>
__global__ void __launch_bounds__(256) k_search_f32_table(const float4* __restrict__ table,
                                                          GridDev g,
                                                          const float* __restrict__ shadow,
                                                          int batch, SearchCtl ctl) {
    constexpr int R = 64 / BT;
    const int lane = threadIdx.x & (kWave - 1);
    const int cg = blockIdx.y;
    // a channel group is skipped in the rerun pass unless one of its channels overflowed
    if (RERUN) {
        bool any = false;
#pragma unroll
        for (int b = 0; b < BT; ++b)
            if (cg * BT + b < batch && ctl.need_rerun[cg * BT + b]) any = true;
        if (!any) return;
    }
    const int rows_per_row4 = g.n_pad / 4;
    float4 rr[BT][NCH];
#pragma unroll
    for (int b = 0; b < BT; ++b) {
        const int ch = cg * BT + b;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            rr[b][c] = ch < batch ? reinterpret_cast<const float4*>(shadow + (size_t)ch * g.n_pad)[c * kWave + lane]
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const long long total = ctl.dump ? ctl.dump_count : g.atoms;
    const long long base0 = ctl.dump ? ctl.dump_begin : 0;
    const long long nbatch = (total + R - 1) / R;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const long long nwaves = (long long)gridDim.x * blockDim.x / kWave;
    for (long long bt = wave; bt < nbatch; bt += nwaves) {
        float acc[64];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            long long row = bt * R + j;
            row = row < total ? row : total - 1;
            const float4* rp = table + (size_t)(base0 + row) * rows_per_row4 + lane;
            f32x4 v[NCH];
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                v[c] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(rp + c * kWave));
#pragma unroll
            for (int b = 0; b < BT; ++b) {
                float s = 0.0f;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    s = fmaf(v[c].x, rr[b][c].x, s);
                    s = fmaf(v[c].y, rr[b][c].y, s);
                    s = fmaf(v[c].z, rr[b][c].z, s);
                    s = fmaf(v[c].w, rr[b][c].w, s);
                }
                acc[j * BT + b] = s;
            }
        }
        reduce_scatter64(acc, lane);
        const int j = lane / BT, b = lane % BT;
        const long long row = bt * R + j;
        const bool valid = row < total && cg * BT + b < batch;
        if (ctl.dump) {
            if (valid) ctl.dump[(size_t)(cg * BT + b) * ctl.dump_count + row] = acc[0];
            continue;
        }
        // emission, one channel of the group at a time (uniform per wave)
#pragma unroll
        for (int bb = 0; bb < BT; ++bb) {
            if (cg * BT + bb >= batch) break;
            emit_uniform(ctl, cg * BT + bb, base0 + row, acc[0], valid && b == bb);
        }
    }
}

template <int NCH, int BT>
static void launch_f32t(act_plan_s* p, int batch, hipStream_t s, const SearchCtl& ctl, int cus) {
    const int groups = (batch + BT - 1) / BT;
    const long long total = ctl.dump ? ctl.dump_count : p->atoms;
    const long long nbatch = (total + (64 / BT) - 1) / (64 / BT);
    long long blocks = (nbatch + 3) / 4;
    const long long cap = grid_cap(p, 8);
    (void)cus;
    blocks = blocks < cap ? blocks : cap;
    if (blocks < 1) blocks = 1;
    if (ctl.pass)
        hipLaunchKernelGGL((k_search_f32_table<NCH, BT, true>), dim3((unsigned)blocks, groups), dim3(256), 0,
                           s, (const float4*)p->table, p->grid, (const float*)p->shadow, batch, ctl);
    else
        hipLaunchKernelGGL((k_search_f32_table<NCH, BT, false>), dim3((unsigned)blocks, groups), dim3(256), 0,
                           s, (const float4*)p->table, p->grid, (const float*)p->shadow, batch, ctl);
}

template <int NCH>
static void launch_f32t_bt(act_plan_s* p, int batch, hipStream_t s, const SearchCtl& ctl, int cus) {
    if (batch == 1)
        launch_f32t<NCH, 1>(p, batch, s, ctl, cus);
    else if (batch == 2)
        launch_f32t<NCH, 2>(p, batch, s, ctl, cus);
    else
        launch_f32t<NCH, 4>(p, batch, s, ctl, cus);
}


act_status launch_search_f32t(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s) {
    const int cus = device_cus();
    switch (p->n_pad / 256) {
        case 1: launch_f32t_bt<1>(p, batch, s, ctl, cus); break;
        case 2: launch_f32t_bt<2>(p, batch, s, ctl, cus); break;
        case 3: launch_f32t_bt<3>(p, batch, s, ctl, cus); break;
        case 4: launch_f32t_bt<4>(p, batch, s, ctl, cus); break;
        case 5: launch_f32t_bt<5>(p, batch, s, ctl, cus); break;
        case 6: launch_f32t_bt<6>(p, batch, s, ctl, cus); break;
        case 7: launch_f32t_bt<7>(p, batch, s, ctl, cus); break;
        case 8: launch_f32t_bt<8>(p, batch, s, ctl, cus); break;
        default:
            set_error("FP32 table search supports n_samples <= 2048");
            return ACT_ERR_UNSUPPORTED;
    }
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

// number of products + tree levels in one FP32 score (for the certified margin)
int f32_chain_length(int n_pad) { return 4 * (n_pad / 256) + 6; }

}  // namespace act
