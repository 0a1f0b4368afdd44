// act_emit.h -- shared pieces of the search kernels: the candidate-emission
// control block and the fused certified emission (see act_search.hip).
#pragma once

#include "act_common.h"

namespace act {

struct SearchCtl {
    unsigned* cand_idx;
    float* cand_score;
    int* cand_count;
    unsigned* gmax;
    const double* ebound;
    const int* need_rerun;
    int cap;
    int pass;           // 0: running-max emission, 1: rerun of overflowed channels
    double* dump;       // act_correlate: scores [batch][dump_count] (no emission)
    long long dump_begin, dump_count;
    const int* len;         // ragged plans: channel lengths and offsets
    const long long* off;
};

// Candidate emission for one lane's score (channel b, atom i).  All lanes of
// the wave call this with the same b (uniform control flow).
__device__ __forceinline__ void emit_uniform(const SearchCtl& c, int b, long long i, float p,
                                             bool valid) {
    const float a = valid ? fabsf(p) : 0.0f;
    const double eb = c.ebound[b];
    if (eb < 0.0) return;  // zero or non-finite channel: handled by the selector
    float M;
    if (c.pass == 0) {
        float wm = wave_max(a);
        float old = 0.0f;
        if ((threadIdx.x & (kWave - 1)) == 0) old = bitsf(atomicMax(&c.gmax[b], fbits(wm)));
        old = __shfl(old, 0, kWave);
        M = fmaxf(old, wm);
    } else {
        M = bitsf(c.gmax[b]);
    }
    const double T = (double)M - 2.0 * eb;
    if (valid && (double)a >= T) {
        int j = atomicAdd(&c.cand_count[b], 1);
        if (j < c.cap) {
            c.cand_idx[(size_t)b * c.cap + j] = (unsigned)i;
            c.cand_score[(size_t)b * c.cap + j] = p;
        }
    }
}

// Channel's current running maximum, read coherently at device scope.
__device__ __forceinline__ float load_gmax(const unsigned* p) {
    return bitsf(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

int device_cus();
act_status launch_search_f64(act_plan_s* p, int batch, const SearchCtl& ctl, const double* resid,
                             hipStream_t s);
act_status launch_search_f32t(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s);
act_status launch_search_bf16t(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s);
act_status launch_search_synth_f32(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s);
act_status launch_search_h16(act_plan_s* p, int batch, const SearchCtl& ctl, hipStream_t s);

}  // namespace act
