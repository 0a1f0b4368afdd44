// act_search.hip -- the coarse search (Sec. III-A "i* = argmax |<g_i, r_k>|";
// the projection P = D X^T of Sec. IV-A) with a fused, certified candidate
// selection.
//
// Every search kernel computes scores p~_i (approximations of <g_hat_i, r>)
// and, instead of materialising P, keeps per channel
//   gmax  = running max |p~| (atomicMax on the float bit pattern), and
//   cands = every (i, p~_i) with |p~_i| >= M - 2 E_b, where M is the running
//           max seen when the score is produced (M <= final max), and E_b is a
//           proven bound on |p~_i - p_i| for this channel and arithmetic.
// Since M never exceeds the final max, the list contains every atom whose
// exact score can still be the maximum; the FP64 rescoring then decides the
// winner exactly.  If more than `cap` atoms qualify, the channel is searched
// once more with the final threshold (pass 1).
#include "act_emit.h"

namespace act {

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
    }
    return cus;
}

int device_lds_per_block() {
    static int bytes = 0;
    if (!bytes) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (bytes <= 0) bytes = 65536;
    }
    return bytes;
}

static act_status dispatch(act_plan_s* p, int batch, hipStream_t s, const SearchCtl& ctl,
                           const double* resid64) {
    if (p->desc.dict == ACT_DICT_LAG) return launch_search_lag(p, batch, ctl, s);
    if (p->desc.prec == ACT_PREC_F64) return launch_search_f64(p, batch, ctl, resid64, s);
    if (p->desc.prec == ACT_PREC_F32 && p->desc.dict == ACT_DICT_TABLE)
        return launch_search_f32t(p, batch, ctl, s);
    if (p->desc.prec == ACT_PREC_BF16 && p->desc.dict == ACT_DICT_TABLE)
        return launch_search_bf16t(p, batch, ctl, s);
    if (p->desc.prec == ACT_PREC_F32 && p->desc.dict == ACT_DICT_SYNTH)
        return launch_search_synth_f32(p, batch, ctl, s);
    if (p->desc.prec == ACT_PREC_F16 && p->desc.dict == ACT_DICT_SYNTH)
        return launch_search_h16(p, batch, ctl, s);
    set_error("search: unsupported precision / dictionary");
    return ACT_ERR_UNSUPPORTED;
}

act_status launch_search(act_plan_s* p, int batch, int pass, hipStream_t s) {
    SearchCtl ctl{p->cand_idx, p->cand_score, p->cand_count, p->gmax, p->ebound, p->need_rerun,
                  p->cap, pass, nullptr, 0, 0, p->call_len, p->call_off};
    return dispatch(p, batch, s, ctl, p->search_resid);
}

act_status launch_correlate(act_plan_s* p, int batch, const double* resid, long long begin,
                            long long count, double* out, hipStream_t s) {
    SearchCtl ctl{p->cand_idx, p->cand_score, p->cand_count, p->gmax, p->ebound, p->need_rerun,
                  p->cap, 0, out, begin, count, nullptr, nullptr};
    return dispatch(p, batch, s, ctl, resid);
}

}  // namespace act
