// act_api.hip -- C ABI entry points: argument checks on the host, then the
// stream-ordered launch sequence of the matching pursuit.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "act_common.h"

namespace act {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace act

using namespace act;

extern "C" const char* act_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* act_status_string(act_status s) {
    switch (s) {
        case ACT_OK: return "ACT_OK";
        case ACT_ERR_INVALID: return "ACT_ERR_INVALID";
        case ACT_ERR_NOMEM: return "ACT_ERR_NOMEM";
        case ACT_ERR_HIP: return "ACT_ERR_HIP";
        case ACT_ERR_UNSUPPORTED: return "ACT_ERR_UNSUPPORTED";
        default: return "ACT_ERR_UNKNOWN";
    }
}

// One order of the residue-based pursuit for every channel (Sec. III-A, Fig.
// "simplified residue-driven ACT iteration"):
//   search (fused certified candidates) -> overflow check -> exact-threshold
//   search of overflowed channels -> FP64 rescoring -> select, refine,
//   coefficient, update.
// Bracket one launch by a pair of events when timing is enabled.
template <typename F>
static act_status timed(act_plan_s* p, int phase, hipStream_t s, F&& launch) {
    if (!p->timing) return launch();
    if (p->ev_used == p->ev_pool.size()) {
        hipEvent_t a, b;
        ACT_HIP(hipEventCreate(&a));
        ACT_HIP(hipEventCreate(&b));
        p->ev_pool.push_back({a, b});
        p->ev_phase.push_back(0);
    }
    auto& ev = p->ev_pool[p->ev_used];
    p->ev_phase[p->ev_used] = phase;
    ++p->ev_used;
    ACT_HIP(hipEventRecord(ev.first, s));
    act_status st = launch();
    if (st != ACT_OK) return st;
    ACT_HIP(hipEventRecord(ev.second, s));
    return ACT_OK;
}

static act_status enqueue_order(act_plan_s* p, int batch, int k, int order, double* resid,
                                double* approx, double* theta, double* coef, long long* index,
                                double* energy, double* gap, int* flags, hipStream_t s) {
    act_status st;
    if ((st = timed(p, 0, s, [&] { return launch_search(p, batch, 0, s); })) != ACT_OK) return st;
    if (!search_emits_certified_set(p, batch) && (st = launch_overflow_check(p, batch, s)) != ACT_OK) return st;
    if ((st = timed(p, 1, s, [&] { return launch_search(p, batch, 1, s); })) != ACT_OK) return st;
    if ((st = timed(p, 2, s, [&] { return launch_rescore(p, batch, resid, s); })) != ACT_OK) return st;
    return timed(p, 3, s, [&] {
        return launch_select_refine_update(p, batch, k, order, resid, approx, theta, coef, index,
                                           energy, gap, flags, s);
    });
}

extern "C" act_status act_timing_enable(act_plan_t p, int32_t enable) {
    ACT_REQUIRE(p != nullptr, "act_timing_enable: plan is NULL");
    p->timing = enable != 0;
    return ACT_OK;
}

extern "C" act_status act_timing_read(act_plan_t p, double* ms, int64_t* launches) {
    ACT_REQUIRE(p != nullptr && ms != nullptr && launches != nullptr, "act_timing_read: NULL argument");
    for (int i = 0; i < 4; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    for (size_t i = 0; i < p->ev_used; ++i) {
        ACT_HIP(hipEventSynchronize(p->ev_pool[i].second));
        float t = 0.0f;
        ACT_HIP(hipEventElapsedTime(&t, p->ev_pool[i].first, p->ev_pool[i].second));
        ms[p->ev_phase[i]] += t;
        launches[p->ev_phase[i]] += 1;
    }
    p->ev_used = 0;
    return ACT_OK;
}

extern "C" act_status act_decompose(act_plan_t p, int32_t batch, const int32_t* len_dev,
                                    const int64_t* off_dev, double* resid_dev, double* approx_dev,
                                    int32_t order, double* theta_dev, double* coef_dev,
                                    int64_t* index_dev, double* energy_dev, double* gap_dev,
                                    int32_t* flags_dev, void* stream) {
    ACT_REQUIRE(p != nullptr, "act_decompose: plan is NULL");
    ACT_REQUIRE(batch >= 1 && batch <= p->max_batch, "act_decompose: batch outside [1, max_batch]");
    ACT_REQUIRE(order >= 1, "act_decompose: order must be >= 1");
    ACT_REQUIRE(resid_dev && theta_dev && coef_dev && index_dev && energy_dev && flags_dev,
                "act_decompose: NULL output pointer");
    if (p->desc.ragged) {
        ACT_REQUIRE(len_dev && off_dev, "act_decompose: ragged plans need len_dev and off_dev");
    } else {
        ACT_REQUIRE(!len_dev && !off_dev, "act_decompose: len_dev/off_dev are for ragged plans only");
    }
    hipStream_t s = (hipStream_t)stream;
    p->last_stream = s;
    p->search_resid = resid_dev;
    p->call_len = len_dev;
    p->call_off = (const long long*)off_dev;
    select_shape(p, batch);
    auto enqueue_all = [&](hipStream_t q) -> act_status {
        act_status st = launch_init(p, batch, resid_dev, approx_dev, energy_dev, flags_dev, order, q);
        if (st != ACT_OK) return st;
        if (p->desc.prior_act) {  // contrast mode: every order works on the original signal
            if ((st = launch_prior_init(p, batch, resid_dev, q)) != ACT_OK) return st;
            for (int k = 0; k < order; ++k) {
                st = timed(p, 3, q, [&] {
                    return launch_prior_order(p, batch, k, order, resid_dev, approx_dev, theta_dev, coef_dev,
                                              (long long*)index_dev, energy_dev, gap_dev, flags_dev, q);
                });
                if (st != ACT_OK) return st;
            }
            return ACT_OK;
        }
        if ((st = launch_ragged_items(p, batch, q)) != ACT_OK) return st;
        for (int k = 0; k < order; ++k) {
            st = enqueue_order(p, batch, k, order, resid_dev, approx_dev, theta_dev, coef_dev,
                               (long long*)index_dev, energy_dev, gap_dev, flags_dev, q);
            if (st != ACT_OK) return st;
        }
        return ACT_OK;
    };
    if (p->timing || !p->use_graphs) return enqueue_all(s);

    // One captured graph per argument signature, replayed on the caller's
    // stream: the whole pursuit becomes a single launch from the host.
    std::vector<uintptr_t> key = {(uintptr_t)batch, (uintptr_t)order, (uintptr_t)len_dev,
                                  (uintptr_t)off_dev, (uintptr_t)resid_dev,
                                  (uintptr_t)approx_dev, (uintptr_t)theta_dev, (uintptr_t)coef_dev,
                                  (uintptr_t)index_dev, (uintptr_t)energy_dev, (uintptr_t)gap_dev,
                                  (uintptr_t)flags_dev};
    for (auto& ge : p->graphs) {
        if (ge.key == key) {
            ge.last_use = ++p->graph_clock;
            ACT_HIP(hipGraphLaunch(ge.exec, s));
            return ACT_OK;
        }
    }
    // capture records without executing; the graph then runs in order on `s`
    if (!p->cap_stream) ACT_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    ACT_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    act_status st = enqueue_all(p->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(p->cap_stream, &graph);
    if (st != ACT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (ce != hipSuccess) {
        set_error(std::string("act_decompose: graph capture failed: ") + hipGetErrorString(ce));
        return ACT_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        set_error(std::string("act_decompose: graph instantiation failed: ") + hipGetErrorString(ie));
        return ACT_ERR_HIP;
    }
    if (p->graphs.size() >= 4) {  // evict the least recently used graph
        size_t lru = 0;
        for (size_t i = 1; i < p->graphs.size(); ++i)
            if (p->graphs[i].last_use < p->graphs[lru].last_use) lru = i;
        ACT_HIP(hipGraphExecDestroy(p->graphs[lru].exec));
        ACT_HIP(hipGraphDestroy(p->graphs[lru].graph));
        p->graphs.erase(p->graphs.begin() + lru);
    }
    p->graphs.push_back({key, graph, exec, ++p->graph_clock});
    ACT_HIP(hipGraphLaunch(exec, s));
    return ACT_OK;
}

// Host checks shared by both LEM entry points; *cap = candidates per stage.
static act_status check_lem(act_plan_t p, const act_lem_desc* cfg, int32_t batch, const double* lhs_dev,
                            double* resid_dev, int32_t order, double* theta_dev, double* coef_dev,
                            double* energy_dev, int32_t* flags_dev, const char* who, long long* cap) {
    const std::string w(who);
    ACT_REQUIRE(p != nullptr && cfg != nullptr, w + ": plan or settings NULL");
    if (!(p->desc.dict == ACT_DICT_SYNTH && p->desc.prec == ACT_PREC_F64 && !p->desc.ragged && !p->desc.prior_act &&
          !p->desc.complex_atoms)) {
        set_error(w + ": needs a plain ACT_DICT_SYNTH + ACT_PREC_F64 plan of real atoms");
        return ACT_ERR_UNSUPPORTED;
    }
    ACT_REQUIRE(batch >= 1 && batch <= p->max_batch, w + ": batch outside [1, max_batch]");
    ACT_REQUIRE(order >= 1, w + ": order must be >= 1");
    ACT_REQUIRE(cfg->samples >= 1 && cfg->levels >= 0 && cfg->levels <= 7 && cfg->topk >= 1 && cfg->topk <= 16,
                w + ": samples >= 1, levels in [0, 7], topk in [1, 16]");
    long long fam = 1;
    for (int d = 0; d < 4; ++d) {
        ACT_REQUIRE(cfg->radius[d] >= 0 && cfg->radius[d] <= 64, w + ": radius outside [0, 64]");
        fam *= 2 * cfg->radius[d] + 1;
    }
    for (int l = 0; l <= cfg->levels; ++l)
        for (int d = 0; d < 4; ++d)
            ACT_REQUIRE(std::isfinite(cfg->step[l][d]) && cfg->step[l][d] > 0.0, w + ": steps must be > 0");
    *cap = std::max<long long>(cfg->samples, cfg->topk * fam);
    ACT_REQUIRE(*cap <= 8192, w + ": more than 8192 candidates per stage");
    ACT_REQUIRE(lhs_dev && resid_dev && theta_dev && coef_dev && energy_dev && flags_dev, w + ": NULL pointer");
    return ACT_OK;
}

extern "C" act_status act_lem_decompose(act_plan_t p, const act_lem_desc* cfg, int32_t batch,
                                        const double* lhs_dev, double* resid_dev, double* approx_dev,
                                        int32_t order, double* theta_dev, double* coef_dev, double* energy_dev,
                                        int32_t* flags_dev, void* stream) {
    long long cap = 0;
    act_status st = check_lem(p, cfg, batch, lhs_dev, resid_dev, order, theta_dev, coef_dev, energy_dev, flags_dev,
                              "act_lem_decompose", &cap);
    if (st != ACT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    p->last_stream = s;
    if (p->lem_cap < cap) {  // workspace: candidates, scores and marks per channel
        ACT_HIP(hipStreamSynchronize(s));
        if (p->lem_cand) ACT_HIP(hipFree(p->lem_cand));
        if (p->lem_score) ACT_HIP(hipFree(p->lem_score));
        p->lem_cand = nullptr;
        p->lem_score = nullptr;
        p->lem_cap = 0;
        ACT_HIP(hipMalloc((void**)&p->lem_cand, (size_t)p->max_batch * cap * 4 * sizeof(double)));
        ACT_HIP(hipMalloc((void**)&p->lem_score, (size_t)p->max_batch * cap * (sizeof(double) + 1)));
        p->lem_cap = (int)cap;
    }
    char* used = (char*)(p->lem_score + (size_t)p->max_batch * p->lem_cap);
    st = launch_init(p, batch, resid_dev, approx_dev, energy_dev, flags_dev, order, s);
    if (st != ACT_OK) return st;
    for (int k = 0; k < order; ++k) {
        st = timed(p, 3, s, [&] {
            return launch_lem_order(p, cfg, p->lem_cap, p->lem_cand, p->lem_score, used, batch, k, order, lhs_dev,
                                    resid_dev, approx_dev, theta_dev, coef_dev, energy_dev, flags_dev, s);
        });
        if (st != ACT_OK) return st;
    }
    return ACT_OK;
}

// Workspace of act_lem_decompose_noalloc: one array per device, held until
// the process ends.  Host code never passes `scratch` itself (on the host it
// names a stand-in, not device memory); it takes the device address from
// hipGetSymbolAddress, once per device with that device current.
static __device__ __align__(256) char scratch[ACT_LEM_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static act_status scratch_for_current_device(char** out) {
    int dev = -1;
    ACT_HIP(hipGetDevice(&dev));
    ACT_REQUIRE(dev >= 0 && dev < kMaxDevices, "act_lem_decompose_noalloc: device index outside [0, 64)");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        ACT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        ACT_REQUIRE(ptr != nullptr, "act_lem_decompose_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = (char*)g_scratch_ptr[dev];
    return ACT_OK;
}

extern "C" act_status act_lem_decompose_noalloc(act_plan_t p, const act_lem_desc* cfg, int32_t batch,
                                                const double* lhs_dev, double* resid_dev, double* approx_dev,
                                                int32_t order, double* theta_dev, double* coef_dev,
                                                double* energy_dev, int32_t* flags_dev, void* stream) {
    long long cap = 0;
    act_status st = check_lem(p, cfg, batch, lhs_dev, resid_dev, order, theta_dev, coef_dev, energy_dev, flags_dev,
                              "act_lem_decompose_noalloc", &cap);
    if (st != ACT_OK) return st;
    const unsigned long long need = (unsigned long long)batch * (unsigned long long)cap * (4 * sizeof(double) +
                                                                                          sizeof(double) + 1);
    if (need > (unsigned long long)ACT_LEM_SCRATCH_BYTES) {
        set_error("act_lem_decompose_noalloc: batch x candidates per stage x 41 bytes = " + std::to_string(need) +
                  " exceeds the " + std::to_string((unsigned long long)ACT_LEM_SCRATCH_BYTES) +
                  "-byte scratch array; use act_lem_decompose");
        return ACT_ERR_INVALID;
    }
    char* base = nullptr;
    if ((st = scratch_for_current_device(&base)) != ACT_OK) return st;
    // [batch][cap][4] parameters, then [batch][cap] scores, then [batch][cap] marks;
    // every entry is written by the kernel before it is read, so no clearing
    double* cand = (double*)base;
    double* score = cand + (size_t)batch * cap * 4;
    char* used = (char*)(score + (size_t)batch * cap);
    hipStream_t s = (hipStream_t)stream;
    p->last_stream = s;
    st = launch_init(p, batch, resid_dev, approx_dev, energy_dev, flags_dev, order, s);
    if (st != ACT_OK) return st;
    for (int k = 0; k < order; ++k) {
        st = launch_lem_order(p, cfg, (int)cap, cand, score, used, batch, k, order, lhs_dev, resid_dev, approx_dev,
                              theta_dev, coef_dev, energy_dev, flags_dev, s);
        if (st != ACT_OK) return st;
    }
    return ACT_OK;
}

extern "C" act_status act_refine(act_plan_t p, int32_t m, const double* resid_dev,
                                 const double* theta0_dev, int32_t steps, double* theta_dev,
                                 double* value_dev, int32_t* flags_dev, void* stream) {
    ACT_REQUIRE(p != nullptr, "act_refine: plan is NULL");
    ACT_REQUIRE(!p->desc.ragged, "act_refine: ragged plans are not supported");
    ACT_REQUIRE(m >= 1 && steps >= 0, "act_refine: m must be >= 1 and steps >= 0");
    ACT_REQUIRE(resid_dev && theta0_dev && theta_dev && value_dev, "act_refine: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    p->last_stream = s;
    return launch_refine_many(p, m, resid_dev, theta0_dev, steps, theta_dev, value_dev, flags_dev, s);
}

extern "C" act_status act_refine_f32(act_plan_t p, int32_t m, const float* resid_dev, const double* theta0_dev,
                                     int32_t steps, double* theta_dev, double* value_dev, int32_t* flags_dev,
                                     void* stream) {
    ACT_REQUIRE(p != nullptr, "act_refine_f32: plan is NULL");
    ACT_REQUIRE(!p->desc.ragged, "act_refine_f32: ragged plans are not supported");
    ACT_REQUIRE(m >= 1 && steps >= 0, "act_refine_f32: m must be >= 1 and steps >= 0");
    ACT_REQUIRE(resid_dev && theta0_dev && theta_dev && value_dev, "act_refine_f32: NULL pointer");
    if (p->desc.complex_atoms || p->desc.prior_act) {
        set_error("act_refine_f32: the FP32 refinement is for the real atoms of the residue-based ACT");
        return ACT_ERR_UNSUPPORTED;
    }
    hipStream_t s = (hipStream_t)stream;
    p->last_stream = s;
    return launch_refine_many_f32(p, m, resid_dev, theta0_dev, steps, theta_dev, value_dev, flags_dev, s);
}

extern "C" act_status act_value_and_grad(act_plan_t p, int32_t m, int32_t dtype,
                                         const void* resid_dev, const double* theta_dev,
                                         double* value_dev, double* dtheta_dev, void* dr_dev,
                                         void* stream) {
    ACT_REQUIRE(p != nullptr, "act_value_and_grad: plan is NULL");
    ACT_REQUIRE(!p->desc.ragged, "act_value_and_grad: ragged plans are not supported");
    ACT_REQUIRE(m >= 1, "act_value_and_grad: m must be >= 1");
    ACT_REQUIRE(dtype == ACT_PREC_F64 || dtype == ACT_PREC_F32, "act_value_and_grad: dtype must be F64 or F32");
    ACT_REQUIRE(resid_dev && theta_dev && value_dev && dtheta_dev, "act_value_and_grad: NULL pointer");
    if (p->desc.complex_atoms) {
        set_error("act_value_and_grad: the forward/adjoint is for real atoms; complex plans refine with act_refine");
        return ACT_ERR_UNSUPPORTED;
    }
    hipStream_t s = (hipStream_t)stream;
    p->last_stream = s;
    return launch_value_and_grad(p, m, dtype, resid_dev, theta_dev, value_dev, dtheta_dev, dr_dev, s);
}

extern "C" act_status act_reconstruct(act_plan_t p, int32_t batch, int32_t order,
                                      const double* theta_dev, const double* coef_dev,
                                      const int32_t* len_dev, const int64_t* off_dev,
                                      double* out_dev, void* stream) {
    ACT_REQUIRE(p != nullptr, "act_reconstruct: plan is NULL");
    ACT_REQUIRE(batch >= 1 && order >= 0, "act_reconstruct: batch must be >= 1, order >= 0");
    ACT_REQUIRE(theta_dev && coef_dev && out_dev, "act_reconstruct: NULL pointer");
    if (p->desc.ragged)
        ACT_REQUIRE(len_dev && off_dev, "act_reconstruct: ragged plans need len_dev and off_dev");
    else
        ACT_REQUIRE(!len_dev && !off_dev, "act_reconstruct: len_dev/off_dev are for ragged plans only");
    hipStream_t s = (hipStream_t)stream;
    p->last_stream = s;
    return launch_reconstruct(p, batch, order, theta_dev, coef_dev, len_dev, (const long long*)off_dev,
                              out_dev, s);
}

extern "C" act_status act_correlate(act_plan_t p, int32_t batch, const double* resid_dev,
                                    int64_t atom_begin, int64_t atom_count, double* score_dev,
                                    void* stream) {
    ACT_REQUIRE(p != nullptr, "act_correlate: plan is NULL");
    ACT_REQUIRE(!p->desc.ragged, "act_correlate: ragged plans are not supported");
    ACT_REQUIRE(batch >= 1 && batch <= p->max_batch, "act_correlate: batch outside [1, max_batch]");
    ACT_REQUIRE(atom_begin >= 0 && atom_count >= 1 && atom_begin + atom_count <= p->atoms,
                "act_correlate: atom range outside the dictionary");
    ACT_REQUIRE(resid_dev && score_dev, "act_correlate: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    p->last_stream = s;
    select_shape(p, batch);
    if (p->desc.prec != ACT_PREC_F64) {
        act_status st = launch_to_shadow(p, batch, resid_dev, s);
        if (st != ACT_OK) return st;
    }
    return launch_correlate(p, batch, resid_dev, atom_begin, atom_count, score_dev, s);
}
