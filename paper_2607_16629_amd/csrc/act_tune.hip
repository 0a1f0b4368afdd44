// act_tune.hip -- launch-shape autotuner of the coarse search.
//
// The search kernels run persistent grids over their tiles; how many
// workgroups per CU pay off (latency hiding against L2 locality and the tail),
// and for the FP16 synthesis of several channels how a tile's 128 columns are
// split between f_c values and channels, depend on the plan and the batch.
// act_tune times the pass-0 search of each candidate on the caller's residual
// and keeps the fastest per batch size.  Shapes never change results: each
// score's arithmetic is fixed by the kernel, and the certified candidate
// selection plus FP64 rescoring decide the winner exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "act_common.h"

namespace act {

void select_shape(act_plan_s* p, int batch) {
    p->shape = act_launch_shape{};
    for (const auto& e : p->shapes)
        if (e.first == batch) p->shape = e.second;
}

long long grid_cap(const act_plan_s* p, int def) {
    const int g = p->shape.grid_per_cu > 0 ? p->shape.grid_per_cu : def;
    return (long long)device_cus() * g;
}

// candidate shapes of the plan's search kernel
static std::vector<act_launch_shape> candidates(const act_plan_s* p, int batch) {
    std::vector<int> grids;
    std::vector<int> cpfs = {0};
    const auto& d = p->desc;
    if (d.dict == ACT_DICT_LAG) {
        grids = {1, 2};
    } else if (d.prec == ACT_PREC_F64) {
        grids = {4, 8, 16, 32};
    } else if (d.dict == ACT_DICT_TABLE && d.prec == ACT_PREC_F32) {
        grids = {2, 4, 8, 16};
    } else if (d.dict == ACT_DICT_TABLE) {  // BF16 table
        grids = {1, 2, 4};
    } else if (d.prec == ACT_PREC_F32) {  // FP32 synthesis
        grids = d.ragged ? std::vector<int>{1, 2, 4} : std::vector<int>{1, 2, 4, 8};
    } else {  // FP16 synthesis
        grids = d.ragged ? std::vector<int>{1, 2, 3, 4} : std::vector<int>{1, 2, 4};
        if (!d.ragged && batch > 1) {
            int top = 1;
            while (top < batch && top < 64) top *= 2;
            cpfs.clear();
            for (int c = top; c >= 1 && (int)cpfs.size() < 4; c /= 2) cpfs.push_back(c);
        }
    }
    std::vector<act_launch_shape> out;
    // lag-table search: the resident-residual form (its own grid) where it
    // applies, then the staged tiles
    const bool rs = d.dict == ACT_DICT_LAG && p->lag_rs_cp && batch >= 32;
    if (rs) {
        act_launch_shape s{};
        s.grid_per_cu = 1;
        out.push_back(s);
    }
    for (int g : grids)
        for (int c : cpfs) {
            act_launch_shape s{};
            s.grid_per_cu = g;
            s.chan_per_fc = c;
            s.form = rs ? 1 : 0;
            out.push_back(s);
        }
    return out;
}

// the cache key: device, plan shape, batch
static std::string cache_key(const act_plan_s* p, int batch) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        for (char& ch : arch)
            if (ch == ' ') ch = '_';
    }
    const auto& d = p->desc;
    std::ostringstream k;
    k << arch << ' ' << device_cus() << ' ' << d.dict << ' ' << d.prec << ' ' << d.grid.n_samples << ' '
      << d.grid.tc_s.count << ' ' << d.grid.fc_hz.count << ' ' << d.grid.c_hz_per_s.count << ' '
      << d.grid.logdt_ln_s.count << ' ' << d.ragged << ' ' << (d.ragged ? d.ragged_tc_div : 0) << ' '
      << d.support_cut << ' ' << d.complex_atoms << ' ' << batch;
    return k.str();
}

static constexpr int kKeyFields = 14;

static bool cache_lookup(const char* path, const std::string& key, act_launch_shape* s) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream in(line);
        std::string tok, k;
        for (int i = 0; i < kKeyFields && (in >> tok); ++i) k += (i ? " " : "") + tok;
        act_launch_shape v{};
        if (k == key && (in >> v.grid_per_cu >> v.chan_per_fc >> v.form >> v.ms) && v.grid_per_cu > 0 &&
            v.grid_per_cu <= 64 && v.chan_per_fc >= 0 && v.chan_per_fc <= 64 && (v.form == 0 || v.form == 1)) {
            v.from_cache = 1;
            *s = v;  // the last matching line wins
            found = true;
        }
    }
    return found;
}

static void cache_append(const char* path, const std::string& key, const act_launch_shape& s) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;  // the choice still applies; the cache is best effort
    std::fprintf(f, "%s %d %d %d %.6f\n", key.c_str(), s.grid_per_cu, s.chan_per_fc, s.form, s.ms);
    std::fclose(f);
}

static void drop_graphs(act_plan_s* p) {
    for (auto& ge : p->graphs) {
        if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
        if (ge.graph) (void)hipGraphDestroy(ge.graph);
    }
    p->graphs.clear();
}

static void keep_shape(act_plan_s* p, int batch, const act_launch_shape& s) {
    for (auto& e : p->shapes)
        if (e.first == batch) {
            e.second = s;
            drop_graphs(p);
            return;
        }
    p->shapes.push_back({batch, s});
    drop_graphs(p);
}

}  // namespace act

using namespace act;

extern "C" act_status act_set_launch_shape(act_plan_t p, int32_t batch, const act_launch_shape* shape) {
    ACT_REQUIRE(p != nullptr && shape != nullptr, "act_set_launch_shape: plan or shape is NULL");
    ACT_REQUIRE(batch >= 1 && batch <= p->max_batch, "act_set_launch_shape: batch outside [1, max_batch]");
    ACT_REQUIRE(shape->grid_per_cu >= 1 && shape->grid_per_cu <= 64 && shape->chan_per_fc >= 0 &&
                    shape->chan_per_fc <= 64 && (shape->form == 0 || shape->form == 1),
                "act_set_launch_shape: grid_per_cu outside [1, 64], chan_per_fc outside [0, 64] or form not 0/1");
    act_launch_shape v = *shape;
    v.from_cache = 0;
    v.ms = 0.0;
    keep_shape(p, batch, v);
    return ACT_OK;
}

extern "C" act_status act_tune(act_plan_t p, int32_t batch, const int32_t* len_dev, const int64_t* off_dev,
                               const double* resid_dev, int32_t reps, const char* cache_path,
                               act_launch_shape* out, void* stream) {
    ACT_REQUIRE(p != nullptr, "act_tune: plan is NULL");
    ACT_REQUIRE(batch >= 1 && batch <= p->max_batch, "act_tune: batch outside [1, max_batch]");
    ACT_REQUIRE(reps >= 1 && reps <= 100, "act_tune: reps outside [1, 100]");
    ACT_REQUIRE(resid_dev != nullptr, "act_tune: resid_dev is NULL");
    if (p->desc.ragged) {
        ACT_REQUIRE(len_dev && off_dev, "act_tune: ragged plans need len_dev and off_dev");
    } else {
        ACT_REQUIRE(!len_dev && !off_dev, "act_tune: len_dev/off_dev are for ragged plans only");
    }
    if (p->desc.prior_act) {
        set_error("act_tune: the prior ACT's search has no tunable launch shape");
        return ACT_ERR_UNSUPPORTED;
    }
    hipStream_t s = (hipStream_t)stream;
    p->last_stream = s;
    const std::string key = cache_key(p, batch);
    act_launch_shape best{};
    if (cache_path && cache_lookup(cache_path, key, &best)) {
        keep_shape(p, batch, best);
        if (out) *out = best;
        return ACT_OK;
    }

    // per-channel outputs of the init pass (|s|^2, flags): scratch of the tuner
    double* energy = nullptr;
    int* flags = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&] {
        if (energy) (void)hipFree(energy);
        if (flags) (void)hipFree(flags);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    act_status st = ACT_OK;
    auto hip_ok = [&](hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        set_error(std::string("act_tune: ") + what + ": " + hipGetErrorString(e));
        st = ACT_ERR_HIP;
        return false;
    };
    if (!hip_ok(hipMalloc((void**)&energy, sizeof(double) * batch), "hipMalloc") ||
        !hip_ok(hipMalloc((void**)&flags, sizeof(int) * batch), "hipMalloc") ||
        !hip_ok(hipEventCreate(&e0), "hipEventCreate") || !hip_ok(hipEventCreate(&e1), "hipEventCreate")) {
        release();
        return st;
    }
    p->search_resid = resid_dev;
    p->call_len = len_dev;
    p->call_off = (const long long*)off_dev;
    double best_ms = -1.0;
    for (const act_launch_shape& cand : candidates(p, batch)) {
        p->shape = cand;
        double total = 0.0;
        for (int r = 0; r < reps && st == ACT_OK; ++r) {
            // fresh search state (running maxima, candidate counts, queues)
            if ((st = launch_init(p, batch, const_cast<double*>(resid_dev), nullptr, energy, flags, 0, s)) != ACT_OK)
                break;
            if ((st = launch_ragged_items(p, batch, s)) != ACT_OK) break;
            if (!hip_ok(hipEventRecord(e0, s), "hipEventRecord")) break;
            if ((st = launch_search(p, batch, 0, s)) != ACT_OK) break;
            if (!hip_ok(hipEventRecord(e1, s), "hipEventRecord")) break;
            if (!hip_ok(hipEventSynchronize(e1), "hipEventSynchronize")) break;
            float ms = 0.0f;
            if (!hip_ok(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) break;
            total += ms;
        }
        if (st != ACT_OK) break;
        const double mean = total / reps;
        if (best_ms < 0.0 || mean < best_ms) {
            best_ms = mean;
            best = cand;
            best.ms = mean;
        }
    }
    release();
    p->shape = act_launch_shape{};
    if (st != ACT_OK) return st;
    keep_shape(p, batch, best);
    if (cache_path) cache_append(cache_path, key, best);
    if (out) *out = best;
    return ACT_OK;
}
