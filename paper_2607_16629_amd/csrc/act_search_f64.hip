// act_search_f64.hip -- coarse search with FP64 atoms synthesised on the fly.
#include "act_emit.h"

namespace act {

// --------------------------------------------------------------------------
// FP64: one lane per atom, atoms synthesised from Eq. (1) in FP64 on the fly,
// p = <g, r> / |g| with the norm taken over the same samples (complex atoms:
// p = |<g, r>| / |E|).  blockIdx.y = channel.
// --------------------------------------------------------------------------
template <bool RERUN, bool CPLX>
__global__ void __launch_bounds__(256) k_search_f64(GridDev g0, const double* __restrict__ resid,
                                                   SearchCtl ctl) {
    const int b = blockIdx.y;
    if (RERUN && ctl.need_rerun[b] == 0) return;
    const ChanGeom cg = chan_geom(g0, b, ctl.len, ctl.off);
    const GridDev& g = cg.g;
    const double* r = resid + cg.off;
    const long long total = ctl.dump ? ctl.dump_count : g.atoms;
    const long long base0 = ctl.dump ? ctl.dump_begin : 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long j0 = (long long)blockIdx.x * blockDim.x; j0 < total; j0 += stride) {
        const long long j = j0 + threadIdx.x;
        const bool valid = j < total;
        const long long i = base0 + (valid ? j : 0);
        double th[4];
        grid_theta(g, i, th);
        const double inv_dt = 1.0 / exp(th[3]);
        double s = 0.0, q = 0.0, sb = 0.0;
        for (int k = 0; k < g.n; ++k) {
            if constexpr (CPLX) {
                double re, im, e;
                atom_parts64(sample_time(k, g.fs), th[0], th[1], th[2], inv_dt, re, im, e);
                s += re * r[k];
                sb += im * r[k];
                q += e * e;
            } else {
                double v = atom_sample64(sample_time(k, g.fs), th[0], th[1], th[2], inv_dt);
                s += v * r[k];
                q += v * v;
            }
        }
        if constexpr (CPLX) s = sqrt(s * s + sb * sb);
        const double p = q > 0.0 ? s / sqrt(q) : 0.0;
        if (ctl.dump) {
            if (valid) ctl.dump[(size_t)b * ctl.dump_count + j] = p;
        } else {
            emit_uniform(ctl, b, i, (float)p, valid);
        }
    }
}


act_status launch_search_f64(act_plan_s* p, int batch, const SearchCtl& ctl, const double* resid,
                             hipStream_t s) {
    // ragged plans: every channel's dictionary is at most the widest one
    const long long total = ctl.dump ? ctl.dump_count : p->atoms;
    long long blocks = (total + 255) / 256;
    const long long cap = grid_cap(p, 16);
    blocks = blocks < cap ? blocks : cap;
    if (blocks < 1) blocks = 1;
    const bool cx = p->desc.complex_atoms != 0;
    if (ctl.pass)
        hipLaunchKernelGGL((cx ? k_search_f64<true, true> : k_search_f64<true, false>), dim3((unsigned)blocks, batch),
                           dim3(256), 0, s, p->grid, resid, ctl);
    else
        hipLaunchKernelGGL((cx ? k_search_f64<false, true> : k_search_f64<false, false>),
                           dim3((unsigned)blocks, batch), dim3(256), 0, s, p->grid, resid, ctl);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

}  // namespace act
