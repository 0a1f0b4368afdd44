// act_probe.hip -- measurement probes for the achievable peaks of the chip the
// library runs on, reported beside the datasheet peaks: a streaming read of a
// large buffer (HBM bandwidth) and dependent-free MFMA loops (matrix-core
// rate).  Not part of the method; the caller times each launch on its stream.
#include "act_common.h"

namespace act {

typedef _Float16 p16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 pb16x8 __attribute__((ext_vector_type(8)));
typedef float p32x16 __attribute__((ext_vector_type(16)));
typedef float p32x4 __attribute__((ext_vector_type(4)));

// Grid-stride read of n4 float4 (16-byte) elements, 8 loads in flight per
// thread; the sum is stored only if it hits an impossible value, which keeps
// the loads without writing anything.
__global__ void __launch_bounds__(256) k_probe_read(const p32x4* __restrict__ src, long long n4,
                                                    float* __restrict__ sink) {
    constexpr int U = 8;
    const long long stride = (long long)gridDim.x * 256;
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    float acc = 0.0f;
    for (; i + (U - 1) * stride < n4; i += U * stride) {
        p32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    for (; i < n4; i += stride) {
        const p32x4 v = __builtin_nontemporal_load(src + i);
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (acc == -1.2345e-37f) sink[0] = acc;
}

// Four independent 32x32 accumulators per wave, `iters` rounds of four MFMAs.
// KIND 0: v_mfma_f32_32x32x16_bf16, 1: _f16, 2: v_mfma_f32_32x32x2_f32.
template <int KIND>
__global__ void __launch_bounds__(256) k_probe_mfma(int iters, float* __restrict__ sink) {
    const float x = 1.0f + 1e-3f * (float)(threadIdx.x & 63);
    p32x16 c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) c[j][v] = 0.0f;
    if constexpr (KIND == 2) {
        const float a = x, b = 1.0f - x;
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int j = 0; j < 4; ++j) c[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c[j], 0, 0, 0);
    } else {
        p16x8 a16, b16;
        pb16x8 a_b, b_b;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a16[k] = (_Float16)(x + 0.01f * k);
            b16[k] = (_Float16)(x - 0.01f * k);
            a_b[k] = (__bf16)(x + 0.01f * k);
            b_b[k] = (__bf16)(x - 0.01f * k);
        }
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if constexpr (KIND == 0)
                    c[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_b, b_b, c[j], 0, 0, 0);
                else
                    c[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a16, b16, c[j], 0, 0, 0);
            }
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) s += c[j][v];
    if (s == -1.2345e-37f) sink[0] = s;
}

}  // namespace act

using namespace act;

extern "C" act_status act_probe_read(const void* buf_dev, int64_t bytes, int32_t blocks_per_cu, float* sink_dev,
                                     void* stream) {
    ACT_REQUIRE(buf_dev && sink_dev, "act_probe_read: NULL pointer");
    ACT_REQUIRE(bytes >= 16 && bytes % 16 == 0 && ((uintptr_t)buf_dev & 15) == 0,
                "act_probe_read: bytes must be a positive multiple of 16 and the buffer 16-byte aligned");
    ACT_REQUIRE(blocks_per_cu >= 1 && blocks_per_cu <= 64, "act_probe_read: blocks_per_cu outside [1, 64]");
    const long long n4 = bytes / 16;
    long long blocks = (long long)device_cus() * blocks_per_cu;
    const long long need = (n4 + 255) / 256;
    if (blocks > need) blocks = need;
    hipLaunchKernelGGL(k_probe_read, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const p32x4*)buf_dev, n4, sink_dev);
    ACT_HIP(hipGetLastError());
    return ACT_OK;
}

extern "C" act_status act_probe_mfma(int32_t prec, int32_t iters, int32_t blocks_per_cu, float* sink_dev,
                                     double* flops, void* stream) {
    ACT_REQUIRE(sink_dev && flops, "act_probe_mfma: NULL pointer");
    ACT_REQUIRE(prec == ACT_PREC_BF16 || prec == ACT_PREC_F16 || prec == ACT_PREC_F32,
                "act_probe_mfma: prec must be ACT_PREC_BF16, ACT_PREC_F16 or ACT_PREC_F32");
    ACT_REQUIRE(iters >= 1 && iters <= (1 << 24), "act_probe_mfma: iters outside [1, 2^24]");
    ACT_REQUIRE(blocks_per_cu >= 1 && blocks_per_cu <= 16, "act_probe_mfma: blocks_per_cu outside [1, 16]");
    const long long blocks = (long long)device_cus() * blocks_per_cu;
    const dim3 grid((unsigned)blocks), blk(256);
    hipStream_t s = (hipStream_t)stream;
    double per_mfma;
    if (prec == ACT_PREC_BF16) {
        hipLaunchKernelGGL(k_probe_mfma<0>, grid, blk, 0, s, iters, sink_dev);
        per_mfma = 32.0 * 32.0 * 16.0 * 2.0;
    } else if (prec == ACT_PREC_F16) {
        hipLaunchKernelGGL(k_probe_mfma<1>, grid, blk, 0, s, iters, sink_dev);
        per_mfma = 32.0 * 32.0 * 16.0 * 2.0;
    } else {
        hipLaunchKernelGGL(k_probe_mfma<2>, grid, blk, 0, s, iters, sink_dev);
        per_mfma = 32.0 * 32.0 * 2.0 * 2.0;
    }
    ACT_HIP(hipGetLastError());
    // blocks x 4 waves x 4 accumulators x iters MFMAs
    *flops = (double)blocks * 4.0 * 4.0 * (double)iters * per_mfma;
    return ACT_OK;
}
