// Achievable matrix-core throughput on this device: every wave issues long runs
// of independent MFMAs on register operands (eight accumulation chains, no
// memory traffic inside the loop), four waves per SIMD.  Measurement support
// for the roofline figures; not part of the method.
#pragma once

#include <hip/hip_runtime.h>

#include "gemm_bf16x3.hpp"

namespace cpa {

constexpr int kPeakChains = 8;

// KIND 0: v_mfma_f32_16x16x4f32 (2048 flop), 1: v_mfma_f32_16x16x32_bf16 (16384 flop).
// clk (nullable): the first wave of the first workgroup stores the shader-clock
// counter and the constant-rate wall counter before and after its MFMA loop, so
// the host can tell the clock the matrix cores ran at.
template <int KIND>
__global__ void __launch_bounds__(256) peak_mfma_kernel(int iters, float* out, unsigned long long* clk) {
    const bool timer = clk != nullptr && blockIdx.x == 0 && threadIdx.x == 0;
    unsigned long long cyc0 = 0, wall0 = 0;
    if (timer) {
        cyc0 = clock64();
        wall0 = wall_clock64();
    }
    f32x4 c[kPeakChains];
#pragma unroll
    for (int i = 0; i < kPeakChains; ++i) c[i] = (f32x4){0.f, 0.f, 0.f, 0.f};
    if (KIND == 0) {
        const float a = 1e-3f * (float)threadIdx.x, b = 1.f - 1e-4f * (float)threadIdx.x;
        for (int t = 0; t < iters; ++t) {
#pragma unroll
            for (int i = 0; i < kPeakChains; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[i], 0, 0, 0);
        }
    } else {
        typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
        u16x8 ua, ub;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            ua[e] = bf16_bits(1e-3f * (float)(threadIdx.x + e));
            ub[e] = bf16_bits(1.f);
        }
        const bf16x8 a = __builtin_bit_cast(bf16x8, ua), b = __builtin_bit_cast(bf16x8, ub);
        for (int t = 0; t < iters; ++t) {
#pragma unroll
            for (int i = 0; i < kPeakChains; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[i], 0, 0, 0);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kPeakChains; ++i) s += (c[i][0] + c[i][1]) + (c[i][2] + c[i][3]);
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
    if (timer) {
        const unsigned long long cyc1 = clock64(), wall1 = wall_clock64();
        clk[0] = cyc1 - cyc0;
        clk[1] = wall1 - wall0;
    }
}

}  // namespace cpa
