// Elementwise parts of the RPCA ADMM iteration (Appendix B, eq. admm_algorithm_mod):
// the closed-form (K^T K)^{-1} K^T (z - u) update, the l1 prox, the projection
// onto the observed data and the dual update, with the stopping quantity
// E_t = ||l_{t+1} - l_t|| / ||l_{t+1}|| (Sec. V-B.2) reduced in FP64.
// Arrays are contiguous m*n float blocks processed by grid-stride loops
// (consecutive lanes touch consecutive elements).  The two E_t sums are
// per-workgroup partials (part[2 * block], part[2 * block + 1]) added in a fixed
// order by the first workgroup of the post kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spectral.hpp"

namespace cpa {

struct AdmmPtrs {
    float* l;
    float* s;
    float* z1;
    float* z2;
    float* u1;
    float* u2;
    float* u3;
    const float* I;
    float* x;   // shrink input l + u1
};

__device__ inline void admm_pre_elem(const AdmmPtrs& P, int64_t e, double& dn, double& dd) {
    const float Ie = P.I[e], u3 = P.u3[e];
    const float a = (P.z1[e] - P.u1[e]) + (Ie - u3);
    const float b = (P.z2[e] - P.u2[e]) + (Ie - u3);
    const float l = (2.f * a - b) * (1.f / 3.f);
    const float s = (2.f * b - a) * (1.f / 3.f);
    const float dl = l - P.l[e];
    dn += (double)dl * dl;
    dd += (double)l * l;
    P.l[e] = l;
    P.s[e] = s;
    P.x[e] = l + P.u1[e];
}

// l, s <- (K^T K)^{-1} K^T (z - u); x <- l + u1; E_t partial sums.
__global__ void __launch_bounds__(256) admm_pre_kernel(AdmmPtrs P, int64_t total, double* part) {
    __shared__ double red[8];
    double dn = 0.0, dd = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride)
        admm_pre_elem(P, e, dn, dd);
    dn = block_sum(dn, red);
    dd = block_sum(dd, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = dn;
        part[2 * blockIdx.x + 1] = dd;
    }
}

// z1 already holds the shrink of x.  z2 = soft(s + u2); u1 += l - z1; u2 += s - z2;
// u3 += l + s - I.  The first workgroup also stores E_t (the pre kernel completed).
// E_t goes to Et_base[*counter] and the counter advances, so the same launch
// (or a replayed graph of it) fills consecutive entries.
__global__ void __launch_bounds__(256) admm_post_kernel(AdmmPtrs P, int64_t total, float t2, const double* part,
                                                        int npart, double* Et_base, int* counter) {
    __shared__ double red[8];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
        const float l = P.l[e], s = P.s[e];
        const float v = s + P.u2[e];
        const float av = fabsf(v) - t2;
        const float z2 = av > 0.f ? copysignf(av, v) : 0.f;
        P.z2[e] = z2;
        P.u1[e] = P.u1[e] + l - P.z1[e];
        P.u2[e] = P.u2[e] + s - z2;
        P.u3[e] = P.u3[e] + l + s - P.I[e];
    }
    if (Et_base && blockIdx.x == 0) {
        double num = 0.0, den = 0.0;
        for (int i = threadIdx.x; i < npart; i += blockDim.x) {
            num += part[2 * i];
            den += part[2 * i + 1];
        }
        num = block_sum(num, red);
        den = block_sum(den, red);
        if (threadIdx.x == 0) {
            const int t = *counter;
            Et_base[t] = den > 0.0 ? sqrt(num / den) : 0.0;
            *counter = t + 1;
        }
    }
}

__global__ void fill_i32_kernel(int* p, int n, int v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace cpa
