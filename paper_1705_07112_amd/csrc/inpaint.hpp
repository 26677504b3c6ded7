// Elementwise parts of the texture-inpainting ADMM (Appendix A, eq.
// admm_algorithm_inp) on z = K l, K = [Id; Psi; Omega; Id; Omega_bar]:
//   l  = (K^T K)^{-1} K^T (z - u), with K^T K = 3 Id + Omega + Omega_bar (= 4 Id)
//        when the mean term is on and 3 Id + Omega without it; the Psi^T (z2 - u2)
//        term arrives from two products with the DCT matrices;
//   z1 = the CPA shrink of l + u1 (the library's dense shrinkage);
//   z2 = soft(Psi l + u2, eta/rho), Psi l from two products;
//   z3 = Omega i (the observed pixels), z4 = clip(l + u4, 0, 1),
//   z5 = y + Omega_bar (c - mean of y over the region), y = Omega_bar l + u5,
//        c = the mean of the observed image over the surrounding pixels;
//   u += K l - z, and E_t = ||l_{t+1} - l_t|| / ||l_{t+1}|| in FP64.
// Arrays are contiguous m*n float blocks processed by grid-stride loops; the
// FP64 sums are per-workgroup partials added in a fixed order, so every
// workgroup of the post kernel computes the same region mean.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spectral.hpp"

namespace cpa {

constexpr int kInpGrid = 1024;   // workgroups of the elementwise kernels (at most)

struct InpPtrs {
    float* l;
    float* z[5];
    float* u[5];
    const float* I;
    const float* om;   // 1 on the observed pixels, 0 on the region to recover
    float* x;          // shrink input l + u1
    const float* T;    // Psi^T (z2 - u2) before the shrink, Psi l after it
    int ave;           // the mean term (z5, u5) is on
};

// A = z2 - u2 (the input of Psi^T).
__global__ void __launch_bounds__(256) inp_diff_kernel(int64_t total, const float* a, const float* b, float* out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = a[e] - b[e];
}

// l, x, E_t partials and the region sum of y = Omega_bar l + u5 (old u5).
__global__ void __launch_bounds__(256) inp_pre_kernel(InpPtrs P, int64_t total, double* part) {
    __shared__ double red[8];
    double dn = 0.0, dd = 0.0, sy = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
        const float w = P.om[e], wb = 1.f - w;
        float r = ((P.z[0][e] - P.u[0][e]) + P.T[e]) + w * (P.z[2][e] - P.u[2][e]) + (P.z[3][e] - P.u[3][e]);
        float dg = 3.f + w;
        if (P.ave) {
            r += wb * (P.z[4][e] - P.u[4][e]);
            dg += wb;
        }
        const float l = r / dg;
        const float dl = l - P.l[e];
        dn += (double)dl * dl;
        dd += (double)l * l;
        if (P.ave && w == 0.f) sy += (double)(wb * l + P.u[4][e]);
        P.l[e] = l;
        P.x[e] = l + P.u[0][e];
    }
    dn = block_sum(dn, red);
    dd = block_sum(dd, red);
    sy = block_sum(sy, red);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = dn;
        part[3 * blockIdx.x + 1] = dd;
        part[3 * blockIdx.x + 2] = sy;
    }
}

// z2..z5 and every u from l, z1 (the shrink) and T = Psi l.  cst: [0] the mean of
// I over the surrounding pixels, [1] the number of region pixels (0: no shift).
// The first workgroup also stores E_t (the pre kernel completed).
__global__ void __launch_bounds__(256) inp_post_kernel(InpPtrs P, int64_t total, float eta, const double* part,
                                                       int npart, const double* cst, double* Et_base, int* counter) {
    __shared__ double red[8];
    __shared__ float s_shift;
    double sy = 0.0;
    for (int i = threadIdx.x; i < npart; i += blockDim.x) sy += part[3 * i + 2];
    sy = block_sum(sy, red);
    if (threadIdx.x == 0) {
        const double cnt = cst[1];
        s_shift = (P.ave && cnt > 0.0) ? (float)(cst[0] - sy / cnt) : 0.f;
        if (blockIdx.x == 0 && Et_base) {
            double dn = 0.0, dd = 0.0;
            for (int i = 0; i < npart; ++i) {
                dn += part[3 * i];
                dd += part[3 * i + 1];
            }
            const int t = *counter;
            Et_base[t] = dd > 0.0 ? sqrt(dn) / sqrt(dd) : 0.0;
            *counter = t + 1;
        }
    }
    __syncthreads();
    const float shift = s_shift;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
        const float l = P.l[e], w = P.om[e], wb = 1.f - w;
        P.u[0][e] += l - P.z[0][e];
        const float p = P.T[e];
        const float y2 = p + P.u[1][e];
        const float z2 = y2 > eta ? y2 - eta : (y2 < -eta ? y2 + eta : 0.f);
        P.z[1][e] = z2;
        P.u[1][e] += p - z2;
        const float z3 = w * P.I[e];
        P.z[2][e] = z3;
        P.u[2][e] += w * l - z3;
        const float y4 = l + P.u[3][e];
        const float z4 = fminf(fmaxf(y4, 0.f), 1.f);
        P.z[3][e] = z4;
        P.u[3][e] += l - z4;
        if (P.ave) {
            const float y5 = wb * l + P.u[4][e];
            const float z5 = w == 0.f ? y5 + shift : y5;
            P.z[4][e] = z5;
            P.u[4][e] += wb * l - z5;
        }
    }
}

// Per-workgroup partials of the constants: [3 b] sum of I over the surrounding
// pixels (border != 0), [3 b + 1] their number, [3 b + 2] the number of region
// pixels (om == 0).
__global__ void __launch_bounds__(256) inp_const_kernel(int64_t total, const float* I, const float* om,
                                                        const float* border, double* part) {
    __shared__ double red[8];
    double sb = 0.0, nb = 0.0, nr = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
        if (border && border[e] != 0.f) {
            sb += (double)I[e];
            nb += 1.0;
        }
        if (om[e] == 0.f) nr += 1.0;
    }
    sb = block_sum(sb, red);
    nb = block_sum(nb, red);
    nr = block_sum(nr, red);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = sb;
        part[3 * blockIdx.x + 1] = nb;
        part[3 * blockIdx.x + 2] = nr;
    }
}

// cst[0] = mean of I over the surrounding pixels, cst[1] = number of region
// pixels; cst[1] = 0 when either set is empty or there is no border mask.  The
// partials are added in a fixed order (one workgroup).
__global__ void __launch_bounds__(256) inp_const_finish_kernel(const double* part, int npart, int has_border,
                                                               double* cst) {
    __shared__ double red[8];
    double sb = 0.0, nb = 0.0, nr = 0.0;
    for (int i = threadIdx.x; i < npart; i += blockDim.x) {
        sb += part[3 * i];
        nb += part[3 * i + 1];
        nr += part[3 * i + 2];
    }
    sb = block_sum(sb, red);
    nb = block_sum(nb, red);
    nr = block_sum(nr, red);
    if (threadIdx.x == 0) {
        const bool ok = has_border && nb > 0.0 && nr > 0.0;
        cst[0] = ok ? sb / nb : 0.0;
        cst[1] = ok ? nr : 0.0;
    }
}

// Start: l = u = 1, z1 = z4 = 1, z3 = Omega 1, z5 = Omega_bar 1, z2 = 1 (the
// caller overwrites z2 with Psi 1).
__global__ void __launch_bounds__(256) inp_init_kernel(int64_t total, const float* om, float* state) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const float w = om[e];
        state[e] = 1.f;                  // l
        state[total + e] = 1.f;          // z1
        state[2 * total + e] = 1.f;      // z2
        state[3 * total + e] = w;        // z3
        state[4 * total + e] = 1.f;      // z4
        state[5 * total + e] = 1.f - w;  // z5
        for (int k = 6; k < 11; ++k) state[k * total + e] = 1.f;   // u1..u5
    }
}

}  // namespace cpa
