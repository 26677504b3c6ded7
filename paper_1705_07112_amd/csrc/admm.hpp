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

// Returns x = l + u1, the element of the shrink input.
__device__ inline float admm_pre_elem(const AdmmPtrs& P, int64_t e, double& dn, double& dd) {
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
    const float x = l + P.u1[e];
    P.x[e] = x;
    return x;
}

// admm_pre_elem on four consecutive elements e .. e + 3 (16-byte accesses; the
// partial sums take them in order).
__device__ inline f32x4 admm_pre_elem4(const AdmmPtrs& P, int64_t e, double& dn, double& dd) {
    const f32x4 Ie = *reinterpret_cast<const f32x4*>(P.I + e);
    const f32x4 u3 = *reinterpret_cast<const f32x4*>(P.u3 + e);
    const f32x4 z1 = *reinterpret_cast<const f32x4*>(P.z1 + e);
    const f32x4 u1 = *reinterpret_cast<const f32x4*>(P.u1 + e);
    const f32x4 z2 = *reinterpret_cast<const f32x4*>(P.z2 + e);
    const f32x4 u2 = *reinterpret_cast<const f32x4*>(P.u2 + e);
    const f32x4 lo = *reinterpret_cast<const f32x4*>(P.l + e);
    f32x4 l, s, x;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float a = (z1[r] - u1[r]) + (Ie[r] - u3[r]);
        const float b = (z2[r] - u2[r]) + (Ie[r] - u3[r]);
        l[r] = (2.f * a - b) * (1.f / 3.f);
        s[r] = (2.f * b - a) * (1.f / 3.f);
        const float dl = l[r] - lo[r];
        dn += (double)dl * dl;
        dd += (double)l[r] * l[r];
        x[r] = l[r] + u1[r];
    }
    *reinterpret_cast<f32x4*>(P.l + e) = l;
    *reinterpret_cast<f32x4*>(P.s + e) = s;
    *reinterpret_cast<f32x4*>(P.x + e) = x;
    return x;
}

// One element of the post-step: z2 = soft(s + u2); u1 += l - z1; u2 += s - z2;
// u3 += l + s - I.
__device__ inline void admm_post_vals(float l, float s, float z1, float Ie, float t2, float& z2, float& u1, float& u2,
                                      float& u3) {
    const float v = s + u2;
    const float av = fabsf(v) - t2;
    z2 = av > 0.f ? copysignf(av, v) : 0.f;
    u1 = u1 + l - z1;
    u2 = u2 + s - z2;
    u3 = u3 + l + s - Ie;
}

// z1 already holds the shrink of x; the post-step on every element (vec: every
// array 16-byte aligned, checked by the host: four elements per thread and step,
// 16-byte loads and stores).  The first workgroup also stores E_t (the pre-step
// completed).  E_t goes to Et_base[*counter] and the counter advances, so the same
// launch (or a replayed graph of it) fills consecutive entries.
__global__ void __launch_bounds__(256) admm_post_kernel(AdmmPtrs P, int64_t total, float t2, const double* part,
                                                        int npart, double* Et_base, int* counter, int vec) {
    __shared__ double red[8];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t head = 0;
    if (vec) {
        const int64_t nq = total / 4;
        for (int64_t q = tid; q < nq; q += stride) {
            const int64_t e = 4 * q;
            const f32x4 l = *reinterpret_cast<const f32x4*>(P.l + e);
            const f32x4 s = *reinterpret_cast<const f32x4*>(P.s + e);
            const f32x4 z1 = *reinterpret_cast<const f32x4*>(P.z1 + e);
            const f32x4 Ie = *reinterpret_cast<const f32x4*>(P.I + e);
            f32x4 u1 = *reinterpret_cast<const f32x4*>(P.u1 + e);
            f32x4 u2 = *reinterpret_cast<const f32x4*>(P.u2 + e);
            f32x4 u3 = *reinterpret_cast<const f32x4*>(P.u3 + e);
            f32x4 z2;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float a = 0.f, b = u1[r], c = u2[r], dd = u3[r];
                admm_post_vals(l[r], s[r], z1[r], Ie[r], t2, a, b, c, dd);
                z2[r] = a;
                u1[r] = b;
                u2[r] = c;
                u3[r] = dd;
            }
            *reinterpret_cast<f32x4*>(P.z2 + e) = z2;
            *reinterpret_cast<f32x4*>(P.u1 + e) = u1;
            *reinterpret_cast<f32x4*>(P.u2 + e) = u2;
            *reinterpret_cast<f32x4*>(P.u3 + e) = u3;
        }
        head = 4 * nq;
    }
    for (int64_t e = head + tid; e < total; e += stride) {
        float z2, u1 = P.u1[e], u2 = P.u2[e], u3 = P.u3[e];
        admm_post_vals(P.l[e], P.s[e], P.z1[e], P.I[e], t2, z2, u1, u2, u3);
        P.z2[e] = z2;
        P.u1[e] = u1;
        P.u2[e] = u2;
        P.u3[e] = u3;
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

// The work before a dense shrink in one launch.  Workgroups 0 .. ntile_wg - 1
// take 32 x 32 tiles of the m x n input (grid-stride; small tiles keep many
// waves in flight, the kernel being bound by memory latency): with admm set they
// run the ADMM pre-step on them (admm_pre_elem: l, s, x = l + u1 and the E_t
// partials, one pair per workgroup in part) and the tile's shrink input is that
// x, else it is read from X.  With xt set, each tile is also stored transposed,
// Xt[j][i] = X[i][j], the rows i from m to ldt (the contraction padded to a
// multiple of 64) as zeros: the tiles then cover ldt rows.  Workgroup ntile_wg
// clears the scalar block and, with d > 0, writes the power iteration's start
// vector (power_init_body).  256 threads.
struct PrepArgs {
    int m, n;
    const float* X;
    int64_t ldx;
    AdmmPtrs P;
    int admm;
    int vec;   // admm arrays 16-byte aligned and n % 4 == 0: four elements per access
    double* part;
    float* xt;
    int64_t ldt;
    double* scal;
    int nscal;
    int d;
    uint64_t seed;
    const double* warm;
    double* w0;
    int pw_w2;
    int ntile_wg;
};

constexpr int kPrepTile = 32;

__global__ void __launch_bounds__(256) prep_kernel(PrepArgs a) {
    constexpr int T = kPrepTile, RPW = 256 / T;   // rows per pass
    __shared__ float blk[T][T + 1];
    __shared__ double red[16];
    if ((int)blockIdx.x == a.ntile_wg) {
        for (int i = threadIdx.x; i < a.nscal; i += blockDim.x) a.scal[i] = 0.0;
        if (a.d > 0) {
            __syncthreads();   // the cleared block before the start vector's norm is stored in it
            power_init_body(a.d, a.seed, a.warm, a.w0, a.scal, a.pw_w2, red);
        }
        return;
    }
    const int tx = threadIdx.x % T, ty = threadIdx.x / T;
    const int rows = a.xt ? (int)(a.ldt / T) : (a.m + T - 1) / T;
    const int cols = (a.n + T - 1) / T;
    double dn = 0.0, dd = 0.0;
    for (int t = blockIdx.x; t < rows * cols; t += a.ntile_wg) {
        const int i0 = (t / cols) * T, j0 = (t % cols) * T;
        if (a.admm && a.vec) {
            // the tile in one pass: 32 rows x 8 groups of four columns
            const int r = threadIdx.x / (T / 4), c4 = (threadIdx.x % (T / 4)) * 4;
            const int i = i0 + r, j = j0 + c4;
            f32x4 v = (f32x4){0.f, 0.f, 0.f, 0.f};
            if (i < a.m && j < a.n) v = admm_pre_elem4(a.P, (int64_t)i * a.n + j, dn, dd);
#pragma unroll
            for (int e = 0; e < 4; ++e) blk[r][c4 + e] = v[e];
        } else {
#pragma unroll
            for (int q = 0; q < T / RPW; ++q) {
                const int i = i0 + ty + RPW * q, j = j0 + tx;
                float v = 0.f;
                if (i < a.m && j < a.n) {
                    if (a.admm)
                        v = admm_pre_elem(a.P, (int64_t)i * a.n + j, dn, dd);
                    else
                        v = a.X[(int64_t)i * a.ldx + j];
                }
                blk[ty + RPW * q][tx] = v;
            }
        }
        if (!a.xt) continue;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < T / RPW; ++q) {
            const int j = j0 + ty + RPW * q, i = i0 + tx;
            if (j < a.n) a.xt[(int64_t)j * a.ldt + i] = blk[tx][ty + RPW * q];
        }
        __syncthreads();   // the block is reused by the next tile
    }
    if (a.admm) {
        dn = block_sum(dn, red);
        dd = block_sum(dd, red);
        if (threadIdx.x == 0) {
            a.part[2 * blockIdx.x] = dn;
            a.part[2 * blockIdx.x + 1] = dd;
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
