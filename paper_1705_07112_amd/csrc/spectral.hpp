// Spectral bound (Algorithm 1, the maximum-eigenvalue step) and the per-call
// scalar block: power iteration on the Gram with FP64 accumulation, the bound
// rule, and the FP64 Chebyshev coefficients (Sec. III-A,
// eq. chebychev_coeff_shifted) computed on the device from that bound.
//
// Power iteration, one launch per Gram-vector product, so every workgroup sees
// the previous product complete:
//   w_0 = v_0 (SplitMix64 start vector or the warm-start vector)
//   product t: v_t = w_{t-1} / ||w_{t-1}||, w_t = G v_t,
//              mu_t = v_t . w_t and ||w_t||^2 accumulated in FP64.
//   stop before product t when |mu_{t-1} - mu_{t-2}| <= tol mu_{t-1} (t >= 3) or
//   ||w_{t-1}|| == 0; later launches return at once.
// The finishing kernel forms ||r|| = sqrt(max(||w_T||^2 - mu_T^2, 0)) and
//   Lambda = min(mu_T + max(margin mu_T, ||r||), ||G||_F).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shrink_fn.hpp"

namespace cpa {

// Scalar block layout (doubles).  Every per-call quantity lives here so a whole
// shrink is enqueued without host round trips.
enum : int {
    SC_FRO2 = 0,      // ||G||_F^2
    SC_TRACE = 1,     // trace G = ||X||_F^2
    SC_LAMBDA = 2,
    SC_MU = 3,
    SC_RESID = 4,
    SC_ITERS = 5,
    SC_STOP = 6,      // product index after which iteration stopped (0: not yet)
    SC_VANISH = 7,    // 1 if a product vanished while ||G||_F > 0
    SC_A1 = 8,        // 2 / Lambda (0 if Lambda == 0)
    SC_A2 = 9,        // 4 / Lambda
    SC_ET_NUM = 10,   // ADMM: ||l_new - l_old||^2
    SC_ET_DEN = 11,   // ADMM: ||l_new||^2
    SC_COEF = 16      // K coefficients, then K norms, then power slots
};

struct ScalarLayout {
    int K, maxit;
    int coef() const { return SC_COEF; }
    int norms() const { return SC_COEF + K; }              // ||Y_k||^2, k = 0..K-1
    int pw_mu() const { return SC_COEF + 2 * K; }          // mu_t, t = 0..maxit
    int pw_w2() const { return SC_COEF + 2 * K + maxit + 1; }  // ||w_t||^2
    int total() const { return SC_COEF + 2 * K + 2 * (maxit + 1); }
};

__global__ void fill_f64_kernel(double* p, int n, double v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__device__ inline uint64_t splitmix64_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// w0 = start vector; ||w0||^2 into pw_w2[0].  warm != nullptr: copy it.
__global__ void power_init_kernel(int d, uint64_t seed, const double* warm, double* w0, double* scal, int pw_w2) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d; i += gridDim.x * blockDim.x) {
        double v;
        if (warm) {
            v = warm[i];
        } else {
            const uint64_t out = splitmix64_out(seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
            v = 2.0 * ((double)(out >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
        }
        w0[i] = v;
        acc += v * v;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0 && acc != 0.0) atomicAdd(scal + pw_w2, acc);
}

// One product w_t = G v_t (G symmetric d x d, row-major, FP32), one wave per row.
__global__ void __launch_bounds__(256) power_step_kernel(int d, const float* G, int64_t ldg, const double* wprev,
                                                         double* wnext, double* scal, int t, double tol,
                                                         int pw_mu, int pw_w2) {
    if (scal[SC_STOP] != 0.0) return;
    const double w2p = scal[pw_w2 + t - 1];
    if (t >= 3) {
        const double m1 = scal[pw_mu + t - 1], m2 = scal[pw_mu + t - 2];
        if (fabs(m1 - m2) <= tol * m1) {
            // all workgroups read the same completed slots and return; one records it
            if (blockIdx.x == 0 && threadIdx.x == 0) scal[SC_STOP] = t - 1;
            return;
        }
    }
    if (!(w2p > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[SC_STOP] = t - 1;
            scal[SC_VANISH] = 1.0;
        }
        return;
    }
    const double inv = 1.0 / sqrt(w2p);
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int nw = gridDim.x * (blockDim.x >> 6);
    double mu_part = 0.0, w2_part = 0.0;
    for (int i = gw; i < d; i += nw) {
        const float* row = G + (int64_t)i * ldg;
        double s = 0.0;
        for (int j = lane; j < d; j += 64) s += (double)row[j] * (wprev[j] * inv);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) {
            wnext[i] = s;
            mu_part += (wprev[i] * inv) * s;
            w2_part += s * s;
        }
    }
    if (lane == 0) {
        if (mu_part != 0.0) atomicAdd(scal + pw_mu + t, mu_part);
        if (w2_part != 0.0) atomicAdd(scal + pw_w2 + t, w2_part);
    }
}

// Bound rule + coefficients + recurrence scalars.  Single workgroup.
//   mode 0: power iteration result (products 1..maxit in the slots)
//   mode 1: Lambda given
//   mode 2: Lambda = ||G||_F
// For mode 0 the warm-start buffer receives v_T (the unit vector of the last product).
__global__ void finish_bound_kernel(int mode, double Lambda_given, int d, int maxit, double margin,
                                    const double* wbuf0, const double* wbuf1, double* warm_out, double* scal,
                                    ShrinkParams sp, int K, int pw_mu, int pw_w2) {
    __shared__ double sLambda;
    __shared__ int sT;
    if (threadIdx.x == 0) {
        const double fro = sqrt(scal[SC_FRO2] > 0.0 ? scal[SC_FRO2] : 0.0);
        double Lam = 0.0;
        int T = 0;
        if (mode == 1) {
            Lam = Lambda_given;
        } else if (mode == 2) {
            Lam = fro;
        } else if (fro > 0.0) {
            T = (scal[SC_STOP] != 0.0) ? (int)scal[SC_STOP] : maxit;
            if (scal[SC_VANISH] != 0.0 || T < 1) {
                Lam = fro;
                T = 0;
            } else {
                const double mu = scal[pw_mu + T];
                const double w2 = scal[pw_w2 + T];
                const double r2 = w2 - mu * mu;
                const double r = sqrt(r2 > 0.0 ? r2 : 0.0);
                const double add = (margin * mu > r) ? margin * mu : r;
                Lam = mu + add;
                if (Lam > fro) Lam = fro;
                scal[SC_MU] = mu;
                scal[SC_RESID] = r;
            }
        }
        scal[SC_ITERS] = T;
        scal[SC_LAMBDA] = Lam;
        scal[SC_A1] = Lam > 0.0 ? 2.0 / Lam : 0.0;
        scal[SC_A2] = Lam > 0.0 ? 4.0 / Lam : 0.0;
        sLambda = Lam;
        sT = T;
    }
    __syncthreads();
    const double Lam = sLambda;
    for (int k = threadIdx.x; k < K; k += blockDim.x) scal[SC_COEF + k] = cheb_coeff(sp, Lam, K, k);
    if (mode == 0 && warm_out && sT >= 1) {
        // v_T = w_{T-1} / ||w_{T-1}||; w_{T-1} sits in buffer (T-1) % 2
        const double* src = ((sT - 1) & 1) ? wbuf1 : wbuf0;
        const double inv = 1.0 / sqrt(scal[pw_w2 + sT - 1]);
        for (int i = threadIdx.x; i < d; i += blockDim.x) warm_out[i] = src[i] * inv;
    }
}

// K == 1: Y = c_0/2 X.
__global__ void scale_copy_kernel(int m, int n, const float* X, int64_t ldx, float* Y, int64_t ldy,
                                  const double* scal) {
    const float c = (float)(0.5 * scal[SC_COEF]);
    const int64_t total = (int64_t)m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        Y[i * ldy + j] = c * X[i * ldx + j];
    }
}

}  // namespace cpa
