// Learned bound / order predictor: a 3 -> 64 -> 64 -> 2 perceptron with tanh
// hidden units (not in the paper; it replaces the power iteration of the
// maximum-eigenvalue step of Algorithm 1 and picks the order per matrix).
//
// Model buffer (float, kModelFloats entries, 16-byte aligned):
//   W1[64][3] | b1[64] | W2[64][64] | b2[64] | W3[2][64] | b3[2]   (out x in, row-major)
//   | mean[3] | inv_std[3] | 2 unused
// Input features f (per matrix): log ||X||_F, log ||Gram||_F^2, log(m n); the
// network sees x = (f - mean) * inv_std.  Outputs: y0 ~ log(lambda_max / ||Gram||_F),
// y1 ~ log K.
//
// Training: pinball loss per output, L = mean over samples and outputs of
// max(q_o r, (q_o - 1) r), r = t - y, minimised with Adam (Kingma and Ba).
// mlp_tile_kernel processes 64-sample tiles: the three 64 x 64 x 64 products of
// a tile (layer-2 forward, layer-2 input gradient, layer-2 weight gradient) run
// on FP32 MFMA, the rest on the vector ALU; every workgroup leaves one partial
// gradient, and mlp_reduce_kernel sums the partials in a fixed order (the
// result does not depend on scheduling) and applies the Adam update.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gemm_f32.hpp"

namespace cpa {

constexpr int kMlpH = 64;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = 192;
constexpr int kOffW2 = 256;
constexpr int kOffB2 = 4352;
constexpr int kOffW3 = 4416;
constexpr int kOffB3 = 4544;
constexpr int kMlpParams = 4546;
constexpr int kOffNorm = 4546;
constexpr int kModelFloats = 4554;
constexpr int kMlpThreads = 256;
constexpr int kMlpMaxWg = 256;     // gradient partial slots
constexpr int kMP = 65;            // LDS pitch of the 64 x 64 tiles

struct MlpArgs {
    const float* feat;   // n x 3 raw features
    const float* targ;   // n x 2 targets (gradient mode)
    const float* model;
    float* y;            // n x 2 outputs (nullable in gradient mode)
    float* part;         // gridDim.x x kMlpParams gradient partials
    double* lpart;       // gridDim.x loss partials
    int64_t s0, count;   // samples [s0, s0 + count)
    float q0, q1;        // quantiles of the two outputs
    float dscale;        // 1 / (2 count): derivative of the mean
};

// acc[jb] += A(rows 16 w .. +15, k) * B(k, 16 jb .. +15) over k = 0..63, with
// A(i, k) = A[i * ai + k * ak] (A already offset to the wave's first row) and
// B(k, j) = B[k * bk + j * bj].  Output position of acc[jb][r]:
// row 4 (lane / 16) + r, column 16 jb + lane % 16.
__device__ inline void mlp_mm16x64(const float* A, int ai, int ak, const float* B, int bk, int bj, f32x4 (&acc)[4]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
#pragma unroll 4
    for (int k0 = 0; k0 < kMlpH; k0 += 4) {
        const int k = k0 + g;
        const float av = A[c * ai + k * ak];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const float bv = B[k * bk + (16 * jb + c) * bj];
            acc[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[jb], 0, 0, 0);
        }
    }
}

template <bool GRAD>
__global__ void __launch_bounds__(kMlpThreads) mlp_tile_kernel(MlpArgs a) {
    __shared__ float W2s[kMlpH * kMP];
    __shared__ float A1[kMlpH * kMP];
    __shared__ float A2[kMlpH * kMP];   // layer-2 activations, later dZ1
    __shared__ float DZ[kMlpH * kMP];   // dL/dz2
    __shared__ float W1s[192], b1s[64], b2s[64], W3s[128], b3s[2], nrm[6];
    __shared__ float Fs[kMlpH][4];
    __shared__ float DY[kMlpH][2];
    __shared__ double red[4];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const float* M = a.model;
    for (int p = tid; p < kMlpH * kMlpH; p += kMlpThreads) W2s[(p >> 6) * kMP + (p & 63)] = M[kOffW2 + p];
    if (tid < 192) W1s[tid] = M[kOffW1 + tid];
    if (tid < 64) {
        b1s[tid] = M[kOffB1 + tid];
        b2s[tid] = M[kOffB2 + tid];
    }
    if (tid < 128) W3s[tid] = M[kOffW3 + tid];
    if (tid < 2) b3s[tid] = M[kOffB3 + tid];
    if (tid < 6) nrm[tid] = M[kOffNorm + tid];

    f32x4 gw2[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) gw2[jb] = f32x4{0.f, 0.f, 0.f, 0.f};
    float gw3 = 0.f, gb3 = 0.f, gb2 = 0.f, gw1 = 0.f, gb1 = 0.f;
    double loss = 0.0;
    __syncthreads();

    const int64_t ntiles = (a.count + kMlpH - 1) / kMlpH;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t base = a.s0 + t * kMlpH;
        const int nv = (int)((a.count - t * kMlpH) < kMlpH ? (a.count - t * kMlpH) : kMlpH);
        // ---- normalised features of the tile (rows past the end are zero)
        if (tid < kMlpH * 3) {
            const int S = tid / 3, i = tid % 3;
            Fs[S][i] = S < nv ? (a.feat[(base + S) * 3 + i] - nrm[i]) * nrm[3 + i] : 0.f;
        }
        __syncthreads();
        // ---- layer 1: A1[S][h] = tanh(b1[h] + W1[h] . x_S)
        {
            const int S = tid >> 2, h0 = (tid & 3) * 16;
            const float x0 = Fs[S][0], x1 = Fs[S][1], x2 = Fs[S][2];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int h = h0 + q;
                A1[S * kMP + h] = tanhf(b1s[h] + W1s[3 * h] * x0 + W1s[3 * h + 1] * x1 + W1s[3 * h + 2] * x2);
            }
        }
        __syncthreads();
        // ---- layer 2: Z2 = A1 W2^T (MFMA), A2 = tanh(Z2 + b2); this wave's rows S = 16 wave ..
        f32x4 a2r[4];
        {
            f32x4 acc[4];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) acc[jb] = f32x4{0.f, 0.f, 0.f, 0.f};
            mlp_mm16x64(A1 + 16 * wave * kMP, kMP, 1, W2s, 1, kMP, acc);
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const int h = 16 * jb + c;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float v = tanhf(acc[jb][r] + b2s[h]);
                    a2r[jb][r] = v;
                    A2[(16 * wave + 4 * g + r) * kMP + h] = v;
                }
            }
        }
        __syncthreads();
        // ---- output layer, loss and dL/dy
        if (tid < 128) {
            const int S = tid >> 1, o = tid & 1;
            float y = b3s[o];
            for (int h = 0; h < kMlpH; ++h) y += W3s[o * kMlpH + h] * A2[S * kMP + h];
            if (!GRAD) {
                if (S < nv) a.y[(base + S) * 2 + o] = y;
            } else {
                float d = 0.f;
                if (S < nv) {
                    if (a.y) a.y[(base + S) * 2 + o] = y;
                    const float q = o == 0 ? a.q0 : a.q1;
                    const float r = a.targ[(base + S) * 2 + o] - y;
                    loss += (double)(r >= 0.f ? q * r : (q - 1.f) * r);
                    d = (r >= 0.f ? -q : 1.f - q) * a.dscale;
                }
                DY[S][o] = d;
            }
        }
        if (!GRAD) {
            __syncthreads();
            continue;
        }
        __syncthreads();
        // ---- dZ2 = (dY W3) * (1 - A2^2) at this thread's MFMA positions
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const int h = 16 * jb + c;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int S = 16 * wave + 4 * g + r;
                const float v = a2r[jb][r];
                DZ[S * kMP + h] = (DY[S][0] * W3s[h] + DY[S][1] * W3s[kMlpH + h]) * (1.f - v * v);
            }
        }
        __syncthreads();
        // ---- small reductions over the tile's samples
        if (tid < 128) {
            const int o = tid >> 6, h = tid & 63;
            float s = 0.f;
            for (int S = 0; S < kMlpH; ++S) s += DY[S][o] * A2[S * kMP + h];
            gw3 += s;
        } else if (tid < 130) {
            const int o = tid - 128;
            float s = 0.f;
            for (int S = 0; S < kMlpH; ++S) s += DY[S][o];
            gb3 += s;
        } else if (tid >= 192) {
            const int h = tid - 192;
            float s = 0.f;
            for (int S = 0; S < kMlpH; ++S) s += DZ[S * kMP + h];
            gb2 += s;
        }
        // ---- gW2 += dZ2^T A1 (rows h = 16 wave ..), dA1 = dZ2 W2 (rows S = 16 wave ..)
        mlp_mm16x64(DZ + 16 * wave, 1, kMP, A1, kMP, 1, gw2);
        f32x4 da1[4];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) da1[jb] = f32x4{0.f, 0.f, 0.f, 0.f};
        mlp_mm16x64(DZ + 16 * wave * kMP, kMP, 1, W2s, kMP, 1, da1);
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const int j = 16 * jb + c;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float v = A1[(16 * wave + 4 * g + r) * kMP + j];
                da1[jb][r] *= 1.f - v * v;
            }
        }
        __syncthreads();   // A2 is free from here on
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) A2[(16 * wave + 4 * g + r) * kMP + 16 * jb + c] = da1[jb][r];
        __syncthreads();
        if (tid < 192) {
            const int h = tid / 3, i = tid % 3;
            float s = 0.f;
            for (int S = 0; S < kMlpH; ++S) s += A2[S * kMP + h] * Fs[S][i];
            gw1 += s;
        } else {
            const int h = tid - 192;
            float s = 0.f;
            for (int S = 0; S < kMlpH; ++S) s += A2[S * kMP + h];
            gb1 += s;
        }
        __syncthreads();
    }
    if (!GRAD) return;

    // ---- this workgroup's partial gradient and loss
    float* P = a.part + (int64_t)blockIdx.x * kMlpParams;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) P[kOffW2 + (16 * wave + 4 * g + r) * kMlpH + 16 * jb + c] = gw2[jb][r];
    if (tid < 128) P[kOffW3 + tid] = gw3;
    else if (tid < 130) P[kOffB3 + tid - 128] = gb3;
    if (tid >= 192) {
        P[kOffB2 + tid - 192] = gb2;
        P[kOffB1 + tid - 192] = gb1;
    } else {
        P[kOffW1 + tid] = gw1;   // tid = 3 h + i
    }
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
    if (lane == 0) red[wave] = loss;
    __syncthreads();
    if (tid == 0) a.lpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

struct AdamArgs {
    const float* part;
    int nwg;
    const double* lpart;
    float* model;        // parameters updated in place (adam != 0)
    float* m;            // first moments
    float* v;            // second moments
    float lr, beta1, beta2, eps;
    double bc1, bc2;     // 1 - beta^t
    float* grad_out;     // nullable: the summed gradient
    double* loss_dst;    // nullable: *loss_dst += loss_mul * sum(lpart)
    double loss_mul;
    int adam;
};

// One thread per parameter: g = sum of the partials in workgroup order (FP64),
// then the Adam step with bias correction.
__global__ void __launch_bounds__(256) mlp_reduce_kernel(AdamArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.loss_dst) {
        double s = 0.0;
        for (int w = 0; w < a.nwg; ++w) s += a.lpart[w];
        *a.loss_dst += a.loss_mul * s;
    }
    if (p >= kMlpParams) return;
    double gs = 0.0;
    for (int w = 0; w < a.nwg; ++w) gs += (double)a.part[(int64_t)w * kMlpParams + p];
    const float gr = (float)gs;
    if (a.grad_out) a.grad_out[p] = gr;
    if (!a.adam) return;
    const float m = a.beta1 * a.m[p] + (1.f - a.beta1) * gr;
    const float v = a.beta2 * a.v[p] + (1.f - a.beta2) * gr * gr;
    a.m[p] = m;
    a.v[p] = v;
    const float mh = (float)(m / a.bc1);
    const float vh = (float)(v / a.bc2);
    a.model[p] -= a.lr * mh / (sqrtf(vh) + a.eps);
}

// Inference for one matrix inside a 256-thread workgroup: every thread calls it
// with the same raw features; y receives the two outputs (all threads).  `h`
// is 128 floats of LDS scratch, `yb` two floats of LDS.
__device__ inline void mlp_infer_wg(const float* __restrict__ M, float f0, float f1, float f2, float* h, float* yb,
                                    float& y0, float& y1) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float x0 = (f0 - M[kOffNorm]) * M[kOffNorm + 3];
    const float x1 = (f1 - M[kOffNorm + 1]) * M[kOffNorm + 4];
    const float x2 = (f2 - M[kOffNorm + 2]) * M[kOffNorm + 5];
    if (tid < kMlpH)
        h[tid] = tanhf(M[kOffB1 + tid] + M[kOffW1 + 3 * tid] * x0 + M[kOffW1 + 3 * tid + 1] * x1 +
                       M[kOffW1 + 3 * tid + 2] * x2);
    __syncthreads();
    {
        // unit u = 16 wave + lane % 16; lane / 16 selects 16 of the 64 inputs
        const int u = 16 * wave + (lane & 15), q = lane >> 4;
        const f32x4* row = reinterpret_cast<const f32x4*>(M + kOffW2 + u * kMlpH + 16 * q);
        float s = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f32x4 w = row[t];
            s += w[0] * h[16 * q + 4 * t] + w[1] * h[16 * q + 4 * t + 1] + w[2] * h[16 * q + 4 * t + 2] +
                 w[3] * h[16 * q + 4 * t + 3];
        }
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        if (q == 0) h[kMlpH + u] = tanhf(s + M[kOffB2 + u]);
    }
    __syncthreads();
    if (wave == 0) {
        float p0 = M[kOffW3 + lane] * h[kMlpH + lane];
        float p1 = M[kOffW3 + kMlpH + lane] * h[kMlpH + lane];
        for (int off = 32; off > 0; off >>= 1) {
            p0 += __shfl_xor(p0, off, 64);
            p1 += __shfl_xor(p1, off, 64);
        }
        if (lane == 0) {
            yb[0] = p0 + M[kOffB3];
            yb[1] = p1 + M[kOffB3 + 1];
        }
    }
    __syncthreads();
    y0 = yb[0];
    y1 = yb[1];
}

}  // namespace cpa
