// FP64 shrinkage (the dense path with FP64 inputs, outputs and arithmetic):
// the Gram, Algorithm 1's recurrence distributed over X (Y_{k+1} = 2 Y_k Ghat -
// Y_{k-1}, Ghat = (2/Lambda) G - I, out = c_0/2 X + sum c_k Y_k; eq.
// recurrence_our_method) and the Gram statistics of the Frobenius bound, all in
// double precision.  The bound and the coefficients come from the same FP64
// kernels as the FP32 path (power iteration on the FP64 Gram).
//
// gemm_f64_kernel: C = op(A) op(B) with 64 x 64 output tiles, K-steps of 32,
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64): eight waves, two per 32 x 32
// output (2 x 2 blocks of 16 x 16), each taking half of every K-step, their
// partial sums added through LDS at the end; operand tiles go through two LDS
// stages ([k][i] and [k][j], zero fill outside the matrix), the next tile's
// global reads in flight in registers while the current tile is multiplied.  op(A)[i][k] is A[k][i] when TA (the
// Gram X^T X reads X transposed), op(B)[k][j] is B[j][k] when TB (X X^T).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spectral.hpp"

namespace cpa {

constexpr int F64_BM = 64, F64_BN = 64, F64_BK = 32;
constexpr int F64_THREADS = 512;                            // 8 waves: 2 x 2 output blocks x K-split 2
constexpr int F64_LOADS = F64_BM * F64_BK / F64_THREADS;    // operand elements per thread and tile
constexpr int F64_PITCH = F64_BM + 1;
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Operand element r of thread tid for the K-tile at k0: (row or column index,
// k index) inside the tile, chosen so that consecutive threads read consecutive
// addresses of the operand.
template <bool KMAJOR>
__device__ inline void f64_tile_pos(int tid, int r, int& x, int& k) {
    const int e = tid + F64_THREADS * r;
    if (KMAJOR) {   // the operand's row index runs along k: consecutive x are adjacent
        x = e % F64_BM;
        k = e / F64_BM;
    } else {        // k is contiguous
        x = e / F64_BK;
        k = e % F64_BK;
    }
}

template <bool TA, bool TB>
__global__ void __launch_bounds__(F64_THREADS) gemm_f64_kernel(int M, int N, int Kd, const double* A, int64_t lda,
                                                               const double* B, int64_t ldb, double* C, int64_t ldc) {
    // two stages of [k][i] and [k][j] tiles; the epilogue reuses stage 0 for the
    // K-split sum
    __shared__ double lds[2][2][F64_BK][F64_PITCH];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wo = wave & 3, kh = wave >> 2;   // output block, half of each K-tile
    const int wr = wo >> 1, wc = wo & 1;       // the wave's 32 x 32 output
    const int i0 = blockIdx.y * F64_BM, j0 = blockIdx.x * F64_BN;
    f64x4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = (f64x4){0.0, 0.0, 0.0, 0.0};
    // the next K-tile is read into registers while the current one is multiplied,
    // then written to the other stage (last read one step earlier)
    double ra[F64_LOADS], rb[F64_LOADS];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < F64_LOADS; ++r) {
            int ii, jj, kk;
            f64_tile_pos<TA>(tid, r, ii, kk);
            const int gi = i0 + ii, gk = k0 + kk;
            ra[r] = (gi < M && gk < Kd) ? (TA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk]) : 0.0;
            f64_tile_pos<!TB>(tid, r, jj, kk);
            const int gj = j0 + jj, gk2 = k0 + kk;
            rb[r] = (gj < N && gk2 < Kd) ? (TB ? B[(int64_t)gj * ldb + gk2] : B[(int64_t)gk2 * ldb + gj]) : 0.0;
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int r = 0; r < F64_LOADS; ++r) {
            int ii, jj, kk;
            f64_tile_pos<TA>(tid, r, ii, kk);
            lds[st][0][kk][ii] = ra[r];
            f64_tile_pos<!TB>(tid, r, jj, kk);
            lds[st][1][kk][jj] = rb[r];
        }
    };
    fetch(0);
    stash(0);
    __syncthreads();
    int st = 0;
    for (int k0 = 0; k0 < Kd; k0 += F64_BK) {
        const bool more = k0 + F64_BK < Kd;
        if (more) fetch(k0 + F64_BK);
        // this wave's k sub-steps of 4: lane l supplies row (or column) l % 16 at k = l / 16
#pragma unroll
        for (int ks = 0; ks < F64_BK / 8; ++ks) {
            const int kk = kh * (F64_BK / 2) + 4 * ks + (lane >> 4);
            double a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) a[x] = lds[st][0][kk][wr * 32 + x * 16 + (lane & 15)];
#pragma unroll
            for (int y = 0; y < 2; ++y) b[y] = lds[st][1][kk][wc * 32 + y * 16 + (lane & 15)];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
        if (more) stash(st ^ 1);
        __syncthreads();
        st ^= 1;
    }
    // lane l holds rows l / 16 + 4 r and column l % 16 of each 16 x 16 block (the
    // FP64 instruction interleaves the rows; the FP32 one gives 4 (l / 16) + r).
    // The second K half adds its partial sums to the first's through LDS.
    double (*red)[F64_PITCH] = reinterpret_cast<double (*)[F64_PITCH]>(&lds[0][0][0][0]);
    if (kh == 1) {
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    red[wr * 32 + x * 16 + (lane >> 4) + 4 * r][wc * 32 + y * 16 + (lane & 15)] = acc[x][y][r];
    }
    __syncthreads();
    if (kh == 0) {
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int li = wr * 32 + x * 16 + (lane >> 4) + 4 * r;
                    const int lj = wc * 32 + y * 16 + (lane & 15);
                    const int i = i0 + li, j = j0 + lj;
                    if (i < M && j < N) C[(int64_t)i * ldc + j] = acc[x][y][r] + red[li][lj];
                }
    }
}

// One recurrence step on an m x n matrix, element (r, c) per thread:
//   step 0: Y_1 = a1 Z - X,               out = c_0/2 X + c_1 Y_1
//   step k: Y_{k+1} = a2 Z - 2 Y_k - Y_{k-1}, out += c_{k+1} Y_{k+1}
// Z = Y_k G (or G Y_k); Yk has pitch ldk (X at step 0), Yo holds Y_{k-1} and
// receives Y_{k+1} (pitch n, same element, same thread); out has pitch ldo.
__global__ void __launch_bounds__(256) cheb64_step_kernel(int m, int n, const double* Z, const double* Yk, int64_t ldk,
                                                          double* Yo, double* out, int64_t ldo, const double* scal,
                                                          int step) {
    const double a = step == 0 ? scal[SC_A1] : scal[SC_A2];
    const double ck = scal[SC_COEF + step + 1];
    const double c0h = 0.5 * scal[SC_COEF];
    const int64_t total = (int64_t)m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / n, c = e % n;
        const double yk = Yk[r * ldk + c];
        double y;
        if (step == 0) {
            y = a * Z[e] - yk;
            out[r * ldo + c] = c0h * yk + ck * y;
        } else {
            y = a * Z[e] - 2.0 * yk - Yo[e];
            out[r * ldo + c] += ck * y;
        }
        Yo[e] = y;
    }
}

// dst (pitch n) = X (pitch ldx).
__global__ void __launch_bounds__(256) copy64_kernel(int m, int n, const double* X, int64_t ldx, double* dst) {
    const int64_t total = (int64_t)m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = X[(e / n) * ldx + e % n];
}

// out = c_0/2 X (K = 1).
__global__ void __launch_bounds__(256) scale64_kernel(int m, int n, const double* X, int64_t ldx, double* out,
                                                      int64_t ldo, const double* scal) {
    const double c0h = 0.5 * scal[SC_COEF];
    const int64_t total = (int64_t)m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / n, c = e % n;
        out[r * ldo + c] = c0h * X[r * ldx + c];
    }
}

// Per-workgroup partials of ||G||_F^2 and tr G (d x d, pitch d), 2 per workgroup,
// in the layout the bound kernel reads.
__global__ void __launch_bounds__(256) gram64_stats_kernel(int d, const double* G, double* gpart) {
    __shared__ double red[8];
    double f2 = 0.0, tr = 0.0;
    const int64_t total = (int64_t)d * d;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const double g = G[e];
        f2 += g * g;
        if (e / d == e % d) tr += g;
    }
    f2 = block_sum(f2, red);
    tr = block_sum(tr, red);
    if (threadIdx.x == 0) {
        gpart[2 * blockIdx.x] = f2;
        gpart[2 * blockIdx.x + 1] = tr;
    }
}

}  // namespace cpa
