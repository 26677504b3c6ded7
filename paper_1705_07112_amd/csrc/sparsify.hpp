// The sparsifying transform and component truncation of Algorithm 1 (Sec. III-B):
//   Phi = T G T^T with T the 8 x 8 block DCT (kron(I, D_8), eq. sing_shrink_exact_sparse)
//         or the identity,
//   underline Phi_ij = Phi_ij if |Phi_ij| >= eps (eq. threshold_components), with
//         eps = the k-th largest |Phi_ij| (the threshold rule of eq. recommendation_epsilon),
//   hat H(underline Phi) by the three-term recurrence with underline Phi in CSR
//         (spmm_cheb_kernel, one sparse product per step),
//   M = T^T hat H T, then hat G = X M (or M X).
//
// Kernels:
//   bt_forward_kernel   one workgroup per pair of 8 x 8 tiles (I <= J):
//                       P = D G_IJ D^T in FP64 from the FP32 Gram, written to tile
//                       (I, J) and transposed to (J, I); diagonal tiles are
//                       symmetrised ((P + P^T)/2).  Phi is therefore exactly
//                       symmetric, so an entry and its mirror always fall on the
//                       same side of eps.  D is passed in (the DCT table, or I).
//   sel_hist_kernel /   radix selection of the k-th largest |Phi| on the FP32 bit
//   sel_pick_kernel     patterns of |Phi| (monotone as unsigned integers): three
//                       passes of 11, 11 and 9 bits; exact integer histograms, so
//                       the threshold is the same on every run.
//   trunc_count_kernel, one wave per row: counts the kept entries; after an
//   trunc_fill_kernel   exclusive scan, writes (column, value) in column order
//                       (ballot + prefix popcount) and zeroes the dropped entries of
//                       Phi in place (the dense underline Phi feeds the power
//                       iteration).
//   bt_inverse_kernel   M_IJ = D^T H_IJ D for every tile, FP64 inside.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpa {

// 8 x 8 transform table D[a][i] (rows are the basis functions), by value.
struct Dct8 {
    double d[64];
};

// Digits of the key: bits 30..20, 19..9, 8..0 (bit 31, the sign, is cleared).
constexpr int kSelBins = 2048;
__device__ inline int sel_bits(int pass) { return pass == 2 ? 9 : 11; }
__device__ inline int sel_shift(int pass) { return pass == 0 ? 20 : (pass == 1 ? 9 : 0); }

// Selection state: [0] prefix bits found so far, [1] their mask, [2] k remaining
// among the entries that match the prefix.
struct SelState {
    uint32_t prefix, mask, krem, pad;
};

__device__ inline uint32_t abs_key(float x) { return __float_as_uint(x) & 0x7fffffffu; }

__global__ void __launch_bounds__(64) bt_forward_kernel(int d, const float* G, int64_t ldg, float* Phi, int64_t ldp,
                                                        Dct8 D) {
    __shared__ double g[8][9];
    __shared__ double t[8][9];
    // tile pair index -> (I, J), I <= J, row-major over the upper triangle
    const int nt = d / 8;
    int p = blockIdx.x, I = 0;
    while (p >= nt - I) {
        p -= nt - I;
        ++I;
    }
    const int J = I + p;
    const int a = threadIdx.x >> 3, b = threadIdx.x & 7;
    g[a][b] = (double)G[(int64_t)(8 * I + a) * ldg + 8 * J + b];
    __syncthreads();
    // t = G_IJ D^T: t[a][b] = sum_j g[a][j] D[b][j]
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += g[a][j] * D.d[8 * b + j];
    t[a][b] = s;
    __syncthreads();
    // P = D t: P[a][b] = sum_i D[a][i] t[i][b]
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) v += D.d[8 * a + i] * t[i][b];
    if (I == J) {
        __syncthreads();
        g[a][b] = v;   // reuse: the tile's P
        __syncthreads();
        const double sym = 0.5 * (g[a][b] + g[b][a]);
        Phi[(int64_t)(8 * I + a) * ldp + 8 * J + b] = (float)sym;
    } else {
        const float f = (float)v;
        Phi[(int64_t)(8 * I + a) * ldp + 8 * J + b] = f;
        Phi[(int64_t)(8 * J + b) * ldp + 8 * I + a] = f;
    }
}

__global__ void __launch_bounds__(64) bt_inverse_kernel(int d, const float* H, int64_t ldh, float* M, int64_t ldm,
                                                        Dct8 D) {
    __shared__ double h[8][9];
    __shared__ double t[8][9];
    const int nt = d / 8;
    const int I = blockIdx.x / nt, J = blockIdx.x % nt;
    const int a = threadIdx.x >> 3, b = threadIdx.x & 7;
    h[a][b] = (double)H[(int64_t)(8 * I + a) * ldh + 8 * J + b];
    __syncthreads();
    // t = H_IJ D: t[a][b] = sum_j h[a][j] D[j][b]
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += h[a][j] * D.d[8 * j + b];
    t[a][b] = s;
    __syncthreads();
    // M = D^T t: M[a][b] = sum_i D[i][a] t[i][b]
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) v += D.d[8 * i + a] * t[i][b];
    M[(int64_t)(8 * I + a) * ldm + 8 * J + b] = (float)v;
}

// Histogram of the next digit of |Phi| over the entries matching the prefix.
__global__ void __launch_bounds__(256) sel_hist_kernel(int d, const float* Phi, int64_t ldp, int pass,
                                                       const SelState* st, unsigned* hist) {
    __shared__ unsigned lh[kSelBins];
    for (int i = threadIdx.x; i < kSelBins; i += 256) lh[i] = 0u;
    __syncthreads();
    const uint32_t prefix = st->prefix, mask = st->mask;
    const int shift = sel_shift(pass), nb = (1 << sel_bits(pass)) - 1;
    const int64_t total = (int64_t)d * d;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int r = (int)(e / d), c = (int)(e % d);
        const uint32_t key = abs_key(Phi[(int64_t)r * ldp + c]);
        if ((key & mask) == prefix) atomicAdd(&lh[(key >> shift) & nb], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += 256)
        if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

// The bin holding the krem-th largest key (counting from the top), appended to
// the prefix; clears the histogram for the next pass.  One workgroup.
__global__ void __launch_bounds__(256) sel_pick_kernel(int pass, SelState* st, unsigned* hist) {
    __shared__ unsigned h[kSelBins];
    __shared__ uint32_t s_bin, s_above;
    for (int i = threadIdx.x; i < kSelBins; i += 256) {
        h[i] = hist[i];
        hist[i] = 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nbin = 1 << sel_bits(pass);
        uint32_t above = 0, bin = 0;
        for (int i = nbin - 1; i >= 0; --i) {
            if (above + h[i] >= st->krem) {
                bin = (uint32_t)i;
                break;
            }
            above += h[i];
        }
        s_bin = bin;
        s_above = above;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int shift = sel_shift(pass);
        st->prefix |= s_bin << shift;
        st->mask |= (uint32_t)((1 << sel_bits(pass)) - 1) << shift;
        st->krem -= s_above;
    }
}

// Kept entries per row (|Phi_ij| >= eps, eps = the selected key).
__global__ void __launch_bounds__(256) trunc_count_kernel(int d, const float* Phi, int64_t ldp, const SelState* st,
                                                          int32_t* cnt) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (r >= d) return;
    const uint32_t eps = st->prefix;
    int c = 0;
    for (int j = lane; j < d; j += 64) c += abs_key(Phi[(int64_t)r * ldp + j]) >= eps ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) cnt[r] = c;
}

// CSR of the kept entries (columns ascending) and the dense truncated matrix in place.
__global__ void __launch_bounds__(256) trunc_fill_kernel(int d, float* Phi, int64_t ldp, const SelState* st,
                                                         const int32_t* rowptr, int32_t* colidx, float* val) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (r >= d) return;
    const uint32_t eps = st->prefix;
    int32_t pos = rowptr[r];
    for (int j0 = 0; j0 < d; j0 += 64) {
        const int j = j0 + lane;
        float v = 0.f;
        bool keep = false;
        if (j < d) {
            v = Phi[(int64_t)r * ldp + j];
            keep = abs_key(v) >= eps;
        }
        const uint64_t bal = __ballot(keep);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (keep) {
            colidx[pos + before] = j;
            val[pos + before] = v;
        } else if (j < d) {
            Phi[(int64_t)r * ldp + j] = 0.f;
        }
        pos += __popcll(bal);
    }
}

// Selection start: nothing fixed yet, the k-th largest of all entries; clears the histogram.
__global__ void sel_init_kernel(SelState* st, uint32_t k, unsigned* hist) {
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) hist[i] = 0u;
    if (threadIdx.x == 0) {
        st->prefix = 0u;
        st->mask = 0u;
        st->krem = k;
        st->pad = 0u;
    }
}

// Dense identity (pitch ld) for Psi_0.
__global__ void eye_kernel(int d, float* P, int64_t ld) {
    const int64_t total = (int64_t)d * ld;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / ld, c = e % ld;
        P[e] = (r == c) ? 1.f : 0.f;
    }
}

}  // namespace cpa
