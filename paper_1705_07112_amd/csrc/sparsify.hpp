// The sparsifying transform and component truncation of Algorithm 1 (Sec. III-B):
//   Phi = T G T^T with T the 8 x 8 block DCT (kron(I, D_8), eq. sing_shrink_exact_sparse),
//         the one-level Haar DWT (optionally with every high-frequency component
//         set to zero, as in the experiments of Sec. V), the identity, or the
//         full DCT (dense: two FP32 products each way, see dct_fill_kernel),
//   underline Phi_ij = Phi_ij if |Phi_ij| >= eps (eq. threshold_components), with
//         eps = the k-th largest |Phi_ij| (the threshold rule of eq. recommendation_epsilon),
//   hat H(underline Phi) by the three-term recurrence with underline Phi in CSR
//         (psi_step_kernel, one sparse product per step),
//   M = T^T hat H T, then hat G = X M (or M X).
//
// Kernels:
//   bt_forward_kernel   one wave per pair of 8 x 8 tiles (I <= J), four to a workgroup
//                       (bt_forward_blk_kernel: one workgroup per 64 x 64 block,
//                       the same values, when d is a multiple of 64):
//                       P = D G_IJ D^T in FP64 from the FP32 Gram, written to tile
//                       (I, J) and transposed to (J, I); diagonal tiles are
//                       symmetrised ((P + P^T)/2).  Phi is therefore exactly
//                       symmetric, so an entry and its mirror always fall on the
//                       same side of eps.  D is passed in (the DCT table, the
//                       one-level Haar table with the four low-pass rows first,
//                       or I); with the Haar table the high-frequency rows and
//                       columns can be zeroed.
//   sel_hist_kernel /   radix selection of the k-th largest |Phi| on the FP32 bit
//   sel_pick_kernel     patterns of |Phi| (monotone as unsigned integers): three
//                       passes of 11, 11 and 9 bits over the upper triangle (an
//                       entry above the diagonal counted twice); exact integer
//                       histograms, so the threshold is the same on every run.  The
//                       pick finds the digit with a suffix scan over the bins (one
//                       workgroup).
//   trunc_count_kernel, one wave per row: counts the kept entries; after an
//   trunc_fill_kernel   exclusive scan, writes (column, value) in column order
//                       (ballot + prefix popcount) and zeroes the dropped entries of
//                       Phi in place (the dense underline Phi feeds the power
//                       iteration).
//   compact_rows_kernel the rows with kept entries; the recurrence runs on that
//   remap_cols_kernel   block only (an empty row of the symmetric truncated matrix
//   eye_compact_kernel  is an empty column too: an eigenvector with eigenvalue 0).
//   psi_step_kernel     one recurrence step on the CSR matrix: a workgroup per row
//                       and 128-column panel, the row's entries spread over its
//                       8 lane groups (the kept rows are very uneven).
//   bt_inverse_kernel   M_IJ = D^T H_IJ D for every tile (one wave each; by 64 x 64
//                       blocks in bt_inverse_blk_kernel), FP64 inside; expands the
//                       compact hat H (hat h(0) on the empty diagonal entries).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f32.hpp"
#include "spectral.hpp"

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

// zero_high: rows 4..7 of the table are high-frequency components (the Haar
// table); every entry of Phi in such a row or column is set to zero.
// Wave w of the workgroup takes tile pair 4 blockIdx.x + w (waves past the last
// pair only join the barriers).
__global__ void __launch_bounds__(256) bt_forward_kernel(int d, const float* G, int64_t ldg, float* Phi, int64_t ldp,
                                                         Dct8 D, int zero_high) {
    __shared__ double g[4][8][9];
    __shared__ double t[4][8][9];
    const int wv = threadIdx.x >> 6;
    // tile pair index -> (I, J), I <= J, row-major over the upper triangle
    const int nt = d / 8;
    const int npair = nt * (nt + 1) / 2;
    const int pair = blockIdx.x * 4 + wv;
    const bool valid = pair < npair;
    int p = valid ? pair : 0, I = 0;
    while (p >= nt - I) {
        p -= nt - I;
        ++I;
    }
    const int J = I + p;
    const int a = (threadIdx.x & 63) >> 3, b = threadIdx.x & 7;
    g[wv][a][b] = valid ? (double)G[(int64_t)(8 * I + a) * ldg + 8 * J + b] : 0.0;
    __syncthreads();
    // t = G_IJ D^T: t[a][b] = sum_j g[a][j] D[b][j]
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += g[wv][a][j] * D.d[8 * b + j];
    t[wv][a][b] = s;
    __syncthreads();
    // P = D t: P[a][b] = sum_i D[a][i] t[i][b]
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) v += D.d[8 * a + i] * t[wv][i][b];
    if (zero_high && (a >= 4 || b >= 4)) v = 0.0;
    g[wv][a][b] = v;   // reuse: the tile's P (every wave reaches the barrier)
    __syncthreads();
    if (!valid) return;
    if (I == J) {
        const double sym = 0.5 * (g[wv][a][b] + g[wv][b][a]);
        Phi[(int64_t)(8 * I + a) * ldp + 8 * J + b] = (float)sym;
    } else {
        const float f = (float)v;
        Phi[(int64_t)(8 * I + a) * ldp + 8 * J + b] = f;
        Phi[(int64_t)(8 * J + b) * ldp + 8 * I + a] = f;
    }
}

// The forward transform by 64 x 64 blocks (d a multiple of 64): one workgroup of
// 256 per block (BI, BJ), BI <= BJ; thread t owns row t / 4 of the block and its
// 16 columns 16 (t % 4) .. + 15 (two 8-column tile groups).  The same FP64
// operations in the same order as bt_forward_kernel, so Phi is bit for bit the
// same:  t = G_IJ D^T per tile in registers, t through LDS, P = D t, P through
// LDS; every global access is a contiguous row segment: the block's P to
// (BI, BJ) and its transpose to (BJ, BI); on a diagonal block each tile takes
// the upper tile's values (a diagonal tile (P + P^T) / 2).
constexpr int kBtPad = 65;
__global__ void __launch_bounds__(256) bt_forward_blk_kernel(int d, const float* G, int64_t ldg, float* Phi,
                                                             int64_t ldp, Dct8 D, int zero_high) {
    __shared__ double ts[64 * kBtPad];
    const int nbk = d / 64;
    int p = blockIdx.x, BI = 0;
    while (p >= nbk - BI) {
        p -= nbk - BI;
        ++BI;
    }
    const int BJ = BI + p;
    const int r = threadIdx.x >> 2, c0 = 16 * (threadIdx.x & 3);
    const int a = r & 7;
    // this thread's 16 entries of G (row r, columns c0 .. c0 + 15)
    double g[16];
    {
        const float* src = G + (int64_t)(64 * BI + r) * ldg + 64 * BJ + c0;
        const bool vec = ((ldg & 3) == 0) && ((reinterpret_cast<uintptr_t>(G) & 15) == 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (vec) {
                const f32x4 x = *reinterpret_cast<const f32x4*>(src + 4 * q);
                for (int e = 0; e < 4; ++e) g[4 * q + e] = (double)x[e];
            } else {
                for (int e = 0; e < 4; ++e) g[4 * q + e] = (double)src[4 * q + e];
            }
        }
    }
    // t[r][c] = sum_j G[r][8 (c / 8) + j] D[c % 8][j]
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < 8; ++j) s += g[8 * h + j] * D.d[8 * b + j];
            ts[r * kBtPad + c0 + 8 * h + b] = s;
        }
    __syncthreads();
    // P[r][c] = sum_i D[r % 8][i] t[8 (r / 8) + i][c]
    double pv[16];
    const int rb = r & ~7;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int c = c0 + k;
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) v += D.d[8 * a + i] * ts[(rb + i) * kBtPad + c];
        if (zero_high && (a >= 4 || (c & 7) >= 4)) v = 0.0;
        pv[k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) ts[r * kBtPad + c0 + k] = pv[k];
    __syncthreads();
    float* dst = Phi + (int64_t)(64 * BI + r) * ldp + 64 * BJ + c0;
    if (BI == BJ) {
        const int I = r >> 3;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int c = c0 + k, J = c >> 3;
            double v;
            if (I < J)
                v = ts[r * kBtPad + c];
            else if (I > J)
                v = ts[c * kBtPad + r];
            else
                v = 0.5 * (ts[r * kBtPad + c] + ts[c * kBtPad + r]);
            dst[k] = (float)v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) dst[k] = (float)ts[r * kBtPad + c0 + k];
        // the mirror: row r of block (BJ, BI) is column r of P
        float* mir = Phi + (int64_t)(64 * BJ + r) * ldp + 64 * BI + c0;
#pragma unroll
        for (int k = 0; k < 16; ++k) mir[k] = (float)ts[(c0 + k) * kBtPad + r];
    }
}

// hat h(0) with the arithmetic of the recurrence on a row with no kept entries
// (Z = 0, Psi_0 = 1): Psi_k = (-1)^k exactly, summed in FP32 in step order.
__device__ inline float hhat_at_zero(const double* scal, int K) {
    const float c0h = (float)(0.5 * scal[SC_COEF]);
    if (K < 2) return c0h;
    float yp = 1.f, yk = -1.f;
    float out = c0h + (float)scal[SC_COEF + 1] * yk;
    for (int k = 1; k + 1 <= K - 1; ++k) {
        const float y = -2.f * yk - yp;
        out += (float)scal[SC_COEF + k + 1] * y;
        yp = yk;
        yk = y;
    }
    return out;
}

// M_IJ = D^T H_IJ D.  With pos != nullptr, H holds hat H of the nonempty rows and
// columns only (row r of the full matrix is row pos[r] there, pos[r] < 0 for an
// empty row): an empty row r of the truncated matrix is an eigenvector with
// eigenvalue 0, so the full hat H is the compact one on the nonempty indices and
// hat h(0) on the diagonal of the empty ones.
// Wave w of the workgroup takes tile 4 blockIdx.x + w.
__global__ void __launch_bounds__(256) bt_inverse_kernel(int d, const float* H, int64_t ldh, float* M, int64_t ldm,
                                                         Dct8 D, const int32_t* pos, const double* scal, int K) {
    __shared__ double hs[4][8][9];
    __shared__ double ts[4][8][9];
    const int wv = threadIdx.x >> 6;
    double(*h)[9] = hs[wv];
    double(*t)[9] = ts[wv];
    const int nt = d / 8;
    const int tile = blockIdx.x * 4 + wv;
    const bool valid = tile < nt * nt;
    const int I = valid ? tile / nt : 0, J = valid ? tile % nt : 0;
    const int a = (threadIdx.x & 63) >> 3, b = threadIdx.x & 7;
    const int r = 8 * I + a, c = 8 * J + b;
    float hv = 0.f;
    if (valid) {
        if (pos) {
            const int pr = pos[r], pc = pos[c];
            if (pr >= 0 && pc >= 0)
                hv = H[(int64_t)pr * ldh + pc];
            else
                hv = r == c ? hhat_at_zero(scal, K) : 0.f;
        } else {
            hv = H[(int64_t)r * ldh + c];
        }
    }
    h[a][b] = (double)hv;
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
    if (valid) M[(int64_t)r * ldm + c] = (float)v;
}

// The inverse transform by 64 x 64 blocks (d a multiple of 64): one workgroup of
// 256 per block, thread t owning row t / 4 and 16 columns as in the forward
// kernel, the same FP64 operations in the same order as bt_inverse_kernel
// (t = H_IJ D per tile in registers, through LDS, M = D^T t), rows of M written
// contiguously.
__global__ void __launch_bounds__(256) bt_inverse_blk_kernel(int d, const float* H, int64_t ldh, float* M,
                                                             int64_t ldm, Dct8 D, const int32_t* pos,
                                                             const double* scal, int K) {
    __shared__ double ts[64 * kBtPad];
    const int nbk = d / 64;
    const int BI = blockIdx.x / nbk, BJ = blockIdx.x % nbk;
    const int r = threadIdx.x >> 2, c0 = 16 * (threadIdx.x & 3);
    const int a = r & 7;
    const int gr = 64 * BI + r;
    double h[16];
    {
        const float hz = pos ? hhat_at_zero(scal, K) : 0.f;
        const int pr = pos ? pos[gr] : gr;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int gc = 64 * BJ + c0 + k;
            float hv;
            if (pos) {
                const int pc = pos[gc];
                hv = (pr >= 0 && pc >= 0) ? H[(int64_t)pr * ldh + pc] : (gr == gc ? hz : 0.f);
            } else {
                hv = H[(int64_t)gr * ldh + gc];
            }
            h[k] = (double)hv;
        }
    }
    // t[r][c] = sum_j H[r][8 (c / 8) + j] D[j][c % 8]
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < 8; ++j) s += h[8 * hh + j] * D.d[8 * j + b];
            ts[r * kBtPad + c0 + 8 * hh + b] = s;
        }
    __syncthreads();
    // M[r][c] = sum_i D[i][r % 8] t[8 (r / 8) + i][c]
    const int rb = r & ~7;
    float* dst = M + (int64_t)gr * ldm + 64 * BJ + c0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int c = c0 + k;
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) v += D.d[8 * i + a] * ts[(rb + i) * kBtPad + c];
        dst[k] = (float)v;
    }
}

// Histogram of the next digit of |Phi| over the entries matching the prefix.
// Phi is exactly symmetric, so the upper triangle suffices: an entry above the
// diagonal counts twice (itself and its mirror), a diagonal entry once; the
// counts are those of all d^2 entries.  Workgroup b takes rows b and d - 1 - b
// (equal work), four columns to a thread (16-byte loads when aligned).
__global__ void __launch_bounds__(256) sel_hist_kernel(int d, const float* Phi, int64_t ldp, int pass,
                                                       const SelState* st, unsigned* hist) {
    __shared__ unsigned lh[kSelBins];
    for (int i = threadIdx.x; i < kSelBins; i += 256) lh[i] = 0u;
    __syncthreads();
    const uint32_t prefix = st->prefix, mask = st->mask;
    const int shift = sel_shift(pass), nb = (1 << sel_bits(pass)) - 1;
    const bool vec = (d & 3) == 0 && (ldp & 3) == 0 && ((reinterpret_cast<uintptr_t>(Phi) & 15) == 0);
    for (int b = blockIdx.x; 2 * b < d; b += gridDim.x) {
        for (int side = 0; side < 2; ++side) {
            const int r = side == 0 ? b : d - 1 - b;
            if (side == 1 && r == b) break;
            const float* row = Phi + (int64_t)r * ldp;
            // columns r .. d - 1, from the 4-aligned column at or below r
            for (int c0 = r & ~3; c0 < d; c0 += 1024) {
                const int c = c0 + 4 * threadIdx.x;
                float v[4] = {0.f, 0.f, 0.f, 0.f};
                if (vec && c + 3 < d) {
                    const f32x4 x = *reinterpret_cast<const f32x4*>(row + c);
                    for (int e = 0; e < 4; ++e) v[e] = x[e];
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (c + e < d) v[e] = row[c + e];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ce = c + e;
                    if (ce < r || ce >= d) continue;
                    const uint32_t key = abs_key(v[e]);
                    if ((key & mask) == prefix) atomicAdd(&lh[(key >> shift) & nb], ce == r ? 1u : 2u);
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += 256)
        if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

// The bin holding the krem-th largest key (counting from the top), appended to
// the prefix; clears the histogram for the next pass.  One workgroup.
__global__ void __launch_bounds__(256) sel_pick_kernel(int pass, SelState* st, unsigned* hist) {
    __shared__ unsigned h[kSelBins];
    __shared__ uint32_t part[256];
    __shared__ uint32_t s_bin, s_above;
    const int t = threadIdx.x;
    const int nbin = 1 << sel_bits(pass), per = nbin / 256;
    for (int i = t; i < kSelBins; i += 256) {
        h[i] = hist[i];
        hist[i] = 0u;
    }
    __syncthreads();
    // thread t owns bins [hi - per, hi): thread 0 the largest digits
    const int hi = nbin - per * t;
    uint32_t sum = 0;
    for (int u = 1; u <= per; ++u) sum += h[hi - u];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    // entries above thread t's bins: excl; the digit is in the one thread where the
    // count reaches krem (1 <= krem <= the entries matching the prefix)
    const uint32_t krem = st->krem;
    const uint32_t incl = part[t], excl = incl - sum;
    if (excl < krem && incl >= krem) {
        uint32_t above = excl;
        int bin = hi - 1;
        for (int u = 1; u <= per; ++u) {
            const int i = hi - u;
            if (above + h[i] >= krem) {
                bin = i;
                break;
            }
            above += h[i];
        }
        s_bin = (uint32_t)bin;
        s_above = above;
    }
    __syncthreads();
    if (t == 0) {
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
    const float* row = Phi + (int64_t)r * ldp;
    int c = 0;
    if ((d & 3) == 0 && (ldp & 3) == 0 && ((reinterpret_cast<uintptr_t>(Phi) & 15) == 0)) {
        // 16-byte loads, four of them in flight per lane
#pragma unroll 4
        for (int j = 4 * lane; j < d; j += 256) {
            const f32x4 x = *reinterpret_cast<const f32x4*>(row + j);
#pragma unroll
            for (int e = 0; e < 4; ++e) c += abs_key(x[e]) >= eps ? 1 : 0;
        }
    } else {
        for (int j = lane; j < d; j += 64) c += abs_key(row[j]) >= eps ? 1 : 0;
    }
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

// A given threshold: the key of |eps| (FP32), every bit fixed.
__global__ void sel_fixed_kernel(SelState* st, float eps) {
    if (threadIdx.x == 0) {
        st->prefix = abs_key(eps);
        st->mask = 0xffffffffu;
        st->krem = 0u;
        st->pad = 0u;
    }
}

// One step of the recurrence on the truncated matrix (CSR):
//   Z = underline Phi Psi_k,  Psi_{k+1} = a Z + b Psi_k + c Psi_{k-1},
//   out = c_0/2 Psi_0 + c_1 Psi_1 (step 0) or out += c_{k+1} Psi_{k+1}
// with a, b, c = 2/Lambda, -1, 0 (step 0) or 4/Lambda, -2, -1 and the coefficients
// from the scalar block.  The rows of the truncated matrix are very uneven (under
// the block DCT the kept entries gather on the block-DC rows), so a workgroup
// takes one row and 128-column panel at a time and spreads the row's entries over
// its 8 groups of 32 lanes (entry e to group e mod 8); the 8 partial sums are
// added in LDS in a fixed order.
// Compact form (rows != nullptr): the matrices are n x n with n = *nrows, row i
// of the recurrence is CSR row rows[i] and the column indices are compact; the
// columns up to the next multiple of 4 are computed too (they never mix with the
// others).  Pprev and Pdst may alias (same element, same thread).  Row pitch ld,
// rows 16-byte aligned, d % 4 == 0.
constexpr int kPsiJ = 128;

__global__ void __launch_bounds__(256) psi_step_kernel(int d, const int32_t* rows, const int32_t* nrows,
                                                       const int32_t* rowptr, const int32_t* colidx, const float* val,
                                                       const float* Pk, const float* Pprev, float* Pdst, int64_t ld,
                                                       float* out, const double* scal, int step, int last) {
    __shared__ f32x4 red[8][32];
    const int n = rows ? *nrows : d;
    const int w4 = (n + 3) & ~3;
    const int panels = (w4 + kPsiJ - 1) / kPsiJ;
    const int items = n * panels;
    const int g = threadIdx.x >> 5, q = threadIdx.x & 31;
    float a, b, cc;
    if (step == 0) {
        a = (float)scal[SC_A1];
        b = -1.f;
        cc = 0.f;
    } else {
        a = (float)scal[SC_A2];
        b = -2.f;
        cc = -1.f;
    }
    const float ck = (float)scal[SC_COEF + step + 1];
    const float c0h = (float)(0.5 * scal[SC_COEF]);
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int r = it / panels, panel = it - r * panels;
        const int j = panel * kPsiJ + 4 * q;
        const bool in = j < w4;
        const int rr = rows ? rows[r] : r;
        const int e0 = rowptr[rr], e1 = rowptr[rr + 1];
        f32x4 z = {0.f, 0.f, 0.f, 0.f};
        if (e1 > e0) {   // the same for the whole workgroup
            if (in) {
                f32x4 acc[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] = (f32x4){0.f, 0.f, 0.f, 0.f};
                int e = e0 + g;
                for (; e + 24 < e1; e += 32) {
                    f32x4 w[4];
                    float sv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        sv[u] = val[e + 8 * u];
                        w[u] = *reinterpret_cast<const f32x4*>(Pk + (int64_t)colidx[e + 8 * u] * ld + j);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[u] += sv[u] * w[u];
                }
                for (; e < e1; e += 8)
                    acc[0] += val[e] * *reinterpret_cast<const f32x4*>(Pk + (int64_t)colidx[e] * ld + j);
                z = (acc[0] + acc[1]) + (acc[2] + acc[3]);
            }
            red[g][q] = z;
            __syncthreads();
            if (g == 0) {
                z = red[0][q];
#pragma unroll
                for (int u = 1; u < 8; ++u) z += red[u][q];
            }
            __syncthreads();   // red is refilled by the next item
        }
        if (g != 0 || !in) continue;
        const int64_t o = (int64_t)r * ld + j;
        const f32x4 yk = *reinterpret_cast<const f32x4*>(Pk + o);
        f32x4 yp = {0.f, 0.f, 0.f, 0.f}, ov = {0.f, 0.f, 0.f, 0.f};
        if (step > 0) {
            yp = *reinterpret_cast<const f32x4*>(Pprev + o);
            ov = *reinterpret_cast<const f32x4*>(out + o);
        }
        f32x4 yn, on;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float y = a * z[t] + b * yk[t];
            if (step > 0) y += cc * yp[t];
            yn[t] = y;
            on[t] = step == 0 ? c0h * yk[t] + ck * y : ov[t] + ck * y;
        }
        *reinterpret_cast<f32x4*>(out + o) = on;
        if (!last) *reinterpret_cast<f32x4*>(Pdst + o) = yn;
    }
}

// The nonempty rows of the truncated matrix (cnt[r] > 0), single workgroup of
// 256: pos[r] = compact index or -1, rows[i] = the i-th nonempty row,
// nrows[0] = their number, nrows[1] = the kept entries (sum of cnt).
__global__ void __launch_bounds__(256) compact_rows_kernel(int d, const int32_t* cnt, int32_t* pos, int32_t* rows,
                                                           int32_t* nrows) {
    __shared__ int32_t part[256];
    __shared__ int32_t tot[256];
    const int t = threadIdx.x;
    const int per = (d + 255) / 256;
    const int lo = min(d, t * per), hi = min(d, lo + per);
    int32_t sum = 0, all = 0;
    for (int i = lo; i < hi; ++i) {
        sum += cnt[i] > 0 ? 1 : 0;
        all += cnt[i];
    }
    part[t] = sum;
    tot[t] = all;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) tot[t] += tot[t + off];
        __syncthreads();
    }
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - sum;
    for (int i = lo; i < hi; ++i) {
        if (cnt[i] > 0) {
            pos[i] = run;
            rows[run] = i;
            ++run;
        } else {
            pos[i] = -1;
        }
    }
    if (t == 255) {
        nrows[0] = part[255];
        nrows[1] = tot[0];
    }
}

// Column indices of the CSR to compact ones (every kept column is a nonempty row:
// the matrix is symmetric).
__global__ void remap_cols_kernel(int d, const int32_t* rowptr, int32_t* colidx, const int32_t* pos) {
    const int32_t nnz = rowptr[d];
    for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x)
        colidx[e] = pos[colidx[e]];
}

// The orthonormal DCT-II matrix D[k][j] = s_k cos(pi (2 j + 1) k / (2 d)),
// s_0 = sqrt(1/d), s_k = sqrt(2/d), and its transpose, in FP32 from FP64 values
// (the angle reduced exactly in integers first).
__global__ void dct_fill_kernel(int d, float* Dm, float* Dt) {
    const int64_t total = (int64_t)d * d;
    const double s0 = sqrt(1.0 / d), s1 = sqrt(2.0 / d);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e / d), j = (int)(e % d);
        const int64_t q = ((int64_t)(2 * j + 1) * k) % (4 * (int64_t)d);   // angle = pi q / (2 d)
        const float v = (float)((k == 0 ? s0 : s1) * cos(M_PI * (double)q / (2.0 * d)));
        Dm[(int64_t)k * d + j] = v;
        Dt[(int64_t)j * d + k] = v;
    }
}

// P <- (P + P^T) / 2 in place (d x d, pitch ld).
__global__ void symmetrize_kernel(int d, float* P, int64_t ld) {
    const int64_t total = (int64_t)d * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / d), j = (int)(e % d);
        if (j <= i) continue;
        const float a = P[(int64_t)i * ld + j], b = P[(int64_t)j * ld + i];
        const float v = 0.5f * (a + b);
        P[(int64_t)i * ld + j] = v;
        P[(int64_t)j * ld + i] = v;
    }
}

// The compact block of the truncated matrix, Phi_S[i][j] = Phi[rows[i]][rows[j]]
// where |Phi| >= eps (the selected key) and 0 elsewhere, for i, j < ns, zero up to
// nb x nb (pitch nb); Phi itself is untruncated.
__global__ void gather_compact_kernel(int ns, int nb, const int32_t* rows, const float* Phi, int64_t ldp,
                                      const SelState* st, float* out) {
    const uint32_t eps = st->prefix;
    const int64_t total = (int64_t)nb * nb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / nb), c = (int)(e % nb);
        float v = 0.f;
        if (r < ns && c < ns) {
            v = Phi[(int64_t)rows[r] * ldp + rows[c]];
            if (abs_key(v) < eps) v = 0.f;
        }
        out[e] = v;
    }
}

// Compact identity: the leading n x n block (n = *nrows, columns up to the next
// multiple of 4) of a matrix with pitch ld.
__global__ void eye_compact_kernel(const int32_t* nrows, float* P, int64_t ld) {
    const int n = *nrows, w4 = (n + 3) & ~3;
    const int64_t total = (int64_t)n * w4;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / w4, c = e % w4;
        P[r * ld + c] = (r == c) ? 1.f : 0.f;
    }
}

// Warm start of the compact block's power iteration across calls, kept in the
// coordinates of the full transformed Gram (the block's rows change from call to
// call): before the bound, compact[i] = full[rows[i]] for the ns kept rows and 0 on
// the padding rows up to nb; after it, full[j] = compact[pos[j]] on kept rows, 0 on
// empty ones.
__global__ void warm_gather_kernel(int ns, int nb, const int32_t* rows, const double* full, double* compact) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x)
        compact[i] = i < ns ? full[rows[i]] : 0.0;
}

__global__ void warm_scatter_kernel(int d, const int32_t* pos, const double* compact, double* full) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d; j += gridDim.x * blockDim.x)
        full[j] = pos[j] >= 0 ? compact[pos[j]] : 0.0;
}

}  // namespace cpa
