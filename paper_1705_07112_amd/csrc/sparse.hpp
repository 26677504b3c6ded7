// Sparse X: the shrinkage of a CSR matrix S (m x n, m >= n) in operator form.
//
// The identity X p(X^T X) = p(X X^T) X (from eq. sing_shrink_from_eig_shrink)
// gives Y_k = T_k(Ghat_L) S with Ghat_L = (2/Lambda) S S^T - I, so one
// recurrence step is
//   W = S^T Y_k            (n x n, SpMM with the transposed pattern)
//   Y_{k+1} = 2 ((2/Lambda) S W - Y_k) - Y_{k-1}   (SpMM + fused Chebyshev epilogue)
// and neither S^T S nor S S^T is ever formed.  Y_0 = S (densified).
//
// Kernels
//   csc_*            the transposed pattern (column pointers, row indices and the
//                    CSR position of each entry, rows ascending within a column),
//                    built once per pattern on the device;
//   spmm_t_kernel    W[c][:] = sum_{(r,c) in S} s_rc Y[r][:], one wave per output
//                    column c and 32-column panel of Y, panels outermost: a panel of
//                    Y (m x 32 floats, 2.5 MB at m = 20000) stays in each XCD's 4 MB
//                    L2 while every wave gathers from it; 8 nonzeros in flight per
//                    wave (8 lanes x float4 per gathered 128-byte row segment);
//   spmm_cheb_kernel Z[r][:] = sum_{(r,c)} s_rc W[c][:] with the recurrence epilogue,
//                    one wave per output row and 128-column panel of W (n x 128
//                    floats, 2 MB at n = 4000), 2 nonzeros in flight per wave.
// Both kernels read the pattern and the streamed operands with non-temporal
// loads and stores so that they do not evict the gathered panel; partial sums
// are combined in a fixed order (xor shuffles), so results do not depend on
// scheduling.
//   power_op_kernel  power iteration on S^T S through two sparse products per step,
//                    one launch of resident workgroups (two grid barriers per product); the
//                    vectors and partial sums go through agent-scope atomic
//                    accesses, so the barriers flush no cache and the pattern
//                    stays in L2 from one product to the next.
//   lanczos_op_kernel  the k-step Lanczos bound on S^T S in the same way.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spectral.hpp"

namespace cpa {

constexpr int SP_THREADS = 256;
constexpr int SP_WAVES = SP_THREADS / 64;   // output rows (or columns) per workgroup, one per wave
constexpr int SPT_J = 32;                   // panel width of S^T Y_k
constexpr int SPC_J = 128;                  // panel width of S W

// Flags a malformed CSR (rowptr[0] != 0, rowptr[m] != nnz, decreasing row
// pointers, a column index outside [0, n), or columns of a row not strictly
// increasing).  Reads only rowptr[0..m] and colidx[0..nnz) (row extents are
// clamped to [0, nnz] before a row's columns are read).
__global__ void csr_validate_kernel(int m, int n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                                    int* bad) {
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (tid == 0 && (rowptr[0] != 0 || rowptr[m] != nnz)) atomicOr(bad, 1);
    for (int64_t r = tid; r < m; r += stride) {
        const int64_t lo = rowptr[r], hi = rowptr[r + 1];
        if (lo > hi) atomicOr(bad, 1);
        const int64_t a = lo < 0 ? 0 : (lo > nnz ? nnz : lo), z = hi < 0 ? 0 : (hi > nnz ? nnz : hi);
        for (int64_t e = a + 1; e < z; ++e)
            if (colidx[e] <= colidx[e - 1]) {
                atomicOr(bad, 1);
                break;
            }
    }
    for (int64_t e = tid; e < nnz; e += stride)
        if (colidx[e] < 0 || colidx[e] >= n) atomicOr(bad, 1);
}

__global__ void csc_count_kernel(int64_t nnz, const int32_t* colidx, int32_t* cnt) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(cnt + colidx[e], 1);
}

// Exclusive scan of cnt[0..n) into colptr[0..n], single workgroup.
__global__ void csc_scan_kernel(int n, const int32_t* cnt, int32_t* colptr) {
    __shared__ int32_t part[SP_THREADS];
    const int per = (n + SP_THREADS - 1) / SP_THREADS;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    int32_t s = 0;
    for (int i = lo; i < hi; ++i) s += cnt[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int t = 0; t < SP_THREADS; ++t) {
            const int32_t v = part[t];
            part[t] = run;
            run += v;
        }
        colptr[n] = run;
    }
    __syncthreads();
    int32_t run = part[threadIdx.x];
    for (int i = lo; i < hi; ++i) {
        colptr[i] = run;
        run += cnt[i];
    }
}

// Places every entry in its column (order within a column arbitrary here).
__global__ void csc_scatter_kernel(int m, const int32_t* rowptr, const int32_t* colidx, const int32_t* colptr,
                                   int32_t* fill, int32_t* crow, int32_t* csrc) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < m; r += gridDim.x * blockDim.x) {
        for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
            const int32_t c = colidx[e];
            const int32_t p = colptr[c] + atomicAdd(fill + c, 1);
            crow[p] = r;
            csrc[p] = e;
        }
    }
}

// Sorts each column by row: the rank of an entry is the number of entries of
// its column with a smaller row (rows are distinct within a column).  One wave
// per column; results go to the second pair of arrays.
__global__ void csc_sort_kernel(int n, const int32_t* colptr, const int32_t* crow_in, const int32_t* csrc_in,
                                int32_t* crow, int32_t* csrc) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (c >= n) return;
    const int32_t b = colptr[c], len = colptr[c + 1] - b;
    for (int32_t i = lane; i < len; i += 64) {
        const int32_t r = crow_in[b + i];
        int32_t rank = 0;
        for (int32_t j = 0; j < len; ++j) rank += crow_in[b + j] < r ? 1 : 0;
        crow[b + rank] = r;
        csrc[b + rank] = csrc_in[b + i];
    }
}

// Y0 = S (dense m x n, ld = ldy), the buffer already zeroed.
__global__ void densify_kernel(int m, const int32_t* rowptr, const int32_t* colidx, const float* val, float* Y,
                               int64_t ldy) {
    for (int r = blockIdx.x; r < m; r += gridDim.x)
        for (int32_t e = rowptr[r] + threadIdx.x; e < rowptr[r + 1]; e += blockDim.x)
            Y[(int64_t)r * ldy + colidx[e]] = val[e];
}

// cval[p] = val[csrc[p]]: the values in column order, gathered once per shrink.
__global__ void csc_values_kernel(int64_t nnz, const int32_t* csrc, const float* val, float* cval) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        cval[p] = val[csrc[p]];
}

__device__ inline f32x4 sp_shfl_xor4(f32x4 v, int off) {
    f32x4 r;
    r[0] = __shfl_xor(v[0], off, 64);
    r[1] = __shfl_xor(v[1], off, 64);
    r[2] = __shfl_xor(v[2], off, 64);
    r[3] = __shfl_xor(v[3], off, 64);
    return r;
}

// W[c][j] = sum over column c of S of s_rc * Y[r][j], j in this wave's 32-column
// panel.  Lane = 8 * g + q: row group g and float4 q of the panel.  Grid: ceil(n / 4) x ceil(ncols / 32) workgroups,
// panels outermost.
__global__ void __launch_bounds__(SP_THREADS) spmm_t_kernel(int n, int ncols, const int32_t* colptr,
                                                            const int32_t* crow, const float* cval,
                                                            const float* Y, int64_t ldy, float* W, int64_t ldw) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int groups = (n + SP_WAVES - 1) / SP_WAVES;
    const int panel = blockIdx.x / groups;
    const int c = (blockIdx.x - panel * groups) * SP_WAVES + wave;
    if (c >= n) return;
    const int g = lane >> 3;
    const int j = panel * SPT_J + 4 * (lane & 7);
    const bool full = j + 3 < ncols;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int32_t p0 = colptr[c], p1 = colptr[c + 1];
    // chunks of 64 entries: one coalesced load of (row, value) per lane, then
    // row group g gathers entries g, g + 8, ..., g + 56 with all eight in flight
    for (int32_t base = p0; base < p1; base += 64) {
        const int cnt = p1 - base < 64 ? (int)(p1 - base) : 64;
        int32_t rl = 0;
        float sl = 0.f;
        if (lane < cnt) {
            rl = __builtin_nontemporal_load(crow + base + lane);
            sl = __builtin_nontemporal_load(cval + base + lane);
        }
        f32x4 y[8];
        float sv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = g + 8 * u;
            const int32_t r = __shfl(rl, i, 64);
            sv[u] = __shfl(sl, i, 64);
            y[u] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (i < cnt) {
                const float* yr = Y + (int64_t)r * ldy + j;
                if (full) {
                    y[u] = *reinterpret_cast<const f32x4*>(yr);
                } else {
                    for (int q = 0; q < 4; ++q)
                        if (j + q < ncols) y[u][q] = yr[q];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += sv[u] * y[u];
    }
    acc += sp_shfl_xor4(acc, 8);
    acc += sp_shfl_xor4(acc, 16);
    acc += sp_shfl_xor4(acc, 32);
    if (g != 0 || j >= ncols) return;
    float* wr = W + (int64_t)c * ldw + j;
    if (full) {
        *reinterpret_cast<f32x4*>(wr) = acc;
    } else {
        for (int q = 0; q < 4; ++q)
            if (j + q < ncols) wr[q] = acc[q];
    }
}

// sum over row r of S of s_rc B[c][j..j+3] for entry group g (entries g, g + 2, ...
// of every 64-entry chunk); the caller adds the two groups with one shuffle.
__device__ inline f32x4 sp_row_gather(int r, int g, int j, bool full, int ncols, const int32_t* rowptr,
                                      const int32_t* colidx, const float* val, const float* W, int64_t ldw) {
    const int lane = threadIdx.x & 63;
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
    const int32_t e0 = rowptr[r], e1 = rowptr[r + 1];
    // chunks of 64 entries: one coalesced load of (column, value) per lane, then
    // entry group g gathers entries g, g + 2, ..., eight at a time in flight
    for (int32_t base = e0; base < e1; base += 64) {
        const int cnt = e1 - base < 64 ? (int)(e1 - base) : 64;
        int32_t cl = 0;
        float sl = 0.f;
        if (lane < cnt) {
            cl = __builtin_nontemporal_load(colidx + base + lane);
            sl = __builtin_nontemporal_load(val + base + lane);
        }
        // the trip count is uniform across the wave (shuffles read every lane)
        for (int u0 = 0; u0 < 32 && 2 * u0 < cnt; u0 += 8) {
            f32x4 w[8];
            float sv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = g + 2 * (u0 + u);
                const int32_t c = __shfl(cl, i, 64);
                sv[u] = __shfl(sl, i, 64);
                w[u] = f32x4{0.f, 0.f, 0.f, 0.f};
                if (i < cnt) {
                    const float* wr = W + (int64_t)c * ldw + j;
                    if (full) {
                        w[u] = *reinterpret_cast<const f32x4*>(wr);
                    } else {
                        for (int q = 0; q < 4; ++q)
                            if (j + q < ncols) w[u][q] = wr[q];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) z += sv[u] * w[u];
        }
    }
    return z;
}

// Z[r][j] = sum over row r of S of s_rc W[c][j], then the recurrence epilogue:
//   first step: Ynew = a1 Z - Yk,  out = c0/2 Yk + c1 Ynew
//   later:      Ynew = a2 Z - 2 Yk - Yprev,  out += c_{k+1} Ynew
// Ynew goes to Ydst (may equal Yprev) unless this is the last step.
// Lane = 32 * g + q: entry group g and float4 q of the 128-column panel.  Grid: ceil(m / 4) x ceil(ncols / 128), panels
// outermost.  The workspace buffers (W, Y*) have row pitches % 32 == 0 and
// aligned bases; `out_vec` says whether the caller's output allows 16-byte
// accesses too.
__global__ void __launch_bounds__(SP_THREADS) spmm_cheb_kernel(int m, int ncols, const int32_t* rowptr,
                                                               const int32_t* colidx, const float* val,
                                                               const float* W, int64_t ldw, const float* Yk,
                                                               const float* Yprev, float* Ydst, int64_t ldy,
                                                               float* out, int64_t ldo, const double* scal,
                                                               int step, int last, int out_vec) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int groups = (m + SP_WAVES - 1) / SP_WAVES;
    const int panel = blockIdx.x / groups;
    const int r = (blockIdx.x - panel * groups) * SP_WAVES + wave;
    if (r >= m) return;
    const int g = lane >> 5;
    const int j = panel * SPC_J + 4 * (lane & 31);
    const bool full = j + 3 < ncols;
    f32x4 z = sp_row_gather(r, g, j, full, ncols, rowptr, colidx, val, W, ldw);
    z += sp_shfl_xor4(z, 32);
    if (g != 0 || j >= ncols) return;
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
    const int64_t oy = (int64_t)r * ldy + j, oo = (int64_t)r * ldo + j;
    const int cnt = full ? 4 : ncols - j;
    f32x4 yk = {0.f, 0.f, 0.f, 0.f}, yp = {0.f, 0.f, 0.f, 0.f}, o = {0.f, 0.f, 0.f, 0.f};
    if (full) {
        yk = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(Yk + oy));
        if (step > 0) yp = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(Yprev + oy));
    } else {
        for (int q = 0; q < cnt; ++q) {
            yk[q] = Yk[oy + q];
            if (step > 0) yp[q] = Yprev[oy + q];
        }
    }
    if (step > 0) {
        if (full && out_vec) {
            o = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(out + oo));
        } else {
            for (int q = 0; q < cnt; ++q) o[q] = out[oo + q];
        }
    }
    f32x4 yn;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float y = a * z[q] + b * yk[q];
        if (step > 0) y += cc * yp[q];
        yn[q] = y;
        o[q] = step == 0 ? c0h * yk[q] + ck * y : o[q] + ck * y;
    }
    if (full && out_vec) {
        __builtin_nontemporal_store(o, reinterpret_cast<f32x4*>(out + oo));
    } else {
        for (int q = 0; q < cnt; ++q) out[oo + q] = o[q];
    }
    if (!last) {
        if (full) {
            __builtin_nontemporal_store(yn, reinterpret_cast<f32x4*>(Ydst + oy));
        } else {
            for (int q = 0; q < cnt; ++q) Ydst[oy + q] = yn[q];
        }
    }
}

// Y[r][j] = sum over row r of S of s_rc F[c][j] (the matrix-polynomial route's
// final product S p).  Same decomposition as spmm_cheb_kernel.
__global__ void __launch_bounds__(SP_THREADS) spmm_out_kernel(int m, int ncols, const int32_t* rowptr,
                                                              const int32_t* colidx, const float* val,
                                                              const float* F, int64_t ldf, float* Y, int64_t ldy,
                                                              int f_vec, int out_vec) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int groups = (m + SP_WAVES - 1) / SP_WAVES;
    const int panel = blockIdx.x / groups;
    const int r = (blockIdx.x - panel * groups) * SP_WAVES + wave;
    if (r >= m) return;
    const int g = lane >> 5;
    const int j = panel * SPC_J + 4 * (lane & 31);
    // 16-byte loads of F need ldf % 4 == 0 (f_vec); otherwise element loads
    const bool full = f_vec && j + 3 < ncols;
    f32x4 z = sp_row_gather(r, g, j, full, ncols, rowptr, colidx, val, F, ldf);
    z += sp_shfl_xor4(z, 32);
    if (g != 0 || j >= ncols) return;
    float* yr = Y + (int64_t)r * ldy + j;
    if (full && out_vec) {
        __builtin_nontemporal_store(z, reinterpret_cast<f32x4*>(yr));
    } else {
        for (int q = 0; q < 4; ++q)
            if (j + q < ncols) yr[q] = z[q];
    }
}

// ||S||_F^2 (= trace of S^T S) as per-workgroup partials in the trace slots of the
// Gram-partial layout: part[2 b] = 0, part[2 b + 1] = partial of workgroup b.
__global__ void sq_norm_kernel(int64_t nnz, const float* val, double* part) {
    __shared__ double red[16];
    double s = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        s += (double)val[e] * val[e];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = 0.0;
        part[2 * blockIdx.x + 1] = s;
    }
}

// Power iteration on G = S^T S without forming it: t = S v, w = S^T t.
// Same stopping rule, partial-sum scheme and data exchange (agent-scope atomic
// accesses, v staged in LDS when n <= kPowerVecLds) as power_coop_kernel; the cap of
// the bound uses tr(G) = ||S||_F^2 >= ||G||_F (written to SC_FRO2 as its square
// by the caller's reduction: SC_FRO2 holds tr(G)^2).
__global__ void __launch_bounds__(kPowerThreads) power_op_kernel(int m, int n, const int32_t* rowptr,
                                                                 const int32_t* colidx, const float* val,
                                                                 const int32_t* colptr, const int32_t* crow,
                                                                 const int32_t* csrc, double* tvec, double* wb0,
                                                                 double* wb1, double* part, unsigned* counter,
                                                                 double* scal, int maxit, double tol, int pw_mu,
                                                                 int pw_w2) {
    __shared__ double red[kPowerThreads / 64];
    __shared__ double bcast[2];
    __shared__ __attribute__((aligned(16))) double vl[kPowerVecLds];
    const bool in_lds = n <= kPowerVecLds;
    const int P = gridDim.x;
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (kPowerThreads / 64) + (threadIdx.x >> 6);
    const int nw = P * (kPowerThreads / 64);
    double w2prev = scal[pw_w2 + 0];
    double muprev = 0.0;
    int stop = 0, vanish = !(w2prev > 0.0);
    unsigned bar = 0;
    int t = 1;
    for (; !vanish && t <= maxit; ++t) {
        const double* wp = (t & 1) ? wb0 : wb1;
        double* wn = (t & 1) ? wb1 : wb0;
        if (in_lds) {
            for (int j = threadIdx.x; j < n; j += kPowerThreads) vl[j] = ld_agent(wp + j);
            __syncthreads();
        }
        const double inv = 1.0 / sqrt(w2prev);
        // t = S v   (rows over waves)
        for (int r = gw; r < m; r += nw) {
            double acc = 0.0;
            for (int32_t e = rowptr[r] + lane; e < rowptr[r + 1]; e += 64) {
                const int32_t c = colidx[e];
                acc += (double)val[e] * ((in_lds ? vl[c] : ld_agent(wp + c)) * inv);
            }
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) st_agent(tvec + r, acc);
        }
        if (!grid_barrier_coherent(counter, (++bar) * P, scal)) return;
        // w = S^T t  (columns over waves), rows ascending within a column
        double mu_part = 0.0, w2_part = 0.0;
        for (int c = gw; c < n; c += nw) {
            double acc = 0.0;
            for (int32_t p = colptr[c] + lane; p < colptr[c + 1]; p += 64) acc += (double)val[csrc[p]] * ld_agent(tvec + crow[p]);
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) {
                st_agent(wn + c, acc);
                mu_part += ((in_lds ? vl[c] : ld_agent(wp + c)) * inv) * acc;
                w2_part += acc * acc;
            }
        }
        mu_part = block_sum(mu_part, red);
        w2_part = block_sum(w2_part, red);
        double* pt = part + (t & 1) * 2 * P;
        if (threadIdx.x == 0) {
            st_agent(pt + blockIdx.x, mu_part);
            st_agent(pt + P + blockIdx.x, w2_part);
        }
        if (!grid_barrier_coherent(counter, (++bar) * P, scal)) return;
        double smu = 0.0, sw2 = 0.0;
        for (int i = threadIdx.x; i < P; i += kPowerThreads) {
            smu += ld_agent(pt + i);
            sw2 += ld_agent(pt + P + i);
        }
        const double mu = block_sum(smu, red);
        const double w2 = block_sum(sw2, red);
        if (threadIdx.x == 0) {
            bcast[0] = mu;
            bcast[1] = w2;
            if (blockIdx.x == 0) {
                scal[pw_mu + t] = mu;
                scal[pw_w2 + t] = w2;
            }
        }
        __syncthreads();
        const double mu_t = bcast[0], w2_t = bcast[1];
        __syncthreads();
        if (!(w2_t > 0.0)) {
            vanish = 1;
            break;
        }
        if (t >= 2 && fabs(mu_t - muprev) <= tol * mu_t) {
            stop = t;
            break;
        }
        muprev = mu_t;
        w2prev = w2_t;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[SC_STOP] = stop ? stop : (vanish ? 0 : maxit);
        scal[SC_VANISH] = vanish;
    }
}

// k-step Lanczos on S^T S through two sparse products per step, the operator
// form's counterpart of lanczos_coop_kernel (n <= kPowerVecLds): in step j
//   t = S q_j (rows over waves, q_j in LDS), stored with agent scope; grid barrier;
//   u_c = (S^T t)_c - beta_{j-1} q_{j-1,c} for each wave's columns (rows ascending
//   within a column), stored with q_{j,c}, and q_{j,c} u_c into the workgroup's
//   alpha partial; grid barrier;
//   every workgroup adds the partials in a fixed order (alpha_j), loads all of u,
//   forms u - alpha_j q_j and ||.||^2 over the n entries itself (the same
//   operations in every workgroup) and keeps q_{j+1} = u / beta_j in LDS.
// The Ritz pair, the stop and the result slots as in lanczos_coop_kernel; entry c
// of the Ritz vector is formed by the thread that stored Q[.][c].  Q holds
// steps + 2 vectors of n: the Lanczos vectors, then U by step parity.
__global__ void __launch_bounds__(kPowerThreads) lanczos_op_kernel(int m, int n, const int32_t* rowptr,
                                                                   const int32_t* colidx, const float* val,
                                                                   const int32_t* colptr, const int32_t* crow,
                                                                   const int32_t* csrc, double* tvec, double* wb0,
                                                                   double* wb1, double* Q, double* part,
                                                                   unsigned* counter, double* scal, int steps,
                                                                   double tol, int pw_mu, int pw_w2) {
    __shared__ double red[kPowerThreads / 64];
    __shared__ double rz[3][kLzSlot];   // Ritz pairs: by step parity, then the final one
    __shared__ __attribute__((aligned(16))) double va[kPowerVecLds];
    __shared__ __attribute__((aligned(16))) double vb[kPowerVecLds];
    const int P = gridDim.x;
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (kPowerThreads / 64) + (threadIdx.x >> 6);
    const int nw = P * (kPowerThreads / 64);
    const double n0 = scal[pw_w2 + 0];
    if (!(n0 > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[SC_STOP] = 0;
            scal[SC_VANISH] = 1;
        }
        return;
    }
    const double inv0 = 1.0 / sqrt(n0);
    for (int i = threadIdx.x; i < n; i += kPowerThreads) {
        va[i] = wb0[i] * inv0;   // q_1
        vb[i] = 0.0;             // q_0
    }
    __syncthreads();
    double* vq = va;   // q_j
    double* vp = vb;   // q_{j-1}, then u
    double bprev = 0.0;
    double al = 0.0, be = 0.0, th_prev = 0.0;
    int k = 0, vanish = 0, slot = -1;
    unsigned bar = 0;
    for (int j = 0; j < steps; ++j) {
        const int par = j & 1;
        double* U = Q + (int64_t)(steps + par) * n;
        // t = S q_j
        for (int r = gw; r < m; r += nw) {
            double acc = 0.0;
            for (int32_t e = rowptr[r] + lane; e < rowptr[r + 1]; e += 64) acc += (double)val[e] * vq[colidx[e]];
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) st_agent(tvec + r, acc);
        }
        if (!grid_barrier_coherent(counter, (++bar) * P, scal)) return;
        // u = S^T t - beta_{j-1} q_{j-1} on this wave's columns
        double apart = 0.0;
        for (int c = gw; c < n; c += nw) {
            double acc = 0.0;
            for (int32_t p = colptr[c] + lane; p < colptr[c + 1]; p += 64)
                acc += (double)val[csrc[p]] * ld_agent(tvec + crow[p]);
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) {
                const double uc = acc - bprev * vp[c];
                st_agent(U + c, uc);
                st_agent(Q + (int64_t)j * n + c, vq[c]);
                apart += vq[c] * uc;
            }
        }
        apart = block_sum(apart, red);
        double* pt = part + par * 2 * P;
        if (threadIdx.x == 0) st_agent(pt + blockIdx.x, apart);
        if (!grid_barrier_coherent(counter, (++bar) * P, scal)) return;
        double sa = 0.0;
        for (int p = threadIdx.x; p < P; p += kPowerThreads) sa += ld_agent(pt + p);
        const double alpha = block_sum(sa, red);
        // u - alpha q_j over all n entries, into vp (q_{j-1} is no longer needed)
        double b2 = 0.0;
        for (int i = threadIdx.x; i < n; i += kPowerThreads) {
            const double ui = ld_agent(U + i) - alpha * vq[i];
            vp[i] = ui;
            b2 += ui * ui;
        }
        const double beta = sqrt(block_sum(b2, red));
        if (lane == j) {
            al = alpha;
            be = beta;
        }
        k = j + 1;
        if (j == 0 && alpha == 0.0 && beta == 0.0) {
            vanish = 1;
            break;
        }
        if (beta == 0.0) break;
        if (tol > 0.0) {
            // the Ritz pair of T_{j+1}; kept when the run ends here
            if (threadIdx.x < 64) {
                double theta, resid, sv;
                lz_ritz(al, be, k, theta, resid, sv);
                const bool stop = j >= 1 && fabs(theta - th_prev) <= tol * theta;
                th_prev = theta;
                if (lane < k) rz[par][lane] = sv;
                if (lane == 0) {
                    rz[par][kLanczosMax] = theta;
                    rz[par][kLanczosMax + 1] = resid;
                    rz[par][kLanczosMax + 2] = stop ? 1.0 : 0.0;
                }
            }
            __syncthreads();
            if (rz[par][kLanczosMax + 2] != 0.0) {
                slot = par;
                break;
            }
        }
        // q_{j+1} = u / beta; the roles of the two LDS vectors swap
        const double ib = 1.0 / beta;
        for (int i = threadIdx.x; i < n; i += kPowerThreads) vp[i] *= ib;
        __syncthreads();
        double* t = vq;
        vq = vp;
        vp = t;
        bprev = beta;
    }
    if (vanish) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[SC_STOP] = 0;
            scal[SC_VANISH] = 1;
        }
        return;
    }
    if (slot < 0) {
        // the Ritz pair of T_k
        slot = 2;
        if (threadIdx.x < 64) {
            double theta, resid, sv;
            lz_ritz(al, be, k, theta, resid, sv);
            if (lane < k) rz[2][lane] = sv;
            if (lane == 0) {
                rz[2][kLanczosMax] = theta;
                rz[2][kLanczosMax + 1] = resid;
            }
        }
        __syncthreads();
    }
    // the Ritz vector: entry c from the stores of the thread that owns column c
    double* yb = ((k - 1) & 1) ? wb1 : wb0;
    if (lane == 0) {
        for (int c = gw; c < n; c += nw) {
            double y = 0.0;
            for (int q = 0; q < k; ++q) y += rz[slot][q] * Q[(int64_t)q * n + c];
            yb[c] = y;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double theta = rz[slot][kLanczosMax], resid = rz[slot][kLanczosMax + 1];
        scal[pw_mu + k] = theta;
        scal[pw_w2 + k] = theta * theta + resid * resid;
        scal[pw_w2 + k - 1] = 1.0;
        scal[SC_STOP] = k;
        scal[SC_VANISH] = 0;
    }
}

// SVT update on the observed set (values in CSR order):
//   r_e = M_e - X[row(e)][col(e)],  Yv_e += delta r_e,  partial sums of r^2.
__global__ void svt_update_kernel(int m, const int32_t* rowptr, const int32_t* colidx, const float* Mv,
                                  const float* X, int64_t ldx, float* Yv, float delta, double* part) {
    __shared__ double red[16];
    double s = 0.0;
    for (int r = blockIdx.x; r < m; r += gridDim.x)
        for (int32_t e = rowptr[r] + threadIdx.x; e < rowptr[r + 1]; e += blockDim.x) {
            const float res = Mv[e] - X[(int64_t)r * ldx + colidx[e]];
            Yv[e] += delta * res;
            s += (double)res * res;
        }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// resid[t] = sqrt(sum part) / norm_M (fixed order), single workgroup.
__global__ void svt_resid_kernel(const double* part, int np, double normM, double* resid_out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0 && resid_out) *resid_out = normM > 0.0 ? sqrt(s) / normM : 0.0;
}

// ---- the matrix-polynomial route without the densified S -----------------------
//
// sp_gram_kernel   G = S^T S by rows of S: row i of G is the sum, over the rows r
//                  of column i of S, of s_ri times row r of S (nnz_r entries), i.e.
//                  sum_r nnz_r^2 products instead of the 2 nnz n of a product with
//                  the densified S.  One workgroup per row i of G; the column's
//                  rows are split into SPG_WAVES contiguous runs, each wave adds its
//                  run's scaled rows in ascending row order into its own LDS copy of
//                  the output row (the entries of one row of S have distinct
//                  columns, so the lanes' read-modify-writes never collide) and the
//                  copies are added in wave order: the sum order is fixed.
// sp_sddmm_kernel  the observed entries of S p, (S p)[r][c] for (r, c) in the
//                  pattern: the sum over row r of S of s_rk p[c][k] -- row c of p,
//                  as the dense route's last product reads p (p is a polynomial in
//                  the symmetric Gram, so p = p^T in exact arithmetic).  One
//                  workgroup per column c with row c of p staged in LDS; the
//                  column's rows go four to a wave (16 lanes each), partial sums
//                  added by xor shuffles.  Output in CSR order (through csrc).
constexpr int SPG_WAVES = 2;
constexpr int SPS_WAVES = 4;
constexpr int SPG_MAXN = 4096;   // the LDS rows of both kernels hold n floats

__global__ void __launch_bounds__(64 * SPG_WAVES) sp_gram_kernel(int n, const int32_t* colptr, const int32_t* crow,
                                                                 const float* cval, const int32_t* rowptr,
                                                                 const int32_t* colidx, const float* val, float* G,
                                                                 int64_t ldg) {
    __shared__ float acc[SPG_WAVES][SPG_MAXN];
    const int i = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* a_row = acc[wave];
    for (int j = lane; j < n; j += 64) a_row[j] = 0.f;
    const int32_t b = colptr[i], len = colptr[i + 1] - b;
    const int32_t chunk = (len + SPG_WAVES - 1) / SPG_WAVES;
    const int32_t lo = b + min(len, wave * chunk), hi = b + min(len, (wave + 1) * chunk);
    for (int32_t p0 = lo; p0 < hi; p0 += 64) {
        const int cnt = min(64, hi - p0);
        // lane l holds the scale and the extent of the batch's row l
        float a_l = 0.f;
        int32_t rb_l = 0, re_l = 0;
        if (lane < cnt) {
            const int32_t r = crow[p0 + lane];
            a_l = cval[p0 + lane];
            rb_l = rowptr[r];
            re_l = rowptr[r + 1];
        }
        // the first 128 entries of the next row are loaded while the current one is added
        int32_t rb = __shfl(rb_l, 0, 64), re = __shfl(re_l, 0, 64);
        int32_t c0 = 0, c1 = 0;
        float v0 = 0.f, v1 = 0.f;
        if (rb + lane < re) { c0 = colidx[rb + lane]; v0 = val[rb + lane]; }
        if (rb + 64 + lane < re) { c1 = colidx[rb + 64 + lane]; v1 = val[rb + 64 + lane]; }
        for (int q = 0; q < cnt; ++q) {
            const float a = __shfl(a_l, q, 64);
            const int32_t qb = rb, qe = re;
            const int32_t qc0 = c0, qc1 = c1;
            const float qv0 = v0, qv1 = v1;
            if (q + 1 < cnt) {
                rb = __shfl(rb_l, q + 1, 64);
                re = __shfl(re_l, q + 1, 64);
                c0 = c1 = 0;
                v0 = v1 = 0.f;
                if (rb + lane < re) { c0 = colidx[rb + lane]; v0 = val[rb + lane]; }
                if (rb + 64 + lane < re) { c1 = colidx[rb + 64 + lane]; v1 = val[rb + 64 + lane]; }
            }
            if (qb + lane < qe) a_row[qc0] += a * qv0;
            if (qb + 64 + lane < qe) a_row[qc1] += a * qv1;
            for (int32_t e = qb + 128 + lane; e < qe; e += 64) a_row[colidx[e]] += a * val[e];
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += 64 * SPG_WAVES) {
        float sum = acc[0][j];
        for (int w = 1; w < SPG_WAVES; ++w) sum += acc[w][j];
        G[(int64_t)i * ldg + j] = sum;
    }
}

__global__ void __launch_bounds__(64 * SPS_WAVES) sp_sddmm_kernel(int n, const int32_t* colptr, const int32_t* crow,
                                                                  const int32_t* csrc, const int32_t* rowptr,
                                                                  const int32_t* colidx, const float* val,
                                                                  const float* F, int64_t ldf, float* out) {
    __shared__ float fr[SPG_MAXN];
    const int c = blockIdx.x;
    for (int j = threadIdx.x; j < n; j += 64 * SPS_WAVES) fr[j] = F[(int64_t)c * ldf + j];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, q = lane & 15;
    const int32_t b = colptr[c], end = colptr[c + 1];
    for (int32_t base = b + 4 * wave; base < end; base += 4 * SPS_WAVES) {
        const int32_t p = base + g;
        const bool valid = p < end;
        float sum = 0.f;
        if (valid) {
            const int32_t r = crow[p];
            const int32_t re = rowptr[r + 1];
            for (int32_t e = rowptr[r] + q; e < re; e += 16) sum += val[e] * fr[colidx[e]];
        }
        sum += __shfl_xor(sum, 8, 64);
        sum += __shfl_xor(sum, 4, 64);
        sum += __shfl_xor(sum, 2, 64);
        sum += __shfl_xor(sum, 1, 64);
        if (valid && q == 0) out[csrc[p]] = sum;
    }
}

// SVT update from the observed values of X (CSR order): r_e = M_e - Xv_e,
// Yv_e += delta r_e, per-workgroup partial sums of r^2 (grid-stride, fixed grid).
__global__ void svt_update_vals_kernel(int64_t nnz, const float* Mv, const float* Xv, float* Yv, float delta,
                                       double* part) {
    __shared__ double red[16];
    double s = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const float res = Mv[e] - Xv[e];
        Yv[e] += delta * res;
        s += (double)res * res;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// dst[t] = src[0] (the bound of an iteration copied into a caller's history).
__global__ void copy_f64_kernel(const double* src, double* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

__global__ void scale_vals_kernel(int64_t nnz, const float* src, float* dst, float f) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = f * src[e];
}

}  // namespace cpa
