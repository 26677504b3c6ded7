// Batched shrinkage of many small matrices in one persistent launch.
//
// Each matrix X_j (m_j x n_j, row-major at X + off_j) is shrunk by Algorithm 1
// (T = Id) in the Y-form, entirely inside one workgroup:
//   Z = X_j viewed so that its short side is first: Z = X_j when m_j <= n_j,
//       Z = X_j^T otherwise (d = min(m_j, n_j) <= 64 rows, e = max <= 128 columns);
//   Gram G = Z Z^T (d x d) with MFMA, ||G||_F^2 in FP64;
//   bound: power iteration or k-step Lanczos on G in LDS (FP64), Lambda given,
//       (1+delta)||G||_F, or the learned predictor (features of G -> perceptron ->
//       Lambda and K_j);
//   coefficients c_k in FP64 (eq. chebychev_coeff_shifted);
//   Y_0 = Z, Y_1 = Ghat Y_0, Y_{k+1} = 2 Ghat Y_k - Y_{k-1}, out = sum c_k Y_k with
//   Ghat = (2/Lambda) G - I fused as (2/Lambda) G Y - Y.
// With the growth check on, ||Y_{K-1}||_F <= (1 + tol) ||X||_F is tested after
// the recurrence (for eigenvalues inside [0, Lambda] every |T_k| <= 1, and above
// Lambda T_k grows with k, so the last Y_k is the largest); on failure the
// matrix is redone once with a safer bound (predictor -> power iteration,
// power or given -> Frobenius).
// Workgroups take matrix indices from an atomic counter until the batch is
// exhausted (every wave reaches the exit).
//
// Split-precision variant (SPLIT = true): each recurrence product G Y_k runs as
// G_hi Y_hi + G_hi Y_lo + G_lo Y_hi on the BF16 matrix cores (16x16x32, FP32
// accumulation, hi = bf16(x), lo = bf16(x - hi) rounded to nearest even); the
// rows of G this lane supplies are split once per matrix and kept in registers,
// and every element of Y_k is split once, by the thread that produced it, into
// bf16 hi / lo planes that replace the FP32 copy in LDS (row j: hi of the 64
// contraction entries, then lo).  The Gram, the bound and the coefficients stay
// FP32 / FP64, and the recurrence values themselves stay FP32 in registers.
//
// LDS: Y_k is kept transposed, YT[j][i] (j < e, i < d, k contiguous), so that
// both MFMA operands (G rows and YT rows) are 16-byte reads along the
// contraction index and a thread's own output positions are contiguous.  Y_k,
// Y_{k-1} and the accumulator also live in the registers of the thread that owns
// the positions (the MFMA output layout is the same at every step); the LDS
// copy of Y_k is only the operand of the next product.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_bf16x3.hpp"
#include "gemm_f32.hpp"
#include "mlp.hpp"
#include "shrink_fn.hpp"
#include "spectral.hpp"

namespace cpa {

constexpr int BT_THREADS = 256;       // 4 waves
constexpr int BT_DMAX = 64;           // short side
constexpr int BT_EMAX = 128;          // long side
constexpr int BT_DP = BT_DMAX + 4;    // LDS pitch (floats) of G and YT rows
constexpr int BT_JB = BT_EMAX / 16;   // column blocks per wave (each wave owns one row block)

// Device mirror of cpa_shrinkage (same layout).
struct ShrinkRec {
    int32_t kind;
    int32_t reserved;
    double tau, w_c, w_sigma, w_eps;
};

struct BatchArgs {
    int batch;
    const int32_t* m;
    const int32_t* n;
    const int64_t* off;
    const float* X;
    float* Y;
    const ShrinkRec* shrink;   // per matrix, or nullptr
    ShrinkParams shrink0;      // used when shrink == nullptr
    int K;                     // order (the maximum order in mode 3)
    int mode;                  // 0 power, 1 given, 2 Frobenius, 3 predictor, 4 features only
    const double* lambda_in;   // mode 1
    double* lambda_out;        // nullable
    int32_t* status;           // nullable: 0 done, 1 redone with the fallback bound,
                               //           2 shape unsupported, 3 growth check failed at the last bound
    float* feat_out;           // nullable: 3 features per matrix
    const float* model;        // mode 3: predictor model
    int K_min;                 // mode 3: smallest order
    int32_t* K_out;            // nullable: order used
    int check;                 // growth check on/off
    double growth_tol;
    int power_iters;
    int lanczos;               // mode 0: 0 power iteration, > 0 Lanczos steps
    double tol, margin;
    uint64_t seed;
    int* queue;                // next queue position (zeroed before launch)
    const int32_t* order;      // nullable: matrix index of every queue position
};

typedef unsigned short bt_u16x8 __attribute__((ext_vector_type(8)));

// Eight consecutive floats -> bf16 hi and lo parts (round to nearest even).
__device__ inline void bt_split8(const float* p, bf16x8& hi, bf16x8& lo) {
    const f32x4 a = *reinterpret_cast<const f32x4*>(p);
    const f32x4 b = *reinterpret_cast<const f32x4*>(p + 4);
    bt_u16x8 h, l;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        unsigned short x, y;
        split2(a[e], x, y);
        h[e] = x;
        l[e] = y;
        split2(b[e], x, y);
        h[e + 4] = x;
        l[e + 4] = y;
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

// Split rows of the bf16 planes: row j holds hi of entries 0..63, then lo.
constexpr int BT_BP = 2 * BT_DP;   // row pitch in bf16 elements (same bytes as an FP32 row)

// Four consecutive entries (i0 .. i0 + 3 of row j) -> the hi and lo planes.
__device__ inline void bt_store_split4(unsigned short* YB, int j, int i0, const f32x4& v) {
    unsigned short h[4], l[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) split2(v[r], h[r], l[r]);
    uint2 hh, ll;
    hh.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
    hh.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
    ll.x = (unsigned)l[0] | ((unsigned)l[1] << 16);
    ll.y = (unsigned)l[2] | ((unsigned)l[3] << 16);
    *reinterpret_cast<uint2*>(YB + j * BT_BP + i0) = hh;
    *reinterpret_cast<uint2*>(YB + j * BT_BP + BT_DMAX + i0) = ll;
}

// Value of v held by lane l (l uniform across the wave).
__device__ inline double bt_readlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// v of the lane selected by the DPP pattern CTRL (within rows of 16 lanes).
template <int CTRL>
__device__ inline double bt_dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes, equal in every lane.  Within each row of 16 lanes:
// swap neighbours, swap pairs, mirror halves of 8, mirror the row -- each step
// adds the same two values in either order, so all lanes of a row end with the
// same bits; the four row sums are then read from lanes 0, 16, 32, 48 and added
// in a fixed order.  VALU data movement only (no LDS round trips).
__device__ inline double bt_wave_sum(double v) {
    v += bt_dpp<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += bt_dpp<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += bt_dpp<0x141>(v);   // row_half_mirror
    v += bt_dpp<0x140>(v);   // row_mirror
    return (bt_readlane(v, 0) + bt_readlane(v, 16)) + (bt_readlane(v, 32) + bt_readlane(v, 48));
}

// Two independent wave sums with their steps interleaved (same operations and
// order as bt_wave_sum on each value).
__device__ inline void bt_wave_sum2(double& a, double& b) {
    a += bt_dpp<0xB1>(a);
    b += bt_dpp<0xB1>(b);
    a += bt_dpp<0x4E>(a);
    b += bt_dpp<0x4E>(b);
    a += bt_dpp<0x141>(a);
    b += bt_dpp<0x141>(b);
    a += bt_dpp<0x140>(a);
    b += bt_dpp<0x140>(b);
    a = (bt_readlane(a, 0) + bt_readlane(a, 16)) + (bt_readlane(a, 32) + bt_readlane(a, 48));
    b = (bt_readlane(b, 0) + bt_readlane(b, 16)) + (bt_readlane(b, 32) + bt_readlane(b, 48));
}

// 1 / sqrt(x) for a positive FP64 x: the hardware estimate refined by two
// Newton steps y <- y (3 - x y^2) / 2 (a few ulp) inside [2^-1000, 2^1000], the
// correctly rounded quotient outside that range.  Only the length of the
// normalised iterate depends on it, never its direction.
__device__ inline double bt_rsqrt(double x) {
    if (x > 0x1p-1000 && x < 0x1p1000) {
        double y = __builtin_amdgcn_rsq(x);
        const double hx = 0.5 * x;
        y = y * (1.5 - hx * y * y);
        y = y * (1.5 - hx * y * y);
        return y;
    }
    return 1.0 / sqrt(x);
}

__device__ inline double bt_block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// Recurrence product of NBLK adjacent 16 x 16 output blocks (column blocks
// jb0 .. jb0 + NBLK - 1 of this wave's row block): the blocks' MFMA chains are
// independent and issued interleaved, so one block's LDS reads and MFMA latency
// overlap the others' work.  Blocks past the matrix's last column read the zero
// padding of YT and produce zeros.
template <bool SPLIT, int NBLK>
__device__ inline void bt_product(const float* YT, int jb0, int lane, const float (&fa)[16], const bf16x8 (&gah)[2],
                                  const bf16x8 (&gal)[2], f32x4 (&acc)[NBLK]) {
    const int g = lane >> 4;
    const float* row[NBLK];
#pragma unroll
    for (int u = 0; u < NBLK; ++u) {
        row[u] = &YT[((jb0 + u) * 16 + (lane & 15)) * BT_DP + 16 * g];
        acc[u] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
    if (SPLIT) {
        const unsigned short* YB = reinterpret_cast<const unsigned short*>(YT);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            bf16x8 yh[NBLK], yl[NBLK];
#pragma unroll
            for (int u = 0; u < NBLK; ++u) {
                const unsigned short* rb = YB + ((jb0 + u) * 16 + (lane & 15)) * BT_BP + 16 * g + 8 * b;
                yh[u] = *reinterpret_cast<const bf16x8*>(rb);
                yl[u] = *reinterpret_cast<const bf16x8*>(rb + BT_DMAX);
            }
#pragma unroll
            for (int u = 0; u < NBLK; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gal[b], yh[u], acc[u], 0, 0, 0);
#pragma unroll
            for (int u = 0; u < NBLK; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gah[b], yl[u], acc[u], 0, 0, 0);
#pragma unroll
            for (int u = 0; u < NBLK; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gah[b], yh[u], acc[u], 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 16; q += 4) {
            f32x4 bv[NBLK];
#pragma unroll
            for (int u = 0; u < NBLK; ++u) bv[u] = *reinterpret_cast<const f32x4*>(row[u] + q);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int u = 0; u < NBLK; ++u)
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[q + r], bv[u][r], acc[u], 0, 0, 0);
        }
    }
}

// Two workgroups per CU (the register budget is capped accordingly): one
// matrix's barriers and power iteration overlap another's recurrence.
// PAIR: recurrence output blocks per MFMA group (1 or 2; a tuning choice, the
// results are the same bits either way: every block's products and adds run
// in the same order).
template <bool SPLIT, int PAIR>
__global__ void __launch_bounds__(BT_THREADS, 2) batched_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) float YT[BT_EMAX * BT_DP];
    __shared__ __attribute__((aligned(16))) float Gs[BT_DMAX * BT_DP];
    __shared__ double vv[BT_DMAX], coef[64], red[4];   // vv: scratch of the predictor network
    __shared__ double ctab[4 * 64], hval[64];            // coefficient tables (K <= 64)
    __shared__ double pw[2 * BT_THREADS];                 // power iteration: partial rows, by parity
    __shared__ int s_idx;
    __shared__ double s_scal[4];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;   // = row block of this wave
    const int g = lane >> 4;
    f32x4 yprev[BT_JB], ycur[BT_JB], outv[BT_JB];

    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(a.queue, 1);
        __syncthreads();
        const int qpos = s_idx;
        __syncthreads();
        if (qpos >= a.batch) break;
        const int idx = a.order ? a.order[qpos] : qpos;

        const int mj = a.m[idx], nj = a.n[idx];
        const bool trans = mj > nj;              // Z = X^T
        const int d = trans ? nj : mj, e = trans ? mj : nj;
        if (d < 1 || d > BT_DMAX || e > BT_EMAX) {
            if (threadIdx.x == 0 && a.status) a.status[idx] = 2;
            continue;
        }
        const float* X = a.X + a.off[idx];
        float* Yo = a.Y + a.off[idx];
        ShrinkParams sp = a.shrink0;
        if (a.shrink) {
            const ShrinkRec r = a.shrink[idx];
            sp.kind = r.kind;
            sp.tau = r.tau;
            sp.w_c = r.w_c;
            sp.w_sigma = r.w_sigma;
            sp.w_eps = r.w_eps;
        }

        auto load_z = [&]() {
            // YT[j][i] = Z[i][j], zero padding up to 128 x 64.  Threads walk X in its
            // own row-major order (consecutive threads, consecutive addresses) over a
            // padded view of 128 x 64 (X = Z^T: YT's rows are X's rows) or 64 x 128
            // (X = Z: X's rows become YT's columns), eight loads in flight per thread
            const int lc = trans ? 6 : 7;
            for (int p0 = threadIdx.x; p0 < BT_EMAX * BT_DMAX; p0 += 8 * BT_THREADS) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int p = p0 + u * BT_THREADS;
                    const int row = p >> lc, col = p & ((1 << lc) - 1);
                    v[u] = (row < mj && col < nj) ? X[(int64_t)row * nj + col] : 0.f;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int p = p0 + u * BT_THREADS;
                    const int row = p >> lc, col = p & ((1 << lc) - 1);
                    YT[trans ? row * BT_DP + col : col * BT_DP + row] = v[u];
                }
            }
            __syncthreads();
        };
        load_z();

        // ---- Gram G[i][i'] = sum_j YT[j][i] YT[j][i'] (MFMA, k = j), wave = row block
        const int ib = wave * 16;
        double fro2 = 0.0, tr = 0.0;
        {
            // the four column blocks as independent chains; the contraction stops at e
            // rounded up to 4 (YT rows past e are zero)
            f32x4 acc[4];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) acc[jb] = (f32x4){0.f, 0.f, 0.f, 0.f};
            const int kend = (e + 3) & ~3;
            for (int k0 = 0; k0 < kend; k0 += 4) {
                const float* yr = &YT[(k0 + g) * BT_DP + (lane & 15)];
                const float av = yr[ib];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) acc[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, yr[jb * 16], acc[jb], 0, 0, 0);
            }
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = ib + 4 * g + r, j = jb * 16 + (lane & 15);
                    Gs[i * BT_DP + j] = acc[jb][r];
                    fro2 += (double)acc[jb][r] * acc[jb][r];
                    if (i == j) tr += (double)acc[jb][r];
                }
            }
        }
        fro2 = bt_block_sum(fro2, red);
        tr = bt_block_sum(tr, red);
        const double fro = sqrt(fro2);
        // features: log ||X||_F (= log sqrt(tr Gram)), log ||Gram||_F^2, log(m n)
        const float f0 = (float)(0.5 * log(tr)), f1 = (float)log(fro2), f2 = (float)log((double)mj * (double)nj);
        if (a.feat_out && threadIdx.x == 0) {
            a.feat_out[3 * (int64_t)idx] = f0;
            a.feat_out[3 * (int64_t)idx + 1] = f1;
            a.feat_out[3 * (int64_t)idx + 2] = f2;
        }
        if (a.mode == 4) {
            if (threadIdx.x == 0 && a.status) a.status[idx] = 0;
            continue;
        }

        int mode = a.mode;
        int Kj = a.K;
        double Lam = 0.0;
        if (mode == 3) {
            if (fro > 0.0) {
                float y0, y1;
                mlp_infer_wg(a.model, f0, f1, f2, reinterpret_cast<float*>(vv), reinterpret_cast<float*>(s_scal), y0, y1);
                const double r = exp((double)(y0 < 0.f ? y0 : 0.f));   // Lambda <= (1 + margin) ||G||_F
                Lam = (1.0 + a.margin) * fro * r;
                const double kf = ceil(exp((double)y1));
                Kj = kf > (double)a.K ? a.K : (kf < (double)a.K_min ? a.K_min : (int)kf);
            } else {
                Kj = a.K_min;
            }
        }
        int status = 0;
        for (int attempt = 0;; ++attempt) {
            if (attempt > 0) load_z();
            // ---- bound
            if (mode == 1) {
                Lam = a.lambda_in[idx];
            } else if (mode == 2 || !(fro > 0.0)) {
                Lam = (1.0 + a.margin) * fro;
            } else if (mode == 0 && a.lanczos > 0) {
                // k-step Lanczos on G (the dense path's rule; the power branch's start
                // vector, layout and products): after each product's barrier every wave
                // forms u, alpha and beta alike, so the stop decisions agree; lane j keeps
                // alpha_j and beta_j for the Ritz pair (lz_ritz)
                double q = 0.0;
                if (lane < d) {
                    const uint64_t z = a.seed + (uint64_t)(lane + 1) * 0x9E3779B97F4A7C15ull;
                    uint64_t o = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                    o = (o ^ (o >> 27)) * 0x94D049BB133111EBull;
                    o ^= o >> 31;
                    q = 2.0 * ((double)(o >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
                }
                const double nv = bt_wave_sum(q * q);
                bool vanish = !(nv > 0.0);
                double al = 0.0, be = 0.0, theta = 0.0, r = 0.0, sv = 0.0, th_prev = 0.0;
                int k = 0;
                bool fresh = false;   // theta and r belong to T_k
                if (!vanish) {
                    q = q / sqrt(nv);
                    const int j0 = __builtin_amdgcn_readfirstlane(16 * wave);
                    f32x4 grow[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) grow[t] = *reinterpret_cast<const f32x4*>(&Gs[lane * BT_DP + j0 + 4 * t]);
                    double qprev = 0.0, bprev = 0.0;
                    const int steps = a.lanczos < d ? a.lanczos : d;
                    for (int j = 0; j < steps; ++j) {
                        double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int u = 0; u < 16; ++u) p4[u & 3] += (double)grow[u >> 2][u & 3] * bt_readlane(q, j0 + u);
                        double* pb = pw + (j & 1) * BT_THREADS;
                        pb[threadIdx.x] = (p4[0] + p4[1]) + (p4[2] + p4[3]);
                        __syncthreads();
                        double uu = ((pb[lane] + pb[64 + lane]) + (pb[128 + lane] + pb[192 + lane])) - bprev * qprev;
                        const double alpha = bt_wave_sum(q * uu);
                        uu -= alpha * q;
                        const double beta = sqrt(bt_wave_sum(uu * uu));
                        if (lane == j) {
                            al = alpha;
                            be = beta;
                        }
                        k = j + 1;
                        int stop = (j == 0 && alpha == 0.0 && beta == 0.0) ? 2 : (beta == 0.0 ? 1 : 0);
                        stop = __builtin_amdgcn_readfirstlane(stop);
                        if (stop == 2) {
                            vanish = true;
                            break;
                        }
                        fresh = false;
                        if (stop == 1) break;
                        if (a.tol > 0.0) {
                            // early stop: successive Ritz values within tol (same in every wave)
                            lz_ritz(al, be, k, theta, r, sv);
                            fresh = true;
                            if (j >= 1 && fabs(theta - th_prev) <= a.tol * theta) break;
                            th_prev = theta;
                        }
                        qprev = q;
                        q = uu / beta;
                        bprev = beta;
                    }
                }
                if (vanish) {
                    Lam = (1.0 + a.margin) * fro;
                } else {
                    if (!fresh) lz_ritz(al, be, k, theta, r, sv);
                    Lam = theta + (a.margin * theta > r ? a.margin * theta : r);
                    if (Lam > (1.0 + a.margin) * fro) Lam = (1.0 + a.margin) * fro;
                }
            } else if (mode == 0) {
                // power iteration on G (d x d), FP64, start vector as in the dense path.
                // Lane i owns row i; wave w adds the columns j in [16 w, 16 w + 16)
                // (four 16-byte reads of row i, conflict-free at pitch 68) with v_j
                // broadcast by readlane.  Rows and columns of G past d and entries of v
                // past d are zero, so every wave takes all 16 columns without a
                // bound test (the zero terms leave the sums unchanged); the four
                // partial rows meet in LDS
                // (one barrier per product, buffers alternating by parity), and every
                // wave then forms the same w, mu, ||w||^2 and stop decision: the
                // values are bitwise equal across lanes and waves (same operations on
                // the same data), and the stop flag goes through readfirstlane so the
                // loop exit is a scalar branch.
                double v = 0.0;
                if (lane < d) {
                    const uint64_t z = a.seed + (uint64_t)(lane + 1) * 0x9E3779B97F4A7C15ull;
                    uint64_t o = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                    o = (o ^ (o >> 27)) * 0x94D049BB133111EBull;
                    o ^= o >> 31;
                    v = 2.0 * ((double)(o >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
                }
                double nv = bt_wave_sum(v * v);
                double mu = 0.0, w2 = 0.0, muprev = 0.0;
                bool vanish = !(nv > 0.0);
                const int j0 = __builtin_amdgcn_readfirstlane(16 * wave);   // scalar lane base
                f32x4 grow[4];   // G[lane][j0 .. j0 + 15], fixed for the whole iteration
#pragma unroll
                for (int t = 0; t < 4; ++t) grow[t] = *reinterpret_cast<const f32x4*>(&Gs[lane * BT_DP + j0 + 4 * t]);
                for (int t = 1; !vanish && t <= a.power_iters; ++t) {
                    const double vs = v * bt_rsqrt(nv);
                    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int u = 0; u < 16; ++u) q[u & 3] += (double)grow[u >> 2][u & 3] * bt_readlane(vs, j0 + u);
                    double* pb = pw + (t & 1) * BT_THREADS;
                    pb[threadIdx.x] = (q[0] + q[1]) + (q[2] + q[3]);
                    __syncthreads();
                    const double wi = (pb[lane] + pb[64 + lane]) + (pb[128 + lane] + pb[192 + lane]);
                    mu = vs * wi;
                    w2 = wi * wi;
                    bt_wave_sum2(mu, w2);
                    int stop = !(w2 > 0.0) ? 2 : ((t >= 2 && fabs(mu - muprev) <= a.tol * mu) ? 1 : 0);
                    stop = __builtin_amdgcn_readfirstlane(stop);
                    if (stop == 2) {
                        vanish = true;
                        break;
                    }
                    if (stop == 1) break;
                    muprev = mu;
                    v = wi;
                    nv = w2;
                }
                if (vanish) {
                    Lam = (1.0 + a.margin) * fro;
                } else {
                    const double r2 = w2 - mu * mu;
                    const double r = sqrt(r2 > 0.0 ? r2 : 0.0);
                    Lam = mu + (a.margin * mu > r ? a.margin * mu : r);
                    if (Lam > (1.0 + a.margin) * fro) Lam = (1.0 + a.margin) * fro;
                }
            }

            // ---- coefficients (FP64, l ascending per k): k theta_l = pi k (2l + 1) / (2K)
            // takes only the 4K angles pi m / (2K), m = k (2l + 1) mod 4K, so their cosines
            // and the K values of h are formed once, in parallel, and each c_k sums its row
            __syncthreads();   // coef and the tables are rewritten on a second attempt
            {
                const double pi = 3.14159265358979323846;
                const int M4 = 4 * Kj;
                for (int q = threadIdx.x; q < M4; q += BT_THREADS) ctab[q] = cos(pi * q / (2.0 * Kj));
                for (int l = threadIdx.x; l < Kj; l += BT_THREADS)
                    hval[l] = Lam > 0.0 ? shrink_h(sp, 0.5 * Lam * (cos(pi * (l + 0.5) / Kj) + 1.0)) : 0.0;
                __syncthreads();
                for (int k = threadIdx.x; k < Kj; k += BT_THREADS) {
                    double acc = 0.0;
                    int idx = k;
                    const int step2 = (2 * k) % M4;
                    for (int l = 0; l < Kj; ++l) {
                        acc += ctab[idx] * hval[l];
                        idx += step2;
                        if (idx >= M4) idx -= M4;
                    }
                    coef[k] = Lam > 0.0 ? 2.0 / Kj * acc : 0.0;
                }
            }
            __syncthreads();
            const float a1 = Lam > 0.0 ? (float)(2.0 / Lam) : 0.f;
            const float a2 = Lam > 0.0 ? (float)(4.0 / Lam) : 0.f;

            // ---- recurrence: this wave owns row block ib and every column block jb
            const int nb = (e + 15) / 16;
            const float c0h = (float)(0.5 * coef[0]);
#pragma unroll
            for (int jb = 0; jb < BT_JB; ++jb) {
                // own positions (i = ib + 4g + r, j = jb*16 + lane%16): YT[j][ib + 4g .. +3]
                const int j = jb * 16 + (lane & 15);
                const f32x4 y0 = *reinterpret_cast<const f32x4*>(&YT[j * BT_DP + ib + 4 * g]);
                ycur[jb] = y0;
                outv[jb] = c0h * y0;
            }
            if (SPLIT) {
                // Y_0 into the bf16 planes (every FP32 entry has been read)
                __syncthreads();
#pragma unroll
                for (int jb = 0; jb < BT_JB; ++jb)
                    if (jb < nb)
                        bt_store_split4(reinterpret_cast<unsigned short*>(YT), jb * 16 + (lane & 15), ib + 4 * g, ycur[jb]);
                __syncthreads();
            }
            float last2 = 0.f;   // ||Y_{K-1}||^2 over this thread's positions
            // split precision: rows ib + lane%16 of G, k = 16 g + 8 b + 0..7, split once per matrix
            bf16x8 gah[2], gal[2];
            if (SPLIT) {
#pragma unroll
                for (int b = 0; b < 2; ++b) bt_split8(&Gs[(ib + (lane & 15)) * BT_DP + 16 * g + 8 * b], gah[b], gal[b]);
            }
            for (int step = 0; step + 1 < Kj; ++step) {
                const float aa = step == 0 ? a1 : a2;
                const float bb = step == 0 ? -1.f : -2.f;
                const float cc = step == 0 ? 0.f : -1.f;
                const float ck = (float)coef[step + 1];
                const bool final_step = step + 2 == Kj;
                // A fragments: G rows ib + lane%16, k = 16 g + kk
                float fa[16];
                if (!SPLIT) {
                    const float* row = &Gs[(ib + (lane & 15)) * BT_DP + 16 * g];
#pragma unroll
                    for (int q = 0; q < 16; q += 4) {
                        const f32x4 t = *reinterpret_cast<const f32x4*>(row + q);
                        fa[q] = t[0];
                        fa[q + 1] = t[1];
                        fa[q + 2] = t[2];
                        fa[q + 3] = t[3];
                    }
                }
                // three-term update of this thread's positions in block jb
                auto update = [&](int jb, const f32x4& acc) {
                    const f32x4 yk = ycur[jb];
                    f32x4 yn;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float y = aa * acc[r] + bb * yk[r];
                        if (step > 0) y += cc * yprev[jb][r];
                        yn[r] = y;
                        outv[jb][r] += ck * y;
                        if (final_step) last2 += y * y;
                    }
                    ycur[jb] = yn;
                    yprev[jb] = yk;
                };
                // column blocks in groups of PAIR (interleaved chains), a lone last block alone
#pragma unroll
                for (int jb = 0; jb < BT_JB; jb += PAIR) {
                    if (PAIR == 2 && jb + 1 < nb) {
                        f32x4 acc[2];
                        bt_product<SPLIT, 2>(YT, jb, lane, fa, gah, gal, acc);
                        update(jb, acc[0]);
                        update(jb + 1, acc[1]);
                    } else if (jb < nb) {
                        f32x4 acc[1];
                        bt_product<SPLIT, 1>(YT, jb, lane, fa, gah, gal, acc);
                        update(jb, acc[0]);
                    }
                }
                if (final_step) break;   // Y_{K-1} is not an operand
                __syncthreads();         // every wave has read Y_k
#pragma unroll
                for (int jb = 0; jb < BT_JB; ++jb) {
                    if (jb < nb) {
                        const int j = jb * 16 + (lane & 15);
                        if (SPLIT)
                            bt_store_split4(reinterpret_cast<unsigned short*>(YT), j, ib + 4 * g, ycur[jb]);
                        else
                            *reinterpret_cast<f32x4*>(&YT[j * BT_DP + ib + 4 * g]) = ycur[jb];
                    }
                }
                __syncthreads();
            }
            if (!a.check || Kj < 2) break;
            const double grow2 = bt_block_sum((double)last2, red);
            const double lim = (1.0 + a.growth_tol) * (1.0 + a.growth_tol) * tr;
            if (grow2 <= lim) break;
            if (attempt > 0 || mode == 2) {
                status = 3;
                break;
            }
            mode = mode == 3 ? 0 : 2;
            status = 1;
        }
        if (threadIdx.x == 0) {
            if (a.lambda_out) a.lambda_out[idx] = Lam;
            if (a.K_out) a.K_out[idx] = Kj;
            if (a.status) a.status[idx] = status;
        }

        // ---- store the accumulator (out(i, j) = Y_j[i][j], or Y_j[j][i] when transposed)
        {
            const int nb = (e + 15) / 16;
#pragma unroll
            for (int jb = 0; jb < BT_JB; ++jb) {
                if (jb < nb) {
                    const int j = jb * 16 + (lane & 15);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = ib + 4 * g + r;
                        if (i < d && j < e) {
                            if (trans)
                                Yo[(int64_t)j * nj + i] = outv[jb][r];
                            else
                                Yo[(int64_t)i * nj + j] = outv[jb][r];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace cpa
