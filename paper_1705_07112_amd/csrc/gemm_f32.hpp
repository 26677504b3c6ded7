// FP32 MFMA GEMM tile engine for the Gram (Algorithm 1, step 1 with T = Id) and
// the Chebyshev recurrence products (Algorithm 1, steps 8-10, distributed over
// X), with fused epilogues.
//
// C(i, j) = sum_k A(i, k) B(k, j),  0 <= i < M, 0 <= j < N, 0 <= k < Kd.
//
// Operand addressing (x is i for A, j for B):
//   XCONTIG  element (x, k) at p[k * ld + x]   (x runs contiguously)
//   KCONTIG  element (x, k) at p[x * ld + k]   (k runs contiguously)
// Each operand is staged through LDS in the layout that matches its global
// layout, so the global loads are 16-byte vectors and the LDS stores need no
// transposition.  The MFMA fragment reader adapts to the LDS layout instead:
// v_mfma_f32_16x16x4f32 takes A(i = lane%16, k = lane/16) and
// B(k = lane/16, j = lane%16); the contraction index seen by lane group
// g = lane/16 at sub-step kk is mapped to tile column k = 8 g + kk for both
// operands (any bijection is valid as long as A and B agree).  With that map a
// KCONTIG LDS row yields eight sub-steps of a lane in two 16-byte reads.
//
// Pipeline: K-tiles of 64, two LDS stages, MFMA fragments double-buffered in
// registers, global loads issued three tiles ahead (see the step description
// above the kernel).
// Workgroup: 8 waves (two per SIMD) in a 2 x 4 arrangement; each wave owns a
// (BM/2) x (BN/4) sub-tile of 16 x 16 MFMA blocks.
//
// Accuracy: each K-tile is accumulated into a fresh partial sum that is then
// added to the running sum with an FP32 add, instead of chaining all Kd
// products through one accumulator.  Chaining 1024 positive products grows the
// rounding error several-fold; the two-level sum keeps the 1024^3 recurrence
// inside the FP32 tolerance.  Two partial sets alternate so the add of tile t
// waits on MFMAs issued a whole tile earlier.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpa {

typedef float f32x4 __attribute__((ext_vector_type(4)));

enum Layout { XCONTIG = 0, KCONTIG = 1 };

#ifndef CPA_GEMM_BK
#define CPA_GEMM_BK 64
#endif
constexpr int GBK = CPA_GEMM_BK; // K-tile depth

// Keeps the compiler's scheduler from sinking the next tiles' global loads below
// the MFMA block that is meant to hide their latency.
#ifndef CPA_SCHED_FENCE
#define CPA_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
#endif

// Instruction-group order for one pipeline step: the LDS fragment reads of the
// next tile and the LDS stores are spread between the MFMAs of the current tile
// so the LDS traffic runs under the matrix-core work instead of in a burst
// before the barrier.  (sched_group_barrier masks: 0x8 MFMA, 0x100 DS read,
// 0x200 DS write.)
#ifndef CPA_READ_SHARE
#define CPA_READ_SHARE 2   // quarters of the step's MFMAs spread over the DS reads
#endif
template <int NMFMA, int NREAD, int NWRITE>
__device__ inline void interleave_step() {
    constexpr int per_read = (NMFMA * CPA_READ_SHARE / 4) / (NREAD > 0 ? NREAD : 1);
    constexpr int used_r = per_read * NREAD;
    constexpr int per_write = (NMFMA - used_r) / (NWRITE + 1);
#pragma unroll
    for (int i = 0; i < NREAD; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, per_read, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
#pragma unroll
    for (int i = 0; i < NWRITE; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, per_write, 0);
        __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, NMFMA - used_r - per_write * NWRITE, 0);
    // the partial-sum adds (VALU, mask 0x2) last: their inputs were produced a
    // whole step earlier, so they never wait on the matrix cores
    __builtin_amdgcn_sched_group_barrier(0x002, 1000, 0);
}
constexpr int GWAVES = 8;        // waves per workgroup (2 x 4)
constexpr int GTHREADS = 64 * GWAVES;
constexpr int KG = GBK / 4;      // sub-steps per lane group and K-tile

template <int BX, int L>
struct TileGeom {
    // LDS pitch (floats) and size of one buffer.
    static constexpr int pitch = (L == XCONTIG) ? (BX + 4) : (GBK + 4);
    static constexpr int rows = (L == XCONTIG) ? GBK : BX;
    static constexpr int size = rows * pitch;
    // float4 vectors per tile and per thread
    static constexpr int vecs = BX * GBK / 4;
    static constexpr int per_thread = vecs / GTHREADS;
    static_assert(per_thread >= 1 && vecs % GTHREADS == 0, "tile too small for the workgroup");
};

struct Operand {
    const float* p;
    int64_t ld;
    int xdim;     // M for A, N for B
};

// Loads the float4 groups of one tile (x0.., k0..) into registers; elements
// outside the matrix read as zero.  The instruction stream is the same for
// every tile: out-of-range groups load from a clamped in-range address and are
// zeroed by a select, so the K loop has no branches and the compiler can keep
// the next tiles' loads in flight across the LDS stores.
//   VEC: 16-byte loads; requires ld % 4 == 0, a 16-byte aligned base, and the
//        vectorised extent (xdim for XCONTIG, Kd for KCONTIG) % 4 == 0 and >= 4.
//   otherwise: four 4-byte loads per group with per-element clamping.
template <int BX, int L, bool VEC>
__device__ inline void tile_load(const Operand& op, int x0, int k0, int Kd, f32x4 (&r)[TileGeom<BX, L>::per_thread]) {
#pragma unroll
    for (int q = 0; q < TileGeom<BX, L>::per_thread; ++q) {
        const int f = threadIdx.x + q * GTHREADS;
        int gx, gk;
        if (L == XCONTIG) {
            gk = k0 + f / (BX / 4);
            gx = x0 + (f % (BX / 4)) * 4;
        } else {
            gx = x0 + f / (GBK / 4);
            gk = k0 + (f % (GBK / 4)) * 4;
        }
        // L == XCONTIG: the group runs along x; KCONTIG: along k
        const int lim_run = (L == XCONTIG) ? op.xdim : Kd;
        const int lim_fix = (L == XCONTIG) ? Kd : op.xdim;
        const int run = (L == XCONTIG) ? gx : gk;
        const int fix = (L == XCONTIG) ? gk : gx;
        const int fixc = fix < lim_fix ? fix : lim_fix - 1;
        const bool fix_ok = fix < lim_fix;
        if (VEC) {
            const bool ok = fix_ok && run < lim_run;
            const int runc = ok ? run : lim_run - 4;
            const float* src = (L == XCONTIG) ? op.p + (int64_t)fixc * op.ld + runc
                                              : op.p + (int64_t)fixc * op.ld + runc;
            const f32x4 v = *reinterpret_cast<const f32x4*>(src);
            const f32x4 z = {0.f, 0.f, 0.f, 0.f};
            r[q] = ok ? v : z;
        } else {
            f32x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool ok = fix_ok && run + e < lim_run;
                const int rc = (run + e < lim_run) ? run + e : lim_run - 1;
                const float t = op.p[(int64_t)fixc * op.ld + rc];
                v[e] = ok ? t : 0.f;
            }
            r[q] = v;
        }
    }
}

template <int BX, int L>
__device__ inline void tile_store(float* lds, const f32x4 (&r)[TileGeom<BX, L>::per_thread]) {
#pragma unroll
    for (int q = 0; q < TileGeom<BX, L>::per_thread; ++q) {
        const int f = threadIdx.x + q * GTHREADS;
        int off;
        if (L == XCONTIG) {
            off = (f / (BX / 4)) * TileGeom<BX, L>::pitch + (f % (BX / 4)) * 4;
        } else {
            off = (f / (GBK / 4)) * TileGeom<BX, L>::pitch + (f % (GBK / 4)) * 4;
        }
        *reinterpret_cast<f32x4*>(lds + off) = r[q];
    }
}

// The Q sub-step operands of one lane for the 16-row block starting at xb,
// sub-steps kk = koff .. koff + Q - 1 of the tile (tile column k = KG g + kk).
template <int BX, int L, int Q>
__device__ inline void frag_read(const float* lds, int xb, int lane, int koff, float (&v)[Q]) {
    const int xi = xb + (lane & 15);
    const int g = lane >> 4;
    if (L == XCONTIG) {
        constexpr int P = TileGeom<BX, L>::pitch;
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = lds[(KG * g + koff + q) * P + xi];
    } else {
        const float* row = lds + xi * TileGeom<BX, L>::pitch + KG * g + koff;
#pragma unroll
        for (int q = 0; q < Q; q += 4) {
            const f32x4 t = *reinterpret_cast<const f32x4*>(row + q);
            v[q] = t[0];
            v[q + 1] = t[1];
            v[q + 2] = t[2];
            v[q + 3] = t[3];
        }
    }
}

// Maps the hardware workgroup id to a tile so that the workgroups that share
// an XCD (dispatch is round-robin over 8 XCDs) cover a compact block of tiles
// and reuse their operand panels from that XCD's L2.
__device__ inline void tile_coords(int ntm, int ntn, int& tm, int& tn) {
    const int T = ntm * ntn;
    int t = blockIdx.x;
    if (T % 8 == 0) t = (t % 8) * (T / 8) + t / 8;
    constexpr int GM = 4;
    const int per_group = GM * ntn;
    const int grp = t / per_group;
    const int first = grp * GM;
    const int rows = min(GM, ntm - first);
    const int r = t % per_group;
    tm = first + r % rows;
    tn = r / rows;
}

// Upper-triangle tiles (tm <= tn) of a square product whose result is symmetric,
// in bands of GM tile rows: each band's tiles column by column (its first GM
// columns are triangular), bands in order; the XCD interleave of tile_coords is
// applied to the linear index first.  nt (nt + 1) / 2 workgroups.
__device__ inline void tile_coords_sym(int nt, int& tm, int& tn) {
    const int T = nt * (nt + 1) / 2;
    int t = blockIdx.x;
    if (T % 8 == 0) t = (t % 8) * (T / 8) + t / 8;
    constexpr int GM = 4;
    int first = 0;
    tm = tn = 0;
    while (first < nt) {
        const int rows = min(GM, nt - first);
        const int tri = rows * (rows + 1) / 2;
        const int cnt = tri + rows * (nt - first - rows);
        if (t < cnt) {
            if (t < tri) {
                int k = 0;
                while ((k + 1) * (k + 2) / 2 <= t) ++k;
                tn = first + k;
                tm = first + (t - k * (k + 1) / 2);
            } else {
                const int r = t - tri;
                tn = first + rows + r / rows;
                tm = first + r % rows;
            }
            return;
        }
        t -= cnt;
        first += rows;
    }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup of two values; the result is valid in thread 0.
__device__ inline void block_sum2(double& a, double& b) {
    __shared__ double red[2][GWAVES];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = a;
        red[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = 0.0;
        for (int i = 0; i < GWAVES; ++i) {
            a += red[0][i];
            b += red[1][i];
        }
    }
}

// block_sum2 for NW waves.
template <int NW>
__device__ inline void block_sum2_w(double& a, double& b) {
    __shared__ double red[2][NW];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = a;
        red[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = 0.0;
        for (int i = 0; i < NW; ++i) {
            a += red[0][i];
            b += red[1][i];
        }
    }
}

// Epilogues run after the K loop on a tile staged in LDS (row-major, pitch
// BN + 4), so that every thread handles whole float4 groups of a row: all
// global loads of a thread are issued before any arithmetic, and each wave
// reads and writes full 256-byte row segments.  `vec` says whether the
// operands allow 16-byte accesses (row pitches % 4 == 0, aligned bases, and
// the group lies inside the matrix); otherwise the group is handled per element.

// Gram: C = acc.  Each workgroup also stores its FP64 partial sums of C(i,j)^2
// and of the diagonal to part[2 * blockIdx.x] and part[2 * blockIdx.x + 1]; the
// bound kernel adds them in a fixed order (no atomics: a single address hit by
// every workgroup serialises in the memory system).
struct EpiGram {
    float* C;
    int64_t ldc;
    double* part;
    bool vec_ok;

    template <int BM, int BN, int NG>
    __device__ inline void run(const float* tile, int m0, int n0, int M, int N, const double*, int, int, int) const {
        constexpr int P = BN + 4, GPR = BN / 4;   // float4 groups per tile row
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int g = threadIdx.x + q * GTHREADS;
            const int r = g / GPR, c = (g % GPR) * 4;
            const int i = m0 + r, j = n0 + c;
            const f32x4 v = *reinterpret_cast<const f32x4*>(tile + r * P + c);
            if (i >= M) continue;
            if (vec_ok && j + 3 < N) {
                *reinterpret_cast<f32x4*>(C + (int64_t)i * ldc + j) = v;
            } else {
                for (int e = 0; e < 4; ++e)
                    if (j + e < N) C[(int64_t)i * ldc + j + e] = v[e];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (j + e < N) {
                    s1 += (double)v[e] * v[e];
                    if (i == j + e) s2 += v[e];
                }
            }
        }
        block_sum2(s1, s2);
        if (threadIdx.x == 0) {
            part[2 * blockIdx.x] = s1;
            part[2 * blockIdx.x + 1] = s2;
        }
    }

    // One piece of the Gram computed as a symmetric product (gemm_f32_piece_kernel,
    // 1024 threads; C % 16 bytes and ldc % 4 checked by the host): the piece and its
    // mirror are stored; the workgroup's partial sums count every stored entry once
    // (||G||_F^2 with the mirrored entries twice, the trace from the diagonal).
    __device__ inline void run_piece(float* tile, int m0, int n0, int half) const {
        constexpr int P = 68;
        const int t = threadIdx.x;
        double s1 = 0.0, s2 = 0.0;
        if (half < 0) {
            const int r = t / 16, cc = (t % 16) * 4;
            f32x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = cc + e;
                v[e] = r <= c ? tile[r * P + c] : tile[c * P + r];
                if (r <= c) s1 += (r == c ? 1.0 : 2.0) * (double)v[e] * v[e];
                if (r == c) s2 += v[e];
            }
            *reinterpret_cast<f32x4*>(C + (int64_t)(m0 + r) * ldc + n0 + cc) = v;
        } else {
            const int c0 = 32 * half;
            if (t < 512) {
                const int r = t / 8, cc = c0 + (t % 8) * 4;
                const f32x4 v = *reinterpret_cast<const f32x4*>(tile + r * P + cc);
                *reinterpret_cast<f32x4*>(C + (int64_t)(m0 + r) * ldc + n0 + cc) = v;
#pragma unroll
                for (int e = 0; e < 4; ++e) s1 += 2.0 * (double)v[e] * v[e];
                const int r2 = t / 16, c2 = (t % 16) * 4;
                f32x4 w;
#pragma unroll
                for (int e = 0; e < 4; ++e) w[e] = tile[(c2 + e) * P + c0 + r2];
                *reinterpret_cast<f32x4*>(C + (int64_t)(n0 + c0 + r2) * ldc + m0 + c2) = w;
            }
        }
        block_sum2_w<16>(s1, s2);
        if (t == 0) {
            part[2 * blockIdx.x] = s1;
            part[2 * blockIdx.x + 1] = s2;
        }
    }
};

// One recurrence step:
//   Ynew = a * acc + b * Yk + c * Yprev
//   first step:  out = c0/2 * Yk + c1 * Ynew      (Yk = X)
//   later steps: out += c_{k+1} * Ynew
//   Ynew is stored to Ydst unless this is the last step (Ydst may equal Yprev:
//   each element is read and then written by the same thread).
//   ||Ynew||_F^2 is accumulated for the growth check only when nrm2 is set: each
//   workgroup adds its partial to one of 64 slots (blockIdx % 64), which keeps
//   the atomics uncontended; the host adds the slots.
// The scalars are read from device memory, so a bound computed on the device
// is consumed without a host round trip.
struct EpiCheb {
    const float* Yk;
    int64_t ldk;
    const float* Yprev;
    int64_t ldp;
    float* Ydst;
    int64_t ldd;
    float* out;
    int64_t ldo;
    const double* scal;   // scalar block
    int step;             // k: this launch produces Y_{k+1}
    int last;
    double* nrm2;         // 64 slots for ||Y_{k+1}||^2, or nullptr
    bool vec_ok;

    template <int BM, int BN, int NG>
    __device__ inline void run(const float* tile, int m0, int n0, int M, int N, const double* sc, int sc_a1,
                               int sc_a2, int sc_coef) const {
        constexpr int P = BN + 4, GPR = BN / 4;
        float a, b, c, c0h;
        if (step == 0) {
            a = (float)sc[sc_a1];
            b = -1.f;
            c = 0.f;
            c0h = (float)(0.5 * sc[sc_coef]);
        } else {
            a = (float)sc[sc_a2];
            b = -2.f;
            c = -1.f;
            c0h = 0.f;
        }
        const float ck1 = (float)sc[sc_coef + step + 1];
        f32x4 vk[NG], vp[NG], vo[NG];
        bool full[NG];
        // issue every load first
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int g = threadIdx.x + q * GTHREADS;
            const int i = m0 + g / GPR, j = n0 + (g % GPR) * 4;
            full[q] = vec_ok && i < M && j + 3 < N;
            vk[q] = vp[q] = vo[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
            if (full[q]) {
                vk[q] = *reinterpret_cast<const f32x4*>(Yk + (int64_t)i * ldk + j);
                if (step > 0) {
                    vp[q] = *reinterpret_cast<const f32x4*>(Yprev + (int64_t)i * ldp + j);
                    vo[q] = *reinterpret_cast<const f32x4*>(out + (int64_t)i * ldo + j);
                }
            } else if (i < M) {
                for (int e = 0; e < 4; ++e) {
                    if (j + e < N) {
                        vk[q][e] = Yk[(int64_t)i * ldk + j + e];
                        if (step > 0) {
                            vp[q][e] = Yprev[(int64_t)i * ldp + j + e];
                            vo[q][e] = out[(int64_t)i * ldo + j + e];
                        }
                    }
                }
            }
        }
        double s1 = 0.0;
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int g = threadIdx.x + q * GTHREADS;
            const int r = g / GPR, cc = (g % GPR) * 4;
            const int i = m0 + r, j = n0 + cc;
            const f32x4 acc = *reinterpret_cast<const f32x4*>(tile + r * P + cc);
            f32x4 yn, o;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float y = a * acc[e] + b * vk[q][e];
                if (step > 0) y += c * vp[q][e];
                yn[e] = y;
                o[e] = (step == 0) ? c0h * vk[q][e] + ck1 * y : vo[q][e] + ck1 * y;
            }
            if (full[q]) {
                *reinterpret_cast<f32x4*>(out + (int64_t)i * ldo + j) = o;
                if (!last) *reinterpret_cast<f32x4*>(Ydst + (int64_t)i * ldd + j) = yn;
#pragma unroll
                for (int e = 0; e < 4; ++e) s1 += (double)yn[e] * yn[e];
            } else if (i < M) {
                for (int e = 0; e < 4; ++e) {
                    if (j + e < N) {
                        out[(int64_t)i * ldo + j + e] = o[e];
                        if (!last) Ydst[(int64_t)i * ldd + j + e] = yn[e];
                        s1 += (double)yn[e] * yn[e];
                    }
                }
            }
        }
        if (nrm2) {
            double unused = 0.0;
            block_sum2(s1, unused);
            if (threadIdx.x == 0 && s1 != 0.0) atomicAdd(nrm2 + (blockIdx.x & 63), s1);
        }
    }
};

// D = alpha acc + beta C + gamma Mx + delta I (the matrix polynomial steps):
// row-major D (pitch ldd), C (pitch ldc, read when beta != 0; may be D), Mx (pitch
// ldm, read when gamma != 0), I the identity (delta added where row == column).
struct EpiLin {
    float* D;
    int64_t ldd;
    const float* C;
    int64_t ldc;
    const float* Mx;
    int64_t ldm;
    float alpha, beta, gamma, delta;
    bool vec_ok;
    // sym: the product is square and its result symmetric (a polynomial in one
    // symmetric matrix); the grid covers the upper-triangle tiles only
    // (tile_coords_sym), C and Mx are read there, and each result tile is written
    // twice, as itself and mirrored, a diagonal tile from its upper half: D comes
    // out exactly symmetric
    int sym = 0;

    template <int BM, int BN, int NG>
    __device__ inline void run(float* tile, int m0, int n0, int M, int N, const double* sc, int a1, int a2,
                               int cf) const {
        if (sym) {
            run_sym<BM, BN, NG>(tile, m0, n0, M);
            return;
        }
        run_plain<BM, BN, NG>(tile, m0, n0, M, N);
    }

    // o = alpha acc + beta C + gamma Mx + delta I of the thread's float4 groups
    template <int BM, int BN, int NG>
    __device__ inline void values(const float* tile, int m0, int n0, int M, int N, f32x4 (&o)[NG],
                                  bool (&full)[NG]) const {
        constexpr int P = BN + 4, GPR = BN / 4;
        f32x4 vd[NG], vm[NG];
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int g = threadIdx.x + q * GTHREADS;
            const int i = m0 + g / GPR, j = n0 + (g % GPR) * 4;
            full[q] = vec_ok && i < M && j + 3 < N;
            vd[q] = vm[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
            if (full[q]) {
                if (beta != 0.f) vd[q] = *reinterpret_cast<const f32x4*>(C + (int64_t)i * ldc + j);
                if (gamma != 0.f) vm[q] = *reinterpret_cast<const f32x4*>(Mx + (int64_t)i * ldm + j);
            } else if (i < M) {
                for (int e = 0; e < 4; ++e) {
                    if (j + e < N) {
                        if (beta != 0.f) vd[q][e] = C[(int64_t)i * ldc + j + e];
                        if (gamma != 0.f) vm[q][e] = Mx[(int64_t)i * ldm + j + e];
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int g = threadIdx.x + q * GTHREADS;
            const int r = g / GPR, cc = (g % GPR) * 4;
            const int i = m0 + r, j = n0 + cc;
            const f32x4 acc = *reinterpret_cast<const f32x4*>(tile + r * P + cc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float v = alpha * acc[e] + beta * vd[q][e] + gamma * vm[q][e];
                if (i == j + e) v += delta;
                o[q][e] = v;
            }
        }
    }

    __device__ inline void store4(int i, int j, int M, int N, bool vec, const f32x4& v) const {
        if (i >= M) return;
        if (vec && j + 3 < N) {
            *reinterpret_cast<f32x4*>(D + (int64_t)i * ldd + j) = v;
        } else {
            for (int e = 0; e < 4; ++e)
                if (j + e < N) D[(int64_t)i * ldd + j + e] = v[e];
        }
    }

    template <int BM, int BN, int NG>
    __device__ inline void run_sym(float* tile, int m0, int n0, int M) const {
        constexpr int P = BN + 4, GPR = BN / 4;
        f32x4 o[NG];
        bool full[NG];
        values<BM, BN, NG>(tile, m0, n0, M, M, o, full);
        __syncthreads();   // every accumulator is read before the tile is overwritten
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int g = threadIdx.x + q * GTHREADS;
            *reinterpret_cast<f32x4*>(tile + (g / GPR) * P + (g % GPR) * 4) = o[q];
        }
        __syncthreads();
        const bool diag = m0 == n0;
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int g = threadIdx.x + q * GTHREADS;
            const int r = g / GPR, cc = (g % GPR) * 4;
            f32x4 v, w;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = cc + e;
                v[e] = (!diag || r <= c) ? tile[r * P + c] : tile[c * P + r];
                w[e] = tile[c * P + r];
            }
            store4(m0 + r, n0 + cc, M, M, vec_ok, v);
            if (!diag) store4(n0 + r, m0 + cc, M, M, vec_ok, w);
        }
    }

    // Epilogue of one piece of a symmetric product (gemm_f32_piece_kernel, 1024
    // threads; M % 64 == 0 and vec_ok, both checked by the host).  half >= 0: the
    // 64 x 32 block at (m0, n0 + 32 half) above the diagonal, stored and mirrored;
    // half < 0: the diagonal tile at (m0, m0), its upper triangle mirrored onto
    // the lower one.  tile: 64 x 68 floats, the product at its tile positions.
    __device__ inline void run_piece(float* tile, int m0, int n0, int half) const {
        constexpr int P = 68;
        const int t = threadIdx.x;
        // values o = alpha acc + beta C + gamma Mx (+ delta on the diagonal) at the
        // stored positions: 64 rows x 8 groups (half piece) or 64 x 16 (diagonal)
        const int gpr = half >= 0 ? 8 : 16;
        const int c0 = half >= 0 ? 32 * half : 0;
        const bool mine = t < 64 * gpr;
        const int r = t / gpr, cc = c0 + (t % gpr) * 4;
        const int i = m0 + r, j = n0 + cc;
        f32x4 o = (f32x4){0.f, 0.f, 0.f, 0.f};
        if (mine) {
            const f32x4 a = *reinterpret_cast<const f32x4*>(tile + r * P + cc);
            f32x4 vd = (f32x4){0.f, 0.f, 0.f, 0.f}, vm = vd;
            if (beta != 0.f) vd = *reinterpret_cast<const f32x4*>(C + (int64_t)i * ldc + j);
            if (gamma != 0.f) vm = *reinterpret_cast<const f32x4*>(Mx + (int64_t)i * ldm + j);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float v = alpha * a[e] + beta * vd[e] + gamma * vm[e];
                if (i == j + e) v += delta;
                o[e] = v;
            }
        }
        __syncthreads();   // every product value read before the tile is overwritten
        if (mine) *reinterpret_cast<f32x4*>(tile + r * P + cc) = o;
        __syncthreads();
        if (half < 0) {
            // the full diagonal tile from its upper triangle
            f32x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = r <= cc + e ? tile[r * P + cc + e] : tile[(cc + e) * P + r];
            *reinterpret_cast<f32x4*>(D + (int64_t)i * ldd + j) = v;
            return;
        }
        if (mine) *reinterpret_cast<f32x4*>(D + (int64_t)i * ldd + j) = o;
        // the mirror: rows n0 + c0 .. + 31, columns m0 .. m0 + 63 (32 x 16 groups)
        if (t < 512) {
            const int r2 = t / 16, c2 = (t % 16) * 4;
            f32x4 w;
#pragma unroll
            for (int e = 0; e < 4; ++e) w[e] = tile[(c2 + e) * P + c0 + r2];
            *reinterpret_cast<f32x4*>(D + (int64_t)(n0 + c0 + r2) * ldd + m0 + c2) = w;
        }
    }

    template <int BM, int BN, int NG>
    __device__ inline void run_plain(const float* tile, int m0, int n0, int M, int N) const {
        constexpr int GPR = BN / 4;
        f32x4 o[NG];
        bool full[NG];
        values<BM, BN, NG>(tile, m0, n0, M, N, o, full);
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int g = threadIdx.x + q * GTHREADS;
            store4(m0 + g / GPR, n0 + (g % GPR) * 4, M, N, vec_ok, o[q]);
        }
    }
};

__device__ inline const double* epi_scal(const EpiLin&) { return nullptr; }
__device__ inline const double* epi_scal(const EpiGram&) { return nullptr; }
__device__ inline const double* epi_scal(const EpiCheb& e) { return e.scal; }
// The symmetric tile order applies to linear-epilogue products flagged sym.
template <class E>
__host__ __device__ inline bool epi_sym(const E&) { return false; }
template <>
__host__ __device__ inline bool epi_sym<EpiLin>(const EpiLin& e) { return e.sym != 0; }

// Tile of this workgroup: the upper-triangle order for symmetric products.
template <class E>
__device__ inline void tile_of(const E& epi, int ntm, int ntn, int& tm, int& tn) {
    if (epi_sym(epi))
        tile_coords_sym(ntm, tm, tn);
    else
        tile_coords(ntm, ntn, tm, tn);
}

// Wave layout: WM x WN waves over the output tile, times KS waves that split
// each K-tile's sub-steps between them (their partial sums are added once,
// in LDS, before the epilogue).  64 x 64 tiles use 2 x 2 x 2: each wave owns a
// 32 x 32 output (2 x 2 MFMA blocks, four independent accumulation chains) over
// half of every K-tile, which reads a third less from LDS than eight waves with
// 32 x 16 outputs over whole K-tiles.  128 x 128 tiles use 2 x 4 x 1.
template <int BM, int BN>
struct WaveLayout {
    static constexpr int WM = 2;
    static constexpr int WN = (BM == 64 && BN == 64) ? 2 : 4;
    static constexpr int KS = GWAVES / (WM * WN);
};

// NWAVES: waves of the workgroup (the K-split KS takes the waves beyond WM x WN).
template <int BM, int BN, int LA, int LB, int NWAVES = GWAVES>
struct GemmCore {
    using GA = TileGeom<BM, LA>;
    using GB = TileGeom<BN, LB>;
    static constexpr int WM = WaveLayout<BM, BN>::WM, WN = WaveLayout<BM, BN>::WN, KS = NWAVES / (WM * WN);
    static constexpr int MB = BM / WM / 16, NB = BN / WN / 16;   // 16x16 blocks per wave
    static constexpr int KQ = KG / KS;                            // sub-steps per wave and K-tile
    static_assert(MB >= 1 && NB >= 1 && KS >= 1 && WM * WN * KS == NWAVES, "bad wave layout");
    static_assert(KQ % 4 == 0, "sub-steps per wave must be a multiple of 4");

    struct Frags {
        float a[MB][KQ];
        float b[NB][KQ];
    };

    // instruction counts of one pipeline step (per wave)
    static constexpr int kMfma = MB * NB * KQ;
    static constexpr int kReads = (LA == KCONTIG ? MB * KQ / 4 : MB * KQ) + (LB == KCONTIG ? NB * KQ / 4 : NB * KQ);
    static constexpr int kWrites = GA::per_thread + GB::per_thread;

    static __device__ inline void read(const float* la, const float* lb, int wr, int wc, int kh, int lane, Frags& f) {
#pragma unroll
        for (int i = 0; i < MB; ++i) frag_read<BM, LA, KQ>(la, wr * (BM / WM) + i * 16, lane, kh * KQ, f.a[i]);
#pragma unroll
        for (int j = 0; j < NB; ++j) frag_read<BN, LB, KQ>(lb, wc * (BN / WN) + j * 16, lane, kh * KQ, f.b[j]);
    }

    // One K-tile (this wave's sub-steps) into the fresh partial `part`.
    static __device__ inline void mfma(const Frags& f, f32x4 (&part)[MB][NB]) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) part[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < KQ; ++kk)
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(f.a[i][kk], f.b[j][kk], part[i][j], 0, 0, 0);
    }

    static __device__ inline void add_into(f32x4 (&acc)[MB][NB], const f32x4 (&part)[MB][NB]) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[i][j] += part[i][j];
    }
};

// Pipeline of step t (tiles past the end are clamped to the last one: loaded,
// stored and read, never used):
//   issue the global loads of tile t+3 into register set (t+1)%2
//   MFMAs of tile t from fragment set t%2 (read during step t-1)
//   read the fragments of tile t+1 from LDS stage (t+1)%2 into set (t+1)%2
//   store tile t+2 (register set t%2, loaded during step t-1) to LDS stage t%2
//   barrier
// Stage t%2 is free at step t: its last reader was the fragment read of tile t
// during step t-1 (the prologue for t = 0), which the barrier of step t-1 (the
// prologue's second barrier) completed.  Every global load
// has about two steps to land and every LDS read one step of MFMAs to hide.
template <int BM, int BN, int LA, int LB, bool VEC, class Epi>
__global__ void __launch_bounds__(GTHREADS) gemm_f32_kernel(Operand A, Operand B, int M, int N, int Kd, Epi epi,
                                                            int sc_a1, int sc_a2, int sc_coef) {
    using C = GemmCore<BM, BN, LA, LB>;
    using GA = typename C::GA;
    using GB = typename C::GB;
    using Frags = typename C::Frags;
    constexpr int MB = C::MB, NB = C::NB;
    __shared__ __attribute__((aligned(16))) float lds_a[2][GA::size];
    __shared__ __attribute__((aligned(16))) float lds_b[2][GB::size];
    static_assert(BM * (BN + 4) <= 2 * GA::size, "the epilogue tile must fit the A buffers");

    const int ntm = (M + BM - 1) / BM;
    const int ntn = (N + BN - 1) / BN;
    int tm, tn;
    tile_of(epi, ntm, ntn, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wo = wave % (C::WM * C::WN);          // output sub-tile of this wave
    const int kh = wave / (C::WM * C::WN);          // its share of each K-tile
    const int wr = wo / C::WN, wc = wo % C::WN;

    f32x4 acc[MB][NB], p0[MB][NB], p1[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = p1[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

    f32x4 ra0[GA::per_thread], rb0[GB::per_thread], ra1[GA::per_thread], rb1[GB::per_thread];
    Frags f0, f1;
    const int nkt = (Kd + GBK - 1) / GBK;
    const int last = nkt - 1;
    auto kof = [&](int t) { return min(t, last) * GBK; };

    // prologue: tiles 0 and 1 into LDS, tile 2 in flight, fragments of tile 0
    tile_load<BM, LA, VEC>(A, m0, kof(0), Kd, ra0);
    tile_load<BN, LB, VEC>(B, n0, kof(0), Kd, rb0);
    tile_load<BM, LA, VEC>(A, m0, kof(1), Kd, ra1);
    tile_load<BN, LB, VEC>(B, n0, kof(1), Kd, rb1);
    tile_store<BM, LA>(lds_a[0], ra0);
    tile_store<BN, LB>(lds_b[0], rb0);
    tile_store<BM, LA>(lds_a[1], ra1);
    tile_store<BN, LB>(lds_b[1], rb1);
    __syncthreads();
    tile_load<BM, LA, VEC>(A, m0, kof(2), Kd, ra0);
    tile_load<BN, LB, VEC>(B, n0, kof(2), Kd, rb0);
    C::read(lds_a[0], lds_b[0], wr, wc, kh, lane, f0);
    // every wave has its tile-0 fragments before step 0 overwrites stage 0
    __syncthreads();

    for (int kt = 0; kt < nkt; kt += 2) {
        // ---- step kt (even): fragments f0, partial p0, loads into set 1, store set 0
        tile_load<BM, LA, VEC>(A, m0, kof(kt + 3), Kd, ra1);
        tile_load<BN, LB, VEC>(B, n0, kof(kt + 3), Kd, rb1);
        CPA_SCHED_FENCE();
        C::mfma(f0, p0);
        C::add_into(acc, p1);
        C::read(lds_a[1], lds_b[1], wr, wc, kh, lane, f1);
        tile_store<BM, LA>(lds_a[0], ra0);
        tile_store<BN, LB>(lds_b[0], rb0);
        interleave_step<C::kMfma, C::kReads, C::kWrites>();
        __syncthreads();
        if (kt + 1 >= nkt) {
            C::add_into(acc, p0);
            break;
        }
        // ---- step kt+1 (odd): fragments f1, partial p1, loads into set 0, store set 1
        tile_load<BM, LA, VEC>(A, m0, kof(kt + 4), Kd, ra0);
        tile_load<BN, LB, VEC>(B, n0, kof(kt + 4), Kd, rb0);
        CPA_SCHED_FENCE();
        C::mfma(f1, p1);
        C::add_into(acc, p0);
        C::read(lds_a[0], lds_b[0], wr, wc, kh, lane, f0);
        tile_store<BM, LA>(lds_a[1], ra1);
        tile_store<BN, LB>(lds_b[1], rb1);
        interleave_step<C::kMfma, C::kReads, C::kWrites>();
        __syncthreads();
        if (kt + 2 >= nkt) C::add_into(acc, p1);
    }

    // stage the accumulator tile in LDS (reusing the operand buffers)
    float* tile = &lds_a[0][0];
#pragma unroll
    for (int h = 0; h < C::KS; ++h) {
        if (kh == h) {
#pragma unroll
            for (int a = 0; a < MB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = wr * (BM / C::WM) + a * 16 + 4 * (lane >> 4) + r;
                        const int j = wc * (BN / C::WN) + b * 16 + (lane & 15);
                        float* t = tile + i * (BN + 4) + j;
                        *t = (h == 0) ? acc[a][b][r] : *t + acc[a][b][r];
                    }
        }
        if (C::KS > 1) __syncthreads();
    }
    __syncthreads();
    constexpr int NG = BM * BN / 4 / GTHREADS;   // float4 groups per thread
    static_assert(NG * 4 * GTHREADS == BM * BN, "tile must split evenly into float4 groups");
    epi.template run<BM, BN, NG>(tile, m0, n0, M, N, epi_scal(epi), sc_a1, sc_a2, sc_coef);
}

}  // namespace cpa
