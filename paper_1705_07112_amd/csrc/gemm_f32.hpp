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
// g = lane/16 at sub-step kk is mapped to tile column k = 4 g + kk for both
// operands (any bijection is valid as long as A and B agree).  With that map a
// KCONTIG LDS row yields the four sub-steps of a lane in one 16-byte read.
//
// Workgroup: 256 threads = 4 waves in a 2 x 2 arrangement; each wave owns a
// (BM/2) x (BN/2) sub-tile made of 16 x 16 MFMA blocks.  K-tiles of 16 are
// double-buffered in LDS with register prefetch of the next tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpa {

typedef float f32x4 __attribute__((ext_vector_type(4)));

enum Layout { XCONTIG = 0, KCONTIG = 1 };

constexpr int GBK = 16;          // K-tile depth
constexpr int GTHREADS = 256;    // threads per workgroup

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
    bool vec_ok;  // ld % 4 == 0 and p 16-byte aligned
};

// Loads the float4 vectors of one tile (x0.., k0..) into registers, zero outside bounds.
template <int BX, int L>
__device__ inline void tile_load(const Operand& op, int x0, int k0, int Kd, f32x4 (&r)[TileGeom<BX, L>::per_thread]) {
#pragma unroll
    for (int q = 0; q < TileGeom<BX, L>::per_thread; ++q) {
        const int f = threadIdx.x + q * GTHREADS;
        int x, k;
        if (L == XCONTIG) {
            k = f / (BX / 4);
            x = (f % (BX / 4)) * 4;
        } else {
            x = f / (GBK / 4);
            k = (f % (GBK / 4)) * 4;
        }
        const int gx = x0 + x, gk = k0 + k;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (L == XCONTIG) {
            if (gk < Kd) {
                const float* src = op.p + (int64_t)gk * op.ld + gx;
                if (op.vec_ok && gx + 3 < op.xdim) {
                    v = *reinterpret_cast<const f32x4*>(src);
                } else {
                    if (gx + 0 < op.xdim) v[0] = src[0];
                    if (gx + 1 < op.xdim) v[1] = src[1];
                    if (gx + 2 < op.xdim) v[2] = src[2];
                    if (gx + 3 < op.xdim) v[3] = src[3];
                }
            }
        } else {
            if (gx < op.xdim) {
                const float* src = op.p + (int64_t)gx * op.ld + gk;
                if (op.vec_ok && gk + 3 < Kd) {
                    v = *reinterpret_cast<const f32x4*>(src);
                } else {
                    if (gk + 0 < Kd) v[0] = src[0];
                    if (gk + 1 < Kd) v[1] = src[1];
                    if (gk + 2 < Kd) v[2] = src[2];
                    if (gk + 3 < Kd) v[3] = src[3];
                }
            }
        }
        r[q] = v;
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

// The four sub-step operands of one lane for the 16-row block starting at xb.
template <int BX, int L>
__device__ inline f32x4 frag_read(const float* lds, int xb, int lane) {
    const int xi = xb + (lane & 15);
    const int g = lane >> 4;
    if (L == XCONTIG) {
        constexpr int P = TileGeom<BX, L>::pitch;
        f32x4 v;
        v[0] = lds[(4 * g + 0) * P + xi];
        v[1] = lds[(4 * g + 1) * P + xi];
        v[2] = lds[(4 * g + 2) * P + xi];
        v[3] = lds[(4 * g + 3) * P + xi];
        return v;
    } else {
        return *reinterpret_cast<const f32x4*>(lds + xi * TileGeom<BX, L>::pitch + 4 * g);
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

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Epilogue of the Gram: C = acc, with ||C||_F^2 and trace(C) accumulated in FP64.
struct EpiGram {
    float* C;
    int64_t ldc;
    double* fro2;    // += sum C(i,j)^2
    double* trace;   // += sum C(i,i)
    __device__ inline void load_scalars(int, int, int) {}
    __device__ inline void apply(int i, int j, float v, double& s1, double& s2) const {
        C[(int64_t)i * ldc + j] = v;
        s1 += (double)v * v;
        if (i == j) s2 += v;
    }
    __device__ inline void finish(double s1, double s2) const {
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        if ((threadIdx.x & 63) == 0) {
            if (s1 != 0.0) atomicAdd(fro2, s1);
            if (s2 != 0.0) atomicAdd(trace, s2);
        }
    }
};

// Epilogue of one recurrence step:
//   Ynew = a * acc + b * Yk + c * Yprev
//   first step:  out = c0/2 * Yk + c1 * Ynew      (Yk = X)
//   later steps: out += c_{k+1} * Ynew
//   Ynew is stored to Ydst unless this is the last step (Ydst may equal Yprev:
//   each element is read and then written by the same lane).
//   ||Ynew||_F^2 is accumulated for the growth check.
// Scalars come from device memory so that a bound computed on the device is
// consumed without a host round trip.
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
    double* nrm2;         // slot for ||Y_{k+1}||^2
    // resolved per launch
    float a, b, c, ck1, c0h;

    __device__ inline void load_scalars(int sc_a1, int sc_a2, int sc_coef) {
        if (step == 0) {
            a = (float)scal[sc_a1];
            b = -1.f;
            c = 0.f;
            c0h = (float)(0.5 * scal[sc_coef + 0]);
        } else {
            a = (float)scal[sc_a2];
            b = -2.f;
            c = -1.f;
            c0h = 0.f;
        }
        ck1 = (float)scal[sc_coef + step + 1];
    }
    __device__ inline void apply(int i, int j, float v, double& s1, double&) const {
        const float yk = Yk[(int64_t)i * ldk + j];
        float yn = a * v + b * yk;
        if (step > 0) yn += c * Yprev[(int64_t)i * ldp + j];
        float* o = out + (int64_t)i * ldo + j;
        if (step == 0)
            *o = c0h * yk + ck1 * yn;
        else
            *o += ck1 * yn;
        if (!last) Ydst[(int64_t)i * ldd + j] = yn;
        s1 += (double)yn * yn;
    }
    __device__ inline void finish(double s1, double) const {
        s1 = wave_sum(s1);
        if ((threadIdx.x & 63) == 0 && s1 != 0.0) atomicAdd(nrm2, s1);
    }
};

template <int BM, int BN, int LA, int LB, class Epi>
__global__ void __launch_bounds__(GTHREADS) gemm_f32_kernel(Operand A, Operand B, int M, int N, int Kd, Epi epi,
                                                            int sc_a1, int sc_a2, int sc_coef) {
    using GA = TileGeom<BM, LA>;
    using GB = TileGeom<BN, LB>;
    __shared__ __attribute__((aligned(16))) float lds_a[2][GA::size];
    __shared__ __attribute__((aligned(16))) float lds_b[2][GB::size];

    const int ntm = (M + BM - 1) / BM;
    const int ntn = (N + BN - 1) / BN;
    int tm, tn;
    tile_coords(ntm, ntn, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    constexpr int MB = BM / 32, NB = BN / 32;   // 16x16 blocks per wave

    f32x4 acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};

    f32x4 ra[GA::per_thread], rb[GB::per_thread];
    const int nkt = (Kd + GBK - 1) / GBK;
    if (nkt > 0) {
        tile_load<BM, LA>(A, m0, 0, Kd, ra);
        tile_load<BN, LB>(B, n0, 0, Kd, rb);
        tile_store<BM, LA>(lds_a[0], ra);
        tile_store<BN, LB>(lds_b[0], rb);
    }
    __syncthreads();

    for (int kt = 0; kt < nkt; ++kt) {
        const int cur = kt & 1;
        const bool more = (kt + 1) < nkt;
        if (more) {
            tile_load<BM, LA>(A, m0, (kt + 1) * GBK, Kd, ra);
            tile_load<BN, LB>(B, n0, (kt + 1) * GBK, Kd, rb);
        }
        f32x4 fa[MB], fb[NB];
#pragma unroll
        for (int a = 0; a < MB; ++a) fa[a] = frag_read<BM, LA>(lds_a[cur], wr * (BM / 2) + a * 16, lane);
#pragma unroll
        for (int b = 0; b < NB; ++b) fb[b] = frag_read<BN, LB>(lds_b[cur], wc * (BN / 2) + b * 16, lane);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int a = 0; a < MB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a][kk], fb[b][kk], acc[a][b], 0, 0, 0);
        if (more) {
            tile_store<BM, LA>(lds_a[cur ^ 1], ra);
            tile_store<BN, LB>(lds_b[cur ^ 1], rb);
        }
        __syncthreads();
    }

    epi.load_scalars(sc_a1, sc_a2, sc_coef);
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wr * (BM / 2) + a * 16 + 4 * (lane >> 4) + r;
                const int j = n0 + wc * (BN / 2) + b * 16 + (lane & 15);
                if (i < M && j < N) epi.apply(i, j, acc[a][b][r], s1, s2);
            }
    epi.finish(s1, s2);
}

}  // namespace cpa
