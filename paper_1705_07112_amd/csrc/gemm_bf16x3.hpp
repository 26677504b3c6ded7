// Split-precision recurrence GEMM: C = A B with FP32 operands evaluated as
//   A_hi B_hi + A_hi B_lo + A_lo B_hi,   x_hi = bf16(x), x_lo = bf16(x - x_hi)
// (round to nearest even), on the gfx950 BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation.  The dropped A_lo B_lo
// term is below 2^-16 relative; the three products carry about 16 mantissa bits
// of each operand.
//
// Operands stay FP32 in HBM (the same traffic as the FP32 path); the split
// happens when a K-tile is written to LDS, where hi and lo live in separate
// bf16 tiles laid out row = output index, k contiguous (an XCONTIG operand is
// transposed on the way in).  The pipeline, wave layout (2 x 2 output x 2
// K-halves, one 32-wide MFMA step per wave and tile), two-level summation and
// epilogues are those of the FP32 engine in gemm_f32.hpp.
//
// MFMA operand map: lane l supplies row l%16 of A (column l%16 of B) and eight
// consecutive k of lane group g = l/16; sub-step s of a 64-wide tile covers tile
// columns k = 16 g + 8 s + e, e = 0..7, for both operands.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f32.hpp"

namespace cpa {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

constexpr int BPITCH = GBK + 8;   // bf16 elements per LDS row (144 bytes: conflict-free 16-byte reads)

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ inline unsigned short bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ inline float bf16_value(unsigned short b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline void split2(float x, unsigned short& hi, unsigned short& lo) {
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_value(hi));
}

template <int BX>
struct SplitTile {
    static constexpr int size = BX * BPITCH;   // bf16 elements per buffer
};

// Registers of one K-tile (FP32, as loaded) -> hi/lo bf16 tiles in LDS.
template <int BX, int L>
__device__ inline void tile_store_split(unsigned short* hi, unsigned short* lo,
                                        const f32x4 (&r)[TileGeom<BX, L>::per_thread]) {
#pragma unroll
    for (int q = 0; q < TileGeom<BX, L>::per_thread; ++q) {
        const int f = threadIdx.x + q * GTHREADS;
        if (L == KCONTIG) {
            const int x = f / (GBK / 4), k = (f % (GBK / 4)) * 4;
            u16x4 h, l;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                unsigned short a, b;
                split2(r[q][e], a, b);
                h[e] = a;
                l[e] = b;
            }
            *reinterpret_cast<u16x4*>(hi + x * BPITCH + k) = h;
            *reinterpret_cast<u16x4*>(lo + x * BPITCH + k) = l;
        } else {
            const int k = f / (BX / 4), x = (f % (BX / 4)) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                unsigned short a, b;
                split2(r[q][e], a, b);
                hi[(x + e) * BPITCH + k] = a;
                lo[(x + e) * BPITCH + k] = b;
            }
        }
    }
}

template <int BM, int BN, int LA, int LB>
struct SplitCore {
    static constexpr int WM = 2, WN = 2, KS = 2;          // 8 waves
    static constexpr int MB = BM / WM / 16, NB = BN / WN / 16;
    static_assert(GBK == 64, "one 32-wide MFMA step per wave and tile needs 64-wide tiles");
    static_assert(MB >= 1 && NB >= 1 && WM * WN * KS == GWAVES, "bad wave layout");

    struct Frags {
        bf16x8 ah[MB], al[MB], bh[NB], bl[NB];
    };

    static constexpr int kMfma = 3 * MB * NB;
    static constexpr int kReads = 2 * (MB + NB);
    static constexpr int kWrites = (LA == KCONTIG ? 2 : 8) * TileGeom<BM, LA>::per_thread +
                                   (LB == KCONTIG ? 2 : 8) * TileGeom<BN, LB>::per_thread;

    static __device__ inline bf16x8 rd(const unsigned short* t, int row, int lane, int s) {
        return *reinterpret_cast<const bf16x8*>(t + row * BPITCH + 16 * (lane >> 4) + 8 * s);
    }

    static __device__ inline void read(const unsigned short* ah, const unsigned short* al, const unsigned short* bh,
                                       const unsigned short* bl, int wr, int wc, int kh, int lane, Frags& f) {
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int row = wr * (BM / WM) + i * 16 + (lane & 15);
            f.ah[i] = rd(ah, row, lane, kh);
            f.al[i] = rd(al, row, lane, kh);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int row = wc * (BN / WN) + j * 16 + (lane & 15);
            f.bh[j] = rd(bh, row, lane, kh);
            f.bl[j] = rd(bl, row, lane, kh);
        }
    }

    // this wave's MFMA step of one K-tile into the fresh partial (small terms first)
    static __device__ inline void mfma(const Frags& f, f32x4 (&part)[MB][NB]) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                f32x4 p = {0.f, 0.f, 0.f, 0.f};
                p = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.al[i], f.bh[j], p, 0, 0, 0);
                p = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[i], f.bl[j], p, 0, 0, 0);
                part[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[i], f.bh[j], p, 0, 0, 0);
            }
    }

    static __device__ inline void add_into(f32x4 (&acc)[MB][NB], const f32x4 (&part)[MB][NB]) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[i][j] += part[i][j];
    }
};

// Same step structure as gemm_f32_kernel (see there): loads three tiles ahead,
// fragments of tile t+1 read during tile t's MFMAs, one barrier per tile.
template <int BM, int BN, int LA, int LB, bool VEC, class Epi>
__global__ void __launch_bounds__(GTHREADS) gemm_bf16x3_kernel(Operand A, Operand B, int M, int N, int Kd, Epi epi,
                                                               int sc_a1, int sc_a2, int sc_coef) {
    using C = SplitCore<BM, BN, LA, LB>;
    using GA = TileGeom<BM, LA>;
    using GB = TileGeom<BN, LB>;
    using Frags = typename C::Frags;
    constexpr int MB = C::MB, NB = C::NB;
    constexpr int SA = SplitTile<BM>::size, SB = SplitTile<BN>::size;
    // [stage][hi, lo] tiles of A, then of B; reused as the FP32 epilogue tile
    __shared__ __attribute__((aligned(16))) unsigned short lds[2 * 2 * (SA + SB)];
    static_assert(BM * (BN + 4) * 2 <= 2 * 2 * (SA + SB), "the epilogue tile must fit the LDS block");
    auto a_hi = [&](int st) { return lds + st * 2 * SA; };
    auto a_lo = [&](int st) { return lds + st * 2 * SA + SA; };
    auto b_hi = [&](int st) { return lds + 4 * SA + st * 2 * SB; };
    auto b_lo = [&](int st) { return lds + 4 * SA + st * 2 * SB + SB; };

    const int ntm = (M + BM - 1) / BM;
    const int ntn = (N + BN - 1) / BN;
    int tm, tn;
    tile_coords(ntm, ntn, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wo = wave % (C::WM * C::WN);
    const int kh = wave / (C::WM * C::WN);
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

    tile_load<BM, LA, VEC>(A, m0, kof(0), Kd, ra0);
    tile_load<BN, LB, VEC>(B, n0, kof(0), Kd, rb0);
    tile_load<BM, LA, VEC>(A, m0, kof(1), Kd, ra1);
    tile_load<BN, LB, VEC>(B, n0, kof(1), Kd, rb1);
    tile_store_split<BM, LA>(a_hi(0), a_lo(0), ra0);
    tile_store_split<BN, LB>(b_hi(0), b_lo(0), rb0);
    tile_store_split<BM, LA>(a_hi(1), a_lo(1), ra1);
    tile_store_split<BN, LB>(b_hi(1), b_lo(1), rb1);
    __syncthreads();
    tile_load<BM, LA, VEC>(A, m0, kof(2), Kd, ra0);
    tile_load<BN, LB, VEC>(B, n0, kof(2), Kd, rb0);
    C::read(a_hi(0), a_lo(0), b_hi(0), b_lo(0), wr, wc, kh, lane, f0);
    __syncthreads();

    for (int kt = 0; kt < nkt; kt += 2) {
        tile_load<BM, LA, VEC>(A, m0, kof(kt + 3), Kd, ra1);
        tile_load<BN, LB, VEC>(B, n0, kof(kt + 3), Kd, rb1);
        CPA_SCHED_FENCE();
        C::mfma(f0, p0);
        C::add_into(acc, p1);
        C::read(a_hi(1), a_lo(1), b_hi(1), b_lo(1), wr, wc, kh, lane, f1);
        tile_store_split<BM, LA>(a_hi(0), a_lo(0), ra0);
        tile_store_split<BN, LB>(b_hi(0), b_lo(0), rb0);
        interleave_step<C::kMfma, C::kReads, C::kWrites>();
        __syncthreads();
        if (kt + 1 >= nkt) {
            C::add_into(acc, p0);
            break;
        }
        tile_load<BM, LA, VEC>(A, m0, kof(kt + 4), Kd, ra0);
        tile_load<BN, LB, VEC>(B, n0, kof(kt + 4), Kd, rb0);
        CPA_SCHED_FENCE();
        C::mfma(f1, p1);
        C::add_into(acc, p0);
        C::read(a_hi(0), a_lo(0), b_hi(0), b_lo(0), wr, wc, kh, lane, f0);
        tile_store_split<BM, LA>(a_hi(1), a_lo(1), ra1);
        tile_store_split<BN, LB>(b_hi(1), b_lo(1), rb1);
        interleave_step<C::kMfma, C::kReads, C::kWrites>();
        __syncthreads();
        if (kt + 2 >= nkt) C::add_into(acc, p1);
    }

    // the two K-halves meet in the FP32 epilogue tile
    float* tile = reinterpret_cast<float*>(lds);
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
        __syncthreads();
    }
    constexpr int NG = BM * BN / 4 / GTHREADS;
    epi.template run<BM, BN, NG>(tile, m0, n0, M, N, epi_scal(epi), sc_a1, sc_a2, sc_coef);
}

}  // namespace cpa
