// FP32 MFMA GEMM for full tiles of two k-contiguous operands, with the operand
// tiles moved from global memory to LDS by the load unit itself
// (global_load_lds_dwordx4: each lane's 16 bytes land at a consecutive LDS
// address, no staging registers, no LDS store instructions).  Used for the
// linear-epilogue products of the matrix-polynomial route.
//
// Same product, MFMA sequence, two-level partial sums and epilogues as
// gemm_f32_kernel (gemm_f32.hpp) for A and B in the KCONTIG layout; it differs
// in how tiles reach LDS and in the wave count:
//   * four LDS stages (tile i in stage i % 4, 32 KB each) and the copy of tile
//     t + 3 issued at step t, so a copy has two whole steps to land -- the
//     operand panels are first touched by all workgroups of an XCD at about the
//     same time, so many copies come from the MALL or HBM;
//   * rows are stored unpadded (64 floats, 16 chunks of 16 bytes) with chunk c
//     of row r at position c ^ (r % 16): a 16-byte fragment read by 16 lanes of
//     16 consecutive rows then touches 16 different chunk positions, i.e. all
//     64 banks once, and each lane's copy address is still a permutation of
//     its row's 256 bytes (coalesced);
//   * the waits are explicit: at the end of step t each wave waits until only
//     its copies of tile t + 3 are outstanding (vmcnt), then the workgroup
//     barrier makes tile t + 2 visible to every wave before step t + 1 reads it.
//     The barrier is the bare s_barrier: a fence would wait for every
//     outstanding copy, including the ones meant to stay in flight;
//   * NW = 16 waves (four per SIMD, K-split 4) hide more of the LDS and MFMA
//     latency than eight, at 110 registers per wave.
// Requirements (checked by the host): M % 64 == 0, N % 64 == 0, Kd % 64 == 0,
// 16-byte aligned bases, leading dimensions % 4 == 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gemm_f32.hpp"

namespace cpa {

constexpr int LDS_STAGES = 4;
// copy instructions per wave for one K-tile of both operands (four rows each)
template <int NW>
constexpr int dma_per_tile() { return 2 * (64 / NW / 4); }
constexpr int kDmaPerTile = dma_per_tile<GWAVES>();

// Waits until at most N of this wave's vector-memory operations are outstanding
// (N: the copies of one K-tile), optionally with all LDS operations done.
template <int N>
__device__ inline void wait_vm();
template <>
__device__ inline void wait_vm<2>() { asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); }
template <>
__device__ inline void wait_vm<4>() { asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); }
template <int N>
__device__ inline void wait_vm_lds();
template <>
__device__ inline void wait_vm_lds<2>() { asm volatile("s_waitcnt vmcnt(2) lgkmcnt(0)" ::: "memory"); }
template <>
__device__ inline void wait_vm_lds<4>() { asm volatile("s_waitcnt vmcnt(4) lgkmcnt(0)" ::: "memory"); }
constexpr int LDS_TILE = 64 * GBK;   // floats per operand tile (64 rows x 64 k, unpadded)
static_assert(GBK == 64, "the swizzled LDS layout assumes K-tiles of 64");

// Copy of one 64 x 64 k-contiguous tile (rows x0.., k0..) into an LDS stage:
// wave w copies rows 8 w .. 8 w + 7, four rows (64 lanes x 16 bytes) per
// instruction; lane L takes row R = R0 + L / 16 and stores its chunk at
// position L % 16, so it reads logical chunk (L % 16) ^ (R % 16).
template <int NW = GWAVES>
__device__ inline void tile_dma(const Operand& op, int x0, int k0, float* stage, int wave, int lane) {
    constexpr int ROWS_PER_WAVE = 64 / NW;
    static_assert(ROWS_PER_WAVE % 4 == 0, "four rows per copy instruction");
#pragma unroll
    for (int i = 0; i < ROWS_PER_WAVE / 4; ++i) {
        const int R0 = wave * ROWS_PER_WAVE + 4 * i;
        const int R = R0 + (lane >> 4);
        const int c = (lane & 15) ^ (R & 15);
        const float* src = op.p + (int64_t)(x0 + R) * op.ld + k0 + 4 * c;
        __builtin_amdgcn_global_load_lds(src, stage + R0 * GBK, 16, 0, 0);
    }
}

// Fragments of one lane for the 16-row block at xb (tile column k = KG g + kk,
// kk = koff .. koff + Q - 1), from a swizzled stage.
template <int Q>
__device__ inline void frag_read_swz(const float* stage, int xb, int lane, int koff, float (&v)[Q]) {
    const int xi = xb + (lane & 15);
    const int g = lane >> 4;
    const float* row = stage + xi * GBK;
#pragma unroll
    for (int q = 0; q < Q; q += 4) {
        const int c = (KG * g + koff + q) >> 2;
        const f32x4 t = *reinterpret_cast<const f32x4*>(row + ((c ^ (xi & 15)) << 2));
        v[q] = t[0];
        v[q + 1] = t[1];
        v[q + 2] = t[2];
        v[q + 3] = t[3];
    }
}

// The K-split partial tiles summed into lds (pitch BN + 4): every K-slice group
// stores its partials in a tile of its own (the stages are free once the loop has
// drained), then each thread adds its positions' KS values in the order K-slice
// 0, 1, ... -- the sums of the one-tile-at-a-time accumulation, with one barrier
// instead of KS.  (r0, c0): the wave's output corner in the tile.
template <class C, int BM, int BN, int NT>
__device__ inline void ksplit_sum(float* lds, const f32x4 (&acc)[C::MB][C::NB], int kh, int r0, int c0, int lane) {
    constexpr int P = BN + 4, TS = BM * P;
    static_assert(C::KS * TS <= LDS_STAGES * 2 * LDS_TILE, "the partial tiles must fit the stages");
#pragma unroll
    for (int a = 0; a < C::MB; ++a)
#pragma unroll
        for (int b = 0; b < C::NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                lds[kh * TS + (r0 + a * 16 + 4 * (lane >> 4) + r) * P + c0 + b * 16 + (lane & 15)] = acc[a][b][r];
    __syncthreads();
    if (C::KS > 1) {
        for (int p = threadIdx.x; p < BM * BN; p += NT) {
            const int q = (p / BN) * P + p % BN;
            float v = lds[q];
#pragma unroll
            for (int h = 1; h < C::KS; ++h) v += lds[h * TS + q];
            lds[q] = v;
        }
        __syncthreads();
    }
}

// NW: waves per workgroup (8: K-split 2, two waves per SIMD; 16: K-split 4,
// four waves per SIMD, half the fragment registers per wave).
template <int BM, int BN, class Epi, int NW = GWAVES>
__global__ void __launch_bounds__(64 * NW) gemm_f32_lds_kernel(Operand A, Operand B, int M, int N, int Kd, Epi epi,
                                                               int sc_a1, int sc_a2, int sc_coef) {
    static_assert(BM == 64 && BN == 64, "64 x 64 output tiles");
    constexpr int NT = 64 * NW;
    constexpr int DMA = dma_per_tile<NW>();
    using C = GemmCore<BM, BN, KCONTIG, KCONTIG, NW>;
    using Frags = typename C::Frags;
    constexpr int MB = C::MB, NB = C::NB;
    // stage s: A tile at lds + 2 s LDS_TILE, B tile right after it
    __shared__ __attribute__((aligned(16))) float lds[LDS_STAGES * 2 * LDS_TILE];
    static_assert(BM * (BN + 4) <= LDS_STAGES * 2 * LDS_TILE, "the epilogue tile must fit");

    const int ntm = M / BM;
    const int ntn = N / BN;
    int tm, tn;
    tile_of(epi, ntm, ntn, tm, tn);
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

    Frags f0, f1;
    const int nkt = Kd / GBK;
    const int last = nkt - 1;
    auto kof = [&](int t) { return min(t, last) * GBK; };
    auto sa = [&](int t) { return lds + (t % LDS_STAGES) * 2 * LDS_TILE; };
    auto sb = [&](int t) { return lds + (t % LDS_STAGES) * 2 * LDS_TILE + LDS_TILE; };
    auto copy = [&](int t) {
        tile_dma<NW>(A, m0, kof(t), sa(t), wave, lane);
        tile_dma<NW>(B, n0, kof(t), sb(t), wave, lane);
    };
    auto read = [&](int t, Frags& f) {
#pragma unroll
        for (int i = 0; i < MB; ++i) frag_read_swz<C::KQ>(sa(t), wr * (BM / C::WM) + i * 16, lane, kh * C::KQ, f.a[i]);
#pragma unroll
        for (int j = 0; j < NB; ++j) frag_read_swz<C::KQ>(sb(t), wc * (BN / C::WN) + j * 16, lane, kh * C::KQ, f.b[j]);
    };

    // prologue: tiles 0, 1, 2 in flight; wait for 0 and 1 (4 copies per tile and wave)
    copy(0);
    copy(1);
    copy(2);
    wait_vm<DMA>();
    __builtin_amdgcn_s_barrier();
    read(0, f0);

    // step t: copy tile t+3 into the stage tile t-1 used (its fragments were read
    // during step t-2), MFMAs of tile t, fragments of tile t+1, wait for tile t+2
    for (int kt = 0; kt < nkt; kt += 2) {
        copy(kt + 3);
        CPA_SCHED_FENCE();
        C::mfma(f0, p0);
        C::add_into(acc, p1);
        read(kt + 1, f1);
        interleave_step<C::kMfma, C::kReads, 0>();
        wait_vm_lds<DMA>();
        __builtin_amdgcn_s_barrier();
        if (kt + 1 >= nkt) {
            C::add_into(acc, p0);
            break;
        }
        copy(kt + 4);
        CPA_SCHED_FENCE();
        C::mfma(f1, p1);
        C::add_into(acc, p0);
        read(kt + 2, f0);
        interleave_step<C::kMfma, C::kReads, 0>();
        wait_vm_lds<DMA>();
        __builtin_amdgcn_s_barrier();
        if (kt + 2 >= nkt) C::add_into(acc, p1);
    }
    // the clamped copies past the last tile may still be landing: drain them
    // before the stages are reused for the epilogue tile
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __syncthreads();

    float* tile = lds;
    ksplit_sum<C, BM, BN, NT>(lds, acc, kh, wr * (BM / C::WM), wc * (BN / C::WN), lane);
    constexpr int NG = BM * BN / 4 / NT;
    static_assert(NG * 4 * NT == BM * BN, "tile must split evenly into float4 groups");
    static_assert(NG == 1 || NT == GTHREADS, "epilogues index float4 groups in steps of GTHREADS");
    epi.template run<BM, BN, NG>(tile, m0, n0, M, N, epi_scal(epi), sc_a1, sc_a2, sc_coef);
}

// ---------------------------------------------------------------------------
// Symmetric products in pieces.  A product whose result is symmetric (every
// product of the matrix-polynomial route is a polynomial in one symmetric
// matrix) needs only the tiles on and above the diagonal: nt (nt + 1) / 2 of the
// nt x nt tiles of 64.  At nt = 16 that is 136 tiles for 256 CUs, one round
// either way.  The pieces below give every CU less work instead: each tile above
// the diagonal is split into its two 64 x 32 column halves (eight 16 x 16 MFMA
// blocks each) and each diagonal tile keeps the blocks on or above its diagonal
// (ten): nt^2 pieces, as many as the tiles of the full product, with at most 10
// of 16 blocks per workgroup.
//
// Waves: the 64 x 64 tile is four 32 x 32 quadrants of 2 x 2 blocks.  A half
// piece has two quadrants, a diagonal piece three ((0,0), (0,1), (1,1)); wave w
// < 4 nq takes quadrant slot w / 4 over K-slice w % 4 (the K-split of the full
// kernel), so each SIMD (w % 4) holds one wave of every quadrant and the MFMA
// count per SIMD is even: 32 blocks x K-steps on a half piece, 40 on a diagonal
// one (whose diagonal quadrants skip the block below their diagonal).  Waves past
// 4 nq only copy tiles.  Operand tiles are copied whole (the B tile of a half
// piece is used in one half), by the same four-stage direct global-to-LDS
// pipeline as gemm_f32_lds_kernel.
//
// Stores: each piece writes its blocks and their mirror images, a diagonal piece
// its upper triangle mirrored onto the lower one, so the result is exactly
// symmetric (Epi::run_piece: the linear epilogue reads C and Mx at the stored,
// upper positions only; the Gram epilogue adds the piece's share of ||G||_F^2
// and of the trace).

// X^T into a k-contiguous operand: Xt[j][i] = X[i][j] (i < m, j < n), and 0 for
// m <= i < ldt, the padding of the contraction length to a multiple of 64.  One
// 64 x 64 block per workgroup (256 threads) through LDS, so that both the reads
// of X and the writes of Xt are row segments.  Grid (ldt / 64, ceil(n / 64)).
__global__ void __launch_bounds__(256) transpose_pad_kernel(int m, int n, const float* X, int64_t ldx, float* Xt,
                                                            int64_t ldt) {
    __shared__ float blk[64][65];
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = i0 + ty + 4 * q, j = j0 + tx;
        blk[ty + 4 * q][tx] = (i < m && j < n) ? X[(int64_t)i * ldx + j] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int j = j0 + ty + 4 * q, i = i0 + tx;
        if (j < n) Xt[(int64_t)j * ldt + i] = blk[tx][ty + 4 * q];
    }
}

// Piece of workgroup blockIdx.x among the nt^2: the diagonal pieces (the longest,
// ten blocks) come first, so they are dispatched first, and, when nt^2 % 8 == 0,
// they take the first slots of every XCD's range (dispatch is round-robin over
// the 8 XCDs and workgroup b runs on XCD b % 8: range x holds the virtual pieces
// x nt^2 / 8 ..), spreading them over the XCDs' L2 caches; the half pieces follow,
// half h % 2 of the h / 2-th tile above the diagonal in row-major order, so
// neighbouring workgroups of an XCD share operand panels.  half = -1 on a
// diagonal piece.
__device__ inline void piece_of(int nt, int& tm, int& tn, int& half) {
    const int P = nt * nt;
    int h;
    const int b = blockIdx.x;
    if (P % 8 == 0) {
        const int per = P / 8, x = b % 8, slot = b / 8;
        const int ndx = (nt - x + 7) / 8;   // diagonal tiles t with t % 8 == x
        if (slot < ndx) {
            tm = tn = x + 8 * slot;
            half = -1;
            return;
        }
        // diagonal pieces in the ranges 0..x (those of range x precede this slot)
        int before = 0;
        for (int y = 0; y <= x; ++y) before += (nt - y + 7) / 8;
        h = x * per + slot - before;
    } else {
        if (b < nt) {
            tm = tn = b;
            half = -1;
            return;
        }
        h = b - nt;
    }
    int q = h >> 1;
    half = h & 1;
    int r = 0;
    while (q >= nt - 1 - r) {
        q -= nt - 1 - r;
        ++r;
    }
    tm = r;
    tn = r + 1 + q;
}

// MFMAs of one K-tile for a wave's quadrant into the fresh partial `part`; on a
// diagonal quadrant the block below its diagonal (i = 1, j = 0) is skipped.
template <class C, bool DIAG>
__device__ inline void mfma_quadrant(const typename C::Frags& f, f32x4 (&part)[C::MB][C::NB]) {
#pragma unroll
    for (int i = 0; i < C::MB; ++i)
#pragma unroll
        for (int j = 0; j < C::NB; ++j) part[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < C::KQ; ++kk)
#pragma unroll
        for (int i = 0; i < C::MB; ++i)
#pragma unroll
            for (int j = 0; j < C::NB; ++j)
                if (!(DIAG && i > j))
                    part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(f.a[i][kk], f.b[j][kk], part[i][j], 0, 0, 0);
}

template <class Epi>
__global__ void __launch_bounds__(1024) gemm_f32_piece_kernel(Operand A, Operand B, int M, int Kd, Epi epi) {
    constexpr int NW = 16, BM = 64, BN = 64;
    constexpr int DMA = dma_per_tile<NW>();
    using C = GemmCore<BM, BN, KCONTIG, KCONTIG, NW>;
    using Frags = typename C::Frags;
    constexpr int MB = C::MB, NB = C::NB;
    static_assert(MB == 2 && NB == 2 && C::KS == 4, "quadrants of 2 x 2 blocks over a K-split of four");
    __shared__ __attribute__((aligned(16))) float lds[LDS_STAGES * 2 * LDS_TILE];

    const int nt = M / 64;
    int tm, tn, half;
    piece_of(nt, tm, tn, half);
    const int m0 = tm * 64, n0 = tn * 64;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nq = half < 0 ? 3 : 2;
    const bool active = wave < 4 * nq;
    const int qi = wave >> 2, kh = wave & 3;
    // quadrant (qr, qc) of the tile: a half piece's column half, or (0,0), (0,1), (1,1)
    const int qr = half >= 0 ? qi : (qi == 2 ? 1 : 0);
    const int qc = half >= 0 ? half : (qi >= 1 ? 1 : 0);
    const bool diagq = half < 0 && qr == qc;

    f32x4 acc[MB][NB], p0[MB][NB], p1[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = p0[i][j] = p1[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

    Frags f0, f1;
    const int nkt = Kd / GBK;
    const int last = nkt - 1;
    auto kof = [&](int t) { return min(t, last) * GBK; };
    auto sa = [&](int t) { return lds + (t % LDS_STAGES) * 2 * LDS_TILE; };
    auto sb = [&](int t) { return lds + (t % LDS_STAGES) * 2 * LDS_TILE + LDS_TILE; };
    auto copy = [&](int t) {
        tile_dma<NW>(A, m0, kof(t), sa(t), wave, lane);
        tile_dma<NW>(B, n0, kof(t), sb(t), wave, lane);
    };
    auto read = [&](int t, Frags& f) {
#pragma unroll
        for (int i = 0; i < MB; ++i) frag_read_swz<C::KQ>(sa(t), qr * 32 + i * 16, lane, kh * C::KQ, f.a[i]);
#pragma unroll
        for (int j = 0; j < NB; ++j) frag_read_swz<C::KQ>(sb(t), qc * 32 + j * 16, lane, kh * C::KQ, f.b[j]);
    };

    // the pipeline of gemm_f32_lds_kernel in three straight-line variants (MODE 0:
    // copies only, 1: a full quadrant, 2: a diagonal quadrant); every wave runs the
    // same sequence of copies and barriers
    auto pipeline = [&](auto mode) {
        constexpr int MODE = decltype(mode)::value;
        constexpr int NMF = MODE == 2 ? C::kMfma * 3 / 4 : C::kMfma;
        copy(0);
        copy(1);
        copy(2);
        wait_vm<DMA>();
        __builtin_amdgcn_s_barrier();
        if constexpr (MODE > 0) read(0, f0);
        for (int kt = 0; kt < nkt; kt += 2) {
            copy(kt + 3);
            CPA_SCHED_FENCE();
            if constexpr (MODE > 0) {
                mfma_quadrant<C, MODE == 2>(f0, p0);
                C::add_into(acc, p1);
                read(kt + 1, f1);
                interleave_step<NMF, C::kReads, 0>();
            }
            wait_vm_lds<DMA>();
            __builtin_amdgcn_s_barrier();
            if (kt + 1 >= nkt) {
                if constexpr (MODE > 0) C::add_into(acc, p0);
                break;
            }
            copy(kt + 4);
            CPA_SCHED_FENCE();
            if constexpr (MODE > 0) {
                mfma_quadrant<C, MODE == 2>(f1, p1);
                C::add_into(acc, p0);
                read(kt + 2, f0);
                interleave_step<NMF, C::kReads, 0>();
            }
            wait_vm_lds<DMA>();
            __builtin_amdgcn_s_barrier();
            if constexpr (MODE > 0)
                if (kt + 2 >= nkt) C::add_into(acc, p1);
        }
    };
    if (!active)
        pipeline(std::integral_constant<int, 0>());
    else if (diagq)
        pipeline(std::integral_constant<int, 2>());
    else
        pipeline(std::integral_constant<int, 1>());
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __syncthreads();

    // K-split partials summed in a fixed order (K-slice 0, 1, 2, 3) into the tile
    // (waves without a quadrant store nothing: the positions they would cover are
    // never stored)
    float* tile = lds;
    if (active) {
        constexpr int TS = BM * (BN + 4);
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    lds[kh * TS + (qr * 32 + a * 16 + 4 * (lane >> 4) + r) * (BN + 4) + qc * 32 + b * 16 + (lane & 15)] =
                        acc[a][b][r];
    }
    __syncthreads();
    for (int p = threadIdx.x; p < BM * BN; p += 1024) {
        constexpr int TS = BM * (BN + 4);
        const int q = (p / BN) * (BN + 4) + p % BN;
        lds[q] = ((lds[q] + lds[TS + q]) + lds[2 * TS + q]) + lds[3 * TS + q];
    }
    __syncthreads();
    epi.run_piece(tile, m0, n0, half);
}

// Symmetric products of side M <= kSymSmallMax (the linear epilogue, Kd = M, both
// operands k-contiguous with 16-byte rows).  In pieces such a product has only
// (M / 64)^2 <= 64 workgroups, each with the whole K loop of a 64 x 64 piece
// behind its pipeline's fill.  Here each workgroup takes one 32 x 32 tile on or
// above the diagonal (nt (nt + 1) / 2 of them, nt = M / 32) and loads its 32 rows
// of A and of B whole into LDS (one round trip: every load is issued before the
// first store).  Wave w computes the 16 x 16 block w % 4 of the tile over half of
// K (w / 4), one fresh partial sum per 64 k added into its accumulator; the two
// halves are added in LDS in a fixed order (first half + second half).  The
// epilogue is EpiLin's: o = alpha acc + beta C + gamma Mx (+ delta on the
// diagonal), read at the tile's positions, stored as the tile and its mirror (a
// diagonal tile from its upper triangle), so D comes out exactly symmetric; C may
// be D (no other workgroup reads this tile's positions).
constexpr int kSymSmallMax = 512;
constexpr int kSymSmallThreads = 512;

__global__ void __launch_bounds__(kSymSmallThreads) gemm_f32_sym_small_kernel(Operand A, Operand B, int M, EpiLin epi) {
    constexpr int T = 32;                    // tile side
    constexpr int KP = kSymSmallMax + 4;     // LDS pitch of the operand rows (floats)
    constexpr int TP = T + 4;                // LDS pitch of the result tile
    __shared__ __attribute__((aligned(16))) float sa[T * KP];
    __shared__ __attribute__((aligned(16))) float sb[T * KP];
    __shared__ __attribute__((aligned(16))) float tile[T * TP];
    const int nt = M / T;
    // the tile of this workgroup: upper-triangle tiles in row order
    int tm = 0, rem = blockIdx.x;
    while (rem >= nt - tm) {
        rem -= nt - tm;
        ++tm;
    }
    const int tn = tm + rem;
    const int m0 = tm * T, n0 = tn * T;
    const int Kd = M;
    const int gpr = Kd / 4;   // float4 groups per row
    {
        // thread t: float4 column group t % CG of rows t / CG + RPH u (every load
        // issued before the first store)
        constexpr int CG = kSymSmallMax / 4;          // groups of a full-width row
        constexpr int RPH = kSymSmallThreads / CG;    // row phases
        constexpr int NR = T / RPH;                   // rows per thread
        const int cg = threadIdx.x % CG, rp = threadIdx.x / CG;
        if (cg < gpr) {
            const float* ga = A.p + (int64_t)(m0 + rp) * A.ld + 4 * cg;
            const float* gb = B.p + (int64_t)(n0 + rp) * B.ld + 4 * cg;
            f32x4 ra[NR], rb[NR];
#pragma unroll
            for (int u = 0; u < NR; ++u) {
                ra[u] = *reinterpret_cast<const f32x4*>(ga + (int64_t)(RPH * u) * A.ld);
                rb[u] = *reinterpret_cast<const f32x4*>(gb + (int64_t)(RPH * u) * B.ld);
            }
#pragma unroll
            for (int u = 0; u < NR; ++u) {
                *reinterpret_cast<f32x4*>(sa + (rp + RPH * u) * KP + 4 * cg) = ra[u];
                *reinterpret_cast<f32x4*>(sb + (rp + RPH * u) * KP + 4 * cg) = rb[u];
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int br = ((wave & 3) >> 1) * 16, bc = (wave & 1) * 16, kh = wave >> 2;
    const int li = lane & 15, lg = lane >> 4;
    const int khalf = Kd / 2;   // a multiple of 16
    const float* pa = sa + (br + li) * KP + kh * khalf + 4 * lg;
    const float* pb = sb + (bc + li) * KP + kh * khalf + 4 * lg;
    f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < khalf; k0 += 64) {
        f32x4 part = (f32x4){0.f, 0.f, 0.f, 0.f};
        const int kend = min(khalf - k0, 64);
        for (int kk = 0; kk < kend; kk += 16) {
            // lane group lg supplies k = k0 + kk + 4 lg + t to the t-th product
            const f32x4 a4 = *reinterpret_cast<const f32x4*>(pa + k0 + kk);
            const f32x4 b4 = *reinterpret_cast<const f32x4*>(pb + k0 + kk);
#pragma unroll
            for (int t = 0; t < 4; ++t) part = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[t], b4[t], part, 0, 0, 0);
        }
        acc += part;
    }
    // lane (li, lg) holds rows br + 4 lg + r, column bc + li of the tile
    if (kh == 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tile[(br + 4 * lg + r) * TP + bc + li] = acc[r];
    }
    __syncthreads();
    if (kh == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float& t = tile[(br + 4 * lg + r) * TP + bc + li];
            t = acc[r] + t;
        }
    }
    __syncthreads();
    // epilogue: 32 rows x 8 float4 groups on the first 256 threads
    const bool mine = threadIdx.x < T * (T / 4);
    const int r = threadIdx.x / (T / 4), cc = (threadIdx.x % (T / 4)) * 4;
    const int i = m0 + r, j = n0 + cc;
    f32x4 o = (f32x4){0.f, 0.f, 0.f, 0.f};
    if (mine) {
        const f32x4 a = *reinterpret_cast<const f32x4*>(tile + r * TP + cc);
        f32x4 vd = (f32x4){0.f, 0.f, 0.f, 0.f}, vm = vd;
        if (epi.beta != 0.f) vd = *reinterpret_cast<const f32x4*>(epi.C + (int64_t)i * epi.ldc + j);
        if (epi.gamma != 0.f) vm = *reinterpret_cast<const f32x4*>(epi.Mx + (int64_t)i * epi.ldm + j);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float v = epi.alpha * a[e] + epi.beta * vd[e] + epi.gamma * vm[e];
            if (i == j + e) v += epi.delta;
            o[e] = v;
        }
    }
    __syncthreads();   // every product value read before the tile is overwritten
    if (mine) *reinterpret_cast<f32x4*>(tile + r * TP + cc) = o;
    __syncthreads();
    if (!mine) return;
    const bool diag = m0 == n0;
    f32x4 v, w;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = cc + e;
        v[e] = (!diag || r <= c) ? tile[r * TP + c] : tile[c * TP + r];
        w[e] = tile[c * TP + r];
    }
    *reinterpret_cast<f32x4*>(epi.D + (int64_t)i * epi.ldd + j) = v;
    if (!diag) *reinterpret_cast<f32x4*>(epi.D + (int64_t)(n0 + r) * epi.ldd + m0 + cc) = w;
}

}  // namespace cpa
