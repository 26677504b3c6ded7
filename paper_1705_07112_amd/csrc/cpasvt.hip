// Host side of the C ABI declared in include/cpasvt.h: argument checks,
// workspace, and the launch sequence of one shrink
//   Gram (MFMA) -> bound (power iteration / given / Frobenius) -> FP64
//   coefficients on the device -> K-1 fused recurrence GEMMs
// plus the RPCA ADMM driver around it.  Everything is enqueued on the
// caller's stream; only calls that report host values synchronise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/cpasvt.h"
#include "admm.hpp"
#include "batched.hpp"
#include "design.hpp"
#include "sparse.hpp"
#include "sparsify.hpp"
#include "inpaint.hpp"
#include "fp64.hpp"
#include "gemm_bf16x3.hpp"
#include "gemm_f32.hpp"
#include "gemm_lds.hpp"
#include "peak.hpp"
#include "shrink_fn.hpp"
#include "spectral.hpp"

using namespace cpa;

namespace {

thread_local char g_err[512] = "";

cpa_status fail(cpa_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return fail(CPA_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxPowerIters = 1000;
constexpr int kAdmmGrid = 2048;   // workgroups of the ADMM elementwise kernels
constexpr int kAdmmChunk = 8;     // ADMM iterations in the longer captured graph (one launch between them)
constexpr int kMaxK = 4096;
constexpr int kMaxDesignK = 1024;        // cpa_design_coeffs orders
constexpr int kMaxDesignN = 1 << 20;     // and sample / grid points
constexpr int64_t kMaxDesignNK = int64_t(1) << 26;   // n K: 512 MiB of basis values

}  // namespace

// Event pairs bracketing individual launches of one kernel family, for
// per-launch timing with HIP events on the caller's stream.
struct TimingLog {
    std::vector<hipEvent_t> ev;   // start/end pairs, reused between records
    size_t used = 0;              // pairs recorded since the last reset
};

// ---- scratch of the allocation-free dense shrink ---------------------------------
// The workspace of cpa_shrink_dense_noalloc lives in this array.  Every GPU that
// loads the library holds its own copy until the process ends.  In host code the
// name only identifies the symbol: kernels receive the device address that
// hipGetSymbolAddress returned for that device (kept per device at cpa_create),
// never the name.  Layout: the power iteration's warm-start vector at offset 0
// (kScratchWarmBytes, for d <= kScratchMaxD), then the shrink's workspace.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchMaxD = 4096;
constexpr size_t kScratchWarmBytes = sizeof(double) * kScratchMaxD;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];      // device address of `scratch` on each device (nullptr: not yet)
int g_scratch_warm_d[kMaxDevices];     // length of the warm vector stored there (-1: none)
}  // namespace

struct cpa_ctx {
    int device = 0;
    void* scratch = nullptr;   // this device's address of the allocation-free entry point's scratch
    int timing = 0;               // 1: bracket launches with events
    TimingLog tlog[3];            // 0: recurrence and full polynomial GEMMs, 1: Gram GEMMs, 2: symmetric pieces
    void* ws = nullptr;        // main workspace
    size_t ws_bytes = 0;
    double* warm = nullptr;    // warm-start vector for power iteration
    int warm_cap = 0;
    int warm_d = -1;           // length of the stored vector, -1 if none
    int coop_max = 0;          // co-resident power-iteration workgroups (0: not queried)
    void* spf = nullptr;       // sparsified path: Phi, CSR of the truncated matrix, Psi buffers, H, M, selection state
    size_t spf_bytes = 0;
    int spf_dct_d = 0;         // the full-DCT matrices in spf are built for this side (0: none)
    int spf_last_d = 0;        // the side of the last sparsified call (the layout depends on it)
    int spf_warm_d = -1;       // side of the full-coordinate warm vector in spf (-1: none)
    int32_t* spf_host = nullptr;   // pinned host word: the compact block's size, read back per call
    void* inp = nullptr;       // inpainting driver: DCT matrices, product scratch, partial sums
    size_t inp_bytes = 0;
    void* f64 = nullptr;       // FP64 shrink: Gram, two Y buffers, product buffer
    size_t f64_bytes = 0;
    void* rpca = nullptr;      // one-call RPCA driver: its state and E_t slot
    size_t rpca_bytes = 0;
    int batch_per_cu = 0;      // co-resident workgroups of the batched kernel per CU (0: not queried)
    int cus = 0;
    int* queue = nullptr;      // work-queue counter of the batched kernel
    void* mlp_ws = nullptr;    // predictor training: gradient partials | loss partials
    // sparse path: its own workspace and the cached transposed pattern
    void* sws = nullptr;
    size_t sws_bytes = 0;
    int32_t* csc = nullptr;    // colptr[n+1] | crow[nnz] | csrc[nnz] | scratch[max(n, 2 nnz)]
    size_t csc_bytes = 0;
    const int32_t* csc_rowptr = nullptr;
    const int32_t* csc_colidx = nullptr;
    int csc_m = -1, csc_n = -1;
    int64_t csc_nnz = -1;
    // captured ADMM iterations (one, and kAdmmChunk in a row), replayed while their
    // key matches
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t admm_exec = nullptr;
    hipGraphExec_t admm_exec_chunk = nullptr;
    std::vector<char> admm_key;
};

namespace {

// Returns the event pair for the next launch of family `which` (nullptrs when timing is off).
cpa_status timing_pair(cpa_ctx* ctx, int which, hipEvent_t& a, hipEvent_t& b) {
    a = b = nullptr;
    if (!ctx || !ctx->timing) return CPA_OK;
    TimingLog& L = ctx->tlog[which];
    if (2 * (L.used + 1) > L.ev.size()) {
        for (int q = 0; q < 2; ++q) {
            // timing only: no system-scope fence (cache write-back) when the event is recorded
            hipEvent_t e;
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            L.ev.push_back(e);
        }
    }
    a = L.ev[2 * L.used];
    b = L.ev[2 * L.used + 1];
    ++L.used;
    return CPA_OK;
}

struct Work {
    float* G;
    float* Yb[2];
    double* w[2];
    double* scal;
    float* x;      // ADMM shrink input
    double* admm;  // ADMM E_t partial sums (2 per pre-kernel workgroup)
    int* et_counter;  // next E_t slot
    float* poly;      // matrix-polynomial route: T_1..T_s, R_0..R_{J-1}, three Clenshaw buffers (d x d each)
    int poly_s;       // s of that route (0: not allocated)
    float* xt = nullptr;   // room for X^T (padded) while the Gram is formed: the polynomial buffers on
                           // that route, else the first Y buffer of the recurrence (free until then)
    int64_t xt_cap = 0;    // its capacity in floats (0: none)
    int64_t yb_cap = 0;    // floats in each Y buffer (0: none)
    bool right;       // Gram = X^T X (n x n) and products on the right; else X X^T (m x m), on the left
    int d;            // side of the Gram
    ScalarLayout lay;
    // warm-start vector of the power iteration and the length of what it holds
    // (-1: nothing); nullptr: the context's
    double* warm_vec = nullptr;
    int* warm_len = nullptr;
};

// The Gram side: CPA_SIDE_AUTO takes the smaller one (X^T X when m >= n).
bool right_side(const cpa_opts* o, int m, int n) {
    return o->side == CPA_SIDE_AUTO ? m >= n : o->side == CPA_SIDE_RIGHT;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Matrices of d x d held by the matrix-polynomial route: T_1..T_s, R_0..R_{J-1},
// three Clenshaw buffers.
int poly_mats(int K, int s) { return s + (K + s - 1) / s + 3; }

int gram_grid(int d) {
    return ((d + 63) / 64) * ((d + 63) / 64);
}

// The power kernels synchronise their workgroups with a bounded grid barrier.
// With at most one workgroup per CU every workgroup runs, or starts as soon as a
// CU frees up (the waiting ones hold at most `grid` CUs, and other work on the
// device ends), so a plain launch reaches every barrier; the cooperative launch,
// which leaves the device idle around it in a captured graph, is kept for larger
// grids.
cpa_status launch_power(cpa_ctx* ctx, const void* fn, int grid, void** args, hipStream_t st) {
    if (ctx->cus == 0) {
        int cus = 0;
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        ctx->cus = std::max(1, cus);
    }
    if (grid <= ctx->cus)
        HIP_TRY(hipLaunchKernel(fn, dim3(grid), dim3(kPowerThreads), args, 0, st));
    else
        HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kPowerThreads), args, 0, st));
    return CPA_OK;
}

// Power-iteration workgroups: about 16 rows each, at most 64 (the grid barrier
// is one counter; few arrivals keep it cheap), never above what is co-resident.
int power_grid(cpa_ctx* ctx, int d) {
    int want = std::max(1, std::min(64, (d + 15) / 16));
    if (ctx->coop_max > 0) want = std::min(want, ctx->coop_max);
    return want;
}

// Co-resident workgroups of the power kernel (queried once per context).
cpa_status query_coop(cpa_ctx* ctx) {
    if (ctx->coop_max == 0) {
        int per_cu = 0, cus = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, power_coop_kernel<float>, kPowerThreads, 0));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        ctx->coop_max = std::max(1, per_cu * cus);
    }
    return CPA_OK;
}

// Byte offsets of the dense workspace regions.  need_y: the two m x n ping-pong
// buffers of the recurrence over X (the matrix-polynomial route does without).
// warm: a d-double warm-start vector at the end (the allocation-free entry point
// keeps it there; the other entry points keep theirs in the context).
struct WsPlan {
    size_t oG = 0, oY0 = 0, oY1 = 0, ow0 = 0, ow1 = 0, os = 0, opl = 0, ox = 0, oa = 0, owarm = 0, total = 0;
};

WsPlan plan_ws(int m, int n, int K, int maxit, bool admm, Work& w, bool right, int poly_s, int pwg, bool need_y,
               bool warm) {
    const int d = right ? n : m;
    w.right = right;
    w.d = d;
    const int64_t mn = (int64_t)m * n;
    w.lay.K = K;
    w.lay.maxit = maxit;
    w.lay.gwg = gram_grid(d);
    w.lay.pwg = pwg;
    WsPlan p;
    size_t off = 0;
    p.oG = off; off = align_up(off + sizeof(float) * (size_t)d * d);
    if (need_y) {
        p.oY0 = off; off = align_up(off + sizeof(float) * (size_t)mn);
        p.oY1 = off; off = align_up(off + sizeof(float) * (size_t)mn);
    }
    p.ow0 = off; off = align_up(off + sizeof(double) * (size_t)d);
    p.ow1 = off; off = align_up(off + sizeof(double) * (size_t)d);
    p.os = off; off = align_up(off + sizeof(double) * (size_t)w.lay.total());
    if (poly_s > 0) { p.opl = off; off = align_up(off + sizeof(float) * (size_t)poly_mats(K, poly_s) * d * d); }
    if (admm) {
        p.ox = off; off = align_up(off + sizeof(float) * (size_t)mn);
        p.oa = off; off = align_up(off + sizeof(double) * 2 * kAdmmGrid + 256);
    }
    if (warm) { p.owarm = off; off = align_up(off + sizeof(double) * (size_t)std::max(d, 1)); }
    p.total = off;
    return p;
}

void bind_ws(Work& w, char* b, const WsPlan& p, bool admm, int poly_s, bool need_y) {
    w.G = reinterpret_cast<float*>(b + p.oG);
    w.Yb[0] = need_y ? reinterpret_cast<float*>(b + p.oY0) : nullptr;
    w.Yb[1] = need_y ? reinterpret_cast<float*>(b + p.oY1) : nullptr;
    w.w[0] = reinterpret_cast<double*>(b + p.ow0);
    w.w[1] = reinterpret_cast<double*>(b + p.ow1);
    w.scal = reinterpret_cast<double*>(b + p.os);
    w.x = admm ? reinterpret_cast<float*>(b + p.ox) : nullptr;
    w.admm = admm ? reinterpret_cast<double*>(b + p.oa) : nullptr;
    w.et_counter = admm ? reinterpret_cast<int*>(b + p.oa + sizeof(double) * 2 * kAdmmGrid) : nullptr;
    w.poly = poly_s > 0 ? reinterpret_cast<float*>(b + p.opl) : nullptr;
    w.poly_s = poly_s;
    w.yb_cap = need_y ? (int64_t)(p.oY1 - p.oY0) / (int64_t)sizeof(float) : 0;
    if (poly_s > 0) {
        w.xt = w.poly;
        w.xt_cap = (int64_t)poly_mats(w.lay.K, poly_s) * w.d * w.d;
    } else {
        w.xt = w.Yb[0];
        w.xt_cap = w.Yb[0] ? (int64_t)(p.oY1 - p.oY0) / (int64_t)sizeof(float) : 0;
    }
}

// size_only != nullptr: report the bytes of the main workspace and the power
// vector this call needs and allocate nothing.
cpa_status ensure_ws(cpa_ctx* ctx, int m, int n, int K, int maxit, bool admm, Work& w, bool right, int poly_s = 0,
                     size_t* size_only = nullptr) {
    cpa_status s;
    if ((s = query_coop(ctx)) != CPA_OK) return s;
    const int d = right ? n : m;
    const WsPlan p = plan_ws(m, n, K, maxit, admm, w, right, poly_s, power_grid(ctx, d), true, false);
    const size_t off = p.total;
    if (size_only) {
        *size_only = off + sizeof(double) * (size_t)std::max(d, 1);
        return CPA_OK;
    }
    if (off > ctx->ws_bytes) {
        if (ctx->ws) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ctx->ws));
            ctx->ws = nullptr;
            ctx->ws_bytes = 0;
        }
        if (hipMalloc(&ctx->ws, off) != hipSuccess) {
            ctx->ws = nullptr;
            return fail(CPA_ERR_ALLOC, "workspace allocation of %zu bytes failed", off);
        }
        ctx->ws_bytes = off;
    }
    bind_ws(w, static_cast<char*>(ctx->ws), p, admm, poly_s, true);
    if (d > ctx->warm_cap) {
        if (ctx->warm) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ctx->warm));
        }
        ctx->warm = nullptr;
        if (hipMalloc(&ctx->warm, sizeof(double) * (size_t)std::max(d, 1)) != hipSuccess) {
            ctx->warm_cap = 0;
            ctx->warm_d = -1;
            return fail(CPA_ERR_ALLOC, "warm-start vector allocation failed");
        }
        ctx->warm_cap = std::max(d, 1);
        ctx->warm_d = -1;
    }
    return CPA_OK;
}

bool aligned16(const float* p, int64_t ld) {
    return (ld % 4 == 0) && ((reinterpret_cast<uintptr_t>(p) & 15) == 0);
}

Operand make_op(const float* p, int64_t ld, int xdim) {
    Operand o;
    o.p = p;
    o.ld = ld;
    o.xdim = xdim;
    return o;
}

// 16-byte tile loads need an aligned base, ld % 4 == 0, and a vectorised extent
// (x for XCONTIG, k for KCONTIG) that is a multiple of 4 and at least 4.
bool vec_operand(const Operand& o, int layout, int Kd) {
    const int run = layout == XCONTIG ? o.xdim : Kd;
    return aligned16(o.p, o.ld) && run % 4 == 0 && run >= 4;
}

// Workgroups of a product: every tile, or the upper-triangle tiles of a
// symmetric one (M == N).
template <class Epi>
int gemm_grid(int ntm, int ntn, const Epi& epi) {
    return epi_sym(epi) ? ntm * (ntm + 1) / 2 : ntm * ntn;
}

// A symmetric product that cannot run in pieces runs as upper-triangle tiles.
template <class Epi>
Epi tiles_not_pieces(const Epi& e) {
    return e;
}
template <>
EpiLin tiles_not_pieces<EpiLin>(const EpiLin& e) {
    EpiLin r = e;
    if (r.sym == 2) r.sym = 1;
    return r;
}

template <int BM, int BN, int LA, int LB, class Epi>
cpa_status launch_gemm(hipStream_t st, const Operand& A, const Operand& B, int M, int N, int Kd, const Epi& epi,
                       int sc_a1, int sc_a2, int sc_coef) {
    const int ntm = (M + BM - 1) / BM, ntn = (N + BN - 1) / BN;
    if (epi_sym(epi) && M != N) return fail(CPA_ERR_ARG, "internal: a symmetric product must be square");
    const Epi et = tiles_not_pieces(epi);
    const int grid = gemm_grid(ntm, ntn, et);
    if (grid <= 0 || Kd <= 0) return CPA_OK;
    if (vec_operand(A, LA, Kd) && vec_operand(B, LB, Kd))
        hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, LA, LB, true, Epi>), dim3(grid), dim3(GTHREADS), 0, st, A, B, M,
                           N, Kd, et, sc_a1, sc_a2, sc_coef);
    else
        hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, LA, LB, false, Epi>), dim3(grid), dim3(GTHREADS), 0, st, A, B,
                           M, N, Kd, et, sc_a1, sc_a2, sc_coef);
    HIP_TRY(hipGetLastError());
    return CPA_OK;
}

template <int LA, int LB, class Epi>
cpa_status launch_gemm_split(hipStream_t st, const Operand& A, const Operand& B, int M, int N, int Kd,
                             const Epi& epi, int sc_a1, int sc_a2, int sc_coef) {
    if (epi_sym(epi)) return fail(CPA_ERR_ARG, "internal: the split-precision products have no symmetric mode");
    const int grid = ((M + 63) / 64) * ((N + 63) / 64);
    if (grid <= 0 || Kd <= 0) return CPA_OK;
    if (vec_operand(A, LA, Kd) && vec_operand(B, LB, Kd))
        hipLaunchKernelGGL((gemm_bf16x3_kernel<64, 64, LA, LB, true, Epi>), dim3(grid), dim3(GTHREADS), 0, st, A, B,
                           M, N, Kd, epi, sc_a1, sc_a2, sc_coef);
    else
        hipLaunchKernelGGL((gemm_bf16x3_kernel<64, 64, LA, LB, false, Epi>), dim3(grid), dim3(GTHREADS), 0, st, A, B,
                           M, N, Kd, epi, sc_a1, sc_a2, sc_coef);
    HIP_TRY(hipGetLastError());
    return CPA_OK;
}

// Full 64 x 64 tiles of two k-contiguous operands: the direct global-to-LDS
// pipeline applies.
bool lds_pipeline_ok(const Operand& A, const Operand& B, int M, int N, int Kd) {
    return M > 0 && N > 0 && Kd > 0 && M % 64 == 0 && N % 64 == 0 && Kd % GBK == 0 && aligned16(A.p, A.ld) &&
           aligned16(B.p, B.ld);
}

// All products use 64 x 64 output tiles: at 1024 x 1024 that is 256 workgroups,
// one per CU, and larger outputs simply have more of them.
template <int LA, int LB, class Epi>
cpa_status gemm_dispatch(hipStream_t st, const Operand& A, const Operand& B, int M, int N, int Kd, const Epi& epi,
                         int sc_a1, int sc_a2, int sc_coef) {
    // the linear-epilogue products of the matrix-polynomial route: direct
    // global-to-LDS copies, 16 waves (measured: 27.2 us vs 27.8 us at 1024^3;
    // the Chebyshev and Gram epilogues run faster on the register-staged kernel)
    if constexpr (LA == KCONTIG && LB == KCONTIG && std::is_same<Epi, EpiLin>::value) {
        if (lds_pipeline_ok(A, B, M, N, Kd)) {
            if (epi_sym(epi) && M != N) return fail(CPA_ERR_ARG, "internal: a symmetric product must be square");
            if (epi.sym == 2 && epi.vec_ok && M <= kSymSmallMax && Kd == M) {
                // small symmetric product: one 32 x 32 tile on or above the diagonal per workgroup
                const int nt = M / 32;
                hipLaunchKernelGGL(gemm_f32_sym_small_kernel, dim3(nt * (nt + 1) / 2), dim3(kSymSmallThreads), 0, st,
                                   A, B, M, epi);
                HIP_TRY(hipGetLastError());
                return CPA_OK;
            }
            if (epi.sym == 2 && epi.vec_ok) {
                // symmetric product in pieces: (M / 64)^2 workgroups
                hipLaunchKernelGGL(gemm_f32_piece_kernel<EpiLin>, dim3((M / 64) * (M / 64)), dim3(1024), 0, st, A, B,
                                   M, Kd, epi);
                HIP_TRY(hipGetLastError());
                return CPA_OK;
            }
            const Epi et = tiles_not_pieces(epi);
            const int grid = gemm_grid(M / 64, N / 64, et);
            hipLaunchKernelGGL((gemm_f32_lds_kernel<64, 64, Epi, 16>), dim3(grid), dim3(1024), 0, st, A, B, M, N, Kd,
                               et, sc_a1, sc_a2, sc_coef);
            HIP_TRY(hipGetLastError());
            return CPA_OK;
        }
    }
    return launch_gemm<64, 64, LA, LB>(st, A, B, M, N, Kd, epi, sc_a1, sc_a2, sc_coef);
}

ShrinkParams to_params(const cpa_shrinkage* s) {
    ShrinkParams p;
    p.kind = s->kind;
    p.tau = s->tau;
    p.w_c = s->w_c;
    p.w_sigma = s->w_sigma;
    p.w_eps = s->w_eps;
    return p;
}

cpa_status check_shrinkage(const cpa_shrinkage* s) {
    if (!s) return fail(CPA_ERR_ARG, "shrinkage is NULL");
    if (s->kind < 0 || s->kind > 3) return fail(CPA_ERR_ARG, "unknown shrinkage kind %d", s->kind);
    if (s->kind != CPA_WEIGHTED_FN && !(std::isfinite(s->tau) && s->tau >= 0.0))
        return fail(CPA_ERR_ARG, "tau must be finite and >= 0");
    if (s->kind == CPA_WEIGHTED_FN &&
        !(std::isfinite(s->w_c) && std::isfinite(s->w_sigma) && s->w_eps > 0.0 && s->w_c >= 0.0))
        return fail(CPA_ERR_ARG, "weighted function needs finite w_c >= 0, w_sigma and w_eps > 0");
    return CPA_OK;
}

// The learned bound rule is the dense single-matrix paths' (the batched path
// takes the predictor through cpa_shrink_batched_predicted); caller-given
// coefficients are the single-matrix FP32 shrinks' (dense and CSR).
cpa_status no_given_coeffs(const cpa_opts* o) {
    if (o->coeffs)
        return fail(CPA_ERR_UNSUPPORTED, "caller-given coefficients are taken by cpa_shrink_dense(_noalloc) and "
                                         "cpa_shrink_csr only");
    return CPA_OK;
}

cpa_status learned_bound_unsupported(const cpa_opts* o) {
    if (o->bound == CPA_BOUND_LEARNED)
        return fail(CPA_ERR_UNSUPPORTED, "the learned bound rule is available on cpa_shrink_dense(_noalloc) and "
                                         "cpa_spectral_bound only");
    return CPA_OK;
}

cpa_status no_learned_bound(const cpa_opts* o) {
    const cpa_status s = learned_bound_unsupported(o);
    return s != CPA_OK ? s : no_given_coeffs(o);
}

// Lanczos steps of the Lanczos rule (0 selects the default).
int lanczos_steps(const cpa_opts* o) { return o->lanczos_steps > 0 ? o->lanczos_steps : kLanczosDefault; }

// Power-iteration slots of the scalar block: the power rule, and the learned
// rule, whose check falls back to power iteration; the Lanczos rule's steps.
int power_slots(const cpa_opts* o) {
    if (o->bound == CPA_BOUND_LANCZOS) return lanczos_steps(o);
    return (o->bound == CPA_BOUND_POWER || o->bound == CPA_BOUND_LEARNED) ? o->power_iters : 1;
}

cpa_status check_opts(const cpa_opts* o) {
    if (!o) return fail(CPA_ERR_ARG, "opts is NULL");
    if (o->K < 1 || o->K > kMaxK) return fail(CPA_ERR_ARG, "K must be in [1, %d], got %d", kMaxK, o->K);
    if (o->bound < 0 || o->bound > 4) return fail(CPA_ERR_ARG, "unknown bound rule %d", o->bound);
    if (o->bound == CPA_BOUND_LEARNED && !o->model) return fail(CPA_ERR_ARG, "the learned bound needs opts.model");
    if (o->bound == CPA_BOUND_GIVEN && !(std::isfinite(o->Lambda) && o->Lambda >= 0.0))
        return fail(CPA_ERR_ARG, "given Lambda must be finite and >= 0");
    if (o->bound == CPA_BOUND_POWER || o->bound == CPA_BOUND_LEARNED) {
        if (o->power_iters < 1 || o->power_iters > kMaxPowerIters)
            return fail(CPA_ERR_ARG, "power_iters must be in [1, %d]", kMaxPowerIters);
        if (!(o->power_tol >= 0.0) || !(o->margin >= 0.0)) return fail(CPA_ERR_ARG, "power_tol and margin must be >= 0");
    }
    if (o->lanczos_steps < 0 || o->lanczos_steps > kLanczosMax)
        return fail(CPA_ERR_ARG, "lanczos_steps must be in [0, %d]", kLanczosMax);
    if (o->bound == CPA_BOUND_LANCZOS && !(o->margin >= 0.0)) return fail(CPA_ERR_ARG, "margin must be >= 0");
    if (o->precision != CPA_PREC_FP32 && o->precision != CPA_PREC_BF16X3)
        return fail(CPA_ERR_UNSUPPORTED, "precision %d not supported", o->precision);
    if (o->eval < CPA_EVAL_AUTO || o->eval > CPA_EVAL_POLYNOMIAL) return fail(CPA_ERR_ARG, "unknown eval %d", o->eval);
    if (o->eval == CPA_EVAL_POLYNOMIAL && o->K > kPsMaxS * kPsMaxS)
        return fail(CPA_ERR_UNSUPPORTED, "the matrix-polynomial route supports K <= %d", kPsMaxS * kPsMaxS);
    if (o->side < CPA_SIDE_AUTO || o->side > CPA_SIDE_LEFT) return fail(CPA_ERR_ARG, "unknown side %d", o->side);
    if (o->damping < CPA_DAMP_NONE || o->damping > CPA_DAMP_LANCZOS)
        return fail(CPA_ERR_ARG, "unknown damping %d", o->damping);
    if (o->coeffs) {
        if (o->bound != CPA_BOUND_GIVEN)
            return fail(CPA_ERR_ARG, "caller-given coefficients need the given bound (they belong to one Lambda)");
        if (o->check || o->damping != CPA_DAMP_NONE)
            return fail(CPA_ERR_UNSUPPORTED, "caller-given coefficients take neither the check nor damping");
    }
    return CPA_OK;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + bbytes && pb < pa + abytes;
}

cpa_status fill_scalars(hipStream_t st, const Work& w) {
    const int n = w.lay.total();
    hipLaunchKernelGGL(fill_f64_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w.scal, n, 0.0);
    HIP_TRY(hipGetLastError());
    return CPA_OK;
}

// Gram into w.G (d x d, ld = d) with ||G||_F^2 and trace accumulated.
cpa_status enqueue_gram_impl(hipStream_t st, int m, int n, const float* X, int64_t ldx, const Work& w, bool xt_ready);

cpa_status enqueue_gram(cpa_ctx* ctx, hipStream_t st, int m, int n, const float* X, int64_t ldx, const Work& w,
                        bool xt_ready = false) {
    hipEvent_t a, b;
    cpa_status s = timing_pair(ctx, 1, a, b);
    if (s != CPA_OK) return s;
    if (a) HIP_TRY(hipEventRecord(a, st));
    s = enqueue_gram_impl(st, m, n, X, ldx, w, xt_ready);
    if (s != CPA_OK) return s;
    if (b) HIP_TRY(hipEventRecord(b, st));
    return CPA_OK;
}

// Leading dimension of X^T when the right-side Gram is formed from it as a
// symmetric product in pieces (its side a multiple of 64, room for X^T with the
// contraction padded to a multiple of 64), else 0.
int64_t gram_xt_ld(const Work& w, int m, int n) {
    const int d = w.d;
    if (!w.right || d % 64 != 0 || !aligned16(w.G, d) || gram_grid(d) != w.lay.gwg || !w.xt) return 0;
    const int64_t ldt = ((int64_t)m + 63) / 64 * 64;
    if (!aligned16(w.xt, ldt) || (int64_t)n * ldt > w.xt_cap || ldt > INT32_MAX) return 0;
    return ldt;
}

cpa_status enqueue_gram_impl(hipStream_t st, int m, int n, const float* X, int64_t ldx, const Work& w, bool xt_ready) {
    EpiGram epi;
    const int d = w.d;
    epi.C = w.G;
    epi.ldc = d;
    epi.part = w.scal + w.lay.gpart();
    epi.vec_ok = aligned16(w.G, d);
    // the Gram as a symmetric product in pieces (gemm_f32_piece_kernel) when its
    // side is a multiple of 64: on the right side from X^T (transposed, the
    // contraction padded with zeros to a multiple of 64; xt_ready: already there),
    // on the left from X itself
    if (d % 64 == 0 && epi.vec_ok && gram_grid(d) == w.lay.gwg) {
        const int nt = d / 64;
        if (w.right) {
            const int64_t ldt = gram_xt_ld(w, m, n);
            if (ldt > 0) {
                if (!xt_ready) {
                    hipLaunchKernelGGL(transpose_pad_kernel, dim3((unsigned)(ldt / 64), (unsigned)(n / 64)), dim3(256),
                                       0, st, m, n, X, ldx, w.xt, ldt);
                    HIP_TRY(hipGetLastError());
                }
                const Operand T = make_op(w.xt, ldt, n);
                hipLaunchKernelGGL(gemm_f32_piece_kernel<EpiGram>, dim3(nt * nt), dim3(1024), 0, st, T, T, n, (int)ldt,
                                   epi);
                HIP_TRY(hipGetLastError());
                return CPA_OK;
            }
        } else if (n % 64 == 0 && aligned16(X, ldx)) {
            const Operand A = make_op(X, ldx, m);
            hipLaunchKernelGGL(gemm_f32_piece_kernel<EpiGram>, dim3(nt * nt), dim3(1024), 0, st, A, A, m, n, epi);
            HIP_TRY(hipGetLastError());
            return CPA_OK;
        }
    }
    if (w.right) {
        // G(i, j) = sum_r X[r][i] X[r][j]
        Operand A = make_op(X, ldx, n), B = make_op(X, ldx, n);
        return gemm_dispatch<XCONTIG, XCONTIG>(st, A, B, n, n, m, epi, 0, 0, 0);
    }
    // G(i, j) = sum_c X[i][c] X[j][c]
    Operand A = make_op(X, ldx, m), B = make_op(X, ldx, m);
    return gemm_dispatch<KCONTIG, KCONTIG>(st, A, B, m, m, n, epi, 0, 0, 0);
}

// G64 != nullptr: the power iteration reads that FP64 Gram (pitch d) instead of w.G.
// A Work that carries the matrix-polynomial route gets its coefficients rewritten
// for that route by the bound's finish kernel (enqueue_poly_core then skips it).
bool poly_fused(const Work& w, int K) { return w.poly_s > 0 && K >= 2; }

// The finish kernel's bound mode of a rule: 0 power, 1 given, 2 Frobenius, 3 learned.
int bound_mode(int rule) {
    return (rule == CPA_BOUND_POWER || rule == CPA_BOUND_LANCZOS) ? 0
           : rule == CPA_BOUND_GIVEN                              ? 1
           : rule == CPA_BOUND_FROBENIUS                          ? 2
                                                                  : 3;
}

// logmn: log(m n) of the input (the learned rule's third feature).
cpa_status enqueue_bound(cpa_ctx* ctx, hipStream_t st, int d, const cpa_shrinkage* sh, const cpa_opts* o,
                         const Work& w, int mode_override, const double* G64 = nullptr, double logmn = 0.0,
                         bool start_ready = false, double* Q64 = nullptr, size_t q64_doubles = 0) {
    int mode = bound_mode(o->bound);
    if (mode_override >= 0) mode = mode_override;
    double* warm_vec = w.warm_vec ? w.warm_vec : ctx->warm;
    int& warm_len = w.warm_len ? *w.warm_len : ctx->warm_d;
    if (mode == 0) {
        const bool warm = o->warm_start && warm_len == d;
        if (!start_ready) {
            hipLaunchKernelGGL(power_init_kernel, dim3(1), dim3(256), 0, st, d, (uint64_t)o->seed,
                               warm ? (const double*)warm_vec : nullptr, w.w[0], w.scal, w.lay.pw_w2());
            HIP_TRY(hipGetLastError());
        }
        int d_ = d, maxit_ = o->power_iters, pw_mu = w.lay.pw_mu(), pw_w2 = w.lay.pw_w2();
        // every product or step has its slots in the scalar block
        const int slots = o->bound == CPA_BOUND_LANCZOS ? std::min(lanczos_steps(o), d) : maxit_;
        if (slots > w.lay.maxit)
            return fail(CPA_ERR_ARG, "internal: %d bound slots laid out for %d products", w.lay.maxit, slots);
        const float* G = w.G;
        int64_t ldg = d;
        double* wb0 = w.w[0];
        double* wb1 = w.w[1];
        double* part = w.scal + w.lay.ppart();
        unsigned* counter = reinterpret_cast<unsigned*>(w.scal + SC_BARRIER);
        double* scal = w.scal;
        double tol = o->power_tol;
        cpa_status ls;
        if (G64 && o->bound == CPA_BOUND_LANCZOS) {
            // the FP64 Gram: the grid kernel at every side, its vectors in the caller's idle buffer
            int steps = std::min(lanczos_steps(o), d);
            if (d > kPowerVecLds)
                return fail(CPA_ERR_UNSUPPORTED, "the Lanczos bound takes Gram sides up to %d (got %d)", kPowerVecLds,
                            d);
            if (!Q64 || (size_t)(steps + 2) * d > q64_doubles)
                return fail(CPA_ERR_UNSUPPORTED, "no room for the Lanczos vectors in this workspace");
            void* args[] = {&d_, &G64, &ldg, &wb0, &wb1, &Q64, &part, &counter, &scal, &steps, &tol, &pw_mu, &pw_w2};
            ls = launch_power(ctx, reinterpret_cast<const void*>(lanczos_coop_kernel<double>), w.lay.pwg, args, st);
        } else if (G64) {
            void* args[] = {&d_, &G64, &ldg, &wb0, &wb1, &part, &counter, &scal, &maxit_, &tol, &pw_mu, &pw_w2};
            ls = launch_power(ctx, reinterpret_cast<const void*>(power_coop_kernel<double>), w.lay.pwg, args, st);
        } else if (o->bound == CPA_BOUND_LANCZOS) {
            int steps = std::min(lanczos_steps(o), d);
            if (d <= kPowerWgMaxD) {
                hipLaunchKernelGGL(lanczos_wg_kernel, dim3(1), dim3(kPowerWgThreads), 0, st, d, G, ldg, wb0, wb1, scal,
                                   steps, o->power_tol, pw_mu, pw_w2);
                HIP_TRY(hipGetLastError());
                ls = CPA_OK;
            } else {
                // the Lanczos vectors (and the shared u by parity) in a buffer that is
                // idle while the bound runs: the second recurrence buffer, or the
                // matrix-polynomial region (read again only after the bound)
                if (d > kPowerVecLds)
                    return fail(CPA_ERR_UNSUPPORTED, "the Lanczos bound takes Gram sides up to %d (got %d)",
                                kPowerVecLds, d);
                const size_t need = sizeof(double) * (size_t)(steps + 2) * d;
                double* Q = nullptr;
                if (w.Yb[1] && need <= sizeof(float) * (size_t)w.yb_cap)
                    Q = reinterpret_cast<double*>(w.Yb[1]);
                else if (w.poly && need <= sizeof(float) * (size_t)poly_mats(w.lay.K, w.poly_s) * w.d * w.d)
                    Q = reinterpret_cast<double*>(w.poly);
                if (!Q) return fail(CPA_ERR_UNSUPPORTED, "no room for the Lanczos vectors in this workspace");
                double tol = o->power_tol;
                void* args[] = {&d_, &G, &ldg, &wb0, &wb1, &Q, &part, &counter, &scal, &steps, &tol, &pw_mu, &pw_w2};
                ls = launch_power(ctx, reinterpret_cast<const void*>(lanczos_coop_kernel<float>), w.lay.pwg, args, st);
            }
        } else if (d <= kPowerWgMaxD) {
            // small sides: one workgroup with G in registers, no grid barrier
            hipLaunchKernelGGL(power_wg_kernel, dim3(1), dim3(kPowerWgThreads), 0, st, d, G, ldg, wb0, wb1, scal,
                               maxit_, tol, pw_mu, pw_w2);
            HIP_TRY(hipGetLastError());
            ls = CPA_OK;
        } else {
            void* args[] = {&d_, &G, &ldg, &wb0, &wb1, &part, &counter, &scal, &maxit_, &tol, &pw_mu, &pw_w2};
            ls = launch_power(ctx, reinterpret_cast<const void*>(power_coop_kernel<float>), w.lay.pwg, args, st);
        }
        if (ls != CPA_OK) return ls;
    }
    // on the matrix-polynomial route the finish kernel also forms T1 (extra workgroups)
    const bool shift = poly_fused(w, o->K);
    const int shift_wg = shift ? (int)std::min<int64_t>(4096, ((int64_t)d * d / 16 + 255) / 256 + 1) : 0;
    hipLaunchKernelGGL(finish_bound_kernel, dim3(1 + shift_wg), dim3(256), 0, st, mode, o->Lambda, d, o->power_iters,
                       o->margin, (const double*)w.w[0], (const double*)w.w[1], mode == 0 ? warm_vec : nullptr, w.scal,
                       to_params(sh), o->K, w.lay.pw_mu(), w.lay.pw_w2(), (const double*)(w.scal + w.lay.gpart()),
                       w.lay.gwg, 0, o->damping, w.poly_s, poly_fused(w, o->K) ? w.lay.ps() : -1,
                       mode == 3 ? o->model : nullptr, logmn, o->coeffs, shift ? (const float*)w.G : nullptr,
                       (int64_t)d, shift ? w.poly : nullptr);
    HIP_TRY(hipGetLastError());
    if (mode == 0) warm_len = d;
    return CPA_OK;
}

// K-1 recurrence steps (or the K == 1 scaling), accumulating into Y.
cpa_status enqueue_recurrence(cpa_ctx* ctx, hipStream_t st, int m, int n, const float* X, int64_t ldx, float* Y, int64_t ldy,
                              int K, const Work& w, bool norms_needed, int precision) {
    if (K == 1) {
        const int64_t total = (int64_t)m * n;
        const int grid = (int)std::min<int64_t>(4096, (total + 255) / 256);
        hipLaunchKernelGGL(scale_copy_kernel, dim3(std::max(grid, 1)), dim3(256), 0, st, m, n, X, ldx, Y, ldy,
                           (const double*)w.scal);
        HIP_TRY(hipGetLastError());
        return CPA_OK;
    }
    const int d = w.d;
    const int norms = w.lay.norms();
    if (!w.Yb[0] || !w.Yb[1]) return fail(CPA_ERR_ARG, "internal: the recurrence has no Y buffers in this workspace");
    for (int k = 0; k + 1 <= K - 1; ++k) {
        EpiCheb epi;
        const float* yk = k == 0 ? X : w.Yb[(k - 1) & 1];
        const int64_t ldk = k == 0 ? ldx : n;
        const float* yp = k <= 1 ? X : w.Yb[k & 1];
        const int64_t ldp = k <= 1 ? ldx : n;
        epi.Yk = yk;
        epi.ldk = ldk;
        epi.Yprev = yp;
        epi.ldp = ldp;
        epi.Ydst = w.Yb[k & 1];
        epi.ldd = n;
        epi.out = Y;
        epi.ldo = ldy;
        epi.scal = w.scal;
        epi.step = k;
        epi.last = (k + 1 == K - 1) ? 1 : 0;
        epi.nrm2 = norms_needed ? w.scal + norms + (k + 1) * kNormSlots : nullptr;
        epi.vec_ok = aligned16(yk, ldk) && aligned16(yp, ldp) && aligned16(epi.Ydst, n) && aligned16(Y, ldy);
        hipEvent_t ea, eb;
        cpa_status s = timing_pair(ctx, 0, ea, eb);
        if (s != CPA_OK) return s;
        if (ea) HIP_TRY(hipEventRecord(ea, st));
        if (w.right) {
            // Y_k G: A = Y_k (k contiguous); B(k, j) = G[k][j] = G[j][k] (G symmetric),
            // read along k so both operands take 16-byte LDS fragment reads
            Operand A = make_op(yk, ldk, m), B = make_op(w.G, d, n);
            s = precision == CPA_PREC_BF16X3
                    ? launch_gemm_split<KCONTIG, KCONTIG>(st, A, B, m, n, n, epi, SC_A1, SC_A2, SC_COEF)
                    : gemm_dispatch<KCONTIG, KCONTIG>(st, A, B, m, n, n, epi, SC_A1, SC_A2, SC_COEF);
        } else {
            // G Y_k: A(i, k) = G[k][i] (G symmetric; i contiguous), B = Y_k (j contiguous)
            Operand A = make_op(w.G, d, m), B = make_op(yk, ldk, n);
            s = precision == CPA_PREC_BF16X3
                    ? launch_gemm_split<XCONTIG, XCONTIG>(st, A, B, m, n, m, epi, SC_A1, SC_A2, SC_COEF)
                    : gemm_dispatch<XCONTIG, XCONTIG>(st, A, B, m, n, m, epi, SC_A1, SC_A2, SC_COEF);
        }
        if (s != CPA_OK) return s;
        if (eb) HIP_TRY(hipEventRecord(eb, st));
    }
    return CPA_OK;
}

// ---- matrix-polynomial route ---------------------------------------------------
//
// The same polynomial as the recurrence, p(Ghat) = c_0/2 I + sum_k c_k T_k(Ghat), is
// formed on the d x d side (as Algorithm 1's H = sum c_k Psi_k) with baby steps and
// giant steps in the Chebyshev basis:
//   T_1 = Ghat, T_{i+1} = 2 T_1 T_i - T_{i-1}            (i < s: s - 1 products)
//   p = sum_j R_j T_j(y), y = T_s, R_j = sum_i r_{j,i} T_i   (Clenshaw in y: J - 1 products)
//   Y = X p (right side) or p X (left side)                 (one product)
// with s = ceil(sqrt(K)) and J = ceil(K / s) (K <= 1024, so s, J <= 32): about
// 2 sqrt(K) products instead of K - 1.  All matrices of the route are polynomials
// in Ghat, hence symmetric in exact arithmetic, and the engine reads the second
// operand along k, i.e. transposed.  Only the fixed operands (T_1 in the baby
// steps, y in the giant steps) are taken that way: a transposed T_1 or y is one
// fixed, slightly different operator for the whole chain, whereas transposing
// the operand that changes from step to step lets its rounding asymmetry grow
// (about 3e-5 at s = 10 in FP32, and relative errors near 1e-3 at K = 144).

constexpr int kPolyMaxK = kPsMaxS * kPsMaxS;   // 1024

int poly_s_of(int K) {
    int s = 1;
    while (s * s < K) ++s;
    return std::min(s, kPsMaxS);
}

// s of the matrix-polynomial route when `o` selects it for an m x n input, else 0.
int poly_choice(const cpa_opts* o, int m, int n) {
    if (o->K < 2 || o->K > kPolyMaxK || o->eval == CPA_EVAL_RECURRENCE) return 0;
    const int s = poly_s_of(o->K), J = (o->K + s - 1) / s;
    if (o->eval == CPA_EVAL_POLYNOMIAL) return s;
    const bool right = right_side(o, m, n);
    const double d = right ? n : m, e = right ? m : n;
    const double cost_poly = (double)(s - 1 + J - 1) * d * d * d + e * d * d;
    const double cost_rec = (double)(o->K - 1) * e * d * d;
    return cost_poly < cost_rec ? s : 0;
}

// Timing family of a matrix-polynomial product: 2 for a symmetric product in
// pieces, else 0 (with the recurrence products).
template <class Epi>
int poly_family(const Epi&) {
    return 0;
}
template <>
int poly_family<EpiLin>(const EpiLin& e) {
    return e.sym == 2 ? 2 : 0;
}

template <class Epi>
cpa_status poly_gemm(cpa_ctx* ctx, hipStream_t st, const Operand& A, const Operand& B, int M, int N, int Kd,
                     const Epi& epi, int precision, bool kk) {
    hipEvent_t ea, eb;
    cpa_status s = timing_pair(ctx, poly_family(epi), ea, eb);
    if (s != CPA_OK) return s;
    if (ea) HIP_TRY(hipEventRecord(ea, st));
    if (kk)
        s = precision == CPA_PREC_BF16X3 ? launch_gemm_split<KCONTIG, KCONTIG>(st, A, B, M, N, Kd, epi, SC_A1, SC_A2, SC_COEF)
                                         : gemm_dispatch<KCONTIG, KCONTIG>(st, A, B, M, N, Kd, epi, SC_A1, SC_A2, SC_COEF);
    else
        s = precision == CPA_PREC_BF16X3 ? launch_gemm_split<XCONTIG, XCONTIG>(st, A, B, M, N, Kd, epi, SC_A1, SC_A2, SC_COEF)
                                         : gemm_dispatch<XCONTIG, XCONTIG>(st, A, B, M, N, Kd, epi, SC_A1, SC_A2, SC_COEF);
    if (s != CPA_OK) return s;
    if (eb) HIP_TRY(hipEventRecord(eb, st));
    return CPA_OK;
}

EpiLin lin_epi(float* D, int64_t ldd, const float* Mx, int64_t ldm, float alpha, float beta, float gamma, float delta) {
    EpiLin e;
    e.D = D;
    e.ldd = ldd;
    e.C = D;
    e.ldc = ldd;
    e.Mx = Mx;
    e.ldm = ldm;
    e.alpha = alpha;
    e.beta = beta;
    e.gamma = gamma;
    e.delta = delta;
    e.vec_ok = aligned16(D, ldd) && (gamma == 0.f || aligned16(Mx, ldm));
    return e;
}

// The polynomial p(Ghat) (d x d, pitch d) from the Gram G (pitch ldg) and the
// coefficients in scal; `poly` holds poly_mats(K, s) matrices of d x d.  Returns p's buffer.
// How the symmetric products of the route run (EpiLin::sym): 0 all tiles, 1 the
// upper-triangle tiles, 2 in pieces (gemm_f32_piece_kernel; d % 64 == 0).  Cost
// in MFMA blocks per CU: rounds of workgroups over the CUs times the blocks of
// the largest workgroup (16 for a tile, 10 for a diagonal piece).  d = 1024 on
// 256 CUs: 16 (all tiles or the 136 upper ones, one round) against 10 (256
// pieces); d = 1344: 2 x 16 and 2 x 10 against 16 for the 231 upper tiles.
int sym_mode(cpa_ctx* ctx, int d) {
    if (ctx->cus == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) return 0;
        ctx->cus = std::max(1, cus);
    }
    const int64_t nt = (d + 63) / 64, full = nt * nt, tri = nt * (nt + 1) / 2, c = ctx->cus;
    const int64_t cost_full = (full + c - 1) / c * 16, cost_tri = (tri + c - 1) / c * 16;
    const int64_t cost_piece = d % 64 == 0 ? (full + c - 1) / c * 10 : INT64_MAX;
    if (cost_piece < cost_tri && cost_piece < cost_full) return 2;
    return cost_tri < cost_full ? 1 : 0;
}

// check_off >= 0: after the baby steps, the Gram-weighted means of T_2..T_s go
// to the scalar block at check_off (ps_check_kernel).
cpa_status enqueue_poly_core(cpa_ctx* ctx, hipStream_t st, int d, const float* G, int64_t ldg, double* scal,
                             int roff, float* poly, int s, int K, int precision, float** F_out, bool coeff_ready,
                             int check_off = -1, bool shift_ready = false) {
    const int J = (K + s - 1) / s;
    const int sym = precision == CPA_PREC_FP32 ? sym_mode(ctx, d) : 0;
    const int64_t dd = (int64_t)d * d;
    float* T1 = poly;                         // T_q at T1 + (q - 1) dd, q = 1..s
    float* R = poly + (int64_t)s * dd;        // R_j at R + j dd
    float* Bf[3] = {R + (int64_t)J * dd, R + (int64_t)(J + 1) * dd, R + (int64_t)(J + 2) * dd};
    const int ge = (int)std::min<int64_t>(4096, (dd + 255) / 256);
    if (!coeff_ready) {
        hipLaunchKernelGGL(ps_coeff_kernel, dim3(1), dim3(256), 0, st, K, s, J, scal, roff);
        HIP_TRY(hipGetLastError());
    }
    if (!shift_ready) {
        hipLaunchKernelGGL(ps_shift_kernel, dim3(ge), dim3(256), 0, st, d, G, ldg, T1, (const double*)scal);
        HIP_TRY(hipGetLastError());
    }
    cpa_status r;
    auto Tq = [&](int q) { return T1 + (int64_t)(q - 1) * dd; };
    // baby steps: T_{i+1} = 2 T_i T_1 - T_{i-1}, T_0 = I (T_1 is the operand read transposed)
    for (int i = 1; i < s; ++i) {
        EpiLin e = lin_epi(Tq(i + 1), d, i > 1 ? Tq(i - 1) : nullptr, d, 2.f, 0.f, i > 1 ? -1.f : 0.f,
                           i > 1 ? 0.f : -1.f);
        e.sym = sym;
        if ((r = poly_gemm(ctx, st, make_op(Tq(i), d, d), make_op(T1, d, d), d, d, d, e, precision, true)) != CPA_OK)
            return r;
    }
    if (check_off >= 0 && s >= 2) {
        hipLaunchKernelGGL(ps_check_kernel, dim3(kPsCheckWg), dim3(256), 0, st, d, G, ldg, (const float*)T1, s,
                           scal + check_off);
        HIP_TRY(hipGetLastError());
    }
    // every R_j = sum_i r_{j,i} T_i in one pass
    const dim3 glc((int)std::min<int64_t>(4096, (dd / 4 + 255) / 256 + 1));
    if (s <= 16)
        hipLaunchKernelGGL(ps_lincomb_kernel<16>, glc, dim3(256), 0, st, d, s, J, (const float*)T1,
                           (const double*)scal, roff, R);
    else if (s <= 24)
        hipLaunchKernelGGL(ps_lincomb_kernel<24>, glc, dim3(256), 0, st, d, s, J, (const float*)T1,
                           (const double*)scal, roff, R);
    else
        hipLaunchKernelGGL(ps_lincomb_kernel<kPsMaxS>, glc, dim3(256), 0, st, d, s, J, (const float*)T1,
                           (const double*)scal, roff, R);
    HIP_TRY(hipGetLastError());
    if (J == 1) {
        *F_out = R;
        return CPA_OK;
    }
    // giant steps (Clenshaw in y = T_s): b_{J-1} = R_{J-1}; b_j = R_j + 2 b_{j+1} y - b_{j+2};
    // p = R_0 + b_1 y - b_2
    const float* y = Tq(s);
    const float* cur = R + (int64_t)(J - 1) * dd;   // b_{j+1}
    const float* prev = nullptr;                     // b_{j+2}
    for (int j = J - 2; j >= 0; --j) {
        float* dst = Bf[0];
        for (int q = 0; q < 3; ++q)
            if (Bf[q] != cur && Bf[q] != prev) {
                dst = Bf[q];
                break;
            }
        EpiLin e = lin_epi(dst, d, prev, d, j > 0 ? 2.f : 1.f, 1.f, prev ? -1.f : 0.f, 0.f);
        e.sym = sym;
        e.C = R + (int64_t)j * dd;
        e.ldc = d;
        e.vec_ok = e.vec_ok && aligned16(e.C, d);
        // b_{j+1} y with y read transposed
        if ((r = poly_gemm(ctx, st, make_op(cur, d, d), make_op(y, d, d), d, d, d, e, precision, true)) != CPA_OK)
            return r;
        prev = cur;
        cur = dst;
    }
    *F_out = const_cast<float*>(cur);
    return CPA_OK;
}

cpa_status enqueue_poly(cpa_ctx* ctx, hipStream_t st, int m, int n, const float* X, int64_t ldx, float* Y,
                        int64_t ldy, int K, const Work& w, int precision, bool check = false) {
    const int d = w.d;
    float* F = nullptr;
    // enqueue_bound on this Work rewrote the coefficients and formed T1 already
    cpa_status r = enqueue_poly_core(ctx, st, d, w.G, d, w.scal, w.lay.ps(), w.poly, w.poly_s, K, precision, &F,
                                     poly_fused(w, K), check ? w.lay.pchk() : -1, poly_fused(w, K));
    if (r != CPA_OK) return r;
    // Y = X p (right) or p X (left); p read transposed (it is the fixed operand)
    const EpiLin e = lin_epi(Y, ldy, nullptr, 0, 1.f, 0.f, 0.f, 0.f);
    if (w.right)
        return poly_gemm(ctx, st, make_op(X, ldx, m), make_op(F, d, n), m, n, n, e, precision, true);
    return poly_gemm(ctx, st, make_op(F, d, m), make_op(X, ldx, n), m, n, m, e, precision, false);
}

// Reads the scalar block's header and the growth-check norms through a fixed
// host buffer (no heap allocation; one copy while K <= 48, else a few).
cpa_status read_info(hipStream_t st, const Work& w, int K, int m, int n, cpa_info* info, double* growth_out) {
    constexpr int kBuf = 3200;
    double h[kBuf];
    const int nrm = w.lay.norms();
    const int first = std::min(kBuf, nrm + std::max(K, 1) * kNormSlots);
    HIP_TRY(hipMemcpyAsync(h, w.scal, sizeof(double) * first, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double hdr[SC_COEF];
    std::memcpy(hdr, h, sizeof(hdr));
    double g = 0.0;
    const double x2 = hdr[SC_TRACE];
    int base = 0, have = first;   // h holds scal[base, base + have)
    for (int k = 1; k < K; ++k) {
        const int at = nrm + k * kNormSlots;
        if (at + kNormSlots > base + have) {
            base = at;
            have = std::min(kBuf / kNormSlots, K - k) * kNormSlots;
            HIP_TRY(hipMemcpyAsync(h, w.scal + base, sizeof(double) * have, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        double nk = 0.0;
        for (int q = 0; q < kNormSlots; ++q) nk += h[at - base + q];
        const double r = x2 > 0.0 ? std::sqrt(nk / x2) : 0.0;
        g = std::max(g, r);
    }
    if (growth_out) *growth_out = g;
    if (info) {
        info->Lambda = hdr[SC_LAMBDA];
        info->mu = hdr[SC_MU];
        info->resid = hdr[SC_RESID];
        info->fro_gram = std::sqrt(std::max(hdr[SC_FRO2], 0.0));
        info->max_growth = g;
        info->power_iters_done = (int)hdr[SC_ITERS];
        info->fallback = 0;
        info->side = w.right ? 0 : 1;
        info->reserved = 0;
    }
    if (hdr[SC_TIMEOUT] != 0.0) return fail(CPA_ERR_HIP, "power iteration grid barrier timed out");
    if (!std::isfinite(hdr[SC_TRACE]) || !std::isfinite(hdr[SC_FRO2]))
        return fail(CPA_ERR_NONFINITE, "X holds NaN or infinite entries (or its Gram overflows FP32)");
    if (!std::isfinite(hdr[SC_LAMBDA])) return fail(CPA_ERR_NONFINITE, "spectral bound is not finite");
    return CPA_OK;
}

// max_q mu_q of the matrix-polynomial route's check (ps_check_kernel), from the
// scalar block (synchronising); 0 when tr G = 0.
cpa_status read_poly_check(hipStream_t st, const Work& w, double* growth) {
    constexpr int kMaxPart = (kPsMaxS - 1) * kPsCheckWg;
    double h[kMaxPart];
    double tr = 0.0;
    const int s = w.poly_s;
    *growth = 0.0;
    if (s < 2) return CPA_OK;
    HIP_TRY(hipMemcpyAsync(h, w.scal + w.lay.pchk(), sizeof(double) * (s - 1) * kPsCheckWg, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&tr, w.scal + SC_TRACE, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (!(tr > 0.0)) return CPA_OK;
    double g = -INFINITY;
    for (int q = 2; q <= s; ++q) {
        double sum = 0.0;
        for (int b = 0; b < kPsCheckWg; ++b) sum += h[(q - 2) * kPsCheckWg + b];
        g = std::max(g, sum / tr);
    }
    *growth = g;
    return CPA_OK;
}

// What enqueue_prep has done for the shrink that follows it.
struct PrepDone {
    bool xt = false;      // X^T stored for the Gram (gram_xt_ld)
    bool start = false;   // the power iteration's start vector written
};

// One launch before a shrink (prep_kernel): clears the scalar block, writes the
// power iteration's start vector when the bound `mode` (0: power) needs it, and
// stores X^T when the Gram is formed from it; with P, the ADMM pre-step runs on
// the same tiles (its E_t partials into part, *npart of them) and the shrink
// input is P->x.
cpa_status enqueue_prep(cpa_ctx* ctx, hipStream_t st, int m, int n, const float* X, int64_t ldx, const Work& w,
                        const cpa_opts* o, int mode, const AdmmPtrs* P, double* part, int* npart, PrepDone& done) {
    PrepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.m = m;
    a.n = n;
    a.X = X;
    a.ldx = ldx;
    if (P) {
        a.P = *P;
        a.admm = 1;
        a.part = part;
        auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
        a.vec = n % 4 == 0 && al(P->l) && al(P->s) && al(P->z1) && al(P->z2) && al(P->u1) && al(P->u2) &&
                al(P->u3) && al(P->I) && al(P->x);
    }
    const int64_t ldt = gram_xt_ld(w, m, n);
    a.xt = ldt > 0 ? w.xt : nullptr;
    a.ldt = ldt;
    a.scal = w.scal;
    a.nscal = w.lay.total();
    const int d = w.d;
    if (mode == 0) {
        const double* warm_vec = w.warm_vec ? w.warm_vec : ctx->warm;
        const int warm_len = w.warm_len ? *w.warm_len : ctx->warm_d;
        a.d = d;
        a.seed = (uint64_t)o->seed;
        a.warm = o->warm_start && warm_len == d ? warm_vec : nullptr;
        a.w0 = w.w[0];
        a.pw_w2 = w.lay.pw_w2();
    }
    const int64_t rows = ldt > 0 ? ldt / kPrepTile : ((int64_t)m + kPrepTile - 1) / kPrepTile,
                  cols = ((int64_t)n + kPrepTile - 1) / kPrepTile;
    const int64_t tiles = (P || ldt > 0) ? rows * cols : 0;
    a.ntile_wg = (int)std::min<int64_t>(tiles, P ? kAdmmGrid : 4096);
    hipLaunchKernelGGL(prep_kernel, dim3(a.ntile_wg + 1), dim3(256), 0, st, a);
    HIP_TRY(hipGetLastError());
    if (npart) *npart = a.ntile_wg;
    done.xt = ldt > 0;
    done.start = mode == 0;
    return CPA_OK;
}

cpa_status shrink_impl(cpa_ctx* ctx, hipStream_t st, int m, int n, const float* X, int64_t ldx, float* Y,
                       int64_t ldy, const cpa_shrinkage* sh, const cpa_opts* o, cpa_info* info, const Work& w,
                       const PrepDone* pre = nullptr) {
    const int d = w.d;
    const double logmn = std::log((double)m * n);
    // the check's recompute: power iteration after the learned bound (the fallback
    // the predictor stands in for), the guaranteed ||G||_F after the others
    const int redo_mode = o->bound == CPA_BOUND_LEARNED ? 0 : 2;
    cpa_status s;
    PrepDone pd;
    if (pre) {
        pd = *pre;
    } else if ((s = enqueue_prep(ctx, st, m, n, X, ldx, w, o, bound_mode(o->bound), nullptr, nullptr, nullptr, pd)) !=
               CPA_OK) {
        return s;
    }
    if ((s = enqueue_gram(ctx, st, m, n, X, ldx, w, pd.xt)) != CPA_OK) return s;
    if ((s = enqueue_bound(ctx, st, d, sh, o, w, -1, nullptr, logmn, pd.start)) != CPA_OK) return s;
    if (w.poly_s > 0 && o->K >= 2) {
        if ((s = enqueue_poly(ctx, st, m, n, X, ldx, Y, ldy, o->K, w, o->precision, o->check != 0)) != CPA_OK)
            return s;
        if (!info && !o->check) return CPA_OK;
        if ((s = read_info(st, w, 1, m, n, info, nullptr)) != CPA_OK) return s;
        if (!o->check) return CPA_OK;
        double growth = 0.0;
        if ((s = read_poly_check(st, w, &growth)) != CPA_OK) return s;
        if (info) info->max_growth = growth;
        if (growth <= 1.0 + o->growth_tol) return CPA_OK;
        // bound too small: redo with the safer bound (Gram still valid)
        if ((s = fill_scalars(st, w)) != CPA_OK) return s;
        if ((s = enqueue_gram(ctx, st, m, n, X, ldx, w)) != CPA_OK) return s;
        if ((s = enqueue_bound(ctx, st, d, sh, o, w, redo_mode, nullptr, logmn)) != CPA_OK) return s;
        if ((s = enqueue_poly(ctx, st, m, n, X, ldx, Y, ldy, o->K, w, o->precision, true)) != CPA_OK) return s;
        if ((s = read_info(st, w, 1, m, n, info, nullptr)) != CPA_OK) return s;
        if ((s = read_poly_check(st, w, &growth)) != CPA_OK) return s;
        if (info) {
            info->fallback = 1;
            info->max_growth = growth;
        }
        if (growth > 1.0 + o->growth_tol)
            return fail(CPA_ERR_BOUND, "weighted mean %.6g exceeds 1 + %.3g even after the recompute", growth,
                        o->growth_tol);
        return CPA_OK;
    } else if ((s = enqueue_recurrence(ctx, st, m, n, X, ldx, Y, ldy, o->K, w, info != nullptr || o->check,
                                       o->precision)) != CPA_OK) {
        return s;
    }
    if (!info && !o->check) return CPA_OK;
    double growth = 0.0;
    if ((s = read_info(st, w, o->K, m, n, info, &growth)) != CPA_OK) return s;
    if (o->check && growth > 1.0 + o->growth_tol) {
        // bound too small: redo with the safer bound (Gram is still valid)
        if ((s = fill_scalars(st, w)) != CPA_OK) return s;
        if ((s = enqueue_gram(ctx, st, m, n, X, ldx, w)) != CPA_OK) return s;
        if ((s = enqueue_bound(ctx, st, d, sh, o, w, redo_mode, nullptr, logmn)) != CPA_OK) return s;
        if ((s = enqueue_recurrence(ctx, st, m, n, X, ldx, Y, ldy, o->K, w, info != nullptr || o->check, o->precision)) != CPA_OK) return s;
        if ((s = read_info(st, w, o->K, m, n, info, &growth)) != CPA_OK) return s;
        if (info) info->fallback = 1;
        if (growth > 1.0 + o->growth_tol)
            return fail(CPA_ERR_BOUND, "growth %.6g exceeds 1 + %.3g even after the recompute", growth, o->growth_tol);
    }
    return CPA_OK;
}

// ---- sparse path ----------------------------------------------------------------

constexpr int kSqGrid = 512;   // workgroups of the ||S||_F^2 reduction

struct SpWork {
    float* Y[2];
    float* W;
    int64_t ld;        // row pitch of Y and W (n rounded up to 32: 128-byte rows)
    float* cval;       // values of S in column order (nnz)
    double* tvec;
    double* w[2];
    double* scal;
    float* yv;         // SVT iterate values (nnz), when requested
    float* xv;         // SVT: observed entries of the shrink (nnz), when requested
    float* poly;       // matrix-polynomial route: poly_mats(K, s) matrices of n x n (or nullptr)
    int poly_s;
    ScalarLayout lay;
};

cpa_status ensure_sparse_ws(cpa_ctx* ctx, int m, int n, int64_t nnz, int K, int maxit, bool svt, SpWork& w,
                            int poly_s = 0) {
    if (ctx->coop_max == 0) {
        int per_cu = 0, cus = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, power_coop_kernel<float>, kPowerThreads, 0));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        ctx->coop_max = std::max(1, per_cu * cus);
    }
    w.ld = (n + 31) & ~int64_t(31);
    w.lay.K = K;
    w.lay.maxit = maxit;
    w.lay.gwg = kSqGrid;
    w.lay.pwg = std::max(1, std::min({64, (m + 63) / 64, ctx->coop_max}));
    size_t off = 0;
    const size_t oY0 = off; off = align_up(off + sizeof(float) * (size_t)m * w.ld);
    const size_t oY1 = off; off = align_up(off + sizeof(float) * (size_t)m * w.ld);
    const size_t oW = off; off = align_up(off + sizeof(float) * (size_t)n * w.ld);
    const size_t oT = off; off = align_up(off + sizeof(double) * (size_t)std::max(m, 1));
    const size_t ow0 = off; off = align_up(off + sizeof(double) * (size_t)std::max(n, 1));
    const size_t ow1 = off; off = align_up(off + sizeof(double) * (size_t)std::max(n, 1));
    const size_t os = off; off = align_up(off + sizeof(double) * (size_t)w.lay.total());
    const size_t ocv = off; off = align_up(off + sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
    size_t oy = 0;
    size_t oxv = 0;
    if (svt) {
        oy = off; off = align_up(off + sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
        oxv = off; off = align_up(off + sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
    }
    size_t opl = 0;
    if (poly_s > 0) { opl = off; off = align_up(off + sizeof(float) * (size_t)poly_mats(K, poly_s) * n * n); }
    if (off > ctx->sws_bytes) {
        if (ctx->sws) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ctx->sws));
            ctx->sws = nullptr;
            ctx->sws_bytes = 0;
        }
        if (hipMalloc(&ctx->sws, off) != hipSuccess) {
            ctx->sws = nullptr;
            return fail(CPA_ERR_ALLOC, "sparse workspace allocation of %zu bytes failed", off);
        }
        ctx->sws_bytes = off;
    }
    char* b = static_cast<char*>(ctx->sws);
    w.Y[0] = reinterpret_cast<float*>(b + oY0);
    w.Y[1] = reinterpret_cast<float*>(b + oY1);
    w.W = reinterpret_cast<float*>(b + oW);
    w.cval = reinterpret_cast<float*>(b + ocv);
    w.poly = poly_s > 0 ? reinterpret_cast<float*>(b + opl) : nullptr;
    w.poly_s = poly_s;
    w.tvec = reinterpret_cast<double*>(b + oT);
    w.w[0] = reinterpret_cast<double*>(b + ow0);
    w.w[1] = reinterpret_cast<double*>(b + ow1);
    w.scal = reinterpret_cast<double*>(b + os);
    w.yv = svt ? reinterpret_cast<float*>(b + oy) : nullptr;
    w.xv = svt ? reinterpret_cast<float*>(b + oxv) : nullptr;
    if (n > ctx->warm_cap) {
        if (ctx->warm) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ctx->warm));
        }
        ctx->warm = nullptr;
        if (hipMalloc(&ctx->warm, sizeof(double) * (size_t)std::max(n, 1)) != hipSuccess) {
            ctx->warm_cap = 0;
            ctx->warm_d = -1;
            return fail(CPA_ERR_ALLOC, "warm-start vector allocation failed");
        }
        ctx->warm_cap = std::max(n, 1);
        ctx->warm_d = -1;
    }
    return CPA_OK;
}

// The transposed pattern, rebuilt only when the CSR arrays or sizes change.
cpa_status ensure_csc(cpa_ctx* ctx, hipStream_t st, int m, int n, int64_t nnz, const int32_t* rowptr,
                      const int32_t* colidx) {
    if (ctx->csc && ctx->csc_rowptr == rowptr && ctx->csc_colidx == colidx && ctx->csc_m == m && ctx->csc_n == n &&
        ctx->csc_nnz == nnz)
        return CPA_OK;
    const size_t need = sizeof(int32_t) * ((size_t)n + 1 + 2 * (size_t)nnz + std::max<size_t>(n, 2 * (size_t)nnz));
    if (need > ctx->csc_bytes) {
        if (ctx->csc) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ctx->csc));
            ctx->csc = nullptr;
            ctx->csc_bytes = 0;
        }
        if (hipMalloc(&ctx->csc, need) != hipSuccess) {
            ctx->csc = nullptr;
            return fail(CPA_ERR_ALLOC, "pattern transpose allocation failed");
        }
        ctx->csc_bytes = need;
    }
    int32_t* colptr = ctx->csc;
    int32_t* crow = colptr + n + 1;
    int32_t* csrc = crow + nnz;
    int32_t* scratch = csrc + nnz;   // counts, then the unsorted (row, src) pairs
    // a new pattern is validated once (one synchronisation) before any kernel indexes with it
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, st, scratch, 1, 0);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(csr_validate_kernel, dim3(1024), dim3(256), 0, st, m, n, nnz, rowptr, colidx, scratch);
    HIP_TRY(hipGetLastError());
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, scratch, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return fail(CPA_ERR_ARG, "malformed CSR (row pointers or column indices)");
    hipLaunchKernelGGL(fill_i32_kernel, dim3(std::max(1, std::min(1024, (n + 255) / 256))), dim3(256), 0, st, scratch,
                       n, 0);
    HIP_TRY(hipGetLastError());
    const int ge = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (nnz + 255) / 256));
    if (nnz > 0) hipLaunchKernelGGL(csc_count_kernel, dim3(ge), dim3(256), 0, st, nnz, colidx, scratch);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(csc_scan_kernel, dim3(1), dim3(SP_THREADS), 0, st, n, (const int32_t*)scratch, colptr);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(fill_i32_kernel, dim3(std::max(1, std::min(1024, (n + 255) / 256))), dim3(256), 0, st, scratch,
                       n, 0);
    HIP_TRY(hipGetLastError());
    // unsorted pairs go to crow/csrc first, then sorted into scratch, then copied back
    hipLaunchKernelGGL(csc_scatter_kernel, dim3(std::max(1, std::min(4096, (m + 255) / 256))), dim3(256), 0, st, m,
                       rowptr, colidx, (const int32_t*)colptr, scratch, crow, csrc);
    HIP_TRY(hipGetLastError());
    int32_t* srow = scratch;
    int32_t* ssrc = scratch + nnz;
    hipLaunchKernelGGL(csc_sort_kernel, dim3(std::max(1, (n + 3) / 4)), dim3(256), 0, st, n, (const int32_t*)colptr,
                       (const int32_t*)crow, (const int32_t*)csrc, srow, ssrc);
    HIP_TRY(hipGetLastError());
    if (nnz > 0) {
        HIP_TRY(hipMemcpyAsync(crow, srow, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(csrc, ssrc, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, st));
    }
    ctx->csc_rowptr = rowptr;
    ctx->csc_colidx = colidx;
    ctx->csc_m = m;
    ctx->csc_n = n;
    ctx->csc_nnz = nnz;
    return CPA_OK;
}

// One sparse shrink, Y = hat G(S) (dense m x n at Y, ldy), everything enqueued.
// s of the matrix-polynomial route for a CSR input (0: operator-form recurrence).
// The route costs one sparse product for the Gram S^T S, s - 1 + J - 1 dense n x n
// products and one sparse product S p; the recurrence costs two sparse products per
// step.  AUTO takes the route when it has fewer products and its n x n buffers fit
// in 16 GiB.
int sparse_poly_choice(const cpa_opts* o, int n) {
    if (o->K < 2 || o->K > kPolyMaxK || o->eval == CPA_EVAL_RECURRENCE) return 0;
    const int s = poly_s_of(o->K), J = (o->K + s - 1) / s;
    if (o->eval == CPA_EVAL_POLYNOMIAL) return s;
    const double bytes = 4.0 * poly_mats(o->K, s) * (double)n * n;
    if (bytes > 16.0 * (1 << 30)) return 0;
    return (s - 1 + J - 1 + 2) < 2 * (o->K - 1) ? s : 0;
}

// xv != nullptr (the SVT driver, matrix-polynomial route only): the observed
// entries of the result go to xv (nnz, CSR order) and Y is not written.
cpa_status shrink_csr_impl(cpa_ctx* ctx, hipStream_t st, int m, int n, int64_t nnz, const int32_t* rowptr,
                           const int32_t* colidx, const float* val, float* Y, int64_t ldy,
                           const cpa_shrinkage* sh, const cpa_opts* o, const SpWork& w, float* xv = nullptr) {
    const int32_t* colptr = ctx->csc;
    const int32_t* crow = colptr + n + 1;
    const int32_t* csrc = crow + nnz;
    const int n_tot = w.lay.total();
    hipLaunchKernelGGL(fill_f64_kernel, dim3((n_tot + 255) / 256), dim3(256), 0, st, w.scal, n_tot, 0.0);
    HIP_TRY(hipGetLastError());
    // tr(S^T S) = ||S||_F^2 into the odd partial slots (even slots stay zero)
    double* gpart = w.scal + w.lay.gpart();
    hipLaunchKernelGGL(sq_norm_kernel, dim3(kSqGrid), dim3(256), 0, st, nnz, val, gpart);
    HIP_TRY(hipGetLastError());
    int mode = bound_mode(o->bound);
    if (mode == 0) {
        const bool warm = o->warm_start && ctx->warm_d == n;
        hipLaunchKernelGGL(power_init_kernel, dim3(1), dim3(256), 0, st, n, (uint64_t)o->seed,
                           warm ? (const double*)ctx->warm : nullptr, w.w[0], w.scal, w.lay.pw_w2());
        HIP_TRY(hipGetLastError());
        int m_ = m, n_ = n, maxit_ = o->power_iters, pw_mu = w.lay.pw_mu(), pw_w2 = w.lay.pw_w2();
        double* tvec = w.tvec;
        double* wb0 = w.w[0];
        double* wb1 = w.w[1];
        double* part = w.scal + w.lay.ppart();
        unsigned* counter = reinterpret_cast<unsigned*>(w.scal + SC_BARRIER);
        double* scal = w.scal;
        double tol = o->power_tol;
        cpa_status ls;
        if (o->bound == CPA_BOUND_LANCZOS) {
            // the Lanczos vectors (and u by parity) in a buffer idle until the
            // evaluation: W (n rows), else the second recurrence buffer (m rows)
            if (n > kPowerVecLds)
                return fail(CPA_ERR_UNSUPPORTED, "the Lanczos bound takes Gram sides up to %d (got %d)", kPowerVecLds,
                            n);
            int steps = std::min(lanczos_steps(o), n);
            const size_t need = sizeof(double) * (size_t)(steps + 2) * n;
            double* Q = nullptr;
            if (need <= sizeof(float) * (size_t)n * w.ld)
                Q = reinterpret_cast<double*>(w.W);
            else if (need <= sizeof(float) * (size_t)m * w.ld)
                Q = reinterpret_cast<double*>(w.Y[1]);
            if (!Q) return fail(CPA_ERR_UNSUPPORTED, "no room for the Lanczos vectors in this workspace");
            void* args[] = {&m_, &n_, &rowptr, &colidx, &val, &colptr, &crow, &csrc, &tvec, &wb0, &wb1,
                            &Q, &part, &counter, &scal, &steps, &tol, &pw_mu, &pw_w2};
            ls = launch_power(ctx, reinterpret_cast<const void*>(lanczos_op_kernel), w.lay.pwg, args, st);
        } else {
            void* args[] = {&m_, &n_, &rowptr, &colidx, &val, &colptr, &crow, &csrc, &tvec, &wb0, &wb1,
                            &part, &counter, &scal, &maxit_, &tol, &pw_mu, &pw_w2};
            ls = launch_power(ctx, reinterpret_cast<const void*>(power_op_kernel), w.lay.pwg, args, st);
        }
        if (ls != CPA_OK) return ls;
    }
    hipLaunchKernelGGL(finish_bound_kernel, dim3(1), dim3(256), 0, st, mode, o->Lambda, n, o->power_iters, o->margin,
                       (const double*)w.w[0], (const double*)w.w[1], mode == 0 ? ctx->warm : nullptr, w.scal,
                       to_params(sh), o->K, w.lay.pw_mu(), w.lay.pw_w2(), (const double*)gpart, kSqGrid, 1, o->damping, 0, -1,
                       nullptr, 0.0, o->coeffs, nullptr, (int64_t)0, nullptr);
    HIP_TRY(hipGetLastError());
    if (mode == 0) ctx->warm_d = n;
    const bool poly = w.poly_s > 0 && o->K >= 2;
    // the Gram by rows of S (no densified copy) when its LDS rows hold n floats
    const bool row_gram = poly && n <= SPG_MAXN;
    if (xv && !row_gram) return fail(CPA_ERR_ARG, "internal: observed-entry output needs the row-Gram route");
    const int64_t total = (int64_t)m * w.ld;
    if (!row_gram) {
        // Y_0 = S densified
        hipLaunchKernelGGL(fill_f32_kernel, dim3((int)std::min<int64_t>(8192, (total + 255) / 256)), dim3(256), 0, st,
                           w.Y[0], total, 0.f);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(densify_kernel, dim3(std::min(m, 8192)), dim3(256), 0, st, m, rowptr, colidx, val, w.Y[0],
                           w.ld);
        HIP_TRY(hipGetLastError());
    }
    if (o->K == 1) {
        hipLaunchKernelGGL(scale_copy_kernel, dim3((int)std::min<int64_t>(4096, (total + 255) / 256)), dim3(256), 0,
                           st, m, n, (const float*)w.Y[0], w.ld, Y, ldy, (const double*)w.scal);
        HIP_TRY(hipGetLastError());
        return CPA_OK;
    }
    if (nnz > 0) {
        hipLaunchKernelGGL(csc_values_kernel, dim3((int)std::min<int64_t>(4096, (nnz + 255) / 256)), dim3(256), 0, st,
                           nnz, csrc, val, w.cval);
        HIP_TRY(hipGetLastError());
    }
    if (poly) {
        // matrix-polynomial route: Gram S^T S (by rows of S, or one sparse product with
        // the densified S for n above the LDS rows), the polynomial on the n x n side,
        // then Y = S p (or its observed entries)
        if (row_gram)
            hipLaunchKernelGGL(sp_gram_kernel, dim3(n), dim3(64 * SPG_WAVES), 0, st, n, colptr, crow,
                               (const float*)w.cval, rowptr, colidx, val, w.W, w.ld);
        else
            hipLaunchKernelGGL(spmm_t_kernel, dim3(((n + SP_WAVES - 1) / SP_WAVES) * ((n + SPT_J - 1) / SPT_J)),
                               dim3(SP_THREADS), 0, st, n, n, colptr, crow, (const float*)w.cval,
                               (const float*)w.Y[0], w.ld, w.W, w.ld);
        HIP_TRY(hipGetLastError());
        float* F = nullptr;
        cpa_status r = enqueue_poly_core(ctx, st, n, w.W, w.ld, w.scal, w.lay.ps(), w.poly, w.poly_s, o->K,
                                         CPA_PREC_FP32, &F, false);
        if (r != CPA_OK) return r;
        if (xv) {
            hipLaunchKernelGGL(sp_sddmm_kernel, dim3(n), dim3(64 * SPS_WAVES), 0, st, n, colptr, crow, csrc, rowptr,
                               colidx, val, (const float*)F, (int64_t)n, xv);
            HIP_TRY(hipGetLastError());
            return CPA_OK;
        }
        hipLaunchKernelGGL(spmm_out_kernel, dim3(((m + SP_WAVES - 1) / SP_WAVES) * ((n + SPC_J - 1) / SPC_J)),
                           dim3(SP_THREADS), 0, st, m, n, rowptr, colidx, val, (const float*)F, (int64_t)n, Y, ldy,
                           aligned16(F, n) ? 1 : 0, aligned16(Y, ldy) ? 1 : 0);
        HIP_TRY(hipGetLastError());
        return CPA_OK;
    }
    const int grid_t = ((n + SP_WAVES - 1) / SP_WAVES) * ((n + SPT_J - 1) / SPT_J);
    const int grid_c = ((m + SP_WAVES - 1) / SP_WAVES) * ((n + SPC_J - 1) / SPC_J);
    for (int k = 0; k + 1 <= o->K - 1; ++k) {
        const float* yk = w.Y[k & 1];
        const float* yp = w.Y[(k + 1) & 1];
        float* ydst = w.Y[(k + 1) & 1];
        hipEvent_t ea, eb;
        cpa_status s = timing_pair(ctx, 0, ea, eb);
        if (s != CPA_OK) return s;
        if (ea) HIP_TRY(hipEventRecord(ea, st));
        hipLaunchKernelGGL(spmm_t_kernel, dim3(grid_t), dim3(SP_THREADS), 0, st, n, n, colptr, crow,
                           (const float*)w.cval, yk, w.ld, w.W, w.ld);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(spmm_cheb_kernel, dim3(grid_c), dim3(SP_THREADS), 0, st, m, n, rowptr, colidx, val,
                           (const float*)w.W, w.ld, yk, yp, ydst, w.ld, Y, ldy, (const double*)w.scal, k,
                           (k + 1 == o->K - 1) ? 1 : 0, aligned16(Y, ldy) ? 1 : 0);
        HIP_TRY(hipGetLastError());
        if (eb) HIP_TRY(hipEventRecord(eb, st));
    }
    return CPA_OK;
}

cpa_status check_csr_args(cpa_ctx* ctx, int m, int n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                          const float* val, float* Y, int64_t ldy) {
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (m < 0 || n < 0 || nnz < 0) return fail(CPA_ERR_SHAPE, "negative size");
    if (m < n) return fail(CPA_ERR_UNSUPPORTED, "sparse path needs m >= n; shrink the transpose (CSC) instead");
    if (nnz > INT32_MAX || (int64_t)m * n > ((int64_t)1 << 33)) return fail(CPA_ERR_SHAPE, "sparse matrix too large");
    if (m == 0 || n == 0) return CPA_OK;
    if (!rowptr || (nnz > 0 && (!colidx || !val)) || !Y) return fail(CPA_ERR_ARG, "NULL array");
    if (ldy < n) return fail(CPA_ERR_SHAPE, "ldy < n");
    return CPA_OK;
}

cpa_status check_dense_args(cpa_ctx* ctx, int m, int n, const float* X, int64_t ldx) {
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (m < 0 || n < 0) return fail(CPA_ERR_SHAPE, "negative size %d x %d", m, n);
    if ((int64_t)m * n > (int64_t)1 << 31) return fail(CPA_ERR_SHAPE, "matrix too large");
    if (m > 0 && n > 0) {
        if (!X) return fail(CPA_ERR_ARG, "X is NULL");
        if (ldx < n) return fail(CPA_ERR_SHAPE, "ldx %lld < n %d", (long long)ldx, n);
    }
    return CPA_OK;
}

}  // namespace

extern "C" {

cpa_status cpa_create(cpa_ctx** ctx_out, int device) {
    if (!ctx_out) return fail(CPA_ERR_ARG, "ctx_out is NULL");
    *ctx_out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(CPA_ERR_ARG, "device %d out of range (%d devices)", device, count);
    HIP_TRY(hipSetDevice(device));
    void* scratch_ptr = nullptr;
    if (device < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(CPA_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
            g_scratch_ptr[device] = p;
            g_scratch_warm_d[device] = -1;
        }
        scratch_ptr = g_scratch_ptr[device];
    }
    cpa_ctx* c = new (std::nothrow) cpa_ctx();
    if (!c) return fail(CPA_ERR_ALLOC, "context allocation failed");
    c->device = device;
    c->scratch = scratch_ptr;
    *ctx_out = c;
    return CPA_OK;
}

cpa_status cpa_destroy(cpa_ctx* ctx) {
    if (!ctx) return CPA_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->warm) (void)hipFree(ctx->warm);
    for (auto& L : ctx->tlog)
        for (hipEvent_t e : L.ev) (void)hipEventDestroy(e);
    if (ctx->admm_exec) (void)hipGraphExecDestroy(ctx->admm_exec);
    if (ctx->admm_exec_chunk) (void)hipGraphExecDestroy(ctx->admm_exec_chunk);
    if (ctx->queue) (void)hipFree(ctx->queue);
    if (ctx->spf) (void)hipFree(ctx->spf);
    if (ctx->spf_host) (void)hipHostFree(ctx->spf_host);
    if (ctx->inp) (void)hipFree(ctx->inp);
    if (ctx->f64) (void)hipFree(ctx->f64);
    if (ctx->rpca) (void)hipFree(ctx->rpca);
    if (ctx->mlp_ws) (void)hipFree(ctx->mlp_ws);
    if (ctx->sws) (void)hipFree(ctx->sws);
    if (ctx->csc) (void)hipFree(ctx->csc);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return CPA_OK;
}

const char* cpa_status_string(cpa_status s) {
    switch (s) {
        case CPA_OK: return "CPA_OK";
        case CPA_ERR_ARG: return "CPA_ERR_ARG";
        case CPA_ERR_SHAPE: return "CPA_ERR_SHAPE";
        case CPA_ERR_ALLOC: return "CPA_ERR_ALLOC";
        case CPA_ERR_HIP: return "CPA_ERR_HIP";
        case CPA_ERR_NONFINITE: return "CPA_ERR_NONFINITE";
        case CPA_ERR_BOUND: return "CPA_ERR_BOUND";
        case CPA_ERR_UNSUPPORTED: return "CPA_ERR_UNSUPPORTED";
        case CPA_ERR_IO: return "CPA_ERR_IO";
    }
    return "CPA_ERR_UNKNOWN";
}

const char* cpa_last_error(void) { return g_err; }

cpa_status cpa_workspace_bytes(cpa_ctx* ctx, int m, int n, const cpa_opts* opts, size_t* bytes_host) {
    cpa_status s;
    if (!ctx || !bytes_host) return fail(CPA_ERR_ARG, "NULL argument");
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if (m < 0 || n < 0) return fail(CPA_ERR_SHAPE, "negative size");
    *bytes_host = 0;
    if (m == 0 || n == 0) return CPA_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    Work w;
    const int maxit = power_slots(opts);
    return ensure_ws(ctx, m, n, opts->K, maxit, false, w, right_side(opts, m, n), poly_choice(opts, m, n), bytes_host);
}

void cpa_default_opts(cpa_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->K = 16;
    o->bound = CPA_BOUND_POWER;
    o->Lambda = 0.0;
    o->power_iters = 100;
    o->warm_start = 0;
    o->power_tol = 1e-7;
    o->margin = 0.01;
    o->seed = 0;
    o->check = 0;
    o->precision = CPA_PREC_FP32;
    o->growth_tol = 1e-3;
    o->eval = CPA_EVAL_AUTO;
    o->side = CPA_SIDE_AUTO;
}

cpa_status cpa_damping_factors(int K, int kind, double* g_host) {
    if (K < 1 || K > kMaxK) return fail(CPA_ERR_ARG, "K must be in [1, %d], got %d", kMaxK, K);
    if (kind < CPA_DAMP_NONE || kind > CPA_DAMP_LANCZOS) return fail(CPA_ERR_ARG, "unknown damping %d", kind);
    if (!g_host) return fail(CPA_ERR_ARG, "output pointer is NULL");
    for (int k = 0; k < K; ++k) g_host[k] = damping_factor(kind, K, k);
    return CPA_OK;
}

cpa_status cpa_chebyshev_coeffs(const cpa_shrinkage* shrink, double Lambda, int K, double* c_host) {
    cpa_status s = check_shrinkage(shrink);
    if (s != CPA_OK) return s;
    if (!c_host) return fail(CPA_ERR_ARG, "c_host is NULL");
    if (K < 1 || K > kMaxK) return fail(CPA_ERR_ARG, "K must be in [1, %d]", kMaxK);
    if (!(std::isfinite(Lambda) && Lambda >= 0.0)) return fail(CPA_ERR_ARG, "Lambda must be finite and >= 0");
    const ShrinkParams p = to_params(shrink);
    for (int k = 0; k < K; ++k) c_host[k] = cheb_coeff(p, Lambda, K, k);
    return CPA_OK;
}

cpa_status cpa_design_coeffs(const cpa_shrinkage* shrink, double Lambda, int K, int design_kind, int n,
                             double* c_host, double* err_host) {
    cpa_status s = check_shrinkage(shrink);
    if (s != CPA_OK) return s;
    if (!c_host) return fail(CPA_ERR_ARG, "c_host is NULL");
    if (K < 1 || K > kMaxDesignK) return fail(CPA_ERR_ARG, "K must be in [1, %d], got %d", kMaxDesignK, K);
    if (!(std::isfinite(Lambda) && Lambda >= 0.0)) return fail(CPA_ERR_ARG, "Lambda must be finite and >= 0");
    if (design_kind < CPA_DESIGN_CHEBYSHEV || design_kind > CPA_DESIGN_MINIMAX)
        return fail(CPA_ERR_ARG, "unknown design %d", design_kind);
    if (n == 0) n = design_kind == CPA_DESIGN_MINIMAX ? 8000 : 2000;
    if (design_kind == CPA_DESIGN_LSQ && (n < K || n < 2 || n > kMaxDesignN))
        return fail(CPA_ERR_ARG, "least squares needs K <= n <= %d samples (n >= 2), got %d", kMaxDesignN, n);
    if (design_kind == CPA_DESIGN_MINIMAX && (n < 2 * K + 1 || n > kMaxDesignN))
        return fail(CPA_ERR_ARG, "minimax needs 2 K + 1 <= n <= %d grid points, got %d", kMaxDesignN, n);
    if (design_kind != CPA_DESIGN_CHEBYSHEV && (int64_t)n * K > kMaxDesignNK)
        return fail(CPA_ERR_ARG, "n K = %lld exceeds %lld (the n x K basis matrix is held in host memory)",
                    (long long)n * K, (long long)kMaxDesignNK);
    const ShrinkParams p = to_params(shrink);
    double err = 0.0;
    if (!(Lambda > 0.0)) {
        for (int k = 0; k < K; ++k) c_host[k] = 0.0;
    } else if (design_kind == CPA_DESIGN_CHEBYSHEV) {
        for (int k = 0; k < K; ++k) c_host[k] = cheb_coeff(p, Lambda, K, k);
        for (int l = 0; l < K; ++l) {
            const double th = design::kPi * (l + 0.5) / K;
            double v = 0.5 * c_host[0];
            for (int k = 1; k < K; ++k) v += c_host[k] * cos(k * th);
            err = std::max(err, fabs(shrink_h(p, 0.5 * Lambda * (cos(th) + 1.0)) - v));
        }
    } else {
        err = design_kind == CPA_DESIGN_LSQ ? design::lsq(p, Lambda, K, n, c_host)
                                            : design::minimax(p, Lambda, K, n, 200, 1e-10, c_host);
        if (err < 0.0) return fail(CPA_ERR_NONFINITE, "a reference system of the Remez exchange is singular");
        c_host[0] *= 2.0;   // plain coefficients -> the c_0 / 2 convention
    }
    if (err_host) *err_host = err;
    return CPA_OK;
}

cpa_status cpa_spectral_bound(cpa_ctx* ctx, void* stream, int m, int n, const float* X_dev, int64_t ldx,
                              const cpa_opts* opts, double* Lambda_host, cpa_info* info_host) {
    cpa_status s;
    if ((s = check_dense_args(ctx, m, n, X_dev, ldx)) != CPA_OK) return s;
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if (!Lambda_host) return fail(CPA_ERR_ARG, "Lambda_host is NULL");
    if (m == 0 || n == 0) {
        *Lambda_host = 0.0;
        if (info_host) std::memset(info_host, 0, sizeof(*info_host));
        return CPA_OK;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Work w;
    const int maxit = power_slots(opts);
    if ((s = ensure_ws(ctx, m, n, opts->K, maxit, false, w, right_side(opts, m, n))) != CPA_OK) return s;
    cpa_shrinkage soft0 = {CPA_SOFT, 0, 0.0, 0.0, 0.0, 1.0};
    if ((s = fill_scalars(st, w)) != CPA_OK) return s;
    if ((s = enqueue_gram(ctx, st, m, n, X_dev, ldx, w)) != CPA_OK) return s;
    if ((s = enqueue_bound(ctx, st, w.d, &soft0, opts, w, -1, nullptr, std::log((double)m * n))) != CPA_OK) return s;
    cpa_info tmp;
    if ((s = read_info(st, w, 1, m, n, &tmp, nullptr)) != CPA_OK) return s;
    *Lambda_host = tmp.Lambda;
    if (info_host) *info_host = tmp;
    return CPA_OK;
}

cpa_status cpa_shrink_dense(cpa_ctx* ctx, void* stream, int m, int n, const float* X_dev, int64_t ldx, float* Y_dev,
                            int64_t ldy, const cpa_shrinkage* shrink, const cpa_opts* opts, cpa_info* info_host) {
    cpa_status s;
    if ((s = check_dense_args(ctx, m, n, X_dev, ldx)) != CPA_OK) return s;
    if ((s = check_shrinkage(shrink)) != CPA_OK) return s;
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if (m == 0 || n == 0) {
        if (info_host) std::memset(info_host, 0, sizeof(*info_host));
        return CPA_OK;
    }
    if (!Y_dev) return fail(CPA_ERR_ARG, "Y is NULL");
    if (ldy < n) return fail(CPA_ERR_SHAPE, "ldy %lld < n %d", (long long)ldy, n);
    const size_t xb = sizeof(float) * ((size_t)(m - 1) * ldx + n);
    const size_t yb = sizeof(float) * ((size_t)(m - 1) * ldy + n);
    if (overlaps(X_dev, xb, Y_dev, yb)) return fail(CPA_ERR_ARG, "Y overlaps X");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Work w;
    const int maxit = power_slots(opts);
    if ((s = ensure_ws(ctx, m, n, opts->K, maxit, false, w, right_side(opts, m, n), poly_choice(opts, m, n))) != CPA_OK)
        return s;
    return shrink_impl(ctx, st, m, n, X_dev, ldx, Y_dev, ldy, shrink, opts, info_host, w);
}

cpa_status cpa_shrink_dense_noalloc(cpa_ctx* ctx, void* stream, int m, int n, const float* X_dev, int64_t ldx,
                                    float* Y_dev, int64_t ldy, const cpa_shrinkage* shrink, const cpa_opts* opts,
                                    cpa_info* info_host) {
    cpa_status s;
    if ((s = check_dense_args(ctx, m, n, X_dev, ldx)) != CPA_OK) return s;
    if ((s = check_shrinkage(shrink)) != CPA_OK) return s;
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if (m == 0 || n == 0) {
        if (info_host) std::memset(info_host, 0, sizeof(*info_host));
        return CPA_OK;
    }
    if (!Y_dev) return fail(CPA_ERR_ARG, "Y is NULL");
    if (ldy < n) return fail(CPA_ERR_SHAPE, "ldy %lld < n %d", (long long)ldy, n);
    const size_t xb = sizeof(float) * ((size_t)(m - 1) * ldx + n);
    const size_t yb = sizeof(float) * ((size_t)(m - 1) * ldy + n);
    if (overlaps(X_dev, xb, Y_dev, yb)) return fail(CPA_ERR_ARG, "Y overlaps X");
    if (!ctx->scratch) return fail(CPA_ERR_UNSUPPORTED, "no scratch on device %d", ctx->device);
    const bool right = right_side(opts, m, n);
    const int d = right ? n : m;
    if (d > kScratchMaxD)
        return fail(CPA_ERR_SHAPE, "Gram side %d exceeds the allocation-free limit of %d", d, kScratchMaxD);
    HIP_TRY(hipSetDevice(ctx->device));
    if ((s = query_coop(ctx)) != CPA_OK) return s;
    Work w;
    const int maxit = power_slots(opts);
    const int ps = poly_choice(opts, m, n);
    const bool need_y = ps == 0;   // the recurrence over X (and the growth check's redo) needs the Y pair
    const WsPlan p = plan_ws(m, n, opts->K, maxit, false, w, right, ps, power_grid(ctx, d), need_y, false);
    if (p.total > kScratchBytes - kScratchWarmBytes)
        return fail(CPA_ERR_SHAPE, "this shrink needs %zu bytes of workspace; the allocation-free entry point has %zu",
                    p.total, kScratchBytes - kScratchWarmBytes);
    char* base = static_cast<char*>(ctx->scratch);
    bind_ws(w, base + kScratchWarmBytes, p, false, ps, need_y);
    w.warm_vec = reinterpret_cast<double*>(base);
    w.warm_len = &g_scratch_warm_d[ctx->device];
    // per-launch timing would create events: off for this call
    struct TimingOff {
        cpa_ctx* c;
        int saved;
        ~TimingOff() { c->timing = saved; }
    } guard{ctx, ctx->timing};
    ctx->timing = 0;
    return shrink_impl(ctx, static_cast<hipStream_t>(stream), m, n, X_dev, ldx, Y_dev, ldy, shrink, opts, info_host, w);
}

cpa_status cpa_timing_enable(cpa_ctx* ctx, int enable) {
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    ctx->timing = enable ? 1 : 0;
    for (auto& L : ctx->tlog) L.used = 0;
    return CPA_OK;
}

cpa_status cpa_timing_read(cpa_ctx* ctx, int which, double* total_ms_host, int64_t* launches_host) {
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (which < 0 || which > 2) return fail(CPA_ERR_ARG, "unknown kernel family %d", which);
    if (!total_ms_host || !launches_host) return fail(CPA_ERR_ARG, "output pointer is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    TimingLog& L = ctx->tlog[which];
    double tot = 0.0;
    for (size_t i = 0; i < L.used; ++i) {
        HIP_TRY(hipEventSynchronize(L.ev[2 * i + 1]));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, L.ev[2 * i], L.ev[2 * i + 1]));
        tot += ms;
    }
    *total_ms_host = tot;
    *launches_host = (int64_t)L.used;
    return CPA_OK;
}

namespace {

// Checks shared by the batched entry points; fills the common kernel arguments.
cpa_status batched_prepare(cpa_ctx* ctx, int batch, const int32_t* m_dev, const int32_t* n_dev,
                           const int64_t* off_dev, const float* X_dev, BatchArgs& a) {
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (batch < 0) return fail(CPA_ERR_SHAPE, "batch < 0");
    if (batch > 0 && (!m_dev || !n_dev || !off_dev || !X_dev)) return fail(CPA_ERR_ARG, "NULL array");
    std::memset(&a, 0, sizeof(a));
    a.batch = batch;
    a.m = m_dev;
    a.n = n_dev;
    a.off = off_dev;
    a.X = X_dev;
    a.K = 1;
    a.K_min = 1;
    a.shrink0 = ShrinkParams{0, 0.0, 0.0, 0.0, 1.0};
    return CPA_OK;
}

// Launch shape of the batched kernel (the autotuner's search space).
struct BatchConfig {
    int per_cu;   // persistent workgroups per CU (1 or the occupancy limit)
    int pair;     // recurrence output blocks per MFMA group (1 or 2)
    int order;    // 0: queue in index order, 1: largest d^2 e first
};

cpa_status batched_query(cpa_ctx* ctx) {
    if (ctx->batch_per_cu == 0) {
        int per_cu = 0, cus = 0;
        // every instantiation has the same LDS and the same register cap
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel<false, 2>, BT_THREADS, 0));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        ctx->batch_per_cu = std::max(1, per_cu);
        ctx->cus = std::max(1, cus);
    }
    return CPA_OK;
}

// Queue reset (a fill kernel, so the pair can be captured in a graph) and the kernel.
cpa_status batched_enqueue(hipStream_t st, const BatchArgs& a, bool split, int pair, int grid) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, st, a.queue, 1, 0);
    HIP_TRY(hipGetLastError());
    grid = std::max(1, std::min(a.batch, grid));
    if (split && pair == 2)
        hipLaunchKernelGGL((batched_kernel<true, 2>), dim3(grid), dim3(BT_THREADS), 0, st, a);
    else if (split)
        hipLaunchKernelGGL((batched_kernel<true, 1>), dim3(grid), dim3(BT_THREADS), 0, st, a);
    else if (pair == 2)
        hipLaunchKernelGGL((batched_kernel<false, 2>), dim3(grid), dim3(BT_THREADS), 0, st, a);
    else
        hipLaunchKernelGGL((batched_kernel<false, 1>), dim3(grid), dim3(BT_THREADS), 0, st, a);
    HIP_TRY(hipGetLastError());
    return CPA_OK;
}

// Direct calls: the default configuration (occupancy-limit grid, pairs, index order).
cpa_status batched_launch(cpa_ctx* ctx, void* stream, BatchArgs& a, bool split = false) {
    HIP_TRY(hipSetDevice(ctx->device));
    cpa_status s;
    if ((s = batched_query(ctx)) != CPA_OK) return s;
    if (!ctx->queue && hipMalloc(&ctx->queue, 256) != hipSuccess) {
        ctx->queue = nullptr;
        return fail(CPA_ERR_ALLOC, "queue allocation failed");
    }
    a.queue = ctx->queue;
    a.order = nullptr;
    return batched_enqueue(static_cast<hipStream_t>(stream), a, split, 2, ctx->batch_per_cu * ctx->cus);
}

cpa_status batched_shrink_args(const cpa_opts* opts, const float* X_dev, float* Y_dev,
                               const cpa_shrinkage* shrink_dev, const cpa_shrinkage* shrink_host, BatchArgs& a) {
    cpa_status s;
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if ((s = no_learned_bound(opts)) != CPA_OK) return s;
    if (opts->K > 64) return fail(CPA_ERR_ARG, "batched shrinkage supports K <= 64");
    if (opts->side != CPA_SIDE_AUTO) return fail(CPA_ERR_UNSUPPORTED, "batched shrinkage takes the smaller Gram (side auto)");
    if (opts->damping != CPA_DAMP_NONE) return fail(CPA_ERR_UNSUPPORTED, "batched shrinkage takes undamped coefficients");

    if (opts->check && !(opts->growth_tol >= 0.0)) return fail(CPA_ERR_ARG, "growth_tol must be >= 0");
    if (a.batch > 0 && !Y_dev) return fail(CPA_ERR_ARG, "NULL array");
    if (a.batch > 0 && X_dev == Y_dev) return fail(CPA_ERR_ARG, "Y aliases X");
    if (!shrink_dev && (s = check_shrinkage(shrink_host)) != CPA_OK) return s;
    a.Y = Y_dev;
    a.shrink = reinterpret_cast<const ShrinkRec*>(shrink_dev);
    if (!shrink_dev) a.shrink0 = to_params(shrink_host);
    a.K = opts->K;
    a.power_iters = opts->power_iters;
    a.lanczos = opts->bound == CPA_BOUND_LANCZOS ? lanczos_steps(opts) : 0;
    a.tol = opts->power_tol;
    a.margin = opts->margin;
    a.seed = opts->seed;
    a.check = opts->check ? 1 : 0;
    a.growth_tol = opts->growth_tol;
    return CPA_OK;
}

}  // namespace

cpa_status cpa_shrink_batched(cpa_ctx* ctx, void* stream, int batch, const int32_t* m_dev, const int32_t* n_dev,
                              const int64_t* off_dev, const float* X_dev, float* Y_dev,
                              const cpa_shrinkage* shrink_dev, const cpa_shrinkage* shrink_host,
                              const cpa_opts* opts, const double* Lambda_dev, double* Lambda_out_dev,
                              int32_t* status_dev) {
    cpa_status s;
    BatchArgs a;
    if ((s = batched_prepare(ctx, batch, m_dev, n_dev, off_dev, X_dev, a)) != CPA_OK) return s;
    if ((s = batched_shrink_args(opts, X_dev, Y_dev, shrink_dev, shrink_host, a)) != CPA_OK) return s;
    if (opts->bound == CPA_BOUND_GIVEN && !Lambda_dev) return fail(CPA_ERR_ARG, "Lambda_dev is NULL");
    if (batch == 0) return CPA_OK;
    a.mode = (opts->bound == CPA_BOUND_POWER || opts->bound == CPA_BOUND_LANCZOS) ? 0
             : opts->bound == CPA_BOUND_GIVEN                                     ? 1
                                                                                  : 2;
    a.lambda_in = Lambda_dev;
    a.lambda_out = Lambda_out_dev;
    a.status = status_dev;
    return batched_launch(ctx, stream, a, opts->precision == CPA_PREC_BF16X3);
}

cpa_status cpa_batched_features(cpa_ctx* ctx, void* stream, int batch, const int32_t* m_dev, const int32_t* n_dev,
                                const int64_t* off_dev, const float* X_dev, float* feat_dev, int32_t* status_dev) {
    cpa_status s;
    BatchArgs a;
    if ((s = batched_prepare(ctx, batch, m_dev, n_dev, off_dev, X_dev, a)) != CPA_OK) return s;
    if (batch > 0 && !feat_dev) return fail(CPA_ERR_ARG, "feat_dev is NULL");
    if (batch == 0) return CPA_OK;
    a.mode = 4;
    a.feat_out = feat_dev;
    a.status = status_dev;
    return batched_launch(ctx, stream, a);
}

cpa_status cpa_shrink_batched_predicted(cpa_ctx* ctx, void* stream, int batch, const int32_t* m_dev,
                                        const int32_t* n_dev, const int64_t* off_dev, const float* X_dev,
                                        float* Y_dev, const cpa_shrinkage* shrink_dev,
                                        const cpa_shrinkage* shrink_host, const cpa_opts* opts,
                                        const float* model_dev, int32_t K_min, double* Lambda_out_dev,
                                        int32_t* K_out_dev, int32_t* status_dev) {
    cpa_status s;
    BatchArgs a;
    if ((s = batched_prepare(ctx, batch, m_dev, n_dev, off_dev, X_dev, a)) != CPA_OK) return s;
    if ((s = batched_shrink_args(opts, X_dev, Y_dev, shrink_dev, shrink_host, a)) != CPA_OK) return s;
    if (!model_dev) return fail(CPA_ERR_ARG, "model_dev is NULL");
    if (reinterpret_cast<uintptr_t>(model_dev) % 16 != 0) return fail(CPA_ERR_ARG, "model_dev must be 16-byte aligned");
    if (K_min < 1 || K_min > opts->K) return fail(CPA_ERR_ARG, "K_min must be in [1, opts->K]");
    if (opts->power_iters < 1 || opts->power_iters > kMaxPowerIters)
        return fail(CPA_ERR_ARG, "power_iters must be in [1, %d] (used by the fallback)", kMaxPowerIters);
    if (!(opts->power_tol >= 0.0) || !(opts->margin >= 0.0)) return fail(CPA_ERR_ARG, "power_tol and margin must be >= 0");
    if (batch == 0) return CPA_OK;
    a.mode = 3;
    a.model = model_dev;
    a.K_min = K_min;
    a.lambda_out = Lambda_out_dev;
    a.K_out = K_out_dev;
    a.status = status_dev;
    return batched_launch(ctx, stream, a, opts->precision == CPA_PREC_BF16X3);
}

}  // extern "C"

struct cpa_batched_plan {
    int device = 0;
    BatchArgs a;                  // bound buffers; queue and order are the plan's own
    bool split = false;
    BatchConfig cfg{2, 2, 0};
    int grid = 1;
    int* queue = nullptr;
    int32_t* order = nullptr;     // largest-first queue order (used when cfg.order == 1)
    hipGraphExec_t exec = nullptr;
    cpa_batched_tuning tun{};
};

namespace {

void plan_free(cpa_batched_plan* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->queue) (void)hipFree(p->queue);
    if (p->order) (void)hipFree(p->order);
    delete p;
}

// Largest-first queue order by the recurrence work d^2 e of every matrix (stable;
// shapes outside the limits last).
cpa_status plan_order(cpa_batched_plan* p, hipStream_t st) {
    const int b = p->a.batch;
    std::vector<int32_t> m(b), n(b);
    HIP_TRY(hipMemcpyAsync(m.data(), p->a.m, sizeof(int32_t) * b, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(n.data(), p->a.n, sizeof(int32_t) * b, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int64_t> cost(b);
    for (int j = 0; j < b; ++j) {
        const int64_t d = std::min(m[j], n[j]), e = std::max(m[j], n[j]);
        cost[j] = (d >= 1 && d <= BT_DMAX && e <= BT_EMAX) ? d * d * e : -1;
    }
    std::vector<int32_t> ord(b);
    for (int j = 0; j < b; ++j) ord[j] = j;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
    HIP_TRY(hipMemcpyAsync(p->order, ord.data(), sizeof(int32_t) * b, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return CPA_OK;
}

cpa_status plan_enqueue(cpa_batched_plan* p, hipStream_t st, const BatchConfig& c, int per_cu_max, int cus) {
    BatchArgs a = p->a;
    a.queue = p->queue;
    a.order = c.order ? p->order : nullptr;
    return batched_enqueue(st, a, p->split, c.pair, std::min(c.per_cu, per_cu_max) * cus);
}

// Mean time of `reps` launches of configuration c (after one untimed launch), in us.
cpa_status plan_time(cpa_batched_plan* p, hipStream_t st, const BatchConfig& c, int per_cu_max, int cus, int reps,
                     double& us) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(CPA_ERR_HIP, "event creation failed");
    }
    cpa_status s = plan_enqueue(p, st, c, per_cu_max, cus);
    if (s == CPA_OK && hipEventRecord(e0, st) != hipSuccess) s = fail(CPA_ERR_HIP, "event record failed");
    for (int r = 0; s == CPA_OK && r < reps; ++r) s = plan_enqueue(p, st, c, per_cu_max, cus);
    if (s == CPA_OK && hipEventRecord(e1, st) != hipSuccess) s = fail(CPA_ERR_HIP, "event record failed");
    if (s == CPA_OK && hipEventSynchronize(e1) != hipSuccess) s = fail(CPA_ERR_HIP, "event wait failed");
    float ms = 0.f;
    if (s == CPA_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = fail(CPA_ERR_HIP, "event timing failed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    us = 1e3 * (double)ms / reps;
    return s;
}

}  // namespace

extern "C" {

cpa_status cpa_batched_plan_create(cpa_ctx* ctx, void* stream, int batch, const int32_t* m_dev, const int32_t* n_dev,
                                   const int64_t* off_dev, const float* X_dev, float* Y_dev,
                                   const cpa_shrinkage* shrink_dev, const cpa_shrinkage* shrink_host,
                                   const cpa_opts* opts, const double* Lambda_dev, double* Lambda_out_dev,
                                   int32_t* status_dev, int32_t tune, cpa_batched_plan** plan_out) {
    if (!plan_out) return fail(CPA_ERR_ARG, "plan_out is NULL");
    *plan_out = nullptr;
    cpa_status s;
    BatchArgs a;
    if ((s = batched_prepare(ctx, batch, m_dev, n_dev, off_dev, X_dev, a)) != CPA_OK) return s;
    if ((s = batched_shrink_args(opts, X_dev, Y_dev, shrink_dev, shrink_host, a)) != CPA_OK) return s;
    if (opts->bound == CPA_BOUND_GIVEN && !Lambda_dev) return fail(CPA_ERR_ARG, "Lambda_dev is NULL");
    if (tune != 0 && tune != 1) return fail(CPA_ERR_ARG, "tune must be 0 or 1");
    a.mode = (opts->bound == CPA_BOUND_POWER || opts->bound == CPA_BOUND_LANCZOS) ? 0
             : opts->bound == CPA_BOUND_GIVEN                                     ? 1
                                                                                  : 2;
    a.lambda_in = Lambda_dev;
    a.lambda_out = Lambda_out_dev;
    a.status = status_dev;
    HIP_TRY(hipSetDevice(ctx->device));
    if ((s = batched_query(ctx)) != CPA_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);

    cpa_batched_plan* p = new (std::nothrow) cpa_batched_plan();
    if (!p) return fail(CPA_ERR_ALLOC, "plan allocation failed");
    p->device = ctx->device;
    p->a = a;
    p->split = opts->precision == CPA_PREC_BF16X3;
    const BatchConfig dflt{ctx->batch_per_cu, 2, 0};
    p->cfg = dflt;
    if (hipMalloc(&p->queue, 256) != hipSuccess) {
        p->queue = nullptr;
        plan_free(p);
        return fail(CPA_ERR_ALLOC, "queue allocation failed");
    }
    if (batch > 0) {
        if (hipMalloc(&p->order, sizeof(int32_t) * (size_t)batch) != hipSuccess) {
            p->order = nullptr;
            plan_free(p);
            return fail(CPA_ERR_ALLOC, "order allocation failed");
        }
        if ((s = plan_order(p, st)) != CPA_OK) {
            plan_free(p);
            return s;
        }
    }
    if (tune && batch > 0) {
        // every configuration computes the same results; keep the fastest
        double best = 0.0;
        int ncand = 0;
        for (int per_cu = 1; per_cu <= std::min(2, ctx->batch_per_cu); ++per_cu)
            for (int pair = 1; pair <= 2; ++pair)
                for (int ord = 0; ord <= 1; ++ord) {
                    const BatchConfig c{per_cu, pair, ord};
                    double us = 0.0;
                    if ((s = plan_time(p, st, c, ctx->batch_per_cu, ctx->cus, 3, us)) != CPA_OK) {
                        plan_free(p);
                        return s;
                    }
                    ++ncand;
                    if (per_cu == dflt.per_cu && pair == dflt.pair && ord == dflt.order) p->tun.default_us = us;
                    if (ncand == 1 || us < best) {
                        best = us;
                        p->cfg = c;
                    }
                }
        p->tun.candidates = ncand;
        p->tun.best_us = best;
    }
    p->grid = std::max(1, std::min(batch, p->cfg.per_cu * ctx->cus));
    p->tun.grid = p->grid;
    p->tun.pair = p->cfg.pair;
    p->tun.order = p->cfg.order;

    // capture the chosen launch (queue reset + kernel) once; replays bake in every argument
    if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        ctx->cap_stream = nullptr;
        plan_free(p);
        return fail(CPA_ERR_HIP, "capture stream creation failed");
    }
    if (batch > 0) {
        hipGraph_t g;
        if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            plan_free(p);
            return fail(CPA_ERR_HIP, "graph capture could not start");
        }
        const cpa_status cs = plan_enqueue(p, ctx->cap_stream, p->cfg, ctx->batch_per_cu, ctx->cus);
        const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
        if (cs != CPA_OK || ce != hipSuccess) {
            if (ce == hipSuccess) (void)hipGraphDestroy(g);
            plan_free(p);
            return cs != CPA_OK ? cs : fail(CPA_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ce));
        }
        const hipError_t ie = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            p->exec = nullptr;
            plan_free(p);
            return fail(CPA_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
        }
    }
    *plan_out = p;
    return CPA_OK;
}

cpa_status cpa_batched_plan_execute(cpa_batched_plan* plan, void* stream) {
    if (!plan) return fail(CPA_ERR_ARG, "plan is NULL");
    if (!plan->exec) return CPA_OK;   // empty batch
    HIP_TRY(hipSetDevice(plan->device));
    HIP_TRY(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
    return CPA_OK;
}

cpa_status cpa_batched_plan_tuning(const cpa_batched_plan* plan, cpa_batched_tuning* out) {
    if (!plan || !out) return fail(CPA_ERR_ARG, "NULL argument");
    *out = plan->tun;
    return CPA_OK;
}

cpa_status cpa_batched_plan_destroy(cpa_batched_plan* plan) {
    plan_free(plan);
    return CPA_OK;
}

namespace {

cpa_status ensure_mlp_ws(cpa_ctx* ctx, float*& part, double*& lpart) {
    const size_t pbytes = align_up(sizeof(float) * (size_t)kMlpMaxWg * kMlpParams);
    if (!ctx->mlp_ws) {
        if (hipMalloc(&ctx->mlp_ws, pbytes + sizeof(double) * kMlpMaxWg) != hipSuccess) {
            ctx->mlp_ws = nullptr;
            return fail(CPA_ERR_ALLOC, "predictor workspace allocation failed");
        }
    }
    part = static_cast<float*>(ctx->mlp_ws);
    lpart = reinterpret_cast<double*>(static_cast<char*>(ctx->mlp_ws) + pbytes);
    return CPA_OK;
}

cpa_status check_model(const float* model_dev) {
    if (!model_dev) return fail(CPA_ERR_ARG, "model_dev is NULL");
    if (reinterpret_cast<uintptr_t>(model_dev) % 16 != 0) return fail(CPA_ERR_ARG, "model_dev must be 16-byte aligned");
    return CPA_OK;
}

cpa_status check_quantiles(const float* q) {
    if (!q) return fail(CPA_ERR_ARG, "quantiles_host is NULL");
    for (int o = 0; o < 2; ++o)
        if (!(q[o] > 0.f && q[o] < 1.f)) return fail(CPA_ERR_ARG, "quantiles must lie in (0, 1)");
    return CPA_OK;
}

}  // namespace

cpa_status cpa_predictor_forward(cpa_ctx* ctx, void* stream, int64_t n, const float* feat_dev,
                                 const float* model_dev, float* y_dev) {
    cpa_status s;
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (n < 0) return fail(CPA_ERR_SHAPE, "n < 0");
    if ((s = check_model(model_dev)) != CPA_OK) return s;
    if (n == 0) return CPA_OK;
    if (!feat_dev || !y_dev) return fail(CPA_ERR_ARG, "NULL array");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    MlpArgs a;
    std::memset(&a, 0, sizeof(a));
    a.feat = feat_dev;
    a.model = model_dev;
    a.y = y_dev;
    a.s0 = 0;
    a.count = n;
    const int64_t tiles = (n + kMlpH - 1) / kMlpH;
    const int grid = (int)std::min<int64_t>(tiles, 2048);
    hipLaunchKernelGGL(mlp_tile_kernel<false>, dim3(grid), dim3(kMlpThreads), 0, st, a);
    HIP_TRY(hipGetLastError());
    return CPA_OK;
}

cpa_status cpa_predictor_grad(cpa_ctx* ctx, void* stream, int64_t n, const float* feat_dev, const float* targ_dev,
                              const float* quantiles_host, const float* model_dev, float* grad_dev,
                              double* loss_dev) {
    cpa_status s;
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (n < 1) return fail(CPA_ERR_SHAPE, "n must be >= 1");
    if ((s = check_model(model_dev)) != CPA_OK) return s;
    if ((s = check_quantiles(quantiles_host)) != CPA_OK) return s;
    if (!feat_dev || !targ_dev || !grad_dev) return fail(CPA_ERR_ARG, "NULL array");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    float* part;
    double* lpart;
    if ((s = ensure_mlp_ws(ctx, part, lpart)) != CPA_OK) return s;
    MlpArgs a;
    std::memset(&a, 0, sizeof(a));
    a.feat = feat_dev;
    a.targ = targ_dev;
    a.model = model_dev;
    a.part = part;
    a.lpart = lpart;
    a.s0 = 0;
    a.count = n;
    a.q0 = quantiles_host[0];
    a.q1 = quantiles_host[1];
    a.dscale = (float)(1.0 / (2.0 * (double)n));
    const int64_t tiles = (n + kMlpH - 1) / kMlpH;
    const int grid = (int)std::min<int64_t>(tiles, kMlpMaxWg);
    hipLaunchKernelGGL(mlp_tile_kernel<true>, dim3(grid), dim3(kMlpThreads), 0, st, a);
    HIP_TRY(hipGetLastError());
    if (loss_dev) {
        hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(64), 0, st, loss_dev, 1, 0.0);
        HIP_TRY(hipGetLastError());
    }
    AdamArgs r;
    std::memset(&r, 0, sizeof(r));
    r.part = part;
    r.nwg = grid;
    r.lpart = lpart;
    r.grad_out = grad_dev;
    r.loss_dst = loss_dev;
    r.loss_mul = 1.0 / (2.0 * (double)n);
    r.adam = 0;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, r);
    HIP_TRY(hipGetLastError());
    return CPA_OK;
}

cpa_status cpa_predictor_train(cpa_ctx* ctx, void* stream, int64_t n, const float* feat_dev, const float* targ_dev,
                               const float* quantiles_host, int32_t batch_size, int32_t epochs, float lr,
                               float* model_dev, float* adam_dev, int64_t* step_io_host, double* epoch_loss_dev) {
    cpa_status s;
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (n < 1) return fail(CPA_ERR_SHAPE, "n must be >= 1");
    if ((s = check_model(model_dev)) != CPA_OK) return s;
    if ((s = check_quantiles(quantiles_host)) != CPA_OK) return s;
    if (!feat_dev || !targ_dev || !adam_dev || !step_io_host) return fail(CPA_ERR_ARG, "NULL argument");
    if (batch_size < 1 || batch_size > kMlpH * kMlpMaxWg)
        return fail(CPA_ERR_ARG, "batch_size must be in [1, %d]", kMlpH * kMlpMaxWg);
    if (epochs < 0) return fail(CPA_ERR_ARG, "epochs < 0");
    if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(CPA_ERR_ARG, "lr must be finite and >= 0");
    if (*step_io_host < 0) return fail(CPA_ERR_ARG, "*step_io_host < 0");
    if (epochs == 0) return CPA_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    float* part;
    double* lpart;
    if ((s = ensure_mlp_ws(ctx, part, lpart)) != CPA_OK) return s;
    if (epoch_loss_dev) {
        hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(256), 0, st, epoch_loss_dev, epochs, 0.0);
        HIP_TRY(hipGetLastError());
    }
    const int64_t steps = (n + batch_size - 1) / batch_size;
    const double beta1 = 0.9, beta2 = 0.999;
    int64_t t = *step_io_host;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t b = 0; b < steps; ++b) {
            const int64_t s0 = b * batch_size;
            const int64_t cnt = std::min<int64_t>(batch_size, n - s0);
            MlpArgs a;
            std::memset(&a, 0, sizeof(a));
            a.feat = feat_dev;
            a.targ = targ_dev;
            a.model = model_dev;
            a.part = part;
            a.lpart = lpart;
            a.s0 = s0;
            a.count = cnt;
            a.q0 = quantiles_host[0];
            a.q1 = quantiles_host[1];
            a.dscale = (float)(1.0 / (2.0 * (double)cnt));
            const int grid = (int)((cnt + kMlpH - 1) / kMlpH);
            hipLaunchKernelGGL(mlp_tile_kernel<true>, dim3(grid), dim3(kMlpThreads), 0, st, a);
            HIP_TRY(hipGetLastError());
            ++t;
            AdamArgs r;
            std::memset(&r, 0, sizeof(r));
            r.part = part;
            r.nwg = grid;
            r.lpart = lpart;
            r.model = model_dev;
            r.m = adam_dev;
            r.v = adam_dev + kMlpParams;
            r.lr = lr;
            r.beta1 = (float)beta1;
            r.beta2 = (float)beta2;
            r.eps = 1e-8f;
            r.bc1 = 1.0 - std::pow(beta1, (double)t);
            r.bc2 = 1.0 - std::pow(beta2, (double)t);
            r.loss_dst = epoch_loss_dev ? epoch_loss_dev + ep : nullptr;
            r.loss_mul = 1.0 / (2.0 * (double)cnt * (double)steps);
            r.adam = 1;
            hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, r);
            HIP_TRY(hipGetLastError());
        }
    }
    *step_io_host = t;
    return CPA_OK;
}

cpa_status cpa_shrink_csr(cpa_ctx* ctx, void* stream, int m, int n, int64_t nnz, const int32_t* rowptr_dev,
                          const int32_t* colidx_dev, const float* val_dev, float* Y_dev, int64_t ldy,
                          const cpa_shrinkage* shrink, const cpa_opts* opts, cpa_info* info_host) {
    cpa_status s;
    if ((s = check_csr_args(ctx, m, n, nnz, rowptr_dev, colidx_dev, val_dev, Y_dev, ldy)) != CPA_OK) return s;
    if (opts && opts->side == CPA_SIDE_LEFT) return fail(CPA_ERR_UNSUPPORTED, "sparse path forms S^T S (side right)");
    if ((s = check_shrinkage(shrink)) != CPA_OK) return s;
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if ((s = learned_bound_unsupported(opts)) != CPA_OK) return s;
    if (opts->precision != CPA_PREC_FP32) return fail(CPA_ERR_UNSUPPORTED, "sparse path is FP32");
    if (opts->check) return fail(CPA_ERR_UNSUPPORTED, "the growth check is not available on the sparse path");
    if (m == 0 || n == 0) {
        if (info_host) std::memset(info_host, 0, sizeof(*info_host));
        return CPA_OK;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    SpWork w;
    const int maxit = power_slots(opts);
    if ((s = ensure_sparse_ws(ctx, m, n, nnz, opts->K, maxit, false, w, sparse_poly_choice(opts, n))) != CPA_OK)
        return s;
    if ((s = ensure_csc(ctx, st, m, n, nnz, rowptr_dev, colidx_dev)) != CPA_OK) return s;
    if ((s = shrink_csr_impl(ctx, st, m, n, nnz, rowptr_dev, colidx_dev, val_dev, Y_dev, ldy, shrink, opts, w)) != CPA_OK)
        return s;
    if (info_host) {
        double h[SC_COEF];
        HIP_TRY(hipMemcpyAsync(h, w.scal, sizeof(h), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        std::memset(info_host, 0, sizeof(*info_host));
        info_host->Lambda = h[SC_LAMBDA];
        info_host->mu = h[SC_MU];
        info_host->resid = h[SC_RESID];
        info_host->fro_gram = h[SC_TRACE];
        info_host->power_iters_done = (int)h[SC_ITERS];
        if (h[SC_TIMEOUT] != 0.0) return fail(CPA_ERR_HIP, "power iteration grid barrier timed out");
        if (!std::isfinite(h[SC_TRACE])) return fail(CPA_ERR_NONFINITE, "S holds NaN or infinite values");
        if (!std::isfinite(h[SC_LAMBDA])) return fail(CPA_ERR_NONFINITE, "spectral bound is not finite");
    }
    return CPA_OK;
}

cpa_status cpa_svt_complete(cpa_ctx* ctx, void* stream, int m, int n, int64_t nnz, const int32_t* rowptr_dev,
                            const int32_t* colidx_dev, const float* Mobs_dev, double tau, double delta, int iters,
                            float* X_dev, int64_t ldx, const cpa_opts* opts, double* resid_dev, double* k0_host,
                            const float* Y0_vals_dev, float* Y_vals_dev, double* Lambda_dev) {
    cpa_status s;
    if ((s = check_csr_args(ctx, m, n, nnz, rowptr_dev, colidx_dev, Mobs_dev, X_dev, ldx)) != CPA_OK) return s;
    if (opts && opts->side == CPA_SIDE_LEFT) return fail(CPA_ERR_UNSUPPORTED, "sparse path forms S^T S (side right)");
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if ((s = no_learned_bound(opts)) != CPA_OK) return s;
    if (opts->precision != CPA_PREC_FP32 || opts->check) return fail(CPA_ERR_UNSUPPORTED, "unsupported option");
    if (!(std::isfinite(tau) && tau >= 0.0 && std::isfinite(delta) && delta > 0.0) || iters < 0)
        return fail(CPA_ERR_ARG, "tau >= 0, delta > 0 and iters >= 0 required");
    if (k0_host) *k0_host = 0.0;
    if (m == 0 || n == 0 || iters == 0) return CPA_OK;
    if (Y_vals_dev && Y0_vals_dev && Y_vals_dev != Y0_vals_dev &&
        overlaps(Y_vals_dev, sizeof(float) * nnz, Y0_vals_dev, sizeof(float) * nnz))
        return fail(CPA_ERR_ARG, "Y_vals overlaps Y0_vals (pass the same buffer to update in place)");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    SpWork w;
    const int maxit = power_slots(opts);
    const int ps = sparse_poly_choice(opts, n);
    if ((s = ensure_sparse_ws(ctx, m, n, nnz, opts->K, std::max(maxit, 200), true, w, ps)) != CPA_OK) return s;
    if ((s = ensure_csc(ctx, st, m, n, nnz, rowptr_dev, colidx_dev)) != CPA_OK) return s;
    const int gv = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (nnz + 255) / 256));
    if (Y0_vals_dev) {
        // continue from the caller's iterate
        if (nnz > 0) HIP_TRY(hipMemcpyAsync(w.yv, Y0_vals_dev, sizeof(float) * nnz, hipMemcpyDeviceToDevice, st));
    } else {
        // k0 = ceil(tau / (delta ||P_Omega M||_2)) from a converged power iteration (one sync)
        cpa_opts ob = *opts;
        ob.bound = CPA_BOUND_POWER;
        ob.power_iters = 200;
        ob.power_tol = 1e-9;
        ob.warm_start = 0;
        ob.K = 1;
        cpa_shrinkage s0 = {CPA_SOFT, 0, 0.0, 0.0, 0.0, 1.0};
        if ((s = shrink_csr_impl(ctx, st, m, n, nnz, rowptr_dev, colidx_dev, Mobs_dev, X_dev, ldx, &s0, &ob, w)) !=
            CPA_OK)
            return s;
        double mu = 0.0;
        HIP_TRY(hipMemcpyAsync(&mu, w.scal + SC_MU, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const double nrm2 = std::sqrt(std::max(mu, 0.0));
        const double k0 = nrm2 > 0.0 ? std::ceil(tau / (delta * nrm2)) : 1.0;
        if (k0_host) *k0_host = k0;
        hipLaunchKernelGGL(scale_vals_kernel, dim3(gv), dim3(256), 0, st, nnz, Mobs_dev, w.yv, (float)(k0 * delta));
        HIP_TRY(hipGetLastError());
    }
    // ||P_Omega M||_F for the residual normalisation (host, once)
    std::vector<float> hv(nnz);
    HIP_TRY(hipMemcpyAsync(hv.data(), Mobs_dev, sizeof(float) * nnz, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double nm = 0.0;
    for (float v : hv) nm += (double)v * v;
    nm = std::sqrt(nm);
    cpa_shrinkage sh = {CPA_SOFT, 0, tau, 0.0, 0.0, 1.0};
    // iterations before the last need only the observed entries of X^t (on the
    // matrix-polynomial route with the row Gram); the last one forms X^iters
    const bool observed_only = ps > 0 && opts->K >= 2 && n <= SPG_MAXN;
    const int gu = std::min(m, 4096);
    const int gvu = std::max(1, std::min(gv, gu));   // partials go to tvec (m doubles)
    for (int t = 0; t < iters; ++t) {
        const bool last = t + 1 == iters;
        if (observed_only && !last) {
            if ((s = shrink_csr_impl(ctx, st, m, n, nnz, rowptr_dev, colidx_dev, w.yv, X_dev, ldx, &sh, opts, w,
                                     w.xv)) != CPA_OK)
                return s;
            hipLaunchKernelGGL(svt_update_vals_kernel, dim3(gvu), dim3(256), 0, st, nnz, Mobs_dev, (const float*)w.xv,
                               w.yv, (float)delta, w.tvec);
            HIP_TRY(hipGetLastError());
            hipLaunchKernelGGL(svt_resid_kernel, dim3(1), dim3(256), 0, st, (const double*)w.tvec, gvu, nm,
                               resid_dev ? resid_dev + t : nullptr);
        } else {
            if ((s = shrink_csr_impl(ctx, st, m, n, nnz, rowptr_dev, colidx_dev, w.yv, X_dev, ldx, &sh, opts, w)) !=
                CPA_OK)
                return s;
            // residual partials reuse the power-iteration vector buffer (m doubles >= gu)
            hipLaunchKernelGGL(svt_update_kernel, dim3(gu), dim3(256), 0, st, m, rowptr_dev, colidx_dev, Mobs_dev,
                               (const float*)X_dev, ldx, w.yv, (float)delta, w.tvec);
            HIP_TRY(hipGetLastError());
            hipLaunchKernelGGL(svt_resid_kernel, dim3(1), dim3(256), 0, st, (const double*)w.tvec, gu, nm,
                               resid_dev ? resid_dev + t : nullptr);
        }
        HIP_TRY(hipGetLastError());
        if (Lambda_dev) {
            hipLaunchKernelGGL(copy_f64_kernel, dim3(1), dim3(64), 0, st, (const double*)(w.scal + SC_LAMBDA),
                               Lambda_dev + t);
            HIP_TRY(hipGetLastError());
        }
    }
    if (Y_vals_dev && nnz > 0)
        HIP_TRY(hipMemcpyAsync(Y_vals_dev, w.yv, sizeof(float) * nnz, hipMemcpyDeviceToDevice, st));
    return CPA_OK;
}

int64_t cpa_rpca_state_floats(int m, int n) {
    if (m < 0 || n < 0) return 0;
    return 7 * (int64_t)m * n;
}

cpa_status cpa_rpca_init(cpa_ctx* ctx, void* stream, int m, int n, float* state_dev) {
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (m < 0 || n < 0) return fail(CPA_ERR_SHAPE, "negative size");
    if (m == 0 || n == 0) return CPA_OK;
    if (!state_dev) return fail(CPA_ERR_ARG, "state is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t total = cpa_rpca_state_floats(m, n);
    hipLaunchKernelGGL(fill_f32_kernel, dim3(2048), dim3(256), 0, static_cast<hipStream_t>(stream), state_dev, total, 1.f);
    HIP_TRY(hipGetLastError());
    ctx->warm_d = -1;
    return CPA_OK;
}

cpa_status cpa_rpca_iterate(cpa_ctx* ctx, void* stream, int m, int n, const float* I_dev, float* state_dev, int iters,
                            double inv_rho, double eta_over_rho, const cpa_opts* opts, double* Et_dev) {
    cpa_status s;
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (m < 0 || n < 0) return fail(CPA_ERR_SHAPE, "negative size");
    if (iters < 0) return fail(CPA_ERR_ARG, "iters < 0");
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if ((s = no_learned_bound(opts)) != CPA_OK) return s;
    if (!(std::isfinite(inv_rho) && inv_rho >= 0.0 && std::isfinite(eta_over_rho) && eta_over_rho >= 0.0))
        return fail(CPA_ERR_ARG, "inv_rho and eta_over_rho must be finite and >= 0");
    if (m == 0 || n == 0 || iters == 0) return CPA_OK;
    if (!I_dev || !state_dev) return fail(CPA_ERR_ARG, "I or state is NULL");
    const int64_t mn = (int64_t)m * n;
    if (overlaps(I_dev, sizeof(float) * mn, state_dev, sizeof(float) * 7 * mn))
        return fail(CPA_ERR_ARG, "I overlaps the state");
    if (opts->check) return fail(CPA_ERR_UNSUPPORTED, "the growth check is not available inside the ADMM driver");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Work w;
    const int maxit = power_slots(opts);
    if ((s = ensure_ws(ctx, m, n, opts->K, maxit, true, w, right_side(opts, m, n), poly_choice(opts, m, n))) != CPA_OK)
        return s;
    AdmmPtrs P;
    P.l = state_dev;
    P.s = state_dev + mn;
    P.z1 = state_dev + 2 * mn;
    P.z2 = state_dev + 3 * mn;
    P.u1 = state_dev + 4 * mn;
    P.u2 = state_dev + 5 * mn;
    P.u3 = state_dev + 6 * mn;
    P.I = I_dev;
    P.x = w.x;
    cpa_shrinkage sh = {CPA_SOFT, 0, inv_rho, 0.0, 0.0, 1.0};
    const int grid = (int)std::min<int64_t>(kAdmmGrid, (mn + 255) / 256);
    (void)grid;
    auto one_iteration = [&](hipStream_t q) -> cpa_status {
        cpa_status r;
        // the ADMM pre-step, fused with the shrink's preparation (prep_kernel)
        PrepDone pd;
        int npart = 0;
        if ((r = enqueue_prep(ctx, q, m, n, w.x, n, w, opts, bound_mode(opts->bound), &P, w.admm, &npart, pd)) !=
            CPA_OK)
            return r;
        if ((r = shrink_impl(ctx, q, m, n, w.x, n, P.z1, n, &sh, opts, nullptr, w, &pd)) != CPA_OK) return r;
        // 16-byte accesses when every array is aligned (the state's blocks are mn floats apart)
        const int vec = (mn % 4 == 0) && ((reinterpret_cast<uintptr_t>(state_dev) & 15) == 0) &&
                        ((reinterpret_cast<uintptr_t>(I_dev) & 15) == 0);
        const int pgrid = (int)std::min<int64_t>(kAdmmGrid, ((vec ? mn / 4 : mn) + 255) / 256);
        hipLaunchKernelGGL(admm_post_kernel, dim3(std::max(pgrid, 1)), dim3(256), 0, q, P, mn, (float)eta_over_rho,
                           (const double*)w.admm, npart, Et_dev, w.et_counter, vec);
        HIP_TRY(hipGetLastError());
        return CPA_OK;
    };
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, st, w.et_counter, 1, 0);
    HIP_TRY(hipGetLastError());
    int t = 0;
    // A cold power-iteration start is run directly; the captured graph always
    // takes the warm start (or the seeded start when warm starts are off).
    const int d = w.d;
    if ((opts->bound == CPA_BOUND_POWER || opts->bound == CPA_BOUND_LANCZOS) && opts->warm_start &&
        ctx->warm_d != d) {
        if ((s = one_iteration(st)) != CPA_OK) return s;
        ++t;
    }
    if (t == iters) return CPA_OK;
    if (ctx->timing) {
        // per-launch event timing needs direct launches
        for (; t < iters; ++t)
            if ((s = one_iteration(st)) != CPA_OK) return s;
        return CPA_OK;
    }
    // key of the captured iteration: every pointer and scalar its launches bake in
    std::vector<char> key;
    auto put = [&](const void* p, size_t nb) {
        const char* c = static_cast<const char*>(p);
        key.insert(key.end(), c, c + nb);
    };
    put(&m, sizeof m); put(&n, sizeof n); put(&I_dev, sizeof I_dev); put(&state_dev, sizeof state_dev);
    put(&Et_dev, sizeof Et_dev); put(&ctx->ws, sizeof ctx->ws); put(&ctx->warm, sizeof ctx->warm);
    put(opts, sizeof *opts); put(&inv_rho, sizeof inv_rho); put(&eta_over_rho, sizeof eta_over_rho);
    // one graph of `reps` iterations in a row
    auto capture = [&](int reps, hipGraphExec_t* exec) -> cpa_status {
        if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipGraph_t g;
        HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        cpa_status cs = CPA_OK;
        for (int r = 0; r < reps && cs == CPA_OK; ++r) cs = one_iteration(ctx->cap_stream);
        const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
        if (cs != CPA_OK) {
            if (ce == hipSuccess) (void)hipGraphDestroy(g);
            return cs;
        }
        if (ce != hipSuccess) return fail(CPA_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ce));
        const hipError_t ie = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            *exec = nullptr;
            return fail(CPA_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
        }
        return CPA_OK;
    };
    if (!ctx->admm_exec || !ctx->admm_exec_chunk || key != ctx->admm_key) {
        for (hipGraphExec_t* e : {&ctx->admm_exec, &ctx->admm_exec_chunk})
            if (*e) {
                HIP_TRY(hipGraphExecDestroy(*e));
                *e = nullptr;
            }
        ctx->admm_key.clear();
        // both graphs now, so that a later call with many iterations does not
        // capture inside its caller's timing
        if ((s = capture(1, &ctx->admm_exec)) != CPA_OK) return s;
        if ((s = capture(kAdmmChunk, &ctx->admm_exec_chunk)) != CPA_OK) return s;
        ctx->admm_key = key;
    }
    for (; iters - t >= kAdmmChunk; t += kAdmmChunk) HIP_TRY(hipGraphLaunch(ctx->admm_exec_chunk, st));
    for (; t < iters; ++t) HIP_TRY(hipGraphLaunch(ctx->admm_exec, st));
    return CPA_OK;
}

}  // extern "C"

extern "C" {

cpa_status cpa_peak_mfma(cpa_ctx* ctx, void* stream, int kind, int iters, double* tflops_host,
                         double* clock_ghz_host) {
    if (!ctx || !tflops_host) return fail(CPA_ERR_ARG, "NULL argument");
    if (kind != 0 && kind != 1) return fail(CPA_ERR_ARG, "kind must be 0 (FP32) or 1 (BF16)");
    if (iters < 1 || iters > (1 << 20)) return fail(CPA_ERR_ARG, "iters must be in [1, 2^20]");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int grid = 4 * cus;   // four 4-wave workgroups per CU: four waves per SIMD
    int wall_khz = 0;
    if (clock_ghz_host) HIP_TRY(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, ctx->device));
    float* out = nullptr;
    // the two counter spans follow the per-thread outputs
    const size_t out_bytes = sizeof(float) * (size_t)grid * 256;
    if (hipMalloc(&out, out_bytes + 2 * sizeof(unsigned long long)) != hipSuccess)
        return fail(CPA_ERR_ALLOC, "allocation failed");
    unsigned long long* clk =
        clock_ghz_host ? reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(out) + out_bytes) : nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    cpa_status s = CPA_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) s = fail(CPA_ERR_HIP, "event creation failed");
    float ms = 0.f;
    for (int r = 0; s == CPA_OK && r < 2; ++r) {   // the first launch warms the clocks up
        if (hipEventRecord(e0, st) != hipSuccess) s = fail(CPA_ERR_HIP, "event record failed");
        if (kind == 0)
            hipLaunchKernelGGL(peak_mfma_kernel<0>, dim3(grid), dim3(256), 0, st, iters, out, clk);
        else
            hipLaunchKernelGGL(peak_mfma_kernel<1>, dim3(grid), dim3(256), 0, st, iters, out, clk);
        if (s == CPA_OK && hipGetLastError() != hipSuccess) s = fail(CPA_ERR_HIP, "launch failed");
        if (s == CPA_OK && hipEventRecord(e1, st) != hipSuccess) s = fail(CPA_ERR_HIP, "event record failed");
        if (s == CPA_OK && hipEventSynchronize(e1) != hipSuccess) s = fail(CPA_ERR_HIP, "event wait failed");
        if (s == CPA_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = fail(CPA_ERR_HIP, "event timing failed");
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    unsigned long long span[2] = {0, 0};
    if (s == CPA_OK && clk && hipMemcpy(span, clk, sizeof(span), hipMemcpyDeviceToHost) != hipSuccess)
        s = fail(CPA_ERR_HIP, "counter read failed");
    (void)hipFree(out);
    if (s != CPA_OK) return s;
    if (clock_ghz_host)
        *clock_ghz_host = (span[1] > 0 && wall_khz > 0) ? (double)span[0] / ((double)span[1] / (wall_khz * 1e3)) / 1e9
                                                        : 0.0;
    const double flop = (double)grid * 4 /* waves */ * iters * kPeakChains * (kind == 0 ? 2048.0 : 16384.0);
    *tflops_host = flop / (1e-3 * ms) / 1e12;
    return CPA_OK;
}

}  // extern "C"

namespace {

// 8 x 8 transform table: the orthonormal DCT-II, D[a][i] = s_a cos(pi (2i + 1) a / 16),
// s_0 = sqrt(1/8), s_a = 1/2; or the identity.
// Rows of the 8 x 8 transform block.  Haar: one level on the pairs (2q, 2q + 1)
// of the block, the four low-pass rows (sum / sqrt 2) first, then the four
// high-pass rows (difference / sqrt 2).  Over the whole vector this is the usual
// one-level Haar DWT with its outputs permuted; a permutation P of T's rows leaves
// T^T hat H(T G T^T) T unchanged (hat H(P A P^T) = P hat H(A) P^T, and the kept set
// is the same), so the block order gives the same result.
Dct8 transform_table(int transform) {
    Dct8 t;
    const double r2 = std::sqrt(0.5);
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 8; ++i) {
            if (transform == CPA_TRANSFORM_BLOCK_DCT8) {
                t.d[8 * a + i] = (a == 0 ? std::sqrt(1.0 / 8.0) : 0.5) * std::cos(M_PI * (2 * i + 1) * a / 16.0);
            } else if (transform == CPA_TRANSFORM_HAAR1 || transform == CPA_TRANSFORM_HAAR1_LOWPASS) {
                const int q = a & 3;
                const bool high = a >= 4;
                t.d[8 * a + i] = (i == 2 * q) ? r2 : (i == 2 * q + 1 ? (high ? -r2 : r2) : 0.0);
            } else {
                t.d[8 * a + i] = (a == i) ? 1.0 : 0.0;
            }
        }
    return t;
}

struct SpfWork {
    float* Phi;      // d x d: Phi, then the dense truncated matrix
    int32_t* cnt;    // d
    int32_t* rowptr; // d + 1
    int32_t* colidx; // d^2 (capacity)
    float* val;      // d^2
    float* P[2];     // Psi ping-pong, d x d
    float* H;        // d x d
    float* M;        // d x d
    unsigned* hist;  // kSelBins
    SelState* sel;
    int32_t* pos;    // d: compact index of a nonempty row, -1 for an empty one
    int32_t* rows;   // d: the nonempty rows
    int32_t* nrows;  // 2: the nonempty rows, the kept entries
    float* Dm;       // d x d, the full DCT (dense transform only, else null)
    float* Dt;       // its transpose
    double* warm;    // d: the compact block's power vector in full coordinates (warm start)
};

cpa_status ensure_spf(cpa_ctx* ctx, int d, bool dense_t, SpfWork& s) {
    const size_t dd = (size_t)d * d;
    size_t off = 0;
    const size_t oPhi = off; off = align_up(off + sizeof(float) * dd);
    const size_t oC = off; off = align_up(off + sizeof(int32_t) * d);
    const size_t oR = off; off = align_up(off + sizeof(int32_t) * (d + 1));
    const size_t oI = off; off = align_up(off + sizeof(int32_t) * dd);
    const size_t oV = off; off = align_up(off + sizeof(float) * dd);
    const size_t oP0 = off; off = align_up(off + sizeof(float) * dd);
    const size_t oP1 = off; off = align_up(off + sizeof(float) * dd);
    const size_t oH = off; off = align_up(off + sizeof(float) * dd);
    const size_t oM = off; off = align_up(off + sizeof(float) * dd);
    const size_t oHi = off; off = align_up(off + sizeof(unsigned) * kSelBins);
    const size_t oS = off; off = align_up(off + sizeof(SelState));
    const size_t oPos = off; off = align_up(off + sizeof(int32_t) * d);
    const size_t oRows = off; off = align_up(off + sizeof(int32_t) * d);
    const size_t oN = off; off = align_up(off + 2 * sizeof(int32_t));
    const size_t oW = off; off = align_up(off + sizeof(double) * d);
    size_t oDm = 0, oDt = 0;
    if (dense_t) {
        oDm = off; off = align_up(off + sizeof(float) * dd);
        oDt = off; off = align_up(off + sizeof(float) * dd);
    }
    // another side moves every buffer: the DCT matrices must be rebuilt and the warm
    // vector is gone
    if (d != ctx->spf_last_d) {
        ctx->spf_dct_d = 0;
        ctx->spf_warm_d = -1;
    }
    ctx->spf_last_d = d;
    if (off > ctx->spf_bytes) {
        ctx->spf_dct_d = 0;
        ctx->spf_warm_d = -1;
        if (ctx->spf) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ctx->spf));
            ctx->spf = nullptr;
            ctx->spf_bytes = 0;
        }
        if (hipMalloc(&ctx->spf, off) != hipSuccess) {
            ctx->spf = nullptr;
            return fail(CPA_ERR_ALLOC, "sparsified-path workspace allocation of %zu bytes failed", off);
        }
        ctx->spf_bytes = off;
    }
    char* b = static_cast<char*>(ctx->spf);
    s.Phi = reinterpret_cast<float*>(b + oPhi);
    s.cnt = reinterpret_cast<int32_t*>(b + oC);
    s.rowptr = reinterpret_cast<int32_t*>(b + oR);
    s.colidx = reinterpret_cast<int32_t*>(b + oI);
    s.val = reinterpret_cast<float*>(b + oV);
    s.P[0] = reinterpret_cast<float*>(b + oP0);
    s.P[1] = reinterpret_cast<float*>(b + oP1);
    s.H = reinterpret_cast<float*>(b + oH);
    s.M = reinterpret_cast<float*>(b + oM);
    s.hist = reinterpret_cast<unsigned*>(b + oHi);
    s.sel = reinterpret_cast<SelState*>(b + oS);
    s.pos = reinterpret_cast<int32_t*>(b + oPos);
    s.rows = reinterpret_cast<int32_t*>(b + oRows);
    s.nrows = reinterpret_cast<int32_t*>(b + oN);
    s.Dm = dense_t ? reinterpret_cast<float*>(b + oDm) : nullptr;
    s.Dt = dense_t ? reinterpret_cast<float*>(b + oDt) : nullptr;
    s.warm = reinterpret_cast<double*>(b + oW);
    return CPA_OK;
}

}  // namespace

extern "C" {

cpa_status cpa_shrink_dense_sparsified(cpa_ctx* ctx, void* stream, int m, int n, const float* X_dev, int64_t ldx,
                                       float* Y_dev, int64_t ldy, const cpa_shrinkage* shrink, const cpa_opts* opts,
                                       const cpa_sparsify* sp, cpa_info* info_host, double* eps_host,
                                       int64_t* nnz_host) {
    cpa_status s;
    if ((s = check_dense_args(ctx, m, n, X_dev, ldx)) != CPA_OK) return s;
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if ((s = no_learned_bound(opts)) != CPA_OK) return s;
    if ((s = check_shrinkage(shrink)) != CPA_OK) return s;
    if (!sp) return fail(CPA_ERR_ARG, "sparsify is NULL");
    if (sp->transform != CPA_TRANSFORM_IDENTITY && sp->transform != CPA_TRANSFORM_BLOCK_DCT8 &&
        sp->transform != CPA_TRANSFORM_HAAR1 && sp->transform != CPA_TRANSFORM_HAAR1_LOWPASS &&
        sp->transform != CPA_TRANSFORM_DCT)
        return fail(CPA_ERR_ARG, "unknown transform %d", sp->transform);
    if (sp->threshold != CPA_THRESHOLD_KEEP && sp->threshold != CPA_THRESHOLD_ABSOLUTE)
        return fail(CPA_ERR_ARG, "unknown threshold mode %d", sp->threshold);
    const bool abs_eps = sp->threshold == CPA_THRESHOLD_ABSOLUTE;
    if (abs_eps && !(std::isfinite(sp->eps) && sp->eps >= 0.0))
        return fail(CPA_ERR_ARG, "eps must be finite and >= 0");
    if (opts->check) return fail(CPA_ERR_UNSUPPORTED, "the growth check is not available on the sparsified path");
    if (opts->precision != CPA_PREC_FP32) return fail(CPA_ERR_UNSUPPORTED, "the sparsified path is FP32");
    if (m == 0 || n == 0) {
        if (info_host) std::memset(info_host, 0, sizeof(*info_host));
        if (eps_host) *eps_host = 0.0;
        if (nnz_host) *nnz_host = 0;
        return CPA_OK;
    }
    if (!Y_dev) return fail(CPA_ERR_ARG, "Y is NULL");
    if (ldy < n) return fail(CPA_ERR_SHAPE, "ldy < n");
    if (overlaps(X_dev, sizeof(float) * ((size_t)(m - 1) * ldx + n), Y_dev, sizeof(float) * ((size_t)(m - 1) * ldy + n)))
        return fail(CPA_ERR_ARG, "Y overlaps X");
    const bool right = right_side(opts, m, n);
    const int d = right ? n : m;
    if (d % 8 != 0) return fail(CPA_ERR_SHAPE, "the Gram side (%d) must be a multiple of 8 (8 x 8 tiles)", d);
    if (!abs_eps && (sp->keep < 1 || sp->keep > (int64_t)d * d)) return fail(CPA_ERR_ARG, "keep must be in [1, d^2]");
    if ((int64_t)d * d > INT32_MAX) return fail(CPA_ERR_SHAPE, "Gram too large for 32-bit indices");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Work w;
    const int maxit = power_slots(opts);
    // hat H by the matrix polynomial on the compact block, or by the sparse recurrence
    const bool poly = opts->K >= 2 && opts->K <= kPolyMaxK && opts->eval != CPA_EVAL_RECURRENCE;
    const int ps = poly ? poly_s_of(opts->K) : 0;
    if ((s = ensure_ws(ctx, m, n, opts->K, maxit, false, w, right, ps)) != CPA_OK) return s;
    SpfWork f;
    const bool dense_t = sp->transform == CPA_TRANSFORM_DCT;
    if ((s = ensure_spf(ctx, d, dense_t, f)) != CPA_OK) return s;
    const Dct8 D = transform_table(sp->transform);
    const int nt = d / 8;

    if ((s = fill_scalars(st, w)) != CPA_OK) return s;
    if ((s = enqueue_gram(ctx, st, m, n, X_dev, ldx, w)) != CPA_OK) return s;
    // Phi = T G T^T (exactly symmetric)
    const int gd = (int)std::min<int64_t>(4096, ((int64_t)d * d + 255) / 256);
    if (dense_t) {
        // full DCT: C = D G, Phi = C D^T (FP32 products), then (Phi + Phi^T)/2
        const EpiLin ec = lin_epi(f.P[0], d, nullptr, 0, 1.f, 0.f, 0.f, 0.f);
        const EpiLin ep = lin_epi(f.Phi, d, nullptr, 0, 1.f, 0.f, 0.f, 0.f);
        if (ctx->spf_dct_d != d) {
            hipLaunchKernelGGL(dct_fill_kernel, dim3(gd), dim3(256), 0, st, d, f.Dm, f.Dt);
            HIP_TRY(hipGetLastError());
            ctx->spf_dct_d = d;
        }
        if ((s = poly_gemm(ctx, st, make_op(f.Dt, d, d), make_op(w.G, d, d), d, d, d, ec, CPA_PREC_FP32, false)) !=
            CPA_OK)
            return s;
        if ((s = poly_gemm(ctx, st, make_op(f.P[0], d, d), make_op(f.Dm, d, d), d, d, d, ep, CPA_PREC_FP32, true)) !=
            CPA_OK)
            return s;
        hipLaunchKernelGGL(symmetrize_kernel, dim3(gd), dim3(256), 0, st, d, f.Phi, (int64_t)d);
        HIP_TRY(hipGetLastError());
    } else {
        const int zh = sp->transform == CPA_TRANSFORM_HAAR1_LOWPASS ? 1 : 0;
        if (d % 64 == 0)   // 64 x 64 blocks, rows written whole
            hipLaunchKernelGGL(bt_forward_blk_kernel, dim3((d / 64) * (d / 64 + 1) / 2), dim3(256), 0, st, d,
                               (const float*)w.G, (int64_t)d, f.Phi, (int64_t)d, D, zh);
        else
            hipLaunchKernelGGL(bt_forward_kernel, dim3((nt * (nt + 1) / 2 + 3) / 4), dim3(256), 0, st, d,
                               (const float*)w.G, (int64_t)d, f.Phi, (int64_t)d, D, zh);
        HIP_TRY(hipGetLastError());
    }
    // M = T^T hat H T from the compact hat H (pitch ldh; hat h(0) on the empty diagonal)
    auto inverse = [&](const float* Hc, int64_t ldh) -> cpa_status {
        if (!dense_t) {
            if (d % 64 == 0)
                hipLaunchKernelGGL(bt_inverse_blk_kernel, dim3((d / 64) * (d / 64)), dim3(256), 0, st, d, Hc, ldh, f.M,
                                   (int64_t)d, D, (const int32_t*)f.pos, (const double*)w.scal, opts->K);
            else
                hipLaunchKernelGGL(bt_inverse_kernel, dim3((nt * nt + 3) / 4), dim3(256), 0, st, d, Hc, ldh, f.M,
                                   (int64_t)d, D, (const int32_t*)f.pos, (const double*)w.scal, opts->K);
            HIP_TRY(hipGetLastError());
            return CPA_OK;
        }
        // expand to the full hat H (identity table), then C = hat H D, M = D^T C
        hipLaunchKernelGGL(d % 64 == 0 ? bt_inverse_blk_kernel : bt_inverse_kernel,
                           dim3(d % 64 == 0 ? (d / 64) * (d / 64) : (nt * nt + 3) / 4), dim3(256), 0, st, d, Hc, ldh,
                           f.P[0], (int64_t)d,
                           transform_table(CPA_TRANSFORM_IDENTITY), (const int32_t*)f.pos, (const double*)w.scal,
                           opts->K);
        HIP_TRY(hipGetLastError());
        const EpiLin ec = lin_epi(f.P[1], d, nullptr, 0, 1.f, 0.f, 0.f, 0.f);
        const EpiLin em = lin_epi(f.M, d, nullptr, 0, 1.f, 0.f, 0.f, 0.f);
        cpa_status r;
        if ((r = poly_gemm(ctx, st, make_op(f.P[0], d, d), make_op(f.Dt, d, d), d, d, d, ec, CPA_PREC_FP32, true)) !=
            CPA_OK)
            return r;
        return poly_gemm(ctx, st, make_op(f.Dm, d, d), make_op(f.P[1], d, d), d, d, d, em, CPA_PREC_FP32, false);
    };
    if (abs_eps) {
        // the given eps, as the key of its FP32 value
        hipLaunchKernelGGL(sel_fixed_kernel, dim3(1), dim3(64), 0, st, f.sel, (float)sp->eps);
        HIP_TRY(hipGetLastError());
    } else {
        // eps = the keep-th largest |Phi|
        hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, st, f.sel, (uint32_t)sp->keep, f.hist);
        HIP_TRY(hipGetLastError());
        const int gh = std::max(1, std::min(1024, (d + 1) / 2));   // pairs of rows (upper triangle)
        for (int pass = 0; pass < 3; ++pass) {
            hipLaunchKernelGGL(sel_hist_kernel, dim3(gh), dim3(256), 0, st, d, (const float*)f.Phi, (int64_t)d,
                               pass, (const SelState*)f.sel, f.hist);
            HIP_TRY(hipGetLastError());
            hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(256), 0, st, pass, f.sel, f.hist);
            HIP_TRY(hipGetLastError());
        }
    }
    // the truncated matrix: kept entries per row; the recurrence route also builds
    // its CSR and the dense truncated matrix in place (the polynomial route gathers
    // the compact block with the threshold applied)
    const int gr = (d + 3) / 4;
    hipLaunchKernelGGL(trunc_count_kernel, dim3(gr), dim3(256), 0, st, d, (const float*)f.Phi, (int64_t)d,
                       (const SelState*)f.sel, f.cnt);
    HIP_TRY(hipGetLastError());
    if (!poly) {
        hipLaunchKernelGGL(csc_scan_kernel, dim3(1), dim3(SP_THREADS), 0, st, d, (const int32_t*)f.cnt, f.rowptr);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(trunc_fill_kernel, dim3(gr), dim3(256), 0, st, d, f.Phi, (int64_t)d,
                           (const SelState*)f.sel, (const int32_t*)f.rowptr, f.colidx, f.val);
        HIP_TRY(hipGetLastError());
    }
    // hat H is computed on the nonempty rows and columns only
    hipLaunchKernelGGL(compact_rows_kernel, dim3(1), dim3(256), 0, st, d, (const int32_t*)f.cnt, f.pos, f.rows,
                       f.nrows);
    HIP_TRY(hipGetLastError());
    const EpiLin ey = lin_epi(Y_dev, ldy, nullptr, 0, 1.f, 0.f, 0.f, 0.f);
    Work wi = w;   // the layout read_info uses
    // the requested host results: info, the threshold and the kept count
    auto report = [&](const Work& wr) -> cpa_status {
        cpa_status r;
        if (info_host) {
            if ((r = read_info(st, wr, opts->K, m, n, info_host, nullptr)) != CPA_OK) return r;
        }
        if (eps_host || nnz_host) {
            SelState hs;
            int32_t nnz = 0;
            HIP_TRY(hipMemcpyAsync(&hs, f.sel, sizeof(hs), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(&nnz, f.nrows + 1, sizeof(nnz), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (eps_host) {
                float e;
                std::memcpy(&e, &hs.prefix, sizeof(e));
                *eps_host = (double)e;
            }
            if (nnz_host) *nnz_host = nnz;
        }
        return CPA_OK;
    };
    // the block's size: it sets every launch of the polynomial route, and with a
    // given eps it may be zero -- one wait for the stream in either case
    int32_t ns = -1;
    if (poly || abs_eps) {
        // into pinned memory: a direct copy, not the staged one of pageable memory
        if (!ctx->spf_host) HIP_TRY(hipHostMalloc((void**)&ctx->spf_host, sizeof(int32_t), hipHostMallocDefault));
        HIP_TRY(hipMemcpyAsync(ctx->spf_host, f.nrows, sizeof(ns), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        ns = *ctx->spf_host;
        if (ns < 0 || ns > d || (ns == 0 && !abs_eps))
            return fail(CPA_ERR_HIP, "compact block size %d read back out of range", ns);
        if (ns == 0) {
            // nothing kept (a given eps above every |Phi_ij|): the truncated matrix is
            // zero, so is its largest eigenvalue, and the shrink is zero on either
            // route (h(0) = 0 for every shrink function; the bound stays 0)
            HIP_TRY(hipMemset2DAsync(Y_dev, sizeof(float) * (size_t)ldy, 0, sizeof(float) * (size_t)n, m, st));
            return report(w);
        }
    }
    if (poly) {
        // zero rows and columns appended to the block are empty ones too (eigenvalue 0,
        // never read back): a multiple of 64 gives full tiles to every product
        int nb = (ns + 63) / 64 * 64;
        if (nb > d) nb = (ns + 3) / 4 * 4;   // d % 8 == 0, so this fits
        const int gg = (int)std::min<int64_t>(4096, ((int64_t)nb * nb + 255) / 256);
        hipLaunchKernelGGL(gather_compact_kernel, dim3(gg), dim3(256), 0, st, ns, nb, (const int32_t*)f.rows,
                           (const float*)f.Phi, (int64_t)d, (const SelState*)f.sel, w.G);
        HIP_TRY(hipGetLastError());
        // bound, coefficients and p(Phi_S) on the nb x nb block (pitch nb, in the Gram's buffer);
        // the Gram partials keep their place (they depend on K and maxit only)
        Work wc = w;
        wc.d = nb;
        wc.lay.pwg = power_grid(ctx, nb);
        // warm start: the previous call's vector, mapped from full coordinates onto this
        // call's block
        const bool warm_map =
            opts->warm_start && (opts->bound == CPA_BOUND_POWER || opts->bound == CPA_BOUND_LANCZOS);
        if (warm_map) {
            if (ctx->spf_warm_d == d) {
                hipLaunchKernelGGL(warm_gather_kernel, dim3((nb + 255) / 256), dim3(256), 0, st, ns, nb,
                                   (const int32_t*)f.rows, (const double*)f.warm, ctx->warm);
                HIP_TRY(hipGetLastError());
                ctx->warm_d = nb;
            } else {
                ctx->warm_d = -1;
            }
        }
        if ((s = enqueue_bound(ctx, st, nb, shrink, opts, wc, -1)) != CPA_OK) return s;
        if (warm_map) {
            hipLaunchKernelGGL(warm_scatter_kernel, dim3((d + 255) / 256), dim3(256), 0, st, d,
                               (const int32_t*)f.pos, (const double*)ctx->warm, f.warm);
            HIP_TRY(hipGetLastError());
            ctx->spf_warm_d = d;
        }
        float* F = nullptr;
        if ((s = enqueue_poly_core(ctx, st, nb, w.G, nb, w.scal, wc.lay.ps(), w.poly, ps, opts->K, CPA_PREC_FP32,
                                   &F, poly_fused(wc, opts->K), -1, poly_fused(wc, opts->K))) != CPA_OK)
            return s;
        // M = T^T hat H T (hat h(0) on the empty diagonal), then Y = X M (right) or M X (left)
        if ((s = inverse(F, nb)) != CPA_OK) return s;
        if (right)
            s = poly_gemm(ctx, st, make_op(X_dev, ldx, m), make_op(f.M, d, n), m, n, n, ey, CPA_PREC_FP32, true);
        else
            s = poly_gemm(ctx, st, make_op(f.M, d, m), make_op(X_dev, ldx, n), m, n, m, ey, CPA_PREC_FP32, false);
        if (s != CPA_OK) return s;
        wi = wc;
    } else {
        hipLaunchKernelGGL(remap_cols_kernel, dim3(1024), dim3(256), 0, st, d, (const int32_t*)f.rowptr, f.colidx,
                           (const int32_t*)f.pos);
        HIP_TRY(hipGetLastError());

        // bound and coefficients from the (dense) truncated matrix
        Work wb = w;
        wb.G = f.Phi;
        if ((s = enqueue_bound(ctx, st, d, shrink, opts, wb, -1)) != CPA_OK) return s;
        if (opts->K == 1) {
            // hat H = c_0/2 I, and T^T (c_0/2 I) T = c_0/2 I: Y = c_0/2 X
            if ((s = enqueue_recurrence(ctx, st, m, n, X_dev, ldx, Y_dev, ldy, 1, w, false, CPA_PREC_FP32)) != CPA_OK)
                return s;
        } else {
            // compact hat H: Psi_0 = I, Psi_{k+1} = 2 ((2/Lambda) Phi_ Psi_k - Psi_k) - Psi_{k-1}, H = sum c_k Psi_k
            const int ge = (int)std::min<int64_t>(4096, ((int64_t)d * d + 255) / 256);
            hipLaunchKernelGGL(eye_compact_kernel, dim3(ge), dim3(256), 0, st, (const int32_t*)f.nrows, f.P[0],
                               (int64_t)d);
            HIP_TRY(hipGetLastError());
            // row-and-panel items loop over a grid of at most 2048 workgroups
            const int grid_c = (int)std::min<int64_t>(2048, (int64_t)d * ((d + kPsiJ - 1) / kPsiJ));
            int cur = 0;
            for (int k = 0; k + 1 <= opts->K - 1; ++k) {
                const float* yk = f.P[cur];
                float* yo = f.P[cur ^ 1];   // Psi_{k-1} (unused at k = 0), overwritten by Psi_{k+1}
                hipLaunchKernelGGL(psi_step_kernel, dim3(grid_c), dim3(256), 0, st, d, (const int32_t*)f.rows,
                                   (const int32_t*)f.nrows, (const int32_t*)f.rowptr,
                                   (const int32_t*)f.colidx, (const float*)f.val, yk, (const float*)yo, yo, (int64_t)d,
                                   f.H, (const double*)w.scal, k, (k + 1 == opts->K - 1) ? 1 : 0);
                HIP_TRY(hipGetLastError());
                cur ^= 1;
            }
            // M = T^T hat H T, then Y = X M (right) or M X (left)
            if ((s = inverse(f.H, d)) != CPA_OK) return s;
            if (right)
                s = poly_gemm(ctx, st, make_op(X_dev, ldx, m), make_op(f.M, d, n), m, n, n, ey, CPA_PREC_FP32, true);
            else
                s = poly_gemm(ctx, st, make_op(f.M, d, m), make_op(X_dev, ldx, n), m, n, m, ey, CPA_PREC_FP32, false);
            if (s != CPA_OK) return s;
        }
    }
    return report(wi);
}

}  // extern "C"

// ---- Texture inpainting (Appendix A) ----

namespace {

struct InpWork {
    float* Dm;    // m x m DCT-II matrix
    float* Dtm;   // its transpose
    float* Dn;    // n x n
    float* Dtn;
    float* A;     // m x n product scratch
    float* B;     // m x n product scratch
    float* T;     // m x n: Psi^T (z2 - u2), then Psi l
    float* x;     // m x n shrink input
    double* part; // 3 per elementwise workgroup
    double* cst;  // mean over the surrounding pixels, region size
    int* counter; // next E_t slot
};

cpa_status ensure_inp(cpa_ctx* ctx, int m, int n, InpWork& s) {
    const size_t mm = (size_t)m * m, nn = (size_t)n * n, mn = (size_t)m * n;
    size_t off = 0;
    const size_t oDm = off; off = align_up(off + sizeof(float) * mm);
    const size_t oDtm = off; off = align_up(off + sizeof(float) * mm);
    const size_t oDn = off; off = align_up(off + sizeof(float) * nn);
    const size_t oDtn = off; off = align_up(off + sizeof(float) * nn);
    const size_t oA = off; off = align_up(off + sizeof(float) * mn);
    const size_t oB = off; off = align_up(off + sizeof(float) * mn);
    const size_t oT = off; off = align_up(off + sizeof(float) * mn);
    const size_t oX = off; off = align_up(off + sizeof(float) * mn);
    const size_t oP = off; off = align_up(off + sizeof(double) * 3 * kInpGrid);
    const size_t oC = off; off = align_up(off + sizeof(double) * 4);
    const size_t oK = off; off = align_up(off + sizeof(int));
    if (off > ctx->inp_bytes) {
        if (ctx->inp) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ctx->inp));
            ctx->inp = nullptr;
            ctx->inp_bytes = 0;
        }
        if (hipMalloc(&ctx->inp, off) != hipSuccess) {
            ctx->inp = nullptr;
            return fail(CPA_ERR_ALLOC, "inpainting workspace allocation of %zu bytes failed", off);
        }
        ctx->inp_bytes = off;
    }
    char* b = static_cast<char*>(ctx->inp);
    s.Dm = reinterpret_cast<float*>(b + oDm);
    s.Dtm = reinterpret_cast<float*>(b + oDtm);
    s.Dn = reinterpret_cast<float*>(b + oDn);
    s.Dtn = reinterpret_cast<float*>(b + oDtn);
    s.A = reinterpret_cast<float*>(b + oA);
    s.B = reinterpret_cast<float*>(b + oB);
    s.T = reinterpret_cast<float*>(b + oT);
    s.x = reinterpret_cast<float*>(b + oX);
    s.part = reinterpret_cast<double*>(b + oP);
    s.cst = reinterpret_cast<double*>(b + oC);
    s.counter = reinterpret_cast<int*>(b + oK);
    return CPA_OK;
}

// The DCT matrices of both sides (D and D^T for m and for n).
cpa_status inp_dct(hipStream_t st, int m, int n, const InpWork& f) {
    const int gm = (int)std::min<int64_t>(4096, ((int64_t)m * m + 255) / 256);
    const int gn = (int)std::min<int64_t>(4096, ((int64_t)n * n + 255) / 256);
    hipLaunchKernelGGL(dct_fill_kernel, dim3(gm), dim3(256), 0, st, m, f.Dm, f.Dtm);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(dct_fill_kernel, dim3(gn), dim3(256), 0, st, n, f.Dn, f.Dtn);
    HIP_TRY(hipGetLastError());
    return CPA_OK;
}

// out = Psi src = D_m src D_n^T (forward) or Psi^T src = D_m^T src D_n, via f.B.
cpa_status inp_psi(cpa_ctx* ctx, hipStream_t st, int m, int n, const float* src, float* out, bool forward,
                   const InpWork& f) {
    const EpiLin eb = lin_epi(f.B, n, nullptr, 0, 1.f, 0.f, 0.f, 0.f);
    const EpiLin eo = lin_epi(out, n, nullptr, 0, 1.f, 0.f, 0.f, 0.f);
    cpa_status s;
    // B = D_m src (forward: A stored D_m^T, read transposed) or D_m^T src (A stored D_m)
    if ((s = poly_gemm(ctx, st, make_op(forward ? f.Dtm : f.Dm, m, m), make_op(src, n, n), m, n, m, eb,
                       CPA_PREC_FP32, false)) != CPA_OK)
        return s;
    // out = B D_n^T (B operand stored D_n) or B D_n (stored D_n^T)
    return poly_gemm(ctx, st, make_op(f.B, n, m), make_op(forward ? f.Dn : f.Dtn, n, n), m, n, n, eo,
                     CPA_PREC_FP32, true);
}

// eq. (recommendation_epsilon) with Table IV's counts: k = d^2 / 20000 (0.5e-4 d^2)
// while E_t > E_l, 3 d^2 / 20000 (1.5e-4 d^2) while E_t > E_m, d^2 / 2000 (0.5e-3 d^2)
// after that; a fractional count is rounded up, exactly, and the result lies in [1, d^2].
int64_t schedule_keep(double E_t, int d, double E_l, double E_m) {
    const unsigned __int128 dd = (unsigned __int128)d * (unsigned __int128)d;
    unsigned __int128 num, den;
    if (E_t > E_l) {
        num = dd;
        den = 20000;
    } else if (E_t > E_m) {
        num = 3 * dd;
        den = 20000;
    } else {
        num = dd;
        den = 2000;
    }
    unsigned __int128 k = (num + den - 1) / den;
    if (k < 1) k = 1;
    if (k > dd) k = dd;
    return (int64_t)k;
}

// The adaptive sparsified shrink of the inpainting driver: transform, the E_t
// before the first iteration, the switch points, and where the keeps go.
struct InpSchedule {
    int32_t transform;
    double E_prev, E_l, E_m;
    int64_t* keep_host;
};

cpa_status inpaint_run(cpa_ctx* ctx, void* stream, int m, int n, const float* I_dev, const float* omega_dev,
                       const float* border_dev, float* state_dev, int iters, double inv_rho, double eta_over_rho,
                       const cpa_opts* opts, double* Et_dev, const InpSchedule* sched) {
    cpa_status s;
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (m < 0 || n < 0) return fail(CPA_ERR_SHAPE, "negative size");
    if (iters < 0) return fail(CPA_ERR_ARG, "iters < 0");
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if ((s = no_learned_bound(opts)) != CPA_OK) return s;
    if (!(std::isfinite(inv_rho) && inv_rho >= 0.0 && std::isfinite(eta_over_rho) && eta_over_rho >= 0.0))
        return fail(CPA_ERR_ARG, "inv_rho and eta_over_rho must be finite and >= 0");
    if (m == 0 || n == 0 || iters == 0) return CPA_OK;
    if (!I_dev || !omega_dev || !state_dev) return fail(CPA_ERR_ARG, "I, omega or state is NULL");
    if (opts->check) return fail(CPA_ERR_UNSUPPORTED, "the growth check is not available inside the ADMM driver");
    const int64_t mn = (int64_t)m * n;
    const size_t sb = sizeof(float) * 11 * mn, ib = sizeof(float) * mn;
    if (overlaps(I_dev, ib, state_dev, sb) || overlaps(omega_dev, ib, state_dev, sb) ||
        (border_dev && overlaps(border_dev, ib, state_dev, sb)))
        return fail(CPA_ERR_ARG, "an input overlaps the state");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Work w;
    const int maxit = power_slots(opts);
    const int d = right_side(opts, m, n) ? n : m;
    if (sched) {
        // the sparsified shrink's own checks, before anything is launched
        if (d % 8 != 0) return fail(CPA_ERR_SHAPE, "the Gram side (%d) must be a multiple of 8 (8 x 8 tiles)", d);
        if ((int64_t)d * d > INT32_MAX) return fail(CPA_ERR_SHAPE, "Gram too large for 32-bit indices");
        if (opts->precision != CPA_PREC_FP32) return fail(CPA_ERR_UNSUPPORTED, "the sparsified path is FP32");
    } else if ((s = ensure_ws(ctx, m, n, opts->K, maxit, false, w, right_side(opts, m, n), poly_choice(opts, m, n))) !=
               CPA_OK) {
        return s;
    }
    InpWork f;
    if ((s = ensure_inp(ctx, m, n, f)) != CPA_OK) return s;
    if ((s = inp_dct(st, m, n, f)) != CPA_OK) return s;
    const int grid = (int)std::min<int64_t>(kInpGrid, (mn + 255) / 256);
    hipLaunchKernelGGL(inp_const_kernel, dim3(grid), dim3(256), 0, st, mn, I_dev, omega_dev, border_dev, f.part);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(inp_const_finish_kernel, dim3(1), dim3(256), 0, st, (const double*)f.part, grid,
                       border_dev ? 1 : 0, f.cst);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, st, f.counter, 1, 0);
    HIP_TRY(hipGetLastError());
    InpPtrs P;
    P.l = state_dev;
    for (int k = 0; k < 5; ++k) {
        P.z[k] = state_dev + (1 + k) * mn;
        P.u[k] = state_dev + (6 + k) * mn;
    }
    P.I = I_dev;
    P.om = omega_dev;
    P.x = f.x;
    P.T = f.T;
    P.ave = border_dev ? 1 : 0;
    cpa_shrinkage sh = {CPA_SOFT, 0, inv_rho, 0.0, 0.0, 1.0};
    double e_prev = sched ? sched->E_prev : 0.0;
    for (int t = 0; t < iters; ++t) {
        // T = Psi^T (z2 - u2)
        hipLaunchKernelGGL(inp_diff_kernel, dim3(grid), dim3(256), 0, st, mn, (const float*)P.z[1],
                           (const float*)P.u[1], f.A);
        HIP_TRY(hipGetLastError());
        if ((s = inp_psi(ctx, st, m, n, f.A, f.T, false, f)) != CPA_OK) return s;
        hipLaunchKernelGGL(inp_pre_kernel, dim3(grid), dim3(256), 0, st, P, mn, f.part);
        HIP_TRY(hipGetLastError());
        // z1 = the CPA shrink of x = l + u1 (sparsified: keep from the previous E_t)
        if (sched) {
            const cpa_sparsify sp = {sched->transform, CPA_THRESHOLD_KEEP, schedule_keep(e_prev, d, sched->E_l, sched->E_m),
                                     0.0};
            if (sched->keep_host) sched->keep_host[t] = sp.keep;
            if ((s = cpa_shrink_dense_sparsified(ctx, stream, m, n, f.x, n, P.z[0], n, &sh, opts, &sp, nullptr,
                                                 nullptr, nullptr)) != CPA_OK)
                return s;
        } else if ((s = shrink_impl(ctx, st, m, n, f.x, n, P.z[0], n, &sh, opts, nullptr, w)) != CPA_OK) {
            return s;
        }
        // T = Psi l
        if ((s = inp_psi(ctx, st, m, n, P.l, f.T, true, f)) != CPA_OK) return s;
        hipLaunchKernelGGL(inp_post_kernel, dim3(grid), dim3(256), 0, st, P, mn, (float)eta_over_rho,
                           (const double*)f.part, grid, (const double*)f.cst, Et_dev, f.counter);
        HIP_TRY(hipGetLastError());
        if (sched) {
            HIP_TRY(hipMemcpyAsync(&e_prev, Et_dev + t, sizeof(double), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
    }
    return CPA_OK;
}


}  // namespace

extern "C" {

int64_t cpa_inpaint_state_floats(int m, int n) {
    if (m <= 0 || n <= 0) return 0;
    return 11 * (int64_t)m * n;
}

cpa_status cpa_inpaint_init(cpa_ctx* ctx, void* stream, int m, int n, const float* omega_dev, float* state_dev) {
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (m < 0 || n < 0) return fail(CPA_ERR_SHAPE, "negative size");
    if (m == 0 || n == 0) return CPA_OK;
    if (!omega_dev || !state_dev) return fail(CPA_ERR_ARG, "omega or state is NULL");
    const int64_t mn = (int64_t)m * n;
    if (overlaps(omega_dev, sizeof(float) * mn, state_dev, sizeof(float) * 11 * mn))
        return fail(CPA_ERR_ARG, "omega overlaps the state");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    InpWork f;
    cpa_status s;
    if ((s = ensure_inp(ctx, m, n, f)) != CPA_OK) return s;
    const int grid = (int)std::min<int64_t>(kInpGrid, (mn + 255) / 256);
    hipLaunchKernelGGL(inp_init_kernel, dim3(grid), dim3(256), 0, st, mn, omega_dev, state_dev);
    HIP_TRY(hipGetLastError());
    // z2 = Psi 1 (the init kernel left ones in z2; the product reads them from there)
    if ((s = inp_dct(st, m, n, f)) != CPA_OK) return s;
    return inp_psi(ctx, st, m, n, state_dev + 2 * mn, state_dev + 2 * mn, true, f);
}

cpa_status cpa_inpaint_iterate(cpa_ctx* ctx, void* stream, int m, int n, const float* I_dev, const float* omega_dev,
                               const float* border_dev, float* state_dev, int iters, double inv_rho,
                               double eta_over_rho, const cpa_opts* opts, double* Et_dev) {
    return inpaint_run(ctx, stream, m, n, I_dev, omega_dev, border_dev, state_dev, iters, inv_rho, eta_over_rho, opts,
                       Et_dev, nullptr);
}

cpa_status cpa_keep_schedule(double E_t, int d, double E_l, double E_m, int64_t* keep) {
    if (!keep) return fail(CPA_ERR_ARG, "keep is NULL");
    if (std::isnan(E_t)) return fail(CPA_ERR_ARG, "E_t is NaN");
    if (d <= 0) return fail(CPA_ERR_SHAPE, "d must be positive");
    if (!(std::isfinite(E_l) && std::isfinite(E_m) && E_m >= 0.0 && E_l >= E_m))
        return fail(CPA_ERR_ARG, "the switch points must satisfy 0 <= E_m <= E_l (finite)");
    *keep = schedule_keep(E_t, d, E_l, E_m);
    return CPA_OK;
}

cpa_status cpa_inpaint_iterate_scheduled(cpa_ctx* ctx, void* stream, int m, int n, const float* I_dev,
                                         const float* omega_dev, const float* border_dev, float* state_dev, int iters,
                                         double inv_rho, double eta_over_rho, const cpa_opts* opts, int32_t transform,
                                         double E_prev, double E_l, double E_m, double* Et_dev, int64_t* keep_host) {
    if (transform != CPA_TRANSFORM_IDENTITY && transform != CPA_TRANSFORM_BLOCK_DCT8 &&
        transform != CPA_TRANSFORM_HAAR1 && transform != CPA_TRANSFORM_HAAR1_LOWPASS && transform != CPA_TRANSFORM_DCT)
        return fail(CPA_ERR_ARG, "unknown transform %d", transform);
    if (std::isnan(E_prev)) return fail(CPA_ERR_ARG, "E_prev is NaN");
    if (!(std::isfinite(E_l) && std::isfinite(E_m) && E_m >= 0.0 && E_l >= E_m))
        return fail(CPA_ERR_ARG, "the switch points must satisfy 0 <= E_m <= E_l (finite)");
    if (!Et_dev && iters > 0 && m > 0 && n > 0) return fail(CPA_ERR_ARG, "Et is required (the schedule reads E_t)");
    InpSchedule sc{transform, E_prev, E_l, E_m, keep_host};
    return inpaint_run(ctx, stream, m, n, I_dev, omega_dev, border_dev, state_dev, iters, inv_rho, eta_over_rho, opts,
                       Et_dev, &sc);
}

}  // extern "C"

// ---- FP64 dense shrinkage ----

namespace {

struct F64Work {
    double* G;      // d x d
    double* Yb[2];  // m x n: Y_k ping-pong (Y_0 = a copy of X)
    double* Z;      // m x n product
};

cpa_status ensure_f64(cpa_ctx* ctx, int d, int m, int n, F64Work& f) {
    const size_t dd = (size_t)d * d, mn = (size_t)m * n;
    size_t off = 0;
    const size_t oG = off; off = align_up(off + sizeof(double) * dd);
    const size_t oY0 = off; off = align_up(off + sizeof(double) * mn);
    const size_t oY1 = off; off = align_up(off + sizeof(double) * mn);
    const size_t oZ = off; off = align_up(off + sizeof(double) * mn);
    if (off > ctx->f64_bytes) {
        if (ctx->f64) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ctx->f64));
            ctx->f64 = nullptr;
            ctx->f64_bytes = 0;
        }
        if (hipMalloc(&ctx->f64, off) != hipSuccess) {
            ctx->f64 = nullptr;
            return fail(CPA_ERR_ALLOC, "FP64 workspace allocation of %zu bytes failed", off);
        }
        ctx->f64_bytes = off;
    }
    char* b = static_cast<char*>(ctx->f64);
    f.G = reinterpret_cast<double*>(b + oG);
    f.Yb[0] = reinterpret_cast<double*>(b + oY0);
    f.Yb[1] = reinterpret_cast<double*>(b + oY1);
    f.Z = reinterpret_cast<double*>(b + oZ);
    return CPA_OK;
}

template <bool TA, bool TB>
cpa_status gemm64(hipStream_t st, int M, int N, int Kd, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double* C, int64_t ldc) {
    const dim3 grid((N + F64_BN - 1) / F64_BN, (M + F64_BM - 1) / F64_BM);
    hipLaunchKernelGGL((gemm_f64_kernel<TA, TB>), grid, dim3(F64_THREADS), 0, st, M, N, Kd, A, lda, B, ldb, C, ldc);
    HIP_TRY(hipGetLastError());
    return CPA_OK;
}

}  // namespace

extern "C" {

cpa_status cpa_shrink_dense_f64(cpa_ctx* ctx, void* stream, int m, int n, const double* X_dev, int64_t ldx,
                                double* Y_dev, int64_t ldy, const cpa_shrinkage* shrink, const cpa_opts* opts_in,
                                cpa_info* info_host) {
    cpa_status s;
    if ((s = check_dense_args(ctx, m, n, reinterpret_cast<const float*>(X_dev), ldx)) != CPA_OK) return s;
    if ((s = check_shrinkage(shrink)) != CPA_OK) return s;
    if (!opts_in) return fail(CPA_ERR_ARG, "opts is NULL");
    cpa_opts o = *opts_in;
    if (o.precision == CPA_PREC_FP64) o.precision = CPA_PREC_FP32;   // the arithmetic here is FP64 in any case
    if ((s = check_opts(&o)) != CPA_OK) return s;
    if ((s = no_learned_bound(&o)) != CPA_OK) return s;
    if (o.precision != CPA_PREC_FP32) return fail(CPA_ERR_UNSUPPORTED, "the FP64 path has no split precision");
    if (o.check) return fail(CPA_ERR_UNSUPPORTED, "the growth check is not available on the FP64 path");
    if (o.eval == CPA_EVAL_POLYNOMIAL) return fail(CPA_ERR_UNSUPPORTED, "the FP64 path evaluates by the recurrence");
    if (m == 0 || n == 0) {
        if (info_host) std::memset(info_host, 0, sizeof(*info_host));
        return CPA_OK;
    }
    if (!Y_dev) return fail(CPA_ERR_ARG, "Y is NULL");
    if (ldy < n) return fail(CPA_ERR_SHAPE, "ldy < n");
    if (overlaps(X_dev, sizeof(double) * ((size_t)(m - 1) * ldx + n), Y_dev, sizeof(double) * ((size_t)(m - 1) * ldy + n)))
        return fail(CPA_ERR_ARG, "Y overlaps X");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool right = right_side(&o, m, n);
    const int d = right ? n : m;
    Work w;
    const int maxit = power_slots(&o);
    if ((s = ensure_ws(ctx, m, n, o.K, maxit, false, w, right, 0)) != CPA_OK) return s;
    F64Work f;
    if ((s = ensure_f64(ctx, d, m, n, f)) != CPA_OK) return s;
    if ((s = fill_scalars(st, w)) != CPA_OK) return s;
    // Gram X^T X (n x n) or X X^T (m x m), FP64
    if (right)
        s = gemm64<true, false>(st, n, n, m, X_dev, ldx, X_dev, ldx, f.G, n);
    else
        s = gemm64<false, true>(st, m, m, n, X_dev, ldx, X_dev, ldx, f.G, m);
    if (s != CPA_OK) return s;
    hipLaunchKernelGGL(gram64_stats_kernel, dim3(w.lay.gwg), dim3(256), 0, st, d, (const double*)f.G,
                       w.scal + w.lay.gpart());
    HIP_TRY(hipGetLastError());
    // the Lanczos vectors (if that rule is asked for) in the product buffer Z, idle until the recurrence
    if ((s = enqueue_bound(ctx, st, d, shrink, &o, w, -1, f.G, 0.0, false, f.Z, (size_t)m * n)) != CPA_OK) return s;
    const int64_t mn = (int64_t)m * n;
    const int ge = (int)std::min<int64_t>(4096, (mn + 255) / 256);
    if (o.K == 1) {
        hipLaunchKernelGGL(scale64_kernel, dim3(ge), dim3(256), 0, st, m, n, X_dev, ldx, Y_dev, ldy,
                           (const double*)w.scal);
        HIP_TRY(hipGetLastError());
    } else {
        hipLaunchKernelGGL(copy64_kernel, dim3(ge), dim3(256), 0, st, m, n, X_dev, ldx, f.Yb[0]);
        HIP_TRY(hipGetLastError());
        int cur = 0;
        for (int k = 0; k + 1 <= o.K - 1; ++k) {
            const double* yk = f.Yb[cur];
            // Z = Y_k G (right) or G Y_k (left)
            if (right)
                s = gemm64<false, false>(st, m, n, n, yk, n, f.G, n, f.Z, n);
            else
                s = gemm64<false, false>(st, m, n, m, f.G, m, yk, n, f.Z, n);
            if (s != CPA_OK) return s;
            hipLaunchKernelGGL(cheb64_step_kernel, dim3(ge), dim3(256), 0, st, m, n, (const double*)f.Z, yk,
                               (int64_t)n, f.Yb[cur ^ 1], Y_dev, ldy, (const double*)w.scal, k);
            HIP_TRY(hipGetLastError());
            cur ^= 1;
        }
    }
    if (info_host) {
        if ((s = read_info(st, w, o.K, m, n, info_host, nullptr)) != CPA_OK) return s;
        info_host->side = right ? 0 : 1;
    }
    return CPA_OK;
}

}  // extern "C"

// ---- One-call RPCA driver ----

extern "C" {

cpa_status cpa_rpca_admm(cpa_ctx* ctx, void* stream, int m, int n, const float* I_dev, float* L_dev, float* S_dev,
                         double inv_rho, double eta_over_rho, int max_iters, double tol, const cpa_opts* opts,
                         double* Et_host, int* iters_done) {
    cpa_status s;
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (m < 0 || n < 0) return fail(CPA_ERR_SHAPE, "negative size");
    if (max_iters < 0) return fail(CPA_ERR_ARG, "max_iters < 0");
    if (!(tol >= 0.0)) return fail(CPA_ERR_ARG, "tol must be >= 0");
    if ((s = check_opts(opts)) != CPA_OK) return s;
    if ((s = no_learned_bound(opts)) != CPA_OK) return s;
    if (iters_done) *iters_done = 0;
    if (m == 0 || n == 0 || max_iters == 0) return CPA_OK;
    if (!I_dev || !L_dev || !S_dev) return fail(CPA_ERR_ARG, "I, L or S is NULL");
    const int64_t mn = (int64_t)m * n;
    const size_t b = sizeof(float) * (size_t)mn;
    if (overlaps(L_dev, b, S_dev, b) || overlaps(L_dev, b, I_dev, b) || overlaps(S_dev, b, I_dev, b))
        return fail(CPA_ERR_ARG, "I, L and S must not overlap");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t need = align_up(sizeof(float) * 7 * (size_t)mn) + sizeof(double);
    if (need > ctx->rpca_bytes) {
        if (ctx->rpca) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ctx->rpca));
            ctx->rpca = nullptr;
            ctx->rpca_bytes = 0;
        }
        if (hipMalloc(&ctx->rpca, need) != hipSuccess) {
            ctx->rpca = nullptr;
            return fail(CPA_ERR_ALLOC, "RPCA state allocation of %zu bytes failed", need);
        }
        ctx->rpca_bytes = need;
    }
    float* state = static_cast<float*>(ctx->rpca);
    double* et_dev = reinterpret_cast<double*>(static_cast<char*>(ctx->rpca) + align_up(sizeof(float) * 7 * (size_t)mn));
    if ((s = cpa_rpca_init(ctx, stream, m, n, state)) != CPA_OK) return s;
    int t = 0;
    while (t < max_iters) {
        if ((s = cpa_rpca_iterate(ctx, stream, m, n, I_dev, state, 1, inv_rho, eta_over_rho, opts, et_dev)) != CPA_OK)
            return s;
        double e = 0.0;
        HIP_TRY(hipMemcpyAsync(&e, et_dev, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (Et_host) Et_host[t] = e;
        ++t;
        if (e <= tol) break;
    }
    if (iters_done) *iters_done = t;
    HIP_TRY(hipMemcpyAsync(L_dev, state, b, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(S_dev, state + mn, b, hipMemcpyDeviceToDevice, st));
    return CPA_OK;
}

}  // extern "C"

// ---- Predictor model files ----

extern "C" {

static const char kModelMagic[8] = {'C', 'P', 'A', 'P', 'R', 'E', 'D', '1'};

cpa_status cpa_predictor_save(cpa_ctx* ctx, void* stream, const float* model_dev, const char* path) {
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (!model_dev || !path) return fail(CPA_ERR_ARG, "model or path is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<float> h(CPA_PRED_MODEL_FLOATS);
    HIP_TRY(hipMemcpyAsync(h.data(), model_dev, sizeof(float) * h.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return fail(CPA_ERR_IO, "cannot open %s for writing", path);
    const int32_t hdr[2] = {1, CPA_PRED_MODEL_FLOATS};
    bool ok = std::fwrite(kModelMagic, 1, 8, fp) == 8 && std::fwrite(hdr, sizeof(int32_t), 2, fp) == 2 &&
              std::fwrite(h.data(), sizeof(float), h.size(), fp) == h.size();
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return fail(CPA_ERR_IO, "write to %s failed", path);
    return CPA_OK;
}

cpa_status cpa_predictor_load(cpa_ctx* ctx, void* stream, const char* path, float* model_dev) {
    if (!ctx) return fail(CPA_ERR_ARG, "context is NULL");
    if (!model_dev || !path) return fail(CPA_ERR_ARG, "model or path is NULL");
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(CPA_ERR_IO, "cannot open %s", path);
    char magic[8];
    int32_t hdr[2] = {0, 0};
    std::vector<float> h(CPA_PRED_MODEL_FLOATS);
    const bool head = std::fread(magic, 1, 8, fp) == 8 && std::fread(hdr, sizeof(int32_t), 2, fp) == 2;
    const bool good = head && std::memcmp(magic, kModelMagic, 8) == 0 && hdr[0] == 1 &&
                      hdr[1] == CPA_PRED_MODEL_FLOATS && std::fread(h.data(), sizeof(float), h.size(), fp) == h.size();
    std::fclose(fp);
    if (!good) return fail(CPA_ERR_IO, "%s is not a version-1 model file of %d floats", path, CPA_PRED_MODEL_FLOATS);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(model_dev, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return CPA_OK;
}

}  // extern "C"
