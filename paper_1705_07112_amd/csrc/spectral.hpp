// Spectral bound (Algorithm 1, the maximum-eigenvalue step) and the per-call
// scalar block: power iteration or k-step Lanczos on the Gram with FP64
// accumulation, the bound rule, and the FP64 Chebyshev coefficients (Sec. III-A,
// eq. chebychev_coeff_shifted) computed on the device from that bound.
//
// Gram sides up to 256 run either iteration in one workgroup that holds G in
// registers (power_wg_kernel, lanczos_wg_kernel).  Larger sides run in one launch
// whose workgroups are all resident (at most one per CU, or a cooperative
// launch) with a grid barrier per product (power_coop_kernel, lanczos_coop_kernel).
// The power iteration:
//   w_0 = v_0 (SplitMix64 start vector or the warm-start vector)
//   product t: v_t = w_{t-1} / ||w_{t-1}||, w_t = G v_t,
//              mu_t = v_t . w_t and ||w_t||^2 in FP64: each workgroup stores its
//              partial sums, and after the barrier every workgroup adds all
//              partials in the same order, so all of them take the same
//              stopping decision;
//   stop after product t when |mu_t - mu_{t-1}| <= tol mu_t (t >= 2) or
//   ||w_t|| == 0, or after maxit products.
// The finishing kernel forms ||r|| = sqrt(max(||w_T||^2 - mu_T^2, 0)) and
//   Lambda = min(mu_T + max(margin mu_T, ||r||), (1 + margin) ||G||_F).
// ||G||_F >= lambda_max caps runaway residual terms without removing the
// margin: a bound equal to lambda_max would place the top eigenvalue on the
// endpoint of [-1, 1] where T_k has slope k^2 and FP32 rounding is amplified.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mlp.hpp"
#include "shrink_fn.hpp"

namespace cpa {

// Scalar block layout (doubles).  Every per-call quantity lives here so a whole
// shrink is enqueued without host round trips.
enum : int {
    SC_FRO2 = 0,      // ||G||_F^2
    SC_TRACE = 1,     // trace G = ||X||_F^2
    SC_LAMBDA = 2,
    SC_MU = 3,
    SC_RESID = 4,
    SC_ITERS = 5,
    SC_STOP = 6,      // product index after which iteration stopped (0: not yet)
    SC_VANISH = 7,    // 1 if a product vanished while ||G||_F > 0
    SC_A1 = 8,        // 2 / Lambda (0 if Lambda == 0)
    SC_A2 = 9,        // 4 / Lambda
    SC_ET_NUM = 10,   // ADMM: ||l_new - l_old||^2
    SC_ET_DEN = 11,   // ADMM: ||l_new||^2
    SC_TIMEOUT = 12,  // 1 if a grid barrier gave up waiting
    SC_BARRIER = 13,  // grid-barrier arrival counter (first 4 bytes, zeroed with the block)
    SC_COEF = 16      // K coefficients, then the other regions below
};

constexpr int kNormSlots = 64;   // partial-sum slots per growth-check norm

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPsMaxS = 32;   // largest baby-step count of the matrix-polynomial route (K <= 1024)
constexpr int kPsCheckWg = 64;   // workgroups of the matrix-polynomial route's a-posteriori check

struct ScalarLayout {
    int K, maxit, gwg, pwg;      // gwg: Gram workgroups, pwg: power-iteration workgroups
    int coef() const { return SC_COEF; }
    int norms() const { return SC_COEF + K; }                          // K x kNormSlots
    int pw_mu() const { return norms() + K * kNormSlots; }            // mu_t, t = 0..maxit
    int pw_w2() const { return pw_mu() + maxit + 1; }                 // ||w_t||^2
    int gpart() const { return pw_w2() + maxit + 1; }                 // 2 per Gram workgroup
    int ppart() const { return gpart() + 2 * gwg; }                   // 2 x 2 per power workgroup
    int ps() const { return ppart() + 4 * pwg; }                       // matrix-polynomial coefficients
    int pchk() const { return ps() + K + kPsMaxS; }                     // check partials, (q - 2) x kPsCheckWg
    int total() const { return pchk() + (kPsMaxS - 1) * kPsCheckWg; }
};

__global__ void fill_f64_kernel(double* p, int n, double v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__device__ inline uint64_t splitmix64_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// w0 = start vector; ||w0||^2 into pw_w2[0].  warm != nullptr: copy it (unless its
// norm is zero).
// Single workgroup (fixed summation order).
__device__ inline void power_init_body(int d, uint64_t seed, const double* warm, double* w0, double* scal, int pw_w2,
                                       double* red) {
    if (warm) {
        // a warm vector without weight (e.g. mapped from rows that are all gone) gives
        // way to the seeded start
        double wn = 0.0;
        for (int i = threadIdx.x; i < d; i += blockDim.x) wn += warm[i] * warm[i];
        wn = block_sum(wn, red);
        if (!(wn > 0.0)) warm = nullptr;
    }
    double acc = 0.0;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        double v;
        if (warm) {
            v = warm[i];
        } else {
            const uint64_t out = splitmix64_out(seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
            v = 2.0 * ((double)(out >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
        }
        w0[i] = v;
        acc += v * v;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) scal[pw_w2] = acc;
}

__global__ void power_init_kernel(int d, uint64_t seed, const double* warm, double* w0, double* scal, int pw_w2) {
    __shared__ double red[16];
    power_init_body(d, seed, warm, w0, scal, pw_w2, red);
}

constexpr int kPowerThreads = 512;

// Grid barrier: a monotonically increasing arrival counter (zeroed before the
// launch); barrier number b completes when the counter reaches b * gridDim.x.
// Every workgroup of the grid must become resident (a cooperative launch, or at
// most one workgroup per CU).  The wait is bounded: on time-out the workgroup
// records SC_TIMEOUT and reports failure, so every wave exits.
__device__ inline bool grid_barrier(unsigned* counter, unsigned target, double* scal) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > (1u << 22)) {
                good = 0;
                scal[SC_TIMEOUT] = 1.0;
                break;
            }
        }
        __threadfence();
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// Grid barrier for kernels that exchange data only through agent-scope atomic
// accesses (coherent across the XCDs' L2 caches without flushing them): each
// thread's stores have completed (vmcnt) before its workgroup arrives, and the
// spin reads the counter with relaxed loads.  Unlike grid_barrier it writes back
// and invalidates no cache, so G stays in L2 from one product to the next.
__device__ inline bool grid_barrier_coherent(unsigned* counter, unsigned target, double* scal) {
    __shared__ int ok;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > (1u << 22)) {
                good = 0;
                scal[SC_TIMEOUT] = 1.0;
                break;
            }
        }
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

__device__ inline double ld_agent(const double* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void st_agent(double* p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Sum of part[0..n) in a fixed order (same result in every workgroup).
__device__ inline double ordered_sum(const double* part, int n, double* red) {
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a += part[i];
    return block_sum(a, red);
}

// All products of the power iteration in one launch (see top).
// The iterate and the partial sums written during the launch are exchanged
// through agent-scope atomic stores and loads (grid_barrier_coherent); each
// workgroup copies w_{t-1} into LDS once per product (d <= kPowerVecLds; above
// that the matvec reads it with agent-scope loads).
constexpr int kPowerVecLds = 4096;

// TG: the Gram's element type (float, or double for the FP64 path).
template <class TG>
__global__ void __launch_bounds__(kPowerThreads) power_coop_kernel(int d, const TG* G, int64_t ldg, double* wb0,
                                                                   double* wb1, double* part, unsigned* counter,
                                                                   double* scal, int maxit, double tol, int pw_mu,
                                                                   int pw_w2) {
    __shared__ double red[kPowerThreads / 64];
    __shared__ double bcast[2];
    __shared__ __attribute__((aligned(16))) double vl[kPowerVecLds];
    const int P = gridDim.x;
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (kPowerThreads / 64) + (threadIdx.x >> 6);
    const int nw = P * (kPowerThreads / 64);
    const bool in_lds = d <= kPowerVecLds;
    double w2prev = scal[pw_w2 + 0];
    double muprev = 0.0;
    int stop = 0, vanish = 0;
    if (!(w2prev > 0.0)) vanish = 1;
    int t = 1;
    // the iterate in LDS: w_0 here, then w_t right after each barrier (its loads
    // overlap the loads of the partial sums)
    if (in_lds && !vanish) {
        for (int j = threadIdx.x; j < d; j += kPowerThreads) vl[j] = ld_agent(wb0 + j);
        __syncthreads();
    }
    for (; !vanish && t <= maxit; ++t) {
        const double* wp = (t & 1) ? wb0 : wb1;   // w_{t-1}
        double* wn = (t & 1) ? wb1 : wb0;         // w_t
        const double inv = 1.0 / sqrt(w2prev);
        double mu_part = 0.0, w2_part = 0.0;
        const bool vec = std::is_same<TG, float>::value && ((ldg & 3) == 0) &&
                         ((reinterpret_cast<uintptr_t>(G) & 15) == 0) && in_lds;
        for (int i = gw; i < d; i += nw) {
            const TG* row = G + (int64_t)i * ldg;
            // four independent partial sums, 16-byte loads of G when rows are aligned,
            // several loads in flight per lane (the sum is scaled by 1/||w|| at the end)
            double a[4] = {0.0, 0.0, 0.0, 0.0};
            int j = 4 * lane;
            if constexpr (std::is_same<TG, float>::value) {
                if (vec) {
#pragma unroll 4
                    for (; j + 3 < d; j += 256) {
                        const f32x4 g = *reinterpret_cast<const f32x4*>(row + j);
                        const double2 v01 = *reinterpret_cast<const double2*>(vl + j);
                        const double2 v23 = *reinterpret_cast<const double2*>(vl + j + 2);
                        a[0] += (double)g[0] * v01.x;
                        a[1] += (double)g[1] * v01.y;
                        a[2] += (double)g[2] * v23.x;
                        a[3] += (double)g[3] * v23.y;
                    }
                }
            }
            for (; j < d; j += 256)
                for (int e = 0; e < 4; ++e)
                    if (j + e < d) a[e] += (double)row[j + e] * (in_lds ? vl[j + e] : ld_agent(wp + j + e));
            double acc = (a[0] + a[1]) + (a[2] + a[3]);
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            acc *= inv;
            if (lane == 0) {
                st_agent(wn + i, acc);
                mu_part += ((in_lds ? vl[i] : ld_agent(wp + i)) * inv) * acc;
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
        if (!grid_barrier_coherent(counter, (unsigned)t * P, scal)) return;
        double smu = 0.0, sw2 = 0.0;
        for (int i = threadIdx.x; i < P; i += kPowerThreads) {
            smu += ld_agent(pt + i);
            sw2 += ld_agent(pt + P + i);
        }
        // vl (w_{t-1}) was last read before the barrier; the block sums below
        // synchronise the workgroup before the next product reads w_t
        if (in_lds)
            for (int j = threadIdx.x; j < d; j += kPowerThreads) vl[j] = ld_agent(wn + j);
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

// Power iteration for a Gram of side d <= kPowerWgMaxD in one workgroup: the same
// products, Rayleigh quotients, stopping rule and outputs as power_coop_kernel
// (w_t in the buffer of t's parity, mu_t and ||w_t||^2 in their slots, the stop
// record), with G held in registers for the whole iteration, so that a product
// costs two workgroup barriers instead of device-wide round trips.  Wave w takes
// the 64 x 64 block of G at row block w % 4 and column block w / 4: lane l holds
// row 64 (w % 4) + l of that block (64 floats) and v's entry for column
// 64 (w / 4) + l, which the products broadcast by readlane.  Entries past d are
// zero, so every wave runs the same steps.  The four partial row sums meet in LDS
// and are added in a fixed order; each sum over the d rows is four wave sums
// (DPP, fixed order) added in a fixed order, so every wave takes the same
// stopping decision.
constexpr int kPowerWgMaxD = 256;
constexpr int kPowerWgThreads = 1024;

__device__ inline double pw_readlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL>
__device__ inline double pw_dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// a[j % 4] += g[j] * (v of lane j), j = 0..63 in order: this lane's row slice
// against the wave's 64 entries of the vector.  The broadcasts are taken eight at
// a time ahead of their products, so the scalar registers they fill are not
// reused back to back.
__device__ inline void pw_rowdot(const float (&g)[64], double v, double (&a)[4]) {
#pragma unroll
    for (int j0 = 0; j0 < 64; j0 += 8) {
        double vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) vv[u] = pw_readlane(v, j0 + u);
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u & 3] += (double)g[j0 + u] * vv[u];
    }
}

// Sums of a and b over the 64 lanes (equal in every lane): within rows of 16
// lanes swap neighbours, swap pairs, mirror halves, mirror the row; then the
// four row sums in a fixed order.
__device__ inline void pw_wave_sum2(double& a, double& b) {
    a += pw_dpp<0xB1>(a);
    b += pw_dpp<0xB1>(b);
    a += pw_dpp<0x4E>(a);
    b += pw_dpp<0x4E>(b);
    a += pw_dpp<0x141>(a);
    b += pw_dpp<0x141>(b);
    a += pw_dpp<0x140>(a);
    b += pw_dpp<0x140>(b);
    a = (pw_readlane(a, 0) + pw_readlane(a, 16)) + (pw_readlane(a, 32) + pw_readlane(a, 48));
    b = (pw_readlane(b, 0) + pw_readlane(b, 16)) + (pw_readlane(b, 32) + pw_readlane(b, 48));
}

__global__ void __launch_bounds__(kPowerWgThreads) power_wg_kernel(int d, const float* G, int64_t ldg, double* wb0,
                                                                 double* wb1, double* scal, int maxit, double tol,
                                                                 int pw_mu, int pw_w2) {
    __shared__ double rowp[2][4][kPowerWgMaxD];   // partial row sums by column block, by parity
    __shared__ double red[2][2][4];               // per column block: v.w and ||w||^2 parts, by parity
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rb = wave & 3, cb = wave >> 2;
    const int row = 64 * rb + lane, col = 64 * cb + lane;
    const bool live = 64 * rb < d && 64 * cb < d;   // uniform per wave
    float g[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) g[j] = 0.f;
    if (live && row < d) {
        const float* gr = G + (int64_t)row * ldg + 64 * cb;
        if (((ldg & 3) == 0) && ((reinterpret_cast<uintptr_t>(G) & 15) == 0) && 64 * cb + 64 <= d) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const f32x4 x = *reinterpret_cast<const f32x4*>(gr + 4 * q);
                g[4 * q] = x[0];
                g[4 * q + 1] = x[1];
                g[4 * q + 2] = x[2];
                g[4 * q + 3] = x[3];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 64; ++j)
                if (64 * cb + j < d) g[j] = gr[j];
        }
    }
    double v = col < d ? wb0[col] : 0.0;   // w_{t-1} for this lane's column (unnormalised)
    double w2prev = scal[pw_w2 + 0];
    double muprev = 0.0;
    int stop = 0, vanish = !(w2prev > 0.0);
    int t = 1;
    for (; !vanish && t <= maxit; ++t) {
        const int par = t & 1;
        const double inv = 1.0 / sqrt(w2prev);
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        if (live) {
            // the empty asm keeps the FP64 conversions of G inside the loop (hoisted,
            // they would take 128 registers)
#pragma unroll
            for (int j = 0; j < 64; ++j) asm volatile("" : "+v"(g[j]));
            pw_rowdot(g, v, a);
        }
        rowp[par][cb][row] = (a[0] + a[1]) + (a[2] + a[3]);
        __syncthreads();
        // w_t for this lane's column, the new iterate (rows and columns share the index)
        const double wi = ((rowp[par][0][col] + rowp[par][1][col]) + (rowp[par][2][col] + rowp[par][3][col])) * inv;
        if (rb == 0) {
            // the sums over this column block (the other waves hold the same wi)
            double mu_p = (v * inv) * wi, w2_p = wi * wi;
            pw_wave_sum2(mu_p, w2_p);
            if (lane == 0) {
                red[par][0][cb] = mu_p;
                red[par][1][cb] = w2_p;
            }
            if (col < d) ((t & 1) ? wb1 : wb0)[col] = wi;
        }
        __syncthreads();
        const double mu = (red[par][0][0] + red[par][0][1]) + (red[par][0][2] + red[par][0][3]);
        const double w2 = (red[par][1][0] + red[par][1][1]) + (red[par][1][2] + red[par][1][3]);
        if (threadIdx.x == 0) {
            scal[pw_mu + t] = mu;
            scal[pw_w2 + t] = w2;
        }
        if (!(w2 > 0.0)) {
            vanish = 1;
            break;
        }
        if (t >= 2 && fabs(mu - muprev) <= tol * mu) {
            stop = t;
            break;
        }
        muprev = mu;
        w2prev = w2;
        v = wi;
    }
    if (threadIdx.x == 0) {
        scal[SC_STOP] = stop ? stop : (vanish ? 0 : maxit);
        scal[SC_VANISH] = vanish;
    }
}

// ---- k-step Lanczos bound (a second reading of the maximum-eigenvalue step)
//   q_1 = w_0 / ||w_0||, beta_0 = 0; step j: u = G q_j - beta_{j-1} q_{j-1},
//   alpha_j = q_j.u, u <- u - alpha_j q_j, beta_j = ||u||, q_{j+1} = u / beta_j
//   (no reorthogonalisation; an exactly vanishing beta_j ends the run, and with
//   tol > 0 so does the first step j >= 2 whose Ritz value moved by at most
//   tol theta_j), then the largest eigenvalue theta of the tridiagonal T_k, its
//   unit eigenvector s, the
//   Ritz residual ||r|| = beta_k |s_k| and the Ritz vector y = sum_j s_j q_j.  The
//   power slots receive mu_T = theta and ||w_T||^2 = theta^2 + ||r||^2, so the
//   finishing kernel's rule gives Lambda = min(theta + max(margin theta, ||r||),
//   (1 + margin) ||G||_F), and y goes where the power iteration leaves its last
//   vector (the warm start of the next call).
constexpr int kLanczosMax = 32;
constexpr int kLanczosDefault = 12;

__device__ inline double pw_wave_sum(double a) {
    a += pw_dpp<0xB1>(a);
    a += pw_dpp<0x4E>(a);
    a += pw_dpp<0x141>(a);
    a += pw_dpp<0x140>(a);
    return (pw_readlane(a, 0) + pw_readlane(a, 16)) + (pw_readlane(a, 32) + pw_readlane(a, 48));
}

// 1 / x: the hardware estimate and one Newton step (relative error near 2^-44,
// a relative perturbation of that size of the pivots' quotients).
__device__ inline double lz_rcp(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// Ritz pair of T_k for its largest eigenvalue, by one wave: lane i < k holds
// al = alpha_i and be = beta_i (T(i, i+1) for i < k - 1; lane k - 1 holds beta_k,
// the coupling to the next Krylov vector, which is not part of T_k).
//   theta: multisection -- each round the 64 lanes count the eigenvalues above 64
//     equispaced points of the bracket [max alpha_i, Gershgorin bound] by the signs
//     of the LDL^T pivots of T - x I (a zero pivot taken as -pivmin), and the
//     bracket shrinks to the gap above the highest point with a count of at least
//     one, until it is 2^-30 of theta wide (the bound adds a relative margin of
//     about 1e-2, so theta is kept to about 1e-9; five rounds from a bracket of
//     theta's size);
//   s: the backward three-term recurrence s_{k-1} = 1,
//     s_{i-1} = ((theta - alpha_i) s_i - beta_i s_{i+1}) / beta_{i-1} (the direction
//     in which the top Ritz vector's entries grow), rescaled by 2^-400 whenever an
//     entry passes 2^400, then normalised; lane i receives s_i;
//   resid = beta_k |s_{k-1}|.
// theta and resid are the same in every lane (same operations on the same data).
__device__ inline void lz_ritz(double al, double be, int k, double& theta, double& resid, double& s_out) {
    const int lane = threadIdx.x & 63;
    const double bsq = be * be;
    double lo = pw_readlane(al, 0), hi = lo, bmax2 = 0.0;
    for (int i = 0; i < k; ++i) {
        const double a = pw_readlane(al, i);
        const double b0 = i > 0 ? fabs(pw_readlane(be, i - 1)) : 0.0;
        const double b1 = i + 1 < k ? fabs(pw_readlane(be, i)) : 0.0;
        lo = fmax(lo, a);
        hi = fmax(hi, a + b0 + b1);
        if (i + 1 < k) bmax2 = fmax(bmax2, pw_readlane(bsq, i));
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, bmax2);
    for (int round = 0; round < 12; ++round) {
        if (!(hi - lo > 0x1p-30 * fmax(fabs(lo), fabs(hi)))) break;
        const double x = lo + (hi - lo) * ((double)(lane + 1) * (1.0 / 65.0));
        int neg = 0;
        double q = 1.0;
        for (int i = 0; i < k; ++i) {
            q = (pw_readlane(al, i) - x) - (i > 0 ? pw_readlane(bsq, i - 1) * lz_rcp(q) : 0.0);
            if (fabs(q) < pivmin) q = -pivmin;
            neg += q < 0.0 ? 1 : 0;
        }
        const uint64_t mask = __ballot(k - neg >= 1);
        const int L = mask ? 63 - __clzll(mask) : -1;
        const double xl = pw_readlane(x, L < 0 ? 0 : L);
        const double xh = pw_readlane(x, L < 63 ? L + 1 : 63);
        if (L >= 0) lo = xl;
        if (L < 63) hi = xh;
    }
    theta = 0.5 * (lo + hi);
    double s_mine = lane == k - 1 ? 1.0 : 0.0;
    double s_next = 0.0, s_cur = 1.0;
    for (int i = k - 1; i >= 1; --i) {
        const double bi = i + 1 < k ? pw_readlane(be, i) : 0.0;
        double s_prev = ((theta - pw_readlane(al, i)) * s_cur - bi * s_next) * lz_rcp(pw_readlane(be, i - 1));
        if (fabs(s_prev) > 0x1p400) {
            s_prev *= 0x1p-400;
            s_cur *= 0x1p-400;
            s_mine *= 0x1p-400;
        }
        if (lane == i - 1) s_mine = s_prev;
        s_next = s_cur;
        s_cur = s_prev;
    }
    const double nrm = sqrt(pw_wave_sum(s_mine * s_mine));
    s_out = s_mine / nrm;
    resid = fabs(pw_readlane(be, k - 1)) * fabs(pw_readlane(s_out, k - 1));
}

// The Ritz pair of T_j is formed by the first wave only, during step j (while
// the other waves take their rows of G q_j), into LDS slots by step parity; the
// step's barrier publishes it together with the stopping decision, and a run
// that stops there keeps k = j (the products of step j are dropped).  A run
// that ends by its step count or a vanishing beta forms the pair of T_k after
// the loop, into a third slot.  kLzSlot: s_0..s_{k-1}, then theta, ||r|| and the
// stop flag.
constexpr int kLzSlot = kLanczosMax + 3;

// k-step Lanczos for a Gram of side d <= kPowerWgMaxD in one workgroup, steps <=
// kLanczosMax: the register layout of power_wg_kernel for the products; the
// Lanczos vectors stay in LDS (for the Ritz vector).  Each step takes one
// workgroup barrier: after it every wave forms u on all d entries from the four
// partial row sums and adds alpha and ||u||^2 itself (the same operations in every
// wave, so every wave holds the same alpha_j and beta_j).
__global__ void __launch_bounds__(kPowerWgThreads) lanczos_wg_kernel(int d, const float* G, int64_t ldg, double* wb0,
                                                                   double* wb1, double* scal, int steps, double tol,
                                                                   int pw_mu, int pw_w2) {
    __shared__ double rowp[2][4][kPowerWgMaxD];   // partial row sums by column block, by parity
    __shared__ double Q[kLanczosMax][kPowerWgMaxD];
    __shared__ double rz[3][kLzSlot];             // Ritz pairs: by step parity, then the final one
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rb = wave & 3, cb = wave >> 2;
    const int row = 64 * rb + lane, col = 64 * cb + lane;
    const bool live = 64 * rb < d && 64 * cb < d;
    float g[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) g[j] = 0.f;
    if (live && row < d) {
        const float* gr = G + (int64_t)row * ldg + 64 * cb;
        if (((ldg & 3) == 0) && ((reinterpret_cast<uintptr_t>(G) & 15) == 0) && 64 * cb + 64 <= d) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const f32x4 x = *reinterpret_cast<const f32x4*>(gr + 4 * q);
                g[4 * q] = x[0];
                g[4 * q + 1] = x[1];
                g[4 * q + 2] = x[2];
                g[4 * q + 3] = x[3];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 64; ++j)
                if (64 * cb + j < d) g[j] = gr[j];
        }
    }
    const double n0 = scal[pw_w2 + 0];
    if (!(n0 > 0.0)) {
        // no start vector: the finishing kernel falls back to ||G||_F
        if (threadIdx.x == 0) {
            scal[SC_STOP] = 0;
            scal[SC_VANISH] = 1;
        }
        return;
    }
    double q = col < d ? wb0[col] / sqrt(n0) : 0.0;   // q_j at this lane's column
    double bprev = 0.0;
    double al = 0.0, be = 0.0;   // lane j: alpha_j, beta_j
    double th_prev = 0.0;        // first wave: the Ritz value of T_{j-1}
    int k = 0, vanish = 0, slot = -1;
    for (int j = 0; j < steps; ++j) {
        const int par = j & 1;
        if (rb == 0) Q[j][col] = q;
        if (tol > 0.0 && j >= 1 && wave == 0) {
            double theta, resid, s;
            lz_ritz(al, be, j, theta, resid, s);
            const bool stop = j >= 2 && fabs(theta - th_prev) <= tol * theta;
            th_prev = theta;
            if (lane < j) rz[par][lane] = s;
            if (lane == 0) {
                rz[par][kLanczosMax] = theta;
                rz[par][kLanczosMax + 1] = resid;
                rz[par][kLanczosMax + 2] = stop ? 1.0 : 0.0;
            }
        }
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        if (live) {
#pragma unroll
            for (int jj = 0; jj < 64; ++jj) asm volatile("" : "+v"(g[jj]));
            pw_rowdot(g, q, a);
        }
        rowp[par][cb][row] = (a[0] + a[1]) + (a[2] + a[3]);
        __syncthreads();
        if (tol > 0.0 && j >= 1 && rz[par][kLanczosMax + 2] != 0.0) {
            slot = par;   // k = j
            break;
        }
        double u[4], qc[4];
        double pa = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int cc = 64 * c + lane;
            const double gq = (rowp[par][0][cc] + rowp[par][1][cc]) + (rowp[par][2][cc] + rowp[par][3][cc]);
            qc[c] = Q[j][cc];
            u[c] = gq - (j > 0 ? bprev * Q[j - 1][cc] : 0.0);
            pa += qc[c] * u[c];
        }
        const double alpha = pw_wave_sum(pa);
        double pb = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            u[c] -= alpha * qc[c];
            pb += u[c] * u[c];
        }
        const double beta = sqrt(pw_wave_sum(pb));
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
        const double uc = cb == 0 ? u[0] : (cb == 1 ? u[1] : (cb == 2 ? u[2] : u[3]));
        q = uc / beta;
        bprev = beta;
    }
    if (vanish) {
        if (threadIdx.x == 0) {
            scal[SC_STOP] = 0;
            scal[SC_VANISH] = 1;
        }
        return;
    }
    if (slot < 0) {
        // the Ritz pair of T_k
        slot = 2;
        if (wave == 0) {
            double theta, resid, s;
            lz_ritz(al, be, k, theta, resid, s);
            if (lane < k) rz[2][lane] = s;
            if (lane == 0) {
                rz[2][kLanczosMax] = theta;
                rz[2][kLanczosMax + 1] = resid;
            }
        }
        __syncthreads();
    }
    // the Ritz vector into the buffer the finishing kernel reads the last vector
    // from (slot T - 1 holds its squared length: s is a unit vector)
    double* yb = ((k - 1) & 1) ? wb1 : wb0;
    if (threadIdx.x < d) {
        double y = 0.0;
        for (int i = 0; i < k; ++i) y += rz[slot][i] * Q[i][threadIdx.x];
        yb[threadIdx.x] = y;
    }
    if (threadIdx.x == 0) {
        const double theta = rz[slot][kLanczosMax], resid = rz[slot][kLanczosMax + 1];
        scal[pw_mu + k] = theta;
        scal[pw_w2 + k] = theta * theta + resid * resid;
        scal[pw_w2 + k - 1] = 1.0;
        scal[SC_STOP] = k;
        scal[SC_VANISH] = 0;
    }
}

// k-step Lanczos for Gram sides kPowerWgMaxD < d <= kPowerVecLds, in the power
// iteration's resident grid with one grid barrier per step:
//   before it, each workgroup's waves take rows of G q_j (q_j and q_{j-1} in
//   LDS), form u_i = (G q_j)_i - beta_{j-1} q_{j-1,i}, store u_i and q_{j,i}
//   (U and Q, agent scope) and add q_{j,i} u_i into the workgroup's partial;
//   after it, every workgroup adds the partials in a fixed order (alpha_j), loads
//   all of u, forms u - alpha_j q_j and ||.||^2 over the d entries itself (same
//   operations in every workgroup) and keeps q_{j+1} = u / beta_j in LDS.
// Every workgroup holds the same alpha and beta; with the early stop its first
// wave forms the Ritz pair of T_{j+1} once beta_j is known (a grid step costs
// several times the pair, so the pair is not deferred into the next step as in
// lanczos_wg_kernel), and every workgroup takes the same stopping decision; the
// Ritz vector's entry i is formed by the thread that stored Q[.][i].  Q holds steps + 2 vectors of d:
// the Lanczos vectors, then U by step parity (a workgroup that runs ahead writes
// the other one while the rest still read theirs; the same parity rule as the
// partial sums).
// TG: the Gram's element type (float, or double for the FP64 path).
template <class TG>
__global__ void __launch_bounds__(kPowerThreads) lanczos_coop_kernel(int d, const TG* G, int64_t ldg, double* wb0,
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
    for (int i = threadIdx.x; i < d; i += kPowerThreads) {
        va[i] = wb0[i] * inv0;   // q_1
        vb[i] = 0.0;             // q_0
    }
    __syncthreads();
    double* vq = va;   // q_j
    double* vp = vb;   // q_{j-1}, then u
    const bool vec = std::is_same<TG, float>::value && ((ldg & 3) == 0) && ((reinterpret_cast<uintptr_t>(G) & 15) == 0);
    double bprev = 0.0;
    double al = 0.0, be = 0.0, th_prev = 0.0;
    int k = 0, vanish = 0, slot = -1;
    for (int j = 0; j < steps; ++j) {
        const int par = j & 1;
        double* U = Q + (int64_t)(steps + par) * d;
        double apart = 0.0;
        for (int i = gw; i < d; i += nw) {
            const TG* row = G + (int64_t)i * ldg;
            double a[4] = {0.0, 0.0, 0.0, 0.0};
            int c = 4 * lane;
            if constexpr (std::is_same<TG, float>::value) {
                if (vec) {
#pragma unroll 4
                    for (; c + 3 < d; c += 256) {
                        const f32x4 g = *reinterpret_cast<const f32x4*>(row + c);
                        const double2 v01 = *reinterpret_cast<const double2*>(vq + c);
                        const double2 v23 = *reinterpret_cast<const double2*>(vq + c + 2);
                        a[0] += (double)g[0] * v01.x;
                        a[1] += (double)g[1] * v01.y;
                        a[2] += (double)g[2] * v23.x;
                        a[3] += (double)g[3] * v23.y;
                    }
                }
            }
            for (; c < d; c += 256)
                for (int e = 0; e < 4; ++e)
                    if (c + e < d) a[e] += (double)row[c + e] * vq[c + e];
            double acc = (a[0] + a[1]) + (a[2] + a[3]);
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) {
                const double ui = acc - bprev * vp[i];
                st_agent(U + i, ui);
                st_agent(Q + (int64_t)j * d + i, vq[i]);
                apart += vq[i] * ui;
            }
        }
        apart = block_sum(apart, red);
        double* pt = part + (j & 1) * 2 * P;
        if (threadIdx.x == 0) st_agent(pt + blockIdx.x, apart);
        if (!grid_barrier_coherent(counter, (unsigned)(j + 1) * P, scal)) return;
        double sa = 0.0;
        for (int p = threadIdx.x; p < P; p += kPowerThreads) sa += ld_agent(pt + p);
        const double alpha = block_sum(sa, red);
        // u - alpha q_j over all d entries, into vp (q_{j-1} is no longer needed)
        double b2 = 0.0;
        for (int i = threadIdx.x; i < d; i += kPowerThreads) {
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
                double theta, resid, s;
                lz_ritz(al, be, k, theta, resid, s);
                const bool stop = j >= 1 && fabs(theta - th_prev) <= tol * theta;
                th_prev = theta;
                if (lane < k) rz[par][lane] = s;
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
        for (int i = threadIdx.x; i < d; i += kPowerThreads) vp[i] *= ib;
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
            double theta, resid, s;
            lz_ritz(al, be, k, theta, resid, s);
            if (lane < k) rz[2][lane] = s;
            if (lane == 0) {
                rz[2][kLanczosMax] = theta;
                rz[2][kLanczosMax + 1] = resid;
            }
        }
        __syncthreads();
    }
    // the Ritz vector: entry i from the stores of the thread that owns row i
    double* yb = ((k - 1) & 1) ? wb1 : wb0;
    if (lane == 0) {
        for (int i = gw; i < d; i += nw) {
            double y = 0.0;
            for (int q = 0; q < k; ++q) y += rz[slot][q] * Q[(int64_t)q * d + i];
            yb[i] = y;
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

constexpr int kCoefLds = 1024;   // orders up to this use the cosine-table coefficient path

// Bound rule + coefficients + recurrence scalars.  Single workgroup.
//   mode 0: power iteration result (products 1..maxit in the slots)
//   mode 1: Lambda given
//   mode 2: Lambda = ||G||_F (tr G when cap_trace)
// For mode 0 the warm-start buffer receives v_T (the unit vector of the last product).
__device__ inline void ps_coeff_block(int K, int s, int J, double* scal, int out);

// coeffs != nullptr: c_0..c_{K-1} are copied from there instead of computed.
// Workgroups past the first (launched when T1s is set) form the
// matrix-polynomial route's T1 = (2 / Lambda) G - I from G (pitch ldgs), the
// work of ps_shift_kernel, once each has the bound.
// ps_out >= 0: the coefficients are also rewritten for the matrix-polynomial route
// with baby steps of ps_s (ps_coeff_block), saving that route a launch.
// mode: 0 power iteration, 1 given, 2 Frobenius, 3 the predictor network
// `model` on the features (log ||X||_F, log ||G||_F^2, log mn) (logmn = log mn):
// Lambda = (1 + margin) ||G||_F exp(min(y0, 0)), never above the Frobenius cap.
__global__ void finish_bound_kernel(int mode, double Lambda_given, int d, int maxit, double margin,
                                    const double* wbuf0, const double* wbuf1, double* warm_out, double* scal,
                                    ShrinkParams sp, int K, int pw_mu, int pw_w2, const double* gpart, int gwg,
                                    int cap_trace, int damping, int ps_s, int ps_out, const float* model,
                                    double logmn, const double* coeffs, const float* Gs, int64_t ldgs, float* T1s) {
    __shared__ double sLambda;
    __shared__ int sT;
    __shared__ double red[16];
    __shared__ float mlp_h[2 * kMlpH], mlp_y[2];
    // Gram statistics from the per-workgroup partials, in a fixed order
    double f2 = 0.0, tr = 0.0;
    for (int i = threadIdx.x; i < gwg; i += blockDim.x) {
        f2 += gpart[2 * i];
        tr += gpart[2 * i + 1];
    }
    f2 = block_sum(f2, red);
    tr = block_sum(tr, red);
    float y0 = 0.f;
    if (mode == 3 && f2 > 0.0 && tr > 0.0) {
        float y1;
        mlp_infer_wg(model, (float)(0.5 * log(tr)), (float)log(f2), (float)logmn, mlp_h, mlp_y, y0, y1);
    }
    // workgroup 0 stores the bound and the coefficients; the others (T1s set)
    // arrive at the same Lambda from the same inputs and form T1 = (2 / Lambda) G - I
    const bool lead = blockIdx.x == 0;
    if (threadIdx.x == 0) {
        if (lead) {
            scal[SC_FRO2] = f2;
            scal[SC_TRACE] = tr;
        }
        // cap_trace: only tr(G) is known (operator form); tr(G) >= ||G||_F >= lambda_max
        const double fro = cap_trace ? tr : sqrt(f2 > 0.0 ? f2 : 0.0);
        double Lam = 0.0;
        int T = 0;
        if (mode == 1) {
            Lam = Lambda_given;
        } else if (mode == 2) {
            Lam = fro;
        } else if (mode == 3) {
            Lam = fro > 0.0 ? (1.0 + margin) * fro * exp((double)(y0 < 0.f ? y0 : 0.f)) : 0.0;
        } else if (fro > 0.0) {
            T = (int)scal[SC_STOP];
            if (scal[SC_VANISH] != 0.0 || scal[SC_TIMEOUT] != 0.0 || T < 1) {
                Lam = fro;
                T = 0;
            } else {
                const double mu = scal[pw_mu + T];
                const double w2 = scal[pw_w2 + T];
                const double r2 = w2 - mu * mu;
                const double r = sqrt(r2 > 0.0 ? r2 : 0.0);
                const double add = (margin * mu > r) ? margin * mu : r;
                Lam = mu + add;
                if (Lam > (1.0 + margin) * fro) Lam = (1.0 + margin) * fro;
                if (lead) {
                    scal[SC_MU] = mu;
                    scal[SC_RESID] = r;
                }
            }
        }
        if (lead) {
            scal[SC_ITERS] = T;
            scal[SC_LAMBDA] = Lam;
            scal[SC_A1] = Lam > 0.0 ? 2.0 / Lam : 0.0;
            scal[SC_A2] = Lam > 0.0 ? 4.0 / Lam : 0.0;
        }
        sLambda = Lam;
        sT = T;
    }
    __syncthreads();
    const double Lam = sLambda;
    if (!lead) {
        // T1 = (2 / Lambda) G - I (d x d, pitch d; G with pitch ldgs), the scale
        // rounded to FP32 as the polynomial's products read it
        const float a1 = (float)(Lam > 0.0 ? 2.0 / Lam : 0.0);
        const int64_t stride = (int64_t)(gridDim.x - 1) * blockDim.x;
        const int64_t first = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x;
        if ((d & 3) == 0 && (ldgs & 3) == 0 && ((uintptr_t)Gs & 15) == 0 && ((uintptr_t)T1s & 15) == 0) {
            // four elements of one row per access, four accesses per thread in flight
            // (all loads before the first store)
            const int64_t total4 = (int64_t)d * d / 4;
            for (int64_t q0 = first; q0 < total4; q0 += 4 * stride) {
                float4 g[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t q = q0 + u * stride;
                    if (q < total4) {
                        const int64_t i = (4 * q) / d, j = 4 * q - i * d;
                        g[u] = *reinterpret_cast<const float4*>(Gs + i * ldgs + j);
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t q = q0 + u * stride;
                    if (q < total4) {
                        const int64_t i = (4 * q) / d, j = 4 * q - i * d;
                        float4 t;
                        t.x = a1 * g[u].x - (i == j ? 1.f : 0.f);
                        t.y = a1 * g[u].y - (i == j + 1 ? 1.f : 0.f);
                        t.z = a1 * g[u].z - (i == j + 2 ? 1.f : 0.f);
                        t.w = a1 * g[u].w - (i == j + 3 ? 1.f : 0.f);
                        *reinterpret_cast<float4*>(T1s + 4 * q) = t;
                    }
                }
            }
        } else {
            const int64_t total = (int64_t)d * d;
            for (int64_t p = first; p < total; p += stride) {
                const int64_t i = p / d, j = p - i * d;
                T1s[p] = a1 * Gs[i * ldgs + j] - (i == j ? 1.f : 0.f);
            }
        }
        return;
    }
    if (coeffs) {
        // caller-given coefficients (another polynomial design for this Lambda)
        for (int k = threadIdx.x; k < K; k += blockDim.x) scal[SC_COEF + k] = Lam > 0.0 ? coeffs[k] : 0.0;
    } else if (K <= kCoefLds) {
        // k theta_l = pi k (2l + 1) / (2K): only the 4K angles pi m / (2K), m = k (2l + 1)
        // mod 4K, occur, so their cosines are tabled once, h is evaluated once per node,
        // and each c_k sums its row with l ascending (the order of the definition)
        __shared__ double ctab[4 * kCoefLds];
        __shared__ double hval[kCoefLds];
        const double pi = 3.14159265358979323846;
        const int M4 = 4 * K;
        for (int m = threadIdx.x; m < M4; m += blockDim.x) ctab[m] = cos(pi * m / (2.0 * K));
        for (int l = threadIdx.x; l < K; l += blockDim.x) {
            const double th = pi * (l + 0.5) / K;
            hval[l] = Lam > 0.0 ? shrink_h(sp, 0.5 * Lam * (cos(th) + 1.0)) : 0.0;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            double acc = 0.0;
            int idx = k;                       // k (2l + 1) mod 4K at l = 0
            const int step = (2 * k) % M4;
            for (int l = 0; l < K; ++l) {
                acc += ctab[idx] * hval[l];
                idx += step;
                if (idx >= M4) idx -= M4;
            }
            scal[SC_COEF + k] = Lam > 0.0 ? 2.0 / K * acc * damping_factor(damping, K, k) : 0.0;
        }
    } else {
        for (int k = threadIdx.x; k < K; k += blockDim.x)
            scal[SC_COEF + k] = cheb_coeff(sp, Lam, K, k) * damping_factor(damping, K, k);
    }
    if (mode == 0 && warm_out && sT >= 1) {
        // v_T = w_{T-1} / ||w_{T-1}||; w_{T-1} sits in buffer (T-1) % 2
        const double* src = ((sT - 1) & 1) ? wbuf1 : wbuf0;
        const double inv = 1.0 / sqrt(scal[pw_w2 + sT - 1]);
        for (int i = threadIdx.x; i < d; i += blockDim.x) warm_out[i] = src[i] * inv;
    }
    if (ps_out >= 0) {
        __syncthreads();   // every c_k stored
        ps_coeff_block(K, ps_s, (K + ps_s - 1) / ps_s, scal, ps_out);
    }
}

// K == 1: Y = c_0/2 X.
__global__ void scale_copy_kernel(int m, int n, const float* X, int64_t ldx, float* Y, int64_t ldy,
                                  const double* scal) {
    const float c = (float)(0.5 * scal[SC_COEF]);
    const int64_t total = (int64_t)m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        Y[i * ldy + j] = c * X[i * ldx + j];
    }
}

// Matrix-polynomial route (baby steps / giant steps in the Chebyshev basis).
// p(x) = c_0/2 + sum_{k>=1} c_k T_k(x) is rewritten as
//   p(x) = sum_{j<J} R_j(x) T_j(y),  y = T_s(x),  R_j = sum_{i<s} r_{j,i} T_i(x),
// using T_j(T_s(x)) = T_{js}(x) and T_i T_{js} = (T_{js+i} + T_{js-i}) / 2: from
// the highest degree down, r_{j,i} = 2 w_{js+i} and w_{js-i} -= w_{js+i} (i >= 1),
// r_{j,0} = w_{js}, r_{0,i} = w_i.  One thread, FP64; r is written row by row.
__device__ inline void ps_coeff_block(int K, int s, int J, double* scal, int out) {
    __shared__ double w[kPsMaxS * kPsMaxS + kPsMaxS];
    const int n = J * s;   // <= K + s - 1 <= 271
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        w[k] = k < K ? scal[SC_COEF + k] * (k == 0 ? 0.5 : 1.0) : 0.0;
    __syncthreads();
    // in place: entry (j, i) of r lives at w[j s + i]; rows from the last down, the
    // s - 1 updates of a row in parallel (their sources lie in row j and their
    // targets w[j s - i] are distinct entries of row j - 1)
    for (int j = J - 1; j >= 1; --j) {
        const int i = (int)threadIdx.x + 1;
        if (i < s) {
            const int k = j * s + i;
            const double v = w[k];
            w[k] = 2.0 * v;
            w[j * s - i] -= v;
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x) scal[out + k] = w[k];
}

__global__ void ps_coeff_kernel(int K, int s, int J, double* scal, int out) { ps_coeff_block(K, s, J, scal, out); }

// T1 = (2 / Lambda) G - I, d x d (G with pitch ldg, T1 with pitch d).
__global__ void ps_shift_kernel(int d, const float* G, int64_t ldg, float* T1, const double* scal) {
    const float a1 = (float)scal[SC_A1];
    const int64_t total = (int64_t)d * d;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = p / d, j = p - i * d;
        T1[p] = a1 * G[i * ldg + j] - (i == j ? 1.f : 0.f);
    }
}

// A-posteriori check of the matrix-polynomial route: the Gram-weighted means
//   mu_q = <G, T_q(Ghat)>_F / tr G = sum_i lambda_i T_q(x_i) / sum_i lambda_i,  q = 2..s,
// over the baby steps already formed (T_q at T1 + (q - 1) d^2, pitch d).  With
// Lambda >= lambda_max every x_i = 2 lambda_i / Lambda - 1 lies in [-1, 1], so
// |T_q(x_i)| <= 1 and mu_q <= 1; a bound below lambda_max puts the top eigenvalue,
// which carries the largest weight, beyond 1, where T_q grows like cosh.  Per
// workgroup FP64 partials of <G, T_q> at part[(q - 2) kPsCheckWg + b] (grid
// kPsCheckWg, fixed element split, so the sums do not depend on scheduling).
__global__ void ps_check_kernel(int d, const float* G, int64_t ldg, const float* T1, int s, double* part) {
    __shared__ double red[16];
    const int64_t dd = (int64_t)d * d;
    double acc[kPsMaxS];
#pragma unroll
    for (int q = 0; q < kPsMaxS; ++q) acc[q] = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < dd; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = p / d, j = p - i * d;
        const double g = G[i * ldg + j];
#pragma unroll
        for (int q = 2; q < kPsMaxS + 1; ++q)
            if (q <= s) acc[q - 1] += g * (double)T1[(int64_t)(q - 1) * dd + p];
    }
    for (int q = 2; q <= s; ++q) {
        const double v = block_sum(acc[q - 1], red);
        if (threadIdx.x == 0) part[(q - 2) * kPsCheckWg + blockIdx.x] = v;
    }
}

// R_j = r_{j,0} I + sum_{q=1}^{s-1} r_{j,q} T_q for every j < J in one pass: each
// element of T_1..T_{s-1} is read once (T_q at T1 + (q - 1) d^2, pitch d) and R_j
// goes to R + j d^2.  Four consecutive elements per thread (16-byte accesses when
// d % 4 == 0).  MAXS >= s: the register block of the T_q (launched with 16, 24
// or 32, the smallest that holds s).
template <int MAXS>
__global__ void ps_lincomb_kernel(int d, int s, int J, const float* T1, const double* scal, int roff, float* R) {
    __shared__ float rc[MAXS * MAXS];
    for (int k = threadIdx.x; k < J * s; k += blockDim.x) rc[k] = (float)scal[roff + k];
    __syncthreads();
    const int64_t dd = (int64_t)d * d;
    const bool vec = (d & 3) == 0;
    const int64_t nq = (dd + 3) / 4;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < nq; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p0 = 4 * g;
        f32x4 t[MAXS];
#pragma unroll
        for (int q = 1; q < MAXS; ++q) {
            t[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
            if (q < s) {
                const float* src = T1 + (int64_t)(q - 1) * dd + p0;
                if (vec) {
                    t[q] = *reinterpret_cast<const f32x4*>(src);
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (p0 + e < dd) t[q][e] = src[e];
                }
            }
        }
        // which of the four entries lie on the diagonal (with d % 4 == 0 they share
        // one row: a single division, 32-bit where d^2 allows)
        bool on_diag[4];
        if (vec) {
            int64_t r0;
            if (dd <= 0x7fffffff)
                r0 = (int64_t)((uint32_t)p0 / (uint32_t)d);
            else
                r0 = p0 / d;
            const int64_t c0 = p0 - r0 * d;
#pragma unroll
            for (int e = 0; e < 4; ++e) on_diag[e] = r0 == c0 + e;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t p = p0 + e;
                on_diag[e] = p / d == p % d;
            }
        }
        for (int j = 0; j < J; ++j) {
            f32x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = on_diag[e] ? rc[j * s] : 0.f;
#pragma unroll
            for (int q = 1; q < MAXS; ++q)
                if (q < s) v += rc[j * s + q] * t[q];
            float* dst = R + (int64_t)j * dd + p0;
            if (vec) {
                *reinterpret_cast<f32x4*>(dst) = v;
            } else {
                for (int e = 0; e < 4; ++e)
                    if (p0 + e < dd) dst[e] = v[e];
            }
        }
    }
}

}  // namespace cpa
