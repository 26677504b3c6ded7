// Shrinkage response and Chebyshev coefficients in FP64, compiled for both the
// host (cpa_chebyshev_coeffs) and the device (per-call coefficient kernel, so a
// bound computed on the GPU never has to travel to the host).
//
// Response family: Sec. IV-A, eq. (filter_response_ours).  Coefficients:
// Sec. III-A, eq. (chebychev_coeff_shifted) -- the discrete cosine sums of h at
// the K Chebyshev-Gauss nodes theta_l = pi (l - 1/2) / K mapped to [0, Lambda].
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace cpa {

struct ShrinkParams {
    int kind;        // 0 soft, 1 hard, 2 weighted constant, 3 weighted function
    double tau;
    double w_c;
    double w_sigma;
    double w_eps;
};

// h(x) on the Gram's eigenvalue x = s^2.  Strict threshold on sqrt(x); x <= 0 -> 0.
__host__ __device__ inline double shrink_h(const ShrinkParams& p, double x) {
    if (!(x > 0.0)) return 0.0;
    const double s = sqrt(x);
    double w, t;
    switch (p.kind) {
        case 0:
        case 2: w = p.tau; t = p.tau; break;
        case 1: w = 0.0; t = p.tau; break;
        default: {
            const double e = x - p.w_sigma;
            w = p.w_c / (sqrt(e > 0.0 ? e : 0.0) + p.w_eps);
            t = w;
        }
    }
    return s > t ? (s - w) / s : 0.0;
}

// c_k for one k: (2/K) sum_{l=1..K} cos(k theta_l) h(Lambda/2 (cos theta_l + 1)),
// summed with l ascending.
__host__ __device__ inline double cheb_coeff(const ShrinkParams& p, double Lambda, int K, int k) {
    if (!(Lambda > 0.0)) return 0.0;
    const double pi = 3.14159265358979323846;
    double acc = 0.0;
    for (int l = 1; l <= K; ++l) {
        const double th = pi * (l - 0.5) / K;
        const double x = 0.5 * Lambda * (cos(th) + 1.0);
        acc += cos(k * th) * shrink_h(p, x);
    }
    return 2.0 / K * acc;
}

// Optional damping factor g_k of c_k (not in the paper; the kernel polynomial
// method's factors for degree N = K - 1): kind 0 none, 1 Jackson
// ((N - k + 1) cos(pi k/(N+1)) + sin(pi k/(N+1)) cot(pi/(N+1))) / (N + 1),
// 2 Lanczos sin(pi k/(N+1)) / (pi k/(N+1)); g_0 = 1.
__host__ __device__ inline double damping_factor(int kind, int K, int k) {
    if (kind == 0 || k == 0 || K < 2) return 1.0;
    const double pi = 3.14159265358979323846;
    const double n1 = (double)K;   // N + 1
    const double a = pi * k / n1;
    if (kind == 1) return ((n1 - k) * cos(a) + sin(a) / tan(pi / n1)) / n1;
    return sin(a) / a;
}

}  // namespace cpa
