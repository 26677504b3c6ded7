// Host FP64 polynomial designs on [0, Lambda] other than Chebyshev interpolation,
// for the comparison of Sec. IV-B (least squares and minimax,
// eq. (l_p_norm_for_approximation)).  Each returns coefficients in the shrink's
// convention p(x) = c_0/2 + sum_{k>=1} c_k T_k(2x/Lambda - 1), so the device
// evaluation runs them unchanged (opts.coeffs).
//
//   least squares: minimise sum_i (h(x_i) - p(x_i))^2 over the n uniform samples
//     x_i = Lambda i / (n - 1), by Householder QR of the n x K Chebyshev matrix
//     (the minimiser is unique and basis independent; the Chebyshev basis keeps the
//     problem well conditioned where the paper's monomial Vandermonde matrix is not);
//   minimax: minimise max_i |h(x_i) - p(x_i)| over the grid
//     x_i = (Lambda/2)(1 - cos(pi i / (n - 1))) by the Remez exchange: on a
//     reference of K + 1 grid points solve p(x_j) + (-1)^j E = h(x_j) (with the
//     signs of the last error), move the reference onto the largest error of each
//     run of one sign, keeping K + 1 alternating points, until the largest grid
//     error is within a relative `tol` of |E|.
#pragma once

#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "shrink_fn.hpp"

namespace cpa {
namespace design {

constexpr double kPi = 3.14159265358979323846;

// Rows of T_0..T_{K-1} at t (cos form; t clamped to [-1, 1]).
inline void cheb_row(double t, int K, double* row) {
    const double th = acos(t < -1.0 ? -1.0 : (t > 1.0 ? 1.0 : t));
    for (int k = 0; k < K; ++k) row[k] = cos(k * th);
}

inline double eval_plain(const double* a, const double* row, int K) {
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += a[k] * row[k];
    return s;
}

// Least squares: returns the plain coefficients a (p = sum a_k T_k) in a[0..K-1]
// and the largest sample residual.  Requires n >= K >= 1.
inline double lsq(const ShrinkParams& sp, double Lambda, int K, int n, double* a) {
    // column-major n x K matrix and right-hand side
    std::vector<double> V((size_t)n * K), b(n), row(K);
    for (int i = 0; i < n; ++i) {
        const double x = Lambda * i / (n - 1);
        cheb_row(2.0 * x / Lambda - 1.0, K, row.data());
        for (int k = 0; k < K; ++k) V[(size_t)k * n + i] = row[k];
        b[i] = shrink_h(sp, x);
    }
    std::vector<double> h = b;
    // Householder QR, applied to b as it goes
    std::vector<double> rdiag(K);
    for (int j = 0; j < K; ++j) {
        double* col = &V[(size_t)j * n];
        double nrm = 0.0;
        for (int i = j; i < n; ++i) nrm += col[i] * col[i];
        nrm = sqrt(nrm);
        const double alpha = col[j] > 0.0 ? -nrm : nrm;   // R_jj, sign opposite to the pivot
        rdiag[j] = alpha;
        if (nrm == 0.0) continue;
        col[j] -= alpha;                                  // v = x - alpha e_1
        const double vnorm2 = -2.0 * alpha * col[j];      // ||v||^2 = 2 nrm (nrm + |x_j|)
        if (vnorm2 == 0.0) continue;
        auto reflect = [&](double* y) {
            double dot = 0.0;
            for (int i = j; i < n; ++i) dot += col[i] * y[i];
            const double f = 2.0 * dot / vnorm2;
            for (int i = j; i < n; ++i) y[i] -= f * col[i];
        };
        for (int c = j + 1; c < K; ++c) reflect(&V[(size_t)c * n]);
        reflect(b.data());
    }
    // R a = (Q^T b)[0..K-1]; R's off-diagonal entries sit above the diagonal of V
    for (int j = K - 1; j >= 0; --j) {
        double s = b[j];
        for (int c = j + 1; c < K; ++c) s -= V[(size_t)c * n + j] * a[c];
        a[j] = rdiag[j] != 0.0 ? s / rdiag[j] : 0.0;
    }
    double emax = 0.0;
    for (int i = 0; i < n; ++i) {
        const double x = Lambda * i / (n - 1);
        cheb_row(2.0 * x / Lambda - 1.0, K, row.data());
        emax = std::max(emax, fabs(h[i] - eval_plain(a, row.data(), K)));
    }
    return emax;
}

// Dense (K+1) x (K+1) solve by Gaussian elimination with partial pivoting
// (row-major A, overwritten; x receives the solution).  False if singular.
inline bool solve(std::vector<double>& A, std::vector<double>& rhs, int N, double* x) {
    for (int c = 0; c < N; ++c) {
        int p = c;
        for (int r = c + 1; r < N; ++r)
            if (fabs(A[(size_t)r * N + c]) > fabs(A[(size_t)p * N + c])) p = r;
        if (A[(size_t)p * N + c] == 0.0) return false;
        if (p != c) {
            for (int k = 0; k < N; ++k) std::swap(A[(size_t)p * N + k], A[(size_t)c * N + k]);
            std::swap(rhs[p], rhs[c]);
        }
        const double inv = 1.0 / A[(size_t)c * N + c];
        for (int r = c + 1; r < N; ++r) {
            const double f = A[(size_t)r * N + c] * inv;
            if (f == 0.0) continue;
            for (int k = c; k < N; ++k) A[(size_t)r * N + k] -= f * A[(size_t)c * N + k];
            rhs[r] -= f * rhs[c];
        }
    }
    for (int r = N - 1; r >= 0; --r) {
        double s = rhs[r];
        for (int k = r + 1; k < N; ++k) s -= A[(size_t)r * N + k] * x[k];
        x[r] = s / A[(size_t)r * N + r];
    }
    return true;
}

// Minimax by the Remez exchange: plain coefficients in a[0..K-1]; returns the
// largest grid error (= |E| within tol at convergence), or -1 if a reference
// system was singular.  Requires n >= K + 1.
inline double minimax(const ShrinkParams& sp, double Lambda, int K, int n, int max_iter, double tol, double* a) {
    std::vector<double> x(n), h(n), T((size_t)n * K), e(n);
    double hscale = 1.0;
    for (int i = 0; i < n; ++i) {
        x[i] = 0.5 * Lambda * (1.0 - cos(kPi * i / (n - 1)));
        cheb_row(2.0 * x[i] / Lambda - 1.0, K, &T[(size_t)i * K]);
        h[i] = shrink_h(sp, x[i]);
        hscale = std::max(hscale, fabs(h[i]));
    }
    // start: the grid points nearest the extrema of T_K, i.e. nearest (Lambda/2)(1 - cos(pi j / K))
    std::vector<int> ref(K + 1);
    for (int j = 0; j <= K; ++j) {
        const double target = 0.5 * Lambda * (1.0 - cos(kPi * j / K));
        const int i0 = (int)(std::lower_bound(x.begin(), x.end(), target) - x.begin());
        int best = std::min(i0, n - 1);
        if (i0 > 0 && fabs(x[i0 - 1] - target) <= fabs(x[best] - target)) best = i0 - 1;
        ref[j] = best;
    }
    for (int j = 1; j <= K; ++j)
        if (ref[j] <= ref[j - 1]) return -2.0;   // grid too coarse for K + 1 distinct points
    std::vector<double> sign(K + 1), A((size_t)(K + 1) * (K + 1)), rhs(K + 1), sol(K + 1);
    for (int j = 0; j <= K; ++j) sign[j] = (j % 2) ? -1.0 : 1.0;
    const int N = K + 1;
    double emax = 0.0;
    for (int it = 0; it < max_iter; ++it) {
        for (int j = 0; j < N; ++j) {
            for (int k = 0; k < K; ++k) A[(size_t)j * N + k] = T[(size_t)ref[j] * K + k];
            A[(size_t)j * N + K] = sign[j];
            rhs[j] = h[ref[j]];
        }
        if (!solve(A, rhs, N, sol.data())) return -1.0;
        for (int k = 0; k < K; ++k) a[k] = sol[k];
        const double E = fabs(sol[K]);
        emax = 0.0;
        for (int i = 0; i < n; ++i) {
            e[i] = h[i] - eval_plain(a, &T[(size_t)i * K], K);
            emax = std::max(emax, fabs(e[i]));
        }
        if (emax <= E * (1.0 + tol) + 1e-14 * hscale) break;
        // largest |e| of each maximal run of one sign (zero counts as positive)
        std::vector<int> cand;
        int start = 0;
        for (int i = 1; i <= n; ++i) {
            if (i == n || (e[i] >= 0.0) != (e[start] >= 0.0)) {
                int best = start;
                for (int r = start + 1; r < i; ++r)
                    if (fabs(e[r]) > fabs(e[best])) best = r;
                cand.push_back(best);
                start = i;
            }
        }
        // keep K + 1 of them: drop the smaller end until the count fits
        size_t lo = 0, hi = cand.size();
        while (hi - lo > (size_t)N) {
            if (fabs(e[cand[lo]]) < fabs(e[cand[hi - 1]])) ++lo;
            else --hi;
        }
        if (hi - lo < (size_t)N) break;
        bool same = true;
        for (int j = 0; j < N; ++j) same = same && ref[j] == cand[lo + j];
        if (same) break;
        for (int j = 0; j < N; ++j) {
            ref[j] = cand[lo + j];
            sign[j] = e[ref[j]] >= 0.0 ? 1.0 : -1.0;
        }
    }
    return emax;
}

}  // namespace design
}  // namespace cpa
