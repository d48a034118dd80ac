// Dense FP64 helpers of the host setup:
//  * Cholesky factorisation and explicit inverse of the coarsest matrix
//    (Algorithm 1, last step: a direct solver for A_L; the inverse turns the
//    coarsest solve into one dense matrix-vector product on the GPU);
//  * Householder thin QR used for the tentative prolongation (the per-
//    aggregate factorisation B_a = Q_a R_a of the near-nullspace block).
#include <algorithm>
#include <cmath>
#include <vector>

#include "setup_internal.hpp"

namespace saamg {

// In-place lower Cholesky of a row-major symmetric n x n matrix, right-looking
// with NB-wide panels; the trailing update is split over rows across threads.
static void cholesky_lower(std::vector<double> &a, int n, int nthreads) {
    const int NB = 96;
    for (int k0 = 0; k0 < n; k0 += NB) {
        int kb = std::min(NB, n - k0);
        // diagonal block
        for (int k = k0; k < k0 + kb; ++k) {
            double d = a[(size_t)k * n + k];
            for (int p = k0; p < k; ++p) d -= a[(size_t)k * n + p] * a[(size_t)k * n + p];
            if (!(d > 0.0) || !std::isfinite(d))
                throw AmgError{AMG_ERR_NOT_SPD, "coarsest matrix is not positive definite"};
            d = std::sqrt(d);
            a[(size_t)k * n + k] = d;
            for (int i = k + 1; i < k0 + kb; ++i) {
                double s = a[(size_t)i * n + k];
                for (int p = k0; p < k; ++p) s -= a[(size_t)i * n + p] * a[(size_t)k * n + p];
                a[(size_t)i * n + k] = s / d;
            }
        }
        int rest = n - (k0 + kb);
        if (rest <= 0) break;
        // panel rows below the diagonal block
        parallel_for(rest, nthreads, [&](int64_t b, int64_t e) {
            for (int64_t ii = b; ii < e; ++ii) {
                size_t i = (size_t)(k0 + kb + ii);
                for (int k = k0; k < k0 + kb; ++k) {
                    double s = a[i * n + k];
                    for (int p = k0; p < k; ++p) s -= a[i * n + p] * a[(size_t)k * n + p];
                    a[i * n + k] = s / a[(size_t)k * n + k];
                }
            }
        });
        // trailing update of the lower triangle, balanced by area
        int64_t total = (int64_t)rest * (rest + 1) / 2;
        int T = std::max(1, nthreads);
        std::vector<int> split(T + 1, 0);
        split[T] = rest;
        for (int t = 1; t < T; ++t) {
            double target = (double)total * t / T;
            split[t] = std::min(rest, (int)std::sqrt(2.0 * target));
        }
        parallel_tasks(T, [&](int t) {
                for (int ii = split[t]; ii < split[t + 1]; ++ii) {
                    size_t i = (size_t)(k0 + kb + ii);
                    const double *li = &a[i * n + k0];
                    for (int jj = 0; jj <= ii; ++jj) {
                        size_t j = (size_t)(k0 + kb + jj);
                        const double *lj = &a[j * n + k0];
                        double s = 0.0;
                        for (int p = 0; p < kb; ++p) s += li[p] * lj[p];
                        a[i * n + j] -= s;
                    }
                }
        });
    }
}

void dense_spd_inverse(std::vector<double> &a, int n, int nthreads) {
    cholesky_lower(a, n, nthreads);
    // W = L^{-1}, stored by columns: wc[j] holds rows j..n-1 of column j
    std::vector<double> wc((size_t)n * n, 0.0);
    parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
        std::vector<double> w(n);
        for (int64_t j = b; j < e; ++j) {
            for (int i = (int)j; i < n; ++i) {
                double s = (i == j) ? 1.0 : 0.0;
                const double *li = &a[(size_t)i * n];
                for (int k = (int)j; k < i; ++k) s -= li[k] * w[k];
                w[i] = s / li[i];
            }
            std::copy(w.begin() + j, w.end(), wc.begin() + (size_t)j * n + j);
        }
    });
    // A^{-1} = W^T W
    parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i)
            for (int j = 0; j <= i; ++j) {
                int k0 = (int)std::max<int64_t>(i, j);
                const double *wi = &wc[(size_t)i * n];
                const double *wj = &wc[(size_t)j * n];
                double s = 0.0;
                for (int k = k0; k < n; ++k) s += wi[k] * wj[k];
                a[(size_t)i * n + j] = s;
            }
    });
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) a[(size_t)i * n + j] = a[(size_t)j * n + i];
}

void householder_qr(const double *a, int m, int k, double *Q, double *R) {
    std::vector<double> A(a, a + (size_t)m * k);  // column-major copy
    std::vector<double> V((size_t)m * k, 0.0);     // Householder vectors
    std::vector<double> beta(k, 0.0);
    for (int j = 0; j < k; ++j) {
        double *x = &A[(size_t)j * m];
        double nrm = 0.0;
        for (int i = j; i < m; ++i) nrm += x[i] * x[i];
        nrm = std::sqrt(nrm);
        double *v = &V[(size_t)j * m];
        if (nrm == 0.0) {
            beta[j] = 0.0;
            continue;
        }
        double alpha = x[j] >= 0 ? -nrm : nrm;
        for (int i = j; i < m; ++i) v[i] = x[i];
        v[j] -= alpha;
        double vv = 0.0;
        for (int i = j; i < m; ++i) vv += v[i] * v[i];
        beta[j] = vv > 0 ? 2.0 / vv : 0.0;
        for (int c = j; c < k; ++c) {
            double *y = &A[(size_t)c * m];
            double s = 0.0;
            for (int i = j; i < m; ++i) s += v[i] * y[i];
            s *= beta[j];
            for (int i = j; i < m; ++i) y[i] -= s * v[i];
        }
    }
    // R (row-major k x k) and Q = H_0 ... H_{k-1} [I; 0]
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) R[r * k + c] = (c >= r) ? A[(size_t)c * m + r] : 0.0;
    for (int c = 0; c < k; ++c) {
        double *q = &Q[(size_t)c * m];
        for (int i = 0; i < m; ++i) q[i] = (i == c) ? 1.0 : 0.0;
        for (int j = k - 1; j >= 0; --j) {
            if (beta[j] == 0.0) continue;
            const double *v = &V[(size_t)j * m];
            double s = 0.0;
            for (int i = j; i < m; ++i) s += v[i] * q[i];
            s *= beta[j];
            for (int i = j; i < m; ++i) q[i] -= s * v[i];
        }
    }
    // positive diagonal of R
    for (int r = 0; r < k; ++r)
        if (R[r * k + r] < 0.0) {
            for (int c = 0; c < k; ++c) R[r * k + c] = -R[r * k + c];
            double *q = &Q[(size_t)r * m];
            for (int i = 0; i < m; ++i) q[i] = -q[i];
        }
}

}  // namespace saamg
