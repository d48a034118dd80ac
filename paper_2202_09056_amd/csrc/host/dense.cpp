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

// The three cubic loops of the inverse.  Each is built twice, for the
// baseline x86-64 instruction set and for x86-64-v3 (AVX2 with fused
// multiply-add), and the loader picks the one the processor runs.  They
// work on register tiles of 4 x 8 entries held as eight 4-wide vectors (on
// the baseline build each vector is two SSE registers), so every step issues
// eight independent multiply-adds.  Within one build every entry's sum runs
// over its index range in a fixed order, so the result does not depend on
// the thread count (the build with fused multiply-adds differs from the
// baseline one in the last bits).
#define SAAMG_DENSE_CLONES __attribute__((target_clones("arch=x86-64-v3", "default")))

typedef double d4 __attribute__((vector_size(32)));
typedef double d4u __attribute__((vector_size(32), aligned(8)));  // unaligned access

// (no helper functions taking or returning d4: on the baseline build that
// would change the calling convention; a scalar operand is broadcast)
#define LOAD4(p) (*(const d4u *)(p))

constexpr int kGroup = 32;  // columns of W per forward-substitution group

// a_ij -= sum_p L_ip L_jp over panel columns k0..k0+kb-1 for the lower
// triangle of the trailing rows (k1 = k0 + kb on): row blocks [bi0, bi1) of
// four rows, column blocks of eight; pt holds the panel transposed,
// pt[p * ldp + jj] = L[k1 + jj][k0 + p], zero beyond the last row.
SAAMG_DENSE_CLONES
static void trailing_update(double *a, int n, int k0, int kb, int rest, const double *pt, int ldp, int bi0,
                            int bi1) {
    const int k1 = k0 + kb;
    for (int bi = bi0; bi < bi1; ++bi) {
        const double *l[4];
        for (int r = 0; r < 4; ++r) l[r] = &a[(size_t)(k1 + std::min(4 * bi + r, rest - 1)) * n + k0];
        const int nbj = (4 * bi + 3) / 8 + 1;
        for (int bj = 0; bj < nbj; ++bj) {
            d4 acc[4][2] = {};
            for (int p = 0; p < kb; ++p) {
                const double *v = &pt[(size_t)p * ldp + 8 * bj];
                const d4 v0 = LOAD4(v), v1 = LOAD4(v + 4);
                for (int r = 0; r < 4; ++r) {
                    const double lr = l[r][p];
                    acc[r][0] += lr * v0;
                    acc[r][1] += lr * v1;
                }
            }
            for (int r = 0; r < 4; ++r) {
                const int ii = 4 * bi + r;
                if (ii >= rest) break;
                double *row = &a[(size_t)(k1 + ii) * n + k1];
                for (int c = 0; c < 8 && 8 * bj + c <= ii; ++c) row[8 * bj + c] -= acc[r][c / 4][c % 4];
            }
        }
    }
}

// Columns j0..j0+31 of W = L^{-1} by forward substitution into
// wg[(i - j0) * 32 + c] for rows i = j0..n-1 (L is the lower triangle of a;
// columns past n come out zero).
SAAMG_DENSE_CLONES
static void forward_group(const double *a, int n, int j0, double *wg) {
    for (int i = j0; i < n; ++i) {
        d4 s[8];
        for (int q = 0; q < 8; ++q)
            for (int e = 0; e < 4; ++e) s[q][e] = (i == j0 + 4 * q + e) ? 1.0 : 0.0;
        const double *li = &a[(size_t)i * n];
        for (int k = j0; k < i; ++k) {
            const double lk = li[k];
            const double *w = &wg[(size_t)(k - j0) * kGroup];
            for (int q = 0; q < 8; ++q) s[q] -= lk * LOAD4(w + 4 * q);
        }
        const double d = li[i];
        double *w = &wg[(size_t)(i - j0) * kGroup];
        for (int q = 0; q < 8; ++q) *(d4u *)(w + 4 * q) = s[q] / d;
    }
}

// (W^T W)_ij = sum_{k >= i} W_ki W_kj for the lower triangle: row blocks
// [bi0, bi1) of four rows, column blocks of eight.  wg[g] holds
// W[k][32g..32g+31] for k = 32g..n-1 (row k at (k - 32g) * 32).
SAAMG_DENSE_CLONES
static void gram_lower(double *a, int n, const double *const *wg, int bi0, int bi1) {
    for (int bi = bi0; bi < bi1; ++bi) {
        const int k0 = 4 * bi;
        const int gi = k0 / kGroup;
        const double *wi = wg[gi] + (size_t)(k0 - kGroup * gi) * kGroup + (k0 % kGroup);
        const int nbj = (4 * bi + 3) / 8 + 1;
        for (int bj = 0; bj < nbj; ++bj) {
            const int j0 = 8 * bj, gj = j0 / kGroup;
            const double *wj = wg[gj] + (size_t)(k0 - kGroup * gj) * kGroup + (j0 % kGroup);
            d4 acc[4][2] = {};
            for (int k = k0; k < n; ++k) {
                const double *u = wi + (size_t)(k - k0) * kGroup;
                const double *v = wj + (size_t)(k - k0) * kGroup;
                const d4 v0 = LOAD4(v), v1 = LOAD4(v + 4);
                for (int r = 0; r < 4; ++r) {
                    const double ur = u[r];
                    acc[r][0] += ur * v0;
                    acc[r][1] += ur * v1;
                }
            }
            for (int r = 0; r < 4; ++r) {
                const int i = k0 + r;
                if (i >= n) break;
                for (int c = 0; c < 8 && j0 + c <= i; ++c) a[(size_t)i * n + j0 + c] = acc[r][c / 4][c % 4];
            }
        }
    }
}

// Splits [0, nblk) into T contiguous ranges of about equal cost, the cost
// of block b being cost(b); the ranges depend on T only through where they
// are cut, never through what a block computes.
template <typename F>
static std::vector<int> balanced_split(int nblk, int T, F cost) {
    std::vector<double> acc(nblk + 1, 0.0);
    for (int b = 0; b < nblk; ++b) acc[b + 1] = acc[b] + cost(b);
    std::vector<int> cut(T + 1, nblk);
    cut[0] = 0;
    int b = 0;
    for (int t = 1; t < T; ++t) {
        const double target = acc[nblk] * t / T;
        while (b < nblk && acc[b + 1] <= target) ++b;
        cut[t] = b;
    }
    return cut;
}

static int task_count(int nthreads, int nblk) { return std::max(1, std::min(nthreads, nblk)); }

// In-place lower Cholesky of a row-major symmetric n x n matrix, right-looking
// with NB-wide panels.  Every entry is formed by one thread in a fixed order,
// so the factor does not depend on the thread count.  The trailing update
// reads the panel in transposed form so the eight columns of a tile are
// adjacent.
static void cholesky_lower(std::vector<double> &a, int n, int nthreads) {
    const int NB = 96;
    std::vector<double> pt;
    for (int k0 = 0; k0 < n; k0 += NB) {
        const int kb = std::min(NB, n - k0);
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
        const int k1 = k0 + kb, rest = n - k1;
        if (rest <= 0) break;
        // panel rows below the diagonal block, and their transposed copy
        // (zero-padded to whole column blocks of eight)
        const int nbr = (rest + 3) / 4, ldp = 8 * ((rest + 7) / 8);
        pt.assign((size_t)kb * ldp, 0.0);
        {
            const int T = task_count(nthreads, nbr);
            parallel_tasks(T, [&](int t) {
                const int64_t lo = (int64_t)rest * t / T, hi = (int64_t)rest * (t + 1) / T;
                for (int64_t ii = lo; ii < hi; ++ii) {
                    const size_t i = (size_t)(k1 + ii);
                    for (int k = k0; k < k1; ++k) {
                        double s = a[i * n + k];
                        for (int p = k0; p < k; ++p) s -= a[i * n + p] * a[(size_t)k * n + p];
                        a[i * n + k] = s / a[(size_t)k * n + k];
                    }
                    for (int p = 0; p < kb; ++p) pt[(size_t)p * ldp + ii] = a[i * n + k0 + p];
                }
            });
        }
        // trailing update a_ij -= sum_p L_ip L_jp (j <= i); row block bi
        // holds about bi / 2 + 1 tiles
        const int T = task_count(nthreads, nbr);
        const std::vector<int> cut = balanced_split(nbr, T, [](int b) { return (double)((4 * b + 3) / 8 + 1); });
        parallel_tasks(T, [&](int t) { trailing_update(a.data(), n, k0, kb, rest, pt.data(), ldp, cut[t], cut[t + 1]); });
    }
}

// A^{-1} = W^T W with W = L^{-1}.  W is formed by forward substitution in
// groups of 32 columns (each group's rows from its first column on, in a
// buffer of its own; the groups spread over threads), then the product runs
// over 4 x 8 tiles of the lower triangle reading those buffers.  The sums of
// a group's columns, and of a tile's entries, start at the group's or the
// tile's first row: the extra terms meet entries of W above its diagonal,
// which are zero and leave the sums unchanged.
void dense_spd_inverse(std::vector<double> &a, int n, int nthreads) {
    cholesky_lower(a, n, nthreads);
    const int ng = (n + kGroup - 1) / kGroup;
    std::vector<std::vector<double>> wg(ng);
    std::vector<const double *> wptr(ng);
    for (int g = 0; g < ng; ++g) {
        wg[g].assign((size_t)(n - kGroup * g) * kGroup, 0.0);
        wptr[g] = wg[g].data();
    }
    {
        const int T = task_count(nthreads, ng);
        const std::vector<int> cut = balanced_split(ng, T, [&](int g) {
            const double m = n - (double)kGroup * g;
            return m * m;
        });
        parallel_tasks(T, [&](int t) {
            for (int g = cut[t]; g < cut[t + 1]; ++g) forward_group(a.data(), n, kGroup * g, wg[g].data());
        });
    }
    // (A^{-1})_ij = sum_{k >= i} W_ki W_kj for j <= i, then mirrored
    {
        const int nbi = (n + 3) / 4;
        const int T = task_count(nthreads, nbi);
        const std::vector<int> cut =
            balanced_split(nbi, T, [&](int b) { return (double)((4 * b + 3) / 8 + 1) * (double)(n - 4 * b); });
        parallel_tasks(T, [&](int t) { gram_lower(a.data(), n, wptr.data(), cut[t], cut[t + 1]); });
    }
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
