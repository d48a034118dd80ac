// Scalar CSR kernels of the hybrid setup (Section 3: the hierarchy built in
// scalar arithmetic and every matrix converted to the 3x3 block format
// afterwards, the construction behind the paper's "NS Hybrid" solvers),
// FP64 on the host: conversion between scalar CSR and BSR3, the sparse
// product and transpose in scalar form.
#include <algorithm>
#include <cstring>
#include <vector>

#include "setup_internal.hpp"

namespace saamg {

Csr unblock(const Bsr3 &A, int nthreads) {
    Csr S;
    S.rows = 3 * A.rows;
    S.cols = 3 * A.cols;
    S.ptr.assign((size_t)S.rows + 1, 0);
    // count, then fill each scalar row (block columns are sorted, so each row comes out sorted)
    parallel_for(A.rows, nthreads, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i)
            for (int r = 0; r < 3; ++r) {
                int64_t c = 0;
                for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                    for (int q = 0; q < 3; ++q) c += A.val[9 * k + 3 * r + q] != 0.0;  // exact zeros not stored
                S.ptr[3 * i + r + 1] = c;
            }
    });
    for (int32_t i = 0; i < S.rows; ++i) S.ptr[i + 1] += S.ptr[i];
    S.col.resize(S.ptr[S.rows]);
    S.val.resize(S.ptr[S.rows]);
    parallel_for(A.rows, nthreads, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i)
            for (int r = 0; r < 3; ++r) {
                int64_t d = S.ptr[3 * i + r];
                for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                    for (int q = 0; q < 3; ++q) {
                        const double v = A.val[9 * k + 3 * r + q];
                        if (v == 0.0) continue;
                        S.col[d] = 3 * A.col[k] + q;
                        S.val[d++] = v;
                    }
            }
    });
    return S;
}

Bsr3 reblock(const Csr &S, int nthreads) {
    if (S.rows % 3 || S.cols % 3) throw AmgError{AMG_ERR_ARG, "internal: scalar size not a multiple of 3"};
    Bsr3 B;
    B.rows = S.rows / 3;
    B.cols = S.cols / 3;
    B.ptr.assign((size_t)B.rows + 1, 0);
    // block columns of block row I: the merged block columns of its three scalar rows
    auto block_cols = [&](int32_t I, std::vector<int32_t> &cols) {
        cols.clear();
        for (int r = 0; r < 3; ++r)
            for (int64_t k = S.ptr[3 * I + r]; k < S.ptr[3 * I + r + 1]; ++k) cols.push_back(S.col[k] / 3);
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    };
    parallel_for(B.rows, nthreads, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> cols;
        for (int64_t I = lo; I < hi; ++I) {
            block_cols((int32_t)I, cols);
            B.ptr[I + 1] = (int64_t)cols.size();
        }
    });
    for (int32_t I = 0; I < B.rows; ++I) B.ptr[I + 1] += B.ptr[I];
    B.col.resize(B.ptr[B.rows]);
    B.val.assign(9 * (size_t)B.ptr[B.rows], 0.0);
    parallel_for(B.rows, nthreads, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> cols;
        for (int64_t I = lo; I < hi; ++I) {
            block_cols((int32_t)I, cols);
            const int64_t base = B.ptr[I];
            std::copy(cols.begin(), cols.end(), B.col.begin() + base);
            for (int r = 0; r < 3; ++r)
                for (int64_t k = S.ptr[3 * I + r]; k < S.ptr[3 * I + r + 1]; ++k) {
                    const int32_t J = S.col[k] / 3;
                    const int64_t q = base + (std::lower_bound(cols.begin(), cols.end(), J) - cols.begin());
                    B.val[9 * q + 3 * r + S.col[k] % 3] = S.val[k];
                }
        }
    });
    return B;
}

// C = A B row by row with a dense accumulator per thread (Gustavson); the
// columns of each row come out sorted.
Csr csr_multiply(const Csr &A, const Csr &B, int nthreads) {
    Csr C;
    C.rows = A.rows;
    C.cols = B.cols;
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads, A.rows / 512 + 1));
    struct Part {
        std::vector<int32_t> col;
        std::vector<double> val;
        std::vector<int64_t> cnt;
    };
    std::vector<Part> parts(T);
    std::vector<int64_t> rb(T + 1);
    for (int t = 0; t <= T; ++t) rb[t] = (int64_t)A.rows * t / T;
    parallel_tasks(T, [&](int t) {
        Part &p = parts[t];
        std::vector<double> acc(B.cols, 0.0);
        std::vector<int64_t> mark(B.cols, -1);
        std::vector<int32_t> touched;
        p.cnt.resize(rb[t + 1] - rb[t]);
        for (int64_t i = rb[t]; i < rb[t + 1]; ++i) {
            touched.clear();
            for (int64_t ka = A.ptr[i]; ka < A.ptr[i + 1]; ++ka) {
                const int32_t k = A.col[ka];
                const double a = A.val[ka];
                for (int64_t kb = B.ptr[k]; kb < B.ptr[k + 1]; ++kb) {
                    const int32_t j = B.col[kb];
                    if (mark[j] != i) {
                        mark[j] = i;
                        touched.push_back(j);
                        acc[j] = 0.0;
                    }
                    acc[j] += a * B.val[kb];
                }
            }
            std::sort(touched.begin(), touched.end());
            for (int32_t j : touched) {
                p.col.push_back(j);
                p.val.push_back(acc[j]);
            }
            p.cnt[i - rb[t]] = (int64_t)touched.size();
        }
    });
    C.ptr.assign((size_t)A.rows + 1, 0);
    for (int t = 0; t < T; ++t)
        for (int64_t i = rb[t]; i < rb[t + 1]; ++i) C.ptr[i + 1] = parts[t].cnt[i - rb[t]];
    for (int64_t i = 0; i < A.rows; ++i) C.ptr[i + 1] += C.ptr[i];
    C.col.resize(C.ptr[A.rows]);
    C.val.resize(C.ptr[A.rows]);
    parallel_tasks(T, [&](int t) {
        const int64_t off = C.ptr[rb[t]];
        std::copy(parts[t].col.begin(), parts[t].col.end(), C.col.begin() + off);
        std::copy(parts[t].val.begin(), parts[t].val.end(), C.val.begin() + off);
    });
    return C;
}

Csr csr_transpose(const Csr &A) {
    Csr T;
    T.rows = A.cols;
    T.cols = A.rows;
    T.ptr.assign((size_t)T.rows + 1, 0);
    for (int32_t c : A.col) ++T.ptr[c + 1];
    for (int32_t i = 0; i < T.rows; ++i) T.ptr[i + 1] += T.ptr[i];
    T.col.resize(A.col.size());
    T.val.resize(A.val.size());
    std::vector<int64_t> fill(T.ptr.begin(), T.ptr.end() - 1);
    for (int32_t i = 0; i < A.rows; ++i)  // rows in order: the transposed rows come out sorted
        for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            const int64_t q = fill[A.col[k]]++;
            T.col[q] = i;
            T.val[q] = A.val[k];
        }
    return T;
}

}  // namespace saamg
