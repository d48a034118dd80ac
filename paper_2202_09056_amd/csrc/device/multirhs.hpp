// Multi-right-hand-side solve: k <= 32 columns stored row-major (column index
// fastest, X[i*k + j]), every operator read once per product for all columns.
#pragma once

#include "kernels.hpp"

namespace saamg {

constexpr int kMaxRhs = 32;
constexpr int kMaxMGrid = 2048;      // workgroups of a multi-column product
constexpr int kMSplit = 32;          // ranges of the first stage of a multi-column finalize
// partials of the multi-column kernels: kMaxMGrid + kMSplit entries of 64 doubles
constexpr int kMaxGemmSlices = 16;   // split of the inner dimension of the coarsest GEMM

// Per-column CG state (device resident).
struct MState {
    double rz[kMaxRhs];
    double pq[kMaxRhs];
    double rr[kMaxRhs];
    double bb[kMaxRhs];
    double alpha[kMaxRhs];
    double beta[kMaxRhs];
    double tol2bb[kMaxRhs];
    double rz_prev[kMaxRhs];
    int32_t iter[kMaxRhs];
    int32_t done[kMaxRhs];
    int32_t status[kMaxRhs];
    int32_t all_done;
    int32_t k;
    int32_t maxiter;
    int32_t flexible;
};

template <typename V, typename T>
void launch_spmm(const SellView<V> &A, int C, int mode, int k, const T *x, const T *f, T *y, const T *M,
                 double *partials, MState *st, int gated, int site, hipStream_t s);
template <typename T>
void launch_jacobi0_m(int64_t rows, int k, const T *M, const T *f, T *x, MState *st, int gated, hipStream_t s);
// Y = Ainv F (n x k, row-major); part: scratch of kMaxGemmSlices * n * 32 doubles
template <typename T>
void launch_dense_gemm(int n, int k, const double *Ainv, const T *f, T *y, double *part, MState *st, int gated,
                       hipStream_t s);
int dense_gemm_slices(int n, int k);
// outer FP64 CG pieces; TV is the V-cycle vector type
template <typename TV>
void launch_cg_update_m(int64_t rows, int k, double *x, const double *p, double *r, const double *q,
                        const TV *M, TV *rv, TV *x1, const TV *zold, double *partials, MState *st,
                        hipStream_t s);
template <typename TV>
void launch_cg_dir_m(int64_t rows, int k, const TV *z, double *p, MState *st, hipStream_t s);
void launch_mstate_init(MState *st, int k, int maxiter, int flexible, hipStream_t s);
void launch_mstate_arm(MState *st, double tol, hipStream_t s);
int spmm_grid(int rows);

enum MSite : int32_t {
    MSITE_NONE = 0,
    MSITE_PQ = 1,
    MSITE_RR = 2,
    MSITE_RZ = 3,
    MSITE_INIT = 4,
    MSITE_RZ0 = 5,
};

}  // namespace saamg
