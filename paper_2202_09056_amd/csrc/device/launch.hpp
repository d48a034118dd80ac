// Host-side launchers of the solve-phase kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace saamg {

int sell_grid(int nslices);
int product_grid(int rows, int nslices, int C);

template <typename V, typename T>
void launch_sell(const SellView<V> &A, int C, int mode, const T *x, const T *f, T *y, const T *M,
                 double *partials, DevState *st, int gated, int site, hipStream_t s);

template <typename T>
void launch_jacobi0(int64_t rows, const T *M, const T *f, T *x, DevState *st, int gated,
                    hipStream_t s);

// G = GP - M GAP record by record (three operators with one pattern and one
// layout; cs = rows per slice of the storage, M planar smoother blocks).
template <typename V, typename T>
void launch_g_rebuild(const SellView<V> &G, const SellView<V> &GP, const SellView<V> &GAP, int cs, const T *M,
                      hipStream_t s);

template <typename T>
void launch_cg_update(int64_t rows, T *x, const T *p, T *r, const T *q, const T *M, T *x1,
                      const T *zold, double *partials, DevState *st, hipStream_t s);
template <typename T>
void launch_cg_dir(int64_t n, const T *z, T *p, DevState *st, hipStream_t s);
template <typename T>
void launch_add_to(int64_t n, const T *d, double *x, hipStream_t s);
void launch_cg_update_mixed(int64_t rows, double *x, const double *p, double *r, const double *q,
                            const float *M, float *rv, float *x1, const float *zold, double *partials,
                            DevState *st, hipStream_t s);
void launch_cg_dir_mixed(int64_t n, const float *z, double *p, DevState *st, hipStream_t s);
void launch_state_inner(DevState *st, double tol2abs, int maxiter, hipStream_t s);

template <typename Ts, typename Td>
void launch_copy(int64_t n, const Ts *src, Td *dst, hipStream_t s);

template <typename T>
void launch_dot(int64_t n, const T *a, const T *b, double *partials, DevState *st, int gated, int site,
                int max_grid, hipStream_t s);
template <typename T>
void launch_fill(int64_t n, T v, T *d, hipStream_t s);
// out = a + b (n entries); with site != SITE_NONE also f . out into the state
// (partials needs one pair per 256 entries)
template <typename T>
void launch_add2(int64_t n, const T *a, const T *b, T *out, const T *f, double *partials, DevState *st, int gated,
                 int site, hipStream_t s);

void launch_state_init(DevState *st, double tol, int maxiter, int flexible, hipStream_t s);
// norms[0..1] (device) = (bb, rr) of the state
void launch_state_norms(const DevState *st, double *norms, hipStream_t s);
void launch_state_arm(DevState *st, double tol, hipStream_t s);

template <typename T>
void launch_dense_gemv(int n, const double *Ainv, const T *f, T *y, DevState *st, int gated,
                       hipStream_t s);
// y = W f for a dense m x n FP64 W (row-major), one workgroup per row
template <typename T>
void launch_dense_rect(int m, int n, const double *W, const T *f, T *y, DevState *st, int gated, hipStream_t s);

}  // namespace saamg
