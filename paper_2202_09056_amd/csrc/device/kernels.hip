// HIP kernels for gfx950 (see kernels.hpp for the data layout).
//
// Every product kernel streams a sliced-ELL 3x3-block matrix once, gathers
// the input vector (cache resident), and fuses the level's vector work into
// the same pass: residual f - A x, one block-Jacobi sweep x + M (f - A x),
// correction x += P x_c, and the dot products CG needs.  Device-wide sums are
// two-stage and deterministic: every workgroup writes its partial sum, and the
// last workgroup to finish (counted with one atomic increment) adds the
// partials in a fixed order and applies the CG scalar update on the device,
// so the host never waits inside an iteration.
#include <algorithm>

#include "kernels.hpp"
#include "launch.hpp"

namespace saamg {

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) s += lds[i];
    }
    __syncthreads();
    return s;
}

__device__ __forceinline__ double load_coherent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void finalize(int site, double t0, double t1, DevState *st) {
    switch (site) {
        case SITE_PQ:
            st->pq = t0;
            if (!(t0 > 0.0)) {
                st->status = isfinite(t0) ? ST_BREAKDOWN : ST_NONFINITE;
                st->done = 1;
            } else {
                st->alpha = st->rz / t0;
            }
            break;
        case SITE_RR:
            st->rr = t0;
            st->rz_prev = t1;
            st->iter += 1;
            if (!isfinite(t0)) {
                st->status = ST_NONFINITE;
                st->done = 1;
            } else if (t0 <= st->tol2bb) {
                st->status = ST_CONVERGED;
                st->done = 1;
            } else if (st->iter >= st->maxiter) {
                st->status = ST_MAXITER;
                st->done = 1;
            }
            break;
        case SITE_RZ:
            st->beta = st->flexible ? (t0 - st->rz_prev) / st->rz : t0 / st->rz;
            st->rz = t0;
            if (!isfinite(t0)) {
                st->status = ST_NONFINITE;
                st->done = 1;
            }
            break;
        case SITE_RZ0:
            st->rz = t0;
            break;
        case SITE_INIT:
            st->bb = t0;
            st->rr = t1;
            break;
        case SITE_TRUE:
            st->rr = t1;
            break;
        default:
            break;
    }
}

// Two simultaneous device-wide sums; the last workgroup finalises `site`.
__device__ void reduce2_finalize(double v0, double v1, double *partials, DevState *st,
                                 int site) {
    __shared__ double lds0[kBlock / 64];
    __shared__ double lds1[kBlock / 64];
    __shared__ int last;
    const double b0 = block_sum(v0, lds0);
    const double b1 = block_sum(v1, lds1);
    const int nblk = gridDim.x;
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = b0;
        partials[nblk + blockIdx.x] = b1;
        __threadfence();
        const uint32_t prev = atomicAdd(&st->counter, 1u);
        last = (prev == (uint32_t)(nblk - 1));
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double s0 = 0.0, s1 = 0.0;
    for (int j = threadIdx.x; j < nblk; j += kBlock) {
        s0 += load_coherent(partials + j);
        s1 += load_coherent(partials + nblk + j);
    }
    const double t0 = block_sum(s0, lds0);
    const double t1 = block_sum(s1, lds1);
    if (threadIdx.x == 0) {
        st->counter = 0;
        finalize(site, t0, t1, st);
    }
}

// Workgroups are dealt to the 8 XCDs round-robin; remap so each XCD walks a
// contiguous range of slices and its L2 keeps the matching window of x.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int xcd = b & 7, idx = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// ---------------------------------------------------------------------------
// sliced-ELL block products
// ---------------------------------------------------------------------------

template <typename V, typename T, int C, int MODE>
__global__ __launch_bounds__(kBlock) void k_sell(SellView<V> A, const T *__restrict__ x,
                                                 const T *__restrict__ f, T *__restrict__ y,
                                                 const T *__restrict__ M, double *partials,
                                                 DevState *st, int gated, int site) {
    if (gated && st->done) return;
    constexpr int G = 64 / C;
    const int lane = threadIdx.x & 63;
    const int g = lane / C;
    const int r = lane % C;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t slice = (int64_t)tile * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t row = slice * C + r;
    const bool has_row = slice < A.nslices && row < A.rows;
    T s0 = 0, s1 = 0, s2 = 0;
    if (has_row) {
        const int len = A.rowlen[row];
        const int64_t base = A.slice_ptr[slice];
        for (int k = g; k < len; k += G) {
            const int64_t slot = base + k;
            const int c = A.col[slot * C + r];
            const V *v = A.val + slot * (9 * C) + r;
            const T a0 = to_compute(v[0], T()), a1 = to_compute(v[C], T()), a2 = to_compute(v[2 * C], T());
            const T a3 = to_compute(v[3 * C], T()), a4 = to_compute(v[4 * C], T()), a5 = to_compute(v[5 * C], T());
            const T a6 = to_compute(v[6 * C], T()), a7 = to_compute(v[7 * C], T()), a8 = to_compute(v[8 * C], T());
            const T *xc = x + 3 * (int64_t)c;
            const T x0 = xc[0], x1 = xc[1], x2 = xc[2];
            s0 = fma(a0, x0, fma(a1, x1, fma(a2, x2, s0)));
            s1 = fma(a3, x0, fma(a4, x1, fma(a5, x2, s1)));
            s2 = fma(a6, x0, fma(a7, x1, fma(a8, x2, s2)));
        }
    }
#pragma unroll
    for (int off = C; off < 64; off <<= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
        s2 += __shfl_xor(s2, off, 64);
    }
    double d0 = 0.0, d1 = 0.0;
    if (has_row && g == 0) {
        T *yr = y + 3 * row;
        if constexpr (MODE == MODE_SPMV) {
            yr[0] = s0; yr[1] = s1; yr[2] = s2;
        } else if constexpr (MODE == MODE_ADD) {
            yr[0] += s0; yr[1] += s1; yr[2] += s2;
        } else if constexpr (MODE == MODE_SPMV_DOT) {
            yr[0] = s0; yr[1] = s1; yr[2] = s2;
            const T *xr = x + 3 * row;
            d0 = (double)xr[0] * s0 + (double)xr[1] * s1 + (double)xr[2] * s2;
        } else {
            const T *fr = f + 3 * row;
            const T e0 = fr[0] - s0, e1 = fr[1] - s1, e2 = fr[2] - s2;
            if constexpr (MODE == MODE_RESID || MODE == MODE_RESID_NORM) {
                yr[0] = e0; yr[1] = e1; yr[2] = e2;
                if constexpr (MODE == MODE_RESID_NORM) {
                    d0 = (double)fr[0] * fr[0] + (double)fr[1] * fr[1] + (double)fr[2] * fr[2];
                    d1 = (double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2;
                }
            } else {  // smoothing sweep
                const T *m = M + (row / kMSlice) * (9 * kMSlice) + (row % kMSlice);
                const T *xr = x + 3 * row;
                const T z0 = xr[0] + (m[0] * e0 + m[kMSlice] * e1 + m[2 * kMSlice] * e2);
                const T z1 = xr[1] + (m[3 * kMSlice] * e0 + m[4 * kMSlice] * e1 + m[5 * kMSlice] * e2);
                const T z2 = xr[2] + (m[6 * kMSlice] * e0 + m[7 * kMSlice] * e1 + m[8 * kMSlice] * e2);
                yr[0] = z0; yr[1] = z1; yr[2] = z2;
                if constexpr (MODE == MODE_SMOOTH_DOT)
                    d0 = (double)fr[0] * z0 + (double)fr[1] * z1 + (double)fr[2] * z2;
            }
        }
    }
    if constexpr (MODE == MODE_SPMV_DOT || MODE == MODE_SMOOTH_DOT || MODE == MODE_RESID_NORM)
        reduce2_finalize(d0, d1, partials, st, site);
}

// ---------------------------------------------------------------------------
// vector kernels (one thread per block row)
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void apply_m(const T *__restrict__ M, int64_t row, T e0, T e1, T e2,
                                        T &z0, T &z1, T &z2) {
    const T *m = M + (row / kMSlice) * (9 * kMSlice) + (row % kMSlice);
    z0 = m[0] * e0 + m[kMSlice] * e1 + m[2 * kMSlice] * e2;
    z1 = m[3 * kMSlice] * e0 + m[4 * kMSlice] * e1 + m[5 * kMSlice] * e2;
    z2 = m[6 * kMSlice] * e0 + m[7 * kMSlice] * e1 + m[8 * kMSlice] * e2;
}

// x = M f (first smoothing sweep from a zero guess)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi0(int64_t rows, const T *__restrict__ M,
                                                    const T *__restrict__ f, T *__restrict__ x,
                                                    DevState *st, int gated) {
    if (gated && st->done) return;
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (row >= rows) return;
    T z0, z1, z2;
    apply_m(M, row, f[3 * row], f[3 * row + 1], f[3 * row + 2], z0, z1, z2);
    x[3 * row] = z0;
    x[3 * row + 1] = z1;
    x[3 * row + 2] = z2;
}

// CG update: x += alpha p, r -= alpha q, ||r||^2 (and r . z_old for the
// flexible variant), and the level-1 pre-smoothing sweep x1 = M r.
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t rows, double *__restrict__ x,
                                                      const double *__restrict__ p,
                                                      double *__restrict__ r,
                                                      const double *__restrict__ q,
                                                      const double *__restrict__ M,
                                                      double *__restrict__ x1,
                                                      const double *__restrict__ zold,
                                                      double *partials, DevState *st) {
    if (st->done) return;
    const double alpha = st->alpha;
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double d0 = 0.0, d1 = 0.0;
    if (row < rows) {
        double e[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t i = 3 * row + c;
            x[i] += alpha * p[i];
            e[c] = r[i] - alpha * q[i];
            r[i] = e[c];
            d0 += e[c] * e[c];
            if (zold) d1 += e[c] * zold[i];
        }
        if (M) {
            double z0, z1, z2;
            apply_m(M, row, e[0], e[1], e[2], z0, z1, z2);
            x1[3 * row] = z0;
            x1[3 * row + 1] = z1;
            x1[3 * row + 2] = z2;
        }
    }
    reduce2_finalize(d0, d1, partials, st, SITE_RR);
}

// p = z + beta p
__global__ __launch_bounds__(kBlock) void k_cg_dir(int64_t n, const double *__restrict__ z,
                                                   double *__restrict__ p, DevState *st) {
    if (st->done) return;
    const double beta = st->beta;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = z[i] + beta * p[i];
}

// device-wide a . b into `site` (used when no product kernel carries the dot)
__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, const double *__restrict__ a,
                                                const double *__restrict__ b, double *partials,
                                                DevState *st, int gated, int site) {
    if (gated && st->done) return;
    const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double d = 0.0;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * kBlock) d += a[i] * b[i];
    reduce2_finalize(d, 0.0, partials, st, site);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, T v, T *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) d[i] = v;
}

template <typename Ts, typename Td>
__global__ __launch_bounds__(kBlock) void k_copy(int64_t n, const Ts *__restrict__ s,
                                                 Td *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) d[i] = (Td)s[i];
}

__global__ void k_state_init(DevState *st, double tol, int maxiter, int flexible) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->rz = st->pq = st->rr = st->bb = st->alpha = st->beta = st->rz_prev = 0.0;
        st->tol2bb = tol;  // scaled by ||b||^2 in k_state_arm
        st->iter = 0;
        st->maxiter = maxiter;
        st->done = 0;
        st->status = ST_RUNNING;
        st->counter = 0;
        st->flexible = flexible;
    }
}

// after the initial residual: tol2bb = tol^2 ||b||^2, restart the loop flags
__global__ void k_state_arm(DevState *st, double tol) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->tol2bb = tol * tol * st->bb;
        st->done = 0;
        st->status = ST_RUNNING;
    }
}

// Dense y = Ainv f (coarsest level), FP64, one wavefront per row.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_gemv(int n, const double *__restrict__ Ainv,
                                                       const T *__restrict__ f,
                                                       T *__restrict__ y, DevState *st,
                                                       int gated) {
    if (gated && st->done) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double *a = Ainv + (int64_t)row * n;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += a[j] * (double)f[j];
    s = wave_sum(s);
    if (lane == 0) y[row] = (T)s;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

template <typename V, typename T, int C>
static void launch_sell_c(const SellView<V> &A, int mode, const T *x, const T *f, T *y,
                          const T *M, double *partials, DevState *st, int gated, int site,
                          hipStream_t s) {
    const int slices_per_block = kBlock / 64;
    const int grid = (A.nslices + slices_per_block - 1) / slices_per_block;
    if (grid == 0) return;
    switch (mode) {
#define SAAMG_CASE(MD)                                                                     \
    case MD:                                                                               \
        hipLaunchKernelGGL((k_sell<V, T, C, MD>), dim3(grid), dim3(kBlock), 0, s, A, x, f, y, M, \
                           partials, st, gated, site);                                     \
        break;
        SAAMG_CASE(MODE_SPMV)
        SAAMG_CASE(MODE_RESID)
        SAAMG_CASE(MODE_SMOOTH)
        SAAMG_CASE(MODE_ADD)
        SAAMG_CASE(MODE_SPMV_DOT)
        SAAMG_CASE(MODE_SMOOTH_DOT)
        SAAMG_CASE(MODE_RESID_NORM)
#undef SAAMG_CASE
    }
}

template <typename V, typename T>
void launch_sell(const SellView<V> &A, int C, int mode, const T *x, const T *f, T *y, const T *M,
                 double *partials, DevState *st, int gated, int site, hipStream_t s) {
    switch (C) {
        case 16: launch_sell_c<V, T, 16>(A, mode, x, f, y, M, partials, st, gated, site, s); break;
        case 32: launch_sell_c<V, T, 32>(A, mode, x, f, y, M, partials, st, gated, site, s); break;
        default: launch_sell_c<V, T, 64>(A, mode, x, f, y, M, partials, st, gated, site, s); break;
    }
}

int sell_grid(int nslices) { return (nslices + kBlock / 64 - 1) / (kBlock / 64); }

template void launch_sell<double, double>(const SellView<double> &, int, int, const double *,
                                          const double *, double *, const double *, double *,
                                          DevState *, int, int, hipStream_t);
template void launch_sell<float, float>(const SellView<float> &, int, int, const float *,
                                        const float *, float *, const float *, double *,
                                        DevState *, int, int, hipStream_t);
template void launch_sell<bf16_t, float>(const SellView<bf16_t> &, int, int, const float *,
                                         const float *, float *, const float *, double *,
                                         DevState *, int, int, hipStream_t);

template <typename T>
void launch_jacobi0(int64_t rows, const T *M, const T *f, T *x, DevState *st, int gated,
                    hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_jacobi0<T>, dim3((rows + kBlock - 1) / kBlock), dim3(kBlock), 0, s, rows,
                       M, f, x, st, gated);
}
template void launch_jacobi0<double>(int64_t, const double *, const double *, double *,
                                     DevState *, int, hipStream_t);
template void launch_jacobi0<float>(int64_t, const float *, const float *, float *, DevState *,
                                    int, hipStream_t);

void launch_cg_update(int64_t rows, double *x, const double *p, double *r, const double *q,
                      const double *M, double *x1, const double *zold, double *partials,
                      DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update, dim3((rows + kBlock - 1) / kBlock), dim3(kBlock), 0, s, rows,
                       x, p, r, q, M, x1, zold, partials, st);
}

void launch_cg_dir(int64_t n, const double *z, double *p, DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_dir, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, z, p, st);
}

template <typename Ts, typename Td>
void launch_copy(int64_t n, const Ts *src, Td *dst, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_copy<Ts, Td>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n,
                       src, dst);
}
template void launch_copy<double, double>(int64_t, const double *, double *, hipStream_t);
template void launch_copy<double, float>(int64_t, const double *, float *, hipStream_t);
template void launch_copy<float, double>(int64_t, const float *, double *, hipStream_t);

void launch_dot(int64_t n, const double *a, const double *b, double *partials, DevState *st, int gated,
                int site, int max_grid, hipStream_t s) {
    int64_t grid = std::min<int64_t>((n + kBlock - 1) / kBlock, max_grid);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_dot, dim3(grid), dim3(kBlock), 0, s, n, a, b, partials, st, gated, site);
}

template <typename T>
void launch_fill(int64_t n, T v, T *d, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, v, d);
}
template void launch_fill<double>(int64_t, double, double *, hipStream_t);
template void launch_fill<float>(int64_t, float, float *, hipStream_t);

void launch_state_init(DevState *st, double tol, int maxiter, int flexible, hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, tol, maxiter, flexible);
}
void launch_state_arm(DevState *st, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_state_arm, dim3(1), dim3(64), 0, s, st, tol);
}

template <typename T>
void launch_dense_gemv(int n, const double *Ainv, const T *f, T *y, DevState *st, int gated,
                       hipStream_t s) {
    if (n <= 0) return;
    const int rows_per_block = kBlock / 64;
    hipLaunchKernelGGL(k_dense_gemv<T>, dim3((n + rows_per_block - 1) / rows_per_block),
                       dim3(kBlock), 0, s, n, Ainv, f, y, st, gated);
}
template void launch_dense_gemv<double>(int, const double *, const double *, double *,
                                        DevState *, int, hipStream_t);
template void launch_dense_gemv<float>(int, const double *, const float *, float *, DevState *,
                                       int, hipStream_t);

}  // namespace saamg
