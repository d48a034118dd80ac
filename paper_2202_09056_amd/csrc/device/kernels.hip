// HIP kernels for gfx950 (see kernels.hpp for the data layout).
//
// Every product kernel streams a 3x3-block matrix once, gathers the input
// vector (cache resident), and fuses the level's vector work into the same
// pass (the SellMode epilogues): residual f - A x, one smoothing sweep
// x + M (f - A x), correction x += P x_c, the fused post-sweep
// G e + M (f + t), and the dot products CG needs.  Device-wide sums are
// two-stage and deterministic: every workgroup writes its partial sum, and a
// one-workgroup kernel (k_finalize) adds the partials in a fixed order and
// applies the CG scalar update on the device, so the host never waits inside
// an iteration.
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

// Matrix entries are streamed once per product: load them non-temporally so
// they do not evict the gathered vector from the caches.
__device__ __forceinline__ double ld_nt(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_nt(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int ld_nt(const int *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ bf16_t ld_nt(const bf16_t *p) {
    return bf16_t{__builtin_nontemporal_load(&p->bits)};
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

// Per-workgroup partial sums of two values; k_finalize adds them up.  No
// device-scope fence is needed inside the streaming kernels: the kernel
// boundary orders the partial stores before the finalize kernel reads them.
__device__ __forceinline__ void reduce2_partial(double v0, double v1, double *partials) {
    __shared__ double lds0[kBlock / 64];
    __shared__ double lds1[kBlock / 64];
    const double b0 = block_sum(v0, lds0);
    const double b1 = block_sum(v1, lds1);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = b0;
        partials[gridDim.x + blockIdx.x] = b1;
    }
}

// One workgroup: deterministic fixed-order sum of `nblk` partial pairs, then
// the CG scalar update for `site`.  A thread loads eight of its partials of
// each sum before adding them (in the same order), so the loads overlap
// instead of costing one memory round trip each.
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ partials, int nblk,
                                                     DevState *st, int gated, int site) {
    if (gated && st->done) return;
    __shared__ double lds0[kBlock / 64];
    __shared__ double lds1[kBlock / 64];
    double s0 = 0.0, s1 = 0.0;
    int j = threadIdx.x;
    for (; j + 7 * kBlock < nblk; j += 8 * kBlock) {
        double p0[8], p1[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            p0[q] = partials[j + q * kBlock];
            p1[q] = partials[nblk + j + q * kBlock];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            s0 += p0[q];
            s1 += p1[q];
        }
    }
    for (; j < nblk; j += kBlock) {
        s0 += partials[j];
        s1 += partials[nblk + j];
    }
    const double t0 = block_sum(s0, lds0);
    const double t1 = block_sum(s1, lds1);
    if (threadIdx.x == 0) finalize(site, t0, t1, st);
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

template <int MODE>
constexpr bool mode_reduces() {
    return MODE == MODE_SPMV_DOT || MODE == MODE_SMOOTH_DOT || MODE == MODE_RESID_NORM || MODE == MODE_POST_DOT ||
           MODE == MODE_POST2_DOT || MODE == MODE_POSTP_DOT;
}

// The fused post-sweep z = G e + M (f + t) (M indexed by row, or by slice
// position for the P modes: a copy of the blocks in the operator's own row
// order, so a slice reads them contiguously when its rows are sorted).
template <int MODE>
constexpr bool mode_post() {
    return MODE == MODE_POST || MODE == MODE_POST_DOT || MODE == MODE_POSTP || MODE == MODE_POSTP_DOT;
}

// Operands of a row's epilogue, loaded before the product loop so their
// latency hides behind the matrix stream.
template <typename T>
struct RowPre {
    T f0, f1, f2, x0, x1, x2, y0, y1, y2;
    T m[9];
    T m2[9];  // post-sweep blocks of the two-block fused post-sweep
};

// Modes whose epilogue reads f, a row-local vector and the smoother block
// (15 operands): the smoothing sweeps (x) and the fused post-sweep (t, held
// in y).
template <int MODE>
constexpr bool mode_smooths() {
    return MODE == MODE_SMOOTH || MODE == MODE_SMOOTH_DOT || mode_post<MODE>();
}

// The two-block fused post-sweep: f, t (in y) and the pre- and post-sweep
// blocks (24 operands; M points at an 18-entry planar array).
template <int MODE>
constexpr bool mode_post2() {
    return MODE == MODE_POST2 || MODE == MODE_POST2_DOT;
}

// The epilogue operands of a row (f, x, y and the smoother block, as the mode
// needs them) are loaded before the product loop so their latency hides behind
// the matrix stream, spread over the lanes that serve the row (lane q of the
// row loads operands q, q + G, ...) so that no lane holds all of them through
// the loop; the row's first lane collects them by shuffles afterwards.
template <int MODE>
constexpr int pre_items() {
    if constexpr (MODE == MODE_SPMV) return 0;
    else if constexpr (mode_post2<MODE>()) return 24;    // f (3), t (3), M (9), Mt (9)
    else if constexpr (mode_smooths<MODE>()) return 15;  // f (3), x (3), M (9)
    else if constexpr (MODE == MODE_MSOLVE) return 12;   // f (3), M (9)
    else return 3;                                       // f, y or x
}

template <typename T, int MODE>
__device__ __forceinline__ T pre_load(int64_t row, int64_t pos, int j, const T *__restrict__ x,
                                      const T *__restrict__ f, const T *__restrict__ y, const T *__restrict__ M) {
    if constexpr (mode_post2<MODE>()) {
        if (j < 3) return f[3 * row + j];
        if (j < 6) return y[3 * row + j - 3];
        return M[(row / kMSlice) * (18 * kMSlice) + (j - 6) * kMSlice + (row % kMSlice)];
    } else if constexpr (mode_smooths<MODE>()) {
        if (j < 3) return f[3 * row + j];
        if (j < 6) return mode_post<MODE>() ? y[3 * row + j - 3] : x[3 * row + j - 3];
        const int64_t mi = (MODE == MODE_POSTP || MODE == MODE_POSTP_DOT) ? pos : row;
        return M[(mi / kMSlice) * (9 * kMSlice) + (j - 6) * kMSlice + (mi % kMSlice)];
    } else if constexpr (MODE == MODE_MSOLVE) {
        if (j < 3) return f[3 * row + j];
        return M[(row / kMSlice) * (9 * kMSlice) + (j - 3) * kMSlice + (row % kMSlice)];
    } else if constexpr (MODE == MODE_ADD) {
        return y[3 * row + j];
    } else if constexpr (MODE == MODE_SPMV_DOT) {
        return x[3 * row + j];
    } else {
        return f[3 * row + j];
    }
}

template <typename T, int MODE>
__device__ __forceinline__ void pre_assign(RowPre<T> &p, int j, T v) {
    if constexpr (mode_post2<MODE>()) {
        if (j == 0) p.f0 = v;
        else if (j == 1) p.f1 = v;
        else if (j == 2) p.f2 = v;
        else if (j == 3) p.x0 = v;
        else if (j == 4) p.x1 = v;
        else if (j == 5) p.x2 = v;
        else if (j < 15) p.m[j - 6] = v;
        else p.m2[j - 15] = v;
    } else if constexpr (mode_smooths<MODE>()) {
        if (j == 0) p.f0 = v;
        else if (j == 1) p.f1 = v;
        else if (j == 2) p.f2 = v;
        else if (j == 3) p.x0 = v;
        else if (j == 4) p.x1 = v;
        else if (j == 5) p.x2 = v;
        else p.m[j - 6] = v;
    } else if constexpr (MODE == MODE_MSOLVE) {
        if (j == 0) p.f0 = v;
        else if (j == 1) p.f1 = v;
        else if (j == 2) p.f2 = v;
        else p.m[j - 3] = v;
    } else if constexpr (MODE == MODE_ADD) {
        if (j == 0) p.y0 = v; else if (j == 1) p.y1 = v; else p.y2 = v;
    } else if constexpr (MODE == MODE_SPMV_DOT) {
        if (j == 0) p.x0 = v; else if (j == 1) p.x1 = v; else p.x2 = v;
    } else {
        if (j == 0) p.f0 = v; else if (j == 1) p.f1 = v; else p.f2 = v;
    }
}

// Operands held by lane `q` of a row served by G lanes.  Only the smoothing
// modes (15 operands) spread them; the 3 operands of the other modes stay in
// the row's first lane (measured faster: the spread buys occupancy the
// product loop of those modes does not need).
template <typename T, int MODE, int G>
struct PreSpread {
    static constexpr int NP = pre_items<MODE>();
    static constexpr int GE = NP > 3 ? G : 1;  // lanes that hold operands
    static constexpr int PQ = NP > 0 ? (NP + GE - 1) / GE : 1;
    T v[PQ];
    __device__ __forceinline__ void load(bool has_row, int64_t row, int64_t pos, int q, const T *__restrict__ x,
                                         const T *__restrict__ f, const T *__restrict__ y,
                                         const T *__restrict__ M) {
#pragma unroll
        for (int i = 0; i < PQ; ++i) {
            const int j = q + GE * i;
            v[i] = (has_row && q < GE && j < NP) ? pre_load<T, MODE>(row, pos, j, x, f, y, M) : T(0);
        }
    }
    // every lane must call this; the result is meaningful in lanes with q == 0.
    // Operand j of row lane (q', r) sits in lane q' * stride + r.
    __device__ __forceinline__ RowPre<T> gather(int r, int stride) const {
        RowPre<T> p;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            if constexpr (GE == 1)
                pre_assign<T, MODE>(p, j, v[j]);
            else
                pre_assign<T, MODE>(p, j, __shfl(v[j / GE], (j % GE) * stride + r, 64));
        }
        return p;
    }
};

// Row epilogue shared by the product kernels: (s0, s1, s2) = (A x)_row.
template <typename T, int MODE>
__device__ __forceinline__ void row_epilogue(int64_t row, T s0, T s1, T s2, const RowPre<T> &p,
                                             T *__restrict__ y, double &d0, double &d1) {
    T *yr = y + 3 * row;
    if constexpr (MODE == MODE_SPMV) {
        yr[0] = s0; yr[1] = s1; yr[2] = s2;
    } else if constexpr (MODE == MODE_ADD) {
        yr[0] = p.y0 + s0; yr[1] = p.y1 + s1; yr[2] = p.y2 + s2;
    } else if constexpr (MODE == MODE_SPMV_DOT) {
        yr[0] = s0; yr[1] = s1; yr[2] = s2;
        d0 = (double)p.x0 * s0 + (double)p.x1 * s1 + (double)p.x2 * s2;
    } else if constexpr (mode_post<MODE>()) {
        // z = (G e) + M (f + t), t in the x slot of the operands
        const T e0 = p.f0 + p.x0, e1 = p.f1 + p.x1, e2 = p.f2 + p.x2;
        const T z0 = s0 + (p.m[0] * e0 + p.m[1] * e1 + p.m[2] * e2);
        const T z1 = s1 + (p.m[3] * e0 + p.m[4] * e1 + p.m[5] * e2);
        const T z2 = s2 + (p.m[6] * e0 + p.m[7] * e1 + p.m[8] * e2);
        yr[0] = z0; yr[1] = z1; yr[2] = z2;
        if constexpr (MODE == MODE_POST_DOT || MODE == MODE_POSTP_DOT)
            d0 = (double)p.f0 * z0 + (double)p.f1 * z1 + (double)p.f2 * z2;
    } else if constexpr (mode_post2<MODE>()) {
        // z = (G e) + M f + Mt t, t in the x slot of the operands
        const T z0 = s0 + (p.m[0] * p.f0 + p.m[1] * p.f1 + p.m[2] * p.f2) +
                     (p.m2[0] * p.x0 + p.m2[1] * p.x1 + p.m2[2] * p.x2);
        const T z1 = s1 + (p.m[3] * p.f0 + p.m[4] * p.f1 + p.m[5] * p.f2) +
                     (p.m2[3] * p.x0 + p.m2[4] * p.x1 + p.m2[5] * p.x2);
        const T z2 = s2 + (p.m[6] * p.f0 + p.m[7] * p.f1 + p.m[8] * p.f2) +
                     (p.m2[6] * p.x0 + p.m2[7] * p.x1 + p.m2[8] * p.x2);
        yr[0] = z0; yr[1] = z1; yr[2] = z2;
        if constexpr (MODE == MODE_POST2_DOT)
            d0 = (double)p.f0 * z0 + (double)p.f1 * z1 + (double)p.f2 * z2;
    } else {
        const T e0 = p.f0 - s0, e1 = p.f1 - s1, e2 = p.f2 - s2;
        if constexpr (MODE == MODE_MSOLVE) {
            yr[0] = p.m[0] * e0 + p.m[1] * e1 + p.m[2] * e2;
            yr[1] = p.m[3] * e0 + p.m[4] * e1 + p.m[5] * e2;
            yr[2] = p.m[6] * e0 + p.m[7] * e1 + p.m[8] * e2;
        } else if constexpr (MODE == MODE_RESID || MODE == MODE_RESID_NORM) {
            yr[0] = e0; yr[1] = e1; yr[2] = e2;
            if constexpr (MODE == MODE_RESID_NORM) {
                d0 = (double)p.f0 * p.f0 + (double)p.f1 * p.f1 + (double)p.f2 * p.f2;
                d1 = (double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2;
            }
        } else {  // smoothing sweep
            const T z0 = p.x0 + (p.m[0] * e0 + p.m[1] * e1 + p.m[2] * e2);
            const T z1 = p.x1 + (p.m[3] * e0 + p.m[4] * e1 + p.m[5] * e2);
            const T z2 = p.x2 + (p.m[6] * e0 + p.m[7] * e1 + p.m[8] * e2);
            yr[0] = z0; yr[1] = z1; yr[2] = z2;
            if constexpr (MODE == MODE_SMOOTH_DOT)
                d0 = (double)p.f0 * z0 + (double)p.f1 * z1 + (double)p.f2 * z2;
        }
    }
}

// Elements 0..7 of a block, one aligned 16-byte load per group.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef unsigned int uvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load8(const double *__restrict__ val, int64_t gstride, int64_t rec, double a[8]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const dvec2 v = __builtin_nontemporal_load((const dvec2 *)(val + q * gstride + rec * 2));
        a[2 * q] = v.x;
        a[2 * q + 1] = v.y;
    }
}
__device__ __forceinline__ void load8(const float *__restrict__ val, int64_t gstride, int64_t rec, float a[8]) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const fvec4 v = __builtin_nontemporal_load((const fvec4 *)(val + q * gstride + rec * 4));
        a[4 * q] = v.x;
        a[4 * q + 1] = v.y;
        a[4 * q + 2] = v.z;
        a[4 * q + 3] = v.w;
    }
}
__device__ __forceinline__ void load8(const bf16_t *__restrict__ val, int64_t, int64_t rec, float a[8]) {
    const uvec4 v = __builtin_nontemporal_load((const uvec4 *)(val + rec * 8));
    const unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // the lower address holds the lower half
        a[2 * i] = __uint_as_float(w[i] << 16);
        a[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
}

template <typename V, typename T, int C>
__device__ __forceinline__ void block_fma(const SellView<V> &A, int64_t slot, int r,
                                          const T *__restrict__ x, T &s0, T &s1, T &s2) {
    const int64_t rec = slot * C + r;
    const int c = ld_nt(A.col + rec);
    T a[8];
    load8(A.val, A.gstride, rec, a);
    const T a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3], a4 = a[4], a5 = a[5], a6 = a[6], a7 = a[7];
    const T a8 = to_compute(ld_nt(A.val8 + rec), T());
    const T *xc = x + 3 * (int64_t)c;
    const T x0 = xc[0], x1 = xc[1], x2 = xc[2];
    s0 = fma(a0, x0, fma(a1, x1, fma(a2, x2, s0)));
    s1 = fma(a3, x0, fma(a4, x1, fma(a5, x2, s1)));
    s2 = fma(a6, x0, fma(a7, x1, fma(a8, x2, s2)));
}

// Sliced-ELL product, G = 64 / C lanes per block row.
template <typename V, typename T, int C, int MODE>
__global__ __launch_bounds__(kBlock) void k_sell(SellView<V> A, const T *__restrict__ x,
                                                 const T *__restrict__ f, T *__restrict__ y,
                                                 const T *__restrict__ M, double *partials,
                                                 DevState *st, int gated) {
    if (gated && st->done) return;
    constexpr int G = 64 / C;
    const int lane = threadIdx.x & 63;
    const int g = lane / C;
    const int r = lane % C;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t slice = (int64_t)tile * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t pos = slice * C + r;
    const bool has_row = slice < A.nslices && pos < A.rows;
    const int64_t row = has_row ? (A.perm ? (int64_t)A.perm[pos] : pos) : 0;
    T s0 = 0, s1 = 0, s2 = 0;
    T u0 = 0, u1 = 0, u2 = 0;
    PreSpread<T, MODE, G> spread;
    spread.load(has_row, row, pos, g, x, f, y, M);
    if (has_row) {
        const int len = A.rowlen[pos];
        const int64_t base = A.slice_ptr[slice];
        int k = g;
        if constexpr (C <= 16) {
            // several lanes per row: four blocks in flight per lane (measured:
            // level-2 operators 4.8 -> 5.4 TB/s on the 64^3 cube, where few
            // wavefronts per SIMD have to cover the memory latency)
            T w0 = 0, w1 = 0, w2 = 0, v0 = 0, v1 = 0, v2 = 0;
            for (; k + 3 * G < len; k += 4 * G) {
                block_fma<V, T, C>(A, base + k, r, x, s0, s1, s2);
                block_fma<V, T, C>(A, base + k + G, r, x, u0, u1, u2);
                block_fma<V, T, C>(A, base + k + 2 * G, r, x, w0, w1, w2);
                block_fma<V, T, C>(A, base + k + 3 * G, r, x, v0, v1, v2);
            }
            s0 += w0; s1 += w1; s2 += w2;
            u0 += v0; u1 += v1; u2 += v2;
        }
        for (; k + G < len; k += 2 * G) {
            block_fma<V, T, C>(A, base + k, r, x, s0, s1, s2);
            block_fma<V, T, C>(A, base + k + G, r, x, u0, u1, u2);
        }
        if (k < len) block_fma<V, T, C>(A, base + k, r, x, s0, s1, s2);
        s0 += u0;
        s1 += u1;
        s2 += u2;
    }
#pragma unroll
    for (int off = C; off < 64; off <<= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
        s2 += __shfl_xor(s2, off, 64);
    }
    const RowPre<T> pre = spread.gather(r, C);
    double d0 = 0.0, d1 = 0.0;
    if (has_row && g == 0) row_epilogue<T, MODE>(row, s0, s1, s2, pre, y, d0, d1);
    if constexpr (mode_reduces<MODE>()) reduce2_partial(d0, d1, partials);
}

constexpr int kRowPass = 4;  // passes of 7 blocks issued together (even)

// Sum over blocks [0, len) starting at record `base` of a contiguous (C = 1)
// operator, one wavefront: 63 lanes cover 7 blocks x 9 entries per pass, so
// lane l always accumulates entry e = l % 9 of its blocks (column c = e % 3).
// Chunks of up to 128 blocks: the chunk's column indices are loaded first
// (two per lane) and handed out by shuffles, so the value loads and the
// gathers of every pass can be issued together.  The trip count is uniform
// across the wavefront (every lane takes part in every shuffle); a pass
// beyond the end re-reads block 0 of the chunk with weight 0.
template <typename V, typename T>
__device__ __forceinline__ T rowwave_sum(const SellView<V> &A, const T *__restrict__ x, int64_t base, int len,
                                         int lane) {
    const int e = lane % 9;
    const int kb = lane / 9;  // 0..6, 7 = idle lane 63
    const int c = e % 3;
    const bool active = lane < 63;
    T acc = 0, acc2 = 0;
    for (int k0 = 0; k0 < len; k0 += 128) {
        const int n = min(len - k0, 128);
        const int64_t cb = base + k0;
        const int ci0 = lane < n ? ld_nt(A.col + cb + lane) : 0;
        const int ci1 = 64 + lane < n ? ld_nt(A.col + cb + 64 + lane) : 0;
        for (int p0 = 0; 7 * p0 < n; p0 += kRowPass) {
            T vs[kRowPass], xs[kRowPass];
#pragma unroll
            for (int q = 0; q < kRowPass; ++q) {
                const int kk = kb + 7 * (p0 + q);
                const bool ok = active && kk < n;
                const int ks = ok ? kk : 0;
                const int a = __shfl(ci0, ks & 63, 64), b = __shfl(ci1, ks & 63, 64);
                const int col = ks < 64 ? a : b;
                const T v = to_compute(ld_nt(A.val + (cb + ks) * 9 + e), T());  // contiguous blocks
                vs[q] = ok ? v : T(0);
                xs[q] = x[3 * (int64_t)col + c];
            }
#pragma unroll
            for (int q = 0; q < kRowPass; q += 2) {
                acc = fma(vs[q], xs[q], acc);
                acc2 = fma(vs[q + 1], xs[q + 1], acc2);
            }
        }
    }
    return acc + acc2;
}

// Folds the per-lane entry sums of rowwave_sum into the row's three sums
// (returned in every lane): first the 7 block groups (lanes e, e+9, ...,
// e+54), then the 3 columns of each block row.
template <typename T>
__device__ __forceinline__ void rowwave_fold(T acc, int lane, T &s0, T &s1, T &s2) {
    T se = acc;
#pragma unroll
    for (int m = 1; m < 7; ++m) se += __shfl(acc, (lane + 9 * m) & 63, 64);
    const T sr = se + __shfl(se, (lane + 1) & 63, 64) + __shfl(se, (lane + 2) & 63, 64);
    s0 = __shfl(sr, 0, 64);
    s1 = __shfl(sr, 3, 64);
    s2 = __shfl(sr, 6, 64);
}

// Long rows: one wavefront per block row over the row's contiguous blocks
// (layout code 1).
template <typename V, typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_rowwave(SellView<V> A, const T *__restrict__ x,
                                                    const T *__restrict__ f, T *__restrict__ y,
                                                    const T *__restrict__ M, double *partials,
                                                    DevState *st, int gated) {
    if (gated && st->done) return;
    const int lane = threadIdx.x & 63;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t row = (int64_t)tile * (kBlock / 64) + (threadIdx.x >> 6);
    const bool has_row = row < A.rows;
    PreSpread<T, MODE, 64> spread;
    spread.load(has_row, row, row, lane, x, f, y, M);
    T acc = 0;
    if (has_row) acc = rowwave_sum<V, T>(A, x, A.slice_ptr[row], A.rowlen[row], lane);
    T s0, s1, s2;
    rowwave_fold(acc, lane, s0, s1, s2);
    const RowPre<T> pre = spread.gather(0, 1);
    double d0 = 0.0, d1 = 0.0;
    if (has_row && lane == 0) row_epilogue<T, MODE>(row, s0, s1, s2, pre, y, d0, d1);
    if constexpr (mode_reduces<MODE>()) reduce2_partial(d0, d1, partials);
}

// Few long rows (coarse levels): one workgroup per block row over the same
// contiguous storage (layout code 2).  Wave w of the kBlock/64 waves takes
// the w-th share of the row's blocks (shares of whole 7-block passes), and
// the waves' sums are added in wave order through LDS, so the result does
// not depend on timing.  Four times the wavefronts of a row wave keep more
// loads in flight when the level has too few rows to fill the chip.
template <typename V, typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_rowgroup(SellView<V> A, const T *__restrict__ x,
                                                     const T *__restrict__ f, T *__restrict__ y,
                                                     const T *__restrict__ M, double *partials,
                                                     DevState *st, int gated) {
    if (gated && st->done) return;
    constexpr int S = kBlock / 64;
    __shared__ T part[S][3];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t row = xcd_tile(blockIdx.x, gridDim.x);
    const bool has_row = row < A.rows;
    PreSpread<T, MODE, 64> spread;
    spread.load(has_row && w == 0, row, row, lane, x, f, y, M);
    T acc = 0;
    if (has_row) {
        const int len = A.rowlen[row];
        const int share = 7 * ((len + 7 * S - 1) / (7 * S));
        const int lo = min(len, w * share);
        const int hi = min(len, lo + share);
        acc = rowwave_sum<V, T>(A, x, (int64_t)A.slice_ptr[row] + lo, hi - lo, lane);
    }
    T s0, s1, s2;
    rowwave_fold(acc, lane, s0, s1, s2);
    if (lane == 0) {
        part[w][0] = s0;
        part[w][1] = s1;
        part[w][2] = s2;
    }
    __syncthreads();
    const RowPre<T> pre = spread.gather(0, 1);
    double d0 = 0.0, d1 = 0.0;
    if (has_row && threadIdx.x == 0) {
        T t0 = part[0][0], t1 = part[0][1], t2 = part[0][2];
#pragma unroll
        for (int q = 1; q < S; ++q) {
            t0 += part[q][0];
            t1 += part[q][1];
            t2 += part[q][2];
        }
        row_epilogue<T, MODE>(row, t0, t1, t2, pre, y, d0, d1);
    }
    if constexpr (mode_reduces<MODE>()) reduce2_partial(d0, d1, partials);
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
// flexible variant), and the level-1 pre-smoothing sweep x1 = M r.  Dot
// products accumulate in FP64 whatever the vector type.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t rows, T *__restrict__ x,
                                                      const T *__restrict__ p, T *__restrict__ r,
                                                      const T *__restrict__ q,
                                                      const T *__restrict__ M, T *__restrict__ x1,
                                                      const T *__restrict__ zold, double *partials,
                                                      DevState *st) {
    if (st->done) return;
    const T alpha = (T)st->alpha;
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double d0 = 0.0, d1 = 0.0;  // ||r||^2, r . z_old
    if (row < rows) {
        T e[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t i = 3 * row + c;
            x[i] += alpha * p[i];
            e[c] = r[i] - alpha * q[i];
            r[i] = e[c];
            d0 += (double)e[c] * e[c];
            if (zold) d1 += (double)e[c] * zold[i];
        }
        if (M) {
            T z0, z1, z2;
            apply_m(M, row, e[0], e[1], e[2], z0, z1, z2);
            x1[3 * row] = z0;
            x1[3 * row + 1] = z1;
            x1[3 * row + 2] = z2;
        }
    }
    reduce2_partial(d0, d1, partials);
}

// Outer FP64 CG around a reduced-precision V-cycle: the update also writes
// the FP32 copy of r the V-cycle reads, and its level-1 pre-smoothing sweep.
template <typename TV>
__global__ __launch_bounds__(kBlock) void k_cg_update_mixed(
    int64_t rows, double *__restrict__ x, const double *__restrict__ p, double *__restrict__ r,
    const double *__restrict__ q, const TV *__restrict__ M, TV *__restrict__ rv, TV *__restrict__ x1,
    const TV *__restrict__ zold, double *partials, DevState *st) {
    if (st->done) return;
    const double alpha = st->alpha;
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double d0 = 0.0, d1 = 0.0;
    if (row < rows) {
        TV e[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t i = 3 * row + c;
            x[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            d0 += ri * ri;
            e[c] = (TV)ri;
            rv[i] = e[c];
            if (zold) d1 += (double)e[c] * zold[i];
        }
        if (M) {
            TV z0, z1, z2;
            apply_m(M, row, e[0], e[1], e[2], z0, z1, z2);
            x1[3 * row] = z0;
            x1[3 * row + 1] = z1;
            x1[3 * row + 2] = z2;
        }
    }
    reduce2_partial(d0, d1, partials);
}

// p (FP64) = z (V-cycle precision) + beta p
template <typename TV>
__global__ __launch_bounds__(kBlock) void k_cg_dir_mixed(int64_t n, const TV *__restrict__ z,
                                                         double *__restrict__ p, DevState *st) {
    if (st->done) return;
    const double beta = st->beta;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = (double)z[i] + beta * p[i];
}

// p = z + beta p
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_dir(int64_t n, const T *__restrict__ z,
                                                   T *__restrict__ p, DevState *st) {
    if (st->done) return;
    const T beta = (T)st->beta;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = z[i] + beta * p[i];
}

// x (FP64) += d (any type)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add_to(int64_t n, const T *__restrict__ d,
                                                   double *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] += (double)d[i];
}

// device-wide a . b into `site` (used when no product kernel carries the dot)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, const T *__restrict__ a,
                                                const T *__restrict__ b, double *partials,
                                                DevState *st, int gated) {
    if (gated && st->done) return;
    const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double d = 0.0;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * kBlock) d += (double)a[i] * b[i];
    reduce2_partial(d, 0.0, partials);
}

// out = a + b (out may be a or b); with a reduction site, also the partial
// sums of f . out
template <typename T, bool DOT>
__global__ __launch_bounds__(kBlock) void k_add2(int64_t n, const T *a, const T *b, T *out,
                                                 const T *__restrict__ f, double *partials,
                                                 DevState *st, int gated) {
    if (gated && st->done) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double d = 0.0;
    if (i < n) {
        const T v = a[i] + b[i];
        out[i] = v;
        if constexpr (DOT) d = (double)f[i] * v;
    }
    if constexpr (DOT) reduce2_partial(d, 0.0, partials);
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

// inner solve of the mixed-precision form: fresh counters, absolute target
__global__ void k_state_inner(DevState *st, double tol2abs, int maxiter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->tol2bb = tol2abs;
        st->iter = 0;
        st->maxiter = maxiter;
        st->done = 0;
        st->status = ST_RUNNING;
        st->rz = st->pq = st->alpha = st->beta = st->rz_prev = 0.0;
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

// Dense y = W f for a short, wide W (m x n, FP64, row-major: the coarsest
// inverse times the last restriction), one workgroup per row: the row's n
// entries are read in 256-wide coalesced sweeps with four accumulators per
// thread, then added in fixed order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_rect(int m, int n, const double *__restrict__ W,
                                                       const T *__restrict__ f, T *__restrict__ y, DevState *st,
                                                       int gated) {
    if (gated && st->done) return;
    __shared__ double lds[kBlock / 64];
    const int row = blockIdx.x;
    const double *w = W + (int64_t)row * n;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = threadIdx.x;
    for (; j + 3 * kBlock < n; j += 4 * kBlock) {
        a0 += w[j] * (double)f[j];
        a1 += w[j + kBlock] * (double)f[j + kBlock];
        a2 += w[j + 2 * kBlock] * (double)f[j + 2 * kBlock];
        a3 += w[j + 3 * kBlock] * (double)f[j + 3 * kBlock];
    }
    for (; j < n; j += kBlock) a0 += w[j] * (double)f[j];
    const double s = block_sum((a0 + a1) + (a2 + a3), lds);
    if (threadIdx.x == 0 && row < m) y[row] = (T)s;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

static void launch_finalize(const double *partials, int nblk, DevState *st, int gated, int site,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partials, nblk, st, gated, site);
}

template <typename V, typename T, int C>
static int launch_sell_c(const SellView<V> &A, int mode, const T *x, const T *f, T *y, const T *M,
                         double *partials, DevState *st, int gated, hipStream_t s) {
    const int grid = product_grid(A.rows, A.nslices, C);
    if (grid == 0) return 0;
    switch (mode) {
#define SAAMG_CASE(MD)                                                                            \
    case MD:                                                                                      \
        if constexpr (C == 1)                                                                     \
            hipLaunchKernelGGL((k_rowwave<V, T, MD>), dim3(grid), dim3(kBlock), 0, s, A, x, f, y, M, \
                               partials, st, gated);                                              \
        else if constexpr (C == 2)                                                                \
            hipLaunchKernelGGL((k_rowgroup<V, T, MD>), dim3(grid), dim3(kBlock), 0, s, A, x, f, y, M, \
                               partials, st, gated);                                              \
        else                                                                                      \
            hipLaunchKernelGGL((k_sell<V, T, C, MD>), dim3(grid), dim3(kBlock), 0, s, A, x, f, y, M, \
                               partials, st, gated);                                              \
        break;
        SAAMG_CASE(MODE_SPMV)
        SAAMG_CASE(MODE_RESID)
        SAAMG_CASE(MODE_SMOOTH)
        SAAMG_CASE(MODE_ADD)
        SAAMG_CASE(MODE_SPMV_DOT)
        SAAMG_CASE(MODE_SMOOTH_DOT)
        SAAMG_CASE(MODE_RESID_NORM)
        SAAMG_CASE(MODE_POST)
        SAAMG_CASE(MODE_POST_DOT)
        SAAMG_CASE(MODE_POST2)
        SAAMG_CASE(MODE_POST2_DOT)
        SAAMG_CASE(MODE_MSOLVE)
        SAAMG_CASE(MODE_POSTP)
        SAAMG_CASE(MODE_POSTP_DOT)
#undef SAAMG_CASE
    }
    return grid;
}

template <typename V, typename T>
void launch_sell(const SellView<V> &A, int C, int mode, const T *x, const T *f, T *y, const T *M,
                 double *partials, DevState *st, int gated, int site, hipStream_t s) {
    int grid = 0;
    switch (C) {
        case 1: grid = launch_sell_c<V, T, 1>(A, mode, x, f, y, M, partials, st, gated, s); break;
        case 2: grid = launch_sell_c<V, T, 2>(A, mode, x, f, y, M, partials, st, gated, s); break;
        case 4: grid = launch_sell_c<V, T, 4>(A, mode, x, f, y, M, partials, st, gated, s); break;
        case 8: grid = launch_sell_c<V, T, 8>(A, mode, x, f, y, M, partials, st, gated, s); break;
        case 16: grid = launch_sell_c<V, T, 16>(A, mode, x, f, y, M, partials, st, gated, s); break;
        case 32: grid = launch_sell_c<V, T, 32>(A, mode, x, f, y, M, partials, st, gated, s); break;
        default: grid = launch_sell_c<V, T, 64>(A, mode, x, f, y, M, partials, st, gated, s); break;
    }
    const bool reduces = mode == MODE_SPMV_DOT || mode == MODE_SMOOTH_DOT || mode == MODE_RESID_NORM ||
                         mode == MODE_POST_DOT || mode == MODE_POST2_DOT || mode == MODE_POSTP_DOT;
    if (reduces && site != SITE_NONE && grid > 0) launch_finalize(partials, grid, st, gated, site, s);
}

int sell_grid(int nslices) { return (nslices + kBlock / 64 - 1) / (kBlock / 64); }

// Workgroups of one product launch: a wavefront per row (code 1), a
// workgroup per row (code 2), or a wavefront per slice.
int product_grid(int rows, int nslices, int C) {
    if (C == 1) return (rows + kBlock / 64 - 1) / (kBlock / 64);
    if (C == 2) return rows;
    return sell_grid(nslices);
}

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

// One thread per row position of G: G_IJ = GP_IJ - M_I GAP_IJ for each of
// the row's blocks (the learned level-1 operator G = (I - S A) P after the
// blocks S change).  The three operators share pattern and layout, so a
// record index addresses the same block in each.
template <typename V, typename T>
__global__ __launch_bounds__(kBlock) void k_g_rebuild(SellView<V> G, SellView<V> GP, SellView<V> GAP, int cs,
                                                      const T *__restrict__ M) {
    const int64_t pos = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pos >= G.rows) return;
    const int64_t row = G.perm ? (int64_t)G.perm[pos] : pos;
    const T *mr = M + (row / kMSlice) * (9 * kMSlice) + (row % kMSlice);
    T m[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = mr[e * kMSlice];
    const int len = G.rowlen[pos];
    const int64_t base = G.slice_ptr[pos / cs];
    const int r = (int)(pos % cs);
    for (int k = 0; k < len; ++k) {
        const int64_t rec = (base + k) * cs + r;
        T a[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) a[e] = to_compute(*elem_ptr(GAP, rec, e), T());
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int e = 3 * i + j;
                const T g = to_compute(*elem_ptr(GP, rec, e), T()) -
                            (m[3 * i] * a[j] + m[3 * i + 1] * a[3 + j] + m[3 * i + 2] * a[6 + j]);
                *const_cast<V *>(elem_ptr(G, rec, e)) = (V)g;
            }
    }
}

template <typename V, typename T>
void launch_g_rebuild(const SellView<V> &G, const SellView<V> &GP, const SellView<V> &GAP, int cs, const T *M,
                      hipStream_t s) {
    if (G.rows <= 0) return;
    hipLaunchKernelGGL((k_g_rebuild<V, T>), dim3((G.rows + kBlock - 1) / kBlock), dim3(kBlock), 0, s, G, GP, GAP,
                       cs, M);
}
template void launch_g_rebuild<double, double>(const SellView<double> &, const SellView<double> &,
                                               const SellView<double> &, int, const double *, hipStream_t);
template void launch_g_rebuild<float, float>(const SellView<float> &, const SellView<float> &,
                                             const SellView<float> &, int, const float *, hipStream_t);

template <typename T>
void launch_cg_update(int64_t rows, T *x, const T *p, T *r, const T *q, const T *M, T *x1,
                      const T *zold, double *partials, DevState *st, hipStream_t s) {
    const int grid = (int)((rows + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_cg_update<T>, dim3(grid), dim3(kBlock), 0, s, rows, x, p, r, q, M, x1, zold,
                       partials, st);
    launch_finalize(partials, grid, st, 1, SITE_RR, s);
}
template void launch_cg_update<double>(int64_t, double *, const double *, double *, const double *,
                                       const double *, double *, const double *, double *, DevState *,
                                       hipStream_t);
template void launch_cg_update<float>(int64_t, float *, const float *, float *, const float *,
                                      const float *, float *, const float *, double *, DevState *,
                                      hipStream_t);

template <typename T>
void launch_cg_dir(int64_t n, const T *z, T *p, DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_dir<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, z, p, st);
}
template void launch_cg_dir<double>(int64_t, const double *, double *, DevState *, hipStream_t);
template void launch_cg_dir<float>(int64_t, const float *, float *, DevState *, hipStream_t);

void launch_cg_update_mixed(int64_t rows, double *x, const double *p, double *r, const double *q,
                            const float *M, float *rv, float *x1, const float *zold, double *partials,
                            DevState *st, hipStream_t s) {
    const int grid = (int)((rows + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_cg_update_mixed<float>, dim3(grid), dim3(kBlock), 0, s, rows, x, p, r, q, M, rv, x1,
                       zold, partials, st);
    launch_finalize(partials, grid, st, 1, SITE_RR, s);
}

void launch_cg_dir_mixed(int64_t n, const float *z, double *p, DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_dir_mixed<float>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, z, p, st);
}

template <typename T>
void launch_add_to(int64_t n, const T *d, double *x, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_add_to<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, d, x);
}
template void launch_add_to<float>(int64_t, const float *, double *, hipStream_t);
template void launch_add_to<double>(int64_t, const double *, double *, hipStream_t);

void launch_state_inner(DevState *st, double tol2abs, int maxiter, hipStream_t s) {
    hipLaunchKernelGGL(k_state_inner, dim3(1), dim3(64), 0, s, st, tol2abs, maxiter);
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
template void launch_copy<float, float>(int64_t, const float *, float *, hipStream_t);

template <typename T>
void launch_dot(int64_t n, const T *a, const T *b, double *partials, DevState *st, int gated, int site,
                int max_grid, hipStream_t s) {
    int64_t grid = std::min<int64_t>((n + kBlock - 1) / kBlock, max_grid);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_dot<T>, dim3(grid), dim3(kBlock), 0, s, n, a, b, partials, st, gated);
    launch_finalize(partials, (int)grid, st, gated, site, s);
}
template void launch_dot<double>(int64_t, const double *, const double *, double *, DevState *, int, int,
                                 int, hipStream_t);
template void launch_dot<float>(int64_t, const float *, const float *, double *, DevState *, int, int,
                                int, hipStream_t);

template <typename T>
void launch_add2(int64_t n, const T *a, const T *b, T *out, const T *f, double *partials, DevState *st, int gated,
                 int site, hipStream_t s) {
    if (n <= 0) return;
    const int grid = (int)((n + kBlock - 1) / kBlock);
    if (site == SITE_NONE) {
        hipLaunchKernelGGL((k_add2<T, false>), dim3(grid), dim3(kBlock), 0, s, n, a, b, out, f, partials, st, gated);
    } else {
        hipLaunchKernelGGL((k_add2<T, true>), dim3(grid), dim3(kBlock), 0, s, n, a, b, out, f, partials, st, gated);
        launch_finalize(partials, grid, st, gated, site, s);
    }
}
template void launch_add2<double>(int64_t, const double *, const double *, double *, const double *, double *,
                                  DevState *, int, int, hipStream_t);
template void launch_add2<float>(int64_t, const float *, const float *, float *, const float *, double *,
                                 DevState *, int, int, hipStream_t);

template <typename T>
void launch_fill(int64_t n, T v, T *d, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, v, d);
}
template void launch_fill<double>(int64_t, double, double *, hipStream_t);
template void launch_fill<float>(int64_t, float, float *, hipStream_t);

// norms[0] = ||b||^2, norms[1] = ||r||^2 from a state after SITE_INIT
__global__ void k_state_norms(const DevState *st, double *norms) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        norms[0] = st->bb;
        norms[1] = st->rr;
    }
}
void launch_state_norms(const DevState *st, double *norms, hipStream_t s) {
    hipLaunchKernelGGL(k_state_norms, dim3(1), dim3(64), 0, s, st, norms);
}

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

template <typename T>
void launch_dense_rect(int m, int n, const double *W, const T *f, T *y, DevState *st, int gated, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_dense_rect<T>, dim3(m), dim3(kBlock), 0, s, m, n, W, f, y, st, gated);
}
template void launch_dense_rect<double>(int, int, const double *, const double *, double *, DevState *, int,
                                        hipStream_t);
template void launch_dense_rect<float>(int, int, const double *, const float *, float *, DevState *, int,
                                       hipStream_t);
template void launch_dense_gemv<float>(int, const double *, const float *, float *, DevState *,
                                       int, hipStream_t);

}  // namespace saamg
