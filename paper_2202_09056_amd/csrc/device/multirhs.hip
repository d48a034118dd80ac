// Multi-right-hand-side kernels: block SpMM over the same device operators as
// the single-vector path, one 32-lane half-wavefront per block row; with k
// columns each column gets 32/kp lanes (kp = the power of two >= k) that split
// the row's blocks.  The half-wavefront stages its row's blocks in LDS with
// coalesced loads (32 blocks at a time), and every column's lanes read them
// back as broadcasts, so each block is fetched once for all columns; the
// input columns of a block column are k contiguous values, so the gathers
// stay coalesced.  A lane takes four of its blocks per step, so twelve
// gathers are in flight before the first product (the gathers hit L2 or the
// MALL and set the pace, not HBM).  The epilogues follow the single-vector modes (residual,
// smoothing, correction, fused post-sweeps, dot products).
// Per-column dot products reduce per workgroup and are added up in fixed
// order by a one-workgroup finalize kernel, which also applies the CG scalar
// update of every column (alpha_j, beta_j, convergence mask).
#include <algorithm>
#include <atomic>
#include <cstdint>

#include "multirhs.hpp"

namespace saamg {

constexpr int kRowsPerBlockM = kBlock / 32;  // 8 half-wavefronts, one block row each

__device__ __forceinline__ double to_d(double v) { return v; }
__device__ __forceinline__ double to_d(float v) { return (double)v; }

template <typename V, typename T>
__device__ __forceinline__ T cvt_v(const V *p) {
    return to_compute(*p, T());
}

// Workgroups are dispatched to the eight XCDs in turn (b % 8).  The tiles are
// split into eight contiguous ranges, one per XCD, sized by the XCD's share
// of the grid, and an XCD's workgroups walk their range in order: every round
// of an XCD follows the rows of its previous round, so the X columns of the
// plane below (already in that XCD's L2) are read again from L2.
struct TileRange {
    int64_t first, end;
    int step;
};
__device__ __forceinline__ TileRange xcd_range_m(int b, int nb, int64_t ntiles) {
    const int xcd = b & 7, per = nb >> 3, rem = nb & 7;
    const int nx = per + (xcd < rem ? 1 : 0);        // workgroups on this XCD (>= 1: b is one)
    const int before = xcd * per + min(xcd, rem);    // workgroups on lower XCDs
    return {ntiles * before / nb + (b >> 3), ntiles * (before + nx) / nb, nx};
}

// Per-column sums over the workgroup's 8 rows -> partials[block][2][32].
__device__ __forceinline__ void mreduce(double d0, double d1, double *partials) {
    __shared__ double l0[kRowsPerBlockM][32];
    __shared__ double l1[kRowsPerBlockM][32];
    const int hw = threadIdx.x >> 5, j = threadIdx.x & 31;
    l0[hw][j] = d0;
    l1[hw][j] = d1;
    __syncthreads();
    if (threadIdx.x < 32) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int h = 0; h < kRowsPerBlockM; ++h) {
            s0 += l0[h][threadIdx.x];
            s1 += l1[h][threadIdx.x];
        }
        partials[(int64_t)blockIdx.x * 64 + threadIdx.x] = s0;
        partials[(int64_t)blockIdx.x * 64 + 32 + threadIdx.x] = s1;
    }
}

// The row's blocks are staged in LDS kStage at a time: the 32 lanes of the
// half-wavefront load distinct values (coalesced per slice) instead of every
// lane loading every value of every block, then the column lanes read them
// back as broadcasts.
constexpr int kStage = 32;

// Output of column j of block row `row` from its three sums s0..s2 (the
// products of the row with the input column), per epilogue mode; the dot
// products of the reducing modes are added to d0 (and d1).
template <typename T, int MODE>
__device__ __forceinline__ void spmm_row_out(int64_t row, int j, int k, T s0, T s1, T s2, const T *__restrict__ X,
                                             const T *__restrict__ F, T *__restrict__ Y, const T *__restrict__ M,
                                             double &d0, double &d1) {
    T *yr = Y + 3 * row * k + j;
    if constexpr (MODE == MODE_SPMV) {
        yr[0] = s0; yr[k] = s1; yr[2 * k] = s2;
    } else if constexpr (MODE == MODE_ADD) {
        yr[0] += s0; yr[k] += s1; yr[2 * k] += s2;
    } else if constexpr (MODE == MODE_SPMV_DOT) {
        yr[0] = s0; yr[k] = s1; yr[2 * k] = s2;
        const T *xr = X + 3 * row * k + j;
        d0 += to_d(xr[0]) * s0 + to_d(xr[k]) * s1 + to_d(xr[2 * k]) * s2;
    } else if constexpr (MODE == MODE_POST || MODE == MODE_POST_DOT) {
        // fused post-sweep: Y holds t on entry, z = (G e) + M (f + t)
        const T *fr = F + 3 * row * k + j;
        const T f0 = fr[0], f1 = fr[k], f2 = fr[2 * k];
        const T e0 = f0 + yr[0], e1 = f1 + yr[k], e2 = f2 + yr[2 * k];
        const T *m = M + (row / kMSlice) * (9 * kMSlice) + (row % kMSlice);
        const T z0 = s0 + (m[0] * e0 + m[kMSlice] * e1 + m[2 * kMSlice] * e2);
        const T z1 = s1 + (m[3 * kMSlice] * e0 + m[4 * kMSlice] * e1 + m[5 * kMSlice] * e2);
        const T z2 = s2 + (m[6 * kMSlice] * e0 + m[7 * kMSlice] * e1 + m[8 * kMSlice] * e2);
        yr[0] = z0; yr[k] = z1; yr[2 * k] = z2;
        if constexpr (MODE == MODE_POST_DOT) d0 += to_d(f0) * z0 + to_d(f1) * z1 + to_d(f2) * z2;
    } else if constexpr (MODE == MODE_POST2 || MODE == MODE_POST2_DOT) {
        // two-block fused post-sweep: z = (G e) + M f + Mt t, M and Mt in
        // one 18-entry planar array
        const T *fr = F + 3 * row * k + j;
        const T f0 = fr[0], f1 = fr[k], f2 = fr[2 * k];
        const T t0 = yr[0], t1 = yr[k], t2 = yr[2 * k];
        const T *m = M + (row / kMSlice) * (18 * kMSlice) + (row % kMSlice);
        const T *q = m + 9 * kMSlice;
        const T z0 = s0 + (m[0] * f0 + m[kMSlice] * f1 + m[2 * kMSlice] * f2) +
                     (q[0] * t0 + q[kMSlice] * t1 + q[2 * kMSlice] * t2);
        const T z1 = s1 + (m[3 * kMSlice] * f0 + m[4 * kMSlice] * f1 + m[5 * kMSlice] * f2) +
                     (q[3 * kMSlice] * t0 + q[4 * kMSlice] * t1 + q[5 * kMSlice] * t2);
        const T z2 = s2 + (m[6 * kMSlice] * f0 + m[7 * kMSlice] * f1 + m[8 * kMSlice] * f2) +
                     (q[6 * kMSlice] * t0 + q[7 * kMSlice] * t1 + q[8 * kMSlice] * t2);
        yr[0] = z0; yr[k] = z1; yr[2 * k] = z2;
        if constexpr (MODE == MODE_POST2_DOT) d0 += to_d(f0) * z0 + to_d(f1) * z1 + to_d(f2) * z2;
    } else {
        const T *fr = F + 3 * row * k + j;
        const T f0 = fr[0], f1 = fr[k], f2 = fr[2 * k];
        const T e0 = f0 - s0, e1 = f1 - s1, e2 = f2 - s2;
        if constexpr (MODE == MODE_RESID || MODE == MODE_RESID_NORM) {
            yr[0] = e0; yr[k] = e1; yr[2 * k] = e2;
            if constexpr (MODE == MODE_RESID_NORM) {
                d0 += to_d(f0) * f0 + to_d(f1) * f1 + to_d(f2) * f2;
                d1 += to_d(e0) * e0 + to_d(e1) * e1 + to_d(e2) * e2;
            }
        } else {
            const T *m = M + (row / kMSlice) * (9 * kMSlice) + (row % kMSlice);
            const T *xr = X + 3 * row * k + j;
            const T z0 = xr[0] + (m[0] * e0 + m[kMSlice] * e1 + m[2 * kMSlice] * e2);
            const T z1 = xr[k] + (m[3 * kMSlice] * e0 + m[4 * kMSlice] * e1 + m[5 * kMSlice] * e2);
            const T z2 = xr[2 * k] + (m[6 * kMSlice] * e0 + m[7 * kMSlice] * e1 + m[8 * kMSlice] * e2);
            yr[0] = z0; yr[k] = z1; yr[2 * k] = z2;
            if constexpr (MODE == MODE_SMOOTH_DOT) d0 += to_d(f0) * z0 + to_d(f1) * z1 + to_d(f2) * z2;
        }
    }
}

// Products of the staged blocks [0, nb) of one row with the input columns:
// lane group g takes blocks g, g + L, ... (four per step, their twelve gathers
// issued together; the blocks reach the two accumulators s and u in the same
// order in both loops).
template <typename T>
__device__ __forceinline__ void spmm_chunk(const T *__restrict__ sv_, const int32_t *__restrict__ sc_, int nb,
                                           int g, int L, const T *__restrict__ X, int k, int j, T &s0, T &s1,
                                           T &s2, T &u0, T &u1, T &u2) {
    int b = g;
    // four blocks per step, their twelve gathers issued together (the blocks
    // reach the two accumulators in the same order as in the loop below)
    for (; b + 3 * L < nb; b += 4 * L) {
        const T *sa = &sv_[9 * b];
        const T *sb = &sv_[9 * (b + L)];
        const T *sc = &sv_[9 * (b + 2 * L)];
        const T *sd = &sv_[9 * (b + 3 * L)];
        const T *pa = X + 3 * (int64_t)sc_[b] * k + j;
        const T *pb = X + 3 * (int64_t)sc_[b + L] * k + j;
        const T *pc = X + 3 * (int64_t)sc_[b + 2 * L] * k + j;
        const T *pd = X + 3 * (int64_t)sc_[b + 3 * L] * k + j;
        const T a0 = pa[0], a1 = pa[k], a2 = pa[2 * k];
        const T b0 = pb[0], b1 = pb[k], b2 = pb[2 * k];
        const T c0 = pc[0], c1 = pc[k], c2 = pc[2 * k];
        const T e0 = pd[0], e1 = pd[k], e2 = pd[2 * k];
        s0 = fma(sa[0], a0, fma(sa[1], a1, fma(sa[2], a2, s0)));
        s1 = fma(sa[3], a0, fma(sa[4], a1, fma(sa[5], a2, s1)));
        s2 = fma(sa[6], a0, fma(sa[7], a1, fma(sa[8], a2, s2)));
        u0 = fma(sb[0], b0, fma(sb[1], b1, fma(sb[2], b2, u0)));
        u1 = fma(sb[3], b0, fma(sb[4], b1, fma(sb[5], b2, u1)));
        u2 = fma(sb[6], b0, fma(sb[7], b1, fma(sb[8], b2, u2)));
        s0 = fma(sc[0], c0, fma(sc[1], c1, fma(sc[2], c2, s0)));
        s1 = fma(sc[3], c0, fma(sc[4], c1, fma(sc[5], c2, s1)));
        s2 = fma(sc[6], c0, fma(sc[7], c1, fma(sc[8], c2, s2)));
        u0 = fma(sd[0], e0, fma(sd[1], e1, fma(sd[2], e2, u0)));
        u1 = fma(sd[3], e0, fma(sd[4], e1, fma(sd[5], e2, u1)));
        u2 = fma(sd[6], e0, fma(sd[7], e1, fma(sd[8], e2, u2)));
    }
    for (; b < nb; b += 2 * L) {
        {
            const T *sv = &sv_[9 * b];
            const T *xc = X + 3 * (int64_t)sc_[b] * k + j;
            const T x0 = xc[0], x1 = xc[k], x2 = xc[2 * k];
            s0 = fma(sv[0], x0, fma(sv[1], x1, fma(sv[2], x2, s0)));
            s1 = fma(sv[3], x0, fma(sv[4], x1, fma(sv[5], x2, s1)));
            s2 = fma(sv[6], x0, fma(sv[7], x1, fma(sv[8], x2, s2)));
        }
        if (b + L < nb) {
            const T *sv = &sv_[9 * (b + L)];
            const T *xc = X + 3 * (int64_t)sc_[b + L] * k + j;
            const T x0 = xc[0], x1 = xc[k], x2 = xc[2 * k];
            u0 = fma(sv[0], x0, fma(sv[1], x1, fma(sv[2], x2, u0)));
            u1 = fma(sv[3], x0, fma(sv[4], x1, fma(sv[5], x2, u1)));
            u2 = fma(sv[6], x0, fma(sv[7], x1, fma(sv[8], x2, u2)));
        }
    }
}

// One 32-lane half-wavefront per block row.  With kp = the power of two >= k,
// lane l serves column j = l % kp and takes every (32/kp)-th staged block of
// the row starting at l / kp (four per step, then two); the partial sums of a
// column's lanes are added by shuffles, and the lanes with l < kp write the
// row.  The tile and chunk loops have uniform trip counts per workgroup (the
// chunk count comes from the operator's longest row), so every thread reaches
// every barrier.
//
// FP32 and BF16 instantiations ask for six waves per SIMD: they fit in 67-74
// VGPRs without spills (seven waves for most modes, five to four before), and
// more resident waves keep more of the gathers in flight.  FP64 would spill
// at five, so it keeps the compiler's choice, and so does the plain product
// (the restriction, whose long rows ran slower with the extra waves).
template <typename V, typename T, int MODE>
constexpr int spmm_min_waves() { return (sizeof(T) == 8 || MODE == MODE_SPMV) ? 1 : 6; }

template <typename V, typename T, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(spmm_min_waves<V, T, MODE>(), 8)))
void k_spmm(SellView<V> A, int C, int k, int kp, const T *__restrict__ X, const T *__restrict__ F,
            T *__restrict__ Y, const T *__restrict__ M, double *partials, MState *st, int gated) {
    if (gated && st->all_done) return;
    __shared__ T sval[kRowsPerBlockM][kStage * 9];
    __shared__ int32_t scol[kRowsPerBlockM][kStage];
    const int hw = threadIdx.x >> 5;
    const int lane = threadIdx.x & 31;
    const int j = lane & (kp - 1);
    const int g = lane / kp;
    const int L = 32 / kp;
    const bool col_on = j < k && !(gated && st->done[j]);
    const int64_t ntiles = ((int64_t)A.rows + kRowsPerBlockM - 1) / kRowsPerBlockM;
    const int nchunks = (A.maxlen + kStage - 1) / kStage;
    double d0 = 0.0, d1 = 0.0;
    // tiles of 8 rows: this XCD's range, strided by its workgroups
    const TileRange tr = xcd_range_m(blockIdx.x, gridDim.x, ntiles);
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
    const int64_t pos = tile * kRowsPerBlockM + hw;
    const bool has_row = pos < A.rows;
    const bool on = has_row && col_on;
    const int64_t row = has_row ? (A.perm ? (int64_t)A.perm[pos] : pos) : 0;
    const int len = has_row ? A.rowlen[pos] : 0;
    const int r = (int)(pos % C);
    const int64_t base = has_row ? (int64_t)A.slice_ptr[pos / C] : 0;
    T s0 = 0, s1 = 0, s2 = 0;
    T u0 = 0, u1 = 0, u2 = 0;
    for (int ch = 0; ch < nchunks; ++ch) {
        const int k0 = ch * kStage;
        const int nb = min(kStage, len - k0);  // <= 0 once the row is done
        for (int v = lane; v < kStage * 9; v += 32) {
            const int b = v / 9, e = v - 9 * b;
            if (b < nb) {
                const int64_t rec = (base + k0 + b) * C + r;
                sval[hw][v] = cvt_v<V, T>(elem_ptr(A, rec, e));
            }
        }
        if (lane < nb) scol[hw][lane] = A.col[(base + k0 + lane) * C + r];
        __syncthreads();
        if (on) spmm_chunk<T>(sval[hw], scol[hw], nb, g, L, X, k, j, s0, s1, s2, u0, u1, u2);
        __syncthreads();
    }
    s0 += u0;
    s1 += u1;
    s2 += u2;
    // add the lanes of each column (offsets below 32 stay inside the half-wave)
    for (int off = kp; off < 32; off <<= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
        s2 += __shfl_xor(s2, off, 64);
    }
    if (on && g == 0) spmm_row_out<T, MODE>(row, j, k, s0, s1, s2, X, F, Y, M, d0, d1);
    }
    if constexpr (MODE == MODE_SPMV_DOT || MODE == MODE_SMOOTH_DOT || MODE == MODE_RESID_NORM ||
                  MODE == MODE_POST_DOT || MODE == MODE_POST2_DOT)
        mreduce(d0, d1, partials);
}

// Long rows (restrictions and the coarse operators, whose rows hold many
// blocks while the operator has few rows): one workgroup per block row.  The
// eight half-wavefronts take the row's blocks kStageLong at a time in turn
// (half-wave h stages and multiplies blocks h*kStageLong ... of each round of
// 8*kStageLong), their sums are added in LDS in fixed half-wave order, and
// half-wave 0 applies the epilogue.  Every thread works on the same row, so
// the rounds (from that row's length) and barriers are the same for all.
constexpr int kStageLong = 8;

template <typename V, typename T, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(spmm_min_waves<V, T, MODE>(), 8)))
void k_spmm_long(SellView<V> A, int C, int k, int kp, const T *__restrict__ X, const T *__restrict__ F,
                 T *__restrict__ Y, const T *__restrict__ M, double *partials, MState *st, int gated) {
    if (gated && st->all_done) return;
    __shared__ T sval[kRowsPerBlockM][kStageLong * 9];
    __shared__ int32_t scol[kRowsPerBlockM][kStageLong];
    __shared__ T red[kRowsPerBlockM][3][32];
    const int hw = threadIdx.x >> 5;
    const int lane = threadIdx.x & 31;
    const int j = lane & (kp - 1);
    const int g = lane / kp;
    const int L = 32 / kp;
    const bool col_on = j < k && !(gated && st->done[j]);
    const int per_round = kRowsPerBlockM * kStageLong;
    double d0 = 0.0, d1 = 0.0;
    // one row per workgroup: this XCD's range of rows, strided by its workgroups
    const TileRange tr = xcd_range_m(blockIdx.x, gridDim.x, A.rows);
    for (int64_t pos = tr.first; pos < tr.end; pos += tr.step) {
        const int64_t row = A.perm ? (int64_t)A.perm[pos] : pos;
        const int len = A.rowlen[pos];
        const int r = (int)(pos % C);
        const int64_t base = (int64_t)A.slice_ptr[pos / C];
        const int nrounds = (len + per_round - 1) / per_round;  // the whole workgroup's row
        T s0 = 0, s1 = 0, s2 = 0;
        T u0 = 0, u1 = 0, u2 = 0;
        for (int rd = 0; rd < nrounds; ++rd) {
            const int k0 = rd * per_round + hw * kStageLong;
            const int nb = min(kStageLong, len - k0);  // <= 0 past the row's end
            for (int v = lane; v < kStageLong * 9; v += 32) {
                const int b = v / 9, e = v - 9 * b;
                if (b < nb) {
                    const int64_t rec = (base + k0 + b) * C + r;
                    sval[hw][v] = cvt_v<V, T>(elem_ptr(A, rec, e));
                }
            }
            if (lane < nb) scol[hw][lane] = A.col[(base + k0 + lane) * C + r];
            __syncthreads();
            if (col_on) spmm_chunk<T>(sval[hw], scol[hw], nb, g, L, X, k, j, s0, s1, s2, u0, u1, u2);
            __syncthreads();
        }
        s0 += u0;
        s1 += u1;
        s2 += u2;
        for (int off = kp; off < 32; off <<= 1) {
            s0 += __shfl_xor(s0, off, 64);
            s1 += __shfl_xor(s1, off, 64);
            s2 += __shfl_xor(s2, off, 64);
        }
        if (g == 0) {
            red[hw][0][j] = s0;
            red[hw][1][j] = s1;
            red[hw][2][j] = s2;
        }
        __syncthreads();
        if (hw == 0 && g == 0 && col_on) {
            T t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
            for (int h = 0; h < kRowsPerBlockM; ++h) {
                t0 += red[h][0][j];
                t1 += red[h][1][j];
                t2 += red[h][2][j];
            }
            spmm_row_out<T, MODE>(row, j, k, t0, t1, t2, X, F, Y, M, d0, d1);
        }
        __syncthreads();  // red is written again for the next row
    }
    if constexpr (MODE == MODE_SPMV_DOT || MODE == MODE_SMOOTH_DOT || MODE == MODE_RESID_NORM ||
                  MODE == MODE_POST_DOT || MODE == MODE_POST2_DOT)
        mreduce(d0, d1, partials);
}

// Vector-column form (k a multiple of VW, X aligned to 16 bytes): each lane
// owns VW adjacent columns and loads them as one 16-byte vector per block row
// of a gathered block column (VW = 2 FP64 values), so a lane keeps 16 bytes
// in flight per load instead of one value.  kpv = kp / VW lanes
// cover the row's columns; the L = 32 / kpv lane groups split the row's
// blocks (two per step) and are added by shuffles, as in k_spmm.  Two
// blocks per step keep the kernel within 96 VGPRs, five wavefronts per SIMD
// (four blocks per step needed 123 and ran 10% slower at four wavefronts);
// the order in which a lane adds its blocks is the same either way.
template <typename T, int VW>
struct VecOf;
template <>
struct VecOf<double, 2> {
    typedef double type __attribute__((ext_vector_type(2)));
};

// acc + a0 x0 + a1 x1 + a2 x2 per component, in the order of the scalar kernel
template <int VW, typename T, typename TV>
__device__ __forceinline__ TV vfma3(const TV &acc, T a0, T a1, T a2, const TV &x0, const TV &x1, const TV &x2) {
    TV r;
#pragma unroll
    for (int v = 0; v < VW; ++v) r[v] = fma(a0, x0[v], fma(a1, x1[v], fma(a2, x2[v], acc[v])));
    return r;
}

// Per-column sums -> partials[block][2][32] (as mreduce) when the lane that
// holds column j's sums is not lane j: `owner` lanes hold column j.
__device__ __forceinline__ void mreduce_cols(double d0, double d1, bool owner, int j, double *partials) {
    __shared__ double l0[kRowsPerBlockM][32];
    __shared__ double l1[kRowsPerBlockM][32];
    const int hw = threadIdx.x >> 5, lane = threadIdx.x & 31;
    l0[hw][lane] = 0.0;
    l1[hw][lane] = 0.0;
    __syncthreads();
    if (owner) {
        l0[hw][j] = d0;
        l1[hw][j] = d1;
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int h = 0; h < kRowsPerBlockM; ++h) {
            s0 += l0[h][threadIdx.x];
            s1 += l1[h][threadIdx.x];
        }
        partials[(int64_t)blockIdx.x * 64 + threadIdx.x] = s0;
        partials[(int64_t)blockIdx.x * 64 + 32 + threadIdx.x] = s1;
    }
}

// component v of a vector by a select chain (no dynamic register indexing)
template <int VW, typename TV>
__device__ __forceinline__ auto pick(const TV &x, int v) -> decltype(x[0] + 0) {
    auto r = x[0];
#pragma unroll
    for (int q = 1; q < VW; ++q)
        if (v == q) r = x[q];
    return r;
}

template <typename V, typename T, int MODE, int VW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5, 8)))
void k_spmm_v(SellView<V> A, int C, int k, int kpv, const T *__restrict__ X, const T *__restrict__ F,
              T *__restrict__ Y, const T *__restrict__ M, double *partials, MState *st, int gated) {
    using TV = typename VecOf<T, VW>::type;
    if (gated && st->all_done) return;
    __shared__ T sval[kRowsPerBlockM][kStage * 9];
    __shared__ int32_t scol[kRowsPerBlockM][kStage];
    const int hw = threadIdx.x >> 5;
    const int lane = threadIdx.x & 31;
    const int jv = lane & (kpv - 1);
    const int g = lane / kpv;
    const int L = 32 / kpv;
    const int j0 = VW * jv;
    bool any = false;  // some column of this lane's vector is live
#pragma unroll
    for (int v = 0; v < VW; ++v) any = any || (j0 + v < k && !(gated && st->done[j0 + v]));
    // after the butterfly below every lane group holds the full sums, and
    // group g < VW writes column j0 + g: the epilogue keeps one column per lane
    // and the half-wave's 32 lanes cover 32 adjacent columns (L >= VW since kp <= 32)
    const int jo = j0 + g;
    const bool out_col = g < VW && jo < k && !(gated && st->done[jo]);
    const int64_t ntiles = ((int64_t)A.rows + kRowsPerBlockM - 1) / kRowsPerBlockM;
    const int nchunks = (A.maxlen + kStage - 1) / kStage;
    double d0 = 0.0, d1 = 0.0;
    // tiles of 8 rows: this XCD's range, strided by its workgroups
    const TileRange tr = xcd_range_m(blockIdx.x, gridDim.x, ntiles);
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
        const int64_t pos = tile * kRowsPerBlockM + hw;
        const bool has_row = pos < A.rows;
        const bool on = has_row && any;
        const int64_t row = has_row ? (A.perm ? (int64_t)A.perm[pos] : pos) : 0;
        const int len = has_row ? A.rowlen[pos] : 0;
        const int r = (int)(pos % C);
        const int64_t base = has_row ? (int64_t)A.slice_ptr[pos / C] : 0;
        TV s0 = {}, s1 = {}, s2 = {};
        for (int ch = 0; ch < nchunks; ++ch) {
            const int k0 = ch * kStage;
            const int nb = min(kStage, len - k0);  // <= 0 once the row is done
            for (int v = lane; v < kStage * 9; v += 32) {
                const int b = v / 9, e = v - 9 * b;
                if (b < nb) {
                    const int64_t rec = (base + k0 + b) * C + r;
                    sval[hw][v] = cvt_v<V, T>(elem_ptr(A, rec, e));
                }
            }
            if (lane < nb) scol[hw][lane] = A.col[(base + k0 + lane) * C + r];
            __syncthreads();
            if (on) {
                int b = g;
                // two blocks per step, their six vector gathers issued together
                for (; b + L < nb; b += 2 * L) {
                    const T *sa = &sval[hw][9 * b];
                    const T *sb = &sval[hw][9 * (b + L)];
                    const T *pa = X + 3 * (int64_t)scol[hw][b] * k + j0;
                    const T *pb = X + 3 * (int64_t)scol[hw][b + L] * k + j0;
                    const TV a0 = *(const TV *)pa, a1 = *(const TV *)(pa + k), a2 = *(const TV *)(pa + 2 * k);
                    const TV b0 = *(const TV *)pb, b1 = *(const TV *)(pb + k), b2 = *(const TV *)(pb + 2 * k);
                    s0 = vfma3<VW>(s0, sa[0], sa[1], sa[2], a0, a1, a2);
                    s1 = vfma3<VW>(s1, sa[3], sa[4], sa[5], a0, a1, a2);
                    s2 = vfma3<VW>(s2, sa[6], sa[7], sa[8], a0, a1, a2);
                    s0 = vfma3<VW>(s0, sb[0], sb[1], sb[2], b0, b1, b2);
                    s1 = vfma3<VW>(s1, sb[3], sb[4], sb[5], b0, b1, b2);
                    s2 = vfma3<VW>(s2, sb[6], sb[7], sb[8], b0, b1, b2);
                }
                for (; b < nb; b += L) {
                    const T *sv = &sval[hw][9 * b];
                    const T *xc = X + 3 * (int64_t)scol[hw][b] * k + j0;
                    const TV x0 = *(const TV *)xc, x1 = *(const TV *)(xc + k), x2 = *(const TV *)(xc + 2 * k);
                    s0 = vfma3<VW>(s0, sv[0], sv[1], sv[2], x0, x1, x2);
                    s1 = vfma3<VW>(s1, sv[3], sv[4], sv[5], x0, x1, x2);
                    s2 = vfma3<VW>(s2, sv[6], sv[7], sv[8], x0, x1, x2);
                }
            }
            __syncthreads();
        }
        // add the lane groups of each column set (offsets below 32 stay inside the half-wave)
        for (int off = kpv; off < 32; off <<= 1) {
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                s0[v] += __shfl_xor(s0[v], off, 64);
                s1[v] += __shfl_xor(s1[v], off, 64);
                s2[v] += __shfl_xor(s2[v], off, 64);
            }
        }
        if (has_row && out_col)
            spmm_row_out<T, MODE>(row, jo, k, pick<VW>(s0, g), pick<VW>(s1, g), pick<VW>(s2, g), X, F, Y, M, d0,
                                  d1);
    }
    if constexpr (MODE == MODE_SPMV_DOT || MODE == MODE_SMOOTH_DOT || MODE == MODE_RESID_NORM ||
                  MODE == MODE_POST_DOT || MODE == MODE_POST2_DOT)
        mreduce_cols(d0, d1, out_col, jo, partials);
}

// x = M f for every column (first smoothing sweep from zero)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi0_m(int64_t rows, int k, const T *__restrict__ M,
                                                      const T *__restrict__ f, T *__restrict__ x, MState *st,
                                                      int gated) {
    if (gated && st->all_done) return;
    const int64_t row = (int64_t)blockIdx.x * kRowsPerBlockM + (threadIdx.x >> 5);
    const int j = threadIdx.x & 31;
    if (row >= rows || j >= k) return;
    const T *m = M + (row / kMSlice) * (9 * kMSlice) + (row % kMSlice);
    const T *fr = f + 3 * row * k + j;
    const T e0 = fr[0], e1 = fr[k], e2 = fr[2 * k];
    T *xr = x + 3 * row * k + j;
    xr[0] = m[0] * e0 + m[kMSlice] * e1 + m[2 * kMSlice] * e2;
    xr[k] = m[3 * kMSlice] * e0 + m[4 * kMSlice] * e1 + m[5 * kMSlice] * e2;
    xr[2 * k] = m[6 * kMSlice] * e0 + m[7 * kMSlice] * e1 + m[8 * kMSlice] * e2;
}

// Y = Ainv F on the coarsest level with FP64 matrix cores.  Each wavefront
// owns one 16x16 tile of Y and one of S slices of the inner dimension
// (split-K: S = up to 16 slices so that a few thousand wavefronts stream Ainv),
// v_mfma_f64_16x16x4f64 over k-steps of 4 with two accumulator chains; a second
// kernel adds the S partial tiles in fixed order.  Operand layout per lane l:
// A element (row l % 16, k l / 16), B element (k l / 16, column l % 16);
// accumulator entry v (v = 0..3) holds row 4 v + l / 16, column l % 16 (layout
// measured on gfx950).
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_gemm_part(int n, int k, int S, const double *__restrict__ Ainv,
                                                            const T *__restrict__ F, double *__restrict__ part,
                                                            MState *st, int gated) {
    if (gated && st->all_done) return;
    const int lane = threadIdx.x & 63;
    const int tiles_k = (k + 15) / 16;
    const int tiles = ((n + 15) / 16) * tiles_k;
    const int w = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (w >= tiles * S) return;
    const int t = w % tiles, sl = w / tiles;
    const int ti = t / tiles_k, tj = t % tiles_k;
    const int i = ti * 16 + (lane & 15);
    const int kq = lane >> 4;
    const int j = tj * 16 + (lane & 15);
    // inner range of this slice, a multiple of 8 long (two k-steps per pass)
    const int steps = (n + 7) / 8;
    const int per = (steps + S - 1) / S;
    const int q_lo = sl * per * 8, q_hi = min(n, (sl + 1) * per * 8);
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    for (int q0 = q_lo; q0 < q_hi; q0 += 8) {
        const int qa = q0 + kq, qb = q0 + 4 + kq;
        const double a0 = (i < n && qa < q_hi) ? Ainv[(int64_t)i * n + qa] : 0.0;
        const double a1 = (i < n && qb < q_hi) ? Ainv[(int64_t)i * n + qb] : 0.0;
        const double b0 = (qa < q_hi && j < k) ? to_d(F[(int64_t)qa * k + j]) : 0.0;
        const double b1 = (qb < q_hi && j < k) ? to_d(F[(int64_t)qb * k + j]) : 0.0;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
    }
    // partial tile, layout [slice][row][16 * tiles_k]
    const int ld = 16 * tiles_k;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = ti * 16 + 4 * v + kq;
        if (row < n) part[((int64_t)sl * n + row) * ld + j] = acc0[v] + acc1[v];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_gemm_sum(int n, int k, int S, const double *__restrict__ part,
                                                           T *__restrict__ Y, MState *st, int gated) {
    if (gated && st->all_done) return;
    const int ld = 16 * ((k + 15) / 16);
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)n * k) return;
    const int64_t row = idx / k;
    const int j = (int)(idx % k);
    double s = 0.0;
    for (int sl = 0; sl < S; ++sl) s += part[((int64_t)sl * n + row) * ld + j];
    Y[idx] = (T)s;
}

// Outer FP64 CG update for every column not yet done: x += a_j p,
// r -= a_j q, ||r_j||^2 (and r_j . z_old,j), the V-cycle copy rv of r and the
// level-1 pre-smoothing sweep x1 = M rv.
template <typename TV>
__global__ __launch_bounds__(kBlock) void k_cg_update_m(int64_t rows, int k, double *__restrict__ x,
                                                        const double *__restrict__ p, double *__restrict__ r,
                                                        const double *__restrict__ q, const TV *__restrict__ M,
                                                        TV *__restrict__ rv, TV *__restrict__ x1,
                                                        const TV *__restrict__ zold, double *partials,
                                                        MState *st) {
    if (st->all_done) return;
    const int j = threadIdx.x & 31;
    const bool col_on = j < k && !st->done[j];
    double d0 = 0.0, d1 = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * kRowsPerBlockM + (threadIdx.x >> 5); row < rows;
         row += (int64_t)gridDim.x * kRowsPerBlockM) {
    if (col_on) {
        const double alpha = st->alpha[j];
        TV e[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t i = (3 * row + c) * k + j;
            x[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            d0 += ri * ri;
            e[c] = (TV)ri;
            rv[i] = e[c];
            if (zold) d1 += to_d(e[c]) * zold[i];
        }
        if (M) {
            const TV *m = M + (row / kMSlice) * (9 * kMSlice) + (row % kMSlice);
            TV *xr = x1 + 3 * row * k + j;
            xr[0] = m[0] * e[0] + m[kMSlice] * e[1] + m[2 * kMSlice] * e[2];
            xr[k] = m[3 * kMSlice] * e[0] + m[4 * kMSlice] * e[1] + m[5 * kMSlice] * e[2];
            xr[2 * k] = m[6 * kMSlice] * e[0] + m[7 * kMSlice] * e[1] + m[8 * kMSlice] * e[2];
        }
    }
    }
    mreduce(d0, d1, partials);
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_cg_dir_m(int64_t n, int k, const TV *__restrict__ z,
                                                     double *__restrict__ p, MState *st) {
    if (st->all_done) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n * k) return;
    const int j = (int)(i % k);
    if (st->done[j]) return;
    p[i] = to_d(z[i]) + st->beta[j] * p[i];
}

// One workgroup of 32 x 32 threads: thread (t, j) sums the partials of
// column j over blocks t, t+32, ... in order (loading eight blocks' partials
// before adding them, so the loads overlap), the 32 sums of a column are then
// added in order (deterministic), and the CG scalar update of `site` is
// applied; finally the all-done flag is refreshed.
__global__ __launch_bounds__(1024) void k_mfinalize(const double *__restrict__ partials, int nblk, MState *st,
                                                    int gated, int site) {
    if (gated && st->all_done) return;
    __shared__ double l0[32][33];
    __shared__ double l1[32][33];
    __shared__ int any_running;
    const int j = threadIdx.x & 31, t = threadIdx.x >> 5;
    double a0 = 0.0, a1 = 0.0;
    int b = t;
    for (; b + 7 * 32 < nblk; b += 8 * 32) {
        double p0[8], p1[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double *pp = partials + (int64_t)(b + 32 * q) * 64 + j;
            p0[q] = pp[0];
            p1[q] = pp[32];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            a0 += p0[q];
            a1 += p1[q];
        }
    }
    for (; b < nblk; b += 32) {
        a0 += partials[(int64_t)b * 64 + j];
        a1 += partials[(int64_t)b * 64 + 32 + j];
    }
    l0[t][j] = a0;
    l1[t][j] = a1;
    if (threadIdx.x == 0) any_running = 0;
    __syncthreads();
    if (threadIdx.x < 32 && j < st->k && !(gated && st->done[j])) {
        double t0 = 0.0, t1 = 0.0;
        for (int q = 0; q < 32; ++q) {
            t0 += l0[q][j];
            t1 += l1[q][j];
        }
        switch (site) {
            case MSITE_PQ:
                st->pq[j] = t0;
                if (!(t0 > 0.0)) {
                    st->status[j] = isfinite(t0) ? ST_BREAKDOWN : ST_NONFINITE;
                    st->done[j] = 1;
                } else {
                    st->alpha[j] = st->rz[j] / t0;
                }
                break;
            case MSITE_RR:
                st->rr[j] = t0;
                st->rz_prev[j] = t1;
                st->iter[j] += 1;
                if (!isfinite(t0)) {
                    st->status[j] = ST_NONFINITE;
                    st->done[j] = 1;
                } else if (t0 <= st->tol2bb[j]) {
                    st->status[j] = ST_CONVERGED;
                    st->done[j] = 1;
                } else if (st->iter[j] >= st->maxiter) {
                    st->status[j] = ST_MAXITER;
                    st->done[j] = 1;
                }
                break;
            case MSITE_RZ:
                st->beta[j] = st->flexible ? (t0 - st->rz_prev[j]) / st->rz[j] : t0 / st->rz[j];
                st->rz[j] = t0;
                break;
            case MSITE_RZ0:
                st->rz[j] = t0;
                break;
            case MSITE_INIT:
                st->bb[j] = t0;
                st->rr[j] = t1;
                break;
            default:
                break;
        }
    }
    __syncthreads();
    if (threadIdx.x < 32 && j < st->k && !st->done[j]) atomicOr(&any_running, 1);
    __syncthreads();
    if (threadIdx.x == 0) st->all_done = any_running ? 0 : 1;
}

__global__ void k_mstate_init(MState *st, int k, int maxiter, int flexible) {
    const int j = threadIdx.x;
    if (j < kMaxRhs) {
        st->rz[j] = st->pq[j] = st->rr[j] = st->bb[j] = st->alpha[j] = st->beta[j] = st->rz_prev[j] = 0.0;
        st->tol2bb[j] = 0.0;
        st->iter[j] = 0;
        st->done[j] = j < k ? 0 : 1;
        st->status[j] = ST_RUNNING;
    }
    if (j == 0) {
        st->all_done = 0;
        st->k = k;
        st->maxiter = maxiter;
        st->flexible = flexible;
    }
}

// after the initial residuals: per-column targets; zero right-hand sides and
// columns already below the target are done
__global__ void k_mstate_arm(MState *st, double tol) {
    const int j = threadIdx.x;
    __shared__ int any_running;
    if (j == 0) any_running = 0;
    __syncthreads();
    if (j < st->k) {
        st->tol2bb[j] = tol * tol * st->bb[j];
        const bool fin = st->bb[j] == 0.0 || st->rr[j] <= st->tol2bb[j];
        st->done[j] = fin ? 1 : 0;
        st->status[j] = fin ? ST_CONVERGED : ST_RUNNING;
        if (!fin) atomicOr(&any_running, 1);
    }
    __syncthreads();
    if (j == 0) st->all_done = any_running ? 0 : 1;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// Grid bound of the multi-column kernels: at most kMaxMGrid workgroups
// striding over the rows, so the per-column dot products leave few partial
// sums (the partials buffers are sized by it); a launch takes no more than the
// device holds at once (spmm_resident).
int spmm_grid(int rows) { return std::min((rows + kRowsPerBlockM - 1) / kRowsPerBlockM, kMaxMGrid); }

// k_spmm_long takes operators whose rows hold more than kLongRow blocks on
// average and whose gathered input (cols x 3 x k values) fits one XCD's L2.
// Measured on the 48^3 cube at 32 FP32 columns: level-2 restriction (476 rows
// of 154 blocks) 69 -> 16 us, level-2 residual (9,378 rows of 58) 52 -> 39 us;
// the level-1 restriction (rows of 104 blocks, but a 45 MB input) went
// 56 -> 64 us and the level-2 post-sweep (rows of 25) 23 -> 32 us, so those
// stay with k_spmm.
constexpr int kLongRow = 32;
constexpr int64_t kLongInputBytes = 4 << 20;

// Fixed-order sums of contiguous ranges of per-workgroup partials (one range
// per workgroup), so that the one-workgroup finalize reads kMSplit entries
// instead of up to kMaxMGrid: a single CU reading the ~1 MB of a full grid's
// partials took about 15 us per finalize.
__global__ __launch_bounds__(kBlock) void k_mpartial(const double *__restrict__ partials, int nblk,
                                                     double *__restrict__ out, const MState *st, int gated) {
    if (gated && st->all_done) return;
    const int s = blockIdx.x, S = gridDim.x;
    const int b0 = (int)((int64_t)nblk * s / S), b1 = (int)((int64_t)nblk * (s + 1) / S);
    const int e = threadIdx.x & 63, grp = threadIdx.x >> 6;
    double a = 0.0;
    for (int b = b0 + grp; b < b1; b += kBlock / 64) a += partials[(int64_t)b * 64 + e];
    __shared__ double l[kBlock / 64][64];
    l[grp][e] = a;
    __syncthreads();
    if (threadIdx.x < 64) {
        double t = 0.0;
#pragma unroll
        for (int g = 0; g < kBlock / 64; ++g) t += l[g][threadIdx.x];
        out[(int64_t)s * 64 + threadIdx.x] = t;
    }
}

// partials holds kMaxMGrid + kMSplit entries of 64 values: the per-workgroup
// sums, then the range sums of k_mpartial
static void launch_mfinalize(double *partials, int nblk, MState *st, int gated, int site, hipStream_t s) {
    if (nblk > 2 * kMSplit) {
        double *ranges = partials + (size_t)kMaxMGrid * 64;
        hipLaunchKernelGGL(k_mpartial, dim3(kMSplit), dim3(kBlock), 0, s, partials, nblk, ranges, st, gated);
        partials = ranges;
        nblk = kMSplit;
    }
    hipLaunchKernelGGL(k_mfinalize, dim3(1), dim3(1024), 0, s, partials, nblk, st, gated, site);
}

// Workgroups of k_spmm<V, T, MODE> that the whole device holds at once
// (occupancy API, taken once per instantiation; every device of a process is
// the same part).  A grid beyond it would run a second, mostly idle round of
// workgroups after the first.  Contexts on other threads may ask at the same
// time: they compute the same value, and the atomic keeps that race defined.
template <typename Kernel>
static int resident_of(Kernel kernel, std::atomic<int> &resident) {
    int r = resident.load(std::memory_order_relaxed);
    if (r == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || cus <= 0 ||
            per_cu <= 0)
            return kMaxMGrid;
        r = cus * per_cu;
        resident.store(r, std::memory_order_relaxed);
    }
    return r;
}
template <typename V, typename T, int MODE>
static int spmm_resident() {
    static std::atomic<int> resident{0};
    return resident_of(k_spmm<V, T, MODE>, resident);
}
template <typename V, typename T, int MODE>
static int spmm_long_resident() {
    static std::atomic<int> resident{0};
    return resident_of(k_spmm_long<V, T, MODE>, resident);
}
template <typename V, typename T, int MODE, int VW>
static int spmm_v_resident() {
    static std::atomic<int> resident{0};
    return resident_of(k_spmm_v<V, T, MODE, VW>, resident);
}

template <typename V, typename T>
void launch_spmm(const SellView<V> &A, int C, int mode, int k, const T *x, const T *f, T *y, const T *M,
                 double *partials, MState *st, int gated, int site, hipStream_t s) {
    if (C == 2) C = 1;  // row groups keep the row-wave storage: one row per slice
    int grid = spmm_grid(A.rows);
    if (grid == 0) return;
    // long rows over an L2-resident input: a workgroup per row, so that each
    // row's blocks spread over eight half-wavefronts
    const bool long_rows = A.meanlen > kLongRow && (int64_t)A.cols * 3 * k * (int64_t)sizeof(T) <= kLongInputBytes;
    int kp = 1;
    while (kp < k) kp <<= 1;
    // FP64: two columns per lane as 16-byte vectors when the columns split
    // evenly and X is aligned (FP32 keeps one column per lane: its four-column
    // vectors measured slower, 131 -> 135 us for the level-1 residual and
    // 132 -> 158 us for the fused post-sweep of the 48^3 cube at 32 columns)
    const bool vec = sizeof(T) == 8 && k % 2 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0;
    switch (mode) {
#define SAAMG_MCASE(MD)                                                                                    \
    case MD:                                                                                               \
        if (long_rows) {                                                                                   \
            grid = (int)std::min<int64_t>({(int64_t)A.rows, (int64_t)spmm_long_resident<V, T, MD>(),      \
                                           (int64_t)kMaxMGrid});                                          \
            hipLaunchKernelGGL((k_spmm_long<V, T, MD>), dim3(grid), dim3(kBlock), 0, s, A, C, k, kp, x, f, \
                               y, M, partials, st, gated);                                                 \
            break;                                                                                         \
        }                                                                                                  \
        if constexpr (sizeof(T) == 8) {                                                                    \
            if (vec) {                                                                                     \
                grid = std::min(grid, spmm_v_resident<V, T, MD, 2>());                                     \
                hipLaunchKernelGGL((k_spmm_v<V, T, MD, 2>), dim3(grid), dim3(kBlock), 0, s, A, C, k, kp / 2, \
                                   x, f, y, M, partials, st, gated);                                       \
                break;                                                                                     \
            }                                                                                              \
        }                                                                                                  \
        grid = std::min(grid, spmm_resident<V, T, MD>());                                                  \
        hipLaunchKernelGGL((k_spmm<V, T, MD>), dim3(grid), dim3(kBlock), 0, s, A, C, k, kp, x, f, y, M,    \
                           partials, st, gated);                                                           \
        break;
        SAAMG_MCASE(MODE_SPMV)
        SAAMG_MCASE(MODE_RESID)
        SAAMG_MCASE(MODE_SMOOTH)
        SAAMG_MCASE(MODE_ADD)
        SAAMG_MCASE(MODE_SPMV_DOT)
        SAAMG_MCASE(MODE_SMOOTH_DOT)
        SAAMG_MCASE(MODE_RESID_NORM)
        SAAMG_MCASE(MODE_POST)
        SAAMG_MCASE(MODE_POST_DOT)
        SAAMG_MCASE(MODE_POST2)
        SAAMG_MCASE(MODE_POST2_DOT)
#undef SAAMG_MCASE
    }
    const bool reduces = mode == MODE_SPMV_DOT || mode == MODE_SMOOTH_DOT || mode == MODE_RESID_NORM ||
                         mode == MODE_POST_DOT || mode == MODE_POST2_DOT;
    if (reduces && site != MSITE_NONE) launch_mfinalize(partials, grid, st, gated, site, s);
}

template void launch_spmm<double, double>(const SellView<double> &, int, int, int, const double *, const double *,
                                          double *, const double *, double *, MState *, int, int, hipStream_t);
template void launch_spmm<float, float>(const SellView<float> &, int, int, int, const float *, const float *,
                                        float *, const float *, double *, MState *, int, int, hipStream_t);
template void launch_spmm<bf16_t, float>(const SellView<bf16_t> &, int, int, int, const float *, const float *,
                                         float *, const float *, double *, MState *, int, int, hipStream_t);

template <typename T>
void launch_jacobi0_m(int64_t rows, int k, const T *M, const T *f, T *x, MState *st, int gated, hipStream_t s) {
    if (rows <= 0) return;
    // one block row per half-wavefront over the whole level (no grid cap: this
    // kernel has no dot product and no row loop)
    hipLaunchKernelGGL(k_jacobi0_m<T>, dim3((unsigned)((rows + kRowsPerBlockM - 1) / kRowsPerBlockM)), dim3(kBlock), 0, s,
                       rows, k, M, f, x, st,
                       gated);
}
template void launch_jacobi0_m<double>(int64_t, int, const double *, const double *, double *, MState *, int,
                                       hipStream_t);
template void launch_jacobi0_m<float>(int64_t, int, const float *, const float *, float *, MState *, int,
                                      hipStream_t);

int dense_gemm_slices(int n, int k) {
    const int tiles = ((n + 15) / 16) * ((k + 15) / 16);
    const int steps = (n + 7) / 8;
    return std::max(1, std::min({kMaxGemmSlices, 4096 / std::max(tiles, 1), steps}));
}

template <typename T>
void launch_dense_gemm(int n, int k, const double *Ainv, const T *f, T *y, double *part, MState *st, int gated,
                       hipStream_t s) {
    if (n <= 0) return;
    const int tiles = ((n + 15) / 16) * ((k + 15) / 16);
    const int S = dense_gemm_slices(n, k);
    const int waves = kBlock / 64;
    hipLaunchKernelGGL(k_dense_gemm_part<T>, dim3((tiles * S + waves - 1) / waves), dim3(kBlock), 0, s, n, k, S,
                       Ainv, f, part, st, gated);
    const int64_t nk = (int64_t)n * k;
    hipLaunchKernelGGL(k_dense_gemm_sum<T>, dim3((unsigned)((nk + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, k,
                       S, part, y, st, gated);
}
template void launch_dense_gemm<double>(int, int, const double *, const double *, double *, double *, MState *,
                                        int, hipStream_t);
template void launch_dense_gemm<float>(int, int, const double *, const float *, float *, double *, MState *, int,
                                       hipStream_t);

template <typename TV>
void launch_cg_update_m(int64_t rows, int k, double *x, const double *p, double *r, const double *q, const TV *M,
                        TV *rv, TV *x1, const TV *zold, double *partials, MState *st, hipStream_t s) {
    const int grid = spmm_grid((int)rows);
    hipLaunchKernelGGL(k_cg_update_m<TV>, dim3(grid), dim3(kBlock), 0, s, rows, k, x, p, r, q, M, rv, x1, zold,
                       partials, st);
    launch_mfinalize(partials, grid, st, 1, MSITE_RR, s);
}
template void launch_cg_update_m<double>(int64_t, int, double *, const double *, double *, const double *,
                                         const double *, double *, double *, const double *, double *, MState *,
                                         hipStream_t);
template void launch_cg_update_m<float>(int64_t, int, double *, const double *, double *, const double *,
                                        const float *, float *, float *, const float *, double *, MState *,
                                        hipStream_t);

template <typename TV>
void launch_cg_dir_m(int64_t rows, int k, const TV *z, double *p, MState *st, hipStream_t s) {
    const int64_t n = 3 * rows * k;
    hipLaunchKernelGGL(k_cg_dir_m<TV>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, 3 * rows, k, z, p, st);
}
template void launch_cg_dir_m<double>(int64_t, int, const double *, double *, MState *, hipStream_t);
template void launch_cg_dir_m<float>(int64_t, int, const float *, double *, MState *, hipStream_t);

void launch_mstate_init(MState *st, int k, int maxiter, int flexible, hipStream_t s) {
    hipLaunchKernelGGL(k_mstate_init, dim3(1), dim3(64), 0, s, st, k, maxiter, flexible);
}
void launch_mstate_arm(MState *st, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_mstate_arm, dim3(1), dim3(64), 0, s, st, tol);
}

}  // namespace saamg
