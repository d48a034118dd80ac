// HIP kernels of the solve phase (gfx950): BSR3 sliced-ELL products fused with
// residual / smoothing / dot products, CG vector updates, the dense coarsest
// solve, and deterministic device-wide reductions.
//
// Device layout of a 3x3-block matrix ("sliced ELL", one slice = C block
// rows): slot k of slice s holds the k-th block of each of its C rows; with
// rec = slot*C + r the column index of row r is col[rec].  Values (element e
// row-major in the 3x3 block) in 16-byte groups: W = 16 / sizeof(value)
// elements per group (2 FP64, 4 FP32, 8 BF16); element e < 8 sits in group
// q = e / W at val[q*gstride + rec*W + e % W] (gstride = records * W), element
// 8 in val8[rec].  A lane reads a block with one aligned 16-byte load per
// group (5 / 3 / 2 loads per block instead of 9) and the lanes of a wavefront
// read consecutive 16-byte chunks of a group, so every load instruction
// streams contiguous memory.  Row-wave operators (C = 1, where 63 lanes read
// the 9 entries of 7 blocks at once) keep each block's 9 values contiguous,
// val[rec*9 + e] (marked by gstride = 0, no val8).  A wavefront of 64 lanes serves one
// slice with G = 64/C lanes per row: lane g of a row takes blocks g, g+G, ...
// so every load instruction streams G contiguous segments of C values, and
// the G partial sums of a row are combined with cross-lane shuffles.  With
// C = 1 the layout is plain block CSR (each row's blocks contiguous) and a
// whole wavefront streams one long row; layout code 2 (row groups) keeps that
// storage and gives each row a workgroup of four wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace saamg {

constexpr int kBlock = 256;        // threads per workgroup
constexpr int kMSlice = 64;        // slice height of smoother blocks / row vectors

// ---------------------------------------------------------------------------
// value types
// ---------------------------------------------------------------------------

struct bf16_t {
    uint16_t bits;
};

// elements of a value type per 16-byte group
template <typename V>
constexpr int group_width() {
    return 16 / (int)sizeof(V);
}

__device__ __forceinline__ double to_compute(double v, double) { return v; }
__device__ __forceinline__ float to_compute(float v, float) { return v; }
__device__ __forceinline__ double to_compute(float v, double) { return (double)v; }
__device__ __forceinline__ float to_compute(bf16_t v, float) {
    return __uint_as_float(((uint32_t)v.bits) << 16);
}

template <typename V>
struct SellView {
    int32_t rows;
    int32_t nslices;
    const int32_t *__restrict__ slice_ptr;  // [nslices+1] slot offsets
    const int32_t *__restrict__ rowlen;     // [rows] blocks of the row at each slice position
    const int32_t *__restrict__ col;        // [slots*C]
    const V *__restrict__ val;              // [8 * records] elements 0..7 in 16-byte groups
    const V *__restrict__ val8;             // [records] element 8 of each block
    const int32_t *__restrict__ perm;       // [rows] row at each slice position, or null
    int32_t maxlen;                         // longest row (blocks)
    int64_t gstride;                        // elements per 16-byte group plane (records * W); 0: C = 1
    int32_t cols;                           // block columns (launch choices only)
    int32_t meanlen;                        // stored blocks / rows, rounded up (launch choices only)
};

// Address of element e of the block at record rec (see the layout above).
template <typename V>
__device__ __forceinline__ const V *elem_ptr(const SellView<V> &A, int64_t rec, int e) {
    constexpr int W = group_width<V>();
    if (A.gstride == 0) return A.val + rec * 9 + e;
    return e < 8 ? A.val + (e / W) * A.gstride + rec * W + (e % W) : A.val8 + rec;
}

// CG / reduction state resident on the device.
struct DevState {
    double rz;        // r . z of the current iterate
    double pq;        // p . A p
    double rr;        // ||r||^2
    double bb;        // ||b||^2
    double alpha;
    double beta;
    double tol2bb;    // tol^2 ||b||^2
    double rz_prev;   // r_new . z_old (flexible CG)
    int32_t iter;
    int32_t maxiter;
    int32_t done;     // gates every iteration kernel
    int32_t status;   // see StateStatus
    int32_t flexible;
};

enum StateStatus : int32_t {
    ST_RUNNING = 0,
    ST_CONVERGED = 1,   // recursive residual met the target
    ST_BREAKDOWN = 2,
    ST_NONFINITE = 3,
    ST_MAXITER = 4,
};

// What the last block of a reduction does with the device-wide sum.
enum ReduceSite : int32_t {
    SITE_NONE = 0,
    SITE_PQ = 1,      // alpha = rz / pq
    SITE_RR = 2,      // iteration count, convergence test
    SITE_RZ = 3,      // beta = rz_new / rz
    SITE_INIT = 4,    // (bb, rr) of the initial residual
    SITE_RZ0 = 5,     // first r . z (no beta)
    SITE_TRUE = 6,    // true residual norm into rr
    SITE_RZOLD = 7,   // r_new . z_old (flexible CG), stored for SITE_RZ
};

enum SellMode : int32_t {
    MODE_SPMV = 0,        // y = A x
    MODE_RESID = 1,       // y = f - A x
    MODE_SMOOTH = 2,      // y = x + M (f - A x)
    MODE_ADD = 3,         // y += A x
    MODE_SPMV_DOT = 4,    // y = A x, reduce x . y
    MODE_SMOOTH_DOT = 5,  // y = x + M (f - A x), reduce f . y
    MODE_RESID_NORM = 6,  // y = f - A x, reduce (f . f, y . y)
    MODE_POST = 7,        // y = A x + M (f + y): y holds t on entry (fused post-sweep)
    MODE_POST_DOT = 8,    // same + reduce f . y (level 1)
    MODE_POST2 = 9,       // y = A x + M f + Mt y with M, Mt in one 18-entry planar array (block SPAI-0)
    MODE_POST2_DOT = 10,  // same + reduce f . y (level 1)
    MODE_MSOLVE = 11,     // y = M (f - A x); y may alias x when A never reads the rows it writes
                          // (a colour pass of a block triangular solve)
    MODE_POSTP = 12,      // MODE_POST with M stored in the operator's slice-position order
    MODE_POSTP_DOT = 13,  // same + reduce f . y (level 1)
};

}  // namespace saamg
