// Numeric phase of the block sparse products of the setup on the device:
// C = A B for 3x3 block CSR matrices whose product pattern was formed on the
// host (symbolic phase), used for the Galerkin product A_{l+1} = R (A P) of
// Algorithm 1.  One thread per output block (i, j): it walks row i of A in
// increasing column order and, for each block A_ik, finds j in row k of B by
// binary search, accumulating A_ik B_kj in FP64 -- the order in which the
// host product adds the same terms, so the two agree to the last bits of the
// 3x3 products.  No atomics: every output block has one writer.
#include <hip/hip_runtime.h>

#include "galerkin.hpp"

namespace saamg {

constexpr int kGBlock = 256;

__global__ __launch_bounds__(kGBlock) void k_bsr_product(int64_t nout, const int32_t *__restrict__ crow,
                                                         const int32_t *__restrict__ ccol,
                                                         const int64_t *__restrict__ aptr,
                                                         const int32_t *__restrict__ acol,
                                                         const double *__restrict__ aval,
                                                         const int64_t *__restrict__ bptr,
                                                         const int32_t *__restrict__ bcol,
                                                         const double *__restrict__ bval, double *__restrict__ cval) {
    const int64_t q = (int64_t)blockIdx.x * kGBlock + threadIdx.x;
    if (q >= nout) return;
    const int32_t i = crow[q], j = ccol[q];
    double c[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) c[e] = 0.0;
    for (int64_t ka = aptr[i]; ka < aptr[i + 1]; ++ka) {
        const int32_t k = acol[ka];
        int64_t lo = bptr[k], hi = bptr[k + 1];
        while (lo < hi) {  // first entry of row k with column >= j
            const int64_t mid = (lo + hi) >> 1;
            if (bcol[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        if (lo == bptr[k + 1] || bcol[lo] != j) continue;
        const double *a = aval + 9 * ka;
        const double *b = bval + 9 * lo;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                const double ar = a[3 * r + kk];
                c[3 * r + 0] += ar * b[3 * kk + 0];
                c[3 * r + 1] += ar * b[3 * kk + 1];
                c[3 * r + 2] += ar * b[3 * kk + 2];
            }
    }
    double *out = cval + 9 * q;
#pragma unroll
    for (int e = 0; e < 9; ++e) out[e] = c[e];
}

void launch_bsr_product(const DevBsr &A, const DevBsr &B, const int32_t *crow, const int32_t *ccol, int64_t nout,
                        double *cval, hipStream_t s) {
    if (nout <= 0) return;
    const int64_t grid = (nout + kGBlock - 1) / kGBlock;
    hipLaunchKernelGGL(k_bsr_product, dim3((unsigned)grid), dim3(kGBlock), 0, s, nout, crow, ccol, A.ptr, A.col,
                       A.val, B.ptr, B.col, B.val, cval);
}

}  // namespace saamg
