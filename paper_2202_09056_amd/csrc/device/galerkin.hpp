// Device numeric phase of the setup's block sparse products (galerkin.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace saamg {

// A 3x3 block CSR matrix in device memory (plain layout: row offsets, sorted
// block columns, 9 row-major values per block).
struct DevBsr {
    int32_t rows = 0;
    const int64_t *ptr = nullptr;
    const int32_t *col = nullptr;
    const double *val = nullptr;
};

// cval[q] = sum_k A(crow[q], k) B(k, ccol[q]) for the nout output blocks of a
// product pattern (blocks of C in row-major order: crow is the row of each).
void launch_bsr_product(const DevBsr &A, const DevBsr &B, const int32_t *crow, const int32_t *ccol, int64_t nout,
                        double *cval, hipStream_t s);

}  // namespace saamg
