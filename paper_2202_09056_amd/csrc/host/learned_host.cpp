// Host inputs of the learned level-1 smoother blocks, built with the
// hierarchy (FP64, then stored as the device consumes them).
//
// Features of node i (90, scale free): the diagonal block D_i / ||D_i||_F
// (row-major) and, for every stored block A_ij, the diagonal of A_ij divided
// by ||D_i||_F at the slot k = 9 (sx+1) + 3 (sy+1) + (sz+1) given by the signs
// of the coordinate differences x_j - x_i (a difference within 1e-8 of the
// largest bounding-box extent counts as 0); empty slots are 0.  A node with
// two neighbours in one slot is not a brick-grid node: AMG_ERR_UNSUPPORTED.
// Cholesky factors: M_i = L_i L_i^T of the block-Jacobi block, lower triangle
// stored as (L00, L10, L11, L20, L21, L22).
#include <algorithm>
#include <array>
#include <cmath>

#include "setup_internal.hpp"

namespace saamg {

void learned_inputs(const Bsr3 &A, const double *coords, const std::vector<double> &Minv,
                    std::vector<float> &phi, std::vector<double> &Lchol, int nthreads) {
    const int32_t nb = A.rows;
    if (!coords) throw AmgError{AMG_ERR_ARG, "the learned smoother needs node coordinates"};
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = coords[d];
    for (int32_t i = 0; i < nb; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], coords[3 * (size_t)i + d]);
            hi[d] = std::max(hi[d], coords[3 * (size_t)i + d]);
        }
    const double tau = 1e-8 * std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
    phi.assign((size_t)nb * 90, 0.0f);
    Lchol.assign((size_t)nb * 6, 0.0);
    parallel_for(nb, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            const double *D = nullptr;
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                if (A.col[k] == i) D = &A.val[9 * k];
            if (!D) throw AmgError{AMG_ERR_ARG, "missing diagonal block"};
            double dn = 0.0;
            for (int q = 0; q < 9; ++q) dn += D[q] * D[q];
            dn = std::sqrt(dn);
            float *f = &phi[90 * (size_t)i];
            for (int q = 0; q < 9; ++q) f[q] = (float)(D[q] / dn);
            std::array<bool, 27> used{};
            const double *xi = coords + 3 * i;
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                const double *xj = coords + 3 * (size_t)A.col[k];
                int slot = 0;
                for (int d = 0; d < 3; ++d) {
                    const double diff = xj[d] - xi[d];
                    const int sg = diff > tau ? 1 : (diff < -tau ? -1 : 0);
                    slot = 3 * slot + (sg + 1);
                }
                if (used[slot])
                    throw AmgError{AMG_ERR_UNSUPPORTED, "two neighbours of one node fall into the same slot"};
                used[slot] = true;
                const double *a = &A.val[9 * k];
                for (int c = 0; c < 3; ++c) f[9 + 3 * slot + c] = (float)(a[4 * c] / dn);
            }
            // Cholesky of the symmetric block M_i (lower triangle)
            const double *m = &Minv[9 * i];
            double *L = &Lchol[6 * i];
            const double d0 = m[0];
            if (!(d0 > 0.0)) throw AmgError{AMG_ERR_NOT_SPD, "smoother block not positive definite"};
            L[0] = std::sqrt(d0);
            L[1] = m[3] / L[0];
            const double d1 = m[4] - L[1] * L[1];
            if (!(d1 > 0.0)) throw AmgError{AMG_ERR_NOT_SPD, "smoother block not positive definite"};
            L[2] = std::sqrt(d1);
            L[3] = m[6] / L[0];
            L[4] = (m[7] - L[3] * L[1]) / L[2];
            const double d2 = m[8] - L[3] * L[3] - L[4] * L[4];
            if (!(d2 > 0.0)) throw AmgError{AMG_ERR_NOT_SPD, "smoother block not positive definite"};
            L[5] = std::sqrt(d2);
        }
    });
}

}  // namespace saamg
