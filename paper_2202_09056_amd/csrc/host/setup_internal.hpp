// Internal host-side data structures of the SA-AMG setup (FP64).
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "../../../include/saamg.h"

namespace saamg {

// Allocator whose resize() leaves new elements uninitialised (explicit
// values, as in assign(n, v) or push_back, are still constructed): the block
// values of the large setup matrices are written in parallel right after
// they are sized, and a serial zero fill of hundreds of MB would cost more
// than the parallel fill itself.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <typename U>
    NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
    template <typename U>
    void construct(U *p) noexcept {
        ::new (static_cast<void *>(p)) U;
    }
    template <typename U, typename... Args>
    void construct(U *p, Args &&...args) {
        ::new (static_cast<void *>(p)) U(std::forward<Args>(args)...);
    }
};
using ValVec = std::vector<double, NoInitAlloc<double>>;

// 3x3 block CSR with 64-bit row offsets (host).  Every writer of val that
// sizes it with resize() writes all of its entries.
struct Bsr3 {
    int32_t rows = 0;               // block rows
    int32_t cols = 0;               // block columns
    std::vector<int64_t> ptr;       // rows + 1
    std::vector<int32_t> col;       // nnzb
    ValVec val;                     // 9 * nnzb, row-major blocks
    int64_t nnzb() const { return (int64_t)col.size(); }
};

// Scalar CSR with 64-bit row offsets (host; the hybrid setup path).
struct Csr {
    int32_t rows = 0;
    int32_t cols = 0;
    std::vector<int64_t> ptr;       // rows + 1
    std::vector<int32_t> col;       // sorted within each row
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)col.size(); }
};

struct HostLevel {
    Bsr3 A;                         // level operator
    Bsr3 P, R;                      // transfer operators (empty on the coarsest level)
    std::vector<double> Minv;       // 9 * rows: pre-sweep smoother blocks M_I (row-major 3x3)
    std::vector<double> Mpost;      // post-sweep blocks M_I^T when they differ (SPAI-0), else empty
    // Fused sweeps (one pre- and one post-sweep; empty otherwise):
    // G = (I - Mt A) P with Mt the post-sweep blocks, the post-smoothed
    // iterate being z = G e + M f + Mt t for the residual t of the
    // pre-smoothed iterate and the coarse correction e (every level but the
    // coarsest); AM = A M (block A_IJ M_J), t = f - AM f (levels below the
    // first).  GP, GAP: P and A P on G's pattern (level 1 of the learned
    // smoother, whose blocks S change after setup: G = GP - S GAP).
    Bsr3 AM, G, GP, GAP;
    // Block ILU(0) in a greedy multicolour order (smoother = AMG_SMOOTHER_ILU0
    // on this level; empty otherwise): colour of each block row, the strictly
    // lower factor L (blocks L_IJ with colour(J) < colour(I), unit diagonal
    // implied), the strictly upper part of U (colour(J) > colour(I)) and the
    // inverted diagonal blocks of U, all in the level's own row numbering.
    std::vector<int32_t> ilu_colour;
    int32_t ilu_ncolours = 0;
    Bsr3 ilu_L, ilu_U;
    std::vector<double> ilu_Dinv;   // 9 * rows
    std::vector<double> ilu_D;      // 9 * rows: diagonal blocks of U (export)
    double omega_j = 0.0;
    double eps = 0.0;
    int node_size = 3;              // 3 on level 1, m (6 or 3) above
    int32_t n_agg = 0;
    std::vector<int32_t> agg;       // aggregate per node, -1 isolated
};

struct Hierarchy {
    std::vector<HostLevel> levels;
    int32_t n_coarse = 0;           // unknowns of the coarsest level
    std::vector<double> coarse_inv; // n_coarse^2, row-major symmetric inverse
    amg_params prm{};
    double setup_ms = 0.0;
    // wall time of each setup phase summed over the levels (ms), indexed by SetupPhase
    double phase_ms[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    // inputs of the learned level-1 smoother (smoother = AMG_SMOOTHER_LEARNED)
    std::vector<float> learn_phi;   // nb * 90 per-node features
    std::vector<double> learn_L;    // nb * 6 Cholesky factors of M_i (L00 L10 L11 L20 L21 L22)
};

// Phases of the setup timed separately (Hierarchy::phase_ms).
enum SetupPhase {
    PH_STRENGTH_AGGREGATE = 0,  // strength graph and aggregation
    PH_TENTATIVE = 1,           // per-aggregate QR of the near-nullspace (scalar space)
    PH_SMOOTH_P = 2,            // filtered matrix and P = (I - omega D^-1 A_F) P^
    PH_TRANSPOSE = 3,           // R = P^T
    PH_GALERKIN = 4,            // A P and R (A P)
    PH_SMOOTHER = 5,            // smoother blocks and the power estimate of the damping
    PH_FUSED = 6,               // AM = A M and G = (I - M A) P
    PH_ILU = 7,                 // colouring and ILU(0) factors
    PH_COARSEST = 8,            // dense inverse of the coarsest matrix
    PH_OTHER = 9,               // input checks, near-nullspace, learned-smoother inputs
    PH_CONVERT = 10,            // scalar <-> 3x3 block conversions (hybrid setup only)
};

// thread-local error message
void set_error(const std::string &msg);

// status-carrying exception used inside the setup
struct AmgError {
    amg_status status;
    std::string msg;
};

// Run fn(begin, end) over [0, n) split into contiguous chunks (at most
// nthreads, at least ~1024 items each) on a persistent thread pool.
void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t, int64_t)> &fn);
// Run fn(t) for t in [0, ntasks) on the pool, one task per worker.
void parallel_tasks(int ntasks, const std::function<void(int)> &fn);
int resolve_threads(int requested);

// The Galerkin products of one level, AP = A P and Ac = R (A P), formed
// elsewhere (the device numeric phase); the default is the host product.
using GalerkinFn = std::function<void(const Bsr3 &A, const Bsr3 &P, const Bsr3 &R, Bsr3 &AP, Bsr3 &Ac)>;

// Steps of Algorithm 1 (hierarchy.cpp).  With invert = false the coarsest
// matrix is left assembled in coarse_inv for a later invert_coarsest (a batch
// builds its problems one per thread, then inverts each coarsest matrix with
// every thread).
void build_hierarchy(const amg_bsr3 &A, const double *coords, const amg_params &prm,
                     Hierarchy &H, const GalerkinFn *galerkin = nullptr, bool invert = true);
void invert_coarsest(Hierarchy &H, int nthreads);

// Per-node features and Cholesky factors of the level-1 smoother blocks for
// the learned smoother (learned_host.cpp).
void learned_inputs(const Bsr3 &A, const double *coords, const std::vector<double> &Minv,
                    std::vector<float> &phi, std::vector<double> &Lchol, int nthreads);

// Dense FP64 Cholesky and inverse (dense.cpp). Throws AmgError(AMG_ERR_NOT_SPD).
void dense_spd_inverse(std::vector<double> &a, int n, int nthreads);

// Householder thin QR of an m x k column-major matrix (m >= k): Q (m x k,
// column-major) and R (k x k, row-major) with R_jj >= 0.
void householder_qr(const double *a, int m, int k, double *Q, double *R);

// Scalar CSR kernels of the hybrid setup path (scalar.cpp): unblock drops
// exact zeros; reblock forms a 3x3 block wherever one of its entries is stored.
Csr unblock(const Bsr3 &A, int nthreads);
Bsr3 reblock(const Csr &S, int nthreads);
Csr csr_multiply(const Csr &A, const Csr &B, int nthreads);
Csr csr_transpose(const Csr &A);

// Sparse products in block arithmetic (sparse.cpp).
Bsr3 bsr_multiply(const Bsr3 &A, const Bsr3 &B, int nthreads);
Bsr3 bsr_symbolic(const Bsr3 &A, const Bsr3 &B, int nthreads);  // pattern of A B, val empty
Bsr3 bsr_transpose(const Bsr3 &A, int nthreads = 1);
void bsr_spmv(const Bsr3 &A, const double *x, double *y, int nthreads);

}  // namespace saamg

// Opaque handle of the C ABI: a host hierarchy.
struct amg_hierarchy {
    saamg::Hierarchy H;
};
