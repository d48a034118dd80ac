// Device context: upload of the host hierarchy into the device layouts (with
// the autotuner), the V-cycle launch sequence (Algorithm 2, evaluated with the
// fused sweeps where a level has them), the CG driver (Section 4) and the
// device entry points of the C ABI.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <type_traits>
#include <vector>

#include "../host/setup_internal.hpp"
#include "launch.hpp"
#include "learned.hpp"
#include "multirhs.hpp"

namespace saamg {

#define HIP_CHECK(call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw AmgError{e_ == hipErrorOutOfMemory ? AMG_ERR_OOM : AMG_ERR_HIP,          \
                           std::string(#call) + ": " + hipGetErrorString(e_)};             \
    } while (0)

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

struct DevAlloc {
    std::vector<void *> ptrs;
    size_t bytes = 0;
    template <typename T>
    T *get(size_t count) {
        if (count == 0) count = 1;
        void *p = nullptr;
        HIP_CHECK(hipMalloc(&p, count * sizeof(T)));
        ptrs.push_back(p);
        bytes += count * sizeof(T);
        return static_cast<T *>(p);
    }
    ~DevAlloc() {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

template <typename V>
V to_storage(double v);
template <>
double to_storage<double>(double v) { return v; }
template <>
float to_storage<float>(double v) { return (float)v; }
template <>
bf16_t to_storage<bf16_t>(double v) {
    // round to nearest even from the FP32 value
    float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return bf16_t{(uint16_t)(u >> 16)};
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return bf16_t{(uint16_t)(u >> 16)};
}

template <typename V>
struct DevSell {
    SellView<V> v{};
    int C = 64;
    bool sorted = false;
    int32_t cols = 0;
    int64_t nnzb = 0;
    int64_t slots = 0;
};

// Host copies of what a setup uploads, kept until the stream has consumed
// them; a buffer sized without contents is left uninitialised for its writer.
using Staging = std::vector<std::vector<char, NoInitAlloc<char>>>;

// Host threads the upload running on this thread may use: amg_params.nthreads
// of the setup call in progress (set for its duration), else all of them.
static thread_local int t_setup_threads = 0;
struct SetupThreads {
    int prev;
    explicit SetupThreads(int requested) : prev(t_setup_threads) { t_setup_threads = resolve_threads(requested); }
    ~SetupThreads() { t_setup_threads = prev; }
};
static int setup_threads() { return t_setup_threads > 0 ? t_setup_threads : resolve_threads(0); }

// Sliced-ELL copy of a host BSR3 matrix (C rows per slice; layout codes 1 and
// 2, row waves and row groups, keep one row per slice with each block's 9
// values contiguous).  With `sorted`, rows are ordered by
// decreasing length inside windows of 256 slices (SELL-C-sigma) so that the
// rows sharing a slice have similar lengths and little padding; the kernel
// then reads the row index of each slice position from `perm`.
// Slices per window of the SELL-C-sigma sort (rows are ordered by length
// within windows of this many slices): 256, or SAAMG_SORT_WINDOW (1 to 4096).
// On the 64^3 cube windows of 256 slices (4096 rows of SELL-16) ran the
// level-1 fused post-sweep in 111.5 us against 114 us with 64 and 112 us
// with 512: wider windows pad less, narrower ones keep the epilogue's
// permuted reads of f, t and z closer together.
static int sort_window_slices() {
    static const int w = [] {
        const char *e = std::getenv("SAAMG_SORT_WINDOW");
        const int v = e ? std::atoi(e) : 256;
        return (v >= 1 && v <= 4096) ? v : 256;
    }();
    return w;
}

// With `row_ids` (sliced ELL only, C > 2) the matrix holds a subset of the
// rows of a larger operator: local row i writes row (*row_ids)[i] of the
// output, and `perm` carries those ids.
template <typename V>
DevSell<V> upload_sell(const Bsr3 &A, int C, DevAlloc &al, hipStream_t s,
                       Staging &staging, bool sorted = false,
                       const std::vector<int32_t> *row_ids = nullptr) {
    DevSell<V> d;
    d.C = C;
    d.cols = A.cols;
    d.nnzb = A.nnzb();
    d.sorted = sorted && C > 2;
    if (row_ids && (C <= 2 || (int64_t)row_ids->size() != A.rows))
        throw AmgError{AMG_ERR_ARG, "row subset needs a sliced-ELL layout and one id per row"};
    const bool contiguous = C <= 2;  // row waves / row groups: 9 contiguous values per block
    if (contiguous) C = 1;           // one row per slice
    const int32_t rows = A.rows;
    const int32_t nsl = (rows + C - 1) / C;
    std::vector<int32_t> perm(rows);
    for (int32_t i = 0; i < rows; ++i) perm[i] = i;
    auto rlen = [&](int32_t i) { return (int32_t)(A.ptr[i + 1] - A.ptr[i]); };
    if (d.sorted) {
        const int32_t win = sort_window_slices() * C;
        for (int32_t w0 = 0; w0 < rows; w0 += win) {
            const int32_t w1 = std::min(rows, w0 + win);
            std::stable_sort(perm.begin() + w0, perm.begin() + w1,
                             [&](int32_t a, int32_t b) { return rlen(a) > rlen(b); });
        }
    }
    std::vector<int32_t> sp(nsl + 1, 0), len(rows);
    for (int32_t q = 0; q < rows; ++q) len[q] = rlen(perm[q]);
    int64_t slots = 0;
    for (int32_t sl = 0; sl < nsl; ++sl) {
        int32_t w = 0;
        for (int32_t q = sl * C; q < std::min(rows, (sl + 1) * C); ++q) w = std::max(w, len[q]);
        sp[sl] = (int32_t)slots;
        slots += w;
        if (slots > INT32_MAX) throw AmgError{AMG_ERR_ARG, "matrix too large for 32-bit slot offsets"};
    }
    sp[nsl] = (int32_t)slots;
    d.slots = slots;
    constexpr int W = group_width<V>();
    const int64_t nrec = slots * C;
    const int64_t gstride = contiguous ? 0 : nrec * W;
    // the layout arrays are built in place in their staging buffers, the
    // slices spread over the host threads; every record of a slice is
    // written, the ones past a row's length (and past the last row) as zero
    auto buffer = [&](size_t bytes) -> char * {
        staging.emplace_back(bytes);
        return staging.back().data();
    };
    const size_t nval = (size_t)nrec * (contiguous ? 9 : 8);
    int32_t *col = (int32_t *)buffer((size_t)nrec * 4);
    V *val = (V *)buffer(nval * sizeof(V));
    V *val8 = contiguous ? nullptr : (V *)buffer((size_t)nrec * sizeof(V));
    const V zero = to_storage<V>(0.0);
    parallel_for(nsl, setup_threads(), [&](int64_t s0, int64_t s1) {
        for (int64_t sl = s0; sl < s1; ++sl) {
            const int32_t width = sp[sl + 1] - sp[sl];
            for (int rl = 0; rl < C; ++rl) {
                const int32_t q = (int32_t)sl * C + rl;
                const int32_t n_here = q < rows ? len[q] : 0;
                const int64_t first = q < rows ? A.ptr[perm[q]] : 0;
                for (int32_t k = 0; k < width; ++k) {
                    const int64_t rec = ((int64_t)sp[sl] + k) * C + rl;
                    const bool has = k < n_here;
                    const int64_t src = first + k;
                    col[rec] = has ? A.col[src] : 0;
                    if (contiguous) {
                        for (int e = 0; e < 9; ++e) val[rec * 9 + e] = has ? to_storage<V>(A.val[9 * src + e]) : zero;
                    } else {
                        for (int e = 0; e < 8; ++e)
                            val[(e / W) * gstride + rec * W + e % W] = has ? to_storage<V>(A.val[9 * src + e]) : zero;
                        val8[rec] = has ? to_storage<V>(A.val[9 * src + 8]) : zero;
                    }
                }
            }
        }
    });
    int32_t *dsp = al.get<int32_t>(sp.size());
    int32_t *dlen = al.get<int32_t>(len.size());
    int32_t *dcol = al.get<int32_t>((size_t)nrec);
    V *dval = al.get<V>(nval);
    V *dval8 = contiguous ? nullptr : al.get<V>((size_t)nrec);
    if (row_ids)
        for (auto &q : perm) q = (*row_ids)[q];
    int32_t *dperm = (d.sorted || row_ids) ? al.get<int32_t>(perm.size()) : nullptr;
    auto stage = [&](const void *p, size_t bytes) {
        staging.emplace_back((const char *)p, (const char *)p + bytes);
        return (const void *)staging.back().data();
    };
    HIP_CHECK(hipMemcpyAsync(dsp, stage(sp.data(), sp.size() * 4), sp.size() * 4, hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(dlen, stage(len.data(), len.size() * 4), len.size() * 4, hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(dcol, col, (size_t)nrec * 4, hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(dval, val, nval * sizeof(V), hipMemcpyHostToDevice, s));
    if (!contiguous) HIP_CHECK(hipMemcpyAsync(dval8, val8, (size_t)nrec * sizeof(V), hipMemcpyHostToDevice, s));
    if (dperm)
        HIP_CHECK(hipMemcpyAsync(dperm, stage(perm.data(), perm.size() * 4), perm.size() * 4,
                                 hipMemcpyHostToDevice, s));
    int32_t maxlen = 0;
    for (int32_t q = 0; q < rows; ++q) maxlen = std::max(maxlen, len[q]);
    const int32_t meanlen = rows > 0 ? (int32_t)((A.nnzb() + rows - 1) / rows) : 0;
    d.v = SellView<V>{rows, nsl, dsp, dlen, dcol, dval, dval8, dperm, maxlen, gstride, A.cols, meanlen};
    return d;
}

// Smoother blocks in the planar slice layout [row/64][e][row%64].
template <typename T>
T *upload_m(const std::vector<double> &Minv, int32_t rows, DevAlloc &al, hipStream_t s,
            Staging &staging) {
    const int64_t nsl = (rows + kMSlice - 1) / kMSlice;
    std::vector<T> m((size_t)nsl * 9 * kMSlice, T(0));
    for (int32_t r = 0; r < rows; ++r)
        for (int e = 0; e < 9; ++e) m[((r / kMSlice) * 9 + e) * kMSlice + r % kMSlice] = (T)Minv[9 * (size_t)r + e];
    T *d = al.get<T>(m.size());
    staging.emplace_back((const char *)m.data(), (const char *)(m.data() + m.size()));
    HIP_CHECK(hipMemcpyAsync(d, staging.back().data(), m.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

// Pre- and post-sweep blocks of one level in one planar array
// [row/64][e][row%64] with e = 0..8 the pre-sweep and 9..17 the post-sweep
// block (the two-block fused post-sweep of block SPAI-0).
template <typename T>
T *upload_mm(const std::vector<double> &Mpre, const std::vector<double> &Mpost, int32_t rows, DevAlloc &al,
             hipStream_t s, Staging &staging) {
    const int64_t nsl = (rows + kMSlice - 1) / kMSlice;
    std::vector<T> m((size_t)nsl * 18 * kMSlice, T(0));
    for (int32_t r = 0; r < rows; ++r)
        for (int e = 0; e < 18; ++e)
            m[((r / kMSlice) * 18 + e) * kMSlice + r % kMSlice] =
                (T)(e < 9 ? Mpre[9 * (size_t)r + e] : Mpost[9 * (size_t)r + e - 9]);
    T *d = al.get<T>(m.size());
    staging.emplace_back((const char *)m.data(), (const char *)(m.data() + m.size()));
    HIP_CHECK(hipMemcpyAsync(d, staging.back().data(), m.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

// ---------------------------------------------------------------------------
// V-cycle over one precision
// ---------------------------------------------------------------------------

template <typename V, typename T>
struct Level {
    int32_t rows = 0;
    DevSell<V> A, P, R;
    T *M = nullptr;   // pre-sweep smoother blocks (planar)
    T *Mt = nullptr;  // post-sweep blocks: M itself, or M^T for block SPAI-0
    // fused sweeps (see HostLevel): t = f - AM f on the way down (has_am),
    // z = G e + M f + Mt t in place of t on the way up (has_g)
    DevSell<V> AM, G;
    DevSell<V> GP, GAP;  // P and A P on G's pattern and layout (level 1 of the learned smoother)
    bool has_am = false, has_g = false;
    T *MM = nullptr;  // [M | Mt] (18-entry planar) when the post-sweep blocks differ
    T *Mg = nullptr;  // M in G's slice-position order (G sorted, fixed symmetric blocks)
    // block ILU(0) smoother in colour order: per colour, the rows of that
    // colour with their blocks of L (lower colours) and of U (higher
    // colours), and the inverted diagonal blocks of U (planar)
    bool ilu = false;
    std::vector<DevSell<V>> iluL, iluU;
    T *Dinv = nullptr;
    T *f = nullptr, *x = nullptr, *t = nullptr, *y = nullptr;
    T *out = nullptr;  // where V_l leaves its result
    // out = (L U)^{-1} rhs: a forward pass per colour (w_I = rhs_I - sum L_IJ
    // w_J over lower colours) into w, then a backward pass per colour from the
    // highest (out_I = U_II^{-1} (w_I - sum U_IJ out_J) over higher colours).
    // Rows of one colour are not coupled, so each pass reads only rows
    // written by earlier passes.  w differs from rhs and out; out may be rhs
    // (the forward passes have consumed rhs before the first backward pass).
    void ilu_solve(const T *rhs, T *w, T *o, double *partials, DevState *st, int gated, hipStream_t s) const {
        for (size_t c = 0; c < iluL.size(); ++c)
            launch_sell<V, T>(iluL[c].v, iluL[c].C, MODE_RESID, w, rhs, w, nullptr, partials, st, gated, SITE_NONE, s);
        for (size_t c = iluU.size(); c-- > 0;)
            launch_sell<V, T>(iluU[c].v, iluU[c].C, MODE_MSOLVE, o, w, o, Dinv, partials, st, gated, SITE_NONE, s);
    }
    // mode and block array of the fused post-sweep (single-vector kernels)
    int post_mode(bool dot) const {
        if (Mg) return dot ? MODE_POSTP_DOT : MODE_POSTP;
        return post_mode_rows(dot);
    }
    const T *post_m() const { return Mg ? Mg : post_m_rows(); }
    // the same with the blocks indexed by row (the multi-column kernels)
    int post_mode_rows(bool dot) const {
        return MM ? (dot ? MODE_POST2_DOT : MODE_POST2) : (dot ? MODE_POST_DOT : MODE_POST);
    }
    const T *post_m_rows() const { return MM ? MM : M; }
};

template <typename V, typename T>
struct Vcycle {
    std::vector<Level<V, T>> lv;
    int n_coarse = 0;
    const double *Ainv = nullptr;
    int npre = 1, npost = 1;
    // The last restriction folded into the coarsest solve: W = A_L^{-1} R_{L-1}
    // (dense FP64, n_coarse x unknowns of level w_level = L-2), applied to
    // that level's residual t in one launch instead of the restriction and
    // the coarsest product (levels with fused sweeps only; -1: not folded).
    const double *W = nullptr;
    int w_level = -1;
    bool folded(int first) const { return W && w_level > first; }

    // z = V(f1) from level `first` down (first = 0: the whole cycle).  If
    // pre_done, x of level `first` already holds M f1.
    void run(const T *f1, T *z, bool pre_done, int gated, int final_site, double *partials,
             DevState *st, hipStream_t s, int first = 0) {
        const int L = (int)lv.size();
        std::vector<T *> cur(L);
        for (int l = first; l + 1 < L; ++l) {
            auto &v = lv[l];
            const T *f = l == first ? f1 : v.f;
            if (l > first && v.has_am && v.has_g) {
                launch_sell<V, T>(v.AM.v, v.AM.C, MODE_RESID, f, f, v.t, nullptr, partials, st, gated, SITE_NONE, s);
                if (!(folded(first) && l == w_level))
                    launch_sell<V, T>(v.R.v, v.R.C, MODE_SPMV, v.t, nullptr, lv[l + 1].f, nullptr, partials, st,
                                      gated, SITE_NONE, s);
                continue;
            }
            if (v.ilu) {
                // x = (L U)^{-1} f (w in y), t = f - A x, restriction
                v.ilu_solve(f, v.y, v.x, partials, st, gated, s);
                cur[l] = v.x;
                launch_sell<V, T>(v.A.v, v.A.C, MODE_RESID, v.x, f, v.t, nullptr, partials, st, gated, SITE_NONE, s);
                launch_sell<V, T>(v.R.v, v.R.C, MODE_SPMV, v.t, nullptr, lv[l + 1].f, nullptr, partials, st, gated,
                                  SITE_NONE, s);
                continue;
            }
            if (!(l == first && pre_done)) launch_jacobi0<T>(v.rows, v.M, f, v.x, st, gated, s);
            T *c = v.x;
            for (int k = 1; k < npre; ++k) {
                T *o = (c == v.x) ? v.y : v.x;
                launch_sell<V, T>(v.A.v, v.A.C, MODE_SMOOTH, c, f, o, v.M, partials, st, gated, SITE_NONE, s);
                c = o;
            }
            cur[l] = c;
            // with G the top level's residual is kept in z, which the fused
            // post-sweep then overwrites in place
            T *t = (l == first && v.has_g && npost == 1) ? z : v.t;
            launch_sell<V, T>(v.A.v, v.A.C, MODE_RESID, c, f, t, nullptr, partials, st, gated, SITE_NONE, s);
            launch_sell<V, T>(v.R.v, v.R.C, MODE_SPMV, t, nullptr, lv[l + 1].f, nullptr, partials, st, gated,
                              SITE_NONE, s);
        }
        auto &cl = lv[L - 1];
        const bool direct = L - 1 == first;
        if (folded(first))
            launch_dense_rect<T>(n_coarse, 3 * lv[w_level].rows, W, lv[w_level].t, cl.y, st, gated, s);
        else
            launch_dense_gemv<T>(n_coarse, Ainv, direct ? f1 : cl.f, direct ? z : cl.y, st, gated, s);
        cl.out = direct ? z : cl.y;
        for (int l = L - 2; l >= first; --l) {
            auto &v = lv[l];
            const T *f = l == first ? f1 : v.f;
            if (l > first && v.has_am && v.has_g) {
                launch_sell<V, T>(v.G.v, v.G.C, v.post_mode(false), lv[l + 1].out, f, v.t, v.post_m(), partials, st,
                                  gated, SITE_NONE, s);
                v.out = v.t;
                continue;
            }
            if (l == first && v.has_g && npost == 1) {
                const bool dot = final_site != SITE_NONE;
                launch_sell<V, T>(v.G.v, v.G.C, v.post_mode(dot), lv[l + 1].out, f, z, v.post_m(), partials, st,
                                  gated, dot ? final_site : SITE_NONE, s);
                v.out = z;
                continue;
            }
            T *c = cur[l];
            launch_sell<V, T>(v.P.v, v.P.C, MODE_ADD, lv[l + 1].out, nullptr, c, nullptr, partials, st, gated,
                              SITE_NONE, s);
            if (v.ilu) {
                // t = f - A x, d = (L U)^{-1} t (w in y, d over t), out = x + d
                launch_sell<V, T>(v.A.v, v.A.C, MODE_RESID, c, f, v.t, nullptr, partials, st, gated, SITE_NONE, s);
                v.ilu_solve(v.t, v.y, v.t, partials, st, gated, s);
                const bool dot = (l == first && final_site != SITE_NONE);
                T *dest = l == first ? z : v.y;
                launch_add2<T>(3 * (int64_t)v.rows, c, v.t, dest, f, partials, st, gated,
                               dot ? final_site : SITE_NONE, s);
                v.out = dest;
                continue;
            }
            T *spare = (c == v.x) ? v.y : v.x;
            T *dest = l == first ? z : spare;
            T *src = c;
            for (int k = 0; k + 1 < npost; ++k) {
                T *o = (src == c) ? v.t : c;
                launch_sell<V, T>(v.A.v, v.A.C, MODE_SMOOTH, src, f, o, v.Mt, partials, st, gated, SITE_NONE, s);
                src = o;
            }
            const bool dot = (l == first && final_site != SITE_NONE);
            launch_sell<V, T>(v.A.v, v.A.C, dot ? MODE_SMOOTH_DOT : MODE_SMOOTH, src, f, dest, v.Mt, partials, st,
                              gated, dot ? final_site : SITE_NONE, s);
            v.out = dest;
        }
    }
};

// Layout per matrix: short rows (the fine operator, P) take one lane per row
// over 64-row slices; long rows (R, coarse operators) take one wavefront per
// row over contiguous block rows.
int choose_c(const Bsr3 &A) {
    const double avg = A.rows ? (double)A.nnzb() / A.rows : 0.0;
    return avg > 40.0 ? 1 : 64;
}

// Autotuner: upload each candidate layout, time it with HIP events
// (residuals t = f - A x for square operators, y = A x otherwise), keep the
// fastest (with a 5 % margin in favour of the fixed rule).  Small operators keep the fixed rule (their
// products are latency bound and the differences are noise).
// Optional persistent record of the autotuner's choices: the file named by
// the environment variable SAAMG_TUNE_CACHE holds one line per operator,
// "rows cols nnzb value_bytes C sorted"; a hit skips the timing.  The file
// named by SAAMG_TUNE_LOG, if set, receives every candidate's time:
// "rows cols nnzb value_bytes mode C sorted ms_per_10_launches".
struct TuneCache {
    std::mutex mu;
    std::string loaded;  // file the entries were read from (reread when the variable changes)
    std::map<std::string, std::pair<int, int>> entries;
    static std::string key(const Bsr3 &A, size_t vbytes) {
        return std::to_string(A.rows) + " " + std::to_string(A.cols) + " " + std::to_string(A.nnzb()) + " " +
               std::to_string(vbytes);
    }
    const char *path() { return std::getenv("SAAMG_TUNE_CACHE"); }
    bool lookup(const std::string &k, int &C, bool &sorted) {
        std::lock_guard<std::mutex> lk(mu);
        const char *p = path();
        if (!p) return false;
        if (loaded != p) {
            loaded = p;
            entries.clear();
            std::ifstream in(p);
            int64_t r, c, n, vb;
            int cc, so;
            while (in >> r >> c >> n >> vb >> cc >> so)
                entries[std::to_string(r) + " " + std::to_string(c) + " " + std::to_string(n) + " " +
                        std::to_string(vb)] = {cc, so};
        }
        auto it = entries.find(k);
        if (it == entries.end()) return false;
        C = it->second.first;
        sorted = it->second.second != 0;
        return C == 1 || C == 2 || C == 4 || C == 8 || C == 16 || C == 32 || C == 64;
    }
    void store(const std::string &k, int C, bool sorted) {
        std::lock_guard<std::mutex> lk(mu);
        const char *p = path();
        if (!p) return;
        entries[k] = {C, sorted ? 1 : 0};
        std::ofstream out(p, std::ios::app);
        out << k << " " << C << " " << (sorted ? 1 : 0) << "\n";
    }
};
static TuneCache g_tune_cache;

template <typename V>
// post_m: the level's smoother blocks when A is a fused post-sweep operator G
// (timed in that mode, whose epilogue reads 15 operands per row).
DevSell<V> tuned_sell(const Bsr3 &A, bool tune, DevAlloc &al, hipStream_t s,
                      Staging &staging, double *partials, DevState *st,
                      const void *post_m = nullptr, int post_mode = MODE_POST) {
    if (!tune || A.nnzb() < 4000) return upload_sell<V>(A, choose_c(A), al, s, staging);
    const std::string ckey = TuneCache::key(A, sizeof(V));
    {
        int cc = 0;
        bool so = false;
        if (g_tune_cache.lookup(ckey, cc, so)) return upload_sell<V>(A, cc, al, s, staging, so);
    }
    struct Cand {
        int C;
        bool sorted;
    };
    std::vector<Cand> cands = {{64, false}, {32, false}, {16, false}, {1, false}};
    int64_t mx = 0;
    for (int32_t i = 0; i < A.rows; ++i) mx = std::max<int64_t>(mx, A.ptr[i + 1] - A.ptr[i]);
    const double avg = A.rows ? (double)A.nnzb() / A.rows : 0.0;
    // long rows: narrower slices put 8 or 16 lanes on each row, row groups a
    // whole workgroup
    if (avg > 24.0) cands.insert(cands.end(), {{8, false}, {4, false}, {2, false}});
    // row-length spread: try the sorted slices too
    if (mx > 1.25 * avg) {
        cands.insert(cands.end(), {{64, true}, {32, true}, {16, true}});
        if (avg > 24.0) cands.insert(cands.end(), {{8, true}, {4, true}});
    }
    Cand best{choose_c(A), false};
    float best_ms = 1e30f;
    DevAlloc tmp;
    using T = typename std::conditional<std::is_same<V, double>::value, double, float>::type;
    T *x = tmp.get<T>(3 * (size_t)A.cols);
    T *y = tmp.get<T>(3 * (size_t)A.rows);
    launch_fill<T>(3 * (int64_t)A.cols, T(1), x, s);
    launch_fill<T>(3 * (int64_t)A.rows, T(1), y, s);
    // level operators run as residual / smoothing sweeps in the V-cycle, the
    // transfer operators as plain products, G as the fused post-sweep: time
    // the mode they will run in
    const T *M = (const T *)post_m;
    const int mode = M ? post_mode : A.rows == A.cols ? MODE_RESID : MODE_SPMV;
    T *fp = M ? tmp.get<T>(3 * (size_t)A.rows) : nullptr;  // f of the post-sweep (y holds t)
    if (fp) launch_fill<T>(3 * (int64_t)A.rows, T(1), fp, s);
    const T *f = M ? fp : A.rows == A.cols ? x : nullptr;
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    // the fixed rule is timed first; another layout must beat it by 5 % (the
    // timings of small operators are noisy), or by 2 % once a launch takes
    // more than 50 us; each candidate keeps the best of three batches of 10
    // launches
    std::stable_partition(cands.begin(), cands.end(),
                          [&](const Cand &c) { return c.C == best.C && !c.sorted; });
    for (const Cand &c : cands) {
        DevAlloc cand;
        Staging st_c;
        DevSell<V> d = upload_sell<V>(A, c.C, cand, s, st_c, c.sorted);
        launch_sell<V, T>(d.v, c.C, mode, x, f, y, M, partials, st, 0, SITE_NONE, s);
        float ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HIP_CHECK(hipEventRecord(e0, s));
            for (int i = 0; i < 10; ++i)
                launch_sell<V, T>(d.v, c.C, mode, x, f, y, M, partials, st, 0, SITE_NONE, s);
            HIP_CHECK(hipEventRecord(e1, s));
            HIP_CHECK(hipEventSynchronize(e1));
            float t = 0.f;
            HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t);
        }
        if (const char *log = std::getenv("SAAMG_TUNE_LOG")) {
            std::ofstream out(log, std::ios::app);
            out << ckey << " " << mode << " " << c.C << " " << (c.sorted ? 1 : 0) << " " << ms << "\n";
        }
        const float margin = best_ms > 0.5f ? 0.98f : 0.95f;  // 10 launches
        if (best_ms == 1e30f || ms < margin * best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_CHECK(hipStreamSynchronize(s));
    g_tune_cache.store(ckey, best.C, best.sorted);
    return upload_sell<V>(A, best.C, al, s, staging, best.sorted);
}

// ---------------------------------------------------------------------------
// Krylov vectors and the context
// ---------------------------------------------------------------------------

template <typename T>
struct Krylov {
    T *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;
};

// Buffers of the multi-right-hand-side solve (k <= 32 columns, row-major),
// allocated on the first multi solve and kept by the context.
struct MultiBufs {
    bool ready = false;
    double *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr;  // outer FP64 CG
    void *rv = nullptr, *zv = nullptr;                              // V-cycle precision
    std::vector<void *> f, x, t, y;                                 // per level, V-cycle precision
    double *partials = nullptr;
    double *gemm_part = nullptr;  // split-K partial tiles of the coarsest GEMM
    MState *st = nullptr;
    MState *hst = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_k = 0;
};

// Learned level-1 smoother blocks (smoother = AMG_SMOOTHER_LEARNED).
struct LearnedBufs {
    bool available = false;  // inputs uploaded (hierarchy of at least two levels)
    bool active = false;     // learned blocks installed in the level-1 smoother array
    bool g_stale = false;    // level-1 G not yet formed with the blocks now installed
    int nb = 0;
    size_t mlen = 0;         // elements of the planar level-1 smoother array
    float *phi = nullptr;    // nb x 90 features
    float *theta32 = nullptr;  // FP32 copy of BF16 parameters (AMG_MLP_PARAMS)
    double *L = nullptr;     // nb x 6 Cholesky factors of M_i
    float *g = nullptr;      // nb x 6 network outputs
    void *Mbj = nullptr;     // block-Jacobi blocks in the V-cycle precision (planar)
    int *nbad = nullptr;
    int *hbad = nullptr;     // pinned mirror
    double *x0 = nullptr;    // caller's initial guess, kept for the fallback
    // training buffers, allocated by the first amg_mlp_loss_grad
    bool train_ready = false;
    float *z1 = nullptr, *z2 = nullptr, *t = nullptr, *dg = nullptr, *dz1 = nullptr, *dz2 = nullptr;
    double *U = nullptr, *pgrad = nullptr, *scal = nullptr, *hscal = nullptr;
    double *r = nullptr, *w = nullptr, *y = nullptr, *y2 = nullptr, *q = nullptr, *xc = nullptr;
};

// run_loop's verdict when the learned smoother let the residual grow
constexpr int ST_GROWTH = 100;
// residual norm this many times above the smallest seen at a check
constexpr double kGrowthFactor = 100.0;

}  // namespace saamg

using namespace saamg;

// ---------------------------------------------------------------------------
// static scratch of amg_true_residual_noalloc: the reduction state (first
// 256 bytes) and the per-workgroup partial sums, one copy per device
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[AMG_NOALLOC_SCRATCH_BYTES];

namespace saamg {

static_assert(sizeof(DevState) <= 256, "reduction state must fit the scratch header");
constexpr size_t kScratchHeader = 256;

// Device address of `scratch` on `device` (which must be current), looked up
// once per device; host code uses only this address, never the symbol.
static void *scratch_address(int device) {
    static std::mutex mu;
    static std::map<int, void *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) return it->second;
    void *p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw AmgError{AMG_ERR_HIP, "no device address for the static scratch array"};
    addr[device] = p;
    return p;
}

}  // namespace saamg

struct amg_ctx {
    int device = 0;
    void *scratch = nullptr;  // this device's static scratch array (amg_true_residual_noalloc)
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;  // used when the caller passes the null stream
    amg_params prm{};
    DevAlloc al;
    amg_stats_t stats{};
    int32_t nb = 0;
    int64_t n = 0;
    int precision = AMG_FP64;
    // FP64 finest operator: outer products and true residuals in every form
    DevSell<double> A64;
    // V-cycle in the chosen storage precision
    Vcycle<double, double> v64;
    Vcycle<float, float> v32;
    Vcycle<bf16_t, float> v16;
    // inner Krylov operator of the mixed forms (FP32 values)
    DevSell<float> A32;
    Krylov<double> k64;    // FP64 CG (k64.x is the solution)
    Krylov<float> k32;     // inner FP32 CG of the mixed forms (k32.x is the correction)
    double *R64 = nullptr; // FP64 residual of the outer iteration
    double *Ainv = nullptr;
    double *partials = nullptr;
    int max_grid = 1;
    DevState *st = nullptr;
    DevState *hst = nullptr;  // pinned mirror
    hipEvent_t ev0 = nullptr, ev1 = nullptr, fence_in = nullptr, fence_out = nullptr;
    hipGraphExec_t iter_exec = nullptr;
    hipGraph_t iter_graph = nullptr;
    int iter_graph_k = 0;
    MultiBufs mb;
    LearnedBufs lr;

    ~amg_ctx() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (lr.hbad) (void)hipHostFree(lr.hbad);
        if (lr.hscal) (void)hipHostFree(lr.hscal);
        if (mb.exec) (void)hipGraphExecDestroy(mb.exec);
        if (mb.graph) (void)hipGraphDestroy(mb.graph);
        if (mb.hst) (void)hipHostFree(mb.hst);
        if (iter_exec) (void)hipGraphExecDestroy(iter_exec);
        if (iter_graph) (void)hipGraphDestroy(iter_graph);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (fence_in) (void)hipEventDestroy(fence_in);
        if (fence_out) (void)hipEventDestroy(fence_out);
        if (hst) (void)hipHostFree(hst);
        if (own_stream) (void)hipStreamDestroy(own_stream);
    }
};

namespace saamg {

// ---------------------------------------------------------------------------
// upload
// ---------------------------------------------------------------------------

// Rows of one colour of an ILU(0) factor (in the level's numbering) as a
// sliced-ELL operator that writes those rows of the output.
static Bsr3 colour_rows(const Bsr3 &F, const std::vector<int32_t> &rows) {
    Bsr3 S;
    S.rows = (int32_t)rows.size();
    S.cols = F.cols;
    S.ptr.assign(rows.size() + 1, 0);
    for (size_t q = 0; q < rows.size(); ++q) {
        const int32_t i = rows[q];
        S.col.insert(S.col.end(), F.col.begin() + F.ptr[i], F.col.begin() + F.ptr[i + 1]);
        S.val.insert(S.val.end(), F.val.begin() + 9 * F.ptr[i], F.val.begin() + 9 * F.ptr[i + 1]);
        S.ptr[q + 1] = (int64_t)S.col.size();
    }
    return S;
}

// Rows per slice of a colour pass: narrow slices for long rows; rows sorted
// by length within windows when their lengths vary.
static int ilu_slice_rows(const Bsr3 &S) {
    const double avg = S.rows ? (double)S.nnzb() / S.rows : 0.0;
    return avg > 48.0 ? 4 : avg > 24.0 ? 8 : 16;
}

template <typename V, typename T>
static void upload_ilu(amg_ctx *ctx, const HostLevel &hl, Level<V, T> &dl, Staging &staging) {
    hipStream_t s = ctx->stream;
    const int nc = hl.ilu_ncolours;
    std::vector<std::vector<int32_t>> rows(nc);
    for (int32_t i = 0; i < hl.A.rows; ++i) rows[hl.ilu_colour[i]].push_back(i);
    dl.iluL.clear();
    dl.iluU.clear();
    for (int c = 0; c < nc; ++c) {
        const Bsr3 Lc = colour_rows(hl.ilu_L, rows[c]);
        const Bsr3 Uc = colour_rows(hl.ilu_U, rows[c]);
        dl.iluL.push_back(upload_sell<V>(Lc, ilu_slice_rows(Lc), ctx->al, s, staging, true, &rows[c]));
        dl.iluU.push_back(upload_sell<V>(Uc, ilu_slice_rows(Uc), ctx->al, s, staging, true, &rows[c]));
    }
    dl.Dinv = upload_m<T>(hl.ilu_Dinv, hl.A.rows, ctx->al, s, staging);
    dl.ilu = true;
}

template <typename V, typename T>
static void upload_vcycle(amg_ctx *ctx, const Hierarchy &H, Vcycle<V, T> &vc,
                          Staging &staging, const DevSell<V> *finest_given) {
    hipStream_t s = ctx->stream;
    const bool tune = ctx->prm.autotune != 0;
    const int L = (int)H.levels.size();
    vc.lv.resize(L);
    vc.npre = H.prm.npre;
    vc.npost = H.prm.npost;
    for (int l = 0; l < L; ++l) {
        const auto &hl = H.levels[l];
        auto &dl = vc.lv[l];
        dl.rows = hl.A.rows;
        const size_t vlen = 3 * (size_t)hl.A.rows;
        dl.f = ctx->al.get<T>(vlen);
        dl.x = ctx->al.get<T>(vlen);
        dl.t = ctx->al.get<T>(vlen);
        dl.y = ctx->al.get<T>(vlen);
        if (l + 1 < L) {
            if (l == 0 && finest_given)
                dl.A = *finest_given;
            else
                dl.A = tuned_sell<V>(hl.A, tune, ctx->al, s, staging, ctx->partials, ctx->st);
            dl.P = tuned_sell<V>(hl.P, tune, ctx->al, s, staging, ctx->partials, ctx->st);
            dl.R = tuned_sell<V>(hl.R, tune, ctx->al, s, staging, ctx->partials, ctx->st);
            dl.M = upload_m<T>(hl.Minv, hl.A.rows, ctx->al, s, staging);
            if (!hl.ilu_colour.empty()) {
                if (std::is_same<V, bf16_t>::value)
                    throw AmgError{AMG_ERR_UNSUPPORTED, "the ILU(0) smoother needs an FP64 or FP32 V-cycle"};
                upload_ilu<V, T>(ctx, hl, dl, staging);
            }
            dl.Mt = hl.Mpost.empty() ? dl.M : upload_m<T>(hl.Mpost, hl.A.rows, ctx->al, s, staging);
            // BF16 storage keeps the plain sweeps: G = P - M A P is a
            // difference of like-sized terms, which 8 mantissa bits do not
            // resolve (the V-cycle loses ~40 % in iterations)
            constexpr bool fuse = !std::is_same<V, bf16_t>::value;
            if (fuse && !hl.AM.ptr.empty()) {
                dl.AM = tuned_sell<V>(hl.AM, tune, ctx->al, s, staging, ctx->partials, ctx->st);
                dl.has_am = true;
            }
            if (fuse && !hl.G.ptr.empty()) {
                if (!hl.Mpost.empty()) dl.MM = upload_mm<T>(hl.Minv, hl.Mpost, hl.A.rows, ctx->al, s, staging);
                dl.G = tuned_sell<V>(hl.G, tune, ctx->al, s, staging, ctx->partials, ctx->st, dl.post_m(),
                                     dl.post_mode(false));
                dl.has_g = true;
                // rows sorted within windows: the post-sweep reads a copy of M in
                // G's slice-position order (contiguous per slice); not for the
                // learned level-1 blocks, which change after setup
                const bool learned1 = l == 0 && ctx->prm.smoother == AMG_SMOOTHER_LEARNED;
                if (dl.G.sorted && dl.G.C > 2 && hl.Mpost.empty() && !learned1) {
                    std::vector<int32_t> perm(hl.A.rows);
                    HIP_CHECK(hipMemcpyAsync(perm.data(), dl.G.v.perm, perm.size() * 4, hipMemcpyDeviceToHost, s));
                    HIP_CHECK(hipStreamSynchronize(s));
                    std::vector<double> mp(hl.Minv.size());
                    for (size_t q = 0; q < perm.size(); ++q)
                        std::memcpy(&mp[9 * q], &hl.Minv[9 * (size_t)perm[q]], 9 * sizeof(double));
                    dl.Mg = upload_m<T>(mp, hl.A.rows, ctx->al, s, staging);
                }
                if (!hl.GP.ptr.empty()) {  // same pattern, same layout: records line up
                    dl.GP = upload_sell<V>(hl.GP, dl.G.C, ctx->al, s, staging, dl.G.sorted);
                    dl.GAP = upload_sell<V>(hl.GAP, dl.G.C, ctx->al, s, staging, dl.G.sorted);
                }
            }
        }
    }
    vc.n_coarse = H.n_coarse;
    vc.Ainv = ctx->Ainv;
    // fold the last restriction into the coarsest solve when the level above
    // the coarsest runs the fused sweeps (three or more levels) and the dense
    // W streams at most kFoldSlack bytes more than R and the inverse it
    // replaces (about what the launch it saves costs at the tail of a cycle)
    constexpr double kFoldSlack = 16e6;
    const int wl = L - 2;
    const bool fold_cheap =
        L >= 3 && (double)H.n_coarse * 3.0 * H.levels[wl].A.rows * 8.0 <=
                      (double)H.levels[wl].R.nnzb() * (9.0 * 8 + 4) + 4.0 * H.levels[wl].R.rows +
                          (double)H.n_coarse * H.n_coarse * 8.0 + kFoldSlack;
    if (fold_cheap && vc.lv[wl].has_am && vc.lv[wl].has_g) {
        const Bsr3 &R = H.levels[wl].R;
        const int nc = H.n_coarse, nf = 3 * H.levels[wl].A.rows;
        std::vector<double> W((size_t)nc * nf, 0.0);
        for (int32_t I = 0; I < R.rows; ++I)
            for (int64_t k = R.ptr[I]; k < R.ptr[I + 1]; ++k)
                for (int r = 0; r < 3; ++r)
                    for (int cc = 0; cc < 3; ++cc) {
                        const double v = R.val[9 * k + 3 * r + cc];
                        if (v == 0.0) continue;
                        const int kk = 3 * I + r, j = 3 * R.col[k] + cc;
                        for (int i = 0; i < nc; ++i) W[(size_t)i * nf + j] += H.coarse_inv[(size_t)i * nc + kk] * v;
                    }
        double *dW = ctx->al.get<double>(W.size());
        HIP_CHECK(hipMemcpyAsync(dW, W.data(), W.size() * 8, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));  // W is released on return
        vc.W = dW;
        vc.w_level = wl;
    }
}

template <typename T>
static void alloc_krylov(amg_ctx *ctx, Krylov<T> &k) {
    k.x = ctx->al.get<T>(ctx->n);
    k.r = ctx->al.get<T>(ctx->n);
    k.p = ctx->al.get<T>(ctx->n);
    k.q = ctx->al.get<T>(ctx->n);
    k.z = ctx->al.get<T>(ctx->n);
}

template <typename V>
static double sell_bytes(const DevSell<V> &M, double vec_bytes) {
    return (double)M.nnzb * (9.0 * sizeof(V) + 4) + 4.0 * M.v.rows + vec_bytes;
}

// Algorithmic HBM bytes of one V-cycle with value size sv, smoother size sm
// and vector size s (each stored block, index and vector entry once).
static double vcycle_bytes(const Hierarchy &H, double sv, double sm, double s, bool fused, int w_level = -1) {
    double b = 0.0;
    for (size_t l = 0; l + 1 < H.levels.size(); ++l) {
        const auto &L = H.levels[l];
        const double rows = L.A.rows, crow = L.P.cols;
        const double a = (double)L.A.nnzb() * (9 * sv + 4) + 4 * rows;
        const double p = (double)L.P.nnzb() * (9 * sv + 4);
        const double g = (double)L.G.nnzb() * (9 * sv + 4) + 4 * rows + 3 * s * crow + 9 * s * rows +
                         (L.Mpost.empty() ? 9 : 18) * sm * rows;
        if (!L.ilu_colour.empty()) {
            // ILU(0): (L U)^{-1} f; residual; restriction; prolongation add;
            // residual; (L U)^{-1} t; x + d.  A triangular solve reads L and U
            // once (row lengths and row ids, rhs, w twice, the output and the
            // inverted diagonal blocks)
            const double solve = (double)(L.ilu_L.nnzb() + L.ilu_U.nnzb()) * (9 * sv + 4) + 16 * rows +
                                 9 * sm * rows + 12 * s * rows;
            b += 2 * solve + 2 * (a + 9 * s * rows);
            b += p + 4 * crow + 3 * s * rows + 3 * s * crow;
            b += p + 4 * rows + 3 * s * crow + 6 * s * rows;
            b += 9 * s * rows;
            continue;
        }
        if (fused && l > 0 && !L.AM.ptr.empty() && !L.G.ptr.empty()) {
            // fused sweeps: t = f - AM f; restriction (folded into the
            // coarsest product on level w_level); z = G e + M (f + t)
            b += (double)L.AM.nnzb() * (9 * sv + 4) + 4 * rows + 6 * s * rows;
            if ((int)l != w_level) b += p + 4 * crow + 3 * s * rows + 3 * s * crow;
            b += g;
            continue;
        }
        if (fused && l == 0 && !L.G.ptr.empty()) {
            // first level: residual (pre-sweep fused into the CG update);
            // restriction; z = G e + M (f + t)
            b += a + 9 * s * rows;
            b += p + 4 * crow + 3 * s * rows + 3 * s * crow;
            b += g;
            continue;
        }
        if (l > 0) b += 9 * sm * rows + 6 * s * rows;      // pre-sweep from zero (level 1: fused)
        b += a + 9 * s * rows;                              // residual: A, x, f, t
        b += p + 4 * crow + 3 * s * rows + 3 * s * crow;    // restriction
        b += p + 4 * rows + 3 * s * crow + 6 * s * rows;    // prolongation add
        b += a + 9 * sm * rows + 9 * s * rows;              // post-sweep: A, M, x, f, y
    }
    if (w_level >= 0) {  // W = A_L^{-1} R applied to the level's residual
        const double nf = 3.0 * H.levels[w_level].A.rows;
        return b + (double)H.n_coarse * nf * 8.0 + s * (nf + H.n_coarse);
    }
    return b + (double)H.n_coarse * H.n_coarse * 8.0 + 2 * s * H.n_coarse;
}

static void compute_stats(amg_ctx *ctx, const Hierarchy &H) {
    amg_stats_t &st = ctx->stats;
    std::memset(&st, 0, sizeof(st));
    st.levels = (int32_t)H.levels.size();
    double tot = 0.0;
    for (size_t l = 0; l < H.levels.size(); ++l) {
        const auto &L = H.levels[l];
        st.nb[l] = L.A.rows;
        st.nnzb_A[l] = L.A.nnzb();
        st.nnzb_P[l] = L.P.nnzb();
        st.n_agg[l] = L.n_agg;
        st.omega_j[l] = L.omega_j;
        tot += (double)L.A.nnzb();
    }
    double sv = 8, sm = 8, s = 8, sa = 8;  // values, smoother, vectors, Krylov operator
    if (ctx->precision == AMG_FP32) sv = sm = s = sa = 4;
    if (ctx->precision == AMG_BF16) {
        sv = 2;
        sm = s = sa = 4;
    }
    const double n = 3.0 * H.levels[0].A.rows;
    const double rows = H.levels[0].A.rows;
    const double a1 = (double)H.levels[0].A.nnzb() * (9 * sa + 4) + 4.0 * rows;
    st.n_coarse = H.n_coarse;
    st.operator_complexity = tot / (double)H.levels[0].A.nnzb();
    st.setup_ms = H.setup_ms;
    for (int q = 0; q < 11; ++q) st.setup_phase_ms[q] = H.phase_ms[q];
    const int wl = ctx->precision == AMG_FP64   ? ctx->v64.w_level
                   : ctx->precision == AMG_FP32 ? ctx->v32.w_level
                                                : ctx->v16.w_level;
    st.vcycle_bytes = vcycle_bytes(H, sv, sm, s, ctx->precision != AMG_BF16, wl);
    // the level-1 zero-guess sweep rides on the CG update unless level 1 is ILU(0)
    const double pre1 = H.levels[0].ilu_colour.empty() ? 9 * sm * rows : -3 * s * rows;
    if (ctx->precision == AMG_FP64 || ctx->prm.krylov == AMG_KRYLOV_IR) {
        st.iter_bytes = st.vcycle_bytes + (a1 + 2 * s * n)      // q = A p
                        + 7 * s * n + pre1                      // update + level-1 pre-sweep
                        + 3 * s * n;                            // p = z + beta p
    } else {
        // outer FP64 CG: FP64 product, update writing the FP32 r and pre-sweep,
        // FP32 z into the FP64 direction
        const double a64 = (double)H.levels[0].A.nnzb() * (9 * 8 + 4) + 4.0 * rows;
        st.iter_bytes = st.vcycle_bytes + (a64 + 16 * n) + 6 * 8 * n + 2 * s * n + pre1 +
                        (s * n + 16 * n);
    }
    st.device_bytes = (double)ctx->al.bytes;
    auto code = [](int C, bool sorted) { return sorted ? -C : C; };
    auto fill = [&](const auto &vc) {
        for (size_t l = 0; l + 1 < H.levels.size(); ++l) {
            const auto &v = vc.lv[l];
            st.layout_A[l] = code(v.A.C, v.A.sorted);
            st.layout_P[l] = code(v.P.C, v.P.sorted);
            st.layout_R[l] = code(v.R.C, v.R.sorted);
            st.layout_AM[l] = v.has_am ? code(v.AM.C, v.AM.sorted) : 0;
            st.layout_G[l] = v.has_g ? code(v.G.C, v.G.sorted) : 0;
        }
    };
    if (ctx->precision == AMG_FP64)
        fill(ctx->v64);
    else if (ctx->precision == AMG_FP32)
        fill(ctx->v32);
    else
        fill(ctx->v16);
}

static void upload(amg_ctx *ctx, const Hierarchy &H) {
    hipStream_t s = ctx->stream;
    Staging staging;
    staging.reserve(64);
    ctx->precision = ctx->prm.precision;
    if (ctx->precision < AMG_FP64 || ctx->precision > AMG_BF16) throw AmgError{AMG_ERR_ARG, "unknown precision"};
    int max_grid = 1;
    for (const auto &hl : H.levels) max_grid = std::max(max_grid, hl.A.rows);  // up to a workgroup per row
    ctx->max_grid = max_grid;
    ctx->partials = ctx->al.get<double>(2 * (size_t)max_grid);
    ctx->st = ctx->al.get<DevState>(1);
    ctx->nb = H.levels[0].A.rows;
    ctx->n = 3 * (int64_t)ctx->nb;
    ctx->Ainv = ctx->al.get<double>(H.coarse_inv.size());
    HIP_CHECK(hipMemcpyAsync(ctx->Ainv, H.coarse_inv.data(), H.coarse_inv.size() * 8, hipMemcpyHostToDevice, s));
    const bool tune = ctx->prm.autotune != 0;
    ctx->A64 = tuned_sell<double>(H.levels[0].A, tune, ctx->al, s, staging, ctx->partials, ctx->st);
    alloc_krylov<double>(ctx, ctx->k64);
    ctx->R64 = ctx->al.get<double>(ctx->n);
    if (ctx->precision == AMG_FP64) {
        upload_vcycle<double, double>(ctx, H, ctx->v64, staging, &ctx->A64);
    } else {
        alloc_krylov<float>(ctx, ctx->k32);
        const bool ir = ctx->prm.krylov == AMG_KRYLOV_IR;
        // the inner CG of iterative refinement needs an FP32 finest operator;
        // the FP32 V-cycle shares it
        if (ir || ctx->precision == AMG_FP32)
            ctx->A32 = tuned_sell<float>(H.levels[0].A, tune, ctx->al, s, staging, ctx->partials, ctx->st);
        if (ctx->precision == AMG_FP32)
            upload_vcycle<float, float>(ctx, H, ctx->v32, staging, &ctx->A32);
        else
            upload_vcycle<bf16_t, float>(ctx, H, ctx->v16, staging, nullptr);
    }
    if (!H.learn_phi.empty() && H.levels.size() > 1) {
        auto &lr = ctx->lr;
        lr.nb = ctx->nb;
        lr.mlen = (size_t)((ctx->nb + kMSlice - 1) / kMSlice) * 9 * kMSlice;
        lr.phi = ctx->al.get<float>(H.learn_phi.size());
        HIP_CHECK(hipMemcpyAsync(lr.phi, H.learn_phi.data(), H.learn_phi.size() * 4, hipMemcpyHostToDevice, s));
        lr.L = ctx->al.get<double>(H.learn_L.size());
        HIP_CHECK(hipMemcpyAsync(lr.L, H.learn_L.data(), H.learn_L.size() * 8, hipMemcpyHostToDevice, s));
        lr.g = ctx->al.get<float>((size_t)ctx->nb * kOut);
        lr.theta32 = ctx->al.get<float>(kParams);
        lr.nbad = ctx->al.get<int>(1);
        lr.x0 = ctx->al.get<double>(ctx->n);
        const size_t esz = ctx->precision == AMG_FP64 ? 8 : 4;
        const void *m = ctx->precision == AMG_FP64   ? (const void *)ctx->v64.lv[0].M
                        : ctx->precision == AMG_FP32 ? (const void *)ctx->v32.lv[0].M
                                                     : (const void *)ctx->v16.lv[0].M;
        lr.Mbj = esz == 8 ? (void *)ctx->al.get<double>(lr.mlen) : (void *)ctx->al.get<float>(lr.mlen);
        HIP_CHECK(hipMemcpyAsync(lr.Mbj, m, lr.mlen * esz, hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipHostMalloc((void **)&lr.hbad, sizeof(int), hipHostMallocDefault));
        lr.available = true;
    }
    HIP_CHECK(hipHostMalloc((void **)&ctx->hst, sizeof(DevState), hipHostMallocDefault));
    HIP_CHECK(hipEventCreate(&ctx->ev0));
    HIP_CHECK(hipEventCreate(&ctx->ev1));
    launch_state_init(ctx->st, 0.0, 1, 0, s);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));  // staging buffers may be released now
    compute_stats(ctx, H);
}

static void read_state(amg_ctx *ctx) {
    HIP_CHECK(hipMemcpyAsync(ctx->hst, ctx->st, sizeof(DevState), hipMemcpyDeviceToHost, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
}

// Level-1 smoother array of the V-cycle (planar blocks, V-cycle precision).
static void *level1_m(amg_ctx *ctx) {
    if (ctx->precision == AMG_FP64) return ctx->v64.lv[0].M;
    return ctx->precision == AMG_FP32 ? ctx->v32.lv[0].M : ctx->v16.lv[0].M;
}

// Put the block-Jacobi blocks back (same array, so captured graphs stay valid).
static void restore_jacobi(amg_ctx *ctx) {
    auto &lr = ctx->lr;
    if (!lr.available) return;
    const size_t esz = ctx->precision == AMG_FP64 ? 8 : 4;
    HIP_CHECK(hipMemcpyAsync(level1_m(ctx), lr.Mbj, lr.mlen * esz, hipMemcpyDeviceToDevice, ctx->stream));
    lr.active = false;
    lr.g_stale = true;
}

// Level-1 G = P - S (A P) for the blocks S now in the smoother array, before
// any V-cycle that starts on level 1 (installing or restoring blocks only
// marks it stale: the training steps do not run such V-cycles).
static void ensure_g(amg_ctx *ctx) {
    auto &lr = ctx->lr;
    if (!lr.g_stale) return;
    auto go = [&](auto &vc) {
        auto &v = vc.lv[0];
        if (v.has_g && v.GP.v.rows > 0)
            launch_g_rebuild(v.G.v, v.GP.v, v.GAP.v, v.G.C <= 2 ? 1 : v.G.C, v.M, ctx->stream);
    };
    if (ctx->precision == AMG_FP64)
        go(ctx->v64);
    else if (ctx->precision == AMG_FP32)
        go(ctx->v32);
    HIP_CHECK(hipGetLastError());
    lr.g_stale = false;
}

// S(theta) into the level-1 smoother array; returns the number of nodes that
// kept their block-Jacobi block (check = 1 only).  t: tanh of the outputs
// (training) or null.  z1, z2: pre-activations (training) or null.
static int install_learned(amg_ctx *ctx, const float *theta, int check, float *z1, float *z2, float *t) {
    auto &lr = ctx->lr;
    hipStream_t s = ctx->stream;
    launch_mlp_forward(lr.nb, lr.phi, theta, z1, z2, lr.g, s);
    HIP_CHECK(hipMemsetAsync(lr.nbad, 0, sizeof(int), s));
    if (ctx->precision == AMG_FP64)
        launch_assemble_blocks<double>(lr.nb, lr.g, lr.L, (double *)level1_m(ctx), (const double *)lr.Mbj, t,
                                       check, lr.nbad, s);
    else
        launch_assemble_blocks<float>(lr.nb, lr.g, lr.L, (float *)level1_m(ctx), (const float *)lr.Mbj, t, check,
                                      lr.nbad, s);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(lr.hbad, lr.nbad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    lr.active = true;
    lr.g_stale = true;
    return *lr.hbad;
}

// ---------------------------------------------------------------------------
// CG engine for one vector precision
// ---------------------------------------------------------------------------

// z = V(r) and r . z into `site`; handles the single-level (dense) case
template <typename V, typename T>
static void precondition(amg_ctx *ctx, Vcycle<V, T> &vc, const T *r, T *z, bool pre_done, int gated,
                         int site) {
    hipStream_t s = ctx->stream;
    if (vc.lv.size() > 1) {
        vc.run(r, z, pre_done, gated, site, ctx->partials, ctx->st, s);
    } else {
        launch_dense_gemv<T>(vc.n_coarse, vc.Ainv, r, z, ctx->st, gated, s);
        if (site != SITE_NONE) launch_dot<T>(ctx->n, r, z, ctx->partials, ctx->st, gated, site, ctx->max_grid, s);
    }
}

template <typename VA, typename V, typename T>
static void cg_iteration(amg_ctx *ctx, const DevSell<VA> &A, Vcycle<V, T> &vc, Krylov<T> &k) {
    hipStream_t s = ctx->stream;
    launch_sell<VA, T>(A.v, A.C, MODE_SPMV_DOT, k.p, nullptr, k.q, nullptr, ctx->partials, ctx->st, 1, SITE_PQ,
                       s);
    const bool multi = vc.lv.size() > 1;
    // the level-1 zero-guess sweep x1 = M r rides on the update (block-diagonal smoothers)
    const bool pre = multi && !vc.lv[0].ilu;
    launch_cg_update<T>(ctx->nb, k.x, k.p, k.r, k.q, pre ? vc.lv[0].M : nullptr, pre ? vc.lv[0].x : k.z,
                        ctx->prm.krylov == AMG_KRYLOV_FCG ? k.z : nullptr, ctx->partials, ctx->st, s);
    precondition<V, T>(ctx, vc, k.r, k.z, pre, 1, SITE_RZ);
    launch_cg_dir<T>(ctx->n, k.z, k.p, ctx->st, s);
}

// FP64 CG preconditioned by a V-cycle stored in FP32/BF16: FP64 product q =
// A p with the FP64 operator, FP32 copies of r in, FP32 z out of the V-cycle.
template <typename V>
static void cg_iteration_mixed(amg_ctx *ctx, Vcycle<V, float> &vc) {
    hipStream_t s = ctx->stream;
    auto &k = ctx->k64;
    launch_sell<double, double>(ctx->A64.v, ctx->A64.C, MODE_SPMV_DOT, k.p, nullptr, k.q, nullptr, ctx->partials,
                                ctx->st, 1, SITE_PQ, s);
    const bool multi = vc.lv.size() > 1;
    const bool pre = multi && !vc.lv[0].ilu;
    launch_cg_update_mixed(ctx->nb, k.x, k.p, k.r, k.q, pre ? vc.lv[0].M : nullptr, ctx->k32.r,
                           pre ? vc.lv[0].x : ctx->k32.z,
                           ctx->prm.krylov == AMG_KRYLOV_FCG ? ctx->k32.z : nullptr, ctx->partials, ctx->st, s);
    precondition<V, float>(ctx, vc, ctx->k32.r, ctx->k32.z, pre, 1, SITE_RZ);
    launch_cg_dir_mixed(ctx->n, ctx->k32.z, k.p, ctx->st, s);
}

static bool iterative_refinement(const amg_ctx *ctx) {
    return ctx->precision != AMG_FP64 && ctx->prm.krylov == AMG_KRYLOV_IR;
}

// one iteration of the context's own form
static void form_iteration(amg_ctx *ctx) {
    if (ctx->precision == AMG_FP64) {
        cg_iteration<double, double, double>(ctx, ctx->A64, ctx->v64, ctx->k64);
    } else if (iterative_refinement(ctx)) {  // inner FP32 CG
        if (ctx->precision == AMG_FP32)
            cg_iteration<float, float, float>(ctx, ctx->A32, ctx->v32, ctx->k32);
        else
            cg_iteration<float, bf16_t, float>(ctx, ctx->A32, ctx->v16, ctx->k32);
    } else if (ctx->precision == AMG_FP32) {
        cg_iteration_mixed<float>(ctx, ctx->v32);
    } else {
        cg_iteration_mixed<bf16_t>(ctx, ctx->v16);
    }
}

template <typename V, typename T>
static void start_direction(amg_ctx *ctx, Vcycle<V, T> &vc, Krylov<T> &k) {
    precondition<V, T>(ctx, vc, k.r, k.z, false, 0, SITE_RZ0);
    launch_copy<T, T>(ctx->n, k.z, k.p, ctx->stream);
}

// z = V(r) for the outer FP64 CG of a mixed form: r64 -> FP32, V-cycle, p = z
template <typename V>
static void start_direction_mixed(amg_ctx *ctx, Vcycle<V, float> &vc) {
    launch_copy<double, float>(ctx->n, ctx->k64.r, ctx->k32.r, ctx->stream);
    precondition<V, float>(ctx, vc, ctx->k32.r, ctx->k32.z, false, 0, SITE_RZ0);
    launch_copy<float, double>(ctx->n, ctx->k32.z, ctx->k64.p, ctx->stream);
}

static void form_start(amg_ctx *ctx) {
    if (ctx->precision == AMG_FP64) {
        start_direction<double, double>(ctx, ctx->v64, ctx->k64);
    } else if (iterative_refinement(ctx)) {
        if (ctx->precision == AMG_FP32)
            start_direction<float, float>(ctx, ctx->v32, ctx->k32);
        else
            start_direction<bf16_t, float>(ctx, ctx->v16, ctx->k32);
    } else if (ctx->precision == AMG_FP32) {
        start_direction_mixed<float>(ctx, ctx->v32);
    } else {
        start_direction_mixed<bf16_t>(ctx, ctx->v16);
    }
}

// A caller on the null stream gets the context's own stream (graphs cannot
// capture the null stream); events order it after the caller's prior work and
// the caller's later work after it.
struct StreamFence {
    amg_ctx *ctx;
    explicit StreamFence(amg_ctx *c) : ctx(c) {
        if (ctx->own_stream) {
            HIP_CHECK(hipEventRecord(ctx->fence_in, nullptr));
            HIP_CHECK(hipStreamWaitEvent(ctx->own_stream, ctx->fence_in, 0));
        }
    }
    ~StreamFence() {
        if (ctx->own_stream) {
            (void)hipEventRecord(ctx->fence_out, ctx->own_stream);
            (void)hipStreamWaitEvent(nullptr, ctx->fence_out, 0);
        }
    }
};

template <typename F>
static amg_status guarded(F &&fn) {
    set_error("");
    try {
        return fn();
    } catch (const AmgError &e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return AMG_ERR_OOM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return AMG_ERR_ARG;
    }
}

static void ensure_iter_graph(amg_ctx *ctx) {
    const int k = std::max(1, ctx->prm.check_every);
    if (ctx->iter_exec && ctx->iter_graph_k == k) return;
    if (ctx->iter_exec) {
        HIP_CHECK(hipGraphExecDestroy(ctx->iter_exec));
        ctx->iter_exec = nullptr;
    }
    if (ctx->iter_graph) {
        HIP_CHECK(hipGraphDestroy(ctx->iter_graph));
        ctx->iter_graph = nullptr;
    }
    HIP_CHECK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < k; ++i) form_iteration(ctx);
    hipGraph_t g = nullptr;
    HIP_CHECK(hipStreamEndCapture(ctx->stream, &g));
    ctx->iter_graph = g;
    HIP_CHECK(hipGraphInstantiate(&ctx->iter_exec, g, nullptr, nullptr, 0));
    ctx->iter_graph_k = k;
}

static void run_chunk(amg_ctx *ctx) {
    if (ctx->prm.use_graphs) {
        ensure_iter_graph(ctx);
        HIP_CHECK(hipGraphLaunch(ctx->iter_exec, ctx->stream));
    } else {
        const int k = std::max(1, ctx->prm.check_every);
        for (int i = 0; i < k; ++i) form_iteration(ctx);
    }
    HIP_CHECK(hipGetLastError());
}

// FP64 true residual R64 = b - A x; state (bb, rr) on the host afterwards
static void true_residual(amg_ctx *ctx, const double *b, const double *x, double &bb, double &rr) {
    launch_sell<double, double>(ctx->A64.v, ctx->A64.C, MODE_RESID_NORM, x, b, ctx->R64, nullptr, ctx->partials,
                                ctx->st, 0, SITE_INIT, ctx->stream);
    HIP_CHECK(hipGetLastError());
    read_state(ctx);
    bb = ctx->hst->bb;
    rr = ctx->hst->rr;
}

// Run the armed CG loop until the state says done; returns the device status.
// With learned smoother blocks installed, a non-finite residual norm or one
// kGrowthFactor above the smallest seen at an earlier check ends the loop
// with ST_GROWTH (the caller then falls back to block Jacobi).
static int run_loop(amg_ctx *ctx) {
    double best = std::numeric_limits<double>::infinity();
    for (;;) {
        run_chunk(ctx);
        read_state(ctx);
        if (ctx->hst->done) return ctx->hst->status;
        if (ctx->lr.active) {
            const double rr = ctx->hst->rr;
            if (!std::isfinite(rr) || rr > kGrowthFactor * kGrowthFactor * best) return ST_GROWTH;
            best = std::min(best, rr);
        }
    }
}

// FP64 CG (the FP64 form, and the outer iteration of the mixed forms)
static amg_status solve_fp64(amg_ctx *ctx, const double *b, double *x, double tol, amg_solve_info &inf) {
    hipStream_t s = ctx->stream;
    auto &k = ctx->k64;
    const double tol2 = tol * tol;
    launch_state_init(ctx->st, tol, ctx->prm.maxiter, ctx->prm.krylov == AMG_KRYLOV_FCG, s);
    launch_copy<double, double>(ctx->n, x, k.x, s);
    launch_sell<double, double>(ctx->A64.v, ctx->A64.C, MODE_RESID_NORM, k.x, b, k.r, nullptr, ctx->partials,
                                ctx->st, 0, SITE_INIT, s);
    launch_state_arm(ctx->st, tol, s);
    HIP_CHECK(hipGetLastError());
    read_state(ctx);
    const double bb = ctx->hst->bb, rr0 = ctx->hst->rr;
    if (!std::isfinite(bb)) throw AmgError{AMG_ERR_ARG, "right-hand side has non-finite entries"};
    if (bb == 0.0) {
        launch_fill<double>(ctx->n, 0.0, x, s);
        inf.converged = 1;
        return AMG_OK;
    }
    if (!std::isfinite(rr0)) throw AmgError{AMG_ERR_ARG, "initial residual is not finite (check x0 and A)"};
    if (rr0 <= tol2 * bb) {
        inf.converged = 1;
        inf.rel_true_residual = std::sqrt(rr0 / bb);
        return AMG_OK;
    }
    amg_status status = AMG_OK;
    form_start(ctx);
    int restarts = 0;
    for (;;) {
        const int stt = run_loop(ctx);
        if (stt == ST_BREAKDOWN || stt == ST_NONFINITE || stt == ST_GROWTH) {
            status = AMG_ERR_BREAKDOWN;
            set_error(stt == ST_BREAKDOWN   ? "CG breakdown: p^T A p <= 0"
                      : stt == ST_GROWTH ? "residual growth with the learned smoother"
                                         : "CG produced a non-finite value");
            break;
        }
        const int iters = ctx->hst->iter;
        double bbt, rt;
        true_residual(ctx, b, k.x, bbt, rt);
        ctx->hst->iter = iters;
        if (rt <= tol2 * bb) {
            inf.converged = 1;
            break;
        }
        if (ctx->prm.accept_recurrence && stt == ST_CONVERGED) {
            inf.converged = 2;  // the recurrence residual met tol, the FP64 true residual did not
            break;
        }
        if (stt == ST_MAXITER || restarts >= ctx->prm.max_restarts) {
            status = AMG_NOT_CONVERGED;
            set_error("iteration limit or restart limit reached");
            break;
        }
        ++restarts;
        launch_copy<double, double>(ctx->n, ctx->R64, k.r, s);
        launch_state_arm(ctx->st, tol, s);  // keeps the iteration count, clears the flags
        form_start(ctx);
    }
    // state after true_residual holds rr of the final iterate
    launch_copy<double, double>(ctx->n, k.x, x, s);
    inf.iters = ctx->hst->iter;
    inf.restarts = restarts;
    inf.rel_true_residual = std::sqrt(ctx->hst->rr / bb);
    return status;
}

// Mixed precision by iterative refinement (krylov = IR): FP64 residuals around
// an inner CG on FP32 vectors (dot products accumulated in FP64) preconditioned
// by the FP32 or BF16-storage V-cycle; the coarsest solve stays FP64.
static amg_status solve_mixed(amg_ctx *ctx, const double *b, double *x, double tol, amg_solve_info &inf) {
    hipStream_t s = ctx->stream;
    auto &k = ctx->k32;
    double *X = ctx->k64.x;
    const double tol2 = tol * tol;
    launch_state_init(ctx->st, tol, ctx->prm.maxiter, ctx->prm.krylov == AMG_KRYLOV_FCG, s);
    launch_copy<double, double>(ctx->n, x, X, s);
    double bb, rr;
    true_residual(ctx, b, X, bb, rr);
    if (!std::isfinite(bb)) throw AmgError{AMG_ERR_ARG, "right-hand side has non-finite entries"};
    if (bb == 0.0) {
        launch_fill<double>(ctx->n, 0.0, x, s);
        inf.converged = 1;
        return AMG_OK;
    }
    if (!std::isfinite(rr)) throw AmgError{AMG_ERR_ARG, "initial residual is not finite (check x0 and A)"};
    amg_status status = AMG_OK;
    int total = 0, outer = 0;
    const int max_outer = 30;
    double prev = rr;
    while (rr > tol2 * bb) {
        if (outer >= max_outer || total >= ctx->prm.maxiter) {
            status = AMG_NOT_CONVERGED;
            set_error("iteration limit reached");
            break;
        }
        // inner target: at least 1e-5 relative, no tighter than needed for tol
        const double rel = std::max(1e-5, 0.5 * std::sqrt(tol2 * bb / rr));
        launch_copy<double, float>(ctx->n, ctx->R64, k.r, s);
        launch_fill<float>(ctx->n, 0.0f, k.x, s);
        launch_state_inner(ctx->st, rel * rel * rr, ctx->prm.maxiter - total, s);
        form_start(ctx);
        const int stt = run_loop(ctx);
        total += ctx->hst->iter;
        ++outer;
        if (stt == ST_NONFINITE || stt == ST_GROWTH) {
            status = AMG_ERR_BREAKDOWN;
            set_error("inner CG produced a non-finite value");
            break;
        }
        // keep the iterate: a correction that does not reduce the FP64
        // residual is taken back (k64.p is free in this form)
        launch_copy<double, double>(ctx->n, X, ctx->k64.p, s);
        launch_add_to<float>(ctx->n, k.x, X, s);
        true_residual(ctx, b, X, bb, rr);
        if (!(rr < prev)) {
            launch_copy<double, double>(ctx->n, ctx->k64.p, X, s);
            rr = prev;
            status = stt == ST_BREAKDOWN ? AMG_ERR_BREAKDOWN : AMG_NOT_CONVERGED;
            set_error("iterative refinement stopped reducing the residual");
            break;
        }
        prev = rr;
    }
    if (rr <= tol2 * bb) inf.converged = 1;
    launch_copy<double, double>(ctx->n, X, x, s);
    inf.iters = total;
    inf.restarts = outer;
    inf.rel_true_residual = std::sqrt(rr / bb);
    return status;
}

}  // namespace saamg

extern "C" {

amg_status amg_upload(const amg_hierarchy *h, const amg_params *prm, void *hip_stream, amg_ctx **out) {
    return guarded([&]() -> amg_status {
        if (!h || !out) throw AmgError{AMG_ERR_ARG, "null argument"};
        *out = nullptr;
        std::unique_ptr<amg_ctx> ctx(new amg_ctx());
        ctx->prm = prm ? *prm : h->H.prm;
        const SetupThreads threads(ctx->prm.nthreads);
        ctx->prm.npre = h->H.prm.npre;
        ctx->prm.npost = h->H.prm.npost;
        HIP_CHECK(hipGetDevice(&ctx->device));
        ctx->scratch = scratch_address(ctx->device);
        ctx->stream = (hipStream_t)hip_stream;
        HIP_CHECK(hipEventCreateWithFlags(&ctx->fence_in, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&ctx->fence_out, hipEventDisableTiming));
        if (!ctx->stream) {
            HIP_CHECK(hipStreamCreate(&ctx->own_stream));
            ctx->stream = ctx->own_stream;
        }
        StreamFence fence(ctx.get());
        upload(ctx.get(), h->H);
        *out = ctx.release();
        return AMG_OK;
    });
}

amg_status amg_setup(const amg_bsr3 *A, const double *coords, const amg_params *prm, void *hip_stream,
                     amg_ctx **out) {
    amg_hierarchy *h = nullptr;
    amg_status s = (prm && prm->setup_device) ? amg_hierarchy_build_device(A, coords, prm, hip_stream, &h)
                                              : amg_hierarchy_build(A, coords, prm, &h);
    if (s != AMG_OK) return s;
    s = amg_upload(h, prm, hip_stream, out);
    amg_hierarchy_free(h);
    return s;
}

void amg_destroy(amg_ctx *ctx) { delete ctx; }

amg_status amg_stats(const amg_ctx *ctx, amg_stats_t *st) {
    if (!ctx || !st) {
        set_error("null argument");
        return AMG_ERR_ARG;
    }
    *st = ctx->stats;
    return AMG_OK;
}

amg_status amg_solve(amg_ctx *ctx, const double *b, double *x, double tol, amg_solve_info *info) {
    return guarded([&]() -> amg_status {
        if (!ctx || !b || !x) throw AmgError{AMG_ERR_ARG, "null argument"};
        if (!(tol > 0.0) || !std::isfinite(tol)) throw AmgError{AMG_ERR_ARG, "tol must be positive"};
        StreamFence fence(ctx);
        ensure_g(ctx);
        HIP_CHECK(hipEventRecord(ctx->ev0, ctx->stream));
        amg_solve_info inf{};
        const bool learned = ctx->lr.active;
        if (learned) HIP_CHECK(hipMemcpyAsync(ctx->lr.x0, x, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
        auto run = [&](amg_solve_info &i) {
            return iterative_refinement(ctx) ? solve_mixed(ctx, b, x, tol, i) : solve_fp64(ctx, b, x, tol, i);
        };
        amg_status st = run(inf);
        if (learned && st == AMG_ERR_BREAKDOWN) {
            // fallback: block Jacobi, restart from the caller's initial guess
            restore_jacobi(ctx);
            ensure_g(ctx);
            HIP_CHECK(hipMemcpyAsync(x, ctx->lr.x0, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
            amg_solve_info again{};
            set_error("");
            st = run(again);
            again.iters += inf.iters;
            again.fell_back = 1;
            inf = again;
        }
        HIP_CHECK(hipEventRecord(ctx->ev1, ctx->stream));
        HIP_CHECK(hipEventSynchronize(ctx->ev1));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        inf.solve_ms = ms;
        if (info) *info = inf;
        return st;
    });
}

// V-cycle of the context's form with FP64 input and output (conversion in and
// out of the context's level-1 buffers for the mixed forms).
amg_status amg_vcycle(amg_ctx *ctx, const double *r, double *z) {
    return guarded([&]() -> amg_status {
        if (!ctx || !r || !z || r == z) throw AmgError{AMG_ERR_ARG, "invalid vectors"};
        StreamFence fence(ctx);
        ensure_g(ctx);
        hipStream_t s = ctx->stream;
        if (ctx->precision == AMG_FP64) {
            precondition<double, double>(ctx, ctx->v64, r, z, false, 0, SITE_NONE);
        } else {
            launch_copy<double, float>(ctx->n, r, ctx->k32.r, s);
            if (ctx->precision == AMG_FP32)
                precondition<float, float>(ctx, ctx->v32, ctx->k32.r, ctx->k32.z, false, 0, SITE_NONE);
            else
                precondition<bf16_t, float>(ctx, ctx->v16, ctx->k32.r, ctx->k32.z, false, 0, SITE_NONE);
            launch_copy<float, double>(ctx->n, ctx->k32.z, z, s);
        }
        HIP_CHECK(hipGetLastError());
        return AMG_OK;
    });
}

amg_status amg_true_residual(amg_ctx *ctx, const double *b, const double *x, double *rel) {
    return guarded([&]() -> amg_status {
        if (!ctx || !b || !x || !rel) throw AmgError{AMG_ERR_ARG, "null argument"};
        StreamFence fence(ctx);
        double bb, rr;
        true_residual(ctx, b, x, bb, rr);
        *rel = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        return AMG_OK;
    });
}

amg_status amg_true_residual_noalloc(amg_ctx *ctx, const double *b, const double *x, double *r,
                                     double *norms, double *rel) {
    return guarded([&]() -> amg_status {
        if (!ctx || !b || !x || !r || !norms) throw AmgError{AMG_ERR_ARG, "null argument"};
        if (r == b || r == x) throw AmgError{AMG_ERR_ARG, "r must not alias b or x"};
        const auto &A = ctx->A64;
        const int64_t grid = product_grid(A.v.rows, A.v.nslices, A.C);
        const int64_t cap = (int64_t)((AMG_NOALLOC_SCRATCH_BYTES - kScratchHeader) / (2 * sizeof(double)));
        if (grid > cap)
            throw AmgError{AMG_ERR_ARG, "the finest operator's product needs " + std::to_string(grid) +
                                            " workgroup partial sums; the static scratch holds " +
                                            std::to_string(cap)};
        StreamFence fence(ctx);
        hipStream_t s = ctx->stream;
        DevState *st = static_cast<DevState *>(ctx->scratch);
        double *partials = reinterpret_cast<double *>(static_cast<char *>(ctx->scratch) + kScratchHeader);
        // every partial the finalize adds and both norms it sets are written
        // by this call first: nothing in the array needs clearing
        launch_sell<double, double>(A.v, A.C, MODE_RESID_NORM, x, b, r, nullptr, partials, st, 0, SITE_INIT, s);
        launch_state_norms(st, norms, s);
        HIP_CHECK(hipGetLastError());
        if (rel) {
            HIP_CHECK(hipMemcpyAsync(ctx->hst, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            const double bb = ctx->hst->bb, rr = ctx->hst->rr;
            *rel = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        }
        return AMG_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// single kernels for tests and timing
// ---------------------------------------------------------------------------

namespace saamg {

// A vector of level v that is none of the given ones (work space of the
// ILU(0) sweeps in the single-kernel entry points).
template <typename V, typename T>
static T *spare_buffer(const Level<V, T> &v, const void *a, const void *b, const void *c) {
    for (T *p : {v.f, v.x, v.t, v.y})
        if ((const void *)p != a && (const void *)p != b && (const void *)p != c) return p;
    throw AmgError{AMG_ERR_ARG, "no free level buffer"};
}

// Launch op on level l of a V-cycle in its own precision; buffers are the
// level's (in, in2 -> out as documented for amg_debug_apply).
template <typename V, typename T>
static void level_op(amg_ctx *ctx, Vcycle<V, T> &vc, int l, int op, const T *in, const T *in2, T *out) {
    hipStream_t s = ctx->stream;
    if (op == 5) {
        launch_dense_gemv<T>(vc.n_coarse, vc.Ainv, in, out, ctx->st, 0, s);
        return;
    }
    auto &v = vc.lv[l];
    switch (op) {
        case 0: launch_sell<V, T>(v.A.v, v.A.C, MODE_SPMV, in, nullptr, out, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s); break;
        case 1: launch_sell<V, T>(v.R.v, v.R.C, MODE_SPMV, in, nullptr, out, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s); break;
        case 2: launch_sell<V, T>(v.P.v, v.P.C, MODE_SPMV, in, nullptr, out, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s); break;
        case 3:
            if (v.ilu)
                v.ilu_solve(in, spare_buffer(v, in, nullptr, out), out, ctx->partials, ctx->st, 0, s);
            else
                launch_jacobi0<T>(v.rows, v.M, in, out, ctx->st, 0, s);
            break;
        case 4:
            if (v.ilu) {
                // out = in2 + (L U)^{-1} (in - A in2), the residual and the correction in out
                T *w = spare_buffer(v, in, in2, out);
                launch_sell<V, T>(v.A.v, v.A.C, MODE_RESID, in2, in, out, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s);
                v.ilu_solve(out, w, out, ctx->partials, ctx->st, 0, s);
                launch_add2<T>(3 * (int64_t)v.rows, in2, out, out, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s);
            } else {
                launch_sell<V, T>(v.A.v, v.A.C, MODE_SMOOTH, in2, in, out, v.M, ctx->partials, ctx->st, 0, SITE_NONE, s);
            }
            break;
        case 6: launch_sell<V, T>(v.A.v, v.A.C, MODE_RESID, in2, in, out, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s); break;
        case 7: launch_sell<V, T>(v.A.v, v.A.C, MODE_SMOOTH_DOT, in2, in, out, v.M, ctx->partials, ctx->st, 0, SITE_NONE, s); break;
        case 8: launch_sell<V, T>(v.A.v, v.A.C, MODE_SPMV_DOT, in, nullptr, out, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s); break;
        case 11: launch_sell<V, T>(v.AM.v, v.AM.C, MODE_RESID, in, in, out, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s); break;
        case 12: launch_sell<V, T>(v.G.v, v.G.C, v.post_mode(false), in, in2, out, v.post_m(), ctx->partials, ctx->st, 0, SITE_NONE, s); break;
        case 13: launch_sell<V, T>(v.G.v, v.G.C, v.post_mode(true), in, in2, out, v.post_m(), ctx->partials, ctx->st, 0, SITE_NONE, s); break;
        default: throw AmgError{AMG_ERR_ARG, "unknown op"};
    }
}

// whether level l of the context's V-cycle uses the fused sweeps
// whether level l of the context's V-cycle has the fused sweep for op 11
// (AM) or 12 / 13 (G)
static bool level_fused(const amg_ctx *ctx, int l, int op) {
    if (l < 0 || l + 1 >= ctx->stats.levels) return false;
    auto has = [op](const auto &v) { return op == 11 ? v.has_am : v.has_g; };
    if (ctx->precision == AMG_FP64) return has(ctx->v64.lv[l]);
    return ctx->precision == AMG_FP32 ? has(ctx->v32.lv[l]) : has(ctx->v16.lv[l]);
}

// sizes (in units of the level vectors) of an op's input and output
static void op_sizes(const amg_ctx *ctx, int l, int op, int64_t &nin, int64_t &nout) {
    const amg_stats_t &st = ctx->stats;
    if (op == 5) {
        nin = nout = st.n_coarse;
        return;
    }
    const int64_t nf = 3 * (int64_t)st.nb[l], nc = 3 * (int64_t)st.nb[l + 1];
    nin = (op == 2 || op == 12) ? nc : nf;
    nout = op == 1 ? nc : nf;
}

template <typename V, typename T>
static void debug_op_mixed(amg_ctx *ctx, Vcycle<V, T> &vc, int l, int op, const double *in, const double *in2,
                           double *out) {
    hipStream_t s = ctx->stream;
    int64_t nin, nout;
    op_sizes(ctx, l, op, nin, nout);
    // level scratch: coarse-side vectors live on level l+1 (or the coarsest level)
    const int lc = op == 5 ? (int)vc.lv.size() - 1 : l + 1;
    T *ti = (op == 2 || op == 12) ? vc.lv[lc].t : (op == 5 ? vc.lv[lc].f : vc.lv[l].t);
    T *ti2 = vc.lv[op == 5 ? lc : l].x;
    T *to = (op == 1) ? vc.lv[lc].y : (op == 5 ? vc.lv[lc].y : vc.lv[l].y);
    launch_copy<double, T>(nin, in, ti, s);
    if (in2) launch_copy<double, T>(nout, in2, ti2, s);
    if (op == 12) launch_copy<double, T>(nout, out, to, s);  // t, updated in place
    level_op<V, T>(ctx, vc, l, op, ti, in2 ? ti2 : nullptr, to);
    launch_copy<T, double>(nout, to, out, s);
}

}  // namespace saamg

extern "C" amg_status amg_debug_apply(amg_ctx *ctx, int32_t level, int32_t op, const double *in,
                                      const double *in2, double *out) {
    return guarded([&]() -> amg_status {
        if (!ctx || !in || !out) throw AmgError{AMG_ERR_ARG, "null argument"};
        if (op < 0 || (op > 6 && op != 11 && op != 12)) throw AmgError{AMG_ERR_ARG, "unknown op"};
        const int L = ctx->stats.levels;
        if (op != 5 && (level < 0 || level + 1 >= L))
            throw AmgError{AMG_ERR_ARG, "level has no sparse operators (coarsest or out of range)"};
        if ((op == 4 || op == 6 || op == 12) && (!in2 || in2 == out)) throw AmgError{AMG_ERR_ARG, "op needs in2 != out"};
        if ((op == 11 || op == 12) && !level_fused(ctx, level, op))
            throw AmgError{AMG_ERR_ARG, "level has no fused sweeps"};
        if ((op == 11 || op == 12) && in == out) throw AmgError{AMG_ERR_ARG, "op needs in != out"};
        StreamFence fence(ctx);
        ensure_g(ctx);
        if (ctx->precision == AMG_FP64)
            level_op<double, double>(ctx, ctx->v64, level, op, in, in2, out);
        else if (ctx->precision == AMG_FP32)
            debug_op_mixed<float, float>(ctx, ctx->v32, level, op, in, in2, out);
        else
            debug_op_mixed<bf16_t, float>(ctx, ctx->v16, level, op, in, in2, out);
        HIP_CHECK(hipGetLastError());
        return AMG_OK;
    });
}

namespace saamg {

static Krylov<double> &krylov_of(amg_ctx *ctx, double *) { return ctx->k64; }
static Krylov<float> &krylov_of(amg_ctx *ctx, float *) { return ctx->k32; }

template <typename V, typename T>
static double time_level_op(amg_ctx *ctx, Vcycle<V, T> &vc, int level, int op, int reps, double &nb) {
    hipStream_t s = ctx->stream;
    const double sv = sizeof(V), st = sizeof(T);
    const int L = (int)vc.lv.size();
    std::function<void()> launch;
    if (op == 9) {
        if (L < 2) throw AmgError{AMG_ERR_ARG, "single-level hierarchy has no V-cycle"};
        Krylov<T> &k = krylov_of(ctx, (T *)nullptr);
        T *r = k.r, *z = k.z;
        launch_fill<T>(ctx->n, T(1), r, s);
        launch = [&, r, z]() { vc.run(r, z, false, 0, SITE_NONE, ctx->partials, ctx->st, s); };
        nb = ctx->stats.vcycle_bytes;
    } else if (op == 5) {
        auto &cl = vc.lv[L - 1];
        launch_fill<T>(vc.n_coarse, T(1), cl.f, s);
        launch = [&]() { launch_dense_gemv<T>(vc.n_coarse, vc.Ainv, cl.f, cl.y, ctx->st, 0, s); };
        nb = (double)vc.n_coarse * vc.n_coarse * 8.0 + 2.0 * st * vc.n_coarse;
    } else if (op == 16) {
        if (!vc.W) throw AmgError{AMG_ERR_ARG, "no folded coarsest product in this V-cycle"};
        auto &cl = vc.lv[L - 1];
        auto &wl = vc.lv[vc.w_level];
        const int nf = 3 * wl.rows;
        launch_fill<T>(nf, T(1), wl.t, s);
        launch = [&, nf]() { launch_dense_rect<T>(vc.n_coarse, nf, vc.W, wl.t, cl.y, ctx->st, 0, s); };
        nb = (double)vc.n_coarse * nf * 8.0 + st * (nf + vc.n_coarse);
    } else {
        auto &v = vc.lv[level];
        auto &c = vc.lv[level + 1];
        const double rows = v.rows, crow = c.rows, sm = st;
        launch_fill<T>(3 * (int64_t)v.rows, T(1), v.x, s);
        launch_fill<T>(3 * (int64_t)v.rows, T(1), v.f, s);
        launch_fill<T>(3 * (int64_t)c.rows, T(1), c.y, s);
        switch (op) {
            case 0: launch = [&]() { level_op<V, T>(ctx, vc, level, 0, v.x, nullptr, v.t); }; nb = sell_bytes(v.A, 6 * st * rows); break;
            case 1: launch = [&]() { level_op<V, T>(ctx, vc, level, 1, v.x, nullptr, c.f); }; nb = sell_bytes(v.R, 3 * st * (rows + crow)); break;
            case 2:
                launch = [&]() { launch_sell<V, T>(v.P.v, v.P.C, MODE_ADD, c.y, nullptr, v.t, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s); };
                nb = sell_bytes(v.P, 3 * st * crow + 6 * st * rows);
                break;
            case 3: launch = [&]() { level_op<V, T>(ctx, vc, level, 3, v.f, nullptr, v.t); }; nb = (9 * sm + 6 * st) * rows; break;
            case 4: launch = [&]() { level_op<V, T>(ctx, vc, level, 4, v.f, v.x, v.t); }; nb = sell_bytes(v.A, 9 * sm * rows + 9 * st * rows); break;
            case 6: launch = [&]() { level_op<V, T>(ctx, vc, level, 6, v.f, v.x, v.t); }; nb = sell_bytes(v.A, 9 * st * rows); break;
            case 7: launch = [&]() { level_op<V, T>(ctx, vc, level, 7, v.f, v.x, v.t); }; nb = sell_bytes(v.A, 9 * sm * rows + 9 * st * rows); break;
            case 8: launch = [&]() { level_op<V, T>(ctx, vc, level, 8, v.x, nullptr, v.t); }; nb = sell_bytes(v.A, 6 * st * rows); break;
            case 11: launch = [&]() { level_op<V, T>(ctx, vc, level, 11, v.f, nullptr, v.t); }; nb = sell_bytes(v.AM, 6 * st * rows); break;
            case 12:
            case 13:
                // in place on y: the value it holds does not change the work
                launch = [&, op]() { level_op<V, T>(ctx, vc, level, op, c.y, v.f, v.t); };
                nb = sell_bytes(v.G, 3 * st * crow + 9 * st * rows + (v.MM ? 18 : 9) * sm * rows);
                break;
            case 14:  // G's stream alone: the fused operator as a plain product
                launch = [&]() { launch_sell<V, T>(v.G.v, v.G.C, MODE_SPMV, c.y, nullptr, v.t, nullptr, ctx->partials, ctx->st, 0, SITE_NONE, s); };
                nb = sell_bytes(v.G, 3 * st * crow + 3 * st * rows);
                break;
            case 15:  // A's stream with the fused post-sweep's epilogue z = A x + M (f + y)
                launch = [&]() { launch_sell<V, T>(v.A.v, v.A.C, MODE_POST, v.x, v.f, v.t, v.M, ctx->partials, ctx->st, 0, SITE_NONE, s); };
                nb = sell_bytes(v.A, 3 * st * rows + 9 * st * rows + 9 * sm * rows);
                break;
            default: throw AmgError{AMG_ERR_ARG, "unknown op"};
        }
    }
    launch();  // warm-up
    HIP_CHECK(hipEventRecord(ctx->ev0, s));
    for (int i = 0; i < reps; ++i) launch();
    HIP_CHECK(hipEventRecord(ctx->ev1, s));
    HIP_CHECK(hipEventSynchronize(ctx->ev1));
    HIP_CHECK(hipGetLastError());
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    return ms / reps;
}

}  // namespace saamg

extern "C" amg_status amg_time_op(amg_ctx *ctx, int32_t level, int32_t op, int32_t reps, double *avg_ms,
                                  double *bytes) {
    return guarded([&]() -> amg_status {
        if (!ctx || !avg_ms || !bytes || reps < 1) throw AmgError{AMG_ERR_ARG, "invalid argument"};
        if (op < 0 || op > 16) throw AmgError{AMG_ERR_ARG, "unknown op"};
        const int L = ctx->stats.levels;
        const bool sparse_op = op != 5 && op != 9 && op != 10 && op != 16;
        if (sparse_op && (level < 0 || level + 1 >= L)) throw AmgError{AMG_ERR_ARG, "level has no sparse operators"};
        if ((op >= 11 && op <= 14) && !level_fused(ctx, level, op == 14 ? 12 : op))
            throw AmgError{AMG_ERR_ARG, "level has no fused sweeps"};
        if (op == 13 && level != 0) throw AmgError{AMG_ERR_ARG, "op 13 exists on level 0 only"};
        if ((op == 7 || op == 8) && level != 0) throw AmgError{AMG_ERR_ARG, "ops 7 and 8 exist on level 0 only"};
        StreamFence fence(ctx);
        ensure_g(ctx);
        hipStream_t s = ctx->stream;
        double nb = 0.0, ms = 0.0;
        if (op == 10) {
            // one iteration of the context's CG from a consistent state, re-armed
            // so no iteration is skipped
            launch_state_init(ctx->st, 0.0, 1 << 30, 0, s);
            launch_fill<double>(ctx->n, 1.0, ctx->k64.r, s);
            launch_fill<double>(ctx->n, 0.0, ctx->k64.x, s);
            if (ctx->precision != AMG_FP64) {
                launch_fill<float>(ctx->n, 1.0f, ctx->k32.r, s);
                launch_fill<float>(ctx->n, 0.0f, ctx->k32.x, s);
            }
            form_start(ctx);
            form_iteration(ctx);
            HIP_CHECK(hipEventRecord(ctx->ev0, s));
            for (int i = 0; i < reps; ++i) form_iteration(ctx);
            HIP_CHECK(hipEventRecord(ctx->ev1, s));
            HIP_CHECK(hipEventSynchronize(ctx->ev1));
            HIP_CHECK(hipGetLastError());
            float f = 0.f;
            HIP_CHECK(hipEventElapsedTime(&f, ctx->ev0, ctx->ev1));
            ms = f / reps;
            nb = ctx->stats.iter_bytes;
        } else if (ctx->precision == AMG_FP64) {
            ms = time_level_op<double, double>(ctx, ctx->v64, level, op, reps, nb);
        } else if (ctx->precision == AMG_FP32) {
            ms = time_level_op<float, float>(ctx, ctx->v32, level, op, reps, nb);
        } else {
            ms = time_level_op<bf16_t, float>(ctx, ctx->v16, level, op, reps, nb);
        }
        *avg_ms = ms;
        *bytes = nb;
        return AMG_OK;
    });
}

// ---------------------------------------------------------------------------
// multi-right-hand-side solve
// ---------------------------------------------------------------------------

namespace saamg {

template <typename V, typename T>
static void alloc_multi(amg_ctx *ctx, Vcycle<V, T> &vc) {
    MultiBufs &m = ctx->mb;
    if (m.ready) return;
    const size_t nk = (size_t)ctx->n * kMaxRhs;
    m.X = ctx->al.get<double>(nk);
    m.R = ctx->al.get<double>(nk);
    m.P = ctx->al.get<double>(nk);
    m.Q = ctx->al.get<double>(nk);
    m.rv = ctx->al.get<T>(nk);
    m.zv = ctx->al.get<T>(nk);
    for (auto &lv : vc.lv) {
        const size_t len = 3 * (size_t)lv.rows * kMaxRhs;
        m.f.push_back(ctx->al.get<T>(len));
        m.x.push_back(ctx->al.get<T>(len));
        m.t.push_back(ctx->al.get<T>(len));
        m.y.push_back(ctx->al.get<T>(len));
    }
    // per-workgroup column sums of any multi-column launch (at most kMaxMGrid
    // workgroups), then the finalize's range sums
    m.partials = ctx->al.get<double>((size_t)(kMaxMGrid + kMSplit) * 64);
    m.gemm_part = ctx->al.get<double>((size_t)kMaxGemmSlices * std::max(vc.n_coarse, 1) * kMaxRhs);
    m.st = ctx->al.get<MState>(1);
    HIP_CHECK(hipHostMalloc((void **)&m.hst, sizeof(MState), hipHostMallocDefault));
    m.ready = true;
    ctx->stats.device_bytes = (double)ctx->al.bytes;
}

// z = V(f1) for k columns at once (same sequence as Vcycle::run)
template <typename V, typename T>
static void vcycle_multi(amg_ctx *ctx, Vcycle<V, T> &vc, int k, const T *f1, T *z, bool pre_done, int gated,
                         int site) {
    MultiBufs &m = ctx->mb;
    hipStream_t s = ctx->stream;
    const int L = (int)vc.lv.size();
    std::vector<T *> cur(L), out(L);
    for (int l = 0; l + 1 < L; ++l) {
        auto &v = vc.lv[l];
        const T *f = l == 0 ? f1 : (T *)m.f[l];
        T *x = (T *)m.x[l], *y = (T *)m.y[l], *t = (T *)m.t[l];
        if (l > 0 && v.has_am && v.has_g) {  // fused sweeps (as in Vcycle::run)
            launch_spmm<V, T>(v.AM.v, v.AM.C, MODE_RESID, k, f, f, t, nullptr, m.partials, m.st, gated, MSITE_NONE,
                              s);
            launch_spmm<V, T>(v.R.v, v.R.C, MODE_SPMV, k, t, nullptr, (T *)m.f[l + 1], nullptr, m.partials, m.st,
                              gated, MSITE_NONE, s);
            continue;
        }
        if (l == 0 && v.has_g && vc.npost == 1) t = z;  // the fused post-sweep overwrites it in place
        if (!(l == 0 && pre_done)) launch_jacobi0_m<T>(v.rows, k, v.M, f, x, m.st, gated, s);
        T *c = x;
        for (int q = 1; q < vc.npre; ++q) {
            T *o = (c == x) ? y : x;
            launch_spmm<V, T>(v.A.v, v.A.C, MODE_SMOOTH, k, c, f, o, v.M, m.partials, m.st, gated, MSITE_NONE, s);
            c = o;
        }
        cur[l] = c;
        launch_spmm<V, T>(v.A.v, v.A.C, MODE_RESID, k, c, f, t, nullptr, m.partials, m.st, gated, MSITE_NONE, s);
        launch_spmm<V, T>(v.R.v, v.R.C, MODE_SPMV, k, t, nullptr, (T *)m.f[l + 1], nullptr, m.partials, m.st, gated,
                          MSITE_NONE, s);
    }
    launch_dense_gemm<T>(vc.n_coarse, k, vc.Ainv, (T *)m.f[L - 1], (T *)m.y[L - 1], m.gemm_part, m.st, gated, s);
    out[L - 1] = (T *)m.y[L - 1];
    for (int l = L - 2; l >= 0; --l) {
        auto &v = vc.lv[l];
        const T *f = l == 0 ? f1 : (T *)m.f[l];
        T *c = cur[l];
        T *x = (T *)m.x[l], *y = (T *)m.y[l], *t = (T *)m.t[l];
        if (l > 0 && v.has_am && v.has_g) {
            launch_spmm<V, T>(v.G.v, v.G.C, v.post_mode_rows(false), k, out[l + 1], f, t, v.post_m_rows(), m.partials, m.st,
                              gated, MSITE_NONE, s);
            out[l] = t;
            continue;
        }
        if (l == 0 && v.has_g && vc.npost == 1) {
            const bool dot = site != MSITE_NONE;
            launch_spmm<V, T>(v.G.v, v.G.C, v.post_mode_rows(dot), k, out[1], f, z, v.post_m_rows(), m.partials, m.st, gated,
                              dot ? site : MSITE_NONE, s);
            out[0] = z;
            continue;
        }
        launch_spmm<V, T>(v.P.v, v.P.C, MODE_ADD, k, out[l + 1], nullptr, c, nullptr, m.partials, m.st, gated,
                          MSITE_NONE, s);
        T *spare = (c == x) ? y : x;
        T *dest = l == 0 ? z : spare;
        T *src = c;
        for (int q = 0; q + 1 < vc.npost; ++q) {
            T *o = (src == c) ? t : c;
            launch_spmm<V, T>(v.A.v, v.A.C, MODE_SMOOTH, k, src, f, o, v.Mt, m.partials, m.st, gated, MSITE_NONE, s);
            src = o;
        }
        const bool dot = (l == 0 && site != MSITE_NONE);
        launch_spmm<V, T>(v.A.v, v.A.C, dot ? MODE_SMOOTH_DOT : MODE_SMOOTH, k, src, f, dest, v.Mt, m.partials, m.st,
                          gated, dot ? site : MSITE_NONE, s);
        out[l] = dest;
    }
}

template <typename V, typename T>
static void multi_iteration(amg_ctx *ctx, Vcycle<V, T> &vc, int k) {
    MultiBufs &m = ctx->mb;
    hipStream_t s = ctx->stream;
    launch_spmm<double, double>(ctx->A64.v, ctx->A64.C, MODE_SPMV_DOT, k, m.P, nullptr, m.Q, nullptr, m.partials,
                                m.st, 1, MSITE_PQ, s);
    launch_cg_update_m<T>(ctx->nb, k, m.X, m.P, m.R, m.Q, vc.lv[0].M, (T *)m.rv, (T *)m.x[0],
                          ctx->prm.krylov == AMG_KRYLOV_FCG ? (const T *)m.zv : nullptr, m.partials, m.st, s);
    vcycle_multi<V, T>(ctx, vc, k, (const T *)m.rv, (T *)m.zv, true, 1, MSITE_RZ);
    launch_cg_dir_m<T>(ctx->nb, k, (const T *)m.zv, m.P, m.st, s);
}

template <typename V, typename T>
static amg_status solve_multi_t(amg_ctx *ctx, Vcycle<V, T> &vc, int k, const double *B, double *Xout, double tol,
                                amg_solve_info *info) {
    if (vc.lv.size() < 2) throw AmgError{AMG_ERR_UNSUPPORTED, "multi-RHS solve needs a hierarchy of two or more levels"};
    alloc_multi<V, T>(ctx, vc);
    MultiBufs &m = ctx->mb;
    hipStream_t s = ctx->stream;
    const int64_t nk = ctx->n * k;
    launch_mstate_init(m.st, k, ctx->prm.maxiter, ctx->prm.krylov == AMG_KRYLOV_FCG, s);
    launch_copy<double, double>(nk, Xout, m.X, s);
    launch_spmm<double, double>(ctx->A64.v, ctx->A64.C, MODE_RESID_NORM, k, m.X, B, m.R, nullptr, m.partials, m.st,
                                0, MSITE_INIT, s);
    launch_mstate_arm(m.st, tol, s);
    HIP_CHECK(hipMemcpyAsync(m.hst, m.st, sizeof(MState), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j) {
        if (!std::isfinite(m.hst->bb[j])) throw AmgError{AMG_ERR_ARG, "right-hand side has non-finite entries"};
        if (!std::isfinite(m.hst->rr[j])) throw AmgError{AMG_ERR_ARG, "initial residual is not finite"};
    }
    if (!m.hst->all_done) {
        launch_copy<double, T>(nk, m.R, (T *)m.rv, s);
        vcycle_multi<V, T>(ctx, vc, k, (const T *)m.rv, (T *)m.zv, false, 0, MSITE_RZ0);
        launch_copy<T, double>(nk, (const T *)m.zv, m.P, s);
        const int chunk = std::max(1, ctx->prm.check_every);
        if (ctx->prm.use_graphs && (!m.exec || m.graph_k != k)) {
            if (m.exec) HIP_CHECK(hipGraphExecDestroy(m.exec));
            if (m.graph) HIP_CHECK(hipGraphDestroy(m.graph));
            m.exec = nullptr;
            m.graph = nullptr;
            HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < chunk; ++i) multi_iteration<V, T>(ctx, vc, k);
            HIP_CHECK(hipStreamEndCapture(s, &m.graph));
            HIP_CHECK(hipGraphInstantiate(&m.exec, m.graph, nullptr, nullptr, 0));
            m.graph_k = k;
        }
        for (;;) {
            if (ctx->prm.use_graphs)
                HIP_CHECK(hipGraphLaunch(m.exec, s));
            else
                for (int i = 0; i < chunk; ++i) multi_iteration<V, T>(ctx, vc, k);
            HIP_CHECK(hipGetLastError());
            HIP_CHECK(hipMemcpyAsync(m.hst, m.st, sizeof(MState), hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            if (m.hst->all_done) break;
        }
    }
    std::vector<int32_t> iters(m.hst->iter, m.hst->iter + k), status(m.hst->status, m.hst->status + k);
    // FP64 true residual of every column
    launch_spmm<double, double>(ctx->A64.v, ctx->A64.C, MODE_RESID_NORM, k, m.X, B, m.R, nullptr, m.partials, m.st,
                                0, MSITE_INIT, s);
    HIP_CHECK(hipMemcpyAsync(m.hst, m.st, sizeof(MState), hipMemcpyDeviceToHost, s));
    launch_copy<double, double>(nk, m.X, Xout, s);
    HIP_CHECK(hipStreamSynchronize(s));
    amg_status res = AMG_OK;
    const double tol2 = tol * tol;
    for (int j = 0; j < k; ++j) {
        const double bb = m.hst->bb[j], rr = m.hst->rr[j];
        const bool truly = bb == 0.0 || rr <= tol2 * bb;
        const bool conv = truly || (ctx->prm.accept_recurrence && status[j] == ST_CONVERGED);
        if (status[j] == ST_BREAKDOWN || status[j] == ST_NONFINITE) {
            res = AMG_ERR_BREAKDOWN;
            set_error("CG breakdown in column " + std::to_string(j));
        } else if (!conv && res == AMG_OK) {
            res = AMG_NOT_CONVERGED;
            set_error("column " + std::to_string(j) + " did not reach the tolerance");
        }
        if (info) {
            info[j] = amg_solve_info{};
            info[j].iters = iters[j];
            info[j].converged = truly ? 1 : conv ? 2 : 0;
            info[j].rel_true_residual = bb > 0 ? std::sqrt(rr / bb) : 0.0;
        }
    }
    return res;
}

// Z = V(R) for k columns: FP64 in and out, the V-cycle in the context's precision
template <typename V, typename T>
static void vcycle_multi_entry(amg_ctx *ctx, Vcycle<V, T> &vc, int k, const double *R, double *Z) {
    alloc_multi<V, T>(ctx, vc);
    MultiBufs &m = ctx->mb;
    hipStream_t s = ctx->stream;
    const int64_t nk = ctx->n * k;
    launch_copy<double, T>(nk, R, (T *)m.rv, s);
    if (vc.lv.size() > 1)
        vcycle_multi<V, T>(ctx, vc, k, (const T *)m.rv, (T *)m.zv, false, 0, MSITE_NONE);
    else
        launch_dense_gemm<T>(vc.n_coarse, k, vc.Ainv, (const T *)m.rv, (T *)m.zv, m.gemm_part, m.st, 0, s);
    launch_copy<T, double>(nk, (const T *)m.zv, Z, s);
}

}  // namespace saamg

extern "C" amg_status amg_vcycle_multi(amg_ctx *ctx, int32_t k, const double *R, double *Z) {
    return guarded([&]() -> amg_status {
        if (!ctx || !R || !Z || R == Z) throw AmgError{AMG_ERR_ARG, "invalid vectors"};
        if (k < 1 || k > kMaxRhs) throw AmgError{AMG_ERR_ARG, "k must be in [1, 32]"};
        if (ctx->prm.smoother == AMG_SMOOTHER_ILU0)
            throw AmgError{AMG_ERR_UNSUPPORTED, "the multi-column V-cycle has no ILU(0) smoother"};
        StreamFence fence(ctx);
        ensure_g(ctx);
        if (ctx->precision == AMG_FP64)
            vcycle_multi_entry<double, double>(ctx, ctx->v64, k, R, Z);
        else if (ctx->precision == AMG_FP32)
            vcycle_multi_entry<float, float>(ctx, ctx->v32, k, R, Z);
        else
            vcycle_multi_entry<bf16_t, float>(ctx, ctx->v16, k, R, Z);
        HIP_CHECK(hipGetLastError());
        return AMG_OK;
    });
}

extern "C" amg_status amg_solve_multi(amg_ctx *ctx, int32_t k, const double *B, double *X, double tol,
                                      amg_solve_info *info_k) {
    return guarded([&]() -> amg_status {
        if (!ctx || !B || !X) throw AmgError{AMG_ERR_ARG, "null argument"};
        if (k < 1 || k > kMaxRhs) throw AmgError{AMG_ERR_ARG, "k must be in [1, 32]"};
        if (!(tol > 0.0) || !std::isfinite(tol)) throw AmgError{AMG_ERR_ARG, "tol must be positive"};
        if (ctx->prm.smoother == AMG_SMOOTHER_ILU0)
            throw AmgError{AMG_ERR_UNSUPPORTED, "the multi-right-hand-side solve has no ILU(0) smoother"};
        StreamFence fence(ctx);
        ensure_g(ctx);
        HIP_CHECK(hipEventRecord(ctx->ev0, ctx->stream));
        amg_status st;
        if (ctx->precision == AMG_FP64)
            st = solve_multi_t<double, double>(ctx, ctx->v64, k, B, X, tol, info_k);
        else if (ctx->precision == AMG_FP32)
            st = solve_multi_t<float, float>(ctx, ctx->v32, k, B, X, tol, info_k);
        else
            st = solve_multi_t<bf16_t, float>(ctx, ctx->v16, k, B, X, tol, info_k);
        HIP_CHECK(hipEventRecord(ctx->ev1, ctx->stream));
        HIP_CHECK(hipEventSynchronize(ctx->ev1));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        if (info_k)
            for (int j = 0; j < k; ++j) info_k[j].solve_ms = ms;
        return st;
    });
}

// ---------------------------------------------------------------------------
// batch of independent problems in one solve
// ---------------------------------------------------------------------------
//
// Each problem keeps its own hierarchy (built on the host exactly as for a
// single solve).  On the device the level-l operators of all problems are
// concatenated block-diagonally, problems still coarsening first and the
// problems whose coarsest level is l after them, so every V-cycle step is one
// launch for the whole batch; the coarsest solves of level l run as one
// batched dense product.  The outer FP64 CG keeps one alpha, beta and
// convergence flag per problem (segmented fixed-order reductions).

namespace saamg {

struct BLevel {
    int32_t rows = 0;  // block rows of all problems active at this level
    int32_t m = 0;     // block rows of problems that coarsen further
    // coarsest solves at this level (rows m..rows)
    int32_t ncs = 0;   // scalar rows
    int32_t *cmap = nullptr;        // scalar coarse row -> entry of the coarse table
    int64_t *c_off = nullptr;       // per entry: scalar offset of the problem in this level's vectors
    int32_t *c_n = nullptr;         // per entry: size
    int64_t *c_a = nullptr;         // per entry: offset of its inverse in the Ainv pool
    int32_t *c_slot = nullptr;      // per entry: the problem's slot (its convergence flag)
};

template <typename V, typename T>
struct BatchDev {
    Vcycle<V, T> vc;        // level operators (rows 0..m of each level)
    std::vector<BLevel> bl;
};

}  // namespace saamg

struct amg_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    amg_params prm{};
    saamg::DevAlloc al;
    int np = 0;
    int precision = AMG_FP32;
    std::vector<int64_t> off0;   // problem -> scalar offset in level-0 vectors
    std::vector<int64_t> n0;     // problem -> scalar size
    int64_t n = 0;               // scalar size of level 0
    int32_t nb = 0;
    saamg::DevSell<double> A64;  // block-diagonal FP64 operator of all problems
    saamg::BatchDev<double, double> d64;
    saamg::BatchDev<float, float> d32;
    double *Ainv = nullptr;      // pool of coarsest inverses
    double *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr;  // outer FP64 CG
    void *rv = nullptr, *zv = nullptr;                              // V-cycle precision
    int64_t *seg = nullptr;      // np+1 scalar segment offsets (level 0 order)
    int32_t *rowprob = nullptr;  // block row (level 0) -> problem slot
    double *partials = nullptr;
    saamg::DevState *st = nullptr;  // gate: done = every problem finished
    double *bsc = nullptr;          // per-problem scalars: 8 arrays of np
    int32_t *bint = nullptr;        // per-problem ints: iter, done, status (3 arrays of np)
    double *hsc = nullptr;          // pinned mirrors
    int32_t *hint = nullptr;
    saamg::DevState *hst = nullptr;
    const double **hptr = nullptr;  // pinned: the caller's b and x pointers per slot (2 np)
    const double **dptr = nullptr;  // device copy of hptr
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<int> slot_of;    // user problem index -> level-0 slot
    ~amg_batch() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (hsc) (void)hipHostFree(hsc);
        if (hint) (void)hipHostFree(hint);
        if (hst) (void)hipHostFree(hst);
        if (hptr) (void)hipHostFree(hptr);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (own_stream) (void)hipStreamDestroy(own_stream);
    }
};

namespace saamg {

// per-problem scalar arrays inside bsc: index k * np + p
enum BScalar { B_RZ = 0, B_PQ, B_RR, B_BB, B_ALPHA, B_BETA, B_TOL2, B_RZPREV, B_NSCALAR };
enum BInt { B_ITER = 0, B_DONE, B_STATUS, B_NINT };

__global__ __launch_bounds__(kBlock) void k_segdot_d(const double *__restrict__ a, const double *__restrict__ b,
                                                     const int64_t *__restrict__ seg, int np, int sub,
                                                     double *partials, const DevState *st, int gated) {
    if (gated && st->done) return;
    const int p = blockIdx.x / sub, sidx = blockIdx.x % sub;
    const int64_t s0 = seg[p], s1 = seg[p + 1];
    double d = 0.0;
    for (int64_t i = s0 + (int64_t)sidx * kBlock + threadIdx.x; i < s1; i += (int64_t)sub * kBlock) d += a[i] * b[i];
    __shared__ double lds[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += lds[w];
        partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_segdot_f(const float *__restrict__ a, const float *__restrict__ b,
                                                     const int64_t *__restrict__ seg, int np, int sub,
                                                     double *partials, const DevState *st, int gated) {
    if (gated && st->done) return;
    const int p = blockIdx.x / sub, sidx = blockIdx.x % sub;
    const int64_t s0 = seg[p], s1 = seg[p + 1];
    double d = 0.0;
    for (int64_t i = s0 + (int64_t)sidx * kBlock + threadIdx.x; i < s1; i += (int64_t)sub * kBlock)
        d += (double)a[i] * (double)b[i];
    __shared__ double lds[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += lds[w];
        partials[blockIdx.x] = t;
    }
}

// Per-problem CG scalar updates from the segmented partials (sub per problem,
// fixed order), then the batch gate.  Two sums per site are kept in
// partials[0..np*sub) and partials[np*sub..2*np*sub) when `two` is set.
__global__ __launch_bounds__(kBlock) void k_bfinalize(const double *__restrict__ partials, int np, int sub, int two,
                                                      double *sc, int32_t *in, DevState *st, int gated, int site) {
    if (gated && st->done) return;
    __shared__ int running;
    if (threadIdx.x == 0) running = 0;
    __syncthreads();
    for (int p = threadIdx.x; p < np; p += kBlock) {
        int32_t *done = in + B_DONE * np, *iter = in + B_ITER * np, *status = in + B_STATUS * np;
        if (gated && done[p]) continue;
        // eight partials of each sum loaded before they are added (same order)
        const double *pa = partials + (int64_t)p * sub;
        const double *pb = partials + (int64_t)np * sub + (int64_t)p * sub;
        double t0 = 0.0, t1 = 0.0;
        int q = 0;
        for (; q + 8 <= sub; q += 8) {
            double u[8], v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                u[e] = pa[q + e];
                v[e] = two ? pb[q + e] : 0.0;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                t0 += u[e];
                if (two) t1 += v[e];
            }
        }
        for (; q < sub; ++q) {
            t0 += pa[q];
            if (two) t1 += pb[q];
        }
        double *rz = sc + B_RZ * np, *pq = sc + B_PQ * np, *rr = sc + B_RR * np, *bb = sc + B_BB * np;
        double *alpha = sc + B_ALPHA * np, *beta = sc + B_BETA * np, *tol2 = sc + B_TOL2 * np;
        switch (site) {
            case SITE_PQ:
                pq[p] = t0;
                if (!(t0 > 0.0)) {
                    status[p] = isfinite(t0) ? ST_BREAKDOWN : ST_NONFINITE;
                    done[p] = 1;
                } else {
                    alpha[p] = rz[p] / t0;
                }
                break;
            case SITE_RR:
                rr[p] = t0;
                iter[p] += 1;
                if (!isfinite(t0)) {
                    status[p] = ST_NONFINITE;
                    done[p] = 1;
                } else if (t0 <= tol2[p]) {
                    status[p] = ST_CONVERGED;
                    done[p] = 1;
                } else if (iter[p] >= st->maxiter) {
                    status[p] = ST_MAXITER;
                    done[p] = 1;
                }
                break;
            case SITE_RZ:
                beta[p] = t0 / rz[p];
                rz[p] = t0;
                break;
            case SITE_RZ0:
                rz[p] = t0;
                break;
            case SITE_INIT:
                bb[p] = t0;
                rr[p] = t1;
                break;
            default:
                break;
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < np; p += kBlock)
        if (!in[B_DONE * np + p]) atomicOr(&running, 1);
    __syncthreads();
    if (threadIdx.x == 0) st->done = running ? 0 : 1;
}

// after the initial residuals: targets per problem, zero right-hand sides and
// problems already at the target are done
__global__ __launch_bounds__(kBlock) void k_barm(int np, double tol, double *sc, int32_t *in, DevState *st,
                                                 int maxiter) {
    __shared__ int running;
    if (threadIdx.x == 0) running = 0;
    __syncthreads();
    for (int p = threadIdx.x; p < np; p += kBlock) {
        const double bb = sc[B_BB * np + p], rr = sc[B_RR * np + p];
        sc[B_TOL2 * np + p] = tol * tol * bb;
        const bool fin = bb == 0.0 || rr <= tol * tol * bb;
        in[B_DONE * np + p] = fin ? 1 : 0;
        in[B_STATUS * np + p] = fin ? ST_CONVERGED : ST_RUNNING;
        in[B_ITER * np + p] = 0;
        if (!fin) atomicOr(&running, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->done = running ? 0 : 1;
        st->maxiter = maxiter;
    }
}

// x += a_p p, r -= a_p q on the rows of unfinished problems; V-cycle copy rv
// of r, and the level-1 pre-smoothing sweep for rows that have a smoother
template <typename TV>
__global__ __launch_bounds__(kBlock) void k_bupdate(int64_t rows, int64_t mrows, const int32_t *__restrict__ rowprob,
                                                    int np, double *__restrict__ x, const double *__restrict__ p,
                                                    double *__restrict__ r, const double *__restrict__ q,
                                                    const TV *__restrict__ M, TV *__restrict__ rv, TV *__restrict__ x1,
                                                    const double *sc, const int32_t *in, const DevState *st) {
    if (st->done) return;
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (row >= rows) return;
    const int pr = rowprob[row];
    TV e[3];
    const bool act = !in[B_DONE * np + pr];
    const double alpha = sc[B_ALPHA * np + pr];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t i = 3 * row + c;
        double ri = r[i];
        if (act) {
            x[i] += alpha * p[i];
            ri -= alpha * q[i];
            r[i] = ri;
        }
        e[c] = (TV)ri;
        rv[i] = e[c];
    }
    if (row < mrows) {
        const TV *m = M + (row / kMSlice) * (9 * kMSlice) + (row % kMSlice);
        x1[3 * row] = m[0] * e[0] + m[kMSlice] * e[1] + m[2 * kMSlice] * e[2];
        x1[3 * row + 1] = m[3 * kMSlice] * e[0] + m[4 * kMSlice] * e[1] + m[5 * kMSlice] * e[2];
        x1[3 * row + 2] = m[6 * kMSlice] * e[0] + m[7 * kMSlice] * e[1] + m[8 * kMSlice] * e[2];
    }
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_bdir(int64_t rows, const int32_t *__restrict__ rowprob, int np,
                                                 const TV *__restrict__ z, double *__restrict__ p, const double *sc,
                                                 const int32_t *in, const DevState *st) {
    if (st->done) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= 3 * rows) return;
    const int pr = rowprob[i / 3];
    if (in[B_DONE * np + pr]) return;
    p[i] = (double)z[i] + sc[B_BETA * np + pr] * p[i];
}

// coarsest solves of several problems: scalar row i of the coarse part
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bgemv(int ncs, int64_t base, const int32_t *__restrict__ cmap,
                                                  const int64_t *__restrict__ c_off, const int32_t *__restrict__ c_n,
                                                  const int64_t *__restrict__ c_a, const int32_t *__restrict__ c_slot,
                                                  const int32_t *__restrict__ done, const double *__restrict__ Ainv,
                                                  const T *__restrict__ f, T *__restrict__ y, const DevState *st,
                                                  int gated) {
    if (gated && st->done) return;
    const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= ncs) return;
    const int e = cmap[i];
    // a finished problem's z is never read again (its direction, scalars and
    // iterate are frozen), so its dense inverse is not streamed either
    if (gated && done[c_slot[e]]) return;
    const int64_t s = c_off[e];
    const int n = c_n[e];
    const int64_t gi = base + i;
    const int64_t li = gi - s;
    const double *a = Ainv + c_a[e] + li * n;
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc += a[j] * (double)f[s + j];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) y[gi] = (T)acc;
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_gather_cast(int64_t n, const double *__restrict__ s,
                                                        TV *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) d[i] = (TV)s[i];
}

constexpr int kSegSub = 16;

static void bseg_dot(amg_batch *B, const double *a, const double *b, int gated, int site) {
    hipLaunchKernelGGL(k_segdot_d, dim3(B->np * kSegSub), dim3(kBlock), 0, B->stream, a, b, B->seg, B->np, kSegSub,
                       B->partials, B->st, gated);
    hipLaunchKernelGGL(k_bfinalize, dim3(1), dim3(kBlock), 0, B->stream, B->partials, B->np, kSegSub, 0, B->bsc,
                       B->bint, B->st, gated, site);
}
static void bseg_dot(amg_batch *B, const float *a, const float *b, int gated, int site) {
    hipLaunchKernelGGL(k_segdot_f, dim3(B->np * kSegSub), dim3(kBlock), 0, B->stream, a, b, B->seg, B->np, kSegSub,
                       B->partials, B->st, gated);
    hipLaunchKernelGGL(k_bfinalize, dim3(1), dim3(kBlock), 0, B->stream, B->partials, B->np, kSegSub, 0, B->bsc,
                       B->bint, B->st, gated, site);
}

// z = V(f) over all problems (rows of level-l vectors: smoothing part first)
template <typename V, typename T>
static void bvcycle(amg_batch *B, BatchDev<V, T> &d, const T *f0, T *z, bool pre_done, int gated) {
    hipStream_t s = B->stream;
    auto &vc = d.vc;
    const int L = (int)vc.lv.size();
    std::vector<T *> out(L);
    for (int l = 0; l < L; ++l) {
        auto &v = vc.lv[l];
        auto &bl = d.bl[l];
        const T *f = l == 0 ? f0 : v.f;
        T *o = l == 0 ? z : v.y;
        out[l] = o;
        if (bl.m > 0 && l + 1 < L && l > 0 && v.has_am && v.has_g) {
            // fused sweeps: t = f - AM f kept in the output rows of the
            // continuing problems (the post-sweep overwrites it in place; the
            // problems that end here own the rows after bl.m)
            launch_sell<V, T>(v.AM.v, v.AM.C, MODE_RESID, f, f, o, nullptr, B->partials, B->st, gated, SITE_NONE, s);
            launch_sell<V, T>(v.R.v, v.R.C, MODE_SPMV, o, nullptr, vc.lv[l + 1].f, nullptr, B->partials, B->st,
                              gated, SITE_NONE, s);
        } else if (bl.m > 0 && l + 1 < L) {
            // with G on the first level the residual goes to the output rows
            // of the continuing problems as well
            T *t = (l == 0 && v.has_g) ? o : v.t;
            if (!(l == 0 && pre_done)) launch_jacobi0<T>(bl.m, v.M, f, v.x, B->st, gated, s);
            launch_sell<V, T>(v.A.v, v.A.C, MODE_RESID, v.x, f, t, nullptr, B->partials, B->st, gated, SITE_NONE, s);
            launch_sell<V, T>(v.R.v, v.R.C, MODE_SPMV, t, nullptr, vc.lv[l + 1].f, nullptr, B->partials, B->st,
                              gated, SITE_NONE, s);
        }
        if (bl.ncs > 0) {
            const int waves = kBlock / 64;
            hipLaunchKernelGGL(k_bgemv<T>, dim3((bl.ncs + waves - 1) / waves), dim3(kBlock), 0, s, bl.ncs,
                               (int64_t)3 * bl.m, bl.cmap, bl.c_off, bl.c_n, bl.c_a, bl.c_slot,
                               B->bint + B_DONE * B->np, B->Ainv, f, o, B->st, gated);
        }
    }
    for (int l = L - 2; l >= 0; --l) {
        auto &v = vc.lv[l];
        auto &bl = d.bl[l];
        if (bl.m == 0) continue;
        const T *f = l == 0 ? f0 : v.f;
        if ((l > 0 && v.has_am && v.has_g) || (l == 0 && v.has_g)) {
            launch_sell<V, T>(v.G.v, v.G.C, MODE_POST, out[l + 1], f, out[l], v.M, B->partials, B->st, gated,
                              SITE_NONE, s);
            continue;
        }
        launch_sell<V, T>(v.P.v, v.P.C, MODE_ADD, out[l + 1], nullptr, v.x, nullptr, B->partials, B->st, gated,
                          SITE_NONE, s);
        launch_sell<V, T>(v.A.v, v.A.C, MODE_SMOOTH, v.x, f, out[l], v.Mt, B->partials, B->st, gated, SITE_NONE, s);
    }
}

template <typename V, typename T>
static void biteration(amg_batch *B, BatchDev<V, T> &d) {
    hipStream_t s = B->stream;
    launch_sell<double, double>(B->A64.v, B->A64.C, MODE_SPMV, B->P, nullptr, B->Q, nullptr, B->partials, B->st, 1,
                                SITE_NONE, s);
    bseg_dot(B, B->P, B->Q, 1, SITE_PQ);
    const int m0 = d.bl[0].m;
    hipLaunchKernelGGL(k_bupdate<T>, dim3((B->nb + kBlock - 1) / kBlock), dim3(kBlock), 0, s, (int64_t)B->nb,
                       (int64_t)m0, B->rowprob, B->np, B->X, B->P, B->R, B->Q, d.vc.lv[0].M, (T *)B->rv,
                       d.vc.lv[0].x, B->bsc, B->bint, B->st);
    bseg_dot(B, B->R, B->R, 1, SITE_RR);
    bvcycle<V, T>(B, d, (const T *)B->rv, (T *)B->zv, true, 1);
    bseg_dot(B, (const T *)B->rv, (const T *)B->zv, 1, SITE_RZ);
    hipLaunchKernelGGL(k_bdir<T>, dim3((3 * (int64_t)B->nb + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       (int64_t)B->nb, B->rowprob, B->np, (const T *)B->zv, B->P, B->bsc, B->bint, B->st);
}

static void bform_iteration(amg_batch *B) {
    if (B->precision == AMG_FP64)
        biteration<double, double>(B, B->d64);
    else
        biteration<float, float>(B, B->d32);
}

template <typename V, typename T>
static void bstart(amg_batch *B, BatchDev<V, T> &d) {
    hipStream_t s = B->stream;
    hipLaunchKernelGGL(k_gather_cast<T>, dim3((B->n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, B->n, B->R,
                       (T *)B->rv);
    bvcycle<V, T>(B, d, (const T *)B->rv, (T *)B->zv, false, 0);
    bseg_dot(B, (const T *)B->rv, (const T *)B->zv, 0, SITE_RZ0);
    launch_copy<T, double>(B->n, (const T *)B->zv, B->P, s);
}

static void concat_level(const std::vector<const Bsr3 *> &mats, const std::vector<int64_t> &row_off,
                         const std::vector<int64_t> &col_off, int64_t rows, int64_t cols, Bsr3 &out) {
    out.rows = (int32_t)rows;
    out.cols = (int32_t)cols;
    out.ptr.assign((size_t)rows + 1, 0);
    int64_t nnz = 0;
    for (auto *m : mats) nnz += m->nnzb();
    out.col.resize(nnz);
    out.val.resize(9 * (size_t)nnz);
    // rows are filled problem by problem; problems occupy disjoint row ranges
    std::vector<int64_t> cnt((size_t)rows, 0);
    for (size_t q = 0; q < mats.size(); ++q)
        for (int32_t i = 0; i < mats[q]->rows; ++i) cnt[row_off[q] + i] = mats[q]->ptr[i + 1] - mats[q]->ptr[i];
    for (int64_t i = 0; i < rows; ++i) out.ptr[i + 1] = out.ptr[i] + cnt[i];
    const int T = std::max(1, std::min<int>((int)mats.size(), setup_threads()));
    parallel_tasks(T, [&](int t) {
        for (size_t q = t; q < mats.size(); q += T) {
            const Bsr3 &m = *mats[q];
            for (int32_t i = 0; i < m.rows; ++i) {
                int64_t d = out.ptr[row_off[q] + i];
                for (int64_t k = m.ptr[i]; k < m.ptr[i + 1]; ++k, ++d) {
                    out.col[d] = (int32_t)(m.col[k] + col_off[q]);
                    std::memcpy(&out.val[9 * d], &m.val[9 * k], 9 * sizeof(double));
                }
            }
        }
    });
}

template <typename V, typename T>
static void upload_batch(amg_batch *B, const std::vector<Hierarchy> &H, BatchDev<V, T> &d,
                         Staging &staging, std::vector<double> &ainv_pool,
                         const std::vector<std::vector<int64_t>> &off, const std::vector<std::vector<int>> &order,
                         const std::vector<int> &msplit) {
    hipStream_t s = B->stream;
    const bool tune = B->prm.autotune != 0;
    const int L = (int)order.size();
    auto &vc = d.vc;
    vc.lv.resize(L);
    vc.npre = 1;
    vc.npost = 1;
    d.bl.resize(L);
    for (int l = 0; l < L; ++l) {
        auto &v = vc.lv[l];
        auto &bl = d.bl[l];
        const std::vector<int> &ord = order[l];
        int64_t rows = 0;
        for (int p : ord) rows += H[p].levels[l].A.rows;
        bl.rows = (int32_t)rows;
        bl.m = msplit[l];
        v.rows = bl.m;
        const size_t vlen = 3 * (size_t)rows;
        v.f = B->al.get<T>(vlen);
        v.x = B->al.get<T>(vlen);
        v.t = B->al.get<T>(vlen);
        v.y = B->al.get<T>(vlen);
        // smoothing part
        std::vector<const Bsr3 *> As, Ps, Rs, AMs, Gs;
        std::vector<int64_t> ro, co_next, co_here;
        std::vector<double> Mall, Mtall;
        bool post_differs = false;
        // fused sweeps when every continuing problem has G here (and AM below
        // the first level); the batch keeps one block array per level, so
        // only symmetric smoother blocks
        bool fuse_g = true, fuse_am = l > 0;
        for (int p : ord) {
            if ((int)H[p].levels.size() <= l + 1) continue;
            As.push_back(&H[p].levels[l].A);
            Ps.push_back(&H[p].levels[l].P);
            AMs.push_back(&H[p].levels[l].AM);
            Gs.push_back(&H[p].levels[l].G);
            fuse_g = fuse_g && !H[p].levels[l].G.ptr.empty() && H[p].levels[l].Mpost.empty();
            fuse_am = fuse_am && !H[p].levels[l].AM.ptr.empty();
            ro.push_back(off[l][p]);
            co_next.push_back(off[l + 1][p]);
            const HostLevel &hl = H[p].levels[l];
            Mall.insert(Mall.end(), hl.Minv.begin(), hl.Minv.end());
            const std::vector<double> &mt = hl.Mpost.empty() ? hl.Minv : hl.Mpost;
            Mtall.insert(Mtall.end(), mt.begin(), mt.end());
            post_differs = post_differs || !hl.Mpost.empty();
        }
        if (bl.m > 0) {
            Bsr3 A, P, R;
            concat_level(As, ro, ro, bl.m, bl.m, A);
            const int64_t next_rows = [&] {
                int64_t r = 0;
                for (int p : order[l + 1]) r += H[p].levels[l + 1].A.rows;
                return r;
            }();
            concat_level(Ps, ro, co_next, bl.m, next_rows, P);
            R = bsr_transpose(P, setup_threads());
            v.A = tuned_sell<V>(A, tune, B->al, s, staging, B->partials, B->st);
            v.P = tuned_sell<V>(P, tune, B->al, s, staging, B->partials, B->st);
            v.R = tuned_sell<V>(R, tune, B->al, s, staging, B->partials, B->st);
            v.M = upload_m<T>(Mall, bl.m, B->al, s, staging);
            v.Mt = post_differs ? upload_m<T>(Mtall, bl.m, B->al, s, staging) : v.M;
            if (fuse_g && (l == 0 || fuse_am)) {
                Bsr3 G;
                concat_level(Gs, ro, co_next, bl.m, next_rows, G);
                v.G = tuned_sell<V>(G, tune, B->al, s, staging, B->partials, B->st, v.M);
                v.has_g = true;
                if (l > 0) {
                    Bsr3 AM;
                    concat_level(AMs, ro, ro, bl.m, bl.m, AM);
                    v.AM = tuned_sell<V>(AM, tune, B->al, s, staging, B->partials, B->st);
                    v.has_am = true;
                }
            }
        }
        // coarsest part
        std::vector<int32_t> cmap;
        std::vector<int64_t> c_off, c_a;
        std::vector<int32_t> c_n, c_slot;
        for (int p : ord) {
            if ((int)H[p].levels.size() != l + 1) continue;
            const int e = (int)c_off.size();
            c_off.push_back(3 * off[l][p]);
            c_n.push_back(H[p].n_coarse);
            c_slot.push_back(B->slot_of[p]);
            c_a.push_back((int64_t)ainv_pool.size());
            ainv_pool.insert(ainv_pool.end(), H[p].coarse_inv.begin(), H[p].coarse_inv.end());
            for (int i = 0; i < H[p].n_coarse; ++i) cmap.push_back(e);
        }
        bl.ncs = (int32_t)cmap.size();
        if (bl.ncs > 0) {
            auto put = [&](auto &vec, auto *&dst) {
                using E = typename std::remove_reference<decltype(vec)>::type::value_type;
                dst = B->al.get<E>(vec.size());
                staging.emplace_back((const char *)vec.data(), (const char *)(vec.data() + vec.size()));
                HIP_CHECK(hipMemcpyAsync(dst, staging.back().data(), vec.size() * sizeof(E), hipMemcpyHostToDevice, s));
            };
            put(cmap, bl.cmap);
            put(c_off, bl.c_off);
            put(c_n, bl.c_n);
            put(c_a, bl.c_a);
            put(c_slot, bl.c_slot);
        }
    }
}

static void build_batch(amg_batch *B, const std::vector<Hierarchy> &H) {
    hipStream_t s = B->stream;
    const int np = B->np;
    int L = 0;
    for (auto &h : H) L = std::max<int>(L, (int)h.levels.size());
    // per level: problems still active, coarsening ones first
    std::vector<std::vector<int>> order(L);
    std::vector<std::vector<int64_t>> off(L, std::vector<int64_t>(np, -1));
    std::vector<int> msplit(L, 0);
    for (int l = 0; l < L; ++l) {
        int64_t o = 0;
        for (int p = 0; p < np; ++p)
            if ((int)H[p].levels.size() > l + 1) order[l].push_back(p);
        for (int p : order[l]) {
            off[l][p] = o;
            o += H[p].levels[l].A.rows;
        }
        msplit[l] = (int)o;
        for (int p = 0; p < np; ++p)
            if ((int)H[p].levels.size() == l + 1) {
                order[l].push_back(p);
                off[l][p] = o;
                o += H[p].levels[l].A.rows;
            }
    }
    Staging staging;
    int max_rows = 1;
    for (int l = 0; l < L; ++l) {
        int64_t r = 0;
        for (int p : order[l]) r += H[p].levels[l].A.rows;
        max_rows = std::max<int64_t>(max_rows, r);
    }
    const int grid_max = std::max(max_rows, np * kSegSub);  // up to a workgroup per row
    B->partials = B->al.get<double>(2 * (size_t)grid_max);
    B->st = B->al.get<DevState>(1);
    launch_state_init(B->st, 0.0, B->prm.maxiter, 0, s);
    // level-0 layout of the user's problems
    B->off0.assign(np, 0);
    B->n0.assign(np, 0);
    B->slot_of.assign(np, 0);
    std::vector<int64_t> seg(np + 1, 0);
    std::vector<int32_t> rowprob;
    for (size_t q = 0; q < order[0].size(); ++q) {
        const int p = order[0][q];
        B->slot_of[p] = (int)q;
        B->off0[p] = 3 * off[0][p];
        B->n0[p] = 3 * (int64_t)H[p].levels[0].A.rows;
        seg[q + 1] = seg[q] + B->n0[p];
        for (int32_t i = 0; i < H[p].levels[0].A.rows; ++i) rowprob.push_back((int32_t)q);
    }
    B->n = seg[np];
    B->nb = (int32_t)(B->n / 3);
    // FP64 finest operator of all problems (level-0 order)
    {
        std::vector<const Bsr3 *> As;
        std::vector<int64_t> ro;
        for (int p : order[0]) {
            As.push_back(&H[p].levels[0].A);
            ro.push_back(off[0][p]);
        }
        Bsr3 A;
        concat_level(As, ro, ro, B->nb, B->nb, A);
        B->A64 = tuned_sell<double>(A, B->prm.autotune != 0, B->al, s, staging, B->partials, B->st);
    }
    std::vector<double> pool;
    if (B->precision == AMG_FP64)
        upload_batch<double, double>(B, H, B->d64, staging, pool, off, order, msplit);
    else
        upload_batch<float, float>(B, H, B->d32, staging, pool, off, order, msplit);
    B->Ainv = B->al.get<double>(pool.size());
    HIP_CHECK(hipMemcpyAsync(B->Ainv, pool.data(), pool.size() * 8, hipMemcpyHostToDevice, s));
    B->d64.vc.Ainv = B->Ainv;
    B->d32.vc.Ainv = B->Ainv;
    B->seg = B->al.get<int64_t>(seg.size());
    HIP_CHECK(hipMemcpyAsync(B->seg, seg.data(), seg.size() * 8, hipMemcpyHostToDevice, s));
    B->rowprob = B->al.get<int32_t>(rowprob.size());
    HIP_CHECK(hipMemcpyAsync(B->rowprob, rowprob.data(), rowprob.size() * 4, hipMemcpyHostToDevice, s));
    B->X = B->al.get<double>(B->n);
    B->R = B->al.get<double>(B->n);
    B->P = B->al.get<double>(B->n);
    B->Q = B->al.get<double>(B->n);
    if (B->precision == AMG_FP64) {
        B->rv = B->al.get<double>(B->n);
        B->zv = B->al.get<double>(B->n);
    } else {
        B->rv = B->al.get<float>(B->n);
        B->zv = B->al.get<float>(B->n);
    }
    B->bsc = B->al.get<double>((size_t)B_NSCALAR * np);
    B->bint = B->al.get<int32_t>((size_t)B_NINT * np);
    HIP_CHECK(hipHostMalloc((void **)&B->hsc, sizeof(double) * B_NSCALAR * np, hipHostMallocDefault));
    HIP_CHECK(hipHostMalloc((void **)&B->hint, sizeof(int32_t) * B_NINT * np, hipHostMallocDefault));
    HIP_CHECK(hipHostMalloc((void **)&B->hst, sizeof(DevState), hipHostMallocDefault));
    HIP_CHECK(hipHostMalloc((void **)&B->hptr, sizeof(double *) * 2 * np, hipHostMallocDefault));
    B->dptr = B->al.get<const double *>(2 * (size_t)np);
    HIP_CHECK(hipEventCreate(&B->ev0));
    HIP_CHECK(hipEventCreate(&B->ev1));
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
}

// Between the caller's per-problem vectors and the concatenated level-0
// vector (slot order): entry i belongs to the slot q with seg[q] <= i <
// seg[q+1] (binary search over the np+1 offsets), whose vector is ptr[q].
__global__ __launch_bounds__(kBlock) void k_bgather(int64_t n, int np, const int64_t *__restrict__ seg,
                                                    const double *const *__restrict__ ptr, double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = np;  // seg[lo] <= i < seg[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= i) lo = mid; else hi = mid;
    }
    dst[i] = ptr[lo][i - seg[lo]];
}
__global__ __launch_bounds__(kBlock) void k_bscatter(int64_t n, int np, const int64_t *__restrict__ seg,
                                                     double *const *__restrict__ ptr, const double *__restrict__ src) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = np;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= i) lo = mid; else hi = mid;
    }
    ptr[lo][i - seg[lo]] = src[i];
}

// The caller's b and x pointers in slot order, copied to the device once per solve.
static void bpointers(amg_batch *B, const double *const *b, double *const *x) {
    for (int p = 0; p < B->np; ++p) {
        if (!b[p] || !x[p]) throw AmgError{AMG_ERR_ARG, "null vector in the batch"};
        B->hptr[B->slot_of[p]] = b[p];
        B->hptr[B->np + B->slot_of[p]] = x[p];
    }
    HIP_CHECK(hipMemcpyAsync(B->dptr, B->hptr, sizeof(double *) * 2 * B->np, hipMemcpyHostToDevice, B->stream));
}
static void bgather(amg_batch *B, int which, double *dst) {
    hipLaunchKernelGGL(k_bgather, dim3((unsigned)((B->n + kBlock - 1) / kBlock)), dim3(kBlock), 0, B->stream, B->n,
                       B->np, B->seg, B->dptr + (size_t)which * B->np, dst);
}
static void bscatter_x(amg_batch *B) {
    hipLaunchKernelGGL(k_bscatter, dim3((unsigned)((B->n + kBlock - 1) / kBlock)), dim3(kBlock), 0, B->stream, B->n,
                       B->np, B->seg, const_cast<double *const *>(B->dptr + B->np), B->X);
}

static void bread(amg_batch *B) {
    HIP_CHECK(hipMemcpyAsync(B->hst, B->st, sizeof(DevState), hipMemcpyDeviceToHost, B->stream));
    HIP_CHECK(hipMemcpyAsync(B->hsc, B->bsc, sizeof(double) * B_NSCALAR * B->np, hipMemcpyDeviceToHost, B->stream));
    HIP_CHECK(hipMemcpyAsync(B->hint, B->bint, sizeof(int32_t) * B_NINT * B->np, hipMemcpyDeviceToHost, B->stream));
    HIP_CHECK(hipStreamSynchronize(B->stream));
}

// FP64 residual of every problem into R, (bb, rr) per problem
static void btrue_residual(amg_batch *B) {
    launch_sell<double, double>(B->A64.v, B->A64.C, MODE_RESID, B->X, B->Q, B->R, nullptr, B->partials, B->st, 0,
                                SITE_NONE, B->stream);
    // bb and rr: two segmented dots, both into the INIT slots
    hipLaunchKernelGGL(k_segdot_d, dim3(B->np * kSegSub), dim3(kBlock), 0, B->stream, B->Q, B->Q, B->seg, B->np,
                       kSegSub, B->partials, B->st, 0);
    hipLaunchKernelGGL(k_segdot_d, dim3(B->np * kSegSub), dim3(kBlock), 0, B->stream, B->R, B->R, B->seg, B->np,
                       kSegSub, B->partials + (int64_t)B->np * kSegSub, B->st, 0);
    hipLaunchKernelGGL(k_bfinalize, dim3(1), dim3(kBlock), 0, B->stream, B->partials, B->np, kSegSub, 1, B->bsc,
                       B->bint, B->st, 0, SITE_INIT);
}

static amg_status solve_batch(amg_batch *B, const double *const *b, double *const *x, double tol,
                              amg_solve_info *info) {
    hipStream_t s = B->stream;
    const int np = B->np;
    // gather b (into Q, reused as the right-hand side of the batch) and x
    bpointers(B, b, x);
    bgather(B, 0, B->Q);
    bgather(B, 1, B->X);
    // the right-hand side must survive: keep it in P until the residual is formed
    btrue_residual(B);
    hipLaunchKernelGGL(k_barm, dim3(1), dim3(kBlock), 0, s, np, tol, B->bsc, B->bint, B->st, B->prm.maxiter);
    bread(B);
    for (int p = 0; p < np; ++p)
        if (!std::isfinite(B->hsc[B_BB * np + p]) || !std::isfinite(B->hsc[B_RR * np + p]))
            throw AmgError{AMG_ERR_ARG, "non-finite right-hand side or initial guess in the batch"};
    // keep b: copy Q (the gathered b) aside in the FP64 X slots is not possible; regather at the end
    if (!B->hst->done) {
        if (B->precision == AMG_FP64)
            bstart<double, double>(B, B->d64);
        else
            bstart<float, float>(B, B->d32);
        const int chunk = std::max(1, B->prm.check_every);
        if (B->prm.use_graphs && !B->exec) {
            HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < chunk; ++i) bform_iteration(B);
            HIP_CHECK(hipStreamEndCapture(s, &B->graph));
            HIP_CHECK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
        }
        for (;;) {
            if (B->prm.use_graphs)
                HIP_CHECK(hipGraphLaunch(B->exec, s));
            else
                for (int i = 0; i < chunk; ++i) bform_iteration(B);
            HIP_CHECK(hipGetLastError());
            HIP_CHECK(hipMemcpyAsync(B->hst, B->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            if (B->hst->done) break;
        }
    }
    bread(B);
    std::vector<int32_t> iters(B->hint + B_ITER * np, B->hint + B_ITER * np + np);
    std::vector<int32_t> status(B->hint + B_STATUS * np, B->hint + B_STATUS * np + np);
    // FP64 true residuals: re-gather b into Q
    bgather(B, 0, B->Q);
    btrue_residual(B);
    bread(B);
    bscatter_x(B);
    HIP_CHECK(hipStreamSynchronize(s));
    amg_status res = AMG_OK;
    const double tol2 = tol * tol;
    for (int p = 0; p < np; ++p) {
        const int q = B->slot_of[p];
        const double bb = B->hsc[B_BB * np + q], rr = B->hsc[B_RR * np + q];
        const bool conv = bb == 0.0 || rr <= tol2 * bb;
        if (status[q] == ST_BREAKDOWN || status[q] == ST_NONFINITE) {
            res = AMG_ERR_BREAKDOWN;
            set_error("CG breakdown in problem " + std::to_string(p));
        } else if (!conv && res == AMG_OK) {
            res = AMG_NOT_CONVERGED;
            set_error("problem " + std::to_string(p) + " did not reach the tolerance");
        }
        if (info) {
            info[p] = amg_solve_info{};
            info[p].iters = iters[q];
            info[p].converged = conv ? 1 : 0;
            info[p].rel_true_residual = bb > 0 ? std::sqrt(rr / bb) : 0.0;
        }
    }
    return res;
}

}  // namespace saamg

extern "C" {

amg_status amg_setup_batch(int32_t np, const amg_bsr3 *A, const double *const *coords, const amg_params *prm,
                           void *hip_stream, amg_batch **out) {
    return guarded([&]() -> amg_status {
        if (np < 1 || !A || !coords || !out) throw AmgError{AMG_ERR_ARG, "invalid batch arguments"};
        *out = nullptr;
        std::unique_ptr<amg_batch> B(new amg_batch());
        amg_default_params(&B->prm);
        if (prm) B->prm = *prm;
        B->np = np;
        const SetupThreads threads(B->prm.nthreads);
        if (B->prm.smoother == AMG_SMOOTHER_ILU0 || B->prm.smoother == AMG_SMOOTHER_LEARNED)
            throw AmgError{AMG_ERR_UNSUPPORTED, "batches use block Jacobi or block SPAI-0"};
        B->precision = B->prm.precision == AMG_FP64 ? AMG_FP64 : AMG_FP32;
        // one host thread per problem group; each problem builds single-threaded
        // up to its coarsest matrix, whose dense inverses (cubic in its size,
        // the largest part of a small problem's setup) then run one after
        // another, largest first, each on every thread (the inverse does not
        // depend on the thread count)
        std::vector<Hierarchy> H(np);
        amg_params one = B->prm;
        one.nthreads = 1;
        const int nthr = resolve_threads(B->prm.nthreads);
        const int T = std::max(1, std::min(np, nthr));
        std::vector<std::exception_ptr> errs(T);
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t)
            th.emplace_back([&, t]() {
                try {
                    for (int p = t; p < np; p += T) build_hierarchy(A[p], coords[p], one, H[p], nullptr, false);
                } catch (...) {
                    errs[t] = std::current_exception();
                }
            });
        for (auto &x : th) x.join();
        for (auto &e : errs)
            if (e) std::rethrow_exception(e);
        std::vector<int> order(np);
        for (int p = 0; p < np; ++p) order[p] = p;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return H[x].n_coarse > H[y].n_coarse; });
        for (int p : order) invert_coarsest(H[p], nthr);
        HIP_CHECK(hipGetDevice(&B->device));
        B->stream = (hipStream_t)hip_stream;
        if (!B->stream) {
            HIP_CHECK(hipStreamCreate(&B->own_stream));
            B->stream = B->own_stream;
        }
        build_batch(B.get(), H);
        *out = B.release();
        return AMG_OK;
    });
}

amg_status amg_solve_batch(amg_batch *B, const double *const *b, double *const *x, double tol,
                           amg_solve_info *info) {
    return guarded([&]() -> amg_status {
        if (!B || !b || !x) throw AmgError{AMG_ERR_ARG, "null argument"};
        if (!(tol > 0.0) || !std::isfinite(tol)) throw AmgError{AMG_ERR_ARG, "tol must be positive"};
        if (B->own_stream) HIP_CHECK(hipStreamSynchronize(nullptr));
        HIP_CHECK(hipEventRecord(B->ev0, B->stream));
        amg_status st = solve_batch(B, b, x, tol, info);
        HIP_CHECK(hipEventRecord(B->ev1, B->stream));
        HIP_CHECK(hipEventSynchronize(B->ev1));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, B->ev0, B->ev1));
        if (info)
            for (int p = 0; p < B->np; ++p) info[p].solve_ms = ms;
        return st;
    });
}

// z[p] = V_p(r[p]) for every problem of the batch in one batched V-cycle (the
// sequence of every iteration of amg_solve_batch).
amg_status amg_vcycle_batch(amg_batch *B, const double *const *r, double *const *z) {
    return guarded([&]() -> amg_status {
        if (!B || !r || !z) throw AmgError{AMG_ERR_ARG, "null argument"};
        for (int p = 0; p < B->np; ++p)
            if (!r[p] || !z[p] || r[p] == z[p]) throw AmgError{AMG_ERR_ARG, "invalid vector in the batch"};
        if (B->own_stream) HIP_CHECK(hipStreamSynchronize(nullptr));
        hipStream_t s = B->stream;
        for (int p = 0; p < B->np; ++p) launch_copy<double, double>(B->n0[p], r[p], B->Q + B->off0[p], s);
        if (B->precision == AMG_FP64) {
            bvcycle<double, double>(B, B->d64, B->Q, B->P, false, 0);
        } else {
            launch_copy<double, float>(B->n, B->Q, (float *)B->rv, s);
            bvcycle<float, float>(B, B->d32, (const float *)B->rv, (float *)B->zv, false, 0);
            launch_copy<float, double>(B->n, (const float *)B->zv, B->P, s);
        }
        for (int p = 0; p < B->np; ++p) launch_copy<double, double>(B->n0[p], B->P + B->off0[p], z[p], s);
        HIP_CHECK(hipGetLastError());
        if (B->own_stream) HIP_CHECK(hipStreamSynchronize(s));
        return AMG_OK;
    });
}

void amg_batch_destroy(amg_batch *B) { delete B; }

}  // extern "C"

// ---------------------------------------------------------------------------
// learned level-1 smoother blocks: installation and training
// ---------------------------------------------------------------------------

namespace saamg {

static void require_learned(const amg_ctx *ctx) {
    if (!ctx->lr.available)
        throw AmgError{AMG_ERR_UNSUPPORTED,
                       "learned smoother needs smoother = AMG_SMOOTHER_LEARNED at setup and two or more levels"};
}

static void require_training(const amg_ctx *ctx) {
    require_learned(ctx);
    if (ctx->precision != AMG_FP64) throw AmgError{AMG_ERR_UNSUPPORTED, "training needs an FP64 context"};
}

static void alloc_training(amg_ctx *ctx) {
    auto &lr = ctx->lr;
    if (lr.train_ready) return;
    const size_t nb = lr.nb;
    lr.z1 = ctx->al.get<float>(nb * kHid);
    lr.z2 = ctx->al.get<float>(nb * kHid);
    lr.dz1 = ctx->al.get<float>(nb * kHid);
    lr.dz2 = ctx->al.get<float>(nb * kHid);
    lr.t = ctx->al.get<float>(nb * kOut);
    lr.dg = ctx->al.get<float>(nb * kOut);
    lr.U = ctx->al.get<double>(nb * 9);
    const size_t nchunks = std::max<size_t>(1, (nb + kGradChunk - 1) / kGradChunk);
    lr.pgrad = ctx->al.get<double>(nchunks * kParams);
    lr.scal = ctx->al.get<double>(4);
    lr.r = ctx->al.get<double>(ctx->n);
    lr.w = ctx->al.get<double>(ctx->n);
    lr.y = ctx->al.get<double>(ctx->n);
    lr.y2 = ctx->al.get<double>(ctx->n);
    lr.q = ctx->al.get<double>(ctx->n);
    lr.xc = ctx->al.get<double>(3 * (size_t)ctx->v64.lv[1].rows);
    HIP_CHECK(hipHostMalloc((void **)&lr.hscal, 4 * sizeof(double), hipHostMallocDefault));
    lr.train_ready = true;
}

// out = (I - P V_2(R A .)) w on the FP64 hierarchy (out != w)
static void coarse_correct(amg_ctx *ctx, const double *w, double *out) {
    hipStream_t s = ctx->stream;
    auto &vc = ctx->v64;
    auto &l0 = vc.lv[0];
    auto &l1 = vc.lv[1];
    launch_sell<double, double>(l0.A.v, l0.A.C, MODE_SPMV, w, nullptr, l0.t, nullptr, ctx->partials, ctx->st, 0,
                                SITE_NONE, s);
    launch_sell<double, double>(l0.R.v, l0.R.C, MODE_SPMV, l0.t, nullptr, l1.f, nullptr, ctx->partials, ctx->st, 0,
                                SITE_NONE, s);
    vc.run(l1.f, ctx->lr.xc, false, 0, SITE_NONE, ctx->partials, ctx->st, s, 1);
    launch_sell<double, double>(l0.P.v, l0.P.C, MODE_RESID, ctx->lr.xc, w, out, nullptr, ctx->partials, ctx->st, 0,
                                SITE_NONE, s);
}

static void spmv1(amg_ctx *ctx, const double *x, double *y) {
    auto &l0 = ctx->v64.lv[0];
    launch_sell<double, double>(l0.A.v, l0.A.C, MODE_SPMV, x, nullptr, y, nullptr, ctx->partials, ctx->st, 0,
                                SITE_NONE, ctx->stream);
}

}  // namespace saamg

extern "C" {

amg_status amg_smoother_set_weights(amg_ctx *ctx, const void *theta, size_t bytes, int32_t dtype, int32_t check,
                                    int32_t *n_fallback) {
    return guarded([&]() -> amg_status {
        if (!ctx) throw AmgError{AMG_ERR_ARG, "null context"};
        require_learned(ctx);
        if (theta) {
            if (dtype != AMG_FP32 && dtype != AMG_BF16)
                throw AmgError{AMG_ERR_ARG, "weights must be AMG_FP32 or AMG_BF16"};
            const size_t want = (size_t)AMG_MLP_PARAMS * (dtype == AMG_FP32 ? 4 : 2);
            if (bytes != want)
                throw AmgError{AMG_ERR_ARG, "weights need " + std::to_string(want) + " bytes, got " +
                                                std::to_string(bytes)};
        }
        StreamFence fence(ctx);
        int bad = 0;
        if (theta) {
            const float *t32 = static_cast<const float *>(theta);
            if (dtype == AMG_BF16) {
                launch_bf16_widen(kParams, static_cast<const uint16_t *>(theta), ctx->lr.theta32, ctx->stream);
                t32 = ctx->lr.theta32;
            }
            bad = install_learned(ctx, t32, check != 0, nullptr, nullptr, nullptr);
        } else {
            restore_jacobi(ctx);
        }
        HIP_CHECK(hipStreamSynchronize(ctx->stream));
        if (n_fallback) *n_fallback = bad;
        return AMG_OK;
    });
}

amg_status amg_mlp_loss_grad(amg_ctx *ctx, const float *theta, const double *E, int32_t k, float scale,
                             int32_t accumulate, double *loss, float *grad) {
    return guarded([&]() -> amg_status {
        if (!ctx || !theta || !E || !grad || k < 1) throw AmgError{AMG_ERR_ARG, "invalid argument"};
        require_training(ctx);
        StreamFence fence(ctx);
        alloc_training(ctx);
        auto &lr = ctx->lr;
        hipStream_t s = ctx->stream;
        const int64_t n = ctx->n;
        install_learned(ctx, theta, 1, lr.z1, lr.z2, lr.t);
        const double *S = ctx->v64.lv[0].M;
        launch_fill<double>((int64_t)lr.nb * 9, 0.0, lr.U, s);
        launch_fill<double>(4, 0.0, lr.scal, s);
        for (int j = 0; j < k; ++j) {
            const double *e = E + (size_t)j * n;
            spmv1(ctx, e, lr.r);                                                   // r = A e
            launch_dot_out(n, e, lr.r, ctx->partials, ctx->max_grid, lr.scal + 0, s);  // e^T A e
            launch_block_resid(lr.nb, S, e, lr.r, lr.w, s);                        // w = e - S r
            coarse_correct(ctx, lr.w, lr.y);                                       // y = (I - Pi) w
            spmv1(ctx, lr.y, lr.q);
            launch_dot_out(n, lr.y, lr.q, ctx->partials, ctx->max_grid, lr.scal + 1, s);  // y^T A y
            launch_loss_acc(lr.scal, s);
            coarse_correct(ctx, lr.y, lr.y2);                                      // (I - Pi) y
            spmv1(ctx, lr.y2, lr.q);                                               // A (I - Pi) y
            launch_outer_acc(lr.nb, lr.U, lr.q, lr.r, lr.scal + 3, s);             // dl/dS += -2/den q r^T
        }
        launch_block_grad(lr.nb, lr.U, lr.L, lr.t, 1.0 / k, lr.dg, s);
        launch_mlp_backward(lr.nb, theta, lr.z1, lr.z2, lr.dg, lr.dz1, lr.dz2, s);
        launch_param_grad(lr.nb, lr.phi, lr.z1, lr.z2, lr.dg, lr.dz1, lr.dz2, lr.pgrad, grad, scale, accumulate != 0,
                          s);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(lr.hscal, lr.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (loss) *loss = lr.hscal[2] / k;
        return AMG_OK;
    });
}

amg_status amg_mlp_adam(amg_ctx *ctx, float *theta, const float *grad, float *m, float *v, int32_t n,
                        int32_t step, float lr, float beta1, float beta2, float eps) {
    return guarded([&]() -> amg_status {
        if (!ctx || !theta || !grad || !m || !v || n < 1 || step < 1)
            throw AmgError{AMG_ERR_ARG, "invalid argument"};
        StreamFence fence(ctx);
        const float bc1 = (float)(1.0 - std::pow((double)beta1, step));
        const float bc2 = (float)(1.0 - std::pow((double)beta2, step));
        launch_adam(n, theta, grad, m, v, lr, beta1, beta2, eps, bc1, bc2, ctx->stream);
        HIP_CHECK(hipGetLastError());
        return AMG_OK;
    });
}

amg_status amg_training_errors(amg_ctx *ctx, double *E, int32_t k, int32_t cycles) {
    return guarded([&]() -> amg_status {
        if (!ctx || !E || k < 1 || cycles < 0) throw AmgError{AMG_ERR_ARG, "invalid argument"};
        if (ctx->precision != AMG_FP64) throw AmgError{AMG_ERR_UNSUPPORTED, "training errors need an FP64 context"};
        StreamFence fence(ctx);
        ensure_g(ctx);
        hipStream_t s = ctx->stream;
        auto &kk = ctx->k64;
        for (int j = 0; j < k; ++j) {
            double *e = E + (size_t)j * ctx->n;
            for (int c = 0; c < cycles; ++c) {
                launch_sell<double, double>(ctx->A64.v, ctx->A64.C, MODE_SPMV, e, nullptr, kk.r, nullptr,
                                            ctx->partials, ctx->st, 0, SITE_NONE, s);
                precondition<double, double>(ctx, ctx->v64, kk.r, kk.z, false, 0, SITE_NONE);
                launch_sub_from(ctx->n, kk.z, e, s);
            }
        }
        HIP_CHECK(hipGetLastError());
        return AMG_OK;
    });
}

}  // extern "C"
