// Host setup of the smoothed-aggregation hierarchy (Algorithm 1), FP64.
//
// Structure of the paper's "NS Block" solver (Section 3): the matrix stays
// in 3x3 block form; only the construction of the tentative prolongation,
// which needs the near-nullspace, is done in scalar space (per aggregate,
// on the scalar rows of its nodes), and the resulting operator is reblocked.
// Prolongation smoothing, R = P^T, the Galerkin product R A P and the
// smoother are block operations.
//
// Readings where the paper gives no formula (the same rules are written out
// in the test oracle, independently):
//  * node size b = 3 on level 1, m (= near-nullspace columns, 6 or 3) above;
//    a node of size 6 is a pair of consecutive block rows;
//  * strength: s_IJ = Frobenius norm of the node block; J != I strong for I
//    iff s_IJ > 0 and s_IJ^2 >= eps_l^2 s_II s_JJ (1 - 1e-12),
//    eps_l = eps_strong * eps_decay^(l-1);
//  * aggregation: (1) in increasing node order, a non-isolated node whose
//    strong neighbours are all unaggregated seeds an aggregate with its
//    non-isolated strong neighbours; (2) every other non-isolated node joins
//    the aggregate (as of the end of phase 1) of its strongest strong
//    neighbour, ratio s_IJ^2/(s_II s_JJ) with 1e-12 relative slack, ties to
//    the lowest aggregate id; (3) aggregates whose near-nullspace block is
//    rank deficient (fewer rows than columns, or min|R_kk| < 1e-10 max|R_kk|)
//    merge into the neighbouring aggregate with the largest summed s_IJ over
//    strong links (ties to the lowest id), repeated in increasing id until
//    none merges, then survivors are renumbered in order;
//  * tentative P: per aggregate, thin QR with positive diag(R) of the
//    near-nullspace rows ordered by node then component;
//  * P = (I - omega_p D^{-1} A_F) P^, A_F = A with weak node blocks removed
//    and their scalar row sums added to the scalar diagonal, D = diag(A);
//  * smoother: M_I = omega_j M0_I on 3x3 diagonal blocks, with M0_I =
//    inv(A_II) (block Jacobi) or M0_I = A_II inv(sum_J A_IJ A_IJ^T) (block
//    SPAI-0, the block-diagonal minimiser of ||I - M0 A||_F; the post-sweep
//    uses its transpose); omega_j = 4/(3 lambda^) with lambda^ from 30 power
//    steps on M0 A starting at x_i = (-1)^i (or the user's fixed omega_j);
//  * stop when n_l <= coarse_enough, at max_levels, or when coarsening leaves
//    more than 0.9 n_l unknowns; the coarsest matrix is inverted densely.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "setup_internal.hpp"

namespace saamg {

namespace {

constexpr double kTieSlack = 1e-12;
constexpr double kRankTol = 1e-10;

struct Strength {
    int32_t N = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> nbr;     // strong neighbours, increasing
    std::vector<double> ratio;    // s_IJ^2 / (s_II s_JJ)
    std::vector<double> norm;     // s_IJ
    bool strong(int32_t I, int32_t J) const {
        auto b = nbr.begin() + ptr[I], e = nbr.begin() + ptr[I + 1];
        auto it = std::lower_bound(b, e, J);
        return it != e && *it == J;
    }
};

inline double blk_sq(const double *v) {
    double s = 0.0;
    for (int e = 0; e < 9; ++e) s += v[e] * v[e];
    return s;
}

// s_IJ^2 for node blocks made of bpn x bpn 3x3 blocks (bpn = node_size / 3).
Strength strength_graph(const Bsr3 &A, int bpn, double eps, int nthreads) {
    Strength G;
    int32_t N = A.rows / bpn;
    G.N = N;
    std::vector<double> sdiag(N, 0.0);
    parallel_for(N, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t I = b; I < e; ++I) {
            double s = 0.0;
            for (int r = 0; r < bpn; ++r) {
                int64_t i = I * bpn + r;
                for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                    if (A.col[k] / bpn == I) s += blk_sq(&A.val[9 * k]);
            }
            sdiag[I] = std::sqrt(s);
        }
    });
    // per-node lists, built in parallel chunks then concatenated
    int T = std::max(1, std::min(nthreads, N / 256 + 1));
    std::vector<std::vector<int32_t>> pn(T);
    std::vector<std::vector<double>> pr(T), pm(T);
    std::vector<std::vector<int64_t>> pc(T);
    parallel_tasks(T, [&](int t) {
        {
            int64_t I0 = (int64_t)N * t / T, I1 = (int64_t)N * (t + 1) / T;
            std::vector<std::pair<int32_t, double>> acc;
            for (int64_t I = I0; I < I1; ++I) {
                acc.clear();
                for (int r = 0; r < bpn; ++r) {
                    int64_t i = I * bpn + r;
                    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                        int32_t J = A.col[k] / bpn;
                        if (J == I) continue;
                        acc.emplace_back(J, blk_sq(&A.val[9 * k]));
                    }
                }
                std::stable_sort(acc.begin(), acc.end(),
                                 [](const auto &x, const auto &y) { return x.first < y.first; });
                int64_t cnt = 0;
                for (size_t q = 0; q < acc.size();) {
                    int32_t J = acc[q].first;
                    double s2 = 0.0;
                    while (q < acc.size() && acc[q].first == J) s2 += acc[q++].second;
                    double prod = sdiag[I] * sdiag[J];
                    if (s2 > 0.0 && s2 >= eps * eps * prod * (1.0 - kTieSlack)) {
                        pn[t].push_back(J);
                        pr[t].push_back(prod > 0 ? s2 / prod : 0.0);
                        pm[t].push_back(std::sqrt(s2));
                        ++cnt;
                    }
                }
                pc[t].push_back(cnt);
            }
        }
    });
    G.ptr.assign((size_t)N + 1, 0);
    int64_t I = 0;
    for (int t = 0; t < T; ++t)
        for (int64_t c : pc[t]) {
            G.ptr[I + 1] = G.ptr[I] + c;
            ++I;
        }
    for (int t = 0; t < T; ++t) {
        G.nbr.insert(G.nbr.end(), pn[t].begin(), pn[t].end());
        G.ratio.insert(G.ratio.end(), pr[t].begin(), pr[t].end());
        G.norm.insert(G.norm.end(), pm[t].begin(), pm[t].end());
    }
    return G;
}

// Rows of the near-nullspace block of the given nodes (sorted), scalar space.
void local_B(const std::vector<double> &B, int m, int b, const int32_t *nodes, int cnt,
             std::vector<double> &Ba /* column-major (cnt*b) x m */) {
    int rows = cnt * b;
    Ba.assign((size_t)rows * m, 0.0);
    for (int q = 0; q < cnt; ++q)
        for (int c = 0; c < b; ++c) {
            size_t src = ((size_t)nodes[q] * b + c) * m;
            for (int j = 0; j < m; ++j) Ba[(size_t)j * rows + q * b + c] = B[src + j];
        }
}

bool rank_deficient(const std::vector<double> &Ba, int rows, int m) {
    if (rows < m) return true;
    std::vector<double> Q((size_t)rows * m), R((size_t)m * m);
    householder_qr(Ba.data(), rows, m, Q.data(), R.data());
    double mx = 0.0, mn = INFINITY;
    for (int k = 0; k < m; ++k) {
        double d = std::fabs(R[k * m + k]);
        mx = std::max(mx, d);
        mn = std::min(mn, d);
    }
    return !(mx > 0.0 && mn >= kRankTol * mx);
}

// Phases 1-3 of the aggregation rule.
int32_t aggregate(const Strength &G, const std::vector<double> &B, int m, int b,
                  std::vector<int32_t> &agg, int nthreads) {
    const int32_t N = G.N;
    agg.assign(N, -1);
    std::vector<uint8_t> isolated(N);
    for (int32_t I = 0; I < N; ++I) isolated[I] = G.ptr[I + 1] == G.ptr[I];
    int32_t n_agg = 0;
    for (int32_t I = 0; I < N; ++I) {
        if (isolated[I] || agg[I] >= 0) continue;
        bool free_nb = true;
        for (int64_t k = G.ptr[I]; k < G.ptr[I + 1]; ++k)
            if (agg[G.nbr[k]] >= 0) {
                free_nb = false;
                break;
            }
        if (!free_nb) continue;
        agg[I] = n_agg;
        for (int64_t k = G.ptr[I]; k < G.ptr[I + 1]; ++k)
            if (!isolated[G.nbr[k]]) agg[G.nbr[k]] = n_agg;
        ++n_agg;
    }
    std::vector<int32_t> snap(agg);
    for (int32_t I = 0; I < N; ++I) {
        if (isolated[I] || snap[I] >= 0) continue;
        double rmax = -1.0;
        for (int64_t k = G.ptr[I]; k < G.ptr[I + 1]; ++k)
            if (snap[G.nbr[k]] >= 0) rmax = std::max(rmax, G.ratio[k]);
        if (rmax < 0.0) continue;
        int32_t best = -1;
        for (int64_t k = G.ptr[I]; k < G.ptr[I + 1]; ++k) {
            int32_t a = snap[G.nbr[k]];
            if (a >= 0 && G.ratio[k] >= rmax * (1.0 - kTieSlack) && (best < 0 || a < best))
                best = a;
        }
        agg[I] = best;
    }
    // phase 3: merge rank-deficient aggregates
    std::vector<std::vector<int32_t>> members(n_agg);
    for (int32_t I = 0; I < N; ++I)
        if (agg[I] >= 0) members[agg[I]].push_back(I);
    std::vector<uint8_t> alive(n_agg, 1);
    // the rank test of every aggregate's members as formed above, in parallel
    // (members are in increasing order); the sequential passes below test an
    // aggregate again only after it has grown by a merge, so the outcome is
    // that of testing every aggregate on every pass
    std::vector<uint8_t> deficient(n_agg, 0), grown(n_agg, 0);
    parallel_for(n_agg, nthreads, [&](int64_t lo, int64_t hi) {
        std::vector<double> Bt;
        for (int64_t a = lo; a < hi; ++a) {
            local_B(B, m, b, members[a].data(), (int)members[a].size(), Bt);
            deficient[a] = rank_deficient(Bt, (int)members[a].size() * b, m);
        }
    });
    std::vector<double> Ba;
    bool changed = true;
    while (changed) {
        changed = false;
        for (int32_t a = 0; a < n_agg; ++a) {
            if (!alive[a]) continue;
            auto &mem = members[a];
            if (grown[a]) {
                std::sort(mem.begin(), mem.end());
                local_B(B, m, b, mem.data(), (int)mem.size(), Ba);
                deficient[a] = rank_deficient(Ba, (int)mem.size() * b, m);
                grown[a] = 0;
            }
            if (!deficient[a]) continue;
            std::vector<std::pair<int32_t, double>> sums;
            for (int32_t I : mem)
                for (int64_t k = G.ptr[I]; k < G.ptr[I + 1]; ++k) {
                    int32_t t = agg[G.nbr[k]];
                    if (t >= 0 && t != a) sums.emplace_back(t, G.norm[k]);
                }
            if (sums.empty()) continue;
            std::sort(sums.begin(), sums.end(),
                      [](const auto &x, const auto &y) { return x.first < y.first; });
            std::vector<std::pair<int32_t, double>> tot;
            for (auto &p : sums) {
                if (!tot.empty() && tot.back().first == p.first)
                    tot.back().second += p.second;
                else
                    tot.push_back(p);
            }
            double smax = 0.0;
            for (auto &p : tot) smax = std::max(smax, p.second);
            int32_t target = -1;
            for (auto &p : tot)
                if (p.second >= smax * (1.0 - kTieSlack)) {
                    target = p.first;
                    break;
                }
            for (int32_t I : mem) agg[I] = target;
            members[target].insert(members[target].end(), mem.begin(), mem.end());
            grown[target] = 1;
            mem.clear();
            alive[a] = 0;
            changed = true;
        }
    }
    std::vector<int32_t> remap(n_agg, -1);
    int32_t cnt = 0;
    for (int32_t a = 0; a < n_agg; ++a)
        if (alive[a]) remap[a] = cnt++;
    for (int32_t I = 0; I < N; ++I)
        if (agg[I] >= 0) agg[I] = remap[agg[I]];
    return cnt;
}

// Tentative prolongation (scalar QR per aggregate) reblocked to BSR3, and
// the next level's near-nullspace B_c (n_agg*m x m, row-major).
void tentative(const std::vector<int32_t> &agg, int32_t n_agg, const std::vector<double> &B,
               int m, int b, int32_t fine_rows, Bsr3 &Pt, std::vector<double> &Bc,
               int nthreads) {
    const int bpn = b / 3;        // block rows per fine node
    const int cpa = m / 3;        // block columns per aggregate
    const int32_t N = (int32_t)agg.size();
    std::vector<std::vector<int32_t>> members(n_agg);
    for (int32_t I = 0; I < N; ++I)
        if (agg[I] >= 0) members[agg[I]].push_back(I);
    // position of each node inside its aggregate
    std::vector<int32_t> pos(N, -1);
    for (int32_t a = 0; a < n_agg; ++a)
        for (size_t q = 0; q < members[a].size(); ++q) pos[members[a][q]] = (int32_t)q;
    Pt.rows = fine_rows;
    Pt.cols = n_agg * cpa;
    Pt.ptr.assign((size_t)fine_rows + 1, 0);
    for (int32_t i = 0; i < fine_rows; ++i) Pt.ptr[i + 1] = Pt.ptr[i] + (agg[i / bpn] >= 0 ? cpa : 0);
    Pt.col.assign(Pt.ptr[fine_rows], 0);
    Pt.val.assign(9 * (size_t)Pt.ptr[fine_rows], 0.0);
    Bc.assign((size_t)n_agg * m * m, 0.0);
    parallel_for(n_agg, nthreads, [&](int64_t ab, int64_t ae) {
        std::vector<double> Ba, Q, R;
        for (int64_t a = ab; a < ae; ++a) {
            const auto &mem = members[a];
            int cnt = (int)mem.size();
            int rows = cnt * b;
            local_B(B, m, b, mem.data(), cnt, Ba);
            Q.assign((size_t)rows * m, 0.0);
            R.assign((size_t)m * m, 0.0);
            householder_qr(Ba.data(), rows, m, Q.data(), R.data());
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) Bc[((size_t)a * m + r) * m + c] = R[r * m + c];
            for (int q = 0; q < cnt; ++q) {
                int32_t I = mem[q];
                for (int s = 0; s < bpn; ++s) {
                    int32_t i = I * bpn + s;
                    for (int cb = 0; cb < cpa; ++cb) {
                        int64_t k = Pt.ptr[i] + cb;
                        Pt.col[k] = (int32_t)(a * cpa + cb);
                        double *blk = &Pt.val[9 * k];
                        for (int r = 0; r < 3; ++r)
                            for (int c = 0; c < 3; ++c)
                                blk[3 * r + c] = Q[(size_t)(cb * 3 + c) * rows + q * b + s * 3 + r];
                    }
                }
            }
        }
    });
    (void)pos;
}

// P = P^ - omega D^{-1} A_F P^ in block arithmetic.
Bsr3 smooth_prolongation(const Bsr3 &A, const Strength &G, int bpn, const Bsr3 &Pt,
                         double omega, int nthreads) {
    const int32_t n = A.rows;
    // filtered A: kept blocks; lumped row sums of weak blocks
    Bsr3 AF;
    AF.rows = A.rows;
    AF.cols = A.cols;
    AF.ptr.assign((size_t)n + 1, 0);
    std::vector<uint8_t> keep(A.col.size());
    std::vector<double> lump((size_t)3 * n, 0.0), dinv((size_t)3 * n, 0.0);
    parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            int32_t I = (int32_t)(i / bpn);
            int64_t cnt = 0;
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                int32_t J = A.col[k] / bpn;
                bool kp = (J == I) || G.strong(I, J);
                keep[k] = kp;
                if (kp) {
                    ++cnt;
                } else {
                    const double *v = &A.val[9 * k];
                    for (int r = 0; r < 3; ++r) lump[3 * i + r] += v[3 * r] + v[3 * r + 1] + v[3 * r + 2];
                }
                if (A.col[k] == i) {
                    const double *v = &A.val[9 * k];
                    for (int r = 0; r < 3; ++r) {
                        double d = v[4 * r];
                        if (!(d > 0.0))
                            throw AmgError{AMG_ERR_NOT_SPD, "non-positive diagonal entry at block row " +
                                                                std::to_string(i)};
                        dinv[3 * i + r] = 1.0 / d;
                    }
                }
            }
            AF.ptr[i + 1] = cnt;
        }
    });
    for (int32_t i = 0; i < n; ++i) AF.ptr[i + 1] += AF.ptr[i];
    AF.col.resize(AF.ptr[n]);
    AF.val.resize(9 * (size_t)AF.ptr[n]);
    parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            int64_t d = AF.ptr[i];
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                if (!keep[k]) continue;
                AF.col[d] = A.col[k];
                std::memcpy(&AF.val[9 * d], &A.val[9 * k], 9 * sizeof(double));
                if (A.col[k] == i)
                    for (int r = 0; r < 3; ++r) AF.val[9 * d + 4 * r] += lump[3 * i + r];
                ++d;
            }
        }
    });
    Bsr3 AP = bsr_multiply(AF, Pt, nthreads);
    // P = Pt - omega D^{-1} AP, union pattern (Pt's pattern is contained in AP's
    // wherever the diagonal block is kept, which it always is)
    Bsr3 P;
    P.rows = Pt.rows;
    P.cols = Pt.cols;
    P.ptr = AP.ptr;
    P.col = AP.col;
    P.val.resize(AP.val.size());
    parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            int64_t kt = Pt.ptr[i];
            for (int64_t k = AP.ptr[i]; k < AP.ptr[i + 1]; ++k) {
                const double *ap = &AP.val[9 * k];
                double *out = &P.val[9 * k];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) out[3 * r + c] = -omega * dinv[3 * i + r] * ap[3 * r + c];
                while (kt < Pt.ptr[i + 1] && Pt.col[kt] < AP.col[k]) ++kt;
                if (kt < Pt.ptr[i + 1] && Pt.col[kt] == AP.col[k]) {
                    const double *pt = &Pt.val[9 * kt];
                    for (int e2 = 0; e2 < 9; ++e2) out[e2] = pt[e2] + out[e2];
                }
            }
            // a tentative block outside AP's pattern would need a union; it
            // cannot happen since A_F keeps every diagonal block
            for (int64_t q = Pt.ptr[i]; q < Pt.ptr[i + 1]; ++q) {
                bool found = std::binary_search(AP.col.begin() + AP.ptr[i], AP.col.begin() + AP.ptr[i + 1],
                                                Pt.col[q]);
                if (!found) throw AmgError{AMG_ERR_ARG, "internal: tentative block outside A_F P^"};
            }
        }
    });
    return P;
}

// ---- the same transfer-operator steps in scalar CSR (hybrid setup) --------

// Strong links between b x b node blocks of the scalar matrix A (the rule of
// strength_graph, the squared Frobenius norms summed entry by entry).
Strength strength_scalar(const Csr &A, int b, double eps, int nthreads) {
    Strength G;
    const int32_t N = A.rows / b;
    G.N = N;
    std::vector<double> sdiag(N, 0.0);
    parallel_for(N, nthreads, [&](int64_t lo, int64_t hi) {
        for (int64_t I = lo; I < hi; ++I) {
            double s = 0.0;
            for (int64_t i = I * b; i < (I + 1) * b; ++i)
                for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                    if (A.col[k] / b == I) s += A.val[k] * A.val[k];
            sdiag[I] = std::sqrt(s);
        }
    });
    std::vector<std::vector<int32_t>> nb(N);
    std::vector<std::vector<double>> rt(N), nm(N);
    parallel_for(N, nthreads, [&](int64_t lo, int64_t hi) {
        std::vector<std::pair<int32_t, double>> acc;
        for (int64_t I = lo; I < hi; ++I) {
            acc.clear();
            for (int64_t i = I * b; i < (I + 1) * b; ++i)
                for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                    const int32_t J = A.col[k] / b;
                    if (J != I) acc.emplace_back(J, A.val[k] * A.val[k]);
                }
            std::stable_sort(acc.begin(), acc.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
            for (size_t q = 0; q < acc.size();) {
                const int32_t J = acc[q].first;
                double s2 = 0.0;
                while (q < acc.size() && acc[q].first == J) s2 += acc[q++].second;
                const double prod = sdiag[I] * sdiag[J];
                if (s2 > 0.0 && s2 >= eps * eps * prod * (1.0 - kTieSlack)) {
                    nb[I].push_back(J);
                    rt[I].push_back(prod > 0 ? s2 / prod : 0.0);
                    nm[I].push_back(std::sqrt(s2));
                }
            }
        }
    });
    G.ptr.assign((size_t)N + 1, 0);
    for (int32_t I = 0; I < N; ++I) {
        G.ptr[I + 1] = G.ptr[I] + (int64_t)nb[I].size();
        G.nbr.insert(G.nbr.end(), nb[I].begin(), nb[I].end());
        G.ratio.insert(G.ratio.end(), rt[I].begin(), rt[I].end());
        G.norm.insert(G.norm.end(), nm[I].begin(), nm[I].end());
    }
    return G;
}

// P = P^ - omega D^{-1} A_F P^ in scalar CSR: A_F keeps the entries of the
// diagonal and strong node blocks, the row sum of every weak entry goes to
// the scalar diagonal, D = diag(A).
Csr smooth_prolongation_scalar(const Csr &A, const Strength &G, int b, const Csr &Pt, double omega,
                               int nthreads) {
    const int32_t n = A.rows;
    Csr AF;
    AF.rows = AF.cols = n;
    AF.ptr.assign((size_t)n + 1, 0);
    std::vector<double> dinv(n, 0.0), lump(n, 0.0);
    std::vector<uint8_t> keep(A.col.size());
    parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            const int32_t I = (int32_t)(i / b);
            int64_t cnt = 0;
            bool diag = false;
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                const int32_t J = A.col[k] / b;
                const bool kp = J == I || G.strong(I, J);
                keep[k] = kp;
                if (kp)
                    ++cnt;
                else
                    lump[i] += A.val[k];
                if (A.col[k] == i) {
                    diag = true;
                    if (!(A.val[k] > 0.0))
                        throw AmgError{AMG_ERR_NOT_SPD, "non-positive diagonal entry at row " + std::to_string(i)};
                    dinv[i] = 1.0 / A.val[k];
                }
            }
            if (!diag) throw AmgError{AMG_ERR_NOT_SPD, "missing diagonal entry at row " + std::to_string(i)};
            AF.ptr[i + 1] = cnt;
        }
    });
    for (int32_t i = 0; i < n; ++i) AF.ptr[i + 1] += AF.ptr[i];
    AF.col.resize(AF.ptr[n]);
    AF.val.resize(AF.ptr[n]);
    parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            int64_t d = AF.ptr[i];
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                if (!keep[k]) continue;
                AF.col[d] = A.col[k];
                AF.val[d] = A.val[k] + (A.col[k] == i ? lump[i] : 0.0);
                ++d;
            }
        }
    });
    Csr AP = csr_multiply(AF, Pt, nthreads);
    // P = Pt - omega D^{-1} AP on the union of the two patterns
    Csr P;
    P.rows = Pt.rows;
    P.cols = Pt.cols;
    P.ptr.assign((size_t)n + 1, 0);
    std::vector<std::vector<int32_t>> pc(n);
    std::vector<std::vector<double>> pv(n);
    parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            int64_t a = AP.ptr[i], t = Pt.ptr[i];
            const int64_t ae = AP.ptr[i + 1], te = Pt.ptr[i + 1];
            while (a < ae || t < te) {
                const int32_t ca = a < ae ? AP.col[a] : INT32_MAX, ct = t < te ? Pt.col[t] : INT32_MAX;
                const int32_t c = std::min(ca, ct);
                double v = 0.0;
                if (ct == c) v += Pt.val[t++];
                if (ca == c) v -= omega * dinv[i] * AP.val[a++];
                pc[i].push_back(c);
                pv[i].push_back(v);
            }
        }
    });
    for (int32_t i = 0; i < n; ++i) {
        P.ptr[i + 1] = P.ptr[i] + (int64_t)pc[i].size();
        P.col.insert(P.col.end(), pc[i].begin(), pc[i].end());
        P.val.insert(P.val.end(), pv[i].begin(), pv[i].end());
    }
    return P;
}

bool inv3(const double *a, double *out) {
    double c00 = a[4] * a[8] - a[5] * a[7];
    double c01 = a[5] * a[6] - a[3] * a[8];
    double c02 = a[3] * a[7] - a[4] * a[6];
    double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    double nrm = 0.0;
    for (int e = 0; e < 9; ++e) nrm = std::max(nrm, std::fabs(a[e]));
    if (!(std::fabs(det) > 1e-14 * nrm * nrm * nrm) || !std::isfinite(det)) return false;
    double id = 1.0 / det;
    out[0] = c00 * id;
    out[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    out[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    out[3] = c01 * id;
    out[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    out[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    out[6] = c02 * id;
    out[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    out[8] = (a[0] * a[4] - a[1] * a[3]) * id;
    return true;
}

// c = a b for row-major 3x3 blocks.
static void mul3(const double *a, const double *b, double *c) {
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
            c[3 * r + q] = a[3 * r] * b[q] + a[3 * r + 1] * b[3 + q] + a[3 * r + 2] * b[6 + q];
}

// Operators of the fused sweeps of a level below the first (one pre- and one
// post-sweep with symmetric blocks M): with x = M f the pre-smoothed iterate
// and t = f - A x = f - (A M) f its residual, the coarse correction e and the
// post-sweep give
//   z = x + P e + M (f - A (x + P e)) = M (f + t) + (P - M A P) e,
// so the level needs AM = A M (same pattern as A) and G = P - M (A P)
// (pattern of P and A P).  With a post-sweep Mt != M (block SPAI-0 applies
// M^T) the same steps give z = M f + Mt t + (P - Mt A P) e.  Mathematically
// the V-cycle is unchanged.  The first level keeps its own pre-sweep (fused
// into the CG update) and residual and takes G only.
static void am_operator(HostLevel &L, int nthreads) {
    const Bsr3 &A = L.A;
    const std::vector<double> &M = L.Minv;
    L.AM.rows = A.rows;
    L.AM.cols = A.cols;
    L.AM.ptr = A.ptr;
    L.AM.col = A.col;
    L.AM.val.resize(A.val.size());  // every block is written below
    parallel_for(A.rows, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i)
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                mul3(&A.val[9 * k], &M[9 * (size_t)A.col[k]], &L.AM.val[9 * k]);
    });
}

// G = (I - Mt A) P with Mt the post-sweep blocks (M itself, or M^T for block
// SPAI-0, where the post-smoothed iterate is z = G e + M f + M^T t).
static void g_operator(HostLevel &L, const Bsr3 &AP, int nthreads) {
    const Bsr3 &P = L.P;
    const std::vector<double> &M = L.Mpost.empty() ? L.Minv : L.Mpost;
    // G row i = P row i - Mt_i (A P) row i, columns merged in increasing order
    Bsr3 &G = L.G;
    G.rows = P.rows;
    G.cols = P.cols;
    G.ptr.assign(P.rows + 1, 0);
    for (int32_t i = 0; i < P.rows; ++i) {
        int64_t a = P.ptr[i], c = AP.ptr[i], n = 0;
        while (a < P.ptr[i + 1] || c < AP.ptr[i + 1]) {
            const int32_t ja = a < P.ptr[i + 1] ? P.col[a] : INT32_MAX;
            const int32_t jc = c < AP.ptr[i + 1] ? AP.col[c] : INT32_MAX;
            if (ja <= jc) ++a;
            if (jc <= ja) ++c;
            ++n;
        }
        G.ptr[i + 1] = G.ptr[i] + n;
    }
    G.col.resize(G.ptr[P.rows]);
    G.val.resize(9 * (size_t)G.ptr[P.rows]);  // every block is written below
    parallel_for(P.rows, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            const double *mi = &M[9 * (size_t)i];
            int64_t a = P.ptr[i], c = AP.ptr[i], o = G.ptr[i];
            while (a < P.ptr[i + 1] || c < AP.ptr[i + 1]) {
                const int32_t ja = a < P.ptr[i + 1] ? P.col[a] : INT32_MAX;
                const int32_t jc = c < AP.ptr[i + 1] ? AP.col[c] : INT32_MAX;
                double *g = &G.val[9 * o];
                G.col[o] = std::min(ja, jc);
                if (ja <= jc) {
                    for (int q = 0; q < 9; ++q) g[q] = P.val[9 * a + q];
                    ++a;
                } else {
                    for (int q = 0; q < 9; ++q) g[q] = 0.0;
                }
                if (jc <= ja) {
                    double t[9];
                    mul3(mi, &AP.val[9 * c], t);
                    for (int q = 0; q < 9; ++q) g[q] -= t[q];
                    ++c;
                }
                ++o;
            }
        }
    });
}

// The two parts of G on its pattern, for a level whose smoother blocks change
// after setup (learned blocks S on level 1): GP holds P's blocks and GAP the
// blocks of A P, so the device can form G = GP - S GAP for any S.
static void g_parts(HostLevel &L, const Bsr3 &AP) {
    const Bsr3 &P = L.P, &G = L.G;
    for (Bsr3 *X : {&L.GP, &L.GAP}) {
        X->rows = G.rows;
        X->cols = G.cols;
        X->ptr = G.ptr;
        X->col = G.col;
        X->val.assign(G.val.size(), 0.0);
    }
    for (int32_t i = 0; i < G.rows; ++i) {
        int64_t a = P.ptr[i], c = AP.ptr[i];
        for (int64_t o = G.ptr[i]; o < G.ptr[i + 1]; ++o) {
            if (a < P.ptr[i + 1] && P.col[a] == G.col[o]) {
                std::memcpy(&L.GP.val[9 * o], &P.val[9 * a], 9 * sizeof(double));
                ++a;
            }
            if (c < AP.ptr[i + 1] && AP.col[c] == G.col[o]) {
                std::memcpy(&L.GAP.val[9 * o], &AP.val[9 * c], 9 * sizeof(double));
                ++c;
            }
        }
    }
}

// Smoother blocks of one level (block Jacobi or block SPAI-0): Minv holds the
// pre-sweep blocks, Mpost the post-sweep blocks when they differ (SPAI-0:
// the transposes; empty otherwise).  Returns omega_j.
double smoother_blocks(const Bsr3 &A, int32_t kind, double omega_user, std::vector<double> &Minv,
                       std::vector<double> &Mpost, int nthreads) {
    const int32_t n = A.rows;
    std::vector<double> Dinv(9 * (size_t)n);  // undamped blocks M0_I
    std::vector<int> bad(1, -1);
    parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            const double *d = nullptr;
            double G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                const double *a = &A.val[9 * k];
                if (A.col[k] == i) d = a;
                if (kind == AMG_SMOOTHER_SPAI0)
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < 3; ++c)
                            G[3 * r + c] += a[3 * r] * a[3 * c] + a[3 * r + 1] * a[3 * c + 1] +
                                            a[3 * r + 2] * a[3 * c + 2];
            }
            if (kind != AMG_SMOOTHER_SPAI0) {
                if (!d || !inv3(d, &Dinv[9 * i])) bad[0] = (int)i;
                continue;
            }
            double Gi[9];
            if (!d || !inv3(G, Gi)) {
                bad[0] = (int)i;
                continue;
            }
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    Dinv[9 * i + 3 * r + c] = d[3 * r] * Gi[c] + d[3 * r + 1] * Gi[3 + c] + d[3 * r + 2] * Gi[6 + c];
        }
    });
    if (bad[0] >= 0)
        throw AmgError{AMG_ERR_SINGULAR_BLOCK,
                       "diagonal block " + std::to_string(bad[0]) + " is singular"};
    double omega = omega_user;
    if (!(omega > 0.0)) {
        // lambda^ of M0 A: 30 power steps from x_i = (-1)^i
        std::vector<double> x(3 * (size_t)n), y(3 * (size_t)n), t(3 * (size_t)n);
        for (size_t i = 0; i < x.size(); ++i) x[i] = (i & 1) ? -1.0 : 1.0;
        double lam = 0.0;
        for (int it = 0; it < 30; ++it) {
            bsr_spmv(A, x.data(), t.data(), nthreads);
            parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
                for (int64_t i = b; i < e; ++i) {
                    const double *d = &Dinv[9 * i];
                    const double *v = &t[3 * i];
                    for (int r = 0; r < 3; ++r)
                        y[3 * i + r] = d[3 * r] * v[0] + d[3 * r + 1] * v[1] + d[3 * r + 2] * v[2];
                }
            });
            // ||y||^2 and ||x||^2 as sums of kNormChunks fixed index ranges added
            // in order (the same result for any thread count)
            constexpr int kNormChunks = 64;
            double py[kNormChunks], px[kNormChunks];
            const int64_t len = (int64_t)y.size();
            parallel_tasks(std::min(kNormChunks, std::max(1, nthreads)), [&](int t) {
                const int T = std::min(kNormChunks, std::max(1, nthreads));
                for (int c = t; c < kNormChunks; c += T) {
                    double sy = 0.0, sx = 0.0;
                    for (int64_t i = len * c / kNormChunks; i < len * (c + 1) / kNormChunks; ++i) {
                        sy += y[i] * y[i];
                        sx += x[i] * x[i];
                    }
                    py[c] = sy;
                    px[c] = sx;
                }
            });
            double ny = 0.0, nx = 0.0;
            for (int c = 0; c < kNormChunks; ++c) {
                ny += py[c];
                nx += px[c];
            }
            ny = std::sqrt(ny);
            nx = std::sqrt(nx);
            lam = ny / nx;
            parallel_for(len, nthreads, [&](int64_t b, int64_t e) {
                for (int64_t i = b; i < e; ++i) x[i] = y[i] / ny;
            });
        }
        omega = 4.0 / (3.0 * lam);
    }
    Minv.resize(Dinv.size());
    parallel_for((int64_t)Dinv.size(), nthreads, [&](int64_t b, int64_t e) {
        for (int64_t q = b; q < e; ++q) Minv[q] = omega * Dinv[q];
    });
    Mpost.clear();
    if (kind == AMG_SMOOTHER_SPAI0) {
        Mpost.resize(Minv.size());
        for (int32_t i = 0; i < n; ++i)
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) Mpost[9 * (size_t)i + 3 * r + c] = Minv[9 * (size_t)i + 3 * c + r];
    }
    return omega;
}

// Block ILU(0) of a level in a greedy multicolour order (the smoother of the
// paper's experiments: Section 3, ILU(0) with 3x3 block values).  Colours:
// in increasing block-row order, the smallest colour not yet taken by a
// block row the row is coupled to (A's block pattern).  The rows are then
// eliminated in the order (colour, row): the incomplete factors keep A's
// pattern, L_IK = A_IK U_KK^{-1} for the coupled K of a lower colour, taken
// in that order, each followed by A_IJ -= L_IK U_KJ for every J after K in
// the order that row K and row I both hold.  Rows of one colour are never
// coupled, so they are eliminated independently (in parallel here), and each
// triangular solve of the smoother is one dependent pass per colour.
static void ilu0_multicolour(HostLevel &L, int nthreads) {
    const Bsr3 &A = L.A;
    const int32_t n = A.rows;
    std::vector<int32_t> colour(n, -1);
    std::vector<int32_t> seen;  // stamp per colour: last row that found it taken
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            const int32_t c = colour[A.col[k]];
            if (c >= 0) seen[c] = i;
        }
        int32_t c = 0;
        while (c < nc && seen[c] == i) ++c;
        if (c == nc) {
            ++nc;
            seen.push_back(-1);
        }
        colour[i] = c;
    }
    // rows grouped by colour, increasing row id inside a colour
    std::vector<int32_t> cptr(nc + 1, 0), order(n);
    for (int32_t i = 0; i < n; ++i) ++cptr[colour[i] + 1];
    for (int32_t c = 0; c < nc; ++c) cptr[c + 1] += cptr[c];
    {
        std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
        for (int32_t i = 0; i < n; ++i) order[fill[colour[i]]++] = i;
    }
    // elimination on a copy of A's values
    std::vector<double> a(A.val.begin(), A.val.end());
    std::vector<int64_t> diag(n, -1);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (A.col[k] == i) diag[i] = k;
    std::vector<double> Uinv(9 * (size_t)n);
    std::vector<int> bad(1, -1);
    auto before = [&](int32_t p, int32_t q) {  // p eliminated before q
        return colour[p] < colour[q] || (colour[p] == colour[q] && p < q);
    };
    for (int32_t c = 0; c < nc; ++c) {
        parallel_for(cptr[c + 1] - cptr[c], nthreads, [&](int64_t b, int64_t e) {
            std::vector<int64_t> low;
            for (int64_t q = cptr[c] + b; q < cptr[c] + e; ++q) {
                const int32_t i = order[q];
                low.clear();
                for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                    if (colour[A.col[k]] < c) low.push_back(k);
                std::sort(low.begin(), low.end(),
                          [&](int64_t p, int64_t r) { return before(A.col[p], A.col[r]); });
                for (int64_t p : low) {
                    const int32_t kk = A.col[p];
                    double lik[9];
                    mul3(&a[9 * p], &Uinv[9 * (size_t)kk], lik);
                    std::memcpy(&a[9 * p], lik, sizeof(lik));
                    // row kk's entries after kk in the order, where row i has them too
                    for (int64_t r = A.ptr[kk]; r < A.ptr[kk + 1]; ++r) {
                        const int32_t j = A.col[r];
                        if (!before(kk, j)) continue;
                        const int32_t *rb = A.col.data() + A.ptr[i], *re = A.col.data() + A.ptr[i + 1];
                        const int32_t *hit = std::lower_bound(rb, re, j);
                        if (hit == re || *hit != j) continue;
                        double prod[9];
                        mul3(lik, &a[9 * r], prod);
                        double *aij = &a[9 * (A.ptr[i] + (hit - rb))];
                        for (int t = 0; t < 9; ++t) aij[t] -= prod[t];
                    }
                }
                if (diag[i] < 0 || !inv3(&a[9 * diag[i]], &Uinv[9 * (size_t)i])) bad[0] = i;
            }
        });
        if (bad[0] >= 0)
            throw AmgError{AMG_ERR_SINGULAR_BLOCK,
                           "ILU(0) pivot block " + std::to_string(bad[0]) + " is singular"};
    }
    // split into L (lower colours), U (higher colours) and the diagonal
    auto split = [&](bool lower, Bsr3 &M) {
        M.rows = M.cols = n;
        M.ptr.assign(n + 1, 0);
        M.col.clear();
        M.val.clear();
        for (int32_t i = 0; i < n; ++i) {
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                const int32_t j = A.col[k];
                if (j == i || (colour[j] < colour[i]) != lower) continue;
                M.col.push_back(j);
                M.val.insert(M.val.end(), &a[9 * k], &a[9 * k] + 9);
            }
            M.ptr[i + 1] = (int64_t)M.col.size();
        }
    };
    split(true, L.ilu_L);
    split(false, L.ilu_U);
    L.ilu_D.resize(9 * (size_t)n);
    for (int32_t i = 0; i < n; ++i) std::memcpy(&L.ilu_D[9 * (size_t)i], &a[9 * diag[i]], 9 * sizeof(double));
    L.ilu_Dinv = std::move(Uinv);
    L.ilu_colour = std::move(colour);
    L.ilu_ncolours = nc;
}

void check_input(const amg_bsr3 &A, const double *coords, int nthreads) {
    if (A.nb <= 0 || A.nnzb <= 0 || !A.row_ptr || !A.col || !A.val)
        throw AmgError{AMG_ERR_ARG, "null or empty matrix"};
    if (!coords) throw AmgError{AMG_ERR_ARG, "coords is null"};
    if (A.row_ptr[0] != 0 || A.row_ptr[A.nb] != A.nnzb)
        throw AmgError{AMG_ERR_ARG, "row_ptr must start at 0 and end at nnzb"};
    // rows in parallel; the first failing row (lowest index) is reported
    enum { OK = 0, NOT_MONOTONE, OUT_OF_RANGE, UNSORTED, NO_DIAGONAL, NON_FINITE };
    std::mutex mu;
    int64_t bad_row = INT64_MAX;
    int bad_kind = OK;
    parallel_for(A.nb, nthreads, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            const int64_t b = A.row_ptr[i], e = A.row_ptr[i + 1];
            int kind = OK;
            if (e < b) {
                kind = NOT_MONOTONE;
            } else {
                bool diag = false;
                for (int64_t k = b; k < e && kind == OK; ++k) {
                    const int32_t c = A.col[k];
                    if (c < 0 || c >= A.nb) kind = OUT_OF_RANGE;
                    else if (k > b && c <= A.col[k - 1]) kind = UNSORTED;
                    diag |= (c == i);
                }
                if (kind == OK && !diag) kind = NO_DIAGONAL;
                for (int64_t q = 9 * b; q < 9 * e && kind == OK; ++q)
                    if (!std::isfinite(A.val[q])) kind = NON_FINITE;
                for (int q = 0; q < 3 && kind == OK; ++q)
                    if (!std::isfinite(coords[3 * i + q])) kind = NON_FINITE + 1;
            }
            if (kind != OK) {
                std::lock_guard<std::mutex> g(mu);
                if (i < bad_row) {
                    bad_row = i;
                    bad_kind = kind;
                }
                return;  // later rows of this range cannot be lower
            }
        }
    });
    if (bad_kind == OK) return;
    const std::string row = std::to_string(bad_row);
    switch (bad_kind) {
        case NOT_MONOTONE: throw AmgError{AMG_ERR_ARG, "row_ptr is not monotone at row " + row};
        case OUT_OF_RANGE: throw AmgError{AMG_ERR_ARG, "column index out of range in row " + row};
        case UNSORTED: throw AmgError{AMG_ERR_ARG, "columns not sorted/unique in row " + row};
        case NO_DIAGONAL: throw AmgError{AMG_ERR_ARG, "missing diagonal block in row " + row};
        case NON_FINITE: throw AmgError{AMG_ERR_ARG, "non-finite matrix value"};
        default: throw AmgError{AMG_ERR_ARG, "non-finite coordinate"};
    }
}

}  // namespace

// Adds the wall time since the previous mark to one setup phase.
struct PhaseClock {
    double *ms;
    std::chrono::steady_clock::time_point last = std::chrono::steady_clock::now();
    void mark(int phase) {
        const auto now = std::chrono::steady_clock::now();
        ms[phase] += std::chrono::duration<double, std::milli>(now - last).count();
        last = now;
    }
};

void invert_coarsest(Hierarchy &H, int nthreads) {
    const auto t0 = std::chrono::steady_clock::now();
    dense_spd_inverse(H.coarse_inv, H.n_coarse, nthreads);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    H.phase_ms[PH_COARSEST] += ms;
    H.setup_ms += ms;
}

void build_hierarchy(const amg_bsr3 &Ain, const double *coords, const amg_params &prm,
                     Hierarchy &H, const GalerkinFn *galerkin, bool invert) {
    auto t0 = std::chrono::steady_clock::now();
    for (double &v : H.phase_ms) v = 0.0;
    PhaseClock clk{H.phase_ms};
    check_input(Ain, coords, resolve_threads(prm.nthreads));
    if (prm.max_levels < 1 || prm.max_levels > AMG_MAX_LEVELS || prm.npre < 1 || prm.npost < 1)
        throw AmgError{AMG_ERR_ARG, "invalid level or sweep parameters"};
    if (prm.smoother != AMG_SMOOTHER_JACOBI && prm.smoother != AMG_SMOOTHER_LEARNED &&
        prm.smoother != AMG_SMOOTHER_SPAI0 && prm.smoother != AMG_SMOOTHER_ILU0)
        throw AmgError{AMG_ERR_ARG, "unknown smoother"};
    if (prm.smoother_levels < 0) throw AmgError{AMG_ERR_ARG, "smoother_levels must be >= 0"};
    if (prm.setup_path != AMG_SETUP_BLOCK && prm.setup_path != AMG_SETUP_SCALAR)
        throw AmgError{AMG_ERR_ARG, "unknown setup path"};
    const int nthreads = resolve_threads(prm.nthreads);
    H.prm = prm;
    H.levels.clear();
    // level 1 operator
    Bsr3 A;
    A.rows = A.cols = Ain.nb;
    A.ptr.assign(Ain.row_ptr, Ain.row_ptr + Ain.nb + 1);
    A.col.assign(Ain.col, Ain.col + Ain.nnzb);
    A.val.resize(9 * (size_t)Ain.nnzb);
    parallel_for(Ain.nb, nthreads, [&](int64_t b, int64_t e) {
        const int64_t k0 = Ain.row_ptr[b], k1 = Ain.row_ptr[e];
        std::memcpy(A.val.data() + 9 * k0, Ain.val + 9 * k0, 9 * (k1 - k0) * sizeof(double));
    });
    // near-nullspace B_1 (n x m, row-major)
    const int32_t nb = Ain.nb;
    int m = prm.use_nullspace ? 6 : 3;
    std::vector<double> B((size_t)3 * nb * m, 0.0);
    if (prm.use_nullspace) {
        double cx = 0, cy = 0, cz = 0;
        for (int32_t i = 0; i < nb; ++i) {
            cx += coords[3 * i];
            cy += coords[3 * i + 1];
            cz += coords[3 * i + 2];
        }
        cx /= nb;
        cy /= nb;
        cz /= nb;
        for (int32_t i = 0; i < nb; ++i) {
            double dx = coords[3 * i] - cx, dy = coords[3 * i + 1] - cy, dz = coords[3 * i + 2] - cz;
            double *bx = &B[(3 * (size_t)i + 0) * m];
            double *by = &B[(3 * (size_t)i + 1) * m];
            double *bz = &B[(3 * (size_t)i + 2) * m];
            bx[0] = 1.0;
            by[1] = 1.0;
            bz[2] = 1.0;
            // rotations about x, y, z: (0,-dz,dy), (dz,0,-dx), (-dy,dx,0)
            by[3] = -dz;
            bz[3] = dy;
            bx[4] = dz;
            bz[4] = -dx;
            bx[5] = -dy;
            by[5] = dx;
        }
    } else {
        for (int32_t i = 0; i < nb; ++i)
            for (int c = 0; c < 3; ++c) B[(3 * (size_t)i + c) * m + c] = 1.0;
    }
    int b = 3;
    const bool scalar = prm.setup_path == AMG_SETUP_SCALAR && !galerkin;
    Csr As_next;  // the next level's matrix in scalar CSR (hybrid setup)
    for (int l = 1;; ++l) {
        H.levels.emplace_back();
        HostLevel &L = H.levels.back();
        L.node_size = b;
        L.eps = prm.eps_strong * std::pow(prm.eps_decay, l - 1);
        L.A = std::move(A);
        const int64_t nl = 3 * (int64_t)L.A.rows;
        if (nl <= prm.coarse_enough || l >= prm.max_levels) break;
        const int bpn = b / 3;
        clk.mark(PH_OTHER);
        // the hybrid setup keeps the level matrix in scalar CSR as well
        Csr As;
        if (scalar) {
            As = l == 1 ? unblock(L.A, nthreads) : std::move(As_next);
            clk.mark(PH_CONVERT);
        }
        Strength G = scalar ? strength_scalar(As, b, L.eps, nthreads) : strength_graph(L.A, bpn, L.eps, nthreads);
        int32_t n_agg = aggregate(G, B, m, b, L.agg, nthreads);
        clk.mark(PH_STRENGTH_AGGREGATE);
        if (n_agg == 0 || (double)m * n_agg > 0.9 * (double)nl) {
            L.agg.clear();
            break;
        }
        L.n_agg = n_agg;
        Bsr3 Pt;
        std::vector<double> Bc;
        tentative(L.agg, n_agg, B, m, b, L.A.rows, Pt, Bc, nthreads);
        clk.mark(PH_TENTATIVE);
        Bsr3 AP;
        if (scalar) {
            // Section 3's hybrid construction: smoothing, transpose and the
            // Galerkin product in scalar CSR, every result converted to 3x3
            // blocks afterwards
            const Csr Pts = unblock(Pt, nthreads);
            clk.mark(PH_CONVERT);
            const Csr Ps = smooth_prolongation_scalar(As, G, b, Pts, prm.omega_p, nthreads);
            clk.mark(PH_SMOOTH_P);
            const Csr Rs = csr_transpose(Ps);
            clk.mark(PH_TRANSPOSE);
            const Csr APs = csr_multiply(As, Ps, nthreads);
            As_next = csr_multiply(Rs, APs, nthreads);
            clk.mark(PH_GALERKIN);
            L.P = reblock(Ps, nthreads);
            L.R = reblock(Rs, nthreads);
            AP = reblock(APs, nthreads);
            A = reblock(As_next, nthreads);
            clk.mark(PH_CONVERT);
        } else {
            L.P = smooth_prolongation(L.A, G, bpn, Pt, prm.omega_p, nthreads);
            clk.mark(PH_SMOOTH_P);
            L.R = bsr_transpose(L.P, nthreads);
            clk.mark(PH_TRANSPOSE);
            if (galerkin) {
                (*galerkin)(L.A, L.P, L.R, AP, A);
            } else {
                AP = bsr_multiply(L.A, L.P, nthreads);
                A = bsr_multiply(L.R, AP, nthreads);
            }
            clk.mark(PH_GALERKIN);
        }
        // block-Jacobi blocks are kept on ILU(0) levels too (export, and the
        // levels below smoother_levels use them)
        L.omega_j = smoother_blocks(L.A, prm.smoother, prm.omega_j, L.Minv, L.Mpost, nthreads);
        clk.mark(PH_SMOOTHER);
        const bool ilu = prm.smoother == AMG_SMOOTHER_ILU0 && (prm.smoother_levels == 0 || l <= prm.smoother_levels);
        if (ilu) ilu0_multicolour(L, nthreads);
        clk.mark(PH_ILU);
        // fused sweeps need one pre- and one post-sweep (and a block-diagonal
        // smoother); level 1 of the learned smoother also keeps G's parts (its
        // blocks change after setup)
        if (prm.npre == 1 && prm.npost == 1 && !ilu) {
            if (l >= 2) am_operator(L, nthreads);
            g_operator(L, AP, nthreads);
            if (l == 1 && prm.smoother == AMG_SMOOTHER_LEARNED) g_parts(L, AP);
        }
        clk.mark(PH_FUSED);
        B.swap(Bc);
        b = m;
    }
    // coarsest: dense inverse
    clk.mark(PH_OTHER);
    HostLevel &C = H.levels.back();
    const int nc = 3 * C.A.rows;
    if (nc > 20000) throw AmgError{AMG_ERR_ARG, "coarsening stalled: coarsest level too large for a dense solve"};
    H.n_coarse = nc;
    H.coarse_inv.assign((size_t)nc * nc, 0.0);
    for (int32_t i = 0; i < C.A.rows; ++i)
        for (int64_t k = C.A.ptr[i]; k < C.A.ptr[i + 1]; ++k) {
            int32_t j = C.A.col[k];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    H.coarse_inv[(size_t)(3 * i + r) * nc + 3 * j + c] = C.A.val[9 * k + 3 * r + c];
        }
    if (invert) dense_spd_inverse(H.coarse_inv, nc, nthreads);
    clk.mark(PH_COARSEST);
    if (prm.smoother == AMG_SMOOTHER_LEARNED && H.levels.size() > 1)
        learned_inputs(H.levels[0].A, coords, H.levels[0].Minv, H.learn_phi, H.learn_L, nthreads);
    clk.mark(PH_OTHER);
    H.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace saamg
