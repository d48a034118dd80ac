// C ABI: parameters, errors and the host-only hierarchy entry points.
#include <cstring>
#include <new>
#include <string>

#include "setup_internal.hpp"

namespace saamg {
static thread_local std::string g_error;
void set_error(const std::string &msg) { g_error = msg; }
const char *get_error() { return g_error.c_str(); }
}  // namespace saamg

extern "C" {

void amg_default_params(amg_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->eps_strong = 0.08;
    p->eps_decay = 0.5;
    p->omega_p = 2.0 / 3.0;
    p->omega_j = 0.0;
    p->npre = 1;
    p->npost = 1;
    p->coarse_enough = 3000;
    p->max_levels = 10;
    p->use_nullspace = 1;
    p->precision = AMG_FP64;
    p->krylov = AMG_KRYLOV_CG;
    p->maxiter = 1000;
    p->check_every = 8;
    p->max_restarts = 2;
    p->use_graphs = 1;
    p->nthreads = 0;
    p->autotune = 1;
    p->smoother_levels = 1;
    p->setup_path = AMG_SETUP_BLOCK;
    p->setup_device = 0;
}

const char *amg_last_error(void) { return saamg::get_error(); }

amg_status amg_hierarchy_build(const amg_bsr3 *A, const double *coords, const amg_params *prm,
                               amg_hierarchy **out) {
    saamg::set_error("");
    if (!A || !out) {
        saamg::set_error("null argument");
        return AMG_ERR_ARG;
    }
    *out = nullptr;
    amg_params def;
    amg_default_params(&def);
    const amg_params &p = prm ? *prm : def;
    try {
        auto *h = new amg_hierarchy();
        try {
            saamg::build_hierarchy(*A, coords, p, h->H);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
        return AMG_OK;
    } catch (const saamg::AmgError &e) {
        saamg::set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        saamg::set_error("host allocation failed during setup");
        return AMG_ERR_OOM;
    } catch (const std::exception &e) {
        saamg::set_error(e.what());
        return AMG_ERR_ARG;
    }
}

void amg_hierarchy_free(amg_hierarchy *h) { delete h; }

amg_status amg_hierarchy_stats(const amg_hierarchy *h, amg_stats_t *st) {
    if (!h || !st) {
        saamg::set_error("null argument");
        return AMG_ERR_ARG;
    }
    std::memset(st, 0, sizeof(*st));
    const auto &H = h->H;
    st->levels = (int32_t)H.levels.size();
    double nnz1 = (double)H.levels[0].A.nnzb(), tot = 0.0;
    for (size_t l = 0; l < H.levels.size(); ++l) {
        const auto &L = H.levels[l];
        st->nb[l] = L.A.rows;
        st->nnzb_A[l] = L.A.nnzb();
        st->nnzb_P[l] = L.P.nnzb();
        st->n_agg[l] = L.n_agg;
        st->omega_j[l] = L.omega_j;
        tot += (double)L.A.nnzb();
    }
    st->n_coarse = H.n_coarse;
    st->operator_complexity = tot / nnz1;
    st->setup_ms = H.setup_ms;
    for (int q = 0; q < 11; ++q) st->setup_phase_ms[q] = H.phase_ms[q];
    return AMG_OK;
}

amg_status amg_hierarchy_level_shape(const amg_hierarchy *h, int32_t level, int32_t which,
                                     int32_t *rows, int32_t *cols, int64_t *nnzb) {
    if (!h || !rows || !cols || !nnzb) {
        saamg::set_error("null argument");
        return AMG_ERR_ARG;
    }
    const auto &H = h->H;
    if (which == 5) {
        *rows = *cols = H.n_coarse;
        *nnzb = (int64_t)H.n_coarse * H.n_coarse;
        return AMG_OK;
    }
    if (which == 6 || which == 7) {  // learned-smoother inputs (level ignored)
        const int per = which == 6 ? 90 : 6;
        const size_t len = which == 6 ? H.learn_phi.size() : H.learn_L.size();
        *rows = (int32_t)(len / per);
        *cols = per;
        *nnzb = (int64_t)len;
        return AMG_OK;
    }
    if (level < 0 || level >= (int32_t)H.levels.size()) {
        saamg::set_error("level out of range");
        return AMG_ERR_ARG;
    }
    const auto &L = H.levels[level];
    const saamg::Bsr3 *M = nullptr;
    switch (which) {
        case 0: M = &L.A; break;
        case 1: M = &L.P; break;
        case 2: M = &L.R; break;
        case 9: M = &L.AM; break;
        case 10: M = &L.G; break;
        case 12: M = &L.ilu_L; break;
        case 13:
            *rows = *cols = L.ilu_colour.empty() ? 0 : L.A.rows;
            *nnzb = L.ilu_colour.empty() ? 0 : L.ilu_U.nnzb() + L.A.rows;
            return AMG_OK;
        case 11:
            *rows = *cols = L.A.rows;
            *nnzb = (int64_t)L.ilu_colour.size();
            return AMG_OK;
        case 3:
        case 8:
            *rows = *cols = L.A.rows;
            *nnzb = L.Minv.empty() ? 0 : L.A.rows;
            return AMG_OK;
        case 4:
            *rows = (int32_t)L.agg.size();
            *cols = L.n_agg;
            *nnzb = (int64_t)L.agg.size();
            return AMG_OK;
        default: saamg::set_error("unknown export kind"); return AMG_ERR_ARG;
    }
    *rows = M->rows;
    *cols = M->cols;
    *nnzb = M->nnzb();
    return AMG_OK;
}

amg_status amg_hierarchy_export(const amg_hierarchy *h, int32_t level, int32_t which,
                                int32_t *row_ptr, int32_t *col, double *val) {
    int32_t rows, cols;
    int64_t nnzb;
    amg_status s = amg_hierarchy_level_shape(h, level, which, &rows, &cols, &nnzb);
    if (s != AMG_OK) return s;
    const auto &H = h->H;
    if (which == 5) {
        if (!val) return AMG_ERR_ARG;
        std::memcpy(val, H.coarse_inv.data(), H.coarse_inv.size() * sizeof(double));
        return AMG_OK;
    }
    if (which == 6) {
        if (!val) return AMG_ERR_ARG;
        for (size_t i = 0; i < H.learn_phi.size(); ++i) val[i] = (double)H.learn_phi[i];
        return AMG_OK;
    }
    if (which == 7) {
        if (!val) return AMG_ERR_ARG;
        std::memcpy(val, H.learn_L.data(), H.learn_L.size() * sizeof(double));
        return AMG_OK;
    }
    const auto &L = H.levels[level];
    if (which == 3 || which == 8) {
        if (!val) return AMG_ERR_ARG;
        const std::vector<double> &M = (which == 8 && !L.Mpost.empty()) ? L.Mpost : L.Minv;
        std::memcpy(val, M.data(), M.size() * sizeof(double));
        return AMG_OK;
    }
    if (which == 4) {
        if (!val) return AMG_ERR_ARG;
        for (size_t i = 0; i < L.agg.size(); ++i) val[i] = (double)L.agg[i];
        return AMG_OK;
    }
    if (which == 11) {
        if (!val) return AMG_ERR_ARG;
        for (size_t i = 0; i < L.ilu_colour.size(); ++i) val[i] = (double)L.ilu_colour[i];
        return AMG_OK;
    }
    if (!row_ptr || !col || !val) {
        saamg::set_error("null output array");
        return AMG_ERR_ARG;
    }
    if (which == 13) {  // U with its diagonal blocks, columns sorted
        if (L.ilu_colour.empty()) {
            row_ptr[0] = 0;
            return AMG_OK;
        }
        const saamg::Bsr3 &U = L.ilu_U;
        int64_t q = 0;
        row_ptr[0] = 0;
        for (int32_t i = 0; i < U.rows; ++i) {
            bool placed = false;
            for (int64_t k = U.ptr[i]; k <= U.ptr[i + 1]; ++k) {
                if (!placed && (k == U.ptr[i + 1] || U.col[k] > i)) {
                    col[q] = i;
                    std::memcpy(val + 9 * q, &L.ilu_D[9 * (size_t)i], 9 * sizeof(double));
                    ++q;
                    placed = true;
                }
                if (k == U.ptr[i + 1]) break;
                col[q] = U.col[k];
                std::memcpy(val + 9 * q, &U.val[9 * k], 9 * sizeof(double));
                ++q;
            }
            row_ptr[i + 1] = (int32_t)q;
        }
        return AMG_OK;
    }
    const saamg::Bsr3 &M = which == 0   ? L.A
                           : which == 1 ? L.P
                           : which == 2 ? L.R
                           : which == 9 ? L.AM
                           : which == 12 ? L.ilu_L
                                         : L.G;
    if (M.ptr.empty()) {  // an operator this level does not have
        row_ptr[0] = 0;
        return AMG_OK;
    }
    for (int32_t i = 0; i <= M.rows; ++i) row_ptr[i] = (int32_t)M.ptr[i];
    std::memcpy(col, M.col.data(), M.col.size() * sizeof(int32_t));
    std::memcpy(val, M.val.data(), M.val.size() * sizeof(double));
    return AMG_OK;
}

}  // extern "C"
