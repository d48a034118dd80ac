// Block-arithmetic sparse kernels for the host setup: BSR3 products,
// transposes and matrix-vector products (FP64).  Used for the Galerkin
// product A_{i+1} = R_i A_i P_i of Algorithm 1 in block form, as the paper's
// "NS Block" variant does (Section 3).
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <exception>
#include <mutex>
#include <thread>

#include "setup_internal.hpp"

namespace saamg {

int resolve_threads(int requested) {
    if (requested > 0) return requested;
    unsigned hc = std::thread::hardware_concurrency();
    return hc ? (int)std::min(hc, 64u) : 4;
}

namespace {

// Fork-join pool kept for the life of the process: creating threads is the
// dominant cost of small setups otherwise.  parallel_for splits [0, n) into
// contiguous chunks, the calling thread takes part, and calls are serialised.
// The chunk counter holds the call's generation in its upper half, and a
// thread claims a chunk only while the counter still belongs to the call it
// woke for: a thread that is late from one call can never take (and run a
// second time) a chunk of the next one.
class Pool {
  public:
    static Pool &get() {
        static Pool p;
        return p;
    }
    void run(int chunks, const std::function<void(int)> &job) {
        std::lock_guard<std::mutex> call(call_mu_);
        ensure(chunks - 1);
        uint32_t g;
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &job;
            chunks_ = chunks;
            pending_ = chunks;
            g = (uint32_t)++gen_;
            next_.store((uint64_t)g << 32);
        }
        cv_.notify_all();
        work(g, chunks, &job);
        std::exception_ptr err;
        {
            std::unique_lock<std::mutex> lk(mu_);
            done_cv_.wait(lk, [&] { return pending_ == 0; });
            job_ = nullptr;
            err = error_;
            error_ = nullptr;
        }
        if (err) std::rethrow_exception(err);
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            ++gen_;
        }
        cv_.notify_all();
        for (auto &t : threads_) t.join();
    }

  private:
    void ensure(int workers) {
        while ((int)threads_.size() < workers) threads_.emplace_back([this] { loop(); });
    }
    // Runs chunks of call g until none is left (or the counter has moved on).
    void work(uint32_t g, int chunks, const std::function<void(int)> *job) {
        for (;;) {
            uint64_t v = next_.load();
            int c;
            for (;;) {
                if ((uint32_t)(v >> 32) != g) return;
                c = (int)(uint32_t)v;
                if (c >= chunks) return;
                if (next_.compare_exchange_weak(v, v + 1)) break;
            }
            std::exception_ptr err;
            try {
                (*job)(c);
            } catch (...) {
                err = std::current_exception();
            }
            std::lock_guard<std::mutex> lk(mu_);
            if (err && !error_) error_ = err;
            if (--pending_ == 0) done_cv_.notify_all();
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            uint32_t g;
            int chunks;
            const std::function<void(int)> *job;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                g = (uint32_t)gen_;
                chunks = chunks_;
                job = job_;
            }
            if (job) work(g, chunks, job);
        }
    }
    std::mutex call_mu_, mu_;
    std::condition_variable cv_, done_cv_;
    std::vector<std::thread> threads_;
    const std::function<void(int)> *job_ = nullptr;
    int chunks_ = 0;
    int pending_ = 0;
    std::atomic<uint64_t> next_{0};
    uint64_t gen_ = 0;
    bool stop_ = false;
    std::exception_ptr error_;
};

}  // namespace

void parallel_tasks(int ntasks, const std::function<void(int)> &fn) {
    if (ntasks <= 0) return;
    if (ntasks == 1) {
        fn(0);
        return;
    }
    Pool::get().run(ntasks, fn);
}

void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t, int64_t)> &fn) {
    if (n <= 0) return;
    int T = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads, n / 1024));
    if (T == 1) {
        fn(0, n);
        return;
    }
    parallel_tasks(T, [&](int t) { fn(n * t / T, n * (t + 1) / T); });
}

static inline void gemm3_acc(const double *a, const double *b, double *c) {
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double ar = a[3 * r + k];
            c[3 * r + 0] += ar * b[3 * k + 0];
            c[3 * r + 1] += ar * b[3 * k + 1];
            c[3 * r + 2] += ar * b[3 * k + 2];
        }
}

// C = A B, row by row with a dense accumulator over the block columns of B.
Bsr3 bsr_multiply(const Bsr3 &A, const Bsr3 &B, int nthreads) {
    Bsr3 C;
    C.rows = A.rows;
    C.cols = B.cols;
    int T = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads, A.rows / 256 + 1));
    struct Part {
        std::vector<int32_t> col;
        std::vector<double> val;
        std::vector<int64_t> cnt;
    };
    std::vector<Part> parts(T);
    std::vector<int64_t> rb(T + 1);
    for (int t = 0; t <= T; ++t) rb[t] = (int64_t)A.rows * t / T;
    auto work = [&](int t) {
        Part &p = parts[t];
        std::vector<double> acc((size_t)B.cols * 9, 0.0);
        std::vector<int32_t> mark(B.cols, -1);
        std::vector<int32_t> touched;
        p.cnt.resize(rb[t + 1] - rb[t]);
        for (int64_t i = rb[t]; i < rb[t + 1]; ++i) {
            touched.clear();
            for (int64_t ka = A.ptr[i]; ka < A.ptr[i + 1]; ++ka) {
                int32_t k = A.col[ka];
                const double *a = &A.val[9 * ka];
                for (int64_t kb = B.ptr[k]; kb < B.ptr[k + 1]; ++kb) {
                    int32_t j = B.col[kb];
                    if (mark[j] != (int32_t)i) {
                        mark[j] = (int32_t)i;
                        touched.push_back(j);
                        std::fill(&acc[9 * (size_t)j], &acc[9 * (size_t)j] + 9, 0.0);
                    }
                    gemm3_acc(a, &B.val[9 * kb], &acc[9 * (size_t)j]);
                }
            }
            std::sort(touched.begin(), touched.end());
            for (int32_t j : touched) {
                p.col.push_back(j);
                p.val.insert(p.val.end(), &acc[9 * (size_t)j], &acc[9 * (size_t)j] + 9);
            }
            p.cnt[i - rb[t]] = (int64_t)touched.size();
        }
    };
    parallel_tasks(T, work);
    C.ptr.assign((size_t)A.rows + 1, 0);
    for (int t = 0; t < T; ++t)
        for (int64_t i = rb[t]; i < rb[t + 1]; ++i) C.ptr[i + 1] = parts[t].cnt[i - rb[t]];
    for (int64_t i = 0; i < A.rows; ++i) C.ptr[i + 1] += C.ptr[i];
    C.col.resize(C.ptr[A.rows]);
    C.val.resize(9 * (size_t)C.ptr[A.rows]);
    parallel_tasks(T, [&](int t) {
        int64_t off = C.ptr[rb[t]];
        std::copy(parts[t].col.begin(), parts[t].col.end(), C.col.begin() + off);
        std::copy(parts[t].val.begin(), parts[t].val.end(), C.val.begin() + 9 * off);
    });
    return C;
}

// Pattern of A B (block columns sorted per row, no values).
Bsr3 bsr_symbolic(const Bsr3 &A, const Bsr3 &B, int nthreads) {
    Bsr3 C;
    C.rows = A.rows;
    C.cols = B.cols;
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads, A.rows / 256 + 1));
    std::vector<std::vector<int32_t>> cols(T);
    std::vector<std::vector<int64_t>> cnt(T);
    std::vector<int64_t> rb(T + 1);
    for (int t = 0; t <= T; ++t) rb[t] = (int64_t)A.rows * t / T;
    parallel_tasks(T, [&](int t) {
        std::vector<int32_t> mark(B.cols, -1), touched;
        for (int64_t i = rb[t]; i < rb[t + 1]; ++i) {
            touched.clear();
            for (int64_t ka = A.ptr[i]; ka < A.ptr[i + 1]; ++ka) {
                const int32_t k = A.col[ka];
                for (int64_t kb = B.ptr[k]; kb < B.ptr[k + 1]; ++kb) {
                    const int32_t j = B.col[kb];
                    if (mark[j] != (int32_t)i) {
                        mark[j] = (int32_t)i;
                        touched.push_back(j);
                    }
                }
            }
            std::sort(touched.begin(), touched.end());
            cols[t].insert(cols[t].end(), touched.begin(), touched.end());
            cnt[t].push_back((int64_t)touched.size());
        }
    });
    C.ptr.assign((size_t)A.rows + 1, 0);
    for (int t = 0; t < T; ++t)
        for (int64_t i = rb[t]; i < rb[t + 1]; ++i) C.ptr[i + 1] = cnt[t][i - rb[t]];
    for (int64_t i = 0; i < A.rows; ++i) C.ptr[i + 1] += C.ptr[i];
    C.col.resize(C.ptr[A.rows]);
    for (int t = 0; t < T; ++t) std::copy(cols[t].begin(), cols[t].end(), C.col.begin() + C.ptr[rb[t]]);
    return C;
}

// Rows of A are split into contiguous ranges, one per task; task t's blocks of
// column j go after those of the earlier tasks, so every transposed row keeps
// the increasing order of the serial scatter whatever the task count.
Bsr3 bsr_transpose(const Bsr3 &A, int nthreads) {
    Bsr3 T;
    T.rows = A.cols;
    T.cols = A.rows;
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(std::max(nthreads, 1), A.nnzb() / 65536 + 1));
    std::vector<int64_t> rb(nt + 1);
    for (int t = 0; t <= nt; ++t) rb[t] = (int64_t)A.rows * t / nt;
    std::vector<std::vector<int64_t>> cnt(nt, std::vector<int64_t>((size_t)A.cols, 0));
    parallel_tasks(nt, [&](int t) {
        for (int64_t k = A.ptr[rb[t]]; k < A.ptr[rb[t + 1]]; ++k) ++cnt[t][A.col[k]];
    });
    // T.ptr from the column totals; cnt[t][j] becomes task t's first slot in row j
    T.ptr.assign((size_t)A.cols + 1, 0);
    for (int32_t j = 0; j < A.cols; ++j) {
        int64_t o = T.ptr[j];
        for (int t = 0; t < nt; ++t) {
            const int64_t n = cnt[t][j];
            cnt[t][j] = o;
            o += n;
        }
        T.ptr[j + 1] = o;
    }
    T.col.resize(A.col.size());
    T.val.resize(A.val.size());  // every block is written below
    parallel_tasks(nt, [&](int t) {
        std::vector<int64_t> &pos = cnt[t];
        for (int64_t i = rb[t]; i < rb[t + 1]; ++i)
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                const int64_t d = pos[A.col[k]]++;
                T.col[d] = (int32_t)i;
                const double *s = &A.val[9 * k];
                double *tv = &T.val[9 * d];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) tv[3 * r + c] = s[3 * c + r];
            }
    });
    return T;
}

void bsr_spmv(const Bsr3 &A, const double *x, double *y, int nthreads) {
    parallel_for(A.rows, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            double s0 = 0, s1 = 0, s2 = 0;
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                const double *a = &A.val[9 * k];
                const double *xv = &x[3 * (size_t)A.col[k]];
                s0 += a[0] * xv[0] + a[1] * xv[1] + a[2] * xv[2];
                s1 += a[3] * xv[0] + a[4] * xv[1] + a[5] * xv[2];
                s2 += a[6] * xv[0] + a[7] * xv[1] + a[8] * xv[2];
            }
            y[3 * i] = s0;
            y[3 * i + 1] = s1;
            y[3 * i + 2] = s2;
        }
    });
}

}  // namespace saamg
