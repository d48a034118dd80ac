// Host setup with the numeric Galerkin products on the GPU: the hierarchy is
// built as by amg_hierarchy_build (Algorithm 1, block construction), except
// that on every level the values of A P and A_{l+1} = R (A P) are computed by
// the device kernels of galerkin.hip; their patterns (symbolic phase) are
// formed on the host, and the values come back to the host for the next
// level's strength graph and aggregation.
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../host/setup_internal.hpp"
#include "galerkin.hpp"

namespace saamg {

namespace {

#define SD_CHECK(call)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw AmgError{e_ == hipErrorOutOfMemory ? AMG_ERR_OOM : AMG_ERR_HIP,          \
                           std::string(#call) + ": " + hipGetErrorString(e_)};             \
    } while (0)

// Device buffers of one product step, released when it ends.
struct Buffers {
    std::vector<void *> p;
    template <typename T>
    T *get(size_t n) {
        void *q = nullptr;
        SD_CHECK(hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)));
        p.push_back(q);
        return static_cast<T *>(q);
    }
    ~Buffers() {
        for (void *q : p) (void)hipFree(q);
    }
};

struct Uploaded {
    DevBsr m;
    int32_t *crow = nullptr;  // row of each block (product outputs)
    double *val = nullptr;
};

Uploaded upload(const Bsr3 &M, bool values, bool rows_of_blocks, Buffers &buf, hipStream_t s) {
    Uploaded u;
    int64_t *ptr = buf.get<int64_t>(M.ptr.size());
    int32_t *col = buf.get<int32_t>(M.col.size());
    double *val = buf.get<double>(9 * M.col.size());
    SD_CHECK(hipMemcpyAsync(ptr, M.ptr.data(), M.ptr.size() * 8, hipMemcpyHostToDevice, s));
    SD_CHECK(hipMemcpyAsync(col, M.col.data(), M.col.size() * 4, hipMemcpyHostToDevice, s));
    if (values) SD_CHECK(hipMemcpyAsync(val, M.val.data(), M.val.size() * 8, hipMemcpyHostToDevice, s));
    if (rows_of_blocks) {
        std::vector<int32_t> r(M.col.size());
        for (int32_t i = 0; i < M.rows; ++i)
            for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) r[k] = i;
        u.crow = buf.get<int32_t>(r.size());
        SD_CHECK(hipMemcpyAsync(u.crow, r.data(), r.size() * 4, hipMemcpyHostToDevice, s));
        SD_CHECK(hipStreamSynchronize(s));  // r is released on return
    }
    u.m = DevBsr{M.rows, ptr, col, val};
    u.val = val;
    return u;
}

}  // namespace

// AP = A P and Ac = R AP: patterns on the host, values on the device.
void device_galerkin(hipStream_t s, int nthreads, const Bsr3 &A, const Bsr3 &P, const Bsr3 &R, Bsr3 &AP,
                     Bsr3 &Ac) {
    AP = bsr_symbolic(A, P, nthreads);
    Ac = bsr_symbolic(R, AP, nthreads);
    Buffers buf;
    const Uploaded dA = upload(A, true, false, buf, s);
    const Uploaded dP = upload(P, true, false, buf, s);
    const Uploaded dR = upload(R, true, false, buf, s);
    const Uploaded dAP = upload(AP, false, true, buf, s);
    const Uploaded dAc = upload(Ac, false, true, buf, s);
    launch_bsr_product(dA.m, dP.m, dAP.crow, dAP.m.col, AP.nnzb(), dAP.val, s);
    launch_bsr_product(dR.m, dAP.m, dAc.crow, dAc.m.col, Ac.nnzb(), dAc.val, s);
    SD_CHECK(hipGetLastError());
    AP.val.resize(9 * (size_t)AP.nnzb());
    Ac.val.resize(9 * (size_t)Ac.nnzb());
    SD_CHECK(hipMemcpyAsync(AP.val.data(), dAP.val, AP.val.size() * 8, hipMemcpyDeviceToHost, s));
    SD_CHECK(hipMemcpyAsync(Ac.val.data(), dAc.val, Ac.val.size() * 8, hipMemcpyDeviceToHost, s));
    SD_CHECK(hipStreamSynchronize(s));
}

}  // namespace saamg

extern "C" amg_status amg_hierarchy_build_device(const amg_bsr3 *A, const double *coords, const amg_params *prm,
                                                 void *hip_stream, amg_hierarchy **out) {
    using namespace saamg;
    set_error("");
    if (!A || !out) {
        set_error("null argument");
        return AMG_ERR_ARG;
    }
    *out = nullptr;
    amg_params def;
    amg_default_params(&def);
    const amg_params &p = prm ? *prm : def;
    try {
        std::unique_ptr<amg_hierarchy> h(new amg_hierarchy());
        const hipStream_t s = (hipStream_t)hip_stream;
        const int nthreads = resolve_threads(p.nthreads);
        const GalerkinFn fn = [&](const Bsr3 &Al, const Bsr3 &P, const Bsr3 &R, Bsr3 &AP, Bsr3 &Ac) {
            device_galerkin(s, nthreads, Al, P, R, AP, Ac);
        };
        build_hierarchy(*A, coords, p, h->H, &fn);
        *out = h.release();
        return AMG_OK;
    } catch (const AmgError &e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed during setup");
        return AMG_ERR_OOM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return AMG_ERR_ARG;
    }
}
