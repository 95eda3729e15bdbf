// Setup-time eigendecomposition of the kinship matrix on the device
// (gwas_eigh): Phi = Z diag(w) Z^T in FP64 by rocSOLVER's divide-and-conquer
// symmetric eigensolver. The solver library is large and only setup needs it,
// so it is opened on the first call rather than linked; its headers supply
// the types and enumerations only.
#include <dlfcn.h>

#include <mutex>

#include <rocsolver/rocsolver.h>

#include "ctx.h"

using gw::fail;

namespace {

struct Solver {
    decltype(&rocblas_create_handle) create = nullptr;
    decltype(&rocblas_destroy_handle) destroy = nullptr;
    decltype(&rocblas_set_stream) set_stream = nullptr;
    decltype(&rocsolver_dsyevd) dsyevd = nullptr;
    std::string error;
};

const Solver &solver() {
    static Solver s;
    static std::once_flag once;
    std::call_once(once, [] {
        void *h = dlopen("librocsolver.so.0", RTLD_NOW | RTLD_LOCAL);
        if (!h) h = dlopen("/opt/rocm/lib/librocsolver.so.0", RTLD_NOW | RTLD_LOCAL);
        if (!h) {
            const char *e = dlerror();
            s.error = std::string("cannot open librocsolver.so.0: ") + (e ? e : "");
            return;
        }
        s.create = (decltype(s.create))dlsym(h, "rocblas_create_handle");
        s.destroy = (decltype(s.destroy))dlsym(h, "rocblas_destroy_handle");
        s.set_stream = (decltype(s.set_stream))dlsym(h, "rocblas_set_stream");
        s.dsyevd = (decltype(s.dsyevd))dlsym(h, "rocsolver_dsyevd");
        if (!s.create || !s.destroy || !s.set_stream || !s.dsyevd) s.error = "rocSOLVER/rocBLAS symbols not found";
    });
    return s;
}

}  // namespace

extern "C" gwas_status gwas_eigh(int32_t n, const double *Phi, double *Z, double *w, int32_t on_device,
                                 void *stream) {
    gw::last_error().clear();
    if (n < 1 || n > 16384) return fail(GWAS_EINVAL, "n = %d outside [1, 16384]", n);
    if (!Phi || !Z || !w) return fail(GWAS_EINVAL, "NULL argument");
    const Solver &sv = solver();
    if (!sv.error.empty()) return fail(GWAS_EHIP, "%s", sv.error.c_str());
    hipStream_t s = (hipStream_t)stream;
    const size_t nn = (size_t)n * n;
    double *dA = nullptr, *dD = nullptr, *dE = nullptr;
    rocblas_int *dinfo = nullptr;
    rocblas_handle handle = nullptr;
    gwas_status st = GWAS_OK;
    rocblas_int info = 0;
    auto run = [&]() -> gwas_status {
        HIP_TRY(hipMalloc(&dA, sizeof(double) * nn));
        HIP_TRY(hipMalloc(&dD, sizeof(double) * n));
        HIP_TRY(hipMalloc(&dE, sizeof(double) * n));
        HIP_TRY(hipMalloc(&dinfo, sizeof(rocblas_int)));
        HIP_TRY(hipMemcpyAsync(dA, Phi, sizeof(double) * nn,
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        if (sv.create(&handle) != rocblas_status_success) return fail(GWAS_EHIP, "rocblas_create_handle failed");
        if (sv.set_stream(handle, s) != rocblas_status_success) return fail(GWAS_EHIP, "rocblas_set_stream failed");
        const rocblas_status rs =
            sv.dsyevd(handle, rocblas_evect_original, rocblas_fill_lower, n, dA, n, dD, dE, dinfo);
        if (rs != rocblas_status_success) return fail(GWAS_EHIP, "rocsolver_dsyevd failed (status %d)", (int)rs);
        HIP_TRY(hipMemcpyAsync(&info, dinfo, sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (info != 0) return fail(GWAS_EHIP, "eigensolver did not converge (info %d)", (int)info);
        const hipMemcpyKind out = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        HIP_TRY(hipMemcpyAsync(Z, dA, sizeof(double) * nn, out, s));
        HIP_TRY(hipMemcpyAsync(w, dD, sizeof(double) * n, out, s));
        HIP_TRY(hipStreamSynchronize(s));
        return GWAS_OK;
    };
    st = run();
    if (handle) sv.destroy(handle);
    for (void *p : {(void *)dA, (void *)dD, (void *)dE, (void *)dinfo})
        if (p) (void)hipFree(p);
    return st;
}
