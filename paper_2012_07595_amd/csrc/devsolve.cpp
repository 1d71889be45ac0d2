// Cholesky solve of the (shifted) Newton system of the inner solve on the
// device, for systems too large for the host (N = r(k1 - r) + r3(k3 - r3)
// reaches 2750 at rank (10,10,10)).  rocSOLVER's FP64 potrf/potrs on the
// ctx's stream; the matrix is symmetric, so row-major input is its own
// column-major transpose.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "bks_internal.h"

namespace bks {

DevSolver::~DevSolver() {
    if (handle) rocblas_destroy_handle(static_cast<rocblas_handle>(handle));
}

bool DevSolver::solve(hipStream_t s, int N, const double *H, double *b) {
    if (!handle) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) fail(BKS_EDEVICE, "rocblas handle");
        handle = h;
    }
    rocblas_handle h = static_cast<rocblas_handle>(handle);
    if (rocblas_set_stream(h, s) != rocblas_status_success) fail(BKS_EDEVICE, "rocblas stream");
    dA.ensure((size_t)N * N * 8);
    db.ensure((size_t)N * 8 + 64);
    HIPCHECK(hipMemcpyAsync(dA.ptr, H, (size_t)N * N * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(db.ptr, b, (size_t)N * 8, hipMemcpyHostToDevice, s));
    rocblas_int *dinfo = reinterpret_cast<rocblas_int *>(db.as<char>() + (size_t)N * 8);
    if (rocsolver_dpotrf(h, rocblas_fill_lower, N, dA.as<double>(), N, dinfo) !=
        rocblas_status_success)
        fail(BKS_EDEVICE, "rocsolver_dpotrf");
    rocblas_int info = 0;
    HIPCHECK(hipMemcpyAsync(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (info != 0) return false;
    if (rocsolver_dpotrs(h, rocblas_fill_lower, N, 1, dA.as<double>(), N, db.as<double>(), N) !=
        rocblas_status_success)
        fail(BKS_EDEVICE, "rocsolver_dpotrs");
    HIPCHECK(hipMemcpyAsync(b, db.ptr, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    return true;
}

}  // namespace bks
