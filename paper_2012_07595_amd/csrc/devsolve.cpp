// Device help for the inner solve (Algorithm 5 step (i)) of large cores:
//  - Cholesky solve of the (shifted) Newton system, for systems too large for
//    the host (N = r(k1 - r) + r3(k3 - r3) reaches 2750 at rank (10,10,10),
//    17000 at rank 20): the blocked factorisation of cholesky.hip up to
//    order kSmallCholMax (the forward substitution riding along; 256-column
//    panels with a rocBLAS dsyrk update from order 8192) and rocSOLVER's
//    FP64 potrf beyond, then the remaining triangular solves (after ours
//    only the backward one: one workgroup of trisolve.hip up to order
//    kSolveWgMax, rocBLAS's trsv up to kPotrsMax, the multi-launch blocked
//    solve beyond; after potrf, potrs up to kPotrsMax and the blocked
//    solves beyond), all on the ctx's stream with one
//    synchronisation per solve; the matrix is symmetric, so row-major
//    input is its own column-major transpose;
//  - the dense products of the core (HOSVD Grams, mode-3 products, the
//    rotation into [P P_perp], [S S_perp] coordinates) as rocBLAS FP64
//    GEMMs.  Device matrices are column-major; a row-major host matrix
//    uploaded as is reads as its transpose.
#include <algorithm>
#include <cstring>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "bks_internal.h"

namespace bks {

DevSolver::~DevSolver() {
    if (handle) rocblas_destroy_handle(static_cast<rocblas_handle>(handle));
}

void *DevSolver::get_handle(hipStream_t s) {
    if (!handle) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) fail(BKS_EDEVICE, "rocblas handle");
        // no atomics: every product sums in a fixed order, run to run
        if (rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed) != rocblas_status_success)
            fail(BKS_EDEVICE, "rocblas atomics mode");
        handle = h;
    }
    rocblas_handle h = static_cast<rocblas_handle>(handle);
    if (rocblas_set_stream(h, s) != rocblas_status_success) fail(BKS_EDEVICE, "rocblas stream");
    return handle;
}

bool DevSolver::solve(hipStream_t s, int N, const double *H, double mu, bool new_matrix,
                      double *b) {
    const size_t bytes = (size_t)N * N * 8;
    if (new_matrix || dH.bytes < bytes) {
        dH.ensure(bytes);
        HIPCHECK(hipMemcpyAsync(dH.ptr, H, bytes, hipMemcpyHostToDevice, s));
    }
    return solve_resident(s, N, mu, b);
}

bool DevSolver::solve_resident(hipStream_t s, int N, double mu, double *b) {
    const size_t bytes = (size_t)N * N * 8;
    if (dH.bytes < bytes) fail(BKS_EINVAL, "Newton matrix not on the device");
    dA.ensure(bytes);
    // b, then info (64 bytes), then the factorisation's workspace
    db.ensure((size_t)N * 8 + 64 + kCholWork * 8);
    pin.ensure((size_t)N * 8 + 64);
    double *st = reinterpret_cast<double *>(pin.ptr);
    shift_copy_dev(s, dA.as<double>(), dH.as<double>(), N, mu);
    std::memcpy(st, b, (size_t)N * 8);
    HIPCHECK(hipMemcpyAsync(db.ptr, st, (size_t)N * 8, hipMemcpyHostToDevice, s));
    int *dinfo = reinterpret_cast<int *>(db.as<char>() + (size_t)N * 8);
    // our blocked factorisation up to kSmallCholMax (0.30 against 1.18 ms on
    // potrf at order 500, 2.6 against 7.8 ms at 2750, 61 against 106 ms at
    // 17000), with the forward substitution riding along (db becomes
    // L^{-1} b); rocSOLVER's potrf beyond
    const bool own = N <= kSmallCholMax;
    if (own) {
        double *dwork = reinterpret_cast<double *>(db.as<char>() + (size_t)N * 8 + 64);
        chol_factor_dev(s, dA.as<double>(), N, dinfo, db.as<double>(), dwork, get_handle(s));
    } else {
        static_assert(sizeof(rocblas_int) == sizeof(int), "info is an int");
        rocblas_handle h = static_cast<rocblas_handle>(get_handle(s));
        if (rocsolver_dpotrf(h, rocblas_fill_lower, N, dA.as<double>(), N,
                             reinterpret_cast<rocblas_int *>(dinfo)) != rocblas_status_success)
            fail(BKS_EDEVICE, "rocsolver_dpotrf");
    }
    // the remaining triangular solves, enqueued behind the factorisation:
    // after our factorisation only L^T x = y, in one workgroup for small
    // orders (it skips itself after a failed factorisation) or rocBLAS's
    // trsv; after potrf both, by potrs up to kPotrsMax and by the
    // multi-launch blocked solves beyond (potrs ran each triangular solve
    // at ~15-20 ms at order 17000).  All but the one-workgroup solve run on
    // after a failure and their result is dropped.
    if (own && N <= kSolveWgMax) {
        chol_solve_small(s, dA.as<double>(), N, db.as<double>(), dinfo, false);
    } else if (own && N > kPotrsMax) {
        chol_solve_dev(s, dA.as<double>(), N, db.as<double>(), false);
    } else if (own) {
        rocblas_handle h = static_cast<rocblas_handle>(get_handle(s));
        if (rocblas_dtrsv(h, rocblas_fill_lower, rocblas_operation_transpose,
                          rocblas_diagonal_non_unit, N, dA.as<double>(), N, db.as<double>(),
                          1) != rocblas_status_success)
            fail(BKS_EDEVICE, "rocblas_dtrsv");
    } else if (N <= kPotrsMax) {
        rocblas_handle h = static_cast<rocblas_handle>(get_handle(s));
        if (rocsolver_dpotrs(h, rocblas_fill_lower, N, 1, dA.as<double>(), N, db.as<double>(),
                             N) != rocblas_status_success)
            fail(BKS_EDEVICE, "rocsolver_dpotrs");
    } else {
        chol_solve_dev(s, dA.as<double>(), N, db.as<double>());
    }
    // the solution and info in one transfer, one synchronisation
    HIPCHECK(hipMemcpyAsync(st, db.ptr, (size_t)N * 8 + sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    int info = 0;
    std::memcpy(&info, st + N, sizeof(int));
    if (info != 0) return false;
    std::memcpy(b, st, (size_t)N * 8);
    return true;
}


// ---------------------------------------------------------------- DevInner
namespace {
void check_rb(rocblas_status st, const char *what) {
    if (st != rocblas_status_success) fail(BKS_EDEVICE, what);
}
void dgemm_sb(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
              const double *A, int lda, int64_t sA, const double *B, int ldb, int64_t sB,
              double *C, int ldc, int64_t sC, int batch) {
    const double one = 1.0, zero = 0.0;
    check_rb(rocblas_dgemm_strided_batched(h, ta, tb, m, n, k, &one, A, lda, sA, B, ldb, sB, &zero,
                                           C, ldc, sC, batch),
             "rocblas_dgemm_strided_batched");
}
}  // namespace

// Small transfers of the inner solve go through a pinned staging buffer
// (one copy per call for several operands; every DevInner call ends with a
// stream synchronisation, so the buffer is free again on return).
double *DevInner::stage(size_t count) {
    pin.ensure(count * 8);
    return reinterpret_cast<double *>(pin.ptr);
}

void DevInner::set_core(const double *C, int k1_, int k3_) {
    k1 = k1_;
    k3 = k3_;
    rot_r = rot_r3 = -1;
    newton_n = 0;
    const size_t n = (size_t)k1 * k1 * k3;
    dC.ensure(n * 8);
    HIPCHECK(hipMemcpyAsync(dC.ptr, C, n * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipStreamSynchronize(s));
}

// A single GEMM with a k1 x k1 (or k3 x k3) result and an inner dimension
// of k1 k3 (k1^2) runs on one or two workgroups; the Grams are formed as
// batched partial products over the core's slices instead, summed in a fixed
// order by a matrix-vector product with ones.
void DevInner::sum_parts(const double *parts, int len, int nparts, double *out_host) {
    rocblas_handle h = static_cast<rocblas_handle>(ds->get_handle(s));
    if (dOnes.bytes < (size_t)nparts * 8) {
        // ones over the whole allocation, slack included (see DevSolver::solve)
        dOnes.ensure((size_t)nparts * 8);
        std::vector<double> ones(dOnes.bytes / 8, 1.0);
        HIPCHECK(hipMemcpyAsync(dOnes.ptr, ones.data(), ones.size() * 8, hipMemcpyHostToDevice, s));
        HIPCHECK(hipStreamSynchronize(s));
    }
    dOut.ensure((size_t)len * 8);
    const double one = 1.0, zero = 0.0;
    check_rb(rocblas_dgemv(h, rocblas_operation_none, len, nparts, &one, parts, len,
                           dOnes.as<double>(), 1, &zero, dOut.as<double>(), 1),
             "rocblas_dgemv");
    double *hs = stage(len);
    HIPCHECK(hipMemcpyAsync(hs, dOut.ptr, (size_t)len * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    std::memcpy(out_host, hs, (size_t)len * 8);
}

void DevInner::gram1(double *G1) {
    rocblas_handle h = static_cast<rocblas_handle>(ds->get_handle(s));
    const int64_t sl = (int64_t)k1 * k1;
    dT.ensure((size_t)sl * k3 * 8);
    // part c = X_c X_c^T with X_c = C(:, :, c) (column-major k1 x k1)
    dgemm_sb(h, rocblas_operation_none, rocblas_operation_transpose, k1, k1, k1, dC.as<double>(),
             k1, sl, dC.as<double>(), k1, sl, dT.as<double>(), k1, sl, k3);
    sum_parts(dT.as<double>(), (int)sl, k3, G1);
}

void DevInner::gram3(double *G3) {
    rocblas_handle h = static_cast<rocblas_handle>(ds->get_handle(s));
    const int sl = k1 * k1;
    const int64_t g = (int64_t)k3 * k3;
    dT.ensure((size_t)g * k1 * 8);
    // C is the column-major (k1^2) x k3 matrix C_(3)^T; part b is the product
    // of its rows b k1 .. b k1 + k1 - 1 (the fibres C(:, b, c)) with themselves
    dgemm_sb(h, rocblas_operation_transpose, rocblas_operation_none, k3, k3, k1, dC.as<double>(), sl,
             k1, dC.as<double>(), sl, k1, dT.as<double>(), k3, g, k1);
    sum_parts(dT.as<double>(), (int)g, k1, G3);
}

void DevInner::mode3p(const double *Sv, int ldS, int l0, int nl, const double *P, int r,
                      double *out) {
    rocblas_handle h = static_cast<rocblas_handle>(ds->get_handle(s));
    const int sl = k1 * k1;
    const size_t ns = (size_t)k3 * nl, np = (size_t)k1 * r, no = (size_t)k1 * r * nl;
    // staging: [Sc (column-major k3 x nl) | P], then the result
    double *hs = stage(ns + np + no);
    for (int c = 0; c < k3; ++c)
        for (int l = 0; l < nl; ++l) hs[c + (size_t)k3 * l] = Sv[(size_t)c * ldS + l0 + l];
    std::memcpy(hs + ns, P, np * 8);
    dA.ensure((ns + np) * 8);
    dT.ensure((size_t)sl * nl * 8);
    dOut.ensure(no * 8);
    HIPCHECK(hipMemcpyAsync(dA.ptr, hs, (ns + np) * 8, hipMemcpyHostToDevice, s));
    const double *dS = dA.as<double>(), *dP = dA.as<double>() + ns;
    // CS = C_(3)^T Sc (k1^2 x nl), then M_l = CS_l P with CS_l the k1 x k1
    // slice l; P row-major k1 x r reads as the column-major r x k1 matrix P^T
    dgemm_sb(h, rocblas_operation_none, rocblas_operation_none, sl, nl, k3, dC.as<double>(), sl, 0,
             dS, k3, 0, dT.as<double>(), sl, 0, 1);
    dgemm_sb(h, rocblas_operation_none, rocblas_operation_transpose, k1, r, k1, dT.as<double>(), k1,
             sl, dP, r, 0, dOut.as<double>(), k1, (int64_t)k1 * r, nl);
    HIPCHECK(hipMemcpyAsync(hs + ns + np, dOut.ptr, no * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    std::memcpy(out, hs + ns + np, no * 8);
}

void DevInner::hooi3(const double *P, int r, double *M3) {
    rocblas_handle h = static_cast<rocblas_handle>(ds->get_handle(s));
    const int64_t sl = (int64_t)k1 * k1;
    // P row-major k1 x r reads as the column-major r x k1 matrix P^T
    dA.ensure((size_t)k1 * r * 8);
    dT.ensure((size_t)k1 * r * k3 * 8);
    dOut.ensure((size_t)r * r * k3 * 8);
    const size_t np = (size_t)k1 * r, no = (size_t)r * r * k3;
    double *hs = stage(np + no);
    std::memcpy(hs, P, np * 8);
    HIPCHECK(hipMemcpyAsync(dA.ptr, hs, np * 8, hipMemcpyHostToDevice, s));
    // CP_c = C_c P (k1 x r), then M_c = P^T CP_c (r x r, M_c(i, j) at i + r j)
    dgemm_sb(h, rocblas_operation_none, rocblas_operation_transpose, k1, r, k1, dC.as<double>(), k1,
             sl, dA.as<double>(), r, 0, dT.as<double>(), k1, (int64_t)k1 * r, k3);
    dgemm_sb(h, rocblas_operation_none, rocblas_operation_none, r, r, k1, dA.as<double>(), r, 0,
             dT.as<double>(), k1, (int64_t)k1 * r, dOut.as<double>(), r, (int64_t)r * r, k3);
    HIPCHECK(hipMemcpyAsync(hs + np, dOut.ptr, no * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    std::memcpy(M3, hs + np, no * 8);
}

void DevInner::rotate(const double *Qp, const double *Qs, int r, int r3, double *Y, double *Y2,
                      bool partial) {
    rocblas_handle h = static_cast<rocblas_handle>(ds->get_handle(s));
    const int64_t sl = (int64_t)k1 * k1;
    const int C1 = k3 - r3;
    // row-major Qp, Qs read as Qp^T, Qs^T; one upload [Qp | Qs], one
    // download [Y | Y2] through the pinned staging buffer
    const size_t nqp = (size_t)k1 * k1, nqs = (size_t)k3 * k3;
    const size_t ny = (size_t)sl * r3, ny2 = (size_t)k1 * r * C1;
    double *hs = stage(std::max(nqp + nqs, ny + ny2));
    std::memcpy(hs, Qp, nqp * 8);
    std::memcpy(hs + nqp, Qs, nqs * 8);
    dA.ensure((nqp + nqs) * 8);
    dOut.ensure((size_t)sl * k3 * 8);
    dT.ensure((size_t)std::max<int64_t>(sl * r3, (int64_t)k1 * r * C1) * 8);
    dY.ensure((ny + ny2) * 8);
    HIPCHECK(hipMemcpyAsync(dA.ptr, hs, (nqp + nqs) * 8, hipMemcpyHostToDevice, s));
    const double *dQs = dA.as<double>() + nqp;
    // X_l = C.(I, I, Qs(:, l)) for every l: (k1^2 x k3) times Qs
    dgemm_sb(h, rocblas_operation_none, rocblas_operation_transpose, (int)sl, k3, k3,
             dC.as<double>(), (int)sl, 0, dQs, k3, 0, dOut.as<double>(), (int)sl, 0, 1);
    double *dYl = dY.as<double>(), *dY2 = dY.as<double>() + sl * r3;
    // Y_l = Qp^T (X_l Qp), l < r3
    dgemm_sb(h, rocblas_operation_none, rocblas_operation_transpose, k1, k1, k1, dOut.as<double>(),
             k1, sl, dA.as<double>(), k1, 0, dT.as<double>(), k1, sl, r3);
    dgemm_sb(h, rocblas_operation_none, rocblas_operation_none, k1, k1, k1, dA.as<double>(), k1, 0,
             dT.as<double>(), k1, sl, dYl, k1, sl, r3);
    if (C1 > 0) {
        // Y2_z = Qp^T (X_{r3+z} Qp(:, :r)); Qp(:, :r)^T is the first r rows of the array
        dgemm_sb(h, rocblas_operation_none, rocblas_operation_transpose, k1, r, k1,
                 dOut.as<double>() + sl * r3, k1, sl, dA.as<double>(), k1, 0, dT.as<double>(), k1,
                 (int64_t)k1 * r, C1);
        dgemm_sb(h, rocblas_operation_none, rocblas_operation_none, k1, r, k1, dA.as<double>(), k1, 0,
                 dT.as<double>(), k1, (int64_t)k1 * r, dY2, k1, (int64_t)k1 * r, C1);
    }
    // (the upload has been consumed before the download lands: same stream)
    const size_t py = (size_t)k1 * r * r3, py2 = (size_t)r * r * C1;
    if (partial) {
        // the first r columns of each Y_l and the first r rows of each Y2
        // column: the gradient's blocks (the Newton matrix reads dY here)
        HIPCHECK(hipMemcpy2DAsync(hs, (size_t)k1 * r * 8, dYl, (size_t)sl * 8, (size_t)k1 * r * 8,
                                  (size_t)r3, hipMemcpyDeviceToHost, s));
        if (C1 > 0)
            HIPCHECK(hipMemcpy2DAsync(hs + py, (size_t)r * 8, dY2, (size_t)k1 * 8, (size_t)r * 8,
                                      (size_t)r * C1, hipMemcpyDeviceToHost, s));
    } else {
        HIPCHECK(hipMemcpyAsync(hs, dYl, (ny + ny2) * 8, hipMemcpyDeviceToHost, s));
    }
    HIPCHECK(hipStreamSynchronize(s));
    // dY keeps [Y | Y2] of this rank for newton_matrix
    // (the Newton matrix in ds->dH stays: the inner solve forms it once per
    // iteration and rotates trial points before it solves again with
    // another shift)
    rot_r = r;
    rot_r3 = r3;
    if (partial) {
        std::memcpy(Y, hs, py * 8);
        if (C1 > 0) std::memcpy(Y2, hs + py, py2 * 8);
    } else {
        std::memcpy(Y, hs, ny * 8);
        if (C1 > 0) std::memcpy(Y2, hs + ny, ny2 * 8);
    }
}

}  // namespace bks
