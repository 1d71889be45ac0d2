// Triangular solves with a Cholesky factor on the device: x <- (L L^T)^{-1} x
// for the lower factor L (N x N, column-major, leading dimension N) that
// rocSOLVER's potrf leaves, one right-hand side (the Newton step of the inner
// solve).  Blocked by 64 rows: each diagonal block is solved by one wave
// (the lanes hold the block's unknowns, the pivot value is broadcast by a
// lane shuffle), the rest of the vector is updated by a matrix-vector pass
// over the block's panel.  Forward: L y = x, then backward: L^T x = y.
// Every sum runs in a fixed order (no atomics), so the result does not
// change from run to run.
#include <algorithm>

#include "bks_internal.h"

namespace bks {

namespace {

constexpr int kTriB = 64;

// L[k0:k0+nb, k0:k0+nb] y = x[k0:k0+nb] in place (forward), one wave
__global__ __launch_bounds__(64) void tri_block_lower(const double *__restrict__ L, int64_t N,
                                                      int64_t k0, int nb, double *__restrict__ x) {
    const int i = threadIdx.x;
    double xi = i < nb ? x[k0 + i] : 0.0;
    for (int j = 0; j < nb; ++j) {
        const int64_t col = (k0 + j) * N + k0;
        double xj = __shfl(xi, j);
        xj = xj / L[col + j];
        if (i == j) xi = xj;
        if (i > j && i < nb) xi -= L[col + i] * xj;
    }
    if (i < nb) x[k0 + i] = xi;
}

// L[k0:k0+nb, k0:k0+nb]^T y = x[k0:k0+nb] in place (backward), one wave
__global__ __launch_bounds__(64) void tri_block_upper_t(const double *__restrict__ L, int64_t N,
                                                        int64_t k0, int nb, double *__restrict__ x) {
    const int i = threadIdx.x;
    double xi = i < nb ? x[k0 + i] : 0.0;
    for (int j = nb - 1; j >= 0; --j) {
        double xj = __shfl(xi, j);
        xj = xj / L[(k0 + j) * N + k0 + j];
        if (i == j) xi = xj;
        // (L^T)(i, j) = L(j, i) for i < j
        if (i < j) xi -= L[(k0 + i) * N + k0 + j] * xj;
    }
    if (i < nb) x[k0 + i] = xi;
}

// x[r] -= sum_{c < nb} L[r, k0 + c] x[k0 + c] for the rows r >= k0 + nb
__global__ __launch_bounds__(256) void tri_update_lower(const double *__restrict__ L, int64_t N,
                                                        int64_t k0, int nb, double *__restrict__ x) {
    __shared__ double xs[kTriB];
    if (threadIdx.x < nb) xs[threadIdx.x] = x[k0 + threadIdx.x];
    __syncthreads();
    const int64_t r = k0 + nb + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    double s = 0.0;
    for (int c = 0; c < nb; ++c) s = fma(L[(k0 + c) * N + r], xs[c], s);
    x[r] -= s;
}

// x[k0 + c] -= sum_{r >= k0 + nb} L[r, k0 + c] x[r] for c < nb: one
// workgroup per column, a strided sum per thread and a tree over the threads
__global__ __launch_bounds__(256) void tri_update_upper_t(const double *__restrict__ L, int64_t N,
                                                          int64_t k0, int nb,
                                                          double *__restrict__ x) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    const double *col = L + (k0 + c) * N;
    double s = 0.0;
    for (int64_t r = k0 + nb + threadIdx.x; r < N; r += 256) s = fma(col[r], x[r], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) x[k0 + c] -= red[0];
}

}  // namespace

void chol_solve_dev(hipStream_t s, const double *L, int N, double *x) {
    const int64_t n = N;
    const int64_t nblk = (n + kTriB - 1) / kTriB;
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t k0 = b * kTriB;
        const int nb = (int)std::min<int64_t>(kTriB, n - k0);
        hipLaunchKernelGGL(tri_block_lower, dim3(1), dim3(64), 0, s, L, n, k0, nb, x);
        const int64_t rest = n - k0 - nb;
        if (rest > 0)
            hipLaunchKernelGGL(tri_update_lower, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0,
                               s, L, n, k0, nb, x);
    }
    for (int64_t b = nblk - 1; b >= 0; --b) {
        const int64_t k0 = b * kTriB;
        const int nb = (int)std::min<int64_t>(kTriB, n - k0);
        if (n - k0 - nb > 0)
            hipLaunchKernelGGL(tri_update_upper_t, dim3((unsigned)nb), dim3(256), 0, s, L, n, k0,
                               nb, x);
        hipLaunchKernelGGL(tri_block_upper_t, dim3(1), dim3(64), 0, s, L, n, k0, nb, x);
    }
    HIPCHECK(hipGetLastError());
}

}  // namespace bks
