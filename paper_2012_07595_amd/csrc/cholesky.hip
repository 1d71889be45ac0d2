// Cholesky factorisation A = L L^T on the device for the Newton systems of
// the inner solve up to order kSmallCholMax (rocSOLVER's potrf is slower
// there: its small kernels are launch-bound).  Right-looking in 32-column
// blocks with two launches per block column:
//   chol_panel   every workgroup factors the 32 x 32 diagonal block itself
//                (one wave, a row per lane in registers, pivots broadcast
//                by lane shuffles), then solves its 256 rows of the panel,
//                x L_kk^T = a (a row per thread, in registers); workgroup 0
//                also writes the diagonal block back;
//   chol_update  the trailing lower triangle -= P P^T in 32 x 32 tiles.
// A is column-major with leading dimension N (the symmetric Newton matrix,
// whose row-major layout reads the same); only its lower triangle is read
// and L overwrites it.  A non-positive (or NaN) pivot stops the
// factorisation: its 1-based index goes to *info and every later kernel
// returns at once.  Every sum has a fixed order, and the diagonal block is
// factored by the same code in every workgroup, so all of them use the same
// L_kk.
#include <algorithm>

#include "bks_internal.h"

namespace bks {

namespace {

constexpr int kCB = 32;  // block columns (= trailing-update tile)

__global__ __launch_bounds__(256) void chol_panel(double *__restrict__ A, int64_t N, int64_t k0,
                                                  int nb, int *__restrict__ info) {
    __shared__ double Lk[kCB][kCB + 1];
    __shared__ int bad;
    if (*info != 0) return;
    const int tid = threadIdx.x;
    if (tid < 64) {
        // wave 0: lane i < nb holds row i of the diagonal block
        const int i = tid;
        double row[kCB];
#pragma unroll
        for (int j = 0; j < kCB; ++j)
            row[j] = (i < nb && j <= i) ? A[(k0 + j) * N + k0 + i] : (i == j ? 1.0 : 0.0);
        // no branches on the pivot inside the unrolled loop: a bad pivot is
        // recorded and the (then meaningless) arithmetic runs on; columns
        // past nb are identity rows and leave the block unchanged
        int fail = 0;
#pragma unroll
        for (int j = 0; j < kCB; ++j) {
            const double p = __shfl(row[j], j);
            fail = (fail == 0 && j < nb && !(p > 0.0)) ? j + 1 : fail;
            const double d = sqrt(p);
            row[j] = i == j ? d : (i > j ? row[j] / d : row[j]);
#pragma unroll
            for (int l = j + 1; l < kCB; ++l) {
                const double c = __shfl(row[j], l);  // L(l, j)
                row[l] = i >= l ? row[l] - row[j] * c : row[l];
            }
        }
        if (i < kCB) {
#pragma unroll
            for (int j = 0; j < kCB; ++j) Lk[i][j] = row[j];
        }
        if (i == 0) bad = fail;
    }
    __syncthreads();
    if (bad != 0) {
        if (blockIdx.x == 0 && tid == 0) *info = (int)(k0 + bad);
        return;
    }
    if (blockIdx.x == 0) {
        for (int idx = tid; idx < nb * nb; idx += 256) {
            const int i = idx % nb, j = idx / nb;
            if (i >= j) A[(k0 + j) * N + k0 + i] = Lk[i][j];
        }
    }
    // panel rows exist only below a full block (nb = kCB): a block with
    // nb < kCB is the last one and has none
    const int64_t r = k0 + nb + (int64_t)blockIdx.x * 256 + tid;
    if (r >= N || nb != kCB) return;
    double x[kCB];
#pragma unroll
    for (int j = 0; j < kCB; ++j) x[j] = A[(k0 + j) * N + r];
#pragma unroll
    for (int j = 0; j < kCB; ++j) {
        double v = x[j];
#pragma unroll
        for (int l = 0; l < j; ++l) v -= x[l] * Lk[j][l];
        x[j] = v / Lk[j][j];
    }
#pragma unroll
    for (int j = 0; j < kCB; ++j) A[(k0 + j) * N + r] = x[j];
}

// trailing lower triangle: A[i, j] -= sum_l A[i, k0 + l] A[j, k0 + l] for
// j0 <= j <= i < N, j0 = k0 + nb; one 32 x 32 tile (ti >= tj) per workgroup
__global__ __launch_bounds__(256) void chol_update(double *__restrict__ A, int64_t N, int64_t k0,
                                                   int nb, const int *__restrict__ info) {
    __shared__ double Pi[kCB][kCB + 1], Pj[kCB][kCB + 1];
    if (*info != 0) return;
    const int64_t b = blockIdx.x;
    int64_t ti = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > b) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    const int64_t tj = b - ti * (ti + 1) / 2;
    const int64_t j0 = k0 + nb;
    const int64_t i0 = j0 + ti * kCB, c0 = j0 + tj * kCB;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < kCB * kCB; idx += 256) {
        const int rr = idx % kCB, l = idx / kCB;
        const int64_t ri = i0 + rr, rj = c0 + rr;
        Pi[l][rr] = (l < nb && ri < N) ? A[(k0 + l) * N + ri] : 0.0;
        Pj[l][rr] = (l < nb && rj < N) ? A[(k0 + l) * N + rj] : 0.0;
    }
    __syncthreads();
    const int ty = tid / 16, tx = tid % 16;  // 2 x 2 outputs per thread
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int l = 0; l < nb; ++l) {
        const double a0 = Pi[l][2 * ty], a1 = Pi[l][2 * ty + 1];
        const double b0 = Pj[l][2 * tx], b1 = Pj[l][2 * tx + 1];
        acc[0][0] = fma(a0, b0, acc[0][0]);
        acc[0][1] = fma(a0, b1, acc[0][1]);
        acc[1][0] = fma(a1, b0, acc[1][0]);
        acc[1][1] = fma(a1, b1, acc[1][1]);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int64_t i = i0 + 2 * ty + u, j = c0 + 2 * tx + v;
            if (i < N && j < N && i >= j) A[j * N + i] -= acc[u][v];
        }
}

__global__ void clear_info(int *info) { *info = 0; }

}  // namespace

void chol_factor_dev(hipStream_t s, double *A, int N, int *info) {
    const int64_t n = N;
    hipLaunchKernelGGL(clear_info, dim3(1), dim3(1), 0, s, info);
    for (int64_t k0 = 0; k0 < n; k0 += kCB) {
        const int nb = (int)std::min<int64_t>(kCB, n - k0);
        const int64_t rest = n - k0 - nb;
        hipLaunchKernelGGL(chol_panel, dim3((unsigned)std::max<int64_t>(1, (rest + 255) / 256)),
                           dim3(256), 0, s, A, n, k0, nb, info);
        if (rest <= 0) continue;
        const int64_t T = (rest + kCB - 1) / kCB;
        hipLaunchKernelGGL(chol_update, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, s, A, n,
                           k0, nb, info);
    }
    HIPCHECK(hipGetLastError());
}

}  // namespace bks
