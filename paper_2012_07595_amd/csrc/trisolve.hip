// Triangular solves with a Cholesky factor on the device: x <- (L L^T)^{-1} x
// for a lower factor L (N x N, column-major, leading dimension N), one
// right-hand side (the Newton step of the inner solve).  Forward: L y = x,
// then backward: L^T x = y.  Two forms:
//  - chol_solve_wg: one workgroup of 512 threads with x resident in LDS,
//    for small orders (one compute unit's bandwidth bounds it beyond a
//    thousand or so); per 64-row block one wave solves the
//    diagonal block (staged in LDS, unknowns in lanes, each solved value
//    broadcast by a lane read) and all threads update the rest of x from
//    the block's panel.  One launch for both solves, so no gaps between
//    kernels.
//  - chol_solve_dev: the same blocking over several launches, with
//    multi-workgroup panel passes, for the largest orders.
// Both can skip the forward solve (after a factorisation that substituted
// forward already).
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


// ---------------------------------------------------------------- one workgroup

constexpr int kWgB = 64;        // diagonal block
constexpr int kWgT = 512;       // threads (two waves per SIMD: 256 registers each)
constexpr int kWgHalf = kWgB / 2;  // columns per thread in the forward panel pass
constexpr int kWgCols = 8;      // threads per column in the backward panel pass
constexpr int kWgBatch = 32;    // rows per thread and backward pass

__device__ inline double lane_read(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Ld[c][r] = L(k0 + r, k0 + c) for r >= c, zero above the diagonal, identity
// outside the matrix (the last block may be short); dinv[c] = 1 / L(c, c).
__device__ void stage_diag(const double *__restrict__ L, int64_t N, int64_t k0, int nb,
                           double (*Ld)[kWgB + 1], double *dinv) {
    for (int idx = threadIdx.x; idx < kWgB * kWgB; idx += kWgT) {
        const int r = idx % kWgB, c = idx / kWgB;
        double v;
        if (r < nb && c < nb)
            v = r >= c ? L[(k0 + c) * N + k0 + r] : 0.0;
        else
            v = r == c ? 1.0 : 0.0;
        Ld[c][r] = v;
    }
    if (threadIdx.x < kWgB)
        dinv[threadIdx.x] =
            threadIdx.x < nb ? 1.0 / L[(k0 + threadIdx.x) * N + k0 + threadIdx.x] : 1.0;
}

// forward panel pass over kWgT rows: two threads per row, each with half of
// the block's columns, for the rows base + t/2 and base + kWgT/2 + t/2,
// loaded into registers in one batch.  Rows past the end read the last row
// instead (no branch per load) and their sums are dropped.
__device__ inline void fwd_load(const double *__restrict__ L, int64_t N, int64_t k0, int64_t base,
                                double (*v)[kWgHalf]) {
    const int h = threadIdx.x % 2;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        // each column's start is uniform and the row a 32-bit offset, so a
        // load needs no address register of its own
        const uint32_t r = (uint32_t)min(base + p * (kWgT / 2) + threadIdx.x / 2, N - 1);
#pragma unroll
        for (int c = 0; c < kWgHalf; ++c) {
            const double *__restrict__ colc = L + (k0 + h * kWgHalf + c) * N;
            v[p][c] = colc[r];
        }
    }
}

// xs[r] -= sum_c L(r, k0 + c) y_c for those rows; the pair of threads of a
// row adds its two halves by a lane exchange (the same sum in both lanes)
__device__ inline void fwd_apply(double *xs, int64_t N, int64_t k0, int64_t base,
                                 const double (*v)[kWgHalf]) {
    const int h = threadIdx.x % 2;
    const double *y = xs + k0 + h * kWgHalf;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int64_t r = base + p * (kWgT / 2) + threadIdx.x / 2;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < kWgHalf; ++c) s = fma(v[p][c], y[c], s);
        s += __shfl_xor(s, 1);
        if (h == 0 && r < N) xs[r] -= s;
    }
}

__global__ __launch_bounds__(512) void chol_solve_wg(const double *__restrict__ L, int64_t N,
                                                     double *__restrict__ x,
                                                     const int *__restrict__ info, int forward) {
    extern __shared__ double xs[];  // N
    __shared__ double Ld[kWgB][kWgB + 1];
    __shared__ double dinv[kWgB];
    if (*info != 0) return;
    const int tid = threadIdx.x;
    for (int64_t r = tid; r < N; r += kWgT) xs[r] = x[r];
    const int64_t nblk = (N + kWgB - 1) / kWgB;
    double v[2][kWgHalf];
    // forward: L y = x.  The first pass's panel entries are loaded before
    // the diagonal block is solved (they do not depend on it).  A block
    // with rows below it is a full one (nb = kWgB).
    for (int64_t b = 0; forward && b < nblk; ++b) {
        const int64_t k0 = b * kWgB;
        const int nb = (int)min((int64_t)kWgB, N - k0);
        __syncthreads();
        stage_diag(L, N, k0, nb, Ld, dinv);
        if (k0 + nb < N) fwd_load(L, N, k0, k0 + nb, v);
        __syncthreads();
        if (tid < 64) {
            // lane i holds unknown i; Ld's zero upper triangle leaves the
            // lanes already solved unchanged
            const int i = tid;
            double xi = i < nb ? xs[k0 + i] : 0.0;
#pragma unroll 8
            for (int j = 0; j < kWgB; ++j) {
                const double yj = lane_read(xi, j) * dinv[j];
                xi = i == j ? yj : fma(-Ld[j][i], yj, xi);
            }
            if (i < nb) xs[k0 + i] = xi;
        }
        __syncthreads();
        for (int64_t base = k0 + nb; base < N; base += kWgT) {
            if (base != k0 + nb) fwd_load(L, N, k0, base, v);
            fwd_apply(xs, N, k0, base, v);
        }
    }
    // backward: L^T x = y.  x_c -= sum_{r below the block} L(r, k0 + c) x_r:
    // kWgCols neighbouring threads per column, each with kWgBatch rows of a
    // pass in registers (rows past the end read the last row, weighted by
    // zero), then a butterfly over those threads (every lane ends with the
    // same sum)
    const int c = tid / kWgCols, q = tid % kWgCols;
    for (int64_t b = nblk - 1; b >= 0; --b) {
        const int64_t k0 = b * kWgB;
        const int nb = (int)min((int64_t)kWgB, N - k0);
        __syncthreads();
        stage_diag(L, N, k0, nb, Ld, dinv);
        double s = 0.0;
        if (c < nb) {
            const double *__restrict__ col = L + (k0 + c) * N;
            for (int64_t base = k0 + nb + q; base < N; base += (int64_t)kWgCols * kWgBatch) {
                double w[kWgBatch];
                if (base + (int64_t)kWgCols * (kWgBatch - 1) < N) {
                    // a full batch: one address, constant offsets
                    const double *__restrict__ p = col + base;
#pragma unroll
                    for (int m = 0; m < kWgBatch; ++m) w[m] = p[kWgCols * m];
#pragma unroll
                    for (int m = 0; m < kWgBatch; ++m) s = fma(w[m], xs[base + kWgCols * m], s);
                } else {
#pragma unroll
                    for (int m = 0; m < kWgBatch; ++m) w[m] = col[min(base + kWgCols * m, N - 1)];
#pragma unroll
                    for (int m = 0; m < kWgBatch; ++m) {
                        const int64_t r = base + kWgCols * m;
                        s = fma(w[m], r < N ? xs[r] : 0.0, s);
                    }
                }
            }
        }
#pragma unroll
        for (int w = kWgCols / 2; w > 0; w >>= 1) s += __shfl_xor(s, w);
        __syncthreads();
        if (q == 0 && c < nb) xs[k0 + c] -= s;
        __syncthreads();
        if (tid < 64) {
            // (L^T)(i, j) = L(j, i) = Ld[i][j], zero for i > j
            const int i = tid;
            double xi = i < nb ? xs[k0 + i] : 0.0;
#pragma unroll 8
            for (int j = kWgB - 1; j >= 0; --j) {
                const double yj = lane_read(xi, j) * dinv[j];
                xi = i == j ? yj : fma(-Ld[i][j], yj, xi);
            }
            if (i < nb) xs[k0 + i] = xi;
        }
    }
    __syncthreads();
    for (int64_t r = tid; r < N; r += kWgT) x[r] = xs[r];
}

}  // namespace

void chol_solve_dev(hipStream_t s, const double *L, int N, double *x, bool forward) {
    const int64_t n = N;
    const int64_t nblk = (n + kTriB - 1) / kTriB;
    for (int64_t b = 0; forward && b < nblk; ++b) {
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

void chol_solve_small(hipStream_t s, const double *L, int N, double *x, const int *info,
                      bool forward) {
    if (N < 1 || N > kSolveWgLimit) fail(BKS_EINVAL, "chol_solve_small: order out of range");
    hipLaunchKernelGGL(chol_solve_wg, dim3(1), dim3(kWgT), (size_t)N * sizeof(double), s, L,
                       (int64_t)N, x, info, forward ? 1 : 0);
    HIPCHECK(hipGetLastError());
}

}  // namespace bks
