// Cholesky factorisation A = L L^T on the device for the Newton systems of
// the inner solve up to order kSmallCholMax (rocSOLVER's potrf is slower
// at every order measured, 256 to 17000: its small kernels are launch-bound
// at small orders, its panel work at large ones).  Right-looking in 32-column
// blocks with one launch per block column (chol_step): the panel of block
// column k, into which the update by panel k-1 is folded, and, in other
// workgroups of the same launch, the update by panel k-1 of the trailing
// columns beyond block k (in a launch of its own, chol_trail, where those
// tiles are too many for one round of the compute units).  From order
// kHybridMin the blocks are grouped in panels of kPanel columns: the steps
// update only the panel's columns and one rank-kPanel dsyrk (rocBLAS)
// updates the rest of the matrix after each panel.  A is column-major with
// leading dimension N (the symmetric Newton matrix, whose row-major layout
// reads the same); only its lower triangle is read and L overwrites it.
// Given a right-hand side b, the forward substitution L y = b rides along:
// step k solves block k of y with L_kk and subtracts its terms from the
// rows below, so b holds y at the end.  A non-positive (or NaN) pivot
// stops the factorisation: its 1-based index goes to *info and every later
// kernel returns at once.  Every sum has a fixed order, and the diagonal
// block is factored by the same code in every workgroup, so all of them
// use the same L_kk.
#include <algorithm>

#include <rocblas/rocblas.h>

#include "bks_internal.h"

namespace bks {

namespace {

constexpr int kCB = 32;  // block columns (= trailing-update tile)
static_assert(kCholWork == kCB * kCB + kCB, "a diagonal block and its unknowns");

// lane `l` (the same for every lane) of a wave's double
__device__ inline double lane_read(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// 1 / sqrt(p) for p > 0: the hardware estimate and two Newton steps
// y <- y + y (1 - p y^2) / 2 (each about doubles the correct bits; the
// result is within an ulp or two, which the factorisation's backward
// stability does not notice)
__device__ inline double rsqrt_nr(double p) {
    double y = __builtin_amdgcn_rsq(p);
#pragma unroll
    for (int k = 0; k < 2; ++k) y = fma(0.5 * y, fma(-p * y, y, 1.0), y);
    return y;
}

constexpr int kRowsPerWg = 192;  // panel rows per workgroup (waves 1-3)
constexpr int kFuseMaxWg = 512;  // one fused step's workgroups: two per compute unit
constexpr int64_t kPanel = 256;     // panel width of the large-order form
constexpr int64_t kHybridMin = 8192;  // orders from which it is used

// A block column's panel with the previous panel's update folded in (the
// workgroups of one launch below the panel count): the diagonal block
// D = A_kk - P_k-1,k P_k-1,k^T is formed in LDS by all threads and
// factored by wave 0 (a row per lane in registers, column entries
// broadcast by lane reads, pivots from a refined reciprocal square root);
// waves 1-3 meanwhile subtract the previous panel from their rows of the
// block column (loaded at the start), then solve x L_kk^T = a (a row per
// thread, right-looking, times the pivots' reciprocals).  Workgroup 0 writes the diagonal
// block's factor L_kk and the block's forward-substituted unknowns: in place
// when it is the step's only panel workgroup (`direct`), else to `work`,
// since the other panel workgroups read A_kk and b_k at their own start,
// which may come after workgroup 0 has finished (nothing orders workgroups
// of one launch); the next step's workgroup 0 moves them into place.
__device__ __forceinline__ void panel_part(double *__restrict__ A, int64_t N, int64_t k0, int nb,
                                           int64_t p, bool fold, bool direct,
                                           double *__restrict__ bvec, double *__restrict__ work,
                                           int *__restrict__ info, double (*Lp)[kCB + 1],
                                           double (*Lk)[kCB + 1], double *rd, double *yb,
                                           int *bad) {
    const int tid = threadIdx.x;
    // the previous block column's panel to apply (not when a panel's first
    // step follows the rank-kPanel update of the whole trailing matrix)
    const bool fuse = fold && k0 > 0;
    const int64_t kp = k0 - kCB;
    // this thread's panel row.  Panel rows exist only below a full block
    // (nb = kCB): a block with nb < kCB is the last one and has none.
    const int64_t r = k0 + nb + p * kRowsPerWg + (tid - 64);
    const bool has_row = tid >= 64 && r < N && nb == kCB;
    const bool solve_b = bvec != nullptr;
    double x[kCB], xp[kCB];
    double bv = 0.0;  // b at this thread's panel row, or (wave 0) at row k0 + tid of the block
    if (solve_b && (has_row || (tid < nb)))
        bv = bvec[has_row ? r : k0 + tid];
    if (has_row) {
#pragma unroll
        for (int j = 0; j < kCB; ++j) x[j] = A[(k0 + j) * N + r];
        if (fuse) {
#pragma unroll
            for (int l = 0; l < kCB; ++l) xp[l] = A[(kp + l) * N + r];
        }
    }
    // the diagonal block's entries this thread forms (idx = tid + 256 m)
    double dk[kCB * kCB / 256];
#pragma unroll
    for (int m = 0; m < kCB * kCB / 256; ++m) {
        const int idx = tid + 256 * m, i = idx % kCB, j = idx / kCB;
        dk[m] = (i < nb && j <= i) ? A[(k0 + j) * N + k0 + i] : 0.0;
    }
    if (fuse) {
        for (int idx = tid; idx < kCB * kCB; idx += 256) {
            const int i = idx % kCB, l = idx / kCB;
            Lp[i][l] = i < nb ? A[(kp + l) * N + k0 + i] : 0.0;
        }
    }
    __syncthreads();
    // D into Lk (lower triangle; wave 0 reads it before it writes L_kk there)
#pragma unroll
    for (int m = 0; m < kCB * kCB / 256; ++m) {
        const int idx = tid + 256 * m, i = idx % kCB, j = idx / kCB;
        double v = dk[m];
        if (fuse && i < nb && j <= i) {
#pragma unroll 8
            for (int l = 0; l < kCB; ++l) v = fma(-Lp[i][l], Lp[j][l], v);
        }
        Lk[i][j] = v;
    }
    __syncthreads();
    if (tid < 64) {
        // lane i < nb holds row i of D, lanes nb <= i < kCB an identity
        // row (they leave the block unchanged)
        const int i = tid;
        double row[kCB];
#pragma unroll
        for (int j = 0; j < kCB; ++j)
            row[j] = (i < nb && j <= i) ? Lk[i][j] : (i == j ? 1.0 : 0.0);
        // Step j takes the pivot from lane j and column j's entries from
        // lanes l > j; those are lower-triangle values.  The updates run on
        // every lane without a mask, so a lane's entries right of its
        // diagonal turn to garbage, which no lane ever reads.  No branches
        // on the pivot inside the unrolled loop: a bad one is recorded and
        // the (then meaningless) arithmetic runs on.
        int fail = 0;
        double myrd = 1.0;
#pragma unroll
        for (int j = 0; j < kCB; ++j) {
            const double pv = lane_read(row[j], j);
            fail = (fail == 0 && j < nb && !(pv > 0.0)) ? j + 1 : fail;
            const double rj = rsqrt_nr(pv);
            row[j] = i == j ? pv * rj : row[j] * rj;
            myrd = i == j ? rj : myrd;
#pragma unroll
            for (int l = j + 1; l < kCB; ++l) row[l] = fma(-row[j], lane_read(row[j], l), row[l]);
        }
        if (i < kCB) {
#pragma unroll
            for (int j = 0; j < kCB; ++j) Lk[i][j] = row[j];
            rd[i] = myrd;
        }
        if (i == 0) *bad = fail;
    } else if (has_row && fuse) {
        // x_j -= sum_l xp_l Lp[j][l], term by term over l (32 independent
        // updates per term)
#pragma unroll
        for (int l = 0; l < kCB; ++l) {
#pragma unroll
            for (int j = 0; j < kCB; ++j) x[j] = fma(-xp[l], Lp[j][l], x[j]);
        }
    }
    __syncthreads();
    if (*bad != 0) {
        if (p == 0 && tid == 0) *info = (int)(k0 + *bad);
        return;
    }
    if (p == 0) {
        for (int idx = tid; idx < nb * nb; idx += 256) {
            const int i = idx % nb, j = idx / nb;
            if (i < j) continue;
            if (direct)
                A[(k0 + j) * N + k0 + i] = Lk[i][j];
            else
                work[j * kCB + i] = Lk[i][j];
        }
    }
    if (tid < 64) {
        if (solve_b) {
            // forward substitution of the block: y = L_kk^{-1} b_k, b_k final
            // (every earlier step has subtracted its terms); lane i holds
            // unknown i, lanes past nb hold zero
            const int i = tid, ic = min(i, kCB - 1);
            double yi = i < nb ? bv : 0.0;
#pragma unroll
            for (int j = 0; j < kCB; ++j) {
                const double yj = lane_read(yi, j) * rd[j];
                yi = i == j ? yj : ((i > j && i < nb) ? fma(-Lk[ic][j], yj, yi) : yi);
            }
            if (i < kCB) yb[i] = yi;
            if (p == 0 && i < nb) {
                if (direct)
                    bvec[k0 + i] = yi;
                else
                    work[kCB * kCB + i] = yi;
            }
        }
    } else if (has_row) {
        // right-looking: once x_j is final, its terms leave the later
        // unknowns (independent updates, where a per-unknown sum is one
        // dependent chain)
#pragma unroll
        for (int j = 0; j < kCB; ++j) {
            x[j] *= rd[j];
#pragma unroll
            for (int l = j + 1; l < kCB; ++l) x[l] = fma(-x[j], Lk[l][j], x[l]);
        }
#pragma unroll
        for (int j = 0; j < kCB; ++j) A[(k0 + j) * N + r] = x[j];
    }
    if (solve_b) {
        // the block's solved unknowns leave the rows below: b_r -= L(r, k) y
        __syncthreads();
        if (has_row) {
            double sb = bv;
#pragma unroll
            for (int j = 0; j < kCB; ++j) sb = fma(-x[j], yb[j], sb);
            bvec[r] = sb;
        }
    }
}

// One 32 x 32 tile of the trailing update with the panel of block column
// kp: A[i, j] -= sum_l A[i, kp + l] A[j, kp + l] for j0 <= j <= i < N, j in
// the first cp tile columns: tiles (ti >= tj, tj < cp) numbered by rows of
// the triangle while ti < cp (b = ti (ti + 1) / 2 + tj), then cp per row.
__device__ __forceinline__ void update_tile(double *__restrict__ A, int64_t N, int64_t kp, int64_t j0,
                                            int64_t b, int64_t cp, double (*Pi)[kCB + 1],
                                            double (*Pj)[kCB + 1]) {
    int64_t ti, tj;
    const int64_t tri = cp * (cp + 1) / 2;
    if (b < tri) {
        ti = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
        while (ti * (ti + 1) / 2 > b) --ti;
        while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
        tj = b - ti * (ti + 1) / 2;
    } else {
        ti = cp + (b - tri) / cp;
        tj = (b - tri) % cp;
    }
    const int64_t i0 = j0 + ti * kCB, c0 = j0 + tj * kCB;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < kCB * kCB; idx += 256) {
        const int rr = idx % kCB, l = idx / kCB;
        const int64_t ri = i0 + rr, rj = c0 + rr;
        Pi[l][rr] = ri < N ? A[(kp + l) * N + ri] : 0.0;
        Pj[l][rr] = rj < N ? A[(kp + l) * N + rj] : 0.0;
    }
    __syncthreads();
    const int ty = tid / 16, tx = tid % 16;  // 2 x 2 outputs per thread
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    // partly unrolled: fully unrolled, the LDS reads of all 32 steps are
    // hoisted and take every register
#pragma unroll 4
    for (int l = 0; l < kCB; ++l) {
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

// Step k of the factorisation (k0 = 32 k): workgroups [0, gp) factor block
// column k with panel k-1 folded in (panel_part); the rest apply panel k-1
// to the trailing columns beyond block k (update_tile), which panel k does
// not touch.  Every column thus receives every earlier panel's update before
// its own step.  kflush >= 0: the full diagonal block at kflush (an earlier
// step's) and its unknowns wait in `work`; workgroup 0 moves them into place
// before it does anything else (no workgroup of this launch reads either).
__global__ __launch_bounds__(256) void chol_step(double *__restrict__ A, int64_t N, int64_t k0,
                                                 int nb, int64_t gp, int fold, int64_t cp,
                                                 int64_t kflush, double *__restrict__ bvec,
                                                 double *__restrict__ work,
                                                 int *__restrict__ info) {
    __shared__ double sm[2][kCB][kCB + 1];
    __shared__ double rd[kCB];  // 1 / L(j, j)
    __shared__ double yb[kCB];  // the block's forward-substituted unknowns
    __shared__ int bad;
    if (*info != 0) return;
    const int64_t w = blockIdx.x;
    if (w == 0 && kflush >= 0) {
        for (int idx = threadIdx.x; idx < kCB * kCB; idx += 256) {
            const int i = idx % kCB, j = idx / kCB;
            if (i >= j) A[(kflush + j) * N + kflush + i] = work[idx];
        }
        if (bvec != nullptr && threadIdx.x < kCB)
            bvec[kflush + threadIdx.x] = work[kCB * kCB + threadIdx.x];
    }
    if (w < gp)
        panel_part(A, N, k0, nb, w, fold != 0, gp == 1, bvec, work, info, sm[0], sm[1], rd, yb,
                   &bad);
    else
        update_tile(A, N, k0 - kCB, k0 + nb, w - gp, cp, sm[0], sm[1]);
}

// The trailing update alone (the tiles of a step too many for one round of
// the fused kernel, whose register use allows two workgroups per compute
// unit)
__global__ __launch_bounds__(256) void chol_trail(double *__restrict__ A, int64_t N, int64_t kp,
                                                  int64_t j0, int64_t cp,
                                                  const int *__restrict__ info) {
    __shared__ double sm[2][kCB][kCB + 1];
    if (*info != 0) return;
    update_tile(A, N, kp, j0, blockIdx.x, cp, sm[0], sm[1]);
}

__global__ void clear_info(int *info) { *info = 0; }

// dst = src + mu I (N x N, leading dimension N): columns over grid.y,
// rows over threads
__global__ __launch_bounds__(256) void shift_copy(double *__restrict__ dst,
                                                  const double *__restrict__ src, int64_t N,
                                                  double mu) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    for (int64_t j = blockIdx.y; j < N; j += gridDim.y) {
        const int64_t e = j * N + i;
        dst[e] = i == j ? src[e] + mu : src[e];
    }
}

}  // namespace

void chol_factor_dev(hipStream_t s, double *A, int N, int *info, double *b, double *work,
                     void *blas) {
    const int64_t n = N;
    if (work == nullptr) fail(BKS_EINVAL, "chol_factor_dev: no workspace");
    // large orders: panels of kPanel columns factored by the steps below
    // (their trailing tiles restricted to the panel's columns), each followed
    // by one rank-kPanel update of the rest of the matrix on rocBLAS (dsyrk)
    const int64_t panel = (blas && n >= kHybridMin) ? kPanel : n;
    hipLaunchKernelGGL(clear_info, dim3(1), dim3(1), 0, s, info);
    // the block whose factor and unknowns wait in `work` (a step with more
    // than one panel workgroup leaves them there), or -1.  The last step has
    // no rows below its block, hence one panel workgroup: nothing is left.
    int64_t pending = -1;
    for (int64_t p0 = 0; p0 < n; p0 += panel) {
        const int64_t p1 = std::min(n, p0 + panel);
        for (int64_t k0 = p0; k0 < p1; k0 += kCB) {
            const int nb = (int)std::min<int64_t>(kCB, n - k0);
            const int64_t rest = n - k0 - nb;
            const int64_t gp = std::max<int64_t>(1, (rest + kRowsPerWg - 1) / kRowsPerWg);
            // panel k-1 folded into block column k, and its update of the
            // columns beyond block k within this panel: in the same launch
            // while the whole grid fits one round of the compute units, else
            // in a launch of their own.  A panel's first step has neither
            // (the rank-kPanel update covered them).
            const bool fold = k0 > p0;
            const int64_t T = fold ? (rest + kCB - 1) / kCB : 0;
            const int64_t cp = std::min<int64_t>(T, (p1 - k0 - nb + kCB - 1) / kCB);
            const int64_t tiles = cp * (cp + 1) / 2 + (T - cp) * cp;
            const bool fused = gp + tiles <= kFuseMaxWg;
            hipLaunchKernelGGL(chol_step, dim3((unsigned)(gp + (fused ? tiles : 0))), dim3(256), 0,
                               s, A, n, k0, nb, gp, fold ? 1 : 0, cp, pending, b, work, info);
            pending = gp == 1 ? -1 : k0;
            if (!fused && tiles > 0)
                hipLaunchKernelGGL(chol_trail, dim3((unsigned)tiles), dim3(256), 0, s, A, n,
                                   k0 - kCB, k0 + nb, cp, info);
        }
        if (p1 < n) {
            const double alpha = -1.0, beta = 1.0;
            if (rocblas_dsyrk(static_cast<rocblas_handle>(blas), rocblas_fill_lower,
                              rocblas_operation_none, (rocblas_int)(n - p1), (rocblas_int)(p1 - p0),
                              &alpha, A + p0 * n + p1, (rocblas_int)n, &beta, A + p1 * n + p1,
                              (rocblas_int)n) != rocblas_status_success)
                fail(BKS_EDEVICE, "rocblas_dsyrk");
        }
    }
    HIPCHECK(hipGetLastError());
}

void shift_copy_dev(hipStream_t s, double *dst, const double *src, int N, double mu) {
    const int64_t n = N;
    hipLaunchKernelGGL(shift_copy, dim3((unsigned)((n + 255) / 256), (unsigned)std::min<int64_t>(n, 4096)),
                       dim3(256), 0, s, dst, src, n, mu);
    HIPCHECK(hipGetLastError());
}

}  // namespace bks
