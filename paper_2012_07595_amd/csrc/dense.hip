// Dense tall-skinny kernels for the block orthogonalisation (Algorithm 3
// steps (ii)-(iv), Appendix B), core formation (eq. tkd) and restart
// (eq. tks1).  All accumulate in FP64; these products are HBM-bound
// (one pass over the tall operand per call), so they use vector FP64 FMA
// rather than matrix cores.
//
// gram_dd forms B^T B in double-double (a compensated product/sum per term):
// the in-block part of the orthogonalisation must resolve directions that
// are ~1e-12 of the block's norm (the G-gradient near convergence, Proposition
// 3.2), which an FP64 Gram matrix (error ~1e-16 of its largest entry) cannot.
#include <algorithm>

#include "bks_internal.h"

namespace bks {

namespace {

// ------------------------------------------------------------- gemm_tn
constexpr int TN_T = 32;   // output tile (k x q)
constexpr int TN_R = 32;   // rows staged per step

template <typename TB>
__global__ __launch_bounds__(256) void gemm_tn_kernel(const double *__restrict__ A, int64_t lda,
                                                      const TB *__restrict__ B, int64_t ldb,
                                                      int64_t rows, int k, int q,
                                                      int64_t rows_per_split,
                                                      double *__restrict__ part, int ntk,
                                                      int ntq) {
    __shared__ double As[TN_R][TN_T + 1];
    __shared__ double Bs[TN_R][TN_T + 1];
    const int tile = blockIdx.x;
    const int tk = tile % ntk, tq = tile / ntk;
    const int split = blockIdx.y;
    const int64_t r0 = (int64_t)split * rows_per_split;
    const int64_t r1 = min(rows, r0 + rows_per_split);
    const int tid = threadIdx.x;
    const int ty = tid / 16, tx = tid % 16;  // 2x2 outputs per thread
    double acc[2][2] = {{0, 0}, {0, 0}};
    for (int64_t rb = r0; rb < r1; rb += TN_R) {
        for (int x = tid; x < TN_R * TN_T; x += 256) {
            const int rr = x / TN_T, cc = x % TN_T;
            const int64_t row = rb + rr;
            const int ka = tk * TN_T + cc, qb = tq * TN_T + cc;
            As[rr][cc] = (row < r1 && ka < k) ? A[row * lda + ka] : 0.0;
            Bs[rr][cc] = (row < r1 && qb < q) ? (double)B[row * ldb + qb] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int rr = 0; rr < TN_R; ++rr) {
            const double a0 = As[rr][ty * 2], a1 = As[rr][ty * 2 + 1];
            const double b0 = Bs[rr][tx * 2], b1 = Bs[rr][tx * 2 + 1];
            acc[0][0] = fma(a0, b0, acc[0][0]);
            acc[0][1] = fma(a0, b1, acc[0][1]);
            acc[1][0] = fma(a1, b0, acc[1][0]);
            acc[1][1] = fma(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int kk = tk * TN_T + ty * 2 + a, qq = tq * TN_T + tx * 2 + b;
            if (kk < k && qq < q) part[((int64_t)split * k + kk) * q + qq] = acc[a][b];
        }
}

__global__ void reduce_splits(const double *__restrict__ part, int nsplit, int k, int q,
                              double *__restrict__ out, int64_t ldo) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)k * q) return;
    const int kk = (int)(idx / q), qq = (int)(idx % q);
    double s = 0.0;
    for (int x = 0; x < nsplit; ++x) s += part[((int64_t)x * k + kk) * q + qq];
    out[(int64_t)kk * ldo + qq] = s;
}

// Many splits: one 256-thread block per output, strided partial sums and a
// fixed-order tree in LDS (deterministic).
__global__ __launch_bounds__(256) void reduce_splits_wide(const double *__restrict__ part,
                                                          int nsplit, int k, int q,
                                                          double *__restrict__ out, int64_t ldo) {
    __shared__ double red[256];
    const int64_t o = blockIdx.x;
    const int kk = (int)(o / q), qq = (int)(o % q);
    double s = 0.0;
    for (int x = threadIdx.x; x < nsplit; x += 256) s += part[((int64_t)x * k + kk) * q + qq];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)kk * ldo + qq] = red[0];
}

// A^T B for k <= 256 and q <= 64 (the basis against a block of at most 64
// columns): one block holds the whole k x q product of its row range, so
// every row of A and B is read once (the 32 x 32 tiling above reads A once
// per column tile of B and B once per row tile of A).  Thread (ty, tx) owns
// outputs (ty + 16 i, tx + 16 j), i < KI, j < 4; rows are staged 16 at a
// time.
constexpr int TR_ROWS = 16;
constexpr int TR_KMAX = 256, TR_QMAX = 64;

template <typename TB, int KI>
__global__ __launch_bounds__(256) void gemm_tn_rows_kernel(const double *__restrict__ A,
                                                           int64_t lda, const TB *__restrict__ B,
                                                           int64_t ldb, int64_t rows, int k,
                                                           int q, int64_t rows_per_split,
                                                           double *__restrict__ part) {
    __shared__ double As[TR_ROWS][16 * KI + 1];
    __shared__ double Bs[TR_ROWS][TR_QMAX + 1];
    const int split = blockIdx.x;
    const int64_t r0 = (int64_t)split * rows_per_split;
    const int64_t r1 = min(rows, r0 + rows_per_split);
    const int tid = threadIdx.x;
    const int ty = tid / 16, tx = tid % 16;
    double acc[KI][4];
#pragma unroll
    for (int i = 0; i < KI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int64_t rb = r0; rb < r1; rb += TR_ROWS) {
        const int nr = (int)min<int64_t>(TR_ROWS, r1 - rb);
        for (int x = tid; x < TR_ROWS * k; x += 256) {
            const int rr = x / k, cc = x - (x / k) * k;
            As[rr][cc] = rr < nr ? A[(rb + rr) * lda + cc] : 0.0;
        }
        for (int x = tid; x < TR_ROWS * q; x += 256) {
            const int rr = x / q, cc = x - (x / q) * q;
            Bs[rr][cc] = rr < nr ? (double)B[(rb + rr) * ldb + cc] : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < nr; ++rr) {
            double a[KI], b[4];
#pragma unroll
            for (int i = 0; i < KI; ++i) a[i] = ty + 16 * i < k ? As[rr][ty + 16 * i] : 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = tx + 16 * j < q ? Bs[rr][tx + 16 * j] : 0.0;
#pragma unroll
            for (int i = 0; i < KI; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < KI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int kk = ty + 16 * i, qq = tx + 16 * j;
            if (kk < k && qq < q) part[((int64_t)split * k + kk) * q + qq] = acc[i][j];
        }
}

template <typename TB, int KI>
void launch_tn_rows(int64_t nsplit, const double *A, int64_t lda, const TB *B, int64_t ldb,
                    int64_t rows, int k, int q, int64_t rps, double *part, hipStream_t s) {
    hipLaunchKernelGGL((gemm_tn_rows_kernel<TB, KI>), dim3((unsigned)nsplit), dim3(256), 0, s, A,
                       lda, B, ldb, rows, k, q, rps, part);
}

void launch_reduce(const double *part, int nsplit, int k, int q, double *out, int64_t ldo,
                   hipStream_t s) {
    const int64_t n = (int64_t)k * q;
    if (nsplit > 32 && n <= 65536)
        hipLaunchKernelGGL(reduce_splits_wide, dim3((unsigned)n), dim3(256), 0, s, part, nsplit, k,
                           q, out, ldo);
    else
        hipLaunchKernelGGL(reduce_splits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part,
                           nsplit, k, q, out, ldo);
}

template <typename TB>
void gemm_tn_impl(const double *A, int64_t lda, const TB *B, int64_t ldb, int64_t rows, int k,
                  int q, double *out, int64_t ldo, Ctx &c, hipStream_t s) {
    if (k <= 0 || q <= 0) return;
    if (rows > 0 && k <= TR_KMAX && q <= TR_QMAX) {
        // ~64 rows per block (fewer blocks only for short operands)
        int64_t nsplit = std::min<int64_t>(1024, std::max<int64_t>(1, rows / 64));
        const int64_t rps = (rows + nsplit - 1) / nsplit;
        nsplit = (rows + rps - 1) / rps;
        c.ws_pack2.ensure((size_t)nsplit * k * q * sizeof(double));
        double *part = c.ws_pack2.as<double>();
        if (k <= 32)
            launch_tn_rows<TB, 2>(nsplit, A, lda, B, ldb, rows, k, q, rps, part, s);
        else if (k <= 64)
            launch_tn_rows<TB, 4>(nsplit, A, lda, B, ldb, rows, k, q, rps, part, s);
        else if (k <= 128)
            launch_tn_rows<TB, 8>(nsplit, A, lda, B, ldb, rows, k, q, rps, part, s);
        else
            launch_tn_rows<TB, 16>(nsplit, A, lda, B, ldb, rows, k, q, rps, part, s);
        launch_reduce(part, (int)nsplit, k, q, out, ldo, s);
        HIPCHECK(hipGetLastError());
        return;
    }
    const int ntk = (k + TN_T - 1) / TN_T, ntq = (q + TN_T - 1) / TN_T;
    const int tiles = ntk * ntq;
    int64_t nsplit = std::max<int64_t>(1, 2048 / tiles);
    nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, rows / 128));
    int64_t rps = (rows + nsplit - 1) / nsplit;
    rps = std::max<int64_t>(rps, 1);
    nsplit = (rows + rps - 1) / rps;
    if (nsplit < 1) nsplit = 1;
    const size_t need = (size_t)nsplit * k * q * sizeof(double);
    c.ws_pack2.ensure(need);
    double *part = c.ws_pack2.as<double>();
    if (rows == 0) {
        HIPCHECK(hipMemsetAsync(part, 0, (size_t)k * q * sizeof(double), s));
        nsplit = 1;
    } else {
        hipLaunchKernelGGL(gemm_tn_kernel<TB>, dim3(tiles, (unsigned)nsplit), dim3(256), 0, s, A,
                           lda, B, ldb, rows, k, q, rps, part, ntk, ntq);
    }
    launch_reduce(part, (int)nsplit, k, q, out, ldo, s);
    HIPCHECK(hipGetLastError());
}

// ------------------------------------------------------------- gemm_nn
constexpr int NN_R = 64, NN_Q = 16, NN_K = 32;

__global__ __launch_bounds__(256) void gemm_nn_kernel(const double *__restrict__ A, int64_t lda,
                                                      const double *__restrict__ H, int64_t ldh,
                                                      int64_t rows, int k, int q, double alpha,
                                                      double beta, double *__restrict__ C,
                                                      int64_t ldc) {
    __shared__ double As[NN_R][NN_K + 1];
    __shared__ double Hs[NN_K][NN_Q];
    const int64_t r0 = (int64_t)blockIdx.x * NN_R;
    const int q0 = blockIdx.y * NN_Q;
    const int tid = threadIdx.x;
    const int tr = tid / 4, tq = (tid % 4) * 4;
    double acc[4] = {0, 0, 0, 0};
    for (int k0 = 0; k0 < k; k0 += NN_K) {
        for (int x = tid; x < NN_R * NN_K; x += 256) {
            const int rr = x / NN_K, kk = x % NN_K;
            const int64_t row = r0 + rr;
            As[rr][kk] = (row < rows && k0 + kk < k) ? A[row * lda + k0 + kk] : 0.0;
        }
        for (int x = tid; x < NN_K * NN_Q; x += 256) {
            const int kk = x / NN_Q, cc = x % NN_Q;
            Hs[kk][cc] = (k0 + kk < k && q0 + cc < q) ? H[(int64_t)(k0 + kk) * ldh + q0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < NN_K; ++kk) {
            const double a = As[tr][kk];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) acc[cc] = fma(a, Hs[kk][tq + cc], acc[cc]);
        }
        __syncthreads();
    }
    const int64_t row = r0 + tr;
    if (row < rows)
        for (int cc = 0; cc < 4; ++cc) {
            const int col = q0 + tq + cc;
            if (col < q) {
                double *p = &C[row * ldc + col];
                *p = (beta == 0.0 ? 0.0 : beta * *p) + alpha * acc[cc];
            }
        }
}

// ------------------------------------------------------------- gram_dd
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void dd_add(double &hi, double &lo, double x, double xe) {
    double s, e;
    two_sum(hi, x, s, e);
    e += lo + xe;
    hi = s + e;
    lo = e - (hi - s);
}

constexpr int DD_ROWS = 32;
constexpr int DD_MAXQ = 64;

__global__ __launch_bounds__(256) void gram_dd_kernel(const double *__restrict__ B, int64_t ldb,
                                                      int64_t rows, int q,
                                                      int64_t rows_per_block,
                                                      double *__restrict__ phi,
                                                      double *__restrict__ plo) {
    __shared__ double Bs[DD_ROWS][DD_MAXQ + 1];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(rows, r0 + rows_per_block);
    const int npair = q * (q + 1) / 2;
    const int tid = threadIdx.x;
    // each thread owns up to 9 pairs (q <= 64 gives at most 2080 pairs)
    double hi[9], lo[9];
    int pc[9], pd[9];
    int np = 0;
    for (int p = tid; p < npair && np < 9; p += 256, ++np) {
        int d = 0;
        while ((d + 1) * (d + 2) / 2 <= p) ++d;
        pc[np] = p - d * (d + 1) / 2;
        pd[np] = d;
        hi[np] = 0.0;
        lo[np] = 0.0;
    }
    for (int64_t rb = r0; rb < r1; rb += DD_ROWS) {
        for (int x = tid; x < DD_ROWS * q; x += 256) {
            const int rr = x / q, cc = x % q;
            const int64_t row = rb + rr;
            Bs[rr][cc] = row < r1 ? B[row * ldb + cc] : 0.0;
        }
        __syncthreads();
        for (int t = 0; t < np; ++t) {
            const int c = pc[t], d = pd[t];
            for (int rr = 0; rr < DD_ROWS; ++rr) {
                const double a = Bs[rr][c], b = Bs[rr][d];
                const double p = a * b;
                const double e = fma(a, b, -p);
                dd_add(hi[t], lo[t], p, e);
            }
        }
        __syncthreads();
    }
    for (int t = 0; t < np; ++t) {
        const int p = pd[t] * (pd[t] + 1) / 2 + pc[t];
        phi[(int64_t)blockIdx.x * npair + p] = hi[t];
        plo[(int64_t)blockIdx.x * npair + p] = lo[t];
    }
}

// One 64-thread block per pair: strided double-double partial sums, then a
// fixed-order double-double tree in LDS.
__global__ __launch_bounds__(64) void gram_dd_reduce(const double *__restrict__ phi,
                                                     const double *__restrict__ plo, int nblk,
                                                     int q, double *__restrict__ Ghi,
                                                     double *__restrict__ Glo) {
    __shared__ double rh[64], rl[64];
    const int npair = q * (q + 1) / 2;
    const int p = blockIdx.x;
    double hi = 0.0, lo = 0.0;
    for (int x = threadIdx.x; x < nblk; x += 64)
        dd_add(hi, lo, phi[(int64_t)x * npair + p], plo[(int64_t)x * npair + p]);
    rh[threadIdx.x] = hi;
    rl[threadIdx.x] = lo;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            double h2 = rh[threadIdx.x], l2 = rl[threadIdx.x];
            dd_add(h2, l2, rh[threadIdx.x + w], rl[threadIdx.x + w]);
            rh[threadIdx.x] = h2;
            rl[threadIdx.x] = l2;
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    hi = rh[0];
    lo = rl[0];
    int d = 0;
    while ((d + 1) * (d + 2) / 2 <= p) ++d;
    const int c = p - d * (d + 1) / 2;
    Ghi[c * q + d] = hi;
    Glo[c * q + d] = lo;
    Ghi[d * q + c] = hi;
    Glo[d * q + c] = lo;
}

__global__ void colnorm2_kernel(const double *__restrict__ B, int64_t ldb, int64_t rows, int q,
                                int64_t rows_per_block, double *__restrict__ part) {
    const int c = threadIdx.x % 64;
    const int lane_grp = threadIdx.x / 64;  // 4 row interleaves
    __shared__ double red[4][64];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(rows, r0 + rows_per_block);
    for (int cb = 0; cb < q; cb += 64) {
        double s = 0.0;
        if (cb + c < q)
            for (int64_t r = r0 + lane_grp; r < r1; r += 4) {
                const double v = B[r * ldb + cb + c];
                s = fma(v, v, s);
            }
        red[lane_grp][c] = s;
        __syncthreads();
        if (lane_grp == 0 && cb + c < q)
            part[(int64_t)blockIdx.x * q + cb + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
        __syncthreads();
    }
}

template <typename S, typename D>
__global__ void convert2d(const S *__restrict__ src, int64_t lds, D *__restrict__ dst,
                          int64_t ldd, int64_t rows, int cols) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    const int64_t r = idx / cols;
    const int c = (int)(idx - r * cols);
    dst[r * ldd + c] = static_cast<D>(src[r * lds + c]);
}

}  // namespace

void gemm_tn_f64(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t rows, int k,
                 int q, double *out, int64_t ldo, Ctx &c, hipStream_t s) {
    gemm_tn_impl<double>(A, lda, B, ldb, rows, k, q, out, ldo, c, s);
}

void gemm_tn_f32f64(const double *A, int64_t lda, const float *B, int64_t ldb, int64_t rows,
                    int k, int q, double *out, int64_t ldo, Ctx &c, hipStream_t s) {
    gemm_tn_impl<float>(A, lda, B, ldb, rows, k, q, out, ldo, c, s);
}

void gemm_nn_f64(const double *A, int64_t lda, const double *H, int64_t ldh, int64_t rows, int k,
                 int q, double alpha, double beta, double *C, int64_t ldc, hipStream_t s) {
    if (rows <= 0 || q <= 0) return;
    dim3 grid((unsigned)((rows + NN_R - 1) / NN_R), (unsigned)((q + NN_Q - 1) / NN_Q));
    hipLaunchKernelGGL(gemm_nn_kernel, grid, dim3(256), 0, s, A, lda, H, ldh, rows, k, q, alpha,
                       beta, C, ldc);
    HIPCHECK(hipGetLastError());
}

void gram_dd(const double *B, int64_t ldb, int64_t rows, int q, double *Ghi, double *Glo, Ctx &c,
             hipStream_t s) {
    if (q <= 0) return;
    if (q > DD_MAXQ) fail(BKS_EINVAL, "gram_dd: block wider than 64 columns");
    const int npair = q * (q + 1) / 2;
    // ~64 rows per block: a block's threads own up to 9 column pairs each, so
    // the kernel is bound by its double-double arithmetic, not by HBM, and
    // needs many blocks (m = 2e4 rows: 313 blocks; 256 rows per block kept
    // 3/4 of the chip idle)
    int64_t nblk = std::min<int64_t>(1024, std::max<int64_t>(1, (rows + 63) / 64));
    int64_t rpb = std::max<int64_t>(1, (rows + nblk - 1) / nblk);
    nblk = std::max<int64_t>(1, (rows + rpb - 1) / rpb);
    c.ws_pack2.ensure((size_t)nblk * npair * 2 * sizeof(double));
    double *phi = c.ws_pack2.as<double>();
    double *plo = phi + nblk * npair;
    hipLaunchKernelGGL(gram_dd_kernel, dim3((unsigned)nblk), dim3(256), 0, s, B, ldb, rows, q, rpb,
                       phi, plo);
    hipLaunchKernelGGL(gram_dd_reduce, dim3(npair), dim3(64), 0, s, phi, plo, (int)nblk, q, Ghi,
                       Glo);
    HIPCHECK(hipGetLastError());
}

void colnorm2(const double *B, int64_t ldb, int64_t rows, int q, double *out, Ctx &c,
              hipStream_t s) {
    if (q <= 0) return;
    int64_t nblk = std::min<int64_t>(2048, std::max<int64_t>(1, (rows + 63) / 64));
    int64_t rpb = std::max<int64_t>(1, (rows + nblk - 1) / nblk);
    nblk = std::max<int64_t>(1, (rows + rpb - 1) / rpb);
    c.ws_pack1.ensure((size_t)nblk * q * sizeof(double));
    double *part = c.ws_pack1.as<double>();
    hipLaunchKernelGGL(colnorm2_kernel, dim3((unsigned)nblk), dim3(256), 0, s, B, ldb, rows, q, rpb,
                       part);
    launch_reduce(part, (int)nblk, 1, q, out, (int64_t)q, s);
    HIPCHECK(hipGetLastError());
}

void convert_f64_f32(const double *src, int64_t lds, float *dst, int64_t ldd, int64_t rows,
                     int cols, hipStream_t s) {
    const int64_t n = rows * cols;
    if (n <= 0) return;
    hipLaunchKernelGGL((convert2d<double, float>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       s, src, lds, dst, ldd, rows, cols);
    HIPCHECK(hipGetLastError());
}

void convert_f32_f64(const float *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                     int cols, hipStream_t s) {
    const int64_t n = rows * cols;
    if (n <= 0) return;
    hipLaunchKernelGGL((convert2d<float, double>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       s, src, lds, dst, ldd, rows, cols);
    HIPCHECK(hipGetLastError());
}

void copy2d_f64(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows, int cols,
                hipStream_t s) {
    const int64_t n = rows * cols;
    if (n <= 0) return;
    hipLaunchKernelGGL((convert2d<double, double>), dim3((unsigned)((n + 255) / 256)), dim3(256),
                       0, s, src, lds, dst, ldd, rows, cols);
    HIPCHECK(hipGetLastError());
}

}  // namespace bks
