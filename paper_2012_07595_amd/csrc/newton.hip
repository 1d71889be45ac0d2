// The Newton matrix of the inner solve (Algorithm 5 step (i)) formed on the
// device from the rotated core blocks that DevInner::rotate leaves there,
// and factorised where it lies: for large cores the matrix (N = r(k1 - r) +
// r3(k3 - r3) unknowns, N^2 doubles: 2.3 GB at rank (20,20,20) with k1 = 580,
// k3 = 310) is neither assembled on the host nor uploaded.
//
// Blocks of B = C.([P P_perp], [P P_perp], [S S_perp]) as rotate() leaves
// them (column-major): Y(x, y, l) = B(x, y, l) for l < r3 (k1 x k1 x r3) and
// Y2(x, j, z) = B(x, j, r3 + z) for j < r, z < k3 - r3 (k1 x r x C1).  With
// F = B000, M = B100, B110, B001, B101 the negative Hessian H = -2A of the
// second-order model (the host's newton_matrix states the entries) is, in
// Delta (x, a) and Theta (z, c) coordinates:
//   DD  H = -(v(i, j) + v(j, i)),  v((x,a),(y,b)) = 2 sum_c M(y,a,c) M(x,b,c)
//         + 2 sum_c B110(x,y,c) F(a,b,c) + 2 [a=b] MM(x,y) - 2 [x=y] S1(a,b)
//   DT  H = -4 sum_b M(x,b,c) B001(a,b,z) - 4 sum_b B101(x,b,z) F(a,b,c)
//   TT  H = -2 [c=d] G(z,w) + 2 [z=w] S3(c,d)
// with MM(x,y) = <M_x, M_y>, S1 = <F, F>_{-1}, S3 = <F, F>_{-3},
// G(z,w) = <B001_z, B001_w>.  Every entry is a function of its (row, column)
// pair evaluated in a fixed order, and the DD entry is symmetric in them, so
// H is exactly symmetric.
#include <algorithm>
#include <cstring>

#include "bks_internal.h"

namespace bks {

namespace {

struct NewtonDims {
    int k1, r, r3, A1, C1, nd, N;
};

// Compact copies of the small blocks, laid out for the Hessian kernel's
// reads (consecutive threads of a row walk the fastest index):
//   Mb[(c A1 + x) r + b]  = M(x,b,c)      Mc[(x r + b) r3 + c] = M(x,b,c)
//   Fb[(c r + a) r + b]   = F(a,b,c)      Fc[(a r + b) r3 + c] = F(a,b,c)
__global__ void newton_pack(const double *__restrict__ Y, NewtonDims d, double *__restrict__ Mb,
                            double *__restrict__ Mc, double *__restrict__ Fb,
                            double *__restrict__ Fc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nm = (int64_t)d.A1 * d.r * d.r3, nf = (int64_t)d.r * d.r * d.r3;
    const int64_t k1 = d.k1;
    if (t < nm) {
        const int x = (int)(t % d.A1), b = (int)((t / d.A1) % d.r), c = (int)(t / ((int64_t)d.A1 * d.r));
        const double v = Y[(d.r + x) + k1 * (b + k1 * c)];
        Mb[((int64_t)c * d.A1 + x) * d.r + b] = v;
        Mc[((int64_t)x * d.r + b) * d.r3 + c] = v;
    } else if (t < nm + nf) {
        const int64_t u = t - nm;
        const int a = (int)(u % d.r), b = (int)((u / d.r) % d.r), c = (int)(u / ((int64_t)d.r * d.r));
        const double v = Y[a + k1 * (b + k1 * c)];
        Fb[((int64_t)c * d.r + a) * d.r + b] = v;
        Fc[((int64_t)a * d.r + b) * d.r3 + c] = v;
    }
}

// The small Gram matrices: MM (A1 x A1), S1 (r x r), S3 (r3 x r3), G (C1 x
// C1), one thread per entry, summed in a fixed order that does not depend on
// which of (p, q) and (q, p) is computed (products commute), so each is
// exactly symmetric.
__global__ void newton_grams(const double *__restrict__ Y2, const double *__restrict__ Mc,
                             const double *__restrict__ Fc, NewtonDims d, double *__restrict__ MM,
                             double *__restrict__ S1, double *__restrict__ S3,
                             double *__restrict__ G) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n1 = (int64_t)d.A1 * d.A1, n2 = (int64_t)d.r * d.r, n3 = (int64_t)d.r3 * d.r3,
                  n4 = (int64_t)d.C1 * d.C1;
    const int r = d.r, r3 = d.r3;
    const int64_t k1 = d.k1;
    if (t < n1) {
        const int x = (int)(t / d.A1), y = (int)(t % d.A1);
        const double *mx = Mc + (int64_t)x * r * r3, *my = Mc + (int64_t)y * r * r3;
        double s = 0.0;
        for (int q = 0; q < r * r3; ++q) s = fma(mx[q], my[q], s);
        MM[t] = s;
    } else if (t < n1 + n2) {
        const int64_t u = t - n1;
        const int a = (int)(u / r), b = (int)(u % r);
        double s = 0.0;
        // S1(a,b) = sum_{y,c} F(a,y,c) F(b,y,c); Fc rows (a, y) hold c
        for (int y = 0; y < r; ++y) {
            const double *fa = Fc + ((int64_t)a * r + y) * r3, *fb = Fc + ((int64_t)b * r + y) * r3;
            for (int c = 0; c < r3; ++c) s = fma(fa[c], fb[c], s);
        }
        S1[u] = s;
    } else if (t < n1 + n2 + n3) {
        const int64_t u = t - n1 - n2;
        const int c = (int)(u / r3), e = (int)(u % r3);
        double s = 0.0;
        for (int q = 0; q < r * r; ++q) s = fma(Fc[(int64_t)q * r3 + c], Fc[(int64_t)q * r3 + e], s);
        S3[u] = s;
    } else if (t < n1 + n2 + n3 + n4) {
        const int64_t u = t - n1 - n2 - n3;
        const int z = (int)(u / d.C1), w = (int)(u % d.C1);
        double s = 0.0;
        for (int b = 0; b < r; ++b)
            for (int a = 0; a < r; ++a)
                s = fma(Y2[a + k1 * (b + (int64_t)r * z)], Y2[a + k1 * (b + (int64_t)r * w)], s);
        G[u] = s;
    }
}

// v((x,a),(y,b)) of the Delta-Delta block (see the header)
__device__ __forceinline__ double dd_term(const double *__restrict__ Y, const double *__restrict__ Mb,
                                          const double *__restrict__ Fb, const double *__restrict__ MM,
                                          const double *__restrict__ S1, const NewtonDims &d, int x,
                                          int a, int y, int b) {
    const int64_t k1 = d.k1, sl = k1 * k1;
    const int r = d.r;
    double g = 0.0, k = 0.0;
    for (int c = 0; c < d.r3; ++c) {
        const int64_t mc = (int64_t)c * d.A1;
        g = fma(Mb[(mc + y) * r + a], Mb[(mc + x) * r + b], g);
        k = fma(Y[(r + x) + k1 * (r + y) + sl * c], Fb[((int64_t)c * r + a) * r + b], k);
    }
    double v = 2.0 * g + 2.0 * k;
    if (a == b) v += 2.0 * MM[(int64_t)x * d.A1 + y];
    if (x == y) v -= 2.0 * S1[(int64_t)a * r + b];
    return v;
}

// Delta-Theta entry for Delta (x, a), Theta (z, c)
__device__ __forceinline__ double dt_term(const double *__restrict__ Y2, const double *__restrict__ Mc,
                                          const double *__restrict__ Fc, const NewtonDims &d, int x,
                                          int a, int z, int c) {
    const int64_t k1 = d.k1;
    const int r = d.r;
    double t1 = 0.0, t2 = 0.0;
    for (int b = 0; b < r; ++b) {
        const int64_t col = k1 * (b + (int64_t)r * z);
        t1 = fma(Mc[((int64_t)x * r + b) * d.r3 + c], Y2[a + col], t1);
        t2 = fma(Y2[(r + x) + col], Fc[((int64_t)a * r + b) * d.r3 + c], t2);
    }
    double v = -4.0 * t1;
    v -= 4.0 * t2;
    return v;
}

// H (N x N, row-major = column-major: symmetric), one thread per entry of a
// row segment; nbx blocks of 256 threads per row.
__global__ __launch_bounds__(256) void newton_hessian(
    const double *__restrict__ Y, const double *__restrict__ Y2, const double *__restrict__ Mb,
    const double *__restrict__ Mc, const double *__restrict__ Fb, const double *__restrict__ Fc, const double *__restrict__ MM, const double *__restrict__ S1,
    const double *__restrict__ S3, const double *__restrict__ G, NewtonDims d, int nbx,
    double *__restrict__ H) {
    const int64_t i = blockIdx.x / nbx;
    const int64_t j = (int64_t)(blockIdx.x % nbx) * 256 + threadIdx.x;
    if (i >= d.N || j >= d.N) return;
    const int r = d.r, r3 = d.r3, nd = d.nd;
    double h;
    if (i < nd && j < nd) {
        const int x = (int)(i / r), a = (int)(i % r), y = (int)(j / r), b = (int)(j % r);
        // v(i, j) + v(j, i): each evaluated as a function of its own
        // (row, column) pair, so the thread of (j, i) forms the same sum
        const double vij = dd_term(Y, Mb, Fb, MM, S1, d, x, a, y, b);
        const double vji = dd_term(Y, Mb, Fb, MM, S1, d, y, b, x, a);
        h = -(vij + vji);
    } else if (i < nd) {
        const int64_t jt = j - nd;
        h = dt_term(Y2, Mc, Fc, d, (int)(i / r), (int)(i % r), (int)(jt / r3), (int)(jt % r3));
    } else if (j < nd) {
        const int64_t it = i - nd;
        h = dt_term(Y2, Mc, Fc, d, (int)(j / r), (int)(j % r), (int)(it / r3), (int)(it % r3));
    } else {
        const int64_t it = i - nd, jt = j - nd;
        const int z = (int)(it / r3), c = (int)(it % r3), w = (int)(jt / r3), e = (int)(jt % r3);
        h = 0.0;
        if (c == e) h += -2.0 * G[(int64_t)z * d.C1 + w];
        if (z == w) h += 2.0 * S3[(int64_t)c * r3 + e];
    }
    H[i * d.N + j] = h;
}

__global__ void newton_diag(const double *__restrict__ H, int64_t N, double *__restrict__ diag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) diag[i] = H[i * N + i];
}

}  // namespace

bool DevInner::newton_matrix(int r, int r3, double *diag) {
    NewtonDims d;
    d.k1 = k1;
    d.r = r;
    d.r3 = r3;
    d.A1 = k1 - r;
    d.C1 = k3 - r3;
    d.nd = d.A1 * r;
    const int64_t N64 = (int64_t)d.nd + (int64_t)d.C1 * r3;
    if (N64 <= 0 || N64 > (int64_t)1 << 30) return false;
    d.N = (int)N64;
    // rotate() left Y (k1^2 r3) and Y2 (k1 r C1) in dY for this r, r3
    if (rot_r != r || rot_r3 != r3) fail(BKS_EINVAL, "newton_matrix: no rotation for this rank");
    const int64_t sl = (int64_t)k1 * k1;
    const double *Y = dY.as<double>(), *Y2 = Y + sl * r3;
    const int64_t nm = (int64_t)d.A1 * r * r3, nf = (int64_t)r * r * r3;
    const int64_t ng = (int64_t)d.A1 * d.A1 + (int64_t)r * r + (int64_t)r3 * r3 + (int64_t)d.C1 * d.C1;
    dNw.ensure((size_t)(2 * nm + 2 * nf + ng + N64) * 8);
    double *Mb = dNw.as<double>(), *Mc = Mb + nm, *Fb = Mc + nm, *Fc = Fb + nf;
    double *MM = Fc + nf, *S1 = MM + (int64_t)d.A1 * d.A1, *S3 = S1 + (int64_t)r * r,
           *G = S3 + (int64_t)r3 * r3, *dg = G + (int64_t)d.C1 * d.C1;
    const size_t hb = (size_t)N64 * N64 * 8;
    ds->dH.ensure(hb);
    hipLaunchKernelGGL(newton_pack, dim3((unsigned)((nm + nf + 255) / 256)), dim3(256), 0, s, Y, d,
                       Mb, Mc, Fb, Fc);
    HIPCHECK(hipGetLastError());
    hipLaunchKernelGGL(newton_grams, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, Y2, Mc,
                       Fc, d, MM, S1, S3, G);
    HIPCHECK(hipGetLastError());
    const int nbx = (d.N + 255) / 256;
    const int64_t nblk = (int64_t)d.N * nbx;
    if (nblk > 0x7fffffff) return false;
    hipLaunchKernelGGL(newton_hessian, dim3((unsigned)nblk), dim3(256), 0, s, Y, Y2, Mb, Mc, Fb, Fc,
                       MM, S1, S3, G, d, nbx, ds->dH.as<double>());
    HIPCHECK(hipGetLastError());
    hipLaunchKernelGGL(newton_diag, dim3((unsigned)((N64 + 255) / 256)), dim3(256), 0, s,
                       ds->dH.as<double>(), N64, dg);
    HIPCHECK(hipGetLastError());
    double *hs = stage((size_t)N64);
    HIPCHECK(hipMemcpyAsync(hs, dg, (size_t)N64 * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    std::memcpy(diag, hs, (size_t)N64 * 8);
    newton_n = d.N;
    return true;
}

bool DevInner::newton_solve(double mu, double *b) {
    if (newton_n <= 0) fail(BKS_EINVAL, "newton_solve: no device Newton matrix");
    return ds->solve_resident(s, newton_n, mu, b);
}

}  // namespace bks
