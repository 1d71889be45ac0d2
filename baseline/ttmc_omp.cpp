// CPU baseline of the tensor-times-block products: plain FP64 loops over a
// sorted stored-entry layout, parallel over output rows with OpenMP on all
// host cores.  A measurement baseline, written independently of the GPU
// library and checked against the FP64 oracle; not part of the product.
//
//   free3: T3(k, :) = sum over stored (i <= j, k, v) of v X(i,:)^T Y(j,:) and,
//          for i != j, v X(j,:)^T Y(i,:)   (symmetric half: a <= b, column
//          b(b+1)/2 + a; else column a + px b)
//   free1: T1(r, b + py c) = sum over the full entries (r, col, k, v) of
//          v Y(col, b) Z(k, c)             (both orientations given)
//   mode3: t(q, c) = sum over the fibre of stored pair q of v Z(k, c)
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

#include <omp.h>

extern "C" {

void cpu_free3(int64_t n, const int64_t *kptr, const int32_t *ei, const int32_t *ej,
               const double *ev, const double *X, int px, const double *Y, int py, int sym,
               double *out) {
    const int64_t q = sym ? (int64_t)px * (px + 1) / 2 : (int64_t)px * py;
#pragma omp parallel
    {
        std::vector<double> M((std::size_t)px * py);
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < n; ++k) {
            std::fill(M.begin(), M.end(), 0.0);
            for (int64_t e = kptr[k]; e < kptr[k + 1]; ++e) {
                const int64_t i = ei[e], j = ej[e];
                const double v = ev[e], w = i != j ? v : 0.0;
                const double *Xi = X + i * px, *Xj = X + j * px;
                const double *Yi = Y + i * py, *Yj = Y + j * py;
                for (int a = 0; a < px; ++a) {
                    const double s1 = v * Xi[a], s2 = w * Xj[a];
                    double *Ma = M.data() + (std::size_t)a * py;
                    for (int b = 0; b < py; ++b) Ma[b] += s1 * Yj[b] + s2 * Yi[b];
                }
            }
            double *o = out + k * q;
            if (sym) {
                for (int b = 0; b < px; ++b)
                    for (int a = 0; a <= b; ++a) o[b * (b + 1) / 2 + a] = M[(std::size_t)a * py + b];
            } else {
                for (int b = 0; b < py; ++b)
                    for (int a = 0; a < px; ++a) o[a + (int64_t)px * b] = M[(std::size_t)a * py + b];
            }
        }
    }
}

void cpu_free1(int64_t m, const int64_t *rptr, const int32_t *col, const int32_t *kk,
               const double *ev, const double *Y, int py, const double *Z, int pz, double *out) {
    const int64_t q = (int64_t)py * pz;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < m; ++r) {
        double *o = out + r * q;
        for (int64_t c = 0; c < q; ++c) o[c] = 0.0;
        for (int64_t e = rptr[r]; e < rptr[r + 1]; ++e) {
            const double v = ev[e];
            const double *y = Y + (int64_t)col[e] * py, *z = Z + (int64_t)kk[e] * pz;
            for (int c = 0; c < pz; ++c) {
                const double s = v * z[c];
                for (int b = 0; b < py; ++b) o[b + (int64_t)py * c] += s * y[b];
            }
        }
    }
}

void cpu_mode3(int64_t P, const int64_t *pptr, const int32_t *kk, const double *ev,
               const double *Z, int pz, double *out) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < P; ++p) {
        double *o = out + p * pz;
        for (int c = 0; c < pz; ++c) o[c] = 0.0;
        for (int64_t e = pptr[p]; e < pptr[p + 1]; ++e) {
            const double v = ev[e];
            const double *z = Z + (int64_t)kk[e] * pz;
            for (int c = 0; c < pz; ++c) o[c] += v * z[c];
        }
    }
}

int cpu_threads(void) {
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}

}  // extern "C"
