// Small dense FP64 linear algebra (host).  Textbook algorithms: Householder
// reduction to tridiagonal form followed by the implicitly shifted QL
// iteration for symmetric eigenproblems, right-looking Cholesky, Householder
// QR.
#include "linalg.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

namespace bks {
namespace la {

namespace {

// Reduce symmetric A (n x n, row-major, in Z) to tridiagonal T = Q^T A Q;
// on return Z holds Q, d the diagonal and e[i] = T(i, i+1), e[n-1] = 0.
void tridiagonalize(int n, std::vector<double> &Z, std::vector<double> &d,
                    std::vector<double> &e) {
    std::vector<double> A = Z;
    std::vector<std::vector<double>> vs;
    vs.reserve(n);
    std::vector<double> p(n), q(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        std::vector<double> v(len);
        double nrm2 = 0.0;
        for (int i = 0; i < len; ++i) {
            v[i] = A[(size_t)(k + 1 + i) * n + k];
            nrm2 += v[i] * v[i];
        }
        const double nrm = std::sqrt(nrm2);
        if (nrm == 0.0) {
            vs.emplace_back();
            continue;
        }
        const double alpha = v[0] > 0 ? -nrm : nrm;
        v[0] -= alpha;
        double vn2 = 0.0;
        for (int i = 0; i < len; ++i) vn2 += v[i] * v[i];
        if (vn2 == 0.0) {
            vs.emplace_back();
            continue;
        }
        const double inv = 1.0 / std::sqrt(vn2);
        for (int i = 0; i < len; ++i) v[i] *= inv;
        // A22 <- H A22 H with H = I - 2 v v^T
        double K = 0.0;
        for (int i = 0; i < len; ++i) {
            double s = 0.0;
            const double *row = &A[(size_t)(k + 1 + i) * n + k + 1];
            for (int j = 0; j < len; ++j) s += row[j] * v[j];
            p[i] = s;
            K += v[i] * s;
        }
        for (int i = 0; i < len; ++i) q[i] = p[i] - K * v[i];
        for (int i = 0; i < len; ++i) {
            double *row = &A[(size_t)(k + 1 + i) * n + k + 1];
            const double vi = v[i], qi = q[i];
            for (int j = 0; j < len; ++j) row[j] -= 2.0 * (vi * q[j] + qi * v[j]);
        }
        A[(size_t)(k + 1) * n + k] = alpha;
        A[(size_t)k * n + k + 1] = alpha;
        for (int i = 1; i < len; ++i) {
            A[(size_t)(k + 1 + i) * n + k] = 0.0;
            A[(size_t)k * n + k + 1 + i] = 0.0;
        }
        vs.push_back(std::move(v));
    }
    d.assign(n, 0.0);
    e.assign(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)i * n + i + 1];
    // Q = H_0 H_1 ... : start from I and apply each reflector on the right
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    for (int k = 0; k < (int)vs.size(); ++k) {
        const auto &v = vs[k];
        if (v.empty()) continue;
        const int len = n - k - 1;
        for (int i = 0; i < n; ++i) {
            double *row = &Z[(size_t)i * n + k + 1];
            double s = 0.0;
            for (int j = 0; j < len; ++j) s += row[j] * v[j];
            s *= 2.0;
            for (int j = 0; j < len; ++j) row[j] -= s * v[j];
        }
    }
}

// Implicitly shifted QL on the tridiagonal (d, e); rotations accumulated
// into the columns of Z.
void tridiag_ql(int n, std::vector<double> &d, std::vector<double> &e, std::vector<double> &Z) {
    const double eps = std::numeric_limits<double>::epsilon();
    double anorm = 0.0;
    for (int i = 0; i < n; ++i) anorm = std::max(anorm, std::fabs(d[i]) + std::fabs(e[i]));
    if (!std::isfinite(anorm)) throw std::runtime_error("eigensolver: non-finite input");
    // an off-diagonal entry is negligible relative to its neighbours or, for
    // clusters of (near-)zero eigenvalues, relative to the matrix norm
    const double floor_ = eps * 1e-3 * anorm;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        int m;
        do {
            for (m = l; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd || std::fabs(e[m]) <= floor_) break;
            }
            if (m != l) {
                if (++iter > 300) throw std::runtime_error("eigensolver did not converge");
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = std::hypot(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
                double s = 1.0, c = 1.0, p = 0.0;
                int i;
                bool early = false;
                for (i = m - 1; i >= l; --i) {
                    double f = s * e[i];
                    const double b = c * e[i];
                    r = std::hypot(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) {
                        d[i + 1] -= p;
                        e[m] = 0.0;
                        early = true;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    for (int k = 0; k < n; ++k) {
                        double *zr = &Z[(size_t)k * n];
                        f = zr[i + 1];
                        zr[i + 1] = s * zr[i] + c * f;
                        zr[i] = c * zr[i] - s * f;
                    }
                }
                if (early) continue;
                d[l] -= p;
                e[l] = g;
                e[m] = 0.0;
            }
        } while (m != l);
    }
}

}  // namespace

void sym_eig(int n, const double *A, double *w, double *V) {
    if (n == 0) return;
    if (n == 1) {
        w[0] = A[0];
        V[0] = 1.0;
        return;
    }
    std::vector<double> Z(A, A + (size_t)n * n);
    // symmetrise (callers pass symmetric matrices up to rounding)
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double s = 0.5 * (Z[(size_t)i * n + j] + Z[(size_t)j * n + i]);
            Z[(size_t)i * n + j] = Z[(size_t)j * n + i] = s;
        }
    std::vector<double> d, e;
    tridiagonalize(n, Z, d, e);
    tridiag_ql(n, d, e, Z);
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] > d[b]; });
    for (int j = 0; j < n; ++j) {
        w[j] = d[ord[j]];
        for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = Z[(size_t)i * n + ord[j]];
    }
}

void top_eigvecs(int n, const double *A, int r, double *Vr, double *wr) {
    std::vector<double> w(n), V((size_t)n * n);
    sym_eig(n, A, w.data(), V.data());
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < r; ++j) Vr[(size_t)i * r + j] = V[(size_t)i * n + j];
    if (wr)
        for (int j = 0; j < r; ++j) wr[j] = w[j];
}

bool cholesky(int n, double *A, double *fail_pivot) {
    // Right-looking A = U^T U on the upper triangle (row j of U contiguous,
    // trailing update as row AXPYs), then L = U^T into the lower triangle.
    for (int j = 0; j < n; ++j) {
        double *uj = &A[(size_t)j * n];
        const double s = uj[j];
        if (!(s > 0.0)) {
            if (fail_pivot) *fail_pivot = s;
            return false;
        }
        const double d = std::sqrt(s);
        const double inv = 1.0 / d;
        uj[j] = d;
        for (int k = j + 1; k < n; ++k) uj[k] *= inv;
        for (int i = j + 1; i < n; ++i) {
            const double f = uj[i];
            if (f == 0.0) continue;
            double *ai = &A[(size_t)i * n];
            for (int k = i; k < n; ++k) ai[k] -= f * uj[k];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i];
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) A[(size_t)i * n + j] = 0.0;
    return true;
}

void chol_solve(int n, const double *L, double *b) {
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        const double *ri = &L[(size_t)i * n];
        for (int k = 0; k < i; ++k) s -= ri[k] * b[k];
        b[i] = s / ri[i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * b[k];
        b[i] = s / L[(size_t)i * n + i];
    }
}

void qr_full(int m, int n, const double *Ain, double *Q) {
    std::vector<double> A(Ain, Ain + (size_t)m * n);
    std::vector<std::vector<double>> vs;
    for (int k = 0; k < n && k < m; ++k) {
        const int len = m - k;
        std::vector<double> v(len);
        double nrm2 = 0.0;
        for (int i = 0; i < len; ++i) {
            v[i] = A[(size_t)(k + i) * n + k];
            nrm2 += v[i] * v[i];
        }
        const double nrm = std::sqrt(nrm2);
        const double alpha = v[0] > 0 ? -nrm : nrm;
        v[0] -= alpha;
        double vn2 = 0.0;
        for (int i = 0; i < len; ++i) vn2 += v[i] * v[i];
        if (vn2 > 0.0) {
            const double inv = 1.0 / std::sqrt(vn2);
            for (int i = 0; i < len; ++i) v[i] *= inv;
            for (int j = k; j < n; ++j) {
                double s = 0.0;
                for (int i = 0; i < len; ++i) s += v[i] * A[(size_t)(k + i) * n + j];
                s *= 2.0;
                for (int i = 0; i < len; ++i) A[(size_t)(k + i) * n + j] -= s * v[i];
            }
        } else {
            std::fill(v.begin(), v.end(), 0.0);
        }
        vs.push_back(std::move(v));
    }
    // Q = H_0 H_1 ... H_{n-1} applied to I
    std::fill(Q, Q + (size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
    for (int k = (int)vs.size() - 1; k >= 0; --k) {
        const auto &v = vs[k];
        const int len = m - k;
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
            for (int i = 0; i < len; ++i) s += v[i] * Q[(size_t)(k + i) * m + j];
            s *= 2.0;
            if (s != 0.0)
                for (int i = 0; i < len; ++i) Q[(size_t)(k + i) * m + j] -= s * v[i];
        }
    }
    // keep the column signs so that span(Q(:, :n)) matches A's columns in order
}

void orthonormalize(int m, int n, double *A) {
    std::vector<double> Q((size_t)m * m);
    qr_full(m, n, A, Q.data());
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = Q[(size_t)i * m + j];
}

void gemm(int m, int n, int k, const double *A, const double *B, double *C) {
    std::fill(C, C + (size_t)m * n, 0.0);
    for (int i = 0; i < m; ++i) {
        double *ci = &C[(size_t)i * n];
        for (int l = 0; l < k; ++l) {
            const double a = A[(size_t)i * k + l];
            if (a == 0.0) continue;
            const double *bl = &B[(size_t)l * n];
            for (int j = 0; j < n; ++j) ci[j] += a * bl[j];
        }
    }
}

void gemm_tn(int m, int n, int k, const double *A, const double *B, double *C) {
    std::fill(C, C + (size_t)m * n, 0.0);
    for (int l = 0; l < k; ++l) {
        const double *al = &A[(size_t)l * m];
        const double *bl = &B[(size_t)l * n];
        for (int i = 0; i < m; ++i) {
            const double a = al[i];
            if (a == 0.0) continue;
            double *ci = &C[(size_t)i * n];
            for (int j = 0; j < n; ++j) ci[j] += a * bl[j];
        }
    }
}

}  // namespace la
}  // namespace bks
