// Small dense FP64 linear algebra (host).  Textbook algorithms: Householder
// reduction to tridiagonal form followed by the implicitly shifted QL
// iteration (EISPACK IMTQL2) for symmetric eigenproblems, blocked
// right-looking Cholesky, Householder QR, and a register-blocked product on
// AVX2 FMA.
#include "linalg.h"

#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <mutex>
#include <numeric>
#include <stdexcept>
#include <thread>

namespace bks {
namespace la {

namespace {

// sum_j a[j] b[j] with 16 partial sums in AVX2 registers (fixed order:
// lane sums, then the four registers, then the tail), where a plain loop
// would be one dependent chain of FMAs
inline double dot_avx(const double *a, const double *b, int n) {
    __m256d s0 = _mm256_setzero_pd(), s1 = _mm256_setzero_pd();
    __m256d s2 = _mm256_setzero_pd(), s3 = _mm256_setzero_pd();
    int j = 0;
    for (; j + 16 <= n; j += 16) {
        s0 = _mm256_fmadd_pd(_mm256_loadu_pd(a + j), _mm256_loadu_pd(b + j), s0);
        s1 = _mm256_fmadd_pd(_mm256_loadu_pd(a + j + 4), _mm256_loadu_pd(b + j + 4), s1);
        s2 = _mm256_fmadd_pd(_mm256_loadu_pd(a + j + 8), _mm256_loadu_pd(b + j + 8), s2);
        s3 = _mm256_fmadd_pd(_mm256_loadu_pd(a + j + 12), _mm256_loadu_pd(b + j + 12), s3);
    }
    for (; j + 4 <= n; j += 4) s0 = _mm256_fmadd_pd(_mm256_loadu_pd(a + j), _mm256_loadu_pd(b + j), s0);
    const __m256d s = _mm256_add_pd(_mm256_add_pd(s0, s1), _mm256_add_pd(s2, s3));
    alignas(32) double l[4];
    _mm256_store_pd(l, s);
    double r = (l[0] + l[1]) + (l[2] + l[3]);
    for (; j < n; ++j) r += a[j] * b[j];
    return r;
}
// orders from which top_eigvecs takes the reduced path
constexpr int kTopEigMin = 24;

// Reduce symmetric A (n x n, row-major, in Z) to tridiagonal T = Q^T A Q;
// on return Z holds Q, d the diagonal and e[i] = T(i, i+1), e[n-1] = 0.
// The reduction alone: the reflectors H_k = I - 2 v_k v_k^T (acting on
// indices k+1 .. n-1; empty where the column was already reduced) in vs,
// T in (d, e); A is overwritten.
void tridiag_reduce(int n, std::vector<double> &A, std::vector<double> &d, std::vector<double> &e,
                    std::vector<std::vector<double>> &vs) {
    vs.clear();
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
        for (int i = 0; i < len; ++i) p[i] = dot_avx(&A[(size_t)(k + 1 + i) * n + k + 1], v.data(), len);
        double K = 0.0;
        for (int i = 0; i < len; ++i) K += v[i] * p[i];
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
}

void tridiagonalize(int n, std::vector<double> &Z, std::vector<double> &d,
                    std::vector<double> &e) {
    std::vector<double> A = Z;
    std::vector<std::vector<double>> vs;
    tridiag_reduce(n, A, d, e, vs);
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

// Implicitly shifted QL on the tridiagonal (d, e): the Martin-Wilkinson
// implicit QL algorithm in the form EISPACK publishes as IMTQL2 (from
// Wilkinson and Reinsch's Handbook, vol. II), with its step order and
// underflow exit; rotations accumulated into the rows of Zt = Z^T (row i of
// Zt is column i of Z, so each rotation updates two contiguous rows).
void tridiag_ql(int n, std::vector<double> &d, std::vector<double> &e, std::vector<double> &Zt,
                bool vectors = true) {
    const double eps = std::numeric_limits<double>::epsilon();
    double anorm = 0.0;
    for (int i = 0; i < n; ++i) anorm = std::max(anorm, std::fabs(d[i]) + std::fabs(e[i]));
    if (!std::isfinite(anorm)) throw std::runtime_error("eigensolver: non-finite input");
    // Without vectors: T scaled to unit norm (the eigenvalues scale back),
    // so that sqrt(a^2 + b^2) cannot overflow and replaces the slower
    // library hypot.
    double unscale = 1.0;
    if (!vectors && anorm > 0.0) {
        for (int i = 0; i < n; ++i) {
            d[i] /= anorm;
            e[i] /= anorm;
        }
        unscale = anorm;
        anorm = 1.0;
    }
    auto pyth = [vectors](double a, double b) {
        return vectors ? std::hypot(a, b) : std::sqrt(a * a + b * b);
    };
    // an off-diagonal entry is negligible relative to its neighbours or, for
    // clusters of (near-)zero eigenvalues, relative to the matrix norm (and
    // always below the smallest normal number: a tiny matrix whose relative
    // floor underflows must still converge)
    const double floor_ = std::max(eps * 1e-3 * anorm, std::numeric_limits<double>::min());
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
                double r = pyth(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
                double s = 1.0, c = 1.0, p = 0.0;
                int i;
                bool early = false;
                for (i = m - 1; i >= l; --i) {
                    double f = s * e[i];
                    const double b = c * e[i];
                    r = pyth(f, g);
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
                    if (!vectors) continue;
                    double *zi = &Zt[(size_t)i * n], *zi1 = &Zt[(size_t)(i + 1) * n];
                    for (int k = 0; k < n; ++k) {
                        const double a0 = zi[k], a1 = zi1[k];
                        zi1[k] = s * a0 + c * a1;
                        zi[k] = c * a0 - s * a1;
                    }
                }
                if (early) continue;
                d[l] -= p;
                e[l] = g;
                e[m] = 0.0;
            }
        } while (m != l);
    }
    if (unscale != 1.0)
        for (int q = 0; q < n; ++q) d[q] *= unscale;
}

}  // namespace

namespace {

// Cyclic Jacobi on a symmetric row-major matrix (destroyed): eigenvalues in
// w, eigenvectors as the columns of V (row-major).  Slow but unconditionally
// convergent; the fallback when the QL iteration stalls.
void jacobi_eig(int n, std::vector<double> &A, std::vector<double> &w, std::vector<double> &V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
    double tot = 0.0;
    for (double x : A) tot += x * x;
    const double eps = std::numeric_limits<double>::epsilon();
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += 2.0 * a(p, q) * a(p, q);
        if (off <= eps * eps * tot || off == 0.0) {
            w.resize(n);
            for (int i = 0; i < n; ++i) w[i] = a(i, i);
            return;
        }
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a(p, q);
                if (apq == 0.0) continue;
                // rotation in the (p, q) plane that zeroes A(p, q)
                const double th = (a(q, q) - a(p, p)) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * akq;
                    a(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * aqk;
                    a(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    throw std::runtime_error("eigensolver did not converge");
}

}  // namespace

void sym_eig_jacobi(int n, const double *A, double *w, double *V) {
    if (n == 0) return;
    std::vector<double> Z(A, A + (size_t)n * n), wj, Vj;
    for (double x : Z)
        if (!std::isfinite(x)) throw std::runtime_error("eigensolver: non-finite input");
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double s = 0.5 * (Z[(size_t)i * n + j] + Z[(size_t)j * n + i]);
            Z[(size_t)i * n + j] = Z[(size_t)j * n + i] = s;
        }
    jacobi_eig(n, Z, wj, Vj);
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return wj[a] > wj[b]; });
    for (int j = 0; j < n; ++j) {
        w[j] = wj[ord[j]];
        for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = Vj[(size_t)i * n + ord[j]];
    }
}

void sym_eig(int n, const double *A, double *w, double *V) {
    if (n == 0) return;
    if (n == 1) {
        w[0] = A[0];
        V[0] = 1.0;
        return;
    }
    std::vector<double> Z(A, A + (size_t)n * n);
    for (double x : Z)
        if (!std::isfinite(x)) throw std::runtime_error("eigensolver: non-finite input");
    // symmetrise (callers pass symmetric matrices up to rounding)
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double s = 0.5 * (Z[(size_t)i * n + j] + Z[(size_t)j * n + i]);
            Z[(size_t)i * n + j] = Z[(size_t)j * n + i] = s;
        }
    std::vector<double> d, e;
    const std::vector<double> Asym = Z;
    tridiagonalize(n, Z, d, e);
    std::vector<double> Zt((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Zt[(size_t)j * n + i] = Z[(size_t)i * n + j];
    try {
        tridiag_ql(n, d, e, Zt);
    } catch (const std::runtime_error &) {
        // QL stalled: cyclic Jacobi on the symmetrised input
        sym_eig_jacobi(n, Asym.data(), w, V);
        return;
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] > d[b]; });
    for (int j = 0; j < n; ++j) {
        w[j] = d[ord[j]];
        const double *zc = &Zt[(size_t)ord[j] * n];
        for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = zc[i];
    }
}

namespace {

// Eigenvectors of the symmetric tridiagonal T (d0, e0; e0[i] = T(i, i+1))
// for the eigenvalues lam0[0..r) by inverse iteration: (T - sigma I) x = b by
// Gaussian elimination with partial pivoting (U with two superdiagonals),
// three solves from a fixed start vector.  Eigenvalues closer than 1e-3 |T|
// form a cluster: their shifts are kept apart by 10 eps |T| and each solve
// is orthogonalised against the cluster's earlier vectors (modified
// Gram-Schmidt).  Y is n x r row-major.
void tridiag_inverse_iteration(int n, const std::vector<double> &d0, const std::vector<double> &e0,
                               const double *lam0, int r, std::vector<double> &Y) {
    const double eps = std::numeric_limits<double>::epsilon();
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i)
        tnorm = std::max(tnorm, std::fabs(d0[i]) + (i > 0 ? std::fabs(e0[i - 1]) : 0.0) +
                                    (i + 1 < n ? std::fabs(e0[i]) : 0.0));
    // T / |T| (the vectors do not change), so that the solves' growth of up
    // to 1 / eps cannot overflow a sum of squares
    const double sc = tnorm > 0.0 ? 1.0 / tnorm : 1.0;
    std::vector<double> d(n), e(n), lamv(r);
    for (int i = 0; i < n; ++i) {
        d[i] = d0[i] * sc;
        e[i] = e0[i] * sc;
    }
    for (int j = 0; j < r; ++j) lamv[j] = lam0[j] * sc;
    const double *lam = lamv.data();
    const double eps3 = eps;
    const double ortol = 1e-3;
    Y.assign((size_t)n * r, 0.0);
    std::vector<double> u0(n), u1(n), u2(n), mult(n), x(n), b(n);
    std::vector<char> swp(n);
    double sigma_prev = 0.0;
    int c0 = 0;  // first index of the current cluster
    for (int j = 0; j < r; ++j) {
        double sigma = lam[j];
        if (j > 0 && lam[j - 1] - lam[j] < ortol) {
            sigma = std::min(sigma, sigma_prev - 10.0 * eps3);
        } else {
            c0 = j;
        }
        sigma_prev = sigma;
        // T - sigma I = P L U
        double a = d[0] - sigma, bb = n > 1 ? e[0] : 0.0;
        for (int i = 0; i + 1 < n; ++i) {
            const double ei = e[i], dn = d[i + 1] - sigma, en = i + 2 < n ? e[i + 1] : 0.0;
            if (std::fabs(a) >= std::fabs(ei)) {
                swp[i] = 0;
                if (a == 0.0) a = eps3;
                u0[i] = a;
                u1[i] = bb;
                u2[i] = 0.0;
                mult[i] = ei / a;
                a = dn - mult[i] * bb;
                bb = en;
            } else {
                swp[i] = 1;
                u0[i] = ei;
                u1[i] = dn;
                u2[i] = en;
                mult[i] = a / ei;
                a = bb - mult[i] * dn;
                bb = -mult[i] * en;
            }
        }
        if (a == 0.0) a = eps3;
        u0[n - 1] = a;
        // fixed start vector (a small linear congruential sequence)
        uint64_t st = 0x9e3779b97f4a7c15ull * (uint64_t)(j + 1);
        for (int i = 0; i < n; ++i) {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            b[i] = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        }
        for (int it = 0; it < 3; ++it) {
            // L^{-1} with the row swaps, then U x = y
            for (int i = 0; i + 1 < n; ++i) {
                if (swp[i]) std::swap(b[i], b[i + 1]);
                b[i + 1] -= mult[i] * b[i];
            }
            for (int i = n - 1; i >= 0; --i) {
                double s = b[i];
                if (i + 1 < n) s -= u1[i] * x[i + 1];
                if (i + 2 < n) s -= u2[i] * x[i + 2];
                x[i] = s / u0[i];
            }
            for (int k = c0; k < j; ++k) {
                double dot = 0.0;
                for (int i = 0; i < n; ++i) dot += x[i] * Y[(size_t)i * r + k];
                for (int i = 0; i < n; ++i) x[i] -= dot * Y[(size_t)i * r + k];
            }
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) nrm += x[i] * x[i];
            nrm = std::sqrt(nrm);
            if (!(nrm > 0.0) || !std::isfinite(nrm)) break;
            for (int i = 0; i < n; ++i) b[i] = x[i] / nrm;
        }
        for (int i = 0; i < n; ++i) Y[(size_t)i * r + j] = b[i];
    }
}

}  // namespace

void top_eigvecs(int n, const double *A, int r, double *Vr, double *wr) {
    auto full = [&] {
        std::vector<double> w(n), V((size_t)n * n);
        sym_eig(n, A, w.data(), V.data());
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < r; ++j) Vr[(size_t)i * r + j] = V[(size_t)i * n + j];
        if (wr)
            for (int j = 0; j < r; ++j) wr[j] = w[j];
    };
    // small orders, or most of the spectrum wanted: the full decomposition
    if (n < kTopEigMin || 2 * r > n) return full();
    // Householder reduction (reflectors kept), eigenvalues alone by the QL
    // iteration, the r wanted vectors of T by inverse iteration, then back
    // through the reflectors: 4/3 n^3 + O(n^2 r) instead of the ~6 n^3 of
    // accumulating every rotation into n vectors
    std::vector<double> Z(A, A + (size_t)n * n);
    for (double x : Z)
        if (!std::isfinite(x)) throw std::runtime_error("eigensolver: non-finite input");
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double s = 0.5 * (Z[(size_t)i * n + j] + Z[(size_t)j * n + i]);
            Z[(size_t)i * n + j] = Z[(size_t)j * n + i] = s;
        }
    const std::vector<double> Asym = Z;
    std::vector<double> d, e, none;
    std::vector<std::vector<double>> vs;
    tridiag_reduce(n, Z, d, e, vs);
    std::vector<double> dq = d, eq = e;
    try {
        tridiag_ql(n, dq, eq, none, false);
    } catch (const std::runtime_error &) {
        return full();
    }
    std::sort(dq.begin(), dq.end(), std::greater<double>());
    std::vector<double> Y;
    tridiag_inverse_iteration(n, d, e, dq.data(), r, Y);
    // X = H_0 (H_1 (... H_{n-3} Y)), a reflector at a time over whole rows
    std::vector<double> sv(r);
    for (int k = (int)vs.size() - 1; k >= 0; --k) {
        const auto &v = vs[k];
        if (v.empty()) continue;
        const int len = n - k - 1;
        std::fill(sv.begin(), sv.end(), 0.0);
        for (int i = 0; i < len; ++i) {
            const double vi = v[i];
            const double *yr = &Y[(size_t)(k + 1 + i) * r];
            for (int j = 0; j < r; ++j) sv[j] += vi * yr[j];
        }
        for (int i = 0; i < len; ++i) {
            const double vi2 = 2.0 * v[i];
            double *yr = &Y[(size_t)(k + 1 + i) * r];
            for (int j = 0; j < r; ++j) yr[j] -= vi2 * sv[j];
        }
    }
    // accept only eigenpairs of the input to working accuracy: residuals
    // |A x - lam x| and the departure from orthonormality within
    // 64 n eps (relative to max_i sum_j |A(i, j)|); else the full solver
    const double eps = std::numeric_limits<double>::epsilon();
    double anorm = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += std::fabs(Asym[(size_t)i * n + j]);
        anorm = std::max(anorm, s);
    }
    const double tol = 64.0 * n * eps;
    std::vector<double> AY((size_t)n * r);
    dgemm(false, false, n, r, n, 1.0, Asym.data(), n, Y.data(), r, 0.0, AY.data(), r);
    for (int j = 0; j < r; ++j) {
        double rn = 0.0;
        for (int i = 0; i < n; ++i) {
            const double ri = AY[(size_t)i * r + j] - dq[j] * Y[(size_t)i * r + j];
            rn += ri * ri;
        }
        if (!(std::sqrt(rn) <= tol * std::max(anorm, std::numeric_limits<double>::min())))
            return full();
        for (int k = 0; k <= j; ++k) {
            double o = 0.0;
            for (int i = 0; i < n; ++i) o += Y[(size_t)i * r + j] * Y[(size_t)i * r + k];
            if (!(std::fabs(o - (k == j ? 1.0 : 0.0)) <= tol)) return full();
        }
    }
    std::copy(Y.begin(), Y.end(), Vr);
    if (wr)
        for (int j = 0; j < r; ++j) wr[j] = dq[j];
}

bool cholesky(int n, double *A, double *fail_pivot) {
    // Blocked right-looking A = U^T U on the upper triangle (row j of U
    // contiguous): factor the rows of one diagonal block (row AXPYs inside
    // the block), update the trailing upper triangle with dgemm; the lower
    // triangle is cleared.  Both triangular solves then read rows of U.
    constexpr int NB = 48, RB = 64;
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int r0 = std::min(n, j0 + NB), jb = r0 - j0;
        for (int j = j0; j < r0; ++j) {
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
            for (int i = j + 1; i < r0; ++i) {
                const double f = uj[i];
                if (f == 0.0) continue;
                double *ai = &A[(size_t)i * n];
                for (int k = i; k < n; ++k) ai[k] -= f * uj[k];
            }
        }
        if (r0 < n) {
            // A(i, k) -= sum_{t in block} U(t, i) U(t, k), rows in panels of RB
            const int nrb = (n - r0 + RB - 1) / RB;
            parallel_for(nrb, [&](int b) {
                const int i0 = r0 + b * RB, i1 = std::min(n, i0 + RB);
                dgemm(true, false, i1 - i0, n - i0, jb, -1.0, &A[(size_t)j0 * n + i0], n,
                      &A[(size_t)j0 * n + i0], n, 1.0, &A[(size_t)i0 * n + i0], n);
            });
        }
    }
    for (int i = 0; i < n; ++i) std::fill(A + (size_t)i * n, A + (size_t)i * n + i, 0.0);
    return true;
}

void chol_solve(int n, const double *U, double *b) {
    // U^T y = b by columns of U^T (rows of U), then U x = y by rows of U
    for (int k = 0; k < n; ++k) {
        const double *uk = &U[(size_t)k * n];
        const double yk = b[k] / uk[k];
        b[k] = yk;
        for (int i = k + 1; i < n; ++i) b[i] -= yk * uk[i];
    }
    for (int i = n - 1; i >= 0; --i) {
        const double *ui = &U[(size_t)i * n];
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= ui[k] * b[k];
        b[i] = s / ui[i];
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

// ---------------------------------------------------------------- threads
namespace {
thread_local int t_threads = 0;
thread_local bool t_in_pool = false;

int default_threads() {
    if (const char *e = std::getenv("BKS_HOST_THREADS")) {
        const int v = std::atoi(e);
        if (v > 0) return v;
    }
    const int hw = (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(hw > 0 ? hw : 1, 8));
}

// A persistent pool of workers that runs one index loop at a time; the
// caller works on the loop too.  A caller that finds the pool busy (another
// host thread's loop) or is itself inside a loop runs its loop inline, so
// the host is never oversubscribed.  The pool lives until the process ends.
struct Pool {
    std::mutex run_mu, mu;
    std::condition_variable cv_work, cv_done;
    const std::function<void(int)> *job = nullptr;
    int n = 0, pending = 0;
    std::atomic<int> next{0};
    uint64_t gen = 0;
    int nworkers = 0;

    explicit Pool(int nw) : nworkers(nw) {
        for (int w = 0; w < nw; ++w) std::thread([this] { loop(); }).detach();
    }
    void loop() {
        t_in_pool = true;
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int)> *f;
            int cnt;
            {
                std::unique_lock<std::mutex> g(mu);
                cv_work.wait(g, [&] { return gen != seen; });
                seen = gen;
                f = job;
                cnt = n;
            }
            for (int i; (i = next.fetch_add(1)) < cnt;) (*f)(i);
            std::lock_guard<std::mutex> g(mu);
            if (--pending == 0) cv_done.notify_one();
        }
    }
    void run(int cnt, const std::function<void(int)> &f) {
        {
            std::lock_guard<std::mutex> g(mu);
            job = &f;
            n = cnt;
            next = 0;
            pending = nworkers;
            ++gen;
        }
        cv_work.notify_all();
        t_in_pool = true;
        for (int i; (i = next.fetch_add(1)) < cnt;) f(i);
        t_in_pool = false;
        std::unique_lock<std::mutex> g(mu);
        cv_done.wait(g, [&] { return pending == 0; });
    }
};

Pool *pool() {
    static Pool *p = new Pool(std::max(0, default_threads() - 1));
    return p;
}
}  // namespace

void set_threads(int n) { t_threads = n; }

int threads() {
    if (t_threads > 0) return t_threads;
    static const int def = default_threads();
    return def;
}

void parallel_for(int n, const std::function<void(int)> &fn) {
    if (n <= 0) return;
    Pool *p = (n > 1 && threads() > 1 && !t_in_pool) ? pool() : nullptr;
    if (p && p->nworkers > 0 && p->run_mu.try_lock()) {
        p->run(n, fn);
        p->run_mu.unlock();
        return;
    }
    for (int i = 0; i < n; ++i) fn(i);
}

// ---------------------------------------------------------------- dgemm
namespace {

constexpr int MR = 4, NR = 8;

// acc(4 x 8) = sum_l a(l, 0:4)^T b(l, 0:8), l in order; a(l, r) at
// Ap[l * sa + r], b(l, c) at Bp[l * sb + c]
inline void micro_4x8(int k, const double *Ap, int sa, const double *Bp, int sb, double *acc) {
    __m256d c0a = _mm256_setzero_pd(), c0b = _mm256_setzero_pd();
    __m256d c1a = _mm256_setzero_pd(), c1b = _mm256_setzero_pd();
    __m256d c2a = _mm256_setzero_pd(), c2b = _mm256_setzero_pd();
    __m256d c3a = _mm256_setzero_pd(), c3b = _mm256_setzero_pd();
    for (int l = 0; l < k; ++l) {
        const double *bl = Bp + (size_t)l * sb, *al = Ap + (size_t)l * sa;
        const __m256d b0 = _mm256_loadu_pd(bl), b1 = _mm256_loadu_pd(bl + 4);
        __m256d a = _mm256_broadcast_sd(al);
        c0a = _mm256_fmadd_pd(a, b0, c0a);
        c0b = _mm256_fmadd_pd(a, b1, c0b);
        a = _mm256_broadcast_sd(al + 1);
        c1a = _mm256_fmadd_pd(a, b0, c1a);
        c1b = _mm256_fmadd_pd(a, b1, c1b);
        a = _mm256_broadcast_sd(al + 2);
        c2a = _mm256_fmadd_pd(a, b0, c2a);
        c2b = _mm256_fmadd_pd(a, b1, c2b);
        a = _mm256_broadcast_sd(al + 3);
        c3a = _mm256_fmadd_pd(a, b0, c3a);
        c3b = _mm256_fmadd_pd(a, b1, c3b);
    }
    _mm256_storeu_pd(acc + 0, c0a);
    _mm256_storeu_pd(acc + 4, c0b);
    _mm256_storeu_pd(acc + 8, c1a);
    _mm256_storeu_pd(acc + 12, c1b);
    _mm256_storeu_pd(acc + 16, c2a);
    _mm256_storeu_pd(acc + 20, c2b);
    _mm256_storeu_pd(acc + 24, c3a);
    _mm256_storeu_pd(acc + 28, c3b);
}

}  // namespace

void dgemm(bool ta, bool tb, int m, int n, int k, double alpha, const double *A, int lda,
           const double *B, int ldb, double beta, double *C, int ldc, bool parallel) {
    if (m <= 0 || n <= 0) return;
    if (k <= 0 || alpha == 0.0) {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j)
                C[(size_t)i * ldc + j] = beta == 0.0 ? 0.0 : beta * C[(size_t)i * ldc + j];
        return;
    }
    const int mp = (m + MR - 1) / MR, np = (n + NR - 1) / NR;
    // A panel ip holds rows ip*MR.. of op(A) as a(l, r); B panel jp holds
    // columns jp*NR.. of op(B) as b(l, c).  Full panels of A^T (ta) and of a
    // row-major B (!tb) are read in place; the others are packed.
    auto a_at = [&](int i, int l) {
        return ta ? A[(size_t)l * lda + i] : A[(size_t)i * lda + l];
    };
    auto b_at = [&](int l, int j) {
        return tb ? B[(size_t)j * ldb + l] : B[(size_t)l * ldb + j];
    };
    std::vector<const double *> ap(mp), bp(np);
    std::vector<int> as(mp), bs(np);
    int npa = 0, npb = 0;
    for (int ip = 0; ip < mp; ++ip)
        if (!(ta && ip * MR + MR <= m)) ++npa;
    for (int jp = 0; jp < np; ++jp)
        if (!(!tb && jp * NR + NR <= n)) ++npb;
    std::vector<double> Apk((size_t)npa * k * MR), Bpk((size_t)npb * k * NR);
    for (int ip = 0, q = 0; ip < mp; ++ip) {
        if (ta && ip * MR + MR <= m) {
            ap[ip] = A + ip * MR;
            as[ip] = lda;
            continue;
        }
        double *dst = &Apk[(size_t)q++ * k * MR];
        for (int l = 0; l < k; ++l)
            for (int r = 0; r < MR; ++r) {
                const int i = ip * MR + r;
                dst[(size_t)l * MR + r] = i < m ? a_at(i, l) : 0.0;
            }
        ap[ip] = dst;
        as[ip] = MR;
    }
    for (int jp = 0, q = 0; jp < np; ++jp) {
        if (!tb && jp * NR + NR <= n) {
            bp[jp] = B + jp * NR;
            bs[jp] = ldb;
            continue;
        }
        double *dst = &Bpk[(size_t)q++ * k * NR];
        for (int l = 0; l < k; ++l)
            for (int c = 0; c < NR; ++c) {
                const int j = jp * NR + c;
                dst[(size_t)l * NR + c] = j < n ? b_at(l, j) : 0.0;
            }
        bp[jp] = dst;
        bs[jp] = NR;
    }
    auto tile = [&](int ip, int jp) {
        alignas(32) double acc[MR * NR];
        micro_4x8(k, ap[ip], as[ip], bp[jp], bs[jp], acc);
        const int i0 = ip * MR, j0 = jp * NR;
        if (i0 + MR <= m && j0 + NR <= n) {
            for (int r = 0; r < MR; ++r) {
                double *ci = C + (size_t)(i0 + r) * ldc + j0;
                const double *ar = acc + r * NR;
                if (beta == 0.0)
                    for (int c = 0; c < NR; ++c) ci[c] = alpha * ar[c];
                else
                    for (int c = 0; c < NR; ++c) ci[c] = beta * ci[c] + alpha * ar[c];
            }
            return;
        }
        for (int r = 0; r < MR; ++r) {
            const int i = i0 + r;
            if (i >= m) break;
            double *ci = C + (size_t)i * ldc;
            for (int c = 0; c < NR; ++c) {
                const int j = j0 + c;
                if (j >= n) break;
                const double v = alpha * acc[r * NR + c];
                ci[j] = beta == 0.0 ? v : beta * ci[j] + v;
            }
        }
    };
    // parallel tasks: groups of row panels (at most ~4 tasks per thread), or
    // single tiles when there are few row panels
    if (parallel && (double)m * n * k > 2e5 && threads() > 1) {
        const int want = 4 * threads();
        if (mp >= want / 2) {
            const int per = (mp + want - 1) / want;
            parallel_for((mp + per - 1) / per, [&](int t) {
                for (int ip = t * per; ip < std::min(mp, t * per + per); ++ip)
                    for (int jp = 0; jp < np; ++jp) tile(ip, jp);
            });
        } else {
            parallel_for(mp * np, [&](int t) { tile(t / np, t % np); });
        }
        return;
    }
    for (int ip = 0; ip < mp; ++ip)
        for (int jp = 0; jp < np; ++jp) tile(ip, jp);
}

}  // namespace la
}  // namespace bks
