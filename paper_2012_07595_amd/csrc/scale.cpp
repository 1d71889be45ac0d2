// Slice scalings applied at upload (host logic): see scale.h.
#include "scale.h"

#include <algorithm>
#include <cmath>
#include <vector>

#include "linalg.h"

namespace bks {

double sym_frobenius(int64_t cnt, const int64_t *lo, const int64_t *hi, const double *v) {
    double s = 0.0;
    for (int64_t e = 0; e < cnt; ++e) s += (lo[e] == hi[e] ? 1.0 : 2.0) * v[e] * v[e];
    return std::sqrt(s);
}

double sym_spectral_radius(int64_t cnt, const int64_t *lo, const int64_t *hi, const double *v) {
    if (cnt == 0) return 0.0;
    std::vector<int64_t> rows(lo, lo + cnt);
    rows.insert(rows.end(), hi, hi + cnt);
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    const int d = (int)rows.size();
    auto loc = [&](int64_t r) {
        return (int)(std::lower_bound(rows.begin(), rows.end(), r) - rows.begin());
    };
    if (d <= kDenseRows) {
        std::vector<double> A((size_t)d * d, 0.0), w(d), V((size_t)d * d);
        for (int64_t e = 0; e < cnt; ++e) {
            const int a = loc(lo[e]), b = loc(hi[e]);
            A[(size_t)a * d + b] += v[e];
            if (a != b) A[(size_t)b * d + a] += v[e];
        }
        la::sym_eig(d, A.data(), w.data(), V.data());
        return std::max(std::fabs(w[0]), std::fabs(w[d - 1]));
    }
    // local CSR over both orientations
    std::vector<int64_t> ptr(d + 1, 0);
    std::vector<int> ra(cnt), rb(cnt);
    for (int64_t e = 0; e < cnt; ++e) {
        ra[e] = loc(lo[e]);
        rb[e] = loc(hi[e]);
        ptr[ra[e] + 1]++;
        if (ra[e] != rb[e]) ptr[rb[e] + 1]++;
    }
    for (int r = 0; r < d; ++r) ptr[r + 1] += ptr[r];
    std::vector<int> col(ptr[d]);
    std::vector<double> val(ptr[d]);
    {
        std::vector<int64_t> at(ptr.begin(), ptr.end() - 1);
        for (int64_t e = 0; e < cnt; ++e) {
            col[at[ra[e]]] = rb[e];
            val[at[ra[e]]++] = v[e];
            if (ra[e] != rb[e]) {
                col[at[rb[e]]] = ra[e];
                val[at[rb[e]]++] = v[e];
            }
        }
    }
    const int K = std::min(d, kLanczosSteps);
    std::vector<double> Q((size_t)K * d), alpha, beta, w(d);
    // a fixed start with positive entries (it overlaps the Perron vector of
    // a nonnegative slice)
    double nq = 0.0;
    for (int i = 0; i < d; ++i) {
        Q[i] = 1.0 + 0.5 * std::sin(3.7 * (i + 1));
        nq += Q[i] * Q[i];
    }
    nq = std::sqrt(nq);
    for (int i = 0; i < d; ++i) Q[i] /= nq;
    double best = 0.0;
    for (int j = 0; j < K; ++j) {
        const double *q = &Q[(size_t)j * d];
        for (int r = 0; r < d; ++r) {
            double s = 0.0;
            for (int64_t x = ptr[r]; x < ptr[r + 1]; ++x) s += val[x] * q[col[x]];
            w[r] = s;
        }
        double a = 0.0;
        for (int r = 0; r < d; ++r) a += w[r] * q[r];
        alpha.push_back(a);
        // full reorthogonalisation (twice)
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i <= j; ++i) {
                const double *qi = &Q[(size_t)i * d];
                double c = 0.0;
                for (int r = 0; r < d; ++r) c += w[r] * qi[r];
                for (int r = 0; r < d; ++r) w[r] -= c * qi[r];
            }
        double b = 0.0;
        for (int r = 0; r < d; ++r) b += w[r] * w[r];
        b = std::sqrt(b);
        const bool last = j + 1 == K || b == 0.0;
        if (j % 8 == 7 || last) {
            // Ritz values of the tridiagonal T_j
            const int n = j + 1;
            std::vector<double> T((size_t)n * n, 0.0), th(n), S((size_t)n * n);
            for (int i = 0; i < n; ++i) {
                T[(size_t)i * n + i] = alpha[i];
                if (i + 1 < n) T[(size_t)i * n + i + 1] = T[(size_t)(i + 1) * n + i] = beta[i];
            }
            la::sym_eig(n, T.data(), th.data(), S.data());
            const int x = std::fabs(th[0]) >= std::fabs(th[n - 1]) ? 0 : n - 1;
            best = std::fabs(th[x]);
            // residual of the Ritz pair: beta_j |last component of its vector|
            const double res = b * std::fabs(S[(size_t)(n - 1) * n + x]);
            if (last || res <= 1e-14 * best) break;
        }
        beta.push_back(b);
        double *qn = &Q[(size_t)(j + 1) * d];
        for (int r = 0; r < d; ++r) qn[r] = w[r] / b;
    }
    return best;
}

}  // namespace bks
