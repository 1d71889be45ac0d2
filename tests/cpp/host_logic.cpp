// Host-logic checks of libbks (no GPU): work schedules and the partial-row
// reduction tree, and the host dense kernels used by the inner solve.
// Prints one "ok <check>" line per passed check; exits 1 on the first failure.
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "inner.h"
#include "linalg.h"
#include "scale.h"
#include "schedule.h"

using namespace bks;

static void require(bool c, const char *what) {
    if (!c) {
        std::printf("FAIL %s\n", what);
        std::exit(1);
    }
}

static std::vector<int64_t> random_segptr(std::mt19937_64 &g, int nseg) {
    std::vector<int64_t> sp(nseg + 1, 0);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int s = 0; s < nseg; ++s) {
        const double x = u(g);
        int64_t len = x < 0.15 ? 0 : x < 0.7 ? (int64_t)(u(g) * 48) : x < 0.95 ? (int64_t)(u(g) * 5000)
                                                                            : (int64_t)(u(g) * 300000);
        sp[s + 1] = sp[s] + len;
    }
    return sp;
}

static void check_schedule() {
    std::mt19937_64 g(7);
    for (int E : {1, 3, 12, 21, 64}) {
        const auto sp = random_segptr(g, 3000);
        const int64_t nseg = (int64_t)sp.size() - 1;
        std::vector<Item> items;
        std::vector<Fixup> fix;
        int64_t nslots = 0;
        build_schedule(sp, E, items, fix, nslots);
        std::vector<int> covered(sp.back(), 0);
        std::vector<int> seg_done(nseg, 0);
        std::vector<int> slot_seen(nslots, 0);
        const int64_t CH = std::max<int64_t>((int64_t)E * kHeavySteps, 2048);
        for (const Item &it : items) {
            if (it.seg_end < 0) {
                require(it.beg < it.end && it.end - it.beg <= CH, "heavy chunk size");
                require(it.beg >= sp[it.seg] && it.end <= sp[it.seg + 1], "heavy chunk in segment");
                for (int64_t e = it.beg; e < it.end; ++e) covered[e]++;
                if (it.slot >= 0) {
                    require(it.slot < nslots && !slot_seen[it.slot], "slot unique");
                    slot_seen[it.slot] = 1;
                } else {
                    require(it.beg == sp[it.seg] && it.end == sp[it.seg + 1], "unsplit heavy whole");
                    seg_done[it.seg]++;
                }
            } else {
                require(it.seg_end > it.seg && it.seg_end - it.seg <= E, "light run size");
                for (int64_t s = it.seg; s < it.seg_end; ++s) {
                    require(sp[s + 1] - sp[s] <= kLightMax, "light segment short");
                    for (int64_t e = sp[s]; e < sp[s + 1]; ++e) covered[e]++;
                    seg_done[s]++;
                }
            }
        }
        for (const Fixup &f : fix) {
            int64_t n = 0;
            for (int32_t x = 0; x < f.nslots; ++x) {
                require(slot_seen[f.first_slot + x] == 1, "fixup slots are chunk slots");
                slot_seen[f.first_slot + x] = 2;
                ++n;
            }
            require(n >= 2, "split segments have several chunks");
            seg_done[f.seg]++;
        }
        for (int64_t e = 0; e < sp.back(); ++e) require(covered[e] == 1, "every entry exactly once");
        for (int64_t s = 0; s < nseg; ++s)
            require(seg_done[s] == 1 || sp[s + 1] == sp[s], "every nonempty segment written once");
        for (int64_t x = 0; x < nslots; ++x) require(slot_seen[x] == 2, "every slot summed");
    }
    std::printf("ok schedule\n");
}

// Group schedules of the register-direct kernel: every entry exactly once,
// every segment (empty ones included) written once, group widths powers of
// two that hold every segment at <= kGroupLPE entries per lane, 64 / L
// segments at most per light item, heavy chunks equal (+-1) and whole waves.
static void check_group_schedule() {
    std::mt19937_64 g(17);
    for (int rep = 0; rep < 4; ++rep) {
        auto sp = random_segptr(g, 4000);
        if (rep == 3) {
            // many short segments of mixed lengths (pair fibres, pair rows)
            std::uniform_int_distribution<int> len(0, 40);
            for (size_t s = 0; s + 1 < sp.size(); ++s) sp[s + 1] = sp[s] + len(g);
        }
        const int64_t nseg = (int64_t)sp.size() - 1;
        std::vector<Item> items;
        std::vector<Fixup> fix;
        int64_t nslots = 0;
        build_group_schedule(sp, items, fix, nslots);
        std::vector<int> covered(sp.back(), 0), seg_done(nseg, 0), slot_seen(nslots, 0);
        for (const Item &it : items) {
            if (it.seg_end < 0) {
                require(it.pad == 64, "group: heavy items take the whole wave");
                require(sp[it.seg + 1] - sp[it.seg] > 64 * kGroupLPE, "group: heavy only when long");
                require(it.beg < it.end && it.end - it.beg <= kGroupChunk, "group: chunk size");
                require(it.beg >= sp[it.seg] && it.end <= sp[it.seg + 1], "group: chunk in segment");
                for (int64_t e = it.beg; e < it.end; ++e) covered[e]++;
                if (it.slot >= 0) {
                    require(it.slot < nslots && !slot_seen[it.slot], "group: slot unique");
                    slot_seen[it.slot] = 1;
                } else {
                    require(it.beg == sp[it.seg] && it.end == sp[it.seg + 1], "group: whole");
                    seg_done[it.seg]++;
                }
            } else {
                const int L = it.pad;
                require(L >= 1 && L <= 64 && (L & (L - 1)) == 0, "group: L a power of two");
                require(it.seg_end > it.seg && (it.seg_end - it.seg) * L <= 64, "group: 64 / L segments");
                for (int64_t s = it.seg; s < it.seg_end; ++s) {
                    require(sp[s + 1] - sp[s] <= (int64_t)L * kGroupLPE, "group: entries per lane");
                    for (int64_t e = sp[s]; e < sp[s + 1]; ++e) covered[e]++;
                    seg_done[s]++;
                }
            }
        }
        for (const Fixup &f : fix) {
            int64_t lo = INT64_MAX, hi = 0;
            for (int32_t x = 0; x < f.nslots; ++x) {
                require(slot_seen[f.first_slot + x] == 1, "group: fixup slots are chunk slots");
                slot_seen[f.first_slot + x] = 2;
            }
            for (const Item &it : items)
                if (it.seg_end < 0 && it.seg == f.seg) {
                    lo = std::min(lo, it.end - it.beg);
                    hi = std::max(hi, it.end - it.beg);
                }
            require(f.nslots >= 2 && hi - lo <= 1, "group: equal chunks");
            seg_done[f.seg]++;
        }
        for (int64_t e = 0; e < sp.back(); ++e) require(covered[e] == 1, "group: every entry once");
        for (int64_t s = 0; s < nseg; ++s) require(seg_done[s] == 1, "group: every segment once");
        for (int64_t x = 0; x < nslots; ++x) require(slot_seen[x] == 2, "group: every slot summed");
    }
    std::printf("ok group_schedule\n");
}

// Slice scalings: the spectral radius by the dense path and by Lanczos
// (more than kDenseRows touched rows) against a dense eigensolve of the same
// matrix, and the closed form of a complete graph; the Frobenius norm.
static void check_scale() {
    std::mt19937_64 g(23);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int d : {37, 900}) {
        std::vector<int64_t> lo, hi;
        std::vector<double> v;
        std::vector<double> A((size_t)d * d, 0.0);
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b)
                if (u(g) < 12.0 / d || b == a + 1) {
                    const double x = u(g);   // nonnegative, connected (a path)
                    lo.push_back(3 * a + 1); // arbitrary labels
                    hi.push_back(3 * b + 1);
                    v.push_back(x);
                    A[(size_t)a * d + b] = A[(size_t)b * d + a] = x;
                }
        std::vector<double> w(d), V((size_t)d * d);
        la::sym_eig(d, A.data(), w.data(), V.data());
        const double want = std::max(std::fabs(w[0]), std::fabs(w[d - 1]));
        const double got = sym_spectral_radius((int64_t)v.size(), lo.data(), hi.data(), v.data());
        require(std::fabs(got - want) <= 1e-12 * want, "scale: spectral radius");
        double f = 0.0;
        for (double x : A) f += x * x;
        require(std::fabs(sym_frobenius((int64_t)v.size(), lo.data(), hi.data(), v.data()) -
                          std::sqrt(f)) <= 1e-13 * std::sqrt(f), "scale: frobenius");
    }
    // c K_q: largest eigenvalue c (q - 1); 500 nodes takes the Lanczos path
    for (int q : {9, 500}) {
        std::vector<int64_t> lo, hi;
        std::vector<double> v;
        for (int a = 0; a < q; ++a)
            for (int b = a + 1; b < q; ++b) {
                lo.push_back(a);
                hi.push_back(b);
                v.push_back(2.5);
            }
        const double got = sym_spectral_radius((int64_t)v.size(), lo.data(), hi.data(), v.data());
        require(std::fabs(got - 2.5 * (q - 1)) <= 1e-12 * 2.5 * (q - 1), "scale: complete graph");
    }
    require(sym_spectral_radius(0, nullptr, nullptr, nullptr) == 0.0, "scale: empty");
    std::printf("ok scale\n");
}

static void check_wide_schedule() {
    std::mt19937_64 g(9);
    const auto sp = random_segptr(g, 500);
    for (int CW : {300, 2048, 10000}) {
        std::vector<Item> items;
        std::vector<Fixup> fix;
        int64_t nslots = 0;
        build_wide_schedule(sp, CW, items, fix, nslots);
        require((int64_t)fix.size() == (int64_t)sp.size() - 1, "one fix per slice");
        require(nslots == (int64_t)items.size(), "slot per item");
        std::vector<int> covered(sp.back(), 0);
        for (size_t q = 0; q < items.size(); ++q) {
            const Item &it = items[q];
            require(it.slot == (int32_t)q && it.end - it.beg <= CW + CW / 2 + 1 && it.beg < it.end,
                    "wide item");
            for (int64_t e = it.beg; e < it.end; ++e) covered[e]++;
        }
        for (const Fixup &f : fix) {
            const int64_t len = sp[f.seg + 1] - sp[f.seg];
            require(f.nslots == (len == 0 ? 0 : std::max<int64_t>(1, (len + CW / 2) / CW)),
                    "wide: round(len / CW) chunks");
            int64_t lo = len, hi = 0;
            for (int32_t x = 0; x < f.nslots; ++x) {
                const Item &it = items[f.first_slot + x];
                require(it.seg == f.seg, "fix lists the slice's items");
                lo = std::min(lo, it.end - it.beg);
                hi = std::max(hi, it.end - it.beg);
            }
            require(f.nslots < 2 || (hi - lo <= 1 && lo >= CW / 2), "wide: equal chunks");
        }
        for (int64_t e = 0; e < sp.back(); ++e) require(covered[e] == 1, "wide: every entry once");
    }
    std::printf("ok wide_schedule\n");
}

static void check_fix_tree() {
    std::mt19937_64 g(11);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    std::vector<Fixup> fix;
    int64_t nslots = 0;
    const int counts[] = {2, 64, 65, 127, 4096, 4097, 300000, 5};
    for (int s = 0; s < 8; ++s) {
        fix.push_back({s, (int32_t)nslots, counts[s], 0});
        nslots += counts[s];
    }
    const int64_t base = nslots;
    std::vector<double> val(nslots);
    for (double &v : val) v = u(g);
    std::vector<double> direct(8, 0.0);
    for (const Fixup &f : fix)
        for (int32_t x = 0; x < f.nslots; ++x) direct[f.seg] += val[f.first_slot + x];
    std::vector<std::vector<Fixup>> levels;
    build_fix_tree(fix, nslots, levels);
    require(nslots > base, "tree adds slots");
    val.resize(nslots, NAN);
    for (const auto &lv : levels) {
        for (const Fixup &f : lv) {
            require(f.nslots <= kFixFan && f.seg >= base && f.seg < nslots, "level fixup");
            double s = 0.0;
            for (int32_t x = 0; x < f.nslots; ++x) {
                require(f.first_slot + x < f.seg, "reads precede the slot written");
                s += val[f.first_slot + x];
            }
            val[f.seg] = s;
        }
    }
    for (const Fixup &f : fix) {
        require(f.nslots <= kFixFan, "final fixups are shallow");
        double s = 0.0;
        for (int32_t x = 0; x < f.nslots; ++x) s += val[f.first_slot + x];
        require(std::isfinite(s) && std::fabs(s - direct[f.seg]) <= 1e-9 * (1 + std::fabs(direct[f.seg])),
                "tree sum equals direct sum");
    }
    std::printf("ok fix_tree levels=%zu\n", levels.size());
}

static void check_dgemm() {
    std::mt19937_64 g(13);
    std::normal_distribution<double> nd;
    const int sizes[] = {1, 3, 4, 5, 8, 9, 33, 70};
    for (int m : sizes)
        for (int n : sizes)
            for (int k : {1, 2, 7, 40})
                for (int ta = 0; ta < 2; ++ta)
                    for (int tb = 0; tb < 2; ++tb) {
                        const int lda = (ta ? m : k) + 3, ldb = (tb ? k : n) + 1, ldc = n + 2;
                        std::vector<double> A((size_t)(ta ? k : m) * lda), B((size_t)(tb ? n : k) * ldb),
                            C((size_t)m * ldc), C0;
                        for (double &x : A) x = nd(g);
                        for (double &x : B) x = nd(g);
                        for (double &x : C) x = nd(g);
                        C0 = C;
                        const double alpha = 0.75, beta = (m + n + k) % 2 ? 0.0 : -0.5;
                        la::dgemm(ta, tb, m, n, k, alpha, A.data(), lda, B.data(), ldb, beta, C.data(),
                                  ldc, (m * n * k) % 3 == 0);
                        for (int i = 0; i < m; ++i)
                            for (int j = 0; j < n; ++j) {
                                double s = 0.0, sa = 0.0;
                                for (int l = 0; l < k; ++l) {
                                    const double a = ta ? A[(size_t)l * lda + i] : A[(size_t)i * lda + l];
                                    const double b = tb ? B[(size_t)j * ldb + l] : B[(size_t)l * ldb + j];
                                    s += a * b;
                                    sa += std::fabs(a * b);
                                }
                                const double want = alpha * s + (beta == 0.0 ? 0.0 : beta * C0[(size_t)i * ldc + j]);
                                require(std::fabs(C[(size_t)i * ldc + j] - want) <= 1e-13 * (sa + 1.0),
                                        "dgemm matches the triple loop");
                            }
                        for (int i = 0; i < m; ++i)
                            for (int j = n; j < ldc; ++j)
                                require(C[(size_t)i * ldc + j] == C0[(size_t)i * ldc + j],
                                        "dgemm leaves the padding alone");
                    }
    std::printf("ok dgemm\n");
}

static void check_cholesky_and_threads() {
    std::mt19937_64 g(17);
    std::normal_distribution<double> nd;
    for (int n : {1, 5, 47, 48, 49, 100, 130}) {
        std::vector<double> G((size_t)n * (n + 3)), A((size_t)n * n);
        for (double &x : G) x = nd(g);
        la::dgemm(false, true, n, n, n + 3, 1.0, G.data(), n + 3, G.data(), n + 3, 0.0, A.data(), n);
        std::vector<double> U = A;
        double piv = 0.0;
        require(la::cholesky(n, U.data(), &piv), "SPD factorises");
        double anorm = 0.0;
        for (double x : A) anorm = std::max(anorm, std::fabs(x));
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += U[(size_t)l * n + i] * U[(size_t)l * n + j];
                require(std::fabs(s - A[(size_t)i * n + j]) <= 1e-12 * anorm * n, "U^T U = A");
                if (j < i) require(U[(size_t)i * n + j] == 0.0, "U upper");
            }
        // chol_solve against a known solution
        std::vector<double> x0(n), bb(n, 0.0);
        for (double &x : x0) x = nd(g);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) bb[i] += A[(size_t)i * n + j] * x0[j];
        la::chol_solve(n, U.data(), bb.data());
        double xerr = 0.0, xn = 0.0;
        for (int i = 0; i < n; ++i) {
            xerr = std::max(xerr, std::fabs(bb[i] - x0[i]));
            xn = std::max(xn, std::fabs(x0[i]));
        }
        require(xerr <= 1e-8 * xn, "chol_solve recovers x");
        // thread count does not change a bit
        std::vector<double> L1 = A, L4 = A;
        la::set_threads(1);
        la::cholesky(n, L1.data());
        la::set_threads(4);
        la::cholesky(n, L4.data());
        la::set_threads(0);
        for (size_t x = 0; x < L1.size(); ++x) require(L1[x] == L4[x], "cholesky bitwise across threads");
        // an indefinite matrix is refused with a nonpositive pivot
        std::vector<double> Bm = A;
        for (int i = 0; i < n; ++i) Bm[(size_t)i * n + i] -= 2.0 * anorm * n;
        piv = 1.0;
        require(!la::cholesky(n, Bm.data(), &piv) && piv <= 0.0, "indefinite refused");
    }
    // dgemm across thread counts
    const int m = 90, n = 75, k = 300;
    std::vector<double> A((size_t)m * k), B((size_t)k * n), C1((size_t)m * n), C4((size_t)m * n);
    for (double &x : A) x = nd(g);
    for (double &x : B) x = nd(g);
    la::set_threads(1);
    la::dgemm(false, false, m, n, k, 1.0, A.data(), k, B.data(), n, 0.0, C1.data(), n, true);
    la::set_threads(4);
    la::dgemm(false, false, m, n, k, 1.0, A.data(), k, B.data(), n, 0.0, C4.data(), n, true);
    la::set_threads(0);
    for (size_t x = 0; x < C1.size(); ++x) require(C1[x] == C4[x], "dgemm bitwise across threads");
    std::printf("ok cholesky_threads\n");
}

static void check_eig() {
    std::mt19937_64 g(19);
    std::normal_distribution<double> nd;
    for (int n : {1, 2, 7, 40, 70}) {
        std::vector<double> A((size_t)n * n), w(n), V((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = nd(g);
        la::sym_eig(n, A.data(), w.data(), V.data());
        for (int i = 1; i < n; ++i) require(w[i - 1] >= w[i], "descending eigenvalues");
        // the Jacobi fallback gives the same spectrum and a valid basis
        std::vector<double> wj(n), Vj((size_t)n * n);
        la::sym_eig_jacobi(n, A.data(), wj.data(), Vj.data());
        for (int i = 0; i < n; ++i) {
            require(std::fabs(wj[i] - w[i]) <= 1e-12 * n * std::max(1.0, std::fabs(w[0])),
                    "Jacobi eigenvalues");
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += Vj[(size_t)i * n + l] * wj[l] * Vj[(size_t)j * n + l];
                require(std::fabs(s - A[(size_t)i * n + j]) <= 1e-12 * n, "Jacobi V W V^T = A");
            }
        }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0, o = 0.0;
                for (int l = 0; l < n; ++l) {
                    s += V[(size_t)i * n + l] * w[l] * V[(size_t)j * n + l];
                    o += V[(size_t)l * n + i] * V[(size_t)l * n + j];
                }
                require(std::fabs(s - A[(size_t)i * n + j]) <= 1e-12 * n, "V W V^T = A");
                require(std::fabs(o - (i == j ? 1.0 : 0.0)) <= 1e-12 * n, "V orthogonal");
            }
    }
    // far-from-unit scales and matrices with many zero eigenvalues converge
    // (squares stay normal: the Householder norms are plain sums of squares)
    for (double scale : {1e-150, 1.0, 1e150}) {
        const int n = 30;
        std::vector<double> A((size_t)n * n), w(n), V((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j)
                A[(size_t)i * n + j] = A[(size_t)j * n + i] = scale * nd(g) * (i < 5 && j < 5);
        la::sym_eig(n, A.data(), w.data(), V.data());
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double o = 0.0;
                for (int l = 0; l < n; ++l) o += V[(size_t)l * n + i] * V[(size_t)l * n + j];
                require(std::fabs(o - (i == j ? 1.0 : 0.0)) <= 1e-12 * n, "V orthogonal (scaled)");
            }
        double wmax = 0.0;
        for (double x : w) wmax = std::max(wmax, std::fabs(x));
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += V[(size_t)i * n + l] * w[l] * V[(size_t)j * n + l];
                require(std::fabs(s - A[(size_t)i * n + j]) <= 1e-12 * n * wmax,
                        "V W V^T = A (scaled)");
            }
    }
    std::printf("ok sym_eig\n");
}

// The leading r eigenvectors (reduced path: tridiagonal eigenvalues, inverse
// iteration, back-transformation) against the full decomposition: the same
// eigenvalues, the same projector onto the leading subspace, orthonormal
// columns, small residuals; clustered spectra with the cut beside and inside
// a cluster; extreme scales.
static void check_top_eigvecs() {
    std::mt19937_64 g(31);
    std::normal_distribution<double> nd;
    auto residual_ok = [](int n, const std::vector<double> &A, int r, const std::vector<double> &V,
                          const std::vector<double> &w, double tol) {
        double an = 0.0;
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += std::fabs(A[(size_t)i * n + j]);
            an = std::max(an, s);
        }
        for (int c = 0; c < r; ++c) {
            double rn = 0.0;
            for (int i = 0; i < n; ++i) {
                double s = -w[c] * V[(size_t)i * r + c];
                for (int j = 0; j < n; ++j) s += A[(size_t)i * n + j] * V[(size_t)j * r + c];
                rn += s * s;
            }
            if (!(std::sqrt(rn) <= tol * an)) return false;
            for (int c2 = 0; c2 <= c; ++c2) {
                double o = 0.0;
                for (int i = 0; i < n; ++i) o += V[(size_t)i * r + c] * V[(size_t)i * r + c2];
                if (!(std::fabs(o - (c == c2 ? 1.0 : 0.0)) <= tol)) return false;
            }
        }
        return true;
    };
    auto projector_gap = [](int n, int r, const std::vector<double> &V1, int ld1,
                            const std::vector<double> &V2) {
        double m = 0.0;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                double a = 0.0, b = 0.0;
                for (int j = 0; j < r; ++j) {
                    a += V1[(size_t)i * ld1 + j] * V1[(size_t)k * ld1 + j];
                    b += V2[(size_t)i * r + j] * V2[(size_t)k * r + j];
                }
                m = std::max(m, std::fabs(a - b));
            }
        return m;
    };
    // random symmetric matrices
    for (int n : {24, 31, 70, 190})
        for (int r : {1, 5, 10}) {
            std::vector<double> A((size_t)n * n), w(n), V((size_t)n * n), wr(r), Vr((size_t)n * r);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = nd(g);
            la::sym_eig(n, A.data(), w.data(), V.data());
            la::top_eigvecs(n, A.data(), r, Vr.data(), wr.data());
            const double scale = std::max(std::fabs(w[0]), std::fabs(w[n - 1]));
            for (int j = 0; j < r; ++j)
                require(std::fabs(wr[j] - w[j]) <= 1e-13 * n * scale, "top_eigvecs: eigenvalues");
            require(residual_ok(n, A, r, Vr, wr, 1e-12 * n), "top_eigvecs: residual");
            // the leading subspace is determined up to rounding / gap
            const double gap = (w[r - 1] - w[r]) / scale;
            require(projector_gap(n, r, V, n, Vr) <= 1e-13 * n / std::max(gap, 1e-3),
                    "top_eigvecs: leading subspace");
        }
    // clustered spectra: Q diag(5, 5, 5, 3, 3, 1, ...) Q^T
    for (int n : {40, 100}) {
        std::vector<double> M((size_t)n * n), Q((size_t)n * n), A((size_t)n * n, 0.0);
        for (auto &x : M) x = nd(g);
        la::qr_full(n, n, M.data(), Q.data());
        std::vector<double> lam(n);
        for (int i = 0; i < n; ++i) lam[i] = i < 3 ? 5.0 : i < 5 ? 3.0 : 1.0 / (1.0 + i);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += Q[(size_t)i * n + k] * lam[k] * Q[(size_t)j * n + k];
                A[(size_t)i * n + j] = s;
            }
        for (int r : {2, 3, 5}) {
            std::vector<double> wr(r), Vr((size_t)n * r);
            la::top_eigvecs(n, A.data(), r, Vr.data(), wr.data());
            for (int j = 0; j < r; ++j)
                require(std::fabs(wr[j] - lam[j]) <= 1e-13 * n * 5.0, "top_eigvecs: cluster values");
            require(residual_ok(n, A, r, Vr, wr, 1e-12 * n), "top_eigvecs: cluster residual");
            if (r != 2)  // a cut between clusters fixes the subspace: Q(:, :r)
                require(projector_gap(n, r, Q, n, Vr) <= 1e-12 * n, "top_eigvecs: cluster subspace");
        }
    }
    // far-from-unit scales
    for (double scale : {1e-150, 1e150}) {
        const int n = 60, r = 4;
        std::vector<double> A((size_t)n * n), wr(r), Vr((size_t)n * r), w(n), V((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = scale * nd(g);
        la::sym_eig(n, A.data(), w.data(), V.data());
        la::top_eigvecs(n, A.data(), r, Vr.data(), wr.data());
        for (int j = 0; j < r; ++j)
            require(std::fabs(wr[j] - w[j]) <= 1e-13 * n * std::fabs(w[0]), "top_eigvecs: scaled values");
        require(residual_ok(n, A, r, Vr, wr, 1e-12 * n), "top_eigvecs: scaled residual");
    }
    std::printf("ok top_eigvecs\n");
}

// The device interface of the inner solve, implemented with plain loops from
// its contract (inner.h): the inner solve must reach the same point through
// it as through its own host products.
struct LoopDevice : InnerDevice {
    std::vector<double> C;
    int k1 = 0, k3 = 0;
    int calls = 0, partial_calls = 0;
    double at(int a, int b, int c) const { return C[a + (size_t)k1 * (b + (size_t)k1 * c)]; }
    void set_core(const double *Cp, int k1_, int k3_) override {
        k1 = k1_;
        k3 = k3_;
        C.assign(Cp, Cp + (size_t)k1 * k1 * k3);
    }
    void gram1(double *G1) override {
        ++calls;
        for (int a = 0; a < k1; ++a)
            for (int b = 0; b < k1; ++b) {
                double s = 0.0;
                for (int c = 0; c < k3; ++c)
                    for (int x = 0; x < k1; ++x) s += at(a, x, c) * at(b, x, c);
                G1[(size_t)a * k1 + b] = s;
            }
    }
    void gram3(double *G3) override {
        ++calls;
        for (int c = 0; c < k3; ++c)
            for (int d = 0; d < k3; ++d) {
                double s = 0.0;
                for (int b = 0; b < k1; ++b)
                    for (int a = 0; a < k1; ++a) s += at(a, b, c) * at(a, b, d);
                G3[(size_t)c * k3 + d] = s;
            }
    }
    void mode3p(const double *Sv, int ldS, int l0, int nl, const double *P, int r,
                double *out) override {
        ++calls;
        for (int l = 0; l < nl; ++l)
            for (int j = 0; j < r; ++j)
                for (int a = 0; a < k1; ++a) {
                    double s = 0.0;
                    for (int b = 0; b < k1; ++b) {
                        double cs = 0.0;
                        for (int c = 0; c < k3; ++c) cs += at(a, b, c) * Sv[(size_t)c * ldS + l0 + l];
                        s += cs * P[(size_t)b * r + j];
                    }
                    out[a + (size_t)k1 * (j + (size_t)r * l)] = s;
                }
    }
    void hooi3(const double *P, int r, double *M3) override {
        ++calls;
        for (int c = 0; c < k3; ++c)
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < r; ++j) {
                    double s = 0.0;
                    for (int b = 0; b < k1; ++b)
                        for (int a = 0; a < k1; ++a) s += at(a, b, c) * P[(size_t)a * r + i] * P[(size_t)b * r + j];
                    M3[(size_t)c * r * r + i + r * j] = s;
                }
    }
    void rotate(const double *Qp, const double *Qs, int r, int r3, double *Y, double *Y2,
                bool partial) override {
        ++calls;
        if (partial) {
            // the whole rotation, then the blocks the contract returns
            ++partial_calls;
            std::vector<double> Yf((size_t)k1 * k1 * r3), Y2f((size_t)k1 * r * (k3 - r3));
            rotate(Qp, Qs, r, r3, Yf.data(), Y2f.data(), false);
            for (int l = 0; l < r3; ++l)
                for (int y = 0; y < r; ++y)
                    for (int x = 0; x < k1; ++x)
                        Y[x + (size_t)k1 * (y + (size_t)r * l)] = Yf[x + (size_t)k1 * (y + (size_t)k1 * l)];
            for (int z = 0; z < k3 - r3; ++z)
                for (int j = 0; j < r; ++j)
                    for (int x = 0; x < r; ++x)
                        Y2[x + (size_t)r * (j + (size_t)r * z)] = Y2f[x + (size_t)k1 * (j + (size_t)r * z)];
            return;
        }
        std::vector<double> X((size_t)k1 * k1), T((size_t)k1 * k1);
        for (int l = 0; l < k3; ++l) {
            for (int b = 0; b < k1; ++b)
                for (int a = 0; a < k1; ++a) {
                    double s = 0.0;
                    for (int c = 0; c < k3; ++c) s += at(a, b, c) * Qs[(size_t)c * k3 + l];
                    X[(size_t)a * k1 + b] = s;
                }
            const int ncol = l < r3 ? k1 : r;
            for (int a = 0; a < k1; ++a)  // T = X Qp(:, :ncol)
                for (int y = 0; y < ncol; ++y) {
                    double s = 0.0;
                    for (int b = 0; b < k1; ++b) s += X[(size_t)a * k1 + b] * Qp[(size_t)b * k1 + y];
                    T[(size_t)a * k1 + y] = s;
                }
            for (int x = 0; x < k1; ++x)  // Qp^T T
                for (int y = 0; y < ncol; ++y) {
                    double s = 0.0;
                    for (int a = 0; a < k1; ++a) s += Qp[(size_t)a * k1 + x] * T[(size_t)a * k1 + y];
                    if (l < r3) Y[x + (size_t)k1 * (y + (size_t)k1 * l)] = s;
                    else Y2[x + (size_t)k1 * (y + (size_t)r * (l - r3))] = s;
                }
        }
    }
};

// claims to form the Newton matrix itself (so the inner solve asks for
// partial rotations) but declines each time: the inner solve must then
// rotate again in full and form the matrix on the host
struct DecliningNewtonDevice : LoopDevice {
    bool forms_newton() const override { return true; }
};

static void check_inner_device() {
    // planted core: C = sum_t f_t u_t o u_t o w_t + small symmetric noise
    const int k1 = 30, k3 = 20, r = 3, r3 = 3;
    std::mt19937_64 g(23);
    std::normal_distribution<double> nd;
    std::vector<double> U((size_t)k1 * r), W((size_t)k3 * r3);
    for (double &x : U) x = nd(g);
    for (double &x : W) x = nd(g);
    la::orthonormalize(k1, r, U.data());
    la::orthonormalize(k3, r3, W.data());
    std::vector<double> C((size_t)k1 * k1 * k3);
    for (int c = 0; c < k3; ++c)
        for (int b = 0; b < k1; ++b)
            for (int a = 0; a <= b; ++a) {
                double v = 1e-2 * nd(g);
                for (int t = 0; t < r; ++t)
                    v += (10.0 - 2.0 * t) * U[(size_t)a * r + t] * U[(size_t)b * r + t] * W[(size_t)c * r3 + t];
                C[a + (size_t)k1 * (b + (size_t)k1 * c)] = C[b + (size_t)k1 * (a + (size_t)k1 * c)] = v;
            }
    std::vector<double> P0, S0, P1, S1;
    InnerInfo i0, i1;
    inner_solve(C, k1, k3, r, r3, 1e-13, 5, 50, false, P0, S0, i0);
    LoopDevice dev;
    inner_solve(C, k1, k3, r, r3, 1e-13, 5, 50, false, P1, S1, i1, BigSolve(), &dev, 0.0);
    require(dev.calls > 0, "device path taken");
    require(i0.rel <= 1e-12 && i1.rel <= 1e-12, "both paths converge");
    const double g0 = inner_objective(C, k1, k3, P0, S0, r, r3);
    const double g1 = inner_objective(C, k1, k3, P1, S1, r, r3);
    require(std::fabs(g0 - g1) <= 1e-12 * g0, "same objective through the device interface");
    // same subspace: ||(I - P0 P0^T) P1||_F
    double d2 = 0.0;
    for (int j = 0; j < r; ++j)
        for (int i = 0; i < k1; ++i) {
            double s = P1[(size_t)i * r + j];
            for (int t = 0; t < r; ++t) {
                double pt = 0.0;
                for (int x = 0; x < k1; ++x) pt += P0[(size_t)x * r + t] * P1[(size_t)x * r + j];
                s -= P0[(size_t)i * r + t] * pt;
            }
            d2 += s * s;
        }
    require(std::sqrt(d2) <= 1e-10, "same subspace through the device interface");
    // partial rotations (Newton systems from order 1, a host solver as the
    // large-system solve) give the same solution
    setenv("BKS_DEVICE_SOLVE_MIN", "1", 1);
    const BigSolve hostbig = [](int N, const double *H, double mu, bool, double *b) {
        std::vector<double> A(H, H + (size_t)N * N);
        for (int q = 0; q < N; ++q) A[(size_t)q * N + q] += mu;
        if (!la::cholesky(N, A.data())) return false;
        la::chol_solve(N, A.data(), b);
        return true;
    };
    std::vector<double> P2, S2;
    InnerInfo i2;
    DecliningNewtonDevice devp;
    inner_solve(C, k1, k3, r, r3, 1e-13, 5, 50, false, P2, S2, i2, hostbig, &devp, 0.0);
    require(devp.partial_calls > 0, "partial rotations taken");
    require(i2.rel <= 1e-12, "partial-rotation path converges");
    const double g2 = inner_objective(C, k1, k3, P2, S2, r, r3);
    require(std::fabs(g0 - g2) <= 1e-12 * g0, "same objective with partial rotations");
    double d3 = 0.0;
    for (int j = 0; j < r; ++j)
        for (int q = 0; q < k1; ++q) {
            double s = P2[(size_t)q * r + j];
            for (int u = 0; u < r; ++u) {
                double pt = 0.0;
                for (int x = 0; x < k1; ++x) pt += P0[(size_t)x * r + u] * P2[(size_t)x * r + j];
                s -= P0[(size_t)q * r + u] * pt;
            }
            d3 += s * s;
        }
    require(std::sqrt(d3) <= 1e-10, "same subspace with partial rotations");
    std::printf("ok inner_device calls=%d partial=%d\n", dev.calls, devp.partial_calls);
}

int main() {
    check_schedule();
    check_group_schedule();
    check_scale();
    check_wide_schedule();
    check_fix_tree();
    check_dgemm();
    check_cholesky_and_threads();
    check_eig();
    check_top_eigvecs();
    check_inner_device();
    return 0;
}
