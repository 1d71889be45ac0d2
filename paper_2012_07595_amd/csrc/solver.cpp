// Block Krylov-Schur (Algorithm 5, symmetric case U = V) and symmetric HOOI
// (section "Higher Order Orthogonal Iteration") driven from the host; every product with the large tensor
// and every tall-skinny operation runs on the device, the small projected
// problems on the host in FP64.
//
// Precision modes
//   FP64:  every tensor product in FP64; the gradient-defining slices of the
//          core are taken from the step-(iii) products as below.
//   MIXED: block-Krylov expansion products and the core product A.(X, X)_{1,2}
//          in FP32; the step-(iii) products T1 = A.(U0, W0)_{2,3} and
//          T3 = A.(U0, U0)_{1,2} with FP32 values, FP64 factors and FP64
//          accumulation.  By Proposition 3.2 and Lemma 3.1 the G-gradient
//          of the projected problem at the restart point depends only on the
//          slices C(:, U0, W0) = X^T T1 and C(U0, U0, :) = Z^T T3, so those
//          slices of the FP32-formed core are overwritten with FP64-accurate
//          ones: a stationary point of the full problem is then an exact
//          fixed point of the mixed iteration.  The basis itself is always
//          kept and orthogonalised in FP64 (with an FP32 shadow copy feeding
//          the FP32 products).  The other slices carry FP32 rounding, which
//          leaves the gradient wandering at a floor (~1e-11 relative at the
//          C3 shape); once it is below 1e-9 and an outer iteration fails to
//          halve the best value so far, the remaining iterations run their
//          products in FP64 (bks_info.fp64_from).
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>

#include "bks_internal.h"
#include "inner.h"
#include "linalg.h"

namespace bks {

// BKS_DEBUG_INNER=1: one line per inner solve on stderr (iterations, final
// local gradient, phase times)
static bool debug_inner() {
    static const bool on = [] {
        const char *e = std::getenv("BKS_DEBUG_INNER");
        return e && e[0] == '1';
    }();
    return on;
}

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ double-double
struct dd {
    double hi, lo;
};
inline dd dd_from(double a) { return {a, 0.0}; }
inline dd two_sum(double a, double b) {
    double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
inline dd dd_norm(double s, double e) {
    double h = s + e;
    return {h, e - (h - s)};
}
inline dd add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = dd_norm(s.hi, s.lo);
    s.lo += t.lo;
    return dd_norm(s.hi, s.lo);
}
inline dd neg(dd a) { return {-a.hi, -a.lo}; }
inline dd sub(dd a, dd b) { return add(a, neg(b)); }
inline dd mul(dd a, dd b) {
    double p = a.hi * b.hi;
    double e = std::fma(a.hi, b.hi, -p);
    e += a.hi * b.lo + a.lo * b.hi;
    return dd_norm(p, e);
}
inline dd divd(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = sub(a, mul(b, dd_from(q1)));
    double q2 = r.hi / b.hi;
    r = sub(r, mul(b, dd_from(q2)));
    double q3 = r.hi / b.hi;
    return add(dd_norm(q1, q2), dd_from(q3));
}
inline dd sqrtd(dd a) {
    if (a.hi <= 0) return {0, 0};
    double x = std::sqrt(a.hi);
    dd xx = mul(dd_from(x), dd_from(x));
    dd r = sub(a, xx);
    return add(dd_from(x), dd_from(r.hi / (2.0 * x)));
}

// Ordered Cholesky of a DD Gram matrix G (q x q, row-major hi/lo) with
// column dropping; returns kept columns and T (q x q', row-major) with
// Q = B T having orthonormal columns spanning the kept part.
//   drop column c if its residual^2 <= (tau * before_c)^2, or once the basis
//   is full (room columns already kept).
void chol_drop(int q, const std::vector<double> &Ghi, const std::vector<double> &Glo,
               const std::vector<double> &before2, double tau, int room, std::vector<int> &kept,
               std::vector<double> &T) {
    std::vector<dd> G((size_t)q * q);
    for (size_t i = 0; i < G.size(); ++i) G[i] = {Ghi[i], Glo[i]};
    std::vector<dd> R((size_t)q * q, dd{0, 0});
    kept.clear();
    for (int c = 0; c < q; ++c) {
        if ((int)kept.size() >= room) break;
        dd d = G[(size_t)c * q + c];
        for (int e : kept) d = sub(d, mul(R[(size_t)e * q + c], R[(size_t)e * q + c]));
        const double thr = tau * tau * before2[c];
        if (!(d.hi > thr) || d.hi <= 0.0) continue;
        dd rcc = sqrtd(d);
        R[(size_t)c * q + c] = rcc;
        for (int x = c + 1; x < q; ++x) {
            dd s = G[(size_t)c * q + x];
            for (int e : kept) s = sub(s, mul(R[(size_t)e * q + c], R[(size_t)e * q + x]));
            R[(size_t)c * q + x] = divd(s, rcc);
        }
        kept.push_back(c);
    }
    const int k = (int)kept.size();
    // Rk = R(kept, kept) upper triangular; T = Rk^{-1} (DD back substitution)
    std::vector<dd> Ti((size_t)k * k, dd{0, 0});
    for (int j = 0; j < k; ++j) {
        // solve Rk t = e_j
        for (int i = j; i >= 0; --i) {
            dd s = (i == j) ? dd_from(1.0) : dd{0, 0};
            for (int l = i + 1; l <= j; ++l)
                s = sub(s, mul(R[(size_t)kept[i] * q + kept[l]], Ti[(size_t)l * k + j]));
            Ti[(size_t)i * k + j] = divd(s, R[(size_t)kept[i] * q + kept[i]]);
        }
    }
    T.assign((size_t)q * k, 0.0);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) T[(size_t)kept[i] * k + j] = Ti[(size_t)i * k + j].hi + Ti[(size_t)i * k + j].lo;
}

int sym_idx(int a, int b) { return b * (b + 1) / 2 + a; }  // a <= b

struct Solver {
    Ctx &c;
    Tensor &t;
    hipStream_t s;
    int64_t m, n;
    int r, r3, p, stages, variant;
    bool mixed;
    bool fp32;  // expansion and core products in FP32 (mixed, until the floor)
    double tau64 = 1e-14, tau32 = 1e-5;

    int k1cap = 0, k3cap = 0, qcap = 0;
    DevBuf X64, X32, Z64, Z32;
    int k1 = 0, k3 = 0;
    std::vector<int> uoff, uw, woff, ww;
    std::set<std::pair<int, int>> used_u, used_w;

    DevBuf P32, P64, W64a, W64b;  // product / work buffers (rows x qcap)
    DevBuf T1, T3h;               // FP64 step-(iii) products
    DevBuf T3core, Cdev;          // core product and Z^T T3core
    DevBuf Hd, Hd2, Gd;           // small device scratch
    std::vector<double> hbuf;

    Solver(Ctx &c_, Tensor &t_, hipStream_t s_, int r_, int r3_, int p_, int st, int var, bool mx)
        : c(c_), t(t_), s(s_), m(t_.m), n(t_.n), r(r_), r3(r3_), p(p_), stages(st),
          variant(var), mixed(mx), fp32(mx) {}

    // Pinned staging for the small host <-> device copies of the
    // orthogonalisation: uploads are queued without a wait (their staging
    // bytes stay untouched until the next synchronisation), downloads land
    // in pinned memory first.
    // (the ctx's staging buffer: solves on one ctx do not overlap)
    static constexpr size_t kPinBytes = (size_t)1 << 20;
    size_t pin_used = 0;
    void sync() {
        HIPCHECK(hipStreamSynchronize(s));
        pin_used = 0;
    }
    char *pin_take(size_t bytes) {
        if (c.pin.bytes < kPinBytes) {
            sync();
            c.pin.ensure(kPinBytes);
        }
        if (pin_used + bytes > kPinBytes) sync();
        char *q = c.pin.ptr + pin_used;
        pin_used += (bytes + 255) & ~(size_t)255;
        return q;
    }

    template <class T_>
    void d2h(T_ *h, const void *d, size_t count) {
        const size_t bytes = count * sizeof(T_);
        if (bytes > kPinBytes / 2) {
            HIPCHECK(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
            sync();
            return;
        }
        char *q = pin_take(bytes);
        HIPCHECK(hipMemcpyAsync(q, d, bytes, hipMemcpyDeviceToHost, s));
        sync();
        std::memcpy(h, q, bytes);
    }
    template <class T_>
    void h2d(void *d, const T_ *h, size_t count) {
        const size_t bytes = count * sizeof(T_);
        if (bytes > kPinBytes / 2) {
            HIPCHECK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
            sync();
            return;
        }
        char *q = pin_take(bytes);
        std::memcpy(q, h, bytes);
        HIPCHECK(hipMemcpyAsync(d, q, bytes, hipMemcpyHostToDevice, s));
    }

    // -------------------------------------------------------- capacities
    int ubar_w(int a) const {
        if (a == 0 || variant == BKS_VARIANT_MAX) return uw[a];
        return std::min(p, uw[a]);
    }
    int wbar_w(int b) const {
        if (b == 0 || variant == BKS_VARIANT_MAX) return ww[b];
        return std::min(p, ww[b]);
    }

    std::vector<std::array<int, 3>> stage_products(int stage) const {
        std::vector<std::array<int, 3>> out;  // {kind 0=U 1=W, a, b}
        if (stage == 1) return {{0, 0, 0}, {1, 0, 0}};
        const int nu = (int)uw.size(), nw = (int)ww.size();
        if (variant == BKS_VARIANT_MIN) {
            int q = stage - 1;
            if (q < nu && q < nw) out.push_back({0, q, q});
            if (q < nu) out.push_back({1, q, q});
            return out;
        }
        if (variant == BKS_VARIANT_BK) {
            int q = stage - 1;
            for (int a = 0; a < q; ++a) {
                if (a < nu && q < nw) out.push_back({0, a, q});
                if (q < nu && a < nw) out.push_back({0, q, a});
            }
            for (int a = 0; a < q; ++a)
                if (q < nu) out.push_back({1, a, q});
            return out;
        }
        for (int s_ = 1; s_ < std::max(nu, nw); ++s_) {
            for (int a = 0; a < s_; ++a) {
                if (a < nu && s_ < nw && !used_u.count({a, s_})) out.push_back({0, a, s_});
                if (s_ < nu && a < nw && !used_u.count({s_, a})) out.push_back({0, s_, a});
            }
            if (s_ < nu && s_ < nw && !used_u.count({s_, s_})) out.push_back({0, s_, s_});
        }
        for (int s_ = 0; s_ < nu; ++s_)
            for (int a = 0; a <= s_; ++a)
                if (!used_w.count({a, s_})) out.push_back({1, a, s_});
        return out;
    }

    // Simulate the schedule without deflation to size the device buffers.
    void plan() {
        uw = {r};
        ww = {r3};
        used_u.clear();
        used_w.clear();
        int qmax = std::max(r * r3, r * (r + 1) / 2);
        int64_t K1 = r, K3 = r3;
        for (int st = 1; st <= stages; ++st) {
            auto prods = stage_products(st);
            std::vector<int> nu, nw;
            for (auto &pr : prods) {
                if (pr[0] == 0) {
                    used_u.insert({pr[1], pr[2]});
                    int q = ubar_w(pr[1]) * wbar_w(pr[2]);
                    qmax = std::max(qmax, q);
                    nu.push_back(q);
                } else {
                    used_w.insert({pr[1], pr[2]});
                    int pa = ubar_w(pr[1]), pb = ubar_w(pr[2]);
                    int q = pr[1] == pr[2] ? pa * (pa + 1) / 2 : pa * pb;
                    qmax = std::max(qmax, q);
                    nw.push_back(q);
                }
            }
            for (int q : nu) {
                int w = (int)std::min<int64_t>(q, m - K1);
                uw.push_back(w);
                K1 += w;
            }
            for (int q : nw) {
                int w = (int)std::min<int64_t>(q, n - K3);
                ww.push_back(w);
                K3 += w;
            }
        }
        k1cap = (int)std::min<int64_t>(m, K1);
        k3cap = (int)std::min<int64_t>(n, K3);
        qcap = qmax;
        if (k1cap > 4096 || k3cap > 4096) fail(BKS_EINVAL, "basis would exceed 4096 columns");
    }

    void allocate() {
        X64.alloc((size_t)m * k1cap * 8);
        Z64.alloc((size_t)n * k3cap * 8);
        if (mixed) {
            X32.alloc((size_t)m * k1cap * 4);
            Z32.alloc((size_t)n * k3cap * 4);
        }
        const int64_t rows = std::max(m, n);
        P64.alloc((size_t)rows * qcap * 8);
        if (mixed) P32.alloc((size_t)rows * qcap * 4);
        W64a.alloc((size_t)rows * std::max(qcap, std::max(r, r3)) * 8);
        W64b.alloc((size_t)rows * std::max(qcap, std::max(r, r3)) * 8);
        T1.alloc((size_t)m * r * r3 * 8);
        T3h.alloc((size_t)n * (r * (r + 1) / 2) * 8);
        const size_t Q = (size_t)k1cap * (k1cap + 1) / 2;
        // FP64 wide even in mixed mode: its last iterations may form the
        // core in FP64
        T3core.alloc((size_t)n * Q * 8);
        Cdev.alloc((size_t)k3cap * Q * 8);
        const size_t small = (size_t)std::max(k1cap, k3cap) * std::max(qcap, 64) * 8 + 4096;
        Hd.alloc(small);
        Hd2.alloc(small);
        Gd.alloc((size_t)64 * 64 * 8 * 2 + 64 * 8);
    }

    double *Xcol(int col) { return X64.as<double>() + col; }
    double *Zcol(int col) { return Z64.as<double>() + col; }

    // Orthonormalise B (rows x q, ld) against the basis and append the kept
    // columns; B is left projected off the old basis.  Returns kept count.
    // hi and lo parts of a q x q double-double Gram at Gd, Gd + 64*64 (and,
    // with `norms`, nn column norms at Gd + 2*64*64): one copy
    void gram_dd_download(int q, std::vector<double> &hi, std::vector<double> &lo,
                          std::vector<double> *norms = nullptr, int nn = 0) {
        const size_t len = norms ? (size_t)2 * 64 * 64 + nn : (size_t)64 * 64 + (size_t)q * q;
        std::vector<double> all(len);
        d2h(all.data(), Gd.ptr, all.size());
        hi.assign(all.begin(), all.begin() + (size_t)q * q);
        lo.assign(all.begin() + 64 * 64, all.begin() + 64 * 64 + (size_t)q * q);
        if (norms) norms->assign(all.begin() + 2 * 64 * 64, all.begin() + 2 * 64 * 64 + nn);
    }

    int orth_append(bool isU, double *B, int64_t ldb, int q, double tau) {
        const int64_t rows = isU ? m : n;
        int &k = isU ? k1 : k3;
        const int cap = isU ? k1cap : k3cap;
        DevBuf &Bas = isU ? X64 : Z64;
        const int64_t ldbas = isU ? k1cap : k3cap;
        int total = 0;
        for (int c0 = 0; c0 < q; c0 += 64) {
            const int qc = std::min(64, q - c0);
            double *Bc = B + c0;
            const int room = cap - k;
            if (room <= 0) break;
            // squared column norms before the projection (downloaded with the Gram)
            std::vector<double> before2;
            colnorm2(Bc, ldb, rows, qc, Gd.as<double>() + 2 * 64 * 64, c, s);
            double *H = Hd.as<double>();
            for (int pass = 0; pass < 2 && k > 0; ++pass) {
                gemm_tn_f64(Bas.as<double>(), ldbas, Bc, ldb, rows, k, qc, H, qc, c, s);
                gemm_nn_f64(Bas.as<double>(), ldbas, H, qc, rows, k, qc, -1.0, 1.0, Bc, ldb, s);
            }
            std::vector<double> Ghi, Glo;
            gram_dd(Bc, ldb, rows, qc, Gd.as<double>(), Gd.as<double>() + 64 * 64, c, s);
            gram_dd_download(qc, Ghi, Glo, &before2, qc);
            std::vector<int> kept;
            std::vector<double> T;
            chol_drop(qc, Ghi, Glo, before2, tau, room, kept, T);
            const int qk = (int)kept.size();
            if (qk == 0) continue;
            // Q1 = B T into W64a (rows x qk)
            double *Q1 = W64a.as<double>();
            h2d(H, T.data(), T.size());
            gemm_nn_f64(Bc, ldb, H, qk, rows, qc, qk, 1.0, 0.0, Q1, qk, s);
            // second pass: off the old basis, then CholQR on the block
            if (k > 0) {
                gemm_tn_f64(Bas.as<double>(), ldbas, Q1, qk, rows, k, qk, H, qk, c, s);
                gemm_nn_f64(Bas.as<double>(), ldbas, H, qk, rows, k, qk, -1.0, 1.0, Q1, qk, s);
            }
            std::vector<double> G2h, G2l;
            gram_dd(Q1, qk, rows, qk, Gd.as<double>(), Gd.as<double>() + 64 * 64, c, s);
            gram_dd_download(qk, G2h, G2l);
            std::vector<double> ones(qk, 1.0);
            std::vector<int> kept2;
            std::vector<double> T2;
            chol_drop(qk, G2h, G2l, ones, 0.0, qk, kept2, T2);
            if ((int)kept2.size() != qk) fail(BKS_EDEVICE, "orthogonalisation lost rank");
            h2d(H, T2.data(), T2.size());
            gemm_nn_f64(Q1, qk, H, qk, rows, qk, qk, 1.0, 0.0, Bas.as<double>() + k, ldbas, s);
            if (mixed) {
                DevBuf &B32 = isU ? X32 : Z32;
                convert_f64_f32(Bas.as<double>() + k, ldbas, B32.as<float>() + k, ldbas, rows, qk, s);
            }
            k += qk;
            total += qk;
        }
        return total;
    }

    // Append a new block of `w` columns starting at `off`.
    void add_block(bool isU, int off, int w) {
        if (isU) {
            uoff.push_back(off);
            uw.push_back(w);
        } else {
            woff.push_back(off);
            ww.push_back(w);
        }
    }

    // A block's bars: first columns of block a (U) or b (W).
    // product (kind U: FREE1(Ubar_a, Wbar_b); kind W: FREE3(Ubar_a, Ubar_b))
    // into P64 (rows x q).  prec: BKS_F32 / BKS_F64 / BKS_F32IN_F64ACC.
    int product(int kind, int a, int b, int prec, double *dst, int64_t ldd) {
        if (kind == 0) {
            const int py = ubar_w(a), pz = wbar_w(b);
            if (py == 0 || pz == 0) return 0;
            const int q = py * pz;
            if (prec == BKS_F32) {
                ttmc(c, t, BKS_FREE1, X32.as<float>() + uoff[a], k1cap, py, Z32.as<float>() + woff[b],
                     k3cap, pz, false, BKS_F32, P32.ptr, q, s);
                convert_f32_f64(P32.as<float>(), q, dst, ldd, m, q, s);
            } else {
                ttmc(c, t, BKS_FREE1, Xcol(uoff[a]), k1cap, py, Zcol(woff[b]), k3cap, pz, false, prec,
                     dst, ldd, s);
            }
            return q;
        }
        const int pa = ubar_w(a), pb = ubar_w(b);
        if (pa == 0 || pb == 0) return 0;
        const bool sym = (a == b);
        const int q = sym ? pa * (pa + 1) / 2 : pa * pb;
        if (prec == BKS_F32) {
            ttmc(c, t, BKS_FREE3, X32.as<float>() + uoff[a], k1cap, pa,
                 sym ? nullptr : (const void *)(X32.as<float>() + uoff[b]), k1cap, pb, sym, BKS_F32,
                 P32.ptr, q, s);
            convert_f32_f64(P32.as<float>(), q, dst, ldd, n, q, s);
        } else {
            ttmc(c, t, BKS_FREE3, Xcol(uoff[a]), k1cap, pa,
                 sym ? nullptr : (const void *)Xcol(uoff[b]), k1cap, pb, sym, prec, dst, ldd, s);
        }
        return q;
    }

    // Load a host column-major start (rows x w) into the basis and orthonormalise.
    void load_start(bool isU, const double *h, int w) {
        const int64_t rows = isU ? m : n;
        const int64_t ld = isU ? k1cap : k3cap;
        std::vector<double> rm((size_t)rows * ld, 0.0);
        for (int64_t i = 0; i < rows; ++i)
            for (int j = 0; j < w; ++j) rm[(size_t)i * ld + j] = h[(size_t)j * rows + i];
        DevBuf &Bas = isU ? X64 : Z64;
        h2d(Bas.ptr, rm.data(), rm.size());
        reset_basis(isU, w);
    }

    // Orthonormalise columns [0, w) of the basis in place (CholQR twice) and
    // make them the only block.
    void reset_basis(bool isU, int w) {
        const int64_t rows = isU ? m : n;
        const int64_t ld = isU ? k1cap : k3cap;
        DevBuf &Bas = isU ? X64 : Z64;
        double *W = W64b.as<double>();
        for (int pass = 0; pass < 2; ++pass) {
            copy2d_f64(Bas.as<double>(), ld, W, w, rows, w, s);
            std::vector<double> Gh((size_t)w * w), Gl((size_t)w * w);
            gram_dd(W, w, rows, w, Gd.as<double>(), Gd.as<double>() + 64 * 64, c, s);
            gram_dd_download(w, Gh, Gl);
            std::vector<double> ones(w, 1.0), T;
            std::vector<int> kept;
            chol_drop(w, Gh, Gl, ones, 0.0, w, kept, T);
            if ((int)kept.size() != w) fail(BKS_EINVAL, "start matrix is rank deficient");
            h2d(Hd.ptr, T.data(), T.size());
            gemm_nn_f64(W, w, Hd.as<double>(), w, rows, w, w, 1.0, 0.0, Bas.as<double>(), ld, s);
        }
        if (mixed) {
            DevBuf &B32 = isU ? X32 : Z32;
            convert_f64_f32(Bas.as<double>(), ld, B32.as<float>(), ld, rows, w, s);
        }
        if (isU) {
            k1 = w;
            uoff = {0};
            uw = {w};
            used_u.clear();
        } else {
            k3 = w;
            woff = {0};
            ww = {w};
            used_w.clear();
        }
    }

    // ------------------------------------------------------ step (iii)/(iv)
    struct StepOut {
        double rel, normF;
        std::vector<double> F1;   // r x r*r3 (row-major)
        std::vector<double> s1, s3;
    };

    StepOut bk_step() {
        // FP64 accumulation over the tensor's own values (FP32 values are exact in FP64)
        const int prec = BKS_F64;
        const int q1 = r * r3, q3 = r * (r + 1) / 2;
        StepOut o;
        // T1 = A.(U0, W0)_{2,3};  T3 = A.(U0, U0)_{1,2} (sym-half)
        ttmc(c, t, BKS_FREE1, Xcol(0), k1cap, r, Zcol(0), k3cap, r3, false, prec, T1.ptr, q1, s);
        ttmc(c, t, BKS_FREE3, Xcol(0), k1cap, r, nullptr, 0, 0, true, prec, T3h.ptr, q3, s);
        // F_(1) = U0^T T1
        o.F1.assign((size_t)r * q1, 0.0);
        gemm_tn_f64(Xcol(0), k1cap, T1.as<double>(), q1, m, r, q1, Hd.as<double>(), q1, c, s);
        d2h(o.F1.data(), Hd.ptr, o.F1.size());
        // U1, W1 and the R factors
        // R1 = U1^T (I - U0 U0^T) T1 = U1^T T1 and R3 = W1^T T3 since U1 is
        // orthogonal to U0 and W1 to W0.
        double *B = P64.as<double>();
        copy2d_f64(T1.as<double>(), q1, B, q1, m, q1, s);
        const int kU = orth_append(true, B, q1, q1, tau64);
        add_block(true, r, kU);
        std::vector<double> R1((size_t)kU * q1, 0.0);
        if (kU > 0) {
            gemm_tn_f64(Xcol(r), k1cap, T1.as<double>(), q1, m, kU, q1, Hd.as<double>(), q1, c, s);
            d2h(R1.data(), Hd.ptr, R1.size());
        }
        copy2d_f64(T3h.as<double>(), q3, B, q3, n, q3, s);
        const int kW = orth_append(false, B, q3, q3, tau64);
        add_block(false, r3, kW);
        std::vector<double> R3h((size_t)kW * q3, 0.0);
        if (kW > 0) {
            gemm_tn_f64(Zcol(r3), k3cap, T3h.as<double>(), q3, n, kW, q3, Hd.as<double>(), q3, c, s);
            d2h(R3h.data(), Hd.ptr, R3h.size());
        }
        used_u.insert({0, 0});
        used_w.insert({0, 0});
        // F(a,b,c) = F1[a][b + r c];  F_(3)[c][a + r b]
        std::vector<double> F3((size_t)r3 * r * r);
        double f2 = 0.0;
        for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b)
                for (int cc = 0; cc < r3; ++cc) {
                    const double v = o.F1[(size_t)a * q1 + b + r * cc];
                    F3[(size_t)cc * r * r + a + r * b] = v;
                    f2 += v * v;
                }
        // <H0, H1^1>_{-1} = R1 F_(1)^T ; <H0, H1^3>_{-3} = R3full F_(3)^T
        double g1 = 0.0, g3 = 0.0;
        for (int i = 0; i < kU; ++i)
            for (int a = 0; a < r; ++a) {
                double sacc = 0.0;
                for (int x = 0; x < q1; ++x) sacc += R1[(size_t)i * q1 + x] * o.F1[(size_t)a * q1 + x];
                g1 += sacc * sacc;
            }
        std::vector<double> R3f((size_t)kW * r * r, 0.0);
        for (int i = 0; i < kW; ++i)
            for (int b = 0; b < r; ++b)
                for (int a = 0; a <= b; ++a) {
                    const double v = R3h[(size_t)i * q3 + sym_idx(a, b)];
                    R3f[(size_t)i * r * r + a + r * b] = v;
                    R3f[(size_t)i * r * r + b + r * a] = v;
                }
        for (int i = 0; i < kW; ++i)
            for (int cc = 0; cc < r3; ++cc) {
                double sacc = 0.0;
                for (int x = 0; x < r * r; ++x) sacc += R3f[(size_t)i * r * r + x] * F3[(size_t)cc * r * r + x];
                g3 += sacc * sacc;
            }
        o.normF = std::sqrt(f2);
        o.rel = o.normF > 0 ? std::sqrt(2.0 * g1 + g3) / o.normF : INFINITY;
        // S-values (section "Conditioning of the best approximation problem")
        auto svals = [](int rows_, int cols, const std::vector<double> &M, int nv) {
            // singular values of M (rows_ x cols) via eig of M M^T
            std::vector<double> G((size_t)rows_ * rows_, 0.0), w(rows_), V((size_t)rows_ * rows_);
            for (int i = 0; i < rows_; ++i)
                for (int j = 0; j < rows_; ++j) {
                    double sacc = 0.0;
                    for (int x = 0; x < cols; ++x) sacc += M[(size_t)i * cols + x] * M[(size_t)j * cols + x];
                    G[(size_t)i * rows_ + j] = sacc;
                }
            if (rows_ > 0) la::sym_eig(rows_, G.data(), w.data(), V.data());
            std::vector<double> out;
            for (int i = 0; i < std::min(nv, rows_); ++i) out.push_back(std::sqrt(std::max(w[i], 0.0)));
            return out;
        };
        o.s1 = svals(r, q1, o.F1, r);
        auto t1 = svals(kU, q1, R1, 1);
        o.s1.push_back(t1.empty() ? 0.0 : t1[0]);
        o.s3 = svals(r3, r * r, F3, r3);
        auto t3 = svals(kW, r * r, R3f, 1);
        o.s3.push_back(t3.empty() ? 0.0 : t3[0]);
        return o;
    }

    void expand(int from_stage) {
        for (int st = from_stage; st <= stages; ++st) {
            auto prods = stage_products(st);
            // bars are taken from blocks existing at the start of the stage
            struct P_ {
                int kind, a, b;
            };
            std::vector<P_> us, ws;
            for (auto &pr : prods) {
                if (pr[0] == 0) {
                    used_u.insert({pr[1], pr[2]});
                    us.push_back({0, pr[1], pr[2]});
                } else {
                    used_w.insert({pr[1], pr[2]});
                    ws.push_back({1, pr[1], pr[2]});
                }
            }
            const int prec = fp32 ? BKS_F32 : BKS_F64;
            const double tau = fp32 ? tau32 : tau64;
            double *B = P64.as<double>();
            for (auto &pr : us) {
                int q = 0;
                const int off = k1;
                if (k1 < k1cap) q = product(0, pr.a, pr.b, prec, B, qcap);
                const int got = q > 0 ? orth_append(true, B, qcap, q, tau) : 0;
                add_block(true, off, got);
            }
            for (auto &pr : ws) {
                int q = 0;
                const int off = k3;
                if (k3 < k3cap) q = product(1, pr.a, pr.b, prec, B, qcap);
                const int got = q > 0 ? orth_append(false, B, qcap, q, tau) : 0;
                add_block(false, off, got);
            }
        }
    }

    // C = A.(X, X, Z) as a k1 x k1 x k3 column-major host array.
    void form_core(std::vector<double> &C) {
        const int Q = k1 * (k1 + 1) / 2;
        if (fp32) {
            ttmc(c, t, BKS_FREE3, X32.ptr, k1cap, k1, nullptr, 0, 0, true, BKS_F32, T3core.ptr, Q, s);
            gemm_tn_f32f64(Zcol(0), k3cap, T3core.as<float>(), Q, n, k3, Q, Cdev.as<double>(), Q, c, s);
        } else {
            ttmc(c, t, BKS_FREE3, X64.ptr, k1cap, k1, nullptr, 0, 0, true, BKS_F64, T3core.ptr, Q, s);
            gemm_tn_f64(Zcol(0), k3cap, T3core.as<double>(), Q, n, k3, Q, Cdev.as<double>(), Q, c, s);
        }
        std::vector<double> Ch((size_t)k3 * Q);
        d2h(Ch.data(), Cdev.ptr, Ch.size());
        C.assign((size_t)k1 * k1 * k3, 0.0);
        for (int cc = 0; cc < k3; ++cc)
            for (int b = 0; b < k1; ++b)
                for (int a = 0; a <= b; ++a) {
                    const double v = Ch[(size_t)cc * Q + sym_idx(a, b)];
                    C[a + (size_t)k1 * (b + (size_t)k1 * cc)] = v;
                    C[b + (size_t)k1 * (a + (size_t)k1 * cc)] = v;
                }
        {
            // Gradient-defining slices from the step-(iii) products (FP64
            // accumulation in both modes): the gradient is evaluated from
            // these same products, so a stationary point of the full problem
            // is an exact fixed point of the iteration (in mixed mode they
            // also replace FP32-formed values)
            const int q1 = r * r3, q3 = r * (r + 1) / 2;
            std::vector<double> XT1((size_t)k1 * q1), ZT3((size_t)k3 * q3);
            gemm_tn_f64(Xcol(0), k1cap, T1.as<double>(), q1, m, k1, q1, Hd.as<double>(), q1, c, s);
            d2h(XT1.data(), Hd.ptr, XT1.size());
            gemm_tn_f64(Zcol(0), k3cap, T3h.as<double>(), q3, n, k3, q3, Hd.as<double>(), q3, c, s);
            d2h(ZT3.data(), Hd.ptr, ZT3.size());
            for (int a = 0; a < k1; ++a)
                for (int b = 0; b < r; ++b)
                    for (int cc = 0; cc < r3; ++cc) {
                        const double v = XT1[(size_t)a * q1 + b + r * cc];
                        C[a + (size_t)k1 * (b + (size_t)k1 * cc)] = v;
                        C[b + (size_t)k1 * (a + (size_t)k1 * cc)] = v;
                    }
            for (int cc = 0; cc < k3; ++cc)
                for (int b = 0; b < r; ++b)
                    for (int a = 0; a <= b; ++a) {
                        const double v = ZT3[(size_t)cc * q3 + sym_idx(a, b)];
                        C[a + (size_t)k1 * (b + (size_t)k1 * cc)] = v;
                        C[b + (size_t)k1 * (a + (size_t)k1 * cc)] = v;
                    }
        }
    }

    // U0 = X P, W0 = Z S (eq. tks1), orthonormalised, as the new single blocks.
    void restart(const std::vector<double> &P, const std::vector<double> &S) {
        double *W = W64a.as<double>();
        h2d(Hd.ptr, P.data(), P.size());
        gemm_nn_f64(Xcol(0), k1cap, Hd.as<double>(), r, m, k1, r, 1.0, 0.0, W, r, s);
        copy2d_f64(W, r, Xcol(0), k1cap, m, r, s);
        reset_basis(true, r);
        h2d(Hd.ptr, S.data(), S.size());
        gemm_nn_f64(Zcol(0), k3cap, Hd.as<double>(), r3, n, k3, r3, 1.0, 0.0, W, r3, s);
        copy2d_f64(W, r3, Zcol(0), k3cap, n, r3, s);
        reset_basis(false, r3);
    }

    void outputs(double *U, double *W, double *F, const std::vector<double> &F1) {
        std::vector<double> h((size_t)m * k1cap);
        if (U) {
            d2h(h.data(), X64.ptr, (size_t)m * k1cap);
            for (int64_t i = 0; i < m; ++i)
                for (int j = 0; j < r; ++j) U[(size_t)j * m + i] = h[(size_t)i * k1cap + j];
        }
        if (W) {
            std::vector<double> hz((size_t)n * k3cap);
            d2h(hz.data(), Z64.ptr, hz.size());
            for (int64_t i = 0; i < n; ++i)
                for (int j = 0; j < r3; ++j) W[(size_t)j * n + i] = hz[(size_t)i * k3cap + j];
        }
        if (F)
            for (int a = 0; a < r; ++a)
                for (int b = 0; b < r; ++b)
                    for (int cc = 0; cc < r3; ++cc)
                        F[a + (size_t)r * (b + (size_t)r * cc)] = F1[(size_t)a * r * r3 + b + r * cc];
    }
};

void draw_start(uint64_t seed, int64_t rows, int w, std::vector<double> &out) {
    std::mt19937_64 g(seed);
    std::normal_distribution<double> N(0.0, 1.0);
    out.resize((size_t)rows * w);
    for (auto &v : out) v = N(g);
}

void fill_info(bks_info *info, const Solver::StepOut &o, int iters, bool conv, int k1, int k3,
               double normA) {
    if (!info) return;
    info->fp64_from = -1;
    info->outer_iters = iters;
    info->converged = conv ? 1 : 0;
    info->k1 = k1;
    info->k3 = k3;
    info->rel_grad = o.rel;
    info->normF = o.normF;
    info->normA = normA;
    for (int i = 0; i < 65; ++i) {
        info->svals1[i] = i < (int)o.s1.size() ? o.s1[i] : 0.0;
        info->svals2[i] = info->svals1[i];  // U = V
        info->svals3[i] = i < (int)o.s3.size() ? o.s3[i] : 0.0;
    }
}

}  // namespace

// Device bytes a bks_solve of an m x m x n tensor allocates (the buffers of
// Solver::allocate plus the product workspaces), for admission control.
size_t solve_footprint(int64_t m, int64_t n, int64_t nnz, const bks_params &prm) {
    Ctx c;
    Tensor t;
    t.m = m;
    t.n = n;
    const bool mixed = prm.precision == BKS_PREC_MIXED;
    Solver S(c, t, nullptr, prm.r, prm.r3, prm.p > 0 ? prm.p : 4, prm.s > 0 ? prm.s : 2,
             prm.variant, mixed);
    S.plan();
    const size_t k1 = S.k1cap, k3 = S.k3cap, q = S.qcap, rows = (size_t)std::max(m, n);
    const size_t Q = k1 * (k1 + 1) / 2;
    size_t b = (size_t)m * k1 * 8 + (size_t)n * k3 * 8;
    if (mixed) b += (size_t)m * k1 * 4 + (size_t)n * k3 * 4 + rows * q * 4;
    b += rows * q * 8 + 2 * rows * std::max<size_t>(q, std::max(prm.r, prm.r3)) * 8;
    b += (size_t)m * prm.r * prm.r3 * 8 + (size_t)n * (prm.r * (prm.r + 1) / 2) * 8;
    b += (size_t)n * Q * 8 + k3 * Q * 8;
    b += 2 * std::max(k1, k3) * std::max<size_t>(q, 64) * 8 + 64 * 64 * 16;
    // product partials and the split reductions (grow-only workspaces, 25%
    // slack each): a core product wider than 24 columns keeps one k1 x k1
    // partial per slice chunk, counted as the product counts its chunks
    // (chunk width clamp(nnz / 4096, 256, 2048), widened so that at most
    // max(n + 1, 512 MB / partial) chunks exist, every slice at least one),
    // plus a block-packed copy of X
    const size_t cts = 8;  // FP64 partials also in mixed mode (its last iterations)
    if (k1 > 24) {
        const double per_item = (double)k1 * k1 * cts;
        const int64_t max_items = std::max<int64_t>(n + 1, (int64_t)(536870912.0 / per_item));
        int64_t cw = std::min<int64_t>(2048, std::max<int64_t>(256, nnz / 4096));
        cw = std::max<int64_t>(cw, nnz / std::max<int64_t>(1, max_items - n) + 1);
        const int64_t items = std::min<int64_t>(max_items, n + nnz / cw + 1);
        b += (size_t)items * k1 * k1 * cts / 4 * 5 + (size_t)m * (k1 + 16) * cts / 4 * 5;
    }
    b += (size_t)n * Q * 8 / 4 + rows * 64 * 8 + (size_t)(1 << 20) * 8;
    // inner solve on the device: the core and its rotated blocks (each at
    // most k1^2 k3 doubles) for large cores, and the Newton matrix with its
    // shifted copy for large Newton systems (grow-only, 25% slack)
    const size_t core = k1 * k1 * k3 * 8;
    if ((double)k1 * k1 * k3 >= device_core_min())
        b += 4 * core / 4 * 5 + (k1 * k1 + k3 * k3) * 8 / 4 * 5;
    const size_t N = (size_t)prm.r * (k1 - std::min<size_t>(k1, prm.r)) +
                     (size_t)prm.r3 * (k3 - std::min<size_t>(k3, prm.r3));
    if ((int64_t)N >= device_solve_min()) b += 2 * N * N * 8 / 4 * 5 + N * 16 + 16384;
    return b;
}

int run_bks(Ctx &c, Tensor &t, const bks_params &prm, double *U, double *W, double *F,
            bks_info *info, hipStream_t s) {
    const double t0 = now_s();
    const int r = prm.r, r3 = prm.r3;
    if (t.general) fail(BKS_EINVAL, "a general tensor: use bks_gsolve");
    if (r < 1 || r3 < 1 || r > t.m || r3 > t.n || r3 > r * (r + 1) / 2)
        fail(BKS_EINVAL, "need 1 <= r <= m, 1 <= r3 <= min(n, r(r+1)/2)");
    if (r > 64 || r3 > 64) fail(BKS_EINVAL, "r and r3 are limited to 64");
    const int st = prm.s > 0 ? prm.s : 2;
    const int p = prm.p > 0 ? prm.p : 4;
    if (prm.variant < 0 || prm.variant > 2) fail(BKS_EINVAL, "variant");
    if (prm.precision != BKS_PREC_FP64 && prm.precision != BKS_PREC_MIXED) fail(BKS_EINVAL, "precision");
    const bool mixed = prm.precision == BKS_PREC_MIXED;
    const double tol = prm.tol > 0 ? prm.tol : (mixed ? 1e-11 : 1e-13);
    const double itol = prm.inner_tol > 0 ? prm.inner_tol : 1e-13;
    const int max_outer = prm.max_outer > 0 ? prm.max_outer : 200;
    const int hooi_warm = prm.hooi_warm >= 0 ? prm.hooi_warm : 5;
    const int ng_max = prm.ng_max > 0 ? prm.ng_max : 50;

    Solver S(c, t, s, r, r3, p, st, prm.variant, mixed);
    S.plan();
    S.allocate();
    std::vector<double> h0;
    if (prm.U0) {
        S.load_start(true, prm.U0, r);
    } else {
        draw_start(prm.seed * 2 + 1, t.m, r, h0);
        S.load_start(true, h0.data(), r);
    }
    if (prm.W0) {
        S.load_start(false, prm.W0, r3);
    } else {
        draw_start(prm.seed * 2 + 2, t.n, r3, h0);
        S.load_start(false, h0.data(), r3);
    }
    double te = 0, tc = 0, ti = 0, ts = 0;
    double a = now_s();
    Solver::StepOut o = S.bk_step();  // stage 1 of the initial expansion
    ts += now_s() - a;
    a = now_s();
    S.expand(2);
    te += now_s() - a;
    int it = 0;
    bool conv = false;
    std::vector<double> C, P, Sm;
    std::vector<double> rel_hist, f_hist;
    int fp64_from = -1;
    long inner_newton = 0;
    int last_k1 = S.k1, last_k3 = S.k3;
    bool cancelled = false;
    while (true) {
        // a served request that was cancelled stops here, at the point of its
        // last restart (or its start), which is returned
        if (c.cancel && c.cancel->load()) {
            cancelled = true;
            break;
        }
        last_k1 = S.k1;
        last_k3 = S.k3;
        a = now_s();
        S.form_core(C);
        tc += now_s() - a;
        for (double v : C)
            if (!std::isfinite(v))
                fail(BKS_EDEVICE, "non-finite projected core at outer iteration " +
                                      std::to_string(it) + " (k1 " + std::to_string(S.k1) +
                                      ", k3 " + std::to_string(S.k3) + ")");
        a = now_s();
        InnerInfo ii;
        const bool warm = prm.inner_start == 1;
        if (warm) {
            // the restart point U0, W0 is the leading block of X, Z
            P.assign((size_t)S.k1 * r, 0.0);
            Sm.assign((size_t)S.k3 * r3, 0.0);
            for (int j = 0; j < r; ++j) P[(size_t)j * r + j] = 1.0;
            for (int j = 0; j < r3; ++j) Sm[(size_t)j * r3 + j] = 1.0;
        }
        if (c.host_acquire) c.host_acquire();
        try {
            const BigSolve big = [&](int N, const double *H, double mu, bool fresh, double *b) {
                return c.devsolve.solve(s, N, H, mu, fresh, b);
            };
            c.devinner.ds = &c.devsolve;
            c.devinner.s = s;
            InnerDevice *dev = &c.devinner;
            inner_solve(C, S.k1, S.k3, r, r3, itol, hooi_warm, ng_max, warm, P, Sm, ii, big, dev,
                        device_core_min());
            if (!warm) {
                // keep the outer objective non-decreasing (eq. Fnon-decr): if
                // the HOSVD-started solve ends below the current point E0,
                // solve again from E0 (accepted steps only increase g)
                std::vector<double> P0((size_t)S.k1 * r, 0.0), S0((size_t)S.k3 * r3, 0.0);
                for (int j = 0; j < r; ++j) P0[(size_t)j * r + j] = 1.0;
                for (int j = 0; j < r3; ++j) S0[(size_t)j * r3 + j] = 1.0;
                // (the device holds this C when the inner solve used it)
                InnerDevice *gdev =
                    (double)S.k1 * S.k1 * S.k3 >= device_core_min() ? dev : nullptr;
                const double g_new = inner_objective(C, S.k1, S.k3, P, Sm, r, r3, gdev);
                const double g_cur = inner_objective(C, S.k1, S.k3, P0, S0, r, r3, gdev);
                if (g_new < g_cur * (1.0 - 1e-14)) {
                    InnerInfo i2;
                    inner_solve(C, S.k1, S.k3, r, r3, itol, hooi_warm, ng_max, true, P0, S0, i2,
                                big, dev, device_core_min());
                    P.swap(P0);
                    Sm.swap(S0);
                    ii.newton += i2.newton;
                }
            }
        } catch (...) {
            if (c.host_release) c.host_release();
            throw;
        }
        if (c.host_release) c.host_release();
        inner_newton += ii.newton;
        ti += now_s() - a;
        if (debug_inner())
            std::fprintf(stderr,
                         "[bks] outer %d k1 %d k3 %d inner iters %d newton %d rel %.3e  "
                         "start %.2f rotate %.2f hess %.2f chol %.2f total %.2f ms\n",
                         it, S.k1, S.k3, ii.iters, ii.newton, ii.rel, 1e3 * ii.t_start,
                         1e3 * ii.t_rotate, 1e3 * ii.t_hess, 1e3 * ii.t_chol, 1e3 * (now_s() - a));
        a = now_s();
        S.restart(P, Sm);
        o = S.bk_step();
        ts += now_s() - a;
        ++it;
        rel_hist.push_back(o.rel);
        f_hist.push_back(o.normF);
        if (o.rel <= tol) {
            conv = true;
            break;
        }
        if (it >= max_outer) break;
        // mixed precision at its floor: below 1e-9 an outer iteration that
        // does not halve the best gradient so far switches the remaining
        // expansion and core products to FP64
        if (S.fp32 && o.rel < 1e-9 && rel_hist.size() >= 2) {
            const double best_before = *std::min_element(rel_hist.begin(), rel_hist.end() - 1);
            if (o.rel > 0.5 * best_before) {
                S.fp32 = false;
                fp64_from = it;
            }
        }
        // stagnation at the rounding floor above tol: once below 1e-10, 30
        // outer iterations without halving the best gradient end the solve
        // (not converged; the iterate is returned).  Slow linear convergence
        // halves it far more often.
        constexpr int kWin = 30;
        if (it > kWin) {
            const double best_recent =
                *std::min_element(rel_hist.end() - kWin, rel_hist.end());
            const double best_before =
                *std::min_element(rel_hist.begin(), rel_hist.end() - kWin);
            if (best_before < 1e-10 && best_recent > 0.5 * best_before) break;
        }
        a = now_s();
        S.expand(2);
        te += now_s() - a;
    }
    S.outputs(U, W, F, o.F1);
    fill_info(info, o, it, conv, last_k1, last_k3, std::sqrt(t.frob2));
    if (info) {
        info->fp64_from = fp64_from;
        info->t_expand = te;
        info->t_core = tc;
        info->t_inner = ti;
        info->t_step = ts;
        info->t_total = now_s() - t0;
        info->n_hist = (int)std::min<size_t>(512, rel_hist.size());
        for (int i = 0; i < info->n_hist; ++i) {
            info->rel_hist[i] = rel_hist[i];
            info->normF_hist[i] = f_hist[i];
        }
    }
    if (cancelled) return BKS_ECANCELED;
    return conv ? BKS_OK : BKS_ENOTCONV;
}

// Symmetric HOOI (section "Higher Order Orthogonal Iteration"): U from the r leading left singular vectors
// of T1 = A.(U, W)_{2,3}, then W from A.(U, U)_{1,2} with the new U (its
// sym-half unfolding with off-diagonal columns weighted by sqrt(2) has the
// Gram matrix of the full unfolding).  Singular vectors come from the small
// Gram matrix: U = T1 V_r diag(sigma)^{-1}, then re-orthonormalised in FP64.
// The G-gradient (global coordinates, section "Gradient on the product manifold") is evaluated every
// `grad_every` iterations with FP64-accurate products.  In mixed precision
// the iteration products are FP32 until the measured relative gradient is
// below 1e-4, then FP64-accurate.
int run_hooi(Ctx &c, Tensor &t, const hooi_params &prm, double *U, double *W, double *F,
             bks_info *info, hipStream_t s) {
    const double t0 = now_s();
    const int r = prm.r, r3 = prm.r3;
    if (t.general) fail(BKS_EINVAL, "a general tensor: use bks_gsolve");
    if (r < 1 || r3 < 1 || r > t.m || r3 > t.n || r3 > r * (r + 1) / 2)
        fail(BKS_EINVAL, "need 1 <= r <= m, 1 <= r3 <= min(n, r(r+1)/2)");
    if (r > 64 || r3 > 64) fail(BKS_EINVAL, "r and r3 are limited to 64");
    const bool mixed = prm.precision == BKS_PREC_MIXED;
    const double tol = prm.tol > 0 ? prm.tol : 1e-13;
    const int max_iter = prm.max_iter > 0 ? prm.max_iter : 2000;
    const int every = prm.grad_every > 0 ? prm.grad_every : 10;
    // the basis buffers of a Solver hold U (k1cap = r) and W (k3cap = r3)
    Solver S(c, t, s, r, r3, 1, 1, BKS_VARIANT_BK, mixed);
    S.k1cap = r;
    S.k3cap = r3;
    S.qcap = std::max(r * r3, r * (r + 1) / 2);
    S.X64.alloc((size_t)t.m * r * 8);
    S.Z64.alloc((size_t)t.n * r3 * 8);
    if (mixed) {
        S.X32.alloc((size_t)t.m * r * 4);
        S.Z32.alloc((size_t)t.n * r3 * 4);
        S.P32.alloc((size_t)std::max(t.m, t.n) * S.qcap * 4);
    }
    S.P64.alloc((size_t)std::max(t.m, t.n) * S.qcap * 8);
    S.W64a.alloc((size_t)std::max(t.m, t.n) * S.qcap * 8);
    S.W64b.alloc((size_t)std::max(t.m, t.n) * S.qcap * 8);
    S.T1.alloc((size_t)t.m * r * r3 * 8);
    S.T3h.alloc((size_t)t.n * (r * (r + 1) / 2) * 8);
    const int qa = r * r3, qb = r * (r + 1) / 2;
    // small scratch: Gram (q x q) / right factors, then a second region at
    // offset `hoff` for the projection coefficients of the gradient
    const size_t hoff = (size_t)std::max(qa, qb) * std::max(qa, qb) + (size_t)qa * r + 4096;
    S.Hd.alloc((hoff + 64 * 64) * 8);
    S.Gd.alloc((size_t)64 * 64 * 8 * 2 + 64 * 8);
    std::vector<double> h0;
    if (prm.U0) S.load_start(true, prm.U0, r);
    else {
        draw_start(prm.seed * 2 + 1, t.m, r, h0);
        S.load_start(true, h0.data(), r);
    }
    if (prm.W0) S.load_start(false, prm.W0, r3);
    else {
        draw_start(prm.seed * 2 + 2, t.n, r3, h0);
        S.load_start(false, h0.data(), r3);
    }
    const int q1 = r * r3, q3 = r * (r + 1) / 2;
    // top `w` left singular vectors of M (rows x q, FP64 device, ld q) into
    // the basis columns [0, w) via the Gram matrix, weights applied to columns
    auto left_sv = [&](bool isU, double *M, int64_t rows, int q, int w,
                       const std::vector<double> &colw) {
        std::vector<double> G((size_t)q * q);
        gemm_tn_f64(M, q, M, q, rows, q, q, S.Hd.as<double>(), q, c, s);
        S.d2h(G.data(), S.Hd.ptr, G.size());
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) G[(size_t)i * q + j] *= colw[i] * colw[j];
        std::vector<double> V((size_t)q * w), ev(w);
        la::top_eigvecs(q, G.data(), w, V.data(), ev.data());
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < w; ++j) {
                const double sg = std::sqrt(std::max(ev[j], 1e-300));
                V[(size_t)i * w + j] *= colw[i] / sg;
            }
        S.h2d(S.Hd.ptr, V.data(), V.size());
        DevBuf &Bas = isU ? S.X64 : S.Z64;
        gemm_nn_f64(M, q, S.Hd.as<double>(), w, rows, q, w, 1.0, 0.0, Bas.as<double>(), w, s);
        S.reset_basis(isU, w);
    };
    std::vector<double> w1(q1, 1.0), w3(q3, 1.0);
    for (int b = 0; b < r; ++b)
        for (int a = 0; a < b; ++a) w3[sym_idx(a, b)] = std::sqrt(2.0);
    // global gradient at the current (U, W); also returns F_(1)
    auto gradient = [&](std::vector<double> &F1, double &normF) {
        // FP64 accumulation over the tensor's own values (FP32 values are exact in FP64)
        const int prec = BKS_F64;
        ttmc(c, t, BKS_FREE1, S.X64.ptr, r, r, S.Z64.ptr, r3, r3, false, prec, S.T1.ptr, q1, s);
        ttmc(c, t, BKS_FREE3, S.X64.ptr, r, r, nullptr, 0, 0, true, prec, S.T3h.ptr, q3, s);
        F1.assign((size_t)r * q1, 0.0);
        gemm_tn_f64(S.X64.as<double>(), r, S.T1.as<double>(), q1, t.m, r, q1, S.Hd.as<double>(), q1, c, s);
        S.d2h(F1.data(), S.Hd.ptr, F1.size());
        // Gamma1 = T1 F_(1)^T (m x r); Gamma3 = T3full F_(3)^T via the sym-half columns
        std::vector<double> F1t((size_t)q1 * r), M3((size_t)q3 * r3, 0.0);
        double f2 = 0.0;
        for (int a = 0; a < r; ++a)
            for (int x = 0; x < q1; ++x) {
                F1t[(size_t)x * r + a] = F1[(size_t)a * q1 + x];
                f2 += F1[(size_t)a * q1 + x] * F1[(size_t)a * q1 + x];
            }
        for (int b = 0; b < r; ++b)
            for (int a = 0; a <= b; ++a)
                for (int cc = 0; cc < r3; ++cc) {
                    double v = F1[(size_t)a * q1 + b + r * cc];
                    if (a != b) v += F1[(size_t)b * q1 + a + r * cc];
                    M3[(size_t)sym_idx(a, b) * r3 + cc] = v;
                }
        normF = std::sqrt(f2);
        double g2[2];
        for (int mode = 0; mode < 2; ++mode) {
            const bool isU = mode == 0;
            const int64_t rows = isU ? t.m : t.n;
            const int w = isU ? r : r3;
            const int q = isU ? q1 : q3;
            double *Gm = S.W64a.as<double>();
            S.h2d(S.Hd.ptr, isU ? F1t.data() : M3.data(), (size_t)q * w);
            gemm_nn_f64(isU ? S.T1.as<double>() : S.T3h.as<double>(), q, S.Hd.as<double>(), w, rows,
                        q, w, 1.0, 0.0, Gm, w, s);
            DevBuf &Bas = isU ? S.X64 : S.Z64;
            double *H = S.Hd.as<double>() + hoff;
            gemm_tn_f64(Bas.as<double>(), w, Gm, w, rows, w, w, H, w, c, s);
            gemm_nn_f64(Bas.as<double>(), w, H, w, rows, w, w, -1.0, 1.0, Gm, w, s);
            std::vector<double> n2(w);
            colnorm2(Gm, w, rows, w, S.Gd.as<double>(), c, s);
            S.d2h(n2.data(), S.Gd.ptr, w);
            g2[mode] = 0.0;
            for (double v : n2) g2[mode] += v;
        }
        return normF > 0 ? std::sqrt(2.0 * g2[0] + g2[1]) / normF : INFINITY;
    };
    std::vector<double> F1;
    double normF = 0.0;
    double rel = gradient(F1, normF);
    int it = 0;
    std::vector<double> rel_hist;
    bool conv = rel <= tol;
    int fp64_from = -1;
    while (!conv && it < max_iter) {
        const bool fp32 = mixed && rel > 1e-4;
        if (mixed && !fp32 && fp64_from < 0) fp64_from = it;
        const int prec = fp32 ? BKS_F32 : BKS_F64;
        double *T = S.P64.as<double>();
        if (fp32) {
            ttmc(c, t, BKS_FREE1, S.X32.ptr, r, r, S.Z32.ptr, r3, r3, false, BKS_F32, S.P32.ptr, q1, s);
            convert_f32_f64(S.P32.as<float>(), q1, T, q1, t.m, q1, s);
        } else {
            ttmc(c, t, BKS_FREE1, S.X64.ptr, r, r, S.Z64.ptr, r3, r3, false, prec, T, q1, s);
        }
        left_sv(true, T, t.m, q1, r, w1);
        if (fp32) {
            ttmc(c, t, BKS_FREE3, S.X32.ptr, r, r, nullptr, 0, 0, true, BKS_F32, S.P32.ptr, q3, s);
            convert_f32_f64(S.P32.as<float>(), q3, T, q3, t.n, q3, s);
        } else {
            ttmc(c, t, BKS_FREE3, S.X64.ptr, r, r, nullptr, 0, 0, true, prec, T, q3, s);
        }
        left_sv(false, T, t.n, q3, r3, w3);
        ++it;
        if (it % every == 0 || it >= max_iter) {
            rel = gradient(F1, normF);
            rel_hist.push_back(rel);
            conv = rel <= tol;
        }
    }
    S.outputs(U, W, nullptr, F1);
    if (F)
        for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b)
                for (int cc = 0; cc < r3; ++cc)
                    F[a + (size_t)r * (b + (size_t)r * cc)] = F1[(size_t)a * q1 + b + r * cc];
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->fp64_from = fp64_from;
        info->outer_iters = it;
        info->converged = conv ? 1 : 0;
        info->rel_grad = rel;
        info->normF = normF;
        info->normA = std::sqrt(t.frob2);
        info->t_total = now_s() - t0;
        info->n_hist = (int)std::min<size_t>(512, rel_hist.size());
        for (int i = 0; i < info->n_hist; ++i) info->rel_hist[i] = rel_hist[i];
    }
    return conv ? BKS_OK : BKS_ENOTCONV;
}

// ---------------------------------------------------------------- general tensors
// Algorithm 5 for a general (non-symmetric) tensor A in R^{l x m x n}
// (section "A Tensor Krylov-Schur like method"): three bases X, Y, Z grown
// by the mode-1, -2, -3 block-Krylov steps of Algorithm 3 (section
// "Block-Krylov methods"), the core C = A.(X, Y, Z), its best rank-(r1, r2,
// r3) approximation, the restart and one block-Krylov step per mode with the
// three-term G-gradient of Proposition 3.2.  Schedule (the paper gives the BK
// diagrams for the (1,2)-symmetric case only): min-BK in every mode -- stage
// t: U_t from (Vbar_{t-1}, Wbar_{t-1}), V_t from (Ubar_{t-1}, Wbar_{t-1}),
// W_t from (Ubar_{t-1}, Vbar_{t-1}); U0, V0, W0 whole, later blocks their
// first p columns.  Inner solve: truncated HOSVD, then HOOI until the
// projected problem's relative gradient reaches the tolerance (the paper's
// alternative to Newton-Grassmann, with the same fixed points).
namespace {

// dense core helpers (host, small sizes): C is k0 x k1 x k2, column-major
struct GCore {
    int k[3];
    std::vector<double> C;
    double at(int a, int b, int c) const { return C[a + (size_t)k[0] * (b + (size_t)k[1] * c)]; }
};

// M = mode-`md` unfolding of C.(P0, P1, P2) with the factor of mode md the
// identity: rows k[md], columns (first remaining fastest) r_b * r_c
static std::vector<double> partial_unfold(const GCore &G, int md, const std::vector<double> *P[3],
                                          const int r[3]) {
    const int k0 = G.k[0], k1 = G.k[1], k2 = G.k[2];
    // contract the two other modes one at a time
    int d[3] = {k0, k1, k2};
    std::vector<double> cur = G.C;
    for (int mode = 0; mode < 3; ++mode) {
        if (mode == md) continue;
        const std::vector<double> &Pm = *P[mode];  // k[mode] x r[mode], row-major
        int nd[3] = {d[0], d[1], d[2]};
        nd[mode] = r[mode];
        std::vector<double> nxt((size_t)nd[0] * nd[1] * nd[2], 0.0);
        for (int c = 0; c < d[2]; ++c)
            for (int b = 0; b < d[1]; ++b)
                for (int a = 0; a < d[0]; ++a) {
                    const double v = cur[a + (size_t)d[0] * (b + (size_t)d[1] * c)];
                    if (v == 0.0) continue;
                    const int idx[3] = {a, b, c};
                    for (int x = 0; x < r[mode]; ++x) {
                        int o[3] = {a, b, c};
                        o[mode] = x;
                        nxt[o[0] + (size_t)nd[0] * (o[1] + (size_t)nd[1] * o[2])] +=
                            v * Pm[(size_t)idx[mode] * r[mode] + x];
                    }
                }
        cur.swap(nxt);
        d[0] = nd[0];
        d[1] = nd[1];
        d[2] = nd[2];
    }
    // unfold in mode md: rows d[md], columns the other two (first fastest)
    const int o1 = md == 0 ? 1 : 0, o2 = md == 2 ? 1 : 2;
    std::vector<double> M((size_t)d[md] * d[o1] * d[o2]);
    for (int c = 0; c < d[2]; ++c)
        for (int b = 0; b < d[1]; ++b)
            for (int a = 0; a < d[0]; ++a) {
                const int idx[3] = {a, b, c};
                M[(size_t)idx[md] * d[o1] * d[o2] + idx[o1] + (size_t)d[o1] * idx[o2]] =
                    cur[a + (size_t)d[0] * (b + (size_t)d[1] * c)];
            }
    return M;
}

// leading r left singular vectors of M (rows x cols, row-major), rows x r row-major
static std::vector<double> top_left(const std::vector<double> &M, int rows, int cols, int r) {
    std::vector<double> G((size_t)rows * rows);
    la::dgemm(false, true, rows, rows, cols, 1.0, M.data(), cols, M.data(), cols, 0.0, G.data(), rows);
    std::vector<double> V((size_t)rows * r);
    la::top_eigvecs(rows, G.data(), r, V.data());
    return V;
}

// relative G-gradient of ||C.(P0, P1, P2)||^2 and ||F||^2
static double g_gradient(const GCore &G, const std::vector<double> *P[3], const int r[3],
                         double *f2out) {
    double g2 = 0.0, f2 = 0.0;
    for (int md = 0; md < 3; ++md) {
        const int rows = G.k[md];
        const int o1 = md == 0 ? 1 : 0, o2 = md == 2 ? 1 : 2;
        const int cols = r[o1] * r[o2];
        const std::vector<double> M = partial_unfold(G, md, P, r);      // rows x cols
        const std::vector<double> &B = *P[md];                            // rows x r[md]
        // F_(md) = B^T M (r x cols); G = (M - B F) F^T
        std::vector<double> F((size_t)r[md] * cols), R = M, Gm((size_t)rows * r[md]);
        la::dgemm(true, false, r[md], cols, rows, 1.0, B.data(), r[md], M.data(), cols, 0.0, F.data(), cols);
        la::dgemm(false, false, rows, cols, r[md], -1.0, B.data(), r[md], F.data(), cols, 1.0, R.data(), cols);
        la::dgemm(false, true, rows, r[md], cols, 1.0, R.data(), cols, F.data(), cols, 0.0, Gm.data(), r[md]);
        for (double v : Gm) g2 += v * v;
        if (md == 0)
            for (double v : F) f2 += v * v;
    }
    if (f2out) *f2out = f2;
    return f2 > 0 ? std::sqrt(g2 / f2) : INFINITY;
}

static void g_inner(const GCore &G, const int r[3], double tol, int max_iter, bool from_e0,
                    std::vector<double> out[3]) {
    std::vector<double> P[3];
    const std::vector<double> *pp[3] = {&P[0], &P[1], &P[2]};
    for (int md = 0; md < 3; ++md) {
        if (from_e0) {
            P[md].assign((size_t)G.k[md] * r[md], 0.0);
            for (int j = 0; j < r[md]; ++j) P[md][(size_t)j * r[md] + j] = 1.0;
        } else {
            // truncated HOSVD: leading left singular vectors of the unfoldings
            std::vector<double> I3[3];
            int rr[3] = {G.k[0], G.k[1], G.k[2]};
            for (int x = 0; x < 3; ++x) {
                I3[x].assign((size_t)G.k[x] * G.k[x], 0.0);
                for (int j = 0; j < G.k[x]; ++j) I3[x][(size_t)j * G.k[x] + j] = 1.0;
            }
            const std::vector<double> *ip[3] = {&I3[0], &I3[1], &I3[2]};
            const int o1 = md == 0 ? 1 : 0, o2 = md == 2 ? 1 : 2;
            const std::vector<double> M = partial_unfold(G, md, ip, rr);
            P[md] = top_left(M, G.k[md], G.k[o1] * G.k[o2], r[md]);
        }
    }
    double rel = g_gradient(G, pp, r, nullptr);
    for (int it = 1; rel > tol && it <= max_iter; ++it) {
        for (int md = 0; md < 3; ++md) {
            const int o1 = md == 0 ? 1 : 0, o2 = md == 2 ? 1 : 2;
            const std::vector<double> M = partial_unfold(G, md, pp, r);
            P[md] = top_left(M, G.k[md], r[o1] * r[o2], r[md]);
        }
        if (it % 5 == 0 || it == max_iter) rel = g_gradient(G, pp, r, nullptr);
    }
    for (int md = 0; md < 3; ++md) out[md] = P[md];
}

struct GSolver {
    Ctx &c;
    Tensor &t;
    hipStream_t s;
    int64_t dim[3];
    int r[3], p, stages;
    bool mixed;
    double tau64 = 1e-14, tau32 = 1e-5;
    int kcap[3] = {0, 0, 0}, k[3] = {0, 0, 0}, qcap = 0;
    DevBuf B64[3], B32[3], P32, P64, W64a, T64[3], Hd, Gd, Tb32, Tb64, Cb;
    std::vector<int> off[3], w[3];

    GSolver(Ctx &c_, Tensor &t_, hipStream_t s_, const int r_[3], int p_, int st, bool mx)
        : c(c_), t(t_), s(s_), p(p_), stages(st), mixed(mx) {
        dim[0] = t.l;
        dim[1] = t.m;
        dim[2] = t.n;
        for (int x = 0; x < 3; ++x) r[x] = r_[x];
    }

    void sync() { HIPCHECK(hipStreamSynchronize(s)); }
    template <class T_> void d2h(T_ *h, const void *d, size_t count) {
        HIPCHECK(hipMemcpyAsync(h, d, count * sizeof(T_), hipMemcpyDeviceToHost, s));
        sync();
    }
    template <class T_> void h2d(void *d, const T_ *h, size_t count) {
        HIPCHECK(hipMemcpyAsync(d, h, count * sizeof(T_), hipMemcpyHostToDevice, s));
        sync();
    }
    double *col(int md, int j) { return B64[md].as<double>() + j; }
    static int other1(int md) { return md == 0 ? 1 : 0; }
    static int other2(int md) { return md == 2 ? 1 : 2; }
    int bar(int md, int blk) const { return blk == 0 ? w[md][0] : std::min(p, w[md][blk]); }

    void plan() {
        int64_t K[3];
        int wd[3][16];
        for (int x = 0; x < 3; ++x) {
            K[x] = r[x];
            wd[x][0] = r[x];
        }
        qcap = std::max({r[1] * r[2], r[0] * r[2], r[0] * r[1]});
        for (int st = 1; st <= stages && st < 16; ++st) {
            int q[3];
            for (int md = 0; md < 3; ++md) {
                auto b = [&](int x) { return st - 1 == 0 ? wd[x][0] : std::min(p, wd[x][st - 1]); };
                q[md] = b(other1(md)) * b(other2(md));
                qcap = std::max(qcap, q[md]);
            }
            for (int md = 0; md < 3; ++md) {
                const int ww = (int)std::min<int64_t>(q[md], dim[md] - K[md]);
                wd[md][st] = ww;
                K[md] += ww;
            }
        }
        for (int x = 0; x < 3; ++x) {
            kcap[x] = (int)std::min<int64_t>(dim[x], K[x]);
            if (kcap[x] > 4096) fail(BKS_EINVAL, "basis would exceed 4096 columns");
        }
    }

    void allocate() {
        const int64_t rows = std::max({dim[0], dim[1], dim[2]});
        for (int x = 0; x < 3; ++x) {
            B64[x].alloc((size_t)dim[x] * kcap[x] * 8);
            if (mixed) B32[x].alloc((size_t)dim[x] * kcap[x] * 4);
            const int q = r[other1(x)] * r[other2(x)];
            T64[x].alloc((size_t)dim[x] * q * 8);
        }
        P64.alloc((size_t)rows * qcap * 8);
        if (mixed) P32.alloc((size_t)rows * qcap * 4);
        W64a.alloc((size_t)rows * std::max(qcap, std::max({r[0], r[1], r[2]})) * 8);
        const int kmax = std::max({kcap[0], kcap[1], kcap[2]});
        Hd.alloc((size_t)kmax * std::max(qcap, 64) * 8 + 4096);
        Gd.alloc((size_t)64 * 64 * 8 * 2 + 64 * 8);
        // core blocks: (n x 20*20) products and their k2 x 400 projections
        Tb64.alloc((size_t)dim[2] * 400 * 8);
        if (mixed) Tb32.alloc((size_t)dim[2] * 400 * 4);
        Cb.alloc((size_t)kcap[2] * 400 * 8);
    }

    int orth_append(int md, double *B, int64_t ldb, int q, double tau) {
        const int64_t rows = dim[md];
        int &kk = k[md];
        const int cap = kcap[md];
        const int64_t ldbas = kcap[md];
        int total = 0;
        for (int c0 = 0; c0 < q; c0 += 64) {
            const int qc = std::min(64, q - c0);
            double *Bc = B + c0;
            const int room = cap - kk;
            if (room <= 0) break;
            colnorm2(Bc, ldb, rows, qc, Gd.as<double>() + 2 * 64 * 64, c, s);
            double *H = Hd.as<double>();
            for (int pass = 0; pass < 2 && kk > 0; ++pass) {
                gemm_tn_f64(B64[md].as<double>(), ldbas, Bc, ldb, rows, kk, qc, H, qc, c, s);
                gemm_nn_f64(B64[md].as<double>(), ldbas, H, qc, rows, kk, qc, -1.0, 1.0, Bc, ldb, s);
            }
            gram_dd(Bc, ldb, rows, qc, Gd.as<double>(), Gd.as<double>() + 64 * 64, c, s);
            std::vector<double> all((size_t)2 * 64 * 64 + qc);
            d2h(all.data(), Gd.ptr, all.size());
            std::vector<double> Ghi(all.begin(), all.begin() + (size_t)qc * qc),
                Glo(all.begin() + 64 * 64, all.begin() + 64 * 64 + (size_t)qc * qc),
                before2(all.begin() + 2 * 64 * 64, all.begin() + 2 * 64 * 64 + qc);
            std::vector<int> kept;
            std::vector<double> T;
            chol_drop(qc, Ghi, Glo, before2, tau, room, kept, T);
            const int qk = (int)kept.size();
            if (qk == 0) continue;
            double *Q1 = W64a.as<double>();
            h2d(H, T.data(), T.size());
            gemm_nn_f64(Bc, ldb, H, qk, rows, qc, qk, 1.0, 0.0, Q1, qk, s);
            if (kk > 0) {
                gemm_tn_f64(B64[md].as<double>(), ldbas, Q1, qk, rows, kk, qk, H, qk, c, s);
                gemm_nn_f64(B64[md].as<double>(), ldbas, H, qk, rows, kk, qk, -1.0, 1.0, Q1, qk, s);
            }
            gram_dd(Q1, qk, rows, qk, Gd.as<double>(), Gd.as<double>() + 64 * 64, c, s);
            std::vector<double> all2((size_t)64 * 64 + (size_t)qk * qk);
            d2h(all2.data(), Gd.ptr, all2.size());
            std::vector<double> G2h(all2.begin(), all2.begin() + (size_t)qk * qk),
                G2l(all2.begin() + 64 * 64, all2.begin() + 64 * 64 + (size_t)qk * qk);
            std::vector<double> ones(qk, 1.0), T2;
            std::vector<int> kept2;
            chol_drop(qk, G2h, G2l, ones, 0.0, qk, kept2, T2);
            if ((int)kept2.size() != qk) fail(BKS_EDEVICE, "orthogonalisation lost rank");
            h2d(H, T2.data(), T2.size());
            gemm_nn_f64(Q1, qk, H, qk, rows, qk, qk, 1.0, 0.0, B64[md].as<double>() + kk, ldbas, s);
            if (mixed)
                convert_f64_f32(B64[md].as<double>() + kk, ldbas, B32[md].as<float>() + kk, ldbas,
                                rows, qk, s);
            kk += qk;
            total += qk;
        }
        return total;
    }

    // orthonormalise columns [0, ww) of basis md (CholQR twice) as its only block
    void reset_basis(int md, int ww) {
        const int64_t rows = dim[md], ld = kcap[md];
        double *W = W64a.as<double>();
        for (int pass = 0; pass < 2; ++pass) {
            copy2d_f64(B64[md].as<double>(), ld, W, ww, rows, ww, s);
            gram_dd(W, ww, rows, ww, Gd.as<double>(), Gd.as<double>() + 64 * 64, c, s);
            std::vector<double> all((size_t)64 * 64 + (size_t)ww * ww);
            d2h(all.data(), Gd.ptr, all.size());
            std::vector<double> Gh(all.begin(), all.begin() + (size_t)ww * ww),
                Gl(all.begin() + 64 * 64, all.begin() + 64 * 64 + (size_t)ww * ww), ones(ww, 1.0), T;
            std::vector<int> kept;
            chol_drop(ww, Gh, Gl, ones, 0.0, ww, kept, T);
            if ((int)kept.size() != ww) fail(BKS_EINVAL, "start matrix is rank deficient");
            h2d(Hd.ptr, T.data(), T.size());
            gemm_nn_f64(W, ww, Hd.as<double>(), ww, rows, ww, ww, 1.0, 0.0, B64[md].as<double>(), ld, s);
        }
        if (mixed) convert_f64_f32(B64[md].as<double>(), ld, B32[md].as<float>(), ld, rows, ww, s);
        k[md] = ww;
        off[md] = {0};
        w[md] = {ww};
    }

    void load_start(int md, const double *h) {
        const int64_t rows = dim[md], ld = kcap[md];
        std::vector<double> rm((size_t)rows * ld, 0.0);
        for (int64_t i = 0; i < rows; ++i)
            for (int j = 0; j < r[md]; ++j) rm[(size_t)i * ld + j] = h[(size_t)j * rows + i];
        h2d(B64[md].ptr, rm.data(), rm.size());
        reset_basis(md, r[md]);
    }

    // product for a new block of mode md from blocks (b1 of the first other
    // mode, b2 of the second), into dst (dim[md] x q, FP64)
    int product(int md, int b1, int b2, int prec, double *dst, int64_t ldd) {
        const int m1 = other1(md), m2 = other2(md);
        const int p1 = bar(m1, b1), p2 = bar(m2, b2);
        if (p1 == 0 || p2 == 0) return 0;
        const int q = p1 * p2;
        if (prec == BKS_F32) {
            gttmc(c, t, md, B32[m1].as<float>() + off[m1][b1], kcap[m1], p1,
                  B32[m2].as<float>() + off[m2][b2], kcap[m2], p2, BKS_F32, P32.ptr, q, s);
            convert_f32_f64(P32.as<float>(), q, dst, ldd, dim[md], q, s);
        } else {
            gttmc(c, t, md, col(m1, off[m1][b1]), kcap[m1], p1, col(m2, off[m2][b2]), kcap[m2], p2,
                  prec, dst, ldd, s);
        }
        return q;
    }

    void expand(int from_stage) {
        const int prec = mixed ? BKS_F32 : BKS_F64;
        const double tau = mixed ? tau32 : tau64;
        for (int st = from_stage; st <= stages; ++st) {
            const int src = st - 1;
            // bars from the blocks existing at the start of the stage
            int have[3];
            for (int md = 0; md < 3; ++md) have[md] = (int)w[md].size();
            for (int md = 0; md < 3; ++md) {
                int got = 0, o = k[md];
                if (src < have[other1(md)] && src < have[other2(md)] && k[md] < kcap[md]) {
                    double *B = P64.as<double>();
                    const int q = product(md, src, src, prec, B, qcap);
                    got = q > 0 ? orth_append(md, B, qcap, q, tau) : 0;
                }
                off[md].push_back(o);
                w[md].push_back(got);
            }
        }
    }

    // C = A.(X, Y, Z), column-major k0 x k1 x k2, formed in 20 x 20 blocks
    // of the first two modes (T = A.(X_a, Y_b)_{1,2}, then Z^T T); the
    // slices that define the gradient at (U0, V0, W0) are then replaced by
    // the FP64-accumulated step-(iii) products (see form_core above)
    void form_core(GCore &G) {
        const int k0 = k[0], k1 = k[1], k2 = k[2];
        G.k[0] = k0;
        G.k[1] = k1;
        G.k[2] = k2;
        G.C.assign((size_t)k0 * k1 * k2, 0.0);
        constexpr int BW = 20;
        std::vector<double> h((size_t)k2 * BW * BW);
        for (int a0 = 0; a0 < k0; a0 += BW)
            for (int b0 = 0; b0 < k1; b0 += BW) {
                const int pa = std::min(BW, k0 - a0), pb = std::min(BW, k1 - b0), q = pa * pb;
                if (mixed) {
                    gttmc(c, t, 2, B32[0].as<float>() + a0, kcap[0], pa, B32[1].as<float>() + b0,
                          kcap[1], pb, BKS_F32, Tb32.ptr, q, s);
                    gemm_tn_f32f64(col(2, 0), kcap[2], Tb32.as<float>(), q, dim[2], k2, q,
                                   Cb.as<double>(), q, c, s);
                } else {
                    gttmc(c, t, 2, col(0, a0), kcap[0], pa, col(1, b0), kcap[1], pb, BKS_F64,
                          Tb64.ptr, q, s);
                    gemm_tn_f64(col(2, 0), kcap[2], Tb64.as<double>(), q, dim[2], k2, q,
                                Cb.as<double>(), q, c, s);
                }
                d2h(h.data(), Cb.ptr, (size_t)k2 * q);
                for (int cc = 0; cc < k2; ++cc)
                    for (int b = 0; b < pb; ++b)
                        for (int a = 0; a < pa; ++a)
                            G.C[(a0 + a) + (size_t)k0 * ((b0 + b) + (size_t)k1 * cc)] =
                                h[(size_t)cc * q + a + pa * b];
            }
        // gradient-defining slices from the step-(iii) products: mode md's
        // product T_md (dim[md] x r_o1 r_o2) projected on basis md gives C
        // with the other two indices in their leading r
        for (int md = 0; md < 3; ++md) {
            const int o1 = other1(md), o2 = other2(md);
            const int q = r[o1] * r[o2];
            std::vector<double> P((size_t)k[md] * q);
            gemm_tn_f64(col(md, 0), kcap[md], T64[md].as<double>(), q, dim[md], k[md], q,
                        Hd.as<double>(), q, c, s);
            d2h(P.data(), Hd.ptr, P.size());
            for (int x = 0; x < k[md]; ++x)
                for (int b = 0; b < r[o2]; ++b)
                    for (int a = 0; a < r[o1]; ++a) {
                        int idx[3];
                        idx[md] = x;
                        idx[o1] = a;
                        idx[o2] = b;
                        G.C[idx[0] + (size_t)k0 * (idx[1] + (size_t)k1 * idx[2])] =
                            P[(size_t)x * q + a + r[o1] * b];
                    }
        }
    }

    // U0 = X P, V0 = Y Q, W0 = Z S (eq. tks1), orthonormalised, single blocks
    void restart(const std::vector<double> Pm[3]) {
        for (int md = 0; md < 3; ++md) {
            double *W = W64a.as<double>();
            h2d(Hd.ptr, Pm[md].data(), Pm[md].size());
            gemm_nn_f64(col(md, 0), kcap[md], Hd.as<double>(), r[md], dim[md], k[md], r[md], 1.0,
                        0.0, W, r[md], s);
            copy2d_f64(W, r[md], col(md, 0), kcap[md], dim[md], r[md], s);
            reset_basis(md, r[md]);
        }
    }

    struct StepOut {
        double rel = INFINITY, normF = 0.0;
        std::vector<double> F;  // r0 x r1 x r2 column-major
        std::vector<double> sv[3];
    };

    // step (iii)/(iv): one block-Krylov step per mode from (U0, V0, W0)
    // (FP64 accumulation), the new blocks U1, V1, W1, and Proposition 3.2
    StepOut bk_step() {
        StepOut o;
        const int prec = BKS_F64;
        for (int md = 0; md < 3; ++md) {
            const int o1 = other1(md), o2 = other2(md), q = r[o1] * r[o2];
            gttmc(c, t, md, col(o1, 0), kcap[o1], r[o1], col(o2, 0), kcap[o2], r[o2], prec,
                  T64[md].ptr, q, s);
        }
        // F_(1) = U0^T T_0 : r0 x r1 r2 (column b + r1 c), i.e. F(a, b, c)
        const int q0 = r[1] * r[2];
        std::vector<double> F1((size_t)r[0] * q0);
        gemm_tn_f64(col(0, 0), kcap[0], T64[0].as<double>(), q0, dim[0], r[0], q0, Hd.as<double>(),
                    q0, c, s);
        d2h(F1.data(), Hd.ptr, F1.size());
        o.F.assign((size_t)r[0] * q0, 0.0);
        double f2 = 0.0;
        for (int a = 0; a < r[0]; ++a)
            for (int x = 0; x < q0; ++x) {
                o.F[a + (size_t)r[0] * x] = F1[(size_t)a * q0 + x];
                f2 += F1[(size_t)a * q0 + x] * F1[(size_t)a * q0 + x];
            }
        o.normF = std::sqrt(f2);
        auto Fat = [&](int a, int b, int cc) { return o.F[a + (size_t)r[0] * (b + (size_t)r[1] * cc)]; };
        double g2 = 0.0;
        for (int md = 0; md < 3; ++md) {
            const int o1 = other1(md), o2 = other2(md), q = r[o1] * r[o2];
            double *B = P64.as<double>();
            copy2d_f64(T64[md].as<double>(), q, B, q, dim[md], q, s);
            const int kn = orth_append(md, B, q, q, tau64);
            off[md].push_back(r[md]);
            w[md].push_back(kn);
            // H1 = B1^T T_md (kn x q): B1 is orthogonal to U0, so this is
            // B1^T (I - U0 U0^T) T_md
            std::vector<double> H1((size_t)kn * q);
            if (kn > 0) {
                gemm_tn_f64(col(md, r[md]), kcap[md], T64[md].as<double>(), q, dim[md], kn, q,
                            Hd.as<double>(), q, c, s);
                d2h(H1.data(), Hd.ptr, H1.size());
            }
            // F_(md): r[md] x q with columns a + r[o1] b
            std::vector<double> Fm((size_t)r[md] * q);
            for (int x = 0; x < r[md]; ++x)
                for (int b = 0; b < r[o2]; ++b)
                    for (int a = 0; a < r[o1]; ++a) {
                        int idx[3];
                        idx[md] = x;
                        idx[o1] = a;
                        idx[o2] = b;
                        Fm[(size_t)x * q + a + r[o1] * b] = Fat(idx[0], idx[1], idx[2]);
                    }
            // <H0, H1^md>_{-md} = H1 F_(md)^T
            for (int i = 0; i < kn; ++i)
                for (int x = 0; x < r[md]; ++x) {
                    double acc = 0.0;
                    for (int y = 0; y < q; ++y) acc += H1[(size_t)i * q + y] * Fm[(size_t)x * q + y];
                    g2 += acc * acc;
                }
            // S-values: singular values of F_(md), then sigma_max(H1)
            auto svals = [](int rows, int cols, const std::vector<double> &M, int nv) {
                std::vector<double> G((size_t)rows * rows, 0.0), wv(rows), V((size_t)rows * rows);
                if (rows > 0) {
                    la::dgemm(false, true, rows, rows, cols, 1.0, M.data(), cols, M.data(), cols,
                              0.0, G.data(), rows);
                    la::sym_eig(rows, G.data(), wv.data(), V.data());
                }
                std::vector<double> out;
                for (int i = 0; i < std::min(nv, rows); ++i) out.push_back(std::sqrt(std::max(wv[i], 0.0)));
                return out;
            };
            o.sv[md] = svals(r[md], q, Fm, r[md]);
            auto t1 = svals(kn, q, H1, 1);
            o.sv[md].push_back(t1.empty() ? 0.0 : t1[0]);
        }
        o.rel = o.normF > 0 ? std::sqrt(g2) / o.normF : INFINITY;
        return o;
    }

    void outputs(double *U, double *V, double *W) {
        double *outs[3] = {U, V, W};
        for (int md = 0; md < 3; ++md) {
            if (!outs[md]) continue;
            std::vector<double> h((size_t)dim[md] * kcap[md]);
            d2h(h.data(), B64[md].ptr, h.size());
            for (int64_t i = 0; i < dim[md]; ++i)
                for (int j = 0; j < r[md]; ++j)
                    outs[md][(size_t)j * dim[md] + i] = h[(size_t)i * kcap[md] + j];
        }
    }
};

}  // namespace

int run_gbks(Ctx &c, Tensor &t, const bks_gparams &prm, double *U, double *V, double *W,
             double *F, bks_info *info, hipStream_t s) {
    const double t0 = now_s();
    if (!t.general) fail(BKS_EINVAL, "not a general tensor (use bks_solve)");
    const int r[3] = {prm.r1, prm.r2, prm.r3};
    const int64_t dim[3] = {t.l, t.m, t.n};
    for (int x = 0; x < 3; ++x) {
        if (r[x] < 1 || r[x] > dim[x] || r[x] > 64) fail(BKS_EINVAL, "need 1 <= r_k <= min(dim_k, 64)");
        const int o1 = x == 0 ? 1 : 0, o2 = x == 2 ? 1 : 2;
        if (r[x] > r[o1] * r[o2]) fail(BKS_EINVAL, "need r_k <= product of the other two ranks");
    }
    if (prm.precision != BKS_PREC_FP64 && prm.precision != BKS_PREC_MIXED) fail(BKS_EINVAL, "precision");
    const bool mixed = prm.precision == BKS_PREC_MIXED;
    const int st = prm.s > 0 ? prm.s : 2, p = prm.p > 0 ? prm.p : 4;
    const double tol = prm.tol > 0 ? prm.tol : (mixed ? 1e-11 : 1e-13);
    const double itol = prm.inner_tol > 0 ? prm.inner_tol : 1e-13;
    const int max_outer = prm.max_outer > 0 ? prm.max_outer : 200;
    GSolver S(c, t, s, r, p, st, mixed);
    S.plan();
    S.allocate();
    const double *starts[3] = {prm.U0, prm.V0, prm.W0};
    std::vector<double> h;
    for (int md = 0; md < 3; ++md) {
        if (starts[md]) {
            S.load_start(md, starts[md]);
        } else {
            draw_start(prm.seed * 3 + 1 + md, dim[md], r[md], h);
            S.load_start(md, h.data());
        }
    }
    double te = 0, tc = 0, ti = 0, ts = 0, a = now_s();
    GSolver::StepOut o = S.bk_step();
    ts += now_s() - a;
    a = now_s();
    S.expand(2);
    te += now_s() - a;
    int it = 0;
    bool conv = false;
    std::vector<double> rel_hist, f_hist;
    int last_k[3] = {S.k[0], S.k[1], S.k[2]};
    while (true) {
        for (int x = 0; x < 3; ++x) last_k[x] = S.k[x];
        a = now_s();
        GCore G;
        S.form_core(G);
        tc += now_s() - a;
        a = now_s();
        std::vector<double> Pm[3];
        g_inner(G, r, itol, 5000, false, Pm);
        // keep the outer objective non-decreasing (eq. Fnon-decr)
        {
            std::vector<double> E[3];
            for (int x = 0; x < 3; ++x) {
                E[x].assign((size_t)G.k[x] * r[x], 0.0);
                for (int j = 0; j < r[x]; ++j) E[x][(size_t)j * r[x] + j] = 1.0;
            }
            const std::vector<double> *pp[3] = {&Pm[0], &Pm[1], &Pm[2]};
            const std::vector<double> *pe[3] = {&E[0], &E[1], &E[2]};
            double g_new = 0, g_cur = 0;
            g_gradient(G, pp, r, &g_new);
            g_gradient(G, pe, r, &g_cur);
            if (g_new < g_cur * (1.0 - 1e-14)) g_inner(G, r, itol, 5000, true, Pm);
        }
        ti += now_s() - a;
        a = now_s();
        S.restart(Pm);
        o = S.bk_step();
        ts += now_s() - a;
        ++it;
        rel_hist.push_back(o.rel);
        f_hist.push_back(o.normF);
        if (o.rel <= tol) {
            conv = true;
            break;
        }
        if (it >= max_outer) break;
        a = now_s();
        S.expand(2);
        te += now_s() - a;
    }
    S.outputs(U, V, W);
    if (F) std::copy(o.F.begin(), o.F.end(), F);
    if (info) {
        info->fp64_from = -1;
        info->outer_iters = it;
        info->converged = conv ? 1 : 0;
        info->k1 = last_k[0];
        info->k3 = last_k[2];
        info->rel_grad = o.rel;
        info->normF = o.normF;
        info->normA = std::sqrt(t.frob2);
        for (int i = 0; i < 65; ++i) {
            info->svals1[i] = i < (int)o.sv[0].size() ? o.sv[0][i] : 0.0;
            info->svals2[i] = i < (int)o.sv[1].size() ? o.sv[1][i] : 0.0;
            info->svals3[i] = i < (int)o.sv[2].size() ? o.sv[2][i] : 0.0;
        }
        info->t_expand = te;
        info->t_core = tc;
        info->t_inner = ti;
        info->t_step = ts;
        info->t_total = now_s() - t0;
        info->n_hist = (int)std::min<size_t>(512, rel_hist.size());
        for (int i = 0; i < info->n_hist; ++i) {
            info->rel_hist[i] = rel_hist[i];
            info->normF_hist[i] = f_hist[i];
        }
    }
    return conv ? BKS_OK : BKS_ENOTCONV;
}

}  // namespace bks

using namespace bks;

namespace {
template <class F>
int guard_solve(bks_ctx ctx, F f) {
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    try {
        return f();
    } catch (const Error &e) {
        c->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        c->last_error = "host allocation failed";
        return BKS_ENOMEM;
    } catch (const std::exception &e) {
        c->last_error = e.what();
        return BKS_EDEVICE;
    }
}
}  // namespace

extern "C" {

int bks_solve(bks_ctx ctx, bks_tensor t, const bks_params *prm, double *U, double *W, double *F,
              bks_info *info) {
    if (!ctx || !t || !prm) return BKS_EINVAL;
    return guard_solve(ctx, [&] {
        Ctx *c = reinterpret_cast<Ctx *>(ctx);
        std::lock_guard<std::mutex> g(c->mu);
        HIPCHECK(hipSetDevice(c->device));
        if (info) std::memset(info, 0, sizeof(*info));
        return run_bks(*c, *reinterpret_cast<Tensor *>(t), *prm, U, W, F, info, c->stream);
    });
}

int bks_gsolve(bks_ctx ctx, bks_tensor t, const bks_gparams *prm, double *U, double *V, double *W,
               double *F, bks_info *info) {
    if (!ctx || !t || !prm) return BKS_EINVAL;
    return guard_solve(ctx, [&] {
        Ctx *c = reinterpret_cast<Ctx *>(ctx);
        std::lock_guard<std::mutex> g(c->mu);
        HIPCHECK(hipSetDevice(c->device));
        if (info) std::memset(info, 0, sizeof(*info));
        return run_gbks(*c, *reinterpret_cast<Tensor *>(t), *prm, U, V, W, F, info, c->stream);
    });
}

int hooi_solve(bks_ctx ctx, bks_tensor t, const hooi_params *prm, double *U, double *W, double *F,
               bks_info *info) {
    if (!ctx || !t || !prm) return BKS_EINVAL;
    return guard_solve(ctx, [&] {
        Ctx *c = reinterpret_cast<Ctx *>(ctx);
        std::lock_guard<std::mutex> g(c->mu);
        HIPCHECK(hipSetDevice(c->device));
        return run_hooi(*c, *reinterpret_cast<Tensor *>(t), *prm, U, W, F, info, c->stream);
    });
}

}  // extern "C"
