// Inner solve of Algorithm 5 step (i) on the host in FP64.
//
// g(P, S) = ||C.(P, P, S)||^2 on Gr(k1, r) x Gr(k3, r3).  Start: truncated
// HOSVD of C and `hooi_warm` symmetric HOOI iterations (section "Experiments"), then
// Newton-Grassmann.  The paper cites Newton-Grassmann without giving it; the
// step used here comes from the second-order expansion of g in the local
// coordinates of Appendix A.  With [P P_perp], [S S_perp] orthogonal and
// B = C.([P P_perp], [P P_perp], [S S_perp]) split into blocks (0 = first r or
// r3 coordinates, 1 = the rest), F = B000 and, along P(D) = [I; D] M,
// S(T) = [I; T] N with M, N the normalisations,
//   g = ||F||^2 + 4<Gamma1, D> + 2<Gamma3, T> + d^T A d + O(|d|^3)
//   Gamma1 = <B100, F>_{-1},  Gamma3 = <B001, F>_{-3}
//   d^T A d = ||G1||^2 + 2<F, G2> - 2 tr(D S1 D^T) - tr(T S3 T^T)
// where G1, G2 are the first and second order parts of B.([I;D],[I;D],[I;T])
// and S1 = <F, F>_{-1}, S3 = <F, F>_{-3}.  The blocks of A are formed in
// closed form from B100, B001, B110, B101 and F; the Newton step solves
// (-2A) d = (4 Gamma1, 2 Gamma3) by Cholesky and retracts with a thin QR.
// If -2A is not positive definite a HOOI iteration is taken instead.
#include "inner.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>

#include "linalg.h"

namespace bks {

namespace {

struct View {
    const double *C;
    int k1, k3;
    InnerDevice *dev = nullptr;  // large cores: dense products on the device
    bool hooi_dev = true;        // the HOOI and objective products too
    double at(int a, int b, int c) const { return C[a + (size_t)k1 * (b + (size_t)k1 * c)]; }
};

// CS(a, b, l) = sum_c C(a, b, c) Sv(c, l) for the columns [l0, l0+nl) of Sv
// (k3 x ldS row-major).  Output layout: a + k1*(b + k1*l).  The slices of C
// (a, b) are exactly symmetric, so so is every CS(:, :, l), and row a of a
// slice is contiguous at a * k1.
void mode3_product(const View &V, const double *Sv, int ldS, int l0, int nl,
                   std::vector<double> &out) {
    const int k1 = V.k1, k3 = V.k3;
    const int sl = k1 * k1;
    out.resize((size_t)sl * nl);
    la::dgemm(true, false, nl, sl, k3, 1.0, Sv + l0, ldS, V.C, sl, 0.0, out.data(), sl, true);
}

void hosvd(const View &V, int r, int r3, std::vector<double> &P, std::vector<double> &S) {
    const int k1 = V.k1, k3 = V.k3;
    const size_t sl = (size_t)k1 * k1;
    // G1 = C_(1) C_(1)^T: the mode-1 fibres C(:, b, c) are the rows of a
    // (k1 k3) x k1 matrix; G3 = C_(3) C_(3)^T: slice c is row c of k3 x k1^2
    std::vector<double> G1((size_t)k1 * k1), G3((size_t)k3 * k3);
    if (V.dev) {
        V.dev->gram1(G1.data());
        V.dev->gram3(G3.data());
        // exact symmetry (the device sums G(i, j) and G(j, i) separately)
        for (int a = 0; a < k1; ++a)
            for (int b = 0; b < a; ++b)
                G1[(size_t)a * k1 + b] = G1[(size_t)b * k1 + a] =
                    0.5 * (G1[(size_t)a * k1 + b] + G1[(size_t)b * k1 + a]);
        for (int a = 0; a < k3; ++a)
            for (int b = 0; b < a; ++b)
                G3[(size_t)a * k3 + b] = G3[(size_t)b * k3 + a] =
                    0.5 * (G3[(size_t)a * k3 + b] + G3[(size_t)b * k3 + a]);
    } else {
        la::dgemm(true, false, k1, k1, k1 * k3, 1.0, V.C, k1, V.C, k1, 0.0, G1.data(), k1, true);
        la::dgemm(false, true, k3, k3, (int)sl, 1.0, V.C, (int)sl, V.C, (int)sl, 0.0, G3.data(),
                  k3, true);
    }
    P.assign((size_t)k1 * r, 0.0);
    S.assign((size_t)k3 * r3, 0.0);
    la::top_eigvecs(k1, G1.data(), r, P.data());
    la::top_eigvecs(k3, G3.data(), r3, S.data());
}

// Leading w left singular vectors of M (rows x cols, row-major) through the
// small Gram matrix: U = M V diag(sigma)^-1, re-orthonormalised.
void lead_left(const std::vector<double> &M, int rows, int cols, int w, std::vector<double> &U) {
    std::vector<double> G((size_t)cols * cols);
    la::dgemm(true, false, cols, cols, rows, 1.0, M.data(), cols, M.data(), cols, 0.0, G.data(),
              cols, true);
    std::vector<double> Vv((size_t)cols * w), ev(w);
    la::top_eigvecs(cols, G.data(), w, Vv.data(), ev.data());
    for (int j = 0; j < w; ++j) {
        const double sc = 1.0 / std::sqrt(std::max(ev[j], 1e-300));
        for (int a = 0; a < cols; ++a) Vv[(size_t)a * w + j] *= sc;
    }
    U.resize((size_t)rows * w);
    la::dgemm(false, false, rows, w, cols, 1.0, M.data(), cols, Vv.data(), w, 0.0, U.data(), w);
    la::orthonormalize(rows, w, U.data());
}

// One symmetric HOOI iteration on the core (section "Higher Order Orthogonal Iteration").
void hooi_step(const View &V, int r, int r3, std::vector<double> &P, std::vector<double> &S) {
    const int k1 = V.k1, k3 = V.k3;
    const size_t sl = (size_t)k1 * k1;
    // M1(a, j + r*l) = sum_b CS(a, b, l) P(b, j), CS = C x_3 S (k1 x k1 x r3)
    const int w1 = r * r3;
    std::vector<double> M1((size_t)k1 * w1);
    if (V.dev && V.hooi_dev) {
        std::vector<double> out((size_t)k1 * w1);
        V.dev->mode3p(S.data(), r3, 0, r3, P.data(), r, out.data());
        for (int a = 0; a < k1; ++a)
            for (int x = 0; x < w1; ++x) M1[(size_t)a * w1 + x] = out[a + (size_t)k1 * x];
    } else {
        std::vector<double> CS;
        mode3_product(V, S.data(), r3, 0, r3, CS);
        la::parallel_for(r3, [&](int l) {
            la::dgemm(false, false, k1, r, k1, 1.0, &CS[sl * l], k1, P.data(), r, 0.0,
                      &M1[(size_t)r * l], w1);
        });
    }
    lead_left(M1, k1, w1, r, P);
    // M3(c, i + r*j) = sum_{a,b} C(a,b,c) P(a,i) P(b,j)
    const int w3 = r * r;
    std::vector<double> M3((size_t)k3 * w3);
    if (V.dev && V.hooi_dev) {
        V.dev->hooi3(P.data(), r, M3.data());
        lead_left(M3, k3, w3, r3, S);
        return;
    }
    la::parallel_for(k3, [&](int c) {
        std::vector<double> CP((size_t)k1 * r), T((size_t)r * r);
        la::dgemm(false, false, k1, r, k1, 1.0, V.C + sl * c, k1, P.data(), r, 0.0, CP.data(), r);
        la::dgemm(true, false, r, r, k1, 1.0, P.data(), r, CP.data(), r, 0.0, T.data(), r);
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < r; ++j) M3[(size_t)c * w3 + i + r * j] = T[(size_t)i * r + j];
    });
    lead_left(M3, k3, w3, r3, S);
}

struct Blocks {
    int r, r3, A1, C1;
    std::vector<double> Qp, Qs;   // k1 x k1, k3 x k3 (row-major), first columns span P, S
    std::vector<double> F;        // r x r x r3     F(a,b,c)   at a + r*(b + r*c)
    std::vector<double> B100;     // A1 x r x r3    (x,b,c)    at x + A1*(b + r*c)
    std::vector<double> B110;     // A1 x A1 x r3   (x,y,c)    at x + A1*(y + A1*c)
    std::vector<double> B001;     // r x r x C1     (a,b,z)    at a + r*(b + r*z)
    std::vector<double> B101;     // A1 x r x C1    (x,b,z)    at x + A1*(b + r*z)
    bool partial = false;         // B110, B101 left on the device (not filled)
};

// `partial` (device path only): the device keeps B110 and B101, which only
// the Newton matrix reads, and forms that matrix itself.
void rotate(const View &V, const std::vector<double> &P, const std::vector<double> &S, int r,
            int r3, Blocks &B, bool partial = false) {
    const int k1 = V.k1, k3 = V.k3;
    B.r = r;
    B.r3 = r3;
    B.A1 = k1 - r;
    B.C1 = k3 - r3;
    B.Qp.resize((size_t)k1 * k1);
    B.Qs.resize((size_t)k3 * k3);
    la::qr_full(k1, r, P.data(), B.Qp.data());
    la::qr_full(k3, r3, S.data(), B.Qs.data());
    const int A1 = B.A1, C1 = B.C1;
    B.F.assign((size_t)r * r * r3, 0.0);
    B.B100.assign((size_t)A1 * r * r3, 0.0);
    B.B001.assign((size_t)r * r * C1, 0.0);
    B.partial = partial && V.dev;
    if (B.partial) {
        B.B110.clear();
        B.B101.clear();
        std::vector<double> Y((size_t)k1 * r * r3), Y2((size_t)r * r * C1);
        V.dev->rotate(B.Qp.data(), B.Qs.data(), r, r3, Y.data(), Y2.data(), true);
        for (int l = 0; l < r3; ++l)
            for (int y = 0; y < r; ++y)
                for (int x = 0; x < k1; ++x) {
                    const double v = Y[x + (size_t)k1 * (y + (size_t)r * l)];
                    if (x < r) B.F[x + r * (y + (size_t)r * l)] = v;
                    else B.B100[(x - r) + (size_t)A1 * (y + (size_t)r * l)] = v;
                }
        std::copy(Y2.begin(), Y2.end(), B.B001.begin());
        return;
    }
    B.B110.assign((size_t)A1 * A1 * r3, 0.0);
    B.B101.assign((size_t)A1 * r * C1, 0.0);
    if (V.dev) {
        std::vector<double> Y((size_t)k1 * k1 * r3), Y2((size_t)k1 * r * C1);
        V.dev->rotate(B.Qp.data(), B.Qs.data(), r, r3, Y.data(), Y2.data(), false);
        for (int l = 0; l < r3; ++l)
            for (int y = 0; y < k1; ++y)
                for (int x = 0; x < k1; ++x) {
                    const double v = Y[x + (size_t)k1 * (y + (size_t)k1 * l)];
                    if (x < r && y < r) B.F[x + r * (y + (size_t)r * l)] = v;
                    else if (x >= r && y < r) B.B100[(x - r) + (size_t)A1 * (y + (size_t)r * l)] = v;
                    else if (x >= r && y >= r)
                        B.B110[(x - r) + (size_t)A1 * ((y - r) + (size_t)A1 * l)] = v;
                }
        for (int z = 0; z < C1; ++z)
            for (int j = 0; j < r; ++j)
                for (int x = 0; x < k1; ++x) {
                    const double v = Y2[x + (size_t)k1 * (j + (size_t)r * z)];
                    if (x < r) B.B001[x + r * (j + (size_t)r * z)] = v;
                    else B.B101[(x - r) + (size_t)A1 * (j + (size_t)r * z)] = v;
                }
        return;
    }
    // CS(:, :, l) = C.(I, I, Qs(:, l)) for all k3 columns: the first r3 give
    // R0 = C.(Qp, Qp, S), the rest R1 = C.(Qp, P, S_perp)
    std::vector<double> CS;
    mode3_product(V, B.Qs.data(), k3, 0, k3, CS);
    const size_t sl = (size_t)k1 * k1;
    la::parallel_for(k3, [&](int l) {
        const double *Xl = &CS[sl * l];  // symmetric: row a contiguous
        if (l < r3) {
            // Y = Qp^T X_l Qp, split into F, B100, B110
            std::vector<double> tmp(sl), Y(sl);
            la::dgemm(false, false, k1, k1, k1, 1.0, Xl, k1, B.Qp.data(), k1, 0.0, tmp.data(), k1);
            la::dgemm(true, false, k1, k1, k1, 1.0, B.Qp.data(), k1, tmp.data(), k1, 0.0, Y.data(),
                      k1);
            for (int x = 0; x < k1; ++x)
                for (int y = 0; y < k1; ++y) {
                    const double v = Y[(size_t)x * k1 + y];
                    if (x < r && y < r) B.F[x + r * (y + (size_t)r * l)] = v;
                    else if (x >= r && y < r) B.B100[(x - r) + (size_t)A1 * (y + (size_t)r * l)] = v;
                    else if (x >= r && y >= r)
                        B.B110[(x - r) + (size_t)A1 * ((y - r) + (size_t)A1 * l)] = v;
                }
        } else {
            // Y2 = Qp^T X_z P (P = the first r columns of Qp), split into B001, B101
            const int z = l - r3;
            std::vector<double> t2((size_t)k1 * r), Y2((size_t)k1 * r);
            la::dgemm(false, false, k1, r, k1, 1.0, Xl, k1, B.Qp.data(), k1, 0.0, t2.data(), r);
            la::dgemm(true, false, k1, r, k1, 1.0, B.Qp.data(), k1, t2.data(), r, 0.0, Y2.data(), r);
            for (int x = 0; x < k1; ++x)
                for (int j = 0; j < r; ++j) {
                    const double v = Y2[(size_t)x * r + j];
                    if (x < r) B.B001[x + r * (j + (size_t)r * z)] = v;
                    else B.B101[(x - r) + (size_t)A1 * (j + (size_t)r * z)] = v;
                }
        }
    });
}

double local_gradient(const Blocks &B, std::vector<double> &G1, std::vector<double> &G3,
                      double &normF) {
    const int r = B.r, r3 = B.r3, A1 = B.A1, C1 = B.C1;
    G1.assign((size_t)A1 * r, 0.0);
    G3.assign((size_t)C1 * r3, 0.0);
    for (int x = 0; x < A1; ++x)
        for (int a = 0; a < r; ++a) {
            double s = 0.0;
            for (int c = 0; c < r3; ++c)
                for (int b = 0; b < r; ++b)
                    s += B.B100[x + (size_t)A1 * (b + (size_t)r * c)] * B.F[a + r * (b + (size_t)r * c)];
            G1[(size_t)x * r + a] = s;
        }
    for (int z = 0; z < C1; ++z)
        for (int c = 0; c < r3; ++c) {
            double s = 0.0;
            for (int b = 0; b < r; ++b)
                for (int a = 0; a < r; ++a)
                    s += B.B001[a + r * (b + (size_t)r * z)] * B.F[a + r * (b + (size_t)r * c)];
            G3[(size_t)z * r3 + c] = s;
        }
    double f2 = 0.0, g1 = 0.0, g3 = 0.0;
    for (double v : B.F) f2 += v * v;
    for (double v : G1) g1 += v * v;
    for (double v : G3) g3 += v * v;
    normF = std::sqrt(f2);
    return normF > 0 ? std::sqrt(2.0 * g1 + g3) / normF : INFINITY;
}

// Negative Hessian H = -2A (N x N row-major) of the second-order model.
// The sums over one core index are products of rearranged blocks:
//   Delta-Delta  A[(x,a),(y,b)] = 2 [a=b] <M_x, M_y> + 2 sum_c M(x,b,c) M(y,a,c)
//                                + 2 sum_c F(a,b,c) B110(x,y,c) - 2 [x=y] S1(a,b)
//   Delta-Theta  A[(x,a),(z,c)] = 2 sum_b (M(x,b,c) B001(a,b,z) + F(a,b,c) B101(x,b,z))
//   Theta-Theta  A[(z,c),(w,d)] = [c=d] <B001_z, B001_w> - [z=w] S3(c,d)
// with M = B100, S1 = <F, F>_{-1}, S3 = <F, F>_{-3}.
void newton_matrix(const Blocks &B, std::vector<double> &H) {
    const int r = B.r, r3 = B.r3, A1 = B.A1, C1 = B.C1;
    const int nd = A1 * r, nt = C1 * r3, N = nd + nt;
    const int rr = r * r;
    // every Delta row is written in full below; the Theta rows accumulate
    H.resize((size_t)N * N);
    std::fill(H.begin() + (size_t)nd * N, H.end(), 0.0);
    auto Fv = [&](int a, int b, int c) { return B.F[a + r * (b + (size_t)r * c)]; };
    auto M = [&](int x, int b, int c) { return B.B100[x + (size_t)A1 * (b + (size_t)r * c)]; };
    auto B001 = [&](int a, int b, int z) { return B.B001[a + r * (b + (size_t)r * z)]; };
    std::vector<double> S1((size_t)r * r, 0.0), S3((size_t)r3 * r3, 0.0);
    for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b) {
            double s = 0.0;
            for (int c = 0; c < r3; ++c)
                for (int y = 0; y < r; ++y) s += Fv(a, y, c) * Fv(b, y, c);
            S1[(size_t)a * r + b] = s;
        }
    for (int c = 0; c < r3; ++c)
        for (int d = 0; d < r3; ++d) {
            double s = 0.0;
            for (int a = 0; a < r; ++a)
                for (int b = 0; b < r; ++b) s += Fv(a, b, c) * Fv(a, b, d);
            S3[(size_t)c * r3 + d] = s;
        }
    // Delta-Delta: Gx[(x,b),(y,a)] = sum_c M(x,b,c) M(y,a,c); K[(x,y),(a,b)] =
    // sum_c B110(x,y,c) F(a,b,c)
    // thread-local workspaces: reused across calls (large cores need ~60 MB,
    // whose first touch would otherwise dominate)
    // (the lambdas below run on pool threads: they must see the caller's
    // instances, hence the local references)
    struct Work {
        std::vector<double> Mt, B110t, Ft, Gx, K, MM, Mxc, B001t, B101t, Fb, T1, T2;
    };
    static thread_local Work tl_work;
    Work &w_ = tl_work;
    auto &Mt = w_.Mt, &B110t = w_.B110t, &Ft = w_.Ft, &Gx = w_.Gx, &K = w_.K, &MM = w_.MM;
    auto &Mxc = w_.Mxc, &B001t = w_.B001t, &B101t = w_.B101t, &Fb = w_.Fb, &T1 = w_.T1,
         &T2 = w_.T2;
    Mt.resize((size_t)nd * r3);
    B110t.resize((size_t)A1 * A1 * r3);
    Ft.resize((size_t)r3 * rr);
    for (int x = 0; x < A1; ++x)
        for (int b = 0; b < r; ++b)
            for (int c = 0; c < r3; ++c) Mt[((size_t)x * r + b) * r3 + c] = M(x, b, c);
    for (int c = 0; c < r3; ++c)
        for (int y = 0; y < A1; ++y)
            for (int x = 0; x < A1; ++x)
                B110t[((size_t)x * A1 + y) * r3 + c] = B.B110[x + (size_t)A1 * (y + (size_t)A1 * c)];
    for (int c = 0; c < r3; ++c)
        for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b) Ft[(size_t)c * rr + a * r + b] = Fv(a, b, c);
    Gx.resize((size_t)nd * nd);
    K.resize((size_t)A1 * A1 * rr);
    la::dgemm(false, true, nd, nd, r3, 1.0, Mt.data(), r3, Mt.data(), r3, 0.0, Gx.data(), nd, true);
    la::dgemm(false, false, A1 * A1, rr, r3, 1.0, B110t.data(), r3, Ft.data(), rr, 0.0, K.data(), rr,
              true);
    // MM = <M_x, M_y> = Mflat Mflat^T, Mflat(x, (b,c)) = M(x,b,c) (contiguous: Mt)
    MM.resize((size_t)A1 * A1);
    la::dgemm(false, true, A1, A1, r * r3, 1.0, Mt.data(), r * r3, Mt.data(), r * r3, 0.0,
              MM.data(), A1, true);
    // Delta-Theta: T1[(x,c),(a,z)] = sum_b M(x,b,c) B001(a,b,z);
    // T2[(x,z),(a,c)] = sum_b B101(x,b,z) F(a,b,c)
    Mxc.resize((size_t)A1 * r3 * r);
    B001t.resize((size_t)r * r * C1);
    B101t.resize((size_t)A1 * C1 * r);
    Fb.resize((size_t)r * r * r3);
    for (int x = 0; x < A1; ++x)
        for (int c = 0; c < r3; ++c)
            for (int b = 0; b < r; ++b) Mxc[((size_t)x * r3 + c) * r + b] = M(x, b, c);
    for (int b = 0; b < r; ++b)
        for (int a = 0; a < r; ++a)
            for (int z = 0; z < C1; ++z) B001t[(size_t)b * (r * C1) + a * C1 + z] = B001(a, b, z);
    for (int x = 0; x < A1; ++x)
        for (int z = 0; z < C1; ++z)
            for (int b = 0; b < r; ++b)
                B101t[((size_t)x * C1 + z) * r + b] = B.B101[x + (size_t)A1 * (b + (size_t)r * z)];
    for (int b = 0; b < r; ++b)
        for (int a = 0; a < r; ++a)
            for (int c = 0; c < r3; ++c) Fb[(size_t)b * (r * r3) + a * r3 + c] = Fv(a, b, c);
    T1.resize((size_t)A1 * r3 * r * C1);
    T2.resize((size_t)A1 * C1 * r * r3);
    if (C1 > 0) {
        la::dgemm(false, false, A1 * r3, r * C1, r, 1.0, Mxc.data(), r, B001t.data(), r * C1, 0.0,
                  T1.data(), r * C1, true);
        la::dgemm(false, false, A1 * C1, r * r3, r, 1.0, B101t.data(), r, Fb.data(), r * r3, 0.0,
                  T2.data(), r * r3, true);
    }
    // assemble H = -2A (rows of the Delta part; Theta rows by symmetry below)
    la::parallel_for(A1, [&](int x) {
        for (int a = 0; a < r; ++a) {
            double *h = &H[((size_t)x * r + a) * N];
            for (int y = 0; y < A1; ++y) {
                const double *k = &K[((size_t)x * A1 + y) * rr + (size_t)a * r];
                // Gx[(x,b),(y,a)] = Gx[(y,a),(x,b)] (exactly symmetric): contiguous in b
                const double *g = &Gx[((size_t)y * r + a) * nd + (size_t)x * r];
                for (int b = 0; b < r; ++b) {
                    double v = 2.0 * g[b] + 2.0 * k[b];
                    if (a == b) v += 2.0 * MM[(size_t)x * A1 + y];
                    if (x == y) v -= 2.0 * S1[(size_t)a * r + b];
                    h[y * r + b] = -2.0 * v;
                }
            }
            // two passes, each reading its product contiguously
            for (int c = 0; c < r3; ++c) {
                const double *t1 = &T1[((size_t)x * r3 + c) * (r * C1) + (size_t)a * C1];
                for (int z = 0; z < C1; ++z) h[nd + z * r3 + c] = -4.0 * t1[z];
            }
            for (int z = 0; z < C1; ++z) {
                const double *t2 = &T2[((size_t)x * C1 + z) * (r * r3) + (size_t)a * r3];
                for (int c = 0; c < r3; ++c) h[nd + z * r3 + c] -= 4.0 * t2[c];
            }
        }
    });
    // Theta-Theta
    for (int z = 0; z < C1; ++z)
        for (int w = 0; w <= z; ++w) {
            double s = 0.0;
            for (int b = 0; b < r; ++b)
                for (int a = 0; a < r; ++a) s += B001(a, b, z) * B001(a, b, w);
            for (int c = 0; c < r3; ++c) {
                const int i1 = nd + z * r3 + c, j1 = nd + w * r3 + c;
                H[(size_t)i1 * N + j1] += -2.0 * s;
                if (w != z) H[(size_t)j1 * N + i1] += -2.0 * s;
            }
        }
    for (int z = 0; z < C1; ++z)
        for (int c = 0; c < r3; ++c)
            for (int d = 0; d < r3; ++d)
                H[(size_t)(nd + z * r3 + c) * N + nd + z * r3 + d] -= -2.0 * S3[(size_t)c * r3 + d];
    // exact symmetry, in 32 x 32 tiles (tile row ti owns the tiles (ti, tj >= ti));
    // the Theta rows' Delta columns are only filled here, by copy
    const int TS = 32, nt_ = (N + TS - 1) / TS;
    la::parallel_for(nt_, [&](int ti) {
        for (int tj = ti; tj < nt_; ++tj)
            for (int i = ti * TS; i < std::min(N, ti * TS + TS); ++i)
                for (int j = std::max(i + 1, tj * TS); j < std::min(N, tj * TS + TS); ++j) {
                    if (i < nd && j >= nd) {
                        H[(size_t)j * N + i] = H[(size_t)i * N + j];
                        continue;
                    }
                    const double s = 0.5 * (H[(size_t)i * N + j] + H[(size_t)j * N + i]);
                    H[(size_t)i * N + j] = H[(size_t)j * N + i] = s;
                }
    });
}

// g(P, S) = ||C.(P, P, S)||^2
double objective(const View &V, const std::vector<double> &P, const std::vector<double> &S, int r,
                 int r3) {
    const int k1 = V.k1;
    const size_t sl = (size_t)k1 * k1;
    std::vector<double> gl(r3, 0.0);
    if (V.dev && V.hooi_dev) {
        // M_l = CS_l P on the device; g = sum_l ||P^T M_l||^2
        std::vector<double> M((size_t)k1 * r * r3);
        V.dev->mode3p(S.data(), r3, 0, r3, P.data(), r, M.data());
        for (int l = 0; l < r3; ++l)
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < r; ++j) {
                    double t = 0.0;
                    for (int a = 0; a < k1; ++a)
                        t += P[(size_t)a * r + i] * M[a + (size_t)k1 * (j + (size_t)r * l)];
                    gl[l] += t * t;
                }
        double g = 0.0;
        for (double v : gl) g += v;
        return g;
    }
    std::vector<double> CS;
    mode3_product(V, S.data(), r3, 0, r3, CS);
    la::parallel_for(r3, [&](int l) {
        std::vector<double> t((size_t)k1 * r), T((size_t)r * r);
        la::dgemm(false, false, k1, r, k1, 1.0, &CS[sl * l], k1, P.data(), r, 0.0, t.data(), r);
        la::dgemm(true, false, r, r, k1, 1.0, P.data(), r, t.data(), r, 0.0, T.data(), r);
        double g = 0.0;
        for (double v : T) g += v * v;
        gl[l] = g;
    });
    double g = 0.0;
    for (double v : gl) g += v;
    return g;
}

// orth(Q(:, :r) + Q(:, r:) D), Q k x k row-major, D (k-r) x r row-major
void retract(int k, int r, const std::vector<double> &Q, const double *D, std::vector<double> &out) {
    out.assign((size_t)k * r, 0.0);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < r; ++j) {
            double s = Q[(size_t)i * k + j];
            for (int x = 0; x < k - r; ++x) s += Q[(size_t)i * k + r + x] * D[(size_t)x * r + j];
            out[(size_t)i * r + j] = s;
        }
    la::orthonormalize(k, r, out.data());
}

}  // namespace

double device_core_min() {
    static const double v = [] {
        const char *e = std::getenv("BKS_DEVICE_CORE_MIN");
        return e ? std::atof(e) : kDeviceCoreMin;
    }();
    return v;
}

double device_hooi_min() {
    static const double v = [] {
        const char *e = std::getenv("BKS_DEVICE_HOOI_MIN");
        return e ? std::atof(e) : kDeviceHooiMin;
    }();
    return v;
}

int device_solve_min() {
    static const int v = [] {
        const char *e = std::getenv("BKS_DEVICE_SOLVE_MIN");
        return e ? std::atoi(e) : kDeviceSolveMin;
    }();
    return v;
}

double inner_objective(const std::vector<double> &C, int k1, int k3, const std::vector<double> &P,
                       const std::vector<double> &S, int r, int r3, InnerDevice *dev) {
    View V{C.data(), k1, k3, dev};
    return objective(V, P, S, r, r3);
}

void inner_solve(const std::vector<double> &C, int k1, int k3, int r, int r3, double tol,
                 int hooi_warm, int ng_max, bool warm, std::vector<double> &P,
                 std::vector<double> &S, InnerInfo &info, const BigSolve &big,
                 InnerDevice *dev, double dev_min) {
    View V{C.data(), k1, k3, nullptr};
    if (dev && (double)k1 * k1 * k3 >= dev_min) {
        dev->set_core(C.data(), k1, k3);
        V.dev = dev;
        V.hooi_dev = (double)k1 * k1 * k3 >= device_hooi_min();
    }
    info = InnerInfo{};
    auto clk = [] {
        return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
            .count();
    };
    double t0 = clk();
    if (!warm) {
        hosvd(V, r, r3, P, S);
        for (int it = 0; it < hooi_warm; ++it) hooi_step(V, r, r3, P, S);
    }
    info.t_start = clk() - t0;
    Blocks B, Bn;
    // with the products on the device, a trial point is judged from its
    // rotation (g = ||F||^2 of the rotated core, the same sum of squares the
    // objective forms), which an accepted step keeps for the next iteration
    bool have_B = false;
    // a device that forms the Newton matrix itself returns only the blocks
    // the gradient reads from each rotation
    const int n_newton = (k1 - r) * r + (k3 - r3) * r3;
    const bool partial = big && V.dev && V.dev->forms_newton() && n_newton >= device_solve_min();
    std::vector<double> G1, G3, d, Pn, Sn;
    // the Newton matrices (60 MB at rank (10,10,10)) are reused across calls
    static thread_local std::vector<double> tl_H, tl_Hs;
    std::vector<double> &H = tl_H, &Hs = tl_Hs;
    std::vector<double> hdiag;
    double mu = 0.0;
    double prev = INFINITY;
    int stall = 0;
    bool last_plain = false;
    while (true) {
        t0 = clk();
        if (!have_B) rotate(V, P, S, r, r3, B, partial);
        have_B = false;
        double nf;
        info.rel = local_gradient(B, G1, G3, nf);
        info.t_rotate += clk() - t0;
        if (info.rel <= tol || info.iters >= ng_max) break;
        // at the rounding floor the gradient stops shrinking: two steps in a
        // row that do not halve it below 1e-9 end the iteration (above 1e-9
        // only undamped steps count: damped ones may legitimately progress
        // slowly far from the maximum)
        const bool at_floor = info.rel < 1e-9;
        stall = ((last_plain || at_floor) && at_floor && info.rel > 0.5 * prev) ? stall + 1 : 0;
        if (stall >= 2) break;
        prev = info.rel;
        if (B.A1 * r + B.C1 * r3 == 0) break;
        const int nd = B.A1 * r, N = nd + B.C1 * r3;
        t0 = clk();
        // large systems: the matrix is formed and factorised on the device
        // when the device provides it, else formed here
        hdiag.resize(N);
        const bool dev_h = big && V.dev && N >= device_solve_min() &&
                           V.dev->newton_matrix(r, r3, hdiag.data());
        if (!dev_h) {
            // the host forms H: it needs the whole rotation
            if (B.partial) rotate(V, P, S, r, r3, B, false);
            newton_matrix(B, H);
            for (int i = 0; i < N; ++i) hdiag[i] = H[(size_t)i * N + i];
        }
        info.t_hess += clk() - t0;
        // Safeguarded Newton step (a reading: the paper cites the method
        // only): solve (-2A + mu I) d = b with the smallest tried shift that
        // makes the matrix positive definite and the step increase g; mu = 0
        // near a maximum gives the plain Newton step.
        double hmax = 0.0;
        for (int i = 0; i < N; ++i) hmax = std::max(hmax, std::fabs(hdiag[i]));
        const double mu0 = 1e-8 * std::max(hmax, 1e-300);
        const double g0 = nf * nf;
        bool accepted = false;
        // far below 1e-9 no ascent direction survives rounding after a few
        // shifts: there a rejected step ends the iteration
        const bool deep_floor = info.rel < 1e-10;
        const int max_attempts = deep_floor ? 4 : 12;
        for (int attempt = 0; attempt < max_attempts && !accepted; ++attempt) {
            const bool on_device = big && N >= device_solve_min();
            if (!on_device) {
                Hs = H;
                for (int i = 0; i < N; ++i) Hs[(size_t)i * N + i] += mu;
            }
            d.assign(N, 0.0);
            for (int i = 0; i < nd; ++i) d[i] = 4.0 * G1[i];
            for (int i = 0; i < N - nd; ++i) d[nd + i] = 2.0 * G3[i];
            t0 = clk();
            if (on_device) {
                const bool pd = dev_h ? V.dev->newton_solve(mu, d.data())
                                      : big(N, H.data(), mu, attempt == 0, d.data());
                info.t_chol += clk() - t0;
                if (!pd) {
                    // no pivot from the device factorisation: escalate by 10
                    mu = std::max(10.0 * mu, mu0);
                    continue;
                }
            } else {
                double piv = 0.0;
                const bool pd = la::cholesky(N, Hs.data(), &piv);
                info.t_chol += clk() - t0;
                if (!pd) {
                    // the failed pivot bounds how far the spectrum reaches below 0
                    mu = std::max({4.0 * mu, mu0, mu + 2.0 * std::fabs(piv)});
                    continue;
                }
                la::chol_solve(N, Hs.data(), d.data());
            }
            retract(k1, r, B.Qp, d.data(), Pn);
            retract(k3, r3, B.Qs, d.data() + nd, Sn);
            double g1;
            if (V.dev) {
                t0 = clk();
                rotate(V, Pn, Sn, r, r3, Bn, partial);
                info.t_rotate += clk() - t0;
                g1 = 0.0;
                for (double v : Bn.F) g1 += v * v;
            } else {
                g1 = objective(V, Pn, Sn, r, r3);
            }
            // g is a sum of ~k1^2 k3 rounded products: changes below 1e-13
            // relative are rounding noise, not descent
            if (g1 >= g0 * (1.0 - 1e-13)) {
                accepted = true;
                last_plain = (mu == 0.0);
                P.swap(Pn);
                S.swap(Sn);
                if (V.dev) {
                    std::swap(B, Bn);
                    have_B = true;
                }
                mu = mu > mu0 ? mu / 4.0 : 0.0;
            } else {
                mu = std::max(4.0 * mu, mu0);
            }
        }
        ++info.iters;
        if (accepted) {
            ++info.newton;
        } else {
            // no step raises g: at the floor that is the maximum to rounding
            if (deep_floor) break;
            last_plain = false;
            hooi_step(V, r, r3, P, S);
        }
    }
}

}  // namespace bks
