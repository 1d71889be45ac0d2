// Best rank-(r, r, r3) approximation of the dense projected core
// C = A.(X, X, Z) (Algorithm 5 step (i), eq. maxrC).
#pragma once

#include <functional>
#include <vector>

namespace bks {

// Optional solver for large Newton systems: solve (H + mu I) x = b in place
// of b (H N x N symmetric row-major); returns false if H + mu I is not
// positive definite.  `new_matrix` is false when H is the same as in the
// previous call (only mu changed).
using BigSolve = std::function<bool(int N, const double *H, double mu, bool new_matrix, double *b)>;
constexpr int kDeviceSolveMin = 256;

// Optional device for the dense products of large cores.  After set_core
// (C uploaded, layout as below) every call is synchronous and returns host
// results:
//   gram1:  G1 = C_(1) C_(1)^T (k1 x k1)          gram3: G3 = C_(3) C_(3)^T (k3 x k3)
//   mode3p: out(a + k1*(j + r*l)) = sum_b [sum_c C(a,b,c) Sv(c, l0 + l)] P(b, j),
//           l < nl (Sv k3 x ldS, P k1 x r, row-major): the mode-3 product
//           times P in mode 2
//   hooi3:  M3(c, i + r*j) = sum_{a,b} C(a,b,c) P(a,i) P(b,j) (P k1 x r row-major)
//   rotate: with Qp (k1 x k1) and Qs (k3 x k3) row-major orthogonal,
//           X_l = C.(I, I, Qs(:,l)); Y(x, y, l) = (Qp^T X_l Qp)(x, y) for l < r3
//           at x + k1*(y + k1*l), Y2(x, j, z) = (Qp^T X_{r3+z} Qp(:, :r))(x, j)
//           at x + k1*(j + r*z), z < k3 - r3; with `partial`, only the
//           blocks the gradient reads: Y(x, y, l) for y < r at
//           x + k1*(y + r*l) and Y2(x, j, z) for x < r at x + r*(j + r*z)
//           (a device that forms the Newton matrix keeps the rest)
// Results equal the host products up to rounding order.
struct InnerDevice {
    virtual ~InnerDevice() = default;
    virtual void set_core(const double *C, int k1, int k3) = 0;
    virtual void gram1(double *G1) = 0;
    virtual void gram3(double *G3) = 0;
    virtual void mode3p(const double *Sv, int ldS, int l0, int nl, const double *P, int r,
                        double *out) = 0;
    virtual void hooi3(const double *P, int r, double *M3) = 0;
    virtual void rotate(const double *Qp, const double *Qs, int r, int r3, double *Y,
                        double *Y2, bool partial) = 0;
    // true if newton_matrix forms the Newton matrix on the device (the inner
    // solve then asks rotate for partial results)
    virtual bool forms_newton() const { return false; }
    // The Newton matrix H of the last rotate() (the entries newton_matrix
    // states) formed and kept on the device, its N diagonal entries copied
    // to diag; false if the device does not provide it (the host forms H).
    virtual bool newton_matrix(int r, int r3, double *diag) {
        (void)r, (void)r3, (void)diag;
        return false;
    }
    // Solve (H + mu I) x = b with that matrix, in place of b; false if the
    // shifted matrix is not positive definite.
    virtual bool newton_solve(double mu, double *b) {
        (void)mu, (void)b;
        return false;
    }
};
// Cores with at least this many entries (k1^2 k3) use the device when given
// (BKS_DEVICE_CORE_MIN overrides); Newton systems of at least
// device_solve_min() unknowns are factorised on the device
// (BKS_DEVICE_SOLVE_MIN overrides).
constexpr double kDeviceCoreMin = 1.0e5;
double device_core_min();
// ... of which those with k1^2 k3 >= device_hooi_min() (BKS_DEVICE_HOOI_MIN)
// also run the HOOI steps' and the objective's products there
constexpr double kDeviceHooiMin = kDeviceCoreMin;
double device_hooi_min();
int device_solve_min();

struct InnerInfo {
    int iters = 0;        // Newton-Grassmann iterations (incl. HOOI fallbacks)
    int newton = 0;       // Newton steps taken
    double rel = 0.0;     // final relative local gradient
    double t_start = 0, t_rotate = 0, t_hess = 0, t_chol = 0;  // seconds
};

// C: k1 x k1 x k3, column-major (a + k1*(b + k1*c)), symmetric in a, b.
// P (k1 x r) and S (k3 x r3), row-major, are outputs; with `warm` they are
// also the start (else HOSVD + hooi_warm HOOI steps, section "Experiments").
// g(P, S) = ||C.(P, P, S)||^2 (P k1 x r, S k3 x r3, row-major)
double inner_objective(const std::vector<double> &C, int k1, int k3, const std::vector<double> &P,
                       const std::vector<double> &S, int r, int r3, InnerDevice *dev = nullptr);

void inner_solve(const std::vector<double> &C, int k1, int k3, int r, int r3, double tol,
                 int hooi_warm, int ng_max, bool warm, std::vector<double> &P,
                 std::vector<double> &S, InnerInfo &info, const BigSolve &big = BigSolve(),
                 InnerDevice *dev = nullptr, double dev_min = kDeviceCoreMin);

}  // namespace bks
