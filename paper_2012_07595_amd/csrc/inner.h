// Best rank-(r, r, r3) approximation of the dense projected core
// C = A.(X, X, Z) (Algorithm 5 step (i), eq. maxrC).
#pragma once

#include <functional>
#include <vector>

namespace bks {

// Optional solver for large Newton systems: solve H x = b in place of b
// (H N x N symmetric row-major); returns false if H is not positive definite.
using BigSolve = std::function<bool(int N, const double *H, double *b)>;
constexpr int kDeviceSolveMin = 512;

struct InnerInfo {
    int iters = 0;        // Newton-Grassmann iterations (incl. HOOI fallbacks)
    int newton = 0;       // Newton steps taken
    double rel = 0.0;     // final relative local gradient
    double t_start = 0, t_rotate = 0, t_hess = 0, t_chol = 0;  // seconds
};

// C: k1 x k1 x k3, column-major (a + k1*(b + k1*c)), symmetric in a, b.
// P (k1 x r) and S (k3 x r3), row-major, are outputs; with `warm` they are
// also the start (else HOSVD + hooi_warm HOOI steps, Section 5.2).
// g(P, S) = ||C.(P, P, S)||^2 (P k1 x r, S k3 x r3, row-major)
double inner_objective(const std::vector<double> &C, int k1, int k3, const std::vector<double> &P,
                       const std::vector<double> &S, int r, int r3);

void inner_solve(const std::vector<double> &C, int k1, int k3, int r, int r3, double tol,
                 int hooi_warm, int ng_max, bool warm, std::vector<double> &P,
                 std::vector<double> &S, InnerInfo &info, const BigSolve &big = BigSolve());

}  // namespace bks
