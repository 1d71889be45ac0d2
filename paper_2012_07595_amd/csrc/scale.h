// Slice scalings of a (1,2)-symmetric tensor applied at upload (host logic,
// no HIP): section "Experiments", Example 3 (every slice scaled so that its
// largest eigenvalue is 1) and Example 4 (every slice scaled to Frobenius
// norm 1).
#pragma once

#include <cstdint>

namespace bks {

// Largest eigenvalue magnitude of the symmetric matrix whose stored entries
// are (lo[e] <= hi[e], v[e]), e < cnt, each off-diagonal entry standing for
// both (lo, hi) and (hi, lo); rows are arbitrary labels.  Dense symmetric
// eigensolver on the touched rows up to kDenseRows of them, else Lanczos
// with full reorthogonalisation until the largest Ritz value's residual is
// below 1e-14 of it (at most kLanczosSteps steps).  0 for an empty matrix.
constexpr int kDenseRows = 400;
constexpr int kLanczosSteps = 400;
double sym_spectral_radius(int64_t cnt, const int64_t *lo, const int64_t *hi, const double *v);

// Frobenius norm of the full symmetric matrix (off-diagonal entries twice).
double sym_frobenius(int64_t cnt, const int64_t *lo, const int64_t *hi, const double *v);

}  // namespace bks
