// Host float64 pieces of the fits that device code also uses.
#pragma once

#include <cstdint>

namespace lv {

// Projection onto the spectral-norm ball (Eq. stiefel_convex_hull) from the
// d x d Gram matrix M M^T: T (d x d, row-major) with T M the projection of M.
// Returns false, leaving T untouched, when no singular value exceeds 1.
bool clip_factor(int32_t d, const double *MMt, double *T);

}  // namespace lv
