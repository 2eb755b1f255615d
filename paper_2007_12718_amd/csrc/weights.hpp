// Corrected-trapezoidal (Duan-Rokhlin order 4/6/8/10) weights, host side.
#pragma once
#include <vector>

#include "common.hpp"

namespace lsh {

// Dimensionless correction tau_d at stencil offset (dx, dy): the matrix entry
// coupling a target to the source at offset d is h^2 (G(h|d|)[d != 0] + tau_d).
struct StencilEntry {
  int dx, dy;
  double re, im;
};

// kappa-independent orbit weights tau' (1, 2, 4 or 6 values).
std::vector<double> orbit_weights(int order);
// All stencil points of the given order (1, 5, 13 or 25) at this kappa*h.
std::vector<StencilEntry> correction_stencil(int order, double kh);

}  // namespace lsh
