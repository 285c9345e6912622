// Power-series coefficients of the Chebyshev polynomials (ChebConv basis,
// paper Sec. 3.2): T_k(t) = sum_m t[k][m] t^m for k, m <= 8.  Shared by the
// host-side parameter conversion and the device gradient conversion.
#pragma once

namespace mgl {

struct ChebTab {
  double t[9][9];
};

}  // namespace mgl
