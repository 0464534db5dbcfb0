// Device-side Rotne-Prager-Yamakawa block, Eqs. 7-9 of arXiv 2208.06559.
#pragma once
#include <hip/hip_runtime.h>

namespace bd {

// Coefficients of D_ij = cI * I + cRR * R R^T for R = r_i - r_j, i != j.
//  far field  (|R| >= 2a, Eq. 8): (3h*/4R) [(1 + 2a^2/3R^2) I + (1 - 2a^2/R^2) RR^T/R^2]
//  near field (|R| <  2a, Eq. 9): (3h*/8a) [(8/3 - 3R/4a) I + RR^T/(4aR)], where
//  (3h*/4R)(R/2a) = 3h*/8a; the RR^T term is taken as 0 at R = 0.
__device__ __forceinline__ void rpy_coeffs(double R2, double hstar, double a, double& cI,
                                           double& cRR) {
  const double R = sqrt(R2);
  if (R >= 2.0 * a) {
    const double pre = 3.0 * hstar / (4.0 * R);
    const double a2 = a * a;
    cI = pre * (1.0 + 2.0 * a2 / (3.0 * R2));
    cRR = pre * (1.0 - 2.0 * a2 / R2) / R2;
  } else {
    const double pre = 3.0 * hstar / (8.0 * a);
    cI = pre * (8.0 / 3.0 - 3.0 * R / (4.0 * a));
    cRR = (R > 0.0) ? pre / (4.0 * a * R) : 0.0;
  }
}

}  // namespace bd
