// Device-resident LSQR state (one per right-hand side being iterated).
#pragma once
#include <cstdint>

namespace rfmls {
struct LsqrDev {
  double alpha, beta, alpha_prev, rhobar, phibar, bnorm, anorm2, ddnorm;
  double normr, normar, acond, ynorm, phi_rho, theta_rho;
  double atol, btol, conlim;
  int64_t itn, itmax;
  int32_t istop, pending, done, pad;
};
}  // namespace rfmls
