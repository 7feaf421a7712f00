// Internal declarations shared by the library's translation units.
#pragma once
#include <cstdint>

#include "lbm.h"

namespace lbm {

// Equation-of-state constants, FP64.
//   C-S:  p = rho RT (1 + e + e^2 - e^3)/(1 - e)^3 - c2 rho^2,  e = c1 rho (c1 = b/4, c2 = a)
//   P-R:  p = rho RT/(1 - c1 rho) - c2 rho^2/(1 + c1 rho (2 - c1 rho))  (c1 = b, c2 = a alpha(T))
// psi^2 = (p - rho/3) * two_over_G   (Eq. 8, c = 1)
struct EosConst {
  int32_t kind;
  double RT, c1, c2, two_over_G;
};

double pr_kappa(double omega);
int critical_point(int32_t eos, double a, double b, double R, double omega, double* Tc, double* rc);
int maxwell(int32_t eos, double a, double b, double R, double omega, double T, double* rl,
            double* rg, double* p0);
int eos_constants(const lbm_params& p, EosConst* k);
double pressure(const EosConst& k, double rho);

}  // namespace lbm
