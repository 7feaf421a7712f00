// Host-side thermodynamics of the library: equations of state, critical
// points and the Maxwell construction (paper Sec. II Eq. 7, Sec. III.C Eq. 23).
//
// The critical point is reduced to one equation in the packing variable and
// solved by bisection; the Maxwell construction is solved as equality of
// pressure and chemical potential, bracketing the pressure between the two
// spinodal pressures.
#include <cmath>
#include <cstdint>

#include "lbm.h"
#include "lbm_internal.h"

namespace lbm {

double pr_kappa(double omega) { return 0.37464 + 1.54226 * omega - 0.26992 * omega * omega; }

namespace {

// Carnahan-Starling: p = rho R T Z(eta) - a rho^2, Z = (1+eta+eta^2-eta^3)/(1-eta)^3, eta = b rho/4.
struct CS {
  double a, b, R, T;
  double p(double r) const {
    double e = b * r / 4, m = 1 - e;
    return r * R * T * (1 + e + e * e - e * e * e) / (m * m * m) - a * r * r;
  }
  double dp(double r) const {
    double e = b * r / 4, m = 1 - e;
    return R * T * (1 + 4 * e + 4 * e * e - 4 * e * e * e + e * e * e * e) / (m * m * m * m) - 2 * a * r;
  }
  double mu(double r) const {
    double e = b * r / 4, m = 1 - e;
    return R * T * (std::log(r) + (8 * e - 9 * e * e + 3 * e * e * e) / (m * m * m)) - 2 * a * r;
  }
  double rmax() const { return 4 / b; }
};

// Peng-Robinson with the attraction already multiplied by alpha(T).
struct PR {
  double aa, b, R, T;
  double p(double r) const {
    return r * R * T / (1 - b * r) - aa * r * r / (1 + 2 * b * r - b * b * r * r);
  }
  double dp(double r) const {
    double D = 1 + 2 * b * r - b * b * r * r, m = 1 - b * r;
    return R * T / (m * m) - aa * 2 * r * (1 + b * r) / (D * D);
  }
  double mu(double r) const {
    const double s2 = std::sqrt(2.0);
    double D = 1 + 2 * b * r - b * b * r * r, m = 1 - b * r;
    return R * T * (std::log(r / m) + 1 / m) +
           aa / (2 * s2 * b) * std::log((1 + (1 - s2) * b * r) / (1 + (1 + s2) * b * r)) - aa * r / D;
  }
  double rmax() const { return 1 / b; }
};

template <class F>
double bisect(F f, double lo, double hi, int iters = 200) {
  double flo = f(lo);
  for (int i = 0; i < iters; ++i) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    double fm = f(mid);
    if ((fm > 0) == (flo > 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

// Maxwell construction for one EOS object: returns false when T >= Tc.
template <class E>
bool maxwell_eos(const E& e, double* rl, double* rg, double* p0) {
  const int n = 4000;
  double rm = e.rmax();
  double sp[2];
  int ns = 0;
  double prev = e.dp(rm / n);
  for (int k = 2; k < n && ns < 2; ++k) {
    double r = rm * k / n, v = e.dp(r);
    if ((prev > 0) != (v > 0)) {
      double lo = rm * (k - 1) / n;
      sp[ns++] = bisect([&](double s) { return e.dp(s); }, lo, r);
    }
    prev = v;
  }
  if (ns < 2) return false;
  double pmax = e.p(sp[0]), pmin = e.p(sp[1]);
  if (pmin < pmax * 1e-12) pmin = pmax * 1e-12;
  auto gas = [&](double q) { return bisect([&](double s) { return e.p(s) - q; }, 0.0, sp[0]); };
  auto liq = [&](double q) {
    double hi = sp[1] + 0.5 * (rm - sp[1]);
    double step = 0.5 * (rm - sp[1]);
    while (e.p(hi) < q && step > 1e-300) {  // walk towards rho_max until p exceeds q
      step *= 0.5;
      hi += step;
    }
    return bisect([&](double s) { return e.p(s) - q; }, sp[1], hi);
  };
  // mu(liquid) - mu(gas) increases with the trial pressure q
  auto resid = [&](double q) { return e.mu(liq(q)) - e.mu(gas(q)); };
  double q = bisect(resid, pmin, pmax, 120);
  *rl = liq(q);
  *rg = gas(q);
  *p0 = q;
  return true;
}

// C-S critical packing: eta N'(eta)(1 - eta) + N(eta)(5 eta - 1) = 0 with
// N = 1 + 4e + 4e^2 - 4e^3 + e^4 (from dp = 0 and d2p = 0 eliminating T).
void cs_critical(double a, double b, double R, double* Tc, double* rc) {
  auto N = [](double e) { return 1 + 4 * e + 4 * e * e - 4 * e * e * e + e * e * e * e; };
  auto Np = [](double e) { return 4 + 8 * e - 12 * e * e + 4 * e * e * e; };
  double eta = bisect([&](double e) { return e * Np(e) * (1 - e) + N(e) * (5 * e - 1); }, 0.01, 0.5);
  double m = 1 - eta;
  double A = N(eta) / (m * m * m * m);
  *rc = 4 * eta / b;
  *Tc = 8 * a * eta / (b * R * A);
}

// P-R (alpha = 1) critical point in x = b rho: h'(x) (1 - x) = 2 h(x),
// h = x (1 + x) / D^2, D = 1 + 2x - x^2; then R Tc = (a/b) 2 h (1 - x)^2.
void pr_critical(double a, double b, double R, double* Tc, double* rc) {
  auto h = [](double x) {
    double D = 1 + 2 * x - x * x;
    return x * (1 + x) / (D * D);
  };
  auto hp = [](double x) {
    double D = 1 + 2 * x - x * x, Dp = 2 - 2 * x;
    return ((1 + 2 * x) * D - 2 * x * (1 + x) * Dp) / (D * D * D);
  };
  double x = bisect([&](double s) { return hp(s) * (1 - s) - 2 * h(s); }, 0.05, 0.6);
  *rc = x / b;
  *Tc = a / (b * R) * 2 * h(x) * (1 - x) * (1 - x);
}

}  // namespace

int critical_point(int32_t eos, double a, double b, double R, double /*omega*/, double* Tc,
                   double* rc) {
  if (!(a > 0) || !(b > 0) || !(R > 0)) return LBM_EINVAL;
  if (eos == LBM_EOS_CS)
    cs_critical(a, b, R, Tc, rc);
  else if (eos == LBM_EOS_PR)
    pr_critical(a, b, R, Tc, rc);
  else
    return LBM_EINVAL;
  return LBM_OK;
}

int eos_constants(const lbm_params& p, EosConst* k) {
  k->kind = p.eos;
  k->RT = p.R * p.T;
  k->two_over_G = 2.0 / p.G;
  if (p.eos == LBM_EOS_CS) {
    k->c1 = p.b / 4;
    k->c2 = p.a;
    return LBM_OK;
  }
  if (p.eos == LBM_EOS_PR) {
    double Tc, rc;
    pr_critical(p.a, p.b, p.R, &Tc, &rc);
    double s = 1 + pr_kappa(p.omega) * (1 - std::sqrt(p.T / Tc));
    k->c1 = p.b;
    k->c2 = p.a * s * s;
    return LBM_OK;
  }
  return LBM_EINVAL;
}

double pressure(const EosConst& k, double rho) {
  if (k.kind == LBM_EOS_CS) {
    double e = k.c1 * rho, m = 1 - e;
    return rho * k.RT * (1 + e * (1 + e * (1 - e))) / (m * m * m) - k.c2 * rho * rho;
  }
  return rho * k.RT / (1 - k.c1 * rho) - k.c2 * rho * rho / (1 + k.c1 * rho * (2 - k.c1 * rho));
}

int maxwell(int32_t eos, double a, double b, double R, double omega, double T, double* rl,
            double* rg, double* p0) {
  if (!(T > 0)) return LBM_EINVAL;
  bool ok;
  if (eos == LBM_EOS_CS) {
    ok = maxwell_eos(CS{a, b, R, T}, rl, rg, p0);
  } else if (eos == LBM_EOS_PR) {
    double Tc, rc;
    pr_critical(a, b, R, &Tc, &rc);
    double s = 1 + pr_kappa(omega) * (1 - std::sqrt(T / Tc));
    ok = maxwell_eos(PR{a * s * s, b, R, T}, rl, rg, p0);
  } else {
    return LBM_EINVAL;
  }
  return ok ? LBM_OK : LBM_EINVAL;
}

}  // namespace lbm

extern "C" int lbm_critical_point(int32_t eos, double a, double b, double R, double omega,
                                  double* Tc, double* rho_c) {
  if (!Tc || !rho_c) return LBM_EINVAL;
  return lbm::critical_point(eos, a, b, R, omega, Tc, rho_c);
}

extern "C" int lbm_maxwell(int32_t eos, double a, double b, double R, double omega, double T,
                           double* rho_l, double* rho_g, double* p0) {
  double l, g, q;
  int st = lbm::maxwell(eos, a, b, R, omega, T, &l, &g, &q);
  if (st != LBM_OK) return st;
  if (rho_l) *rho_l = l;
  if (rho_g) *rho_g = g;
  if (p0) *p0 = q;
  return LBM_OK;
}

extern "C" int lbm_pressure(const lbm_params* p, double rho, double* out) {
  if (!p || !out) return LBM_EINVAL;
  lbm::EosConst k;
  int st = lbm::eos_constants(*p, &k);
  if (st != LBM_OK) return st;
  *out = lbm::pressure(k, rho);
  return LBM_OK;
}
