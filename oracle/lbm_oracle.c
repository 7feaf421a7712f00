/*
 * Plain FP64 CPU oracle of the pseudopotential lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or table with the GPU path.
 *
 * It is written to be checked against the paper by eye: one function per
 * equation, separate sweeps for moments, potential, force, collision and
 * streaming, no fusion and no reordering beyond what each equation states.
 * Build with -O2 -ffp-contract=off (no fused multiply-add contraction).
 *
 * Paper: Q. Li, K. H. Luo, X. J. Li, "Forcing scheme in pseudopotential
 * lattice Boltzmann model for multiphase flows" (arXiv:1204.4098).
 *   Sec. II, Eq. (1)   BGK evolution with forcing term
 *   Sec. II, Eq. (2)   D2Q9 equilibrium, weights 4/9, 1/9, 1/36
 *   Sec. II, Eq. (3)   interaction force, w(1)=1/3, w(2)=1/12
 *   Sec. II, Eq. (8)   potential from the equation of state
 *   Sec. III.A, Eqs. (9)-(10)  Shan-Chen velocity shift
 *   Sec. III.A, Eq. (11)       exact-difference method (EDM)
 *   Sec. III.C, Eq. (23)       Carnahan-Starling equation of state
 *   Sec. IV.B, Eq. (31)        improved forcing scheme (sigma = 0: Guo et al.)
 *   Sec. III.B, Eq. (12)       general form of a forcing term, used literally for
 *                              Ladd's scheme (Table I: equilibrium and forcing
 *                              velocity u, B_e = C_e = 1) and the modified EDM
 *                              (Sec. III.C: EDM with C_e = 1/tau)
 * Peng-Robinson is not written in the paper; its standard form is used
 * (alpha(T) = [1 + kappa (1 - sqrt(T/Tc))]^2,
 *  kappa = 0.37464 + 1.54226 w - 0.26992 w^2).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - c = delta_t = 1 and c_s^2 = 1/3 (D2Q9).
 *   - Direction numbering e0=(0,0), e1=(1,0), e2=(0,1), e3=(-1,0), e4=(0,-1),
 *     e5=(1,1), e6=(-1,1), e7=(-1,-1), e8=(1,-1).
 *   - In Eq. (31), upsilon = tau - 1/2 exactly.
 *   - The velocity in the equilibrium of the improved scheme is the actual
 *     fluid velocity v = u + F/(2 rho), as in Guo et al.'s scheme.
 *   - Modified EDM: only C_e changes; B_e = 1, the forcing velocity is EDM's
 *     v = u + F/(2 rho) and the equilibrium is taken at u, as in EDM.
 *   - Periodic boundaries in x and y.
 *   - Divergence: a non-finite or non-positive density, or a non-positive
 *     (or non-finite) argument of the square root in Eq. (8).
 *
 * Layout: populations f[a][y][x] (a = direction), x fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_EOS_CS = 0, OR_EOS_PR = 1 };
enum { OR_SCHEME_SC = 0, OR_SCHEME_EDM = 1, OR_SCHEME_IMPROVED = 2, OR_SCHEME_EDM_MODIFIED = 3,
       OR_SCHEME_LADD = 4 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_EPSI = -2, OR_EDIVERGED = -3, OR_ENOMEM = -5 };

typedef struct {
  int32_t nx, ny;
  double tau;       /* relaxation time, Eq. (1) */
  double G;         /* interaction strength, Eq. (3) */
  int32_t eos;      /* OR_EOS_CS or OR_EOS_PR */
  double a, b, R, T;
  double omega;     /* acentric factor, Peng-Robinson only */
  double Tc;        /* critical temperature, Peng-Robinson alpha(T) only */
  int32_t scheme;   /* OR_SCHEME_* */
  double sigma;     /* constant of the improved scheme, Eq. (31) */
  /* Collision: 0 = BGK (Eq. 1); 1 = multiple relaxation times (see or_mrt_collide),
   * with rates s_e (energy), s_eps (energy square) and s_q (energy flux); the
   * density, momentum and stress moments relax at 1/tau. */
  int32_t mrt;
  double s_e, s_eps, s_q;
} or_params;

static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WEQ[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

/* Interaction weights of Eq. (3): w(|e|^2 = 1) = 1/3, w(|e|^2 = 2) = 1/12. */
static double w_int(int a) {
  int e2 = EX[a] * EX[a] + EY[a] * EY[a];
  return e2 == 1 ? 1.0 / 3.0 : 1.0 / 12.0;
}

/* Equation of state p_EOS(rho). */
double or_p_eos(const or_params* p, double rho) {
  if (p->eos == OR_EOS_CS) {
    /* Eq. (23): p = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2, eta = b rho / 4 */
    double eta = p->b * rho / 4.0;
    double one_m = 1.0 - eta;
    return rho * p->R * p->T * (1.0 + eta + eta * eta - eta * eta * eta) /
               (one_m * one_m * one_m) -
           p->a * rho * rho;
  } else {
    /* Peng-Robinson: p = rho R T / (1 - b rho) - a alpha(T) rho^2 / (1 + 2 b rho - b^2 rho^2) */
    double kappa = 0.37464 + 1.54226 * p->omega - 0.26992 * p->omega * p->omega;
    double s = 1.0 + kappa * (1.0 - sqrt(p->T / p->Tc));
    double alpha = s * s;
    return rho * p->R * p->T / (1.0 - p->b * rho) -
           p->a * alpha * rho * rho / (1.0 + 2.0 * p->b * rho - p->b * p->b * rho * rho);
  }
}

/* Eq. (8) with c = 1: psi = sqrt(2 (p_EOS - rho c_s^2) / G).
 * Returns OR_EPSI when the argument is not a positive finite number. */
int or_psi(const or_params* p, double rho, double* psi) {
  double arg = 2.0 * (or_p_eos(p, rho) - rho * CS2) / p->G;
  if (!(arg > 0.0) || !isfinite(arg)) return OR_EPSI;
  *psi = sqrt(arg);
  return OR_OK;
}

/* Eq. (2): f_eq = w rho [1 + e.u/c_s^2 + uu:(ee - c_s^2 I)/(2 c_s^4)] */
void or_feq(double rho, double ux, double uy, double* feq) {
  for (int a = 0; a < 9; ++a) {
    double eu = EX[a] * ux + EY[a] * uy;
    double quad = (EX[a] * EX[a] - CS2) * ux * ux + 2.0 * EX[a] * EY[a] * ux * uy +
                  (EY[a] * EY[a] - CS2) * uy * uy;
    feq[a] = WEQ[a] * rho * (1.0 + eu / CS2 + quad / (2.0 * CS2 * CS2));
  }
}

/* Density and velocity u = sum f e / rho (Sec. III.A). */
static void node_moments(const double* f9, double* rho, double* ux, double* uy) {
  double r = 0.0, jx = 0.0, jy = 0.0;
  for (int a = 0; a < 9; ++a) r += f9[a];
  for (int a = 0; a < 9; ++a) {
    jx += f9[a] * EX[a];
    jy += f9[a] * EY[a];
  }
  *rho = r;
  *ux = jx / r;
  *uy = jy / r;
}

/* Eq. (3): F(x) = -G psi(x) sum_{a=1..8} w(|e_a|^2) psi(x + e_a) e_a, periodic. */
void or_interaction_force(const or_params* p, const double* psi, double* Fx, double* Fy) {
  int nx = p->nx, ny = p->ny;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double sx = 0.0, sy = 0.0;
      for (int a = 1; a < 9; ++a) {
        int xn = (x + EX[a] + nx) % nx, yn = (y + EY[a] + ny) % ny;
        double t = w_int(a) * psi[(size_t)yn * nx + xn];
        sx += t * EX[a];
        sy += t * EY[a];
      }
      double c = -p->G * psi[(size_t)y * nx + x];
      Fx[(size_t)y * nx + x] = c * sx;
      Fy[(size_t)y * nx + x] = c * sy;
    }
}

/* Forcing term F_a and the velocity used in the equilibrium, per scheme.
 *   SC (Eqs. 9-10):   u_eq = u + tau F / rho, F_a = 0
 *   EDM (Eq. 11):     u_eq = u, F_a = f_eq(rho, u + F/rho) - f_eq(rho, u)
 *   improved (Eq. 31): u_eq = v = u + F/(2 rho), v' = v + sigma F / ((tau - 1/2) psi^2),
 *                     F_a = w (1 - 1/(2 tau)) [(e - v')/c_s^2 + (e.v') e / c_s^4] . F
 * psi2 is psi^2 (used by the improved scheme only). */
/* Eq. (12): F_a = w_a [B.e_a / c_s^2 + C:(e_a e_a - c_s^2 I) / (2 c_s^4)], with
 * the vector B and the symmetric 2x2 tensor C (row-major Cxx, Cxy, Cyx, Cyy). */
void or_general_form(const double B[2], const double C[4], double* Fa) {
  for (int a = 0; a < 9; ++a) {
    double e[2] = {EX[a], EY[a]};
    double first = (B[0] * e[0] + B[1] * e[1]) / CS2;
    double second = 0.0;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) second += C[2 * i + j] * (e[i] * e[j] - (i == j ? CS2 : 0.0));
    Fa[a] = WEQ[a] * (first + second / (2.0 * CS2 * CS2));
  }
}

void or_forcing(const or_params* p, double rho, double ux, double uy, double Fx, double Fy,
                double psi2, double* ueqx, double* ueqy, double* Fa) {
  if (p->scheme == OR_SCHEME_EDM_MODIFIED || p->scheme == OR_SCHEME_LADD) {
    /* forcing velocity: EDM's v = u + F/(2 rho) (modified EDM) or u (Ladd) */
    double vx = ux, vy = uy, Ce = 1.0;
    if (p->scheme == OR_SCHEME_EDM_MODIFIED) {
      vx = ux + Fx / (2.0 * rho);
      vy = uy + Fy / (2.0 * rho);
      Ce = 1.0 / p->tau;
    }
    double B[2] = {Fx, Fy};  /* B_e = 1 */
    double C[4] = {Ce * (vx * Fx + Fx * vx), Ce * (vx * Fy + Fx * vy),
                   Ce * (vy * Fx + Fy * vx), Ce * (vy * Fy + Fy * vy)};
    *ueqx = ux;
    *ueqy = uy;
    or_general_form(B, C, Fa);
  } else if (p->scheme == OR_SCHEME_SC) {
    *ueqx = ux + p->tau * Fx / rho;
    *ueqy = uy + p->tau * Fy / rho;
    for (int a = 0; a < 9; ++a) Fa[a] = 0.0;
  } else if (p->scheme == OR_SCHEME_EDM) {
    double f1[9], f0[9];
    or_feq(rho, ux + Fx / rho, uy + Fy / rho, f1);
    or_feq(rho, ux, uy, f0);
    *ueqx = ux;
    *ueqy = uy;
    for (int a = 0; a < 9; ++a) Fa[a] = f1[a] - f0[a];
  } else {
    double vx = ux + Fx / (2.0 * rho), vy = uy + Fy / (2.0 * rho);
    double ups = p->tau - 0.5;
    double vpx = vx + p->sigma * Fx / (ups * psi2);
    double vpy = vy + p->sigma * Fy / (ups * psi2);
    *ueqx = vx;
    *ueqy = vy;
    for (int a = 0; a < 9; ++a) {
      double ev = EX[a] * vpx + EY[a] * vpy;
      double cx = (EX[a] - vpx) / CS2 + ev * EX[a] / (CS2 * CS2);
      double cy = (EY[a] - vpy) / CS2 + ev * EY[a] / (CS2 * CS2);
      Fa[a] = WEQ[a] * (1.0 - 1.0 / (2.0 * p->tau)) * (cx * Fx + cy * Fy);
    }
  }
}

/* ---- multiple-relaxation-time collision -------------------------------------
 * The paper states that the improved scheme extends to the MRT form of the
 * model (Sec. IV.B, last paragraph) without writing it out.  This is the D2Q9
 * MRT collision of Lallemand and Luo (Phys. Rev. E 61, 6546, 2000): moments
 * m = M f with the rows (for e of squared length e2)
 *   rho: 1;  e: -4 + 3 e2;  eps: 4 - (21/2) e2 + (9/2) e2^2;
 *   j_x: ex;  q_x: (-5 + 3 e2) ex;  j_y: ey;  q_y: (-5 + 3 e2) ey;
 *   p_xx: ex^2 - ey^2;  p_xy: ex ey,
 * relaxed one by one, m* = m - s_k (m - m_eq) + (1 - s_k/2) S_k, f* = M^-1 m*.
 * Reading of "readily extended": the equilibrium moments are M f_eq of Eq. (2)
 * at v = u + F/(2 rho), and the source S is M applied to Eq. (31)'s bracket
 * (the forcing term without its factor 1 - 1/(2 tau)), taken for moment k with
 * the modified velocity v'_k = v + sigma F / ((1/s_k - 1/2) psi^2), i.e. with
 * the moment's own relaxation time in place of tau.  With every rate equal to
 * 1/tau this is the BGK improved scheme exactly. */

/* Row k of the moment matrix at direction a (the polynomials above). */
double or_mrt_row(int k, int a) {
  double ex = EX[a], ey = EY[a], e2 = ex * ex + ey * ey;
  switch (k) {
    case 0: return 1.0;
    case 1: return -4.0 + 3.0 * e2;
    case 2: return 4.0 - 10.5 * e2 + 4.5 * e2 * e2;
    case 3: return ex;
    case 4: return (-5.0 + 3.0 * e2) * ex;
    case 5: return ey;
    case 6: return (-5.0 + 3.0 * e2) * ey;
    case 7: return ex * ex - ey * ey;
    default: return ex * ey;
  }
}

/* Relaxation rate of moment k. */
static double mrt_rate(const or_params* p, int k) {
  switch (k) {
    case 1: return p->s_e;
    case 2: return p->s_eps;
    case 4: case 6: return p->s_q;
    default: return 1.0 / p->tau;
  }
}

/* Eq. (31)'s bracket w [(e - v')/c_s^2 + (e.v') e/c_s^4] . F at every direction. */
static void improved_bracket(double vpx, double vpy, double Fx, double Fy, double* out) {
  for (int a = 0; a < 9; ++a) {
    double ev = EX[a] * vpx + EY[a] * vpy;
    double cx = (EX[a] - vpx) / CS2 + ev * EX[a] / (CS2 * CS2);
    double cy = (EY[a] - vpy) / CS2 + ev * EY[a] / (CS2 * CS2);
    out[a] = WEQ[a] * (cx * Fx + cy * Fy);
  }
}

/* One MRT collision of the populations f9 at a node (improved scheme). */
void or_mrt_collide(const or_params* p, const double* f9, double rho, double ux, double uy,
                    double Fx, double Fy, double psi2, double* out9) {
  double vx = ux + Fx / (2.0 * rho), vy = uy + Fy / (2.0 * rho);
  double feq[9], m[9], meq[9], ms[9], D[9];
  or_feq(rho, vx, vy, feq);
  for (int k = 0; k < 9; ++k) {
    double sk = mrt_rate(p, k);
    double vpx = vx + p->sigma * Fx / ((1.0 / sk - 0.5) * psi2);
    double vpy = vy + p->sigma * Fy / ((1.0 / sk - 0.5) * psi2);
    double br[9];
    improved_bracket(vpx, vpy, Fx, Fy, br);
    double S = 0.0;
    m[k] = meq[k] = D[k] = 0.0;
    for (int a = 0; a < 9; ++a) {
      double Mka = or_mrt_row(k, a);
      m[k] += Mka * f9[a];
      meq[k] += Mka * feq[a];
      S += Mka * br[a];
      D[k] += Mka * Mka;
    }
    ms[k] = m[k] - sk * (m[k] - meq[k]) + (1.0 - sk / 2.0) * S;
  }
  /* the rows are orthogonal, so M^-1 = M^T diag(1 / |row k|^2) */
  for (int a = 0; a < 9; ++a) {
    double v = 0.0;
    for (int k = 0; k < 9; ++k) v += or_mrt_row(k, a) * ms[k] / D[k];
    out9[a] = v;
  }
}

static int valid_params(const or_params* p) {
  if (p->nx < 3 || p->ny < 3) return 0;
  if (p->mrt) {
    if (p->scheme != OR_SCHEME_IMPROVED) return 0;
    if (!(p->s_e > 0.0 && p->s_e < 2.0) || !(p->s_eps > 0.0 && p->s_eps < 2.0) ||
        !(p->s_q > 0.0 && p->s_q < 2.0))
      return 0;
  }
  if (!(p->tau > 0.5)) return 0;
  if (p->eos != OR_EOS_CS && p->eos != OR_EOS_PR) return 0;
  if (p->scheme < OR_SCHEME_SC || p->scheme > OR_SCHEME_LADD) return 0;
  if (p->eos == OR_EOS_PR && !(p->Tc > 0.0)) return 0;
  if (!(p->G != 0.0)) return 0;
  return 1;
}

/* f = f_eq(rho0, u0) at every node (u0 may be NULL for rest). */
void or_init_equilibrium(int32_t nx, int32_t ny, const double* rho0, const double* ux0,
                         const double* uy0, double* f) {
  size_t n = (size_t)nx * ny;
  for (size_t i = 0; i < n; ++i) {
    double feq[9];
    or_feq(rho0[i], ux0 ? ux0[i] : 0.0, uy0 ? uy0[i] : 0.0, feq);
    for (int a = 0; a < 9; ++a) f[(size_t)a * n + i] = feq[a];
  }
}

/* Potential field psi(x) from the current populations; returns OR_EPSI and the
 * flat index of the first failing node when the state has left the EOS range. */
static int psi_field(const or_params* p, const double* f, double* rho, double* ux, double* uy,
                     double* psi, size_t* bad) {
  size_t n = (size_t)p->nx * p->ny;
  for (size_t i = 0; i < n; ++i) {
    double f9[9];
    for (int a = 0; a < 9; ++a) f9[a] = f[(size_t)a * n + i];
    node_moments(f9, &rho[i], &ux[i], &uy[i]);
    if (!(rho[i] > 0.0) || !isfinite(rho[i]) || or_psi(p, rho[i], &psi[i]) != OR_OK) {
      *bad = i;
      return OR_EPSI;
    }
  }
  return OR_OK;
}

/* Advance f by nsteps time steps of Eq. (1).  On divergence returns
 * OR_EDIVERGED, leaves f at the last finite state and sets *diverged_at to
 * the index of the step that could not be taken. */
int or_step(const or_params* p, double* f, int64_t nsteps, int64_t* diverged_at) {
  if (!valid_params(p)) return OR_EINVAL;
  size_t n = (size_t)p->nx * p->ny;
  double* rho = malloc(n * sizeof(double));
  double* ux = malloc(n * sizeof(double));
  double* uy = malloc(n * sizeof(double));
  double* psi = malloc(n * sizeof(double));
  double* Fx = malloc(n * sizeof(double));
  double* Fy = malloc(n * sizeof(double));
  double* fs = malloc(9 * n * sizeof(double));
  int status = OR_OK;
  if (!rho || !ux || !uy || !psi || !Fx || !Fy || !fs) {
    status = OR_ENOMEM;
    goto done;
  }
  if (diverged_at) *diverged_at = -1;
  for (int64_t t = 0; t < nsteps; ++t) {
    size_t bad = 0;
    /* sweep 1+2: moments and potential */
    if (psi_field(p, f, rho, ux, uy, psi, &bad) != OR_OK) {
      if (diverged_at) *diverged_at = t;
      status = OR_EDIVERGED;
      goto done;
    }
    /* sweep 3: interaction force, Eq. (3) */
    or_interaction_force(p, psi, Fx, Fy);
    /* sweep 4: collision, Eq. (1) right-hand side */
    for (size_t i = 0; i < n; ++i) {
      double f9[9], feq[9], Fa[9], ueqx, ueqy;
      for (int a = 0; a < 9; ++a) f9[a] = f[(size_t)a * n + i];
      if (p->mrt) {
        double out9[9];
        or_mrt_collide(p, f9, rho[i], ux[i], uy[i], Fx[i], Fy[i], psi[i] * psi[i], out9);
        for (int a = 0; a < 9; ++a) fs[(size_t)a * n + i] = out9[a];
        continue;
      }
      or_forcing(p, rho[i], ux[i], uy[i], Fx[i], Fy[i], psi[i] * psi[i], &ueqx, &ueqy, Fa);
      or_feq(rho[i], ueqx, ueqy, feq);
      for (int a = 0; a < 9; ++a)
        fs[(size_t)a * n + i] = f9[a] - (f9[a] - feq[a]) / p->tau + Fa[a];
    }
    /* sweep 5: streaming, f_a(x + e_a, t + 1) = f*_a(x, t), periodic */
    for (int a = 0; a < 9; ++a)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          int xd = (x + EX[a] + p->nx) % p->nx, yd = (y + EY[a] + p->ny) % p->ny;
          f[(size_t)a * n + (size_t)yd * p->nx + xd] = fs[(size_t)a * n + (size_t)y * p->nx + x];
        }
  }
done:
  free(rho); free(ux); free(uy); free(psi); free(Fx); free(Fy); free(fs);
  return status;
}

/* Macroscopic output: rho, actual velocity v = u + F/(2 rho) (Table I, all
 * schemes), pressure p = p_EOS(rho) (Eqs. 5 and 8).  Any pointer may be NULL. */
int or_moments(const or_params* p, const double* f, double* rho_out, double* vx_out,
               double* vy_out, double* p_out) {
  if (!valid_params(p)) return OR_EINVAL;
  size_t n = (size_t)p->nx * p->ny;
  double* rho = malloc(n * sizeof(double));
  double* ux = malloc(n * sizeof(double));
  double* uy = malloc(n * sizeof(double));
  double* psi = malloc(n * sizeof(double));
  double* Fx = malloc(n * sizeof(double));
  double* Fy = malloc(n * sizeof(double));
  int status = OR_OK;
  size_t bad;
  if (!rho || !ux || !uy || !psi || !Fx || !Fy) { status = OR_ENOMEM; goto done; }
  status = psi_field(p, f, rho, ux, uy, psi, &bad);
  if (status != OR_OK) goto done;
  or_interaction_force(p, psi, Fx, Fy);
  for (size_t i = 0; i < n; ++i) {
    if (rho_out) rho_out[i] = rho[i];
    if (vx_out) vx_out[i] = ux[i] + Fx[i] / (2.0 * rho[i]);
    if (vy_out) vy_out[i] = uy[i] + Fy[i] / (2.0 * rho[i]);
    if (p_out) p_out[i] = or_p_eos(p, rho[i]);
  }
done:
  free(rho); free(ux); free(uy); free(psi); free(Fx); free(Fy);
  return status;
}

/* Total mass: the plain double sum of rho over nodes (row-major order), and the
 * fixed-point sum of round-to-nearest-even(rho * 2^40) in 128-bit integer,
 * returned as (low 64 bits, high 64 bits).  rho = sum_a f_a in a = 0..8 order. */
void or_mass(int32_t nx, int32_t ny, const double* f, double* mass, int64_t* fixed_lo_hi) {
  size_t n = (size_t)nx * ny;
  double m = 0.0;
  __int128 acc = 0;
  for (size_t i = 0; i < n; ++i) {
    double r = 0.0;
    for (int a = 0; a < 9; ++a) r += f[(size_t)a * n + i];
    m += r;
    acc += (__int128)llrint(ldexp(r, 40));
  }
  if (mass) *mass = m;
  if (fixed_lo_hi) {
    fixed_lo_hi[0] = (int64_t)(uint64_t)(unsigned __int128)acc;
    fixed_lo_hi[1] = (int64_t)(acc >> 64);
  }
}
