/* Driver for the sanitizer build of the C oracle (test infrastructure): runs
 * every entry point of oracle/lbm_oracle.c on small odd lattice shapes, every
 * forcing scheme, both equations of state, the MRT collision and the
 * divergence path, so that AddressSanitizer and UndefinedBehaviorSanitizer see
 * every index computation.  Exit status 0 when every call returned as expected. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int32_t nx, ny;
  double tau, G;
  int32_t eos;
  double a, b, R, T, omega, Tc;
  int32_t scheme;
  double sigma;
  int32_t mrt;
  double s_e, s_eps, s_q;
} or_params;

int or_step(const or_params* p, double* f, int64_t nsteps, int64_t* diverged_at);
int or_moments(const or_params* p, const double* f, double* rho, double* vx, double* vy, double* pr);
void or_mass(int32_t nx, int32_t ny, const double* f, double* mass, int64_t* fixed);
void or_init_equilibrium(int32_t nx, int32_t ny, const double* rho0, const double* ux0,
                         const double* uy0, double* f);

static int run(int nx, int ny, int eos, int scheme, int mrt, double t) {
  or_params p = {nx, ny, 0.8, -1.0, eos, 1.0, 4.0, 1.0, 0.0, 0.344, 0.0, scheme, 0.1, mrt, 1.3, 1.1, 1.2};
  if (eos == 1) {
    p.a = 2.0 / 49.0;
    p.b = 2.0 / 21.0;
    p.Tc = 0.0729190;
  }
  p.T = t * (eos == 1 ? p.Tc : 0.0943287);
  size_t n = (size_t)nx * ny;
  double* rho0 = malloc(n * sizeof(double));
  double* f = malloc(9 * n * sizeof(double));
  double* out = malloc(4 * n * sizeof(double));
  double lo = eos == 1 ? 0.5 : 0.05, hi = eos == 1 ? 4.0 : 0.25;
  for (size_t i = 0; i < n; ++i) rho0[i] = lo + (hi - lo) * (double)((i * 7919) % 97) / 96.0;
  or_init_equilibrium(nx, ny, rho0, NULL, NULL, f);
  int64_t div = -1;
  int st = or_step(&p, f, 7, &div);
  if (st == 0) st = or_moments(&p, f, out, out + n, out + 2 * n, out + 3 * n);
  double m;
  int64_t fixed[2];
  or_mass(nx, ny, f, &m, fixed);
  free(rho0);
  free(f);
  free(out);
  return st;
}

int main(void) {
  const int shapes[][2] = {{3, 3}, {5, 4}, {4, 7}, {17, 9}};
  int bad = 0;
  for (int s = 0; s < 4; ++s)
    for (int eos = 0; eos < 2; ++eos)
      for (int scheme = 0; scheme < 5; ++scheme) {
        int st = run(shapes[s][0], shapes[s][1], eos, scheme, 0, 0.95);
        if (st != 0 && st != -3) bad++;
      }
  for (int s = 0; s < 4; ++s)
    if (run(shapes[s][0], shapes[s][1], 0, 2, 1, 0.95) != 0) bad++;
  /* divergence: a density beyond the equation of state's range */
  {
    or_params p = {8, 5, 1.0, -1.0, 0, 1.0, 4.0, 1.0, 0.08, 0.0, 0.0, 2, 0.0, 0, 1.0, 1.0, 1.0};
    double rho0[40], f[360];
    for (int i = 0; i < 40; ++i) rho0[i] = 0.1;
    or_init_equilibrium(8, 5, rho0, NULL, NULL, f);
    f[4 * 40 + 13] = NAN;
    int64_t div = -1;
    if (or_step(&p, f, 3, &div) != -3 || div != 0) bad++;
  }
  printf("oracle sanitizer driver: %d unexpected results\n", bad);
  return bad != 0;
}
