/*
 * lbm.h -- C ABI of the MI355X pseudopotential lattice Boltzmann library.
 *
 * The library advances the D2Q9 BGK lattice Boltzmann equation with the
 * Shan-Chen pseudopotential interaction force on AMD Instinct MI355X
 * (gfx950).  Method: Q. Li, K. H. Luo, X. J. Li, "Forcing scheme in
 * pseudopotential lattice Boltzmann model for multiphase flows",
 * arXiv:1204.4098.  One time step (lbm_step) is, at every node:
 *
 *   1. streaming (pull form of Eq. 1):   f_a(x, t) = f*_a(x - e_a, t - 1)
 *   2. moments:                          rho = sum f_a, u = sum f_a e_a / rho
 *   3. potential, Eq. (8) with c = 1:    psi = sqrt(2 (p_EOS(rho) - rho/3) / G)
 *      p_EOS is Carnahan-Starling (Eq. 23) or Peng-Robinson (standard form)
 *   4. interaction force, Eq. (3):       F = -G psi(x) sum_a w(|e_a|^2) psi(x + e_a) e_a,
 *                                        w(1) = 1/3, w(2) = 1/12
 *   5. forcing scheme and BGK collision, Eqs. (1), (2), (9)-(11), (31):
 *        Shan-Chen:  u_eq = u + tau F / rho, no forcing term
 *        EDM:        u_eq = u, F_a = f_eq(rho, u + F/rho) - f_eq(rho, u)
 *        improved:   u_eq = v = u + F / (2 rho),
 *                    F_a = w_a (1 - 1/(2 tau)) [(e_a - v')/c_s^2 + (e_a.v') e_a / c_s^4] . F,
 *                    v' = v + sigma F / ((tau - 1/2) psi^2)   (sigma = 0: Guo et al.)
 *        f*_a = f_a - (f_a - f_eq_a(rho, u_eq)) / tau + F_a
 *
 * Units: c = delta_t = 1, c_s^2 = 1/3.  Boundaries are periodic in x and y.
 * Directions: e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0) e4=(0,-1)
 *             e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1).
 *
 * Host arrays are row-major [y][x] (x fastest); population arrays are
 * [a][y][x].  Device memory is owned by the caller: the library never
 * allocates device memory; it works inside a caller-provided workspace whose
 * size the *_workspace_bytes functions report.  The workspace must stay
 * allocated, and must not be used by anyone else, until the matching
 * *_destroy call.  All work is enqueued on the caller's HIP stream
 * (hipStream_t passed as void*; NULL = the null stream).  A context must not
 * be used from two threads at once.
 *
 * Every function returns an int status: LBM_OK (0) or a negative error code
 * (lbm_strerror gives its text).  No C++ exception crosses this boundary.
 * A non-finite or non-positive density, or a non-positive argument of the
 * square root of Eq. (8), during a step marks the run as diverged: kernels
 * record the first such step on the device, and the next call that
 * synchronises (lbm_status, lbm_moments, lbm_mass, lbm_get_populations,
 * lbm_batch_coexistence, the lbm_batch_* accessors) reports it.  A diverged
 * run is frozen: every later launch copies its stored populations unchanged,
 * so the state read back is the one the diverging launch wrote, whatever the
 * number of steps requested after it.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;      /* one lattice; opaque, host-side */
typedef struct lbm_batch lbm_batch;  /* many independent lattices; opaque */

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* invalid argument or parameter */
  LBM_EPSI = -2,        /* initial density outside the EOS range: 2(p - rho/3)/G <= 0 */
  LBM_EDIVERGED = -3,   /* the run diverged (see lbm_status) */
  LBM_EHIP = -4,        /* a HIP runtime call failed */
  LBM_ENOSPACE = -5,    /* workspace smaller than *_workspace_bytes reports */
  LBM_ENOTSUP = -6      /* request not supported by this build */
};

enum { LBM_EOS_CS = 0, LBM_EOS_PR = 1 };
/* Forcing schemes.  SHANCHEN: velocity shift, Eqs. (9)-(10).  EDM: exact
 * difference method, Eq. (11).  IMPROVED: Eq. (31) (sigma = 0 is Guo et al.'s
 * scheme, Eq. (13)).  EDM_MODIFIED: EDM with C_e = 1/tau in the general form of
 * Eq. (12) (Sec. III.C).  LADD: Table I, equilibrium and forcing velocity u,
 * B_e = C_e = 1. */
enum {
  LBM_SCHEME_SHANCHEN = 0,
  LBM_SCHEME_EDM = 1,
  LBM_SCHEME_IMPROVED = 2,
  LBM_SCHEME_EDM_MODIFIED = 3,
  LBM_SCHEME_LADD = 4
};
/* Storage of populations: FP64, or deviations d_a = f_a - w_a rho_ref stored
 * in FP32 / FP16 with FP32 collision arithmetic (the EOS, psi and force stay
 * FP64), or FP32 deviations with FP64 collision arithmetic.  rho_ref = 0 stores
 * the populations themselves.  With FP32 storage and FP32 arithmetic, the mass
 * of each node and its momentum change (exactly F) are restored in FP64 after
 * the collision, so FP32 rounding is not a persistent mass or momentum source.
 * Device layout of every precision: element (a, y, x) at (9 y + a) pitch + x,
 * pitch = nx rounded up to a multiple of 64 (the nine direction rows of a
 * lattice row are consecutive). */
enum { LBM_PREC_F64 = 0, LBM_PREC_F32DEV = 1, LBM_PREC_F16DEV = 2, LBM_PREC_F32DEV_F64 = 3 };

typedef struct {
  int32_t nx, ny;    /* lattice size, periodic; 3 <= nx, ny; nx*ny < 2^31 */
  double tau;        /* relaxation time, Eq. (1); > 0.5 */
  double G;          /* interaction strength, Eq. (3); nonzero (the paper: -1) */
  int32_t eos;       /* LBM_EOS_* */
  double a, b, R;    /* EOS constants (C-S: a=1, b=4, R=1 in the paper) */
  double T;          /* absolute temperature (use lbm_critical_point for T/Tc) */
  double omega;      /* acentric factor (Peng-Robinson only) */
  int32_t scheme;    /* LBM_SCHEME_* */
  double sigma;      /* sigma of the improved scheme, Eq. (31); ignored otherwise */
  int32_t precision; /* LBM_PREC_* */
  double rho_ref;    /* reference density of deviation storage; NaN = mean of rho0 */
} lbm_params;

/* ---- thermodynamics (host only; no GPU needed) ---------------------------- */

/* Critical point of the EOS (dp/drho = d2p/drho2 = 0; Peng-Robinson with
 * alpha = 1).  Sec. III.C gives Tc ~ 0.094, rho_c = 0.13044 for C-S a=1, b=4, R=1. */
int lbm_critical_point(int32_t eos, double a, double b, double R, double omega,
                       double* Tc, double* rho_c);

/* Maxwell-construction coexistence densities, Eq. (7), at absolute T < Tc. */
int lbm_maxwell(int32_t eos, double a, double b, double R, double omega, double T,
                double* rho_l, double* rho_g, double* p0);

/* Equation of state p_EOS(rho) at the parameters' T (host, FP64). */
int lbm_pressure(const lbm_params* p, double rho, double* p_out);

/* ---- single lattice -------------------------------------------------------- */

/* Bytes of device workspace lbm_init needs for these parameters. */
int lbm_workspace_bytes(const lbm_params* p, size_t* bytes);

/* Create a context.  rho0 (host, ny*nx) is the initial density; ux0/uy0
 * (host, ny*nx, nullable = 0) the initial velocity; populations start at
 * f_eq(rho0, u0) (Eq. 2).  dev_workspace must be 256-byte aligned.
 * Returns LBM_EPSI when some rho0 lies outside the EOS range. */
int lbm_init(const lbm_params* p, const double* rho0, const double* ux0, const double* uy0,
             void* dev_workspace, size_t ws_bytes, void* hip_stream, lbm_ctx** out);

/* Enqueue n time steps on the context's stream (asynchronous). */
int lbm_step(lbm_ctx* c, int64_t n);

/* Synchronise; *step = steps taken so far, *diverged_at = first diverged step
 * or -1.  Returns LBM_EDIVERGED if the run diverged, else LBM_OK. */
int lbm_status(lbm_ctx* c, int64_t* step, int64_t* diverged_at);

/* Macroscopic fields of the current state into host arrays (ny*nx each,
 * nullable): rho, actual velocity v = u + F/(2 rho) (Table I), and pressure
 * p = p_EOS(rho) (Eqs. 5 and 8).  Synchronous. */
int lbm_moments(lbm_ctx* c, double* rho, double* vx, double* vy, double* p);

/* Same, into device arrays (ny*nx each, FP64, non-null), asynchronous. */
int lbm_moments_device(lbm_ctx* c, double* rho, double* vx, double* vy, double* p);

/* Flat-interface diagnostic for an interface whose normal is x (the slab
 * initial condition).  rho_bar (nx host doubles, non-null) = mean of rho over
 * y for each column.  p_n (nx host doubles, nullable) = normal pressure of
 * Eq. (25) with alpha = 0, beta = 3 (nearest-neighbour stencil, Sec. IV.A)
 * plus the improved scheme's 2 G^2 sigma psi'^2 (Eq. 35), from psi(rho_bar)
 * of Eq. (8) with central differences psi' = (psi[x+1] - psi[x-1])/2 and
 * psi'' = psi[x+1] - 2 psi[x] + psi[x-1], periodic.  At equilibrium p_n is
 * constant across the interface.  The paper fixes the scheme's contribution
 * to p_n only for the improved scheme (sigma = 0: Guo et al.), so p_n for
 * any other scheme returns LBM_ENOTSUP.  Uses the context's device scratch;
 * synchronous.  A column mean outside the range of Eq. (8) gives NaN there. */
int lbm_flat_profile(lbm_ctx* c, double* rho_bar, double* p_n);

/* Surface tension of the same flat interface (normal x), per interface of the
 * periodic slab: gamma = integral of (P_n - P_t) across it.  After Eq. (35) the
 * paper writes the pressure tensor as P_b delta_ij + kappa d_i psi d_j psi with
 * the improved scheme adding 2 G^2 sigma to kappa, so P_n - P_t = (kappa +
 * 2 G^2 sigma) psi'^2; kappa is not given there, and is taken as -G/6, the only
 * value for which a tensor of that form has the second-order expansion of
 * Eq. (3) on this stencil as its divergence.  gamma = (-G/6 + 2 G^2 sigma)
 * sum_x psi'(x)^2 / 2 over the column-mean profile, psi' as in
 * lbm_flat_profile.  The improved scheme only (LBM_ENOTSUP otherwise; with
 * the MRT collision the stress moments relax at 1/tau, so the same gamma
 * holds, while p_n of lbm_flat_profile is not supported there).  Synchronous. */
int lbm_surface_tension(lbm_ctx* c, double* gamma);

/* Total mass: fixed[0..1] = the 128-bit integer sum over nodes of
 * round-to-nearest-even(rho * 2^40) as (low, high) 64-bit words, with
 * rho = sum_a f_a summed in direction order 0..8 in FP64 (populations decoded
 * to FP64 first); *mass = FP64 sum.  Either pointer may be NULL.  Synchronous. */
int lbm_mass(lbm_ctx* c, int64_t* fixed, double* mass);

/* Allocation-free variant of lbm_mass, for callers that cannot allocate
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  It needs no context or workspace: dev_populations is a
 * population buffer in the library's storage layout (as lbm_device_buffers
 * returns it; nx, ny, precision and, for deviation storage, rho_ref as in the
 * lbm_params that made it; rho_ref is ignored for FP64).  Outputs as lbm_mass,
 * bit for bit.  The work-group partials live in a static device array of
 * 24,608 bytes that every GPU the library runs on holds until the process
 * ends; each call overwrites it entirely, so calls that overlap on one GPU
 * (two streams or threads at once) race.  Calls no allocator: two kernels,
 * one 24-byte copy to the host and a synchronisation of hip_stream (NULL = the
 * null stream).  nx, ny >= 3 and nx*ny <= LBM_NOALLOC_MAX_NODES, else
 * LBM_EINVAL (shape, precision, rho_ref) or LBM_ENOSPACE (too many nodes). */
#define LBM_NOALLOC_MAX_NODES 2147483647LL
int lbm_mass_noalloc(const void* dev_populations, int32_t nx, int32_t ny, int32_t precision,
                     double rho_ref, void* hip_stream, int64_t* fixed, double* mass);

/* Current populations f_a(x, t) decoded to FP64, host array 9*ny*nx [a][y][x]. */
int lbm_get_populations(lbm_ctx* c, double* f, int64_t* step);

/* Replace the state by f (host 9*ny*nx), re-encoded to the storage type with
 * round-to-nearest-even; sets the step counter and clears divergence. */
int lbm_set_populations(lbm_ctx* c, const double* f, int64_t step);

/* Bitwise checkpoint of the raw storage plus header (step, parameters). */
int lbm_state_bytes(lbm_ctx* c, size_t* bytes);
int lbm_save_state(lbm_ctx* c, void* host_buf, size_t bytes);
int lbm_load_state(lbm_ctx* c, const void* host_buf, size_t bytes);

/* Launch shape ("tile") of the step kernel.  A work-group of 64*waves threads
 * owns a strip of 64*waves columns (one column per thread) and marches up
 * `rows` rows; rows = 0 selects the balanced schedule, in which a grid sized
 * to the GPU's resident capacity splits all strip rows evenly.  `depth` (1 or
 * 2) is how many rows of loads are in flight while a row is collided.
 * `steps` (1, 2 or 3) is the number of time steps one launch advances: with
 * 2, the populations of the intermediate step stay on chip (registers and
 * LDS), so they cross HBM once per two steps; its strips are at most
 * 64*waves - 6 columns wide (the six extra columns are recomputed), spread
 * evenly over nx (FP64: strip edges on 64-byte boundaries), waves in {4, 8}.
 * With 3 (FP64 and FP32-storage-FP64-collision lattices of at least 5 x 5;
 * waves 4 or 8, depth 1; else LBM_ENOTSUP or LBM_EINVAL) they cross HBM once per
 * three steps, strips at most 64*waves - 10 columns wide.  A remainder of
 * lbm_step(n) smaller than `steps` runs as one launch of that many steps.
 * waves in {1, 2, 4, 8, 16}; rows in [0, 128].  lbm_tune times the candidates
 * on the current state without advancing it and keeps the fastest per lattice
 * step; the choice is cached per (nx, ny, precision, collision operator) for
 * the life of the process.  Every tile gives bitwise identical results. */
int lbm_tune(lbm_ctx* c, int32_t* waves, int32_t* rows, int32_t* depth, int32_t* steps);
int lbm_set_tile(lbm_ctx* c, int32_t waves, int32_t rows, int32_t depth, int32_t steps);
int lbm_get_tile(lbm_ctx* c, int32_t* waves, int32_t* rows, int32_t* depth, int32_t* steps);

/* Replay n steps through captured HIP graphs of k steps each (k even, >= 2;
 * 0 disables; a graph holds k / steps launches of the tile and one launch for
 * a remainder).  Needs a non-null stream.  The graphs of both buffer parities
 * are captured, instantiated and uploaded by this call (and again by
 * lbm_set_tile / lbm_tune when the tile changes), so lbm_step only replays
 * them; synchronous.  Results are bitwise identical to eager launches. */
int lbm_set_graph_steps(lbm_ctx* c, int32_t k);

/* Collision operator.  rates = NULL: BGK (Eq. 1, the default).  Otherwise the
 * D2Q9 multiple-relaxation-time collision of Lallemand and Luo (Phys. Rev. E
 * 61, 6546, 2000) with the improved forcing scheme carried into moment space,
 * the extension the paper names at the end of Sec. IV.B: rates[0..2] = s_e,
 * s_eps, s_q, the relaxation rates of the energy, energy-square and energy-flux
 * moments (each in (0, 2)); density, momentum and stress relax at 1/tau, so
 * the shear viscosity stays c_s^2 (tau - 1/2) and the bulk viscosity becomes
 * c_s^2 (1/s_e - 1/2).  Each moment gets Eq. (31)'s forcing moment with
 * v' = v + sigma F / ((1/s - 1/2) psi^2) for its own rate s, so rates all equal
 * to 1/tau give the BGK improved scheme.  Improved scheme only, FP64 or FP32
 * deviation storage (else LBM_ENOTSUP); every tile of the lattice's precision
 * (one, two and, for FP64, three steps per launch), bitwise equal to one
 * another.  Captured graphs are rebuilt. */
int lbm_set_mrt(lbm_ctx* c, const double* rates);

/* Number of graphs captured over the context's life (a tool can check that a
 * timed lbm_step call captured none). */
int lbm_graph_captures(lbm_ctx* c, int64_t* n);

/* Index-checked builds only (liblbm_hip_check.so, compiled with
 * LBM_CHECK_INDEX): the number of out-of-range global accesses or tile shapes
 * the kernels have met since the last call (the accesses were skipped), then
 * reset to 0.  Synchronises the device.  Release builds return LBM_ENOTSUP. */
int lbm_debug_index_faults(uint64_t* count);

/* The context's parameters, with rho_ref resolved (the mean initial density
 * when NaN was given; 0 for FP64 storage). */
int lbm_get_params(lbm_ctx* c, lbm_params* out);

/* Raw device addresses of the two population buffers (for timing and
 * profiling tools) and which one holds the current state (0 or 1). */
int lbm_device_buffers(lbm_ctx* c, void** buf0, void** buf1, int32_t* current);

int lbm_destroy(lbm_ctx* c);
const char* lbm_strerror(int status);

/* ---- batch of independent lattices ---------------------------------------- */

/* nruns parameter sets p[0..nruns-1] (one precision for all), initial
 * densities rho0[i] (host, p[i].ny * p[i].nx each).  One persistent kernel
 * launch advances every run by one step; a diverged run is frozen at the
 * step it diverged and the others continue unchanged. */
int lbm_batch_workspace_bytes(int32_t nruns, const lbm_params* p, size_t* bytes);
int lbm_batch_init(int32_t nruns, const lbm_params* p, const double* const* rho0,
                   void* dev_workspace, size_t ws_bytes, void* hip_stream, lbm_batch** out);
int lbm_batch_step(lbm_batch* b, int64_t n);

/* Coexistence densities of flat-interface runs (Sec. IV.B, slab of Eq. 36
 * with normal x): rho_l = mean density over y of the column at x = nx/2,
 * rho_g = the same at x = 0 (slab in [nx/4, 3nx/4)).  Reduced on the device in
 * FP64 by one launch over all runs (fixed summation order); only 2 doubles and
 * the status per run cross to the host.  rho_l = rho_g = NaN for a diverged
 * run.  status[i] = LBM_OK or LBM_EDIVERGED; diverged_at[i] = first diverged
 * step or -1.  Arrays of nruns (nullable).  Synchronous. */
int lbm_batch_coexistence(lbm_batch* b, double* rho_l, double* rho_g, int32_t* status,
                          int64_t* diverged_at);
/* Moments (as lbm_moments) and FP64 populations (as lbm_get_populations) of
 * one run; host arrays sized for that run.  Synchronous.  They return
 * LBM_EDIVERGED, with the outputs filled from the frozen state, when the run
 * has diverged. */
int lbm_batch_moments(lbm_batch* b, int32_t run, double* rho, double* vx, double* vy, double* p);
int lbm_batch_get_populations(lbm_batch* b, int32_t run, double* f);
/* Tiles of the batch work list (rows >= 4: items of that many rows, spread
 * over the grid; rows = 0: the balanced schedule, in which the rows of all
 * whole-run strips, concatenated, are split evenly over a grid sized to the
 * resident capacity), tuned over the whole batch like lbm_tune;
 * waves in {1, 2, 4, 8}; steps = 2 (waves 2, 4 or 8) runs two time steps per
 * launch as for a single lattice, with strips of at most 64*waves - 6
 * columns. */
int lbm_batch_tune(lbm_batch* b, int32_t* waves, int32_t* rows, int32_t* depth, int32_t* steps);
int lbm_batch_set_tile(lbm_batch* b, int32_t waves, int32_t rows, int32_t depth, int32_t steps);
int lbm_batch_get_tile(lbm_batch* b, int32_t* waves, int32_t* rows, int32_t* depth, int32_t* steps);
/* As lbm_set_graph_steps: captures the graphs of both parities now. */
int lbm_batch_set_graph_steps(lbm_batch* b, int32_t k);
/* The MRT collision of lbm_set_mrt for every run of the batch: rates[3*i ..
 * 3*i+2] = s_e, s_eps, s_q of run i (each in (0, 2), else LBM_EINVAL);
 * rates = NULL restores BGK.  Every run must use the improved scheme and the
 * batch FP64 or FP32 deviation storage (else LBM_ENOTSUP; nothing changes on
 * an error).  One- and two-step batch tiles; each run's results are bitwise
 * those of a single lattice with the same rates.  The descriptor table is
 * uploaded and captured graphs are rebuilt (synchronous). */
int lbm_batch_set_mrt(lbm_batch* b, const double* rates);
int lbm_batch_graph_captures(lbm_batch* b, int64_t* n);
/* Lattice updates per step summed over runs that are still active. */
int lbm_batch_nodes(lbm_batch* b, int64_t* nodes);
int lbm_batch_destroy(lbm_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
