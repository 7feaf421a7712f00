// Device code of the fused pseudopotential D2Q9 step for gfx950.
//
// One work-group owns a strip of SW = 64*NW lattice columns (one column per
// thread) and a chunk of L rows, and marches up the chunk one row at a time:
//
//   * streaming is done on load (pull): f_a(x, y) = f*_a(x - e_a, y - e_a)
//     from the source buffer (paper Eq. 1);
//   * each loaded row gives rho and, in FP64, psi^2 = 2 (p_EOS - rho/3)/G
//     (Eqs. 8, 23); psi goes to a 4-row ring in LDS;
//   * the row below is then complete (psi at y-1, y, y+1), so its force
//     (Eq. 3), forcing scheme (Eqs. 9-11, 31) and BGK collision (Eqs. 1, 2)
//     are computed and its 9 populations stored, coalesced, to the
//     destination buffer at the same node.
//
// psi of the two halo columns x0-1 and x0+SW is computed once per chunk in a
// prologue; the halo rows y0-1 and y0+L are recomputed by the chunks on
// either side.  Populations are read once from HBM and written once (the
// neighbour strips' halo reads hit L2), so a step moves 2*9*sizeof(storage)
// bytes per node.  The paper gives no kernel design; this layout is ours.
//
// k_step2 advances two time steps per launch with the intermediate
// populations kept on chip (registers and LDS), so the populations cross HBM
// once per two steps; k_batch_step runs many lattices from one work list.
// All kernels share the node arithmetic below and give identical bits.
//
// Storage: FP64 populations, or deviations s_a = f_a - w_a rho_ref in FP32 /
// FP16 with FP32 collision arithmetic, or FP32 deviations with FP64
// collision arithmetic.  The EOS, psi and force stencil are always evaluated
// in FP64.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "host_layout.hpp"  // Item

namespace lbm {

constexpr int LMAX = 128;  // largest chunk height (rows) k_step marches (halo arrays in LDS)

// Per-lattice constants, prepared on the host.
struct RunDev {
  int32_t nx, ny, pitch, eos;
  int64_t plane;            // elements between direction a and a+1 at one node
  int64_t rs;               // elements between row y and y+1 of one direction
  int64_t elems;            // elements of the lattice's population buffer
  int64_t off;              // element offset of this lattice in the population pool
  double RT, c1, c2;        // EOS constants (see EosConst)
  double two_over_G, mG;    // 2/G and -G
  double inv_tau;
  // forcing scheme in general form: u_eq = u + c_eq F/rho,
  // F_a = w_a [3 Be e.F + Ce (9 (e.vf)(e.F) - 3 vf.F)], vf = u + c_f F/rho + sig F/psi^2
  double c_eq, c_f, sig, Be, Ce;
  // products used by the collision: w0 Ce, w1 Ce, w2 Ce and 3 w1 Be, 3 w2 Be
  // (w0, w1, w2 = 4/9, 1/9, 1/36); om w0, om w1, om w2, 3 om w1, 3 om w2 and
  // 1 - om with om = 1/tau
  double wCe0, wCe1, wCe2, wBe3_1, wBe3_2;
  double om_w0, om_w1, om_w2, om_3w1, om_3w2, om1;
  double rho_ref;           // deviation reference density (0 for FP64 storage)
  int32_t run;
  int32_t mrt;              // 1: multiple-relaxation-time collision (collide_mrt)
  // MRT rates of the energy, energy-square and energy-flux moments (the others
  // relax at inv_tau) and the improved scheme's sigma / (1/s - 1/2) for the
  // energy and energy-square moments (sig above is the stress moments' value)
  double s_e, s_eps, s_q, sig_e, sig_eps;
};


// Balanced schedule of a batch: the concatenated rows of all strips, [0,
// total), are split evenly over the grid; block t (XCD-remapped) marches its
// share, one piece per item it overlaps (at most `cap` rows per piece), and
// calls piece(item, first row in the item, rows).
template <class Piece>
__device__ __forceinline__ void balanced_pieces(const Item* __restrict__ items, int nitems, int total,
                                                int t, int cap, Piece&& piece) {
  int64_t r = (int64_t)total * t / gridDim.x;
  const int64_t e = (int64_t)total * (t + 1) / gridDim.x;
  if (r >= e) return;
  int lo = 0, hi = nitems - 1;  // last item whose row0 <= r
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].row0 <= r) lo = mid;
    else hi = mid - 1;
  }
  int i = lo;
  while (r < e) {
    const Item it = items[i];
    const int y = (int)(r - it.row0);
    const int n = (int)min(min(e - r, (int64_t)(it.nrows - y)), (int64_t)cap);
    piece(it, y, n);
    r += n;
    if (y + n >= it.nrows) ++i;
    __syncthreads();  // LDS is reused by the next piece
  }
}

// Storage traits: E = element type in memory, R = collision arithmetic type;
// round(v) = the value a store followed by a load would give.  Cache policy
// per type, measured on the 4096 x 4096 droplet workload with the two-step
// kernel: FP64 populations stream with non-temporal loads and stores (plain
// stores cost 10 %); FP32 deviations use plain loads and stores (9 % faster
// than non-temporal); FP32 storage with FP64 arithmetic and FP16 deviations
// show no difference.
struct f32s_f64a {};  // FP32 deviation storage with FP64 collision arithmetic
template <typename S> struct Store;
// E: stored type; R: collision arithmetic; P: type of psi, of the force and of
// the density they are evaluated at (FP64 for every storage type: the EOS and
// psi stay FP64 in the reduced-precision forms).  kConserve: after the FP32
// collision, restore the node's mass and momentum change exactly (see
// conserve()).
template <> struct Store<double> {
  using E = double;
  using R = double;
  using P = double;
  static constexpr bool kConserve = false;
  static __device__ __forceinline__ R ld(const E* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ void st(E* p, R v) { __builtin_nontemporal_store(v, p); }
  static __device__ __forceinline__ R round(R v) { return v; }
};
template <> struct Store<float> {
  using E = float;
  using R = float;
  using P = double;
  static constexpr bool kConserve = true;
  static __device__ __forceinline__ R ld(const E* p) { return *p; }
  static __device__ __forceinline__ void st(E* p, R v) { *p = v; }
  static __device__ __forceinline__ R round(R v) { return v; }
};
template <> struct Store<f32s_f64a> {
  using E = float;
  using R = double;
  using P = double;
  static constexpr bool kConserve = false;
  static __device__ __forceinline__ R ld(const E* p) { return double(__builtin_nontemporal_load(p)); }
  static __device__ __forceinline__ void st(E* p, R v) { __builtin_nontemporal_store(float(v), p); }
  static __device__ __forceinline__ R round(R v) { return double(float(v)); }
};
template <> struct Store<__half> {
  using E = __half;
  using R = float;
  using P = double;
  static constexpr bool kConserve = false;
  // The narrowing to FP16 takes its operand through an empty asm statement:
  // the backend otherwise folds it into the FMA that produced the operand (a
  // mixed-precision FMA with an FP16 result, one rounding instead of two) at
  // some call sites only, whatever the contraction setting, which breaks the
  // bitwise identity of the one- and two-step kernels.
  static __device__ __forceinline__ _Float16 narrow(R v) {
    asm volatile("" : "+v"(v));
    return static_cast<_Float16>(v);
  }
  static __device__ __forceinline__ R ld(const E* p) { return __half2float(*p); }
  static __device__ __forceinline__ void st(E* p, R v) {
    __half_raw h;
    h.data = narrow(v);
    *p = h;
  }
  static __device__ __forceinline__ R round(R v) { return static_cast<float>(narrow(v)); }
};

// Index-checked build (LBM_CHECK_INDEX): every global load and store of the
// step, copy and mass kernels checks its element offset against the lattice's
// buffer, and every tile its shape against the kernel's limits; a violation
// is counted in g_index_faults (read by lbm_debug_index_faults) and the access
// is skipped.  Release builds compile none of this.
#ifdef LBM_CHECK_INDEX
__device__ unsigned long long g_index_faults;
__device__ __forceinline__ bool index_ok(int64_t off, int64_t n) {
  if (off >= 0 && off < n) return true;
  atomicAdd(&g_index_faults, 1ull);
  return false;
}
#define LBM_TILE_CHECK(cond)                            \
  do {                                                  \
    if (!(cond)) atomicAdd(&g_index_faults, 1ull);      \
  } while (0)
#else
__device__ __forceinline__ bool index_ok(int64_t, int64_t) { return true; }
#define LBM_TILE_CHECK(cond) \
  do {                       \
  } while (0)
#endif

// D2Q9 directions e0=(0,0), e1=(1,0), e2=(0,1), e3=(-1,0), e4=(0,-1), e5=(1,1),
// e6=(-1,1), e7=(-1,-1), e8=(1,-1) (pull9, collide and the moments use this
// numbering); weights of Eq. (2):
__device__ constexpr double kW[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Reciprocals: the hardware estimate refined by two Newton steps (FP64, about
// 1 ulp), or the single-precision estimate (FP32 arithmetic paths, 1 ulp).
// Arguments are positive normal numbers (or non-finite in a diverged state).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Column indices of one thread: its own column and the periodic neighbours.
struct Cols {
  unsigned x, xm, xp;
};
__device__ __forceinline__ Cols cols_of(int x, int nx) {
  return Cols{(unsigned)x, (unsigned)(x == 0 ? nx - 1 : x - 1), (unsigned)(x == nx - 1 ? 0 : x + 1)};
}

// Pull the 9 populations of node (c.x, y) from the post-collision field.  Row
// and plane offsets are uniform across the block (scalar registers); only the
// 32-bit column index varies per lane.
template <typename S>
__device__ __forceinline__ void pull9(const typename Store<S>::E* __restrict__ src, const RunDev& d,
                                      const Cols& c, int y, typename Store<S>::R (&f)[9]) {
  const int ym = y == 0 ? d.ny - 1 : y - 1;
  const int yp = y == d.ny - 1 ? 0 : y + 1;
  const int64_t P = d.plane;
  using T = Store<S>;
  const typename T::E* r0 = src + (int64_t)y * d.rs;
  const typename T::E* rm = src + (int64_t)ym * d.rs;
  const typename T::E* rp = src + (int64_t)yp * d.rs;
#ifdef LBM_CHECK_INDEX
  const typename T::E* p9[9] = {r0 + c.x,         r0 + P + c.xm,     rm + 2 * P + c.x,
                                r0 + 3 * P + c.xp, rp + 4 * P + c.x,  rm + 5 * P + c.xm,
                                rm + 6 * P + c.xp, rp + 7 * P + c.xp, rp + 8 * P + c.xm};
  for (int a = 0; a < 9; ++a) f[a] = index_ok(p9[a] - src, d.elems) ? T::ld(p9[a]) : typename T::R(0);
#else
  f[0] = T::ld(r0 + c.x);
  f[1] = T::ld(r0 + P + c.xm);
  f[2] = T::ld(rm + 2 * P + c.x);
  f[3] = T::ld(r0 + 3 * P + c.xp);
  f[4] = T::ld(rp + 4 * P + c.x);
  f[5] = T::ld(rm + 5 * P + c.xm);
  f[6] = T::ld(rm + 6 * P + c.xp);
  f[7] = T::ld(rp + 7 * P + c.xp);
  f[8] = T::ld(rp + 8 * P + c.xm);
#endif
}

// The arithmetic of one node update below is written with explicit fma()
// where a fused multiply-add is wanted and compiled with contraction off, so
// every kernel that inlines it performs the same operations and rounds the
// same way (the single-step, two-step and batched kernels give identical bits).

// Density deviation sum_a s_a in the arithmetic type (pairwise order).
template <typename R>
__device__ __forceinline__ R sum9(const R (&s)[9]) {
#pragma clang fp contract(off)
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])) + s[8];
}

// psi^2 = 2 (p_EOS(rho) - rho/3) / G (Eq. 8 with Eq. 23 or Peng-Robinson), in
// the type P.
template <typename P>
__device__ __forceinline__ P psi2_of(P rho, const RunDev& d) {
#pragma clang fp contract(off)
  P p;
  const P one = P(1);
  if (d.eos == 0) {
    // rho RT (1 + e + e^2 - e^3)/(1 - e)^3 - c2 rho^2, e = b rho / 4
    const P e = P(d.c1) * rho, m = one - e;
    const P poly = fma(e, fma(e, one - e, one), one);
    p = fma((rho * P(d.RT)) * poly, rcp((m * m) * m), -((P(d.c2) * rho) * rho));
  } else {
    // rho RT/(1 - b) - c2 rho^2/(1 + b(2 - b)) over one common reciprocal
    const P b = P(d.c1) * rho;
    const P q1 = one - b, q2 = fma(b, P(2) - b, one);
    p = fma(rho * P(d.RT), q2, -(((P(d.c2) * rho) * rho) * q1)) * rcp(q1 * q2);
  }
  return fma(rho, P(-1.0 / 3.0), p) * P(d.two_over_G);
}

// psi from psi^2 (the correctly rounded FP64 square root).
__device__ __forceinline__ double psi_root(double x) { return sqrt(x); }

__device__ __forceinline__ double pressure_of(double rho, const RunDev& d) {
  if (d.eos == 0) {
    const double e = d.c1 * rho, m = 1.0 - e;
    return rho * d.RT * (1.0 + e * (1.0 + e * (1.0 - e))) / (m * m * m) - d.c2 * rho * rho;
  }
  return rho * d.RT / (1.0 - d.c1 * rho) - d.c2 * rho * rho / (1.0 + d.c1 * rho * (2.0 - d.c1 * rho));
}

// Interaction force of Eq. (3) from the 3x3 psi neighbourhood (row-major:
// s = y-1, c = y, n = y+1; index 0 = x-1, 1 = x, 2 = x+1), w(1)=1/3, w(2)=1/12.
template <typename P>
__device__ __forceinline__ void force3x3(const P* rs, const P* rc, const P* rn, int i, P mG, P& Fx,
                                         P& Fy) {
#pragma clang fp contract(off)
  const P w1 = P(1.0 / 3.0), w2 = P(1.0 / 12.0);
  const P dNE = rn[i + 1] - rs[i - 1];   // psi(x+e5) - psi(x-e5)
  const P dNW = rn[i - 1] - rs[i + 1];   // psi(x+e6) - psi(x-e6)
  const P Sx = fma(w1, rc[i + 1] - rc[i - 1], w2 * (dNE - dNW));
  const P Sy = fma(w1, rn[i] - rs[i], w2 * (dNE + dNW));
  const P c = mG * rc[i];
  Fx = c * Sx;
  Fy = c * Sy;
}

// BGK collision with the forcing scheme in general form (see RunDev).
//
// For direction a the update is s_a + om (seq_a - s_a) + F_a with
//   seq_a = w (drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u))        (Eq. 2, deviation form)
//   F_a   = w [3 B_e e.F + C_e (9 (e.v)(e.F) - 3 v.F)]             (Eq. 12)
// The opposite direction (e -> -e) flips the odd terms only, so each pair is
// evaluated once: om seq = om w X +- 3 om w rho e.u with X = drho + rho (4.5
// (e.u)^2 - 1.5 u.u), F_a = C +- D, and s' = (1 - om) s + (P +- Q) with
// P = om w X + C, Q = 3 om w rho e.u + D (the products of om and the weights
// are per-lattice constants).
template <typename R>
__device__ __forceinline__ void collide_pair(R& sa, R& sb, R eu, R eF, R ev, R omw, R omwr3, R wCe,
                                             R wBe3, R rho, R drho, R usq, R vF3, R om1) {
#pragma clang fp contract(off)
  const R X = fma(rho, fma(R(4.5) * eu, eu, -usq), drho);
  const R C = wCe * fma(R(9) * ev, eF, -vF3);
  const R P = fma(omw, X, C);
  const R Q = fma(omwr3, eu, wBe3 * eF);
  sa = fma(om1, sa, P + Q);
  sb = fma(om1, sb, P - Q);
}

template <typename R>
__device__ __forceinline__ void collide(R (&s)[9], R drho, R rho, R jx, R jy, R Fx, R Fy,
                                        R inv_psi2, const RunDev& d) {
#pragma clang fp contract(off)
  const R inv_rho = rcp(rho);
  const R ux = jx * inv_rho, uy = jy * inv_rho;
  const R Fr_x = Fx * inv_rho, Fr_y = Fy * inv_rho;
  const R wx = fma(R(d.c_eq), Fr_x, ux), wy = fma(R(d.c_eq), Fr_y, uy);
  const R sg = R(d.sig) * inv_psi2;
  const R vx = fma(sg, Fx, fma(R(d.c_f), Fr_x, ux)), vy = fma(sg, Fy, fma(R(d.c_f), Fr_y, uy));
  const R om1 = R(d.om1);
  const R usq = R(1.5) * fma(wx, wx, wy * wy);
  const R vF3 = R(3) * fma(vx, Fx, vy * Fy);
  const R omw1 = R(d.om_w1), omw2 = R(d.om_w2);
  const R omwr3_1 = R(d.om_3w1) * rho, omwr3_2 = R(d.om_3w2) * rho;
  const R wCe1 = R(d.wCe1), wBe3_1 = R(d.wBe3_1), wCe2 = R(d.wCe2), wBe3_2 = R(d.wBe3_2);
  // rest direction: e = 0
  s[0] = fma(om1, s[0], fma(R(d.om_w0), fma(rho, -usq, drho), R(d.wCe0) * -vF3));
  // axis pairs (e1, e3 = -e1), (e2, e4 = -e2)
  collide_pair(s[1], s[3], wx, Fx, vx, omw1, omwr3_1, wCe1, wBe3_1, rho, drho, usq, vF3, om1);
  collide_pair(s[2], s[4], wy, Fy, vy, omw1, omwr3_1, wCe1, wBe3_1, rho, drho, usq, vF3, om1);
  // diagonal pairs (e5 = (1,1), e7 = -e5), (e6 = (-1,1), e8 = -e6)
  collide_pair(s[5], s[7], wx + wy, Fx + Fy, vx + vy, omw2, omwr3_2, wCe2, wBe3_2, rho, drho, usq,
               vF3, om1);
  collide_pair(s[6], s[8], wy - wx, Fy - Fx, vy - vx, omw2, omwr3_2, wCe2, wBe3_2, rho, drho, usq,
               vF3, om1);
}

// Multiple-relaxation-time collision with the improved forcing scheme, on the
// D2Q9 moments of Lallemand and Luo (2000): rho, e, eps, j_x, q_x, j_y, q_y,
// p_xx, p_xy (squared row norms 9, 36, 36, 6, 12, 6, 12, 4, 4).  Each moment
// relaxes at its own rate toward the moments of the Eq. (2) equilibrium at
// v = u + F/(2 rho),
//   e_eq = rho(-2 + 3|v|^2), eps_eq = rho(1 - 3|v|^2), q_eq = -rho v,
//   p_xx,eq = rho(vx^2 - vy^2), p_xy,eq = rho vx vy,
// and receives (1 - s/2) times the moment of Eq. (31)'s bracket taken with the
// moment's own modified velocity v' = v + sigma F / ((1/s - 1/2) psi^2):
//   S_e = 6 v'.F, S_eps = -6 v'.F, S_q = -F, S_xx = 2(v'x Fx - v'y Fy), S_xy = v'x Fy + v'y Fx.
// The conserved moments need no relaxation: rho' = rho and j' = j + F (any
// momentum rate gives this).  In deviation storage the moments of w rho_ref,
// rho_ref (1, -2, 1, 0, ...), are taken out of rho, e and eps.  With every rate
// 1/tau this is the BGK update of collide() up to rounding.
template <typename R>
__device__ __forceinline__ void collide_mrt(R (&s)[9], R drho, R rho, R jx, R jy, R Fx, R Fy,
                                            R inv_psi2, const RunDev& d) {
#pragma clang fp contract(off)
  const R inv_rho = rcp(rho);
  const R vx = fma(R(0.5) * Fx, inv_rho, jx * inv_rho), vy = fma(R(0.5) * Fy, inv_rho, jy * inv_rho);
  const R v2 = fma(vx, vx, vy * vy), vF = fma(vx, Fx, vy * Fy);
  const R FF = fma(Fx, Fx, Fy * Fy) * inv_psi2;
  // moments of the stored values
  const R ax = s[1] + s[3], ay = s[2] + s[4], a = ax + ay;
  const R dg = (s[5] + s[7]) + (s[6] + s[8]);
  const R e = fma(R(-4), s[0], fma(R(2), dg, -a));
  const R ep = fma(R(4), s[0], fma(R(-2), a, dg));
  const R qx = fma(R(-2), s[1] - s[3], (s[5] - s[7]) + (s[8] - s[6]));
  const R qy = fma(R(-2), s[2] - s[4], (s[5] - s[7]) + (s[6] - s[8]));
  const R pxx = ax - ay;
  const R pxy = (s[5] + s[7]) - (s[6] + s[8]);
  // equilibria (deviation form: rho_ref (1, -2, 1) removed from rho, e, eps)
  const R r3v2 = R(3) * rho * v2;
  const R e_eq = fma(R(-2), drho, r3v2), ep_eq = drho - r3v2;
  const R se = R(d.s_e), sp = R(d.s_eps), sq = R(d.s_q), sn = R(d.inv_tau);
  const R S_e = R(6) * fma(R(d.sig_e), FF, vF);
  const R S_ep = R(-6) * fma(R(d.sig_eps), FF, vF);
  const R sgn = R(2) * R(d.sig) * inv_psi2;
  const R S_xx = fma(R(2), fma(vx, Fx, -(vy * Fy)), sgn * fma(Fx, Fx, -(Fy * Fy)));
  const R S_xy = fma(vx, Fy, vy * Fx) + sgn * (Fx * Fy);
  // m' = m - s (m - m_eq) + (1 - s/2) S
  const R e1 = fma(-se, e - e_eq, e) + (R(1) - R(0.5) * se) * S_e;
  const R ep1 = fma(-sp, ep - ep_eq, ep) + (R(1) - R(0.5) * sp) * S_ep;
  const R hq = R(1) - R(0.5) * sq;
  const R qx1 = fma(-sq, fma(rho, vx, qx), qx) - hq * Fx;
  const R qy1 = fma(-sq, fma(rho, vy, qy), qy) - hq * Fy;
  const R hn = R(1) - R(0.5) * sn;
  const R pxx1 = fma(-sn, pxx - rho * fma(vx, vx, -(vy * vy)), pxx) + hn * S_xx;
  const R pxy1 = fma(-sn, pxy - (rho * vx) * vy, pxy) + hn * S_xy;
  const R jx1 = jx + Fx, jy1 = jy + Fy;
  // back to populations: f = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m'
  const R r0 = drho * R(1.0 / 9.0), r1 = e1 * R(1.0 / 36.0), r2 = ep1 * R(1.0 / 36.0);
  const R r3 = jx1 * R(1.0 / 6.0), r4 = qx1 * R(1.0 / 12.0), r5 = jy1 * R(1.0 / 6.0),
          r6 = qy1 * R(1.0 / 12.0), r7 = pxx1 * R(0.25), r8 = pxy1 * R(0.25);
  s[0] = fma(R(4), r2 - r1, r0);
  const R A = fma(R(-2), r2, r0 - r1), Dg = fma(R(2), r1, r0 + r2);
  const R ox = fma(R(-2), r4, r3), oy = fma(R(-2), r6, r5);
  s[1] = (A + ox) + r7;
  s[3] = (A - ox) + r7;
  s[2] = (A + oy) - r7;
  s[4] = (A - oy) - r7;
  const R X = r3 + r4, Y = r5 + r6;
  s[5] = (Dg + (X + Y)) + r8;
  s[6] = (Dg - (X - Y)) - r8;
  s[7] = (Dg - (X + Y)) + r8;
  s[8] = (Dg + (X - Y)) - r8;
}

// The collision of a node: BGK (collide) or MRT (collide_mrt).
template <bool MRT, typename R>
__device__ __forceinline__ void collide_any(R (&s)[9], R drho, R rho, R jx, R jy, R Fx, R Fy,
                                            R inv_psi2, const RunDev& d) {
  if constexpr (MRT)
    collide_mrt<R>(s, drho, rho, jx, jy, Fx, Fy, inv_psi2, d);
  else
    collide<R>(s, drho, rho, jx, jy, Fx, Fy, inv_psi2, d);
}

template <typename R>
__device__ __forceinline__ R mom_x(const R (&s)[9]) {
  return ((s[1] - s[3]) + (s[5] - s[7])) + (s[8] - s[6]);
}
template <typename R>
__device__ __forceinline__ R mom_y(const R (&s)[9]) {
  return ((s[2] - s[4]) + (s[5] - s[7])) + (s[6] - s[8]);
}

// Momentum of FP32 values (as FP64 t) summed in FP64: exact unless the
// values span more than 29 binary orders of magnitude, and then wrong only by
// an FP64 rounding of the largest, far below an FP32 rounding; being exact,
// the sums do not depend on their order.
__device__ __forceinline__ void exact_momentum(const double (&t)[9], double& jx, double& jy) {
#pragma clang fp contract(off)
  const double u = t[5] - t[7], v = t[8] - t[6];
  jx = ((t[1] - t[3]) + u) + v;
  jy = ((t[2] - t[4]) + u) - v;
}
// Mass and momentum of nine FP32 values, exactly (as exact_momentum).
__device__ __forceinline__ void exact_moments(const float (&s)[9], double& m, double& jx, double& jy) {
#pragma clang fp contract(off)
  double t[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) t[a] = double(s[a]);
  m = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7])) + t[8];
  exact_momentum(t, jx, jy);
}

// The collision conserves mass and changes the momentum by exactly F (every
// forcing scheme here, BGK or MRT).  In FP32 arithmetic each updated
// population carries its own rounding, and at a steady state the same
// roundings recur every step: a persistent mass and momentum source at every
// node that the slow bulk dynamics integrate into visibly shifted coexistence
// densities.  conserve() puts the momentum change of the new populations back
// to exactly F (half the x defect on e1 and -e1, likewise y on e2, -e4) and the
// mass back to exactly the old mass on the rest population, computed in FP64;
// what remains is one FP32 rounding of five values.
__device__ __forceinline__ void conserve(float (&s)[9], double m_t, double jx_t, double jy_t) {
#pragma clang fp contract(off)
  double t[9], jx, jy;
  t[0] = 0.0;  // the rest population carries no momentum
#pragma unroll
  for (int a = 1; a < 9; ++a) t[a] = double(s[a]);
  exact_momentum(t, jx, jy);
  const double dx = 0.5 * (jx_t - jx), dy = 0.5 * (jy_t - jy);
  s[1] = float(t[1] + dx);
  s[3] = float(t[3] - dx);
  s[2] = float(t[2] + dy);
  s[4] = float(t[4] - dy);
#pragma unroll
  for (int a = 1; a < 5; ++a) t[a] = double(s[a]);
  const double rest = ((t[1] + t[2]) + (t[3] + t[4])) + ((t[5] + t[6]) + (t[7] + t[8]));
  s[0] = float(m_t - rest);
}

// One node update: collision (BGK or MRT) of the pulled values s with the
// force (Fx, Fy) (FP64), then, for FP32 storage, conserve().
template <typename S, bool MRT>
__device__ __forceinline__ void update_node(typename Store<S>::R (&s)[9],
                                            typename Store<S>::R drho, typename Store<S>::P rho,
                                            typename Store<S>::P Fx, typename Store<S>::P Fy,
                                            typename Store<S>::R ip2, const RunDev& d) {
  using R = typename Store<S>::R;
  if constexpr (Store<S>::kConserve) {
    double m0, jx0, jy0;
    exact_moments(s, m0, jx0, jy0);
    collide_any<MRT, R>(s, drho, R(rho), mom_x(s), mom_y(s), R(Fx), R(Fy), ip2, d);
    conserve(s, m0, jx0 + double(Fx), jy0 + double(Fy));
  } else {
    collide_any<MRT, R>(s, drho, R(rho), mom_x(s), mom_y(s), R(Fx), R(Fy), ip2, d);
  }
}

// One tile: columns [x0, x0+ncols), rows [y0, y0+nrows), nrows <= LMAX.
// All threads of the block call it (barriers inside); ring is [4][SW+2],
// haloL/haloR [LMAX+2].  PF is the number of rows whose loads are in flight
// while a row is collided: with PF = 2 the loads of row y+2 are issued before
// the psi of row y+1 is evaluated and row y is collided.
template <typename S, int NW, int PF, bool MRT = false>
__device__ __forceinline__ void tile_step(const typename Store<S>::E* __restrict__ src,
                                          typename Store<S>::E* __restrict__ dst,
                                          const RunDev& d, int x0, int y0, int ncols, int nrows,
                                          unsigned long long step,
                                          unsigned long long* __restrict__ flag,
                                          typename Store<S>::P (*ring)[64 * NW + 2],
                                          typename Store<S>::P* haloL, typename Store<S>::P* haloR) {
  using T = Store<S>;
  using R = typename T::R;
  using P = typename T::P;
  constexpr int SW = 64 * NW;
  const int tid = threadIdx.x;
  LBM_TILE_CHECK(ncols >= 1 && ncols <= SW && nrows >= 1 && nrows <= LMAX && x0 >= 0 &&
                 x0 + ncols <= d.nx && y0 >= 0 && y0 + nrows <= d.ny);
  const bool act = tid < ncols;
  const int x = x0 + tid;
  const Cols cx = cols_of(act ? x : x0, d.nx);
  const int xl = x0 == 0 ? d.nx - 1 : x0 - 1;
  const int xr = x0 + ncols >= d.nx ? 0 : x0 + ncols;
  const P rref = P(d.rho_ref);
  bool bad = false;

  // preload rows y0-1 (ring slot 0) and y0 (slot 1); with PF = 2 also issue row
  // y0+1.  The loads are issued before the halo prologue so that both wait on
  // memory together.
  R fc[9], fn[9], fp[9];
  if (act) {
    pull9<S>(src, d, cx, y0 == 0 ? d.ny - 1 : y0 - 1, fp);
    pull9<S>(src, d, cx, y0, fc);
    if (PF == 2) pull9<S>(src, d, cx, y0 + 1 == d.ny ? 0 : y0 + 1, fn);
  }

  // prologue: psi of the two halo columns for rows y0-1 .. y0+nrows
  for (int i = tid; i < 2 * (nrows + 2); i += SW) {
    const int k = i >> 1;
    int yy = y0 - 1 + k;
    yy = yy < 0 ? yy + d.ny : (yy >= d.ny ? yy - d.ny : yy);
    R f[9];
    pull9<S>(src, d, cols_of((i & 1) ? xr : xl, d.nx), yy, f);
    const P rho = rref + P(sum9(f));
    ((i & 1) ? haloR : haloL)[k] = psi_root(psi2_of(rho, d));
  }

  P psi2c = P(0);
  if (act) {
    ring[0][tid + 1] = psi_root(psi2_of(rref + P(sum9(fp)), d));
    psi2c = psi2_of(rref + P(sum9(fc)), d);
    ring[1][tid + 1] = psi_root(psi2c);
  }
  __syncthreads();  // the halo columns are in LDS
  if (tid == 0) {
    ring[0][0] = haloL[0];
    ring[0][ncols + 1] = haloR[0];
    ring[1][0] = haloL[1];
    ring[1][ncols + 1] = haloR[1];
  }

  for (int j = 0; j < nrows; ++j) {
    const int y = y0 + j;
    const int yn = y + 1 == d.ny ? 0 : y + 1;
    const int sl = (j + 2) & 3;
    R fnn[9];
    P psi2n = P(0);
    if (act) {
      if (PF == 2) {
        if (j + 1 < nrows) pull9<S>(src, d, cx, yn + 1 == d.ny ? 0 : yn + 1, fnn);
      } else {
        pull9<S>(src, d, cx, yn, fn);
      }
      psi2n = psi2_of(rref + P(sum9(fn)), d);
      ring[sl][tid + 1] = psi_root(psi2n);
    }
    if (tid == 0) {
      ring[sl][0] = haloL[j + 2];
      ring[sl][ncols + 1] = haloR[j + 2];
    }
    __syncthreads();
    if (act) {
      P Fx, Fy;
      force3x3(ring[j & 3], ring[(j + 1) & 3], ring[sl], tid + 1, P(d.mG), Fx, Fy);
      const R drho = sum9(fc);
      const P rho = rref + P(drho);
      bad |= !(psi2c > P(0)) || !(rho > P(0));
      const R ip2 = d.sig != 0.0 ? rcp(R(psi2c)) : R(0);
      update_node<S, MRT>(fc, drho, rho, Fx, Fy, ip2, d);
      typename T::E* row = dst + (int64_t)y * d.rs;
#pragma unroll
      for (int a = 0; a < 9; ++a)
        if (index_ok(row + a * d.plane + cx.x - dst, d.elems)) T::st(row + a * d.plane + cx.x, fc[a]);
#pragma unroll
      for (int a = 0; a < 9; ++a) fc[a] = fn[a];
      psi2c = psi2n;
      if (PF == 2 && j + 1 < nrows) {
#pragma unroll
        for (int a = 0; a < 9; ++a) fn[a] = fnn[a];
      }
    }
  }
  // divergence: one atomic per wave that saw a bad node
  if (__ballot(bad) != 0 && __lane_id() == 0) atomicMin(flag, step);
}

// A run that diverged at an earlier launch is frozen: instead of a time step
// its tiles copy the stored populations unchanged from src to dst, so both
// buffers hold the state the diverging launch wrote, whatever the parity of
// later launches.  Columns [x0, x0+ncols), rows [y0, y0+nrows), SW threads.
template <typename S, int SW>
__device__ __forceinline__ void copy_tile(const typename Store<S>::E* __restrict__ src,
                                          typename Store<S>::E* __restrict__ dst, const RunDev& d,
                                          int x0, int y0, int ncols, int nrows) {
  if ((int)threadIdx.x >= ncols) return;
  const int x = x0 + (int)threadIdx.x;
  for (int j = 0; j < nrows; ++j) {
    const int64_t o = (int64_t)(y0 + j) * d.rs + x;
#pragma unroll
    for (int a = 0; a < 9; ++a)
      if (index_ok(o + a * d.plane, d.elems)) dst[o + a * d.plane] = src[o + a * d.plane];
  }
}

// XCD-aware block order: consecutive tiles go to the same XCD (blocks are
// dispatched round-robin over the 8 XCDs), so halo rows/columns shared by
// neighbouring tiles are found in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7, k = b & 7, i = b >> 3;
  return k * q + (k < r ? k : r) + i;
}

// Single-lattice step.  L > 0: one block per (strip, L-row chunk).  L == 0:
// balanced schedule, the strip-major row space [0, nstrips*ny) is split evenly
// over the grid (sized to the resident capacity) and each block marches its
// share in pieces of at most LMAX rows.
template <typename S, int NW, int PF, bool MRT = false>
__global__ __launch_bounds__(64 * NW) void k_step(const typename Store<S>::E* __restrict__ src,
                                                  typename Store<S>::E* __restrict__ dst,
                                                  RunDev d, int L, int nstrips,
                                                  const unsigned long long* stepbase,
                                                  unsigned long long steplocal,
                                                  unsigned long long* flag) {
  __shared__ typename Store<S>::P ring[4][64 * NW + 2];
  __shared__ typename Store<S>::P haloL[LMAX + 2], haloR[LMAX + 2];
  constexpr int SW = 64 * NW;
  const unsigned long long step = (stepbase ? *stepbase : 0ull) + steplocal;
  const bool frozen = *flag < step;  // diverged at an earlier step
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  if (L > 0) {
    const int sy = t / nstrips, sx = t - sy * nstrips;
    const int x0 = sx * SW, y0 = sy * L;
    if (frozen)
      copy_tile<S, SW>(src, dst, d, x0, y0, min(SW, d.nx - x0), min(L, d.ny - y0));
    else
      tile_step<S, NW, PF, MRT>(src, dst, d, x0, y0, min(SW, d.nx - x0), min(L, d.ny - y0), step, flag,
                           ring, haloL, haloR);
    return;
  }
  const int64_t total = (int64_t)nstrips * d.ny;
  int64_t r = total * t / gridDim.x;
  const int64_t e = total * (t + 1) / gridDim.x;
  while (r < e) {
    const int s = (int)(r / d.ny), y = (int)(r - (int64_t)s * d.ny);
    int n = (int)min(e - r, (int64_t)(d.ny - y));
    n = min(n, LMAX);
    const int x0 = s * SW;
    if (frozen)
      copy_tile<S, SW>(src, dst, d, x0, y, min(SW, d.nx - x0), n);
    else
      tile_step<S, NW, PF, MRT>(src, dst, d, x0, y, min(SW, d.nx - x0), n, step, flag, ring, haloL,
                           haloR);
    r += n;
    __syncthreads();  // LDS is reused by the next piece
  }
}

// ---- two time steps per launch ------------------------------------------------

// Row modes of tile_step2 (bit set): a steady row, and the phases that run
// on every lane of the block instead of on their own lane range.
constexpr int kRowPsi = 1, kRowPull2 = 2, kRowCollide1 = 4, kRowCollide2 = 8, kRowSteady = 16;
// Mode of the steady rows per storage type, chosen by measurement on the
// 4096 x 4096 droplet workload.
template <typename S> struct SteadyMode
    : std::integral_constant<int, kRowSteady | kRowPsi | kRowPull2 | kRowCollide1 | kRowCollide2> {};
template <> struct SteadyMode<double> : std::integral_constant<int, kRowSteady | kRowPull2> {};
// The batched kernel unmasks every phase for every storage type: on the
// 256-run sweep (2-wave strips of 16-64-row lattices) that is 2 % faster for
// FP64 storage (44.3 -> 45.3 GLUPS), while on the 4096 x 4096 lattice it makes
// the single-lattice FP64 kernel 5 % slower (485 -> 513 us per launch).
constexpr int kBatchSteadyMode = kRowSteady | kRowPsi | kRowPull2 | kRowCollide1 | kRowCollide2;
// Steady rows per loop iteration (1 to 3), measured likewise.  Unrolling by 3
// removes the rotation moves but adds registers; it pays for FP32 storage with
// FP64 arithmetic and for FP16 storage (261 -> 251 us per launch, 161-167
// VGPRs: still 3 waves per SIMD); FP64 storage: 7 % fewer VALU instructions
// per row yet 5 % slower; FP32 storage would fall from 3 to 2 waves per SIMD
// (241 VGPRs).
template <typename S> struct SteadyUnroll : std::integral_constant<int, 1> {};
template <> struct SteadyUnroll<f32s_f64a> : std::integral_constant<int, 3> {};
template <> struct SteadyUnroll<__half> : std::integral_constant<int, 3> {};

// The populations cross HBM once per two steps.  Lane i of a block owns
// column c = x0 - 3 + i for both steps, i < ncols + 6:
//   * every lane pulls its column and evaluates psi(t);
//   * lanes 1 .. ncols+4 run step one (t -> t+1) exactly as tile_step does and
//     keep f*(t+1) in registers, rounded to the storage type;
//   * lanes 2 .. ncols+3 pull f*(t+1) for step two and evaluate psi(t+1);
//   * lanes 3 .. ncols+2 finish step two and write the columns [x0, x0+ncols),
// so neighbouring strips overlap by six columns of recomputed work and no
// halo column is loaded apart from the coalesced row loads.  Rows: step two
// writes [y0, y0 + L); it needs psi(t+1) on rows y0-1 .. y0+L, hence f*(t+1)
// on rows y0-2 .. y0+L+1, hence psi(t) on rows y0-3 .. y0+L+2.  Step two
// pulls f*(t+1) from registers for the x-unshifted directions (0, 2, 4) and
// from an LDS exchange row for the six shifted ones, and runs three rows
// behind step one; one row of the march takes two barriers.  Both steps use
// the same arithmetic, in the same order, as two single-step launches, so the
// result is bitwise identical.
template <typename S, int NW, int PF, int MODE = SteadyMode<S>::value, bool MRT = false>
__device__ __forceinline__ void tile_step2(const typename Store<S>::E* __restrict__ src,
                                           typename Store<S>::E* __restrict__ dst,
                                           const RunDev& d, int x0, int y0, int ncols, int nrows,
                                           unsigned long long step,
                                           unsigned long long* __restrict__ flag,
                                           typename Store<S>::P (*ring1)[64 * NW],
                                           typename Store<S>::P (*ring2)[64 * NW],
                                           typename Store<S>::R (*xch)[64 * NW]) {
  using T = Store<S>;
  using R = typename T::R;
  using P = typename T::P;
  const int tid = threadIdx.x;
  LBM_TILE_CHECK(ncols >= 1 && ncols <= 64 * NW - 6 && nrows >= 1 && x0 >= 0 &&
                 x0 + ncols <= d.nx && y0 >= 0 && y0 + nrows <= d.ny);
  const int n0 = ncols + 6;                         // lanes that evaluate psi(t)
  const bool act0 = tid < n0;
  const bool act1 = tid >= 1 && tid < n0 - 1;       // lanes that run step one
  const bool pull2 = tid >= 2 && tid < n0 - 2;      // lanes that pull for step two
  const bool out = tid >= 3 && tid < ncols + 3;     // lanes that write step two
  // LDS neighbour index: tid on every lane of the ranges above, kept inside
  // the rows for lanes 0 and 64*NW-1
  const int tc = min(max(tid, 1), 64 * NW - 2);
  auto wrapx = [&](int x) { return x < 0 ? x + d.nx : (x >= d.nx ? x - d.nx : x); };
  auto wrapy = [&](int y) { return y < 0 ? y + d.ny : (y >= d.ny ? y - d.ny : y); };
  const Cols cx = cols_of(wrapx(x0 - 3 + min(tid, n0 - 1)), d.nx);
  const P rref = P(d.rho_ref);
  bool bad1 = false, bad2 = false;
  const int ya = y0 - 3;                            // first psi(t) row

  // preload: psi(t) of rows y0-3 (ring slot 0) and y0-2 (slot 1); pulled row y0-2
  R fc[9] = {}, fn[9] = {};
  P psi2c = P(0);
  if (act0) {
    R f[9];
    pull9<S>(src, d, cx, wrapy(ya), f);
    pull9<S>(src, d, cx, wrapy(ya + 1), fc);
    if (PF == 2) pull9<S>(src, d, cx, wrapy(ya + 2), fn);
    ring1[0][tid] = psi_root(psi2_of(rref + P(sum9(f)), d));
    psi2c = psi2_of(rref + P(sum9(fc)), d);
    ring1[1][tid] = psi_root(psi2c);
  }

  // f*(t+1) of the last three step-one rows, kept for step two:
  // gA = row y1-1 (all 9), gB = row y1-2 (0,1,3,2,5,6), gC = row y1-3 (2,5,6)
  R gA[9] = {}, gB[6] = {}, gC[3] = {};
  R hp[9] = {};     // step-two pulled populations of the row collided next
  P psi2p = P(0);
  const int n_one = nrows + 4;                      // step-one rows y0-2 .. y0+nrows+1
  // One row of the march.  Mode (MODE: SteadyMode, or kBatchSteadyMode in the
  // batched kernel) bit 16 marks a steady row, in
  // which every row condition below holds; bits 1, 2, 4, 8 make a phase run
  // on every lane of the block: lanes outside the phase's range compute values
  // that no lane in range reads (their LDS slots are read only by lanes
  // outside the ranges too, and tc keeps their neighbour reads inside the
  // rows), so that phase carries no per-lane branch apart from the store.
  auto row = [&](const int j, auto mode) __attribute__((always_inline)) {
    constexpr int M = decltype(mode)::value;
    constexpr bool St = (M & kRowSteady) != 0;
    const int y1 = y0 - 2 + j;                      // step-one row collided at this j
    // ---- phase 1: psi(t) of row y1+1; exchange of the rows step two pulls
    R fnn[9];
    P psi2n = P(0);
    if ((St || j < n_one) && ((M & kRowPsi) || act0)) {
      // the row loads go out at raised wave priority, so a wave about to issue
      // them is not held behind the other wave's arithmetic (FP64: 1 % faster)
      __builtin_amdgcn_s_setprio(2);
      if (PF == 2) {
        if (St || j + 1 < n_one) pull9<S>(src, d, cx, wrapy(y1 + 2), fnn);
      } else {
        pull9<S>(src, d, cx, wrapy(y1 + 1), fn);
      }
      __builtin_amdgcn_s_setprio(0);
      psi2n = psi2_of(rref + P(sum9(fn)), d);
      ring1[(j + 2) & 3][tid] = psi_root(psi2n);
    }
    if ((St || j >= 3) && ((M & kRowPsi) || act1)) {  // step two pulls row q = y1 - 2 below
      xch[0][tid] = gB[1];
      xch[1][tid] = gB[2];
      xch[2][tid] = gC[1];
      xch[3][tid] = gC[2];
      xch[4][tid] = gA[7];
      xch[5][tid] = gA[8];
    }
    __syncthreads();
    // ---- phase 2: step-two pull of row q = y1-2 and its psi(t+1); step-one collide of row y1
    const int q = y1 - 2;
    R hn[9];
    P psi2q = P(0);
    if ((St || j >= 3) && ((M & kRowPull2) || pull2)) {
      hn[0] = gB[0];
      hn[1] = xch[0][tc - 1];
      hn[2] = gC[0];
      hn[3] = xch[1][tc + 1];
      hn[4] = gA[4];
      hn[5] = xch[2][tc - 1];
      hn[6] = xch[3][tc + 1];
      hn[7] = xch[4][tc + 1];
      hn[8] = xch[5][tc - 1];
      psi2q = psi2_of(rref + P(sum9(hn)), d);
      ring2[(q - (y0 - 1)) & 3][tid] = psi_root(psi2q);
    }
    if (St || j >= 1) {  // rotate the kept step-one rows (gA was produced at j-1)
      gC[0] = gB[3]; gC[1] = gB[4]; gC[2] = gB[5];
      gB[0] = gA[0]; gB[1] = gA[1]; gB[2] = gA[3];
      gB[3] = gA[2]; gB[4] = gA[5]; gB[5] = gA[6];
    }
    if ((St || j < n_one) && ((M & kRowCollide1) || act0)) {
      if ((M & kRowCollide1) || act1) {
        P Fx, Fy;
        force3x3(ring1[j & 3], ring1[(j + 1) & 3], ring1[(j + 2) & 3], tc, P(d.mG), Fx, Fy);
        const R drho = sum9(fc);
        const P rho = rref + P(drho);
        const bool chk = out && y1 >= y0 && y1 < y0 + nrows;
        bad1 |= chk && (!(psi2c > P(0)) || !(rho > P(0)));
        const R ip2 = d.sig != 0.0 ? rcp(R(psi2c)) : R(0);
        update_node<S, MRT>(fc, drho, rho, Fx, Fy, ip2, d);
#pragma unroll
        for (int a = 0; a < 9; ++a) gA[a] = T::round(fc[a]);
      }
#pragma unroll
      for (int a = 0; a < 9; ++a) fc[a] = fn[a];
      psi2c = psi2n;
      if (PF == 2 && (St || j + 1 < n_one)) {
#pragma unroll
        for (int a = 0; a < 9; ++a) fn[a] = fnn[a];
      }
    }
    __syncthreads();
    // ---- phase 3: step-two collide of row r = q-1 and store
    const int r = q - 1;
    if ((St || (j >= 4 && r >= y0 && r < y0 + nrows)) && ((M & kRowCollide2) || out)) {
      P Fx, Fy;
      force3x3(ring2[(r - 1 - (y0 - 1)) & 3], ring2[(r - (y0 - 1)) & 3], ring2[(q - (y0 - 1)) & 3],
               tc, P(d.mG), Fx, Fy);
      const R drho = sum9(hp);
      const P rho = rref + P(drho);
      bad2 |= out && (!(psi2p > P(0)) || !(rho > P(0)));
      const R ip2 = d.sig != 0.0 ? rcp(R(psi2p)) : R(0);
      update_node<S, MRT>(hp, drho, rho, Fx, Fy, ip2, d);
      if (out) {
        typename T::E* orow = dst + (int64_t)wrapy(r) * d.rs;
#pragma unroll
        for (int a = 0; a < 9; ++a)
          if (index_ok(orow + a * d.plane + cx.x - dst, d.elems)) T::st(orow + a * d.plane + cx.x, hp[a]);
      }
    }
    if (St || j >= 3) {
#pragma unroll
      for (int a = 0; a < 9; ++a) hp[a] = hn[a];
      psi2p = psi2q;
    }
  };
  // rows 0..4 fill the pipeline, 5 .. n_one-2 are steady, the last two drain it
  using Edge = std::integral_constant<int, 0>;
  using Steady = std::integral_constant<int, MODE>;
  for (int j = 0; j < 5; ++j) row(j, Edge{});
  // Steady rows U at a time (a loop with barriers is not unrolled by the
  // compiler): with U = 3, the period of the kept-row rotations (gA -> gB ->
  // gC, fnn -> fn -> fc), those rotations become register renaming instead of
  // moves.
  // The steady rows end where the row loads one row ahead would pass the last
  // step-one row.
  constexpr int U = SteadyUnroll<S>::value;
  const int js_end = n_one - 1;
  int js = 5;
  for (; js + U <= js_end; js += U) {
    row(js, Steady{});
    if constexpr (U > 1) row(js + 1, Steady{});
    if constexpr (U > 2) row(js + 2, Steady{});
  }
  if constexpr (U > 1)
    for (; js < js_end; ++js) row(js, Steady{});
  for (int j = max(5, js_end); j < n_one + 1; ++j) row(j, Edge{});
  // divergence: the first step that saw a bad node (one atomic per wave)
  const auto b1 = __ballot(bad1), b2 = __ballot(bad2);
  if (__lane_id() == 0 && (b1 | b2) != 0) atomicMin(flag, b1 != 0 ? step : step + 1);
}

// Strip edges of the two-step kernel are rounded down to multiples of this
// many columns (FP64: 8 columns = 64 B, so no 64-byte segment of a population
// row is written by two blocks; 3 % faster on the 4096 x 4096 droplet
// workload).  Strips then span at most nx / nstrips + A - 1 columns, which the
// launcher's strip count keeps within 64*NW - 6.
template <typename S> struct Step2Align : std::integral_constant<int, 1> {};
template <> struct Step2Align<double> : std::integral_constant<int, 8> {};

// Two steps per launch over the single lattice; strips of at most 64*NW - 6
// columns, spread evenly over nx (edges aligned as Step2Align says).  L > 0: one block per (strip, L-row chunk);
// L == 0: balanced schedule, every block marches one contiguous share of the
// strip-major row space (no length cap: the tile holds no per-row arrays); a
// share is split where it crosses a strip boundary.  (With the row-interleaved
// layout a band-major order -- the blocks of one XCD marching one band of rows
// across all strips -- measured no faster for any storage type.)
template <typename S, int NW, int PF, bool MRT = false>
__global__ __launch_bounds__(64 * NW) void k_step2(const typename Store<S>::E* __restrict__ src,
                                                   typename Store<S>::E* __restrict__ dst,
                                                   RunDev d, int L, int nstrips,
                                                   const unsigned long long* stepbase,
                                                   unsigned long long steplocal,
                                                   unsigned long long* flag) {
  using R = typename Store<S>::R;
  __shared__ typename Store<S>::P ring1[4][64 * NW];
  __shared__ typename Store<S>::P ring2[4][64 * NW];
  __shared__ R xch[6][64 * NW];
  const unsigned long long step = (stepbase ? *stepbase : 0ull) + steplocal;
  const bool frozen = *flag < step;  // diverged at an earlier step
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  auto strip = [&](int sx, int& x0, int& nc) {
    constexpr int A = Step2Align<S>::value;
    auto edge = [&](int k) {
      return k >= nstrips ? d.nx : (int)((int64_t)k * d.nx / nstrips) / A * A;
    };
    x0 = edge(sx);
    nc = edge(sx + 1) - x0;
  };
  if (L > 0) {
    const int sy = t / nstrips, sx = t - sy * nstrips;
    int x0, nc;
    strip(sx, x0, nc);
    const int y0 = sy * L;
    if (frozen)
      copy_tile<S, 64 * NW>(src, dst, d, x0, y0, nc, min(L, d.ny - y0));
    else
      tile_step2<S, NW, PF, SteadyMode<S>::value, MRT>(src, dst, d, x0, y0, nc, min(L, d.ny - y0),
                                                       step, flag, ring1, ring2,
                            xch);
    return;
  }
  const int64_t total = (int64_t)nstrips * d.ny;
  int64_t r = total * t / gridDim.x;
  const int64_t e = total * (t + 1) / gridDim.x;
  while (r < e) {
    const int s = (int)(r / d.ny), y = (int)(r - (int64_t)s * d.ny);
    const int n = (int)min(e - r, (int64_t)(d.ny - y));
    int x0, nc;
    strip(s, x0, nc);
    if (frozen)
      copy_tile<S, 64 * NW>(src, dst, d, x0, y, nc, n);
    else
      tile_step2<S, NW, PF, SteadyMode<S>::value, MRT>(src, dst, d, x0, y, nc, n, step, flag, ring1,
                                                       ring2, xch);
    r += n;
    __syncthreads();  // LDS is reused by the next piece
  }
}

// ---- three time steps per launch ----------------------------------------------

// Three steps per launch: the pipeline of tile_step2 with a third level.  Lane
// i of a block owns column c = x0 - 5 + i for all three steps, i < ncols + 10:
//   * every lane pulls its column and evaluates psi(t);
//   * lanes 1 .. ncols+8 run step one and keep f*(t+1) (the last three rows);
//   * lanes 2 .. ncols+7 pull f*(t+1) and evaluate psi(t+1), lanes 3 ..
//     ncols+6 run step two and keep f*(t+2) likewise;
//   * lanes 4 .. ncols+5 pull f*(t+2) and evaluate psi(t+2), lanes 5 ..
//     ncols+4 run step three and write the columns [x0, x0+ncols).
// Rows: step three writes [y0, y0+nrows), so step two produces rows y0-2 ..
// y0+nrows+1, step one rows y0-4 .. y0+nrows+3, and psi(t) is evaluated on
// rows y0-5 .. y0+nrows+4.  At march row j step one collides y1 = y0-4+j,
// step two pulls y1-2 and collides y1-3, step three pulls y1-5 and collides
// y1-6.  Each step pulls the x-unshifted directions of the previous step's
// rows from the lane's own registers and the six shifted ones through an LDS
// exchange row, as in tile_step2; two barriers per march row.  Same
// arithmetic in the same order as three single-step launches: bitwise equal.
template <typename S, int NW, bool MRT = false>
__device__ __forceinline__ void tile_step3(const typename Store<S>::E* __restrict__ src,
                                           typename Store<S>::E* __restrict__ dst,
                                           const RunDev& d, int x0, int y0, int ncols, int nrows,
                                           unsigned long long step,
                                           unsigned long long* __restrict__ flag,
                                           typename Store<S>::P (*ring1)[64 * NW],
                                           typename Store<S>::P (*ring2)[64 * NW],
                                           typename Store<S>::P (*ring3)[64 * NW],
                                           typename Store<S>::R (*xch1)[64 * NW],
                                           typename Store<S>::R (*xch2)[64 * NW]) {
  using T = Store<S>;
  using R = typename T::R;
  using P = typename T::P;
  const int tid = threadIdx.x;
  LBM_TILE_CHECK(ncols >= 1 && ncols <= 64 * NW - 10 && nrows >= 1 && x0 >= 0 &&
                 x0 + ncols <= d.nx && y0 >= 0 && y0 + nrows <= d.ny);
  const int n0 = ncols + 10;                        // lanes that evaluate psi(t)
  const bool act0 = tid < n0;
  const bool act1 = tid >= 1 && tid < n0 - 1;       // step one
  const bool pull2 = tid >= 2 && tid < n0 - 2;      // step-two pull, psi(t+1)
  const bool act2 = tid >= 3 && tid < n0 - 3;       // step two
  const bool pull3 = tid >= 4 && tid < n0 - 4;      // step-three pull, psi(t+2)
  const bool out = tid >= 5 && tid < n0 - 5;        // step three and the store
  const int tc = min(max(tid, 1), 64 * NW - 2);     // LDS neighbour index inside the rows
  auto wrapx = [&](int x) { return x < 0 ? x + d.nx : (x >= d.nx ? x - d.nx : x); };
  auto wrapy = [&](int y) { return y < 0 ? y + d.ny : (y >= d.ny ? y - d.ny : y); };
  const Cols cx = cols_of(wrapx(x0 - 5 + min(tid, n0 - 1)), d.nx);
  const P rref = P(d.rho_ref);
  bool bad1 = false, bad2 = false, bad3 = false;
  const int ya = y0 - 5;                            // first psi(t) row (ring1 slot 0)
  const int yb = y0 - 3;                            // first psi(t+1) row (ring2 slot 0)
  const int yc = y0 - 1;                            // first psi(t+2) row (ring3 slot 0)

  R fc[9] = {}, fn[9] = {};
  P psi2c = P(0);
  if (act0) {
    R f[9];
    pull9<S>(src, d, cx, wrapy(ya), f);
    pull9<S>(src, d, cx, wrapy(ya + 1), fc);
    ring1[0][tid] = psi_root(psi2_of(rref + P(sum9(f)), d));
    psi2c = psi2_of(rref + P(sum9(fc)), d);
    ring1[1][tid] = psi_root(psi2c);
  }
  // f*(t+1) kept for step two: gA = row y1-1 (all 9), gB = y1-2 (0,1,3,2,5,6),
  // gC = y1-3 (2,5,6); f*(t+2) kept for step three likewise (kA, kB, kC, rows
  // produced one, two and three march rows ago)
  R gA[9] = {}, gB[6] = {}, gC[3] = {};
  R kA[9] = {}, kB[6] = {}, kC[3] = {};
  R hp[9] = {}, hp3[9] = {};   // pulled rows of steps two and three collided next
  P psi2p = P(0), psi3p = P(0);
  const int n_one = nrows + 8;                      // step-one rows y0-4 .. y0+nrows+3
  auto row = [&](const int j, auto steady) __attribute__((always_inline)) {
    constexpr bool St = decltype(steady)::value;
    const int y1 = y0 - 4 + j;
    // ---- phase 1: psi(t) of row y1+1; exchange rows for steps two and three
    P psi2n = P(0);
    if ((St || j < n_one) && act0) {
      __builtin_amdgcn_s_setprio(2);
      pull9<S>(src, d, cx, wrapy(y1 + 1), fn);
      __builtin_amdgcn_s_setprio(0);
      psi2n = psi2_of(rref + P(sum9(fn)), d);
      ring1[(j + 2) & 3][tid] = psi_root(psi2n);
    }
    const bool lv2 = St || (j >= 3 && j <= n_one);  // step two pulls q2 = y1-2
    const bool lv3 = St || j >= 8;                  // step three pulls q3 = y1-5
    // In steady rows the exchange writes and the pulls of steps two and three
    // run on every lane: a lane outside a range writes and reads only LDS slots
    // that no lane inside the range reads (tc keeps its neighbour reads inside
    // the rows), so its values are never used.
    if (lv2 && (St || act1)) {
      xch1[0][tid] = gB[1];
      xch1[1][tid] = gB[2];
      xch1[2][tid] = gC[1];
      xch1[3][tid] = gC[2];
      xch1[4][tid] = gA[7];
      xch1[5][tid] = gA[8];
    }
    if (lv3 && (St || act2)) {
      xch2[0][tid] = kB[1];
      xch2[1][tid] = kB[2];
      xch2[2][tid] = kC[1];
      xch2[3][tid] = kC[2];
      xch2[4][tid] = kA[7];
      xch2[5][tid] = kA[8];
    }
    __syncthreads();
    // ---- phase 2: pulls of steps two and three and their psi; step-one collide
    const int q2 = y1 - 2, q3 = y1 - 5;
    R hn[9], hn3[9];
    P psi2q = P(0), psi3q = P(0);
    if (lv2 && (St || pull2)) {
      hn[0] = gB[0];
      hn[1] = xch1[0][tc - 1];
      hn[2] = gC[0];
      hn[3] = xch1[1][tc + 1];
      hn[4] = gA[4];
      hn[5] = xch1[2][tc - 1];
      hn[6] = xch1[3][tc + 1];
      hn[7] = xch1[4][tc + 1];
      hn[8] = xch1[5][tc - 1];
      psi2q = psi2_of(rref + P(sum9(hn)), d);
      ring2[(q2 - yb) & 3][tid] = psi_root(psi2q);
    }
    if (lv3 && (St || pull3)) {
      hn3[0] = kB[0];
      hn3[1] = xch2[0][tc - 1];
      hn3[2] = kC[0];
      hn3[3] = xch2[1][tc + 1];
      hn3[4] = kA[4];
      hn3[5] = xch2[2][tc - 1];
      hn3[6] = xch2[3][tc + 1];
      hn3[7] = xch2[4][tc + 1];
      hn3[8] = xch2[5][tc - 1];
      psi3q = psi2_of(rref + P(sum9(hn3)), d);
      ring3[(q3 - yc) & 3][tid] = psi_root(psi3q);
    }
    if (St || j >= 1) {  // rotate the kept step-one rows (gA was produced at j-1)
      gC[0] = gB[3]; gC[1] = gB[4]; gC[2] = gB[5];
      gB[0] = gA[0]; gB[1] = gA[1]; gB[2] = gA[3];
      gB[3] = gA[2]; gB[4] = gA[5]; gB[5] = gA[6];
    }
    if ((St || j < n_one) && act0) {
      if (act1) {
        P Fx, Fy;
        force3x3(ring1[j & 3], ring1[(j + 1) & 3], ring1[(j + 2) & 3], tc, P(d.mG), Fx, Fy);
        const R drho = sum9(fc);
        const P rho = rref + P(drho);
        const bool chk = out && y1 >= y0 && y1 < y0 + nrows;
        bad1 |= chk && (!(psi2c > P(0)) || !(rho > P(0)));
        const R ip2 = d.sig != 0.0 ? rcp(R(psi2c)) : R(0);
        update_node<S, MRT>(fc, drho, rho, Fx, Fy, ip2, d);
#pragma unroll
        for (int a = 0; a < 9; ++a) gA[a] = T::round(fc[a]);
      }
#pragma unroll
      for (int a = 0; a < 9; ++a) fc[a] = fn[a];
      psi2c = psi2n;
    }
    __syncthreads();
    // ---- phase 3: step-two collide of row r2 = q2-1; step-three collide of r3 = q3-1 and store
    const int r2 = q2 - 1, r3 = q3 - 1;
    if (St || (j >= 5 && j <= n_one)) {
      // rotate the kept step-two rows (kA was produced at j-1)
      kC[0] = kB[3]; kC[1] = kB[4]; kC[2] = kB[5];
      kB[0] = kA[0]; kB[1] = kA[1]; kB[2] = kA[3];
      kB[3] = kA[2]; kB[4] = kA[5]; kB[5] = kA[6];
      if (act2) {
        P Fx, Fy;
        force3x3(ring2[(r2 - 1 - yb) & 3], ring2[(r2 - yb) & 3], ring2[(q2 - yb) & 3], tc, P(d.mG),
                 Fx, Fy);
        const R drho = sum9(hp);
        const P rho = rref + P(drho);
        const bool chk = out && r2 >= y0 && r2 < y0 + nrows;
        bad2 |= chk && (!(psi2p > P(0)) || !(rho > P(0)));
        const R ip2 = d.sig != 0.0 ? rcp(R(psi2p)) : R(0);
        update_node<S, MRT>(hp, drho, rho, Fx, Fy, ip2, d);
#pragma unroll
        for (int a = 0; a < 9; ++a) kA[a] = T::round(hp[a]);
      }
    }
    if (lv2) {
#pragma unroll
      for (int a = 0; a < 9; ++a) hp[a] = hn[a];
      psi2p = psi2q;
    }
    if ((St || j >= 10) && out) {
      P Fx, Fy;
      force3x3(ring3[(r3 - 1 - yc) & 3], ring3[(r3 - yc) & 3], ring3[(q3 - yc) & 3], tc, P(d.mG),
               Fx, Fy);
      const R drho = sum9(hp3);
      const P rho = rref + P(drho);
      bad3 |= !(psi3p > P(0)) || !(rho > P(0));
      const R ip2 = d.sig != 0.0 ? rcp(R(psi3p)) : R(0);
      update_node<S, MRT>(hp3, drho, rho, Fx, Fy, ip2, d);
      typename T::E* orow = dst + (int64_t)wrapy(r3) * d.rs;
#pragma unroll
      for (int a = 0; a < 9; ++a)
        if (index_ok(orow + a * d.plane + cx.x - dst, d.elems)) T::st(orow + a * d.plane + cx.x, hp3[a]);
    }
    if (lv3) {
#pragma unroll
      for (int a = 0; a < 9; ++a) hp3[a] = hn3[a];
      psi3p = psi3q;
    }
  };
  // rows 0..9 fill the pipeline, 10 .. n_one-1 are steady (every row condition
  // above holds), the last two drain it
  using Edge = std::integral_constant<bool, false>;
  using Steady = std::integral_constant<bool, true>;
  for (int j = 0; j < 10; ++j) row(j, Edge{});
  for (int j = 10; j < n_one; ++j) row(j, Steady{});
  for (int j = max(10, n_one); j < n_one + 2; ++j) row(j, Edge{});
  const auto b1 = __ballot(bad1), b2 = __ballot(bad2), b3 = __ballot(bad3);
  if (__lane_id() == 0 && (b1 | b2 | b3) != 0)
    atomicMin(flag, b1 != 0 ? step : (b2 != 0 ? step + 1 : step + 2));
}

// Three steps per launch over the single lattice (FP64 collision arithmetic):
// strips of at most 64*NW - 10 columns spread evenly over nx, edges aligned as
// for the two-step kernel; L > 0: one block per (strip, L-row chunk); L == 0:
// the balanced schedule of k_step2.
template <typename S, int NW, bool MRT = false>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2))) void k_step3(const typename Store<S>::E* __restrict__ src,
                                                   typename Store<S>::E* __restrict__ dst,
                                                   RunDev d, int L, int nstrips,
                                                   const unsigned long long* stepbase,
                                                   unsigned long long steplocal,
                                                   unsigned long long* flag) {
  using R = typename Store<S>::R;
  using P = typename Store<S>::P;
  __shared__ P ring1[4][64 * NW];
  __shared__ P ring2[4][64 * NW];
  __shared__ P ring3[4][64 * NW];
  __shared__ R xch1[6][64 * NW];
  __shared__ R xch2[6][64 * NW];
  const unsigned long long step = (stepbase ? *stepbase : 0ull) + steplocal;
  const bool frozen = *flag < step;  // diverged at an earlier step
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  auto strip = [&](int sx, int& x0, int& nc) {
    constexpr int A = Step2Align<S>::value;
    auto edge = [&](int k) {
      return k >= nstrips ? d.nx : (int)((int64_t)k * d.nx / nstrips) / A * A;
    };
    x0 = edge(sx);
    nc = edge(sx + 1) - x0;
  };
  if (L > 0) {
    const int sy = t / nstrips, sx = t - sy * nstrips;
    int x0, nc;
    strip(sx, x0, nc);
    const int y0 = sy * L;
    if (frozen)
      copy_tile<S, 64 * NW>(src, dst, d, x0, y0, nc, min(L, d.ny - y0));
    else
      tile_step3<S, NW, MRT>(src, dst, d, x0, y0, nc, min(L, d.ny - y0), step, flag, ring1, ring2, ring3,
                        xch1, xch2);
    return;
  }
  const int64_t total = (int64_t)nstrips * d.ny;
  int64_t r = total * t / gridDim.x;
  const int64_t e = total * (t + 1) / gridDim.x;
  while (r < e) {
    const int s = (int)(r / d.ny), y = (int)(r - (int64_t)s * d.ny);
    const int n = (int)min(e - r, (int64_t)(d.ny - y));
    int x0, nc;
    strip(s, x0, nc);
    if (frozen)
      copy_tile<S, 64 * NW>(src, dst, d, x0, y, nc, n);
    else
      tile_step3<S, NW, MRT>(src, dst, d, x0, y, nc, n, step, flag, ring1, ring2, ring3, xch1, xch2);
    r += n;
    __syncthreads();  // LDS is reused by the next piece
  }
}

// Persistent batched step: blocks of XCD k walk the k-th contiguous eighth of
// the work list.  Grid must be a multiple of 8.
template <typename S, int NW, int PF, bool MRT = false>
__global__ __launch_bounds__(64 * NW) void k_batch_step(const typename Store<S>::E* __restrict__ src,
                                                        typename Store<S>::E* __restrict__ dst,
                                                        const RunDev* __restrict__ runs,
                                                        const Item* __restrict__ items, int nitems,
                                                        int total,
                                                        const unsigned long long* stepbase,
                                                        unsigned long long steplocal,
                                                        unsigned long long* flags) {
  __shared__ typename Store<S>::P ring[4][64 * NW + 2];
  __shared__ typename Store<S>::P haloL[LMAX + 2], haloR[LMAX + 2];
  const unsigned long long step = (stepbase ? *stepbase : 0ull) + steplocal;
  if (total > 0) {  // balanced schedule over whole-strip items
    balanced_pieces(items, nitems, total, xcd_remap(blockIdx.x, gridDim.x), LMAX,
                    [&](const Item& it, int y, int n) {
                      const RunDev d = runs[it.run];
                      if (flags[it.run] < step)
                        copy_tile<S, 64 * NW>(src + d.off, dst + d.off, d, it.x0, it.y0 + y, it.ncols, n);
                      else
                        tile_step<S, NW, PF, MRT>(src + d.off, dst + d.off, d, it.x0, it.y0 + y, it.ncols,
                                                  n, step, &flags[it.run], ring, haloL, haloR);
                    });
    return;
  }
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, nb = gridDim.x >> 3;
  const int lo = (int)((int64_t)nitems * xcd / 8), hi = (int)((int64_t)nitems * (xcd + 1) / 8);
  for (int i = lo + slot; i < hi; i += nb) {
    const Item it = items[i];
    const RunDev d = runs[it.run];
    if (flags[it.run] < step)  // frozen run
      copy_tile<S, 64 * NW>(src + d.off, dst + d.off, d, it.x0, it.y0, it.ncols, it.nrows);
    else
      tile_step<S, NW, PF, MRT>(src + d.off, dst + d.off, d, it.x0, it.y0, it.ncols, it.nrows, step,
                           &flags[it.run], ring, haloL, haloR);
    __syncthreads();  // LDS is reused by the next item
  }
}

// Persistent batched launch of two steps (tile_step2) over a work list whose
// items are at most 64*NW - 6 columns wide.  A run frozen by divergence at an
// earlier launch is copied unchanged; grid must be a multiple of 8.
template <typename S, int NW, int PF, bool MRT = false>
__global__ __launch_bounds__(64 * NW) void k_batch_step2(const typename Store<S>::E* __restrict__ src,
                                                         typename Store<S>::E* __restrict__ dst,
                                                         const RunDev* __restrict__ runs,
                                                         const Item* __restrict__ items, int nitems,
                                                         int total,
                                                         const unsigned long long* stepbase,
                                                         unsigned long long steplocal,
                                                         unsigned long long* flags) {
  using R = typename Store<S>::R;
  __shared__ typename Store<S>::P ring1[4][64 * NW];
  __shared__ typename Store<S>::P ring2[4][64 * NW];
  __shared__ R xch[6][64 * NW];
  const unsigned long long step = (stepbase ? *stepbase : 0ull) + steplocal;
  if (total > 0) {  // balanced schedule over whole-strip items (no row cap: no per-row arrays)
    balanced_pieces(items, nitems, total, xcd_remap(blockIdx.x, gridDim.x), 1 << 30,
                    [&](const Item& it, int y, int n) {
                      const RunDev d = runs[it.run];
                      if (flags[it.run] < step)
                        copy_tile<S, 64 * NW>(src + d.off, dst + d.off, d, it.x0, it.y0 + y, it.ncols, n);
                      else
                        tile_step2<S, NW, PF, kBatchSteadyMode, MRT>(src + d.off, dst + d.off, d,
                                                                     it.x0, it.y0 + y, it.ncols, n,
                                                                     step, &flags[it.run], ring1,
                                                                     ring2, xch);
                    });
    return;
  }
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, nb = gridDim.x >> 3;
  const int lo = (int)((int64_t)nitems * xcd / 8), hi = (int)((int64_t)nitems * (xcd + 1) / 8);
  for (int i = lo + slot; i < hi; i += nb) {
    const Item it = items[i];
    const RunDev d = runs[it.run];
    if (flags[it.run] < step)  // frozen run
      copy_tile<S, 64 * NW>(src + d.off, dst + d.off, d, it.x0, it.y0, it.ncols, it.nrows);
    else
      tile_step2<S, NW, PF, kBatchSteadyMode, MRT>(src + d.off, dst + d.off, d, it.x0, it.y0,
                                                   it.ncols, it.nrows, step, &flags[it.run], ring1,
                                                   ring2, xch);
    __syncthreads();  // LDS is reused by the next item
  }
}

// Coexistence densities of flat interfaces with normal x, for every run of a
// batch: out[2r] = mean over y of rho at column nx/2 (liquid), out[2r+1] = the
// same at column 0 (vapour), in FP64 with rho decoded as the step kernels do
// (rho_ref + sum of the pulled populations).  One block per run; per-thread
// partial sums over rows tid, tid+256, ... then a fixed-order tree, so the
// result does not depend on timing.  A diverged run gives NaN.
template <typename S>
__global__ __launch_bounds__(256) void k_batch_coex(const typename Store<S>::E* __restrict__ pool,
                                                    const RunDev* __restrict__ runs,
                                                    const unsigned long long* __restrict__ flags,
                                                    double* __restrict__ out) {
  using R = typename Store<S>::R;
  __shared__ double sl[256], sg[256];
  const int r = blockIdx.x;
  const RunDev d = runs[r];
  const typename Store<S>::E* src = pool + d.off;
  const Cols cl = cols_of(d.nx / 2, d.nx), cg = cols_of(0, d.nx);
  double al = 0.0, ag = 0.0;
  for (int y = threadIdx.x; y < d.ny; y += 256) {
    R f[9];
    pull9<S>(src, d, cl, y, f);
    al += d.rho_ref + double(sum9(f));
    pull9<S>(src, d, cg, y, f);
    ag += d.rho_ref + double(sum9(f));
  }
  sl[threadIdx.x] = al;
  sg[threadIdx.x] = ag;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      sl[threadIdx.x] += sl[threadIdx.x + k];
      sg[threadIdx.x] += sg[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const bool div = flags[r] != ~0ull;
    out[2 * r] = div ? __builtin_nan("") : sl[0] / d.ny;
    out[2 * r + 1] = div ? __builtin_nan("") : sg[0] / d.ny;
  }
}

// Graph helper: advance the device step counter after k steps.
__global__ void k_counter_add(unsigned long long* ctr, unsigned long long k) { *ctr += k; }
__global__ void k_counter_set(unsigned long long* ctr, unsigned long long v) { *ctr = v; }

// ---- diagnostics (rare; simple one-node-per-thread kernels) ---------------

// Pass 1: rho, u = j/rho and psi at every node (rho/ux/uy/psi planes, [y][x]).
// Rows blockIdx.y, blockIdx.y + gridDim.y, ... (the grid's y extent is capped).
template <typename S>
__global__ void k_moments1(const typename Store<S>::E* __restrict__ src, RunDev d, double* rho, double* ux,
                           double* uy, double* psi) {
  using R = typename Store<S>::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= d.nx) return;
  for (int y = blockIdx.y; y < d.ny; y += gridDim.y) {
    R f[9];
    pull9<S>(src, d, cols_of(x, d.nx), y, f);
    const R drho = sum9(f);
    const double r = d.rho_ref + double(drho);
    const int64_t o = (int64_t)y * d.nx + x;
    rho[o] = r;
    ux[o] = double(mom_x(f) / R(r));
    uy[o] = double(mom_y(f) / R(r));
    psi[o] = sqrt(psi2_of(r, d));
  }
}

// Pass 2: v = u + F/(2 rho) (Table I, actual velocity) and p = p_EOS(rho).
__global__ void k_moments2(RunDev d, const double* __restrict__ psi, const double* rho, double* vx,
                           double* vy, double* p) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= d.nx) return;
  const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
  for (int y = blockIdx.y; y < d.ny; y += gridDim.y) {
    const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
    const double* rs = psi + (int64_t)ym * d.nx;
    const double* rc = psi + (int64_t)y * d.nx;
    const double* rn = psi + (int64_t)yp * d.nx;
    const double s[3] = {rs[xm], rs[x], rs[xp]}, c[3] = {rc[xm], rc[x], rc[xp]},
                 n[3] = {rn[xm], rn[x], rn[xp]};
    double Fx, Fy;
    force3x3(s, c, n, 1, d.mG, Fx, Fy);
    const int64_t o = (int64_t)y * d.nx + x;
    const double r = rho[o];
    vx[o] += Fx / (2.0 * r);
    vy[o] += Fy / (2.0 * r);
    p[o] = pressure_of(r, d);
  }
}

// Flat interface with normal x: mean density of each column (fixed order in y).
__global__ void k_colmean(const double* __restrict__ rho, int nx, int ny, double* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  double s = 0.0;
  for (int y = 0; y < ny; ++y) s += rho[(int64_t)y * nx + x];
  out[x] = s / ny;
}

// Normal pressure across the profile (Eq. 25 with alpha = 0, beta = 3, plus the
// improved scheme's 2 G^2 sigma psi'^2 of Eq. 35); psi' and psi'' are central
// differences, periodic in x.
__global__ void k_normal_pressure(const double* __restrict__ rbar, RunDev d, double sigma,
                                  double* __restrict__ pn) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= d.nx) return;
  const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
  const double pm = sqrt(psi2_of(rbar[xm], d)), pc = sqrt(psi2_of(rbar[x], d)),
               pp = sqrt(psi2_of(rbar[xp], d));
  const double d1 = 0.5 * (pp - pm), d2 = (pp - 2.0 * pc) + pm;
  const double G = -d.mG;
  pn[x] = rbar[x] * (1.0 / 3.0) + 0.5 * G * pc * pc + (G / 12.0) * (3.0 * pc * d2) +
          2.0 * G * G * sigma * d1 * d1;
}

// Surface tension of one interface of a periodic flat slab with normal x, from
// the column-mean profile: gamma = (kappa + 2 G^2 sigma) sum_x psi'(x)^2 / 2,
// psi' central differences of psi(rbar) (Eq. 8), kappa = -G/6 (the
// P_b I + kappa grad psi grad psi form of the pressure tensor that Eq. (35)
// modifies, with kappa fixed by the second-order expansion of Eq. 3).  One
// block of 256 threads, fixed summation order.
__global__ __launch_bounds__(256) void k_surface_tension(const double* __restrict__ rbar, RunDev d,
                                                         double sigma, double* __restrict__ out) {
  __shared__ double sm[256];
  double acc = 0.0;
  for (int x = threadIdx.x; x < d.nx; x += 256) {
    const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
    const double d1 = 0.5 * (sqrt(psi2_of(rbar[xp], d)) - sqrt(psi2_of(rbar[xm], d)));
    acc += d1 * d1;
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double G = -d.mG;
    out[0] = (-G / 6.0 + 2.0 * G * G * sigma) * sm[0] * 0.5;
  }
}

// Decode one stored population to FP64 exactly as the host decoder does:
// f = s + (w * rho_ref), two separately rounded operations.
__device__ __forceinline__ double decode(double v, int, double) { return v; }
__device__ __forceinline__ double decode(float v, int a, double rref) {
#pragma clang fp contract(off)
  const double wr = kW[a] * rref;
  return double(v) + wr;
}
__device__ __forceinline__ double decode(__half v, int a, double rref) {
#pragma clang fp contract(off)
  const double wr = kW[a] * rref;
  return double(__half2float(v)) + wr;
}

// Mass: per block, sum of round-to-nearest-even(rho * 2^40) (exact, 128-bit)
// and the FP64 sum; rho = sum_a f_a in direction order of the decoded
// populations.  A thread's int64 sum holds at most ceil(nodes / (blocks * 256))
// terms, 8192 for 2^31 nodes and 1024 blocks, so it cannot overflow for
// densities below 1000; the block sums are 128-bit.
template <typename S>
__global__ __launch_bounds__(256) void k_mass(const typename Store<S>::E* __restrict__ src, RunDev d,
                                              __int128* part_i, double* part_d) {
  __shared__ __int128 si[256];
  __shared__ double sd[256];
  const int64_t n = (int64_t)d.nx * d.ny;
  long long acc_i = 0;
  double acc_d = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    const int y = (int)(k / d.nx), x = (int)(k - (int64_t)y * d.nx);
    const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
    const int64_t P = d.plane;
    const int64_t r0 = (int64_t)y * d.rs, rm = (int64_t)ym * d.rs, rp = (int64_t)yp * d.rs;
    const int64_t idx[9] = {r0 + x,          P + r0 + xm,     2 * P + rm + x,
                            3 * P + r0 + xp, 4 * P + rp + x,  5 * P + rm + xm,
                            6 * P + rm + xp, 7 * P + rp + xp, 8 * P + rp + xm};
    double r = 0.0;
    for (int a = 0; a < 9; ++a)
      if (index_ok(idx[a], d.elems)) r += decode(src[idx[a]], a, d.rho_ref);
    acc_i += __double2ll_rn(r * 1099511627776.0);  // 2^40, exact scaling
    acc_d += r;
  }
  si[threadIdx.x] = acc_i;
  sd[threadIdx.x] = acc_d;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      si[threadIdx.x] += si[threadIdx.x + s];
      sd[threadIdx.x] += sd[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_i[blockIdx.x] = si[0];
    part_d[blockIdx.x] = sd[0];
  }
}

// Final mass sums over the block partials, in block order (one thread):
// out[0], out[1] = low and high 64-bit words of the 128-bit integer sum, out[2]
// = the bits of the FP64 sum.
__global__ void k_mass_final(const __int128* __restrict__ part_i, const double* __restrict__ part_d,
                             int nblocks, unsigned long long* __restrict__ out) {
  __int128 acc = 0;
  double m = 0.0;
  for (int i = 0; i < nblocks; ++i) {
    acc += part_i[i];
    m += part_d[i];
  }
  out[0] = (unsigned long long)acc;
  out[1] = (unsigned long long)(acc >> 64);
  out[2] = __double_as_longlong(m);
}

}  // namespace lbm
