// Host side of the library: contexts, launches, graphs, tile tuning, batch
// runs and the C ABI declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_kernels.hpp"

namespace lbm {
namespace {

constexpr int kEXh[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEYh[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double kWh[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                       1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
constexpr size_t kAlign = 256;
constexpr int kMassBlocks = 1024;
constexpr unsigned long long kNoDiv = ~0ull;

#define HIPCHK(x)                        \
  do {                                   \
    if ((x) != hipSuccess) return LBM_EHIP; \
  } while (0)

// Launch shape of the step kernels: waves per block (strip of 64*nw columns),
// rows per block (0 = balanced schedule over the resident grid), the row
// prefetch depth (1 or 2) and the time steps per launch (1, or 2 for the
// two-step kernel of the single lattice).
struct Tile {
  int nw, L, pf;
  int ts = 1;
};

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
int esize_of(int prec) { return prec == LBM_PREC_F64 ? 8 : prec == LBM_PREC_F16DEV ? 2 : 4; }
using layout::elems_of;
using layout::pitch_of;
using layout::plane_of;
using layout::rs_of;

int validate(const lbm_params& p) {
  if (p.nx < 3 || p.ny < 3) return LBM_EINVAL;
  if ((int64_t)p.nx * p.ny >= (1ll << 31)) return LBM_EINVAL;
  if (!(p.tau > 0.5) || !std::isfinite(p.tau)) return LBM_EINVAL;
  if (!(p.G != 0.0) || !std::isfinite(p.G)) return LBM_EINVAL;
  if (p.eos != LBM_EOS_CS && p.eos != LBM_EOS_PR) return LBM_EINVAL;
  if (p.scheme < LBM_SCHEME_SHANCHEN || p.scheme > LBM_SCHEME_LADD) return LBM_EINVAL;
  if (p.precision < LBM_PREC_F64 || p.precision > LBM_PREC_F32DEV_F64) return LBM_EINVAL;
  if (!(p.a > 0) || !(p.b > 0) || !(p.R > 0) || !(p.T > 0)) return LBM_EINVAL;
  if (!std::isfinite(p.sigma)) return LBM_EINVAL;
  return LBM_OK;
}

double host_psi2(const EosConst& k, double rho) { return (pressure(k, rho) - rho / 3.0) * k.two_over_G; }

// Host equilibrium, Eq. (2) with c_s^2 = 1/3.
void host_feq(double rho, double ux, double uy, double* f) {
  const double usq = ux * ux + uy * uy;
  for (int a = 0; a < 9; ++a) {
    const double eu = kEXh[a] * ux + kEYh[a] * uy;
    f[a] = kWh[a] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
  }
}

// Fill the device-side constants of one lattice.
RunDev make_rundev(const lbm_params& p, const EosConst& k, double rho_ref, int64_t off, int run) {
  RunDev d{};
  d.nx = p.nx;
  d.ny = p.ny;
  d.pitch = pitch_of(p.nx);
  d.eos = p.eos;
  d.plane = plane_of(p.nx);
  d.rs = rs_of(p.nx);
  d.elems = elems_of(p.nx, p.ny);
  d.off = off;
  d.RT = k.RT;
  d.c1 = k.c1;
  d.c2 = k.c2;
  d.two_over_G = k.two_over_G;
  d.mG = -p.G;
  d.inv_tau = 1.0 / p.tau;
  switch (p.scheme) {
    case LBM_SCHEME_SHANCHEN:  // Eqs. (9)-(10): u_eq = u + tau F/rho, no forcing term
      d.c_eq = p.tau;
      d.c_f = 0.0;
      d.sig = 0.0;
      d.Be = d.Ce = 0.0;
      break;
    case LBM_SCHEME_EDM:  // Eq. (11) = Eq. (16): B_e = C_e = 1, velocity u + F/(2 rho)
      d.c_eq = 0.0;
      d.c_f = 0.5;
      d.sig = 0.0;
      d.Be = d.Ce = 1.0;
      break;
    case LBM_SCHEME_EDM_MODIFIED:  // Sec. III.C: EDM with C_e = 1/tau
      d.c_eq = 0.0;
      d.c_f = 0.5;
      d.sig = 0.0;
      d.Be = 1.0;
      d.Ce = 1.0 / p.tau;
      break;
    case LBM_SCHEME_LADD:  // Table I: u in the equilibrium and in F_a, B_e = C_e = 1
      d.c_eq = 0.0;
      d.c_f = 0.0;
      d.sig = 0.0;
      d.Be = d.Ce = 1.0;
      break;
    default:  // Eq. (31): u_eq = v, B_e = C_e = 1 - 1/(2 tau), v' = v + sigma F/((tau - 1/2) psi^2)
      d.c_eq = 0.5;
      d.c_f = 0.5;
      d.sig = p.sigma / (p.tau - 0.5);
      d.Be = d.Ce = 1.0 - 0.5 / p.tau;
      break;
  }
  d.wCe0 = 4.0 / 9.0 * d.Ce;
  d.wCe1 = 1.0 / 9.0 * d.Ce;
  d.wCe2 = 1.0 / 36.0 * d.Ce;
  d.wBe3_1 = 3.0 / 9.0 * d.Be;
  d.wBe3_2 = 3.0 / 36.0 * d.Be;
  d.om_w0 = 4.0 / 9.0 * d.inv_tau;
  d.om_w1 = 1.0 / 9.0 * d.inv_tau;
  d.om_w2 = 1.0 / 36.0 * d.inv_tau;
  d.om_3w1 = 3.0 / 9.0 * d.inv_tau;
  d.om_3w2 = 3.0 / 36.0 * d.inv_tau;
  d.om1 = 1.0 - d.inv_tau;
  d.rho_ref = rho_ref;
  d.run = run;
  d.mrt = 0;
  d.s_e = d.s_eps = d.s_q = d.inv_tau;
  d.sig_e = d.sig_eps = d.sig;
  return d;
}

// Switch a lattice's constants to the MRT collision with energy, energy-square
// and energy-flux rates r[0..2] (the density, momentum and stress moments relax
// at 1/tau): sigma / (1/s - 1/2) of the improved scheme per moment.
void set_mrt(RunDev& d, const lbm_params& p, const double* r) {
  d.mrt = 1;
  d.s_e = r[0];
  d.s_eps = r[1];
  d.s_q = r[2];
  d.sig_e = p.sigma / (1.0 / r[0] - 0.5);
  d.sig_eps = p.sigma / (1.0 / r[1] - 0.5);
}

// Encode FP64 populations into the storage buffer (layout::encode): FP64 as
// is, deviations f - w rho_ref rounded to FP32 (and then to FP16).
template <typename S>
void encode_buffer(const lbm_params& p, double rref, const double* f, std::vector<char>& out) {
  out.assign(elems_of(p.nx, p.ny) * sizeof(S), 0);
  S* b = reinterpret_cast<S*>(out.data());
  layout::encode(p.nx, p.ny, f, b, [&](int a, double v) -> S {
    if constexpr (std::is_same<S, double>::value)
      return v;
    else if constexpr (std::is_same<S, float>::value)
      return (float)(v - kWh[a] * rref);
    else  // RNE to FP32, then RNE to FP16
      return __float2half_rn((float)(v - kWh[a] * rref));
  });
}

// Decode the storage buffer to FP64 populations: f = s + (w rho_ref), two
// separately rounded operations (as the device decoder of the mass does).
template <typename S>
void decode_buffer(const lbm_params& p, double rref, const char* raw, double* f) {
  const S* b = reinterpret_cast<const S*>(raw);
  layout::decode(p.nx, p.ny, b, f, [&](int a, S v) -> double {
    if constexpr (std::is_same<S, double>::value) {
      return v;
    } else {
      volatile double wr = kWh[a] * rref;  // keep the two roundings separate
      if constexpr (std::is_same<S, float>::value)
        return (double)v + wr;
      else
        return (double)__half2float(v) + wr;
    }
  });
}

void encode_any(int prec, const lbm_params& p, double rref, const double* f, std::vector<char>& o) {
  if (prec == LBM_PREC_F64) encode_buffer<double>(p, rref, f, o);
  else if (prec == LBM_PREC_F16DEV) encode_buffer<__half>(p, rref, f, o);
  else encode_buffer<float>(p, rref, f, o);
}
void decode_any(int prec, const lbm_params& p, double rref, const char* raw, double* f) {
  if (prec == LBM_PREC_F64) decode_buffer<double>(p, rref, raw, f);
  else if (prec == LBM_PREC_F16DEV) decode_buffer<__half>(p, rref, raw, f);
  else decode_buffer<float>(p, rref, raw, f);
}

// ---- launches ---------------------------------------------------------------

// Resident blocks per CU times the CU count for one kernel (cached per kernel).
int resident_blocks(const void* fn, int threads) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(fn);
  if (it != cache.end()) return it->second;
  int dev = 0, ncu = 256, occ = 1;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, threads, 0) != hipSuccess || occ < 1)
    occ = 1;
  return cache[fn] = ncu * occ;
}

template <typename S, int NW, int PF, bool MRT>
hipError_t launch_step_t(const void* src, void* dst, const RunDev& d, int L,
                         const unsigned long long* base, unsigned long long local,
                         unsigned long long* flag, hipStream_t st) {
  const int SW = 64 * NW;
  const int nstrips = (d.nx + SW - 1) / SW;
  int grid;
  if (L > 0) {
    grid = nstrips * ((d.ny + L - 1) / L);
  } else {  // balanced: resident capacity, at least 8 rows per block
    const int64_t rows = (int64_t)nstrips * d.ny;
    grid = resident_blocks((const void*)k_step<S, NW, PF, MRT>, SW);
    grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, rows / 8));
  }
  using E = typename Store<S>::E;
  hipLaunchKernelGGL((k_step<S, NW, PF, MRT>), dim3(grid), dim3(SW), 0, st, static_cast<const E*>(src),
                     static_cast<E*>(dst), d, L, nstrips, base, local, flag);
  return hipGetLastError();
}

template <typename S, bool MRT = false>
hipError_t launch_step_s(const Tile& t, const void* src, void* dst, const RunDev& d,
                         const unsigned long long* base, unsigned long long local,
                         unsigned long long* flag, hipStream_t st) {
  switch (t.nw * 10 + t.pf) {
    case 11: return launch_step_t<S, 1, 1, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 12: return launch_step_t<S, 1, 2, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 21: return launch_step_t<S, 2, 1, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 22: return launch_step_t<S, 2, 2, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 41: return launch_step_t<S, 4, 1, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 42: return launch_step_t<S, 4, 2, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 81: return launch_step_t<S, 8, 1, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 82: return launch_step_t<S, 8, 2, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 161: return launch_step_t<S, 16, 1, MRT>(src, dst, d, t.L, base, local, flag, st);
    default: return launch_step_t<S, 16, 2, MRT>(src, dst, d, t.L, base, local, flag, st);
  }
}

template <typename S, int NW, int PF, bool MRT = false>
hipError_t launch_step2_t(const void* src, void* dst, const RunDev& d, int L,
                          const unsigned long long* base, unsigned long long local,
                          unsigned long long* flag, hipStream_t st) {
  const int SW = 64 * NW;
  // strips of at most SW - 6 columns after their edges are aligned down to A columns
  constexpr int A = Step2Align<S>::value;
  const int nstrips = (d.nx + SW - 7 - (A - 1)) / (SW - 6 - (A - 1));
  int grid;
  if (L > 0) {
    grid = nstrips * ((d.ny + L - 1) / L);
  } else {
    const int64_t rows = (int64_t)nstrips * d.ny;
    grid = resident_blocks((const void*)k_step2<S, NW, PF, MRT>, SW);
    grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, rows / 8));
  }
  using E = typename Store<S>::E;
  hipLaunchKernelGGL((k_step2<S, NW, PF, MRT>), dim3(grid), dim3(SW), 0, st,
                     static_cast<const E*>(src), static_cast<E*>(dst), d, L, nstrips, base, local, flag);
  return hipGetLastError();
}

template <typename S, bool MRT = false>
hipError_t launch_step2_s(const Tile& t, const void* src, void* dst, const RunDev& d,
                          const unsigned long long* base, unsigned long long local,
                          unsigned long long* flag, hipStream_t st) {
  switch (t.nw * 10 + t.pf) {
    case 41: return launch_step2_t<S, 4, 1, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 42: return launch_step2_t<S, 4, 2, MRT>(src, dst, d, t.L, base, local, flag, st);
    case 81: return launch_step2_t<S, 8, 1, MRT>(src, dst, d, t.L, base, local, flag, st);
    default: return launch_step2_t<S, 8, 2, MRT>(src, dst, d, t.L, base, local, flag, st);
  }
}

template <typename S, int NW, bool MRT = false>
hipError_t launch_step3_t(const void* src, void* dst, const RunDev& d, int L,
                          const unsigned long long* base, unsigned long long local,
                          unsigned long long* flag, hipStream_t st) {
  const int SW = 64 * NW;
  // strips of at most SW - 10 columns after their edges are aligned down to A columns
  constexpr int A = Step2Align<S>::value;
  const int nstrips = (d.nx + SW - 11 - (A - 1)) / (SW - 10 - (A - 1));
  int grid;
  if (L > 0) {
    grid = nstrips * ((d.ny + L - 1) / L);
  } else {
    const int64_t rows = (int64_t)nstrips * d.ny;
    grid = resident_blocks((const void*)k_step3<S, NW, MRT>, SW);
    grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, rows / 8));
  }
  using E = typename Store<S>::E;
  hipLaunchKernelGGL((k_step3<S, NW, MRT>), dim3(grid), dim3(SW), 0, st, static_cast<const E*>(src),
                     static_cast<E*>(dst), d, L, nstrips, base, local, flag);
  return hipGetLastError();
}

// Storage types with a three-step kernel: those with FP64 collision arithmetic
// (the FP32 and FP16 arithmetic paths are bound by instruction issue, where
// the recomputed halo of a third step costs more than the traffic it saves).
bool has_step3(int prec) { return prec == LBM_PREC_F64 || prec == LBM_PREC_F32DEV_F64; }

// One launch of the tile: t.ts time steps (1, 2 or 3) from src into dst.
hipError_t launch_step(int prec, const Tile& t, const void* src, void* dst, const RunDev& d,
                       const unsigned long long* base, unsigned long long local,
                       unsigned long long* flag, hipStream_t st) {
  if (t.ts == 3 && d.mrt)  // FP64 only: the one precision with both MRT and three steps
    return t.nw == 8 ? launch_step3_t<double, 8, true>(src, dst, d, t.L, base, local, flag, st)
                     : launch_step3_t<double, 4, true>(src, dst, d, t.L, base, local, flag, st);
  if (t.ts == 3) {
    if (prec == LBM_PREC_F64)
      return t.nw == 8 ? launch_step3_t<double, 8>(src, dst, d, t.L, base, local, flag, st)
                       : launch_step3_t<double, 4>(src, dst, d, t.L, base, local, flag, st);
    if (prec == LBM_PREC_F32DEV_F64)
      return t.nw == 8 ? launch_step3_t<f32s_f64a, 8>(src, dst, d, t.L, base, local, flag, st)
                       : launch_step3_t<f32s_f64a, 4>(src, dst, d, t.L, base, local, flag, st);
    return hipErrorInvalidValue;
  }
  if (t.ts == 2 && d.mrt) {  // FP64 or FP32 deviation storage (checked by lbm_set_mrt)
    if (prec == LBM_PREC_F64) return launch_step2_s<double, true>(t, src, dst, d, base, local, flag, st);
    return launch_step2_s<float, true>(t, src, dst, d, base, local, flag, st);
  }
  if (t.ts == 2) {
    if (prec == LBM_PREC_F64) return launch_step2_s<double>(t, src, dst, d, base, local, flag, st);
    if (prec == LBM_PREC_F32DEV) return launch_step2_s<float>(t, src, dst, d, base, local, flag, st);
    if (prec == LBM_PREC_F32DEV_F64)
      return launch_step2_s<f32s_f64a>(t, src, dst, d, base, local, flag, st);
    return launch_step2_s<__half>(t, src, dst, d, base, local, flag, st);
  }
  if (d.mrt) {  // one step per launch; FP64 or FP32 deviation storage (checked by lbm_set_mrt)
    if (prec == LBM_PREC_F64) return launch_step_s<double, true>(t, src, dst, d, base, local, flag, st);
    return launch_step_s<float, true>(t, src, dst, d, base, local, flag, st);
  }
  if (prec == LBM_PREC_F64) return launch_step_s<double>(t, src, dst, d, base, local, flag, st);
  if (prec == LBM_PREC_F32DEV) return launch_step_s<float>(t, src, dst, d, base, local, flag, st);
  if (prec == LBM_PREC_F32DEV_F64) return launch_step_s<f32s_f64a>(t, src, dst, d, base, local, flag, st);
  return launch_step_s<__half>(t, src, dst, d, base, local, flag, st);
}

// Grid of a batch launch: item lists take at most one block per item (a
// multiple of 8, one eighth of the list per XCD); the balanced schedule
// (total > 0 rows) the resident capacity, at least 8 rows per block.
int batch_grid(const void* fn, int threads, int nitems, int total) {
  int g = resident_blocks(fn, threads);
  if (total > 0) return (int)std::max<int64_t>(1, std::min<int64_t>(g, total / 8));
  g = std::min(g, (nitems + 7) / 8 * 8);
  return std::max(8, g / 8 * 8);
}

template <typename S, int NW, int PF, bool MRT>
hipError_t launch_batch_t(const void* src, void* dst, const RunDev* runs, const Item* items,
                          int nitems, int total, const unsigned long long* base,
                          unsigned long long local, unsigned long long* flags, hipStream_t st) {
  const int g = batch_grid((const void*)k_batch_step<S, NW, PF, MRT>, 64 * NW, nitems, total);
  using E = typename Store<S>::E;
  hipLaunchKernelGGL((k_batch_step<S, NW, PF, MRT>), dim3(g), dim3(64 * NW), 0, st,
                     static_cast<const E*>(src), static_cast<E*>(dst), runs, items, nitems, total,
                     base, local, flags);
  return hipGetLastError();
}

template <typename S, bool MRT = false>
hipError_t launch_batch_s(const Tile& t, const void* src, void* dst, const RunDev* runs,
                          const Item* items, int nitems, int total, const unsigned long long* base,
                          unsigned long long local, unsigned long long* flags, hipStream_t st) {
  switch (t.nw * 10 + t.pf) {
    case 11: return launch_batch_t<S, 1, 1, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 12: return launch_batch_t<S, 1, 2, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 21: return launch_batch_t<S, 2, 1, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 22: return launch_batch_t<S, 2, 2, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 41: return launch_batch_t<S, 4, 1, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 42: return launch_batch_t<S, 4, 2, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 81: return launch_batch_t<S, 8, 1, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    default: return launch_batch_t<S, 8, 2, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
  }
}

template <typename S, int NW, int PF, bool MRT>
hipError_t launch_batch2_t(const void* src, void* dst, const RunDev* runs, const Item* items,
                           int nitems, int total, const unsigned long long* base,
                           unsigned long long local, unsigned long long* flags, hipStream_t st) {
  const int g = batch_grid((const void*)k_batch_step2<S, NW, PF, MRT>, 64 * NW, nitems, total);
  using E = typename Store<S>::E;
  hipLaunchKernelGGL((k_batch_step2<S, NW, PF, MRT>), dim3(g), dim3(64 * NW), 0, st,
                     static_cast<const E*>(src), static_cast<E*>(dst), runs, items, nitems, total,
                     base, local, flags);
  return hipGetLastError();
}

template <typename S, bool MRT = false>
hipError_t launch_batch2_s(const Tile& t, const void* src, void* dst, const RunDev* runs,
                           const Item* items, int nitems, int total, const unsigned long long* base,
                           unsigned long long local, unsigned long long* flags, hipStream_t st) {
  switch (t.nw * 10 + t.pf) {
    case 21: return launch_batch2_t<S, 2, 1, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 22: return launch_batch2_t<S, 2, 2, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 41: return launch_batch2_t<S, 4, 1, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 42: return launch_batch2_t<S, 4, 2, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    case 81: return launch_batch2_t<S, 8, 1, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
    default: return launch_batch2_t<S, 8, 2, MRT>(src, dst, runs, items, nitems, total, base, local, flags, st);
  }
}

// One launch of the batch tile: t.ts time steps (1 or 2) of every active run;
// mrt: the runs' descriptors carry the MRT collision (FP64 or FP32 deviation
// storage, checked by lbm_batch_set_mrt).
hipError_t launch_batch(int prec, bool mrt, const Tile& t, const void* src, void* dst,
                        const RunDev* runs, const Item* items, int nitems, int total,
                        const unsigned long long* base, unsigned long long local,
                        unsigned long long* flags, hipStream_t st) {
  if (mrt) {
    if (t.ts == 2) {
      if (prec == LBM_PREC_F64)
        return launch_batch2_s<double, true>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
      return launch_batch2_s<float, true>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
    }
    if (prec == LBM_PREC_F64)
      return launch_batch_s<double, true>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
    return launch_batch_s<float, true>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
  }
  if (t.ts == 2) {
    if (prec == LBM_PREC_F64)
      return launch_batch2_s<double>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
    if (prec == LBM_PREC_F32DEV)
      return launch_batch2_s<float>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
    if (prec == LBM_PREC_F32DEV_F64)
      return launch_batch2_s<f32s_f64a>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
    return launch_batch2_s<__half>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
  }
  if (prec == LBM_PREC_F64)
    return launch_batch_s<double>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
  if (prec == LBM_PREC_F32DEV)
    return launch_batch_s<float>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
  if (prec == LBM_PREC_F32DEV_F64)
    return launch_batch_s<f32s_f64a>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
  return launch_batch_s<__half>(t, src, dst, runs, items, nitems, total, base, local, flags, st);
}

template <typename S>
hipError_t launch_moments_s(const void* src, const RunDev& d, double* rho, double* vx, double* vy,
                            double* p, double* psi, hipStream_t st) {
  // rows beyond the grid's y extent (at most 65535 here) are looped in the kernels
  dim3 blk(64), grd((d.nx + 63) / 64, std::min(d.ny, 65535));
  hipLaunchKernelGGL(k_moments1<S>, grd, blk, 0, st, static_cast<const typename Store<S>::E*>(src), d, rho,
                     vx, vy, psi);
  hipLaunchKernelGGL(k_moments2, grd, blk, 0, st, d, (const double*)psi, (const double*)rho, vx, vy, p);
  return hipGetLastError();
}

hipError_t launch_moments(int prec, const void* src, const RunDev& d, double* rho, double* vx,
                          double* vy, double* p, double* psi, hipStream_t st) {
  if (prec == LBM_PREC_F64) return launch_moments_s<double>(src, d, rho, vx, vy, p, psi, st);
  if (prec == LBM_PREC_F32DEV) return launch_moments_s<float>(src, d, rho, vx, vy, p, psi, st);
  if (prec == LBM_PREC_F32DEV_F64) return launch_moments_s<f32s_f64a>(src, d, rho, vx, vy, p, psi, st);
  return launch_moments_s<__half>(src, d, rho, vx, vy, p, psi, st);
}

// Mass partials of kMassBlocks work-groups into part_i/part_d, then the final
// sums into out[0..2] (see k_mass_final).
hipError_t launch_mass(int prec, const void* src, const RunDev& d, __int128* pi, double* pd,
                       unsigned long long* out, hipStream_t st) {
  if (prec == LBM_PREC_F64)
    hipLaunchKernelGGL(k_mass<double>, dim3(kMassBlocks), dim3(256), 0, st, (const double*)src, d, pi, pd);
  else if (prec == LBM_PREC_F32DEV)
    hipLaunchKernelGGL(k_mass<float>, dim3(kMassBlocks), dim3(256), 0, st, (const float*)src, d, pi, pd);
  else if (prec == LBM_PREC_F32DEV_F64)
    hipLaunchKernelGGL(k_mass<f32s_f64a>, dim3(kMassBlocks), dim3(256), 0, st, (const float*)src, d, pi, pd);
  else
    hipLaunchKernelGGL(k_mass<__half>, dim3(kMassBlocks), dim3(256), 0, st, (const __half*)src, d, pi, pd);
  hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(1), 0, st, (const __int128*)pi, (const double*)pd,
                     kMassBlocks, out);
  return hipGetLastError();
}

// Bytes of mass scratch: 128-bit and FP64 partials per work-group, then the
// three result words.
constexpr size_t kMassScratch = kMassBlocks * (sizeof(__int128) + sizeof(double)) + 4 * sizeof(unsigned long long);

}  // namespace
}  // namespace lbm

// Device scratch of lbm_mass_noalloc (the mass partials and result words,
// kMassScratch = 24,608 bytes), one copy per GPU, held until the process ends.
// Host code never uses this name as an address: it uses the per-device
// pointer hipGetSymbolAddress returned for it.
static __device__ __align__(256) unsigned char scratch[lbm::kMassScratch];

namespace lbm {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` per device (null until set up)

// The current device's address of `scratch`, looked up on the first call on
// that device (with it current) and kept.
hipError_t scratch_of_current_device(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = static_cast<char*>(g_scratch[dev]);
  return hipSuccess;
}

hipError_t launch_batch_coex(int prec, const void* pool, const RunDev* runs, int nruns,
                             const unsigned long long* flags, double* out, hipStream_t st) {
  const dim3 g(nruns), b(256);
  if (prec == LBM_PREC_F64)
    hipLaunchKernelGGL(k_batch_coex<double>, g, b, 0, st, (const double*)pool, runs, flags, out);
  else if (prec == LBM_PREC_F32DEV)
    hipLaunchKernelGGL(k_batch_coex<float>, g, b, 0, st, (const float*)pool, runs, flags, out);
  else if (prec == LBM_PREC_F32DEV_F64)
    hipLaunchKernelGGL(k_batch_coex<f32s_f64a>, g, b, 0, st, (const float*)pool, runs, flags, out);
  else
    hipLaunchKernelGGL(k_batch_coex<__half>, g, b, 0, st, (const __half*)pool, runs, flags, out);
  return hipGetLastError();
}

// ---- tile heuristics and tuning cache -----------------------------------------

Tile default_tile(int nx, int ny) {
  Tile t{nx >= 1024 ? 4 : nx >= 256 ? 2 : 1, 0, 2};
  const int SW = 64 * t.nw;
  const int64_t rows = (int64_t)((nx + SW - 1) / SW) * ny;
  if (rows < 8 * 1024) {  // small lattices: short chunks give more blocks
    int l = 64;
    while (l > 4 && ((nx + SW - 1) / SW) * ((ny + l - 1) / l) < 1024) l /= 2;
    t.L = std::min(l, std::max(1, ny));
  }
  return t;
}

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, Tile> g_tune;

}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm_ctx {
  lbm_params p;
  EosConst k;
  RunDev d;
  int esize;
  size_t pop_bytes, raw_bytes;
  char* ws;
  size_t ws_bytes;
  void* buf[2];
  int cur;
  double* aux;  // 5 planes of nx*ny doubles: rho, vx, vy, p, psi
  __int128* part_i;   // mass scratch: partials and the result words
  double* part_d;
  unsigned long long* mass_out;
  unsigned long long* flag;
  unsigned long long* ctr;
  hipStream_t st;
  int64_t step;
  Tile tile;
  int graph_k;
  hipGraphExec_t gexec[2];
  Tile gtile;
  int64_t captures;  // graphs captured so far
};

namespace {

size_t raw_bytes_of(const lbm_params& p) {
  const int es = esize_of(p.precision);
  return (size_t)elems_of(p.nx, p.ny) * es;
}

size_t ctx_layout(const lbm_params& p, size_t* pop, size_t* aux, size_t* parts, size_t* misc) {
  *pop = align_up(raw_bytes_of(p));
  *aux = align_up(5 * (size_t)p.nx * p.ny * sizeof(double));
  *parts = align_up(kMassScratch);
  *misc = align_up(2 * sizeof(unsigned long long));
  return 2 * *pop + *aux + *parts + *misc;
}

bool same_tile(const Tile& a, const Tile& b) {
  return a.nw == b.nw && a.L == b.L && a.pf == b.pf && a.ts == b.ts;
}

// Strip widths of the single-lattice kernel (64 to 1024 columns) and of the
// batched one (64 to 512 columns; batched lattices are at most a few hundred
// columns wide).
constexpr int kStepWaves[] = {1, 2, 4, 8, 16};
constexpr int kBatchWaves[] = {1, 2, 4, 8};
constexpr int kStep2Waves[] = {4, 8};  // two-step kernel: 250- and 506-column strips
// The batched two-step kernel also has 2-wave blocks (122-column strips): the
// lattices of a sweep are 64 to 512 columns wide, and a 250-column strip of a
// narrow one leaves most lanes of its block idle.
constexpr int kBatchStep2Waves[] = {2, 4, 8};

// A launch shape; ts2_min_nw is the smallest wave count of the two-step kernel
// (2 for the batched launch, 4 for a single lattice).
// The three-step kernel (single lattice only) has 4- and 8-wave blocks and
// row prefetch depth 1.
bool valid_tile(int nw, int L, int pf, int maxnw, int ts = 1, int ts2_min_nw = 4) {
  if (ts == 2 && (nw < ts2_min_nw || (nw != 2 && nw != 4 && nw != 8))) return false;
  if (ts == 3 && (ts2_min_nw != 4 || (nw != 4 && nw != 8) || pf != 1)) return false;
  return (nw == 1 || nw == 2 || nw == 4 || nw == 8 || nw == 16) && nw <= maxnw && L >= 0 &&
         L <= LMAX && (pf == 1 || pf == 2) && ts >= 1 && ts <= 3;
}

// A remainder of r < t.ts steps of a multi-step tile: one launch of r steps
// (the two-step kernel for two, with the same waves, rows and depth, which
// every three-step tile also suits).
Tile remainder_tile(Tile t, int r) {
  t.ts = r;
  return t;
}

// Launches in a graph of k steps: k / ts full launches and one for the remainder.
int graph_launches(int k, int ts) { return k / ts + (k % ts != 0 ? 1 : 0); }

void drop_graphs(lbm_ctx* c) {
  for (int i = 0; i < 2; ++i)
    if (c->gexec[i]) {
      (void)hipGraphExecDestroy(c->gexec[i]);
      c->gexec[i] = nullptr;
    }
}

int upload_state(lbm_ctx* c, const std::vector<char>& raw, int64_t step) {
  HIPCHK(hipMemcpyAsync(c->buf[0], raw.data(), raw.size(), hipMemcpyHostToDevice, c->st));
  c->cur = 0;
  c->step = step;
  hipLaunchKernelGGL(k_counter_set, dim3(1), dim3(1), 0, c->st, c->flag, kNoDiv);
  hipLaunchKernelGGL(k_counter_set, dim3(1), dim3(1), 0, c->st, c->ctr, (unsigned long long)step);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return LBM_OK;
}

int capture_graph(lbm_ctx* c, int parity) {
  hipGraph_t g;
  HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  const int full = c->graph_k / c->tile.ts, rest = c->graph_k % c->tile.ts;
  for (int i = 0; i < graph_launches(c->graph_k, c->tile.ts) && e == hipSuccess; ++i) {
    const int s = (parity + i) & 1;
    const Tile t = i < full ? c->tile : remainder_tile(c->tile, rest);
    e = launch_step(c->p.precision, t, c->buf[s], c->buf[s ^ 1], c->d, c->ctr,
                    (unsigned long long)i * c->tile.ts, c->flag, c->st);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_counter_add, dim3(1), dim3(1), 0, c->st, c->ctr,
                       (unsigned long long)c->graph_k);
    e = hipGetLastError();
  }
  hipError_t e2 = hipStreamEndCapture(c->st, &g);
  if (e != hipSuccess || e2 != hipSuccess) return LBM_EHIP;
  e = hipGraphInstantiate(&c->gexec[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e == hipSuccess) e = hipGraphUpload(c->gexec[parity], c->st);
  if (e != hipSuccess) {
    if (c->gexec[parity]) (void)hipGraphExecDestroy(c->gexec[parity]);
    c->gexec[parity] = nullptr;
    return LBM_EHIP;
  }
  c->gtile = c->tile;
  ++c->captures;
  return LBM_OK;
}

// Capture (or re-capture after a tile change) the graphs of both buffer
// parities now, so that no later lbm_step call pays for a capture.
int prepare_graphs(lbm_ctx* c) {
  if (c->graph_k <= 0) return LBM_OK;
  if (!same_tile(c->gtile, c->tile)) drop_graphs(c);
  for (int parity = 0; parity < 2; ++parity)
    if (!c->gexec[parity]) {
      int st = capture_graph(c, parity);
      if (st != LBM_OK) return st;
    }
  HIPCHK(hipStreamSynchronize(c->st));
  return LBM_OK;
}

// Time `reps` launches of one candidate tile (reads the current buffer, writes
// the other, so the state does not advance).  Returns ms or a negative value.
template <class Launch>
float time_launches(hipStream_t st, Launch&& launch, int reps) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.f;
  }
  hipError_t e = hipSuccess;
  for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = -1.f;
  if (e == hipSuccess && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = -1.f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e == hipSuccess ? ms : -1.f;
}

// Pick the fastest tile per lattice step (tuning::pick_best); time_one(t)
// returns ms per lattice step, negative on a HIP error, +inf to skip the tile.
// Returns LBM_OK (best_tile unchanged if every tile was skipped) or LBM_EHIP.
template <class TimeOne>
int pick_tile(const std::vector<Tile>& cand, TimeOne&& time_one, Tile& best_tile) {
  const int k = tuning::pick_best((int)cand.size(), [&](int i) { return time_one(cand[i]); });
  if (k == -2) return LBM_EHIP;
  if (k >= 0) best_tile = cand[k];
  return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_strerror(int s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_EPSI: return "density outside the equation-of-state range (2(p - rho/3)/G <= 0)";
    case LBM_EDIVERGED: return "the run diverged";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ENOSPACE: return "workspace too small";
    case LBM_ENOTSUP: return "not supported";
    default: return "unknown error";
  }
}

int lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
  if (!p || !bytes) return LBM_EINVAL;
  int st = validate(*p);
  if (st != LBM_OK) return st;
  size_t a, b, c2, d2;
  *bytes = ctx_layout(*p, &a, &b, &c2, &d2);
  return LBM_OK;
}

int lbm_init(const lbm_params* p, const double* rho0, const double* ux0, const double* uy0,
             void* ws, size_t ws_bytes, void* stream, lbm_ctx** out) {
  if (!p || !rho0 || !ws || !out) return LBM_EINVAL;
  *out = nullptr;
  int st = validate(*p);
  if (st != LBM_OK) return st;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return LBM_EINVAL;
  size_t pop, aux, parts, misc;
  const size_t need = ctx_layout(*p, &pop, &aux, &parts, &misc);
  if (ws_bytes < need) return LBM_ENOSPACE;
  EosConst k;
  st = eos_constants(*p, &k);
  if (st != LBM_OK) return st;
  const size_t n = (size_t)p->nx * p->ny;
  double mean = 0.0;
  for (size_t i = 0; i < n; ++i) {
    if (!(rho0[i] > 0) || !(host_psi2(k, rho0[i]) > 0)) return LBM_EPSI;
    mean += rho0[i];
  }
  mean /= (double)n;
  double rref = 0.0;
  if (p->precision != LBM_PREC_F64) rref = std::isnan(p->rho_ref) ? mean : p->rho_ref;
  std::vector<double> f(9 * n);
  for (size_t i = 0; i < n; ++i) {
    double fe[9];
    host_feq(rho0[i], ux0 ? ux0[i] : 0.0, uy0 ? uy0[i] : 0.0, fe);
    for (int a = 0; a < 9; ++a) f[a * n + i] = fe[a];
  }
  lbm_ctx* c = new lbm_ctx{};
  c->p = *p;
  c->p.rho_ref = rref;
  c->k = k;
  c->d = make_rundev(*p, k, rref, 0, 0);
  c->esize = esize_of(p->precision);
  c->pop_bytes = pop;
  c->raw_bytes = raw_bytes_of(*p);
  c->ws = static_cast<char*>(ws);
  c->ws_bytes = ws_bytes;
  c->buf[0] = c->ws;
  c->buf[1] = c->ws + pop;
  c->aux = reinterpret_cast<double*>(c->ws + 2 * pop);
  c->part_i = reinterpret_cast<__int128*>(c->ws + 2 * pop + aux);
  c->part_d = reinterpret_cast<double*>(c->part_i + kMassBlocks);
  c->mass_out = reinterpret_cast<unsigned long long*>(c->part_d + kMassBlocks);
  c->flag = reinterpret_cast<unsigned long long*>(c->ws + 2 * pop + aux + parts);
  c->ctr = c->flag + 1;
  c->st = static_cast<hipStream_t>(stream);
  c->tile = default_tile(p->nx, p->ny);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({p->nx, p->ny, p->precision, 0});
    if (it != g_tune.end()) c->tile = it->second;
  }
  // the second buffer is written only at lattice nodes: clear its row padding once
  // so that checkpoints of either buffer are deterministic
  if (hipMemsetAsync(c->buf[1], 0, c->raw_bytes, c->st) != hipSuccess) {
    delete c;
    return LBM_EHIP;
  }
  std::vector<char> raw;
  encode_any(p->precision, c->p, rref, f.data(), raw);
  st = upload_state(c, raw, 0);
  if (st != LBM_OK) {
    delete c;
    return st;
  }
  *out = c;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) {
  if (!c || n < 0) return LBM_EINVAL;
  int64_t done = 0;
  if (c->graph_k > 0 && n >= c->graph_k) {
    if (!same_tile(c->gtile, c->tile)) drop_graphs(c);
    hipLaunchKernelGGL(k_counter_set, dim3(1), dim3(1), 0, c->st, c->ctr, (unsigned long long)c->step);
    HIPCHK(hipGetLastError());
    while (n - done >= c->graph_k) {
      if (!c->gexec[c->cur]) {
        int st = capture_graph(c, c->cur);
        if (st != LBM_OK) return st;
      }
      HIPCHK(hipGraphLaunch(c->gexec[c->cur], c->st));
      done += c->graph_k;
      c->step += c->graph_k;
      c->cur ^= graph_launches(c->graph_k, c->tile.ts) & 1;  // one buffer swap per launch
    }
  }
  while (done < n) {
    const int s = c->cur;
    Tile t = c->tile;
    if (n - done < t.ts) t = remainder_tile(t, (int)(n - done));  // fewer steps than the tile's
    HIPCHK(launch_step(c->p.precision, t, c->buf[s], c->buf[s ^ 1], c->d, nullptr,
                       (unsigned long long)c->step, c->flag, c->st));
    c->cur ^= 1;
    c->step += t.ts;
    done += t.ts;
  }
  return LBM_OK;
}

int lbm_status(lbm_ctx* c, int64_t* step, int64_t* diverged_at) {
  if (!c) return LBM_EINVAL;
  unsigned long long f = 0;
  HIPCHK(hipMemcpyAsync(&f, c->flag, sizeof f, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (step) *step = c->step;
  if (diverged_at) *diverged_at = f == kNoDiv ? -1 : (int64_t)f;
  return f == kNoDiv ? LBM_OK : LBM_EDIVERGED;
}

int lbm_moments_device(lbm_ctx* c, double* rho, double* vx, double* vy, double* p) {
  if (!c || !rho || !vx || !vy || !p) return LBM_EINVAL;
  const size_t n = (size_t)c->p.nx * c->p.ny;
  HIPCHK(launch_moments(c->p.precision, c->buf[c->cur], c->d, rho, vx, vy, p, c->aux + 4 * n, c->st));
  return LBM_OK;
}

int lbm_moments(lbm_ctx* c, double* rho, double* vx, double* vy, double* p) {
  if (!c) return LBM_EINVAL;
  const size_t n = (size_t)c->p.nx * c->p.ny;
  double* a = c->aux;
  int st = lbm_moments_device(c, a, a + n, a + 2 * n, a + 3 * n);
  if (st != LBM_OK) return st;
  double* outs[4] = {rho, vx, vy, p};
  for (int i = 0; i < 4; ++i)
    if (outs[i]) HIPCHK(hipMemcpyAsync(outs[i], a + i * n, n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return lbm_status(c, nullptr, nullptr);
}

int lbm_flat_profile(lbm_ctx* c, double* rho_bar, double* p_n) {
  if (!c || !rho_bar) return LBM_EINVAL;
  if (p_n && (c->p.scheme != LBM_SCHEME_IMPROVED || c->d.mrt)) return LBM_ENOTSUP;
  const size_t n = (size_t)c->p.nx * c->p.ny;
  double* a = c->aux;
  // rho plane at a; the column means and the pressure reuse the velocity plane
  double* rb = a + n;
  double* pn = rb + c->p.nx;
  HIPCHK(launch_moments(c->p.precision, c->buf[c->cur], c->d, a, a + n, a + 2 * n, a + 3 * n,
                        a + 4 * n, c->st));
  const dim3 blk(256), grd((c->p.nx + 255) / 256);
  hipLaunchKernelGGL(k_colmean, grd, blk, 0, c->st, (const double*)a, c->p.nx, c->p.ny, rb);
  if (p_n)
    hipLaunchKernelGGL(k_normal_pressure, grd, blk, 0, c->st, (const double*)rb, c->d, c->p.sigma, pn);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(rho_bar, rb, c->p.nx * sizeof(double), hipMemcpyDeviceToHost, c->st));
  if (p_n) HIPCHK(hipMemcpyAsync(p_n, pn, c->p.nx * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return lbm_status(c, nullptr, nullptr);
}

// The three result words of the mass kernels into the caller's outputs.
static void mass_words(const unsigned long long w[3], int64_t* fixed, double* mass) {
  if (fixed) {
    fixed[0] = (int64_t)w[0];
    fixed[1] = (int64_t)w[1];
  }
  if (mass) std::memcpy(mass, &w[2], sizeof(double));
}

int lbm_surface_tension(lbm_ctx* c, double* gamma) {
  if (!c || !gamma) return LBM_EINVAL;
  if (c->p.scheme != LBM_SCHEME_IMPROVED) return LBM_ENOTSUP;
  const size_t n = (size_t)c->p.nx * c->p.ny;
  double* a = c->aux;
  double* rb = a + n;  // column means and the result reuse the velocity plane
  double* g = rb + c->p.nx;
  HIPCHK(launch_moments(c->p.precision, c->buf[c->cur], c->d, a, a + n, a + 2 * n, a + 3 * n,
                        a + 4 * n, c->st));
  hipLaunchKernelGGL(k_colmean, dim3((c->p.nx + 255) / 256), dim3(256), 0, c->st, (const double*)a,
                     c->p.nx, c->p.ny, rb);
  hipLaunchKernelGGL(k_surface_tension, dim3(1), dim3(256), 0, c->st, (const double*)rb, c->d,
                     c->p.sigma, g);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(gamma, g, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return lbm_status(c, nullptr, nullptr);
}

int lbm_mass(lbm_ctx* c, int64_t* fixed, double* mass) {
  if (!c) return LBM_EINVAL;
  HIPCHK(launch_mass(c->p.precision, c->buf[c->cur], c->d, c->part_i, c->part_d, c->mass_out, c->st));
  unsigned long long w[3];
  HIPCHK(hipMemcpyAsync(w, c->mass_out, sizeof w, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  mass_words(w, fixed, mass);
  return lbm_status(c, nullptr, nullptr);
}

int lbm_mass_noalloc(const void* dev_populations, int32_t nx, int32_t ny, int32_t precision,
                     double rho_ref, void* hip_stream, int64_t* fixed, double* mass) {
  if (!dev_populations || nx < 3 || ny < 3) return LBM_EINVAL;
  if (precision < LBM_PREC_F64 || precision > LBM_PREC_F32DEV_F64 || !std::isfinite(rho_ref))
    return LBM_EINVAL;
  if ((int64_t)nx * ny > LBM_NOALLOC_MAX_NODES) return LBM_ENOSPACE;
  char* base = nullptr;
  HIPCHK(scratch_of_current_device(&base));
  RunDev d{};
  d.nx = nx;
  d.ny = ny;
  d.pitch = pitch_of(nx);
  d.plane = plane_of(nx);
  d.rs = rs_of(nx);
  d.elems = elems_of(nx, ny);
  d.rho_ref = precision == LBM_PREC_F64 ? 0.0 : rho_ref;
  __int128* pi = reinterpret_cast<__int128*>(base);
  double* pd = reinterpret_cast<double*>(pi + kMassBlocks);
  unsigned long long* out = reinterpret_cast<unsigned long long*>(pd + kMassBlocks);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  HIPCHK(launch_mass(precision, dev_populations, d, pi, pd, out, st));
  unsigned long long w[3];
  HIPCHK(hipMemcpyAsync(w, out, sizeof w, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  mass_words(w, fixed, mass);
  return LBM_OK;
}

int lbm_get_populations(lbm_ctx* c, double* f, int64_t* step) {
  if (!c || !f) return LBM_EINVAL;
  std::vector<char> raw(c->raw_bytes);
  HIPCHK(hipMemcpyAsync(raw.data(), c->buf[c->cur], raw.size(), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  decode_any(c->p.precision, c->p, c->p.rho_ref, raw.data(), f);
  if (step) *step = c->step;
  return lbm_status(c, nullptr, nullptr);
}

int lbm_set_populations(lbm_ctx* c, const double* f, int64_t step) {
  if (!c || !f || step < 0) return LBM_EINVAL;
  std::vector<char> raw;
  encode_any(c->p.precision, c->p, c->p.rho_ref, f, raw);
  return upload_state(c, raw, step);
}

// Checkpoint: a header {magic, version, step, precision, nx, ny, rho_ref, raw
// bytes} followed by the raw storage of the current buffer.
struct CkptHeader {
  uint64_t magic, version;
  int64_t step;
  int32_t precision, nx, ny, pad;
  double rho_ref;
  uint64_t raw_bytes;
};
static_assert(sizeof(CkptHeader) == 56, "header layout");
constexpr uint64_t kCkptMagic = 0x4C424D434B505431ull;

int lbm_state_bytes(lbm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return LBM_EINVAL;
  *bytes = sizeof(CkptHeader) + c->raw_bytes;
  return LBM_OK;
}

int lbm_save_state(lbm_ctx* c, void* host, size_t bytes) {
  if (!c || !host || bytes < sizeof(CkptHeader) + c->raw_bytes) return LBM_EINVAL;
  CkptHeader h{kCkptMagic, 2, c->step, c->p.precision, c->p.nx, c->p.ny, 0, c->p.rho_ref, c->raw_bytes};
  std::memcpy(host, &h, sizeof h);
  HIPCHK(hipMemcpyAsync(static_cast<char*>(host) + sizeof h, c->buf[c->cur], c->raw_bytes,
                        hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return LBM_OK;
}

int lbm_load_state(lbm_ctx* c, const void* host, size_t bytes) {
  if (!c || !host || bytes < sizeof(CkptHeader)) return LBM_EINVAL;
  CkptHeader h;
  std::memcpy(&h, host, sizeof h);
  if (h.magic != kCkptMagic || h.version != 2 || h.precision != c->p.precision || h.nx != c->p.nx ||
      h.ny != c->p.ny || h.raw_bytes != c->raw_bytes || bytes < sizeof h + c->raw_bytes ||
      !(h.rho_ref == c->p.rho_ref) || h.step < 0)
    return LBM_EINVAL;
  std::vector<char> raw(static_cast<const char*>(host) + sizeof h,
                        static_cast<const char*>(host) + sizeof h + c->raw_bytes);
  return upload_state(c, raw, h.step);
}

int lbm_set_tile(lbm_ctx* c, int32_t nw, int32_t L, int32_t depth, int32_t steps) {
  if (!c || !valid_tile(nw, L, depth, 16, steps)) return LBM_EINVAL;
  if (steps == 3 && !has_step3(c->p.precision)) return LBM_ENOTSUP;
  if (steps == 3 && (c->p.nx < 5 || c->p.ny < 5)) return LBM_EINVAL;  // halo of 5 wraps once
  c->tile = Tile{nw, L, depth, steps};
  return prepare_graphs(c);
}

int lbm_get_tile(lbm_ctx* c, int32_t* nw, int32_t* L, int32_t* depth, int32_t* steps) {
  if (!c) return LBM_EINVAL;
  if (nw) *nw = c->tile.nw;
  if (L) *L = c->tile.L;
  if (depth) *depth = c->tile.pf;
  if (steps) *steps = c->tile.ts;
  return LBM_OK;
}

int lbm_tune(lbm_ctx* c, int32_t* nw_out, int32_t* L_out, int32_t* depth_out, int32_t* steps_out) {
  if (!c) return LBM_EINVAL;
  Tile bt = c->tile;
  const int s = c->cur;
  const int64_t nodes = (int64_t)c->p.nx * c->p.ny;
  const int reps = nodes >= (1 << 22) ? 3 : 10;
  std::vector<Tile> cand;
  for (int nw : kStepWaves) {
    if (nw > 1 && 64 * (nw / 2) >= c->p.nx) continue;
    for (int pf : {1, 2})
      for (int L : {0, 1, 2, 4, 8, 16, 32, 64, 128})
        if (L <= 2 * c->p.ny && (L == 0 || L > 2 || nodes < (1 << 20)))  // 1-2 rows: small lattices
          cand.push_back(Tile{nw, L, pf, 1});
  }
  for (int nw : kStep2Waves) {
    if (nw > 4 && 64 * (nw / 2) >= c->p.nx) continue;
    for (int pf : {1, 2})
      for (int L : {0, 32, 64, 128})
        if (L <= 2 * c->p.ny) cand.push_back(Tile{nw, L, pf, 2});
  }
  if (has_step3(c->p.precision) && c->p.nx >= 16 && c->p.ny >= 16)
    for (int nw : {4, 8}) {
      if (nw > 4 && 64 * (nw / 2) >= c->p.nx) continue;
      for (int L : {0, 64, 128})
        if (L <= 2 * c->p.ny) cand.push_back(Tile{nw, L, 1, 3});
    }
  const int pst = pick_tile(
      cand,
      [&](const Tile& t) {
        const float ms = time_launches(
            c->st,
            [&] {
              return launch_step(c->p.precision, t, c->buf[s], c->buf[s ^ 1], c->d, nullptr,
                                 (unsigned long long)c->step, c->flag, c->st);
            },
            reps);
        return ms < 0 ? ms : ms / t.ts;  // time per lattice step
      },
      bt);
  if (pst != LBM_OK) return pst;
  c->tile = bt;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[{c->p.nx, c->p.ny, c->p.precision, c->d.mrt}] = bt;
  }
  const int gst = prepare_graphs(c);
  if (gst != LBM_OK) return gst;
  if (nw_out) *nw_out = bt.nw;
  if (L_out) *L_out = bt.L;
  if (depth_out) *depth_out = bt.pf;
  if (steps_out) *steps_out = bt.ts;
  return LBM_OK;
}

int lbm_set_graph_steps(lbm_ctx* c, int32_t k) {
  if (!c || k < 0 || (k > 0 && (k < 2 || k % 2))) return LBM_EINVAL;
  if (k > 0 && c->st == nullptr) return LBM_EINVAL;  // the null stream cannot be captured
  drop_graphs(c);
  c->graph_k = k;
  return prepare_graphs(c);
}

int lbm_set_mrt(lbm_ctx* c, const double* rates) {
  if (!c) return LBM_EINVAL;
  if (!rates) {
    const int mrt = c->d.mrt;
    c->d = make_rundev(c->p, c->k, c->p.rho_ref, 0, 0);
    if (mrt) drop_graphs(c);
    return prepare_graphs(c);
  }
  if (c->p.scheme != LBM_SCHEME_IMPROVED) return LBM_ENOTSUP;
  if (c->p.precision != LBM_PREC_F64 && c->p.precision != LBM_PREC_F32DEV) return LBM_ENOTSUP;
  for (int i = 0; i < 3; ++i)
    if (!(rates[i] > 0.0 && rates[i] < 2.0)) return LBM_EINVAL;
  c->d = make_rundev(c->p, c->k, c->p.rho_ref, 0, 0);
  set_mrt(c->d, c->p, rates);
  drop_graphs(c);  // the captured launches carry the old constants
  return prepare_graphs(c);
}

int lbm_graph_captures(lbm_ctx* c, int64_t* n) {
  if (!c || !n) return LBM_EINVAL;
  *n = c->captures;
  return LBM_OK;
}

int lbm_debug_index_faults(uint64_t* count) {
  if (!count) return LBM_EINVAL;
#ifdef LBM_CHECK_INDEX
  unsigned long long v = 0, zero = 0;
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_index_faults), sizeof v));
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(g_index_faults), &zero, sizeof zero));
  *count = v;
  return LBM_OK;
#else
  *count = 0;
  return LBM_ENOTSUP;
#endif
}

int lbm_get_params(lbm_ctx* c, lbm_params* out) {
  if (!c || !out) return LBM_EINVAL;
  *out = c->p;
  return LBM_OK;
}

int lbm_device_buffers(lbm_ctx* c, void** b0, void** b1, int32_t* cur) {
  if (!c) return LBM_EINVAL;
  if (b0) *b0 = c->buf[0];
  if (b1) *b1 = c->buf[1];
  if (cur) *cur = c->cur;
  return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  (void)hipStreamSynchronize(c->st);
  drop_graphs(c);
  delete c;
  return LBM_OK;
}

}  // extern "C"

// ============================================================================
// Batch of independent lattices.
// ============================================================================

struct lbm_batch {
  int nruns;
  int prec, esize;
  std::vector<lbm_params> p;
  std::vector<EosConst> k;
  std::vector<RunDev> d;  // host copy of the descriptor table
  std::vector<int64_t> nodes;
  char* ws;
  size_t pool_bytes;
  void* buf[2];
  int cur;
  RunDev* d_runs;
  Item* d_items;
  int nitems, items_cap;
  int total_rows;  // balanced schedule: rows of all strip items (0 for item lists)
  unsigned long long* flags;
  unsigned long long* ctr;
  double* aux;
  size_t aux_nodes;
  hipStream_t st;
  int64_t step;
  Tile tile;
  int graph_k;
  hipGraphExec_t gexec[2];
  Tile gtile;
  int64_t captures;  // graphs captured so far
  double* coex;      // 2 * nruns doubles: (rho_l, rho_g) per run
  int mrt;           // 1: every run's descriptor carries the MRT collision
};

namespace {

struct BatchLayout {
  size_t pool, runs, items, flags, aux, coex, total;
  int items_cap;
  size_t aux_nodes;
};

int64_t run_elems(const lbm_params& q) { return layout::run_elems(q.nx, q.ny); }

BatchLayout batch_layout(int n, const lbm_params* p) {
  BatchLayout L{};
  size_t elems = 0, maxn = 0;
  int cap = 0;
  const size_t es = esize_of(p[0].precision);
  for (int i = 0; i < n; ++i) {
    elems += run_elems(p[i]);
    maxn = std::max(maxn, (size_t)p[i].nx * p[i].ny);
    cap += layout::max_items(p[i].nx, p[i].ny);
  }
  L.pool = align_up(elems * es);
  L.runs = align_up(n * sizeof(RunDev));
  L.items_cap = cap;
  L.items = align_up((size_t)cap * sizeof(Item));
  L.flags = align_up((n + 1) * sizeof(unsigned long long));
  L.aux_nodes = maxn;
  L.aux = align_up(5 * maxn * sizeof(double));
  L.coex = align_up(2 * (size_t)n * sizeof(double));
  L.total = 2 * L.pool + L.runs + L.items + L.flags + L.aux + L.coex;
  return L;
}

// Work list of a tile (layout::build_items), uploaded to the device.
int batch_items(lbm_batch* b, const Tile& t) {
  std::vector<Item> items;
  std::vector<int> nx(b->nruns), ny(b->nruns);
  for (int r = 0; r < b->nruns; ++r) {
    nx[r] = b->p[r].nx;
    ny[r] = b->p[r].ny;
  }
  // two-step strips of FP64 lattices start on 64-byte boundaries, as for a single lattice
  const int64_t rows = layout::build_items(b->nruns, nx.data(), ny.data(), t.nw, t.L, t.ts, items,
                                           b->prec == LBM_PREC_F64 ? Step2Align<double>::value : 1);
  if ((int)items.size() > b->items_cap) return LBM_ENOSPACE;
  if (rows >= INT32_MAX) return LBM_EINVAL;
  b->total_rows = t.L > 0 ? 0 : (int)rows;
  HIPCHK(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  b->nitems = (int)items.size();
  b->tile = t;
  return LBM_OK;
}

void batch_drop_graphs(lbm_batch* b) {
  for (int i = 0; i < 2; ++i)
    if (b->gexec[i]) {
      (void)hipGraphExecDestroy(b->gexec[i]);
      b->gexec[i] = nullptr;
    }
}

int batch_capture(lbm_batch* b, int parity) {
  hipGraph_t g;
  HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  const int launches = b->graph_k / b->tile.ts;  // graph_k is even
  for (int i = 0; i < launches && e == hipSuccess; ++i) {
    const int s = (parity + i) & 1;
    e = launch_batch(b->prec, b->mrt != 0, b->tile, b->buf[s], b->buf[s ^ 1], b->d_runs, b->d_items, b->nitems, b->total_rows,
                     b->ctr, (unsigned long long)i * b->tile.ts, b->flags, b->st);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_counter_add, dim3(1), dim3(1), 0, b->st, b->ctr, (unsigned long long)b->graph_k);
    e = hipGetLastError();
  }
  hipError_t e2 = hipStreamEndCapture(b->st, &g);
  if (e != hipSuccess || e2 != hipSuccess) return LBM_EHIP;
  e = hipGraphInstantiate(&b->gexec[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e == hipSuccess) e = hipGraphUpload(b->gexec[parity], b->st);
  if (e != hipSuccess) {
    if (b->gexec[parity]) (void)hipGraphExecDestroy(b->gexec[parity]);
    b->gexec[parity] = nullptr;
    return LBM_EHIP;
  }
  b->gtile = b->tile;
  ++b->captures;
  return LBM_OK;
}

int batch_prepare_graphs(lbm_batch* b) {
  if (b->graph_k <= 0) return LBM_OK;
  if (!same_tile(b->gtile, b->tile)) batch_drop_graphs(b);
  for (int parity = 0; parity < 2; ++parity)
    if (!b->gexec[parity]) {
      int st = batch_capture(b, parity);
      if (st != LBM_OK) return st;
    }
  HIPCHK(hipStreamSynchronize(b->st));
  return LBM_OK;
}

std::tuple<int, int, int, int> batch_key(const lbm_batch* b) {
  int64_t tot = 0;
  int maxnx = 0;
  for (int r = 0; r < b->nruns; ++r) {
    tot += b->nodes[r];
    maxnx = std::max(maxnx, b->p[r].nx);
  }
  return {(int)std::min<int64_t>(tot, INT32_MAX), maxnx, b->prec | (b->mrt << 8), b->nruns};
}

}  // namespace

extern "C" {

int lbm_batch_workspace_bytes(int32_t n, const lbm_params* p, size_t* bytes) {
  if (n < 1 || !p || !bytes) return LBM_EINVAL;
  for (int i = 0; i < n; ++i) {
    int st = validate(p[i]);
    if (st != LBM_OK) return st;
    if (p[i].precision != p[0].precision) return LBM_EINVAL;
  }
  *bytes = batch_layout(n, p).total;
  return LBM_OK;
}

int lbm_batch_init(int32_t n, const lbm_params* p, const double* const* rho0, void* ws,
                   size_t ws_bytes, void* stream, lbm_batch** out) {
  if (n < 1 || !p || !rho0 || !ws || !out) return LBM_EINVAL;
  *out = nullptr;
  size_t need;
  int st = lbm_batch_workspace_bytes(n, p, &need);
  if (st != LBM_OK) return st;
  if (ws_bytes < need) return LBM_ENOSPACE;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return LBM_EINVAL;
  for (int r = 0; r < n; ++r)
    if (!rho0[r]) return LBM_EINVAL;
  const BatchLayout Lay = batch_layout(n, p);
  lbm_batch* b = new lbm_batch{};
  b->nruns = n;
  b->prec = p[0].precision;
  b->esize = esize_of(b->prec);
  b->p.assign(p, p + n);
  b->k.resize(n);
  b->ws = static_cast<char*>(ws);
  b->pool_bytes = Lay.pool;
  b->buf[0] = b->ws;
  b->buf[1] = b->ws + Lay.pool;
  b->d_runs = reinterpret_cast<RunDev*>(b->ws + 2 * Lay.pool);
  b->d_items = reinterpret_cast<Item*>(b->ws + 2 * Lay.pool + Lay.runs);
  b->items_cap = Lay.items_cap;
  b->flags = reinterpret_cast<unsigned long long*>(b->ws + 2 * Lay.pool + Lay.runs + Lay.items);
  b->ctr = b->flags + n;
  b->aux = reinterpret_cast<double*>(b->ws + 2 * Lay.pool + Lay.runs + Lay.items + Lay.flags);
  b->aux_nodes = Lay.aux_nodes;
  b->coex = reinterpret_cast<double*>(b->ws + 2 * Lay.pool + Lay.runs + Lay.items + Lay.flags + Lay.aux);
  b->st = static_cast<hipStream_t>(stream);
  std::vector<char> pool(Lay.pool, 0);
  int64_t off = 0;
  for (int r = 0; r < n && st == LBM_OK; ++r) {
    const lbm_params& q = p[r];
    st = eos_constants(q, &b->k[r]);
    if (st != LBM_OK) break;
    const size_t nn = (size_t)q.nx * q.ny;
    double mean = 0;
    for (size_t i = 0; i < nn; ++i) {
      if (!(rho0[r][i] > 0) || !(host_psi2(b->k[r], rho0[r][i]) > 0)) st = LBM_EPSI;
      mean += rho0[r][i];
    }
    if (st != LBM_OK) break;
    mean /= (double)nn;
    const double rref = b->prec == LBM_PREC_F64 ? 0.0 : (std::isnan(q.rho_ref) ? mean : q.rho_ref);
    b->p[r].rho_ref = rref;
    b->d.push_back(make_rundev(q, b->k[r], rref, off, r));
    b->nodes.push_back((int64_t)nn);
    std::vector<double> f(9 * nn);
    for (size_t i = 0; i < nn; ++i) {
      double fe[9];
      host_feq(rho0[r][i], 0.0, 0.0, fe);
      for (int a = 0; a < 9; ++a) f[a * nn + i] = fe[a];
    }
    std::vector<char> raw;
    encode_any(b->prec, q, rref, f.data(), raw);
    std::memcpy(pool.data() + off * b->esize, raw.data(), raw.size());
    off += run_elems(q);
  }
  if (st != LBM_OK) {
    delete b;
    return st;
  }
  hipError_t e = hipMemcpyAsync(b->buf[0], pool.data(), pool.size(), hipMemcpyHostToDevice, b->st);
  if (e == hipSuccess) e = hipMemsetAsync(b->buf[1], 0, pool.size(), b->st);  // row padding
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_runs, b->d.data(), n * sizeof(RunDev), hipMemcpyHostToDevice, b->st);
  std::vector<unsigned long long> fl(n + 1, kNoDiv);
  fl[n] = 0;  // step counter
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->flags, fl.data(), fl.size() * sizeof(unsigned long long), hipMemcpyHostToDevice, b->st);
  if (e == hipSuccess) e = hipStreamSynchronize(b->st);
  if (e != hipSuccess) {
    delete b;
    return LBM_EHIP;
  }
  Tile t{1, 16, 2};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(batch_key(b));
    if (it != g_tune.end()) t = it->second;
  }
  st = batch_items(b, t);
  if (st != LBM_OK) {
    delete b;
    return st;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int64_t n) {
  if (!b || n < 0) return LBM_EINVAL;
  int64_t done = 0;
  if (b->graph_k > 0 && n >= b->graph_k) {
    if (!same_tile(b->gtile, b->tile)) batch_drop_graphs(b);
    hipLaunchKernelGGL(k_counter_set, dim3(1), dim3(1), 0, b->st, b->ctr, (unsigned long long)b->step);
    HIPCHK(hipGetLastError());
    while (n - done >= b->graph_k) {
      if (!b->gexec[b->cur]) {
        int st = batch_capture(b, b->cur);
        if (st != LBM_OK) return st;
      }
      HIPCHK(hipGraphLaunch(b->gexec[b->cur], b->st));
      done += b->graph_k;
      b->step += b->graph_k;
      b->cur ^= (b->graph_k / b->tile.ts) & 1;  // one buffer swap per launch
    }
  }
  while (done < n) {
    const int s = b->cur;
    Tile t = b->tile;
    if (n - done < t.ts) t.ts = 1;  // odd remainder of a two-step tile (its items suit both)
    HIPCHK(launch_batch(b->prec, b->mrt != 0, t, b->buf[s], b->buf[s ^ 1], b->d_runs, b->d_items, b->nitems, b->total_rows,
                        nullptr, (unsigned long long)b->step, b->flags, b->st));
    b->cur ^= 1;
    b->step += t.ts;
    done += t.ts;
  }
  return LBM_OK;
}

int lbm_batch_set_tile(lbm_batch* b, int32_t nw, int32_t L, int32_t depth, int32_t steps) {
  if (!b || !valid_tile(nw, L, depth, 8, steps, 2) || (L > 0 && L < 4)) return LBM_EINVAL;
  batch_drop_graphs(b);
  const int st = batch_items(b, Tile{nw, L, depth, steps});
  return st != LBM_OK ? st : batch_prepare_graphs(b);
}

int lbm_batch_get_tile(lbm_batch* b, int32_t* nw, int32_t* L, int32_t* depth, int32_t* steps) {
  if (!b) return LBM_EINVAL;
  if (steps) *steps = b->tile.ts;
  if (nw) *nw = b->tile.nw;
  if (L) *L = b->tile.L;
  if (depth) *depth = b->tile.pf;
  return LBM_OK;
}

int lbm_batch_set_graph_steps(lbm_batch* b, int32_t k) {
  if (!b || k < 0 || (k > 0 && (k < 2 || k % 2))) return LBM_EINVAL;
  if (k > 0 && b->st == nullptr) return LBM_EINVAL;
  batch_drop_graphs(b);
  b->graph_k = k;
  return batch_prepare_graphs(b);
}

int lbm_batch_set_mrt(lbm_batch* b, const double* rates) {
  if (!b) return LBM_EINVAL;
  if (rates) {
    if (b->prec != LBM_PREC_F64 && b->prec != LBM_PREC_F32DEV) return LBM_ENOTSUP;
    for (int r = 0; r < b->nruns; ++r) {
      if (b->p[r].scheme != LBM_SCHEME_IMPROVED) return LBM_ENOTSUP;
      for (int i = 0; i < 3; ++i)
        if (!(rates[3 * r + i] > 0.0 && rates[3 * r + i] < 2.0)) return LBM_EINVAL;
    }
  }
  for (int r = 0; r < b->nruns; ++r) {
    RunDev& d = b->d[r];
    // back to the BGK values make_rundev sets, then the run's MRT rates
    d.mrt = 0;
    d.s_e = d.s_eps = d.s_q = d.inv_tau;
    d.sig_e = d.sig_eps = d.sig;
    if (rates) set_mrt(d, b->p[r], rates + 3 * r);
  }
  HIPCHK(hipMemcpyAsync(b->d_runs, b->d.data(), b->nruns * sizeof(RunDev), hipMemcpyHostToDevice, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  b->mrt = rates ? 1 : 0;
  batch_drop_graphs(b);  // the captured launches are of the other kernels
  return batch_prepare_graphs(b);
}

int lbm_batch_graph_captures(lbm_batch* b, int64_t* n) {
  if (!b || !n) return LBM_EINVAL;
  *n = b->captures;
  return LBM_OK;
}

int lbm_batch_tune(lbm_batch* b, int32_t* nw_out, int32_t* L_out, int32_t* depth_out,
                   int32_t* steps_out) {
  if (!b) return LBM_EINVAL;
  Tile bt = b->tile;
  const int s = b->cur;
  int maxnx = 0;
  for (int r = 0; r < b->nruns; ++r) maxnx = std::max(maxnx, b->p[r].nx);
  std::vector<Tile> cand;
  for (int nw : kBatchWaves) {
    if (nw > 1 && 64 * (nw / 2) >= maxnx) continue;
    for (int pf : {1, 2})
      for (int L : {0, 4, 8, 16, 32, 64}) cand.push_back(Tile{nw, L, pf, 1});
  }
  for (int nw : kBatchStep2Waves) {
    if (nw > 4 && 64 * (nw / 2) >= maxnx) continue;
    for (int pf : {1, 2})
      for (int L : {0, 32, 64}) cand.push_back(Tile{nw, L, pf, 2});
  }
  int ist = LBM_OK;
  const int pst = pick_tile(
      cand,
      [&](const Tile& t) {
        ist = batch_items(b, t);
        if (ist == LBM_ENOSPACE) return 1e30f;  // too many items for the work list: skipped
        if (ist != LBM_OK) return -1.f;
        const float ms = time_launches(
            b->st,
            [&] {
              return launch_batch(b->prec, b->mrt != 0, t, b->buf[s], b->buf[s ^ 1], b->d_runs, b->d_items,
                                  b->nitems, b->total_rows, nullptr, (unsigned long long)b->step,
                                  b->flags, b->st);
            },
            5);
        return ms < 0 ? ms : ms / t.ts;  // time per lattice step
      },
      bt);
  if (pst != LBM_OK) return ist != LBM_OK && ist != LBM_ENOSPACE ? ist : pst;
  batch_drop_graphs(b);
  int st = batch_items(b, bt);
  if (st != LBM_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[batch_key(b)] = bt;
  }
  st = batch_prepare_graphs(b);
  if (st != LBM_OK) return st;
  if (nw_out) *nw_out = bt.nw;
  if (L_out) *L_out = bt.L;
  if (depth_out) *depth_out = bt.pf;
  if (steps_out) *steps_out = bt.ts;
  return LBM_OK;
}

int lbm_batch_nodes(lbm_batch* b, int64_t* nodes) {
  if (!b || !nodes) return LBM_EINVAL;
  std::vector<unsigned long long> fl(b->nruns);
  HIPCHK(hipMemcpyAsync(fl.data(), b->flags, b->nruns * sizeof(unsigned long long), hipMemcpyDeviceToHost, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  int64_t t = 0;
  for (int r = 0; r < b->nruns; ++r)
    if (fl[r] == kNoDiv) t += b->nodes[r];
  *nodes = t;
  return LBM_OK;
}

// LBM_EDIVERGED when the run is frozen by divergence, else LBM_OK (synchronises).
static int batch_run_status(lbm_batch* b, int32_t run) {
  unsigned long long f = 0;
  HIPCHK(hipMemcpyAsync(&f, b->flags + run, sizeof f, hipMemcpyDeviceToHost, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  return f == kNoDiv ? LBM_OK : LBM_EDIVERGED;
}

int lbm_batch_moments(lbm_batch* b, int32_t run, double* rho, double* vx, double* vy, double* p) {
  if (!b || run < 0 || run >= b->nruns) return LBM_EINVAL;
  const RunDev& d = b->d[run];
  const size_t n = (size_t)d.nx * d.ny;
  double* a = b->aux;
  const char* src = static_cast<const char*>(b->buf[b->cur]) + d.off * b->esize;
  HIPCHK(launch_moments(b->prec, src, d, a, a + n, a + 2 * n, a + 3 * n, a + 4 * n, b->st));
  double* outs[4] = {rho, vx, vy, p};
  for (int i = 0; i < 4; ++i)
    if (outs[i]) HIPCHK(hipMemcpyAsync(outs[i], a + i * n, n * sizeof(double), hipMemcpyDeviceToHost, b->st));
  return batch_run_status(b, run);
}

int lbm_batch_get_populations(lbm_batch* b, int32_t run, double* f) {
  if (!b || run < 0 || run >= b->nruns || !f) return LBM_EINVAL;
  const RunDev& d = b->d[run];
  std::vector<char> raw(raw_bytes_of(b->p[run]));
  const char* src = static_cast<const char*>(b->buf[b->cur]) + d.off * b->esize;
  HIPCHK(hipMemcpyAsync(raw.data(), src, raw.size(), hipMemcpyDeviceToHost, b->st));
  const int st = batch_run_status(b, run);
  if (st != LBM_OK && st != LBM_EDIVERGED) return st;
  decode_any(b->prec, b->p[run], d.rho_ref, raw.data(), f);
  return st;
}

int lbm_batch_coexistence(lbm_batch* b, double* rho_l, double* rho_g, int32_t* status,
                          int64_t* diverged_at) {
  if (!b) return LBM_EINVAL;
  HIPCHK(launch_batch_coex(b->prec, b->buf[b->cur], b->d_runs, b->nruns, b->flags, b->coex, b->st));
  std::vector<unsigned long long> fl(b->nruns);
  std::vector<double> lg(2 * (size_t)b->nruns);
  HIPCHK(hipMemcpyAsync(fl.data(), b->flags, b->nruns * sizeof(unsigned long long), hipMemcpyDeviceToHost, b->st));
  HIPCHK(hipMemcpyAsync(lg.data(), b->coex, lg.size() * sizeof(double), hipMemcpyDeviceToHost, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  for (int r = 0; r < b->nruns; ++r) {
    const bool div = fl[r] != kNoDiv;
    if (status) status[r] = div ? LBM_EDIVERGED : LBM_OK;
    if (diverged_at) diverged_at[r] = div ? (int64_t)fl[r] : -1;
    if (rho_l) rho_l[r] = lg[2 * r];
    if (rho_g) rho_g[r] = lg[2 * r + 1];
  }
  return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_EINVAL;
  (void)hipStreamSynchronize(b->st);
  batch_drop_graphs(b);
  delete b;
  return LBM_OK;
}

}  // extern "C"
