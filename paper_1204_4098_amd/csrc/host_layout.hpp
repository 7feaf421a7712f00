// Host-side storage layout, batch work lists and the tuner's selection rule of
// the library, in plain C++ (no HIP), so that they can also be built with the
// host sanitizers.  Used by lbm_lib.hip.
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

namespace lbm {

// A tile of the batched launch.  In the balanced schedule an item is a whole
// strip of one run and row0 is its first row in the concatenated row space of
// all items (rows of earlier items summed); item lists leave it 0.
struct Item {
  int32_t run, x0, y0, ncols, nrows, row0;
};

namespace layout {

constexpr int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Population storage, row-interleaved: element (a, y, x) at a * plane + y * rs
// + x with rows of pitch elements (nx rounded up to 64), plane = pitch and rs =
// 9 pitch, so the nine direction rows of one lattice row are consecutive in
// memory.  A row of the march then reads and writes three 9-row blocks close
// together instead of 18 rows in nine planes far apart: on the 4096 x 4096
// FP64 workload the two-step kernel runs 491 us per launch against 525 us with
// plane-major storage (plane = ny pitch, rs = pitch), and a memory-only
// marching probe reaches 5.5 against 5.2 TB/s.
inline int pitch_of(int nx) { return (nx + 63) / 64 * 64; }
inline int64_t plane_of(int nx) { return (int64_t)pitch_of(nx); }
inline int64_t rs_of(int nx) { return 9 * (int64_t)pitch_of(nx); }
inline int64_t elems_of(int nx, int ny) { return 9 * (int64_t)pitch_of(nx) * ny; }

// Encode FP64 populations f[a][y][x] (nx*ny per direction) into the
// pre-streamed storage b (elems_of elements, padding left as it is): b holds
// f*_a(x, y) at node (x, y), and the kernel's pull reads it at (x + e_a, y +
// e_a); so b(a, y, x) = f[a][y + ey][x + ex] (periodic).  enc(a, v) converts
// one value to the storage type.
template <typename S, class Enc>
void encode(int nx, int ny, const double* f, S* b, Enc&& enc) {
  const int64_t plane = plane_of(nx), rs = rs_of(nx), n = (int64_t)nx * ny;
  for (int a = 0; a < 9; ++a)
    for (int y = 0; y < ny; ++y) {
      const int ys = (y + kEY[a] + ny) % ny;
      for (int x = 0; x < nx; ++x) {
        const int xs = (x + kEX[a] + nx) % nx;
        b[a * plane + (int64_t)y * rs + x] = enc(a, f[a * n + (int64_t)ys * nx + xs]);
      }
    }
}

// The inverse: dec(a, s) converts one stored value to FP64.
template <typename S, class Dec>
void decode(int nx, int ny, const S* b, double* f, Dec&& dec) {
  const int64_t plane = plane_of(nx), rs = rs_of(nx), n = (int64_t)nx * ny;
  for (int a = 0; a < 9; ++a)
    for (int y = 0; y < ny; ++y) {
      const int ys = (y - kEY[a] + ny) % ny;
      for (int x = 0; x < nx; ++x) {
        const int xs = (x - kEX[a] + nx) % nx;
        f[a * n + (int64_t)y * nx + x] = dec(a, b[a * plane + (int64_t)ys * rs + xs]);
      }
    }
}

// Elements of one run in the batch pool (rounded up to 64).
inline int64_t run_elems(int nx, int ny) { return (elems_of(nx, ny) + 63) / 64 * 64; }

// The most items any offered tile can produce for a run (1 wave, 4 rows).
inline int max_items(int nx, int ny) { return ((nx + 63) / 64) * ((ny + 3) / 4); }

// Work list of a batch tile: per run, chunks of L rows times strips of 64*nw
// columns, or for the two-step tile (ts = 2) strips of at most 64*nw - 6
// columns spread evenly over the run's width with their edges rounded down to
// multiples of `align` columns (such items also suit the one-step kernel,
// which runs an odd remainder step).  L = 0: whole-height strips with row0 set
// for the balanced schedule.  Returns the rows of all items (the balanced
// schedule's row space).
inline int64_t build_items(int nruns, const int* nx, const int* ny, int nw, int L, int ts,
                           std::vector<Item>& items, int align = 1) {
  items.clear();
  const int SW = 64 * nw, A = ts == 2 ? std::max(1, align) : 1;
  int64_t rows = 0;
  for (int r = 0; r < nruns; ++r) {
    const int Lr = L > 0 ? L : ny[r];
    // strips of at most SW - 6 columns once their edges are rounded down to A
    const int ns = ts == 2 ? (nx[r] + SW - 7 - (A - 1)) / (SW - 6 - (A - 1)) : (nx[r] + SW - 1) / SW;
    auto edge = [&](int k) { return k >= ns ? nx[r] : (int)((int64_t)k * nx[r] / ns) / A * A; };
    for (int y0 = 0; y0 < ny[r]; y0 += Lr)
      for (int sx = 0; sx < ns; ++sx) {
        const int x0 = ts == 2 ? edge(sx) : sx * SW;
        const int x1 = ts == 2 ? edge(sx + 1) : std::min(nx[r], x0 + SW);
        const int n = std::min(Lr, ny[r] - y0);
        items.push_back(Item{r, x0, y0, x1 - x0, n, L > 0 ? 0 : (int32_t)std::min<int64_t>(rows, INT32_MAX)});
        rows += n;
      }
  }
  return rows;
}

}  // namespace layout

namespace tuning {

// Index of the fastest of n candidates.  time_one(i) times candidate i
// (milliseconds per lattice step; negative on an error; >= 1e30 to skip it).
// A single pass in candidate order is biased by the GPU's clocks drifting down
// over a long back-to-back run (a kernel trace of the FP64 4096 x 4096 tune
// showed candidates late in the list running up to 40 % slower than the same
// kernels before or after the tune).  So the first pass only shortlists the
// kRefine fastest; they are then timed again in kRefine rounds, each round
// starting one candidate later, so that every finalist is timed once at every
// position of a round, and they are ranked by the sum of those times: a drift
// that grows linearly over the calls then adds the same to every finalist's
// sum.  Returns the index, -1 if every candidate was skipped, or -2 after an
// error.
constexpr int kRefine = 6;
template <class TimeOne>
int pick_best(int n, TimeOne&& time_one) {
  std::vector<std::pair<float, int>> first;
  for (int i = 0; i < n; ++i) {
    const float ms = time_one(i);
    if (ms < 0) return -2;
    if (ms < 1e30f) first.push_back({ms, i});
  }
  if (first.empty()) return -1;
  std::sort(first.begin(), first.end());
  const int m = std::min<int>(kRefine, (int)first.size());
  if (m == 1) return first[0].second;
  std::vector<double> sum(m, 0.0);
  for (int r = 0; r < m; ++r)
    for (int q = 0; q < m; ++q) {
      const int k = (q + r) % m;
      const float ms = time_one(first[k].second);
      if (ms < 0) return -2;
      sum[k] += ms;
    }
  int kb = 0;
  for (int k = 1; k < m; ++k)
    if (sum[k] < sum[kb]) kb = k;
  return first[kb].second;
}

}  // namespace tuning
}  // namespace lbm
