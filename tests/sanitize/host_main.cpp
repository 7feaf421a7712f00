// Driver for the sanitizer build of the library's host-side layout and work
// lists (paper_1204_4098_amd/csrc/host_layout.hpp; test infrastructure): round
// trips through encode/decode on odd shapes and checks that the batch work
// lists of every offered tile cover each node of each run exactly once and stay
// inside the runs, so that AddressSanitizer and UndefinedBehaviorSanitizer see
// every index computation.  Exit status 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "host_layout.hpp"

using namespace lbm;

static int failures = 0;
#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      std::printf("check failed: %s (line %d)\n", #c, __LINE__);       \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static void round_trips(int nx, int ny, std::mt19937_64& rng) {
  std::uniform_real_distribution<double> u(0.01, 0.5);
  const size_t n = (size_t)nx * ny;
  std::vector<double> f(9 * n), g(9 * n);
  for (auto& v : f) v = u(rng);
  std::vector<double> b(layout::elems_of(nx, ny), -1.0);
  layout::encode(nx, ny, f.data(), b.data(), [](int, double v) { return v; });
  layout::decode(nx, ny, b.data(), g.data(), [](int, double v) { return v; });
  CHECK(f == g);
  // every stored element written once at most: the stored values are a permutation
  size_t written = 0;
  for (double v : b) written += v >= 0.0;
  CHECK(written == 9 * n);
  std::vector<float> bf(layout::elems_of(nx, ny), 0.f);
  layout::encode(nx, ny, f.data(), bf.data(), [](int, double v) { return (float)v; });
  layout::decode(nx, ny, bf.data(), g.data(), [](int, float v) { return (double)v; });
  for (size_t i = 0; i < 9 * n; ++i) CHECK(g[i] == (double)(float)f[i]);
}

static void work_lists(std::mt19937_64& rng) {
  for (int trial = 0; trial < 40; ++trial) {
    const int nruns = 1 + (int)(rng() % 12);
    std::vector<int> nx(nruns), ny(nruns);
    int cap = 0;
    for (int r = 0; r < nruns; ++r) {
      nx[r] = 3 + (int)(rng() % 600);
      ny[r] = 3 + (int)(rng() % 130);
      cap += layout::max_items(nx[r], ny[r]);
    }
    for (int nw : {1, 2, 4, 8})
      for (int ts : {1, 2})
        for (int align : {1, 8}) {
        if ((ts == 1 && align != 1) || (ts == 2 && nw < 2)) continue;  // tiles the library offers
        for (int L : {0, 4, 5, 8, 32, 128}) {
          std::vector<Item> items;
          const int64_t rows = layout::build_items(nruns, nx.data(), ny.data(), nw, L, ts, items, align);
          CHECK((int)items.size() <= cap);
          std::vector<std::vector<int>> cover(nruns);
          for (int r = 0; r < nruns; ++r) cover[r].assign((size_t)nx[r] * ny[r], 0);
          int64_t prefix = 0;
          for (const Item& it : items) {
            CHECK(it.run >= 0 && it.run < nruns);
            if (it.run < 0 || it.run >= nruns) continue;
            const int r = it.run;
            CHECK(it.x0 >= 0 && it.ncols >= 1 && it.x0 + it.ncols <= nx[r]);
            CHECK(it.y0 >= 0 && it.nrows >= 1 && it.y0 + it.nrows <= ny[r]);
            CHECK(it.ncols <= (ts == 2 ? 64 * nw - 6 : 64 * nw));
            CHECK(it.x0 % align == 0);
            if (L > 0) CHECK(it.nrows <= L && it.row0 == 0);
            else CHECK(it.row0 == prefix && it.nrows == ny[r] && it.y0 == 0);
            prefix += it.nrows;
            for (int y = it.y0; y < it.y0 + it.nrows && y < ny[r]; ++y)
              for (int x = it.x0; x < it.x0 + it.ncols && x < nx[r]; ++x) ++cover[r][(size_t)y * nx[r] + x];
          }
          CHECK(prefix == rows);
          for (int r = 0; r < nruns; ++r)
            for (int c : cover[r]) CHECK(c == 1);
        }
      }
  }
}

int main() {
  std::mt19937_64 rng(0x12044098);
  const int shapes[][2] = {{3, 3}, {5, 4}, {64, 16}, {70, 9}, {130, 7}, {257, 3}};
  for (const auto& s : shapes) round_trips(s[0], s[1], rng);
  work_lists(rng);
  std::printf("host layout sanitizer driver: %d failed checks\n", failures);
  return failures != 0;
}
