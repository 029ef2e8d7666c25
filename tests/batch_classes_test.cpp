// CPU test of the batch's binning launch classes (batch_classes.h): the
// class of a tile's or grid's LDS, and the merging of classes too small to
// fill the device.  Built and run by tests/test_batch_classes.py; exits
// nonzero with a message on the first broken expectation.
#include <cstdio>
#include <map>
#include <random>
#include <vector>

#include "../paper_2310_02926_amd/csrc/batch_classes.h"

using binimpl::lds_class;
using binimpl::merge_small_classes;

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                            \
  do {                                                              \
    if (!(cond)) {                                                  \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);     \
      std::fprintf(stderr, __VA_ARGS__);                            \
      std::fprintf(stderr, "\n");                                   \
      ++g_fail;                                                     \
      return;                                                       \
    }                                                               \
  } while (0)

const size_t kCu = 163840;  // LDS per CU on gfx950

void class_cases() {
  const int tiles[3] = {8, 4, 2}, grids[2] = {4, 2};
  struct Case {
    size_t lds;
    int tile, grid;
  } cases[] = {{1, 0, 0},          {20480, 0, 0},     {20481, 1, 0},     {40960, 1, 0},
               {40961, 2, 1},      {81920, 2, 1},     {81921, 3, 2},     {163840, 3, 2}};
  for (const Case& c : cases) {
    CHECK(lds_class(c.lds, kCu, tiles, 3) == c.tile, "tile class of %zu bytes", c.lds);
    CHECK(lds_class(c.lds, kCu, grids, 2) == c.grid, "grid class of %zu bytes", c.lds);
  }
}

std::vector<uint32_t> blocks(uint32_t tag, size_t n) {
  std::vector<uint32_t> v(n);
  for (size_t i = 0; i < n; ++i) v[i] = tag << 16 | (uint32_t)i;
  return v;
}

void merge_cases() {
  {  // every class fills the device: nothing moves
    std::vector<uint32_t> c[4] = {blocks(0, 300), blocks(1, 256), blocks(2, 999), blocks(3, 1)};
    size_t l[4] = {10, 20, 30, 40};
    merge_small_classes(c, l, 4, 256);
    CHECK(c[0].size() == 300 && c[1].size() == 256 && c[2].size() == 999 && c[3].size() == 1, "large classes moved");
    CHECK(l[3] == 40, "lds changed");
  }
  {  // a small class skips an empty one and lands after the next class's own blocks
    std::vector<uint32_t> c[4] = {blocks(0, 5), {}, blocks(2, 300), blocks(3, 400)};
    size_t l[4] = {50, 0, 30, 90};
    merge_small_classes(c, l, 4, 256);
    CHECK(c[0].empty() && c[1].empty() && c[2].size() == 305 && c[3].size() == 400, "sizes after merge");
    CHECK(c[2][299] == (2u << 16 | 299u) && c[2][300] == 0u, "appended after the class's own blocks");
    CHECK(l[2] == 50, "merged class keeps the larger LDS (%zu)", l[2]);
  }
  {  // all small: everything ends in the largest non-empty class
    std::vector<uint32_t> c[4] = {blocks(0, 3), blocks(1, 4), blocks(2, 5), {}};
    size_t l[4] = {1, 2, 3, 0};
    merge_small_classes(c, l, 4, 256);
    CHECK(c[0].empty() && c[1].empty() && c[2].size() == 12 && c[3].empty(), "all into class 2");
    CHECK(l[2] == 3, "lds %zu", l[2]);
  }
}

// Random classes: the blocks are kept (each in a class at least its own),
// only the largest non-empty class may stay below the minimum, and a
// class's LDS covers every block it holds.
void random_cases() {
  std::mt19937 rng(7);
  for (int it = 0; it < 2000 && !g_fail; ++it) {
    const int ncls = 2 + (int)(rng() % 3);
    const size_t minb = 1 + rng() % 300;
    std::vector<std::vector<uint32_t>> c(ncls);
    std::vector<size_t> l(ncls, 0);
    std::map<uint32_t, int> orig;
    std::map<uint32_t, size_t> need;
    for (int q = 0; q < ncls; ++q) {
      const size_t n = rng() % 4 == 0 ? 0 : rng() % 500;
      c[q] = blocks((uint32_t)q, n);
      l[q] = n ? 1 + rng() % 100000 : 0;
      for (uint32_t b : c[q]) {
        orig[b] = q;
        need[b] = l[q];
      }
    }
    merge_small_classes(c.data(), l.data(), ncls, minb);
    size_t total = 0;
    int last = -1;
    for (int q = 0; q < ncls; ++q)
      if (!c[q].empty()) last = q;
    for (int q = 0; q < ncls; ++q) {
      total += c[q].size();
      CHECK(c[q].empty() || c[q].size() >= minb || q == last, "iteration %d: class %d keeps %zu < %zu blocks", it,
            q, c[q].size(), minb);
      for (uint32_t b : c[q]) {
        CHECK(orig.count(b) && orig[b] <= q, "iteration %d: block moved down or appeared", it);
        CHECK(l[q] >= need[b], "iteration %d: class %d LDS %zu below its block's %zu", it, q, l[q], need[b]);
      }
    }
    CHECK(total == orig.size(), "iteration %d: %zu blocks instead of %zu", it, total, orig.size());
  }
}

}  // namespace

int main() {
  class_cases();
  if (!g_fail) merge_cases();
  if (!g_fail) random_cases();
  if (g_fail) return 1;
  std::printf("ok\n");
  return 0;
}
