// Launch classes of a batch's binning stage, as pure functions: no HIP, so
// they are tested on the CPU (tests/batch_classes_test.cpp).
//
// A batch group's tile binning (or whole-grid binning) runs as one launch
// per class of the LDS its requests' tiles (or grids) take: class q holds
// the requests whose LDS fits 'shares[q]' times in a CU's LDS, the last
// class the rest.  Smaller LDS classes run more, smaller workgroups per CU.
// The class launches run one after another, so a class with fewer blocks
// than the device has CUs would leave most of it idle for its launch: its
// blocks join the next larger non-empty class instead, whose workgroups
// are larger and whose LDS covers theirs.  (The largest non-empty class
// keeps its own launch.)  A batch of a few requests the server gathered
// then runs as one or two launches, as a batch of hundreds runs as one per
// class.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace binimpl {

// The class of a request whose tile or grid takes 'lds' bytes: the first q
// with shares[q] * lds <= cu_lds (shares decreasing), else nshares.
inline int lds_class(size_t lds, size_t cu_lds, const int* shares, int nshares) {
  for (int q = 0; q < nshares; ++q)
    if ((size_t)shares[q] * lds <= cu_lds) return q;
  return nshares;
}

// Moves the blocks of every class with fewer than min_blocks blocks into the
// next larger non-empty class (in order, after that class's own blocks) and
// raises that class's LDS to cover them.
inline void merge_small_classes(std::vector<uint32_t>* cls, size_t* lds, int ncls, size_t min_blocks) {
  for (int q = 0; q + 1 < ncls; ++q) {
    if (cls[q].empty() || cls[q].size() >= min_blocks) continue;
    int up = q + 1;
    while (up < ncls && cls[up].empty()) ++up;
    if (up == ncls) continue;
    cls[up].insert(cls[up].end(), cls[q].begin(), cls[q].end());
    lds[up] = std::max(lds[up], lds[q]);
    cls[q].clear();
  }
}

}  // namespace binimpl
