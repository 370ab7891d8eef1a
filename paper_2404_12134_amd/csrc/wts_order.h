// wts_order.h -- pop order of the persistent strip sweeps (host code).
//
// A sweep's waves pop (pair, strip) items from one list in list order.  A
// strip waits on its neighbour strip of the same pair (the one above it in a
// forward sweep, below it in the Soft-DTW backward), so the list must put
// every strip after that neighbour: a wait is then always on an item some
// running wave already holds, and no order of completion can deadlock.
//
// Within that constraint the order is a critical-path list schedule.  Every
// strip is keyed by the length, in sweep steps, of the chain it heads: its
// own columns plus kStripSpacing for each strip of its pair still to come
// after it.  Strips are popped by decreasing key.  Long pairs start early and
// finish early instead of forming the tail, and pairs of similar length
// interleave strip by strip, so a strip is rarely popped before the strip it
// waits on has moved ahead.  Keys strictly shrink along a pair's own order,
// so the constraint above holds by construction.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace wts {

// Assumed spacing, in sweep steps, between the starts of two consecutive
// strips of one pair in the schedule model.  A strip can start about one
// wave skew (64 steps) plus a row handoff after its neighbour; the order
// keeps about ten times that.  Spacings of 400 to 800 time alike on pairs of
// even lengths; 800 is the fastest on lengths spread 1k-20k.
constexpr int64_t kStripSpacing = 800;

// cols[q]: steps one strip of pair q takes (its columns plus the wave skew);
// strips[q]: its strip count (0 allowed).  Calls emit(q, s) once per strip,
// in pop order; with `reverse` each pair's strips come last-first.
// Ties: the strip earlier in its pair's own order, then the lower pair.
template <class Emit>
void pop_order(const std::vector<int64_t>& cols, const std::vector<int>& strips, bool reverse,
               Emit emit) {
  struct Head {
    int64_t key;
    int q, k;   // pair, position of the strip in its pair's own order
  };
  auto after = [](const Head& a, const Head& b) {   // max-heap on key
    if (a.key != b.key) return a.key < b.key;
    if (a.k != b.k) return a.k > b.k;
    return a.q > b.q;
  };
  auto head = [&](int q, int k) {
    return Head{cols[q] + (int64_t)(strips[q] - 1 - k) * kStripSpacing, q, k};
  };
  std::vector<Head> heap;
  heap.reserve(strips.size());
  for (size_t q = 0; q < strips.size(); ++q)
    if (strips[q] > 0) heap.push_back(head((int)q, 0));
  std::make_heap(heap.begin(), heap.end(), after);
  while (!heap.empty()) {
    std::pop_heap(heap.begin(), heap.end(), after);
    const Head h = heap.back();
    heap.pop_back();
    const int S = strips[h.q];
    emit(h.q, reverse ? S - 1 - h.k : h.k);
    if (h.k + 1 < S) {
      heap.push_back(head(h.q, h.k + 1));
      std::push_heap(heap.begin(), heap.end(), after);
    }
  }
}

}  // namespace wts
