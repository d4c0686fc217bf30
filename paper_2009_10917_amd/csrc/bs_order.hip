// Element visiting order from the connectivity of the scatter map (host code
// of the plan set-up).  The gather of Section 5 sums, for every global node,
// the copies of that node in the elements around it; when neighbouring
// elements are visited close together in time their lines of x_L are still
// in the caches when the next row needs them.  Nothing here uses coordinates
// or the numbering of the global ids: only which elements share corners.
//
//   1. (corner id, element) pairs of every unmasked corner, radix-sorted by
//      id: each run of equal ids lists the elements around one mesh vertex.
//   2. Element graph: e and f are neighbours when they share a face, found
//      as the other element holding both ends of a diagonal of that face.
//   3. Recursive bisection: a part is ordered breadth first from a far
//      element (the last one reached by a breadth-first sweep from its first
//      element), split at the median of that order into a near and a far
//      half, and the halves are ordered the same way, near half first.  The
//      order of a part of at most `leaf` elements is its breadth-first order.

#include <algorithm>
#include <new>

#include "bs_order.h"

namespace bs {
namespace {

// LSD radix sort of 64-bit keys, 16 bits per pass, passes over zero digits skipped.
void radix_sort_u64(std::vector<uint64_t>& a, std::vector<uint64_t>& tmp) {
  const size_t n = a.size();
  tmp.resize(n);
  uint64_t any = 0;
  for (uint64_t v : a) any |= v;
  std::vector<size_t> count(1 << 16);
  for (int shift = 0; shift < 64; shift += 16) {
    if (((any >> shift) & 0xffff) == 0) continue;
    std::fill(count.begin(), count.end(), 0);
    for (uint64_t v : a) ++count[(v >> shift) & 0xffff];
    size_t run = 0;
    for (auto& c : count) {
      const size_t k = c;
      c = run;
      run += k;
    }
    for (uint64_t v : a) tmp[count[(v >> shift) & 0xffff]++] = v;
    a.swap(tmp);
  }
}

// Up to six face neighbours per element (-1: none).
struct Graph {
  std::vector<int32_t> nbr;  // [6 n]
};

// Corners c = i + 2j + 4k of a hexahedron; per face, its two diagonals.
constexpr int kFaceDiag[6][2][2] = {
    {{0, 6}, {2, 4}}, {{1, 7}, {3, 5}},  // i = 0, i = 1
    {{0, 5}, {1, 4}}, {{2, 7}, {3, 6}},  // j = 0, j = 1
    {{0, 3}, {1, 2}}, {{4, 7}, {5, 6}},  // k = 0, k = 1
};

// The face neighbours: the other element holding both corners of a
// diagonal of the face (in a conforming hexahedral mesh only the two
// elements sharing that face hold both).  A diagonal with a masked corner is
// replaced by the other one.
void build_graph(const int32_t* corners, int64_t n_elem, Graph& g) {
  std::vector<uint64_t> pairs, tmp;
  pairs.reserve(static_cast<size_t>(n_elem) * 8);
  for (int64_t e = 0; e < n_elem; ++e)
    for (int c = 0; c < 8; ++c) {
      const int32_t id = corners[8 * e + c];
      if (id >= 0) pairs.push_back(static_cast<uint64_t>(id) << 32 | static_cast<uint64_t>(e));
    }
  radix_sort_u64(pairs, tmp);
  tmp.clear();
  tmp.shrink_to_fit();
  // run [run_b, run_e) of the sorted pairs holding each (element, corner)
  const size_t np = pairs.size();
  std::vector<int64_t> run_b(static_cast<size_t>(n_elem) * 8, 0), run_e(static_cast<size_t>(n_elem) * 8, 0);
  for (size_t a = 0; a < np;) {
    const uint64_t id = pairs[a] >> 32;
    size_t b = a + 1;
    while (b < np && (pairs[b] >> 32) == id) ++b;
    for (size_t m = a; m < b; ++m) {
      const int64_t e = static_cast<int64_t>(pairs[m] & 0xffffffffu);
      for (int c = 0; c < 8; ++c)
        if (static_cast<uint64_t>(static_cast<uint32_t>(corners[8 * e + c])) == id && corners[8 * e + c] >= 0) {
          run_b[8 * e + c] = static_cast<int64_t>(a);
          run_e[8 * e + c] = static_cast<int64_t>(b);
        }
    }
    a = b;
  }
  g.nbr.assign(static_cast<size_t>(n_elem) * 6, -1);
  for (int64_t e = 0; e < n_elem; ++e)
    for (int f = 0; f < 6; ++f)
      for (int d = 0; d < 2; ++d) {
        const int c0 = kFaceDiag[f][d][0], c1 = kFaceDiag[f][d][1];
        if (corners[8 * e + c0] < 0 || corners[8 * e + c1] < 0) continue;
        int32_t found = -1;
        for (int64_t m = run_b[8 * e + c0]; m < run_e[8 * e + c0] && found < 0; ++m) {
          const int32_t h = static_cast<int32_t>(pairs[m] & 0xffffffffu);
          if (h == e) continue;
          for (int64_t q = run_b[8 * e + c1]; q < run_e[8 * e + c1]; ++q)
            if (static_cast<int32_t>(pairs[q] & 0xffffffffu) == h) {
              found = h;
              break;
            }
        }
        g.nbr[6 * e + f] = found;
        break;
      }
}

struct Mark {
  int32_t label;
  uint32_t stamp;
};

struct Bfs {
  const Graph& g;
  std::vector<Mark>& mark;
  uint32_t cur = 0;
  std::vector<int32_t> queue;

  Bfs(const Graph& g_, std::vector<Mark>& mark_) : g(g_), mark(mark_) {}

  // Breadth-first order of the elements labelled `lab` reachable from s.
  void run(int32_t s, int32_t lab) {
    ++cur;
    queue.clear();
    queue.push_back(s);
    mark[s].stamp = cur;
    for (size_t h = 0; h < queue.size(); ++h) {
      const int32_t v = queue[h];
      for (int f = 0; f < 6; ++f) {
        const int32_t w = g.nbr[6 * static_cast<int64_t>(v) + f];
        if (w < 0) continue;
        Mark& m = mark[w];
        if (m.label == lab && m.stamp != cur) {
          m.stamp = cur;
          queue.push_back(w);
        }
      }
    }
  }
};

}  // namespace

bool element_order_bisection(const int32_t* corners, int64_t n_elem, int64_t leaf, std::vector<int32_t>& rank,
                             std::string& err) {
  try {
    rank.assign(static_cast<size_t>(n_elem), 0);
    if (n_elem == 0) return true;
    if (leaf < 1) leaf = 1;
    Graph g;
    build_graph(corners, n_elem, g);
    std::vector<int32_t> ord(static_cast<size_t>(n_elem));
    std::vector<Mark> mark(static_cast<size_t>(n_elem), Mark{0, 0});
    for (int64_t e = 0; e < n_elem; ++e) ord[e] = static_cast<int32_t>(e);
    Bfs bfs(g, mark);
    struct Part {
      int64_t b, e;
      int32_t lab;
    };
    std::vector<Part> stack{{0, n_elem, 0}};
    std::vector<int32_t> old;
    int32_t next_label = 1;
    while (!stack.empty()) {
      const Part p = stack.back();
      stack.pop_back();
      const int64_t size = p.e - p.b;
      if (size <= leaf) continue;
      // a far element of the part, then the breadth-first order from it;
      // members the sweep does not reach (the part is not connected) follow
      // in their previous order
      old.assign(ord.begin() + p.b, ord.begin() + p.e);
      bfs.run(ord[p.b], p.lab);
      bfs.run(bfs.queue.back(), p.lab);
      int64_t k = p.b;
      for (int32_t v : bfs.queue) ord[k++] = v;
      if (k < p.e)
        for (int32_t v : old)
          if (mark[v].stamp != bfs.cur) ord[k++] = v;
      const int64_t mid = p.b + size / 2;
      for (int64_t i = mid; i < p.e; ++i) mark[ord[i]].label = next_label;
      stack.push_back({mid, p.e, next_label});
      stack.push_back({p.b, mid, p.lab});
      ++next_label;
    }
    for (int64_t i = 0; i < n_elem; ++i) rank[ord[i]] = static_cast<int32_t>(i);
    return true;
  } catch (const std::bad_alloc&) {
    err = "out of host memory";
    return false;
  }
}

}  // namespace bs
