// Element visiting order derived from the scatter map alone (bs_order.hip):
// host code of the plan set-up, used by bs_gs_order_elements.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace bs {

// Elements are the n_elem groups of 8 corner ids in `corners` (global ids,
// negative when a corner is masked; corner c is local node (c & 1,
// (c >> 1) & 1, c >> 2) scaled to the element's degree); two elements are
// neighbours when they share a face.  Returns in rank[e] (0 .. n_elem-1, a permutation) the
// position of element e in an order that keeps neighbours close: recursive
// bisection of the element graph, each part split at the median of its
// breadth-first distances from a far (pseudo-peripheral) element of the
// part, parts visited depth first; parts of at most `leaf` elements keep
// their breadth-first order.  Deterministic.  Returns false (with `err`)
// when memory runs out.
bool element_order_bisection(const int32_t* corners, int64_t n_elem, int64_t leaf, std::vector<int32_t>& rank,
                             std::string& err);

}  // namespace bs
