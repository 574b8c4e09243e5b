// Host-side geometry of the recursive partition (no device code).
//
// Level 0 nodes are the time steps of every instance.  Level 0 is cut into
// chunks of L0 nodes and every higher level into chunks of L1 nodes.  Every
// chunk but an instance's last one ends in a separator node, and the
// separators of level l are the nodes of level l+1.  An instance with no more
// nodes than the chunk length at some level is a single chunk there and is
// solved directly by that level's back-substitution.
#pragma once

#include <stdint.h>

#include <vector>

namespace smnn {

struct Level {
  std::vector<int64_t> n;          // nodes per instance
  std::vector<int64_t> node_off;   // [N+1] exclusive prefix sum of n
  std::vector<int64_t> chunk_off;  // [N+1] exclusive prefix sum of chunks per instance
  std::vector<int32_t> chunk_inst; // [chunks] owning instance of each chunk
  int64_t nodes = 0, chunks = 0;
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Levels for step counts T (all >= 1) and chunk lengths L0 (level 0) and
// L1 (levels >= 1), both >= 2.
inline std::vector<Level> build_levels(const std::vector<int64_t>& T, int L0, int L1) {
  std::vector<Level> lv;
  std::vector<int64_t> n = T;
  const size_t N = T.size();
  for (;;) {
    const int L = lv.empty() ? L0 : L1;
    Level l;
    l.n = n;
    l.node_off.assign(N + 1, 0);
    l.chunk_off.assign(N + 1, 0);
    std::vector<int64_t> next(N, 0);
    bool any_next = false;
    for (size_t i = 0; i < N; ++i) {
      const int64_t g = n[i] > 0 ? ceil_div(n[i], L) : 0;
      l.node_off[i + 1] = l.node_off[i] + n[i];
      l.chunk_off[i + 1] = l.chunk_off[i] + g;
      next[i] = n[i] > L ? g - 1 : 0;
      any_next = any_next || next[i] > 0;
    }
    l.nodes = l.node_off[N];
    l.chunks = l.chunk_off[N];
    l.chunk_inst.resize(l.chunks);
    for (size_t i = 0; i < N; ++i)
      for (int64_t c = l.chunk_off[i]; c < l.chunk_off[i + 1]; ++c) l.chunk_inst[c] = (int32_t)i;
    lv.push_back(std::move(l));
    if (!any_next) break;
    n = next;
  }
  return lv;
}

// Time step (0-based, within its instance) of node `node` of level `level`:
// separator j of level l is node (j+1) L - 1 of level l-1, L the chunk
// length of level l-1.
inline int64_t node_step(int level, int64_t node, int L0, int L1) {
  int64_t s = node;
  for (int l = level; l > 0; --l) s = (s + 1) * (l == 1 ? L0 : L1) - 1;
  return s;
}

}  // namespace smnn
