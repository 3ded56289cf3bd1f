// Host-side symbolic analysis of the block-sparse normal equations (solver
// SPARSE), done once per problem structure, the way sparse Cholesky solvers
// separate symbolic analysis from the numeric factorisation (Section 4.2).
//
// 1. Fill-reducing ordering of the pose graph: minimum degree on the
//    elimination graph, kept explicitly as adjacency bitsets (eliminating v
//    joins its remaining neighbours into a clique).  Ties go to the smallest
//    index, so the ordering is deterministic.
// 2. Tile structure of the factor: the permuted scalar matrix (d scalars per
//    pose) is cut into ts x ts tiles; a tile is structurally non-zero if some
//    Hessian block touches it, and the set is closed under tile-level
//    elimination (the non-zero tiles below the diagonal of column J are added
//    to column parent(J) = the first of them).
// 3. Per tile column J the sorted list of non-zero tile rows (diagonal first),
//    from which the numeric phase takes its panel tasks: the triangular solve
//    of every tile in the column and the update of every pair of them.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace dnls {
namespace sym {

inline int popcount64(uint64_t x) { return __builtin_popcountll(x); }

// Minimum-degree elimination order of an undirected graph with n nodes.
// adj[v] lists the neighbours of v (duplicates and self loops are ignored).
inline std::vector<int> min_degree_order(int n, const std::vector<std::vector<int>>& adj) {
  const int W = (n + 63) / 64;
  std::vector<uint64_t> bits((size_t)n * W, 0);
  auto row = [&](int v) { return bits.data() + (size_t)v * W; };
  for (int v = 0; v < n; ++v)
    for (int u : adj[v])
      if (u != v) {
        row(v)[u >> 6] |= uint64_t(1) << (u & 63);
        row(u)[v >> 6] |= uint64_t(1) << (v & 63);
      }
  std::vector<int> deg(n), order;
  std::vector<char> done(n, 0);
  order.reserve(n);
  for (int v = 0; v < n; ++v) {
    int c = 0;
    for (int w = 0; w < W; ++w) c += popcount64(row(v)[w]);
    deg[v] = c;
  }
  std::vector<int> nb;
  for (int step = 0; step < n; ++step) {
    int best = -1;
    for (int v = 0; v < n; ++v)
      if (!done[v] && (best < 0 || deg[v] < deg[best])) best = v;
    const int v = best;
    done[v] = 1;
    order.push_back(v);
    nb.clear();
    const uint64_t* rv = row(v);
    for (int w = 0; w < W; ++w) {
      uint64_t x = rv[w];
      while (x) {
        const int b = __builtin_ctzll(x);
        nb.push_back(w * 64 + b);
        x &= x - 1;
      }
    }
    for (int u : nb) {
      uint64_t* ru = row(u);
      for (int w = 0; w < W; ++w) ru[w] |= rv[w];
      ru[u >> 6] &= ~(uint64_t(1) << (u & 63));
      ru[v >> 6] &= ~(uint64_t(1) << (v & 63));
      int c = 0;
      for (int w = 0; w < W; ++w) c += popcount64(ru[w]);
      deg[u] = c;
    }
    uint64_t* rvm = row(v);
    for (int w = 0; w < W; ++w) rvm[w] = 0;
  }
  return order;
}

// Elimination tree of the matrix with the given pattern in elimination
// order pos[] (Liu's algorithm with path compression), then a postorder of
// it: an equivalent elimination order (same fill) in which every subtree is
// contiguous, so that fixed-size tiles group related columns.
inline std::vector<int> postorder_positions(int n, const std::vector<std::vector<int>>& adj,
                                            const std::vector<int>& pos) {
  std::vector<int> inv(n);
  for (int v = 0; v < n; ++v) inv[pos[v]] = v;
  std::vector<int> parent(n, -1), anc(n, -1);
  for (int j = 0; j < n; ++j) {
    const int v = inv[j];
    for (int u : adj[v]) {
      int r = pos[u];
      if (r >= j) continue;
      while (anc[r] != -1 && anc[r] != j) {
        const int next = anc[r];
        anc[r] = j;
        r = next;
      }
      if (anc[r] == -1) {
        anc[r] = j;
        parent[r] = j;
      }
    }
  }
  std::vector<std::vector<int>> children(n);
  std::vector<int> roots;
  for (int j = 0; j < n; ++j) (parent[j] >= 0 ? children[parent[j]] : roots).push_back(j);
  std::vector<int> post;
  post.reserve(n);
  std::vector<std::pair<int, int>> stack;
  for (auto it = roots.rbegin(); it != roots.rend(); ++it) stack.emplace_back(*it, 0);
  while (!stack.empty()) {
    auto& top = stack.back();
    const int v = top.first;
    if (top.second < (int)children[v].size()) {
      const int c = children[v][top.second++];
      stack.emplace_back(c, 0);
    } else {
      post.push_back(v);
      stack.pop_back();
    }
  }
  std::vector<int> newpos(n);
  for (int k = 0; k < n; ++k) newpos[inv[post[k]]] = k;
  return newpos;
}

// Number of off-diagonal non-zero blocks in every block column of the
// Cholesky factor when the graph is eliminated in the order pos[] (bitset
// elimination: each eliminated node joins its later neighbours into a
// clique).  Indexed by elimination position.
inline std::vector<int> block_column_counts(int n, const std::vector<std::vector<int>>& adj,
                                            const std::vector<int>& pos) {
  const int W = (n + 63) / 64;
  std::vector<uint64_t> bits((size_t)n * W, 0);
  auto row = [&](int j) { return bits.data() + (size_t)j * W; };
  for (int v = 0; v < n; ++v)
    for (int u : adj[v]) {
      const int a = pos[v], b = pos[u];
      if (a < b) row(a)[b >> 6] |= uint64_t(1) << (b & 63);
      else if (b < a) row(b)[a >> 6] |= uint64_t(1) << (a & 63);
    }
  std::vector<int> cnt(n, 0);
  for (int j = 0; j < n; ++j) {
    const uint64_t* rj = row(j);
    int c = 0, first = -1;
    for (int w = 0; w < W; ++w) {
      c += popcount64(rj[w]);
      if (first < 0 && rj[w]) first = w * 64 + __builtin_ctzll(rj[w]);
    }
    cnt[j] = c;
    // the structure of column j (minus its first row) joins the first row's column
    if (first >= 0) {
      uint64_t* rp = row(first);
      for (int w = 0; w < W; ++w) rp[w] |= rj[w];
      rp[first >> 6] &= ~(uint64_t(1) << (first & 63));
    }
  }
  return cnt;
}

// Flops of the block Cholesky with d x d blocks, given the off-diagonal
// block count m_j of every block column: diagonal factor d^3/3, triangular
// solves m_j d^3, updates of the m_j (m_j + 1) / 2 block pairs 2 d^3 each.
inline double block_flops(const std::vector<int>& cnt, int d) {
  const double d3 = double(d) * d * d;
  double f = 0.0;
  for (int m : cnt) f += d3 / 3.0 + m * d3 + double(m) * (m + 1) * d3;
  return f;
}

struct TileStructure {
  int P = 0;                       // tile rows = tile columns
  std::vector<int> col_ptr;        // [P+1]
  std::vector<int> row_idx;        // tile rows of column J, sorted, diagonal first
};

// Tile pattern of the Cholesky factor of a matrix of n scalars whose
// variables occupy the scalar ranges [start[v], start[v] + size[v]) in
// elimination order; blocks lists the (variable a, variable b) pairs of the
// Hessian's non-zero off-diagonal blocks (every diagonal block is non-zero).
inline TileStructure tile_symbolic_vars(int n, int ts, const std::vector<int>& start, const std::vector<int>& size,
                                        const std::vector<std::pair<int, int>>& blocks) {
  TileStructure t;
  t.P = (n + ts - 1) / ts;
  std::vector<std::vector<int>> cols(t.P);
  auto add = [&](int I, int J) {
    if (I < J) std::swap(I, J);
    cols[J].push_back(I);
  };
  for (size_t k = 0; k < start.size(); ++k) {
    const int s0 = start[k], s1 = s0 + size[k] - 1;
    for (int I = s0 / ts; I <= s1 / ts; ++I)
      for (int J = s0 / ts; J <= s1 / ts; ++J) add(I, J);
  }
  for (const auto& ab : blocks) {
    const int ra0 = start[ab.first], ra1 = ra0 + size[ab.first] - 1;
    const int rb0 = start[ab.second], rb1 = rb0 + size[ab.second] - 1;
    for (int I = ra0 / ts; I <= ra1 / ts; ++I)
      for (int J = rb0 / ts; J <= rb1 / ts; ++J) add(I, J);
  }
  for (int J = 0; J < t.P; ++J) cols[J].push_back(J);
  // closure under tile-level elimination
  for (int J = 0; J < t.P; ++J) {
    auto& c = cols[J];
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
    if (c.size() > 1) {
      const int parent = c[1];
      for (size_t k = 1; k < c.size(); ++k) cols[parent].push_back(c[k]);
    }
  }
  t.col_ptr.assign(t.P + 1, 0);
  for (int J = 0; J < t.P; ++J) {
    t.col_ptr[J + 1] = t.col_ptr[J] + (int)cols[J].size();
    for (int I : cols[J]) t.row_idx.push_back(I);
  }
  return t;
}

// The same for npose variables of d scalars each; perm_pos[v] = position
// of pose v in the elimination order.
inline TileStructure tile_symbolic(int npose, int d, int ts, const std::vector<int>& perm_pos,
                                   const std::vector<std::pair<int, int>>& blocks) {
  std::vector<int> start(npose), size(npose, d);
  for (int k = 0; k < npose; ++k) start[k] = perm_pos[k] * d;
  return tile_symbolic_vars(npose * d, ts, start, size, blocks);
}

// Work of the numeric factorisation on this structure, in flops
// (diagonal factor + triangular solves + updates, full tiles).
inline double tile_flops(const TileStructure& t, int ts) {
  const double tile3 = double(ts) * ts * ts;
  double f = 0.0;
  for (int J = 0; J < t.P; ++J) {
    const double m = t.col_ptr[J + 1] - t.col_ptr[J] - 1;
    f += tile3 / 3.0 + m * tile3 + m * (m + 1) / 2.0 * 2.0 * tile3;
  }
  return f;
}

}  // namespace sym
}  // namespace dnls
