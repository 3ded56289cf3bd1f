// CPU driver for the host symbolic analysis (tests only): reads
//   npose d ts m  then m lines "a b" (pose pairs)
// and prints the minimum-degree order, the tile structure and the block
// column counts of the factor.
#include <cstdio>
#include <utility>
#include <vector>

#include "../../paper_2207_09442_amd/csrc/symbolic.hpp"

int main(int argc, char**) {
  int n, d, ts, m;
  if (std::scanf("%d %d %d %d", &n, &d, &ts, &m) != 4) return 1;
  std::vector<std::vector<int>> adj(n);
  std::vector<std::pair<int, int>> blocks;
  for (int k = 0; k < m; ++k) {
    int a, b;
    if (std::scanf("%d %d", &a, &b) != 2) return 1;
    adj[a].push_back(b);
    adj[b].push_back(a);
    blocks.emplace_back(a, b);
  }
  const std::vector<int> order = dnls::sym::min_degree_order(n, adj);
  std::vector<int> pos(n);
  for (int k = 0; k < n; ++k) pos[order[k]] = k;
  const bool post = (argc > 1);
  if (post) pos = dnls::sym::postorder_positions(n, adj, pos);
  std::vector<int> final_order(n);
  for (int v = 0; v < n; ++v) final_order[pos[v]] = v;
  const dnls::sym::TileStructure t = dnls::sym::tile_symbolic(n, d, ts, pos, blocks);
  std::printf("order");
  for (int v : (post ? final_order : order)) std::printf(" %d", v);
  std::printf("\nP %d\ncol_ptr", t.P);
  for (int v : t.col_ptr) std::printf(" %d", v);
  std::printf("\nrow_idx");
  for (int v : t.row_idx) std::printf(" %d", v);
  std::printf("\nflops %.6e\n", dnls::sym::tile_flops(t, ts));
  const std::vector<int> cnt = dnls::sym::block_column_counts(n, adj, pos);
  std::printf("counts");
  for (int v : cnt) std::printf(" %d", v);
  std::printf("\nblock_flops %.6e\n", dnls::sym::block_flops(cnt, d));
  return 0;
}
