// Site -> row-bit order of the internal storage (the row layout the H.V
// pass walks).  Kept apart from the API code: the stored traffic figures of
// the H.V pass are tied to this file and the kernel source.
#include <algorithm>
#include <tuple>
#include <vector>

#include "lrei_internal.h"

namespace lrei {

// Site -> row-bit map of the internal storage order.  The n - 14 highest bits
// (the bits that change between the row blocks an XCD works on at one time)
// go to sites that share no term where possible, so that every flip mask
// touches at most one of them and the rows gathered across blocks fall into
// few distinct partner blocks.  Greedy: minimum-degree sites first.
std::vector<int> choose_site_order(int n, int n_bonds, const int32_t *bond_ij) {
  std::vector<int> pos(n);
  const int nh = n > 14 ? n - 14 : 0;
  std::vector<std::vector<int>> adj(n);
  for (int b = 0; b < n_bonds; ++b) {
    const int i = bond_ij[2 * b], j = bond_ij[2 * b + 1];
    if (i == j) continue;
    adj[i].push_back(j);
    adj[j].push_back(i);
  }
  std::vector<char> inH(n, 0), blocked(n, 0);
  int cnt = 0;
  while (cnt < nh) {
    int best = -1;
    for (int q = n - 1; q >= 0; --q)
      if (!blocked[q] && (best < 0 || adj[q].size() < adj[best].size())) best = q;
    if (best < 0) break;
    inH[best] = blocked[best] = 1;
    for (int nb : adj[best]) blocked[nb] = 1;
    ++cnt;
  }
  while (cnt < nh) {
    int best = -1, bestc = 1 << 30;
    for (int q = n - 1; q >= 0; --q) {
      if (inH[q]) continue;
      int c = 0;
      for (int nb : adj[q]) c += inH[nb];
      if (c < bestc) {
        bestc = c;
        best = q;
      }
    }
    inH[best] = 1;
    ++cnt;
  }
  // The top three row bits pick the XCD that owns a row, so every bond of
  // those three "selector" sites gathers from another XCD's rows.  Take as
  // selectors the three high sites with the fewest distinct neighbours, and
  // give the low row bits first to the selectors' neighbours, then to the
  // other high sites' neighbours: the bonds of one far site then read the
  // same remote lines for rows that are processed close together, and those
  // lines are still in L2 (on the 4 x 5 lattice: 12 % less fabric traffic).
  std::vector<int> H, S;
  for (int q = 0; q < n; ++q)
    if (inH[q]) H.push_back(q);
  auto nbr_union = [&](const std::vector<int> &set) {
    std::vector<char> m(n, 0);
    int c = 0;
    for (int h : set)
      for (int nb : adj[h])
        if (!m[nb]) {
          m[nb] = 1;
          ++c;
        }
    return c;
  };
  if ((int)H.size() <= 3) {
    S = H;
  } else {
    int best = 1 << 30;
    const int m = (int)H.size();
    for (int a = 0; a < m; ++a)
      for (int b = a + 1; b < m; ++b)
        for (int c = b + 1; c < m; ++c) {
          const int u = nbr_union({H[a], H[b], H[c]});
          if (u < best) {
            best = u;
            S = {H[a], H[b], H[c]};
          }
        }
  }
  std::vector<char> inS(n, 0);
  for (int q : S) inS[q] = 1;
  std::vector<int> low;
  for (int q = 0; q < n; ++q)
    if (!inH[q]) low.push_back(q);
  auto cls = [&](int q) {
    int sel = 0, high = 0;
    for (int nb : adj[q]) {
      sel += inS[nb];
      high += inH[nb];
    }
    return std::make_tuple(sel > 0 ? 0 : (high > 0 ? 1 : 2), -high, q);
  };
  std::stable_sort(low.begin(), low.end(), [&](int x, int y) { return cls(x) < cls(y); });
  int k = 0;
  for (int q : low) pos[q] = k++;
  for (int q : H)
    if (!inS[q]) pos[q] = k++;
  for (int q : S) pos[q] = k++;
  return pos;
}

}  // namespace lrei
