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

// Site -> row-bit map for the tiled H.V pass, which keeps the 2^k rows that
// share their bits above k in LDS, so a bond whose two sites both map to the
// low k bits reads its partner rows there.  The low bits therefore go to the
// k-site set with the most bonds inside it (searched exhaustively where the
// number of k-subsets is small, else by greedy growth from every site plus
// improving swaps), k = min(k_cluster, n); within that set and after it the
// sites follow greedy growth order (most bonds into the sites already placed),
// so every shorter prefix is a dense cluster too and the next row bits go to
// the remote sites most tied to the tile (their partner tiles are the nearest
// ones).  The last sites of the order -- the fewest ties -- take the top bits,
// which pick the XCD a row block runs on.
std::vector<int> choose_site_order_cluster(int n, int n_bonds, const int32_t *bond_ij, int k_cluster) {
  std::vector<uint32_t> bm;
  std::vector<std::vector<int>> adj(n);
  for (int b = 0; b < n_bonds; ++b) {
    const int i = bond_ij[2 * b], j = bond_ij[2 * b + 1];
    if (i == j) continue;
    bm.push_back((1u << i) | (1u << j));
    adj[i].push_back(j);
    adj[j].push_back(i);
  }
  const int k = std::max(0, std::min(k_cluster, n));
  auto inside = [&](uint32_t set) {
    int c = 0;
    for (uint32_t m : bm) c += (m & ~set) == 0;
    return c;
  };
  uint32_t best = 0;
  int bestc = -1;
  double combos = 1;
  for (int i = 0; i < k; ++i) combos = combos * (n - i) / (i + 1);
  if (k > 0 && combos <= 3e6) {
    // every k-subset in lexicographic order (Gosper's hack on the bit set)
    uint32_t set = (k == 32) ? ~0u : ((1u << k) - 1);
    const uint32_t limit = (n == 32) ? ~0u : (1u << n);
    while (true) {
      const int c = inside(set);
      if (c > bestc) {
        bestc = c;
        best = set;
      }
      const uint32_t lo = set & (~set + 1), hi = set + lo;
      if (hi == 0 || hi >= limit) break;
      set = (((hi ^ set) >> 2) / lo) | hi;
      if (set >= limit) break;
    }
  } else if (k > 0) {
    for (int s0 = 0; s0 < n; ++s0) {
      uint32_t set = 1u << s0;
      for (int c = 1; c < k; ++c) {
        int bq = -1, bt = -1;
        for (int q = 0; q < n; ++q) {
          if (set & (1u << q)) continue;
          int t = 0;
          for (int nb : adj[q]) t += (set >> nb) & 1;
          if (t > bt) {
            bt = t;
            bq = q;
          }
        }
        set |= 1u << bq;
      }
      for (bool improved = true; improved;) {  // swaps that add inside bonds
        improved = false;
        const int c0 = inside(set);
        for (int a = 0; a < n && !improved; ++a) {
          if (!(set & (1u << a))) continue;
          for (int b = 0; b < n && !improved; ++b) {
            if (set & (1u << b)) continue;
            const uint32_t t = (set & ~(1u << a)) | (1u << b);
            if (inside(t) > c0) {
              set = t;
              improved = true;
            }
          }
        }
      }
      const int c = inside(set);
      if (c > bestc) {
        bestc = c;
        best = set;
      }
    }
  }
  // growth order: inside the cluster first, then the rest; ties to the site
  // with the fewest bonds to unplaced sites, then the lower index
  std::vector<int> order;
  uint32_t placed = 0;
  for (int phase = 0; phase < 2; ++phase) {
    while (true) {
      int bq = -1, bt = -1, bo = 1 << 30;
      for (int q = 0; q < n; ++q) {
        if (placed & (1u << q)) continue;
        if (phase == 0 && !(best & (1u << q))) continue;
        int t = 0, o = 0;
        for (int nb : adj[q]) {
          if ((placed >> nb) & 1) ++t;
          else ++o;
        }
        if (t > bt || (t == bt && o < bo)) {
          bt = t;
          bo = o;
          bq = q;
        }
      }
      if (bq < 0) break;
      placed |= 1u << bq;
      order.push_back(bq);
    }
  }
  std::vector<int> pos(n);
  for (int i = 0; i < n; ++i) pos[order[i]] = i;
  return pos;
}

}  // namespace lrei
