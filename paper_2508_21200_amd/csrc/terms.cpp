// Host-side construction of the matrix-free Hamiltonian term table.
//
// The Pauli-form Hamiltonian (Sec. 5, eq. 5.1 with S = hbar s / 2)
//   H = sum_b 1/2 sum_{a,c} J_b[a][c] s^a_i s^c_j + 1/2 sum_i h_i . s_i
// maps basis row x to rows x ^ mask with coefficients fixed by a few bits of
// x.  Matrix elements used (basis |0> = up, |1> = down):
//   <b| s^x |1-b> = 1,  <b| s^y |1-b> = -i (b = 0), +i (b = 1),  <b| s^z |b> = 1 - 2b.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <tuple>

#include "lrei_internal.h"

namespace lrei {

namespace {

using cd = std::complex<double>;

cd flip_elem(int axis, int b) {  // <b| s^axis |1-b> for axis in {x, y}
  if (axis == 0) return cd(1.0, 0.0);
  return b == 0 ? cd(0.0, -1.0) : cd(0.0, 1.0);
}

struct Acc {
  cd c[4] = {cd(0), cd(0), cd(0), cd(0)};
};

}  // namespace

bool build_terms(int n, int n_bonds, const int32_t *bond_ij, const double *bond_J,
                 const double *site_h, TermTable &out, std::string &err) {
  if (n < 1 || n > 30) {
    err = "n_spins must be in [1, 30]";
    return false;
  }
  if (n_bonds < 0 || (n_bonds > 0 && (!bond_ij || !bond_J))) {
    err = "invalid bond arrays";
    return false;
  }
  std::map<std::tuple<uint32_t, uint32_t, uint32_t>, Acc> off;  // (mask, sa, sb)
  std::vector<DiagTerm> diag;
  for (int k = 0; k < n_bonds; ++k) {
    int i = bond_ij[2 * k], j = bond_ij[2 * k + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i >= j) {
      err = "bond " + std::to_string(k) + " must satisfy 0 <= i < j < n";
      return false;
    }
    const double *J = bond_J + 9 * k;
    for (int q = 0; q < 9; ++q)
      if (!std::isfinite(J[q])) {
        err = "non-finite coupling in bond " + std::to_string(k);
        return false;
      }
    const uint32_t mi = 1u << i, mj = 1u << j;
    if (J[8] != 0.0) diag.push_back({(uint32_t)i, (uint32_t)j, 0.5 * J[8]});
    for (int a = 0; a < 3; ++a) {
      for (int c = 0; c < 3; ++c) {
        double w = 0.5 * J[3 * a + c];
        if (w == 0.0 || (a == 2 && c == 2)) continue;
        for (int bi = 0; bi < 2; ++bi) {
          for (int bj = 0; bj < 2; ++bj) {
            if (a < 2 && c < 2) {
              off[{mi | mj, (uint32_t)i, (uint32_t)j}].c[bi + 2 * bj] +=
                  w * flip_elem(a, bi) * flip_elem(c, bj);
            } else if (a < 2) {  // flip site i, s^z on site j
              off[{mi, (uint32_t)i, (uint32_t)j}].c[bi + 2 * bj] +=
                  w * flip_elem(a, bi) * double(1 - 2 * bj);
            } else {  // s^z on site i, flip site j
              off[{mj, (uint32_t)j, (uint32_t)i}].c[bj + 2 * bi] +=
                  w * double(1 - 2 * bi) * flip_elem(c, bj);
            }
          }
        }
      }
    }
  }
  if (site_h) {
    for (int i = 0; i < n; ++i) {
      const double *h = site_h + 3 * i;
      for (int q = 0; q < 3; ++q)
        if (!std::isfinite(h[q])) {
          err = "non-finite field on site " + std::to_string(i);
          return false;
        }
      if (h[2] != 0.0) diag.push_back({(uint32_t)i, 31u, 0.5 * h[2]});
      if (h[0] == 0.0 && h[1] == 0.0) continue;
      cd f0 = 0.5 * (h[0] * flip_elem(0, 0) + h[1] * flip_elem(1, 0));
      cd f1 = 0.5 * (h[0] * flip_elem(0, 1) + h[1] * flip_elem(1, 1));
      const uint32_t mi = 1u << i;
      // Fold into an existing one-flip term on the same site (any partner bit).
      bool folded = false;
      for (auto &kv : off) {
        if (std::get<0>(kv.first) == mi && std::get<1>(kv.first) == (uint32_t)i) {
          for (int bj = 0; bj < 2; ++bj) {
            kv.second.c[0 + 2 * bj] += f0;
            kv.second.c[1 + 2 * bj] += f1;
          }
          folded = true;
          break;
        }
      }
      if (!folded) {
        Acc &acc = off[{mi, (uint32_t)i, (uint32_t)i}];
        acc.c[0] += f0;  // index b + 2b with sa = sb = i
        acc.c[3] += f1;
      }
    }
  }
  out.off.clear();
  out.diag = diag;
  double bound = 0.0;
  for (const auto &d : diag) bound += std::fabs(d.w);
  for (const auto &kv : off) {
    OffTerm t;
    t.mask = std::get<0>(kv.first);
    t.sa = std::get<1>(kv.first);
    t.sb = std::get<2>(kv.first);
    double mx = 0.0;
    for (int q = 0; q < 4; ++q) {
      t.re[q] = kv.second.c[q].real();
      t.im[q] = kv.second.c[q].imag();
      mx = std::max(mx, std::abs(kv.second.c[q]));
    }
    if (mx == 0.0) continue;
    bound += mx;
    out.off.push_back(t);
  }
  out.gershgorin = bound;
  // Tr(H^2) / N = mean over rows of d(x)^2 + sum_t |c_t(x)|^2.  Distinct
  // z-strings (parities of bit sets {si, sj}) are orthogonal over the rows, so
  // mean d^2 is the sum over distinct strings of their summed weight squared;
  // a one-site term's coefficient takes its two diagonal entries with equal
  // frequency, a two-site term's its four.
  std::map<std::pair<uint32_t, uint32_t>, double> zw;
  for (const auto &d : diag) {
    const uint32_t a = std::min(d.si, d.sj), b = std::max(d.si, d.sj);
    zw[{a, b}] += d.w;
  }
  double tr2 = 0.0;
  for (const auto &kv : zw) tr2 += kv.second * kv.second;
  for (const auto &t : out.off) {
    auto m2 = [&](int q) { return t.re[q] * t.re[q] + t.im[q] * t.im[q]; };
    tr2 += t.sa == t.sb ? 0.5 * (m2(0) + m2(3)) : 0.25 * (m2(0) + m2(1) + m2(2) + m2(3));
  }
  out.spread = std::sqrt(tr2);
  return true;
}

}  // namespace lrei
