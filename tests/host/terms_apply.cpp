// Host-only harness for the CPU tests: builds the library's Hamiltonian term
// table and applies it to a block on the CPU with the same indexing rules the
// GPU kernel uses (coefficient index = bit(x, sa) + 2 bit(x, sb) of the
// destination row).  Lets the term construction be checked without a GPU.
#include <complex>
#include <string>

#include "../../paper_2508_21200_amd/csrc/lrei_internal.h"

extern "C" __attribute__((visibility("default"))) int terms_apply(int n, int nb, const int32_t *bonds,
                                                                    const double *J, const double *h, int r,
                                                                    const double *V, double *Y, double *bound) {
  lrei::TermTable t;
  std::string err;
  if (!lrei::build_terms(n, nb, bonds, J, h, t, err)) return 1;
  const long long N = 1LL << n;
  using cd = std::complex<double>;
  const cd *X = reinterpret_cast<const cd *>(V);
  cd *out = reinterpret_cast<cd *>(Y);
  for (long long x = 0; x < N; ++x) {
    double d = 0;
    for (const auto &dt : t.diag) d += (((x >> dt.si) ^ (x >> dt.sj)) & 1) ? -dt.w : dt.w;
    for (int c = 0; c < r; ++c) out[x * r + c] = d * X[x * r + c];
    for (const auto &ot : t.off) {
      const int idx = (int)((x >> ot.sa) & 1) | ((int)((x >> ot.sb) & 1) << 1);
      const cd coef(ot.re[idx], ot.im[idx]);
      if (coef == cd(0)) continue;
      for (int c = 0; c < r; ++c) out[x * r + c] += coef * X[(x ^ (long long)ot.mask) * r + c];
    }
  }
  *bound = t.gershgorin;
  return 0;
}

// sqrt(Tr(H^2) / N) as the term table computes it (the scale of the Krylov
// recurrence).
extern "C" __attribute__((visibility("default"))) int terms_spread(int n, int nb, const int32_t *bonds,
                                                                     const double *J, const double *h,
                                                                     double *spread) {
  lrei::TermTable t;
  std::string err;
  if (!lrei::build_terms(n, nb, bonds, J, h, t, err)) return 1;
  *spread = t.spread;
  return 0;
}

// The site -> row-bit map of the tiled pass's cluster order.
extern "C" __attribute__((visibility("default"))) void site_order_cluster(int n, int nb, const int32_t *bonds,
                                                                          int k, int *pos) {
  const std::vector<int> p = lrei::choose_site_order_cluster(n, nb, bonds, k);
  for (int i = 0; i < n; ++i) pos[i] = p[i];
}
