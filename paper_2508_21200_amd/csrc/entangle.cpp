// Entanglement measures of a two-spin reduced density matrix (Sec. 3.6: the
// paper takes concurrence, negativity and nonlocality of the 4 x 4 R_kl).
// Host code on 4 x 4 complex matrices, index q = 2 b_k + b_l.
#include <algorithm>
#include <cmath>
#include <complex>

#include "lrei_internal.h"

namespace {

using cd = std::complex<double>;

// Hermitian n x n (n <= 4) eigen-decomposition by cyclic Jacobi rotations:
// on return A is diagonal (w its diagonal) and A_in = V diag(w) V*.
void herm_eig(int n, cd A[4][4], double w[4], cd V[4][4]) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0, dia = 0;
    for (int i = 0; i < n; ++i) {
      dia += std::norm(A[i][i]);
      for (int j = i + 1; j < n; ++j) off += std::norm(A[i][j]);
    }
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double b = std::abs(A[p][q]);
        if (b == 0.0) continue;
        // D = diag(1, e^{-i phi}) makes the 2 x 2 block real; then a real
        // rotation [[c, s], [-s, c]] zeroes it: U = D R
        const cd ph = A[p][q] / b;
        const double tau = (A[q][q].real() - A[p][p].real()) / (2.0 * b);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        const cd u00 = c, u01 = s, u10 = -s * std::conj(ph), u11 = c * std::conj(ph);
        for (int k = 0; k < n; ++k) {  // A <- A U, V <- V U
          const cd ap = A[k][p], aq = A[k][q];
          A[k][p] = ap * u00 + aq * u10;
          A[k][q] = ap * u01 + aq * u11;
          const cd vp = V[k][p], vq = V[k][q];
          V[k][p] = vp * u00 + vq * u10;
          V[k][q] = vp * u01 + vq * u11;
        }
        for (int k = 0; k < n; ++k) {  // A <- U* A
          const cd ap = A[p][k], aq = A[q][k];
          A[p][k] = std::conj(u00) * ap + std::conj(u10) * aq;
          A[q][k] = std::conj(u01) * ap + std::conj(u11) * aq;
        }
        A[p][q] = A[q][p] = 0.0;
      }
  }
  for (int i = 0; i < n; ++i) w[i] = A[i][i].real();
}

}  // namespace

extern "C" lrei_status lrei_pair_entanglement(const double *R, double *concurrence, double *negativity,
                                              double *chsh) {
  if (!R) return LREI_E_INVALID;
  cd M[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) M[i][j] = cd(R[2 * (4 * i + j)], R[2 * (4 * i + j) + 1]);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      if (!std::isfinite(M[i][j].real()) || !std::isfinite(M[i][j].imag())) return LREI_E_INVALID;
  if (concurrence) {
    // eigenvalues of sqrt(R) Rt sqrt(R), Rt = (sy x sy) conj(R) (sy x sy),
    // equal those of R Rt (Wootters)
    cd A[4][4], V[4][4];
    double w[4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) A[i][j] = 0.5 * (M[i][j] + std::conj(M[j][i]));
    herm_eig(4, A, w, V);
    cd S[4][4];  // sqrt(R)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        cd x = 0;
        for (int k = 0; k < 4; ++k) x += V[i][k] * std::sqrt(std::max(w[k], 0.0)) * std::conj(V[j][k]);
        S[i][j] = x;
      }
    // sy x sy = antidiagonal (-1, 1, 1, -1): (Y X Y)[i][j] = y_i y_j X[3-i][3-j]
    const double y[4] = {-1, 1, 1, -1};
    cd Rt[4][4], T[4][4], B[4][4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) Rt[i][j] = y[i] * y[j] * std::conj(M[3 - i][3 - j]);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        cd x = 0;
        for (int k = 0; k < 4; ++k) x += Rt[i][k] * S[k][j];
        T[i][j] = x;
      }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        cd x = 0;
        for (int k = 0; k < 4; ++k) x += S[i][k] * T[k][j];
        B[i][j] = x;
      }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) A[i][j] = 0.5 * (B[i][j] + std::conj(B[j][i]));
    herm_eig(4, A, w, V);
    double l[4];
    for (int i = 0; i < 4; ++i) l[i] = std::sqrt(std::max(w[i], 0.0));
    std::sort(l, l + 4, [](double a, double b) { return a > b; });
    *concurrence = std::max(0.0, l[0] - l[1] - l[2] - l[3]);
  }
  if (negativity) {
    // partial transpose on the second spin: PT[(i j)][(i' j')] = R[(i j')][(i' j)]
    cd A[4][4], V[4][4];
    double w[4];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int i2 = 0; i2 < 2; ++i2)
          for (int j2 = 0; j2 < 2; ++j2) A[2 * i + j][2 * i2 + j2] = M[2 * i + j2][2 * i2 + j];
    for (int i = 0; i < 4; ++i)
      for (int j = i; j < 4; ++j) {
        const cd h = 0.5 * (A[i][j] + std::conj(A[j][i]));
        A[i][j] = h;
        A[j][i] = std::conj(h);
      }
    herm_eig(4, A, w, V);
    double ng = 0;
    for (int i = 0; i < 4; ++i)
      if (w[i] < 0) ng -= w[i];
    *negativity = ng;
  }
  if (chsh) {
    // T_ij = Re Tr(R s_i x s_j); the largest CHSH value is 2 sqrt(m1 + m2),
    // m1 >= m2 the two largest eigenvalues of T^T T (Horodecki)
    const cd I(0, 1);
    const cd s[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    double Tm[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        cd tr = 0;  // Tr(R (s_a x s_b)) = sum_{pq} R[p][q] (s_a x s_b)[q][p]
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            for (int i2 = 0; i2 < 2; ++i2)
              for (int j2 = 0; j2 < 2; ++j2) tr += M[2 * i + j][2 * i2 + j2] * s[a][i2][i] * s[b][j2][j];
        Tm[a][b] = tr.real();
      }
    cd A[4][4], V[4][4];
    double w[4];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double x = 0;
        for (int k = 0; k < 3; ++k) x += Tm[k][i] * Tm[k][j];
        A[i][j] = x;
      }
    herm_eig(3, A, w, V);
    std::sort(w, w + 3, [](double a, double b) { return a > b; });
    *chsh = 2.0 * std::sqrt(std::max(w[0] + w[1], 0.0));
  }
  return LREI_OK;
}
