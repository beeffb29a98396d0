// Projected (small-space) part of one LREI-RK step, in FP64 on one workgroup.
//
// All stage factors of one RK step lie in the block Krylov space of H started
// from the current support V_1: V_1 is in it, f(K_j) = Z_j V_j* + V_j W_j*
// only adds H V_j, and V_{j+1} is spanned by V_1..V_j, W_1..W_j.  The N-space
// passes build that space as the Chebyshev blocks P_0 = V_1, P_1, ..., P_s and
// measure their Gram products; this kernel then runs the paper's step
// (eqs. 3.2/4.1, 3.3, 3.4, 3.7-3.9 and the partial eigendecomposition with the
// spectrum reset to Lambda_0) exactly, in the coordinates of an orthonormal
// basis of that space, and returns the coefficients C with V_new = [P_0..P_s] C.
//
// Steps:
//  1. Assemble the Gram matrix Gamma of the blocks from the measured products
//     and the Chebyshev recurrence; Cholesky Gamma = R* R with directions whose
//     pivot falls below 1e-13 of the diagonal treated as dependent (dropped).
//  2. Coordinates: V_1 = B R^{-1} u_1 with u_1 = R[:, :r] (R_00* R_00)^{-1/2};
//     the projected Hamiltonian acts as y = R That R^{-1} u, That being the
//     block-tridiagonal Chebyshev relation H P_j = c P_j + e (P_{j+1} + P_{j-1})/2.
//  3. For each stage: G = u* y, X11 = Phi o G, X12 coefficients c_a; the
//     complement action W = Vhat X12* through r Householder reflectors of u
//     (Sec. 3.4) (or the projector form); Z = u X11 + W; the stage matrix
//     k = u_1 Lambda_0 u_1* + h sum a_l (z_l u_l* + u_l w_l*) and its r largest
//     eigenvectors by a cyclic two-sided complex Jacobi method.
//  4. C = R^{-1} u_final.
#include <hip/hip_runtime.h>

#include "lrei_internal.h"

namespace lrei {

namespace {

constexpr int NT = 1024;
constexpr int kMaxPairs = kMaxDim / 2;

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// phi(delta): q-LL (delta/hbar)(i - kappa delta) (eq. 4.1); q-LLG (i delta/hbar)/(1 - i kappa delta)
// (eq. 3.2: D / (E + L + L*)).  X11_ab = phi(lam_a - lam_b) G_ab, X12 = diag(phi(lam)) V* H Vhat.
__device__ inline double2 phi(double d, int model, double kappa, double hbar) {
  if (model == 0) return make_double2(-kappa * d * d / hbar, d / hbar);
  // (i d / hbar) / (1 - i kappa d) = (i d / hbar)(1 + i kappa d) / (1 + kappa^2 d^2)
  const double den = hbar * (1.0 + kappa * kappa * d * d);
  return make_double2(-kappa * d * d / den, d / den);
}

// ----- workgroup-wide small dense helpers (row-major, leading dimension ld) ---

// C (m x n) = A (m x k) * B (k x n)
__device__ void gemm_nn(double2 *C, int ldc, const double2 *A, int lda, const double2 *B, int ldb,
                        int m, int n, int k) {
  for (int e = threadIdx.x; e < m * n; e += NT) {
    const int i = e / n, j = e % n;
    double2 s = make_double2(0, 0);
    for (int q = 0; q < k; ++q) s = cadd(s, cmul(A[i * lda + q], B[q * ldb + j]));
    C[i * ldc + j] = s;
  }
}
// C (m x n) = A^H (A: k x m) * B (k x n)
__device__ void gemm_hn(double2 *C, int ldc, const double2 *A, int lda, const double2 *B, int ldb,
                        int m, int n, int k) {
  for (int e = threadIdx.x; e < m * n; e += NT) {
    const int i = e / n, j = e % n;
    double2 s = make_double2(0, 0);
    for (int q = 0; q < k; ++q) s = cadd(s, cmulc(A[q * lda + i], B[q * ldb + j]));
    C[i * ldc + j] = s;
  }
}

// out[c] = sum_{i < m} conj(v[i * ldv]) M[i * ldm + c], c < nc (nc <= 32), via LDS partials
__device__ void col_dots(double2 *out, const double2 *v, int ldv, const double2 *M, int ldm, int m,
                         int nc, double2 *s_red /* NT entries */) {
  const int c = threadIdx.x % nc, slice = threadIdx.x / nc, S = NT / nc;
  double2 s = make_double2(0, 0);
  if (slice < S)
    for (int i = slice; i < m; i += S) s = cadd(s, cmulc(v[i * ldv], M[i * ldm + c]));
  s_red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < nc) {
    double2 t = make_double2(0, 0);
    for (int q = 0; q < S; ++q) t = cadd(t, s_red[q * nc + threadIdx.x]);
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// ----- complex Hermitian Jacobi (round-robin parallel ordering) ---------------

struct JacobiShared {
  int p[kMaxPairs], q[kMaxPairs];
  double cs[kMaxPairs], sn[kMaxPairs], t[kMaxPairs];
  double2 e[kMaxPairs];
  int rotated;
  int order[kMaxR];
};

__device__ inline int rr_player(int pos, int round, int mp) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (mp - 1);
}

// Diagonalises the Hermitian m x m matrix A (row-major, ld m) in place and
// accumulates V = product of rotations (V starts as identity).  Returns the
// sweep count, or -1 when max_sweeps is reached.
__device__ int jacobi(double2 *A, double2 *V, int m, double tol, int max_sweeps, JacobiShared &js) {
  const int mp = m + (m & 1), np = mp / 2;
  for (int e = threadIdx.x; e < m * m; e += NT)
    V[e] = make_double2((e / m) == (e % m) ? 1.0 : 0.0, 0.0);
  // scale = max |A_ii|
  __shared__ double s_scale;
  if (threadIdx.x == 0) {
    double sc = 0;
    for (int i = 0; i < m; ++i) sc = fmax(sc, fabs(A[i * m + i].x));
    s_scale = sc > 0 ? sc : 1.0;
  }
  __syncthreads();
  const double thresh = tol * s_scale;
  if (m == 1) return 0;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) js.rotated = 0;
    __syncthreads();
    for (int round = 0; round < mp - 1; ++round) {
      if (threadIdx.x < np) {
        const int i = threadIdx.x;
        int a = rr_player(i, round, mp), b = rr_player(mp - 1 - i, round, mp);
        const int p = a < b ? a : b, q = a < b ? b : a;
        js.p[i] = p;
        js.q[i] = q;
        double cs = 1, sn = 0, t = 0;
        double2 e = make_double2(1, 0);
        if (q < m) {
          const double2 c = A[p * m + q];
          const double x = sqrt(cabs2(c));
          if (x > thresh) {
            const double app = A[p * m + p].x, aqq = A[q * m + q].x;
            const double tau = (aqq - app) / (2.0 * x);
            t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            cs = 1.0 / sqrt(1.0 + t * t);
            sn = t * cs;
            e = make_double2(c.x / x, -c.y / x);  // e^{-i arg c}
            js.rotated = 1;
          }
        }
        js.cs[i] = cs;
        js.sn[i] = sn;
        js.t[i] = t;
        js.e[i] = e;
      }
      __syncthreads();
      // two-sided update of 2x2 blocks (P rows, Q cols); diagonal blocks exact
      for (int blk = threadIdx.x; blk < np * np; blk += NT) {
        const int P = blk / np, Q = blk % np;
        const int pP = js.p[P], qP = js.q[P], pQ = js.p[Q], qQ = js.q[Q];
        if (js.sn[P] == 0.0 && js.sn[Q] == 0.0) continue;
        if (P == Q) {
          if (qP >= m) continue;
          const double x = sqrt(cabs2(A[pP * m + qP]));
          const double app = A[pP * m + pP].x, aqq = A[qP * m + qP].x;
          A[pP * m + pP] = make_double2(app - js.t[P] * x, 0.0);
          A[qP * m + qP] = make_double2(aqq + js.t[P] * x, 0.0);
          A[pP * m + qP] = make_double2(0, 0);
          A[qP * m + pP] = make_double2(0, 0);
          continue;
        }
        const bool hq = qP < m, hqq = qQ < m;
        const double2 z = make_double2(0, 0);
        double2 a = A[pP * m + pQ];
        double2 b = hqq ? A[pP * m + qQ] : z;
        double2 c = hq ? A[qP * m + pQ] : z;
        double2 d = (hq && hqq) ? A[qP * m + qQ] : z;
        // rows: J_P^H
        const double csP = js.cs[P], snP = js.sn[P];
        const double2 ebP = cconj(js.e[P]);
        const double2 a1 = csub(cscale(csP, a), cscale(snP, cmul(ebP, c)));
        const double2 b1 = csub(cscale(csP, b), cscale(snP, cmul(ebP, d)));
        const double2 c1 = cadd(cscale(snP, a), cscale(csP, cmul(ebP, c)));
        const double2 d1 = cadd(cscale(snP, b), cscale(csP, cmul(ebP, d)));
        // cols: J_Q
        const double csQ = js.cs[Q], snQ = js.sn[Q];
        const double2 eQ = js.e[Q];
        A[pP * m + pQ] = csub(cscale(csQ, a1), cscale(snQ, cmul(eQ, b1)));
        if (hqq) A[pP * m + qQ] = cadd(cscale(snQ, a1), cscale(csQ, cmul(eQ, b1)));
        if (hq) A[qP * m + pQ] = csub(cscale(csQ, c1), cscale(snQ, cmul(eQ, d1)));
        if (hq && hqq) A[qP * m + qQ] = cadd(cscale(snQ, c1), cscale(csQ, cmul(eQ, d1)));
      }
      for (int e = threadIdx.x; e < np * m; e += NT) {
        const int P = e / m, i = e % m;
        if (js.sn[P] == 0.0) continue;
        const int p = js.p[P], q = js.q[P];
        const double2 vp = V[i * m + p], vq = V[i * m + q];
        const double cs = js.cs[P], sn = js.sn[P];
        const double2 ee = js.e[P];
        V[i * m + p] = csub(cscale(cs, vp), cscale(sn, cmul(ee, vq)));
        V[i * m + q] = cadd(cscale(sn, vp), cscale(cs, cmul(ee, vq)));
      }
      __syncthreads();
    }
    const int rot = js.rotated;
    __syncthreads();
    if (!rot) return sweep + 1;
  }
  return -1;
}

// Largest-r eigenvalues of a diagonalised A (descending) -> columns of V into u.
__device__ void take_top(const double2 *A, const double2 *V, int m, int r, double2 *u, int ldu,
                         int rows_out, JacobiShared &js) {
  if (threadIdx.x == 0) {
    bool used[kMaxDim];
    for (int i = 0; i < m; ++i) used[i] = false;
    for (int k = 0; k < r; ++k) {
      int best = -1;
      double bv = 0;
      for (int i = 0; i < m; ++i)
        if (!used[i] && (best < 0 || A[i * m + i].x > bv)) {
          best = i;
          bv = A[i * m + i].x;
        }
      used[best] = true;
      js.order[k] = best;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows_out * r; e += NT) {
    const int i = e / r, k = e % r;
    u[i * ldu + k] = i < m ? V[i * m + js.order[k]] : make_double2(0, 0);
  }
  __syncthreads();
}

}  // namespace

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(NT) void k_small_rk(SmallRkParams p, SmallWs ws) {
  extern __shared__ __align__(16) double2 s_mat[];
  __shared__ JacobiShared js;
  __shared__ double2 s_red[NT];
  __shared__ double2 s_vec[kMaxDim];
  __shared__ double s_beta[kMaxR];
  __shared__ int s_drop[kMaxDim];
  __shared__ double s_minpiv;
  __shared__ int s_ndrop;
  __shared__ double s_alpha;

  const int r = p.r, s = p.s, nb = p.nblocks, D = nb * r, rr = r * r;
  double2 *G = ws.gamma, *R = ws.R, *Ri = ws.Rinv;
  double2 *y = ws.work;                 // D x r
  double2 *t1 = y + D * r;              // D x r
  double2 *Uh = t1 + D * r;             // D x r Householder vectors
  double2 *Yc = Uh + D * r;             // D x r
  double2 *Vj = Yc + D * r;             // D x D Jacobi rotations
  double2 *Kg = Vj + D * D;             // D x D stage matrix (global fallback)
  double2 *X11 = Kg + D * D;            // r x r
  double2 *Gr = X11 + rr;               // r x r
  double2 *tmp = Gr + rr;               // r x r
  double2 *Lw = tmp + rr;               // r x r Lowdin factor
  double *stats = ws.stats;

  // ---- 1. Gram matrix of the Chebyshev blocks --------------------------------
  auto gblk = [&](int bi, int bj) { return G + (bi * r) * D + bj * r; };
  for (int e = threadIdx.x; e < D * D; e += NT) G[e] = make_double2(0, 0);
  __syncthreads();
  auto put = [&](int bi, int bj, const double2 *M) {
    for (int e = threadIdx.x; e < rr; e += NT) gblk(bi, bj)[(e / r) * D + e % r] = M[e];
  };
  put(0, 0, ws.meas + 0 * rr);
  put(0, 1, ws.meas + 1 * rr);
  put(1, 1, ws.meas + 2 * rr);
  for (int j = 1; j < s; ++j) {
    put(j - 1, j + 1, ws.meas + (3 * j + 0) * rr);
    put(j, j + 1, ws.meas + (3 * j + 1) * rr);
    put(j + 1, j + 1, ws.meas + (3 * j + 2) * rr);
  }
  __syncthreads();
  for (int j = 1; j < s; ++j) {
    // Gamma_{i, j+1} for i <= j-2 from P_{j+1} = 2 H~ P_j - P_{j-1}
    for (int e = threadIdx.x; e < (j - 1) * rr; e += NT) {
      const int i = e / rr, a = (e % rr) / r, b = e % r;
      double2 v;
      if (i == 0)
        v = csub(cscale(2.0, gblk(1, j)[a * D + b]), gblk(0, j - 1)[a * D + b]);
      else
        v = csub(cadd(gblk(i + 1, j)[a * D + b], gblk(i - 1, j)[a * D + b]), gblk(i, j - 1)[a * D + b]);
      gblk(i, j + 1)[a * D + b] = v;
    }
    __syncthreads();
  }
  // Hermitian completion (diagonal blocks symmetrised)
  for (int e = threadIdx.x; e < D * D; e += NT) {
    const int i = e / D, j = e % D;
    const int bi = i / r, bj = j / r;
    if (bi > bj) G[e] = cconj(G[j * D + i]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < D * D; e += NT) {
    const int i = e / D, j = e % D;
    if (i / r == j / r && i < j) {
      const double2 a = G[e], b = G[j * D + i];
      const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      G[e] = h;
      G[j * D + i] = cconj(h);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < D; e += NT) G[e * D + e].y = 0.0;
  __syncthreads();

  // ---- Cholesky Gamma = R^H R (R upper), dependent directions dropped -------
  for (int e = threadIdx.x; e < D * D; e += NT) R[e] = G[e];
  if (threadIdx.x == 0) {
    s_minpiv = 1.0;
    s_ndrop = 0;
  }
  __syncthreads();
  for (int k = 0; k < D; ++k) {
    if (threadIdx.x == 0) {
      const double piv = R[k * D + k].x, orig = G[k * D + k].x;
      const double ratio = orig > 0 ? piv / orig : 0.0;
      if (!(piv > 1e-13 * orig) || !(orig > 0)) {
        s_drop[k] = 1;
        s_ndrop += 1;
      } else {
        s_drop[k] = 0;
        s_minpiv = fmin(s_minpiv, ratio);
      }
    }
    __syncthreads();
    const bool dropped = s_drop[k];
    const double rkk = dropped ? 1.0 : sqrt(R[k * D + k].x);
    // row k of R
    for (int j = k + 1 + threadIdx.x; j < D; j += NT)
      R[k * D + j] = dropped ? make_double2(0, 0) : cscale(1.0 / rkk, R[k * D + j]);
    __syncthreads();
    if (threadIdx.x == 0) R[k * D + k] = make_double2(rkk, 0.0);
    // trailing update
    if (!dropped) {
      const int w = D - k - 1;
      for (int e = threadIdx.x; e < w * w; e += NT) {
        const int i = k + 1 + e / w, j = k + 1 + e % w;
        if (j >= i) R[i * D + j] = csub(R[i * D + j], cmulc(R[k * D + i], R[k * D + j]));
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < D * D; e += NT)
    if (e / D > e % D) R[e] = make_double2(0, 0);
  __syncthreads();
  // R^{-1}: column c by back substitution (one thread per column)
  for (int e = threadIdx.x; e < D * D; e += NT) Ri[e] = make_double2(0, 0);
  __syncthreads();
  for (int c = threadIdx.x; c < D; c += NT) {
    Ri[c * D + c] = cdiv(make_double2(1, 0), R[c * D + c]);
    for (int i = c - 1; i >= 0; --i) {
      double2 sum = make_double2(0, 0);
      for (int k = i + 1; k <= c; ++k) sum = cadd(sum, cmul(R[i * D + k], Ri[k * D + c]));
      Ri[i * D + c] = cdiv(make_double2(-sum.x, -sum.y), R[i * D + i]);
    }
  }
  __syncthreads();

  // ---- 2. u_1 = R[:, :r] Gamma_00^{-1/2} ------------------------------------
  double2 *u1 = ws.stage;  // stage 0, slot u
  {
    // Lowdin factor from Gamma_00 (r x r) by Jacobi; skip when already orthonormal
    __shared__ double s_dev;
    if (threadIdx.x == 0) {
      double dev = 0;
      for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b) {
          double2 g = G[a * D + b];
          if (a == b) g.x -= 1.0;
          dev = fmax(dev, sqrt(cabs2(g)));
        }
      s_dev = dev;
    }
    __syncthreads();
    const double dev = s_dev;
    if (threadIdx.x == 0) stats[4] = dev;
    if (dev > 1e-14) {
      double2 *A = s_mat;
      for (int e = threadIdx.x; e < rr; e += NT) A[e] = G[(e / r) * D + e % r];
      __syncthreads();
      jacobi(A, Vj, r, 1e-16, 60, js);
      // Lw = E diag(mu^{-1/2}) E^H
      for (int e = threadIdx.x; e < rr; e += NT) {
        const int a = e / r, b = e % r;
        double2 sacc = make_double2(0, 0);
        for (int k = 0; k < r; ++k) {
          const double mu = A[k * r + k].x;
          sacc = cadd(sacc, cscale(1.0 / sqrt(mu), cmul(Vj[a * r + k], cconj(Vj[b * r + k]))));
        }
        Lw[e] = sacc;
      }
      __syncthreads();
      gemm_nn(u1, r, R, D, Lw, r, D, r, r);
    } else {
      for (int e = threadIdx.x; e < D * r; e += NT) u1[e] = R[(e / r) * D + e % r];
    }
    __syncthreads();
  }

  // ---- 3. stages -------------------------------------------------------------
  const double h = p.h;
  double2 *cvec = s_vec;  // c_a = phi(lam_a) in s_vec[0..r)
  if (threadIdx.x < r) cvec[threadIdx.x] = phi(p.lam[threadIdx.x], p.model, p.kappa, p.hbar);
  __syncthreads();
  int total_sweeps = 0, max_sw = 0, failed = 0;
  for (int j = 0; j < s; ++j) {
    double2 *u = ws.stage + (3 * j + 0) * D * r;
    double2 *z = ws.stage + (3 * j + 1) * D * r;
    double2 *w = ws.stage + (3 * j + 2) * D * r;
    const int mi = (j + 1) * r;           // support of u
    const int mo = (j + 2) * r;           // support of y = H u
    // y = R That R^{-1} u
    gemm_nn(t1, r, Ri, D, u, r, mi, r, mi);  // rows >= mi of R^{-1} u vanish (upper triangular)
    __syncthreads();
    for (int e = threadIdx.x; e < mo * r; e += NT) {
      const int row = e / r, col = e % r, bi = row / r, a = row % r;
      double2 v = cscale(p.shift, bi <= j ? t1[e] : make_double2(0, 0));
      if (bi >= 1 && bi - 1 <= j) {
        const double coef = (bi - 1 == 0) ? p.halfwidth : 0.5 * p.halfwidth;
        v = cadd(v, cscale(coef, t1[((bi - 1) * r + a) * r + col]));
      }
      if (bi + 1 <= j) v = cadd(v, cscale(0.5 * p.halfwidth, t1[((bi + 1) * r + a) * r + col]));
      Yc[e] = v;  // That * t1 (temporarily in Yc)
    }
    __syncthreads();
    gemm_nn(y, r, R, D, Yc, r, mo, r, mo);
    __syncthreads();
    for (int e = threadIdx.x; e < mo * r; e += NT)
      if (s_drop[e / r]) y[e] = make_double2(0, 0);
    __syncthreads();
    // G = u^H y ; X11
    gemm_hn(Gr, r, u, r, y, r, r, r, mo);
    __syncthreads();
    for (int e = threadIdx.x; e < rr; e += NT) {
      const int a = e / r, b = e % r;
      const double2 g1 = Gr[a * r + b], g2 = Gr[b * r + a];
      const double2 gs = make_double2(0.5 * (g1.x + g2.x), 0.5 * (g1.y - g2.y));
      X11[e] = cmul(phi(p.lam[a] - p.lam[b], p.model, p.kappa, p.hbar), gs);
      if (a == b) X11[e] = make_double2(0, 0);
    }
    if (j == 0 && threadIdx.x == 0) {
      double en = 0;
      for (int a = 0; a < r; ++a) en += p.lam[a] * Gr[a * r + a].x;
      stats[5] = en;
    }
    __syncthreads();
    // W = Vhat X12^*  (coordinates)
    for (int e = threadIdx.x; e < mo * r; e += NT) Yc[e] = cmul(y[e], cconj(cvec[e % r]));
    __syncthreads();
    if (p.householder_mode == 1) {
      // Householder vectors of u (mo x r), eq. (3.3); working copy in w
      for (int e = threadIdx.x; e < mo * r; e += NT) w[e] = u[e];
      __syncthreads();
      for (int k = 0; k < r; ++k) {
        // norm of w[k:mo, k]
        col_dots(s_vec + r, w + k * r + k, r, w + k * r + k, r, mo - k, 1, s_red);
        if (threadIdx.x == 0) s_alpha = sqrt(s_vec[r].x);
        __syncthreads();
        const double alpha = s_alpha;
        const double2 x0 = w[k * r + k];
        const double ax0 = sqrt(cabs2(x0));
        const double2 ph = ax0 > 0 ? cscale(1.0 / ax0, x0) : make_double2(1, 0);
        for (int i = threadIdx.x; i < mo; i += NT) {
          double2 v = i < k ? make_double2(0, 0) : w[i * r + k];
          if (i == k) v = cadd(v, cscale(alpha, ph));
          Uh[i * r + k] = v;
        }
        if (threadIdx.x == 0) s_beta[k] = alpha > 0 ? 1.0 / (alpha * alpha + alpha * ax0) : 0.0;
        __syncthreads();
        // apply P_k to the working copy columns k+1..r-1
        if (k + 1 < r) {
          col_dots(s_vec + r, Uh + k, r, w, r, mo, r, s_red);
          for (int e = threadIdx.x; e < mo * r; e += NT) {
            const int i = e / r, c = e % r;
            if (c > k) w[e] = csub(w[e], cscale(s_beta[k], cmul(Uh[i * r + k], s_vec[r + c])));
          }
          __syncthreads();
        }
      }
      // Q^H Yc = P_r ... P_1 Yc  (P_1 first)
      for (int k = 0; k < r; ++k) {
        col_dots(s_vec + r, Uh + k, r, Yc, r, mo, r, s_red);
        for (int e = threadIdx.x; e < mo * r; e += NT)
          Yc[e] = csub(Yc[e], cscale(s_beta[k], cmul(Uh[(e / r) * r + k], s_vec[r + e % r])));
        __syncthreads();
      }
      for (int e = threadIdx.x; e < r * r; e += NT) Yc[e] = make_double2(0, 0);
      __syncthreads();
      // W = Q [0; .] = P_1 ... P_r (.)  (P_r first)
      for (int k = r - 1; k >= 0; --k) {
        col_dots(s_vec + r, Uh + k, r, Yc, r, mo, r, s_red);
        for (int e = threadIdx.x; e < mo * r; e += NT)
          Yc[e] = csub(Yc[e], cscale(s_beta[k], cmul(Uh[(e / r) * r + k], s_vec[r + e % r])));
        __syncthreads();
      }
      for (int e = threadIdx.x; e < D * r; e += NT) w[e] = e < mo * r ? Yc[e] : make_double2(0, 0);
    } else {
      // projector form: W = (y - u G_raw) diag(conj c)
      gemm_nn(t1, r, u, r, Gr, r, mo, r, r);
      __syncthreads();
      for (int e = threadIdx.x; e < D * r; e += NT)
        w[e] = e < mo * r ? cmul(csub(y[e], t1[e]), cconj(cvec[e % r])) : make_double2(0, 0);
    }
    __syncthreads();
    // Z = u X11 + W
    gemm_nn(z, r, u, r, X11, r, mo, r, r);
    __syncthreads();
    for (int e = threadIdx.x; e < D * r; e += NT) z[e] = e < mo * r ? cadd(z[e], w[e]) : make_double2(0, 0);
    __syncthreads();
    // stage matrix k (mo x mo): u1 Lam u1^H + h sum coef_l (z_l u_l^H + u_l w_l^H)
    const bool last = (j + 1 == s);
    const int m = mo;
    double2 *K = (m * m <= p.lds_elems) ? s_mat : Kg;
    for (int e = threadIdx.x; e < m * m; e += NT) {
      const int a = e / m, b = e % m;
      double2 sacc = make_double2(0, 0);
      for (int c = 0; c < r; ++c)
        sacc = cadd(sacc, cscale(p.lam[c], cmul(u1[a * r + c], cconj(u1[b * r + c]))));
      for (int l = 0; l <= j; ++l) {
        const double coef = h * (last ? p.b[l] : p.a[j + 1][l]);
        if (coef == 0.0) continue;
        const double2 *ul = ws.stage + (3 * l + 0) * D * r;
        const double2 *zl = ws.stage + (3 * l + 1) * D * r;
        const double2 *wl = ws.stage + (3 * l + 2) * D * r;
        double2 t = make_double2(0, 0);
        for (int c = 0; c < r; ++c)
          t = cadd(t, cadd(cmul(zl[a * r + c], cconj(ul[b * r + c])), cmul(ul[a * r + c], cconj(wl[b * r + c]))));
        sacc = cadd(sacc, cscale(coef, t));
      }
      K[e] = sacc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * m; e += NT) {
      const int a = e / m, b = e % m;
      if (a < b) {
        const double2 x1 = K[e], x2 = K[b * m + a];
        const double2 hh = make_double2(0.5 * (x1.x + x2.x), 0.5 * (x1.y - x2.y));
        K[e] = hh;
        K[b * m + a] = cconj(hh);
      } else if (a == b) {
        K[e].y = 0.0;
      }
    }
    __syncthreads();
    const int sw = jacobi(K, Vj, m, p.eig_tol, p.max_sweeps, js);
    if (sw < 0) failed = 1;
    total_sweeps += sw < 0 ? p.max_sweeps : sw;
    max_sw = max(max_sw, sw < 0 ? p.max_sweeps : sw);
    double2 *unext = last ? ws.Cfin /* temporary */ : ws.stage + (3 * (j + 1) + 0) * D * r;
    take_top(K, Vj, m, r, unext, r, D, js);
    if (last) {
      // C = R^{-1} u_final
      for (int e = threadIdx.x; e < D * r; e += NT) t1[e] = ws.Cfin[e];
      __syncthreads();
      gemm_nn(ws.Cfin, r, Ri, D, t1, r, D, r, D);
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    int bad = 0;
    for (int e = 0; e < D * r; ++e)
      if (!isfinite(ws.Cfin[e].x) || !isfinite(ws.Cfin[e].y)) bad = 1;
    stats[0] = total_sweeps;
    stats[1] = max_sw;
    stats[2] = s_ndrop;
    stats[3] = s_minpiv;
    stats[6] = failed;
    stats[7] = bad;
    stats[8] = s;  // eigensolves this step
    // running totals over the steps of one call (zeroed by the host per call)
    stats[10] += total_sweeps;
    stats[11] += s;
    stats[12] = fmax(stats[12], (double)max_sw);
    stats[13] += failed;
    stats[14] += bad;
    stats[15] += 1;
  }
}

void launch_small_rk(const SmallRkParams &p, const SmallWs &ws, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_small_rk, hipFuncAttributeMaxDynamicSharedMemorySize,
                        kSmallLdsBytes);
    attr = true;
  }
  const size_t lds = (size_t)p.lds_elems * sizeof(double2);
  hipLaunchKernelGGL(k_small_rk, dim3(1), dim3(NT), lds, s, p, ws);
}

}  // namespace lrei
