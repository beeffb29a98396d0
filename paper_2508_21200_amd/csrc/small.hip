// Projected (small-space) part of one LREI-RK step, in FP64 on one workgroup.
//
// All stage factors of one RK step lie in the block Krylov space of H started
// from the current support V_1: V_1 is in it, f(K_j) = Z_j V_j* + V_j W_j*
// only adds H V_j, and V_{j+1} is spanned by V_1..V_j, W_1..W_j.  The N-space
// passes build that space as the blocks P_0 = V_1, P_{j+1} = beta (H P_j - P_j D_j)
// (D_j diagonal per-column shifts, beta the inverse spectral width of H) and
// measure their Gram products; this kernel then runs the paper's step
// (eqs. 3.2/4.1, 3.3, 3.4, 3.7-3.9 and the partial eigendecomposition with the
// spectrum reset to Lambda_0) exactly, in the coordinates of an orthonormal
// basis of that space, and returns the coefficients C with V_new = [P_0..P_s] C.
//
// Steps:
//  1. Assemble the Gram matrix Gamma of the blocks from the measured products
//     and the recurrence (P_i* P_{j+1} = P_{i+1}* P_j + beta (D_i P_i* P_j - P_i* P_j D_j));
//     Cholesky Gamma = R* R with directions whose pivot falls below 1e-13 of
//     the diagonal treated as dependent (dropped).
//  2. Coordinates: V_1 = B R^{-1} u_1 with u_1 = R[:, :r] (R_00* R_00)^{-1/2};
//     the projected Hamiltonian acts as y = R That R^{-1} u, That being the
//     block-bidiagonal relation H P_j = P_j D_j + P_{j+1} / beta.
//  3. For each stage: G = u* y, X11 = Phi o G, X12 coefficients c_a; the
//     complement action W = Vhat X12* through r Householder reflectors of u
//     (Sec. 3.4) (or the projector form); Z = u X11 + W; the stage matrix
//     k = u_1 Lambda_0 u_1* + h sum a_l (z_l u_l* + u_l w_l*) and its r largest
//     eigenvectors: subspace iteration from u with a spectral-gap certificate,
//     or the direct solve (Householder tridiagonalisation, multisection on
//     Sturm counts, inverse iteration, back-transformation).
//  4. C = R^{-1} u_final; the last kernel of the step refreshes D_j.
//
// Every phase is latency bound (one workgroup): the stage matrix (packed
// upper triangle) and the solver's work arrays live in LDS.
#include <hip/hip_runtime.h>

#include "lrei_internal.h"
#include "learned_dev.h"

namespace lrei {

namespace {

constexpr int NT = 512;
constexpr int NW = NT / 64;
constexpr int kMaxPairs = kMaxR / 2 + 1;  // Jacobi is used for r x r problems only

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

// Barrier for LDS traffic only: global memory operations may stay in flight.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Cross-lane reductions on DPP row operations (quad_perm, row_half_mirror,
// row_mirror within 16 lanes), a swizzle for the swap of 16-lane halves, and
// readlane across the two halves of the wave.  Every lane of the group must
// be active.  Results are identical in all lanes of the group.
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline double swap16_d(double v) {  // lane i <-> lane i ^ 16 within each 32 lanes
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
  return __hiloint2double(hi, lo);
}
__device__ inline double readlane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ inline double sum16(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}
__device__ inline double sum32(double v) {
  v = sum16(v);
  return v + swap16_d(v);
}
__device__ inline double sum64(double v) {
  v = sum32(v);
  return readlane_d(v, 0) + readlane_d(v, 32);
}
__device__ inline double max16(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  return fmax(v, dpp_d<0x140>(v));
}
__device__ inline double min16(double v) {
  v = fmin(v, dpp_d<0xB1>(v));
  v = fmin(v, dpp_d<0x4E>(v));
  v = fmin(v, dpp_d<0x141>(v));
  return fmin(v, dpp_d<0x140>(v));
}
__device__ inline double max32(double v) { v = max16(v); return fmax(v, swap16_d(v)); }
__device__ inline double min32(double v) { v = min16(v); return fmin(v, swap16_d(v)); }
__device__ inline double max64(double v) {
  v = max32(v);
  return fmax(readlane_d(v, 0), readlane_d(v, 32));
}

__device__ inline double2 wave_sum(double2 v) { return make_double2(sum64(v.x), sum64(v.y)); }

// phi(delta): q-LL (delta/hbar)(i - kappa delta) (eq. 4.1); q-LLG (i delta/hbar)/(1 - i kappa delta)
// (eq. 3.2: D / (E + L + L*)).  X11_ab = phi(lam_a - lam_b) G_ab, X12 = diag(phi(lam)) V* H Vhat.
__device__ inline double2 phi(double d, int model, double kappa, double hbar) {
  if (model == 0) return make_double2(-kappa * d * d / hbar, d / hbar);
  const double den = hbar * (1.0 + kappa * kappa * d * d);
  return make_double2(-kappa * d * d / den, d / den);
}

// ----- workgroup-wide small dense helpers (row-major, leading dimension ld) ---

// C (M x N, ldc) = op(A) B, op(A) = A (M x K, lda) or, with ah, A^H (A is K x M);
// complex FP64 on 16x16x4 MFMA, one 16 x 16 tile of C per wave at a time,
// operands read from memory (LDS or global).  C must not overlap A or B.
// Ends with a barrier.
typedef double d4v_g __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void zgemm(double2 *C, int ldc, const double2 *A, int lda, bool ah, const double2 *B, int ldb, int M,
                      int N, int K) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int mt = (M + 15) / 16, nt = (N + 15) / 16;
  for (int t = wave; t < mt * nt; t += NW) {
    const int ti = t / nt, tj = t % nt;
    const int row = ti * 16 + li, col = tj * 16 + li;
    d4v_g cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    // four k-steps of operands are loaded before their products, so that the
    // loads (global memory here, mostly L2 hits) overlap
    for (int kk = 0; kk < K; kk += 16) {
      double2 a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kk + 4 * q + lk;
        a[q] = make_double2(0, 0);
        b[q] = make_double2(0, 0);
        if (k < K && row < M) a[q] = ah ? cconj(A[k * lda + row]) : A[row * lda + k];
        if (k < K && col < N) b[q] = B[k * ldb + col];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cre = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].x, b[q].x, cre, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[q].y, b[q].y, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].x, b[q].y, cim, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].y, b[q].x, cim, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * 16 + 4 * v + lk, j = tj * 16 + li;
      if (i < M && j < N) C[i * ldc + j] = make_double2(cre[v], cim[v]);
    }
  }
  __syncthreads();
}

// out[c] = sum_{i < m} conj(v[i * ldv]) M[i * ldm + c] for c < nc, one wave per
// column (wave-level reduction, no LDS).  Ends with a barrier.
__device__ void col_dots(double2 *out, const double2 *v, int ldv, const double2 *M, int ldm, int m, int nc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < nc; c += NW) {
    double2 s = make_double2(0, 0);
    for (int i = lane; i < m; i += 64) s = cadd(s, cmulc(v[i * ldv], M[i * ldm + c]));
    s = wave_sum(s);
    if (lane == 0) out[c] = s;
  }
  __syncthreads();
}

// ----- complex Hermitian Jacobi (round-robin parallel ordering) ---------------

struct JacobiShared {
  int p[kMaxPairs], q[kMaxPairs];
  double cs[kMaxPairs], sn[kMaxPairs], t[kMaxPairs];
  double2 e[kMaxPairs];
  int rotated;
  double scale;
  int order[kMaxR];
};

__device__ inline int rr_player(int pos, int round, int mp) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (mp - 1);
}
// packed upper triangle, column-major: element (i, j), i <= j
__device__ inline int pk(int i, int j) { return j * (j + 1) / 2 + i; }
__device__ inline double2 aget(const double2 *A, int i, int j) {
  return i <= j ? A[pk(i, j)] : cconj(A[pk(j, i)]);
}
__device__ inline void aset(double2 *A, int i, int j, double2 v) {
  if (i <= j)
    A[pk(i, j)] = v;
  else
    A[pk(j, i)] = cconj(v);
}

// Diagonalises the Hermitian m x m matrix A (packed upper triangle) in place and
// accumulates V = product of rotations (m x m row-major, starts as identity).
// A and V may live in LDS or global memory (lds says which barrier suffices).
// Returns the sweep count, or -1 when max_sweeps is reached.
__device__ int jacobi(double2 *A, double2 *V, int m, double tol, int max_sweeps, JacobiShared &js, bool lds) {
  const int mp = m + (m & 1), np = mp / 2;
  for (int e = threadIdx.x; e < m * m; e += NT)
    V[e] = make_double2((e / m) == (e % m) ? 1.0 : 0.0, 0.0);
  if (threadIdx.x == 0) {
    double sc = 0;
    for (int i = 0; i < m; ++i) sc = fmax(sc, fabs(A[pk(i, i)].x));
    js.scale = sc > 0 ? sc : 1.0;
  }
  __syncthreads();
  const double thresh = tol * js.scale;
  if (m == 1) return 0;
  const int nblk = np * (np + 1) / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) js.rotated = 0;
    __syncthreads();
    for (int round = 0; round < mp - 1; ++round) {
      if (threadIdx.x < np) {
        const int i = threadIdx.x;
        const int a = rr_player(i, round, mp), b = rr_player(mp - 1 - i, round, mp);
        const int p = a < b ? a : b, q = a < b ? b : a;
        js.p[i] = p;
        js.q[i] = q;
        double cs = 1, sn = 0, t = 0;
        double2 e = make_double2(1, 0);
        if (q < m) {
          const double2 c = A[pk(p, q)];
          const double x = sqrt(cabs2(c));
          if (x > thresh) {
            const double app = A[pk(p, p)].x, aqq = A[pk(q, q)].x;
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
      if (lds) lds_barrier(); else __syncthreads();
      // two-sided update of the 2x2 blocks (P rows, Q cols), P <= Q; the
      // (Q, P) blocks are their adjoints in the packed storage
      for (int blk = threadIdx.x; blk < nblk; blk += NT) {
        int P = 0, rem = blk;
        while (rem >= np - P) {
          rem -= np - P;
          ++P;
        }
        const int Q = P + rem;
        const double snP = js.sn[P], snQ = js.sn[Q];
        if (snP == 0.0 && snQ == 0.0) continue;
        const int pP = js.p[P], qP = js.q[P], pQ = js.p[Q], qQ = js.q[Q];
        if (P == Q) {
          if (qP >= m) continue;
          const double x = sqrt(cabs2(A[pk(pP, qP)]));
          const double app = A[pk(pP, pP)].x, aqq = A[pk(qP, qP)].x;
          A[pk(pP, pP)] = make_double2(app - js.t[P] * x, 0.0);
          A[pk(qP, qP)] = make_double2(aqq + js.t[P] * x, 0.0);
          A[pk(pP, qP)] = make_double2(0, 0);
          continue;
        }
        const bool hq = qP < m, hqq = qQ < m;
        const double2 z = make_double2(0, 0);
        const double2 a = aget(A, pP, pQ);
        const double2 b = hqq ? aget(A, pP, qQ) : z;
        const double2 c = hq ? aget(A, qP, pQ) : z;
        const double2 d = (hq && hqq) ? aget(A, qP, qQ) : z;
        const double csP = js.cs[P];
        const double2 ebP = cconj(js.e[P]);
        const double2 a1 = csub(cscale(csP, a), cscale(snP, cmul(ebP, c)));
        const double2 b1 = csub(cscale(csP, b), cscale(snP, cmul(ebP, d)));
        const double2 c1 = cadd(cscale(snP, a), cscale(csP, cmul(ebP, c)));
        const double2 d1 = cadd(cscale(snP, b), cscale(csP, cmul(ebP, d)));
        const double csQ = js.cs[Q];
        const double2 eQ = js.e[Q];
        aset(A, pP, pQ, csub(cscale(csQ, a1), cscale(snQ, cmul(eQ, b1))));
        if (hqq) aset(A, pP, qQ, cadd(cscale(snQ, a1), cscale(csQ, cmul(eQ, b1))));
        if (hq) aset(A, qP, pQ, csub(cscale(csQ, c1), cscale(snQ, cmul(eQ, d1))));
        if (hq && hqq) aset(A, qP, qQ, cadd(cscale(snQ, c1), cscale(csQ, cmul(eQ, d1))));
      }
      for (int e = threadIdx.x; e < np * m; e += NT) {
        const int P = e / m, i = e % m;
        const double sn = js.sn[P];
        if (sn == 0.0) continue;
        const int p = js.p[P], q = js.q[P];
        const double2 vp = V[i * m + p], vq = V[i * m + q];
        const double cs = js.cs[P];
        const double2 ee = js.e[P];
        V[i * m + p] = csub(cscale(cs, vp), cscale(sn, cmul(ee, vq)));
        V[i * m + q] = cadd(cscale(sn, vp), cscale(cs, cmul(ee, vq)));
      }
      if (lds) lds_barrier(); else __syncthreads();
    }
    __syncthreads();
    if (!js.rotated) return sweep + 1;
  }
  return -1;
}

// The same Jacobi iteration run by one wave (called by the 64 lanes of one
// wave only; A, V and js in LDS): each round costs wave-level
// synchronisation instead of workgroup barriers, which is what dominates
// for r x r problems.  Same rotations, same arithmetic per element.
__device__ __forceinline__ int jacobi_wave(double2 *A, double2 *V, int m, double tol, int max_sweeps, JacobiShared &js) {
  const int lane = threadIdx.x & 63;
  const int mp = m + (m & 1), np = mp / 2;
  for (int e = lane; e < m * m; e += 64)
    V[e] = make_double2((e / m) == (e % m) ? 1.0 : 0.0, 0.0);
  if (lane == 0) {
    double sc = 0;
    for (int i = 0; i < m; ++i) sc = fmax(sc, fabs(A[pk(i, i)].x));
    js.scale = sc > 0 ? sc : 1.0;
  }
  __builtin_amdgcn_wave_barrier();
  const double thresh = tol * js.scale;
  if (m == 1) return 0;
  const int nblk = np * (np + 1) / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (lane == 0) js.rotated = 0;
    __builtin_amdgcn_wave_barrier();
    for (int round = 0; round < mp - 1; ++round) {
      if (lane < np) {
        const int i = lane;
        const int a = rr_player(i, round, mp), b = rr_player(mp - 1 - i, round, mp);
        const int p = a < b ? a : b, q = a < b ? b : a;
        js.p[i] = p;
        js.q[i] = q;
        double cs = 1, sn = 0, t = 0;
        double2 e = make_double2(1, 0);
        if (q < m) {
          const double2 c = A[pk(p, q)];
          const double x = sqrt(cabs2(c));
          if (x > thresh) {
            const double app = A[pk(p, p)].x, aqq = A[pk(q, q)].x;
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
      __builtin_amdgcn_wave_barrier();
      // two-sided update of the 2x2 blocks (P rows, Q cols), P <= Q; the
      // (Q, P) blocks are their adjoints in the packed storage
      for (int blk = lane; blk < nblk; blk += 64) {
        int P = 0, rem = blk;
        while (rem >= np - P) {
          rem -= np - P;
          ++P;
        }
        const int Q = P + rem;
        const double snP = js.sn[P], snQ = js.sn[Q];
        if (snP == 0.0 && snQ == 0.0) continue;
        const int pP = js.p[P], qP = js.q[P], pQ = js.p[Q], qQ = js.q[Q];
        if (P == Q) {
          if (qP >= m) continue;
          const double x = sqrt(cabs2(A[pk(pP, qP)]));
          const double app = A[pk(pP, pP)].x, aqq = A[pk(qP, qP)].x;
          A[pk(pP, pP)] = make_double2(app - js.t[P] * x, 0.0);
          A[pk(qP, qP)] = make_double2(aqq + js.t[P] * x, 0.0);
          A[pk(pP, qP)] = make_double2(0, 0);
          continue;
        }
        const bool hq = qP < m, hqq = qQ < m;
        const double2 z = make_double2(0, 0);
        const double2 a = aget(A, pP, pQ);
        const double2 b = hqq ? aget(A, pP, qQ) : z;
        const double2 c = hq ? aget(A, qP, pQ) : z;
        const double2 d = (hq && hqq) ? aget(A, qP, qQ) : z;
        const double csP = js.cs[P];
        const double2 ebP = cconj(js.e[P]);
        const double2 a1 = csub(cscale(csP, a), cscale(snP, cmul(ebP, c)));
        const double2 b1 = csub(cscale(csP, b), cscale(snP, cmul(ebP, d)));
        const double2 c1 = cadd(cscale(snP, a), cscale(csP, cmul(ebP, c)));
        const double2 d1 = cadd(cscale(snP, b), cscale(csP, cmul(ebP, d)));
        const double csQ = js.cs[Q];
        const double2 eQ = js.e[Q];
        aset(A, pP, pQ, csub(cscale(csQ, a1), cscale(snQ, cmul(eQ, b1))));
        if (hqq) aset(A, pP, qQ, cadd(cscale(snQ, a1), cscale(csQ, cmul(eQ, b1))));
        if (hq) aset(A, qP, pQ, csub(cscale(csQ, c1), cscale(snQ, cmul(eQ, d1))));
        if (hq && hqq) aset(A, qP, qQ, cadd(cscale(snQ, c1), cscale(csQ, cmul(eQ, d1))));
      }
      for (int e = lane; e < np * m; e += 64) {
        const int P = e / m, i = e % m;
        const double sn = js.sn[P];
        if (sn == 0.0) continue;
        const int p = js.p[P], q = js.q[P];
        const double2 vp = V[i * m + p], vq = V[i * m + q];
        const double cs = js.cs[P];
        const double2 ee = js.e[P];
        V[i * m + p] = csub(cscale(cs, vp), cscale(sn, cmul(ee, vq)));
        V[i * m + q] = cadd(cscale(sn, vp), cscale(cs, cmul(ee, vq)));
      }
      __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();
    if (!js.rotated) return sweep + 1;
  }
  return -1;
}

__device__ inline uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// ----- top-r eigenpairs by Householder tridiagonalisation ---------------------
//
// A (m x m Hermitian, packed lower triangle, column-major) is reduced to a
// Hermitian tridiagonal T = Q^H A Q with m-2 Householder reflectors (vectors
// kept in A's columns below the subdiagonal), T is made real by a diagonal
// phase scaling, the r largest eigenvalues are found by multisection on Sturm
// counts, their eigenvectors by inverse iteration with partial-pivoting
// tridiagonal solves (re-orthogonalised within clusters of close eigenvalues),
// and are mapped back through the phases and reflectors.

constexpr int kTriDim = (kMaxStages + 1) * kMaxR;  // bound on m
constexpr int kGroup = 16;                         // lanes per eigenvalue in the multisection

struct TriShared {
  double d[kTriDim], e2[kTriDim], ae[kTriDim], beta[kTriDim];
  double2 e[kTriDim], ph[kTriDim], p[kTriDim], v[kTriDim];
  double2 kpart[NT / 32];
  double lam[kMaxR];
  double glo, ghi, tnorm;
  uint64_t tmark;
  double tacc[7];  // real-time ticks: tridiagonalisation, multisection, inverse iteration, back-transform,
                   // (unused), and the warm-started solver: whole, its Ritz step
};

// packed lower triangle, column-major: element (i, j), i >= j
__device__ inline int pl(int i, int j, int m) { return j * m - (j * (j - 1)) / 2 + (i - j); }

__device__ inline double wave_sum_d(double v) { return sum64(v); }

// 1/b from the hardware reciprocal refined by one Newton step (|b| >= pivmin,
// so b is normal); within a couple of ulp of the correctly rounded quotient.
__device__ inline double rcp_nr(double b) {
  const double r = __builtin_amdgcn_rcp(b);
  return r * fma(-b, r, 2.0);
}

// 1/sqrt(a) (a > 0 and normal) from the hardware reciprocal square root refined
// by one Newton step, y (3 - a y^2) / 2.
__device__ inline double rsq_nr(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  return y * fma(-0.5 * a * y, y, 1.5);
}

// Number of eigenvalues of the real symmetric tridiagonal (d, e) below s, by
// the ratio form of the Sturm sequence (pivots of LDL^T of T - s I).  The
// recurrence is a serial chain; (d, e^2) are read eight entries ahead of it.
__device__ inline int sturm_count(const TriShared &ts, int m, double s, double pivmin) {
  constexpr int B = 8;
  double q = ts.d[0] - s;
  int c = q < 0.0;
  for (int i0 = 1; i0 < m; i0 += B) {
    double dd[B], ee[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = i0 + u < m ? i0 + u : m - 1;
      dd[u] = ts.d[i];
      ee[u] = ts.e2[i - 1];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (i0 + u < m) {
        if (fabs(q) < pivmin) q = -pivmin;
        q = (dd[u] - s) - ee[u] * rcp_nr(q);
        c += q < 0.0;
      }
    }
  }
  return c;
}

// u (rows_out x r, ld ldu) <- eigenvectors of the r largest eigenvalues of A,
// descending.  scr: >= 4 * m * SL doubles (SL = 16 for r <= 16, else 32), used
// for the inverse-iteration LU and the back-transform.
__device__ __forceinline__ void eig_top(double2 *A, int m, int r, double2 *u, int ldu, int rows_out, double *scr,
                                        bool lds, TriShared &ts) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto tlap = [&](int slot) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint64_t t = now_ticks();
      ts.tacc[slot] += (double)(t - ts.tmark);
      ts.tmark = t;
    }
  };
  if (threadIdx.x == 0) ts.tmark = now_ticks();
  // ---- Householder tridiagonalisation.  A v and the rank-2 update give each
  // trailing row to a group of 8 lanes (64 rows at a time), the lanes of a
  // group walking the row's columns with stride 8: at m <= 64 every thread
  // has at most 8 elements and the row sums are 3-step DPP reductions.
  const int grow = threadIdx.x >> 3, gsub = threadIdx.x & 7;
  for (int k = 0; k + 2 < m; ++k) {
    if (wave == 0) {
      double s2 = 0;
      for (int i = k + 1 + lane; i < m; i += 64) {
        const double2 x = A[pl(i, k, m)];
        s2 += cabs2(x);
        ts.v[i] = x;
      }
      s2 = wave_sum_d(s2);
      if (lane == 0) {
        const double2 x0 = A[pl(k + 1, k, m)];
        if (!(s2 > 1e-300)) {
          // column already reduced (below any meaningful scale): no reflector,
          // the negligible remainder below the subdiagonal is dropped
          ts.beta[k] = 0.0;
          ts.e[k] = x0;
        } else {
          // alpha = -|x| x0 / |x0|, v0 = x0 - alpha = (1 + |x| / |x0|) x0, so
          // |v|^2 = |v0|^2 + |x|^2 - |x0|^2 = nx^2 + 2 nx ax0 + s2 with the
          // computed nx = |x|; square roots and quotients as reciprocal square
          // roots and reciprocals with a Newton step (short dependent chains)
          const double c2 = cabs2(x0);
          const double nx = s2 * rsq_nr(s2);
          double2 alpha, v0;
          double ax0 = 0.0;
          if (c2 > 1e-300) {
            const double ia = rsq_nr(c2);
            ax0 = c2 * ia;
            const double q = nx * ia;
            alpha = cscale(-q, x0);
            v0 = cscale(1.0 + q, x0);
          } else {
            alpha = make_double2(-nx, 0.0);
            v0 = make_double2(nx, 0.0);
          }
          ts.beta[k] = 2.0 * rcp_nr(fma(nx, nx + 2.0 * ax0, s2));
          ts.e[k] = alpha;
          A[pl(k + 1, k, m)] = v0;  // the reflector vector stays in column k
          ts.v[k + 1] = v0;
        }
      }
    }
    if (lds) lds_barrier(); else __syncthreads();
    const double beta = ts.beta[k];
    if (beta != 0.0) {
      // p = beta A22 v, and this wave's part of v^H p
      double2 kp = make_double2(0, 0);
      for (int i0 = k + 1; i0 < m; i0 += NT / 8) {
        const int i = i0 + grow;
        double sr = 0, si = 0, sr2 = 0, si2 = 0;  // two chains: FP64 adds wait on each other
        if (i < m) {
          for (int j = k + 1 + gsub; j < m; j += 16) {
            const int hi = i > j ? i : j, lo = i > j ? j : i;
            double2 a = A[pl(hi, lo, m)];
            if (i < j) a.y = -a.y;
            const double2 v = ts.v[j];
            sr = fma(a.x, v.x, fma(-a.y, v.y, sr));
            si = fma(a.x, v.y, fma(a.y, v.x, si));
            const int j2 = j + 8;
            if (j2 < m) {
              const int hi2 = i > j2 ? i : j2, lo2 = i > j2 ? j2 : i;
              double2 a2 = A[pl(hi2, lo2, m)];
              if (i < j2) a2.y = -a2.y;
              const double2 v2 = ts.v[j2];
              sr2 = fma(a2.x, v2.x, fma(-a2.y, v2.y, sr2));
              si2 = fma(a2.x, v2.y, fma(a2.y, v2.x, si2));
            }
          }
        }
        sr += sr2;
        si += si2;
        sr += dpp_d<0xB1>(sr);  // sum over the 8 lanes of the group
        si += dpp_d<0xB1>(si);
        sr += dpp_d<0x4E>(sr);
        si += dpp_d<0x4E>(si);
        sr += dpp_d<0x141>(sr);
        si += dpp_d<0x141>(si);
        if (i < m && gsub == 0) {
          const double2 pi = make_double2(beta * sr, beta * si);
          ts.p[i] = pi;
          kp = cadd(kp, cmulc(ts.v[i], pi));
        }
      }
      kp = wave_sum(kp);
      if (lane == 0) ts.kpart[wave] = kp;
      if (lds) lds_barrier(); else __syncthreads();
      // K = (beta/2) v^H p (fixed summation order); w = p - K v
      double2 kq[NW];
#pragma unroll
      for (int q = 0; q < NW; ++q) kq[q] = ts.kpart[q];
#pragma unroll
      for (int h = NW / 2; h > 0; h >>= 1)  // pairwise, fixed order
#pragma unroll
        for (int q = 0; q < h; ++q) kq[q] = cadd(kq[q], kq[q + h]);
      const double2 ks = kq[0];
      const double2 K = cscale(0.5 * beta, ks);
      // lower triangle of the trailing block: A_ij -= v_i conj(w_j) + w_i conj(v_j)
      for (int i = k + 1 + grow; i < m; i += NT / 8) {
        const double2 vi = ts.v[i], wi = csub(ts.p[i], cmul(K, vi));
        for (int j = k + 1 + gsub; j <= i; j += 8) {
          const double2 vj = ts.v[j], wj = csub(ts.p[j], cmul(K, vj));
          const int q = pl(i, j, m);
          A[q] = csub(A[q], cadd(cmul(vi, cconj(wj)), cmul(wi, cconj(vj))));
        }
      }
      if (lds) lds_barrier(); else __syncthreads();
    }
  }
  tlap(0);
  // ---- real tridiagonal: d, |e|, phases.  The moduli and unit phase factors
  // in parallel; their running product (ph_i = prod_{k<i} e_k / |e_k|) by one
  // thread, in the same order; the Gershgorin bounds by wave reductions.
  if (threadIdx.x == 0 && m >= 2) ts.e[m - 2] = A[pl(m - 1, m - 2, m)];
  __syncthreads();
  double2 *unit = ts.p;  // free after the tridiagonalisation
  for (int i = threadIdx.x; i < m; i += NT) {
    ts.d[i] = A[pl(i, i, m)].x;
    if (i + 1 < m) {
      const double a = sqrt(cabs2(ts.e[i]));
      ts.ae[i] = a;
      ts.e2[i] = a * a;
      unit[i] = a > 0 ? cscale(1.0 / a, ts.e[i]) : make_double2(1, 0);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 ph = make_double2(1, 0);
    for (int i = 0; i < m; ++i) {
      ts.ph[i] = ph;
      if (i + 1 < m && ts.ae[i] > 0) ph = cmul(ph, unit[i]);
    }
  }
  if (wave == 0) {
    double lo = 1e300, hi = -1e300;
    for (int i = lane; i < m; i += 64) {
      const double rad = (i > 0 ? ts.ae[i - 1] : 0.0) + (i + 1 < m ? ts.ae[i] : 0.0);
      lo = fmin(lo, ts.d[i] - rad);
      hi = fmax(hi, ts.d[i] + rad);
    }
    lo = -max64(-lo);
    hi = max64(hi);
    if (lane == 0) {
      const double tn = fmax(fabs(lo), fabs(hi));
      ts.tnorm = tn > 0 ? tn : 1.0;
      ts.glo = lo - 1e-14 * ts.tnorm;
      ts.ghi = hi + 1e-14 * ts.tnorm;
    }
  }
  __syncthreads();
  // ---- multisection: G lanes per eigenvalue (32 when r <= 16, else 16), all
  // within one wave; each round splits the bracket into G + 1 parts.  The
  // shifts only seed the inverse iteration below: 33^8 and 17^10 parts bring
  // them within ~1e-12 of the Gershgorin width, and two inverse iterations
  // then shrink a component along another eigenvector by (shift error / gap)^2,
  // below FP64 rounding for any gap above 1e-6 of the norm (eigenvalues closer
  // than 1e-3 of the norm are re-orthogonalised as a cluster).
  {
    const int G = r <= NT / 32 ? 32 : kGroup;
    const int rounds = G == 32 ? 8 : 10;
    const int k = threadIdx.x / G, t = threadIdx.x % G;
    const double pivmin = 1e-290;
    if (k < r) {
      double a = ts.glo, b = ts.ghi;
      const int target = m - 1 - k;
      for (int round = 0; round < rounds; ++round) {
        const double x = a + (b - a) * (double)(t + 1) / (double)(G + 1);
        const bool ok = sturm_count(ts, m, x, pivmin) <= target;  // lambda_target >= x
        double na = ok ? x : -1e300, nb = ok ? 1e300 : x;
        if (G == 32) {
          na = max32(na);
          nb = min32(nb);
        } else {
          na = max16(na);
          nb = min16(nb);
        }
        if (na > -1e300) a = na;
        if (nb < 1e300) b = nb;
      }
      if (t == 0) ts.lam[k] = 0.5 * (a + b);
    }
  }
  __syncthreads();
  tlap(1);
  // ---- inverse iteration (wave 0, lane k < r), interleaved per-lane arrays
  const int SL = r <= 16 ? 16 : 32;
  double *U0 = scr, *U1 = scr + m * SL, *U2 = scr + 2 * m * SL, *X = scr + 3 * m * SL;
  if (wave == 0) {
    const int k = lane;
    const bool act = k < r;
    const double lam = act ? ts.lam[k] : 0.0;
    const double tiny = 1e-15 * ts.tnorm;
    if (act)
      for (int i = 0; i < m; ++i) X[i * SL + k] = 1.0 + 0.25 * (double)((7 * i + 3 * k) % 11);
    bool near = false;  // lane k: some eigenvalue j < k lies within 1e-3 of the norm
    if (act)
      for (int j = 0; j < k; ++j) near = near || fabs(lam - ts.lam[j]) < 1e-3 * ts.tnorm;
    const unsigned long long close = __ballot(near);
    for (int it = 0; it < 2; ++it) {
      if (act) {
        double u0 = ts.d[0] - lam, u1 = m > 1 ? ts.ae[0] : 0.0;
        double rc = X[0 * SL + k];
        // Elimination with row interchanges: the chain runs through u0, u1
        // and rc; the tridiagonal and the right-hand side are read a block of
        // IB rows ahead (row i + 1 of X is read before row i is written).  U0
        // keeps the reciprocal of each pivot (hardware reciprocal refined by a
        // Newton step), so no division sits on the chain here or in the
        // back-substitution.  Pivots below 1e-290 are replaced by tiny.
        constexpr int IB = 8;
        constexpr double kFloor = 1e-290;
        for (int i0 = 0; i0 + 1 < m; i0 += IB) {
          double an_[IB], ian_[IB], bn_[IB], cn_[IB], rn_[IB];
#pragma unroll
          for (int q = 0; q < IB; ++q) {
            const int i = i0 + q + 1 < m ? i0 + q : m - 2;
            an_[q] = ts.ae[i];
            ian_[q] = an_[q] > kFloor ? rcp_nr(an_[q]) : 0.0;
            bn_[q] = ts.d[i + 1] - lam;
            cn_[q] = (i + 2 < m) ? ts.ae[i + 1] : 0.0;
            rn_[q] = X[(i + 1) * SL + k];
          }
#pragma unroll
          for (int q = 0; q < IB; ++q) {
            const int i = i0 + q;
            if (i + 1 >= m) break;
            const double an = an_[q], bn = bn_[q], cn = cn_[q], rn = rn_[q];
            // keep row i as the pivot row unless the subdiagonal is larger
            const bool keep = fabs(u0) >= an || !(an > kFloor);
            const double piv = fabs(u0) > kFloor ? u0 : tiny;
            const double ip = keep ? rcp_nr(piv) : ian_[q];
            const double f = (keep ? an : u0) * ip;
            U0[i * SL + k] = ip;
            U1[i * SL + k] = keep ? u1 : bn;
            U2[i * SL + k] = keep ? 0.0 : cn;
            X[i * SL + k] = keep ? rc : rn;
            const double nu0 = keep ? bn - f * u1 : u1 - f * bn;
            const double nu1 = keep ? cn : -f * cn;
            rc = keep ? rn - f * rc : rc - f * rn;
            u0 = nu0;
            u1 = nu1;
          }
        }
        const double ipl = rcp_nr(fabs(u0) > kFloor ? u0 : tiny);
        double x2 = 0.0, x1 = rc * ipl;
        X[(m - 1) * SL + k] = x1;
        double nrm = x1 * x1;
        // back-substitution, rows read a block ahead of the chain through x1, x2
        for (int i0 = m - 2; i0 >= 0; i0 -= IB) {
          double r_[IB], a_[IB], b_[IB], c_[IB];
#pragma unroll
          for (int q = 0; q < IB; ++q) {
            const int i = i0 - q >= 0 ? i0 - q : 0;
            r_[q] = X[i * SL + k];
            a_[q] = U0[i * SL + k];
            b_[q] = U1[i * SL + k];
            c_[q] = U2[i * SL + k];
          }
#pragma unroll
          for (int q = 0; q < IB; ++q) {
            const int i = i0 - q;
            if (i < 0) break;
            const double xi = (r_[q] - b_[q] * x1 - c_[q] * x2) * a_[q];
            X[i * SL + k] = xi;
            nrm += xi * xi;
            x2 = x1;
            x1 = xi;
          }
        }
        const double inv = 1.0 / sqrt(nrm);
        for (int i = 0; i < m; ++i) X[i * SL + k] *= inv;
      }
      // modified Gram-Schmidt within clusters of close eigenvalues (whole wave);
      // `close` (bit kk: eigenvalue kk has a close earlier one) skips the rest
      for (int kk = 1; kk < r; ++kk) {
        if (!((close >> kk) & 1ull)) continue;  // the same in every lane
        bool any = false;
        for (int j = 0; j < kk; ++j) {
          if (fabs(ts.lam[kk] - ts.lam[j]) >= 1e-3 * ts.tnorm) continue;
          any = true;
          double dt = 0;
          for (int i = lane; i < m; i += 64) dt += X[i * SL + kk] * X[i * SL + j];
          dt = wave_sum_d(dt);
          for (int i = lane; i < m; i += 64) X[i * SL + kk] -= dt * X[i * SL + j];
        }
        if (any) {
          double nn = 0;
          for (int i = lane; i < m; i += 64) nn += X[i * SL + kk] * X[i * SL + kk];
          nn = wave_sum_d(nn);
          const double inv = 1.0 / sqrt(nn);
          for (int i = lane; i < m; i += 64) X[i * SL + kk] *= inv;
        }
      }
    }
  }
  __syncthreads();
  tlap(2);
  // ---- back-transform: u = Q (ph o X), Q = H_0 ... H_{m-3}.  One half-wave per
  // column: lane l of the half holds rows l, l + 32, ... in registers, so each
  // reflector costs one half-wave reduction and no barrier.
  {
    const int half = threadIdx.x >> 5, hl = threadIdx.x & 31;
    constexpr int kSlots = (kTriDim + 31) / 32;
    for (int c = half; c < r; c += NT / 32) {
      double2 y[kSlots];
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        const int l = hl + 32 * q;
        y[q] = l < m ? cscale(X[l * SL + c], ts.ph[l]) : make_double2(0, 0);
      }
      for (int k = m - 3; k >= 0; --k) {
        const double beta = ts.beta[k];
        if (beta == 0.0) continue;
        double sr = 0, si = 0;
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
          const int l = hl + 32 * q;
          if (l > k && l < m) {
            const double2 t = cmulc(A[pl(l, k, m)], y[q]);
            sr += t.x;
            si += t.y;
          }
        }
        sr = sum32(sr);
        si = sum32(si);
        const double2 f = make_double2(beta * sr, beta * si);
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
          const int l = hl + 32 * q;
          if (l > k && l < m) y[q] = csub(y[q], cmul(A[pl(l, k, m)], f));
        }
      }
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        const int l = hl + 32 * q;
        if (l < rows_out) u[l * ldu + c] = l < m ? y[q] : make_double2(0, 0);
      }
    }
  }
  tlap(3);
}

// ----- top-r eigenvectors by subspace iteration from a predicted basis -------
//
// The r largest eigenvalues of a stage matrix stay close to Lambda_0 while the
// rest of its spectrum is small (the tangent part of f vanishes on the
// complement of the support, so that part is second order in the step; for
// the later stages of a step it is smaller still).  The span of the r
// eigenvectors is then reached by subspace iteration X <- orth(K X D^-1) from
// the stage's input basis in a few iterations: the error shrinks by
// max|rest| / lambda_r per iteration.  Convergence is judged by the subspace
// residual Res = K X - X G, G = X* K X.  The result is kept only with a
// certificate that no other eigenvalue of K reaches the r found: the rest of
// the spectrum lies within T + |Res| of zero, T^2 = |K|_F^2 - |G|_F^2 -
// 2 |Res|_F^2 (the squared Frobenius norm of the compression of K to the
// complement of X), and the r eigenvalues near G's lie above a Gershgorin
// lower bound of G minus |Res|.  The eigenvectors then come from the r x r
// eigenproblem of G.  Otherwise (slow contraction, a failed
// orthonormalisation, no certificate) the caller runs the direct solver; K is
// left intact for it.

__device__ inline double2 kget(const double2 *K, int i, int j, int m) {
  return i >= j ? K[pl(i, j, m)] : cconj(K[pl(j, i, m)]);
}

// Sum over the workgroup of one value per thread, fixed order; every thread
// gets the result.
__device__ double block_sum(double v, double *red) {
  v = sum64(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < NW; ++w) t += red[w];
  return t;
}

// Y (m x r, ld r) = K X for the packed Hermitian K; one 16 x 16 MFMA tile per
// wave.  Ends with a barrier.
__device__ __forceinline__ void hemm_packed(double2 *Y, const double2 *K, int m, const double2 *X, int r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int mt = (m + 15) / 16, nt = (r + 15) / 16;
  for (int t = wave; t < mt * nt; t += NW) {
    const int ti = t / nt, tj = t % nt;
    const int row = ti * 16 + li, col = tj * 16 + li;
    d4v_g cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    for (int kk = 0; kk < m; kk += 4) {
      const int k = kk + lk;
      double2 a = make_double2(0, 0), b = make_double2(0, 0);
      if (k < m && row < m) a = kget(K, row, k, m);
      if (k < m && col < r) b = X[k * r + col];
      cre = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cre, 0, 0, 0);
      cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, cim, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, cim, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * 16 + 4 * v + lk, j = tj * 16 + li;
      if (i < m && j < r) Y[i * r + j] = make_double2(cre[v], cim[v]);
    }
  }
  __syncthreads();
}

// Per-thread partial of |Y - X G|_F^2 (X, Y: m x r; G: r x r; all ld r),
// formed tile by tile in MFMA registers.
__device__ double resid_part(const double2 *Y, const double2 *X, const double2 *G, int m, int r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int mt = (m + 15) / 16, nt = (r + 15) / 16;
  double acc = 0;
  for (int t = wave; t < mt * nt; t += NW) {
    const int ti = t / nt, tj = t % nt;
    const int row = ti * 16 + li, col = tj * 16 + li;
    d4v_g cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    for (int kk = 0; kk < r; kk += 4) {
      const int k = kk + lk;
      double2 a = make_double2(0, 0), b = make_double2(0, 0);
      if (k < r && row < m) a = X[row * r + k];
      if (k < r && col < r) b = G[k * r + col];
      cre = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cre, 0, 0, 0);
      cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, cim, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, cim, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * 16 + 4 * v + lk, j = tj * 16 + li;
      if (i < m && j < r) {
        const double2 y = Y[i * r + j];
        const double dr = y.x - cre[v], di = y.y - cim[v];
        acc += dr * dr + di * di;
      }
    }
  }
  return acc;
}

// X (m x r) <- X R^{-1} with X* X = R* R (Cholesky QR); C: r x r scratch.
// Returns false (workgroup-uniform) if X* X is not numerically positive definite.
__device__ __forceinline__ bool chol_qr(double2 *X, int m, int r, double2 *C) {
  zgemm(C, r, X, r, true, X, r, r, r, m);  // C = X* X (ends with a barrier)
  // upper Cholesky factor in place, right-looking, all threads on each update
  for (int k = 0; k < r; ++k) {
    const double piv = C[k * r + k].x;
    if (!(piv > 1e-280)) return false;  // every thread read the same pivot
    const double inv = 1.0 / sqrt(piv);
    __syncthreads();
    for (int j = k + 1 + threadIdx.x; j < r; j += NT) C[k * r + j] = cscale(inv, C[k * r + j]);
    if (threadIdx.x == 0) C[k * r + k] = make_double2(sqrt(piv), 0.0);
    __syncthreads();
    const int w = r - k - 1;
    for (int e = threadIdx.x; e < w * w; e += NT) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      if (j >= i) C[i * r + j] = csub(C[i * r + j], cmulc(C[k * r + i], C[k * r + j]));
    }
    __syncthreads();
  }
  // rows of X times R^{-1}, in place: x_c = (y_c - sum_{k<c} x_k R_kc) / R_cc
  for (int i = threadIdx.x; i < m; i += NT) {
    double2 *x = X + i * r;
    for (int c = 0; c < r; ++c) {
      double2 v = x[c];
      for (int k = 0; k < c; ++k) v = csub(v, cmul(x[k], C[k * r + c]));
      x[c] = cscale(1.0 / C[c * r + c].x, v);
    }
  }
  __syncthreads();
  return true;
}

// X (m x r) <- its polar factor X (X* X)^{-1/2} by Newton-Schulz steps
// X <- X (3 I - X* X) / 2 (products on MFMA; the error squares each step:
// a step taken from |X* X - I| <= 1e-8 is the last one).
// X and Y (m x r) swap roles as the iteration proceeds.  Returns false
// (workgroup-uniform; X spans the same space) if X* X is too far from I for
// the iteration or it does not settle.  For r <= 16 one wave forms X* X, its
// distance from I and the step matrix in registers: two barriers per step.
__device__ __forceinline__ bool polar_ns(double2 *&X, double2 *&Y, int m, int r, double2 *C, double *red, int *flag) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < 8; ++k) {
    if (r <= 16) {
      if (wave == 0) {
        const int li = lane & 15, lk = lane >> 4;
        d4v_g cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
        for (int kk = 0; kk < m; kk += 16) {
          double2 a[4], b[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int kr = kk + 4 * q + lk;
            a[q] = (kr < m && li < r) ? cconj(X[kr * r + li]) : make_double2(0, 0);
            b[q] = (kr < m && li < r) ? X[kr * r + li] : make_double2(0, 0);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].x, b[q].x, cre, 0, 0, 0);
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[q].y, b[q].y, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].x, b[q].y, cim, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].y, b[q].x, cim, 0, 0, 0);
          }
        }
        double dv = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 4 * v + lk, j = li;
          if (i < r && j < r) {
            const double cr = cre[v] - (i == j ? 1.0 : 0.0);
            dv = fmax(dv, fmax(fabs(cr), fabs(cim[v])));
            C[i * r + j] = make_double2((i == j ? 1.0 : 0.0) - 0.5 * cr, -0.5 * cim[v]);  // (3 I - X* X) / 2
          }
        }
        dv = max64(dv);
        if (lane == 0) *flag = dv <= 4e-16 ? 1 : (dv <= 1e-8 ? 3 : ((!(dv < 0.25) || k == 7) ? 2 : 0));
      }
      __syncthreads();
    } else {
      zgemm(C, r, X, r, true, X, r, r, r, m);  // C = X* X
      double dv = 0;
      for (int e = threadIdx.x; e < r * r; e += NT) {
        double2 c = C[e];
        if (e / r == e % r) c.x -= 1.0;
        dv = fmax(dv, fmax(fabs(c.x), fabs(c.y)));
      }
      dv = max64(dv);
      __syncthreads();
      if (lane == 0) red[wave] = dv;
      __syncthreads();
      double dev = 0;
      for (int w = 0; w < NW; ++w) dev = fmax(dev, red[w]);
      for (int e = threadIdx.x; e < r * r; e += NT)  // C <- (3 I - C) / 2
        C[e] = e / r == e % r ? make_double2(1.5 - 0.5 * C[e].x, -0.5 * C[e].y) : cscale(-0.5, C[e]);
      if (threadIdx.x == 0) *flag = dev <= 4e-16 ? 1 : (dev <= 1e-8 ? 3 : ((!(dev < 0.25) || k == 7) ? 2 : 0));
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();  // every thread has read the flag before it is rewritten
    if (f == 1) return true;
    if (f == 2) return false;
    zgemm(Y, r, X, r, false, C, r, m, r, r);  // Y = X (3 I - X* X) / 2
    double2 *t = X;
    X = Y;
    Y = t;
    if (f == 3) return true;  // |X* X - I| <= 1e-8 before the step: about 1e-16 after it
  }
  return false;
}

// Largest value over the workgroup of one value per thread; every thread
// gets the result.
__device__ double block_max(double v, double *red) {
  v = max64(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < NW; ++w) t = fmax(t, red[w]);
  return t;
}

// Eigenvectors of the Hermitian r x r G (ld r) by Newton refinement from
// Z = I: with P = Z* Z, S = Z* G Z and theta_i = S_ii / P_ii, the correction
// Z <- Z (I + E), E_ij = (S_ij - theta_j P_ij) / (theta_j - theta_i) (i != j),
// E_ii = (1 - P_ii) / 2, removes the off-diagonal of S and the departure of
// Z from orthonormality to first order together (the iterative refinement
// of an eigendecomposition of Ogita and Aishima), so that the error squares
// each step while the off-diagonal of G is small against the gaps of its
// eigenvalues.  The Ritz step's G is close to diagonal (the subspace
// iteration starts from the previous stage's eigenvectors), where this takes
// three or four steps of three small products instead of Jacobi sweeps.
// ZT (r x 2r, ld 2r) holds Z and G Z, PS (r x 2r, ld 2r) P and S, E (r x r)
// the correction; theta (r) the eigenvalues.  On return Z (first r columns of
// ZT) is orthonormal to rounding and diagonalises G to the same order.
// Returns false (workgroup-uniform) if the step does not contract (close
// eigenvalues), leaving G intact for another method.
__device__ bool ritz_refine(const double2 *G, int r, double2 *ZT, double2 *PS, double2 *E, double *theta,
                            double *red) {
  const int r2 = 2 * r;
  for (int e = threadIdx.x; e < r * r; e += NT) {
    const int i = e / r, c = e % r;
    ZT[i * r2 + c] = make_double2(i == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int it = 0; it < 8; ++it) {
    zgemm(ZT + r, r2, G, r, false, ZT, r2, r, r, r);  // G Z beside Z
    zgemm(PS, r2, ZT, r2, true, ZT, r2, r, r2, r);    // [P | S] = Z* [Z | G Z]
    for (int i = threadIdx.x; i < r; i += NT) theta[i] = PS[i * r2 + r + i].x / PS[i * r2 + i].x;
    __syncthreads();
    double off = 0;
    for (int e = threadIdx.x; e < r * r; e += NT) {
      const int i = e / r, j = e % r;
      const double2 pij = PS[i * r2 + j];
      double2 v;
      if (i == j) {
        v = make_double2(0.5 * (1.0 - pij.x), 0.0);
      } else {
        const double2 sij = PS[i * r2 + r + j];
        const double inv = 1.0 / (theta[j] - theta[i]);
        v = make_double2((sij.x - theta[j] * pij.x) * inv, (sij.y - theta[j] * pij.y) * inv);
        const double a = sqrt(cabs2(v));
        off = fmax(off, a == a ? a : 1e300);  // a NaN counts as no contraction
      }
      E[e] = v;
    }
    off = block_max(off, red);  // ends with a barrier: E is visible
    if (!(off < 0.5)) return false;
    zgemm(ZT + r, r2, ZT, r2, false, E, r, r, r, r);  // Z E
    for (int e = threadIdx.x; e < r * r; e += NT) {
      const int i = e / r, c = e % r;
      ZT[i * r2 + c] = cadd(ZT[i * r2 + c], ZT[i * r2 + r + c]);
    }
    __syncthreads();
    if (off < 1e-8) return true;  // the update just applied leaves an error of order off^2
  }
  return false;
}

// Words (double2) of arena the subspace iteration needs beyond K, and whether
// the arena holds them and the small eigenproblem (after C, or over K).
__device__ inline int warm_need(int m, int r) { return 2 * m * r + 2 * r * r; }
__device__ inline int warm_small(int r) { return r * (r + 1) / 2 + 2 * r * r; }
__device__ inline bool warm_fits(int m, int r, int arena_elems) {
  const int npl = m * (m + 1) / 2;
  return npl + warm_need(m, r) <= arena_elems &&
         (npl + warm_need(m, r) + warm_small(r) <= arena_elems || npl >= warm_small(r));
}

// u (rows_out x r, ld ldu, global) <- eigenvectors of the r largest eigenvalues
// of the Hermitian K (m x m, packed lower, in the LDS arena at K), descending,
// or false.  S: m x r start with orthonormal columns (ld lds_in).  The arena
// must hold K (npl words), then X, Y (m x r) and G, C (r x r); after the
// certificate the small eigenproblem's scratch goes after C if it fits there,
// else over K.  iters: iterations run.
__device__ __forceinline__ bool warm_top(double2 *K, int m, int r, const double2 *S, int lds_in, double2 *u, int ldu,
                         int rows_out, double2 *arena, int arena_elems, int maxit, double tol, JacobiShared &js,
                         int &iters, const double2 *rot = nullptr, const double *lam = nullptr,
                         double *ritz_ticks = nullptr, bool refine = true) {
  __shared__ double red[NW];
  __shared__ double s_lb[kMaxR];
  __shared__ int s_flag;
  const int npl = m * (m + 1) / 2;
  double2 *X = K + npl, *Y = X + m * r, *G = Y + m * r, *C = G + r * r;
  for (int e = threadIdx.x; e < m * r; e += NT) X[e] = S[(e / r) * lds_in + e % r];
  double kp = 0;
  for (int e = threadIdx.x; e < npl; e += NT) kp += cabs2(K[e]);
  double kd = 0;
  for (int i = threadIdx.x; i < m; i += NT) kd += cabs2(K[pl(i, i, m)]);
  const double kn2 = 2.0 * block_sum(kp, red) - block_sum(kd, red);  // ends with a barrier: X is visible
  int pre = 0;  // block products spent on the start
  if (rot) {
    // first-order predictor in the rotated basis (one block product):
    // X <- orth(S R + (I - S S*) K S R diag(1 / lam))
    zgemm(X, r, S, lds_in, false, rot, r, m, r, r);  // X = S R
    hemm_packed(Y, K, m, X, r);                      // Y = K X
    zgemm(C, r, S, lds_in, true, Y, r, r, r, m);     // C = S* Y
    for (int e = threadIdx.x; e < m * r; e += NT) {
      const int i = e / r, a = e % r;
      double2 v = Y[e];
      for (int c = 0; c < r; ++c) v = csub(v, cmul(S[i * lds_in + c], C[c * r + a]));
      X[e] = cadd(X[e], cscale(1.0 / lam[a], v));
    }
    __syncthreads();
    pre = 1;
    if (!polar_ns(X, Y, m, r, C, red, &s_flag) && !chol_qr(X, m, r, C)) {
      iters = pre;
      return false;
    }
  }
  double prev = 0, res2 = 0, g2 = 0;
  bool conv = false;
  int it = 0;
  for (; it < maxit; ++it) {
    hemm_packed(Y, K, m, X, r);                  // Y = K X
    zgemm(C, r, X, r, true, Y, r, r, r, m);      // C = X* Y
    double gp = 0;
    for (int e = threadIdx.x; e < r * r; e += NT) {  // G = Hermitian part
      const int a = e / r, b = e % r;
      const double2 x1 = C[a * r + b], x2 = C[b * r + a];
      const double2 g = make_double2(0.5 * (x1.x + x2.x), 0.5 * (x1.y - x2.y));
      G[e] = g;
      gp += cabs2(g);
    }
    g2 = block_sum(gp, red);
    res2 = block_sum(resid_part(Y, X, G, m, r), red);
    // converged: |Res| <= tol |G|, or stalled at rounding level below 100 tol |G|
    const double tol2 = tol * tol;
    conv = res2 <= tol2 * g2 || (it > 0 && res2 <= 1e4 * tol2 * g2 && res2 >= 0.25 * prev);
    if (conv) break;
    // give up early when the contraction measured from two residuals leaves
    // too many iterations
    if (it >= 1) {
      const double q = sqrt(res2 / prev);
      const double need = q < 1.0 ? log(sqrt(tol2 * g2 / res2)) / log(q) : 1e30;
      if (!(need <= (double)(maxit - it - 1))) {
        iters = pre + it + 1;
        return false;
      }
    }
    prev = res2;
    // X <- orth(Y diag(1 / G_aa)): the scaling keeps the columns near unit length
    for (int e = threadIdx.x; e < m * r; e += NT) {
      const double d = G[(e % r) * (r + 1)].x;
      X[e] = cscale(fabs(d) > 1e-280 ? 1.0 / d : 1.0, Y[e]);
    }
    __syncthreads();
    if (!polar_ns(X, Y, m, r, C, red, &s_flag) && !chol_qr(X, m, r, C)) {
      iters = pre + it + 1;
      return false;
    }
  }
  iters = pre + it + (conv ? 1 : 0);
  if (!conv) return false;
  // certificate (K still intact for the direct solver if it fails)
  {
    const double T = sqrt(fmax(kn2 - g2 - 2.0 * res2, 0.0)), res = sqrt(res2);
    for (int a = threadIdx.x; a < r; a += NT) {  // Gershgorin lower end of row a
      double rad = 0;
      for (int b = 0; b < r; ++b)
        if (b != a) rad += sqrt(cabs2(G[a * r + b]));
      s_lb[a] = G[a * (r + 1)].x - rad;
    }
    __syncthreads();
    double lb = 1e300;
    for (int a = 0; a < r; ++a) lb = fmin(lb, s_lb[a]);
    if (!(lb - res > T + res + 1e-13 * sqrt(kn2))) return false;
  }
  // Ritz vectors: G = Z diag(theta) Z*, theta descending, by Newton refinement
  // (ZT over Y, [P | S] over the small problem's scratch, E over C), else by
  // cyclic Jacobi (G is close to diagonal: few sweeps) on its packed upper
  // triangle
  double2 *Gp = (npl + warm_need(m, r) + warm_small(r) <= arena_elems) ? C + r * r : K;
  double2 *Zj = Gp + r * (r + 1) / 2, *Z = Zj + r * r;
  __shared__ double s_theta[kMaxR];
  uint64_t t_ritz = 0;
  if (threadIdx.x == 0) t_ritz = now_ticks();
  auto ritz_done = [&] {
    if (threadIdx.x == 0 && ritz_ticks) *ritz_ticks += (double)(now_ticks() - t_ritz);
  };
  if (refine && m >= 2 * r && ritz_refine(G, r, Y, Gp, C, s_theta, red)) {
    if (threadIdx.x < r) {  // rank by eigenvalue, descending (ties by index)
      const int a = threadIdx.x;
      int rank = 0;
      for (int b = 0; b < r; ++b)
        rank += (s_theta[b] > s_theta[a] || (s_theta[b] == s_theta[a] && b < a)) ? 1 : 0;
      js.order[rank] = a;
    }
    __syncthreads();
    // each column's phase: its component along the corresponding vector of X
    // real and positive (the vectors stay in the phases of the stage's start
    // basis, independent of the rounding of the refinement)
    for (int e = threadIdx.x; e < r * r; e += NT) {
      const int a = js.order[e % r];
      const double2 d = Y[a * 2 * r + a];
      const double n = sqrt(cabs2(d));
      const double2 ph = n > 0 ? make_double2(d.x / n, -d.y / n) : make_double2(1, 0);
      C[e] = cmul(Y[(e / r) * 2 * r + a], ph);
    }
    __syncthreads();
    zgemm(u, ldu, X, r, false, C, r, m, r, r);  // u = X Z
    for (int e = threadIdx.x; e < (rows_out - m) * r; e += NT) u[(m + e / r) * ldu + e % r] = make_double2(0, 0);
    __syncthreads();
    ritz_done();
    return true;
  }
  for (int e = threadIdx.x; e < r * r; e += NT) {
    const int i = e / r, j = e % r;
    if (i <= j) Gp[pk(i, j)] = G[e];
  }
  __syncthreads();
  if (threadIdx.x < 64) jacobi_wave(Gp, Zj, r, 4e-16, 12, js);
  __syncthreads();
  if (threadIdx.x == 0) {  // columns by eigenvalue, descending
    for (int k = 0; k < r; ++k) js.order[k] = k;
    for (int k = 0; k < r; ++k)
      for (int l = k + 1; l < r; ++l)
        if (Gp[pk(js.order[l], js.order[l])].x > Gp[pk(js.order[k], js.order[k])].x) {
          const int t = js.order[k];
          js.order[k] = js.order[l];
          js.order[l] = t;
        }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r * r; e += NT) Z[e] = Zj[(e / r) * r + js.order[e % r]];
  __syncthreads();
  zgemm(u, ldu, X, r, false, Z, r, m, r, r);  // u = X Z
  for (int e = threadIdx.x; e < (rows_out - m) * r; e += NT) u[(m + e / r) * ldu + e % r] = make_double2(0, 0);
  __syncthreads();
  ritz_done();
  return true;
}

// ----- pieces shared by the RK and AB projected-step kernels -------------------

// 1 if any of the n complex values is not finite (workgroup-uniform).
__device__ __forceinline__ int any_nonfinite(const double2 *x, int n) {
  int bad = 0;
  for (int e = threadIdx.x; e < n; e += NT)
    if (!isfinite(x[e].x) || !isfinite(x[e].y)) bad = 1;
  return __syncthreads_or(bad);
}

struct StepShared {
  JacobiShared js;
  TriShared ts;
  double2 vec[4 * kMaxR];
  double hbeta[kTriDim];
  unsigned char drop[kTriDim];
  double rkk[kTriDim];  // Cholesky: the diagonal of R (1 for a dropped direction)
  double gdiag[kTriDim];  // Cholesky: the full Gram's diagonal entries of the factored columns
  double minpiv, dev;
  int ndrop;
  double coef[kMaxStages > kMaxAb ? kMaxStages : kMaxAb];  // stage or AB weights, or error weights
};

// Cholesky of the n x n Hermitian block G (leading dimension ldg) into the
// upper triangle of R (ldr): G = R* R.  A direction whose pivot falls below
// 1e-13 of its diagonal in the full Gram matrix (orig[c * ldo]) is dependent on
// the earlier ones: its row of R is zeroed, its pivot set to 1 and drop[c] = 1.
// sh.minpiv / sh.ndrop report the smallest kept pivot ratio and the drops.
__device__ void chol_drop(const double2 *G, int ldg, const double2 *orig, int ldo, double2 *R, int ldr, int n,
                          double2 *arena, int arena_elems, unsigned char *drop, StepShared &sh) {
  const bool in_lds = n * n <= arena_elems;
  double2 *C = in_lds ? arena : R;
  const int ldc = in_lds ? n : ldr;
  for (int e = threadIdx.x; e < n * n; e += NT) C[(e / n) * ldc + e % n] = G[(e / n) * ldg + e % n];
  // the reference diagonal, read once instead of once per column
  for (int k = threadIdx.x; k < n; k += NT) sh.gdiag[k] = orig[k * ldo].x;
  if (threadIdx.x == 0) {
    sh.minpiv = 1.0;
    sh.ndrop = 0;
  }
  __syncthreads();
  // Right-looking elimination with one barrier per column: the trailing
  // block is updated with the unscaled row k, C_ij -= conj(C_ki) C_kj / piv,
  // and the rows are scaled by 1 / R_kk only at the end (row k is not written
  // again after step k).  Threads form a 16 x 32 grid over the upper triangle.
  for (int k = 0; k < n; ++k) {
    const double piv = C[k * ldc + k].x, og = sh.gdiag[k];
    const bool dropped = !(piv > 1e-13 * og) || !(og > 0);
    if (threadIdx.x == 0) {
      drop[k] = dropped;
      sh.rkk[k] = dropped ? 1.0 : sqrt(piv);
      if (dropped)
        sh.ndrop += 1;
      else
        sh.minpiv = fmin(sh.minpiv, piv / og);
    }
    if (!dropped) {
      const double ip = 1.0 / piv;
      for (int i = k + 1 + (threadIdx.x >> 5); i < n; i += NT / 32) {
        const double2 cki = cscale(ip, cconj(C[k * ldc + i]));
        for (int j = i + (threadIdx.x & 31); j < n; j += 32)
          C[i * ldc + j] = csub(C[i * ldc + j], cmul(cki, C[k * ldc + j]));
      }
    }
    if (in_lds) lds_barrier(); else __syncthreads();
  }
  // R: diagonal rkk, row k above it C_kj / rkk (zero for a dropped direction),
  // zero below (in place when C is R: each entry is read and written by one
  // thread)
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    double2 v = make_double2(0, 0);
    if (i == j)
      v = make_double2(sh.rkk[i], 0.0);
    else if (i < j && !drop[i])
      v = cscale(1.0 / sh.rkk[i], C[i * ldc + j]);
    R[i * ldr + j] = v;
  }
  __syncthreads();
}

// Ri = R^{-1} for the n x n upper triangular R: thread c owns column c and
// back-substitutes bottom-up; the column's own earlier results are re-read by
// the same thread only.  The substitution is a chain of dependent reads, so R
// and Ri are staged in the LDS arena when 2 n^2 elements fit there (in global
// memory otherwise).  Begins and ends with a barrier; the arena is scratch.
__device__ void upper_inverse(const double2 *R, int ldr, double2 *Ri, int ldi, int n, double2 *arena,
                              int arena_elems) {
  const bool in_lds = 2 * n * n <= arena_elems;
  const double2 *Rs = R;
  double2 *Is = Ri;
  int lr = ldr, li = ldi;
  if (in_lds) {
    for (int e = threadIdx.x; e < n * n; e += NT) arena[e] = R[(e / n) * ldr + e % n];
    Rs = arena;
    Is = arena + n * n;
    lr = li = n;
  }
  for (int e = threadIdx.x; e < n * n; e += NT) Is[(e / n) * li + e % n] = make_double2(0, 0);
  __syncthreads();
  // In LDS, G lanes (4, 8 or 16, an aligned part of a 16-lane row) share a
  // column: each sums every G-th product and a DPP reduction within the group
  // completes the sum, so the chain per entry is n / G products long.  Lane 0
  // of the group writes the entry, which the group's lanes read back in the
  // next steps (LDS accesses of one wave complete in order).
  const int lg = n <= 16 ? 4 : n <= 32 ? 4 : n <= 64 ? 3 : n <= 128 ? 2 : 0;
  if (in_lds && lg > 0 && (n << lg) <= NT) {
    const int G = 1 << lg, c = threadIdx.x >> lg, t = threadIdx.x & (G - 1);
    if (c < n) {
      if (t == 0) Is[c * li + c] = cdiv(make_double2(1, 0), Rs[c * lr + c]);
      for (int i = c - 1; i >= 0; --i) {
        double sr = 0, si = 0;
        for (int k = i + 1 + t; k <= c; k += G) {
          const double2 a = Rs[i * lr + k], b = Is[k * li + c];
          sr += a.x * b.x - a.y * b.y;
          si += a.x * b.y + a.y * b.x;
        }
        sr += dpp_d<0xB1>(sr);
        si += dpp_d<0xB1>(si);
        sr += dpp_d<0x4E>(sr);
        si += dpp_d<0x4E>(si);
        if (lg >= 3) {
          sr += dpp_d<0x141>(sr);
          si += dpp_d<0x141>(si);
        }
        if (lg >= 4) {
          sr += dpp_d<0x140>(sr);
          si += dpp_d<0x140>(si);
        }
        if (t == 0) Is[i * li + c] = cdiv(make_double2(-sr, -si), Rs[i * lr + i]);
      }
    }
  } else
  for (int c = threadIdx.x; c < n; c += NT) {
    Is[c * li + c] = cdiv(make_double2(1, 0), Rs[c * lr + c]);
    for (int i = c - 1; i >= 0; --i) {
      double sr = 0, si = 0;
#pragma unroll 8
      for (int k = i + 1; k <= c; ++k) {
        const double2 a = Rs[i * lr + k], b = Is[k * li + c];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
      }
      Is[i * li + c] = cdiv(make_double2(-sr, -si), Rs[i * lr + i]);
    }
  }
  __syncthreads();
  if (in_lds) {
    for (int e = threadIdx.x; e < n * n; e += NT) Ri[(e / n) * ldi + e % n] = Is[e];
    __syncthreads();
  }
}

// u (m x r) <- u (u* u)^{-1/2} when max|u* u - I| > 1e-14 (Lowdin), by the
// series below or an r x r Jacobi eigendecomposition.  S, Lw, T: r x r, r x r,
// m x r scratch (in the LDS arena after its first 3 r^2 elements where they
// fit, else global); u is copied to T once and every product reads T; the
// packed Jacobi matrices and the series terms use the arena's start.
__device__ __forceinline__ void lowdin(double2 *u, int m, int r, double2 *S, double2 *Lw, double2 *T,
                                       double2 *arena, StepShared &sh, double tol, int max_sweeps) {
  const int rr = r * r;
  for (int e = threadIdx.x; e < m * r; e += NT) T[e] = u[e];
  __syncthreads();
  zgemm(S, r, T, r, true, T, r, r, r, m);
  __syncthreads();
  {  // max |S - I| over the entries, by every thread and a workgroup maximum
    __shared__ double red[NW];
    double dev = 0;
    for (int e = threadIdx.x; e < rr; e += NT) {
      double2 g = S[e];
      if (e / r == e % r) g.x -= 1.0;
      dev = fmax(dev, sqrt(cabs2(g)));
    }
    dev = block_max(dev, red);
    if (threadIdx.x == 0) sh.dev = dev;
  }
  __syncthreads();
  if (!(sh.dev > 1e-14)) return;
  if (sh.dev <= 1e-6) {
    // S = I + E with |E|_2 <= r * 1e-6: S^{-1/2} = I - E/2 + 3/8 E^2 - 5/16 E^3,
    // the next term below 1e-19
    double2 *E = arena, *E2 = arena + rr, *E3 = arena + 2 * rr;
    for (int e = threadIdx.x; e < rr; e += NT) {
      const int a = e / r, b = e % r;
      const double2 x1 = S[a * r + b], x2 = S[b * r + a];
      E[e] = a == b ? make_double2(x1.x - 1.0, 0.0) : make_double2(0.5 * (x1.x + x2.x), 0.5 * (x1.y - x2.y));
    }
    __syncthreads();
    zgemm(E2, r, E, r, false, E, r, r, r, r);
    zgemm(E3, r, E2, r, false, E, r, r, r, r);
    for (int e = threadIdx.x; e < rr; e += NT) {
      const double2 t = cadd(cscale(-0.5, E[e]), cadd(cscale(0.375, E2[e]), cscale(-0.3125, E3[e])));
      Lw[e] = (e / r == e % r) ? make_double2(1.0 + t.x, t.y) : t;
    }
  } else {
    double2 *A = arena, *E = arena + rr;
    for (int e = threadIdx.x; e < rr; e += NT) {
      const int a = e / r, b = e % r;
      if (a <= b) {
        const double2 x1 = S[a * r + b], x2 = S[b * r + a];
        A[pk(a, b)] = a == b ? make_double2(x1.x, 0.0) : make_double2(0.5 * (x1.x + x2.x), 0.5 * (x1.y - x2.y));
      }
    }
    __syncthreads();
    jacobi(A, E, r, tol, max_sweeps, sh.js, true);
    __syncthreads();
    for (int e = threadIdx.x; e < rr; e += NT) {
      const int a = e / r, b = e % r;
      double2 acc = make_double2(0, 0);
      for (int k = 0; k < r; ++k)
        acc = cadd(acc, cscale(1.0 / sqrt(A[pk(k, k)].x), cmul(E[a * r + k], cconj(E[b * r + k]))));
      Lw[e] = acc;
    }
  }
  __syncthreads();
  zgemm(u, r, T, r, false, Lw, r, m, r, r);
  __syncthreads();
}

struct ModelCoef {
  int model;
  double kappa, hbar;
  const double *lam;
};

// Right-hand side f(rho) = z u* + u w* in coordinates (eqs. 3.2 / 4.1, 3.3-3.5):
// u (m x r, orthonormal columns) are the coordinates of V, y those of H V;
// G = u* y (symmetrised), X11 = Phi o G, c = phi(lam), w = (I - u u*) y diag(conj c)
// through the r Householder reflectors of u (hmode 1) or the projector (hmode 0),
// z = u X11 + w.  z, w are written with D rows (rows >= m zero).
// Scratch: Gr, X11 (r x r), t1, Uh, Yc (m x r, global); LDS arena >= 3 m r
// elements keeps the reflector work in LDS.  *energy (if set) = sum lam_a G_aa.
__device__ __forceinline__ void rhs_coords(const double2 *u, const double2 *y, int m, int D, int r, const ModelCoef &mc, int hmode,
                           double2 *z, double2 *w, double2 *Gr, double2 *X11, double2 *t1, double2 *Uh,
                           double2 *Yc, double2 *arena, int arena_elems, StepShared &sh, double *energy) {
  const int rr = r * r;
  double2 *cvec = sh.vec;  // c_a = phi(lam_a)
  double2 *dots = sh.vec + kMaxR;
  if (threadIdx.x < r) cvec[threadIdx.x] = phi(mc.lam[threadIdx.x], mc.model, mc.kappa, mc.hbar);
  zgemm(Gr, r, u, r, true, y, r, r, r, m);
  __syncthreads();
  for (int e = threadIdx.x; e < rr; e += NT) {
    const int a = e / r, b = e % r;
    const double2 g1 = Gr[a * r + b], g2 = Gr[b * r + a];
    const double2 gs = make_double2(0.5 * (g1.x + g2.x), 0.5 * (g1.y - g2.y));
    X11[e] = a == b ? make_double2(0, 0) : cmul(phi(mc.lam[a] - mc.lam[b], mc.model, mc.kappa, mc.hbar), gs);
  }
  if (energy && threadIdx.x == 0) {
    double en = 0;
    for (int a = 0; a < r; ++a) en += mc.lam[a] * Gr[a * r + a].x;
    *energy = en;
  }
  __syncthreads();
  if (hmode == 1 && r <= NT / 32 && m <= kTriDim) {
    // Householder vectors of u (m x r), eq. (3.3).  Half-wave c owns column c
    // of u (and later of y diag(conj c)) in registers, rows lane + 32 q; the
    // reflector vectors go to Vr (LDS when they fit), one barrier per reflector.
    constexpr int kS = (kTriDim + 31) / 32;
    const int hw = threadIdx.x >> 5, hl = threadIdx.x & 31, hbase = threadIdx.x & 32;
    const bool own = hw < r;
    double2 *Vr = (m * r <= arena_elems) ? arena : Uh;
    double2 x[kS];
#pragma unroll
    for (int q = 0; q < kS; ++q) {
      const int l = hl + 32 * q;
      x[q] = (own && l < m) ? u[l * r + hw] : make_double2(0, 0);
    }
    auto hsum = [&](double2 v) { return make_double2(sum32(v.x), sum32(v.y)); };
    for (int k = 0; k < r; ++k) {
      if (hw == k) {
        double s2 = 0;
#pragma unroll
        for (int q = 0; q < kS; ++q) {
          const int l = hl + 32 * q;
          if (l >= k && l < m) s2 += cabs2(x[q]);
        }
        s2 = sum32(s2);
        const double alpha = sqrt(s2);
        // x0 = row k of this column, held by lane k % 32 of the half-wave, slot k / 32
        double2 x0 = make_double2(0, 0);
#pragma unroll
        for (int q = 0; q < kS; ++q)
          if (q == k / 32) x0 = x[q];
        x0.x = __shfl(x0.x, hbase | (k & 31));
        x0.y = __shfl(x0.y, hbase | (k & 31));
        const double ax0 = sqrt(cabs2(x0));
        const double2 ph = ax0 > 0 ? cscale(1.0 / ax0, x0) : make_double2(1, 0);
#pragma unroll
        for (int q = 0; q < kS; ++q) {
          const int l = hl + 32 * q;
          if (l < m) {
            double2 v = l < k ? make_double2(0, 0) : x[q];
            if (l == k) v = cadd(v, cscale(alpha, ph));
            Vr[l * r + k] = v;
          }
        }
        if (hl == 0) sh.hbeta[k] = alpha > 1e-150 ? 1.0 / (alpha * alpha + alpha * ax0) : 0.0;
      }
      __syncthreads();
      if (own && hw > k) {  // apply P_k to the remaining columns
        double2 d = make_double2(0, 0);
#pragma unroll
        for (int q = 0; q < kS; ++q) {
          const int l = hl + 32 * q;
          if (l >= k && l < m) d = cadd(d, cmulc(Vr[l * r + k], x[q]));
        }
        d = cscale(sh.hbeta[k], hsum(d));
#pragma unroll
        for (int q = 0; q < kS; ++q) {
          const int l = hl + 32 * q;
          if (l >= k && l < m) x[q] = csub(x[q], cmul(Vr[l * r + k], d));
        }
      }
    }
    // w = Q [0; (Q^H y diag(conj c))_{r:}]: P_0 first, zero rows < r, then P_{r-1} first
    if (own) {
      const double2 cc = cconj(cvec[hw]);
#pragma unroll
      for (int q = 0; q < kS; ++q) {
        const int l = hl + 32 * q;
        x[q] = l < m ? cmul(y[l * r + hw], cc) : make_double2(0, 0);
      }
      for (int pass = 0; pass < 2; ++pass) {
        for (int kk = 0; kk < r; ++kk) {
          const int k = pass == 0 ? kk : r - 1 - kk;
          double2 d = make_double2(0, 0);
#pragma unroll
          for (int q = 0; q < kS; ++q) {
            const int l = hl + 32 * q;
            if (l >= k && l < m) d = cadd(d, cmulc(Vr[l * r + k], x[q]));
          }
          d = cscale(sh.hbeta[k], hsum(d));
#pragma unroll
          for (int q = 0; q < kS; ++q) {
            const int l = hl + 32 * q;
            if (l >= k && l < m) x[q] = csub(x[q], cmul(Vr[l * r + k], d));
          }
        }
        if (pass == 0) {
#pragma unroll
          for (int q = 0; q < kS; ++q)
            if (hl + 32 * q < r) x[q] = make_double2(0, 0);
        }
      }
#pragma unroll
      for (int q = 0; q < kS; ++q) {
        const int l = hl + 32 * q;
        if (l < D) w[l * r + hw] = l < m ? x[q] : make_double2(0, 0);
      }
    }
  } else if (hmode == 1) {
    // Householder vectors of u (m x r), eq. (3.3), column-parallel form (r > 16);
    // work arrays in LDS when they fit
    const bool hl = 3 * m * r <= arena_elems;
    double2 *Wk = hl ? arena : w;
    double2 *U_ = hl ? arena + m * r : Uh;
    double2 *Y_ = hl ? arena + 2 * m * r : Yc;
    for (int e = threadIdx.x; e < m * r; e += NT) {
      Wk[e] = u[e];
      Y_[e] = cmul(y[e], cconj(cvec[e % r]));
    }
    __syncthreads();
    for (int k = 0; k < r; ++k) {
      col_dots(dots, Wk + k * r + k, r, Wk + k * r + k, r, m - k, 1);
      const double alpha = sqrt(dots[0].x);
      const double2 x0 = Wk[k * r + k];
      const double ax0 = sqrt(cabs2(x0));
      const double2 ph = ax0 > 0 ? cscale(1.0 / ax0, x0) : make_double2(1, 0);
      for (int i = threadIdx.x; i < m; i += NT) {
        double2 v = i < k ? make_double2(0, 0) : Wk[i * r + k];
        if (i == k) v = cadd(v, cscale(alpha, ph));
        U_[i * r + k] = v;
      }
      if (threadIdx.x == 0) sh.hbeta[k] = alpha > 1e-150 ? 1.0 / (alpha * alpha + alpha * ax0) : 0.0;
      __syncthreads();
      if (k + 1 < r) {
        col_dots(dots, U_ + k, r, Wk, r, m, r);
        for (int e = threadIdx.x; e < m * r; e += NT) {
          const int i = e / r, c = e % r;
          if (c > k) Wk[e] = csub(Wk[e], cscale(sh.hbeta[k], cmul(U_[i * r + k], dots[c])));
        }
        __syncthreads();
      }
    }
    // Q^H Y = P_r ... P_1 Y (P_1 first), zero the span of u, then Q (P_r first)
    for (int k = 0; k < r; ++k) {
      col_dots(dots, U_ + k, r, Y_, r, m, r);
      for (int e = threadIdx.x; e < m * r; e += NT)
        Y_[e] = csub(Y_[e], cscale(sh.hbeta[k], cmul(U_[(e / r) * r + k], dots[e % r])));
      __syncthreads();
    }
    for (int e = threadIdx.x; e < rr; e += NT) Y_[e] = make_double2(0, 0);
    __syncthreads();
    for (int k = r - 1; k >= 0; --k) {
      col_dots(dots, U_ + k, r, Y_, r, m, r);
      for (int e = threadIdx.x; e < m * r; e += NT)
        Y_[e] = csub(Y_[e], cscale(sh.hbeta[k], cmul(U_[(e / r) * r + k], dots[e % r])));
      __syncthreads();
    }
    for (int e = threadIdx.x; e < D * r; e += NT) w[e] = e < m * r ? Y_[e] : make_double2(0, 0);
  } else {
    // projector form: W = (y - u G_raw) diag(conj c)
    zgemm(t1, r, u, r, false, Gr, r, m, r, r);
    __syncthreads();
    for (int e = threadIdx.x; e < D * r; e += NT)
      w[e] = e < m * r ? cmul(csub(y[e], t1[e]), cconj(cvec[e % r])) : make_double2(0, 0);
  }
  __syncthreads();
  zgemm(z, r, u, r, false, X11, r, m, r, r);
  __syncthreads();
  for (int e = threadIdx.x; e < D * r; e += NT) z[e] = e < m * r ? cadd(z[e], w[e]) : make_double2(0, 0);
  __syncthreads();
}

// The stage's y = R That R^{-1} u and f = z u* + u w* (projector form of the
// complement action; eqs. 3.2 / 4.1, 3.3-3.5) with every operand but R and
// R^{-1} in the LDS arena L (>= 4 D r + 2 r^2 words): the same products as
// rhs_coords, without the global round trips of its scratch blocks.  Writes
// z, w (D rows, rows >= mo zero) and Gr; bad[0..2] report non-finite u, y,
// z or w (workgroup-uniform).  Part one: u to LDS and y; part two: the rest.
struct StageLds {
  double2 *u, *y, *t, *c, *G, *X;
};
__device__ __forceinline__ StageLds stage_lds_layout(double2 *L, int D, int mo, int r) {
  StageLds a;
  a.u = L;
  a.y = a.u + mo * r;
  a.t = a.y + mo * r;
  a.c = a.t + D * r;
  a.G = a.c + mo * r;
  a.X = a.G + r * r;
  return a;
}
__device__ __forceinline__ void stage_hu_lds(const StageLds &a, const double2 *u, const double2 *R, const double2 *Ri,
                                             const double *shifts, double beta, int j, int mi, int mo, int D, int r,
                                             const unsigned char *drop, int *bad) {
  int b0 = 0;
  for (int e = threadIdx.x; e < mo * r; e += NT) {
    const double2 v = u[e];
    if (!isfinite(v.x) || !isfinite(v.y)) b0 = 1;
    a.u[e] = v;
  }
  bad[0] = __syncthreads_or(b0);
  zgemm(a.t, r, Ri, D, false, a.u, r, mi, r, mi);  // t = R^{-1} u
  const double ib = 1.0 / beta;
  for (int e = threadIdx.x; e < mo * r; e += NT) {
    const int row = e / r, col = e % r, bi = row / r, q = row % r;
    double2 v = bi <= j ? cscale(shifts[bi * r + q], a.t[e]) : make_double2(0, 0);
    if (bi >= 1 && bi - 1 <= j) v = cadd(v, cscale(ib, a.t[((bi - 1) * r + q) * r + col]));
    a.c[e] = v;  // That t
  }
  __syncthreads();
  zgemm(a.y, r, R, D, false, a.c, r, mo, r, mo);
  int b1 = 0;
  for (int e = threadIdx.x; e < mo * r; e += NT) {
    if (drop[e / r]) a.y[e] = make_double2(0, 0);
    const double2 v = a.y[e];
    if (!isfinite(v.x) || !isfinite(v.y)) b1 = 1;
  }
  bad[1] = __syncthreads_or(b1);
}
__device__ __forceinline__ void stage_rhs_lds(const StageLds &a, int mo, int D, int r, const ModelCoef &mc,
                                              double2 *z, double2 *w, double2 *Gr, StepShared &sh, double *energy,
                                              int *bad) {
  const int rr = r * r;
  double2 *cvec = sh.vec;  // c_a = phi(lam_a)
  if (threadIdx.x < r) cvec[threadIdx.x] = phi(mc.lam[threadIdx.x], mc.model, mc.kappa, mc.hbar);
  zgemm(a.G, r, a.u, r, true, a.y, r, r, r, mo);  // G = u* y
  for (int e = threadIdx.x; e < rr; e += NT) {
    const int p = e / r, q = e % r;
    const double2 g1 = a.G[p * r + q], g2 = a.G[q * r + p];
    const double2 gs = make_double2(0.5 * (g1.x + g2.x), 0.5 * (g1.y - g2.y));
    a.X[e] = p == q ? make_double2(0, 0) : cmul(phi(mc.lam[p] - mc.lam[q], mc.model, mc.kappa, mc.hbar), gs);
    Gr[e] = g1;
  }
  if (energy && threadIdx.x == 0) {
    double en = 0;
    for (int q = 0; q < r; ++q) en += mc.lam[q] * a.G[q * r + q].x;
    *energy = en;
  }
  __syncthreads();
  zgemm(a.t, r, a.u, r, false, a.G, r, mo, r, r);  // u G
  zgemm(a.c, r, a.u, r, false, a.X, r, mo, r, r);  // u X11
  int b2 = 0;
  for (int e = threadIdx.x; e < D * r; e += NT) {
    double2 wv = make_double2(0, 0), zv = make_double2(0, 0);
    if (e < mo * r) {
      wv = cmul(csub(a.y[e], a.t[e]), cconj(cvec[e % r]));  // w = (y - u G) diag(conj c)
      zv = cadd(a.c[e], wv);                                // z = u X11 + w
      if (!isfinite(wv.x) || !isfinite(wv.y) || !isfinite(zv.x) || !isfinite(zv.y)) b2 = 1;
    }
    w[e] = wv;
    z[e] = zv;
  }
  bad[2] = __syncthreads_or(b2);
}

// Packed (lower, column-major) Hermitian stage matrix of order m:
// K = u1 diag(lam) u1* + sum_l coef_l (z_l u_l* + u_l w_l*)   (eqs. 3.7-3.9;
// lam == nullptr: without the first term),
// formed as K = (P Q* + Q P*) / 2 over the factor pairs (P, Q) = (u1 diag(lam),
// u1), (coef_l z_l, u_l), (coef_l u_l, w_l), so that K is Hermitian to the last
// bit.  Lower 16 x 16 tiles, one per wave at a time, on FP64 MFMA with the
// factor rows (m x r, row-major) read straight from memory.
typedef double d4v_s __attribute__((ext_vector_type(4)));
__device__ inline d4v_s mfma_d(double a, double b, d4v_s c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Term l's factors are u0 + l*su, z0 + l*sz, w0 + l*sw; coef[l] may be in LDS.
__device__ __forceinline__ void stage_matrix(double2 *K, int m, int r, const double2 *u1, const double *lam, int nterm,
                             const double2 *u0, size_t su, const double2 *z0, size_t sz, const double2 *w0,
                             size_t sw, const double *coef, double2 *stg = nullptr, int stg_words = 0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mt = (m + 15) / 16, ntile = mt * (mt + 1) / 2;
  const int li = lane & 15, lk = lane >> 4;
  const int ldp = r + 1;  // odd row pitch in 16-byte words: the 16 rows of a tile fall on distinct banks
  if (stg && ntile <= 2 * NW && 2 * m * ldp <= stg_words) {
    // Channel by channel: the workgroup copies the channel's two factor blocks
    // (global, m x r each) into LDS with coalesced loads, then every wave adds
    // the channel to its (at most two) tiles, kept in registers across the
    // channels.  The factors are read from global memory once per channel
    // instead of once per tile.  stg may overlap K.
    double2 *Ps = stg, *Qs = stg + m * ldp;
    d4v_s kre[2], kim[2];
    int ra[2], rb[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      kre[q] = d4v_s{0, 0, 0, 0};
      kim[q] = d4v_s{0, 0, 0, 0};
      int ta = 0, rem = wave + q * NW;
      while (rem > ta) {
        rem -= ta + 1;
        ++ta;
      }
      ra[q] = ta * 16 + li;
      rb[q] = rem * 16 + li;
    }
    for (int ch = 0; ch < 1 + 2 * nterm; ++ch) {
      const double2 *P, *Q;
      double sc = 1.0;
      if (ch == 0) {
        if (!lam) continue;  // no u1 diag(lam) u1* term
        P = u1;
        Q = u1;
      } else {
        const int l = (ch - 1) / 2;
        sc = coef[l];
        if (sc == 0.0) continue;
        P = (ch & 1) ? z0 + l * sz : u0 + l * su;
        Q = (ch & 1) ? u0 + l * su : w0 + l * sw;
      }
      __syncthreads();  // the previous channel's products have read the blocks
      for (int e = threadIdx.x; e < m * r; e += NT) {
        const int i = e / r, c = e % r;
        Ps[i * ldp + c] = P[e];
        if (ch > 0) Qs[i * ldp + c] = Q[e];
      }
      __syncthreads();
      const double2 *Qx = ch > 0 ? Qs : Ps;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (wave + q * NW >= ntile) break;  // the same for the whole wave
        for (int kk = 0; kk < r; kk += 4) {
          const int c = kk + lk;
          const double sv = ch == 0 ? (c < r ? lam[c] : 0.0) : sc;
          const bool ok = c < r;
          const double2 z = make_double2(0, 0);
          const double2 pa = (ok && ra[q] < m) ? Ps[ra[q] * ldp + c] : z, qa = (ok && ra[q] < m) ? Qx[ra[q] * ldp + c] : z;
          const double2 pb = (ok && rb[q] < m) ? Ps[rb[q] * ldp + c] : z, qb = (ok && rb[q] < m) ? Qx[rb[q] * ldp + c] : z;
          // (s pa) conj(qb) + qa conj(s pb)
          const double a1r = sv * pa.x, a1i = sv * pa.y, b1r = qb.x, b1i = -qb.y;
          const double a2r = qa.x, a2i = qa.y, b2r = sv * pb.x, b2i = -sv * pb.y;
          kre[q] = mfma_d(a1r, b1r, kre[q]);
          kre[q] = mfma_d(-a1i, b1i, kre[q]);
          kim[q] = mfma_d(a1r, b1i, kim[q]);
          kim[q] = mfma_d(a1i, b1r, kim[q]);
          kre[q] = mfma_d(a2r, b2r, kre[q]);
          kre[q] = mfma_d(-a2i, b2i, kre[q]);
          kim[q] = mfma_d(a2r, b2i, kim[q]);
          kim[q] = mfma_d(a2i, b2r, kim[q]);
        }
      }
    }
    __syncthreads();  // K may overlap the staging blocks
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (wave + q * NW >= ntile) break;
      const int ta = (ra[q] - li) / 16, tb = (rb[q] - li) / 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ta * 16 + 4 * v + lk, col = tb * 16 + li;
        if (row < m && col <= row)
          K[pl(row, col, m)] = make_double2(0.5 * kre[q][v], row == col ? 0.0 : 0.5 * kim[q][v]);
      }
    }
    __syncthreads();
    return;
  }
  for (int t = wave; t < ntile; t += NW) {
    int ta = 0, rem = t;
    while (rem > ta) {
      rem -= ta + 1;
      ++ta;
    }
    const int tb = rem;  // ta >= tb
    d4v_s kre = {0, 0, 0, 0}, kim = {0, 0, 0, 0};
    const int ra = ta * 16 + li, rb = tb * 16 + li;
    for (int ch = 0; ch < 1 + 2 * nterm; ++ch) {
      const double2 *P, *Q;
      double sc = 1.0;
      if (ch == 0) {
        if (!lam) continue;  // no u1 diag(lam) u1* term
        P = u1;
        Q = u1;
      } else {
        const int l = (ch - 1) / 2;
        sc = coef[l];
        if (sc == 0.0) continue;
        P = (ch & 1) ? z0 + l * sz : u0 + l * su;
        Q = (ch & 1) ? u0 + l * su : w0 + l * sw;
      }
      for (int kk = 0; kk < r; kk += 4) {
        const int c = kk + lk;
        const double s = ch == 0 ? (c < r ? lam[c] : 0.0) : sc;
        const bool ok = c < r;
        const double2 z = make_double2(0, 0);
        const double2 pa = (ok && ra < m) ? P[ra * r + c] : z, qa = (ok && ra < m) ? Q[ra * r + c] : z;
        const double2 pb = (ok && rb < m) ? P[rb * r + c] : z, qb = (ok && rb < m) ? Q[rb * r + c] : z;
        // (s pa) conj(qb) + qa conj(s pb)
        const double a1r = s * pa.x, a1i = s * pa.y, b1r = qb.x, b1i = -qb.y;
        const double a2r = qa.x, a2i = qa.y, b2r = s * pb.x, b2i = -s * pb.y;
        kre = mfma_d(a1r, b1r, kre);
        kre = mfma_d(-a1i, b1i, kre);
        kim = mfma_d(a1r, b1i, kim);
        kim = mfma_d(a1i, b1r, kim);
        kre = mfma_d(a2r, b2r, kre);
        kre = mfma_d(-a2i, b2i, kre);
        kim = mfma_d(a2r, b2i, kim);
        kim = mfma_d(a2i, b2r, kim);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = ta * 16 + 4 * v + lk, col = tb * 16 + li;
      if (row < m && col <= row) K[pl(row, col, m)] = make_double2(0.5 * kre[v], row == col ? 0.0 : 0.5 * kim[v]);
    }
  }
  __syncthreads();
}

// Householder QR of M (m x q, row-major ld q, overwritten), m >= q:
// Q (m x q, orthonormal columns, explicit) and Rm (q x q upper) with M = Q Rm.
// Vh (m x q) holds the reflector vectors.
__device__ void householder_qr(double2 *M, int m, int q, double2 *Q, double2 *Rm, double2 *Vh, StepShared &sh) {
  double2 *dots = sh.vec;  // >= q entries needed: use Q's last row block as scratch when q > 4 r
  for (int e = threadIdx.x; e < m * q; e += NT) Vh[e] = make_double2(0, 0);
  __syncthreads();
  for (int k = 0; k < q; ++k) {
    col_dots(Rm + k * q + k, M + k * q + k, q, M + k * q + k, q, m - k, 1);  // |x|^2 parked in Rm
    const double alpha = sqrt(Rm[k * q + k].x);
    const double2 x0 = M[k * q + k];
    const double ax0 = sqrt(cabs2(x0));
    const double2 ph = ax0 > 0 ? cscale(1.0 / ax0, x0) : make_double2(1, 0);
    for (int i = k + threadIdx.x; i < m; i += NT) {
      double2 v = M[i * q + k];
      if (i == k) v = cadd(v, cscale(alpha, ph));
      Vh[i * q + k] = v;
    }
    if (threadIdx.x == 0) sh.hbeta[k] = alpha > 1e-150 ? 1.0 / (alpha * alpha + alpha * ax0) : 0.0;
    __syncthreads();
    // columns c > k: M[:, c] -= beta v (v* M[:, c]); column k becomes -ph alpha e_k
    for (int c = k + 1 + (threadIdx.x >> 6); c < q; c += NW) {
      const int lane = threadIdx.x & 63;
      double2 s = make_double2(0, 0);
      for (int i = k + lane; i < m; i += 64) s = cadd(s, cmulc(Vh[i * q + k], M[i * q + c]));
      s = wave_sum(s);
      const double2 f = cscale(sh.hbeta[k], s);
      for (int i = k + lane; i < m; i += 64) M[i * q + c] = csub(M[i * q + c], cmul(Vh[i * q + k], f));
    }
    __syncthreads();
    if (threadIdx.x == 0) M[k * q + k] = cscale(-alpha, ph);
    for (int i = k + 1 + threadIdx.x; i < m; i += NT) M[i * q + k] = make_double2(0, 0);
    __syncthreads();
  }
  for (int e = threadIdx.x; e < q * q; e += NT) Rm[e] = (e / q > e % q) ? make_double2(0, 0) : M[e];
  // Q = P_0 ... P_{q-1} [I; 0], reflectors applied last-first
  for (int e = threadIdx.x; e < m * q; e += NT) Q[e] = make_double2((e / q) == (e % q) ? 1.0 : 0.0, 0.0);
  __syncthreads();
  (void)dots;
  for (int k = q - 1; k >= 0; --k) {
    for (int c = k + (threadIdx.x >> 6); c < q; c += NW) {
      const int lane = threadIdx.x & 63;
      double2 s = make_double2(0, 0);
      for (int i = k + lane; i < m; i += 64) s = cadd(s, cmulc(Vh[i * q + k], Q[i * q + c]));
      s = wave_sum(s);
      const double2 f = cscale(sh.hbeta[k], s);
      for (int i = k + lane; i < m; i += 64) Q[i * q + c] = csub(Q[i * q + c], cmul(Vh[i * q + k], f));
    }
    __syncthreads();
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// LREI-RK projected step, one launch per stage j = 0 .. s-1.  Stage j needs
// only the Gram products of P_0 .. P_{j+1}, so it can run as soon as pass j
// is reduced, while the later passes proceed.  Each launch extends the Gram
// matrix, its Cholesky factor R (bordered form: R12 = R11^{-*} G12,
// R22 = chol(G22 - R12* R12)) and R^{-1} by the new Krylov block, then runs
// the stage.  State between launches lives in the workspace.
//
// The two halves are separate device functions: the basis extension (Gram
// columns, Cholesky, R^{-1}) needs only the Grams of pass j, the stage itself
// also the output of stage j - 1.  The single-trajectory step runs them as two
// kernels on two streams, so that the basis extension of stage j + 1 runs
// while stage j does; the batch kernel runs both in one launch.  They share no
// scratch: the extension writes columns [k0, k1) of the Gram, R and R^{-1}
// (rows and columns below k0 are all stage j reads of them), the drop flags
// of those columns, and its own scratch in the Hh block.
// ---------------------------------------------------------------------------

// phase timers (100 MHz real-time counter): slots 0..2 the extension, 3..7 the
// stage, each part adding only its own slots into stats[16..23]
// steps a stage goes to the direct eigensolver after a rejected warm start
constexpr int kWarmRetry = 8;     // steps on the direct solve after a first rejected warm start
constexpr int kWarmRetryMax = 64;  // ... doubled after each further rejection, up to this

// ---- learned start rotation: features and rotation of a stage -------------
//
// Stage j maps its input basis u (the state at c_in h, c_in = sum_l a_jl) to
// the eigenvectors of its stage matrix (the state at c_out h, c_out =
// sum_l a_{j+1,l}, or sum_l b_l at the last stage); s = (c_out - c_in) h /
// hbar is the step the in-span rotation covers.  Features: Re, Im of G / |G|_F
// (G = Herm(u* y), y = H u), s |G|_F, kappa.

// The step of the current attempt: fixed, or the controller's (adaptive).
__device__ inline double step_size(const SmallRkParams &p) { return p.ctl ? p.ctl[kCtlH] : p.h; }

__device__ double stage_step(const SmallRkParams &p, int j) {
  double cin = 0, cout = 0;
  for (int l = 0; l < p.s; ++l) {
    cin += j > 0 ? p.a[j][l] : 0.0;
    cout += (j + 1 == p.s) ? p.b[l] : p.a[j + 1][l];
  }
  return (cout - cin) * step_size(p) / p.hbar;
}

// G (r x r, Hermitian part of Gu = u* y, global) -> features f (2 r^2 + 2, LDS).
__device__ __forceinline__ void stage_features(const SmallRkParams &p, int j, const double2 *Gu, int r,
                                                       float *f, double *s_nrm) {
  if (threadIdx.x == 0) {
    double n2 = 0;
    for (int a = 0; a < r; ++a)
      for (int b = 0; b < r; ++b) {
        const double2 x = Gu[a * r + b], y = Gu[b * r + a];
        const double gr = 0.5 * (x.x + y.x), gi = 0.5 * (x.y - y.y);
        n2 += gr * gr + gi * gi;
      }
    *s_nrm = sqrt(n2);
  }
  __syncthreads();
  const double nrm = *s_nrm, inv = nrm > 0 ? 1.0 / nrm : 0.0;
  for (int e = threadIdx.x; e < r * r; e += NT) {
    const int a = e / r, b = e % r;
    const double2 x = Gu[a * r + b], y = Gu[b * r + a];
    f[e] = (float)(0.5 * (x.x + y.x) * inv);
    f[r * r + e] = (float)(0.5 * (x.y - y.y) * inv);
  }
  if (threadIdx.x == 0) {
    f[2 * r * r] = (float)(stage_step(p, j) * nrm);
    f[2 * r * r + 1] = (float)p.kappa;
  }
  __syncthreads();
}

// Scratch of the rotation at the arena's start, in floats (every region a
// multiple of 4 floats, so the FP64 regions stay 16-byte aligned): features,
// two hidden layers, NT partial sums, r^2 outputs, then [I - A/2 | I] and R.
struct RotScratch {
  int f, h0, h1, part, out, aug, R, total;
};
__device__ inline RotScratch rot_scratch(int r) {
  RotScratch q;
  q.f = 0;
  q.h0 = 4 * ((net_in(r) + 3) / 4);
  q.h1 = q.h0 + kNetWidth;
  q.part = q.h1 + kNetWidth;
  q.out = q.part + NT;
  q.aug = q.out + 4 * ((r * r + 3) / 4);
  q.R = q.aug + 4 * 2 * r * r;
  q.total = q.R + 4 * r * r;
  return q;
}

// The predictor's rotation R (r x r, written to Rg in global memory): I,
// Cayley(-i s G), or the network's.  ar: the arena (features at its start).
// Ends with a barrier.
__device__ __forceinline__ void stage_rotation(const SmallRkParams &p, int j, const double2 *Gu, int r,
                                                       float *ar, double2 *Rg) {
  const RotScratch q = rot_scratch(r);
  float *f = ar + q.f, *h0 = ar + q.h0, *h1 = ar + q.h1, *part = ar + q.part, *out = ar + q.out;
  double2 *aug = reinterpret_cast<double2 *>(ar + q.aug), *R = reinterpret_cast<double2 *>(ar + q.R);
  if (p.warm == LREI_WARM_LEARNED) {
    net_forward_wg(p.net, r, f, h0, h1, part, out, NT);  // ends with a barrier
    for (int e = threadIdx.x; e < r * r; e += NT) out[e] += analytic_param(f, r, e);
    __syncthreads();
  } else if (p.warm == LREI_WARM_PREDICT_CAYLEY) {
    // A = -i s G: o_a = -s G_aa; upper pairs (re, im) = (s Im G_ab, -s Re G_ab)
    const double st = stage_step(p, j);
    for (int e = threadIdx.x; e < r * r; e += NT) {
      const int a = e / r, b = e % r;
      const double2 x = Gu[a * r + b], y = Gu[b * r + a];
      const double gr = 0.5 * (x.x + y.x), gi = 0.5 * (x.y - y.y);
      if (a == b) {
        out[a] = (float)(-st * gr);
      } else if (a < b) {
        const int k = r + 2 * (a * r - a * (a + 1) / 2 + (b - a - 1));
        out[k] = (float)(st * gi);
        out[k + 1] = (float)(-st * gr);
      }
    }
    __syncthreads();
  } else {
    for (int e = threadIdx.x; e < r * r; e += NT) out[e] = 0.0f;  // A = 0: R = I
    __syncthreads();
  }
  if (threadIdx.x < 64) cayley_wave(out, r, aug, R, nullptr);
  __syncthreads();
  for (int e = threadIdx.x; e < r * r; e += NT) Rg[e] = R[e];
  __syncthreads();
}

struct PhaseClock {
  uint64_t mark;
  double acc[8];
};

// ---- adaptive stepping: error estimate and step-size controller -----------
//
// The two candidate matrices of eq. 3.9 (weights b and the embedded b_hat)
// differ by E = h sum_l e_l (z_l u_l* + u_l w_l*), e = b - b_hat, over the
// right-hand sides f_0 .. f_k.  The projection onto the fixed spectrum keeps,
// to first order, the part of E tangent to the fixed-spectrum manifold at the
// new state ub:  |T(E)|^2 = 2 |E ub - ub M|^2 + sum_{i != j, lam_i != lam_j}
// |M_ij|^2 with M = ub* E ub.  The estimate |T(E)|_F decides the attempt
// (accept when <= tol) and the next step, h min(facmax, max(facmin,
// 0.9 (tol / err)^(1 / (q + 1)))) clamped to [h_min, h_max] and to the time
// left (Hairer, Norsett & Wanner, Sec. II.4); a rejected attempt keeps the
// state (C = [I; 0]: V_new = P_0 = V).
constexpr double kFac = 0.9, kFacMin = 0.2, kFacMax = 5.0;

__device__ __forceinline__ void adapt_control(const SmallRkParams &p, const SmallWs &ws, int k, double h, const double2 *ub,
                              double2 *E, double2 *EV, double2 *M, double *coef) {
  __shared__ double red[NW];
  __shared__ int s_accept;
  const int r = p.r, D = p.nblocks * r;
  if (threadIdx.x <= k) coef[threadIdx.x] = h * p.e[threadIdx.x];
  __syncthreads();
  stage_matrix(E, D, r, nullptr, nullptr, k + 1, ws.stage, (size_t)3 * D * r, ws.stage + D * r, (size_t)3 * D * r,
               ws.stage + 2 * D * r, (size_t)3 * D * r, coef);
  hemm_packed(EV, E, D, ub, r);
  zgemm(M, r, ub, r, true, EV, r, r, r, D);  // M = ub* E ub
  double part = 2.0 * resid_part(EV, ub, M, D, r);
  for (int e = threadIdx.x; e < r * r; e += NT) {
    const int i = e / r, c = e % r;
    if (i != c && p.lam[i] != p.lam[c]) part += cabs2(M[e]);
  }
  int bad = 0;
  for (int e = threadIdx.x; e < D * r; e += NT)
    if (!isfinite(ws.Cfin[e].x) || !isfinite(ws.Cfin[e].y)) bad = 1;
  bad = __syncthreads_or(bad);
  const double sum = block_sum(part, red);
  const double err = bad ? NAN : sqrt(sum);
  if (threadIdx.x == 0) {
    double *c = p.ctl;
    const double t = c[kCtlT], t_end = c[kCtlTEnd], tol = c[kCtlTol];
    const double h_min = c[kCtlHMin], h_max = c[kCtlHMax];
    const bool last = h >= t_end - t;  // this attempt was clamped to end on t_end
    const bool finite = isfinite(err);
    const bool accept = finite && err <= tol;
    double fac = !finite ? kFacMin : (err > 0.0 ? kFac * pow(tol / err, 1.0 / (p.order_low + 1)) : kFacMax);
    fac = fmin(c[kCtlAfterReject] != 0.0 ? 1.0 : kFacMax, fmax(kFacMin, fac));
    double h_new = fmin(h * fac, h_max);
    double t_new = t;
    if (accept) {
      t_new = last ? t_end : t + h;
      c[kCtlAccepted] += 1.0;
      c[kCtlErrMax] = fmax(c[kCtlErrMax], err);
    } else {
      c[kCtlRejected] += 1.0;
      if (h <= h_min) c[kCtlFailed] = 1.0;
    }
    h_new = fmax(h_new, h_min);
    const bool done = accept && last;
    c[kCtlH] = done ? h_new : fmin(h_new, t_end - t_new);
    c[kCtlT] = t_new;
    c[kCtlDone] = done ? 1.0 : 0.0;
    c[kCtlErr] = err;
    c[kCtlAfterReject] = accept ? 0.0 : 1.0;
    c[kCtlAttempts] += 1.0;
    s_accept = accept ? 1 : 0;
  }
  __syncthreads();
  if (!s_accept)
    for (int e = threadIdx.x; e < D * r; e += NT)
      ws.Cfin[e] = make_double2(e / r == e % r ? 1.0 : 0.0, 0.0);
  __syncthreads();
}

__device__ __forceinline__ void rk_basis(const SmallRkParams &p, const SmallWs &ws, int j, double2 *s_arena,
                                         StepShared &sh, PhaseClock &pc) {
  if (p.ctl && p.ctl[kCtlSkip] != 0.0) return;  // an attempt after the end (uniform)
  const int r = p.r, nb = p.nblocks, D = nb * r, rr = r * r;
  double2 *G = ws.gamma, *R = ws.R, *Ri = ws.Rinv;
  double2 *S22 = ws.Hh;                 // 2r x 2r Schur complement / R22^{-1} scratch
  double2 *t1 = ws.Hh + 4 * rr;         // k0 x r products (k0 <= s r; fits after S22 in D x D)
  double *flags = ws.flags;             // [D] dropped directions
  double *stats = ws.stats;
  const int arena = small_basis_lds_elems(p.lds_elems, r);
  const int k0 = j == 0 ? 0 : (j + 1) * r;  // first new column of the Gram matrix
  const int k1 = (j + 2) * r;               // end of the new columns
  const int nn = k1 - k0;
  if (threadIdx.x == 0) {
    pc.mark = now_ticks();
    for (int k = 0; k < 3; ++k) pc.acc[k] = 0.0;
  }
  auto lap = [&](int slot) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint64_t t = now_ticks();
      pc.acc[slot] += (double)(t - pc.mark);
      pc.mark = t;
    }
  };
  // ---- 1. Gram columns [k0, k1) -----------------------------------------------
  // pass 0 measured P0*P0, P0*P1, P1*P1; pass j >= 1 measured P_j*P_{j+1}, P_{j+1}*P_{j+1};
  // the other blocks of column j+1 follow from P_{i+1} = beta (H P_i - P_i D_i):
  // P_i* P_{j+1} = P_{i+1}* P_j + beta (D_i P_i* P_j - P_i* P_j D_j)
  auto gblk = [&](int bi, int bj) { return G + (bi * r) * D + bj * r; };
  auto put = [&](int bi, int bj, const double2 *M) {
    for (int e = threadIdx.x; e < rr; e += NT) gblk(bi, bj)[(e / r) * D + e % r] = M[e];
  };
  if (j == 0) {
    put(0, 0, ws.meas + 0 * rr);
    put(0, 1, ws.meas + 1 * rr);
    put(1, 1, ws.meas + 2 * rr);
  } else {
    put(j, j + 1, ws.meas + (3 * j + 0) * rr);
    put(j + 1, j + 1, ws.meas + (3 * j + 1) * rr);
  }
  __syncthreads();
  // symmetrise the measured diagonal blocks before they enter the recurrence
  for (int bi = (j == 0 ? 0 : j + 1); bi <= j + 1; ++bi) {
    for (int e = threadIdx.x; e < rr; e += NT) {
      const int a = e / r, b = e % r;
      double2 *M = gblk(bi, bi);
      if (a < b) {
        const double2 x1 = M[a * D + b], x2 = M[b * D + a];
        const double2 hh = make_double2(0.5 * (x1.x + x2.x), 0.5 * (x1.y - x2.y));
        M[a * D + b] = hh;
        M[b * D + a] = cconj(hh);
      } else if (a == b) {
        M[a * D + a].y = 0.0;
      }
    }
    __syncthreads();
  }
  auto gget = [&](int bi, int bj, int a, int b) {  // any block, via Hermitian symmetry
    return bi <= bj ? gblk(bi, bj)[a * D + b] : cconj(gblk(bj, bi)[b * D + a]);
  };
  if (j >= 1) {
    const double *Dsh = ws.shifts;  // [block][r]
    for (int e = threadIdx.x; e < j * rr; e += NT) {
      const int i = e / rr, a = (e % rr) / r, b = e % r;
      const double2 gij = gget(i, j, a, b);
      const double d = p.beta * (Dsh[i * r + a] - Dsh[j * r + b]);
      gblk(i, j + 1)[a * D + b] = cadd(gget(i + 1, j, a, b), cscale(d, gij));
    }
    __syncthreads();
  }
  // lower part of the new columns' rows
  for (int e = threadIdx.x; e < nn * k1; e += NT) {
    const int i = k0 + e / k1, c = e % k1;  // row i of the new block, column c
    if (i / r > c / r) G[i * D + c] = cconj(G[c * D + i]);
  }
  __syncthreads();

  lap(0);
  // ---- 2. Cholesky of the new columns (dependent directions dropped) -----------
  if (j == 0) {
    for (int c = threadIdx.x; c < D; c += NT) flags[c] = 0.0;
    chol_drop(G, D, G, D + 1, R, D, k1, s_arena, arena, sh.drop, sh);
    for (int c = threadIdx.x; c < k1; c += NT) flags[c] = sh.drop[c];
    // rows and columns beyond k1 stay zero until their stage
    for (int e = threadIdx.x; e < D * D; e += NT)
      if (e / D >= k1 || e % D >= k1) R[e] = make_double2(0, 0);
  } else {
    // R12 = Ri11^* G12 (dropped rows of R12 are zero), S = G22 - R12^* R12
    zgemm(t1, nn, Ri, D, true, G + k0, D, k0, nn, k0);
    for (int e = threadIdx.x; e < k0 * nn; e += NT) {
      const int i = e / nn, c = e % nn;
      R[i * D + k0 + c] = flags[i] != 0.0 ? make_double2(0, 0) : t1[e];
    }
    __syncthreads();
    zgemm(S22, nn, R + k0, D, true, R + k0, D, nn, nn, k0);
    for (int e = threadIdx.x; e < nn * nn; e += NT) {
      const int i = e / nn, c = e % nn;
      S22[e] = csub(G[(k0 + i) * D + k0 + c], S22[e]);
    }
    __syncthreads();
    chol_drop(S22, nn, G + k0 * (D + 1), D + 1, R + k0 * (D + 1), D, nn, s_arena, arena, sh.drop, sh);
    for (int c = threadIdx.x; c < nn; c += NT) flags[k0 + c] = sh.drop[c];
  }
  if (threadIdx.x == 0) {
    if (j == 0) {
      stats[2] = sh.ndrop;
      stats[3] = sh.minpiv;
    } else {
      stats[2] += sh.ndrop;
      stats[3] = fmin(stats[3], sh.minpiv);
    }
  }
  lap(1);
  // ---- 3. R^{-1} for the new columns: Ri22 = R22^{-1}, Ri12 = -Ri11 R12 Ri22 ------
  if (j == 0) {
    for (int e = threadIdx.x; e < D * D; e += NT) Ri[e] = make_double2(0, 0);
    upper_inverse(R, D, Ri, D, k1, s_arena, arena);
  } else {
    upper_inverse(R + k0 * (D + 1), D, Ri + k0 * (D + 1), D, nn, s_arena, arena);
    zgemm(t1, nn, Ri, D, false, R + k0, D, k0, nn, k0);       // Ri11 R12
    zgemm(S22, nn, t1, nn, false, Ri + k0 * (D + 1), D, k0, nn, nn);  // (Ri11 R12) Ri22
    for (int e = threadIdx.x; e < k0 * nn; e += NT) {
      const int i = e / nn, c = e % nn;
      Ri[i * D + k0 + c] = make_double2(-S22[e].x, -S22[e].y);
    }
    __syncthreads();
  }
  lap(2);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) stats[16 + k] += pc.acc[k] * 1e-5;  // ms
}

__device__ __forceinline__ void rk_stage(const SmallRkParams &p, const SmallWs &ws, int j, double2 *s_arena,
                                         StepShared &sh, PhaseClock &pc) {
  const int r = p.r, s = p.s, nb = p.nblocks, D = nb * r, rr = r * r;
  double2 *R = ws.R, *Ri = ws.Rinv;
  double2 *y = ws.work;                 // D x r
  double2 *t1 = y + D * r;              // D x r
  double2 *Uh = t1 + D * r;             // D x r Householder vectors (global fallback)
  double2 *Yc = Uh + D * r;             // D x r
  double2 *Vj = Yc + D * r;             // D x D eigensolver scratch (global fallback)
  double2 *Kg = Vj + D * D;             // D x D stage matrix (global fallback)
  double2 *X11 = Kg + D * D;            // r x r
  double2 *Gr = X11 + rr;               // r x r
  double2 *tmp = Gr + rr;               // r x r
  double2 *Lw = tmp + rr;               // r x r Lowdin factor
  double *flags = ws.flags;             // [D] dropped directions
  double *stats = ws.stats;
  const int arena = p.lds_elems;
  const int k1 = (j + 2) * r;
  if (p.ctl && p.ctl[kCtlSkip] != 0.0) return;  // an attempt after the end (uniform)
  if (threadIdx.x == 0) {
    pc.mark = now_ticks();
    for (int k = 3; k < 8; ++k) pc.acc[k] = 0.0;
    for (int k = 0; k < 7; ++k) sh.ts.tacc[k] = 0.0;
  }
  auto lap = [&](int slot) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint64_t t = now_ticks();
      pc.acc[slot] += (double)(t - pc.mark);
      pc.mark = t;
    }
  };
  for (int c = threadIdx.x; c < k1; c += NT) sh.drop[c] = flags[c] != 0.0;
  __syncthreads();
  // ---- u_1 = R[:, :r] (Lowdin re-orthonormalised), at the first stage -------------
  double2 *u1 = ws.stage;  // stage 0, slot u
  if (j == 0) {
    for (int e = threadIdx.x; e < D * r; e += NT) u1[e] = R[(e / r) * D + e % r];
    __syncthreads();
    if (D * r + 5 * rr <= arena)  // scratch in the arena, after the series' three terms
      lowdin(u1, D, r, s_arena + 3 * rr + D * r, s_arena + 4 * rr + D * r, s_arena + 3 * rr, s_arena, sh,
             p.eig_tol, p.max_sweeps);
    else
      lowdin(u1, D, r, tmp, Lw, t1, s_arena, sh, p.eig_tol, p.max_sweeps);
    if (threadIdx.x == 0) stats[4] = sh.dev;
  }

  // ---- 3. stage j -------------------------------------------------------------
  const double h = step_size(p);
  const ModelCoef mc{p.model, p.kappa, p.hbar, p.lam};
  {
    double2 *u = ws.stage + (3 * j + 0) * D * r;
    double2 *z = ws.stage + (3 * j + 1) * D * r;
    double2 *w = ws.stage + (3 * j + 2) * D * r;
    const int mi = (j + 1) * r;  // support of u
    const int mo = (j + 2) * r;  // support of y = H u
    // first non-finite value: stats[28] = 10 * stage + phase (1 u, 2 y, 3 z/w, 4 K, 5 eigenvectors)
    if (threadIdx.x == 0 && j == 0) stats[28] = -1;
    if (p.householder_mode == 0 && 4 * D * r + 2 * rr <= arena) {
      // the stage's right-hand side with its operands in LDS
      const StageLds a = stage_lds_layout(s_arena, D, mo, r);
      int bad[3];
      stage_hu_lds(a, u, R, Ri, ws.shifts, p.beta, j, mi, mo, D, r, sh.drop, bad);
      lap(3);
      stage_rhs_lds(a, mo, D, r, mc, z, w, Gr, sh, j == 0 ? &stats[5] : nullptr, bad);
      if (threadIdx.x == 0 && stats[28] < 0 && (bad[0] | bad[1] | bad[2]))
        stats[28] = 10 * j + (bad[0] ? 1 : (bad[1] ? 2 : 3));
    } else {
    // y = R That R^{-1} u, That the block-bidiagonal relation H P_i = P_i D_i + P_{i+1} / beta
    zgemm(t1, r, Ri, D, false, u, r, mi, r, mi);
    {
      const double ib = 1.0 / p.beta;
      for (int e = threadIdx.x; e < mo * r; e += NT) {
        const int row = e / r, col = e % r, bi = row / r, a = row % r;
        double2 v = bi <= j ? cscale(ws.shifts[bi * r + a], t1[e]) : make_double2(0, 0);
        if (bi >= 1 && bi - 1 <= j) v = cadd(v, cscale(ib, t1[((bi - 1) * r + a) * r + col]));
        Yc[e] = v;  // That * t1
      }
    }
    __syncthreads();
    zgemm(y, r, R, D, false, Yc, r, mo, r, mo);
    for (int e = threadIdx.x; e < mo * r; e += NT)
      if (sh.drop[e / r]) y[e] = make_double2(0, 0);
    lap(3);
    rhs_coords(u, y, mo, D, r, mc, p.householder_mode, z, w, Gr, X11, t1, Uh, Yc, s_arena, arena, sh,
               j == 0 ? &stats[5] : nullptr);
    {
      const int f1 = any_nonfinite(u, D * r), f2 = any_nonfinite(y, D * r);
      const int f3 = any_nonfinite(z, D * r) | any_nonfinite(w, D * r);
      if (threadIdx.x == 0 && stats[28] < 0 && (f1 | f2 | f3)) stats[28] = 10 * j + (f1 ? 1 : (f2 ? 2 : 3));
    }
    }
    lap(4);
    if (j == s) {
      // error stage of a pair that also weights f at the new state (u = that
      // state): the estimate and the controller, no stage matrix
      const int npl = D * (D + 1) / 2;
      adapt_control(p, ws, j, h, u, npl <= arena ? s_arena : Kg, Yc, X11, sh.coef);
    } else {
    // learned start rotation: the stage's features (recorded as a training
    // sample and/or fed to the network) and the predictor's rotation R (into
    // tmp), in the arena before the stage matrix takes it
    __shared__ int s_slot;
    __shared__ double s_nrm;
    const bool fits = r <= kNetMaxR && rot_scratch(r).total <= 4 * arena;
    const bool record = p.rec != nullptr && fits;
    const bool use_rot = fits && (p.warm == LREI_WARM_PREDICT_IDENTITY || p.warm == LREI_WARM_PREDICT_CAYLEY ||
                                  (p.warm == LREI_WARM_LEARNED && p.net != nullptr));
    if (use_rot || record) {
      float *ar = reinterpret_cast<float *>(s_arena);
      stage_features(p, j, Gr, r, ar, &s_nrm);
      if (record) {
        if (threadIdx.x == 0) s_slot = atomicAdd(p.rec_count, 1);
        __syncthreads();
        if (s_slot < p.rec_cap) {
          float *dst = p.rec + (size_t)s_slot * net_sample_floats(r);
          for (int e = threadIdx.x; e < net_in(r); e += NT) dst[e] = ar[e];
        }
      }
      if (use_rot) stage_rotation(p, j, Gr, r, ar, tmp);
      __syncthreads();
    }
    // stage matrix (eqs. 3.7-3.9) and its top-r eigenvectors
    const bool last = (j + 1 == s);
    const int m = mo;
    const int SL = r <= 16 ? 16 : 32;
    const int npl = m * (m + 1) / 2;
    const bool jl = (npl + 2 * m * SL <= arena);
    double2 *K = jl ? s_arena : Kg;
    double *scr = jl ? reinterpret_cast<double *>(s_arena + npl) : reinterpret_cast<double *>(Vj);
    if (threadIdx.x <= j) sh.coef[threadIdx.x] = h * (last ? p.b[threadIdx.x] : p.a[j + 1][threadIdx.x]);
    __syncthreads();
    // the arena branch passes s_arena itself, so that the compiler sees LDS
    // accesses (a pointer chosen at run time is generic: flat instructions)
    if (jl)
      stage_matrix(s_arena, m, r, u1, p.lam, j + 1, ws.stage, (size_t)3 * D * r, ws.stage + D * r,
                   (size_t)3 * D * r, ws.stage + 2 * D * r, (size_t)3 * D * r, sh.coef, s_arena, arena);
    else
      stage_matrix(Kg, m, r, u1, p.lam, j + 1, ws.stage, (size_t)3 * D * r, ws.stage + D * r, (size_t)3 * D * r,
                   ws.stage + 2 * D * r, (size_t)3 * D * r, sh.coef);
    lap(5);
    {
      int fk = 0;
      for (int e = threadIdx.x; e < m * (m + 1) / 2; e += NT)
        if (!isfinite(K[e].x) || !isfinite(K[e].y)) fk = 1;
      fk = __syncthreads_or(fk);
      if (threadIdx.x == 0 && stats[28] < 0 && fk) stats[28] = 10 * j + 4;
    }
    double2 *unext = last ? ws.Cfin /* temporary */ : ws.stage + (3 * (j + 1) + 0) * D * r;
    bool solved = false;
    if ((p.warm == LREI_WARM_ANALYTIC || use_rot) && jl && K == s_arena && warm_fits(m, r, arena)) {
      // subspace iteration from the stage's input basis u, in the LDS arena
      // after K (over the direct solver's scratch, which it rebuilds if it
      // runs).  A stage whose last attempt was rejected goes to the direct
      // solver for the next kWarmRetry steps, twice as many after each
      // further rejection in a row (up to kWarmRetryMax; an accepted attempt
      // resets it): the spectrum of a stage matrix changes little from one
      // step to the next.  warm_skip[kMaxStages + j] keeps the current span.
      const double skip = ws.warm_skip[j];
      __syncthreads();  // every thread has read the counter before it changes
      if (skip > 0.0) {
        if (threadIdx.x == 0) ws.warm_skip[j] = skip - 1.0;
      } else {
        int its = 0;
        uint64_t t_w = 0;
        if (threadIdx.x == 0) t_w = now_ticks();
        solved = warm_top(s_arena, m, r, u, r, unext, r, D, s_arena, arena, 10, p.warm_tol, sh.js, its,
                          use_rot ? tmp : nullptr, p.lam, &sh.ts.tacc[6],
                          // the learned start's inputs depend on the eigenvectors'
                          // phases: the paths that record or use it keep the phase
                          // convention of the Jacobi rotations it was trained with
                          !(record || use_rot));
        if (threadIdx.x == 0) sh.ts.tacc[5] += (double)(now_ticks() - t_w);
        if (threadIdx.x == 0) {
          stats[solved ? 9 : 31] += 1;
          stats[12] += its;
          const double span = solved ? 0.0 : fmin((double)kWarmRetryMax, fmax((double)kWarmRetry,
                                                                               2.0 * ws.warm_skip[kMaxStages + j]));
          ws.warm_skip[j] = span;
          ws.warm_skip[kMaxStages + j] = span;
        }
      }
    }
    if (!solved) {
      if (jl)
        eig_top(s_arena, m, r, unext, r, D, reinterpret_cast<double *>(s_arena + npl), true, sh.ts);
      else
        eig_top(Kg, m, r, unext, r, D, scr, false, sh.ts);
    }
    if (record && s_slot < p.rec_cap) {  // training target T = u* u_next
      zgemm(X11, r, u, r, true, unext, r, r, r, D);
      float *dst = p.rec + (size_t)s_slot * net_sample_floats(r) + net_in(r);
      for (int e = threadIdx.x; e < r * r; e += NT) {
        dst[2 * e] = (float)X11[e].x;
        dst[2 * e + 1] = (float)X11[e].y;
      }
    }
    {
      const int fe = any_nonfinite(unext, D * r);
      if (threadIdx.x == 0 && stats[28] < 0 && fe) stats[28] = 10 * j + 5;
    }
    lap(6);
    if (last) {
      for (int e = threadIdx.x; e < D * r; e += NT) t1[e] = ws.Cfin[e];
      __syncthreads();
      zgemm(ws.Cfin, r, Ri, D, false, t1, r, D, r, D);  // C = R^{-1} u_final
      if (p.ctl && p.err_stage == s) {
        // the error stage starts from the new state
        double2 *un = ws.stage + (3 * s + 0) * D * r;
        for (int e = threadIdx.x; e < D * r; e += NT) un[e] = t1[e];
        __syncthreads();
      } else if (p.ctl) {
        const int npl = D * (D + 1) / 2;
        adapt_control(p, ws, j, h, t1, npl <= arena ? s_arena : Kg, Yc, X11, sh.coef);
      }
    }
    }  // stage j < s
  }
  lap(7);
  int bad = 0;
  if (j + 1 == s) {
    int bad_local = 0;
    for (int e = threadIdx.x; e < D * r; e += NT)
      if (!isfinite(ws.Cfin[e].x) || !isfinite(ws.Cfin[e].y)) bad_local = 1;
    bad = __syncthreads_or(bad_local);
  }
  if (threadIdx.x == 0) {
    for (int k = 3; k < 8; ++k) stats[16 + k] += pc.acc[k] * 1e-5;  // ms
    for (int k = 0; k < 4; ++k) stats[24 + k] += sh.ts.tacc[k] * 1e-5;
    stats[29] += sh.ts.tacc[5] * 1e-5;
    stats[30] += sh.ts.tacc[6] * 1e-5;
    if (j + 1 == s) {
      stats[0] = 0;
      stats[1] = 0;
      stats[6] = 0;
      stats[7] = bad;
      stats[8] = s;  // eigensolves this step
      // running totals over the steps of one call (zeroed by the host per call)
      stats[11] += s;
      if (!p.ctl) stats[14] += bad;  // adaptive: the controller rejects the attempt instead
      stats[15] += 1;
    }
  }
  // The step's last kernel refreshes the Krylov column shifts for the next
  // step: D_i[a] becomes the Rayleigh quotient of column a of block i,
  // (P_i* H P_i)_aa / (P_i* P_i)_aa = D_i[a] + Re (P_i* P_{i+1})_aa / (beta (P_i* P_i)_aa),
  // so that the next blocks carry the part of H P_i that is new.  Only the
  // conditioning of the stored blocks depends on the shifts, not the space.
  const int last_kernel = (p.ctl && p.err_stage == p.s) ? p.s : p.s - 1;
  if (j == last_kernel) {
    const double2 *G = ws.gamma;
    for (int e = threadIdx.x; e < (nb - 1) * r; e += NT) {
      const int i = e / r, a = e % r;
      const double gii = G[(i * r + a) * D + i * r + a].x;
      const double gnext = G[(i * r + a) * D + (i + 1) * r + a].x;
      const double dn = ws.shifts[e] + gnext / (p.beta * gii);
      if (gii > 1e-280 && isfinite(dn)) ws.shifts[e] = dn;
    }
  }
}

// Basis extension of stage j (one workgroup).
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6))) void k_small_rk_basis(SmallRkParams p, SmallWs ws, int j) {
  extern __shared__ __align__(16) double2 s_arena[];
  __shared__ StepShared sh;
  __shared__ PhaseClock pc;
  rk_basis(p, ws, j, s_arena, sh, pc);
}

// Stage j after its basis extension (one workgroup).
__global__ __launch_bounds__(NT) void k_small_rk(SmallRkParams p, SmallWs ws, int j) {
  extern __shared__ __align__(16) double2 s_arena[];
  __shared__ StepShared sh;
  __shared__ PhaseClock pc;
  rk_stage(p, ws, j, s_arena, sh, pc);
}

// One workgroup per job of a batch: extension and stage in one launch.
__global__ __launch_bounds__(NT) void k_small_rk_batch(const SmallRkParams *__restrict__ ps,
                                                      const SmallWs *__restrict__ wss, int j) {
  extern __shared__ __align__(16) double2 s_arena[];
  __shared__ StepShared sh;
  __shared__ PhaseClock pc;
  const SmallRkParams &p = ps[blockIdx.x];
  const SmallWs &ws = wss[blockIdx.x];
  rk_basis(p, ws, j, s_arena, sh, pc);
  __syncthreads();  // the stage reads the flags, R and R^{-1} the extension wrote
  rk_stage(p, ws, j, s_arena, sh, pc);
}

void launch_small_rk_stage_batch(const SmallRkParams *p, const SmallWs *ws, int n_jobs, int lds_elems, int j,
                                 hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_small_rk_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kSmallLdsBytes);
    attr = true;
  }
  hipLaunchKernelGGL(k_small_rk_batch, dim3(n_jobs), dim3(NT), (size_t)lds_elems * sizeof(double2), s, p, ws, j);
}

namespace {
void small_rk_attrs() {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_small_rk, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kSmallLdsBytes);
    (void)hipFuncSetAttribute((const void *)k_small_rk_basis, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kSmallLdsBytes);
    attr = true;
  }
}
}  // namespace

void launch_small_rk(const SmallRkParams &p, const SmallWs &ws, hipStream_t s) {
  small_rk_attrs();
  const size_t lds = (size_t)p.lds_elems * sizeof(double2);
  const size_t lds_basis = (size_t)small_basis_lds_elems(p.lds_elems, p.r) * sizeof(double2);
  for (int j = 0; j < p.s; ++j) {
    hipLaunchKernelGGL(k_small_rk_basis, dim3(1), dim3(NT), lds_basis, s, p, ws, j);
    hipLaunchKernelGGL(k_small_rk, dim3(1), dim3(NT), lds, s, p, ws, j);
  }
}

void launch_small_rk_basis(const SmallRkParams &p, const SmallWs &ws, int j, hipStream_t s) {
  small_rk_attrs();
  hipLaunchKernelGGL(k_small_rk_basis, dim3(1), dim3(NT),
                     (size_t)small_basis_lds_elems(p.lds_elems, p.r) * sizeof(double2), s, p, ws, j);
}

void launch_small_rk_stage(const SmallRkParams &p, const SmallWs &ws, int j, hipStream_t s) {
  small_rk_attrs();
  hipLaunchKernelGGL(k_small_rk, dim3(1), dim3(NT), (size_t)p.lds_elems * sizeof(double2), s, p, ws, j);
}

namespace {
// Start of an adaptive attempt: every kernel of the attempt does nothing if
// the integration has already ended or failed.
__global__ void k_attempt_begin(double *ctl) {
  if (threadIdx.x == 0) ctl[kCtlSkip] = (ctl[kCtlDone] != 0.0 || ctl[kCtlFailed] != 0.0) ? 1.0 : 0.0;
}
}  // namespace

void launch_attempt_begin(double *ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_attempt_begin, dim3(1), dim3(64), 0, s, ctl);
}

// ---------------------------------------------------------------------------
// LREI-AB projected step and history update
//
// The history of an ABm run, f(rho_{k-l}) for l = 1..m-1 (Sec. 3.8), needs the
// supports V_{k-l} and H V_{k-l}.  Those blocks are nearly dependent (V_{k-1}
// differs from V_k by O(dt)), so they are kept as an orthonormal basis U of
// span{V_k, V_{k-l}, H V_{k-l}} in N-space together with their coordinates in
// U.  One step: X = H V_k (or, after an RK start-up step, X = [H V_j, V_{j+1}]
// and at the very first step also V_j) is orthogonalised against U in N-space,
// Y = X - U (U* X), with the products U* Y, Y* Y measured again; the basis
// B = [U, Y] then has a well-conditioned Gram matrix [[U*U, U*Y], [Y*U, Y*Y]].
// In its orthonormal coordinates this kernel forms the AB stage matrix
// rho_k + dt sum_l b_l f(rho_{k-l}), its top-r eigenvectors (spectrum reset to
// Lambda_0), and a new orthonormal history basis for the next step by a
// Householder QR of the coordinates of [V_{k+1}, V_k, H V_k, older pairs];
// the N-space rotation U_new = B T and V_{k+1} = B C run in the block pass.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(NT) void k_small_ab(SmallAbParams p, SmallAbWs ws) {
  extern __shared__ __align__(16) double2 s_arena[];
  __shared__ StepShared sh;
  const int r = p.r, rr = r * r, nU = p.nU, qx = p.qx, DU = nU * r, D = DU + qx * r;
  const int npk = p.npairs_keep, qn = (3 + 2 * npk) * r, ldc = qn + r;
  const int arena = p.lds_elems;
  double2 *G = ws.work;                 // D x D
  double2 *R = G + D * D;               // D x D
  double2 *Ri = R + D * D;              // D x D
  double2 *Mq = Ri + D * D;             // D x qn
  double2 *Qm = Mq + D * qn;            // D x qn
  double2 *Vh = Qm + D * qn;            // D x qn
  double2 *Rm = Vh + D * qn;            // qn x qn
  double2 *cu = Rm + qn * qn;           // [kMaxAb][2] x (D x r): u_l, y_l
  double2 *cz = cu + 2 * kMaxAb * D * r;  // [kMaxAb][2] x (D x r): z_l, w_l
  double2 *unew = cz + 2 * kMaxAb * D * r;  // D x r
  double2 *t1 = unew + D * r, *Uh = t1 + D * r, *Yc = Uh + D * r;  // D x r each
  double2 *Kg = Yc + D * r;             // D x D
  double2 *Sg = Kg + D * D;             // D x D scratch (eigensolver, global fallback)
  double2 *X11 = Sg + D * D, *Gr = X11 + rr, *tmp = Gr + rr, *Lw = tmp + rr;
  double *stats = ws.stats;
  if (threadIdx.x == 0)
    for (int k = 0; k < 7; ++k) sh.ts.tacc[k] = 0.0;

  // ---- Gram of B = [U, Y] from the measured products
  for (int e = threadIdx.x; e < D * D; e += NT) {
    const int i = e / D, j = e % D;
    const int bi = i / r, bj = j / r, a = i % r, b = j % r;
    double2 v;
    if (bi < nU && bj < nU) {
      const int lo = bi < bj ? bi : bj, hi = bi < bj ? bj : bi;
      const int g = lo * nU - lo * (lo - 1) / 2 + (hi - lo);
      v = bi <= bj ? ws.UUg[(g * r + a) * r + b] : cconj(ws.UUg[(g * r + b) * r + a]);
    } else if (bi < nU || bj < nU) {
      const int ui = bi < nU ? bi : bj, yq = (bi < nU ? bj : bi) - nU;
      const int g = ui * qx + yq;
      v = bi < nU ? ws.gBg[(g * r + a) * r + b] : cconj(ws.gBg[(g * r + b) * r + a]);
    } else {
      const int q1 = bi - nU, q2 = bj - nU;
      const int lo = q1 < q2 ? q1 : q2, hi = q1 < q2 ? q2 : q1;
      const int g = nU * qx + lo * qx - lo * (lo - 1) / 2 + (hi - lo);
      v = q1 <= q2 ? ws.gBg[(g * r + a) * r + b] : cconj(ws.gBg[(g * r + b) * r + a]);
    }
    G[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < D * D; e += NT) {  // exact Hermitian symmetry
    const int i = e / D, j = e % D;
    if (i < j) {
      const double2 x1 = G[e], x2 = G[j * D + i];
      const double2 hh = make_double2(0.5 * (x1.x + x2.x), 0.5 * (x1.y - x2.y));
      G[e] = hh;
      G[j * D + i] = cconj(hh);
    } else if (i == j) {
      G[e].y = 0.0;
    }
  }
  __syncthreads();
  chol_drop(G, D, G, D + 1, R, D, D, s_arena, arena, sh.drop, sh);
  upper_inverse(R, D, Ri, D, D, s_arena, arena);

  // ---- coordinates in the orthonormal basis B R^{-1}
  // of a vector held as U-coordinates x (DU x r): R[:, :DU] x
  auto coord_u = [&](double2 *out, const double2 *x) {
    for (int e = threadIdx.x; e < D * r; e += NT) {
      const int i = e / r, c = e % r;
      double sr = 0, si = 0;
      if (!sh.drop[i])
        for (int k = i; k < DU; ++k) {
          const double2 a = R[i * D + k], b = x[k * r + c];
          sr += a.x * b.x - a.y * b.y;
          si += a.x * b.y + a.y * b.x;
        }
      out[e] = make_double2(sr, si);
    }
    __syncthreads();
  };
  // of X block q = U c1_q + Y_q: R[:, :DU] c1_q + R[:, DU + q r + (0..r)], times scale
  auto coord_x = [&](double2 *out, int q, double scale) {
    for (int e = threadIdx.x; e < D * r; e += NT) {
      const int i = e / r, c = e % r;
      double sr = 0, si = 0;
      if (!sh.drop[i]) {
        for (int k = i; k < DU; ++k) {
          const int ui = k / r, a = k % r;
          const double2 cc = ws.c1g[((ui * qx + q) * r + a) * r + c];
          const double2 rv = R[i * D + k];
          sr += rv.x * cc.x - rv.y * cc.y;
          si += rv.x * cc.y + rv.y * cc.x;
        }
        const int col = DU + q * r + c;
        if (col >= i) {
          sr += R[i * D + col].x;
          si += R[i * D + col].y;
        }
      }
      out[e] = make_double2(scale * sr, scale * si);
    }
    __syncthreads();
  };
  double2 *u0 = cu, *y0 = cu + D * r;
  const double2 *vc_in = ws.coords_in;
  if (p.x_v0 >= 0) coord_x(u0, p.x_v0, 1.0); else coord_u(u0, vc_in);
  coord_x(y0, p.x_hv, p.hv_scale);
  const ModelCoef mc{p.model, p.kappa, p.hbar, p.lam};
  if (p.mode == 1) {
    lowdin(u0, D, r, tmp, Lw, t1, s_arena, sh, p.eig_tol, p.max_sweeps);
    if (threadIdx.x == 0) stats[4] = sh.dev;
    const int m = p.m_ab;
    for (int l = 1; l < m; ++l) {
      coord_u(cu + (2 * l) * D * r, vc_in + (1 + 2 * (l - 1)) * DU * r);
      coord_u(cu + (2 * l + 1) * D * r, vc_in + (2 + 2 * (l - 1)) * DU * r);
    }
    for (int l = 0; l < m; ++l)
      rhs_coords(cu + (2 * l) * D * r, cu + (2 * l + 1) * D * r, D, D, r, mc, p.householder_mode,
                 cz + (2 * l) * D * r, cz + (2 * l + 1) * D * r, Gr, X11, t1, Uh, Yc, s_arena, arena, sh,
                 l == 0 ? &stats[5] : nullptr);
    if (threadIdx.x < m) sh.coef[threadIdx.x] = p.h * p.bcoef[threadIdx.x];
    __syncthreads();
    const int SL = r <= 16 ? 16 : 32;
    const int npl = D * (D + 1) / 2;
    const bool jl = (npl + 2 * D * SL <= arena);
    double2 *K = jl ? s_arena : Kg;
    double *scr = jl ? reinterpret_cast<double *>(s_arena + npl) : reinterpret_cast<double *>(Sg);
    stage_matrix(K, D, r, u0, p.lam, m, cu, (size_t)2 * D * r, cz, (size_t)2 * D * r, cz + D * r,
                 (size_t)2 * D * r, sh.coef);
    eig_top(K, D, r, unew, r, D, scr, jl, sh.ts);
  } else {
    coord_x(unew, p.x_vnew, 1.0);
  }
  // ---- new history basis: Householder QR of [V_{k+1}, V_k, H V_k, pairs 1..npk]
  for (int e = threadIdx.x; e < D * qn; e += NT) {
    const int i = e / qn, col = e % qn, blk = col / r, c = col % r;
    double2 v;
    if (blk == 0) v = unew[i * r + c];
    else if (blk == 1) v = u0[i * r + c];
    else if (blk == 2) v = y0[i * r + c];
    else {
      const int l = (blk - 3) / 2 + 1, which = (blk - 3) % 2;
      v = p.mode == 1 ? cu[(2 * l + which) * D * r + i * r + c] : make_double2(0, 0);
    }
    Mq[e] = v;
  }
  __syncthreads();
  if (p.mode == 0 && npk > 0) {
    // bootstrap: older pairs come straight from their U-coordinates
    for (int l = 1; l <= npk; ++l)
      for (int which = 0; which < 2; ++which) {
        coord_u(t1, vc_in + (1 + 2 * (l - 1) + which) * DU * r);
        const int blk = 3 + 2 * (l - 1) + which;
        for (int e = threadIdx.x; e < D * r; e += NT) Mq[(e / r) * qn + blk * r + e % r] = t1[e];
        __syncthreads();
      }
  }
  householder_qr(Mq, D, qn, Qm, Rm, Vh, sh);
  // ---- outputs: T = R^{-1} Q (new U), C = R^{-1} u_new (new V), coordinates = Rm
  for (int e = threadIdx.x; e < D * ldc; e += NT) {
    const int i = e / ldc, col = e % ldc;
    double sr = 0, si = 0;
    if (col < qn || p.mode == 1)
      for (int k = i; k < D; ++k) {
        const double2 a = Ri[i * D + k];
        const double2 b = col < qn ? Qm[k * qn + col] : unew[k * r + (col - qn)];
        if (sh.drop[k]) continue;
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
      }
    ws.Cc[e] = make_double2(sr, si);
  }
  for (int e = threadIdx.x; e < (1 + 2 * (npk + 1)) * qn * r; e += NT) {
    const int slot = e / (qn * r), rem = e % (qn * r), i = rem / r, c = rem % r;
    ws.coords_out[e] = Rm[i * qn + slot * r + c];
  }
  __syncthreads();
  int bad_local = 0;
  for (int e = threadIdx.x; e < D * ldc; e += NT)
    if (!isfinite(ws.Cc[e].x) || !isfinite(ws.Cc[e].y)) bad_local = 1;
  const int bad = __syncthreads_or(bad_local);
  if (threadIdx.x == 0) {
    stats[2] = sh.ndrop;
    stats[3] = sh.minpiv;
    stats[7] = bad;
    stats[14] += bad;
    if (p.mode == 1) {
      stats[8] = 1;
      stats[11] += 1;
      stats[15] += 1;
    }
  }
}

void launch_small_ab(const SmallAbParams &p, const SmallAbWs &ws, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_small_ab, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kSmallLdsBytes);
    attr = true;
  }
  hipLaunchKernelGGL(k_small_ab, dim3(1), dim3(NT), (size_t)p.lds_elems * sizeof(double2), s, p, ws);
}

size_t small_ab_work_elems(int D, int qn, int r) {
  return 5 * (size_t)D * D + 3 * (size_t)D * qn + (size_t)qn * qn + 4 * (size_t)kMaxAb * D * r + 4 * (size_t)D * r +
         4 * (size_t)r * r;
}

// Gram-Schmidt coefficients of the block pass: rows [U blocks..., X blocks...],
// columns the Y blocks: C = [-c1; I] with c1_q = U* X_q.
__global__ void k_ab_cgs_coef(const double2 *c1g, int nU, int qx, int r, double2 *C) {
  const int DU = nU * r, D = DU + qx * r, ldc = qx * r;
  for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < D * ldc; e += blockDim.x * gridDim.x) {
    const int i = e / ldc, col = e % ldc;
    double2 v;
    if (i < DU) {
      const int ui = i / r, a = i % r, q = col / r, c = col % r;
      const double2 g = c1g[((ui * qx + q) * r + a) * r + c];
      v = make_double2(-g.x, -g.y);
    } else {
      v = make_double2(i - DU == col ? 1.0 : 0.0, 0.0);
    }
    C[e] = v;
  }
}

void launch_ab_cgs_coef(const double2 *c1g, int nU, int qx, int r, double2 *C, hipStream_t s) {
  hipLaunchKernelGGL(k_ab_cgs_coef, dim3(4), dim3(256), 0, s, c1g, nU, qx, r, C);
}

// ---------------------------------------------------------------------------
// Initial state from a non-orthogonal factor A (N x m): the run starts from
// the partial eigendecomposition of rho_0 = A A* / Tr(A A*) (Sec. 3.7).  The
// eigenpairs of rho_0 are those of the Gram matrix G = A* A (the same
// nonzero eigenvalues times Tr), with eigenvectors A W diag(w)^{-1/2}.
// ---------------------------------------------------------------------------

namespace {

// partials[block][pk(i, j)] = sum over the block's rows x of conj(A[x, i]) A[x, j], i <= j
__global__ __launch_bounds__(NT) void k_factor_gram(const double2 *__restrict__ A, long long N, int m,
                                                   double2 *__restrict__ partials) {
  const int np = m * (m + 1) / 2;
  for (int e = threadIdx.x; e < np; e += NT) {
    int j = 0;
    while ((j + 1) * (j + 2) / 2 <= e) ++j;
    const int i = e - j * (j + 1) / 2;
    double2 acc = make_double2(0, 0);
    for (long long x = blockIdx.x; x < N; x += gridDim.x) acc = cadd(acc, cmulc(A[x * m + i], A[x * m + j]));
    partials[(long long)blockIdx.x * np + e] = acc;
  }
}

// One workgroup: G = the partials summed in block order, its eigenpairs by
// Jacobi, descending; rank = #{w_a > 1e-14 w_1}; lam_a = w_a / sum_b w_b over
// the kept ones; C (m x m, row-major) = W[:, a] / sqrt(w_a) for a < rank, 0
// beyond.  info[0] = rank.
__global__ __launch_bounds__(NT) void k_factor_eig(const double2 *__restrict__ partials, int grid, int m,
                                                  double2 *__restrict__ C, double *__restrict__ lam,
                                                  int *__restrict__ info) {
  __shared__ double2 G[kMaxR * (kMaxR + 1) / 2], W[kMaxR * kMaxR];
  __shared__ JacobiShared js;
  __shared__ double w[kMaxR];
  __shared__ int s_rank;
  const int np = m * (m + 1) / 2;
  for (int e = threadIdx.x; e < np; e += NT) {
    double2 acc = make_double2(0, 0);
    for (int b = 0; b < grid; ++b) acc = cadd(acc, partials[(long long)b * np + e]);
    G[e] = acc;
  }
  __syncthreads();
  jacobi(G, W, m, 1e-16, 60, js, true);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < m; ++k) js.order[k] = k;
    for (int k = 0; k < m; ++k)
      for (int l = k + 1; l < m; ++l)
        if (G[pk(js.order[l], js.order[l])].x > G[pk(js.order[k], js.order[k])].x) {
          const int t = js.order[k];
          js.order[k] = js.order[l];
          js.order[l] = t;
        }
    const double top = G[pk(js.order[0], js.order[0])].x;
    int rank = 0;
    double tr = 0;
    for (int k = 0; k < m; ++k) {
      w[k] = G[pk(js.order[k], js.order[k])].x;
      if (w[k] > 1e-14 * top && top > 0) {
        rank = k + 1;
        tr += w[k];
      }
    }
    for (int k = 0; k < m; ++k) lam[k] = k < rank ? w[k] / tr : 0.0;
    s_rank = rank;
    info[0] = rank;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const int i = e / m, a = e % m;
    C[e] = a < s_rank ? cscale(1.0 / sqrt(w[a]), W[i * m + js.order[a]]) : make_double2(0, 0);
  }
}

// V[x, b] = sum_i A[x, i] C[i, b] (N x r, row-major; C has leading dimension m)
__global__ void k_factor_apply(const double2 *__restrict__ A, long long N, int m, const double2 *__restrict__ C,
                               int r, double2 *__restrict__ V) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < N * r;
       t += (long long)gridDim.x * blockDim.x) {
    const long long x = t / r;
    const int b = (int)(t % r);
    double2 acc = make_double2(0, 0);
    for (int i = 0; i < m; ++i) acc = cadd(acc, cmul(A[x * m + i], C[i * m + b]));
    V[t] = acc;
  }
}

}  // namespace

void launch_factor_eig(const double2 *A, long long N, int m, double2 *partials, int grid, double2 *C, double *lam,
                       int *info, hipStream_t s) {
  hipLaunchKernelGGL(k_factor_gram, dim3(grid), dim3(NT), 0, s, A, N, m, partials);
  hipLaunchKernelGGL(k_factor_eig, dim3(1), dim3(NT), 0, s, (const double2 *)partials, grid, m, C, lam, info);
}

void launch_factor_apply(const double2 *A, long long N, int m, const double2 *C, int r, double2 *V, hipStream_t s) {
  const long long total = N * r;
  const int grid = (int)std::min<long long>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(k_factor_apply, dim3(grid), dim3(256), 0, s, A, N, m, C, r, V);
}

}  // namespace lrei
