// Host-side helpers shared by the single-trajectory context (api.hip) and the
// batch context (batch.hip): owned device buffers, the RK tableaux, and the
// upload of a Hamiltonian's term tables.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lrei_internal.h"

namespace lrei {

constexpr int kStatsLen = 32;  // per-trajectory statistics slots of the projected step

// An owned device allocation.  Copies share the pointer; release() frees it.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  bool ensure(size_t b) {
    if (b <= bytes && p) return true;
    release();
    if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
      return false;
    }
    bytes = b;
    return true;
  }
};

// The two streams of a context: the work stream (N-space passes; the
// caller's, or one owned by the library) and the side stream the projected
// step runs on, both non-blocking and at the default priority.
inline hipError_t create_streams(bool own_work, hipStream_t *work, hipStream_t *side) {
  if (own_work) {
    hipError_t e = hipStreamCreateWithFlags(work, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  return hipStreamCreateWithFlags(side, hipStreamNonBlocking);
}

// Butcher tableaux (Sec. 3.7).  RK2: the paper's Heun tableau; RK3: Kutta;
// RK4: classical.
inline void tableau(int scheme, int &s, double a[kMaxStages][kMaxStages], double b[kMaxStages]) {
  for (int i = 0; i < kMaxStages; ++i) {
    b[i] = 0;
    for (int j = 0; j < kMaxStages; ++j) a[i][j] = 0;
  }
  switch (scheme) {
    case LREI_RK1: s = 1; b[0] = 1; break;
    case LREI_RK2: s = 2; a[1][0] = 1; b[0] = b[1] = 0.5; break;
    case LREI_RK3:
      s = 3; a[1][0] = 0.5; a[2][0] = -1; a[2][1] = 2;
      b[0] = 1.0 / 6; b[1] = 4.0 / 6; b[2] = 1.0 / 6;
      break;
    default:
      s = 4; a[1][0] = 0.5; a[2][1] = 0.5; a[3][2] = 1;
      b[0] = 1.0 / 6; b[1] = 2.0 / 6; b[2] = 2.0 / 6; b[3] = 1.0 / 6;
      break;
  }
}

// Embedded pairs for adaptive stepping: the tableau (a, b) that advances the
// state, the error weights e = b - b_hat over the right-hand sides the
// estimate uses, the stage that forms the estimate (s - 1, or s when b_hat
// also weights f at the new state) and the order q of the embedded solution.
// HE21: Heun with Euler embedded.  BS32: Bogacki-Shampine 3(2),
// b_hat = (7/24, 1/4, 1/3, 1/8).  RK43: classical RK4, b_hat of order 3.
inline bool pair_tableau(int pair, int &s, double a[kMaxStages][kMaxStages], double b[kMaxStages],
                         double e[kMaxStages], int &err_stage, int &q) {
  for (int i = 0; i < kMaxStages; ++i) {
    b[i] = e[i] = 0;
    for (int j = 0; j < kMaxStages; ++j) a[i][j] = 0;
  }
  switch (pair) {
    case LREI_PAIR_HE21:
      s = 2; a[1][0] = 1; b[0] = b[1] = 0.5;
      e[0] = 0.5 - 1.0; e[1] = 0.5;
      err_stage = 1; q = 1;
      return true;
    case LREI_PAIR_BS32:
      s = 3; a[1][0] = 0.5; a[2][1] = 0.75;
      b[0] = 2.0 / 9; b[1] = 3.0 / 9; b[2] = 4.0 / 9;
      e[0] = 2.0 / 9 - 7.0 / 24; e[1] = 3.0 / 9 - 0.25; e[2] = 4.0 / 9 - 1.0 / 3; e[3] = -0.125;
      err_stage = 3; q = 2;
      return true;
    case LREI_PAIR_RK43:
      // the classical RK4 step; b_hat = (1, 2, 2, 0, 1) / 6 moves the last
      // weight to f at the new state
      tableau(LREI_RK4, s, a, b);
      e[3] = 1.0 / 6; e[4] = -1.0 / 6;
      err_stage = 4; q = 3;
      return true;
    default:
      return false;
  }
}

// Device copies of a term table: off-diagonal records in FP64 and FP32, the
// diagonal terms and the per-row diagonal d(x) in both precisions.
struct DevTerms {
  DevBuf off64, off32, diag, d64, d32;
  int n_off = 0, n_diag = 0;
  int cplx = 0;  // some off-diagonal coefficient has an imaginary part
  void release() {
    off64.release();
    off32.release();
    diag.release();
    d64.release();
    d32.release();
  }
};

// Uploads t for N = 2^n rows on stream s and waits for it.  On failure nothing
// is left allocated in out and err says why (LREI_E_INVALID: too many terms,
// LREI_E_NOMEM, LREI_E_DEVICE).
inline lrei_status upload_terms(const TermTable &t, long long N, hipStream_t s, DevTerms &out, std::string &err) {
  std::vector<DevOffTerm> off(t.off.size());
  std::vector<DevTerm<float>> off32(t.off.size());
  int cplx = 0;
  for (size_t i = 0; i < t.off.size(); ++i) {
    off[i].mask = off32[i].mask = t.off[i].mask;
    off[i].sa = off32[i].sa = t.off[i].sa;
    off[i].sb = off32[i].sb = t.off[i].sb;
    off[i].act = off32[i].act = 0;
    for (int q = 0; q < 4; ++q) {
      off[i].re[q] = t.off[i].re[q];
      off[i].im[q] = t.off[i].im[q];
      off32[i].re[q] = (float)t.off[i].re[q];
      off32[i].im[q] = (float)t.off[i].im[q];
      if (t.off[i].im[q] != 0.0) cplx = 1;
      if (off[i].re[q] != 0.0 || off[i].im[q] != 0.0) off[i].act |= 1u << q;
      if (off32[i].re[q] != 0.0f || off32[i].im[q] != 0.0f) off32[i].act |= 1u << q;
    }
  }
  std::vector<DevDiagTerm> dg(t.diag.size());
  for (size_t i = 0; i < t.diag.size(); ++i) dg[i] = {t.diag[i].si, t.diag[i].sj, t.diag[i].w};
  if (off.size() > 256 || dg.size() > 512) {
    err = "too many Hamiltonian terms (max 256 off-diagonal, 512 diagonal)";
    return LREI_E_INVALID;
  }
  DevTerms d;
  if (!d.off64.ensure(std::max<size_t>(1, off.size()) * sizeof(DevOffTerm)) ||
      !d.off32.ensure(std::max<size_t>(1, off.size()) * sizeof(DevTerm<float>)) ||
      !d.diag.ensure(std::max<size_t>(1, dg.size()) * sizeof(DevDiagTerm)) ||
      !d.d64.ensure((size_t)N * sizeof(double)) || !d.d32.ensure((size_t)N * sizeof(float))) {
    d.release();
    err = "device allocation failed";
    return LREI_E_NOMEM;
  }
  hipError_t he = hipSuccess;
  if (!off.empty()) {
    he = hipMemcpy(d.off64.p, off.data(), off.size() * sizeof(DevOffTerm), hipMemcpyHostToDevice);
    if (he == hipSuccess)
      he = hipMemcpy(d.off32.p, off32.data(), off32.size() * sizeof(DevTerm<float>), hipMemcpyHostToDevice);
  }
  if (he == hipSuccess && !dg.empty())
    he = hipMemcpy(d.diag.p, dg.data(), dg.size() * sizeof(DevDiagTerm), hipMemcpyHostToDevice);
  if (he == hipSuccess) {
    launch_diag_values((const DevDiagTerm *)d.diag.p, (int)dg.size(), N, (double *)d.d64.p, (float *)d.d32.p, s);
    he = hipGetLastError();
  }
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    d.release();
    err = std::string("upload Hamiltonian tables: ") + hipGetErrorString(he);
    return LREI_E_DEVICE;
  }
  d.n_off = (int)off.size();
  d.n_diag = (int)dg.size();
  d.cplx = cplx;
  out = d;
  return LREI_OK;
}

}  // namespace lrei
