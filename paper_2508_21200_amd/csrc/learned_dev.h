// Device pieces of the learned start rotation shared by the training kernels
// and the stage kernel: the network's forward pass for one sample by one
// workgroup, and the Cayley map by one wave.
//
// Network: x (2 r^2 + 2 reals) -> 3 hidden layers of width 256 with SiLU ->
// r^2 reals o.  Parameters in one flat FP32 vector: W1 [in x 256] row-major,
// b1, W2 [256 x 256], b2, W3, b3, W4 [256 x r^2], b4; a layer is h W + b.
// The network's output is a correction to the analytic generator -i s G
// (G / |G| and s |G| are features): the skew-Hermitian A is unpacked from
// o + o_an(x), with A_aa = i o_a, then the upper off-diagonal entries row by
// row as (re, im) pairs, A_ba = -conj(A_ab).
// R = (I - A/2)^{-1} (I + A/2) = 2 (I - A/2)^{-1} - I.
#pragma once

#include <hip/hip_runtime.h>

#include "lrei_internal.h"

namespace lrei {

constexpr int kNetWidth = 256;
constexpr int kNetMaxR = 16;  // networks are built for r <= 16 (r^2 <= width)
__host__ __device__ inline int net_in(int r) { return 2 * r * r + 2; }
__host__ __device__ inline long long net_param_count(int r) {
  const long long a = net_in(r), w = kNetWidth, o = (long long)r * r;
  return a * w + w + 2 * (w * w + w) + w * o + o;
}
// one training sample: features, then T = u* u_next as r x r (re, im) pairs, row-major
__host__ __device__ inline int net_sample_floats(int r) { return net_in(r) + 2 * r * r; }

__device__ inline float silu_f(float z) { return z / (1.0f + __expf(-z)); }

// Entry e of o_an(x), the parametrisation of -i s G: -s G_aa on the diagonal,
// (s Im G_ab, -s Re G_ab) for the upper pairs; x = (Re G/|G|, Im G/|G|, s |G|, kappa).
__device__ inline float analytic_param(const float *x, int r, int e) {
  const float sg = x[2 * r * r];
  if (e < r) return -sg * x[e * r + e];
  const int k = e - r, pidx = k >> 1;
  int a = 0, rem = pidx;
  while (rem >= r - a - 1) {
    rem -= r - a - 1;
    ++a;
  }
  const int b = a + 1 + rem;
  return (k & 1) ? -sg * x[a * r + b] : sg * x[r * r + a * r + b];
}

// Forward pass of one sample by a workgroup of nt threads (nt a multiple of
// 2 * kNetWidth is not required; every thread takes part).  x: inputs (LDS),
// h0, h1: kNetWidth floats each (LDS), part: nt floats (LDS), out: r^2 floats.
// Begins and ends with a barrier.
__device__ inline void net_forward_wg(const float *__restrict__ P, int r, const float *x, float *h0, float *h1,
                                      float *part, float *out, int nt) {
  const int nin = net_in(r), no = r * r, W = kNetWidth;
  const float *in = x;
  long long off = 0;
  __syncthreads();
  for (int l = 0; l < 4; ++l) {
    const int K = l == 0 ? nin : W, N = l == 3 ? no : W;
    const float *Wt = P + off, *b = P + off + (long long)K * N;
    off += (long long)K * N + N;
    float *dst = l == 3 ? out : (l % 2 == 0 ? h0 : h1);
    // thread t: output o = t % N of slice s = t / N over the inputs
    const int slices = nt / N;
    const int o = threadIdx.x % N, sl = threadIdx.x / N;
    float acc = 0.0f;
    if (sl < slices) {
      const int k0 = (int)((long long)K * sl / slices), k1 = (int)((long long)K * (sl + 1) / slices);
      int k = k0;
      for (; k + 8 <= k1; k += 8) {
        float w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = Wt[(long long)(k + u) * N + o];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += in[k + u] * w[u];
      }
      for (; k < k1; ++k) acc += in[k] * Wt[(long long)k * N + o];
      part[threadIdx.x] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N; e += nt) {
      float s = b[e];
      for (int q = 0; q < slices; ++q) s += part[q * N + e];
      dst[e] = l == 3 ? s : silu_f(s);
    }
    __syncthreads();
    in = dst;
  }
}

// R = Cayley(A(o)) by the 64 lanes of one wave, in FP64: Gauss-Jordan with
// partial pivoting on [I - A/2 | I] (aug: r x 2r, LDS), then R = 2 M^{-1} - I.
// Minv (optional, r x r) receives M^{-1}.  Lanes synchronise at wave level.
__device__ inline void cayley_wave(const float *o, int r, double2 *aug, double2 *R, double2 *Minv) {
  const int lane = threadIdx.x & 63, w2 = 2 * r;
  for (int e = lane; e < r * w2; e += 64) {
    const int i = e / w2, c = e % w2;
    double2 v = make_double2(0, 0);
    if (c < r) {
      // M = I - A/2
      if (i == c) {
        v = make_double2(1.0, -0.5 * (double)o[i]);
      } else {
        const int a = i < c ? i : c, b = i < c ? c : i;
        const int k = r + 2 * (a * r - a * (a + 1) / 2 + (b - a - 1));
        const double re = o[k], im = o[k + 1];
        // A_ab = re + i im (a < b), A_ba = -re + i im
        v = i < c ? make_double2(-0.5 * re, -0.5 * im) : make_double2(0.5 * re, -0.5 * im);
      }
    } else {
      v = make_double2(c - r == i ? 1.0 : 0.0, 0.0);
    }
    aug[e] = v;
  }
  __builtin_amdgcn_wave_barrier();
  for (int k = 0; k < r; ++k) {
    // pivot: the largest |aug[i][k]|, i >= k (lowest index on ties)
    double best = -1.0;
    int bi = k;
    for (int i = k; i < r; ++i) {
      const double2 z = aug[i * w2 + k];
      const double a = z.x * z.x + z.y * z.y;
      if (a > best) {
        best = a;
        bi = i;
      }
    }
    if (bi != k)
      for (int c = lane; c < w2; c += 64) {
        const double2 t = aug[k * w2 + c];
        aug[k * w2 + c] = aug[bi * w2 + c];
        aug[bi * w2 + c] = t;
      }
    __builtin_amdgcn_wave_barrier();
    const double2 pv = aug[k * w2 + k];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const double2 ip = make_double2(pv.x / den, -pv.y / den);
    __builtin_amdgcn_wave_barrier();
    for (int c = lane; c < w2; c += 64) {
      const double2 z = aug[k * w2 + c];
      aug[k * w2 + c] = make_double2(z.x * ip.x - z.y * ip.y, z.x * ip.y + z.y * ip.x);
    }
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < r * w2; e += 64) {
      const int i = e / w2, c = e % w2;
      if (i == k) continue;
      const double2 f = aug[i * w2 + k], pk = aug[k * w2 + c];
      const double2 z = aug[e];
      aug[e] = make_double2(z.x - (f.x * pk.x - f.y * pk.y), z.y - (f.x * pk.y + f.y * pk.x));
    }
    __builtin_amdgcn_wave_barrier();
  }
  for (int e = lane; e < r * r; e += 64) {
    const int i = e / r, c = e % r;
    const double2 mi = aug[i * w2 + r + c];
    if (Minv) Minv[e] = mi;
    R[e] = make_double2(2.0 * mi.x - (i == c ? 1.0 : 0.0), 2.0 * mi.y);
  }
  __builtin_amdgcn_wave_barrier();
}

}  // namespace lrei
