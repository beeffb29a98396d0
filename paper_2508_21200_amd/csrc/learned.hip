// Learned start rotation for the stage eigensolve: training kernels and the
// network API.
//
// A network (learned_dev.h) is built for one rank r (<= 16).  Training
// samples are recorded by the RK stage kernel (features of the stage and the
// overlap T = u* u_next of its input basis with its output eigenvectors);
// training minimises the mean over a batch of sum_a (1 - |(R* T)_aa|^2) with
// Adam.  Forward: four layer products (tiled FP32 GEMM on MFMA with the bias
// and SiLU fused); per-sample Cayley map, loss and its gradient with respect to the
// network outputs (one wave per sample, FP64); backward: the layer products
// transposed, with SiLU' fused, and column sums for the biases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_common.h"
#include "learned_dev.h"

struct lrei_net {
  int device = 0, r = 0;
  long long np = 0;
  hipStream_t stream = nullptr;
  lrei::DevBuf params, grads, m1, m2;
  // batch buffers
  int cap = 0;
  lrei::DevBuf X, T, Z[3], H[3], O, gO, gH, gZ, loss, perm;
  long long adam_t = 0;
  std::string err;
  lrei_status fail(lrei_status s, const std::string &m) {
    err = m;
    return s;
  }
};

namespace lrei {
namespace {

constexpr int kGemmT = 64, kGemmK = 16;

typedef float f4_t __attribute__((ext_vector_type(4)));

// C[M x N] = op(A)[M x K] op(B)[K x N]; op(A)(m, k) = ta ? A[k lda + m] : A[m lda + k],
// op(B)(k, n) = tb ? B[n ldb + k] : B[k ldb + n].  Epilogue ep: 0 store; 1 add
// bias[n], store Z = C and H = silu(C); 2 multiply by silu'(Zp[m ldc + n]).
// A workgroup of four waves forms a 64 x 64 tile of C: K is walked in chunks
// of 16 staged in LDS (transposed operands are gathered there), and each wave
// accumulates a 32 x 32 quarter as 2 x 2 FP32 16 x 16 x 4 MFMA tiles.  Operand
// lanes: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k; the result
// D[4 g + v][j] sits in lane j + 16 g, register v.
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *__restrict__ A, int lda, int ta,
                                              const float *__restrict__ B, int ldb, int tb, float *__restrict__ C,
                                              int ldc, int ep, const float *__restrict__ bias, float *__restrict__ H,
                                              const float *__restrict__ Zp) {
  __shared__ float As[kGemmK][kGemmT + 4], Bs[kGemmK][kGemmT + 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;  // the wave's quarter of the tile
  const int m0 = blockIdx.y * kGemmT, n0 = blockIdx.x * kGemmT;
  f4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += kGemmK) {
    for (int e = threadIdx.x; e < kGemmK * kGemmT; e += 256) {
      // consecutive threads walk the operand's contiguous index (k for A
      // stored by rows of op(A), m for a transposed A; likewise for B)
      const int kk = ta ? e / kGemmT : e % kGemmK, mm = ta ? e % kGemmT : e / kGemmK;
      const int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < M && gk < K) ? (ta ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk]) : 0.0f;
      const int kb = tb ? e % kGemmK : e / kGemmT, nn = tb ? e / kGemmK : e % kGemmT;
      const int gn = n0 + nn, gkb = k0 + kb;
      Bs[kb][nn] = (gn < N && gkb < K) ? (tb ? B[(long long)gn * ldb + gkb] : B[(long long)gkb * ldb + gn]) : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmK; kk += 4) {
      float a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[kk + lk][wm + 16 * t + li];
        b[t] = Bs[kk + lk][wn + 16 * t + li];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm + 16 * ti + 4 * lk + v, gn = n0 + wn + 16 * tj + li;
        if (gm >= M || gn >= N) continue;
        const long long q = (long long)gm * ldc + gn;
        float val = acc[ti][tj][v];
        if (ep == 1) {
          val += bias[gn];
          C[q] = val;
          H[q] = silu_f(val);
        } else if (ep == 2) {
          const float z = Zp[q];
          const float sg = 1.0f / (1.0f + __expf(-z));
          C[q] = val * sg * (1.0f + z * (1.0f - sg));
        } else {
          C[q] = val;
        }
      }
}

void gemm(int M, int N, int K, const float *A, int lda, int ta, const float *B, int ldb, int tb, float *C, int ldc,
          int ep, const float *bias, float *H, const float *Zp, hipStream_t s) {
  dim3 grid((N + kGemmT - 1) / kGemmT, (M + kGemmT - 1) / kGemmT);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, M, N, K, A, lda, ta, B, ldb, tb, C, ldc, ep, bias, H, Zp);
}

// X, T of a batch: samples perm[b0 .. b0 + B)
__global__ void k_gather(const float *__restrict__ samples, const int *__restrict__ perm, int b0, int B, int r,
                         float *__restrict__ X, float *__restrict__ T) {
  const int nin = net_in(r), nt = 2 * r * r, sf = net_sample_floats(r);
  const long long total = (long long)B * sf;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e / sf), c = (int)(e % sf);
    const float v = samples[(long long)perm[b0 + b] * sf + c];
    if (c < nin)
      X[(long long)b * nin + c] = v;
    else
      T[(long long)b * nt + (c - nin)] = v;
  }
}

// One wave per sample: R = Cayley(A(o)), loss_b = sum_a (1 - |(R* T)_aa|^2),
// gO_b = d(loss_b / B)/d o (through gA = M^{-H} gR (I + R)^H / 2,
// gR = -2 T diag(conj s), s_a = (R* T)_aa).  Rout (optional): R as FP64 pairs.
__global__ __launch_bounds__(64) void k_cayley_loss(const float *__restrict__ O, const float *__restrict__ X,
                                                    const float *__restrict__ T, int B, int r,
                                                    float *__restrict__ gO, double *__restrict__ loss,
                                                    double *__restrict__ Rout) {
  __shared__ double2 aug[kNetMaxR * 2 * kNetMaxR], R[kNetMaxR * kNetMaxR], Mi[kNetMaxR * kNetMaxR];
  __shared__ double2 Tm[kNetMaxR * kNetMaxR], S[kNetMaxR], gA[kNetMaxR * kNetMaxR], Q[kNetMaxR * kNetMaxR];
  __shared__ float o[kNetMaxR * kNetMaxR];
  const int b = blockIdx.x, lane = threadIdx.x, rr = r * r;
  if (b >= B) return;
  const float *x = X + (long long)b * net_in(r);
  for (int e = lane; e < rr; e += 64) o[e] = O[(long long)b * rr + e] + analytic_param(x, r, e);
  __builtin_amdgcn_wave_barrier();
  cayley_wave(o, r, aug, R, Mi);
  if (Rout)
    for (int e = lane; e < rr; e += 64) {
      Rout[((long long)b * rr + e) * 2] = R[e].x;
      Rout[((long long)b * rr + e) * 2 + 1] = R[e].y;
    }
  if (!T) return;
  for (int e = lane; e < rr; e += 64)
    Tm[e] = make_double2(T[((long long)b * rr + e) * 2], T[((long long)b * rr + e) * 2 + 1]);
  __builtin_amdgcn_wave_barrier();
  // s_a = sum_c conj(R_ca) T_ca
  if (lane < r) {
    double2 s = make_double2(0, 0);
    for (int c = 0; c < r; ++c) {
      const double2 x = R[c * r + lane], t = Tm[c * r + lane];
      s.x += x.x * t.x + x.y * t.y;
      s.y += x.x * t.y - x.y * t.x;
    }
    S[lane] = s;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) {
    double l = 0;
    for (int a = 0; a < r; ++a) l += 1.0 - (S[a].x * S[a].x + S[a].y * S[a].y);
    loss[b] = l;
  }
  // Q = gR (I + R)^H, gR_ca = -2 T_ca conj(s_a)
  for (int e = lane; e < rr; e += 64) {
    const int c = e / r, d = e % r;
    double2 q = make_double2(0, 0);
    for (int a = 0; a < r; ++a) {
      const double2 t = Tm[c * r + a], s = S[a];
      const double2 g = make_double2(-2.0 * (t.x * s.x + t.y * s.y), -2.0 * (t.y * s.x - t.x * s.y));
      // (I + R)^H [a][d] = conj((I + R)[d][a])
      double2 ir = R[d * r + a];
      if (d == a) ir.x += 1.0;
      q.x += g.x * ir.x + g.y * ir.y;
      q.y += g.y * ir.x - g.x * ir.y;
    }
    Q[e] = q;
  }
  __builtin_amdgcn_wave_barrier();
  // gA = M^{-H} Q / 2
  for (int e = lane; e < rr; e += 64) {
    const int i = e / r, d = e % r;
    double2 g = make_double2(0, 0);
    for (int c = 0; c < r; ++c) {
      const double2 mi = Mi[c * r + i], q = Q[c * r + d];  // conj(Minv[c][i])
      g.x += mi.x * q.x + mi.y * q.y;
      g.y += mi.x * q.y - mi.y * q.x;
    }
    gA[e] = make_double2(0.5 * g.x, 0.5 * g.y);
  }
  __builtin_amdgcn_wave_barrier();
  // gradient with respect to the r^2 reals, divided by the batch size
  const double sc = 1.0 / B;
  float *g = gO + (long long)b * rr;
  for (int a = lane; a < r; a += 64) g[a] = (float)(sc * gA[a * r + a].y);
  for (int e = lane; e < r * (r - 1) / 2; e += 64) {
    int a = 0, rem = e;
    while (rem >= r - a - 1) {
      rem -= r - a - 1;
      ++a;
    }
    const int bb = a + 1 + rem;
    const double2 x = gA[a * r + bb], y = gA[bb * r + a];
    const double qx = x.x - y.x, qy = -x.y - y.y;  // q = conj(gA_ab) - gA_ba
    g[r + 2 * e] = (float)(sc * qx);
    g[r + 2 * e + 1] = (float)(-sc * qy);
  }
}

// O[b][e] += bias[e] (output layer)
__global__ void k_add_bias(float *__restrict__ O, const float *__restrict__ bias, int B, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < B * n) O[e] += bias[e % n];
}

// out[n] = sum_m G[m ldg + n]
__global__ void k_colsum(const float *__restrict__ G, int M, int N, int ldg, float *__restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0;
  for (int m = 0; m < M; ++m) s += G[(long long)m * ldg + n];
  out[n] = s;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi, v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  }
}

struct Layers {
  const float *W[4], *b[4];
  float *gW[4], *gb[4];
  int K[4], N[4];
};

Layers layers(lrei_net *m) {
  Layers L{};
  const int r = m->r, W = kNetWidth;
  long long off = 0;
  for (int l = 0; l < 4; ++l) {
    L.K[l] = l == 0 ? net_in(r) : W;
    L.N[l] = l == 3 ? r * r : W;
    L.W[l] = (const float *)m->params.p + off;
    L.gW[l] = (float *)m->grads.p + off;
    off += (long long)L.K[l] * L.N[l];
    L.b[l] = (const float *)m->params.p + off;
    L.gb[l] = (float *)m->grads.p + off;
    off += L.N[l];
  }
  return L;
}

bool ensure_batch(lrei_net *m, int B) {
  if (B <= m->cap) return true;
  const int r = m->r, W = kNetWidth;
  bool ok = m->X.ensure((size_t)B * net_in(r) * 4) && m->T.ensure((size_t)B * 2 * r * r * 4) &&
            m->O.ensure((size_t)B * r * r * 4) && m->gO.ensure((size_t)B * r * r * 4) &&
            m->gH.ensure((size_t)B * W * 4) && m->gZ.ensure((size_t)B * W * 4) && m->loss.ensure((size_t)B * 8);
  for (int l = 0; l < 3; ++l) ok = ok && m->Z[l].ensure((size_t)B * W * 4) && m->H[l].ensure((size_t)B * W * 4);
  if (ok) m->cap = B;
  return ok;
}

// forward + loss + backward of the batch already gathered into X, T
void batch_pass(lrei_net *m, int B, bool backward, double *Rout) {
  const int r = m->r, W = kNetWidth, rr = r * r;
  const Layers L = layers(m);
  hipStream_t s = m->stream;
  const float *in = (const float *)m->X.p;
  int ldin = net_in(r);
  for (int l = 0; l < 3; ++l) {
    gemm(B, W, L.K[l], in, ldin, 0, L.W[l], W, 0, (float *)m->Z[l].p, W, 1, L.b[l], (float *)m->H[l].p, nullptr, s);
    in = (const float *)m->H[l].p;
    ldin = W;
  }
  gemm(B, rr, W, in, W, 0, L.W[3], rr, 0, (float *)m->O.p, rr, 0, nullptr, nullptr, nullptr, s);
  hipLaunchKernelGGL(k_add_bias, dim3((B * rr + 255) / 256), dim3(256), 0, s, (float *)m->O.p, L.b[3], B, rr);
  hipLaunchKernelGGL(k_cayley_loss, dim3(B), dim3(64), 0, s, (const float *)m->O.p, (const float *)m->X.p,
                     Rout ? (const float *)nullptr : (const float *)m->T.p, B, r, (float *)m->gO.p,
                     (double *)m->loss.p, Rout);
  if (!backward) return;
  // output layer
  gemm(W, rr, B, (const float *)m->H[2].p, W, 1, (const float *)m->gO.p, rr, 0, L.gW[3], rr, 0, nullptr, nullptr,
       nullptr, s);
  hipLaunchKernelGGL(k_colsum, dim3((rr + 255) / 256), dim3(256), 0, s, (const float *)m->gO.p, B, rr, rr, L.gb[3]);
  const float *g = (const float *)m->gO.p;
  int ldg = rr, Ng = rr;
  for (int l = 2; l >= 0; --l) {
    // gZ_l = (g W_{l+1}^T) o silu'(Z_l)
    gemm(B, W, Ng, g, ldg, 0, L.W[l + 1], Ng, 1, (float *)m->gZ.p, W, 2, nullptr, nullptr, (const float *)m->Z[l].p,
         s);
    const float *hin = l == 0 ? (const float *)m->X.p : (const float *)m->H[l - 1].p;
    const int ldh = l == 0 ? net_in(r) : W;
    gemm(L.K[l], W, B, hin, ldh, 1, (const float *)m->gZ.p, W, 0, L.gW[l], W, 0, nullptr, nullptr, nullptr, s);
    hipLaunchKernelGGL(k_colsum, dim3((W + 255) / 256), dim3(256), 0, s, (const float *)m->gZ.p, B, W, W, L.gb[l]);
    // the next layer down reads gZ through gH (gZ is overwritten)
    (void)hipMemcpyAsync(m->gH.p, m->gZ.p, (size_t)B * W * 4, hipMemcpyDeviceToDevice, s);
    g = (const float *)m->gH.p;
    ldg = W;
    Ng = W;
  }
}

uint64_t splitmix64(uint64_t &x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double unit(uint64_t &x) { return (double)(splitmix64(x) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace
}  // namespace lrei

using namespace lrei;

extern "C" {

long long lrei_net_param_count(int r) { return (r >= 1 && r <= kNetMaxR) ? net_param_count(r) : -1; }

lrei_status lrei_net_create(lrei_net **out, int hip_device, int r, const float *init, uint64_t seed) {
  if (!out) return LREI_E_INVALID;
  *out = nullptr;
  if (r < 1 || r > kNetMaxR) return LREI_E_INVALID;
  if (hipSetDevice(hip_device) != hipSuccess) return LREI_E_DEVICE;
  auto *m = new lrei_net;
  m->device = hip_device;
  m->r = r;
  m->np = net_param_count(r);
  if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) {
    delete m;
    return LREI_E_DEVICE;
  }
  const size_t bytes = (size_t)m->np * 4;
  if (!m->params.ensure(bytes) || !m->grads.ensure(bytes) || !m->m1.ensure(bytes) || !m->m2.ensure(bytes)) {
    lrei_net_destroy(m);
    return LREI_E_NOMEM;
  }
  std::vector<float> p((size_t)m->np);
  if (init) {
    std::memcpy(p.data(), init, bytes);
  } else {
    // hidden layers: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights; output
    // layer zero (the untrained network gives the analytic rotation); zero biases
    uint64_t st = seed;
    long long off = 0;
    for (int l = 0; l < 4; ++l) {
      const int K = l == 0 ? net_in(r) : kNetWidth, N = l == 3 ? r * r : kNetWidth;
      const double a = (l == 3 ? 0.0 : 1.0) / std::sqrt((double)K);
      for (long long i = 0; i < (long long)K * N; ++i) p[off + i] = (float)((2.0 * unit(st) - 1.0) * a);
      off += (long long)K * N;
      for (int i = 0; i < N; ++i) p[off + i] = 0.0f;
      off += N;
    }
  }
  if (hipMemcpy(m->params.p, p.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->m1.p, 0, bytes) != hipSuccess || hipMemset(m->m2.p, 0, bytes) != hipSuccess) {
    lrei_net_destroy(m);
    return LREI_E_DEVICE;
  }
  *out = m;
  return LREI_OK;
}

void lrei_net_destroy(lrei_net *m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  for (DevBuf *b : {&m->params, &m->grads, &m->m1, &m->m2, &m->X, &m->T, &m->O, &m->gO, &m->gH, &m->gZ, &m->loss,
                    &m->perm})
    b->release();
  for (int l = 0; l < 3; ++l) {
    m->Z[l].release();
    m->H[l].release();
  }
  if (m->stream) (void)hipStreamDestroy(m->stream);
  delete m;
}

const char *lrei_net_last_error(const lrei_net *m) { return m ? m->err.c_str() : "null network"; }

int lrei_net_rank(const lrei_net *m) { return m ? m->r : -1; }

const void *lrei_net_device_params(const lrei_net *m) { return m ? m->params.p : nullptr; }

lrei_status lrei_net_get_params(lrei_net *m, float *host) {
  if (!m || !host) return LREI_E_INVALID;
  (void)hipSetDevice(m->device);
  if (hipStreamSynchronize(m->stream) != hipSuccess ||
      hipMemcpy(host, m->params.p, (size_t)m->np * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return m->fail(LREI_E_DEVICE, "copy of the parameters failed");
  return LREI_OK;
}

lrei_status lrei_net_set_params(lrei_net *m, const float *host) {
  if (!m || !host) return LREI_E_INVALID;
  (void)hipSetDevice(m->device);
  if (hipStreamSynchronize(m->stream) != hipSuccess ||
      hipMemcpy(m->params.p, host, (size_t)m->np * 4, hipMemcpyHostToDevice) != hipSuccess)
    return m->fail(LREI_E_DEVICE, "copy of the parameters failed");
  m->adam_t = 0;
  (void)hipMemset(m->m1.p, 0, (size_t)m->np * 4);
  (void)hipMemset(m->m2.p, 0, (size_t)m->np * 4);
  return LREI_OK;
}

// Loss (mean over the n samples) and, if grad_host, its gradient; one batch.
lrei_status lrei_net_loss_grad(lrei_net *m, const float *samples, int n, double *loss_out, float *grad_host) {
  if (!m || !samples || n < 1 || n > (1 << 16)) return LREI_E_INVALID;
  (void)hipSetDevice(m->device);
  if (!ensure_batch(m, n) || !m->perm.ensure((size_t)n * 4)) return m->fail(LREI_E_NOMEM, "device allocation failed");
  std::vector<int> id(n);
  for (int i = 0; i < n; ++i) id[i] = i;
  hipStream_t s = m->stream;
  (void)hipMemcpyAsync(m->perm.p, id.data(), (size_t)n * 4, hipMemcpyHostToDevice, s);
  hipLaunchKernelGGL(k_gather, dim3(256), dim3(256), 0, s, samples, (const int *)m->perm.p, 0, n, m->r,
                     (float *)m->X.p, (float *)m->T.p);
  batch_pass(m, n, grad_host != nullptr, nullptr);
  std::vector<double> l(n);
  hipError_t e = hipMemcpyAsync(l.data(), m->loss.p, (size_t)n * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && grad_host) e = hipMemcpyAsync(grad_host, m->grads.p, (size_t)m->np * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return m->fail(LREI_E_DEVICE, std::string("network pass: ") + hipGetErrorString(e));
  double t = 0;
  for (double v : l) t += v;
  if (loss_out) *loss_out = t / n;
  return LREI_OK;
}

// Rotations R (n x r x r complex, FP64 (re, im) pairs) the network gives for
// the features of n samples.
lrei_status lrei_net_rotations(lrei_net *m, const float *samples, int n, double *R_host) {
  if (!m || !samples || !R_host || n < 1 || n > (1 << 16)) return LREI_E_INVALID;
  (void)hipSetDevice(m->device);
  const size_t rb = (size_t)n * m->r * m->r * 16;
  DevBuf Rd;
  if (!ensure_batch(m, n) || !m->perm.ensure((size_t)n * 4) || !Rd.ensure(rb))
    return m->fail(LREI_E_NOMEM, "device allocation failed");
  std::vector<int> id(n);
  for (int i = 0; i < n; ++i) id[i] = i;
  hipStream_t s = m->stream;
  (void)hipMemcpyAsync(m->perm.p, id.data(), (size_t)n * 4, hipMemcpyHostToDevice, s);
  hipLaunchKernelGGL(k_gather, dim3(256), dim3(256), 0, s, samples, (const int *)m->perm.p, 0, n, m->r,
                     (float *)m->X.p, (float *)m->T.p);
  batch_pass(m, n, false, (double *)Rd.p);
  hipError_t e = hipMemcpyAsync(R_host, Rd.p, rb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  Rd.release();
  if (e != hipSuccess) return m->fail(LREI_E_DEVICE, std::string("network rotations: ") + hipGetErrorString(e));
  return LREI_OK;
}

// Adam over `epochs` passes of the n samples in batches of `batch`, shuffled
// per epoch (splitmix64 Fisher-Yates from shuffle_seed); epoch_loss[e] = the
// mean training loss of epoch e (before each batch's update).
lrei_status lrei_net_train(lrei_net *m, const float *samples, int n, int batch, int epochs, float lr,
                             uint64_t shuffle_seed, double *epoch_loss) {
  if (!m || !samples || n < 1 || batch < 1 || batch > 4096 || epochs < 0 || !(lr > 0)) return LREI_E_INVALID;
  (void)hipSetDevice(m->device);
  const int B = std::min(batch, n);
  if (!ensure_batch(m, B) || !m->perm.ensure((size_t)n * 4)) return m->fail(LREI_E_NOMEM, "device allocation failed");
  hipStream_t s = m->stream;
  std::vector<int> perm(n);
  std::vector<double> l(B);
  uint64_t st = shuffle_seed;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int i = n - 1; i > 0; --i) std::swap(perm[i], perm[splitmix64(st) % (uint64_t)(i + 1)]);
    if (hipMemcpyAsync(m->perm.p, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s) != hipSuccess)
      return m->fail(LREI_E_DEVICE, "upload of the sample order failed");
    double tot = 0;
    int cnt = 0;
    for (int b0 = 0; b0 + B <= n; b0 += B) {
      hipLaunchKernelGGL(k_gather, dim3(256), dim3(256), 0, s, samples, (const int *)m->perm.p, b0, B, m->r,
                         (float *)m->X.p, (float *)m->T.p);
      batch_pass(m, B, true, nullptr);
      ++m->adam_t;
      const float c1 = 1.0f - std::pow(b1, (float)m->adam_t), c2 = 1.0f - std::pow(b2, (float)m->adam_t);
      hipLaunchKernelGGL(k_adam, dim3(512), dim3(256), 0, s, (float *)m->params.p, (const float *)m->grads.p,
                         (float *)m->m1.p, (float *)m->m2.p, m->np, lr, b1, b2, eps, c1, c2);
      if (epoch_loss) {
        if (hipMemcpyAsync(l.data(), m->loss.p, (size_t)B * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return m->fail(LREI_E_DEVICE, "loss read-back failed");
        for (double v : l) tot += v;
        cnt += B;
      }
    }
    if (epoch_loss) epoch_loss[ep] = cnt ? tot / cnt : 0.0;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return m->fail(LREI_E_DEVICE, std::string("training: ") + hipGetErrorString(e));
  return LREI_OK;
}

}  // extern "C"
