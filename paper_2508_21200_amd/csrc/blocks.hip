// Generic N-space block pass: outputs that are linear combinations of input
// blocks, and Gram products among inputs and outputs, in one read of the
// inputs.  It carries the orthonormal history basis of the multistep (AB)
// schemes: the Gram products of history and new blocks, the block classical
// Gram-Schmidt step Y = X - U c, and the rotation U_new = [U, Y] T that keeps
// the history basis orthonormal.
//
// Precision: block storage is T (complex FP32 or FP64); every product runs on
// 16x16x4 FP64 MFMA with T values widened exactly to FP64, so the Gram
// products of FP32 blocks are exact products accumulated in FP64, and the
// combination outputs are formed in FP64 before they are rounded to T.  The
// Gram-Schmidt difference X - U c is therefore accurate relative to its own
// (possibly small) size, which the history basis relies on.
//
// Layout: as everywhere, N x r blocks are row-major complex (re, im
// interleaved).  r <= 16 here (one 16x16 MFMA tile per block pair).
#include <hip/hip_runtime.h>

#include "lrei_internal.h"

namespace lrei {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kBT = 512;         // threads per workgroup
constexpr int kBW = kBT / 64;    // waves
constexpr int kBR = 16;          // rows per tile
constexpr int kBP = 16;          // padded columns (r <= 16)
constexpr int kPlane = kBR * kBP;

template <typename T> struct Cx;
template <> struct Cx<double> { using type = double2; };
template <> struct Cx<float> { using type = float2; };

__device__ inline d4v mfma64(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Workgroup w runs on XCD w % 8; each XCD walks a contiguous eighth of the tiles.
__device__ inline long long btile(long long k, long long num_tiles, int grid) {
  const int w = blockIdx.x;
  if ((grid & 7) == 0 && (num_tiles & 7) == 0 && num_tiles >= grid) {
    const long long per = num_tiles >> 3;
    const long long t = (long long)(w >> 3) + k * (grid >> 3);
    return t < per ? (long long)(w & 7) * per + t : -1;
  }
  const long long t = (long long)w + k * grid;
  return t < num_tiles ? t : -1;
}

// MI: Gram work items per wave (items = n_gram <= MI * kBW).
template <typename T, int MI>
__global__ __launch_bounds__(kBT) void k_blocks(BlocksArgs a) {
  using C2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  T *planes = reinterpret_cast<T *>(smem);  // block q: re at 2q*kPlane, im at (2q+1)*kPlane
  const int r = a.r, nin = a.n_in, nout = a.n_out, nb = nin + nout;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 2 * nb * kPlane; i += kBT) planes[i] = T(0);
  __syncthreads();

  double acc[MI][8];
#pragma unroll
  for (int q = 0; q < MI; ++q)
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[q][v] = 0.0;

  const long long N = a.N;
  const long long num_tiles = (N + kBR - 1) / kBR;
  for (long long k = 0;; ++k) {
    const long long tile = btile(k, num_tiles, a.grid);
    if (tile < 0) break;
    const long long row0 = tile * kBR;
    // 1. input tiles -> LDS (coalesced: consecutive threads take consecutive columns of a row)
    for (int e = threadIdx.x; e < nin * kBR * r; e += kBT) {
      const int q = e / (kBR * r), rem = e % (kBR * r), lr = rem / r, c = rem % r;
      const long long x = row0 + lr;
      C2 v;
      v.x = 0; v.y = 0;
      if (x < N) v = reinterpret_cast<const C2 *>(a.in[q])[x * r + c];
      planes[(2 * q) * kPlane + lr * kBP + c] = v.x;
      planes[(2 * q + 1) * kPlane + lr * kBP + c] = v.y;
    }
    __syncthreads();
    // 2. outputs: out_o = sum_i in_i C[i, o]; one 16x16 tile per (wave, output)
    for (int o = wave; o < nout; o += kBW) {
      d4v ore = {0, 0, 0, 0}, oim = {0, 0, 0, 0};
      const int j = lane & 15;
      for (int i = 0; i < nin; ++i) {
        const T *xr = planes + (2 * i) * kPlane, *xi = planes + (2 * i + 1) * kPlane;
        for (int kk = 0; kk < kBP; kk += 4) {
          const int ak = kk + (lane >> 4);
          const double ar = (double)xr[(lane & 15) * kBP + ak], ai = (double)xi[(lane & 15) * kBP + ak];
          double2 c = make_double2(0, 0);
          if (ak < r && j < r) c = a.C[(size_t)(i * r + ak) * a.ldc + o * r + j];
          ore = mfma64(ar, c.x, ore);
          ore = mfma64(-ai, c.y, ore);
          oim = mfma64(ar, c.y, oim);
          oim = mfma64(ai, c.x, oim);
        }
      }
      T *yr = planes + (2 * (nin + o)) * kPlane, *yi = planes + (2 * (nin + o) + 1) * kPlane;
      C2 *out = reinterpret_cast<C2 *>(a.out[o]);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * v + (lane >> 4);  // f64 MFMA result row
        const long long x = row0 + i;
        if (j < r) {
          C2 w;
          w.x = (T)ore[v];
          w.y = (T)oim[v];
          yr[i * kBP + j] = w.x;  // the rounded value, as stored
          yi[i * kBP + j] = w.y;
          if (x < N) out[x * r + j] = w;
        }
      }
    }
    if (nout > 0) __syncthreads();
    // 3. Gram products G_g += X_a^H X_b over the tile's rows
#pragma unroll
    for (int q = 0; q < MI; ++q) {
      const int g = wave + kBW * q;
      if (g >= a.n_gram) break;
      const int ba = a.ga[g], bb = a.gb[g];
      const T *xr = planes + (2 * ba) * kPlane, *xi = planes + (2 * ba + 1) * kPlane;
      const T *yr = planes + (2 * bb) * kPlane, *yi = planes + (2 * bb + 1) * kPlane;
      d4v cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
      for (int kk = 0; kk < kBR; kk += 4) {
        const int row = kk + (lane >> 4), col = lane & 15;
        const double ar = (double)xr[row * kBP + col], ai = (double)xi[row * kBP + col];
        const double br = (double)yr[row * kBP + col], bi = (double)yi[row * kBP + col];
        cre = mfma64(ar, br, cre);
        cre = mfma64(ai, bi, cre);
        cim = mfma64(ar, bi, cim);
        cim = mfma64(-ai, br, cim);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[q][v] += cre[v];
        acc[q][4 + v] += cim[v];
      }
    }
    __syncthreads();
  }
  // 4. per-workgroup partials, entry-major: partials[e * grid + wg], e = (g * r + a) * r + b
#pragma unroll
  for (int q = 0; q < MI; ++q) {
    const int g = wave + kBW * q;
    if (g >= a.n_gram) break;
    const int b = lane & 15;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ar = 4 * v + (lane >> 4);
      if (ar < r && b < r) {
        const long long e = ((long long)g * r + ar) * r + b;
        a.partials[e * a.grid + blockIdx.x] = make_double2(acc[q][v], acc[q][4 + v]);
      }
    }
  }
}

}  // namespace

int blocks_grid(long long N) {
  const long long tiles = (N + kBR - 1) / kBR;
  long long g = tiles < 512 ? tiles : 512;
  if (g >= 8) g &= ~7LL;
  return (int)(g < 1 ? 1 : g);
}

size_t blocks_lds(bool fp32, int n_blocks) { return (size_t)2 * n_blocks * kPlane * (fp32 ? 4 : 8); }

bool launch_blocks(bool fp32, const BlocksArgs &a, hipStream_t s) {
  if (a.r < 1 || a.r > kBP || a.n_in < 0 || a.n_in > kMaxIoBlocks || a.n_out < 0 || a.n_out > kMaxIoBlocks ||
      a.n_gram < 0 || a.n_gram > kMaxGrams || a.grid < 1)
    return false;
  const size_t lds = blocks_lds(fp32, a.n_in + a.n_out);
  static bool attr = false;
  if (!attr) {
    const int cap = 160 * 1024;
    (void)hipFuncSetAttribute((const void *)k_blocks<float, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void *)k_blocks<float, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void *)k_blocks<double, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void *)k_blocks<double, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    attr = true;
  }
  if (lds > 160 * 1024) return false;
  const bool few = a.n_gram <= kBW;
  if (fp32) {
    if (few) hipLaunchKernelGGL((k_blocks<float, 1>), dim3(a.grid), dim3(kBT), lds, s, a);
    else hipLaunchKernelGGL((k_blocks<float, 4>), dim3(a.grid), dim3(kBT), lds, s, a);
  } else {
    if (few) hipLaunchKernelGGL((k_blocks<double, 1>), dim3(a.grid), dim3(kBT), lds, s, a);
    else hipLaunchKernelGGL((k_blocks<double, 4>), dim3(a.grid), dim3(kBT), lds, s, a);
  }
  return true;
}

}  // namespace lrei
