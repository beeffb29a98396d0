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

// The combination coefficients C (n_in r x n_out r) are the same for every
// tile: they are staged once per workgroup in LDS after the tile planes when
// the two fit in kBlocksLdsCap bytes (else every tile reads them from memory).
constexpr size_t kBlocksLdsCap = 64 * 1024;
__host__ __device__ inline size_t blocks_planes_bytes(bool fp32, int nb) { return (size_t)2 * nb * kPlane * (fp32 ? 4 : 8); }
__host__ __device__ inline bool blocks_c_in_lds(bool fp32, int nin, int nout, int r) {
  return blocks_planes_bytes(fp32, nin + nout) + (size_t)nin * nout * r * r * 16 <= kBlocksLdsCap;
}

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
  const bool c_lds = blocks_c_in_lds(sizeof(T) == 4, nin, nout, r);
  const int ldc = c_lds ? nout * r : a.ldc;
  double2 *Cs = reinterpret_cast<double2 *>(smem + blocks_planes_bytes(sizeof(T) == 4, nb));
  if (c_lds)
    for (int e = threadIdx.x; e < nin * r * nout * r; e += kBT) Cs[e] = a.C[(size_t)(e / (nout * r)) * a.ldc + e % (nout * r)];
  const double2 *Cm = c_lds ? Cs : a.C;
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
        double2 c[kBP / 4];
#pragma unroll
        for (int q = 0; q < kBP / 4; ++q) {  // the four coefficient loads together
          const int ak = 4 * q + (lane >> 4);
          c[q] = (ak < r && j < r) ? Cm[(size_t)(i * r + ak) * ldc + o * r + j] : make_double2(0, 0);
        }
#pragma unroll
        for (int q = 0; q < kBP / 4; ++q) {
          const int ak = 4 * q + (lane >> 4);
          const double ar = (double)xr[(lane & 15) * kBP + ak], ai = (double)xi[(lane & 15) * kBP + ak];
          ore = mfma64(ar, c[q].x, ore);
          ore = mfma64(-ai, c[q].y, ore);
          oim = mfma64(ar, c[q].y, oim);
          oim = mfma64(ai, c[q].x, oim);
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

// The same pass for small r on FP64 vector FMAs: with 16 x 16 MFMA tiles an
// r-column block uses (r/16)^2 of each product, and on this chip the FP64
// matrix rate is no higher than the vector rate, so up to r = 8 exact-size
// vector products are faster.  Tiles of kSR = 64 rows with the blocks packed
// at their own width r in LDS (block q: re at 2q kSR r, im at (2q + 1) kSR r,
// row-major), the coefficients in LDS when planes and coefficients fit in
// kSmallLdsCap bytes, the same partials layout; thread t accumulates Gram
// entries t, t + kBT, ... in registers.
constexpr int kSR = 64;
constexpr size_t kSmallLdsCap = 96 * 1024;
constexpr int kSmallEntries = (kMaxGrams * 8 * 8 + kBT - 1) / kBT;  // r <= 8
__host__ __device__ inline size_t small_planes_bytes(bool fp32, int nb, int r) {
  return (size_t)2 * nb * kSR * r * (fp32 ? 4 : 8);
}
__host__ __device__ inline bool small_c_in_lds(bool fp32, int nin, int nout, int r) {
  return small_planes_bytes(fp32, nin + nout, r) + (size_t)nin * nout * r * r * 16 <= kSmallLdsCap;
}

// R: the block width r, a compile-time constant so that every index folds and
// the inner products unroll; each thread's output and Gram entries are the
// same in every tile, so their coordinates are computed once.
constexpr int kOutPerThread = (kMaxIoBlocks * kSR * 8 + kBT - 1) / kBT;
template <typename T, int R>
__global__ __launch_bounds__(kBT) void k_blocks_small(BlocksArgs a) {
  using C2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  T *planes = reinterpret_cast<T *>(smem);
  constexpr int rr = R * R, pl = kSR * R;
  const int nin = a.n_in, nout = a.n_out, nb = nin + nout;
  const bool c_lds = small_c_in_lds(sizeof(T) == 4, nin, nout, R);
  const int ldc = c_lds ? nout * R : a.ldc;
  double2 *Cs = reinterpret_cast<double2 *>(smem + small_planes_bytes(sizeof(T) == 4, nb, R));
  if (c_lds)
    for (int e = threadIdx.x; e < nin * R * nout * R; e += kBT) Cs[e] = a.C[(size_t)(e / (nout * R)) * a.ldc + e % (nout * R)];
  const double2 *Cm = c_lds ? Cs : a.C;
  const int n_ent = a.n_gram * rr;
  double accr[kSmallEntries], acci[kSmallEntries];
  int gx[kSmallEntries], gy[kSmallEntries];  // plane offsets of the entry's two columns
#pragma unroll
  for (int m = 0; m < kSmallEntries; ++m) {
    accr[m] = acci[m] = 0.0;
    const int e = threadIdx.x + m * kBT;
    const int g = e < n_ent ? e / rr : 0, i = (e % rr) / R, j = e % R;
    gx[m] = 2 * a.ga[g] * pl + i;
    gy[m] = 2 * a.gb[g] * pl + j;
  }
  const int n_out_ent = nout * pl;
  const long long N = a.N;
  const long long num_tiles = (N + kSR - 1) / kSR;
  for (long long k = 0;; ++k) {
    const long long tile = btile(k, num_tiles, a.grid);
    if (tile < 0) break;
    const long long row0 = tile * kSR;
    const bool full = row0 + kSR <= N;
    // one tile of every input: kSR R consecutive complex values per block
    for (int e = threadIdx.x; e < nin * pl; e += kBT) {
      const int q = e / pl, rem = e - q * pl;
      C2 v;
      v.x = 0;
      v.y = 0;
      if (full || row0 + rem / R < N) v = reinterpret_cast<const C2 *>(a.in[q])[row0 * R + rem];
      planes[(2 * q) * pl + rem] = v.x;
      planes[(2 * q + 1) * pl + rem] = v.y;
    }
    __syncthreads();
    // outputs: out_o[row][c] = sum_{i, k} in_i[row][k] C[i R + k][o R + c]
#pragma unroll
    for (int m = 0; m < kOutPerThread; ++m) {
      const int e = threadIdx.x + m * kBT;
      if (e >= n_out_ent) break;
      const int o = e / pl, rem = e - o * pl, lr = rem / R, c = rem - lr * R;
      double sr = 0, si = 0;
      for (int i = 0; i < nin; ++i) {
        const T *xr = planes + (2 * i) * pl + lr * R, *xi = xr + pl;
        const double2 *cf = Cm + (size_t)(i * R) * ldc + o * R + c;
#pragma unroll
        for (int kk = 0; kk < R; ++kk) {
          const double2 w = cf[kk * ldc];
          const double ar = (double)xr[kk], ai = (double)xi[kk];
          sr += ar * w.x - ai * w.y;
          si += ar * w.y + ai * w.x;
        }
      }
      C2 w;
      w.x = (T)sr;
      w.y = (T)si;
      planes[(2 * (nin + o)) * pl + rem] = w.x;  // the rounded value, as stored
      planes[(2 * (nin + o) + 1) * pl + rem] = w.y;
      if (full || row0 + lr < N) reinterpret_cast<C2 *>(a.out[o])[row0 * R + rem] = w;
    }
    if (nout > 0) __syncthreads();
    // Gram entries (g, i, j) += sum over the tile's rows of conj(X_a[row][i]) X_b[row][j]
#pragma unroll
    for (int m = 0; m < kSmallEntries; ++m) {
      const int e = threadIdx.x + m * kBT;
      if (e >= n_ent) break;
      const T *xa = planes + gx[m], *xb = planes + gy[m];
#pragma unroll 8
      for (int lr = 0; lr < kSR; ++lr) {
        const double ar = (double)xa[lr * R], ai = (double)xa[lr * R + pl];
        const double br = (double)xb[lr * R], bi = (double)xb[lr * R + pl];
        accr[m] += ar * br + ai * bi;
        acci[m] += ar * bi - ai * br;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < kSmallEntries; ++m) {
    const int e = threadIdx.x + m * kBT;
    if (e >= n_ent) break;
    a.partials[(long long)e * a.grid + blockIdx.x] = make_double2(accr[m], acci[m]);
  }
}

template <typename T>
void launch_small(int r, const BlocksArgs &a, size_t lds, hipStream_t s) {
  switch (r) {
    case 1: hipLaunchKernelGGL((k_blocks_small<T, 1>), dim3(a.grid), dim3(kBT), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_blocks_small<T, 2>), dim3(a.grid), dim3(kBT), lds, s, a); break;
    case 3: hipLaunchKernelGGL((k_blocks_small<T, 3>), dim3(a.grid), dim3(kBT), lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_blocks_small<T, 4>), dim3(a.grid), dim3(kBT), lds, s, a); break;
    case 5: hipLaunchKernelGGL((k_blocks_small<T, 5>), dim3(a.grid), dim3(kBT), lds, s, a); break;
    case 6: hipLaunchKernelGGL((k_blocks_small<T, 6>), dim3(a.grid), dim3(kBT), lds, s, a); break;
    case 7: hipLaunchKernelGGL((k_blocks_small<T, 7>), dim3(a.grid), dim3(kBT), lds, s, a); break;
    default: hipLaunchKernelGGL((k_blocks_small<T, 8>), dim3(a.grid), dim3(kBT), lds, s, a); break;
  }
}

template <typename T, int R>
void set_small_attr(int cap) {
  (void)hipFuncSetAttribute((const void *)k_blocks_small<T, R>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
}

template <typename T>
void set_small_attrs(int cap) {
  set_small_attr<T, 1>(cap);
  set_small_attr<T, 2>(cap);
  set_small_attr<T, 3>(cap);
  set_small_attr<T, 4>(cap);
  set_small_attr<T, 5>(cap);
  set_small_attr<T, 6>(cap);
  set_small_attr<T, 7>(cap);
  set_small_attr<T, 8>(cap);
}

}  // namespace

int blocks_grid(long long N) {
  const long long tiles = (N + kBR - 1) / kBR;
  long long g = tiles < 1024 ? tiles : 1024;
  if (g >= 8) g &= ~7LL;
  return (int)(g < 1 ? 1 : g);
}

namespace {
// the small-r path when r <= 8 and its planes fit in the LDS of a CU
bool use_small(bool fp32, int nin, int nout, int r) {
  return r <= 8 && small_planes_bytes(fp32, nin + nout, r) <= 160 * 1024;
}
}  // namespace

size_t blocks_lds(bool fp32, int nin, int nout, int r) {
  if (use_small(fp32, nin, nout, r))
    return small_planes_bytes(fp32, nin + nout, r) +
           (small_c_in_lds(fp32, nin, nout, r) ? (size_t)nin * nout * r * r * 16 : 0);
  return blocks_planes_bytes(fp32, nin + nout) +
         (blocks_c_in_lds(fp32, nin, nout, r) ? (size_t)nin * nout * r * r * 16 : 0);
}

bool launch_blocks(bool fp32, const BlocksArgs &a, hipStream_t s) {
  if (a.r < 1 || a.r > kBP || a.n_in < 0 || a.n_in > kMaxIoBlocks || a.n_out < 0 || a.n_out > kMaxIoBlocks ||
      a.n_gram < 0 || a.n_gram > kMaxGrams || a.grid < 1)
    return false;
  const size_t lds = blocks_lds(fp32, a.n_in, a.n_out, a.r);
  static bool attr = false;
  if (!attr) {
    const int cap = 160 * 1024;
    (void)hipFuncSetAttribute((const void *)k_blocks<float, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void *)k_blocks<float, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void *)k_blocks<double, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void *)k_blocks<double, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    set_small_attrs<float>(cap);
    set_small_attrs<double>(cap);
    attr = true;
  }
  if (lds > 160 * 1024) return false;
  if (use_small(fp32, a.n_in, a.n_out, a.r)) {
    if (fp32)
      launch_small<float>(a.r, a, lds, s);
    else
      launch_small<double>(a.r, a, lds, s);
    return true;
  }
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
