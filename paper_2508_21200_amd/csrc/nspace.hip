// N-space kernels of the LREI step on gfx950: the matrix-free Hamiltonian
// apply in the Krylov block recurrence P_{j+1} = beta (H P_j - P_j D_j) with
// fused Gram products, the
// basis combination that forms the new support, a deterministic reduction of
// per-workgroup partial sums, and the magnetisation pass.
//
// Layout: every N x r block is row-major complex (re, im interleaved), so the
// r columns of a basis row are one contiguous segment (256 B for r = 16 in
// FP64, 128 B in FP32) and any row gather is a coalesced segment load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lrei_internal.h"

namespace lrei {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kTile = 64;     // rows per tile
constexpr int kMaxLds = 150 * 1024;

__host__ __device__ inline int pow2ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
__host__ __device__ inline int pad16(int v) { return (v + 15) & ~15; }

// bfloat16 (the upper half of an IEEE float) for the low part of a
// compensated state: round to nearest even on the way in (finite values).
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// 16x16x4 MFMA wrappers.  Operand lanes: A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k.  Result D[i][j] sits in lane j + 16g, register v, with
// i = 4v + g for f64 and i = 4g + v for f32 (measured on gfx950).
__device__ inline d4v mfma(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4v mfma(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> __device__ inline int mfma_row(int lane, int v);
template <> __device__ inline int mfma_row<double>(int lane, int v) { return 4 * v + (lane >> 4); }
template <> __device__ inline int mfma_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }

template <typename T> struct Acc4;
template <> struct Acc4<double> { using type = d4v; };
template <> struct Acc4<float> { using type = f4v; };

// Tile -> workgroup assignment.  When possible each of the 8 XCDs (workgroup
// w runs on XCD w % 8) walks one contiguous eighth of the rows, so the
// partner rows of low-bit flips stay in that XCD's L2.
__device__ inline long long tile_of(long long k, long long num_tiles, int grid, int w) {
  if ((grid & 7) == 0 && (num_tiles & 7) == 0 && num_tiles >= grid) {
    const long long per = num_tiles >> 3;
    const int g8 = grid >> 3;
    const long long t = (long long)(w >> 3) + k * g8;
    return t < per ? (long long)(w & 7) * per + t : -1;
  }
  const long long t = (long long)w + k * grid;
  return t < num_tiles ? t : -1;
}

// Gram products over one LDS tile: G_g += X_g^H Y_g for up to 3 (X, Y) pairs.
// Planes hold re / im parts [kTile][RP] of type T.  Items are (gram, a-tile,
// b-tile, row split) distributed round-robin over the waves.
template <typename T>
struct GramPlan {
  int ng, ta, rs, items;
};

template <typename T, int MI>
__device__ inline void gram_tile(const T *const *xre, const T *const *xim, const T *const *yre,
                                 const T *const *yim, const GramPlan<T> &gp, int RP,
                                 double (&acc)[MI][8]) {
  using A4 = typename Acc4<T>::type;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows_per_split = kTile / gp.rs;
#pragma unroll
  for (int q = 0; q < MI; ++q) {
    const int it = wave + kWaves * q;
    if (it >= gp.items) break;
    int t = it;
    const int split = t % gp.rs; t /= gp.rs;
    const int tb = t % gp.ta; t /= gp.ta;
    const int ta = t % gp.ta; t /= gp.ta;
    const int g = t;
    const T *Xr = xre[g], *Xi = xim[g], *Yr = yre[g], *Yi = yim[g];
    const int a = ta * 16 + (lane & 15), b = tb * 16 + (lane & 15);
    A4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    const int row0 = split * rows_per_split;
    for (int kk = 0; kk < rows_per_split; kk += 4) {
      const int row = row0 + kk + (lane >> 4);
      const T xr = Xr[row * RP + a], xi = Xi[row * RP + a];
      const T yr = Yr[row * RP + b], yi = Yi[row * RP + b];
      cre = mfma(xr, yr, cre);
      cre = mfma(xi, yi, cre);
      cim = mfma(xr, yi, cim);
      cim = mfma(-xi, yr, cim);
    }
    // Per-tile products in T, accumulated across tiles in FP64.
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc[q][v] += (double)cre[v];
      acc[q][4 + v] += (double)cim[v];
    }
  }
}

// As gram_tile with one work item per wave, the per-tile products added to the
// FP64 accumulators in LDS (lacc[v * kThreads + thread], v < 8) instead of registers.
template <typename T>
__device__ inline void gram_tile_lds(const T *const *xre, const T *const *xim, const T *const *yre,
                                     const T *const *yim, const GramPlan<T> &gp, int RP, double *lacc) {
  using A4 = typename Acc4<T>::type;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows_per_split = kTile / gp.rs;
  const int it = wave;
  if (it >= gp.items) return;
  int t = it;
  const int split = t % gp.rs; t /= gp.rs;
  const int tb = t % gp.ta; t /= gp.ta;
  const int ta = t % gp.ta; t /= gp.ta;
  const int g = t;
  const T *Xr = xre[g], *Xi = xim[g], *Yr = yre[g], *Yi = yim[g];
  const int a = ta * 16 + (lane & 15), b = tb * 16 + (lane & 15);
  A4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
  const int row0 = split * rows_per_split;
  for (int kk = 0; kk < rows_per_split; kk += 4) {
    const int row = row0 + kk + (lane >> 4);
    const T xr = Xr[row * RP + a], xi = Xi[row * RP + a];
    const T yr = Yr[row * RP + b], yi = Yi[row * RP + b];
    cre = mfma(xr, yr, cre);
    cre = mfma(xi, yi, cre);
    cim = mfma(xr, yi, cim);
    cim = mfma(-xi, yr, cim);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    lacc[v * kThreads + threadIdx.x] += (double)cre[v];
    lacc[(4 + v) * kThreads + threadIdx.x] += (double)cim[v];
  }
}

// Writes the workgroup's Gram partial sums, entry-major: partials[e * grid + wg]
// with e = g * r * r + a * r + b.  Row splits (held by different waves) are
// summed through LDS in a fixed wave order, so the result is deterministic.
template <typename T, int MI>
__device__ inline void gram_store(const GramPlan<T> &gp, const double (&acc)[MI][8], int r,
                                  double2 *partials, double2 *stage /* LDS, ng * r * r */, int grid, int wg) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int w = 0; w < kWaves; ++w) {
    if (gp.rs == 1 || wave == w) {
#pragma unroll
      for (int q = 0; q < MI; ++q) {
        const int it = wave + kWaves * q;
        if (it >= gp.items) break;
        int t = it;
        const int split = t % gp.rs; t /= gp.rs;
        const int tb = t % gp.ta; t /= gp.ta;
        const int ta = t % gp.ta; t /= gp.ta;
        const int g = t;
        const int b = tb * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = ta * 16 + mfma_row<T>(lane, v);
          if (a < r && b < r) {
            const int e = (g * r + a) * r + b;
            const double2 val = make_double2(acc[q][v], acc[q][4 + v]);
            if (gp.rs == 1 || split == 0) {
              stage[e] = val;
            } else {
              stage[e].x += val.x;
              stage[e].y += val.y;
            }
          }
        }
      }
    }
    __syncthreads();
    if (gp.rs == 1) break;
  }
  for (int e = threadIdx.x; e < gp.ng * r * r; e += kThreads) partials[(long long)e * grid + wg] = stage[e];
}

template <typename T>
__device__ inline GramPlan<T> make_plan(int ng, int RP) {
  GramPlan<T> gp;
  gp.ng = ng;
  gp.ta = RP / 16;
  const int base = ng * gp.ta * gp.ta;
  gp.rs = base >= kWaves ? 1 : kWaves / base;  // rows per split stays a multiple of 16
  gp.items = base * gp.rs;
  return gp;
}

// ---------------------------------------------------------------------------
// Krylov pass with the Hamiltonian applied matrix-free:
//   P+ = alpha (H P - P diag(colshift)), colshift the per-column shifts of P
//   mode 0: first block     Grams P*P, P*P+, P+*P+
//   mode 1: later blocks    Grams P*P+, P+*P+
//   mode 2: Y = alpha H X   (no Grams, no shift)
//
// A row x of the output is d(x) X[x] + sum_t c_t(x) X[x ^ mask_t].  L lanes
// share a row, each holding E consecutive complex columns (16-byte loads), so
// the per-term index and coefficient work is done once per E columns.  The
// diagonal d(x) is precomputed per row.  The term table is read with uniform
// (scalar) loads; a coefficient is picked from the term's four entries by the
// two destination bits.  Terms with a zero coefficient for the row skip the load.
// ---------------------------------------------------------------------------
template <typename T, int E>
__device__ inline void load_ce(const T *p, T (&v)[2 * E]) {
  if constexpr (sizeof(T) == 4 && E == 1) {
    const float2 q = *reinterpret_cast<const float2 *>(p);
    v[0] = q.x; v[1] = q.y;
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < E / 2; ++k) {
      const float4 q = reinterpret_cast<const float4 *>(p)[k];
      v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const double2 q = reinterpret_cast<const double2 *>(p)[k];
      v[2 * k] = q.x; v[2 * k + 1] = q.y;
    }
  }
}
// Streaming stores of a pass's output block: written once, read by the next
// pass; the non-temporal hint keeps them from displacing the L2 lines that
// are reused (the pass's partner rows, the projected step's workspace).
typedef float f2n_t __attribute__((ext_vector_type(2)));
typedef float f4n_t __attribute__((ext_vector_type(4)));
typedef double d2n_t __attribute__((ext_vector_type(2)));
template <typename T, int E>
__device__ inline void store_ce_nt(T *p, const T (&v)[2 * E]) {
  if constexpr (sizeof(T) == 4 && E == 1) {
    __builtin_nontemporal_store(f2n_t{v[0], v[1]}, reinterpret_cast<f2n_t *>(p));
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < E / 2; ++k)
      __builtin_nontemporal_store(f4n_t{v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]},
                                  reinterpret_cast<f4n_t *>(p) + k);
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k)
      __builtin_nontemporal_store(d2n_t{v[2 * k], v[2 * k + 1]}, reinterpret_cast<d2n_t *>(p) + k);
  }
}
template <typename T, int E>
__device__ inline void store_ce(T *p, const T (&v)[2 * E]) {
  if constexpr (sizeof(T) == 4 && E == 1) {
    *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < E / 2; ++k)
      reinterpret_cast<float4 *>(p)[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k) reinterpret_cast<double2 *>(p)[k] = make_double2(v[2 * k], v[2 * k + 1]);
  }
}
template <typename T>
__device__ inline T pick4(int idx, T c0, T c1, T c2, T c3) {
  const T lo = (idx & 1) ? c1 : c0, hi = (idx & 1) ? c3 : c2;
  return (idx & 2) ? hi : lo;
}

// E complex columns per lane, CPLX: some coefficient has an imaginary part,
// MI: Gram work items per wave, WIN: row-bit window sweeps allowed, CMP:
// compacted gathers (below).  wg is the workgroup's index among the a.grid
// workgroups of this pass.
//
// Compacted gathers: a row needs the partner rows of the terms whose
// coefficient is non-zero for its two destination bits only (for an XXZ bond,
// about half of them).  With the term loop shared by the wave, every load
// instruction is issued for every term and carries only the lanes whose rows
// need it.  In the compacted form each row first marks its active terms in a
// 64-bit mask (the term's active pattern over the four destination-bit values
// is kept in the record), then every lane walks its own active
// terms in increasing order, reading the records from a copy in LDS, so that
// the wave issues max over its rows of the active-term count of loads per
// batch slot instead of the full term count.  The accumulation order of a row
// is the same in both forms, so their results are identical.
template <typename T, int E, bool CPLX, int MI, bool WIN, bool DYN, bool CMP = false>
__device__ __forceinline__ void hv_body(const HvArgs &a, int wg, unsigned char *smem) {
  static_assert(!DYN || (MI == 1 && !WIN), "the dynamic schedule keeps one Gram item per wave in LDS");
  // row gathers in flight per lane: kept small so that four waves fit per SIMD
  constexpr int B = (sizeof(T) == 4 ? 16 : 8) / E > 1 ? (sizeof(T) == 4 ? 16 : 8) / E : 2;
  const int r = a.r;
  const int L = a.lanes;   // lanes per row, power of two, L * E >= r
  const int RW = 64 / L;   // rows per wave per iteration
  const int RP = pad16(r);
  const bool grams = a.mode != 2 && !a.acc_out;

  // LDS: four planes [kTile][RP] (cur, next) x (re, im) for the Gram products
  T *planes = reinterpret_cast<T *>(smem);
  const int plane = kTile * RP;
  T *cre = planes, *cim = planes + plane, *nre = planes + 2 * plane, *nim = planes + 3 * plane;
  if (grams)
    for (int i = threadIdx.x; i < 4 * plane; i += kThreads) planes[i] = T(0);
  __syncthreads();

  const T *__restrict__ Pc = reinterpret_cast<const T *>(a.Pcur);
  T *__restrict__ Pn = reinterpret_cast<T *>(a.Pnext);
  // The term table is read-only during the launch and every lane of a wave
  // reads the same record: reading it through the constant address space
  // makes these scalar loads, which are waited for separately from the row
  // gathers, so the gathers of several terms stay in flight together.
  using TermC = const __attribute__((address_space(4))) DevTerm<T>;
  TermC *terms = (TermC *)(a.terms);
  const T *__restrict__ dv = reinterpret_cast<const T *>(a.diagv);
  const T *__restrict__ Yin = reinterpret_cast<const T *>(a.acc_in);

  // compacted gathers: the terms t0 .. t1 - 1 (at most 64) copied to LDS
  DevTerm<T> *lterm = reinterpret_cast<DevTerm<T> *>(smem + a.cmp_off);
  if constexpr (CMP) {
    const int nt = a.t1 - a.t0;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(a.terms) + (size_t)a.t0 * (sizeof(DevTerm<T>) / 4);
    uint32_t *dst = reinterpret_cast<uint32_t *>(lterm);
    for (int i = threadIdx.x; i < nt * (int)(sizeof(DevTerm<T>) / 4); i += kThreads) dst[i] = src[i];
    __syncthreads();
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane % L, rsub = lane / L;
  const int col0 = cl * E;
  const bool active = col0 < r;
  const T alpha = (T)a.alpha;
  // column shifts of this block (the recurrence subtracts P_j diag(shift))
  T csh[E];
#pragma unroll
  for (int e = 0; e < E; ++e) csh[e] = (a.colshift && col0 + e < r) ? (T)a.colshift[col0 + e] : T(0);

  const int ng = a.mode == 2 ? 0 : (a.mode == 0 ? 3 : 2);
  GramPlan<T> gp = make_plan<T>(ng > 0 ? ng : 1, RP);
  const T *xre[3], *xim[3], *yre[3], *yim[3];
  if (a.mode == 0) {
    xre[0] = cre; xim[0] = cim; yre[0] = cre; yim[0] = cim;
    xre[1] = cre; xim[1] = cim; yre[1] = nre; yim[1] = nim;
    xre[2] = nre; xim[2] = nim; yre[2] = nre; yim[2] = nim;
  } else {
    xre[0] = cre; xim[0] = cim; yre[0] = nre; yim[0] = nim;
    xre[1] = nre; xim[1] = nim; yre[1] = nre; yim[1] = nim;
    xre[2] = nre; xim[2] = nim; yre[2] = nre; yim[2] = nim;
  }
  double acc[MI][8];
#pragma unroll
  for (int q = 0; q < MI; ++q)
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[q][v] = 0.0;

  const long long N = a.N;
  const int t0 = a.t0, t1 = a.t1;
  // Tiles of 64 rows.  One window (the default): the natural row order, each
  // XCD walking a contiguous eighth.  Several windows (a sweep confined to the
  // window bits of its terms): the XCD x = wg % 8 takes windows x, x + 8, ...,
  // and its workgroups share each window's tiles, so the window's rows stay in
  // that XCD's L2 while its partner rows are gathered.
  const int nw = a.win_bits;
  const long long nwin = 1LL << a.n_fix;
  const long long tiles_per_win = ((1LL << nw) + kTile - 1) / kTile;
  auto deposit = [&](long long v, const unsigned char *pos, int nb) {
    uint32_t x = 0;
    for (int i = 0; i < nb; ++i) x |= (uint32_t)((v >> i) & 1) << pos[i];
    return x;
  };
  const int xcd = wg & 7, slot = wg >> 3, g8 = a.grid >> 3;
  const bool by_window = WIN && nwin >= 8 && (a.grid & 7) == 0;
  long long wi = by_window ? xcd : 0, lt = by_window ? slot : 0;
  uint32_t wbase = by_window ? deposit(wi, a.fix_pos, a.n_fix) : 0;
  const long long num_tiles = (N + kTile - 1) / kTile;
  // Dynamic schedule: the tiles of XCD slot x = wg % 8 (a contiguous eighth of
  // the rows) form cpx chunks, chunk c holding tiles c, c + cpx, ... of the
  // slot (so the chunks being worked on at one time cover consecutive tiles).
  // The slot's workgroups take chunks from counter sched[x]: a workgroup on a
  // CU shared with other work takes fewer, instead of holding up the pass.
  // Gram partial sums are kept per chunk (accumulated in LDS), so the result
  // does not depend on which workgroup took which chunk.  Each workgroup
  // makes one failing take; the slot's last one to finish (counted in
  // sched[8 + x]) resets both counters for the next launch.
  // Chunk c of a slot holds tiles c, c + cpx, ... below per: per / cpx or one
  // more, so any chunk count up to per covers the slot.
  const int cpx = DYN ? a.chunks >> 3 : 1;
  const long long per = num_tiles >> 3;
  // dynamic schedule only (r <= 16): the staged partial sums fit in the planes
  double *lacc = reinterpret_cast<double *>(smem + 4 * (size_t)plane * sizeof(T));
  __shared__ int s_chunk;
  int chunk = -1;
  long long kc = 0, kn = 0;  // tiles of the current chunk done / in it
  if constexpr (DYN) {
    for (int v = 0; v < 8; ++v) lacc[v * kThreads + threadIdx.x] = 0.0;
  }
  for (long long k = 0;; ++k) {
    long long row0 = 0;
    uint32_t tbase = 0;
    if constexpr (DYN) {
      if (kc == kn) {
        if (grams && chunk >= 0) {  // the finished chunk's partial sums
          double av[1][8];
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            av[0][v] = lacc[v * kThreads + threadIdx.x];
            lacc[v * kThreads + threadIdx.x] = 0.0;
          }
          gram_store<T, 1>(gp, av, r, a.partials, reinterpret_cast<double2 *>(planes), a.chunks, xcd * cpx + chunk);
          __syncthreads();
          for (int i = threadIdx.x; i < 4 * plane; i += kThreads) planes[i] = T(0);
        }
        if (threadIdx.x == 0) s_chunk = atomicAdd(&a.sched[xcd], 1);
        __syncthreads();
        chunk = s_chunk;
        __syncthreads();
        if (chunk >= cpx) {
          if (threadIdx.x == 0 && atomicAdd(&a.sched[8 + xcd], 1) == g8 - 1) {
            atomicExch(&a.sched[xcd], 0);
            atomicExch(&a.sched[8 + xcd], 0);
          }
          break;
        }
        kc = 0;
        kn = (per - chunk + cpx - 1) / cpx;
      }
      row0 = ((long long)xcd * per + chunk + kc * cpx) * kTile;
      ++kc;
    } else if (by_window) {
      while (wi < nwin && lt >= tiles_per_win) {
        wi += 8;
        lt = slot;
        if (wi < nwin) wbase = deposit(wi, a.fix_pos, a.n_fix);
      }
      if (wi >= nwin) break;
      tbase = wbase | deposit(lt * kTile, a.win_pos, nw);
      lt += g8;
    } else {
      const long long tile = tile_of(k, num_tiles, a.grid, wg);
      if (tile < 0) break;
      row0 = tile * kTile;
    }
    for (int it = 0; it * kWaves * RW < kTile; ++it) {
      const int lr = it * kWaves * RW + wave * RW + rsub;  // local row
      if (lr >= kTile) continue;
      const long long x = by_window ? (long long)(tbase | deposit(lr, a.win_pos, nw < 6 ? nw : 6)) : row0 + lr;
      if (x >= N || !active || (by_window && (lr >> (nw < 6 ? nw : 6)) != 0)) continue;
      const uint32_t xu = (uint32_t)x;
      const size_t rowo = (size_t)xu * r;           // row offset (complex)
      const size_t base = rowo + col0;
      auto ld = [&](const T *P, size_t ro, T(&v)[2 * E]) { load_ce<T, E>(P + 2 * (ro + col0), v); };
      T own[2 * E], o[2 * E];
      ld(Pc, rowo, own);
      if (a.use_diag) {
        const T d = dv[xu];
#pragma unroll
        for (int e = 0; e < 2 * E; ++e) o[e] = d * own[e];
      } else {
#pragma unroll
        for (int e = 0; e < 2 * E; ++e) o[e] = T(0);
      }
      if (Yin) {
        T yv[2 * E];
        ld(Yin, rowo, yv);
#pragma unroll
        for (int e = 0; e < 2 * E; ++e) o[e] += yv[e];
      }
      auto fma_batch = [&](const T (&y)[B][2 * E], const T (&cr)[B], const T (&ci)[B]) {
#pragma unroll
        for (int u = 0; u < B; ++u)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            o[2 * e] += cr[u] * y[u][2 * e];
            o[2 * e + 1] += cr[u] * y[u][2 * e + 1];
            if (CPLX) {
              o[2 * e] -= ci[u] * y[u][2 * e + 1];
              o[2 * e + 1] += ci[u] * y[u][2 * e];
            }
          }
      };
      if constexpr (CMP) {
        // active terms of this row: bit k for term t0 + k
        uint32_t am0 = 0, am1 = 0;
        for (int t = t0; t < t1; ++t) {
          TermC &tm = terms[t];
          const uint32_t idx = ((xu >> tm.sa) & 1u) | (((xu >> tm.sb) & 1u) << 1);
          const uint32_t bit = (tm.act >> idx) & 1u;
          const int k = t - t0;
          if (k < 32) am0 |= bit << k;
          else am1 |= bit << (k - 32);
        }
        uint64_t act = ((uint64_t)am1 << 32) | am0;
        while (__any(act != 0)) {
          T y[B][2 * E];
          T cr[B], ci[B];
#pragma unroll
          for (int u = 0; u < B; ++u) {
            cr[u] = T(0);
            ci[u] = T(0);
#pragma unroll
            for (int e = 0; e < 2 * E; ++e) y[u][e] = T(0);
            if (act != 0) {
              const int k = __builtin_ctzll(act);
              act &= act - 1;
              const DevTerm<T> &tm = lterm[k];
              const int idx = (int)(((xu >> tm.sa) & 1u) | (((xu >> tm.sb) & 1u) << 1));
              cr[u] = tm.re[idx];
              if (CPLX) ci[u] = tm.im[idx];
              ld(Pc, (size_t)(xu ^ tm.mask) * r, y[u]);
            }
          }
          fma_batch(y, cr, ci);
        }
      } else {
        for (int t = t0; t < t1; t += B) {
          T y[B][2 * E];
          T cr[B], ci[B];
#pragma unroll
          for (int u = 0; u < B; ++u) {
            cr[u] = T(0);
            ci[u] = T(0);
#pragma unroll
            for (int e = 0; e < 2 * E; ++e) y[u][e] = T(0);
            if (t + u < t1) {
              TermC &tm = terms[t + u];
              const int idx = (int)(((xu >> tm.sa) & 1u) | (((xu >> tm.sb) & 1u) << 1));
              cr[u] = pick4(idx, tm.re[0], tm.re[1], tm.re[2], tm.re[3]);
              if (CPLX) ci[u] = pick4(idx, tm.im[0], tm.im[1], tm.im[2], tm.im[3]);
              if (cr[u] != T(0) || ci[u] != T(0)) ld(Pc, (size_t)(xu ^ tm.mask) * r, y[u]);
            }
          }
          fma_batch(y, cr, ci);
        }
      }
      if (!a.acc_out) {
#pragma unroll
        for (int e = 0; e < 2 * E; ++e) o[e] = alpha * (o[e] - csh[e >> 1] * own[e]);
      }
      store_ce_nt<T, E>(Pn + 2 * base, o);
      if (grams) {
        const int gl = by_window ? lr : (int)(x - row0);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int c = col0 + e;
          if (c < r) {
            cre[gl * RP + c] = own[2 * e];
            cim[gl * RP + c] = own[2 * e + 1];
            nre[gl * RP + c] = o[2 * e];
            nim[gl * RP + c] = o[2 * e + 1];
          }
        }
      }
    }
    if (grams) {
      __syncthreads();
      // rows beyond N keep the zeros written at start only for the first tile;
      // N is a power of two >= 2 so a partial tile is always the only tile.
      if constexpr (DYN)
        gram_tile_lds<T>(xre, xim, yre, yim, gp, RP, lacc);
      else
        gram_tile<T, MI>(xre, xim, yre, yim, gp, RP, acc);
      __syncthreads();
    }
  }
  if constexpr (!DYN) {
    if (grams) {
      __syncthreads();
      gram_store<T, MI>(gp, acc, r, a.partials, reinterpret_cast<double2 *>(planes), a.grid, wg);
    }
  }
}

template <typename T, int E, bool CPLX, int MI, bool DYN, bool CMP>
__global__ __launch_bounds__(kThreads) void k_hv(HvArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (a.skip && *a.skip != 0.0) return;  // the same for every workgroup of the launch
  hv_body<T, E, CPLX, MI, !DYN, DYN, CMP>(a, blockIdx.x, smem);
}

// Many independent passes in one launch (one per trajectory of a batch): the
// workgroup's job and its index within that job come from the launch tables;
// every job's workgroups start at a multiple of 8, so a workgroup keeps its
// XCD slot within the job.
template <typename T, int E, bool CPLX, int MI, bool DYN>
__global__ __launch_bounds__(kThreads) void k_hv_batch(BatchLaunch b) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int j = b.wg_job[blockIdx.x];
  if (j < 0) return;  // alignment padding
  const HvArgs a = reinterpret_cast<const HvArgs *>(b.jobs)[j];
  hv_body<T, E, CPLX, MI, false, DYN>(a, blockIdx.x - b.job_wg0[j], smem);
}

// ---------------------------------------------------------------------------
// Tiled Krylov pass.  A workgroup of W waves walks tiles of R = 2^k
// consecutive rows: it loads the tile of P_j into LDS (each row's 16-byte
// chunks XOR-swizzled by the low row bits, so the rows that one load
// instruction gathers fall on different banks), then every row's output
//   P+[x] = alpha (d(x) P[x] + sum_t c_t(x) P[x ^ m_t] - P[x] diag(shift))
// takes the partner rows of the terms t < n_local (flip masks below 2^k) from
// LDS and gathers those of the other terms from global memory.  Each wave
// stages its RW output rows in an LDS slice of its own and adds their Gram
// products (P*P+, P+*P+; P*P too in mode 0) on MFMA, per tile in T and across
// tiles in FP64; the waves' sums meet in LDS in a fixed order at the end.
// Rows are 16-byte multiples (FP32: r even), r <= 16.
// ---------------------------------------------------------------------------
template <typename T, int E, bool CPLX, int W>
__global__ __launch_bounds__(64 * W) void k_hv_tile(HvArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (a.skip && *a.skip != 0.0) return;
  using A4 = typename Acc4<T>::type;
  constexpr int NTH = 64 * W;
  constexpr int CB = 2 * sizeof(T);  // bytes per complex
  constexpr int LB = E * CB;         // bytes per lane per row
  constexpr int B = (sizeof(T) == 4 ? 16 : 8) / E > 1 ? (sizeof(T) == 4 ? 16 : 8) / E : 2;
  static_assert(LB % 16 == 0, "lanes move whole 16-byte chunks");
  const int r = a.r;
  const int L = a.lanes, RW = 64 / L;
  const int kb = a.tile_bits, R = 1 << kb;
  const int rowb = r * CB, cpr = rowb >> 4;
  const int smask = (cpr & (cpr - 1)) == 0 ? cpr - 1 : 0;
  unsigned char *tile = smem;
  T *stage = reinterpret_cast<T *>(smem + (size_t)R * rowb);  // [W][RW][r] complex
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane % L, rsub = lane / L;
  const int col0 = cl * E;
  const bool active = col0 < r;
  const T alpha = (T)a.alpha;
  T csh[E];
#pragma unroll
  for (int e = 0; e < E; ++e) csh[e] = (a.colshift && col0 + e < r) ? (T)a.colshift[col0 + e] : T(0);
  const T *__restrict__ Pc = reinterpret_cast<const T *>(a.Pcur);
  T *__restrict__ Pn = reinterpret_cast<T *>(a.Pnext);
  using TermC = const __attribute__((address_space(4))) DevTerm<T>;
  TermC *terms = (TermC *)(a.terms);
  const T *__restrict__ dv = reinterpret_cast<const T *>(a.diagv);
  const int nloc = a.n_local, noff = a.n_off;
  const int ng = a.mode == 0 ? 3 : 2;

  // LDS row access: the E complex columns of this lane (LB / 16 chunks)
  auto lds_ld = [&](int row, T (&v)[2 * E]) {
    const unsigned char *rp = tile + (size_t)row * rowb;
    const int c0 = (col0 * CB) >> 4;
#pragma unroll
    for (int q = 0; q < LB / 16; ++q) {
      const uint4 w = *reinterpret_cast<const uint4 *>(rp + (((c0 + q) ^ (row & smask)) << 4));
      const T *f = reinterpret_cast<const T *>(&w);
#pragma unroll
      for (int h = 0; h < 16 / (int)sizeof(T); ++h) v[q * (16 / sizeof(T)) + h] = f[h];
    }
  };
  auto g_ld = [&](const T *P, size_t ro, T (&v)[2 * E]) { load_ce<T, E>(P + 2 * (ro + col0), v); };

  double acc[3][8];
#pragma unroll
  for (int g = 0; g < 3; ++g)
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[g][v] = 0.0;

  const long long num_tiles = a.N >> kb;
  const int wg = blockIdx.x;
  for (long long k = 0;; ++k) {
    const long long tid = tile_of(k, num_tiles, a.grid, wg);
    if (tid < 0) break;
    const long long base = tid << kb;
    __syncthreads();  // the previous tile's rows are no longer read
    {
      const unsigned char *src = reinterpret_cast<const unsigned char *>(Pc) + (size_t)base * rowb;
      for (int j = threadIdx.x; j < R * cpr; j += NTH) {
        const int row = j / cpr, c = j - row * cpr;
        *reinterpret_cast<uint4 *>(tile + (size_t)row * rowb + ((c ^ (row & smask)) << 4)) =
            *reinterpret_cast<const uint4 *>(src + ((size_t)j << 4));
      }
    }
    __syncthreads();
    A4 tre[3], tim[3];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      tre[g] = A4{0, 0, 0, 0};
      tim[g] = A4{0, 0, 0, 0};
    }
    for (int it = 0; it < R / (W * RW); ++it) {
      const int lr0 = it * W * RW + wave * RW;  // this wave's first row of the iteration
      const int lr = lr0 + rsub;
      const uint32_t xu = (uint32_t)(base + lr);
      T own[2 * E], o[2 * E];
#pragma unroll
      for (int e = 0; e < 2 * E; ++e) own[e] = o[e] = T(0);
      if (active) {
        lds_ld(lr, own);
        const T d = dv[xu];
#pragma unroll
        for (int e = 0; e < 2 * E; ++e) o[e] = d * own[e];
        // terms inside the tile: partners from LDS; the others from global memory
        for (int part = 0; part < 2; ++part) {
          const int t0 = part == 0 ? 0 : nloc, t1 = part == 0 ? nloc : noff;
          for (int t = t0; t < t1; t += B) {
            T y[B][2 * E];
            T cr[B], ci[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
              cr[u] = T(0);
              ci[u] = T(0);
#pragma unroll
              for (int e = 0; e < 2 * E; ++e) y[u][e] = T(0);
              if (t + u < t1) {
                TermC &tm = terms[t + u];
                const int idx = (int)(((xu >> tm.sa) & 1u) | (((xu >> tm.sb) & 1u) << 1));
                cr[u] = pick4(idx, tm.re[0], tm.re[1], tm.re[2], tm.re[3]);
                if (CPLX) ci[u] = pick4(idx, tm.im[0], tm.im[1], tm.im[2], tm.im[3]);
                if (cr[u] != T(0) || ci[u] != T(0)) {
                  if (part == 0)
                    lds_ld(lr ^ (int)tm.mask, y[u]);
                  else
                    g_ld(Pc, (size_t)(xu ^ tm.mask) * r, y[u]);
                }
              }
            }
#pragma unroll
            for (int u = 0; u < B; ++u)
#pragma unroll
              for (int e = 0; e < E; ++e) {
                o[2 * e] += cr[u] * y[u][2 * e];
                o[2 * e + 1] += cr[u] * y[u][2 * e + 1];
                if (CPLX) {
                  o[2 * e] -= ci[u] * y[u][2 * e + 1];
                  o[2 * e + 1] += ci[u] * y[u][2 * e];
                }
              }
          }
        }
#pragma unroll
        for (int e = 0; e < 2 * E; ++e) o[e] = alpha * (o[e] - csh[e >> 1] * own[e]);
        store_ce<T, E>(Pn + 2 * ((size_t)xu * r + col0), o);
        // this wave's slice of the output rows for the Gram products
        T *sp = stage + 2 * ((size_t)(wave * RW + rsub) * r + col0);
#pragma unroll
        for (int e = 0; e < 2 * E; ++e) sp[e] = o[e];
      }
      __builtin_amdgcn_wave_barrier();  // the slice is read across lanes of this wave below
      // Grams over the wave's RW rows: lane i + 16 q holds column i of row 4 s + q
      const int gi = lane & 15, gq = lane >> 4;
      for (int s4 = 0; s4 < RW; s4 += 4) {
        T xr = T(0), xi = T(0), yr = T(0), yi = T(0);
        if (gi < r) {
          const int row = lr0 + s4 + gq;
          const int byte = gi * CB;
          const T *xp = reinterpret_cast<const T *>(tile + (size_t)row * rowb +
                                                    ((((byte >> 4) ^ (row & smask)) << 4) | (byte & 15)));
          xr = xp[0];
          xi = xp[1];
          const T *yp = stage + 2 * ((size_t)(wave * RW + s4 + gq) * r + gi);
          yr = yp[0];
          yi = yp[1];
        }
        // G_XY = sum conj(x) y, G_YY, G_XX (mode 0)
        tre[0] = mfma(xr, yr, tre[0]);
        tre[0] = mfma(xi, yi, tre[0]);
        tim[0] = mfma(xr, yi, tim[0]);
        tim[0] = mfma(-xi, yr, tim[0]);
        tre[1] = mfma(yr, yr, tre[1]);
        tre[1] = mfma(yi, yi, tre[1]);
        tim[1] = mfma(yr, yi, tim[1]);
        tim[1] = mfma(-yi, yr, tim[1]);
        if (ng == 3) {
          tre[2] = mfma(xr, xr, tre[2]);
          tre[2] = mfma(xi, xi, tre[2]);
          tim[2] = mfma(xr, xi, tim[2]);
          tim[2] = mfma(-xi, xr, tim[2]);
        }
      }
      __builtin_amdgcn_wave_barrier();  // the slice is rewritten next iteration
    }
#pragma unroll
    for (int g = 0; g < 3; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[g][v] += (double)tre[g][v];
        acc[g][4 + v] += (double)tim[g][v];
      }
  }
  // waves' sums in a fixed order, then the workgroup's partials (entry-major;
  // Gram order of the pass: mode 0 P*P, P*P+, P+*P+; mode 1 P*P+, P+*P+)
  __syncthreads();
  double2 *red = reinterpret_cast<double2 *>(smem);
  for (int w = 0; w < W; ++w) {
    if (wave == w) {
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        if (g >= ng) break;
        const int slot = ng == 3 ? (g == 2 ? 0 : (g == 0 ? 1 : 2)) : (g == 0 ? 0 : 1);
        const int b = lane & 15;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int arow = mfma_row<T>(lane, v);
          if (arow < r && b < r) {
            const int e = (slot * r + arow) * r + b;
            const double2 val = make_double2(acc[g][v], acc[g][4 + v]);
            if (w == 0) {
              red[e] = val;
            } else {
              red[e].x += val.x;
              red[e].y += val.y;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < ng * r * r; e += NTH) a.partials[(long long)e * a.grid + wg] = red[e];
}

// Diagonal of H per row: d(x) = sum_k w_k (1 - 2 (b_{i_k}(x) xor b_{j_k}(x))),
// bit 31 of a row index being 0 (one-site terms use j_k = 31).
__global__ void k_diag_values(const DevDiagTerm *diag, int n_diag, long long N, double *d64, float *d32) {
  for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < N; x += (long long)gridDim.x * blockDim.x) {
    const uint32_t xu = (uint32_t)x;
    double s = 0.0;
    for (int t = 0; t < n_diag; ++t) {
      const DevDiagTerm dt = diag[t];
      s += (((xu >> dt.si) ^ (xu >> dt.sj)) & 1u) ? -dt.w : dt.w;
    }
    d64[x] = s;
    if (d32) d32[x] = (float)s;
  }
}

// ---------------------------------------------------------------------------
// out (N x r) = [B_0 ... B_{nb-1}] (N x nb r) * C (nb r x r), C complex FP64.
// In place over B_0 is allowed: a tile's rows are read before they are written.
// ---------------------------------------------------------------------------

// Each wave forms 16 output rows at a time with 16x16x4 MFMA.  The MFMA inner
// index is permuted so that lane (i, q) of the A operand holds CPL consecutive
// complex columns q*CPL .. q*CPL+CPL-1 of row i (one contiguous vector load);
// step s of the product uses column q*CPL + s, and C is read with the same
// permutation.  C sits in LDS.  In place over block 0 is allowed: a wave reads
// all of its rows before it writes them, and no other wave touches them.
template <typename T, int RP>
__device__ __forceinline__ void combine_body(const CombineArgs &a, int wg, unsigned char *smem) {
  using A4 = typename Acc4<T>::type;
  const int r = a.r, nb = a.nb;
  const int K = nb * RP;
  T *cre = reinterpret_cast<T *>(smem);  // [K][RP]
  T *cim = cre + K * RP;
  for (int i = threadIdx.x; i < K * RP; i += kThreads) {
    const int kk = i / RP, j = i % RP;
    const int blk = kk / RP, ak = kk % RP;
    double2 c = make_double2(0.0, 0.0);
    if (ak < r && j < r) c = a.C[(blk * r + ak) * r + j];
    if (a.lo_in && blk == 0 && ak == j && j < r) c.x -= 1.0;  // compensated state: the update only
    cre[i] = (T)c.x;
    cim[i] = (T)c.y;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  constexpr int CPL = RP / 4;  // 4 or 8 complex columns per lane
  constexpr int TA = RP / 16;
  T *out = reinterpret_cast<T *>(a.out);
  const long long N = a.N;
  const long long num_tiles = (N + kTile - 1) / kTile;
  for (long long k = 0;; ++k) {
    const long long tile = tile_of(k, num_tiles, a.grid, wg);
    if (tile < 0) break;
    const long long x = tile * kTile + wave * 16 + i16;  // this lane's A row
    A4 ore[2], oim[2];
    for (int t = 0; t < 2; ++t) { ore[t] = A4{0, 0, 0, 0}; oim[t] = A4{0, 0, 0, 0}; }
    for (int blk = 0; blk < nb; ++blk) {
      const T *B = reinterpret_cast<const T *>(a.blocks[blk]);
      T v[16];  // up to 8 complex
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = T(0);
      const int c0 = q * CPL;
      if (x < N) {
        if (c0 + CPL <= r) {
          if constexpr (CPL == 4) {
            load_ce<T, 4>(B + 2 * ((size_t)x * r + c0), *reinterpret_cast<T(*)[8]>(v));
          } else {
            load_ce<T, 4>(B + 2 * ((size_t)x * r + c0), *reinterpret_cast<T(*)[8]>(v));
            load_ce<T, 4>(B + 2 * ((size_t)x * r + c0 + 4), *reinterpret_cast<T(*)[8]>(v + 8));
          }
        } else {
          for (int e = 0; e < CPL; ++e)
            if (c0 + e < r) {
              v[2 * e] = B[2 * ((size_t)x * r + c0 + e)];
              v[2 * e + 1] = B[2 * ((size_t)x * r + c0 + e) + 1];
            }
        }
      }
#pragma unroll
      for (int st = 0; st < CPL; ++st) {
        const T ar = v[2 * st], ai = v[2 * st + 1];
        const int crow = blk * RP + c0 + st;
        for (int tb = 0; tb < TA; ++tb) {
          const int ccol = tb * 16 + i16;
          const T br = cre[crow * RP + ccol], bi = cim[crow * RP + ccol];
          ore[tb] = mfma(ar, br, ore[tb]);
          ore[tb] = mfma(-ai, bi, ore[tb]);
          oim[tb] = mfma(ar, bi, oim[tb]);
          oim[tb] = mfma(ai, br, oim[tb]);
        }
      }
    }
    // D[i][j] in lane j + 16 g, register v: row mfma_row(lane, v), column j = lane % 16
#pragma unroll
    for (int tb = 0; tb < TA; ++tb) {
      const int j = tb * 16 + i16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long long xo = tile * kTile + wave * 16 + mfma_row<T>(lane, v);
        if (j < r && xo < N) {
          const size_t o = 2 * ((size_t)xo * r + j);
          if constexpr (sizeof(T) == 4) {
            if (a.lo_in) {
              // hi + lo + update in FP64, split again (this wave read row xo of
              // blocks[0] above; out may be blocks[0]); lo is bfloat16
              const float2 h = *reinterpret_cast<const float2 *>(reinterpret_cast<const T *>(a.blocks[0]) + o);
              const ushort2 l = reinterpret_cast<const ushort2 *>(a.lo_in)[o / 2];
              const double vr = (double)h.x + (double)from_bf16(l.x) + (double)ore[tb][v];
              const double vi = (double)h.y + (double)from_bf16(l.y) + (double)oim[tb][v];
              const float hr = (float)vr, hm = (float)vi;
              *reinterpret_cast<float2 *>(out + o) = make_float2(hr, hm);
              reinterpret_cast<ushort2 *>(a.lo_out)[o / 2] =
                  make_ushort2(to_bf16((float)(vr - (double)hr)), to_bf16((float)(vi - (double)hm)));
              continue;
            }
          }
          out[o] = ore[tb][v];
          out[o + 1] = oim[tb][v];
        }
      }
    }
  }
}

template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_combine(CombineArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (a.skip && *a.skip != 0.0) return;
  combine_body<T, RP>(a, blockIdx.x, smem);
}

template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_combine_batch(BatchLaunch b) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int j = b.wg_job[blockIdx.x];
  if (j < 0) return;  // alignment padding
  // read in place: a copy of the block-pointer array would live in scratch
  const CombineArgs &a = reinterpret_cast<const CombineArgs *>(b.jobs)[j];
  combine_body<T, RP>(a, blockIdx.x - b.job_wg0[j], smem);
}

// Deterministic reduction of entry-major partials: out[e] = sum_c in[e * count + c],
// one workgroup per entry, strided per-thread sums then a fixed tree.
__device__ __forceinline__ void reduce_body(const double2 *in, int count, double2 *out, int e) {
  __shared__ double2 part[256];
  double sr = 0.0, si = 0.0;
  for (int c = threadIdx.x; c < count; c += 256) {
    const double2 v = in[(long long)e * count + c];
    sr += v.x;
    si += v.y;
  }
  part[threadIdx.x] = make_double2(sr, si);
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      part[threadIdx.x].x += part[threadIdx.x + w].x;
      part[threadIdx.x].y += part[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[e] = part[0];
}

__global__ __launch_bounds__(256) void k_reduce(const double2 *in, int count, int len, double2 *out) {
  (void)len;
  reduce_body(in, count, out, blockIdx.x);
}

// One workgroup per entry of every job.
__global__ __launch_bounds__(256) void k_reduce_batch(BatchLaunch b) {
  const int j = b.wg_job[blockIdx.x];
  if (j < 0) return;
  const ReduceJob q = reinterpret_cast<const ReduceJob *>(b.jobs)[j];
  reduce_body(q.in, q.count, q.out, blockIdx.x - b.job_wg0[j]);
}

// Row permutation by a bit map: y(x) = sum_i bit_i(x) << pos[i].
// forward: dst[y(x)] = src[x]; inverse: dst[x] = src[y(x)].
struct PermArgs {
  unsigned char pos[32];
  int n;
};
template <typename C2>
__global__ void k_permute_rows(const C2 *src, C2 *dst, long long N, int r, PermArgs pa, int inverse) {
  const long long total = N * r;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long x = e / r;
    const int c = (int)(e % r);
    uint32_t y = 0;
    for (int i = 0; i < pa.n; ++i) y |= (uint32_t)((x >> i) & 1) << pa.pos[i];
    if (inverse)
      dst[e] = src[(long long)y * r + c];
    else
      dst[(long long)y * r + c] = src[e];
  }
}

__global__ void k_convert_d2f(const double2 *src, float2 *dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}
__global__ void k_split_d2f(const double2 *src, float2 *hi, ushort2 *lo, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double2 v = src[i];
    const float2 h = make_float2((float)v.x, (float)v.y);
    hi[i] = h;
    lo[i] = make_ushort2(to_bf16((float)(v.x - (double)h.x)), to_bf16((float)(v.y - (double)h.y)));
  }
}
__global__ void k_merge_f2d(const float2 *hi, const ushort2 *lo, double2 *dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = make_double2((double)hi[i].x + (double)from_bf16(lo[i].x), (double)hi[i].y + (double)from_bf16(lo[i].y));
}
__global__ void k_convert_f2d(const float2 *src, double2 *dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = make_double2((double)src[i].x, (double)src[i].y);
}

// Magnetisation partials: per workgroup (sum_x,a lam_a conj(V[x,a]) s^v_i V)
// summed over sites i, for v = x, y, z; written as [grid][2] double2 =
// (mx, my), (mz, 0).  The 1/n and hbar/2 factors are applied on the host.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_magnet(const void *Vp, const double *lam, long long N,
                                                     int r, int n, double2 *partials) {
  using C2 = typename Cplx<T>::type;
  const C2 *V = reinterpret_cast<const C2 *>(Vp);
  const int L = pow2ceil(r), RW = 64 / L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane % L, rsub = lane / L;
  double mx = 0, my = 0, mz = 0;
  if (col < r) {
    const double lm = lam[col];
    const long long rows_per_block = (long long)kWaves * RW;
    for (long long x0 = (long long)blockIdx.x * rows_per_block; x0 < N;
         x0 += (long long)gridDim.x * rows_per_block) {
      const long long x = x0 + wave * RW + rsub;
      if (x >= N) continue;
      const C2 v = V[x * r + col];
      const double vr = v.x, vi = v.y;
      const double w = lm * (vr * vr + vi * vi);
      int up = 0;
      for (int i = 0; i < n; ++i) {
        const int b = (int)((x >> i) & 1);
        up += b ? -1 : 1;
        const C2 u = V[(x ^ (1LL << i)) * r + col];
        // conj(v) * u
        const double pr = vr * u.x + vi * u.y, pi = vr * u.y - vi * u.x;
        mx += lm * pr;
        // <b|s^y|1-b> = -i (b = 0), +i (b = 1): contributes Re(conj(v) * (+-i) u)
        my += lm * (b ? -pi : pi);
      }
      mz += w * up;
    }
  }
  __shared__ double red[3][kThreads];
  red[0][threadIdx.x] = mx;
  red[1][threadIdx.x] = my;
  red[2][threadIdx.x] = mz;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = make_double2(red[0][0], red[1][0]);
    partials[2 * blockIdx.x + 1] = make_double2(red[2][0], 0.0);
  }
}

// Two-spin reduced density matrices (Sec. 3.6), pair p = blockIdx.y with row
// bits (bk, bl): the N/4 groups of rows that differ only in those two bits
// each hold the four rows x_q (q = 2 b_k + b_l), and
// R[q][q'] = sum over groups and columns a of lam_a V[x_q, a] conj(V[x_q', a]).
// Lanes share a group as the magnetisation kernel shares a row (one column
// each); the ten entries q <= q' are summed in FP64 and reduced in the
// workgroup in a fixed order: partials[(p * gridDim.x + block) * 10 + e].
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pair_density(const void *Vp, const double *lam, long long N, int r,
                                                           const int *bits, double2 *partials) {
  using C2 = typename Cplx<T>::type;
  const C2 *V = reinterpret_cast<const C2 *>(Vp);
  const int p = blockIdx.y, bk = bits[2 * p], bl = bits[2 * p + 1];
  const int lo = bk < bl ? bk : bl, hi = bk < bl ? bl : bk;
  const int L = pow2ceil(r), RW = 64 / L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane % L, rsub = lane / L;
  double acc[20];
#pragma unroll
  for (int e = 0; e < 20; ++e) acc[e] = 0.0;
  const long long G = N >> 2;
  if (col < r) {
    const double lm = lam[col];
    const long long per_block = (long long)kWaves * RW;
    for (long long g0 = (long long)blockIdx.x * per_block; g0 < G; g0 += (long long)gridDim.x * per_block) {
      const long long g = g0 + wave * RW + rsub;
      if (g >= G) continue;
      // g with zero bits inserted at lo, then at hi
      long long x = ((g >> lo) << (lo + 1)) | (g & ((1LL << lo) - 1));
      x = ((x >> hi) << (hi + 1)) | (x & ((1LL << hi) - 1));
      C2 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long long xq = x | ((long long)(q >> 1) << bk) | ((long long)(q & 1) << bl);
        v[q] = V[xq * r + col];
      }
      int e = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int q2 = q; q2 < 4; ++q2, ++e) {
          // lam * v_q * conj(v_q2)
          const double ar = v[q].x, ai = v[q].y, br = v[q2].x, bi = v[q2].y;
          acc[2 * e] += lm * (ar * br + ai * bi);
          acc[2 * e + 1] += lm * (ai * br - ar * bi);
        }
    }
  }
  __shared__ double red[kThreads];
  for (int c = 0; c < 20; ++c) {
    red[threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double *out = reinterpret_cast<double *>(partials + ((long long)p * gridDim.x + blockIdx.x) * 10);
      out[c] = red[0];
    }
    __syncthreads();
  }
}

// out[p] (4 x 4 complex, row-major) = scale * (the sum over the pair's
// workgroup partials in block order) + shift * I; the lower triangle by
// Hermitian symmetry.
__global__ void k_pair_reduce(const double2 *partials, int grid, int n_pairs, double scale, double shift,
                              double2 *out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pairs * 10) return;
  const int p = t / 10, e = t % 10;
  double2 s = make_double2(0, 0);
  for (int b = 0; b < grid; ++b) {
    const double2 v = partials[((long long)p * grid + b) * 10 + e];
    s.x += v.x;
    s.y += v.y;
  }
  int q = 0, q2 = 0, k = e;
  while (k >= 4 - q) {
    k -= 4 - q;
    ++q;
  }
  q2 = q + k;
  s = make_double2(scale * s.x + (q == q2 ? shift : 0.0), scale * s.y);
  out[p * 16 + q * 4 + q2] = s;
  if (q2 != q) out[p * 16 + q2 * 4 + q] = make_double2(s.x, -s.y);
}

// LDS of a pass: the four Gram planes [kTile][RP] of the tile, which also
// stage the workgroup's Gram partial sums (up to 3 r^2 complex FP64 values)
// when it stores them -- the larger of the two.
size_t hv_lds(bool fp32, int r) {
  const size_t planes = 4 * (size_t)kTile * pad16(r) * (fp32 ? 4 : 8);
  const size_t stage = 3 * (size_t)r * r * sizeof(double2);
  return planes > stage ? planes : stage;
}

}  // namespace

int hv_partial_splits(int r) {
  (void)r;
  return 1;  // row splits are summed inside the workgroup
}

int nspace_grid(long long N, int r) {
  (void)r;
  const long long tiles = (N + kTile - 1) / kTile;
  long long g = tiles < 1024 ? tiles : 1024;
  if (g >= 8) g &= ~7LL;
  return (int)(g < 1 ? 1 : g);
}

// Complex columns per lane for the H.V pass: 16-byte lanes, E | r, and at
// least four lanes per row where r allows, so that the four waves of a
// 64-row tile all have rows.
int hv_elems_per_lane(bool fp32, int r) {
  int e;
  if (r > 16) e = (fp32 && r % 2 == 0) ? 2 : 1;
  else if (fp32) e = r % 4 == 0 ? 4 : (r % 2 == 0 ? 2 : 1);
  else e = r % 2 == 0 ? 2 : 1;
  while (e > 1 && r / e < 4) e >>= 1;
  return e;
}

size_t hv_lds_bytes(bool fp32, int r) { return hv_lds(fp32, r); }

size_t hv_lds_dyn_extra() { return (size_t)8 * kThreads * sizeof(double); }

template <typename T, int E, bool C, int MI, bool DYN, bool CMP>
static void launch_one_v(const HvArgs &a, size_t lds, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_hv<T, E, C, MI, DYN, CMP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxLds);
    attr = true;
  }
  hipLaunchKernelGGL((k_hv<T, E, C, MI, DYN, CMP>), dim3(a.grid), dim3(kThreads), lds, s, a);
}

template <typename T, int E, bool C, int MI, bool DYN>
static void launch_one(const HvArgs &a, size_t lds, hipStream_t s) {
  if constexpr (MI == 1) {  // compacted gathers: r <= 16
    if (a.compact) {
      launch_one_v<T, E, C, MI, DYN, true>(a, lds, s);
      return;
    }
  }
  launch_one_v<T, E, C, MI, DYN, false>(a, lds, s);
}

template <typename T, int E, bool C, int MI, bool DYN>
static void launch_one_batch(const BatchLaunch &b, int total_wg, size_t lds, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_hv_batch<T, E, C, MI, DYN>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    attr = true;
  }
  hipLaunchKernelGGL((k_hv_batch<T, E, C, MI, DYN>), dim3(total_wg), dim3(kThreads), lds, s, b);
}

// Dispatches on (precision, E, complex coefficients, Gram items per wave,
// schedule).  f is called as f.template operator()<T, E, C, MI, DYN>().  The
// dynamic schedule exists for FP32 storage with one Gram item per wave.
template <typename Fn>
static bool dispatch_hv(bool fp32, int E, bool cplx, bool big, bool dyn, Fn &&f) {
  if (dyn && (!fp32 || big)) return false;
  auto c = [&](auto tag_t, auto tag_e, auto tag_mi) {
    using T = typename decltype(tag_t)::type;
    constexpr int EE = decltype(tag_e)::value, MI = decltype(tag_mi)::value;
    if constexpr (std::is_same_v<T, float> && MI == 1) {
      if (dyn) {
        if (cplx) f.template operator()<T, EE, true, MI, true>();
        else f.template operator()<T, EE, false, MI, true>();
        return;
      }
    }
    if (cplx) f.template operator()<T, EE, true, MI, false>();
    else f.template operator()<T, EE, false, MI, false>();
  };
  struct F32 { using type = float; };
  struct F64 { using type = double; };
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  using I4 = std::integral_constant<int, 4>;
  using I8 = std::integral_constant<int, 8>;
  if (fp32) {
    if (big) {
      if (E == 2) c(F32{}, I2{}, I3{});
      else if (E == 1) c(F32{}, I1{}, I3{});
      else return false;
    } else {
      switch (E) {
        case 8: c(F32{}, I8{}, I1{}); break;
        case 4: c(F32{}, I4{}, I1{}); break;
        case 2: c(F32{}, I2{}, I1{}); break;
        case 1: c(F32{}, I1{}, I1{}); break;
        default: return false;
      }
    }
  } else {
    if (big) {
      if (E != 1) return false;
      c(F64{}, I1{}, I3{});
    } else {
      switch (E) {
        case 4: c(F64{}, I4{}, I1{}); break;
        case 2: c(F64{}, I2{}, I1{}); break;
        case 1: c(F64{}, I1{}, I1{}); break;
        default: return false;
      }
    }
  }
  return true;
}

// Whether `epl` complex columns per lane is a launchable H.V shape for rank r
// in this precision (0 = the default shape, always valid for 1 <= r <= 32).
bool hv_epl_valid(bool fp32, int r, int epl) {
  if (r < 1 || r > kMaxR) return false;
  if (epl == 0) return true;
  if (epl < 0 || r % epl != 0) return false;
  int L = 1;
  while (L * epl < r) L <<= 1;
  if (L > 64) return false;
  const bool big = r > 16;
  if (fp32) return big ? (epl == 1 || epl == 2) : (epl == 1 || epl == 2 || epl == 4 || epl == 8);
  return big ? epl == 1 : (epl == 1 || epl == 2 || epl == 4);
}

// Lanes per row of the tiled pass for E columns per lane.
static int tile_lanes(int r, int E) {
  int L = 1;
  while (L * E < r) L <<= 1;
  return L;
}

size_t hv_tile_lds(bool fp32, int r, int E, int tile_bits, int waves) {
  const size_t cb = fp32 ? 8 : 16;
  const int L = tile_lanes(r, E);
  return ((size_t)1 << tile_bits) * r * cb + (size_t)waves * (64 / L) * r * cb;
}

bool hv_tile_ok(bool fp32, int r, int E, int tile_bits, int waves, long long N, int grid) {
  if (r < 1 || r > 16 || E < 1 || r % E != 0) return false;
  if (fp32 ? (r % 2 != 0 || (E != 2 && E != 4)) : (E != 1 && E != 2)) return false;
  if (waves != 8 && waves != 16) return false;
  const int L = tile_lanes(r, E);
  if (L > 16) return false;  // at least 4 rows per wave for the 16 x 16 x 4 Gram products
  const long long R = 1LL << tile_bits;
  if (tile_bits < 4 || R < (long long)waves * (64 / L) || N % R != 0) return false;
  const long long tiles = N / R;
  if (tiles % 8 != 0 || grid < 8 || grid % 8 != 0 || grid > tiles || grid > kMaxHvGrid) return false;
  const size_t red = 3 * (size_t)r * r * sizeof(double2);  // the final reduction reuses the tile's LDS
  return hv_tile_lds(fp32, r, E, tile_bits, waves) <= (size_t)kMaxTileLds && R * r * (fp32 ? 8 : 16) >= (long long)red;
}

bool prepare_hv(bool fp32, HvArgs &a) {
  if (a.win_bits == 0) {  // default: one window over all row bits, every term, the diagonal
    a.t0 = 0;
    a.t1 = a.n_off;
    a.use_diag = 1;
    a.n_fix = 0;
    a.win_bits = 31;
  }
  if (!hv_epl_valid(fp32, a.r, a.epl)) return false;
  const int E = a.epl > 0 ? a.epl : hv_elems_per_lane(fp32, a.r);
  if (a.tile_bits > 0) {  // tiled pass: one window, static tile schedule, Grams always
    if (a.mode == 2 || a.acc_out || a.n_fix != 0 || a.t0 != 0 || a.t1 != a.n_off ||
        !hv_tile_ok(fp32, a.r, E, a.tile_bits, a.tile_waves, a.N, a.grid) || a.n_local < 0 || a.n_local > a.n_off)
      return false;
    a.epl = E;
    a.lanes = tile_lanes(a.r, E);
    a.terms = fp32 ? (const void *)a.terms32 : (const void *)a.terms64;
    a.diagv = fp32 ? (const void *)a.diag32 : (const void *)a.diag64;
    a.chunks = 0;
    return true;
  }
  if (a.r % E != 0) return false;
  int L = 1;
  while (L * E < a.r) L <<= 1;
  if (L > 64) return false;
  const bool big = a.r > 16;  // three Gram work items per wave above r = 16
  if (fp32 ? (big && E > 2) || (!big && E > 8) : (big && E != 1) || (!big && E > 4)) return false;
  if (a.compact && (big || a.t1 - a.t0 > 64)) return false;
  a.lanes = L;
  a.epl = E;
  a.terms = fp32 ? (const void *)a.terms32 : (const void *)a.terms64;
  a.diagv = fp32 ? (const void *)a.diag32 : (const void *)a.diag64;
  // dynamic schedule with two chunks per workgroup where the partial buffer
  // holds them (one per workgroup otherwise); single window, grid a multiple of 8
  a.chunks = 0;
  const long long tiles = (a.N + kTile - 1) / kTile;
  const bool grams = a.mode != 2 && !a.acc_out;
  const long long cap = grams ? (a.partial_cap > 0 ? a.partial_cap : a.grid) : (1LL << 40);
  if (fp32 && !big && a.sched && a.n_fix == 0 && a.grid >= 8 && a.grid % 8 == 0 && tiles % 8 == 0) {
    for (long long ch = 2LL * a.grid; ch >= a.grid; ch /= 2)
      if (ch <= cap && ch <= tiles) {  // every chunk holds at least one tile
        a.chunks = (int)ch;
        break;
      }
  }
  return true;
}

size_t hv_launch_lds(bool fp32, const HvArgs &a) {
  if (a.tile_bits > 0) return hv_tile_lds(fp32, a.r, a.epl, a.tile_bits, a.tile_waves);
  const size_t base = hv_lds(fp32, a.r) + (a.chunks > 0 ? hv_lds_dyn_extra() : 0);
  if (!a.compact) return base;
  return base + (size_t)(a.t1 - a.t0) * (fp32 ? sizeof(DevTerm<float>) : sizeof(DevTerm<double>));
}

template <typename T, int E, bool C, int W>
static void launch_tile_one(const HvArgs &a, size_t lds, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_hv_tile<T, E, C, W>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxTileLds);
    attr = true;
  }
  hipLaunchKernelGGL((k_hv_tile<T, E, C, W>), dim3(a.grid), dim3(64 * W), lds, s, a);
}

static bool launch_tile(bool fp32, const HvArgs &a, size_t lds, hipStream_t s) {
  const bool c = a.cplx != 0, w16 = a.tile_waves == 16;
  auto go = [&](auto tag_t, auto tag_e) {
    using T = typename decltype(tag_t)::type;
    constexpr int EE = decltype(tag_e)::value;
    if (c) {
      if (w16) launch_tile_one<T, EE, true, 16>(a, lds, s);
      else launch_tile_one<T, EE, true, 8>(a, lds, s);
    } else {
      if (w16) launch_tile_one<T, EE, false, 16>(a, lds, s);
      else launch_tile_one<T, EE, false, 8>(a, lds, s);
    }
  };
  struct F32 { using type = float; };
  struct F64 { using type = double; };
  if (fp32) {
    if (a.epl == 4) go(F32{}, std::integral_constant<int, 4>{});
    else if (a.epl == 2) go(F32{}, std::integral_constant<int, 2>{});
    else return false;
  } else {
    if (a.epl == 2) go(F64{}, std::integral_constant<int, 2>{});
    else if (a.epl == 1) go(F64{}, std::integral_constant<int, 1>{});
    else return false;
  }
  return true;
}

int launch_hv(bool fp32, const HvArgs &a0, hipStream_t s) {
  HvArgs a = a0;
  if (!prepare_hv(fp32, a)) return 0;
  const size_t lds = hv_launch_lds(fp32, a);
  a.cmp_off = (int)(hv_lds(fp32, a.r) + (a.chunks > 0 ? hv_lds_dyn_extra() : 0));
  if (a.tile_bits > 0) return launch_tile(fp32, a, lds, s) ? a.grid : 0;
  const bool ok = dispatch_hv(fp32, a.epl, a.cplx != 0, a.r > 16, a.chunks > 0,
                                [&]<typename T, int E, bool C, int MI, bool DYN>() {
                                  launch_one<T, E, C, MI, DYN>(a, lds, s);
                                });
  return ok ? (a.chunks > 0 ? a.chunks : a.grid) : 0;
}

int hv_resident_per_cu(bool fp32, const HvArgs &a0, bool *dynamic) {
  HvArgs a = a0;
  *dynamic = false;
  if (!prepare_hv(fp32, a) || a.tile_bits > 0) return 0;
  const size_t lds = hv_launch_lds(fp32, a);
  int n = 0;
  const bool ok = dispatch_hv(fp32, a.epl, a.cplx != 0, a.r > 16, a.chunks > 0,
                              [&]<typename T, int E, bool C, int MI, bool DYN>() {
                                const void *f = (const void *)k_hv<T, E, C, MI, DYN, false>;
                                if constexpr (MI == 1)
                                  if (a.compact) f = (const void *)k_hv<T, E, C, MI, DYN, true>;
                                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kThreads, lds) != hipSuccess)
                                  n = 0;
                              });
  *dynamic = ok && a.chunks > 0;
  return ok ? n : 0;
}

bool launch_hv_batch(bool fp32, int epl, bool cplx, bool big, bool dyn, const BatchLaunch &b, int total_wg,
                       size_t lds, hipStream_t s) {
  return dispatch_hv(fp32, epl, cplx, big, dyn, [&]<typename T, int E, bool C, int MI, bool DYN>() {
    launch_one_batch<T, E, C, MI, DYN>(b, total_wg, lds, s);
  });
}

void launch_diag_values(const DevDiagTerm *diag, int n_diag, long long N, double *d64, float *d32, hipStream_t s) {
  long long blocks = (N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_diag_values, dim3((unsigned)blocks), dim3(256), 0, s, diag, n_diag, N, d64, d32);
}

void launch_combine(bool fp32, const void *const *blocks, int nblocks, const double2 *C, void *out,
                    long long N, int r, int grid, hipStream_t s, const double *skip, const void *lo_in,
                    void *lo_out) {
  CombineArgs a;
  a.skip = skip;
  a.lo_in = fp32 ? lo_in : nullptr;
  a.lo_out = fp32 ? lo_out : nullptr;
  for (int i = 0; i < kMaxBlocks; ++i) a.blocks[i] = i < nblocks ? blocks[i] : nullptr;
  a.nb = nblocks;
  a.C = C;
  a.out = out;
  a.N = N;
  a.r = r;
  a.grid = grid;
  const int RP = pad16(r);
  const size_t lds = (size_t)(2 * nblocks * RP * RP) * (fp32 ? 4 : 8);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_combine<float, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    (void)hipFuncSetAttribute((const void *)k_combine<float, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    (void)hipFuncSetAttribute((const void *)k_combine<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    (void)hipFuncSetAttribute((const void *)k_combine<double, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    attr = true;
  }
  if (fp32) {
    if (RP == 16) hipLaunchKernelGGL((k_combine<float, 16>), dim3(grid), dim3(kThreads), lds, s, a);
    else hipLaunchKernelGGL((k_combine<float, 32>), dim3(grid), dim3(kThreads), lds, s, a);
  } else {
    if (RP == 16) hipLaunchKernelGGL((k_combine<double, 16>), dim3(grid), dim3(kThreads), lds, s, a);
    else hipLaunchKernelGGL((k_combine<double, 32>), dim3(grid), dim3(kThreads), lds, s, a);
  }
}

void launch_combine_batch(bool fp32, int RP, int nblocks, const BatchLaunch &b, int total_wg, hipStream_t s) {
  const size_t lds = (size_t)(2 * nblocks * RP * RP) * (fp32 ? 4 : 8);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_combine_batch<float, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    (void)hipFuncSetAttribute((const void *)k_combine_batch<float, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    (void)hipFuncSetAttribute((const void *)k_combine_batch<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    (void)hipFuncSetAttribute((const void *)k_combine_batch<double, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    attr = true;
  }
  if (fp32) {
    if (RP == 16) hipLaunchKernelGGL((k_combine_batch<float, 16>), dim3(total_wg), dim3(kThreads), lds, s, b);
    else hipLaunchKernelGGL((k_combine_batch<float, 32>), dim3(total_wg), dim3(kThreads), lds, s, b);
  } else {
    if (RP == 16) hipLaunchKernelGGL((k_combine_batch<double, 16>), dim3(total_wg), dim3(kThreads), lds, s, b);
    else hipLaunchKernelGGL((k_combine_batch<double, 32>), dim3(total_wg), dim3(kThreads), lds, s, b);
  }
}

void launch_reduce_batch(const BatchLaunch &b, int total_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_batch, dim3(total_wg), dim3(256), 0, s, b);
}

void launch_reduce(const double2 *partials, int count, int len, double2 *out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(len), dim3(256), 0, s, partials, count, len, out);
}

void launch_split(const double2 *src, float2 *hi, void *lo, long long n, hipStream_t s) {
  const long long blocks = std::max<long long>(1, std::min<long long>(4096, (n + 255) / 256));
  hipLaunchKernelGGL(k_split_d2f, dim3((unsigned)blocks), dim3(256), 0, s, src, hi, (ushort2 *)lo, n);
}

void launch_merge(const float2 *hi, const void *lo, double2 *dst, long long n, hipStream_t s) {
  const long long blocks = std::max<long long>(1, std::min<long long>(4096, (n + 255) / 256));
  hipLaunchKernelGGL(k_merge_f2d, dim3((unsigned)blocks), dim3(256), 0, s, hi, (const ushort2 *)lo, dst, n);
}

void launch_convert(bool to_fp32, const void *src, void *dst, long long n, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  if (to_fp32)
    hipLaunchKernelGGL(k_convert_d2f, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const double2 *)src, (float2 *)dst, n);
  else
    hipLaunchKernelGGL(k_convert_f2d, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float2 *)src, (double2 *)dst, n);
}

void launch_permute(bool fp32, const void *src, void *dst, long long N, int r, const int *pos, int n, bool inverse,
                    hipStream_t s) {
  PermArgs pa{};
  pa.n = n;
  for (int i = 0; i < n; ++i) pa.pos[i] = (unsigned char)pos[i];
  long long blocks = (N * r + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (fp32)
    hipLaunchKernelGGL(k_permute_rows<float2>, dim3((unsigned)blocks), dim3(256), 0, s, (const float2 *)src,
                       (float2 *)dst, N, r, pa, (int)inverse);
  else
    hipLaunchKernelGGL(k_permute_rows<double2>, dim3((unsigned)blocks), dim3(256), 0, s, (const double2 *)src,
                       (double2 *)dst, N, r, pa, (int)inverse);
}

void launch_pair_density(bool fp32, const void *V, const double *lam, long long N, int r, const int *bits,
                         int n_pairs, int grid, double2 *partials, double2 *out, double scale, double shift,
                         hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_pair_density<float>, dim3(grid, n_pairs), dim3(kThreads), 0, s, V, lam, N, r, bits, partials);
  else
    hipLaunchKernelGGL(k_pair_density<double>, dim3(grid, n_pairs), dim3(kThreads), 0, s, V, lam, N, r, bits,
                       partials);
  hipLaunchKernelGGL(k_pair_reduce, dim3((n_pairs * 10 + 255) / 256), dim3(256), 0, s, (const double2 *)partials,
                     grid, n_pairs, scale, shift, out);
}

void launch_magnetization(bool fp32, const void *V, const double *lam, long long N, int r, int n,
                          double2 *partials, int grid, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_magnet<float>, dim3(grid), dim3(kThreads), 0, s, V, lam, N, r, n, partials);
  else
    hipLaunchKernelGGL(k_magnet<double>, dim3(grid), dim3(kThreads), 0, s, V, lam, N, r, n, partials);
}

}  // namespace lrei
