// Internal declarations shared by the LREI library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lrei.h"

namespace lrei {

// ---------------------------------------------------------------------------
// Hamiltonian term tables (built on the host from the Pauli-form couplings).
//
// Y[x] = d(x) X[x] + sum_t c_t[b_a(x) + 2 b_b(x)] X[x ^ mask_t]
//   d(x) = sum_k w_k (1 - 2 (b_{i_k}(x) xor b_{j_k}(x)))   (j_k = 31 for a field)
// b_s(x) is bit s of x.  A coefficient table is indexed by the bits of the
// destination row x at sites a, b (b = a for a one-site term).
// ---------------------------------------------------------------------------
struct OffTerm {
  uint32_t mask;
  uint32_t sa, sb;
  double re[4], im[4];
};
struct DiagTerm {
  uint32_t si, sj;
  double w;
};

struct TermTable {
  std::vector<OffTerm> off;
  std::vector<DiagTerm> diag;
  double gershgorin = 0.0;  // bound on the spectral radius of H
  double spread = 0.0;      // sqrt(Tr(H^2) / N): the spectral width of H seen by a random state
};

// Builds the term table; returns false with `err` set on invalid input.
bool build_terms(int n, int n_bonds, const int32_t *bond_ij, const double *bond_J,
                 const double *site_h, TermTable &out, std::string &err);

// Device-side term record in the storage precision T of the pass.
template <typename T>
struct DevTerm {
  // act: bit q set when the coefficient for destination bits q = b_sa + 2 b_sb
  // is non-zero (the rows for which the term gathers a partner)
  uint32_t mask, sa, sb, act;
  T re[4], im[4];
};
using DevOffTerm = DevTerm<double>;
struct DevDiagTerm {
  uint32_t si, sj;
  double w;
};

// Maximum supported sizes.
constexpr int kMaxR = 32;
constexpr int kMaxStages = 5;               // RK4, and the error stage of its embedded pair
constexpr int kMaxBlocks = 8;               // Krylov blocks in the projected basis
constexpr int kMaxDim = kMaxBlocks * kMaxR; // projected dimension bound

// Launch helpers implemented in nspace.hip / small.hip.
struct HvArgs {
  const void *Pcur;    // P_j
  void *Pnext;         // P_{j+1}
  const DevTerm<double> *terms64;  // off-diagonal terms
  const DevTerm<float> *terms32;
  const double *diag64;            // d(x) per row
  const float *diag32;
  int n_off;
  int cplx;             // some coefficient has a non-zero imaginary part
  int epl;              // complex columns per lane (0: default)
  int lanes;            // set by the launcher
  const void *terms, *diagv;  // set by the launcher
  // sweep over a window of row bits (default: one window of all bits, all terms)
  int t0, t1;                   // off-diagonal terms of this sweep
  int use_diag;                 // add d(x) X[x]
  const void *acc_in;           // add this partial sum (or nullptr)
  int acc_out;                  // write the raw sum, no combination, no Grams
  int win_bits, n_fix;          // window bits (traversal order) and fixed bits
  unsigned char win_pos[32], fix_pos[32];
  long long N;
  int r;
  // Krylov block recurrence P_{j+1} = alpha (H P_j - P_j diag(colshift)),
  // colshift[c] the shift of column c of block j (nullptr: all zero)
  double alpha;
  const double *colshift;
  int mode;             // 0: first block (Grams P0*P0, P0*P1, P1*P1), 1: later blocks
                        // (Grams P*P+, P+*P+), 2: plain Y = alpha H X (no Grams)
  double2 *partials;    // Gram partial sums, entry-major [entry][slot]
  int grid;
  // dynamic tile schedule: counters (16 ints, zero between launches; nullptr:
  // static schedule) and the number of partial-sum slots the buffer holds
  int *sched;
  int partial_cap;
  int chunks;           // set by prepare_hv: Gram partial slots used (0: one per workgroup)
  const double *skip;   // the pass does nothing while *skip != 0 (nullptr: always runs)
  // tiled pass (tile_bits > 0): workgroups of 64 * tile_waves threads hold
  // 2^tile_bits rows of P_j in LDS; terms [0, n_local) flip bits below
  // tile_bits only (the term table is sorted by highest flipped bit)
  int tile_bits;
  int tile_waves;
  int n_local;
  // compacted gathers (untiled pass, r <= 16, at most 64 terms per launch):
  // each row walks only its active terms; the term records sit in LDS at
  // byte offset cmp_off (set by the launcher)
  int compact;
  int cmp_off;
};

// Launches one H.V pass; returns the number of Gram partial slots written
// (the reduction's count), 0 if the shape is unsupported.
int launch_hv(bool fp32, const HvArgs &a, hipStream_t s);
bool hv_epl_valid(bool fp32, int r, int epl);
// Fills the launcher-set fields of a (columns per lane, lanes, table pointers,
// the default single window); false if the shape is unsupported.
bool prepare_hv(bool fp32, HvArgs &a);
size_t hv_lds_bytes(bool fp32, int r);
size_t hv_launch_lds(bool fp32, const HvArgs &a);  // dynamic LDS of a prepared pass
// Workgroups of the (unprepared) pass a that fit on one CU at once, 0 if the
// shape is unsupported or is a tiled pass; *dynamic tells whether the pass
// takes the dynamic chunk schedule.
int hv_resident_per_cu(bool fp32, const HvArgs &a, bool *dynamic);

// Launch tables of a batched kernel (many independent jobs in one launch):
// workgroup w runs job wg_job[w] as that job's workgroup w - job_wg0[job].
// jobs points to a device array of the kernel's per-job argument records.
struct BatchLaunch {
  const void *jobs;
  const int *wg_job;
  const int *job_wg0;
};
// Batched Krylov passes: every job is a HvArgs prepared by prepare_hv
// with the same precision, columns per lane epl, complex flag and r > 16 flag.
bool launch_hv_batch(bool fp32, int epl, bool cplx, bool big, bool dyn, const BatchLaunch &b, int total_wg,
                       size_t lds, hipStream_t s);
size_t hv_lds_dyn_extra();  // LDS added by the dynamic schedule (Gram accumulators)
// Basis combination out = [B_0 ... B_{nb-1}] C (nspace.hip).
struct CombineArgs {
  const void *blocks[kMaxBlocks];
  int nb;
  const double2 *C;
  void *out;
  long long N;
  int r, grid;
  const double *skip;  // nothing is written while *skip != 0 (nullptr: always runs)
  // compensated FP32 state (FP32 blocks only; nullptr: plain): the state is
  // blocks[0] + lo_in (lo as bfloat16 pairs); the kernel forms
  // blocks[0] + lo_in + [B_0..B_{nb-1}] (C - [I; 0]) in FP64 and writes it split
  // again as out + lo_out
  const void *lo_in;
  void *lo_out;
};
// Batched combinations: every job has the same nb and padded width RP (16 or 32).
void launch_combine_batch(bool fp32, int RP, int nblocks, const BatchLaunch &b, int total_wg, hipStream_t s);
// Batched reductions: job q sums q.count partials per entry into q.out; one
// workgroup per entry.
struct ReduceJob {
  const double2 *in;
  int count;
  double2 *out;
};
void launch_reduce_batch(const BatchLaunch &b, int total_wg, hipStream_t s);
// Compensated FP32 state: hi = fl32(v), lo = bf16(v - hi) as (re, im) pairs of
// uint16 (split); v = hi + lo (merge).  hi + lo holds v to ~2^-33 relative.
void launch_split(const double2 *src, float2 *hi, void *lo, long long n, hipStream_t s);
void launch_merge(const float2 *hi, const void *lo, double2 *dst, long long n, hipStream_t s);
void launch_diag_values(const DevDiagTerm *diag, int n_diag, long long N, double *d64, float *d32, hipStream_t s);
int hv_elems_per_lane(bool fp32, int r);
void launch_combine(bool fp32, const void *const *blocks, int nblocks, const double2 *C, void *out,
                    long long N, int r, int grid, hipStream_t s, const double *skip = nullptr,
                    const void *lo_in = nullptr, void *lo_out = nullptr);
void launch_reduce(const double2 *partials, int count, int len, double2 *out, hipStream_t s);
void launch_convert(bool to_fp32, const void *src, void *dst, long long n_complex, hipStream_t s);
// dst rows = src rows moved by the site -> bit map pos (forward) or gathered back (inverse).
void launch_permute(bool fp32, const void *src, void *dst, long long N, int r, const int *pos, int n, bool inverse,
                    hipStream_t s);
// Initial state from a factor A (N x m, device, natural row order): Gram
// partials (grid x m(m+1)/2) and the one-workgroup eigensolve giving C
// (m x m), lam (m) and info[0] = rank; then V = A C[:, :r].
void launch_factor_eig(const double2 *A, long long N, int m, double2 *partials, int grid, double2 *C, double *lam,
                       int *info, hipStream_t s);
void launch_factor_apply(const double2 *A, long long N, int m, const double2 *C, int r, double2 *V, hipStream_t s);

// Two-spin reduced density matrices of n_pairs (bit k, bit l) pairs (bits:
// device, 2 per pair) into out (device, n_pairs x 16 double2), each
// scale * R + shift * I; partials: at least n_pairs * grid * 10 double2.
void launch_pair_density(bool fp32, const void *V, const double *lam, long long N, int r, const int *bits,
                         int n_pairs, int grid, double2 *partials, double2 *out, double scale, double shift,
                         hipStream_t s);
void launch_magnetization(bool fp32, const void *V, const double *lam, long long N, int r, int n,
                          double2 *partials, int grid, hipStream_t s);
int nspace_grid(long long N, int r);
constexpr int kMaxHvGrid = 2048;  // largest H.V launch the partial-sum buffer holds
constexpr int kMaxTileLds = 160 * 1024;  // LDS of one workgroup on gfx950
// Tiled pass: LDS bytes of a launch shape, and whether the shape is launchable
// (rank, columns per lane, tile bits, waves, rows, workgroups).
size_t hv_tile_lds(bool fp32, int r, int E, int tile_bits, int waves);
bool hv_tile_ok(bool fp32, int r, int E, int tile_bits, int waves, long long N, int grid);

// Generic block pass (blocks.hip): out_o = sum_i in_i C[i, o] and Gram
// products over the listed (a, b) pairs of [inputs..., outputs...], r <= 16.
constexpr int kMaxIoBlocks = 10;
constexpr int kMaxGrams = 32;
struct BlocksArgs {
  const void *in[kMaxIoBlocks];
  void *out[kMaxIoBlocks];
  int n_in, n_out;
  const double2 *C;      // row (i * r + a), column (o * r + b), leading dimension ldc
  int ldc;
  signed char ga[kMaxGrams], gb[kMaxGrams];
  int n_gram;
  double2 *partials;     // [n_gram * r * r][grid], entry-major
  long long N;
  int r, grid;
};
bool launch_blocks(bool fp32, const BlocksArgs &a, hipStream_t s);
int blocks_grid(long long N);
size_t blocks_lds(bool fp32, int nin, int nout, int r);

// Site -> row-bit order of the internal storage (site_order.cpp): pos[site]
// is the row bit that holds the site.
std::vector<int> choose_site_order(int n, int n_bonds, const int32_t *bond_ij);
// The same for the tiled H.V pass: the k_cluster-site set with the most inner
// bonds in the low bits, greedy growth order within and after it.
std::vector<int> choose_site_order_cluster(int n, int n_bonds, const int32_t *bond_ij, int k_cluster);
constexpr int kClusterBits = 10;  // tile rows of the tiled pass at r = 16 in FP32: 2^10

// Device-resident state of the step-size controller (adaptive stepping, one
// double each).  The stage that forms the error estimate reads the step from
// kCtlH, decides, and writes the next step; every kernel of an attempt does
// nothing while kCtlSkip is set (copied from kCtlDone | kCtlFailed when the
// attempt begins).
enum CtlSlot {
  kCtlH = 0,         // step of the next attempt
  kCtlT,             // time reached (accepted steps)
  kCtlTEnd,          // time to reach
  kCtlTol,           // tolerance on the error estimate
  kCtlHMin,
  kCtlHMax,
  kCtlErr,           // estimate of the last attempt
  kCtlAccepted,
  kCtlRejected,
  kCtlDone,          // t_end reached
  kCtlFailed,        // rejected at h <= h_min
  kCtlSkip,
  kCtlAfterReject,   // the last attempt was rejected (no growth of h next)
  kCtlErrMax,        // largest estimate among accepted steps
  kCtlAttempts,      // attempts that ran
  kCtlLen = 16
};
void launch_attempt_begin(double *ctl, hipStream_t s);

// Parameters of the projected (small-space) step kernel.
struct SmallRkParams {
  int r, s, nblocks;      // nblocks = s + 1
  int model;              // 0 qLL, 1 qLLG
  int householder_mode;
  int max_sweeps;
  int warm;
  int lds_elems;          // double2 capacity of the dynamic LDS matrix
  double kappa, hbar, h, eig_tol;
  double warm_tol;        // relative subspace residual at which the warm-started eigensolve stops
  double beta;            // Krylov recurrence P_{j+1} = beta (H P_j - P_j diag(D_j)), D_j in SmallWs.shifts
  double a[kMaxStages][kMaxStages];
  double b[kMaxStages];
  double lam[kMaxR];
  // learned start rotation: network parameters (LREI_WARM_LEARNED) and the
  // training-sample recorder (rec == nullptr: off)
  const float *net;
  float *rec;
  int *rec_count;
  int rec_cap;
  // adaptive stepping (ctl == nullptr: fixed step h): controller state, the
  // stage that forms the error estimate (s - 1, or s for a pair that also
  // weights the right-hand side at the new state; that stage then forms no
  // stage matrix), the error weights b - b_hat over f_0 .. f_{err_stage} and
  // the order q of the embedded solution
  double *ctl;
  int err_stage;
  int order_low;
  double e[kMaxStages];
};

// Device layout of the small workspace (doubles).
struct SmallWs {
  double2 *meas;     // [kMaxStages][3][r*r]: measured Grams per pass
  double2 *gamma;    // [D*D] Gram of the Krylov basis
  double2 *R;        // [D*D] Cholesky factor
  double2 *Rinv;     // [D*D]
  double2 *Hh;       // [D*D] projected Hamiltonian
  double2 *work;     // [8*D*D] scratch
  double2 *stage;    // [kMaxStages][3][D*r] u, z, w per stage
  double2 *Cfin;     // [D*r] combination coefficients for the new V
  double *flags;     // [D] directions dropped as dependent
  double *warm_skip; // [2][kMaxStages] steps left before stage j tries the warm start again,
                     // and the span of stage j's last skip (doubled on each rejection in a row)
  double *shifts;    // [kMaxBlocks][r] column shifts D_j of the Krylov recurrence (read by the
                     // passes; refreshed from the measured Rayleigh quotients by the step's last stage)
  double *stats;     // [32]
};

// LDS arena of the projected-step kernel: an 80 x 80 Cholesky factor, or the
// packed stage matrix plus inverse-iteration scratch (the largest problems kept
// in LDS; bigger ones fall back to global memory).
constexpr int kSmallLdsElems = 80 * 80;
constexpr int kSmallLdsBytes = kSmallLdsElems * 16;
// LDS capacity (double2 elements) to request for a projected dimension D.
inline int small_lds_elems(int D, int r) {
  const int sl = r <= 16 ? 16 : 32;
  int need = D * D;
  const int tri = D * (D + 1) / 2 + 2 * D * sl;
  if (tri > need) need = tri;
  if (3 * D * r > need) need = 3 * D * r;
  if (2 * r * r > need) need = 2 * r * r;
  return need < kSmallLdsElems ? need : kSmallLdsElems;
}
// LDS capacity (double2 elements) of a basis extension: its Cholesky factor
// and triangular inverse stage at most 2 (2r)^2 elements (the first stage's two
// blocks), so it asks for no more than that and fits on a CU beside more
// workgroups of a running pass than a stage does.
__host__ __device__ inline int small_basis_lds_elems(int lds_elems, int r) {
  const int need = 8 * r * r;
  return need < lds_elems ? need : lds_elems;
}
void launch_small_rk(const SmallRkParams &p, const SmallWs &ws, hipStream_t s);
// Stage j of an RK step in two launches: the basis extension (needs the Grams
// of pass j), then the stage (needs the extension and stage j - 1).
void launch_small_rk_basis(const SmallRkParams &p, const SmallWs &ws, int j, hipStream_t s);
void launch_small_rk_stage(const SmallRkParams &p, const SmallWs &ws, int j, hipStream_t s);
// Stage j of many independent projected steps, one workgroup per job;
// lds_elems is the largest p.lds_elems among the jobs.
void launch_small_rk_stage_batch(const SmallRkParams *p, const SmallWs *ws, int n_jobs, int lds_elems, int j,
                                 hipStream_t s);

// Projected AB step / history update (small.hip).
constexpr int kMaxAb = 4;  // AB4
struct SmallAbParams {
  int r, m_ab;             // rank, AB order m
  int mode;                // 0: history update after an RK start-up step, 1: AB step
  int nU, qx;              // history basis blocks U, new blocks X (and Y)
  int x_v0, x_hv, x_vnew;  // X block holding V_k (-1: V_k is in U), H V_k (scaled), V_{k+1} (mode 0)
  double hv_scale;         // H V_k = hv_scale * X[x_hv]
  int npairs_keep;         // older history pairs carried into the new basis (<= m - 2)
  int model, householder_mode, lds_elems;
  int max_sweeps;          // Jacobi sweep limit of the Lowdin step
  double kappa, hbar, h;
  double eig_tol;          // Jacobi tolerance of the Lowdin step
  double bcoef[kMaxAb];
  double lam[kMaxR];
};
struct SmallAbWs {
  const double2 *UUg;        // Grams of the U blocks, pairs i <= j in row order, r x r each
  const double2 *c1g;        // U_i* X_q, index i * qx + q
  const double2 *gBg;        // U_i* Y_q (index i * qx + q), then Y_q* Y_q' (q <= q', row order)
  const double2 *coords_in;  // U-coordinates: V_k, then (V_{k-l}, H V_{k-l}) pairs, each nU r x r
  double2 *coords_out;       // the same for the new basis (qn x r each)
  double2 *Cc;               // [(nU + qx) r] x [qn + r]: new U blocks, then V_{k+1}
  double2 *work;
  double *stats;
};
void launch_small_ab(const SmallAbParams &p, const SmallAbWs &ws, hipStream_t s);
size_t small_ab_work_elems(int D, int qn, int r);
void launch_ab_cgs_coef(const double2 *c1g, int nU, int qx, int r, double2 *C, hipStream_t s);
int hv_partial_splits(int r);

}  // namespace lrei

// Device address of a model's parameters (learned.hip).
extern "C" const void *lrei_net_device_params(const lrei_net *m);
