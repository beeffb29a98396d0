// C ABI of the LREI library: context management, validation, and the step
// driver that sequences the N-space passes and the projected step kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <tuple>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "host_common.h"
#include "lrei_internal.h"

using namespace lrei;

namespace {

constexpr uint64_t kStateMagic = 0x4c52454953543031ull;  // "LREIST01"

// Device scratch of lrei_apply_hamiltonian_noalloc: the input and the product
// in the internal site order, 2 N r complex128 values at most.  Each GPU the
// library runs on holds its own copy until the process ends; host code never
// uses the array's name as an address, only the per-device address that
// hipGetSymbolAddress returns (resolved when a context is created).
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
void *g_scratch_addr[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Resolves this device's address of the scratch array (hip_device current).
hipError_t resolve_scratch(int hip_device) {
  if (hip_device < 0 || hip_device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[hip_device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) g_scratch_addr[hip_device] = ptr;
  return e == hipSuccess && !ptr ? hipErrorInvalidSymbol : e;
}

}  // namespace

struct lrei_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // the projected-step stages run on a second stream, each after its pass;
  // their basis extensions on a third, each after its pass
  hipStream_t side = nullptr, basis = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join_basis = nullptr;
  hipEvent_t ev_pass[kMaxStages] = {}, ev_basis[kMaxStages] = {};
  lrei_options opt{};
  std::string err;

  // Hamiltonian
  bool have_h = false;
  std::vector<int> site_pos;     // physical site -> row bit of the internal storage order
  int n = 0;
  long long N = 0;
  double hbar = 1.0;
  TermTable terms;
  DevTerms dt;                    // device term tables and d(x) per row
  int epl = 0;                    // H.V columns per lane (0: default)
  int hv_grid = 0;                // H.V workgroups per launch (0: default)
  int hv_tile_bits = 0;           // tiled pass: 2^bits rows per LDS tile (0: untiled)
  int hv_tile_waves = 16;         // tiled pass: waves per workgroup
  int hv_compact = 0;             // untiled pass with compacted gathers
  int num_cus = 0;                // compute units of the device
  // grid of the passes that overlap stage kernels, cached for one pass shape
  struct {
    int grid = -1, epl = -1, r = -1, compact = -1, fp32 = -1, tile_bits = -1, sweeps = -1, result = 0;
  } overlap;
  // H.V sweep plan: each sweep applies the terms whose flip masks lie in its
  // window of row bits (one sweep = all bits, all terms)
  struct HvSweep {
    std::vector<int> win, fix;
    int t0 = 0, t1 = 0;
  };
  int hv_w = 0;                   // window bits (0: one sweep)
  std::vector<HvSweep> sweeps;
  DevBuf acc;                     // partial sums between sweeps
  DevBuf sched;                   // H.V tile-scheduling counters (16 ints, zero between launches)
  bool hv_launch_failed = false;  // an H.V launch was refused (shape invalid for the rank)

  // weight p of the maximally mixed part: the state is p I / N + (1 - p) V Lambda V*
  double mix_p = 0.0;

  // learned start rotation: attached network, training-sample recorder
  const float *net = nullptr;
  int net_r = 0;
  float *rec = nullptr;
  int rec_cap = 0;
  DevBuf rec_count;               // one int

  // state
  bool have_rho = false;
  int r = 0;
  std::vector<double> lam;
  bool fp32 = false;
  DevBuf blocks[kMaxStages + 1];
  DevBuf save;       // state at the start of a step call (rollback)
  // LREI_MIXED: the state is the compensated pair blocks[0] (FP32) + lo
  // (bfloat16 pairs, 4 bytes per element)
  DevBuf lo, save_lo;
  size_t lo_bytes() const { return (size_t)N * r * 4; }
  DevBuf partials;
  DevBuf ws_buf;
  DevBuf stats_buf;
  DevBuf lam_dev;
  SmallWs ws{};
  int grid = 1;
  int64_t steps_done = 0;
  lrei_stats stats{};

  // ABm history (Sec. 3.8): orthonormal basis U of the recent supports and
  // H-images, its Gram products and the U-coordinates of the history
  struct AbState {
    bool valid = false;
    int scheme = 0, m = 0, model = -1;
    double dt = 0, kappa = 0;
    int count = 0;   // steps of this AB run so far (start-up steps included)
    int nU = 0;      // blocks in U
    int npairs = 0;  // history pairs held in coordinates
    int cur = 0;     // current U set / coordinate buffer
  } ab;
  DevBuf ab_U[2][2 * kMaxAb - 1];
  DevBuf ab_coords[2], ab_UUg, ab_c1g, ab_gBg, ab_Cb, ab_Cc, ab_work, ab_partials;
  int ab_grid = 1;

  // adaptive stepping: device-resident controller state (kCtlLen doubles);
  // pass_skip is handed to the N-space passes of an attempt being enqueued
  DevBuf ctl;
  const double *pass_skip = nullptr;

  // captured step graph (g_dt < 0: an adaptive attempt)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int g_model = -1, g_scheme = -1;
  double g_dt = 0, g_kappa = 0;

  lrei_status fail(lrei_status st, const std::string &m) {
    err = m;
    return st;
  }
  size_t elem() const { return fp32 ? sizeof(float2) : sizeof(double2); }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    g_model = g_scheme = -1;
  }
};

namespace {

lrei_status check_hip(lrei_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return LREI_OK;
  return c->fail(LREI_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                        \
  do {                                                      \
    lrei_status _st = check_hip(ctx, (expr), #expr);        \
    if (_st != LREI_OK) return _st;                         \
  } while (0)

// Allocates every buffer the state of rank r needs.
lrei_status alloc_state(lrei_ctx *ctx, int r, bool fp32) {
  const size_t el = fp32 ? sizeof(float2) : sizeof(double2);
  const size_t blk = (size_t)ctx->N * r * el;
  for (int i = 0; i <= kMaxStages; ++i)
    if (!ctx->blocks[i].ensure(blk)) return ctx->fail(LREI_E_NOMEM, "device allocation of Krylov blocks failed");
  if (!ctx->save.ensure(blk)) return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  const size_t lob = (size_t)ctx->N * r * 4;  // bfloat16 (re, im) per element
  if (fp32 && (!ctx->lo.ensure(lob) || !ctx->save_lo.ensure(lob)))
    return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  if (!ctx->acc.ensure(blk)) return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  ctx->grid = nspace_grid(ctx->N, r);
  if (ctx->hv_grid <= 0) ctx->hv_grid = ctx->grid;
  const size_t pcount = (size_t)kMaxHvGrid * hv_partial_splits(r) * 3 * r * r;
  if (!ctx->partials.ensure(pcount * sizeof(double2) + 2 * kMaxHvGrid * sizeof(double2)))
    return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  const int D = (kMaxStages + 1) * r;
  const size_t ws_elems = (size_t)kMaxStages * 3 * r * r      // meas
                          + 4 * (size_t)D * D                  // gamma, R, Rinv, Hh
                          + (4 * (size_t)D * r + 2 * (size_t)D * D + 4 * (size_t)r * r)  // work
                          + (size_t)kMaxStages * 3 * D * r     // stage
                          + (size_t)D * r                      // Cfin
                          + (size_t)D                          // flags (as complex slots)
                          + (size_t)kMaxStages                 // warm_skip: 2 kMaxStages doubles
                          + (size_t)kMaxBlocks * r;            // column shifts (as complex slots)
  if (!ctx->ws_buf.ensure(ws_elems * sizeof(double2))) return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  if (!ctx->stats_buf.ensure(kStatsLen * sizeof(double))) return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  if (!ctx->lam_dev.ensure(kMaxR * sizeof(double))) return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  double2 *w = (double2 *)ctx->ws_buf.p;
  ctx->ws.meas = w; w += (size_t)kMaxStages * 3 * r * r;
  ctx->ws.gamma = w; w += (size_t)D * D;
  ctx->ws.R = w; w += (size_t)D * D;
  ctx->ws.Rinv = w; w += (size_t)D * D;
  ctx->ws.Hh = w; w += (size_t)D * D;
  ctx->ws.work = w; w += 4 * (size_t)D * r + 2 * (size_t)D * D + 4 * (size_t)r * r;
  ctx->ws.stage = w; w += (size_t)kMaxStages * 3 * D * r;
  ctx->ws.Cfin = w; w += (size_t)D * r;
  ctx->ws.flags = (double *)w; w += (size_t)D;
  ctx->ws.warm_skip = (double *)w; w += (size_t)kMaxStages;
  ctx->ws.shifts = (double *)w;
  ctx->ws.stats = (double *)ctx->stats_buf.p;
  return LREI_OK;
}

// Scale of the Krylov recurrence P_{j+1} = beta (H P_j - P_j D_j): the
// inverse spectral width sqrt(N / Tr(H^2)), so that the blocks keep norms of
// order one.  The space spanned does not depend on it.
double krylov_beta(const lrei_ctx *ctx) { return ctx->terms.spread > 0 ? 1.0 / ctx->terms.spread : 1.0; }

// Off-diagonal terms that flip only bits below k (a prefix of the table,
// which is sorted by the highest bit a term flips).
int local_terms(const lrei_ctx *ctx, int k) {
  int c = 0;
  for (const auto &t : ctx->terms.off)
    if ((t.mask >> k) == 0) ++c;
    else break;
  return c;
}

// Hamiltonian tables of an H.V pass.
void hv_args(lrei_ctx *ctx, HvArgs &a) {
  a.terms64 = (const DevTerm<double> *)ctx->dt.off64.p;
  a.terms32 = (const DevTerm<float> *)ctx->dt.off32.p;
  a.diag64 = (const double *)ctx->dt.d64.p;
  a.diag32 = (const float *)ctx->dt.d32.p;
  a.n_off = ctx->dt.n_off;
  a.cplx = ctx->dt.cplx;
  a.epl = ctx->epl;
  a.sched = (int *)ctx->sched.p;
  a.partial_cap = kMaxHvGrid;  // ctx->partials holds this many slots
}

// One Krylov pass with fused Grams, reduced into meas.  With a sweep plan
// (sweeps = true and more than one sweep), the pass runs as one launch per
// sweep: the first adds the diagonal, each writes its partial sum to ctx->acc,
// the last adds its terms to that sum and forms the recurrence combination and
// the Grams.
int hv_launches(lrei_ctx *ctx, int r, int grid, int mode, const void *cur, void *next, double2 *partials,
                bool sweeps, int partial_cap = kMaxHvGrid, const double *colshift = nullptr) {
  HvArgs a{};
  a.Pcur = cur;
  a.Pnext = next;
  hv_args(ctx, a);
  a.N = ctx->N;
  a.r = r;
  if (!hv_epl_valid(ctx->fp32, r, a.epl)) a.epl = 0;  // a shape tuned for another rank
  a.alpha = krylov_beta(ctx);
  a.colshift = colshift;
  a.mode = mode;
  a.partials = partials;
  a.grid = grid;
  a.partial_cap = partial_cap;
  a.skip = ctx->pass_skip;
  const size_t ns = ctx->sweeps.size();
  int slots = 0;
  if (mode != 2 && ns <= 1 && ctx->hv_tile_bits > 0) {  // the tiled pass
    a.tile_bits = ctx->hv_tile_bits;
    a.tile_waves = ctx->hv_tile_waves;
    a.n_local = local_terms(ctx, ctx->hv_tile_bits);
  } else if (ctx->hv_compact && r <= 16) {
    a.compact = 1;
  }
  if (!sweeps || ns <= 1) {
    slots = launch_hv(ctx->fp32, a, ctx->stream);
  } else {
    for (size_t i = 0; i < ns; ++i) {
      const auto &sw = ctx->sweeps[i];
      HvArgs b = a;
      b.t0 = sw.t0;
      b.t1 = sw.t1;
      b.use_diag = i == 0;
      b.acc_in = i == 0 ? nullptr : ctx->acc.p;
      b.acc_out = i + 1 < ns;
      if (b.acc_out) b.Pnext = ctx->acc.p;
      b.win_bits = (int)sw.win.size();
      b.n_fix = (int)sw.fix.size();
      for (size_t q = 0; q < sw.win.size(); ++q) b.win_pos[q] = (unsigned char)sw.win[q];
      for (size_t q = 0; q < sw.fix.size(); ++q) b.fix_pos[q] = (unsigned char)sw.fix[q];
      slots = launch_hv(ctx->fp32, b, ctx->stream);
    }
  }
  if (slots <= 0) ctx->hv_launch_failed = true;
  return slots;  // Gram partial slots written by the (last) launch
}

bool hv_pass_into(lrei_ctx *ctx, int r, int grid, int mode, const void *cur, void *next, double2 *partials,
                    double2 *meas, bool sweeps = false, int partial_cap = kMaxHvGrid,
                    const double *colshift = nullptr) {
  const int slots = hv_launches(ctx, r, grid, mode, cur, next, partials, sweeps, partial_cap, colshift);
  if (slots <= 0) return false;
  if (mode != 2) launch_reduce(partials, slots, (mode == 0 ? 3 : 2) * r * r, meas, ctx->stream);
  return true;
}

// Forgets the tuned H.V launch shape (it was chosen for one rank and
// precision) and the captured step graph that baked it in.
void reset_hv_tuning(lrei_ctx *ctx) {
  ctx->epl = 0;
  ctx->hv_grid = 0;
  ctx->overlap = {};
  ctx->hv_tile_bits = 0;
  ctx->hv_compact = 0;
  ctx->drop_graph();
}

// Workgroups of the basis combination.  A CU holds twice as many of its
// workgroups as of the H.V pass's, and the combination's block reads need
// that many waves in flight: twice the pass grid, at most the tile count.
int combine_grid(const lrei_ctx *ctx) {
  const long long tiles = (ctx->N + 63) / 64;
  long long g = 2LL * ctx->grid;
  if (g > tiles) g = tiles >= 8 ? (tiles & ~7LL) : tiles;
  return (int)(g < 1 ? 1 : g);
}

// Grid of a pass that runs beside the step's stage kernels.  A stage kernel
// is one workgroup that needs most of a CU's vector registers and LDS (room
// for at most one pass workgroup beside it); while a pass holds every slot
// of every CU the stage waits for the pass to drain.  When the
// tuned grid fills the chip, such passes leave two CUs of each of the 8 XCDs
// free: (CUs - 16) x the workgroups a CU holds.  Only the dynamic chunk
// schedule, which balances any grid that is a multiple of 8, takes it.
int overlap_grid(lrei_ctx *ctx) {
  auto &o = ctx->overlap;
  const int r = ctx->r, fp32 = ctx->fp32 ? 1 : 0;
  const int ns = (int)ctx->sweeps.size();
  if (o.grid == ctx->hv_grid && o.epl == ctx->epl && o.r == r && o.compact == ctx->hv_compact && o.fp32 == fp32 &&
      o.tile_bits == ctx->hv_tile_bits && o.sweeps == ns)
    return o.result;
  o.tile_bits = ctx->hv_tile_bits;
  o.sweeps = ns;
  o.grid = ctx->hv_grid;
  o.epl = ctx->epl;
  o.r = r;
  o.compact = ctx->hv_compact;
  o.fp32 = fp32;
  o.result = ctx->hv_grid;
  const int cus = ctx->num_cus;
  if (ctx->hv_tile_bits > 0 || ns > 1 || cus <= 16 || cus % 8 != 0) return o.result;
  HvArgs a{};
  hv_args(ctx, a);
  a.N = ctx->N;
  a.r = r;
  if (!hv_epl_valid(ctx->fp32, r, a.epl)) a.epl = 0;
  a.mode = 1;
  a.grid = ctx->hv_grid;
  a.compact = ctx->hv_compact && r <= 16;
  bool dyn = false;
  const int per_cu = hv_resident_per_cu(ctx->fp32, a, &dyn);
  if (!dyn || per_cu <= 0 || ctx->hv_grid < cus * per_cu) return o.result;
  a.grid = (cus - 16) * per_cu;
  if (hv_resident_per_cu(ctx->fp32, a, &dyn) > 0 && dyn) o.result = a.grid;
  return o.result;
}

// Krylov pass j of a step: P_{j+1} = beta (H P_j - P_j diag(D_j)) into
// blocks[j + 1] with its Gram products into slot j of ws.meas; D_j is the
// context's column shift of block j (zero when `shifted` is false).
void krylov_pass(lrei_ctx *ctx, int j, bool shifted = true) {
  hv_pass_into(ctx, ctx->r, j == 0 ? ctx->hv_grid : overlap_grid(ctx), j == 0 ? 0 : 1, ctx->blocks[j].p, ctx->blocks[j + 1].p,
                 (double2 *)ctx->partials.p, ctx->ws.meas + (size_t)j * 3 * ctx->r * ctx->r, true, kMaxHvGrid,
                 shifted ? ctx->ws.shifts + (size_t)j * ctx->r : nullptr);
}

// Sweep plan for windows of w row bits: repeatedly choose the n - w fixed bits
// that the fewest remaining flip masks touch (exhaustively when the choice is
// small, else greedily bit by bit), give those masks' terms to a sweep, and
// upload the term tables in sweep order.  w >= n (or 0) is one sweep.
lrei_status hv_set_plan(lrei_ctx *ctx, int w) {
  const int n = ctx->n;
  const auto &off = ctx->terms.off;
  std::vector<int> order;
  std::vector<lrei_ctx::HvSweep> plan;
  if (w <= 0 || w >= n) {
    lrei_ctx::HvSweep sw;
    for (int b = 0; b < n; ++b) sw.win.push_back(b);
    sw.t0 = 0;
    sw.t1 = (int)off.size();
    for (size_t t = 0; t < off.size(); ++t) order.push_back((int)t);
    plan.push_back(sw);
    w = 0;
  } else {
    std::vector<int> left;
    for (size_t t = 0; t < off.size(); ++t) left.push_back((int)t);
    const int nf = n - w;
    auto hits = [&](uint32_t fmask) {
      int c = 0;
      for (int t : left) c += (off[t].mask & fmask) != 0;
      return c;
    };
    double combos = 1;
    for (int i = 0; i < nf; ++i) combos = combos * (n - i) / (i + 1);
    while (!left.empty()) {
      uint32_t best = 0;
      if (combos <= 2e5) {
        int bestc = 1 << 30;
        std::vector<int> idx(nf);
        for (int i = 0; i < nf; ++i) idx[i] = i;
        while (true) {
          uint32_t fm = 0;
          for (int i : idx) fm |= 1u << i;
          const int c = hits(fm);
          if (c < bestc) {
            bestc = c;
            best = fm;
          }
          int i = nf - 1;
          while (i >= 0 && idx[i] == n - nf + i) --i;
          if (i < 0) break;
          ++idx[i];
          for (int q = i + 1; q < nf; ++q) idx[q] = idx[q - 1] + 1;
        }
      } else {
        for (int i = 0; i < nf; ++i) {
          int bestc = 1 << 30, bb = -1;
          for (int b = 0; b < n; ++b) {
            if (best & (1u << b)) continue;
            const int c = hits(best | (1u << b));
            if (c < bestc) {
              bestc = c;
              bb = b;
            }
          }
          best |= 1u << bb;
        }
      }
      lrei_ctx::HvSweep sw;
      for (int b = 0; b < n; ++b) (best & (1u << b) ? sw.fix : sw.win).push_back(b);
      sw.t0 = (int)order.size();
      std::vector<int> rest;
      for (int t : left) {
        if ((off[t].mask & best) == 0)
          order.push_back(t);
        else
          rest.push_back(t);
      }
      sw.t1 = (int)order.size();
      if (sw.t1 == sw.t0) return ctx->fail(LREI_E_INVALID, "H.V sweep plan: a term does not fit any window");
      plan.push_back(sw);
      left.swap(rest);
    }
  }
  // term tables in sweep order
  std::vector<DevOffTerm> o64(off.size());
  std::vector<DevTerm<float>> o32(off.size());
  for (size_t q = 0; q < order.size(); ++q) {
    const OffTerm &t = off[order[q]];
    o64[q].mask = o32[q].mask = t.mask;
    o64[q].sa = o32[q].sa = t.sa;
    o64[q].sb = o32[q].sb = t.sb;
    o64[q].act = o32[q].act = 0;
    for (int k = 0; k < 4; ++k) {
      o64[q].re[k] = t.re[k];
      o64[q].im[k] = t.im[k];
      o32[q].re[k] = (float)t.re[k];
      o32[q].im[k] = (float)t.im[k];
      if (o64[q].re[k] != 0.0 || o64[q].im[k] != 0.0) o64[q].act |= 1u << k;
      if (o32[q].re[k] != 0.0f || o32[q].im[k] != 0.0f) o32[q].act |= 1u << k;
    }
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (!o64.empty()) {
    HIPCHK(hipMemcpy(ctx->dt.off64.p, o64.data(), o64.size() * sizeof(DevOffTerm), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->dt.off32.p, o32.data(), o32.size() * sizeof(DevTerm<float>), hipMemcpyHostToDevice));
  }
  ctx->sweeps = plan;
  ctx->hv_w = w;
  ctx->drop_graph();
  return LREI_OK;
}

SmallRkParams rk_params(lrei_ctx *ctx, int model, int scheme, double dt, double kappa) {
  SmallRkParams p{};
  int s;
  tableau(scheme, s, p.a, p.b);
  p.r = ctx->r;
  p.s = s;
  p.nblocks = s + 1;
  p.model = model;
  p.householder_mode = ctx->opt.householder_mode;
  p.max_sweeps = ctx->opt.eig_max_sweeps;
  p.warm = ctx->opt.warm;
  p.net = ctx->net;
  p.rec = ctx->rec_cap > 0 ? ctx->rec : nullptr;
  p.rec_count = (int *)ctx->rec_count.p;
  p.rec_cap = ctx->rec_cap;
  p.kappa = kappa;
  p.hbar = ctx->hbar;
  p.h = dt;
  p.eig_tol = ctx->opt.eig_tol;
  // the warm-started eigensolve stops well below the storage rounding of the path
  p.warm_tol = ctx->fp32 ? 1e-11 : 1e-14;
  p.beta = krylov_beta(ctx);
  for (int i = 0; i < ctx->r; ++i) p.lam[i] = ctx->lam[i];
  p.lds_elems = small_lds_elems(p.nblocks * ctx->r, ctx->r);
  return p;
}

// Enqueues one LREI-RK step: the Krylov passes on the context
// stream; as soon as pass j is reduced (stage j needs the Grams of
// P_0 .. P_{j+1} only) the basis extension of stage j on the basis stream,
// then stage j itself on the side stream, so that the extension of stage
// j + 1 and the later passes overlap stage j; the combination after the last
// stage.
void enqueue_stages(lrei_ctx *ctx, const SmallRkParams &p);

void enqueue_rk_step(lrei_ctx *ctx, int model, int scheme, double dt, double kappa) {
  enqueue_stages(ctx, rk_params(ctx, model, scheme, dt, kappa));
}

// One attempt of an adaptive step: the stages of the pair's tableau (and the
// error stage), the controller's decision on the device, the combination
// (the old state again when the attempt is rejected).  Every kernel of the
// attempt does nothing once the controller has reached t_end or failed.
void enqueue_attempt(lrei_ctx *ctx, const SmallRkParams &p) {
  launch_attempt_begin(p.ctl, ctx->stream);
  ctx->pass_skip = p.ctl + kCtlSkip;
  enqueue_stages(ctx, p);
  ctx->pass_skip = nullptr;
}

// Passes, basis extensions and stages of one RK step (or adaptive attempt),
// then the combination V_new = [P_0 .. P_{nblocks-1}] C.
void enqueue_stages(lrei_ctx *ctx, const SmallRkParams &p) {
  // an error stage that weights f at the new state needs one more pass
  const int s = (p.ctl && p.err_stage == p.s) ? p.s + 1 : p.s;
  (void)hipEventRecord(ctx->ev_fork, ctx->stream);
  (void)hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0);
  (void)hipStreamWaitEvent(ctx->basis, ctx->ev_fork, 0);
  for (int j = 0; j < s; ++j) {
    krylov_pass(ctx, j);
    (void)hipEventRecord(ctx->ev_pass[j], ctx->stream);
    (void)hipStreamWaitEvent(ctx->basis, ctx->ev_pass[j], 0);
    launch_small_rk_basis(p, ctx->ws, j, ctx->basis);
    (void)hipEventRecord(ctx->ev_basis[j], ctx->basis);
    (void)hipStreamWaitEvent(ctx->side, ctx->ev_basis[j], 0);
    launch_small_rk_stage(p, ctx->ws, j, ctx->side);
  }
  (void)hipEventRecord(ctx->ev_join_basis, ctx->basis);
  (void)hipStreamWaitEvent(ctx->stream, ctx->ev_join_basis, 0);
  (void)hipEventRecord(ctx->ev_join, ctx->side);
  (void)hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0);
  const void *bl[kMaxBlocks];
  for (int i = 0; i < p.nblocks; ++i) bl[i] = ctx->blocks[i].p;
  launch_combine(ctx->fp32, bl, p.nblocks, ctx->ws.Cfin, ctx->blocks[0].p, ctx->N, ctx->r, combine_grid(ctx),
                 ctx->stream,
                 p.ctl ? p.ctl + kCtlSkip : nullptr, ctx->fp32 ? ctx->lo.p : nullptr,
                 ctx->fp32 ? ctx->lo.p : nullptr);
}

// Steps between two checks of the mixed-precision conditioning floor.
constexpr int kGuardSteps = 16;

// k RK steps: replays of the captured step graph (captured first if the step
// differs from the last one captured), or eager launches.
lrei_status run_rk_steps(lrei_ctx *ctx, int model, int scheme, double dt, double kappa, int k) {
  if (ctx->opt.use_graph == 0) {
    for (int i = 0; i < k; ++i) enqueue_rk_step(ctx, model, scheme, dt, kappa);
    return LREI_OK;
  }
  int first = 0;
  if (!(ctx->exec && ctx->g_model == model && ctx->g_scheme == scheme && ctx->g_dt == dt && ctx->g_kappa == kappa)) {
    ctx->drop_graph();
    // launch attributes are set on first use, outside capture; this eager
    // step counts as the first step
    enqueue_rk_step(ctx, model, scheme, dt, kappa);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    enqueue_rk_step(ctx, model, scheme, dt, kappa);
    HIPCHK(hipStreamEndCapture(ctx->stream, &ctx->graph));
    HIPCHK(hipGraphInstantiate(&ctx->exec, ctx->graph, nullptr, nullptr, 0));
    ctx->g_model = model;
    ctx->g_scheme = scheme;
    ctx->g_dt = dt;
    ctx->g_kappa = kappa;
    first = 1;
  }
  for (int i = first; i < k; ++i) HIPCHK(hipGraphLaunch(ctx->exec, ctx->stream));
  return LREI_OK;
}

void ab_reset(lrei_ctx *ctx);

// Moves a LREI_MIXED context to FP64 storage: the state and the rollback
// copy of the current call (its start-of-call state) are widened exactly,
// the N-space buffers are reallocated for FP64, the captured graphs, the
// tuned H.V shape and the AB history are dropped.
lrei_status promote_fp64(lrei_ctx *ctx) {
  const size_t n = (size_t)ctx->N * ctx->r;
  void *wide = nullptr, *wide_save = nullptr;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (hipMalloc(&wide, n * sizeof(double2)) != hipSuccess)
    return ctx->fail(LREI_E_NOMEM, "device allocation for the FP64 promotion failed");
  if (hipMalloc(&wide_save, n * sizeof(double2)) != hipSuccess) {
    (void)hipFree(wide);
    return ctx->fail(LREI_E_NOMEM, "device allocation for the FP64 promotion failed");
  }
  launch_merge((const float2 *)ctx->blocks[0].p, ctx->lo.p, (double2 *)wide, (long long)n,
               ctx->stream);
  launch_merge((const float2 *)ctx->save.p, ctx->save_lo.p, (double2 *)wide_save, (long long)n,
               ctx->stream);  // the start-of-call state
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(wide);
    (void)hipFree(wide_save);
    return check_hip(ctx, e, "FP64 promotion");
  }
  ctx->drop_graph();
  ab_reset(ctx);
  ctx->fp32 = false;
  ctx->epl = 0;
  ctx->hv_grid = 0;
  ctx->overlap = {};
  ctx->hv_tile_bits = 0;
  ctx->hv_compact = 0;
  lrei_status st = alloc_state(ctx, ctx->r, false);
  if (st == LREI_OK) {
    e = hipMemcpyAsync(ctx->blocks[0].p, wide, n * sizeof(double2), hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ctx->save.p, wide_save, n * sizeof(double2), hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) st = check_hip(ctx, e, "FP64 promotion");
  }
  (void)hipFree(wide);
  (void)hipFree(wide_save);
  if (st == LREI_OK) ctx->stats.precision_promoted = 1;
  return st;
}

// Projected-step parameters of an adaptive attempt with an embedded pair.
SmallRkParams adapt_params(lrei_ctx *ctx, int model, int pair, double kappa) {
  SmallRkParams p = rk_params(ctx, model, LREI_RK4, 0.0, kappa);
  int s = 0, err_stage = 0, q = 0;
  pair_tableau(pair, s, p.a, p.b, p.e, err_stage, q);
  p.s = s;
  p.nblocks = err_stage == s ? s + 2 : s + 1;
  p.err_stage = err_stage;
  p.order_low = q;
  p.ctl = (double *)ctx->ctl.p;
  p.h = 0.0;  // the step comes from the controller state
  p.lds_elems = small_lds_elems(p.nblocks * ctx->r, ctx->r);
  return p;
}

// ---- ABm schemes -------------------------------------------------------------

int ab_order(int scheme) { return scheme - 10; }  // LREI_AB2 = 12 -> m = 2

// Allocates the AB history buffers for order m at the current rank.
lrei_status ab_alloc(lrei_ctx *ctx, int m) {
  const int r = ctx->r;
  const size_t blk = (size_t)ctx->N * r * ctx->elem();
  for (auto &set : ctx->ab_U)
    for (int i = 0; i < 2 * m - 1; ++i)
      if (!set[i].ensure(blk)) return ctx->fail(LREI_E_NOMEM, "device allocation of the AB history failed");
  const int Dmax = 2 * m * r, qmax = (2 * m - 1) * r, rr = r * r;
  const size_t coords = (size_t)(2 * m - 1) * qmax * r;
  bool ok = ctx->ab_coords[0].ensure(coords * sizeof(double2)) && ctx->ab_coords[1].ensure(coords * sizeof(double2)) &&
            ctx->ab_UUg.ensure((size_t)kMaxGrams * rr * sizeof(double2)) &&
            ctx->ab_c1g.ensure((size_t)kMaxGrams * rr * sizeof(double2)) &&
            ctx->ab_gBg.ensure((size_t)kMaxGrams * rr * sizeof(double2)) &&
            ctx->ab_Cb.ensure((size_t)Dmax * 3 * r * sizeof(double2)) &&
            ctx->ab_Cc.ensure((size_t)Dmax * (qmax + r) * sizeof(double2)) &&
            ctx->ab_work.ensure(small_ab_work_elems(Dmax, qmax, r) * sizeof(double2));
  ctx->ab_grid = blocks_grid(ctx->N);
  ok = ok && ctx->ab_partials.ensure((size_t)kMaxGrams * rr * ctx->ab_grid * sizeof(double2));
  if (!ok) return ctx->fail(LREI_E_NOMEM, "device allocation of the AB workspace failed");
  return LREI_OK;
}

void ab_reset(lrei_ctx *ctx) {
  ctx->ab = lrei_ctx::AbState{};
}

// One block pass plus the reduction of its Gram products into dst.
void block_pass(lrei_ctx *ctx, const std::vector<const void *> &in, const std::vector<void *> &out,
                const double2 *C, int ldc, const std::vector<std::pair<int, int>> &grams, double2 *dst) {
  BlocksArgs a{};
  for (size_t i = 0; i < in.size(); ++i) a.in[i] = in[i];
  for (size_t i = 0; i < out.size(); ++i) a.out[i] = out[i];
  a.n_in = (int)in.size();
  a.n_out = (int)out.size();
  a.C = C;
  a.ldc = ldc;
  for (size_t g = 0; g < grams.size(); ++g) {
    a.ga[g] = (signed char)grams[g].first;
    a.gb[g] = (signed char)grams[g].second;
  }
  a.n_gram = (int)grams.size();
  a.partials = (double2 *)ctx->ab_partials.p;
  a.N = ctx->N;
  a.r = ctx->r;
  a.grid = ctx->ab_grid;
  launch_blocks(ctx->fp32, a, ctx->stream);
  if (a.n_gram > 0) launch_reduce(a.partials, a.grid, a.n_gram * ctx->r * ctx->r, dst, ctx->stream);
}

// Orthogonalises the new blocks X against the history basis U and rotates
// [U, Y] into the next basis (after an RK start-up step, mode 0, or as the AB
// step itself, mode 1).
void ab_update(lrei_ctx *ctx, const std::vector<const void *> &X, SmallAbParams p) {
  auto &ab = ctx->ab;
  const int r = ctx->r, nU = ab.nU, qx = (int)X.size();
  std::vector<const void *> U;
  for (int i = 0; i < nU; ++i) U.push_back(ctx->ab_U[ab.cur][i].p);
  std::vector<const void *> ux = U;
  ux.insert(ux.end(), X.begin(), X.end());
  std::vector<const void *> Y;
  if (nU > 0) {
    std::vector<std::pair<int, int>> ga;
    for (int i = 0; i < nU; ++i)
      for (int q = 0; q < qx; ++q) ga.push_back({i, nU + q});
    block_pass(ctx, ux, {}, nullptr, 0, ga, (double2 *)ctx->ab_c1g.p);
    launch_ab_cgs_coef((const double2 *)ctx->ab_c1g.p, nU, qx, r, (double2 *)ctx->ab_Cb.p, ctx->stream);
    std::vector<void *> yout;
    for (int q = 0; q < qx; ++q) yout.push_back(ctx->blocks[2 + q].p);
    std::vector<std::pair<int, int>> gb;
    const int y0 = nU + qx;
    for (int i = 0; i < nU; ++i)
      for (int q = 0; q < qx; ++q) gb.push_back({i, y0 + q});
    for (int q = 0; q < qx; ++q)
      for (int q2 = q; q2 < qx; ++q2) gb.push_back({y0 + q, y0 + q2});
    block_pass(ctx, ux, yout, (const double2 *)ctx->ab_Cb.p, qx * r, gb, (double2 *)ctx->ab_gBg.p);
    for (auto *y : yout) Y.push_back(y);
  } else {
    std::vector<std::pair<int, int>> gb;
    for (int q = 0; q < qx; ++q)
      for (int q2 = q; q2 < qx; ++q2) gb.push_back({q, q2});
    block_pass(ctx, X, {}, nullptr, 0, gb, (double2 *)ctx->ab_gBg.p);
    Y = X;
  }
  p.nU = nU;
  p.qx = qx;
  p.npairs_keep = std::min(ab.npairs, ab.m - 2);
  if (p.npairs_keep < 0) p.npairs_keep = 0;
  const int qn = (3 + 2 * p.npairs_keep) * r, nUn = qn / r;
  p.lds_elems = small_lds_elems((nU + qx) * r, r);
  SmallAbWs w{};
  w.UUg = (const double2 *)ctx->ab_UUg.p;
  w.c1g = (const double2 *)ctx->ab_c1g.p;
  w.gBg = (const double2 *)ctx->ab_gBg.p;
  w.coords_in = (const double2 *)ctx->ab_coords[ab.cur].p;
  w.coords_out = (double2 *)ctx->ab_coords[1 - ab.cur].p;
  w.Cc = (double2 *)ctx->ab_Cc.p;
  w.work = (double2 *)ctx->ab_work.p;
  w.stats = (double *)ctx->stats_buf.p;
  launch_small_ab(p, w, ctx->stream);
  std::vector<const void *> uy = U;
  uy.insert(uy.end(), Y.begin(), Y.end());
  std::vector<void *> out;
  for (int i = 0; i < nUn; ++i) out.push_back(ctx->ab_U[1 - ab.cur][i].p);
  if (p.mode == 1) out.push_back(ctx->blocks[0].p);
  const int b0 = nU + qx;
  std::vector<std::pair<int, int>> gc;
  for (int i = 0; i < nUn; ++i)
    for (int j = i; j < nUn; ++j) gc.push_back({b0 + i, b0 + j});
  block_pass(ctx, uy, out, (const double2 *)ctx->ab_Cc.p, qn + r, gc, (double2 *)ctx->ab_UUg.p);
  ab.cur ^= 1;
  ab.nU = nUn;
  ab.npairs = p.npairs_keep + 1;
}

SmallAbParams ab_params(lrei_ctx *ctx, int mode) {
  SmallAbParams p{};
  const auto &ab = ctx->ab;
  p.r = ctx->r;
  p.m_ab = ab.m;
  p.mode = mode;
  p.model = ab.model;
  p.householder_mode = ctx->opt.householder_mode;
  p.max_sweeps = ctx->opt.eig_max_sweeps;
  p.eig_tol = ctx->opt.eig_tol;
  p.kappa = ab.kappa;
  p.hbar = ctx->hbar;
  p.h = ab.dt;
  static const double b2[2] = {3.0 / 2, -1.0 / 2}, b3[3] = {23.0 / 12, -16.0 / 12, 5.0 / 12},
                      b4[4] = {55.0 / 24, -59.0 / 24, 37.0 / 24, -9.0 / 24};
  const double *b = ab.m == 2 ? b2 : (ab.m == 3 ? b3 : b4);
  for (int l = 0; l < kMaxAb; ++l) p.bcoef[l] = l < ab.m ? b[l] : 0.0;
  for (int i = 0; i < ctx->r; ++i) p.lam[i] = ctx->lam[i];
  return p;
}

// One step of an ABm run: an RK start-up step plus a history update while
// fewer than m - 1 steps are done, else the AB step.
void enqueue_ab_step(lrei_ctx *ctx) {
  auto &ab = ctx->ab;
  const double e = 1.0 / krylov_beta(ctx);
  if (ab.count < ab.m - 1) {
    const int j = ab.count;
    int bs = ctx->opt.ab_bootstrap;
    if (!(bs >= LREI_RK1 && bs <= LREI_RK4)) bs = LREI_RK4;
    // V_j is needed after the combine overwrote blocks[0]: keep a copy at the first step
    if (j == 0)
      (void)hipMemcpyAsync(ctx->ab_U[1 - ab.cur][0].p, ctx->blocks[0].p, (size_t)ctx->N * ctx->r * ctx->elem(),
                           hipMemcpyDeviceToDevice, ctx->stream);
    // the history takes blocks[1] as a multiple of H V_j: no column shift on
    // the first Krylov block of a start-up step (AB steps are never captured)
    (void)hipMemsetAsync(ctx->ws.shifts, 0, ctx->r * sizeof(double), ctx->stream);
    enqueue_rk_step(ctx, ab.model, bs, ab.dt, ab.kappa);
    SmallAbParams p = ab_params(ctx, 0);
    std::vector<const void *> X;
    if (j == 0) {
      // U is empty: the copy of V_0 sits in a block of the set that the rotation writes;
      // move it to a Krylov block first (blocks[1] holds alpha H V_0, blocks[0] V_1)
      (void)hipMemcpyAsync(ctx->blocks[4].p, ctx->ab_U[1 - ab.cur][0].p, (size_t)ctx->N * ctx->r * ctx->elem(),
                           hipMemcpyDeviceToDevice, ctx->stream);
      X = {ctx->blocks[4].p, ctx->blocks[1].p, ctx->blocks[0].p};
      p.x_v0 = 0;
      p.x_hv = 1;
      p.x_vnew = 2;
    } else {
      X = {ctx->blocks[1].p, ctx->blocks[0].p};
      p.x_v0 = -1;
      p.x_hv = 0;
      p.x_vnew = 1;
    }
    p.hv_scale = e;  // blocks[1] = beta H V_j, e = 1 / beta
    ab_update(ctx, X, p);
  } else {
    HvArgs a{};
    a.Pcur = ctx->blocks[0].p;
    a.Pnext = ctx->blocks[1].p;
    hv_args(ctx, a);
    a.N = ctx->N;
    a.r = ctx->r;
    if (!hv_epl_valid(ctx->fp32, a.r, a.epl)) a.epl = 0;
    a.alpha = 1.0;
    a.mode = 2;
    a.grid = ctx->grid;
    if (launch_hv(ctx->fp32, a, ctx->stream) <= 0) ctx->hv_launch_failed = true;
    SmallAbParams p = ab_params(ctx, 1);
    p.x_v0 = -1;
    p.x_hv = 0;
    p.x_vnew = -1;
    p.hv_scale = 1.0;
    ab_update(ctx, {ctx->blocks[1].p}, p);
    // the AB step writes the new state in the storage precision only: the
    // compensation of a mixed state restarts at zero (AB steps are never captured)
    if (ctx->fp32) (void)hipMemsetAsync(ctx->lo.p, 0, ctx->lo_bytes(), ctx->stream);
  }
  ab.count += 1;
}


lrei_status read_stats(lrei_ctx *ctx, double *h) {
  HIPCHK(hipMemcpyAsync(h, ctx->stats_buf.p, kStatsLen * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LREI_OK;
}

}  // namespace

extern "C" {

void lrei_default_options(lrei_options *o) {
  if (!o) return;
  o->precision = LREI_FP64;
  o->eig_tol = 1e-15;
  o->eig_max_sweeps = 40;
  o->warm = LREI_WARM_ANALYTIC;
  o->ab_bootstrap = LREI_RK4;
  o->householder_mode = 0;
  o->use_graph = 1;
  o->deterministic = 1;
  o->autotune_cache = nullptr;
  o->mixed_pivot_floor = 2e-6;
  o->fail_after_steps = 0;
  o->site_order = 0;
}

lrei_status lrei_create(lrei_ctx **out, int hip_device, void *hip_stream, const lrei_options *opt) {
  if (!out) return LREI_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return LREI_E_DEVICE;
  if (hip_device < 0 || hip_device >= ndev) return LREI_E_INVALID;
  lrei_ctx *ctx = new lrei_ctx();
  lrei_default_options(&ctx->opt);
  if (opt) ctx->opt = *opt;
  if (ctx->opt.precision != LREI_FP64 && ctx->opt.precision != LREI_MIXED) {
    delete ctx;
    return LREI_E_INVALID;
  }
  if (!(ctx->opt.mixed_pivot_floor >= 0) || !std::isfinite(ctx->opt.mixed_pivot_floor)) {
    delete ctx;
    return LREI_E_INVALID;
  }
  if (ctx->opt.site_order != 0 && ctx->opt.site_order != 1) {
    delete ctx;
    return LREI_E_INVALID;
  }
  if (!(ctx->opt.eig_tol > 0) || ctx->opt.eig_max_sweeps < 1 ||
      ctx->opt.warm < LREI_WARM_PLAIN || ctx->opt.warm > LREI_WARM_PREDICT_CAYLEY) {
    delete ctx;
    return LREI_E_INVALID;
  }
  ctx->fp32 = ctx->opt.precision == LREI_MIXED;
  ctx->device = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess) {
    delete ctx;
    return LREI_E_DEVICE;
  }
  if (hip_stream) ctx->stream = (hipStream_t)hip_stream;
  ctx->own_stream = !hip_stream;
  if (hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess) {
    delete ctx;
    return LREI_E_DEVICE;
  }
  if (create_streams(!hip_stream, &ctx->stream, &ctx->side) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->basis, hipStreamNonBlocking) != hipSuccess) {
    lrei_destroy(ctx);
    return LREI_E_DEVICE;
  }
  bool ok = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&ctx->ev_join_basis, hipEventDisableTiming) == hipSuccess;
  for (auto &e : ctx->ev_pass) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  for (auto &e : ctx->ev_basis) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  ok = ok && ctx->sched.ensure(16 * sizeof(int)) && hipMemset(ctx->sched.p, 0, 16 * sizeof(int)) == hipSuccess;
  ok = ok && resolve_scratch(hip_device) == hipSuccess;
  if (!ok) {
    lrei_destroy(ctx);
    return LREI_E_DEVICE;
  }
  *out = ctx;
  return LREI_OK;
}

void lrei_destroy(lrei_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->drop_graph();
  for (auto &b : ctx->blocks) b.release();
  ctx->save.release();
  ctx->acc.release();
  ctx->sched.release();
  ctx->partials.release();
  ctx->ws_buf.release();
  ctx->stats_buf.release();
  ctx->ctl.release();
  ctx->lam_dev.release();
  ctx->dt.release();
  for (auto &set : ctx->ab_U)
    for (auto &b : set) b.release();
  for (auto &b : ctx->ab_coords) b.release();
  ctx->ab_UUg.release();
  ctx->ab_c1g.release();
  ctx->ab_gBg.release();
  ctx->ab_Cb.release();
  ctx->ab_Cc.release();
  ctx->ab_work.release();
  ctx->ab_partials.release();
  for (hipStream_t *st : {&ctx->side, &ctx->basis})
    if (*st) {
      (void)hipStreamSynchronize(*st);
      (void)hipStreamDestroy(*st);
    }
  for (hipEvent_t e : {ctx->ev_fork, ctx->ev_join, ctx->ev_join_basis})
    if (e) (void)hipEventDestroy(e);
  for (auto &e : ctx->ev_pass)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : ctx->ev_basis)
    if (e) (void)hipEventDestroy(e);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char *lrei_last_error(const lrei_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

lrei_status lrei_record(lrei_ctx *ctx, float *samples, int capacity) {
  if (!ctx) return LREI_E_INVALID;
  if (capacity < 0 || (capacity > 0 && !samples)) return ctx->fail(LREI_E_INVALID, "invalid sample buffer");
  (void)hipSetDevice(ctx->device);
  if (!ctx->rec_count.ensure(sizeof(int))) return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipMemset(ctx->rec_count.p, 0, sizeof(int));
  if (e != hipSuccess) return ctx->fail(LREI_E_DEVICE, std::string("record: ") + hipGetErrorString(e));
  ctx->rec = capacity > 0 ? samples : nullptr;
  ctx->rec_cap = capacity;
  ctx->drop_graph();  // the recorder is a launch argument of the stage kernel
  return LREI_OK;
}

lrei_status lrei_record_count(lrei_ctx *ctx, int *count) {
  if (!ctx || !count) return LREI_E_INVALID;
  *count = 0;
  if (!ctx->rec_count.p) return LREI_OK;
  (void)hipSetDevice(ctx->device);
  int c = 0;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(&c, ctx->rec_count.p, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return ctx->fail(LREI_E_DEVICE, std::string("record count: ") + hipGetErrorString(e));
  *count = std::min(c, ctx->rec_cap);
  return LREI_OK;
}

lrei_status lrei_attach_net(lrei_ctx *ctx, const lrei_net *m) {
  if (!ctx) return LREI_E_INVALID;
  if (m && ctx->have_rho && lrei_net_rank(m) != ctx->r)
    return ctx->fail(LREI_E_INVALID, "the network's rank differs from the state's");
  ctx->net = m ? (const float *)lrei_net_device_params(m) : nullptr;
  ctx->net_r = m ? lrei_net_rank(m) : 0;
  ctx->drop_graph();
  return LREI_OK;
}

lrei_status lrei_set_hamiltonian(lrei_ctx *ctx, int n_spins, int n_bonds, const int32_t *bond_ij,
                                 const double *bond_J, const double *site_h, double hbar) {
  if (!ctx) return LREI_E_INVALID;
  if (!(hbar > 0) || !std::isfinite(hbar)) return ctx->fail(LREI_E_INVALID, "hbar must be positive and finite");
  if (n_spins < 1 || n_spins > 30) return ctx->fail(LREI_E_INVALID, "n_spins must be in [1, 30]");
  if (n_bonds < 0 || (n_bonds > 0 && (!bond_ij || !bond_J))) return ctx->fail(LREI_E_INVALID, "bad bond arrays");
  for (int b = 0; b < 2 * n_bonds; ++b)
    if (bond_ij[b] < 0 || bond_ij[b] >= n_spins) return ctx->fail(LREI_E_INVALID, "bond site out of range");
  if (ctx->have_rho && n_spins != ctx->n)
    return ctx->fail(LREI_E_STATE, "n_spins differs from the current state; set a new rho after changing n");
  // terms in the internal site order
  const std::vector<int> pos = ctx->opt.site_order == 1
                                   ? choose_site_order_cluster(n_spins, n_bonds, bond_ij, kClusterBits)
                                   : choose_site_order(n_spins, n_bonds, bond_ij);
  // a bond whose sites swap order gets the transposed tensor (J^{ab} s^a_i s^b_j)
  std::vector<int32_t> pbonds(2 * (size_t)n_bonds);
  std::vector<double> pJ(bond_J ? bond_J : (const double *)nullptr, bond_J ? bond_J + 9 * (size_t)n_bonds : nullptr);
  for (int b = 0; b < n_bonds; ++b) {
    int i = pos[bond_ij[2 * b]], j = pos[bond_ij[2 * b + 1]];
    if (i > j) {
      std::swap(i, j);
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < a; ++c) std::swap(pJ[9 * b + 3 * a + c], pJ[9 * b + 3 * c + a]);
    }
    pbonds[2 * b] = i;
    pbonds[2 * b + 1] = j;
  }
  std::vector<double> ph;
  if (site_h) {
    ph.assign(3 * (size_t)n_spins, 0.0);
    for (int q = 0; q < n_spins; ++q)
      for (int c = 0; c < 3; ++c) ph[3 * pos[q] + c] = site_h[3 * q + c];
  }
  TermTable t;
  std::string e;
  if (!build_terms(n_spins, n_bonds, pbonds.data(), pJ.data(), site_h ? ph.data() : nullptr, t, e))
    return ctx->fail(LREI_E_INVALID, e);
  // terms by the highest row bit they flip: for any tile of 2^k rows the
  // terms that stay inside it are a prefix of the table
  std::stable_sort(t.off.begin(), t.off.end(), [](const OffTerm &x, const OffTerm &y) {
    return 31 - __builtin_clz(x.mask) < 31 - __builtin_clz(y.mask);
  });
  HIPCHK(hipSetDevice(ctx->device));
  DevTerms dt;
  const lrei_status ust = upload_terms(t, 1LL << n_spins, ctx->stream, dt, e);
  if (ust != LREI_OK) return ctx->fail(ust, e);
  ctx->dt.release();
  ctx->dt = dt;
  ctx->sweeps.clear();  // term tables are in their natural order: one sweep
  ctx->hv_w = 0;
  ctx->terms = t;
  if (ctx->have_rho && ctx->site_pos != pos) {
    // the stored state follows the previous site order: move it to the new one
    const size_t vb = (size_t)ctx->N * ctx->r * ctx->elem();
    (void)vb;
    launch_permute(ctx->fp32, ctx->blocks[0].p, ctx->acc.p, ctx->N, ctx->r, ctx->site_pos.data(), n_spins, true,
                   ctx->stream);
    launch_permute(ctx->fp32, ctx->acc.p, ctx->blocks[0].p, ctx->N, ctx->r, pos.data(), n_spins, false, ctx->stream);
    // the low part of a compensated state is not moved: it restarts at zero
    if (ctx->fp32) HIPCHK(hipMemsetAsync(ctx->lo.p, 0, ctx->lo_bytes(), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ab_reset(ctx);
  }
  ctx->site_pos = pos;
  ctx->n = n_spins;
  ctx->N = 1LL << n_spins;
  ctx->hbar = hbar;
  ctx->have_h = true;
  ctx->drop_graph();
  return LREI_OK;
}

lrei_status lrei_set_rho(lrei_ctx *ctx, int r, const double *lambda, const void *V, int v_is_device) {
  if (!ctx) return LREI_E_INVALID;
  if (!ctx->have_h) return ctx->fail(LREI_E_STATE, "set a Hamiltonian before rho");
  if (r < 1 || r > kMaxR) return ctx->fail(LREI_E_INVALID, "r must be in [1, 32]");
  if ((long long)r > ctx->N) return ctx->fail(LREI_E_INVALID, "r exceeds the Hilbert dimension");
  if (!lambda || !V) return ctx->fail(LREI_E_INVALID, "null lambda or V");
  for (int i = 0; i < r; ++i) {
    if (!std::isfinite(lambda[i]) || !(lambda[i] > 0))
      return ctx->fail(LREI_E_INVALID, "lambda must be finite and strictly positive");
    if (i > 0 && lambda[i] > lambda[i - 1]) return ctx->fail(LREI_E_INVALID, "lambda must be non-increasing");
  }
  HIPCHK(hipSetDevice(ctx->device));
  // Validate in temporaries first so that a rejected V leaves the state intact.
  const size_t el = ctx->elem();
  const size_t vbytes = (size_t)ctx->N * r * el;
  const int grid = nspace_grid(ctx->N, r);
  // FP64: V -> tv, natural -> internal site order into tp.  Mixed: V (FP64)
  // -> internal order in tw, split into the compensated FP32 pair tp (hi) +
  // tlo (lo).  The validation pass below measures V* V and V* (beta H V) on
  // tp with the context's term tables (tv: its scratch output).
  const size_t n64 = (size_t)ctx->N * r * sizeof(double2);
  DevBuf tv, tp, tpart, tmeas, tstage, tw, tlo;
  auto release_tmp = [&]() {
    tv.release(); tp.release(); tpart.release(); tmeas.release(); tstage.release(); tw.release(); tlo.release();
  };
  if (!tv.ensure(vbytes) || !tp.ensure(vbytes) ||
      !tpart.ensure((size_t)grid * hv_partial_splits(r) * 3 * r * r * sizeof(double2)) ||
      !tmeas.ensure(3 * (size_t)r * r * sizeof(double2)) ||
      (ctx->fp32 && (!tw.ensure(n64) || !tlo.ensure((size_t)ctx->N * r * 4) ||
                     (!v_is_device && !tstage.ensure(n64))))) {
    release_tmp();
    return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  }
  {
    const size_t n = (size_t)ctx->N * r;
    hipError_t e1 = hipSuccess;
    if (!ctx->fp32) {
      e1 = hipMemcpyAsync(tv.p, V, n * sizeof(double2), v_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          ctx->stream);
      if (e1 == hipSuccess)
        launch_permute(false, tv.p, tp.p, ctx->N, r, ctx->site_pos.data(), ctx->n, false, ctx->stream);
    } else {
      const void *src = V;
      if (!v_is_device) {
        e1 = hipMemcpyAsync(tstage.p, V, n * sizeof(double2), hipMemcpyHostToDevice, ctx->stream);
        src = tstage.p;
      }
      if (e1 == hipSuccess) {
        launch_permute(false, src, tw.p, ctx->N, r, ctx->site_pos.data(), ctx->n, false, ctx->stream);
        launch_split((const double2 *)tw.p, (float2 *)tp.p, tlo.p, (long long)n, ctx->stream);
      }
    }
    if (e1 != hipSuccess) {
      release_tmp();
      return check_hip(ctx, e1, "upload V");
    }
  }
  if (!hv_pass_into(ctx, r, grid, 0, tp.p, tv.p, (double2 *)tpart.p, (double2 *)tmeas.p, false, grid)) {
    release_tmp();
    return ctx->fail(LREI_E_INVALID, "no H.V launch shape for rank " + std::to_string(r));
  }
  std::vector<double2> g(3 * r * r);
  hipError_t e2 = hipGetLastError();
  if (e2 == hipSuccess)
    e2 = hipMemcpyAsync(g.data(), tmeas.p, g.size() * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream);
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(ctx->stream);
  if (e2 != hipSuccess) {
    release_tmp();
    return check_hip(ctx, e2, "validate V");
  }
  double dev = 0;
  bool finite = true;
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) {
      double2 v = g[a * r + b];
      if (!std::isfinite(v.x) || !std::isfinite(v.y)) finite = false;
      if (a == b) v.x -= 1.0;
      dev = std::max(dev, std::sqrt(v.x * v.x + v.y * v.y));
    }
  const double tol = ctx->fp32 ? 1e-5 : 1e-10;
  if (!finite || !(dev <= tol)) {
    release_tmp();
    return ctx->fail(LREI_E_INVALID, "V must have finite orthonormal columns (max |V*V - I| = " +
                                         std::to_string(dev) + ")");
  }
  if (!ctx->have_rho || ctx->r != r) reset_hv_tuning(ctx);  // the tuned shape belongs to the old rank
  lrei_status st = alloc_state(ctx, r, ctx->fp32);
  if (st != LREI_OK) {
    release_tmp();
    ctx->have_rho = false;
    return st;
  }
  ctx->r = r;
  // a new state: every stage tries the warm-started eigensolve again
  e2 = hipMemsetAsync(ctx->ws.warm_skip, 0, 2 * kMaxStages * sizeof(double), ctx->stream);
  // a new state: the first Krylov block's column shifts are the Rayleigh
  // quotients of V's columns (the validation pass measured P0* P1 with
  // P1 = beta H V), the later blocks' start at zero; every step refreshes them
  std::vector<double> sh0((size_t)kMaxBlocks * r, 0.0);
  for (int a = 0; a < r; ++a) {
    const double gaa = g[a * r + a].x, haa = g[r * r + a * r + a].x / krylov_beta(ctx);
    if (gaa > 0 && std::isfinite(haa / gaa)) sh0[a] = haa / gaa;
  }
  if (e2 == hipSuccess)
    e2 = hipMemcpyAsync(ctx->ws.shifts, sh0.data(), sh0.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(ctx->stream);  // sh0 is host stack memory
  if (e2 == hipSuccess) e2 = hipMemcpyAsync(ctx->blocks[0].p, tp.p, vbytes, hipMemcpyDeviceToDevice, ctx->stream);
  if (e2 == hipSuccess && ctx->fp32)
    e2 = hipMemcpyAsync(ctx->lo.p, tlo.p, (size_t)ctx->N * r * 4, hipMemcpyDeviceToDevice, ctx->stream);
  if (e2 == hipSuccess) e2 = hipGetLastError();
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(ctx->stream);
  release_tmp();
  HIPCHK(e2);
  ctx->lam.assign(lambda, lambda + r);
  ctx->have_rho = true;
  ctx->steps_done = 0;
  ab_reset(ctx);
  ctx->drop_graph();
  return LREI_OK;
}

lrei_status lrei_step(lrei_ctx *ctx, int model, int scheme, double dt, double kappa, int n_steps) {
  if (!ctx) return LREI_E_INVALID;
  if (!ctx->have_rho) return ctx->fail(LREI_E_STATE, "set rho before stepping");
  if (model != LREI_QLL && model != LREI_QLLG) return ctx->fail(LREI_E_INVALID, "unknown model");
  const bool is_ab = scheme >= LREI_AB2 && scheme <= LREI_AB4;
  if (!(scheme >= LREI_RK1 && scheme <= LREI_RK4) && !is_ab)
    return ctx->fail(LREI_E_INVALID, "unsupported scheme (RK1..RK4, AB2..AB4)");
  if (!(dt > 0) || !std::isfinite(dt)) return ctx->fail(LREI_E_INVALID, "dt must be positive and finite");
  if (!(kappa >= 0) || !std::isfinite(kappa)) return ctx->fail(LREI_E_INVALID, "kappa must be >= 0 and finite");
  if (n_steps < 0) return ctx->fail(LREI_E_INVALID, "n_steps must be >= 0");
  // the low-rank part of a state with a maximally mixed admixture evolves with
  // damping (1 - p) kappa (Sec. 5, a full-rank state)
  kappa *= 1.0 - ctx->mix_p;
  if (!is_ab && ctx->opt.warm == LREI_WARM_LEARNED && (!ctx->net || ctx->net_r != ctx->r))
    return ctx->fail(LREI_E_STATE, "LREI_WARM_LEARNED needs an attached network of the state's rank");
  if (is_ab) {
    const int m = ab_order(scheme);
    if (ctx->r > 16) return ctx->fail(LREI_E_INVALID, "AB schemes support r <= 16");
    if ((long long)(2 * m + 2) * ctx->r > ctx->N)
      return ctx->fail(LREI_E_INVALID, "AB schemes need N >= (2m + 2) r");
  }
  if (n_steps == 0) return LREI_OK;
  HIPCHK(hipSetDevice(ctx->device));
  if (is_ab) {
    auto &ab = ctx->ab;
    if (!(ab.valid && ab.scheme == scheme && ab.model == model && ab.dt == dt && ab.kappa == kappa)) {
      // a new AB run: the history is rebuilt from the current state
      ab_reset(ctx);
      ab.scheme = scheme;
      ab.m = ab_order(scheme);
      ab.model = model;
      ab.dt = dt;
      ab.kappa = kappa;
      lrei_status st = ab_alloc(ctx, ab.m);
      if (st != LREI_OK) return st;
      ab.valid = true;
    }
  } else {
    ab_reset(ctx);  // an RK step moves the state outside any AB history
  }
  const auto t0 = std::chrono::steady_clock::now();
  const size_t vbytes = (size_t)ctx->N * ctx->r * ctx->elem();
  HIPCHK(hipMemcpyAsync(ctx->save.p, ctx->blocks[0].p, vbytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (ctx->fp32) HIPCHK(hipMemcpyAsync(ctx->save_lo.p, ctx->lo.p, ctx->lo_bytes(), hipMemcpyDeviceToDevice, ctx->stream));
  double zeros[kStatsLen] = {0};
  HIPCHK(hipMemcpyAsync(ctx->stats_buf.p, zeros, sizeof(zeros), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->hv_launch_failed = false;
  if (is_ab) {
    for (int k = 0; k < n_steps; ++k) enqueue_ab_step(ctx);
  } else {
    // mixed precision: every kGuardSteps steps (and at the end) the smallest
    // Cholesky pivot ratio of the last step is checked against the floor
    // below which the FP32 blocks no longer resolve the Krylov directions
    const bool guard = ctx->fp32 && ctx->opt.mixed_pivot_floor > 0;
    int left = n_steps;
    while (left > 0) {
      const int k = guard && ctx->fp32 ? std::min(left, kGuardSteps) : left;
      lrei_status rs = run_rk_steps(ctx, model, scheme, dt, kappa, k);
      if (rs != LREI_OK) return rs;
      left -= k;
      if (guard && ctx->fp32) {
        double piv = 1.0;
        HIPCHK(hipMemcpyAsync(&piv, ctx->ws.stats + 3, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (piv < ctx->opt.mixed_pivot_floor) {
          rs = promote_fp64(ctx);
          if (rs != LREI_OK) return rs;
        }
      }
    }
  }
  HIPCHK(hipGetLastError());
  double h[kStatsLen];
  lrei_status st = read_stats(ctx, h);
  if (st != LREI_OK) return st;
  const auto t1 = std::chrono::steady_clock::now();
  // stats[0..8] describe the last step, stats[10..15] the whole call
  const bool bad = h[14] != 0 || (ctx->opt.fail_after_steps > 0 && n_steps >= ctx->opt.fail_after_steps);
  if (bad || ctx->hv_launch_failed) {
    ab_reset(ctx);  // the history no longer matches the restored state
    HIPCHK(hipMemcpyAsync(ctx->blocks[0].p, ctx->save.p, (size_t)ctx->N * ctx->r * ctx->elem(),
                          hipMemcpyDeviceToDevice, ctx->stream));
    if (ctx->fp32)
      HIPCHK(hipMemcpyAsync(ctx->lo.p, ctx->save_lo.p, ctx->lo_bytes(), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->hv_launch_failed) {
      ctx->hv_launch_failed = false;
      return ctx->fail(LREI_E_INVALID, "an H.V pass could not be launched for this rank; state restored to the "
                                       "start of the call");
    }
    char where[96] = "";
    if (h[28] >= 0)
      std::snprintf(where, sizeof(where), " (first at stage %d, %s)", (int)h[28] / 10,
                    (const char *[]){"", "u", "H u", "z/w", "stage matrix", "eigenvectors"}[(int)h[28] % 10]);
    return ctx->fail(LREI_E_NUMERIC,
                     std::string("non-finite values in the step") + where + "; state restored to the start of the call");
  }
  ctx->steps_done += n_steps;
  ctx->stats.steps_done = ctx->steps_done;
  ctx->stats.eigensolves += (int64_t)h[11];
  ctx->stats.warm_accepted += (int64_t)h[9];
  ctx->stats.warm_rejected += (int64_t)h[31];
  ctx->stats.warm_iterations += (int64_t)h[12];
  ctx->stats.dropped_directions = (int32_t)h[2];
  ctx->stats.min_pivot_ratio = h[3];
  ctx->stats.ortho_error = h[4];
  ctx->stats.energy = h[5];
  ctx->stats.last_step_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  for (int k = 0; k < 8; ++k) ctx->stats.phase_ms[k] = h[16 + k];
  for (int k = 0; k < 4; ++k) ctx->stats.eig_phase_ms[k] = h[24 + k];
  ctx->stats.eig_phase_ms[4] = h[29];
  ctx->stats.eig_phase_ms[5] = h[30];
  return LREI_OK;
}

lrei_status lrei_evolve_adaptive(lrei_ctx *ctx, int model, int pair, double kappa, double t_span, double tol,
                                 double h_init, double h_min, double h_max, int max_attempts,
                                 lrei_adapt_result *out) {
  if (!ctx) return LREI_E_INVALID;
  if (out) {
    *out = lrei_adapt_result{};
    out->err_last = NAN;
  }
  if (!ctx->have_rho) return ctx->fail(LREI_E_STATE, "set rho before stepping");
  if (model != LREI_QLL && model != LREI_QLLG) return ctx->fail(LREI_E_INVALID, "unknown model");
  if (pair != LREI_PAIR_HE21 && pair != LREI_PAIR_BS32 && pair != LREI_PAIR_RK43)
    return ctx->fail(LREI_E_INVALID, "unknown embedded pair (LREI_PAIR_HE21, LREI_PAIR_BS32, LREI_PAIR_RK43)");
  if (!(t_span > 0) || !std::isfinite(t_span)) return ctx->fail(LREI_E_INVALID, "t_span must be positive and finite");
  if (!(tol > 0) || !std::isfinite(tol)) return ctx->fail(LREI_E_INVALID, "tol must be positive and finite");
  if (!(h_min > 0) || !(h_init >= h_min) || !(h_max >= h_min) || !std::isfinite(h_init) || std::isnan(h_max))
    return ctx->fail(LREI_E_INVALID, "need 0 < h_min <= h_init and h_min <= h_max");
  if (max_attempts < 1) return ctx->fail(LREI_E_INVALID, "max_attempts must be >= 1");
  if (!(kappa >= 0) || !std::isfinite(kappa)) return ctx->fail(LREI_E_INVALID, "kappa must be >= 0 and finite");
  kappa *= 1.0 - ctx->mix_p;  // damping of the low-rank part (full-rank admixture)
  if (ctx->opt.warm == LREI_WARM_LEARNED && (!ctx->net || ctx->net_r != ctx->r))
    return ctx->fail(LREI_E_STATE, "LREI_WARM_LEARNED needs an attached network of the state's rank");
  HIPCHK(hipSetDevice(ctx->device));
  ab_reset(ctx);
  if (!ctx->ctl.ensure(kCtlLen * sizeof(double))) return ctx->fail(LREI_E_NOMEM, "allocation failed");
  const auto t0 = std::chrono::steady_clock::now();
  const size_t vbytes = (size_t)ctx->N * ctx->r * ctx->elem();
  HIPCHK(hipMemcpyAsync(ctx->save.p, ctx->blocks[0].p, vbytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (ctx->fp32) HIPCHK(hipMemcpyAsync(ctx->save_lo.p, ctx->lo.p, ctx->lo_bytes(), hipMemcpyDeviceToDevice, ctx->stream));
  double zeros[kStatsLen] = {0};
  HIPCHK(hipMemcpyAsync(ctx->stats_buf.p, zeros, sizeof(zeros), hipMemcpyHostToDevice, ctx->stream));
  double c[kCtlLen] = {0};
  c[kCtlH] = std::min(std::min(h_init, h_max), t_span);
  c[kCtlTEnd] = t_span;
  c[kCtlTol] = tol;
  c[kCtlHMin] = h_min;
  c[kCtlHMax] = h_max;
  HIPCHK(hipMemcpyAsync(ctx->ctl.p, c, sizeof(c), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->hv_launch_failed = false;
  SmallRkParams p = adapt_params(ctx, model, pair, kappa);
  const bool use_graph = ctx->opt.use_graph != 0;
  const bool guard = ctx->fp32 && ctx->opt.mixed_pivot_floor > 0;
  int launched = 0;
  // the captured attempt (captured first when the attempt differs from the
  // last one captured; the eager attempt that sets the launch attributes,
  // outside capture, is an attempt of its own)
  auto ensure_graph = [&]() -> lrei_status {
    if (!use_graph || (ctx->exec && ctx->g_model == model && ctx->g_scheme == pair && ctx->g_dt < 0 &&
                       ctx->g_kappa == kappa))
      return LREI_OK;
    ctx->drop_graph();
    enqueue_attempt(ctx, p);
    HIPCHK(hipGetLastError());
    ++launched;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    enqueue_attempt(ctx, p);
    HIPCHK(hipStreamEndCapture(ctx->stream, &ctx->graph));
    HIPCHK(hipGraphInstantiate(&ctx->exec, ctx->graph, nullptr, nullptr, 0));
    ctx->g_model = model;
    ctx->g_scheme = pair;
    ctx->g_dt = -1.0;
    ctx->g_kappa = kappa;
    return LREI_OK;
  };
  // batches of attempts between reads of the controller state: as many as
  // the current step needs to reach t_span (at most 16); attempts queued
  // after the end do nothing.  Mixed precision: the conditioning floor is
  // checked after every batch (the last attempt's smallest pivot ratio).
  for (;;) {
    lrei_status gs = ensure_graph();
    if (gs != LREI_OK) return gs;
    HIPCHK(hipMemcpyAsync(c, ctx->ctl.p, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (guard && ctx->fp32 && c[kCtlAttempts] > 0) {
      double piv = 1.0;
      HIPCHK(hipMemcpyAsync(&piv, ctx->ws.stats + 3, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      if (piv < ctx->opt.mixed_pivot_floor) {
        gs = promote_fp64(ctx);
        if (gs != LREI_OK) return gs;
        p = adapt_params(ctx, model, pair, kappa);
        gs = ensure_graph();
        if (gs != LREI_OK) return gs;
        HIPCHK(hipMemcpyAsync(c, ctx->ctl.p, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
      }
    }
    if (c[kCtlDone] != 0.0 || c[kCtlFailed] != 0.0 || launched >= max_attempts) break;
    const double need = std::ceil((t_span - c[kCtlT]) / c[kCtlH]);
    int batch = need >= 16.0 ? 16 : (need < 1.0 ? 1 : (int)need);
    batch = std::min(batch, max_attempts - launched);
    for (int k = 0; k < batch; ++k) {
      if (use_graph)
        HIPCHK(hipGraphLaunch(ctx->exec, ctx->stream));
      else
        enqueue_attempt(ctx, p);
    }
    HIPCHK(hipGetLastError());
    launched += batch;
  }
  double h[kStatsLen];
  lrei_status st = read_stats(ctx, h);
  if (st != LREI_OK) return st;
  const auto t1 = std::chrono::steady_clock::now();
  if (ctx->hv_launch_failed) {
    ctx->hv_launch_failed = false;
    HIPCHK(hipMemcpyAsync(ctx->blocks[0].p, ctx->save.p, (size_t)ctx->N * ctx->r * ctx->elem(),
                          hipMemcpyDeviceToDevice, ctx->stream));
    if (ctx->fp32)
      HIPCHK(hipMemcpyAsync(ctx->lo.p, ctx->save_lo.p, ctx->lo_bytes(), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return ctx->fail(LREI_E_INVALID,
                     "an H.V pass could not be launched for this rank; state restored to the start of the call");
  }
  const bool reached = c[kCtlDone] != 0.0;
  if (out) {
    out->t = c[kCtlT];
    out->h_next = c[kCtlH];
    out->err_last = c[kCtlErr];
    out->err_max = c[kCtlErrMax];
    out->accepted = (int)c[kCtlAccepted];
    out->rejected = (int)c[kCtlRejected];
    out->attempts = (int)c[kCtlAttempts];
    out->reached = reached ? 1 : 0;
  }
  ctx->steps_done += (int64_t)c[kCtlAccepted];
  ctx->stats.steps_done = ctx->steps_done;
  ctx->stats.eigensolves += (int64_t)h[11];
  ctx->stats.warm_accepted += (int64_t)h[9];
  ctx->stats.warm_rejected += (int64_t)h[31];
  ctx->stats.warm_iterations += (int64_t)h[12];
  ctx->stats.dropped_directions = (int32_t)h[2];
  ctx->stats.min_pivot_ratio = h[3];
  ctx->stats.ortho_error = h[4];
  ctx->stats.energy = h[5];
  ctx->stats.last_step_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  for (int k = 0; k < 8; ++k) ctx->stats.phase_ms[k] = h[16 + k];
  for (int k = 0; k < 4; ++k) ctx->stats.eig_phase_ms[k] = h[24 + k];
  ctx->stats.eig_phase_ms[4] = h[29];
  ctx->stats.eig_phase_ms[5] = h[30];
  if (reached) return LREI_OK;
  char msg[160];
  if (c[kCtlFailed] != 0.0)
    std::snprintf(msg, sizeof(msg), "an attempt at h <= h_min was rejected at t = %.6g; state of the last accepted step",
                  c[kCtlT]);
  else
    std::snprintf(msg, sizeof(msg), "max_attempts reached at t = %.6g; state of the last accepted step", c[kCtlT]);
  return ctx->fail(LREI_E_NOTCONVERGED, msg);
}

lrei_status lrei_get_rho(lrei_ctx *ctx, double *lambda, void *V, int v_is_device) {
  if (!ctx) return LREI_E_INVALID;
  if (!ctx->have_rho) return ctx->fail(LREI_E_STATE, "no state");
  if (lambda) std::memcpy(lambda, ctx->lam.data(), ctx->r * sizeof(double));
  if (!V) return LREI_OK;
  HIPCHK(hipSetDevice(ctx->device));
  const size_t n = (size_t)ctx->N * ctx->r;
  if (!ctx->fp32) {  // back to the physical site order
    launch_permute(false, ctx->blocks[0].p, ctx->acc.p, ctx->N, ctx->r, ctx->site_pos.data(), ctx->n, true,
                   ctx->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(V, ctx->acc.p, n * sizeof(double2),
                          v_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return LREI_OK;
  }
  // the compensated pair hi + lo in FP64, then the physical site order
  DevBuf w64, p64;
  if (!w64.ensure(n * sizeof(double2)) || (!v_is_device && !p64.ensure(n * sizeof(double2))))
    return ctx->fail(LREI_E_NOMEM, "allocation failed");
  launch_merge((const float2 *)ctx->blocks[0].p, ctx->lo.p, (double2 *)w64.p, (long long)n,
               ctx->stream);
  void *dst = v_is_device ? V : p64.p;
  launch_permute(false, w64.p, dst, ctx->N, ctx->r, ctx->site_pos.data(), ctx->n, true, ctx->stream);
  HIPCHK(hipGetLastError());
  if (!v_is_device) HIPCHK(hipMemcpyAsync(V, p64.p, n * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LREI_OK;
}

lrei_status lrei_get_rank(lrei_ctx *ctx, int *r) {
  if (!ctx || !r) return LREI_E_INVALID;
  if (!ctx->have_rho) return ctx->fail(LREI_E_STATE, "no state");
  *r = ctx->r;
  return LREI_OK;
}

lrei_status lrei_set_rho_factor(lrei_ctx *ctx, int m, const void *A, int a_is_device) {
  if (!ctx) return LREI_E_INVALID;
  if (ctx->N <= 0) return ctx->fail(LREI_E_STATE, "set the Hamiltonian first");
  if (m < 1 || m > kMaxR || m > ctx->N || !A) return ctx->fail(LREI_E_INVALID, "need 1 <= m <= min(32, N) and A");
  HIPCHK(hipSetDevice(ctx->device));
  const long long N = ctx->N;
  const int np = m * (m + 1) / 2;
  const int grid = (int)std::min<long long>(256, std::max<long long>(1, N / 256));
  DevBuf ad, part, cm, lamd, info, vd;
  if ((!a_is_device && !ad.ensure((size_t)N * m * sizeof(double2))) ||
      !part.ensure((size_t)grid * np * sizeof(double2)) || !cm.ensure((size_t)m * m * sizeof(double2)) ||
      !lamd.ensure((size_t)m * sizeof(double)) || !info.ensure(sizeof(int)))
    return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  const double2 *Ad = a_is_device ? (const double2 *)A : (const double2 *)ad.p;
  hipError_t e = hipSuccess;
  if (!a_is_device)
    e = hipMemcpyAsync(ad.p, A, (size_t)N * m * sizeof(double2), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    launch_factor_eig(Ad, N, m, (double2 *)part.p, grid, (double2 *)cm.p, (double *)lamd.p, (int *)info.p,
                      ctx->stream);
    e = hipGetLastError();
  }
  int rank = 0;
  std::vector<double> lam(m);
  if (e == hipSuccess) e = hipMemcpyAsync(&rank, info.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(lam.data(), lamd.p, m * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return ctx->fail(LREI_E_DEVICE, std::string("factor eigensolve: ") + hipGetErrorString(e));
  if (rank < 1) return ctx->fail(LREI_E_INVALID, "the factor is zero or not finite");
  if (!vd.ensure((size_t)N * rank * sizeof(double2))) return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  launch_factor_apply(Ad, N, m, (const double2 *)cm.p, rank, (double2 *)vd.p, ctx->stream);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  ad.release();
  part.release();
  if (e != hipSuccess) return ctx->fail(LREI_E_DEVICE, std::string("factor apply: ") + hipGetErrorString(e));
  lam.resize(rank);
  return lrei_set_rho(ctx, rank, lam.data(), vd.p, 1);
}

lrei_status lrei_set_mixing(lrei_ctx *ctx, double p) {
  if (!ctx) return LREI_E_INVALID;
  if (!(p >= 0.0 && p < 1.0)) return ctx->fail(LREI_E_INVALID, "p must be in [0, 1)");
  ctx->mix_p = p;
  ab_reset(ctx);      // the AB history holds right-hand sides at the old damping
  ctx->drop_graph();  // the damping is a launch argument
  return LREI_OK;
}

lrei_status lrei_pair_density(lrei_ctx *ctx, int n_pairs, const int *pairs, double *out) {
  if (!ctx) return LREI_E_INVALID;
  if (!ctx->have_rho) return ctx->fail(LREI_E_STATE, "no state");
  if (n_pairs < 1 || n_pairs > 4096 || !pairs || !out)
    return ctx->fail(LREI_E_INVALID, "n_pairs must be 1..4096 with host pair and output arrays");
  std::vector<int> bits(2 * (size_t)n_pairs);
  for (int p = 0; p < n_pairs; ++p) {
    const int k = pairs[2 * p], l = pairs[2 * p + 1];
    if (k < 0 || l < 0 || k >= ctx->n || l >= ctx->n || k == l)
      return ctx->fail(LREI_E_INVALID, "pair " + std::to_string(p) + ": sites must be distinct and < n");
    bits[2 * p] = ctx->site_pos[k];
    bits[2 * p + 1] = ctx->site_pos[l];
  }
  HIPCHK(hipSetDevice(ctx->device));
  const int r = ctx->r;
  const int grid = (int)std::min<long long>(256, std::max<long long>(1, (ctx->N / 4) / 1024));
  DevBuf db, part, res;
  if (!db.ensure(bits.size() * sizeof(int)) || !part.ensure((size_t)n_pairs * grid * 10 * sizeof(double2)) ||
      !res.ensure((size_t)n_pairs * 16 * sizeof(double2)))
    return ctx->fail(LREI_E_NOMEM, "device allocation failed");
  hipError_t e = hipMemcpyAsync(ctx->lam_dev.p, ctx->lam.data(), r * sizeof(double), hipMemcpyHostToDevice,
                                ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(db.p, bits.data(), bits.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    launch_pair_density(ctx->fp32, ctx->blocks[0].p, (const double *)ctx->lam_dev.p, ctx->N, r, (const int *)db.p,
                        n_pairs, grid, (double2 *)part.p, (double2 *)res.p, 1.0 - ctx->mix_p, 0.25 * ctx->mix_p,
                        ctx->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, res.p, (size_t)n_pairs * 16 * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  db.release();
  part.release();
  res.release();
  if (e != hipSuccess) return ctx->fail(LREI_E_DEVICE, std::string("pair density: ") + hipGetErrorString(e));
  return LREI_OK;
}

lrei_status lrei_observables(lrei_ctx *ctx, double *energy, double magnetization[3]) {
  if (!ctx) return LREI_E_INVALID;
  if (!ctx->have_rho) return ctx->fail(LREI_E_STATE, "no state");
  HIPCHK(hipSetDevice(ctx->device));
  const int r = ctx->r;
  if (energy) {
    // the step's first pass without column shifts, P1 = beta H P0, and its
    // Gram P0* P1 = beta V* H V
    krylov_pass(ctx, 0, false);
    HIPCHK(hipGetLastError());
    std::vector<double2> g(3 * r * r);
    HIPCHK(hipMemcpyAsync(g.data(), ctx->ws.meas, g.size() * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double e = 1.0 / krylov_beta(ctx);
    double en = 0;
    for (int a = 0; a < r; ++a) en += ctx->lam[a] * g[r * r + a * r + a].x * e;
    // Tr(H) = 0 (every Pauli-string term is traceless): the maximally mixed
    // part adds nothing
    *energy = (1.0 - ctx->mix_p) * en;
  }
  if (magnetization) {
    HIPCHK(hipMemcpyAsync(ctx->lam_dev.p, ctx->lam.data(), r * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    const int grid = std::min<long long>(1024, std::max<long long>(1, ctx->N / 64));
    double2 *part = (double2 *)ctx->partials.p;
    launch_magnetization(ctx->fp32, ctx->blocks[0].p, (const double *)ctx->lam_dev.p, ctx->N, r, ctx->n, part, grid,
                         ctx->stream);
    HIPCHK(hipGetLastError());
    std::vector<double2> h(2 * grid);
    HIPCHK(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double mx = 0, my = 0, mz = 0;
    for (int i = 0; i < grid; ++i) {
      mx += h[2 * i].x;
      my += h[2 * i].y;
      mz += h[2 * i + 1].x;
    }
    const double f = (1.0 - ctx->mix_p) * 0.5 * ctx->hbar / ctx->n;
    magnetization[0] = f * mx;
    magnetization[1] = f * my;
    magnetization[2] = f * mz;
  }
  return LREI_OK;
}

lrei_status lrei_get_stats(lrei_ctx *ctx, lrei_stats *s) {
  if (!ctx || !s) return LREI_E_INVALID;
  *s = ctx->stats;
  return LREI_OK;
}

}  // extern "C"

namespace {

// Y = H X on the context stream for device blocks in the natural site order:
// X -> internal order (ta), H (FP64 pass, mode 2) into tb, back to the natural
// order into Y (Y may alias ta).  Returns false if no launch shape fits r.
bool enqueue_apply_h(lrei_ctx *ctx, int r, const void *X, void *Y, void *ta, void *tb) {
  launch_permute(false, X, ta, ctx->N, r, ctx->site_pos.data(), ctx->n, false, ctx->stream);
  HvArgs a{};
  a.Pcur = ta;
  a.Pnext = tb;
  hv_args(ctx, a);
  a.N = ctx->N;
  a.r = r;
  if (!hv_epl_valid(false, r, a.epl)) a.epl = 0;  // FP64 launch; the tuned shape may be FP32's
  a.alpha = 1.0;
  a.mode = 2;
  a.grid = nspace_grid(ctx->N, r);
  if (launch_hv(false, a, ctx->stream) <= 0) return false;
  launch_permute(false, tb, Y, ctx->N, r, ctx->site_pos.data(), ctx->n, true, ctx->stream);
  return true;
}

}  // namespace

extern "C" {

lrei_status lrei_apply_hamiltonian_noalloc(lrei_ctx *ctx, int r, const void *X, void *Y) {
  if (!ctx) return LREI_E_INVALID;
  if (!ctx->have_h) return ctx->fail(LREI_E_STATE, "no Hamiltonian");
  if (r < 1 || r > kMaxR || !X || !Y) return ctx->fail(LREI_E_INVALID, "bad arguments");
  const size_t bytes = (size_t)ctx->N * r * sizeof(double2);
  if (2 * bytes > kScratchBytes)
    return ctx->fail(LREI_E_INVALID, "N r = " + std::to_string(ctx->N * r) + " complex values exceed the " +
                                         std::to_string(kScratchBytes / (2 * sizeof(double2))) +
                                         " that the static scratch holds (2 N r complex128 <= 64 MiB)");
  char *base = (char *)g_scratch_addr[ctx->device];  // resolved by lrei_create on this device
  if (!base) return ctx->fail(LREI_E_DEVICE, "scratch address not resolved on this device");
  HIPCHK(hipSetDevice(ctx->device));
  if (!enqueue_apply_h(ctx, r, X, Y, base, base + bytes))
    return ctx->fail(LREI_E_INVALID, "no H.V launch shape for this rank");
  return check_hip(ctx, hipGetLastError(), "apply_hamiltonian_noalloc launch");
}

lrei_status lrei_apply_hamiltonian(lrei_ctx *ctx, int r, const void *X, void *Y, int is_device) {
  if (!ctx) return LREI_E_INVALID;
  if (!ctx->have_h) return ctx->fail(LREI_E_STATE, "no Hamiltonian");
  if (r < 1 || r > kMaxR || !X || !Y) return ctx->fail(LREI_E_INVALID, "bad arguments");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t bytes = (size_t)ctx->N * r * sizeof(double2);
  DevBuf dx, dy, dp;
  auto release_all = [&]() {
    dx.release();
    dy.release();
    dp.release();
  };
  if (!dy.ensure(bytes) || !dp.ensure(bytes) || (!is_device && !dx.ensure(bytes))) {
    release_all();
    return ctx->fail(LREI_E_NOMEM, "allocation failed");
  }
  const void *px = X;
  if (!is_device) {
    lrei_status st0 = check_hip(ctx, hipMemcpyAsync(dx.p, X, bytes, hipMemcpyHostToDevice, ctx->stream), "upload X");
    if (st0 != LREI_OK) {
      release_all();
      return st0;
    }
    px = dx.p;
  }
  void *py = is_device ? Y : dp.p;
  if (!enqueue_apply_h(ctx, r, px, py, dp.p, dy.p)) {
    release_all();
    return ctx->fail(LREI_E_INVALID, "no H.V launch shape for this rank");
  }
  lrei_status st = check_hip(ctx, hipGetLastError(), "apply_hamiltonian launch");
  if (st == LREI_OK && !is_device)
    st = check_hip(ctx, hipMemcpyAsync(Y, dp.p, bytes, hipMemcpyDeviceToHost, ctx->stream), "copy back");
  if (st == LREI_OK) st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "sync");
  release_all();
  return st;
}

// Checkpoint layout (little-endian): 16 x uint64 header {magic, n, r, steps_done,
// fp32, ab_valid, ab_scheme, ab_model, ab_count, ab_nU, ab_npairs, dt bits,
// kappa bits, shifts flag, 0, 0}; lambda (r doubles); V (N x r complex128); with
// a valid AB history also the U Gram products, the U-coordinates of the history
// and the U blocks in the context's storage precision; then (shifts flag 1) the
// Krylov column shifts, kMaxBlocks x r doubles.  Buffers without the shifts
// (flag 0) are read too; their shifts start as set_rho's.
namespace {
constexpr uint64_t kStateMagic2 = 0x4c52454953543032ull;  // "LREIST02"
size_t ab_blob_bytes(const lrei_ctx::AbState &ab, size_t r, long long N, size_t elem) {
  if (!ab.valid) return 0;
  const size_t DU = (size_t)ab.nU * r;
  return ((size_t)ab.nU * (ab.nU + 1) / 2 * r * r + (1 + 2 * (size_t)ab.npairs) * DU * r) * sizeof(double2) +
         (size_t)ab.nU * (size_t)N * r * elem;
}
}  // namespace

lrei_status lrei_get_state(lrei_ctx *ctx, void *buf, size_t *len) {
  if (!ctx || !len) return LREI_E_INVALID;
  if (!ctx->have_rho) return ctx->fail(LREI_E_STATE, "no state");
  const size_t vbytes = (size_t)ctx->N * ctx->r * sizeof(double2);
  const size_t head = 16 * 8 + ctx->r * sizeof(double);
  const size_t abb = ab_blob_bytes(ctx->ab, ctx->r, ctx->N, ctx->elem());
  const size_t shb = (size_t)kMaxBlocks * ctx->r * sizeof(double);  // Krylov column shifts
  const size_t need = head + vbytes + abb + shb;
  if (!buf) {
    *len = need;
    return LREI_OK;
  }
  if (*len < need) return ctx->fail(LREI_E_INVALID, "buffer too small");
  const auto &ab = ctx->ab;
  uint64_t hdr[16] = {kStateMagic2, (uint64_t)ctx->n, (uint64_t)ctx->r, (uint64_t)ctx->steps_done,
                      (uint64_t)ctx->fp32, (uint64_t)ab.valid, (uint64_t)ab.scheme, (uint64_t)ab.model,
                      (uint64_t)ab.count, (uint64_t)ab.nU, (uint64_t)ab.npairs, 0, 0, 1, 0, 0};
  std::memcpy(&hdr[11], &ab.dt, 8);
  std::memcpy(&hdr[12], &ab.kappa, 8);
  std::memcpy(buf, hdr, sizeof(hdr));
  std::memcpy((char *)buf + 128, ctx->lam.data(), ctx->r * sizeof(double));
  *len = need;
  lrei_status st = lrei_get_rho(ctx, nullptr, (char *)buf + head, 0);
  if (st != LREI_OK) return st;
  // the column shifts of the Krylov recurrence (hdr[13] = 1), after the AB
  // blob: a resumed run then rounds exactly as the uninterrupted one
  HIPCHK(hipMemcpyAsync((char *)buf + head + vbytes + abb, ctx->ws.shifts, shb, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (!ab.valid) return LREI_OK;
  char *q = (char *)buf + head + vbytes;
  const size_t r = ctx->r, DU = (size_t)ab.nU * r;
  const size_t ub = (size_t)ab.nU * (ab.nU + 1) / 2 * r * r * sizeof(double2);
  const size_t cb = (1 + 2 * (size_t)ab.npairs) * DU * r * sizeof(double2);
  if (ub) HIPCHK(hipMemcpyAsync(q, ctx->ab_UUg.p, ub, hipMemcpyDeviceToHost, ctx->stream));
  q += ub;
  if (cb) HIPCHK(hipMemcpyAsync(q, ctx->ab_coords[ab.cur].p, cb, hipMemcpyDeviceToHost, ctx->stream));
  q += cb;
  const size_t blk = (size_t)ctx->N * r * ctx->elem();
  for (int i = 0; i < ab.nU; ++i, q += blk)
    HIPCHK(hipMemcpyAsync(q, ctx->ab_U[ab.cur][i].p, blk, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LREI_OK;
}

lrei_status lrei_set_state(lrei_ctx *ctx, const void *buf, size_t len) {
  if (!ctx || !buf || len < 32) return LREI_E_INVALID;
  uint64_t magic;
  std::memcpy(&magic, buf, 8);
  if (magic == kStateMagic) {  // rank-r state without AB history
    uint64_t hdr[4];
    std::memcpy(hdr, buf, sizeof(hdr));
    if (!ctx->have_h || (int)hdr[1] != ctx->n) return ctx->fail(LREI_E_STATE, "Hamiltonian with matching n required");
    const int r = (int)hdr[2];
    if (r < 1 || r > kMaxR) return ctx->fail(LREI_E_INVALID, "bad rank in state buffer");
    const size_t need = 32 + r * sizeof(double) + (size_t)ctx->N * r * sizeof(double2);
    if (len < need) return ctx->fail(LREI_E_INVALID, "state buffer truncated");
    const double *lam = (const double *)((const char *)buf + 32);
    lrei_status st = lrei_set_rho(ctx, r, lam, (const char *)buf + 32 + r * sizeof(double), 0);
    if (st != LREI_OK) return st;
    ctx->steps_done = (int64_t)hdr[3];
    return LREI_OK;
  }
  if (magic != kStateMagic2 || len < 128) return ctx->fail(LREI_E_INVALID, "not an LREI state buffer");
  uint64_t hdr[16];
  std::memcpy(hdr, buf, sizeof(hdr));
  if (!ctx->have_h || (int)hdr[1] != ctx->n) return ctx->fail(LREI_E_STATE, "Hamiltonian with matching n required");
  const int r = (int)hdr[2];
  if (r < 1 || r > kMaxR) return ctx->fail(LREI_E_INVALID, "bad rank in state buffer");
  const size_t head = 128 + r * sizeof(double), vbytes = (size_t)ctx->N * r * sizeof(double2);
  if (len < head + vbytes) return ctx->fail(LREI_E_INVALID, "state buffer truncated");
  lrei_ctx::AbState ab{};
  ab.valid = hdr[5] != 0;
  if (ab.valid) {
    if ((hdr[4] != 0) != ctx->fp32)
      return ctx->fail(LREI_E_INVALID, "AB history was saved at another storage precision");
    ab.scheme = (int)hdr[6];
    ab.m = ab_order(ab.scheme);
    ab.model = (int)hdr[7];
    ab.count = (int)hdr[8];
    ab.nU = (int)hdr[9];
    ab.npairs = (int)hdr[10];
    std::memcpy(&ab.dt, &hdr[11], 8);
    std::memcpy(&ab.kappa, &hdr[12], 8);
    if (ab.m < 2 || ab.m > kMaxAb || ab.nU < 0 || ab.nU > 2 * ab.m - 1 || ab.npairs < 0 || ab.npairs > ab.m - 1 ||
        r > 16)
      return ctx->fail(LREI_E_INVALID, "corrupt AB history in state buffer");
  }
  const lrei_ctx::AbState saved = ab;
  if (len < head + vbytes + ab_blob_bytes(ab, r, ctx->N, ctx->elem()))
    return ctx->fail(LREI_E_INVALID, "state buffer truncated");
  const double *lam = (const double *)((const char *)buf + 128);
  const size_t abb = ab_blob_bytes(ab, r, ctx->N, ctx->elem()), shb = (size_t)kMaxBlocks * r * sizeof(double);
  const bool with_shifts = hdr[13] == 1;
  if (with_shifts && len < head + vbytes + abb + shb) return ctx->fail(LREI_E_INVALID, "state buffer truncated");
  lrei_status st = lrei_set_rho(ctx, r, lam, (const char *)buf + head, 0);
  if (st != LREI_OK) return st;
  ctx->steps_done = (int64_t)hdr[3];
  if (with_shifts) {
    HIPCHK(hipMemcpyAsync(ctx->ws.shifts, (const char *)buf + head + vbytes + abb, shb, hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  if (!saved.valid) return LREI_OK;
  ctx->ab = saved;
  st = ab_alloc(ctx, saved.m);
  if (st != LREI_OK) {
    ab_reset(ctx);
    return st;
  }
  ctx->ab.cur = 0;
  const char *q = (const char *)buf + head + vbytes;
  const size_t DU = (size_t)saved.nU * r;
  const size_t ub = (size_t)saved.nU * (saved.nU + 1) / 2 * r * r * sizeof(double2);
  const size_t cb = (1 + 2 * (size_t)saved.npairs) * DU * r * sizeof(double2);
  if (ub) HIPCHK(hipMemcpyAsync(ctx->ab_UUg.p, q, ub, hipMemcpyHostToDevice, ctx->stream));
  q += ub;
  if (cb) HIPCHK(hipMemcpyAsync(ctx->ab_coords[0].p, q, cb, hipMemcpyHostToDevice, ctx->stream));
  q += cb;
  const size_t blk = (size_t)ctx->N * r * ctx->elem();
  for (int i = 0; i < saved.nU; ++i, q += blk)
    HIPCHK(hipMemcpyAsync(ctx->ab_U[0][i].p, q, blk, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LREI_OK;
}

lrei_status lrei_profile_kernels(lrei_ctx *ctx, int model, int scheme, double dt, double kappa, int iters,
                                 double ms[4]) {
  if (!ctx || !ms || iters < 1) return LREI_E_INVALID;
  if (!ctx->have_rho || ctx->steps_done < 1) return ctx->fail(LREI_E_STATE, "run one step first");
  if (!(scheme >= LREI_RK1 && scheme <= LREI_RK4)) return ctx->fail(LREI_E_INVALID, "RK schemes only");
  HIPCHK(hipSetDevice(ctx->device));
  const SmallRkParams p = rk_params(ctx, model, scheme, dt, kappa);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int r = ctx->r;
  int slots = ctx->hv_grid;  // Gram partial slots of the timed pass (set by its launch)
  auto timed = [&](int which) -> double {
    // one untimed launch, then `iters` timed ones
    for (int k = 0; k <= iters; ++k) {
      if (k == 1) (void)hipEventRecord(e0, ctx->stream);
      switch (which) {
        case 0:
          slots = hv_launches(ctx, r, ctx->hv_grid, 1, ctx->blocks[1].p, ctx->blocks[4].p,
                              (double2 *)ctx->partials.p, true, kMaxHvGrid, ctx->ws.shifts + r);
          break;
        case 1:
          launch_reduce((const double2 *)ctx->partials.p, slots, 2 * r * r,
                        ctx->ws.work, ctx->stream);  // scratch target: the step's Grams stay intact
          break;
        case 2:
          launch_small_rk(p, ctx->ws, ctx->stream);
          break;
        default: {
          const void *bl[kMaxBlocks];
          for (int i = 0; i <= p.s; ++i) bl[i] = ctx->blocks[i].p;
          launch_combine(ctx->fp32, bl, p.s + 1, ctx->ws.Cfin, ctx->save.p, ctx->N, r, combine_grid(ctx), ctx->stream,
                         nullptr, ctx->fp32 ? ctx->lo.p : nullptr, ctx->fp32 ? ctx->acc.p : nullptr);
        }
      }
    }
    (void)hipEventRecord(e1, ctx->stream);
    (void)hipEventSynchronize(e1);
    float t = 0;
    (void)hipEventElapsedTime(&t, e0, e1);
    return (double)t / iters;
  };
  for (int w = 0; w < 4; ++w) ms[w] = timed(w);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipGetLastError());
  return LREI_OK;
}

// Key of an H.V tuning result: device, problem shape and term table.
static std::string tune_key(lrei_ctx *ctx) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, ctx->device);
  std::string arch = prop.gcnArchName;
  for (auto &c : arch)
    if (c == ' ') c = '_';
  char buf[256];
  std::snprintf(buf, sizeof(buf), "lrei-hv %s %d %d %d %s %d %d", arch.c_str(), prop.multiProcessorCount, ctx->n,
                ctx->r, ctx->fp32 ? "mixed" : "fp64", ctx->dt.n_off, ctx->dt.cplx);
  return buf;
}

constexpr int kTuneMax = LREI_TUNE_MAX;

lrei_status lrei_autotune(lrei_ctx *ctx, lrei_tune_result *out) {
  if (!ctx) return LREI_E_INVALID;
  if (!ctx->have_rho) return ctx->fail(LREI_E_STATE, "set rho before tuning");
  HIPCHK(hipSetDevice(ctx->device));
  lrei_tune_result res{};
  const std::string key = tune_key(ctx);
  const char *cache = ctx->opt.autotune_cache;
  const int r = ctx->r;
  // variant code: 0 untiled, 1 untiled with compacted gathers, 100 k + w the
  // tiled pass with 2^k-row tiles and w waves
  const bool compact_ok = r <= 16 && ctx->dt.n_off <= 64;
  auto tile_valid = [&](int e, int g, int tile) {
    if (tile == 0) return true;
    if (tile == 1) return compact_ok;
    if (tile < 100) return false;
    const int tb = tile / 100, tw = tile % 100;
    return hv_tile_ok(ctx->fp32, r, e, tb, tw, ctx->N, g);
  };
  if (cache) {
    if (FILE *f = std::fopen(cache, "r")) {
      char line[512];
      while (std::fgets(line, sizeof(line), f)) {
        const std::string l(line);
        if (l.compare(0, key.size(), key) != 0 || l.size() <= key.size() || l[key.size()] != ' ') continue;
        int e = 0, g = 0, w = 0, tile = 0;
        double ms = 0;
        if (std::sscanf(l.c_str() + key.size(), " %d %d %d %d %lf", &e, &g, &w, &tile, &ms) == 5 && e > 0 &&
            hv_epl_valid(ctx->fp32, r, e) && g > 0 && g <= kMaxHvGrid && w >= 0 && w < ctx->n && tile >= 0 &&
            (tile == 0 || w == 0) && tile_valid(e, g, tile)) {
          res.epl = e;
          res.grid = g;
          res.win_bits = w;
          res.tile_bits = tile >= 100 ? tile / 100 : 0;
          res.tile_waves = tile >= 100 ? tile % 100 : 0;
          res.compact = tile == 1;
          res.ms = ms;
          res.from_cache = 1;
        }
      }
      std::fclose(f);
    }
  }
  if (!res.from_cache) {
    // candidates (epl, grid, window, tile = 100 tile_bits + waves): the untiled
    // pass over columns per lane and grids, and the tiled pass over columns per
    // lane, waves, the three largest tiles that fit LDS and one or two
    // workgroups per CU
    struct Cand { int e, g, w, tile; };
    std::vector<Cand> cands;
    std::vector<int> epls;
    for (int e : {1, 2, 4, 8}) {
      if (!hv_epl_valid(ctx->fp32, r, e)) continue;
      if (r > 16 && e != hv_elems_per_lane(ctx->fp32, r)) continue;
      epls.push_back(e);
    }
    const long long tiles64 = (ctx->N + 63) / 64;
    for (int e : epls)
      for (int g : {256, 512, 768, 1024, 1280, 1536, 2048})
        if (g <= tiles64 && g <= kMaxHvGrid) cands.push_back({e, g, 0, 0});
    if (cands.empty())
      for (int e : epls) cands.push_back({e, nspace_grid(ctx->N, r), 0, 0});
    if (compact_ok) {  // the same shapes with compacted gathers
      const size_t nu = cands.size();
      for (size_t i = 0; i < nu; ++i) cands.push_back({cands[i].e, cands[i].g, 0, 1});
    }
    for (int e : epls)
      for (int waves : {16, 8}) {
        int kmax = 0;
        for (int kb = 4; kb <= ctx->n; ++kb)
          if (hv_tile_ok(ctx->fp32, r, e, kb, waves, ctx->N, 8)) kmax = kb;
        for (int kb = kmax; kb >= 4 && kb > kmax - 3; --kb) {
          const long long ntile = ctx->N >> kb;  // small problems: one workgroup per tile
          for (int g : {256, 512, (int)std::min<long long>(ntile, 255)})
            if (hv_tile_ok(ctx->fp32, r, e, kb, waves, ctx->N, g) &&
                (g <= 256 || 2 * hv_tile_lds(ctx->fp32, r, e, kb, waves) <= (size_t)kMaxTileLds))
              cands.push_back({e, g, 0, 100 * kb + waves});
        }
      }
    // valid data in the pass input: the current state
    const size_t vbytes = (size_t)ctx->N * r * ctx->elem();
    HIPCHK(hipMemcpyAsync(ctx->blocks[1].p, ctx->blocks[0].p, vbytes, hipMemcpyDeviceToDevice, ctx->stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = 1e300;
    lrei_status st0 = hv_set_plan(ctx, 0);
    if (st0 != LREI_OK) return st0;
    for (const Cand &c : cands) {
      if (res.n_tried >= kTuneMax) break;
      ctx->epl = c.e;
      ctx->hv_tile_bits = c.tile >= 100 ? c.tile / 100 : 0;
      ctx->hv_tile_waves = c.tile >= 100 ? c.tile % 100 : 16;
      ctx->hv_compact = c.tile == 1;
      const int iters = 5;
      bool launched = true;
      auto pass = [&]() {
        launched = hv_pass_into(ctx, r, c.g, 1, ctx->blocks[1].p, ctx->blocks[4].p, (double2 *)ctx->partials.p,
                                ctx->ws.work, true, kMaxHvGrid, ctx->ws.shifts + r) &&
                   launched;
      };
      pass();
      if (!launched) {
        ctx->hv_launch_failed = false;
        continue;
      }
      (void)hipEventRecord(e0, ctx->stream);
      for (int k = 0; k < iters; ++k) pass();
      (void)hipEventRecord(e1, ctx->stream);
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipGetLastError());
      float t = 0;
      (void)hipEventElapsedTime(&t, e0, e1);
      const double ms = (double)t / iters;
      res.tried_epl[res.n_tried] = c.e;
      res.tried_grid[res.n_tried] = c.g;
      res.tried_win[res.n_tried] = c.w;
      res.tried_tile[res.n_tried] = c.tile;
      res.tried_ms[res.n_tried] = ms;
      res.n_tried++;
      if (ms < best) {
        best = ms;
        res.epl = c.e;
        res.grid = c.g;
        res.win_bits = c.w;
        res.tile_bits = c.tile >= 100 ? c.tile / 100 : 0;
        res.tile_waves = c.tile >= 100 ? c.tile % 100 : 0;
        res.compact = c.tile == 1;
        res.ms = ms;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (res.epl == 0) return ctx->fail(LREI_E_DEVICE, "no H.V variant could be launched");
    if (cache)
      if (FILE *f = std::fopen(cache, "a")) {
        std::fprintf(f, "%s %d %d %d %d %.6f\n", key.c_str(), res.epl, res.grid, res.win_bits,
                     res.tile_bits > 0 ? 100 * res.tile_bits + res.tile_waves : (res.compact ? 1 : 0), res.ms);
        std::fclose(f);
      }
  }
  lrei_status st = hv_set_plan(ctx, res.win_bits);
  if (st != LREI_OK) return st;
  res.n_sweeps = (int)ctx->sweeps.size();
  ctx->epl = res.epl;
  ctx->hv_grid = res.grid;
  ctx->hv_tile_bits = res.tile_bits;
  ctx->hv_tile_waves = res.tile_bits > 0 ? res.tile_waves : 16;
  ctx->hv_compact = res.compact;
  res.overlap_grid = overlap_grid(ctx);
  ctx->drop_graph();
  if (out) *out = res;
  return LREI_OK;
}

lrei_status lrei_synchronize(lrei_ctx *ctx) {
  if (!ctx) return LREI_E_INVALID;
  return check_hip(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
}

}  // extern "C"
