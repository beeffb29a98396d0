// Batched LREI-RK trajectories: many independent problems (each its own
// Hamiltonian, rank, model and damping) advanced with one launch per kernel
// and launch shape for the whole batch.
//
// A step is the single-trajectory step (Sec. 3.7 in the block Krylov space of
// the trajectory's own H and V) run for every trajectory at once:
//   for each pass j: batched Krylov H.V passes with fused Grams (one launch
//   per columns-per-lane class), one batched reduction, then on the second
//   stream the batched projected-step stage j (one workgroup per trajectory);
//   after the last stage, batched basis combinations.
// The kernels are the single-trajectory kernels' bodies; a workgroup finds
// its trajectory in per-launch tables.  Each trajectory's workgroups start at
// a multiple of 8, so the XCD-aware tile mapping holds within a trajectory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "host_common.h"
#include "lrei_internal.h"

using namespace lrei;

namespace {

constexpr int kMaxTraj = 1024;
constexpr int kBatchMaxGrid = 256;  // default cap on workgroups per trajectory and pass

// Tables of one batched launch: per-job records and the workgroup -> job map.
struct LaunchTables {
  DevBuf jobs, wg_job, job_wg0;
  int total_wg = 0;
  BatchLaunch view() const {
    return BatchLaunch{jobs.p, (const int *)wg_job.p, (const int *)job_wg0.p};
  }
  void release() {
    jobs.release();
    wg_job.release();
    job_wg0.release();
    total_wg = 0;
  }
};

// Builds the tables for jobs with the given workgroup counts; align pads each
// job's first workgroup to a multiple of 8 (padding workgroups get job -1).
template <typename Rec>
bool build_tables(const std::vector<Rec> &recs, const std::vector<int> &wgs, bool align, LaunchTables &t) {
  std::vector<int> wg_job, wg0(recs.size());
  for (size_t j = 0; j < recs.size(); ++j) {
    if (align)
      while (wg_job.size() % 8) wg_job.push_back(-1);
    wg0[j] = (int)wg_job.size();
    for (int w = 0; w < wgs[j]; ++w) wg_job.push_back((int)j);
  }
  t.release();
  if (recs.empty()) return true;
  if (!t.jobs.ensure(recs.size() * sizeof(Rec)) || !t.wg_job.ensure(wg_job.size() * sizeof(int)) ||
      !t.job_wg0.ensure(wg0.size() * sizeof(int)))
    return false;
  if (hipMemcpy(t.jobs.p, recs.data(), recs.size() * sizeof(Rec), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.wg_job.p, wg_job.data(), wg_job.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.job_wg0.p, wg0.data(), wg0.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return false;
  t.total_wg = (int)wg_job.size();
  return true;
}

// Workgroups of one trajectory's pass: one per 64-row tile up to cap, a
// multiple of 8 from 8 on (the XCD slots).
int batch_grid(long long N, int cap = kBatchMaxGrid) {
  const long long tiles = (N + 63) / 64;
  long long g = tiles < cap ? tiles : cap;
  if (g >= 8) g &= ~7LL;
  return (int)(g < 1 ? 1 : g);
}

std::string g_create_error;  // message of the last failed lrei_batch_create

}  // namespace

struct lrei_batch {
  int device = 0;
  hipStream_t stream = nullptr, side = nullptr;
  bool own_stream = false;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_pass[kMaxStages] = {};
  lrei_options opt{};
  std::string err;
  double hbar = 1.0;
  bool fp32 = false;

  struct Traj {
    int n = 0, r = 0, model = 0, grid = 1;
    int hv_epl = 0, hv_cap = kBatchMaxGrid;  // H.V pass shape: columns per lane (0: default), workgroup cap
    long long N = 0;
    double kappa = 0;
    std::vector<double> lam;
    TermTable terms;
    DevTerms dt;
    DevBuf blocks[kMaxStages + 1], save, partials, ws_buf;
    SmallWs ws{};
    void release() {
      dt.release();
      for (auto &b : blocks) b.release();
      save.release();
      partials.release();
      ws_buf.release();
    }
  };
  std::vector<Traj> tr;
  DevBuf stats;    // [n_traj][kStatsLen]
  DevBuf scratch;  // complex128 staging, max N r

  // launch tables: Krylov pass j by (columns per lane, r > 16) class,
  // reduction of pass j, projected step, combination by padded width
  struct HvGroup {
    int epl = 1;
    bool cplx = false, big = false, dyn = false;
    size_t lds = 0;
    LaunchTables t;
  };
  std::vector<HvGroup> hv[kMaxStages];
  LaunchTables reduce[kMaxStages];
  DevBuf small_p, small_ws;
  int small_lds = 0;
  struct CombGroup {
    int RP = 16;
    LaunchTables t;
  };
  std::vector<CombGroup> comb;
  std::vector<CombGroup> comb_prof;  // the same combinations written to the rollback copies
  int cur_scheme = -1, cur_s = 0;
  double cur_dt = 0;

  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool unusable = false;  // launch tables could not be rebuilt after a failed autotune

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
  }
};

namespace {

lrei_status bchk(lrei_batch *b, hipError_t e, const char *what) {
  if (e == hipSuccess) return LREI_OK;
  return b->fail(LREI_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define BCHK(expr)                                   \
  do {                                               \
    lrei_status _st = bchk(b, (expr), #expr);        \
    if (_st != LREI_OK) return _st;                  \
  } while (0)

// Per-trajectory device state: Krylov blocks, rollback copy, Gram partials and
// the projected-step workspace (the single-trajectory layout).
lrei_status alloc_traj(lrei_batch *b, lrei_batch::Traj &t, int idx) {
  const size_t blk = (size_t)t.N * t.r * b->elem();
  for (auto &bl : t.blocks)
    if (!bl.ensure(blk)) return b->fail(LREI_E_NOMEM, "device allocation of Krylov blocks failed");
  if (!t.save.ensure(blk)) return b->fail(LREI_E_NOMEM, "device allocation failed");
  t.grid = batch_grid(t.N);
  const int r = t.r, D = (kMaxStages + 1) * r;
  if (!t.partials.ensure((size_t)t.grid * 3 * r * r * sizeof(double2)))
    return b->fail(LREI_E_NOMEM, "device allocation failed");
  const size_t ws_elems = (size_t)kMaxStages * 3 * r * r + 4 * (size_t)D * D +
                          (4 * (size_t)D * r + 2 * (size_t)D * D + 4 * (size_t)r * r) +
                          (size_t)kMaxStages * 3 * D * r + (size_t)D * r + (size_t)D + (size_t)kMaxStages +
                          (size_t)kMaxBlocks * r;
  if (!t.ws_buf.ensure(ws_elems * sizeof(double2))) return b->fail(LREI_E_NOMEM, "device allocation failed");
  double2 *w = (double2 *)t.ws_buf.p;
  t.ws.meas = w; w += (size_t)kMaxStages * 3 * r * r;
  t.ws.gamma = w; w += (size_t)D * D;
  t.ws.R = w; w += (size_t)D * D;
  t.ws.Rinv = w; w += (size_t)D * D;
  t.ws.Hh = w; w += (size_t)D * D;
  t.ws.work = w; w += 4 * (size_t)D * r + 2 * (size_t)D * D + 4 * (size_t)r * r;
  t.ws.stage = w; w += (size_t)kMaxStages * 3 * D * r;
  t.ws.Cfin = w; w += (size_t)D * r;
  t.ws.flags = (double *)w; w += (size_t)D;
  t.ws.warm_skip = (double *)w; w += (size_t)kMaxStages;
  t.ws.shifts = (double *)w;
  if (hipMemset(t.ws.warm_skip, 0, 2 * kMaxStages * sizeof(double)) != hipSuccess ||
      hipMemset(t.ws.shifts, 0, (size_t)kMaxBlocks * r * sizeof(double)) != hipSuccess)
    return b->fail(LREI_E_DEVICE, "device memset failed");
  t.ws.stats = (double *)b->stats.p + (size_t)idx * kStatsLen;
  return LREI_OK;
}

// Tables of the Krylov passes and their reductions (independent of the scheme):
// every pass, or pass j_only alone.  Each trajectory's pass takes its own
// shape (hv_epl, hv_cap); its Gram partial buffer grows to the grid.
lrei_status build_pass_tables(lrei_batch *b, int j_only = -1) {
  for (int j = 0; j < kMaxStages; ++j) {
    if (j_only >= 0 && j != j_only) continue;
    std::map<std::tuple<int, int, int>, std::vector<int>> cls;  // (epl, big, dynamic) -> trajectories
    std::vector<HvArgs> args(b->tr.size());
    for (size_t q = 0; q < b->tr.size(); ++q) {
      auto &t = b->tr[q];
      HvArgs a{};
      a.Pcur = t.blocks[j].p;
      a.Pnext = t.blocks[j + 1].p;
      a.terms64 = (const DevTerm<double> *)t.dt.off64.p;
      a.terms32 = (const DevTerm<float> *)t.dt.off32.p;
      a.diag64 = (const double *)t.dt.d64.p;
      a.diag32 = (const float *)t.dt.d32.p;
      a.n_off = t.dt.n_off;
      a.cplx = t.dt.cplx;
      a.N = t.N;
      a.r = t.r;
      a.alpha = t.terms.spread > 0 ? 1.0 / t.terms.spread : 1.0;
      a.colshift = t.ws.shifts + (size_t)j * t.r;
      a.mode = j == 0 ? 0 : 1;
      a.epl = t.hv_epl;
      a.grid = batch_grid(t.N, t.hv_cap);
      if (!t.partials.ensure((size_t)a.grid * 3 * t.r * t.r * sizeof(double2)))
        return b->fail(LREI_E_NOMEM, "device allocation failed");
      a.partials = (double2 *)t.partials.p;
      // static tile schedule: a batched launch holds many workgroups per CU
      // slot, which the hardware dispatcher balances by itself
      a.sched = nullptr;
      a.partial_cap = a.grid;
      if (!prepare_hv(b->fp32, a)) return b->fail(LREI_E_INVALID, "unsupported rank for the H.V pass");
      args[q] = a;
      cls[{a.epl, a.r > 16 ? 1 : 0, a.chunks > 0 ? 1 : 0}].push_back((int)q);
    }
    for (auto &g : b->hv[j]) g.t.release();
    b->hv[j].clear();
    for (auto &kv : cls) {
      lrei_batch::HvGroup g;
      g.epl = std::get<0>(kv.first);
      g.big = std::get<1>(kv.first) != 0;
      g.dyn = std::get<2>(kv.first) != 0;
      std::vector<HvArgs> recs;
      std::vector<int> wgs;
      for (int q : kv.second) {
        recs.push_back(args[q]);
        wgs.push_back(args[q].grid);
        g.cplx = g.cplx || args[q].cplx;
        g.lds = std::max(g.lds, hv_launch_lds(b->fp32, args[q]));
      }
      if (!build_tables(recs, wgs, true, g.t)) return b->fail(LREI_E_NOMEM, "launch table upload failed");
      b->hv[j].push_back(std::move(g));
    }
    std::vector<ReduceJob> rj;
    std::vector<int> lens;
    for (size_t q = 0; q < b->tr.size(); ++q) {
      auto &t = b->tr[q];
      const int rr = t.r * t.r;
      const int slots = args[q].chunks > 0 ? args[q].chunks : args[q].grid;
      rj.push_back(ReduceJob{(const double2 *)t.partials.p, slots, t.ws.meas + (size_t)j * 3 * rr});
      lens.push_back((j == 0 ? 3 : 2) * rr);
    }
    if (!build_tables(rj, lens, false, b->reduce[j])) return b->fail(LREI_E_NOMEM, "launch table upload failed");
  }
  return LREI_OK;
}

// Tables that depend on the scheme and step: projected-step parameters and
// the combinations (their block count is s + 1).
lrei_status build_step_tables(lrei_batch *b, int scheme, double dt) {
  std::vector<SmallRkParams> ps;
  std::vector<SmallWs> wss;
  int s = 0;
  int lds = 0;
  for (auto &t : b->tr) {
    SmallRkParams p{};
    tableau(scheme, s, p.a, p.b);
    p.r = t.r;
    p.s = s;
    p.nblocks = s + 1;
    p.model = t.model;
    p.householder_mode = b->opt.householder_mode;
    p.max_sweeps = b->opt.eig_max_sweeps;
    p.warm = b->opt.warm;
    p.kappa = t.kappa;
    p.hbar = b->hbar;
    p.h = dt;
    p.eig_tol = b->opt.eig_tol;
    p.warm_tol = b->fp32 ? 1e-11 : 1e-14;
    p.beta = t.terms.spread > 0 ? 1.0 / t.terms.spread : 1.0;
    for (int i = 0; i < t.r; ++i) p.lam[i] = t.lam[i];
    p.lds_elems = small_lds_elems(p.nblocks * t.r, t.r);
    lds = std::max(lds, p.lds_elems);
    ps.push_back(p);
    wss.push_back(t.ws);
  }
  if (!b->small_p.ensure(ps.size() * sizeof(SmallRkParams)) || !b->small_ws.ensure(wss.size() * sizeof(SmallWs)))
    return b->fail(LREI_E_NOMEM, "device allocation failed");
  BCHK(hipMemcpy(b->small_p.p, ps.data(), ps.size() * sizeof(SmallRkParams), hipMemcpyHostToDevice));
  BCHK(hipMemcpy(b->small_ws.p, wss.data(), wss.size() * sizeof(SmallWs), hipMemcpyHostToDevice));
  b->small_lds = lds;
  std::map<int, std::vector<int>> cls;  // padded width -> trajectories
  for (size_t q = 0; q < b->tr.size(); ++q) cls[b->tr[q].r <= 16 ? 16 : 32].push_back((int)q);
  for (auto &g : b->comb) g.t.release();
  for (auto &g : b->comb_prof) g.t.release();
  b->comb.clear();
  b->comb_prof.clear();
  for (int prof = 0; prof < 2; ++prof) {
    for (auto &kv : cls) {
      lrei_batch::CombGroup g;
      g.RP = kv.first;
      std::vector<CombineArgs> recs;
      std::vector<int> wgs;
      for (int q : kv.second) {
        auto &t = b->tr[q];
        CombineArgs a{};
        for (int i = 0; i < kMaxBlocks; ++i) a.blocks[i] = i <= s ? t.blocks[i].p : nullptr;
        a.nb = s + 1;
        a.C = t.ws.Cfin;
        a.out = prof ? t.save.p : t.blocks[0].p;
        a.N = t.N;
        a.r = t.r;
        a.grid = t.grid;
        recs.push_back(a);
        wgs.push_back(t.grid);
    }
      if (!build_tables(recs, wgs, true, g.t)) return b->fail(LREI_E_NOMEM, "launch table upload failed");
      (prof ? b->comb_prof : b->comb).push_back(std::move(g));
    }
  }
  b->cur_scheme = scheme;
  b->cur_s = s;
  b->cur_dt = dt;
  b->drop_graph();
  return LREI_OK;
}

// Pass j of every trajectory: H.V with fused Grams, then the reduction into meas.
void enqueue_pass(lrei_batch *b, int j, hipStream_t s) {
  for (auto &g : b->hv[j])
    launch_hv_batch(b->fp32, g.epl, g.cplx, g.big, g.dyn, g.t.view(), g.t.total_wg, g.lds, s);
  launch_reduce_batch(b->reduce[j].view(), b->reduce[j].total_wg, s);
}

// One LREI-RK step of every trajectory; stage j of the projected steps runs
// on the second stream as soon as pass j is reduced.
void enqueue_step(lrei_batch *b) {
  const int s = b->cur_s, n = (int)b->tr.size();
  (void)hipEventRecord(b->ev_fork, b->stream);
  (void)hipStreamWaitEvent(b->side, b->ev_fork, 0);
  for (int j = 0; j < s; ++j) {
    enqueue_pass(b, j, b->stream);
    (void)hipEventRecord(b->ev_pass[j], b->stream);
    (void)hipStreamWaitEvent(b->side, b->ev_pass[j], 0);
    launch_small_rk_stage_batch((const SmallRkParams *)b->small_p.p, (const SmallWs *)b->small_ws.p, n,
                                b->small_lds, j, b->side);
  }
  (void)hipEventRecord(b->ev_join, b->side);
  (void)hipStreamWaitEvent(b->stream, b->ev_join, 0);
  for (auto &g : b->comb) launch_combine_batch(b->fp32, g.RP, s + 1, g.t.view(), g.t.total_wg, b->stream);
}

void destroy_batch(lrei_batch *b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->side) (void)hipStreamSynchronize(b->side);
  b->drop_graph();
  for (auto &t : b->tr) t.release();
  b->stats.release();
  b->scratch.release();
  for (auto &v : b->hv)
    for (auto &g : v) g.t.release();
  for (auto &t : b->reduce) t.release();
  for (auto &g : b->comb) g.t.release();
  for (auto &g : b->comb_prof) g.t.release();
  b->small_p.release();
  b->small_ws.release();
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  for (auto &e : b->ev_pass)
    if (e) (void)hipEventDestroy(e);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

// Validates descriptor q on the host (the orthonormality of V is checked on
// the device after upload).
bool check_desc(const lrei_traj_desc &d, int q, std::string &err) {
  auto bad = [&](const std::string &m) {
    err = "trajectory " + std::to_string(q) + ": " + m;
    return false;
  };
  if (d.n_spins < 1 || d.n_spins > 30) return bad("n_spins must be in [1, 30]");
  if (d.r < 1 || d.r > kMaxR) return bad("r must be in [1, 32]");
  if ((long long)d.r > (1LL << d.n_spins)) return bad("r exceeds the Hilbert dimension");
  if (!d.lambda || !d.V) return bad("null lambda or V");
  for (int i = 0; i < d.r; ++i) {
    if (!std::isfinite(d.lambda[i]) || !(d.lambda[i] > 0)) return bad("lambda must be finite and strictly positive");
    if (i > 0 && d.lambda[i] > d.lambda[i - 1]) return bad("lambda must be non-increasing");
  }
  if (d.model != LREI_QLL && d.model != LREI_QLLG) return bad("unknown model");
  if (!(d.kappa >= 0) || !std::isfinite(d.kappa)) return bad("kappa must be >= 0 and finite");
  return true;
}

}  // namespace

extern "C" {

lrei_status lrei_batch_create(lrei_batch **out, int hip_device, void *hip_stream, const lrei_options *opt,
                              int n_traj, const lrei_traj_desc *traj, double hbar) {
  g_create_error.clear();
  auto cfail = [](lrei_status st, const std::string &m) {
    g_create_error = m;
    return st;
  };
  if (!out) return cfail(LREI_E_INVALID, "null output pointer");
  *out = nullptr;
  if (n_traj < 1 || n_traj > kMaxTraj || !traj) return cfail(LREI_E_INVALID, "n_traj must be in [1, 1024]");
  if (!(hbar > 0) || !std::isfinite(hbar)) return cfail(LREI_E_INVALID, "hbar must be positive and finite");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return cfail(LREI_E_DEVICE, "no HIP device");
  if (hip_device < 0 || hip_device >= ndev) return cfail(LREI_E_INVALID, "bad device index");
  lrei_options o;
  lrei_default_options(&o);
  if (opt) o = *opt;
  if (o.precision != LREI_FP64 && o.precision != LREI_MIXED) return cfail(LREI_E_INVALID, "unknown precision");
  if (!(o.eig_tol > 0) || o.eig_max_sweeps < 1) return cfail(LREI_E_INVALID, "bad eigensolver options");
  if (o.warm != LREI_WARM_PLAIN && o.warm != LREI_WARM_ANALYTIC)
    return cfail(LREI_E_INVALID, "warm must be LREI_WARM_PLAIN or LREI_WARM_ANALYTIC");
  std::vector<TermTable> tabs(n_traj);
  for (int q = 0; q < n_traj; ++q) {
    std::string e;
    if (!check_desc(traj[q], q, e)) return cfail(LREI_E_INVALID, e);
    const auto &d = traj[q];
    if (d.n_bonds < 0 || (d.n_bonds > 0 && (!d.bond_ij || !d.bond_J)))
      return cfail(LREI_E_INVALID, "trajectory " + std::to_string(q) + ": bad bond arrays");
    if (!build_terms(d.n_spins, d.n_bonds, d.bond_ij, d.bond_J, d.site_h, tabs[q], e))
      return cfail(LREI_E_INVALID, "trajectory " + std::to_string(q) + ": " + e);
  }
  if (hipSetDevice(hip_device) != hipSuccess) return cfail(LREI_E_DEVICE, "hipSetDevice failed");

  lrei_batch *b = new lrei_batch();
  b->device = hip_device;
  b->opt = o;
  b->fp32 = o.precision == LREI_MIXED;
  b->hbar = hbar;
  auto bail = [&](lrei_status st) {
    const std::string m = b->err;
    destroy_batch(b);
    return cfail(st, m);
  };
  if (hip_stream) b->stream = (hipStream_t)hip_stream;
  b->own_stream = !hip_stream;
  if (create_streams(!hip_stream, &b->stream, &b->side) != hipSuccess) {
    b->err = "stream creation failed";
    return bail(LREI_E_DEVICE);
  }
  bool ok = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) == hipSuccess;
  for (auto &e : b->ev_pass) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    b->err = "stream/event creation failed";
    return bail(LREI_E_DEVICE);
  }
  if (!b->stats.ensure((size_t)n_traj * kStatsLen * sizeof(double))) {
    b->err = "device allocation failed";
    return bail(LREI_E_NOMEM);
  }
  b->tr.resize(n_traj);
  size_t max_nr = 0;
  for (int q = 0; q < n_traj; ++q) {
    auto &t = b->tr[q];
    const auto &d = traj[q];
    t.n = d.n_spins;
    t.N = 1LL << d.n_spins;
    t.r = d.r;
    t.model = d.model;
    t.kappa = d.kappa;
    t.lam.assign(d.lambda, d.lambda + d.r);
    t.terms = tabs[q];
    std::string e;
    const lrei_status ust = upload_terms(t.terms, t.N, b->stream, t.dt, e);
    if (ust != LREI_OK) {
      b->err = "trajectory " + std::to_string(q) + ": " + e;
      return bail(ust);
    }
    lrei_status st = alloc_traj(b, t, q);
    if (st != LREI_OK) return bail(st);
    max_nr = std::max(max_nr, (size_t)t.N * t.r);
  }
  if (!b->scratch.ensure(max_nr * sizeof(double2))) {
    b->err = "device allocation failed";
    return bail(LREI_E_NOMEM);
  }
  // upload the states (complex128 -> storage precision)
  for (int q = 0; q < n_traj; ++q) {
    auto &t = b->tr[q];
    const size_t n = (size_t)t.N * t.r;
    hipError_t e = hipSuccess;
    if (!b->fp32) {
      e = hipMemcpyAsync(t.blocks[0].p, traj[q].V, n * sizeof(double2), hipMemcpyHostToDevice, b->stream);
    } else {
      e = hipMemcpyAsync(b->scratch.p, traj[q].V, n * sizeof(double2), hipMemcpyHostToDevice, b->stream);
      if (e == hipSuccess) launch_convert(true, b->scratch.p, t.blocks[0].p, (long long)n, b->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // scratch is reused by the next trajectory
    }
    if (e != hipSuccess) {
      bchk(b, e, "upload V");
      return bail(LREI_E_DEVICE);
    }
  }
  lrei_status st = build_pass_tables(b);
  if (st != LREI_OK) return bail(st);
  // orthonormality of every V from the pass-0 Gram P0* P0
  enqueue_pass(b, 0, b->stream);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess) he = hipStreamSynchronize(b->stream);
  if (he != hipSuccess) {
    bchk(b, he, "validate V");
    return bail(LREI_E_DEVICE);
  }
  const double tol = b->fp32 ? 1e-5 : 1e-10;
  for (int q = 0; q < n_traj; ++q) {
    auto &t = b->tr[q];
    std::vector<double2> g((size_t)t.r * t.r);
    if (hipMemcpy(g.data(), t.ws.meas, g.size() * sizeof(double2), hipMemcpyDeviceToHost) != hipSuccess) {
      b->err = "read Gram";
      return bail(LREI_E_DEVICE);
    }
    double dev = 0;
    bool finite = true;
    for (int a = 0; a < t.r; ++a)
      for (int c = 0; c < t.r; ++c) {
        double2 v = g[(size_t)a * t.r + c];
        if (!std::isfinite(v.x) || !std::isfinite(v.y)) finite = false;
        if (a == c) v.x -= 1.0;
        dev = std::max(dev, std::sqrt(v.x * v.x + v.y * v.y));
      }
    if (!finite || !(dev <= tol)) {
      b->err = "trajectory " + std::to_string(q) + ": V must have finite orthonormal columns (max |V*V - I| = " +
               std::to_string(dev) + ")";
      return bail(LREI_E_INVALID);
    }
  }
  *out = b;
  return LREI_OK;
}

void lrei_batch_destroy(lrei_batch *b) { destroy_batch(b); }

const char *lrei_batch_last_error(const lrei_batch *b) { return b ? b->err.c_str() : g_create_error.c_str(); }

lrei_status lrei_batch_step(lrei_batch *b, int scheme, double dt, int n_steps) {
  if (!b) return LREI_E_INVALID;
  if (b->unusable) return b->fail(LREI_E_STATE, "batch unusable: its launch tables could not be rebuilt");
  if (!(scheme >= LREI_RK1 && scheme <= LREI_RK4))
    return b->fail(LREI_E_INVALID, "batched stepping supports RK1..RK4");
  if (!(dt > 0) || !std::isfinite(dt)) return b->fail(LREI_E_INVALID, "dt must be positive and finite");
  if (n_steps < 0) return b->fail(LREI_E_INVALID, "n_steps must be >= 0");
  if (n_steps == 0) return LREI_OK;
  BCHK(hipSetDevice(b->device));
  if (scheme != b->cur_scheme || dt != b->cur_dt) {
    lrei_status st = build_step_tables(b, scheme, dt);
    if (st != LREI_OK) return st;
  }
  for (auto &t : b->tr)
    BCHK(hipMemcpyAsync(t.save.p, t.blocks[0].p, (size_t)t.N * t.r * b->elem(), hipMemcpyDeviceToDevice, b->stream));
  std::vector<double> zeros(b->tr.size() * kStatsLen, 0.0);
  BCHK(hipMemcpyAsync(b->stats.p, zeros.data(), zeros.size() * sizeof(double), hipMemcpyHostToDevice, b->stream));
  BCHK(hipStreamSynchronize(b->stream));
  if (b->opt.use_graph) {
    int k0 = 0;
    if (!b->exec) {
      // launch attributes are set on first use, outside capture; this eager
      // step counts as the first step
      enqueue_step(b);
      BCHK(hipGetLastError());
      BCHK(hipStreamSynchronize(b->stream));
      BCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      enqueue_step(b);
      BCHK(hipStreamEndCapture(b->stream, &b->graph));
      BCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      k0 = 1;
    }
    for (int k = k0; k < n_steps; ++k) BCHK(hipGraphLaunch(b->exec, b->stream));
  } else {
    for (int k = 0; k < n_steps; ++k) enqueue_step(b);
  }
  BCHK(hipGetLastError());
  std::vector<double> h(b->tr.size() * kStatsLen);
  BCHK(hipMemcpyAsync(h.data(), b->stats.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BCHK(hipStreamSynchronize(b->stream));
  for (size_t q = 0; q < b->tr.size(); ++q) {
    if (h[q * kStatsLen + 14] != 0) {
      for (auto &t : b->tr)
        BCHK(hipMemcpyAsync(t.blocks[0].p, t.save.p, (size_t)t.N * t.r * b->elem(), hipMemcpyDeviceToDevice,
                            b->stream));
      BCHK(hipStreamSynchronize(b->stream));
      return b->fail(LREI_E_NUMERIC, "trajectory " + std::to_string(q) +
                                         ": non-finite values in the step; every trajectory restored to the "
                                         "start of the call");
    }
  }
  return LREI_OK;
}

lrei_status lrei_batch_get_rho(lrei_batch *b, int traj, double *lambda, void *V, int v_is_device) {
  if (!b) return LREI_E_INVALID;
  if (traj < 0 || traj >= (int)b->tr.size()) return b->fail(LREI_E_INVALID, "trajectory index out of range");
  auto &t = b->tr[traj];
  if (lambda) std::memcpy(lambda, t.lam.data(), t.r * sizeof(double));
  if (!V) return LREI_OK;
  BCHK(hipSetDevice(b->device));
  const size_t n = (size_t)t.N * t.r;
  const void *src = t.blocks[0].p;
  if (b->fp32) {
    launch_convert(false, t.blocks[0].p, b->scratch.p, (long long)n, b->stream);
    BCHK(hipGetLastError());
    src = b->scratch.p;
  }
  BCHK(hipMemcpyAsync(V, src, n * sizeof(double2), v_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                      b->stream));
  BCHK(hipStreamSynchronize(b->stream));
  return LREI_OK;
}

lrei_status lrei_batch_energies(lrei_batch *b, double *energy) {
  if (!b || !energy) return LREI_E_INVALID;
  if (b->unusable) return b->fail(LREI_E_STATE, "batch unusable: its launch tables could not be rebuilt");
  BCHK(hipSetDevice(b->device));
  // pass 0 measures P0* P0 and P0* P1 with P1 = beta (H P0 - P0 D0) (scratch block 1;
  // the state is untouched), so (P0* H P0)_aa = (P0* P1)_aa / beta + D0_a (P0* P0)_aa
  enqueue_pass(b, 0, b->stream);
  BCHK(hipGetLastError());
  BCHK(hipStreamSynchronize(b->stream));
  for (size_t q = 0; q < b->tr.size(); ++q) {
    auto &t = b->tr[q];
    const int rr = t.r * t.r;
    std::vector<double2> g(2 * rr);
    std::vector<double> d0(t.r);
    BCHK(hipMemcpy(g.data(), t.ws.meas, 2 * rr * sizeof(double2), hipMemcpyDeviceToHost));
    BCHK(hipMemcpy(d0.data(), t.ws.shifts, t.r * sizeof(double), hipMemcpyDeviceToHost));
    const double e = t.terms.spread > 0 ? t.terms.spread : 1.0;
    double en = 0;
    for (int a = 0; a < t.r; ++a)
      en += t.lam[a] * (g[rr + a * t.r + a].x * e + d0[a] * g[a * t.r + a].x);
    energy[q] = en;
  }
  return LREI_OK;
}

lrei_status lrei_batch_profile_kernels(lrei_batch *b, int scheme, double dt, int iters, double ms[4]) {
  if (!b || !ms || iters < 1) return LREI_E_INVALID;
  if (b->unusable) return b->fail(LREI_E_STATE, "batch unusable: its launch tables could not be rebuilt");
  if (scheme != b->cur_scheme || dt != b->cur_dt)
    return b->fail(LREI_E_STATE, "run lrei_batch_step with this scheme and dt first");
  BCHK(hipSetDevice(b->device));
  BCHK(hipStreamSynchronize(b->stream));
  BCHK(hipStreamSynchronize(b->side));
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  const int n = (int)b->tr.size(), s = b->cur_s;
  auto timed = [&](auto &&fn) -> double {
    fn();  // warm
    (void)hipEventRecord(e0, b->stream);
    for (int i = 0; i < iters; ++i) fn();
    (void)hipEventRecord(e1, b->stream);
    (void)hipEventSynchronize(e1);
    float t = 0;
    (void)hipEventElapsedTime(&t, e0, e1);
    return (double)t / iters;
  };
  const int j = s > 1 ? 1 : 0;  // the recurrence-form pass where it exists
  ms[0] = timed([&] {
    for (auto &g : b->hv[j])
      launch_hv_batch(b->fp32, g.epl, g.cplx, g.big, g.dyn, g.t.view(), g.t.total_wg, g.lds, b->stream);
  });
  ms[1] = timed([&] { launch_reduce_batch(b->reduce[j].view(), b->reduce[j].total_wg, b->stream); });
  ms[2] = timed([&] {
    for (int q = 0; q < s; ++q)
      launch_small_rk_stage_batch((const SmallRkParams *)b->small_p.p, (const SmallWs *)b->small_ws.p, n,
                                  b->small_lds, q, b->stream);
  });
  ms[3] = timed([&] {
    for (auto &g : b->comb_prof) launch_combine_batch(b->fp32, g.RP, s + 1, g.t.view(), g.t.total_wg, b->stream);
  });
  const hipError_t he = hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  BCHK(he);
  return LREI_OK;
}

lrei_status lrei_batch_autotune(lrei_batch *b, int iters, lrei_batch_tune_result *out) {
  if (!b || iters < 1) return LREI_E_INVALID;
  if (b->unusable) return b->fail(LREI_E_STATE, "batch unusable: its launch tables could not be rebuilt");
  BCHK(hipSetDevice(b->device));
  BCHK(hipStreamSynchronize(b->stream));
  BCHK(hipStreamSynchronize(b->side));
  std::vector<int> ranks;
  for (auto &t : b->tr)
    if (std::find(ranks.begin(), ranks.end(), t.r) == ranks.end()) ranks.push_back(t.r);
  std::sort(ranks.begin(), ranks.end());
  std::vector<std::pair<int, int>> saved;
  for (auto &t : b->tr) saved.push_back({t.hv_epl, t.hv_cap});
  auto set_class = [&](int r, int epl, int cap) {
    for (auto &t : b->tr)
      if (t.r == r) {
        t.hv_epl = epl;
        t.hv_cap = cap;
      }
  };
  // on any failure: the shapes from before the call, every table rebuilt
  auto restore = [&](lrei_status st) {
    (void)hipStreamSynchronize(b->stream);
    for (size_t q = 0; q < b->tr.size(); ++q) {
      b->tr[q].hv_epl = saved[q].first;
      b->tr[q].hv_cap = saved[q].second;
    }
    const std::string e = b->err;
    if (build_pass_tables(b) != LREI_OK) b->unusable = true;
    b->drop_graph();
    b->err = e;
    return st;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return b->fail(LREI_E_DEVICE, "event creation failed");
  }
  // one recurrence-form pass of every trajectory (all launch classes) and its
  // reduction, on the batch stream; the state block is only read
  constexpr int j = 1;
  auto timed = [&](double &ms) -> bool {
    auto once = [&] {
      for (auto &g : b->hv[j])
        launch_hv_batch(b->fp32, g.epl, g.cplx, g.big, g.dyn, g.t.view(), g.t.total_wg, g.lds, b->stream);
      launch_reduce_batch(b->reduce[j].view(), b->reduce[j].total_wg, b->stream);
    };
    once();
    (void)hipEventRecord(e0, b->stream);
    for (int i = 0; i < iters; ++i) once();
    (void)hipEventRecord(e1, b->stream);
    if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) return false;
    float t = 0;
    (void)hipEventElapsedTime(&t, e0, e1);
    ms = (double)t / iters;
    return true;
  };
  auto finish = [&](lrei_status st) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st == LREI_OK ? st : restore(st);
  };
  lrei_batch_tune_result res{};
  lrei_status st = build_pass_tables(b, j);
  if (st != LREI_OK) return finish(st);
  double best = 0;
  if (!timed(best)) return finish(b->fail(LREI_E_DEVICE, "timing the batched pass failed"));
  res.ms_default = best;
  static const int kCaps[] = {16, 32, 64, 128, 256, 512, 1024};
  for (int r : ranks) {
    int best_epl = 0, best_cap = kBatchMaxGrid;
    for (auto &t : b->tr)
      if (t.r == r) {
        best_epl = t.hv_epl;
        best_cap = t.hv_cap;
        break;
      }
    std::vector<std::vector<int>> seen_grids[9];  // per columns-per-lane value
    for (int epl : {1, 2, 4, 8}) {
      if (!hv_epl_valid(b->fp32, r, epl)) continue;
      for (int cap : kCaps) {
        std::vector<int> grids;
        for (auto &t : b->tr)
          if (t.r == r) grids.push_back(batch_grid(t.N, cap));
        auto &seen = seen_grids[epl];
        if (std::find(seen.begin(), seen.end(), grids) != seen.end()) continue;  // same launch as a smaller cap
        seen.push_back(grids);
        set_class(r, epl, cap);
        st = build_pass_tables(b, j);
        if (st != LREI_OK) return finish(st);
        double ms = 0;
        if (!timed(ms)) return finish(b->fail(LREI_E_DEVICE, "timing the batched pass failed"));
        if (res.n_tried < LREI_TUNE_MAX) {
          res.tried_rank[res.n_tried] = r;
          res.tried_epl[res.n_tried] = epl;
          res.tried_cap[res.n_tried] = cap;
          res.tried_ms[res.n_tried] = ms;
          ++res.n_tried;
        }
        if (ms < best) {
          best = ms;
          best_epl = epl;
          best_cap = cap;
        }
      }
    }
    set_class(r, best_epl, best_cap);
    if (res.n_classes < LREI_BATCH_TUNE_CLASSES) {
      res.rank[res.n_classes] = r;
      res.epl[res.n_classes] = best_epl;
      res.wg_cap[res.n_classes] = best_cap;
      ++res.n_classes;
    }
  }
  st = build_pass_tables(b, j);
  if (st != LREI_OK) return finish(st);
  if (!timed(res.ms)) return finish(b->fail(LREI_E_DEVICE, "timing the batched pass failed"));
  st = build_pass_tables(b);  // every pass with the chosen shapes
  if (st != LREI_OK) return finish(st);
  b->drop_graph();
  finish(LREI_OK);
  if (out) *out = res;
  return LREI_OK;
}

lrei_status lrei_batch_synchronize(lrei_batch *b) {
  if (!b) return LREI_E_INVALID;
  BCHK(hipSetDevice(b->device));
  BCHK(hipStreamSynchronize(b->stream));
  BCHK(hipStreamSynchronize(b->side));
  return LREI_OK;
}

}  // extern "C"
