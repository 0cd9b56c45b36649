// Host side of the gqd C ABI: validation, item planning, twiddle table, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gqd.h"
#include "gqd_internal.h"
#include "gqd_compositions.h"

using namespace gqd;

namespace {

thread_local std::string g_last_error;

gqd_status fail(gqd_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

gqd_status hip_fail(hipError_t e, const char* what) {
  return fail(GQD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define GQD_HIP(call)                                 \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

int class_of(int n) {
  for (int c = 0; c < kNumClasses; ++c)
    if (kClassN[c] == n) return c;
  return -1;
}

constexpr size_t kLdsMax = 160 * 1024;
// a T_max above which an automatic call preconditions a size class (resolve_precond)
constexpr double kPrecondStiffness = 1.25;

}  // namespace

struct gqd_handle {
  int dims = 1;
  int batch = 0;
  double mass = 0.0;
  // 2D grids (dims = 2): n x n points per item, line size class, device tables
  int n2 = 0;
  int line_cls = -1;
  double mass2[2] = {0.0, 0.0};
  std::vector<Item2> items2;
  Item2* d_items2 = nullptr;
  double2* d_tw2 = nullptr;
  unsigned* d_sync = nullptr;
  double* d_part = nullptr;
  int resident_cap = 0;  // workgroups the partial and sync areas are sized for
  int stats_roles = 1;   // groups per item of the last 2D launch (2: merge their statistics)
  int stats_precond = 0; // the last launch's solves were preconditioned (byte count)
  int stats_literal = 0; // the last launch ran the literal explicit half-steps (byte count)
  // precond = 2 (automatic): the choice of each size class for the current call
  bool precond_auto = false;
  int class_precond[kNumClasses] = {};
  int spin_limit = 0;    // polls of a 2D grid wait before it gives up (0: the default)
  std::vector<ItemMeta> items;
  long long total_complex = 0;
  std::vector<int> class_lists[kNumClasses];
  ItemMeta* d_items = nullptr;
  int* d_lists[kNumClasses] = {};
  double2* d_tw = nullptr;
  long long tw_off[kNumPlans] = {};
  int plan[kNumClasses] = {};  // transform plan of each size class (kPlans index)
  ItemStats* d_stats = nullptr;
  std::vector<ItemStats> h_stats;
  const double* V = nullptr;
  const double* F = nullptr;
  void* work = nullptr;
  size_t work_bytes = 0;
  int* solve_log = nullptr;  // optional per-solve iteration counts, log_cap per item
  long long log_cap = 0;
  void* scratch = nullptr;   // this device's static scratch (gqd_propagate_noalloc)
  hipStream_t side[kNumClasses] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kNumClasses] = {};
  bool streams_ready = false;
};

namespace {

gqd_status check_opts(const gqd_handle* h, const gqd_solver_opts* o) {
  if (!o) return fail(GQD_ERR_INVALID, "solver options are NULL");
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(GQD_ERR_INVALID, "tol must be finite and > 0");
  if (o->restart < 1 || o->restart > kMaxRestart) return fail(GQD_ERR_INVALID, "restart must be in 1..64");
  if (o->maxit < 1) return fail(GQD_ERR_INVALID, "maxit must be >= 1");
  if (o->precond < 0 || o->precond > 2) return fail(GQD_ERR_INVALID, "precond must be 0, 1 or 2");
  if (h->dims == 2) {
    if (o->precond == 1) return fail(GQD_ERR_UNSUPPORTED, "the kinetic preconditioner is available on 1D grids");
    if (lds_bytes2(h->n2, o->restart) > kLdsMax)
      return fail(GQD_ERR_UNSUPPORTED, "restart " + std::to_string(o->restart) +
                                           " needs more than 160 KB of LDS at n = " + std::to_string(h->n2) +
                                           " x " + std::to_string(h->n2));
    return GQD_OK;
  }
  for (int c = 0; c < kNumClasses; ++c) {
    if (!h->class_lists[c].empty() && lds_bytes(h->plan[c], o->restart) > kLdsMax)
      return fail(GQD_ERR_UNSUPPORTED, "restart " + std::to_string(o->restart) +
                                           " needs more than 160 KB of LDS at n = " +
                                           std::to_string(kClassN[c]));
  }
  return GQD_OK;
}

size_t work_need(const gqd_handle* h, int m) {
  // 2D: two regions per item, as the reverse sweep solves phi and mu on two groups at once
  if (h->dims == 2) return 2 * (size_t)h->total_complex * (size_t)(kWork2Extra + m + 1) * sizeof(double2);
  return (size_t)h->total_complex * (size_t)(m + kWorkExtra) * sizeof(double2);
}

constexpr int kSpinLimit = 1 << 22;  // polls of one grid barrier (seconds) before abort

// Launch the 2D kernel over all items: groups of G workgroups per item (two groups per
// item for the reverse sweep, which solves phi and mu side by side), as many items per
// cooperative launch as can be resident together.
gqd_status run2d(gqd_handle* h, K2Args a, hipStream_t stream) {
  int resident = 0;
  GQD_HIP(max_resident2d(h->line_cls, a.sc.m, &resident));
  if (resident < 1) return fail(GQD_ERR_UNSUPPORTED, "2D kernel cannot be resident");
  if (resident > h->resident_cap) resident = h->resident_cap;
  const int roles = (a.mode == kM2Adjoint && resident >= 2) ? 2 : 1;
  const long long vec = 2LL * h->n2 * h->n2;
  long long gmax = 2LL * (h->n2 / kLineWaves);
  if (vec / kThreads2 < gmax) gmax = vec / kThreads2;
  long long per_item = resident / h->batch;
  if (per_item < 1) per_item = 1;
  if (per_item < gmax) gmax = per_item;
  int G = 1;
  while (2LL * G <= gmax) G *= 2;
  // two groups share what one would have had: every grid barrier writes back and
  // invalidates the L2 of each XCD it spans, so more workgroups per XCD make each
  // barrier dearer (at 256 x 256: 128 + 128 workgroups lost to 64 + 64)
  if (roles == 2 && G > 1) G /= 2;
  const int per_launch = resident / (G * roles);
  a.G = G;
  a.roles = roles;
  a.work_stride = (long long)(kWork2Extra + a.sc.m + 1) * vec;
  h->stats_roles = roles;
  double* out0 = a.out;
  for (int base = 0; base < h->batch; base += per_launch) {
    const int cnt = (h->batch - base < per_launch) ? h->batch - base : per_launch;
    K2Args b = a;
    b.items = h->d_items2 + base;
    b.batch = cnt;
    b.stats = h->d_stats + base;
    b.stats1 = h->d_stats + h->batch + base;
    if (out0) b.out = out0 + (a.mode == kM2Inner ? 2 : 4) * (size_t)base;
    // per group [arrivals, abort]; per item [mu ready, gradient done]
    GQD_HIP(hipMemsetAsync(h->d_sync, 0, sizeof(unsigned) * 2 * (size_t)cnt * (roles + 1), stream));
    GQD_HIP(launch_run2d(h->line_cls, b, stream));
  }
  return GQD_OK;
}

K2Args base_args2(const gqd_handle* h) {
  K2Args a;
  std::memset(&a, 0, sizeof(a));
  a.V = h->V;
  a.F = h->F;
  a.tw = h->d_tw2;
  a.inv2m0 = 1.0 / (2.0 * h->mass2[0]);
  a.inv2m1 = 1.0 / (2.0 * h->mass2[1]);
  a.mass0 = h->mass2[0];
  a.mass1 = h->mass2[1];
  a.sync = h->d_sync;
  a.part = h->d_part;
  a.spin_limit = h->spin_limit > 0 ? h->spin_limit : kSpinLimit;
  a.roles = 1;
  return a;
}

void release_streams(gqd_handle* h) {
  for (int c = 0; c < kNumClasses; ++c) {
    if (h->side[c]) (void)hipStreamDestroy(h->side[c]);
    if (h->ev_join[c]) (void)hipEventDestroy(h->ev_join[c]);
    h->side[c] = nullptr;
    h->ev_join[c] = nullptr;
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  h->ev_fork = nullptr;
  h->streams_ready = false;
}

// Side streams and events, created on first use; a failure part way releases what was
// created, so that a later call starts again from nothing.
gqd_status ensure_streams(gqd_handle* h) {
  if (h->streams_ready) return GQD_OK;
  hipError_t e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
  for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) {
    e = hipStreamCreateWithFlags(&h->side[c], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join[c], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    release_streams(h);
    return hip_fail(e, "creating side streams");
  }
  h->streams_ready = true;
  return GQD_OK;
}

// Launch `fn` once per non-empty size class.  Several classes run concurrently on
// side streams forked from and joined back into the caller's stream, largest first.
// class_precond (solves of an automatic call): the preconditioner flag of each class.
template <class Fn>
gqd_status for_each_class(gqd_handle* h, hipStream_t stream, KArgs a, Fn fn, const int* class_precond = nullptr) {
  int active = 0;
  for (int c = 0; c < kNumClasses; ++c) active += h->class_lists[c].empty() ? 0 : 1;
  if (active == 1) {
    for (int c = 0; c < kNumClasses; ++c) {
      if (h->class_lists[c].empty()) continue;
      a.list = h->d_lists[c];
      a.nlist = (int)h->class_lists[c].size();
      a.tw = h->d_tw + h->tw_off[h->plan[c]];
      if (class_precond) a.sc.precond = class_precond[c];
      GQD_HIP(fn(h->plan[c], a, stream));
    }
    return GQD_OK;
  }
  gqd_status st = ensure_streams(h);
  if (st != GQD_OK) return st;
  GQD_HIP(hipEventRecord(h->ev_fork, stream));
  // largest grids first: they carry most of the work, and side streams that share a
  // hardware queue run their kernels one after the other
  for (int c = kNumClasses - 1; c >= 0; --c) {
    if (h->class_lists[c].empty()) continue;
    GQD_HIP(hipStreamWaitEvent(h->side[c], h->ev_fork, 0));
    a.list = h->d_lists[c];
    a.nlist = (int)h->class_lists[c].size();
    a.tw = h->d_tw + h->tw_off[h->plan[c]];
    if (class_precond) a.sc.precond = class_precond[c];
    GQD_HIP(fn(h->plan[c], a, h->side[c]));
    GQD_HIP(hipEventRecord(h->ev_join[c], h->side[c]));
    GQD_HIP(hipStreamWaitEvent(stream, h->ev_join[c], 0));
  }
  return GQD_OK;
}

KArgs base_args(const gqd_handle* h) {
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.items = h->d_items;
  a.V = h->V;
  a.F = h->F;
  a.inv2m = 1.0 / (2.0 * h->mass);
  a.mass = h->mass;
  a.stats = h->d_stats;
  return a;
}

gqd_status make_gammas(gqd_scheme s, int order, GammaTab* gt) {
  if (order < 2 || order % 2 || order > 2 * (kMaxLevels + 1))
    return fail(GQD_ERR_INVALID, "order must be even, 2..10");
  if (s != GQD_TRIPLE_JUMP && s != GQD_SUZUKI && s != GQD_OPTIMAL)
    return fail(GQD_ERR_INVALID, "unknown composition scheme");
  std::memset(gt, 0, sizeof(*gt));
  if (s == GQD_OPTIMAL && order > 2) {
    // one level of fractions over the second-order method (gqd_compositions.h)
    for (int k = 0; k < kNumFlat; ++k)
      if (kFlatComps[k].order == order) {
        gt->flat = 1 + kFlatComps[k].offset;
        gt->count = kFlatComps[k].count;
        gt->arity = kFlatComps[k].count;
        gt->levels = 1;
        return GQD_OK;
      }
    return fail(GQD_ERR_UNSUPPORTED, "no non-recursive composition of order " + std::to_string(order));
  }
  gt->arity = (s == GQD_TRIPLE_JUMP) ? 3 : 5;
  gt->levels = order / 2 - 1;
  gt->count = 1;
  for (int l = 0; l < gt->levels; ++l) {
    const int p = 2 * l + 2;  // order of the method being composed
    if (s == GQD_TRIPLE_JUMP) {
      const double r = std::pow(2.0, 1.0 / (p + 1));
      gt->side[l] = 1.0 / (2.0 - r);
      gt->mid[l] = -r / (2.0 - r);
    } else {
      const double r = std::pow(4.0, 1.0 / (p + 1));
      gt->side[l] = 1.0 / (4.0 - r);
      gt->mid[l] = -r / (4.0 - r);
    }
    gt->count *= gt->arity;
  }
  return GQD_OK;
}

// Largest |tau_c| of a composition's substeps (tau_c dt is the substep).
double max_abs_tau(const GammaTab& gt) {
  if (gt.flat) {
    static const double flat[kFlatTauLen] = {GQD_FLAT_TAU_VALUES};
    double t = 0.0;
    for (int c = 0; c < gt.count; ++c) t = std::max(t, std::fabs(flat[gt.flat - 1 + c]));
    return t;
  }
  double t = 1.0;
  for (int l = 0; l < gt.levels; ++l) t *= std::max(std::fabs(gt.side[l]), std::fabs(gt.mid[l]));
  return t;
}

// Solver option precond (0 off, 1 on, 2 automatic) resolved for one call (the byte
// counts of the call's statistics also note its literal flag here); returns the
// flag the launch arguments carry (for automatic calls, each size class then takes its
// own from class_precond).  The kinetic part sets the stiffness of 1 + i a H: with
// T_max = (pi / dq)^2 / 2m the largest kinetic energy of a class's grids and a the
// largest half-substep, a T_max is the largest eigenvalue of a T.  The preconditioner
// removes it at the price of one more transform pair per iteration, which pays once
// a T_max exceeds about 1.25 (per-class timings of the ragged batch at Suzuki-6,
// 2.5 a.u.: the plain solver is 24 % faster at a T_max = 0.35, the preconditioned one
// 6 % faster at 1.4 and twice as fast at 5.7; the 8th-order batch at 20 a.u.,
// a T_max = 5.0, 1.8x; the gradient workload at 1.15 ran faster plain).
// With per-item steps (not read back from the device) an automatic call
// preconditions every class.
int resolve_precond(gqd_handle* h, const gqd_solver_opts* o, const GammaTab& gt, double dt, bool item_steps) {
  const int precond = o->precond;
  h->stats_literal = o->literal ? 1 : 0;
  h->precond_auto = precond == 2 && h->dims == 1;
  if (precond != 2) {
    h->stats_precond = precond;
    return precond;
  }
  if (h->dims == 2) {
    h->stats_precond = 0;
    return 0;
  }
  const double a = 0.5 * std::fabs(dt) * max_abs_tau(gt);
  for (int c = 0; c < kNumClasses; ++c) {
    double tmax = 0.0;
    for (int b : h->class_lists[c]) {
      const double pmax = M_PI / h->items[b].dq;
      tmax = std::max(tmax, pmax * pmax / (2.0 * h->mass));
    }
    h->class_precond[c] = (item_steps || a * tmax > kPrecondStiffness) ? 1 : 0;
  }
  h->stats_precond = 0;
  return 0;
}

// Longest-first dispatch: the hardware starts workgroups in launch-list order and a
// launch ends with its slowest CU, so the items measured most expensive in the last
// call (H applications plus squared Arnoldi counts, the Gram-Schmidt part) go first.
// Items are independent, so the order changes no result.  Called with the device idle.
gqd_status reorder_by_cost(gqd_handle* h) {
  if (h->dims != 1) return GQD_OK;
  for (int c = 0; c < kNumClasses; ++c) {
    std::vector<int>& L = h->class_lists[c];
    if (L.size() < 2) continue;
    auto cost = [&](int b) {
      const ItemStats& s = h->h_stats[b];
      return (double)s.h_applies + 0.5 * (double)s.iterations_sq;
    };
    std::vector<int> sorted = L;
    std::stable_sort(sorted.begin(), sorted.end(), [&](int x, int y) { return cost(x) > cost(y); });
    if (sorted == L) continue;
    L = sorted;
    GQD_HIP(hipMemcpy(h->d_lists[c], L.data(), sizeof(int) * L.size(), hipMemcpyHostToDevice));
  }
  return GQD_OK;
}

gqd_status collect_stats(gqd_handle* h, hipStream_t stream, gqd_stats* st) {
  GQD_HIP(hipStreamSynchronize(stream));
  GQD_HIP(hipMemcpy(h->h_stats.data(), h->d_stats, sizeof(ItemStats) * h->batch, hipMemcpyDeviceToHost));
  if (h->dims == 2 && h->stats_roles == 2) {
    // the second group's solves (mu) of a two-group reverse sweep
    std::vector<ItemStats> s1(h->batch);
    GQD_HIP(hipMemcpy(s1.data(), h->d_stats + h->batch, sizeof(ItemStats) * h->batch, hipMemcpyDeviceToHost));
    for (int b = 0; b < h->batch; ++b) {
      ItemStats& s = h->h_stats[b];
      s.h_applies += s1[b].h_applies;
      s.iterations += s1[b].iterations;
      s.iterations_sq += s1[b].iterations_sq;
      s.extra_vecs += s1[b].extra_vecs;
      s.solves += s1[b].solves;
      if (s1[b].max_iters > s.max_iters) s.max_iters = s1[b].max_iters;
      s.failures += s1[b].failures;
      if (s1[b].nonfinite > s.nonfinite) s.nonfinite = s1[b].nonfinite;
      if (s1[b].max_resid > s.max_resid) s.max_resid = s1[b].max_resid;
    }
  }
  {
    const gqd_status rs = reorder_by_cost(h);
    if (rs != GQD_OK) return rs;
  }
  std::memset(st, 0, sizeof(*st));
  st->failed_item = -1;
  for (int b = 0; b < h->batch; ++b) {
    const ItemStats& s = h->h_stats[b];
    st->h_applies += s.h_applies;
    st->iterations += s.iterations;
    st->iterations_sq += s.iterations_sq;
    st->solves += s.solves;
    if (s.max_iters > st->max_iters) st->max_iters = s.max_iters;
    st->failures += s.failures;
    st->nonfinite += s.nonfinite;
    if (s.max_resid > st->max_true_resid) st->max_true_resid = s.max_resid;
    // 32 (I^2 + 4 I + 8) bytes per grid point per solve (S = 2 complex128 vectors);
    // preconditioned: each iteration also writes and reads z_j = M^-1 v_j, and the
    // cycle's update passes V y through M^-1: 32 (I^2 + 6 I + 10)
    const double pts = h->dims == 2 ? (double)h->n2 * h->n2 : (double)h->items[b].n;
    const bool pc = h->dims == 1 && h->precond_auto ? h->class_precond[h->items[b].cls] != 0 : h->stats_precond != 0;
    const double per_it = pc ? 6.0 : 4.0, per_solve = pc ? 10.0 : 8.0;
    const double alg = 32.0 * pts *
                       ((double)s.iterations_sq + per_it * (double)s.iterations + per_solve * (double)s.solves);
    st->alg_bytes += alg;
    // implementation bytes: the extra Gram-Schmidt sweeps, and in literal mode the
    // explicit half-step's own H application (read and write, per solve)
    st->impl_bytes += alg + 32.0 * pts * ((double)s.extra_vecs + (h->stats_literal ? 2.0 * (double)s.solves : 0.0));
    if ((s.failures || s.nonfinite) && st->failed_item < 0) st->failed_item = b;
  }
  for (int b = 0; b < h->batch; ++b)
    if (h->h_stats[b].nonfinite == 2)
      return fail(GQD_ERR_HIP, "grid barrier timed out (item " + std::to_string(b) + ")");
  if (st->nonfinite) return fail(GQD_ERR_NONFINITE, "a norm became non-finite (first item " +
                                                         std::to_string(st->failed_item) + ")");
  if (st->failures) return fail(GQD_ERR_NOT_CONVERGED, "GMRES hit maxit in " + std::to_string(st->failures) +
                                                           " solves (first item " +
                                                           std::to_string(st->failed_item) + ")");
  return GQD_OK;
}

gqd_status ready(const gqd_handle* h, bool need_work, const gqd_solver_opts* o) {
  if (!h) return fail(GQD_ERR_INVALID, "handle is NULL");
  if (!h->V || !h->F) return fail(GQD_ERR_STATE, "surfaces not set (gqd_set_surfaces)");
  if (need_work) {
    gqd_status s = check_opts(h, o);
    if (s != GQD_OK) return s;
    if (!h->work) return fail(GQD_ERR_STATE, "workspace not set (gqd_set_workspace)");
    if (h->work_bytes < work_need(h, o->restart))
      return fail(GQD_ERR_STATE, "workspace too small for this restart length");
  }
  return GQD_OK;
}

}  // namespace

extern "C" {

const char* gqd_last_error(void) { return g_last_error.c_str(); }

static gqd_status create2d(gqd_handle** out, const gqd_grid_desc* g);

gqd_status gqd_create(gqd_handle** out, const gqd_grid_desc* g) {
  if (!out || !g) return fail(GQD_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (g->dims == 2) return create2d(out, g);
  if (g->dims != 1) return fail(GQD_ERR_UNSUPPORTED, "dims must be 1 or 2");
  if (g->surfaces != 2) return fail(GQD_ERR_UNSUPPORTED, "only surfaces = 2 is supported");
  if (g->batch < 1) return fail(GQD_ERR_INVALID, "batch must be >= 1");
  if (!g->n || !g->qmin || !g->qmax || !g->mass) return fail(GQD_ERR_INVALID, "NULL grid array");
  if (!(g->mass[0] > 0.0) || !std::isfinite(g->mass[0])) return fail(GQD_ERR_INVALID, "mass must be > 0");
  gqd_handle* h = new (std::nothrow) gqd_handle();
  if (!h) return fail(GQD_ERR_NOMEM, "out of host memory");
  h->batch = g->batch;
  h->mass = g->mass[0];
  h->items.resize(g->batch);
  long long off = 0;
  for (int b = 0; b < g->batch; ++b) {
    const int n = g->n[b];
    const int cls = class_of(n);
    const double L = g->qmax[b] - g->qmin[b];
    if (cls < 0) {
      delete h;
      return fail(GQD_ERR_UNSUPPORTED, "item " + std::to_string(b) + ": n = " + std::to_string(n) +
                                           " (supported: 256, 512, 1024, 2048, 4096)");
    }
    if (!(L > 0.0) || !std::isfinite(L)) {
      delete h;
      return fail(GQD_ERR_INVALID, "item " + std::to_string(b) + ": qmax must exceed qmin");
    }
    ItemMeta& m = h->items[b];
    m.n = n;
    m.cls = cls;
    m.off = off;
    m.voff = off;
    m.foff = off / 2;
    m.dq = L / n;
    m.pscale = 2.0 * M_PI / L;
    off += 2LL * n;
    h->class_lists[cls].push_back(b);
  }
  h->total_complex = off;
  h->h_stats.resize(g->batch);
  auto cleanup = [&](gqd_status s) {
    gqd_destroy(h);
    return s;
  };
  hipError_t e;
  if ((e = hipMalloc(&h->d_items, sizeof(ItemMeta) * g->batch)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc items"));
  if ((e = hipMemcpy(h->d_items, h->items.data(), sizeof(ItemMeta) * g->batch, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy items"));
  for (int c = 0; c < kNumClasses; ++c) {
    if (h->class_lists[c].empty()) continue;
    const size_t bytes = sizeof(int) * h->class_lists[c].size();
    if ((e = hipMalloc(&h->d_lists[c], bytes)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc lists"));
    if ((e = hipMemcpy(h->d_lists[c], h->class_lists[c].data(), bytes, hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMemcpy lists"));
  }
  // per-pass twiddle tables of every plan, evaluated in extended precision and rounded
  // once: entry k (R - 1) + r - 1 of a pass = exp(-2 pi i r k / (Ns R))
  std::vector<double2> tw;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int p = 0; p < kNumPlans; ++p) {
    h->tw_off[p] = (long long)tw.size();
    PassNR ps[6] = {};
    const int np = twiddle_passes(p, ps);
    for (int q = 0; q < np; ++q) {
      const long double L = (long double)ps[q].Ns * ps[q].R;
      for (int k = 0; k < ps[q].Ns; ++k)
        for (int r = 1; r < ps[q].R; ++r) {
          const long double ang = 2.0L * pi * (long double)(r * k) / L;
          tw.push_back(make_double2((double)cosl(ang), (double)-sinl(ang)));
        }
    }
    if ((long long)tw.size() - h->tw_off[p] != plan_table_size(p)) {
      gqd_destroy(h);
      return fail(GQD_ERR_INVALID, "internal: twiddle table size mismatch");
    }
  }
  for (int c = 0; c < kNumClasses; ++c) h->plan[c] = kClassPlans[c][0];
  if ((e = hipMalloc(&h->d_tw, sizeof(double2) * tw.size())) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc twiddles"));
  if ((e = hipMemcpy(h->d_tw, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy twiddles"));
  if ((e = hipMalloc(&h->d_stats, sizeof(ItemStats) * g->batch)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc stats"));
  if ((e = hipMemset(h->d_stats, 0, sizeof(ItemStats) * g->batch)) != hipSuccess) return cleanup(hip_fail(e, "hipMemset stats"));
  if ((e = configure_kernels(kMaxRestart)) != hipSuccess) return cleanup(hip_fail(e, "configure kernels"));
  {
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return cleanup(hip_fail(e, "hipGetDevice"));
    if ((e = scratch_address(dev, &h->scratch)) != hipSuccess) return cleanup(hip_fail(e, "hipGetSymbolAddress scratch"));
  }
  *out = h;
  return GQD_OK;
}

// 2D: every item is an n x n grid with the same n in {64, 128, 256, 512}; qmin, qmax
// per item and axis, one mass per axis.
static gqd_status create2d(gqd_handle** out, const gqd_grid_desc* g) {
  if (g->surfaces != 2) return fail(GQD_ERR_UNSUPPORTED, "only surfaces = 2 is supported");
  if (g->batch < 1) return fail(GQD_ERR_INVALID, "batch must be >= 1");
  if (!g->n || !g->qmin || !g->qmax || !g->mass) return fail(GQD_ERR_INVALID, "NULL grid array");
  for (int d = 0; d < 2; ++d)
    if (!(g->mass[d] > 0.0) || !std::isfinite(g->mass[d])) return fail(GQD_ERR_INVALID, "mass must be > 0");
  const int n = g->n[0];
  int cls = -1;
  for (int c = 0; c < kNumLine2; ++c)
    if (kLine2N[c] == n) cls = c;
  for (int b = 0; b < g->batch; ++b) {
    if (g->n[2 * b] != n || g->n[2 * b + 1] != n || cls < 0)
      return fail(GQD_ERR_UNSUPPORTED, "item " + std::to_string(b) +
                                           ": 2D grids must be n x n with one n in {64, 128, 256, 512}");
    for (int d = 0; d < 2; ++d) {
      const double L = g->qmax[2 * b + d] - g->qmin[2 * b + d];
      if (!(L > 0.0) || !std::isfinite(L))
        return fail(GQD_ERR_INVALID, "item " + std::to_string(b) + ": qmax must exceed qmin");
    }
  }
  gqd_handle* h = new (std::nothrow) gqd_handle();
  if (!h) return fail(GQD_ERR_NOMEM, "out of host memory");
  h->dims = 2;
  h->batch = g->batch;
  h->n2 = n;
  h->line_cls = cls;
  h->mass2[0] = g->mass[0];
  h->mass2[1] = g->mass[1];
  h->items2.resize(g->batch);
  const long long vec = 2LL * n * n;
  for (int b = 0; b < g->batch; ++b) {
    Item2& it = h->items2[b];
    const double L1 = g->qmax[2 * b] - g->qmin[2 * b], L2 = g->qmax[2 * b + 1] - g->qmin[2 * b + 1];
    it.off = b * vec;
    it.dv = (L1 / n) * (L2 / n);
    it.ps0 = 2.0 * M_PI / L1;
    it.ps1 = 2.0 * M_PI / L2;
  }
  h->total_complex = g->batch * vec;
  h->h_stats.resize(g->batch);
  auto cleanup = [&](gqd_status s) {
    gqd_destroy(h);
    return s;
  };
  hipError_t e;
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return cleanup(hip_fail(e, "hipGetDevice"));
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return cleanup(hip_fail(e, "hipDeviceGetAttribute"));
  h->resident_cap = cus * (2048 / kThreads2);
  if ((e = hipMalloc(&h->d_items2, sizeof(Item2) * g->batch)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc items"));
  if ((e = hipMemcpy(h->d_items2, h->items2.data(), sizeof(Item2) * g->batch, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy items"));
  // line twiddles exp(-2 pi i t / n) in extended precision, rounded once
  std::vector<double2> tw(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int t = 0; t < n; ++t) {
    const long double ang = 2.0L * pi * (long double)t / (long double)n;
    tw[t] = make_double2((double)cosl(ang), (double)-sinl(ang));
  }
  if ((e = hipMalloc(&h->d_tw2, sizeof(double2) * n)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc twiddles"));
  if ((e = hipMemcpy(h->d_tw2, tw.data(), sizeof(double2) * n, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy twiddles"));
  // sync: two words per group and two per item, at most resident_cap of each
  if ((e = hipMalloc(&h->d_sync, sizeof(unsigned) * 4 * (size_t)h->resident_cap)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMalloc sync"));
  if ((e = hipMalloc(&h->d_part, sizeof(double) * 2 * (size_t)h->resident_cap * kPart2)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMalloc partials"));
  // statistics of the first group of each item, then of the second (reverse sweep)
  if ((e = hipMalloc(&h->d_stats, 2 * sizeof(ItemStats) * g->batch)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc stats"));
  if ((e = hipMemset(h->d_stats, 0, 2 * sizeof(ItemStats) * g->batch)) != hipSuccess) return cleanup(hip_fail(e, "hipMemset stats"));
  if ((e = configure_kernels2d(kMaxRestart)) != hipSuccess) return cleanup(hip_fail(e, "configure kernels"));
  *out = h;
  return GQD_OK;
}

void gqd_destroy(gqd_handle* h) {
  if (!h) return;
  if (h->d_items2) (void)hipFree(h->d_items2);
  if (h->d_tw2) (void)hipFree(h->d_tw2);
  if (h->d_sync) (void)hipFree(h->d_sync);
  if (h->d_part) (void)hipFree(h->d_part);
  if (h->d_items) (void)hipFree(h->d_items);
  for (int c = 0; c < kNumClasses; ++c)
    if (h->d_lists[c]) (void)hipFree(h->d_lists[c]);
  if (h->d_tw) (void)hipFree(h->d_tw);
  if (h->d_stats) (void)hipFree(h->d_stats);
  release_streams(h);
  delete h;
}

gqd_status gqd_state_size(const gqd_handle* h, long long* n) {
  if (!h || !n) return fail(GQD_ERR_INVALID, "NULL argument");
  *n = h->total_complex;
  return GQD_OK;
}

gqd_status gqd_state_offset(const gqd_handle* h, int item, long long* off) {
  if (!h || !off) return fail(GQD_ERR_INVALID, "NULL argument");
  if (item < 0 || item >= h->batch) return fail(GQD_ERR_INVALID, "item out of range");
  *off = h->dims == 2 ? h->items2[item].off : h->items[item].off;
  return GQD_OK;
}

gqd_status gqd_workspace_size(const gqd_handle* h, const gqd_solver_opts* o, size_t* bytes) {
  if (!h || !bytes) return fail(GQD_ERR_INVALID, "NULL argument");
  gqd_status s = check_opts(h, o);
  if (s != GQD_OK) return s;
  *bytes = work_need(h, o->restart);
  return GQD_OK;
}

gqd_status gqd_set_workspace(gqd_handle* h, void* p, size_t bytes) {
  if (!h || !p) return fail(GQD_ERR_INVALID, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(p) & 15) != 0) return fail(GQD_ERR_INVALID, "workspace must be 16-byte aligned");
  h->work = p;
  h->work_bytes = bytes;
  return GQD_OK;
}

gqd_status gqd_set_surfaces(gqd_handle* h, const double* V, const double* F) {
  if (!h || !V || !F) return fail(GQD_ERR_INVALID, "NULL argument");
  h->V = V;
  h->F = F;
  return GQD_OK;
}

gqd_status gqd_apply_H(gqd_handle* h, const void* in, void* out, void* stream) {
  gqd_status s = ready(h, false, nullptr);
  if (s != GQD_OK) return s;
  if (!in || !out) return fail(GQD_ERR_INVALID, "NULL state pointer");
  if (in == out) return fail(GQD_ERR_INVALID, "psi_in and psi_out must differ");
  if (h->dims == 2) {
    if (!h->work || h->work_bytes < work_need(h, 0))
      return fail(GQD_ERR_STATE, "2D grids need the workspace (gqd_set_workspace) for gqd_apply_H");
    K2Args a = base_args2(h);
    a.mode = kM2ApplyH;
    a.psi = (double2*)in;
    a.aux = (double2*)out;
    a.work = (double2*)h->work;
    return run2d(h, a, (hipStream_t)stream);
  }
  KArgs a = base_args(h);
  a.psi = (double2*)in;
  a.aux = (double2*)out;
  return for_each_class(h, (hipStream_t)stream, a, launch_apply_h);
}

static bool elementary(gqd_method m) { return m == GQD_EULER_EXPLICIT || m == GQD_EULER_IMPLICIT || m == GQD_SOD; }

static int method_code(gqd_method m) {
  switch (m) {
    case GQD_TRAP: return kTrap;
    case GQD_EULER_EXPLICIT: return kEulerExpl;
    case GQD_EULER_IMPLICIT: return kEulerImpl;
    case GQD_SOD: return kSod;
    case GQD_SPLIT_OPERATOR: return kSplit;
    default: return kMidp;
  }
}

static gqd_status propagate_impl(gqd_handle* h, gqd_method m, gqd_scheme sch, int order, double dt,
                                 long long nsteps, const double* dt_item, const long long* nsteps_item,
                                 void* psi, const gqd_solver_opts* o, gqd_stats* st, void* stream) {
  gqd_status s = ready(h, true, o);
  if (s != GQD_OK) return s;
  if (!psi) return fail(GQD_ERR_INVALID, "NULL state pointer");
  if (m != GQD_TRAP && m != GQD_MIDP && m != GQD_SPLIT_OPERATOR && !elementary(m))
    return fail(GQD_ERR_INVALID, "unknown method");
  if (elementary(m) && order != (m == GQD_SOD ? 2 : 1))
    return fail(GQD_ERR_INVALID, "the Euler methods take order 1 and second-order differencing order 2");
  if (!std::isfinite(dt)) return fail(GQD_ERR_INVALID, "dt must be finite");
  if (nsteps < 0) return fail(GQD_ERR_INVALID, "nsteps must be >= 0");
  hipStream_t strm = (hipStream_t)stream;
  if (h->dims == 2) {
    if (elementary(m) || m == GQD_SPLIT_OPERATOR)
      return fail(GQD_ERR_UNSUPPORTED, "the elementary and split-operator methods run on 1D grids");
    if (dt_item || nsteps_item) return fail(GQD_ERR_UNSUPPORTED, "per-item steps are available on 1D grids");
    K2Args a = base_args2(h);
    s = make_gammas(sch, order, &a.gt);
    if (s != GQD_OK) return s;
    a.mode = kM2Propagate;
    a.psi = (double2*)psi;
    a.work = (double2*)h->work;
    a.sc = SolveCfg{o->tol, o->restart, o->maxit, o->literal ? 1 : 0, o->verify ? 1 : 0, o->precond ? 1 : 0};
    a.sc.precond = resolve_precond(h, o, a.gt, dt, false);
    a.method = (m == GQD_TRAP) ? kTrap : kMidp;
    a.dt = dt;
    a.nsteps = nsteps;
    s = run2d(h, a, strm);
    if (s != GQD_OK) return s;
    return st ? collect_stats(h, strm, st) : GQD_OK;
  }
  KArgs a = base_args(h);
  // the elementary methods take whole steps: a one-substep table (tau = 1)
  s = elementary(m) ? make_gammas(GQD_SUZUKI, 2, &a.gt) : make_gammas(sch, order, &a.gt);
  if (s != GQD_OK) return s;
  a.psi = (double2*)psi;
  a.work = (double2*)h->work;
  a.sc = SolveCfg{o->tol, o->restart, o->maxit, o->literal ? 1 : 0, o->verify ? 1 : 0, o->precond ? 1 : 0};
  // (the implicit Euler step solves 1 + i dt H: its half-substep is the whole step)
  a.sc.precond = resolve_precond(h, o, a.gt, elementary(m) ? 2.0 * dt : dt, dt_item != nullptr);
  a.mode = 0;
  a.method = method_code(m);
  a.dt = dt;
  a.nsteps = nsteps;
  a.dt_item = dt_item;
  a.nsteps_item = nsteps_item;
  a.hpsi_valid = 0;
  s = for_each_class(h, strm, a, m == GQD_SPLIT_OPERATOR ? launch_split : launch_run,
                     h->precond_auto ? h->class_precond : nullptr);
  if (s != GQD_OK) return s;
  return st ? collect_stats(h, strm, st) : GQD_OK;
}

gqd_status gqd_propagate(gqd_handle* h, gqd_method m, gqd_scheme sch, int order, double dt,
                         long long nsteps, void* psi, const gqd_solver_opts* o, gqd_stats* st,
                         void* stream) {
  return propagate_impl(h, m, sch, order, dt, nsteps, nullptr, nullptr, psi, o, st, stream);
}

gqd_status gqd_propagate_noalloc(gqd_handle* h, gqd_method m, gqd_scheme sch, int order, double dt,
                                 long long nsteps, void* psi, const gqd_solver_opts* o, gqd_stats* st,
                                 void* stream) {
  if (!h) return fail(GQD_ERR_INVALID, "handle is NULL");
  if (h->dims != 1) return fail(GQD_ERR_UNSUPPORTED, "the allocation-free propagation runs 1D batches");
  if (!h->V || !h->F) return fail(GQD_ERR_STATE, "surfaces not set (gqd_set_surfaces)");
  gqd_status s = check_opts(h, o);
  if (s != GQD_OK) return s;
  if (!psi) return fail(GQD_ERR_INVALID, "NULL state pointer");
  if (m != GQD_TRAP && m != GQD_MIDP && m != GQD_SPLIT_OPERATOR && !elementary(m))
    return fail(GQD_ERR_INVALID, "unknown method");
  if (elementary(m) && order != (m == GQD_SOD ? 2 : 1))
    return fail(GQD_ERR_INVALID, "the Euler methods take order 1 and second-order differencing order 2");
  if (!std::isfinite(dt)) return fail(GQD_ERR_INVALID, "dt must be finite");
  if (nsteps < 0) return fail(GQD_ERR_INVALID, "nsteps must be >= 0");
  const size_t need = work_need(h, o->restart);
  if (need > kScratchBytes)
    return fail(GQD_ERR_INVALID, "this batch needs " + std::to_string(need) + " bytes of workspace at restart " +
                                     std::to_string(o->restart) + "; the static scratch holds " +
                                     std::to_string(kScratchBytes));
  if (!h->scratch) return fail(GQD_ERR_STATE, "no scratch address for this handle's device");
  KArgs a = base_args(h);
  s = elementary(m) ? make_gammas(GQD_SUZUKI, 2, &a.gt) : make_gammas(sch, order, &a.gt);
  if (s != GQD_OK) return s;
  a.psi = (double2*)psi;
  a.work = (double2*)h->scratch;  // nothing in the scratch is read before it is written
  a.sc = SolveCfg{o->tol, o->restart, o->maxit, o->literal ? 1 : 0, o->verify ? 1 : 0, o->precond ? 1 : 0};
  a.sc.precond = resolve_precond(h, o, a.gt, elementary(m) ? 2.0 * dt : dt, false);
  a.mode = 0;
  a.method = method_code(m);
  a.dt = dt;
  a.nsteps = nsteps;
  a.hpsi_valid = 0;
  // every size class on the caller's stream, one after another: no side streams or
  // events are created
  hipStream_t strm = (hipStream_t)stream;
  for (int c = kNumClasses - 1; c >= 0; --c) {
    if (h->class_lists[c].empty()) continue;
    a.list = h->d_lists[c];
    a.nlist = (int)h->class_lists[c].size();
    a.tw = h->d_tw + h->tw_off[h->plan[c]];
    if (h->precond_auto) a.sc.precond = h->class_precond[c];
    GQD_HIP(m == GQD_SPLIT_OPERATOR ? launch_split(h->plan[c], a, strm) : launch_run(h->plan[c], a, strm));
  }
  return st ? collect_stats(h, strm, st) : GQD_OK;
}

gqd_status gqd_propagate_items(gqd_handle* h, gqd_method m, gqd_scheme sch, int order, const double* dt,
                               const long long* nsteps, void* psi, const gqd_solver_opts* o,
                               gqd_stats* st, void* stream) {
  if (!dt || !nsteps) return fail(GQD_ERR_INVALID, "NULL per-item dt or nsteps");
  return propagate_impl(h, m, sch, order, 0.0, 0, dt, nsteps, psi, o, st, stream);
}

gqd_status gqd_list_plans(int n, int* radices, int max_plans, int* count) {
  if (!count) return fail(GQD_ERR_INVALID, "NULL argument");
  const int c = class_of(n);
  if (c < 0) return fail(GQD_ERR_UNSUPPORTED, "no 1D size class n = " + std::to_string(n));
  int k = 0;
  for (int i = 0; i < kMaxPlansPerClass; ++i) {
    const int p = kClassPlans[c][i];
    if (p < 0) continue;
    if (radices && k < max_plans) {
      radices[4 * k] = kPlans[p].R0;
      radices[4 * k + 1] = kPlans[p].R1;
      radices[4 * k + 2] = kPlans[p].R2;
      radices[4 * k + 3] = kPlans[p].R3;
    }
    ++k;
  }
  *count = k;
  return GQD_OK;
}

gqd_status gqd_set_solve_log(gqd_handle* h, int* log, long long per_item) {
  if (!h) return fail(GQD_ERR_INVALID, "NULL handle");
  if (per_item < 0 || (per_item > 0 && !log)) return fail(GQD_ERR_INVALID, "solve log needs a buffer and a size >= 0");
  h->solve_log = per_item > 0 ? log : nullptr;
  h->log_cap = per_item > 0 ? per_item : 0;
  // the kernels read each item's log from its statistics record (2D: both groups')
  const int recs = h->dims == 2 ? 2 * h->batch : h->batch;
  std::vector<ItemStats> st(recs);
  GQD_HIP(hipDeviceSynchronize());
  GQD_HIP(hipMemcpy(st.data(), h->d_stats, sizeof(ItemStats) * recs, hipMemcpyDeviceToHost));
  for (int r = 0; r < recs; ++r) {
    const int b = r % h->batch;
    st[r].log = h->solve_log ? h->solve_log + (size_t)b * h->log_cap : nullptr;
    st[r].log_cap = h->log_cap;
  }
  GQD_HIP(hipMemcpy(h->d_stats, st.data(), sizeof(ItemStats) * recs, hipMemcpyHostToDevice));
  return GQD_OK;
}

gqd_status gqd_composition(gqd_scheme s, int order, double* tau, int max_tau, int* count) {
  if (!count) return fail(GQD_ERR_INVALID, "NULL argument");
  GammaTab gt;
  gqd_status st = make_gammas(s, order, &gt);
  if (st != GQD_OK) return st;
  *count = gt.count;
  if (!tau) return GQD_OK;
  if (max_tau < gt.count) return fail(GQD_ERR_INVALID, "tau holds fewer than the substeps of one step");
  static const double flat_tau[kFlatTauLen] = {GQD_FLAT_TAU_VALUES};
  for (int c = 0; c < gt.count; ++c) {
    if (gt.flat) {
      tau[c] = flat_tau[gt.flat - 1 + c];
      continue;
    }
    // the kernels' product, innermost level first (digit l of c picks level l's gamma)
    double t = 1.0;
    int cc = c;
    for (int l = 0; l < gt.levels; ++l) {
      const int d = cc % gt.arity;
      cc /= gt.arity;
      t = (d == gt.arity / 2 ? gt.mid[l] : gt.side[l]) * t;
    }
    tau[c] = t;
  }
  return GQD_OK;
}

gqd_status gqd_set_wait_limit(gqd_handle* h, int polls) {
  if (!h) return fail(GQD_ERR_INVALID, "NULL handle");
  if (polls < 0) return fail(GQD_ERR_INVALID, "wait limit must be >= 0");
  h->spin_limit = polls;
  return GQD_OK;
}

gqd_status gqd_set_plan(gqd_handle* h, int n, const int* radices) {
  if (!h || !radices) return fail(GQD_ERR_INVALID, "NULL argument");
  if (h->dims != 1) return fail(GQD_ERR_UNSUPPORTED, "transform plans are chosen per 1D size class");
  const int c = class_of(n);
  if (c < 0) return fail(GQD_ERR_UNSUPPORTED, "no 1D size class n = " + std::to_string(n));
  for (int i = 0; i < kMaxPlansPerClass; ++i) {
    const int p = kClassPlans[c][i];
    if (p < 0) continue;
    const Plan& P = kPlans[p];
    if (P.R0 == radices[0] && P.R1 == radices[1] && P.R2 == radices[2] && P.R3 == radices[3]) {
      h->plan[c] = p;
      return GQD_OK;
    }
  }
  return fail(GQD_ERR_UNSUPPORTED, "no plan with these radices for n = " + std::to_string(n));
}

gqd_status gqd_autotune(gqd_handle* h, gqd_method m, gqd_scheme sch, int order, double dt, long long nsteps,
                        void* psi, const gqd_solver_opts* o, int* radices, void* stream) {
  gqd_status s = ready(h, true, o);
  if (s != GQD_OK) return s;
  if (!psi) return fail(GQD_ERR_INVALID, "NULL state pointer");
  if (m != GQD_TRAP && m != GQD_MIDP)
    return fail(GQD_ERR_INVALID, "the autotuner takes the trapezoidal rule or the implicit midpoint");
  if (!std::isfinite(dt)) return fail(GQD_ERR_INVALID, "dt must be finite");
  if (nsteps < 1) return fail(GQD_ERR_INVALID, "nsteps must be >= 1");
  if (radices)
    for (int i = 0; i < 4 * kNumClasses; ++i) radices[i] = 0;
  if (h->dims != 1) return GQD_OK;  // 2D items have one line transform per size
  KArgs a = base_args(h);
  s = make_gammas(sch, order, &a.gt);
  if (s != GQD_OK) return s;
  a.psi = (double2*)psi;
  a.work = (double2*)h->work;
  a.sc = SolveCfg{o->tol, o->restart, o->maxit, o->literal ? 1 : 0, o->verify ? 1 : 0, o->precond ? 1 : 0};
  a.sc.precond = resolve_precond(h, o, a.gt, dt, false);
  a.mode = 0;
  a.method = (m == GQD_TRAP) ? kTrap : kMidp;
  a.dt = dt;
  a.nsteps = nsteps;
  hipStream_t strm = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GQD_HIP(hipEventCreate(&e0));
  GQD_HIP(hipEventCreate(&e1));
  gqd_status result = GQD_OK;
  for (int c = 0; c < kNumClasses && result == GQD_OK; ++c) {
    if (h->class_lists[c].empty()) continue;
    a.list = h->d_lists[c];
    a.nlist = (int)h->class_lists[c].size();
    if (h->precond_auto) a.sc.precond = h->class_precond[c];
    float best[kMaxPlansPerClass];
    for (int k = 0; k < kMaxPlansPerClass; ++k) best[k] = -1.0f;
    // three rounds over the plans that fit in LDS, keeping each plan's fastest launch
    for (int round = 0; round < 3 && result == GQD_OK; ++round)
      for (int k = 0; k < kMaxPlansPerClass && result == GQD_OK; ++k) {
        const int p = kClassPlans[c][k];
        if (p < 0 || lds_bytes(p, o->restart) > kLdsMax) continue;
        a.tw = h->d_tw + h->tw_off[p];
        hipError_t e;
        float ms = 0.0f;
        if ((e = hipEventRecord(e0, strm)) != hipSuccess || (e = launch_run(p, a, strm)) != hipSuccess ||
            (e = hipEventRecord(e1, strm)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
          result = hip_fail(e, "autotune launch");
          break;
        }
        if (best[k] < 0.0f || ms < best[k]) best[k] = ms;
      }
    int pick = -1;
    for (int k = 0; k < kMaxPlansPerClass; ++k)
      if (best[k] >= 0.0f && (pick < 0 || best[k] < best[pick])) pick = k;
    if (pick >= 0) h->plan[c] = kClassPlans[c][pick];
    if (radices) {
      const Plan& P = kPlans[h->plan[c]];
      radices[4 * c] = P.R0;
      radices[4 * c + 1] = P.R1;
      radices[4 * c + 2] = P.R2;
      radices[4 * c + 3] = P.R3;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return result;
}

gqd_status gqd_implicit_step(gqd_handle* h, gqd_method m, double dt, void* psi, const gqd_solver_opts* o,
                             gqd_stats* st, void* stream) {
  if (m != GQD_TRAP && m != GQD_MIDP)
    return fail(GQD_ERR_INVALID, "gqd_implicit_step takes the trapezoidal rule or the implicit midpoint");
  return gqd_propagate(h, m, GQD_SUZUKI, 2, dt, 1, psi, o, st, stream);
}

gqd_status gqd_adjoint(gqd_handle* h, gqd_scheme sch, int order, double dt, long long nsteps, void* psi,
                       void* lambda, double* gF, const gqd_solver_opts* o, gqd_stats* st, void* stream) {
  gqd_status s = ready(h, true, o);
  if (s != GQD_OK) return s;
  if (!psi || !lambda || !gF) return fail(GQD_ERR_INVALID, "NULL pointer");
  if (!std::isfinite(dt)) return fail(GQD_ERR_INVALID, "dt must be finite");
  if (nsteps < 0) return fail(GQD_ERR_INVALID, "nsteps must be >= 0");
  if (h->dims == 2) {
    K2Args a = base_args2(h);
    s = make_gammas(sch, order, &a.gt);
    if (s != GQD_OK) return s;
    a.mode = kM2Adjoint;
    a.method = kMidp;
    a.psi = (double2*)psi;
    a.aux = (double2*)lambda;
    a.gF = gF;
    a.work = (double2*)h->work;
    a.sc = SolveCfg{o->tol, o->restart, o->maxit, o->literal ? 1 : 0, o->verify ? 1 : 0, o->precond ? 1 : 0};
    a.sc.precond = resolve_precond(h, o, a.gt, dt, false);
    a.dt = dt;
    a.nsteps = nsteps;
    hipStream_t strm = (hipStream_t)stream;
    s = run2d(h, a, strm);
    if (s != GQD_OK) return s;
    return st ? collect_stats(h, strm, st) : GQD_OK;
  }
  KArgs a = base_args(h);
  s = make_gammas(sch, order, &a.gt);
  if (s != GQD_OK) return s;
  a.psi = (double2*)psi;
  a.aux = (double2*)lambda;
  a.gF = gF;
  a.work = (double2*)h->work;
  a.sc = SolveCfg{o->tol, o->restart, o->maxit, o->literal ? 1 : 0, o->verify ? 1 : 0, o->precond ? 1 : 0};
  a.sc.precond = resolve_precond(h, o, a.gt, dt, false);
  a.dt = dt;
  a.nsteps = nsteps;
  hipStream_t strm = (hipStream_t)stream;
  a.mode = 1;
  a.method = kMidp;
  s = for_each_class(h, strm, a, launch_run, h->precond_auto ? h->class_precond : nullptr);
  if (s != GQD_OK) return s;
  return st ? collect_stats(h, strm, st) : GQD_OK;
}

gqd_status gqd_diag(gqd_handle* h, const void* psi, double* out, void* stream) {
  gqd_status s = ready(h, false, nullptr);
  if (s != GQD_OK) return s;
  if (!psi || !out) return fail(GQD_ERR_INVALID, "NULL pointer");
  if (h->dims == 2) {
    if (!h->work || h->work_bytes < work_need(h, 0))
      return fail(GQD_ERR_STATE, "2D grids need the workspace (gqd_set_workspace) for gqd_diag");
    K2Args a = base_args2(h);
    a.mode = kM2Diag;
    a.psi = (double2*)psi;
    a.out = out;
    a.work = (double2*)h->work;
    return run2d(h, a, (hipStream_t)stream);
  }
  KArgs a = base_args(h);
  a.psi = (double2*)psi;
  a.out = out;
  return for_each_class(h, (hipStream_t)stream, a, launch_diag);
}

gqd_status gqd_inner(gqd_handle* h, const void* psi, const void* phi, double* out, void* stream) {
  gqd_status s = ready(h, false, nullptr);
  if (s != GQD_OK) return s;
  if (!psi || !phi || !out) return fail(GQD_ERR_INVALID, "NULL pointer");
  if (h->dims == 2) {
    K2Args a = base_args2(h);
    a.mode = kM2Inner;
    a.psi = (double2*)psi;
    a.aux = (double2*)phi;
    a.out = out;
    return run2d(h, a, (hipStream_t)stream);
  }
  KArgs a = base_args(h);
  a.psi = (double2*)psi;
  a.aux = (double2*)phi;
  a.out = out;
  return for_each_class(h, (hipStream_t)stream, a, launch_inner);
}

}  // extern "C"
