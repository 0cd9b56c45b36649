// Structures shared by the host API (gqd_api.cpp) and the kernels (gqd_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gqd {

constexpr int kMaxLevels = 4;  // compositions up to order 10
constexpr int kMaxArity = 5;   // Suzuki fractal has 5 substeps per level
constexpr int kMaxRestart = 64;
// Gram-Schmidt takes a second pass when the first leaves less than this fraction of
// |w|^2 (the classical 1/2 criterion).  A looser threshold repeats fewer passes, but
// the orthogonality lost by consecutive single passes compounds: on 12-iteration solves
// it reached 1e-13 at a threshold of 1e-2, against 2e-15 at 1/2.
constexpr double kReorthRatio = 0.5;
// workspace per item: m + kWorkExtra state vectors (basis m+1, four slots, one parking slot)
constexpr int kWorkExtra = 6;
constexpr int kNumClasses = 5;  // N = 256, 512, 1024, 2048, 4096
constexpr int kClassN[kNumClasses] = {256, 512, 1024, 2048, 4096};

// Per-item description, resident on the device.
struct ItemMeta {
  int n;                // grid points (1D)
  int cls;              // index into kClassN
  long long off;        // offset of the item's state, in complex elements (= sum of 2n before it)
  long long voff;       // offset into V (doubles), [2][n] per item
  long long foff;       // offset into F (doubles), [n] per item
  double dq;            // grid spacing
  double pscale;        // 2 pi / L: momentum p_k = pscale * k'
};

// Per-item counters written by the propagation kernels.
struct ItemStats {
  long long h_applies;
  long long iterations;
  long long iterations_sq;  // sum over solves of (iterations of the solve)^2
  // vector passes beyond the algorithmic count: the three-term pre-projection's dot
  // products, the preconditioned Arnoldi step's read of v_j for its shift and both
  // sweeps of every second Gram-Schmidt pass
  long long extra_vecs;
  int solves;
  int max_iters;
  int failures;         // solves that hit maxit
  int nonfinite;        // 1 if a norm became NaN/Inf (the item stops there)
  double max_resid;     // largest |b - X x| / |b| of a solve that ended on its true residual
  // set by the host (gqd_set_solve_log), read by the kernels: the Arnoldi iterations of
  // the item's solve s go to log[s] for s < log_cap (two-group reverse sweep: phi
  // solves at even s, mu solves at odd s)
  int* log;
  long long log_cap;
};

struct SolveCfg {
  double tol;
  int m;        // restart length
  int maxit;    // iterations per solve
  int literal;  // 1: perform every explicit half-step
  int verify;   // 1: a solve that converges by its residual estimate ends only once
                // its true residual meets the tolerance (else GMRES restarts from x)
  int precond;  // 1: GMRES right-preconditioned by (1 + i a p^2 / 2m)^-1 (1D)
};

// Composition coefficients per recursion level l (raising order 2l+2 to 2l+4).  Both
// schemes are symmetric with one distinct middle coefficient: triple jump
// (g1, g2, g1), Suzuki (g1, g1, g3, g1, g1).  Digit d of a substep index selects
// mid[l] when d == arity/2 and side[l] otherwise.
// A non-recursive composition lists its substep fractions instead: flat > 0 is one
// plus the offset of its first fraction in the device table of such lists, count its
// length.
struct GammaTab {
  int arity;    // 3 (triple jump) or 5 (Suzuki)
  int levels;   // order/2 - 1
  int count;    // arity^levels substeps per step (flat: the length of the list)
  int flat;     // 0: recursive; else 1 + offset of the list
  double side[kMaxLevels];
  double mid[kMaxLevels];
};

// geometric base methods (composed), then the elementary controls (not composed)
// (kSplit: the split-operator method of the diabatic representation, composed)
enum Method { kTrap = 0, kMidp = 1, kEulerExpl = 2, kEulerImpl = 3, kSod = 4, kSplit = 5 };

struct KArgs {
  const ItemMeta* items;
  const int* list;      // item indices of this launch's size class
  int nlist;
  const double* V;
  const double* F;
  double2* psi;         // state (in-place) / input
  double2* aux;         // second state: H psi output, or lambda for the adjoint
  double* gF;           // adjoint: dL/dF12 accumulation [n] per item (foff layout)
  double* out;          // diagnostics output
  double2* work;        // workspace base, (m + kWorkExtra) vectors of 2n per item
  const double2* tw;    // per-pass twiddle tables of this launch's plan
  double inv2m;         // 1 / (2 mass)
  double mass;
  SolveCfg sc;
  int mode;             // 0 propagate, 1 reverse sweep
  int method;
  double dt;
  long long nsteps;
  const double* dt_item;        // optional per-item step (device), overrides dt
  const long long* nsteps_item; // optional per-item step count (device), overrides nsteps
  GammaTab gt;
  int hpsi_valid;       // trapezoid economy: HPSI slot already holds H psi
  ItemStats* stats;
};

// Stockham plans: radices (R0, R1, R2, R3) of one transform of N points (R3 = 1 means
// three passes), T = N / R0 threads per item (every pass has 2N/R butterflies, a
// multiple of T), and whether the transform ping-pongs between two LDS buffers (one
// barrier per pass, the operator input kept in registers) or works in place.  Each
// size class has one or more plans; the first is the default and gqd_autotune picks
// among them by timing them on the caller's batch.
struct Plan {
  int N, R0, R1, R2, R3;
  bool two_buf;
  // four-step form: the radix-R0 stage on owned points, one exchange through LDS, then
  // the (N/R0)-point transforms of the 2 R0 (surface, k1) slabs, each inside one wave's
  // own LDS region (radices R1, R2, R3); workgroup barriers only around the exchanges
  bool four_step = false;
};
constexpr int kNumPlans = 11;
constexpr Plan kPlans[kNumPlans] = {
    {256, 4, 8, 8, 1, true, true},     // 0
    {256, 4, 4, 4, 4, true},     // 1
    {512, 4, 8, 4, 4, true, true},     // 2
    {512, 8, 8, 8, 1, true},     // 3
    {1024, 4, 8, 8, 4, true, true},    // 4
    {1024, 8, 8, 4, 4, true},    // 5
    {1024, 8, 8, 16, 1, true},   // 6
    {2048, 4, 8, 8, 8, true, true},  // 7
    {2048, 8, 8, 8, 4, true},    // 8
    {2048, 8, 16, 16, 1, true},  // 9
    {4096, 8, 8, 8, 8, false, true},   // 10
};
constexpr int kMaxPlansPerClass = 3;
// plans of each size class, default first; -1 ends a list
constexpr int kClassPlans[kNumClasses][kMaxPlansPerClass] = {
    {0, 1, -1}, {2, 3, -1}, {4, 5, 6}, {7, 8, 9}, {10, -1, -1}};

constexpr int plan_threads(int p) { return kPlans[p].N / kPlans[p].R0; }

// Twiddled passes of one application of p, in execution order (the first forward pass
// has Ns = 1 and needs none): (Ns, R) of each.  Both the host table builder and the
// kernels enumerate them with this function.
struct PassNR {
  int Ns, R;
};
constexpr int twiddle_passes(int plan, PassNR* out) {
  const int R0 = kPlans[plan].R0, R1 = kPlans[plan].R1, R2 = kPlans[plan].R2, R3 = kPlans[plan].R3;
  int n = 0;
  if (kPlans[plan].four_step) {
    // the outer twiddles exp(-2 pi i t k1 / N) (t < N/R0, k1 < R0), then the twiddled
    // passes of the slab transform (forward, the fused one included, then inverse)
    out[n++] = PassNR{kPlans[plan].N / R0, R0};
    if (R3 == 1) {
      out[n++] = PassNR{R1, R2};  // fused
      out[n++] = PassNR{R2, R1};
    } else {
      out[n++] = PassNR{R1, R2};
      out[n++] = PassNR{R1 * R2, R3};  // fused
      out[n++] = PassNR{R3, R2};
      out[n++] = PassNR{R3 * R2, R1};
    }
  } else if (R3 == 1) {
    out[n++] = PassNR{R0, R1};            // forward
    out[n++] = PassNR{R0 * R1, R2};       // forward, fused with the first inverse pass
    out[n++] = PassNR{R2, R1};            // inverse
    out[n++] = PassNR{R2 * R1, R0};       // inverse, to owned points
  } else {
    out[n++] = PassNR{R0, R1};
    out[n++] = PassNR{R0 * R1, R2};
    out[n++] = PassNR{R0 * R1 * R2, R3};  // fused
    out[n++] = PassNR{R3, R2};
    out[n++] = PassNR{R3 * R2, R1};
    out[n++] = PassNR{R3 * R2 * R1, R0};
  }
  return n;
}
// Per-pass twiddle table: entry k (R - 1) + r - 1 = exp(-2 pi i r k / (Ns R)), k < Ns.
constexpr int pass_table_size(PassNR p) { return p.Ns * (p.R - 1); }
constexpr int plan_table_size(int plan) {
  PassNR ps[6] = {};
  const int n = twiddle_passes(plan, ps);
  int t = 0;
  for (int i = 0; i < n; ++i) t += pass_table_size(ps[i]);
  return t;
}
constexpr int pass_table_offset(int plan, int pass) {
  PassNR ps[6] = {};
  twiddle_passes(plan, ps);
  int t = 0;
  for (int i = 0; i < pass; ++i) t += pass_table_size(ps[i]);
  return t;
}

// LDS bytes needed by a launch of a plan with restart length m.
inline size_t lds_bytes(int plan, int m) {
  const int N = kPlans[plan].N;
  const int W = plan_threads(plan) / 64;
  const size_t fft = kPlans[plan].two_buf ? 4 * (size_t)N : 2 * (size_t)N;
  // fft, part [W][m+1], hcol [m+1], g [m+1], sn [m], y [m+1], R [m(m+1)/2]; cs [m], scal [16]
  const size_t c = fft + (size_t)W * (m + 1) + 3 * (size_t)(m + 1) + (size_t)m + (size_t)m * (m + 1) / 2;
  return c * 16 + (size_t)m * 8 + 16 * 8;
}

// ------------------------------------------------------------------ 2D grids
// A 2D item is an n x n grid (n = kLine2N[c]), state [2][n][n] with the second index
// fastest.  A group of G workgroups shares one item: each H application runs as
// "line blocks" (kLineWaves adjacent rows or columns, one wave per line) and every
// vector operation on contiguous chunks of VEC / G elements, with grid barriers
// between the phases.
constexpr int kNumLine2 = 4;
constexpr int kLine2N[kNumLine2] = {64, 128, 256, 512};
constexpr int kLineWaves = 4;                   // lines per block = waves per workgroup
constexpr int kThreads2 = 64 * kLineWaves;
// workspace per 2D item: kWork2Extra fixed slots, then the m + 1 basis vectors
constexpr int kWork2Extra = 10;
// reduction slots per workgroup: m + 1 complex dots plus a few reals
constexpr int kPart2 = 2 * (kMaxRestart + 1) + 8;

struct Item2 {
  long long off;        // state offset (complex elements) = V offset (doubles) = F offset
  double dv;            // volume element dq1 dq2
  double ps0, ps1;      // 2 pi / L along q1 (slow index) and q2 (fast index)
};

enum Mode2 { kM2Propagate = 0, kM2Adjoint = 1, kM2ApplyH = 2, kM2Diag = 3, kM2Inner = 4 };

struct K2Args {
  const Item2* items;
  int batch;
  int G;                // workgroups per item (power of two)
  const double* V;      // [2][n][n] per item
  const double* F;      // [2][n][n] per item: F12 along q1, along q2
  double2* psi;
  double2* aux;         // H psi output / lambda / second state of an inner product
  double* gF;           // adjoint: [2][n][n] per item
  double* out;          // diagnostics / inner product output
  double2* work;        // (kWork2Extra + m + 1) vectors of 2 n^2 per item
  long long work_stride;
  const double2* tw;    // exp(-2 pi i t / n), t < n
  double inv2m0, inv2m1;
  double mass0, mass1;
  SolveCfg sc;
  int mode;
  int method;
  double dt;
  long long nsteps;
  GammaTab gt;
  ItemStats* stats;
  ItemStats* stats1;    // roles = 2: the second group's statistics
  // groups of G workgroups per item: 1, or 2 for the reverse sweep (phi and mu solved
  // side by side, each on its own group with its own workspace region)
  int roles;
  unsigned* sync;       // per group: [0] arrivals, [1] abort flag; then per item, when
                        // roles = 2: [0] mu ready, [1] gradient done (zeroed before launch)
  double* part;         // per group: [2][G][kPart2]
  int spin_limit;       // polls of a grid barrier before it gives up and aborts
};

// LDS bytes of the 2D kernel at line length n and restart length m.
inline size_t lds_bytes2(int n, int m) {
  const size_t lines = 4 * (size_t)kLineWaves * n;  // two buffers x two surfaces per wave
  const size_t c = lines + n + 2 * (size_t)(m + 1) + 2 * (size_t)m + (size_t)m * (m + 1) / 2 + (m + 1);
  const size_t d = (size_t)(kLineWaves + 1) * kPart2 + m + 16;
  return c * 16 + d * 8 + 64;
}

// The allocation-free entry point's workspace: a static device array of this size per
// GPU (gqd_kernels.hip), its address resolved once per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
hipError_t scratch_address(int device, void** ptr);

// Kernel launchers (gqd_kernels.hip).  Each launches the items of a.list with one plan
// (kPlans index) on `stream`.
hipError_t launch_apply_h(int plan, const KArgs& a, hipStream_t stream);
hipError_t launch_run(int plan, const KArgs& a, hipStream_t stream);  // propagate / adjoint
hipError_t launch_split(int plan, const KArgs& a, hipStream_t stream);  // diabatic split-operator
hipError_t launch_diag(int plan, const KArgs& a, hipStream_t stream);
hipError_t launch_inner(int plan, const KArgs& a, hipStream_t stream);
hipError_t configure_kernels(int m_max);
// 2D launcher (gqd_kernels2d.hip): cooperative launch of batch * G workgroups.
hipError_t launch_run2d(int line_cls, const K2Args& a, hipStream_t stream);
hipError_t configure_kernels2d(int m_max);
// Most workgroups of the 2D kernel that can be resident at once on the current device.
hipError_t max_resident2d(int line_cls, int m, int* blocks);

}  // namespace gqd
