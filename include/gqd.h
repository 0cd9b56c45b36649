/* gqd: implicit, exactly unitary geometric integrators for nonadiabatic quantum
 * dynamics in the adiabatic representation, on AMD Instinct MI355X (gfx950), FP64.
 *
 * Method: S. Choi and J. Vanicek, "Efficient geometric integrators for nonadiabatic
 * quantum dynamics. I. The adiabatic representation", J. Chem. Phys. 150, 204112
 * (2019), arXiv:1902.04661.  Atomic units with hbar = 1 (the paper's App. A).
 *
 * Problem.  A batch of independent wavepackets ("items").  Item b is an S = 2
 * component wavefunction on a uniform periodic grid of n_b points on [qmin_b, qmax_b)
 * (right end excluded, dq = L/n, L = qmax - qmin), with
 *   H = (1/2m) [p 1 - i F(q)]^dag [p 1 - i F(q)] + V(q)                   (Eq. 22)
 * where V = diag(V_1, V_2) (adiabatic surfaces) and F is the antisymmetric
 * nonadiabatic coupling, F12 = -F21, F11 = F22 = 0 (Eq. 28).  p acts by the dynamic
 * Fourier method (Sec. II.E): forward DFT sum_j x_j exp(-2 pi i j k/n), multiply by
 * p_k = 2 pi k'/L with k' = k for k < n/2 and k - n otherwise, inverse DFT with 1/n.
 *
 * Memory.  Every buffer argument is a DEVICE pointer owned by the caller (for example
 * torch tensors); the library never frees them and keeps only the V and F pointers
 * given to gqd_set_surfaces, which must stay valid while the handle uses them.
 * Layouts, items concatenated in batch order:
 *   psi  complex128 (interleaved re, im) [item][surface 2][n_b]      ("state vector")
 *   V    float64 [item][surface 2][n_b]
 *   F    float64 [item][n_b]           (F12 along q)
 *   gF   float64 [item][n_b]           (gradient with respect to F12)
 * gqd_state_offset() gives each item's offset in complex elements; V uses the same
 * offsets in doubles; F and gF use half of it.
 *
 * Two dimensions (dims = 2).  Every item is an n x n grid with one n for the whole
 * batch, n in {64, 128, 256, 512}, on [qmin_b1, qmax_b1) x [qmin_b2, qmax_b2) with
 * masses m_1, m_2, and H = sum_d (1/2m_d) A_d^dag A_d + V, A_d = p_d 1 - i F^(d) (the
 * multidimensional form of Eq. 22; p_d acts along axis d as above).  Layouts, q1 the
 * slow and q2 the fast index:
 *   psi  complex128 [item][surface 2][n][n]
 *   V    float64 [item][surface 2][n][n]
 *   F    float64 [item][d 2][n][n]      (F12 along q1, then along q2)
 *   gF   float64 [item][d 2][n][n]
 * so V, F and gF all use the state offsets (in doubles).  A group of workgroups shares
 * each item (cooperative launches); gqd_apply_H and gqd_diag then also need the
 * workspace, gqd_propagate_items is unsupported.  gqd_adjoint gives each item two
 * groups, one for the phi solves and one for the mu solves of every substep, so a 2D
 * workspace holds two regions per item.  The group crosses grid barriers with
 * a bounded wait: if one ever times out the item stops, its state is left unspecified
 * (within a call the midpoint rule may hold it in the workspace), and a call given a
 * gqd_stats pointer returns GQD_ERR_HIP.  With GQD_2D_PLAIN_LAUNCH=1 in the environment the 2D
 * kernel is launched as an ordinary kernel of the same grid instead (for profilers
 * that fail on cooperative launches); the grid never exceeds what can be resident, so
 * on an otherwise idle GPU nothing changes, and a workgroup that could not start would
 * end the call through that time-out rather than hang it.
 *
 * Streams and errors.  Calls are asynchronous on the given hipStream_t (NULL = the
 * null stream) unless they take a gqd_stats pointer that is not NULL: then the call
 * waits for its own work and reports GMRES failures through its return value.
 * Such a call also records each item's cost, and later launches on 1D grids start
 * the most expensive items first (workgroups are dispatched in list order and a launch
 * lasts until its slowest CU finishes); items are independent, so no result changes.
 * A 1D call with a NULL gqd_stats pointer only launches kernels and orders side
 * streams with events, so it can be captured into a HIP graph and replayed (each
 * replay advances the captured state in place); 2D calls launch cooperatively and are
 * not capture-safe.
 * Every call returns a gqd_status; on failure gqd_last_error() (thread-local) holds
 * a message.  Nothing throws across this interface.
 */
#ifndef GQD_H
#define GQD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GQD_OK = 0,
  GQD_ERR_INVALID = -1,       /* bad argument (null pointer, size, option) */
  GQD_ERR_HIP = -2,           /* a HIP runtime call failed */
  GQD_ERR_NOMEM = -3,         /* a host or small device table could not be allocated */
  GQD_ERR_NOT_CONVERGED = -4, /* some GMRES solve hit maxit (Sec. III: large steps stall GMRES) */
  GQD_ERR_UNSUPPORTED = -5,   /* grid size or dimensionality without a kernel */
  GQD_ERR_NONFINITE = -6,     /* a norm became NaN or Inf; that item stopped there */
  GQD_ERR_STATE = -7          /* surfaces or workspace not set */
} gqd_status;

/* Base method.  The geometric second-order methods (Sec. II.C) are composed to higher
 * orders; the elementary methods of Sec. II.B are the paper's non-geometric controls
 * and are not composed. */
typedef enum {
  GQD_TRAP = 0,           /* trapezoidal rule, U_impl(h/2) U_expl(h/2), Eq. (18) */
  GQD_MIDP = 1,           /* implicit midpoint, U_expl(h/2) U_impl(h/2), Eq. (19) */
  GQD_EULER_EXPLICIT = 2, /* psi' = (1 - i dt H) psi, Eq. (13) */
  GQD_EULER_IMPLICIT = 3, /* psi' = (1 + i dt H)^-1 psi, Eq. (14), GMRES as for TRAP/MIDP */
  GQD_SOD = 4,            /* second-order differencing psi(t + dt) = psi(t - dt)
                             - 2 i dt H psi(t), Eq. (16) */
  GQD_SPLIT_OPERATOR = 5  /* DIABATIC representation: H = p^2/2m + W(q) with the real
                             symmetric W read from the surfaces as V = (W11, W22),
                             F = W12; the second-order splitting exp(-i W h/2)
                             exp(-i T h) exp(-i W h/2) of Table I, composed like
                             TRAP and MIDP (Sec. II.D).  1D only. */
} gqd_method;

/* Symmetric composition of the second-order methods (Sec. II.D). */
typedef enum {
  GQD_TRIPLE_JUMP = 0, /* recursive, M = 3 per level, Eq. (20) */
  GQD_SUZUKI = 1,      /* recursive, M = 5 per level, Eq. (21) */
  GQD_OPTIMAL = 2      /* non-recursive: one symmetric composition of the second-order
                          method, the schemes Sec. II.D calls optimal: M = 5, 9, 17
                          substeps with the smallest largest |substep| at orders 4, 6, 8
                          (Suzuki's fractal at order 4; Kahan and Li's at 6 and 8) and
                          M = 35 with the smallest sum of |substeps| at order 10
                          (Sofroniou and Spaletta's).  The fractions come from solving
                          the order and optimality conditions (gqd_composition returns
                          them); order 2 is the method itself */
} gqd_scheme;

typedef struct {
  int dims;           /* D: number of nuclear degrees of freedom, 1 or 2 */
  int surfaces;       /* S: must be 2 */
  int batch;          /* number of items, >= 1 */
  const int* n;       /* host [batch*dims]: grid points per axis; 1D: each one of 256, 512,
                         1024, 2048, 4096; 2D: all equal, one of 64, 128, 256, 512 */
  const double* qmin; /* host [batch*dims] */
  const double* qmax; /* host [batch*dims], > qmin */
  const double* mass; /* host [dims], > 0 */
} gqd_grid_desc;

typedef struct {
  double tol;  /* GMRES stops when its residual estimate <= tol * ||b|| (Euclidean); > 0 */
  int restart; /* Krylov dimension m before a restart, 1..64 */
  int maxit;   /* Arnoldi iterations allowed per solve, >= 1 */
  int literal; /* 1: perform every explicit half-step (3 + I H-applications per substep,
                  Table I); 0: use the Cayley identities (midpoint psi' = 2x - psi,
                  trapezoid reuses H psi' = (b - psi')/(i a)), 2 + I per substep */
  int verify;  /* 1: when the residual estimate meets the tolerance, form x, compute the
                  TRUE residual b - (1 + i a H) x (one more H application) and end the
                  solve only if it meets the tolerance too, else restart GMRES from x;
                  gqd_stats.max_true_resid then covers every solve.  0: stop on the
                  estimate (Sec. II.C solves to machine accuracy; the estimate is the
                  usual GMRES stop test) */
  int precond; /* 1: right-precondition GMRES by the exact inverse of the kinetic part,
                  M = 1 + i a p^2 / 2m (diagonal in momentum space, applied by one more
                  transform pair per iteration): the Arnoldi process runs on
                  (1 + i a H) M^-1 and a cycle ends with x += M^-1 V y, so the residual
                  tested is still that of (1 + i a H) x = b.  The kinetic term sets the
                  stiffness of the system on fine grids: about 4.6 iterations per solve
                  instead of 10 at N = 2048 and 21 at N = 4096.  1D grids only
                  (GQD_ERR_UNSUPPORTED on 2D).  0: plain GMRES, as in Sec. II.C.
                  2: automatic, per size class: preconditioned where a T_max > 1.25, with
                  a the call's largest half-substep |tau_c dt| / 2 and T_max the
                  largest kinetic energy (pi / dq)^2 / 2m of the class's grids, plain
                  elsewhere (where the extra transforms cost more than the saved
                  iterations); with per-item steps every class is preconditioned; on
                  2D grids the same as 0.  gqd_stats.alg_bytes counts each class with
                  its own solver.  Any other value: GQD_ERR_INVALID */
} gqd_solver_opts;

typedef struct {
  long long h_applies;  /* H applications, all items */
  long long iterations; /* Arnoldi iterations, all items */
  long long iterations_sq; /* sum over solves of the squared iteration count */
  long long solves;     /* GMRES solves, all items */
  int max_iters;        /* largest iteration count of one solve */
  int failures;         /* solves that hit maxit */
  int failed_item;      /* first item with a failure or non-finite norm, else -1 */
  int nonfinite;        /* items stopped by a non-finite norm */
  double alg_bytes;     /* algorithmic memory traffic of the call: 32 (I^2 + 4I + 8) bytes
                           per grid point per solve of I iterations (two complex128
                           surfaces, one Gram-Schmidt pass, fused H application);
                           32 (I^2 + 6I + 10) with precond (each iteration writes and
                           reads M^-1 v_j, the cycle's update M^-1 V y once more) */
  double max_true_resid; /* largest |b - (1 + i a H) x| / |b| over the solves that ended
                            on a true residual: every solve with verify = 1; without it
                            only those that ended at their initial residual or after a
                            restart (0 if none did) */
  double impl_bytes;    /* alg_bytes plus the vector passes this implementation makes
                           beyond them, 32 bytes per grid point each: both sweeps (dot
                           products and update) of every second Gram-Schmidt pass, 2(j + 1)
                           vectors at Arnoldi step j; the dot products of the plain 1D
                           solver's three-term pre-projection (v_j, v_(j-1)); the
                           preconditioned solver's second read of v_j, which its
                           shifted Arnoldi step subtracts (1 per iteration); with
                           literal = 1, the explicit half-step's H application (2 per
                           solve).  Reads served from LDS count as well */
} gqd_stats;

typedef struct gqd_handle gqd_handle;

/* Builds host plans and small device tables (item descriptors, twiddles, per-item
 * counters).  The handle owns those tables and frees them in gqd_destroy. */
gqd_status gqd_create(gqd_handle** h, const gqd_grid_desc* g);
void gqd_destroy(gqd_handle* h);

/* Total complex elements of one state vector (all items), and item b's offset. */
gqd_status gqd_state_size(const gqd_handle* h, long long* n_complex);
gqd_status gqd_state_offset(const gqd_handle* h, int item, long long* offset);

/* Workspace for the solver: (restart + 6) state vectors in 1D, (restart + 11) in 2D
 * (gqd_apply_H and gqd_diag on 2D grids need it too).  The caller allocates it
 * (bytes from gqd_workspace_size) and passes it once; it must stay valid. */
gqd_status gqd_workspace_size(const gqd_handle* h, const gqd_solver_opts* o, size_t* bytes);
gqd_status gqd_set_workspace(gqd_handle* h, void* dev_ptr, size_t bytes);

/* Adiabatic surfaces V and coupling F12 (device pointers, layouts above). */
gqd_status gqd_set_surfaces(gqd_handle* h, const double* V, const double* F);

/* psi_out = H psi_in (Eq. 22); psi_in and psi_out must not overlap. */
gqd_status gqd_apply_H(gqd_handle* h, const void* psi_in, void* psi_out, void* stream);

/* One base step of length dt in place: trapezoidal rule or implicit midpoint, each
 * with its implicit half solved by GMRES from the explicit-Euler guess (Sec. II.C).
 * (The elementary methods step through gqd_propagate.) */
gqd_status gqd_implicit_step(gqd_handle* h, gqd_method m, double dt, void* psi,
                             const gqd_solver_opts* o, gqd_stats* st, void* stream);

/* nsteps steps of length dt in place, each the recursive symmetric composition of the
 * base method to the given even order (2, 4, 6, 8, 10): 3^(order/2-1) triple-jump or
 * 5^(order/2-1) Suzuki substeps, gamma_1 applied first (Sec. II.D).  dt may be
 * negative (backward propagation).
 * The elementary methods take order 1 (both Euler methods) or 2 (GQD_SOD), ignore the
 * scheme and run on 1D grids only (GQD_ERR_UNSUPPORTED in 2D).  GQD_SOD carries two
 * states; every call starts it afresh from psi(0) = psi and
 * psi(-dt) = (1 + i dt H - dt^2 H^2 / 2) psi(0), one second-order Runge-Kutta step
 * backwards (Sec. III), so one run is one call with its total step count.  It is
 * stable only for |dt| < 1 / E_max, E_max the largest |eigenvalue| of H (Eq. A48);
 * beyond it the state grows without bound (GQD_ERR_NONFINITE once it overflows). */
gqd_status gqd_propagate(gqd_handle* h, gqd_method m, gqd_scheme s, int order, double dt,
                         long long nsteps, void* psi, const gqd_solver_opts* o,
                         gqd_stats* st, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gqd_propagate on a 1D handle without
 * the caller's workspace.  The solver works in a static device array that the library
 * holds on every GPU it runs on until the process ends (64 MiB; its address is resolved
 * in gqd_create), so the call needs no gqd_set_workspace and calls no hipMalloc, hipFree
 * or other allocating routine, and creates no streams or events: the size classes run
 * one after another on `stream`.  The batch must fit: (restart + 6) state vectors of
 * 32 bytes per grid point (gqd_workspace_size) at most 64 MiB, else GQD_ERR_INVALID.
 * Inputs, outputs, statistics and errors as gqd_propagate.  Every call on one GPU shares
 * that GPU's array and leaves its contents behind (nothing in it is read before the call
 * writes it), so calls that overlap in time on one GPU, on any streams or handles, race
 * and must not be issued.  2D handles: GQD_ERR_UNSUPPORTED. */
gqd_status gqd_propagate_noalloc(gqd_handle* h, gqd_method m, gqd_scheme s, int order, double dt,
                                 long long nsteps, void* psi, const gqd_solver_opts* o,
                                 gqd_stats* st, void* stream);

/* As gqd_propagate, but item b takes its own step dt[b] and step count nsteps[b]
 * (DEVICE arrays of length batch; a negative dt propagates backward).  One launch
 * covers the whole batch, so items with different steps run side by side.  1D only. */
gqd_status gqd_propagate_items(gqd_handle* h, gqd_method m, gqd_scheme s, int order,
                               const double* dt, const long long* nsteps, void* psi,
                               const gqd_solver_opts* o, gqd_stats* st, void* stream);

/* Transform plans of a 1D size n: radices (R0, R1, R2, R3; R3 = 1 means three
 * passes) of each plan, 4 ints per plan in host radices[4 * max_plans] (may be NULL),
 * their number in *count; the first is the default.  Needs no handle or device. */
gqd_status gqd_list_plans(int n, int* radices, int max_plans, int* count);

/* Use the plan with these radices (host int[4]) for every item of size n on this
 * handle from the next call on.  GQD_ERR_UNSUPPORTED if n has no such plan. */
gqd_status gqd_set_plan(gqd_handle* h, int n, const int* radices);

/* Per-solve record (optional): from the next call on, the Arnoldi iteration count of
 * the s-th GMRES solve of item b within a call is written to log[b * per_item + s]
 * for s < per_item (later solves are not recorded).  log is a DEVICE int array of
 * batch * per_item entries owned by the caller; it must stay valid while set.  Solves
 * are numbered in the order the item performs them (substeps in order of application;
 * a reverse sweep solves phi, then mu, per substep: phi at even and mu at odd s).
 * per_item = 0 (log may be NULL) switches the record off.  GQD_ERR_INVALID if
 * per_item < 0, or per_item > 0 with a NULL log. */
gqd_status gqd_set_solve_log(gqd_handle* h, int* log, long long per_item);

/* The substep fractions tau_c (step c has length tau_c dt) of one composed step, in
 * the order they are applied: tau (host) receives *count values when it is not NULL and
 * max_tau >= *count.  Needs no handle or device.  GQD_ERR_UNSUPPORTED for an order
 * without such a scheme. */
gqd_status gqd_composition(gqd_scheme s, int order, double* tau, int max_tau, int* count);

/* Polls a 2D grid barrier (or a hand-off between the two groups of a 2D reverse sweep)
 * makes before it gives up (polls >= 1; 0 restores the default of 2^22, about seconds).
 * When a wait gives up, every workgroup of the item leaves at its next check, the item's
 * state is left part-way, and a call given a gqd_stats pointer returns GQD_ERR_HIP.  A
 * small limit makes a stuck launch fail fast (and lets a test reach that path from the
 * host).  1D handles have no such waits and ignore it.  GQD_ERR_INVALID if polls < 0. */
gqd_status gqd_set_wait_limit(gqd_handle* h, int polls);

/* Transform autotuner.  Each 1D size class has several Stockham plans (radix orders
 * and threads per item, compiled in); this times every plan that fits in LDS at this
 * restart length on the handle's own items (nsteps composed steps of the given method
 * and scheme per launch, three rounds, fastest launch kept) and uses the fastest plan
 * of each class in every later call on the handle.  psi is a SCRATCH state (for
 * example a copy of the initial state): it is propagated in place 3 x (plans) times.
 * radices: optional host int[20]; row c (N = 256, 512, 1024, 2048, 4096) receives the
 * chosen plan's radices (R0, R1, R2, R3; R3 = 1 means three passes), zeros for empty
 * classes.  The results of later calls do not depend on the plan beyond rounding.
 * Synchronous.  2D handles have nothing to tune and return GQD_OK. */
gqd_status gqd_autotune(gqd_handle* h, gqd_method m, gqd_scheme s, int order, double dt, long long nsteps,
                        void* psi, const gqd_solver_opts* o, int* radices, void* stream);

/* Reverse sweep of gqd_propagate for a real loss L(psi(T)), with no stored
 * trajectory: every substep's Cayley map is inverted exactly (time reversibility,
 * App. A, Eq. A40).  On entry psi holds psi(T) and lambda holds dL/dpsi*(T) in the
 * Euclidean sense (dL = 2 Re sum conj(lambda) dpsi); on return psi holds the
 * reconstructed psi(0), lambda holds dL/dpsi*(0), and dL/dF12 on the grid (2D: of each
 * component F^(d)) has been ADDED to gF.  The same sweep serves both base methods (they share the Cayley map). */
gqd_status gqd_adjoint(gqd_handle* h, gqd_scheme s, int order, double dt, long long nsteps,
                       void* psi, void* lambda, double* gF, const gqd_solver_opts* o,
                       gqd_stats* st, void* stream);

/* Per item: out[4b..4b+3] = (||psi||, <psi|H|psi>, P_1, P_2) with the grid inner product
 * <a|b> = dq sum conj(a) b (2D: dq1 dq2 sum) (Sec. II.A, Eq. 6).  out: device float64
 * [batch*4]. */
gqd_status gqd_diag(gqd_handle* h, const void* psi, double* out, void* stream);

/* Per item: out[2b], out[2b+1] = Re, Im <psi|phi>.  out: device float64 [batch*2]. */
gqd_status gqd_inner(gqd_handle* h, const void* psi, const void* phi, double* out, void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* gqd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GQD_H */
