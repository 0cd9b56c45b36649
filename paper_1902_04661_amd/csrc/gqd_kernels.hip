// gfx950 kernels for the implicit geometric integrators of Choi & Vanicek,
// J. Chem. Phys. 150, 204112 (2019).  One workgroup owns one 1D two-surface
// wavepacket for a whole call: every H application, every Arnoldi iteration and
// every composition substep of that item runs inside the workgroup, with vectors
// on owned points in registers, the Fourier passes in LDS and the Krylov basis in
// the item's slice of the workspace.
#include "gqd_device.hpp"
#include "gqd_internal.h"
#include "gqd_compositions.h"

#include <mutex>

namespace gqd {

// The preconditioned Arnoldi step takes a second Gram-Schmidt pass when the first keeps
// less than this fraction of |w|^2 (|w'| < |w| / 2).  A kept fraction f leaves the new
// vector's components along the basis at about eps / sqrt(f) of its norm, so passes
// that keep 25-50 % (the common case on the shifted operator) lose at most twice the
// orthogonality of a pass that keeps all; the plain solver's 1/2 would repeat them.  On
// a drawn N = 2048 packet over one Suzuki-8 step of 20 a.u. the largest |V^H V - 1| is
// 4.5e-15 against 5.1e-15 at 1/2, the true residuals and iteration counts unchanged.
constexpr double kReorthRatioPrec = 0.25;


template <int PLAN>
struct Eng {
  static constexpr int N = kPlans[PLAN].N;
  static constexpr int R0 = kPlans[PLAN].R0, R1 = kPlans[PLAN].R1, R2 = kPlans[PLAN].R2, R3 = kPlans[PLAN].R3;
  static constexpr int T = N / R0;
  static constexpr int W = T / 64;
  static_assert(T % 64 == 0, "whole waves only");
  static constexpr int RF = (R3 == 1) ? R2 : R3;  // radix of the fused k-space pass
  static constexpr size_t VEC = 2 * (size_t)N;    // complex elements of one state vector
  // two-buffer classes: ping-pong LDS transform buffers (one barrier per pass) and the
  // operator input kept in registers; in-place classes: one buffer, the input re-read
  // and the partial H result parked in the workspace
  static constexpr bool kPP = kPlans[PLAN].two_buf;
  static constexpr bool kFS = kPlans[PLAN].four_step;
  // four-step form: slabs of M = N / R0 points, 2 R0 of them, SPW per wave
  static constexpr int M = N / R0;
  static constexpr int SPW = (2 * R0) / W;
  static_assert(!kFS || SPW * W == 2 * R0, "four-step plans: whole slabs per wave");
  // waves per SIMD the register allocation must leave room for.  Plans whose threads
  // own R0 <= 4 points per surface are held to 256 VGPRs (two waves per SIMD): with
  // the Gram-Schmidt loads issued in bursts the allocator would otherwise spill into
  // AGPRs and halve the occupancy.
  static constexpr int WPE = R0 <= 4 ? 2 : 1;
  // Gram-Schmidt sweeps take two basis vectors per turn when a thread owns few points
  static constexpr int GSV = (R0 <= 4) ? 2 : 1;
  // surfaces per burst of Gram-Schmidt loads: GSV * SB * R0 loads in flight per lane
  static constexpr int SB = (R0 <= 4) ? 2 : 1;

  struct OV {
    cplx v[2][R0];
  };

  using LP = GQD_L cplx*;
  struct Ctx {
    GQD_L cplx* fft;   // [2N] (in-place) or [4N] (two buffers)
    GQD_L cplx* part;  // [W][kmax]
    GQD_L cplx* hcol;  // [kmax]
    GQD_L cplx* g;     // [kmax]
    GQD_L cplx* sn;    // [m]
    GQD_L cplx* y;     // [m + 1]
    GQD_L cplx* R;     // [m(m+1)/2], column j at j(j+1)/2
    GQD_L double* cs;     // [m]
    GQD_L double* scal;   // [16]
    int kmax;
    const double* V;   // item's V, [2][N]
    const double* F;   // item's F12, [N]
    const cplx* tw;
    double pscale;
    double inv2m;
  };

  // LDS slot of transform element i in a swizzled buffer: the 8-element block index
  // (bits 3-5) is XORed into the low three bits.  Two writes of the transform give each
  // thread a run of R consecutive elements (the register-held first pass and the fused
  // k-space pass); unswizzled, eight lanes of such a 16-byte store hit the same four
  // banks.  Only those two outputs are swizzled, and only the passes that read them
  // apply the map; where a butterfly's inputs are a multiple of 64 elements apart the
  // XOR term is the same for all of them and is computed once.
  static __device__ __forceinline__ int swz(int i) { return i ^ ((i >> 3) & 7); }

  // owned point r of this lane; lane_tid() keeps address arithmetic local to its use
  static __device__ __forceinline__ int pt(int r) { return lane_tid() + r * T; }

  static __device__ Ctx make_ctx(GQD_L cplx* smem, int m, const KArgs& a, const ItemMeta& im) {
    Ctx c;
    const int kmax = m + 1;
    c.kmax = kmax;
    c.fft = smem;
    c.part = c.fft + (kPP ? 4 : 2) * N;
    c.hcol = c.part + W * kmax;
    c.g = c.hcol + kmax;
    c.sn = c.g + kmax;
    c.y = c.sn + m;
    c.R = c.y + (m + 1);
    c.cs = (GQD_L double*)(c.R + (m * (m + 1)) / 2);
    c.scal = c.cs + m;
    c.V = a.V + im.voff;
    c.F = a.F + im.foff;
    c.tw = (const cplx*)a.tw;
    c.pscale = im.pscale;
    c.inv2m = a.inv2m;
    return c;
  }

  // ------------------------------------------------------------ owned-point vectors
  static __device__ __forceinline__ void load(OV& x, const cplx* __restrict__ gp) {
    const GQD_G cplx* g = opaque(gp);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int r = 0; r < R0; ++r) x.v[s][r] = g[s * N + pt(r)];
    __builtin_amdgcn_sched_barrier(0);
  }
  static __device__ __forceinline__ void store(const OV& x, cplx* __restrict__ gp) {
    GQD_G cplx* g = opaque(gp);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int r = 0; r < R0; ++r) g[s * N + pt(r)] = x.v[s][r];
  }
  static __device__ __forceinline__ double norm2(const OV& x) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int r = 0; r < R0; ++r) acc += cabs2(x.v[s][r]);
    return acc;
  }

  // ------------------------------------------------------------------- reductions
  // Workgroup sum of one real; every thread returns the same value (same order).
  static __device__ double block_sum1(double v, const Ctx& c) {
    v = wave_sum(v);
    GQD_L double* p = (GQD_L double*)c.part;
    if ((threadIdx.x & 63) == 0) p[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += p[w];
    __syncthreads();
    return uniform_d(s);
  }

  // Gram-Schmidt stash (four-step plans): between transforms the LDS transform buffers
  // are idle, so the sweep's last turn (the newest one or two basis vectors) is parked
  // there at each thread's own points (slot q at fft + q 2N; in-place plans sweep one
  // vector per turn and use slot 0 only) by the first dot-product sweep and read back
  // by the update and by a second pass.  Each location is only ever touched by its own
  // thread here, and the four-step transform touches it only from the same thread or
  // behind its workgroup barriers.
  static constexpr bool kStash = kFS && (kPP || GSV == 1);
  enum { kStashOff = 0, kStashFill = 1, kStashUse = 2 };

  // dst[i] = sum conj(V_i) w over the item, i < K (V_i = basis + i*VEC); dst in LDS.
  // With with_norm, dst[K] = (||w||^2, 0) comes out of the same reduction.  MODE: fill
  // the stash from the last turn, or read the last turn from it.
  template <int MODE = kStashOff>
  static __device__ void block_dots(const cplx* __restrict__ basis, const OV& w, int K,
                                    const Ctx& c, GQD_L cplx* dst, bool with_norm = false) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (with_norm) {
      const double nn = wave_sum(norm2(w));
      if (lane == 0) c.part[wv * c.kmax + K] = mk(nn, 0.0);
    }
    // two basis vectors per turn so that their loads and reductions overlap; all loads
    // of a turn (or of one surface, for R0 = 8) are issued before the first use
#pragma unroll 1
    for (int i = 0; i < K; i += GSV) {
      const bool two = GSV == 2 && i + 1 < K;
      const bool last = kStash && MODE != kStashOff && i + GSV >= K;
      const GQD_G cplx* Va = opaque(basis + (size_t)i * VEC);
      const GQD_G cplx* Vb = opaque(basis + (size_t)(two ? i + 1 : i) * VEC);
      const GQD_L cplx* Sa = c.fft;
      const GQD_L cplx* Sb = c.fft + (two ? 2 * N : 0);
      double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
#pragma unroll
      for (int s0 = 0; s0 < 2; s0 += SB) {
        cplx a[SB][R0], b[SB][R0];
        if (MODE == kStashUse && last) {
#pragma unroll
          for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              a[s][r] = Sa[(s0 + s) * N + pt(r)];
              if constexpr (GSV == 2) b[s][r] = Sb[(s0 + s) * N + pt(r)];
            }
        } else {
#pragma unroll
          for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              a[s][r] = Va[(s0 + s) * N + pt(r)];
              if constexpr (GSV == 2) b[s][r] = Vb[(s0 + s) * N + pt(r)];
            }
          if (MODE == kStashFill && last) {
            GQD_L cplx* Wa = c.fft;
            GQD_L cplx* Wb = c.fft + 2 * N;
#pragma unroll
            for (int s = 0; s < SB; ++s)
#pragma unroll
              for (int r = 0; r < R0; ++r) {
                Wa[(s0 + s) * N + pt(r)] = a[s][r];
                if constexpr (GSV == 2) {
                  if (two) Wb[(s0 + s) * N + pt(r)] = b[s][r];
                }
              }
          }
        }
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) {
            const cplx z = w.v[s0 + s][r];
            ax += a[s][r].x * z.x + a[s][r].y * z.y;
            ay += a[s][r].x * z.y - a[s][r].y * z.x;
            if constexpr (GSV == 2) {
              bx += b[s][r].x * z.x + b[s][r].y * z.y;
              by += b[s][r].x * z.y - b[s][r].y * z.x;
            }
          }
      }
      ax = wave_sum(ax);
      ay = wave_sum(ay);
      if constexpr (GSV == 2) {
        bx = wave_sum(bx);
        by = wave_sum(by);
      }
      if (lane == 0) {
        c.part[wv * c.kmax + i] = mk(ax, ay);
        if (two) c.part[wv * c.kmax + i + 1] = mk(bx, by);
      }
    }
    __syncthreads();
    const int Kt = with_norm ? K + 1 : K;
    for (int i = threadIdx.x; i < Kt; i += T) {
      cplx s = mk(0.0, 0.0);
#pragma unroll
      for (int w2 = 0; w2 < W; ++w2) s = cadd(s, c.part[w2 * c.kmax + i]);
      dst[i] = s;
    }
    __syncthreads();
  }

  // w -= sum_i h[i] V_i, i < K (h in LDS).  All loads of a turn are issued before the
  // first use, so that a wave keeps them in flight together.  USE: the last turn comes
  // from the stash (filled by the dot-product sweep over the same K).
  template <bool USE = false>
  static __device__ void block_axpy(const cplx* __restrict__ basis, const GQD_L cplx* h, int K, OV& w,
                                    const Ctx& c) {
#pragma unroll 1
    for (int i = 0; i < K; i += GSV) {
      const bool two = GSV == 2 && i + 1 < K;
      const bool last = kStash && USE && i + GSV >= K;
      const GQD_G cplx* Va = opaque(basis + (size_t)i * VEC);
      const GQD_G cplx* Vb = opaque(basis + (size_t)(two ? i + 1 : i) * VEC);
      const GQD_L cplx* Sa = c.fft;
      const GQD_L cplx* Sb = c.fft + (two ? 2 * N : 0);
      const cplx ha = h[i];
      const cplx hb = two ? h[i + 1] : mk(0.0, 0.0);
#pragma unroll
      for (int s0 = 0; s0 < 2; s0 += SB) {
        cplx a[SB][R0], b[SB][R0];
        if (last) {
#pragma unroll
          for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              a[s][r] = Sa[(s0 + s) * N + pt(r)];
              if constexpr (GSV == 2) b[s][r] = Sb[(s0 + s) * N + pt(r)];
            }
        } else {
#pragma unroll
          for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              a[s][r] = Va[(s0 + s) * N + pt(r)];
              if constexpr (GSV == 2) b[s][r] = Vb[(s0 + s) * N + pt(r)];
            }
        }
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) {
            w.v[s0 + s][r] = csub(w.v[s0 + s][r], cmul(ha, a[s][r]));
            if constexpr (GSV == 2) w.v[s0 + s][r] = csub(w.v[s0 + s][r], cmul(hb, b[s][r]));
          }
      }
    }
  }

  // --------------------------------------------------------------- Fourier passes
  // Twiddles come from per-pass tables (built by the host): butterfly k of a pass with
  // stride Ns and radix R finds exp(-2 pi i r k / (Ns R)), r = 1..R-1, contiguously at
  // tw + offset + k (R - 1).  Inverse passes multiply by the conjugate.
  template <int S>
  static __device__ __forceinline__ cplx twmul(cplx x, cplx w) {
    return S < 0 ? cmul(x, w) : mk(x.x * w.x + x.y * w.y, x.y * w.x - x.x * w.y);
  }

  // Twiddles of the butterflies this thread handles in pass P (radix R, stride Ns): the
  // kinetic loop loads them one pass ahead, before the barrier that closes the previous
  // pass, so their latency overlaps the wait.
  template <int R, int Ns>
  struct TwS {
    static constexpr int PER = (2 * N / R) / T;
    cplx w[PER][R - 1];
  };
  template <int R, int Ns, int P>
  static __device__ __forceinline__ void tw_load(TwS<R, Ns>& t, const GQD_G cplx* tw) {
    constexpr int OFF = pass_table_offset(PLAN, P);
    const int tid = lane_tid();
#pragma unroll
    for (int q = 0; q < TwS<R, Ns>::PER; ++q) {
      const int b = tid + q * T;
      const int k = (b % (N / R)) % Ns;
      const GQD_G cplx* tk = tw + OFF + k * (R - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) t.w[q][r - 1] = tk[r - 1];
    }
  }

  // One Stockham pass over both surfaces, src -> dst (dst == src when in place).
  // Butterfly j (< N/R) of surface s reads x[j + r N/R], twiddles by w_{Ns R}^{r k}
  // (k = j mod Ns), applies the radix-R DFT and writes y[(j/Ns) Ns R + k + r Ns].
  // `next` issues the next pass's twiddle loads before the closing barrier.
  template <int R, int Ns, int S, bool SWIN = false, class Next>
  static __device__ __forceinline__ void pass(const GQD_L cplx* src, GQD_L cplx* dst, const TwS<R, Ns>& tw,
                                              Next&& next) {
    constexpr int NB = 2 * N / R;
    static_assert(NB % T == 0, "butterflies must be a multiple of the thread count");
    constexpr int PER = NB / T;
    cplx x[PER][R];
    int tid = lane_tid();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int b = tid + q * T;
      const int s = b / (N / R), j = b % (N / R);
      if constexpr (SWIN && (N / R) % 64 == 0) {
        const int i0 = s * N + swz(j);  // inputs 64k apart share the XOR term
#pragma unroll
        for (int r = 0; r < R; ++r) x[q][r] = src[i0 + r * (N / R)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = s * N + j + r * (N / R);
          x[q][r] = src[SWIN ? swz(i) : i];
        }
      }
    }
    if constexpr (!kPP) __syncthreads();  // in place: all reads before any write
    tid = lane_tid();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int b = tid + q * T;
      const int s = b / (N / R), j = b % (N / R);
      const int k = j % Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) x[q][r] = twmul<S>(x[q][r], tw.w[q][r - 1]);
      DFT<R, S>::run(x[q]);
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[s * N + base + r * Ns] = x[q][r];
    }
    next();
    __syncthreads();
  }

  // Fused last forward pass (radix RF, Ns = N/RF), momentum multiply and first
  // inverse pass (radix RF, Ns = 1): butterfly j's forward outputs are the k-space
  // points j + r N/RF, exactly the inputs of the inverse butterfly j.
  // KM = 1: multiply by exp(-i ktau p_k^2) / N (the kinetic factor of a split-operator
  // step, ktau = tau / 2m); KM = 2: by (1 + i ktau p_k^2)^-1 / N (the inverse of the
  // kinetic part of 1 + i a H, ktau = a / 2m); KM = 0: by p_k / N
  template <int KM = 0, class Next>
  static __device__ __forceinline__ void fused_kspace(const GQD_L cplx* src, GQD_L cplx* dst,
                                                      const TwS<RF, N / RF>& tw, const Ctx& c, Next&& next,
                                                      double ktau = 0.0) {
    constexpr int NB = 2 * N / RF;
    static_assert(NB % T == 0, "fused pass butterflies");
    constexpr int PER = NB / T;
    constexpr int Ns = N / RF;
    cplx x[PER][RF];
    int tid = lane_tid();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int b = tid + q * T;
      const int s = b / Ns, j = b % Ns;
#pragma unroll
      for (int r = 0; r < RF; ++r) x[q][r] = src[s * N + j + r * Ns];
    }
    if constexpr (!kPP) __syncthreads();
    const double scale = opaque_d(c.pscale) / (double)N;
    tid = lane_tid();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int b = tid + q * T;
      const int s = b / Ns, j = b % Ns;
#pragma unroll
      for (int r = 1; r < RF; ++r) x[q][r] = cmul(x[q][r], tw.w[q][r - 1]);
      DFT<RF, -1>::run(x[q]);
#pragma unroll
      for (int r = 0; r < RF; ++r) {
        const int kk = j + r * Ns;                      // k-space index
        const int kp = (kk < N / 2) ? kk : kk - N;      // signed wavenumber
        if constexpr (KM == 1) {
          const double pk = scale * (double)N * (double)kp;
          double sn, cs;
          sincos(-ktau * pk * pk, &sn, &cs);
          x[q][r] = cscale(cmul(x[q][r], mk(cs, sn)), 1.0 / (double)N);
        } else if constexpr (KM == 2) {
          // (1 + i ktau p^2)^-1 / N = (1 - i q) / (N (1 + q^2)), q = ktau p^2
          const double pk = scale * (double)N * (double)kp;
          const double qk = ktau * pk * pk;
          const double inv = 1.0 / ((double)N * (1.0 + qk * qk));
          x[q][r] = mk((x[q][r].x + qk * x[q][r].y) * inv, (x[q][r].y - qk * x[q][r].x) * inv);
        } else {
          x[q][r] = cscale(x[q][r], scale * (double)kp);  // p_k / N
        }
      }
      DFT<RF, +1>::run(x[q]);
#pragma unroll
      for (int r = 0; r < RF; ++r) dst[s * N + swz(j * RF + r)] = x[q][r];
    }
    next();
    __syncthreads();
  }

  // ---------------------------------------------------------- four-step transform
  // n = M n1 + n2 and k = k1 + R0 k2 (n1, k1 < R0; n2, k2 < M = N / R0):
  //   X[k1 + R0 k2] = sum_n2 w_M^(n2 k2) w_N^(n2 k1) sum_n1 x[M n1 + n2] w_R0^(n1 k1).
  // Thread t = n2 owns x[M n1 + t]: the inner sums are a radix-R0 DFT in registers.
  // One exchange writes the (surface s, k1) slab q = s R0 + k1 at q M; wave w then owns
  // slabs w SPW ... w SPW + SPW - 1 and runs the outer sums as a Stockham transform of M
  // points (radices R1, R2, R3) in its own region, the k-space factor inside the fused
  // pass as in the whole-transform form.  The inverse ends with the outer twiddle
  // w_N^(-n2 k1) and returns through one exchange to owned points.  Passes inside a wave
  // are ordered by wave-level synchronisation; only the exchanges need workgroup
  // barriers.  Two-buffer plans exchange forward through b0 and work and exchange back
  // in b1; in-place plans do all of it in b0 (and end with a barrier, as the next
  // application's exchange overwrites it).
  static __device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // One Stockham pass of radix R (stride Ns, sign S) over the wave's slabs: butterfly
  // b = lane + 64 q is butterfly j = b mod (M/R) of slab e = b / (M/R); it reads
  // x[e M + j + r M/R], twiddles by table TP (none for TP < 0), applies the DFT and writes
  // y[e M + (j/Ns) Ns R + j mod Ns + r Ns].  All of the wave's loads come before its
  // stores, so src may equal dst.  SWIN / SWOUT route the input / output index through
  // swz; OUTER multiplies output n2 = j + r M/R by conj(w_N^(n2 k1)) of the slab's k1.
  template <int R, int Ns, int S, int TP, bool SWIN, bool SWOUT, bool OUTER>
  static __device__ __forceinline__ void wpass(const GQD_L cplx* src, GQD_L cplx* dst, const Ctx& c,
                                               int slab0) {
    constexpr int NR = M / R;
    constexpr int NB = SPW * NR;
    static_assert(NB % 64 == 0, "whole butterflies per lane");
    constexpr int PER = NB / 64;
    cplx x[PER][R];
    {
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int b = l + 64 * q, e = b / NR, j = b % NR;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = e * M + j + r * NR;
          x[q][r] = src[SWIN ? swz(i) : i];
        }
      }
    }
    if constexpr (TP >= 0) {
      const GQD_G cplx* tw = opaque(c.tw) + pass_table_offset(PLAN, TP);
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int k = ((l + 64 * q) % NR) % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) x[q][r] = twmul<S>(x[q][r], tw[k * (R - 1) + r - 1]);
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) DFT<R, S>::run(x[q]);
    if constexpr (OUTER) {
      const GQD_G cplx* tw0 = opaque(c.tw) + pass_table_offset(PLAN, 0);
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int b = l + 64 * q, e = b / NR, j = b % NR;
        const int k1 = (slab0 + e) % R0;
        if (k1 != 0) {
#pragma unroll
          for (int r = 0; r < R; ++r) x[q][r] = twmul<+1>(x[q][r], tw0[(j + r * NR) * (R0 - 1) + k1 - 1]);
        }
      }
    }
    {
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int b = l + 64 * q, e = b / NR, j = b % NR;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int o = e * M + (j / Ns) * Ns * R + j % Ns + r * Ns;
          dst[SWOUT ? swz(o) : o] = x[q][r];
        }
      }
    }
  }
  // Fused last forward pass (radix RF, Ns = M/RF, table TP), k-space factor and first
  // inverse pass (radix RF, Ns = 1) over the wave's slabs: forward output r of butterfly
  // j of slab e is X[k1 + R0 (j + r M/RF)]; the inverse writes y[e M + j RF + r] through swz.
  template <int KM, int TP, bool SWIN>
  static __device__ __forceinline__ void wfused(const GQD_L cplx* src, GQD_L cplx* dst, const Ctx& c,
                                                int slab0, double ktau) {
    constexpr int NR = M / RF;
    constexpr int NB = SPW * NR;
    static_assert(NB % 64 == 0, "whole butterflies per lane");
    constexpr int PER = NB / 64;
    cplx x[PER][RF];
    {
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int b = l + 64 * q, e = b / NR, j = b % NR;
#pragma unroll
        for (int r = 0; r < RF; ++r) {
          const int i = e * M + j + r * NR;
          x[q][r] = src[SWIN ? swz(i) : i];
        }
      }
    }
    {
      const GQD_G cplx* tw = opaque(c.tw) + pass_table_offset(PLAN, TP);
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = (l + 64 * q) % NR;
#pragma unroll
        for (int r = 1; r < RF; ++r) x[q][r] = cmul(x[q][r], tw[j * (RF - 1) + r - 1]);
      }
    }
    const double scale = opaque_d(c.pscale) / (double)N;
    {
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int b = l + 64 * q, e = b / NR, j = b % NR;
        const int k1 = (slab0 + e) % R0;
        DFT<RF, -1>::run(x[q]);
#pragma unroll
        for (int r = 0; r < RF; ++r) {
          const int kk = k1 + R0 * (j + r * NR);          // k-space index
          const int kp = (kk < N / 2) ? kk : kk - N;      // signed wavenumber
          if constexpr (KM == 1) {
            const double pk = scale * (double)N * (double)kp;
            double sn, cs;
            sincos(-ktau * pk * pk, &sn, &cs);
            x[q][r] = cscale(cmul(x[q][r], mk(cs, sn)), 1.0 / (double)N);
          } else if constexpr (KM == 2) {
            // (1 + i ktau p^2)^-1 / N = (1 - i q) / (N (1 + q^2)), q = ktau p^2
            const double pk = scale * (double)N * (double)kp;
            const double qk = ktau * pk * pk;
            const double inv = 1.0 / ((double)N * (1.0 + qk * qk));
            x[q][r] = mk((x[q][r].x + qk * x[q][r].y) * inv, (x[q][r].y - qk * x[q][r].x) * inv);
          } else {
            x[q][r] = cscale(x[q][r], scale * (double)kp);  // p_k / N
          }
        }
        DFT<RF, +1>::run(x[q]);
      }
    }
    {
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int b = l + 64 * q, e = b / NR, j = b % NR;
#pragma unroll
        for (int r = 0; r < RF; ++r) dst[swz(e * M + j * RF + r)] = x[q][r];
      }
    }
  }
  // wfused with two results from one forward transform: dst gets the inverse's first
  // pass of M^-1 X and dst2 that of p M^-1 X, M = 1 + i ktau p^2 (the preconditioner and
  // the momentum of its result, for the fused first turn of a preconditioned Arnoldi
  // step).  dst2 is the wave's own region of the other buffer.
  template <int TP, bool SWIN>
  static __device__ __forceinline__ void wfused2(const GQD_L cplx* src, GQD_L cplx* dst, GQD_L cplx* dst2,
                                                 const Ctx& c, int slab0, double ktau) {
    constexpr int NR = M / RF;
    constexpr int NB = SPW * NR;
    static_assert(NB % 64 == 0, "whole butterflies per lane");
    constexpr int PER = NB / 64;
    cplx x[PER][RF], z[PER][RF];
    {
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int b = l + 64 * q, e = b / NR, j = b % NR;
#pragma unroll
        for (int r = 0; r < RF; ++r) {
          const int i = e * M + j + r * NR;
          x[q][r] = src[SWIN ? swz(i) : i];
        }
      }
    }
    {
      const GQD_G cplx* tw = opaque(c.tw) + pass_table_offset(PLAN, TP);
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = (l + 64 * q) % NR;
#pragma unroll
        for (int r = 1; r < RF; ++r) x[q][r] = cmul(x[q][r], tw[j * (RF - 1) + r - 1]);
      }
    }
    const double scale = opaque_d(c.pscale) / (double)N;
    {
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int b = l + 64 * q, e = b / NR, j = b % NR;
        const int k1 = (slab0 + e) % R0;
        DFT<RF, -1>::run(x[q]);
#pragma unroll
        for (int r = 0; r < RF; ++r) {
          const int kk = k1 + R0 * (j + r * NR);          // k-space index
          const int kp = (kk < N / 2) ? kk : kk - N;      // signed wavenumber
          // (1 + i ktau p^2)^-1 / N = (1 - i q) / (N (1 + q^2)), q = ktau p^2; times p
          const double pk = scale * (double)N * (double)kp;
          const double qk = ktau * pk * pk;
          const double inv = 1.0 / ((double)N * (1.0 + qk * qk));
          x[q][r] = mk((x[q][r].x + qk * x[q][r].y) * inv, (x[q][r].y - qk * x[q][r].x) * inv);
          z[q][r] = cscale(x[q][r], pk);
        }
        DFT<RF, +1>::run(x[q]);
        DFT<RF, +1>::run(z[q]);
      }
    }
    {
      const int l = lane_tid() & 63;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int b = l + 64 * q, e = b / NR, j = b % NR;
#pragma unroll
        for (int r = 0; r < RF; ++r) {
          dst[swz(e * M + j * RF + r)] = x[q][r];
          dst2[swz(e * M + j * RF + r)] = z[q][r];
        }
      }
    }
  }
  // uz = M^-1 x and upz = p M^-1 x, M = 1 + i ktau p^2, from one forward transform
  // (four-step, two-buffer plans): the forward exchange goes through b0 and the slab
  // passes run in b1 as in kinetic_fs; the fused pass leaves M^-1 X in b1 and p M^-1 X in
  // the wave's region of b0, the inverse passes run on both, and both return through
  // the exchange.  x is read before uz or upz is written, so either may alias it.
  static __device__ void kinetic_fs_mz(const OV& x, OV& uz, OV& upz, const Ctx& c, double ktau) {
    static_assert(kFS && kPP, "two results need the two-buffer four-step form");
    GQD_L cplx* b0 = c.fft;
    GQD_L cplx* b1 = c.fft + 2 * N;
    cplx wo[R0 - 1];
    {
      const GQD_G cplx* tk = opaque(c.tw) + pass_table_offset(PLAN, 0) + lane_tid() * (R0 - 1);
#pragma unroll
      for (int k1 = 1; k1 < R0; ++k1) wo[k1 - 1] = tk[k1 - 1];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      cplx y[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) y[r] = x.v[s][r];
      DFT<R0, -1>::run(y);
#pragma unroll
      for (int k1 = 1; k1 < R0; ++k1) y[k1] = cmul(y[k1], wo[k1 - 1]);
      const int t = lane_tid();
#pragma unroll
      for (int k1 = 0; k1 < R0; ++k1) b0[(s * R0 + k1) * M + t] = y[k1];
    }
    __syncthreads();
    const int slab0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * SPW;
    GQD_L cplx* X = b0 + slab0 * M;
    GQD_L cplx* Y = b1 + slab0 * M;
    if constexpr (R3 == 1) {
      wpass<R1, 1, -1, -1, false, true, false>(X, Y, c, slab0);
      wave_sync();
      wfused2<1, true>(Y, Y, X, c, slab0, ktau);
      wave_sync();
      wpass<R1, R2, +1, 2, true, false, true>(Y, Y, c, slab0);
      wpass<R1, R2, +1, 2, true, false, true>(X, X, c, slab0);
    } else {
      wpass<R1, 1, -1, -1, false, true, false>(X, Y, c, slab0);
      wave_sync();
      wpass<R2, R1, -1, 1, true, false, false>(Y, Y, c, slab0);
      wave_sync();
      wfused2<2, false>(Y, Y, X, c, slab0, ktau);
      wave_sync();
      wpass<R2, R3, +1, 3, true, false, false>(Y, Y, c, slab0);
      wpass<R2, R3, +1, 3, true, false, false>(X, X, c, slab0);
      wave_sync();
      wpass<R1, R3 * R2, +1, 4, false, false, true>(Y, Y, c, slab0);
      wpass<R1, R3 * R2, +1, 4, false, false, true>(X, X, c, slab0);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      cplx y[R0], w[R0];
      const int t = lane_tid();
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        y[q] = b1[(s * R0 + q) * M + t];
        w[q] = b0[(s * R0 + q) * M + t];
      }
      DFT<R0, +1>::run(y);
      DFT<R0, +1>::run(w);
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        uz.v[s][r] = y[r];
        upz.v[s][r] = w[r];
      }
    }
    __syncthreads();  // b0 was read above; the next application's exchange writes it
  }

  template <int KM = 0>
  static __device__ void kinetic_fs(const OV& x, OV& u, const Ctx& c, double ktau) {
    GQD_L cplx* b0 = c.fft;                          // forward exchange
    GQD_L cplx* b1 = kPP ? c.fft + 2 * N : c.fft;    // slab work and the way back
    // inner radix-R0 DFT on owned points, outer twiddle w_N^(t k1) (the same for both
    // surfaces, loaded once), exchange
    cplx wo[R0 - 1];
    {
      const GQD_G cplx* tk = opaque(c.tw) + pass_table_offset(PLAN, 0) + lane_tid() * (R0 - 1);
#pragma unroll
      for (int k1 = 1; k1 < R0; ++k1) wo[k1 - 1] = tk[k1 - 1];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      cplx y[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) y[r] = x.v[s][r];
      DFT<R0, -1>::run(y);
#pragma unroll
      for (int k1 = 1; k1 < R0; ++k1) y[k1] = cmul(y[k1], wo[k1 - 1]);
      const int t = lane_tid();
#pragma unroll
      for (int k1 = 0; k1 < R0; ++k1) b0[(s * R0 + k1) * M + t] = y[k1];
    }
    __syncthreads();
    const int slab0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * SPW;
    const GQD_L cplx* X = b0 + slab0 * M;
    GQD_L cplx* Y = b1 + slab0 * M;
    if constexpr (R3 == 1) {
      wpass<R1, 1, -1, -1, false, true, false>(X, Y, c, slab0);
      wave_sync();
      wfused<KM, 1, true>(Y, Y, c, slab0, ktau);
      wave_sync();
      wpass<R1, R2, +1, 2, true, false, true>(Y, Y, c, slab0);
    } else {
      wpass<R1, 1, -1, -1, false, true, false>(X, Y, c, slab0);
      wave_sync();
      wpass<R2, R1, -1, 1, true, false, false>(Y, Y, c, slab0);
      wave_sync();
      wfused<KM, 2, false>(Y, Y, c, slab0, ktau);
      wave_sync();
      wpass<R2, R3, +1, 3, true, false, false>(Y, Y, c, slab0);
      wave_sync();
      wpass<R1, R3 * R2, +1, 4, false, false, true>(Y, Y, c, slab0);
    }
    __syncthreads();
    // inverse radix-R0 DFT over k1 back to owned points
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      cplx y[R0];
      const int t = lane_tid();
#pragma unroll
      for (int q = 0; q < R0; ++q) y[q] = b1[(s * R0 + q) * M + t];
      DFT<R0, +1>::run(y);
#pragma unroll
      for (int r = 0; r < R0; ++r) u.v[s][r] = y[r];
    }
    if constexpr (!kPP) __syncthreads();  // the next application's exchange reuses b0
  }

  // u = p x on both surfaces (forward DFT, multiply by p_k, inverse DFT / N); with
  // KM = 1, u = exp(-i ktau p^2) x instead (the kinetic factor of a split-operator step),
  // with KM = 2, u = (1 + i ktau p^2)^-1 x (the GMRES preconditioner).
  template <int KM = 0>
  static __device__ void kinetic(const OV& x, OV& u, const Ctx& c, double ktau = 0.0) {
    if constexpr (kFS) {
      kinetic_fs<KM>(x, u, c, ktau);
    } else {
      kinetic_sh<KM>(x, u, c, ktau);
    }
  }

  // Stockham form: every pass over the whole transform, one barrier each
  template <int KM = 0>
  static __device__ void kinetic_sh(const OV& x, OV& u, const Ctx& c, double ktau = 0.0) {
    GQD_L cplx* b0 = c.fft;
    GQD_L cplx* b1 = kPP ? c.fft + 2 * N : c.fft;
    constexpr int PL = (R3 == 1) ? 3 : 5;  // table index of the last pass
    TwS<R1, R0> t0;
    // pass A: radix R0, Ns = 1, from owned registers (butterfly j = thread)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      cplx y[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) y[r] = x.v[s][r];
      DFT<R0, -1>::run(y);
#pragma unroll
      for (int r = 0; r < R0; ++r) b0[s * N + swz(lane_tid() * R0 + r)] = y[r];
    }
    tw_load<R1, R0, 0>(t0, opaque(c.tw));
    __syncthreads();
    TwS<R0, T> tl;
    if constexpr (R3 == 1) {
      TwS<RF, N / RF> tf;
      TwS<R1, R2> t2;
      pass<R1, R0, -1, true>(b0, b1, t0, [&] { tw_load<RF, N / RF, 1>(tf, opaque(c.tw)); });
      fused_kspace<KM>(b1, b0, tf, c, [&] { tw_load<R1, R2, 2>(t2, opaque(c.tw)); }, ktau);
      pass<R1, R2, +1, true>(b0, b1, t2, [&] { tw_load<R0, T, PL>(tl, opaque(c.tw)); });
    } else {
      TwS<R2, R0 * R1> t1;
      TwS<RF, N / RF> tf;
      TwS<R2, R3> t3;
      TwS<R1, R3 * R2> t4;
      pass<R1, R0, -1, true>(b0, b1, t0, [&] { tw_load<R2, R0 * R1, 1>(t1, opaque(c.tw)); });
      pass<R2, R0 * R1, -1>(b1, b0, t1, [&] { tw_load<RF, N / RF, 2>(tf, opaque(c.tw)); });
      fused_kspace<KM>(b0, b1, tf, c, [&] { tw_load<R2, R3, 3>(t3, opaque(c.tw)); }, ktau);
      pass<R2, R3, +1, true>(b1, b0, t3, [&] { tw_load<R1, R3 * R2, 4>(t4, opaque(c.tw)); });
      pass<R1, R3 * R2, +1>(b0, b1, t4, [&] { tw_load<R0, T, PL>(tl, opaque(c.tw)); });
    }
    // last inverse pass: radix R0, Ns = T, butterfly j = thread -> owned points
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      cplx y[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) y[r] = b1[s * N + pt(r)];
#pragma unroll
      for (int r = 1; r < R0; ++r) y[r] = twmul<+1>(y[r], tl.w[0][r - 1]);
      DFT<R0, +1>::run(y);
#pragma unroll
      for (int r = 0; r < R0; ++r) u.v[s][r] = y[r];
    }
    // in place, the buffer is reused by the next pass A; with two buffers the next
    // writer of b1 comes after a barrier
    if constexpr (!kPP) __syncthreads();
  }

  // y = [p - i F] x for x at xg (F12 couples surface 2 into surface 1, F21 = -F12).
  // The input is re-read at owned points after the transform.
  static __device__ void apply_A(const cplx* xg, OV& y, const Ctx& c) {
    {
      OV t;
      load(t, xg);
      kinetic(t, y, c);
    }
    const GQD_G double* F = opaque(c.F);
    const GQD_G cplx* xq = opaque(xg);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const double f = F[pt(r)];
      const cplx x0 = xq[pt(r)], x1 = xq[N + pt(r)];
      // -i f x2 added to surface 1, +i f x1 added to surface 2
      y.v[0][r] = cadd(y.v[0][r], cmul_is(x1, -f));
      y.v[1][r] = cadd(y.v[1][r], cmul_is(x0, f));
    }
  }

  // y <- y / (2m) + V x: completes H x = A (A x) / (2m) + V x after the second A pass.
  static __device__ __forceinline__ void finish_H(OV& y, const cplx* xg, const Ctx& c) {
    const GQD_G double* V = opaque(c.V);
    const GQD_G cplx* xq = opaque(xg);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int r = 0; r < R0; ++r)
        y.v[s][r] = cadd(cscale(y.v[s][r], c.inv2m), cscale(xq[s * N + pt(r)], V[s * N + pt(r)]));
  }

  // y <- exp(-i W tau) y on owned points for the diabatic matrix W = [[W11, W12],
  // [W12, W22]] held as V = (W11, W22), F = W12: with W = wbar 1 + dz sz + W12 sx and
  // r = (dz^2 + W12^2)^(1/2), exp(-i W tau) = exp(-i wbar tau) [cos(r tau) 1
  // - i sin(r tau) / r (dz sz + W12 sx)].
  static __device__ __forceinline__ void expW(OV& y, double tau, const Ctx& c) {
    const GQD_G double* V = opaque(c.V);
    const GQD_G double* F = opaque(c.F);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const double w11 = V[pt(r)], w22 = V[N + pt(r)], w12 = F[pt(r)];
      const double wbar = 0.5 * (w11 + w22), dz = 0.5 * (w11 - w22);
      const double rr = sqrt(dz * dz + w12 * w12);
      double sr, cr, sb, cb;
      sincos(rr * tau, &sr, &cr);
      sincos(-wbar * tau, &sb, &cb);
      const double sinc = rr > 0.0 ? sr / rr : tau;
      const cplx a = mk(cr, -sinc * dz), d = mk(cr, sinc * dz), b = mk(0.0, -sinc * w12);
      const cplx y0 = y.v[0][r], y1 = y.v[1][r];
      const cplx phase = mk(cb, sb);
      y.v[0][r] = cmul(phase, cadd(cmul(a, y0), cmul(b, y1)));
      y.v[1][r] = cmul(phase, cadd(cmul(b, y0), cmul(d, y1)));
    }
  }

  // y += -i F x on owned points (x read from a global vector)
  template <class P>
  static __device__ __forceinline__ void couple(OV& y, P xs, const Ctx& c) {
    const GQD_G double* F = opaque(c.F);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const double f = F[pt(r)];
      const cplx x0 = xs[pt(r)], x1 = xs[N + pt(r)];
      y.v[0][r] = cadd(y.v[0][r], cmul_is(x1, -f));
      y.v[1][r] = cadd(y.v[1][r], cmul_is(x0, f));
    }
  }

  // pre = (-i F chi) / (2m) + (V - shift) x written to dst (global), x read from xs;
  // the outer A's coupling and the potential, formed before the second transform.
  template <class P, class Q>
  static __device__ __forceinline__ void make_pre(const OV& chi, P xs, Q dst, double shift, const Ctx& c) {
    const GQD_G double* F = opaque(c.F);
    const GQD_G double* V = opaque(c.V);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const double f = F[pt(r)];
      const double v0 = V[pt(r)] - shift, v1 = V[N + pt(r)] - shift;
      const cplx x0 = xs[pt(r)], x1 = xs[N + pt(r)];
      const cplx p0 = cadd(cscale(cmul_is(chi.v[1][r], -f), c.inv2m), cscale(x0, v0));
      const cplx p1 = cadd(cscale(cmul_is(chi.v[0][r], f), c.inv2m), cscale(x1, v1));
      dst[pt(r)] = p0;
      dst[N + pt(r)] = p1;
    }
  }

  // register forms: x (then pre) held at owned points
  static __device__ __forceinline__ void couple(OV& y, const OV& x, const Ctx& c) {
    const GQD_G double* F = opaque(c.F);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const double f = F[pt(r)];
      y.v[0][r] = cadd(y.v[0][r], cmul_is(x.v[1][r], -f));
      y.v[1][r] = cadd(y.v[1][r], cmul_is(x.v[0][r], f));
    }
  }
  static __device__ __forceinline__ void make_pre(const OV& chi, OV& xp, double shift, const Ctx& c) {
    const GQD_G double* F = opaque(c.F);
    const GQD_G double* V = opaque(c.V);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const double f = F[pt(r)];
      const double v0 = V[pt(r)] - shift, v1 = V[N + pt(r)] - shift;
      const cplx p0 = cadd(cscale(cmul_is(chi.v[1][r], -f), c.inv2m), cscale(xp.v[0][r], v0));
      const cplx p1 = cadd(cscale(cmul_is(chi.v[0][r], f), c.inv2m), cscale(xp.v[1][r], v1));
      xp.v[0][r] = p0;
      xp.v[1][r] = p1;
    }
  }
  static __device__ __forceinline__ void add_pre(OV& y, const OV& pre, const Ctx& c) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int r = 0; r < R0; ++r) y.v[s][r] = cadd(cscale(y.v[s][r], c.inv2m), pre.v[s][r]);
  }

  // y <- y / (2m) + pre
  template <class P>
  static __device__ __forceinline__ void add_pre(OV& y, P pre, const Ctx& c) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int r = 0; r < R0; ++r) y.v[s][r] = cadd(cscale(y.v[s][r], c.inv2m), pre[s * N + pt(r)]);
  }

  // --------------------------------------------------------------------- GMRES
  static __device__ void givens_update(int j, double hn, const Ctx& c) { gm_givens(j, hn, c); }
  static __device__ void back_solve(int k, const Ctx& c) { gm_back_solve(k, c); }

  // |g_(j+1)| that givens_update would leave for the column hcol + dj e_j and the
  // subdiagonal hn, in the same arithmetic, writing nothing (thread 0's value counts)
  static __device__ double givens_probe(int j, double hn, cplx dj, const Ctx& c) {
    const GQD_L cplx* h = c.hcol;
    cplx a = j == 0 ? cadd(h[0], dj) : h[0];
    for (int i = 0; i < j; ++i) {
      const double ci = c.cs[i];
      const cplx si = c.sn[i];
      const cplx hi1 = i + 1 == j ? cadd(h[j], dj) : h[i + 1];
      a = cadd(cmul(cneg(mk(si.x, -si.y)), a), cscale(hi1, ci));
    }
    cplx sj;
    if (hn == 0.0) {
      sj = mk(0.0, 0.0);
    } else if (a.x == 0.0 && a.y == 0.0) {
      sj = mk(1.0, 0.0);
    } else {
      const double absa = hypot(a.x, a.y);
      const double rho = sqrt(absa * absa + hn * hn);
      sj = cscale(mk(a.x / absa, a.y / absa), hn / rho);
    }
    const cplx g1 = cmul(cneg(mk(sj.x, -sj.y)), c.g[j]);
    return hypot(g1.x, g1.y);
  }
};

// composition fraction tau_c: product of one gamma per level, innermost level first
// (the flattened list of Sec. II.D with gamma_1 applied first)
// substep fractions of the non-recursive compositions (gqd_compositions.h)
static __constant__ double kFlatTau[kFlatTauLen] = {GQD_FLAT_TAU_VALUES};

__device__ __forceinline__ double substep_tau(int c, const GammaTab& gt) {
  if (gt.flat) return kFlatTau[gt.flat - 1 + c];
  double t = 1.0;
  int cc = c;
  const int mid = gt.arity / 2;
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) {
    if (l < gt.levels) {
      const int d = cc % gt.arity;
      cc /= gt.arity;
      t = (d == mid ? gt.mid[l] : gt.side[l]) * t;
    }
  }
  return t;
}

// ------------------------------------------------------------------------ kernels

// Program counter values of the propagation machine (see k_run).
enum Pc {
  kSubstep,       // start the next substep (or finish)
  kSolveGuess,    // have H b: form x0 = (1 - i al H) b, ask for H x0
  kSolveResid,    // have H x: true residual, restart or finish the solve
  kSolveArnoldi,  // have (H - s) v_j: Arnoldi step j
  kMidpAfter,     // midpoint: x solved
  kMidpExplicit,  // midpoint, literal: have H x
  kTrapHpsi,      // trapezoid: have H psi
  kTrapAfter,     // trapezoid: psi' solved
  kAdjAfterPhi,   // adjoint: phi solved
  kAdjAfterMu,    // adjoint: mu solved
  kAdjAphi,       // adjoint: have A phi
  kAdjAmu,        // adjoint: have A mu
  kExplAfter,     // explicit Euler: have H psi
  kImplAfter,     // implicit Euler: x solved
  kSodStart,      // second-order differencing: have H psi(0)
  kSodStart2,     // second-order differencing: have H H psi(0)
  kSodStep,       // second-order differencing: have H psi(t)
  kPrecZ,         // preconditioned GMRES: have z_j = M^-1 v_j, ask for H z_j
  kPrecArnoldi,   // preconditioned GMRES: have H z_j: Arnoldi step j on X M^-1
  kPrecUpdate     // preconditioned GMRES: have M^-1 V y: x += it
};

// Whole-call propagation (mode 0) or reverse sweep (mode 1) of one item per workgroup.
//
// The kernel is a small machine around a single operator application so that the
// Fourier-transform code exists once: each loop turn applies A = p - iF to a global
// vector (H takes two turns, the inner A x kept in registers between them), then the current
// program counter consumes the result and requests the next application.
//
// Propagation, per substep of length h = tau_c dt, alpha = h/2 (Sec. II.C-D):
//   midpoint (Eq. 19):  x = (1 + i alpha H)^-1 psi;  psi' = (1 - i alpha H) x, or 2x - psi
//   trapezoid (Eq. 18): b = (1 - i alpha H) psi;     psi' = (1 + i alpha H)^-1 b
// Each inverse is restarted GMRES(m) from x0 = (1 - i alpha H) b, with the Arnoldi
// basis built from H - s, s a real shift near the Rayleigh quotient of the first basis
// vector (classical Gram-Schmidt, a second pass on cancellation) and
// Givens rotations on the Hessenberg matrix of 1 + i alpha H; it stops when the
// residual estimate is <= tol ||b||.
//
// Reverse sweep, substeps in reverse order: phi = (1 - i alpha H)^-1 psi,
// mu = (1 - i alpha H)^-1 lambda, psi <- 2 phi - psi, lambda <- 2 mu - lambda,
// gF += -(2 alpha / m) Re[conj(mu1)(A phi)2 - conj(mu2)(A phi)1 + conj(A mu)1 phi2 - conj(A mu)2 phi1].
// PC: the solves are right-preconditioned (a separate instantiation, so that the plain
// solver's register allocation does not carry the preconditioned states)
template <int P, bool PC = false>
__global__ void __launch_bounds__(Eng<P>::T) __attribute__((amdgpu_waves_per_eu(Eng<P>::WPE))) k_run(KArgs a) {
  using E = Eng<P>;
  constexpr int N = E::N;
  using OV = typename E::OV;
  constexpr int R0 = E::R0;
  constexpr int T = E::T;
  if ((int)blockIdx.x >= a.nlist) return;
  extern __shared__ double2 smem_raw[];
  GQD_L cplx* smem = (GQD_L cplx*)smem_raw;
  const int item = a.list[blockIdx.x];
  const ItemMeta im = a.items[item];
  const int m = a.sc.m;
  cplx* work = (cplx*)a.work + im.off * (long long)(m + kWorkExtra);
  const auto c = E::make_ctx(smem, m, a, im);
  cplx* psi = (cplx*)a.psi + im.off;
  cplx* lam = (cplx*)a.aux + im.off;
  cplx* basis = work;
  cplx* S0 = work + (size_t)(m + 1) * E::VEC;  // X (solve output)  | PHI
  cplx* S1 = S0 + E::VEC;                       // B (rhs, H x)      | MU
  cplx* S2 = S1 + E::VEC;                       // HPSI              | A phi
  cplx* S3 = S2 + E::VEC;                       //                   | (spare: A mu stays in registers)
  cplx* CHI = S3 + E::VEC;                      // inner A x of an H application
  const bool adj = a.mode == 1;
  const bool midp = a.method == kMidp;
  const double dt = a.dt_item ? uniform_d(a.dt_item[item]) : a.dt;
  const long long nsteps = a.nsteps_item ? a.nsteps_item[item] : a.nsteps;
  const bool literal = a.sc.literal != 0;

  long long napply = 0, iters_total = 0, iters_sq = 0, extra_vecs = 0;
  int solves = 0, max_iters = 0, failures = 0;
  bool bad = false;
  bool have_hpsi = a.hpsi_valid != 0;

  long long n = 0;
  int cc = adj ? a.gt.count - 1 : 0;
  double alpha = 0.0;  // half the substep (geometric methods), the whole step (elementary)
  bool sod_started = false;

  // operator request: H - opshift applied to opsrc (opshift = 0 outside Arnoldi), or
  // (opK) the preconditioner (1 + i ktau p^2)^-1, one transform pair, no coupling
  bool pending = false, opH = false, op_in_y = false, opK = false, opKH = false;
  double opktau = 0.0;
  bool prec_cv = false;  // preconditioned cycle: converged by the estimate
  bool psi_in_y = false;  // y holds psi at owned points (set by the midpoint update)
  int half = 0;
  const cplx* opsrc = nullptr;
  double opshift = 0.0;
  // Arnoldi runs on H - s, s the Rayleigh quotient of the first basis vector of the
  // previous solve of the same kind (sig0: psi or phi, sig1: the adjoint's mu)
  double sig0 = 0.0, sig1 = 0.0;
  // preconditioned solves run Arnoldi on X M^-1 - (1 + i al e), e = (h_00 - 1) / (i al)
  // taken from the first column of the previous solve of the same kind
  cplx pe0 = mk(0.0, 0.0), pe1 = mk(0.0, 0.0);
  bool kind_mu = false;
  // solve state
  const cplx* bg = nullptr;
  cplx* xg = nullptr;
  double al = 0.0, tolb = 0.0;
  // thread 0 alone keeps the largest true relative residual a solve ended on, as a
  // numerator/denominator pair (tol |r|, tol |b|; divided once at the end), in LDS:
  // no register is held through the loop
  GQD_L double* const max_resid = c.scal + 11;
  if (threadIdx.x == 0) {
    max_resid[0] = 0.0;
    max_resid[1] = 1.0;
  }
  int j = 0, iters = 0, after = kSubstep;

  int pc = kSubstep;
  OV y, keep;

  // in_y: the operand was just stored from y, which still holds it at owned points
  auto request = [&](const cplx* src, bool h, double shift = 0.0, bool in_y = false) {
    pending = true;
    opsrc = src;
    opH = h;
    opshift = shift;
    op_in_y = in_y;
    opK = false;
    opKH = false;
    half = 0;
  };
  // H M^-1 on y (two-buffer four-step plans): the first turn makes z = M^-1 y (stored to
  // S3) and A z from one forward transform, the second turn A A z as usual
  auto request_prec_h = [&]() {
    request(nullptr, true, 0.0, true);
    opKH = true;
    opktau = al * a.inv2m;
  };
  // the preconditioner M^-1 = (1 + i al p^2 / 2m)^-1 of the current solve on y
  auto request_prec = [&]() {
    pending = true;
    opsrc = nullptr;
    opH = false;
    opshift = 0.0;
    op_in_y = true;
    opK = true;
    opKH = false;
    opktau = al * a.inv2m;
    half = 0;
  };
  // start a solve of (1 + i al H) x = b: ||b||, then ask for H b.  b_in_y: y holds b
  // (the midpoint's new state, just stored), so neither needs to read it back.
  auto solve_begin = [&](const cplx* b, cplx* x, double alv, int ret, bool b_in_y = false) {
    bg = b;
    xg = x;
    al = alv;
    after = ret;
    kind_mu = ret == kAdjAfterMu;
    iters = 0;
    OV t;
    if (b_in_y) {
      t = y;
    } else {
      E::load(t, b);
    }
    const double bnorm = sqrt(E::block_sum1(E::norm2(t), c));
    if (!isfinite(bnorm)) bad = true;
    tolb = a.sc.tol * bnorm;
    request(b, true, 0.0, b_in_y);
    pc = kSolveGuess;
  };
  auto solve_end = [&](bool conv) {
    if (threadIdx.x == 0) log_solve(a.stats ? a.stats + item : nullptr, solves, iters);
    ++solves;
    iters_total += iters;
    iters_sq += (long long)iters * iters;
    if (iters > max_iters) max_iters = iters;
    if (!conv) ++failures;
    pc = after;
  };
  auto advance = [&]() {
    if (adj) {
      if (--cc < 0) {
        cc = a.gt.count - 1;
        ++n;
      }
    } else if (++cc == a.gt.count) {
      cc = 0;
      ++n;
    }
    pc = kSubstep;
  };

  for (;;) {
    if (bad) break;
    if constexpr (PC) {
      if (pending && opK) {
        // (the transform reads all of its input before it writes any of its output)
        E::template kinetic<2>(y, y, c, opktau);
        pending = false;
      }
    }
    if (pending) {
      // one transform per turn: turn 1 takes the input from opsrc, turn 2 (H only) takes
      // chi = A x from registers; x and then the partial result are kept in registers
      // (two-buffer mode) or read from opsrc / parked in the CHI slot (larger N)
      OV t;
      if (half == 0) {
        if (op_in_y) {
          t = y;
        } else {
          E::load(t, opsrc);
        }
        if constexpr (E::kPP) keep = t;
      } else {
        t = y;
      }
      if constexpr (PC && E::kFS && E::kPP) {
        if (half == 0 && opKH) {
          // preconditioned Arnoldi step: z = M^-1 v and p z from one forward transform;
          // z becomes the operand of H (kept for the second turn and in S3 for w)
          E::kinetic_fs_mz(t, keep, y, c, opktau);
          E::store(keep, S3);
        } else {
          E::kinetic(t, y, c);
        }
      } else {
        E::kinetic(t, y, c);
      }
      if (half == 0) {
        if constexpr (E::kPP) {
          E::couple(y, keep, c);
          if (opH) E::make_pre(y, keep, opshift, c);
        } else {
          E::couple(y, opaque(opsrc), c);
          if (opH) E::make_pre(y, opaque(opsrc), opaque(CHI), opshift, c);
        }
        if (opH) {
          half = 1;
          continue;
        }
      } else {
        if constexpr (E::kPP) {
          E::add_pre(y, keep, c);
        } else {
          E::add_pre(y, opaque(CHI), c);
        }
        ++napply;
      }
      pending = false;
    }
    switch (pc) {
      case kSubstep: {
        if (n >= nsteps) goto done;
        if (a.method >= kEulerExpl) {  // elementary methods: whole steps, tau = 1
          alpha = substep_tau(cc, a.gt) * dt;
          if (a.method == kEulerImpl) {
            solve_begin(psi, S0, alpha, kImplAfter);
          } else {
            request(psi, true, 0.0, psi_in_y);
            psi_in_y = false;
            pc = a.method == kEulerExpl ? kExplAfter : (sod_started ? kSodStep : kSodStart);
          }
          break;
        }
        alpha = 0.5 * (substep_tau(cc, a.gt) * dt);
        if (adj) {
          solve_begin(psi, S0, -alpha, kAdjAfterPhi);
        } else if (midp) {
          solve_begin(psi, S0, alpha, kMidpAfter, psi_in_y);
          psi_in_y = false;
        } else if (literal || !have_hpsi) {
          request(psi, true);
          pc = kTrapHpsi;
        } else {
          pc = kTrapHpsi;  // H psi already in S2
        }
        break;
      }
      case kTrapHpsi: {
        OV p, q;
        if (literal || !have_hpsi) {
          E::store(y, S2);
          q = y;
        } else {
          E::load(q, S2);
        }
        E::load(p, psi);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) p.v[s][r] = csub(p.v[s][r], cmul_is(q.v[s][r], alpha));
        E::store(p, S1);  // b = (1 - i alpha H) psi
        solve_begin(S1, psi, alpha, kTrapAfter);
        break;
      }
      case kTrapAfter: {
        if (!literal) {
          // H psi' = (b - psi') / (i alpha), reused by the next substep's explicit half
          OV p, q;
          E::load(p, S1);
          E::load(q, psi);
#pragma unroll
          for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              const cplx d = csub(p.v[s][r], q.v[s][r]);
              q.v[s][r] = mk(d.y / alpha, -d.x / alpha);
            }
          E::store(q, S2);
          have_hpsi = true;
        }
        advance();
        break;
      }
      case kMidpAfter: {
        if (literal) {
          request(S0, true);
          pc = kMidpExplicit;
          break;
        }
        OV q;  // psi' = 2x - psi, left in y for the next substep's solve
        E::load(q, S0);
        E::load(y, psi);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) y.v[s][r] = csub(cscale(q.v[s][r], 2.0), y.v[s][r]);
        E::store(y, psi);
        psi_in_y = true;
        advance();
        break;
      }
      case kMidpExplicit: {
        OV q;  // psi' = x - i alpha H x
        E::load(q, S0);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) q.v[s][r] = csub(q.v[s][r], cmul_is(y.v[s][r], alpha));
        E::store(q, psi);
        advance();
        break;
      }
      case kSolveGuess: {
        OV t;
        E::load(t, bg);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) y.v[s][r] = csub(t.v[s][r], cmul_is(y.v[s][r], al));
        E::store(y, xg);  // x0 = (1 - i al H) b
        request(xg, true, 0.0, true);
        pc = kSolveResid;
        break;
      }
      case kSolveResid: {
        OV t;
        E::load(t, xg);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) y.v[s][r] = cadd(t.v[s][r], cmul_is(y.v[s][r], al));
        E::load(t, bg);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) y.v[s][r] = csub(t.v[s][r], y.v[s][r]);  // r = b - X x
        const double beta = sqrt(E::block_sum1(E::norm2(y), c));
        if (!isfinite(beta)) {
          bad = true;
          break;
        }
        if (beta <= tolb) {
          if (threadIdx.x == 0 && tolb > 0.0 && a.sc.tol * beta * max_resid[1] > max_resid[0] * tolb) {
            max_resid[0] = a.sc.tol * beta;
            max_resid[1] = tolb;
          }
          solve_end(true);
          break;
        }
        if (iters >= a.sc.maxit) {
          solve_end(false);
          break;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) y.v[s][r] = mk(y.v[s][r].x / beta, y.v[s][r].y / beta);
        E::store(y, basis);
        if (threadIdx.x == 0) c.g[0] = mk(beta, 0.0);
        // (the next block reduction's barrier orders this write before any read)
        j = 0;
        if constexpr (PC) {
          if constexpr (E::kFS && E::kPP) {
            request_prec_h();
            pc = kPrecArnoldi;
          } else {
            request_prec();
            pc = kPrecZ;
          }
          break;
        }
        request(basis, true, kind_mu ? sig1 : sig0, true);
        pc = kSolveArnoldi;
        break;
      }
      case kPrecZ: {
        if constexpr (PC) {
          // z_j = M^-1 v_j in y: kept in S3 for w = X z_j, then H z_j
          E::store(y, S3);
          request(S3, true, 0.0, true);
          pc = kPrecArnoldi;
          break;
        }
        break;
      }
      case kPrecArnoldi: {
        if constexpr (PC) {
          // Arnoldi step j on X M^-1 (right preconditioning), shifted by s = 1 + i al e:
          // w = z_j + i al H z_j - s v_j, one classical Gram-Schmidt pass over v_0..v_j
          // with |w|^2 from the same reduction (its last turn parked in the stash for the
          // update), a second pass when the first keeps less than kReorthRatioPrec of
          // |w|^2.  X M^-1 = 1 + i al (H - T) M^-1 has no Hermitian structure to exploit.
          // Unshifted, w lies mostly along v_j (the identity and the potential's mean),
          // the pass cancels most of |w|^2 and the second pass runs on nearly every step;
          // with e the Rayleigh energy of the previous solve of the same kind the pass
          // keeps 25-55 % of |w|^2.  The shift changes the Krylov space of no step; the
          // column of X M^-1 gains s on its diagonal below.
          ++iters;
          const cplx pe = kind_mu ? pe1 : pe0;
          const cplx sft = mk(1.0 - al * pe.y, al * pe.x);
          {
            OV z, v;
            E::load(z, S3);
            E::load(v, basis + (size_t)j * E::VEC);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
              for (int r = 0; r < R0; ++r)
                y.v[s][r] = csub(cadd(z.v[s][r], cmul_is(y.v[s][r], al)), cmul(sft, v.v[s][r]));
          }
          extra_vecs += 1;  // v_j read again for the shift
          E::template block_dots<E::kStashFill>(basis, y, j + 1, c, c.hcol, true);
          const double w2 = uniform_d(c.hcol[j + 1].x);
          double hn2 = w2;
          for (int i = 0; i <= j; ++i) hn2 -= cabs2(c.hcol[i]);
          hn2 = uniform_d(hn2);
          E::template block_axpy<true>(basis, c.hcol, j + 1, y, c);
          // The second pass only serves v_(j+1).  Where it is due, the step is most often
          // the cycle's last (the new direction is small against w as the residual
          // estimate reaches the tolerance), which the one-pass column decides as well:
          // the tolerance met, the restart length or maxit reached.  Those steps skip it.
          bool reorth = hn2 < kReorthRatioPrec * w2;
          if (reorth && hn2 > 0.0) {
            if (iters >= a.sc.maxit || j + 1 >= m) {
              reorth = false;
            } else {
              if (threadIdx.x == 0) c.scal[1] = E::givens_probe(j, sqrt(hn2), sft, c);
              __syncthreads();
              reorth = !(uniform_d(c.scal[1]) <= tolb);
            }
          }
          if (reorth) {
            extra_vecs += 2 * (j + 1);
            E::template block_dots<E::kStashUse>(basis, y, j + 1, c, c.y, true);
            double r2 = uniform_d(c.y[j + 1].x);
            for (int i = 0; i <= j; ++i) r2 -= cabs2(c.y[i]);
            hn2 = uniform_d(r2 > 0.0 ? r2 : 0.0);
            E::template block_axpy<true>(basis, c.y, j + 1, y, c);
            // every wave has read the pass's coefficients before the column gains them
            __syncthreads();
            for (int i = threadIdx.x; i <= j; i += T) c.hcol[i] = cadd(c.hcol[i], c.y[i]);
          }
          __syncthreads();
          // the same thread rotates the column next
          if (threadIdx.x == 0) c.hcol[j] = cadd(c.hcol[j], sft);
          const double hn = sqrt(hn2);
          E::givens_update(j, hn, c);
          if (j == 0 && al != 0.0) {  // h_00 is left in place by the first rotation
            const double h0x = uniform_d(c.hcol[0].x), h0y = uniform_d(c.hcol[0].y);
            const cplx e = mk(h0y / al, (1.0 - h0x) / al);  // (h_00 - 1) / (i al)
            if (kind_mu) pe1 = e; else pe0 = e;
          }
          const double gabs = uniform_d(c.scal[0]);
          if (!isfinite(hn) || !isfinite(gabs)) {
            bad = true;
            break;
          }
          const bool cv = gabs <= tolb;
          if (!cv && hn != 0.0 && iters < a.sc.maxit && j + 1 < m) {
            const double sc = 1.0 / hn;
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
              for (int r = 0; r < R0; ++r) y.v[s][r] = cscale(y.v[s][r], sc);
            ++j;
            E::store(y, basis + (size_t)j * E::VEC);
            if constexpr (E::kFS && E::kPP) {
              request_prec_h();
              pc = kPrecArnoldi;
            } else {
              request_prec();
              pc = kPrecZ;
            }
            break;
          }
          // cycle ends: x += M^-1 (V y) over the k = j + 1 basis vectors
          const int k = j + 1;
          E::back_solve(k, c);
#pragma unroll
          for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int r = 0; r < R0; ++r) y.v[s][r] = mk(0.0, 0.0);
          for (int i = 0; i < k; ++i) {
            OV v;
            E::load(v, basis + (size_t)i * E::VEC);
            const cplx yi = c.y[i];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
              for (int r = 0; r < R0; ++r) y.v[s][r] = cadd(y.v[s][r], cmul(yi, v.v[s][r]));
          }
          __syncthreads();  // c.y is read by all before it can be rewritten
          prec_cv = cv;
          request_prec();
          pc = kPrecUpdate;
          break;
        }
        break;
      }
      case kPrecUpdate: {
        if constexpr (PC) {
          {
            OV x;
            E::load(x, xg);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
              for (int r = 0; r < R0; ++r) x.v[s][r] = cadd(x.v[s][r], y.v[s][r]);
            E::store(x, xg);
          }
          if (prec_cv && !a.sc.verify) {
            solve_end(true);
          } else {  // verification, restart, or maxit / breakdown: the true residual decides
            request(xg, true);
            pc = kSolveResid;
          }
          break;
        }
        break;
      }
      case kSolveArnoldi: {
        // Arnoldi on H - s (the Krylov space of 1 + i al H is that of H - s for any real
        // shift s).  H - s is Hermitian, so w = (H - s) v_j lies, up to rounding, in the
        // span of v_j, v_(j-1) and the new direction: those two are projected out first
        // (their dot products in one reduction, the update from the stash that the same
        // sweep filled), then one classical Gram-Schmidt pass over v_0..v_j, with |w1|^2
        // from the same reduction, removes what rounding left along every basis vector.
        // That pass cancels little; another runs only when it keeps less than
        // kReorthRatio of |w1|^2.  (A full first pass would cancel more than half of
        // |w|^2 on most iterations once the Lanczos coefficients settle, and need the
        // second full pass every time.)
        // Column j of the Hessenberg matrix of X = 1 + i al H is delta_ij + i al (h_ij +
        // s delta_ij), and v_(j+1) = i sign(al) w'/|w'| makes its subdiagonal |al| |w'| real.
        ++iters;
        const double sh = opshift;
        const int k0 = j > 0 ? j - 1 : 0;
        const int K0 = j - k0 + 1;
        const cplx* b0 = basis + (size_t)k0 * E::VEC;
        E::template block_dots<E::kStashFill>(b0, y, K0, c, c.y, false);
        E::template block_axpy<true>(b0, c.y, K0, y, c);
        extra_vecs += K0;
        // |w2|^2 = |w1|^2 - sum |c_i|^2 when the pass keeps at least half of |w1|^2 (a
        // few ulp there); a further pass returns its own |w'|^2 from the same reduction
        E::template block_dots<E::kStashFill>(basis, y, j + 1, c, c.hcol, true);
        const double w2 = uniform_d(c.hcol[j + 1].x);
        double hn2 = w2;
        for (int i = 0; i <= j; ++i) hn2 -= cabs2(c.hcol[i]);
        hn2 = uniform_d(hn2);
        if (j == 0) {  // <v_0|H v_0>, the shift of the following columns and solves
          // (read here: the column is rewritten below, behind barriers)
          const double rq = uniform_d(c.hcol[0].x + c.y[0].x) + sh;
          if (kind_mu) sig1 = rq; else sig0 = rq;
        }
        E::template block_axpy<true>(basis, c.hcol, j + 1, y, c);
        // every wave has read the pass's coefficients before the column gains the
        // three-term ones, and the column is whole before anyone reads it below
        __syncthreads();
        if (threadIdx.x < K0) c.hcol[k0 + threadIdx.x] = cadd(c.hcol[k0 + threadIdx.x], c.y[threadIdx.x]);
        __syncthreads();
        if (hn2 < kReorthRatio * w2) {
          extra_vecs += 2 * (j + 1);
          E::template block_dots<E::kStashUse>(basis, y, j + 1, c, c.y, true);
          double r2 = uniform_d(c.y[j + 1].x);
          for (int i = 0; i <= j; ++i) r2 -= cabs2(c.y[i]);
          hn2 = uniform_d(r2 > 0.0 ? r2 : 0.0);
          E::template block_axpy<true>(basis, c.y, j + 1, y, c);
          for (int i = threadIdx.x; i <= j; i += T) c.hcol[i] = cadd(c.hcol[i], c.y[i]);
        }
        const double hn = sqrt(hn2);
        for (int i = threadIdx.x; i <= j; i += T) {
          if (i == j) {
            const cplx hx = cmul_is(mk(c.hcol[i].x + sh, c.hcol[i].y), al);  // i al (h_jj + s)
            c.hcol[i] = mk(1.0 + hx.x, hx.y);
          } else {
            c.hcol[i] = cmul_is(c.hcol[i], al);  // i al h_ij
          }
        }
        __syncthreads();
        E::givens_update(j, fabs(al) * hn, c);
        const double gabs = uniform_d(c.scal[0]);
        if (!isfinite(hn) || !isfinite(gabs)) {
          bad = true;
          break;
        }
        const bool cv = gabs <= tolb;
        if (!cv && hn != 0.0 && iters < a.sc.maxit && j + 1 < m) {
          const double sc = (al >= 0.0 ? 1.0 : -1.0) / hn;
#pragma unroll
          for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int r = 0; r < R0; ++r) y.v[s][r] = cmul_is(y.v[s][r], sc);
          ++j;
          E::store(y, basis + (size_t)j * E::VEC);
          request(basis + (size_t)j * E::VEC, true, kind_mu ? sig1 : sig0, true);
          break;
        }
        // cycle ends: x += V y over the k = j + 1 basis vectors
        const int k = j + 1;
        E::back_solve(k, c);
        {
          OV x;
          E::load(x, xg);
          // the last turn's vectors are still in the Gram-Schmidt stash (the last
          // Arnoldi step swept the same k); not on in-place plans, whose registers
          // are exhausted here
#pragma unroll 1
          for (int i = 0; i < k; i += E::GSV) {
            const bool two = E::GSV == 2 && i + 1 < k;
            const bool last = E::kStash && E::kPP && i + E::GSV >= k;
            const GQD_G cplx* Va = opaque(basis + (size_t)i * E::VEC);
            const GQD_G cplx* Vb = opaque(basis + (size_t)(two ? i + 1 : i) * E::VEC);
            const GQD_L cplx* Sa = c.fft;
            const GQD_L cplx* Sb = c.fft + (two ? 2 * N : 0);
            const cplx ya = c.y[i];
            const cplx yb = two ? c.y[i + 1] : mk(0.0, 0.0);
            constexpr int SB = E::SB;
#pragma unroll
            for (int s0 = 0; s0 < 2; s0 += SB) {
              cplx va[SB][R0], vb[SB][R0];
              if (last) {
#pragma unroll
                for (int s = 0; s < SB; ++s)
#pragma unroll
                  for (int r = 0; r < R0; ++r) {
                    va[s][r] = Sa[(s0 + s) * N + E::pt(r)];
                    if constexpr (E::GSV == 2) vb[s][r] = Sb[(s0 + s) * N + E::pt(r)];
                  }
              } else {
#pragma unroll
                for (int s = 0; s < SB; ++s)
#pragma unroll
                  for (int r = 0; r < R0; ++r) {
                    va[s][r] = Va[(s0 + s) * N + E::pt(r)];
                    if constexpr (E::GSV == 2) vb[s][r] = Vb[(s0 + s) * N + E::pt(r)];
                  }
              }
#pragma unroll
              for (int s = 0; s < SB; ++s)
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                  x.v[s0 + s][r] = cadd(x.v[s0 + s][r], cmul(ya, va[s][r]));
                  if constexpr (E::GSV == 2) x.v[s0 + s][r] = cadd(x.v[s0 + s][r], cmul(yb, vb[s][r]));
                }
            }
          }
          E::store(x, xg);
        }
        __syncthreads();  // y is read by all before it can be rewritten
        if (cv && !a.sc.verify) {
          solve_end(true);
        } else {  // verification, restart, or maxit / breakdown: the true residual decides
          request(xg, true);
          pc = kSolveResid;
        }
        break;
      }
      case kAdjAfterPhi:
        solve_begin(lam, S1, -alpha, kAdjAfterMu);
        break;
      case kAdjAfterMu:
        request(S0, false);
        pc = kAdjAphi;
        break;
      case kAdjAphi:
        E::store(y, S2);
        request(S1, false);
        pc = kAdjAmu;
        break;
      case kAdjAmu: {
        // y = A mu at owned points (surface s of point r in y.v[s][r])
        double* gF = a.gF + im.foff;
        const double coef = -(2.0 * alpha / a.mass);
        double tg[R0], g[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          const int i0 = E::pt(r), i1 = N + E::pt(r);
          tg[r] = cconjmul(S1[i0], S2[i1]).x - cconjmul(S1[i1], S2[i0]).x +
                  cconjmul(y.v[0][r], S0[i1]).x - cconjmul(y.v[1][r], S0[i0]).x;
        }
#pragma unroll
        for (int r = 0; r < R0; ++r) g[r] = gF[E::pt(r)];
        __builtin_amdgcn_sched_barrier(0);  // all loads before the first store
#pragma unroll
        for (int r = 0; r < R0; ++r) gF[E::pt(r)] = g[r] + coef * tg[r];
        OV p, t;
        E::load(p, psi);
        E::load(t, S0);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) p.v[s][r] = csub(cscale(t.v[s][r], 2.0), p.v[s][r]);
        E::store(p, psi);
        E::load(p, lam);
        E::load(t, S1);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) p.v[s][r] = csub(cscale(t.v[s][r], 2.0), p.v[s][r]);
        E::store(p, lam);
        advance();
        break;
      }
      case kExplAfter: {  // psi' = psi - i dt H psi (Eq. 13)
        OV p;
        E::load(p, psi);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) p.v[s][r] = csub(p.v[s][r], cmul_is(y.v[s][r], alpha));
        E::store(p, psi);
        y = p;  // the next step's operator input
        psi_in_y = true;
        advance();
        break;
      }
      case kImplAfter: {  // psi' = (1 + i dt H)^-1 psi (Eq. 14), solved into S0
        OV p;
        E::load(p, S0);
        E::store(p, psi);
        advance();
        break;
      }
      case kSodStart: {  // H psi(0) kept for the start and the first step; ask for H H psi(0)
        E::store(y, S2);
        request(S2, true);
        pc = kSodStart2;
        break;
      }
      case kSodStart2: {
        // psi(-dt) = psi(0) + i dt H psi(0) - dt^2/2 H H psi(0), one second-order
        // Runge-Kutta step backwards (Sec. III); then the first step of Eq. (16),
        // psi(dt) = psi(-dt) - 2 i dt H psi(0); S1 keeps the previous state psi(0)
        OV p, h1, q;
        E::load(p, psi);
        E::load(h1, S2);
        const double half2 = -0.5 * alpha * alpha;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) {
            const cplx prev = cadd(cadd(p.v[s][r], cmul_is(h1.v[s][r], alpha)), cscale(y.v[s][r], half2));
            q.v[s][r] = csub(prev, cmul_is(h1.v[s][r], 2.0 * alpha));
          }
        E::store(p, S1);
        E::store(q, psi);
        sod_started = true;
        advance();
        break;
      }
      case kSodStep: {  // psi(t + dt) = psi(t - dt) - 2 i dt H psi(t) (Eq. 16)
        OV p, q;
        E::load(p, psi);
        E::load(q, S1);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R0; ++r) q.v[s][r] = csub(q.v[s][r], cmul_is(y.v[s][r], 2.0 * alpha));
        E::store(p, S1);
        E::store(q, psi);
        y = q;  // the next step's operator input
        psi_in_y = true;
        advance();
        break;
      }
      default:
        bad = true;
        break;
    }
  }
done:
  if (threadIdx.x == 0 && a.stats) {
    ItemStats* st = a.stats + item;
    st->h_applies = napply;
    st->iterations = iters_total;
    st->iterations_sq = iters_sq;
    st->extra_vecs = extra_vecs;
    st->solves = solves;
    st->max_iters = max_iters;
    st->failures = failures;
    st->nonfinite = bad ? 1 : 0;
    st->max_resid = max_resid[0] / max_resid[1];
  }
}

// aux = H psi; aux doubles as the parking slot of the inner A psi
template <int P>
__global__ void __launch_bounds__(Eng<P>::T) k_apply_h(KArgs a) {
  using E = Eng<P>;
  constexpr int N = E::N;
  if ((int)blockIdx.x >= a.nlist) return;
  extern __shared__ double2 smem_raw[];
  GQD_L cplx* smem = (GQD_L cplx*)smem_raw;
  const ItemMeta im = a.items[a.list[blockIdx.x]];
  const auto c = E::make_ctx(smem, 0, a, im);
  typename E::OV y;
  E::apply_A((cplx*)a.psi + im.off, y, c);
  E::store(y, (cplx*)a.aux + im.off);
  E::apply_A((cplx*)a.aux + im.off, y, c);
  E::finish_H(y, (cplx*)a.psi + im.off, c);
  E::store(y, (cplx*)a.aux + im.off);
}

// Split-operator propagation in the DIABATIC representation (Table I's second-order
// splitting, composed like the implicit methods): W = [[W11, W12], [W12, W22]] is
// read from V = (W11, W22) and F = W12.  Each substep of length tau applies
// exp(-i W tau/2) pointwise, exp(-i T tau) through one transform pair with the phase
// exp(-i tau p_k^2 / 2m) in k-space, and exp(-i W tau/2) again.  The state stays in
// registers for the whole call; only the potential is read per substep.
template <int P>
__global__ void __launch_bounds__(Eng<P>::T) __attribute__((amdgpu_waves_per_eu(Eng<P>::WPE))) k_split(KArgs a) {
  using E = Eng<P>;
  if ((int)blockIdx.x >= a.nlist) return;
  extern __shared__ double2 smem_raw[];
  GQD_L cplx* smem = (GQD_L cplx*)smem_raw;
  const int item = a.list[blockIdx.x];
  const ItemMeta im = a.items[item];
  const auto c = E::make_ctx(smem, 0, a, im);
  cplx* psi = (cplx*)a.psi + im.off;
  const double dt = a.dt_item ? uniform_d(a.dt_item[item]) : a.dt;
  const long long nsteps = a.nsteps_item ? a.nsteps_item[item] : a.nsteps;
  typename E::OV y, t;
  E::load(y, psi);
  for (long long n = 0; n < nsteps; ++n) {
    for (int cc = 0; cc < a.gt.count; ++cc) {
      const double tau = substep_tau(cc, a.gt) * dt;
      E::expW(y, 0.5 * tau, c);
      t = y;
      E::template kinetic<1>(t, y, c, tau * c.inv2m);
      E::expW(y, 0.5 * tau, c);
    }
  }
  E::store(y, psi);
  if (threadIdx.x == 0 && a.stats) {  // no H applications and no solves
    ItemStats* st = a.stats + item;
    st->h_applies = 0;
    st->iterations = 0;
    st->iterations_sq = 0;
    st->solves = 0;
    st->max_iters = 0;
    st->failures = 0;
    st->nonfinite = 0;
    st->max_resid = 0.0;
  }
}

// out[item] = (norm, energy, P1, P2); energy = ||A psi||^2 / (2m) + <psi|V psi>
template <int P>
__global__ void __launch_bounds__(Eng<P>::T) k_diag(KArgs a) {
  using E = Eng<P>;
  constexpr int N = E::N;
  if ((int)blockIdx.x >= a.nlist) return;
  extern __shared__ double2 smem_raw[];
  GQD_L cplx* smem = (GQD_L cplx*)smem_raw;
  const int item = a.list[blockIdx.x];
  const ItemMeta im = a.items[item];
  const auto c = E::make_ctx(smem, 0, a, im);
  const cplx* x = (cplx*)a.psi + im.off;
  double p0 = 0.0, p1 = 0.0, pv = 0.0;
#pragma unroll
  for (int r = 0; r < E::R0; ++r) {
    const double a0 = cabs2(x[E::pt(r)]), a1 = cabs2(x[N + E::pt(r)]);
    p0 += a0;
    p1 += a1;
    pv += c.V[E::pt(r)] * a0 + c.V[N + E::pt(r)] * a1;
  }
  typename E::OV ax;
  E::apply_A(x, ax, c);
  const double ka = E::norm2(ax);
  const double P0 = E::block_sum1(p0, c) * im.dq;
  const double P1 = E::block_sum1(p1, c) * im.dq;
  const double PV = E::block_sum1(pv, c) * im.dq;
  const double KA = E::block_sum1(ka, c) * im.dq;
  if (threadIdx.x == 0) {
    double* o = a.out + 4 * (size_t)item;
    o[0] = sqrt(P0 + P1);
    o[1] = KA * a.inv2m + PV;
    o[2] = P0;
    o[3] = P1;
  }
}

// out[2 item], out[2 item + 1] = Re, Im <psi|aux> = dq * sum conj(psi) aux
template <int P>
__global__ void __launch_bounds__(Eng<P>::T) k_inner(KArgs a) {
  using E = Eng<P>;
  constexpr int N = E::N;
  if ((int)blockIdx.x >= a.nlist) return;
  extern __shared__ double2 smem_raw[];
  GQD_L cplx* smem = (GQD_L cplx*)smem_raw;
  const int item = a.list[blockIdx.x];
  const ItemMeta im = a.items[item];
  const auto c = E::make_ctx(smem, 0, a, im);
  const cplx* x = (cplx*)a.psi + im.off;
  const cplx* y = (cplx*)a.aux + im.off;
  double re = 0.0, imv = 0.0;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int r = 0; r < E::R0; ++r) {
      const cplx z = cconjmul(x[s * N + E::pt(r)], y[s * N + E::pt(r)]);
      re += z.x;
      imv += z.y;
    }
  re = E::block_sum1(re, c) * im.dq;
  imv = E::block_sum1(imv, c) * im.dq;
  if (threadIdx.x == 0) {
    a.out[2 * (size_t)item] = re;
    a.out[2 * (size_t)item + 1] = imv;
  }
}

// --------------------------------------------------------------------- launchers

#define GQD_DISPATCH(plan, EXPR)                 \
  switch (plan) {                                \
    case 0: { constexpr int P = 0; EXPR; } break;   \
    case 1: { constexpr int P = 1; EXPR; } break;   \
    case 2: { constexpr int P = 2; EXPR; } break;   \
    case 3: { constexpr int P = 3; EXPR; } break;   \
    case 4: { constexpr int P = 4; EXPR; } break;   \
    case 5: { constexpr int P = 5; EXPR; } break;   \
    case 6: { constexpr int P = 6; EXPR; } break;   \
    case 7: { constexpr int P = 7; EXPR; } break;   \
    case 8: { constexpr int P = 8; EXPR; } break;   \
    case 9: { constexpr int P = 9; EXPR; } break;   \
    case 10: { constexpr int P = 10; EXPR; } break; \
    default: return hipErrorInvalidValue;        \
  }
static_assert(kNumPlans == 11, "one dispatch case per plan");

template <int P>
static hipError_t set_lds_limit(size_t bytes) {
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_apply_h<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_run<P, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_run<P, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_diag<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_split<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_inner<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Workspace of the allocation-free entry point (gqd_propagate_noalloc): a file-scope
// device array, one copy per GPU, held until the process ends.  Host code never uses
// its name as an address (on the host it names a stand-in, not device memory): the
// device address comes from hipGetSymbolAddress, once per device, with that device
// current, and only that pointer is handed to kernels.
static __device__ __align__(256) double2 scratch[kScratchBytes / sizeof(double2)];

hipError_t scratch_address(int device, void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes it current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t configure_kernels(int m_max) {
  for (int plan = 0; plan < kNumPlans; ++plan) {
    hipError_t e = hipSuccess;
    GQD_DISPATCH(plan, {
      size_t bytes = lds_bytes(P, m_max);
      if (bytes > 160 * 1024) bytes = 160 * 1024;
      e = set_lds_limit<P>(bytes);
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

#define GQD_LAUNCH(KERNEL, M_LDS)                                                                  \
  GQD_DISPATCH(plan, {                                                                            \
    if (a.nlist <= 0) return hipSuccess;                                                          \
    hipLaunchKernelGGL(KERNEL<P>, dim3(a.nlist), dim3(Eng<P>::T), lds_bytes(P, M_LDS), stream, a); \
  });                                                                                             \
  return hipGetLastError();

hipError_t launch_apply_h(int plan, const KArgs& a, hipStream_t stream) { GQD_LAUNCH(k_apply_h, 0) }
hipError_t launch_run(int plan, const KArgs& a, hipStream_t stream) {
  GQD_DISPATCH(plan, {
    if (a.nlist <= 0) return hipSuccess;
    if (a.sc.precond)
      hipLaunchKernelGGL((k_run<P, true>), dim3(a.nlist), dim3(Eng<P>::T), lds_bytes(P, a.sc.m), stream, a);
    else
      hipLaunchKernelGGL((k_run<P, false>), dim3(a.nlist), dim3(Eng<P>::T), lds_bytes(P, a.sc.m), stream, a);
  });
  return hipGetLastError();
}
hipError_t launch_diag(int plan, const KArgs& a, hipStream_t stream) { GQD_LAUNCH(k_diag, 0) }
hipError_t launch_split(int plan, const KArgs& a, hipStream_t stream) { GQD_LAUNCH(k_split, 0) }
hipError_t launch_inner(int plan, const KArgs& a, hipStream_t stream) { GQD_LAUNCH(k_inner, 0) }

}  // namespace gqd
