// gfx950 kernel for two-surface wavepackets on 2D grids (n x n points, q1 the slow
// and q2 the fast index).  A 2 MB state at n = 256 does not fit one workgroup, so a
// group of G workgroups shares one item for a whole call:
//
//   * H = sum_d A_d A_d / (2 m_d) + V with A_d = p_d - i F^(d) (Eq. 22 and its
//     multidimensional form, Sec. II.E) splits into line operations: A_2 acts along
//     rows (fixed q1), A_1 along columns (fixed q2), each line independent.  A line
//     block is kLineWaves adjacent lines, one wave per line: the block is staged
//     through LDS with coalesced loads, each wave runs its line's Stockham transforms
//     (radix 8 where the line allows, the k-space multiply fused between the last
//     forward and the first inverse pass) in its own LDS buffers, and the block is
//     written back.  Row blocks
//     also add V psi; rows and columns write two separate partial results.
//   * every other vector operation (Gram-Schmidt, updates, norms) runs on contiguous
//     chunks of VEC / G elements per workgroup; a reduction writes one partial per
//     workgroup, crosses a grid barrier, and every workgroup then sums the partials
//     in the same fixed order, so all of them take identical decisions.
//
// Grid barriers are an arrival counter per item; a waiting workgroup polls it a
// bounded number of times and on time-out raises the item's abort flag, which makes
// every workgroup of the item leave at its next barrier.  The launch is cooperative,
// so all workgroups are resident.
#include "gqd_device.hpp"
#include "gqd_internal.h"
#include "gqd_compositions.h"

#include <cstdlib>

namespace gqd {

template <int NL>
struct G2 {
  static constexpr int WV = kLineWaves;
  static constexpr int T = kThreads2;
  static constexpr int P = NL / 64;  // points per lane per surface on a line
  static constexpr int NPTS = NL * NL;
  static constexpr long long VEC = 2LL * NPTS;
  static constexpr int NBA = NL / WV;  // line blocks per axis
  static_assert(NL % 64 == 0 && NL >= 64 && NL <= 512, "line length");
};

struct Ctx2 {
  GQD_L cplx* lines;  // [WV][2 buffers][2 surfaces][NL]
  GQD_L cplx* tw;     // [NL]
  GQD_L cplx* hcol;   // [m+1]
  GQD_L cplx* g;      // [m+1]
  GQD_L cplx* sn;     // [m]
  GQD_L cplx* y;      // [m]
  GQD_L cplx* R;      // [m(m+1)/2]
  GQD_L cplx* coef;   // [m+1]
  GQD_L double* wpart;  // [WV][kPart2]
  GQD_L double* red;    // [kPart2]
  GQD_L double* cs;     // [m]
  GQD_L double* scal;   // [16]
};

__device__ Ctx2 make_ctx2(GQD_L cplx* smem, int NL, int m) {
  Ctx2 c;
  c.lines = smem;
  c.tw = c.lines + 4 * kLineWaves * NL;
  c.hcol = c.tw + NL;
  c.g = c.hcol + (m + 1);
  c.sn = c.g + (m + 1);
  c.y = c.sn + m;
  c.R = c.y + m;
  c.coef = c.R + (m * (m + 1)) / 2;
  c.wpart = (GQD_L double*)(c.coef + (m + 1));
  c.red = c.wpart + kLineWaves * kPart2;
  c.cs = c.red + kPart2;
  c.scal = c.cs + m;
  return c;
}

// ------------------------------------------------------------------ grid barrier
struct GridSync {
  unsigned* count;
  unsigned* abort_flag;
  unsigned target;
  int G;
  int limit;
};

// Returns false (in every thread) if the item was aborted or the wait timed out.
__device__ bool grid_barrier(GridSync& s, GQD_L double* flag) {
  __syncthreads();
  s.target += (unsigned)s.G;
  if (threadIdx.x == 0) {
    bool ok = true;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(s.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int polls = 0;
    for (;;) {
      const unsigned c = __hip_atomic_load(s.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((int)(c - s.target) >= 0) break;
      if (__hip_atomic_load(s.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = false;
        break;
      }
      if (++polls > s.limit) {
        __hip_atomic_store(s.abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag = ok ? 1.0 : 0.0;
  }
  __syncthreads();
  return uniform_d(*flag) != 0.0;
}

// One-sided hand-off between the two groups of a reverse sweep: every workgroup of the
// signalling group adds one to `cnt` after its writes (release); every workgroup of the
// waiting group polls until `cnt` reaches `target` (acquire).  The wait is bounded like
// a grid barrier and gives up when either group's abort flag is set.
__device__ void group_signal(unsigned* cnt) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}
__device__ bool group_wait(const unsigned* cnt, unsigned target, unsigned* own_abort, const unsigned* other_abort,
                           int limit, GQD_L double* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    bool ok = true;
    int polls = 0;
    for (;;) {
      const unsigned c = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((int)(c - target) >= 0) break;
      if (__hip_atomic_load(own_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          __hip_atomic_load(other_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = false;
        break;
      }
      if (++polls > limit) {
        __hip_atomic_store(own_abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag = ok ? 1.0 : 0.0;
  }
  __syncthreads();
  return uniform_d(*flag) != 0.0;
}

// ---------------------------------------------------------------- reductions
// Wave-reduce v and record it as slot k of this workgroup's partial.
__device__ __forceinline__ void put_partial(const Ctx2& c, int k, double v) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) c.wpart[(threadIdx.x >> 6) * kPart2 + k] = v;
}

// Sum slots 0..K-1 over the item's workgroups: c.red[k] holds the same value in every
// workgroup afterwards.  `part` is the item's [2][G][kPart2] area; the two halves
// alternate so that a workgroup that runs ahead never overwrites partials another
// one is still reading.
__device__ bool grid_sum(const Ctx2& c, GridSync& s, double* part, int& par, int g, int K) {
  __syncthreads();
  double* mine = part + ((size_t)par * s.G + g) * kPart2;
  for (int k = threadIdx.x; k < K; k += kThreads2) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kLineWaves; ++w) t += c.wpart[w * kPart2 + k];
    mine[k] = t;
  }
  if (!grid_barrier(s, c.scal + 15)) return false;
  const double* all = part + (size_t)par * s.G * kPart2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // wave w sums slots w, w + WV, ...; the loads of four of its slots are issued before
  // any is added (G <= 256: at most four partials per lane and slot), and each slot is
  // summed over the workgroups in increasing order
  for (int kb = wave; kb < K; kb += 4 * kLineWaves) {
    double v[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = kb + q * kLineWaves;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gg = lane + 64 * r;
        v[q][r] = (k < K && gg < s.G) ? all[(size_t)gg * kPart2 + k] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (lane + 64 * r < s.G) t += v[q][r];
      t = wave_sum(t);
      const int k = kb + q * kLineWaves;
      if (lane == 0 && k < K) c.red[k] = t;
    }
  }
  __syncthreads();
  par ^= 1;
  return true;
}

// ------------------------------------------------------------ line transforms
// Line transform plans: radices (L1, L2, L3) with L1 L2 L3 = NL (L3 = 1: two factors).
// The forward transform runs Stockham passes of L1 (and L2), the last forward pass, the
// multiply by p_k / NL and the first inverse pass run as one fused pass, then the
// inverse passes of the remaining radices in reverse order: 3 passes at NL = 64 and 5
// from 128 to 512, each one read and one write of the line through LDS.
template <int NL>
struct LinePlan;
template <>
struct LinePlan<64> {
  static constexpr int L1 = 8, L2 = 8, L3 = 1;
};
template <>
struct LinePlan<128> {
  static constexpr int L1 = 4, L2 = 4, L3 = 8;
};
template <>
struct LinePlan<256> {
  static constexpr int L1 = 4, L2 = 8, L3 = 8;
};
template <>
struct LinePlan<512> {
  static constexpr int L1 = 8, L2 = 8, L3 = 8;
};

// LDS slot of line element i in a swizzled buffer: bits 3-5 are XORed into the low
// three bits.  The passes with Ns = 1 give each lane a run of R consecutive outputs,
// which unswizzled would put eight lanes of a 16-byte store on the same banks; those
// outputs are stored, and read by the next pass, through this map.
__device__ __forceinline__ int lswz(int i) { return i ^ ((i >> 3) & 7); }

// One Stockham pass of radix R (sub-transform size Ns) over both surfaces of the
// wave's line; S = -1 forward, +1 inverse.  Butterfly j of surface s reads
// x[j + r NL/R], twiddles by w_{R Ns}^{r k} (k = j mod Ns) from the line table and
// writes y[(j - k) R + k + r Ns].  SWIN / SWOUT route the input / output index
// through lswz.
template <int NL, int R, int S, bool SWIN, bool SWOUT>
__device__ __forceinline__ void line_pass(const GQD_L cplx* src, GQD_L cplx* dst, int Ns, const Ctx2& c) {
  constexpr int NR = NL / R;
  constexpr int NB = 2 * NR;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int b0 = 0; b0 < NB; b0 += 64) {
    const int bb = b0 + lane;
    if (NB % 64 == 0 || bb < NB) {
      const int s = bb / NR, j = bb % NR;
      const int k = j & (Ns - 1);
      const GQD_L cplx* in = src + s * NL;
      GQD_L cplx* out = dst + s * NL;
      cplx v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = j + r * NR;
        v[r] = in[SWIN ? lswz(idx) : idx];
      }
      const int step = NL / (R * Ns);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cplx t = c.tw[r * k * step];
        if constexpr (S > 0) t.y = -t.y;
        v[r] = cmul(v[r], t);
      }
      DFT<R, S>::run(v);
      const int o = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = o + r * Ns;
        out[SWOUT ? lswz(idx) : idx] = v[r];
      }
    }
  }
}

// Last forward pass (radix R, Ns = NL/R), momentum multiply and first inverse pass
// (radix R, Ns = 1) in registers: butterfly j's forward outputs are the k-space points
// j + r NL/R, which are exactly the inputs of inverse butterfly j.  The inverse pass
// writes y[j R + r] through lswz.
template <int NL, int R, bool SWIN>
__device__ __forceinline__ void line_fused(const GQD_L cplx* src, GQD_L cplx* dst, const Ctx2& c, double pn) {
  constexpr int NR = NL / R;
  constexpr int NB = 2 * NR;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int b0 = 0; b0 < NB; b0 += 64) {
    const int bb = b0 + lane;
    if (NB % 64 == 0 || bb < NB) {
      const int s = bb / NR, j = bb % NR;
      const GQD_L cplx* in = src + s * NL;
      GQD_L cplx* out = dst + s * NL;
      cplx v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = j + r * NR;
        v[r] = in[SWIN ? lswz(idx) : idx];
      }
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], c.tw[r * j]);
      DFT<R, -1>::run(v);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int kk = j + r * NR;  // k-space index
        v[r] = cscale(v[r], pn * (double)(kk < NL / 2 ? kk : kk - NL));
      }
      DFT<R, 1>::run(v);
#pragma unroll
      for (int r = 0; r < R; ++r) out[lswz(j * R + r)] = v[r];
    }
  }
}

// y = IFFT(p FFT x) on the wave's line, both surfaces (x, y: lane's points lane + 64 r).
// Orders a wave's own LDS passes: every line of a block lives in its wave's own
// buffers, so the passes need no workgroup barrier.
__device__ __forceinline__ void line_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NL>
__device__ void line_kinetic(const cplx (&x)[2][NL / 64], cplx (&y)[2][NL / 64], const Ctx2& c, double ps) {
  using E = G2<NL>;
  using L = LinePlan<NL>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  GQD_L cplx* b0 = c.lines + (size_t)wave * 4 * NL;
  GQD_L cplx* b1 = b0 + 2 * NL;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int r = 0; r < E::P; ++r) b0[s * NL + lane + 64 * r] = x[s][r];
  line_wave_sync();
  const double pn = ps / (double)NL;
  GQD_L cplx* out;
  if constexpr (L::L3 == 1) {
    line_pass<NL, L::L1, -1, false, true>(b0, b1, 1, c);
    line_wave_sync();
    line_fused<NL, L::L2, true>(b1, b0, c, pn);
    line_wave_sync();
    line_pass<NL, L::L1, 1, true, false>(b0, b1, L::L2, c);
    line_wave_sync();
    out = b1;
  } else {
    line_pass<NL, L::L1, -1, false, true>(b0, b1, 1, c);
    line_wave_sync();
    line_pass<NL, L::L2, -1, true, false>(b1, b0, L::L1, c);
    line_wave_sync();
    line_fused<NL, L::L3, false>(b0, b1, c, pn);
    line_wave_sync();
    line_pass<NL, L::L2, 1, true, false>(b1, b0, L::L3, c);
    line_wave_sync();
    line_pass<NL, L::L1, 1, false, false>(b0, b1, L::L3 * L::L2, c);
    line_wave_sync();
    out = b1;
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int r = 0; r < E::P; ++r) y[s][r] = out[s * NL + lane + 64 * r];
  line_wave_sync();
}

// y += -i F x coupling of A = p - i F: (A x)_1 gains -i F12 x_2, (A x)_2 gains +i F12 x_1
template <int P>
__device__ __forceinline__ void line_couple(cplx (&y)[2][P], const cplx (&x)[2][P], const double (&f)[P]) {
#pragma unroll
  for (int r = 0; r < P; ++r) {
    y[0][r] = cadd(y[0][r], mk(f[r] * x[1][r].y, -f[r] * x[1][r].x));
    y[1][r] = cadd(y[1][r], mk(-f[r] * x[0][r].y, f[r] * x[0][r].x));
  }
}

// Index of element (surface s, line l, point i) of a row (q1 fixed = l) or column
// (q2 fixed = l) block, in the [2][NL][NL] layout.
template <int NL>
__device__ __forceinline__ int line_gidx(bool row, int s, int l, int i) {
  return s * NL * NL + (row ? l * NL + i : i * NL + l);
}
// Cooperative mapping of element e of a block of kLineWaves lines onto (s, w, i):
// rows are contiguous along i, columns along w.
template <int NL>
__device__ __forceinline__ void block_map(bool row, int e, int& s, int& w, int& i) {
  s = e / (kLineWaves * NL);
  const int rem = e - s * kLineWaves * NL;
  // rows: w = rem / NL, i = rem % NL; columns: i = rem / kLineWaves, w = rem % kLineWaves
  // (selected as values, so that no private array of {w, i} is formed)
  const int qr = rem / NL, qc = rem / kLineWaves;
  w = row ? qr : rem - qc * kLineWaves;
  i = row ? rem - qr * NL : qc;
}

// Line operation request of the propagation machine.
// The operand is x = scale * (srcw src + src2w src2 - i hal (h1 + h2) - sum_{i<K} coef_i basis_i)
// (src2, h1, h2 may be null, coef in LDS); row and column blocks form it with the same
// operations, so both see the same values, and row blocks store it to copy_dst.  The
// h term forms (1 - i al H) b from b and the two halves of H b (or a stored H b), so a
// GMRES guess or a trapezoidal right-hand side needs no pass and no grid barrier of
// its own.
struct LineReq {
  const cplx* src;
  const cplx* src2;
  const cplx* basis;
  int K;
  cplx scale;        // applied when `scaled`
  bool scaled;
  cplx* copy_dst;    // may be null
  bool opH;          // true: H parts; false: A_d x along each axis
  cplx* out_r;       // rows:    A_2 A_2 x / (2 m_2) + (V - shift) x   |  A_2 x
  cplx* out_c;       // columns: A_1 A_1 x / (2 m_1)                   |  A_1 x
  double shift = 0.0;  // H - shift (Arnoldi only)
  const cplx* h1 = nullptr;
  const cplx* h2 = nullptr;
  double hal = 0.0;
  double srcw = 1.0;   // weights of src and src2 (applied only when not 1)
  double src2w = 1.0;
};

template <int NL>
__device__ void line_op(const LineReq& q, const Ctx2& c, const K2Args& a, const Item2& im, int g) {
  using E = G2<NL>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double* V = a.V + im.off;
  const double* F = a.F + im.off;
  for (int b = g; b < 2 * E::NBA; b += a.G) {
    const bool row = b < E::NBA;
    // Column slot j = 16 q + 8 h + r takes column block 2 (8 q + r) + h: the two blocks
    // whose four columns share 128-byte lines (blocks 2k and 2k + 1) go to workgroups
    // eight apart, which the dispatcher places on the same XCD, so one L2 serves both
    // halves of every line.
    const int cj = b - E::NBA;
    const int cb = 2 * (8 * (cj >> 4) + (cj & 7)) + ((cj >> 3) & 1);
    const int l0 = (row ? b : cb) * kLineWaves;
    // EB elements per thread at a time, each source read for all of them before any is
    // used, so that a wave keeps EB loads in flight (per element the operations and
    // their order are those of the formula above)
    constexpr int EPT = 2 * kLineWaves * NL / kThreads2;
    constexpr int EB = EPT < 8 ? EPT : 8;
    static_assert(EPT % EB == 0, "line block elements per thread");
#pragma unroll 1
    for (int e0 = 0; e0 < EPT; e0 += EB) {
      int gi[EB], li[EB];
      cplx v[EB], t[EB];
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        int s, w, i;
        block_map<NL>(row, threadIdx.x + (e0 + u) * kThreads2, s, w, i);
        gi[u] = line_gidx<NL>(row, s, l0 + w, i);
        li[u] = w * 4 * NL + s * NL + i;
      }
      // all sources are requested before any is used (after a grid barrier every read
      // misses the L2, so each round of dependent loads costs a full memory latency)
      cplx t2[EB], t3[EB];
#pragma unroll
      for (int u = 0; u < EB; ++u) v[u] = q.src[gi[u]];
      if (q.src2) {
#pragma unroll
        for (int u = 0; u < EB; ++u) t[u] = q.src2[gi[u]];
      }
      if (q.h1) {
#pragma unroll
        for (int u = 0; u < EB; ++u) t2[u] = q.h1[gi[u]];
      }
      if (q.h2) {
#pragma unroll
        for (int u = 0; u < EB; ++u) t3[u] = q.h2[gi[u]];
      }
      if (q.srcw != 1.0) {
#pragma unroll
        for (int u = 0; u < EB; ++u) v[u] = cscale(v[u], q.srcw);
      }
      if (q.src2) {
        if (q.src2w != 1.0) {
#pragma unroll
          for (int u = 0; u < EB; ++u) t[u] = cscale(t[u], q.src2w);
        }
#pragma unroll
        for (int u = 0; u < EB; ++u) v[u] = cadd(v[u], t[u]);
      }
      if (q.h1) {
        if (q.h2) {
#pragma unroll
          for (int u = 0; u < EB; ++u) t2[u] = cadd(t2[u], t3[u]);
        }
#pragma unroll
        for (int u = 0; u < EB; ++u) v[u] = csub(v[u], cmul_is(t2[u], q.hal));
      }
      // basis vectors two at a time, both loads in flight together
      int k = 0;
      for (; k + 1 < q.K; k += 2) {
        const cplx* bk = q.basis + (size_t)k * E::VEC;
        const cplx* bk1 = bk + E::VEC;
        const cplx ck = c.coef[k], ck1 = c.coef[k + 1];
#pragma unroll
        for (int u = 0; u < EB; ++u) {
          t[u] = bk[gi[u]];
          t2[u] = bk1[gi[u]];
        }
#pragma unroll
        for (int u = 0; u < EB; ++u) v[u] = csub(v[u], cmul(ck, t[u]));
#pragma unroll
        for (int u = 0; u < EB; ++u) v[u] = csub(v[u], cmul(ck1, t2[u]));
      }
      if (k < q.K) {
        const cplx* bk = q.basis + (size_t)k * E::VEC;
        const cplx ck = c.coef[k];
#pragma unroll
        for (int u = 0; u < EB; ++u) t[u] = bk[gi[u]];
#pragma unroll
        for (int u = 0; u < EB; ++u) v[u] = csub(v[u], cmul(ck, t[u]));
      }
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        if (q.scaled) v[u] = cmul(q.scale, v[u]);
        if (row && q.copy_dst) q.copy_dst[gi[u]] = v[u];
        c.lines[li[u]] = v[u];
      }
    }
    __syncthreads();
    const int ln = l0 + wave;
    const GQD_L cplx* mine = c.lines + (size_t)wave * 4 * NL;
    cplx x[2][E::P], y[2][E::P];
    double f[E::P];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int r = 0; r < E::P; ++r) x[s][r] = mine[s * NL + lane + 64 * r];
    const int d = row ? 1 : 0;  // rows move along q2 (F^(2)), columns along q1 (F^(1))
#pragma unroll
    for (int r = 0; r < E::P; ++r) f[r] = F[d * E::NPTS + line_gidx<NL>(row, 0, ln, lane + 64 * r)];
    // (selected as values: a select between two fields would become a private array)
    const double ps0 = im.ps0, ps1 = im.ps1;
    const double ps = row ? ps1 : ps0;
    line_kinetic<NL>(x, y, c, ps);
    line_couple<E::P>(y, x, f);
    if (q.opH) {
      cplx z[2][E::P];
      line_kinetic<NL>(y, z, c, ps);
      line_couple<E::P>(z, y, f);
      const double m0 = a.inv2m0, m1 = a.inv2m1;
      const double inv2m = row ? m1 : m0;
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int r = 0; r < E::P; ++r) {
          y[s][r] = cscale(z[s][r], inv2m);
          if (row) y[s][r] = cadd(y[s][r], cscale(x[s][r], V[line_gidx<NL>(true, s, ln, lane + 64 * r)] - q.shift));
        }
    }
    GQD_L cplx* outl = c.lines + (size_t)wave * 4 * NL;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int r = 0; r < E::P; ++r) outl[s * NL + lane + 64 * r] = y[s][r];
    __syncthreads();
    cplx* out = row ? q.out_r : q.out_c;
    for (int e = threadIdx.x; e < 2 * kLineWaves * NL; e += kThreads2) {
      int s, w, i;
      block_map<NL>(row, e, s, w, i);
      out[line_gidx<NL>(row, s, l0 + w, i)] = c.lines[(size_t)w * 4 * NL + s * NL + i];
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------- propagation
enum Pc2 {
  k2Substep,
  k2SolveGuess,
  k2SolveResid,
  k2SolveArnoldi,
  k2MidpAfter,
  k2MidpExplicit,
  k2TrapHpsi,
  k2TrapAfter,
  k2AdjAfterPhi,
  k2AdjAfterMu,
  k2AdjAphi,
  k2AdjAmu,
  k2AdjPhiDone,   // two groups: role 0 has phi, asks for A phi
  k2AdjGrad,      // two groups: role 0 has A phi; waits for mu, adds the gradient, updates psi
  k2AdjMuDone,    // two groups: role 1 has mu, asks for A mu
  k2AdjMuAfter,   // two groups: role 1 has A mu; updates lambda and signals
  k2ApplyDone,
  k2DiagDone,
  k2Inner
};

// substep fractions of the non-recursive compositions (gqd_compositions.h)
static __constant__ double kFlatTau2[kFlatTauLen] = {GQD_FLAT_TAU_VALUES};

__device__ __forceinline__ double substep_tau2(int cc, const GammaTab& gt) {
  if (gt.flat) return kFlatTau2[gt.flat - 1 + cc];
  double t = 1.0;
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

// One item per group of a.G workgroups; the same machine as the 1D kernel
// (propagation per substep of length h = tau_c dt, alpha = h/2, Sec. II.C-D; reverse
// sweep), with the state in global memory and grid-wide reductions.
//   midpoint (Eq. 19):  x = (1 + i alpha H)^-1 psi;  psi' = (1 - i alpha H) x, or 2x - psi
//   trapezoid (Eq. 18): b = (1 - i alpha H) psi;     psi' = (1 + i alpha H)^-1 b
//   reverse sweep: phi = (1 - i alpha H)^-1 psi, mu = (1 - i alpha H)^-1 lambda,
//   psi <- 2 phi - psi, lambda <- 2 mu - lambda and, per axis d,
//   gF_d += -(2 alpha / m_d) Re[conj(mu1)(A_d phi)2 - conj(mu2)(A_d phi)1
//                                + conj(A_d mu)1 phi2 - conj(A_d mu)2 phi1].
// GMRES(m) from x0 = (1 - i al H) b with an Arnoldi basis of H - s, s a real shift near
// the Rayleigh quotient of v_0 (classical Gram-Schmidt, a second pass when the first
// removes all but kReorthRatio of |w|^2) and
// Givens rotations on the Hessenberg matrix of 1 + i al H; stop at |g_(j+1)| <= tol |b|.
// Chunk loops that sum over basis vectors take kChunkB elements per thread at a time,
// reading each vector for all of them before using any (loads kept in flight together).
constexpr int kChunkB = 4;

template <int NL>
__global__ void __launch_bounds__(kThreads2) k_run2d(K2Args a) {
  using E = G2<NL>;
  constexpr int T = kThreads2;
  const int G = a.G;
  const int R = a.roles;
  const int grp = blockIdx.x / G;
  const int item = grp / R;
  const int role = grp - item * R;
  const int g = blockIdx.x - grp * G;
  if (item >= a.batch) return;
  extern __shared__ double2 smem_raw[];
  const int m = a.sc.m;
  const Ctx2 c = make_ctx2((GQD_L cplx*)smem_raw, NL, m);
  for (int t = threadIdx.x; t < NL; t += T) c.tw[t] = ((const cplx*)a.tw)[t];
  __syncthreads();
  const Item2 im = a.items[item];
  cplx* psi = (cplx*)a.psi + im.off;
  cplx* lam = (cplx*)a.aux + im.off;
  cplx* wk = (cplx*)a.work + (size_t)grp * a.work_stride;
  // with two groups, role 1 keeps mu in its B slot and A mu in its AR, AC slots
  cplx* wk1 = (cplx*)a.work + (size_t)(item * R + R - 1) * a.work_stride;
  cplx* X = wk;                   // solve output | phi
  cplx* B = wk + E::VEC;          // rhs          | mu
  cplx* HP = wk + 2 * E::VEC;     // H psi (trapezoid economy)
  // row and column parts of the last H x (or A_2 phi, A_1 phi), and a spare pair that
  // the next line operation writes while the current one may still be read
  cplx* OR = wk + 3 * E::VEC;
  cplx* OC = wk + 4 * E::VEC;
  cplx* ORs = wk + 8 * E::VEC;
  cplx* OCs = wk + 9 * E::VEC;
  cplx* W = wk + 5 * E::VEC;      // partly orthogonalised Arnoldi vector, residual
  cplx* AR = wk + 6 * E::VEC;     // A_2 mu
  cplx* AC = wk + 7 * E::VEC;     // A_1 mu
  cplx* basis = wk + kWork2Extra * E::VEC;
  static_assert(kWork2Extra == 10, "workspace slots");
  GridSync sy{a.sync + 2 * grp, a.sync + 2 * grp + 1, 0u, G, a.spin_limit};
  unsigned* other_abort = a.sync + 2 * (item * R + (R - 1 - role)) + 1;
  unsigned* hand = a.sync + 2 * (size_t)a.batch * R + 2 * item;  // [0] mu ready, [1] gradient done
  unsigned handoffs = 0;  // substeps this group has completed (two-group reverse sweep)
  double* part = a.part + (size_t)grp * 2 * G * kPart2;
  int par = 0;
  const long long CH = E::VEC / G;
  const long long e0 = (long long)g * CH, e1 = e0 + CH;
  const long long PCH = E::NPTS / G;  // chunk of grid points (both surfaces) for the gradient
  const long long p0 = (long long)g * PCH, p1 = p0 + PCH;

  const bool adj = a.mode == kM2Adjoint;
  const bool midp = a.method == kMidp;
  const bool literal = a.sc.literal != 0;
  const double dt = a.dt;
  const long long nsteps = a.nsteps;

  long long napply = 0, iters_total = 0, iters_sq = 0, extra_vecs = 0;
  int solves = 0, max_iters = 0, failures = 0;
  bool bad = false, aborted = false;
  bool have_hpsi = false;
  bool touched = false;  // chunk work touched global memory since the last barrier

  long long n = 0;
  int cc = adj ? a.gt.count - 1 : 0;
  double alpha = 0.0;

  bool pending = false, swap_after = false;
  // Midpoint fold: a converged solve that is not the call's last leaves x = x0 + V y and
  // psi' = 2 x - psi to the load of the next substep's first H request, which forms
  // psi' = 2 x0 + 2 V y - psi and stores it to the other buffer of the pair (psi, HP);
  // fold_k > 0: pending, with y in LDS and fold_k basis vectors
  int fold_k = 0;
  cplx* psi_cur = psi;
  LineReq rq{};
  const cplx* bg = nullptr;
  cplx* xg = nullptr;
  double al = 0.0, tolb = 0.0, bnrm = 0.0;
  double max_resid = 0.0;  // largest true relative residual a solve ended on
  int j = 0, iters = 0, after = k2Substep;
  int pc = k2Substep;
  // Arnoldi runs on H - s, s the Rayleigh quotient of the first basis vector of the
  // previous solve of the same kind (sig0: psi or phi, sig1: the adjoint's mu)
  double sig0 = 0.0, sig1 = 0.0;
  bool kind_mu = false;
  if (a.mode == kM2ApplyH || a.mode == kM2Diag) {
    rq = LineReq{psi, nullptr, nullptr, 0, mk(1.0, 0.0), false, nullptr, a.mode == kM2ApplyH, ORs, OCs};
    pending = true;
    swap_after = true;
    pc = a.mode == kM2ApplyH ? k2ApplyDone : k2DiagDone;
  } else if (a.mode == kM2Inner) {
    pc = k2Inner;
  }

  // H x (or A_d x) of a global vector into the spare pair, which becomes current
  auto request = [&](const cplx* src, bool h) {
    rq = LineReq{src, nullptr, nullptr, 0, mk(1.0, 0.0), false, nullptr, h, ORs, OCs};
    pending = true;
    swap_after = true;
  };
  auto gsum = [&](int K) -> bool {
    touched = false;
    if (!grid_sum(c, sy, part, par, g, K)) {
      aborted = true;
      return false;
    }
    return true;
  };
  // start a solve of (1 + i al H) x = b: ask for H b.  |b| joins the first residual's
  // reduction; pre (when given) forms b itself in that load as src - i al_b h_1 (+ h_2)
  // and stores it to b, the trapezoid's right-hand side.
  auto solve_begin = [&](const cplx* b, cplx* x, double alv, int ret, const LineReq* pre = nullptr) {
    bg = b;
    xg = x;
    al = alv;
    after = ret;
    kind_mu = ret == k2AdjAfterMu;
    iters = 0;
    if (pre) {
      rq = *pre;
      pending = true;
      swap_after = true;
    } else {
      request(b, true);
    }
    pc = k2SolveGuess;
  };
  auto solve_end = [&](bool conv) {
    // the two groups of a reverse sweep interleave: phi solves even, mu solves odd
    if (g == 0 && threadIdx.x == 0)
      log_solve(a.stats ? a.stats + item : nullptr, R == 2 ? 2LL * solves + role : (long long)solves, iters);
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
    pc = k2Substep;
  };

  // partial sums of <v_i, y> over this chunk, i < K, into slots 2i, 2i+1, with
  // y = y1 (+ y2); with norm_slot >= 0, |y|^2 into that slot (four basis vectors per
  // sweep so that y is read once per four)
  auto chunk_dots = [&](const cplx* y1, const cplx* y2, int K, int norm_slot) {
    double nn = 0.0;
    for (int i0 = 0; i0 < K; i0 += 4) {
      const int nv = K - i0 < 4 ? K - i0 : 4;
      double sx[4] = {0.0, 0.0, 0.0, 0.0}, sv[4] = {0.0, 0.0, 0.0, 0.0};
      // kChunkB elements per thread at a time, all their loads issued before any use
      for (long long eb = e0 + threadIdx.x; eb < e1; eb += kChunkB * T) {
        cplx w[kChunkB], w2[kChunkB], bv[4][kChunkB];
#pragma unroll
        for (int q = 0; q < kChunkB; ++q) {
          const long long e = eb + q * T;
          w[q] = e < e1 ? y1[e] : mk(0.0, 0.0);
          if (y2) w2[q] = e < e1 ? y2[e] : mk(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (u < nv) {
            const cplx* bu = basis + (size_t)(i0 + u) * E::VEC;
#pragma unroll
            for (int q = 0; q < kChunkB; ++q) {
              const long long e = eb + q * T;
              bv[u][q] = e < e1 ? bu[e] : mk(0.0, 0.0);
            }
          }
#pragma unroll
        for (int q = 0; q < kChunkB; ++q) {
          if (eb + q * T >= e1) break;
          if (y2) w[q] = cadd(w[q], w2[q]);
          if (i0 == 0) nn += cabs2(w[q]);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (u < nv) {
              const cplx z = cconjmul(bv[u][q], w[q]);
              sx[u] += z.x;
              sv[u] += z.y;
            }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (u < nv) {
          put_partial(c, 2 * (i0 + u), sx[u]);
          put_partial(c, 2 * (i0 + u) + 1, sv[u]);
        }
    }
    if (norm_slot >= 0) put_partial(c, norm_slot, nn);
  };

  for (;;) {
    if (bad || aborted) break;
    if (pending) {
      if (touched && !grid_barrier(sy, c.scal + 15)) {
        aborted = true;
        break;
      }
      line_op<NL>(rq, c, a, im, g);
      if (rq.opH) ++napply;
      if (swap_after) {
        cplx* t = OR;
        OR = ORs;
        ORs = t;
        t = OC;
        OC = OCs;
        OCs = t;
      }
      pending = false;
      touched = false;
      if (!grid_barrier(sy, c.scal + 15)) {
        aborted = true;
        break;
      }
    }
    switch (pc) {
      case k2Substep: {
        if (n >= nsteps) goto done;
        alpha = 0.5 * (substep_tau2(cc, a.gt) * dt);
        if (adj && R == 2) {
          if (role == 0) {
            solve_begin(psi, X, -alpha, k2AdjPhiDone);
          } else {
            // mu of the previous substep must have been read by the gradient
            if (!group_wait(hand + 1, handoffs * (unsigned)G, sy.abort_flag, other_abort, a.spin_limit,
                            c.scal + 15)) {
              aborted = true;
              break;
            }
            solve_begin(lam, B, -alpha, k2AdjMuDone);
          }
        } else if (adj) {
          solve_begin(psi, X, -alpha, k2AdjAfterPhi);
        } else if (midp) {
          if (fold_k > 0) {
            // b = 2 x0 + 2 V y - psi, formed by the load of H b and stored to the other buffer
            for (int i = threadIdx.x; i < fold_k; i += T) c.coef[i] = cscale(c.y[i], -2.0);
            __syncthreads();
            cplx* nb = psi_cur == psi ? HP : psi;
            LineReq pre{X, psi_cur, basis, fold_k, mk(1.0, 0.0), false, nb, true, ORs, OCs};
            pre.srcw = 2.0;
            pre.src2w = -1.0;
            psi_cur = nb;
            fold_k = 0;
            solve_begin(psi_cur, X, alpha, k2MidpAfter, &pre);
          } else {
            solve_begin(psi_cur, X, alpha, k2MidpAfter);
          }
        } else if (literal || !have_hpsi) {
          request(psi, true);
          pc = k2TrapHpsi;
        } else {
          pc = k2TrapHpsi;
        }
        break;
      }
      case k2TrapHpsi: {
        // b = (1 - i alpha H) psi, formed and stored by the load of H b
        const bool fresh = literal || !have_hpsi;
        LineReq pre{psi, nullptr, nullptr, 0, mk(1.0, 0.0), false, B, true, ORs, OCs};
        pre.h1 = fresh ? OR : HP;
        pre.h2 = fresh ? OC : nullptr;
        pre.hal = alpha;
        solve_begin(B, psi, alpha, k2TrapAfter, &pre);
        break;
      }
      case k2TrapAfter: {
        if (!literal) {
          for (long long e = e0 + threadIdx.x; e < e1; e += T) {
            const cplx d = csub(B[e], psi[e]);  // H psi' = (b - psi') / (i alpha)
            HP[e] = mk(d.y / alpha, -d.x / alpha);
          }
          touched = true;
          have_hpsi = true;
        }
        advance();
        break;
      }
      case k2MidpAfter: {
        if (literal) {
          request(X, true);
          pc = k2MidpExplicit;
          break;
        }
        if (fold_k > 0) {  // the next substep's first load forms psi'
          advance();
          break;
        }
        // into the caller's buffer, whichever of the pair holds psi now
        for (long long e = e0 + threadIdx.x; e < e1; e += T) psi[e] = csub(cscale(X[e], 2.0), psi_cur[e]);
        psi_cur = psi;
        touched = true;
        advance();
        break;
      }
      case k2MidpExplicit: {
        for (long long e = e0 + threadIdx.x; e < e1; e += T)
          psi[e] = csub(X[e], cmul_is(cadd(OR[e], OC[e]), alpha));
        touched = true;
        advance();
        break;
      }
      case k2SolveGuess: {
        // x0 = (1 - i al H) b, formed and stored by the load of H x0
        rq = LineReq{bg, nullptr, nullptr, 0, mk(1.0, 0.0), false, xg, true, ORs, OCs};
        rq.h1 = OR;
        rq.h2 = OC;
        rq.hal = al;
        pending = true;
        swap_after = true;
        pc = k2SolveResid;
        break;
      }
      case k2SolveResid: {
        double acc = 0.0, accb = 0.0;
        for (long long eb = e0 + threadIdx.x; eb < e1; eb += kChunkB * T) {
          cplx bv[kChunkB], xv[kChunkB], o1[kChunkB], o2[kChunkB];
#pragma unroll
          for (int q = 0; q < kChunkB; ++q) {
            const long long e = eb + q * T;
            const bool in = e < e1;
            bv[q] = in ? bg[e] : mk(0.0, 0.0);
            xv[q] = in ? xg[e] : mk(0.0, 0.0);
            o1[q] = in ? OR[e] : mk(0.0, 0.0);
            o2[q] = in ? OC[e] : mk(0.0, 0.0);
          }
#pragma unroll
          for (int q = 0; q < kChunkB; ++q) {
            const long long e = eb + q * T;
            if (e >= e1) break;
            const cplx r = csub(bv[q], cadd(xv[q], cmul_is(cadd(o1[q], o2[q]), al)));  // b - X x
            W[e] = r;
            acc += cabs2(r);
            accb += cabs2(bv[q]);
          }
        }
        put_partial(c, 0, acc);
        put_partial(c, 1, accb);
        if (!gsum(2)) break;
        const double bnorm = sqrt(uniform_d(c.red[1]));
        if (!isfinite(bnorm)) {
          bad = true;
          break;
        }
        tolb = a.sc.tol * bnorm;
        bnrm = bnorm;
        const double beta = sqrt(uniform_d(c.red[0]));
        if (!isfinite(beta)) {
          bad = true;
          break;
        }
        if (beta <= tolb) {
          const double rr = bnrm > 0.0 ? beta / bnrm : 0.0;
          if (rr > max_resid) max_resid = rr;
          solve_end(true);
          break;
        }
        if (iters >= a.sc.maxit) {
          solve_end(false);
          break;
        }
        if (threadIdx.x == 0) c.g[0] = mk(beta, 0.0);
        // v_0 = r / beta: the H request scales the residual on the fly and row blocks
        // store the scaled values as the first basis vector
        rq = LineReq{W, nullptr, nullptr, 0, mk(1.0 / beta, 0.0), true, basis, true, ORs, OCs,
                     kind_mu ? sig1 : sig0};
        pending = true;
        swap_after = true;
        j = 0;
        pc = k2SolveArnoldi;
        break;
      }
      case k2SolveArnoldi: {
        ++iters;
        // w = (H - s) v_j = OR + OC: h_i = <v_i, w> (i <= j) and |w|^2 in one reduction;
        // |w'|^2 = |w|^2 - sum |h_i|^2 when the pass keeps at least half of |w|^2.  The
        // shift s (any real s spans the same Krylov space) shrinks |w| and with it the
        // cancellation, so the second pass is rarely needed.
        const double sh = rq.shift;
        chunk_dots(OR, OC, j + 1, 2 * (j + 1));
        if (!gsum(2 * (j + 1) + 1)) break;
        const double w2 = uniform_d(c.red[2 * (j + 1)]);
        if (j == 0) {  // <v_0|H v_0>, the shift of the following columns and solves
          const double rq0 = uniform_d(c.red[0]) + sh;
          if (kind_mu) sig1 = rq0; else sig0 = rq0;
        }
        for (int i = threadIdx.x; i <= j; i += T) {
          c.hcol[i] = mk(c.red[2 * i], c.red[2 * i + 1]);
          c.coef[i] = c.hcol[i];
        }
        __syncthreads();
        double hn2 = w2;
        for (int i = 0; i <= j; ++i) hn2 -= cabs2(c.coef[i]);
        hn2 = uniform_d(hn2);
        const cplx* base = OR;
        const cplx* base2 = OC;
        if (hn2 < kReorthRatio * w2) {
          extra_vecs += 2 * (j + 1);
          // second pass: W = w - sum h_i v_i, then c_i = <v_i, W> and |W|^2 in one
          // reduction; the update by c is left to the next operand load
          for (long long eb = e0 + threadIdx.x; eb < e1; eb += kChunkB * T) {
            cplx w[kChunkB], t[kChunkB];
#pragma unroll
            for (int u = 0; u < kChunkB; ++u) {
              const long long e = eb + u * T;
              w[u] = e < e1 ? OR[e] : mk(0.0, 0.0);
              t[u] = e < e1 ? OC[e] : mk(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < kChunkB; ++u) w[u] = cadd(w[u], t[u]);
            for (int i = 0; i <= j; ++i) {
              const cplx* bi = basis + (size_t)i * E::VEC;
              const cplx ci = c.coef[i];
#pragma unroll
              for (int u = 0; u < kChunkB; ++u) t[u] = eb + u * T < e1 ? bi[eb + u * T] : mk(0.0, 0.0);
#pragma unroll
              for (int u = 0; u < kChunkB; ++u) w[u] = csub(w[u], cmul(ci, t[u]));
            }
#pragma unroll
            for (int u = 0; u < kChunkB; ++u)
              if (eb + u * T < e1) W[eb + u * T] = w[u];
          }
          chunk_dots(W, nullptr, j + 1, 2 * (j + 1));
          touched = true;
          if (!gsum(2 * (j + 1) + 1)) break;
          double r2 = uniform_d(c.red[2 * (j + 1)]);
          for (int i = threadIdx.x; i <= j; i += T) {
            c.coef[i] = mk(c.red[2 * i], c.red[2 * i + 1]);
            c.hcol[i] = cadd(c.hcol[i], c.coef[i]);
          }
          __syncthreads();
          for (int i = 0; i <= j; ++i) r2 -= cabs2(c.coef[i]);
          hn2 = uniform_d(r2 > 0.0 ? r2 : 0.0);
          base = W;
          base2 = nullptr;
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
        gm_givens(j, fabs(al) * hn, c);
        const double gabs = uniform_d(c.scal[0]);
        if (!isfinite(hn) || !isfinite(gabs)) {
          bad = true;
          break;
        }
        const bool cv = gabs <= tolb;
        if (!cv && hn != 0.0 && iters < a.sc.maxit && j + 1 < m) {
          // v_(j+1) = i sign(al) w' / |w'|, formed while the next H application loads it
          const double sc = (al >= 0.0 ? 1.0 : -1.0) / hn;
          const int K = j + 1;
          ++j;
          rq = LineReq{base, base2, basis, K, mk(0.0, sc), true, basis + (size_t)j * E::VEC, true, ORs, OCs,
                       kind_mu ? sig1 : sig0};
          pending = true;
          swap_after = true;
          break;
        }
        const int k = j + 1;
        gm_back_solve(k, c);
        if (cv && !a.sc.verify && after == k2MidpAfter && !literal && !adj &&
            !(cc + 1 == a.gt.count && n + 1 >= nsteps)) {
          // a midpoint solve with a substep after it in this call: x = x0 + V y and the
          // update psi' = 2x - psi go into the next H request's load (fold_k)
          fold_k = k;
          solve_end(true);
          break;
        }
        for (long long eb = e0 + threadIdx.x; eb < e1; eb += kChunkB * T) {
          cplx x[kChunkB], t[kChunkB];
#pragma unroll
          for (int u = 0; u < kChunkB; ++u) x[u] = eb + u * T < e1 ? xg[eb + u * T] : mk(0.0, 0.0);
          for (int i = 0; i < k; ++i) {
            const cplx* bi = basis + (size_t)i * E::VEC;
            const cplx yi = c.y[i];
#pragma unroll
            for (int u = 0; u < kChunkB; ++u) t[u] = eb + u * T < e1 ? bi[eb + u * T] : mk(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < kChunkB; ++u) x[u] = cadd(x[u], cmul(yi, t[u]));
          }
#pragma unroll
          for (int u = 0; u < kChunkB; ++u)
            if (eb + u * T < e1) xg[eb + u * T] = x[u];
        }
        touched = true;
        if (cv && !a.sc.verify) {
          solve_end(true);
        } else {  // verification, restart, or maxit / breakdown: the true residual decides
          request(xg, true);
          pc = k2SolveResid;
        }
        break;
      }
      case k2AdjAfterPhi:
        solve_begin(lam, B, -alpha, k2AdjAfterMu);
        break;
      case k2AdjAfterMu:
        request(X, false);
        pc = k2AdjAphi;
        break;
      case k2AdjAphi:
        rq = LineReq{B, nullptr, nullptr, 0, mk(1.0, 0.0), false, nullptr, false, AR, AC};
        pending = true;
        swap_after = false;
        pc = k2AdjAmu;
        break;
      case k2AdjAmu: {
        double* gF = a.gF + im.off;
        const double c1 = -(2.0 * alpha / a.mass1), c0 = -(2.0 * alpha / a.mass0);
        for (long long p = p0 + threadIdx.x; p < p1; p += T) {
          const long long i0 = p, i1 = E::NPTS + p;
          const cplx ph0 = X[i0], ph1 = X[i1], mu0 = B[i0], mu1 = B[i1];
          // axis of q2 (rows): A_2 phi in OR, A_2 mu in AR; axis of q1 (columns): OC, AC
          const double t1 = cconjmul(mu0, OR[i1]).x - cconjmul(mu1, OR[i0]).x +
                            cconjmul(AR[i0], ph1).x - cconjmul(AR[i1], ph0).x;
          const double t0 = cconjmul(mu0, OC[i1]).x - cconjmul(mu1, OC[i0]).x +
                            cconjmul(AC[i0], ph1).x - cconjmul(AC[i1], ph0).x;
          gF[p] += c0 * t0;
          gF[E::NPTS + p] += c1 * t1;
        }
        for (long long e = e0 + threadIdx.x; e < e1; e += T) {
          psi[e] = csub(cscale(X[e], 2.0), psi[e]);
          lam[e] = csub(cscale(B[e], 2.0), lam[e]);
        }
        touched = true;
        advance();
        break;
      }
      case k2AdjPhiDone:
        request(X, false);
        pc = k2AdjGrad;
        break;
      case k2AdjMuDone:
        rq = LineReq{B, nullptr, nullptr, 0, mk(1.0, 0.0), false, nullptr, false, AR, AC};
        pending = true;
        swap_after = false;
        pc = k2AdjMuAfter;
        break;
      case k2AdjMuAfter: {
        for (long long e = e0 + threadIdx.x; e < e1; e += T) lam[e] = csub(cscale(B[e], 2.0), lam[e]);
        group_signal(hand);
        ++handoffs;
        touched = true;
        advance();
        break;
      }
      case k2AdjGrad: {
        // mu, A_2 mu, A_1 mu from the other group's slots
        if (!group_wait(hand, (handoffs + 1) * (unsigned)G, sy.abort_flag, other_abort, a.spin_limit,
                        c.scal + 15)) {
          aborted = true;
          break;
        }
        const cplx* MU = wk1 + E::VEC;
        const cplx* MR = wk1 + 6 * E::VEC;
        const cplx* MC = wk1 + 7 * E::VEC;
        double* gF = a.gF + im.off;
        const double c1 = -(2.0 * alpha / a.mass1), c0 = -(2.0 * alpha / a.mass0);
        for (long long p = p0 + threadIdx.x; p < p1; p += T) {
          const long long i0 = p, i1 = E::NPTS + p;
          const cplx ph0 = X[i0], ph1 = X[i1], mu0 = MU[i0], mu1 = MU[i1];
          const double t1 = cconjmul(mu0, OR[i1]).x - cconjmul(mu1, OR[i0]).x +
                            cconjmul(MR[i0], ph1).x - cconjmul(MR[i1], ph0).x;
          const double t0 = cconjmul(mu0, OC[i1]).x - cconjmul(mu1, OC[i0]).x +
                            cconjmul(MC[i0], ph1).x - cconjmul(MC[i1], ph0).x;
          gF[p] += c0 * t0;
          gF[E::NPTS + p] += c1 * t1;
        }
        for (long long e = e0 + threadIdx.x; e < e1; e += T) psi[e] = csub(cscale(X[e], 2.0), psi[e]);
        group_signal(hand + 1);
        ++handoffs;
        touched = true;
        advance();
        break;
      }
      case k2ApplyDone: {
        cplx* out = (cplx*)a.aux + im.off;
        for (long long e = e0 + threadIdx.x; e < e1; e += T) out[e] = cadd(OR[e], OC[e]);
        goto done;
      }
      case k2DiagDone: {
        // OR = A_2 psi, OC = A_1 psi
        const double* V = a.V + im.off;
        double q0 = 0.0, q1 = 0.0, pv = 0.0, k2 = 0.0, k1 = 0.0;
        for (long long p = p0 + threadIdx.x; p < p1; p += T) {
          const double a0 = cabs2(psi[p]), a1 = cabs2(psi[E::NPTS + p]);
          q0 += a0;
          q1 += a1;
          pv += V[p] * a0 + V[E::NPTS + p] * a1;
          k2 += cabs2(OR[p]) + cabs2(OR[E::NPTS + p]);
          k1 += cabs2(OC[p]) + cabs2(OC[E::NPTS + p]);
        }
        put_partial(c, 0, q0);
        put_partial(c, 1, q1);
        put_partial(c, 2, pv);
        put_partial(c, 3, k1);
        put_partial(c, 4, k2);
        if (!gsum(5)) break;
        if (g == 0 && threadIdx.x == 0) {
          const double P0 = c.red[0] * im.dv, P1 = c.red[1] * im.dv;
          double* o = a.out + 4 * (size_t)item;
          o[0] = sqrt(P0 + P1);
          o[1] = (c.red[3] * a.inv2m0 + c.red[4] * a.inv2m1 + c.red[2]) * im.dv;
          o[2] = P0;
          o[3] = P1;
        }
        goto done;
      }
      case k2Inner: {
        const cplx* y = (const cplx*)a.aux + im.off;
        double re = 0.0, imv = 0.0;
        for (long long e = e0 + threadIdx.x; e < e1; e += T) {
          const cplx z = cconjmul(psi[e], y[e]);
          re += z.x;
          imv += z.y;
        }
        put_partial(c, 0, re);
        put_partial(c, 1, imv);
        if (!gsum(2)) break;
        if (g == 0 && threadIdx.x == 0) {
          a.out[2 * (size_t)item] = c.red[0] * im.dv;
          a.out[2 * (size_t)item + 1] = c.red[1] * im.dv;
        }
        goto done;
      }
      default:
        bad = true;
        break;
    }
  }
done:
  // a group that stops early releases the other group of its item from any hand-off wait
  if (R == 2 && (bad || aborted) && threadIdx.x == 0)
    __hip_atomic_store(sy.abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (g == 0 && threadIdx.x == 0 && a.stats) {
    ItemStats* st = (role == 0 ? a.stats : a.stats1) + item;
    st->h_applies = napply;
    st->iterations = iters_total;
    st->iterations_sq = iters_sq;
    st->extra_vecs = extra_vecs;
    st->solves = solves;
    st->max_iters = max_iters;
    st->failures = failures;
    st->nonfinite = aborted ? 2 : (bad ? 1 : 0);
    st->max_resid = max_resid;
  }
}

// --------------------------------------------------------------------- launchers

#define GQD_DISPATCH2(cls, EXPR)                     \
  switch (cls) {                                     \
    case 0: { constexpr int NL = 64;  EXPR; } break; \
    case 1: { constexpr int NL = 128; EXPR; } break; \
    case 2: { constexpr int NL = 256; EXPR; } break; \
    case 3: { constexpr int NL = 512; EXPR; } break; \
    default: return hipErrorInvalidValue;            \
  }

hipError_t configure_kernels2d(int m_max) {
  for (int cls = 0; cls < kNumLine2; ++cls) {
    hipError_t e = hipSuccess;
    GQD_DISPATCH2(cls, {
      size_t bytes = lds_bytes2(NL, m_max);
      if (bytes > 160 * 1024) bytes = 160 * 1024;
      e = hipFuncSetAttribute((const void*)k_run2d<NL>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t max_resident2d(int cls, int m, int* blocks) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  GQD_DISPATCH2(cls, {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_run2d<NL>, kThreads2, lds_bytes2(NL, m));
  });
  if (e != hipSuccess) return e;
  *blocks = per * cus;
  return hipSuccess;
}

// The launch is cooperative, so the runtime guarantees that every workgroup is resident.
// GQD_2D_PLAIN_LAUNCH=1 in the environment makes it an ordinary launch of the same grid
// instead, for profilers that fail on cooperative launches: the grid never exceeds the
// resident capacity (run2d sizes it so), so on an otherwise idle GPU every workgroup
// starts at once; if one could not, the waits of the others end at their poll limit and
// the call fails with the barrier time-out.
static bool plain_launch_2d() {
  const char* v = std::getenv("GQD_2D_PLAIN_LAUNCH");
  return v && v[0] == '1' && v[1] == 0;
}

hipError_t launch_run2d(int cls, const K2Args& a, hipStream_t stream) {
  K2Args args = a;
  void* params[] = {&args};
  const bool plain = plain_launch_2d();
  GQD_DISPATCH2(cls, {
    if (plain) {
      hipLaunchKernelGGL(k_run2d<NL>, dim3(a.batch * a.G * a.roles), dim3(kThreads2), lds_bytes2(NL, a.sc.m),
                         stream, args);
      return hipGetLastError();
    }
    return hipLaunchCooperativeKernel((const void*)k_run2d<NL>, dim3(a.batch * a.G * a.roles), dim3(kThreads2), params,
                                      (unsigned)lds_bytes2(NL, a.sc.m), stream);
  });
  return hipSuccess;
}

}  // namespace gqd
