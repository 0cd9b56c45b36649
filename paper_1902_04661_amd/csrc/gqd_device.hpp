// Device building blocks for the gfx950 path: FP64 complex helpers, small DFT
// butterflies, LDS-staged Stockham passes and workgroup reductions.
//
// Layout used throughout: one workgroup owns one wavepacket (one "item").  A 1D
// item with N grid points has 2 surfaces; thread t of the T = N / R0 threads owns
// the points t + r*T (r < R0) of both surfaces ("owned points").  Pointwise work
// (coupling, potential, Krylov updates, dot products) happens on owned points in
// registers; only the inner passes of the Fourier transforms go through LDS.
#pragma once
#include <hip/hip_runtime.h>

#include "gqd_internal.h"

namespace gqd {

// Address-space qualified pointers: global memory (1) and LDS (3).  Generic pointers
// would compile to flat instructions.
#define GQD_G __attribute__((address_space(1)))
#define GQD_L __attribute__((address_space(3)))

// Complex value: a native two-double vector (loads and stores from any address space
// as one 16-byte access).  Memory layout equals interleaved complex128.
typedef double cplx __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cplx mk(double re, double im) {
  cplx r;
  r.x = re;
  r.y = im;
  return r;
}

// ----------------------------------------------------------------- complex helpers
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return mk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return mk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ cplx cconjmul(cplx a, cplx b) {
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ cplx cscale(cplx a, double s) { return mk(a.x * s, a.y * s); }
// i * s * a
__device__ __forceinline__ cplx cmul_is(cplx a, double s) { return mk(-s * a.y, s * a.x); }
__device__ __forceinline__ double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ cplx cneg(cplx a) { return mk(-a.x, -a.y); }

// ------------------------------------------------------------------- DFT butterflies
// X_k = sum_r x_r exp(S * 2 pi i r k / R), natural order in and out; S = -1 forward.
// Built by radix-2 decimation in time; constant twiddles are cos/sin of multiples of pi/8.
struct TwC {
  static constexpr double C8 = 0.70710678118654752440;   // cos(pi/4)
  static constexpr double C16 = 0.92387953251128675613;  // cos(pi/8)
  static constexpr double S16 = 0.38268343236508977173;  // sin(pi/8)
};

// multiply z by exp(S * 2 pi i K / R) for constant K, R (R <= 16)
template <int R, int S, int K>
__device__ __forceinline__ cplx twc(cplx z) {
  constexpr int k16 = K * (16 / R);  // angle in units of 2 pi / 16, 0..7
  if constexpr (k16 == 0) {
    return z;
  } else if constexpr (k16 == 4) {  // multiply by S*i
    return S > 0 ? mk(-z.y, z.x) : mk(z.y, -z.x);
  } else if constexpr (k16 == 2 || k16 == 6) {
    // (cos, S sin) with cos = +-C8, sin = C8
    constexpr double c = (k16 == 2) ? TwC::C8 : -TwC::C8;
    constexpr double s = S * TwC::C8;
    return mk(c * z.x - s * z.y, c * z.y + s * z.x);
  } else {
    constexpr double c = (k16 == 1) ? TwC::C16 : (k16 == 3) ? TwC::S16 : (k16 == 5) ? -TwC::S16 : -TwC::C16;
    constexpr double s0 = (k16 == 1) ? TwC::S16 : (k16 == 3) ? TwC::C16 : (k16 == 5) ? TwC::C16 : TwC::S16;
    constexpr double s = S * s0;
    return mk(c * z.x - s * z.y, c * z.y + s * z.x);
  }
}

template <int R, int S>
struct DFT {
  template <int K>
  static __device__ __forceinline__ void combine(cplx* x, const cplx* e, const cplx* o) {
    if constexpr (K < R / 2) {
      cplx t = twc<R, S, K>(o[K]);
      x[K] = cadd(e[K], t);
      x[K + R / 2] = csub(e[K], t);
      combine<K + 1>(x, e, o);
    }
  }
  static __device__ __forceinline__ void run(cplx* x) {
    cplx e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    DFT<R / 2, S>::run(e);
    DFT<R / 2, S>::run(o);
    combine<0>(x, e, o);
  }
};
template <int S>
struct DFT<2, S> {
  static __device__ __forceinline__ void run(cplx* x) {
    cplx a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};
template <int S>
struct DFT<1, S> {
  static __device__ __forceinline__ void run(cplx*) {}
};

// Returns p unchanged but opaque to the optimiser, so loads through it cannot be
// hoisted out of the enclosing loop (loop-invariant twiddle and coefficient loads
// would otherwise stay live in registers for the whole kernel).
template <class Tp>
__device__ __forceinline__ GQD_G Tp* opaque(Tp* p) {
  // every pointer passed here is the same in all lanes: broadcast it to a scalar
  // register first (free when the compiler already knows it is uniform)
  const unsigned long long b = reinterpret_cast<unsigned long long>(p);
  unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(b & 0xffffffffull));
  unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi));
  return (GQD_G Tp*)(((unsigned long long)hi << 32) | lo);
}
template <class Tp>
__device__ __forceinline__ GQD_G Tp* opaque(GQD_G Tp* p) {
  return opaque((Tp*)p);
}
// Same for a uniform double and for the lane index: values derived from them
// (addresses, per-lane scale factors) are recomputed where used instead of being
// precomputed once and kept in registers for the whole kernel.
__device__ __forceinline__ double opaque_d(double x) {
  asm volatile("" : "+s"(x));
  return x;
}
// Solve s of an item took `iters` Arnoldi iterations: written to the item's log when
// the host set one (gqd_set_solve_log).  Called by one thread; reads the log pointer
// from the item's statistics record at the time of use, so it holds no register.
__device__ __forceinline__ void log_solve(ItemStats* st, long long s, int iters) {
  if (!st) return;
  const GQD_G ItemStats* p = opaque(st);
  int* lg = p->log;
  if (lg && s < p->log_cap) lg[s] = iters;
}

// A value every lane holds identically, made provably uniform (scalar register).
__device__ __forceinline__ double uniform_d(double x) {
  const unsigned long long b = __double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(b & 0xffffffffull));
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int lane_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// -------------------------------------------------------------------- reductions
template <int T>
struct Block {
  static constexpr int W = (T + 63) / 64;  // waves
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------- GMRES least squares
// The context C holds LDS arrays hcol[m+1] (new Hessenberg column), g[m+1], sn[m],
// cs[m], y[m], R (column j at j(j+1)/2) and scal[16].
//
// Thread 0 applies the stored rotations to the new column, forms the new rotation
// from (column[j], hn), stores column j of R and updates g; scal[0] = |g_(j+1)|.
template <class C>
__device__ void gm_givens(int j, double hn, const C& c) {
  if (threadIdx.x == 0) {
    GQD_L cplx* h = c.hcol;
    for (int i = 0; i < j; ++i) {
      const double ci = c.cs[i];
      const cplx si = c.sn[i];
      const cplx hi = h[i], hi1 = h[i + 1];
      const cplx t = cadd(cscale(hi, ci), cmul(si, hi1));
      h[i + 1] = cadd(cmul(cneg(mk(si.x, -si.y)), hi), cscale(hi1, ci));
      h[i] = t;
    }
    const cplx a = h[j];
    double cj;
    cplx sj, rj;
    if (hn == 0.0) {
      cj = 1.0;
      sj = mk(0.0, 0.0);
      rj = a;
    } else if (a.x == 0.0 && a.y == 0.0) {
      cj = 0.0;
      sj = mk(1.0, 0.0);
      rj = mk(hn, 0.0);
    } else {
      const double absa = hypot(a.x, a.y);
      const double rho = sqrt(absa * absa + hn * hn);
      const cplx ph = mk(a.x / absa, a.y / absa);
      cj = absa / rho;
      sj = cscale(ph, hn / rho);
      rj = cscale(ph, rho);
    }
    c.cs[j] = cj;
    c.sn[j] = sj;
    GQD_L cplx* Rj = c.R + (j * (j + 1)) / 2;
    for (int i = 0; i < j; ++i) Rj[i] = h[i];
    Rj[j] = rj;
    const cplx gj = c.g[j];
    c.g[j + 1] = cmul(cneg(mk(sj.x, -sj.y)), gj);
    c.g[j] = cscale(gj, cj);
    c.scal[0] = hypot(c.g[j + 1].x, c.g[j + 1].y);
  }
  __syncthreads();
}

// Thread 0: y = R^-1 g (upper triangular, k columns).
template <class C>
__device__ void gm_back_solve(int k, const C& c) {
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      cplx s = mk(0.0, 0.0);
      for (int l = i + 1; l < k; ++l) s = cadd(s, cmul(c.R[(l * (l + 1)) / 2 + i], c.y[l]));
      const cplx num = csub(c.g[i], s);
      const cplx d = c.R[(i * (i + 1)) / 2 + i];
      const double dd = d.x * d.x + d.y * d.y;
      c.y[i] = mk((num.x * d.x + num.y * d.y) / dd, (num.y * d.x - num.x * d.y) / dd);
    }
  }
  __syncthreads();
}

}  // namespace gqd
