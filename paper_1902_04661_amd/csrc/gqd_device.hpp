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

// ------------------------------------------------------------------------ FFT plans
// Stockham passes of radices (R0, R1, R2[, R3]) with product N and T = N / R0 threads.
// Every pass has 2N/R butterflies (two surfaces), a whole multiple of T, and T is a
// whole number of 64-lane waves.  R3 = 1 means a three-pass plan.
template <int N> struct Plan;
template <> struct Plan<256>  { static constexpr int R0 = 4, R1 = 8, R2 = 8, R3 = 1; };
template <> struct Plan<512>  { static constexpr int R0 = 4, R1 = 8, R2 = 4, R3 = 4; };
template <> struct Plan<1024> { static constexpr int R0 = 4, R1 = 8, R2 = 8, R3 = 4; };
template <> struct Plan<2048> { static constexpr int R0 = 4, R1 = 8, R2 = 8, R3 = 8; };
template <> struct Plan<4096> { static constexpr int R0 = 8, R1 = 8, R2 = 8, R3 = 8; };

constexpr int TW_N = 4096;  // twiddle table: exp(-2 pi i k / 4096), k < 4096

// Twiddle exp(S * 2 pi i * num / den) for den | TW_N, from the table.
template <int S>
__device__ __forceinline__ cplx tw_lookup(const GQD_G cplx* __restrict__ tw, int idx4096) {
  cplx w = tw[idx4096];
  return S < 0 ? w : mk(w.x, -w.y);
}

// One in-place Stockham pass over 2 sequences of length N in LDS (seq s at lds[s*N]).
// Butterfly j (< N/R) of sequence s reads x[j + r N/R], twiddles by w_{Ns R}^{r k}
// (k = j mod Ns), applies the radix-R DFT and writes y[(j/Ns) Ns R + k + r Ns].
template <int N, int T, int R, int Ns, int S>
__device__ __forceinline__ void stockham_lds(GQD_L cplx* lds, const GQD_G cplx* __restrict__ tw) {
  constexpr int NB = 2 * N / R;
  static_assert(NB % T == 0, "butterflies must be a multiple of the thread count");
  constexpr int PER = NB / T;
  cplx x[PER][R];
  int tid = lane_tid();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * T;
    const int s = b / (N / R), j = b % (N / R);
#pragma unroll
    for (int r = 0; r < R; ++r) x[q][r] = lds[s * N + j + r * (N / R)];
  }
  __syncthreads();
  tid = lane_tid();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * T;
    const int s = b / (N / R), j = b % (N / R);
    const int k = j % Ns;
    if constexpr (Ns > 1) {
      constexpr int step = TW_N / (Ns * R);
#pragma unroll
      for (int r = 1; r < R; ++r) x[q][r] = cmul(x[q][r], tw_lookup<S>(tw, r * k * step));
    }
    DFT<R, S>::run(x[q]);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) lds[s * N + base + r * Ns] = x[q][r];
  }
  __syncthreads();
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

}  // namespace gqd
