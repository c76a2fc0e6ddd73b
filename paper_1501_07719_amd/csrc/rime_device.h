// Device-side numeric helpers shared by the kernels of librime.so: the
// precision traits of the two arithmetic paths (float64, and float32 with an
// accurate sine/cosine of turns and the gfx950 hardware exp2, reciprocal and
// reciprocal square root), the error-free phase argument, and float64
// compensated (two-sum) accumulation with wavefront and workgroup reductions.
#pragma once

#include "rime_internal.h"

namespace rime {

// ---------------------------------------------------------------------------
// Numeric helpers
// ---------------------------------------------------------------------------

constexpr double kInvTwoPi = 0.15915494309189533576888376337251436;
constexpr double kLog2e = 1.44269504088896340735992468100189214;

// Pointers into the constant address space: loads through them at a
// wavefront-uniform address become scalar (SMEM) loads whose results are
// operands in SGPRs.  Only data written by an earlier kernel is read this way.
// (The host compilation pass parses the device code without address spaces.)
#if defined(__HIP_DEVICE_COMPILE__)
#define RIME_CONST __attribute__((address_space(4)))
#else
#define RIME_CONST
#endif

template <class T>
__device__ inline const RIME_CONST T *const_ptr(const void *p) {
  return (const RIME_CONST T *)(p);  // an address-space cast needs the C form
}

// Plain 4-vector for loads through constant-space pointers (the HIP vector
// types have no copy from that address space); copies merge into one wide
// scalar load.
template <class R>
struct alignas(4 * sizeof(R)) Quad {
  R x, y, z, w;
};

// Returns x unchanged in a VGPR the compiler cannot see through, so that a
// constant folded into x (an LDS region offset) stays in the per-lane base
// address instead of being re-added inside a loop.
__device__ inline uint32_t opaque_vgpr(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The set descriptor of a work item, read through the constant space so that
// its fields are wavefront-uniform (scalar) values.
__device__ inline SetDesc load_set(const KParams &p, int set) {
  if (!p.sets) return p.one;
  const RIME_CONST SetDesc *q = const_ptr<SetDesc>(p.sets) + set;
  SetDesc d;
  d.lm = q->lm;
  d.stokes = q->stokes;
  d.alpha = q->alpha;
  d.gshape = q->gshape;
  d.xshape = q->xshape;
  d.npsrc = q->npsrc;
  d.ngsrc = q->ngsrc;
  d.nxsrc = q->nxsrc;
  d.src_off = q->src_off;
  return d;
}

template <class R> struct Num;

template <> struct Num<double> {
  using R2 = double2;
  using R4 = double4;
  // sin and cos of 2 pi r for r in [-1/2, 1/2] turns.
  __device__ static inline void sincos_turns(double r, double *s, double *c) {
    sincospi(2.0 * r, s, c);
  }
  // expb(y) = exp(y / kExpScale): the exponential in the base whose argument
  // scale is kExpScale (e here, 2 in the float version).
  static constexpr double kExpScale = 1.0;
  __device__ static inline double expb(double y) { return exp(y); }
  // the 32 bits packed into the last word of a per-baseline record
  __device__ static inline uint32_t bits(double w) {
    return static_cast<uint32_t>(__double_as_longlong(w));
  }
  __device__ static inline double from_bits(uint32_t b) {
    return __longlong_as_double(static_cast<long long>(b));
  }
  __device__ static inline double rcp(double x) { return 1.0 / x; }
  __device__ static inline double rsqrt_(double x) { return rsqrt(x); }
};

template <> struct Num<float> {
  using R2 = float2;
  using R4 = float4;
  // sin and cos of 2 pi r for r in [-1/2, 1/2] turns, to about one float32
  // unit: the quarter-turn reduction r = q/4 + x is exact in float64, the
  // angle 2 pi x (|2 pi x| <= pi/4) is rounded once to float32, and the Taylor
  // series of sin to degree 9 and of cos to degree 10 leave truncation errors
  // below 2e-9 there; the quadrant then permutes and negates the pair.  (The
  // hardware v_sin_f32 / v_cos_f32 are several float32 units less accurate,
  // which shows in sums that cancel.)
  __device__ static inline void sincos_turns(double r, float *s, float *c) {
    const double q = rint(4.0 * r);
    const float th = static_cast<float>((r - 0.25 * q) * (2.0 * 3.14159265358979323846));
    const float t2 = th * th;
    const float sn =
        th * (1.0f + t2 * (-1.0f / 6.0f +
                           t2 * (1.0f / 120.0f + t2 * (-1.0f / 5040.0f + t2 * (1.0f / 362880.0f)))));
    const float cs =
        1.0f + t2 * (-0.5f + t2 * (1.0f / 24.0f +
                                   t2 * (-1.0f / 720.0f +
                                         t2 * (1.0f / 40320.0f + t2 * (-1.0f / 3628800.0f)))));
    // sin and cos of th + iq pi/2
    const int iq = static_cast<int>(q) & 3;
    const float ss = (iq & 1) ? cs : sn, cc = (iq & 1) ? sn : cs;
    *s = (iq & 2) ? -ss : ss;
    *c = ((iq + 1) & 2) ? -cc : cc;
  }
  static constexpr double kExpScale = kLog2e;
  __device__ static inline float expb(float y) { return __builtin_amdgcn_exp2f(y); }
  __device__ static inline uint32_t bits(float w) { return __float_as_uint(w); }
  __device__ static inline float from_bits(uint32_t b) { return __uint_as_float(b); }
  __device__ static inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  __device__ static inline float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
};

// Error-free transformations for the phase argument of eq. k_term.  The path
// length tau = u l + v m + w (n - 1) times nu / c spans hundreds to thousands of
// turns on the benchmark arrays; carried as an unevaluated float64 pair
// (hi + lo) through exact products and sums, its fraction of a turn is the
// exact fraction of the products of the float64 inputs to about 1e-16 turns,
// whatever the rounding order of a plain evaluation would have been.
// Every function here turns contraction off: fusing a product into a
// following sum (hipcc contracts by default) would round differently from
// the product that the error term is taken against, and break the identity.

// Error-free sum (Knuth): s + e == a + b exactly.
__device__ inline void two_sum(double a, double b, double &s, double &e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

// Error-free product with one fused multiply-add: p + e == a b exactly.
__device__ inline void two_prod(double a, double b, double &p, double &e) {
#pragma clang fp contract(off)
  p = a * b;
  e = fma(a, b, -p);
}

struct Pair {
  double hi, lo;
};

// tau = u l + v m + w (n - 1) (metres) as hi + lo.
__device__ inline Pair path_length(double u, double v, double w, double l, double m,
                                   double nm1) {
#pragma clang fp contract(off)
  double p1, e1, p2, e2, p3, e3, s, es1, es2;
  two_prod(u, l, p1, e1);
  two_prod(v, m, p2, e2);
  two_prod(w, nm1, p3, e3);
  two_sum(p1, p2, s, es1);
  two_sum(s, p3, s, es2);
  Pair t;
  two_sum(s, (e1 + e2 + e3) + (es1 + es2), t.hi, t.lo);
  return t;
}

// tau nu / c in turns minus its nearest integer (ties to even), in
// [-1/2, 1/2] up to rounding: exp(-2 pi i x) has period 1 in x.
__device__ inline double phase_frac(Pair tau, double nuc) {
#pragma clang fp contract(off)
  double xh, xe;
  two_prod(tau.hi, nuc, xh, xe);
  const double xl = xe + tau.lo * nuc;
  return (xh - rint(xh)) + xl;
}

// The phase argument of one (antenna, source) pair, for its channels.
// EXACT (the float64 path): the error-free pair above.  Otherwise (the
// float32 path) one plain float64 evaluation: at a few thousand turns it is
// within about 1e-12 turns of the exact fraction, four orders of magnitude
// below what a float32 sine and cosine resolve, for a fifth of the work.
template <bool EXACT> struct PhaseArg;

template <> struct PhaseArg<true> {
  Pair tau;
  __device__ inline PhaseArg(double u, double v, double w, double l, double m, double nm1)
      : tau(path_length(u, v, w, l, m, nm1)) {}
  __device__ inline double turns(double nuc) const { return phase_frac(tau, nuc); }
};

template <> struct PhaseArg<false> {
  double tau;
  __device__ inline PhaseArg(double u, double v, double w, double l, double m, double nm1)
      : tau(fma(w, nm1, fma(v, m, u * l))) {}
  __device__ inline double turns(double nuc) const {
    const double x = tau * nuc;
    return x - rint(x);
  }
};

// Beam factors of the float32 path for a beam angle x in [0, beam_clip]
// (the plan accepts beam_clip <= 1.5 rad): e = cos^3(x) and, when wanted,
// tan(x)/x, the factor of d ln e / dl.  With z = x^2, cos x = C(z) and
// sin(x)/x = P(z) are their Taylor series to z^6, whose truncation errors
// stay below 5e-8 relative up to 1.5 rad (below 1e-10 up to 1.0881 rad);
// tan(x)/x = P(z) / C(z) needs no special case at x = 0.
__device__ inline void beam_f32(float x, bool want_tan, float *e, float *tx) {
  const float z = x * x;
  const float c =
      1.0f + z * (-1.0f / 2.0f +
                  z * (1.0f / 24.0f +
                       z * (-1.0f / 720.0f +
                            z * (1.0f / 40320.0f +
                                 z * (-1.0f / 3628800.0f + z * (1.0f / 479001600.0f))))));
  *e = c * c * c;
  if (want_tan) {
    const float sx =
        1.0f + z * (-1.0f / 6.0f +
                    z * (1.0f / 120.0f +
                         z * (-1.0f / 5040.0f +
                              z * (1.0f / 362880.0f +
                                   z * (-1.0f / 39916800.0f + z * (1.0f / 6227020800.0f))))));
    *tx = sx * __builtin_amdgcn_rcpf(c);
  }
}

// a^2 + b^2 with each product rounded on its own (l^2 + m^2 as written).
__device__ inline double sumsq_rn(double a, double b) {
#pragma clang fp contract(off)
  return a * a + b * b;
}

// Compensated float64 accumulator.
struct Comp {
  double s = 0.0, c = 0.0;
  __device__ inline void add(double x) {
    double e;
    two_sum(s, x, s, e);
    c += e;
  }
  __device__ inline void merge(double os, double oc) {
    double e;
    two_sum(s, os, s, e);
    c += oc + e;
  }
};

__device__ inline Comp wave_reduce(Comp v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const double os = __shfl_xor(v.s, off, kWave);
    const double oc = __shfl_xor(v.c, off, kWave);
    v.merge(os, oc);
  }
  return v;
}

// Workgroup reduction of a compensated pair; the result is valid in thread 0.
template <int NT>
__device__ inline Comp block_reduce(Comp v, double2 *scratch) {
  constexpr int NW = NT / kWave;
  v = wave_reduce(v);
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  if (NW == 1) return v;
  __syncthreads();
  if (lane == 0) scratch[wave] = make_double2(v.s, v.c);
  __syncthreads();
  Comp r;
  if (wave == 0) {
    if (lane < NW) {
      r.s = scratch[lane].x;
      r.c = scratch[lane].y;
    }
    r = wave_reduce(r);
  }
  return r;
}

constexpr int nat_for(int nbt) { return nbt >= 1024 ? 64 : nbt >= 256 ? 32 : 16; }

// 2x2 complex matrices in float64, entries (xx, xy, yx, yy) = ([0][0], [0][1],
// [1][0], [1][1]).
struct M22 {
  double re[4], im[4];
};

// a b
__device__ inline M22 m22_mul(const M22 &a, const M22 &b) {
  M22 r;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int x = 2 * i + k, y = 2 * k + j;
        sr += a.re[x] * b.re[y] - a.im[x] * b.im[y];
        si += a.re[x] * b.im[y] + a.im[x] * b.re[y];
      }
      r.re[2 * i + j] = sr;
      r.im[2 * i + j] = si;
    }
  return r;
}

// a^H
__device__ inline M22 m22_herm(const M22 &a) {
  M22 r;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      r.re[2 * i + j] = a.re[2 * j + i];
      r.im[2 * i + j] = -a.im[2 * j + i];
    }
  return r;
}

__device__ inline M22 m22_load(const double2 *m) {
  M22 r;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 v = m[k];
    r.re[k] = v.x;
    r.im[k] = v.y;
  }
  return r;
}

}  // namespace rime
