// Device-side numeric helpers shared by the kernels of librime.so: the
// precision traits of the two arithmetic paths (float64, and float32 with the
// gfx950 hardware transcendentals), definition-order products for the phase
// argument, and float64 compensated (two-sum) accumulation with wavefront and
// workgroup reductions.
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
  d.npsrc = q->npsrc;
  d.ngsrc = q->ngsrc;
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
  // sin and cos of x radians, |x| <= 1.1.
  __device__ static inline void sincos_rad(double x, double *s, double *c) { sincos(x, s, c); }
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
  __device__ static inline double sqrt_(double x) { return sqrt(x); }
  __device__ static inline double rcp(double x) { return 1.0 / x; }
};

template <> struct Num<float> {
  using R2 = float2;
  using R4 = float4;
  // v_sin_f32 / v_cos_f32 take the angle in turns.
  __device__ static inline void sincos_turns(double r, float *s, float *c) {
    const float rf = static_cast<float>(r);
    *s = __builtin_amdgcn_sinf(rf);
    *c = __builtin_amdgcn_cosf(rf);
  }
  __device__ static inline void sincos_rad(float x, float *s, float *c) {
    const float t = x * static_cast<float>(kInvTwoPi);
    *s = __builtin_amdgcn_sinf(t);
    *c = __builtin_amdgcn_cosf(t);
  }
  static constexpr double kExpScale = kLog2e;
  __device__ static inline float expb(float y) { return __builtin_amdgcn_exp2f(y); }
  __device__ static inline uint32_t bits(float w) { return __float_as_uint(w); }
  __device__ static inline float from_bits(uint32_t b) { return __uint_as_float(b); }
  __device__ static inline float sqrt_(double x) {
    return __builtin_amdgcn_sqrtf(static_cast<float>(x));
  }
  __device__ static inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
};

// (a0 b0 + a1 b1) + a2 b2 with every product and sum rounded separately (no
// fused multiply-add), i.e. in the order in which the definitions are written.
// The phase argument is hundreds of turns, so the rounding of this sum is
// visible in the phase; evaluating it in definition order keeps the FP64 path
// rounding-compatible with a plain evaluation of the same formula.
__device__ inline double dot3_rn(double a0, double b0, double a1, double b1, double a2,
                                 double b2) {
#pragma clang fp contract(off)
  return (a0 * b0 + a1 * b1) + a2 * b2;
}

__device__ inline double sumsq_rn(double a, double b) {
#pragma clang fp contract(off)
  return a * a + b * b;
}

// Error-free sum: s + e == a + b exactly.
__device__ inline void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
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

}  // namespace rime
