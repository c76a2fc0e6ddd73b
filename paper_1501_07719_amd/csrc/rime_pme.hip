// Matrix-core engine for the point sources of one sky in the float32-mixed
// path (gfx950 MFMA, fp16 inputs, float32 accumulation).
//
// For a point source with no baseline-dependent factor, the source-summed
// coherency of eq. 1 factors over the two antennas of a baseline:
//   S_k[p][q] = sum_s a_ps conj(a_qs) St'_sk,   a_ps = e_ps K_ps,
// i.e. for every (timestep, channel) the four Stokes sums of all baselines
// form the antenna x antenna matrix product A diag(St'_k) A^H.  This file
// evaluates that product, and the corresponding part of the adjoint, on the
// matrix cores:
//   pme_phase    a_ps for every (t, nu, s, p), split into fp16 hi + lo parts
//                (22 significant bits; the phase argument is formed and
//                reduced in float64 as in the float32 per-baseline kernels),
//                and the beam's d ln e / d(l, m) factor;
//   pme_scale    per (channel, Stokes parameter) power-of-two scale of the
//                source-side operand;
//   pme_forward  one Q block of 32 antennas against one or two P blocks per
//                workgroup, one Stokes parameter per wavefront: the real form
//                of the product over (s, re/im) with v_mfma_f32_32x32x16_f16,
//                each fp16 product taken as hi*hi + hi*lo + lo*hi, summed in
//                float32 over 128 sources and in float64 beyond.  The float64
//                Stokes sums of every antenna pair go to HBM, where the
//                per-baseline kernel adds them to the sums of the remaining
//                (Gaussian) sources before forming V and chi^2;
//   pme_mfrag    the residual matrices of the adjoint as fp16 MFMA fragments;
//   pme_adjoint  the gradient of chi^2 with respect to the point-source
//                parameters (see the comment there);
//   pme_fin_items, pme_finalize
//                float64 sums of the adjoint's per-workgroup partials.
// Operand fragments follow the gfx950 lane layout of the 32x32x16 fp16
// instruction: A[i][k] in lane i + 32 (k / 8), element k % 8; B[k][j] in lane
// j + 32 (k / 8), element k % 8; D[i][j] in lane j + 32 ((i / 4) % 2),
// register (i % 4) + 4 (i / 8).
#include "rime_device.h"

namespace rime {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kPmeCh = 32;                 // sources per staged chunk
constexpr int kPmeRow = 2 * kPmeCh + 8;    // fp16 per LDS row: (s, re/im) + 16 B pad
constexpr int kPmeFold = 4;                // chunks summed in float32 before a float64 fold

__device__ inline uint32_t pack_h2(_Float16 re, _Float16 im) {
  return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, re)) |
         (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, im)) << 16);
}

__device__ inline float lo_h(uint32_t w) {
  return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w & 0xffffu)));
}
__device__ inline float hi_h(uint32_t w) {
  return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w >> 16)));
}

// x = h + l with h = fp16(x) and l = fp16(x - h).
__device__ inline void split_h(float x, _Float16 &h, _Float16 &l) {
  h = static_cast<_Float16>(x);
  l = static_cast<_Float16>(x - static_cast<float>(h));
}

// (x0, x1) = h + l as two fp16 pairs.  The hi pair is materialised once, so
// that the lo pair is taken against the very values the products use
// (otherwise the compiler may form the packed hi pair and the hi value the lo
// part is taken against with different conversions, which differ by an ulp
// when the product is rounded once rather than twice).
__device__ inline void split_h2(float x0, float x1, uint32_t &h, uint32_t &l) {
  typedef _Float16 half2v __attribute__((ext_vector_type(2)));
  const half2v hv = {static_cast<_Float16>(x0), static_cast<_Float16>(x1)};
  h = opaque_vgpr(__builtin_bit_cast(uint32_t, hv));
  const half2v lv = {static_cast<_Float16>(x0 - lo_h(h)), static_cast<_Float16>(x1 - hi_h(h))};
  l = __builtin_bit_cast(uint32_t, lv);
}

// fp16 pair (re, im) -> (-im, re): with b in the B operand of the real form
// of a complex product, the column of the imaginary part of a conj(b)
__device__ inline uint32_t rot_h2(uint32_t w) { return ((w >> 16) | (w << 16)) ^ 0x8000u; }

// (re, im) -> (im, -re) on the four pairs of a fragment: with a in the A
// operand, the row of the imaginary part of a conj(b) (the adjoint's residual
// fragments; they do not change over the sources of a channel, and hipcc
// keeps the rotated copies in registers across the source loop)
__device__ inline half8 rot8(half8 v) {
  half8 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    r[2 * e] = v[2 * e + 1];
    r[2 * e + 1] = -v[2 * e];
  }
  return r;
}

// Workgroups are dealt round-robin to the 8 XCDs; renumbering them makes
// consecutive work items (which share operands through L2) land on one XCD.
__device__ inline int xcd_item(int nitems) {
  const int per_xcd = (nitems + 7) / 8;
  return static_cast<int>(blockIdx.x % 8) * per_xcd + static_cast<int>(blockIdx.x / 8);
}

// ---------------------------------------------------------------------------
// Phase planes: thread = (source, antenna) of one timestep and one block of
// p.phase_nc channels, reusing the float64 phase argument tau and the beam
// radius over the block.  Workgroups are dispatched with the (source, antenna)
// index fastest, so the ones in flight write the few planes of one (timestep,
// channel block) at a time.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void pme_phase(const KParams p) {
  using N = Num<float>;
  const SetDesc sd = p.one;
  const int tt = blockIdx.y;
  const int t = p.pme_t0 + tt;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int nap = p.nap;
  const int64_t plane = static_cast<int64_t>(sd.npsrc) * nap;
  if (idx >= plane) return;
  const int cb = blockIdx.z * p.phase_nc;
  const int ce = min(p.nchan, cb + p.phase_nc);
  const int s = static_cast<int>(idx / nap);
  const int a = static_cast<int>(idx - static_cast<int64_t>(s) * nap);
  const int64_t o = static_cast<int64_t>(tt) * p.nchan * plane + idx;
  uint32_t *hi = p.ph_hi + o;
  uint32_t *lo = p.ph_lo + o;
  float *k3p = p.ph_k3 ? p.ph_k3 + o : nullptr;
  if (a >= p.na) {
    for (int c = cb; c < ce; ++c) {
      hi[c * plane] = 0u;
      lo[c * plane] = 0u;
      if (k3p) k3p[c * plane] = 0.0f;
    }
    return;
  }
  const double4 g = p.src_geo[sd.src_off + s];
  const double *x = p.uvw + (static_cast<int64_t>(t) * p.na + a) * 3;
  // tau = u l + v m + w (n - 1), metres (eq. k_term), in float64 to well
  // below the resolution of the float32 sine and cosine
  const PhaseArg<false> tau(x[0], x[1], x[2], g.x, g.y, g.z);
  double r2b = 0.0, rb = 0.0;
  if (p.beam) {
    const double *q = p.pointing + (static_cast<int64_t>(t) * p.na + a) * 2;
    r2b = sumsq_rn(g.x - q[0], g.y - q[1]);
    rb = sqrt(r2b);
  }
  for (int c = cb; c < ce; ++c) {
    const double r = tau.turns(p.nu_c[c]);
    float sn, cs;
    N::sincos_turns(r, &sn, &cs);
    float e = 1.0f, k3 = 0.0f;
    if (p.beam) {
      // cos^3 of beam_k r nu / beam_ref_freq, clipped (eq. e_term); the clip
      // is decided in float64 on r^2 as in the per-baseline kernels
      const double bs = p.bsc[c];
      const bool clipped = r2b >= p.clip_r2[c];
      const double xd = clipped ? p.beam_clip : bs * rb;
      float tx = 0.0f;
      beam_f32(static_cast<float>(xd), k3p != nullptr, &e, &tx);
      // d ln e / dl = -3 bs^2 (l - dl_p) tan(x)/x; zero past the clip
      if (!clipped) k3 = static_cast<float>(p.bk3[c]) * tx;
    }
    _Float16 rh, rl, ih, il;
    split_h(e * cs, rh, rl);
    split_h(-e * sn, ih, il);
    hi[c * plane] = pack_h2(rh, ih);
    lo[c * plane] = pack_h2(rl, il);
    if (k3p) k3p[c * plane] = k3;
  }
}

// St'_k (k = I, Q, U, V) of source s of the set at channel c and timestep t:
// the spectrally scaled Stokes vector, or, with brightness per timestep (ST),
// the spectral factor times that timestep's Stokes vector (rounded as in the
// per-baseline kernels).  The kernels that call it per chunk take ST as a
// template parameter, so that the plain calls do not carry its registers.
template <bool ST>
__device__ inline float4 pme_stokes(const KParams &p, int s, int c, int t) {
  const int64_t gs = p.one.src_off + s;
  if (ST) {
    const int nsrc = p.one.npsrc + p.one.ngsrc + p.one.nxsrc;
    const double *q = p.stokes_t + (static_cast<int64_t>(t) * nsrc + s) * 4;
    const double f = static_cast<double>(static_cast<const float *>(p.src_sf)[gs * p.nchan + c]);
    return make_float4(static_cast<float>(f * q[0]), static_cast<float>(f * q[1]),
                       static_cast<float>(f * q[2]), static_cast<float>(f * q[3]));
  }
  return static_cast<const float4 *>(p.src_st)[gs * p.nchan + c];
}

// ---------------------------------------------------------------------------
// Forward scale: exponent e of max_s |St'_k,s(nu)| (over the timesteps too with
// brightness per timestep), one workgroup per channel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pme_scale(const KParams p) {
  __shared__ float s_m[4][256 / kWave];
  const int c = blockIdx.x;
  const SetDesc sd = p.one;
  const int nt = p.stokes_t ? p.ntime : 1;
  float m[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int t = 0; t < nt; ++t)
    for (int s = threadIdx.x; s < sd.npsrc; s += 256) {
      const float4 v = p.stokes_t ? pme_stokes<true>(p, s, c, t) : pme_stokes<false>(p, s, c, t);
      m[0] = fmaxf(m[0], fabsf(v.x));
      m[1] = fmaxf(m[1], fabsf(v.y));
      m[2] = fmaxf(m[2], fabsf(v.z));
      m[3] = fmaxf(m[3], fabsf(v.w));
    }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m[k] = fmaxf(m[k], __shfl_xor(m[k], off, kWave));
    if (threadIdx.x % kWave == 0) s_m[k][threadIdx.x / kWave] = m[k];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    const float mm = fmaxf(fmaxf(s_m[k][0], s_m[k][1]), fmaxf(s_m[k][2], s_m[k][3]));
    int e = 0;
    if (mm > 0.0f) frexpf(mm, &e);
    p.pme_exp[c * 4 + k] = e;
  }
}

// ---------------------------------------------------------------------------
// Forward: workgroup = (timestep, channel, group of one Q block and NT P
// blocks); wavefront k accumulates S_k of the group's tiles (P, Q).  The P
// side is the plain a as fp16 hi/lo fragments from LDS.  The Q side carries
// St'_k 2^-e(nu, k): each wavefront forms it for its own k from a float32 copy
// of the Q block's a in LDS and splits it in registers, together with its
// rotation (re, im) -> (-im, re), which gives the imaginary part of the
// product; the tiles of a group share the two.  NT = 2 halves that work per
// tile but holds the float64 sums of two tiles (two workgroups per CU);
// NT = 1 runs three workgroups per CU, so that one's products overlap
// another's operand work.  The plan pairs the tiles of a Q block when the
// array has more than three antenna blocks: with fewer, half of the groups
// would hold one tile (64 antennas, 100 timesteps, 64 channels: 2.40 ms with
// NT = 1 against 2.70 ms; 197 antennas, 20 timesteps, 256 channels: 24.3 ms
// against 23.1 ms).
// ---------------------------------------------------------------------------
struct FwdRegs {
  uint4 pah, pal, pbh, pbl, qh, ql;
  float4 st;
};

constexpr int kPmeQRow = 2 * kPmeCh + 4;  // floats per LDS row of the Q block: (s, re/im) + 16 B pad

// Global operands of one chunk for thread (source tid / 8, antennas 4 (tid % 8) ..)
// at channel c and timestep t.
template <bool ST, int NT>
__device__ inline FwdRegs fwd_load(const KParams &p, const uint32_t *hi0, const uint32_t *lo0,
                                   int c, int t, int s0, int cnt, int Q, int Pa, int Pb) {
  const int tid = threadIdx.x;
  const int s = tid >> 3, ag = (tid & 7) * 4;
  FwdRegs r;
  r.pah = r.pal = r.pbh = r.pbl = r.qh = r.ql = make_uint4(0, 0, 0, 0);
  r.st = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (s < cnt) {
    // a P block equal to the Q block (a diagonal tile) reuses the Q operands
    const int64_t row = static_cast<int64_t>(s0 + s) * p.nap;
    r.qh = *reinterpret_cast<const uint4 *>(hi0 + row + Q * kPmeBlk + ag);
    r.ql = *reinterpret_cast<const uint4 *>(lo0 + row + Q * kPmeBlk + ag);
    if (Pa == Q) {
      r.pah = r.qh;
      r.pal = r.ql;
    } else {
      r.pah = *reinterpret_cast<const uint4 *>(hi0 + row + Pa * kPmeBlk + ag);
      r.pal = *reinterpret_cast<const uint4 *>(lo0 + row + Pa * kPmeBlk + ag);
    }
    if (NT == 2) {
      if (Pb == Q) {
        r.pbh = r.qh;
        r.pbl = r.ql;
      } else if (Pb >= 0) {
        r.pbh = *reinterpret_cast<const uint4 *>(hi0 + row + Pb * kPmeBlk + ag);
        r.pbl = *reinterpret_cast<const uint4 *>(lo0 + row + Pb * kPmeBlk + ag);
      }
    }
    r.st = pme_stokes<ST>(p, s0 + s, c, t);
  }
  return r;
}

template <bool ST, int NT>
__global__ __launch_bounds__(256, NT == 1 ? 3 : 2) void pme_forward(const KParams p) {
  const int nitems = p.pme_nt * p.nchan * p.ngroup;
  const int item = xcd_item(nitems);
  if (item >= nitems) return;
  const int grp = item % p.ngroup;
  const int rest = item / p.ngroup;
  const int c = rest % p.nchan;
  const int tt = rest / p.nchan;

  // [P block a/b][antenna][(s, re/im)] as fp16 hi/lo; the Q block's a in
  // float32; the scaled Stokes parameters [k][s]
  __shared__ __attribute__((aligned(16))) _Float16 s_ah[NT][kPmeBlk][kPmeRow];
  __shared__ __attribute__((aligned(16))) _Float16 s_al[NT][kPmeBlk][kPmeRow];
  __shared__ __attribute__((aligned(16))) float s_qf[kPmeBlk][kPmeQRow];
  __shared__ __attribute__((aligned(16))) float s_f[4][kPmeCh];

  const SetDesc sd = p.one;
  const int *gr = p.groups + grp * 5;
  const int Q = gr[0], Pa = gr[1], Pb = NT == 2 ? gr[2] : -1, ida = gr[3], idb = gr[4];
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid % kWave;
  const int k = wave;  // Stokes parameter of this wavefront
  const int row = lane & 31, g = lane >> 5;

  const int64_t plane = static_cast<int64_t>(sd.npsrc) * p.nap;
  const uint32_t *hi0 = p.ph_hi + (static_cast<int64_t>(tt) * p.nchan + c) * plane;
  const uint32_t *lo0 = p.ph_lo + (static_cast<int64_t>(tt) * p.nchan + c) * plane;
  // St'_k 2^-e(nu, k): |scaled| < 1
  float fsc[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) fsc[kk] = ldexpf(1.0f, -p.pme_exp[c * 4 + kk]);
  const double unscale = ldexp(1.0, p.pme_exp[c * 4 + k]);

  floatx16 aR[NT], aI[NT];
  double dR[NT][16], dI[NT][16];
#pragma unroll
  for (int x = 0; x < NT; ++x)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      aR[x][r] = aI[x][r] = 0.0f;
      dR[x][r] = dI[x][r] = 0.0;
    }

  const int nchunk = (sd.npsrc + kPmeCh - 1) / kPmeCh;
  for (int ch = 0; ch < nchunk; ++ch) {
    const FwdRegs cur = fwd_load<ST, NT>(p, hi0, lo0, c, p.pme_t0 + tt, ch * kPmeCh,
                                         min(kPmeCh, sd.npsrc - ch * kPmeCh), Q, Pa, Pb);
    __syncthreads();  // the previous chunk's operands are consumed
    {
      const int s = tid >> 3, ag = (tid & 7) * 4;
      const uint32_t w0[4] = {cur.pah.x, cur.pah.y, cur.pah.z, cur.pah.w};
      const uint32_t w1[4] = {cur.pal.x, cur.pal.y, cur.pal.z, cur.pal.w};
      const uint32_t w2[4] = {cur.pbh.x, cur.pbh.y, cur.pbh.z, cur.pbh.w};
      const uint32_t w3[4] = {cur.pbl.x, cur.pbl.y, cur.pbl.z, cur.pbl.w};
      const uint32_t wq[4] = {cur.qh.x, cur.qh.y, cur.qh.z, cur.qh.w};
      const uint32_t wl[4] = {cur.ql.x, cur.ql.y, cur.ql.z, cur.ql.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        *reinterpret_cast<uint32_t *>(&s_ah[0][ag + j][2 * s]) = w0[j];
        *reinterpret_cast<uint32_t *>(&s_al[0][ag + j][2 * s]) = w1[j];
        if (NT == 2 && Pb >= 0) {
          *reinterpret_cast<uint32_t *>(&s_ah[NT - 1][ag + j][2 * s]) = w2[j];
          *reinterpret_cast<uint32_t *>(&s_al[NT - 1][ag + j][2 * s]) = w3[j];
        }
        // a = hi + lo exactly in float32
        *reinterpret_cast<float2 *>(&s_qf[ag + j][2 * s]) =
            make_float2(lo_h(wq[j]) + lo_h(wl[j]), hi_h(wq[j]) + hi_h(wl[j]));
      }
      if ((tid & 7) == 0) {
        s_f[0][s] = cur.st.x * fsc[0];
        s_f[1][s] = cur.st.y * fsc[1];
        s_f[2][s] = cur.st.z * fsc[2];
        s_f[3][s] = cur.st.w * fsc[3];
      }
    }
    __syncthreads();
#pragma unroll
    for (int step = 0; step < kPmeCh / 8; ++step) {
      // K index (s, re/im) with s = 8 step + 4 g + e / 2 for element e
      const int col = 16 * step + 8 * g;
      half8 bh, bl, rbh, rbl;
      {
        const float4 q0 = *reinterpret_cast<const float4 *>(&s_qf[row][col]);
        const float4 q1 = *reinterpret_cast<const float4 *>(&s_qf[row][col + 4]);
        const float4 f = *reinterpret_cast<const float4 *>(&s_f[k][8 * step + 4 * g]);
        uint32_t hw[4], lw[4];
        split_h2(q0.x * f.x, q0.y * f.x, hw[0], lw[0]);
        split_h2(q0.z * f.y, q0.w * f.y, hw[1], lw[1]);
        split_h2(q1.x * f.z, q1.y * f.z, hw[2], lw[2]);
        split_h2(q1.z * f.w, q1.w * f.w, hw[3], lw[3]);
        bh = __builtin_bit_cast(half8, make_uint4(hw[0], hw[1], hw[2], hw[3]));
        bl = __builtin_bit_cast(half8, make_uint4(lw[0], lw[1], lw[2], lw[3]));
        rbh = __builtin_bit_cast(half8,
                                 make_uint4(rot_h2(hw[0]), rot_h2(hw[1]), rot_h2(hw[2]), rot_h2(hw[3])));
        rbl = __builtin_bit_cast(half8,
                                 make_uint4(rot_h2(lw[0]), rot_h2(lw[1]), rot_h2(lw[2]), rot_h2(lw[3])));
      }
#pragma unroll
      for (int x = 0; x < NT; ++x) {
        if (x == 1 && Pb < 0) break;
        const half8 ah = *reinterpret_cast<const half8 *>(&s_ah[x][row][col]);
        const half8 al = *reinterpret_cast<const half8 *>(&s_al[x][row][col]);
        aR[x] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, aR[x], 0, 0, 0);
        aI[x] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, rbh, aI[x], 0, 0, 0);
        aR[x] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, aR[x], 0, 0, 0);
        aI[x] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, rbl, aI[x], 0, 0, 0);
        aR[x] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, aR[x], 0, 0, 0);
        aI[x] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, rbh, aI[x], 0, 0, 0);
      }
    }
    if ((ch + 1) % kPmeFold == 0 || ch + 1 == nchunk) {
#pragma unroll
      for (int x = 0; x < NT; ++x)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          dR[x][r] += static_cast<double>(aR[x][r]) * unscale;
          dI[x][r] += static_cast<double>(aI[x][r]) * unscale;
          aR[x][r] = aI[x][r] = 0.0f;
        }
    }
  }

  // Stokes sums S_k[i][j] of antennas (32 P + i, 32 Q + j)
  const int64_t slice = (static_cast<int64_t>(p.pme_t0) + tt) * p.nchan + c;
  const int j = lane & 31;
#pragma unroll
  for (int x = 0; x < NT; ++x) {
    if (x == 1 && Pb < 0) break;
    double2 *out =
        p.spts + ((slice * p.npair + (x == 0 ? ida : idb)) * 4 + k) * (kPmeBlk * kPmeBlk);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = (r & 3) + 8 * (r >> 2) + 4 * g;
      out[i * kPmeBlk + j] = make_double2(dR[x][r], dI[x][r]);
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the point sources.  With the weighted residual in Stokes form
// rho_k of every baseline stored in its antenna-pair slot T (rho, or its
// conjugate for a baseline stored as (q, p)), the Hermitian matrix
// M_k = T_k + T_k^H has M_k[p][q] = rho_k for the baseline (p, q) and
// conj(rho_k) for (q, p).  With Z_k = M_k conj(A) (antennas x sources) and
// c_pq = a_p conj(a_q), summing over the baselines (p < q):
//   sum Re(c rho_k)                   = 1/2 sum_p Re(a_ps Z_k[p][s])
//   sum (u_p - u_q) Im(c rho_k)       = sum_p u_p Im(a_ps Z_k[p][s])  (v, w alike)
//   sum (beta_p + beta_q) Re(c rho_k) = sum_p beta_ps Re(a_ps Z_k[p][s])
// and P = c sum_k St'_k rho_k combines the four k with weights St'_k, so the
// per-baseline adjoint's source sums follow from Z_k by reductions over the
// antennas p.  Workgroup = (source range, timestep, kPmeNCW channels,
// antenna block P, kPmeNQ blocks of q); wavefront k holds the fp16 hi/lo
// fragments of rows (p in P, re/im) of M_k for the q range (scaled by a power
// of two so that max |M| < 1) and streams 32-source chunks of A as the B
// operand.
// ---------------------------------------------------------------------------
constexpr int kPmeBRow = 2 * kPmeBlk * kPmeNQ + 8;  // fp16 per B row: (q, re/im) + pad

// Fragments of M_k (rows of block P, columns of the q range) for one
// (timestep, channel): workgroup = (timestep, channel, P, q range),
// wavefront = k.  Element e of K-step st of lane (row, g) is (q, re/im) with
// q = 8 st + 4 g + e / 2 local to the range.  Each wavefront copies the
// residual tile of one q block at a time into LDS with contiguous 16-byte
// loads (slots that hold no baseline read as zero), so that the row-wise and
// the transposed reads of the fragment layout come from LDS.
__global__ __launch_bounds__(256) void pme_mfrag(const KParams p) {
  __shared__ float s_gmax[4];
  __shared__ float2 s_t[4][kPmeBlk][kPmeBlk + 1];  // [k][i][j], one q block at a time
  const int nP = p.nblk, nQR = p.pme_nqr;
  const int item = blockIdx.x;  // ((tt * nchan + c) * nP + P) * nQR + qr
  int rest = item;
  const int qr = rest % nQR;
  rest /= nQR;
  const int P = rest % nP;
  rest /= nP;
  const int c = rest % p.nchan;
  const int tt = rest / p.nchan;
  const int t = p.pme_t0 + tt;
  const int Q0 = qr * kPmeNQ;
  const int nq = min(kPmeNQ, nP - Q0);
  const int tid = threadIdx.x;
  const int k = tid / kWave, lane = tid % kWave;
  const int row = lane & 31, g = lane >> 5;
  const int64_t base =
      ((static_cast<int64_t>(t) * p.nchan + c) * p.npair * 4 + k) * (kPmeBlk * kPmeBlk);
  float2 m[kPmeNQ * 4][4];
  float mx = 0.0f;
#pragma unroll
  for (int b = 0; b < kPmeNQ; ++b) {
    const int qb = Q0 + b;
    const int pr = b < nq ? p.pair_of[min(P, qb) * nP + max(P, qb)] : -1;
    const float4 *src = reinterpret_cast<const float4 *>(
        p.rho_t + base + static_cast<int64_t>(max(pr, 0)) * 4 * kPmeBlk * kPmeBlk);
#pragma unroll
    for (int it = 0; it < kPmeBlk * kPmeBlk / 2 / kWave; ++it) {
      const int idx = it * kWave + lane;  // float4 index: row i, columns j, j + 1
      const int i = idx / (kPmeBlk / 2), j = (idx % (kPmeBlk / 2)) * 2;
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      uint32_t msk = 0u;
      if (pr >= 0) {
        v = src[idx];
        msk = p.pair_mask[pr * kPmeBlk + i] >> j;
      }
      s_t[k][i][j] = (msk & 1u) ? make_float2(v.x, v.y) : make_float2(0.0f, 0.0f);
      s_t[k][i][j + 1] = (msk & 2u) ? make_float2(v.z, v.w) : make_float2(0.0f, 0.0f);
    }
    __syncthreads();
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      const int st = 4 * b + sb;
      const int j0 = 8 * sb + 4 * g;  // q = 8 st + 4 g + e lies in block b at column j0 + e
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = j0 + e;
        float2 v = make_float2(0.0f, 0.0f);
        if (st < nq * 4) {
          if (qb == P) {
            // T + T^H on the diagonal block
            const float2 x = s_t[k][row][j];
            const float2 y = s_t[k][j][row];
            v = make_float2(x.x + y.x, x.y - y.y);
          } else if (P < qb) {
            v = s_t[k][row][j];
          } else {
            // the tile is stored as (qb, P): conjugate transpose
            const float2 y = s_t[k][j][row];
            v = make_float2(y.x, -y.y);
          }
        }
        m[st][e] = v;
        mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
      }
    }
    __syncthreads();  // the tile is consumed before the next one is staged
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
  if (lane == 0) s_gmax[k] = mx;
  __syncthreads();
  const float gmax = fmaxf(fmaxf(s_gmax[0], s_gmax[1]), fmaxf(s_gmax[2], s_gmax[3]));
  int ex = 0;
  if (gmax > 0.0f) frexpf(gmax, &ex);
  const float scl = ldexpf(1.0f, -ex);
  if (tid == 0) p.mscale[item] = gmax > 0.0f ? ldexpf(1.0f, ex) : 0.0f;
  uint4 *dst = p.mfrag + ((static_cast<int64_t>(item) * 4 + k) * (kPmeNQ * 4) * kWave) * 2;
#pragma unroll
  for (int st = 0; st < kPmeNQ * 4; ++st) {
    if (st < nq * 4) {
      uint32_t hw[4], lw[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        _Float16 rh, rl, ih, il;
        split_h(m[st][e].x * scl, rh, rl);
        split_h(m[st][e].y * scl, ih, il);
        hw[e] = pack_h2(rh, ih);
        lw[e] = pack_h2(rl, il);
      }
      dst[(st * kWave + lane) * 2] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      dst[(st * kWave + lane) * 2 + 1] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
  }
}

template <bool ST>
__global__ __launch_bounds__(256, 2) void pme_adjoint(const KParams p) {
  const int nP = p.nblk, nQR = p.pme_nqr, nCG = p.pme_ncg, nT = p.pme_nt;
  const int nitems = p.pme_nsr * nT * nCG * nP * nQR;
  const int item = xcd_item(nitems);
  if (item >= nitems) return;
  int rest = item;
  const int qr = rest % nQR;
  rest /= nQR;
  const int P = rest % nP;
  rest /= nP;
  const int cg = rest % nCG;
  rest /= nCG;
  const int tt = rest % nT;
  const int sr = rest / nT;
  const int t = p.pme_t0 + tt;
  const int Q0 = qr * kPmeNQ;
  const int nq = min(kPmeNQ, nP - Q0);
  const SetDesc sd = p.one;
  const int sbeg = sr * kPmeSR;
  const int send = min(sd.npsrc, sbeg + kPmeSR);

  __shared__ __attribute__((aligned(16))) _Float16 s_bh[kPmeCh][kPmeBRow];
  __shared__ __attribute__((aligned(16))) _Float16 s_bl[kPmeCh][kPmeBRow];
  __shared__ float2 s_ap[kPmeBlk][kPmeCh + 1];  // a of block P (float32)
  __shared__ float s_betl[kPmeBlk][kPmeCh + 1];  // beta_l = k3 (l - dl_p)
  __shared__ float s_betm[kPmeBlk][kPmeCh + 1];  // beta_m = k3 (m - dm_p)
  __shared__ float s_out[4][kPmeCh][6];          // per k: G, u, v, w, beam l, beam m
  __shared__ float s_src[kPmeCh][8];             // St'(nu) I..V, l/n, m/n, (nu/nu_ref)^alpha
  __shared__ float s_acc[kPmeSR][7];
  __shared__ float s_uvw[kPmeBlk][3];
  __shared__ double s_pnt[kPmeBlk][2];

  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid % kWave;
  const int k = wave;
  const int row = lane & 31, g = lane >> 5;
  const int64_t plane = static_cast<int64_t>(sd.npsrc) * p.nap;
  const bool p_in_range = P >= Q0 && P < Q0 + nq;

  for (int i = tid; i < kPmeSR * 7; i += 256) (&s_acc[0][0])[i] = 0.0f;
  if (tid < kPmeBlk) {
    const int a = P * kPmeBlk + tid;
    float u = 0.0f, v = 0.0f, w = 0.0f;
    double pl = 0.0, pm = 0.0;
    if (a < p.na) {
      const double *x = p.uvw + (static_cast<int64_t>(t) * p.na + a) * 3;
      u = static_cast<float>(x[0]);
      v = static_cast<float>(x[1]);
      w = static_cast<float>(x[2]);
      if (p.beam) {
        const double *q = p.pointing + (static_cast<int64_t>(t) * p.na + a) * 2;
        pl = q[0];
        pm = q[1];
      }
    }
    s_uvw[tid][0] = u;
    s_uvw[tid][1] = v;
    s_uvw[tid][2] = w;
    s_pnt[tid][0] = pl;
    s_pnt[tid][1] = pm;
  }

  for (int ci = 0; ci < kPmeNCW; ++ci) {
    const int c = cg * kPmeNCW + ci;
    if (c >= p.nchan) break;
    const int64_t fitem = ((static_cast<int64_t>(tt) * p.nchan + c) * nP + P) * nQR + qr;
    const float unscl = p.mscale[fitem];
    if (unscl == 0.0f) continue;  // the residual of this block row is zero
    half8 mh[kPmeNQ * 4], ml[kPmeNQ * 4];
    {
      const uint4 *src = p.mfrag + ((fitem * 4 + k) * (kPmeNQ * 4) * kWave) * 2;
#pragma unroll
      for (int st = 0; st < kPmeNQ * 4; ++st) {
        uint4 h = make_uint4(0, 0, 0, 0), l = h;
        if (st < nq * 4) {
          h = src[(st * kWave + lane) * 2];
          l = src[(st * kWave + lane) * 2 + 1];
        }
        mh[st] = __builtin_bit_cast(half8, h);
        ml[st] = __builtin_bit_cast(half8, l);
      }
    }
    const uint32_t *hi0 = p.ph_hi + (static_cast<int64_t>(tt) * p.nchan + c) * plane;
    const uint32_t *lo0 = p.ph_lo + (static_cast<int64_t>(tt) * p.nchan + c) * plane;
    const float *k30 =
        p.beam ? p.ph_k3 + (static_cast<int64_t>(tt) * p.nchan + c) * plane : nullptr;
    const float tpnc = static_cast<float>(2.0 * kPi * p.nu_c[c]);
    const float lnfr = static_cast<float>(p.lnfr[c]);

    for (int s0 = sbeg; s0 < send; s0 += kPmeCh) {
      const int cnt = min(kPmeCh, send - s0);
      __syncthreads();  // LDS of the previous chunk is consumed
      {
        // B operand rows: a of the q range for 32 sources; block P in float32
        const int s = tid >> 3, part = tid & 7;
        uint4 h0 = make_uint4(0, 0, 0, 0), h1 = h0, l0 = h0, l1 = h0;
        uint4 ph = h0, pl = h0;
        float4 k3 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        double sl = 0.0, sm = 0.0;
        if (s < cnt) {
          const int64_t rowoff = static_cast<int64_t>(s0 + s) * p.nap;
          const int q0 = Q0 * kPmeBlk + part * 8;  // 8 antennas per thread
          if (q0 < (Q0 + nq) * kPmeBlk) {
            h0 = *reinterpret_cast<const uint4 *>(hi0 + rowoff + q0);
            h1 = *reinterpret_cast<const uint4 *>(hi0 + rowoff + q0 + 4);
            l0 = *reinterpret_cast<const uint4 *>(lo0 + rowoff + q0);
            l1 = *reinterpret_cast<const uint4 *>(lo0 + rowoff + q0 + 4);
          }
          if (!p_in_range) {
            ph = *reinterpret_cast<const uint4 *>(hi0 + rowoff + P * kPmeBlk + part * 4);
            pl = *reinterpret_cast<const uint4 *>(lo0 + rowoff + P * kPmeBlk + part * 4);
          }
          if (k30) {
            k3 = *reinterpret_cast<const float4 *>(k30 + rowoff + P * kPmeBlk + part * 4);
            const double4 geo = p.src_geo[sd.src_off + s0 + s];
            sl = geo.x;
            sm = geo.y;
          }
        }
        if (part == 0) {
          // per-source factors of the assembly below
          float4 sv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          double2 lo = make_double2(0.0, 0.0);
          float f = 0.0f;
          if (s < cnt) {
            const int64_t gs = sd.src_off + s0 + s;
            sv = pme_stokes<ST>(p, s0 + s, c, t);
            lo = p.src_lon[gs];
            f = p.src_f[gs * p.nchan + c];
          }
          s_src[s][0] = sv.x;
          s_src[s][1] = sv.y;
          s_src[s][2] = sv.z;
          s_src[s][3] = sv.w;
          s_src[s][4] = static_cast<float>(lo.x);
          s_src[s][5] = static_cast<float>(lo.y);
          s_src[s][6] = f;
        }
        uint4 *bh = reinterpret_cast<uint4 *>(&s_bh[s][part * 16]);
        uint4 *bl = reinterpret_cast<uint4 *>(&s_bl[s][part * 16]);
        bh[0] = h0;
        bh[1] = h1;
        bl[0] = l0;
        bl[1] = l1;
        const float k3v[4] = {k3.x, k3.y, k3.z, k3.w};
        if (p_in_range) {
          // block P is part of the q range: a from the words just loaded
          const int a0 = Q0 * kPmeBlk + part * 8 - P * kPmeBlk;  // first antenna, local to P
          if (a0 >= 0 && a0 < kPmeBlk) {
            const uint32_t hw[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
            const uint32_t lw[8] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w};
#pragma unroll
            for (int j = 0; j < 8; ++j)
              s_ap[a0 + j][s] =
                  make_float2(lo_h(hw[j]) + lo_h(lw[j]), hi_h(hw[j]) + hi_h(lw[j]));
          }
        } else {
          const uint32_t phw[4] = {ph.x, ph.y, ph.z, ph.w}, plw[4] = {pl.x, pl.y, pl.z, pl.w};
#pragma unroll
          for (int j = 0; j < 4; ++j)
            s_ap[part * 4 + j][s] =
                make_float2(lo_h(phw[j]) + lo_h(plw[j]), hi_h(phw[j]) + hi_h(plw[j]));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = part * 4 + j;
          s_betl[i][s] = k3v[j] * static_cast<float>(sl - s_pnt[i][0]);
          s_betm[i][s] = k3v[j] * static_cast<float>(sm - s_pnt[i][1]);
        }
      }
      __syncthreads();
      floatx16 accR, accI;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accR[r] = 0.0f;
        accI[r] = 0.0f;
      }
#pragma unroll
      for (int st = 0; st < kPmeNQ * 4; ++st) {
        if (st < nq * 4) {
          const int col = 16 * st + 8 * g;
          const half8 bh = *reinterpret_cast<const half8 *>(&s_bh[row][col]);
          const half8 bl = *reinterpret_cast<const half8 *>(&s_bl[row][col]);
          const half8 rh = rot8(mh[st]), rl = rot8(ml[st]);
          accR = __builtin_amdgcn_mfma_f32_32x32x16_f16(mh[st], bh, accR, 0, 0, 0);
          accI = __builtin_amdgcn_mfma_f32_32x32x16_f16(rh, bh, accI, 0, 0, 0);
          accR = __builtin_amdgcn_mfma_f32_32x32x16_f16(mh[st], bl, accR, 0, 0, 0);
          accI = __builtin_amdgcn_mfma_f32_32x32x16_f16(rh, bl, accI, 0, 0, 0);
          accR = __builtin_amdgcn_mfma_f32_32x32x16_f16(ml[st], bh, accR, 0, 0, 0);
          accI = __builtin_amdgcn_mfma_f32_32x32x16_f16(rl, bh, accI, 0, 0, 0);
        }
      }
      // reductions of a_ps Z_k[p][s] over this lane's 16 antennas p --------
      {
        float o[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = (r & 3) + 8 * (r >> 2) + 4 * g;
          const float2 a = s_ap[i][row];
          const float wr = a.x * accR[r] - a.y * accI[r];
          const float wi = a.x * accI[r] + a.y * accR[r];
          o[0] += wr;
          o[1] += s_uvw[i][0] * wi;
          o[2] += s_uvw[i][1] * wi;
          o[3] += s_uvw[i][2] * wi;
          o[4] += s_betl[i][row] * wr;
          o[5] += s_betm[i][row] * wr;
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) o[j] += __shfl_xor(o[j], 32, kWave);
        if (g == 0) {
#pragma unroll
          for (int j = 0; j < 6; ++j) s_out[k][row][j] = o[j];
        }
      }
      __syncthreads();
      if (tid < cnt) {
        const int s = tid;
        const float stv[4] = {s_src[s][0], s_src[s][1], s_src[s][2], s_src[s][3]};
        float G[4], h[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          G[kk] = 0.5f * unscl * s_out[kk][s][0];
#pragma unroll
          for (int j = 0; j < 5; ++j) h[j] += stv[kk] * s_out[kk][s][1 + j];
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) h[j] *= unscl;
        // h = (sum u Im W, sum v Im W, sum w Im W, sum beta_l Re W, sum beta_m Re W)
        const float lon = s_src[s][4], mon = s_src[s][5], f = s_src[s][6];
        float *acc = s_acc[s0 + s - sbeg];
        acc[0] += h[3] + tpnc * (h[0] - lon * h[2]);
        acc[1] += h[4] + tpnc * (h[1] - mon * h[2]);
        acc[2] += G[0] * f;
        acc[3] += G[1] * f;
        acc[4] += G[2] * f;
        acc[5] += G[3] * f;
        acc[6] += (stv[0] * G[0] + stv[1] * G[1] + stv[2] * G[2] + stv[3] * G[3]) * lnfr;
      }
    }
  }
  __syncthreads();
  // partials [sr][t][cg][P][qr][kPmeSR][7]
  float *dst = p.pgrad +
               ((((static_cast<int64_t>(sr) * p.ntime + t) * nCG + cg) * nP + P) * nQR + qr) *
                   (kPmeSR * 7);
  for (int i = tid; i < (send - sbeg) * 7; i += 256) dst[i] = (&s_acc[0][0])[i];
}

// Point-source gradient rows from the adjoint partials, in two float64 passes
// with a fixed order.  pme_fin_items: thread = one column (source, component)
// of the partial rows, workgroup = 256 contiguous columns of one source range
// and one chunk of items, so every item row is read as one contiguous 1 KiB
// run.  pme_finalize: thread = (source, gradient column), summing the chunks;
// columns 7..9 (shape) are zero.
__global__ __launch_bounds__(256) void pme_fin_items(const KParams p) {
  constexpr int kRow = kPmeSR * 7;
  const int sr = blockIdx.y, ch = blockIdx.z;
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= min(kPmeSR, p.one.npsrc - sr * kPmeSR) * 7) return;
  const int64_t nper = static_cast<int64_t>(p.ntime) * p.pme_ncg * p.nblk * p.pme_nqr;
  const int64_t cs = (nper + p.pme_fchunk - 1) / p.pme_fchunk;
  const int64_t i1 = min(nper, (ch + 1) * cs);
  const float *src = p.pgrad + static_cast<int64_t>(sr) * nper * kRow + col;
  Comp acc;
  int64_t i = ch * cs;
  for (; i + 4 <= i1; i += 4) {
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = src[(i + k) * kRow];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.add(static_cast<double>(v[k]));
  }
  for (; i < i1; ++i) acc.add(static_cast<double>(src[i * kRow]));
  p.pfin[(static_cast<int64_t>(sr) * p.pme_fchunk + ch) * kRow + col] = make_double2(acc.s, acc.c);
}

__global__ __launch_bounds__(256) void pme_finalize(const KParams p) {
  constexpr int kRow = kPmeSR * 7;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= static_cast<int64_t>(p.one.npsrc) * 10) return;
  const int s = static_cast<int>(idx / 10), j = static_cast<int>(idx % 10);
  double out = 0.0;
  if (j < 7) {
    const int sr = s / kPmeSR, sl = s % kPmeSR;
    const double2 *src = p.pfin + static_cast<int64_t>(sr) * p.pme_fchunk * kRow + sl * 7 + j;
    Comp r;
    for (int ch = 0; ch < p.pme_fchunk; ++ch) {
      const double2 v = src[static_cast<int64_t>(ch) * kRow];
      r.merge(v.x, v.y);
    }
    out = 2.0 * (r.s + r.c);
  }
  p.grad_out[p.one.src_off * 10 + idx] = out;
}

// ---------------------------------------------------------------------------
// Launchers (timesteps [p.pme_t0, p.pme_t0 + p.pme_nt))
// ---------------------------------------------------------------------------
static hipError_t launch_phase(const KParams &p, hipStream_t stream) {
  const int64_t plane = static_cast<int64_t>(p.one.npsrc) * p.nap;
  // channels per workgroup, as measured.  Planes of 1 MiB and more write
  // fastest in blocks of 4 channels: for 1500 sources x 224 antennas, 20
  // timesteps and 256 channels with the beam, 4.2 ms, against 5.8 ms with 16
  // and 7.8 ms with all 256.  Smaller planes write fastest in blocks of 16:
  // for 1000 x 64, 100 timesteps and 64 channels, 0.61 ms against 0.70 ms.
  KParams q = p;
  q.phase_nc = plane * static_cast<int64_t>(sizeof(uint32_t)) >= (int64_t(1) << 20) ? 4 : 16;
  dim3 g1(static_cast<unsigned>((plane + 255) / 256), static_cast<unsigned>(p.pme_nt),
          static_cast<unsigned>((p.nchan + q.phase_nc - 1) / q.phase_nc));
  hipLaunchKernelGGL(pme_phase, g1, dim3(256), 0, stream, q);
  return hipGetLastError();
}

hipError_t launch_pme_scale(const KParams &p, hipStream_t stream) {
  if (p.one.npsrc <= 0) return hipSuccess;
  hipLaunchKernelGGL(pme_scale, dim3(p.nchan), dim3(256), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_pme(const KParams &p, hipStream_t stream) {
  if (p.one.npsrc <= 0 || p.pme_nt <= 0) return hipSuccess;
  hipError_t e = launch_phase(p, stream);
  if (e != hipSuccess) return e;
  const int64_t nitems = static_cast<int64_t>(p.pme_nt) * p.nchan * p.ngroup;
  const int64_t grid = 8 * ((nitems + 7) / 8);
  const dim3 gd(static_cast<unsigned>(grid)), bd(256);
  if (p.pme_pairs) {
    if (p.stokes_t)
      hipLaunchKernelGGL((pme_forward<true, 2>), gd, bd, 0, stream, p);
    else
      hipLaunchKernelGGL((pme_forward<false, 2>), gd, bd, 0, stream, p);
  } else {
    if (p.stokes_t)
      hipLaunchKernelGGL((pme_forward<true, 1>), gd, bd, 0, stream, p);
    else
      hipLaunchKernelGGL((pme_forward<false, 1>), gd, bd, 0, stream, p);
  }
  return hipGetLastError();
}

hipError_t launch_pme_adjoint(const KParams &p, bool phase, hipStream_t stream) {
  if (p.one.npsrc <= 0 || p.pme_nt <= 0) return hipSuccess;
  hipError_t e = phase ? launch_phase(p, stream) : hipSuccess;
  if (e != hipSuccess) return e;
  const int64_t nfrag = static_cast<int64_t>(p.pme_nt) * p.nchan * p.nblk * p.pme_nqr;
  hipLaunchKernelGGL(pme_mfrag, dim3(static_cast<unsigned>(nfrag)), dim3(256), 0, stream, p);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t nitems =
      static_cast<int64_t>(p.pme_nsr) * p.pme_nt * p.pme_ncg * p.nblk * p.pme_nqr;
  const int64_t grid = 8 * ((nitems + 7) / 8);
  if (p.stokes_t)
    hipLaunchKernelGGL(pme_adjoint<true>, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream,
                       p);
  else
    hipLaunchKernelGGL(pme_adjoint<false>, dim3(static_cast<unsigned>(grid)), dim3(256), 0,
                       stream, p);
  return hipGetLastError();
}

hipError_t launch_pme_finalize(const KParams &p, hipStream_t stream) {
  if (p.one.npsrc <= 0) return hipSuccess;
  const dim3 g1(kPmeSR * 7 / 256, static_cast<unsigned>(p.pme_nsr),
                static_cast<unsigned>(p.pme_fchunk));
  hipLaunchKernelGGL(pme_fin_items, g1, dim3(256), 0, stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = static_cast<int64_t>(p.one.npsrc) * 10;
  hipLaunchKernelGGL(pme_finalize, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     stream, p);
  return hipGetLastError();
}

}  // namespace rime
