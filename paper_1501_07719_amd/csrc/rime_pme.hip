// Matrix-core engine for the point sources of one sky in the float32-mixed
// path (gfx950 MFMA, fp16 inputs, float32 accumulation).
//
// For a point source with no baseline-dependent factor, the source-summed
// coherency of eq. 1 factors over the two antennas of a baseline:
//   S_k[p][q] = sum_s a_ps conj(a_qs) St'_sk,   a_ps = e_ps K_ps,
// i.e. for every (timestep, channel) the four Stokes sums of all baselines
// form the antenna x antenna matrix product A diag(St'_k) A^H.  This file
// evaluates that product on the matrix cores:
//   pme_phase   a_ps for every (t, nu, s, p), split into fp16 hi + lo parts
//               (22 significant bits; the phase argument is reduced in
//               float64 exactly as in the per-baseline kernels);
//   pme_forward one 32 x 32 antenna tile (P, Q) per workgroup, one Stokes
//               parameter per wavefront: the real product over (s, re/im)
//               with v_mfma_f32_32x32x16_f16, each fp16 product taken as
//               hi*hi + hi*lo + lo*hi, summed in float32 within a chunk of 32
//               sources and in float64 across chunks.  The result (float64
//               Stokes sums of every antenna pair of the tile) goes to HBM,
//               where the per-baseline kernel adds it to the sums of the
//               remaining (Gaussian) sources before forming V and chi^2;
//   pme_adjoint the gradient of chi^2 with respect to the point-source
//               parameters from the weighted residual that the per-baseline
//               kernel leaves in the antenna-pair slots, as the product
//               (T + T^H) conj(A) on the matrix cores followed by per-source
//               reductions over the antennas (see the comment there);
//   pme_finalize float64 sums of the adjoint's per-workgroup partials.
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

// (re, im) -> (im, -re) on a packed fp16 pair: the row of the imaginary part
// of a conj(b) in the real form of the complex product.
__device__ inline uint32_t rot_h2(uint32_t w) { return (w >> 16) | ((w ^ 0x8000u) << 16); }

// ---------------------------------------------------------------------------
// Phase planes: thread = (source, antenna) of one timestep; loops over the
// channels reusing the float64 phase argument tau and the beam radius.
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
  const int s = static_cast<int>(idx / nap);
  const int a = static_cast<int>(idx - static_cast<int64_t>(s) * nap);
  uint32_t *hi = p.ph_hi + static_cast<int64_t>(tt) * p.nchan * plane + idx;
  uint32_t *lo = p.ph_lo + static_cast<int64_t>(tt) * p.nchan * plane + idx;
  if (a >= p.na) {
    for (int c = 0; c < p.nchan; ++c) {
      hi[c * plane] = 0u;
      lo[c * plane] = 0u;
    }
    return;
  }
  const double4 g = p.src_geo[sd.src_off + s];
  const double *x = p.uvw + (static_cast<int64_t>(t) * p.na + a) * 3;
  // tau = u l + v m + w (n - 1), metres (eq. k_term)
  const double tau = dot3_rn(x[0], g.x, x[1], g.y, x[2], g.z);
  double r2b = 0.0;
  float rb = 0.0f;
  if (p.beam) {
    const double *q = p.pointing + (static_cast<int64_t>(t) * p.na + a) * 2;
    r2b = sumsq_rn(g.x - q[0], g.y - q[1]);
    rb = N::sqrt_(r2b);
  }
  for (int c = 0; c < p.nchan; ++c) {
    const double xt = tau * p.nu_c[c];
    const double r = xt - rint(xt);
    float sn, cs;
    N::sincos_turns(r, &sn, &cs);
    float e = 1.0f;
    if (p.beam) {
      // cos^3 of beam_k r nu / beam_ref_freq, clipped (eq. e_term); the clip
      // is decided in float64 on r^2 as in the per-baseline kernels
      const double bs = p.beam_k * p.bfr[c];
      const bool clipped = r2b >= p.clip_r2[c];
      const float xr = clipped ? static_cast<float>(p.beam_clip) : static_cast<float>(bs) * rb;
      float sb, cb;
      N::sincos_rad(xr, &sb, &cb);
      e = cb * cb * cb;
    }
    _Float16 rh, rl, ih, il;
    split_h(e * cs, rh, rl);
    split_h(-e * sn, ih, il);
    hi[c * plane] = pack_h2(rh, ih);
    lo[c * plane] = pack_h2(rl, il);
  }
}

// ---------------------------------------------------------------------------
// Antenna-pair product for one (timestep, channel, tile pair).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pme_forward(const KParams p) {
  // Workgroups are dealt round-robin to the 8 XCDs; renumber them so that
  // the tile pairs of one (timestep, channel) share an XCD and its L2.
  const int nitems = p.pme_nt * p.nchan * p.npair;
  const int per_xcd = (nitems + 7) / 8;
  const int item = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (item >= nitems) return;
  const int pair = item % p.npair;
  const int rest = item / p.npair;
  const int c = rest % p.nchan;
  const int tt = rest / p.nchan;

  __shared__ __attribute__((aligned(16))) _Float16 s_ah[kPmeBlk][kPmeRow];
  __shared__ __attribute__((aligned(16))) _Float16 s_al[kPmeBlk][kPmeRow];
  __shared__ __attribute__((aligned(16))) _Float16 s_rh[kPmeBlk][kPmeRow];
  __shared__ __attribute__((aligned(16))) _Float16 s_rl[kPmeBlk][kPmeRow];
  __shared__ __attribute__((aligned(16))) _Float16 s_bh[4][kPmeBlk][kPmeRow];
  __shared__ __attribute__((aligned(16))) _Float16 s_bl[4][kPmeBlk][kPmeRow];
  __shared__ float s_st[4][kPmeCh];
  __shared__ float s_scale[4];

  const SetDesc sd = p.one;
  const int2 pq = p.pair_blk[pair];
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid % kWave;
  const int k = wave;  // Stokes parameter of this wavefront

  const int64_t plane = static_cast<int64_t>(sd.npsrc) * p.nap;
  const uint32_t *hi0 = p.ph_hi + (static_cast<int64_t>(tt) * p.nchan + c) * plane;
  const uint32_t *lo0 = p.ph_lo + (static_cast<int64_t>(tt) * p.nchan + c) * plane;
  const float4 *st = static_cast<const float4 *>(p.src_st);

  floatx16 accR, accI;
  double dR[16], dI[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    accR[r] = 0.0f;
    accI[r] = 0.0f;
    dR[r] = 0.0;
    dI[r] = 0.0;
  }

  const int nchunk = (sd.npsrc + kPmeCh - 1) / kPmeCh;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int s0 = ch * kPmeCh;
    const int cnt = min(kPmeCh, sd.npsrc - s0);
    __syncthreads();  // previous chunk's fragments are consumed
    if (tid < kPmeCh) {
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (tid < cnt) v = st[(sd.src_off + s0 + tid) * p.nchan + c];
      s_st[0][tid] = v.x;
      s_st[1][tid] = v.y;
      s_st[2][tid] = v.z;
      s_st[3][tid] = v.w;
    }
    __syncthreads();
    // per-chunk power-of-two scale of Stokes parameter k: max |St'_k| -> [1/2, 1)
    if (lane < kPmeCh) {
      float m = fabsf(s_st[k][lane]);
#pragma unroll
      for (int off = kPmeCh / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
      if (lane == 0) {
        int e = 0;
        if (m > 0.0f) frexpf(m, &e);
        s_scale[k] = ldexpf(1.0f, -e);
      }
    }
    __syncthreads();
    {
      // staging: thread = (source, 4 antennas) of both antenna blocks
      const int s = tid >> 3, ag = (tid & 7) * 4;
      uint4 ph = make_uint4(0, 0, 0, 0), pl = ph, qh = ph, ql = ph;
      if (s < cnt) {
        const int64_t row = static_cast<int64_t>(s0 + s) * p.nap;
        ph = *reinterpret_cast<const uint4 *>(hi0 + row + pq.x * kPmeBlk + ag);
        pl = *reinterpret_cast<const uint4 *>(lo0 + row + pq.x * kPmeBlk + ag);
        qh = *reinterpret_cast<const uint4 *>(hi0 + row + pq.y * kPmeBlk + ag);
        ql = *reinterpret_cast<const uint4 *>(lo0 + row + pq.y * kPmeBlk + ag);
      }
      const uint32_t phw[4] = {ph.x, ph.y, ph.z, ph.w}, plw[4] = {pl.x, pl.y, pl.z, pl.w};
      const uint32_t qhw[4] = {qh.x, qh.y, qh.z, qh.w}, qlw[4] = {ql.x, ql.y, ql.z, ql.w};
      float f[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) f[kk] = s_st[kk][s] * s_scale[kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        *reinterpret_cast<uint32_t *>(&s_ah[ag + j][2 * s]) = phw[j];
        *reinterpret_cast<uint32_t *>(&s_al[ag + j][2 * s]) = plw[j];
        *reinterpret_cast<uint32_t *>(&s_rh[ag + j][2 * s]) = rot_h2(phw[j]);
        *reinterpret_cast<uint32_t *>(&s_rl[ag + j][2 * s]) = rot_h2(plw[j]);
        const float ar = lo_h(qhw[j]) + lo_h(qlw[j]);
        const float ai = hi_h(qhw[j]) + hi_h(qlw[j]);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          _Float16 rh, rl, ih, il;
          split_h(ar * f[kk], rh, rl);
          split_h(ai * f[kk], ih, il);
          *reinterpret_cast<uint32_t *>(&s_bh[kk][ag + j][2 * s]) = pack_h2(rh, ih);
          *reinterpret_cast<uint32_t *>(&s_bl[kk][ag + j][2 * s]) = pack_h2(rl, il);
        }
      }
    }
    __syncthreads();
    {
      const int row = lane & 31, g = lane >> 5;
#pragma unroll
      for (int step = 0; step < kPmeCh / 8; ++step) {
        // K index (s, re/im) with s = 8 step + 4 g + e / 2 for element e
        const int col = 16 * step + 8 * g;
        const half8 ah = *reinterpret_cast<const half8 *>(&s_ah[row][col]);
        const half8 al = *reinterpret_cast<const half8 *>(&s_al[row][col]);
        const half8 rh = *reinterpret_cast<const half8 *>(&s_rh[row][col]);
        const half8 rl = *reinterpret_cast<const half8 *>(&s_rl[row][col]);
        const half8 bh = *reinterpret_cast<const half8 *>(&s_bh[k][row][col]);
        const half8 bl = *reinterpret_cast<const half8 *>(&s_bl[k][row][col]);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_f16(rh, bh, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_f16(rh, bl, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_f16(rl, bh, accI, 0, 0, 0);
      }
      // fold the chunk into float64, undoing its scale
      const double inv = 1.0 / static_cast<double>(s_scale[k]);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        dR[r] += static_cast<double>(accR[r]) * inv;
        dI[r] += static_cast<double>(accI[r]) * inv;
        accR[r] = 0.0f;
        accI[r] = 0.0f;
      }
    }
  }

  // Stokes sums S_k[i][j] of antennas (32 P + i, 32 Q + j)
  double2 *out = p.spts +
                 ((((static_cast<int64_t>(p.pme_t0) + tt) * p.nchan + c) * p.npair + pair) * 4 + k) *
                     (kPmeBlk * kPmeBlk);
  const int j = lane & 31;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
    out[i * kPmeBlk + j] = make_double2(dR[r], dI[r]);
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the point sources.  With the weighted residual in Stokes form
// rho_k of every baseline stored in its antenna-pair slot T (rho, or its
// conjugate for a baseline stored as (q, p)), the Hermitian matrix
// M_k = T_k + T_k^H has M_k[p][q] = rho_k for the baseline (p, q) and
// conj(rho_k) for (q, p).  Then, with Z_k = M_k conj(A) (antennas x sources):
//   sum_{p<q} Re(c_pq rho_k)            = 1/2 sum_p Re(a_ps Z_k[p][s])
//   W_ps = a_ps sum_k St'_k Z_k[p][s]   sums P = c sum_k St'_k rho_k over
//                                       the baselines of antenna p, so that
//   sum_{p<q} (u_p - u_q) Im P          = sum_p u_p Im W_ps   (v, w alike)
//   sum_{p<q} (beta_p + beta_q) Re P    = sum_p beta_ps Re W_ps
// which are the per-source sums of the per-baseline adjoint.  Workgroup =
// (source range, timestep, kPmeNCW channels, antenna block P, kPmeNQ blocks
// of q); wavefront k holds the fp16 hi/lo fragments of rows (p in P, re/im)
// of M_k (scaled by a power of two per channel so that max |M| < 1) for the
// whole q range and streams 32-source chunks of A as the B operand.
// ---------------------------------------------------------------------------
constexpr int kPmeBRow = 2 * kPmeBlk * kPmeNQ + 8;  // fp16 per B row: (q, re/im) + pad

__device__ inline float2 rho_at(const KParams &p, int64_t base, int pair, int i, int j) {
  if (pair < 0) return make_float2(0.0f, 0.0f);
  if (!((p.pair_mask[pair * kPmeBlk + i] >> j) & 1u)) return make_float2(0.0f, 0.0f);
  return p.rho_t[base + static_cast<int64_t>(pair) * 4 * kPmeBlk * kPmeBlk + i * kPmeBlk + j];
}

__global__ __launch_bounds__(256, 2) void pme_adjoint(const KParams p) {
  using N = Num<float>;
  const int nP = p.nblk, nQR = p.pme_nqr, nCG = p.pme_ncg, nT = p.pme_nt;
  const int nitems = p.pme_nsr * nT * nCG * nP * nQR;
  const int per_xcd = (nitems + 7) / 8;
  const int item = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
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
  __shared__ float2 s_ap[kPmeBlk][kPmeCh + 1];
  __shared__ float2 s_w[kPmeBlk][kPmeCh + 1];
  __shared__ float s_g[4][kPmeCh];
  __shared__ float s_red[4][kPmeCh][5];
  __shared__ float s_acc[kPmeSR][7];
  __shared__ float s_uvw[kPmeBlk][3];
  __shared__ double s_pnt[kPmeBlk][2];
  __shared__ float s_gmax[4];

  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid % kWave;
  const int k = wave;
  const int row = lane & 31, g = lane >> 5;
  const int64_t plane = static_cast<int64_t>(sd.npsrc) * p.nap;

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
    // ---- fragments of M_k for rows (32 P + row) and the q range ------------
    const int64_t base = ((static_cast<int64_t>(t) * p.nchan + c) * p.npair * 4 + k) *
                         (kPmeBlk * kPmeBlk);
    // base + pair * 4 * 1024 addresses T_k of that pair
    // M_k[32 P + row][q] for the four q of element group e of K-step st
    auto fetch = [&](int st, int e) -> float2 {
      const int ql = 8 * st + 4 * g;  // first of four q (local to the range)
      const int qb = Q0 + ql / kPmeBlk;
      const int j = ql % kPmeBlk + e;
      if (qb == P) {
        const int pr = p.pair_of[P * nP + P];
        const float2 a = rho_at(p, base, pr, row, j);
        const float2 b = rho_at(p, base, pr, j, row);
        return make_float2(a.x + b.x, a.y - b.y);
      }
      if (P < qb) return rho_at(p, base, p.pair_of[P * nP + qb], row, j);
      const float2 b = rho_at(p, base, p.pair_of[qb * nP + P], j, row);
      return make_float2(b.x, -b.y);
    };
    float mx = 0.0f;
    for (int st = 0; st < nq * 4; ++st) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float2 v = fetch(st, e);
        mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
      }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
    __syncthreads();  // previous channel's s_gmax readers are done
    if (lane == 0) s_gmax[wave] = mx;
    __syncthreads();
    const float gmax = fmaxf(fmaxf(s_gmax[0], s_gmax[1]), fmaxf(s_gmax[2], s_gmax[3]));
    if (gmax == 0.0f) continue;  // uniform across the workgroup
    int ex = 0;
    frexpf(gmax, &ex);
    const float scl = ldexpf(1.0f, -ex);
    const float unscl = ldexpf(1.0f, ex);
    half8 mh[kPmeNQ * 4], ml[kPmeNQ * 4];
#pragma unroll
    for (int st = 0; st < kPmeNQ * 4; ++st) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float2 v = make_float2(0.0f, 0.0f);
        if (st < nq * 4) v = fetch(st, e);
        _Float16 rh, rl, ih, il;
        split_h(v.x * scl, rh, rl);
        split_h(v.y * scl, ih, il);
        mh[st][2 * e] = rh;
        mh[st][2 * e + 1] = ih;
        ml[st][2 * e] = rl;
        ml[st][2 * e + 1] = il;
      }
    }
    const uint32_t *hi0 = p.ph_hi + (static_cast<int64_t>(tt) * p.nchan + c) * plane;
    const uint32_t *lo0 = p.ph_lo + (static_cast<int64_t>(tt) * p.nchan + c) * plane;
    const float4 *stk = static_cast<const float4 *>(p.src_st);
    const double nuc = p.nu_c[c];
    const float tpnc = static_cast<float>(2.0 * kPi * nuc);
    const double lnfr = p.lnfr[c];
    const double bs = p.beam_k * (p.beam ? p.bfr[c] : 0.0);
    const double clip_r2 = p.beam ? p.clip_r2[c] : 0.0;
    const float k3s = static_cast<float>(-3.0 * bs * bs);

    for (int s0 = sbeg; s0 < send; s0 += kPmeCh) {
      const int cnt = min(kPmeCh, send - s0);
      __syncthreads();  // LDS of the previous chunk is consumed
      {
        // B operand rows: a of the q range for 32 sources; a_p in float32
        const int s = tid >> 3, part = tid & 7;
        uint4 h0 = make_uint4(0, 0, 0, 0), h1 = h0, l0 = h0, l1 = h0;
        uint4 ph = h0, pl = h0;
        if (s < cnt) {
          const int64_t rowoff = static_cast<int64_t>(s0 + s) * p.nap;
          const int q0 = Q0 * kPmeBlk + part * 8;  // 8 antennas per thread
          if (q0 < (Q0 + nq) * kPmeBlk) {
            h0 = *reinterpret_cast<const uint4 *>(hi0 + rowoff + q0);
            h1 = *reinterpret_cast<const uint4 *>(hi0 + rowoff + q0 + 4);
            l0 = *reinterpret_cast<const uint4 *>(lo0 + rowoff + q0);
            l1 = *reinterpret_cast<const uint4 *>(lo0 + rowoff + q0 + 4);
          }
          ph = *reinterpret_cast<const uint4 *>(hi0 + rowoff + P * kPmeBlk + part * 4);
          pl = *reinterpret_cast<const uint4 *>(lo0 + rowoff + P * kPmeBlk + part * 4);
        }
        uint4 *bh = reinterpret_cast<uint4 *>(&s_bh[s][part * 16]);
        uint4 *bl = reinterpret_cast<uint4 *>(&s_bl[s][part * 16]);
        bh[0] = h0;
        bh[1] = h1;
        bl[0] = l0;
        bl[1] = l1;
        const uint32_t phw[4] = {ph.x, ph.y, ph.z, ph.w}, plw[4] = {pl.x, pl.y, pl.z, pl.w};
#pragma unroll
        for (int j = 0; j < 4; ++j)
          s_ap[part * 4 + j][s] =
              make_float2(lo_h(phw[j]) + lo_h(plw[j]), hi_h(phw[j]) + hi_h(plw[j]));
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
          half8 rh, rl;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            rh[2 * e] = mh[st][2 * e + 1];
            rh[2 * e + 1] = -mh[st][2 * e];
            rl[2 * e] = ml[st][2 * e + 1];
            rl[2 * e + 1] = -ml[st][2 * e];
          }
          accR = __builtin_amdgcn_mfma_f32_32x32x16_f16(mh[st], bh, accR, 0, 0, 0);
          accR = __builtin_amdgcn_mfma_f32_32x32x16_f16(mh[st], bl, accR, 0, 0, 0);
          accR = __builtin_amdgcn_mfma_f32_32x32x16_f16(ml[st], bh, accR, 0, 0, 0);
          accI = __builtin_amdgcn_mfma_f32_32x32x16_f16(rh, bh, accI, 0, 0, 0);
          accI = __builtin_amdgcn_mfma_f32_32x32x16_f16(rh, bl, accI, 0, 0, 0);
          accI = __builtin_amdgcn_mfma_f32_32x32x16_f16(rl, bh, accI, 0, 0, 0);
        }
      }
      // Z_k[p][s] (scaled) in lane (s = row, p = i(r)) ------------------------
      float4 st4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (row < cnt) st4 = stk[(sd.src_off + s0 + row) * p.nchan + c];
      const float stk_k = k == 0 ? st4.x : k == 1 ? st4.y : k == 2 ? st4.z : st4.w;
      float gk = 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = (r & 3) + 8 * (r >> 2) + 4 * g;
        const float2 a = s_ap[i][row];
        gk += a.x * accR[r];
        gk -= a.y * accI[r];
      }
      gk += __shfl_xor(gk, 32, kWave);
      if (g == 0) s_g[k][row] = gk;
      // W partial sums: wavefronts add St'_k Z_k in a fixed order
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        if (k == kk) {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int i = (r & 3) + 8 * (r >> 2) + 4 * g;
            float2 w = make_float2(stk_k * accR[r], stk_k * accI[r]);
            if (kk > 0) {
              const float2 o = s_w[i][row];
              w.x += o.x;
              w.y += o.y;
            }
            s_w[i][row] = w;
          }
        }
        __syncthreads();
      }
      // phase and beam sums over the antennas p of block P -------------------
      {
        const int s = tid & 31, pg = tid >> 5;
        float g5 = 0.0f, g6 = 0.0f, g7 = 0.0f, g8 = 0.0f, g9 = 0.0f;
        if (s < cnt) {
          const double4 geo = p.src_geo[sd.src_off + s0 + s];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = pg * 4 + e;
            const float2 a = s_ap[i][s];
            const float2 z = s_w[i][s];
            const float wr = a.x * z.x - a.y * z.y;
            const float wi = a.x * z.y + a.y * z.x;
            g7 += s_uvw[i][0] * wi;
            g8 += s_uvw[i][1] * wi;
            g9 += s_uvw[i][2] * wi;
            if (p.beam) {
              // d ln e / d(l, m) as in the per-baseline adjoint
              const double dl = geo.x - s_pnt[i][0];
              const double dm = geo.y - s_pnt[i][1];
              const double r2b = sumsq_rn(dl, dm);
              const bool clipped = r2b >= clip_r2;
              if (!clipped) {
                const float rb = N::sqrt_(r2b);
                const float xr = static_cast<float>(bs) * rb;
                float sb, cb;
                N::sincos_rad(xr, &sb, &cb);
                const float tx = xr > 1e-4f ? sb * N::rcp(cb * xr) : 1.0f + xr * xr / 3.0f;
                const float k3 = k3s * tx;
                g5 += k3 * static_cast<float>(dl) * wr;
                g6 += k3 * static_cast<float>(dm) * wr;
              }
            }
          }
        }
        g5 += __shfl_xor(g5, 32, kWave);
        g6 += __shfl_xor(g6, 32, kWave);
        g7 += __shfl_xor(g7, 32, kWave);
        g8 += __shfl_xor(g8, 32, kWave);
        g9 += __shfl_xor(g9, 32, kWave);
        if (g == 0) {
          s_red[wave][s][0] = g5;
          s_red[wave][s][1] = g6;
          s_red[wave][s][2] = g7;
          s_red[wave][s][3] = g8;
          s_red[wave][s][4] = g9;
        }
      }
      __syncthreads();
      if (tid < cnt) {
        const int s = tid;
        float gs[5];
#pragma unroll
        for (int j = 0; j < 5; ++j)
          gs[j] = unscl * (((s_red[0][s][j] + s_red[1][s][j]) + s_red[2][s][j]) + s_red[3][s][j]);
        float G[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) G[kk] = 0.5f * unscl * s_g[kk][s];
        const float4 sv = stk[(sd.src_off + s0 + s) * p.nchan + c];
        const double2 lo = p.src_lon[sd.src_off + s0 + s];
        const float f = static_cast<float>(exp(sd.alpha[s0 + s] * lnfr));
        const float lon = static_cast<float>(lo.x), mon = static_cast<float>(lo.y);
        float *acc = s_acc[s0 + s - sbeg];
        acc[0] += gs[0] + tpnc * (gs[2] - lon * gs[4]);
        acc[1] += gs[1] + tpnc * (gs[3] - mon * gs[4]);
        acc[2] += G[0] * f;
        acc[3] += G[1] * f;
        acc[4] += G[2] * f;
        acc[5] += G[3] * f;
        acc[6] += (sv.x * G[0] + sv.y * G[1] + sv.z * G[2] + sv.w * G[3]) *
                  static_cast<float>(lnfr);
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

// Point-source gradient rows from the adjoint partials: one workgroup per
// source, float64 sums in a fixed order; columns 7..9 (shape) are zero.
__global__ __launch_bounds__(256) void pme_finalize(const KParams p) {
  __shared__ double2 scr[256 / kWave];
  const int s = blockIdx.x;
  const int sr = s / kPmeSR, sl = s % kPmeSR;
  const int nper = p.ntime * p.pme_ncg * p.nblk * p.pme_nqr;
  const float *src = p.pgrad + static_cast<int64_t>(sr) * nper * (kPmeSR * 7) + sl * 7;
  for (int j = 0; j < 7; ++j) {
    Comp acc;
    for (int i = threadIdx.x; i < nper; i += 256)
      acc.add(static_cast<double>(src[static_cast<int64_t>(i) * (kPmeSR * 7) + j]));
    const Comp r = block_reduce<256>(acc, scr);
    if (threadIdx.x == 0) p.grad_out[(p.one.src_off + s) * 10 + j] = 2.0 * (r.s + r.c);
    __syncthreads();
  }
  if (threadIdx.x < 3) p.grad_out[(p.one.src_off + s) * 10 + 7 + threadIdx.x] = 0.0;
}

hipError_t launch_pme_adjoint(const KParams &p, hipStream_t stream) {
  const int64_t plane = static_cast<int64_t>(p.one.npsrc) * p.nap;
  if (plane <= 0 || p.pme_nt <= 0) return hipSuccess;
  dim3 g1(static_cast<unsigned>((plane + 255) / 256), static_cast<unsigned>(p.pme_nt));
  hipLaunchKernelGGL(pme_phase, g1, dim3(256), 0, stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nitems =
      static_cast<int64_t>(p.pme_nsr) * p.pme_nt * p.pme_ncg * p.nblk * p.pme_nqr;
  const int64_t grid = 8 * ((nitems + 7) / 8);
  hipLaunchKernelGGL(pme_adjoint, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_pme_finalize(const KParams &p, hipStream_t stream) {
  if (p.one.npsrc <= 0) return hipSuccess;
  hipLaunchKernelGGL(pme_finalize, dim3(p.one.npsrc), dim3(256), 0, stream, p);
  return hipGetLastError();
}

// Phase planes and antenna-pair sums for timesteps [p.pme_t0, p.pme_t0 + p.pme_nt).
hipError_t launch_pme(const KParams &p, hipStream_t stream) {
  const int64_t plane = static_cast<int64_t>(p.one.npsrc) * p.nap;
  if (plane <= 0 || p.pme_nt <= 0) return hipSuccess;
  dim3 g1(static_cast<unsigned>((plane + 255) / 256), static_cast<unsigned>(p.pme_nt));
  hipLaunchKernelGGL(pme_phase, g1, dim3(256), 0, stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nitems = static_cast<int64_t>(p.pme_nt) * p.nchan * p.npair;
  const int64_t grid = 8 * ((nitems + 7) / 8);
  hipLaunchKernelGGL(pme_forward, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, p);
  return hipGetLastError();
}

}  // namespace rime
