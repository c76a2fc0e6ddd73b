// HIP kernels of the RIME chi-squared engine for gfx950 (MI355X).
//
// One work item (= one workgroup) owns a tile of baselines (at most NBT, one
// per thread, drawn from at most NAT antennas), a block of NC channels and a
// chunk of timesteps.  For every source tile of NS sources it
//   1. computes the per-antenna terms a_tps(nu) = e_tps K_tps once per antenna
//      into LDS (the per-antenna-first strategy of the paper, Section 4,
//      fused here with the per-baseline stage instead of going through HBM);
//   2. accumulates, per visibility, the four Stokes-weighted sums
//      sum_s S c_s I'_s, ..., sum_s S c_s V'_s with c_s = a_p conj(a_q)
//      (eq. 1 with B written out; the gains are applied once after the sum,
//      which is exact since they do not depend on the source);
// and then, per visibility, forms V, the residual and the weighted squared
// residual of eq. lhood, reduced in float64 with compensated (two-sum)
// arithmetic.  In gradient mode the weighted residual stays in LDS and a
// second source sweep (lanes over sources x channels, loop over baselines;
// in the float32 kernels with two channels per thread, lanes over sources x
// two baseline halves, each lane with both channels) accumulates
// d chi^2 / d theta_s without ever storing V.
//
// Precision: R = double (plain FP64) or R = float (mixed).  The phase argument
// is formed in float64 (error-free in the FP64 path, in plain float64 within
// about 1e-12 turns in the mixed one) and reduced to [-1/2, 1/2] turns before
// the sine/cosine (in the mixed path a float32 one accurate to about one
// unit); the beam clip decision is taken in float64; the per-visibility source
// sums run in float32 within a source tile and are folded into float64 after
// each tile; chi^2 and gradient sums are float64.
#include "rime_device.h"

namespace rime {


template <class R>
__device__ void prep_baselines(const KParams &p, int nc, int t);

// ---------------------------------------------------------------------------
// Per-call preparation, one launch.  Rows blockIdx.y < nset: per-source data,
// (l, m, n - 1), (l/n, m/n), the spectrally scaled Stokes vector per channel
// (eq. brightness_term) and the Gaussian shape coefficients, one thread per
// source; each workgroup also records whether one of its sources lies outside
// the domain l^2 + m^2 < 1 of n = sqrt(1 - l^2 - m^2) (Section 2.1, after
// eq. k_term), whose geometry is then NaN.  Rows nset + t (gradient mode,
// nc > 0): the adjoint's per-baseline records of timestep t.
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(256) void prep_sources(const KParams p, int nc) {
  using R4 = typename Num<R>::R4;
  const int set = blockIdx.y;
  if (set >= p.nset) {
    prep_baselines<R>(p, nc, set - p.nset);
    return;
  }
  const SetDesc sd = p.sets ? p.sets[set] : p.one;
  const int nsrc = sd.npsrc + sd.ngsrc + sd.nxsrc;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  int outside = 0;
  if (s < nsrc) {
    const double l = sd.lm[2 * s], m = sd.lm[2 * s + 1];
    const double r2 = sumsq_rn(l, m);
    outside = r2 >= 1.0;
    const double nan = __builtin_nan("");
    const double n = outside ? nan : sqrt(1.0 - r2);
    const double nm1 = outside ? nan : -r2 / (1.0 + n);
    const int64_t g = sd.src_off + s;
    p.src_geo[g] = make_double4(l, m, nm1, outside ? 1.0 : 0.0);
    p.src_lon[g] = make_double2(l / n, m / n);
    const double I = sd.stokes[4 * s], Q = sd.stokes[4 * s + 1];
    const double U = sd.stokes[4 * s + 2], V = sd.stokes[4 * s + 3];
    const double a = sd.alpha[s];
    R4 *st = static_cast<R4 *>(p.src_st) + g * p.nchan;
    for (int c = 0; c < p.nchan; ++c) {
      const double f = exp(a * p.lnfr[c]);
      R4 v;
      v.x = static_cast<R>(f * I);
      v.y = static_cast<R>(f * Q);
      v.z = static_cast<R>(f * U);
      v.w = static_cast<R>(f * V);
      st[c] = v;
      if (p.src_f) p.src_f[g * p.nchan + c] = static_cast<float>(f);
      if (p.src_sf) static_cast<R *>(p.src_sf)[g * p.nchan + c] = static_cast<R>(f);
    }
    if (s >= sd.npsrc) {
      // Gaussian or disk shape with the axis ratio folded into the minor-axis
      // pair, so that the quadratic form is A^2 + B^2 with A = du el + dv em
      // and B = du (R em) - dv (R el)
      const int gi = s - sd.npsrc;
      const double *sh = gi < sd.ngsrc ? sd.gshape + 3 * gi : sd.xshape + 3 * (gi - sd.ngsrc);
      const double el = sh[0], em = sh[1], Rr = sh[2];
      R4 v;
      v.x = static_cast<R>(el);
      v.y = static_cast<R>(em);
      v.z = static_cast<R>(Rr * em);
      v.w = static_cast<R>(Rr * el);
      static_cast<R4 *>(p.src_gs)[g] = v;
    }
  }
  if (p.dom) {
    // every workgroup of the set rows writes its flag word (no clearing pass)
    const int any = __syncthreads_or(outside);
    if (threadIdx.x == 0) {
      p.dom[1 + p.dom_off + set * gridDim.x + blockIdx.x] = any;
      if (set == 0 && blockIdx.x == 0 && p.dom_off == 0) p.dom[0] = p.dom_count;
    }
  }
}

// ---------------------------------------------------------------------------
// Per-baseline records of the adjoint, one per (timestep, tile, slot): the
// baseline vector (u_p - u_q, v_p - v_q, w_p - w_q) and, in the bits of the
// last word, the byte offsets of antennas p (low 16 bits) and q (high 16 bits)
// within a source row of the a-tile of a kernel with `nc` channels per thread.
// The adjoint reads them with scalar loads.
// ---------------------------------------------------------------------------
template <class R>
__device__ void prep_baselines(const KParams &p, int nc, int t) {
  using N = Num<R>;
  using R2 = typename N::R2;
  using R4 = typename N::R4;
  const int64_t n = static_cast<int64_t>(p.ntile) * p.nbt;
  R4 *rec = static_cast<R4 *>(const_cast<void *>(p.bl_rec)) + t * n;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * 256) {
    const int tile = static_cast<int>(i / p.nbt);
    R4 r;
    r.x = r.y = r.z = R(0);
    uint32_t off = 0;
    if (p.tile_bl[i] >= 0) {
      const int lpq = p.tile_lpq[i];
      const int lp = lpq & 0xffff, lq = lpq >> 16;
      const int ap = p.tile_ant[tile * p.nat + lp], aq = p.tile_ant[tile * p.nat + lq];
      const double *up = p.uvw + (static_cast<int64_t>(t) * p.na + ap) * 3;
      const double *uq = p.uvw + (static_cast<int64_t>(t) * p.na + aq) * 3;
      r.x = static_cast<R>(up[0] - uq[0]);
      r.y = static_cast<R>(up[1] - uq[1]);
      r.z = static_cast<R>(up[2] - uq[2]);
      const uint32_t row = static_cast<uint32_t>(nc * sizeof(R2));
      off = lp * row | (lq * row) << 16;
    }
    r.w = N::from_bits(off);
    rec[i] = r;
  }
}

// ---------------------------------------------------------------------------
// Main kernel
// ---------------------------------------------------------------------------

// Kernel modes.  MODE_RESID is the forward of the float64-residual mixed
// mode: float64 arithmetic over float32 data and weights, chi^2 partials and,
// when p.rho_b is set, the weighted residual in Stokes form (float32) per
// visibility and, with p.pme_adj, in the antenna-pair slots.  MODE_ADJ is its
// float32 adjoint: pass 2 alone, over the residual read from p.rho_b.
enum { MODE_PREDICT = 0, MODE_CHI2 = 1, MODE_GRAD = 2, MODE_RESID = 3, MODE_ADJ = 4 };

template <bool B, class X, class Y> struct Pick { using T = X; };
template <class X, class Y> struct Pick<false, X, Y> { using T = Y; };

template <class R, int NBT, int NC, int NS, int MODE>
struct Layout {
  using R2 = typename Num<R>::R2;
  using R4 = typename Num<R>::R4;
  static constexpr int NAT = nat_for(NBT);
  static constexpr int NW = NBT / kWave;
  // a-tile row per source: NAT antennas x NC channels, padded by two
  // elements so that the adjoint's lanes (source x channel) hit distinct banks.
  static constexpr int AST = NAT * NC + 2;
  static constexpr bool GRAD = MODE == MODE_GRAD || MODE == MODE_ADJ;
  static constexpr size_t A_BYTES = (sizeof(R2) * NS * AST + 511) / 512 * 512;
  static constexpr size_t BETA_BYTES = GRAD ? A_BYTES : 0;
  static constexpr size_t RED_BYTES = GRAD ? sizeof(R) * NBT * 10 : 0;
  // The float64 gradient with two channels per thread and at least 256
  // threads keeps the residual tile of its work item in global memory (the
  // workspace): the adjoint reads it as a broadcast (the lanes of a wavefront
  // need NC distinct 64-byte rows per baseline, served by the vector cache),
  // and without its 32 KiB the kernel fits two workgroups per CU instead of
  // one (measured at 64 antennas: 140 -> 93 ms).  The other variants keep it
  // in LDS: the float32 ones, and the float64 ones whose registers already
  // allow one wavefront per SIMD only, where the global reads cost time.
  static constexpr bool RHO_GLOBAL = GRAD && sizeof(R) == 8 && NC == 2 && NBT >= 256;
  static constexpr size_t RHO_TILE = GRAD ? sizeof(R2) * NBT * NC * 4 : 0;
  static constexpr size_t RHO_BYTES = RHO_GLOBAL ? 0 : RHO_TILE;
  static_assert(!GRAD || NS * NC == kWave, "the adjoint maps one wavefront to NS x NC");
  // LDS byte offsets.  The residual tile comes first: the adjoint addresses it
  // per lane plus constant offsets, which fold into the 16-bit offset field of
  // ds_read only below 64 KiB.  Beta follows the a-tile at a multiple of 512
  // bytes (one base for both in ds_read2st64); the adjoint's cross-wave
  // reduction buffer reuses the a and beta tiles, which are dead at that point.
  static constexpr size_t OFF_RHO = 0;
  static constexpr size_t OFF_A = OFF_RHO + RHO_BYTES;
  static constexpr size_t OFF_BETA = OFF_A + A_BYTES;
  // per-source records of the tile: NC scaled Stokes rows, then the shape
  static constexpr int SREC = NC + 1;
  static constexpr size_t OFF_SRC = OFF_BETA + BETA_BYTES;
  static constexpr size_t OFF_UVW = OFF_SRC + sizeof(R4) * NS * SREC;
  static constexpr size_t OFF_PNT = OFF_UVW + sizeof(double) * NAT * 3;
  static constexpr size_t OFF_SCR = OFF_PNT + sizeof(double) * NAT * 2;
  static constexpr size_t OFF_RED = OFF_A;
  static constexpr size_t LDS_BYTES = OFF_SCR + sizeof(double2) * (NW > 0 ? NW : 1);
  static_assert(A_BYTES % 512 == 0 && RHO_BYTES % 16 == 0, "alignment of the LDS regions");
  static_assert(RED_BYTES <= A_BYTES + BETA_BYTES, "reduction buffer within the a/beta tiles");
  static_assert(RHO_BYTES <= 65536, "the residual tile must lie below 64 KiB");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS of one CU");
};

// Per-antenna stage for one source tile: a[s][ant][c] = e K (and, for the
// adjoint, beta[s][ant][c] = d ln e / d(l, m)), plus the tile's scaled Stokes
// and Gaussian shapes.
template <class R, int NBT, int NC, int NS, int MODE, bool WITH_BETA, bool TERMS>
__device__ inline void stage_tile(const KParams &p, const SetDesc &sd, int t, int tile, int s0,
                                  int cnt, bool shaped, int c0, int ncv,
                                  const double (*s_uvw)[3],
                                  const double (*s_pnt)[2], typename Num<R>::R2 *s_a,
                                  typename Num<R>::R2 *s_beta, typename Num<R>::R4 *s_src) {
  using L = Layout<R, NBT, NC, NS, MODE>;
  using N = Num<R>;
  using R2 = typename N::R2;
  using R4 = typename N::R4;
  constexpr int NAT = L::NAT;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NS * NAT; idx += NBT) {
    const int s = idx / NAT;
    const int ai = idx - s * NAT;
    const bool ok = s < cnt && p.tile_ant[tile * NAT + ai] >= 0;
    R2 out[NC];
    R2 bet[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      out[c].x = R(0);
      out[c].y = R(0);
      bet[c].x = R(0);
      bet[c].y = R(0);
    }
    if (ok) {
      const double4 g = p.src_geo[sd.src_off + s0 + s];
      // tau = u l + v m + w (n - 1), metres (eq. k_term): error-free in
      // float64, a plain float64 evaluation for the float32 path
      const PhaseArg<sizeof(R) == 8> tau(s_uvw[ai][0], s_uvw[ai][1], s_uvw[ai][2], g.x, g.y,
                                         g.z);
      double r2b = 0.0, dl = 0.0, dm = 0.0, rb = 0.0;
      if (p.beam) {
        dl = g.x - s_pnt[ai][0];
        dm = g.y - s_pnt[ai][1];
        r2b = sumsq_rn(dl, dm);
        rb = sqrt(r2b);
      }
      // The angles of the per-antenna factors are formed in float64 and their
      // sines and cosines to within about a unit of R (N::sincos_turns): each
      // factor is reused by every baseline of the tile that holds the antenna.
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (c < ncv) {
          const double r = tau.turns(p.nu_c[c0 + c]);
          R sn, cs;
          N::sincos_turns(r, &sn, &cs);
          R e = R(1);
          if (p.beam) {
            // x_b = bs r, bs = beam_k nu / beam_ref_freq, clipped at beam_clip
            // (eq. e_term); the clip is decided on r^2 against the per-channel
            // threshold (beam_clip / bs)^2.
            // d ln e / dl = -3 tan(x) dx/dl, dx/dl = bs (l - dl_p) / r
            //             = -3 bs^2 (l - dl_p) tan(x)/x ; zero past the clip.
            const double bs = p.bsc[c0 + c];
            const bool clipped = r2b >= p.clip_r2[c0 + c];
            const double xr = clipped ? p.beam_clip : bs * rb;
            R tx = R(0);
            if constexpr (sizeof(R) == 8) {
              R sb, cb;
              N::sincos_turns(xr * kInvTwoPi, &sb, &cb);
              e = cb * cb * cb;
              if (WITH_BETA && !clipped)
                tx = xr > 1e-4 ? sb * N::rcp(cb * xr) : R(1) + xr * xr * R(1.0 / 3.0);
            } else {
              float txf = 0.0f;
              beam_f32(static_cast<float>(xr), WITH_BETA, &e, &txf);
              if (!clipped) tx = txf;
            }
            if (WITH_BETA) {
              const R k3 = static_cast<R>(p.bk3[c0 + c]) * tx;
              bet[c].x = k3 * static_cast<R>(dl);
              bet[c].y = k3 * static_cast<R>(dm);
            }
          }
          out[c].x = e * cs;
          out[c].y = -e * sn;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      s_a[s * L::AST + ai * NC + c] = out[c];
      if (WITH_BETA) s_beta[s * L::AST + ai * NC + c] = bet[c];
    }
  }
  // per-source records: the NC Stokes rows of the block's channels, then the
  // Gaussian or disk shape (zeros for point sources and past the tile's end);
  // with brightness per timestep, the rows are (nu/nu_ref)^alpha times this
  // timestep's Stokes vector
  const R4 *st = static_cast<const R4 *>(p.src_st);
  const R4 *gs = static_cast<const R4 *>(p.src_gs);
  const int nsrc = sd.npsrc + sd.ngsrc + sd.nxsrc;
  for (int idx = tid; idx < NS * L::SREC; idx += NBT) {
    const int s = idx / L::SREC, c = idx - s * L::SREC;
    R4 v;
    v.x = v.y = v.z = v.w = R(0);
    if (s < cnt) {
      if (c < NC) {
        if (c < ncv) {
          if (TERMS && p.stokes_t) {
            const double *q = p.stokes_t + (static_cast<int64_t>(t) * nsrc + s0 + s) * 4;
            const double f = static_cast<double>(
                static_cast<const R *>(p.src_sf)[(sd.src_off + s0 + s) * p.nchan + c0 + c]);
            v.x = static_cast<R>(f * q[0]);
            v.y = static_cast<R>(f * q[1]);
            v.z = static_cast<R>(f * q[2]);
            v.w = static_cast<R>(f * q[3]);
          } else {
            v = st[(sd.src_off + s0 + s) * p.nchan + c0 + c];
          }
        }
      } else if (shaped) {
        v = gs[sd.src_off + s0 + s];
      }
    }
    s_src[idx] = v;
  }
}

// Pass 1 inner loop over the sources of one tile: adds
// sum_s S c_s (I', Q', U', V')_s to the 8 accumulators of each channel.
// `src` holds the tile's per-source records (NC scaled Stokes rows, then the
// shape coefficients (el, em, R em, R el)).  With A = du el + dv em and
// B = du R em - dv R el, the shape factor is S = expb(gqs[c] (A^2 + B^2)) for
// a Gaussian and S = (1 + gqs[c] (A^2 + B^2))^(-3/2) for an exponential disk
// (gqs: the channel's coefficient of the morphology).  All lanes read the
// same record (an LDS broadcast).
template <class R, int NC, int AST, int SHAPE>
__device__ inline void accumulate(int cnt, const typename Num<R>::R2 *ap_row,
                                  const typename Num<R>::R2 *aq_row,
                                  const typename Num<R>::R4 *src, R du, R dv, const R *gqs,
                                  R (&in)[NC][8]) {
  using N = Num<R>;
  using R2 = typename N::R2;
  using R4 = typename N::R4;
  static_assert(NC % 2 == 0, "channel pairs");
#pragma unroll 2
  for (int s = 0; s < cnt; ++s) {
    const R4 *rs = src + s * (NC + 1);
    R Qf = R(0);
    if (SHAPE != SHAPE_POINT) {
      const R4 g = rs[NC];
      const R A = du * g.x + dv * g.y;
      const R B = du * g.z - dv * g.w;
      Qf = A * A + B * B;
    }
    // the a-terms of channel pairs as one 4-vector load each
    R2 apc[NC], aqc[NC];
#pragma unroll
    for (int c = 0; c < NC; c += 2) {
      const R4 p4 = *reinterpret_cast<const R4 *>(ap_row + s * AST + c);
      const R4 q4 = *reinterpret_cast<const R4 *>(aq_row + s * AST + c);
      apc[c].x = p4.x;
      apc[c].y = p4.y;
      apc[c + 1].x = p4.z;
      apc[c + 1].y = p4.w;
      aqc[c].x = q4.x;
      aqc[c].y = q4.y;
      aqc[c + 1].x = q4.z;
      aqc[c + 1].y = q4.w;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const R2 ap = apc[c];
      const R2 aq = aqc[c];
      const R4 st = rs[c];
      R cr = ap.x * aq.x + ap.y * aq.y;
      R ci = ap.y * aq.x - ap.x * aq.y;
      if (SHAPE == SHAPE_GAUSS) {
        const R S = N::expb(gqs[c] * Qf);
        cr *= S;
        ci *= S;
      } else if (SHAPE == SHAPE_DISK) {
        const R r = N::rsqrt_(R(1) + gqs[c] * Qf);
        const R S = r * r * r;
        cr *= S;
        ci *= S;
      }
      in[c][0] += cr * st.x;
      in[c][1] += ci * st.x;
      in[c][2] += cr * st.y;
      in[c][3] += ci * st.y;
      in[c][4] += cr * st.z;
      in[c][5] += ci * st.z;
      in[c][6] += cr * st.w;
      in[c][7] += ci * st.w;
    }
  }
}

// Pass 2 inner loop over the tile's active baselines, for this lane's
// (source, channel).  Accumulators:
//   g[0..3]  sum Re(c rho_k)                      (Stokes, times f later; also
//            give sum Re P = sum_k St'_k g[k] for alpha)
//   g[5], g[6]   sum (beta_p + beta_q)_{l,m} Re P  (beam part of l, m)
//   g[7], g[8], g[9]  sum (du, dv, dw) Im P        (phase part of l, m)
//   g[10..14]  Gaussian and disk: sum du A h ReP, sum dv B h ReP, sum dv A h ReP,
//              sum du B h ReP, sum B^2 h ReP, with A = du e.x + dv e.y and
//              B = du e.z - dv e.w the lane-scaled shape terms: for a Gaussian
//              S = expb(-(A^2 + B^2)) and h = 1; for a disk
//              S = (1 + A^2 + B^2)^(-3/2) and h = 1 / (1 + A^2 + B^2), the
//              term-dependent part of d ln S / d(A^2 + B^2)
// with P = c Phi, Phi = sum_k St'_k rho_k.  `rec` holds the tile's
// per-baseline records (du, dv, dw, a-tile offsets of p and q), read with
// scalar loads; the beta row of a source lies BETA_OFF bytes after its a row.
template <class R, int NC, int SHAPE, bool BEAM, int BETA_OFF>
__device__ inline void adjoint_loop(int wave, int nw, int nact, const RIME_CONST Quad<R> *rec,
                                    const typename Num<R>::R2 *s_rho, const char *arow,
                                    const typename Num<R>::R4 st,
                                    const typename Num<R>::R4 e, int cl, R (&g)[15]) {
  using N = Num<R>;
  using R2 = typename N::R2;
  using R4 = typename N::R4;
  // records are read one iteration ahead (the record array is padded)
  Quad<R> geo_n = rec[wave];
#pragma unroll 2
  for (int bi = wave; bi < nact; bi += nw) {
    const Quad<R> geo = geo_n;
    geo_n = rec[bi + nw];
    const uint32_t off = N::bits(geo.w);
    const char *pa = arow + (off & 0xffffu);
    const char *qa = arow + (off >> 16);
    const R2 ap = *reinterpret_cast<const R2 *>(pa);
    const R2 aq = *reinterpret_cast<const R2 *>(qa);
    const R2 *rho = s_rho + (bi * NC + cl) * 4;
    const R2 r0 = rho[0], r1 = rho[1], r2 = rho[2], r3 = rho[3];
    R cr = ap.x * aq.x + ap.y * aq.y;
    R ci = ap.y * aq.x - ap.x * aq.y;
    R A = R(0), B = R(0), h = R(1);
    if (SHAPE == SHAPE_GAUSS) {
      A = geo.x * e.x + geo.y * e.y;
      B = geo.x * e.z - geo.y * e.w;
      const R S = N::expb(-(A * A + B * B));
      cr *= S;
      ci *= S;
    } else if (SHAPE == SHAPE_DISK) {
      A = geo.x * e.x + geo.y * e.y;
      B = geo.x * e.z - geo.y * e.w;
      const R r = N::rsqrt_(R(1) + A * A + B * B);
      h = r * r;
      const R S = h * r;
      cr *= S;
      ci *= S;
    }
    // Re(c rho_k) as two fused multiply-adds each
    g[0] += cr * r0.x;
    g[0] -= ci * r0.y;
    g[1] += cr * r1.x;
    g[1] -= ci * r1.y;
    g[2] += cr * r2.x;
    g[2] -= ci * r2.y;
    g[3] += cr * r3.x;
    g[3] -= ci * r3.y;
    const R phr = st.x * r0.x + st.y * r1.x + st.z * r2.x + st.w * r3.x;
    const R phi = st.x * r0.y + st.y * r1.y + st.z * r2.y + st.w * r3.y;
    const R Pr = cr * phr - ci * phi;
    const R Pi = cr * phi + ci * phr;
    if (BEAM) {
      const R2 bp = *reinterpret_cast<const R2 *>(pa + BETA_OFF);
      const R2 bq = *reinterpret_cast<const R2 *>(qa + BETA_OFF);
      g[5] += (bp.x + bq.x) * Pr;
      g[6] += (bp.y + bq.y) * Pr;
    }
    g[7] += geo.x * Pi;
    g[8] += geo.y * Pi;
    g[9] += geo.z * Pi;
    if (SHAPE != SHAPE_POINT) {
      const R hP = SHAPE == SHAPE_DISK ? h * Pr : Pr;
      const R t1 = A * hP, t2 = B * hP;
      g[10] += geo.x * t1;
      g[11] += geo.y * t2;
      g[12] += geo.y * t1;
      g[13] += geo.x * t2;
      g[14] += B * t2;
    }
  }
}

// Pass 2 inner loop of the float32 kernels with two channels per thread,
// with both channels of a (source, baseline) in one lane: lane (source sl,
// half hb) takes the baselines 2 j + hb of this wavefront's pairs j (and the
// wavefront that holds a last, unpaired baseline takes it in half 0).  The
// per-channel sums g[c][0..3] (Re(c rho_k)), g5[c], g6[c] (beam) are as in
// adjoint_loop; the phase and shape sums are merged over the two channels,
// each channel's final factor applied per baseline:
//   G7..G9   sum (du, dv, dw) Pi,        Pi = sum_c tp_c Im P_c
//   G10..G14 sum du A0 H, dv B0 H, dv A0 H, du B0 H, B0^2 H,
//            H = sum_c dk_c h_c Re P_c, with A0 = du e.x + dv e.y and
//            B0 = du e.z - dv e.w of the unscaled shape (el, em, R em, R el),
//            S_c = expb(-kk_c (A0^2 + B0^2)) for a Gaussian and
//            (1 + kk_c (A0^2 + B0^2))^(-3/2), h_c = 1 / (1 + kk_c (A0^2 + B0^2))
//            for a disk (h_c = 1 for a Gaussian).
// The shape coordinates are then formed once per baseline for both channels.
struct PairConst {
  float tp[2], kk[2], dk[2];  // 2 pi nu/c, the shape scale squared, the shape gradient factor
};
struct PairAcc {
  float g[2][4], g5[2], g6[2], G[8];  // G: G7, G8, G9, G10 .. G14
};

template <int SHAPE, bool BEAM, int BETA_OFF>
__device__ inline void adjoint_pair(int wave, int nw, int nact, int hb, const float4 *rec,
                                    const float2 *s_rho, const char *arow, const float4 st0,
                                    const float4 st1, const float4 e, const PairConst &k,
                                    PairAcc &a) {
  auto body = [&](const float4 geo, int bi) {
    const uint32_t off = __float_as_uint(geo.w);
    const char *pa = arow + (off & 0xffffu);
    const char *qa = arow + (off >> 16);
    const float4 ap = *reinterpret_cast<const float4 *>(pa);  // (channel 0, channel 1)
    const float4 aq = *reinterpret_cast<const float4 *>(qa);
    const float4 *rho = reinterpret_cast<const float4 *>(s_rho + bi * 2 * 4);
    const float4 r[4] = {rho[0], rho[1], rho[2], rho[3]};  // channel 0: k 0,1 | 2,3; channel 1
    float cr[2] = {ap.x * aq.x + ap.y * aq.y, ap.z * aq.z + ap.w * aq.w};
    float ci[2] = {ap.y * aq.x - ap.x * aq.y, ap.w * aq.z - ap.z * aq.w};
    float A0 = 0.0f, B0 = 0.0f, h[2] = {1.0f, 1.0f};
    if (SHAPE != SHAPE_POINT) {
      A0 = geo.x * e.x + geo.y * e.y;
      B0 = geo.x * e.z - geo.y * e.w;
      const float Q0 = A0 * A0 + B0 * B0;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        float S;
        if (SHAPE == SHAPE_GAUSS) {
          S = __builtin_amdgcn_exp2f(-(k.kk[c] * Q0));
        } else {
          const float rr = __builtin_amdgcn_rsqf(1.0f + k.kk[c] * Q0);
          h[c] = rr * rr;
          S = h[c] * rr;
        }
        cr[c] *= S;
        ci[c] *= S;
      }
    }
    float Pr[2], Pi[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float4 ra = r[2 * c], rb = r[2 * c + 1];  // (rho_0, rho_1), (rho_2, rho_3)
      const float4 st = c == 0 ? st0 : st1;
      a.g[c][0] += cr[c] * ra.x;
      a.g[c][0] -= ci[c] * ra.y;
      a.g[c][1] += cr[c] * ra.z;
      a.g[c][1] -= ci[c] * ra.w;
      a.g[c][2] += cr[c] * rb.x;
      a.g[c][2] -= ci[c] * rb.y;
      a.g[c][3] += cr[c] * rb.z;
      a.g[c][3] -= ci[c] * rb.w;
      const float phr = st.x * ra.x + st.y * ra.z + st.z * rb.x + st.w * rb.z;
      const float phi = st.x * ra.y + st.y * ra.w + st.z * rb.y + st.w * rb.w;
      Pr[c] = cr[c] * phr - ci[c] * phi;
      Pi[c] = cr[c] * phi + ci[c] * phr;
    }
    if (BEAM) {
      const float4 bp = *reinterpret_cast<const float4 *>(pa + BETA_OFF);
      const float4 bq = *reinterpret_cast<const float4 *>(qa + BETA_OFF);
      a.g5[0] += (bp.x + bq.x) * Pr[0];
      a.g6[0] += (bp.y + bq.y) * Pr[0];
      a.g5[1] += (bp.z + bq.z) * Pr[1];
      a.g6[1] += (bp.w + bq.w) * Pr[1];
    }
    const float Pt = k.tp[0] * Pi[0] + k.tp[1] * Pi[1];
    a.G[0] += geo.x * Pt;
    a.G[1] += geo.y * Pt;
    a.G[2] += geo.z * Pt;
    if (SHAPE != SHAPE_POINT) {
      const float H = k.dk[0] * h[0] * Pr[0] + k.dk[1] * h[1] * Pr[1];
      const float t1 = A0 * H, t2 = B0 * H;
      a.G[3] += geo.x * t1;
      a.G[4] += geo.y * t2;
      a.G[5] += geo.y * t1;
      a.G[6] += geo.x * t2;
      a.G[7] += B0 * t2;
    }
  };
  const int npair = nact >> 1;
  // records are read one pair ahead (the record array is padded)
  float4 geo_n = rec[2 * wave + hb];
  for (int bj = wave; bj < npair; bj += nw) {
    const float4 geo = geo_n;
    geo_n = rec[2 * (bj + nw) + hb];
    body(geo, 2 * bj + hb);
  }
  if ((nact & 1) && hb == 0 && wave == npair % nw) body(rec[nact - 1], nact - 1);
}

// Source tiles of a set: points first, then Gaussians, then disks; tile k
// covers sources [s0, s0 + cnt) of one morphology.
struct SrcTile {
  int shape, s0, cnt;
};

__device__ inline SrcTile src_tile(const SetDesc &sd, int k, int ns, int npt, int ngt) {
  if (k < npt) return {SHAPE_POINT, k * ns, min(ns, sd.npsrc - k * ns)};
  if (k < npt + ngt) {
    const int s0 = sd.npsrc + (k - npt) * ns;
    return {SHAPE_GAUSS, s0, min(ns, sd.npsrc + sd.ngsrc - s0)};
  }
  const int s0 = sd.npsrc + sd.ngsrc + (k - npt - ngt) * ns;
  return {SHAPE_DISK, s0, min(ns, sd.npsrc + sd.ngsrc + sd.nxsrc - s0)};
}

// TERMS: the instantiation that also applies per-call terms (a 2x2 G per
// antenna, brightness per timestep); kept apart so that the plain calls do
// not carry their registers.
// The float64 256-thread forward kernels with two channels per thread ask
// for three workgroups per CU (168 VGPRs, a few dozen spilled outside the
// source loops): they fit that in LDS and were VALU-idle a quarter of the
// time at two (c2: float64-residual forward 29.5 -> 27.5 ms, FP64 chi^2
// 28.5 -> 27.6 ms).  The gradient mode's LDS allows two workgroups anyway.
template <class R, int NBT, int NC, int NS, int MODE, bool TERMS>
__global__ __launch_bounds__(NBT, (NBT == 256 && NC == 2 && sizeof(R) == 8 &&
                                   MODE != MODE_GRAD) ? 3 : 1)
void rime_main(const KParams p) {
  using L = Layout<R, NBT, NC, NS, MODE>;
  using N = Num<R>;
  using R2 = typename N::R2;
  using R4 = typename N::R4;
  // data and weights: float32 in the float64 forward of the float64-residual mode
  using DT = typename Pick<MODE == MODE_RESID, float, R>::T;
  using DT2 = typename Num<DT>::R2;
  constexpr int NAT = L::NAT;
  constexpr int NW = L::NW;

  // one LDS block, laid out by Layout
  __shared__ __attribute__((aligned(16))) char smem[L::LDS_BYTES];
  R2 *s_rho = L::RHO_GLOBAL
                  ? static_cast<R2 *>(p.rho_g) +
                        static_cast<int64_t>(blockIdx.x) * (L::RHO_TILE / sizeof(R2))
                  : reinterpret_cast<R2 *>(smem + L::OFF_RHO);
  R2 *s_a = reinterpret_cast<R2 *>(smem + L::OFF_A);
  R2 *s_beta = reinterpret_cast<R2 *>(smem + L::OFF_BETA);
  R *s_red = reinterpret_cast<R *>(smem + L::OFF_RED);
  R4 *s_src = reinterpret_cast<R4 *>(smem + L::OFF_SRC);
  double(*s_uvw)[3] = reinterpret_cast<double(*)[3]>(smem + L::OFF_UVW);
  double(*s_pnt)[2] = reinterpret_cast<double(*)[2]>(smem + L::OFF_PNT);
  double2 *s_scr = reinterpret_cast<double2 *>(smem + L::OFF_SCR);

  // ---- work item ----------------------------------------------------------
  const int item = blockIdx.x;
  const int set_rank = item / p.items_per_set;
  const int local_item = item - set_rank * p.items_per_set;
  const int set = p.order ? const_ptr<int32_t>(p.order)[set_rank] : set_rank;
  const SetDesc sd = load_set(p, set);
  int rem = local_item;
  const int tile = rem % p.ntile;
  rem /= p.ntile;
  const int chb = rem % p.nchb;
  const int tc = rem / p.nchb;
  // this set's part of the per-visibility residual (float64-residual mode)
  const int64_t rho_set = static_cast<int64_t>(set) * p.ntime * p.nbl * p.nchan * 4;

  const int tid = threadIdx.x;
  const int nact = p.tile_nact[tile];
  const int bl = p.tile_bl[tile * NBT + tid];
  const bool active = bl >= 0;
  const int lpq = active ? p.tile_lpq[tile * NBT + tid] : 0;
  const int lp = lpq & 0xffff, lq = lpq >> 16;
  const int c0 = chb * NC;
  const int ncv = min(NC, p.nchan - c0);
  const int nsrc = sd.npsrc + sd.ngsrc + sd.nxsrc;
  const int t0 = tc * p.tchunk;
  const int t1 = min(p.ntime, t0 + p.tchunk);
  const int npt = (sd.npsrc + NS - 1) / NS;
  const int ngt = (sd.ngsrc + NS - 1) / NS;
  const int nst = npt + ngt + (sd.nxsrc + NS - 1) / NS;

  // per-channel constants of this thread's channels: -pi^2/(4 ln 2) (nu/c)^2
  // in the argument scale of N::expb (Gaussian), (2 pi nu/c)^2 (disk)
  R gqs[NC], dqs[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double nuc = c < ncv ? p.nu_c[c0 + c] : 0.0;
    gqs[c] = static_cast<R>(-kGauss * N::kExpScale * nuc * nuc);
    dqs[c] = static_cast<R>(4.0 * kPi * kPi * nuc * nuc);
  }

  Comp chi;

  for (int t = t0; t < t1; ++t) {
    __syncthreads();
    for (int i = tid; i < NAT; i += NBT) {
      const int a = p.tile_ant[tile * NAT + i];
      double u = 0, v = 0, w = 0, pl = 0, pm = 0;
      if (a >= 0) {
        const double *x = p.uvw + (static_cast<int64_t>(t) * p.na + a) * 3;
        u = x[0];
        v = x[1];
        w = x[2];
        if (p.beam) {
          const double *q = p.pointing + (static_cast<int64_t>(t) * p.na + a) * 2;
          pl = q[0];
          pm = q[1];
        }
      }
      s_uvw[i][0] = u;
      s_uvw[i][1] = v;
      s_uvw[i][2] = w;
      s_pnt[i][0] = pl;
      s_pnt[i][1] = pm;
    }
    __syncthreads();
    const R du = static_cast<R>(s_uvw[lp][0] - s_uvw[lq][0]);
    const R dv = static_cast<R>(s_uvw[lp][1] - s_uvw[lq][1]);

    // ---- epilogue for one channel: V, residual, chi^2 (and rho) ---------------
    // S = the four Stokes sums (re, im) of this thread's baseline.
    // the global antennas of this thread's baseline
    const int gap = active ? p.tile_ant[tile * NAT + lp] : 0;
    const int gaq = active ? p.tile_ant[tile * NAT + lq] : 0;
    auto gains = [&](double2 (&gg)[4]) {
      // V_ij *= g_pi conj(g_qj)
      const double2 gpi[2] = {make_double2(p.gains[4 * gap + 0], p.gains[4 * gap + 1]),
                              make_double2(p.gains[4 * gap + 2], p.gains[4 * gap + 3])};
      const double2 gqj[2] = {make_double2(p.gains[4 * gaq + 0], p.gains[4 * gaq + 1]),
                              make_double2(p.gains[4 * gaq + 2], p.gains[4 * gaq + 3])};
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double2 a = gpi[i], b = gqj[j];
          gg[2 * i + j] = make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
        }
    };
    auto epilogue = [&](int c, const double (&S)[8], const double2 (&gg)[4]) {
      const bool ok = c < ncv;
      // Stokes sums -> 2x2 coherency X (eq. brightness_term)
      const double SIr = S[0], SIi = S[1], SQr = S[2], SQi = S[3];
      const double SUr = S[4], SUi = S[5], SVr = S[6], SVi = S[7];
      M22 X;
      X.re[0] = SIr + SQr;  // xx
      X.im[0] = SIi + SQi;
      X.re[1] = SUr - SVi;  // xy = S_U + i S_V
      X.im[1] = SUi + SVr;
      X.re[2] = SUr + SVi;  // yx = S_U - i S_V
      X.im[2] = SUi - SVr;
      X.re[3] = SIr - SQr;  // yy
      X.im[3] = SIi - SQi;
      double Vr[4], Vi[4];
      // V = G_p X G_q^H (eq. 1's direction-independent term, outside the
      // source sum), or the plan's diagonal gains
      M22 Gp, Gq;
      if (TERMS && p.die) {
        const int64_t gi = (static_cast<int64_t>(t) * p.na) * p.nchan + c0 + min(c, ncv - 1);
        Gp = m22_load(p.die + (gi + static_cast<int64_t>(gap) * p.nchan) * 4);
        Gq = m22_load(p.die + (gi + static_cast<int64_t>(gaq) * p.nchan) * 4);
        const M22 V = m22_mul(m22_mul(Gp, X), m22_herm(Gq));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          Vr[k] = V.re[k];
          Vi[k] = V.im[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          Vr[k] = X.re[k] * gg[k].x - X.im[k] * gg[k].y;
          Vi[k] = X.re[k] * gg[k].y + X.im[k] * gg[k].x;
        }
      }
      const int64_t vidx = ((static_cast<int64_t>(t) * p.nbl + bl) * p.nchan + c0 + c) * 4;
      if (MODE == MODE_PREDICT) {
        if (ok) {
          R2 *out = static_cast<R2 *>(p.vis) + vidx;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            R2 v;
            v.x = static_cast<R>(Vr[k]);
            v.y = static_cast<R>(Vi[k]);
            out[k] = v;
          }
        }
      } else {
        double Yr[4] = {0, 0, 0, 0}, Yi[4] = {0, 0, 0, 0};
        if (ok) {
          const DT2 *D = static_cast<const DT2 *>(p.data) + vidx;
          const DT *W = static_cast<const DT *>(p.weight) + vidx;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const DT2 d = D[k];
            const double w = static_cast<double>(W[k]);
            const double rr = Vr[k] - static_cast<double>(d.x);
            const double ri = Vi[k] - static_cast<double>(d.y);
            chi.add(w * (rr * rr + ri * ri));
            Yr[k] = w * rr;
            Yi[k] = w * ri;
          }
        }
        if (MODE == MODE_GRAD || MODE == MODE_RESID) {
          // the residual carried to the coherency X: Z = G_p^H Y G_q (with
          // diagonal gains Z_ij = Y_ij conj(g_pi) g_qj = Y_ij conj(gg_ij)); then
          // rho_I = conj(Zxx) + conj(Zyy), rho_Q = conj(Zxx) - conj(Zyy),
          // rho_U = conj(Zxy) + conj(Zyx), rho_V = i (conj(Zxy) - conj(Zyx))
          double Zr[4], Zi[4];
          if (TERMS && p.die) {
            M22 Y;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              Y.re[k] = Yr[k];
              Y.im[k] = Yi[k];
            }
            const M22 Z = m22_mul(m22_mul(m22_herm(Gp), Y), Gq);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              Zr[k] = Z.re[k];
              Zi[k] = Z.im[k];
            }
            if (ok && p.die_part) {
              // d chi^2 / d conj(G) of this visibility: Y G_q X^H for antenna
              // p and Y^H G_p X for antenna q
              const M22 Ap = m22_mul(m22_mul(Y, Gq), m22_herm(X));
              const M22 Aq = m22_mul(m22_mul(m22_herm(Y), Gp), X);
              double2 *dp = p.die_part + vidx * 2;
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                dp[k] = make_double2(Ap.re[k], Ap.im[k]);
                dp[4 + k] = make_double2(Aq.re[k], Aq.im[k]);
              }
            }
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              Zr[k] = Yr[k] * gg[k].x + Yi[k] * gg[k].y;
              Zi[k] = Yi[k] * gg[k].x - Yr[k] * gg[k].y;
            }
          }
          // rho_k in the adjoint's precision (float32 in both mixed modes)
          using A = typename Pick<MODE == MODE_RESID, float, R>::T;
          using A2 = typename Num<A>::R2;
          A2 v[4];
          v[0].x = static_cast<A>(Zr[0] + Zr[3]);
          v[0].y = static_cast<A>(-(Zi[0] + Zi[3]));
          v[1].x = static_cast<A>(Zr[0] - Zr[3]);
          v[1].y = static_cast<A>(-(Zi[0] - Zi[3]));
          v[2].x = static_cast<A>(Zr[1] + Zr[2]);
          v[2].y = static_cast<A>(-(Zi[1] + Zi[2]));
          v[3].x = static_cast<A>(Zi[1] - Zi[2]);
          v[3].y = static_cast<A>(Zr[1] - Zr[2]);
          if (MODE == MODE_GRAD) {
            A2 *rho = reinterpret_cast<A2 *>(s_rho) + (tid * NC + c) * 4;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) rho[kk] = v[kk];
          } else if (ok && p.rho_b) {
            float2 *rb = p.rho_b + rho_set + vidx;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) rb[kk] = make_float2(v[kk].x, v[kk].y);
          }
          if (sizeof(A) == 4 && p.pme_adj && ok) {
            // the point-source adjoint on the matrix cores reads rho from its
            // antenna-pair slot (conjugated when the slot holds (q, p))
            const int slot = p.bl_slot[bl];
            const int pair = slot >> 11, si = (slot >> 6) & 31, sj = (slot >> 1) & 31;
            const float cj = (slot & 1) ? -1.0f : 1.0f;
            float2 *rt = p.rho_t +
                         (((static_cast<int64_t>(t) * p.nchan + c0 + c) * p.npair + pair) * 4) *
                             (kPmeBlk * kPmeBlk) +
                         si * kPmeBlk + sj;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
              rt[kk * kPmeBlk * kPmeBlk] =
                  make_float2(static_cast<float>(v[kk].x), cj * static_cast<float>(v[kk].y));
          }
        }
      }
    };

    if constexpr (MODE == MODE_ADJ) {
      // the weighted residual of this thread's baseline from the float64
      // forward (zero past the last channel)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int64_t vidx =
            rho_set + ((static_cast<int64_t>(t) * p.nbl + bl) * p.nchan + c0 + c) * 4;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          s_rho[(tid * NC + c) * 4 + kk] =
              (active && c < ncv) ? p.rho_b[vidx + kk] : make_float2(0.0f, 0.0f);
      }
    } else {
      // ---- pass 1: source sums ----------------------------------------------
      double acc[NC][8];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[c][k] = 0.0;

      // with the matrix-core engine the point-source sums arrive from HBM
      for (int k = p.pme ? npt : 0; k < nst; ++k) {
        const SrcTile st = src_tile(sd, k, NS, npt, ngt);
        const int cnt = st.cnt;
        __syncthreads();
        stage_tile<R, NBT, NC, NS, MODE, false, TERMS>(p, sd, t, tile, st.s0, cnt,
                                                st.shape != SHAPE_POINT, c0, ncv, s_uvw, s_pnt,
                                                s_a, s_beta, s_src);
        __syncthreads();
        R in[NC][8];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int j = 0; j < 8; ++j) in[c][j] = R(0);
        {
          // the per-lane a-tile rows and the record base go through an opaque
          // register, so that the region offsets stay in the base addresses
          // and the loop advances them with immediate offsets
          // (16-byte aligned: NC * sizeof(R2) and the row stride are multiples
          // of 16, so a thread's NC channels load as one 16-byte word)
          static_assert((NC * sizeof(R2)) % 16 == 0 && (L::AST * sizeof(R2)) % 16 == 0 &&
                            L::OFF_A % 16 == 0 && L::OFF_SRC % 16 == 0,
                        "16-byte aligned a-tile rows");
          const R2 *ap_row = static_cast<const R2 *>(__builtin_assume_aligned(
              smem + opaque_vgpr(static_cast<uint32_t>(L::OFF_A + lp * NC * sizeof(R2))), 16));
          const R2 *aq_row = static_cast<const R2 *>(__builtin_assume_aligned(
              smem + opaque_vgpr(static_cast<uint32_t>(L::OFF_A + lq * NC * sizeof(R2))), 16));
          const R4 *src = static_cast<const R4 *>(__builtin_assume_aligned(
              smem + opaque_vgpr(static_cast<uint32_t>(L::OFF_SRC)), 16));
          if (st.shape == SHAPE_GAUSS)
            accumulate<R, NC, L::AST, SHAPE_GAUSS>(cnt, ap_row, aq_row, src, du, dv, gqs, in);
          else if (st.shape == SHAPE_DISK)
            accumulate<R, NC, L::AST, SHAPE_DISK>(cnt, ap_row, aq_row, src, du, dv, dqs, in);
          else
            accumulate<R, NC, L::AST, SHAPE_POINT>(cnt, ap_row, aq_row, src, du, dv, gqs, in);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int j = 0; j < 8; ++j) acc[c][j] += static_cast<double>(in[c][j]);
      }

      // ---- epilogue ------------------------------------------------------------
      if (active) {
        if (p.pme) {
          // point-source Stokes sums of this baseline from the antenna-pair
          // tiles; a baseline stored as (q, p) takes the conjugate
          const int slot = p.bl_slot[bl];
          const int pair = slot >> 11, si = (slot >> 6) & 31, sj = (slot >> 1) & 31;
          const double cj = (slot & 1) ? -1.0 : 1.0;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            if (c < ncv) {
              const double2 *sp =
                  p.spts +
                  (((static_cast<int64_t>(t) * p.nchan + c0 + c) * p.npair + pair) * 4) *
                      (kPmeBlk * kPmeBlk) +
                  si * kPmeBlk + sj;
#pragma unroll
              for (int kk = 0; kk < 4; ++kk) {
                const double2 v = sp[kk * kPmeBlk * kPmeBlk];
                acc[c][2 * kk] += v.x;
                acc[c][2 * kk + 1] += cj * v.y;
              }
            }
          }
        }
        double2 gg[4];
        gains(gg);
#pragma unroll
        for (int c = 0; c < NC; ++c) epilogue(c, acc[c], gg);
      }
    }

    // ---- pass 2: adjoint ----------------------------------------------------
    if (L::GRAD) {
      const int lane = tid % kWave;
      // wavefront index, uniform across the wavefront (scalar loop counters)
      const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
      // float32 with two channels per thread: lane = (source, baseline half)
      // holding both channels (adjoint_pair); otherwise lane = (source, channel)
      constexpr bool kPair = sizeof(R) == 4 && NC == 2;
      const int sl = kPair ? (lane & 31) : lane / NC;
      const int cl = kPair ? 0 : lane - (lane / NC) * NC;
      const int hb = kPair ? (lane >> 5) : 0;
      const bool lane_ok_c = cl < ncv;
      const double nuc_l = lane_ok_c ? p.nu_c[c0 + cl] : 0.0;
      const R tpnc = static_cast<R>(2.0 * kPi * nuc_l);
      // Gaussian lanes scale the shape coefficients by kap = sqrt(kGauss
      // kExpScale) nu/c, so that S = expb(-(A^2 + B^2)); 2 gq / kap with
      // gq = -kGauss (nu/c)^2 turns the accumulated sums into d chi^2 / d shape
      const double kap_l = sqrt(kGauss * N::kExpScale) * nuc_l;
      const double dsc_l = -2.0 * kap_l / N::kExpScale;
      // disk lanes scale by kapd = 2 pi nu/c, so that S = (1 + A^2 + B^2)^(-3/2)
      // and d ln S / d(A^2 + B^2) = -3/2 h: the sums turn into d chi^2 / d shape
      // with -3 kapd in place of 2 gq / kap
      const double kapd_l = 2.0 * kPi * nuc_l;
      const double dscd_l = -3.0 * kapd_l;
      const double lnfr_l = lane_ok_c ? p.lnfr[c0 + cl] : 0.0;
      const RIME_CONST Quad<R> *rec =
          const_ptr<Quad<R>>(p.bl_rec) + (static_cast<int64_t>(t) * p.ntile + tile) * NBT;
      // both channels of a paired lane (zero past the last channel)
      double nuc2[2] = {0.0, 0.0}, lnfr2[2] = {0.0, 0.0};
      PairConst pc{};
      if (kPair) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
          if (c < ncv) {
            nuc2[c] = p.nu_c[c0 + c];
            lnfr2[c] = p.lnfr[c0 + c];
          }
        pc.tp[0] = static_cast<float>(2.0 * kPi * nuc2[0]);
        pc.tp[1] = static_cast<float>(2.0 * kPi * nuc2[1]);
      }
      // gradient partials: [set][item][nsrc][10], sets laid out by src_off
      double *gout = p.grad_part + sd.src_off * p.items_per_set * 10 +
                     static_cast<int64_t>(local_item) * nsrc * 10;
      // with the matrix-core adjoint the point sources are done elsewhere
      for (int k = p.pme_adj ? npt : 0; k < nst; ++k) {
        const SrcTile tl = src_tile(sd, k, NS, npt, ngt);
        const int s0 = tl.s0, cnt = tl.cnt;
        const bool shaped = tl.shape != SHAPE_POINT;
        const bool disk = tl.shape == SHAPE_DISK;
        __syncthreads();
        stage_tile<R, NBT, NC, NS, MODE, true, TERMS>(p, sd, t, tile, s0, cnt, shaped, c0, ncv,
                                                      s_uvw, s_pnt, s_a, s_beta, s_src);
        __syncthreads();
        R gl[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) gl[j] = R(0);
        if constexpr (kPair) {
          if (sl < cnt) {
            const float4 st0 = s_src[sl * L::SREC], st1 = s_src[sl * L::SREC + 1];
            const double2 lo = p.src_lon[sd.src_off + s0 + sl];
            float4 e = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (shaped) e = s_src[sl * L::SREC + NC];
            // the shape scale per channel: kap^2 (Gaussian, kap = sqrt(kGauss
            // kExpScale) nu/c) or kapd^2 (disk, kapd = 2 pi nu/c), and the
            // factor that turns the sums into d chi^2 / d shape (2 gq / kap or
            // -3 kapd, times the scale)
            PairConst pk = pc;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const double kg = sqrt(kGauss * N::kExpScale) * nuc2[c], kd = 2.0 * kPi * nuc2[c];
              pk.kk[c] = static_cast<float>(disk ? kd * kd : kg * kg);
              pk.dk[c] = static_cast<float>(disk ? -3.0 * kd * kd : -2.0 * kg * kg / N::kExpScale);
            }
            const char *arow =
                smem + opaque_vgpr(static_cast<uint32_t>(L::OFF_A + sl * L::AST * sizeof(R2)));
            const float4 *recv = reinterpret_cast<const float4 *>(p.bl_rec) +
                                 (static_cast<int64_t>(t) * p.ntile + tile) * NBT;
            const float2 *rho2 = reinterpret_cast<const float2 *>(s_rho);
            constexpr int BO = static_cast<int>(L::OFF_BETA - L::OFF_A);
            PairAcc a{};
            if (p.beam) {
              if (tl.shape == SHAPE_GAUSS)
                adjoint_pair<SHAPE_GAUSS, true, BO>(wave, NW, nact, hb, recv, rho2, arow, st0, st1,
                                                    e, pk, a);
              else if (disk)
                adjoint_pair<SHAPE_DISK, true, BO>(wave, NW, nact, hb, recv, rho2, arow, st0, st1,
                                                   e, pk, a);
              else
                adjoint_pair<SHAPE_POINT, true, BO>(wave, NW, nact, hb, recv, rho2, arow, st0, st1,
                                                    e, pk, a);
            } else {
              if (tl.shape == SHAPE_GAUSS)
                adjoint_pair<SHAPE_GAUSS, false, BO>(wave, NW, nact, hb, recv, rho2, arow, st0,
                                                     st1, e, pk, a);
              else if (disk)
                adjoint_pair<SHAPE_DISK, false, BO>(wave, NW, nact, hb, recv, rho2, arow, st0, st1,
                                                    e, pk, a);
              else
                adjoint_pair<SHAPE_POINT, false, BO>(wave, NW, nact, hb, recv, rho2, arow, st0,
                                                     st1, e, pk, a);
            }
            // assemble this half's sums over its baselines (both channels)
            const double al = sd.alpha[s0 + sl];
            const float f0 = static_cast<float>(exp(al * lnfr2[0]));
            const float f1 = static_cast<float>(exp(al * lnfr2[1]));
            const float lon = static_cast<float>(lo.x), mon = static_cast<float>(lo.y);
            gl[0] = a.g5[0] + a.g5[1] + (a.G[0] - lon * a.G[2]);
            gl[1] = a.g6[0] + a.g6[1] + (a.G[1] - mon * a.G[2]);
            gl[2] = a.g[0][0] * f0 + a.g[1][0] * f1;
            gl[3] = a.g[0][1] * f0 + a.g[1][1] * f1;
            gl[4] = a.g[0][2] * f0 + a.g[1][2] * f1;
            gl[5] = a.g[0][3] * f0 + a.g[1][3] * f1;
            gl[6] = (st0.x * a.g[0][0] + st0.y * a.g[0][1] + st0.z * a.g[0][2] +
                     st0.w * a.g[0][3]) * static_cast<float>(lnfr2[0]) +
                    (st1.x * a.g[1][0] + st1.y * a.g[1][1] + st1.z * a.g[1][2] +
                     st1.w * a.g[1][3]) * static_cast<float>(lnfr2[1]);
            if (shaped) {
              const int xi = s0 + sl - sd.npsrc;
              const double Rr =
                  disk ? sd.xshape[3 * (xi - sd.ngsrc) + 2] : sd.gshape[3 * xi + 2];
              const float Rf = static_cast<float>(Rr);
              gl[7] = a.G[3] - Rf * a.G[4];
              gl[8] = a.G[5] + Rf * a.G[6];
              gl[9] = Rr > 0.0 ? static_cast<float>(static_cast<double>(a.G[7]) / Rr) : 0.0f;
            }
          }
        } else if (sl < cnt && lane_ok_c) {
          const R4 st = s_src[sl * L::SREC + cl];
          const double2 lo = p.src_lon[sd.src_off + s0 + sl];
          R4 e;
          e.x = e.y = e.z = e.w = R(0);
          if (shaped) {
            const R4 gsh = s_src[sl * L::SREC + NC];
            const R kap = static_cast<R>(disk ? kapd_l : kap_l);
            e.x = kap * gsh.x;
            e.y = kap * gsh.y;
            e.z = kap * gsh.z;
            e.w = kap * gsh.w;
          }
          // per-lane a-tile base with the region offset inside the register
          const char *arow = smem + opaque_vgpr(static_cast<uint32_t>(
                                        L::OFF_A + (sl * L::AST + cl) * sizeof(R2)));
          constexpr int BO = static_cast<int>(L::OFF_BETA - L::OFF_A);
          R g[15];
#pragma unroll
          for (int j = 0; j < 15; ++j) g[j] = R(0);
          if (p.beam) {
            if (tl.shape == SHAPE_GAUSS)
              adjoint_loop<R, NC, SHAPE_GAUSS, true, BO>(wave, NW, nact, rec, s_rho, arow, st, e,
                                                         cl, g);
            else if (disk)
              adjoint_loop<R, NC, SHAPE_DISK, true, BO>(wave, NW, nact, rec, s_rho, arow, st, e,
                                                        cl, g);
            else
              adjoint_loop<R, NC, SHAPE_POINT, true, BO>(wave, NW, nact, rec, s_rho, arow, st, e,
                                                         cl, g);
          } else {
            if (tl.shape == SHAPE_GAUSS)
              adjoint_loop<R, NC, SHAPE_GAUSS, false, BO>(wave, NW, nact, rec, s_rho, arow, st, e,
                                                          cl, g);
            else if (disk)
              adjoint_loop<R, NC, SHAPE_DISK, false, BO>(wave, NW, nact, rec, s_rho, arow, st, e,
                                                         cl, g);
            else
              adjoint_loop<R, NC, SHAPE_POINT, false, BO>(wave, NW, nact, rec, s_rho, arow, st, e,
                                                          cl, g);
          }
          g[4] = st.x * g[0] + st.y * g[1] + st.z * g[2] + st.w * g[3];
          // assemble: Stokes by the spectral factor, alpha by ln(nu/nu_ref),
          // l and m from their beam and phase parts, shape by 2 gq / kap (the
          // sums carry A = kap (du el + dv em) and B = kap R (du em - dv el)):
          //   d/d el = 2 gq / kap (g10 - R g11),  d/d em = 2 gq / kap (g12 + R g13),
          //   d/d R  = 2 gq / kap g14 / (kap R)
          const double al = sd.alpha[s0 + sl];
          const R f = static_cast<R>(exp(al * lnfr_l));
          const R lon = static_cast<R>(lo.x), mon = static_cast<R>(lo.y);
          gl[0] = g[5] + tpnc * (g[7] - lon * g[9]);
          gl[1] = g[6] + tpnc * (g[8] - mon * g[9]);
          gl[2] = g[0] * f;
          gl[3] = g[1] * f;
          gl[4] = g[2] * f;
          gl[5] = g[3] * f;
          gl[6] = g[4] * static_cast<R>(lnfr_l);
          if (shaped) {
            const int xi = s0 + sl - sd.npsrc;
            const double Rr =
                disk ? sd.xshape[3 * (xi - sd.ngsrc) + 2] : sd.gshape[3 * xi + 2];
            const double dl_ = disk ? dscd_l : dsc_l, kl_ = disk ? kapd_l : kap_l;
            const R dsc = static_cast<R>(dl_), Rf = static_cast<R>(Rr);
            gl[7] = dsc * (g[10] - Rf * g[11]);
            gl[8] = dsc * (g[12] + Rf * g[13]);
            gl[9] = (Rr > 0.0 && kl_ > 0.0)
                        ? static_cast<R>(dl_ * static_cast<double>(g[14]) / (kl_ * Rr))
                        : R(0);
          }
        }
        // sum the lanes of each source (its NC channel lanes, adjacent; or
        // its two baseline halves), then across wavefronts through LDS in a
        // fixed order
#pragma unroll
        for (int j = 0; j < 10; ++j) {
          if (kPair) {
            gl[j] += __shfl_xor(gl[j], 32, kWave);
          } else {
#pragma unroll
            for (int d = 1; d < NC; d <<= 1) gl[j] += __shfl_xor(gl[j], d, kWave);
          }
        }
        __syncthreads();  // the reduction buffer aliases the beta, Stokes and shape tiles
        if (cl == 0 && hb == 0) {
#pragma unroll
          for (int j = 0; j < 10; ++j) s_red[(wave * NS + sl) * 10 + j] = gl[j];
        }
        __syncthreads();
        for (int idx = tid; idx < NS * 10; idx += NBT) {
          const int s = idx / 10;
          if (s >= cnt) continue;
          double sum = 0.0;
#pragma unroll 4
          for (int w = 0; w < NW; ++w) sum += static_cast<double>(s_red[w * NS * 10 + idx]);
          double *dst = gout + static_cast<int64_t>(s0) * 10 + idx;
          if (t == t0)
            *dst = sum;
          else
            *dst += sum;
          const int j = idx - s * 10;
          if (TERMS && p.gst_part && j >= 2 && j < 6)
            p.gst_part[((static_cast<int64_t>(local_item) * p.tchunk + (t - t0)) * nsrc + s0 + s) *
                           4 +
                       j - 2] = sum;
        }
      }
    }
  }

  if (MODE != MODE_PREDICT && MODE != MODE_ADJ) {
    const Comp r = block_reduce<NBT>(chi, s_scr);
    if (tid == 0)
      p.chi2_part[static_cast<int64_t>(set) * p.items_per_set + local_item] =
          make_double2(r.s, r.c);
  }
}

// ---------------------------------------------------------------------------
// Finalize: deterministic compensated sums of the per-item partials.
// ---------------------------------------------------------------------------
// chi^2 of one set from its per-item (sum, compensation) partials, in a fixed
// order; all 256 threads of the workgroup take part.
__device__ inline void chi2_reduce(const KParams &p, int set, double2 *scr) {
  Comp acc;
  const double2 *part = p.chi2_part + static_cast<int64_t>(set) * p.items_per_set;
  // each thread merges items tid, tid + 256, ... in that order; four loads are
  // issued before they are merged
  int i = threadIdx.x;
  for (; i + 3 * 256 < p.items_per_set; i += 4 * 256) {
    double2 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = part[i + k * 256];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.merge(v[k].x, v[k].y);
  }
  for (; i < p.items_per_set; i += 256) {
    const double2 v = part[i];
    acc.merge(v.x, v.y);
  }
  const Comp r = block_reduce<256>(acc, scr);
  if (threadIdx.x == 0) p.chi2_out[set] = r.s + r.c;
}

__global__ __launch_bounds__(256) void finalize_chi2(const KParams p) {
  __shared__ double2 scr[256 / kWave];
  chi2_reduce(p, blockIdx.x, scr);
}

// Level 1: grid (source-parameter blocks, item chunks, sets); each thread
// sums `grad_chunks` consecutive items of one (source, parameter).
// In gradient mode the grid has one more row of chunks (blockIdx.y ==
// grad_nchunk) whose first workgroup forms chi^2 instead, which saves a launch.
__global__ __launch_bounds__(256) void finalize_grad1(const KParams p) {
  __shared__ double2 scr[256 / kWave];
  const int set = blockIdx.z;
  if (static_cast<int>(blockIdx.y) == p.grad_nchunk) {
    if (blockIdx.x == 0) chi2_reduce(p, set, scr);
    return;
  }
  const SetDesc sd = p.sets ? p.sets[set] : p.one;
  const int nsrc = sd.npsrc + sd.ngsrc + sd.nxsrc;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nsrc * 10) return;
  const int chunk = blockIdx.y;
  const int i0 = chunk * p.grad_chunks;
  const int i1 = min(p.items_per_set, i0 + p.grad_chunks);
  const int64_t stride = static_cast<int64_t>(nsrc) * 10;
  const double *src = p.grad_part + sd.src_off * p.items_per_set * 10 + idx;
  Comp acc;
  // items in order; eight loads are issued before they are added
  int i = i0;
  for (; i + 8 <= i1; i += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = src[(i + k) * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc.add(v[k]);
  }
  for (; i < i1; ++i) acc.add(src[i * stride]);
  double2 *dst = reinterpret_cast<double2 *>(p.grad_part2) +
                 sd.src_off * p.grad_nchunk * 10 + static_cast<int64_t>(chunk) * stride + idx;
  *dst = make_double2(acc.s, acc.c);
}

// Level 2: one thread per (set, source, parameter) sums the chunks.
__global__ __launch_bounds__(256) void finalize_grad2(const KParams p) {
  const int set = blockIdx.y;
  const SetDesc sd = p.sets ? p.sets[set] : p.one;
  const int nsrc = sd.npsrc + sd.ngsrc + sd.nxsrc;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nsrc * 10) return;
  const int64_t stride = static_cast<int64_t>(nsrc) * 10;
  const double2 *src = reinterpret_cast<const double2 *>(p.grad_part2) +
                       sd.src_off * p.grad_nchunk * 10 + idx;
  Comp acc;
  // chunks in order; eight loads are issued before they are merged
  int j = 0;
  for (; j + 8 <= p.grad_nchunk; j += 8) {
    double2 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = src[(j + k) * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc.merge(v[k].x, v[k].y);
  }
  for (; j < p.grad_nchunk; ++j) {
    const double2 v = src[j * stride];
    acc.merge(v.x, v.y);
  }
  p.grad_out[sd.src_off * 10 + idx] = 2.0 * (acc.s + acc.c);
}

// ---------------------------------------------------------------------------
// Gradient with respect to the direction-independent term: per (timestep,
// antenna, channel, matrix entry), twice the sum of the per-visibility
// partials of the antenna's baselines in baseline order (compensated), i.e.
// d chi^2 / d Re G + i d chi^2 / d Im G.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void die_grad(const KParams p) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t n = static_cast<int64_t>(p.ntime) * p.na * p.nchan * 4;
  if (idx >= n) return;
  const int k = static_cast<int>(idx & 3);
  int64_t rest = idx >> 2;
  const int c = static_cast<int>(rest % p.nchan);
  rest /= p.nchan;
  const int a = static_cast<int>(rest % p.na);
  const int t = static_cast<int>(rest / p.na);
  Comp re, im;
  for (int j = p.ant_off[a]; j < p.ant_off[a + 1]; ++j) {
    const int2 e = p.ant_bl[j];
    const double2 v =
        p.die_part[((static_cast<int64_t>(t) * p.nbl + e.x) * p.nchan + c) * 8 + e.y * 4 + k];
    re.add(v.x);
    im.add(v.y);
  }
  p.grad_die[idx] = make_double2(2.0 * (re.s + re.c), 2.0 * (im.s + im.c));
}

// Gradient with respect to the brightness per timestep: per (timestep,
// source, Stokes parameter), twice the sum over the work items of that
// timestep's chunk (tiles, then channel blocks, in order).
__global__ __launch_bounds__(256) void stokes_t_grad(const KParams p) {
  const int nsrc = p.one.npsrc + p.one.ngsrc + p.one.nxsrc;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= static_cast<int64_t>(p.ntime) * nsrc * 4) return;
  const int64_t sk = idx % (static_cast<int64_t>(nsrc) * 4);
  const int t = static_cast<int>(idx / (static_cast<int64_t>(nsrc) * 4));
  const int tc = t / p.tchunk, tt = t - tc * p.tchunk;
  const int s = static_cast<int>(sk / 4), k = static_cast<int>(sk % 4);
  Comp acc;
  if (p.pme_adj && s < p.one.npsrc) {
    // point sources with the matrix-core adjoint: its per-item partials of
    // timestep t, columns 2..5 (the Stokes sums times the spectral factor)
    const int sr = s / kPmeSR, sl = s - sr * kPmeSR;
    const int64_t nit = static_cast<int64_t>(p.pme_ncg) * p.nblk * p.pme_nqr;
    const float *src =
        p.pgrad + (static_cast<int64_t>(sr) * p.ntime + t) * nit * (kPmeSR * 7) + sl * 7 + 2 + k;
    for (int64_t i = 0; i < nit; ++i) acc.add(static_cast<double>(src[i * (kPmeSR * 7)]));
  } else {
    for (int chb = 0; chb < p.nchb; ++chb)
      for (int tile = 0; tile < p.ntile; ++tile) {
        const int64_t item = tile + static_cast<int64_t>(p.ntile) * (chb + p.nchb * tc);
        acc.add(p.gst_part[(item * p.tchunk + tt) * nsrc * 4 + sk]);
      }
  }
  p.grad_stokes_t[idx] = 2.0 * (acc.s + acc.c);
}

hipError_t launch_stokes_t_grad(const KParams &p, hipStream_t stream) {
  const int64_t n = static_cast<int64_t>(p.ntime) * (p.one.npsrc + p.one.ngsrc + p.one.nxsrc) * 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(stokes_t_grad, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     stream, p);
  return hipGetLastError();
}

hipError_t launch_die_grad(const KParams &p, hipStream_t stream) {
  const int64_t n = static_cast<int64_t>(p.ntime) * p.na * p.nchan * 4;
  hipLaunchKernelGGL(die_grad, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream,
                     p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streamed evaluation: chi^2 and its gradient are additive over time
// (eq. lhood sums over timesteps), so a call over time chunks sums the
// chunks' results, in chunk order, compensated.  part[k] = (chi^2, grad) of
// chunk k, `stride` doubles apart; thread idx sums entry idx of every chunk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sum_chunks(const double *part, int nchunk, int64_t stride,
                                                  int64_t n, double *chi2, double *grad) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= n) return;
  Comp acc;
  for (int k = 0; k < nchunk; ++k) acc.add(part[k * stride + idx]);
  const double v = acc.s + acc.c;
  if (idx == 0)
    chi2[0] = v;
  else
    grad[idx - 1] = v;
}

hipError_t launch_sum_chunks(const double *part, int nchunk, int64_t stride, int64_t n,
                             double *chi2, double *grad, hipStream_t stream) {
  hipLaunchKernelGGL(sum_chunks, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     stream, part, nchunk, stride, n, chi2, grad);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// The instantiation with per-call terms runs only when a call has them.
template <class R, int NBT, int NC, int NS, int MODE>
static hipError_t launch_main(const KParams &p, int nitems, hipStream_t stream) {
  if (p.die || p.stokes_t)
    hipLaunchKernelGGL((rime_main<R, NBT, NC, NS, MODE, true>), dim3(nitems), dim3(NBT), 0,
                       stream, p);
  else
    hipLaunchKernelGGL((rime_main<R, NBT, NC, NS, MODE, false>), dim3(nitems), dim3(NBT), 0,
                       stream, p);
  return hipGetLastError();
}

hipError_t launch_prep(const KParams &p, bool fp64, int max_nsrc, int rec_nc,
                       hipStream_t stream) {
  // rec_nc > 0: also the per-baseline records of every timestep (one grid row
  // per timestep after the per-set rows); one workgroup per set row at least,
  // which writes the set's domain flag also for a sky without sources
  const int nblk = max_nsrc > 0 ? (max_nsrc + 255) / 256 : 1;
  dim3 grid(nblk, p.nset + (rec_nc > 0 ? p.ntime : 0));
  if (fp64)
    hipLaunchKernelGGL(prep_sources<double>, grid, dim3(256), 0, stream, p, rec_nc);
  else
    hipLaunchKernelGGL(prep_sources<float>, grid, dim3(256), 0, stream, p, rec_nc);
  return hipGetLastError();
}

// with_chi2 = false (gradient mode): the gradient only, chi^2 being formed
// from the partials of another launch geometry (the float64-residual mode).
hipError_t launch_finalize(const KParams &p, int mode, int max_nsrc, hipStream_t stream,
                           bool with_chi2) {
  if (mode == MODE_PREDICT) return hipSuccess;
  if (mode == MODE_GRAD && max_nsrc == 0) {
    // a sky without sources has no gradient rows
    if (!with_chi2) return hipSuccess;
    mode = MODE_CHI2;
  }
  if (mode != MODE_GRAD) {
    hipLaunchKernelGGL(finalize_chi2, dim3(p.nset), dim3(256), 0, stream, p);
    return hipGetLastError();
  }
  // level 1 of the gradient, plus chi^2 in the extra row of chunks
  const int nblk = (max_nsrc * 10 + 255) / 256;
  hipLaunchKernelGGL(finalize_grad1, dim3(nblk, p.grad_nchunk + (with_chi2 ? 1 : 0), p.nset),
                     dim3(256), 0, stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finalize_grad2, dim3(nblk, p.nset), dim3(256), 0, stream, p);
  return hipGetLastError();
}

// Compiled variants, indexed per (mode, precision).
struct VariantEntry {
  Variant v;
  hipError_t (*fn)(const KParams &, int, hipStream_t);
};

#define RIME_V(R, NBT, NC, NS, M, PME) \
  { {NBT, NC, NS, PME}, &launch_main<R, NBT, NC, NS, M> }

// Float64 variants 0..3; float32-mixed variants 0..3 plus 4..5 with the
// point-source sums on the matrix cores (single sky only).
constexpr int kMaxVariants = 6;
constexpr int kVariantCount[2] = {4, 6};

static const VariantEntry kVariants[3][2][kMaxVariants] = {
    // MODE_PREDICT
    {{RIME_V(double, 64, 2, 32, MODE_PREDICT, 0), RIME_V(double, 256, 2, 32, MODE_PREDICT, 0),
      RIME_V(double, 1024, 2, 32, MODE_PREDICT, 0), RIME_V(double, 256, 4, 16, MODE_PREDICT, 0)},
     {RIME_V(float, 64, 2, 32, MODE_PREDICT, 0), RIME_V(float, 256, 2, 32, MODE_PREDICT, 0),
      RIME_V(float, 1024, 2, 32, MODE_PREDICT, 0), RIME_V(float, 256, 4, 16, MODE_PREDICT, 0),
      RIME_V(float, 1024, 2, 32, MODE_PREDICT, 1), RIME_V(float, 256, 2, 32, MODE_PREDICT, 1)}},
    // MODE_CHI2
    {{RIME_V(double, 64, 2, 32, MODE_CHI2, 0), RIME_V(double, 256, 2, 32, MODE_CHI2, 0),
      RIME_V(double, 1024, 2, 32, MODE_CHI2, 0), RIME_V(double, 256, 4, 16, MODE_CHI2, 0)},
     {RIME_V(float, 64, 2, 32, MODE_CHI2, 0), RIME_V(float, 256, 2, 32, MODE_CHI2, 0),
      RIME_V(float, 1024, 2, 32, MODE_CHI2, 0), RIME_V(float, 256, 4, 16, MODE_CHI2, 0),
      RIME_V(float, 1024, 2, 32, MODE_CHI2, 1), RIME_V(float, 256, 2, 32, MODE_CHI2, 1)}},
    // MODE_GRAD
    {{RIME_V(double, 64, 2, 32, MODE_GRAD, 0), RIME_V(double, 256, 2, 32, MODE_GRAD, 0),
      RIME_V(double, 256, 4, 16, MODE_GRAD, 0), RIME_V(double, 64, 4, 16, MODE_GRAD, 0)},
     {RIME_V(float, 64, 2, 32, MODE_GRAD, 0), RIME_V(float, 256, 2, 32, MODE_GRAD, 0),
      RIME_V(float, 1024, 2, 32, MODE_GRAD, 0), RIME_V(float, 256, 4, 16, MODE_GRAD, 0),
      RIME_V(float, 1024, 2, 32, MODE_GRAD, 1), RIME_V(float, 256, 2, 32, MODE_GRAD, 1)}},
};

// The float64-residual mode: float64 forwards (the shapes of the float64
// variants) and float32 adjoints (the shapes of the float32-mixed gradient
// variants; 4 and 5 take the point sources on the matrix cores).
static const VariantEntry kResid[4] = {
    RIME_V(double, 64, 2, 32, MODE_RESID, 0), RIME_V(double, 256, 2, 32, MODE_RESID, 0),
    RIME_V(double, 1024, 2, 32, MODE_RESID, 0), RIME_V(double, 256, 4, 16, MODE_RESID, 0)};
static const VariantEntry kAdj[kMaxVariants] = {
    RIME_V(float, 64, 2, 32, MODE_ADJ, 0),   RIME_V(float, 256, 2, 32, MODE_ADJ, 0),
    RIME_V(float, 1024, 2, 32, MODE_ADJ, 0), RIME_V(float, 256, 4, 16, MODE_ADJ, 0),
    RIME_V(float, 1024, 2, 32, MODE_ADJ, 1), RIME_V(float, 256, 2, 32, MODE_ADJ, 1)};

hipError_t launch_resid(int index, const KParams &p, int nitems, hipStream_t stream) {
  return kResid[index].fn(p, nitems, stream);
}

hipError_t launch_adj(int index, const KParams &p, int nitems, hipStream_t stream) {
  return kAdj[index].fn(p, nitems, stream);
}

// Precision 2 is the float64-residual mixed mode: its chi^2 variants are the
// float64 forwards, its gradient variants the float32 adjoints; it has no
// predict variant (model visibilities come from either other precision).
int variant_count(int mode, int prec) {
  if (mode < 0 || mode > 2 || prec < 0 || prec > 2) return 0;
  if (prec == 2) return mode == MODE_PREDICT ? 0 : mode == MODE_CHI2 ? 4 : kMaxVariants;
  return kVariantCount[prec];
}

const Variant *variant_info(int mode, int prec, int index) {
  if (index < 0 || index >= variant_count(mode, prec)) return nullptr;
  if (prec == 2) return mode == MODE_CHI2 ? &kResid[index].v : &kAdj[index].v;
  return &kVariants[mode][prec][index].v;
}

hipError_t launch_variant(int mode, int prec, int index, const KParams &p, int nitems,
                          hipStream_t stream) {
  return kVariants[mode][prec][index].fn(p, nitems, stream);
}

}  // namespace rime
