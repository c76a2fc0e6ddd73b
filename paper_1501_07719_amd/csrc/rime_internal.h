// Internal structures shared by the HIP kernels and the host runtime of
// librime.so.  Not part of the public ABI (include/rime.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rime.h"

namespace rime {

// Speed of light (m/s, exact) and the Gaussian shape constant pi^2 / (4 ln 2).
constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kGauss = (kPi * kPi) / (4.0 * 0.69314718055994530941723212145817657);

// Sources per tile (lanes of one wavefront cover srcs x chans in the adjoint).
constexpr int kWave = 64;

// One sky model as seen by the kernels: npsrc points, then ngsrc Gaussians,
// then nxsrc exponential disks.
struct SetDesc {
  const double *lm;      // [nsrc][2]
  const double *stokes;  // [nsrc][4]
  const double *alpha;   // [nsrc]
  const double *gshape;  // [ngsrc][3]
  const double *xshape;  // [nxsrc][3]
  int32_t npsrc, ngsrc, nxsrc;
  int64_t src_off;       // first source of this set in the concatenated source index
};

// Source morphologies (the shape factor S_tpqs of the source sum).
enum { SHAPE_POINT = 0, SHAPE_GAUSS = 1, SHAPE_DISK = 2 };

// Baseline tiling for one block size: every tile has at most `nbt` baselines
// and at most `nat` distinct antennas.
struct TileSet {
  int32_t nbt = 0, nat = 0, ntile = 0;
  int32_t *bl = nullptr;   // device [ntile][nbt]  global baseline index or -1
  int32_t *lpq = nullptr;  // device [ntile][nbt]  local p | (local q << 16)
  int32_t *ant = nullptr;  // device [ntile][nat]  global antenna index or -1
  int32_t *nact = nullptr; // device [ntile]       active baselines (slots 0..nact-1)
};

// Everything a kernel launch needs (passed by value).
struct KParams {
  // observation
  int32_t ntime, na, nbl, nchan;
  const double *uvw;       // [ntime][na][3]
  const double *nu_c;      // [nchan]  nu / c  (1/m)
  const double *lnfr;      // [nchan]  ln(nu / ref_freq)
  const double *pointing;  // [ntime][na][2]  (zeros when absent)
  const double *gains;     // [na][2][2]  (unity when absent)
  int32_t beam;
  const double *bsc;       // [nchan]  beam_k nu / beam_ref_freq (the beam argument per radian)
  const double *bk3;       // [nchan]  -3 bsc^2 (the beam gradient's factor)
  const double *clip_r2;   // [nchan]  (beam_clip / (beam_k nu / beam_ref_freq))^2
  double beam_k;           // beam argument is beam_k * r * nu / beam_ref_freq
  double beam_clip;
  // tiling
  int32_t nbt, nat, ntile;
  const int32_t *tile_bl, *tile_lpq, *tile_ant, *tile_nact;
  int32_t nchb;            // channel blocks
  int32_t tchunk, ntc;     // timesteps per work item, time chunks
  int32_t items_per_set;   // ntile * nchb * ntc
  // sets
  int32_t nset;
  const SetDesc *sets;     // device [nset] (batched) or nullptr
  SetDesc one;             // the single set when sets == nullptr
  const int32_t *order;    // device [nset] largest-first order, or nullptr
  // per-source derived data in the workspace
  double4 *src_geo;        // [total_src] (l, m, n - 1, 0)
  double2 *src_lon;        // [total_src] (l / n, m / n)
  void *src_st;            // [total_src][nchan] Stokes scaled by (nu/nu_ref)^alpha (R4)
  void *src_gs;            // [total_src] Gaussian shape (el, em, R em, R el) (R4)
  const void *bl_rec;      // [ntime][ntile][nbt] per-baseline records of the adjoint (R4):
                           //   (du, dv, dw, a-tile byte offsets of p | q << 16)
  float *src_f;            // [total_src][nchan] (nu/nu_ref)^alpha, or nullptr
  int64_t total_src;
  // domain flags (workspace header): dom[0] = number of flag words written by
  // the call, dom[1 + dom_off + set * blocks + block] = 1 when a source of that
  // preparation block has l^2 + m^2 >= 1 (outside the domain of n), else 0
  int32_t *dom;
  int32_t dom_off, dom_count;
  // weighted residual in Stokes form per visibility, [set][ntime][nbl][nchan][4]
  // (rho_I, rho_Q, rho_U, rho_V), written by the float64 forward of the
  // float64-residual mixed mode and read by its float32 adjoint
  float2 *rho_b;
  // direction-independent 2x2 term of eq. 1, G_p(t, nu): [ntime][na][nchan][4]
  // complex (xx, xy, yx, yy), or nullptr for the plan's diagonal gains; its
  // gradient (gradient calls with grad_die): per-visibility partials
  // [ntime][nbl][nchan][2][4] (Y G_q X^H for antenna p, Y^H G_p X for q),
  // summed per antenna over the CSR list ant_off / ant_bl (baseline, side)
  const double2 *die;
  double2 *die_part;
  double2 *grad_die;
  const int32_t *ant_off;  // [na + 1]
  const int2 *ant_bl;      // [2 nbl] (baseline, 0 for p / 1 for q), by antenna then baseline
  // brightness per timestep (single sky): stokes_t [ntime][nsrc][4] replaces
  // the sky's Stokes; src_sf [nsrc][nchan] (nu/nu_ref)^alpha in R; the
  // adjoint's per-timestep Stokes partials gst_part [item][tchunk][nsrc][4]
  // and their sums grad_stokes_t [ntime][nsrc][4]
  const double *stokes_t;
  void *src_sf;
  double *gst_part;
  double *grad_stokes_t;
  // per-call data
  const void *data;        // [ntime][nbl][nchan][4] complex
  const void *weight;      // [ntime][nbl][nchan][4] real
  void *vis;               // predict output
  double2 *chi2_part;      // [total items] (sum, compensation)
  double *grad_part;       // gradient partials [set][item][nsrc][10]
  void *rho_g;             // float64 gradient: residual tile per work item
                           //   [item][nbt][nc][4] double2
  double *grad_part2;      // second-level partials [set][chunk][nsrc][10]
  int32_t grad_chunks;     // items per second-level chunk, and chunk count
  int32_t grad_nchunk;
  double *chi2_out;        // [nset]
  double *grad_out;        // [total_src][10]
  // matrix-core point-source engine (single sky, float32-mixed): the source
  // sums of the point sources are formed per (timestep, channel) as the
  // antenna x antenna product A diag(St_k) A^H over 32 x 32 antenna tiles
  int32_t pme;             // 1: the point sources come from `spts`
  int32_t nap;             // antennas padded to a multiple of kPmeBlk
  int32_t npair;           // antenna-block pairs (P <= Q) that hold baselines
  const int2 *pair_blk;    // [npair] (P, Q)
  const int32_t *bl_slot;  // [nbl] pair << 11 | i << 6 | j << 1 | conj
  uint32_t *ph_hi;         // phase planes [pme_nt][nchan][npsrc][nap] half2 (re, im):
  uint32_t *ph_lo;         //   a = hi + lo, a = e exp(-2 pi i tau nu / c)
  float *ph_k3;            // [pme_nt][nchan][npsrc][nap] d ln e / d(l, m) = k3 (l - dl, m - dm)
  int32_t ngroup;          // forward work groups: a Q block with one or two P blocks
  const int32_t *groups;   // [ngroup][5] (Q, Pa, Pb or -1, pair of (Pa, Q), pair of (Pb, Q))
  int32_t pme_pairs;       // 1: groups pair two P blocks of a Q block; 0: one each
  int32_t *pme_exp;        // [nchan][4] exponent of max_s |St'_k| (forward scale 2^-e)
  int32_t pme_t0, pme_nt;  // timesteps held by the phase planes
  int32_t phase_nc;        // channels per workgroup of the phase planes (set at launch)
  double2 *spts;           // [ntime][nchan][npair][4][kPmeBlk][kPmeBlk] Stokes sums
  // matrix-core adjoint of the point sources
  int32_t pme_adj;         // 1: point-source gradient from the antenna-pair product
  int32_t nblk;            // antenna blocks (nap / kPmeBlk)
  const int32_t *pair_of;  // [nblk][nblk] pair index of (P, Q), P <= Q, or -1
  const uint32_t *pair_mask;  // [npair][kPmeBlk] bit j of word i: slot (i, j) used
  float2 *rho_t;           // [ntime][nchan][npair][4][kPmeBlk][kPmeBlk] residual in
                           //   Stokes form (conjugated for baselines stored as (q, p))
  float *pgrad;            // adjoint partials [nsr][ntime][ncg][nblk][nqr][kPmeSR][7]
  int32_t pme_ncg, pme_nqr, pme_nsr;
  double2 *pfin;           // float64 sums of pgrad over item chunks
                           //   [nsr][pme_fchunk][kPmeSR * 7] (sum, compensation)
  int32_t pme_fchunk;      // item chunks of those sums
  uint4 *mfrag;            // [pme_nt][nchan][nblk][nqr][4][8][64][2] fp16 fragments of M
  float *mscale;           // [pme_nt][nchan][nblk][nqr] 2^e undoing the fragment scale
};

// Antenna block of the matrix-core engine (rows and columns of one MFMA tile),
// and the work split of its adjoint: antenna blocks per Q range, sources per
// source range, channels per workgroup.  Four channels per workgroup rather
// than eight halve the idle tail of the last round of workgroups on small
// arrays: 64 antennas, 100 timesteps, 64 channels and 1000 sources take
// 3.33 ms against 3.58 ms; 197 antennas are unchanged.
constexpr int kPmeBlk = 32;
constexpr int kPmeNQ = 2;
constexpr int kPmeSR = 512;
constexpr int kPmeNCW = 4;

// The sums of the adjoint partials over items run as about kPmeFinWG
// workgroups of 256 columns (kPmeSR * 7 = 14 x 256) before one pass over the
// chunks: nsr * chunks <= max(kPmeFinWG, nsr) chunk rows of kPmeSR * 7.
constexpr int kPmeFinWG = 2048 / (kPmeSR * 7 / 256);
inline int pme_fin_nchunk(int nsr, int64_t nper) {
  const int64_t n = kPmeFinWG / (nsr > 0 ? nsr : 1);
  return static_cast<int>(n < 1 ? 1 : n < nper ? n : (nper > 0 ? nper : 1));
}

// Padding (in records) after the per-baseline records of the adjoint, which
// reads one record ahead.
constexpr int kRecPad = 1024;

// Kernel variant descriptor.
struct Variant {
  int32_t threads;         // baselines per work item (one per thread)
  int32_t nc;              // channels per thread
  int32_t ns;              // sources per tile
  int32_t pme;             // 1: point-source sums on the matrix cores
};

}  // namespace rime
