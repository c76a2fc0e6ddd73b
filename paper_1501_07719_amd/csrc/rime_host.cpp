// Host runtime of librime.so: argument validation, observation plans and the
// baseline tiling, workspace layout, kernel-variant selection (with a timing
// autotuner and a JSON cache), batched proposals and their hipGraph capture.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "rime_internal.h"

namespace rime {
hipError_t launch_prep(const KParams &p, bool fp64, int max_nsrc, int rec_nc,
                       hipStream_t stream);
hipError_t launch_finalize(const KParams &p, int mode, int max_nsrc, hipStream_t stream,
                           bool with_chi2);
hipError_t launch_pme(const KParams &p, hipStream_t stream);
hipError_t launch_pme_adjoint(const KParams &p, bool phase, hipStream_t stream);
hipError_t launch_pme_finalize(const KParams &p, hipStream_t stream);
hipError_t launch_pme_scale(const KParams &p, hipStream_t stream);
int variant_count(int mode, int prec);
const Variant *variant_info(int mode, int prec, int index);
hipError_t launch_variant(int mode, int prec, int index, const KParams &p, int nitems,
                          hipStream_t stream);
hipError_t launch_resid(int index, const KParams &p, int nitems, hipStream_t stream);
hipError_t launch_sum_chunks(const double *part, int nchunk, int64_t stride, int64_t n,
                             double *chi2, double *grad, hipStream_t stream);
hipError_t launch_die_grad(const KParams &p, hipStream_t stream);
hipError_t launch_stokes_t_grad(const KParams &p, hipStream_t stream);
hipError_t launch_adj(int index, const KParams &p, int nitems, hipStream_t stream);
}  // namespace rime

using namespace rime;

// Device memory of the allocation-free entry point rime_chi2_grad_noalloc:
// one fixed block on every device the library runs on, held until the
// process ends.  Its name is a host-side stand-in; the device address comes
// from hipGetSymbolAddress, once per device (scratch_ptr below).
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local int32_t g_last_hip = 0;

inline rime_status hip_fail(hipError_t e) {
  g_last_hip = static_cast<int32_t>(e);
  return RIME_ERR_HIP;
}

#define RIME_HIP(call)                        \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

constexpr int kNbt[3] = {64, 256, 1024};
constexpr size_t kAlign = 256;
// Target number of work items per launch (several workgroups per CU).
constexpr int64_t kTargetItems = 8192;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int nat_for_host(int nbt) { return nbt >= 1024 ? 64 : nbt >= 256 ? 32 : 16; }

int nbt_slot(int nbt) {
  for (int i = 0; i < 3; ++i)
    if (kNbt[i] == nbt) return i;
  return -1;
}

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

struct rime_plan {
  int device = 0;
  int32_t ntime = 0, na = 0, nbl = 0, nchan = 0;
  int32_t beam = 0;
  double ref_freq = 0, beam_k = 0, beam_clip = 0;
  double *d_uvw = nullptr, *d_nu_c = nullptr, *d_lnfr = nullptr, *d_bsc = nullptr;
  double *d_bk3 = nullptr, *d_clip_r2 = nullptr;
  double *d_pointing = nullptr, *d_gains = nullptr;
  TileSet tiles[3];
  // antenna-block pairs of the matrix-core point-source engine
  int32_t nap = 0, npair = 0, nblk = 0;
  int2 *d_pair_blk = nullptr;
  int32_t *d_bl_slot = nullptr;
  int32_t *d_pair_of = nullptr;
  uint32_t *d_pair_mask = nullptr;
  int32_t ngroup = 0;
  int32_t pme_pairs = 0;        // forward groups pair two P blocks
  int32_t *d_groups = nullptr;  // [ngroup][5] forward work groups
  bool pme_adj_ok = false;  // every antenna-pair slot holds at most one baseline
  int32_t *d_ant_off = nullptr;  // [na + 1] baselines of each antenna (both sides)
  int2 *d_ant_bl = nullptr;      // [2 nbl] (baseline, 0: p / 1: q)
  int32_t variant[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // [mode][precision]
  std::string signature;  // observation part of the autotune key
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;        // around all compute kernels
  hipEvent_t ev_main0 = nullptr, ev_main1 = nullptr;       // around the per-baseline kernel
  // streamed calls: the upload stream, its fork event and, per staging
  // buffer, "uploaded" and "consumed" events (made with the plan)
  hipStream_t copy = nullptr;
  hipEvent_t ev_fork = nullptr, ev_up[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
};

struct GraphKey {
  const void *data, *weight;
  double *chi2, *grad;
  void *ws;
  size_t ws_bytes;
  void *stream;
  int prec, variant, mode;
  bool operator==(const GraphKey &o) const {
    return data == o.data && weight == o.weight && chi2 == o.chi2 && grad == o.grad &&
           ws == o.ws && ws_bytes == o.ws_bytes && stream == o.stream && prec == o.prec &&
           variant == o.variant && mode == o.mode;
  }
};

struct rime_batch {
  const rime_plan *plan = nullptr;
  int32_t nset = 0;
  int64_t total_src = 0;
  int32_t max_nsrc = 0;
  SetDesc *d_sets = nullptr;
  std::vector<SetDesc> h_sets;  // host copy (per-set launches of matrix-core variants)
  int32_t *d_order = nullptr;
  bool has_graph = false;
  GraphKey key{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t variant[3][3] = {{-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}};  // -1: the plan's
  // second lane of the per-set pipelines (matrix-core variants): a stream of
  // the library's own, forked from and joined to the caller's by two events
  hipStream_t lane = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace {

// ---------------------------------------------------------------------------
// Baseline tiling
// ---------------------------------------------------------------------------
// Antennas are split into nb balanced blocks of at most B = nat/2 antennas.
// The baselines joining block P and block Q (P < Q) form a tile (at most
// B^2 = nbt baselines over at most 2B = nat antennas); the baselines inside
// one block are paired with those inside another block into one tile.  Within
// a tile the baselines are sorted by (local p, local q).
rime_status compute_tiles(int na, int nbl, const std::vector<int32_t> &a1,
                          const std::vector<int32_t> &a2, int nbt, int &ntile_out,
                          std::vector<int32_t> &hbl, std::vector<int32_t> &hlpq,
                          std::vector<int32_t> &hant) {
  const int nat = nat_for_host(nbt);
  const int B = nat / 2;
  const int nb = (na + B - 1) / B;
  std::vector<int> block_of(na), block_start(nb + 1, 0);
  for (int b = 0; b < nb; ++b) block_start[b + 1] = block_start[b] + na / nb + (b < na % nb ? 1 : 0);
  for (int b = 0; b < nb; ++b)
    for (int a = block_start[b]; a < block_start[b + 1]; ++a) block_of[a] = b;
  std::vector<std::vector<int>> bucket(static_cast<size_t>(nb) * nb);
  for (int i = 0; i < nbl; ++i) {
    int P = block_of[a1[i]], Q = block_of[a2[i]];
    if (P > Q) std::swap(P, Q);
    bucket[static_cast<size_t>(P) * nb + Q].push_back(i);
  }
  struct T {
    std::vector<int> ants, bls;
  };
  std::vector<T> tiles;
  auto block_ants = [&](int P, std::vector<int> &out) {
    for (int a = block_start[P]; a < block_start[P + 1]; ++a) out.push_back(a);
  };
  auto emit_chunks = [&](const std::vector<int> &bls, const std::vector<int> &ants) {
    for (size_t o = 0; o < bls.size(); o += nbt) {
      T t;
      t.ants = ants;
      t.bls.assign(bls.begin() + o, bls.begin() + std::min(bls.size(), o + nbt));
      tiles.push_back(std::move(t));
    }
  };
  for (int P = 0; P < nb; ++P)
    for (int Q = P + 1; Q < nb; ++Q) {
      const auto &bk = bucket[static_cast<size_t>(P) * nb + Q];
      if (bk.empty()) continue;
      std::vector<int> ants;
      block_ants(P, ants);
      block_ants(Q, ants);
      emit_chunks(bk, ants);
    }
  int pending = -1;
  for (int P = 0; P < nb; ++P) {
    const auto &bk = bucket[static_cast<size_t>(P) * nb + P];
    if (bk.empty()) continue;
    if (pending < 0) {
      pending = P;
      continue;
    }
    const auto &pk = bucket[static_cast<size_t>(pending) * nb + pending];
    std::vector<int> ants;
    block_ants(pending, ants);
    block_ants(P, ants);
    if (static_cast<int>(pk.size() + bk.size()) <= nbt) {
      std::vector<int> bls(pk);
      bls.insert(bls.end(), bk.begin(), bk.end());
      emit_chunks(bls, ants);
    } else {
      std::vector<int> a0;
      block_ants(pending, a0);
      emit_chunks(pk, a0);
      std::vector<int> a1v;
      block_ants(P, a1v);
      emit_chunks(bk, a1v);
    }
    pending = -1;
  }
  if (pending >= 0) {
    std::vector<int> ants;
    block_ants(pending, ants);
    emit_chunks(bucket[static_cast<size_t>(pending) * nb + pending], ants);
  }
  const int ntile = static_cast<int>(tiles.size());
  hbl.assign(static_cast<size_t>(ntile) * nbt, -1);
  hlpq.assign(hbl.size(), 0);
  hant.assign(static_cast<size_t>(ntile) * nat, -1);
  std::vector<int> local(na, -1);
  for (int ti = 0; ti < ntile; ++ti) {
    T &t = tiles[ti];
    if (static_cast<int>(t.ants.size()) > nat) return RIME_ERR_ARG;
    for (size_t i = 0; i < t.ants.size(); ++i) {
      local[t.ants[i]] = static_cast<int>(i);
      hant[static_cast<size_t>(ti) * nat + i] = t.ants[i];
    }
    std::sort(t.bls.begin(), t.bls.end(), [&](int x, int y) {
      const int px = local[a1[x]], py = local[a1[y]];
      if (px != py) return px < py;
      return local[a2[x]] < local[a2[y]];
    });
    for (size_t i = 0; i < t.bls.size(); ++i) {
      const int b = t.bls[i];
      hbl[static_cast<size_t>(ti) * nbt + i] = b;
      hlpq[static_cast<size_t>(ti) * nbt + i] = local[a1[b]] | (local[a2[b]] << 16);
    }
    for (int a : t.ants) local[a] = -1;
  }
  ntile_out = ntile;
  return RIME_OK;
}

rime_status build_tiles(int na, int nbl, const std::vector<int32_t> &a1,
                        const std::vector<int32_t> &a2, int nbt, TileSet &ts) {
  int ntile = 0;
  std::vector<int32_t> hbl, hlpq, hant;
  rime_status st = compute_tiles(na, nbl, a1, a2, nbt, ntile, hbl, hlpq, hant);
  if (st != RIME_OK) return st;
  const int nat = nat_for_host(nbt);
  ts.nbt = nbt;
  ts.nat = nat;
  ts.ntile = ntile;
  std::vector<int32_t> hnact(ntile, 0);
  for (int t = 0; t < ntile; ++t)
    for (int i = 0; i < nbt; ++i)
      if (hbl[static_cast<size_t>(t) * nbt + i] >= 0) hnact[t] = i + 1;
  hipError_t e;
  if ((e = upload(&ts.nact, hnact)) != hipSuccess) return hip_fail(e);
  if ((e = upload(&ts.bl, hbl)) != hipSuccess) return hip_fail(e);
  if ((e = upload(&ts.lpq, hlpq)) != hipSuccess) return hip_fail(e);
  if ((e = upload(&ts.ant, hant)) != hipSuccess) return hip_fail(e);
  return RIME_OK;
}

// ---------------------------------------------------------------------------
// Launch geometry and workspace layout
// ---------------------------------------------------------------------------
// Work items per second-level chunk of the gradient reduction.
constexpr int kGradChunk = 32;

struct Geometry {
  int ntile = 0, nchb = 0, tchunk = 1, ntc = 1, items_per_set = 0, grad_nchunk = 1;
};

Geometry geometry(const rime_plan *plan, const Variant &v, int nset) {
  Geometry g;
  g.ntile = plan->tiles[nbt_slot(v.threads)].ntile;
  g.nchb = (plan->nchan + v.nc - 1) / v.nc;
  const int64_t per_t = static_cast<int64_t>(g.ntile) * g.nchb * nset;
  int64_t tc = (per_t * plan->ntime + kTargetItems - 1) / kTargetItems;
  tc = std::max<int64_t>(1, std::min<int64_t>(tc, plan->ntime));
  g.tchunk = static_cast<int>(tc);
  g.ntc = (plan->ntime + g.tchunk - 1) / g.tchunk;
  g.items_per_set = g.ntile * g.nchb * g.ntc;
  g.grad_nchunk = (g.items_per_set + kGradChunk - 1) / kGradChunk;
  return g;
}

// Per-call terms beyond the sky (rime_terms): bits of the `terms` argument of
// the layouts.
enum { TERM_DIE_GRAD = 1, TERM_STOKES_T = 2, TERM_STOKES_T_GRAD = 4 };

struct WsLayout {
  size_t dom = 0;
  size_t die_part = 0, src_sf = 0, gst = 0;
  size_t geo = 0, lon = 0, st = 0, gs = 0, rec = 0, chi2 = 0, grad = 0, grad2 = 0;
  size_t ph_hi = 0, ph_lo = 0, ph_k3 = 0, spts = 0, pexp = 0, rho_t = 0, pgrad = 0;
  size_t src_f = 0, mfrag = 0, mscale = 0, rho_g = 0, pfin = 0;
  int32_t pme_tchunk = 0;  // timesteps per phase-plane pass (0: engine off)
  bool pme_adj = false;    // point-source adjoint on the matrix cores
  size_t total = 0;
};

// Upper bound on the workspace of one time pass of the matrix-core engine (phase
// planes and residual fragments); one pass avoids recomputing the planes for
// the adjoint.
constexpr size_t kPmePlaneBytes = size_t(48) << 30;

constexpr int kRes64 = RIME_MIXED_RES64;

int pme_ncg(const rime_plan *plan) { return (plan->nchan + kPmeNCW - 1) / kPmeNCW; }
// bytes of one phase plane of one timestep (all channels)
int64_t plane_bytes_t(const rime_plan *plan, int64_t npsrc) {
  return static_cast<int64_t>(plan->nchan) * npsrc * plan->nap * 4;
}
int pme_nqr(const rime_plan *plan) { return (plan->nblk + kPmeNQ - 1) / kPmeNQ; }

// Whether a call runs point sources on the matrix cores (single sky, one of
// the mixed precisions).
bool pme_active(const Variant &v, int prec, int nset) {
  return v.pme && prec != RIME_FP64 && nset == 1;
}

// Words of the domain-flag header at the start of every workspace: a count,
// then one flag per (set, preparation workgroup of 256 sources).
int64_t dom_words(int nset, int64_t total_src) {
  return 1 + static_cast<int64_t>(nset) * std::max<int64_t>(1, (total_src + 255) / 256);
}

// fwd_sums = false: the point-source sums of the matrix-core forward are not
// needed (the adjoint half of the float64-residual mode).
WsLayout ws_layout(const rime_plan *plan, int mode, int prec, const Geometry &g, int nset,
                   int64_t total_src, const Variant &v, bool fwd_sums = true, int terms = 0) {
  WsLayout L;
  const size_t r4 = prec == RIME_FP64 ? 32 : 16;
  size_t off = 0;
  L.dom = off;
  off += align_up(static_cast<size_t>(dom_words(nset, total_src)) * sizeof(int32_t));
  L.geo = off;
  off += align_up(static_cast<size_t>(total_src) * sizeof(double4));
  L.lon = off;
  off += align_up(static_cast<size_t>(total_src) * sizeof(double2));
  L.st = off;
  off += align_up(static_cast<size_t>(total_src) * plan->nchan * r4);
  L.gs = off;
  off += align_up(static_cast<size_t>(total_src) * r4);
  if (mode == RIME_MODE_CHI2_GRAD) {
    L.rec = off;
    off += align_up((static_cast<size_t>(plan->ntime) * g.ntile * v.threads + kRecPad) * r4);
  }
  L.chi2 = off;
  if (mode != RIME_MODE_PREDICT)
    off += align_up(static_cast<size_t>(nset) * g.items_per_set * sizeof(double2));
  L.grad = off;
  if (mode == RIME_MODE_CHI2_GRAD)
    off += align_up(static_cast<size_t>(g.items_per_set) * total_src * 10 * sizeof(double));
  L.grad2 = off;
  if (mode == RIME_MODE_CHI2_GRAD)
    off += align_up(static_cast<size_t>(g.grad_nchunk) * total_src * 10 * sizeof(double2));
  L.rho_g = off;
  if (mode == RIME_MODE_CHI2_GRAD && prec == RIME_FP64 && v.nc == 2 && v.threads >= 256)
    off += align_up(static_cast<size_t>(nset) * g.items_per_set * v.threads * v.nc * 4 *
                    sizeof(double2));
  // (a sky without sources leaves the engine off)
  if (pme_active(v, prec, nset) && total_src > 0) {
    const bool adj = mode == RIME_MODE_CHI2_GRAD && plan->pme_adj_ok;
    const bool k3 = adj && plan->beam;
    // per timestep: phase planes (total_src bounds the point count) and, for
    // the adjoint, the residual fragments
    const size_t plane_t = static_cast<size_t>(plane_bytes_t(plan, total_src));
    const size_t frag_t = adj ? static_cast<size_t>(plan->nchan) * plan->nblk * pme_nqr(plan) *
                                    (4 * 8 * kWave * 2 * sizeof(uint4) + sizeof(float))
                              : 0;
    const size_t per_t = plane_t * (k3 ? 3 : 2) + frag_t;
    L.pme_tchunk = static_cast<int32_t>(
        std::max<size_t>(1, std::min<size_t>(plan->ntime, kPmePlaneBytes / per_t)));
    L.ph_hi = off;
    off += align_up(plane_t * L.pme_tchunk);
    L.ph_lo = off;
    off += align_up(plane_t * L.pme_tchunk);
    if (fwd_sums) {
      L.spts = off;
      off += align_up(static_cast<size_t>(plan->ntime) * plan->nchan * plan->npair * 4 *
                      kPmeBlk * kPmeBlk * sizeof(double2));
      L.pexp = off;
      off += align_up(static_cast<size_t>(plan->nchan) * 4 * sizeof(int32_t));
    }
    if (adj) {
      L.pme_adj = true;
      if (k3) {
        L.ph_k3 = off;
        off += align_up(plane_t * L.pme_tchunk);
      }
      L.rho_t = off;
      off += align_up(static_cast<size_t>(plan->ntime) * plan->nchan * plan->npair * 4 *
                      kPmeBlk * kPmeBlk * sizeof(float2));
      L.pgrad = off;
      off += align_up(static_cast<size_t>((total_src + kPmeSR - 1) / kPmeSR) * plan->ntime *
                      pme_ncg(plan) * plan->nblk * pme_nqr(plan) * kPmeSR * 7 * sizeof(float));
      L.pfin = off;
      off += align_up(static_cast<size_t>(std::max<int64_t>(kPmeFinWG, (total_src + kPmeSR - 1) /
                                                                           kPmeSR)) *
                      kPmeSR * 7 * sizeof(double2));
      L.src_f = off;
      off += align_up(static_cast<size_t>(total_src) * plan->nchan * sizeof(float));
      const size_t nfrag = static_cast<size_t>(L.pme_tchunk) * plan->nchan * plan->nblk *
                           pme_nqr(plan);
      L.mfrag = off;
      off += align_up(nfrag * 4 * 8 * kWave * 2 * sizeof(uint4));
      L.mscale = off;
      off += align_up(nfrag * sizeof(float));
    }
  }
  if (terms & TERM_DIE_GRAD) {
    L.die_part = off;
    off += align_up(static_cast<size_t>(plan->ntime) * plan->nbl * plan->nchan * 8 *
                    sizeof(double2));
  }
  if (terms & TERM_STOKES_T) {
    L.src_sf = off;
    off += align_up(static_cast<size_t>(total_src) * plan->nchan * (r4 / 4));
  }
  if ((terms & TERM_STOKES_T_GRAD) && mode == RIME_MODE_CHI2_GRAD) {
    L.gst = off;
    off += align_up(static_cast<size_t>(g.items_per_set) * g.tchunk * total_src * 4 *
                    sizeof(double));
  }
  L.total = off;
  return L;
}

// The float64-residual mode composes two layouts: the float64 forward's
// (with the domain header at offset 0) and, in gradient mode, the float32
// adjoint's, followed by the per-visibility residual of every set.
struct Res64Layout {
  WsLayout f, a;
  Variant va{};            // the adjoint variant as run (matrix cores only when usable)
  size_t a_off = 0, rho_b = 0, total = 0;
};

Res64Layout res64_layout(const rime_plan *plan, int mode, const Variant &vf,
                         const Variant *va, int nset, int64_t total_src, int terms = 0) {
  Res64Layout R;
  // the forward writes the partials of the G gradient; both halves stage the
  // brightness per timestep; the adjoint writes its per-timestep partials
  R.f = ws_layout(plan, RIME_MODE_CHI2, RIME_FP64, geometry(plan, vf, nset), nset, total_src,
                  vf, true, terms & (TERM_DIE_GRAD | TERM_STOKES_T));
  size_t off = R.f.total;
  if (mode == RIME_MODE_CHI2_GRAD && va) {
    R.va = *va;
    // the point-source adjoint on the matrix cores needs single-baseline slots
    if (!plan->pme_adj_ok) R.va.pme = 0;
    R.a_off = off;
    R.a = ws_layout(plan, RIME_MODE_CHI2_GRAD, RIME_MIXED, geometry(plan, R.va, nset), nset,
                    total_src, R.va, false, terms & (TERM_STOKES_T | TERM_STOKES_T_GRAD));
    off += R.a.total;
    R.rho_b = off;
    off += align_up(static_cast<size_t>(nset) * plan->ntime * plan->nbl * plan->nchan * 4 *
                    sizeof(float2));
  }
  R.total = off;
  return R;
}

// Workspace of one call of (mode, prec) with kernel variant `vidx` and, for a
// gradient in the float64-residual mode, forward variant `fidx`.
size_t call_ws(const rime_plan *plan, int mode, int prec, int vidx, int fidx, int nset,
               int64_t total_src, int terms = 0) {
  const Variant *v = variant_info(mode, prec, vidx);
  if (!v) return 0;
  if (prec != kRes64)
    return ws_layout(plan, mode, prec, geometry(plan, *v, nset), nset, total_src, *v, true, terms)
        .total;
  if (mode == RIME_MODE_CHI2)
    return res64_layout(plan, mode, *v, nullptr, nset, total_src, terms).total;
  const Variant *vf = variant_info(RIME_MODE_CHI2, kRes64, fidx);
  if (!vf) return 0;
  return res64_layout(plan, mode, *vf, v, nset, total_src, terms).total;
}

// Whether a batched call with this variant runs the single-sky pipeline once
// per set (the matrix-core engine works on one sky at a time).
bool per_set_variant(const rime_plan *plan, int mode, int prec, const Variant &v) {
  if (mode == RIME_MODE_PREDICT || !pme_active(v, prec, 1)) return false;
  return prec == RIME_MIXED || (mode == RIME_MODE_CHI2_GRAD && plan->pme_adj_ok);
}

// Per-set pipelines of the matrix-core variants run in two lanes: sets
// 0, 2, 4, ... on the caller's stream and 1, 3, 5, ... on the batch's own, so
// that the kernels of one set overlap those of the next (small sets leave
// most of the chip idle).
constexpr int kBatchLanes = 2;

size_t ws_max(const rime_plan *plan, int mode, int prec, int nset, int64_t total_src) {
  size_t best = 0;
  const int nf = prec == kRes64 && mode == RIME_MODE_CHI2_GRAD
                     ? variant_count(RIME_MODE_CHI2, kRes64)
                     : 1;
  for (int i = 0; i < variant_count(mode, prec); ++i) {
    const Variant *v = variant_info(mode, prec, i);
    for (int f = 0; f < nf; ++f) {
      best = std::max(best, call_ws(plan, mode, prec, i, f, nset, total_src));
      // a batched call with a matrix-core variant runs one set at a time in
      // up to kBatchLanes lanes after a header of domain flags; no set has
      // more than total_src sources
      if (nset > 1 && per_set_variant(plan, mode, prec, *v))
        best = std::max(best, align_up(static_cast<size_t>(dom_words(nset, total_src)) *
                                       sizeof(int32_t)) +
                                  std::min(kBatchLanes, nset) *
                                      align_up(call_ws(plan, mode, prec, i, f, 1, total_src)));
    }
  }
  return best;
}

int64_t sky_nsrc(const rime_sky *sky) {
  return static_cast<int64_t>(sky->npsrc) + sky->ngsrc + sky->nxsrc;
}

// allow_empty: a sky without sources (single-sky calls: V = 0), whose arrays
// may then be NULL.
rime_status check_sky(const rime_sky *sky, bool allow_empty = false) {
  if (!sky) return RIME_ERR_ARG;
  if (sky->npsrc < 0 || sky->ngsrc < 0 || sky->nxsrc < 0) return RIME_ERR_ARG;
  if (sky_nsrc(sky) > (1 << 24)) return RIME_ERR_ARG;
  if (sky_nsrc(sky) == 0) return allow_empty ? RIME_OK : RIME_ERR_ARG;
  if (!sky->lm || !sky->stokes || !sky->alpha) return RIME_ERR_ARG;
  if (sky->ngsrc > 0 && !sky->gshape) return RIME_ERR_ARG;
  if (sky->nxsrc > 0 && !sky->xshape) return RIME_ERR_ARG;
  return RIME_OK;
}

SetDesc set_of(const rime_sky *sky) {
  SetDesc d;
  d.lm = sky->lm;
  d.stokes = sky->stokes;
  d.alpha = sky->alpha;
  d.gshape = sky->gshape;
  d.xshape = sky->xshape;
  d.npsrc = sky->npsrc;
  d.ngsrc = sky->ngsrc;
  d.nxsrc = sky->nxsrc;
  d.src_off = 0;
  return d;
}

KParams base_params(const rime_plan *plan) {
  KParams p;
  std::memset(&p, 0, sizeof(p));
  p.ntime = plan->ntime;
  p.na = plan->na;
  p.nbl = plan->nbl;
  p.nchan = plan->nchan;
  p.uvw = plan->d_uvw;
  p.nu_c = plan->d_nu_c;
  p.lnfr = plan->d_lnfr;
  p.pointing = plan->d_pointing;
  p.gains = plan->d_gains;
  p.beam = plan->beam;
  p.bsc = plan->d_bsc;
  p.bk3 = plan->d_bk3;
  p.clip_r2 = plan->d_clip_r2;
  p.beam_k = plan->beam_k;
  p.beam_clip = plan->beam_clip;
  return p;
}

// One compute call: the sets, the data and the outputs.
struct Call {
  int mode = 0, prec = 0, nset = 1;
  const SetDesc *d_sets = nullptr;  // device [nset] (batched) or nullptr
  SetDesc one{};                    // the single set when d_sets == nullptr
  const int32_t *d_order = nullptr;
  int max_nsrc = 0;
  int64_t total_src = 0;
  const void *data = nullptr, *weight = nullptr;
  void *vis = nullptr;
  double *chi2 = nullptr, *grad = nullptr;
  // domain flags: nullptr for the header of the call's own workspace, else a
  // batch-level header (per-set pipelines) with this call's first flag word
  // and the batch's total word count
  int32_t *dom = nullptr;
  int32_t dom_off = 0, dom_count = 0;
  // per-call terms (single sky only): G_p(t, nu) and its gradient, the
  // brightness per timestep and its gradient
  const double2 *die = nullptr;
  double2 *grad_die = nullptr;
  const double *stokes_t = nullptr;
  double *grad_stokes_t = nullptr;
  int terms() const {
    return (grad_die ? TERM_DIE_GRAD : 0) | (stokes_t ? TERM_STOKES_T : 0) |
           (grad_stokes_t ? TERM_STOKES_T_GRAD : 0);
  }
};

// Kernel parameters of one launch geometry over workspace region `w` laid out
// by L (matrix-core fields set when L enables the engine).
KParams make_params(const rime_plan *plan, const Call &c, const Variant &v, const Geometry &g,
                    const WsLayout &L, char *w) {
  const TileSet &ts = plan->tiles[nbt_slot(v.threads)];
  KParams p = base_params(plan);
  p.nbt = ts.nbt;
  p.nat = ts.nat;
  p.ntile = ts.ntile;
  p.tile_bl = ts.bl;
  p.tile_lpq = ts.lpq;
  p.tile_ant = ts.ant;
  p.tile_nact = ts.nact;
  p.nchb = g.nchb;
  p.tchunk = g.tchunk;
  p.ntc = g.ntc;
  p.items_per_set = g.items_per_set;
  p.nset = c.nset;
  p.sets = c.d_sets;
  p.one = c.one;
  p.order = c.d_order;
  p.src_geo = reinterpret_cast<double4 *>(w + L.geo);
  p.src_lon = reinterpret_cast<double2 *>(w + L.lon);
  p.src_st = w + L.st;
  p.src_gs = w + L.gs;
  if (c.mode == RIME_MODE_CHI2_GRAD) p.bl_rec = w + L.rec;
  p.total_src = c.total_src;
  if (c.dom) {
    p.dom = c.dom;
    p.dom_off = c.dom_off;
    p.dom_count = c.dom_count;
  } else {
    p.dom = reinterpret_cast<int32_t *>(w + L.dom);
    p.dom_off = 0;
    p.dom_count = c.nset * std::max(1, (c.max_nsrc + 255) / 256);
  }
  p.data = c.data;
  p.weight = c.weight;
  p.vis = c.vis;
  p.chi2_part = reinterpret_cast<double2 *>(w + L.chi2);
  p.grad_part = reinterpret_cast<double *>(w + L.grad);
  p.rho_g = w + L.rho_g;
  p.grad_part2 = reinterpret_cast<double *>(w + L.grad2);
  p.grad_chunks = kGradChunk;
  p.grad_nchunk = g.grad_nchunk;
  p.chi2_out = c.chi2;
  p.grad_out = c.grad;
  p.die = c.die;
  p.grad_die = c.grad_die;
  p.ant_off = plan->d_ant_off;
  p.ant_bl = plan->d_ant_bl;
  if (c.grad_die && c.mode == RIME_MODE_CHI2_GRAD)
    p.die_part = reinterpret_cast<double2 *>(w + L.die_part);
  p.stokes_t = c.stokes_t;
  if (c.stokes_t) p.src_sf = w + L.src_sf;
  p.grad_stokes_t = c.grad_stokes_t;
  if (c.grad_stokes_t && c.mode == RIME_MODE_CHI2_GRAD)
    p.gst_part = reinterpret_cast<double *>(w + L.gst);
  p.pme = 0;
  p.pme_adj = 0;
  if (L.pme_tchunk > 0 && c.one.npsrc > 0) {
    p.pme = 1;
    p.nap = plan->nap;
    p.npair = plan->npair;
    p.pair_blk = plan->d_pair_blk;
    p.bl_slot = plan->d_bl_slot;
    p.ngroup = plan->ngroup;
    p.pme_pairs = plan->pme_pairs;
    p.groups = plan->d_groups;
    p.ph_hi = reinterpret_cast<uint32_t *>(w + L.ph_hi);
    p.ph_lo = reinterpret_cast<uint32_t *>(w + L.ph_lo);
    p.spts = reinterpret_cast<double2 *>(w + L.spts);
    p.pme_exp = reinterpret_cast<int32_t *>(w + L.pexp);
    if (L.pme_adj) {
      p.pme_adj = 1;
      p.nblk = plan->nblk;
      p.pair_of = plan->d_pair_of;
      p.pair_mask = plan->d_pair_mask;
      p.rho_t = reinterpret_cast<float2 *>(w + L.rho_t);
      p.pgrad = reinterpret_cast<float *>(w + L.pgrad);
      p.pme_ncg = pme_ncg(plan);
      p.pme_nqr = pme_nqr(plan);
      p.pme_nsr = (c.one.npsrc + kPmeSR - 1) / kPmeSR;
      p.pfin = reinterpret_cast<double2 *>(w + L.pfin);
      p.pme_fchunk = pme_fin_nchunk(
          p.pme_nsr, static_cast<int64_t>(plan->ntime) * p.pme_ncg * plan->nblk * p.pme_nqr);
      p.src_f = reinterpret_cast<float *>(w + L.src_f);
      p.mfrag = reinterpret_cast<uint4 *>(w + L.mfrag);
      p.mscale = reinterpret_cast<float *>(w + L.mscale);
    }
  }
  return p;
}

// The point-source adjoint on the matrix cores, in passes over time that
// each rebuild their phase planes unless `reuse` (one pass whose planes the
// forward left in place).
rime_status enqueue_pme_adjoint(const rime_plan *plan, KParams p, const WsLayout &L, char *w,
                                bool reuse, hipStream_t stream) {
  if (L.ph_k3) p.ph_k3 = reinterpret_cast<float *>(w + L.ph_k3);
  for (int t0 = 0; t0 < plan->ntime; t0 += L.pme_tchunk) {
    p.pme_t0 = t0;
    p.pme_nt = std::min(L.pme_tchunk, plan->ntime - t0);
    RIME_HIP(launch_pme_adjoint(p, !reuse, stream));
  }
  return RIME_OK;
}

// Enqueue one call of the float64-residual mode: float64 forward (chi^2 and,
// for the gradient, the residual), then the float32 adjoint (per-baseline
// kernel, plus the matrix-core engine for point sources).
rime_status enqueue_res64(const rime_plan *plan, const Call &c, int vidx, void *ws,
                          size_t ws_bytes, hipStream_t stream, bool events) {
  const bool grad = c.mode == RIME_MODE_CHI2_GRAD;
  const int fidx = grad ? plan->variant[RIME_MODE_CHI2][kRes64] : vidx;
  const Variant *vf = variant_info(RIME_MODE_CHI2, kRes64, fidx);
  const Variant *va = grad ? variant_info(RIME_MODE_CHI2_GRAD, kRes64, vidx) : nullptr;
  if (!vf || (grad && !va)) return RIME_ERR_UNSUPPORTED;
  const Res64Layout R = res64_layout(plan, c.mode, *vf, va, c.nset, c.total_src, c.terms());
  if (!ws || ws_bytes < R.total) return RIME_ERR_WORKSPACE;
  const Geometry gf = geometry(plan, *vf, c.nset);
  const Geometry ga = grad ? geometry(plan, R.va, c.nset) : Geometry{};
  const int64_t nf = static_cast<int64_t>(c.nset) * gf.items_per_set;
  const int64_t na = static_cast<int64_t>(c.nset) * ga.items_per_set;
  if (nf <= 0 || nf > 0x7fffffff || (grad && (na <= 0 || na > 0x7fffffff)))
    return RIME_ERR_UNSUPPORTED;
  char *w = static_cast<char *>(ws);
  Call cf = c;
  cf.mode = RIME_MODE_CHI2;
  KParams pf = make_params(plan, cf, *vf, gf, R.f, w);
  KParams pa{};
  if (grad) {
    Call ca = c;
    ca.dom = nullptr;
    pa = make_params(plan, ca, R.va, ga, R.a, w + R.a_off);
    pa.dom = nullptr;  // the forward's preparation records the domain
    pa.pme = 0;        // no forward on the matrix cores
    pa.die = nullptr;  // G enters through the forward's residual
    pa.die_part = nullptr;
    pa.rho_b = reinterpret_cast<float2 *>(w + R.rho_b);
    pf.rho_b = pa.rho_b;
    if (c.grad_die) pf.die_part = reinterpret_cast<double2 *>(w + R.f.die_part);
    if (pa.pme_adj) {
      // the forward also stores the residual in the antenna-pair slots
      pf.pme_adj = 1;
      pf.rho_t = pa.rho_t;
      pf.bl_slot = plan->d_bl_slot;
      pf.npair = plan->npair;
    }
  }
  RIME_HIP(launch_prep(pf, true, c.max_nsrc, 0, stream));
  if (grad) RIME_HIP(launch_prep(pa, false, c.max_nsrc, R.va.nc, stream));
  if (events && plan->ev_start) RIME_HIP(hipEventRecord(plan->ev_start, stream));
  if (events && plan->ev_main0) RIME_HIP(hipEventRecord(plan->ev_main0, stream));
  RIME_HIP(launch_resid(fidx, pf, static_cast<int>(nf), stream));
  if (events && plan->ev_main1) RIME_HIP(hipEventRecord(plan->ev_main1, stream));
  if (grad) {
    if (pa.pme_adj) {
      const rime_status st = enqueue_pme_adjoint(plan, pa, R.a, w + R.a_off, false, stream);
      if (st != RIME_OK) return st;
    }
    RIME_HIP(launch_adj(vidx, pa, static_cast<int>(na), stream));
  }
  if (events && plan->ev_stop) RIME_HIP(hipEventRecord(plan->ev_stop, stream));
  RIME_HIP(launch_finalize(pf, RIME_MODE_CHI2, c.max_nsrc, stream, true));
  if (grad) {
    RIME_HIP(launch_finalize(pa, RIME_MODE_CHI2_GRAD, c.max_nsrc, stream, false));
    if (pa.pme_adj) RIME_HIP(launch_pme_finalize(pa, stream));
    if (pf.die_part) RIME_HIP(launch_die_grad(pf, stream));
    if (pa.gst_part) RIME_HIP(launch_stokes_t_grad(pa, stream));
  }
  return RIME_OK;
}

// Enqueue prep + main + finalize for the sets of `c`.
rime_status enqueue(const rime_plan *plan, const Call &c, int vidx, void *ws, size_t ws_bytes,
                    hipStream_t stream, bool events = true) {
  if (c.prec == kRes64) return enqueue_res64(plan, c, vidx, ws, ws_bytes, stream, events);
  const int mode = c.mode, prec = c.prec;
  const Variant *v = variant_info(mode, prec, vidx);
  if (!v) return RIME_ERR_UNSUPPORTED;
  const Geometry g = geometry(plan, *v, c.nset);
  const WsLayout L = ws_layout(plan, mode, prec, g, c.nset, c.total_src, *v, true, c.terms());
  if (L.total > 0 && (!ws || ws_bytes < L.total)) return RIME_ERR_WORKSPACE;
  const int64_t nitems = static_cast<int64_t>(c.nset) * g.items_per_set;
  if (nitems <= 0 || nitems > 0x7fffffff) return RIME_ERR_UNSUPPORTED;
  char *w = static_cast<char *>(ws);
  KParams p = make_params(plan, c, *v, g, L, w);
  RIME_HIP(launch_prep(p, prec == RIME_FP64, c.max_nsrc,
                       mode == RIME_MODE_CHI2_GRAD ? v->nc : 0, stream));
  if (events && plan->ev_start) RIME_HIP(hipEventRecord(plan->ev_start, stream));
  if (p.pme) {
    RIME_HIP(launch_pme_scale(p, stream));
    KParams pf = p;
    // with one pass over time the adjoint reuses the forward's phase planes,
    // which then carry the beam-derivative plane too
    pf.ph_k3 = (L.pme_adj && L.ph_k3 && L.pme_tchunk >= plan->ntime)
                   ? reinterpret_cast<float *>(w + L.ph_k3)
                   : nullptr;
    for (int t0 = 0; t0 < plan->ntime; t0 += L.pme_tchunk) {
      pf.pme_t0 = t0;
      pf.pme_nt = std::min(L.pme_tchunk, plan->ntime - t0);
      RIME_HIP(launch_pme(pf, stream));
    }
  }
  if (events && plan->ev_main0) RIME_HIP(hipEventRecord(plan->ev_main0, stream));
  RIME_HIP(launch_variant(mode, prec, vidx, p, static_cast<int>(nitems), stream));
  if (events && plan->ev_main1) RIME_HIP(hipEventRecord(plan->ev_main1, stream));
  if (p.pme_adj) {
    const rime_status st =
        enqueue_pme_adjoint(plan, p, L, w, L.pme_tchunk >= plan->ntime, stream);
    if (st != RIME_OK) return st;
  }
  if (events && plan->ev_stop) RIME_HIP(hipEventRecord(plan->ev_stop, stream));
  RIME_HIP(launch_finalize(p, mode, c.max_nsrc, stream, true));
  if (p.pme_adj) RIME_HIP(launch_pme_finalize(p, stream));
  if (p.die_part) RIME_HIP(launch_die_grad(p, stream));
  if (p.gst_part) RIME_HIP(launch_stokes_t_grad(p, stream));
  return RIME_OK;
}

bool valid_prec(int prec) { return prec == RIME_FP64 || prec == RIME_MIXED || prec == kRes64; }

rime_status check_terms(const rime_terms *terms, int mode) {
  if (!terms) return RIME_OK;
  if (terms->grad_die && !terms->die) return RIME_ERR_ARG;
  if (terms->grad_stokes_t && !terms->stokes_t) return RIME_ERR_ARG;
  if ((terms->grad_die || terms->grad_stokes_t) && mode != RIME_MODE_CHI2_GRAD) return RIME_ERR_ARG;
  return RIME_OK;
}

rime_status single(const rime_plan *plan, int mode, rime_precision prec, const rime_sky *sky,
                   const void *data, const void *weight, void *vis, double *chi2, double *grad,
                   void *ws, size_t ws_bytes, void *stream, const rime_terms *terms = nullptr) {
  if (!plan) return RIME_ERR_ARG;
  if (!valid_prec(prec)) return RIME_ERR_ARG;
  if (prec == kRes64 && mode == RIME_MODE_PREDICT) return RIME_ERR_UNSUPPORTED;
  rime_status st = check_sky(sky, true);
  if (st != RIME_OK) return st;
  if ((st = check_terms(terms, mode)) != RIME_OK) return st;
  if (mode == RIME_MODE_PREDICT && !vis) return RIME_ERR_ARG;
  if (mode != RIME_MODE_PREDICT && (!data || !weight || !chi2)) return RIME_ERR_ARG;
  // an empty sky has no gradient rows
  if (mode == RIME_MODE_CHI2_GRAD && !grad && sky_nsrc(sky) > 0) return RIME_ERR_ARG;
  Call c;
  c.mode = mode;
  c.prec = prec;
  c.one = set_of(sky);
  c.max_nsrc = static_cast<int>(sky_nsrc(sky));
  c.total_src = c.max_nsrc;
  c.data = data;
  c.weight = weight;
  c.vis = vis;
  c.chi2 = chi2;
  c.grad = grad;
  if (terms) {
    c.die = reinterpret_cast<const double2 *>(terms->die);
    c.grad_die = reinterpret_cast<double2 *>(terms->grad_die);
    c.stokes_t = terms->stokes_t;
    c.grad_stokes_t = terms->grad_stokes_t;
  }
  int dev = 0;
  RIME_HIP(hipGetDevice(&dev));
  if (dev != plan->device) return RIME_ERR_ARG;
  return enqueue(plan, c, plan->variant[mode][prec], ws, ws_bytes,
                 static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// Streamed (out-of-core) evaluation over time chunks
// ---------------------------------------------------------------------------
// A view of `plan` restricted to timesteps [t0, t0 + nt): the same device
// tables, with the time-dependent arrays offset.  Owns nothing.
rime_plan sub_plan(const rime_plan *plan, int t0, int nt) {
  rime_plan v = *plan;
  v.ntime = nt;
  v.d_uvw = plan->d_uvw + static_cast<size_t>(t0) * plan->na * 3;
  v.d_pointing = plan->d_pointing + static_cast<size_t>(t0) * plan->na * 2;
  v.ev_start = v.ev_stop = v.ev_main0 = v.ev_main1 = nullptr;
  return v;
}

struct StreamLayout {
  int chunk_t = 0, nchunk = 0;
  size_t dbytes_t = 0, wbytes_t = 0;   // data and weight bytes per timestep
  size_t hdr = 0, stage[2] = {0, 0}, wstage = 0, part = 0, chunk_off = 0, chunk_ws = 0;
  int64_t stride = 0;                  // doubles per chunk result (chi^2, gradient)
  size_t total = 0;
};

// Workspace of a streamed call: the domain header, two staging buffers of
// chunk_t timesteps of data and weights, the per-chunk results, and one
// chunk-sized call workspace reused by every chunk in stream order.
StreamLayout stream_layout(const rime_plan *plan, int mode, int prec, int64_t nsrc, int chunk_t) {
  StreamLayout S;
  S.chunk_t = std::max(1, std::min(chunk_t, plan->ntime));
  S.nchunk = (plan->ntime + S.chunk_t - 1) / S.chunk_t;
  const size_t vis_t = static_cast<size_t>(plan->nbl) * plan->nchan * 4;
  S.dbytes_t = vis_t * (prec == RIME_FP64 ? 16 : 8);
  S.wbytes_t = vis_t * (prec == RIME_FP64 ? 8 : 4);
  size_t off = 0;
  S.hdr = off;
  off += align_up(static_cast<size_t>(dom_words(1, nsrc)) * sizeof(int32_t));
  S.wstage = align_up(S.chunk_t * S.dbytes_t);
  for (int b = 0; b < 2; ++b) {
    S.stage[b] = off;
    off += S.wstage + align_up(S.chunk_t * S.wbytes_t);
  }
  S.stride = 1 + (mode == RIME_MODE_CHI2_GRAD ? nsrc * 10 : 0);
  S.part = off;
  off += align_up(static_cast<size_t>(S.nchunk) * S.stride * sizeof(double));
  S.chunk_off = off;
  const rime_plan sp = sub_plan(plan, 0, S.chunk_t);
  S.chunk_ws = align_up(ws_max(&sp, mode, prec, 1, nsrc));
  off += S.chunk_ws;
  S.total = off;
  return S;
}

int default_variant(const rime_plan *plan, int mode, int prec) {
  // index layout of the compiled variants: 0 -> 64 threads, 1 -> 256, 2 -> 1024
  // (FP64 adjoint: 1 -> 256 threads x 2 channels with the residual tile in
  // global memory, the fastest on 64 antennas: 93 ms against 137 ms for
  // 2 -> 256 threads x 4 channels);
  // float32-mixed 4 / 5 -> 1024 / 256 threads with the point sources on the
  // matrix cores (measured faster from 64 antennas up); the 1024-thread one
  // for the gradient from 1024 baselines up (2016 baselines: whole call
  // 22.7 ms against 23.0 ms; 19306 baselines: per-baseline kernel 123.7 ms
  // against 150.6 ms); small arrays take 1 in both
  // precisions (7 antennas, 10 timesteps, 16 channels, 20 sources, one graph
  // launch of chi2 + gradient: FP64 30 us against 34 us for 0, float32-mixed
  // 26 us against 28 us for 0 and 75 us for 5).  The float64-residual mode
  // takes the float64 forward 1 and the float32-mixed gradient's adjoint.
  if (prec == RIME_FP64 || plan->nbl <= 96) return 1;
  if (prec == kRes64 && mode != RIME_MODE_CHI2_GRAD) return 1;
  if (mode == RIME_MODE_CHI2_GRAD && plan->nbl >= 1024) return 4;
  return 5;
}

std::string sky_signature(const rime_sky *sky) {
  std::ostringstream o;
  o << "p" << sky->npsrc << "g" << sky->ngsrc << "x" << sky->nxsrc;
  return o.str();
}

std::mutex g_cache_mu;

// Device address of `scratch` on device `dev` (the current device), looked up
// on the first call for that device and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

rime_status scratch_ptr(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return RIME_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&ptr), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return RIME_OK;
}

std::map<std::string, int> read_cache(const char *path) {
  std::map<std::string, int> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while (true) {
    const size_t k0 = s.find('"', i);
    if (k0 == std::string::npos) break;
    const size_t k1 = s.find('"', k0 + 1);
    if (k1 == std::string::npos) break;
    const size_t c = s.find(':', k1);
    if (c == std::string::npos) break;
    m[s.substr(k0 + 1, k1 - k0 - 1)] = std::atoi(s.c_str() + c + 1);
    i = c + 1;
  }
  return m;
}

void write_cache(const char *path, const std::map<std::string, int> &m) {
  std::ofstream f(path);
  f << "{\n";
  size_t n = 0;
  for (const auto &kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++n < m.size() ? ",\n" : "\n");
  f << "}\n";
}

// Antenna blocks of kPmeBlk antennas and the block pairs (P <= Q) that hold
// baselines, for the matrix-core engine.  A baseline (a1, a2) lives in pair
// (min, max) of its blocks at row i (antenna of block P) and column j
// (antenna of block Q); when a1 lies in the later block the tile holds the
// sums of (a2, a1) and the baseline takes their conjugate.
rime_status build_pairs(int na, int nbl, const std::vector<int32_t> &a1,
                        const std::vector<int32_t> &a2, rime_plan *pl) {
  const int nblk = (na + kPmeBlk - 1) / kPmeBlk;
  pl->nap = nblk * kPmeBlk;
  std::vector<int32_t> pair_id(static_cast<size_t>(nblk) * nblk, -1);
  std::vector<int2> pairs;
  std::vector<int32_t> slot(nbl);
  for (int b = 0; b < nbl; ++b) {
    int P = a1[b] / kPmeBlk, Q = a2[b] / kPmeBlk;
    int i = a1[b] % kPmeBlk, j = a2[b] % kPmeBlk, cj = 0;
    if (P > Q) {
      std::swap(P, Q);
      std::swap(i, j);
      cj = 1;
    }
    int &id = pair_id[static_cast<size_t>(P) * nblk + Q];
    if (id < 0) {
      id = static_cast<int32_t>(pairs.size());
      pairs.push_back(make_int2(P, Q));
    }
    slot[b] = (id << 11) | (i << 6) | (j << 1) | cj;
  }
  pl->npair = static_cast<int32_t>(pairs.size());
  pl->nblk = nblk;
  // slot occupancy: the adjoint needs every slot to hold at most one baseline
  std::vector<uint32_t> mask(static_cast<size_t>(pl->npair) * kPmeBlk, 0u);
  pl->pme_adj_ok = true;
  for (int b = 0; b < nbl; ++b) {
    const int id = slot[b] >> 11, i = (slot[b] >> 6) & 31, j = (slot[b] >> 1) & 31;
    uint32_t &w = mask[static_cast<size_t>(id) * kPmeBlk + i];
    if ((w >> j) & 1u) pl->pme_adj_ok = false;
    w |= 1u << j;
  }
  // forward work groups: every Q block with the P blocks of its pairs, two at
  // a time on arrays of more than three blocks, else one at a time (where
  // half of the pairs would be a lone block, the single-block kernel's higher
  // occupancy wins)
  pl->pme_pairs = nblk > 3 ? 1 : 0;
  std::vector<int32_t> groups;
  for (int Q = 0; Q < nblk; ++Q) {
    std::vector<int> ps;
    for (int P = 0; P <= Q; ++P)
      if (pair_id[static_cast<size_t>(P) * nblk + Q] >= 0) ps.push_back(P);
    const size_t step = pl->pme_pairs ? 2 : 1;
    for (size_t x = 0; x < ps.size(); x += step) {
      const int Pa = ps[x], Pb = step == 2 && x + 1 < ps.size() ? ps[x + 1] : -1;
      groups.push_back(Q);
      groups.push_back(Pa);
      groups.push_back(Pb);
      groups.push_back(pair_id[static_cast<size_t>(Pa) * nblk + Q]);
      groups.push_back(Pb >= 0 ? pair_id[static_cast<size_t>(Pb) * nblk + Q] : -1);
    }
  }
  pl->ngroup = static_cast<int32_t>(groups.size() / 5);
  hipError_t e;
  if ((e = upload(&pl->d_groups, groups)) != hipSuccess ||
      (e = upload(&pl->d_pair_blk, pairs)) != hipSuccess ||
      (e = upload(&pl->d_bl_slot, slot)) != hipSuccess ||
      (e = upload(&pl->d_pair_of, pair_id)) != hipSuccess ||
      (e = upload(&pl->d_pair_mask, mask)) != hipSuccess)
    return e == hipErrorOutOfMemory ? RIME_ERR_NOMEM : hip_fail(e);
  return RIME_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *rime_status_string(rime_status s) {
  switch (s) {
    case RIME_OK: return "ok";
    case RIME_ERR_ARG: return "invalid argument";
    case RIME_ERR_WORKSPACE: return "workspace too small";
    case RIME_ERR_HIP: return "HIP runtime error";
    case RIME_ERR_UNSUPPORTED: return "unsupported request";
    case RIME_ERR_NOMEM: return "device allocation failed";
    case RIME_ERR_DOMAIN: return "source outside the domain l^2 + m^2 < 1";
  }
  return "unknown status";
}

int32_t rime_last_hip_error(void) { return g_last_hip; }

rime_status rime_domain_status(const void *ws, size_t ws_bytes, void *stream) {
  if (!ws || ws_bytes < sizeof(int32_t)) return RIME_ERR_ARG;
  RIME_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  int32_t count = 0;
  RIME_HIP(hipMemcpy(&count, ws, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (count < 0 || (static_cast<size_t>(count) + 1) * sizeof(int32_t) > ws_bytes)
    return RIME_ERR_ARG;
  std::vector<int32_t> flags(static_cast<size_t>(count));
  if (count > 0)
    RIME_HIP(hipMemcpy(flags.data(), static_cast<const int32_t *>(ws) + 1,
                       flags.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int32_t f : flags)
    if (f) return RIME_ERR_DOMAIN;
  return RIME_OK;
}

double rime_loglike_const(const double *weight, size_t n) {
  if (!weight) return 0.0;
  // compensated sum of ln(2 pi / w)
  double s = 0.0, c = 0.0;
  const double two_pi = 2.0 * kPi;
  for (size_t i = 0; i < n; ++i) {
    const double x = std::log(two_pi / weight[i]);
    const double t = s + x;
    c += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  return s + c;
}

void rime_plan_destroy(rime_plan *plan) {
  if (!plan) return;
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  if (have && cur != plan->device) (void)hipSetDevice(plan->device);
  if (plan->copy) (void)hipStreamDestroy(plan->copy);
  for (hipEvent_t e : {plan->ev_fork, plan->ev_up[0], plan->ev_up[1], plan->ev_done[0],
                       plan->ev_done[1]})
    if (e) (void)hipEventDestroy(e);
  (void)hipFree(plan->d_uvw);
  (void)hipFree(plan->d_nu_c);
  (void)hipFree(plan->d_lnfr);
  (void)hipFree(plan->d_bsc);
  (void)hipFree(plan->d_bk3);
  (void)hipFree(plan->d_clip_r2);
  (void)hipFree(plan->d_pointing);
  (void)hipFree(plan->d_gains);
  (void)hipFree(plan->d_pair_blk);
  (void)hipFree(plan->d_bl_slot);
  (void)hipFree(plan->d_pair_of);
  (void)hipFree(plan->d_pair_mask);
  (void)hipFree(plan->d_groups);
  (void)hipFree(plan->d_ant_off);
  (void)hipFree(plan->d_ant_bl);
  for (auto &t : plan->tiles) {
    (void)hipFree(t.bl);
    (void)hipFree(t.lpq);
    (void)hipFree(t.ant);
    (void)hipFree(t.nact);
  }
  if (have && cur != plan->device) (void)hipSetDevice(cur);
  delete plan;
}

rime_status rime_plan_create(const rime_obs_desc *obs, rime_plan **out) {
  if (!obs || !out) return RIME_ERR_ARG;
  *out = nullptr;
  if (obs->ntime < 1 || obs->na < 2 || obs->na > 4096 || obs->nbl < 1 || obs->nchan < 1)
    return RIME_ERR_ARG;
  if (!obs->uvw || !obs->freq) return RIME_ERR_ARG;
  if (!(obs->ref_freq > 0)) return RIME_ERR_ARG;
  if ((obs->ant1 == nullptr) != (obs->ant2 == nullptr)) return RIME_ERR_ARG;
  if (obs->beam != 0 && obs->beam != 1) return RIME_ERR_ARG;
  if (obs->beam == 1 && !(obs->beam_ref_freq > 0 && obs->beam_k >= 0 && obs->beam_clip > 0 &&
                          obs->beam_clip <= 1.5))
    return RIME_ERR_ARG;
  if (static_cast<int64_t>(obs->ntime) * obs->nbl * obs->nchan > (int64_t(1) << 40))
    return RIME_ERR_ARG;
  for (int c = 0; c < obs->nchan; ++c)
    if (!(obs->freq[c] > 0)) return RIME_ERR_ARG;
  std::vector<int32_t> a1(obs->nbl), a2(obs->nbl);
  if (!obs->ant1) {
    if (static_cast<int64_t>(obs->nbl) != static_cast<int64_t>(obs->na) * (obs->na - 1) / 2)
      return RIME_ERR_ARG;
    int b = 0;
    for (int p = 0; p < obs->na; ++p)
      for (int q = p + 1; q < obs->na; ++q) {
        a1[b] = p;
        a2[b] = q;
        ++b;
      }
  } else {
    for (int b = 0; b < obs->nbl; ++b) {
      if (obs->ant1[b] < 0 || obs->ant1[b] >= obs->na || obs->ant2[b] < 0 ||
          obs->ant2[b] >= obs->na)
        return RIME_ERR_ARG;
      a1[b] = obs->ant1[b];
      a2[b] = obs->ant2[b];
    }
  }
  rime_plan *pl = new rime_plan;
  hipError_t e = hipGetDevice(&pl->device);
  if (e != hipSuccess) {
    delete pl;
    return hip_fail(e);
  }
  pl->ntime = obs->ntime;
  pl->na = obs->na;
  pl->nbl = obs->nbl;
  pl->nchan = obs->nchan;
  pl->beam = obs->beam;
  pl->ref_freq = obs->ref_freq;
  pl->beam_k = obs->beam == 1 ? obs->beam_k : 0.0;
  pl->beam_clip = obs->beam == 1 ? obs->beam_clip : 0.0;
  const size_t nuvw = static_cast<size_t>(obs->ntime) * obs->na * 3;
  std::vector<double> uvw(obs->uvw, obs->uvw + nuvw);
  std::vector<double> nu_c(obs->nchan), lnfr(obs->nchan), bsc(obs->nchan, 0.0),
      bk3(obs->nchan, 0.0), clip_r2(obs->nchan, 0.0);
  for (int c = 0; c < obs->nchan; ++c) {
    nu_c[c] = obs->freq[c] / kC;
    lnfr[c] = std::log(obs->freq[c] / obs->ref_freq);
    if (obs->beam == 1) {
      const double bfr = obs->freq[c] / obs->beam_ref_freq;
      // the beam argument's scale beam_k nu / beam_ref_freq and the factor
      // -3 bs^2 of its gradient, per channel
      bsc[c] = obs->beam_k * bfr;
      bk3[c] = -3.0 * bsc[c] * bsc[c];
      // radius at which beam_k r nu / beam_ref_freq reaches the clip
      const double rc = obs->beam_k > 0 ? obs->beam_clip / (obs->beam_k * bfr) : 1e300;
      clip_r2[c] = rc * rc;
    }
  }
  std::vector<double> pnt(static_cast<size_t>(obs->ntime) * obs->na * 2, 0.0);
  if (obs->beam == 1 && obs->pointing) std::copy(obs->pointing, obs->pointing + pnt.size(), pnt.begin());
  std::vector<double> gains(static_cast<size_t>(obs->na) * 4);
  for (int a = 0; a < obs->na; ++a) {
    for (int f = 0; f < 2; ++f) {
      gains[4 * a + 2 * f] = obs->gains ? obs->gains[4 * a + 2 * f] : 1.0;
      gains[4 * a + 2 * f + 1] = obs->gains ? obs->gains[4 * a + 2 * f + 1] : 0.0;
    }
  }
  rime_status st = RIME_OK;
  if ((e = upload(&pl->d_uvw, uvw)) != hipSuccess || (e = upload(&pl->d_nu_c, nu_c)) != hipSuccess ||
      (e = upload(&pl->d_lnfr, lnfr)) != hipSuccess ||
      (e = upload(&pl->d_bsc, bsc)) != hipSuccess || (e = upload(&pl->d_bk3, bk3)) != hipSuccess ||
      (e = upload(&pl->d_clip_r2, clip_r2)) != hipSuccess ||
      (e = upload(&pl->d_pointing, pnt)) != hipSuccess ||
      (e = upload(&pl->d_gains, gains)) != hipSuccess) {
    st = e == hipErrorOutOfMemory ? RIME_ERR_NOMEM : hip_fail(e);
  }
  for (int i = 0; i < 3 && st == RIME_OK; ++i)
    st = build_tiles(obs->na, obs->nbl, a1, a2, kNbt[i], pl->tiles[i]);
  if (st == RIME_OK) st = build_pairs(obs->na, obs->nbl, a1, a2, pl);
  if (st == RIME_OK) {
    // the baselines of every antenna, in baseline order (gradient of G)
    std::vector<int32_t> off(obs->na + 1, 0);
    for (int b = 0; b < obs->nbl; ++b) {
      ++off[a1[b] + 1];
      ++off[a2[b] + 1];
    }
    for (int a = 0; a < obs->na; ++a) off[a + 1] += off[a];
    std::vector<int2> lst(static_cast<size_t>(2) * obs->nbl);
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int b = 0; b < obs->nbl; ++b) {
      lst[fill[a1[b]]++] = make_int2(b, 0);
      lst[fill[a2[b]]++] = make_int2(b, 1);
    }
    if ((e = upload(&pl->d_ant_off, off)) != hipSuccess || (e = upload(&pl->d_ant_bl, lst)) != hipSuccess)
      st = e == hipErrorOutOfMemory ? RIME_ERR_NOMEM : hip_fail(e);
  }
  if (st == RIME_OK) {
    // default priority, non-blocking: the streamed calls' upload lane
    if ((e = hipStreamCreateWithFlags(&pl->copy, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming)) != hipSuccess)
      st = hip_fail(e);
    for (int i = 0; i < 2 && st == RIME_OK; ++i)
      if ((e = hipEventCreateWithFlags(&pl->ev_up[i], hipEventDisableTiming)) != hipSuccess ||
          (e = hipEventCreateWithFlags(&pl->ev_done[i], hipEventDisableTiming)) != hipSuccess)
        st = hip_fail(e);
  }
  if (st != RIME_OK) {
    rime_plan_destroy(pl);
    return st;
  }
  for (int m = 0; m < 3; ++m)
    for (int p = 0; p < 3; ++p) pl->variant[m][p] = default_variant(pl, m, p);
  std::ostringstream sig;
  sig << "t" << obs->ntime << "a" << obs->na << "b" << obs->nbl << "c" << obs->nchan << "e"
      << obs->beam;
  pl->signature = sig.str();
  *out = pl;
  return RIME_OK;
}

size_t rime_workspace_size(const rime_plan *plan, rime_mode mode, rime_precision prec,
                           int32_t nset, int64_t total_src) {
  // total_src 0: one empty sky
  if (!plan || nset < 1 || total_src < (nset == 1 ? 0 : nset) || mode < 0 || mode > 2 ||
      !valid_prec(prec))
    return 0;
  return ws_max(plan, mode, prec, nset, total_src);
}

rime_status rime_predict(const rime_plan *plan, const rime_sky *sky, rime_precision prec,
                         void *vis, void *ws, size_t ws_bytes, void *stream) {
  return single(plan, RIME_MODE_PREDICT, prec, sky, nullptr, nullptr, vis, nullptr, nullptr, ws,
                ws_bytes, stream);
}

rime_status rime_chi2(const rime_plan *plan, const rime_sky *sky, rime_precision prec,
                      const void *data, const void *weight, double *chi2, void *ws,
                      size_t ws_bytes, void *stream) {
  return single(plan, RIME_MODE_CHI2, prec, sky, data, weight, nullptr, chi2, nullptr, ws,
                ws_bytes, stream);
}

rime_status rime_chi2_grad(const rime_plan *plan, const rime_sky *sky, rime_precision prec,
                           const void *data, const void *weight, double *chi2, double *grad,
                           void *ws, size_t ws_bytes, void *stream) {
  return single(plan, RIME_MODE_CHI2_GRAD, prec, sky, data, weight, nullptr, chi2, grad, ws,
                ws_bytes, stream);
}

size_t rime_workspace_size_ex(const rime_plan *plan, rime_mode mode, rime_precision prec,
                              int64_t nsrc, const rime_terms *terms) {
  if (!plan || nsrc < 0 || mode < 0 || mode > 2 || !valid_prec(prec) ||
      check_terms(terms, mode) != RIME_OK)
    return 0;
  int bits = 0;
  if (terms)
    bits = (terms->grad_die ? TERM_DIE_GRAD : 0) | (terms->stokes_t ? TERM_STOKES_T : 0) |
           (terms->grad_stokes_t ? TERM_STOKES_T_GRAD : 0);
  size_t best = 0;
  const int nf = prec == kRes64 && mode == RIME_MODE_CHI2_GRAD
                     ? variant_count(RIME_MODE_CHI2, kRes64)
                     : 1;
  for (int i = 0; i < variant_count(mode, prec); ++i)
    for (int f = 0; f < nf; ++f)
      best = std::max(best, call_ws(plan, mode, prec, i, f, 1, nsrc, bits));
  return best;
}

rime_status rime_predict_ex(const rime_plan *plan, const rime_sky *sky, const rime_terms *terms,
                            rime_precision prec, void *vis, void *ws, size_t ws_bytes,
                            void *stream) {
  return single(plan, RIME_MODE_PREDICT, prec, sky, nullptr, nullptr, vis, nullptr, nullptr, ws,
                ws_bytes, stream, terms);
}

rime_status rime_chi2_ex(const rime_plan *plan, const rime_sky *sky, const rime_terms *terms,
                         rime_precision prec, const void *data, const void *weight, double *chi2,
                         double *grad, void *ws, size_t ws_bytes, void *stream) {
  // a gradient call when `grad` is given or a term's gradient is asked for
  // (an empty sky has no `grad` rows)
  const bool g = grad || (terms && (terms->grad_die || terms->grad_stokes_t));
  return single(plan, g ? RIME_MODE_CHI2_GRAD : RIME_MODE_CHI2, prec, sky, data, weight,
                nullptr, chi2, grad, ws, ws_bytes, stream, terms);
}

rime_status rime_chi2_grad_noalloc(const rime_plan *plan, const rime_sky *sky,
                                   rime_precision prec, const void *data, const void *weight,
                                   double *chi2, double *grad, void *stream) {
  if (!plan || !valid_prec(prec)) return RIME_ERR_ARG;
  int dev = 0;
  RIME_HIP(hipGetDevice(&dev));
  if (dev != plan->device) return RIME_ERR_ARG;
  void *ptr = nullptr;
  const rime_status st = scratch_ptr(dev, &ptr);
  if (st != RIME_OK) return st;
  // the call's own checks reject a workspace need above kScratchBytes with
  // RIME_ERR_WORKSPACE before anything is enqueued
  return single(plan, RIME_MODE_CHI2_GRAD, prec, sky, data, weight, nullptr, chi2, grad, ptr,
                kScratchBytes, stream);
}

size_t rime_streamed_workspace_size(const rime_plan *plan, rime_mode mode, rime_precision prec,
                                    int64_t nsrc, int32_t chunk_t) {
  if (!plan || nsrc < 0 || chunk_t < 1 || (mode != RIME_MODE_CHI2 && mode != RIME_MODE_CHI2_GRAD) ||
      !valid_prec(prec))
    return 0;
  return stream_layout(plan, mode, prec, nsrc, chunk_t).total;
}

rime_status rime_chi2_streamed(const rime_plan *plan, const rime_sky *sky, rime_precision prec,
                               const void *data_host, const void *weight_host, double *chi2,
                               double *grad, int32_t chunk_t, void *ws, size_t ws_bytes,
                               void *stream) {
  if (!plan || !data_host || !weight_host || !chi2 || chunk_t < 1 || !valid_prec(prec))
    return RIME_ERR_ARG;
  rime_status st = check_sky(sky, true);
  if (st != RIME_OK) return st;
  const int mode = grad ? RIME_MODE_CHI2_GRAD : RIME_MODE_CHI2;
  const int64_t nsrc = sky_nsrc(sky);
  const StreamLayout S = stream_layout(plan, mode, prec, nsrc, chunk_t);
  if (!ws || ws_bytes < S.total) return RIME_ERR_WORKSPACE;
  int dev = 0;
  RIME_HIP(hipGetDevice(&dev));
  if (dev != plan->device) return RIME_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStream_t c = plan->copy;
  char *w = static_cast<char *>(ws);
  const char *dh = static_cast<const char *>(data_host);
  const char *wh = static_cast<const char *>(weight_host);
  double *part = reinterpret_cast<double *>(w + S.part);
  Call base;
  base.mode = mode;
  base.prec = prec;
  base.one = set_of(sky);
  base.max_nsrc = static_cast<int>(nsrc);
  base.total_src = nsrc;
  // every chunk writes the same domain flags into the call's header
  base.dom = reinterpret_cast<int32_t *>(w + S.hdr);
  base.dom_count = static_cast<int32_t>(std::max<int64_t>(1, (nsrc + 255) / 256));
  // uploads start after earlier work on the caller's stream, which may still
  // be using this workspace
  RIME_HIP(hipEventRecord(plan->ev_fork, s));
  RIME_HIP(hipStreamWaitEvent(c, plan->ev_fork, 0));
  int last_up = -1;
  for (int k = 0; k < S.nchunk && st == RIME_OK; ++k) {
    const int t0 = k * S.chunk_t;
    const int nt = std::min(S.chunk_t, plan->ntime - t0);
    const int b = k & 1;
    char *dst = w + S.stage[b];
    // double buffering: chunk k reuses the buffer of chunk k - 2 once its
    // compute has consumed it; the upload then overlaps chunk k - 1's compute
    hipError_t e = hipSuccess;
    if (k >= 2) e = hipStreamWaitEvent(c, plan->ev_done[b], 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dst, dh + static_cast<size_t>(t0) * S.dbytes_t, nt * S.dbytes_t,
                         hipMemcpyHostToDevice, c);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dst + S.wstage, wh + static_cast<size_t>(t0) * S.wbytes_t,
                         nt * S.wbytes_t, hipMemcpyHostToDevice, c);
    if (e == hipSuccess) e = hipEventRecord(plan->ev_up[b], c);
    if (e != hipSuccess) {
      st = hip_fail(e);
      break;
    }
    last_up = k;
    if ((e = hipStreamWaitEvent(s, plan->ev_up[b], 0)) != hipSuccess) {
      st = hip_fail(e);
      break;
    }
    const rime_plan sp = sub_plan(plan, t0, nt);
    Call cc = base;
    cc.data = dst;
    cc.weight = dst + S.wstage;
    cc.chi2 = part + k * S.stride;
    cc.grad = grad ? part + k * S.stride + 1 : nullptr;
    st = enqueue(&sp, cc, plan->variant[mode][prec], w + S.chunk_off, S.chunk_ws, s, false);
    if (st == RIME_OK && (e = hipEventRecord(plan->ev_done[b], s)) != hipSuccess)
      st = hip_fail(e);
  }
  // the caller's stream always ends after the last upload (also on failure),
  // so that nothing of this call stays unordered with later work on it
  if (last_up >= 0) {
    const hipError_t e = hipStreamWaitEvent(s, plan->ev_up[last_up & 1], 0);
    if (st == RIME_OK && e != hipSuccess) st = hip_fail(e);
  }
  if (st != RIME_OK) return st;
  RIME_HIP(launch_sum_chunks(part, S.nchunk, S.stride, S.stride, chi2, grad, s));
  return RIME_OK;
}

void rime_batch_destroy(rime_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->lane) (void)hipStreamDestroy(b->lane);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  (void)hipFree(b->d_sets);
  (void)hipFree(b->d_order);
  delete b;
}

rime_status rime_batch_create(const rime_plan *plan, int32_t nset, const rime_sky *skies,
                              rime_batch **out) {
  if (!plan || !out || !skies || nset < 1 || nset > (1 << 20)) return RIME_ERR_ARG;
  *out = nullptr;
  std::vector<SetDesc> sets(nset);
  int64_t off = 0;
  int32_t mx = 0;
  for (int i = 0; i < nset; ++i) {
    rime_status st = check_sky(&skies[i]);
    if (st != RIME_OK) return st;
    SetDesc &d = sets[i];
    d = set_of(&skies[i]);
    d.src_off = off;
    const int n = static_cast<int>(sky_nsrc(&skies[i]));
    off += n;
    mx = std::max(mx, n);
  }
  std::vector<int32_t> order(nset);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    // work estimate: an extended source costs about twice a point source
    return sets[x].npsrc + 2 * (sets[x].ngsrc + sets[x].nxsrc) >
           sets[y].npsrc + 2 * (sets[y].ngsrc + sets[y].nxsrc);
  });
  rime_batch *b = new rime_batch;
  b->plan = plan;
  b->nset = nset;
  b->h_sets = sets;
  b->total_src = off;
  b->max_nsrc = mx;
  hipError_t e;
  if ((e = upload(&b->d_sets, sets)) != hipSuccess || (e = upload(&b->d_order, order)) != hipSuccess) {
    rime_batch_destroy(b);
    return e == hipErrorOutOfMemory ? RIME_ERR_NOMEM : hip_fail(e);
  }
  // the second lane of the per-set pipelines and its fork/join events, made
  // here (outside any capture; default priority) so that a call never
  // creates them
  if (nset > 1) {
    if ((e = hipStreamCreateWithFlags(&b->lane, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming)) != hipSuccess) {
      rime_batch_destroy(b);
      return hip_fail(e);
    }
  }
  *out = b;
  return RIME_OK;
}

static int batch_lanes(const rime_batch *b) { return std::min(kBatchLanes, b->nset); }

// Domain-flag words of a batch whose sets run as separate pipelines: a count,
// then each set's preparation workgroups in set order.
static int64_t batch_dom_words(const rime_batch *b) {
  int64_t n = 1;
  for (const SetDesc &d : b->h_sets) n += (d.npsrc + d.ngsrc + d.nxsrc + 255) / 256;
  return n;
}

// Workspace of one batched call with variant vidx: a matrix-core variant runs
// the single-sky pipeline once per set, after a header of domain flags, with
// one set's layout per lane (each reused in stream order); the others run
// all sets in one launch sequence.
static size_t batch_ws(const rime_batch *b, int mode, int prec, int vidx, int fidx) {
  const Variant *v = variant_info(mode, prec, vidx);
  if (!v) return 0;
  if (per_set_variant(b->plan, mode, prec, *v))
    return align_up(static_cast<size_t>(batch_dom_words(b)) * sizeof(int32_t)) +
           batch_lanes(b) * align_up(call_ws(b->plan, mode, prec, vidx, fidx, 1, b->max_nsrc));
  return call_ws(b->plan, mode, prec, vidx, fidx, b->nset, b->total_src);
}

static int batch_variant(const rime_batch *b, int mode, int prec) {
  return b->variant[mode][prec] >= 0 ? b->variant[mode][prec] : b->plan->variant[mode][prec];
}

size_t rime_batch_workspace_size(const rime_batch *b, rime_mode mode, rime_precision prec) {
  if (!b || mode < 0 || mode > 2 || !valid_prec(prec)) return 0;
  size_t best = 0;
  const int nf = prec == kRes64 && mode == RIME_MODE_CHI2_GRAD
                     ? variant_count(RIME_MODE_CHI2, kRes64)
                     : 1;
  for (int i = 0; i < variant_count(mode, prec); ++i)
    for (int f = 0; f < nf; ++f) best = std::max(best, batch_ws(b, mode, prec, i, f));
  return best;
}

rime_status rime_chi2_batched(rime_batch *b, rime_precision prec, const void *data,
                              const void *weight, double *chi2, double *grad, void *ws,
                              size_t ws_bytes, void *stream, int32_t use_graph) {
  if (!b || !data || !weight || !chi2) return RIME_ERR_ARG;
  if (!valid_prec(prec)) return RIME_ERR_ARG;
  const int mode = grad ? RIME_MODE_CHI2_GRAD : RIME_MODE_CHI2;
  const rime_plan *plan = b->plan;
  const int vidx = batch_variant(b, mode, prec);
  const int fidx = plan->variant[RIME_MODE_CHI2][prec];
  const Variant *v = variant_info(mode, prec, vidx);
  if (!v) return RIME_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < batch_ws(b, mode, prec, vidx, fidx)) return RIME_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool per_set = per_set_variant(plan, mode, prec, *v);
  const int lanes = per_set ? batch_lanes(b) : 1;
  Call base;
  base.mode = mode;
  base.prec = prec;
  base.data = data;
  base.weight = weight;
  auto run = [&]() -> rime_status {
    if (!per_set) {
      Call c = base;
      c.nset = b->nset;
      c.d_sets = b->d_sets;
      c.d_order = b->d_order;
      c.max_nsrc = b->max_nsrc;
      c.total_src = b->total_src;
      c.chi2 = chi2;
      c.grad = grad;
      return enqueue(plan, c, vidx, ws, ws_bytes, s);
    }
    // matrix-core variant: the single-sky pipeline per set, set i in lane
    // i % lanes with that lane's part of the workspace (after the batch's
    // domain header); the timing events (if any) bracket the whole sequence
    // on the caller's stream
    const size_t hdr = align_up(static_cast<size_t>(batch_dom_words(b)) * sizeof(int32_t));
    const size_t lane_bytes = align_up(call_ws(plan, mode, prec, vidx, fidx, 1, b->max_nsrc));
    const int32_t nwords = static_cast<int32_t>(batch_dom_words(b) - 1);
    if (plan->ev_start) RIME_HIP(hipEventRecord(plan->ev_start, s));
    if (lanes > 1) {
      RIME_HIP(hipEventRecord(b->fork, s));
      RIME_HIP(hipStreamWaitEvent(b->lane, b->fork, 0));
    }
    rime_status st = RIME_OK;
    int32_t dom_off = 0;
    for (int i = 0; i < b->nset && st == RIME_OK; ++i) {
      Call c = base;
      c.one = b->h_sets[i];
      const int64_t off = c.one.src_off;
      c.one.src_off = 0;
      c.max_nsrc = c.one.npsrc + c.one.ngsrc + c.one.nxsrc;
      c.total_src = c.max_nsrc;
      c.chi2 = chi2 + i;
      c.grad = grad ? grad + off * 10 : nullptr;
      c.dom = static_cast<int32_t *>(ws);
      c.dom_off = dom_off;
      c.dom_count = nwords;
      dom_off += (c.max_nsrc + 255) / 256;
      const int l = i % lanes;
      void *lws = static_cast<char *>(ws) + hdr + l * lane_bytes;
      st = enqueue(plan, c, vidx, lws, lane_bytes, l == 0 ? s : b->lane, false);
    }
    // the lane always joins back, on the error path too, so that nothing of
    // this call stays unordered with later work on the caller's stream (and
    // a capture sees no unjoined fork)
    if (lanes > 1) {
      const hipError_t e1 = hipEventRecord(b->join, b->lane);
      const hipError_t e2 = hipStreamWaitEvent(s, b->join, 0);
      if (st == RIME_OK && e1 != hipSuccess) return hip_fail(e1);
      if (st == RIME_OK && e2 != hipSuccess) return hip_fail(e2);
    }
    if (st != RIME_OK) return st;
    if (plan->ev_stop) RIME_HIP(hipEventRecord(plan->ev_stop, s));
    return RIME_OK;
  };
  if (!use_graph || s == nullptr) return run();
  GraphKey key{data, weight, chi2, grad, ws, ws_bytes, stream, prec, vidx, mode};
  if (!(b->has_graph && b->key == key)) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    if (b->graph) {
      (void)hipGraphDestroy(b->graph);
      b->graph = nullptr;
    }
    b->has_graph = false;
    RIME_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rime_status st = run();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != RIME_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e);
    b->graph = g;
    RIME_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->key = key;
    b->has_graph = true;
  }
  RIME_HIP(hipGraphLaunch(b->exec, s));
  return RIME_OK;
}

rime_status rime_batch_set_variant(rime_batch *b, rime_mode mode, rime_precision prec,
                                   int32_t index) {
  if (!b || (mode != RIME_MODE_CHI2 && mode != RIME_MODE_CHI2_GRAD) || !valid_prec(prec) ||
      !variant_info(mode, prec, index))
    return RIME_ERR_ARG;
  b->variant[mode][prec] = index;
  return RIME_OK;
}

int32_t rime_batch_get_variant(const rime_batch *b, rime_mode mode, rime_precision prec) {
  if (!b || mode < 0 || mode > 2 || !valid_prec(prec)) return -1;
  return batch_variant(b, mode, prec);
}

rime_status rime_batch_autotune(rime_batch *b, rime_mode mode, rime_precision prec,
                                const void *data, const void *weight, void *ws,
                                size_t ws_bytes) {
  if (!b || !data || !weight || (mode != RIME_MODE_CHI2 && mode != RIME_MODE_CHI2_GRAD) ||
      !valid_prec(prec))
    return RIME_ERR_ARG;
  double *chi2 = nullptr, *grad = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(chi2);
    (void)hipFree(grad);
  };
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&chi2), sizeof(double) * b->nset);
  if (e == hipSuccess && mode == RIME_MODE_CHI2_GRAD)
    e = hipMalloc(reinterpret_cast<void **>(&grad), sizeof(double) * 10 * b->total_src);
  if (e == hipSuccess) e = hipStreamCreate(&s);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    cleanup();
    return e == hipErrorOutOfMemory ? RIME_ERR_NOMEM : hip_fail(e);
  }
  const int32_t saved = b->variant[mode][prec];
  float best_ms = 1e30f;
  int best = -1;
  for (int i = 0; i < variant_count(mode, prec); ++i) {
    b->variant[mode][prec] = i;
    rime_status st = rime_chi2_batched(b, prec, data, weight, chi2, grad, ws, ws_bytes, s, 0);
    if (st != RIME_OK) continue;
    (void)hipEventRecord(e0, s);
    st = rime_chi2_batched(b, prec, data, weight, chi2, grad, ws, ws_bytes, s, 0);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || st != RIME_OK) continue;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      best = i;
    }
  }
  cleanup();
  b->variant[mode][prec] = best >= 0 ? best : saved;
  return best >= 0 ? RIME_OK : RIME_ERR_UNSUPPORTED;
}

rime_status rime_tiling_host(int32_t na, int32_t nbl, const int32_t *ant1, const int32_t *ant2,
                             int32_t threads, int32_t max_tiles, int32_t *ntile,
                             int32_t *tile_bl, int32_t *tile_lpq, int32_t *tile_ant) {
  if (na < 2 || nbl < 1 || !ant1 || !ant2 || !ntile || nbt_slot(threads) < 0) return RIME_ERR_ARG;
  std::vector<int32_t> a1(ant1, ant1 + nbl), a2(ant2, ant2 + nbl);
  for (int b = 0; b < nbl; ++b)
    if (a1[b] < 0 || a1[b] >= na || a2[b] < 0 || a2[b] >= na) return RIME_ERR_ARG;
  int nt = 0;
  std::vector<int32_t> hbl, hlpq, hant;
  rime_status st = compute_tiles(na, nbl, a1, a2, threads, nt, hbl, hlpq, hant);
  if (st != RIME_OK) return st;
  *ntile = nt;
  if (nt > max_tiles) return tile_bl ? RIME_ERR_ARG : RIME_OK;
  if (tile_bl) std::copy(hbl.begin(), hbl.end(), tile_bl);
  if (tile_lpq) std::copy(hlpq.begin(), hlpq.end(), tile_lpq);
  if (tile_ant) std::copy(hant.begin(), hant.end(), tile_ant);
  return RIME_OK;
}

rime_status rime_plan_set_main_events(rime_plan *plan, void *start, void *stop) {
  if (!plan || ((start == nullptr) != (stop == nullptr))) return RIME_ERR_ARG;
  plan->ev_main0 = static_cast<hipEvent_t>(start);
  plan->ev_main1 = static_cast<hipEvent_t>(stop);
  return RIME_OK;
}

rime_status rime_plan_set_timing_events(rime_plan *plan, void *start, void *stop) {
  if (!plan || ((start == nullptr) != (stop == nullptr))) return RIME_ERR_ARG;
  plan->ev_start = static_cast<hipEvent_t>(start);
  plan->ev_stop = static_cast<hipEvent_t>(stop);
  return RIME_OK;
}

int32_t rime_variant_matrix_cores(rime_mode mode, rime_precision prec, int32_t index) {
  const Variant *v = variant_info(mode, prec, index);
  return v ? (v->pme ? 1 : 0) : -1;
}

int32_t rime_variant_count(rime_mode mode, rime_precision prec) {
  if (mode < 0 || mode > 2 || !valid_prec(prec)) return 0;
  return variant_count(mode, prec);
}

rime_status rime_variant_info(rime_mode mode, rime_precision prec, int32_t index,
                              int32_t *threads, int32_t *chans_per_thread,
                              int32_t *srcs_per_tile) {
  const Variant *v = variant_info(mode, prec, index);
  if (!v) return RIME_ERR_ARG;
  if (threads) *threads = v->threads;
  if (chans_per_thread) *chans_per_thread = v->nc;
  if (srcs_per_tile) *srcs_per_tile = v->ns;
  return RIME_OK;
}

rime_status rime_set_variant(rime_plan *plan, rime_mode mode, rime_precision prec,
                             int32_t index) {
  if (!plan || !variant_info(mode, prec, index)) return RIME_ERR_ARG;
  plan->variant[mode][prec] = index;
  return RIME_OK;
}

int32_t rime_get_variant(const rime_plan *plan, rime_mode mode, rime_precision prec) {
  if (!plan || mode < 0 || mode > 2 || !valid_prec(prec)) return -1;
  return plan->variant[mode][prec];
}

rime_status rime_autotune(rime_plan *plan, const rime_sky *sky, rime_mode mode,
                          rime_precision prec, const void *data, const void *weight, void *ws,
                          size_t ws_bytes, const char *cache_path) {
  if (!plan || mode < 0 || mode > 2 || !valid_prec(prec))
    return RIME_ERR_ARG;
  rime_status st = check_sky(sky);
  if (st != RIME_OK) return st;
  std::ostringstream k;
  k << plan->signature << "_" << sky_signature(sky) << "_m" << mode << "_p" << prec;
  const std::string key = k.str();
  if (cache_path) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto m = read_cache(cache_path);
    auto it = m.find(key);
    if (it != m.end() && variant_info(mode, prec, it->second)) {
      plan->variant[mode][prec] = it->second;
      return RIME_OK;
    }
  }
  const int nsrc = static_cast<int>(sky_nsrc(sky));
  // scratch outputs for the trial runs
  void *vis = nullptr;
  double *chi2 = nullptr, *grad = nullptr;
  if (mode == RIME_MODE_PREDICT)
    RIME_HIP(hipMalloc(&vis, static_cast<size_t>(plan->ntime) * plan->nbl * plan->nchan * 4 *
                                 (prec == RIME_FP64 ? 16 : 8)));
  RIME_HIP(hipMalloc(reinterpret_cast<void **>(&chi2), sizeof(double)));
  if (mode == RIME_MODE_CHI2_GRAD)
    RIME_HIP(hipMalloc(reinterpret_cast<void **>(&grad), static_cast<size_t>(nsrc) * 10 * sizeof(double)));
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  RIME_HIP(hipStreamCreate(&s));
  RIME_HIP(hipEventCreate(&e0));
  RIME_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  int best = plan->variant[mode][prec];
  const int saved = plan->variant[mode][prec];
  for (int i = 0; i < variant_count(mode, prec); ++i) {
    plan->variant[mode][prec] = i;
    auto call = [&]() {
      return single(plan, mode, prec, sky, data, weight, vis, chi2, grad, ws, ws_bytes, s);
    };
    st = call();  // warm-up (also rejects variants whose workspace does not fit)
    if (st != RIME_OK) continue;
    float ms_min = 1e30f;
    for (int r = 0; r < 3 && st == RIME_OK; ++r) {
      (void)hipEventRecord(e0, s);
      st = call();
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_min = std::min(ms_min, ms);
    }
    if (st == RIME_OK && ms_min < best_ms) {
      best_ms = ms_min;
      best = i;
    }
  }
  (void)hipStreamSynchronize(s);
  plan->variant[mode][prec] = best_ms < 1e29f ? best : saved;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  (void)hipFree(vis);
  (void)hipFree(chi2);
  (void)hipFree(grad);
  if (best_ms >= 1e29f) return RIME_ERR_UNSUPPORTED;
  if (cache_path) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto m = read_cache(cache_path);
    m[key] = best;
    write_cache(cache_path, m);
  }
  return RIME_OK;
}

}  // extern "C"
