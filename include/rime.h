/*
 * rime.h -- C ABI of the MI355X RIME chi-squared engine (librime.so).
 *
 * The library evaluates the Radio Interferometer Measurement Equation for a
 * parameterised sky of point and Gaussian sources (Perkins et al. 2015,
 * "Montblanc", Section 2.1, eq. 1 with eqs. brightness_term, k_term and
 * e_term), reduces it to the weighted chi-squared of Section 2.3
 * (eq. lhood), and differentiates that chi-squared with respect to every
 * source parameter.
 *
 *   V_tpq(nu) = G_p [ sum_s S_tpqs(nu) e_tps e_tqs K_tps conj(K_tqs) B_s(nu) ] G_q^H
 *   K_tps     = exp(-2 pi i (u l + v m + w (n - 1)) nu / c),  n = sqrt(1 - l^2 - m^2)
 *   B_s(nu)   = (nu / nu_ref)^alpha [[I+Q, U+iV], [U-iV, I-Q]]
 *   e_tps     = cos^3(min(beam_k * |(l,m) - pointing_tp| * nu / beam_ref_freq, beam_clip))
 *   G_p       = diag(g_p0, g_p1)          (constant diagonal complex gain)
 *   S_tpqs    = exp(-(pi^2 / (4 ln 2)) [(u' el + v' em)^2 + R^2 (u' em - v' el)^2])
 *               for Gaussian sources (u' = (u_p - u_q) nu / c),
 *               (1 + (2 pi)^2 [(u' el + v' em)^2 + R^2 (u' em - v' el)^2])^(-3/2)
 *               for exponential disks, 1 for point sources
 *   chi^2     = sum_{t, baseline, nu, corr} w |V - D|^2
 *
 * Conventions shared by every entry point:
 *  - Arrays are dense, row-major, little-endian.  Correlations are ordered
 *    (xx, xy, yx, yy); complex values are interleaved (re, im).
 *  - "host" arrays are read during the call and may be freed afterwards.
 *    "device" arrays are HIP device pointers owned by the caller; they must
 *    stay valid until the work enqueued on `stream` has finished.
 *  - Every compute call is asynchronous on `stream` (a hipStream_t; NULL is
 *    the default stream).  Results are valid once the stream is synchronised.
 *  - Argument validation happens on the host before anything is enqueued; a
 *    non-zero status means nothing was enqueued.  No C++ exception crosses
 *    this boundary.
 *  - Precision RIME_FP64: data/weight/vis are complex128/float64 and all
 *    arithmetic is float64.  RIME_MIXED: data/weight/vis are
 *    complex64/float32; the phase argument (formed error-free and reduced to
 *    [-1/2, 1/2] turns) and the chi-squared and gradient sums across
 *    workgroups are float64; the per-term work is float32, except that the
 *    matrix-core variants (rime_variant_matrix_cores) form the point-source
 *    products from fp16 hi + lo operand pairs (hi*hi + hi*lo + lo*hi, about
 *    22 significant bits) with float32 accumulation.
 *    RIME_MIXED_RES64 (chi-squared and gradient only): data/weight as for
 *    RIME_MIXED; the forward pass (model, residual, chi-squared) is float64
 *    throughout and the adjoint is the float32 one of RIME_MIXED, fed with
 *    the float64 residual.  Its gradient keeps the float32 relative accuracy
 *    when the model fits the data to the noise level, where the float32
 *    model error would otherwise dominate the residual.
 *    Sky parameters are float64 in every precision.
 *  - Sources with l^2 + m^2 >= 1 lie outside the domain of
 *    n = sqrt(1 - l^2 - m^2) (Section 2.1, after eq. k_term).  The sky lives
 *    on the device, so a call does not reject them on the host: their
 *    geometry becomes NaN, which propagates to every output of the call, and
 *    the call records the fact in its workspace; rime_domain_status reports
 *    it (RIME_ERR_DOMAIN) once the call has completed.
 *  - Calls are re-entrant when given distinct workspaces; one batch must not
 *    be used from two host threads at once.
 */
#ifndef RIME_H
#define RIME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rime_status {
  RIME_OK = 0,
  RIME_ERR_ARG = 1,          /* null pointer, bad size, inconsistent dimensions */
  RIME_ERR_WORKSPACE = 2,    /* ws_bytes smaller than rime_workspace_size()    */
  RIME_ERR_HIP = 3,          /* a HIP runtime call failed (see rime_last_hip_error) */
  RIME_ERR_UNSUPPORTED = 4,  /* no kernel variant for this request             */
  RIME_ERR_NOMEM = 5,        /* device allocation inside a create call failed  */
  RIME_ERR_DOMAIN = 6        /* a source has l^2 + m^2 >= 1 (rime_domain_status) */
} rime_status;

typedef enum rime_precision {
  RIME_FP64 = 0,
  RIME_MIXED = 1,
  RIME_MIXED_RES64 = 2       /* float64 forward and residual, float32 adjoint */
} rime_precision;

typedef enum rime_mode {
  RIME_MODE_PREDICT = 0,     /* write model visibilities            */
  RIME_MODE_CHI2 = 1,        /* chi-squared only                    */
  RIME_MODE_CHI2_GRAD = 2    /* chi-squared and its source gradient */
} rime_mode;

/* Observation: the per-observation inputs of Table rime_input (uvw,
 * antenna pairs, frequencies, pointing errors) plus the beam and gain model.
 * All arrays are HOST arrays, copied into the plan by rime_plan_create. */
typedef struct rime_obs_desc {
  int32_t ntime;             /* timesteps, >= 1                                   */
  int32_t na;                /* antennas, 2 .. 4096                               */
  int32_t nbl;               /* baselines, >= 1                                   */
  int32_t nchan;             /* channels, >= 1                                    */
  const int32_t *ant1;       /* host [nbl] antenna p of each baseline, or NULL    */
  const int32_t *ant2;       /* host [nbl] antenna q; NULL with ant1 NULL selects  */
                             /* the canonical p < q row-major order, nbl must then */
                             /* be na (na - 1) / 2                                */
  const double *uvw;         /* host [ntime][na][3] metres                        */
  const double *freq;        /* host [nchan] Hz, > 0                              */
  double ref_freq;           /* spectral-index reference frequency, Hz, > 0       */
  int32_t beam;              /* 0: e = 1; 1: cos^3 beam with pointing errors      */
  const double *pointing;    /* host [ntime][na][2] rad, or NULL (zero); beam == 1 */
  const double *gains;       /* host [na][2][2] (feed, re/im) diagonal gains, or  */
                             /* NULL for unity gains                              */
  double beam_k;             /* 65.0                                              */
  double beam_ref_freq;      /* 1.4e9 Hz                                          */
  double beam_clip;          /* 1.0881 rad; 0 < beam_clip <= 1.5 (RIME_ERR_ARG)   */
} rime_obs_desc;

/* One sky model (one sampler proposal).  Point sources first, then
 * Gaussians, then exponential disks.  All arrays are DEVICE float64 arrays.
 * Single-sky calls (rime_predict, rime_chi2, rime_chi2_grad, their _ex and
 * _noalloc forms, rime_chi2_streamed) accept a sky without sources: all
 * counts 0, the arrays may be NULL; the source sum of eq. 1 is then empty,
 * V = 0, chi^2 = sum w |D|^2, and `grad` (no rows) may be NULL.  Batches and
 * rime_autotune need at least one source per sky (RIME_ERR_ARG). */
typedef struct rime_sky {
  int32_t npsrc;             /* point sources, >= 0                               */
  int32_t ngsrc;             /* Gaussian sources, >= 0                            */
  const double *lm;          /* device [nsrc][2] direction cosines, rad, with      */
                             /* l^2 + m^2 < 1 (see rime_domain_status)            */
  const double *stokes;      /* device [nsrc][4] I, Q, U, V in Jy at ref_freq     */
  const double *alpha;       /* device [nsrc] spectral index                      */
  const double *gshape;      /* device [ngsrc][3] (el, em, R): el = theta_maj sin(pa), */
                             /* em = theta_maj cos(pa), R = theta_min / theta_maj; */
                             /* FWHM in rad; may be NULL when ngsrc == 0          */
  int32_t nxsrc;             /* exponential disks (Sersic index 1), >= 0;         */
                             /* npsrc + ngsrc + nxsrc >= 1                        */
  const double *xshape;      /* device [nxsrc][3] (el, em, R) = (h sin(pa),       */
                             /* h cos(pa), minor/major) with h the scale length   */
                             /* (rad) of exp(-r/h) along the major axis; the shape */
                             /* factor is (1 + (2 pi)^2 [(u' el + v' em)^2 +      */
                             /* R^2 (u' em - v' el)^2])^(-3/2); may be NULL when  */
                             /* nxsrc == 0                                        */
} rime_sky;

typedef struct rime_plan rime_plan;    /* observation resident on one device */
typedef struct rime_batch rime_batch;  /* a fixed set of proposals over one plan */

/* Create a plan on the current HIP device: copies the observation to device
 * memory, derives per-channel constants and builds the baseline tiling.
 * Synchronous.  The plan owns its device memory until rime_plan_destroy. */
rime_status rime_plan_create(const rime_obs_desc *obs, rime_plan **out);
void rime_plan_destroy(rime_plan *plan);

/* Bytes of device workspace that one call of `mode` needs for `nset` sets with
 * `total_src` sources in all (nset = 1 for the single-sky calls, where
 * total_src may be 0; otherwise total_src >= nset).  0 for invalid
 * arguments. */
size_t rime_workspace_size(const rime_plan *plan, rime_mode mode, rime_precision prec,
                           int32_t nset, int64_t total_src);

/* Model visibilities, eq. 1: vis is DEVICE [ntime][nbl][nchan][4] complex
 * (complex128 for RIME_FP64, complex64 for RIME_MIXED; RIME_MIXED_RES64
 * returns RIME_ERR_UNSUPPORTED). */
rime_status rime_predict(const rime_plan *plan, const rime_sky *sky, rime_precision prec,
                         void *vis, void *ws, size_t ws_bytes, void *stream);

/* chi^2 of eq. lhood (without the ln(2 pi / w) constant): data is DEVICE
 * [ntime][nbl][nchan][4] complex, weight DEVICE [ntime][nbl][nchan][4] real
 * (precision as for vis); chi2 is DEVICE double[1]. */
rime_status rime_chi2(const rime_plan *plan, const rime_sky *sky, rime_precision prec,
                      const void *data, const void *weight, double *chi2,
                      void *ws, size_t ws_bytes, void *stream);

/* chi^2 and its gradient: grad is DEVICE double [nsrc][10] with columns
 * d chi^2 / d(l, m, I, Q, U, V, alpha, el, em, R) (the shape columns are the
 * Gaussian's or the disk's, and 0 for point sources).  The model
 * visibilities are never written to memory. */
rime_status rime_chi2_grad(const rime_plan *plan, const rime_sky *sky, rime_precision prec,
                           const void *data, const void *weight, double *chi2, double *grad,
                           void *ws, size_t ws_bytes, void *stream);

/* Per-call terms of eq. 1 beyond the sky model (NULL members are absent):
 *  die           DEVICE [ntime][na][nchan][2][2] complex128 (re, im): the
 *                direction-independent Jones term G_p(t, nu), applied
 *                outside the source sum, V_pq = G_p X_pq G_q^H (eq. 1; the
 *                paper lists it as future work, Section 6).  It replaces the
 *                plan's diagonal gains (fold them into G).
 *  grad_die      DEVICE, same shape: d chi^2 / d Re G + i d chi^2 / d Im G
 *                (gradient calls only; needs die).
 *  stokes_t      DEVICE [ntime][nsrc][4] Stokes I, Q, U, V per timestep (Table
 *                rime_input gives the brightness as an ntime x nsrc array);
 *                replaces the sky's stokes; the spectral index stays per
 *                source.
 *  grad_stokes_t DEVICE [ntime][nsrc][4]: d chi^2 / d stokes_t (gradient
 *                calls only; needs stokes_t); the Stokes columns of `grad`
 *                are then its sum over time. */
typedef struct rime_terms {
  const double *die;
  double *grad_die;
  const double *stokes_t;
  double *grad_stokes_t;
} rime_terms;

/* Workspace of one single-sky call with `terms` (NULL: as rime_workspace_size
 * with nset 1).  0 for invalid arguments. */
size_t rime_workspace_size_ex(const rime_plan *plan, rime_mode mode, rime_precision prec,
                              int64_t nsrc, const rime_terms *terms);
/* rime_predict and rime_chi2 / rime_chi2_grad with per-call terms; terms ==
 * NULL gives the plain calls.  Single sky.  rime_chi2_ex computes chi^2 only
 * when grad is NULL and the terms ask for no gradient (grad_die and
 * grad_stokes_t NULL); otherwise chi^2 and gradients (grad may then be NULL
 * only for a sky without sources). */
rime_status rime_predict_ex(const rime_plan *plan, const rime_sky *sky, const rime_terms *terms,
                            rime_precision prec, void *vis, void *ws, size_t ws_bytes,
                            void *stream);
rime_status rime_chi2_ex(const rime_plan *plan, const rime_sky *sky, const rime_terms *terms,
                         rime_precision prec, const void *data, const void *weight, double *chi2,
                         double *grad, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation):
 * rime_chi2_grad without a workspace argument.  The workspace is a fixed
 * 32 MiB block of device memory inside the library, one per device, held
 * until the process ends; the call allocates nothing.  A call whose
 * workspace need (rime_workspace_size for mode RIME_MODE_CHI2_GRAD, one set,
 * the sky's sources, with the plan's variant) exceeds 32 MiB returns
 * RIME_ERR_WORKSPACE and enqueues nothing.  Every call on one device shares
 * the block: calls that overlap on one device (on different streams, or
 * from different host threads) race and must be serialised by the caller.
 * rime_domain_status is not available for these calls (NaN outputs still
 * mark a source outside the domain).  Arguments otherwise as for
 * rime_chi2_grad. */
rime_status rime_chi2_grad_noalloc(const rime_plan *plan, const rime_sky *sky,
                                   rime_precision prec, const void *data, const void *weight,
                                   double *chi2, double *grad, void *stream);

/* Out-of-core chi^2 (grad == NULL) or chi^2 and gradient, streaming the
 * observed data through the device in time chunks: the paper's subdivision
 * of a problem too large for device memory along time (Section 4 "Scaling the
 * RIME", Fig. async_overlap), with the upload of each chunk overlapping the
 * computation of the previous one.
 *  data_host   HOST [ntime][nbl][nchan][4] complex (complex128 for RIME_FP64,
 *              complex64 otherwise), weight_host HOST [ntime][nbl][nchan][4]
 *              real, read during the call's execution on the device: they
 *              must stay valid and unchanged until `stream` has completed the
 *              call's work.  Page-locked host memory (hipHostMalloc) lets the
 *              uploads run asynchronously; pageable memory gives the same
 *              results without the overlap.
 *  chunk_t     timesteps per chunk (>= 1; clamped to ntime).  Two staging
 *              buffers of chunk_t timesteps live in the workspace, filled on
 *              a stream of the plan's own and consumed on `stream`.
 *  chi2, grad  DEVICE outputs as for rime_chi2_grad: chi^2 is additive over
 *              time, so each chunk's chi^2 and gradient land in the workspace
 *              and one final launch sums them in chunk order (compensated).
 *  ws          DEVICE, rime_streamed_workspace_size bytes.
 * The kernel variant is the plan's for (mode, prec).  Streamed calls on one
 * plan must not be issued from two host threads at once (they share the
 * plan's upload stream and events).  Asynchronous on `stream`. */
size_t rime_streamed_workspace_size(const rime_plan *plan, rime_mode mode, rime_precision prec,
                                    int64_t nsrc, int32_t chunk_t);
rime_status rime_chi2_streamed(const rime_plan *plan, const rime_sky *sky, rime_precision prec,
                               const void *data_host, const void *weight_host, double *chi2,
                               double *grad, int32_t chunk_t, void *ws, size_t ws_bytes,
                               void *stream);

/* Domain check of the last call that used workspace `ws` (Section 2.1: n =
 * sqrt(1 - l^2 - m^2) needs l^2 + m^2 < 1).  Synchronises `stream` (the
 * call's stream), then reads the flags the call wrote at the start of its
 * workspace: RIME_ERR_DOMAIN when a source of any set was outside the domain
 * (that call's outputs are NaN), RIME_OK when none was, RIME_ERR_ARG when
 * `ws` holds no flags (never used by a compute call, or too small),
 * RIME_ERR_HIP on a HIP failure.  Covers rime_predict, rime_chi2,
 * rime_chi2_grad, rime_chi2_streamed and rime_chi2_batched (every set of the
 * batch). */
rime_status rime_domain_status(const void *ws, size_t ws_bytes, void *stream);

/* Batched proposals over one observation.  `skies` is a HOST array of nset
 * sky descriptions whose device pointers and source counts are fixed for the
 * life of the batch (the caller overwrites the parameter values in place
 * between evaluations).  Synchronous; owns a small device table. */
rime_status rime_batch_create(const rime_plan *plan, int32_t nset, const rime_sky *skies,
                              rime_batch **out);
void rime_batch_destroy(rime_batch *batch);

/* chi^2 (and gradient when grad != NULL) of every set in one launch sequence:
 * chi2 DEVICE double[nset]; grad DEVICE double [sum nsrc][10], set-major in
 * the order the sets were given.  With use_graph != 0 the launch sequence is
 * captured into a hipGraph on the first call for a given (data, weight, chi2,
 * grad, ws, stream, precision) and replayed afterwards.  With a matrix-core
 * variant the sets alternate between `stream` and a stream that
 * rime_batch_create makes (default priority, destroyed with the batch); it is
 * forked from and joined back to `stream` by events, so all work of the call
 * is ordered after earlier work on `stream` and before later work on it,
 * also when the call fails part-way. */
rime_status rime_chi2_batched(rime_batch *batch, rime_precision prec, const void *data,
                              const void *weight, double *chi2, double *grad,
                              void *ws, size_t ws_bytes, void *stream, int32_t use_graph);
size_t rime_batch_workspace_size(const rime_batch *batch, rime_mode mode,
                                 rime_precision prec);

/* Variant choice of a batch (mode RIME_MODE_CHI2 or RIME_MODE_CHI2_GRAD):
 * until rime_batch_autotune or rime_batch_set_variant sets one, a batch uses
 * its plan's variant.  rime_batch_autotune times every compiled variant on
 * the batch itself (one untimed and one timed rime_chi2_batched call each,
 * on a private stream; ws as for rime_chi2_batched) and keeps the fastest.
 * Synchronous.  rime_batch_get_variant returns the index in use. */
rime_status rime_batch_autotune(rime_batch *batch, rime_mode mode, rime_precision prec,
                                const void *data, const void *weight, void *ws,
                                size_t ws_bytes);
rime_status rime_batch_set_variant(rime_batch *batch, rime_mode mode, rime_precision prec,
                                   int32_t index);
int32_t rime_batch_get_variant(const rime_batch *batch, rime_mode mode, rime_precision prec);

/* Sum over all weights of ln(2 pi / w): the constant of eq. lhood, so that
 * -2 ln L = chi^2 + rime_loglike_const.  HOST array, n entries. */
double rime_loglike_const(const double *weight, size_t n);

const char *rime_status_string(rime_status s);
/* The last HIP error code seen by this thread (0 if none). */
int32_t rime_last_hip_error(void);

/* Kernel-variant selection.  Every compute call uses the variant chosen
 * here for its (plan, mode, precision); the default is a fixed heuristic.
 * rime_autotune times every compiled variant on the given sky and stores the
 * fastest; with cache_path != NULL the choice is also written to / read from
 * that JSON file, keyed by the problem signature.  Synchronous. */
rime_status rime_autotune(rime_plan *plan, const rime_sky *sky, rime_mode mode,
                          rime_precision prec, const void *data, const void *weight,
                          void *ws, size_t ws_bytes, const char *cache_path);
/* Number of compiled variants for (mode, prec) and their descriptions. */
int32_t rime_variant_count(rime_mode mode, rime_precision prec);
rime_status rime_variant_info(rime_mode mode, rime_precision prec, int32_t index,
                              int32_t *threads, int32_t *chans_per_thread,
                              int32_t *srcs_per_tile);
/* 1 when variant `index` of (mode, prec) forms the point-source sums of a
 * single sky on the matrix cores (the antenna x antenna product of
 * A diag(St'_k) A^H per timestep and channel, fp16 hi/lo-split operands,
 * float32 accumulation within 32 sources, float64 across), 0 when every
 * source goes through the per-baseline kernel, -1 for an invalid index.
 * A batched call with such a variant runs the single-sky pipeline once per
 * set, alternating between two streams (workspace: one set's per stream, as
 * rime_batch_workspace_size counts it; rime_workspace_size with the batch's
 * nset and total source count is never smaller).  For RIME_MIXED_RES64 the
 * chi-squared variants are the float64 forwards and the gradient variants
 * the float32 adjoints (the forward of a gradient call is the plan's
 * RIME_MODE_CHI2 variant of that precision). */
int32_t rime_variant_matrix_cores(rime_mode mode, rime_precision prec, int32_t index);
rime_status rime_set_variant(rime_plan *plan, rime_mode mode, rime_precision prec,
                             int32_t index);
int32_t rime_get_variant(const rime_plan *plan, rime_mode mode, rime_precision prec);

/* Timing hooks.  When start/stop are non-NULL hipEvent_t handles, every later
 * compute call on this plan records them on the call's stream:
 * rime_plan_set_timing_events around all of its compute kernels (the
 * per-baseline kernel and, with a matrix-core variant, the point-source
 * kernels; the small per-source preparation and final-reduction kernels fall
 * outside), rime_plan_set_main_events around the per-baseline kernel alone.
 * NULL turns a hook off.  Used to time the kernels in isolation. */
rime_status rime_plan_set_timing_events(rime_plan *plan, void *start, void *stop);
rime_status rime_plan_set_main_events(rime_plan *plan, void *start, void *stop);

/* Host-only view of the baseline tiling used by the kernels: every baseline
 * index appears in exactly one tile; a tile holds at most `threads`
 * baselines (threads = 64, 256 or 1024) over at most 16, 32 or 64 antennas.
 * Outputs (HOST, may be NULL to query *ntile only): tile_bl [ntile][threads]
 * baseline index or -1, tile_lpq [ntile][threads] local p | (local q << 16),
 * tile_ant [ntile][nat] antenna index or -1.  Returns RIME_ERR_ARG when the
 * outputs are given and *ntile > max_tiles.  Performs no HIP call. */
rime_status rime_tiling_host(int32_t na, int32_t nbl, const int32_t *ant1, const int32_t *ant2,
                             int32_t threads, int32_t max_tiles, int32_t *ntile,
                             int32_t *tile_bl, int32_t *tile_lpq, int32_t *tile_ant);

#ifdef __cplusplus
}
#endif

#endif /* RIME_H */
