/*
 * ktf.h -- C-ABI of libktf: batched Kalman-filter track fitting and
 * combinatorial track building on AMD MI355X (gfx950).
 *
 * The problem statement follows the paper's Kalman-filter tracking (Sec. 2):
 * seeds -- "an initial estimate of the track parameters based on a few hits
 * in a subset of the innermost layers" -- and hits on cylindrical barrel
 * layers go in; building (Sec. 3) collects compatible hits layer by layer,
 * keeping the best candidates per seed by chi2 (the clone engine of
 * Sec. 3.1); fitting runs the filter over each track's hits; fitted track
 * parameters, covariances and chi2 come out.
 *
 * Conventions (all calls):
 *  - Units cm, GeV, tesla; the field is uniform along +z.
 *  - Track state (x, y, z, px, py, pz) in the global frame, on the surface of
 *    the layer it was last propagated to.  Covariances are symmetric 6x6
 *    stored as the 21-value upper triangle in row order
 *    (00,01,02,03,04,05,11,12,13,14,15,22,...,55).
 *  - Device arrays are structure-of-arrays, element-major: component c of
 *    track i is at [c * pitch + i], pitch >= n (a multiple of 64 keeps
 *    loads aligned).  Element type is double for KTF_FP64 and float for
 *    KTF_FP32_BULK and KTF_FP32_PROP unless a field says otherwise.
 *  - Every pointer named "device" must be device memory of the current HIP
 *    device; "host" pointers are ordinary host memory.  The caller owns all
 *    buffers it passes; the library owns its context, its workspace and its
 *    staging copies.
 *  - Calls return KTF_OK (0) or a negative error code; ktf_last_error()
 *    returns a message for the last failure on a context.  Problems of a
 *    single track never fail a call: they set bits in its status word.
 */
#ifndef KTF_H
#define KTF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KTF_VERSION_MAJOR 0
#define KTF_VERSION_MINOR 2

#define KTF_MAX_LAYERS 32
#define KTF_MAX_CANDS 16
#define KTF_MAX_PASSES 16

/* return codes */
#define KTF_OK 0
#define KTF_EINVAL (-1)     /* bad argument: null pointer, pitch < n, bad config   */
#define KTF_ENOMEM (-2)     /* device memory or HBM budget exhausted               */
#define KTF_EAGAIN (-3)     /* ktf_poll: result not ready yet                      */
#define KTF_ENOTFOUND (-4)  /* ktf_poll: unknown or already collected ticket       */
#define KTF_EDEVICE (-5)    /* HIP runtime error (message in ktf_last_error)       */

/* per-track status bits */
#define KTF_ST_NO_REACH 1u   /* helix never reaches the next layer: track stops   */
#define KTF_ST_S_NOT_PD 2u   /* residual covariance S not positive definite: hit skipped */
#define KTF_ST_NONFINITE 4u  /* non-finite state or covariance: track stops       */

typedef enum {
  KTF_FP64 = 0,       /* everything in double                                    */
  KTF_FP32_BULK = 1,  /* float storage, float propagation (path solve, transport,
                         Jacobian, F P F^T); the update (S, S^-1, chi2, gain,
                         state and Joseph covariance update) in double           */
  KTF_FP32_PROP = 2   /* float storage and float state propagation (path solve,
                         transport, Jacobian); the covariance is kept in double
                         between layers, so F P F^T and the update run in double.
                         Fused and persistent fits only (a sweep keeps the
                         covariance in HBM in the storage type: KTF_EINVAL);
                         not accepted by ktf_build or ktf_submit               */
} ktf_precision;

typedef enum {
  KTF_FIT_AUTO = 0,        /* fused kernel with the tuned launch shape            */
  KTF_FIT_FUSED = 1,       /* one kernel: all layers of a track in registers      */
  KTF_FIT_PERSISTENT = 2,  /* fused body, persistent blocks pulling track tiles    */
  KTF_FIT_SWEEP = 3,       /* one launch per layer, state round-trips HBM          */
  KTF_FIT_SWEEP_GRAPH = 4  /* the per-layer launches captured once as a hipGraph
                              and replayed                                        */
} ktf_fit_mode;

typedef struct ktf_ctx ktf_ctx;

/* Detector, resolution and building parameters; copied by ktf_create. */
typedef struct {
  int32_t n_layers;        /* 1..KTF_MAX_LAYERS                                  */
  const double *layer_r;   /* host [n_layers], increasing radii (cm)             */
  double z_half;           /* barrel half-length (cm), binning range             */
  double bz;               /* field (T)                                          */
  double sigma_r;          /* radial hit variance term of V (cm), > 0            */
  double sigma_rphi;       /* hit resolution along phi (cm)                      */
  double sigma_z;          /* hit resolution along z (cm)                        */
  int32_t n_zbins;         /* hit bins along z per layer                         */
  int32_t n_phibins;       /* hit bins along phi per layer                       */
  int32_t max_cands;       /* candidates kept per seed per layer, 1..KTF_MAX_CANDS */
  int32_t max_missed;      /* layers a candidate may skip                        */
  int32_t n_seed_layers;   /* innermost layers fitted with the seed's own hits   */
  double chi2_cut;         /* a hit is compatible when its chi2 increment < cut  */
  uint64_t hbm_budget_bytes; /* serving: device bytes the in-flight events may use */
  int32_t max_inflight;    /* serving: events on the device at once              */
  /* Material (Sec. 2: what the Kalman filter lets a fit take into account).
   * When a track leaves layer l for the next one it crosses the layer's
   * material: t = layer_x0[l] |p| / |p.n| radiation lengths (n the radial
   * normal).  Multiple scattering enters as process noise on the momentum,
   * theta0^2 (|p|^2 I - p p^T), theta0 from the Highland formula for unit
   * charge, 0.0136 GeV / (beta p) sqrt(t) (1 + 0.038 ln(t / beta^2)) (meant
   * for 1e-3 <= t <= 100); then the mean energy loss eloss_per_x0 * t moves
   * |p| to sqrt((E - eloss t)^2 - m^2) along the same direction, with the
   * covariance carried by the Jacobian of that map (t held fixed).  No
   * material is applied before the first layer or after the last.        */
  const double *layer_x0;  /* host [n_layers] thickness in radiation lengths at
                              normal incidence, >= 0; NULL = no material       */
  double eloss_per_x0;     /* mean energy loss per radiation length (GeV), >= 0 */
  double mass;             /* particle mass hypothesis (GeV), > 0 when material */
  /* Building: 1 = work on each event's seeds sorted by where their helix
   * meets the first building layer (a Z-order curve over 256 x 32 phi-z
   * cells), so that a wave's candidates search neighbouring hit bins, and
   * stage each wave's box of bins in LDS (the paper's spatial partition of
   * the hits, Sec. 3, with data loaded into local caches, Sec. 3.1); the
   * outputs are returned in the caller's order.  0 = the caller's order,
   * every window read from the binned hits in memory.  Results are the same
   * either way. */
  int32_t seed_order;
  /* Building: > 0 = bin each layer's hits in n_etabins pseudorapidity bins
   * over |eta| < eta_max (eta = asinh(z / rho) of the hit, seen from the
   * origin; beyond, the edge bins) by n_phibins phi bins, the paper's
   * directionally projective partition (Sec. 3: tracks do not bend in eta),
   * in place of n_zbins z bins.  A candidate searches the eta bins that its
   * window (the same conservative bound on every compatible hit) overlaps:
   * the compatible set, and so the result, does not depend on the binning.
   * 0 = z bins. */
  int32_t n_etabins;
  double eta_max;
} ktf_config;

/* Create a context on the current HIP device.  Returns KTF_EINVAL for an
 * invalid config, KTF_EDEVICE when no device is usable. */
int ktf_create(const ktf_config *cfg, ktf_ctx **out);
/* Destroy a context: stops the serving thread (pending tickets are dropped)
 * and frees its device memory.  NULL is accepted. */
int ktf_destroy(ktf_ctx *ctx);
/* Message for the last failed call on ctx (never NULL; "" if none). */
const char *ktf_last_error(const ktf_ctx *ctx);
/* sizeof(ktf_config) as the library was built: ktf_config grows by
 * appended fields from one minor version to the next, and the library
 * reads the whole structure, so a caller checks this against its own
 * sizeof(ktf_config) before ktf_create. */
size_t ktf_config_bytes(void);

/* ---------------------------------------------------------------- fitting
 * Kalman-filter fit (Sec. 2: "repeatedly apply the KF algorithm without
 * branching" over a fixed hit set).  For each track: start from the seed on
 * layer 0's surface, then for l = 0 .. last: propagate along the helix to
 * layer l's cylinder (the first step takes the root of least |s|, so a seed
 * slightly off the surface is projected onto it), propagate the covariance
 * with the surface-constrained Jacobian, and if the track has a hit there
 * update with it.  The fit ends at the track's last layer with a hit.
 */
typedef struct {
  int64_t n;                /* tracks                                            */
  int64_t pitch;            /* >= n                                              */
  ktf_precision prec;
  const void *seed_state;   /* device [6][pitch]                                 */
  const void *seed_cov;     /* device [21][pitch]                                */
  const int8_t *charge;     /* device [pitch], +1 or -1                          */
  const void *hits;         /* device [n_layers][3][pitch]: x, y, z              */
  const uint8_t *hit_valid; /* device [n_layers][pitch], 0 = no hit; NULL = all   */
  int32_t n_passes;         /* 0 or 1: one pass of the filter.  2..KTF_MAX_PASSES:
                               iterated refit, a re-linearisation for seeds too
                               poor for one pass: each further pass refits from
                               the previous pass's result carried back to the
                               first layer (the helix travelled backwards, the
                               mean energy loss given back), with seed_cov.  A
                               pass that sets a status bit the pass before did
                               not is dropped and ends the refit; so do a result
                               that is non-finite or cannot be carried back.
                               Fused and persistent modes, and a double
                               covariance (KTF_FP64, KTF_FP32_PROP) only, else
                               EINVAL: with a float covariance the passes
                               amplify its rounding on poor seeds.          */
} ktf_fit_in;

typedef struct {
  void *state;              /* device [6][pitch]: filtered state at the last layer */
  void *cov;                /* device [21][pitch]                                */
  double *chi2;             /* device [n]: sum of chi2 increments                */
  int32_t *n_upd;           /* device [n]: hits used (ndf = 2 n_upd for a
                               consistent prior)                                */
  uint32_t *status;         /* device [n]: KTF_ST_* bits                         */
} ktf_fit_out;

/* Enqueue a fit on hip_stream (NULL = default stream); returns once the
 * work is enqueued.  Inputs must stay valid until the stream reaches it.
 * Outputs may not alias inputs.  KTF_EINVAL on null pointers or pitch < n.
 * The sweep modes keep per-track scratch in the context: two sweeps on one
 * context must be ordered (same stream, or synchronized by the caller). */
int ktf_fit(ktf_ctx *ctx, const ktf_fit_in *in, ktf_fit_out *out, ktf_fit_mode mode,
            void *hip_stream);

/* Time each launch shape of the fused fit (block size 64..512 x plain or
 * persistent x a register budget of 1, 2 or 3 waves per SIMD x 1 or 2
 * tracks per lane, the two tracks' layers fitted side by side; two per lane
 * only for one pass without material) on the given inputs, in two rounds
 * keeping each shape's faster one, and keep the fastest shape for this
 * precision and size class; KTF_FIT_AUTO then uses it.  The shapes with one
 * track per lane give bit-identical results; two tracks per lane compile the
 * same arithmetic in another context, where the compiler may fuse other
 * multiply-adds, and agree with them to rounding.  Runs synchronously on
 * hip_stream and overwrites out (with the last shape's results). */
int ktf_autotune_fit(ktf_ctx *ctx, const ktf_fit_in *in, ktf_fit_out *out, void *hip_stream);
/* Describe the chosen launch shape for (prec, n) as JSON into buf (block,
 * waves_per_simd, tracks_per_lane, persistent, blocks_per_cu, ms, tuned,
 * and "trials": one [block, waves_per_simd, persistent, tracks_per_lane,
 * ms] per shape tried).  The text is cut at len - 1 characters; 4096 bytes
 * hold every shape. */
int ktf_tuned_shape(ktf_ctx *ctx, ktf_precision prec, int64_t n, char *buf, size_t len);

/* Bytes of the device scratch array behind ktf_fit_noalloc (one copy per
 * GPU, held until the process ends). */
#define KTF_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

/* ktf_fit without any device allocation, for callers that cannot allocate
 * (code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same inputs, outputs, results and stream semantics as
 * ktf_fit; the caller still owns every input and output buffer.  The modes
 * that need scratch take it from a static device array of
 * KTF_NOALLOC_SCRATCH_BYTES per GPU instead of the context's workspace:
 * KTF_FIT_PERSISTENT its tile counter (256 bytes), KTF_FIT_SWEEP per track
 * the end layer (1 byte) and, for KTF_FP32_BULK, the double position (24
 * bytes), i.e. 256 + pitch rounded up to 256 + 24 * pitch bytes in all.
 * KTF_FIT_AUTO, KTF_FIT_FUSED and the iterated refit need none.  Returns
 * KTF_EINVAL for a sweep that does not fit the array (about 1.34 M tracks
 * of float storage, 33 M of double), for KTF_FIT_SWEEP_GRAPH (building a
 * graph allocates), or when the current device is not the context's.
 * Every call on a GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap in time on one GPU race, so order them on one
 * stream or synchronize between them. */
int ktf_fit_noalloc(ktf_ctx *ctx, const ktf_fit_in *in, ktf_fit_out *out, ktf_fit_mode mode,
                    void *hip_stream);

/* --------------------------------------------------------------- building
 * Combinatorial track building with the clone engine (Sec. 3, 3.1), for a
 * batch of independent events.  Per layer the hits are binned (n_zbins x
 * n_phibins over |z| < z_half and phi in [-pi, pi)) so that each candidate
 * only scores hits near its prediction; the compatible set is by definition
 * every hit with chi2 increment < chi2_cut, the bins only accelerate it.
 * Per seed: fit the seed's hits on the first n_seed_layers layers, then for
 * each further layer propagate every live candidate, score the hits, and
 * record (parent, hit, chi2 total, hits + 1); a candidate with no compatible
 * hit records one missed layer while it has fewer than max_missed, else it
 * ends.  Records are ranked by (more hits, lower chi2 total, lower parent
 * rank, lower hit index, missed layer last); the best max_cands are cloned
 * from their parents and updated with their hits.  The result per seed is
 * the best of the survivors and the ended candidates by (more hits, lower
 * chi2, earlier end, lower rank).  Hit indices are positions within the
 * (event, layer) hit list as given.
 */
typedef struct {
  int32_t n_events;
  const int64_t *seed_off;  /* host [n_events+1]: seeds of event e are
                               [seed_off[e], seed_off[e+1])                     */
  const int64_t *hit_off;   /* host [n_events*n_layers+1]: hits of (event e,
                               layer l) are [hit_off[e*L+l], hit_off[e*L+l+1]) */
  int64_t hit_pitch;        /* >= hit_off[n_events*n_layers]                     */
  const void *hits;         /* device [3][hit_pitch]: x, y, z                    */
  int64_t seed_pitch;       /* >= seed_off[n_events]                              */
  const void *seed_state;   /* device [6][seed_pitch]                            */
  const void *seed_cov;     /* device [21][seed_pitch]                           */
  const int8_t *charge;     /* device [seed_pitch]: > 0 positive, else negative
                               (unit charge)                                     */
  const int32_t *seed_hit;  /* device [n_seed_layers][seed_pitch]: index of the
                               seed's hit on each seed layer, -1 = none         */
  ktf_precision prec;
} ktf_event_batch;

typedef struct {
  int32_t *hit_idx;         /* device [n_layers][seed_pitch], -1 = no hit        */
  void *state;              /* device [6][seed_pitch]: the chosen candidate      */
  void *cov;                /* device [21][seed_pitch]                           */
  double *chi2;             /* device [seed_pitch]                               */
  int32_t *n_hits;          /* device [seed_pitch]                               */
  uint32_t *status;         /* device [seed_pitch]                               */
  int32_t *cand_hist;       /* optional device [n_layers][max_cands][2][seed_pitch]:
                               (parent rank, hit) of each candidate kept after
                               each layer, -1 where none; NULL to skip          */
  int32_t *cand_count;      /* optional device [n_layers][seed_pitch]            */
} ktf_build_out;

/* Enqueue building of all events of the batch on hip_stream.  Host offset
 * arrays are read during the call.  Uses context workspace (grown as
 * needed, KTF_ENOMEM when it cannot be); a call first waits for the device
 * work of the previous ktf_build / ktf_bin_hits on the same context, which
 * shares that workspace.  Calls on one context must not overlap in time
 * from several host threads. */
int ktf_build(ktf_ctx *ctx, const ktf_event_batch *ev, ktf_build_out *out, void *hip_stream);

/* Bin the hits of every (event, layer) of a batch: offsets
 * [n_events*n_layers][rows*n_phibins+1] (rows = n_etabins if > 0, else
 * n_zbins; device int32, CSR within each (event, layer)) and perm
 * [hit_pitch] (device int32: original index, within its (event, layer), of
 * the hit at each binned position; binned positions are ordered by (bin,
 * original index)).  A hit with a coordinate that is not a number is kept:
 * in row 0 when its row has no number, in phi bin 0 when x or y is not a
 * number.  Exposed for tests and tools. */
int ktf_bin_hits(ktf_ctx *ctx, const ktf_event_batch *ev, int32_t *offsets, int32_t *perm,
                 void *hip_stream);

/* ---------------------------------------------------------------- serving
 * Continuous batching: events are submitted from host memory as they
 * arrive; a scheduler thread admits queued events while the sum of the
 * in-flight events' device footprints (an estimate of every buffer their
 * building and fit use; the lanes' grow-only workspaces may hold up to
 * twice that) stays within hbm_budget_bytes and fewer than max_inflight
 * events are in flight, runs build + final fit for each admitted group of
 * one precision on its own stream (groups overlap on the device), and
 * returns results through ktf_poll.  Results are identical to running the
 * event alone.  If a group fails to launch, its events are retried one by
 * one, so a failing event fails alone.
 */
typedef struct {
  int64_t n_seeds;
  const int64_t *hit_off;   /* host [n_layers+1]                                 */
  const void *hits;         /* host [3][hit_off[n_layers]] (SoA), double for
                               KTF_FP64, float for KTF_FP32_BULK                 */
  const void *seed_state;   /* host [6][n_seeds], the same type                  */
  const void *seed_cov;     /* host [21][n_seeds], the same type                 */
  const int8_t *charge;     /* host [n_seeds]: > 0 positive, else negative     */
  const int32_t *seed_hit;  /* host [n_seed_layers][n_seeds]                     */
  ktf_precision prec;       /* arithmetic of build and fit for this event and
                               the type of its values (KTF_FP64 or KTF_FP32_BULK) */
} ktf_event_host;

typedef struct {
  int32_t *hit_idx;         /* host [n_layers][n_seeds]                          */
  void *state;              /* host [6][n_seeds]: final fit over the built hits,
                               in the submitted event's type                     */
  void *cov;                /* host [21][n_seeds], the same type                 */
  double *chi2;             /* host [n_seeds]: final fit chi2                    */
  int32_t *n_hits;          /* host [n_seeds]                                    */
  uint32_t *status;         /* host [n_seeds]                                    */
  double t_submit, t_admit, t_done; /* seconds on the library's monotonic clock:
                                       entry of ktf_submit (the copy-in counts),
                                       admission onto a lane, results ready to
                                       collect (copied out of the batch) */
} ktf_result_host;

/* Copy the event into library staging and queue it; returns a ticket.  The
 * caller may free its buffers after return.  KTF_ENOMEM if the event alone
 * exceeds the HBM budget.  Thread-safe. */
int ktf_submit(ktf_ctx *ctx, const ktf_event_host *ev, uint64_t *ticket);
/* Collect a finished event into the caller's host buffers (sized for the
 * event's n_seeds) and forget the ticket.  KTF_EAGAIN while pending,
 * KTF_ENOTFOUND for an unknown ticket.  Thread-safe. */
int ktf_poll(ktf_ctx *ctx, uint64_t ticket, ktf_result_host *out);
/* Seconds on the clock used for t_submit / t_admit / t_done. */
double ktf_now(void);
/* Events queued, in flight and finished-but-uncollected. */
int ktf_serving_stats(ktf_ctx *ctx, int64_t *queued, int64_t *inflight, int64_t *done);
/* Testing hook for failure isolation: the next event submitted on ctx
 * fails when its group is launched, as a launch failure would, before any
 * device work of the group is enqueued (no kernel ever faults); its
 * ktf_poll returns KTF_EDEVICE and the other events of its group are
 * retried alone and complete normally.  Thread-safe. */
int ktf_debug_fail_next_event(ktf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* KTF_H */
