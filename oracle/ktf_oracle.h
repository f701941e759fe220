/*
 * ktf_oracle.h -- plain FP64 CPU oracle for Kalman-filter track fitting and
 * building.  TEST INFRASTRUCTURE ONLY: the GPU library never includes,
 * links or calls anything here; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or constant with the GPU path.
 *
 * Method (paper Sec. 2): a Kalman filter (Fruhwirth 1987) propagates each
 * track's state (x, y, z, px, py, pz) and its 6x6 covariance to the next
 * barrel layer and updates it with that layer's 3-D hit; the same
 * propagate + chi2 step scores hit candidates while building (Sec. 3), and
 * the clone-engine ordering (Sec. 3.1) keeps the best N candidates per seed.
 * The paper prints no equations; the filter here is the textbook one with a
 * global-frame 3-D measurement H = [I3 0], and the propagation follows the
 * helix of a charged particle in a uniform field along z, constrained to the
 * layer cylinder.  Every function is one track at a time, scalar, FP64,
 * full 6x6 matrices, no structural shortcuts.
 *
 * Units cm, GeV, tesla.  Packed covariances: 21-value upper triangle in row
 * order (00,01,02,03,04,05,11,...,55).
 */
#ifndef KTF_ORACLE_H
#define KTF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* per-track status bits (same meaning as the library's, defined separately) */
#define ORC_NO_REACH  1u  /* helix never reaches the next layer cylinder   */
#define ORC_S_NOT_PD  2u  /* residual covariance not positive definite     */
#define ORC_NONFINITE 4u  /* non-finite value in state or covariance       */

typedef struct {
  int32_t n_layers;
  const double *radii;    /* [n_layers], increasing */
  double bz;              /* tesla */
  double sigma_r, sigma_rphi, sigma_z;  /* hit resolution (cm) */
  const double *x0;       /* [n_layers] layer thickness in radiation lengths
                             at normal incidence; NULL = no material */
  double eloss;           /* mean energy loss per radiation length of path, GeV */
  double mass;            /* particle mass hypothesis, GeV */
} orc_geom;

typedef struct {
  int32_t max_cands;      /* candidates kept per seed per layer */
  int32_t max_missed;     /* layers a candidate may skip        */
  double chi2_cut;        /* compatibility: chi2 increment < cut */
  int32_t n_seed_layers;  /* layers fitted with the seed's own hits */
} orc_build_params;

/* transport of a state along the helix to the cylinder of radius r.
 * nearest != 0: take the root of smallest |s| (first step onto layer 1);
 * otherwise the smallest s > 0.  Writes the new state, the 6x6 constrained
 * Jacobian d(state at surface)/d(state) (row-major) and the transverse arc
 * length.  Returns 0 or ORC_NO_REACH. */
int orc_propagate(const double x[6], int q, double bz, double r, int nearest,
                  double xo[6], double F[36], double *s_out);

/* transport at a fixed transverse arc length s (no surface constraint) */
void orc_transport(const double x[6], int q, double bz, double s, double xo[6]);

/* material of layer l for a state x on that layer, applied when the track
 * leaves the layer for the next one (paper Sec. 2: the filter is what lets
 * multiple-scattering estimates enter the fit).  With t = x0[l] |p| / |p.n|
 * the path through the layer in radiation lengths (n the radial normal):
 * multiple scattering as process noise Q = theta0^2 (|p|^2 I - p p^T) on the
 * momentum block, theta0 from the Highland formula for unit charge,
 * theta0 = 0.0136 / (beta p) sqrt(t) (1 + 0.038 ln(t / beta^2)); then the
 * mean energy loss eloss * t, which takes |p| to p' = sqrt((E - eloss t)^2
 * - m^2) along the same direction; with T its Jacobian (identity on the
 * position, f (I - u u^T) + (dp'/d|p|) u u^T on the momentum, u = p/|p|,
 * f = p'/|p|, t held fixed): Po = T (P + Q) T^T.  A layer with x0 <= 0, or
 * x0 == NULL, leaves state and covariance unchanged. */
void orc_material(const orc_geom *g, int l, const double x[6], const double P[36],
                  double xo[6], double Po[36]);

/* F P F^T with full 6x6 matrices */
void orc_cov_propagate(const double P[36], const double F[36], double Po[36]);

/* hit covariance: diag(sigma_r^2, sigma_rphi^2, sigma_z^2) in the hit's
 * (radial, tangential, z) frame rotated into global x, y, z */
void orc_hit_cov(const double m[3], double sr, double srphi, double sz, double V[9]);

/* Kalman update with a 3-D hit m of covariance V (symmetric Joseph form).
 * Returns 0 or ORC_S_NOT_PD (outputs untouched then). */
int orc_update(const double xp[6], const double Pp[36], const double m[3],
               const double V[9], double xo[6], double Po[36], double *chi2);

/* chi2 increment of hit m for predicted (xp, Pp); returns 0 or ORC_S_NOT_PD */
int orc_chi2(const double xp[6], const double Pp[36], const double m[3],
             const double V[9], double *chi2);

/* fit of one track over hits[L][3] with valid[L] (NULL = all valid).  The
 * fit ends at the last layer with a valid hit.  P0 and Po are packed 21.
 * Between layers l-1 and l the material of layer l-1 is applied first. */
int orc_fit_track(const orc_geom *g, const double x0[6], const double P0[21], int q,
                  const double *hits, const uint8_t *valid,
                  double xo[6], double Po[21], double *chi2, int32_t *nupd,
                  uint32_t *status);

/* a state on layer `from` carried back to layer 0 along its helix
 * (reversed momentum and charge, one layer at a time), giving back the mean
 * energy lost when leaving each crossed layer.  Returns 0 or ORC_NO_REACH. */
int orc_carry_back(const orc_geom *g, int q, int from, const double x[6], double xo[6]);

/* iterated refit (re-linearisation, a remedy for seeds too poor for one
 * pass of the linearised filter): pass 1 is orc_fit_track; each further
 * pass refits from the previous pass's final state carried back to layer 0
 * (orc_carry_back), with the seed covariance P0.  The result is that of the
 * last pass; the refit stops early, keeping the pass before, when that pass
 * ended non-finite, its state cannot be carried back, or the new pass sets a
 * status bit that the one before did not.  n_passes <= 1: one pass. */
int orc_refit_track(const orc_geom *g, const double x0[6], const double P0[21], int q,
                    const double *hits, const uint8_t *valid, int n_passes,
                    double xo[6], double Po[21], double *chi2, int32_t *nupd, uint32_t *status);

/* batched (re)fit: AoS inputs state[n][6], cov[n][21], q[n], hits[n][L][3],
 * valid[n][L] (may be NULL); outputs AoS.  Tracks split over nthreads. */
void orc_fit_batch(const orc_geom *g, int64_t n, const double *state, const double *cov,
                   const int8_t *q, const double *hits, const uint8_t *valid,
                   double *state_o, double *cov_o, double *chi2_o, int32_t *nupd_o,
                   uint32_t *status_o, int n_passes, int nthreads);

/* hit binning of one layer: zbin = floor((z + zh) * nz / (2 zh)) clamped,
 * phibin = floor((atan2(y,x) + pi) * nphi / (2 pi)) mod nphi, bin = zbin *
 * nphi + phibin; offsets[nz*nphi + 1] (CSR), perm[n] = original index of
 * the hit at each binned position, ordered by (bin, original index). */
void orc_bin_layer(int64_t n, const double *hits /* [n][3] */, double z_half,
                   int32_t nz, int32_t nphi, int32_t *offsets, int32_t *perm);

/* pseudorapidity of a point seen from the origin, -ln tan(theta / 2) */
double orc_eta(const double h[3]);
/* the same binning with rows of pseudorapidity: etabin = floor((eta +
 * eta_max) * neta / (2 eta_max)) clamped to 0 .. neta - 1 */
void orc_bin_layer_eta(int64_t n, const double *hits /* [n][3] */, double eta_max,
                       int32_t neta, int32_t nphi, int32_t *offsets, int32_t *perm);

/* building of one seed by brute force over every hit of each layer.
 * hits: AoS [total][3] of one event; layer_off[L+1].  seed_hit[nsl] are
 * indices within each seed layer's hit list.  Outputs hit_idx[L] (-1 =
 * none), state, packed cov, chi2, nhits, status.  Optional diagnostics:
 * dbg_n[L] candidates alive after each layer, dbg[L][max_cands][2] =
 * (parent rank, hit) of each, and margin[L+1]: margin[l] for l < L the
 * smallest relative gap of a decision taken at layer l (the chi2-total gap
 * between neighbours of equal hit count among the first max_cands + 1
 * records in ranked order, which decides the kept set and its order, or a
 * chi2 increment's distance from the cut, both relative to max(1, value)),
 * margin[L] that of the final choice (the chi2 gap between the chosen
 * candidate and every other ended or surviving candidate of its hit count;
 * infinite when it has no such competitor). */
int orc_build_seed(const orc_geom *g, const orc_build_params *bp, const double *hits,
                   const int64_t *layer_off, const double x0[6], const double P0[21],
                   int q, const int32_t *seed_hit, int32_t *hit_idx, double xo[6],
                   double Po[21], double *chi2, int32_t *nhits, uint32_t *status,
                   int32_t *dbg_n, int32_t *dbg, double *margin);

/* building of many seeds of one event, split over nthreads; per-seed
 * outputs are arrays of the per-seed outputs above (dbg* and margin may be
 * NULL).  Seed inputs AoS: state[n][6], cov[n][21], q[n], seed_hit[n][nsl]. */
void orc_build_event(const orc_geom *g, const orc_build_params *bp, const double *hits,
                     const int64_t *layer_off, int64_t n_seeds, const double *state,
                     const double *cov, const int8_t *q, const int32_t *seed_hit,
                     int32_t *hit_idx, double *state_o, double *cov_o, double *chi2_o,
                     int32_t *nhits_o, uint32_t *status_o, int32_t *dbg_n, int32_t *dbg,
                     double *margin, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
