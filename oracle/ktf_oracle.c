/*
 * ktf_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see the
 * header).  Written for readability against the method, not for speed:
 * full 6x6 matrices, literal formulas, one track at a time.
 *
 * Parity pins that tie this file to the mathematics live in the tests:
 * the field-free straight line, the closed-form circle, finite differences
 * of the constrained transport, the Joseph form against the simple form,
 * the batch weighted least-squares solution of a linear-Gaussian chain,
 * pull statistics, and brute-force binning checks.
 */
#include "ktf_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define ORC_CLIGHT 0.00299792458 /* GeV per (cm tesla unit-charge) */
#define ORC_MAXL 64
#define ORC_PI 3.14159265358979323846

/* ---------------------------------------------------------------- matrices */

static void unpack21(const double p[21], double P[36]) {
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      P[i * 6 + j] = p[k];
      P[j * 6 + i] = p[k];
      ++k;
    }
}

static void pack21(const double P[36], double p[21]) {
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) p[k++] = P[i * 6 + j];
}

/* C = A * B for n x m times m x p, row-major */
static void matmul(const double *A, const double *B, double *C, int n, int m, int p) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < p; ++j) {
      double acc = 0.0;
      for (int l = 0; l < m; ++l) acc += A[i * m + l] * B[l * p + j];
      C[i * p + j] = acc;
    }
}

static void transpose(const double *A, double *T, int n, int m) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) T[j * n + i] = A[i * m + j];
}

static int all_finite(const double *a, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

/* --------------------------------------------------------------- transport */

/*
 * Equations of motion in a uniform field B along z: the transverse momentum
 * turns at a constant rate per transverse arc length, d(px,py)/ds =
 * (k/pT) (py, -px) with k = c q Bz, so after arc s it has turned by
 * theta = -k s / pT; pz is constant.  Integrating the unit direction
 * (px, py)/pT over the turn gives the position with A = sin(th)/th and
 * C = (1 - cos(th))/th = 2 sin^2(th/2)/th.
 */
static void helix_terms(double th, double *A, double *C) {
  if (th == 0.0) {
    *A = 1.0;
    *C = 0.0;
  } else {
    double h = sin(0.5 * th);
    *A = sin(th) / th;
    *C = 2.0 * h * h / th;
  }
}

/* dA/dth and dC/dth */
static void helix_terms_d(double th, double *dA, double *dC) {
  if (th == 0.0) {
    *dA = 0.0;
    *dC = 0.5;
  } else {
    double h = sin(0.5 * th);
    *dA = (th * cos(th) - sin(th)) / (th * th);
    *dC = (th * sin(th) - 2.0 * h * h) / (th * th);
  }
}

static void transport_k(const double x[6], double k, double s, double xo[6]) {
  double px = x[3], py = x[4], pz = x[5];
  double pt = sqrt(px * px + py * py);
  double th = -k * s / pt;
  double A, C;
  helix_terms(th, &A, &C);
  double sp = s / pt;
  xo[0] = x[0] + sp * (px * A - py * C);
  xo[1] = x[1] + sp * (py * A + px * C);
  xo[2] = x[2] + sp * pz;
  xo[3] = px * cos(th) - py * sin(th);
  xo[4] = py * cos(th) + px * sin(th);
  xo[5] = pz;
}

void orc_transport(const double x[6], int q, double bz, double s, double xo[6]) {
  transport_k(x, ORC_CLIGHT * q * bz, s, xo);
}

/*
 * Propagation to the cylinder of radius r: solve x'(s)^2 + y'(s)^2 = r^2 for
 * the transverse arc length s by Newton's method started at the straight-line
 * root, then transport.  The Jacobian of the map from the starting state to
 * the state on the surface has two parts: the derivative at fixed s (Fs),
 * plus the change of the arc length itself, v * (ds/dx)^T, where v = dT/ds and
 * ds/dx follows from differentiating the surface condition (implicit
 * function theorem).
 */
int orc_propagate(const double x[6], int q, double bz, double r, int nearest,
                  double xo[6], double F[36], double *s_out) {
  const double k = ORC_CLIGHT * q * bz;
  const double px = x[3], py = x[4], pz = x[5];
  const double pt2 = px * px + py * py;
  const double pt = sqrt(pt2);
  if (!(pt > 0.0)) return ORC_NO_REACH;

  if (k != 0.0) { /* the transverse circle must meet the layer circle */
    double cx = x[0] + py / k, cy = x[1] - px / k;
    double d = sqrt(cx * cx + cy * cy);
    double R = pt / fabs(k);
    if (d + R < r || fabs(d - R) > r) return ORC_NO_REACH;
  }

  /* straight-line root */
  double u = (x[0] * px + x[1] * py) / pt;
  double disc = u * u + r * r - (x[0] * x[0] + x[1] * x[1]);
  double s;
  if (disc < 0.0) {
    if (k == 0.0) return ORC_NO_REACH;
    s = -u;
  } else {
    double sq = sqrt(disc);
    if (nearest)
      s = (fabs(-u + sq) <= fabs(-u - sq)) ? -u + sq : -u - sq;
    else
      s = -u + sq;
  }

  /* Newton on g(s) = x'^2 + y'^2 - r^2, g'(s) = 2 (x' px' + y' py') / pT */
  double t[6];
  int converged = 0;
  for (int it = 0; it < 50; ++it) {
    transport_k(x, k, s, t);
    double g = t[0] * t[0] + t[1] * t[1] - r * r;
    double gp = 2.0 * (t[0] * t[3] + t[1] * t[4]) / pt;
    if (gp == 0.0) return ORC_NO_REACH;
    double ds = g / gp;
    s -= ds;
    /* converged when the step is within 1e-12 (1 + |s|) cm: near grazing
     * incidence g' is small and the rounding of g/g' alone reaches ~1e-13 */
    if (fabs(ds) <= 1e-12 * (1.0 + fabs(s))) {
      converged = 1;
      break;
    }
  }
  if (!converged) return ORC_NO_REACH;
  if (!nearest && !(s > 0.0)) return ORC_NO_REACH;
  transport_k(x, k, s, xo);
  if (s_out) *s_out = s;

  /* Fs = d(transport)/d(x, y, z, px, py, pz) at fixed s */
  double th = -k * s / pt, sp = s / pt;
  double A, C, dA, dC;
  helix_terms(th, &A, &C);
  helix_terms_d(th, &dA, &dC);
  double cth = cos(th), sth = sin(th);
  double dth_dpx = -th * px / pt2, dth_dpy = -th * py / pt2;
  double dsp_dpx = -sp * px / pt2, dsp_dpy = -sp * py / pt2;
  double fx = px * A - py * C, fy = py * A + px * C;
  double dfx = px * dA - py * dC, dfy = py * dA + px * dC; /* d/dth */
  double pxo = xo[3], pyo = xo[4];

  double Fs[36];
  memset(Fs, 0, sizeof Fs);
  for (int i = 0; i < 6; ++i) Fs[i * 6 + i] = 1.0;
  Fs[0 * 6 + 3] = dsp_dpx * fx + sp * (A + dfx * dth_dpx);
  Fs[0 * 6 + 4] = dsp_dpy * fx + sp * (-C + dfx * dth_dpy);
  Fs[1 * 6 + 3] = dsp_dpx * fy + sp * (C + dfy * dth_dpx);
  Fs[1 * 6 + 4] = dsp_dpy * fy + sp * (A + dfy * dth_dpy);
  Fs[2 * 6 + 3] = dsp_dpx * pz;
  Fs[2 * 6 + 4] = dsp_dpy * pz;
  Fs[2 * 6 + 5] = sp;
  Fs[3 * 6 + 3] = cth - pyo * dth_dpx;
  Fs[3 * 6 + 4] = -sth - pyo * dth_dpy;
  Fs[4 * 6 + 3] = sth + pxo * dth_dpx;
  Fs[4 * 6 + 4] = cth + pxo * dth_dpy;

  /* v = dT/ds; ds/dx = -(x' dx'/dx + y' dy'/dx) / (x' v0 + y' v1) */
  double v[6] = {pxo / pt, pyo / pt, pz / pt, k * pyo / pt, -k * pxo / pt, 0.0};
  double den = xo[0] * v[0] + xo[1] * v[1];
  if (den == 0.0) return ORC_NO_REACH;
  double w[6];
  for (int j = 0; j < 6; ++j) w[j] = -(xo[0] * Fs[0 * 6 + j] + xo[1] * Fs[1 * 6 + j]) / den;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) F[i * 6 + j] = Fs[i * 6 + j] + v[i] * w[j];
  return 0;
}

void orc_cov_propagate(const double P[36], const double F[36], double Po[36]) {
  double FP[36], Ft[36];
  matmul(F, P, FP, 6, 6, 6);
  transpose(F, Ft, 6, 6);
  matmul(FP, Ft, Po, 6, 6, 6);
}

/* ------------------------------------------------------------------ update */

void orc_hit_cov(const double m[3], double sr, double srphi, double sz, double V[9]) {
  double rho = sqrt(m[0] * m[0] + m[1] * m[1]);
  double c = m[0] / rho, s = m[1] / rho;
  /* columns of R: radial, tangential, z unit vectors at the hit */
  double R[9] = {c, -s, 0.0, s, c, 0.0, 0.0, 0.0, 1.0};
  double D[9] = {sr * sr, 0.0, 0.0, 0.0, srphi * srphi, 0.0, 0.0, 0.0, sz * sz};
  double RD[9], Rt[9];
  matmul(R, D, RD, 3, 3, 3);
  transpose(R, Rt, 3, 3);
  matmul(RD, Rt, V, 3, 3, 3);
}

/* S = H P H^T + V with H = [I3 0]; inverse by adjugate over determinant.
 * Returns 0, or ORC_S_NOT_PD when a leading minor is not positive. */
static int residual_cov_inv(const double Pp[36], const double V[9], double Sinv[9]) {
  double S[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) S[i * 3 + j] = Pp[i * 6 + j] + V[i * 3 + j];
  double m1 = S[0];
  double m2 = S[0] * S[4] - S[1] * S[3];
  double c00 = S[4] * S[8] - S[5] * S[7];
  double c01 = -(S[3] * S[8] - S[5] * S[6]);
  double c02 = S[3] * S[7] - S[4] * S[6];
  double det = S[0] * c00 + S[1] * c01 + S[2] * c02;
  if (!(m1 > 0.0) || !(m2 > 0.0) || !(det > 0.0)) return ORC_S_NOT_PD;
  double adj[9];
  adj[0] = c00;
  adj[3] = c01;
  adj[6] = c02;
  adj[1] = -(S[1] * S[8] - S[2] * S[7]);
  adj[4] = S[0] * S[8] - S[2] * S[6];
  adj[7] = -(S[0] * S[7] - S[1] * S[6]);
  adj[2] = S[1] * S[5] - S[2] * S[4];
  adj[5] = -(S[0] * S[5] - S[2] * S[3]);
  adj[8] = S[0] * S[4] - S[1] * S[3];
  for (int i = 0; i < 9; ++i) Sinv[i] = adj[i] / det;
  return 0;
}

int orc_chi2(const double xp[6], const double Pp[36], const double m[3],
             const double V[9], double *chi2) {
  double Sinv[9];
  if (residual_cov_inv(Pp, V, Sinv)) return ORC_S_NOT_PD;
  double r[3] = {m[0] - xp[0], m[1] - xp[1], m[2] - xp[2]};
  double Sr[3];
  matmul(Sinv, r, Sr, 3, 3, 1);
  *chi2 = r[0] * Sr[0] + r[1] * Sr[1] + r[2] * Sr[2];
  return 0;
}

/*
 * Kalman update: residual r = m - H x', S = H P' H^T + V, K = P' H^T S^-1,
 * x+ = x' + K r, chi2 = r^T S^-1 r, and the covariance in the symmetric
 * Joseph form P+ = (I - K H) P' (I - K H)^T + K V K^T.
 */
int orc_update(const double xp[6], const double Pp[36], const double m[3],
               const double V[9], double xo[6], double Po[36], double *chi2) {
  double Sinv[9];
  if (residual_cov_inv(Pp, V, Sinv)) return ORC_S_NOT_PD;
  double r[3] = {m[0] - xp[0], m[1] - xp[1], m[2] - xp[2]};
  double Sr[3];
  matmul(Sinv, r, Sr, 3, 3, 1);
  *chi2 = r[0] * Sr[0] + r[1] * Sr[1] + r[2] * Sr[2];

  double PHt[18]; /* P' H^T = first three columns of P' */
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 3; ++j) PHt[i * 3 + j] = Pp[i * 6 + j];
  double K[18];
  matmul(PHt, Sinv, K, 6, 3, 3);
  double Kr[6];
  matmul(K, r, Kr, 6, 3, 1);
  for (int i = 0; i < 6; ++i) xo[i] = xp[i] + Kr[i];

  double IKH[36];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) IKH[i * 6 + j] = (i == j ? 1.0 : 0.0) - (j < 3 ? K[i * 3 + j] : 0.0);
  double T1[36], IKHt[36], T2[36];
  matmul(IKH, Pp, T1, 6, 6, 6);
  transpose(IKH, IKHt, 6, 6);
  matmul(T1, IKHt, T2, 6, 6, 6);
  double KV[18], Kt[18], KVKt[36];
  matmul(K, V, KV, 6, 3, 3);
  transpose(K, Kt, 6, 3);
  matmul(KV, Kt, KVKt, 6, 3, 6);
  for (int i = 0; i < 36; ++i) Po[i] = T2[i] + KVKt[i];
  return 0;
}

/* --------------------------------------------------------------------- fit */

void orc_material(const orc_geom *g, int l, const double x[6], const double P[36],
                  double xo[6], double Po[36]) {
  memcpy(xo, x, 6 * sizeof(double));
  memcpy(Po, P, 36 * sizeof(double));
  if (!g->x0 || g->x0[l] <= 0.0) return;
  const double *p = x + 3;
  const double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  const double pmag = sqrt(p2);
  const double r = sqrt(x[0] * x[0] + x[1] * x[1]);
  const double pn = (x[0] * p[0] + x[1] * p[1]) / r; /* momentum along the normal */
  const double t = g->x0[l] * pmag / fabs(pn);
  const double m2 = g->mass * g->mass;
  const double E = sqrt(p2 + m2);
  const double beta = pmag / E;
  const double theta0 = 0.0136 / (beta * pmag) * sqrt(t) * (1.0 + 0.038 * log(t / (beta * beta)));
  /* process noise on the momentum block */
  double Q[36] = {0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      Q[(3 + i) * 6 + 3 + j] = theta0 * theta0 * ((i == j ? p2 : 0.0) - p[i] * p[j]);
  double A[36];
  for (int i = 0; i < 36; ++i) A[i] = P[i] + Q[i];
  /* mean energy loss: |p| -> g(|p|) = sqrt((E - eloss t)^2 - m^2) along the
   * same direction, t held at its value for this state; its Jacobian on the
   * momentum is f (I - u u^T) + g'(|p|) u u^T with u = p/|p|, f = g/|p| and
   * g' = (E - eloss t) |p| / (g E) */
  double f = 1.0, gp = 1.0;
  if (g->eloss > 0.0) {
    const double E2 = E - g->eloss * t;
    const double gm = E2 > g->mass ? sqrt(E2 * E2 - m2) : 0.0;
    f = gm / pmag;
    gp = gm > 0.0 ? E2 * pmag / (gm * E) : 0.0;
  }
  double T[36] = {0}, Tt[36], TA[36];
  for (int i = 0; i < 3; ++i) T[i * 6 + i] = 1.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      T[(3 + i) * 6 + 3 + j] = (i == j ? f : 0.0) + (gp - f) * p[i] * p[j] / p2;
  transpose(T, Tt, 6, 6);
  matmul(T, A, TA, 6, 6, 6);
  matmul(TA, Tt, Po, 6, 6, 6);
  for (int i = 0; i < 3; ++i) xo[3 + i] = f * x[3 + i];
}

/* the fit of one pass; *last = layer of the final state (-1: none) */
static int fit_pass(const orc_geom *g, const double x0[6], const double P0[21], int q,
                    const double *hits, const uint8_t *valid, double xo[6], double Po[21],
                    double *chi2, int32_t *nupd, uint32_t *status, int *last_layer) {
  const int L = g->n_layers;
  int at = -1;
  int last = -1;
  for (int l = 0; l < L; ++l)
    if (!valid || valid[l]) last = l;
  const int L_end = last < 0 ? 1 : last + 1;

  double x[6], P[36];
  memcpy(x, x0, sizeof x);
  unpack21(P0, P);
  double c2sum = 0.0;
  int n = 0;
  uint32_t st = 0;
  for (int l = 0; l < L_end; ++l) {
    double xp[6], F[36], Pp[36], s, xm[6], Pm[36];
    if (l > 0) {
      orc_material(g, l - 1, x, P, xm, Pm);
    } else {
      memcpy(xm, x, sizeof xm);
      memcpy(Pm, P, sizeof Pm);
    }
    if (orc_propagate(xm, q, g->bz, g->radii[l], l == 0, xp, F, &s)) {
      st |= ORC_NO_REACH;
      break;
    }
    at = l;
    orc_cov_propagate(Pm, F, Pp);
    if (!valid || valid[l]) {
      const double *m = hits + 3 * l;
      double V[9], xn[6], Pn[36], c2;
      orc_hit_cov(m, g->sigma_r, g->sigma_rphi, g->sigma_z, V);
      if (orc_update(xp, Pp, m, V, xn, Pn, &c2)) {
        st |= ORC_S_NOT_PD;
        memcpy(x, xp, sizeof x);
        memcpy(P, Pp, sizeof P);
      } else {
        memcpy(x, xn, sizeof x);
        memcpy(P, Pn, sizeof P);
        c2sum += c2;
        ++n;
      }
    } else {
      memcpy(x, xp, sizeof x);
      memcpy(P, Pp, sizeof P);
    }
    if (!all_finite(x, 6) || !all_finite(P, 36)) {
      st |= ORC_NONFINITE;
      break;
    }
  }
  memcpy(xo, x, sizeof x);
  pack21(P, Po);
  *chi2 = c2sum;
  *nupd = n;
  *status = st;
  *last_layer = at;
  return (int)st;
}

int orc_fit_track(const orc_geom *g, const double x0[6], const double P0[21], int q,
                  const double *hits, const uint8_t *valid,
                  double xo[6], double Po[21], double *chi2, int32_t *nupd,
                  uint32_t *status) {
  int last;
  return fit_pass(g, x0, P0, q, hits, valid, xo, Po, chi2, nupd, status, &last);
}

int orc_carry_back(const orc_geom *g, int q, int from, const double x[6], double xo[6]) {
  double cur[6];
  memcpy(cur, x, sizeof cur);
  for (int l = from - 1; l >= 0; --l) {
    /* the same helix travelled backwards: reversed momentum, opposite charge */
    double xr[6] = {cur[0], cur[1], cur[2], -cur[3], -cur[4], -cur[5]}, xp[6], F[36], s;
    if (orc_propagate(xr, -q, g->bz, g->radii[l], 1, xp, F, &s)) return (int)ORC_NO_REACH;
    for (int i = 0; i < 3; ++i) {
      cur[i] = xp[i];
      cur[3 + i] = -xp[3 + i];
    }
    /* give back the mean energy lost when leaving layer l */
    if (g->x0 && g->x0[l] > 0.0 && g->eloss > 0.0) {
      const double *p = cur + 3;
      const double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2], pm = sqrt(p2);
      const double r = sqrt(cur[0] * cur[0] + cur[1] * cur[1]);
      const double t = g->x0[l] * pm / fabs((cur[0] * p[0] + cur[1] * p[1]) / r);
      const double E = sqrt(p2 + g->mass * g->mass) + g->eloss * t;
      const double f = sqrt(E * E - g->mass * g->mass) / pm;
      for (int i = 0; i < 3; ++i) cur[3 + i] *= f;
    }
  }
  memcpy(xo, cur, sizeof cur);
  return 0;
}

int orc_refit_track(const orc_geom *g, const double x0[6], const double P0[21], int q,
                    const double *hits, const uint8_t *valid, int n_passes,
                    double xo[6], double Po[21], double *chi2, int32_t *nupd, uint32_t *status) {
  double seed[6];
  memcpy(seed, x0, sizeof seed);
  int last;
  fit_pass(g, seed, P0, q, hits, valid, xo, Po, chi2, nupd, status, &last);
  for (int pass = 1; pass < n_passes; ++pass) {
    if ((*status & ORC_NONFINITE) || last < 0 || orc_carry_back(g, q, last, xo, seed)) break;
    double x2[6], P2[21], c2;
    int32_t n2;
    uint32_t st2;
    int last2;
    fit_pass(g, seed, P0, q, hits, valid, x2, P2, &c2, &n2, &st2, &last2);
    if (st2 != 0 && *status == 0) break; /* a clean pass is not replaced by a failed one */
    memcpy(xo, x2, sizeof x2);
    memcpy(Po, P2, sizeof P2);
    *chi2 = c2;
    *nupd = n2;
    *status = st2;
    last = last2;
  }
  return (int)*status;
}

typedef struct {
  const orc_geom *g;
  int64_t lo, hi;
  const double *state, *cov, *hits;
  const int8_t *q;
  const uint8_t *valid;
  double *state_o, *cov_o, *chi2_o;
  int32_t *nupd_o;
  uint32_t *status_o;
  int n_passes;
} fit_job;

static void *fit_worker(void *arg) {
  fit_job *j = (fit_job *)arg;
  const int L = j->g->n_layers;
  for (int64_t i = j->lo; i < j->hi; ++i)
    orc_refit_track(j->g, j->state + 6 * i, j->cov + 21 * i, j->q[i], j->hits + (int64_t)3 * L * i,
                    j->valid ? j->valid + (int64_t)L * i : NULL, j->n_passes, j->state_o + 6 * i,
                    j->cov_o + 21 * i, j->chi2_o + i, j->nupd_o + i, j->status_o + i);
  return NULL;
}

void orc_fit_batch(const orc_geom *g, int64_t n, const double *state, const double *cov,
                   const int8_t *q, const double *hits, const uint8_t *valid,
                   double *state_o, double *cov_o, double *chi2_o, int32_t *nupd_o,
                   uint32_t *status_o, int n_passes, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  fit_job jobs[256];
  for (int t = 0; t < nthreads; ++t) {
    fit_job j = {g, n * t / nthreads, n * (t + 1) / nthreads, state, cov, hits, q, valid,
                 state_o, cov_o, chi2_o, nupd_o, status_o, n_passes};
    jobs[t] = j;
  }
  if (nthreads == 1) {
    fit_worker(&jobs[0]);
    return;
  }
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, fit_worker, &jobs[t]);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ----------------------------------------------------------------- binning */

typedef struct {
  int32_t bin, idx;
} bin_key;

static int cmp_bin_key(const void *a, const void *b) {
  const bin_key *x = (const bin_key *)a, *y = (const bin_key *)b;
  if (x->bin != y->bin) return x->bin < y->bin ? -1 : 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

/* A hit with a coordinate that is not a number has no place in a bin
 * formula; it goes to the first z (eta) row and phi bin 0, so that it is
 * kept, and no window reaches it in a way that matters: its chi2 is not
 * below any cut. */
static int32_t phi_bin(const double *h, int32_t nphi) {
  double phi = atan2(h[1], h[0]);
  double pf = floor((phi + ORC_PI) * nphi / (2.0 * ORC_PI));
  if (!(pf == pf)) return 0;
  int32_t pb = (int32_t)pf;
  return ((pb % nphi) + nphi) % nphi;
}

static int32_t row_of(double f, int32_t nrows) {
  return f >= 0.0 ? (f > nrows - 1 ? nrows - 1 : (int32_t)f) : 0;
}

static void bin_sort(int64_t n, bin_key *keys, int32_t nb, int32_t *offsets, int32_t *perm);

void orc_bin_layer(int64_t n, const double *hits, double z_half, int32_t nz, int32_t nphi,
                   int32_t *offsets, int32_t *perm) {
  bin_key *keys = (bin_key *)malloc(sizeof(bin_key) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    const double *h = hits + 3 * i;
    int32_t zb = row_of(floor((h[2] + z_half) * nz / (2.0 * z_half)), nz);
    keys[i].bin = zb * nphi + phi_bin(h, nphi);
    keys[i].idx = (int32_t)i;
  }
  bin_sort(n, keys, nz * nphi, offsets, perm);
  free(keys);
}

/* pseudorapidity of a hit seen from the origin: eta = -ln tan(theta / 2)
 * with theta the polar angle, i.e. sinh(eta) = cot(theta) = z / rho */
double orc_eta(const double h[3]) { return asinh(h[2] / sqrt(h[0] * h[0] + h[1] * h[1])); }

void orc_bin_layer_eta(int64_t n, const double *hits, double eta_max, int32_t neta, int32_t nphi,
                       int32_t *offsets, int32_t *perm) {
  bin_key *keys = (bin_key *)malloc(sizeof(bin_key) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    const double *h = hits + 3 * i;
    int32_t eb = row_of(floor((orc_eta(h) + eta_max) * neta / (2.0 * eta_max)), neta);
    keys[i].bin = eb * nphi + phi_bin(h, nphi);
    keys[i].idx = (int32_t)i;
  }
  bin_sort(n, keys, neta * nphi, offsets, perm);
  free(keys);
}

/* hits sorted by (bin, original index) and the CSR offsets of the bins */
static void bin_sort(int64_t n, bin_key *keys, int32_t nb, int32_t *offsets, int32_t *perm) {
  for (int32_t b = 0; b <= nb; ++b) offsets[b] = 0;
  qsort(keys, (size_t)n, sizeof(bin_key), cmp_bin_key);
  for (int64_t i = 0; i < n; ++i) {
    perm[i] = keys[i].idx;
    offsets[keys[i].bin + 1] += 1;
  }
  for (int32_t b = 0; b < nb; ++b) offsets[b + 1] += offsets[b];
}

/* ---------------------------------------------------------------- building */

typedef struct {
  double x[6], P[36];
  double chi2;
  int32_t nh, nm, status;
  int32_t hit[ORC_MAXL];
} orc_cand;

typedef struct {
  double chi2;      /* chi2 total after taking the hit */
  int32_t nh, nm;   /* hit count and missed-layer count after the step */
  int32_t parent;   /* rank of the parent candidate */
  int32_t hit;      /* hit index within the layer, -1 = missed layer */
} orc_rec;

/* ranking: more hits first, then lower chi2, then lower parent rank, then
 * lower hit index with a missed layer after every real hit */
static int cmp_rec(const void *a, const void *b) {
  const orc_rec *x = (const orc_rec *)a, *y = (const orc_rec *)b;
  if (x->nh != y->nh) return x->nh > y->nh ? -1 : 1;
  if (x->chi2 != y->chi2) return x->chi2 < y->chi2 ? -1 : 1;
  if (x->parent != y->parent) return x->parent < y->parent ? -1 : 1;
  uint32_t hx = (uint32_t)x->hit, hy = (uint32_t)y->hit; /* -1 sorts last */
  return (hx > hy) - (hx < hy);
}

/* final choice among finished and surviving candidates: more hits, lower
 * chi2, earlier end layer, lower rank at the end */
typedef struct {
  int32_t nh;
  double chi2;
  int32_t end_layer, rank;
} orc_final_key;

static int better_final(const orc_final_key *a, const orc_final_key *b) {
  if (a->nh != b->nh) return a->nh > b->nh;
  if (a->chi2 != b->chi2) return a->chi2 < b->chi2;
  if (a->end_layer != b->end_layer) return a->end_layer < b->end_layer;
  return a->rank < b->rank;
}

static double rel_gap(double a, double b) {
  double d = fabs(a - b);
  double s = fabs(a) > 1.0 ? fabs(a) : 1.0;
  return d / s;
}

int orc_build_seed(const orc_geom *g, const orc_build_params *bp, const double *hits,
                   const int64_t *layer_off, const double x0[6], const double P0[21],
                   int q, const int32_t *seed_hit, int32_t *hit_idx, double xo[6],
                   double Po[21], double *chi2, int32_t *nhits, uint32_t *status,
                   int32_t *dbg_n, int32_t *dbg, double *margin) {
  const int L = g->n_layers;
  const int NC = bp->max_cands;
  const int NSL = bp->n_seed_layers;
  orc_cand *cur = (orc_cand *)calloc((size_t)NC, sizeof(orc_cand));
  orc_cand *nxt = (orc_cand *)calloc((size_t)NC, sizeof(orc_cand));
  orc_cand *prop = (orc_cand *)calloc((size_t)NC, sizeof(orc_cand)); /* propagated parents */
  int *prop_ok = (int *)calloc((size_t)NC, sizeof(int));
  size_t rec_cap = 256, nrec = 0;
  orc_rec *rec = (orc_rec *)malloc(rec_cap * sizeof(orc_rec));
  orc_cand best;
  orc_final_key best_key = {-1, 0.0, 0, 0};
  int have_best = 0;
  uint32_t st = 0;

  if (dbg_n)
    for (int l = 0; l < L; ++l) dbg_n[l] = 0;
  if (dbg)
    for (int i = 0; i < L * NC * 2; ++i) dbg[i] = -1;
  if (margin)
    for (int l = 0; l <= L; ++l) margin[l] = INFINITY;
  /* every candidate that ends (hit count, chi2 total), for the final
   * choice's margin */
  size_t fin_cap = 16, nfin = 0;
  orc_final_key *fin = (orc_final_key *)malloc(fin_cap * sizeof(orc_final_key));

  /* seed phase: fit the seed's own hits on the first NSL layers */
  orc_cand *c = &cur[0];
  memcpy(c->x, x0, sizeof c->x);
  unpack21(P0, c->P);
  c->chi2 = 0.0;
  c->nh = 0;
  c->nm = 0;
  c->status = 0;
  for (int l = 0; l < L; ++l) c->hit[l] = -1;
  int nlive = 1;
  int seed_reached = 0;
  for (int l = 0; l < NSL && l < L; ++l) {
    double xp[6], F[36], Pp[36], s, xm[6], Pm[36];
    if (l > 0) {
      orc_material(g, l - 1, c->x, c->P, xm, Pm);
    } else {
      memcpy(xm, c->x, sizeof xm);
      memcpy(Pm, c->P, sizeof Pm);
    }
    if (orc_propagate(xm, q, g->bz, g->radii[l], l == 0, xp, F, &s)) {
      c->status |= ORC_NO_REACH;
      nlive = 0;
      break;
    }
    seed_reached = l + 1;
    orc_cov_propagate(Pm, F, Pp);
    int h = seed_hit[l];
    memcpy(c->x, xp, sizeof xp);
    memcpy(c->P, Pp, sizeof Pp);
    if (h >= 0) {
      const double *m = hits + 3 * (layer_off[l] + h);
      double V[9], xn[6], Pn[36], c2;
      orc_hit_cov(m, g->sigma_r, g->sigma_rphi, g->sigma_z, V);
      if (orc_update(xp, Pp, m, V, xn, Pn, &c2)) {
        c->status |= ORC_S_NOT_PD;
      } else {
        memcpy(c->x, xn, sizeof xn);
        memcpy(c->P, Pn, sizeof Pn);
        c->chi2 += c2;
        c->nh += 1;
        c->hit[l] = h;
      }
    }
  }
  if (nlive == 0) { /* the seed itself could not be followed */
    best = *c;
    have_best = 1;
  }
  /* debug records of the seed layers: one candidate on each layer the seed
   * reached, with the hit it actually took */
  for (int l = 0; l < NSL && l < L; ++l) {
    const int reached = l < seed_reached;
    if (dbg_n) dbg_n[l] = reached;
    if (dbg && reached) {
      dbg[(l * NC) * 2 + 0] = 0;
      dbg[(l * NC) * 2 + 1] = c->hit[l];
    }
  }

  for (int l = NSL; l < L && nlive > 0; ++l) {
    const int64_t h0 = layer_off[l], h1 = layer_off[l + 1];
    double cut_margin = INFINITY;
    nrec = 0;
    for (int ci = 0; ci < nlive; ++ci) {
      orc_cand *p = &cur[ci];
      double F[36], xm[6], Pm[36];
      double s;
      prop_ok[ci] = 0;
      int finished = 0;
      orc_material(g, l - 1, p->x, p->P, xm, Pm);
      if (orc_propagate(xm, q, g->bz, g->radii[l], 0, prop[ci].x, F, &s)) {
        p->status |= ORC_NO_REACH;
        finished = 1;
      } else {
        prop_ok[ci] = 1;
        orc_cov_propagate(Pm, F, prop[ci].P);
        int ncompat = 0;
        for (int64_t hi = h0; hi < h1; ++hi) {
          const double *m = hits + 3 * hi;
          double V[9], c2;
          orc_hit_cov(m, g->sigma_r, g->sigma_rphi, g->sigma_z, V);
          if (orc_chi2(prop[ci].x, prop[ci].P, m, V, &c2)) continue;
          double gap = fabs(c2 - bp->chi2_cut) / (bp->chi2_cut > 1.0 ? bp->chi2_cut : 1.0);
          if (gap < cut_margin) cut_margin = gap;
          if (c2 < bp->chi2_cut) {
            if (nrec == rec_cap) {
              rec_cap *= 2;
              rec = (orc_rec *)realloc(rec, rec_cap * sizeof(orc_rec));
            }
            orc_rec r = {p->chi2 + c2, p->nh + 1, p->nm, ci, (int32_t)(hi - h0)};
            rec[nrec++] = r;
            ++ncompat;
          }
        }
        if (ncompat == 0) {
          if (p->nm < bp->max_missed) {
            if (nrec == rec_cap) {
              rec_cap *= 2;
              rec = (orc_rec *)realloc(rec, rec_cap * sizeof(orc_rec));
            }
            orc_rec r = {p->chi2, p->nh, p->nm + 1, ci, -1};
            rec[nrec++] = r;
          } else {
            finished = 1;
          }
        }
      }
      if (finished) {
        orc_final_key k = {p->nh, p->chi2, l, ci};
        if (nfin == fin_cap) {
          fin_cap *= 2;
          fin = (orc_final_key *)realloc(fin, fin_cap * sizeof(orc_final_key));
        }
        fin[nfin++] = k;
        if (!have_best || better_final(&k, &best_key)) {
          best = *p;
          best_key = k;
          have_best = 1;
        }
      }
    }
    qsort(rec, nrec, sizeof(orc_rec), cmp_rec);
    int nkeep = (int)nrec < NC ? (int)nrec : NC;
    if (margin) {
      double m = cut_margin;
      int lim = (int)nrec < NC + 1 ? (int)nrec : NC + 1;
      for (int i = 0; i + 1 < lim; ++i)
        if (rec[i].nh == rec[i + 1].nh) {
          double gp = rel_gap(rec[i].chi2, rec[i + 1].chi2);
          if (gp < m) m = gp;
        }
      margin[l] = m;
    }
    for (int i = 0; i < nkeep; ++i) {
      const orc_rec *r = &rec[i];
      orc_cand *ch = &nxt[i];
      const orc_cand *par = &cur[r->parent];
      memcpy(ch->hit, par->hit, sizeof ch->hit);
      ch->status = par->status;
      memcpy(ch->x, prop[r->parent].x, sizeof ch->x);
      memcpy(ch->P, prop[r->parent].P, sizeof ch->P);
      ch->chi2 = r->chi2;
      ch->nh = r->nh;
      ch->nm = r->nm;
      if (r->hit >= 0) {
        const double *m = hits + 3 * (h0 + r->hit);
        double V[9], xn[6], Pn[36], c2;
        orc_hit_cov(m, g->sigma_r, g->sigma_rphi, g->sigma_z, V);
        orc_update(prop[r->parent].x, prop[r->parent].P, m, V, xn, Pn, &c2);
        memcpy(ch->x, xn, sizeof xn);
        memcpy(ch->P, Pn, sizeof Pn);
        ch->hit[l] = r->hit;
      }
      if (dbg) {
        dbg[(l * NC + i) * 2 + 0] = r->parent;
        dbg[(l * NC + i) * 2 + 1] = r->hit;
      }
    }
    if (dbg_n) dbg_n[l] = nkeep;
    orc_cand *t = cur;
    cur = nxt;
    nxt = t;
    nlive = nkeep;
  }

  /* surviving candidates compete with the finished ones */
  for (int ci = 0; ci < nlive; ++ci) {
    orc_final_key k = {cur[ci].nh, cur[ci].chi2, L, ci};
    if (nfin == fin_cap) {
      fin_cap *= 2;
      fin = (orc_final_key *)realloc(fin, fin_cap * sizeof(orc_final_key));
    }
    fin[nfin++] = k;
    if (!have_best || better_final(&k, &best_key)) {
      best = cur[ci];
      best_key = k;
      have_best = 1;
    }
  }
  if (margin && have_best) {
    for (size_t i = 0; i < nfin; ++i) {
      const orc_final_key *k = &fin[i];
      if (k->end_layer == best_key.end_layer && k->rank == best_key.rank) continue; /* the chosen one */
      if (k->nh != best_key.nh) continue;
      const double gp = rel_gap(best_key.chi2, k->chi2);
      if (gp < margin[L]) margin[L] = gp;
    }
  }
  free(fin);
  st = (uint32_t)best.status;
  if (!all_finite(best.x, 6) || !all_finite(best.P, 36)) st |= ORC_NONFINITE;
  for (int l = 0; l < L; ++l) hit_idx[l] = best.hit[l];
  memcpy(xo, best.x, sizeof best.x);
  pack21(best.P, Po);
  *chi2 = best.chi2;
  *nhits = best.nh;
  *status = st;
  free(cur);
  free(nxt);
  free(prop);
  free(prop_ok);
  free(rec);
  return 0;
}

typedef struct {
  const orc_geom *g;
  const orc_build_params *bp;
  const double *hits;
  const int64_t *layer_off;
  int64_t lo, hi;
  const double *state, *cov;
  const int8_t *q;
  const int32_t *seed_hit;
  int32_t *hit_idx;
  double *state_o, *cov_o, *chi2_o;
  int32_t *nhits_o;
  uint32_t *status_o;
  int32_t *dbg_n, *dbg;
  double *margin;
} build_job;

static void *build_worker(void *arg) {
  build_job *j = (build_job *)arg;
  const int L = j->g->n_layers, NC = j->bp->max_cands, NSL = j->bp->n_seed_layers;
  for (int64_t i = j->lo; i < j->hi; ++i)
    orc_build_seed(j->g, j->bp, j->hits, j->layer_off, j->state + 6 * i, j->cov + 21 * i,
                   j->q[i], j->seed_hit + (int64_t)NSL * i, j->hit_idx + (int64_t)L * i,
                   j->state_o + 6 * i, j->cov_o + 21 * i, j->chi2_o + i, j->nhits_o + i,
                   j->status_o + i, j->dbg_n ? j->dbg_n + (int64_t)L * i : NULL,
                   j->dbg ? j->dbg + (int64_t)L * NC * 2 * i : NULL,
                   j->margin ? j->margin + (int64_t)(L + 1) * i : NULL);
  return NULL;
}

void orc_build_event(const orc_geom *g, const orc_build_params *bp, const double *hits,
                     const int64_t *layer_off, int64_t n_seeds, const double *state,
                     const double *cov, const int8_t *q, const int32_t *seed_hit,
                     int32_t *hit_idx, double *state_o, double *cov_o, double *chi2_o,
                     int32_t *nhits_o, uint32_t *status_o, int32_t *dbg_n, int32_t *dbg,
                     double *margin, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  build_job jobs[256];
  for (int t = 0; t < nthreads; ++t) {
    build_job j = {g, bp, hits, layer_off, n_seeds * t / nthreads, n_seeds * (t + 1) / nthreads,
                   state, cov, q, seed_hit, hit_idx, state_o, cov_o, chi2_o, nhits_o, status_o,
                   dbg_n, dbg, margin};
    jobs[t] = j;
  }
  if (nthreads == 1) {
    build_worker(&jobs[0]);
    return;
  }
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, build_worker, &jobs[t]);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}
