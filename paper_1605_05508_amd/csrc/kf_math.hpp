// kf_math.hpp -- per-lane Kalman-filter arithmetic for gfx950.
//
// One track per lane, everything in registers.  The operations are those of
// the paper's Kalman-filter tracking (Sec. 2: propagate to the next layer,
// update with its hit; Sec. 2.1: a chain of 3x3 .. 6x6 matrix operations
// with symmetric matrices and known zero/one patterns exploited).  The
// helix model is a charged particle in a uniform field along z between
// cylindrical barrel layers; the measurement is the hit's global (x, y, z).
//
// Precision is a template parameter: TP is the type of the state
// propagation (path solve, transport, Jacobian), C the type the covariance
// is kept and propagated in (F P F^T); the update (hit covariance, S, its
// inverse, chi2, gain, state and Joseph covariance update) and the layer
// material always run in double.  TP = C = double is the plain FP64 path,
// TP = C = float the FP32-bulk path, TP = float with C = double the FP32
// state propagation with a double covariance.
//
// Packed symmetric 6x6: 21-value upper triangle, row order
// (00,01,02,03,04,05,11,12,13,14,15,22,23,24,25,33,34,35,44,45,55).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define KTF_HD __host__ __device__ __forceinline__

namespace ktf {

constexpr double kCLight = 0.00299792458;  // GeV / (cm T)

// status bits (public values, see ktf.h)
constexpr uint32_t kNoReach = 1u;
constexpr uint32_t kSNotPD = 2u;
constexpr uint32_t kNonFinite = 4u;

KTF_HD constexpr int pidx(int i, int j) {  // packed index, i <= j
  return i * 6 - (i * (i - 1)) / 2 + (j - i);
}
KTF_HD constexpr int sidx(int i, int j) { return i <= j ? pidx(i, j) : pidx(j, i); }

// double reciprocal: hardware estimate refined by two Newton-Raphson steps
// (each doubles the correct bits), in place of the IEEE division sequence
KTF_HD double rcp_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}

template <typename T> KTF_HD T rcp(T x);
template <> KTF_HD double rcp<double>(double x) { return rcp_nr(x); }
template <> KTF_HD float rcp<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);  // 1 ulp
#else
  return 1.0f / x;
#endif
}

template <typename T> KTF_HD T ksqrt(T x);
template <> KTF_HD double ksqrt<double>(double x) { return sqrt(x); }
template <> KTF_HD float ksqrt<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);  // hardware square root, 1 ulp (arguments are normal or 0)
#else
  return sqrtf(x);
#endif
}

template <typename T> KTF_HD void ksincos(T x, T* s, T* c);
template <> KTF_HD void ksincos<double>(double x, double* s, double* c) { sincos(x, s, c); }
template <> KTF_HD void ksincos<float>(float x, float* s, float* c) { sincosf(x, s, c); }

// ---------------------------------------------------------------------------
// Helix functions of the turning angle th:
//   A = sin(th)/th, C = (1 - cos th)/th, dA = dA/dth, dC = dC/dth.
// Small angles use the Maclaurin series (no cancellation, no division);
// larger ones the trigonometric forms.
// ---------------------------------------------------------------------------
template <typename T> struct NewtonTol;
template <> struct NewtonTol<float> { static constexpr float v = 1e-6f; };
template <> struct NewtonTol<double> { static constexpr double v = 1e-12; };

template <typename T> struct SeriesLen;
template <> struct SeriesLen<float> { static constexpr int n = 5; };
template <> struct SeriesLen<double> { static constexpr int n = 9; };

template <typename T>
KTF_HD double fact(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

// A and C only (the Newton iterations need no derivatives)
template <typename T>
KTF_HD void helix_ac(T th, T& A, T& C) {
  const T t2 = th * th;
  if (t2 <= T(0.25)) {
    // A = sum (-1)^n t^2n / (2n+1)!,  C = sum (-1)^n t^(2n+1) / (2n+2)!
    constexpr int N = SeriesLen<T>::n;
    T a = T(0), c = T(0);
#pragma unroll
    for (int n = N - 1; n >= 0; --n) {
      const double sg = (n & 1) ? -1.0 : 1.0;
      a = a * t2 + T(sg / fact<T>(2 * n + 1));
      c = c * t2 + T(sg / fact<T>(2 * n + 2));
    }
    A = a;
    C = c * th;
  } else {
    T s, co;
    ksincos(th, &s, &co);
    const T it = rcp(th);
    A = s * it;
    // 1 - cos th without cancellation when cos th > 0
    const T omc = co > T(0) ? s * s * rcp(T(1) + co) : T(1) - co;
    C = omc * it;
  }
}

// dA/dth and dC/dth given A and C:
//   dA = sum (-1)^n 2n t^(2n-1)/(2n+1)!,  dC = sum (-1)^n (2n+1) t^2n/(2n+2)!
// (series), or dA = (cos th - A)/th, dC = (sin th - C)/th.
template <typename T>
KTF_HD void helix_dac(T th, T A, T C, T& dA, T& dC) {
  const T t2 = th * th;
  if (t2 <= T(0.25)) {
    constexpr int N = SeriesLen<T>::n;
    T da = T(0), dc = T(0);
#pragma unroll
    for (int n = N - 1; n >= 0; --n) {
      const double sg = (n & 1) ? -1.0 : 1.0;
      dc = dc * t2 + T(sg * (2 * n + 1) / fact<T>(2 * n + 2));
      if (n >= 1) da = da * t2 + T(sg * (2 * n) / fact<T>(2 * n + 1));
    }
    dA = da * th;
    dC = dc;
  } else {
    const T it = rcp(th);
    dA = ((T(1) - th * C) - A) * it;
    dC = (th * A - C) * it;
  }
}

// ---------------------------------------------------------------------------
// Track state in registers: the position is accumulated in double (it is
// ~ r ~ 10..100 cm while the information sits in its last micrometres); the
// momentum and all propagation arithmetic use the propagation type T.  The
// transport below therefore works with the displacement between layers
// (a few cm), which T resolves well.
// ---------------------------------------------------------------------------
template <typename T>
struct TrackState {
  double pos[3];
  T mom[3];
};

// ---------------------------------------------------------------------------
// Transport at fixed transverse arc length s in field constant k = c q Bz:
// the transverse momentum turns by th = -k s / pT, pz stays, and the
// position advances by d = (s/pT) (px A - py C, py A + px C, pz).
// ---------------------------------------------------------------------------
template <typename T>
struct Transported {
  T d[3];    // displacement
  T mom[3];  // momentum at s
  T th, sp, A, C, sn, cs;
};

template <typename T>
KTF_HD void transport(const TrackState<T>& x, T k, T ipt, T s, Transported<T>& o) {
  const T sp = s * ipt;
  const T th = -k * sp;
  helix_ac(th, o.A, o.C);
  o.th = th;
  o.sp = sp;
  o.sn = th * o.A;          // sin th
  o.cs = T(1) - th * o.C;   // cos th
  const T px = x.mom[0], py = x.mom[1];
  o.d[0] = sp * (px * o.A - py * o.C);
  o.d[1] = sp * (py * o.A + px * o.C);
  o.d[2] = sp * x.mom[2];
  o.mom[0] = px * o.cs - py * o.sn;
  o.mom[1] = py * o.cs + px * o.sn;
  o.mom[2] = x.mom[2];
}

// Jacobian of the surface-to-surface map with its zero/one structure:
//   rows x', y', px', py' depend only on x, y, px, py;
//   row z' = (f20, f21, 1, f23, f24, f25); row pz' = e_pz; column z = e_z.
template <typename T>
struct Jac {
  T a[4][4];      // rows/cols in order (x, y, px, py)
  T z0, z1, z3, z4, z5;  // row z': d z'/d(x, y, px, py, pz)
};

// Path solve + transport + constrained Jacobian.  nearest: root of least
// |s| (first step onto a layer); otherwise the least positive root.
// NITER Newton steps on g(s) = |pos_T + d_T(s)|^2 - r^2 from the
// straight-line root.  Returns false when the track cannot reach the
// cylinder.
template <typename T, int NITER>
KTF_HD bool propagate(const TrackState<T>& x, T k, double r, bool nearest, TrackState<T>& xo,
                      Jac<T>& F) {
  const T px = x.mom[0], py = x.mom[1];
  const T pt2 = px * px + py * py;
  const T ipt = rcp(ksqrt(pt2));
  const T pt = pt2 * ipt;
  const T x0 = (T)x.pos[0], y0 = (T)x.pos[1];
  const T rf = (T)r;
  bool ok = pt2 > T(0);
  if (k != T(0)) {  // the transverse circle must meet the layer circle
    const T ik = rcp(k);
    const T cx = x0 + py * ik, cy = y0 - px * ik;
    const T d = ksqrt(cx * cx + cy * cy);
    const T R = pt * (ik < T(0) ? -ik : ik);
    const T dr = d - R;
    ok = ok && !(d + R < rf) && !((dr < T(0) ? -dr : dr) > rf);
  }
  // g(s) = c0 + 2 pos.d + |d|^2 with c0 = |pos_T|^2 - r^2 in double
  const double c0 = x.pos[0] * x.pos[0] + x.pos[1] * x.pos[1] - r * r;
  const T u = (x0 * px + y0 * py) * ipt;
  const T disc = u * u - (T)c0;
  T s;
  if (disc < T(0)) {
    ok = ok && (k != T(0));
    s = -u;
  } else {
    const T sq = ksqrt(disc);
    const T s1 = -u + sq, s2 = -u - sq;
    s = (nearest && ((s2 < T(0) ? -s2 : s2) < (s1 < T(0) ? -s1 : s1))) ? s2 : s1;
  }
  Transported<T> t;
  T ds = T(0);
  auto newton_step = [&]() {
    transport(x, k, ipt, s, t);
    const double dx = (double)t.d[0], dy = (double)t.d[1];
    const double g = c0 + (2.0 * x.pos[0] + dx) * dx + (2.0 * x.pos[1] + dy) * dy;
    const T xe = (T)(x.pos[0] + dx), ye = (T)(x.pos[1] + dy);
    const T gp = T(2) * (xe * t.mom[0] + ye * t.mom[1]) * ipt;
    ds = (T)g * rcp(gp);
    s = s - ds;
  };
#pragma unroll
  for (int it = 0; it < NITER; ++it) newton_step();
  // Newton converges quadratically from the straight-line root; a long or
  // strongly curved step may need more: continue while the last step is
  // above the tolerance (1e-12 (1 + |s|) cm in double, 1e-6 (1 + |s|) in
  // float), up to 50 steps in all in double.  A helix that only grazes the
  // layer converges slowly (a double root); one that has not converged
  // within the limit counts as not reaching the layer.
  const T tol = NewtonTol<T>::v * (T(1) + (s < T(0) ? -s : s));
  constexpr int kTail = sizeof(T) == 8 ? 50 - NITER : 8;
  bool conv = (ds < T(0) ? -ds : ds) <= tol;
#pragma unroll 1
  for (int it = 0; it < kTail && !conv; ++it) {
    newton_step();
    conv = (ds < T(0) ? -ds : ds) <= tol;
  }
  transport(x, k, ipt, s, t);
  ok = ok && conv && (nearest || s > T(0));
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    xo.pos[i] = x.pos[i] + (double)t.d[i];
    xo.mom[i] = t.mom[i];
  }
  const T xe = (T)xo.pos[0], ye = (T)xo.pos[1];

  // fixed-s derivatives
  T dA, dC;
  helix_dac(t.th, t.A, t.C, dA, dC);
  const T ipt2 = ipt * ipt;
  const T dth_dpx = -t.th * px * ipt2, dth_dpy = -t.th * py * ipt2;
  const T dsp_dpx = -t.sp * px * ipt2, dsp_dpy = -t.sp * py * ipt2;
  const T fx = px * t.A - py * t.C, fy = py * t.A + px * t.C;
  const T dfx = px * dA - py * dC, dfy = py * dA + px * dC;
  const T s03 = dsp_dpx * fx + t.sp * (t.A + dfx * dth_dpx);
  const T s04 = dsp_dpy * fx + t.sp * (-t.C + dfx * dth_dpy);
  const T s13 = dsp_dpx * fy + t.sp * (t.C + dfy * dth_dpx);
  const T s14 = dsp_dpy * fy + t.sp * (t.A + dfy * dth_dpy);
  const T pz = x.mom[2];
  const T s23 = dsp_dpx * pz, s24 = dsp_dpy * pz;
  const T pxo = t.mom[0], pyo = t.mom[1];
  const T s33 = t.cs - pyo * dth_dpx, s34 = -t.sn - pyo * dth_dpy;
  const T s43 = t.sn + pxo * dth_dpx, s44 = t.cs + pxo * dth_dpy;
  // arc-length change: v = dT/ds, w = ds/dx from the surface condition
  const T v0 = pxo * ipt, v1 = pyo * ipt, v2 = pz * ipt;
  const T v3 = k * pyo * ipt, v4 = -k * pxo * ipt;
  const T den = xe * v0 + ye * v1;
  ok = ok && den != T(0);
  const T iden = -rcp(den);
  const T w0 = xe * iden, w1 = ye * iden;
  const T w3 = (xe * s03 + ye * s13) * iden;
  const T w4 = (xe * s04 + ye * s14) * iden;
  // transverse block, order (x, y, px, py)
  const T vt[4] = {v0, v1, v3, v4};
  const T base[4][4] = {{T(1), T(0), s03, s04},
                        {T(0), T(1), s13, s14},
                        {T(0), T(0), s33, s34},
                        {T(0), T(0), s43, s44}};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    F.a[i][0] = base[i][0] + vt[i] * w0;
    F.a[i][1] = base[i][1] + vt[i] * w1;
    F.a[i][2] = base[i][2] + vt[i] * w3;
    F.a[i][3] = base[i][3] + vt[i] * w4;
  }
  F.z0 = v2 * w0;
  F.z1 = v2 * w1;
  F.z3 = s23 + v2 * w3;
  F.z4 = s24 + v2 * w4;
  F.z5 = t.sp;
  return ok;
}

// P' = F P F^T on packed storage using the Jacobian's structure, in the
// covariance's type T (the Jacobian may be of a narrower type J).
// Index sets: transverse T = {0, 1, 3, 4} (block positions 0..3), z = 2,
// pz = 5.
template <typename T, typename J>
KTF_HD void cov_propagate(const T P[21], const Jac<J>& FJ, T Po[21]) {
  constexpr int tix[4] = {0, 1, 3, 4};
  struct {
    T a[4][4];
    T z5;
  } F;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) F.a[r][c] = (T)FJ.a[r][c];
  F.z5 = (T)FJ.z5;
  const T fz[4] = {(T)FJ.z0, (T)FJ.z1, (T)FJ.z3, (T)FJ.z4};
  // row by row: G_i = (F P)_i, then P'_ij = G_i . F_j for j >= i
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T G[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      T acc;
      if (i == 5) {
        acc = P[sidx(5, m)];
      } else if (i == 2) {
        acc = P[sidx(2, m)] + F.z5 * P[sidx(5, m)];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc += fz[b] * P[sidx(tix[b], m)];
      } else {
        const int ia = (i < 2) ? i : i - 1;  // block position of i in T
        acc = T(0);
#pragma unroll
        for (int b = 0; b < 4; ++b) acc += F.a[ia][b] * P[sidx(tix[b], m)];
      }
      G[m] = acc;
    }
#pragma unroll
    for (int j = i; j < 6; ++j) {
      T acc;
      if (j == 5) {
        acc = G[5];
      } else if (j == 2) {
        acc = G[2] + F.z5 * G[5];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc += G[tix[b]] * fz[b];
      } else {
        const int ja = (j < 2) ? j : j - 1;
        acc = T(0);
#pragma unroll
        for (int b = 0; b < 4; ++b) acc += G[tix[b]] * F.a[ja][b];
      }
      Po[pidx(i, j)] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Update (always double).  V is the hit covariance: diag(sr^2, srphi^2,
// sz^2) in the hit's (radial, tangential, z) frame.  S = P'[0:3,0:3] + V is
// inverted by cofactors; the gain is K = P'[:,0:3] S^-1; the covariance is
// the Joseph form (I-KH) P' (I-KH)^T + K V K^T, expanded as
// P' - K B^T - B K^T + K S K^T with B = P'[:,0:3], for the 21 outputs.
// ---------------------------------------------------------------------------
struct HitRes {
  double sr2, srphi2, sz2;
};

struct Residual {
  double r[3];
  double S[6];   // packed 3x3: 00 01 02 11 12 22
  double Si[6];  // inverse
  double chi2;
};

// Inverse of the symmetric 3x3 S (packed 00 01 02 11 12 22) by cofactors
// over the determinant; returns whether S is positive definite (Sylvester).
KTF_HD bool sym3_inverse(const double S[6], double Si[6]) {
  const double S00 = S[0], S01 = S[1], S02 = S[2], S11 = S[3], S12 = S[4], S22 = S[5];
  const double c00 = S11 * S22 - S12 * S12;
  const double c01 = S02 * S12 - S01 * S22;
  const double c02 = S01 * S12 - S02 * S11;
  const double c11 = S00 * S22 - S02 * S02;
  const double c12 = S01 * S02 - S00 * S12;
  const double c22 = S00 * S11 - S01 * S01;
  const double det = S00 * c00 + S01 * c01 + S02 * c02;
  const bool pd = S00 > 0.0 && c22 > 0.0 && det > 0.0;
  const double idet = rcp_nr(det);
  Si[0] = c00 * idet; Si[1] = c01 * idet; Si[2] = c02 * idet;
  Si[3] = c11 * idet; Si[4] = c12 * idet; Si[5] = c22 * idet;
  return pd;
}

// r^T Si r for the packed symmetric Si
KTF_HD double quad3(const double Si[6], const double r[3]) {
  const double Sr0 = Si[0] * r[0] + Si[1] * r[1] + Si[2] * r[2];
  const double Sr1 = Si[1] * r[0] + Si[3] * r[1] + Si[4] * r[2];
  const double Sr2 = Si[2] * r[0] + Si[4] * r[1] + Si[5] * r[2];
  return r[0] * Sr0 + r[1] * Sr1 + r[2] * Sr2;
}

template <typename T, typename C>
KTF_HD bool residual(const TrackState<T>& xp, const C Pp[21], const double m[3],
                     const HitRes& hr, Residual& o) {
  const double rho2 = m[0] * m[0] + m[1] * m[1];
  const double irho2 = rcp_nr(rho2);
  const double xx = m[0] * m[0] * irho2, yy = m[1] * m[1] * irho2, xy = m[0] * m[1] * irho2;
  const double V00 = hr.sr2 * xx + hr.srphi2 * yy;
  const double V01 = (hr.sr2 - hr.srphi2) * xy;
  const double V11 = hr.sr2 * yy + hr.srphi2 * xx;
  o.r[0] = m[0] - xp.pos[0];
  o.r[1] = m[1] - xp.pos[1];
  o.r[2] = m[2] - xp.pos[2];
  const double S00 = (double)Pp[pidx(0, 0)] + V00, S01 = (double)Pp[pidx(0, 1)] + V01;
  const double S02 = (double)Pp[pidx(0, 2)], S11 = (double)Pp[pidx(1, 1)] + V11;
  const double S12 = (double)Pp[pidx(1, 2)], S22 = (double)Pp[pidx(2, 2)] + hr.sz2;
  o.S[0] = S00; o.S[1] = S01; o.S[2] = S02; o.S[3] = S11; o.S[4] = S12; o.S[5] = S22;
  const bool pd = sym3_inverse(o.S, o.Si);
  o.chi2 = quad3(o.Si, o.r);
  return pd;
}

// State and covariance update given the residual; writes into x (state
// type T) and P (covariance type C), which may be xp and Pp themselves (the
// gain is formed from Pp before any element of P is written, and each
// element of P is written after its own element of Pp is read).
// Joseph form expanded: P+ = P' - K B^T - B K^T + K S K^T
//                          = P' - K D^T - D K^T  with D = B - (K S)/2,
// which needs only K and D per row (S symmetric).
template <typename T, typename C>
KTF_HD void apply_update(const TrackState<T>& xp, const C Pp[21], const Residual& R,
                         TrackState<T>& x, C P[21]) {
  double K[6][3], D[6][3];
  const double* Si = R.Si;
  const double* S = R.S;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double b0 = (double)Pp[sidx(i, 0)], b1 = (double)Pp[sidx(i, 1)],
                 b2 = (double)Pp[sidx(i, 2)];
    const double k0 = b0 * Si[0] + b1 * Si[1] + b2 * Si[2];
    const double k1 = b0 * Si[1] + b1 * Si[3] + b2 * Si[4];
    const double k2 = b0 * Si[2] + b1 * Si[4] + b2 * Si[5];
    K[i][0] = k0;
    K[i][1] = k1;
    K[i][2] = k2;
    // D = B - (K S)/2, as fused multiply-adds on the halved gain
    const double h0 = -0.5 * k0, h1 = -0.5 * k1, h2 = -0.5 * k2;
    D[i][0] = fma(h0, S[0], fma(h1, S[1], fma(h2, S[2], b0)));
    D[i][1] = fma(h0, S[1], fma(h1, S[3], fma(h2, S[4], b1)));
    D[i][2] = fma(h0, S[2], fma(h1, S[4], fma(h2, S[5], b2)));
    const double dx = fma(k0, R.r[0], fma(k1, R.r[1], k2 * R.r[2]));
    if (i < 3)
      x.pos[i] = xp.pos[i] + dx;
    else
      x.mom[i - 3] = (T)((double)xp.mom[i - 3] + dx);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = i; j < 6; ++j) {
      double acc = (double)Pp[pidx(i, j)];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc = fma(-K[i][c], D[j][c], acc);
        acc = fma(-D[i][c], K[j][c], acc);
      }
      P[pidx(i, j)] = (C)acc;
    }
  }
}

// Material of the layer a track leaves (radial position x.pos on it):
// path t = x0 |p| / |p.n| radiation lengths (n the radial normal), multiple
// scattering as process noise theta0^2 (|p|^2 I - p p^T) on the momentum
// with the Highland width theta0 = 0.0136 / (beta p) sqrt(t) (1 + 0.038
// ln(t / beta^2)), then the mean energy loss eloss t: |p| -> g = sqrt((E -
// eloss t)^2 - m^2) along the same direction, the covariance carried by the
// Jacobian J = f (I - u u^T) + g' u u^T on the momentum (u = p / |p|, f = g /
// |p|, g' = (E - eloss t) |p| / (g E), t held fixed).  In double.
template <typename T, typename C>
KTF_HD void apply_material(double x0, double eloss, double mass, TrackState<T>& x, C P[21]) {
  const double p[3] = {(double)x.mom[0], (double)x.mom[1], (double)x.mom[2]};
  const double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  const double pm = sqrt(p2);
  const double r = sqrt(x.pos[0] * x.pos[0] + x.pos[1] * x.pos[1]);
  const double pn = (x.pos[0] * p[0] + x.pos[1] * p[1]) / r;
  const double t = x0 * pm / fabs(pn);
  const double E = sqrt(p2 + mass * mass);
  const double beta = pm / E;
  const double th = 0.0136 / (beta * pm) * sqrt(t) * (1.0 + 0.038 * log(t / (beta * beta)));
  const double th2 = th * th;
  // momentum block plus the process noise; the position-momentum block
  double A[3][3], B[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      A[i][j] = (double)P[sidx(3 + i, 3 + j)] + th2 * ((i == j ? p2 : 0.0) - p[i] * p[j]);
      B[i][j] = (double)P[sidx(i, 3 + j)];
    }
  }
  if (eloss > 0.0) {
    const double E2 = E - eloss * t;
    const double g = E2 > mass ? sqrt(E2 * E2 - mass * mass) : 0.0;
    const double f = g / pm;
    const double gp = g > 0.0 ? E2 * pm / (g * E) : 0.0;
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) J[i][j] = (i == j ? f : 0.0) + (gp - f) * p[i] * p[j] / p2;
    double JA[3][3], BJ[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        JA[i][j] = J[i][0] * A[0][j] + J[i][1] * A[1][j] + J[i][2] * A[2][j];
        BJ[i][j] = B[i][0] * J[j][0] + B[i][1] * J[j][1] + B[i][2] * J[j][2];
      }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        A[i][j] = JA[i][0] * J[j][0] + JA[i][1] * J[j][1] + JA[i][2] * J[j][2];
        B[i][j] = BJ[i][j];
      }
#pragma unroll
    for (int i = 0; i < 3; ++i) x.mom[i] = (T)(f * p[i]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (j >= i) P[pidx(3 + i, 3 + j)] = (C)A[i][j];
      P[pidx(i, 3 + j)] = (C)B[i][j];
    }
  }
}

// Inverse of the mean energy loss of apply_material for a state that has
// just crossed the layer inwards: |p| back to sqrt((E + eloss t)^2 - m^2).
template <typename T>
KTF_HD void undo_energy_loss(double x0, double eloss, double mass, TrackState<T>& x) {
  const double p[3] = {(double)x.mom[0], (double)x.mom[1], (double)x.mom[2]};
  const double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  const double pm = sqrt(p2);
  const double r = sqrt(x.pos[0] * x.pos[0] + x.pos[1] * x.pos[1]);
  const double t = x0 * pm / fabs((x.pos[0] * p[0] + x.pos[1] * p[1]) / r);
  const double E = sqrt(p2 + mass * mass) + eloss * t;
  const double f = sqrt(E * E - mass * mass) / pm;
#pragma unroll
  for (int i = 0; i < 3; ++i) x.mom[i] = (T)(f * p[i]);
}

template <typename T, typename C>
KTF_HD bool finite_state(const TrackState<T>& x, const C P[21]) {
  C acc = (C)(x.pos[0] + x.pos[1] + x.pos[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) acc += (C)x.mom[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) acc += P[i];
  return acc - acc == C(0);  // false for inf and nan
}

}  // namespace ktf
