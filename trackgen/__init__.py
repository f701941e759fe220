"""Seeded synthetic events for Kalman-filter track fitting and building.

This module is the one piece of code shared by the FP64 oracle tests and the
GPU path: it produces inputs only.  It simulates a simplified barrel detector
(concentric cylinders in a uniform solenoidal field, no material) the way the
paper's "simplified experimental environment" is described (Abstract; Sec. 3),
draws truth particles, records where each helix crosses each cylinder, smears
those crossings into hits, adds uniformly distributed noise hits, and prepares
seeds (the "initial estimate of the track parameters based on a few hits",
Sec. 2).  It holds none of the filter's arithmetic: no transport Jacobian, no
covariance propagation, no gain, no chi2.  Truth crossings are found with the
closed-form intersection of the track's transverse circle with the layer
circle, which is a different construction from the arc-length Newton solve the
filter uses.

Every floating-point value handed to a consumer is rounded to the nearest
FP32 value and stored as float64, so an FP64 consumer and an FP32 consumer see
bit-identical inputs and any difference between them is arithmetic only.

Units: cm, GeV, tesla.  Layout convention of the returned arrays follows the
library boundary: structure of arrays, element-major, e.g. ``hits[L, 3, n]``.
Packed symmetric 6x6 covariances use the 21-value upper triangle in row order
(00,01,02,03,04,05,11,12,13,14,15,22,23,24,25,33,34,35,44,45,55).
"""
from __future__ import annotations

import concurrent.futures as _cf
import dataclasses
import math
import os
from typing import Optional

import numpy as np

_CHUNK = 1 << 18


def _threads() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def _chunked(fn, n, *arrays):
    """Run fn over track chunks in threads (numpy releases the GIL in its
    loops); fn(sl) fills its outputs for the slice sl."""
    if n <= _CHUNK:
        fn(slice(0, n))
        return
    sls = [slice(a, min(n, a + _CHUNK)) for a in range(0, n, _CHUNK)]
    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(fn, sls))

C_LIGHT = 0.00299792458  # GeV / (cm T) per unit charge

# index pairs (i, j), i <= j, of the packed upper triangle
PACKED_IJ = [(i, j) for i in range(6) for j in range(i, 6)]


def f32(a):
    """Round to the nearest FP32 value, keep float64 storage."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclasses.dataclass(frozen=True)
class Detector:
    """Cylindrical barrel layers at radii ``radii`` in a uniform field ``bz``."""
    radii: tuple
    z_half: float = 100.0
    bz: float = 3.8
    sigma_rphi: float = 0.01
    sigma_z: float = 0.1
    sigma_r: float = 0.01  # radial hit variance used by the filter only; hits are not smeared radially
    x0: float = 0.0        # thickness of every layer in radiation lengths at normal incidence
    eloss: float = 0.0     # mean energy loss per radiation length of path (GeV)
    mass: float = 0.13957  # particle mass (GeV), for beta in the scattering width and the energy loss

    @property
    def n_layers(self) -> int:
        return len(self.radii)


def barrel(n_layers: int, step: float = 4.0, **kw) -> Detector:
    """Layers at r = step, 2*step, ..., n_layers*step."""
    return Detector(radii=tuple(step * (i + 1) for i in range(n_layers)), **kw)


# --------------------------------------------------------------------------
# truth particles
# --------------------------------------------------------------------------

def sample_truth(rng: np.random.Generator, n: int, *, pt_range=(0.5, 10.0),
                 pt_log=False, eta_max=1.0, sigma_vxy=0.01, sigma_vz=1.0):
    """Truth particles: vertex, momentum at the vertex, charge.

    Returns a dict of float64 arrays of length n: vx, vy, vz, px, py, pz, and
    int8 q.  eta is uniform in (-eta_max, eta_max), so pz = pT sinh(eta)
    (pseudorapidity defined as -ln tan(theta/2)).
    """
    lo, hi = pt_range
    if pt_log:
        pt = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    else:
        pt = rng.uniform(lo, hi, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    eta = rng.uniform(-eta_max, eta_max, n)
    q = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    vx = rng.normal(0.0, sigma_vxy, n)
    vy = rng.normal(0.0, sigma_vxy, n)
    vz = rng.normal(0.0, sigma_vz, n)
    return dict(vx=vx, vy=vy, vz=vz, px=pt * np.cos(phi), py=pt * np.sin(phi),
                pz=pt * np.sinh(eta), q=q)


def truth_crossings(truth: dict, det: Detector):
    """Where each truth helix first crosses each layer cylinder.

    Closed form: the transverse projection is a circle of radius R = pT/|k|,
    k = c q Bz, centred at (vx + py/k, vy - px/k).  Its intersections with the
    layer circle follow from the two-circle intersection; of the two points,
    the one reached first when moving along the momentum is taken.  The
    turning angle to it gives the transverse arc length s, from which z and
    the rotated momentum follow.

    Returns pos[L,3,n], mom[L,3,n] (float64, unrounded) and reached[L,n]
    (bool; False where the circle never reaches the layer).
    """
    n = truth["vx"].shape[0]
    L = det.n_layers
    pos = np.zeros((L, 3, n))
    mom = np.zeros((L, 3, n))
    reached = np.zeros((L, n), dtype=bool)

    def work(sl):
        vx, vy, vz = truth["vx"][sl], truth["vy"][sl], truth["vz"][sl]
        px, py, pz = truth["px"][sl], truth["py"][sl], truth["pz"][sl]
        q = truth["q"][sl].astype(np.float64)
        k = C_LIGHT * q * det.bz
        pt = np.hypot(px, py)
        R = pt / np.abs(k)
        cx = vx + py / k
        cy = vy - px / k
        d = np.hypot(cx, cy)
        # d^2 - R^2 without cancellation: |v + w|^2 - |w|^2 = |v|^2 + 2 v.w
        d2mR2 = vx * vx + vy * vy + 2.0 * (vx * py - vy * px) / k
        ux, uy = cx / d, cy / d
        r0x, r0y = vx - cx, vy - cy  # vertex relative to the circle centre
        m = vx.shape[0]
        for li, r in enumerate(det.radii):
            a = (r * r + d2mR2) / (2.0 * d)
            h2 = r * r - a * a
            ok = h2 >= 0.0
            h = np.sqrt(np.where(ok, h2, 0.0))
            best_s = np.full(m, np.inf)
            best_x = np.zeros(m)
            best_y = np.zeros(m)
            for sgn in (1.0, -1.0):
                X = a * ux - sgn * h * uy
                Y = a * uy + sgn * h * ux
                rx, ry = X - cx, Y - cy
                cross = r0x * ry - r0y * rx
                dot = r0x * rx + r0y * ry
                dlt = np.arctan2(cross, dot)
                # k > 0 turns clockwise (negative angle), k < 0 counter-clockwise
                ang = np.where(k > 0, np.where(dlt <= 0, dlt, dlt - 2 * math.pi),
                               np.where(dlt >= 0, dlt, dlt + 2 * math.pi))
                s = np.abs(ang) * R
                better = s < best_s
                best_s = np.where(better, s, best_s)
                best_x = np.where(better, X, best_x)
                best_y = np.where(better, Y, best_y)
            theta = -k * best_s / pt
            c, sn = np.cos(theta), np.sin(theta)
            pos[li, 0, sl] = best_x
            pos[li, 1, sl] = best_y
            pos[li, 2, sl] = vz + best_s * pz / pt
            mom[li, 0, sl] = px * c - py * sn
            mom[li, 1, sl] = py * c + px * sn
            mom[li, 2, sl] = pz
            reached[li, sl] = ok

    _chunked(work, n)
    return pos, mom, reached


def _cross_layer(x, y, z, px, py, pz, k, r):
    """First forward crossing of the helix from (x, y, z, p) with the cylinder
    of radius r (the two-circle intersection of truth_crossings, from an
    arbitrary start).  Returns x, y, z, px, py, pz at the crossing and ok."""
    pt = np.hypot(px, py)
    R = pt / np.abs(k)
    cx = x + py / k
    cy = y - px / k
    d = np.hypot(cx, cy)
    d2mR2 = x * x + y * y + 2.0 * (x * py - y * px) / k
    ux, uy = cx / d, cy / d
    r0x, r0y = x - cx, y - cy
    a = (r * r + d2mR2) / (2.0 * d)
    h2 = r * r - a * a
    ok = h2 >= 0.0
    h = np.sqrt(np.where(ok, h2, 0.0))
    best_s = np.full(x.shape, np.inf)
    best_x = np.zeros(x.shape)
    best_y = np.zeros(x.shape)
    for sgn in (1.0, -1.0):
        X = a * ux - sgn * h * uy
        Y = a * uy + sgn * h * ux
        rx, ry = X - cx, Y - cy
        cross = r0x * ry - r0y * rx
        dot = r0x * rx + r0y * ry
        dlt = np.arctan2(cross, dot)
        ang = np.where(k > 0, np.where(dlt <= 0, dlt, dlt - 2 * math.pi),
                       np.where(dlt >= 0, dlt, dlt + 2 * math.pi))
        s = np.abs(ang) * R
        better = s < best_s
        best_s = np.where(better, s, best_s)
        best_x = np.where(better, X, best_x)
        best_y = np.where(better, Y, best_y)
    theta = -k * best_s / pt
    c, sn = np.cos(theta), np.sin(theta)
    return best_x, best_y, z + best_s * pz / pt, px * c - py * sn, py * c + px * sn, pz, ok


def scatter_layer(rng, x, y, px, py, pz, det: Detector):
    """Cross one layer's material: rotate p by two independent Gaussian
    angles of width theta0 (Highland formula, unit charge) in the plane
    perpendicular to p, then remove the mean energy loss.  The path through
    the layer is x0 |p| / |p.n| radiation lengths (n the radial normal)."""
    p2 = px * px + py * py + pz * pz
    p = np.sqrt(p2)
    r = np.hypot(x, y)
    t = det.x0 * p / np.abs((x * px + y * py) / r)
    E = np.sqrt(p2 + det.mass ** 2)
    beta = p / E
    th0 = 0.0136 / (beta * p) * np.sqrt(t) * (1.0 + 0.038 * np.log(t / beta ** 2))
    pt = np.hypot(px, py)
    ex, ey, ez = px / p, py / p, pz / p
    ux, uy, uz = py / pt, -px / pt, np.zeros_like(pt)   # unit, perpendicular to p and z
    vx, vy, vz = ey * uz - ez * uy, ez * ux - ex * uz, ex * uy - ey * ux
    a = rng.normal(0.0, 1.0, p.shape) * th0
    b = rng.normal(0.0, 1.0, p.shape) * th0
    dx, dy, dz = ex + a * ux + b * vx, ey + a * uy + b * vy, ez + a * uz + b * vz
    dn = np.sqrt(dx * dx + dy * dy + dz * dz)
    pm = p
    if det.eloss > 0.0:
        E2 = E - det.eloss * t
        pm = np.where(E2 > det.mass, np.sqrt(np.maximum(E2 * E2 - det.mass ** 2, 0.0)), 0.0)
    return pm * dx / dn, pm * dy / dn, pm * dz / dn


def truth_crossings_material(truth: dict, det: Detector, rng: np.random.Generator):
    """Layer by layer from the vertex: the helix to the next cylinder (closed
    form), then that layer's material (scatter_layer) before going on.  The
    crossing point and momentum on each layer are taken before its material.
    Returns pos[L,3,n], mom[L,3,n], reached[L,n] like truth_crossings."""
    n = truth["vx"].shape[0]
    L = det.n_layers
    pos = np.zeros((L, 3, n))
    mom = np.zeros((L, 3, n))
    reached = np.zeros((L, n), dtype=bool)
    x, y, z = truth["vx"].copy(), truth["vy"].copy(), truth["vz"].copy()
    px, py, pz = truth["px"].copy(), truth["py"].copy(), truth["pz"].copy()
    k = C_LIGHT * truth["q"].astype(np.float64) * det.bz
    alive = np.ones(n, dtype=bool)
    for li, r in enumerate(det.radii):
        if li > 0:
            with np.errstate(invalid="ignore", divide="ignore"):  # stopped particles are masked
                npx, npy, npz = scatter_layer(rng, x, y, px, py, pz, det)
            px, py, pz = np.where(alive, npx, px), np.where(alive, npy, py), np.where(alive, npz, pz)
            alive &= np.hypot(px, py) > 0.0
        with np.errstate(invalid="ignore", divide="ignore"):
            cx_, cy_, cz_, cpx, cpy, cpz, ok = _cross_layer(x, y, z, px, py, pz, k, r)
        alive &= ok
        reached[li] = alive
        x, y, z = np.where(alive, cx_, x), np.where(alive, cy_, y), np.where(alive, cz_, z)
        px, py, pz = np.where(alive, cpx, px), np.where(alive, cpy, py), np.where(alive, cpz, pz)
        pos[li] = np.stack([x, y, z])
        mom[li] = np.stack([px, py, pz])
    return pos, mom, reached


def crossings(truth: dict, det: Detector, rng: np.random.Generator):
    """Truth crossings, through the layers' material when the detector has any."""
    if det.x0 > 0.0:
        return truth_crossings_material(truth, det, rng)
    return truth_crossings(truth, det)


def smear_hits(rng: np.random.Generator, pos, det: Detector):
    """Gaussian smearing on the cylinder: phi by N(0, sigma_rphi)/r, z by N(0, sigma_z).

    Hits stay on the layer cylinder (no radial smearing).  Returns hits[L,3,n]
    rounded to FP32-representable values.
    """
    L, _, n = pos.shape
    hits = np.zeros_like(pos)
    for li, r in enumerate(det.radii):
        dphi = rng.normal(0.0, det.sigma_rphi, n) / r
        dz = rng.normal(0.0, det.sigma_z, n)

        def work(sl, li=li, r=r, dphi=dphi, dz=dz):
            phi = np.arctan2(pos[li, 1, sl], pos[li, 0, sl]) + dphi[sl]
            hits[li, 0, sl] = r * np.cos(phi)
            hits[li, 1, sl] = r * np.sin(phi)
            hits[li, 2, sl] = pos[li, 2, sl] + dz[sl]

        _chunked(work, n)
    return f32(hits)


# --------------------------------------------------------------------------
# seeds (input preparation; the filter starts from these)
# --------------------------------------------------------------------------

def _pack(C):
    """C[..., 6, 6] -> packed[21, ...]."""
    return np.stack([C[..., i, j] for (i, j) in PACKED_IJ], axis=0)


def prior_cov(x, y, z, px, py, pz, *, f_par, f_perp, f_pz, f_pzt,
              sig_xy=0.1, sig_z=1.0):
    """Block-diagonal seed covariance, packed [21, n].

    Position: diag(sig_xy^2, sig_xy^2, sig_z^2).  Transverse momentum:
    R(phi_p) diag((f_par pT)^2, (f_perp pT)^2) R(phi_p)^T, i.e. f_par relative
    along the transverse direction and f_perp across it.  pz:
    sigma = f_pz |pz| + f_pzt pT.  No correlations between blocks.
    """
    n = x.shape[0]
    pt = np.hypot(px, py)
    c, s = px / pt, py / pt
    a = (f_par * pt) ** 2
    b = (f_perp * pt) ** 2
    C = np.zeros((n, 6, 6))
    C[:, 0, 0] = sig_xy ** 2
    C[:, 1, 1] = sig_xy ** 2
    C[:, 2, 2] = sig_z ** 2
    C[:, 3, 3] = a * c * c + b * s * s
    C[:, 4, 4] = a * s * s + b * c * c
    C[:, 3, 4] = C[:, 4, 3] = (a - b) * c * s
    C[:, 5, 5] = (f_pz * np.abs(pz) + f_pzt * pt) ** 2
    return _pack(C)


def truth_smeared_seed(rng: np.random.Generator, pos1, mom1, *, f_par=0.1, f_perp=0.01,
                       f_pz=0.1, f_pzt=0.01, sig_xy=0.1, sig_z=1.0):
    """Seed drawn from N(truth at layer 1, C0), with C0 evaluated at the truth.

    pos1, mom1: [3, n] truth crossing of the first layer.  Returns state[6,n]
    and packed cov[21,n], both FP32-representable.  The position is smeared
    off the cylinder, so the filter's first step projects it back.
    """
    x, y, z = pos1
    px, py, pz = mom1
    n = x.shape[0]
    pt = np.hypot(px, py)
    c, s = px / pt, py / pt
    g = rng.normal(size=(6, n))
    dpar = f_par * pt * g[3]
    dperp = f_perp * pt * g[4]
    state = np.stack([
        x + sig_xy * g[0],
        y + sig_xy * g[1],
        z + sig_z * g[2],
        px + c * dpar - s * dperp,
        py + s * dpar + c * dperp,
        pz + (f_pz * np.abs(pz) + f_pzt * pt) * g[5],
    ])
    cov = prior_cov(x, y, z, px, py, pz, f_par=f_par, f_perp=f_perp, f_pz=f_pz,
                    f_pzt=f_pzt, sig_xy=sig_xy, sig_z=sig_z)
    return f32(state), f32(cov)


def three_hit_seed(h1, h2, h3, q, bz, *, pt_cap=1000.0, f_par=0.3, f_perp=0.02,
                   f_pz=0.3, f_pzt=0.02):
    """Seed from the first three hits: circumcircle curvature, chord direction.

    h1, h2, h3: [3, n] hits; q: truth charge.  The transverse radius R comes
    from the circle through the three (x, y) points, pT = c Bz R (capped).  The
    direction at hit 1 is the chord h1->h3 turned by +-alpha/2, where alpha is
    the turning angle between h1 and h3 (sin(alpha/2) = chord/2R), counter-
    clockwise when q Bz > 0.  pz = pT (z3 - z1)/(R alpha).  Position = hit 1.
    The prior is the block-diagonal recipe with looser momentum terms.
    """
    x1, y1, z1 = h1
    x2, y2, _ = h2
    x3, y3, z3 = h3
    a = np.hypot(x2 - x1, y2 - y1)
    b = np.hypot(x3 - x2, y3 - y2)
    cchord = np.hypot(x3 - x1, y3 - y1)
    area2 = np.abs((x2 - x1) * (y3 - y1) - (y2 - y1) * (x3 - x1))  # twice the triangle area
    Rmax = pt_cap / (C_LIGHT * bz)
    with np.errstate(divide="ignore", invalid="ignore"):
        R = np.where(area2 > 0, a * b * cchord / (2.0 * area2), np.inf)
    R = np.minimum(R, Rmax)
    pt = C_LIGHT * bz * R
    half = np.arcsin(np.clip(cchord / (2.0 * R), -1.0, 1.0))
    alpha = 2.0 * half
    ux, uy = (x3 - x1) / cchord, (y3 - y1) / cchord
    sg = np.where(q.astype(np.float64) * bz > 0, 1.0, -1.0)
    ca, sa = np.cos(sg * half), np.sin(sg * half)
    dx = ux * ca - uy * sa
    dy = uy * ca + ux * sa
    arc = R * alpha
    pz = pt * (z3 - z1) / arc
    state = np.stack([x1, y1, z1, pt * dx, pt * dy, pz])
    cov = prior_cov(x1, y1, z1, pt * dx, pt * dy, pz, f_par=f_par, f_perp=f_perp,
                    f_pz=f_pz, f_pzt=f_pzt)
    return f32(state), f32(cov)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass
class FitSet:
    """Inputs of a batched fit plus the truth needed to evaluate it."""
    det: Detector
    state: np.ndarray      # [6, n] seed state at layer 1
    cov: np.ndarray        # [21, n] packed seed covariance
    q: np.ndarray          # [n] int8
    hits: np.ndarray       # [L, 3, n]
    valid: np.ndarray      # [L, n] uint8
    truth_pos: np.ndarray  # [L, 3, n]
    truth_mom: np.ndarray  # [L, 3, n]

    @property
    def n(self) -> int:
        return self.q.shape[0]

    def subset(self, idx):
        idx = np.asarray(idx)
        return FitSet(self.det, self.state[:, idx], self.cov[:, idx], self.q[idx],
                      self.hits[:, :, idx], self.valid[:, idx],
                      self.truth_pos[:, :, idx], self.truth_mom[:, :, idx])


def make_fit_set(rng, n, det: Detector, *, pt_range=(0.5, 10.0), pt_log=False,
                 seed_mode="smeared", drop_out_of_z=True):
    truth = sample_truth(rng, n, pt_range=pt_range, pt_log=pt_log)
    pos, mom, reached = crossings(truth, det, rng)
    hits = smear_hits(rng, pos, det)
    valid = reached.copy()
    if drop_out_of_z:
        valid &= np.abs(pos[:, 2, :]) < det.z_half
    if seed_mode == "smeared":
        state, cov = truth_smeared_seed(rng, pos[0], mom[0])
    elif seed_mode == "3hit":
        state, cov = three_hit_seed(hits[0], hits[1], hits[2], truth["q"], det.bz)
    elif seed_mode == "truth":
        state = f32(np.concatenate([pos[0], mom[0]]))
        _, cov = truth_smeared_seed(rng, pos[0], mom[0])
    else:
        raise ValueError(seed_mode)
    return FitSet(det, state, cov, truth["q"], hits, valid.astype(np.uint8), pos, mom)


def config1(seed_mode="3hit", n=1000, seed=1) -> FitSet:
    """Plain FP64 track fit: 1,000 tracks, 10 layers r=4..40 cm, pT U(0.5,10)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_fit_set(rng, n, barrel(10), seed_mode=seed_mode)


def config2(n=1_000_000, seed=2) -> FitSet:
    """FP32-bulk vs FP64 fit at scale: 1e6 tracks, pT log-uniform 0.5-100 GeV."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_fit_set(rng, n, barrel(10), pt_range=(0.5, 100.0), pt_log=True)


def config2_material(n=1_000_000, seed=6, x0=0.02, eloss=0.036) -> FitSet:
    """The fit at scale through material: layers of 2% X0 with a silicon-like
    mean energy loss (0.036 GeV per X0), pT log-uniform 0.5-100 GeV."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_fit_set(rng, n, barrel(10, x0=x0, eloss=eloss), pt_range=(0.5, 100.0), pt_log=True)


def config4(n_events=2000, seed=4, median=3000.0, sigma=0.8, clip=(50, 50000),
            n_layers=17):
    """Uneven batching: log-normal track counts, 6-17 hits, 0-3 missing layers.

    Per track: n_hits ~ U{6..17}; m ~ U{0..min(3, 17-n_hits)}; the track spans
    layers 1..n_hits+m, of which m distinct layers drawn uniformly from
    4..n_hits+m carry no hit.  Layers beyond the span carry no hit either.
    Returns (FitSet over all events concatenated, event_offsets[n_events+1]).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.clip(np.round(np.exp(rng.normal(math.log(median), sigma, n_events))),
                     clip[0], clip[1]).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(counts)])
    n = int(offs[-1])
    det = barrel(n_layers)
    fs = make_fit_set(rng, n, det)
    nh = rng.integers(6, n_layers + 1, n)
    m = (rng.random(n) * (np.minimum(3, n_layers - nh) + 1)).astype(np.int64)
    span = nh + m
    valid = fs.valid.astype(bool)
    lay = np.arange(n_layers)[:, None]
    valid &= lay < span[None, :]
    keys = rng.random((n_layers - 3, n)).astype(np.float32)
    keys[np.arange(3, n_layers)[:, None] >= span[None, :]] = np.inf
    order = np.argsort(keys, axis=0)
    rankpos = np.empty_like(order)
    np.put_along_axis(rankpos, order, np.arange(n_layers - 3)[:, None], axis=0)
    missing = rankpos < m[None, :]
    valid[3:] &= ~missing
    fs.valid = valid.astype(np.uint8)
    return fs, offs


# --------------------------------------------------------------------------
# building events
# --------------------------------------------------------------------------

@dataclasses.dataclass
class BuildSet:
    """A batch of building events.

    Hits of (event e, layer l) are hits[:, hit_off[e*L+l] : hit_off[e*L+l+1]],
    true hits first in track order, then noise.  Seeds of event e are
    [seed_off[e], seed_off[e+1]).  seed_hit[j, s] is the index, within its
    (event, layer) hit list, of seed s's hit on seed layer j (-1 if absent).
    true_idx[l, s] is the index of the seed's own true hit on layer l (-1 if
    the particle left no hit there).
    """
    det: Detector
    n_events: int
    hit_off: np.ndarray      # int64 [n_events*L + 1]
    hits: np.ndarray         # [3, n_hits_total]
    seed_off: np.ndarray     # int64 [n_events + 1]
    state: np.ndarray        # [6, n_seeds]
    cov: np.ndarray          # [21, n_seeds]
    q: np.ndarray            # int8 [n_seeds]
    seed_hit: np.ndarray     # int32 [3, n_seeds]
    true_idx: np.ndarray     # int32 [L, n_seeds]
    truth_pos: np.ndarray    # [L, 3, n_seeds]
    truth_mom: np.ndarray    # [L, 3, n_seeds]

    @property
    def n_seeds(self) -> int:
        return self.q.shape[0]

    def layer_hits(self, e, l):
        L = self.det.n_layers
        a, b = self.hit_off[e * L + l], self.hit_off[e * L + l + 1]
        return self.hits[:, a:b]

    def event(self, e) -> "BuildSet":
        L = self.det.n_layers
        a, b = self.seed_off[e], self.seed_off[e + 1]
        ho = self.hit_off[e * L:(e + 1) * L + 1]
        return BuildSet(self.det, 1, ho - ho[0], self.hits[:, ho[0]:ho[-1]],
                        np.array([0, b - a], dtype=np.int64), self.state[:, a:b],
                        self.cov[:, a:b], self.q[a:b], self.seed_hit[:, a:b],
                        self.true_idx[:, a:b], self.truth_pos[:, :, a:b],
                        self.truth_mom[:, :, a:b])


def concat_events(events) -> BuildSet:
    det = events[0].det
    L = det.n_layers
    hit_parts, hit_sizes, seeds = [], [], []
    for ev in events:
        assert ev.n_events == 1
        hit_parts.append(ev.hits)
        hit_sizes.append(np.diff(ev.hit_off))
    sizes = np.concatenate(hit_sizes)
    hit_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ns = [ev.n_seeds for ev in events]
    seed_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    cat = lambda name, ax=-1: np.concatenate([getattr(ev, name) for ev in events], axis=ax)
    return BuildSet(det, len(events), hit_off, cat("hits"), seed_off, cat("state"),
                    cat("cov"), cat("q"), cat("seed_hit"), cat("true_idx"),
                    cat("truth_pos"), cat("truth_mom"))


def permute_seeds(bs: BuildSet, perm) -> BuildSet:
    """The same events with the seeds in the order perm (a permutation that
    keeps every event's seeds within the event's range)."""
    perm = np.asarray(perm)
    for e in range(bs.n_events):
        a, b = bs.seed_off[e], bs.seed_off[e + 1]
        assert np.array_equal(np.sort(perm[a:b]), np.arange(a, b)), "perm must stay within events"
    return BuildSet(bs.det, bs.n_events, bs.hit_off, bs.hits, bs.seed_off, bs.state[:, perm],
                    bs.cov[:, perm], bs.q[perm], bs.seed_hit[:, perm], bs.true_idx[:, perm],
                    bs.truth_pos[:, :, perm], bs.truth_mom[:, :, perm])


def eta_order(bs: BuildSet, n_bins=21, eta_max=1.0) -> np.ndarray:
    """A seed order that groups each event's seeds by pseudorapidity bin of
    their momentum (n_bins equal bins over |eta| < eta_max, the outermost
    bins open-ended; stable within a bin), events kept in place: the eta
    partition that the paper's building threads over (Sec. 3), here an
    order in which neighbouring seeds search neighbouring hit bins."""
    px, py, pz = bs.state[3], bs.state[4], bs.state[5]
    eta = np.arcsinh(pz / np.hypot(px, py))
    b = np.clip(np.floor((eta + eta_max) * n_bins / (2.0 * eta_max)), 0, n_bins - 1).astype(np.int64)
    parts = []
    for e in range(bs.n_events):
        a, c = bs.seed_off[e], bs.seed_off[e + 1]
        parts.append(a + np.argsort(b[a:c], kind="stable"))
    return np.concatenate(parts).astype(np.int64) if parts else np.zeros(0, np.int64)


def make_build_event(rng, n_tracks, det: Detector, *, noise_frac=0.2, seed_mode="smeared",
                     pt_range=(0.5, 10.0), pt_log=False):
    """One building event: n_tracks truth tracks plus uniform noise per layer.

    Per layer, the true hits come first in track order (tracks whose crossing
    is missing are skipped), then round(noise_frac * n_true) noise hits with
    phi uniform in [-pi, pi) and z uniform in [-z_half, z_half) on the cylinder.
    """
    truth = sample_truth(rng, n_tracks, pt_range=pt_range, pt_log=pt_log)
    pos, mom, reached = crossings(truth, det, rng)
    hits_t = smear_hits(rng, pos, det)
    present = reached & (np.abs(pos[:, 2, :]) < det.z_half)
    L = det.n_layers
    true_idx = np.full((L, n_tracks), -1, dtype=np.int32)
    layer_hits, sizes = [], []
    for l in range(L):
        sel = np.nonzero(present[l])[0]
        true_idx[l, sel] = np.arange(sel.size, dtype=np.int32)
        nn = int(round(noise_frac * sel.size))
        phi = rng.uniform(-math.pi, math.pi, nn)
        z = rng.uniform(-det.z_half, det.z_half, nn)
        r = det.radii[l]
        noise = f32(np.stack([r * np.cos(phi), r * np.sin(phi), z]))
        layer_hits.append(np.concatenate([hits_t[l][:, sel], noise], axis=1))
        sizes.append(sel.size + nn)
    hit_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    if seed_mode == "smeared":
        state, cov = truth_smeared_seed(rng, pos[0], mom[0])
    elif seed_mode == "3hit":
        state, cov = three_hit_seed(hits_t[0], hits_t[1], hits_t[2], truth["q"], det.bz)
    else:
        raise ValueError(seed_mode)
    return BuildSet(det, 1, hit_off, np.concatenate(layer_hits, axis=1),
                    np.array([0, n_tracks], dtype=np.int64), state, cov, truth["q"],
                    true_idx[:3].copy(), true_idx, pos, mom)


def config3(n_events=100, n_tracks=5000, seed=3, n_layers=17, seed_mode="smeared") -> BuildSet:
    """Combinatorial building: events of 5,000 tracks, 17 layers r=4..68, +20% noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    det = barrel(n_layers)
    return concat_events([make_build_event(rng, n_tracks, det, seed_mode=seed_mode)
                          for _ in range(n_events)])


def config5_stream(n_events=400, rate=1000.0, seed=5, n_layers=17, heavy_frac=0.1,
                   heavy=(20000, 50000), light=5000):
    """Serving load: Poisson arrival times and per-event track counts.

    Returns (arrival_s[n_events], n_tracks[n_events]); events themselves are
    made with make_build_event from the same generator state on demand.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, n_events)
    arrivals = np.cumsum(gaps) - gaps[0]
    heavy_ev = rng.random(n_events) < heavy_frac
    nt = np.where(heavy_ev, rng.integers(heavy[0], heavy[1] + 1, n_events), light)
    return arrivals, nt.astype(np.int64), rng
