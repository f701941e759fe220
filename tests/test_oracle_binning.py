"""Pins of the oracle's hit binning.

Hits of each layer are placed into bins so that a track only examines hits
near its prediction (Sec. 3: hits sorted in phi with phi bins for a fast
look-up).  The building workload bins 64 in z by 512 in phi.
"""
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bins_small.txt")


def load_fixture():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        pe, z, zb, pb = line.split()
        phi = eval(pe, {"pi": math.pi})
        rows.append((phi, float(z), int(zb), int(pb)))
    return rows


def test_hand_worked_bins(orc):
    rows = load_fixture()
    hits = np.array([[10 * math.cos(p), 10 * math.sin(p), z] for p, z, _, _ in rows]).T
    offs, perm = orc.bin_layer(hits, 100.0, 64, 512)
    pos = np.empty_like(perm)
    pos[perm] = np.arange(perm.size)
    for i, (_, _, zb, pb) in enumerate(rows):
        b = zb * 512 + pb
        assert offs[b] <= pos[i] < offs[b + 1], (i, zb, pb)


def test_csr_properties(orc):
    rng = np.random.default_rng(1)
    n = 5000
    phi = rng.uniform(-math.pi, math.pi, n)
    z = rng.uniform(-100, 100, n)
    r = 20.0
    hits = np.stack([r * np.cos(phi), r * np.sin(phi), z]).astype(np.float32).astype(np.float64)
    nz, nphi = 64, 512
    offs, perm = orc.bin_layer(hits, 100.0, nz, nphi)
    assert offs[0] == 0 and offs[-1] == n
    assert np.all(np.diff(offs) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(n))
    # every hit lies inside the phi and z range of its bin
    ph = np.arctan2(hits[1], hits[0])
    dphi = 2 * math.pi / nphi
    dz = 200.0 / nz
    for b in range(nz * nphi):
        a, e = offs[b], offs[b + 1]
        if a == e:
            continue
        idx = perm[a:e]
        zb, pb = divmod(b, nphi)
        assert np.all(ph[idx] >= -math.pi + pb * dphi - 1e-12)
        assert np.all(ph[idx] < -math.pi + (pb + 1) * dphi + 1e-12)
        assert np.all(hits[2, idx] >= -100 + zb * dz - 1e-12)
        assert np.all(hits[2, idx] < -100 + (zb + 1) * dz + 1e-12)
        assert np.all(np.diff(idx) > 0)  # original order within a bin


def test_empty_layer(orc):
    offs, perm = orc.bin_layer(np.zeros((3, 0)), 100.0, 64, 512)
    assert perm.size == 0 and np.all(offs == 0)


def test_not_a_number_hits(orc):
    """A hit with a coordinate that is not a number has no bin by the
    formulas: its row is the first when the row's formula gives no number,
    and its phi bin 0 when x or y is not a number.  The hit is kept; the
    other hits bin as usual."""
    nan = float("nan")
    # 0: a plain hit; 1, 2: x or y not a number; 3: z not a number (phi
    # bin of (5, -5): 192 of 512); 4: nothing a number
    hits = np.array([[10.0, nan, 10.0, 5.0, nan],
                     [0.5, 1.0, nan, -5.0, nan],
                     [20.0, 3.0, -7.0, nan, nan]])
    pb0 = int(np.floor((math.atan2(0.5, 10.0) + math.pi) * 512 / (2 * math.pi)))
    zrow = lambda z: int(np.floor((z + 100.0) * 64 / 200.0))
    offs, perm = orc.bin_layer(hits, 100.0, 64, 512)
    bins = {0: [4], 192: [3], zrow(-7.0) * 512: [2], zrow(3.0) * 512: [1], zrow(20.0) * 512 + pb0: [0]}
    for bb, idx in bins.items():
        assert list(perm[offs[bb]:offs[bb + 1]]) == idx, bb
    assert offs[-1] == 5
    # eta rows: x or y not a number leaves no eta either (row 0, bin 0);
    # hit 0 has eta asinh(20 / 10.01) > 1.2: the last of 21 rows
    offs, perm = orc.bin_layer_eta(hits, 1.2, 21, 512)
    bins = {0: [1, 2, 4], 192: [3], 20 * 512 + pb0: [0]}
    for bb, idx in bins.items():
        assert list(perm[offs[bb]:offs[bb + 1]]) == idx, bb
    assert offs[-1] == 5


def test_eta_is_minus_log_tan_half_theta(orc):
    """The pseudorapidity of the eta partition (Sec. 3): -ln tan(theta / 2)
    with theta the polar angle of the point seen from the origin."""
    rng = np.random.default_rng(12)
    for theta in np.concatenate([rng.uniform(0.05, math.pi - 0.05, 200), [math.pi / 2]]):
        rho = rng.uniform(3.0, 70.0)
        ph = rng.uniform(-math.pi, math.pi)
        h = np.array([rho * math.cos(ph), rho * math.sin(ph), rho / math.tan(theta)])
        assert abs(orc.eta(h) - (-math.log(math.tan(theta / 2)))) <= 1e-12 * max(1.0, abs(math.log(math.tan(theta / 2))))
    assert orc.eta(np.array([4.0, 0.0, 0.0])) == 0.0


def test_eta_bins_closed_form(orc):
    """21 eta bins over |eta| < 1.2 by 8 phi bins: points placed at the
    centre of eta bin k and phi bin j on cylinders of several radii land in
    bin (k, j); points beyond |eta| = 1.2 land in the edge rows; within a
    bin hits stay in index order."""
    ne, nphi, em = 21, 8, 1.2
    w = 2 * em / ne
    pts, want = [], []
    for k in range(ne):
        for j in range(nphi):
            for rho in (4.0, 37.0, 68.0):
                eta = -em + (k + 0.5) * w
                ph = -math.pi + (j + 0.5) * 2 * math.pi / nphi
                pts.append((rho * math.cos(ph), rho * math.sin(ph), rho * math.sinh(eta)))
                want.append(k * nphi + j)
    for eta, row in ((1.5, ne - 1), (-2.0, 0), (3.0, ne - 1)):
        pts.append((10.0, 0.0, 10.0 * math.sinh(eta)))
        want.append(row * nphi + nphi // 2)
    hits = np.array(pts).T
    offs, perm = orc.bin_layer_eta(hits, em, ne, nphi)
    want = np.array(want)
    assert np.array_equal(perm, np.argsort(want, kind="stable"))
    assert np.array_equal(offs, np.concatenate([[0], np.cumsum(np.bincount(want, minlength=ne * nphi))]))
