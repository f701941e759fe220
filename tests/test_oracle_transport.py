"""Pins of the oracle's helix propagation against closed forms.

The paper names the method (a Kalman filter propagating tracks between
barrel layers, Sec. 2) but prints no equations; these tests tie the oracle's
propagation to the geometry of a charged particle in a uniform field:
straight lines without field, circles in the transverse plane with it, and
finite differences of the surface-to-surface map for the Jacobian.
"""
import math

import numpy as np
import pytest

import trackgen as tg

CL = 0.00299792458


def rand_state(rng, pt_lo=0.5, pt_hi=50.0, rho=3.0):
    pt = rng.uniform(pt_lo, pt_hi)
    ph = rng.uniform(0, 2 * math.pi)
    return np.array([rng.uniform(-rho, rho), rng.uniform(-rho, rho), rng.uniform(-5, 5),
                     pt * math.cos(ph), pt * math.sin(ph), rng.uniform(-3, 3)])


def test_straight_line_when_field_off(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        x = rand_state(rng)
        r = rng.uniform(6, 40)
        xo, F, s, rc = orc.propagate(x, 1, 0.0, r)
        assert rc == 0
        pt = math.hypot(x[3], x[4])
        u = (x[0] * x[3] + x[1] * x[4]) / pt
        s_ref = -u + math.sqrt(u * u + r * r - x[0] ** 2 - x[1] ** 2)
        ref = np.array([x[0] + s_ref * x[3] / pt, x[1] + s_ref * x[4] / pt,
                        x[2] + s_ref * x[5] / pt, x[3], x[4], x[5]])
        assert s == pytest.approx(s_ref, rel=1e-14, abs=1e-13)
        np.testing.assert_allclose(xo, ref, rtol=1e-13, atol=1e-13)


def two_circle_first_crossing(x, q, bz, r):
    """First crossing of the track circle with the layer circle, written out
    independently of the oracle (intersection of two circles, then the
    smaller turning angle in the direction of motion)."""
    k = CL * q * bz
    pt = math.hypot(x[3], x[4])
    R = pt / abs(k)
    cx, cy = x[0] + x[4] / k, x[1] - x[3] / k
    d = math.hypot(cx, cy)
    a = (r * r - R * R + d * d) / (2 * d)
    h = math.sqrt(r * r - a * a)
    best = None
    for sg in (1, -1):
        X = a * cx / d - sg * h * cy / d
        Y = a * cy / d + sg * h * cx / d
        v0 = (x[0] - cx, x[1] - cy)
        v1 = (X - cx, Y - cy)
        ang = math.atan2(v0[0] * v1[1] - v0[1] * v1[0], v0[0] * v1[0] + v0[1] * v1[1])
        if k > 0 and ang > 0:
            ang -= 2 * math.pi
        if k < 0 and ang < 0:
            ang += 2 * math.pi
        s = abs(ang) * R
        if best is None or s < best[0]:
            best = (s, X, Y, ang)
    return best, (cx, cy, R)


def test_circle_closed_form(orc):
    rng = np.random.default_rng(2)
    for _ in range(300):
        x = rand_state(rng, 0.5, 100.0)
        q = int(rng.choice([-1, 1]))
        r = rng.uniform(6, 40)
        xo, F, s, rc = orc.propagate(x, q, 3.8, r)
        assert rc == 0
        (s_ref, X, Y, ang), (cx, cy, R) = two_circle_first_crossing(x, q, 3.8, r)
        pt = math.hypot(x[3], x[4])
        assert s == pytest.approx(s_ref, rel=1e-11, abs=1e-11)
        assert xo[0] == pytest.approx(X, abs=1e-10)
        assert xo[1] == pytest.approx(Y, abs=1e-10)
        # on both circles
        assert math.hypot(xo[0], xo[1]) == pytest.approx(r, rel=1e-13)
        assert math.hypot(xo[0] - cx, xo[1] - cy) == pytest.approx(R, rel=1e-11)
        # pT conserved, pz constant, pz/pT constant, z linear in the arc length
        assert math.hypot(xo[3], xo[4]) == pytest.approx(pt, rel=1e-13)
        assert xo[5] == x[5]
        assert xo[2] == pytest.approx(x[2] + s_ref * x[5] / pt, abs=1e-10)
        # the momentum turned by the same angle as the radius vector
        turn = math.atan2(x[3] * xo[4] - x[4] * xo[3], x[3] * xo[3] + x[4] * xo[4])
        assert turn == pytest.approx(ang, abs=1e-11)
        assert turn == pytest.approx(-CL * q * 3.8 * s / pt, abs=1e-11)


def test_matches_generator_truth(orc):
    """The generator finds crossings with a closed-form intersection; the
    oracle's arc-length Newton solve must land on the same points."""
    rng = np.random.default_rng(3)
    det = tg.barrel(10)
    tr = tg.sample_truth(rng, 200, pt_range=(0.5, 100.0), pt_log=True)
    pos, mom, reached = tg.truth_crossings(tr, det)
    for i in range(200):
        x = np.array([tr["vx"][i], tr["vy"][i], tr["vz"][i], tr["px"][i], tr["py"][i], tr["pz"][i]])
        for l, r in enumerate(det.radii):
            xo, F, s, rc = orc.propagate(x, int(tr["q"][i]), det.bz, r)
            assert rc == 0
            np.testing.assert_allclose(xo[:3], pos[l, :, i], atol=1e-9)
            np.testing.assert_allclose(xo[3:], mom[l, :, i], rtol=1e-10, atol=1e-12)
            x = xo


def test_forward_backward_returns(orc):
    rng = np.random.default_rng(4)
    for _ in range(100):
        x = rand_state(rng)
        q = int(rng.choice([-1, 1]))
        s = rng.uniform(1, 60)
        y = orc.transport(x, q, 3.8, s)
        z = orc.transport(y, q, 3.8, -s)
        np.testing.assert_allclose(z, x, rtol=1e-12, atol=1e-12)


def test_no_reach(orc):
    # pT so low that the circle diameter is below the layer radius
    r = 40.0
    pt = 0.9 * CL * 3.8 * r / 2
    x = np.array([0.0, 0.0, 0.0, pt, 0.0, 0.1])
    assert orc.propagate(x, 1, 3.8, r)[3] == orc.NO_REACH
    assert orc.propagate(x, 1, 3.8, 0.5 * r)[3] == 0


def constrained_map(orc, x, q, bz, r, nearest):
    return orc.propagate(x, q, bz, r, nearest)[0]


@pytest.mark.parametrize("nearest", [False, True])
def test_jacobian_finite_differences(orc, nearest):
    rng = np.random.default_rng(5)
    for _ in range(100):
        x = rand_state(rng, 0.5, 50.0)
        q = int(rng.choice([-1, 1]))
        if nearest:
            # a seed-like start: near the layer, on either side, heading
            # roughly outward (within 0.5 rad of radial)
            rho = rng.uniform(3.0, 6.0)
            ph = rng.uniform(0, 2 * math.pi)
            pt = math.hypot(x[3], x[4])
            pd = ph + rng.uniform(-0.5, 0.5)
            x[0], x[1] = rho * math.cos(ph), rho * math.sin(ph)
            x[3], x[4] = pt * math.cos(pd), pt * math.sin(pd)
            r = rho + rng.uniform(-0.3, 0.3)
        else:
            r = rng.uniform(8, 40)
        xo, F, s, rc = orc.propagate(x, q, 3.8, r, nearest)
        assert rc == 0
        Fn = np.zeros((6, 6))
        for j in range(6):
            h = 1e-6 * max(1.0, abs(x[j]))
            a, b = x.copy(), x.copy()
            a[j] += h
            b[j] -= h
            Fn[:, j] = (constrained_map(orc, a, q, 3.8, r, nearest)
                        - constrained_map(orc, b, q, 3.8, r, nearest)) / (2 * h)
        scale = np.maximum(1.0, np.abs(F))
        assert np.all(np.abs(F - Fn) <= 1e-6 * scale)


def test_jacobian_structure(orc):
    rng = np.random.default_rng(6)
    for _ in range(100):
        x = rand_state(rng)
        q = int(rng.choice([-1, 1]))
        xo, F, s, rc = orc.propagate(x, q, 3.8, rng.uniform(8, 40))
        e = np.eye(6)
        np.testing.assert_array_equal(F[:, 2], e[:, 2])  # z enters only z'
        np.testing.assert_array_equal(F[5, :], e[5, :])  # pz' = pz
        # transverse rows do not depend on z or pz
        np.testing.assert_array_equal(F[[0, 1, 3, 4]][:, [2, 5]], 0.0)
        # the surface normal is a left null vector: no state change moves
        # the propagated point off the cylinder to first order
        rho = math.hypot(xo[0], xo[1])
        n = np.array([xo[0] / rho, xo[1] / rho, 0, 0, 0, 0])
        assert np.abs(n @ F).max() <= 1e-12 * np.abs(F).max()
