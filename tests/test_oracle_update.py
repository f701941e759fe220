"""Pins of the oracle's Kalman update and covariance algebra.

Textbook Kalman filter (the method named in Sec. 2; matrices of sizes 3x3
to 6x6 per Sec. 2.1): gain K = P H^T S^-1 with S = H P H^T + V, and the
covariance update.  The pins are special cases with closed forms and
algebraic identities that a dropped term, a sign or a transposed operand
would break.
"""
import math

import numpy as np
import pytest


def spd(rng, n, scale=1.0):
    A = rng.normal(size=(n, n))
    return scale * (A @ A.T + n * np.eye(n))


def test_diagonal_reduces_to_scalar_updates(orc):
    """With P diagonal and V diagonal every coordinate updates on its own:
    x+ = x + p/(p+v) (m-x), P+ = p v/(p+v), chi2 = sum (m-x)^2/(p+v)."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        p = rng.uniform(0.01, 4.0, 6)
        v = rng.uniform(0.01, 4.0, 3)
        x = rng.normal(size=6)
        m = rng.normal(size=3)
        xo, Po, c2, rc = orc.update(x, np.diag(p), m, np.diag(v))
        assert rc == 0
        g = p[:3] / (p[:3] + v)
        np.testing.assert_allclose(xo[:3], x[:3] + g * (m - x[:3]), rtol=1e-13, atol=1e-14)
        np.testing.assert_array_equal(xo[3:], x[3:])
        np.testing.assert_allclose(np.diag(Po)[:3], p[:3] * v / (p[:3] + v), rtol=1e-13)
        np.testing.assert_allclose(np.diag(Po)[3:], p[3:], rtol=1e-15)
        assert c2 == pytest.approx(np.sum((m - x[:3]) ** 2 / (p[:3] + v)), rel=1e-13)


def test_joseph_equals_simple_form(orc):
    """Joseph (I-KH)P(I-KH)^T + KVK^T equals P - K S K^T for the optimal gain."""
    rng = np.random.default_rng(2)
    for _ in range(100):
        P = spd(rng, 6)
        V = spd(rng, 3, 0.1)
        x = rng.normal(size=6)
        m = rng.normal(size=3)
        xo, Po, c2, rc = orc.update(x, P, m, V)
        S = P[:3, :3] + V
        K = P[:, :3] @ np.linalg.inv(S)
        np.testing.assert_allclose(Po, P - K @ S @ K.T, rtol=1e-11, atol=1e-12 * np.abs(P).max())
        np.testing.assert_allclose(xo, x + K @ (m - x[:3]), rtol=1e-12, atol=1e-13)
        r = m - x[:3]
        assert c2 == pytest.approx(r @ np.linalg.solve(S, r), rel=1e-12)
        # symmetric and shrinking in the Loewner order
        np.testing.assert_allclose(Po, Po.T, rtol=0, atol=1e-13 * np.abs(Po).max())
        assert np.linalg.eigvalsh(P - Po).min() >= -1e-10 * np.abs(P).max()


def test_information_form(orc):
    """P+^-1 = P^-1 + H^T V^-1 H, and x+ minimises the two-term quadratic."""
    rng = np.random.default_rng(3)
    H = np.hstack([np.eye(3), np.zeros((3, 3))])
    for _ in range(50):
        P = spd(rng, 6)
        V = spd(rng, 3, 0.3)
        x = rng.normal(size=6)
        m = rng.normal(size=3)
        xo, Po, c2, rc = orc.update(x, P, m, V)
        Ii = np.linalg.inv(P) + H.T @ np.linalg.inv(V) @ H
        np.testing.assert_allclose(np.linalg.inv(Po), Ii, rtol=1e-9, atol=1e-9)
        xs = np.linalg.solve(Ii, np.linalg.solve(P, x) + H.T @ np.linalg.solve(V, m))
        np.testing.assert_allclose(xo, xs, rtol=1e-9, atol=1e-10)
        # chi2 increment = minimum of the objective
        obj = (xs - x) @ np.linalg.solve(P, xs - x) + (m - H @ xs) @ np.linalg.solve(V, m - H @ xs)
        assert c2 == pytest.approx(obj, rel=1e-8)


def test_hit_covariance_axes(orc):
    rng = np.random.default_rng(4)
    for _ in range(50):
        ph = rng.uniform(-math.pi, math.pi)
        r = rng.uniform(4, 70)
        m = np.array([r * math.cos(ph), r * math.sin(ph), rng.uniform(-100, 100)])
        V = orc.hit_cov(m, 0.02, 0.01, 0.1)
        rad = np.array([math.cos(ph), math.sin(ph), 0])
        tan = np.array([-math.sin(ph), math.cos(ph), 0])
        ez = np.array([0, 0, 1.0])
        np.testing.assert_allclose(V @ rad, 0.02 ** 2 * rad, atol=1e-17)
        np.testing.assert_allclose(V @ tan, 0.01 ** 2 * tan, atol=1e-17)
        np.testing.assert_allclose(V @ ez, 0.1 ** 2 * ez, atol=1e-17)


def test_not_positive_definite_is_reported(orc):
    P = np.zeros((6, 6))
    V = np.zeros((3, 3))
    xo, Po, c2, rc = orc.update(np.zeros(6), P, np.ones(3), V)
    assert rc == orc.S_NOT_PD
    assert orc.chi2(np.zeros(6), P, np.ones(3), V)[1] == orc.S_NOT_PD


def test_cov_propagate_definition(orc):
    rng = np.random.default_rng(5)
    F = rng.normal(size=(6, 6))
    P = spd(rng, 6)
    np.testing.assert_allclose(orc.cov_propagate(P, F), F @ P @ F.T, rtol=1e-13, atol=1e-12)


def test_radial_null_direction_and_sigma_r_invariance(orc):
    """After a constrained propagation P' has the surface normal as null
    vector; the radial hit variance then leaves gain, state and covariance
    unchanged to first order and P+ keeps the null vector."""
    rng = np.random.default_rng(6)
    for _ in range(30):
        pt = rng.uniform(0.5, 20)
        ph = rng.uniform(0, 2 * math.pi)
        x = np.array([0.01, -0.02, 0.3, pt * math.cos(ph), pt * math.sin(ph), rng.uniform(-2, 2)])
        P0 = spd(rng, 6, 1e-3)
        xp, F, s, rc = orc.propagate(x, 1, 3.8, 20.0)
        Pp = orc.cov_propagate(P0, F)
        rho = math.hypot(xp[0], xp[1])
        n = np.array([xp[0] / rho, xp[1] / rho, 0, 0, 0, 0])
        assert np.abs(Pp @ n).max() <= 1e-10 * np.abs(Pp).max()
        ev = np.linalg.eigvalsh(Pp)
        assert ev[1] > 1e3 * abs(ev[0])  # rank 5
        # hit exactly on the predicted radial line
        m = np.array([xp[0] + 0.003 * n[1], xp[1] - 0.003 * n[0], xp[2] + 0.05])
        m[:2] *= 20.0 / math.hypot(m[0], m[1])
        outs = []
        for sr in (0.01, 0.05):
            V = orc.hit_cov(m, sr, 0.01, 0.1)
            outs.append(orc.update(xp, Pp, m, V))
        (xa, Pa, ca, _), (xb, Pb, cb, _) = outs
        sig = np.sqrt(np.maximum(np.diag(Pa), 1e-30))
        assert np.all(np.abs(xa - xb) <= 1e-5 * sig + 1e-12)
        assert np.abs(Pa - Pb).max() <= 1e-5 * np.abs(Pa).max()
        assert np.abs(Pa @ n).max() <= 1e-8 * np.abs(Pa).max()
