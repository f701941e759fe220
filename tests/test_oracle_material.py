"""Pins of the oracle's material effects (multiple scattering as process
noise with the Highland width, mean energy loss), the extension the paper
names as what makes the Kalman filter worthwhile (Sec. 2).

Each check ties the oracle to something other than its own formula: the
generator's independent simulation of the kicks and of the energy loss,
a special case where the Highland logarithm vanishes, finite differences
of the energy-loss map, and the statistics of fits to simulated tracks,
with a counter-check that ignoring the material is caught.
"""
import math

import numpy as np
import pytest

import trackgen as tg
from tests.helpers import pulls


def radial_state(p, phi=0.3, r=12.0, pz=0.0):
    """A state on the cylinder r moving outward along the normal."""
    c, s = math.cos(phi), math.sin(phi)
    return np.array([r * c, r * s, 1.5, p * c, p * s, pz])


def test_no_material_is_identity(orc):
    det = tg.barrel(4)
    x = radial_state(1.0, pz=0.4)
    P = np.diag([1e-4, 2e-4, 1e-2, 1e-3, 2e-3, 3e-3])
    xo, Po = orc.material(det, 1, x, P)
    assert np.array_equal(xo, x) and np.array_equal(Po, P)


def test_highland_special_case(orc):
    """Normal incidence with x0 = beta^2: the path is beta^2 radiation
    lengths, the logarithm vanishes and theta0 = 0.0136 / p, so the trace of
    the process noise, 2 theta0^2 |p|^2, is 2 * 0.0136^2 at any momentum."""
    m = 0.13957
    for p in (0.3, 1.0, 7.0):
        beta2 = p * p / (p * p + m * m)
        det = tg.barrel(4, x0=beta2)
        x = radial_state(p)
        xo, Po = orc.material(det, 2, x, np.zeros((6, 6)))
        assert np.array_equal(xo, x)
        assert abs(np.trace(Po) - 2 * 0.0136 ** 2) < 1e-15
        assert np.allclose(Po @ np.r_[0, 0, 0, x[3:]], 0.0, atol=1e-18)  # no change along p


def test_process_noise_matches_simulated_kicks(orc):
    """The oracle's Q against the covariance of 400,000 momentum kicks drawn
    by the generator at one state (oblique incidence, so the path factor
    matters)."""
    det = tg.barrel(4, x0=0.03)
    x = np.array([3.0, 7.0, -2.0, 0.35, 0.55, 0.4])
    _, Q = orc.material(det, 1, x, np.zeros((6, 6)))
    n = 400_000
    rng = np.random.default_rng(11)
    ones = np.ones(n)
    kx, ky, kz = tg.scatter_layer(rng, x[0] * ones, x[1] * ones, x[3] * ones, x[4] * ones,
                                  x[5] * ones, det)
    dp = np.stack([kx - x[3], ky - x[4], kz - x[5]])
    emp = dp @ dp.T / n
    q = Q[3:, 3:]
    scale = np.trace(q) / 2
    assert np.abs(emp - q).max() < 0.01 * scale, (emp, q)
    assert np.abs(Q[:3]).max() == 0.0 and np.abs(Q[:, :3]).max() == 0.0


def test_energy_loss_matches_generator_and_its_jacobian(orc):
    """Energy loss alone (a negligible scattering width): the momentum after
    the layer equals the generator's, and the covariance transform equals
    finite differences of the map at normal incidence."""
    det = tg.barrel(4, x0=1e-12, eloss=4e10)   # 0.04 GeV per unit path, theta0 ~ 1e-8
    x = radial_state(0.6, pz=0.0)
    xo, _ = orc.material(det, 0, x, np.zeros((6, 6)))
    gx, gy, gz = tg.scatter_layer(np.random.default_rng(1), *(np.array([v]) for v in (x[0], x[1], x[3], x[4], x[5])), det)
    g = np.array([gx[0], gy[0], gz[0]])
    assert abs(np.linalg.norm(xo[3:]) / np.linalg.norm(g) - 1) < 1e-12
    assert np.allclose(xo[3:], g, rtol=0, atol=1e-8)   # directions differ by the ~1e-9 kick
    assert np.array_equal(xo[:3], x[:3])
    assert np.linalg.norm(xo[3:]) < 0.6 - 0.03
    _, Q0 = orc.material(det, 0, x, np.zeros((6, 6)))
    h = 1e-6
    for v in (np.r_[0, 0, 0, x[3:] / np.linalg.norm(x[3:])], np.r_[0, 0, 0, -x[4], x[3], 0] / 0.6,
              np.r_[0, 0, 0, 0, 0, 1.0]):
        eps = 1e-8
        _, Pv = orc.material(det, 0, x, eps * np.outer(v, v))
        Tv_sq = (Pv - Q0) / eps
        xp, _ = orc.material(det, 0, x + h * v, np.zeros((6, 6)))
        xm, _ = orc.material(det, 0, x - h * v, np.zeros((6, 6)))
        d = (xp - xm) / (2 * h)
        assert np.allclose(Tv_sq, np.outer(d, d), rtol=1e-5, atol=1e-9), (v, Tv_sq, np.outer(d, d))


def simulated(det, n, pt_range, seed):
    rng = np.random.default_rng(seed)
    truth = tg.sample_truth(rng, n, pt_range=pt_range)
    pos, mom, reached = tg.crossings(truth, det, rng)
    hits = tg.smear_hits(rng, pos, det)
    valid = reached & (np.abs(pos[:, 2, :]) < det.z_half)
    state, cov = tg.truth_smeared_seed(rng, pos[0], mom[0], f_par=0.03, f_perp=0.003)
    return tg.FitSet(det, state, cov, truth["q"], hits, valid.astype(np.uint8), pos, mom)


def test_fit_through_material_has_unit_pulls(orc):
    """Tracks simulated through 2% X0 layers with energy loss: the filter
    that accounts for the material gives unit pulls and chi2/(2n) near 1
    (3% prior); the same filter ignoring the material does not."""
    det = tg.barrel(10, x0=0.02, eloss=0.036)
    fs = simulated(det, 3000, (0.5, 2.0), 21)
    for material in (True, False):
        o = orc.fit(fs, material=material)
        ok = (o["status"] == 0) & (o["nupd"] == 10)
        assert ok.mean() > 0.95
        c2 = o["chi2"][ok].sum() / (2 * o["nupd"][ok]).sum()
        pg = pulls(o["state"][:, ok], o["cov"][:, ok], fs.truth_pos[-1][:, ok], fs.truth_mom[-1][:, ok])
        rms = {k: float(np.sqrt(np.mean(v ** 2))) for k, v in pg.items()}
        pt_t = np.hypot(fs.truth_mom[-1][0], fs.truth_mom[-1][1])[ok]
        bias = float(np.mean(np.hypot(o["state"][3], o["state"][4])[ok] / pt_t - 1))
        if material:
            assert 0.96 < c2 < 1.05, c2
            assert all(0.96 < v < 1.05 for v in rms.values()), rms
            assert abs(bias) < 0.002, bias
        else:  # momentum covariance far too small: pulls of several sigma
            assert c2 > 1.1 and rms["px"] > 2 and rms["py"] > 2, (c2, rms)


def test_build_through_material(orc):
    """Building with material: the oracle still recovers nearly all of each
    particle's hits on a 17-layer event with 1% X0 layers."""
    det = tg.barrel(17, x0=0.01, eloss=0.036)
    bs = tg.make_build_event(np.random.default_rng(8), 400, det)
    o = orc.build_event(bs, 0)
    assert (o["hit_idx"] == bs.true_idx).all(axis=0).mean() > 0.9
