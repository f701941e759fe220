"""GPU parity of fitting and building through layer material (multiple
scattering as process noise with the Highland width, mean energy loss)
against the FP64 oracle: FP64 within 1e-10, float paths within their
tolerances, building indices bit-exact in FP64."""
import numpy as np
import pytest

import trackgen as tg
from helpers import (build_inputs, certified, fit_inputs, fp32_errors, fp64_close, host, oracle_with_spread,
                     pad_pitch, pulls)

pytestmark = pytest.mark.gpu

MODES = ["fused", "persistent", "sweep", "sweep_graph"]


@pytest.fixture(scope="module")
def k():
    import paper_1605_05508_amd as k
    return k


def simulated(det, n, pt_range, seed, missing=0.0):
    rng = np.random.default_rng(seed)
    truth = tg.sample_truth(rng, n, pt_range=pt_range)
    pos, mom, reached = tg.crossings(truth, det, rng)
    hits = tg.smear_hits(rng, pos, det)
    valid = reached & (np.abs(pos[:, 2, :]) < det.z_half)
    if missing > 0:
        valid[1:] &= rng.random(valid[1:].shape) >= missing
    state, cov = tg.truth_smeared_seed(rng, pos[0], mom[0], f_par=0.03, f_perp=0.003)
    return tg.FitSet(det, state, cov, truth["q"], hits, valid.astype(np.uint8), pos, mom)


def test_fp64_fit_through_material(k, orc):
    """Several tiles and a ragged tail, missing layers, every launch mode."""
    det = tg.barrel(10, x0=0.02, eloss=0.036)
    fs = simulated(det, 3000 + 37, (0.5, 10.0), 41, missing=0.1)
    o, oc = oracle_with_spread(orc, fs)
    ctx = k.Context.for_detector(det)
    d = fit_inputs(fs, "fp64", pitch=pad_pitch(fs.n) + 64)
    for mode in MODES:
        g = host(ctx.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode), fs.n)
        fp64_close(g, o, oc)


def test_fp64_fit_energy_loss_stops_tracks(k, orc):
    """Heavy energy loss slows tracks down until they curl up before the
    outer layers: the fits end early, some with NO_REACH (the filter's
    estimate no longer reaches a layer that still has a hit), keeping their
    last filtered state."""
    det = tg.barrel(10, x0=0.05, eloss=0.4)
    fs = simulated(det, 2000, (0.15, 0.6), 42)
    o, oc = oracle_with_spread(orc, fs)
    assert 0.01 < np.mean(o["status"] == orc.NO_REACH) < 0.9
    ctx = k.Context.for_detector(det)
    d = fit_inputs(fs, "fp64")
    # at these momenta the energy loss per layer is several percent and the
    # linearised filter is far from linear (chi2/ndf up to ~40 for some
    # tracks): the oracle's own rounding spread grows to ~5e-9 on such
    # tracks, which then hold to ten times their spread
    for mode in MODES:
        g = host(ctx.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode), fs.n)
        fp64_close(g, o, oc)


def test_float_fits_through_material(k, orc):
    det = tg.barrel(10, x0=0.02, eloss=0.036)
    fs = simulated(det, 50_000, (0.5, 20.0), 43)
    o = orc.fit(fs)
    ctx = k.Context.for_detector(det)
    d = fit_inputs(fs, "fp32b")
    po = pulls(o["state"], o["cov"], fs.truth_pos[-1], fs.truth_mom[-1])
    for prec, mode in (("fp32b", "fused"), ("fp32b", "sweep_graph"), ("fp32p", "persistent")):
        g = host(ctx.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode,
                         prec=None if prec == "fp32b" else prec), fs.n)
        assert np.array_equal(g["nupd"], o["nupd"])
        e_pos, e_mom = fp32_errors(g, o, 40.0)
        assert e_pos.max() < 1e-6
        # FP32 bulk's float covariance leaves a tail above 1e-4 (measured
        # below 2.5e-4); FP32_PROP, the headline float path, holds 1e-4 on
        # every track
        assert np.quantile(e_mom, 0.999) < 1e-4 and e_mom.max() < (2.5e-4 if prec == "fp32b" else 1e-4)
        pg = pulls(g["state"], g["cov"], fs.truth_pos[-1], fs.truth_mom[-1])
        for name in pg:
            rg, ro = np.sqrt(np.mean(pg[name] ** 2)), np.sqrt(np.mean(po[name] ** 2))
            assert abs(rg / ro - 1) < 0.01, (prec, mode, name, rg, ro)


def test_build_through_material(k, orc):
    """Building with 1% X0 layers and energy loss: FP64 hit indices, hit
    counts and the kept (parent, hit) lists of every layer exactly as the
    oracle's; FP32 bulk up to certified near-ties."""
    det = tg.barrel(17, x0=0.01, eloss=0.036)
    rng = np.random.default_rng(44)
    bs = tg.concat_events([tg.make_build_event(rng, 300, det) for _ in range(2)])
    ctx = k.Context.for_detector(det)
    outs = [orc.build_event(bs, e, debug=True) for e in range(bs.n_events)]
    o = {key: np.concatenate([x[key] for x in outs], axis=-1) for key in outs[0]}
    d = build_inputs(bs, "fp64")
    g = host(ctx.build(d, hist=True), bs.n_seeds)
    assert np.array_equal(g["hit_idx"], o["hit_idx"])
    assert np.array_equal(g["nhits"], o["nhits"])
    np.testing.assert_allclose(g["chi2"], o["chi2"], rtol=1e-10)
    assert (g["hit_idx"] == bs.true_idx).all(axis=0).mean() > 0.9
    d = build_inputs(bs, "fp32b")
    g = host(ctx.build(d, hist=True), bs.n_seeds)
    for s in range(bs.n_seeds):
        if np.array_equal(g["hit_idx"][:, s], o["hit_idx"][:, s]):
            continue
        ok, layer = certified(o["dbg_n"][:, s], o["dbg"][:, :, :, s], o["margin"][:, s],
                              g["count"][:, s], g["hist"][:, :, :, s])
        assert ok, (s, layer)
