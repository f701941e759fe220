"""GPU parity of the batched Kalman-filter fit against the FP64 oracle.

The fit is the Kalman filter of Sec. 2 run over each track's layers.  FP64
path: every output within 1e-10 of the oracle (relative to the value plus
its own uncertainty), or within ten times the oracle's own rounding spread
where that is larger; float paths: position error / r and momentum error
/ |p| against the FP64 oracle, and pull widths within 1% of the oracle's.
The float path of the headline, FP32_PROP (float storage and state
propagation, the covariance in double), is held to 1e-4 on every track.
FP32 bulk (the covariance rounded to float between layers) meets 1e-4 at
the 99.9th percentile; its tail, up to ~2e-4 on 1e6 tracks at high pT
where the momentum is known to tens of percent, is the float covariance's
and is held to the measured bound.
"""
import json

import numpy as np
import pytest

import trackgen as tg
from helpers import (fit_inputs, fp32_errors, fp64_close, host, oracle_with_spread, pad_pitch, param_rel_errors,
                     pulls)

pytestmark = pytest.mark.gpu

MODES = ["fused", "persistent", "sweep", "sweep_graph"]


@pytest.fixture(scope="module")
def k():
    import paper_1605_05508_amd as k
    return k


@pytest.fixture(scope="module")
def ctx10(k):
    return k.Context(tg.barrel(10).radii)


@pytest.fixture(scope="module")
def c1(orc):
    fs = tg.config1()
    return (fs,) + oracle_with_spread(orc, fs)


@pytest.mark.parametrize("mode", MODES)
def test_fp64_config1_matches_oracle(ctx10, c1, mode):
    fs, o, oc = c1
    d = fit_inputs(fs, "fp64")
    out = ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode)
    g = host(out, fs.n)
    fp64_close(g, o, oc)


def test_fp64_ragged_and_missing_layers(ctx10, orc):
    """Several tiles plus a ragged tail, tracks with missing layers and early
    ends, pitch larger than n."""
    rng = np.random.default_rng(31)
    fs = tg.make_fit_set(rng, 5000 + 37, tg.barrel(10), pt_range=(0.5, 100.0), pt_log=True)
    v = fs.valid.copy()
    v[rng.random(v.shape) < 0.15] = 0
    v[0] = 1
    fs.valid = v
    o, oc = oracle_with_spread(orc, fs)
    d = fit_inputs(fs, "fp64", pitch=pad_pitch(fs.n) + 128)
    for mode in MODES:
        out = ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode)
        fp64_close(host(out, fs.n), o, oc)


def test_modes_agree(ctx10):
    """The fused and persistent kernels share one per-track body, as do the
    per-layer sweep and its graph replay: each pair is bitwise identical and
    every run repeats bitwise.  Between the two families the compiler may
    contract different multiply-adds, so they agree to rounding."""
    rng = np.random.default_rng(32)
    fs = tg.make_fit_set(rng, 3000, tg.barrel(10), pt_range=(0.5, 100.0), pt_log=True)
    for prec in ("fp64", "fp32b"):
        d = fit_inputs(fs, prec)
        run = lambda m: host(ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=m), fs.n)
        res = {m: run(m) for m in MODES}
        again = {m: run(m) for m in MODES}
        for m in MODES:
            for key in res[m]:
                assert np.array_equal(res[m][key], again[m][key]), (prec, m, key)
        for a, b in (("fused", "persistent"), ("sweep", "sweep_graph")):
            for key in res[a]:
                assert np.array_equal(res[a][key], res[b][key]), (prec, a, b, key)
        # FP32 rounding differs between the families at the level of each
        # one's error against the FP64 oracle (a few 1e-5 relative)
        tol = 1e-12 if prec == "fp64" else 2e-4
        f, w = res["fused"], res["sweep"]
        assert np.array_equal(f["nupd"], w["nupd"]) and np.array_equal(f["status"], w["status"])
        np.testing.assert_allclose(w["state"], f["state"], rtol=tol, atol=tol)
        np.testing.assert_allclose(w["chi2"], f["chi2"], rtol=50 * tol, atol=tol)
    d = fit_inputs(fs, "fp32b")
    run = lambda m: host(ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=m,
                                   prec="fp32p"), fs.n)
    f, p, f2 = run("fused"), run("persistent"), run("fused")
    for key in f:
        assert np.array_equal(f[key], p[key]) and np.array_equal(f[key], f2[key]), ("fp32p", key)


# FP32 bulk's documented tail: on 1e6 tracks the largest momentum error is
# 1.3e-4 of |p| and the largest parameter error 1.9e-4 of |x| + sigma, both
# at pT > 10 GeV (about 1e-3 sigma there)
FP32B_TAIL = 2.5e-4


def test_fp32_bulk_accuracy_and_pulls(ctx10, orc):
    fs = tg.config2(n=200_000)
    o = orc.fit(fs)
    d = fit_inputs(fs, "fp32b")
    g = host(ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"]), fs.n)
    assert np.array_equal(g["nupd"], o["nupd"])
    e_pos, e_mom = fp32_errors(g, o, 40.0)
    assert e_pos.max() < 1e-6
    assert np.quantile(e_mom, 0.999) < 1e-4
    assert e_mom.max() < FP32B_TAIL
    assert np.quantile(param_rel_errors(g, o), 0.999) < 1e-4 and param_rel_errors(g, o).max() < FP32B_TAIL
    assert np.abs(g["chi2"] - o["chi2"]).max() / max(1, o["chi2"].max()) < 1e-2
    pg = pulls(g["state"], g["cov"], fs.truth_pos[-1], fs.truth_mom[-1])
    po = pulls(o["state"], o["cov"], fs.truth_pos[-1], fs.truth_mom[-1])
    for name in pg:
        rg, ro = np.sqrt(np.mean(pg[name] ** 2)), np.sqrt(np.mean(po[name] ** 2))
        assert abs(rg / ro - 1) < 0.01, (name, rg, ro)


def test_fp32_prop_accuracy_and_pulls(ctx10, orc):
    """Float state propagation with the covariance kept in double: every
    track within 1e-4 of the FP64 oracle, pulls within 1%."""
    fs = tg.config2(n=200_000)
    o = orc.fit(fs)
    d = fit_inputs(fs, "fp32b")
    for mode in ("fused", "persistent"):
        g = host(ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode, prec="fp32p"), fs.n)
        assert np.array_equal(g["nupd"], o["nupd"]) and np.all(g["status"] == o["status"])
        e_pos, e_mom = fp32_errors(g, o, 40.0)
        assert e_pos.max() < 1e-6
        assert e_mom.max() < 1e-4
        assert param_rel_errors(g, o).max() < 1e-4
        pg = pulls(g["state"], g["cov"], fs.truth_pos[-1], fs.truth_mom[-1])
        po = pulls(o["state"], o["cov"], fs.truth_pos[-1], fs.truth_mom[-1])
        for name in pg:
            rg, ro = np.sqrt(np.mean(pg[name] ** 2)), np.sqrt(np.mean(po[name] ** 2))
            assert abs(rg / ro - 1) < 0.01, (name, rg, ro)


def test_fp32_prop_rejects_sweep(k, ctx10):
    fs = tg.config2(n=100)
    d = fit_inputs(fs, "fp32b")
    for mode in ("sweep", "sweep_graph"):
        with pytest.raises(k.KtfError):
            ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode, prec="fp32p")


def test_full_size_sampled(ctx10, orc):
    """Config 2 at its full 1e6 tracks in the launch the benchmark times;
    a sample of tracks is checked against the oracle one by one."""
    fs = tg.config2()
    for prec in ("fp64", "fp32b", "fp32p"):
        d = fit_inputs(fs, "fp32b" if prec == "fp32p" else prec)
        pp = None if prec == "fp32b" else prec
        # the benchmark's launch: the tuned shape for this precision and size
        ctx10.autotune_fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], prec=pp)
        g = host(ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode="auto", prec=pp), fs.n)
        idx = np.random.default_rng(7).choice(fs.n, 3000, replace=False)
        sub = fs.subset(idx)
        o = orc.fit(sub)
        gs = {key: v[..., idx] for key, v in g.items()}
        if prec == "fp64":
            fp64_close(gs, o, oracle_with_spread(orc, sub)[1])
        else:
            e_pos, e_mom = fp32_errors(gs, o, 40.0)
            assert e_mom.max() < (FP32B_TAIL if prec == "fp32b" else 1e-4) and e_pos.max() < 1e-6
            if prec == "fp32p":
                assert param_rel_errors(gs, o).max() < 1e-4
        assert np.all(g["status"] == 0)
        assert np.all(g["nupd"] == 10)


def test_status_flags(ctx10, orc):
    """Tracks 0..9 are too soft to reach the layers beyond ~27 cm (tight
    prior, no hits in between so nothing corrects the momentum): NO_REACH,
    with the last state kept.  Tracks 20..24 carry a NaN hit on layer 5: the
    residual covariance is not positive definite there, the hit is skipped
    (S_NOT_PD) and the fit goes on.  Tracks 30..34 have no hit on the first
    layer and a seed covariance with an infinite pz variance (a prior with
    no information on pz): the propagated covariance is not finite before
    any S is formed, so the fit stops there with NONFINITE alone."""
    rng = np.random.default_rng(33)
    fs = tg.make_fit_set(rng, 256, tg.barrel(10))
    st = fs.state.copy()
    ptl = 0.9 * 0.00299792458 * 3.8 * 30.0 / 2
    ph = np.arctan2(st[4, :10], st[3, :10])
    st[3, :10], st[4, :10] = ptl * np.cos(ph), ptl * np.sin(ph)
    cov = fs.cov.copy()
    P0 = np.diag([1e-4, 1e-4, 1e-2, (0.01 * ptl) ** 2, (0.01 * ptl) ** 2, 1e-4])
    for kk, (i, j) in enumerate([(i, j) for i in range(6) for j in range(i, 6)]):
        cov[kk, :10] = P0[i, j]
    valid = fs.valid.copy()
    valid[1:9, :10] = 0
    hits = fs.hits.copy()
    hits[5, 0, 20:25] = np.nan
    cov[20, 30:35] = np.inf
    valid[0, 30:35] = 0
    fs2 = tg.FitSet(fs.det, st, cov, fs.q, hits, valid, fs.truth_pos, fs.truth_mom)
    o, oc = oracle_with_spread(orc, fs2)
    assert np.all(o["status"][:10] == orc.NO_REACH) and np.all(o["status"][20:25] == orc.S_NOT_PD)
    assert np.all(o["status"][30:35] == orc.NONFINITE) and np.all(o["nupd"][30:35] == 0)
    for prec in ("fp64", "fp32b", "fp32p"):
        d = fit_inputs(fs2, "fp32b" if prec == "fp32p" else prec)
        for mode in (MODES if prec != "fp32p" else ["fused", "persistent"]):
            g = host(ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode,
                               prec=None if prec == "fp32b" else prec), fs.n)
            assert np.array_equal(g["status"].astype(np.uint32), o["status"]), (prec, mode)
            assert np.array_equal(g["nupd"], o["nupd"]), (prec, mode)
        if prec == "fp64":
            fp64_close(g, o, oc)


def test_empty_and_single(ctx10, orc):
    import torch
    fs = tg.config1(n=1)
    o = orc.fit(fs)
    d = fit_inputs(fs, "fp64")
    fp64_close(host(ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"]), 1), o)
    e = ctx10.fit(d["state"], d["cov"], d["q"][:0], d["hits"], d["valid"])
    torch.cuda.synchronize()
    assert e["state"].shape[1] == 64


def test_autotune_keeps_results(ctx10):
    """Whatever block size, persistence and register budget the autotuner
    picks with one track per lane, the results are bitwise those of the
    default fused launch; with two tracks per lane they agree to rounding."""
    rng = np.random.default_rng(34)
    fs = tg.make_fit_set(rng, 20000, tg.barrel(10))
    for prec in ("fp32b", "fp64", "fp32p"):
        d = fit_inputs(fs, "fp64" if prec == "fp64" else "fp32b")
        pp = None if prec == "fp32b" else prec
        ref = host(ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode="fused", prec=pp), fs.n)
        # the tuner leaves the outputs of the last shape it timed: 512 per
        # block, persistent, three waves per SIMD, two tracks per lane.  The
        # two tracks' arithmetic is the same but compiled in another context,
        # where the compiler fuses other multiply-adds: agreement to rounding
        last = host(ctx10.autotune_fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], prec=pp), fs.n)
        assert np.array_equal(ref["nupd"], last["nupd"]) and np.array_equal(ref["status"], last["status"])
        tol = 1e-12 if prec == "fp64" else 2e-4
        np.testing.assert_allclose(last["state"], ref["state"], rtol=tol, atol=tol)
        np.testing.assert_allclose(last["chi2"], ref["chi2"], rtol=50 * tol, atol=tol)
        assert '"tuned": true' in ctx10.tuned_shape(prec, fs.n)
        shape = json.loads(ctx10.tuned_shape(prec, fs.n, trials=True))
        trials = shape["trials"]   # [block, waves per SIMD, persistent, tracks per lane, ms] per shape
        assert len(trials) == 48 and len({tuple(t[:4]) for t in trials}) == 48
        chosen = [t for t in trials if [t[0], t[1], bool(t[2]), t[3]] ==
                  [shape["block"], shape["waves_per_simd"], shape["persistent"], shape["tracks_per_lane"]]]
        assert len(chosen) == 1 and chosen[0][4] <= min(t[4] for t in trials) + 1e-6   # the fastest
        assert abs(chosen[0][4] - shape["ms"]) < 1e-6
        g = host(ctx10.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode="auto", prec=pp), fs.n)
        if shape["tracks_per_lane"] == 1:
            for key in ref:
                assert np.array_equal(ref[key], g[key]), (prec, key, ctx10.tuned_shape(prec, fs.n))
        else:
            assert np.array_equal(ref["nupd"], g["nupd"]) and np.array_equal(ref["status"], g["status"])
            np.testing.assert_allclose(g["state"], ref["state"], rtol=tol, atol=tol)


def test_bad_arguments_raise(ctx10):
    import torch
    fs = tg.config1(n=10)
    d = fit_inputs(fs, "fp64")
    with pytest.raises(ValueError):
        ctx10.fit(d["state"].float(), d["cov"], d["q"], d["hits"], d["valid"])
    with pytest.raises(ValueError):
        ctx10.fit(d["state"], d["cov"], d["q"], d["hits"][:5], d["valid"])
