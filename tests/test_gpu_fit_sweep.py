"""A sweep of fit configurations against the FP64 oracle: one layer, the
largest layer count, low-momentum tracks that stop before the outer layers,
random missing layers, material, odd track counts and pitches, radial and
tangential hit resolutions that differ (so the hit covariance is a true
rotation of diag(sr^2, srphi^2, sz^2) by the hit's phi), in every launch
mode.  FP64 within 1e-10 (graded for poorly fitted tracks), status and hit
counts exact."""
import numpy as np
import pytest

import trackgen as tg
from helpers import fit_inputs, fp64_close, host, oracle_with_spread, pad_pitch

pytestmark = pytest.mark.gpu

MODES = ["fused", "persistent", "sweep", "sweep_graph"]
CASES = [
    # (seed, layers, tracks, pT range, missing-layer fraction, x0, detector resolutions)
    (201, 1, 333, (0.5, 10.0), 0.0, 0.0, {}),
    (202, 32, 517, (1.0, 20.0), 0.1, 0.0, {}),
    (203, 10, 1001, (0.12, 0.6), 0.0, 0.0, {}),
    (204, 17, 777, (0.5, 10.0), 0.3, 0.01, {}),
    (205, 6, 64, (2.0, 50.0), 0.0, 0.03, {}),
    (206, 10, 900, (0.5, 10.0), 0.1, 0.0, dict(sigma_r=0.02, sigma_rphi=0.01)),
    (207, 10, 700, (1.0, 50.0), 0.0, 0.0, dict(sigma_r=0.05, sigma_rphi=0.01)),
    (208, 12, 500, (0.5, 10.0), 0.0, 0.01, dict(sigma_r=0.01, sigma_rphi=0.03)),
]


@pytest.fixture(scope="module")
def k():
    import paper_1605_05508_amd as k
    return k


@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_fit_configurations(k, orc, case):
    seed, L, n, pt_range, miss, x0, res = case
    rng = np.random.default_rng(seed)
    det = tg.barrel(L, x0=x0, eloss=0.036 if x0 > 0 else 0.0, **res)
    fs = tg.make_fit_set(rng, n, det, pt_range=pt_range)
    if miss > 0:
        drop = rng.random(fs.valid.shape) < miss
        drop[0] = False
        fs.valid[drop] = 0
    o, oc = oracle_with_spread(orc, fs)
    ctx = k.Context.for_detector(det, n_seed_layers=min(3, L))  # building needs n_seed_layers <= layers
    d = fit_inputs(fs, "fp64", pitch=pad_pitch(n) + 128)
    for mode in MODES:
        g = host(ctx.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode), n)
        assert np.array_equal(g["status"].astype(np.uint32), o["status"]), mode
        assert np.array_equal(g["nupd"], o["nupd"]), mode
        fp64_close(g, o, oc)
    ctx.close()
