"""A sweep of building configurations against the FP64 oracle: for a fixed
list of seeded cases (layer counts, beam widths, missed-layer allowances,
chi2 cuts, with and without layer material, ghost hits that make
candidates branch, several events of uneven size in one batch, radial and
tangential hit resolutions that differ (each hit then gets its own rotated
covariance and S); the beam
widths cover every lanes-per-seed and slots-per-lane form of the merge), the FP64
GPU build must give every seed exactly the oracle's hits, hit count and
status, and its chi2 within 1e-10."""
import numpy as np
import pytest

import trackgen as tg
from helpers import build_inputs, host, with_ghosts

pytestmark = pytest.mark.gpu

CASES = [
    # (seed, layers, max_cands, max_missed, chi2_cut, x0, events' track counts[, resolutions])
    (101, 6, 1, 0, 30.0, 0.0, (120,)),
    (102, 9, 4, 1, 30.0, 0.0, (80, 0, 150)),
    (103, 12, 10, 1, 30.0, 0.01, (200, 60)),
    (104, 17, 16, 2, 30.0, 0.0, (90,)),
    (105, 10, 7, 1, 12.0, 0.0, (140, 140)),
    (106, 8, 10, 2, 60.0, 0.02, (100,)),
    (107, 14, 3, 0, 30.0, 0.005, (60, 220, 10)),
    (108, 17, 10, 1, 30.0, 0.01, (250,)),
    (109, 11, 6, 1, 30.0, 0.0, (150, 90)),
    (110, 9, 12, 2, 40.0, 0.0, (120,)),
    (111, 8, 2, 1, 30.0, 0.0, (200,)),
    (112, 12, 10, 1, 30.0, 0.0, (150, 80), dict(sigma_r=0.02, sigma_rphi=0.01)),
    (113, 9, 5, 1, 30.0, 0.01, (120,), dict(sigma_r=0.05, sigma_rphi=0.01)),
    (114, 10, 3, 1, 30.0, 0.0, (160,), dict(sigma_r=0.01, sigma_rphi=0.03)),
]


@pytest.fixture(scope="module")
def k():
    import paper_1605_05508_amd as k
    return k


@pytest.mark.parametrize("seed_order", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_build_configurations(k, orc, case, seed_order):
    seed, L, nc, missed, cut, x0, sizes = case[:7]
    res = case[7] if len(case) > 7 else {}
    rng = np.random.default_rng(seed)
    det = tg.barrel(L, x0=x0, eloss=0.036 if x0 > 0 else 0.0, **res)
    evs = [with_ghosts(tg.make_build_event(rng, n, det), seed * 10 + i) for i, n in enumerate(sizes)]
    bs = tg.concat_events(evs)
    ctx = k.Context.for_detector(det, max_cands=nc, max_missed=missed, chi2_cut=cut, seed_order=seed_order)
    g = host(ctx.build(build_inputs(bs, "fp64")), bs.n_seeds)
    outs = [orc.build_event(bs, e, max_cands=nc, max_missed=missed, chi2_cut=cut)
            for e in range(bs.n_events)]
    o = {key: np.concatenate([x[key] for x in outs], axis=-1) for key in outs[0]}
    assert np.array_equal(g["hit_idx"], o["hit_idx"])
    assert np.array_equal(g["nhits"], o["nhits"])
    assert np.array_equal(g["status"].astype(np.uint32), o["status"])
    np.testing.assert_allclose(g["chi2"], o["chi2"], rtol=1e-10, atol=1e-12)
    ctx.close()
