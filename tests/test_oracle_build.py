"""Pins of the oracle's combinatorial track building.

Building (Sec. 3) extends each seed layer by layer with compatible hits
(lowest chi2 increments), branching to keep up to N candidates per seed; the
clone engine (Sec. 3.1) scores all (candidate, hit) pairs into a list, sorts
it and copies only the best N.  A beam that keeps every branch is an
exhaustive search, and a beam of one is the greedy "best hit" approach; both
reduce to plain enumerations written here independently of the oracle's
bookkeeping.
"""
import math

import numpy as np
import pytest

import trackgen as tg
from helpers import with_ghosts

CUT = 30.0


def small_event(seed, n_tracks, n_layers=7, noise=0.2, pt=(0.5, 10.0)):
    rng = np.random.default_rng(seed)
    det = tg.barrel(n_layers)
    return tg.make_build_event(rng, n_tracks, det, noise_frac=noise, pt_range=pt)


def layer_hits(bs, l):
    return bs.layer_hits(0, l).T  # [n, 3]


def seed_phase(orc, bs, s, nsl=3):
    det = bs.det
    x = bs.state[:, s].copy()
    P = orc.unpack(bs.cov[:, s:s + 1])[0]
    chi2 = 0.0
    hits = []
    for l in range(nsl):
        xp, F, _, rc = orc.propagate(x, int(bs.q[s]), det.bz, det.radii[l], l == 0)
        assert rc == 0
        Pp = orc.cov_propagate(P, F)
        h = int(bs.seed_hit[l, s])
        m = layer_hits(bs, l)[h]
        V = orc.hit_cov(m, det.sigma_r, det.sigma_rphi, det.sigma_z)
        x, P, c2, rc = orc.update(xp, Pp, m, V)
        chi2 += c2
        hits.append(h)
    return x, P, chi2, hits


def enumerate_paths(orc, bs, s, max_missed=1, nsl=3):
    """All hit sequences the branching rule admits: on each layer every hit
    with chi2 < cut opens a branch; with none, a missed layer if allowed,
    else the path ends.  Returns (nhits, chi2, hits) of every end point."""
    det = bs.det
    x, P, chi2, hits = seed_phase(orc, bs, s, nsl)
    ends = []

    def rec(l, x, P, chi2, nh, nm, hits):
        if l == det.n_layers:
            ends.append((nh, chi2, hits))
            return
        xp, F, _, rc = orc.propagate(x, int(bs.q[s]), det.bz, det.radii[l])
        if rc:
            ends.append((nh, chi2, hits + [-1] * (det.n_layers - l)))
            return
        Pp = orc.cov_propagate(P, F)
        found = False
        for h, m in enumerate(layer_hits(bs, l)):
            V = orc.hit_cov(m, det.sigma_r, det.sigma_rphi, det.sigma_z)
            c2, rc = orc.chi2(xp, Pp, m, V)
            if rc == 0 and c2 < CUT:
                found = True
                xn, Pn, _, _ = orc.update(xp, Pp, m, V)
                rec(l + 1, xn, Pn, chi2 + c2, nh + 1, nm, hits + [h])
        if not found:
            if nm < max_missed:
                rec(l + 1, xp, Pp, chi2, nh, nm + 1, hits + [-1])
            else:
                ends.append((nh, chi2, hits + [-1] * (det.n_layers - l)))

    rec(nsl, x, P, chi2, 3, 0, hits)
    return ends


def test_wide_beam_equals_exhaustive_search(orc):
    bs = with_ghosts(small_event(1, 30, n_layers=7), 11)
    o = orc.build_event(bs, 0, max_cands=4096)
    branched = 0
    for s in range(bs.n_seeds):
        ends = enumerate_paths(orc, bs, s)
        branched += len(ends) > 1
        best = min(ends, key=lambda e: (-e[0], e[1]))
        assert o["nhits"][s] == best[0]
        assert o["chi2"][s] == pytest.approx(best[1], rel=1e-12)
        assert list(o["hit_idx"][:, s]) == best[2]
    assert branched >= bs.n_seeds // 2  # the search really branched


def test_narrow_beam_differs_from_wide_only_by_pruning(orc):
    """Keeping fewer candidates can only lose: the wide beam (an exhaustive
    search) ends at least as high in the ranking as any narrower one."""
    bs = with_ghosts(small_event(5, 30, n_layers=7), 12)
    wide = orc.build_event(bs, 0, max_cands=4096)
    for nc in (1, 2, 10):
        o = orc.build_event(bs, 0, max_cands=nc)
        for s in range(bs.n_seeds):
            kw = (-wide["nhits"][s], wide["chi2"][s])
            kn = (-o["nhits"][s], o["chi2"][s])
            assert kw <= kn


def test_beam_of_one_is_greedy(orc):
    bs = with_ghosts(small_event(2, 30, n_layers=8), 13)
    o = orc.build_event(bs, 0, max_cands=1)
    det = bs.det
    for s in range(bs.n_seeds):
        x, P, chi2, hits = seed_phase(orc, bs, s)
        nh, nm = 3, 0
        for l in range(3, det.n_layers):
            xp, F, _, rc = orc.propagate(x, int(bs.q[s]), det.bz, det.radii[l])
            Pp = orc.cov_propagate(P, F)
            best = None
            for h, m in enumerate(layer_hits(bs, l)):
                V = orc.hit_cov(m, det.sigma_r, det.sigma_rphi, det.sigma_z)
                c2, rc2 = orc.chi2(xp, Pp, m, V)
                if rc2 == 0 and c2 < CUT and (best is None or c2 < best[0]):
                    best = (c2, h, m, V)
            if best is None:
                if nm == 1:
                    break
                nm += 1
                hits.append(-1)
                x, P = xp, Pp
                continue
            x, P, _, _ = orc.update(xp, Pp, best[2], best[3])
            chi2 += best[0]
            nh += 1
            hits.append(best[1])
        hits += [-1] * (det.n_layers - len(hits))
        assert o["nhits"][s] == nh
        assert list(o["hit_idx"][:, s]) == hits
        assert o["chi2"][s] == pytest.approx(chi2, rel=1e-12)


def test_finds_true_hits(orc):
    """On a config-3-like event (17 layers, 20% noise) the built track of
    almost every seed is its own particle's hits; a true hit fails the cut
    only in the chi2 tail."""
    bs = small_event(3, 300, n_layers=17)
    o = orc.build_event(bs, 0)
    match = (o["hit_idx"] == bs.true_idx)
    per_seed = match.mean(axis=0)
    assert np.mean(per_seed == 1.0) > 0.95
    assert np.all(o["nhits"] >= 14)


def test_debug_records_are_consistent(orc):
    bs = small_event(4, 60, n_layers=9)
    o = orc.build_event(bs, 0, debug=True)
    L, NC = 9, 10
    for s in range(bs.n_seeds):
        # backtrack the winning candidate's hits from the per-layer records
        # when it survived to the end
        n_end = o["dbg_n"][L - 1, s]
        if n_end == 0:
            continue
        assert n_end <= NC
        ranks = o["dbg"][:, :, 0, s]
        hits = o["dbg"][:, :, 1, s]
        paths = []
        for r in range(n_end):
            rr, seq = r, []
            for l in range(L - 1, 2, -1):
                seq.append(hits[l, rr])
                rr = ranks[l, rr]
            paths.append(list(bs.seed_hit[:, s]) + seq[::-1])
        assert len({tuple(p) for p in paths}) == n_end  # distinct candidates
        for l in range(3, L):
            for r in range(o["dbg_n"][l, s]):
                assert 0 <= ranks[l, r] < o["dbg_n"][l - 1, s]


def test_seed_order_does_not_change_results(orc):
    """Seeds are built independently given their event's hits (Sec. 3): the
    oracle on a permuted seed order (the eta-bin order, and a random order
    within each event) gives each seed exactly the same result."""
    det = tg.barrel(9)
    rng = np.random.default_rng(12)
    bs = tg.concat_events([tg.make_build_event(rng, 120, det) for _ in range(2)])
    eta_perm = tg.eta_order(bs)
    rnd_perm = np.concatenate([a + rng.permutation(b - a) for a, b in zip(bs.seed_off[:-1], bs.seed_off[1:])])
    base = [orc.build_event(bs, e) for e in range(bs.n_events)]
    for perm in (eta_perm, rnd_perm):
        assert not np.array_equal(perm, np.arange(bs.n_seeds))
        pb = tg.permute_seeds(bs, perm)
        for e in range(bs.n_events):
            a, b = bs.seed_off[e], bs.seed_off[e + 1]
            o = orc.build_event(pb, e)
            inv = np.argsort(perm[a:b] - a)
            for key in ("hit_idx", "nhits", "chi2", "state", "cov", "status"):
                assert np.array_equal(o[key][..., inv], base[e][key]), key


def test_eta_order_groups_seeds_by_eta_bin():
    det = tg.barrel(6)
    rng = np.random.default_rng(13)
    bs = tg.concat_events([tg.make_build_event(rng, n, det) for n in (300, 0, 200)])
    perm = tg.eta_order(bs, n_bins=21)
    eta = np.arcsinh(bs.state[5] / np.hypot(bs.state[3], bs.state[4]))
    bins = np.clip(np.floor((eta + 1.0) * 21 / 2.0), 0, 20)
    for a, b in zip(bs.seed_off[:-1], bs.seed_off[1:]):
        p = perm[a:b]
        assert np.array_equal(np.sort(p), np.arange(a, b))      # a permutation within the event
        assert np.all(np.diff(bins[p]) >= 0)                      # bins in order
        for v in np.unique(bins[p]):                              # stable within a bin
            q = p[bins[p] == v]
            assert np.all(np.diff(q) > 0)


# ------------------------------------------------------------------ margins
# The oracle's decision margins adjudicate FP32-bulk building mismatches:
# per layer the smallest relative gap of a decision (neighbouring chi2
# totals of equal hit count among the first max_cands + 1 ranked records,
# or a chi2 increment's distance from the cut), and the final choice's gap.
# They are pinned on a designed event whose chi2 values are known in closed
# form: one seed, three seed layers and one building layer whose hits sit
# at x' + a u, with x' the propagated candidate and u scaled to
# u^T S^-1 u = 1, so that a hit's chi2 increment is exactly a^2.

def designed_event(orc, a2, seed=91):
    rng = np.random.default_rng(seed)
    det = tg.barrel(4)
    bs = tg.make_build_event(rng, 1, det, noise_frac=0.0, pt_range=(2.0, 3.0))
    x, P, p_chi2, _ = seed_phase(orc, bs, 0)
    xp, F, _, rc = orc.propagate(x, int(bs.q[0]), det.bz, det.radii[3])
    assert rc == 0
    Pp = orc.cov_propagate(P, F)
    # equal radial and tangential resolutions: V = diag(s^2, s^2, sz^2) for any hit
    S = Pp[:3, :3] + np.diag([det.sigma_r ** 2, det.sigma_rphi ** 2, det.sigma_z ** 2])
    v = np.array([-xp[1], xp[0], 0.3 * det.radii[3]])
    u = v / math.sqrt(v @ np.linalg.solve(S, v))
    new = np.stack([xp[:3] + math.sqrt(a) * u for a in a2], axis=1)
    hits = [bs.layer_hits(0, l) for l in range(3)] + [new]
    off = np.concatenate([[0], np.cumsum([h.shape[1] for h in hits])]).astype(np.int64)
    ev = tg.BuildSet(det, 1, off, np.concatenate(hits, axis=1), bs.seed_off, bs.state, bs.cov, bs.q,
                     bs.seed_hit, bs.true_idx, bs.truth_pos, bs.truth_mom)
    return ev, p_chi2


def rel(a, b):
    return abs(b - a) / max(1.0, abs(a))


@pytest.mark.parametrize("nc,a2,expect,expect_final", [
    # two close records decide the order of the kept pair
    (10, [4.0, 4.5, 20.0], lambda p: rel(p + 4.0, p + 4.5), lambda p: rel(p + 4.0, p + 4.5)),
    # a compatible hit 0.3 below the cut (an incompatible one 0.6 above)
    (10, [4.0, 10.0, 29.7, 30.6], lambda p: 0.3 / 30.0, lambda p: rel(p + 4.0, p + 10.0)),
    # an incompatible hit 0.15 above the cut decides too
    (10, [4.0, 10.0, 30.15], lambda p: 0.15 / 30.0, lambda p: rel(p + 4.0, p + 10.0)),
    # one candidate kept: the gap beyond the first dropped record is no decision,
    # and with one survivor the final choice has no competitor
    (1, [4.0, 6.0, 6.1], lambda p: rel(p + 4.0, p + 6.0), lambda p: math.inf),
    # two kept: the gap between the last kept and the first dropped decides
    (2, [4.0, 6.0, 6.1], lambda p: rel(p + 6.0, p + 6.1), lambda p: rel(p + 4.0, p + 6.0)),
])
def test_margin_closed_form(orc, nc, a2, expect, expect_final):
    ev, p = designed_event(orc, a2)
    o = orc.build_event(ev, 0, max_cands=nc, chi2_cut=CUT, debug=True)
    order = np.argsort(a2)
    compatible = [i for i in order if a2[i] < CUT][:nc]
    assert o["dbg_n"][3, 0] == len(compatible)
    assert list(o["dbg"][3, :len(compatible), 1, 0]) == compatible   # kept hits by chi2
    assert o["hit_idx"][3, 0] == compatible[0] and math.isclose(o["chi2"][0], p + a2[compatible[0]],
                                                                rel_tol=1e-12)
    assert math.isclose(o["margin"][3, 0], expect(p), rel_tol=1e-9), (o["margin"][3, 0], expect(p))
    assert np.all(np.isinf(o["margin"][:3, 0]))   # the seed layers take no decision
    ef = expect_final(p)
    if math.isinf(ef):
        assert math.isinf(o["margin"][4, 0])
    else:
        assert math.isclose(o["margin"][4, 0], ef, rel_tol=1e-9), (o["margin"][4, 0], ef)


def test_final_margin_only_among_equal_hit_counts(orc):
    """Two candidates leave the building layer (hits at chi2 4 and 25); on a
    second building layer one hit sits 5 sigma from the second candidate's
    prediction, away from the first's, which finds nothing and (no missed
    layer allowed) ends with one hit fewer.  The final choice is then
    decided by the hit count alone: no chi2 gap is a decision (infinite
    final margin), and the last layer's margin is the hits' distances from
    the cut."""
    det = tg.barrel(5)
    rng = np.random.default_rng(92)
    bs = tg.make_build_event(rng, 1, det, noise_frac=0.0, pt_range=(2.0, 3.0))
    x, P, p, _ = seed_phase(orc, bs, 0)
    q = int(bs.q[0])
    xp, F, _, _ = orc.propagate(x, q, det.bz, det.radii[3])
    Pp = orc.cov_propagate(P, F)
    V = np.diag([det.sigma_r ** 2, det.sigma_rphi ** 2, det.sigma_z ** 2])
    S = Pp[:3, :3] + V
    v = np.array([-xp[1], xp[0], 0.3 * det.radii[3]])
    u = v / math.sqrt(v @ np.linalg.solve(S, v))
    l3 = np.stack([xp[:3] + 2.0 * u, xp[:3] + 5.0 * u], axis=1)
    cand = []
    for i in range(2):
        m = l3[:, i]
        xn, Pn, c2, rc = orc.update(xp, Pp, m, orc.hit_cov(m, det.sigma_r, det.sigma_rphi, det.sigma_z))
        y, F4, _, rc4 = orc.propagate(xn, q, det.bz, det.radii[4])
        assert rc == 0 and rc4 == 0
        cand.append((y, orc.cov_propagate(Pn, F4)))
    (y0, P0), (y1, P1) = cand
    S1 = P1[:3, :3] + V
    d = y1[:3] - y0[:3]
    h4 = y1[:3] + 5.0 * d / math.sqrt(d @ np.linalg.solve(S1, d))   # chi2 25 for the second
    c2_first, _ = orc.chi2(y0, P0, h4, orc.hit_cov(h4, det.sigma_r, det.sigma_rphi, det.sigma_z))
    assert c2_first > CUT
    hits = [bs.layer_hits(0, l) for l in range(3)] + [l3, h4[:, None]]
    off = np.concatenate([[0], np.cumsum([h.shape[1] for h in hits])]).astype(np.int64)
    ev = tg.BuildSet(det, 1, off, np.concatenate(hits, axis=1), bs.seed_off, bs.state, bs.cov, bs.q,
                     bs.seed_hit, bs.true_idx, bs.truth_pos, bs.truth_mom)
    o = orc.build_event(ev, 0, max_cands=2, max_missed=0, chi2_cut=CUT, debug=True)
    assert o["nhits"][0] == 5 and list(o["hit_idx"][3:, 0]) == [1, 0]
    assert math.isclose(o["chi2"][0], p + 25.0 + 25.0, rel_tol=1e-9)
    assert math.isclose(o["margin"][3, 0], min(rel(p + 4.0, p + 25.0), 5.0 / 30.0, 26.0 / 30.0), rel_tol=1e-9)
    assert math.isclose(o["margin"][4, 0], min(5.0 / 30.0, (c2_first - CUT) / CUT), rel_tol=1e-9)
    assert math.isinf(o["margin"][5, 0])
