"""Serving: events submitted from the host as they arrive, admitted onto the
GPU as lanes and HBM budget free up, built and fitted there (the paper's
building then fitting, Sec. 2), collected by ticket.  Each event's result
must be the same alone and in the mix."""
import time

import numpy as np
import pytest

import trackgen as tg
from helpers import build_inputs, fp64_close, host, oracle_with_spread

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def k():
    import paper_1605_05508_amd as k
    return k


def host_event(ev, prec="fp32b"):
    return dict(hit_off=ev.hit_off, hits=ev.hits, state=ev.state, cov=ev.cov, q=ev.q,
                seed_hit=ev.seed_hit, prec=prec)


def wait(ctx, t, n, timeout=60.0):
    t0 = time.time()
    while True:
        r = ctx.poll(t, n)
        if r is not None:
            return r
        assert time.time() - t0 < timeout, "serving timed out"
        time.sleep(0.001)


def events(seed, n_ev, sizes=(200, 500, 50, 800)):
    rng = np.random.default_rng(seed)
    det = tg.barrel(17)
    return det, [tg.make_build_event(rng, sizes[i % len(sizes)], det) for i in range(n_ev)]


@pytest.mark.parametrize("prec", ["fp32b", "fp64"])
def test_alone_equals_mix(k, prec):
    det, evs = events(1, 8)
    ctx = k.Context.for_detector(det)
    alone = []
    for ev in evs:
        t = ctx.submit(host_event(ev, prec))
        alone.append(wait(ctx, t, ev.n_seeds))
    tickets = [ctx.submit(host_event(ev, prec)) for ev in evs]
    mix = [wait(ctx, t, ev.n_seeds) for t, ev in zip(tickets, evs)]
    for a, m in zip(alone, mix):
        for key in ("hit_idx", "state", "cov", "chi2", "nhits", "status"):
            assert np.array_equal(a[key], m[key]), key
    st = ctx.serving_stats()
    assert st == dict(queued=0, inflight=0, done=0)
    ctx.close()


def test_fp64_results_match_oracle(k, orc):
    """An FP64 event comes back in double: its hits exactly the oracle's
    building, its final fit over those hits within the FP64 tolerance."""
    det, evs = events(2, 3, sizes=(300,))
    ctx = k.Context.for_detector(det)
    tickets = [ctx.submit(host_event(ev, "fp64")) for ev in evs]
    for t, ev in zip(tickets, evs):
        r = wait(ctx, t, ev.n_seeds)
        assert r["state"].dtype == np.float64 and r["cov"].dtype == np.float64
        o = orc.build_event(ev, 0)
        assert np.array_equal(r["hit_idx"], o["hit_idx"])
        # the final fit over the built hits
        L = det.n_layers
        hits = np.zeros((L, 3, ev.n_seeds))
        valid = (o["hit_idx"] >= 0).astype(np.uint8)
        for l in range(L):
            lh = ev.layer_hits(0, l)
            idx = np.maximum(o["hit_idx"][l], 0)
            hits[l] = lh[:, idx] * valid[l]
        fs = tg.FitSet(det, ev.state, ev.cov, ev.q, hits, valid, ev.truth_pos, ev.truth_mom)
        of, spread = oracle_with_spread(orc, fs)
        g = dict(state=r["state"], cov=r["cov"], chi2=r["chi2"], nupd=r["nhits"], status=r["status"])
        fp64_close(g, of, spread)
    ctx.close()


def test_failed_event_is_isolated(k):
    """A failure forced from the host on one event (ktf_debug_fail_next_event:
    its group fails to launch, before any device work) fails that event
    alone: the events queued with it are retried one by one and their
    results are bit for bit those of running each alone.  Heavy events
    first keep every lane busy, so that the small events queue up and are
    admitted together."""
    det, evs = events(7, 4, sizes=(300, 600, 200, 400))
    rng = np.random.default_rng(17)
    heavy = [tg.make_build_event(rng, 20000, det) for _ in range(4)]
    probe = k.Context.for_detector(det)
    ref = [wait(probe, probe.submit(host_event(ev)), ev.n_seeds) for ev in evs]
    probe.close()
    ctx = k.Context.for_detector(det)
    th = [ctx.submit(host_event(ev)) for ev in heavy]
    tickets = []
    for i, ev in enumerate(evs):
        if i == 1:
            ctx.debug_fail_next_event()
        tickets.append(ctx.submit(host_event(ev)))
    for i, (t, ev) in enumerate(zip(tickets, evs)):
        if i == 1:
            t0 = time.time()
            while True:
                try:
                    r = ctx.poll(t, ev.n_seeds)
                except k.KtfError as e:
                    assert e.code == k.EDEVICE
                    break
                assert r is None, "the injected failure completed"
                assert time.time() - t0 < 60
                time.sleep(0.001)
            continue
        r = wait(ctx, t, ev.n_seeds)
        for key in ("hit_idx", "state", "cov", "chi2", "nhits", "status"):
            assert np.array_equal(r[key], ref[i][key]), (i, key)
    for t, ev in zip(th, heavy):
        wait(ctx, t, ev.n_seeds)
    # the hook fires once: the next event runs normally
    r = wait(ctx, ctx.submit(host_event(evs[1])), evs[1].n_seeds)
    assert np.array_equal(r["hit_idx"], ref[1]["hit_idx"])
    assert ctx.serving_stats() == dict(queued=0, inflight=0, done=0)
    ctx.close()


def test_small_budget_admission(k):
    """With a budget that holds one event at a time, events wait in the
    queue and still all complete; an event larger than the budget is
    refused at submission."""
    det, evs = events(3, 6, sizes=(300,))
    big = tg.make_build_event(np.random.default_rng(9), 20000, det)
    probe = k.Context.for_detector(det)
    ref = [wait(probe, probe.submit(host_event(ev)), ev.n_seeds) for ev in evs]
    probe.close()
    ctx = k.Context.for_detector(det, hbm_budget_bytes=64 << 20, max_inflight=1)
    tickets = [ctx.submit(host_event(ev)) for ev in evs]
    res = [wait(ctx, t, ev.n_seeds) for t, ev in zip(tickets, evs)]
    for a, b in zip(ref, res):
        assert np.array_equal(a["hit_idx"], b["hit_idx"])
    # admissions never overlapped: each event was admitted after the previous finished
    for a, b in zip(res, res[1:]):
        assert b["t_admit"] >= a["t_done"] - 1e-3
    with pytest.raises(k.KtfError) as ei:
        ctx.submit(host_event(big))
    assert ei.value.code == k.ENOMEM
    ctx.close()


def test_unknown_ticket(k):
    det, evs = events(4, 1)
    ctx = k.Context.for_detector(det)
    with pytest.raises(k.KtfError) as ei:
        ctx.poll(12345, 1)
    assert ei.value.code == k.ENOTFOUND
    t = ctx.submit(host_event(evs[0]))
    wait(ctx, t, evs[0].n_seeds)
    with pytest.raises(k.KtfError):
        ctx.poll(t, evs[0].n_seeds)  # already collected
    ctx.close()


def test_material_and_heavy_event_in_the_mix(k):
    """Serving on a detector with layer material, a mix that holds an event
    whose layers have more than 32,768 hits (the multi-kernel binning path)
    beside small ones: every event's hits equal those of a direct build of
    that event, and its result is the same alone and in the mix."""
    rng = np.random.default_rng(6)
    det = tg.barrel(17, x0=0.01, eloss=0.036)
    evs = [tg.make_build_event(rng, n, det) for n in (300, 28000, 500)]
    assert np.diff(evs[1].hit_off).max() > 32768
    ctx = k.Context.for_detector(det)
    direct = []
    for ev in evs:
        direct.append(host(ctx.build(build_inputs(ev, "fp64")), ev.n_seeds)["hit_idx"])
    alone = [wait(ctx, ctx.submit(host_event(ev, "fp64")), ev.n_seeds) for ev in evs]
    tickets = [ctx.submit(host_event(ev, "fp64")) for ev in evs]
    mix = [wait(ctx, t, ev.n_seeds) for t, ev in zip(tickets, evs)]
    for d, a, m in zip(direct, alone, mix):
        assert np.array_equal(a["hit_idx"], d)
        for key in ("hit_idx", "state", "cov", "chi2", "nhits", "status"):
            assert np.array_equal(a[key], m[key]), key
    ctx.close()
