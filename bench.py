"""Benchmark: batched Kalman-filter track fitting on one MI355X.

Workload: 1,000,000 synthetic tracks on 10 cylindrical barrel layers
(r = 4..40 cm, uniform Bz = 3.8 T, no material), pT log-uniform 0.5-100
GeV, |eta| < 1, hits smeared by 0.01 cm in r-phi and 0.1 cm in z, seeds
drawn around the truth.  One step = one fit of every track (propagate to
each layer along the helix, Kalman update with its hit) on inputs already
resident in HBM.  The headline is the float path that holds the 1e-4
parameter bound on every track (float storage and state propagation, the
covariance in double); FP32 bulk (the covariance in float too), the plain
FP64 path, the per-layer graph sweeps, building, serving, uneven events
and the FP64 CPU oracle are measured beside it.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of the fit per track and layer.  The reference model
# (the scope's measurement table): propagation 680 flops, of which F P F^T
# about 200 FMA, and the update 790 FP64 flops.  FP32 bulk runs the
# propagation in FP32; the headline path moves F P F^T to FP64.  Our own
# count of the implemented formulas (FMA = 2) is reported beside it.
REF_PROP, REF_FPF, REF_UPD = 680, 400, 790
OWN_PROP, OWN_FPF, OWN_UPD = 860, 378, 585  # 3 Newton steps + series helix, 189-FMA F P F^T, 585 update
SWEEP_REF_BYTES = 237          # per track-layer, FP32 sweep: state+cov r/w 216, hit 12, chi2 8, flag 1
PEAK_FP32 = 157.3e12           # MI355X vector FP32 (datasheet, packed issue)
PEAK_FP64 = 78.6e12            # MI355X vector FP64
HBM_PEAK = 8.0e12              # bytes/s


def sweep_bytes_per_track_layer(prec_bytes):
    """HBM bytes of one layer step of one track in the per-layer sweep:
    read + write state (6) and covariance (21), read the hit (3) and its
    valid flag, charge, end layer, status, chi2 and hit count, write status,
    chi2, hit count.  FP32 storage carries the position in double between
    layers instead of its stored float copy, which is written only where
    the track ends."""
    b = 3 * prec_bytes + 1 + 1 + 1 + 2 * (4 + 8 + 4)
    if prec_bytes == 4:
        return b + 2 * 24 * prec_bytes + 2 * 3 * 8
    return b + 2 * 27 * prec_bytes


def fused_bytes_per_track(prec_bytes, n_layers):
    """HBM bytes of one track in the fused fit: seed state + covariance,
    charge, hits and valid flags in; state, covariance, chi2, count, status out."""
    return (27 * prec_bytes + 1 + n_layers * (3 * prec_bytes + 1)) + (27 * prec_bytes + 8 + 4 + 4)


def cpu_model():
    """The host CPU's model name, from /proc/cpuinfo."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("fit.hip", "kf_math.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1605_05508_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of one kernel instance (its full template name)
    from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs, scaled by a
    plain copy of known size, or None when the kernel sources changed since
    those counters were taken or that instance was not measured."""
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
        rd, wr = t["kernels"][kernel][:2]
    except (OSError, KeyError, ValueError):
        return None
    if t.get("source_sha") != kernel_sources_sha():
        return None
    return rd + wr


def fit_kernel_name(ts, tp, tc, launch):
    """Template name of the fused-fit instance a tuned launch runs."""
    b, w, k = launch["block"], launch["waves_per_simd"], launch.get("tracks_per_lane", 1)
    if launch.get("persistent"):
        return f"fit_persistent_kernel<{ts}, {tp}, {tc}, {b}, {w}, false, {k}>"
    return f"fit_fused_kernel<{ts}, {tp}, {tc}, {b}, {w}, false, false, {k}>"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU work of the oracle sample (core-seconds)")
    ap.add_argument("--prec", choices=["fp32p", "fp32b", "fp64"], default="fp32p",
                    help="precision of the --profile fit loop (fp32p: the headline path)")
    ap.add_argument("--profile", choices=["fit", "sweep", "build", "copy"], default=None,
                    help="only one timed loop, for rocprofv3 runs (copy: a plain copy of "
                         "known size to calibrate the HBM byte counters)")
    ap.add_argument("--workload", choices=["fit", "uneven", "dense_events", "material", "shapes"], default="fit",
                    help="fit: the headline line; uneven: events of uneven size in one "
                         "launch versus per-event launches; dense_events: building on "
                         "20,000-track events, combinatorial and best-hit; material: the "
                         "fit at scale through layer material; shapes: the fit's time per "
                         "launch shape and its throughput from 1e3 to 1e7 tracks")
    ap.add_argument("--no-build", action="store_true", help="skip the building measurement")
    ap.add_argument("--seed-order", type=int, default=0, help="--profile build: the library's seed order (1) or not (0)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--serve-events", type=int, default=500)
    ap.add_argument("--rates", type=str, default="200,500,1000,2000")
    ap.add_argument("--budgets-mb", type=str, default="16384,1024,512",
                    help="HBM budgets of the serving sweep (MB); a small one makes admission bind")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-events measurement")
    return ap.parse_args()


def serving_measurement(ktf, tg, n_events, rates, budgets):
    """Poisson arrivals of building events (5,000 tracks, 10% heavy events of
    20,000-50,000 tracks, 17 layers, 20% noise) into the continuous-batching
    loop (build + final fit per event), against the plain FP64 path serving
    one event at a time, both closed-loop (its service time) and under the
    same arrivals (its queueing)."""
    import threading
    arrivals, ntr, rng = tg.config5_stream(n_events=n_events, rate=1.0)
    det = tg.barrel(17)
    evs = [tg.make_build_event(rng, int(n), det) for n in ntr]
    # the client hands over float32 arrays (float64 for the FP64 events,
    # converted by the binding), as the C-ABI takes them
    f32 = lambda x: np.ascontiguousarray(x, np.float32)
    f64 = lambda x: np.ascontiguousarray(x, np.float64)
    host = [dict(hit_off=e.hit_off, hits=f32(e.hits), state=f32(e.state), cov=f32(e.cov), q=e.q,
                 seed_hit=e.seed_hit) for e in evs]
    host64 = [dict(hit_off=e.hit_off, hits=f64(e.hits), state=f64(e.state), cov=f64(e.cov), q=e.q,
                   seed_hit=e.seed_hit) for e in evs]

    def run(ctx, rate, prec, sequential=False):
        lat, tracks = [], 0
        pend = {}
        lock = threading.Lock()
        start = ctx.now() + 0.05

        src = host64 if prec == "fp64" else host

        def submitter():
            for i, ev in enumerate(src):
                if not sequential:
                    t_arr = start + arrivals[i] / rate
                    dt = t_arr - ctx.now()
                    if dt > 0:
                        time.sleep(dt)
                t = ctx.submit(dict(ev, prec=prec))
                with lock:
                    pend[t] = i
                if sequential:
                    while True:
                        with lock:
                            if t not in pend:
                                break
                        time.sleep(0.0002)

        th = threading.Thread(target=submitter)
        th.start()
        done = 0
        t_end = None
        while done < len(host):
            with lock:
                items = list(pend.items())
            for t, i in items:
                r = ctx.poll(t, evs[i].n_seeds)
                if r is not None:
                    with lock:
                        del pend[t]
                    lat.append((r["t_done"] - r["t_submit"]) * 1e3)
                    tracks += evs[i].n_seeds
                    done += 1
                    t_end = r["t_done"]
            time.sleep(0.0002)
        th.join()
        span = t_end - start
        lat = np.array(lat)
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "events_per_s": round(len(host) / span, 1), "tracks_per_s": round(tracks / span)}

    out = {"events": n_events, "mean_tracks_per_event": round(float(np.mean(ntr))),
           "heavy_events": int(np.sum(ntr >= 20000))}
    # the continuous-batching loop at each HBM budget: a large one that never
    # binds, and small ones under which admission waits for memory to free up
    out["fp32b_continuous"] = {}
    for budget in budgets:
        ctx = ktf.Context.for_detector(det, hbm_budget_bytes=budget, max_inflight=64)
        run(ctx, 1e9, "fp32b")  # warm-up: workspaces grow to their working size
        # each rate is run once untimed first: its arrivals batch differently
        # from the warm-up's, and a lane's first batch of a new shape may grow
        # its workspace (a regrowth waits for the device)
        per = {}
        for r in rates:
            run(ctx, r, "fp32b")
            per[str(r)] = run(ctx, r, "fp32b")
        out["fp32b_continuous"][f"budget_{budget >> 20}MB"] = per
        ctx.close()
    ctx1 = ktf.Context.for_detector(det, hbm_budget_bytes=16 << 30, max_inflight=1)
    run(ctx1, 1e9, "fp64", sequential=True)
    # closed loop: each event submitted when the previous one is done (the
    # service time alone); then the same Poisson arrivals, queueing
    out["fp64_one_at_a_time"] = run(ctx1, 1e9, "fp64", sequential=True)
    out["fp64_one_at_a_time_poisson"] = {str(r): run(ctx1, r, "fp64") for r in rates}
    ctx1.close()
    return out


def build_efficiency(hit, true_idx, nsl=3):
    """Track efficiency: seeds whose every layer took exactly their own hit
    (or none where they have none).  Hit efficiency: built layers (beyond
    the seed layers) with a true hit where the seed took it.  Fake rate:
    taken hits that are not the seed's own."""
    h, t = hit[nsl:], true_idx[nsl:]
    has = t >= 0
    took = h >= 0
    return {"all_hits_true_fraction": round(float((hit == true_idx).all(axis=0).mean()), 4),
            "hit_efficiency": round(float((h == t)[has].mean()), 4),
            "fake_hit_rate": round(float((h != t)[took].mean()), 5)}


def time_build(ctx, d, o, reps, torch):
    ctx.build(d, out=o)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        ctx.build(d, out=o)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def build_measurement(ctx_cls, tg, torch, reps=5, orc=None, bs=None, precs=("fp32b", "fp64")):
    """Combinatorial building of 100 events x 5,000 tracks (17 layers, 20%
    noise hits, 64 x 512 bins, 10 candidates, chi2 < 30, one missed layer)
    in one batch, and best-hit building (one candidate per seed) on the same
    events."""
    from tests.helpers import build_inputs
    bs = tg.config3() if bs is None else bs
    ctx = ctx_cls.for_detector(bs.det)
    out = {"events": bs.n_events, "seeds": bs.n_seeds, "hits": int(bs.hits.shape[1])}
    hits_by_prec = {}
    for prec in precs:
        d = build_inputs(bs, prec)
        o = ctx.build(d)
        ms = time_build(ctx, d, o, reps, torch)
        hit = o["hit_idx"].cpu().numpy()[:, :bs.n_seeds]
        hits_by_prec[prec] = hit
        out[prec] = {"ms": round(ms, 3), "seeds_per_s": round(bs.n_seeds / (ms * 1e-3)),
                     "events_per_s": round(bs.n_events / (ms * 1e-3), 1),
                     **build_efficiency(hit, bs.true_idx)}
        if prec == "fp32b":
            ctx1 = ctx_cls.for_detector(bs.det, max_cands=1)
            o1 = ctx1.build(d)
            ms1 = time_build(ctx1, d, o1, reps, torch)
            hit1 = o1["hit_idx"].cpu().numpy()[:, :bs.n_seeds]
            out["fp32b_best_hit"] = {"ms": round(ms1, 3), "seeds_per_s": round(bs.n_seeds / (ms1 * 1e-3)),
                                     "events_per_s": round(bs.n_events / (ms1 * 1e-3), 1),
                                     **build_efficiency(hit1, bs.true_idx)}
            del o1
            ctx1.close()
            # the paper's eta partition (Sec. 3) as a seed order: each event's
            # seeds grouped by eta bin, so neighbouring lanes search
            # neighbouring hit bins; every seed's result is unchanged
            perm = tg.eta_order(bs, n_bins=21)
            de = build_inputs(tg.permute_seeds(bs, perm), prec)
            oe = ctx.build(de)
            mse = time_build(ctx, de, oe, reps, torch)
            inv = np.empty_like(perm)
            inv[perm] = np.arange(bs.n_seeds)
            hite = oe["hit_idx"].cpu().numpy()[:, :bs.n_seeds][:, inv]
            out["fp32b_eta_order"] = {"ms": round(mse, 3), "seeds_per_s": round(bs.n_seeds / (mse * 1e-3)),
                                      "eta_bins": 21, "same_hits_as_generation_order": bool(np.array_equal(hite, hit))}
            del de, oe
            # the library's seed order: seeds sorted by their predicted cell on
            # the first building layer, each wave's window box staged in LDS
            ctx2 = ctx_cls.for_detector(bs.det, seed_order=1)
            o2 = ctx2.build(d)
            ms2 = time_build(ctx2, d, o2, reps, torch)
            hit2 = o2["hit_idx"].cpu().numpy()[:, :bs.n_seeds]
            out["fp32b_seed_order"] = {"ms": round(ms2, 3), "seeds_per_s": round(bs.n_seeds / (ms2 * 1e-3)),
                                       "same_hits": bool(np.array_equal(hit2, hit))}
            del o2
            ctx2.close()
            # the paper's eta partition: 21 eta bins by 512 phi bins
            ctx3 = ctx_cls.for_detector(bs.det, n_etabins=21, eta_max=1.2)
            o3 = ctx3.build(d)
            ms3 = time_build(ctx3, d, o3, reps, torch)
            hit3 = o3["hit_idx"].cpu().numpy()[:, :bs.n_seeds]
            out["fp32b_eta_bins"] = {"ms": round(ms3, 3), "seeds_per_s": round(bs.n_seeds / (ms3 * 1e-3)),
                                     "bins": "21 eta x 512 phi over |eta| < 1.2",
                                     "same_hits": bool(np.array_equal(hit3, hit))}
            del o3
            ctx3.close()
        del d, o
    if "fp32b" in hits_by_prec and "fp64" in hits_by_prec:
        # the FP64 build equals the oracle's bit for bit (tests); FP32 bulk
        # may differ only where a decision was a near-tie
        diff = (hits_by_prec["fp32b"] != hits_by_prec["fp64"]).any(axis=0)
        out["fp32b_seeds_differing_from_fp64"] = int(diff.sum())
    if orc is not None:
        m = 100
        t0 = time.perf_counter()
        orc.build_event(bs, 0, seeds=np.arange(m), nthreads=orc.default_threads())
        t = time.perf_counter() - t0
        out["cpu_oracle"] = {"seeds_per_s": round(m / t, 1), "cores": orc.default_threads(),
                             "sample": f"{m} seeds of one event, brute force over every hit"}
    ctx.close()
    return out


def dense_events_workload(args):
    """Building on 25 events of 20,000 tracks (the occupancy of the paper's
    building plots), 17 layers, 20% noise: combinatorial (10 candidates)
    against best-hit (one candidate), FP32 bulk."""
    import torch
    import paper_1605_05508_amd as ktf
    import trackgen as tg
    print("[bench] generating 25 events x 20,000 tracks", file=sys.stderr, flush=True)
    bs = tg.config3(n_events=25, n_tracks=20_000, seed=4)
    print("[bench] building", file=sys.stderr, flush=True)
    res = build_measurement(ktf.Context, tg, torch, bs=bs, precs=("fp32b",))
    print(json.dumps({"metric": "built seeds/s on 20,000-track events, combinatorial vs best-hit",
                      "value": res["fp32b"]["seeds_per_s"], "unit": "seeds/s", "n_gpus": 1,
                      "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
                      "config": {"workload": "25 events x 20,000 tracks, 17 barrel layers, +20% noise hits, "
                                             "64 x 512 bins, chi2 < 30, one missed layer"},
                      "building": res}), flush=True)


def shapes_workload(args):
    """Launch shape and problem size, the GPU's counterpart of the paper's
    vector-width and thread-count scans (Sec. 3.2): the fused fit's time (in
    the precision of --prec, the headline's by default) for every launch
    shape the tuner tries on 1e6 tracks (tracks per block, register budget in
    waves per SIMD, plain or persistent grid, tracks per lane), and the tuned
    fit's throughput from 1e3 to 1e7 tracks (1e7 as ten copies of the 1e6
    tracks)."""
    import torch
    import paper_1605_05508_amd as ktf
    import trackgen as tg
    from tests.helpers import fit_inputs
    print("[bench] generating 1e6 tracks", file=sys.stderr, flush=True)
    fs = tg.config2()
    n = fs.n
    ctx = ktf.Context.for_detector(fs.det)
    prec = args.prec
    pp = None if prec == "fp32b" else prec
    d = fit_inputs(fs, "fp64" if prec == "fp64" else "fp32b", pitch=n)
    dt = d["state"].dtype
    out = ctx.alloc_fit_out(n, n, dt)
    ctx.autotune_fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], out=out, prec=pp)
    tuned = json.loads(ctx.tuned_shape(prec, n, trials=True))
    trials = [{"block": b, "waves_per_simd": w, "persistent": bool(p), "tracks_per_lane": tp, "ms": ms}
              for b, w, p, tp, ms in tuned.pop("trials")]
    del out
    scan = []
    for m in (1_000, 10_000, 100_000, 1_000_000, 10_000_000):
        print(f"[bench] size {m}", file=sys.stderr, flush=True)
        if m <= n:
            x = dict(d, q=d["q"][:m])
            pitch = n
        else:
            k = m // n
            x = dict(state=d["state"].repeat(1, k), cov=d["cov"].repeat(1, k), q=d["q"].repeat(k),
                     hits=d["hits"].repeat(1, 1, k), valid=d["valid"].repeat(1, k))
            pitch = m
        o = ctx.alloc_fit_out(m, pitch, dt)
        ctx.autotune_fit(x["state"], x["cov"], x["q"], x["hits"], x["valid"], out=o, prec=pp)
        run = lambda: ctx.fit(x["state"], x["cov"], x["q"], x["hits"], x["valid"], out=o, prec=pp)
        ms, _ = timed_loop(run, args.steps, args.warmup, torch)
        scan.append({"tracks": m, "ms": round(ms, 4), "tracks_per_s": round(m / (ms * 1e-3)),
                     "launch": json.loads(ctx.tuned_shape(prec, m))})
        del x, o
        torch.cuda.synchronize()
    print(json.dumps({"metric": f"fused fit ({prec}) time per launch shape and tracks/s per problem size",
                      "value": scan[-2]["tracks_per_s"], "unit": "tracks/s", "n_gpus": 1,
                      "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
                      "config": {"workload": "1,000,000 tracks, 10 barrel layers r=4..40 cm, Bz=3.8 T, "
                                             "pT log-uniform 0.5-100 GeV; sizes 1e3..1e7"},
                      "tuned_1e6": tuned, "shapes_1e6": trials, "size_scan": scan}), flush=True)


def material_workload(args):
    """1e6 tracks x 10 layers through 2% X0 layers with energy loss (multiple
    scattering as process noise, mean energy loss): fused fit throughput in
    the three precisions, against the FP64 oracle on a sample."""
    import torch
    import paper_1605_05508_amd as ktf
    import trackgen as tg
    from tests.helpers import fit_inputs, fp32_errors, pulls
    print("[bench] generating tracks through material", file=sys.stderr, flush=True)
    fs = tg.config2_material()
    n, L = fs.n, fs.det.n_layers
    ctx = ktf.Context.for_detector(fs.det)
    res = {}
    outs = {}
    for prec in ("fp32b", "fp32p", "fp64"):
        d = fit_inputs(fs, "fp64" if prec == "fp64" else "fp32b")
        pp = None if prec == "fp32b" else prec
        out = ctx.alloc_fit_out(n, d["state"].shape[1], d["state"].dtype)
        ctx.autotune_fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], out=out, prec=pp)
        run = lambda: ctx.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], out=out, prec=pp)
        ms, _ = timed_loop(run, args.steps, args.warmup, torch)
        torch.cuda.synchronize()
        outs[prec] = {k: v.cpu().numpy()[..., :n] for k, v in out.items()}
        res[prec] = {"ms": round(ms, 4), "tracks_per_s": round(n / (ms * 1e-3)),
                     "launch": ctx.tuned_shape(prec, n)}
        del d, out
    if not args.no_cpu:
        import oracle
        m = 100_000
        sub = fs.subset(np.arange(m))
        o = oracle.fit(sub)
        po = pulls(o["state"], o["cov"], sub.truth_pos[-1], sub.truth_mom[-1])
        for prec, g in outs.items():
            gs = {k: v[..., :m] for k, v in g.items()}
            e_pos, e_mom = fp32_errors(gs, o, 40.0)
            pg = pulls(gs["state"], gs["cov"], sub.truth_pos[-1], sub.truth_mom[-1])
            res[prec].update({"e_mom_max": float(e_mom.max()), "e_mom_p999": float(np.quantile(e_mom, 0.999)),
                              "pull_rms_ratio": {kk: round(float(np.sqrt(np.mean(pg[kk] ** 2)) /
                                                                 np.sqrt(np.mean(po[kk] ** 2))), 5) for kk in pg}})
        res["oracle_pull_rms"] = {kk: round(float(np.sqrt(np.mean(v ** 2))), 4) for kk, v in po.items()}
        res["oracle_sample"] = m
    print(json.dumps({"metric": "fitted tracks/s through layer material", "value": res["fp32b"]["tracks_per_s"],
                      "unit": "tracks/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32+f64",
                      "data": "synthetic",
                      "config": {"workload": "1,000,000 tracks, 10 barrel layers r=4..40 cm of 2% X0 each, "
                                             "energy loss 0.036 GeV per X0, Bz=3.8 T, pT log-uniform 0.5-100 GeV"},
                      "detail": res}), flush=True)


def uneven_workload(args):
    """Events of uneven size: 2,000 events with log-normal track counts
    (median 3,000, sigma 0.8, clipped 50-50,000), 6-17 hits per track with
    0-3 missing layers, FP32-bulk.  One launch over all events (fused,
    persistent, per-layer graph sweep) against one launch per event."""
    import torch
    import paper_1605_05508_amd as ktf
    import trackgen as tg
    from tests.helpers import fit_inputs
    print("[bench] generating the uneven-events workload", file=sys.stderr, flush=True)
    fs, offs = tg.config4()
    n = fs.n
    ctx = ktf.Context.for_detector(fs.det)
    d = fit_inputs(fs, "fp32b")
    out = ctx.alloc_fit_out(n, d["state"].shape[1], torch.float32)
    print("[bench] autotuning", file=sys.stderr, flush=True)
    ctx.autotune_fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], out=out)
    res = {"events": len(offs) - 1, "tracks": n,
           "hits_per_track": round(float(fs.valid.sum(axis=0).mean()), 3)}
    for mode in ("auto", "fused", "persistent", "sweep_graph"):
        ms, _ = timed_loop(lambda: ctx.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"],
                                           mode=mode, out=out), 10, 2, torch)
        res[mode] = {"ms": round(ms, 4), "tracks_per_s": round(n / (ms * 1e-3))}
    res["tuned_launch"] = ctx.tuned_shape("fp32b", n)
    # per-event launches on views of the same buffers (each event its own pitch window)
    print("[bench] per-event launches", file=sys.stderr, flush=True)
    per = []
    for e in range(len(offs) - 1):
        a, b = int(offs[e]), int(offs[e + 1])
        ev = tg.FitSet(fs.det, fs.state[:, a:b], fs.cov[:, a:b], fs.q[a:b], fs.hits[:, :, a:b],
                       fs.valid[:, a:b], fs.truth_pos[:, :, a:b], fs.truth_mom[:, :, a:b])
        per.append((fit_inputs(ev, "fp32b"), b - a))
    outs = [ctx.alloc_fit_out(m, dd["state"].shape[1], torch.float32) for dd, m in per]

    def all_events():
        for (dd, m), oo in zip(per, outs):
            ctx.fit(dd["state"], dd["cov"], dd["q"], dd["hits"], dd["valid"], mode="fused", out=oo)

    ms, wall = timed_loop(all_events, 3, 1, torch)
    res["per_event_launches"] = {"ms": round(ms, 4), "tracks_per_s": round(n / (ms * 1e-3)),
                                 "launches": len(per), "wall_ms": round(wall, 3)}
    res["one_launch_speedup"] = round(ms / res["auto"]["ms"], 2)
    line = {"metric": "fitted tracks/s, uneven events in one launch vs per-event launches",
            "value": res["auto"]["tracks_per_s"], "unit": "tracks/s", "n_gpus": 1,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "uneven batching: 2,000 events, log-normal track counts, "
                                   "6-17 hits, 0-3 missing layers, 17 layers"},
            "detail": res}
    print(json.dumps(line))


def profile_run(args):
    """One timed loop only, for rocprofv3 (no oracle, no other kernels)."""
    import torch
    import paper_1605_05508_amd as ktf
    import trackgen as tg
    from tests.helpers import build_inputs, fit_inputs
    if args.profile == "copy":
        # a plain device copy of known size: 256 MiB read, 256 MiB written
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "steps": args.steps}))
        return
    if args.profile in ("fit", "sweep"):
        fs = tg.config2(n=args.n)
        ctx = ktf.Context.for_detector(fs.det)
        prec = "fp32b" if args.profile == "sweep" and args.prec == "fp32p" else args.prec
        d = fit_inputs(fs, "fp64" if prec == "fp64" else "fp32b")
        pp = None if prec == "fp32b" else prec
        out = ctx.alloc_fit_out(fs.n, d["state"].shape[1], d["state"].dtype)
        # the same launch the headline times: the tuned shape of the fused
        # kernel (tuning launches appear in the trace under their own names)
        if args.profile == "fit":
            ctx.autotune_fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], out=out, prec=pp)
        mode = "auto" if args.profile == "fit" else "sweep_graph"
        run = lambda: ctx.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode, out=out, prec=pp)
        ms, _ = timed_loop(run, args.steps, args.warmup, torch)
        print(json.dumps({"ms_per_step": ms, "n": fs.n}))
        return
    bs = tg.config3()
    ctx = ktf.Context.for_detector(bs.det, seed_order=args.seed_order)
    d = build_inputs(bs, "fp32b")
    o = ctx.build(d)
    run = lambda: ctx.build(d, out=o)
    ms, _ = timed_loop(run, args.steps, args.warmup, torch)
    print(json.dumps({"ms_per_step": ms, "seeds": bs.n_seeds}))


def roofline_of(f32, f64, ms):
    """Mixed-precision ALU roofline of a launch doing f32 FP32 and f64 FP64
    flops in ms: the time at the published peaks, and the fraction of it
    achieved (t_bound / t_measured)."""
    t_bound = f32 / PEAK_FP32 + f64 / PEAK_FP64
    return {"achieved": (f32 + f64) / (ms * 1e-3), "peak": (f32 + f64) / t_bound,
            "frac": t_bound / (ms * 1e-3), "t_bound_us": t_bound * 1e6}


def timed_loop(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall / steps * 1e3


def per_launch_ms(fn, reps, torch):
    """Average duration of one launch, from events recorded on the stream the
    kernels run on (torch's current stream, which the binding passes down)."""
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(s)
        fn()
        b.record(s)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


def uneven_summary(ktf, tg, torch, steps):
    """Events of uneven size (2,000 events, log-normal track counts, 6-17
    hits, 0-3 missing layers; FP32 bulk) in one launch of the tuned fused
    kernel, against one launch per event: issued from the host, and the
    same 2,000 launches captured once in a graph and replayed (device time
    without host launch overhead)."""
    from tests.helpers import fit_inputs
    print("[bench] uneven events: generating", file=sys.stderr, flush=True)
    fs, offs = tg.config4()
    n = fs.n
    ctx = ktf.Context.for_detector(fs.det)
    d = fit_inputs(fs, "fp32b")
    out = ctx.alloc_fit_out(n, d["state"].shape[1], torch.float32)
    ctx.autotune_fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], out=out)
    res = {"events": len(offs) - 1, "tracks": n,
           "hits_per_track": round(float(fs.valid.sum(axis=0).mean()), 3)}
    for mode in ("auto", "persistent", "sweep_graph"):
        ms, _ = timed_loop(lambda: ctx.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"],
                                           mode=mode, out=out), steps, 2, torch)
        res[mode] = {"ms": round(ms, 4), "tracks_per_s": round(n / (ms * 1e-3))}
    res["tuned_launch"] = json.loads(ctx.tuned_shape("fp32b", n))
    del d, out
    print("[bench] uneven events: per-event launches", file=sys.stderr, flush=True)
    per = []
    for e in range(len(offs) - 1):
        a, b = int(offs[e]), int(offs[e + 1])
        ev = tg.FitSet(fs.det, fs.state[:, a:b], fs.cov[:, a:b], fs.q[a:b], fs.hits[:, :, a:b],
                       fs.valid[:, a:b], fs.truth_pos[:, :, a:b], fs.truth_mom[:, :, a:b])
        per.append((fit_inputs(ev, "fp32b"), b - a))
    outs = [ctx.alloc_fit_out(m, dd["state"].shape[1], torch.float32) for dd, m in per]

    def all_events():
        for (dd, m), oo in zip(per, outs):
            ctx.fit(dd["state"], dd["cov"], dd["q"], dd["hits"], dd["valid"], mode="fused", out=oo)

    ms_host, wall = timed_loop(all_events, 3, 1, torch)
    # the same launches captured once and replayed: a fused launch allocates
    # nothing and records no memset, so it can be captured
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        all_events()
    ms_graph, _ = timed_loop(g.replay, 5, 2, torch)
    res["per_event_launches"] = {"launches": len(per), "host_issued_ms": round(ms_host, 4),
                                 "host_issued_wall_ms": round(wall, 3),
                                 "graph_replay_ms": round(ms_graph, 4),
                                 "graph_replay_tracks_per_s": round(n / (ms_graph * 1e-3))}
    res["one_launch_speedup_vs_graph"] = round(ms_graph / res["auto"]["ms"], 3)
    res["one_launch_speedup_vs_host_issued"] = round(ms_host / res["auto"]["ms"], 2)
    del g, per, outs
    ctx.close()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by tracks/events with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    if args.profile:
        profile_run(args)
        return
    if args.workload == "uneven":
        uneven_workload(args)
        return
    if args.workload == "dense_events":
        dense_events_workload(args)
        return
    if args.workload == "shapes":
        shapes_workload(args)
        return
    if args.workload == "material":
        material_workload(args)
        return
    import torch
    import paper_1605_05508_amd as ktf
    import trackgen as tg
    from tests.helpers import fit_inputs  # device staging of generated arrays

    print(f"[bench] generating {args.n} tracks", file=sys.stderr, flush=True)
    fs = tg.config2(n=args.n)
    n, L = fs.n, fs.det.n_layers
    ctx = ktf.Context.for_detector(fs.det)
    d32 = fit_inputs(fs, "fp32b")
    d64 = fit_inputs(fs, "fp64")
    outp = ctx.alloc_fit_out(n, d32["state"].shape[1], torch.float32)
    out32 = ctx.alloc_fit_out(n, d32["state"].shape[1], torch.float32)
    out64 = ctx.alloc_fit_out(n, d64["state"].shape[1], torch.float64)
    print("[bench] autotuning launch shapes", file=sys.stderr, flush=True)
    ctx.autotune_fit(d32["state"], d32["cov"], d32["q"], d32["hits"], d32["valid"], out=outp, prec="fp32p")
    ctx.autotune_fit(d32["state"], d32["cov"], d32["q"], d32["hits"], d32["valid"], out=out32)
    ctx.autotune_fit(d64["state"], d64["cov"], d64["q"], d64["hits"], d64["valid"], out=out64)
    torch.cuda.synchronize()

    def runp(mode="auto"):
        ctx.fit(d32["state"], d32["cov"], d32["q"], d32["hits"], d32["valid"], mode=mode, out=outp,
                prec="fp32p")

    def run32(mode="auto"):
        ctx.fit(d32["state"], d32["cov"], d32["q"], d32["hits"], d32["valid"], mode=mode, out=out32)

    def run64(mode="auto"):
        ctx.fit(d64["state"], d64["cov"], d64["q"], d64["hits"], d64["valid"], mode=mode, out=out64)

    print("[bench] timing the headline fused fit", file=sys.stderr, flush=True)
    ms, wall_ms = timed_loop(runp, args.steps, args.warmup, torch)
    k_ms = per_launch_ms(runp, 10, torch)

    print("[bench] timing FP32 bulk, FP64, graph sweeps", file=sys.stderr, flush=True)
    ms32, _ = timed_loop(run32, max(3, args.steps // 2), 2, torch)
    k32_ms = per_launch_ms(run32, 10, torch)
    ms64, _ = timed_loop(run64, max(3, args.steps // 2), 2, torch)
    ms32_sw, _ = timed_loop(lambda: run32("sweep_graph"), max(3, args.steps // 2), 2, torch)
    ms64_sw, _ = timed_loop(lambda: run64("sweep_graph"), max(3, args.steps // 2), 2, torch)

    # results of the timed configurations, for the error report
    runp()
    run32()
    run64()
    torch.cuda.synchronize()
    gp = {k: v.cpu().numpy()[..., :n] for k, v in outp.items()}
    g32 = {k: v.cpu().numpy()[..., :n] for k, v in out32.items()}
    g64 = {k: v.cpu().numpy()[..., :n] for k, v in out64.items()}

    # roofline of the headline kernel: ALU bound, the reference flop model
    # with F P F^T in FP64; our own count beside it
    launch_p = json.loads(ctx.tuned_shape("fp32p", n))
    launch_b = json.loads(ctx.tuned_shape("fp32b", n))
    hp = fit_kernel_name("float", "float", "double", launch_p)
    ref = roofline_of((REF_PROP - REF_FPF) * L * n, (REF_UPD + REF_FPF) * L * n, k_ms)
    own = roofline_of((OWN_PROP - OWN_FPF) * L * n, (OWN_UPD + OWN_FPF) * L * n, k_ms)
    traffic = measured_traffic(hp)
    roof = {"bound": "alu", "achieved": round(ref["achieved"] / 1e12, 2), "peak": round(ref["peak"] / 1e12, 1),
            "unit": "TFLOP/s", "frac": round(ref["frac"], 4),
            "traffic": None if traffic is None else round(traffic / 1e6, 1),
            "traffic_unit": "MB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": hp, "kernel_ms": round(k_ms, 4), "t_bound_us": round(ref["t_bound_us"], 1),
            "flop_model": f"per track-layer {REF_PROP - REF_FPF} FP32 + {REF_UPD + REF_FPF} FP64 "
                          "(propagation 680 with F P F^T 400 moved to FP64, update 790)",
            "frac_own_count": round(own["frac"], 4),
            "own_count": f"per track-layer {OWN_PROP - OWN_FPF} FP32 + {OWN_UPD + OWN_FPF} FP64",
            "hbm_GBps": round(fused_bytes_per_track(4, L) * n / (k_ms * 1e-3) / 1e9, 1)}
    r32 = roofline_of(REF_PROP * L * n, REF_UPD * L * n, k32_ms)
    o32 = roofline_of(OWN_PROP * L * n, OWN_UPD * L * n, k32_ms)
    t32 = measured_traffic(fit_kernel_name("float", "float", "float", launch_b))
    sweep = {}
    for name, msv, kern in [("fp32b", ms32_sw, "fit_layer_kernel<float, float, 256, false>"),
                            ("fp64", ms64_sw, "fit_layer_kernel<double, double, 256, false>")]:
        pb = 4 if name == "fp32b" else 8
        by_ref = (SWEEP_REF_BYTES if pb == 4 else 465) * L * n
        by_model = sweep_bytes_per_track_layer(pb) * L * n
        tsw = measured_traffic(kern)
        sweep[name] = {"tracks_per_s": round(n / (msv * 1e-3)), "ms": round(msv, 4),
                       "hbm_frac": round(by_ref / (msv * 1e-3) / HBM_PEAK, 4),
                       "bytes_per_track_layer": SWEEP_REF_BYTES if pb == 4 else 465,
                       "hbm_frac_kernel_bytes": round(by_model / (msv * 1e-3) / HBM_PEAK, 4),
                       "kernel_bytes_per_track_layer": sweep_bytes_per_track_layer(pb),
                       "traffic_MB_per_layer_launch": None if tsw is None else round(tsw / 1e6, 1),
                       "hbm_frac_counters": None if tsw is None else round(tsw * L / (msv * 1e-3) / HBM_PEAK, 4)}

    result = {
        "metric": "fitted tracks/s FP32-bulk vs FP64 plain at pull-RMS match; p50/p99 event ms",
        "value": round(n / (ms * 1e-3)),
        "unit": "tracks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "FP32-bulk vs FP64 fit at scale: 1,000,000 tracks, 10 barrel layers "
                               "r=4..40 cm, Bz=3.8 T, pT log-uniform 0.5-100 GeV",
                   "tracks": n, "layers": L,
                   "precision": "float storage and float state propagation (path solve, helix, transport, "
                                "Jacobian); covariance in double (F P F^T, S^-1, gain, Joseph update)",
                   "launch": launch_p},
        "roofline": roof,
        "fp32_bulk": {"tracks_per_s": round(n / (ms32 * 1e-3)), "ms": round(ms32, 4),
                      "precision": "float propagation including F P F^T, covariance float between layers; "
                                   "S^-1, gain and Joseph update in double",
                      "roofline_frac": round(r32["frac"], 4), "roofline_frac_own_count": round(o32["frac"], 4),
                      "t_bound_us": round(r32["t_bound_us"], 1), "kernel_ms": round(k32_ms, 4),
                      "traffic_MB": None if t32 is None else round(t32 / 1e6, 1),
                      "launch": launch_b},
        "fp64_plain": {"tracks_per_s": round(n / (ms64 * 1e-3)), "ms": round(ms64, 4),
                       "launch": json.loads(ctx.tuned_shape("fp64", n))},
        "speedup_over_fp64": round(ms64 / ms, 3),
        "speedup_fp32b_over_fp64": round(ms64 / ms32, 3),
        "sweep_graph": sweep,
        "wall_ms_per_step": round(wall_ms, 4),
    }

    if not args.no_cpu:
        import oracle
        cores = oracle.default_threads()
        # size the sample for about args.cpu_seconds of CPU work
        probe = 2000
        t0 = time.perf_counter()
        oracle.fit(fs.subset(np.arange(probe)), nthreads=1)
        per_track = (time.perf_counter() - t0) / probe
        m = int(min(n, max(probe, args.cpu_seconds / per_track)))
        sub = fs.subset(np.arange(m))
        print(f"[bench] CPU oracle on {m} tracks x {cores} threads", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        o = oracle.fit(sub, nthreads=cores)
        t_cpu = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(m / t_cpu), "unit": "tracks/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": f"first {m} of the {n} tracks, FP64 scalar C, "
                                            f"{cores} threads, wall {t_cpu:.2f} s",
                                  "value_1core": round(1.0 / per_track),
                                  "sample_1core": f"first {probe} tracks on one thread",
                                  "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        # accuracy of every GPU path on the oracle's sample
        from tests.helpers import fp32_errors, param_rel_errors, pulls
        acc = {}
        ptv = np.hypot(o["state"][3], o["state"][4])
        po = pulls(o["state"], o["cov"], sub.truth_pos[-1], sub.truth_mom[-1])
        for name, g in (("headline_fp32p", gp), ("fp32b", g32), ("fp64", g64)):
            gs = {k: v[..., :m] for k, v in g.items()}
            e_pos, e_mom = fp32_errors(gs, o, 40.0)
            e_rel = param_rel_errors(gs, o)
            c2rel = np.abs(gs["chi2"] - o["chi2"]) / np.maximum(1.0, np.abs(o["chi2"]))
            pg = pulls(gs["state"], gs["cov"], sub.truth_pos[-1], sub.truth_mom[-1])
            acc[name] = {"e_pos_max": float(e_pos.max()), "e_mom_max": float(e_mom.max()),
                         "e_mom_p999": float(np.quantile(e_mom, 0.999)),
                         "e_rel_max": float(e_rel.max()),
                         "tracks_e_mom_above_1e-4": int(np.sum(e_mom > 1e-4)),
                         "tracks_e_rel_above_1e-4": int(np.sum(e_rel > 1e-4)),
                         "chi2_rel_err_p9999": float(np.quantile(c2rel, 0.9999)),
                         "chi2_rel_err_max": float(c2rel.max()),
                         "e_mom_max_by_pt": {f"{lo:g}-{hi:g}": float(e_mom[(ptv >= lo) & (ptv < hi)].max(initial=0.0))
                                             for lo, hi in ((0.5, 2), (2, 10), (10, 30), (30, 100))},
                         "pull_rms_ratio": {kk: round(float(np.sqrt(np.mean(pg[kk] ** 2)) /
                                                            np.sqrt(np.mean(po[kk] ** 2))), 5)
                                            for kk in pg},
                         "status_mismatch": int(np.sum(gs["status"].astype(np.uint32) != o["status"]))}
        acc["oracle_pull_rms"] = {kk: round(float(np.sqrt(np.mean(v ** 2))), 4) for kk, v in po.items()}
        result["accuracy_vs_oracle"] = acc
    del d32, d64, outp, out32, out64, gp, g32, g64
    ctx.close()
    torch.cuda.empty_cache()
    if not args.no_build:
        print("[bench] building", file=sys.stderr, flush=True)
        orc = None
        if not args.no_cpu:
            import oracle as orc
        result["building"] = build_measurement(ktf.Context, tg, torch, orc=orc)
        torch.cuda.empty_cache()
    if not args.no_uneven:
        result["uneven_events"] = uneven_summary(ktf, tg, torch, max(3, args.steps // 2))
        torch.cuda.empty_cache()
    if not args.no_serving:
        print("[bench] serving loop", file=sys.stderr, flush=True)
        rates = [float(r) for r in args.rates.split(",")]
        budgets = [int(b) << 20 for b in args.budgets_mb.split(",")]
        result["serving"] = serving_measurement(ktf, tg, args.serve_events, rates, budgets)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
