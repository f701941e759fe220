"""Building parity over every seed of the combinatorial-building workload
(100 events x 5,000 tracks, 17 layers, 20% noise hits, 64 x 512 bins, 10
candidates, chi2 < 30, one missed layer): the GPU build against the
brute-force FP64 oracle for all 500,000 seeds.

FP64: hit indices, hit counts and status exactly the oracle's, chi2 within
1e-10 relative.  FP32 bulk: every seed whose hits differ from the oracle's is
adjudicated at its first differing decision (the layer whose kept (parent,
hit) list differs, else the final choice) by the oracle's decision margin
against the threshold of the tests (TAU_FP32B).

Minutes of CPU for the oracle (about 1,500 seeds/s on 16 threads); not part
of the pytest suite.  Run on a GPU machine from the repository root:
    python tests/full_build_parity.py [--events N]
Prints progress per event and one JSON summary line at the end.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--events", type=int, default=100)
    args = ap.parse_args()
    import torch  # noqa: F401  (the device runtime first, then the library)
    import oracle
    import paper_1605_05508_amd as ktf
    import trackgen as tg
    from helpers import TAU_FP32B, build_inputs, certified, host

    t0 = time.time()
    bs = tg.config3(n_events=args.events)
    ctx = ktf.Context.for_detector(bs.det)
    g = {}
    for prec in ("fp64", "fp32b"):
        g[prec] = host(ctx.build(build_inputs(bs, prec), hist=True), bs.n_seeds)
    ctx.close()
    print(f"[parity] GPU builds done ({bs.n_seeds} seeds), {time.time() - t0:.1f} s", flush=True)
    fp64_bad, fp32_diff, fp32_uncert, certified_at = 0, 0, 0, []
    margins = []
    max_chi2_rel = 0.0
    for e in range(bs.n_events):
        s0, s1 = int(bs.seed_off[e]), int(bs.seed_off[e + 1])
        o = oracle.build_event(bs, e, debug=True, nthreads=oracle.default_threads())
        sl = slice(s0, s1)
        g64 = {k: v[..., sl] for k, v in g["fp64"].items()}
        bad = ~(g64["hit_idx"] == o["hit_idx"]).all(axis=0)
        bad |= g64["nhits"] != o["nhits"]
        bad |= g64["status"].astype(np.uint32) != o["status"]
        rel = np.abs(g64["chi2"] - o["chi2"]) / np.maximum(1.0, np.abs(o["chi2"]))
        bad |= rel > 1e-10
        max_chi2_rel = max(max_chi2_rel, float(rel.max(initial=0.0)))
        fp64_bad += int(bad.sum())
        g32 = {k: v[..., sl] for k, v in g["fp32b"].items()}
        diff = np.nonzero(~(g32["hit_idx"] == o["hit_idx"]).all(axis=0))[0]
        fp32_diff += len(diff)
        for j in diff:
            ok, layer = certified(o["dbg_n"][:, j], o["dbg"][:, :, :, j], o["margin"][:, j],
                                  g32["count"][:, j], g32["hist"][:, :, :, j], TAU_FP32B)
            margins.append(float(o["margin"][layer, j]))
            certified_at.append(int(layer))
            fp32_uncert += 0 if ok else 1
        print(f"[parity] event {e + 1}/{bs.n_events}: fp64 mismatches {fp64_bad}, fp32 differing "
              f"{fp32_diff} (uncertified {fp32_uncert}), {time.time() - t0:.0f} s", flush=True)
    print(json.dumps({"workload": "100 events x 5,000 tracks, 17 layers, 20% noise, 64 x 512 bins, "
                                  "10 candidates, chi2 < 30, one missed layer",
                      "seeds": int(bs.n_seeds), "fp64_mismatches": fp64_bad,
                      "fp64_chi2_rel_max": max_chi2_rel,
                      "fp32b_seeds_differing": fp32_diff, "fp32b_uncertified": fp32_uncert,
                      "tau": TAU_FP32B, "fp32b_margins": margins, "fp32b_decision_layers": certified_at,
                      "seconds": round(time.time() - t0, 1)}), flush=True)


if __name__ == "__main__":
    main()
