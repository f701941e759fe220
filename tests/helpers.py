"""Shared helpers of the GPU tests: moving generated inputs to the device
and comparing results with the oracle's."""
import numpy as np

import trackgen as tg


def pad_pitch(n, align=64):
    return max(align, (n + align - 1) // align * align)


def to_dev(a, dtype, pitch):
    import torch
    a = np.asarray(a)
    shape = a.shape[:-1] + (pitch,)
    out = np.zeros(shape, dtype=dtype)
    out[..., :a.shape[-1]] = a
    return torch.from_numpy(out).cuda()


def fit_inputs(fs, prec, pitch=None):
    import torch
    dt = np.float64 if prec == "fp64" else np.float32
    pitch = pitch or pad_pitch(fs.n)
    return dict(state=to_dev(fs.state, dt, pitch), cov=to_dev(fs.cov, dt, pitch),
                q=torch.from_numpy(np.ascontiguousarray(fs.q, np.int8)).cuda(),
                hits=to_dev(fs.hits, dt, pitch), valid=to_dev(fs.valid, np.uint8, pitch))


def host(out, n):
    return {k: v.cpu().numpy()[..., :n] for k, v in out.items()}


def sigma_diag(cov):
    idx = [0, 6, 11, 15, 18, 20]
    return np.sqrt(np.abs(cov[idx]))


def diverged(r):
    """Fits the linearised filter lost: a status bit, or chi2/ndf >= 50 with
    the diffuse-prior ndf 2 n - 5."""
    ndf = np.maximum(1, 2 * r["nupd"] - 5)
    return (r["status"] != 0) | (r["chi2"] / ndf >= 50)


_DIAG = [0, 6, 11, 15, 18, 20]


def norm_dev(a, o):
    """Per track, the largest normalized difference of a from o: state
    components |a-b| / (|b| + sigma_i), covariance |dP_ij| / sqrt(P_ii P_jj),
    chi2 |a-b| / max(1, |b|).  Entries non-finite in o count where a's
    finiteness differs (inf), else not at all."""
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        sig = sigma_diag(o["cov"])
        parts = [np.abs(a["state"] - o["state"]) / (np.abs(o["state"]) + sig)]
        k = 0
        rows = []
        for i in range(6):
            for j in range(i, 6):
                scale = np.sqrt(np.abs(o["cov"][_DIAG[i]] * o["cov"][_DIAG[j]]))
                rows.append(np.abs(a["cov"][k] - o["cov"][k]) / scale)
                k += 1
        parts.append(np.stack(rows))
        parts.append((np.abs(a["chi2"] - o["chi2"]) / np.maximum(1.0, np.abs(o["chi2"])))[None])
        d = np.concatenate(parts, axis=0)
        fin_o = np.concatenate([np.isfinite(o["state"]), np.isfinite(o["cov"]), np.isfinite(o["chi2"])[None]])
        fin_a = np.concatenate([np.isfinite(a["state"]), np.isfinite(a["cov"]), np.isfinite(a["chi2"])[None]])
        d = np.where(fin_o & fin_a, np.nan_to_num(d, nan=0.0, posinf=0.0), 0.0)
        d = np.where(fin_o != fin_a, np.inf, d)
    return d.max(axis=0)


def perturb_ulp(fs, seed):
    """The fit set with every seed and hit value moved by one ulp up or down
    (a fixed random pattern per seed)."""
    rng = np.random.default_rng(seed)
    f = lambda a: a * (1 + rng.choice([-1.0, 1.0], a.shape) * 2.0 ** -52)
    return tg.FitSet(fs.det, f(fs.state), f(fs.cov), fs.q, f(fs.hits), fs.valid, fs.truth_pos,
                     fs.truth_mom)


def spread_of(o, alts):
    """Per track, the largest norm_dev from the oracle's result o of other
    results of the same oracle that differ from it only by rounding; they
    must agree with it on status and hit counts."""
    for a in alts:
        assert np.array_equal(a["status"], o["status"]) and np.array_equal(a["nupd"], o["nupd"])
    return np.max(np.stack([norm_dev(a, o) for a in alts]), axis=0)


def oracle_with_spread(orc, fs, n_perturb=4, **kw):
    """The oracle's fit of fs and its own rounding spread per track: the
    largest deviation from that fit of the contracted build of the same
    oracle and of fits of inputs perturbed by one ulp (fixed seeds)."""
    o = orc.fit(fs, **kw)
    alts = [orc.fit(fs, contract=True, **kw)]
    alts += [orc.fit(perturb_ulp(fs, 100 + s), **kw) for s in range(n_perturb)]
    return o, spread_of(o, alts)


def fp64_close(g, o, spread=None, tol=1e-10, k_spread=10.0):
    """FP64 parity of every track: status and hit counts exact, values within
    tol by norm_dev.  spread: the oracle's own rounding spread per track
    (oracle_with_spread); a track whose spread exceeds tol / k_spread --
    large where the linearisation is stretched (refits, heavy energy loss,
    fits the filter lost) -- is held to k_spread times its spread."""
    assert np.array_equal(g["status"].astype(np.uint32), o["status"].astype(np.uint32)), \
        np.nonzero(g["status"].astype(np.uint32) != o["status"].astype(np.uint32))
    assert np.array_equal(g["nupd"], o["nupd"]), np.nonzero(g["nupd"] != o["nupd"])
    t = np.full(o["chi2"].shape, tol)
    if spread is not None:
        t = np.maximum(t, k_spread * spread)
    # a fit that stopped on a non-finite state or covariance (the same bit on
    # both sides, checked above) has no meaningful values: the oracle's full
    # 6x6 products turn a 0 * inf into NaN where the kernels' structured
    # products never form it
    t = np.where(o["status"].astype(np.uint32) & 4, np.inf, t)
    d = norm_dev(g, o)
    bad = np.nonzero(~(d <= t))[0]
    assert bad.size == 0, (bad[:10], d[bad[:10]], t[bad[:10]])


def fp32_errors(g, o, radius):
    """e_pos = |d(x,y,z)| / r_L, e_mom = |dp| / |p| against the FP64 oracle."""
    e_pos = np.linalg.norm(g["state"][:3] - o["state"][:3], axis=0) / radius
    e_mom = np.linalg.norm(g["state"][3:] - o["state"][3:], axis=0) / np.linalg.norm(o["state"][3:], axis=0)
    return e_pos, e_mom


def param_rel_errors(g, o):
    """Per track, the largest |a_i - b_i| / (|b_i| + sigma_i) over the six
    parameters: the measure of the FP64 tolerance, applied to FP32 bulk."""
    sig = sigma_diag(o["cov"])
    return (np.abs(g["state"] - o["state"]) / (np.abs(o["state"]) + sig)).max(axis=0)


def pulls(state, cov, truth_pos, truth_mom):
    """Tangential, z, px, py, pz pulls at the last layer vs the truth crossing."""
    d = state - np.concatenate([truth_pos, truth_mom])
    x, y = truth_pos[0], truth_pos[1]
    r = np.hypot(x, y)
    tx, ty = -y / r, x / r
    vt = tx * tx * cov[0] + 2 * tx * ty * cov[1] + ty * ty * cov[6]
    out = {"t": (d[0] * tx + d[1] * ty) / np.sqrt(vt)}
    for i, name, ci in [(2, "z", 11), (3, "px", 15), (4, "py", 18), (5, "pz", 20)]:
        out[name] = d[i] / np.sqrt(cov[ci])
    return out


def with_ghosts(bs, seed, frac=0.6, spread=0.02):
    """Add, beside a fraction of the true hits, a ghost hit a few sigma away
    along phi and z so that candidates branch."""
    rng = np.random.default_rng(seed)
    det = bs.det
    parts, sizes = [], []
    for l in range(det.n_layers):
        h = bs.layer_hits(0, l)
        n_true = int((bs.true_idx[l] >= 0).sum())
        pick = np.nonzero(rng.random(n_true) < frac)[0] if l >= 3 else np.array([], int)
        r = det.radii[l]
        ph = np.arctan2(h[1, pick], h[0, pick]) + rng.normal(0, spread, pick.size) / r
        z = h[2, pick] + rng.normal(0, 0.2, pick.size)
        g = tg.f32(np.stack([r * np.cos(ph), r * np.sin(ph), z]))
        parts.append(np.concatenate([h, g], axis=1))
        sizes.append(parts[-1].shape[1])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return tg.BuildSet(det, 1, off, np.concatenate(parts, axis=1), bs.seed_off, bs.state,
                       bs.cov, bs.q, bs.seed_hit, bs.true_idx, bs.truth_pos, bs.truth_mom)


def build_inputs(bs, prec, seed_pad=0, hit_pad=0):
    """Device copy of a trackgen.BuildSet in the library's batch layout."""
    import torch
    dt = np.float64 if prec == "fp64" else np.float32
    sp = pad_pitch(bs.n_seeds) + seed_pad
    hp = pad_pitch(bs.hits.shape[1]) + hit_pad
    return dict(seed_off=np.asarray(bs.seed_off, np.int64), hit_off=np.asarray(bs.hit_off, np.int64),
                hits=to_dev(bs.hits, dt, hp), state=to_dev(bs.state, dt, sp), cov=to_dev(bs.cov, dt, sp),
                q=to_dev(bs.q, np.int8, sp), seed_hit=to_dev(bs.seed_hit, np.int32, sp))


# Adjudication threshold of FP32-bulk building mismatches: ten times the
# 99.99th percentile of the FP32-bulk fit's relative chi2 error against the
# FP64 oracle on the 1e6-track fit workload (measured 2.06e-4).
TAU_FP32B = 2.1e-3


def certified(o_dbg_n, o_dbg, o_margin, g_count, g_hist, tau=TAU_FP32B):
    """Adjudication of a building mismatch of one seed: find the first layer
    whose kept (parent, hit) list differs; the mismatch is certified when
    the oracle's smallest decision gap at that layer is within tau.  When
    every layer's list agrees, the difference is the final choice's, judged
    by the oracle's final margin (o_margin[L]).  Returns (certified, layer;
    L for the final choice)."""
    L = o_dbg_n.shape[0]
    for l in range(L):
        n = o_dbg_n[l]
        if g_count[l] != n or not np.array_equal(g_hist[l, :n], o_dbg[l, :n]):
            return bool(o_margin[l] <= tau), l
    return bool(o_margin[L] <= tau), L
